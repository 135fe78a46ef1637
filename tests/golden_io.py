"""Reader for tests/golden/*.txt worked-example fixtures."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _grid(lines, shape, dtype):
    # shape is x-first; rows are x-fastest; 3-D slices separated by "--"
    slices, cur = [], []
    for ln in lines:
        if ln == "--":
            slices.append(cur)
            cur = []
        else:
            cur.append([int(t) for t in ln.split()])
    slices.append(cur)
    arr = np.array(slices, dtype=dtype)
    if len(shape) == 2:
        arr = arr[0]
    expect = tuple(reversed(shape))
    assert arr.shape == expect, (arr.shape, expect)
    return arr


def load_cases(name="worked_examples.txt"):
    cases = []
    with open(os.path.join(GOLDEN, name)) as f:
        lines = [ln.strip() for ln in f]
    i = 0
    while i < len(lines):
        ln = lines[i]
        if not ln.startswith("case "):
            i += 1
            continue
        _, cname, dt, dims, r = ln.split()
        dtype = np.uint8 if dt == "u8" else np.uint16
        i += 1
        shape = [int(t) for t in lines[i].split()[1:]]
        i += 1
        assert lines[i] == "input"
        i += 1
        inp = []
        while lines[i] != "output":
            if lines[i] and not lines[i].startswith("#"):
                inp.append(lines[i])
            i += 1
        i += 1
        out = []
        while lines[i] != "end":
            if lines[i] and not lines[i].startswith("#"):
                out.append(lines[i])
            i += 1
        cases.append(dict(name=cname, dims=int(dims), r=int(r),
                          input=_grid(inp, shape, dtype), output=_grid(out, shape, dtype)))
        i += 1
    return cases
