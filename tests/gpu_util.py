"""Helpers for the GPU tests: host<->device copies of uint8/uint16 images."""
import numpy as np


def to_dev(a: np.ndarray):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if t.dtype == torch.uint16:  # copy as int16 bits, view back
        return t.view(torch.int16).to("cuda:0").view(torch.uint16)
    return t.to("cuda:0")


def to_host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().view(torch.uint16).numpy()
    return t.cpu().numpy()


def first_mismatch(got: np.ndarray, want: np.ndarray) -> str:
    bad = np.argwhere(got != want)
    if len(bad) == 0:
        return "equal"
    i = tuple(bad[0])
    return "%d mismatches; first at %s: got %s want %s" % (len(bad), i, got[i], want[i])


def announce(*parts):
    print("case:", *parts, flush=True)
