"""Independent numpy checkers used to pin the oracle (test code only).

None of these share code with the oracle: windows are gathered with numpy's
edge padding (its own clamp-to-edge), and the median is found by counting,
not by selection.
"""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def windows(img: np.ndarray, r: int, dims: int) -> np.ndarray:
    """(..., N) array of the clamp-to-edge windows of the last `dims` axes."""
    pad = [(0, 0)] * (img.ndim - dims) + [(r, r)] * dims
    p = np.pad(img, pad, mode="edge")
    axes = tuple(range(img.ndim - dims, img.ndim))
    v = sliding_window_view(p, (2 * r + 1,) * dims, axis=axes)
    return v.reshape(v.shape[:img.ndim] + (-1,))


def median_by_counting(img: np.ndarray, r: int, dims: int) -> np.ndarray:
    """Median as the smallest window value m with #{u <= m} >= (N+1)/2."""
    w = windows(img, r, dims).astype(np.int64)
    n = w.shape[-1]
    need = (n + 1) // 2
    le = (w[..., None, :] <= w[..., :, None]).sum(-1)  # le[..., j] = #{u <= w_j}
    big = np.iinfo(np.int64).max
    return np.where(le >= need, w, big).min(-1).astype(img.dtype)


def rank_by_counting(img: np.ndarray, r: int, dims: int, k: int) -> np.ndarray:
    """k-th smallest (0-based): smallest m with #{u <= m} >= k+1."""
    w = windows(img, r, dims).astype(np.int64)
    le = (w[..., None, :] <= w[..., :, None]).sum(-1)
    big = np.iinfo(np.int64).max
    return np.where(le >= k + 1, w, big).min(-1).astype(img.dtype)


def box_count(binary: np.ndarray, r: int) -> np.ndarray:
    """Number of ones in each clamp-to-edge (2r+1)^2 window, via a summed-area table."""
    p = np.pad(binary.astype(np.int64), r, mode="edge")
    s = np.zeros((p.shape[0] + 1, p.shape[1] + 1), dtype=np.int64)
    s[1:, 1:] = p.cumsum(0).cumsum(1)
    h, w = binary.shape
    n = 2 * r + 1
    return s[n:n + h, n:n + w] - s[:h, n:n + w] - s[n:n + h, :w] + s[:h, :w]


def median_by_thresholds_u8(img: np.ndarray, r: int) -> np.ndarray:
    """Threshold decomposition (stacking property) of the median filter:
    med >= t  <=>  #{window values >= t} >= (N+1)/2, so
    med = sum_{t=1}^{255} [box_count(img >= t) >= (N+1)/2]."""
    need = ((2 * r + 1) ** 2 + 1) // 2
    out = np.zeros(img.shape, dtype=np.int64)
    for t in range(1, 256):
        b = img >= t
        if not b.any():
            break
        out += box_count(b, r) >= need
    return out.astype(np.uint8)


def rank_dropped_by_coarse_counts(img: np.ndarray, r: int, dims: int, k: int, b: int) -> np.ndarray:
    """Variable precision (Sec. III-D), from counts alone: a descent of the
    uniform tree stopped b levels above the leaves ends in the aligned block of
    2^b grey values that holds the k-th smallest value m and returns its lower
    bound, 2^b * floor(m / 2^b).  That bound is 2^b times the number of t >= 1
    with t * 2^b <= m, and t * 2^b <= m holds exactly when at least N - k
    window values are >= t * 2^b (the stacking property).  No selection, no
    bit mask."""
    w = windows(img, r, dims).astype(np.int64)
    n = w.shape[-1]
    top = 1 << (8 * img.dtype.itemsize)
    out = np.zeros(img.shape, dtype=np.int64)
    for t in range(1, (top >> b) + 1):
        out += (w >= t << b).sum(-1) >= n - k
    return (out << b).astype(img.dtype)


def certificate_ok(img: np.ndarray, out: np.ndarray, r: int, dims: int, k: int) -> bool:
    """m is in the window and #{u < m} <= k < #{u <= m}."""
    w = windows(img, r, dims).astype(np.int64)
    m = out.astype(np.int64)[..., None]
    lt = (w < m).sum(-1)
    le = (w <= m).sum(-1)
    inwin = (w == m).any(-1)
    return bool(np.all(inwin) and np.all(lt <= k) and np.all(k < le))
