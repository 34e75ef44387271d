"""Alignment discrepancy between two warping paths (Sec. 4.4 of arXiv 2008.02734).

For every cell (i, j) of one path the row error is the smallest |j - k| over
the cells (i, k) of the other path; the column error is defined the same way
along columns.  The paper reports the distribution of both errors together;
at 43 frames per second its thresholds 23 ms, 47 ms, 510 ms and 1 s are 1, 2,
22 and 43 frames.  Host-side numpy, used to report the reduced-precision
forms against the FP64 path.
"""
import numpy as np

THRESHOLDS_FRAMES = (1, 2, 22, 43)


def _axis_errors(p, q, axis):
    """For each cell of p: min |p[other] - q[other]| over cells of q on the same index along `axis`."""
    other = 1 - axis
    n = int(max(p[:, axis].max(), q[:, axis].max())) + 1
    lo = np.full(n, np.iinfo(np.int64).max, dtype=np.int64)
    hi = np.full(n, np.iinfo(np.int64).min, dtype=np.int64)
    np.minimum.at(lo, q[:, axis], q[:, other])
    np.maximum.at(hi, q[:, axis], q[:, other])
    v = p[:, other].astype(np.int64)
    a = p[:, axis]
    # a monotone path visits a contiguous range of `other` on each index
    return np.where(v < lo[a], lo[a] - v, np.where(v > hi[a], v - hi[a], 0))


def discrepancy(path, ref):
    """Row and column errors of `path` against `ref` (both (K, 2) integer arrays
    of (i, j) cells from (0, 0) to (M-1, N-1)), concatenated."""
    p = np.asarray(path, dtype=np.int64)
    q = np.asarray(ref, dtype=np.int64)
    return np.concatenate([_axis_errors(p, q, 0), _axis_errors(p, q, 1)])


def summary(path, ref):
    """Mean and maximum frame deviation and the fraction of errors within the
    paper's thresholds."""
    e = discrepancy(path, ref)
    out = {"mean_frames": float(e.mean()), "max_frames": int(e.max())}
    for t in THRESHOLDS_FRAMES:
        out[f"frac_le_{t}"] = float(np.mean(e <= t))
    return out
