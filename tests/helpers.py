"""Shared test helpers: comparison metrics and GPU availability."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rel_l1(gpu, ref, ch=None):
    """Relative L1 error per component: sum|q - q_ref| / sum|q_ref| for the 8
    MHD components; psi is normalised by c_h * sum|B| (psi starts at zero).
    A component of m or B whose sum|q_ref| is below a tenth of its vector's
    (the sum over the three components) is normalised by that tenth instead:
    a component that starts at zero and is only grown by the dynamics (B_z
    of a z-modulated vortex) would otherwise be judged by its own tiny size.
    Returns the array of 9 values."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    out = np.empty(9)
    sums = [np.abs(ref[q]).sum() for q in range(9)]
    for q in range(8):
        den = sums[q]
        if q in (1, 2, 3, 5, 6, 7):
            v0 = 1 if q < 4 else 5
            den = max(den, 0.1 * (sums[v0] + sums[v0 + 1] + sums[v0 + 2]))
        num = np.abs(gpu[q] - ref[q]).sum()
        out[q] = num / den if den > 0 else num
    den = (ch if ch else 1.0) * sum(np.abs(ref[q]).sum() for q in (5, 6, 7))
    out[8] = np.abs(gpu[8] - ref[8]).sum() / den if den > 0 else np.abs(gpu[8] - ref[8]).sum()
    return out


def rel_l1_own(gpu, ref):
    """Relative L1 error of each of the 9 components against its own size,
    sum|q - q_ref| / sum|q_ref| (no floor; a component that is zero in the
    reference reports its absolute L1 error)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    out = np.empty(gpu.shape[0])
    for q in range(gpu.shape[0]):
        den = np.abs(ref[q]).sum()
        num = np.abs(gpu[q] - ref[q]).sum()
        out[q] = num / den if den > 0 else num
    return out


def max_rel(gpu, ref):
    """Element-wise error of each of the 8 MHD components: max|q - q_ref|
    over the grid divided by max|q_ref| (the largest magnitude of the
    component's vector for m and B, so a component that is zero somewhere
    or everywhere is measured against its vector's scale).  Returns 8
    values."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    amax = [np.abs(ref[q]).max() for q in range(8)]
    out = np.empty(8)
    for q in range(8):
        den = amax[q]
        if q in (1, 2, 3, 5, 6, 7):
            v0 = 1 if q < 4 else 5
            den = max(amax[v0], amax[v0 + 1], amax[v0 + 2])
        num = np.abs(gpu[q] - ref[q]).max()
        out[q] = num / den if den > 0 else num
    return out


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


requires_gpu = pytest.mark.skipif(not have_gpu(), reason="needs a GPU")


def face_divergence(U, dx):
    """Discrete divergence of the face field of a constrained-transport state
    U[12][nz][ny][nx] (components 9..11: the field on each cell's lower x, y
    and z faces) on a periodic grid: sum over axes of (upper face - lower
    face) / dx_d, per cell."""
    U = np.asarray(U, dtype=np.float64)
    div = np.zeros(U.shape[1:])
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        b = U[9 + d]
        div += (np.roll(b, -1, axis=ax) - b) / dx[d]
    return div
