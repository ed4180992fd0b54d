"""Shared test helpers (no solver arithmetic of either side lives here)."""
import numpy as np


def rel_err(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def pack_clover_like_abi(C12):
    """Oracle C(x) [V,12,12] -> the ABI's packed host layout [V][2][36]
    (6 real diagonal entries, then 15 complex upper entries row-major) so the
    device-built clover can be compared with the oracle's."""
    V = C12.shape[0]
    out = np.zeros((V, 2, 36))
    iu = [(a, b) for a in range(6) for b in range(a + 1, 6)]
    for k in range(2):
        blk = C12[:, 6 * k:6 * k + 6, 6 * k:6 * k + 6]
        out[:, k, :6] = np.real(np.diagonal(blk, axis1=1, axis2=2))
        for n, (a, b) in enumerate(iu):
            out[:, k, 6 + 2 * n] = blk[:, a, b].real
            out[:, k, 7 + 2 * n] = blk[:, a, b].imag
    return out
