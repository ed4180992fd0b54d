"""Seeded synthetic inputs for the Wilson-clover solver: gauge links and sources.

This module generates *inputs* only (random SU(3) links and fermion sources) and
holds none of the solver's arithmetic.  Both the HIP path and the CPU oracle are
fed from it; neither one's computation lives here.

Paper context (Sec. 5, results): the benchmark uses "a random gauge
configuration" on a 32^4 lattice and a Gaussian noise source eta; the paper
gives no generator or seed, so the recipe below fixes one:

* links  U_mu(x) = reunitarise(exp(i eps H)),  H = sum_a h_a lambda_a / 2,
  h_a ~ N(0,1) drawn from numpy PCG64 ``default_rng(seed)`` in the order
  (site in canonical order, mu = 0..3, a = 0..7);
* reunitarise: row0 /= |row0|; row1 -= <row0,row1> row0, row1 /= |row1|;
  row2 = conj(row0 x row1), so every link is exactly SU(3) to FP64 rounding
  and the 12-real (two-row) compression is lossless up to rounding;
* Gaussian source: z = default_rng(seed).standard_normal((V,4,3,2)),
  eta = z[...,0] + i z[...,1];
* point sources: x0 = default_rng(seed).integers(V); the 12 unit vectors at
  (x0, spin, colour).

Host layouts (canonical site index x + Lx*(y + Ly*(z + Lz*t))):
  gauge  complex128 [V][4][3][3]     (mu, row, col)
  spinor complex128 [V][4][3]        (spin, colour)
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "gell_mann", "random_gauge", "unit_gauge", "gaussian_source",
    "point_sources", "random_su3_field", "reunitarise",
]


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def gell_mann() -> np.ndarray:
    """The 8 Gell-Mann matrices lambda_a (Tr lambda_a lambda_b = 2 delta_ab)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def reunitarise(W: np.ndarray) -> np.ndarray:
    """Project a batch [...,3,3] onto SU(3) by Gram-Schmidt of rows 0,1 and
    row2 = conj(row0 x row1)."""
    W = np.array(W, dtype=np.complex128, copy=True)
    r0 = W[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = W[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _expi_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    w, Q = np.linalg.eigh(H)
    return (Q * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))


def random_su3_field(shape, eps: float, rng: np.random.Generator) -> np.ndarray:
    """exp(i eps H) with H = sum_a h_a lambda_a/2, h ~ N(0,1), reunitarised."""
    h = rng.standard_normal(tuple(shape) + (8,))
    H = np.einsum("...a,aij->...ij", h, gell_mann() / 2)
    return reunitarise(_expi_hermitian(H, eps))


def random_gauge(dims, eps: float = 0.5, seed: int = 1) -> np.ndarray:
    """Random SU(3) links, complex128 [V][4][3][3] (see module docstring)."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    return random_su3_field((V, 4), eps, rng)


def unit_gauge(dims) -> np.ndarray:
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def gaussian_source(dims, seed: int = 2, nrhs: int = 1) -> np.ndarray:
    """Gaussian complex noise, complex128 [V][4][3] (or [nrhs][V][4][3])."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    shape = (V, 4, 3, 2) if nrhs == 1 else (nrhs, V, 4, 3, 2)
    z = rng.standard_normal(shape)
    return z[..., 0] + 1j * z[..., 1]


def point_sources(dims, seed: int = 3):
    """The 12 spin-colour point sources at one random site.

    Returns (x0, eta) with eta complex128 [12][V][4][3]; source k = 3*spin+colour.
    """
    V = volume(dims)
    x0 = int(np.random.default_rng(seed).integers(V))
    eta = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        eta[k, x0, k // 3, k % 3] = 1.0
    return x0, eta
