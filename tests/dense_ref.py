"""Independent dense assembly of the Wilson-clover matrix for tiny lattices.

Written separately from the oracle (vectorised NumPy, gamma matrices built as
Kronecker products, clover leaves from np.roll) so that the two can be checked
against each other.  Used only by the oracle's pin tests.

Matrix index = 12*site + 3*spin + colour, site = x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import numpy as np

S0 = np.eye(2, dtype=np.complex128)
S1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
S2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
S3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def gammas():
    """Chiral basis: gamma_k = sigma_2 (x) sigma_k, gamma_t = -sigma_1 (x) 1."""
    return np.array([np.kron(S2, S1), np.kron(S2, S2), np.kron(S2, S3), -np.kron(S1, S0)])


def _grid(U, dims):
    Lx, Ly, Lz, Lt = dims
    return U.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)


def _sh(A, mu, n):
    """A(x + n*mu) on the [t,z,y,x,...] grid."""
    return np.roll(A, -n, axis=3 - mu)


def _dg(A):
    return np.conj(np.swapaxes(A, -1, -2))


def clover_dense(U, dims):
    """C(x) = i sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}, shape [V,12,12]."""
    G = gammas()
    Ug = _grid(U, dims)
    V = int(np.prod(dims))
    Cl = np.zeros(Ug.shape[:4] + (12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Um, Un = Ug[..., mu, :, :], Ug[..., nu, :, :]
            q = Um @ _sh(Un, mu, 1) @ _dg(_sh(Um, nu, 1)) @ _dg(Un)
            # the other three leaves are the first one at x-mu, x-nu, x-mu-nu,
            # re-based to start and end at x
            Umm = _sh(Um, mu, -1)
            Unm = _sh(Un, nu, -1)
            q += Un @ _dg(_sh(_sh(Um, nu, 1), mu, -1)) @ _dg(_sh(Un, mu, -1)) @ Umm
            q += _dg(Umm) @ _dg(_sh(_sh(Un, mu, -1), nu, -1)) @ _sh(_sh(Um, mu, -1), nu, -1) @ Unm
            q += _dg(Unm) @ _sh(Um, nu, -1) @ _sh(_sh(Un, mu, 1), nu, -1) @ _dg(Um)
            A = q - _dg(q)
            tr = np.trace(A, axis1=-2, axis2=-1)
            F = (A - tr[..., None, None] / 3 * np.eye(3)) / 8
            sig = 0.5j * (G[mu] @ G[nu] - G[nu] @ G[mu])
            Cl += 1j * np.einsum("ab,...ij->...aibj", sig, F).reshape(F.shape[:4] + (12, 12))
    return Cl.reshape(V, 12, 12)


def dirac_dense(U, dims, kappa, csw, bc=(1, 1, 1, 1)):
    """The 12V x 12V matrix D."""
    G = gammas()
    V = int(np.prod(dims))
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    Cl = clover_dense(U, dims)
    Lx, Ly, Lz, Lt = dims
    L = (Lx, Ly, Lz, Lt)
    coords = np.stack(np.meshgrid(np.arange(Lx), np.arange(Ly), np.arange(Lz), np.arange(Lt), indexing="ij"), -1)
    coords = coords.transpose(3, 2, 1, 0, 4).reshape(V, 4)
    idx = lambda c: c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))
    I4 = np.eye(4)
    for x in range(V):
        blk = slice(12 * x, 12 * x + 12)
        D[blk, blk] += np.eye(12) + csw * kappa * Cl[x]
        c = coords[x]
        for mu in range(4):
            cf = c.copy()
            cf[mu] = (c[mu] + 1) % L[mu]
            phf = bc[mu] if c[mu] + 1 == L[mu] else 1
            xf = idx(cf)
            D[blk, 12 * xf:12 * xf + 12] += -kappa * phf * np.kron(I4 - G[mu], U[x, mu])
            cb = c.copy()
            cb[mu] = (c[mu] - 1) % L[mu]
            phb = bc[mu] if c[mu] == 0 else 1
            xb = idx(cb)
            D[blk, 12 * xb:12 * xb + 12] += -kappa * phb * np.kron(I4 + G[mu], _dg(U[xb, mu]))
    return D
