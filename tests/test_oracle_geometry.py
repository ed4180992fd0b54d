"""Pins of the oracle's extended-domain geometry and of the seeded input recipe.

Omega'_i is built here directly from its definition (Sec. 4: each domain is
extended by s sites in both the upward and the downward direction of every
direction that is split, so its extent there is b + 2s and the overlap depth is
d = 2s; a direction the domain spans whole is not extended).  A site x lies in
Omega'_i when, for every split direction mu, (x_mu - o_mu + s) mod L_mu < b_mu + 2s,
o being the origin of Omega_i.  The oracle lists the sites in lexicographic
order of the local coordinate l_mu = (x_mu - o_mu + s_mu) mod L_mu (l_0
fastest); that order is rebuilt here by sorting, not by the oracle's loop.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1011_3318_amd import inputs as I


def coords(dims, x):
    c = []
    for L in dims:
        c.append(x % L)
        x //= L
    return c


def ext_members(dims, block, s, blk):
    """Omega'_blk from the membership rule, in local lexicographic order."""
    nb = [dims[m] // block[m] for m in range(4)]
    o, q = [], blk
    for m in range(4):
        o.append((q % nb[m]) * block[m])
        q //= nb[m]
    sm = [s if block[m] < dims[m] else 0 for m in range(4)]
    e = [block[m] + 2 * sm[m] for m in range(4)]
    members = []
    for x in range(int(np.prod(dims))):
        c = coords(dims, x)
        loc = [(c[m] - o[m] + sm[m]) % dims[m] for m in range(4)]
        if all(loc[m] < e[m] for m in range(4)):
            key = loc[0] + e[0] * (loc[1] + e[1] * (loc[2] + e[2] * loc[3]))
            members.append((key, x))
    members.sort()
    return [x for _, x in members], e


@pytest.mark.parametrize("dims,block,s", [
    ((8, 4, 4, 4), (4, 2, 2, 2), 0),
    ((8, 8, 4, 4), (4, 4, 2, 2), 1),      # s = 1 in every split direction
    ((12, 8, 6, 4), (4, 4, 2, 2), 1),     # unequal extents
    ((12, 4, 4, 4), (4, 4, 4, 4), 2),     # x-only split, d = 4 (Sec. 4)
    ((16, 4, 2, 2), (4, 4, 2, 2), 1),     # x-only split, d = 2
    ((6, 4, 4, 2), (2, 2, 2, 2), 1),      # e = L in y and z: Omega' wraps onto itself there
    ((4, 4, 4, 4), (4, 4, 4, 4), 1),      # b = L everywhere: one domain, no extension
])
def test_extended_domain_membership_and_order(dims, block, s):
    U = I.unit_gauge(dims)
    o = Oracle(dims, U, precompute_clover=False)
    nb, ev = o.decomp(block, s)
    assert nb == int(np.prod([dims[m] // block[m] for m in range(4)]))
    for blk in range(nb):
        want, e = ext_members(dims, block, s, blk)
        assert ev == int(np.prod(e))
        got = o.block_sites(block, s, blk)
        assert len(want) == ev
        assert list(got) == want, blk


def test_extended_domain_is_symmetric_about_the_block():
    """An asymmetric extension (e.g. [o, o + b + 2s) in x) has the same size;
    the membership rule tells it apart: the sites o - s .. o - 1 must be in."""
    dims, block, s = (16, 4, 2, 2), (4, 4, 2, 2), 2
    o = Oracle(dims, I.unit_gauge(dims), precompute_clover=False)
    for blk in range(4):
        got = set(int(x) for x in o.block_sites(block, s, blk))
        xs = sorted(set(coords(dims, x)[0] for x in got))
        ox = blk * 4
        expect = sorted(((ox + d) % 16) for d in range(-s, 4 + s))
        assert xs == expect


def test_generator_anchors():
    """The input recipe's anchors on 4^4, eps = 0.5, seed 1: the first row of
    U_0 at site 0 and the mean plaquette (1/(6V)) sum Re Tr P_{mu nu} / 3."""
    dims = (4, 4, 4, 4)
    U = I.random_gauge(dims, 0.5, 1)
    row0 = U[0, 0, 0]
    want = np.array([0.885093 + 0.161835j, 0.221929 + 0.090583j, 0.198270 - 0.306025j])
    # six printed decimals: real and imaginary parts each within half a unit
    assert np.abs(row0.real - want.real).max() <= 5.01e-7
    assert np.abs(row0.imag - want.imag).max() <= 5.01e-7
    V = I.volume(dims)
    tot = 0.0
    for x in range(V):
        c = coords(dims, x)
        for mu in range(4):
            for nu in range(mu + 1, 4):
                cm = list(c)
                cm[mu] = (cm[mu] + 1) % dims[mu]
                cn = list(c)
                cn[nu] = (cn[nu] + 1) % dims[nu]
                xm = cm[0] + 4 * (cm[1] + 4 * (cm[2] + 4 * cm[3]))
                xn = cn[0] + 4 * (cn[1] + 4 * (cn[2] + 4 * cn[3]))
                P = U[x, mu] @ U[xm, nu] @ U[xn, mu].conj().T @ U[x, nu].conj().T
                tot += np.trace(P).real / 3
    plaq = tot / (6 * V)
    assert abs(plaq - 0.51008) < 5e-6
    # every link SU(3) to rounding
    assert np.abs(np.einsum("...ij,...kj->...ik", U, U.conj()) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13


def test_gaussian_and_point_sources():
    dims = (4, 4, 4, 4)
    eta = I.gaussian_source(dims, 2)
    z = np.random.default_rng(2).standard_normal((256, 4, 3, 2))
    assert np.array_equal(eta, z[..., 0] + 1j * z[..., 1])
    x0, P = I.point_sources(dims, 3)
    assert x0 == int(np.random.default_rng(3).integers(256))
    assert P.shape == (12, 256, 4, 3)
    for k in range(12):
        nz = np.argwhere(P[k] != 0)
        assert nz.tolist() == [[x0, k // 3, k % 3]]
        assert P[k, x0, k // 3, k % 3] == 1
