"""Pins of the oracle's domain decomposition, block operator, MR domain
solver, RAS iteration (Algorithm 1 / Eq. (2)) and nested solver."""
import numpy as np
import pytest

from oracle import Oracle
from paper_1011_3318_amd import inputs as I
import dense_ref as R


def setup(dims, eps=0.5, seed=1, bc=(1, 1, 1, 1)):
    U = I.random_gauge(dims, eps, seed)
    return U, Oracle(dims, U, bc=bc)


def site_ix(sites):
    return (12 * np.asarray(sites)[:, None] + np.arange(12)[None]).reshape(-1)


@pytest.mark.parametrize("dims,block,s", [
    ((6, 4, 4, 2), (2, 2, 2, 2), 0),
    ((6, 4, 4, 2), (2, 2, 2, 2), 1),     # s=1: x extended to 4 of 6, y,z wrap to the full 4
    ((4, 4, 4, 4), (2, 4, 4, 4), 1),     # x-only split, as in the paper
    ((4, 4, 4, 4), (4, 4, 4, 4), 1),     # one block = whole lattice
])
def test_block_operator_is_principal_submatrix(dims, block, s):
    U, o = setup(dims, bc=(1, 1, 1, -1))
    D = R.dirac_dense(U, dims, 0.12, 1.1, bc=(1, 1, 1, -1))
    nb, ev = o.decomp(block, s)
    V = I.volume(dims)
    owned = np.zeros(V, int)
    rng = np.random.default_rng(3)
    for blk in range(nb):
        sites = o.block_sites(block, s, blk)
        assert len(np.unique(sites)) == ev == len(sites)
        ix = site_ix(sites)
        psi = rng.standard_normal((ev, 4, 3)) + 1j * rng.standard_normal((ev, 4, 3))
        got = o.block_apply(block, s, blk, psi, 0.12, 1.1).reshape(-1)
        assert np.abs(got - D[np.ix_(ix, ix)] @ psi.reshape(-1)).max() < 1e-13
        # owned sites = the un-extended block
        origin = [(blk // int(np.prod([dims[m] // block[m] for m in range(mu)]))) % (dims[mu] // block[mu]) * block[mu]
                  for mu in range(4)]
        for x in sites:
            c = [x % dims[0], x // dims[0] % dims[1], x // (dims[0] * dims[1]) % dims[2], x // (dims[0] * dims[1] * dims[2])]
            if all(origin[m] <= c[m] < origin[m] + block[m] for m in range(4)):
                owned[x] += 1
    assert (owned == 1).all()     # the Omega_i partition the lattice
    if tuple(block) == tuple(dims):
        assert np.abs(D[np.ix_(ix, ix)] - D).max() == 0 or np.array_equal(np.sort(sites), np.arange(V))


def test_decomp_rejects_bad_shapes():
    _, o = setup((4, 4, 4, 4))
    with pytest.raises(ValueError):
        o.decomp((3, 4, 4, 4), 0)           # does not divide L
    with pytest.raises(ValueError):
        o.decomp((2, 2, 2, 2), 2)           # b + 2s > L


def test_mr_properties():
    """MR from zero: after one step the residual is orthogonal to D b (the
    1-D least-squares optimum), the residual norm never increases, and many
    steps reach the exact block solution."""
    dims = (4, 4, 4, 4)
    U, o = setup(dims)
    block, s, blk = (2, 2, 2, 2), 1, 5
    _, ev = o.decomp(block, s)
    sites = o.block_sites(block, s, blk)
    Db = R.dirac_dense(U, dims, 0.12, 1.0)[np.ix_(site_ix(sites), site_ix(sites))]
    b = I.gaussian_source(dims, 4)[sites]
    x1 = o.block_mr(block, s, blk, b, 0.12, 1.0, 1).reshape(-1)
    bb = b.reshape(-1)
    r1 = bb - Db @ x1
    assert abs(np.vdot(Db @ bb, r1)) < 1e-12 * np.linalg.norm(Db @ bb) * np.linalg.norm(r1)
    prev = np.linalg.norm(bb)
    for n in (1, 2, 3, 5, 8, 13):
        r = bb - Db @ o.block_mr(block, s, blk, b, 0.12, 1.0, n).reshape(-1)
        assert np.linalg.norm(r) <= prev * (1 + 1e-12)
        prev = np.linalg.norm(r)
    xe = np.linalg.solve(Db, bb)
    x = o.block_mr(block, s, blk, b, 0.12, 1.0, 400).reshape(-1)
    assert np.linalg.norm(x - xe) < 1e-8 * np.linalg.norm(xe)


def test_ras_one_block_is_exact_solve():
    dims = (4, 4, 4, 4)
    U, o = setup(dims)
    eta = I.gaussian_source(dims, 2)
    phi = o.ras(eta, 0.12, 1.0, block=dims, s=0, n_ras=1, n_dominv=0, exact=True)
    r = eta - o.apply_D(phi, 0.12, 1.0)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(eta)


@pytest.mark.parametrize("s", [0, 1])
def test_ras_equation2_identity(s):
    """With exact domain solves, Algorithm 1 computes
    K_RAS eta = S sum_{j<NRAS} (1 - D S)^j eta,
    S = sum_i R_i D_{Omega'_i}^{-1} P_i (dense construction)."""
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    block = (2, 2, 2, 2)
    V = I.volume(dims)
    D = R.dirac_dense(U, dims, 0.12, 1.0)
    nb, ev = o.decomp(block, s)
    S = np.zeros_like(D)
    for blk in range(nb):
        sites = o.block_sites(block, s, blk)
        ix = site_ix(sites)
        inv = np.linalg.inv(D[np.ix_(ix, ix)])
        own = o.block_sites(block, 0, blk)
        own_pos = np.array([np.where(sites == x)[0][0] for x in own])
        rows = site_ix(own)
        S[np.ix_(rows, ix)] = inv[site_ix(own_pos)]
    eta = I.gaussian_source(dims, 2).reshape(-1)
    for n_ras in (1, 2, 3):
        K = np.zeros_like(D)
        T = np.eye(12 * V) - D @ S
        P = np.eye(12 * V)
        for j in range(n_ras):
            K += S @ P
            P = T @ P
        phi = o.ras(eta.reshape(V, 4, 3), 0.12, 1.0, block, s, n_ras, 0, exact=True).reshape(-1)
        assert np.linalg.norm(phi - K @ eta) < 1e-11 * np.linalg.norm(K @ eta)


@pytest.mark.parametrize("s", [0, 1])
def test_ras_exact_block_invariant(s):
    """After one sweep with exact domain solves, eta - D phi vanishes on every
    site whose 8 neighbours lie in its own Omega_i."""
    dims = (9, 2, 2, 2) if s == 0 else (9, 4, 4, 4)
    block = (3, 2, 2, 2) if s == 0 else (3, 4, 4, 4)
    U, o = setup(dims)
    V = I.volume(dims)
    eta = I.gaussian_source(dims, 2)
    phi = o.ras(eta, 0.12, 1.0, block, s, 1, 0, exact=True)
    r = (eta - o.apply_D(phi, 0.12, 1.0)).reshape(V, 12)
    interior = []
    for x in range(V):
        c = [x % dims[0], x // dims[0] % dims[1], x // (dims[0] * dims[1]) % dims[2], x // (dims[0] * dims[1] * dims[2])]
        ok = True
        for mu in range(4):
            if block[mu] < dims[mu]:
                l = c[mu] % block[mu]
                if l == 0 or l == block[mu] - 1:
                    ok = False
        interior.append(ok)
    interior = np.array(interior)
    assert interior.sum() > 0
    assert np.abs(r[interior]).max() < 1e-12 * np.abs(eta).max()
    assert np.abs(r[~interior]).max() > 1e-3


def test_ras_improves_with_sweeps_and_iterations():
    dims = (8, 4, 4, 4)
    U, o = setup(dims)
    eta = I.gaussian_source(dims, 2)
    res = {}
    for n_ras, nd in [(1, 2), (1, 6), (3, 6)]:
        phi = o.ras(eta, 0.12, 1.0, (4, 4, 4, 4), 0, n_ras, nd)
        res[(n_ras, nd)] = np.linalg.norm(eta - o.apply_D(phi, 0.12, 1.0)) / np.linalg.norm(eta)
    assert res[(1, 6)] < res[(1, 2)] < 1
    assert res[(3, 6)] < res[(1, 6)]


@pytest.mark.parametrize("use_ras", [True, False])
def test_nested_solver_true_residual(use_ras):
    dims = (8, 4, 4, 4)
    U, o = setup(dims)
    eta = I.gaussian_source(dims, 2)
    phi, info = o.nested(eta, 0.12, 1.0, tol=1e-10, tol_inner=1e-3, ras=use_ras, block=(4, 4, 4, 4), s=1,
                         n_ras=3, n_dominv=4)
    assert info["converged"]
    r = eta - o.apply_D(phi, 0.12, 1.0)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(eta) * 1.5
