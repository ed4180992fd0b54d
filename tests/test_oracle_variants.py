"""Pins of the oracle's other readings of the domain solver and of the Schwarz
iteration (Sec. 1-2), and of the even-odd reduction, against dense linear
algebra built independently of the oracle (tests/dense_ref.py, NumPy):

* the site term's inverse A(x)^{-1} = (1 + c_sw kappa C(x))^{-1};
* block Jacobi: n steps from zero equal the truncated Neumann series
  sum_{k<n} (1 - M^{-1} D)^k M^{-1} b, M = the 12x12 diagonal blocks of D_{Omega'};
* truncated BiCGStab: its first iterate satisfies BiCGStab's two defining
  conditions (the BiCG Galerkin condition <b, s> = 0 and the minimal-residual
  step r_1 orthogonal to D s), the identity operator is solved in one
  iteration, a zero right-hand side stays zero, many iterations give the
  dense block solution;
* additive Schwarz with exact domain solves: phi = S sum_{j<n} (1 - D S)^j eta,
  S = sum_i P_i^T D_{Omega'_i}^{-1} P_i (whole extended solutions, overlaps add);
* multiplicative Schwarz with exact domain solves: the error is multiplied by
  E = (1 - S_1 D)(1 - S_0 D) per sweep, S_c the restricted sum over the domains
  of colour c (parity of the block coordinates);
* even-odd: Dhat = D_ee - D_eo D_oo^{-1} D_oe, and the reduced solve with the
  odd-site reconstruction solves D phi = eta.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1011_3318_amd import inputs as I
import dense_ref as R

KAPPA, CSW = 0.12, 1.1


def setup(dims, eps=0.5, seed=1):
    U = I.random_gauge(dims, eps, seed)
    return U, Oracle(dims, U)


def site_ix(sites):
    return (12 * np.asarray(sites)[:, None] + np.arange(12)[None]).reshape(-1)


def test_site_term_inverse():
    dims = (4, 4, 2, 2)
    U, o = setup(dims)
    V = I.volume(dims)
    Cl = R.clover_dense(U, dims)
    Ainv = o.site_term_inverse(KAPPA, CSW)
    for x in range(V):
        A = np.eye(12) + CSW * KAPPA * Cl[x]
        assert np.abs(Ainv[x] @ A - np.eye(12)).max() < 1e-13
        # chiral basis: A and its inverse are two 6x6 blocks
        assert np.abs(Ainv[x][:6, 6:]).max() < 1e-14 and np.abs(Ainv[x][6:, :6]).max() < 1e-14
    assert np.abs(o.site_term_inverse(KAPPA, 0.0) - np.eye(12)).max() == 0


def block_dense(U, dims, o, block, s, blk, kappa=KAPPA, csw=CSW):
    sites = o.block_sites(block, s, blk)
    D = R.dirac_dense(U, dims, kappa, csw)
    ix = site_ix(sites)
    return sites, D[np.ix_(ix, ix)]


@pytest.mark.parametrize("n", [1, 2, 5])
def test_jacobi_is_truncated_neumann_series(n):
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    block, s, blk = (2, 2, 2, 2), 1, 3
    sites, Db = block_dense(U, dims, o, block, s, blk)
    m = len(sites)
    M = np.zeros_like(Db)
    for k in range(m):
        sl = slice(12 * k, 12 * k + 12)
        M[sl, sl] = Db[sl, sl]
    Minv = np.linalg.inv(M)
    b = I.gaussian_source(dims, 4)[sites].reshape(-1)
    T = np.eye(12 * m) - Minv @ Db
    want = np.zeros_like(b)
    term = Minv @ b
    for _ in range(n):
        want += term
        term = T @ term
    got = o.block_solve(block, s, blk, b, KAPPA, CSW, 1, n).reshape(-1)
    assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want)


def test_jacobi_without_hopping_is_exact_in_one_step():
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    block, s, blk = (2, 2, 2, 2), 0, 1
    sites, Db = block_dense(U, dims, o, block, s, blk, kappa=0.0)
    b = I.gaussian_source(dims, 4)[sites].reshape(-1)
    got = o.block_solve(block, s, blk, b, 0.0, CSW, 1, 1).reshape(-1)
    assert np.abs(got - b).max() < 1e-15   # kappa = 0: D = A = 1


def test_truncated_bicgstab_first_iteration_conditions():
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    block, s, blk = (2, 2, 2, 2), 1, 6
    sites, Db = block_dense(U, dims, o, block, s, blk)
    b = I.gaussian_source(dims, 5)[sites].reshape(-1)
    x1 = o.block_solve(block, s, blk, b, KAPPA, CSW, 2, 1).reshape(-1)
    # x1 lies in span{b, s} with s = b - alpha D b; write x1 = c0 b + c1 D b
    K = np.stack([b, Db @ b], axis=1)
    c, *_ = np.linalg.lstsq(K, x1, rcond=None)
    assert np.linalg.norm(K @ c - x1) < 1e-12 * np.linalg.norm(x1)
    # x1 = alpha b + omega s = (alpha + omega) b - omega alpha D b: solve
    # alpha + omega = c0, -alpha omega = c1 for (alpha, omega) and test the two
    # defining conditions for either root assignment
    disc = np.sqrt(c[0] ** 2 + 4 * c[1])
    ok = False
    for alpha in ((c[0] + disc) / 2, (c[0] - disc) / 2):
        omega = c[0] - alpha
        s_vec = b - alpha * (Db @ b)
        r1 = s_vec - omega * (Db @ s_vec)
        galerkin = abs(np.vdot(b, s_vec)) / (np.linalg.norm(b) * np.linalg.norm(s_vec))
        minres = abs(np.vdot(Db @ s_vec, r1)) / (np.linalg.norm(Db @ s_vec) * np.linalg.norm(r1))
        if galerkin < 1e-12 and minres < 1e-12:
            ok = True
    assert ok


def test_truncated_bicgstab_limits():
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    block, s, blk = (2, 2, 2, 2), 1, 2
    sites, Db = block_dense(U, dims, o, block, s, blk)
    b = I.gaussian_source(dims, 6)[sites].reshape(-1)
    # many iterations: the dense block solution
    x = o.block_solve(block, s, blk, b, KAPPA, CSW, 2, 80).reshape(-1)
    xe = np.linalg.solve(Db, b)
    assert np.linalg.norm(x - xe) < 1e-9 * np.linalg.norm(xe)
    # identity operator (kappa = 0, c_sw = 0): one iteration is exact
    x1 = o.block_solve(block, s, blk, b, 0.0, 0.0, 2, 1).reshape(-1)
    assert np.abs(x1 - b).max() < 1e-14
    # zero right-hand side: x stays zero through the guarded coefficients
    z = o.block_solve(block, s, blk, np.zeros_like(b), KAPPA, CSW, 2, 4)
    assert not z.any()


def dense_S(o, U, dims, D, block, s, restricted, colour=None):
    """sum over domains (of one colour) of P^T D_{Omega'}^{-1} P, restricted to
    the owned sites or over the whole extended domain."""
    nb, ev = o.decomp(block, s)
    nbs = [dims[m] // block[m] for m in range(4)]
    S = np.zeros_like(D)
    for blk in range(nb):
        bc, q = [], blk
        for m in range(4):
            bc.append(q % nbs[m])
            q //= nbs[m]
        if colour is not None and sum(bc) % 2 != colour:
            continue
        sites = o.block_sites(block, s, blk)
        ix = site_ix(sites)
        inv = np.linalg.inv(D[np.ix_(ix, ix)])
        if restricted:
            own = o.block_sites(block, 0, blk)
            pos = np.array([np.where(sites == x)[0][0] for x in own])
            S[np.ix_(site_ix(own), ix)] += inv[site_ix(pos)]
        else:
            S[np.ix_(ix, ix)] += inv
    return S


@pytest.mark.parametrize("s", [0, 1])
def test_additive_schwarz_identity(s):
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    block = (2, 2, 2, 2)
    V = I.volume(dims)
    D = R.dirac_dense(U, dims, KAPPA, CSW)
    S = dense_S(o, U, dims, D, block, s, restricted=False)
    eta = I.gaussian_source(dims, 2).reshape(-1)
    T = np.eye(12 * V) - D @ S
    for n in (1, 2):
        K = np.zeros_like(D)
        P = np.eye(12 * V)
        for _ in range(n):
            K += S @ P
            P = T @ P
        phi = o.schwarz(eta, KAPPA, CSW, block, s, n, 0, schwarz=1, exact=True).reshape(-1)
        assert np.linalg.norm(phi - K @ eta) < 1e-11 * np.linalg.norm(K @ eta)
    if s == 0:   # no overlap: additive = restricted additive
        a = o.schwarz(eta, KAPPA, CSW, block, 0, 2, 3, schwarz=1)
        r = o.schwarz(eta, KAPPA, CSW, block, 0, 2, 3, schwarz=0)
        assert np.abs(a - r).max() < 1e-14


@pytest.mark.parametrize("s", [0, 1])
def test_multiplicative_schwarz_error_propagation(s):
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    block = (2, 2, 2, 2)
    V = I.volume(dims)
    D = R.dirac_dense(U, dims, KAPPA, CSW)
    S0 = dense_S(o, U, dims, D, block, s, restricted=True, colour=0)
    S1 = dense_S(o, U, dims, D, block, s, restricted=True, colour=1)
    E = (np.eye(12 * V) - S1 @ D) @ (np.eye(12 * V) - S0 @ D)
    eta = I.gaussian_source(dims, 2).reshape(-1)
    xe = np.linalg.solve(D, eta)
    err = xe.copy()
    for n in (1, 2, 3):
        err = E @ err
        phi = o.schwarz(eta, KAPPA, CSW, block, s, n, 0, schwarz=2, exact=True).reshape(-1)
        assert np.linalg.norm(phi - (xe - err)) < 1e-10 * np.linalg.norm(xe)
    # one colour pass on a colouring where every domain has the same colour
    # would be the additive iteration; here both colours occur
    assert np.abs(S0).max() > 0 and np.abs(S1).max() > 0


@pytest.mark.parametrize("solver", [1, 2])
def test_inexact_domain_solvers_inside_ras_converge_to_exact(solver):
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    eta = I.gaussian_source(dims, 2)
    ex = o.schwarz(eta, KAPPA, CSW, (2, 2, 2, 2), 1, 2, 0, exact=True)
    n = 60 if solver == 2 else 200
    got = o.schwarz(eta, KAPPA, CSW, (2, 2, 2, 2), 1, 2, n, solver=solver)
    assert np.linalg.norm(got - ex) < 1e-8 * np.linalg.norm(ex)


def parity_ix(dims, p):
    V = I.volume(dims)
    par = []
    for x in range(V):
        c, q = [], x
        for L in dims:
            c.append(q % L)
            q //= L
        par.append(sum(c) % 2)
    sites = np.array([x for x in range(V) if par[x] == p])
    return sites, site_ix(sites)


def test_schur_complement_is_dense_identity():
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    D = R.dirac_dense(U, dims, KAPPA, CSW)
    es, e = parity_ix(dims, 0)
    os_, od = parity_ix(dims, 1)
    Dhat = D[np.ix_(e, e)] - D[np.ix_(e, od)] @ np.linalg.solve(D[np.ix_(od, od)], D[np.ix_(od, e)])
    psi = I.gaussian_source(dims, 3)
    got = o.apply_schur(psi, KAPPA, CSW)
    want = Dhat @ psi.reshape(-1)[e]
    assert np.linalg.norm(got.reshape(-1)[e] - want) < 1e-12 * np.linalg.norm(want)
    assert not got.reshape(-1)[od].any()


def test_even_odd_solve_solves_the_full_system():
    dims = (4, 4, 2, 4)
    U, o = setup(dims)
    eta = I.gaussian_source(dims, 2)
    phi, info = o.eo_solve(eta, KAPPA, CSW, tol=1e-12)
    assert info["converged"]
    xe = np.linalg.solve(R.dirac_dense(U, dims, KAPPA, CSW), eta.reshape(-1))
    assert np.linalg.norm(phi.reshape(-1) - xe) < 1e-10 * np.linalg.norm(xe)
    # the reduced system needs fewer iterations than the full one
    _, full = o.bicgstab(eta, KAPPA, CSW, tol=1e-12)
    assert info["iters"] < full["iters"]


def test_even_odd_needs_even_extents():
    dims = (3, 4, 2, 2)
    U, o = setup(dims)
    with pytest.raises(ValueError):
        o.apply_schur(I.gaussian_source(dims, 2), KAPPA, CSW)
