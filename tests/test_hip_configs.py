"""GPU solves at the benchmark's own sizes, each result checked by the FP64
oracle's operator (true residual |eta - D phi| / |eta| recomputed on the host):
the 32^4 FP16-storage solve, the 12 point sources on 16^3x32, the paper's
x-only split at 1e-14 (Sec. 4-5), the per-category timers, and the singular
free-field operator at kappa = 1/8 (a failure path)."""
import numpy as np
import pytest

from oracle import Oracle
from paper_1011_3318_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    from paper_1011_3318_amd import wcl
    return wcl


@pytest.fixture(scope="module")
def ctx(W):
    c = W.Context(0)
    yield c
    c.close()


def oracle_resid(dims, U, eta, sol, kappa, csw):
    o = Oracle(dims, U, precompute_clover=False)
    return float(np.linalg.norm(eta - o.apply_D(sol, kappa, csw)) / np.linalg.norm(eta))


@pytest.mark.parametrize("eps,nd,tol_inner", [(0.3, 5, 1e-5), (1.0, 3, 1e-4)])
def test_solve_32x4_f16(W, ctx, eps, nd, tol_inner):
    """32^4, kappa 0.125, c_sw 1.0, FP16-storage RAS on 4^4 domains (the
    benchmark's configuration and launch shape)."""
    dims = (32, 32, 32, 32)
    kappa, csw = 0.125, 1.0
    U = I.random_gauge(dims, eps, 1)
    eta = I.gaussian_source(dims, 2)
    lat = W.Lattice(ctx, dims)
    lat.upload_gauge(U)
    p = W.SolverParams.make(tol_inner=tol_inner,
                            ras=W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=nd, storage=W.F16))
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_nested(p, kappa, csw, lat.pack(eta, W.F64), phi)
    sol = lat.unpack(phi, W.F64)
    lat.close()
    res = oracle_resid(dims, U, eta, sol, kappa, csw)
    print(f"32^4 eps={eps}: {st}, oracle true residual {res:.3e}")
    assert st["converged"] == 1
    assert res <= 1e-10
    assert abs(st["true_resid"] - res) <= 1e-12


def test_point_sources_16x16x16x32(W, ctx):
    """The 12 spin-colour point sources on 16^3 x 32 in one batch."""
    dims = (16, 16, 16, 32)
    kappa, csw = 0.125, 1.0
    U = I.random_gauge(dims, 0.5, 1)
    x0, eta = I.point_sources(dims, 3)
    lat = W.Lattice(ctx, dims)
    lat.upload_gauge(U)
    p = W.SolverParams.make(ras=W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=W.F16))
    phi = lat.zeros(W.F64, 12)
    rc, st = lat.solve_nested(p, kappa, csw, lat.pack(eta, W.F64, 12), phi, nrhs=12)
    sols = lat.unpack(phi, W.F64, 12)
    lat.close()
    o = Oracle(dims, U)
    for k in range(12):
        res = np.linalg.norm(eta[k] - o.apply_D(sols[k], kappa, csw)) / np.linalg.norm(eta[k])
        assert res <= 1e-10, (k, res)


@pytest.mark.parametrize("s", [0, 1, 2])
def test_x_split_to_1e14(W, ctx, s):
    """The paper's decomposition (Sec. 4): the lattice split in x only, each
    domain extended by s sites up and down in x (d = 2s), NRAS 3, N_dominv 5,
    stopping at |eta - D phi|/|eta| < 1e-14 (Sec. 5), kappa 0.126, c_SW 1.0."""
    dims = (16, 8, 8, 8)
    kappa, csw = 0.126, 1.0
    U = I.random_gauge(dims, 0.3, 1)
    eta = I.gaussian_source(dims, 2)
    lat = W.Lattice(ctx, dims)
    lat.upload_gauge(U)
    p = W.SolverParams.make(tol_outer=1e-14, max_outer=200, max_inner=1000,
                            ras=W.RasParams.make(block=(2, 8, 8, 8), s=s, n_ras=3, n_dominv=5, storage=W.F32))
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_nested(p, kappa, csw, lat.pack(eta, W.F64), phi)
    sol = lat.unpack(phi, W.F64)
    lat.close()
    res = oracle_resid(dims, U, eta, sol, kappa, csw)
    print(f"x split s={s}: {st}, oracle true residual {res:.3e}")
    assert st["converged"] == 1
    assert res <= 1e-13


def test_timers_add_up(W, ctx):
    dims = (16, 16, 16, 32)
    U = I.random_gauge(dims, 0.5, 1)
    lat = W.Lattice(ctx, dims)
    lat.upload_gauge(U)
    e = lat.pack(I.gaussian_source(dims, 2), W.F64)
    p = W.SolverParams.make(timers=1, ras=W.RasParams.make(block=(4, 4, 4, 4), s=0, storage=W.F16))
    phi = lat.zeros(W.F64)
    _, st = lat.solve_nested(p, 0.125, 1.0, e, phi)
    parts = st["ms_dslash"] + st["ms_dominv"] + st["ms_blas"] + st["ms_host"]
    print({k: st[k] for k in ("ms_total", "ms_dslash", "ms_dominv", "ms_blas", "ms_host")})
    assert st["ms_dslash"] > 0 and st["ms_dominv"] > 0 and st["ms_blas"] > 0
    assert abs(parts - st["ms_total"]) <= 0.05 * st["ms_total"] + 0.05
    # without timers the categories stay zero and the solution is the same
    phi2 = lat.zeros(W.F64)
    p.timers = 0
    _, st2 = lat.solve_nested(p, 0.125, 1.0, e, phi2)
    assert st2["ms_dslash"] == 0 and st2["ms_dominv"] == 0
    assert np.array_equal(lat.unpack(phi, W.F64), lat.unpack(phi2, W.F64))
    lat.close()


def test_free_field_zero_mode_fails_cleanly(W, ctx):
    """U = 1 and kappa = 1/8: the constant mode is an exact zero mode of D, so
    a Gaussian source has no solution.  Both solvers stop at their limits and
    report failure (no hang, a finite best iterate, stats filled)."""
    dims = (4, 4, 4, 4)
    lat = W.Lattice(ctx, dims)
    lat.upload_gauge(I.unit_gauge(dims))
    eta = I.gaussian_source(dims, 2)
    e = lat.pack(eta, W.F64)
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_bicgstab_f64(1e-10, 300, 0.125, 1.0, e, phi, raise_on_notconv=False)
    assert rc in (W.ENOTCONV, W.EBREAKDOWN) or (rc == 0 and st["true_resid"] > 1e-10)
    assert np.isfinite(lat.unpack(phi, W.F64)).all()
    p = W.SolverParams.make(max_outer=20, max_inner=50, max_restarts=2,
                            ras=W.RasParams.make(block=(2, 2, 2, 2), s=0))
    try:
        rc, st = lat.solve_nested(p, 0.125, 1.0, e, phi, raise_on_notconv=False)
    except W.WclError as err:
        rc = err.code
        st = None
    assert rc in (W.ENOTCONV, W.EBREAKDOWN)
    if st is not None:
        assert st["converged"] == 0 and st["outer_iters"] >= 1
    lat.close()
