"""GPU parity of the RAS domain operator, K_RAS and the solvers against the
FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from helpers import rel_err
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


def make(W, ctx, dims, eps=0.5, seed=1, bc=(1, 1, 1, 1)):
    U = I.random_gauge(dims, eps, seed)
    lat = W.Lattice(ctx, dims, bc)
    lat.upload_gauge(U)
    return U, lat


BLOCK_CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2), 0),
    ((4, 4, 4, 4), (2, 2, 2, 2), 1),      # e = 4 = L: extended domain wraps onto itself
    ((8, 4, 4, 8), (2, 4, 4, 4), 1),      # x split only in x... and t
    ((8, 8, 8, 8), (4, 4, 4, 4), 1),
    ((6, 4, 10, 4), (6, 4, 10, 4), 1),    # one domain = whole lattice
    ((8, 4, 4, 4), (2, 4, 4, 4), 2),      # the paper's x-only split, d = 4
]


@pytest.mark.parametrize("storage", [1, 2])
@pytest.mark.parametrize("dims,block,s", BLOCK_CASES)
def test_domain_operator(W, ctx, dims, block, s, storage):
    U, lat = make(W, ctx, dims, bc=(1, 1, 1, -1))
    o = Oracle(dims, U, bc=(1, 1, 1, -1))
    psi = I.gaussian_source(dims, 4)
    x = lat.pack(psi, W.F32)
    ras = W.RasParams.make(block=block, s=s, storage=storage)
    got = lat.apply_D_blocks(ras, 0.125, 1.2, x)
    nb, ev = o.decomp(block, s)
    assert got.shape[:2] == (nb, ev)
    tol = 2e-6 if storage == 1 else 5e-3
    for blk in range(nb):
        sites = o.block_sites(block, s, blk)
        ref = o.block_apply(block, s, blk, psi[sites], 0.125, 1.2)
        assert rel_err(got[blk], ref) <= tol, blk
    lat.close()


RAS_CASES = [
    ((8, 8, 8, 8), (4, 4, 4, 4), 0, 3, 4),     # fused (ev = 256)
    ((8, 8, 8, 8), (2, 2, 2, 2), 1, 3, 4),     # fused, overlap (ev = 256)
    ((4, 4, 4, 8), (4, 4, 4, 2), 1, 2, 3),     # fused, domain spans x, y, z (periodic inside)
    ((8, 8, 8, 8), (4, 4, 4, 4), 1, 3, 4),     # split (ev = 1296)
    ((8, 4, 6, 4), (4, 2, 2, 4), 1, 2, 5),     # split
    ((16, 8, 8, 8), (8, 8, 8, 8), 1, 1, 3),    # split, the 8^4 domains of the 16^3x32 benchmark
    ((16, 16, 8, 8), (8, 8, 4, 4), 1, 2, 3),   # split; the residual update runs the x/y exchange D-apply
    ((8, 8, 8, 8), (4, 4, 4, 4), 0, 4, 3),     # fused, 4 sweeps: the v_j / rho_N buffers are reused
    ((8, 8, 8, 8), (2, 2, 2, 2), 1, 4, 2),     # fused, overlap, 4 sweeps: r_j buffers reused
]


@pytest.mark.parametrize("storage,tol", [(1, 1e-4), (2, 2e-2)])
@pytest.mark.parametrize("dims,block,s,n_ras,nd", RAS_CASES)
def test_ras_precondition(W, ctx, dims, block, s, n_ras, nd, storage, tol):
    U, lat = make(W, ctx, dims, bc=(1, 1, 1, -1))
    o = Oracle(dims, U, bc=(1, 1, 1, -1))
    r = I.gaussian_source(dims, 6)
    ras = W.RasParams.make(block=block, s=s, n_ras=n_ras, n_dominv=nd, storage=storage)
    rd = lat.pack(r, W.F32)
    v = lat.empty(W.F32)
    lat.ras_precondition(ras, 0.124, 1.0, rd, v)
    got = lat.unpack(v, W.F32)
    ref = o.ras(r, 0.124, 1.0, block, s, n_ras, nd)
    e = rel_err(got, ref)
    print(f"RAS rel err {e:.2e}")
    assert e <= tol
    # the split path computes the same operator
    ras_split = W.RasParams.make(block=block, s=s, n_ras=n_ras, n_dominv=nd, storage=storage,
                                 kernel=W.BLOCK_SPLIT)
    v2 = lat.empty(W.F32)
    lat.ras_precondition(ras_split, 0.124, 1.0, rd, v2)
    assert rel_err(lat.unpack(v2, W.F32), got) <= (1e-5 if storage == 1 else 5e-3)
    lat.close()


def test_ras_fused_rejects_large_domains(W, ctx):
    dims = (8, 8, 8, 8)
    _, lat = make(W, ctx, dims)
    ras = W.RasParams.make(block=(4, 4, 4, 4), s=1, kernel=W.BLOCK_FUSED)
    with pytest.raises(W.WclError) as e:
        lat.ras_precondition(ras, 0.12, 1.0, lat.zeros(W.F32), lat.empty(W.F32))
    assert e.value.code == W.EINVAL
    lat.close()


@pytest.mark.parametrize("s", [0, 1])
def test_ras_multi_rhs_equals_single(W, ctx, s):
    dims = (8, 8, 8, 8)
    U, lat = make(W, ctx, dims)
    r = I.gaussian_source(dims, 8, nrhs=3)
    ras = W.RasParams.make(block=(4, 4, 4, 4), s=s, n_ras=3, n_dominv=4)
    v = lat.empty(W.F32, 3)
    lat.ras_precondition(ras, 0.12, 1.0, lat.pack(r, W.F32, 3), v, nrhs=3)
    many = lat.unpack(v, W.F32, 3)
    for k in range(3):
        v1 = lat.empty(W.F32)
        lat.ras_precondition(ras, 0.12, 1.0, lat.pack(r[k], W.F32), v1)
        assert np.array_equal(lat.unpack(v1, W.F32), many[k])
    lat.close()


def test_plain_bicgstab_anchor(W, ctx):
    """4^4, eps=0.5 seed 1, kappa=0.12, c_sw=1, eta seed 2: the oracle takes
    32 iterations; the GPU FP64 solver follows the same recursion."""
    dims = (4, 4, 4, 4)
    U, lat = make(W, ctx, dims)
    eta = I.gaussian_source(dims, 2)
    e = lat.pack(eta, W.F64)
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_bicgstab_f64(1e-10, 1000, 0.12, 1.0, e, phi)
    sol = lat.unpack(phi, W.F64)
    o = Oracle(dims, U)
    ref, info = o.bicgstab(eta, 0.12, 1.0, tol=1e-10)
    assert abs(st["outer_iters"] - info["iters"]) <= 1
    assert rel_err(sol, ref) < 1e-8
    res = np.linalg.norm(eta - o.apply_D(sol, 0.12, 1.0)) / np.linalg.norm(eta)
    assert res <= 1e-10
    assert abs(st["true_resid"] - res) < 1e-12
    lat.close()


SOLVE_CASES = [
    # dims, block, s, storage, precond
    ((8, 8, 8, 8), (4, 4, 4, 4), 0, 1, 1),
    ((8, 8, 8, 8), (4, 4, 4, 4), 1, 1, 1),
    ((8, 8, 8, 8), (4, 4, 4, 4), 0, 2, 1),
    ((8, 8, 8, 8), (4, 4, 4, 4), 0, 1, 0),
    ((16, 16, 16, 32), (8, 8, 8, 8), 0, 1, 1),
    ((16, 16, 16, 32), (8, 8, 8, 8), 1, 1, 1),
    ((16, 16, 16, 32), (4, 4, 4, 4), 0, 2, 1),   # the benchmark's tuned configuration (on-chip domains)
]


@pytest.mark.parametrize("dims,block,s,storage,precond", SOLVE_CASES)
def test_nested_solve_true_residual(W, ctx, dims, block, s, storage, precond):
    kappa, csw = 0.125, 1.0
    U, lat = make(W, ctx, dims)
    eta = I.gaussian_source(dims, 2)
    p = W.SolverParams.make(precond=precond,
                            ras=W.RasParams.make(block=block, s=s, n_ras=3, n_dominv=4, storage=storage))
    e = lat.pack(eta, W.F64)
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_nested(p, kappa, csw, e, phi)
    sol = lat.unpack(phi, W.F64)
    o = Oracle(dims, U)
    res = np.linalg.norm(eta - o.apply_D(sol, kappa, csw)) / np.linalg.norm(eta)
    print(f"{dims} block={block} s={s} storage={storage} precond={precond}: {st}, oracle true residual {res:.2e}")
    assert st["converged"] == 1
    assert res <= 1e-10
    assert abs(st["true_resid"] - res) <= 1e-12
    lat.close()


def test_nested_multi_rhs_point_sources(W, ctx):
    """12 spin-colour point sources at one site, batched; each result equals
    the single-rhs solve."""
    dims = (8, 8, 8, 8)
    kappa, csw = 0.125, 1.0
    U, lat = make(W, ctx, dims)
    x0, eta = I.point_sources(dims, 3)
    p = W.SolverParams.make(ras=W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4))
    e = lat.pack(eta, W.F64, 12)
    phi = lat.zeros(W.F64, 12)
    rc, st = lat.solve_nested(p, kappa, csw, e, phi, nrhs=12)
    sols = lat.unpack(phi, W.F64, 12)
    o = Oracle(dims, U)
    for k in range(12):
        res = np.linalg.norm(eta[k] - o.apply_D(sols[k], kappa, csw)) / np.linalg.norm(eta[k])
        assert res <= 1e-10, (k, res)
    for k in (0, 7):
        phi1 = lat.zeros(W.F64)
        lat.solve_nested(p, kappa, csw, lat.pack(eta[k], W.F64), phi1)
        assert np.array_equal(lat.unpack(phi1, W.F64), sols[k])
    lat.close()


def test_nested_batch_with_early_and_zero_rhs(W, ctx):
    """A batch whose right-hand sides finish at different iterations (a zero
    source at once, a point source and a Gaussian source later): the kernels
    skip the finished ones, and every result still equals its single-rhs solve
    bit for bit."""
    dims = (8, 8, 8, 8)
    kappa, csw = 0.125, 1.0
    U, lat = make(W, ctx, dims)
    eta = np.stack([I.gaussian_source(dims, 2), np.zeros((lat.V, 4, 3), np.complex128),
                    I.point_sources(dims, 3)[1][5]])
    p = W.SolverParams.make(ras=W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=2, n_dominv=4, storage=W.F16))
    phi = lat.zeros(W.F64, 3)
    rc, st = lat.solve_nested(p, kappa, csw, lat.pack(eta, W.F64, 3), phi, nrhs=3)
    sols = lat.unpack(phi, W.F64, 3)
    assert not sols[1].any()
    o = Oracle(dims, U)
    for k in (0, 2):
        res = np.linalg.norm(eta[k] - o.apply_D(sols[k], kappa, csw)) / np.linalg.norm(eta[k])
        assert res <= 1e-10, (k, res)
        phi1 = lat.zeros(W.F64)
        lat.solve_nested(p, kappa, csw, lat.pack(eta[k], W.F64), phi1)
        assert np.array_equal(lat.unpack(phi1, W.F64), sols[k]), k
    lat.close()


def test_nested_deterministic(W, ctx):
    dims = (8, 8, 8, 8)
    U, lat = make(W, ctx, dims)
    eta = I.gaussian_source(dims, 2)
    p = W.SolverParams.make(ras=W.RasParams.make(block=(4, 4, 4, 4), s=1))
    e = lat.pack(eta, W.F64)
    out = []
    for _ in range(2):
        phi = lat.zeros(W.F64)
        lat.solve_nested(p, 0.125, 1.0, e, phi)
        out.append(lat.unpack(phi, W.F64))
    assert np.array_equal(out[0], out[1])
    lat.close()


def test_solver_error_paths(W, ctx):
    dims = (8, 8, 8, 8)
    U, lat = make(W, ctx, dims)
    p = W.SolverParams.make(ras=W.RasParams.make(block=(4, 4, 4, 4)))
    # eta = 0 -> phi = 0 at once
    z = lat.zeros(W.F64)
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_nested(p, 0.125, 1.0, z, phi)
    assert rc == 0 and not lat.unpack(phi, W.F64).any()
    # NaN source
    eta = I.gaussian_source(dims, 2)
    bad = eta.copy()
    bad[5, 1, 2] = np.nan
    with pytest.raises(W.WclError) as e:
        lat.solve_nested(p, 0.125, 1.0, lat.pack(bad, W.F64), phi)
    assert e.value.code == W.EINVAL
    # iteration limit: best iterate and stats returned
    p1 = W.SolverParams.make(max_outer=1, max_restarts=0, ras=W.RasParams.make(block=(4, 4, 4, 4)))
    rc, st = lat.solve_nested(p1, 0.125, 1.0, lat.pack(eta, W.F64), phi, raise_on_notconv=False)
    assert rc == W.ENOTCONV and st["converged"] == 0 and 0 < st["true_resid"] < 1
    # block shape that does not tile the lattice
    with pytest.raises(W.WclError) as e:
        lat.solve_nested(W.SolverParams.make(ras=W.RasParams.make(block=(3, 4, 4, 4))), 0.125, 1.0,
                         lat.pack(eta, W.F64), phi)
    assert e.value.code == W.EINVAL
    lat.close()


def test_autotune_and_cache(W, ctx, tmp_path):
    dims = (8, 8, 8, 16)
    U, lat = make(W, ctx, dims)
    eta = I.gaussian_source(dims, 2)
    e = lat.pack(eta, W.F64)
    base = W.SolverParams.make()
    cache = str(tmp_path / "tune.jsonl")
    best, ms = W.autotune(lat, base, 0.125, 1.0, e, cache_path=cache)
    assert ms > 0 and best.precond == W.PRECOND_RAS
    assert tuple(best.ras.block) in {(4, 4, 4, 4), (4, 4, 4, 8), (8, 8, 8, 8)}
    # the tuned parameters solve to tolerance
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_nested(best, 0.125, 1.0, e, phi)
    res = np.linalg.norm(eta - Oracle(dims, U).apply_D(lat.unpack(phi, W.F64), 0.125, 1.0)) / np.linalg.norm(eta)
    assert res <= 1e-10
    # second call reads the cache
    lines = open(cache).read().splitlines()
    assert len(lines) == 1
    best2, ms2 = W.autotune(lat, base, 0.125, 1.0, e, cache_path=cache)
    assert tuple(best2.ras.block) == tuple(best.ras.block) and best2.ras.n_dominv == best.ras.n_dominv
    assert ms2 == pytest.approx(ms, rel=1e-3)
    assert len(open(cache).read().splitlines()) == 1
    lat.close()


def test_autotune_two_sources_and_arith(W, ctx):
    """Tuning on two sources (nsrc = 2, stored one after the other) picks
    parameters that solve a third source to tolerance; the cache line keeps
    the arithmetic of the MR steps; nsrc outside 1..16 is rejected."""
    dims = (8, 8, 8, 16)
    U, lat = make(W, ctx, dims)
    srcs = np.stack([I.gaussian_source(dims, 7), I.gaussian_source(dims, 8)])
    et = lat.pack(srcs, W.F64, 2)
    base = W.SolverParams.make()
    best, ms = W.autotune(lat, base, 0.125, 1.0, et, 1, storage=W.F16, nsrc=2)
    assert ms > 0 and best.ras.storage == W.F16 and best.ras.arith in (W.ARITH_FP32, W.ARITH_DOT2)
    eta = I.gaussian_source(dims, 2)
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_nested(best, 0.125, 1.0, lat.pack(eta, W.F64), phi)
    res = np.linalg.norm(eta - Oracle(dims, U).apply_D(lat.unpack(phi, W.F64), 0.125, 1.0)) / np.linalg.norm(eta)
    assert res <= 1e-10
    for bad in (0, 17):
        with pytest.raises(W.WclError) as e:
            W.autotune(lat, base, 0.125, 1.0, et, 1, nsrc=bad)
        assert e.value.code == W.EINVAL
    lat.close()
