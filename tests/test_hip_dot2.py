"""GPU parity of the on-chip MR domain steps with binary16 operands
(WCL_ARITH_DOT2, FP16 storage) against the FP64 oracle's RAS (Algorithm 1,
Eq. (2)) and nested solve (Sec. 3), through the C ABI.

The binary16-operand steps are an approximation of the same preconditioner:
K_RAS is compared with the oracle to the tolerance of FP16 storage, and the
nested solve must still reach the FP64 true residual.  The per-domain
power-of-two scaling makes the preconditioner exactly homogeneous:
K(2^k r) = 2^k K(r) bit for bit, also where 2^k r itself is far outside the
binary16 range."""
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


FUSED_CASES = [
    ((8, 8, 8, 8), (4, 4, 4, 4), 0, 3, 4),     # the tuned shape, no overlap (boundary residual update)
    ((8, 8, 8, 8), (2, 2, 2, 2), 1, 3, 4),     # overlap: full residual update
    ((4, 4, 4, 8), (4, 4, 4, 2), 1, 2, 3),     # domain spans x, y, z (periodic inside)
    ((8, 8, 8, 8), (4, 4, 4, 4), 0, 4, 3),     # 4 sweeps: buffers reused
    ((8, 8, 8, 8), (2, 2, 2, 2), 1, 4, 2),
    ((12, 8, 8, 4), (4, 4, 4, 4), 0, 2, 6),    # ragged: 3 x 2 x 2 x 1 domains, 6 MR steps
]


@pytest.mark.parametrize("dims,block,s,n_ras,nd", FUSED_CASES)
def test_ras_dot2_matches_oracle(W, ctx, dims, block, s, n_ras, nd):
    U, lat = make(W, ctx, dims, bc=(1, 1, 1, -1))
    o = Oracle(dims, U, bc=(1, 1, 1, -1))
    r = I.gaussian_source(dims, 6)
    rd = lat.pack(r, W.F32)
    ras = W.RasParams.make(block=block, s=s, n_ras=n_ras, n_dominv=nd, storage=W.F16, arith=W.ARITH_DOT2)
    v = lat.empty(W.F32)
    lat.ras_precondition(ras, 0.124, 1.0, rd, v)
    got = lat.unpack(v, W.F32)
    ref = o.ras(r, 0.124, 1.0, block, s, n_ras, nd)
    e = rel_err(got, ref)
    # the FP32-arithmetic steps on the same FP16 storage
    ras32 = W.RasParams.make(block=block, s=s, n_ras=n_ras, n_dominv=nd, storage=W.F16)
    v2 = lat.empty(W.F32)
    lat.ras_precondition(ras32, 0.124, 1.0, rd, v2)
    e2 = rel_err(got, lat.unpack(v2, W.F32))
    print(f"dot2 RAS rel err vs oracle {e:.2e}, vs FP32-arithmetic steps {e2:.2e}")
    assert np.isfinite(got).all()
    # measured 1.3e-4 .. 2.7e-4 for both on these cases
    assert e <= 2e-3
    assert e2 <= 2e-3
    lat.close()


@pytest.mark.parametrize("k", [-40, -20, 0, 20, 40])
def test_ras_dot2_homogeneous(W, ctx, k):
    """K(2^k r) == 2^k K(r) bit for bit: the domain scaling absorbs the
    magnitude (2^40 |r| overflows binary16, 2^-40 |r| flushes it to zero)."""
    dims = (8, 8, 8, 8)
    _, lat = make(W, ctx, dims)
    r = I.gaussian_source(dims, 3)
    ras = W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=W.F16, arith=W.ARITH_DOT2)
    v0 = lat.empty(W.F32)
    lat.ras_precondition(ras, 0.125, 1.0, lat.pack(r, W.F32), v0)
    vk = lat.empty(W.F32)
    lat.ras_precondition(ras, 0.125, 1.0, lat.pack(r * 2.0 ** k, W.F32), vk)
    a, b = lat.unpack(v0, W.F32), lat.unpack(vk, W.F32)
    assert np.isfinite(b).all() and np.abs(a).max() > 0
    assert np.array_equal(b, a * 2.0 ** k)
    lat.close()


def test_ras_dot2_zero_and_point_sources(W, ctx):
    """A zero right-hand side gives zero (no 0/0 in the scaling); a point
    source leaves every domain but one at zero."""
    dims = (8, 8, 8, 8)
    U, lat = make(W, ctx, dims)
    ras = W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=2, n_dominv=4, storage=W.F16, arith=W.ARITH_DOT2)
    z = np.zeros((lat.V, 4, 3), np.complex128)
    v = lat.empty(W.F32)
    lat.ras_precondition(ras, 0.125, 1.0, lat.pack(z, W.F32), v)
    assert not lat.unpack(v, W.F32).any()
    _, eta = I.point_sources(dims, 3)
    lat.ras_precondition(ras, 0.125, 1.0, lat.pack(eta[4], W.F32), v)
    got = lat.unpack(v, W.F32)
    ref = Oracle(dims, U).ras(eta[4], 0.125, 1.0, (4, 4, 4, 4), 0, 2, 4)
    assert np.isfinite(got).all()
    assert rel_err(got, ref) <= 5e-3
    lat.close()


def test_ras_dot2_multi_rhs_equals_single(W, ctx):
    dims = (8, 8, 8, 8)
    _, lat = make(W, ctx, dims)
    r = I.gaussian_source(dims, 8, nrhs=3)
    r[1] *= 1e-9   # a much smaller rhs in the same batch: each (domain, rhs) has its own scale
    ras = W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=W.F16, arith=W.ARITH_DOT2)
    v = lat.empty(W.F32, 3)
    lat.ras_precondition(ras, 0.12, 1.0, lat.pack(r, W.F32, 3), v, nrhs=3)
    many = lat.unpack(v, W.F32, 3)
    for k in range(3):
        v1 = lat.empty(W.F32)
        lat.ras_precondition(ras, 0.12, 1.0, lat.pack(r[k], W.F32), v1)
        assert np.array_equal(lat.unpack(v1, W.F32), many[k]), k
    lat.close()


def test_ras_dot2_noalloc_equals_allocating(W, ctx):
    dims = (8, 8, 8, 8)
    _, lat = make(W, ctx, dims)
    r = lat.pack(I.gaussian_source(dims, 5), W.F32)
    ras = W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=W.F16, arith=W.ARITH_DOT2)
    v1, v2 = lat.empty(W.F32), lat.empty(W.F32)
    lat.ras_precondition(ras, 0.125, 1.0, r, v1)
    lat.ras_precondition_noalloc(ras, 0.125, 1.0, r, v2)
    assert np.array_equal(lat.unpack(v1, W.F32), lat.unpack(v2, W.F32))
    lat.close()


@pytest.mark.parametrize("dims,block,s", [((8, 8, 8, 8), (4, 4, 4, 4), 0), ((8, 8, 8, 8), (2, 2, 2, 2), 1),
                                          ((16, 8, 8, 8), (4, 4, 4, 4), 0)])
def test_nested_dot2_true_residual(W, ctx, dims, block, s):
    kappa, csw = 0.125, 1.0
    U, lat = make(W, ctx, dims)
    eta = I.gaussian_source(dims, 2)
    p = W.SolverParams.make(ras=W.RasParams.make(block=block, s=s, n_ras=3, n_dominv=4, storage=W.F16,
                                                 arith=W.ARITH_DOT2))
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_nested(p, kappa, csw, lat.pack(eta, W.F64), phi)
    sol = lat.unpack(phi, W.F64)
    res = np.linalg.norm(eta - Oracle(dims, U).apply_D(sol, kappa, csw)) / np.linalg.norm(eta)
    print(f"{dims} block={block} s={s} dot2: {st}, oracle true residual {res:.2e}")
    assert st["converged"] == 1
    assert res <= 1e-10
    assert abs(st["true_resid"] - res) <= 1e-12
    lat.close()


@pytest.mark.parametrize("kw", [dict(storage=1), dict(storage=2, kernel=2), dict(storage=2, block_solver=1),
                                dict(storage=2, schwarz=2), dict(storage=2, s=1), dict(storage=2, arith=2)])
def test_dot2_rejects_what_it_cannot_run(W, ctx, kw):
    """FP32 storage, the split path, the other domain solvers or Schwarz
    iterations, an extended domain over 256 sites (4^4 with s = 1) and an
    unknown arithmetic are errors, not silent fallbacks."""
    dims = (8, 8, 8, 8)
    _, lat = make(W, ctx, dims)
    args = dict(block=(4, 4, 4, 4), s=0, n_ras=2, n_dominv=2, arith=W.ARITH_DOT2)
    args.update(kw)
    ras = W.RasParams.make(**args)
    with pytest.raises(W.WclError) as e:
        lat.ras_precondition(ras, 0.12, 1.0, lat.zeros(W.F32), lat.empty(W.F32))
    assert e.value.code == W.EINVAL
    lat.close()


def test_nested_dot2_batch_equals_single(W, ctx):
    """A batched dot2 solve (a Gaussian, a point and another Gaussian source)
    gives every rhs bitwise its single-rhs solution, each to an oracle true
    residual <= 1e-10."""
    dims = (8, 8, 8, 8)
    kappa, csw = 0.125, 1.0
    U, lat = make(W, ctx, dims)
    _, pts = I.point_sources(dims, 3)
    eta = np.stack([I.gaussian_source(dims, 2), pts[4], I.gaussian_source(dims, 9)])
    p = W.SolverParams.make(ras=W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=W.F16,
                                                 arith=W.ARITH_DOT2))
    phi = lat.zeros(W.F64, 3)
    rc, st = lat.solve_nested(p, kappa, csw, lat.pack(eta, W.F64, 3), phi, nrhs=3)
    sols = lat.unpack(phi, W.F64, 3)
    o = Oracle(dims, U)
    for k in range(3):
        res = np.linalg.norm(eta[k] - o.apply_D(sols[k], kappa, csw)) / np.linalg.norm(eta[k])
        assert res <= 1e-10, (k, res)
        phi1 = lat.zeros(W.F64)
        lat.solve_nested(p, kappa, csw, lat.pack(eta[k], W.F64), phi1)
        assert np.array_equal(lat.unpack(phi1, W.F64), sols[k]), k
    lat.close()
