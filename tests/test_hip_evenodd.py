"""GPU parity of the even-odd reduction (the Schur complement on the even
sites with the per-site inverse of the two 6x6 site-term blocks) against the
FP64 oracle, and nested solves of the reduced system whose reconstructed
full solution the oracle checks."""
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


def site_parity(dims):
    """(x + y + z + t) mod 2 in the canonical host site order."""
    x, y, z, t = np.meshgrid(*[np.arange(L) for L in dims], indexing="ij")
    return ((x + y + z + t) % 2).transpose(3, 2, 1, 0).reshape(-1)


def make(W, ctx, dims, eps=0.5, seed=1, bc=(1, 1, 1, 1)):
    U = I.random_gauge(dims, eps, seed)
    lat = W.Lattice(ctx, dims, bc)
    lat.upload_gauge(U)
    return U, lat


SCHUR_CASES = [
    ((4, 4, 4, 4), (1, 1, 1, 1)),
    ((8, 4, 6, 4), (1, 1, 1, -1)),    # column cross-section 8 x 4 x 2, antiperiodic t
    ((2, 4, 4, 2), (1, 1, 1, 1)),     # extent 2: forward and backward neighbours coincide
    ((16, 8, 8, 8), (1, 1, 1, -1)),   # several tiles
]


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 1e-5)])
@pytest.mark.parametrize("dims,bc", SCHUR_CASES)
def test_schur_operator(W, ctx, dims, bc, prec, tol):
    U, lat = make(W, ctx, dims, bc=bc)
    o = Oracle(dims, U, bc=bc)
    psi = I.gaussian_source(dims, 4)
    kappa, csw = 0.126, 1.3
    out = lat.empty(prec)
    lat.apply_schur(prec, kappa, csw, lat.pack(psi, prec), out)
    got = lat.unpack(out, prec)
    ref = o.apply_schur(psi, kappa, csw)
    par = site_parity(dims)
    assert np.abs(got[par == 1]).max() == 0          # odd sites zero
    assert rel_err(got, ref) <= tol
    lat.close()


def test_schur_multi_rhs_equals_single(W, ctx):
    dims = (8, 8, 4, 4)
    U, lat = make(W, ctx, dims)
    psi = I.gaussian_source(dims, 5, nrhs=3)
    out = lat.empty(W.F32, 3)
    lat.apply_schur(W.F32, 0.12, 1.0, lat.pack(psi, W.F32, 3), out, nrhs=3)
    many = lat.unpack(out, W.F32, 3)
    for k in range(3):
        o1 = lat.empty(W.F32)
        lat.apply_schur(W.F32, 0.12, 1.0, lat.pack(psi[k], W.F32), o1)
        assert np.array_equal(lat.unpack(o1, W.F32), many[k])
    lat.close()


def test_schur_rejects_odd_extent_and_half_precision(W, ctx):
    _, lat = make(W, ctx, (5, 4, 4, 4))
    with pytest.raises(W.WclError) as e:
        lat.apply_schur(W.F32, 0.12, 1.0, lat.zeros(W.F32), lat.empty(W.F32))
    assert e.value.code == W.EINVAL
    p = W.SolverParams.make(precond=W.PRECOND_NONE, even_odd=1)
    with pytest.raises(W.WclError) as e:
        lat.solve_nested(p, 0.12, 1.0, lat.zeros(W.F64), lat.zeros(W.F64))
    assert e.value.code == W.EINVAL
    lat.close()
    _, lat = make(W, ctx, (4, 4, 4, 4))
    with pytest.raises(W.WclError) as e:
        lat.apply_schur(W.F16, 0.12, 1.0, lat.zeros(W.F16), lat.empty(W.F16))
    assert e.value.code == W.EINVAL
    # the Schwarz preconditioner is not combined with the reduced system
    p = W.SolverParams.make(precond=W.PRECOND_RAS, even_odd=1)
    with pytest.raises(W.WclError) as e:
        lat.solve_nested(p, 0.12, 1.0, lat.zeros(W.F64), lat.zeros(W.F64))
    assert e.value.code == W.EINVAL
    lat.close()


@pytest.mark.parametrize("dims,kappa,nrhs", [((8, 8, 8, 16), 0.125, 1), ((16, 16, 16, 32), 0.125, 1),
                                             ((8, 8, 8, 8), 0.124, 3)])
def test_even_odd_nested_solve(W, ctx, dims, kappa, nrhs):
    csw = 1.0
    U, lat = make(W, ctx, dims)
    eta = I.gaussian_source(dims, 2, nrhs=nrhs) if nrhs > 1 else I.gaussian_source(dims, 2)
    p = W.SolverParams.make(precond=W.PRECOND_NONE, even_odd=1)
    phi = lat.zeros(W.F64, nrhs)
    rc, st = lat.solve_nested(p, kappa, csw, lat.pack(eta, W.F64, nrhs), phi, nrhs=nrhs)
    sol = lat.unpack(phi, W.F64, nrhs)
    lat.close()
    o = Oracle(dims, U)
    etas, sols = (eta, sol) if nrhs > 1 else ([eta], [sol])
    worst = 0.0
    for e_k, s_k in zip(etas, sols):
        res = np.linalg.norm(e_k - o.apply_D(s_k, kappa, csw)) / np.linalg.norm(e_k)
        worst = max(worst, res)
    print(f"even-odd {dims} x{nrhs}: {st}, oracle true residual {worst:.2e}")
    assert st["converged"] == 1 and worst <= 1e-10
    assert abs(st["true_resid"] - worst) <= 1e-12
