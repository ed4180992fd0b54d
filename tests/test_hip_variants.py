"""GPU parity of the other readings of the paper's domain solver and Schwarz
iteration (Sec. 1-2) against the FP64 oracle, through the C ABI:

* domain solvers: minimal residual, block Jacobi (the site terms as the
  diagonal blocks) and BiCGStab truncated to N_dominv iterations;
* Schwarz iterations: restricted additive (Algorithm 1), additive (whole
  extended solutions summed, Richardson refinement) and multiplicative (two
  colours of domains, residual updated in between);
* the site-term inverse (1 + c_SW kappa C)^{-1} the Jacobi solver uses;
* nested solves preconditioned by each variant, with the true residual
  recomputed by the oracle.
"""
import numpy as np
import pytest

from helpers import rel_err
from oracle import Oracle
from paper_1011_3318_amd import inputs as I

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.124, 1.0


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


CASES = [
    ((8, 8, 8, 8), (4, 4, 4, 4), 0, 3, 4),   # 16 domains of 256 sites, no overlap
    ((8, 8, 8, 8), (2, 2, 2, 2), 1, 2, 3),   # overlap 1: 256 domains of 4^4 extended sites
    ((8, 4, 6, 4), (4, 2, 2, 4), 1, 2, 3),   # 384 extended sites: two workgroups per domain
    ((16, 4, 4, 4), (4, 4, 4, 4), 1, 2, 2),  # the paper's x-only split (domains span y, z, t)
]
SOLVERS = ["MR", "JACOBI", "BICGSTAB"]
SCHWARZ = ["RAS", "AS", "SAP"]


@pytest.mark.parametrize("storage,tol", [(1, 1e-4), (2, 2e-2)])
@pytest.mark.parametrize("schwarz", SCHWARZ)
@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("dims,block,s,n_ras,nd", CASES)
def test_schwarz_variant(W, ctx, dims, block, s, n_ras, nd, solver, schwarz, storage, tol):
    U, lat = make(W, ctx, dims, bc=(1, 1, 1, -1))
    o = Oracle(dims, U, bc=(1, 1, 1, -1))
    r = I.gaussian_source(dims, 6)
    sv, sz = getattr(W, "DOMSOLVE_" + solver), getattr(W, "SCHWARZ_" + schwarz)
    ras = W.RasParams.make(block=block, s=s, n_ras=n_ras, n_dominv=nd, storage=storage, block_solver=sv,
                           schwarz=sz)
    v = lat.empty(W.F32)
    lat.ras_precondition(ras, KAPPA, CSW, lat.pack(r, W.F32), v)
    got = lat.unpack(v, W.F32)
    ref = o.schwarz(r, KAPPA, CSW, block, s, n_ras, nd, solver=sv, schwarz=sz)
    e = rel_err(got, ref)
    print(f"{solver}/{schwarz} storage {storage}: rel err {e:.2e}")
    assert e <= tol
    lat.close()


def test_jacobi_one_step_is_the_site_inverse(W, ctx):
    """One Jacobi step from zero, one sweep: v = A^{-1} r at every site."""
    dims = (4, 4, 4, 8)
    U, lat = make(W, ctx, dims)
    o = Oracle(dims, U)
    r = I.gaussian_source(dims, 3)
    ras = W.RasParams.make(block=(2, 2, 2, 2), s=0, n_ras=1, n_dominv=1, block_solver=W.DOMSOLVE_JACOBI)
    v = lat.empty(W.F32)
    lat.ras_precondition(ras, 0.13, 1.5, lat.pack(r, W.F32), v)
    Ainv = o.site_term_inverse(0.13, 1.5)
    ref = np.einsum("xij,xj->xi", Ainv, r.reshape(-1, 12)).reshape(r.shape)
    assert rel_err(lat.unpack(v, W.F32), ref) <= 2e-6
    lat.close()


def test_site_inverse_follows_kappa_and_clover(W, ctx):
    """The cached inverse is rebuilt when kappa, c_SW or the gauge field change."""
    dims = (4, 4, 4, 4)
    U, lat = make(W, ctx, dims)
    r = I.gaussian_source(dims, 3)
    rd = lat.pack(r, W.F32)
    ras = W.RasParams.make(block=(2, 2, 2, 2), s=0, n_ras=1, n_dominv=1, block_solver=W.DOMSOLVE_JACOBI)
    v = lat.empty(W.F32)
    for kappa, csw in [(0.12, 1.0), (0.13, 1.0), (0.13, 1.5), (0.12, 1.0)]:
        lat.ras_precondition(ras, kappa, csw, rd, v)
        Ainv = Oracle(dims, U).site_term_inverse(kappa, csw)
        ref = np.einsum("xij,xj->xi", Ainv, r.reshape(-1, 12)).reshape(r.shape)
        assert rel_err(lat.unpack(v, W.F32), ref) <= 2e-6
    U2 = I.random_gauge(dims, 0.8, 5)
    lat.upload_gauge(U2)
    lat.ras_precondition(ras, 0.12, 1.0, rd, v)
    Ainv = Oracle(dims, U2).site_term_inverse(0.12, 1.0)
    ref = np.einsum("xij,xj->xi", Ainv, r.reshape(-1, 12)).reshape(r.shape)
    assert rel_err(lat.unpack(v, W.F32), ref) <= 2e-6
    lat.close()


@pytest.mark.parametrize("solver,schwarz", [("BICGSTAB", "RAS"), ("JACOBI", "AS"), ("MR", "SAP")])
def test_variant_multi_rhs_equals_single(W, ctx, solver, schwarz):
    dims = (8, 8, 8, 8)
    U, lat = make(W, ctx, dims)
    r = I.gaussian_source(dims, 8, nrhs=3)
    ras = W.RasParams.make(block=(4, 4, 4, 4), s=1, n_ras=2, n_dominv=3,
                           block_solver=getattr(W, "DOMSOLVE_" + solver), schwarz=getattr(W, "SCHWARZ_" + schwarz))
    v = lat.empty(W.F32, 3)
    lat.ras_precondition(ras, KAPPA, CSW, lat.pack(r, W.F32, 3), v, nrhs=3)
    many = lat.unpack(v, W.F32, 3)
    for k in range(3):
        v1 = lat.empty(W.F32)
        lat.ras_precondition(ras, KAPPA, CSW, lat.pack(r[k], W.F32), v1)
        assert np.array_equal(lat.unpack(v1, W.F32), many[k])
    lat.close()


def test_fused_kernel_rejects_variants(W, ctx):
    dims = (8, 8, 8, 8)
    _, lat = make(W, ctx, dims)
    for sv, sz in [(W.DOMSOLVE_JACOBI, W.SCHWARZ_RAS), (W.DOMSOLVE_MR, W.SCHWARZ_SAP)]:
        ras = W.RasParams.make(block=(4, 4, 4, 4), s=0, kernel=W.BLOCK_FUSED, block_solver=sv, schwarz=sz)
        with pytest.raises(W.WclError) as e:
            lat.ras_precondition(ras, 0.12, 1.0, lat.zeros(W.F32), lat.empty(W.F32))
        assert e.value.code == W.EINVAL
    lat.close()


# The additive iteration with overlap counts the overlap twice, so its
# Richardson refinement diverges; one application (n_ras = 1) is the
# classical additive Schwarz preconditioner.
@pytest.mark.parametrize("solver,schwarz,s,n_ras", [("JACOBI", "RAS", 0, 2), ("BICGSTAB", "RAS", 1, 2),
                                                     ("MR", "AS", 1, 1), ("JACOBI", "AS", 0, 2),
                                                     ("MR", "SAP", 0, 2), ("BICGSTAB", "SAP", 1, 2)])
def test_nested_solve_with_variant(W, ctx, solver, schwarz, s, n_ras):
    dims = (8, 8, 8, 16)
    kappa, csw = 0.125, 1.0
    U, lat = make(W, ctx, dims)
    eta = I.gaussian_source(dims, 2)
    ras = W.RasParams.make(block=(4, 4, 4, 4), s=s, n_ras=n_ras, n_dominv=3, storage=W.F32,
                           block_solver=getattr(W, "DOMSOLVE_" + solver), schwarz=getattr(W, "SCHWARZ_" + schwarz))
    p = W.SolverParams.make(ras=ras)
    phi = lat.zeros(W.F64)
    rc, st = lat.solve_nested(p, kappa, csw, lat.pack(eta, W.F64), phi)
    sol = lat.unpack(phi, W.F64)
    lat.close()
    o = Oracle(dims, U)
    res = np.linalg.norm(eta - o.apply_D(sol, kappa, csw)) / np.linalg.norm(eta)
    print(f"{solver}/{schwarz} s={s}: {st}, oracle true residual {res:.2e}")
    assert st["converged"] == 1 and res <= 1e-10
