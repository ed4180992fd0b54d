"""The entry point for callers that cannot allocate device memory:
wcl_ras_precondition_noalloc against wcl_ras_precondition (same kernels,
bitwise the same result) on two calls in a row, the second on a smaller
input, with the library's and torch's allocation counters unchanged."""
import gc

import numpy as np
import pytest
import torch

from paper_1011_3318_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    from paper_1011_3318_amd import wcl
    return wcl


def test_noalloc_matches_ras_precondition(W):
    ctx = W.Context(0)
    calls = [((8, 8, 8, 8), (4, 4, 4, 4), 0, 3, 4, W.F16, 2),   # no overlap, FP16 storage, 2 rhs
             ((4, 4, 8, 8), (2, 2, 2, 2), 1, 4, 3, W.F32, 1)]   # smaller: overlap 1, 4 sweeps, 1 rhs
    lats, inputs = [], []
    for dims, block, s, n_ras, nd, storage, nrhs in calls:
        lat = W.Lattice(ctx, dims)
        lat.upload_gauge(I.random_gauge(dims, 0.5, 1))
        r = I.gaussian_source(dims, 6, nrhs=nrhs) if nrhs > 1 else I.gaussian_source(dims, 6)
        ras = W.RasParams.make(block=block, s=s, n_ras=n_ras, n_dominv=nd, storage=storage)
        lats.append(lat)
        inputs.append((ras, lat.pack(r, W.F32, nrhs), lat.empty(W.F32, nrhs), lat.empty(W.F32, nrhs), nrhs))
    torch.cuda.synchronize()
    # objects left by earlier tests are collected first, and not while the
    # allocation counters are compared
    gc.collect()
    gc.disable()
    try:
        lib_before = ctx.bytes_in_use()
        torch_before = torch.cuda.memory_allocated()
        # two no-allocation calls in a row, the second smaller
        for lat, (ras, rd, v_na, _, nrhs) in zip(lats, inputs):
            lat.ras_precondition_noalloc(ras, 0.124, 1.0, rd, v_na, nrhs=nrhs)
        torch.cuda.synchronize()
        lib_after = ctx.bytes_in_use()
        torch_after = torch.cuda.memory_allocated()
    finally:
        gc.enable()
    assert lib_after == lib_before
    assert torch_after == torch_before
    # the allocating entry point on the same inputs
    for lat, (ras, rd, v_na, v_ref, nrhs) in zip(lats, inputs):
        lat.ras_precondition(ras, 0.124, 1.0, rd, v_ref, nrhs=nrhs)
        got, ref = lat.unpack(v_na, W.F32, nrhs), lat.unpack(v_ref, W.F32, nrhs)
        assert np.isfinite(ref).all() and np.abs(ref).max() > 0
        assert np.array_equal(got, ref)
    for lat in lats:
        lat.close()
    ctx.close()


def test_noalloc_rejects_what_it_cannot_hold(W):
    ctx = W.Context(0)
    dims = (8, 8, 8, 8)
    lat = W.Lattice(ctx, dims)
    lat.upload_gauge(I.random_gauge(dims, 0.5, 1))
    # 48 rhs x 4 FP32 sweep fields of an 8^4 lattice: 72 MiB > the fixed 64 MiB
    nrhs = 48
    r, v = lat.zeros(W.F32, nrhs), lat.empty(W.F32, nrhs)
    big = W.RasParams.make(block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=2, storage=W.F32)
    with pytest.raises(W.WclError) as e:
        lat.ras_precondition_noalloc(big, 0.12, 1.0, r, v, nrhs=nrhs)
    assert e.value.code == W.EINVAL and "scratch" in str(e.value)
    # the split path (extended domains over 256 sites) and the other readings allocate
    for ras in [W.RasParams.make(block=(4, 4, 4, 4), s=1),
                W.RasParams.make(block=(4, 4, 4, 4), s=0, block_solver=W.DOMSOLVE_JACOBI),
                W.RasParams.make(block=(4, 4, 4, 4), s=0, kernel=W.BLOCK_SPLIT)]:
        with pytest.raises(W.WclError) as e:
            lat.ras_precondition_noalloc(ras, 0.12, 1.0, r[: lat.spinor_bytes(W.F32)], v[: lat.spinor_bytes(W.F32)])
        assert e.value.code == W.EINVAL
    lat.close()
    ctx.close()
