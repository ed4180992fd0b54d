"""Host-side checks of the benchmark script (no GPU): the multi-GPU refusal,
the algorithmic flop count used for the domain-solver roofline, and the hash
that ties the stored HBM counters to the kernel sources and flags."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


class _Ras:
    def __init__(self, block, s, n_dominv):
        self.block, self.s, self.n_dominv = block, s, n_dominv


def test_domain_sweep_flops():
    b = load_bench()
    # Wilson-clover operator: 552 site-term + 8 x 165 hop flops = 1872 per site
    assert b.SITE_TERM_FLOPS + 8 * b.HOP_FLOPS == 1872
    dims = (16, 16, 16, 32)
    # 4^4 domains without overlap: 3 of the 4 forward (and backward) hops per
    # direction stay inside a domain, so 6 of 8 hops are kept
    per_site = b.SITE_TERM_FLOPS + 6 * b.HOP_FLOPS + b.MR_FLOPS
    assert b.domain_sweep_flops(dims, _Ras((4, 4, 4, 4), 0, 4), 512, 256) == per_site * 512 * 256 * 4
    # a domain spanning a whole direction keeps both of its hops (periodic wrap inside the set)
    full_t = b.domain_sweep_flops(dims, _Ras((4, 4, 4, 32), 0, 1), 64, 2048)
    assert full_t == (b.SITE_TERM_FLOPS + (6 * 3 / 4 + 2) * b.HOP_FLOPS + b.MR_FLOPS) * 64 * 2048
    # overlap s = 1 extends 4 -> 6 sites: 5 of 6 hops kept per direction
    ov = b.domain_sweep_flops(dims, _Ras((4, 4, 4, 4), 1, 2), 512, 1296)
    assert abs(ov - (b.SITE_TERM_FLOPS + 8 * 5 / 6 * b.HOP_FLOPS + b.MR_FLOPS) * 512 * 1296 * 2) < 1e-3


def test_valu_peak_from_unit_counts():
    b = load_bench()
    # 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
    assert abs(b.VALU_F32_PEAK_TFLOPS - 78.6432) < 1e-3


def test_counter_hash_follows_sources_and_flags():
    """The stored HBM counters count as this build's only while the hash of
    the kernel sources (comments aside) and the device compiler flags is
    unchanged: a flag that changes the code changes the hash, a comment does
    not."""
    b = load_bench()
    from paper_1011_3318_amd import build
    h0 = b.source_hash(b.DOMAIN_SOURCES)
    assert h0 == b.source_hash(b.DOMAIN_SOURCES)
    assert h0 != b.source_hash(b.DAPPLY_SOURCES)
    saved = list(build.HIPCC_FLAGS)
    try:
        build.HIPCC_FLAGS.append("-DWCL_SOME_SWITCH=1")
        assert b.source_hash(b.DOMAIN_SOURCES) != h0
        build.HIPCC_FLAGS[:] = saved + [f"-I{ROOT}/elsewhere"]   # include paths do not count
        assert b.source_hash(b.DOMAIN_SOURCES) == h0
    finally:
        build.HIPCC_FLAGS[:] = saved
