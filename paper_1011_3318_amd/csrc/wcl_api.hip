// C-ABI entry points: context, lattice, resident fields, spinor layout
// conversion and the operator calls.  Solver entry points live in
// wcl_solver.hip, serving in wcl_server.cpp.
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstring>
#include <atomic>
#include <vector>

#include "wcl_kernels.h"

static thread_local char g_err[512] = "";

void wcl_set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int wcl_dev_alloc(wcl_ctx* ctx, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return WCL_OK;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        if (ctx->in_use + bytes > ctx->budget) {
            wcl_set_error("HBM budget exhausted: %llu in use + %llu requested > %llu budget",
                          (unsigned long long)ctx->in_use, (unsigned long long)bytes,
                          (unsigned long long)ctx->budget);
            return WCL_ENOMEM;
        }
        ctx->in_use += bytes;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->in_use -= bytes;
        wcl_set_error("hipMalloc(%llu) failed: %s", (unsigned long long)bytes, hipGetErrorString(e));
        return WCL_ENOMEM;
    }
    return WCL_OK;
}

void wcl_dev_free(wcl_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->in_use -= bytes;
}

int check_prec(int prec) {
    if (prec != WCL_F64 && prec != WCL_F32 && prec != WCL_F16) {
        wcl_set_error("invalid precision %d", prec);
        return WCL_EINVAL;
    }
    return WCL_OK;
}

static int set_device(const wcl_ctx* ctx) {
    WCL_HIP(hipSetDevice(ctx->device));
    return WCL_OK;
}

extern "C" {

const char* wcl_last_error(void) { return g_err; }

int wcl_init(int device, uint64_t hbm_budget_bytes, wcl_ctx** out) {
    if (!out) {
        wcl_set_error("wcl_init: null output handle");
        return WCL_EINVAL;
    }
    *out = nullptr;
    int n = 0;
    WCL_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) {
        wcl_set_error("wcl_init: device %d out of range (%d devices)", device, n);
        return WCL_EINVAL;
    }
    WCL_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    WCL_HIP(hipGetDeviceProperties(&prop, device));
    size_t free_b = 0, total_b = 0;
    WCL_HIP(hipMemGetInfo(&free_b, &total_b));
    auto* c = new wcl_ctx;
    c->device = device;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)free_b;
    c->in_use = 0;
    c->arch_major = prop.major;
    c->num_cu = prop.multiProcessorCount;
    const int rc = static_scratch_setup(device, &c->scratch);
    if (rc != WCL_OK) {
        delete c;
        return rc;
    }
    *out = c;
    return WCL_OK;
}

int wcl_finalize(wcl_ctx* ctx) {
    delete ctx;
    return WCL_OK;
}

uint64_t wcl_bytes_in_use(wcl_ctx* ctx) { return ctx ? ctx->in_use : 0; }

// Column cross-section: the largest power of two dividing L_mu, at most 32
// in x and y and 8 in z.  Whole x rows keep the x-neighbours of a t-slice
// inside the column (the hops that leave a column are the ones re-fetched
// from memory most often); measured on 32^4 this cross-section beat 16x16x8,
// 8x8x4 and 32x32x32.
static int pow2_divisor(int L, int cap) {
    int c = 1;
    while (c * 2 <= cap && L % (c * 2) == 0) c *= 2;
    return c;
}

int wcl_create_lattice(wcl_ctx* ctx, const int dims[4], const int bc[4], wcl_lattice** out) {
    if (!ctx || !dims || !out) {
        wcl_set_error("wcl_create_lattice: null argument");
        return WCL_EINVAL;
    }
    *out = nullptr;
    int64_t V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 2 || dims[mu] > 4096) {
            wcl_set_error("wcl_create_lattice: dims[%d] = %d out of range [2, 4096]", mu, dims[mu]);
            return WCL_EINVAL;
        }
        if (bc && bc[mu] != 1 && bc[mu] != -1) {
            wcl_set_error("wcl_create_lattice: bc[%d] = %d must be +1 or -1", mu, bc[mu]);
            return WCL_EINVAL;
        }
        V *= dims[mu];
    }
    if (V * 12 * 12 > INT32_MAX) {
        wcl_set_error("wcl_create_lattice: volume %lld too large", (long long)V);
        return WCL_EINVAL;
    }
    static std::atomic<uint64_t> next_uid{1};
    auto* lat = new wcl_lattice;
    lat->ctx = ctx;
    lat->V = V;
    lat->uid = next_uid++;
    Geom& g = lat->g;
    const int caps[3] = {32, 32, 8};
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = dims[mu];
        g.bc[mu] = bc ? bc[mu] : 1;
    }
    g.S = 1;
    for (int d = 0; d < 3; ++d) {
        g.c[d] = pow2_divisor(dims[d], caps[d]);
        g.lc[d] = 0;
        while ((1 << g.lc[d]) < g.c[d]) ++g.lc[d];
        g.nC[d] = dims[d] / g.c[d];
        g.S *= g.c[d];
    }
    g.Vc = g.S * dims[3];
    g.V = (int)V;
    // lanes per site of the D-apply (1, 2 or 4); one lane per site measured
    // fastest on 16^3x32 and 32^4; the autotuner may pick another
    lat->lps = 1;
    *out = lat;
    return WCL_OK;
}

int wcl_destroy_lattice(wcl_lattice* lat) {
    if (!lat) return WCL_OK;
    set_device(lat->ctx);
    (void)hipDeviceSynchronize();
    wcl_free_workspace(lat);
    for (int p = 0; p < 3; ++p) {
        wcl_dev_free(lat->ctx, lat->gauge[p], gauge_bytes(p, lat->V));
        wcl_dev_free(lat->ctx, lat->clover[p], clover_bytes(p, lat->V));
    }
    delete lat;
    return WCL_OK;
}

int64_t wcl_volume(const wcl_lattice* lat) { return lat ? lat->V : 0; }

uint64_t wcl_spinor_bytes(const wcl_lattice* lat, int prec, int nrhs) {
    if (!lat || check_prec(prec) != WCL_OK || nrhs < 1) return 0;
    return spinor_rhs_bytes(prec, lat->V) * (uint64_t)nrhs;
}

// ------------------------------------------------------------- gauge ----
static bool link_is_su3(const double* u) {
    using C = std::complex<double>;
    C m[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            m[a][b] = C(u[2 * (3 * a + b)], u[2 * (3 * a + b) + 1]);
            if (!std::isfinite(m[a][b].real()) || !std::isfinite(m[a][b].imag())) return false;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            C s = 0;
            for (int k = 0; k < 3; ++k) s += m[a][k] * std::conj(m[b][k]);
            if (std::abs(s - C(a == b ? 1.0 : 0.0)) > 1e-12) return false;
        }
    C det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
            m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
    return std::abs(det - 1.0) <= 1e-12;
}

static int ensure_fields(wcl_lattice* lat) {
    for (int p = 0; p < 3; ++p) {
        if (!lat->gauge[p]) WCL_CHECK(wcl_dev_alloc(lat->ctx, &lat->gauge[p], gauge_bytes(p, lat->V)));
        if (!lat->clover[p]) WCL_CHECK(wcl_dev_alloc(lat->ctx, &lat->clover[p], clover_bytes(p, lat->V)));
    }
    return WCL_OK;
}

int wcl_upload_gauge(wcl_lattice* lat, const double* U) {
    if (!lat || !U) {
        wcl_set_error("wcl_upload_gauge: null argument");
        return WCL_EINVAL;
    }
    for (int64_t k = 0; k < lat->V * 4; ++k)
        if (!link_is_su3(U + 18 * k)) {
            wcl_set_error("wcl_upload_gauge: link %lld (site %lld, mu %lld) is not SU(3) to 1e-12", (long long)k,
                          (long long)(k / 4), (long long)(k % 4));
            return WCL_EUNITARITY;
        }
    WCL_CHECK(set_device(lat->ctx));
    WCL_CHECK(ensure_fields(lat));
    const size_t bytes = (size_t)lat->V * 4 * 18 * sizeof(double);
    void* stage = nullptr;
    WCL_CHECK(wcl_dev_alloc(lat->ctx, &stage, bytes));
    int rc = WCL_OK;
    if (hipMemcpy(stage, U, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        wcl_set_error("wcl_upload_gauge: host->device copy failed");
        rc = WCL_EHIP;
    }
    if (rc == WCL_OK) rc = launch_pack_gauge(lat->g, (const double*)stage, lat->gauge[0], lat->gauge[1], lat->gauge[2], 0);
    if (rc == WCL_OK && hipDeviceSynchronize() != hipSuccess) {
        wcl_set_error("wcl_upload_gauge: pack kernel failed");
        rc = WCL_EHIP;
    }
    wcl_dev_free(lat->ctx, stage, bytes);
    if (rc == WCL_OK) {
        lat->has_gauge = true;
        lat->has_clover = false;
    }
    return rc;
}

int wcl_compute_clover(wcl_lattice* lat) {
    if (!lat) return WCL_EINVAL;
    if (!lat->has_gauge) {
        wcl_set_error("wcl_compute_clover: no gauge field uploaded");
        return WCL_ESTATE;
    }
    WCL_CHECK(set_device(lat->ctx));
    WCL_CHECK(launch_clover_build(lat->g, lat->gauge[0], lat->clover[0], lat->clover[1], lat->clover[2], 0));
    WCL_HIP(hipDeviceSynchronize());
    lat->has_clover = true;
    ++lat->clover_gen;
    return WCL_OK;
}

int wcl_upload_clover(wcl_lattice* lat, const double* C) {
    if (!lat || !C) {
        wcl_set_error("wcl_upload_clover: null argument");
        return WCL_EINVAL;
    }
    for (int64_t k = 0; k < lat->V * 72; ++k)
        if (!std::isfinite(C[k])) {
            wcl_set_error("wcl_upload_clover: non-finite entry %lld", (long long)k);
            return WCL_EINVAL;
        }
    WCL_CHECK(set_device(lat->ctx));
    WCL_CHECK(ensure_fields(lat));
    const size_t bytes = (size_t)lat->V * 72 * sizeof(double);
    void* stage = nullptr;
    WCL_CHECK(wcl_dev_alloc(lat->ctx, &stage, bytes));
    int rc = WCL_OK;
    if (hipMemcpy(stage, C, bytes, hipMemcpyHostToDevice) != hipSuccess) rc = WCL_EHIP;
    if (rc == WCL_OK) rc = launch_pack_clover(lat->g, (const double*)stage, lat->clover[0], lat->clover[1], lat->clover[2], 0);
    if (rc == WCL_OK && hipDeviceSynchronize() != hipSuccess) rc = WCL_EHIP;
    wcl_dev_free(lat->ctx, stage, bytes);
    if (rc == WCL_EHIP) wcl_set_error("wcl_upload_clover: device copy or pack failed");
    if (rc == WCL_OK) {
        lat->has_clover = true;
        ++lat->clover_gen;
    }
    return rc;
}

int wcl_download_clover(wcl_lattice* lat, double* C) {
    if (!lat || !C) return WCL_EINVAL;
    if (!lat->has_clover) {
        wcl_set_error("wcl_download_clover: no clover field");
        return WCL_ESTATE;
    }
    WCL_CHECK(set_device(lat->ctx));
    const size_t bytes = (size_t)lat->V * 72 * sizeof(double);
    void* stage = nullptr;
    WCL_CHECK(wcl_dev_alloc(lat->ctx, &stage, bytes));
    int rc = launch_unpack_clover(lat->g, lat->clover[0], (double*)stage, 0);
    if (rc == WCL_OK && hipMemcpy(C, stage, bytes, hipMemcpyDeviceToHost) != hipSuccess) {
        wcl_set_error("wcl_download_clover: copy failed");
        rc = WCL_EHIP;
    }
    wcl_dev_free(lat->ctx, stage, bytes);
    return rc;
}

// ----------------------------------------------------------- spinors ----
int wcl_pack_spinor_dev(wcl_lattice* lat, int prec, int nrhs, const double* dev_aos, void* dev_soa, void* stream) {
    if (!lat || !dev_aos || !dev_soa || nrhs < 1) {
        wcl_set_error("wcl_pack_spinor: bad argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(check_prec(prec));
    WCL_CHECK(set_device(lat->ctx));
    return launch_pack_spinor(lat->g, prec, nrhs, dev_aos, dev_soa, spinor_rhs_bytes(prec, lat->V),
                              (hipStream_t)stream);
}

int wcl_unpack_spinor_dev(wcl_lattice* lat, int prec, int nrhs, const void* dev_soa, double* dev_aos, void* stream) {
    if (!lat || !dev_aos || !dev_soa || nrhs < 1) {
        wcl_set_error("wcl_unpack_spinor: bad argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(check_prec(prec));
    WCL_CHECK(set_device(lat->ctx));
    return launch_unpack_spinor(lat->g, prec, nrhs, dev_soa, spinor_rhs_bytes(prec, lat->V), dev_aos,
                                (hipStream_t)stream);
}

int wcl_pack_spinor(wcl_lattice* lat, int prec, int nrhs, const double* host_aos, void* dev_soa, void* stream) {
    if (!lat || !host_aos || nrhs < 1) {
        wcl_set_error("wcl_pack_spinor: bad argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(check_prec(prec));
    WCL_CHECK(set_device(lat->ctx));
    const size_t bytes = (size_t)lat->V * nrhs * 24 * sizeof(double);
    void* stage = nullptr;
    WCL_CHECK(wcl_dev_alloc(lat->ctx, &stage, bytes));
    hipStream_t st = (hipStream_t)stream;
    int rc = WCL_OK;
    if (hipMemcpyAsync(stage, host_aos, bytes, hipMemcpyHostToDevice, st) != hipSuccess) rc = WCL_EHIP;
    if (rc == WCL_OK) rc = wcl_pack_spinor_dev(lat, prec, nrhs, (const double*)stage, dev_soa, stream);
    if (hipStreamSynchronize(st) != hipSuccess && rc == WCL_OK) rc = WCL_EHIP;
    if (rc == WCL_EHIP) wcl_set_error("wcl_pack_spinor: copy or pack failed");
    wcl_dev_free(lat->ctx, stage, bytes);
    return rc;
}

int wcl_unpack_spinor(wcl_lattice* lat, int prec, int nrhs, const void* dev_soa, double* host_aos, void* stream) {
    if (!lat || !host_aos || nrhs < 1) {
        wcl_set_error("wcl_unpack_spinor: bad argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(check_prec(prec));
    WCL_CHECK(set_device(lat->ctx));
    const size_t bytes = (size_t)lat->V * nrhs * 24 * sizeof(double);
    void* stage = nullptr;
    WCL_CHECK(wcl_dev_alloc(lat->ctx, &stage, bytes));
    hipStream_t st = (hipStream_t)stream;
    int rc = wcl_unpack_spinor_dev(lat, prec, nrhs, dev_soa, (double*)stage, stream);
    if (rc == WCL_OK && hipMemcpyAsync(host_aos, stage, bytes, hipMemcpyDeviceToHost, st) != hipSuccess) rc = WCL_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess && rc == WCL_OK) rc = WCL_EHIP;
    if (rc == WCL_EHIP) wcl_set_error("wcl_unpack_spinor: unpack or copy failed");
    wcl_dev_free(lat->ctx, stage, bytes);
    return rc;
}

// ---------------------------------------------------------- operator ----
int wcl_apply_D(wcl_lattice* lat, int prec, double kappa, double csw, const void* in_dev, void* out_dev, int nrhs,
                void* stream) {
    if (!lat || !in_dev || !out_dev || nrhs < 1 || in_dev == out_dev) {
        wcl_set_error("wcl_apply_D: bad argument (null pointer, nrhs < 1 or in == out)");
        return WCL_EINVAL;
    }
    if (!std::isfinite(kappa) || !std::isfinite(csw)) {
        wcl_set_error("wcl_apply_D: non-finite kappa or csw");
        return WCL_EINVAL;
    }
    WCL_CHECK(check_prec(prec));
    if (!lat->has_clover) {
        wcl_set_error("wcl_apply_D: gauge and clover fields must be resident");
        return WCL_ESTATE;
    }
    WCL_CHECK(set_device(lat->ctx));
    DslashArgs a{};
    a.g = lat->g;
    a.gauge = lat->gauge[prec];
    a.clover = lat->clover[prec];
    a.in = in_dev;
    a.out = out_dev;
    a.in_stride = a.out_stride = spinor_rhs_bytes(prec, lat->V);
    a.kappa = kappa;
    a.csw = csw;
    a.nrhs = nrhs;
    a.lps = lat->lps;
    return launch_dslash(a, prec, prec, prec, DS_PLAIN, prec, (hipStream_t)stream);
}

}  // extern "C"
