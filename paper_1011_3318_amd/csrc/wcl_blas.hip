// Vector kernels of the BiCGStab solvers (FP64 outer, FP32 inner), batched
// over right-hand sides.  The solver scalars live on the device (struct
// Scal per rhs) so that no kernel waits for the host; every reduction writes
// per-workgroup partial sums, which a finalize kernel (or every workgroup of
// the update kernel that needs the scalar) adds in a fixed order, so results
// are bitwise reproducible run to run.
#include "wcl_device.h"
#include "wcl_kernels.h"

template <int P>
struct Vec;
template <>
struct Vec<WCL_F64> {
    using E = d2v;   // one complex number per element
    static constexpr int per_site = 12;
};
template <>
struct Vec<WCL_F32> {
    using E = f4v;   // two complex numbers per element
    static constexpr int per_site = 6;
};

WCL_DEV void cdiv(double ar, double ai, double br, double bi, double& cr, double& ci) {
    double d = br * br + bi * bi;
    cr = (ar * br + ai * bi) / d;
    ci = (ai * br - ar * bi) / d;
}
WCL_DEV void cmul(double ar, double ai, double br, double bi, double& cr, double& ci) {
    cr = ar * br - ai * bi;
    ci = ar * bi + ai * br;
}

// complex scalar * element helpers
WCL_DEV f4v cm(double cr, double ci, f4v a) {
    float r = (float)cr, i = (float)ci;
    return f4v{r * a.x - i * a.y, r * a.y + i * a.x, r * a.z - i * a.w, r * a.w + i * a.z};
}
WCL_DEV d2v cm(double cr, double ci, d2v a) {
    return d2v{cr * a.x - ci * a.y, cr * a.y + ci * a.x};
}

// The G partial triples of one rhs added in a fixed order: thread t takes
// partials t, t + 256, ... in ascending order (four loads in flight), then
// the workgroup sum.  Every thread receives the totals, and every workgroup
// that reduces the same partials obtains the same bits.
WCL_DEV void partial_total(const double* partial, int G, int rhs, double t[3]) {
    double d[3] = {0, 0, 0};
    const double* q = partial + 3 * (size_t)rhs * G;
    int k = threadIdx.x;
    for (; k + 3 * 256 < G; k += 4 * 256) {
        double v[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[u][c] = q[3 * (k + 256 * u) + c];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) d[c] += v[u][c];
    }
    for (; k < G; k += 256)
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] += q[3 * k + c];
    __shared__ double tot[3];
    block_reduce3(d, tot);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) t[c] = tot[c];
}

// alpha = rho / <rhat, v> from the totals (<rhat, v> in t[0], t[1]);
// returns true on breakdown (<rhat, v> = 0, alpha set to 0)
WCL_DEV bool alpha_step(const double rho[2], const double t[3], double& ar, double& ai) {
    if (t[0] == 0.0 && t[1] == 0.0) {
        ar = ai = 0.0;
        return true;
    }
    cdiv(rho[0], rho[1], t[0], t[1], ar, ai);
    return false;
}

// omega = <t, s> / <t, t> from the totals of the partials of <s, t>, |t|^2
WCL_DEV void omega_step(const double t[3], double& wr, double& wi) {
    if (t[2] > 0.0) {
        wr = t[0] / t[2];
        wi = -t[1] / t[2];
    } else {
        wr = wi = 0.0;
    }
}

// <a, b> contributions (re, im) and |b|^2
WCL_DEV void dot_acc(d2v a, d2v b, double d[3]) {
    d[0] += a.x * b.x + a.y * b.y;
    d[1] += a.x * b.y - a.y * b.x;
    d[2] += b.x * b.x + b.y * b.y;
}
WCL_DEV void dot_acc(f4v a, f4v b, double d[3]) {
    float re = a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
    float im = a.x * b.y - a.y * b.x + a.z * b.w - a.w * b.z;
    float nn = b.x * b.x + b.y * b.y + b.z * b.z + b.w * b.w;
    d[0] += re;
    d[1] += im;
    d[2] += nn;
}

struct BlasGrid {
    int n;        // elements per rhs (whole tiles)
    int stride;   // elements between rhs
    int G;        // workgroups per rhs
    int last;     // first element of the last tile
    int rem;      // sites used in the last tile (64 when the volume fills it)
};

#define BLAS_PROLOGUE                                   \
    const int rhs = blockIdx.x / bg.G;                  \
    const int wg = blockIdx.x % bg.G;                   \
    const size_t base = (size_t)rhs * bg.stride;        \
    const int step = bg.G * 256;

// loop over the elements of one rhs, skipping the padding of the last tile
#define BLAS_FOR(k)                                                    \
    for (int k = wg * 256 + threadIdx.x; k < bg.n; k += step)          \
        if (k < bg.last || (k & 63) < bg.rem)

// p = r + beta (p - omega v), beta = (rho/rho_old)(alpha/omega)
template <int P>
__global__ __launch_bounds__(256) void k_p_update(BlasGrid bg, const Scal* sc, const void* r_, void* p_,
                                                   const void* v_) {
    using E = typename Vec<P>::E;
    BLAS_PROLOGUE
    const Scal& S = sc[rhs];
    if (S.active) {
        double t1r, t1i, t2r, t2i, br, bi;
        cdiv(S.rho[0], S.rho[1], S.rho_old[0], S.rho_old[1], t1r, t1i);
        cdiv(S.alpha[0], S.alpha[1], S.omega[0], S.omega[1], t2r, t2i);
        cmul(t1r, t1i, t2r, t2i, br, bi);
        const double wr = S.omega[0], wi = S.omega[1];
        const E* r = (const E*)r_ + base;
        E* p = (E*)p_ + base;
        const E* v = (const E*)v_ + base;
        BLAS_FOR(k) {
            E pv = p[k] - cm(wr, wi, v[k]);
            p[k] = r[k] + cm(br, bi, pv);
        }
    }
}

// s = r - alpha v with alpha = rho / <rhat, v> formed from the partials of
// the D-apply that produced v.  Every workgroup forms the same alpha; the
// first records it, with <rhat, v> and the breakdown flag, for later kernels
// and the host.
template <int P>
__global__ __launch_bounds__(256) void k_s_update_fin(BlasGrid bg, Scal* sc, const double* pv, int Gv,
                                                       const void* r_, const void* v_, void* s_) {
    using E = typename Vec<P>::E;
    BLAS_PROLOGUE
    Scal* S = sc + rhs;
    if (!S->active) return;   // uniform over the workgroup
    const E* r = (const E*)r_ + base;
    const E* v = (const E*)v_ + base;
    E* s = (E*)s_ + base;
    // this thread's first element is requested before the reduction, so that
    // the two load latencies overlap
    const int k0 = wg * 256 + threadIdx.x;
    const bool own0 = k0 < bg.n && (k0 < bg.last || (k0 & 63) < bg.rem);
    E r0{}, v0{};
    if (own0) {
        r0 = r[k0];
        v0 = v[k0];
    }
    const double rho[2] = {S->rho[0], S->rho[1]};
    double tv[3];
    partial_total(pv, Gv, rhs, tv);
    double ar, ai;
    const bool bd = alpha_step(rho, tv, ar, ai);
    if (wg == 0 && threadIdx.x == 0) {
        S->rv[0] = tv[0];
        S->rv[1] = tv[1];
        S->alpha[0] = ar;
        S->alpha[1] = ai;
        if (bd) S->breakdown = 1;
    }
    if (own0) s[k0] = r0 - cm(ar, ai, v0);
    for (int k = k0 + step; k < bg.n; k += step)
        if (k < bg.last || (k & 63) < bg.rem) s[k] = r[k] - cm(ar, ai, v[k]);
}

// x += alpha p^ + omega s^;  r = s - omega t;  partials of <rhat, r>, |r|^2.
// omega = <t, s> / <t, t> is formed from the partials of the D-apply that
// produced t (recorded by the first workgroup).  The new partials go to a
// second buffer, because other workgroups still read pw.
template <int P>
__global__ __launch_bounds__(256) void k_xr_update_fin(BlasGrid bg, Scal* sc, const double* pw, int Gw, void* x_,
                                                        const void* ph_, const void* sh_, const void* s_,
                                                        const void* t_, void* r_, const void* rh_, double* partial) {
    using E = typename Vec<P>::E;
    BLAS_PROLOGUE
    Scal* S = sc + rhs;
    double d[3] = {0, 0, 0};
    if (S->active) {   // uniform over the workgroup
        E* x = (E*)x_ + base;
        const E* ph = (const E*)ph_ + base;
        const E* sh = (const E*)sh_ + base;
        const E* s = (const E*)s_ + base;
        const E* t = (const E*)t_ + base;
        E* r = (E*)r_ + base;
        const E* rh = (const E*)rh_ + base;
        // this thread's first element is requested before the reduction
        const int k0 = wg * 256 + threadIdx.x;
        const bool own0 = k0 < bg.n && (k0 < bg.last || (k0 & 63) < bg.rem);
        E x0{}, ph0{}, sh0{}, s0{}, t0{}, rh0{};
        if (own0) {
            x0 = x[k0];
            ph0 = ph[k0];
            sh0 = sh[k0];
            s0 = s[k0];
            t0 = t[k0];
            rh0 = rh[k0];
        }
        const double ar = S->alpha[0], ai = S->alpha[1];
        double tw[3];
        partial_total(pw, Gw, rhs, tw);
        double wr, wi;
        omega_step(tw, wr, wi);
        if (wg == 0 && threadIdx.x == 0) {
            S->tt = tw[2];
            S->omega[0] = wr;
            S->omega[1] = wi;
        }
        if (own0) {
            x[k0] = x0 + cm(ar, ai, ph0) + cm(wr, wi, sh0);
            E nr = s0 - cm(wr, wi, t0);
            r[k0] = nr;
            dot_acc(rh0, nr, d);
        }
        for (int k = k0 + step; k < bg.n; k += step)
            if (k < bg.last || (k & 63) < bg.rem) {
                x[k] = x[k] + cm(ar, ai, ph[k]) + cm(wr, wi, sh[k]);
                E nr = s[k] - cm(wr, wi, t[k]);
                r[k] = nr;
                dot_acc(rh[k], nr, d);
            }
    }
    block_reduce3(d, partial + 3 * ((size_t)rhs * bg.G + wg));
}

// partials of <a, b> and |b|^2 (only for active rhs)
template <int P>
__global__ __launch_bounds__(256) void k_dot(BlasGrid bg, const Scal* sc, const void* a_, const void* b_,
                                              double* partial) {
    using E = typename Vec<P>::E;
    BLAS_PROLOGUE
    double d[3] = {0, 0, 0};
    if (!sc || sc[rhs].active) {
        const E* a = (const E*)a_ + base;
        const E* b = (const E*)b_ + base;
        BLAS_FOR(k) dot_acc(a[k], b[k], d);
    }
    block_reduce3(d, partial + 3 * ((size_t)rhs * bg.G + wg));
}

// BiCGStab start in one pass: x = p = v = 0, r = rhat = b; partials of
// <b, b> and |b|^2 for the active rhs (the same sums k_dot forms)
template <int P>
__global__ __launch_bounds__(256) void k_init(BlasGrid bg, const Scal* sc, const void* b_, void* x_, void* r_,
                                               void* rh_, void* p_, void* v_, double* partial) {
    using E = typename Vec<P>::E;
    BLAS_PROLOGUE
    double d[3] = {0, 0, 0};
    const bool act = sc[rhs].active;
    const E* b = (const E*)b_ + base;
    E* x = (E*)x_ + base;
    E* r = (E*)r_ + base;
    E* rh = (E*)rh_ + base;
    E* p = (E*)p_ + base;
    E* v = (E*)v_ + base;
    BLAS_FOR(k) {
        const E bv = b[k];
        x[k] = E{};
        p[k] = E{};
        v[k] = E{};
        r[k] = bv;
        rh[k] = bv;
        if (act) dot_acc(bv, bv, d);
    }
    block_reduce3(d, partial + 3 * ((size_t)rhs * bg.G + wg));
}

// FP64 -> FP32 with factor 1/sqrt(S.pp) (inner right-hand side b = p/|p|);
// FP32 -> FP64 with factor sqrt(S.pp) (p^ = |p| y).  One thread per FP32
// element: float4 g of site i holds FP64 components 2g and 2g+1.
__global__ __launch_bounds__(256) void k_to_f32_scaled(int V, int G, const Scal* sc, const void* a_, size_t astride2,
                                                        void* y_, size_t ystride4) {
    const int rhs = blockIdx.x / G, wg = blockIdx.x % G;
    if (!sc[rhs].active) return;
    const double f = sc[rhs].pp > 0 ? 1.0 / sqrt(sc[rhs].pp) : 0.0;
    const d2v* a = (const d2v*)a_ + (size_t)rhs * astride2;
    f4v* y = (f4v*)y_ + (size_t)rhs * ystride4;
    const int n = 6 * ((V + 63) / 64 * 64);
    for (int k = wg * 256 + threadIdx.x; k < n; k += G * 256) {
        const int i = (k / 384) * 64 + (k & 63), g = (k >> 6) % 6;
        if (i >= V) continue;
        d2v u = a[tix(2 * g, i, 12)], w = a[tix(2 * g + 1, i, 12)];
        y[k] = f4v{(float)(u.x * f), (float)(u.y * f), (float)(w.x * f), (float)(w.y * f)};
    }
}

__global__ __launch_bounds__(256) void k_to_f64_scaled(int V, int G, const Scal* sc, const void* a_, size_t astride4,
                                                        void* y_, size_t ystride2) {
    const int rhs = blockIdx.x / G, wg = blockIdx.x % G;
    if (!sc[rhs].active) return;
    const double f = sqrt(sc[rhs].pp);
    const f4v* a = (const f4v*)a_ + (size_t)rhs * astride4;
    d2v* y = (d2v*)y_ + (size_t)rhs * ystride2;
    const int n = 6 * ((V + 63) / 64 * 64);
    for (int k = wg * 256 + threadIdx.x; k < n; k += G * 256) {
        const int i = (k / 384) * 64 + (k & 63), g = (k >> 6) % 6;
        if (i >= V) continue;
        f4v v = a[k];
        y[tix(2 * g, i, 12)] = d2v{(double)v.x * f, (double)v.y * f};
        y[tix(2 * g + 1, i, 12)] = d2v{(double)v.z * f, (double)v.w * f};
    }
}

// ----------------------------------------------------------- finalize ---
// One workgroup per rhs adds the G partial triples in a fixed order and
// applies the scalar step of BiCGStab selected by `kind`.
__global__ __launch_bounds__(256) void k_finalize(const double* partial, int G, Scal* sc, int kind, Scal* mirror) {
    const int rhs = blockIdx.x;
    // thread 0 fetches the solver state now, so that its latency overlaps
    // that of the partial sums
    Scal S;
    if (threadIdx.x == 0) S = sc[rhs];
    double t[3];
    partial_total(partial, G, rhs, t);
    if (threadIdx.x != 0 || !S.active) return;
    const double s0 = t[0], s1 = t[1], s2 = t[2];
    switch (kind) {
        case FIN_RHO: {  // rho_old = rho; rho = <rhat, r>; rr = |r|^2
            S.rho_old[0] = S.rho[0];
            S.rho_old[1] = S.rho[1];
            S.rho[0] = s0;
            S.rho[1] = s1;
            S.rr = s2;
            break;
        }
        case FIN_PP: S.pp = s2; break;
        case FIN_RR: S.rr = s2; break;
        case FIN_RR0: S.rr0 = s2; S.rr = s2; break;
    }
    sc[rhs] = S;
    if (mirror) {
        // the host's pinned copy: the solver loop reads it after a stream
        // synchronisation, with no copy of its own
        mirror[rhs] = S;
        __threadfence_system();
    }
}

// ------------------------------------------------------------ launchers --
static BlasGrid blas_grid(int prec, int64_t V) {
    BlasGrid bg;
    const int nc = prec == WCL_F64 ? 12 : 6;
    const int64_t tiles = (V + 63) / 64;
    bg.n = (int)(tiles * 64 * nc);
    bg.stride = (int)(spinor_rhs_bytes(prec, V) / 16);
    bg.G = (int)std::min<int64_t>((bg.n + 255) / 256, 1024);
    bg.last = (int)((tiles - 1) * 64 * nc);
    bg.rem = (int)(V - (tiles - 1) * 64);
    return bg;
}

int blas_partials(int prec, int64_t V) { return blas_grid(prec, V).G; }

#define DISPATCH_P(prec, KERNEL, ...)                                                       \
    do {                                                                                    \
        BlasGrid bg = blas_grid(prec, V);                                                   \
        if (prec == WCL_F64)                                                                \
            KERNEL<WCL_F64><<<bg.G * nrhs, 256, 0, st>>>(bg, __VA_ARGS__);                  \
        else                                                                                \
            KERNEL<WCL_F32><<<bg.G * nrhs, 256, 0, st>>>(bg, __VA_ARGS__);                  \
        WCL_HIP(hipGetLastError());                                                         \
    } while (0)

int blas_p_update(int prec, int64_t V, int nrhs, const Scal* sc, const void* r, void* p, const void* v,
                  hipStream_t st) {
    DISPATCH_P(prec, k_p_update, sc, r, p, v);
    return WCL_OK;
}
int blas_s_update_fin(int prec, int64_t V, int nrhs, Scal* sc, const double* pv, int Gv, const void* r,
                      const void* v, void* s, hipStream_t st) {
    DISPATCH_P(prec, k_s_update_fin, sc, pv, Gv, r, v, s);
    return WCL_OK;
}
int blas_xr_update_fin(int prec, int64_t V, int nrhs, Scal* sc, const double* pw, int Gw, void* x, const void* ph,
                       const void* sh, const void* s, const void* t, void* r, const void* rh, double* partial,
                       hipStream_t st) {
    DISPATCH_P(prec, k_xr_update_fin, sc, pw, Gw, x, ph, sh, s, t, r, rh, partial);
    return WCL_OK;
}
int blas_dot(int prec, int64_t V, int nrhs, const Scal* sc, const void* a, const void* b, double* partial,
             hipStream_t st) {
    DISPATCH_P(prec, k_dot, sc, a, b, partial);
    return WCL_OK;
}
int blas_init(int prec, int64_t V, int nrhs, const Scal* sc, const void* b, void* x, void* r, void* rh, void* p,
              void* v, double* partial, hipStream_t st) {
    DISPATCH_P(prec, k_init, sc, b, x, r, rh, p, v, partial);
    return WCL_OK;
}
int blas_to_f32_scaled(int64_t V, int nrhs, const Scal* sc, const void* a64, void* y32, hipStream_t st) {
    BlasGrid bg = blas_grid(WCL_F32, V);
    k_to_f32_scaled<<<bg.G * nrhs, 256, 0, st>>>((int)V, bg.G, sc, a64, spinor_rhs_bytes(WCL_F64, V) / 16, y32,
                                                 spinor_rhs_bytes(WCL_F32, V) / 16);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}
int blas_to_f64_scaled(int64_t V, int nrhs, const Scal* sc, const void* a32, void* y64, hipStream_t st) {
    BlasGrid bg = blas_grid(WCL_F32, V);
    k_to_f64_scaled<<<bg.G * nrhs, 256, 0, st>>>((int)V, bg.G, sc, a32, spinor_rhs_bytes(WCL_F32, V) / 16, y64,
                                                 spinor_rhs_bytes(WCL_F64, V) / 16);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}
int blas_finalize(const double* partial, int G, int nrhs, Scal* sc, int kind, hipStream_t st, Scal* mirror) {
    k_finalize<<<nrhs, 256, 0, st>>>(partial, G, sc, kind, mirror);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

// Restart of the rhs flagged with breakdown == 2: r = src (if given),
// rhat = r, v = 0 and p = r (the p update's result after a restart, whose
// scalars give beta (p - omega v) = 0).
template <int P>
__global__ __launch_bounds__(256) void k_restart(BlasGrid bg, const Scal* sc, const void* src_, void* r_, void* rh_,
                                                  void* p_, void* v_) {
    using E = typename Vec<P>::E;
    BLAS_PROLOGUE
    if (sc[rhs].breakdown != 2) return;
    E* r = (E*)r_ + base;
    E* rh = (E*)rh_ + base;
    E* p = (E*)p_ + base;
    E* v = (E*)v_ + base;
    const E* src = src_ ? (const E*)src_ + base : nullptr;
    BLAS_FOR(k) {
        E rv = src ? src[k] : r[k];
        r[k] = rv;
        rh[k] = rv;
        p[k] = rv;
        v[k] = E{};
    }
}

int blas_restart(int prec, int64_t V, int nrhs, const Scal* sc, const void* src, void* r, void* rh, void* p, void* v,
                 hipStream_t st) {
    DISPATCH_P(prec, k_restart, sc, src, r, rh, p, v);
    return WCL_OK;
}
