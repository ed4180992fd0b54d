// Full-lattice Wilson-clover D application (Eq. (1)), one site and one
// right-hand side per lane, templated on the storage precision of the
// links/clover (GP), of the input spinor (SPI), of the output (SPO) and of
// the optional axpy source (SPY).  Epilogues:
//   DS_PLAIN  out = D in
//   DS_AXPY   out = y - D in                       (RAS: r <- r - D v)
//   DS_DOT    out = D in, partial sums of <a, out> and <out, out> per
//             workgroup (BiCGStab: v = A p^, <r^, v>; t = A s^, <t,s>, <t,t>)
#include "wcl_device.h"
#include "wcl_kernels.h"

template <int MU, bool FWD, int GP, int SPI, typename T>
WCL_DEV void hop(const DslashArgs& a, const char* in, int j, int ulink_site, T f, T acc[24]) {
    T s[24], h[12], w[12], u[18];
    SpinorIO<SPI>::load(in, a.g.V, j, s);
    spin_project<MU, FWD>(s, h);
    GaugeIO<GP>::load(a.gauge, a.g.V, MU, ulink_site, u);
    su3_apply2<!FWD>(u, h, w);
    spin_accumulate<MU, FWD>(w, f, acc);
}

template <int MU, int GP, int SPI, typename T>
WCL_DEV void hops_dir(const DslashArgs& a, const char* in, int i, const int x[4], T mk, T acc[24]) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    // forward: (1 - gamma_mu) U_mu(x) psi(x + mu)
    T ph = T(1);
    y[MU] = x[MU] + 1;
    if (y[MU] == a.g.L[MU]) {
        y[MU] = 0;
        ph = T(a.g.bc[MU]);
    }
    hop<MU, true, GP, SPI>(a, in, geom_index(a.g, y), i, mk * ph, acc);
    // backward: (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
    ph = T(1);
    y[MU] = x[MU] - 1;
    if (y[MU] < 0) {
        y[MU] = a.g.L[MU] - 1;
        ph = T(a.g.bc[MU]);
    }
    int jb = geom_index(a.g, y);
    hop<MU, false, GP, SPI>(a, in, jb, jb, mk * ph, acc);
}

template <int GP, int SPI, typename T>
WCL_DEV void dslash_site(const DslashArgs& a, const char* in, int i, T acc[24]) {
    int x[4];
    geom_coords(a.g, i, x);
    {
        T s[24], c[72];
        SpinorIO<SPI>::load(in, a.g.V, i, s);
        CloverIO<GP>::load(a.clover, a.g.V, i, c);
        clover_term(c, s, T(a.csw * a.kappa), acc);
    }
    const T mk = T(-a.kappa);
    hops_dir<0, GP, SPI>(a, in, i, x, mk, acc);
    hops_dir<1, GP, SPI>(a, in, i, x, mk, acc);
    hops_dir<2, GP, SPI>(a, in, i, x, mk, acc);
    hops_dir<3, GP, SPI>(a, in, i, x, mk, acc);
}

template <int GP, int SPI, int SPO, int EPI, int SPY>
__global__ __launch_bounds__(256) void k_dslash(DslashArgs a) {
    using T = typename Real<GP>::T;
    static_assert((GP == WCL_F64) == (SPI == WCL_F64), "FP64 arithmetic needs FP64 spinors and links");
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int rhs = lb % a.nrhs;
    const int i = (lb / a.nrhs) * 256 + threadIdx.x;
    const bool active = i < a.g.V;
    T acc[24];
    if (active) {
        dslash_site<GP, SPI>(a, (const char*)a.in + rhs * a.in_stride, i, acc);
        if (EPI == DS_AXPY) {
            T y[24];
            SpinorIO<SPY>::load((const char*)a.y + rhs * a.y_stride, a.g.V, i, y);
#pragma unroll
            for (int k = 0; k < 24; ++k) acc[k] = y[k] - acc[k];
        }
        SpinorIO<SPO>::store((char*)a.out + rhs * a.out_stride, a.g.V, i, acc);
    }
    if (EPI == DS_DOT) {
        // <a, out> (complex) and <out, out> for this workgroup, fixed tree order
        double d[3] = {0.0, 0.0, 0.0};
        if (active) {
            T v[24];
            SpinorIO<SPO>::load((const char*)a.a + rhs * a.a_stride, a.g.V, i, v);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                T ar = v[2 * k], ai = v[2 * k + 1], br = acc[2 * k], bi = acc[2 * k + 1];
                d[0] += (double)(ar * br + ai * bi);
                d[1] += (double)(ar * bi - ai * br);
                d[2] += (double)(br * br + bi * bi);
            }
        }
        block_reduce3(d, a.partial + 3 * (size_t)((lb / a.nrhs) + (size_t)rhs * (gridDim.x / a.nrhs)));
    }
}

template <int GP, int SPI, int SPO, int EPI, int SPY>
static int launch_t(const DslashArgs& a, hipStream_t st) {
    int tiles = (a.g.V + 255) / 256;
    k_dslash<GP, SPI, SPO, EPI, SPY><<<tiles * a.nrhs, 256, 0, st>>>(a);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int dslash_partials_per_rhs(int V) { return (V + 255) / 256; }

// Runtime dispatch over the instantiated combinations.
int launch_dslash(const DslashArgs& a, int gp, int spi, int spo, int epi, int spy, hipStream_t st) {
#define WCL_TRY(G, I, O, E, Y) \
    if (gp == G && spi == I && spo == O && epi == E && (E != DS_AXPY || spy == Y)) return launch_t<G, I, O, E, Y>(a, st)
    WCL_TRY(WCL_F64, WCL_F64, WCL_F64, DS_PLAIN, WCL_F64);
    WCL_TRY(WCL_F64, WCL_F64, WCL_F64, DS_AXPY, WCL_F64);
    WCL_TRY(WCL_F64, WCL_F64, WCL_F64, DS_DOT, WCL_F64);
    WCL_TRY(WCL_F32, WCL_F32, WCL_F32, DS_PLAIN, WCL_F32);
    WCL_TRY(WCL_F32, WCL_F32, WCL_F32, DS_AXPY, WCL_F32);
    WCL_TRY(WCL_F32, WCL_F32, WCL_F32, DS_DOT, WCL_F32);
    WCL_TRY(WCL_F16, WCL_F16, WCL_F16, DS_PLAIN, WCL_F16);
    WCL_TRY(WCL_F16, WCL_F32, WCL_F32, DS_PLAIN, WCL_F32);
    WCL_TRY(WCL_F16, WCL_F32, WCL_F32, DS_DOT, WCL_F32);
    // RAS residual update with FP16 storage: r_{j+1} = r_j - D v_j
    WCL_TRY(WCL_F16, WCL_F16, WCL_F16, DS_AXPY, WCL_F32);
    WCL_TRY(WCL_F16, WCL_F16, WCL_F16, DS_AXPY, WCL_F16);
#undef WCL_TRY
    wcl_set_error("dslash: unsupported precision combination (%d,%d,%d,%d,%d)", gp, spi, spo, epi, spy);
    return WCL_EINVAL;
}
