// Even-odd reduction of D phi = eta (not in the paper; a standard
// accelerator of the same solve).  With even extents every hop joins sites of
// opposite parity (x+y+z+t mod 2), so with H = the hopping part of D,
//   D = [[A_ee, H_eo], [H_oe, A_oo]],
//   Dhat = A_ee - H_eo A_oo^{-1} H_oe          (Schur complement, even sites)
//   Dhat phi_e = eta_e - H_eo A_oo^{-1} eta_o,
//   phi_o = A_oo^{-1} (eta_o - H_oe phi_e).
// A^{-1} is the per-site inverse of the two 6x6 Hermitian site-term blocks,
// built once per (kappa, c_SW).
//
// Half fields hold the sites of one parity: in the device order the sites
// 2h and 2h + 1 differ only in the lowest bit of x (the column cross-section
// c_x is even when L_x is), so exactly one of them has each parity, and the
// site of parity p is stored at half index h.  A half field is a spinor field
// of V/2 sites in the usual tiled layout.
#include "wcl_device.h"
#include "wcl_kernels.h"

// full index and coordinates of half site h of parity p
WCL_DEV int eo_full(const Geom& g, int h, int p, int x[4]) {
    int i = 2 * h;
    geom_coords(g, i, x);
    if (((x[0] + x[1] + x[2] + x[3]) & 1) != p) {
        ++i;
        x[0] += 1;   // the partner differs in the lowest bit of x only (x even -> x + 1)
    }
    return i;
}

// acc = H in at full site i: the eight hops, reading the neighbours (all of
// the other parity) from the half field `in`, two-deep load pipeline.
template <int P, typename T>
WCL_DEV void eo_hops(const EoArgs& a, const char* in, int i, const int x[4], T acc[24]) {
    int nbr[8], lnk[8];
    T ph[8];
    hop_sites(a.g, i, x, nbr, lnk, ph);
    const T mk = T(-a.kappa);
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = T(0);
    T s0[24], u0[18], s1[24], u1[18];
    SpinorIO<P>::load(in, a.Vh, nbr[0] >> 1, s0);
    GaugeIO<P>::template load_raw<true>(a.gauge, a.g.V, 0, lnk[0], u0);
#define WCL_EHOP(K, SC, UC, SN, UN)                                                              \
    if ((K) < 7) {                                                                               \
        SpinorIO<P>::load(in, a.Vh, nbr[((K) + 1) & 7] >> 1, SN);                                 \
        GaugeIO<P>::template load_raw<true>(a.gauge, a.g.V, ((K) + 1) / 2, lnk[((K) + 1) & 7], UN); \
    }                                                                                            \
    hop_compute<(K) / 2, ((K) % 2) == 0>(SC, UC, mk * ph[K], acc);
    WCL_EHOP(0, s0, u0, s1, u1)
    WCL_EHOP(1, s1, u1, s0, u0)
    WCL_EHOP(2, s0, u0, s1, u1)
    WCL_EHOP(3, s1, u1, s0, u0)
    WCL_EHOP(4, s0, u0, s1, u1)
    WCL_EHOP(5, s1, u1, s0, u0)
    WCL_EHOP(6, s0, u0, s1, u1)
    WCL_EHOP(7, s1, u1, s0, u0)
#undef WCL_EHOP
}

// y = M z for the two packed Hermitian blocks of a clover-layout field at i;
// site = true: M = A = 1 + csw kappa C (from the clover field), else
// M = A^{-1} (from the site-term inverse)
template <int P, bool SITE, typename T>
WCL_DEV void eo_site(const EoArgs& a, int i, const T z[24], T y[24]) {
    const T ck = T(a.csw * a.kappa);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        T c[36], w[12];
        CloverBlk<P>::template load<true>(SITE ? a.clover : a.ainv, a.g.V, i, b, c);
        herm6_apply(c, z + 12 * b, w);
#pragma unroll
        for (int j = 0; j < 12; ++j) y[12 * b + j] = SITE ? fmad(ck, w[j], z[12 * b + j]) : w[j];
    }
}

// One kernel for every step of the reduction; half sites of parity a.parity,
// one per lane, right-hand side from the workgroup index:
//   EO_INV     out_h = A^{-1} H in                 (A_oo^{-1} H_oe psi_e)
//   EO_SCHUR   out_h = A in2_h - H in              (Dhat psi_e, with in = A_oo^{-1} H_oe psi_e)
//              epilogue DS_AXPY: out_h = y_h - that; DS_DOT: partials of <a_h, out_h>, |out_h|^2
//   EO_PREP    out_h = y(i) - H in                 (eta_e - H_eo A_oo^{-1} eta_o; y full)
//   EO_RECON   out(i) = A^{-1} (y(i) - H in)       (phi_o into the full field)
//   EO_SITEINV out_h = A^{-1} y(i)                 (A_oo^{-1} eta_o)
//   EO_EXTRACT out_h = y(i)
//   EO_INSERT  out(i) = in2_h                      (phi_e into the full field)
//   EO_ZERO    out(i) = 0
template <int P, int MODE, int EPI>
__global__ __launch_bounds__(256) void k_eo(EoArgs a) {
    using T = typename Real<P>::T;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int rhs = lb % a.nrhs, tile = lb / a.nrhs;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int h = tile * 256 + threadIdx.x;
    const bool active = h < a.Vh;
    T acc[24];
    if (active) {
        int x[4];
        const int i = eo_full(a.g, h, a.parity, x);
        const char* in = (const char*)a.in + rhs * a.in_stride;
        const char* y = (const char*)a.y + rhs * a.y_stride;
        char* out = (char*)a.out + rhs * a.out_stride;
        if constexpr (MODE == EO_INV) {
            T w[24];
            eo_hops<P>(a, in, i, x, w);
            eo_site<P, false>(a, i, w, acc);
            SpinorIO<P>::store(out, a.Vh, h, acc);
        } else if constexpr (MODE == EO_SCHUR) {
            T w[24], s[24];
            eo_hops<P>(a, in, i, x, w);
            SpinorIO<P>::load((const char*)a.in2 + rhs * a.in2_stride, a.Vh, h, s);
            eo_site<P, true>(a, i, s, acc);
#pragma unroll
            for (int k = 0; k < 24; ++k) acc[k] -= w[k];
            if constexpr (EPI == DS_AXPY) {
                SpinorIO<P>::load(y, a.Vh, h, s);
#pragma unroll
                for (int k = 0; k < 24; ++k) acc[k] = s[k] - acc[k];
            }
            SpinorIO<P>::store(out, a.Vh, h, acc);
        } else if constexpr (MODE == EO_PREP || MODE == EO_RECON) {
            T w[24], s[24];
            eo_hops<P>(a, in, i, x, w);
            SpinorIO<P>::load(y, a.g.V, i, s);
#pragma unroll
            for (int k = 0; k < 24; ++k) s[k] -= w[k];
            if constexpr (MODE == EO_PREP) {
                SpinorIO<P>::store(out, a.Vh, h, s);
            } else {
                eo_site<P, false>(a, i, s, acc);
                SpinorIO<P>::store(out, a.g.V, i, acc);
            }
        } else if constexpr (MODE == EO_SITEINV) {
            T s[24];
            SpinorIO<P>::load(y, a.g.V, i, s);
            eo_site<P, false>(a, i, s, acc);
            SpinorIO<P>::store(out, a.Vh, h, acc);
        } else if constexpr (MODE == EO_EXTRACT) {
            SpinorIO<P>::load(y, a.g.V, i, acc);
            SpinorIO<P>::store(out, a.Vh, h, acc);
        } else if constexpr (MODE == EO_INSERT) {
            SpinorIO<P>::load((const char*)a.in2 + rhs * a.in2_stride, a.Vh, h, acc);
            SpinorIO<P>::store(out, a.g.V, i, acc);
        } else {
#pragma unroll
            for (int k = 0; k < 24; ++k) acc[k] = T(0);
            SpinorIO<P>::store(out, a.g.V, i, acc);
        }
    }
    if constexpr (MODE == EO_SCHUR && EPI == DS_DOT) {
        double d[3] = {0.0, 0.0, 0.0};
        if (active) {
            T v[24];
            SpinorIO<P>::load((const char*)a.a + rhs * a.a_stride, a.Vh, h, v);
            site_dot3(v, acc, d);
        }
        block_reduce3(d, a.partial + 3 * ((size_t)tile + (size_t)rhs * (gridDim.x / a.nrhs)));
    }
}

int eo_partials_per_rhs(int Vh) { return (Vh + 255) / 256; }

template <int P, int MODE, int EPI>
static int launch_eo_t(const EoArgs& a, hipStream_t st) {
    const int tiles = (a.Vh + 255) / 256;
    k_eo<P, MODE, EPI><<<tiles * a.nrhs, 256, 0, st>>>(a);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_eo(const EoArgs& a, int prec, int mode, int epi, hipStream_t st) {
    if (a.g.V % 2 || a.Vh * 2 != a.g.V) {
        wcl_set_error("even-odd: half volume %d does not match the lattice", a.Vh);
        return WCL_EINVAL;
    }
#define WCL_EO(P)                                                                              \
    if (prec == P) {                                                                           \
        switch (mode) {                                                                        \
            case EO_INV: return launch_eo_t<P, EO_INV, DS_PLAIN>(a, st);                       \
            case EO_SCHUR:                                                                     \
                return epi == DS_DOT    ? launch_eo_t<P, EO_SCHUR, DS_DOT>(a, st)              \
                       : epi == DS_AXPY ? launch_eo_t<P, EO_SCHUR, DS_AXPY>(a, st)             \
                                        : launch_eo_t<P, EO_SCHUR, DS_PLAIN>(a, st);           \
            case EO_PREP: return launch_eo_t<P, EO_PREP, DS_PLAIN>(a, st);                     \
            case EO_RECON: return launch_eo_t<P, EO_RECON, DS_PLAIN>(a, st);                   \
            case EO_SITEINV: return launch_eo_t<P, EO_SITEINV, DS_PLAIN>(a, st);               \
            case EO_EXTRACT: return launch_eo_t<P, EO_EXTRACT, DS_PLAIN>(a, st);               \
            case EO_INSERT: return launch_eo_t<P, EO_INSERT, DS_PLAIN>(a, st);                 \
            case EO_ZERO: return launch_eo_t<P, EO_ZERO, DS_PLAIN>(a, st);                     \
            default: break;                                                                    \
        }                                                                                      \
    }
    WCL_EO(WCL_F64)
    WCL_EO(WCL_F32)
#undef WCL_EO
    wcl_set_error("even-odd: unsupported precision %d or mode %d", prec, mode);
    return WCL_EINVAL;
}
