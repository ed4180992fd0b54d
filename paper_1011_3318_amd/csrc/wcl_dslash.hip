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

#ifndef WCL_PIPE_DEPTH
#define WCL_PIPE_DEPTH 2
#endif

// A psi at site i, one 6x6 clover block at a time: acc = psi + c_sw kappa C psi.
// NT: non-temporal loads of the links and clover (fields streamed once per
// launch); cached loads when the launch's data fits the Infinity Cache or
// several right-hand sides share the fields.
template <bool NT, int GP, int SPI, typename T>
WCL_DEV void clover_site(const DslashArgs& a, const char* in, int i, T acc[24]) {
    const int V = a.g.V;
    const T ck = T(a.csw * a.kappa);
    T s[24];
    SpinorIO<SPI>::load(in, V, i, s);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        T c[36], y[12];
        CloverBlk<GP>::template load<NT>(a.clover, V, i, b, c);
        herm6_apply(c, s + 12 * b, y);
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[12 * b + j] = s[12 * b + j] + ck * y[j];
    }
}

// Hops K..7 of a D-deep software pipeline: register slot K % D holds the
// neighbour spinor and link of hop K (requested D hops earlier); once hop K
// is computed the slot is refilled with hop K + D, so D - 1 hops' loads are
// in flight while a hop is computed.
// The spinors are held as stored with their scale in ss (1 but for FP16);
// the hop is linear, so the scale joins the hop's factor.
template <int K, int D, bool NT, int GP, int SPI, typename S, typename T>
WCL_DEV void hop_chain(const DslashArgs& a, const char* in, const int nbr[8], const int lnk[8], const T ph[8], T mk,
                       S sb[D][24], T ss[D], T ub[D][18], T acc[24]) {
    if constexpr (K < 8) {
        constexpr int slot = K % D;
        hop_compute<K / 2, (K % 2) == 0>(sb[slot], ub[slot], mk * ph[K] * ss[slot], acc);
        if constexpr (K + D < 8) {
            ss[slot] = SpinorIO<SPI>::load_s(in, a.g.V, nbr[K + D], sb[slot]);
            GaugeIO<GP>::template load_raw<NT>(a.gauge, a.g.V, (K + D) / 2, lnk[K + D], ub[slot]);
        }
        hop_chain<K + 1, D, NT, GP, SPI>(a, in, nbr, lnk, ph, mk, sb, ss, ub, acc);
    }
}

// (D psi)(x): the site term first, then the eight hops in the order
// (x+, x-, y+, y-, z+, z-, t+, t-) through the load pipeline.
template <bool NT, int GP, int SPI, typename T>
WCL_DEV void dslash_site(const DslashArgs& a, const char* in, int i, T acc[24]) {
    constexpr int D = WCL_PIPE_DEPTH;
    int x[4], nbr[8], lnk[8];
    T ph[8];
    geom_coords(a.g, i, x);
    hop_sites(a.g, i, x, nbr, lnk, ph);
    typename SpinorIO<SPI>::Stored sb[D][24];
    T ss[D], ub[D][18];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        ss[k] = SpinorIO<SPI>::load_s(in, a.g.V, nbr[k], sb[k]);
        GaugeIO<GP>::template load_raw<NT>(a.gauge, a.g.V, k / 2, lnk[k], ub[k]);
    }
    clover_site<NT, GP, SPI>(a, in, i, acc);
    hop_chain<0, D, NT, GP, SPI>(a, in, nbr, lnk, ph, T(-a.kappa), sb, ss, ub, acc);
}

// FP16 storage: the same pipeline on binary16 pairs (the neighbour spinor as
// stored and its scale, the link with row 2 rebuilt from exact binary16
// products), every hop formed by packed binary16 projections and v_dot2
// products with FP32 sums (hop_compute16).
template <int K, int D, bool NT>
WCL_DEV void hop_chain16(const DslashArgs& a, const char* in, const int nbr[8], const int lnk[8], const float ph[8],
                         float mk, float z, h2v sb[D][12], float ss[D], h2v ub[D][9], float acc[24]) {
    if constexpr (K < 8) {
        constexpr int slot = K % D;
        hop_compute16<K / 2, (K % 2) == 0>(sb[slot], ub[slot], mk * ph[K] * ss[slot], z, acc);
        if constexpr (K + D < 8) {
            ss[slot] = load_spinor16(in, a.g.V, nbr[K + D], sb[slot]);
            load_link16<NT>(a.gauge, a.g.V, (K + D) / 2, lnk[K + D], z, ub[slot]);
        }
        hop_chain16<K + 1, D, NT>(a, in, nbr, lnk, ph, mk, z, sb, ss, ub, acc);
    }
}

template <bool NT>
WCL_DEV void dslash_site16(const DslashArgs& a, const char* in, int i, float acc[24]) {
    constexpr int D = WCL_PIPE_DEPTH;
    int x[4], nbr[8], lnk[8];
    float ph[8];
    geom_coords(a.g, i, x);
    hop_sites(a.g, i, x, nbr, lnk, ph);
    float z = 0.f;   // opaque zero: the first product of every chain stays a v_dot2
    asm volatile("" : "+v"(z));
    h2v sb[D][12], ub[D][9];
    float ss[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        ss[k] = load_spinor16(in, a.g.V, nbr[k], sb[k]);
        load_link16<NT>(a.gauge, a.g.V, k / 2, lnk[k], z, ub[k]);
    }
    h2v x16[12];
    const float sc = load_spinor16(in, a.g.V, i, x16);
    clover_site16<NT>(a.clover, a.g.V, i, x16, sc, (float)(a.csw * a.kappa), z, acc);
    hop_chain16<0, D, NT>(a, in, nbr, lnk, ph, (float)(-a.kappa), z, sb, ss, ub, acc);
}

template <int GP, int SPI, int SPO, int EPI, int SPY, bool NT>
#ifndef WCL_DSLASH_MINWAVES
#define WCL_DSLASH_MINWAVES 1
#endif
__global__ __launch_bounds__(256, WCL_DSLASH_MINWAVES) void k_dslash(DslashArgs a) {
    using T = typename Real<GP>::T;
    static_assert((GP == WCL_F64) == (SPI == WCL_F64), "FP64 arithmetic needs FP64 spinors and links");
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int rhs = lb % a.nrhs;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int i = (lb / a.nrhs) * 256 + threadIdx.x;
    const bool active = i < a.g.V;
    T acc[24];
    if (active) {
        if constexpr (GP == WCL_F16 && SPI == WCL_F16)
            dslash_site16<NT>(a, (const char*)a.in + rhs * a.in_stride, i, acc);
        else
            dslash_site<NT, GP, SPI>(a, (const char*)a.in + rhs * a.in_stride, i, acc);
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
            site_dot3(v, acc, d);
        }
        block_reduce3(d, a.partial + 3 * (size_t)((lb / a.nrhs) + (size_t)rhs * (gridDim.x / a.nrhs)));
    }
}

// ------------------------------------- x/y neighbours from the workgroup
// With whole x rows in a wavefront (c_x = L_x lanes, c_x | 64) and 256 / c_x
// consecutive y rows of one (z, t, column) slice per workgroup, the x and y
// hops need no neighbour loads.  Each lane projects its own spinor twice per
// direction: P- psi(s) is what s - mu needs for its forward hop, and
// U_mu(s)^dag P+ psi(s) (built with the link the lane loads anyway for its
// own forward hop) is what s + mu needs for its backward hop.  x hops pick
// these up with a cross-lane permute inside the wavefront, y hops through
// LDS; only the first and last rows of a workgroup load their y neighbour
// from memory, unless the workgroup spans the whole y extent and wraps.
// z and t hops keep the pipelined neighbour loads of k_dslash.
bool dslash_xy_layout(const Geom& g) {
    const int cx = g.c[0];
    if (cx != g.L[0] || cx < 2 || 64 % cx != 0) return false;
    return g.c[1] % (256 / cx) == 0;
}

// Keeps the scheduler from hoisting the next phase's loads above this point
// (which would hold them in registers through the current phase).
#define WCL_PHASE() __builtin_amdgcn_sched_barrier(0)

// Forces v to be computed here: arithmetic is otherwise free to sink below
// a barrier, holding its loaded operands in registers across it.
template <typename T, int N>
WCL_DEV void pin_values(T (&v)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) asm volatile("" : "+v"(v[k]));
}

// v as held by lane `src` of this wavefront
WCL_DEV float lane_fetch(float v, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
WCL_DEV double lane_fetch(double v, int src) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

#ifndef WCL_XY_MINWAVES
#define WCL_XY_MINWAVES 2
#endif
template <int GP, int SPI, int SPO, int EPI, int SPY, bool NT>
__global__ __launch_bounds__(256, WCL_XY_MINWAVES) void k_dslash_xy(DslashArgs a) {
    using T = typename Real<GP>::T;
    static_assert((GP == WCL_F64) == (SPI == WCL_F64), "FP64 arithmetic needs FP64 spinors and links");
    __shared__ T hf_y[12][256];   // P- psi(s): forward y hop of the row below
    __shared__ T hb_y[12][256];   // U_y(s)^dag P+ psi(s): backward y hop of the row above
    const Geom& g = a.g;
    const int V = g.V;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int rhs = lb % a.nrhs;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int t = threadIdx.x;
    const int i = (lb / a.nrhs) * 256 + t;   // V % 256 == 0: every lane has a site
    const char* in = (const char*)a.in + rhs * a.in_stride;
    const int R = g.c[0], NR = 256 / R;      // lanes per x row, rows per workgroup
    const int r = t >> g.lc[0];
    int x[4], nbr[8], lnk[8];
    T ph[8];
    geom_coords(g, i, x);
    hop_sites(g, i, x, nbr, lnk, ph);
    const T mk = T(-a.kappa);

    T psi[24], uy[18];
    SpinorIO<SPI>::load(in, V, i, psi);
    GaugeIO<GP>::template load<NT>(a.gauge, V, 1, i, uy);
    {
        T h[12], w[12];
        spin_project<1, true>(psi, h);
#pragma unroll
        for (int k = 0; k < 12; ++k) hf_y[k][t] = h[k];
        spin_project<1, false>(psi, h);
        su3_apply2<true>(uy, h, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) hb_y[k][t] = w[k];
    }
    WCL_PHASE();

    // x hops through the wavefront
    T wf[12], wb[12];
    {
        T ux[18], h[12], hr[12];
        GaugeIO<GP>::template load<NT>(a.gauge, V, 0, i, ux);
        const int lane = t & 63, row0 = lane & ~(R - 1);
        const int up = row0 | ((lane + 1) & (R - 1)), dn = row0 | ((lane + R - 1) & (R - 1));
        spin_project<0, true>(psi, h);
#pragma unroll
        for (int k = 0; k < 12; ++k) hr[k] = lane_fetch(h[k], up);
        su3_apply2<false>(ux, hr, wf);
        spin_project<0, false>(psi, h);
        su3_apply2<true>(ux, h, hr);
#pragma unroll
        for (int k = 0; k < 12; ++k) wb[k] = lane_fetch(hr[k], dn);
    }
    WCL_PHASE();

    T acc[24];
    if constexpr (GP == WCL_F16) {
        float z = 0.f;
        asm volatile("" : "+v"(z));
        clover_site_f16<NT>(a.clover, V, i, psi, (float)(a.csw * a.kappa), z, acc);
        WCL_PHASE();
    } else {
        const T ck = T(a.csw * a.kappa);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            T c[36], y[12];
            CloverBlk<GP>::template load<NT>(a.clover, V, i, b, c);
            herm6_apply(c, psi + 12 * b, y);
#pragma unroll
            for (int j = 0; j < 12; ++j) acc[12 * b + j] = psi[12 * b + j] + ck * y[j];
            WCL_PHASE();
        }
    }
    spin_accumulate<0, true>(wf, mk * ph[0], acc);
    spin_accumulate<0, false>(wb, mk * ph[1], acc);
    pin_values(acc);   // finish the site term and x hops before the barrier

    // y hops from LDS; the edge rows of a workgroup that does not span y load
    __syncthreads();
    const bool wrap = NR == g.L[1];
    {
        T h[12], w[12];
        if (r + 1 < NR || wrap) {
            const int src = r + 1 < NR ? t + R : t - (NR - 1) * R;
#pragma unroll
            for (int k = 0; k < 12; ++k) h[k] = hf_y[k][src];
        } else {
            T s[24];
            SpinorIO<SPI>::load(in, V, nbr[2], s);
            spin_project<1, true>(s, h);
        }
        su3_apply2<false>(uy, h, w);
        spin_accumulate<1, true>(w, mk * ph[2], acc);
    }
    {
        T w[12];
        if (r > 0 || wrap) {
            const int src = r > 0 ? t - R : t + (NR - 1) * R;
#pragma unroll
            for (int k = 0; k < 12; ++k) w[k] = hb_y[k][src];
        } else {
            T s[24], u[18], h[12];
            SpinorIO<SPI>::load(in, V, nbr[3], s);
            GaugeIO<GP>::template load<NT>(a.gauge, V, 1, lnk[3], u);
            spin_project<1, false>(s, h);
            su3_apply2<true>(u, h, w);
        }
        spin_accumulate<1, false>(w, mk * ph[3], acc);
    }

    WCL_PHASE();
    // z and t hops: the pipelined neighbour loads of k_dslash
    constexpr int D = WCL_PIPE_DEPTH;
    typename SpinorIO<SPI>::Stored sb[D][24];
    T ss[D], ub[D][18];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        ss[(4 + k) % D] = SpinorIO<SPI>::load_s(in, V, nbr[4 + k], sb[(4 + k) % D]);
        GaugeIO<GP>::template load_raw<NT>(a.gauge, V, (4 + k) / 2, lnk[4 + k], ub[(4 + k) % D]);
    }

    hop_chain<4, D, NT, GP, SPI>(a, in, nbr, lnk, ph, mk, sb, ss, ub, acc);

    if (EPI == DS_AXPY) {
        T y[24];
        SpinorIO<SPY>::load((const char*)a.y + rhs * a.y_stride, V, i, y);
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = y[k] - acc[k];
    }
    SpinorIO<SPO>::store((char*)a.out + rhs * a.out_stride, V, i, acc);
    if (EPI == DS_DOT) {
        double d[3] = {0.0, 0.0, 0.0};
        T v[24];
        SpinorIO<SPO>::load((const char*)a.a + rhs * a.a_stride, V, i, v);
        site_dot3(v, acc, d);
        block_reduce3(d, a.partial + 3 * (size_t)((lb / a.nrhs) + (size_t)rhs * (gridDim.x / a.nrhs)));
    }
}

// The exchange kernel for FP16 storage on binary16 pairs: the lanes exchange
// conj(P- psi(s)) as stored pairs (6 words) and U_mu(s)^dag P+ psi(s) in FP32 (12
// words), each with the sender's scale, which joins the receiver's hop
// factor; the products are v_dot2 on pairs, the accumulation FP32.
WCL_DEV h2v lane_fetch16(h2v v, int src) {
    return __builtin_bit_cast(h2v, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
}

template <int SPO, int EPI, int SPY, bool NT>
__global__ __launch_bounds__(256, WCL_XY_MINWAVES) void k_dslash_xy16(DslashArgs a) {
    __shared__ h2v hf_y[6][256];     // conj of P- psi(s), stored pairs: forward y hop of the row below
    __shared__ float hb_y[12][256];  // U_y(s)^dag P+ psi(s) (unscaled): backward y hop of the row above
    __shared__ float sc_y[256];      // psi(s)'s scale
    const Geom& g = a.g;
    const int V = g.V;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int rhs = lb % a.nrhs;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int t = threadIdx.x;
    const int i = (lb / a.nrhs) * 256 + t;   // V % 256 == 0: every lane has a site
    const char* in = (const char*)a.in + rhs * a.in_stride;
    const int R = g.c[0], NR = 256 / R;      // lanes per x row, rows per workgroup
    const int r = t >> g.lc[0];
    int x[4], nbr[8], lnk[8];
    float ph[8];
    geom_coords(g, i, x);
    hop_sites(g, i, x, nbr, lnk, ph);
    const float mk = (float)(-a.kappa);
    float z = 0.f;   // opaque zero: the first product of every chain stays a v_dot2
    asm volatile("" : "+v"(z));

    h2v psi[12], uy[9];
    const float sc = load_spinor16(in, V, i, psi);
    load_link16<NT>(a.gauge, V, 1, i, z, uy);
    {
        h2v ha[6], hb[6];
        float w[12];
        spin_project16<1, true, false>(psi, ha, hb);
#pragma unroll
        for (int k = 0; k < 6; ++k) hf_y[k][t] = ha[k];
        sc_y[t] = sc;
        spin_project16<1, false, true>(psi, ha, hb);
        su3_apply16<true>(uy, ha, hb, z, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) hb_y[k][t] = w[k];
    }
    WCL_PHASE();

    // x hops through the wavefront
    float wf[12], wb[12], s_up, s_dn;
    {
        h2v ux[9], ha[6], hb[6], hr[6], hrs[6];
        load_link16<NT>(a.gauge, V, 0, i, z, ux);
        const int lane = t & 63, row0 = lane & ~(R - 1);
        const int up = row0 | ((lane + 1) & (R - 1)), dn = row0 | ((lane + R - 1) & (R - 1));
        // conj h travels; swp h = i conj h
        spin_project16<0, true, false>(psi, ha, hb);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            hr[k] = lane_fetch16(ha[k], up);
            hrs[k] = mul_i(hr[k]);
        }
        s_up = lane_fetch(sc, up);
        s_dn = lane_fetch(sc, dn);
        su3_apply16<false>(ux, hr, hrs, z, wf);
        float w[12];
        spin_project16<0, false, true>(psi, ha, hb);
        su3_apply16<true>(ux, ha, hb, z, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) wb[k] = lane_fetch(w[k], dn);
    }
    WCL_PHASE();

    float acc[24];
    clover_site16<NT>(a.clover, V, i, psi, sc, (float)(a.csw * a.kappa), z, acc);
    WCL_PHASE();
    spin_accumulate<0, true>(wf, mk * ph[0] * s_up, acc);
    spin_accumulate<0, false>(wb, mk * ph[1] * s_dn, acc);
    pin_values(acc);   // finish the site term and x hops before the barrier

    // y hops from LDS; the edge rows of a workgroup that does not span y load
    __syncthreads();
    const bool wrap = NR == g.L[1];
    {
        h2v ha[6], hb[6];
        float w[12], sy;
        if (r + 1 < NR || wrap) {
            const int src = r + 1 < NR ? t + R : t - (NR - 1) * R;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                ha[k] = hf_y[k][src];
                hb[k] = mul_i(ha[k]);
            }
            sy = sc_y[src];
        } else {
            h2v sn[12];
            sy = load_spinor16(in, V, nbr[2], sn);
            spin_project16<1, true, false>(sn, ha, hb);
        }
        su3_apply16<false>(uy, ha, hb, z, w);
        spin_accumulate<1, true>(w, mk * ph[2] * sy, acc);
    }
    {
        float w[12], sy;
        if (r > 0 || wrap) {
            const int src = r > 0 ? t - R : t + (NR - 1) * R;
#pragma unroll
            for (int k = 0; k < 12; ++k) w[k] = hb_y[k][src];
            sy = sc_y[src];
        } else {
            h2v sn[12], u[9], ha[6], hb[6];
            sy = load_spinor16(in, V, nbr[3], sn);
            load_link16<NT>(a.gauge, V, 1, lnk[3], z, u);
            spin_project16<1, false, true>(sn, ha, hb);
            su3_apply16<true>(u, ha, hb, z, w);
        }
        spin_accumulate<1, false>(w, mk * ph[3] * sy, acc);
    }

    WCL_PHASE();
    // z and t hops: the pipelined neighbour loads
    constexpr int D = WCL_PIPE_DEPTH;
    h2v sb[D][12], ub[D][9];
    float ss[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        ss[(4 + k) % D] = load_spinor16(in, V, nbr[4 + k], sb[(4 + k) % D]);
        load_link16<NT>(a.gauge, V, (4 + k) / 2, lnk[4 + k], z, ub[(4 + k) % D]);
    }
    hop_chain16<4, D, NT>(a, in, nbr, lnk, ph, mk, z, sb, ss, ub, acc);

    if (EPI == DS_AXPY) {
        float y[24];
        SpinorIO<SPY>::load((const char*)a.y + rhs * a.y_stride, V, i, y);
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = y[k] - acc[k];
    }
    SpinorIO<SPO>::store((char*)a.out + rhs * a.out_stride, V, i, acc);
    if (EPI == DS_DOT) {
        double d[3] = {0.0, 0.0, 0.0};
        float v[24];
        SpinorIO<SPO>::load((const char*)a.a + rhs * a.a_stride, V, i, v);
        site_dot3(v, acc, d);
        block_reduce3(d, a.partial + 3 * (size_t)((lb / a.nrhs) + (size_t)rhs * (gridDim.x / a.nrhs)));
    }
}

// ------------------------------------------------ several lanes per site
// Stores the float groups of s that belong to `lane` of LPS lanes.
template <int P>
struct SpinorPart;
template <>
struct SpinorPart<WCL_F64> {
    template <int LPS>
    WCL_DEV static void store(void* base, int V, int i, const double s[24], int lane) {
        d2v* p = (d2v*)base;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            if (k % LPS == lane) st_nt(p + tix(k, i, 12), d2v{s[2 * k], s[2 * k + 1]});
    }
};
template <>
struct SpinorPart<WCL_F32> {
    template <int LPS>
    WCL_DEV static void store(void* base, int V, int i, const float s[24], int lane) {
        f4v* p = (f4v*)base;
#pragma unroll
        for (int g = 0; g < 6; ++g)
            if (g % LPS == lane) st_nt(p + tix(g, i, 6), f4v{s[4 * g], s[4 * g + 1], s[4 * g + 2], s[4 * g + 3]});
    }
};
template <>
struct SpinorPart<WCL_F16> {
    template <int LPS>
    WCL_DEV static void store(void* base, int V, int i, const float s[24], int lane) {
        float m = 0.f;
#pragma unroll
        for (int j = 0; j < 24; ++j) m = fmaxf(m, fabsf(s[j]));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        h8v* p = (h8v*)base;
#pragma unroll
        for (int g = 0; g < 3; ++g)
            if (g % LPS == lane) {
                f8v v;
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = s[8 * g + j] * inv;
                st_nt(p + tix(g, i, 3), __builtin_convertvector(v, h8v));
            }
        if (lane == LPS - 1) st_nt((float*)((char*)base + half_spinor_scale_offset(V)) + i, m);
    }
};

// LPS lanes per site: lane j takes directions j*(4/LPS) .. and, for j < 2,
// clover block j; the partial sums are added across the lanes with xor
// shuffles (identical on every lane, so the result is deterministic).
template <int GP, int SPI, int SPO, int EPI, int SPY, int LPS>
__global__ __launch_bounds__(256) void k_dslash_ml(DslashArgs a) {
    using T = typename Real<GP>::T;
    static_assert((GP == WCL_F64) == (SPI == WCL_F64), "FP64 arithmetic needs FP64 spinors and links");
    constexpr int SPW = 256 / LPS, DPL = 4 / LPS;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int rhs = lb % a.nrhs;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int tile = lb / a.nrhs;
    const int lane = threadIdx.x % LPS;
    const int i = tile * SPW + threadIdx.x / LPS;
    const bool active = i < a.g.V;
    const int V = a.g.V;
    T acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = T(0);
    const char* in = (const char*)a.in + rhs * a.in_stride;
    if (active) {
        int x[4];
        geom_coords(a.g, i, x);
        if (lane < 2) {
            T s[24], c[36], xs[12], y[12];
            SpinorIO<SPI>::load(in, V, i, s);
            CloverBlk<GP>::load(a.clover, V, i, lane, c);
#pragma unroll
            for (int j = 0; j < 12; ++j) xs[j] = lane ? s[12 + j] : s[j];
            herm6_apply(c, xs, y);
            const T ck = T(a.csw * a.kappa);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const T v = xs[j] + ck * y[j];
                acc[j] = lane ? T(0) : v;
                acc[12 + j] = lane ? v : T(0);
            }
        }
        const T mk = T(-a.kappa);
#pragma unroll
        for (int m = 0; m < DPL; ++m) {
            const int mu = lane * DPL + m;
            const int xm = pick(x, mu), Lm = pick(a.g.L, mu);
            const T bcm = T(pick(a.g.bc, mu));
            T s[24], h[12], w[12], u[18];
            {   // forward: (1 - gamma_mu) U_mu(x) psi(x + mu)
                int y[4] = {x[0], x[1], x[2], x[3]};
                const bool wrap = xm + 1 == Lm;
                put(y, mu, wrap ? 0 : xm + 1);
                SpinorIO<SPI>::load(in, V, geom_index(a.g, y), s);
                const RtCoef kf = rt_coef(mu, true);
                spin_project_rt(kf, s, h);
                GaugeIO<GP>::load(a.gauge, V, mu, i, u);
                su3_apply2<false>(u, h, w);
                spin_accumulate_rt(kf, w, wrap ? mk * bcm : mk, acc);
            }
            {   // backward: (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
                int y[4] = {x[0], x[1], x[2], x[3]};
                const bool wrap = xm == 0;
                put(y, mu, wrap ? Lm - 1 : xm - 1);
                const int jb = geom_index(a.g, y);
                SpinorIO<SPI>::load(in, V, jb, s);
                const RtCoef kb = rt_coef(mu, false);
                spin_project_rt(kb, s, h);
                GaugeIO<GP>::load(a.gauge, V, mu, jb, u);
                su3_apply2<true>(u, h, w);
                spin_accumulate_rt(kb, w, wrap ? mk * bcm : mk, acc);
            }
        }
    }
#pragma unroll
    for (int off = 1; off < LPS; off <<= 1)
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] += __shfl_xor(acc[k], off, 64);
    if (active) {
        if (EPI == DS_AXPY) {
            T y[24];
            SpinorIO<SPY>::load((const char*)a.y + rhs * a.y_stride, V, i, y);
#pragma unroll
            for (int k = 0; k < 24; ++k) acc[k] = y[k] - acc[k];
        }
        SpinorPart<SPO>::template store<LPS>((char*)a.out + rhs * a.out_stride, V, i, acc, lane);
    }
    if (EPI == DS_DOT) {
        double d[3] = {0.0, 0.0, 0.0};
        if (active && lane == 0) {
            T v[24];
            SpinorIO<SPO>::load((const char*)a.a + rhs * a.a_stride, V, i, v);
            site_dot3(v, acc, d);
        }
        block_reduce3(d, a.partial + 3 * (size_t)(tile + (size_t)rhs * (gridDim.x / a.nrhs)));
    }
}

static size_t dslash_launch_bytes(int V, int gp, int spi, int spo) {
    return gauge_bytes(gp, V) + clover_bytes(gp, V) + spinor_rhs_bytes(spi, V) + spinor_rhs_bytes(spo, V);
}

template <int GP, int SPI, int SPO, int EPI, int SPY>
static int launch_t(const DslashArgs& a, hipStream_t st) {
    const int tiles = dslash_partials_per_rhs(a.g.V, a.lps);
    switch (a.lps) {
        case 2: k_dslash_ml<GP, SPI, SPO, EPI, SPY, 2><<<tiles * a.nrhs, 256, 0, st>>>(a); break;
        case 4: k_dslash_ml<GP, SPI, SPO, EPI, SPY, 4><<<tiles * a.nrhs, 256, 0, st>>>(a); break;
        default: {
            // non-temporal field loads only for one rhs streaming more than the
            // 256 MB Infinity Cache holds
            const bool nt = a.nrhs == 1 && dslash_launch_bytes(a.g.V, GP, SPI, SPO) > (256u << 20);
            if (dslash_xy_layout(a.g)) {
                if constexpr (GP == WCL_F16 && SPI == WCL_F16) {
                    if (nt) k_dslash_xy16<SPO, EPI, SPY, true><<<tiles * a.nrhs, 256, 0, st>>>(a);
                    else k_dslash_xy16<SPO, EPI, SPY, false><<<tiles * a.nrhs, 256, 0, st>>>(a);
                } else {
                    if (nt) k_dslash_xy<GP, SPI, SPO, EPI, SPY, true><<<tiles * a.nrhs, 256, 0, st>>>(a);
                    else k_dslash_xy<GP, SPI, SPO, EPI, SPY, false><<<tiles * a.nrhs, 256, 0, st>>>(a);
                }
            } else if (nt) {
                k_dslash<GP, SPI, SPO, EPI, SPY, true><<<tiles * a.nrhs, 256, 0, st>>>(a);
            } else {
                k_dslash<GP, SPI, SPO, EPI, SPY, false><<<tiles * a.nrhs, 256, 0, st>>>(a);
            }
            break;
        }
    }
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

// workgroups (= dot-product partial sums) per rhs for lps lanes per site
int dslash_partials_per_rhs(int V, int lps) {
    const int spw = 256 / (lps == 2 || lps == 4 ? lps : 1);
    return (V + spw - 1) / spw;
}

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
