// RAS domain solves (Sec. 2, Algorithm 1): projection P_{Omega'_i}, the
// Dirichlet domain operator D_{Omega'_i}, minimal-residual steps and the
// restriction R_{Omega_i}, for all domains and right-hand sides at once.
//
// Split path: the extended domains are stored one after another in an FP32
// workspace (float4 [6][NE] per rhs, NE = nblocks * ev).  Each workgroup
// covers 256 sites of one domain, so a domain can span several workgroups;
// every MR step is one launch of the domain operator (with per-workgroup
// partial sums of <q, rho>, <q, q>) followed by one update launch that adds
// the domain's partials in a fixed order.
#include "wcl_device.h"
#include "wcl_kernels.h"

// local coordinates of extended-domain site l, and its global coordinates
WCL_DEV void block_site(const Geom& g, const Blocks& B, int blk, int l, int lc[4], int x[4]) {
    int t = l, tb = blk;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        lc[mu] = t % B.e[mu];
        t /= B.e[mu];
        int bc = tb % B.nb[mu];
        tb /= B.nb[mu];
        int v = bc * B.b[mu] - B.s[mu] + lc[mu];
        x[mu] = v < 0 ? v + g.L[mu] : (v >= g.L[mu] ? v - g.L[mu] : v);
    }
}

WCL_DEV int local_index(const Blocks& B, const int lc[4]) {
    return lc[0] + B.e[0] * (lc[1] + B.e[1] * (lc[2] + B.e[2] * lc[3]));
}

WCL_DEV bool block_owned(const Blocks& B, const int lc[4]) {
    bool o = true;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) o = o && lc[mu] >= B.s[mu] && lc[mu] < B.s[mu] + B.b[mu];
    return o;
}

WCL_DEV void ws_load(const f4v* base, int NE, int e, float s[24]) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        f4v v = base[(size_t)q * NE + e];
        s[4 * q] = v.x;
        s[4 * q + 1] = v.y;
        s[4 * q + 2] = v.z;
        s[4 * q + 3] = v.w;
    }
}
WCL_DEV void ws_store(f4v* base, int NE, int e, const float s[24]) {
#pragma unroll
    for (int q = 0; q < 6; ++q) base[(size_t)q * NE + e] = f4v{s[4 * q], s[4 * q + 1], s[4 * q + 2], s[4 * q + 3]};
}

// Colour of a domain for the multiplicative iteration: parity of the sum of
// its block coordinates.
WCL_DEV int block_colour(const Blocks& B, int blk) {
    int c = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        c += blk % B.nb[mu];
        blk /= B.nb[mu];
    }
    return c & 1;
}

WCL_DEV bool skip_colour(const BlockArgs& a, int blk) { return a.colour >= 0 && block_colour(a.B, blk) != a.colour; }

// End of a domain solve at extended site l with solution xv:
//   whole: keep xv in the workspace x (the additive gather sums it);
//   else restriction to the owned sites: out (FP32) = xv, or out += xv when
//   accumulating over sweeps, and vj (storage precision) = xv when requested.
// zero = the domain was not solved in this pass (other colour): its owned
// sites get v = 0 (vj, and out unless accumulating).
template <int VP>
WCL_DEV void blk_finish(const BlockArgs& a, int rhs, int blk, int l, const float xv[24], bool zero) {
    if (a.whole) {
        ws_store((f4v*)a.x + rhs * a.ws_stride, a.NE, blk * a.B.ev + l, xv);
        return;
    }
    int lc[4], x[4];
    block_site(a.g, a.B, blk, l, lc, x);
    if (!block_owned(a.B, lc)) return;
    const int gi = geom_index(a.g, x);
    char* out = (char*)a.out + rhs * a.out_stride;
    float z[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) z[k] = zero ? 0.f : xv[k];
    if (a.accumulate) {
        if (!zero) {
            float o[24];
            SpinorIO<WCL_F32>::load(out, a.g.V, gi, o);
#pragma unroll
            for (int k = 0; k < 24; ++k) o[k] += z[k];
            SpinorIO<WCL_F32>::store(out, a.g.V, gi, o);
        }
    } else {
        SpinorIO<WCL_F32>::store(out, a.g.V, gi, z);
    }
    if (a.vj) SpinorIO<VP>::store((char*)a.vj + rhs * a.vj_stride, a.g.V, gi, z);
}

// Sum of the wpb partial triples of domain blk (fixed order).
WCL_DEV void domain_sum3(const double* part, const BlockArgs& a, int rhs, int blk, double s[3]) {
    const double* p = part + 3 * ((size_t)rhs * a.B.nblocks + blk) * a.wpb;
    s[0] = s[1] = s[2] = 0.0;
    for (int k = 0; k < a.wpb; ++k) {
        s[0] += p[3 * k];
        s[1] += p[3 * k + 1];
        s[2] += p[3 * k + 2];
    }
}

// projection: rho = P r on every extended site, x = 0.  BCG (truncated
// BiCGStab): also rhat = rho and the partial sums of <rhat, rho>.
template <int SRC, bool BCG>
__global__ __launch_bounds__(256) void k_blk_project(BlockArgs a) {
    const int per_rhs = a.B.nblocks * a.wpb;
    const int rhs = blockIdx.x / per_rhs;
    const int blk = (blockIdx.x % per_rhs) / a.wpb;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    if (skip_colour(a, blk)) return;
    const int wl = blockIdx.x % a.wpb;
    const int l = wl * 256 + threadIdx.x;
    double d[3] = {0.0, 0.0, 0.0};
    if (l < a.B.ev) {
        int lc[4], x[4];
        block_site(a.g, a.B, blk, l, lc, x);
        float s[24], z[24];
        SpinorIO<SRC>::load((const char*)a.src + rhs * a.src_stride, a.g.V, geom_index(a.g, x), s);
        const int e = blk * a.B.ev + l;
#pragma unroll
        for (int k = 0; k < 24; ++k) z[k] = 0.f;
        ws_store((f4v*)a.rho + rhs * a.ws_stride, a.NE, e, s);
        ws_store((f4v*)a.x + rhs * a.ws_stride, a.NE, e, z);
        if constexpr (BCG) {
            ws_store((f4v*)a.brh + rhs * a.ws_stride, a.NE, e, s);
            site_dot3(s, s, d);
        }
    }
    if constexpr (BCG) block_reduce3(d, a.bpart[0] + 3 * (((size_t)rhs * a.B.nblocks + blk) * a.wpb + wl));
}

// Workspace index of the neighbour of extended site lc in direction mu
// (forward or backward), or -1 when the hop leaves Omega' (Dirichlet).
WCL_DEV int blk_neighbour(const Geom& g, const Blocks& B, const int lc[4], int mu, bool fwd) {
    int ln[4] = {lc[0], lc[1], lc[2], lc[3]};
    const int e = B.e[mu];
    if (fwd) {
        ln[mu] += 1;
        if (ln[mu] == e) {
            if (e != g.L[mu]) return -1;
            ln[mu] = 0;
        }
    } else {
        ln[mu] -= 1;
        if (ln[mu] < 0) {
            if (e != g.L[mu]) return -1;
            ln[mu] = e - 1;
        }
    }
    return local_index(B, ln);
}

// rho of workspace site n and rows 0,1 of link U_mu at global site li
// (ordinary cached loads: every MR step re-reads them)
template <int GP>
WCL_DEV void blk_fetch(const BlockArgs& a, const f4v* rho, int base, int n, int mu, int li, float s[24], float u[18]) {
    if (n >= 0) {
        ws_load(rho, a.NE, base + n, s);
        GaugeIO<GP>::template load_raw<false>(a.gauge, a.g.V, mu, li, u);
    }
}

// q = D_{Omega'} rho on all extended sites; partials per workgroup of
// <q, rho> and <q, q>, or of <dhat, q> and <q, q> when dhat is set
template <int GP>
__global__ __launch_bounds__(256) void k_blk_dslash(BlockArgs a) {
    const int per_rhs = a.B.nblocks * a.wpb;
    const int rhs = blockIdx.x / per_rhs;
    const int blk = (blockIdx.x % per_rhs) / a.wpb;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    if (skip_colour(a, blk)) return;
    const int wl = blockIdx.x % a.wpb;
    const int l = wl * 256 + threadIdx.x;
    double d[3] = {0, 0, 0};
    if (l < a.B.ev) {
        int lc[4], x[4];
        block_site(a.g, a.B, blk, l, lc, x);
        const int gi = geom_index(a.g, x);
        const int base = blk * a.B.ev;
        const int e = base + l;
        const f4v* rho = (const f4v*)a.rho + rhs * a.ws_stride;
        float acc[24];
        const float mk = (float)(-a.kappa);
        // the eight hops (x+, x-, y+, y-, z+, z-, t+, t-), software-pipelined:
        // hop k+1's neighbour and link are requested before hop k is computed
        int ni[8], li[8];
        float ph[8];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            ni[2 * mu] = blk_neighbour(a.g, a.B, lc, mu, true);
            li[2 * mu] = gi;
            ph[2 * mu] = (x[mu] == a.g.L[mu] - 1) ? (float)a.g.bc[mu] : 1.f;
            ni[2 * mu + 1] = blk_neighbour(a.g, a.B, lc, mu, false);
            int y[4] = {x[0], x[1], x[2], x[3]};
            y[mu] = x[mu] == 0 ? a.g.L[mu] - 1 : x[mu] - 1;
            li[2 * mu + 1] = geom_index(a.g, y);
            ph[2 * mu + 1] = (x[mu] == 0) ? (float)a.g.bc[mu] : 1.f;
        }
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = 0.f;
        float s0[24], u0[18], s1[24], u1[18];
        blk_fetch<GP>(a, rho, base, ni[0], 0, li[0], s0, u0);
#define WCL_BHOP(K, SC, UC, SN, UN)                                                            \
    if ((K) < 7) blk_fetch<GP>(a, rho, base, ni[((K) + 1) & 7], ((K) + 1) / 2, li[((K) + 1) & 7], SN, UN); \
    if (ni[K] >= 0) hop_compute<(K) / 2, ((K) % 2) == 0>(SC, UC, mk * ph[K], acc);
        WCL_BHOP(0, s0, u0, s1, u1)
        WCL_BHOP(1, s1, u1, s0, u0)
        WCL_BHOP(2, s0, u0, s1, u1)
        WCL_BHOP(3, s1, u1, s0, u0)
        WCL_BHOP(4, s0, u0, s1, u1)
        WCL_BHOP(5, s1, u1, s0, u0)
        WCL_BHOP(6, s0, u0, s1, u1)
        WCL_BHOP(7, s1, u1, s0, u0)
#undef WCL_BHOP
        float r0[24];
        ws_load(rho, a.NE, e, r0);
        {
            const float ck = (float)(a.csw * a.kappa);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                float c[36], y[12];
                CloverBlk<GP>::template load<false>(a.clover, a.g.V, gi, b, c);
                herm6_apply(c, r0 + 12 * b, y);
#pragma unroll
                for (int j = 0; j < 12; ++j) acc[12 * b + j] += r0[12 * b + j] + ck * y[j];
            }
        }
        ws_store((f4v*)a.q + rhs * a.ws_stride, a.NE, e, acc);
        if (a.dhat) {
            float h[24];
            ws_load((const f4v*)a.dhat + rhs * a.ws_stride, a.NE, e, h);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                float hr = h[2 * k], hi = h[2 * k + 1], qr = acc[2 * k], qi = acc[2 * k + 1];
                d[0] += (double)(hr * qr + hi * qi);   // <dhat, q>
                d[1] += (double)(hr * qi - hi * qr);
                d[2] += (double)(qr * qr + qi * qi);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                float qr = acc[2 * k], qi = acc[2 * k + 1], rr = r0[2 * k], ri = r0[2 * k + 1];
                d[0] += (double)(qr * rr + qi * ri);   // <q, rho>
                d[1] += (double)(qr * ri - qi * rr);
                d[2] += (double)(qr * qr + qi * qi);   // <q, q>
            }
        }
    }
    block_reduce3(d, a.partial + 3 * (((size_t)rhs * a.B.nblocks + blk) * a.wpb + wl));
}

// Last-step write-out of a workgroup whose domain is not solved in this
// pass (other colour): zeros at its owned sites.
template <int VP>
WCL_DEV bool colour_skip_finish(const BlockArgs& a, int rhs, int blk, int l, int last) {
    if (!skip_colour(a, blk)) return false;
    if (last && l < a.B.ev) {
        float z[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) z[k] = 0.f;
        blk_finish<VP>(a, rhs, blk, l, z, true);
    }
    return true;
}

// alpha = <q,rho>/<q,q> for the domain; x += alpha rho; rho -= alpha q.
// On the last step the solution goes to blk_finish.
template <int VP>
__global__ __launch_bounds__(256) void k_blk_update(BlockArgs a, int last) {
    const int per_rhs = a.B.nblocks * a.wpb;
    const int rhs = blockIdx.x / per_rhs;
    const int blk = (blockIdx.x % per_rhs) / a.wpb;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int l = (blockIdx.x % a.wpb) * 256 + threadIdx.x;
    if (colour_skip_finish<VP>(a, rhs, blk, l, last)) return;
    __shared__ float al[2];
    if (threadIdx.x == 0) {
        double s[3];
        domain_sum3(a.partial, a, rhs, blk, s);
        al[0] = s[2] > 0 ? (float)(s[0] / s[2]) : 0.f;
        al[1] = s[2] > 0 ? (float)(s[1] / s[2]) : 0.f;
    }
    __syncthreads();
    if (l >= a.B.ev) return;
    const float ar = al[0], ai = al[1];
    const int e = blk * a.B.ev + l;
    f4v* rho = (f4v*)a.rho + rhs * a.ws_stride;
    f4v* q = (f4v*)a.q + rhs * a.ws_stride;
    f4v* xs = (f4v*)a.x + rhs * a.ws_stride;
    float xv[24];
#pragma unroll
    for (int g = 0; g < 6; ++g) {
        const size_t k = (size_t)g * a.NE + e;
        f4v r = rho[k], qq = q[k], xx = xs[k];
        xx = xx + f4v{ar * r.x - ai * r.y, ar * r.y + ai * r.x, ar * r.z - ai * r.w, ar * r.w + ai * r.z};
        if (!last) {
            r = r - f4v{ar * qq.x - ai * qq.y, ar * qq.y + ai * qq.x, ar * qq.z - ai * qq.w, ar * qq.w + ai * qq.z};
            rho[k] = r;
            xs[k] = xx;
        }
        xv[4 * g] = xx.x;
        xv[4 * g + 1] = xx.y;
        xv[4 * g + 2] = xx.z;
        xv[4 * g + 3] = xx.w;
    }
    if (last) blk_finish<VP>(a, rhs, blk, l, xv, false);
}

// y = A^{-1} z at global site gi: the two packed Hermitian blocks of the
// site-term inverse applied to the two chiral halves
template <int GP>
WCL_DEV void site_inverse_apply(const BlockArgs& a, int gi, const float z[24], float y[24]) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        float c[36];
        CloverBlk<GP>::template load<false>(a.ainv, a.g.V, gi, b, c);
        herm6_apply(c, z + 12 * b, y + 12 * b);
    }
}

// Block Jacobi step (the diagonal blocks of D_{Omega'} are the site terms):
// x = x + A^{-1} (b - q) with b = rho (the projected residual, unchanged)
// and q = D_{Omega'} x; the first step (x = 0) is x = A^{-1} b.
template <int GP, int VP>
__global__ __launch_bounds__(256) void k_blk_jacobi(BlockArgs a, int first, int last) {
    const int per_rhs = a.B.nblocks * a.wpb;
    const int rhs = blockIdx.x / per_rhs;
    const int blk = (blockIdx.x % per_rhs) / a.wpb;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int l = (blockIdx.x % a.wpb) * 256 + threadIdx.x;
    if (colour_skip_finish<VP>(a, rhs, blk, l, last)) return;
    if (l >= a.B.ev) return;
    const int e = blk * a.B.ev + l;
    int lc[4], x[4];
    block_site(a.g, a.B, blk, l, lc, x);
    const int gi = geom_index(a.g, x);
    float b[24], z[24], y[24], xv[24];
    ws_load((const f4v*)a.rho + rhs * a.ws_stride, a.NE, e, b);
    if (first) {
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            z[k] = b[k];
            xv[k] = 0.f;
        }
    } else {
        float q[24];
        ws_load((const f4v*)a.q + rhs * a.ws_stride, a.NE, e, q);
        ws_load((const f4v*)a.x + rhs * a.ws_stride, a.NE, e, xv);
#pragma unroll
        for (int k = 0; k < 24; ++k) z[k] = b[k] - q[k];
    }
    site_inverse_apply<GP>(a, gi, z, y);
#pragma unroll
    for (int k = 0; k < 24; ++k) xv[k] += y[k];
    if (last) blk_finish<VP>(a, rhs, blk, l, xv, false);
    else ws_store((f4v*)a.x + rhs * a.ws_stride, a.NE, e, xv);
}

// ---- truncated BiCGStab on every domain (exactly N_dominv iterations from
// zero, no restart, no early exit; a vanishing denominator makes its
// coefficient zero).  Workspaces: r = rho, v = q, p = bp, s = bs, t = bt,
// rhat = brh, x.  Per iteration five launches:
//   p:  rho = <rhat, r>, beta = (rho/rho_old)(alpha/omega), p = r + beta (p - omega v)
//   v = D p, partials <rhat, v>           (k_blk_dslash with dhat = rhat)
//   s:  alpha = rho / <rhat, v>, s = r - alpha v
//   t = D s, partials <t, s>, |t|^2        (k_blk_dslash)
//   xr: omega = <t, s> / |t|^2, x += alpha p + omega s, r = s - omega t,
//       partials <rhat, r>
// Every workgroup of a domain forms the domain's scalars from the partials
// itself (fixed order); workgroup 0 of the domain records them in dsc for
// the later launches.
WCL_DEV double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return double2{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
WCL_DEV double2 cmul(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
WCL_DEV bool cnz(double2 a) { return a.x != 0.0 || a.y != 0.0; }

__global__ __launch_bounds__(256) void k_bcg_p(BlockArgs a, int it) {
    const int per_rhs = a.B.nblocks * a.wpb;
    const int rhs = blockIdx.x / per_rhs;
    const int blk = (blockIdx.x % per_rhs) / a.wpb;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    if (skip_colour(a, blk)) return;
    const int wl = blockIdx.x % a.wpb;
    const int l = wl * 256 + threadIdx.x;
    double* ds = a.dsc + 8 * ((size_t)rhs * a.B.nblocks + blk);
    __shared__ float bt[4];   // beta, omega
    if (threadIdx.x == 0) {
        double s[3];
        domain_sum3(a.bpart[0], a, rhs, blk, s);
        const double2 rho{s[0], s[1]};
        double2 beta{0.0, 0.0}, omega{0.0, 0.0};
        if (it > 0) {
            const double2 rho_old{ds[6], ds[7]}, alpha{ds[2], ds[3]};
            omega = double2{ds[4], ds[5]};
            if (cnz(rho_old) && cnz(omega)) beta = cmul(cdiv(rho, rho_old), cdiv(alpha, omega));
        }
        if (wl == 0) {
            ds[0] = rho.x;
            ds[1] = rho.y;
        }
        bt[0] = (float)beta.x;
        bt[1] = (float)beta.y;
        bt[2] = (float)omega.x;
        bt[3] = (float)omega.y;
    }
    __syncthreads();
    if (l >= a.B.ev) return;
    const int e = blk * a.B.ev + l;
    float r[24], p[24];
    ws_load((const f4v*)a.rho + rhs * a.ws_stride, a.NE, e, r);
    if (it == 0) {
        ws_store((f4v*)a.bp + rhs * a.ws_stride, a.NE, e, r);   // p = r (p = v = 0 before)
        return;
    }
    float v[24];
    ws_load((const f4v*)a.bp + rhs * a.ws_stride, a.NE, e, p);
    ws_load((const f4v*)a.q + rhs * a.ws_stride, a.NE, e, v);
    const float br = bt[0], bi = bt[1], wr = bt[2], wi = bt[3];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        // u = p - omega v;  p = r + beta u
        const float ur = p[2 * k] - (wr * v[2 * k] - wi * v[2 * k + 1]);
        const float ui = p[2 * k + 1] - (wr * v[2 * k + 1] + wi * v[2 * k]);
        p[2 * k] = r[2 * k] + (br * ur - bi * ui);
        p[2 * k + 1] = r[2 * k + 1] + (br * ui + bi * ur);
    }
    ws_store((f4v*)a.bp + rhs * a.ws_stride, a.NE, e, p);
}

__global__ __launch_bounds__(256) void k_bcg_s(BlockArgs a) {
    const int per_rhs = a.B.nblocks * a.wpb;
    const int rhs = blockIdx.x / per_rhs;
    const int blk = (blockIdx.x % per_rhs) / a.wpb;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    if (skip_colour(a, blk)) return;
    const int wl = blockIdx.x % a.wpb;
    const int l = wl * 256 + threadIdx.x;
    double* ds = a.dsc + 8 * ((size_t)rhs * a.B.nblocks + blk);
    __shared__ float al[2];
    if (threadIdx.x == 0) {
        double s[3];
        domain_sum3(a.bpart[1], a, rhs, blk, s);
        const double2 rv{s[0], s[1]}, rho{ds[0], ds[1]};
        const double2 alpha = cnz(rv) ? cdiv(rho, rv) : double2{0.0, 0.0};
        if (wl == 0) {
            ds[2] = alpha.x;
            ds[3] = alpha.y;
        }
        al[0] = (float)alpha.x;
        al[1] = (float)alpha.y;
    }
    __syncthreads();
    if (l >= a.B.ev) return;
    const int e = blk * a.B.ev + l;
    float r[24], v[24];
    ws_load((const f4v*)a.rho + rhs * a.ws_stride, a.NE, e, r);
    ws_load((const f4v*)a.q + rhs * a.ws_stride, a.NE, e, v);
    const float ar = al[0], ai = al[1];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const float vr = v[2 * k], vi = v[2 * k + 1];
        r[2 * k] -= ar * vr - ai * vi;
        r[2 * k + 1] -= ar * vi + ai * vr;
    }
    ws_store((f4v*)a.bs + rhs * a.ws_stride, a.NE, e, r);
}

template <int VP>
__global__ __launch_bounds__(256) void k_bcg_xr(BlockArgs a, int last) {
    const int per_rhs = a.B.nblocks * a.wpb;
    const int rhs = blockIdx.x / per_rhs;
    const int blk = (blockIdx.x % per_rhs) / a.wpb;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int wl = blockIdx.x % a.wpb;
    const int l = wl * 256 + threadIdx.x;
    if (colour_skip_finish<VP>(a, rhs, blk, l, last)) return;
    double* ds = a.dsc + 8 * ((size_t)rhs * a.B.nblocks + blk);
    __shared__ float co[4];   // alpha, omega
    if (threadIdx.x == 0) {
        double s[3];
        domain_sum3(a.bpart[2], a, rhs, blk, s);
        const double2 omega = s[2] > 0.0 ? double2{s[0] / s[2], s[1] / s[2]} : double2{0.0, 0.0};
        co[0] = (float)ds[2];
        co[1] = (float)ds[3];
        co[2] = (float)omega.x;
        co[3] = (float)omega.y;
        if (wl == 0) {
            ds[4] = omega.x;
            ds[5] = omega.y;
            ds[6] = ds[0];   // rho_old = rho
            ds[7] = ds[1];
        }
    }
    __syncthreads();
    double d[3] = {0.0, 0.0, 0.0};
    if (l < a.B.ev) {
        const int e = blk * a.B.ev + l;
        const float ar = co[0], ai = co[1], wr = co[2], wi = co[3];
        float xv[24], p[24], s[24];
        ws_load((const f4v*)a.x + rhs * a.ws_stride, a.NE, e, xv);
        ws_load((const f4v*)a.bp + rhs * a.ws_stride, a.NE, e, p);
        ws_load((const f4v*)a.bs + rhs * a.ws_stride, a.NE, e, s);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            xv[2 * k] += (ar * p[2 * k] - ai * p[2 * k + 1]) + (wr * s[2 * k] - wi * s[2 * k + 1]);
            xv[2 * k + 1] += (ar * p[2 * k + 1] + ai * p[2 * k]) + (wr * s[2 * k + 1] + wi * s[2 * k]);
        }
        if (last) {
            blk_finish<VP>(a, rhs, blk, l, xv, false);
        } else {
            ws_store((f4v*)a.x + rhs * a.ws_stride, a.NE, e, xv);
            float t[24], h[24];
            ws_load((const f4v*)a.bt + rhs * a.ws_stride, a.NE, e, t);
            ws_load((const f4v*)a.brh + rhs * a.ws_stride, a.NE, e, h);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const float tr = t[2 * k], ti = t[2 * k + 1];
                s[2 * k] -= wr * tr - wi * ti;
                s[2 * k + 1] -= wr * ti + wi * tr;
            }
            ws_store((f4v*)a.rho + rhs * a.ws_stride, a.NE, e, s);   // r = s - omega t
            site_dot3(h, s, d);                                       // <rhat, r>
        }
    }
    if (!last) block_reduce3(d, a.bpart[0] + 3 * (((size_t)rhs * a.B.nblocks + blk) * a.wpb + wl));
}

// Additive Schwarz sum: one thread per lattice site; v(x) = the sum, over
// every domain whose extended set Omega' holds x (in each split direction
// the own domain and, within s sites of its faces, the neighbour), of that
// domain's extended solution at x.  Fixed order, no atomics.
template <int VP>
__global__ __launch_bounds__(256) void k_blk_gather(BlockArgs a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int rhs = blockIdx.y;
    if (i >= a.g.V) return;
    if (a.sc && !a.sc[rhs].active) return;
    int x[4];
    geom_coords(a.g, i, x);
    // per direction: the candidate domains (block coordinate, local coordinate)
    int cb[4][3], cl[4][3], nc[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int b = a.B.b[mu], sm = a.B.s[mu];
        const int own = x[mu] / b, p = x[mu] - own * b;
        int n = 0;
        cb[mu][n] = own;
        cl[mu][n++] = p + sm;
        if (sm > 0 && p < sm) {   // in the upper extension of the previous domain
            cb[mu][n] = own == 0 ? a.B.nb[mu] - 1 : own - 1;
            cl[mu][n++] = p + sm + b;
        }
        if (sm > 0 && p >= b - sm) {   // in the lower extension of the next domain
            cb[mu][n] = own == a.B.nb[mu] - 1 ? 0 : own + 1;
            cl[mu][n++] = p + sm - b;
        }
        nc[mu] = n;
    }
    const f4v* xs = (const f4v*)a.x + rhs * a.ws_stride;
    float v[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = 0.f;
    for (int i3 = 0; i3 < nc[3]; ++i3)
        for (int i2 = 0; i2 < nc[2]; ++i2)
            for (int i1 = 0; i1 < nc[1]; ++i1)
                for (int i0 = 0; i0 < nc[0]; ++i0) {
                    const int bi[4] = {i0, i1, i2, i3};
                    int blk = 0, loc = 0;
                    for (int mu = 3; mu >= 0; --mu) {
                        blk = blk * a.B.nb[mu] + cb[mu][bi[mu]];
                        loc = loc * a.B.e[mu] + cl[mu][bi[mu]];
                    }
                    float s[24];
                    ws_load(xs, a.NE, blk * a.B.ev + loc, s);
#pragma unroll
                    for (int k = 0; k < 24; ++k) v[k] += s[k];
                }
    char* out = (char*)a.out + rhs * a.out_stride;
    if (a.accumulate) {
        float o[24];
        SpinorIO<WCL_F32>::load(out, a.g.V, i, o);
#pragma unroll
        for (int k = 0; k < 24; ++k) o[k] += v[k];
        SpinorIO<WCL_F32>::store(out, a.g.V, i, o);
    } else {
        SpinorIO<WCL_F32>::store(out, a.g.V, i, v);
    }
    if (a.vj) SpinorIO<VP>::store((char*)a.vj + rhs * a.vj_stride, a.g.V, i, v);
}

// Unpacks the extended-domain workspace q to FP64 AoS (test surface).
__global__ __launch_bounds__(256) void k_blk_unpack(BlockArgs a, const float* ws, double* out) {
    int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= a.NE) return;
    float s[24];
    ws_load((const f4v*)ws, a.NE, e, s);
    for (int k = 0; k < 24; ++k) out[(size_t)e * 24 + k] = s[k];
}

static dim3 blk_grid(const BlockArgs& a) { return dim3((unsigned)(a.B.nblocks * a.wpb * a.nrhs)); }

int launch_blk_project(const BlockArgs& a, int src_prec, int bicgstab, hipStream_t st) {
#define WCL_P(S)                                                                            \
    if (src_prec == S) {                                                                    \
        if (bicgstab) k_blk_project<S, true><<<blk_grid(a), 256, 0, st>>>(a);               \
        else k_blk_project<S, false><<<blk_grid(a), 256, 0, st>>>(a);                      \
        WCL_HIP(hipGetLastError());                                                         \
        return WCL_OK;                                                                      \
    }
    WCL_P(WCL_F32)
    WCL_P(WCL_F16)
#undef WCL_P
    wcl_set_error("domain projection: unsupported source precision");
    return WCL_EINVAL;
}

int launch_blk_dslash(const BlockArgs& a, int gp, hipStream_t st) {
    if (gp == WCL_F32) k_blk_dslash<WCL_F32><<<blk_grid(a), 256, 0, st>>>(a);
    else if (gp == WCL_F16) k_blk_dslash<WCL_F16><<<blk_grid(a), 256, 0, st>>>(a);
    else {
        wcl_set_error("domain operator: unsupported storage precision");
        return WCL_EINVAL;
    }
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_blk_update(const BlockArgs& a, int vj_prec, int last, hipStream_t st) {
    if (vj_prec == WCL_F16) k_blk_update<WCL_F16><<<blk_grid(a), 256, 0, st>>>(a, last);
    else k_blk_update<WCL_F32><<<blk_grid(a), 256, 0, st>>>(a, last);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_blk_jacobi(const BlockArgs& a, int gp, int vj_prec, int first, int last, hipStream_t st) {
    if (!a.ainv) {
        wcl_set_error("block Jacobi: site-term inverse missing");
        return WCL_EINVAL;
    }
    if (gp == WCL_F32 && vj_prec == WCL_F32) k_blk_jacobi<WCL_F32, WCL_F32><<<blk_grid(a), 256, 0, st>>>(a, first, last);
    else if (gp == WCL_F16 && vj_prec == WCL_F16)
        k_blk_jacobi<WCL_F16, WCL_F16><<<blk_grid(a), 256, 0, st>>>(a, first, last);
    else {
        wcl_set_error("block Jacobi: unsupported storage precision");
        return WCL_EINVAL;
    }
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_bcg_p(const BlockArgs& a, int it, hipStream_t st) {
    k_bcg_p<<<blk_grid(a), 256, 0, st>>>(a, it);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_bcg_s(const BlockArgs& a, hipStream_t st) {
    k_bcg_s<<<blk_grid(a), 256, 0, st>>>(a);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_bcg_xr(const BlockArgs& a, int vj_prec, int last, hipStream_t st) {
    if (vj_prec == WCL_F16) k_bcg_xr<WCL_F16><<<blk_grid(a), 256, 0, st>>>(a, last);
    else k_bcg_xr<WCL_F32><<<blk_grid(a), 256, 0, st>>>(a, last);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_blk_gather(const BlockArgs& a, int vj_prec, hipStream_t st) {
    const dim3 grid((unsigned)((a.g.V + 255) / 256), (unsigned)a.nrhs);
    if (vj_prec == WCL_F16) k_blk_gather<WCL_F16><<<grid, 256, 0, st>>>(a);
    else k_blk_gather<WCL_F32><<<grid, 256, 0, st>>>(a);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_blk_unpack(const BlockArgs& a, const float* ws, double* out, hipStream_t st) {
    k_blk_unpack<<<(a.NE + 255) / 256, 256, 0, st>>>(a, ws, out);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

// ----------------------------------------------------------- fused path --
// One workgroup per (domain, rhs) holds the whole extended domain on chip:
// extended site l is thread l; its two-row links U_mu(x) and its clover
// block pair stay in registers for all N_dominv MR steps, and each step
// publishes rho(x) and the backward-hop half-spinors U_mu(x)^dag P+ rho(x)
// in LDS for the neighbours.  Two barriers per step; alpha comes from a
// fixed-order workgroup all-reduce, so every thread holds the same value.
template <int NW>
WCL_DEV void wg_allreduce3(double d[3], double* sh) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = wave_sum(d[k]);
    if (l == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) sh[3 * w + k] = d[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) s += sh[3 * q + k];
        d[k] = s;
    }
}

// The same for FP32 per-thread values: FP32 over each wavefront, FP64
// across the wavefronts, in a fixed order.
template <int NW>
WCL_DEV void wg_allreduce3f(const float f[3], double d[3], double* sh) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    float s[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = wave_sumf(f[k]);
    if (l == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) sh[3 * w + k] = (double)s[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double r = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) r += sh[3 * q + k];
        d[k] = r;
    }
}

// Links U_mu(x) (rows 0, 1) and the clover block pair of one site, held in
// registers (as FP32) for all MR steps.  Cached loads: every sweep of every
// inner iteration reads them again, and at moderate volumes they stay in the
// Infinity Cache.
template <int GP>
struct SiteFields {
    float u[4][12];
    float c[72];
    WCL_DEV void zero() {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int k = 0; k < 12; ++k) u[mu][k] = 0.f;
#pragma unroll
        for (int k = 0; k < 72; ++k) c[k] = 0.f;
    }
    WCL_DEV void load(const BlockArgs& a, int gi) {
        float t[18];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            GaugeIO<GP>::template load_raw<false>(a.gauge, a.g.V, mu, gi, t);
#pragma unroll
            for (int k = 0; k < 12; ++k) u[mu][k] = t[k];
        }
        CloverIO<GP>::template load<false>(a.clover, a.g.V, gi, c);
    }
    template <int MU>
    WCL_DEV void link(float w[18]) const {
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = u[MU][k];
        reconstruct_row2(w);
    }
    WCL_DEV void refresh() {}
    // w = U_mu(x) h (DAG = false) or U_mu(x)^dag h
    template <int MU, bool DAG>
    WCL_DEV void apply(const float h[12], float w[12]) const {
        float t[18];
        link<MU>(t);
        su3_apply2<DAG>(t, h, w);
    }
    // q = A r = r + ck C r
    WCL_DEV void site_term(const float r[24], float ck, float q[24]) const { clover_term(c, r, ck, q); }
    // the forms used inside the MR steps (the same arithmetic here)
    template <int MU, bool DAG>
    WCL_DEV void step_apply(const float h[12], float w[12]) const { apply<MU, DAG>(h, w); }
    WCL_DEV void step_site_term(const float r[24], float ck, float q[24]) const { site_term(r, ck, q); }
};

// FP16 storage: rows 0,1 of the links and the clover stay in registers as the
// stored binary16 values, two per register, and enter the arithmetic through
// mixed-precision FMAs (binary16 operand, FP32 product and sum: the same
// values as widening them first).  Row 2 of each link is rebuilt once per
// launch in FP32 and kept, instead of once per use.  This takes 85 registers
// where FP32 copies of the fields take 120.
template <>
struct SiteFields<WCL_F16> {
    h2v u[4][6];      // rows 0,1 of U_mu(x), binary16
    float r2[4][6];   // row 2 of U_mu(x), FP32
    h2v c[36];        // clover blocks, binary16 of value / scale
    float cs;         // the clover's per-site scale
    // The first product of an FMA chain is an FMA onto this zero, which the
    // compiler cannot see through: a plain multiply has no mixed-precision
    // form and would widen the binary16 operand in a separate instruction.
    float zr;
    WCL_DEV void zero() {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                u[mu][k] = h2v{(_Float16)0.f, (_Float16)0.f};
                r2[mu][k] = 0.f;
            }
#pragma unroll
        for (int k = 0; k < 36; ++k) c[k] = h2v{(_Float16)0.f, (_Float16)0.f};
        cs = 0.f;
        zr = 0.f;
        asm volatile("" : "+v"(zr));
    }
    // Called at the top of every MR step: the packed fields become opaque
    // there, so the compiler cannot hoist their widening out of the step loop
    // (which would hold all of them in FP32 registers) and feeds the binary16
    // halves to the mixed-precision FMAs instead.
    WCL_DEV void refresh() {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int k = 0; k < 6; ++k) asm volatile("" : "+v"(u[mu][k]));
#pragma unroll
        for (int k = 0; k < 36; ++k) asm volatile("" : "+v"(c[k]));
    }
    template <int MU>
    WCL_DEV float uk(int k) const { return (float)((k & 1) ? u[MU][k >> 1].y : u[MU][k >> 1].x); }
    WCL_DEV float ck_(int k) const { return (float)((k & 1) ? c[k >> 1].y : c[k >> 1].x); }
    WCL_DEV void load(const BlockArgs& a, int gi) {
        const h4v* gp = (const h4v*)a.gauge;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            float t[18];
#pragma unroll
            for (int g = 0; g < 3; ++g) {
                const h4v v = gp[tix(3 * mu + g, gi, 12)];
                u[mu][2 * g] = h2v{v.x, v.y};
                u[mu][2 * g + 1] = h2v{v.z, v.w};
                t[4 * g] = (float)v.x;
                t[4 * g + 1] = (float)v.y;
                t[4 * g + 2] = (float)v.z;
                t[4 * g + 3] = (float)v.w;
            }
            reconstruct_row2(t);
#pragma unroll
            for (int k = 0; k < 6; ++k) r2[mu][k] = t[12 + k];
        }
        const h8v* cp = (const h8v*)a.clover;
#pragma unroll
        for (int g = 0; g < 9; ++g) {
            const h8v v = cp[tix(g, gi, 9)];
#pragma unroll
            for (int j = 0; j < 4; ++j) c[4 * g + j] = h2v{v[2 * j], v[2 * j + 1]};
        }
        cs = ((const float*)((const char*)a.clover + half_clover_scale_offset(a.g.V)))[gi];
    }
    // w = U_mu(x) h (DAG = false) or U_mu(x)^dag h
    template <int MU, bool DAG>
    WCL_DEV void apply(const float h[12], float w[12]) const {
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float re = zr, im = zr;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const int row = DAG ? b : a, col = DAG ? a : b;
                    const float ur = row < 2 ? uk<MU>(2 * (3 * row + col)) : r2[MU][2 * col];
                    const float uv = row < 2 ? uk<MU>(2 * (3 * row + col) + 1) : r2[MU][2 * col + 1];
                    const float ui = DAG ? -uv : uv;
                    const float hr = h[6 * sp + 2 * b], hi = h[6 * sp + 2 * b + 1];
                    re = fmad(ur, hr, re);
                    re = fmad(-ui, hi, re);
                    im = fmad(ur, hi, im);
                    im = fmad(ui, hr, im);
                }
                w[6 * sp + 2 * a] = re;
                w[6 * sp + 2 * a + 1] = im;
            }
    }
    // q = A r = r + ck C r, C = cs x (the stored binary16 blocks)
    WCL_DEV void site_term(const float r[24], float ck, float q[24]) const {
        const float f = ck * cs;
#pragma unroll
        for (int bk = 0; bk < 2; ++bk) {
            const int o = 36 * bk;
            const float* x = r + 12 * bk;
            float y[12];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                y[2 * a] = fmad(ck_(o + a), x[2 * a], zr);
                y[2 * a + 1] = fmad(ck_(o + a), x[2 * a + 1], zr);
            }
            int k = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int b = a + 1; b < 6; ++b, ++k) {
                    const float re = ck_(o + 6 + 2 * k), im = ck_(o + 6 + 2 * k + 1);
                    y[2 * a] = fmad(re, x[2 * b], y[2 * a]);
                    y[2 * a] = fmad(-im, x[2 * b + 1], y[2 * a]);
                    y[2 * a + 1] = fmad(re, x[2 * b + 1], y[2 * a + 1]);
                    y[2 * a + 1] = fmad(im, x[2 * b], y[2 * a + 1]);
                    y[2 * b] = fmad(re, x[2 * a], y[2 * b]);
                    y[2 * b] = fmad(im, x[2 * a + 1], y[2 * b]);
                    y[2 * b + 1] = fmad(re, x[2 * a + 1], y[2 * b + 1]);
                    y[2 * b + 1] = fmad(-im, x[2 * a], y[2 * b + 1]);
                }
#pragma unroll
            for (int j = 0; j < 12; ++j) q[12 * bk + j] = fmad(f, y[j], x[j]);
        }
    }
    template <int MU, bool DAG>
    WCL_DEV void step_apply(const float h[12], float w[12]) const { apply<MU, DAG>(h, w); }
    WCL_DEV void step_site_term(const float r[24], float ck, float q[24]) const { site_term(r, ck, q); }
};

// FP16 storage with binary16 operands inside the MR steps: the fields as in
// SiteFields<WCL_F16> (row 2 of each link rebuilt in FP32 at load and
// rounded to binary16 as well); each step's products of the links and the
// clover take rho rounded to binary16 as v_dot2 operands (each pair as its
// conjugate, swap or -i multiple, which carry the signs of the complex
// product), summed in FP32, with the spin projections in packed binary16
// additions, and the backward-hop terms U^dag P+ rho pass between sites as
// binary16 pairs.  Accumulation and the MR vector work stay FP32.  The kernel
// scales each domain's rho by a power of two to an RMS component near 1
// before the steps (MR commutes with
// the scaling), so the binary16 operands neither overflow nor lose precision
// to small magnitudes.  The residual updates between sweeps use the
// mixed-precision FMA forms (FP32 operands, unscaled).
struct SiteFieldsDot {
    h2v u[4][9];   // U_mu(x), element (row, col) at 3 row + col, binary16
    h2v c[36];     // clover blocks, binary16 of value / scale
    float cs;
    float zr;      // an opaque zero: see SiteFields<WCL_F16>
    WCL_DEV void zero() {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int k = 0; k < 9; ++k) u[mu][k] = h2v{(_Float16)0.f, (_Float16)0.f};
#pragma unroll
        for (int k = 0; k < 36; ++k) c[k] = h2v{(_Float16)0.f, (_Float16)0.f};
        cs = 0.f;
        zr = 0.f;
        asm volatile("" : "+v"(zr));
    }
    WCL_DEV void refresh() {
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int k = 0; k < 9; ++k) asm volatile("" : "+v"(u[mu][k]));
#pragma unroll
        for (int k = 0; k < 36; ++k) asm volatile("" : "+v"(c[k]));
    }
    template <int MU>
    WCL_DEV float uk(int k) const { return (float)((k & 1) ? u[MU][k >> 1].y : u[MU][k >> 1].x); }
    WCL_DEV float ck_(int k) const { return (float)((k & 1) ? c[k >> 1].y : c[k >> 1].x); }
    WCL_DEV void load(const BlockArgs& a, int gi) {
        const h4v* gp = (const h4v*)a.gauge;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            float t[18];
#pragma unroll
            for (int g = 0; g < 3; ++g) {
                const h4v v = gp[tix(3 * mu + g, gi, 12)];
                u[mu][2 * g] = h2v{v.x, v.y};
                u[mu][2 * g + 1] = h2v{v.z, v.w};
                t[4 * g] = (float)v.x;
                t[4 * g + 1] = (float)v.y;
                t[4 * g + 2] = (float)v.z;
                t[4 * g + 3] = (float)v.w;
            }
            reconstruct_row2(t);
#pragma unroll
            for (int k = 0; k < 3; ++k) u[mu][6 + k] = pack2(t[12 + 2 * k], t[12 + 2 * k + 1]);
        }
        const h8v* cp = (const h8v*)a.clover;
#pragma unroll
        for (int g = 0; g < 9; ++g) {
            const h8v v = cp[tix(g, gi, 9)];
#pragma unroll
            for (int j = 0; j < 4; ++j) c[4 * g + j] = h2v{v[2 * j], v[2 * j + 1]};
        }
        cs = ((const float*)((const char*)a.clover + half_clover_scale_offset(a.g.V)))[gi];
    }
    // w = U_mu(x) h or U_mu(x)^dag h, FP32 operands (mixed-precision FMAs)
    template <int MU, bool DAG>
    WCL_DEV void apply(const float h[12], float w[12]) const {
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float re = zr, im = zr;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const int e = DAG ? 3 * b + a : 3 * a + b;
                    const float ur = uk<MU>(2 * e), uv = uk<MU>(2 * e + 1);
                    const float ui = DAG ? -uv : uv;
                    const float hr = h[6 * sp + 2 * b], hi = h[6 * sp + 2 * b + 1];
                    re = fmad(ur, hr, re);
                    re = fmad(-ui, hi, re);
                    im = fmad(ur, hi, im);
                    im = fmad(ui, hr, im);
                }
                w[6 * sp + 2 * a] = re;
                w[6 * sp + 2 * a + 1] = im;
            }
    }
    // q = r + ck C r, FP32 operands
    WCL_DEV void site_term(const float r[24], float ck, float q[24]) const {
        const float f = ck * cs;
#pragma unroll
        for (int bk = 0; bk < 2; ++bk) {
            const int o = 36 * bk;
            const float* x = r + 12 * bk;
            float y[12];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                y[2 * a] = fmad(ck_(o + a), x[2 * a], zr);
                y[2 * a + 1] = fmad(ck_(o + a), x[2 * a + 1], zr);
            }
            int k = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int b = a + 1; b < 6; ++b, ++k) {
                    const float re = ck_(o + 6 + 2 * k), im = ck_(o + 6 + 2 * k + 1);
                    y[2 * a] = fmad(re, x[2 * b], y[2 * a]);
                    y[2 * a] = fmad(-im, x[2 * b + 1], y[2 * a]);
                    y[2 * a + 1] = fmad(re, x[2 * b + 1], y[2 * a + 1]);
                    y[2 * a + 1] = fmad(im, x[2 * b], y[2 * a + 1]);
                    y[2 * b] = fmad(re, x[2 * a], y[2 * b]);
                    y[2 * b] = fmad(im, x[2 * a + 1], y[2 * b]);
                    y[2 * b + 1] = fmad(re, x[2 * a + 1], y[2 * b + 1]);
                    y[2 * b + 1] = fmad(-im, x[2 * a], y[2 * b + 1]);
                }
#pragma unroll
            for (int j = 0; j < 12; ++j) q[12 * bk + j] = fmad(f, y[j], x[j]);
        }
    }
    // the same products with h rounded to binary16 (v_dot2): the operand
    // pairs (conj h, swp h) of U h or (h, -i h) of U^dag h
    template <int MU, bool DAG>
    WCL_DEV void step_apply(const float h[12], float w[12]) const {
        h2v ha[6], hb[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float re = h[2 * k], im = h[2 * k + 1];
            ha[k] = DAG ? pack2(re, im) : pack2(re, -im);
            hb[k] = DAG ? pack2(im, -re) : pack2(im, re);
        }
        apply16<MU, DAG>(ha, hb, w);
    }
    // w = U h or U^dag h for h given as the operand pairs of spin_project16
    template <int MU, bool DAG>
    WCL_DEV void apply16(const h2v ha[6], const h2v hb[6], float w[12]) const {
        su3_apply16<DAG>(u[MU], ha, hb, zr, w);
    }
    WCL_DEV void step_site_term(const float r[24], float ck, float q[24]) const {
        h2v rp[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) rp[k] = pack2(r[2 * k], r[2 * k + 1]);
        site_term16(rp, r, ck, q);
    }
    // q = r + ck C r with the products on rp (r as binary16 pairs)
    WCL_DEV void site_term16(const h2v rp[12], const float r[24], float ck, float q[24]) const {
        const float f = ck * cs;
#pragma unroll
        for (int bk = 0; bk < 2; ++bk) {
            const int o = 36 * bk;
            const float* x = r + 12 * bk;
            const h2v* xp = rp + 6 * bk;
            float y[12];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                y[2 * a] = fmad(ck_(o + a), x[2 * a], zr);
                y[2 * a + 1] = fmad(ck_(o + a), x[2 * a + 1], zr);
            }
            int k = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int b = a + 1; b < 6; ++b, ++k) {
                    const h2v C = c[o / 2 + 3 + k];   // C_ab; C_ba = conj(C_ab)
                    y[2 * a] = dot2(C, cj(xp[b]), y[2 * a]);
                    y[2 * a + 1] = dot2(C, swp(xp[b]), y[2 * a + 1]);
                    y[2 * b] = dot2(C, xp[a], y[2 * b]);
                    y[2 * b + 1] = dot2(C, mul_mi(xp[a]), y[2 * b + 1]);
                }
#pragma unroll
            for (int j = 0; j < 12; ++j) q[12 * bk + j] = fmad(f, y[j], x[j]);
        }
    }
};

template <int GP, bool DOT>
struct FusedFields {
    using type = SiteFields<GP>;
};
template <>
struct FusedFields<WCL_F16, true> {
    using type = SiteFieldsDot;
};

#ifndef WCL_FUSED_MINWAVES
#define WCL_FUSED_MINWAVES 2
#endif
// RES: 0 = no residual update (first sweep); 1 = r_j = src - D vprev from
// all eight hops; 2 = r_j = src - (the hops of D vprev that leave the
// domain), src being the previous sweep's final MR residual (no overlap).
// DOT: each site keeps its own rho in registers and publishes it to the
// neighbours as binary16 pairs, with the backward terms as binary16 pairs
// (36 instead of 72 LDS words per site).  Three domains per CU would then
// fit the LDS but not the registers: forced to 168 VGPRs the kernel spills
// and ran slower, so it keeps two.
template <bool DOT>
struct FusedShape {
    static constexpr int lds_words = DOT ? 36 : 72;
    static constexpr int min_waves = WCL_FUSED_MINWAVES;
};

template <int GP, int SRC, int VP, int NT, int RES, bool DOT>
__global__ __launch_bounds__(NT, FusedShape<DOT>::min_waves) void k_blk_fused(BlockArgs a, int write_vj) {
    extern __shared__ float lds[];
    float* s_rho = lds;                 // [24][NT]
    float* s_bwd = lds + 24 * NT;       // [4][12][NT] FP32, or [4][6][NT] binary16 pairs (DOT)
    h2v* s_bwd16 = (h2v*)s_bwd;
    __shared__ double s_red[3 * (NT / 64)];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int rhs = lb % a.nrhs, blk = lb / a.nrhs;
    if (a.sc && !a.sc[rhs].active) return;   // uniform over the workgroup
    const int l = threadIdx.x;
    const bool active = l < a.B.ev;
    int lc[4] = {0, 0, 0, 0}, x[4] = {0, 0, 0, 0}, gi = 0;
    int nf[4], nb[4];
    float phf[4], phb[4];
    float rho[24], xs[24];
    typename FusedFields<GP, DOT>::type F;
    F.zero();
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        rho[k] = 0.f;
        xs[k] = 0.f;
    }
    if (active) {
        block_site(a.g, a.B, blk, l, lc, x);
        gi = geom_index(a.g, x);
        SpinorIO<SRC>::load((const char*)a.src + rhs * a.src_stride, a.g.V, gi, rho);   // projection P r
        F.load(a, gi);
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        int ln[4] = {lc[0], lc[1], lc[2], lc[3]};
        const int e = a.B.e[mu], L = a.g.L[mu];
        // forward neighbour inside Omega'?
        ln[mu] = lc[mu] + 1;
        bool in = true;
        if (ln[mu] == e) {
            if (e == L) ln[mu] = 0;
            else in = false;
        }
        nf[mu] = (active && in) ? local_index(a.B, ln) : -1;
        phf[mu] = (x[mu] == L - 1) ? (float)a.g.bc[mu] : 1.f;
        ln[mu] = lc[mu] - 1;
        in = true;
        if (ln[mu] < 0) {
            if (e == L) ln[mu] = e - 1;
            else in = false;
        }
        nb[mu] = (active && in) ? local_index(a.B, ln) : -1;
        phb[mu] = (x[mu] == 0) ? (float)a.g.bc[mu] : 1.f;
    }
    const float ck = (float)(a.csw * a.kappa), mk = (float)(-a.kappa);
    if constexpr (RES == 2) {
        // Without overlap the MR iteration keeps rho = r_{j-1} - D_Omega x on
        // the domain, and v_{j-1} = x there, so r_j = r_{j-1} - D v_{j-1} is
        // the previous sweep's final rho minus the hops of D v_{j-1} that
        // leave the domain (Dirichlet D_Omega drops exactly those).
        if (active) {
            const char* vp = (const char*)a.vprev + rhs * a.vprev_stride;
            int nbr[8], lnk[8];
            float ph[8];
            hop_sites(a.g, gi, x, nbr, lnk, ph);
            float acc[24];
#pragma unroll
            for (int k = 0; k < 24; ++k) acc[k] = 0.f;
#define WCL_XHOP(K)                                                                       \
    if (((K) % 2 == 0 ? nf[(K) / 2] : nb[(K) / 2]) < 0) {                                 \
        float s[24], h[12], w[12], u[18];                                                 \
        SpinorIO<VP>::load(vp, a.g.V, nbr[K], s);                                         \
        spin_project<(K) / 2, (K) % 2 == 0>(s, h);                                        \
        if ((K) % 2 == 0) {                                                               \
            F.template apply<(K) / 2, false>(h, w);                                       \
        } else {                                                                          \
            GaugeIO<GP>::template load<false>(a.gauge, a.g.V, (K) / 2, lnk[K], u);        \
            su3_apply2<true>(u, h, w);                                                    \
        }                                                                                 \
        spin_accumulate<(K) / 2, (K) % 2 == 0>(w, mk * ph[K], acc);                       \
    }
            WCL_XHOP(0) WCL_XHOP(1) WCL_XHOP(2) WCL_XHOP(3) WCL_XHOP(4) WCL_XHOP(5) WCL_XHOP(6) WCL_XHOP(7)
#undef WCL_XHOP
#pragma unroll
            for (int k = 0; k < 24; ++k) rho[k] -= acc[k];
        }
    }
    if constexpr (RES == 1) {
        // The residual update of the previous sweep (Algorithm 1), fused:
        // r_j = r_{j-1} - D v_{j-1} at this site, with the own links and
        // clover from the registers and the neighbours' v_{j-1} and backward
        // links from memory (every site of Omega' sees the whole lattice).
        if (active) {
            const char* vp = (const char*)a.vprev + rhs * a.vprev_stride;
            int nbr[8], lnk[8];
            float ph[8];
            hop_sites(a.g, gi, x, nbr, lnk, ph);
            float acc[24];
            {
                float vv[24];
                SpinorIO<VP>::load(vp, a.g.V, gi, vv);
                F.site_term(vv, ck, acc);
            }
#define WCL_RHOP(K)                                                                   \
    {                                                                                 \
        float s[24], h[12], w[12], u[18];                                             \
        SpinorIO<VP>::load(vp, a.g.V, nbr[K], s);                                     \
        spin_project<(K) / 2, (K) % 2 == 0>(s, h);                                    \
        if ((K) % 2 == 0) {                                                           \
            F.template apply<(K) / 2, false>(h, w);                                   \
        } else {                                                                      \
            GaugeIO<GP>::template load<false>(a.gauge, a.g.V, (K) / 2, lnk[K], u);    \
            su3_apply2<true>(u, h, w);                                                \
        }                                                                             \
        spin_accumulate<(K) / 2, (K) % 2 == 0>(w, mk * ph[K], acc);                   \
    }
            WCL_RHOP(0) WCL_RHOP(1) WCL_RHOP(2) WCL_RHOP(3) WCL_RHOP(4) WCL_RHOP(5) WCL_RHOP(6) WCL_RHOP(7)
#undef WCL_RHOP
#pragma unroll
            for (int k = 0; k < 24; ++k) rho[k] -= acc[k];
            if (a.rout && block_owned(a.B, lc))
                SpinorIO<VP>::store((char*)a.rout + rhs * a.rout_stride, a.g.V, gi, rho);
        }
    }
    // binary16 operands: scale the domain's rho by 2^-e, 2^e near its RMS
    // component (exact in FP32; the solution and the final residual are
    // scaled back at the end)
    float scale = 1.f;
    if constexpr (DOT) {
        double d[3] = {0.0, 0.0, 0.0};
        if (active) {
            float f = 0.f;
#pragma unroll
            for (int k = 0; k < 24; ++k) f = fmad(rho[k], rho[k], f);
            d[0] = f;
        }
        wg_allreduce3<NT / 64>(d, s_red);
        const double ms = d[0] / (24.0 * a.B.ev);
        if (ms > 0.0 && ms < 1e300) {
            int e = 0;
            frexp(sqrt(ms), &e);
            scale = ldexpf(1.f, e);
            const float inv = ldexpf(1.f, -e);
#pragma unroll
            for (int k = 0; k < 24; ++k) rho[k] *= inv;
        }
    }
    if constexpr (DOT) {
        // own rho in registers (FP32); the neighbours read its binary16 pairs
        h2v* s_rp = (h2v*)lds;               // [12][NT]
        h2v* s_bw = (h2v*)(lds + 12 * NT);   // [4][6][NT]
        for (int step = 0; step < a.B.n_dominv; ++step) {
            F.refresh();
            h2v rp[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                rp[k] = pack2(rho[2 * k], rho[2 * k + 1]);
                s_rp[k * NT + l] = rp[k];
            }
            // opaque: the operand variants below come from the packed pairs
            // (folded into packed-add modifiers), not from re-converting
            // rho's halves one by one
#pragma unroll
            for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(rp[k]));
            // publish the backward-hop contributions U_mu(x)^dag P+ rho(x)
#define WCL_BWD16(MU)                                                           \
    {                                                                           \
        h2v ha[6], hb[6];                                                       \
        float w[12];                                                            \
        spin_project16<MU, false, true>(rp, ha, hb);                            \
        F.template apply16<MU, true>(ha, hb, w);                                \
        _Pragma("unroll") for (int k = 0; k < 6; ++k)                           \
            s_bw[(MU * 6 + k) * NT + l] = pack2(w[2 * k], w[2 * k + 1]);        \
    }
            WCL_BWD16(0) WCL_BWD16(1) WCL_BWD16(2) WCL_BWD16(3)
#undef WCL_BWD16
            __syncthreads();
            // q = D_{Omega'} rho
            float q[24];
            F.site_term16(rp, rho, ck, q);
#define WCL_HOPS16(MU)                                                                           \
    if (nf[MU] >= 0) {                                                                           \
        h2v np[12], ha[6], hb[6];                                                                \
        float w[12];                                                                             \
        _Pragma("unroll") for (int k = 0; k < 12; ++k) np[k] = s_rp[k * NT + nf[MU]];           \
        spin_project16<MU, true, false>(np, ha, hb);                                             \
        F.template apply16<MU, false>(ha, hb, w);                                                \
        spin_accumulate<MU, true>(w, mk * phf[MU], q);                                           \
    }                                                                                            \
    if (nb[MU] >= 0) {                                                                           \
        float w[12];                                                                             \
        _Pragma("unroll") for (int k = 0; k < 6; ++k) {                                          \
            const h2v t = s_bw[(MU * 6 + k) * NT + nb[MU]];                                      \
            w[2 * k] = (float)t.x;                                                               \
            w[2 * k + 1] = (float)t.y;                                                           \
        }                                                                                        \
        spin_accumulate<MU, false>(w, mk * phb[MU], q);                                          \
    }
            WCL_HOPS16(0) WCL_HOPS16(1) WCL_HOPS16(2) WCL_HOPS16(3)
#undef WCL_HOPS16
            // <q, rho> and <q, q>: FP32 over the site's 12 components and
            // over each wavefront, FP64 across the wavefronts
            float f[3] = {0.f, 0.f, 0.f};
            if (active) {
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    const float qr = q[2 * k], qi = q[2 * k + 1];
                    const float rr = rho[2 * k], ri = rho[2 * k + 1];
                    f[0] = fmad(qr, rr, f[0]);
                    f[0] = fmad(qi, ri, f[0]);
                    f[1] = fmad(qr, ri, f[1]);
                    f[1] = fmad(-qi, rr, f[1]);
                    f[2] = fmad(qr, qr, f[2]);
                    f[2] = fmad(qi, qi, f[2]);
                }
            }
            double d[3];
            // every thread has finished reading its neighbours' pairs after
            // this barrier; the next writes of them come after it
            wg_allreduce3f<NT / 64>(f, d, s_red);
            // alpha = <q, rho> / <q, q>: one FP64 reciprocal for both parts
            const double inv = d[2] > 0 ? 1.0 / d[2] : 0.0;
            const float ar = (float)(d[0] * inv), ai = (float)(d[1] * inv);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const float pr = rho[2 * k], pi = rho[2 * k + 1];
                xs[2 * k] = fmad(ar, pr, xs[2 * k]);
                xs[2 * k] = fmad(-ai, pi, xs[2 * k]);
                xs[2 * k + 1] = fmad(ar, pi, xs[2 * k + 1]);
                xs[2 * k + 1] = fmad(ai, pr, xs[2 * k + 1]);
                rho[2 * k] = fmad(ai, q[2 * k + 1], fmad(-ar, q[2 * k], pr));
                rho[2 * k + 1] = fmad(-ai, q[2 * k], fmad(-ar, q[2 * k + 1], pi));
            }
        }
    } else {
    // rho lives in LDS between steps: only its owner thread writes it
#pragma unroll
    for (int k = 0; k < 24; ++k) s_rho[k * NT + l] = rho[k];
    for (int step = 0; step < a.B.n_dominv; ++step) {
        F.refresh();
        // publish the backward-hop contributions U_mu(x)^dag P+ rho(x)
        {
            float r[24], h[12], w[12];
#pragma unroll
            for (int k = 0; k < 24; ++k) r[k] = s_rho[k * NT + l];
#define WCL_BWD(MU)                                                                           \
    spin_project<MU, false>(r, h);                                                            \
    F.template step_apply<MU, true>(h, w);                                                    \
    if constexpr (DOT) {                                                                      \
        _Pragma("unroll") for (int k = 0; k < 6; ++k) s_bwd16[(MU * 6 + k) * NT + l] = pack2(w[2 * k], w[2 * k + 1]); \
    } else {                                                                                  \
        _Pragma("unroll") for (int k = 0; k < 12; ++k) s_bwd[(MU * 12 + k) * NT + l] = w[k]; \
    }
            WCL_BWD(0) WCL_BWD(1) WCL_BWD(2) WCL_BWD(3)
#undef WCL_BWD
        }
        __syncthreads();
        // q = D_{Omega'} rho
        float q[24];
        {
            float r[24];
#pragma unroll
            for (int k = 0; k < 24; ++k) r[k] = s_rho[k * NT + l];
            F.step_site_term(r, ck, q);
        }
        {
            float s[24], h[12], w[12];
#define WCL_HOPS(MU)                                                                            \
    if (nf[MU] >= 0) {                                                                          \
        _Pragma("unroll") for (int k = 0; k < 24; ++k) s[k] = s_rho[k * NT + nf[MU]];         \
        spin_project<MU, true>(s, h);                                                           \
        F.template step_apply<MU, false>(h, w);                                                 \
        spin_accumulate<MU, true>(w, mk * phf[MU], q);                                          \
    }                                                                                           \
    if (nb[MU] >= 0) {                                                                          \
        if constexpr (DOT) {                                                                    \
            _Pragma("unroll") for (int k = 0; k < 6; ++k) {                                     \
                const h2v t = s_bwd16[(MU * 6 + k) * NT + nb[MU]];                              \
                w[2 * k] = (float)t.x;                                                          \
                w[2 * k + 1] = (float)t.y;                                                      \
            }                                                                                   \
        } else {                                                                                \
            _Pragma("unroll") for (int k = 0; k < 12; ++k) w[k] = s_bwd[(MU * 12 + k) * NT + nb[MU]]; \
        }                                                                                       \
        spin_accumulate<MU, false>(w, mk * phb[MU], q);                                         \
    }
            WCL_HOPS(0) WCL_HOPS(1) WCL_HOPS(2) WCL_HOPS(3)
#undef WCL_HOPS
        }
        // <q, rho> and <q, q>: FP32 over the site's 12 components, FP64
        // across the workgroup
        double d[3] = {0.0, 0.0, 0.0};
        if (active) {
            // all 24 LDS reads issued before the arithmetic (one wait, not 12)
            float rv[24];
#pragma unroll
            for (int k = 0; k < 24; ++k) rv[k] = s_rho[k * NT + l];
            __builtin_amdgcn_sched_barrier(0);
            float f0 = 0.f, f1 = 0.f, f2 = 0.f;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const float qr = q[2 * k], qi = q[2 * k + 1];
                const float rr = rv[2 * k], ri = rv[2 * k + 1];
                f0 = fmad(qr, rr, f0);
                f0 = fmad(qi, ri, f0);
                f1 = fmad(qr, ri, f1);
                f1 = fmad(-qi, rr, f1);
                f2 = fmad(qr, qr, f2);
                f2 = fmad(qi, qi, f2);
            }
            d[0] = f0;
            d[1] = f1;
            d[2] = f2;
        }
        // every thread has finished reading its neighbours' rho and backward
        // terms after this barrier; the next reads of them follow the next
        // step's publish barrier, so the update below needs no barrier of its own
        wg_allreduce3<NT / 64>(d, s_red);
        const float ar = d[2] > 0 ? (float)(d[0] / d[2]) : 0.f;
        const float ai = d[2] > 0 ? (float)(d[1] / d[2]) : 0.f;
        float pv[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) pv[k] = s_rho[k * NT + l];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const float pr = pv[2 * k], pi = pv[2 * k + 1];
            xs[2 * k] = fmad(ar, pr, xs[2 * k]);
            xs[2 * k] = fmad(-ai, pi, xs[2 * k]);
            xs[2 * k + 1] = fmad(ar, pi, xs[2 * k + 1]);
            xs[2 * k + 1] = fmad(ai, pr, xs[2 * k + 1]);
            s_rho[(2 * k) * NT + l] = fmad(ai, q[2 * k + 1], fmad(-ar, q[2 * k], pr));
            s_rho[(2 * k + 1) * NT + l] = fmad(-ai, q[2 * k], fmad(-ar, q[2 * k + 1], pi));
        }
    }
    // the final MR residual back in registers
#pragma unroll
    for (int k = 0; k < 24; ++k) rho[k] = s_rho[k * NT + l];
    }   // FP32-operand steps
    // restriction to the owned sites and sum into the output
    if (!active || !block_owned(a.B, lc)) return;
    if constexpr (RES != 1) {
        if (a.rout) {
            // this sweep's final MR residual, the next sweep's starting point
            float rn[24];
#pragma unroll
            for (int k = 0; k < 24; ++k) rn[k] = rho[k] * scale;
            SpinorIO<VP>::store((char*)a.rout + rhs * a.rout_stride, a.g.V, gi, rn);
        }
    }
    if constexpr (DOT) {
#pragma unroll
        for (int k = 0; k < 24; ++k) xs[k] *= scale;
    }
    if (write_vj) SpinorIO<VP>::store((char*)a.vj + rhs * a.vj_stride, a.g.V, gi, xs);
    if (a.skip_out) return;
    char* out = (char*)a.out + rhs * a.out_stride;
    if (a.accumulate || a.vsum_n > 0) {
        // out (+)= the earlier sweeps' corrections, in sweep order, then x
        float o[24];
        if (a.accumulate) {
            SpinorIO<WCL_F32>::load(out, a.g.V, gi, o);
        } else {
#pragma unroll
            for (int k = 0; k < 24; ++k) o[k] = 0.f;
        }
        for (int j = 0; j < a.vsum_n; ++j) {
            float t[24];
            SpinorIO<VP>::load((const char*)a.vsum + j * a.vsum_step + rhs * a.vj_stride, a.g.V, gi, t);
#pragma unroll
            for (int k = 0; k < 24; ++k) o[k] += t[k];
        }
#pragma unroll
        for (int k = 0; k < 24; ++k) o[k] += xs[k];
        SpinorIO<WCL_F32>::store(out, a.g.V, gi, o);
    } else {
        SpinorIO<WCL_F32>::store(out, a.g.V, gi, xs);
    }
}

int fused_threads(int ev) { return ev <= 256 ? 256 : 0; }

template <int GP, int SRC, int VP, int NT, int RES, bool DOT>
static int launch_fused_t(const BlockArgs& a, hipStream_t st) {
    const size_t lds = (size_t)FusedShape<DOT>::lds_words * NT * sizeof(float);
    // dynamic LDS above the 64 KB default; set once per instantiation (thread-safe static)
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_blk_fused<GP, SRC, VP, NT, RES, DOT>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    WCL_HIP(attr);
    k_blk_fused<GP, SRC, VP, NT, RES, DOT><<<a.B.nblocks * a.nrhs, NT, lds, st>>>(a, a.vj != nullptr);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_blk_fused(const BlockArgs& a, int gp, int src_prec, hipStream_t st) {
    const int nt = fused_threads(a.B.ev);
    const int res = a.vprev == nullptr ? 0 : (a.res_boundary ? 2 : 1);
#define WCL_F(G, S, NT, D)                                                                 \
    if (gp == G && src_prec == S && nt == NT && (a.dot2 != 0) == D)                        \
        return res == 0   ? launch_fused_t<G, S, G, NT, 0, D>(a, st)                       \
               : res == 1 ? launch_fused_t<G, S, G, NT, 1, D>(a, st)                       \
                          : launch_fused_t<G, S, G, NT, 2, D>(a, st)
    WCL_F(WCL_F32, WCL_F32, 256, false);
    WCL_F(WCL_F16, WCL_F32, 256, false);
    WCL_F(WCL_F16, WCL_F16, 256, false);
    WCL_F(WCL_F16, WCL_F32, 256, true);
    WCL_F(WCL_F16, WCL_F16, 256, true);
#undef WCL_F
    wcl_set_error("fused domain solver: unsupported case (storage %d, source %d, extended volume %d, dot2 %d)", gp,
                  src_prec, a.B.ev, a.dot2);
    return WCL_EINVAL;
}
