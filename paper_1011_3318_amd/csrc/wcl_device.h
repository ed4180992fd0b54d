// Device building blocks: storage loads/stores for the three precisions,
// two-row link reconstruction, packed-Hermitian clover products, the
// chiral-basis spin projections and the per-site Wilson-clover stencil.
#pragma once

#include "wcl_internal.h"

typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f8v __attribute__((ext_vector_type(8)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

#define WCL_DEV __device__ __forceinline__

// a * b + c with one rounding.  The stencil arithmetic is written as chains
// of these into the accumulators: a sum of products such as
// acc += a*b - c*d would otherwise cost a multiply, an FMA and an add.
WCL_DEV float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
WCL_DEV double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int P>
struct Real {
    using T = float;
};
template <>
struct Real<WCL_F64> {
    using T = double;
};

// Non-temporal loads for data streamed exactly once per launch (links,
// clover); neighbour-shared spinor data uses ordinary cached loads.
#ifndef WCL_NT_LOADS
#define WCL_NT_LOADS 1
#endif
#ifndef WCL_NT_STORES
#define WCL_NT_STORES 1
#endif
#ifndef WCL_XCD_REMAP
#define WCL_XCD_REMAP 1
#endif
template <typename V>
WCL_DEV V ld_nt(const V* p) {
#if WCL_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
// NT = true: non-temporal; false: ordinary cached load (fields that a
// kernel reads several times, e.g. the domain operator's links and clover)
template <bool NT, typename V>
WCL_DEV V ldx(const V* p) {
    if constexpr (NT) return ld_nt(p);
    else return *p;
}
template <typename V>
WCL_DEV void st_nt(V* p, V v) {
#if WCL_NT_STORES
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// ------------------------------------------------------------ spinors ---
// s[24]: component k = 3*spin + colour at s[2k] (re), s[2k+1] (im).
template <int P>
struct SpinorIO;

template <>
struct SpinorIO<WCL_F64> {
    using T = double;
    WCL_DEV static void load(const void* base, int V, int i, T s[24]) {
        const d2v* p = (const d2v*)base;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            d2v v = p[tix(k, i, 12)];
            s[2 * k] = v.x;
            s[2 * k + 1] = v.y;
        }
    }
    // the spinor as stored and its scale (1 here): see SpinorIO<WCL_F16>
    using Stored = T;
    WCL_DEV static T load_s(const void* base, int V, int i, Stored s[24]) {
        load(base, V, i, s);
        return T(1);
    }
    WCL_DEV static void store(void* base, int V, int i, const T s[24]) {
        d2v* p = (d2v*)base;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            d2v v = {s[2 * k], s[2 * k + 1]};
            st_nt(p + tix(k, i, 12), v);
        }
    }
};

template <>
struct SpinorIO<WCL_F32> {
    using T = float;
    WCL_DEV static void load(const void* base, int V, int i, T s[24]) {
        const f4v* p = (const f4v*)base;
#pragma unroll
        for (int g = 0; g < 6; ++g) {
            f4v v = p[tix(g, i, 6)];
            s[4 * g] = v.x;
            s[4 * g + 1] = v.y;
            s[4 * g + 2] = v.z;
            s[4 * g + 3] = v.w;
        }
    }
    using Stored = T;
    WCL_DEV static T load_s(const void* base, int V, int i, Stored s[24]) {
        load(base, V, i, s);
        return T(1);
    }
    WCL_DEV static void store(void* base, int V, int i, const T s[24]) {
        f4v* p = (f4v*)base;
#pragma unroll
        for (int g = 0; g < 6; ++g) {
            f4v v = {s[4 * g], s[4 * g + 1], s[4 * g + 2], s[4 * g + 3]};
            st_nt(p + tix(g, i, 6), v);
        }
    }
};

// FP16 spinor: 24 binary16 values of value/scale plus an FP32 per-site
// scale = max |component| (round-to-nearest-even conversion).
template <>
struct SpinorIO<WCL_F16> {
    using T = float;
    WCL_DEV static const float* scale_ptr(const void* base, int V) {
        return (const float*)((const char*)base + half_spinor_scale_offset(V));
    }
    WCL_DEV static void load(const void* base, int V, int i, T s[24]) {
        const h8v* p = (const h8v*)base;
        float sc = scale_ptr(base, V)[i];
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            f8v v = __builtin_convertvector(p[tix(g, i, 3)], f8v);
#pragma unroll
            for (int j = 0; j < 8; ++j) s[8 * g + j] = v[j] * sc;
        }
    }
    // The stored binary16 values themselves (value / scale; consumers widen
    // them inside mixed-precision FMAs) and the scale, which is returned: a
    // linear consumer applies it once to its result.
    using Stored = _Float16;
    WCL_DEV static T load_s(const void* base, int V, int i, _Float16 s[24]) {
        const h8v* p = (const h8v*)base;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const h8v v = p[tix(g, i, 3)];
#pragma unroll
            for (int j = 0; j < 8; ++j) s[8 * g + j] = v[j];
        }
        return scale_ptr(base, V)[i];
    }
    WCL_DEV static void store(void* base, int V, int i, const T s[24]) {
        float m = 0.f;
#pragma unroll
        for (int j = 0; j < 24; ++j) m = fmaxf(m, fabsf(s[j]));
        float inv = m > 0.f ? 1.0f / m : 0.f;
        h8v* p = (h8v*)base;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            f8v v;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = s[8 * g + j] * inv;
            st_nt(p + tix(g, i, 3), __builtin_convertvector(v, h8v));
        }
        ((float*)scale_ptr(base, V))[i] = m;   // cached store: the 4-byte scales of a wavefront combine into whole lines
    }
};

// ------------------------------------------------------------- links ----
// u[18]: 3x3 complex, row-major, u[2*(3r+c)] = re.  Rows 0,1 are stored;
// row 2 = conj(row0 x row1) (exact for SU(3)).
template <typename T>
WCL_DEV void reconstruct_row2(T u[18]) {
#define RE(r, c) u[2 * (3 * (r) + (c))]
#define IM(r, c) u[2 * (3 * (r) + (c)) + 1]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        // (row0_a row1_b - row0_b row1_a)^*
        T re = RE(0, a) * RE(1, b);
        re = fmad(-IM(0, a), IM(1, b), re);
        re = fmad(-RE(0, b), RE(1, a), re);
        re = fmad(IM(0, b), IM(1, a), re);
        T im = RE(0, a) * IM(1, b);
        im = fmad(IM(0, a), RE(1, b), im);
        im = fmad(-RE(0, b), IM(1, a), im);
        im = fmad(-IM(0, b), RE(1, a), im);
        RE(2, c) = re;
        IM(2, c) = -im;
    }
#undef RE
#undef IM
}

template <int P>
struct GaugeIO;

template <>
struct GaugeIO<WCL_F64> {
    using T = double;
    // rows 0,1 only (u[0..11]); row 2 is rebuilt by load() or by the caller
    template <bool NT = true>
    WCL_DEV static void load_raw(const void* base, int V, int mu, int i, T u[18]) {
        const d2v* p = (const d2v*)base;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            d2v v = ldx<NT>(p + tix(6 * mu + k, i, 24));
            u[2 * k] = v.x;
            u[2 * k + 1] = v.y;
        }
    }
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int mu, int i, T u[18]) {
        load_raw<NT>(base, V, mu, i, u);
        reconstruct_row2(u);
    }
};

template <>
struct GaugeIO<WCL_F32> {
    using T = float;
    // rows 0,1 only (u[0..11]); row 2 is rebuilt by load() or by the caller
    template <bool NT = true>
    WCL_DEV static void load_raw(const void* base, int V, int mu, int i, T u[18]) {
        const f4v* p = (const f4v*)base;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            f4v v = ldx<NT>(p + tix(3 * mu + g, i, 12));
            u[4 * g] = v.x;
            u[4 * g + 1] = v.y;
            u[4 * g + 2] = v.z;
            u[4 * g + 3] = v.w;
        }
    }
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int mu, int i, T u[18]) {
        load_raw<NT>(base, V, mu, i, u);
        reconstruct_row2(u);
    }
};

template <>
struct GaugeIO<WCL_F16> {
    using T = float;
    // rows 0,1 only (u[0..11]); row 2 is rebuilt by load() or by the caller
    template <bool NT = true>
    WCL_DEV static void load_raw(const void* base, int V, int mu, int i, T u[18]) {
        const h4v* p = (const h4v*)base;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            f4v v = __builtin_convertvector(ldx<NT>(p + tix(3 * mu + g, i, 12)), f4v);
            u[4 * g] = v.x;
            u[4 * g + 1] = v.y;
            u[4 * g + 2] = v.z;
            u[4 * g + 3] = v.w;
        }
    }
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int mu, int i, T u[18]) {
        load_raw<NT>(base, V, mu, i, u);
        reconstruct_row2(u);
    }
};

// ------------------------------------------------------------ clover ----
// c[72]: blocks k = 0, 1 of 36 reals (6 diagonal reals, 15 complex upper
// entries row-major (0,1),(0,2)..(0,5),(1,2)..(4,5)).
template <int P>
struct CloverIO;

template <>
struct CloverIO<WCL_F64> {
    using T = double;
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int i, T c[72]) {
        const d2v* p = (const d2v*)base;
#pragma unroll
        for (int k = 0; k < 36; ++k) {
            d2v v = ldx<NT>(p + tix(k, i, 36));
            c[2 * k] = v.x;
            c[2 * k + 1] = v.y;
        }
    }
};

template <>
struct CloverIO<WCL_F32> {
    using T = float;
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int i, T c[72]) {
        const f4v* p = (const f4v*)base;
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            f4v v = ldx<NT>(p + tix(k, i, 18));
            c[4 * k] = v.x;
            c[4 * k + 1] = v.y;
            c[4 * k + 2] = v.z;
            c[4 * k + 3] = v.w;
        }
    }
};

template <>
struct CloverIO<WCL_F16> {
    using T = float;
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int i, T c[72]) {
        const h8v* p = (const h8v*)base;
        const float* sc = (const float*)((const char*)base + half_clover_scale_offset(V));
        float s = sc[i];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            f8v v = __builtin_convertvector(ldx<NT>(p + tix(k, i, 9)), f8v);
#pragma unroll
            for (int j = 0; j < 8; ++j) c[8 * k + j] = v[j] * s;
        }
    }
};

// Clover block k of 36 reals (packed Hermitian 6x6).
template <int P>
struct CloverBlk;
template <>
struct CloverBlk<WCL_F64> {
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int i, int k, double c[36]) {
        const d2v* p = (const d2v*)base;
#pragma unroll
        for (int q = 0; q < 18; ++q) {
            d2v v = ldx<NT>(p + tix(18 * k + q, i, 36));
            c[2 * q] = v.x;
            c[2 * q + 1] = v.y;
        }
    }
};
template <>
struct CloverBlk<WCL_F32> {
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int i, int k, float c[36]) {
        const f4v* p = (const f4v*)base;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            f4v v = ldx<NT>(p + tix(9 * k + q, i, 18));
            c[4 * q] = v.x;
            c[4 * q + 1] = v.y;
            c[4 * q + 2] = v.z;
            c[4 * q + 3] = v.w;
        }
    }
};
template <>
struct CloverBlk<WCL_F16> {
    // block 0 = reals 0..35 (groups 0..4), block 1 = reals 36..71 (groups 4..8)
    template <bool NT = true>
    WCL_DEV static void load(const void* base, int V, int i, int k, float c[36]) {
        const h8v* p = (const h8v*)base;
        const float* sc = (const float*)((const char*)base + half_clover_scale_offset(V));
        const float s = sc[i];
        const int off = 4 * k;   // first real of the block inside group 4k
        float t[40];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            f8v v = __builtin_convertvector(ldx<NT>(p + tix(4 * k + q, i, 9)), f8v);
#pragma unroll
            for (int j = 0; j < 8; ++j) t[8 * q + j] = v[j] * s;
        }
#pragma unroll
        for (int j = 0; j < 36; ++j) c[j] = off ? t[4 + j] : t[j];
    }
};

// y = C_k x for one packed 6x6 Hermitian block (x, y: 6 complex).
template <typename T>
WCL_DEV void herm6_apply(const T* c, const T* x, T* y) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        y[2 * a] = c[a] * x[2 * a];
        y[2 * a + 1] = c[a] * x[2 * a + 1];
    }
    int k = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a + 1; b < 6; ++b, ++k) {
            T re = c[6 + 2 * k], im = c[6 + 2 * k + 1];
            // y_a += c_ab x_b ; y_b += conj(c_ab) x_a
            y[2 * a] = fmad(re, x[2 * b], y[2 * a]);
            y[2 * a] = fmad(-im, x[2 * b + 1], y[2 * a]);
            y[2 * a + 1] = fmad(re, x[2 * b + 1], y[2 * a + 1]);
            y[2 * a + 1] = fmad(im, x[2 * b], y[2 * a + 1]);
            y[2 * b] = fmad(re, x[2 * a], y[2 * b]);
            y[2 * b] = fmad(im, x[2 * a + 1], y[2 * b]);
            y[2 * b + 1] = fmad(re, x[2 * a + 1], y[2 * b + 1]);
            y[2 * b + 1] = fmad(-im, x[2 * a], y[2 * b + 1]);
        }
}

// ----------------------------------------------------- spin projection --
// Chiral basis: gamma_k = [[0,-i s_k],[i s_k,0]], gamma_t = [[0,-1],[-1,0]].
// With psi = (u0,u1,l0,l1) the rank-2 projections are
//   (1 -+ gamma_mu) psi = (h0, h1, lower(h)),
// and after the colour matrix acts on h the lower spins are rebuilt from it.
// FWD = true: (1 - gamma_mu) (forward hop), false: (1 + gamma_mu).
template <int MU, bool FWD, typename T>
WCL_DEV void spin_project(const T s[24], T h[12]) {
    const T* u0 = s;
    const T* u1 = s + 6;
    const T* l0 = s + 12;
    const T* l1 = s + 18;
    const T sg = FWD ? T(1) : T(-1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int r = 2 * c, i = 2 * c + 1;
        if (MU == 0) {  // h0 = u0 +- i l1, h1 = u1 +- i l0
            h[r] = u0[r] - sg * l1[i];
            h[i] = u0[i] + sg * l1[r];
            h[6 + r] = u1[r] - sg * l0[i];
            h[6 + i] = u1[i] + sg * l0[r];
        } else if (MU == 1) {  // h0 = u0 +- l1, h1 = u1 -+ l0
            h[r] = u0[r] + sg * l1[r];
            h[i] = u0[i] + sg * l1[i];
            h[6 + r] = u1[r] - sg * l0[r];
            h[6 + i] = u1[i] - sg * l0[i];
        } else if (MU == 2) {  // h0 = u0 +- i l0, h1 = u1 -+ i l1
            h[r] = u0[r] - sg * l0[i];
            h[i] = u0[i] + sg * l0[r];
            h[6 + r] = u1[r] + sg * l1[i];
            h[6 + i] = u1[i] - sg * l1[r];
        } else {  // h = u +- l
            h[r] = u0[r] + sg * l0[r];
            h[i] = u0[i] + sg * l0[i];
            h[6 + r] = u1[r] + sg * l1[r];
            h[6 + i] = u1[i] + sg * l1[i];
        }
    }
}

typedef _Float16 h2v __attribute__((ext_vector_type(2)));

// Complex products on packed binary16 pairs z = (re, im) as v_dot2_f32_f16
// (both binary16 products are exact in FP32, the sum is FP32).  Every
// v_dot2 goes through the compiler builtin, none through inline asm: the
// hardware needs wait states between a DOT instruction and a different
// instruction that reads its result (or a DOT of another encoding reading
// it), and only the compiler, knowing each such instruction, provides them.
// The signs and the order of the two products sit in the second operand:
//   Re(a b) = dot2(a, conj b),   Im(a b) = dot2(a, swp b),
//   Re(conj(a) b) = dot2(a, b),  Im(conj(a) b) = dot2(a, -i b).
WCL_DEV float dot2(h2v a, h2v b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }
WCL_DEV h2v pack2(float x, float y) { return h2v{(_Float16)x, (_Float16)y}; }
// (im, re), conj z, i z and -i z of a pair: exact, and folded by the
// compiler into the operand modifiers of the packed binary16 addition that
// consumes them
WCL_DEV h2v swp(h2v z) { return __builtin_shufflevector(z, z, 1, 0); }
WCL_DEV h2v cj(h2v z) { return h2v{z.x, -z.y}; }
WCL_DEV h2v mul_i(h2v z) { return h2v{-z.y, z.x}; }
WCL_DEV h2v mul_mi(h2v z) { return h2v{z.y, -z.x}; }

// The half-spinor h = (h0, h1) of spin_project<MU,FWD> for a spinor held as
// 12 binary16 pairs (u0, u1, l0, l1 by colour), given as the operand pairs of
// su3_apply16<DAG>: (conj h, swp h) for U h, (h, -i h) for U^dag h.  Each
// pair is one packed binary16 addition u + y of the projection's two terms
// with the conjugation, swap or -i applied to both (so the rounding is that
// of h itself).
template <int MU, bool FWD, bool DAG>
WCL_DEV void spin_project16(const h2v s[12], h2v ha[6], h2v hb[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const h2v u0 = s[c], u1 = s[3 + c], l0 = s[6 + c], l1 = s[9 + c];
        h2v y0, y1;
        if (MU == 0) {   // h0 = u0 +- i l1, h1 = u1 +- i l0
            y0 = FWD ? mul_i(l1) : mul_mi(l1);
            y1 = FWD ? mul_i(l0) : mul_mi(l0);
        } else if (MU == 1) {   // h0 = u0 +- l1, h1 = u1 -+ l0
            y0 = FWD ? l1 : -l1;
            y1 = FWD ? -l0 : l0;
        } else if (MU == 2) {   // h0 = u0 +- i l0, h1 = u1 -+ i l1
            y0 = FWD ? mul_i(l0) : mul_mi(l0);
            y1 = FWD ? mul_mi(l1) : mul_i(l1);
        } else {   // h = u +- l
            y0 = FWD ? l0 : -l0;
            y1 = FWD ? l1 : -l1;
        }
        if (DAG) {
            ha[c] = u0 + y0;
            ha[3 + c] = u1 + y1;
            hb[c] = mul_mi(u0) + mul_mi(y0);
            hb[3 + c] = mul_mi(u1) + mul_mi(y1);
        } else {
            ha[c] = cj(u0) + cj(y0);
            ha[3 + c] = cj(u1) + cj(y1);
            hb[c] = swp(u0) + swp(y0);
            hb[3 + c] = swp(u1) + swp(y1);
        }
    }
}

// w = U h (DAG = false) or U^dag h, U as nine binary16 pairs (element (row,
// col) at 3 row + col), h as the operand pairs (ha, hb) of spin_project16;
// FP32 sums from the zero z (an opaque zero keeps the first product a v_dot2)
template <bool DAG>
WCL_DEV void su3_apply16(const h2v u[9], const h2v ha[6], const h2v hb[6], float z, float w[12]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re = z, im = z;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const h2v U = u[DAG ? 3 * b + a : 3 * a + b];
                re = dot2(U, ha[3 * sp + b], re);
                im = dot2(U, hb[3 * sp + b], im);
            }
            w[6 * sp + 2 * a] = re;
            w[6 * sp + 2 * a + 1] = im;
        }
}

// ------------------------------------------- FP16 storage on binary16 pairs
// An FP16 spinor as stored: 12 binary16 pairs (re, im) of value / scale in
// (spin, colour) order, and the per-site scale.
WCL_DEV float load_spinor16(const void* base, int V, int i, h2v p[12]) {
    const h8v* q = (const h8v*)base;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const h8v v = q[tix(g, i, 3)];
#pragma unroll
        for (int j = 0; j < 4; ++j) p[4 * g + j] = h2v{v[2 * j], v[2 * j + 1]};
    }
    return ((const float*)((const char*)base + half_spinor_scale_offset(V)))[i];
}

// U_mu(site) from FP16 storage as nine binary16 pairs: rows 0, 1 as stored,
// row 2 = conj(row0 x row1) from exact binary16 products summed in FP32 (z
// an opaque zero), rounded to binary16.
template <bool NT>
WCL_DEV void load_link16(const void* gauge, int V, int mu, int site, float z, h2v u[9]) {
    const h4v* gp = (const h4v*)gauge;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const h4v v = ldx<NT>(gp + tix(3 * mu + g, site, 12));
        u[2 * g] = h2v{v.x, v.y};
        u[2 * g + 1] = h2v{v.z, v.w};
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        // row0_a row1_b - row0_b row1_a, then the conjugate
        const h2v nb = -u[b];
        const float re = dot2(nb, cj(u[3 + a]), dot2(u[a], cj(u[3 + b]), z));
        const float im = dot2(nb, swp(u[3 + a]), dot2(u[a], swp(u[3 + b]), z));
        u[6 + c] = pack2(re, -im);
    }
}

// acc = A(x) psi = sc psi + ck cs sc C psi: psi as stored (12 binary16 pairs,
// scale sc), C the stored binary16 clover blocks (scale cs); the products
// are exact binary16 products summed in FP32.
template <bool NT>
WCL_DEV void clover_site16(const void* base, int V, int i, const h2v x16[12], float sc, float ck, float z,
                           float acc[24]) {
    const h8v* p = (const h8v*)base;
    h8v cv[9];
#pragma unroll
    for (int g = 0; g < 9; ++g) cv[g] = ldx<NT>(p + tix(g, i, 9));
    const float f = ck * sc * ((const float*)((const char*)base + half_clover_scale_offset(V)))[i];
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) {
        // block bk: halves 36 bk + (6 diagonal reals, then 15 complex entries)
        auto hv = [&](int k) { return cv[(36 * bk + k) / 8][(36 * bk + k) % 8]; };
        const h2v* xp = x16 + 6 * bk;
        float y[12];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            y[2 * a] = fmad((float)hv(a), (float)xp[a].x, z);
            y[2 * a + 1] = fmad((float)hv(a), (float)xp[a].y, z);
        }
        int k = 0;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = a + 1; b < 6; ++b, ++k) {
                const h2v C = h2v{hv(6 + 2 * k), hv(7 + 2 * k)};   // C_ab; C_ba = conj(C_ab)
                y[2 * a] = dot2(C, cj(xp[b]), y[2 * a]);
                y[2 * a + 1] = dot2(C, swp(xp[b]), y[2 * a + 1]);
                y[2 * b] = dot2(C, xp[a], y[2 * b]);
                y[2 * b + 1] = dot2(C, mul_mi(xp[a]), y[2 * b + 1]);
            }
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            acc[12 * bk + 2 * a] = fmad(f, y[2 * a], fmad((float)xp[a].x, sc, z));
            acc[12 * bk + 2 * a + 1] = fmad(f, y[2 * a + 1], fmad((float)xp[a].y, sc, z));
        }
    }
}

// acc += f * (w0, w1, lower(w)) for the projection spin_project<MU,FWD>.
template <int MU, bool FWD, typename T>
WCL_DEV void spin_accumulate(const T w[12], T f, T acc[24]) {
    const T sg = FWD ? T(1) : T(-1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int r = 2 * c, i = 2 * c + 1;
        const T w0r = w[r], w0i = w[i], w1r = w[6 + r], w1i = w[6 + i];
        acc[r] += f * w0r;
        acc[i] += f * w0i;
        acc[6 + r] += f * w1r;
        acc[6 + i] += f * w1i;
        if (MU == 0) {  // lower = -+i (w1, w0)
            acc[12 + r] += f * (sg * w1i);
            acc[12 + i] += f * (-sg * w1r);
            acc[18 + r] += f * (sg * w0i);
            acc[18 + i] += f * (-sg * w0r);
        } else if (MU == 1) {  // lower = -+(w1, -w0)
            acc[12 + r] += f * (-sg * w1r);
            acc[12 + i] += f * (-sg * w1i);
            acc[18 + r] += f * (sg * w0r);
            acc[18 + i] += f * (sg * w0i);
        } else if (MU == 2) {  // lower = -+i (w0, -w1)
            acc[12 + r] += f * (sg * w0i);
            acc[12 + i] += f * (-sg * w0r);
            acc[18 + r] += f * (-sg * w1i);
            acc[18 + i] += f * (sg * w1r);
        } else {  // lower = +-(w0, w1)
            acc[12 + r] += f * (sg * w0r);
            acc[12 + i] += f * (sg * w0i);
            acc[18 + r] += f * (sg * w1r);
            acc[18 + i] += f * (sg * w1i);
        }
    }
}

// w = U h (DAG = false) or U^dag h (DAG = true), h/w: 2 colour vectors.
template <bool DAG, typename T>
WCL_DEV void su3_apply2(const T u[18], const T h[12], T w[12]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int ab = DAG ? 2 * (3 * b + a) : 2 * (3 * a + b);
                const T ur = u[ab], ui = DAG ? -u[ab + 1] : u[ab + 1];
                const T hr = h[6 * sp + 2 * b], hi = h[6 * sp + 2 * b + 1];
                re = fmad(ur, hr, re);
                re = fmad(-ui, hi, re);
                im = fmad(ur, hi, im);
                im = fmad(ui, hr, im);
            }
            w[6 * sp + 2 * a] = re;
            w[6 * sp + 2 * a + 1] = im;
        }
}

// acc = s + csw*kappa * C s (the site-diagonal term A(x) s).
template <typename T>
WCL_DEV void clover_term(const T c[72], const T s[24], T ck, T acc[24]) {
    T y[12];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        herm6_apply(c + 36 * k, s + 12 * k, y);
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[12 * k + j] = fmad(ck, y[j], s[12 * k + j]);
    }
}

// acc = psi + ck C psi with the FP16 clover: its 72 stored binary16 values
// (value / scale) feed mixed-precision FMAs directly, and the per-site scale
// joins ck.  z is an opaque zero for the heads of the FMA chains (a plain
// multiply has no mixed-precision form and would widen first).
template <bool NT>
WCL_DEV void clover_site_f16(const void* base, int V, int i, const float psi[24], float ck, float z,
                             float acc[24]) {
    const h8v* p = (const h8v*)base;
    h8v g[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) g[k] = ldx<NT>(p + tix(k, i, 9));
    const float f = ck * ((const float*)((const char*)base + half_clover_scale_offset(V)))[i];
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) {
        const int o = 36 * bk;
        const float* x = psi + 12 * bk;
#define WCL_CV(k) ((float)g[(o + (k)) >> 3][(o + (k)) & 7])
        float y[12];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            y[2 * a] = fmad(WCL_CV(a), x[2 * a], z);
            y[2 * a + 1] = fmad(WCL_CV(a), x[2 * a + 1], z);
        }
        int k = 0;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = a + 1; b < 6; ++b, ++k) {
                const float re = WCL_CV(6 + 2 * k), im = WCL_CV(6 + 2 * k + 1);
                y[2 * a] = fmad(re, x[2 * b], y[2 * a]);
                y[2 * a] = fmad(-im, x[2 * b + 1], y[2 * a]);
                y[2 * a + 1] = fmad(re, x[2 * b + 1], y[2 * a + 1]);
                y[2 * a + 1] = fmad(im, x[2 * b], y[2 * a + 1]);
                y[2 * b] = fmad(re, x[2 * a], y[2 * b]);
                y[2 * b] = fmad(im, x[2 * a + 1], y[2 * b]);
                y[2 * b + 1] = fmad(re, x[2 * a + 1], y[2 * b + 1]);
                y[2 * b + 1] = fmad(-im, x[2 * a], y[2 * b + 1]);
            }
#undef WCL_CV
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[12 * bk + j] = fmad(f, y[j], x[j]);
    }
}

// spin_project from stored binary16 values: each half-spinor component is
// one FMA u +- l with both operands widened inside it (the same value as
// widening first and adding).
template <int MU, bool FWD>
WCL_DEV void spin_project(const _Float16 s[24], float h[12]) {
    const _Float16* u0 = s;
    const _Float16* u1 = s + 6;
    const _Float16* l0 = s + 12;
    const _Float16* l1 = s + 18;
    // an opaque +-1 keeps the compiler from turning the FMA into a widen and add
    float sg = FWD ? 1.f : -1.f;
    asm volatile("" : "+v"(sg));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int r = 2 * c, i = 2 * c + 1;
        if (MU == 0) {
            h[r] = fmad((float)l1[i], -sg, (float)u0[r]);
            h[i] = fmad((float)l1[r], sg, (float)u0[i]);
            h[6 + r] = fmad((float)l0[i], -sg, (float)u1[r]);
            h[6 + i] = fmad((float)l0[r], sg, (float)u1[i]);
        } else if (MU == 1) {
            h[r] = fmad((float)l1[r], sg, (float)u0[r]);
            h[i] = fmad((float)l1[i], sg, (float)u0[i]);
            h[6 + r] = fmad((float)l0[r], -sg, (float)u1[r]);
            h[6 + i] = fmad((float)l0[i], -sg, (float)u1[i]);
        } else if (MU == 2) {
            h[r] = fmad((float)l0[i], -sg, (float)u0[r]);
            h[i] = fmad((float)l0[r], sg, (float)u0[i]);
            h[6 + r] = fmad((float)l1[i], sg, (float)u1[r]);
            h[6 + i] = fmad((float)l1[r], -sg, (float)u1[i]);
        } else {
            h[r] = fmad((float)l0[r], sg, (float)u0[r]);
            h[i] = fmad((float)l0[i], sg, (float)u0[i]);
            h[6 + r] = fmad((float)l1[r], sg, (float)u1[r]);
            h[6 + i] = fmad((float)l1[i], sg, (float)u1[i]);
        }
    }
}

// One hop from already-loaded data: s = neighbour spinor, u = rows 0,1 of
// the link (row 2 rebuilt here).  Forward: (1 - gamma_mu) U_mu(x) psi(x+mu);
// backward: (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu).
template <int MU, bool FWD, typename S, typename T>
WCL_DEV void hop_compute(const S s[24], T u[18], T f, T acc[24]) {
    T h[12], w[12];
    reconstruct_row2(u);
    spin_project<MU, FWD>(s, h);
    su3_apply2<!FWD>(u, h, w);
    spin_accumulate<MU, FWD>(w, f, acc);
}

// One hop on binary16 pairs: s = the neighbour spinor as stored (value /
// scale), u = the link, f = -kappa x phase x the neighbour's scale.
template <int MU, bool FWD>
WCL_DEV void hop_compute16(const h2v s[12], const h2v u[9], float f, float z, float acc[24]) {
    h2v ha[6], hb[6];
    float w[12];
    spin_project16<MU, FWD, !FWD>(s, ha, hb);
    su3_apply16<!FWD>(u, ha, hb, z, w);
    spin_accumulate<MU, FWD>(w, f, acc);
}

// The eight hops in the order (x+, x-, y+, y-, z+, z-, t+, t-): neighbour
// site, link site and boundary phase of each.
template <typename T>
WCL_DEV void hop_sites(const Geom& g, int i, const int x[4], int nbr[8], int lnk[8], T ph[8]) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        int y[4] = {x[0], x[1], x[2], x[3]};
        const bool wf = x[mu] + 1 == g.L[mu];
        y[mu] = wf ? 0 : x[mu] + 1;
        nbr[2 * mu] = geom_index(g, y);
        lnk[2 * mu] = i;
        ph[2 * mu] = wf ? T(g.bc[mu]) : T(1);
        const bool wb = x[mu] == 0;
        y[mu] = wb ? g.L[mu] - 1 : x[mu] - 1;
        nbr[2 * mu + 1] = geom_index(g, y);
        lnk[2 * mu + 1] = nbr[2 * mu + 1];
        ph[2 * mu + 1] = wb ? T(g.bc[mu]) : T(1);
    }
}

// <a, b> (complex) and |b|^2 over one site's 12 components, added to d: FMA
// chains in the arithmetic precision, then one conversion to FP64 each.
template <typename T>
WCL_DEV void site_dot3(const T a[24], const T b[24], double d[3]) {
    T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const T ar = a[2 * k], ai = a[2 * k + 1], br = b[2 * k], bi = b[2 * k + 1];
        s0 = fmad(ar, br, s0);
        s0 = fmad(ai, bi, s0);
        s1 = fmad(ar, bi, s1);
        s1 = fmad(-ai, br, s1);
        s2 = fmad(br, br, s2);
        s2 = fmad(bi, bi, s2);
    }
    d[0] += (double)s0;
    d[1] += (double)s1;
    d[2] += (double)s2;
}

// ------------------------------------------------------ XCD remapping ---
// Workgroups are dispatched round-robin over the 8 XCDs; remap so that
// each XCD walks a contiguous range of logical workgroup ids (and thereby a
// contiguous piece of the column-ordered lattice in its own L2).
WCL_DEV int xcd_remap(int b, int n) {
    if (!WCL_XCD_REMAP) return b;
    const int nx = 8;
    int xcd = b % nx, k = b / nx;
    int q = n / nx, r = n % nx;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// --------------------------------------------------------- reductions ---
// v of the lane selected by the DPP pattern CTRL (both 32-bit halves moved)
template <int CTRL>
WCL_DEV double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
WCL_DEV double lane_read(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes (all active), the same value in every lane: DPP
// butterflies inside each row of 16 (quad_perm [1,0,3,2], quad_perm
// [2,3,0,1], row_half_mirror, row_mirror; each pair adds the same two
// values, so every lane of a row ends with the same bits), then the four
// row sums read in a fixed order.  No LDS traffic and no bpermute latency.
WCL_DEV double wave_sum(double v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    v += dpp_move<0x140>(v);
    return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

// The same butterflies in FP32 (the compiler fuses each move into the add
// that takes it, v_add_f32 with a DPP operand), then the four row sums.
template <int CTRL>
WCL_DEV float dpp_movef(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
WCL_DEV float lane_readf(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
WCL_DEV float wave_sumf(float v) {
    v += dpp_movef<0xB1>(v);
    v += dpp_movef<0x4E>(v);
    v += dpp_movef<0x141>(v);
    v += dpp_movef<0x140>(v);
    return (lane_readf(v, 0) + lane_readf(v, 16)) + (lane_readf(v, 32) + lane_readf(v, 48));
}

// Sum of d[0..2] over the workgroup (up to 1024 threads) in a fixed order;
// thread 0 writes the three sums to out.
WCL_DEV void block_reduce3(double d[3], double* out) {
    __shared__ double sh[16][3];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = wave_sum(d[k]);
    if (l == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) sh[w][k] = d[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int q = 0; q < nw; ++q) s += sh[q][k];
            out[k] = s;
        }
    }
}

// ------------------------------------------- direction-generic stencil --
// Same projections as spin_project / spin_accumulate, but with mu chosen at
// run time, so that the lanes of one wavefront can take different
// directions without diverging.  In the chiral basis
//   (1 -+ gamma_mu) psi:  h0 = u0 + c0 l_p0,  h1 = u1 + c1 l_p1,
//   lower spins       :  (d0 w_q0, d1 w_q1),  q = p,
// with, for the forward hop (1 - gamma_mu) (backward: c, d negated),
//   mu :  c0   c1   p0  d0   d1
//   x  :  i    i    1   -i   -i
//   y  :  1    -1   1   -1   1
//   z  :  i    -i   0   -i   i
//   t  :  1    1    0   1    1
struct RtCoef {
    float c0r, c0i, c1r, c1i, d0r, d0i, d1r, d1i;
    int p0;
};

WCL_DEV RtCoef rt_coef(int mu, bool fwd) {
    RtCoef k;
    const float s = fwd ? 1.f : -1.f;
    const bool ev = (mu & 1) == 0;
    k.c0r = ev ? 0.f : s;
    k.c0i = ev ? s : 0.f;
    k.c1r = mu == 0 ? 0.f : (mu == 1 ? -s : (mu == 2 ? 0.f : s));
    k.c1i = mu == 0 ? s : (mu == 2 ? -s : 0.f);
    k.d0r = mu == 1 ? -s : (mu == 3 ? s : 0.f);
    k.d0i = (mu == 0 || mu == 2) ? -s : 0.f;
    k.d1r = (mu == 1 || mu == 3) ? s : 0.f;
    k.d1i = mu == 0 ? -s : (mu == 2 ? s : 0.f);
    k.p0 = mu < 2 ? 1 : 0;
    return k;
}

template <typename T>
WCL_DEV void spin_project_rt(const RtCoef& k, const T s[24], T h[12]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int r = 2 * c, i = 2 * c + 1;
        const T l0r = s[12 + r], l0i = s[12 + i], l1r = s[18 + r], l1i = s[18 + i];
        const T ar = k.p0 ? l1r : l0r, ai = k.p0 ? l1i : l0i;   // l_p0
        const T br = k.p0 ? l0r : l1r, bi = k.p0 ? l0i : l1i;   // l_p1
        h[r] = s[r] + (T)k.c0r * ar - (T)k.c0i * ai;
        h[i] = s[i] + (T)k.c0r * ai + (T)k.c0i * ar;
        h[6 + r] = s[6 + r] + (T)k.c1r * br - (T)k.c1i * bi;
        h[6 + i] = s[6 + i] + (T)k.c1r * bi + (T)k.c1i * br;
    }
}

template <typename T>
WCL_DEV void spin_accumulate_rt(const RtCoef& k, const T w[12], T f, T acc[24]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int r = 2 * c, i = 2 * c + 1;
        const T w0r = w[r], w0i = w[i], w1r = w[6 + r], w1i = w[6 + i];
        acc[r] += f * w0r;
        acc[i] += f * w0i;
        acc[6 + r] += f * w1r;
        acc[6 + i] += f * w1i;
        const T ar = k.p0 ? w1r : w0r, ai = k.p0 ? w1i : w0i;   // w_q0
        const T br = k.p0 ? w0r : w1r, bi = k.p0 ? w0i : w1i;   // w_q1
        acc[12 + r] += f * ((T)k.d0r * ar - (T)k.d0i * ai);
        acc[12 + i] += f * ((T)k.d0r * ai + (T)k.d0i * ar);
        acc[18 + r] += f * ((T)k.d1r * br - (T)k.d1i * bi);
        acc[18 + i] += f * ((T)k.d1r * bi + (T)k.d1i * br);
    }
}

// component mu of x[4] without dynamic register indexing
WCL_DEV int pick(const int x[4], int mu) { return mu == 0 ? x[0] : mu == 1 ? x[1] : mu == 2 ? x[2] : x[3]; }
WCL_DEV void put(int x[4], int mu, int v) {
    x[0] = mu == 0 ? v : x[0];
    x[1] = mu == 1 ? v : x[1];
    x[2] = mu == 2 ? v : x[2];
    x[3] = mu == 3 ? v : x[3];
}
