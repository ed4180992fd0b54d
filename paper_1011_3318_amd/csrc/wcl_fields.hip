// Field set-up kernels: spinor pack/unpack between the FP64 host-order AoS
// layout and the device SoA layouts, two-row link packing, and the device
// build of the clover field C(x) = i sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}.
#include "wcl_device.h"
#include "wcl_kernels.h"

// ------------------------------------------------------------- spinors ---
template <int P>
__global__ __launch_bounds__(256) void k_pack_spinor(Geom g, int nrhs, const double* __restrict__ aos, char* soa,
                                                     size_t stride) {
    using T = typename SpinorIO<P>::T;
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)g.V * nrhs) return;
    int rhs = (int)(tid / g.V), j = (int)(tid % g.V);
    int x[4];
    canonical_coords(g, j, x);
    int i = geom_index(g, x);
    const double* src = aos + ((size_t)rhs * g.V + j) * 24;
    T s[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) s[k] = (T)src[k];
    SpinorIO<P>::store(soa + rhs * stride, g.V, i, s);
}

template <int P>
__global__ __launch_bounds__(256) void k_unpack_spinor(Geom g, int nrhs, const char* soa, size_t stride,
                                                       double* __restrict__ aos) {
    using T = typename SpinorIO<P>::T;
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)g.V * nrhs) return;
    int rhs = (int)(tid / g.V), j = (int)(tid % g.V);
    int x[4];
    canonical_coords(g, j, x);
    int i = geom_index(g, x);
    T s[24];
    SpinorIO<P>::load(soa + rhs * stride, g.V, i, s);
    double* dst = aos + ((size_t)rhs * g.V + j) * 24;
#pragma unroll
    for (int k = 0; k < 24; ++k) dst[k] = (double)s[k];
}

int launch_pack_spinor(const Geom& g, int prec, int nrhs, const double* aos, void* soa, size_t stride,
                       hipStream_t st) {
    int64_t n = (int64_t)g.V * nrhs;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (prec) {
        case WCL_F64: k_pack_spinor<WCL_F64><<<grid, block, 0, st>>>(g, nrhs, aos, (char*)soa, stride); break;
        case WCL_F32: k_pack_spinor<WCL_F32><<<grid, block, 0, st>>>(g, nrhs, aos, (char*)soa, stride); break;
        default: k_pack_spinor<WCL_F16><<<grid, block, 0, st>>>(g, nrhs, aos, (char*)soa, stride); break;
    }
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_unpack_spinor(const Geom& g, int prec, int nrhs, const void* soa, size_t stride, double* aos,
                         hipStream_t st) {
    int64_t n = (int64_t)g.V * nrhs;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (prec) {
        case WCL_F64: k_unpack_spinor<WCL_F64><<<grid, block, 0, st>>>(g, nrhs, (const char*)soa, stride, aos); break;
        case WCL_F32: k_unpack_spinor<WCL_F32><<<grid, block, 0, st>>>(g, nrhs, (const char*)soa, stride, aos); break;
        default: k_unpack_spinor<WCL_F16><<<grid, block, 0, st>>>(g, nrhs, (const char*)soa, stride, aos); break;
    }
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

// --------------------------------------------------------------- gauge ---
// AoS FP64 [V][4][3][3] (canonical order) -> rows 0,1 of every link in the
// three device layouts.
__global__ __launch_bounds__(256) void k_pack_gauge(Geom g, const double* __restrict__ aos, double* g64, float* g32,
                                                    _Float16* g16) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.V) return;
    int x[4];
    canonical_coords(g, j, x);
    int i = geom_index(g, x);
    const size_t V = g.V;
    for (int mu = 0; mu < 4; ++mu) {
        const double* u = aos + ((size_t)j * 4 + mu) * 18;
        // 12 reals: row 0 (3 complex) then row 1
        for (int k = 0; k < 6; ++k) {
            ((d2v*)g64)[tix(6 * mu + k, i, 24)] = d2v{u[2 * k], u[2 * k + 1]};
        }
        for (int q = 0; q < 3; ++q) {
            f4v v = {(float)u[4 * q], (float)u[4 * q + 1], (float)u[4 * q + 2], (float)u[4 * q + 3]};
            ((f4v*)g32)[tix(3 * mu + q, i, 12)] = v;
            // binary16 directly (|U_ij| <= 1), one rounding from FP64
            h4v hv;
            hv[0] = (_Float16)u[4 * q];
            hv[1] = (_Float16)u[4 * q + 1];
            hv[2] = (_Float16)u[4 * q + 2];
            hv[3] = (_Float16)u[4 * q + 3];
            ((h4v*)g16)[tix(3 * mu + q, i, 12)] = hv;
        }
    }
}

int launch_pack_gauge(const Geom& g, const double* aos, void* g64, void* g32, void* g16, hipStream_t st) {
    k_pack_gauge<<<(g.V + 255) / 256, 256, 0, st>>>(g, aos, (double*)g64, (float*)g32, (_Float16*)g16);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

// -------------------------------------------------------------- clover ---
struct M3d {
    double m[18];
};

__device__ M3d load_link64(const Geom& g, const void* g64, const int x[4], int mu) {
    M3d A;
    GaugeIO<WCL_F64>::load(g64, g.V, mu, geom_index(g, x), A.m);
    return A;
}

// C = A * op(B), op = identity or dagger
template <bool DAGB>
__device__ M3d m3_mul(const M3d& A, const M3d& B) {
    M3d C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double re = 0, im = 0;
            for (int k = 0; k < 3; ++k) {
                double ar = A.m[2 * (3 * i + k)], ai = A.m[2 * (3 * i + k) + 1];
                double br, bi;
                if (DAGB) {
                    br = B.m[2 * (3 * j + k)];
                    bi = -B.m[2 * (3 * j + k) + 1];
                } else {
                    br = B.m[2 * (3 * k + j)];
                    bi = B.m[2 * (3 * k + j) + 1];
                }
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            C.m[2 * (3 * i + j)] = re;
            C.m[2 * (3 * i + j) + 1] = im;
        }
    return C;
}

__device__ M3d m3_dag(const M3d& A) {
    M3d C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            C.m[2 * (3 * i + j)] = A.m[2 * (3 * j + i)];
            C.m[2 * (3 * i + j) + 1] = -A.m[2 * (3 * j + i) + 1];
        }
    return C;
}

__device__ void shifted(const Geom& g, const int x[4], int mu, int dm, int nu, int dn, int y[4]) {
    for (int k = 0; k < 4; ++k) y[k] = x[k];
    y[mu] = (y[mu] + dm + g.L[mu]) % g.L[mu];
    if (dn) y[nu] = (y[nu] + dn + g.L[nu]) % g.L[nu];
}

// Fhat_{mu nu}(x) = (1/8)[(Q - Q^dag) - 1/3 Tr(Q - Q^dag)], Q = sum of the
// four plaquette leaves at x in the (mu, nu) plane (links are periodic).
__device__ M3d fhat(const Geom& g, const void* g64, const int x[4], int mu, int nu) {
    int xpm[4], xpn[4], xmm[4], xmn[4], xpnmm[4], xmmmn[4], xpmmn[4];
    shifted(g, x, mu, 1, nu, 0, xpm);
    shifted(g, x, nu, 1, mu, 0, xpn);
    shifted(g, x, mu, -1, nu, 0, xmm);
    shifted(g, x, nu, -1, mu, 0, xmn);
    shifted(g, x, mu, -1, nu, 1, xpnmm);
    shifted(g, x, mu, -1, nu, -1, xmmmn);
    shifted(g, x, mu, 1, nu, -1, xpmmn);
    M3d Umx = load_link64(g, g64, x, mu), Unx = load_link64(g, g64, x, nu);
    // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    M3d Q = m3_mul<true>(m3_mul<true>(m3_mul<false>(Umx, load_link64(g, g64, xpm, nu)), load_link64(g, g64, xpn, mu)),
                         Unx);
    // leaf 2: U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    M3d Ummm = load_link64(g, g64, xmm, mu);
    M3d L2 = m3_mul<false>(
        m3_mul<true>(m3_mul<true>(Unx, load_link64(g, g64, xpnmm, mu)), load_link64(g, g64, xmm, nu)), Ummm);
    // leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    M3d Unmn = load_link64(g, g64, xmn, nu);
    M3d L3 = m3_mul<false>(
        m3_mul<false>(m3_mul<true>(m3_dag(Ummm), load_link64(g, g64, xmmmn, nu)), load_link64(g, g64, xmmmn, mu)),
        Unmn);
    // leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
    M3d L4 = m3_mul<true>(
        m3_mul<false>(m3_mul<false>(m3_dag(Unmn), load_link64(g, g64, xmn, mu)), load_link64(g, g64, xpmmn, nu)),
        Umx);
    for (int k = 0; k < 18; ++k) Q.m[k] += L2.m[k] + L3.m[k] + L4.m[k];
    M3d F;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            F.m[2 * (3 * i + j)] = Q.m[2 * (3 * i + j)] - Q.m[2 * (3 * j + i)];
            F.m[2 * (3 * i + j) + 1] = Q.m[2 * (3 * i + j) + 1] + Q.m[2 * (3 * j + i) + 1];
        }
    double trr = (F.m[0] + F.m[8] + F.m[16]) / 3.0, tri = (F.m[1] + F.m[9] + F.m[17]) / 3.0;
    for (int i = 0; i < 3; ++i) {
        F.m[2 * (4 * i)] -= trr;
        F.m[2 * (4 * i) + 1] -= tri;
    }
    for (int k = 0; k < 18; ++k) F.m[k] *= 0.125;
    return F;
}

// One chiral block: M = i (s3 (x) A3 + s1 (x) A1 + s2 (x) A2)
//                     = [[iA3, iA1 + A2], [iA1 - A2, -iA3]]  (spin 2x2 of colour 3x3)
// packed as 6 real diagonal entries + 15 complex upper entries.
__device__ void pack_block(const M3d& A3, const M3d& A1, const M3d& A2, double out[36]) {
    double M[6][6][2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            int k = 2 * (3 * a + b);
            double a3r = A3.m[k], a3i = A3.m[k + 1], a1r = A1.m[k], a1i = A1.m[k + 1], a2r = A2.m[k], a2i = A2.m[k + 1];
            // i*z = (-im, re)
            M[a][b][0] = -a3i;
            M[a][b][1] = a3r;
            M[a][3 + b][0] = -a1i + a2r;
            M[a][3 + b][1] = a1r + a2i;
            M[3 + a][b][0] = -a1i - a2r;
            M[3 + a][b][1] = a1r - a2i;
            M[3 + a][3 + b][0] = a3i;
            M[3 + a][3 + b][1] = -a3r;
        }
    for (int a = 0; a < 6; ++a) out[a] = M[a][a][0];
    int k = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = a + 1; b < 6; ++b, ++k) {
            out[6 + 2 * k] = M[a][b][0];
            out[6 + 2 * k + 1] = M[a][b][1];
        }
}

__device__ void store_clover_site(int V, int i, const double c[72], void* c64, void* c32, void* c16) {
    for (int k = 0; k < 36; ++k) ((d2v*)c64)[tix(k, i, 36)] = d2v{c[2 * k], c[2 * k + 1]};
    for (int k = 0; k < 18; ++k)
        ((f4v*)c32)[tix(k, i, 18)] = f4v{(float)c[4 * k], (float)c[4 * k + 1], (float)c[4 * k + 2], (float)c[4 * k + 3]};
    double m = 0;
    for (int k = 0; k < 72; ++k) m = fmax(m, fabs(c[k]));
    double inv = m > 0 ? 1.0 / m : 0.0;
    for (int k = 0; k < 9; ++k) {
        h8v hv;
        for (int j = 0; j < 8; ++j) hv[j] = (_Float16)(float)(c[8 * k + j] * inv);
        ((h8v*)c16)[tix(k, i, 9)] = hv;
    }
    float* sc = (float*)((char*)c16 + half_clover_scale_offset(V));
    sc[i] = (float)m;
}

__global__ __launch_bounds__(128) void k_clover_build(Geom g, const void* g64, void* c64, void* c32, void* c16) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    int x[4];
    geom_coords(g, i, x);
    M3d F01 = fhat(g, g64, x, 0, 1), F02 = fhat(g, g64, x, 0, 2), F03 = fhat(g, g64, x, 0, 3);
    M3d F12 = fhat(g, g64, x, 1, 2), F13 = fhat(g, g64, x, 1, 3), F23 = fhat(g, g64, x, 2, 3);
    M3d A3, A1, A2;
    double c[72];
    // spins 0,1:  sum sigma F = s3(-F_xy - F_zt) + s1(-F_xt - F_yz) + s2(F_xz - F_yt)
    for (int k = 0; k < 18; ++k) {
        A3.m[k] = -F01.m[k] - F23.m[k];
        A1.m[k] = -F03.m[k] - F12.m[k];
        A2.m[k] = F02.m[k] - F13.m[k];
    }
    pack_block(A3, A1, A2, c);
    // spins 2,3:  s3(-F_xy + F_zt) + s1(F_xt - F_yz) + s2(F_xz + F_yt)
    for (int k = 0; k < 18; ++k) {
        A3.m[k] = -F01.m[k] + F23.m[k];
        A1.m[k] = F03.m[k] - F12.m[k];
        A2.m[k] = F02.m[k] + F13.m[k];
    }
    pack_block(A3, A1, A2, c + 36);
    store_clover_site(g.V, i, c, c64, c32, c16);
}

int launch_clover_build(const Geom& g, const void* g64, void* c64, void* c32, void* c16, hipStream_t st) {
    k_clover_build<<<(g.V + 127) / 128, 128, 0, st>>>(g, g64, c64, c32, c16);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

// host-packed clover (canonical order, double[V][72]) -> device layouts
__global__ __launch_bounds__(256) void k_pack_clover(Geom g, const double* __restrict__ host, void* c64, void* c32,
                                                     void* c16) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.V) return;
    int x[4];
    canonical_coords(g, j, x);
    double c[72];
    for (int k = 0; k < 72; ++k) c[k] = host[(size_t)j * 72 + k];
    store_clover_site(g.V, geom_index(g, x), c, c64, c32, c16);
}

__global__ __launch_bounds__(256) void k_unpack_clover(Geom g, const void* c64, double* __restrict__ host) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.V) return;
    int x[4];
    canonical_coords(g, j, x);
    double c[72];
    CloverIO<WCL_F64>::load(c64, g.V, geom_index(g, x), c);
    for (int k = 0; k < 72; ++k) host[(size_t)j * 72 + k] = c[k];
}

int launch_pack_clover(const Geom& g, const double* host_dev, void* c64, void* c32, void* c16, hipStream_t st) {
    k_pack_clover<<<(g.V + 255) / 256, 256, 0, st>>>(g, host_dev, c64, c32, c16);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

int launch_unpack_clover(const Geom& g, const void* c64, double* host_dev, hipStream_t st) {
    k_unpack_clover<<<(g.V + 255) / 256, 256, 0, st>>>(g, c64, host_dev);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}

// ------------------------------------------------- site-term inverse ----
// A(x) = 1 + csw kappa C(x) is block-diagonal in the chiral basis: two 6x6
// Hermitian blocks.  Each block is inverted in FP64 by Gauss-Jordan
// elimination with partial pivoting (A need not be positive definite); the
// inverse is Hermitian and is stored packed exactly like the clover field
// (upper triangle), so the clover loaders and herm6_apply serve it too.
__device__ bool herm6_inverse(const double c[36], double ck, double out[36]) {
    double m[6][6][2], v[6][6][2];
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            m[a][b][0] = m[a][b][1] = 0.0;
            v[a][b][0] = a == b ? 1.0 : 0.0;
            v[a][b][1] = 0.0;
        }
    for (int a = 0; a < 6; ++a) m[a][a][0] = 1.0 + ck * c[a];
    int k = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = a + 1; b < 6; ++b, ++k) {
            m[a][b][0] = ck * c[6 + 2 * k];
            m[a][b][1] = ck * c[6 + 2 * k + 1];
            m[b][a][0] = m[a][b][0];
            m[b][a][1] = -m[a][b][1];
        }
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        double best = m[col][col][0] * m[col][col][0] + m[col][col][1] * m[col][col][1];
        for (int r = col + 1; r < 6; ++r) {
            const double q = m[r][col][0] * m[r][col][0] + m[r][col][1] * m[r][col][1];
            if (q > best) {
                best = q;
                piv = r;
            }
        }
        if (!(best > 0.0) || !isfinite(best)) return false;
        if (piv != col)
            for (int j = 0; j < 6; ++j)
                for (int z = 0; z < 2; ++z) {
                    double t = m[col][j][z];
                    m[col][j][z] = m[piv][j][z];
                    m[piv][j][z] = t;
                    t = v[col][j][z];
                    v[col][j][z] = v[piv][j][z];
                    v[piv][j][z] = t;
                }
        // row col /= pivot
        const double pr = m[col][col][0] / best, pi = -m[col][col][1] / best;   // 1 / pivot
        for (int j = 0; j < 6; ++j) {
            double re = m[col][j][0] * pr - m[col][j][1] * pi, im = m[col][j][0] * pi + m[col][j][1] * pr;
            m[col][j][0] = re;
            m[col][j][1] = im;
            re = v[col][j][0] * pr - v[col][j][1] * pi;
            im = v[col][j][0] * pi + v[col][j][1] * pr;
            v[col][j][0] = re;
            v[col][j][1] = im;
        }
        for (int r = 0; r < 6; ++r) {
            if (r == col) continue;
            const double fr = m[r][col][0], fi = m[r][col][1];
            for (int j = 0; j < 6; ++j) {
                m[r][j][0] -= fr * m[col][j][0] - fi * m[col][j][1];
                m[r][j][1] -= fr * m[col][j][1] + fi * m[col][j][0];
                v[r][j][0] -= fr * v[col][j][0] - fi * v[col][j][1];
                v[r][j][1] -= fr * v[col][j][1] + fi * v[col][j][0];
            }
        }
    }
    for (int a = 0; a < 6; ++a) out[a] = v[a][a][0];
    k = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = a + 1; b < 6; ++b, ++k) {
            out[6 + 2 * k] = v[a][b][0];
            out[6 + 2 * k + 1] = v[a][b][1];
        }
    return true;
}

__global__ __launch_bounds__(64) void k_site_inverse(Geom g, const void* c64, double ck, void* a64, void* a32, void* a16,
                                                     int* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    double c[72], r[72];
    CloverIO<WCL_F64>::load(c64, g.V, i, c);
    bool ok = herm6_inverse(c, ck, r) && herm6_inverse(c + 36, ck, r + 36);
    if (!ok) {
        atomicOr(bad, 1);
        for (int k = 0; k < 72; ++k) r[k] = 0.0;
    }
    store_clover_site(g.V, i, r, a64, a32, a16);
}

int launch_site_inverse(const Geom& g, const void* c64, double kappa, double csw, void* a64, void* a32, void* a16,
                        int* bad, hipStream_t st) {
    k_site_inverse<<<(g.V + 63) / 64, 64, 0, st>>>(g, c64, csw * kappa, a64, a32, a16, bad);
    WCL_HIP(hipGetLastError());
    return WCL_OK;
}
