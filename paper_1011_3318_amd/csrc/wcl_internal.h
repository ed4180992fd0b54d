// Internal definitions shared by the HIP sources of the library: error
// handling, the device site layout, storage formats and small complex
// helpers.  Not part of the public ABI (include/wcl.h).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>

#include "wcl.h"

// ------------------------------------------------------------ errors ----
void wcl_set_error(const char* fmt, ...);

#define WCL_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            wcl_set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                          __LINE__);                                                       \
            return WCL_EHIP;                                                               \
        }                                                                                  \
    } while (0)

#define WCL_CHECK(expr)          \
    do {                         \
        int rc_ = (expr);        \
        if (rc_ != WCL_OK) return rc_; \
    } while (0)

// ---------------------------------------------------------- geometry ----
// Device site order.  The lattice is cut into columns of cross-section
// cx*cy*cz (powers of two dividing Lx, Ly, Lz) that run the full t extent.
// A site's internal index is
//     col * Vc + t * S + (lx + cx*(ly + cy*lz)),   S = cx*cy*cz, Vc = S*Lt,
// with col = Cx + nCx*(Cy + nCy*Cz) the column of (x,y,z).  A wavefront
// streams along x inside one t-slice of one column and consecutive
// workgroups walk a column in t, so neighbouring slices are read close
// together in time (by workgroups of the same XCD, see xcd_remap).
struct Geom {
    int L[4];
    int c[3];
    int lc[3];
    int nC[3];
    int S;
    int Vc;
    int V;
    int bc[4];
};

__host__ __device__ inline void geom_coords(const Geom& g, int i, int x[4]) {
    int col = i / g.Vc;
    int r = i - col * g.Vc;
    int t = r / g.S;
    int l = r - t * g.S;
    int lx = l & (g.c[0] - 1);
    int ly = (l >> g.lc[0]) & (g.c[1] - 1);
    int lz = l >> (g.lc[0] + g.lc[1]);
    int Cx = col % g.nC[0];
    int q = col / g.nC[0];
    int Cy = q % g.nC[1];
    int Cz = q / g.nC[1];
    x[0] = (Cx << g.lc[0]) + lx;
    x[1] = (Cy << g.lc[1]) + ly;
    x[2] = (Cz << g.lc[2]) + lz;
    x[3] = t;
}

__host__ __device__ inline int geom_index(const Geom& g, const int x[4]) {
    int col = (x[0] >> g.lc[0]) + g.nC[0] * ((x[1] >> g.lc[1]) + g.nC[1] * (x[2] >> g.lc[2]));
    int l = (x[0] & (g.c[0] - 1)) + g.c[0] * ((x[1] & (g.c[1] - 1)) + g.c[1] * (x[2] & (g.c[2] - 1)));
    return col * g.Vc + x[3] * g.S + l;
}

__host__ __device__ inline int canonical_index(const Geom& g, const int x[4]) {
    return x[0] + g.L[0] * (x[1] + g.L[1] * (x[2] + g.L[2] * x[3]));
}

__host__ __device__ inline void canonical_coords(const Geom& g, int j, int x[4]) {
    x[0] = j % g.L[0];
    j /= g.L[0];
    x[1] = j % g.L[1];
    j /= g.L[1];
    x[2] = j % g.L[2];
    x[3] = j / g.L[2];
}

// ------------------------------------------------------ domain layout ---
// Domains Omega_i tile the lattice by b from the origin; Omega'_i adds s_mu
// sites per side (s_mu = 0 where b_mu = L_mu).  Extended domains are stored
// one after the other, sites in lexicographic order of the local coordinate
// l_mu in [0, e_mu), e_mu = b_mu + 2 s_mu; global x_mu = o_mu - s_mu + l_mu.
struct Blocks {
    int b[4];
    int s[4];
    int e[4];
    int nb[4];
    int nblocks;
    int ev;  // extended volume
    int n_ras, n_dominv;
    int solver;    // WCL_DOMSOLVE_*
    int schwarz;   // WCL_SCHWARZ_*
    int arith;     // WCL_ARITH_*
};

// ------------------------------------------------------ storage -------
// Tiled structure of arrays: a field with NC vector elements per site is
// stored in tiles of 64 sites (one wavefront), element-major inside a tile:
//     element (k, site i)  at  ((i / 64) * NC + k) * 64 + i % 64.
// A wavefront's load of one element is 64 consecutive vectors, and all the
// elements of a tile are contiguous, so a kernel streams a few long runs
// instead of one run per element array (measured: 7.0 vs 5.4 TB/s for the
// D-apply's byte pattern).  The last tile is padded; padding is never read
// as data.
//
// Spinor (per right-hand side; rhs stride = wcl_spinor_bytes(.., 1)):
//   F64: NC=12 double2, element k = component 3*spin + colour
//   F32: NC=6  float4,  element g = components 2g, 2g+1 (re,im,re,im)
//   F16: NC=3  half8 (reals 8g..8g+7 divided by the site scale) + a plain
//        float[Vp] scale array after the tiles
// Gauge (rows 0,1 of each link; row 2 = conj(row0 x row1) rebuilt on load):
//   F64: NC=24 double2 (element 6 mu + k)   F32: NC=12 float4 (3 mu + g)
//   F16: NC=12 half4 (3 mu + g)
// Clover C (kappa-independent), 72 reals per site = blocks k=0,1 of 36:
//   6 real diagonal entries then 15 complex upper entries, row-major:
//   F64: NC=36 double2   F32: NC=18 float4   F16: NC=9 half8 + float[Vp] scale
__host__ __device__ inline size_t tix(int k, int i, int NC) {
    return ((size_t)(i >> 6) * NC + k) * 64 + (i & 63);
}
inline size_t round_up(size_t n, size_t a) { return (n + a - 1) / a * a; }
inline size_t padded_sites(int64_t V) { return round_up((size_t)V, 64); }

inline size_t spinor_rhs_bytes(int prec, int64_t V) {
    const size_t Vp = padded_sites(V);
    switch (prec) {
        case WCL_F64: return 192 * Vp;
        case WCL_F32: return 96 * Vp;
        default: return 48 * Vp + round_up(4 * Vp, 256);
    }
}
inline size_t gauge_bytes(int prec, int64_t V) {
    return padded_sites(V) * 4 * 12 * (prec == WCL_F64 ? 8 : prec == WCL_F32 ? 4 : 2);
}
inline size_t clover_bytes(int prec, int64_t V) {
    const size_t Vp = padded_sites(V);
    return prec == WCL_F64 ? Vp * 72 * 8 : prec == WCL_F32 ? Vp * 72 * 4 : Vp * 144 + round_up(Vp * 4, 256);
}
// byte offset of the FP16 scale array inside an FP16 spinor (per rhs) / clover
__host__ __device__ inline size_t half_spinor_scale_offset(int V) { return (size_t)48 * ((V + 63) / 64 * 64); }
__host__ __device__ inline size_t half_clover_scale_offset(int V) { return (size_t)144 * ((V + 63) / 64 * 64); }

// ------------------------------------------------------ structures -----
struct wcl_ctx {
    int device;
    uint64_t budget;
    uint64_t in_use;
    int arch_major;
    int num_cu;
    std::mutex mu;   // guards in_use (serving slots allocate concurrently)
    void* scratch = nullptr;   // this device's fixed scratch block (see static_scratch_setup)
};

struct Workspace;  // solver scratch, defined in wcl_solver.hip

struct wcl_lattice {
    wcl_ctx* ctx;
    Geom g;
    int64_t V;
    bool has_gauge = false, has_clover = false;
    void* gauge[3] = {nullptr, nullptr, nullptr};   // indexed by WCL_F64/F32/F16
    void* clover[3] = {nullptr, nullptr, nullptr};
    Workspace* ws = nullptr;
    int lps = 1;   // lanes per site of the full-lattice D-apply (tunable)
    uint64_t uid = 0;         // unique per lattice of the process (never reused)
    uint64_t clover_gen = 0;  // incremented whenever the clover field changes
};

// device memory accounting against the context budget
int wcl_dev_alloc(wcl_ctx* ctx, void** p, size_t bytes);
void wcl_dev_free(wcl_ctx* ctx, void* p, size_t bytes);

int check_prec(int prec);
void wcl_free_workspace(wcl_lattice* lat);  // solver workspace, wcl_solver.hip
int make_blocks(const wcl_lattice* lat, const wcl_ras_params* p, Blocks* B);
// Device address of the fixed scratch block on `device` (current), looked up
// once per device (wcl_solver.hip).
int static_scratch_setup(int device, void** ptr);
