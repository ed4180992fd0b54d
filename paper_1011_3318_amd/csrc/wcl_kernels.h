// Kernel launch interfaces shared between the HIP sources.
#pragma once

#include "wcl_internal.h"

enum { DS_PLAIN = 0, DS_AXPY = 1, DS_DOT = 2 };

// BiCGStab scalars of one right-hand side, resident on the device.
struct Scal {
    double rho[2], rho_old[2], alpha[2], omega[2], rv[2];
    double tt, rr, rr0, pp;
    int active, breakdown;
};

struct DslashArgs {
    Geom g;
    const void* gauge;
    const void* clover;
    const void* in;
    void* out;
    const void* y;       // DS_AXPY source
    const void* a;       // DS_DOT left vector
    size_t in_stride, out_stride, y_stride, a_stride;  // bytes per rhs
    double kappa, csw;
    int nrhs;
    int lps;             // lanes per site: 1, 2 or 4
    double* partial;     // DS_DOT: [nrhs][tiles][3]
    const Scal* sc;      // optional: right-hand sides with sc[rhs].active == 0 are skipped
};

int launch_pack_spinor(const Geom& g, int prec, int nrhs, const double* aos, void* soa, size_t stride,
                       hipStream_t st);
int launch_unpack_spinor(const Geom& g, int prec, int nrhs, const void* soa, size_t stride, double* aos,
                         hipStream_t st);
int launch_pack_gauge(const Geom& g, const double* aos, void* g64, void* g32, void* g16, hipStream_t st);
int launch_clover_build(const Geom& g, const void* g64, void* c64, void* c32, void* c16, hipStream_t st);
int launch_pack_clover(const Geom& g, const double* host_dev, void* c64, void* c32, void* c16, hipStream_t st);
int launch_unpack_clover(const Geom& g, const void* c64, double* host_dev, hipStream_t st);

int dslash_partials_per_rhs(int V, int lps);
int launch_dslash(const DslashArgs& a, int gp, int spi, int spo, int epi, int spy, hipStream_t st);

// --------------------------------------------------------- even-odd ----
// Steps of the even-odd reduction (wcl_evenodd.hip); "half" fields hold the
// V/2 sites of one parity, the site of parity p in pair (2h, 2h+1) at index h.
enum { EO_INV = 0, EO_SCHUR = 1, EO_PREP = 2, EO_RECON = 3, EO_SITEINV = 4, EO_EXTRACT = 5, EO_INSERT = 6,
       EO_ZERO = 7 };
struct EoArgs {
    Geom g;
    int Vh;              // V / 2
    int parity;          // parity of the sites the launch computes
    const void* gauge;   // full-lattice fields, precision of the launch
    const void* clover;
    const void* ainv;    // site-term inverse, clover layout
    const void* in;      // half field of the other parity (hop source)
    const void* in2;     // half field of `parity` (EO_SCHUR site-term operand, EO_INSERT source)
    const void* y;       // full field (EO_PREP/RECON/SITEINV/EXTRACT) or half field (EO_SCHUR axpy)
    const void* a;       // half field: left vector of the DS_DOT partials
    void* out;           // half field, or full field for EO_RECON/INSERT/ZERO
    size_t in_stride, in2_stride, y_stride, a_stride, out_stride;   // bytes per rhs
    double kappa, csw;
    int nrhs;
    double* partial;     // DS_DOT: [nrhs][tiles][3]
    const Scal* sc;      // optional: right-hand sides with sc[rhs].active == 0 are skipped
};
int eo_partials_per_rhs(int Vh);
int launch_eo(const EoArgs& a, int prec, int mode, int epi, hipStream_t st);

// ------------------------------------------------------------- solvers --
enum { FIN_RHO = 2, FIN_PP = 3, FIN_RR = 4, FIN_RR0 = 5 };

int blas_partials(int prec, int64_t V);
int blas_p_update(int prec, int64_t V, int nrhs, const Scal* sc, const void* r, void* p, const void* v,
                  hipStream_t st);
// s = r - alpha v, alpha formed from the partials pv of <rhat, v> (Gv per rhs)
int blas_s_update_fin(int prec, int64_t V, int nrhs, Scal* sc, const double* pv, int Gv, const void* r,
                      const void* v, void* s, hipStream_t st);
// x += alpha p^ + omega s^, r = s - omega t, partials of <rhat, r>, |r|^2 into
// `partial` (which must not alias pw); omega formed from the partials pw of
// <s, t>, |t|^2 (Gw per rhs)
int blas_xr_update_fin(int prec, int64_t V, int nrhs, Scal* sc, const double* pw, int Gw, void* x, const void* ph,
                       const void* sh, const void* s, const void* t, void* r, const void* rh, double* partial,
                       hipStream_t st);
int blas_dot(int prec, int64_t V, int nrhs, const Scal* sc, const void* a, const void* b, double* partial,
             hipStream_t st);
// x = p = v = 0, r = rhat = b, partials of <b, b> for the active rhs
int blas_init(int prec, int64_t V, int nrhs, const Scal* sc, const void* b, void* x, void* r, void* rh, void* p,
              void* v, double* partial, hipStream_t st);
int blas_to_f32_scaled(int64_t V, int nrhs, const Scal* sc, const void* a64, void* y32, hipStream_t st);
int blas_to_f64_scaled(int64_t V, int nrhs, const Scal* sc, const void* a32, void* y64, hipStream_t st);
// mirror (optional): device-visible pinned host array that also receives the
// updated scalars of the active rhs
int blas_finalize(const double* partial, int G, int nrhs, Scal* sc, int kind, hipStream_t st,
                  Scal* mirror = nullptr);

// ------------------------------------------------------ domain solves ---
struct BlockArgs {
    Geom g;
    Blocks B;
    const void* gauge;   // storage precision of the domain solver
    const void* clover;
    const void* src;     // projection source
    size_t src_stride;
    void* rho;           // workspace float4 [rhs][6][NE]
    void* q;
    void* x;
    size_t ws_stride;    // float4 elements per rhs
    int NE;              // nblocks * ev
    int wpb;             // workgroups per domain (split path)
    void* out;           // K_RAS output (FP32), owned sites
    size_t out_stride;
    void* vj;            // optional copy of this sweep's correction (storage precision)
    size_t vj_stride;
    int accumulate;      // out += x instead of out = x
    // fused residual update (on-chip path, sweeps after the first), with
    // vprev = v_{j-1}:
    //   res_boundary == 0: src = r_{j-1}; the kernel forms r_j = src - D vprev
    //     and writes r_j to rout at the owned sites;
    //   res_boundary == 1 (no overlap): src = the previous sweep's final MR
    //     residual rho_N = r_{j-1} - D_Omega v_{j-1}; the kernel adds only the
    //     hops that leave the domain, and writes its own final rho_N to rout.
    const void* vprev;   // storage precision
    size_t vprev_stride;
    void* rout;          // storage precision
    size_t rout_stride;
    int res_boundary;
    double kappa, csw;
    int nrhs;
    double* partial;     // [rhs][nblocks][wpb][3]
    const Scal* sc;      // optional: right-hand sides with sc[rhs].active == 0 are skipped
    // split-path variants (the other readings of Sec. 1-2):
    const void* dhat;    // k_blk_dslash: when set, the dot products are <dhat, q> and |q|^2
                         // instead of <q, rho> and |q|^2 (truncated BiCGStab's <rhat, v>)
    int colour;          // -1: every domain; 0 or 1: only the domains of that colour
                         // (multiplicative Schwarz); the others write zeros at their owned sites
    int whole;           // 1: the last step keeps the whole extended solution in x and the additive
                         // gather sums it (overlaps add up); 0: restriction to the owned sites
    const void* ainv;    // block Jacobi: site-term inverse A^{-1}, clover layout, storage precision
    void* bp;            // truncated BiCGStab workspaces (float4 [rhs][6][NE]): p, s, t, rhat
    void* bs;
    void* bt;
    void* brh;
    double* bpart[3];    // truncated BiCGStab partial sums: <rhat, r>, <rhat, v>, (<t, s>, |t|^2)
    double* dsc;         // truncated BiCGStab per-(rhs, domain) scalars [rhs][nblocks][8]:
                         // rho, alpha, omega, rho_old (complex)
    int dot2;            // on-chip MR steps with binary16 operands and FP32 sums (FP16 storage only)
    // on-chip path, output of the sweeps: skip_out = 1 writes no output (the
    // sweep's correction goes to vj only); vsum_n > 0 writes
    // out = vsum[0] + ... + vsum[vsum_n - 1] + x, vsum[j] at vsum + j * vsum_step
    // (storage precision, per-rhs stride vj_stride)
    int skip_out;
    const void* vsum;
    int vsum_n;
    size_t vsum_step;
};

int launch_blk_project(const BlockArgs& a, int src_prec, int bicgstab, hipStream_t st);
int launch_blk_dslash(const BlockArgs& a, int gp, hipStream_t st);
int launch_blk_update(const BlockArgs& a, int vj_prec, int last, hipStream_t st);
// block Jacobi step: x = x + A^{-1} (b - q) (first: x = A^{-1} b), b = rho
int launch_blk_jacobi(const BlockArgs& a, int gp, int vj_prec, int first, int last, hipStream_t st);
// truncated BiCGStab: p update, s update, x/r update (see wcl_block.hip)
int launch_bcg_p(const BlockArgs& a, int it, hipStream_t st);
int launch_bcg_s(const BlockArgs& a, hipStream_t st);
int launch_bcg_xr(const BlockArgs& a, int vj_prec, int last, hipStream_t st);
// additive Schwarz: v(x) = sum of the extended solutions of every domain whose
// Omega' holds x, out (+)= v, vj = v
int launch_blk_gather(const BlockArgs& a, int vj_prec, hipStream_t st);
// A^{-1} = (1 + csw kappa C)^{-1} per site, stored like the clover field in
// FP64, FP32 and FP16; *bad (device int) is set when some A(x) is singular
int launch_site_inverse(const Geom& g, const void* c64, double kappa, double csw, void* a64, void* a32, void* a16,
                        int* bad, hipStream_t st);
int launch_blk_unpack(const BlockArgs& a, const float* ws, double* out, hipStream_t st);
// ------------------------------------------------------------- solvers --
struct Workspace;
Workspace* wcl_workspace_new(wcl_ctx* ctx);
void wcl_workspace_delete(Workspace* w);
size_t workspace_bytes(const Workspace* w);
void workspace_get(Workspace* w, const char* name, size_t bytes, void** out, int* rc);
// Nested RAS-BiCGStab on an explicit workspace and stream (Sec. 3).
// resid_rhs (optional, nrhs values): |eta_i - D phi_i| / |eta_i| per rhs
// (0 for a zero rhs, -1 where the solve ended on a hard error).
int nested_solve(wcl_lattice* lat, Workspace* ws, const wcl_solver_params* prm, double kappa, double csw,
                 const void* eta, void* phi, int nrhs, wcl_solve_stats* stats, hipStream_t st,
                 double* resid_rhs = nullptr);
// Device bytes a nested solve needs on a fresh workspace (estimate, upper bound).
size_t nested_workspace_bytes(const wcl_lattice* lat, const wcl_solver_params* prm, int nrhs);
int fused_threads(int ev);   // workgroup size of the fused domain solver, 0 if it does not fit
int launch_blk_fused(const BlockArgs& a, int gp, int src_prec, hipStream_t st);
int blas_restart(int prec, int64_t V, int nrhs, const Scal* sc, const void* src, void* r, void* rh, void* p, void* v,
                 hipStream_t st);
