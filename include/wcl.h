/*
 * wcl.h -- C ABI of the MI355X (gfx950) Wilson-clover RAS solver library.
 *
 * The library solves the quark linear system D phi = eta (Sec. 1, Eq. (1))
 * for the O(a)-improved Wilson (clover) operator with parameters kappa and
 * c_SW (Sec. 5), using BiCGStab right-preconditioned by the restricted
 * additive Schwarz iteration K_RAS (Sec. 2, Algorithm 1, Eqs. (2)-(3))
 * inside a mixed-precision nested BiCGStab (Sec. 3): FP64 outer solver,
 * FP32 inner solver, RAS domain solves in FP32 or FP16 storage.
 *
 * Operator (the paper names it but prints no formula; kappa-normalised
 * standard form, chiral gamma basis, periodic links):
 *   (D psi)(x) = [1 + c_SW kappa C(x)] psi(x)
 *                - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                               + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *   C(x) = i sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x), Fhat from the four
 *   plaquette leaves, (1/8)[(Q - Q^dag) - (1/3) Tr(Q - Q^dag)].
 *   gamma_k = [[0,-i sigma_k],[i sigma_k,0]] (k = x,y,z), gamma_t = [[0,-1],[-1,0]].
 *
 * Conventions
 *   - Every function returns an int status: WCL_OK (0) or a negative error
 *     code; wcl_last_error() returns a thread-local message for the last
 *     failure on the calling thread.  WCL_PENDING (> 0) is returned only by
 *     wcl_poll.
 *   - Host layouts are FP64 complex, array-of-structures, canonical site
 *     index x + Lx*(y + Ly*(z + Lz*t)); directions mu = 0,1,2,3 = x,y,z,t:
 *       gauge   double[V][4][3][3][2]   (site, mu, row, col, re/im)
 *       spinor  double[nrhs][V][4][3][2] (rhs, site, spin, colour, re/im)
 *   - Device spinor buffers are caller-owned (e.g. torch tensors), in the
 *     library's internal structure-of-arrays layout for their precision,
 *     which only wcl_pack_spinor* produce and wcl_unpack_spinor* read.
 *     Their size is wcl_spinor_bytes(); alignment must be 256 bytes (any
 *     hipMalloc / torch CUDA allocation satisfies it).
 *   - Streams are HIP streams (hipStream_t passed as void*; NULL = default
 *     stream).  Calls that take a stream are asynchronous on it unless
 *     stated otherwise.
 *   - Handles are not thread-safe, except wcl_submit / wcl_poll.
 *   - The library owns the resident gauge and clover fields and all solver
 *     workspace; it frees them in wcl_destroy_lattice / wcl_finalize.
 */
#ifndef WCL_H
#define WCL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define WCL_OK 0
#define WCL_EINVAL (-1)       /* invalid argument (shape, size, NaN/Inf input, ...) */
#define WCL_ENOMEM (-2)       /* HBM budget or device allocation exhausted */
#define WCL_EUNITARITY (-3)   /* gauge link not SU(3) to 1e-12 */
#define WCL_ENOTCONV (-4)     /* solver hit its iteration limit; best iterate returned */
#define WCL_EBREAKDOWN (-5)   /* BiCGStab breakdown persisted after restarts */
#define WCL_EHIP (-6)         /* HIP runtime error */
#define WCL_ESTATE (-7)       /* call out of order (e.g. no gauge uploaded) */
#define WCL_PENDING 1         /* wcl_poll: request not finished yet */

/* ---- precisions ---- */
#define WCL_F64 0
#define WCL_F32 1
#define WCL_F16 2   /* binary16 storage, per-site FP32 scale for spinors/clover; see wcl_apply_D and
                       WCL_ARITH_* for the arithmetic on it */

/* ---- RAS domain solver kernels ---- */
#define WCL_BLOCK_AUTO 0
#define WCL_BLOCK_FUSED 1   /* one workgroup per (domain, rhs), on chip (extended volume <= 256) */
#define WCL_BLOCK_SPLIT 2   /* several workgroups per domain, two launches per MR step (any shape) */
/* WCL_BLOCK_AUTO takes the fused kernel when the extended domain fits it. */

typedef struct wcl_ctx wcl_ctx;
typedef struct wcl_lattice wcl_lattice;
typedef struct wcl_server wcl_server;

/* ---- domain solvers (Sec. 2: "a fixed iteration solver with N_dominv
 * iterations"; every reading runs exactly n_dominv iterations from zero) ---- */
#define WCL_DOMSOLVE_MR 0        /* minimal residual: q = D rho, alpha = <q,rho>/<q,q> */
#define WCL_DOMSOLVE_JACOBI 1    /* block Jacobi: x <- x + A^-1 (b - D x), A = the site (clover) term */
#define WCL_DOMSOLVE_BICGSTAB 2  /* truncated BiCGStab (no restarts, no early exit) */

/* ---- Schwarz iterations (Sec. 1-2) ---- */
#define WCL_SCHWARZ_RAS 0   /* restricted additive Schwarz, Algorithm 1 */
#define WCL_SCHWARZ_AS 1    /* additive Schwarz: the whole extended solutions are summed (overlaps add up),
                               refined by the Richardson iteration phi += v, r -= D v */
#define WCL_SCHWARZ_SAP 2   /* multiplicative Schwarz (Schwarz alternating procedure): the domains are
                               coloured by the parity of their block coordinates; each sweep solves the
                               colour-0 domains, updates r, then the colour-1 domains, updates r */

/* ---- arithmetic of the on-chip MR domain steps (FP16 storage) ---- */
#define WCL_ARITH_FP32 0   /* FP32 FMAs on the stored fields (binary16 fields widened inside the FMAs) */
#define WCL_ARITH_DOT2 1   /* the link and clover products of each MR step take the domain residual
                              rounded to binary16 (after scaling the domain by a power of two to an RMS
                              component near 1) and sum in FP32 (two-term dot products), the spin
                              projections are binary16 additions of those values, and the
                              backward-hop terms pass between sites as binary16; accumulation, the MR
                              scalars and vector updates stay FP32.  FP16 storage,
                              MR domain solver, RAS, extended domains of at most 256 sites only
                              (WCL_EINVAL otherwise).  The preconditioner stays homogeneous:
                              K(2^k r) = 2^k K(r) exactly */

/* RAS parameters (Sec. 2): domains Omega_i are the tiling of the lattice by
 * `block` from the origin; Omega'_i grows each domain by s sites per side in
 * every direction it does not span (overlap depth d = 2s, Sec. 4).
 * n_ras sweeps of Algorithm 1, each domain solved approximately by n_dominv
 * iterations of the domain solver from zero (the paper's fixed-iteration
 * domain solver; minimal residual by default).  storage = WCL_F32 or WCL_F16
 * for the gauge/clover fields and the sweep-internal residual/correction
 * fields.  block_solver and schwarz select the variants above (0 = the
 * defaults: MR domain solves inside RAS); the Jacobi and BiCGStab domain
 * solvers and the AS and SAP iterations run on the split path.  AS needs
 * s <= block[mu] in every split direction (WCL_EINVAL otherwise); its
 * Richardson refinement (n_ras > 1) diverges when overlaps are counted twice,
 * so as a preconditioner it is normally used with n_ras = 1. */
typedef struct wcl_ras_params {
    int block[4];
    int s;
    int n_ras;
    int n_dominv;
    int storage;
    int kernel;        /* WCL_BLOCK_* */
    int block_solver;  /* WCL_DOMSOLVE_* */
    int schwarz;       /* WCL_SCHWARZ_* */
    int arith;         /* WCL_ARITH_* (0 = FP32) */
} wcl_ras_params;

#define WCL_PRECOND_NONE 0
#define WCL_PRECOND_RAS 1

/* Nested solver parameters (Sec. 3): the outer FP64 BiCGStab stops when its
 * recursive residual is below tol_outer*|eta|, then recomputes the true
 * residual |eta - D phi|/|eta| in FP64 and restarts from phi if it is above
 * tol_outer (at most max_restarts times).  Each outer preconditioner call
 * is an FP32 BiCGStab (right-preconditioned by K_RAS if precond = RAS) that
 * stops at relative residual tol_inner or max_inner iterations. */
typedef struct wcl_solver_params {
    double tol_outer;
    double tol_inner;
    int max_outer;
    int max_inner;
    int max_restarts;
    int precond;            /* WCL_PRECOND_* */
    wcl_ras_params ras;
    int even_odd;           /* 1: both solver levels work on the even-odd reduced system Dhat phi_e = b_e
                               (see wcl_apply_schur; precond must be NONE, every extent even), phi_o is
                               reconstructed, and the true residual reported is that of the full D */
    int timers;             /* 1: per-category HIP-event times into wcl_solve_stats (ms_dslash, ...) */
} wcl_solver_params;

/* Per-solve statistics.  The counters follow the paper's timing chart
 * (Sec. 4/5): dslash_full is its "Dv operation count", dslash_block and
 * ras_sweeps measure the domain inversion work; ms_total is the HIP-event
 * time of the whole solve on its stream.  With wcl_solver_params.timers = 1
 * the solve's stream time is split by HIP events into the chart's compute
 * categories: ms_dslash = full-lattice D applications of every precision
 * (T_Dv^calc; with even_odd, the reduced operator), ms_dominv = the domain
 * solver launches of the Schwarz sweeps, including the residual update
 * r -= D v that the on-chip path forms inside the next sweep (T_dominv^calc),
 * ms_blas = BLAS-1 updates, reductions and precision conversions of both
 * solver levels, ms_host = device idle while the host reads the scalars and
 * decides (one wait per iteration).  The four add up to ms_total. */
typedef struct wcl_solve_stats {
    int outer_iters;
    int inner_iters;        /* summed over all inner solves */
    int restarts;           /* true-residual restarts + breakdown restarts */
    int converged;
    int64_t dslash_full;    /* full-lattice D applications (all precisions) */
    int64_t dslash_block;   /* domain-solver iterations (each = one D_Omega' over all domains) */
    int64_t ras_sweeps;
    double true_resid;      /* |eta - D phi| / |eta| in FP64 at exit */
    double ms_total;
    double ms_dslash, ms_dominv, ms_blas, ms_host;   /* only with timers = 1, else 0 */
} wcl_solve_stats;

/* ---- context and lattice ---- */

/* Opens `device` (HIP ordinal) with an HBM budget for everything the library
 * allocates (0 = free memory at init).  *ctx receives the handle. */
int wcl_init(int device, uint64_t hbm_budget_bytes, wcl_ctx** ctx);
int wcl_finalize(wcl_ctx* ctx);
const char* wcl_last_error(void);
/* Bytes currently allocated by the library on the context's device. */
uint64_t wcl_bytes_in_use(wcl_ctx* ctx);

/* A lattice of dims = {Lx,Ly,Lz,Lt} (each >= 2) with fermion boundary phase
 * bc[mu] = +1 (periodic) or -1 (antiperiodic); bc == NULL means periodic. */
int wcl_create_lattice(wcl_ctx* ctx, const int dims[4], const int bc[4], wcl_lattice** lat);
int wcl_destroy_lattice(wcl_lattice* lat);
int64_t wcl_volume(const wcl_lattice* lat);

/* Uploads U (host gauge layout above), checks |U U^dag - 1| and |det U - 1|
 * <= 1e-12 for every link (WCL_EUNITARITY otherwise), stores it on the
 * device as two-row (12-real) links in FP64, FP32 and FP16.  Synchronous.
 * The clover field of the previous gauge, if any, is invalidated. */
int wcl_upload_gauge(wcl_lattice* lat, const double* U);
/* Builds C(x) = i sum sigma Fhat on the device from the resident links and
 * stores it (kappa-independent) as two packed 6x6 Hermitian blocks per site in
 * FP64, FP32 and FP16.  Synchronous. */
int wcl_compute_clover(wcl_lattice* lat);
/* Alternative to wcl_compute_clover: C given on the host as double[V][2][36],
 * block k (k=0: spins 0,1; k=1: spins 2,3), index 3*(spin mod 2)+colour;
 * 6 real diagonal entries, then the 15 complex strictly-upper entries
 * (re, im) in row-major order.  Synchronous. */
int wcl_upload_clover(wcl_lattice* lat, const double* C);
/* Reads the resident FP64 clover back in the same packed host layout. */
int wcl_download_clover(wcl_lattice* lat, double* C);

/* ---- spinor fields ---- */

/* Size in bytes of a device spinor buffer of nrhs fields at precision prec. */
uint64_t wcl_spinor_bytes(const wcl_lattice* lat, int prec, int nrhs);
/* host/device FP64 AoS -> device internal layout (and back).  The *_dev
 * variants take a device pointer to the AoS data. */
int wcl_pack_spinor(wcl_lattice* lat, int prec, int nrhs, const double* host_aos, void* dev_soa, void* stream);
int wcl_unpack_spinor(wcl_lattice* lat, int prec, int nrhs, const void* dev_soa, double* host_aos, void* stream);
int wcl_pack_spinor_dev(wcl_lattice* lat, int prec, int nrhs, const double* dev_aos, void* dev_soa, void* stream);
int wcl_unpack_spinor_dev(wcl_lattice* lat, int prec, int nrhs, const void* dev_soa, double* dev_aos, void* stream);

/* ---- operators ---- */

/* out = D in for nrhs fields (Eq. (1)), periodic lattice with the bc phases,
 * at storage precision prec for spinors, links and clover.  Arithmetic: FP64
 * for WCL_F64, FP32 for WCL_F32; for WCL_F16 the spin projections are
 * binary16 additions of the stored values, the link and clover products take
 * the stored binary16 values (and the projected half-spinors, rounded to
 * binary16) as two-term dot products with FP32 sums, and the per-site scales
 * and the accumulation are FP32 (relative error a few 1e-4).  in and out
 * must not alias. */
int wcl_apply_D(wcl_lattice* lat, int prec, double kappa, double csw, const void* in_dev, void* out_dev, int nrhs,
                void* stream);

/* Even-odd reduced operator (not in the paper; an accelerator of the same
 * solve): with H the hopping part of D and the sites split by parity
 * (x+y+z+t mod 2; every extent must be even, else WCL_EINVAL),
 *   out_e = Dhat in_e = A_ee in_e - H_eo A_oo^{-1} H_oe in_e,  out_o = 0,
 * A = 1 + c_SW kappa C the site term, inverted per site (two 6x6 Hermitian
 * blocks, built once per (kappa, c_SW); WCL_EINVAL if singular).  in and out
 * are full-lattice fields of nrhs right-hand sides in the internal layout at
 * prec = WCL_F64 or WCL_F32 (the odd sites of in are not read); they must
 * not alias.  May allocate workspace on first use. */
int wcl_apply_schur(wcl_lattice* lat, int prec, double kappa, double csw, const void* in_dev, void* out_dev, int nrhs,
                    void* stream);

/* Domain operator test surface (Sec. 2): for every domain i,
 * out_i = D_{Omega'_i} P_{Omega'_i} in, D_{Omega'} being the principal
 * submatrix of D on the site set Omega' (hops leaving it dropped).  in is an
 * FP32 field (1 rhs); out_host receives double[nblocks][ext_volume][4][3][2],
 * sites of each domain in lexicographic order of their local coordinates
 * l_mu = x_mu - o_mu + s_mu (mod L_mu), o = domain origin.  Synchronous. */
int wcl_apply_D_blocks(wcl_lattice* lat, const wcl_ras_params* ras, double kappa, double csw, const void* in_dev,
                       double* out_host, void* stream);
/* Number of domains and extended-domain volume for ras->block, ras->s. */
int wcl_block_info(const wcl_lattice* lat, const wcl_ras_params* ras, int64_t* nblocks, int64_t* ext_volume);

/* v = K r for nrhs FP32 fields: n_ras sweeps of the Schwarz iteration
 * ras->schwarz (RAS: Algorithm 1 / Eq. (2); AS and SAP: Sec. 1-2, see
 * WCL_SCHWARZ_*) with n_dominv iterations of the domain solver
 * ras->block_solver on every domain.  r and v are FP32 device buffers that
 * must not alias.  The block Jacobi solver builds the site-term inverse
 * (1 + c_SW kappa C)^{-1} once per (kappa, c_SW) and returns WCL_EINVAL if
 * it is singular at some site.  May allocate workspace on first use. */
int wcl_ras_precondition(wcl_lattice* lat, const wcl_ras_params* ras, double kappa, double csw, const void* r_dev,
                         void* v_dev, int nrhs, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * v = K_RAS r as wcl_ras_precondition, with the same kernels and bitwise the
 * same result, but its sweep buffers come from a fixed device array of
 * WCL_NOALLOC_SCRATCH_BYTES per GPU (looked up in wcl_init; held until the
 * process ends) and it calls no allocator.  Only the on-chip path: minimal-
 * residual domain solves inside RAS (block_solver = MR, schwarz = RAS,
 * kernel != SPLIT) with extended domains of at most 256 sites; anything else,
 * or needing more than the fixed size (n_ras + 1 storage-precision fields x
 * nrhs for n_ras >= 3: the kept corrections of all sweeps but the last and
 * two residuals), returns WCL_EINVAL.  Every call on one GPU shares that array,
 * which keeps the last call's contents (nothing in it needs to start at
 * zero): calls that overlap in time on one GPU (other streams or threads)
 * race and must be serialised by the caller.  Asynchronous on stream. */
#define WCL_NOALLOC_SCRATCH_BYTES (64u << 20)
int wcl_ras_precondition_noalloc(wcl_lattice* lat, const wcl_ras_params* ras, double kappa, double csw,
                                 const void* r_dev, void* v_dev, int nrhs, void* stream);

/* ---- solvers ---- */

/* Mixed-precision nested BiCGStab (Sec. 3) for nrhs FP64 fields:
 * eta_dev, phi_dev are FP64 device buffers (internal layout).  phi is
 * overwritten (zero initial guess).  Blocks until done; stats may be NULL
 * (with nrhs > 1 the stats are summed over the right-hand sides and
 * true_resid is the largest).  Returns WCL_ENOTCONV with the best iterate in
 * phi if tol_outer is not reached. */
int wcl_solve_nested_bicgstab(wcl_lattice* lat, const wcl_solver_params* p, double kappa, double csw,
                              const void* eta_dev, void* phi_dev, int nrhs, wcl_solve_stats* stats, void* stream);
/* Plain unpreconditioned FP64 BiCGStab (the baseline): stops when the
 * recursive residual is below tol*|eta| and reports the true residual. */
int wcl_solve_bicgstab_f64(wcl_lattice* lat, double tol, int max_iter, double kappa, double csw, const void* eta_dev,
                           void* phi_dev, wcl_solve_stats* stats, void* stream);

/* ---- autotuner ----
 * Picks the RAS parameters the paper leaves to tuning (Sec. 2: overlap
 * depth, N_dominv, NRAS; Sec. 5 scans them by hand) plus the domain shape,
 * storage precision, inner tolerance and the D-apply's lanes per site, by
 * timing complete nested solves of eta on this lattice: stage 1 scans
 * domain shape {4^4, 4^3x8, 8^4} x overlap {0, 1} x storage and arithmetic
 * (bit 0 of storage_mask: FP32; bit 1: FP16; bit 2: FP16 with
 * WCL_ARITH_DOT2 where the fused solver runs; 0 = all); stage 2 scans N_dominv
 * 2..8 x NRAS 1..8; stage 3 the inner tolerance {1e-2, ..., 1e-6} and lanes
 * per site {1, 2}; stage 4 N_dominv and NRAS one step around the best at the
 * chosen tolerance.  Candidates that do not converge within 10 outer
 * iterations are skipped; the others are ranked by the sum over the nsrc
 * tuning sources of their solve times, each credited for ending below the
 * tolerance by the share of an iteration that geometric convergence would
 * have saved (f = log(tol_outer) / log(achieved true residual), credit
 * min(n (1 - f), 1/2) of n inner iterations): the step of one iteration more
 * or less depends on the source.  eta_dev holds nsrc tuning sources of nrhs
 * right-hand sides each, one after the other (1 <= nsrc <= 16); the chosen
 * parameters serve any source on this lattice.
 * With cache_path != NULL the result is read from / appended to that
 * JSON-lines file, keyed by device architecture, dims, nrhs, kappa, c_sw and
 * storage_mask.  *best receives the chosen parameters (tol_outer, max_* and
 * max_restarts are copied from *base; MR domain solves inside RAS, full D),
 * *best_ms its ranking time; the lattice keeps the chosen lanes per
 * site.  Blocks until done. */
int wcl_autotune(wcl_lattice* lat, const wcl_solver_params* base, double kappa, double csw, const void* eta_dev,
                 int nrhs, int nsrc, int storage_mask, const char* cache_path, wcl_solver_params* best,
                 double* best_ms, void* stream);

/* ---- serving (continuous batching of solve requests) ----
 * A server owns resident gauge/clover fields per registered configuration and
 * max_slots worker slots, each with its own HIP stream and solver workspace.
 * Requests wait in FIFO order and are admitted as soon as a slot is free and
 * the HBM they need fits the budget; admitted requests run concurrently on
 * the device.  With max_batch > 1 the request at the head of the queue takes
 * along up to max_batch - 1 queued requests that have the same configuration,
 * kappa, c_sw and solver parameters: they are solved together as the
 * right-hand sides of one nested solve (Sec. 3, every kernel batched over the
 * rhs), so they share every launch.  Each result is identical (bitwise) to
 * the same solve run alone, batched or not: a solve's arithmetic does not
 * depend on the other requests.  wcl_submit and wcl_poll are thread-safe. */
typedef struct wcl_server_params {
    uint64_t hbm_budget_bytes;  /* total for fields + workspaces; 0 = the context budget */
    int max_slots;              /* concurrent solves (>= 1) */
    int max_queue;              /* waiting requests before WCL_ENOMEM (0 = 4096) */
    int max_batch;              /* requests merged into one solve (0 or 1 = none, at most 64) */
} wcl_server_params;

typedef struct wcl_request {
    uint64_t config_id;         /* registered gauge configuration */
    double kappa, csw;
    const wcl_solver_params* params;  /* NULL = defaults (tol 1e-10, RAS 4^4 domains, FP16 storage) */
    const double* eta_host;     /* host spinor layout, 1 rhs; must stay valid until done */
    double* phi_host;           /* receives the solution; must stay valid until done */
} wcl_request;

typedef struct wcl_result {
    int status;                 /* WCL_OK or the solver's error code */
    wcl_solve_stats stats;      /* of the solve; for a batch: its counters and times, and this request's own
                                   true residual and convergence */
    double t_submit, t_admit, t_done;   /* seconds, steady clock */
    int batch;                  /* requests solved together with this one, itself included (1 = alone) */
} wcl_result;

int wcl_server_create(wcl_ctx* ctx, const wcl_server_params* p, wcl_server** srv);
/* Waits for every admitted and queued request, then frees everything. */
int wcl_server_destroy(wcl_server* srv);
/* Uploads U (host gauge layout) for config_id and builds its clover field;
 * they stay resident until the server is destroyed.  Synchronous. */
int wcl_register_gauge(wcl_server* srv, uint64_t config_id, const int dims[4], const double* U_host);
/* Queues a request; *ticket identifies it.  WCL_EINVAL for an unknown
 * config or bad parameters; WCL_ENOMEM if the request can never fit the
 * budget or the queue is full (other requests are unaffected). */
int wcl_submit(wcl_server* srv, const wcl_request* req, uint64_t* ticket);
/* WCL_PENDING while queued or running; otherwise fills *res, returns WCL_OK
 * and forgets the ticket. */
int wcl_poll(wcl_server* srv, uint64_t ticket, wcl_result* res);
/* Blocks until the ticket is done, then behaves like wcl_poll. */
int wcl_wait(wcl_server* srv, uint64_t ticket, wcl_result* res);

#ifdef __cplusplus
}
#endif
#endif /* WCL_H */
