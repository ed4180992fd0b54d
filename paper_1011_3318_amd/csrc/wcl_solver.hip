// Solvers on the device:
//   * K_RAS (Algorithm 1 / Eq. (2)): n_ras sweeps of projection, domain
//     solves, restriction/sum, phi += v and r -= D v (the last residual
//     update is skipped: it cannot change phi);
//   * BiCGStab, right-preconditioned (Eq. (3)), batched over right-hand
//     sides, in FP32 (inner) or FP64 (outer / plain baseline);
//   * the nested solver of Sec. 3: the FP64 outer BiCGStab's preconditioner
//     is an FP32 inner BiCGStab preconditioned by K_RAS.  The outer loop
//     confirms the true residual |eta - D phi| / |eta| in FP64 and restarts
//     from phi when it is above tolerance.
// The host only sequences launches and reads the per-rhs scalars once per
// iteration for the convergence decision.
#include <cmath>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "wcl_kernels.h"

// ------------------------------------------------------------ timeline --
// Per-category device time of one solve (the paper's timing chart, Sec. 4):
// an event is recorded on the solve's stream whenever the category of the
// enqueued work changes; after the solve the interval from each mark to the
// next is added to the category of the mark.  Off unless requested.
enum { CAT_DSLASH = 0, CAT_DOMINV = 1, CAT_BLAS = 2, CAT_HOST = 3, CAT_N = 4 };
struct Timeline {
    bool on = false;
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> pool;
    std::vector<int> cats;
    int cur = -1;
    void start(hipStream_t s) {
        on = true;
        st = s;
        cats.clear();
        cur = -1;
    }
    void mark(int cat) {
        if (!on || cat == cur) return;
        const size_t k = cats.size();
        if (k == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                on = false;
                return;
            }
            pool.push_back(e);
        }
        if (hipEventRecord(pool[k], st) != hipSuccess) {
            on = false;
            return;
        }
        cats.push_back(cat);
        cur = cat;
    }
    // end: an event recorded after the last work of the solve, completed
    void finish(hipEvent_t end, double ms[CAT_N]) {
        for (int c = 0; c < CAT_N; ++c) ms[c] = 0.0;
        if (!on) return;
        for (size_t k = 0; k < cats.size(); ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, pool[k], k + 1 < cats.size() ? pool[k + 1] : end) == hipSuccess)
                ms[cats[k]] += t;
        }
        on = false;
    }
    ~Timeline() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// ----------------------------------------------------------- workspace --
struct Workspace {
    wcl_ctx* ctx = nullptr;
    Timeline tl;
    // key of the site-term inverse held in "ainv.*" (see site_inverse)
    uint64_t ainv_uid = 0, ainv_gen = 0;
    double ainv_kappa = 0.0, ainv_csw = 0.0;
    const void* ainv_ptr = nullptr;
    struct Item {
        std::string name;
        void* p;
        size_t bytes;
    };
    std::vector<Item> items;
    struct Pinned {
        std::string name;
        Scal* p;
        size_t n;
    };
    std::vector<Pinned> pinned;   // host mirrors of the scalar arrays, one per solver level

    int get(const std::string& name, size_t bytes, void** out) {
        for (auto& it : items)
            if (it.name == name) {
                if (it.bytes >= bytes) {
                    *out = it.p;
                    return WCL_OK;
                }
                wcl_dev_free(ctx, it.p, it.bytes);
                it.p = nullptr;
                it.bytes = 0;
                WCL_CHECK(wcl_dev_alloc(ctx, &it.p, bytes));
                it.bytes = bytes;
                *out = it.p;
                return WCL_OK;
            }
        Item it{name, nullptr, 0};
        WCL_CHECK(wcl_dev_alloc(ctx, &it.p, bytes));
        it.bytes = bytes;
        items.push_back(it);
        *out = it.p;
        return WCL_OK;
    }
    int host_scal(const std::string& name, size_t n, Scal** out) {
        for (auto& pp : pinned)
            if (pp.name == name) {
                if (pp.n < n) {
                    (void)hipHostFree(pp.p);
                    pp.p = nullptr;
                    WCL_HIP(hipHostMalloc((void**)&pp.p, n * sizeof(Scal), hipHostMallocDefault));
                    pp.n = n;
                }
                *out = pp.p;
                return WCL_OK;
            }
        Pinned pp{name, nullptr, n};
        WCL_HIP(hipHostMalloc((void**)&pp.p, n * sizeof(Scal), hipHostMallocDefault));
        pinned.push_back(pp);
        *out = pp.p;
        return WCL_OK;
    }
    void release() {
        for (auto& it : items) wcl_dev_free(ctx, it.p, it.bytes);
        items.clear();
        for (auto& pp : pinned) (void)hipHostFree(pp.p);
        pinned.clear();
    }
    ~Workspace() { release(); }
};

Workspace* wcl_workspace_new(wcl_ctx* ctx) {
    auto* w = new Workspace;
    w->ctx = ctx;
    return w;
}
void wcl_workspace_delete(Workspace* w) { delete w; }

size_t workspace_bytes(const Workspace* w) {
    size_t b = 0;
    for (const auto& it : w->items) b += it.bytes;
    return b;
}

void workspace_get(Workspace* w, const char* name, size_t bytes, void** out, int* rc) {
    *rc = w->get(name, bytes, out);
}

size_t nested_workspace_bytes(const wcl_lattice* lat, const wcl_solver_params* prm, int nrhs) {
    const size_t v64 = spinor_rhs_bytes(WCL_F64, lat->V) * nrhs, v32 = spinor_rhs_bytes(WCL_F32, lat->V) * nrhs;
    size_t b = 8 * v64 + 10 * v32;   // outer and inner BiCGStab vectors, inner rhs/solution
    const size_t ainv = clover_bytes(WCL_F64, lat->V) + clover_bytes(WCL_F32, lat->V) + clover_bytes(WCL_F16, lat->V);
    if (prm && prm->precond == WCL_PRECOND_RAS) {
        Blocks B;
        if (make_blocks(lat, &prm->ras, &B) == WCL_OK) {
            // kept corrections v_j (NRAS - 1 on chip), residuals r_j (ping-pong)
            b += (size_t)(std::max(B.n_ras - 1, 2) + 2) * spinor_rhs_bytes(prm->ras.storage, lat->V) * nrhs;
            const bool split = fused_threads(B.ev) != 256 || B.solver != WCL_DOMSOLVE_MR ||
                               B.schwarz != WCL_SCHWARZ_RAS;
            const int nws = B.solver == WCL_DOMSOLVE_BICGSTAB ? 7 : 3;
            if (split) b += (size_t)nws * 96 * B.nblocks * B.ev * nrhs;   // split workspaces
            if (B.solver == WCL_DOMSOLVE_JACOBI) b += ainv;
        }
    }
    if (prm && prm->even_odd) b += ainv + 5 * v64;   // site-term inverse, half fields, full residual
    const size_t partials = (size_t)24 * nrhs * ((lat->V + 63) / 64);
    return b + 6 * partials + (1 << 20);
}

void wcl_free_workspace(wcl_lattice* lat) {
    delete lat->ws;
    lat->ws = nullptr;
}

static Workspace* lattice_ws(wcl_lattice* lat) {
    if (!lat->ws) lat->ws = wcl_workspace_new(lat->ctx);
    return lat->ws;
}

// ---------------------------------------------------------- validation --
int make_blocks(const wcl_lattice* lat, const wcl_ras_params* p, Blocks* B) {
    if (!p) {
        wcl_set_error("RAS parameters missing");
        return WCL_EINVAL;
    }
    if (p->s < 0 || p->n_ras < 1 || p->n_dominv < 1 || (p->storage != WCL_F32 && p->storage != WCL_F16) ||
        p->kernel < 0 || p->kernel > 2 || p->block_solver < 0 || p->block_solver > 2 || p->schwarz < 0 ||
        p->schwarz > 2) {
        wcl_set_error("RAS parameters invalid (s=%d n_ras=%d n_dominv=%d storage=%d kernel=%d)", p->s, p->n_ras,
                      p->n_dominv, p->storage, p->kernel);
        return WCL_EINVAL;
    }
    B->nblocks = 1;
    B->ev = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int L = lat->g.L[mu], b = p->block[mu];
        if (b < 1 || L % b != 0) {
            wcl_set_error("block[%d] = %d does not divide L = %d", mu, b, L);
            return WCL_EINVAL;
        }
        B->b[mu] = b;
        B->s[mu] = b < L ? p->s : 0;
        B->e[mu] = b + 2 * B->s[mu];
        if (B->e[mu] > L) {
            wcl_set_error("extended block %d + 2*%d exceeds L = %d in direction %d", b, p->s, L, mu);
            return WCL_EINVAL;
        }
        B->nb[mu] = L / b;
        B->nblocks *= B->nb[mu];
        B->ev *= B->e[mu];
    }
    if ((int64_t)B->nblocks * B->ev * 6 > INT32_MAX) {
        wcl_set_error("extended domains too large");
        return WCL_EINVAL;
    }
    B->n_ras = p->n_ras;
    B->n_dominv = p->n_dominv;
    B->solver = p->block_solver;
    B->schwarz = p->schwarz;
    B->arith = p->arith;
    if (p->arith != WCL_ARITH_FP32 && p->arith != WCL_ARITH_DOT2) {
        wcl_set_error("RAS arithmetic %d unknown", p->arith);
        return WCL_EINVAL;
    }
    if (p->arith == WCL_ARITH_DOT2 &&
        (p->storage != WCL_F16 || p->block_solver != WCL_DOMSOLVE_MR || p->schwarz != WCL_SCHWARZ_RAS)) {
        wcl_set_error("binary16-operand MR steps need FP16 storage, the MR domain solver and RAS");
        return WCL_EINVAL;
    }
    // the additive sum gathers each site from its own domain and the two
    // neighbouring ones in every direction, which covers every extended
    // domain holding it when s <= b
    for (int mu = 0; mu < 4; ++mu)
        if (B->schwarz == WCL_SCHWARZ_AS && B->s[mu] > B->b[mu]) {
            wcl_set_error("additive Schwarz needs the overlap s = %d <= the domain extent %d in direction %d",
                          B->s[mu], B->b[mu], mu);
            return WCL_EINVAL;
        }
    return WCL_OK;
}

static int need_fields(const wcl_lattice* lat) {
    if (!lat->has_clover) {
        wcl_set_error("gauge and clover fields must be resident");
        return WCL_ESTATE;
    }
    return WCL_OK;
}

// ------------------------------------------------------------------ RAS --
// The fused (on-chip) domain solver takes extended domains of up to 256
// sites with the default readings (minimal-residual domain solves inside
// the restricted additive iteration); every other case uses the split path.
static int pick_kernel(const Blocks& B, int requested, bool* fused) {
    const bool fits = fused_threads(B.ev) == 256;
    const bool variant = B.solver != WCL_DOMSOLVE_MR || B.schwarz != WCL_SCHWARZ_RAS;
    if (requested == WCL_BLOCK_FUSED && !fits) {
        wcl_set_error("fused domain solver needs an extended domain of at most 256 sites (got %d)", B.ev);
        return WCL_EINVAL;
    }
    if (requested == WCL_BLOCK_FUSED && variant) {
        wcl_set_error("the fused domain solver runs minimal-residual domain solves inside RAS only; "
                      "the other domain solvers and Schwarz iterations use the split path");
        return WCL_EINVAL;
    }
    *fused = requested != WCL_BLOCK_SPLIT && fits && !variant;
    if (B.arith == WCL_ARITH_DOT2 && !*fused) {
        wcl_set_error("binary16-operand MR steps run in the fused domain solver only (extended domains of at most "
                      "256 sites, kernel not forced to the split path)");
        return WCL_EINVAL;
    }
    return WCL_OK;
}

// Device buffers of one Schwarz application.
struct RasBufs {
    void* vj[2] = {nullptr, nullptr};     // corrections v_j (storage precision)
    void* rbuf[2] = {nullptr, nullptr};   // residuals r_j between passes (storage precision)
    void* rho = nullptr;                  // split path: extended-domain workspaces
    void* q = nullptr;
    void* x = nullptr;
    double* partial = nullptr;
    void* bp = nullptr;                   // truncated BiCGStab
    void* bs = nullptr;
    void* bt = nullptr;
    void* brh = nullptr;
    double* bpart[3] = {nullptr, nullptr, nullptr};
    double* dsc = nullptr;
};

struct BufReq {
    const char* name;
    size_t bytes;
    void** slot;
};

static int schwarz_passes(const Blocks& B) { return B.n_ras * (B.schwarz == WCL_SCHWARZ_SAP ? 2 : 1); }

// The buffers an application needs, by name.  The same list serves the
// workspace (named, grown on demand) and the fixed scratch block of the
// no-allocation entry point.
static void ras_buffer_list(const Blocks& B, bool fused, int storage, int64_t V, int nrhs, RasBufs& b,
                            std::vector<BufReq>& out) {
    const size_t sst = spinor_rhs_bytes(storage, V) * nrhs;
    out.clear();
    if (fused) {
        // every sweep but the last keeps its correction v_j (one slot each:
        // the last sweep sums them into the output); the residuals ping-pong
        if (B.n_ras > 1) {
            out.push_back({"ras.vj", sst * (B.n_ras - 1), &b.vj[0]});
            out.push_back({"ras.r0", sst, &b.rbuf[0]});
        }
        if (B.n_ras > 2) out.push_back({"ras.r1", sst, &b.rbuf[1]});
        return;
    }
    const int T = schwarz_passes(B);
    const size_t NE = (size_t)B.nblocks * B.ev, wsb = (size_t)16 * 6 * NE * nrhs;
    const int wpb = (B.ev + 255) / 256;
    const size_t pb = (size_t)24 * nrhs * B.nblocks * wpb;
    out.push_back({"ras.rho", wsb, &b.rho});
    out.push_back({"ras.q", wsb, &b.q});
    out.push_back({"ras.x", wsb, &b.x});
    out.push_back({"ras.partial", pb, (void**)&b.partial});
    if (T > 1) {
        out.push_back({"ras.vj", sst, &b.vj[0]});
        out.push_back({"ras.r0", sst, &b.rbuf[0]});
    }
    if (T > 2) out.push_back({"ras.r1", sst, &b.rbuf[1]});
    if (B.solver == WCL_DOMSOLVE_BICGSTAB) {
        out.push_back({"ras.bp", wsb, &b.bp});
        out.push_back({"ras.bs", wsb, &b.bs});
        out.push_back({"ras.bt", wsb, &b.bt});
        out.push_back({"ras.brh", wsb, &b.brh});
        out.push_back({"ras.bpart0", pb, (void**)&b.bpart[0]});
        out.push_back({"ras.bpart1", pb, (void**)&b.bpart[1]});
        out.push_back({"ras.bpart2", pb, (void**)&b.bpart[2]});
        out.push_back({"ras.dsc", (size_t)64 * nrhs * B.nblocks, (void**)&b.dsc});
    }
}

// A^{-1} = (1 + csw kappa C)^{-1} per site in FP64/FP32/FP16, built on the
// device for (lattice, clover field, kappa, csw) and kept in the workspace
// until one of them changes.
static int site_inverse(wcl_lattice* lat, Workspace* ws, double kappa, double csw, hipStream_t st, void* out[3]) {
    const int64_t V = lat->V;
    WCL_CHECK(ws->get("ainv.f64", clover_bytes(WCL_F64, V), &out[0]));
    WCL_CHECK(ws->get("ainv.f32", clover_bytes(WCL_F32, V), &out[1]));
    WCL_CHECK(ws->get("ainv.f16", clover_bytes(WCL_F16, V), &out[2]));
    if (ws->ainv_uid == lat->uid && ws->ainv_gen == lat->clover_gen && ws->ainv_kappa == kappa &&
        ws->ainv_csw == csw && ws->ainv_ptr == out[0])
        return WCL_OK;
    ws->ainv_uid = 0;
    int* bad = nullptr;
    WCL_CHECK(ws->get("ainv.bad", 256, (void**)&bad));
    int hbad = 0;
    WCL_HIP(hipMemcpyAsync(bad, &hbad, sizeof(int), hipMemcpyHostToDevice, st));
    WCL_CHECK(launch_site_inverse(lat->g, lat->clover[WCL_F64], kappa, csw, out[0], out[1], out[2], bad, st));
    WCL_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    WCL_HIP(hipStreamSynchronize(st));
    if (hbad) {
        wcl_set_error("the site term 1 + c_sw kappa C(x) is singular at some site (kappa %g, c_sw %g)", kappa, csw);
        return WCL_EINVAL;
    }
    ws->ainv_uid = lat->uid;
    ws->ainv_gen = lat->clover_gen;
    ws->ainv_kappa = kappa;
    ws->ainv_csw = csw;
    ws->ainv_ptr = out[0];
    return WCL_OK;
}

static void tl_mark(Timeline* tl, int cat) {
    if (tl) tl->mark(cat);
}

// One domain solve on the split path for the current pass: projection of
// the source, the domain solver's iterations, and the write-out (restriction
// to the owned sites, or the additive gather).
static int split_domain_solve(const BlockArgs& a0, const Blocks& B, int storage, int src_prec, const RasBufs& bf,
                              hipStream_t st) {
    BlockArgs a = a0;
    const int n = B.n_dominv;
    if (B.solver == WCL_DOMSOLVE_MR) {
        WCL_CHECK(launch_blk_project(a, src_prec, 0, st));
        for (int k = 0; k < n; ++k) {
            WCL_CHECK(launch_blk_dslash(a, storage, st));
            WCL_CHECK(launch_blk_update(a, storage, k == n - 1, st));
        }
    } else if (B.solver == WCL_DOMSOLVE_JACOBI) {
        WCL_CHECK(launch_blk_project(a, src_prec, 0, st));
        BlockArgs ax = a;   // q = D_{Omega'} x
        ax.rho = bf.x;
        for (int k = 0; k < n; ++k) {
            if (k > 0) WCL_CHECK(launch_blk_dslash(ax, storage, st));
            WCL_CHECK(launch_blk_jacobi(a, storage, storage, k == 0, k == n - 1, st));
        }
    } else {
        WCL_CHECK(launch_blk_project(a, src_prec, 1, st));
        BlockArgs av = a, at = a;
        av.rho = bf.bp;   // v = D p, partials <rhat, v>
        av.q = bf.q;
        av.dhat = bf.brh;
        av.partial = bf.bpart[1];
        at.rho = bf.bs;   // t = D s, partials <t, s>, |t|^2
        at.q = bf.bt;
        at.partial = bf.bpart[2];
        for (int k = 0; k < n; ++k) {
            WCL_CHECK(launch_bcg_p(a, k, st));
            WCL_CHECK(launch_blk_dslash(av, storage, st));
            WCL_CHECK(launch_bcg_s(a, st));
            WCL_CHECK(launch_blk_dslash(at, storage, st));
            WCL_CHECK(launch_bcg_xr(a, storage, k == n - 1, st));
        }
    }
    if (B.schwarz == WCL_SCHWARZ_AS) WCL_CHECK(launch_blk_gather(a, storage, st));
    return WCL_OK;
}

// v = K r for nrhs FP32 fields: n_ras sweeps of the Schwarz iteration
// (Algorithm 1 for RAS; Sec. 1-2 for the additive and multiplicative ones).
// sc (optional): device scalars of the calling solver; inactive rhs are skipped.
static int ras_run(wcl_lattice* lat, const Blocks& B, bool fused, int storage, double kappa, double csw,
                   const void* r, void* v, int nrhs, hipStream_t st, wcl_solve_stats* stats, const Scal* sc,
                   const RasBufs& bf, const void* ainv, Timeline* tl) {
    const int64_t V = lat->V;
    const size_t s32 = spinor_rhs_bytes(WCL_F32, V), sst = spinor_rhs_bytes(storage, V);
    const int no_overlap = B.s[0] == 0 && B.s[1] == 0 && B.s[2] == 0 && B.s[3] == 0;
    const int NE = fused ? 0 : B.nblocks * B.ev, wpb = (B.ev + 255) / 256;
    BlockArgs a{};
    a.g = lat->g;
    a.B = B;
    a.dot2 = B.arith == WCL_ARITH_DOT2;
    a.gauge = lat->gauge[storage];
    a.clover = lat->clover[storage];
    a.NE = NE;
    a.wpb = wpb;
    a.ws_stride = (size_t)6 * NE;
    a.kappa = kappa;
    a.csw = csw;
    a.nrhs = nrhs;
    a.out = v;
    a.out_stride = s32;
    a.sc = sc;
    a.colour = -1;
    a.rho = bf.rho;
    a.q = bf.q;
    a.x = bf.x;
    a.partial = bf.partial;
    a.ainv = ainv;
    a.bp = bf.bp;
    a.bs = bf.bs;
    a.bt = bf.bt;
    a.brh = bf.brh;
    for (int k = 0; k < 3; ++k) a.bpart[k] = bf.bpart[k];
    a.dsc = bf.dsc;
    a.vj_stride = sst;
    if (fused) {
        // Between sweeps r_{j+1} = r_j - D v_j: the next sweep's kernel forms
        // it from v_j.  phi = sum_j v_j (Algorithm 1) is written once, by the
        // last sweep, from the kept corrections of the earlier ones (storage
        // precision) and its own: the output is not read and written again
        // by every sweep.
        const size_t slot = sst * nrhs;
        for (int j = 0; j < B.n_ras; ++j) {
            const bool last = j == B.n_ras - 1;
            tl_mark(tl, CAT_DOMINV);
            a.accumulate = 0;
            a.skip_out = !last;
            a.vsum = bf.vj[0];
            a.vsum_n = last ? j : 0;
            a.vsum_step = slot;
            a.vprev = j == 0 ? nullptr : (const char*)bf.vj[0] + (j - 1) * slot;
            a.vprev_stride = sst;
            a.rout_stride = sst;
            a.vj = last ? nullptr : (char*)bf.vj[0] + j * slot;
            a.res_boundary = no_overlap;
            int src_prec;
            if (no_overlap) {
                // sweep j > 0 starts from sweep j-1's final MR residual and
                // adds the hops of D v_{j-1} that cross domain boundaries
                a.src = j == 0 ? r : bf.rbuf[(j - 1) % 2];
                a.src_stride = j == 0 ? s32 : sst;
                src_prec = j == 0 ? WCL_F32 : storage;
                a.rout = last ? nullptr : bf.rbuf[j % 2];
            } else {
                // sweep j reads r_{j-1} (r itself for j = 1), forms r_j
                a.src = j <= 1 ? r : bf.rbuf[(j - 1) % 2];
                a.src_stride = j <= 1 ? s32 : sst;
                src_prec = j <= 1 ? WCL_F32 : storage;
                a.rout = (j == 0 || last) ? nullptr : bf.rbuf[j % 2];
            }
            WCL_CHECK(launch_blk_fused(a, storage, src_prec, st));
            if (j > 0 && stats) stats->dslash_full += nrhs;
        }
        if (stats) {
            stats->ras_sweeps += B.n_ras;
            stats->dslash_block += (int64_t)B.n_ras * B.n_dominv;
        }
        return WCL_OK;
    }
    // split path: every pass solves its domains on the current residual; a
    // full-lattice D-apply with the axpy epilogue forms the next one
    const int T = schwarz_passes(B), per = B.schwarz == WCL_SCHWARZ_SAP ? 2 : 1;
    const void* src = r;
    size_t src_stride = s32;
    int src_prec = WCL_F32;
    for (int pass = 0; pass < T; ++pass) {
        const bool lastp = pass == T - 1;
        tl_mark(tl, CAT_DOMINV);
        a.colour = B.schwarz == WCL_SCHWARZ_SAP ? pass % per : -1;
        a.whole = B.schwarz == WCL_SCHWARZ_AS;
        a.accumulate = pass > 0;
        a.vj = lastp ? nullptr : bf.vj[0];
        a.src = src;
        a.src_stride = src_stride;
        WCL_CHECK(split_domain_solve(a, B, storage, src_prec, bf, st));
        if (lastp) break;
        // r_{pass+1} = r_pass - D v_pass
        DslashArgs d{};
        d.g = lat->g;
        d.gauge = lat->gauge[storage];
        d.clover = lat->clover[storage];
        d.in = bf.vj[0];
        d.in_stride = sst;
        d.y = src;
        d.y_stride = src_stride;
        d.out = bf.rbuf[pass % 2];
        d.out_stride = sst;
        d.kappa = kappa;
        d.csw = csw;
        d.nrhs = nrhs;
        d.lps = lat->lps;
        d.sc = sc;
        tl_mark(tl, CAT_DSLASH);
        WCL_CHECK(launch_dslash(d, storage, storage, storage, DS_AXPY, src_prec, st));
        if (stats) stats->dslash_full += nrhs;
        src = bf.rbuf[pass % 2];
        src_stride = sst;
        src_prec = storage;
    }
    if (stats) {
        const int per_pass = B.solver == WCL_DOMSOLVE_MR ? B.n_dominv
                             : B.solver == WCL_DOMSOLVE_JACOBI ? B.n_dominv - 1 : 2 * B.n_dominv;
        stats->ras_sweeps += B.n_ras;
        stats->dslash_block += (int64_t)T * per_pass;
    }
    return WCL_OK;
}

// sc (optional): device scalars of the calling solver; inactive rhs are skipped.
static int ras_apply(wcl_lattice* lat, Workspace* ws, const Blocks& B, int storage, int kernel, double kappa,
                     double csw, const void* r, void* v, int nrhs, hipStream_t st, wcl_solve_stats* stats,
                     const Scal* sc = nullptr) {
    bool fused = false;
    WCL_CHECK(pick_kernel(B, kernel, &fused));
    RasBufs bf;
    std::vector<BufReq> req;
    ras_buffer_list(B, fused, storage, lat->V, nrhs, bf, req);
    for (auto& q : req) WCL_CHECK(ws->get(q.name, q.bytes, q.slot));
    void* ainv = nullptr;
    if (!fused && B.solver == WCL_DOMSOLVE_JACOBI) {
        void* inv[3];
        WCL_CHECK(site_inverse(lat, ws, kappa, csw, st, inv));
        ainv = inv[storage];
    }
    return ras_run(lat, B, fused, storage, kappa, csw, r, v, nrhs, st, stats, sc, bf, ainv, &ws->tl);
}

// ------------------------------------------------- fixed scratch block --
// For callers that cannot allocate (graph capture, tight serving loops):
// the on-chip path's sweep buffers come from this fixed device array
// instead of the workspace.  Each device holds its own copy at its own
// address, looked up once per device when a context opens on it.
static __device__ __align__(256) unsigned char scratch[WCL_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

int static_scratch_setup(int device, void** ptr) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= 64) {
        wcl_set_error("device %d out of range for the fixed scratch block", device);
        return WCL_EINVAL;
    }
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        WCL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return WCL_OK;
}

// ------------------------------------------------------------- BiCGStab --
// Preconditioner: out = K in for the active rhs; sc = the calling engine's
// device scalars, act = its host-side active flags.
using Precond = std::function<int(const void* in, void* out, Scal* sc, const std::vector<int>& act)>;

struct EngineResult {
    int iters = 0;
    int restarts = 0;
    bool converged = false;
    bool breakdown = false;    // some rhs was dropped for a persistent breakdown
    double true_resid = 0.0;   // max over rhs (only with true_check)
    std::vector<double> tres;  // per rhs (only with true_check; 0 for a zero rhs)
};

struct Engine {
    wcl_lattice* lat;
    Workspace* ws;
    std::string tag;
    int P;    // vector precision (F64 or F32)
    int gp;   // link/clover precision of D
    int nrhs;
    double kappa, csw;
    hipStream_t st;
    wcl_solve_stats* stats;
    int64_t V;
    size_t vb;
    int Gb, Gd;
    void *r, *rh, *p, *v, *s, *t, *ph, *sh;
    double* partial;
    double* partial2;   // the x/r update's partials (it reads the D-apply's)
    Scal* d;      // device scalars [nrhs]
    Scal* h;      // pinned host mirror
    Scal* hmap;   // h as the device addresses it (written by the finalize kernels)
    hipEvent_t ev = nullptr;   // recorded after each iteration's last finalize
    // even-odd: the operator is the Schur complement Dhat on the even half
    // fields (vectors of V/2 sites); eo_ainv = site-term inverse at precision P
    int eo = 0;
    const void* eo_ainv = nullptr;
    void* eo_t = nullptr;   // half-field temporary A_oo^{-1} H_oe x
    // |r| / |b| of each rhs at the start of the current iteration (what the
    // preconditioner's accuracy is measured against; 1 before the first)
    std::vector<double> rel_now;

    ~Engine() {
        if (ev) (void)hipEventDestroy(ev);
    }

    int init(const Precond* K) {
        V = eo ? lat->V / 2 : lat->V;
        vb = spinor_rhs_bytes(P, V) * nrhs;
        Gb = blas_partials(P, V);
        Gd = eo ? eo_partials_per_rhs((int)V) : dslash_partials_per_rhs((int)V, lat->lps);
        auto name = [&](const char* n) { return tag + "." + n; };
        if (eo) WCL_CHECK(ws->get(name("eot"), vb, &eo_t));
        WCL_CHECK(ws->get(name("r"), vb, &r));
        WCL_CHECK(ws->get(name("rh"), vb, &rh));
        WCL_CHECK(ws->get(name("p"), vb, &p));
        WCL_CHECK(ws->get(name("v"), vb, &v));
        WCL_CHECK(ws->get(name("s"), vb, &s));
        WCL_CHECK(ws->get(name("t"), vb, &t));
        if (K) {
            WCL_CHECK(ws->get(name("ph"), vb, &ph));
            WCL_CHECK(ws->get(name("sh"), vb, &sh));
        } else {
            ph = p;
            sh = s;
        }
        WCL_CHECK(ws->get(name("partial"), (size_t)24 * nrhs * std::max(Gb, Gd), (void**)&partial));
        WCL_CHECK(ws->get(name("partial2"), (size_t)24 * nrhs * Gb, (void**)&partial2));
        WCL_CHECK(ws->get(name("scal"), sizeof(Scal) * nrhs, (void**)&d));
        if (!ev) WCL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        return WCL_OK;
    }
    // Dhat x in two launches: eo_t = A_oo^{-1} H_oe x (odd sites), then
    // out = A_ee x - H_eo eo_t (even sites) with the epilogue epi
    int apply_schur(const void* in, void* out, const void* a, const void* y, int epi) {
        EoArgs e{};
        e.g = lat->g;
        e.Vh = (int)V;
        e.gauge = lat->gauge[gp];
        e.clover = lat->clover[gp];
        e.ainv = eo_ainv;
        e.in_stride = e.in2_stride = e.y_stride = e.a_stride = e.out_stride = spinor_rhs_bytes(P, V);
        e.kappa = kappa;
        e.csw = csw;
        e.nrhs = nrhs;
        e.sc = d;
        e.parity = 1;
        e.in = in;
        e.out = eo_t;
        if (stats) stats->dslash_full += nrhs;
        ws->tl.mark(CAT_DSLASH);
        WCL_CHECK(launch_eo(e, P, EO_INV, DS_PLAIN, st));
        e.parity = 0;
        e.in = eo_t;
        e.in2 = in;
        e.out = out;
        e.a = a;
        e.y = y;
        e.partial = partial;
        return launch_eo(e, P, EO_SCHUR, epi, st);
    }
    int apply_dot(const void* in, void* out, const void* a) {
        if (eo) return apply_schur(in, out, a, nullptr, DS_DOT);
        DslashArgs x{};
        x.g = lat->g;
        x.gauge = lat->gauge[gp];
        x.clover = lat->clover[gp];
        x.in = in;
        x.out = out;
        x.a = a;
        x.in_stride = x.out_stride = x.a_stride = spinor_rhs_bytes(P, V);
        x.kappa = kappa;
        x.csw = csw;
        x.nrhs = nrhs;
        x.lps = lat->lps;
        x.partial = partial;
        x.sc = d;
        if (stats) stats->dslash_full += nrhs;
        ws->tl.mark(CAT_DSLASH);
        return launch_dslash(x, gp, P, P, DS_DOT, P, st);
    }
    // out = b - D x (FP64 true residual)
    int residual(const void* b, const void* x, void* out) {
        if (eo) return apply_schur(x, out, nullptr, b, DS_AXPY);
        DslashArgs a{};
        a.g = lat->g;
        a.gauge = lat->gauge[gp];
        a.clover = lat->clover[gp];
        a.in = x;
        a.y = b;
        a.out = out;
        a.in_stride = a.out_stride = a.y_stride = spinor_rhs_bytes(P, V);
        a.kappa = kappa;
        a.csw = csw;
        a.nrhs = nrhs;
        a.lps = lat->lps;
        if (stats) stats->dslash_full += nrhs;
        ws->tl.mark(CAT_DSLASH);
        return launch_dslash(a, gp, P, P, DS_AXPY, P, st);
    }
    // The finalize kernel before every pull has written the active rhs'
    // scalars into h already; inactive rhs do not change on the device.
    int pull() {
        ws->tl.mark(CAT_HOST);
        WCL_HIP(hipStreamSynchronize(st));
        return WCL_OK;
    }
    int push() {
        ws->tl.mark(CAT_HOST);
        WCL_HIP(hipMemcpyAsync(d, h, sizeof(Scal) * nrhs, hipMemcpyHostToDevice, st));
        WCL_HIP(hipStreamSynchronize(st));
        return WCL_OK;
    }

    // Solves A x = b (A = D at precision gp) for the rhs with act[i] = 1, to
    // |r| <= tol |b| (or tol_rhs[i] |b| per rhs when given).
    // On return act[i] = 1 marks the rhs that converged.
    int run(const void* b, void* x, double tol, int max_iter, const Precond* K, std::vector<int>& act, bool true_check,
            int max_restarts, EngineResult* res, const std::vector<double>* tol_rhs = nullptr) {
        auto tol_of = [&](int i) { return tol_rhs ? (*tol_rhs)[i] : tol; };
        rel_now.assign(nrhs, 1.0);
        WCL_CHECK(init(K));
        WCL_CHECK(ws->host_scal(tag, nrhs, &h));
        WCL_HIP(hipHostGetDevicePointer((void**)&hmap, h, 0));
        for (int i = 0; i < nrhs; ++i) {
            Scal z{};
            z.rho[0] = z.rho_old[0] = z.alpha[0] = z.omega[0] = 1.0;
            z.active = act[i];
            h[i] = z;
        }
        WCL_CHECK(push());
        ws->tl.mark(CAT_BLAS);
        WCL_CHECK(blas_init(P, V, nrhs, d, b, x, r, rh, p, v, partial, st));
        WCL_CHECK(blas_finalize(partial, Gb, nrhs, d, FIN_RHO, st, hmap));
        WCL_CHECK(pull());
        std::vector<double> bnorm(nrhs, 0.0), rh2(nrhs, 0.0);
        // rhs dropped for a persistent breakdown (reported as WCL_EBREAKDOWN)
        std::vector<int> broke(nrhs, 0);
        std::vector<int> conv(nrhs, 0), restarts(nrhs, 0);
        // |b - D x| / |b| of the rhs whose convergence a true residual
        // confirmed (x does not change afterwards); -1 = not known
        std::vector<double> tres(nrhs, -1.0);
        for (int i = 0; i < nrhs; ++i) {
            if (!act[i]) continue;
            if (!std::isfinite(h[i].rr)) {
                wcl_set_error("right-hand side %d is not finite", i);
                return WCL_EINVAL;
            }
            bnorm[i] = std::sqrt(h[i].rr);
            rh2[i] = h[i].rr;
            h[i].rho_old[0] = 1.0;
            h[i].rho_old[1] = 0.0;
            if (bnorm[i] == 0.0) {  // b = 0: x = 0 is exact
                h[i].active = 0;
                conv[i] = 1;
            }
        }
        WCL_CHECK(push());
        int it = 0, total_restarts = 0;
        auto any_active = [&]() {
            for (int i = 0; i < nrhs; ++i)
                if (h[i].active) return true;
            return false;
        };
        // The next iteration's p update is enqueued before the host check of
        // this one and the host waits on an event recorded before it, so the
        // GPU computes p while the host decides.  That is safe: convergence
        // leaves p unused, and a restart sets p = r itself (what the update
        // gives after a restart), overwriting the speculative p.
        bool p_ready = false;
        while (any_active() && it < max_iter) {
            ++it;
            for (int i = 0; i < nrhs; ++i)
                rel_now[i] = (h[i].active && bnorm[i] > 0) ? std::sqrt(h[i].rr) / bnorm[i] : 0.0;
            ws->tl.mark(CAT_BLAS);
            if (!p_ready) WCL_CHECK(blas_p_update(P, V, nrhs, d, r, p, v, st));
            p_ready = false;
            std::vector<int> a_now(nrhs);
            for (int i = 0; i < nrhs; ++i) a_now[i] = h[i].active;
            if (K) WCL_CHECK((*K)(p, ph, d, a_now));
            WCL_CHECK(apply_dot(ph, v, rh));
            // alpha and omega are formed inside the updates that use them
            ws->tl.mark(CAT_BLAS);
            WCL_CHECK(blas_s_update_fin(P, V, nrhs, d, partial, Gd, r, v, s, st));
            if (K) WCL_CHECK((*K)(s, sh, d, a_now));
            WCL_CHECK(apply_dot(sh, t, s));
            ws->tl.mark(CAT_BLAS);
            WCL_CHECK(blas_xr_update_fin(P, V, nrhs, d, partial, Gd, x, ph, sh, s, t, r, rh, partial2, st));
            WCL_CHECK(blas_finalize(partial2, Gb, nrhs, d, FIN_RHO, st, hmap));
            WCL_HIP(hipEventRecord(ev, st));
            if (it < max_iter) {
                WCL_CHECK(blas_p_update(P, V, nrhs, d, r, p, v, st));
                p_ready = true;
            }
            ws->tl.mark(CAT_HOST);
            WCL_HIP(hipEventSynchronize(ev));
            bool changed = false, want_true = false, dropped = false;
            std::vector<int> restart(nrhs, 0);
            for (int i = 0; i < nrhs; ++i) {
                if (!h[i].active) continue;
                const double rr = h[i].rr;
                if (!std::isfinite(rr)) {
                    h[i].active = 0;
                    changed = dropped = true;
                    continue;
                }
                const double rel = std::sqrt(rr) / bnorm[i];
                if (rel <= tol_of(i)) {
                    if (true_check) {
                        want_true = true;
                        restart[i] = 3;   // candidate
                    } else {
                        h[i].active = 0;
                        conv[i] = 1;
                        changed = true;
                    }
                } else {
                    const double arho = std::hypot(h[i].rho[0], h[i].rho[1]);
                    const bool bd = h[i].breakdown || arho < 1e-30 * std::sqrt(rh2[i] * rr) ||
                                    (h[i].omega[0] == 0.0 && h[i].omega[1] == 0.0);
                    if (bd) restart[i] = 1;
                }
            }
            // A dropped rhs must be inactive on the device before any later
            // finalize copies the device scalars back into the host mirror.
            if (dropped) {
                WCL_CHECK(push());
                changed = false;
            }
            const void* restart_src = nullptr;
            if (want_true) {
                // true residual in the engine's precision: t = b - D x
                WCL_CHECK(residual(b, x, t));
                ws->tl.mark(CAT_BLAS);
                WCL_CHECK(blas_dot(P, V, nrhs, d, t, t, partial, st));
                WCL_CHECK(blas_finalize(partial, Gb, nrhs, d, FIN_RR, st, hmap));
                WCL_CHECK(pull());
                for (int i = 0; i < nrhs; ++i) {
                    if (restart[i] != 3) continue;
                    const double trel = std::sqrt(h[i].rr) / bnorm[i];
                    if (trel <= tol_of(i)) {
                        h[i].active = 0;
                        conv[i] = 1;
                        tres[i] = trel;
                        restart[i] = 0;
                        changed = true;
                    } else if (restarts[i] < max_restarts) {
                        restart[i] = 2;   // defect correction from the true residual
                        restart_src = t;
                    } else {
                        h[i].active = 0;
                        restart[i] = 0;
                        changed = true;
                    }
                }
            }
            bool any_restart = false;
            for (int i = 0; i < nrhs; ++i)
                if (restart[i] == 1 || restart[i] == 2) {
                    if (restart[i] == 1 && restarts[i] >= max_restarts + 50) {
                        h[i].active = 0;   // persistent breakdown
                        broke[i] = 1;
                        changed = true;
                        continue;
                    }
                    any_restart = true;
                    ++restarts[i];
                    ++total_restarts;
                }
            if (any_restart) {
                // rhs restarting from the recursive residual keep r; those
                // restarting from the true residual take r = t.  Two passes
                // when both kinds occur.
                for (int pass = 0; pass < 2; ++pass) {
                    const int kind = pass == 0 ? 1 : 2;
                    bool any = false;
                    for (int i = 0; i < nrhs; ++i) {
                        h[i].breakdown = (restart[i] == kind && h[i].active) ? 2 : 0;
                        any = any || h[i].breakdown == 2;
                    }
                    if (!any) continue;
                    WCL_CHECK(push());
                    ws->tl.mark(CAT_BLAS);
                    WCL_CHECK(blas_restart(P, V, nrhs, d, kind == 2 ? restart_src : nullptr, r, rh, p, v, st));
                }
                for (int i = 0; i < nrhs; ++i) h[i].breakdown = 0;
                WCL_CHECK(push());
                ws->tl.mark(CAT_BLAS);
                WCL_CHECK(blas_dot(P, V, nrhs, d, rh, r, partial, st));
                WCL_CHECK(blas_finalize(partial, Gb, nrhs, d, FIN_RHO, st, hmap));
                WCL_CHECK(pull());
                for (int i = 0; i < nrhs; ++i) {
                    if (restart[i] != 1 && restart[i] != 2) continue;
                    h[i].rho_old[0] = h[i].alpha[0] = h[i].omega[0] = 1.0;
                    h[i].rho_old[1] = h[i].alpha[1] = h[i].omega[1] = 0.0;
                    rh2[i] = h[i].rr;
                }
                changed = true;
            }
            if (changed) WCL_CHECK(push());
        }
        res->iters = it;
        res->restarts = total_restarts;
        res->converged = true;
        res->breakdown = false;
        for (int i = 0; i < nrhs; ++i) {
            if (act[i] && !conv[i]) res->converged = false;
            if (broke[i]) res->breakdown = true;
            act[i] = conv[i];
        }
        if (true_check) {
            // report |b - D x| / |b| for every rhs: computed again only for
            // the rhs that no true-residual check confirmed
            bool any = false;
            for (int i = 0; i < nrhs; ++i) {
                h[i].active = (bnorm[i] > 0 && tres[i] < 0) ? 1 : 0;
                any = any || h[i].active;
            }
            if (any) {
                WCL_CHECK(push());
                WCL_CHECK(residual(b, x, t));
                ws->tl.mark(CAT_BLAS);
                WCL_CHECK(blas_dot(P, V, nrhs, d, t, t, partial, st));
                WCL_CHECK(blas_finalize(partial, Gb, nrhs, d, FIN_RR, st, hmap));
                WCL_CHECK(pull());
                for (int i = 0; i < nrhs; ++i)
                    if (h[i].active) tres[i] = std::sqrt(h[i].rr) / bnorm[i];
            }
            res->true_resid = 0.0;
            res->tres.assign(nrhs, 0.0);
            for (int i = 0; i < nrhs; ++i)
                if (bnorm[i] > 0) {
                    res->true_resid = std::max(res->true_resid, tres[i]);
                    res->tres[i] = tres[i];
                }
        }
        return WCL_OK;
    }
};

static int check_solver_params(const wcl_solver_params* p) {
    if (!p || !(p->tol_outer > 0) || !(p->tol_inner > 0) || p->max_outer < 1 || p->max_inner < 1 ||
        p->max_restarts < 0 || (p->precond != WCL_PRECOND_NONE && p->precond != WCL_PRECOND_RAS) ||
        (p->even_odd != 0 && p->even_odd != 1) || (p->timers != 0 && p->timers != 1)) {
        wcl_set_error("invalid solver parameters");
        return WCL_EINVAL;
    }
    if (p->even_odd && p->precond != WCL_PRECOND_NONE) {
        wcl_set_error("the even-odd reduced system is solved without the Schwarz preconditioner (precond = NONE)");
        return WCL_EINVAL;
    }
    return WCL_OK;
}

// |v_i|^2 of nrhs fields read back to the host (synchronous).
static int host_norms2(Workspace* ws, int prec, int64_t V, int nrhs, const void* v, hipStream_t st,
                       std::vector<double>& out) {
    const int G = blas_partials(prec, V);
    Scal *d = nullptr, *h = nullptr, *hm = nullptr;
    double* part = nullptr;
    WCL_CHECK(ws->get("norm.scal", sizeof(Scal) * nrhs, (void**)&d));
    WCL_CHECK(ws->get("norm.partial", (size_t)24 * nrhs * G, (void**)&part));
    WCL_CHECK(ws->host_scal("norm", nrhs, &h));
    WCL_HIP(hipHostGetDevicePointer((void**)&hm, h, 0));
    for (int i = 0; i < nrhs; ++i) {
        h[i] = Scal{};
        h[i].active = 1;
    }
    WCL_HIP(hipMemcpyAsync(d, h, sizeof(Scal) * nrhs, hipMemcpyHostToDevice, st));
    WCL_CHECK(blas_dot(prec, V, nrhs, d, v, v, part, st));
    WCL_CHECK(blas_finalize(part, G, nrhs, d, FIN_RR, st, hm));
    WCL_HIP(hipStreamSynchronize(st));
    out.assign(nrhs, 0.0);
    for (int i = 0; i < nrhs; ++i) out[i] = h[i].rr;
    return WCL_OK;
}

static EoArgs eo_args(const wcl_lattice* lat, int prec, const void* ainv, double kappa, double csw, int nrhs) {
    EoArgs e{};
    e.g = lat->g;
    e.Vh = (int)(lat->V / 2);
    e.gauge = lat->gauge[prec];
    e.clover = lat->clover[prec];
    e.ainv = ainv;
    e.in_stride = e.in2_stride = e.a_stride = spinor_rhs_bytes(prec, e.Vh);
    e.y_stride = e.out_stride = spinor_rhs_bytes(prec, lat->V);
    e.kappa = kappa;
    e.csw = csw;
    e.nrhs = nrhs;
    return e;
}

static int need_even_extents(const wcl_lattice* lat) {
    for (int mu = 0; mu < 4; ++mu)
        if (lat->g.L[mu] % 2) {
            wcl_set_error("the even-odd reduction needs even extents (L[%d] = %d)", mu, lat->g.L[mu]);
            return WCL_EINVAL;
        }
    return WCL_OK;
}

// The nested solve on an explicit workspace (used by the C ABI with the
// lattice's own workspace and by the serving loop with per-slot ones).
// even_odd: both levels solve the Schur complement Dhat phi_e = b_e on the
// even half fields; phi_o is reconstructed afterwards and the reported true
// residual is |eta - D phi| / |eta| of the full system.
int nested_solve(wcl_lattice* lat, Workspace* ws, const wcl_solver_params* prm, double kappa, double csw,
                 const void* eta, void* phi, int nrhs, wcl_solve_stats* stats, hipStream_t st, double* resid_rhs) {
    WCL_CHECK(check_solver_params(prm));
    WCL_CHECK(need_fields(lat));
    if (!eta || !phi || nrhs < 1 || !std::isfinite(kappa) || !std::isfinite(csw)) {
        wcl_set_error("wcl_solve_nested_bicgstab: bad argument");
        return WCL_EINVAL;
    }
    const bool eo = prm->even_odd != 0;
    if (eo) WCL_CHECK(need_even_extents(lat));
    Blocks B{};
    const bool use_ras = prm->precond == WCL_PRECOND_RAS;
    if (use_ras) WCL_CHECK(make_blocks(lat, &prm->ras, &B));
    const int storage = prm->ras.storage;
    const int64_t Vs = eo ? lat->V / 2 : lat->V;   // sites of the solved system's vectors
    wcl_solve_stats local{};
    wcl_solve_stats* S = stats ? stats : &local;
    *S = wcl_solve_stats{};
    hipEvent_t e0, e1;
    WCL_HIP(hipEventCreate(&e0));
    WCL_HIP(hipEventCreate(&e1));
    WCL_HIP(hipEventRecord(e0, st));
    ws->tl.on = false;
    if (prm->timers) {
        ws->tl.start(st);
        ws->tl.mark(CAT_HOST);
    }

    Engine inner{lat, ws, "in", WCL_F32, WCL_F32, nrhs, kappa, csw, st, S};
    Engine outer{lat, ws, "out", WCL_F64, WCL_F64, nrhs, kappa, csw, st, S};
    // even-odd: b_e = eta_e - H_eo A_oo^{-1} eta_o, solved for x_e
    const void* rhs_vec = eta;
    void* sol_vec = phi;
    const double tol = prm->tol_outer;
    // per-rhs outer tolerance (the even-odd system measures against |b_e|)
    std::vector<double> tol_rhs(nrhs, tol);
    std::vector<double> eta2;
    if (eo) {
        void* inv[3];
        WCL_CHECK(site_inverse(lat, ws, kappa, csw, st, inv));
        inner.eo = outer.eo = 1;
        inner.eo_ainv = inv[WCL_F32];
        outer.eo_ainv = inv[WCL_F64];
        const size_t h64 = spinor_rhs_bytes(WCL_F64, Vs) * nrhs;
        void *be = nullptr, *te = nullptr, *xe = nullptr;
        WCL_CHECK(ws->get("eo.b", h64, &be));
        WCL_CHECK(ws->get("eo.t", h64, &te));
        WCL_CHECK(ws->get("eo.x", h64, &xe));
        EoArgs e = eo_args(lat, WCL_F64, inv[WCL_F64], kappa, csw, nrhs);
        ws->tl.mark(CAT_DSLASH);
        e.parity = 1;   // te = A_oo^{-1} eta_o
        e.y = eta;
        e.out = te;
        e.out_stride = spinor_rhs_bytes(WCL_F64, Vs);
        WCL_CHECK(launch_eo(e, WCL_F64, EO_SITEINV, DS_PLAIN, st));
        e.parity = 0;   // be = eta_e - H_eo te
        e.in = te;
        e.out = be;
        WCL_CHECK(launch_eo(e, WCL_F64, EO_PREP, DS_PLAIN, st));
        // The outer loop measures its residual against |b_e|; |eta - D phi|
        // equals the even part |b_e - Dhat x_e| (the odd part is solved
        // exactly), so it runs to tol |eta| / |b_e|.
        std::vector<double> b2;
        ws->tl.mark(CAT_BLAS);
        WCL_CHECK(host_norms2(ws, WCL_F64, lat->V, nrhs, eta, st, eta2));
        WCL_CHECK(host_norms2(ws, WCL_F64, Vs, nrhs, be, st, b2));
        for (int i = 0; i < nrhs; ++i)
            if (b2[i] > 0 && eta2[i] > 0) tol_rhs[i] = prm->tol_outer * std::sqrt(eta2[i] / b2[i]);
        rhs_vec = be;
        sol_vec = xe;
    }
    void *b32 = nullptr, *y32 = nullptr;
    const size_t v32 = spinor_rhs_bytes(WCL_F32, Vs) * nrhs;
    WCL_CHECK(ws->get("nest.b32", v32, &b32));
    WCL_CHECK(ws->get("nest.y32", v32, &y32));
    Precond Kras = [&](const void* in, void* out, Scal* sc, const std::vector<int>&) -> int {
        return ras_apply(lat, ws, B, storage, prm->ras.kernel, kappa, csw, in, out, nrhs, st, S, sc);
    };
    int outer_partials_G = blas_partials(WCL_F64, Vs);
    Precond Kinner = [&](const void* in, void* out, Scal* sc, const std::vector<int>& act) -> int {
        // b = in/|in| in FP32, inner solve, out = |in| y in FP64
        ws->tl.mark(CAT_BLAS);
        WCL_CHECK(blas_dot(WCL_F64, Vs, nrhs, sc, in, in, outer.partial, st));
        WCL_CHECK(blas_finalize(outer.partial, outer_partials_G, nrhs, sc, FIN_PP, st));
        WCL_CHECK(blas_to_f32_scaled(Vs, nrhs, sc, in, b32, st));
        // The inner solve needs only the accuracy that takes the outer
        // residual to its target: about tol / (|r| / |b|), with a safety
        // factor of 4; never tighter than tol_inner, never looser than 0.1.
        // (An exact preconditioner would end the outer solve in one step.)
        // Per rhs, so that a batched rhs takes the path of its own solve.
        std::vector<double> tin(nrhs, prm->tol_inner);
        for (int i = 0; i < nrhs; ++i) {
            const double want = 0.25 * tol_rhs[i] / std::max(outer.rel_now[i], 1e-300);
            tin[i] = std::max(prm->tol_inner, std::min(0.1, want));
        }
        std::vector<int> a = act;
        EngineResult r;
        WCL_CHECK(inner.run(b32, y32, prm->tol_inner, prm->max_inner, use_ras ? &Kras : nullptr, a, false, 0, &r,
                            &tin));
        S->inner_iters += r.iters;
        ws->tl.mark(CAT_BLAS);
        WCL_CHECK(blas_to_f64_scaled(Vs, nrhs, sc, y32, out, st));
        return WCL_OK;
    };
    std::vector<int> act(nrhs, 1);
    EngineResult res;
    int rc = outer.run(rhs_vec, sol_vec, tol, prm->max_outer, &Kinner, act, true, prm->max_restarts, &res, &tol_rhs);
    if (rc == WCL_OK && eo) {
        // phi_o = A_oo^{-1} (eta_o - H_oe x_e), phi_e = x_e; then the full
        // system's true residual
        void* inv[3];
        WCL_CHECK(site_inverse(lat, ws, kappa, csw, st, inv));
        EoArgs e = eo_args(lat, WCL_F64, inv[WCL_F64], kappa, csw, nrhs);
        ws->tl.mark(CAT_DSLASH);
        e.parity = 1;
        e.in = sol_vec;
        e.y = eta;
        e.out = phi;
        WCL_CHECK(launch_eo(e, WCL_F64, EO_RECON, DS_PLAIN, st));
        e.parity = 0;
        e.in2 = sol_vec;
        WCL_CHECK(launch_eo(e, WCL_F64, EO_INSERT, DS_PLAIN, st));
        void* rfull = nullptr;
        WCL_CHECK(ws->get("eo.res", spinor_rhs_bytes(WCL_F64, lat->V) * nrhs, &rfull));
        DslashArgs d{};
        d.g = lat->g;
        d.gauge = lat->gauge[WCL_F64];
        d.clover = lat->clover[WCL_F64];
        d.in = phi;
        d.y = eta;
        d.out = rfull;
        d.in_stride = d.out_stride = d.y_stride = spinor_rhs_bytes(WCL_F64, lat->V);
        d.kappa = kappa;
        d.csw = csw;
        d.nrhs = nrhs;
        d.lps = lat->lps;
        WCL_CHECK(launch_dslash(d, WCL_F64, WCL_F64, WCL_F64, DS_AXPY, WCL_F64, st));
        S->dslash_full += nrhs;
        std::vector<double> r2;
        ws->tl.mark(CAT_BLAS);
        WCL_CHECK(host_norms2(ws, WCL_F64, lat->V, nrhs, rfull, st, r2));
        res.true_resid = 0.0;
        res.tres.assign(nrhs, 0.0);
        for (int i = 0; i < nrhs; ++i)
            if (eta2[i] > 0) {
                res.tres[i] = std::sqrt(r2[i] / eta2[i]);
                res.true_resid = std::max(res.true_resid, res.tres[i]);
            }
    }
    if (resid_rhs)
        for (int i = 0; i < nrhs; ++i) resid_rhs[i] = i < (int)res.tres.size() ? res.tres[i] : -1.0;
    WCL_HIP(hipEventRecord(e1, st));
    WCL_HIP(hipEventSynchronize(e1));
    float ms = 0;
    WCL_HIP(hipEventElapsedTime(&ms, e0, e1));
    double cat[CAT_N];
    ws->tl.finish(e1, cat);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != WCL_OK) return rc;
    S->outer_iters = res.iters;
    S->restarts += res.restarts;
    S->converged = res.converged;
    S->true_resid = res.true_resid;
    S->ms_total = ms;
    S->ms_dslash = cat[CAT_DSLASH];
    S->ms_dominv = cat[CAT_DOMINV];
    S->ms_blas = cat[CAT_BLAS];
    S->ms_host = cat[CAT_HOST];
    if (!res.converged || !(res.true_resid <= prm->tol_outer)) {
        S->converged = 0;
        if (res.breakdown) {
            wcl_set_error("nested BiCGStab: breakdown persisted after %d restarts (true residual %.3e)",
                          res.restarts, res.true_resid);
            return WCL_EBREAKDOWN;
        }
        wcl_set_error("nested BiCGStab: true residual %.3e above tolerance %.3e after %d outer iterations",
                      res.true_resid, prm->tol_outer, res.iters);
        return WCL_ENOTCONV;
    }
    return WCL_OK;
}

extern "C" {

int wcl_block_info(const wcl_lattice* lat, const wcl_ras_params* ras, int64_t* nblocks, int64_t* ext_volume) {
    if (!lat || !nblocks || !ext_volume) return WCL_EINVAL;
    Blocks B;
    WCL_CHECK(make_blocks(lat, ras, &B));
    *nblocks = B.nblocks;
    *ext_volume = B.ev;
    return WCL_OK;
}

int wcl_apply_D_blocks(wcl_lattice* lat, const wcl_ras_params* ras, double kappa, double csw, const void* in_dev,
                       double* out_host, void* stream) {
    if (!lat || !in_dev || !out_host) {
        wcl_set_error("wcl_apply_D_blocks: null argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(need_fields(lat));
    Blocks B;
    WCL_CHECK(make_blocks(lat, ras, &B));
    WCL_HIP(hipSetDevice(lat->ctx->device));
    hipStream_t st = (hipStream_t)stream;
    Workspace* ws = lattice_ws(lat);
    BlockArgs a{};
    a.g = lat->g;
    a.B = B;
    a.colour = -1;
    a.gauge = lat->gauge[ras->storage];
    a.clover = lat->clover[ras->storage];
    a.NE = B.nblocks * B.ev;
    a.wpb = (B.ev + 255) / 256;
    a.ws_stride = (size_t)6 * a.NE;
    a.kappa = kappa;
    a.csw = csw;
    a.nrhs = 1;
    a.src = in_dev;
    a.src_stride = spinor_rhs_bytes(WCL_F32, lat->V);
    const size_t wsb = (size_t)16 * 6 * a.NE;
    WCL_CHECK(ws->get("ras.rho", wsb, &a.rho));
    WCL_CHECK(ws->get("ras.q", wsb, &a.q));
    WCL_CHECK(ws->get("ras.x", wsb, &a.x));
    WCL_CHECK(ws->get("ras.partial", (size_t)24 * B.nblocks * a.wpb, (void**)&a.partial));
    void* stage = nullptr;
    const size_t ob = (size_t)a.NE * 24 * sizeof(double);
    WCL_CHECK(ws->get("blocks.out", ob, &stage));
    WCL_CHECK(launch_blk_project(a, WCL_F32, 0, st));
    WCL_CHECK(launch_blk_dslash(a, ras->storage, st));
    WCL_CHECK(launch_blk_unpack(a, (const float*)a.q, (double*)stage, st));
    WCL_HIP(hipMemcpyAsync(out_host, stage, ob, hipMemcpyDeviceToHost, st));
    WCL_HIP(hipStreamSynchronize(st));
    return WCL_OK;
}

int wcl_ras_precondition(wcl_lattice* lat, const wcl_ras_params* ras, double kappa, double csw, const void* r_dev,
                         void* v_dev, int nrhs, void* stream) {
    if (!lat || !r_dev || !v_dev || r_dev == v_dev || nrhs < 1) {
        wcl_set_error("wcl_ras_precondition: bad argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(need_fields(lat));
    Blocks B;
    WCL_CHECK(make_blocks(lat, ras, &B));
    WCL_HIP(hipSetDevice(lat->ctx->device));
    return ras_apply(lat, lattice_ws(lat), B, ras->storage, ras->kernel, kappa, csw, r_dev, v_dev, nrhs, (hipStream_t)stream,
                     nullptr);
}

int wcl_ras_precondition_noalloc(wcl_lattice* lat, const wcl_ras_params* ras, double kappa, double csw,
                                 const void* r_dev, void* v_dev, int nrhs, void* stream) {
    if (!lat || !ras || !r_dev || !v_dev || r_dev == v_dev || nrhs < 1) {
        wcl_set_error("wcl_ras_precondition_noalloc: bad argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(need_fields(lat));
    Blocks B;
    WCL_CHECK(make_blocks(lat, ras, &B));
    if (B.solver != WCL_DOMSOLVE_MR || B.schwarz != WCL_SCHWARZ_RAS || ras->kernel == WCL_BLOCK_SPLIT ||
        fused_threads(B.ev) != 256) {
        wcl_set_error("wcl_ras_precondition_noalloc: only the on-chip path (minimal-residual domain solves inside "
                      "RAS, extended domains of at most 256 sites) runs without allocating");
        return WCL_EINVAL;
    }
    if (!lat->ctx->scratch) {
        wcl_set_error("wcl_ras_precondition_noalloc: fixed scratch block not set up on device %d", lat->ctx->device);
        return WCL_ESTATE;
    }
    RasBufs bf;
    std::vector<BufReq> req;
    ras_buffer_list(B, true, ras->storage, lat->V, nrhs, bf, req);
    size_t off = 0;
    for (auto& q : req) off += round_up(q.bytes, 256);
    if (off > (size_t)WCL_NOALLOC_SCRATCH_BYTES) {
        wcl_set_error("wcl_ras_precondition_noalloc: needs %zu bytes of scratch for %d rhs on this lattice, "
                      "more than the fixed %zu", off, nrhs, (size_t)WCL_NOALLOC_SCRATCH_BYTES);
        return WCL_EINVAL;
    }
    off = 0;
    for (auto& q : req) {
        *q.slot = (char*)lat->ctx->scratch + off;
        off += round_up(q.bytes, 256);
    }
    WCL_HIP(hipSetDevice(lat->ctx->device));
    return ras_run(lat, B, true, ras->storage, kappa, csw, r_dev, v_dev, nrhs, (hipStream_t)stream, nullptr, nullptr,
                   bf, nullptr, nullptr);
}

int wcl_apply_schur(wcl_lattice* lat, int prec, double kappa, double csw, const void* in_dev, void* out_dev, int nrhs,
                    void* stream) {
    if (!lat || !in_dev || !out_dev || in_dev == out_dev || nrhs < 1 || (prec != WCL_F64 && prec != WCL_F32) ||
        !std::isfinite(kappa) || !std::isfinite(csw)) {
        wcl_set_error("wcl_apply_schur: bad argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(need_fields(lat));
    WCL_CHECK(need_even_extents(lat));
    WCL_HIP(hipSetDevice(lat->ctx->device));
    hipStream_t st = (hipStream_t)stream;
    Workspace* ws = lattice_ws(lat);
    void* inv[3];
    WCL_CHECK(site_inverse(lat, ws, kappa, csw, st, inv));
    const int64_t Vh = lat->V / 2;
    const size_t hb = spinor_rhs_bytes(prec, Vh) * nrhs;
    void *xe = nullptr, *to = nullptr, *ye = nullptr;
    WCL_CHECK(ws->get("schur.x", hb, &xe));
    WCL_CHECK(ws->get("schur.t", hb, &to));
    WCL_CHECK(ws->get("schur.y", hb, &ye));
    EoArgs e = eo_args(lat, prec, inv[prec], kappa, csw, nrhs);
    const size_t hs = spinor_rhs_bytes(prec, Vh), fs = spinor_rhs_bytes(prec, lat->V);
    e.parity = 0;   // x_e = in on the even sites
    e.y = in_dev;
    e.out = xe;
    e.out_stride = hs;
    WCL_CHECK(launch_eo(e, prec, EO_EXTRACT, DS_PLAIN, st));
    e.parity = 1;   // t_o = A_oo^{-1} H_oe x_e
    e.in = xe;
    e.out = to;
    WCL_CHECK(launch_eo(e, prec, EO_INV, DS_PLAIN, st));
    e.parity = 0;   // y_e = A_ee x_e - H_eo t_o
    e.in = to;
    e.in2 = xe;
    e.out = ye;
    WCL_CHECK(launch_eo(e, prec, EO_SCHUR, DS_PLAIN, st));
    e.out = out_dev;
    e.out_stride = fs;
    e.parity = 1;
    WCL_CHECK(launch_eo(e, prec, EO_ZERO, DS_PLAIN, st));
    e.parity = 0;
    e.in2 = ye;
    WCL_CHECK(launch_eo(e, prec, EO_INSERT, DS_PLAIN, st));
    return WCL_OK;
}

int wcl_solve_nested_bicgstab(wcl_lattice* lat, const wcl_solver_params* p, double kappa, double csw,
                              const void* eta_dev, void* phi_dev, int nrhs, wcl_solve_stats* stats, void* stream) {
    if (!lat) return WCL_EINVAL;
    WCL_HIP(hipSetDevice(lat->ctx->device));
    return nested_solve(lat, lattice_ws(lat), p, kappa, csw, eta_dev, phi_dev, nrhs, stats, (hipStream_t)stream);
}

int wcl_solve_bicgstab_f64(wcl_lattice* lat, double tol, int max_iter, double kappa, double csw, const void* eta_dev,
                           void* phi_dev, wcl_solve_stats* stats, void* stream) {
    if (!lat || !eta_dev || !phi_dev || !(tol > 0) || max_iter < 1) {
        wcl_set_error("wcl_solve_bicgstab_f64: bad argument");
        return WCL_EINVAL;
    }
    WCL_CHECK(need_fields(lat));
    WCL_HIP(hipSetDevice(lat->ctx->device));
    hipStream_t st = (hipStream_t)stream;
    wcl_solve_stats local{};
    wcl_solve_stats* S = stats ? stats : &local;
    *S = wcl_solve_stats{};
    hipEvent_t e0, e1;
    WCL_HIP(hipEventCreate(&e0));
    WCL_HIP(hipEventCreate(&e1));
    WCL_HIP(hipEventRecord(e0, st));
    Engine eng{lat, lattice_ws(lat), "plain", WCL_F64, WCL_F64, 1, kappa, csw, st, S};
    std::vector<int> act(1, 1);
    EngineResult res;
    // plain solver: stop on the recursive residual, no restart; report the true residual
    int rc = eng.run(eta_dev, phi_dev, tol, max_iter, nullptr, act, false, 0, &res);
    if (rc == WCL_OK) {
        // true residual for the report
        eng.h[0].active = 1;
        rc = eng.push();
        if (rc == WCL_OK) rc = eng.residual(eta_dev, phi_dev, eng.t);
        if (rc == WCL_OK) rc = blas_dot(WCL_F64, lat->V, 1, eng.d, eng.t, eng.t, eng.partial, st);
        if (rc == WCL_OK) rc = blas_finalize(eng.partial, eng.Gb, 1, eng.d, FIN_RR, st, eng.hmap);
        if (rc == WCL_OK) rc = eng.pull();
        if (rc == WCL_OK) {
            // |eta|: reuse the dot on the right-hand side
            double rr = eng.h[0].rr;
            rc = blas_dot(WCL_F64, lat->V, 1, eng.d, eta_dev, eta_dev, eng.partial, st);
            if (rc == WCL_OK) rc = blas_finalize(eng.partial, eng.Gb, 1, eng.d, FIN_RR, st, eng.hmap);
            if (rc == WCL_OK) rc = eng.pull();
            if (rc == WCL_OK) S->true_resid = eng.h[0].rr > 0 ? std::sqrt(rr / eng.h[0].rr) : 0.0;
        }
    }
    WCL_HIP(hipEventRecord(e1, st));
    WCL_HIP(hipEventSynchronize(e1));
    float ms = 0;
    WCL_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != WCL_OK) return rc;
    S->outer_iters = res.iters;
    S->restarts = res.restarts;
    S->converged = res.converged;
    S->ms_total = ms;
    if (!res.converged) {
        if (res.breakdown) {
            wcl_set_error("BiCGStab FP64: breakdown persisted after %d restarts", res.restarts);
            return WCL_EBREAKDOWN;
        }
        wcl_set_error("BiCGStab FP64: not converged after %d iterations", res.iters);
        return WCL_ENOTCONV;
    }
    return WCL_OK;
}

}  // extern "C"
