// Host side of libsuppcg: argument validation, geometry tables, workspace
// management and the SupPCG driver (Algorithm 3) behind the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/suppcg.h"
#include "sp_blob.h"
#include "sp_internal.h"
#include "sp_stored.h"

using namespace sp;

namespace {

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Batched solve: per-slice tables and buffers of one batch layout (the
// geometries and preconditioner kind), cached across calls.
struct BatchState {
    std::vector<sp_geometry> geoms;
    int kind = -1;
    int nbmax = 1;
    int bp_px = 2;                   // R^T pixels per lane for the whole batch
    size_t lds_rows = 0, lds_cols = 0;
    std::vector<SliceDev> hs;        // host copies; per-call pointers filled in each call
    DevBuf arena, sl, items, scal, trace_d;
    size_t off[BS_COUNT][2] = {};    // item-table offsets (entries) per stage and order
    int count[BS_COUNT][2] = {};
    int order[BS_COUNT] = {};        // chosen order (0 slice-major, 1 grouped by XCD)
    int wpc[BS_COUNT] = {};          // chosen workgroups per CU (0: one per item)
    bool tuned = false;
    uint64_t epoch = 0;              // launch-shape epoch of the layout
};

}  // namespace

struct sp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char err[512] = {0};   // last failure (fixed storage: reporting an error allocates nothing)

    // geometry cache
    bool have_geom = false;
    uint64_t geom_epoch = 0;   // launch-shape epoch the cached tables were built at
    sp_geometry geom{};
    GeomDev G{};
    std::vector<AngleDev> ang_h;
    DevBuf ang, pwave, xp, xTp, yp, ypd, seg, pord, blob_tab;

    // preconditioner cache
    int fftP = 0;
    DevBuf tw, S;

    // solver vectors and scratch.  vx, vxh, vp, vq and scal carry Algorithm 3's
    // state from one loop body to the next and survive the call (checkpoint /
    // resume); the standalone operators use ox, oxh and oscal instead.
    DevBuf vx, vxh, vp;                   // float64 x_k, x_{k+1/2}, p
    DevBuf vq, vw;                        // float64 q = R p and w = R z (nA x nB)
    DevBuf vg, vz, vtb, vtmp;
    DevBuf vtb2, stv_y;                   // S_TV ping-pong: second t_bar (float), iterate (float64)
    DevBuf ox, oxh, oscal;                // sp_tv, sp_tv_grad, sp_tv_perturb
    DevBuf part_f, part_zh, part_gp, part_qq, part_g, part_t, part_s, part_misc, part_se;
    DevBuf stored_xT;                     // transposed image for the stored R product
    DevBuf art_u, art_nrm, art_sum;       // ART: auxiliary vector, ||R_i||^2, sum of b
    DevBuf scal, trace_d, replay_d, trials_tmp;
    Scalars sc_h{};
    hipStream_t own = nullptr;   // capture stream used when the caller's stream is null
    hipEvent_t own_ev[2] = {nullptr, nullptr};   // orders `own` against the null stream (SP_FLAG_ASYNC)

    // Algorithm 3's state left by the last single-slice solve (or sp_state_load):
    // valid while `ok`, with the parameters it was produced with.
    struct SolverState {
        bool ok = false;
        sp_geometry geom{};
        int32_t K = 0, max_trials = 0, kind = 0;
        double a = 0.0, gamma = 0.0, mu = 0.0, rho = 0.0;
    } st;
    // The last solve, for sp_solve_status: 0 none, 1 single-slice, 2 batched
    // (count slices); its eps; a graph whose launches may still be in flight
    // (SP_FLAG_ASYNC), destroyed once the stream has drained.
    int last_kind = 0, last_count = 0;
    double last_eps = 0.0;
    hipGraph_t pend_graph = nullptr;
    hipGraphExec_t pend_exec = nullptr;

    // host staging of sp_backproject_noalloc's tables, sized at creation, and
    // the event after their last upload (the next call waits on it before
    // writing them again)
    std::vector<AngleDev> na_tab;
    hipEvent_t na_ev = nullptr;
    BatchState* batch = nullptr;
    int n_cu = 0;

    // instrumentation: event pairs around launches (sp_profile_enable)
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct ProfRec {
        int kind;
        size_t e0, e1;
    };
    std::vector<ProfRec> prof_recs;
};

// R and R^T stored on the device as sliced ELLPACK (side 0: R by rays, side
// 1: R^T by pixels): slice offsets sp, row lengths len, entries col / val.
struct sp_matrix {
    int device = 0;
    sp_geometry geom{};
    int64_t rows[2] = {0, 0};
    sp::SellShape shape[2] = {};
    int64_t words[2] = {0, 0};     // 32-bit words of each side's entries, padding included
    int64_t nnz = 0;
    DevBuf sp[2], len[2], ent[2];
    DevBuf segT;                   // R: 1 for angles whose rows index the transposed image
};

// Learned preconditioner: parameters, Adam moments and workspace.
struct sp_learned {
    int device = 0;
    int layers = 0, channels = 16, nparams = 0;
    DevBuf theta, adam_m, adam_v, spsg;   // spsg: softplus(d) [16], sigmoid(d) [16]
    size_t cap_pix = 0;                   // pixels the activation buffers hold
    std::vector<DevBuf> act;              // training: a_1..a_L, b_1..b_L, e_1..e_L
    DevBuf a0, z, e0, ping, pong, partial, rtmp, lpart, gdpart;
    int woff(int l) const { return l == 1 ? 0 : 144 + (l - 2) * 2304; }   // W_l offset
    int doff() const { return 144 + (layers - 1) * 2304; }
};

namespace {

int fail(sp_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) std::memcpy(c->err, buf, sizeof buf);
    return code;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), SP_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

// Grows `b` to at least `bytes` (contents are not preserved); zero-fills new storage.
int ensure(sp_ctx* c, DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes && b.ptr) return SP_OK;
    if (b.ptr) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, SP_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    bytes = std::max<size_t>(bytes, 256);
    if (hipMalloc(&b.ptr, bytes) != hipSuccess) {
        b.ptr = nullptr;
        return fail(c, SP_ERR_ALLOC, "hipMalloc of %zu bytes failed", bytes);
    }
    b.bytes = bytes;
    HIP_TRY(c, hipMemsetAsync(b.ptr, 0, bytes, c->stream));
    return SP_OK;
}

void release(DevBuf& b) {
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

template <class T>
T* dptr(DevBuf& b) { return static_cast<T*>(b.ptr); }

bool same_geom(const sp_geometry& a, const sp_geometry& b) {
    return std::memcmp(&a, &b, sizeof a) == 0;
}

int validate_geometry(sp_ctx* c, const sp_geometry* g) {
    if (!g) return fail(c, SP_ERR_ARG, "geometry is NULL");
    if (g->rows < 1 || g->cols < 1 || g->rows > 8192 || g->cols > 8192)
        return fail(c, SP_ERR_ARG, "rows/cols must be in [1, 8192] (got %d x %d)", g->rows, g->cols);
    if (g->n_angles < 1 || g->n_angles > 65536)
        return fail(c, SP_ERR_ARG, "n_angles must be in [1, 65536] (got %d)", g->n_angles);
    if (g->n_bins < 1 || g->n_bins > 65536)
        return fail(c, SP_ERR_ARG, "n_bins must be in [1, 65536] (got %d)", g->n_bins);
    if (!(g->pixel > 0.0) || !std::isfinite(g->pixel))
        return fail(c, SP_ERR_ARG, "pixel must be positive and finite");
    if (!(g->bin_spacing > 0.0) || !std::isfinite(g->bin_spacing))
        return fail(c, SP_ERR_ARG, "bin_spacing must be positive and finite");
    if (!std::isfinite(g->theta0) || !std::isfinite(g->dtheta) || !std::isfinite(g->bin_offset))
        return fail(c, SP_ERR_ARG, "theta0, dtheta and bin_offset must be finite");
    const double ds = g->bin_spacing / g->pixel;
    if (ds < 0.375) return fail(c, SP_ERR_ARG, "bin_spacing below 0.375 pixel is not supported");
    const double pitchB = (double)g->n_bins + 2 * PAD;
    if ((double)g->n_angles * pitchB > 2.0e9) return fail(c, SP_ERR_ARG, "sinogram too large");
    return SP_OK;
}

// Launch shapes of the projector pair per geometry (sp_tune_shapes,
// sp_tuning_set): R's ray parts and R^T's pixels per lane, process-wide.
// Every table built for a geometry takes its entry, so single and batched
// solves of one geometry use the same shapes; the epoch changes with every
// update, which makes the contexts rebuild their cached tables.
struct ShapeEntry {
    sp_geometry g;
    int32_t parts, px;
};
std::mutex g_shape_mu;
std::vector<ShapeEntry> g_shapes;
std::atomic<uint64_t> g_shape_epoch{1};

bool shape_lookup(const sp_geometry& g, int& parts, int& px) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    for (const ShapeEntry& e : g_shapes)
        if (same_geom(e.g, g)) {
            parts = e.parts;
            px = e.px;
            return true;
        }
    return false;
}

// parts == 0 erases the entry
void shape_store(const sp_geometry& g, int parts, int px) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    for (size_t i = 0; i < g_shapes.size(); ++i)
        if (same_geom(g_shapes[i].g, g)) {
            if (parts == 0) g_shapes.erase(g_shapes.begin() + (long)i);
            else g_shapes[i].parts = parts, g_shapes[i].px = px;
            ++g_shape_epoch;
            return;
        }
    if (parts != 0) g_shapes.push_back(ShapeEntry{g, parts, px});
    ++g_shape_epoch;
}

// Device geometry and class-sorted angle table (geometry.cpp), failures
// reported on the context; tuned launch shapes replace the defaults.
int build_geometry_into(sp_ctx* c, const sp_geometry* g, GeomDev& G, AngleDev* tab) {
    char msg[256];
    const int rc = sp::build_geometry_into(g, c->n_cu, G, tab, msg, sizeof msg);
    if (rc) return fail(c, rc, "%s", msg);
    int parts, px;
    if (shape_lookup(*g, parts, px)) {
        G.parts = parts;
        G.bp_px = px;
    }
    return SP_OK;
}

int build_geometry(sp_ctx* c, const sp_geometry* g, GeomDev& G, std::vector<AngleDev>& tab) {
    tab.assign(g->n_angles, AngleDev{});
    return build_geometry_into(c, g, G, tab.data());
}

int setup_geometry(sp_ctx* c, const sp_geometry* g) {
    int rc = validate_geometry(c, g);
    if (rc) return rc;
    const uint64_t epoch = g_shape_epoch.load();
    if (c->have_geom && same_geom(c->geom, *g) && c->geom_epoch == epoch) return SP_OK;
    GeomDev G{};
    std::vector<AngleDev> tab;
    if ((rc = build_geometry(c, g, G, tab))) return rc;
    const size_t nX = (size_t)g->rows * G.pitchX, nXT = (size_t)g->cols * G.pitchXT;
    const size_t nY = (size_t)g->n_angles * G.pitchB;
    // Padded buffers must have zero pads: re-zero when the layout changes.
    if ((rc = ensure(c, c->ang, tab.size() * sizeof(AngleDev)))) return rc;
    const bool relayout = !c->have_geom || c->G.pitchX != G.pitchX || c->G.pitchXT != G.pitchXT ||
                          c->G.pitchB != G.pitchB || c->G.rows != G.rows || c->G.cols != G.cols ||
                          c->G.nA != G.nA;
    if ((rc = ensure(c, c->xp, nX * 8))) return rc;
    if ((rc = ensure(c, c->xTp, nXT * 8))) return rc;
    if ((rc = ensure(c, c->yp, nY * 4))) return rc;
    if ((rc = ensure(c, c->ypd, nY * 8))) return rc;
    if (G.parts > 1 && (rc = ensure(c, c->seg, (size_t)G.parts * g->n_angles * g->n_bins * 8)))
        return rc;
    if (relayout) {
        HIP_TRY(c, hipMemsetAsync(c->xp.ptr, 0, c->xp.bytes, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->xTp.ptr, 0, c->xTp.bytes, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->yp.ptr, 0, c->yp.bytes, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->ypd.ptr, 0, c->ypd.bytes, c->stream));
    }
    c->ang_h = tab;
    std::vector<WaveDev> waves((size_t)G.nwaves);
    project_waves(G, waves.data());
    if ((rc = ensure(c, c->pwave, waves.size() * sizeof(WaveDev)))) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->pwave.ptr, waves.data(), waves.size() * sizeof(WaveDev),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->ang.ptr, tab.data(), tab.size() * sizeof(AngleDev),
                              hipMemcpyHostToDevice, c->stream));
    const std::vector<int32_t> ord = project_order(G, tab.data(), waves.data(), c->n_cu);
    if ((rc = ensure(c, c->pord, ord.size() * sizeof(int32_t)))) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->pord.ptr, ord.data(), ord.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));  // host tables must outlive the copies
    c->G = G;
    c->geom = *g;
    c->geom_epoch = epoch;
    c->have_geom = true;
    return SP_OK;
}

int pad_size(int rows, int cols) {
    int P = 1;
    while (P < 2 * std::max(rows, cols)) P <<= 1;
    return P;
}

int setup_fft(sp_ctx* c, FFTPlan& F) {
    const sp_geometry& g = c->geom;
    const int P = pad_size(g.rows, g.cols);
    if (P > 4096) return fail(c, SP_ERR_ARG, "preconditioner supports images up to 2048 pixels a side");
    int rc;
    if (c->fftP != P) {
        std::vector<double2> tw(P / 2);
        for (int k = 0; k < P / 2; ++k) {
            const double ang = -2.0 * M_PI * (double)k / (double)P;
            tw[k] = make_double2(std::cos(ang), std::sin(ang));
        }
        if ((rc = ensure(c, c->tw, tw.size() * sizeof(double2)))) return rc;
        HIP_TRY(c, hipMemcpyAsync(c->tw.ptr, tw.data(), tw.size() * sizeof(double2),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->fftP = P;
    }
    const int SP = P / 2 + 1;
    if ((rc = ensure(c, c->S, (size_t)g.rows * SP * sizeof(double2)))) return rc;
    F.P = P;
    F.logP = 0;
    while ((1 << F.logP) < P) ++F.logP;
    F.SP = SP;
    F.rows = g.rows;
    F.cols = g.cols;
    F.CB = std::max(1, 2048 / P);
    F.S = dptr<double2>(c->S);
    F.tw = dptr<double2>(c->tw);
    return SP_OK;
}

int check_precond(sp_ctx* c, const sp_precond* pc) {
    if (!pc) return fail(c, SP_ERR_ARG, "preconditioner is NULL");
    if (pc->kind == SP_PRECOND_NONE) return SP_OK;
    if (pc->kind == SP_PRECOND_RAMP) {
        if (!std::isfinite(pc->mu) || !std::isfinite(pc->rho))
            return fail(c, SP_ERR_ARG, "mu and rho must be finite");
        if (!(pc->mu > 0.0) || !(pc->rho > 0.5) || pc->rho > 1.0)
            return fail(c, SP_ERR_NOT_SPD,
                        "M is positive definite only for mu > 0 and 1/2 < rho <= 1 (mu=%g rho=%g)",
                        pc->mu, pc->rho);
        return SP_OK;
    }
    if (pc->kind == SP_PRECOND_LEARNED) {
        if (!pc->net) return fail(c, SP_ERR_ARG, "SP_PRECOND_LEARNED needs a network");
        if (pc->net->device != c->device) return fail(c, SP_ERR_ARG, "network lives on another GPU");
        if (!std::isfinite(pc->mu) || !std::isfinite(pc->rho) || !(pc->mu > 0.0) ||
            !(pc->rho > 0.5) || pc->rho > 1.0)
            return fail(c, SP_ERR_NOT_SPD,
                        "the fallback Fourier preconditioner needs mu > 0 and 1/2 < rho <= 1");
        return SP_OK;
    }
    return fail(c, SP_ERR_ARG, "unknown preconditioner kind %d", pc->kind);
}

int check_tv(sp_ctx* c, const sp_tv_params* p) {
    if (!p) return SP_OK;
    if (p->K < 0 || p->K > 1000) return fail(c, SP_ERR_ARG, "K must be in [0, 1000]");
    if (p->K == 0) return SP_OK;
    if (!(p->a > 0.0 && p->a < 1.0)) return fail(c, SP_ERR_ARG, "a must be in (0, 1)");
    if (!(p->gamma > 0.0) || !std::isfinite(p->gamma)) return fail(c, SP_ERR_ARG, "gamma must be positive");
    if (p->max_trials < 0 || p->max_trials > 10000) return fail(c, SP_ERR_ARG, "max_trials must be in [0, 10000]");
    return SP_OK;
}

// Solver vectors of n pixels (and the nA x nB ray vectors of the context's
// geometry).
int ensure_vectors(sp_ctx* c, size_t n) {
    int rc;
    const size_t m = (size_t)c->G.nA * c->G.nB;
    for (DevBuf* b : {&c->vg, &c->vz, &c->vtb, &c->vtb2, &c->vtmp})
        if ((rc = ensure(c, *b, n * sizeof(float)))) return rc;
    for (DevBuf* b : {&c->vx, &c->vxh, &c->vp, &c->stv_y})
        if ((rc = ensure(c, *b, n * sizeof(double)))) return rc;
    for (DevBuf* b : {&c->vq, &c->vw})
        if ((rc = ensure(c, *b, m * sizeof(double)))) return rc;
    return SP_OK;
}

int ensure_partials(sp_ctx* c) {
    const GeomDev& G = c->G;
    const int n = G.rows * G.cols;
    int rc;
    if ((rc = ensure(c, c->part_f, (size_t)project_blocks(G) * 8))) return rc;
    if ((rc = ensure(c, c->part_qq, (size_t)vec_blocks(G.nA * G.nB) * 8))) return rc;
    if ((rc = ensure(c, c->part_zh, (size_t)std::max((G.rows + 1) / 2, vec_blocks(n)) * 8))) return rc;
    if ((rc = ensure(c, c->part_gp, (size_t)vec_blocks(n) * 8))) return rc;
    if ((rc = ensure(c, c->part_g, (size_t)tv_blocks(G.rows, G.cols) * 8))) return rc;
    if ((rc = ensure(c, c->part_t, (size_t)tv_blocks(G.rows, G.cols) * 9 * 8))) return rc;
    if ((rc = ensure(c, c->part_s, (size_t)std::max(tv_blocks(G.rows, G.cols), tv_prep_tiles(G.rows, G.cols)) * 8)))
        return rc;
    if ((rc = ensure(c, c->part_misc, (size_t)vec_blocks(n) * 8))) return rc;
    if ((rc = ensure(c, c->part_se, (size_t)vec_blocks(n) * 16))) return rc;
    if ((rc = ensure(c, c->scal, sizeof(Scalars)))) return rc;
    return SP_OK;
}

int upload_scalars(sp_ctx* c, DevBuf& dst) {
    HIP_TRY(c, hipMemcpyAsync(dst.ptr, &c->sc_h, sizeof(Scalars), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SP_OK;
}

// Scratch of the standalone TV operators (never the solver's state).
int ensure_op_vectors(sp_ctx* c, size_t n) {
    int rc;
    if ((rc = ensure(c, c->ox, n * sizeof(double)))) return rc;
    if ((rc = ensure(c, c->oxh, n * sizeof(double)))) return rc;
    if ((rc = ensure(c, c->vtb, n * sizeof(float)))) return rc;
    if ((rc = ensure(c, c->vtb2, n * sizeof(float)))) return rc;
    if ((rc = ensure(c, c->stv_y, n * sizeof(double)))) return rc;
    return ensure(c, c->oscal, sizeof(Scalars));
}

int check_launch(sp_ctx* c) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, SP_ERR_HIP, "kernel launch: %s", hipGetErrorString(e));
    return SP_OK;
}

// Status of a finished run from its scalars (Algorithm 3's outcome).
int run_status(const Scalars& q, double eps) {
    if (q.halt) return q.halt;
    if (eps > 0.0 && !(q.f > eps)) return SP_CONVERGED;   // max_iter ended on the test
    if (q.exhausted) return SP_TRIALS_EXHAUSTED;
    return SP_MAXITER;
}

// Waits for and releases the graph an asynchronous solve left in flight.
int drain_pending(sp_ctx* c) {
    if (!c->pend_exec && !c->pend_graph) return SP_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->own) HIP_TRY(c, hipStreamSynchronize(c->own));
    if (c->pend_exec) (void)hipGraphExecDestroy(c->pend_exec);
    if (c->pend_graph) (void)hipGraphDestroy(c->pend_graph);
    c->pend_exec = nullptr;
    c->pend_graph = nullptr;
    return SP_OK;
}

size_t prof_mark(sp_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return (size_t)-1;
        c->ev_pool.push_back(e);
    }
    (void)hipEventRecord(c->ev_pool[c->ev_used], c->stream);
    return c->ev_used++;
}

// Brackets the launches made in its scope with events when profiling is on.
struct ProfScope {
    sp_ctx* c;
    int kind;
    size_t e0 = (size_t)-1;
    ProfScope(sp_ctx* c_, int k) : c(c_), kind(k) {
        if (c->prof) e0 = prof_mark(c);
    }
    ~ProfScope() {
        if (c->prof && e0 != (size_t)-1) {
            const size_t e1 = prof_mark(c);
            if (e1 != (size_t)-1) c->prof_recs.push_back({kind, e0, e1});
        }
    }
};

// One S_TV call (Algorithm 1) from x into xh, K inner steps.  With snorm the
// partials of ||xh - x||^2 go to part_s, and unless ride_snorm (a later
// kernel carries the step, see ScalarRide) the step norm is traced here.
// Between two inner steps one launch applies the step and forms the next
// t_bar; the iterates then alternate between xh and stv_y (and t_bar
// between vtb and vtb2) so that it never reads what it writes, and the last
// step lands in xh.  With x aliasing xh the steps run unfused.  With xp the
// last step also writes R's padded copies of xh to xp / xTp, and the step norm
// partials are per 32 x 32 tile (tv_prep_tiles).
void enqueue_stv(sp_ctx* c, Scalars* sc, int K, const double* x, double* xh, bool snorm,
                 TraceDev tr, int32_t* trials_out, bool ride_snorm = false, double* xp = nullptr,
                 double* xTp = nullptr) {
    const GeomDev& G = c->G;
    const int n = G.rows * G.cols;
    const int* halt = &sc->halt;
    // partials of ||t_bar||^2 (first inner step / later ones) and of the trials
    const int nb0 = tv_blocks(G.rows, G.cols), nb1 = tv_grad_blocks(G.rows, G.cols), nt = tv_tpx_blocks(G.rows, G.cols);
    ProfScope ps(c, SP_PROF_TV);
    const bool fuse = K > 1 && x != xh && c->stv_y.bytes >= (size_t)n * sizeof(double) &&
                      c->vtb2.bytes >= (size_t)n * sizeof(float);
    const double* src = x;
    float* tb = dptr<float>(c->vtb);
    launch_tv_grad(c->stream, G.rows, G.cols, src, tb, dptr<double>(c->part_g), halt);
    for (int i = 0; i < K; ++i) {
        const int nb = i == 0 ? nb0 : nb1;
        launch_tv_trials(c->stream, G.rows, G.cols, src, tb, dptr<double>(c->part_g), nb, sc, 4,
                         dptr<double>(c->part_t), halt);
        launch_tv_decide(c->stream, G.rows, G.cols, src, tb, dptr<double>(c->part_g), nb,
                         dptr<double>(c->part_t), nt, 4, sc, tr, trials_out, halt);
        const bool last = i == K - 1;
        if (last && xp) {
            launch_tv_apply_prep(c->stream, G, src, xh, tb, sc, snorm ? x : nullptr, dptr<double>(c->part_s),
                                 xp, xTp, halt);
        } else if (last || !fuse) {
            launch_tv_apply(c->stream, n, src, xh, tb, sc, (last && snorm) ? x : nullptr,
                            dptr<double>(c->part_s), halt);
            src = xh;
            if (!last) launch_tv_grad(c->stream, G.rows, G.cols, src, tb, dptr<double>(c->part_g), halt, true);
        } else {
            // iterate i + 1 goes to xh when K - 1 - (i + 1) is even, so iterate K - 1 is in xh
            double* dst = (K - 2 - i) % 2 == 0 ? xh : dptr<double>(c->stv_y);
            float* tbn = tb == dptr<float>(c->vtb) ? dptr<float>(c->vtb2) : dptr<float>(c->vtb);
            launch_tv_apply_grad(c->stream, G.rows, G.cols, src, dst, tb, tbn, sc, dptr<double>(c->part_g),
                                 halt);
            src = dst;
            tb = tbn;
        }
    }
    if (snorm && !ride_snorm)
        launch_scalar(c->stream, OP_SNORM, sc, tr, dptr<double>(c->part_s),
                      xp ? tv_prep_tiles(G.rows, G.cols) : nb0, nullptr, 0);
}

// z = M g with the partial dots z^T dotv (dotv nullable).
// Sizes the learned preconditioner's workspace for npix pixels (training
// buffers only when `train`).
int lp_reserve(sp_ctx* c, sp_learned* net, size_t npix, bool train, int B, int H, int W) {
    int rc;
    const size_t a16 = npix * 16 * sizeof(float);
    if ((rc = ensure(c, net->ping, a16))) return rc;
    if ((rc = ensure(c, net->pong, a16))) return rc;
    if ((rc = ensure(c, net->spsg, 64 * sizeof(float)))) return rc;
    if (!train) return SP_OK;
    if (net->act.size() != (size_t)(3 * net->layers)) net->act.resize(3 * net->layers);
    for (auto& b : net->act)
        if ((rc = ensure(c, b, a16))) return rc;
    for (DevBuf* b : {&net->a0, &net->z, &net->e0})
        if ((rc = ensure(c, *b, npix * sizeof(float)))) return rc;
    if ((rc = ensure(c, net->partial, (size_t)lp_wgrad_blocks(B, H, W) * 2304 * sizeof(float)))) return rc;
    if ((rc = ensure(c, net->rtmp,
                     (size_t)lp_reduce_chunks(lp_wgrad_blocks(B, H, W)) * 2304 * sizeof(double))))
        return rc;
    if ((rc = ensure(c, net->lpart, (size_t)B * sizeof(double)))) return rc;
    if ((rc = ensure(c, net->gdpart, (size_t)lp_gd_blocks() * 16 * sizeof(double)))) return rc;
    return SP_OK;
}

// z = M u for B images of H x W (u, z device).  Gated by halt / run (nullable).
int lp_enqueue_apply(sp_ctx* c, sp_learned* net, int B, int H, int W, const float* u, float* z,
                     const int* halt, const int* run) {
    const size_t npix = (size_t)B * H * W;
    int rc = lp_reserve(c, net, npix, false, B, H, W);
    if (rc) return rc;
    hipStream_t st = c->stream;
    const float* th = dptr<float>(net->theta);
    float* sps = dptr<float>(net->spsg);
    const int L = net->layers;
    float* cur = dptr<float>(net->ping);
    float* nxt = dptr<float>(net->pong);
    lp_softplus(st, th + net->doff(), sps, sps + 16);
    lp_conv_in(st, B, H, W, u, nullptr, B, cur, th + net->woff(1), halt, run);
    if (L == 1) {
        lp_scale(st, (long)npix, cur, sps, nxt);
        std::swap(cur, nxt);
    }
    for (int l = 2; l <= L; ++l) {
        const bool last = l == L;   // b_L = softplus(d) * a_L is all the back path needs
        lp_conv_mid(st, false, B, H, W, cur, last ? nullptr : nxt, th + net->woff(l),
                    last ? sps : nullptr, last ? nxt : nullptr, halt, run);
        std::swap(cur, nxt);
    }
    for (int l = L; l >= 2; --l) {
        lp_conv_mid(st, true, B, H, W, cur, nxt, th + net->woff(l), nullptr, nullptr, halt, run);
        std::swap(cur, nxt);
    }
    lp_conv_out(st, B, H, W, cur, z, th + net->woff(1), halt, run);
    return SP_OK;
}

// z = M g (partial dots z^T dotv when dotv != NULL).  In the solver
// (solver = true) every launch honours the halt flag, and a learned M is
// checked (g^T z > 0 and finite) with the Fourier M as fallback.  With xp,
// R's padded copies of z (xp, xTp) are written too: by the Fourier M's last
// kernel, else by a prep launch.
int enqueue_precond(sp_ctx* c, const sp_precond* pc, const float* g, float* z, const float* dotv,
                    double* partials, int& nparts, bool solver, double* xp = nullptr,
                    double* xTp = nullptr) {
    const GeomDev& G = c->G;
    const int n = G.rows * G.cols;
    Scalars* sc = dptr<Scalars>(c->scal);
    const int* halt = solver ? &sc->halt : nullptr;
    if (pc->kind == SP_PRECOND_NONE) {
        if (g != z) launch_copy(c->stream, n, g, z, halt);
        if (dotv) launch_dot(c->stream, n, z, dotv, partials, halt);
        if (xp) launch_prep(c->stream, G, z, xp, xTp, halt);
        nparts = vec_blocks(n);
        return SP_OK;
    }
    FFTPlan F{};
    int rc = setup_fft(c, F);
    if (rc) return rc;
    if (pc->kind == SP_PRECOND_LEARNED) {
        sp_learned* net = const_cast<sp_learned*>(pc->net);
        ProfScope ps(c, SP_PROF_PRECOND);
        if ((rc = lp_enqueue_apply(c, net, 1, G.rows, G.cols, g, z, halt,
                                   solver ? &sc->gate_learned : nullptr)))
            return rc;
        if (solver) {
            double* pg = dptr<double>(c->part_misc);
            launch_dot(c->stream, n, g, z, pg, halt);
            TraceDev none{};
            launch_scalar(c->stream, OP_LCHECK, sc, none, pg, vec_blocks(n), nullptr, 0);
            launch_precond(c->stream, F, pc->mu, pc->rho, g, z, nullptr, nullptr, halt, &sc->gate_ramp);
        }
        if (dotv) launch_dot(c->stream, n, z, dotv, partials, halt);
        if (xp) launch_prep(c->stream, G, z, xp, xTp, halt);
        nparts = vec_blocks(n);
        return SP_OK;
    }
    {
        ProfScope ps(c, SP_PROF_PRECOND);
        launch_precond(c->stream, F, pc->mu, pc->rho, g, z, dotv, partials, halt, nullptr, xp ? &G : nullptr,
                       xp, xTp);
    }
    nparts = precond_dot_blocks(F);
    return SP_OK;
}


// ---- batched solve -----------------------------------------------------------

constexpr int XCDS = 8;              // workgroup w is dispatched to XCD w % 8
constexpr int TUNE_STAGES[] = {BS_PREP, BS_PROJECT, BS_BACKPROJECT, BS_ROWS, BS_TV, BS_VEC};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Virtual blocks of slice S in a stage (the single-slice grid of that stage).
int stage_blocks(const SliceDev& S, int stage) {
    const GeomDev& G = S.G;
    switch (stage) {
    case BS_PREP: return ((G.cols + 31) / 32) * ((G.rows + 31) / 32);
    case BS_PROJECT: return G.nwg * G.parts;
    case BS_PROJ_COMB: return G.parts > 1 ? project_comb_blocks(G) : 0;
    case BS_BACKPROJECT: return backproject_tiles(G, G.bp_px);
    case BS_ROWS: return (G.rows + 1) / 2;
    case BS_COLS: return S.F.P ? (S.F.SP + S.F.CB - 1) / S.F.CB : 0;
    case BS_TV: return tv_blocks(G.rows, G.cols);
    case BS_TVT: return tv_tpx_blocks(G.rows, G.cols);
    case BS_TVG: return tv_grad_blocks(G.rows, G.cols);
    case BS_VEC: return vec_blocks(S.n);
    case BS_PQ: return vec_blocks(std::max(S.n, S.m));
    default: return 1;
    }
}

// Relative cost of one item of the stage for slice S (load balance only).
double item_cost(const SliceDev& S, int stage) {
    const GeomDev& G = S.G;
    switch (stage) {
    case BS_PROJECT: return (double)std::max(G.rows, G.cols) / G.parts;
    case BS_PROJ_COMB: return (double)G.parts;
    case BS_BACKPROJECT: return (double)G.nA;
    case BS_ROWS:
    case BS_COLS: return S.F.P ? (double)S.F.P * S.F.logP : 0.0;
    case BS_VEC: return (double)S.n / std::max(1, vec_blocks(S.n));
    case BS_PQ: return (double)(S.n + S.m) / std::max(1, vec_blocks(std::max(S.n, S.m)));
    default: return 1.0;
    }
}

// Item tables of a stage.  Order 0: slices by decreasing work, each slice's
// blocks consecutive.  Order 1: slices assigned to the 8 XCDs by decreasing
// work to the least-loaded XCD, and entry 8 j + q holding the j-th item of XCD
// q's queue (shorter queues padded with ITEM_NONE), so a slice's blocks share
// one XCD's L2 under the round-robin dispatch of workgroups to XCDs.
void stage_items(const std::vector<SliceDev>& hs, int stage, std::vector<uint32_t>& o0,
                 std::vector<uint32_t>& o1) {
    const int n = (int)hs.size();
    std::vector<int> idx(n);
    std::vector<double> work(n);
    for (int s = 0; s < n; ++s) {
        idx[s] = s;
        work[s] = stage_blocks(hs[s], stage) * item_cost(hs[s], stage);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work[a] > work[b]; });
    o0.clear();
    for (int s : idx)
        for (int b = 0, nb = stage_blocks(hs[s], stage); b < nb; ++b)
            o0.push_back(((uint32_t)s << ITEM_SHIFT) | (uint32_t)b);
    std::vector<std::vector<uint32_t>> q(XCDS);
    std::vector<double> load(XCDS, 0.0);
    for (int s : idx) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += work[s];
        for (int b = 0, nb = stage_blocks(hs[s], stage); b < nb; ++b)
            q[x].push_back(((uint32_t)s << ITEM_SHIFT) | (uint32_t)b);
    }
    size_t len = 0;
    for (auto& v : q) len = std::max(len, v.size());
    o1.assign(len * XCDS, ITEM_NONE);
    for (int x = 0; x < XCDS; ++x)
        for (size_t j = 0; j < q[x].size(); ++j) o1[j * XCDS + x] = q[x][j];
}

ItemTable table(sp_ctx* c, int stage, int order = -1, int wpc = -1) {
    BatchState& B = *c->batch;
    if (order < 0) order = B.order[stage];
    if (wpc < 0) wpc = B.wpc[stage];
    ItemTable t;
    t.items = dptr<uint32_t>(B.items) + B.off[stage][order];
    t.n = B.count[stage][order];
    const long want = wpc > 0 ? (long)wpc * c->n_cu : (long)t.n;
    t.grid = (int)std::max(1L, std::min<long>(t.n, want));
    return t;
}

// (Re)builds the batch layout: geometry tables, one device arena holding every
// slice's padded copies, vectors, FFT scratch, twiddles and partials, and the
// item tables.  Kept while the geometries and preconditioner kind repeat.
int batch_setup(sp_ctx* c, int n, const sp_geometry* geoms, int kind) {
    const uint64_t epoch = g_shape_epoch.load();
    if (c->batch && c->batch->kind == kind && (int)c->batch->geoms.size() == n &&
        c->batch->epoch == epoch &&
        std::memcmp(c->batch->geoms.data(), geoms, sizeof(sp_geometry) * (size_t)n) == 0)
        return SP_OK;
    if (!c->batch) c->batch = new BatchState();
    BatchState& B = *c->batch;
    B.geoms.clear();     // the cache is valid only once the setup has completed
    B.kind = kind;
    B.tuned = false;
    for (int s = 0; s < BS_COUNT; ++s) B.order[s] = B.wpc[s] = 0;
    B.hs.assign(n, SliceDev{});
    B.nbmax = 1;
    B.lds_rows = B.lds_cols = 0;
    std::vector<std::vector<AngleDev>> tabs(n);
    // sizes
    struct Off {
        size_t ang, pwave, pord, xp, xTp, rpd, seg, dvec, vec, sq, S, tw, pf, pgp, pqq, ptg, ptt, pts;
    };
    std::vector<Off> off(n);
    size_t total = 0;
    int rc;
    for (int s = 0; s < n; ++s) {
        SliceDev& S = B.hs[s];
        if ((rc = build_geometry(c, &geoms[s], S.G, tabs[s]))) return fail(c, rc, "slice %d: %s", s, c->err);
        const GeomDev& G = S.G;
        B.nbmax = std::max(B.nbmax, G.nbmax);
        S.n = G.rows * G.cols;
        S.F = FFTPlan{};
        if (kind == SP_PRECOND_RAMP) {
            const int P = pad_size(G.rows, G.cols);
            if (P > 4096) return fail(c, SP_ERR_ARG, "slice %d: preconditioner supports up to 2048 pixels a side", s);
            S.F.P = P;
            while ((1 << S.F.logP) < P) ++S.F.logP;
            S.F.SP = P / 2 + 1;
            S.F.rows = G.rows;
            S.F.cols = G.cols;
            S.F.CB = std::max(1, 2048 / P);
            B.lds_rows = std::max(B.lds_rows, fft_lds_bytes(P, 1));
            B.lds_cols = std::max(B.lds_cols, fft_lds_bytes(P, S.F.CB));
        }
        S.m = G.nA * G.nB;
        S.nf = project_blocks(G);
        S.ngp = vec_blocks(S.n);
        S.nqq = vec_blocks(S.m);
        S.ntv = tv_blocks(G.rows, G.cols);
        S.ntt = tv_tpx_blocks(G.rows, G.cols);
        S.ntg = tv_grad_blocks(G.rows, G.cols);
        S.nsn = tv_prep_tiles(G.rows, G.cols);
        Off& o = off[s];
        auto take = [&](size_t bytes) {
            const size_t at = total;
            total += align256(bytes);
            return at;
        };
        o.ang = take(tabs[s].size() * sizeof(AngleDev));
        o.pwave = take((size_t)G.nwaves * sizeof(WaveDev));
        o.pord = take((size_t)G.nwg * sizeof(int32_t));
        o.xp = take((size_t)G.rows * G.pitchX * 8);
        o.xTp = take((size_t)G.cols * G.pitchXT * 8);
        o.rpd = take((size_t)G.nA * G.pitchB * 8);
        o.seg = take(G.parts > 1 ? (size_t)G.parts * G.nA * G.nB * 8 : 0);
        o.dvec = take((size_t)S.n * 8 * 3);  // x, x_half, p (float64)
        o.vec = take((size_t)S.n * 4 * 3);   // g, z, t_bar
        o.sq = take((size_t)S.m * 8 * 2);    // q = R p, w = R z
        o.S = kind == SP_PRECOND_RAMP ? take((size_t)G.rows * S.F.SP * sizeof(double2)) : 0;
        o.tw = kind == SP_PRECOND_RAMP ? take((size_t)(S.F.P / 2) * sizeof(double2)) : 0;
        o.pf = take((size_t)S.nf * 8);
        o.pgp = take((size_t)S.ngp * 8);
        o.pqq = take((size_t)S.nqq * 8);
        o.ptg = take((size_t)S.ntv * 8);
        o.ptt = take((size_t)S.ntv * 9 * 8);
        o.pts = take((size_t)std::max(S.ntv, S.nsn) * 8);
    }
    if (B.lds_cols > 65536) return fail(c, SP_ERR_ARG, "FFT column tile exceeds the LDS");
    // one R^T tile shape for the whole batch: four pixels per lane when the
    // batch's 4-pixel tiles still fill half the wave slots (the sums do not
    // depend on it, so batched and single solves stay bitwise equal)
    {
        long waves4 = 0;
        for (const SliceDev& S : B.hs) waves4 += (long)backproject_tiles(S.G, 4) * 4;
        B.bp_px = waves4 >= (long)c->n_cu * 16 ? 4 : 2;
        // tuned shapes that agree for every slice take precedence
        int tpx = 0;
        bool all = true;
        for (int s = 0; s < n && all; ++s) {
            int tp, tx;
            if (!shape_lookup(geoms[s], tp, tx) || (tpx && tx != tpx)) all = false;
            else tpx = tx;
        }
        if (all && tpx) B.bp_px = tpx;
        for (SliceDev& S : B.hs) S.G.bp_px = B.bp_px;
    }
    // a fresh zero-filled arena: the pads of the padded copies must be zero
    release(B.arena);
    if ((rc = ensure(c, B.arena, total))) return rc;
    if ((rc = ensure(c, B.scal, sizeof(Scalars) * (size_t)n))) return rc;
    if ((rc = ensure(c, B.sl, sizeof(SliceDev) * (size_t)n))) return rc;
    char* base = dptr<char>(B.arena);
    std::vector<double2> tw;
    for (int s = 0; s < n; ++s) {
        SliceDev& S = B.hs[s];
        const Off& o = off[s];
        S.ang = reinterpret_cast<const AngleDev*>(base + o.ang);
        std::vector<WaveDev> waves((size_t)S.G.nwaves);
        project_waves(S.G, waves.data());
        S.pwave = reinterpret_cast<const WaveDev*>(base + o.pwave);
        HIP_TRY(c, hipMemcpyAsync(base + o.pwave, waves.data(), waves.size() * sizeof(WaveDev),
                                  hipMemcpyHostToDevice, c->stream));
        const std::vector<int32_t> ord = project_order(S.G, tabs[s].data(), waves.data(), c->n_cu);
        S.pord = reinterpret_cast<const int*>(base + o.pord);
        HIP_TRY(c, hipMemcpyAsync(base + o.pord, ord.data(), ord.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        S.xp = reinterpret_cast<double*>(base + o.xp);
        S.xTp = reinterpret_cast<double*>(base + o.xTp);
        S.rpd = reinterpret_cast<double*>(base + o.rpd);
        S.seg = S.G.parts > 1 ? reinterpret_cast<double*>(base + o.seg) : nullptr;
        double* dv = reinterpret_cast<double*>(base + o.dvec);
        S.x = dv;
        S.xh = dv + (size_t)S.n;
        S.p = dv + 2 * (size_t)S.n;
        float* v = reinterpret_cast<float*>(base + o.vec);
        S.g = v;
        S.z = v + (size_t)S.n;
        S.tb = v + 2 * (size_t)S.n;
        S.q = reinterpret_cast<double*>(base + o.sq);
        S.w = S.q + (size_t)S.m;
        if (kind == SP_PRECOND_RAMP) {
            S.F.S = reinterpret_cast<double2*>(base + o.S);
            S.F.tw = reinterpret_cast<const double2*>(base + o.tw);
            tw.resize(S.F.P / 2);
            for (int k = 0; k < S.F.P / 2; ++k) {
                const double ang = -2.0 * M_PI * (double)k / (double)S.F.P;
                tw[k] = make_double2(std::cos(ang), std::sin(ang));
            }
            HIP_TRY(c, hipMemcpyAsync(base + o.tw, tw.data(), tw.size() * sizeof(double2),
                                      hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
        }
        S.pf = reinterpret_cast<double*>(base + o.pf);
        S.pgp = reinterpret_cast<double*>(base + o.pgp);
        S.pqq = reinterpret_cast<double*>(base + o.pqq);
        S.ptg = reinterpret_cast<double*>(base + o.ptg);
        S.ptt = reinterpret_cast<double*>(base + o.ptt);
        S.pts = reinterpret_cast<double*>(base + o.pts);
        S.sc = dptr<Scalars>(B.scal) + s;
        HIP_TRY(c, hipMemcpyAsync(base + o.ang, tabs[s].data(), tabs[s].size() * sizeof(AngleDev),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));   // host table must outlive the copy
    }
    for (int s = 0; s < n; ++s)
        for (int st = 0; st < BS_COUNT; ++st)
            if (stage_blocks(B.hs[s], st) > (int)ITEM_MASK) {
                B.geoms.clear();
                return fail(c, SP_ERR_ARG, "slice %d: too many work items for a batch", s);
            }
    // item tables
    std::vector<uint32_t> all, o0, o1;
    for (int st = 0; st < BS_COUNT; ++st) {
        if (st == BS_COLS && kind != SP_PRECOND_RAMP) continue;
        stage_items(B.hs, st, o0, o1);
        B.off[st][0] = all.size();
        B.count[st][0] = (int)o0.size();
        all.insert(all.end(), o0.begin(), o0.end());
        B.off[st][1] = all.size();
        B.count[st][1] = (int)o1.size();
        all.insert(all.end(), o1.begin(), o1.end());
    }
    if ((rc = ensure(c, B.items, all.size() * sizeof(uint32_t)))) return rc;
    HIP_TRY(c, hipMemcpyAsync(B.items.ptr, all.data(), all.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    B.geoms.assign(geoms, geoms + n);
    B.epoch = epoch;
    return SP_OK;
}

// One batched stage group, as timed by the tuner and run by the solver.
void batch_stage(sp_ctx* c, int stage, int order, int wpc, double mu, double rho) {
    BatchState& B = *c->batch;
    const SliceDev* sl = dptr<SliceDev>(B.sl);
    hipStream_t st = c->stream;
    const ItemTable t = table(c, stage, order, wpc);
    switch (stage) {
    case BS_PREP: launch_prep_b(st, sl, t, BV_XH); break;
    case BS_PROJECT: launch_project_b(st, sl, t, table(c, BS_PROJ_COMB, order, 0), true); break;
    case BS_BACKPROJECT: launch_backproject_b(st, sl, t, B.nbmax, B.bp_px); break;
    case BS_ROWS:
        launch_precond_b(st, sl, t, table(c, BS_COLS, order, wpc), B.lds_rows, B.lds_cols, mu, rho);
        break;
    case BS_TV:
        launch_tv_grad_b(st, sl, t, BV_X);
        launch_tv_trials_b(st, sl, table(c, BS_TVT, order, wpc), BV_X);
        break;
    case BS_VEC: launch_update_x_b(st, sl, t); break;
    default: break;
    }
}

// Times every (order, grid) choice of the heavy stages and keeps the fastest.
// Runs on the live buffers before the initial steps, which overwrite all that
// the timed kernels write.
int batch_tune(sp_ctx* c, double mu, double rho) {
    BatchState& B = *c->batch;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    const int grids[] = {0, 2, 4, 8};
    for (int stage : TUNE_STAGES) {
        if (stage == BS_ROWS && B.kind != SP_PRECOND_RAMP) continue;
        float best = 1e30f;
        for (int order = 0; order < 2; ++order)
            for (int wpc : grids) {
                batch_stage(c, stage, order, wpc, mu, rho);   // warm
                float tmin = 1e30f;
                for (int r = 0; r < 3; ++r) {
                    (void)hipEventRecord(e0, c->stream);
                    batch_stage(c, stage, order, wpc, mu, rho);
                    (void)hipEventRecord(e1, c->stream);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.0f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    tmin = std::min(tmin, ms);
                }
                if (tmin < best * 0.98f) {
                    best = tmin;
                    B.order[stage] = order;
                    B.wpc[stage] = wpc;
                }
            }
        if (stage == BS_ROWS) {
            B.order[BS_COLS] = B.order[BS_ROWS];
            B.wpc[BS_COLS] = B.wpc[BS_ROWS];
        }
        if (stage == BS_TV) {   // the trials launch is timed with the TV stage
            B.order[BS_TVT] = B.order[BS_TVG] = B.order[BS_TV];
            B.wpc[BS_TVT] = B.wpc[BS_TVG] = B.wpc[BS_TV];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B.tuned = true;
    return check_launch(c);
}

// Preconditioner stage of the batched solver: z = M g.
void batch_precond(sp_ctx* c, double mu, double rho) {
    BatchState& B = *c->batch;
    const SliceDev* sl = dptr<SliceDev>(B.sl);
    if (B.kind == SP_PRECOND_RAMP)
        launch_precond_b(c->stream, sl, table(c, BS_ROWS), table(c, BS_COLS), B.lds_rows, B.lds_cols,
                         mu, rho);
    else
        launch_copy_gz_b(c->stream, sl, table(c, BS_VEC));
}
}  // namespace

// ============================================================================
extern "C" {

const char* sp_version(void) { return "suppcg-gfx950 0.1"; }

int sp_ctx_create(int device, void* hip_stream, sp_ctx** out) {
    if (!out) return SP_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return SP_ERR_HIP;
    if (device < 0 || device >= count) return SP_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return SP_ERR_HIP;
    sp_ctx* c = new sp_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        c->n_cu < 1)
        c->n_cu = 256;
    c->na_tab.resize(NOALLOC_MAX_ANGLES);
    if (hipEventCreateWithFlags(&c->na_ev, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return SP_ERR_HIP;
    }
    void* scr = nullptr;
    (void)noalloc_scratch(device, &scr);   // per-device lookup of the static scratch, once
    *out = c;
    return SP_OK;
}

int sp_ctx_destroy(sp_ctx* c) {
    if (!c) return SP_ERR_ARG;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    (void)drain_pending(c);
    for (DevBuf* b : {&c->ang, &c->pwave, &c->xp, &c->xTp, &c->yp, &c->ypd, &c->seg, &c->pord, &c->blob_tab, &c->tw, &c->S, &c->vx, &c->vxh, &c->vp, &c->vq, &c->vw, &c->ox, &c->oxh, &c->oscal,
                      &c->vg, &c->vz, &c->vtb, &c->vtb2, &c->stv_y, &c->vtmp, &c->part_f, &c->part_zh, &c->part_gp,
                      &c->part_qq, &c->part_g, &c->part_t, &c->part_s, &c->part_misc, &c->part_se, &c->stored_xT, &c->art_u, &c->art_nrm, &c->art_sum, &c->scal,
                      &c->trace_d, &c->replay_d, &c->trials_tmp})
        release(*b);
    if (c->own) (void)hipStreamDestroy(c->own);
    for (hipEvent_t e : c->own_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->na_ev) (void)hipEventDestroy(c->na_ev);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->batch) {
        for (DevBuf* b : {&c->batch->arena, &c->batch->sl, &c->batch->items, &c->batch->scal,
                          &c->batch->trace_d})
            release(*b);
        delete c->batch;
    }
    delete c;
    return SP_OK;
}

int sp_ctx_set_stream(sp_ctx* c, void* hip_stream) {
    if (!c) return SP_ERR_ARG;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return SP_OK;
}

const char* sp_last_error(const sp_ctx* c) { return c ? c->err : "null context"; }
const char* sp_ctx_last_error(const sp_ctx* c) { return sp_last_error(c); }

int sp_profile_enable(sp_ctx* c, int on) {
    if (!c) return SP_ERR_ARG;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->prof = on != 0;
    c->prof_recs.clear();
    c->ev_used = 0;
    return SP_OK;
}

int sp_lp_create(sp_ctx* c, int32_t layers, int32_t channels, sp_learned** out) {
    if (!c || !out) return SP_ERR_ARG;
    *out = nullptr;
    if (channels != 16) return fail(c, SP_ERR_ARG, "only 16 channels are supported");
    if (layers < 1 || layers > 8) return fail(c, SP_ERR_ARG, "layers must be in [1, 8]");
    HIP_TRY(c, hipSetDevice(c->device));
    sp_learned* net = new sp_learned();
    net->device = c->device;
    net->layers = layers;
    net->channels = channels;
    net->nparams = 144 + (layers - 1) * 2304 + 16;
    int rc;
    for (DevBuf* b : {&net->theta, &net->adam_m, &net->adam_v})
        if ((rc = ensure(c, *b, (size_t)net->nparams * sizeof(float)))) {
            delete net;
            return rc;
        }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *out = net;
    return SP_OK;
}

int sp_lp_destroy(sp_learned* net) {
    if (!net) return SP_ERR_ARG;
    (void)hipSetDevice(net->device);
    (void)hipDeviceSynchronize();
    for (DevBuf* b : {&net->theta, &net->adam_m, &net->adam_v, &net->spsg, &net->a0, &net->z,
                      &net->e0, &net->ping, &net->pong, &net->partial, &net->rtmp, &net->lpart,
                      &net->gdpart})
        release(*b);
    for (auto& b : net->act) release(b);
    delete net;
    return SP_OK;
}

int64_t sp_lp_num_params(const sp_learned* net) { return net ? net->nparams : -1; }

int sp_lp_set_params(sp_ctx* c, sp_learned* net, const float* theta, int64_t count) {
    if (!c) return SP_ERR_ARG;
    if (!net || !theta || count != net->nparams)
        return fail(c, SP_ERR_ARG, "sp_lp_set_params: need num_params host values");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(net->theta.ptr, theta, (size_t)count * sizeof(float),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(net->adam_m.ptr, 0, net->adam_m.bytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(net->adam_v.ptr, 0, net->adam_v.bytes, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SP_OK;
}

int sp_lp_get_params(sp_ctx* c, const sp_learned* net, float* theta, int64_t count) {
    if (!c) return SP_ERR_ARG;
    if (!net || !theta || count != net->nparams)
        return fail(c, SP_ERR_ARG, "sp_lp_get_params: need num_params host values");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(theta, net->theta.ptr, (size_t)count * sizeof(float),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SP_OK;
}

int sp_lp_set_weights(sp_ctx* c, sp_learned* net, const float* w, int64_t count) {
    return sp_lp_set_params(c, net, w, count);
}

int sp_lp_get_weights(sp_ctx* c, const sp_learned* net, float* w, int64_t count) {
    return sp_lp_get_params(c, net, w, count);
}

int sp_lp_apply(sp_ctx* c, sp_learned* net, int32_t batch, int32_t rows, int32_t cols,
                const float* u, float* z) {
    if (!c) return SP_ERR_ARG;
    if (!net || !u || !z) return fail(c, SP_ERR_ARG, "sp_lp_apply: null argument");
    if (batch < 1 || rows < 1 || cols < 1 || (double)batch * rows * cols > 1.0e9)
        return fail(c, SP_ERR_ARG, "sp_lp_apply: bad sizes");
    if (net->device != c->device) return fail(c, SP_ERR_ARG, "network lives on another GPU");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = lp_enqueue_apply(c, net, batch, rows, cols, u, z, nullptr, nullptr);
    if (rc) return rc;
    return check_launch(c);
}

int sp_lp_loss_grad(sp_ctx* c, sp_learned* net, int32_t rows, int32_t cols, const float* Av,
                    const float* v, int32_t nprobe, const int32_t* idx, int32_t batch,
                    int32_t margin, double* loss, float* grad) {
    if (!c) return SP_ERR_ARG;
    if (!net || !Av || !v || !idx || !loss || !grad)
        return fail(c, SP_ERR_ARG, "sp_lp_loss_grad: null argument");
    if (rows < 1 || cols < 1 || nprobe < 1 || batch < 1 || (double)batch * rows * cols > 2.0e8)
        return fail(c, SP_ERR_ARG, "sp_lp_loss_grad: bad sizes");
    if (margin < 0 || 2 * margin >= std::min(rows, cols))
        return fail(c, SP_ERR_ARG, "sp_lp_loss_grad: margin must leave interior pixels");
    if (net->device != c->device) return fail(c, SP_ERR_ARG, "network lives on another GPU");
    HIP_TRY(c, hipSetDevice(c->device));
    const int B = batch, H = rows, W = cols, L = net->layers;
    const size_t npix = (size_t)B * H * W;
    int rc = lp_reserve(c, net, npix, true, B, H, W);
    if (rc) return rc;
    hipStream_t st = c->stream;
    const float* th = dptr<float>(net->theta);
    float* sps = dptr<float>(net->spsg);
    float* sg = sps + 16;
    auto A = [&](int l) { return l == 0 ? dptr<float>(net->a0) : dptr<float>(net->act[l - 1]); };
    auto Bb = [&](int l) { return dptr<float>(net->act[L + l - 1]); };
    auto E = [&](int l) { return l == 0 ? dptr<float>(net->e0) : dptr<float>(net->act[2 * L + l - 1]); };
    float* Z = dptr<float>(net->z);
    float* part = dptr<float>(net->partial);
    double* rtmp = dptr<double>(net->rtmp);
    const int nwb = lp_wgrad_blocks(B, H, W);
    lp_softplus(st, th + net->doff(), sps, sg);
    // forward chain a_l = C_l a_{l-1}, b_L = softplus(d) a_L, back chain b_{l-1} = C_l^T b_l
    lp_gather(st, B, H * W, Av, idx, nprobe, A(0));
    lp_conv_in(st, B, H, W, A(0), nullptr, B, A(1), th + net->woff(1), nullptr, nullptr);
    for (int l = 2; l <= L; ++l)
        lp_conv_mid(st, false, B, H, W, A(l - 1), A(l), th + net->woff(l),
                    l == L ? sps : nullptr, l == L ? Bb(L) : nullptr, nullptr, nullptr);
    if (L == 1) lp_scale(st, (long)npix, A(1), sps, Bb(1));
    for (int l = L; l >= 2; --l)
        lp_conv_mid(st, true, B, H, W, Bb(l), Bb(l - 1), th + net->woff(l), nullptr, nullptr, nullptr, nullptr);
    lp_conv_out(st, B, H, W, Bb(1), Z, th + net->woff(1), nullptr, nullptr);
    // loss and e_0 = d loss / dz
    lp_loss(st, B, H, W, margin, Z, v, idx, nprobe, E(0), dptr<double>(net->lpart));
    launch_reduce(st, dptr<double>(net->lpart), B, loss);
    // e_l = C_l e_{l-1}; the back chain contributes wgrad(b_l, e_{l-1}) to W_l
    lp_conv_in(st, B, H, W, E(0), nullptr, B, E(1), th + net->woff(1), nullptr, nullptr);
    for (int l = 2; l <= L; ++l)
        lp_conv_mid(st, false, B, H, W, E(l - 1), E(l), th + net->woff(l), nullptr, nullptr, nullptr, nullptr);
    for (int l = 1; l <= L; ++l) {
        const int fi = l == 1 ? 1 : 16;
        lp_wgrad(st, fi, B, H, W, Bb(l), E(l - 1), part);
        lp_reduce(st, nwb, 16 * fi * 9, part, false, grad + net->woff(l), rtmp);
    }
    // d: sigmoid(d) * sum e_L a_L; then f_L = softplus(d) e_L (into b_L's buffer)
    lp_gd(st, (long)npix, E(L), A(L), dptr<double>(net->gdpart), sg, grad + net->doff());
    lp_scale(st, (long)npix, E(L), sps, Bb(L));
    // forward chain: wgrad(f_l, a_{l-1}) into W_l, f_{l-1} = C_l^T f_l
    for (int l = L; l >= 1; --l) {
        const int fi = l == 1 ? 1 : 16;
        lp_wgrad(st, fi, B, H, W, Bb(l), A(l - 1), part);
        lp_reduce(st, nwb, 16 * fi * 9, part, true, grad + net->woff(l), rtmp);
        if (l >= 2)
            lp_conv_mid(st, true, B, H, W, Bb(l), Bb(l - 1), th + net->woff(l), nullptr, nullptr, nullptr, nullptr);
    }
    return check_launch(c);
}

int sp_lp_adam_step(sp_ctx* c, sp_learned* net, const float* grad, double lr, double beta1,
                    double beta2, double eps, int32_t step) {
    if (!c) return SP_ERR_ARG;
    if (!net || !grad || step < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
        !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(c, SP_ERR_ARG, "sp_lp_adam_step: bad argument");
    HIP_TRY(c, hipSetDevice(c->device));
    lp_adam(c->stream, net->nparams, dptr<float>(net->theta), dptr<float>(net->adam_m),
            dptr<float>(net->adam_v), grad, lr, beta1, beta2, eps, step);
    return check_launch(c);
}

int sp_profile_read(sp_ctx* c, int kind, double* total_ms, int32_t* count) {
    if (!c) return SP_ERR_ARG;
    if (kind < 0 || kind >= SP_PROF_KINDS || !total_ms || !count)
        return fail(c, SP_ERR_ARG, "sp_profile_read: bad kind or null output");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    int32_t n = 0;
    for (const auto& r : c->prof_recs) {
        if (r.kind != kind) continue;
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_pool[r.e0], c->ev_pool[r.e1]));
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *count = n;
    return SP_OK;
}

int sp_project(sp_ctx* c, const sp_geometry* g, const float* x, float* y) {
    if (!c) return SP_ERR_ARG;
    if (!x || !y) return fail(c, SP_ERR_ARG, "x and y must be device pointers");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    const GeomDev& G = c->G;
    launch_prep(c->stream, G, x, dptr<double>(c->xp), dptr<double>(c->xTp), nullptr);
    {
        ProfScope ps(c, SP_PROF_PROJECT);
        launch_project(c->stream, G, dptr<AngleDev>(c->ang), dptr<WaveDev>(c->pwave),
                       dptr<double>(c->xp), dptr<double>(c->xTp),
                       nullptr, y, G.nB, nullptr, nullptr, nullptr, dptr<double>(c->seg),
                       dptr<int>(c->pord), nullptr);
    }
    return check_launch(c);
}

int sp_backproject(sp_ctx* c, const sp_geometry* g, const float* y, float* x) {
    if (!c) return SP_ERR_ARG;
    if (!x || !y) return fail(c, SP_ERR_ARG, "x and y must be device pointers");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    const GeomDev& G = c->G;
    launch_pad_sino(c->stream, G, dptr<AngleDev>(c->ang), y, dptr<float>(c->yp));
    {
        ProfScope ps(c, SP_PROF_BACKPROJECT);
        launch_backproject(c->stream, G, dptr<AngleDev>(c->ang), dptr<float>(c->yp), x, nullptr,
                           nullptr, nullptr);
    }
    return check_launch(c);
}

int sp_backproject_noalloc(sp_ctx* c, const sp_geometry* g, const float* y, float* x) {
    if (!c) return SP_ERR_ARG;
    if (!x || !y) return fail(c, SP_ERR_ARG, "x and y must be device pointers");
    int rc = validate_geometry(c, g);
    if (rc) return rc;
    if (g->n_angles > NOALLOC_MAX_ANGLES)
        return fail(c, SP_ERR_ARG, "sp_backproject_noalloc: at most %d angles (got %d)",
                    NOALLOC_MAX_ANGLES, g->n_angles);
    // scratch layout: angle table | padded sinogram
    const size_t pitchB = (size_t)g->n_bins + 2 * PAD;
    const size_t off_yp = align256((size_t)g->n_angles * sizeof(AngleDev));
    const size_t need = off_yp + (size_t)g->n_angles * pitchB * sizeof(float);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(c, SP_ERR_ARG,
                    "sp_backproject_noalloc: this geometry needs %zu bytes of scratch, the static "
                    "array holds %zu", need, NOALLOC_SCRATCH_BYTES);
    HIP_TRY(c, hipSetDevice(c->device));
    void* scr = nullptr;
    hipError_t es = noalloc_scratch(c->device, &scr);
    if (es != hipSuccess || !scr)
        return fail(c, SP_ERR_HIP, "hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(es));
    HIP_TRY(c, hipEventSynchronize(c->na_ev));   // the previous call's uploads have read the staging
    GeomDev G{};
    if ((rc = build_geometry_into(c, g, G, c->na_tab.data()))) return rc;
    char* base = static_cast<char*>(scr);
    AngleDev* ang = reinterpret_cast<AngleDev*>(base);
    float* yp = reinterpret_cast<float*>(base + off_yp);
    HIP_TRY(c, hipMemcpyAsync(ang, c->na_tab.data(), (size_t)g->n_angles * sizeof(AngleDev),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipEventRecord(c->na_ev, c->stream));
    launch_pad_sino(c->stream, G, ang, y, yp);   // every entry of the rows, pads included
    launch_backproject(c->stream, G, ang, yp, x, nullptr, nullptr, nullptr);
    return check_launch(c);
}

// ---- launch-shape tuning ------------------------------------------------------------

int sp_tune_shapes(sp_ctx* c, const sp_geometry* g, int32_t* parts_out, int32_t* px_out, double* ms) {
    if (!c) return SP_ERR_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = drain_pending(c);
    if (rc) return rc;
    if ((rc = setup_geometry(c, g))) return rc;
    const int def_parts = c->G.parts, def_px = c->G.bp_px;
    int old_parts = 0, old_px = 0;
    const bool had = shape_lookup(*g, old_parts, old_px);
    DevBuf xb, yb;
    struct Tmp {
        DevBuf *a, *b;
        ~Tmp() {
            release(*a);
            release(*b);
        }
    } tmp{&xb, &yb};
    const size_t n = (size_t)g->rows * g->cols, m = (size_t)g->n_angles * g->n_bins;
    if ((rc = ensure(c, xb, n * 4)) || (rc = ensure(c, yb, m * 4))) return rc;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, SP_ERR_HIP, "hipEventCreate failed");
    }
    // fastest of 5 calls after a warm-up (data values do not change the work)
    auto time_call = [&](bool back, float& best) -> int {
        best = 1e30f;
        for (int r = 0; r < 6; ++r) {
            (void)hipEventRecord(e0, c->stream);
            const int q = back ? sp_backproject(c, g, dptr<float>(yb), dptr<float>(xb))
                               : sp_project(c, g, dptr<float>(xb), dptr<float>(yb));
            if (q) return q;
            (void)hipEventRecord(e1, c->stream);
            if (hipEventSynchronize(e1) != hipSuccess) return fail(c, SP_ERR_HIP, "timing the launch shapes failed");
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (r > 0) best = std::min(best, t);
        }
        return SP_OK;
    };
    const int parts_c[4] = {1, 2, 4, 8}, px_c[2] = {2, 4};
    float tr[4], tb[2];
    int best_parts = def_parts, best_px = def_px;
    rc = SP_OK;
    for (int i = 0; i < 4 && !rc; ++i) {
        shape_store(*g, parts_c[i], def_px);
        rc = time_call(false, tr[i]);
    }
    if (!rc) {
        // the default wins ties within 2%
        float tdef = 1e30f;
        for (int i = 0; i < 4; ++i)
            if (parts_c[i] == def_parts) tdef = tr[i];
        float best = tdef;
        for (int i = 0; i < 4; ++i)
            if (tr[i] < 0.98f * best) best = tr[i], best_parts = parts_c[i];
    }
    for (int i = 0; i < 2 && !rc; ++i) {
        shape_store(*g, best_parts, px_c[i]);
        rc = time_call(true, tb[i]);
    }
    if (!rc) {
        float tdef = def_px == 4 ? tb[1] : tb[0], best = tdef;
        for (int i = 0; i < 2; ++i)
            if (tb[i] < 0.98f * best) best = tb[i], best_px = px_c[i];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {   // leave the cache as it was
        if (had) shape_store(*g, old_parts, old_px);
        else shape_store(*g, 0, 0);
        return rc;
    }
    shape_store(*g, best_parts, best_px);
    if (parts_out) *parts_out = best_parts;
    if (px_out) *px_out = best_px;
    if (ms) {
        for (int i = 0; i < 4; ++i) ms[i] = tr[i];
        for (int i = 0; i < 2; ++i) ms[4 + i] = tb[i];
    }
    return SP_OK;
}

int sp_tuning_set(const sp_geometry* g, int32_t parts, int32_t px) {
    if (!g) return SP_ERR_ARG;
    if (parts == 0 && px == 0) {
        shape_store(*g, 0, 0);
        return SP_OK;
    }
    if (parts < 1 || parts > 8 || (px != 2 && px != 4)) return SP_ERR_ARG;
    char msg[128];
    GeomDev G{};
    std::vector<AngleDev> tab((size_t)std::max(g->n_angles, 1));
    if (g->n_angles < 1 || sp::build_geometry_into(g, 256, G, tab.data(), msg, sizeof msg) != SP_OK)
        return SP_ERR_ARG;
    shape_store(*g, parts, px);
    return SP_OK;
}

int sp_tuning_list(sp_geometry* geoms, int32_t* parts, int32_t* px, int32_t cap, int32_t* count) {
    if (!count || cap < 0) return SP_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_shape_mu);
    *count = (int32_t)g_shapes.size();
    for (int32_t i = 0; i < cap && i < (int32_t)g_shapes.size(); ++i) {
        if (geoms) geoms[i] = g_shapes[(size_t)i].g;
        if (parts) parts[i] = g_shapes[(size_t)i].parts;
        if (px) px[i] = g_shapes[(size_t)i].px;
    }
    return SP_OK;
}

int sp_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shapes.clear();
    ++g_shape_epoch;
    return SP_OK;
}

int sp_residual(sp_ctx* c, const sp_geometry* g, const float* x, const float* b, float* r, double* f) {
    if (!c) return SP_ERR_ARG;
    if (!x || !b || !f) return fail(c, SP_ERR_ARG, "x, b and f must be device pointers");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    if ((rc = ensure_partials(c))) return rc;
    const GeomDev& G = c->G;
    launch_prep(c->stream, G, x, dptr<double>(c->xp), dptr<double>(c->xTp), nullptr);
    launch_project(c->stream, G, dptr<AngleDev>(c->ang), dptr<WaveDev>(c->pwave), dptr<double>(c->xp),
                   dptr<double>(c->xTp), b, r,
                   G.nB, nullptr, nullptr, dptr<double>(c->part_f), dptr<double>(c->seg),
                   dptr<int>(c->pord), nullptr);
    launch_reduce(c->stream, dptr<double>(c->part_f), project_blocks(G), f);
    return check_launch(c);
}

int sp_gradient(sp_ctx* c, const sp_geometry* g, const float* x, const float* b, float* grad,
                double* f) {
    if (!c) return SP_ERR_ARG;
    if (!x || !b || !grad) return fail(c, SP_ERR_ARG, "x, b and grad must be device pointers");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    if ((rc = ensure_partials(c))) return rc;
    const GeomDev& G = c->G;
    // the solvers' path: the residual stays float64 between R and R^T
    launch_prep(c->stream, G, x, dptr<double>(c->xp), dptr<double>(c->xTp), nullptr);
    launch_project(c->stream, G, dptr<AngleDev>(c->ang), dptr<WaveDev>(c->pwave), dptr<double>(c->xp),
                   dptr<double>(c->xTp), b,
                   nullptr, 0, nullptr, dptr<double>(c->ypd), dptr<double>(c->part_f),
                   dptr<double>(c->seg), dptr<int>(c->pord), nullptr);
    launch_backproject(c->stream, G, dptr<AngleDev>(c->ang), dptr<double>(c->ypd),
                       grad, nullptr, nullptr, nullptr);
    if (f) launch_reduce(c->stream, dptr<double>(c->part_f), project_blocks(G), f);
    return check_launch(c);
}

int sp_precond_apply(sp_ctx* c, const sp_geometry* g, const sp_precond* pc, const float* gin, float* z) {
    if (!c) return SP_ERR_ARG;
    if (!gin || !z) return fail(c, SP_ERR_ARG, "g and z must be device pointers");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    if ((rc = check_precond(c, pc))) return rc;
    if ((rc = ensure_partials(c))) return rc;
    int np = 0;
    if ((rc = enqueue_precond(c, pc, gin, z, nullptr, nullptr, np, false))) return rc;
    return check_launch(c);
}

int sp_tv(sp_ctx* c, const sp_geometry* g, const float* x, double* tv) {
    if (!c) return SP_ERR_ARG;
    if (!x || !tv) return fail(c, SP_ERR_ARG, "x and tv must be device pointers");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    if ((rc = ensure_partials(c))) return rc;
    if ((rc = ensure_op_vectors(c, (size_t)g->rows * g->cols))) return rc;
    launch_widen(c->stream, g->rows * g->cols, x, dptr<double>(c->ox));
    launch_tv_value(c->stream, g->rows, g->cols, dptr<double>(c->ox), dptr<double>(c->part_g), nullptr);
    launch_reduce(c->stream, dptr<double>(c->part_g), tv_blocks(g->rows, g->cols), tv);
    return check_launch(c);
}

int sp_selective_error(sp_ctx* c, const sp_geometry* g, const float* x, const float* ref,
                       const double* axes, double C, double* se) {
    if (!c) return SP_ERR_ARG;
    if (!x || !ref || !se || !axes) return fail(c, SP_ERR_ARG, "x, ref, axes and se are required");
    if (!(axes[0] > 0.0) || !(axes[1] > 0.0) || !std::isfinite(axes[0]) || !std::isfinite(axes[1]))
        return fail(c, SP_ERR_ARG, "ellipse semi-axes must be positive and finite");
    if (!std::isfinite(C)) return fail(c, SP_ERR_ARG, "C must be finite");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    if ((rc = ensure_partials(c))) return rc;
    launch_se(c->stream, g->rows, g->cols, g->pixel, axes[0], axes[1], x, ref, C,
              dptr<double>(c->part_se), se);
    return check_launch(c);
}

int sp_tv_grad(sp_ctx* c, const sp_geometry* g, const float* x, float* tbar, double* norm2) {
    if (!c) return SP_ERR_ARG;
    if (!x || !tbar) return fail(c, SP_ERR_ARG, "x and tbar must be device pointers");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    if ((rc = ensure_partials(c))) return rc;
    if ((rc = ensure_op_vectors(c, (size_t)g->rows * g->cols))) return rc;
    launch_widen(c->stream, g->rows * g->cols, x, dptr<double>(c->ox));
    launch_tv_grad(c->stream, g->rows, g->cols, dptr<double>(c->ox), tbar, dptr<double>(c->part_g), nullptr);
    if (norm2) launch_reduce(c->stream, dptr<double>(c->part_g), tv_blocks(g->rows, g->cols), norm2);
    return check_launch(c);
}

int sp_tv_perturb(sp_ctx* c, const sp_geometry* g, const sp_tv_params* p, const float* x,
                  int32_t* ell, float* x_half, double* tv_half, int32_t* trials) {
    if (!c) return SP_ERR_ARG;
    if (!p || !x || !ell || !x_half) return fail(c, SP_ERR_ARG, "p, x, ell and x_half are required");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = setup_geometry(c, g);
    if (rc) return rc;
    if ((rc = check_tv(c, p))) return rc;
    const size_t n = (size_t)g->rows * g->cols;
    if ((rc = ensure_op_vectors(c, n))) return rc;
    if ((rc = ensure_partials(c))) return rc;
    Scalars& s = c->sc_h;
    s = Scalars{};
    s.a = p->a;
    s.gamma = p->gamma;
    s.K = p->K;
    s.max_trials = p->max_trials > 0 ? p->max_trials : 100;
    if ((rc = upload_scalars(c, c->oscal))) return rc;
    Scalars* sc = dptr<Scalars>(c->oscal);
    HIP_TRY(c, hipMemcpyAsync(&sc->ell, ell, sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    TraceDev tr{};
    double* xd = dptr<double>(c->ox);
    double* xhd = dptr<double>(c->oxh);
    launch_widen(c->stream, (int)n, x, xd);
    if (p->K == 0) {
        launch_copy(c->stream, (int)n, xd, xhd, nullptr);
    } else {
        enqueue_stv(c, sc, p->K, xd, xhd, false, tr, trials);
    }
    launch_narrow(c->stream, (int)n, xhd, x_half);
    HIP_TRY(c, hipMemcpyAsync(ell, &sc->ell, sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    if (tv_half) {
        if (p->K == 0) {
            launch_tv_value(c->stream, g->rows, g->cols, xhd, dptr<double>(c->part_g), nullptr);
            launch_reduce(c->stream, dptr<double>(c->part_g), tv_blocks(g->rows, g->cols), tv_half);
        } else {
            HIP_TRY(c, hipMemcpyAsync(tv_half, &sc->tv_new, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        }
    }
    return check_launch(c);
}

int sp_suppcg_solve(sp_ctx* c, const sp_geometry* g, const float* b, const float* x0,
                    const sp_tv_params* tv, const sp_precond* pc, const sp_solve_params* sp,
                    float* x_out, float* x_last, int32_t* k_out, sp_trace* trace) {
    if (!c) return SP_ERR_ARG;
    if (!b || !x_out || !k_out || !sp) return fail(c, SP_ERR_ARG, "b, x_out, k_out and params are required");
    const bool async = (sp->flags & SP_FLAG_ASYNC) != 0;
    const bool resume = (sp->flags & SP_FLAG_RESUME) != 0;
    if (async && trace) return fail(c, SP_ERR_ARG, "SP_FLAG_ASYNC returns no trace (trace must be NULL)");
    HIP_TRY(c, hipSetDevice(c->device));
    if ((sp->flags & SP_FLAG_GRAPH) && c->stream == nullptr && !c->prof) {
        // The null stream cannot be captured: run the whole solve on an owned
        // stream, ordered after the caller's prior work and, for an
        // asynchronous solve, with the null stream waiting on its end.
        if (!c->own) HIP_TRY(c, hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
        if (!c->own_ev[0]) {
            HIP_TRY(c, hipEventCreateWithFlags(&c->own_ev[0], hipEventDisableTiming));
            HIP_TRY(c, hipEventCreateWithFlags(&c->own_ev[1], hipEventDisableTiming));
        }
        HIP_TRY(c, hipEventRecord(c->own_ev[0], nullptr));
        HIP_TRY(c, hipStreamWaitEvent(c->own, c->own_ev[0], 0));
        c->stream = c->own;
        int r = sp_suppcg_solve(c, g, b, x0, tv, pc, sp, x_out, x_last, k_out, trace);
        c->stream = nullptr;
        if (async) {
            HIP_TRY(c, hipEventRecord(c->own_ev[1], c->own));
            HIP_TRY(c, hipStreamWaitEvent(nullptr, c->own_ev[1], 0));
        } else {
            (void)hipStreamSynchronize(c->own);
        }
        return r;
    }
    int rc = drain_pending(c);
    if (rc) return rc;
    if ((rc = setup_geometry(c, g))) return rc;
    if ((rc = check_precond(c, pc))) return rc;
    if ((rc = check_tv(c, tv))) return rc;
    if (sp->max_iter < 0) return fail(c, SP_ERR_ARG, "max_iter must be >= 0");
    if (!std::isfinite(sp->eps)) return fail(c, SP_ERR_ARG, "eps must be finite");
    const int K = (tv && tv->K > 0) ? tv->K : 0;
    const int max_trials = K ? (tv->max_trials > 0 ? tv->max_trials : 100) : 0;
    const bool replay = (sp->flags & SP_FLAG_REPLAY) != 0;
    if (replay && !sp->replay_trials) return fail(c, SP_ERR_ARG, "SP_FLAG_REPLAY needs replay_trials");
    if (resume) {
        const sp_ctx::SolverState& S = c->st;
        if (!S.ok) return fail(c, SP_ERR_ARG, "SP_FLAG_RESUME: the context holds no solver state");
        if (!same_geom(S.geom, *g)) return fail(c, SP_ERR_ARG, "SP_FLAG_RESUME: geometry differs from the saved state");
        if (S.K != K || (K && (S.a != tv->a || S.gamma != tv->gamma || S.max_trials != max_trials)))
            return fail(c, SP_ERR_ARG, "SP_FLAG_RESUME: S_TV parameters differ from the saved state");
        if (S.kind != pc->kind || (pc->kind != SP_PRECOND_NONE && (S.mu != pc->mu || S.rho != pc->rho)))
            return fail(c, SP_ERR_ARG, "SP_FLAG_RESUME: preconditioner differs from the saved state");
    }
    if (trace && trace->se_ref) {
        for (double a : trace->se_axes)
            if (!(a > 0.0) || !std::isfinite(a))
                return fail(c, SP_ERR_ARG, "se_axes must be positive and finite");
        if (!std::isfinite(trace->se_c)) return fail(c, SP_ERR_ARG, "se_c must be finite");
    }
    c->st.ok = false;   // the buffers below are rewritten from here on
    const GeomDev& G = c->G;
    const int n = G.rows * G.cols;
    if ((rc = ensure_vectors(c, n))) return rc;
    if ((rc = ensure_partials(c))) return rc;
    if (pc->kind == SP_PRECOND_RAMP || pc->kind == SP_PRECOND_LEARNED) {
        FFTPlan F{};
        if ((rc = setup_fft(c, F))) return rc;
    }
    const int cap = std::max(sp->max_iter, 1);
    // trace arrays: 5 double arrays + ell + trials, then the selective errors
    // (cap loop bodies, then the slots of x_0 and x_1)
    const size_t tr_main = (size_t)cap * (5 * 8 + 4) + (size_t)cap * std::max(K, 1) * 4;
    const size_t se_off = (tr_main + 63) & ~(size_t)63;
    const size_t tr_bytes = se_off + (size_t)(cap + 2) * 8;
    const bool want_se = trace && trace->se_ref;
    if ((rc = ensure(c, c->trace_d, tr_bytes))) return rc;
    HIP_TRY(c, hipMemsetAsync(c->trace_d.ptr, 0, se_off, c->stream));
    // selective errors start as NaN (0x7FF80000 in both halves is a NaN)
    HIP_TRY(c, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(dptr<char>(c->trace_d) + se_off),
                                 0x7FF80000, (size_t)(cap + 2) * 2, c->stream));
    double* se_body = reinterpret_cast<double*>(dptr<char>(c->trace_d) + se_off);
    TraceDev tr{};
    {
        char* base = dptr<char>(c->trace_d);
        tr.f_half = reinterpret_cast<double*>(base);
        tr.tv_half = tr.f_half + cap;
        tr.alpha = tr.tv_half + cap;
        tr.beta = tr.alpha + cap;
        tr.s_norm = tr.beta + cap;
        tr.ell = reinterpret_cast<int32_t*>(tr.s_norm + cap);
        tr.trials = tr.ell + cap;
        tr.cap = cap;
    }
    if (replay && K > 0) {
        const size_t bytes = (size_t)sp->max_iter * K * sizeof(int32_t);
        if ((rc = ensure(c, c->replay_d, bytes))) return rc;
        HIP_TRY(c, hipMemcpyAsync(c->replay_d.ptr, sp->replay_trials, bytes, hipMemcpyHostToDevice, c->stream));
        tr.replay = dptr<int32_t>(c->replay_d);
    }
    Scalars& s = c->sc_h;
    if (resume) {
        // continue from the carried scalars (p^T h, l, k, f, ...): a new call
        // counts its loop bodies from 0; a stop on the eps test is re-taken
        // with this call's eps, a breakdown or non-finite stop is final
        HIP_TRY(c, hipMemcpyAsync(&s, c->scal.ptr, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (s.halt == SP_CONVERGED) s.halt = 0;
        s.iter = 0;
        s.inner = 0;
    } else {
        s = Scalars{};
        s.a = K ? tv->a : 0.5;
        s.gamma = K ? tv->gamma : 0.0;
        s.K = K;
        s.max_trials = max_trials;
        s.first = 1;
        s.gate_learned = pc->kind == SP_PRECOND_LEARNED ? 1 : 0;
        s.gate_ramp = 0;
    }
    s.eps = sp->eps;
    s.max_iter = sp->max_iter;
    s.replay = replay ? 1 : 0;
    if ((rc = upload_scalars(c, c->scal))) return rc;

    hipStream_t st = c->stream;
    // wall-time trace: an event at the start, after steps 1-9 and after every
    // loop body (between graph replays in graph mode)
    std::vector<hipEvent_t> tev;
    struct EvGuard {
        std::vector<hipEvent_t>& v;
        ~EvGuard() {
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
        }
    } ev_guard{tev};
    if (trace && trace->t_ms && !async) {
        tev.resize((size_t)cap + 2, nullptr);
        for (hipEvent_t& e : tev) HIP_TRY(c, hipEventCreate(&e));
        HIP_TRY(c, hipEventRecord(tev[0], st));
    }
    Scalars* sc = dptr<Scalars>(c->scal);
    const int* halt = &sc->halt;
    double* xh = dptr<double>(c->vxh);                  // x_{k+1/2}
    double* x = dptr<double>(c->vx);                    // x_k
    double* p = dptr<double>(c->vp);
    double* q = dptr<double>(c->vq);                    // R p
    double* w = dptr<double>(c->vw);                    // R z
    float* gv = dptr<float>(c->vg);
    float* z = dptr<float>(c->vz);
    double* xp = dptr<double>(c->xp);
    double* xTp = dptr<double>(c->xTp);
    double* seg = dptr<double>(c->seg);
    const int* pord = dptr<int>(c->pord);
    double* rpd = dptr<double>(c->ypd);
    const WaveDev* waves = dptr<WaveDev>(c->pwave);
    const AngleDev* ang = dptr<AngleDev>(c->ang);
    double* pf = dptr<double>(c->part_f);
    double* pzh = dptr<double>(c->part_zh);
    double* pgp = dptr<double>(c->part_gp);
    double* pqq = dptr<double>(c->part_qq);
    const int m = G.nA * G.nB;
    const int nf = project_blocks(G), nqq = vec_blocks(m), ngp = vec_blocks(n);

    const double se_ah = want_se ? trace->se_axes[0] : 0.0, se_av = want_se ? trace->se_axes[1] : 0.0;
    auto se_of_x = [&](double* dst, double* dst_body, const int* hflag) {
        launch_se(st, G.rows, G.cols, g->pixel, se_ah, se_av, x, trace->se_ref, trace->se_c,
                  dptr<double>(c->part_se), dst, dst_body, cap, sc, hflag);
    };
    if (!resume) {
        launch_widen(st, n, x0, xh);
        launch_widen(st, n, x0, x);
        if (want_se) se_of_x(se_body + cap, nullptr, nullptr);                       // SE(x_0)
        // Algorithm 3, steps 1-9 (x_{1/2} = x_0; g_0 = A x_0 - y; z_0 = M g_0;
        // p_0 = -z_0; h_0 = A p_0, carried as q = R p_0 = -R z_0; alpha;
        // x_1 = x_0 + alpha p_0; k = 1; l_1 = 0).
        launch_prep(st, G, xh, xp, xTp, halt);
        launch_project(st, G, ang, waves, xp, xTp, b, nullptr, 0, nullptr, rpd, pf, seg, pord, halt);
        launch_scalar(st, OP_F0, sc, tr, pf, nf, nullptr, 0);
        launch_backproject(st, G, ang, rpd, gv, nullptr, nullptr, halt);
        int nzh = 0;
        if ((rc = enqueue_precond(c, pc, gv, z, nullptr, pzh, nzh, true, xp, xTp))) return rc;   // + R's copies of z
        launch_project(st, G, ang, waves, xp, xTp, nullptr, nullptr, 0, nullptr, nullptr, pf, seg, pord,
                       halt, q, w);                                                // w = R z_0
        launch_update_pq_beta(st, n, m, z, p, gv, w, q, sc, tr, pf, nf, pgp, pqq);   // p_0, q
        launch_update_x_alpha(st, n, xh, p, x, sc, tr, pqq, nqq, pgp, ngp, OP_ALPHA0);
        if (want_se) se_of_x(se_body + cap + 1, nullptr, halt);                      // SE(x_1)
        if ((rc = check_launch(c))) return rc;
    }
    if (!tev.empty()) HIP_TRY(c, hipEventRecord(tev[1], st));

    float* snap = (trace && trace->g_snap && trace->g_snap_count > 0) ? trace->g_snap : nullptr;
    const int snap_count = snap ? trace->g_snap_count : 0;
    // One loop body (steps 10-14); every launch reads device state only, so
    // the body can be replayed from a captured graph.
    // r = R x - b goes to the float64 sinogram rpd with the f partials in pf;
    // w = R z to the float64 w with the partials of w^T q in pf
    auto project = [&](const float* bb) {
        ProfScope ps(c, SP_PROF_PROJECT);
        if (bb) launch_project(st, G, ang, waves, xp, xTp, bb, nullptr, 0, nullptr, rpd, pf, seg, pord, halt);
        else launch_project(st, G, ang, waves, xp, xTp, nullptr, nullptr, 0, nullptr, nullptr, pf, seg, pord,
                            halt, q, w);
    };
    auto backproject = [&](float* out, const ScalarRide& ride) {
        ProfScope ps(c, SP_PROF_BACKPROJECT);
        launch_backproject(st, G, ang, rpd, out, nullptr, nullptr, halt, ride);
    };
    // g = R^T r also carries f(x_{k+1/2}) (and the S_TV step norm when K > 0)
    ScalarRide ride_f;
    ride_f.sc = sc;
    ride_f.tr = tr;
    ride_f.pf = pf;
    ride_f.nf = nf;
    ride_f.ps = K > 0 ? dptr<double>(c->part_s) : nullptr;
    ride_f.ns = tv_prep_tiles(G.rows, G.cols);   // the step norm's partials come from the fused last step
    const bool eps_test = sp->eps > 0.0;
    auto body = [&]() -> int {
        ProfScope ps(c, SP_PROF_ITERATION);
        // step 10: while f(x_{k-1/2}) > eps (the test of the previous body's f)
        if (eps_test) launch_scalar(st, OP_EPS, sc, tr, nullptr, 0, nullptr, 0);
        // S_TV -> x_{k+1/2} (K = 0: x_{k+1/2} = x_k), written with R's padded copies
        if (K > 0) {
            enqueue_stv(c, sc, K, x, xh, true, tr, nullptr, true, xp, xTp);
        } else {
            launch_tv_apply_prep(st, G, x, xh, nullptr, sc, nullptr, nullptr, xp, xTp, halt);
        }
        // U_PCG(x_{k+1/2}, p_{k-1}, h_{k-1}), h_{k-1} carried as q = R p_{k-1}
        project(b);                                                               // r = R x - b
        backproject(gv, ride_f);                                      // g = R^T r, f(x_{k+1/2})
        if (snap) launch_snap(st, n, gv, snap, snap_count, sc);
        int nz = 0;
        int r2 = enqueue_precond(c, pc, gv, z, nullptr, pzh, nz, true, xp, xTp);  // z = M g, R's copies of z
        if (r2) return r2;
        project(nullptr);                                              // w = R z, z^T h = w^T q
        launch_update_pq_beta(st, n, m, z, p, gv, w, q, sc, tr, pf, nf, pgp, pqq);  // beta; p, q
        launch_update_x_alpha(st, n, xh, p, x, sc, tr, pqq, nqq, pgp, ngp, OP_ALPHA);  // alpha; x += alpha p
        if (want_se) se_of_x(nullptr, se_body, halt);                             // SE(x_{k+1})
        return check_launch(c);
    };

    // an asynchronous solve does not wait for the halt flag: bodies after a
    // stop are enqueued and do nothing
    const bool poll = eps_test && !async;
    if ((sp->flags & SP_FLAG_GRAPH) && sp->max_iter > 0 && !c->prof) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int brc = body();
        hipError_t ec = hipStreamEndCapture(st, &graph);
        if (brc) {
            if (graph) (void)hipGraphDestroy(graph);
            return brc;
        }
        if (ec != hipSuccess) return fail(c, SP_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(c, SP_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        }
        int32_t hh = 0;
        for (int it = 0; it < sp->max_iter; ++it) {
            hipError_t el = hipGraphLaunch(exec, st);
            if (el == hipSuccess && !tev.empty()) el = hipEventRecord(tev[2 + it], st);
            if (el != hipSuccess) {
                (void)hipStreamSynchronize(st);
                (void)hipGraphExecDestroy(exec);
                (void)hipGraphDestroy(graph);
                return fail(c, SP_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString(el));
            }
            if (poll && (it & 7) == 7) {
                if (hipMemcpyAsync(&hh, &sc->halt, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess) {
                    (void)hipGraphExecDestroy(exec);
                    (void)hipGraphDestroy(graph);
                    return fail(c, SP_ERR_HIP, "polling the halt flag failed");
                }
                if (hh) break;
            }
        }
        if (async) {
            c->pend_graph = graph;   // released once the stream has drained
            c->pend_exec = exec;
        } else {
            const hipError_t es = hipStreamSynchronize(st);
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            if (es != hipSuccess) return fail(c, SP_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(es));
        }
    } else {
        int32_t hh = 0;
        for (int it = 0; it < sp->max_iter; ++it) {
            if ((rc = body())) return rc;
            if (!tev.empty()) HIP_TRY(c, hipEventRecord(tev[2 + it], st));
            if (poll && (it & 7) == 7) {
                HIP_TRY(c, hipMemcpyAsync(&hh, &sc->halt, 4, hipMemcpyDeviceToHost, st));
                HIP_TRY(c, hipStreamSynchronize(st));
                if (hh) break;
            }
        }
    }
    auto keep_state = [&]() {
        sp_ctx::SolverState& S = c->st;
        S.ok = true;
        S.geom = *g;
        S.K = K;
        S.a = K ? tv->a : 0.0;
        S.gamma = K ? tv->gamma : 0.0;
        S.max_trials = max_trials;
        S.kind = pc->kind;
        S.mu = pc->mu;
        S.rho = pc->rho;
        c->last_kind = 1;
        c->last_count = 1;
        c->last_eps = sp->eps;
    };
    if (async) {
        launch_finish(st, n, xh, x, sc, k_out);
        launch_narrow(st, n, xh, x_out);
        if (x_last) launch_narrow(st, n, x, x_last);
        if ((rc = check_launch(c))) return rc;
        keep_state();
        return SP_OK;
    }
    Scalars out{};
    HIP_TRY(c, hipMemcpyAsync(&out, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    *k_out = out.k;
    const int status = run_status(out, sp->eps);
    if (out.halt == SP_BREAKDOWN_CONVERGED && out.k > 1) {
        // the step could not be formed: x_k = x_{k-1/2}
        launch_copy(st, n, xh, x, nullptr);
    }
    launch_narrow(st, n, xh, x_out);
    if (x_last) launch_narrow(st, n, x, x_last);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(st));
    if (trace) {
        const int cnt = std::min(trace->cap, cap);
        std::vector<char> host(tr_bytes);
        HIP_TRY(c, hipMemcpyAsync(host.data(), c->trace_d.ptr, tr_bytes, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        const double* hf = reinterpret_cast<const double*>(host.data());
        const double* htv = hf + cap;
        const double* hal = htv + cap;
        const double* hbe = hal + cap;
        const double* hsn = hbe + cap;
        const int32_t* hell = reinterpret_cast<const int32_t*>(hsn + cap);
        const int32_t* htr = hell + cap;
        const int done = std::min(cnt, out.iter);
        if (trace->f_half) std::copy(hf, hf + done, trace->f_half);
        if (trace->tv_half) std::copy(htv, htv + done, trace->tv_half);
        if (trace->alpha) std::copy(hal, hal + done, trace->alpha);
        if (trace->beta) std::copy(hbe, hbe + done, trace->beta);
        if (trace->s_norm) std::copy(hsn, hsn + done, trace->s_norm);
        if (trace->ell) std::copy(hell, hell + done, trace->ell);
        if (trace->trials && K > 0) std::copy(htr, htr + (size_t)done * K, trace->trials);
        trace->f0 = out.f0;
        trace->alpha0 = out.alpha0;
        trace->fallbacks = out.fallbacks > 0 ? 1 : 0;
        trace->bodies = out.iter;
        const double* hse = reinterpret_cast<const double*>(host.data() + se_off);
        const double nan = std::numeric_limits<double>::quiet_NaN();
        if (want_se && trace->se) std::copy(hse, hse + done, trace->se);
        trace->se0 = want_se && !resume ? hse[cap] : nan;
        trace->se1 = want_se && !resume ? hse[cap + 1] : nan;
        if (!tev.empty()) {
            float ms = 0.0f;
            HIP_TRY(c, hipEventElapsedTime(&ms, tev[0], tev[1]));
            trace->t1_ms = ms;
            for (int j = 0; j < done; ++j) {
                HIP_TRY(c, hipEventElapsedTime(&ms, tev[0], tev[2 + j]));
                trace->t_ms[j] = ms;
            }
        } else {
            trace->t1_ms = nan;
        }
    }
    keep_state();
    if (out.halt == SP_ERR_NONFINITE) return fail(c, SP_ERR_NONFINITE, "non-finite value in a CG scalar");
    return status;
}

// ---- ART and SupART (Section 3.4) ---------------------------------------------------

namespace {
// ART (pixel basis, with S_TV when tv->K > 0) or BlobART (blob basis): the
// iterate is the pixel image or the blob coefficients, float64 on the device.
int art_solve(sp_ctx* c, const sp_geometry* g, const float* b, const float* x0, const sp_tv_params* tv,
              double r, double lam, const sp_solve_params* sp, float* x_out, sp_trace* trace, bool blob) {
    if (!c) return SP_ERR_ARG;
    if (!b || !x_out || !sp) return fail(c, SP_ERR_ARG, "b, x_out and the solve parameters are required");
    if (!(r > 0.0) || !std::isfinite(r)) return fail(c, SP_ERR_ARG, "r must be positive and finite");
    if (!(lam > 0.0 && lam < 2.0)) return fail(c, SP_ERR_ARG, "lambda must lie in (0, 2)");
    if (sp->max_iter < 0) return fail(c, SP_ERR_ARG, "max_iter must be >= 0");
    if (sp->flags & ~(uint32_t)SP_FLAG_GRAPH)
        return fail(c, SP_ERR_ARG, "only SP_FLAG_GRAPH is supported by the ART solver");
    HIP_TRY(c, hipSetDevice(c->device));
    if ((sp->flags & SP_FLAG_GRAPH) && c->stream == nullptr && !c->prof) {
        // the null stream cannot be captured: run on the owned stream, ordered
        // after the caller's prior work
        if (!c->own) HIP_TRY(c, hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
        if (!c->own_ev[0]) {
            HIP_TRY(c, hipEventCreateWithFlags(&c->own_ev[0], hipEventDisableTiming));
            HIP_TRY(c, hipEventCreateWithFlags(&c->own_ev[1], hipEventDisableTiming));
        }
        HIP_TRY(c, hipEventRecord(c->own_ev[0], nullptr));
        HIP_TRY(c, hipStreamWaitEvent(c->own, c->own_ev[0], 0));
        c->stream = c->own;
        const int r2 = art_solve(c, g, b, x0, tv, r, lam, sp, x_out, trace, blob);
        c->stream = nullptr;
        (void)hipStreamSynchronize(c->own);
        return r2;
    }
    int rc = drain_pending(c);
    if (rc) return rc;
    if ((rc = setup_geometry(c, g))) return rc;
    if ((rc = check_tv(c, tv))) return rc;
    const int K = (tv && tv->K > 0) ? tv->K : 0;
    const GeomDev& G = c->G;
    const int n = G.rows * G.cols, m = G.nA * G.nB;
    if (trace && trace->se_ref) {
        for (double a : trace->se_axes)
            if (!(a > 0.0) || !std::isfinite(a)) return fail(c, SP_ERR_ARG, "se_axes must be positive and finite");
        if (!std::isfinite(trace->se_c)) return fail(c, SP_ERR_ARG, "se_c must be finite");
    }
    c->st.ok = false;   // the solver vectors are reused below
    if ((rc = ensure_vectors(c, n)) || (rc = ensure_partials(c))) return rc;
    if ((rc = ensure(c, c->art_u, (size_t)m * 8)) || (rc = ensure(c, c->art_nrm, (size_t)m * 8)) ||
        (rc = ensure(c, c->art_sum, 8)) || (rc = ensure(c, c->ox, (size_t)std::max(n, m) * 8)))
        return rc;
    std::vector<AngleDev> nat((size_t)G.nA);
    for (const AngleDev& A : c->ang_h) nat[(size_t)A.row] = A;
    DevBuf natd;
    struct Tmp {
        DevBuf* a;
        ~Tmp() { release(*a); }
    } tmp{&natd};
    if ((rc = ensure(c, natd, nat.size() * sizeof(AngleDev)))) return rc;
    hipStream_t st = c->stream;
    HIP_TRY(c, hipMemcpyAsync(natd.ptr, nat.data(), nat.size() * sizeof(AngleDev), hipMemcpyHostToDevice, st));
    const int cap = std::max(sp->max_iter, 1);
    const size_t tr_main = (size_t)cap * (5 * 8 + 4) + (size_t)cap * std::max(K, 1) * 4;
    const size_t se_off = (tr_main + 63) & ~(size_t)63;
    const size_t tr_bytes = se_off + (size_t)(cap + 2) * 8;
    const bool want_se = trace && trace->se_ref;
    if ((rc = ensure(c, c->trace_d, tr_bytes))) return rc;
    HIP_TRY(c, hipMemsetAsync(c->trace_d.ptr, 0, se_off, st));
    HIP_TRY(c, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(dptr<char>(c->trace_d) + se_off), 0x7FF80000,
                                 (size_t)(cap + 2) * 2, st));
    double* se_body = reinterpret_cast<double*>(dptr<char>(c->trace_d) + se_off);
    TraceDev tr{};
    {
        char* base = dptr<char>(c->trace_d);
        tr.f_half = reinterpret_cast<double*>(base);
        tr.tv_half = tr.f_half + cap;
        tr.alpha = tr.tv_half + cap;
        tr.beta = tr.alpha + cap;
        tr.s_norm = tr.beta + cap;
        tr.ell = reinterpret_cast<int32_t*>(tr.s_norm + cap);
        tr.trials = tr.ell + cap;
        tr.cap = cap;
    }
    Scalars& s = c->sc_h;
    s = Scalars{};
    s.a = K ? tv->a : 0.5;
    s.gamma = K ? tv->gamma : 0.0;
    s.K = K;
    s.max_trials = K ? (tv->max_trials > 0 ? tv->max_trials : 100) : 0;
    s.max_iter = sp->max_iter;
    if ((rc = upload_scalars(c, c->scal))) return rc;
    Scalars* sc = dptr<Scalars>(c->scal);
    const int* halt = &sc->halt;
    double* x = dptr<double>(c->vx);
    double* xh = dptr<double>(c->vxh);
    double* u = dptr<double>(c->art_u);
    double* nrm = dptr<double>(c->art_nrm);

    std::vector<hipEvent_t> tev;
    struct EvGuard {
        std::vector<hipEvent_t>& v;
        ~EvGuard() {
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
        }
    } ev_guard{tev};
    if (trace && trace->t_ms) {
        tev.resize((size_t)cap + 1, nullptr);
        for (hipEvent_t& e : tev) HIP_TRY(c, hipEventCreate(&e));
        HIP_TRY(c, hipEventRecord(tev[0], st));
    }
    BlobDev B = blob_constants();
    if (blob) {
        std::vector<double2> tab((size_t)B.ntab + 1);
        blob_table_fill(B.a, B.alpha, B.cproj, B.ntab, tab.data());
        if ((rc = ensure(c, c->blob_tab, tab.size() * sizeof(double2)))) return rc;
        HIP_TRY(c, hipMemcpyAsync(c->blob_tab.ptr, tab.data(), tab.size() * sizeof(double2), hipMemcpyHostToDevice,
                                  st));
        HIP_TRY(c, hipStreamSynchronize(st));   // the host table must outlive the copy
        B.tab = dptr<double2>(c->blob_tab);
    }
    const BlobDev* bp = blob ? &B : nullptr;
    double divisor = 1.0;
    if (blob) {
        divisor = 0.0;
        for (int di = 0; di < 5; ++di)
            for (int dj = 0; dj < 5; ++dj) divisor += B.stencil[di][dj];
    }
    // the image the trace and x_out see: x itself, or the blob image in xh
    double* img = blob ? xh : x;
    launch_art_norms(st, G, dptr<AngleDev>(natd), bp, nrm);
    launch_art_init(st, G, b, x0, divisor, dptr<double>(c->ox), dptr<double>(c->art_sum), x, u);
    if (blob) launch_blob_synth(st, G.rows, G.cols, B, x, img, nullptr);
    if (want_se)
        launch_se(st, G.rows, G.cols, g->pixel, trace->se_axes[0], trace->se_axes[1], img, trace->se_ref,
                  trace->se_c, dptr<double>(c->part_se), se_body + cap, nullptr, 0, nullptr, nullptr);
    if ((rc = check_launch(c))) return rc;
    // one iteration: S_TV (SupART), then a cycle through the rays
    auto body = [&]() -> int {
        double* tgt = x;
        if (K > 0) {
            enqueue_stv(c, sc, K, x, xh, false, tr, nullptr);
            tgt = xh;
        }
        launch_art_sweep(st, G, nat.data(), bp, nrm, b, tgt, u, r, lam, halt);
        if (K > 0) launch_copy(st, n, xh, x, halt);
        if (blob) launch_blob_synth(st, G.rows, G.cols, B, x, img, halt);
        launch_scalar(st, OP_NEXT, sc, tr, nullptr, 0, nullptr, 0);
        if (want_se)
            launch_se(st, G.rows, G.cols, g->pixel, trace->se_axes[0], trace->se_axes[1], img, trace->se_ref,
                      trace->se_c, dptr<double>(c->part_se), nullptr, se_body, cap, sc, halt);
        return check_launch(c);
    };
    if ((sp->flags & SP_FLAG_GRAPH) && sp->max_iter > 0 && !c->prof) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int brc = body();
        const hipError_t ec = hipStreamEndCapture(st, &graph);
        if (brc) {
            if (graph) (void)hipGraphDestroy(graph);
            return brc;
        }
        if (ec != hipSuccess) return fail(c, SP_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(c, SP_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        }
        hipError_t el = hipSuccess;
        for (int it = 0; it < sp->max_iter && el == hipSuccess; ++it) {
            el = hipGraphLaunch(exec, st);
            if (el == hipSuccess && !tev.empty()) el = hipEventRecord(tev[1 + it], st);
        }
        const hipError_t es = hipStreamSynchronize(st);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        if (el != hipSuccess) return fail(c, SP_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString(el));
        if (es != hipSuccess) return fail(c, SP_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(es));
    } else {
        for (int it = 0; it < sp->max_iter; ++it) {
            if ((rc = body())) return rc;
            if (!tev.empty()) HIP_TRY(c, hipEventRecord(tev[1 + it], st));
        }
    }
    launch_narrow(st, n, img, x_out);
    Scalars out{};
    HIP_TRY(c, hipMemcpyAsync(&out, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (trace) {
        const int cnt = std::min(trace->cap, cap);
        const int done = std::min(cnt, out.iter);
        std::vector<char> host(tr_bytes);
        HIP_TRY(c, hipMemcpy(host.data(), c->trace_d.ptr, tr_bytes, hipMemcpyDeviceToHost));
        const double* htv = reinterpret_cast<const double*>(host.data()) + cap;
        const int32_t* hell = reinterpret_cast<const int32_t*>(reinterpret_cast<const double*>(host.data()) + 5 * cap);
        const int32_t* htr = hell + cap;
        if (trace->tv_half && K > 0) std::copy(htv, htv + done, trace->tv_half);
        if (trace->ell && K > 0) std::copy(hell, hell + done, trace->ell);
        if (trace->trials && K > 0) std::copy(htr, htr + (size_t)done * K, trace->trials);
        const double* hse = reinterpret_cast<const double*>(host.data() + se_off);
        const double nan = std::numeric_limits<double>::quiet_NaN();
        if (want_se && trace->se) std::copy(hse, hse + done, trace->se);
        trace->se0 = want_se ? hse[cap] : nan;
        trace->se1 = nan;
        if (!tev.empty()) {
            float ms = 0.0f;
            for (int j = 0; j < done; ++j) {
                HIP_TRY(c, hipEventElapsedTime(&ms, tev[0], tev[1 + j]));
                trace->t_ms[j] = ms;
            }
        }
        trace->t1_ms = nan;
        trace->bodies = out.iter;
    }
    return out.exhausted ? SP_TRIALS_EXHAUSTED : SP_MAXITER;
}
}  // namespace

int sp_supart_solve(sp_ctx* c, const sp_geometry* g, const float* b, const float* x0,
                    const sp_tv_params* tv, double r, double lam, const sp_solve_params* sp, float* x_out,
                    sp_trace* trace) {
    return art_solve(c, g, b, x0, tv, r, lam, sp, x_out, trace, false);
}

int sp_blobart_solve(sp_ctx* c, const sp_geometry* g, const float* b, double r, double lam,
                     const sp_solve_params* sp, float* x_out, sp_trace* trace) {
    return art_solve(c, g, b, nullptr, nullptr, r, lam, sp, x_out, trace, true);
}

// ---- stored matrices ---------------------------------------------------------------

namespace {
void matrix_free(sp_matrix* M) {
    for (int sd = 0; sd < 2; ++sd) {
        release(M->sp[sd]);
        release(M->len[sd]);
        release(M->ent[sd]);
    }
    release(M->segT);
    delete M;
}
}  // namespace

int sp_matrix_build(sp_ctx* c, const sp_geometry* g, sp_matrix** out) {
    if (!c) return SP_ERR_ARG;
    if (!out) return fail(c, SP_ERR_ARG, "out is NULL");
    *out = nullptr;
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = drain_pending(c);
    if (rc) return rc;
    if ((rc = setup_geometry(c, g))) return rc;
    const GeomDev& G = c->G;
    const int64_t m = (int64_t)G.nA * G.nB, n = (int64_t)G.rows * G.cols;
    if (m >= ((int64_t)1 << 31) - 256)
        return fail(c, SP_ERR_ARG, "stored matrices need n_angles * n_bins < 2^31");
    // the angle table in natural order (the projectors' copy is sorted by class)
    std::vector<AngleDev> nat((size_t)G.nA);
    for (const AngleDev& A : c->ang_h) nat[(size_t)A.row] = A;
    sp_matrix* M = new (std::nothrow) sp_matrix;
    if (!M) return fail(c, SP_ERR_ALLOC, "out of host memory");
    M->device = c->device;
    M->geom = *g;
    M->rows[0] = m;
    M->rows[1] = n;
    M->shape[0] = SellShape{G.nA, G.nB, (G.nB + 63) / 64};
    M->shape[1] = SellShape{G.rows, G.cols, (G.cols + 63) / 64};
    DevBuf natd, ssize, offs, sums;
    struct Tmp {
        DevBuf *a, *b, *c, *d;
        ~Tmp() {
            release(*a);
            release(*b);
            release(*c);
            release(*d);
        }
    } tmp{&natd, &ssize, &offs, &sums};
    hipStream_t st = c->stream;
    auto bail = [&](int code) {
        (void)hipStreamSynchronize(st);
        matrix_free(M);
        return code;
    };
    const int64_t big = std::max(m, n);
    if ((rc = ensure(c, natd, nat.size() * sizeof(AngleDev))) ||
        (rc = ensure(c, ssize, (size_t)std::max(M->shape[0].nseg * M->shape[0].spseg,
                                                M->shape[1].nseg * M->shape[1].spseg) * 4)) ||
        (rc = ensure(c, offs, (size_t)(big + 1) * 8)) ||
        (rc = ensure(c, sums, (size_t)scan_blocks(big) * 8)))
        return bail(rc);
    if (hipMemcpyAsync(natd.ptr, nat.data(), nat.size() * sizeof(AngleDev), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return bail(fail(c, SP_ERR_HIP, "copying the angle table failed"));
    std::vector<uint8_t> segT((size_t)G.nA);
    for (int a = 0; a < G.nA; ++a) segT[(size_t)a] = (nat[(size_t)a].flags & ANG_HORIZ) ? 1 : 0;
    if ((rc = ensure(c, M->segT, segT.size())) ||
        hipMemcpyAsync(M->segT.ptr, segT.data(), segT.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return bail(rc ? rc : fail(c, SP_ERR_HIP, "copying the segment table failed"));
    int64_t nnz_side[2] = {0, 0};
    for (int sd = 0; sd < 2; ++sd) {
        const SellShape& S = M->shape[sd];
        const int64_t rows = M->rows[sd], ns = S.nseg * S.spseg;
        if ((rc = ensure(c, M->len[sd], (size_t)rows * 4)) || (rc = ensure(c, M->sp[sd], (size_t)(ns + 1) * 8)))
            return bail(rc);
        int32_t* len = dptr<int32_t>(M->len[sd]);
        launch_stored_count(st, G, dptr<AngleDev>(natd), sd == 1, len);
        launch_scan(st, len, rows, dptr<int64_t>(offs), dptr<int64_t>(sums));          // nonzeros
        launch_slice_sizes(st, len, S, dptr<int32_t>(ssize));
        launch_scan(st, dptr<int32_t>(ssize), ns, dptr<int64_t>(M->sp[sd]), dptr<int64_t>(sums));
        if (hipMemcpyAsync(&nnz_side[sd], dptr<int64_t>(offs) + rows, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&M->words[sd], dptr<int64_t>(M->sp[sd]) + ns, 8, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return bail(fail(c, SP_ERR_HIP, "counting the nonzeros failed: %s",
                             hipGetErrorString(hipGetLastError())));
        // padding: column 0, weight 0 (ensure zero-fills new storage)
        if ((rc = ensure(c, M->ent[sd], (size_t)M->words[sd] * 4))) return bail(rc);
        launch_stored_fill(st, G, S, dptr<AngleDev>(natd), sd == 1, dptr<int64_t>(M->sp[sd]), len,
                           dptr<int32_t>(M->ent[sd]));
    }
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(fail(c, SP_ERR_HIP, "building the matrices: %s", hipGetErrorString(e)));
    if (nnz_side[0] != nnz_side[1])
        return bail(fail(c, SP_ERR_HIP, "R and R^T counts differ (%lld vs %lld)", (long long)nnz_side[0],
                         (long long)nnz_side[1]));
    M->nnz = nnz_side[0];
    *out = M;
    return SP_OK;
}

int sp_matrix_destroy(sp_matrix* M) {
    if (!M) return SP_ERR_ARG;
    (void)hipSetDevice(M->device);
    (void)hipDeviceSynchronize();
    matrix_free(M);
    return SP_OK;
}

int sp_matrix_info(const sp_matrix* M, int64_t* nnz, int64_t* bytes) {
    if (!M) return SP_ERR_ARG;
    if (nnz) *nnz = M->nnz;
    if (bytes) {
        int64_t t = 0;
        for (int sd = 0; sd < 2; ++sd)
            t += (int64_t)(M->sp[sd].bytes + M->len[sd].bytes + M->ent[sd].bytes);
        *bytes = t + (int64_t)M->segT.bytes;
    }
    return SP_OK;
}

namespace {
int matrix_apply(sp_ctx* c, const sp_matrix* M, int side, const float* in, float* out) {
    if (!c) return SP_ERR_ARG;
    if (!M || !in || !out) return fail(c, SP_ERR_ARG, "matrix, input and output are required");
    if (M->device != c->device) return fail(c, SP_ERR_ARG, "the matrix lives on another device");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = drain_pending(c);
    if (rc) return rc;
    sp_matrix* W = const_cast<sp_matrix*>(M);
    const float* inT = nullptr;
    if (side == 0) {
        if ((rc = ensure(c, c->stored_xT, (size_t)M->rows[1] * 4))) return rc;
        inT = dptr<float>(c->stored_xT);
    }
    ProfScope ps(c, side ? SP_PROF_STORED_BACKPROJECT : SP_PROF_STORED_PROJECT);
    if (side == 0) launch_transpose(c->stream, M->geom.rows, M->geom.cols, in, dptr<float>(c->stored_xT));
    launch_sell_spmv(c->stream, M->shape[side], dptr<int64_t>(W->sp[side]), dptr<int32_t>(W->len[side]),
                     dptr<int32_t>(W->ent[side]), in, inT, side == 0 ? dptr<uint8_t>(W->segT) : nullptr, out);
    return check_launch(c);
}
}  // namespace

int sp_matrix_project(sp_ctx* c, const sp_matrix* M, const float* x, float* y) {
    return matrix_apply(c, M, 0, x, y);
}

int sp_matrix_backproject(sp_ctx* c, const sp_matrix* M, const float* y, float* x) {
    return matrix_apply(c, M, 1, y, x);
}

int sp_matrix_export(sp_ctx* c, const sp_matrix* M, int side, int64_t* row_ptr, int32_t* col, float* val) {
    if (!c) return SP_ERR_ARG;
    if (!M || (side != 0 && side != 1)) return fail(c, SP_ERR_ARG, "matrix and side 0 or 1 are required");
    if (M->device != c->device) return fail(c, SP_ERR_ARG, "the matrix lives on another device");
    HIP_TRY(c, hipSetDevice(c->device));
    sp_matrix* W = const_cast<sp_matrix*>(M);
    hipStream_t st = c->stream;
    const SellShape& S = M->shape[side];
    const int64_t rows = M->rows[side], ns = S.nseg * S.spseg, words = M->words[side];
    const int R = M->geom.rows, C = M->geom.cols;
    std::vector<int64_t> hsp((size_t)ns + 1);
    std::vector<int32_t> hlen((size_t)rows), hent;
    HIP_TRY(c, hipMemcpyAsync(hsp.data(), W->sp[side].ptr, hsp.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(hlen.data(), W->len[side].ptr, hlen.size() * 4, hipMemcpyDeviceToHost, st));
    if (col || val) {
        hent.resize((size_t)words);
        HIP_TRY(c, hipMemcpyAsync(hent.data(), W->ent[side].ptr, (size_t)words * 4, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    std::vector<uint8_t> segT;
    if (side == 0) {
        segT.resize((size_t)S.nseg);
        HIP_TRY(c, hipMemcpy(segT.data(), W->segT.ptr, segT.size(), hipMemcpyDeviceToHost));
    }
    int64_t p = 0;
    if (row_ptr) row_ptr[0] = 0;
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t seg = r / S.lseg, k = r % S.lseg;
        const int64_t base = hsp[(size_t)sell_slice(S, r)];
        const int lane = sell_lane(S, r);
        const bool tr = side == 0 && segT[(size_t)seg];
        for (int32_t e = 0; e < hlen[(size_t)r]; ++e, ++p) {
            const size_t at = (size_t)(base + sell_offset(lane, e));
            if (col) {
                const int32_t q = hent[at];
                col[p] = tr ? (q % R) * C + q / R : q;   // transposed index j * rows + i
            }
            if (val) std::memcpy(&val[p], &hent[at + SELL_VAL], 4);
        }
        if (row_ptr) row_ptr[r + 1] = p;
    }
    return SP_OK;
}

// ---- checkpoint / resume -------------------------------------------------------

namespace {
struct StateHeader {
    char magic[8];
    int32_t version, scalars_bytes;
    sp_geometry geom;
    int32_t K, max_trials, kind, pad_;
    double a, gamma, mu, rho;
    int64_t n;
    Scalars sc;
};
constexpr char STATE_MAGIC[8] = {'S', 'P', 'S', 'T', 'A', 'T', 'E', '1'};

// Header, then x_k, x_{k-1/2}, p_{k-1} (n float64 each) and q = R p_{k-1}
// (m = nA nB float64).
int64_t state_bytes(int64_t n, int64_t m) { return (int64_t)sizeof(StateHeader) + n * 3 * 8 + m * 8; }
constexpr int32_t STATE_VERSION = 2;
}  // namespace

int sp_state_save(sp_ctx* c, void* host_blob, int64_t* bytes) {
    if (!c) return SP_ERR_ARG;
    if (!bytes) return fail(c, SP_ERR_ARG, "sp_state_save: bytes is required");
    if (!c->st.ok) return fail(c, SP_ERR_ARG, "sp_state_save: the context holds no solver state");
    HIP_TRY(c, hipSetDevice(c->device));
    const sp_ctx::SolverState& S = c->st;
    const int64_t n = (int64_t)S.geom.rows * S.geom.cols;
    const int64_t m = (int64_t)S.geom.n_angles * S.geom.n_bins;
    const int64_t need = state_bytes(n, m);
    if (!host_blob) {
        *bytes = need;
        return SP_OK;
    }
    if (*bytes < need) return fail(c, SP_ERR_ARG, "sp_state_save: the blob needs %lld bytes", (long long)need);
    int rc = drain_pending(c);
    if (rc) return rc;
    StateHeader hd{};
    std::memcpy(hd.magic, STATE_MAGIC, 8);
    hd.version = STATE_VERSION;
    hd.scalars_bytes = (int32_t)sizeof(Scalars);
    hd.geom = S.geom;
    hd.K = S.K;
    hd.max_trials = S.max_trials;
    hd.kind = S.kind;
    hd.a = S.a;
    hd.gamma = S.gamma;
    hd.mu = S.mu;
    hd.rho = S.rho;
    hd.n = n;
    char* out = static_cast<char*>(host_blob);
    HIP_TRY(c, hipMemcpyAsync(&hd.sc, c->scal.ptr, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
    char* v = out + sizeof(StateHeader);
    HIP_TRY(c, hipMemcpyAsync(v, c->vx.ptr, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(v + n * 8, c->vxh.ptr, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(v + 2 * n * 8, c->vp.ptr, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(v + 3 * n * 8, c->vq.ptr, (size_t)m * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::memcpy(out, &hd, sizeof hd);
    *bytes = need;
    return SP_OK;
}

int sp_state_load(sp_ctx* c, const void* host_blob, int64_t bytes) {
    if (!c) return SP_ERR_ARG;
    if (!host_blob || bytes < (int64_t)sizeof(StateHeader))
        return fail(c, SP_ERR_ARG, "sp_state_load: blob too short");
    StateHeader hd;
    std::memcpy(&hd, host_blob, sizeof hd);
    if (std::memcmp(hd.magic, STATE_MAGIC, 8) != 0 || hd.version != STATE_VERSION ||
        hd.scalars_bytes != (int32_t)sizeof(Scalars))
        return fail(c, SP_ERR_ARG, "sp_state_load: not a state blob of this library version");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = drain_pending(c);
    if (rc) return rc;
    if ((rc = setup_geometry(c, &hd.geom))) return rc;
    const int64_t n = (int64_t)hd.geom.rows * hd.geom.cols;
    const int64_t m = (int64_t)hd.geom.n_angles * hd.geom.n_bins;
    if (hd.n != n || bytes < state_bytes(n, m)) return fail(c, SP_ERR_ARG, "sp_state_load: blob size mismatch");
    c->st.ok = false;
    if ((rc = ensure_vectors(c, (size_t)n))) return rc;
    if ((rc = ensure_partials(c))) return rc;
    const char* v = static_cast<const char*>(host_blob) + sizeof(StateHeader);
    c->sc_h = hd.sc;
    HIP_TRY(c, hipMemcpyAsync(c->scal.ptr, &c->sc_h, sizeof(Scalars), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->vx.ptr, v, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->vxh.ptr, v + n * 8, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->vp.ptr, v + 2 * n * 8, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->vq.ptr, v + 3 * n * 8, (size_t)m * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    sp_ctx::SolverState& S = c->st;
    S.geom = hd.geom;
    S.K = hd.K;
    S.max_trials = hd.max_trials;
    S.kind = hd.kind;
    S.a = hd.a;
    S.gamma = hd.gamma;
    S.mu = hd.mu;
    S.rho = hd.rho;
    S.ok = true;
    c->last_kind = 0;
    return SP_OK;
}

int sp_solve_status(sp_ctx* c, int32_t count, int32_t* k, int32_t* status) {
    if (!c) return SP_ERR_ARG;
    if (!k || !status) return fail(c, SP_ERR_ARG, "sp_solve_status: k and status are required");
    if (c->last_kind == 0) return fail(c, SP_ERR_ARG, "sp_solve_status: no solve has run on this context");
    if (count != c->last_count)
        return fail(c, SP_ERR_ARG, "sp_solve_status: the last solve had %d slice(s)", c->last_count);
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = drain_pending(c);
    if (rc) return rc;
    std::vector<Scalars> q((size_t)count);
    const void* src = c->last_kind == 1 ? c->scal.ptr : c->batch->scal.ptr;
    HIP_TRY(c, hipMemcpyAsync(q.data(), src, sizeof(Scalars) * (size_t)count, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < count; ++i) {
        k[i] = q[(size_t)i].k;
        status[i] = run_status(q[(size_t)i], c->last_eps);
    }
    return SP_OK;
}

int sp_suppcg_solve_batched(sp_ctx* c, int32_t n, const sp_geometry* geoms, const float* const* b,
                            const float* const* x0, const sp_tv_params* tv, const sp_precond* pc,
                            const sp_solve_params* sp, float* const* x_out, float* const* x_last,
                            int32_t* k_out, sp_batch_trace* trace) {
    if (!c) return SP_ERR_ARG;
    if (n < 1 || n > MAX_BATCH) return fail(c, SP_ERR_ARG, "n must be in [1, %d]", MAX_BATCH);
    if (!geoms || !b || !x_out || !k_out || !sp || !pc)
        return fail(c, SP_ERR_ARG, "geoms, b, x_out, k_out, params and preconditioner are required");
    const bool async = (sp->flags & SP_FLAG_ASYNC) != 0;
    if (async && trace) return fail(c, SP_ERR_ARG, "SP_FLAG_ASYNC returns no trace (trace must be NULL)");
    if (sp->flags & SP_FLAG_RESUME)
        return fail(c, SP_ERR_ARG, "SP_FLAG_RESUME is not supported by the batched solver");
    HIP_TRY(c, hipSetDevice(c->device));
    if ((sp->flags & SP_FLAG_GRAPH) && c->stream == nullptr) {
        if (!c->own) HIP_TRY(c, hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
        if (!c->own_ev[0]) {
            HIP_TRY(c, hipEventCreateWithFlags(&c->own_ev[0], hipEventDisableTiming));
            HIP_TRY(c, hipEventCreateWithFlags(&c->own_ev[1], hipEventDisableTiming));
        }
        HIP_TRY(c, hipEventRecord(c->own_ev[0], nullptr));
        HIP_TRY(c, hipStreamWaitEvent(c->own, c->own_ev[0], 0));
        c->stream = c->own;
        int r = sp_suppcg_solve_batched(c, n, geoms, b, x0, tv, pc, sp, x_out, x_last, k_out, trace);
        c->stream = nullptr;
        if (async) {
            HIP_TRY(c, hipEventRecord(c->own_ev[1], c->own));
            HIP_TRY(c, hipStreamWaitEvent(nullptr, c->own_ev[1], 0));
        } else {
            (void)hipStreamSynchronize(c->own);
        }
        return r;
    }
    int rc = drain_pending(c);
    if (rc) return rc;
    for (int s = 0; s < n; ++s) {
        if ((rc = validate_geometry(c, &geoms[s]))) return fail(c, rc, "slice %d: %s", s, c->err);
        if (!b[s] || !x_out[s]) return fail(c, SP_ERR_ARG, "slice %d: b and x_out are required", s);
    }
    if (pc->kind != SP_PRECOND_RAMP && pc->kind != SP_PRECOND_NONE)
        return fail(c, SP_ERR_ARG, "the batched solver supports the Fourier preconditioner and M = I");
    if ((rc = check_precond(c, pc))) return rc;
    if ((rc = check_tv(c, tv))) return rc;
    if (sp->flags & SP_FLAG_REPLAY) return fail(c, SP_ERR_ARG, "SP_FLAG_REPLAY is not supported by the batched solver");
    if (sp->max_iter < 0) return fail(c, SP_ERR_ARG, "max_iter must be >= 0");
    if (!std::isfinite(sp->eps)) return fail(c, SP_ERR_ARG, "eps must be finite");
    if (sp->flags & SP_FLAG_AUTOTUNE) {
        // launch shapes of every geometry the table does not hold yet
        for (int s = 0; s < n; ++s) {
            int tp, tx;
            if (shape_lookup(geoms[s], tp, tx)) continue;
            if ((rc = sp_tune_shapes(c, &geoms[s], nullptr, nullptr, nullptr)))
                return fail(c, rc, "slice %d: tuning its launch shapes: %s", s, c->err);
        }
    }
    if ((rc = batch_setup(c, n, geoms, pc->kind))) return rc;
    BatchState& B = *c->batch;
    const int K = (tv && tv->K > 0) ? tv->K : 0;
    const int cap = std::max(sp->max_iter, 1);
    const size_t tr_slice = align256((size_t)cap * (5 * 8 + 4));
    if ((rc = ensure(c, B.trace_d, tr_slice * (size_t)n))) return rc;
    HIP_TRY(c, hipMemsetAsync(B.trace_d.ptr, 0, tr_slice * (size_t)n, c->stream));
    std::vector<Scalars> sc(n);
    for (int s = 0; s < n; ++s) {
        SliceDev& S = B.hs[s];
        S.b = b[s];
        S.x0 = x0 ? x0[s] : nullptr;
        char* t = dptr<char>(B.trace_d) + tr_slice * s;
        S.tr = TraceDev{};
        S.tr.f_half = reinterpret_cast<double*>(t);
        S.tr.tv_half = S.tr.f_half + cap;
        S.tr.alpha = S.tr.tv_half + cap;
        S.tr.beta = S.tr.alpha + cap;
        S.tr.s_norm = S.tr.beta + cap;
        S.tr.ell = reinterpret_cast<int32_t*>(S.tr.s_norm + cap);
        S.tr.cap = cap;
        Scalars& q = sc[s];
        q = Scalars{};
        q.eps = sp->eps;
        q.a = K ? tv->a : 0.5;
        q.gamma = K ? tv->gamma : 0.0;
        q.K = K;
        q.max_trials = K ? (tv->max_trials > 0 ? tv->max_trials : 100) : 0;
        q.max_iter = sp->max_iter;
        q.first = 1;
    }
    hipStream_t st = c->stream;
    HIP_TRY(c, hipMemcpyAsync(B.sl.ptr, B.hs.data(), sizeof(SliceDev) * (size_t)n, hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipMemcpyAsync(B.scal.ptr, sc.data(), sizeof(Scalars) * (size_t)n, hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipStreamSynchronize(st));   // host arrays must outlive the copies
    const SliceDev* sl = dptr<SliceDev>(B.sl);
    const double mu = pc->mu, rho = pc->rho;

    launch_init_b(st, sl, table(c, BS_VEC));                       // x_{1/2} = x_0
    if ((sp->flags & SP_FLAG_AUTOTUNE) && !B.tuned && (rc = batch_tune(c, mu, rho))) return rc;
    // Algorithm 3, steps 1-9, every slice in each launch
    const ItemTable tprep = table(c, BS_PREP), tproj = table(c, BS_PROJECT),
                    tbp = table(c, BS_BACKPROJECT), tvec = table(c, BS_VEC), ttv = table(c, BS_TV),
                    ttvt = table(c, BS_TVT), ttvg = table(c, BS_TVG),
                    tone = table(c, BS_SLICE, 0, 0), tpq = table(c, BS_PQ),
                    tcomb = table(c, BS_PROJ_COMB, B.order[BS_PROJECT], 0);
    launch_prep_b(st, sl, tprep, BV_XH);
    launch_project_b(st, sl, tproj, tcomb, true);
    launch_scalar_b(st, sl, tone, OP_F0);
    launch_backproject_b(st, sl, tbp, B.nbmax, B.bp_px);
    batch_precond(c, mu, rho);
    launch_prep_b(st, sl, tprep, BV_Z);
    launch_project_b(st, sl, tproj, tcomb, false);                // w = R z
    launch_scalar_b(st, sl, tone, OP_BETA);
    launch_update_pq_b(st, sl, tpq);                             // p = -z, q = R p = -w
    launch_scalar_b(st, sl, tone, OP_ALPHA0);
    launch_update_x_b(st, sl, tvec);
    if ((rc = check_launch(c))) return rc;

    // loop body (steps 10-14)
    const bool eps_test = sp->eps > 0.0;
    auto body = [&]() {
        if (eps_test) launch_scalar_b(st, sl, tone, OP_EPS);
        if (K > 0) {
            for (int i = 0; i < K; ++i) {
                const int src = i == 0 ? BV_X : BV_XH;
                launch_tv_grad_b(st, sl, i == 0 ? ttv : ttvg, src);   // the item count follows src
                launch_tv_trials_b(st, sl, ttvt, src);
                launch_tv_decide_b(st, sl, tone, src);
                if (i == K - 1) launch_tv_apply_prep_b(st, sl, tprep, src, false, true);   // + R's copies
                else launch_tv_apply_b(st, sl, ttv, src, false);
            }
            launch_scalar_b(st, sl, tone, OP_SNORM);
        } else {
            launch_tv_apply_prep_b(st, sl, tprep, BV_X, true, false);   // x_{k+1/2} = x_k, R's copies
        }
        launch_project_b(st, sl, tproj, tcomb, true);
        launch_scalar_b(st, sl, tone, OP_F);
        launch_backproject_b(st, sl, tbp, B.nbmax, B.bp_px);
        batch_precond(c, mu, rho);
        launch_prep_b(st, sl, tprep, BV_Z);
        launch_project_b(st, sl, tproj, tcomb, false);            // w = R z, (R z)^T q
        launch_scalar_b(st, sl, tone, OP_BETA);
        launch_update_pq_b(st, sl, tpq);
        launch_scalar_b(st, sl, tone, OP_ALPHA);
        launch_update_x_b(st, sl, tvec);
    };
    const bool poll = eps_test && !async;
    std::vector<Scalars> out(n);
    auto all_halted = [&]() -> int {
        HIP_TRY(c, hipMemcpyAsync(out.data(), B.scal.ptr, sizeof(Scalars) * (size_t)n,
                                  hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        for (const Scalars& q : out)
            if (!q.halt) return 0;
        return 1;
    };
    if ((sp->flags & SP_FLAG_GRAPH) && sp->max_iter > 0) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        body();
        const hipError_t el0 = hipGetLastError();
        hipError_t ec = hipStreamEndCapture(st, &graph);
        if (ec == hipSuccess && el0 != hipSuccess) ec = el0;
        if (ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(c, SP_ERR_HIP, "capturing the batched loop body: %s", hipGetErrorString(ec));
        }
        hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(c, SP_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        }
        for (int it = 0; it < sp->max_iter; ++it) {
            hipError_t el = hipGraphLaunch(exec, st);
            if (el != hipSuccess) {
                (void)hipStreamSynchronize(st);
                (void)hipGraphExecDestroy(exec);
                (void)hipGraphDestroy(graph);
                return fail(c, SP_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString(el));
            }
            if (poll && (it & 7) == 7) {
                const int h = all_halted();
                if (h < 0 || h > 1) {
                    (void)hipGraphExecDestroy(exec);
                    (void)hipGraphDestroy(graph);
                    return h;
                }
                if (h) break;
            }
        }
        if (async) {
            c->pend_graph = graph;   // released once the stream has drained
            c->pend_exec = exec;
        } else {
            const hipError_t es = hipStreamSynchronize(st);
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            if (es != hipSuccess) return fail(c, SP_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(es));
        }
    } else {
        for (int it = 0; it < sp->max_iter; ++it) {
            body();
            if ((rc = check_launch(c))) return rc;
            if (poll && (it & 7) == 7) {
                const int h = all_halted();
                if (h > 1) return h;
                if (h) break;
            }
        }
    }
    c->last_kind = 2;
    c->last_count = n;
    c->last_eps = sp->eps;
    if (async) {
        for (int s = 0; s < n; ++s) {
            const SliceDev& S = B.hs[s];
            launch_finish(st, S.n, S.xh, S.x, dptr<Scalars>(B.scal) + s, k_out + s);
            launch_narrow(st, S.n, S.xh, x_out[s]);
            if (x_last && x_last[s]) launch_narrow(st, S.n, S.x, x_last[s]);
        }
        return check_launch(c);
    }
    HIP_TRY(c, hipMemcpyAsync(out.data(), B.scal.ptr, sizeof(Scalars) * (size_t)n, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    int first_err = SP_OK;
    std::vector<char> host;
    if (trace) {
        host.resize(tr_slice * (size_t)n);
        HIP_TRY(c, hipMemcpyAsync(host.data(), B.trace_d.ptr, host.size(), hipMemcpyDeviceToHost, st));
    }
    for (int s = 0; s < n; ++s) {
        const Scalars& q = out[s];
        k_out[s] = q.k;
        const int status = run_status(q, sp->eps);
        if (q.halt == SP_BREAKDOWN_CONVERGED && q.k > 1)
            HIP_TRY(c, hipMemcpyAsync(B.hs[s].x, B.hs[s].xh, (size_t)B.hs[s].n * 8, hipMemcpyDeviceToDevice, st));
        launch_narrow(st, B.hs[s].n, B.hs[s].xh, x_out[s]);
        if (x_last && x_last[s]) launch_narrow(st, B.hs[s].n, B.hs[s].x, x_last[s]);
        if (status < 16 && first_err == SP_OK) {
            first_err = status;
            fail(c, status, "slice %d: non-finite value in a CG scalar", s);
        }
        if (trace && trace->status) trace->status[s] = status;
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    if (trace && trace->cap > 0) {
        for (int s = 0; s < n; ++s) {
            const char* t = host.data() + tr_slice * s;
            const double* hf = reinterpret_cast<const double*>(t);
            const double* htv = hf + cap;
            const int32_t* hell = reinterpret_cast<const int32_t*>(htv + 4 * (size_t)cap);
            const int done = std::min(std::min(trace->cap, cap), out[s].iter);
            const size_t o = (size_t)s * trace->cap;
            if (trace->f_half) std::copy(hf, hf + done, trace->f_half + o);
            if (trace->tv_half) std::copy(htv, htv + done, trace->tv_half + o);
            if (trace->ell) std::copy(hell, hell + done, trace->ell + o);
        }
    }
    return first_err;
}

int sp_batch_tuning(sp_ctx* c, int32_t* out, int32_t count) {
    if (!c) return SP_ERR_ARG;
    if (!out || count < 2 * BS_SLICE) return fail(c, SP_ERR_ARG, "sp_batch_tuning: need 16 entries");
    for (int s = 0; s < BS_SLICE; ++s) {
        out[2 * s] = c->batch ? c->batch->order[s] : 0;
        out[2 * s + 1] = c->batch ? c->batch->wpc[s] : 0;
    }
    return SP_OK;
}

}  // extern "C"
