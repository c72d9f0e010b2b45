// C ABI of the library: argument validation, per-call constants, launch
// sequencing and filter handles.  Semantics of every entry point are stated
// in include/prism.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "launch.hpp"

using namespace prism;

namespace {

thread_local char g_err[512] = "";

prism_status fail(prism_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(PRISM_HIP_ERROR, "%s: %s (%d)", #expr, hipGetErrorString(e_), (int)e_); \
    } while (0)

#define REQUIRE(cond, ...)                                        \
    do {                                                          \
        if (!(cond)) return fail(PRISM_INVALID_ARGUMENT, __VA_ARGS__); \
    } while (0)

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// PRISM_CAPTURE_ERROR when `stream` is being captured into a graph (calls
// that wait on the host, record events they later query, or record graphs
// of their own cannot run inside a capture)
prism_status not_capturing(hipStream_t stream, const char* what) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cs));
    if (cs != hipStreamCaptureStatusNone) return fail(PRISM_CAPTURE_ERROR, "%s: stream is being captured", what);
    return PRISM_OK;
}

prism_status check_grid(const prism_grid* g) {
    REQUIRE(g, "grid is NULL");
    if (g->dtype != PRISM_F32 && g->dtype != PRISM_BF16)
        return fail(PRISM_UNSUPPORTED, "grid dtype %d unsupported (PRISM_F32 or PRISM_BF16)", g->dtype);
    if (g->n < 8 || g->n > 1024 || g->n % 8)
        return fail(PRISM_UNSUPPORTED, "grid n=%d unsupported (multiple of 8 in [8, 1024])", g->n);
    REQUIRE(isfinite(g->voxel) && g->voxel > 0, "grid voxel must be finite and > 0");
    REQUIRE(isfinite(g->origin[0]) && isfinite(g->origin[1]) && isfinite(g->origin[2]), "grid origin not finite");
    REQUIRE(isfinite(g->occ_out) && isfinite(g->rgb_out), "grid outside values not finite");
    const long long nb3 = (long long)(g->n / 8) * (g->n / 8) * (g->n / 8);
    REQUIRE(g->capacity >= 0 && g->capacity <= nb3, "grid capacity must be in [0, (n/8)^3]");
    return PRISM_OK;
}

prism_status check_cam(const prism_camera* c) {
    REQUIRE(c, "camera is NULL");
    if (c->width < 1 || c->height < 1 || c->width > 8192 || c->height > 8192)
        return fail(PRISM_UNSUPPORTED, "camera %dx%d unsupported (1..8192 each)", c->width, c->height);
    if (c->n_samples < 2 || c->n_samples > 4096)
        return fail(PRISM_UNSUPPORTED, "n_samples=%d unsupported (2..4096)", c->n_samples);
    REQUIRE(isfinite(c->fx) && isfinite(c->fy) && c->fx > 0 && c->fy > 0, "fx, fy must be finite and > 0");
    REQUIRE(isfinite(c->cx) && isfinite(c->cy), "cx, cy must be finite");
    REQUIRE(isfinite(c->d_near) && isfinite(c->d_far) && c->d_near >= 0 && c->d_far > c->d_near,
            "need 0 <= d_near < d_far (finite)");
    REQUIRE(isfinite(c->tau), "tau must be finite");
    return PRISM_OK;
}

prism_status check_weights(const prism_weights* w) {
    REQUIRE(w, "weights is NULL");
    REQUIRE(isfinite(w->w_depth) && isfinite(w->w_rgb) && w->w_depth >= 0 && w->w_rgb >= 0,
            "weights must be finite and >= 0");
    REQUIRE(!isnan(w->gate_depth) && !isnan(w->gate_rgb), "gates must not be NaN");
    return PRISM_OK;
}

// Constants of the single-precision recipe, formed from the double
// parameters exactly as the recipe states (see common.hpp).
GridC grid_c(const prism_grid* g) {
    GridC o;
    for (int i = 0; i < 3; ++i) o.o[i] = (float)g->origin[i];
    o.s = (float)g->voxel;
    o.inv_s = (float)(1.0 / g->voxel);
    o.occ_out = (float)g->occ_out;
    o.rgb_out = (float)g->rgb_out;
    o.n = g->n;
    o.nb = g->n / 8;
    o.nvox = (long long)g->n * g->n * g->n;
    o.table = nullptr;
    o.pocc = o.occ_out;
    o.prgb = o.rgb_out;
    return o;
}

// a single-precision value as the map's storage type holds it (BF16: round
// to nearest even, as the kernels store)
float stored_host(float v, int dtype) {
    if (dtype != PRISM_BF16) return v;
    uint32_t b;
    memcpy(&b, &v, 4);
    if ((b & 0x7fffffffu) > 0x7f800000u) {
        b = (b | 0x400000u) & 0xffff0000u;
    } else {
        b += 0x7fffu + ((b >> 16) & 1u);
        b &= 0xffff0000u;
    }
    float r;
    memcpy(&r, &b, 4);
    return r;
}

CamC cam_c(const prism_camera* c) {
    CamC o;
    o.ifx = (float)(1.0 / c->fx);
    o.ify = (float)(1.0 / c->fy);
    o.fx = (float)c->fx;
    o.fy = (float)c->fy;
    o.cx = (float)c->cx;
    o.cy = (float)c->cy;
    o.dn = (float)c->d_near;
    o.dstep = (float)((c->d_far - c->d_near) / (c->n_samples - 1));
    o.tau = (float)c->tau;
    o.W = c->width;
    o.H = c->height;
    o.K = c->n_samples;
    return o;
}

GridD grid_d(const prism_grid* g) {
    GridD o;
    for (int i = 0; i < 3; ++i) o.o[i] = g->origin[i];
    o.s = g->voxel;
    o.occ_out = g->occ_out;
    o.rgb_out = g->rgb_out;
    o.inv_s = 1.0 / g->voxel;
    return o;
}

CamD cam_d(const prism_camera* c) {
    CamD o;
    o.fx = c->fx;
    o.fy = c->fy;
    o.cx = c->cx;
    o.cy = c->cy;
    o.dn = c->d_near;
    o.step = (c->d_far - c->d_near) / (c->n_samples - 1);
    o.tau = c->tau;
    o.ifx = 1.0 / c->fx;
    o.ify = 1.0 / c->fy;
    return o;
}

WeightsC weights_c(const prism_weights* w) {
    return WeightsC{w->w_depth, w->w_rgb, w->gate_depth, w->gate_rgb, 0.0f, 0.0f, 1.0f, 1.0f, 0};
}

// the weights of an iteratively reweighted least-squares step of the L1
// objective: h = 1/(2b), f = floor * b with b = 1/sqrt(w) per row kind (a
// zero weight gives h = 0, a row that contributes nothing)
WeightsC weights_irls(const prism_weights* w, double floor) {
    WeightsC o = weights_c(w);
    const double bd = w->w_depth > 0 ? 1.0 / sqrt(w->w_depth) : 1.0;
    const double br = w->w_rgb > 0 ? 1.0 / sqrt(w->w_rgb) : 1.0;
    o.irls_h_depth = w->w_depth > 0 ? (float)(0.5 / bd) : 0.0f;
    o.irls_h_rgb = w->w_rgb > 0 ? (float)(0.5 / br) : 0.0f;
    o.irls_f_depth = (float)(floor * bd);
    o.irls_f_rgb = (float)(floor * br);
    o.irls = 1;
    return o;
}

size_t elem_size(int dtype) { return dtype == PRISM_BF16 ? 2 : 4; }

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// map buffer: 8 planes, then brick summary, free-space bits, update counts,
// frustum brick list, its segment lengths, pose scratch
struct MapLayout {
    size_t bmax, bits, counts, list, segcnt, pose, table, pool, total;
};

MapLayout map_layout(const prism_grid* g) {
    MapLayout L;
    size_t nvox = (size_t)g->n * g->n * g->n;
    size_t nb3 = nvox / 512;
    size_t nseg = (nb3 + 255) / 256;
    size_t plane = g->capacity > 0 ? (size_t)g->capacity * 512 : nvox;
    L.bmax = round_up(8 * plane * elem_size(g->dtype), 256);
    L.bits = L.bmax + round_up(4 * nb3, 256);
    L.counts = L.bits + round_up(8 * ((nb3 + 31) / 32), 256);   // plain and dilated bits
    L.list = L.counts + round_up(4 * (size_t)kUpdateGrid, 256);
    L.segcnt = L.list + round_up(4 * nseg * 256, 256);
    L.pose = L.segcnt + round_up(4 * nseg, 256);
    L.table = L.pose + 256;
    L.pool = L.table + (g->capacity > 0 ? round_up(4 * nb3, 256) : 0);
    L.total = L.pool + (g->capacity > 0 ? 256 : 0);
    return L;
}

MapAux map_aux(const prism_grid* g, const void* map) {
    MapLayout L = map_layout(g);
    char* b = (char*)map;
    MapAux a{(float*)(b + L.bmax), (unsigned*)(b + L.bits), (int*)(b + L.counts),
             (int*)(b + L.list),   (int*)(b + L.segcnt),    (void*)(b + L.pose)};
    a.table = nullptr;
    a.pool = nullptr;
    a.var0 = nullptr;
    a.capacity = 0;
    if (g->capacity > 0) {
        a.table = (int*)(b + L.table);
        a.pool = (int*)(b + L.pool);
        a.var0 = (float*)(b + L.pool + 8);
        a.capacity = (int)g->capacity;
    }
    return a;
}

// constants of a grid bound to one map buffer (brick-pool maps: the slot
// table, the pool's plane stride and the values of voxels without a slot)
GridC grid_cm(const prism_grid* g, const void* map) {
    GridC o = grid_c(g);
    if (g->capacity > 0) {
        o.table = map_aux(g, map).table;
        o.nvox = (long long)g->capacity * 512;
        o.pocc = stored_host(o.occ_out, g->dtype);
        o.prgb = stored_host(o.rgb_out, g->dtype);
    }
    return o;
}

// free-space bits for the renderer, NULL when skipping is not exact (tau != 0)
const unsigned* skip_table(const prism_grid* g, const prism_camera* c, const void* map) {
    return (float)c->tau == 0.0f ? map_aux(g, map).bits : nullptr;
}

size_t reduce_bytes(const CamC& c, int n_frames) {
    int nb = render_blocks(c) > track_blocks(c) ? render_blocks(c) : track_blocks(c);
    nb = nb > vjp_blocks(c) ? nb : vjp_blocks(c);
    return (size_t)nb * n_frames * PRISM_NEQ * sizeof(double);
}

// ---- stage timer (profiling aid for batched steps) -------------------------
// While armed, every batched step records an event pair around each stage's
// launch (up to `cap` pairs per stage); prism_stage_timer_read sums them.
struct StageTimer {
    std::mutex mu;
    bool armed = false;
    int cap = 0;
    std::vector<hipEvent_t> ev[PRISM_N_STAGES];   // pairs: begin, end
    int used[PRISM_N_STAGES] = {};
};
StageTimer g_timer;

// reserves the next event pair of `stage` when the timer is armed and the
// stream is not being captured into a graph
bool timer_pair(int s, hipStream_t st, hipEvent_t* b, hipEvent_t* e) {
    std::lock_guard<std::mutex> lk(g_timer.mu);
    if (!g_timer.armed || g_timer.used[s] >= g_timer.cap) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    int i = g_timer.used[s]++;
    *b = g_timer.ev[s][2 * i];
    *e = g_timer.ev[s][2 * i + 1];
    return true;
}

struct StageScope {
    hipStream_t st;
    hipEvent_t end_ev = nullptr;
    StageScope(int s, hipStream_t stream) : st(stream) {
        hipEvent_t b;
        if (timer_pair(s, stream, &b, &end_ev) && hipEventRecord(b, st) != hipSuccess) end_ev = nullptr;
    }
    ~StageScope() {
        if (end_ev) (void)hipEventRecord(end_ev, st);
    }
};


}  // namespace

// ---------------------------------------------------------------------------
// filter handle
// ---------------------------------------------------------------------------
struct prism_filter {
    prism_filter_cfg cfg;
    GridC g;
    CamC c;
    GridD gd;
    CamD cd;
    WeightsC w;
    WeightsC w_gn;   // rows of a Gauss-Newton iteration (the IRLS weights under PRISM_MODE_IRLS_L1, else w)
    TransC tc;
    double lap_h;    // factor of H in the Laplace precision (2, or 1 under PRISM_MODE_LAPLACE_FACTOR1)
    prism_filter_state* S;
    prism_filter_bias_state* X;   // the 15-D state's bias part (NULL without PRISM_MODE_ACCEL_BIAS)
    float *a_depth, *a_rgb, *a_normals;
    uint8_t *a_mask, *a_nmask;
    double* partials;
    Rel32* rel;   // relative pose of the iterate to the anchor (written by predict / GN)
    void* map;
    int64_t steps;
    prism_filter_state host_state;   // source of prism_filter_reset uploads
    prism_filter_bias_state host_bias;   // source of prism_filter_reset_bias uploads
    double min_inliers;              // contributing pixels below which a step raises PRISM_FLAG_LOW_INLIERS
    // checkpoint header staged on the host, and the event after its last copy
    alignas(64) unsigned char save_hdr[512];
    hipEvent_t save_done;
    // executable graphs of a full step, keyed by the frame's buffer addresses
    struct StepGraph {
        const void *depth, *rgb, *u;
        hipGraphExec_t exec;
        hipEvent_t done;            // recorded after each launch of exec
        hipStream_t last_stream;    // stream of the latest launch (NULL: never launched)
        uint64_t last_use;
    };
    static constexpr int kMaxGraphs = 4;
    StepGraph graphs[kMaxGraphs];
    int n_graphs;
    uint64_t graph_clock;
    // serving input slots (caller memory) and their completion events
    static constexpr int kMaxSlots = 4;
    prism_frame slots[kMaxSlots];
    hipEvent_t slot_done[kMaxSlots];
    int n_slots;
    int64_t submitted, completed;
    hipStream_t submit_stream;
    // descriptor for batched steps: host copy, its place in state_mem, and
    // whether the device copy is stale
    AgentDesc desc;
    AgentDesc* desc_dev;
    bool desc_dirty;
};

namespace {

// releases every recorded batched-step graph that has f as a member
hipError_t release_batch_graphs_of(const prism_filter* f);

// Waits for the graph's last launch, then frees it.  Every earlier launch is
// complete by then: a launch on a new stream first waits for the previous one.
hipError_t release_graph(prism_filter::StepGraph& G) {
    hipError_t e = hipEventSynchronize(G.done);
    (void)hipGraphExecDestroy(G.exec);
    (void)hipEventDestroy(G.done);
    return e;
}

struct StateLayout {
    size_t state, bias, a_depth, a_rgb, a_normals, a_mask, a_nmask, partials, rel, desc, total;
};

StateLayout state_layout(const prism_camera* c) {
    StateLayout L;
    size_t npix = (size_t)c->width * c->height;
    CamC cc = cam_c(c);
    size_t off = 0;
    L.state = off;
    off = round_up(off + sizeof(prism_filter_state), 256);
    L.bias = off;   // the 15-D state's bias part (kept for every filter, a few KB)
    off = round_up(off + sizeof(prism_filter_bias_state), 256);
    L.a_depth = off;
    off = round_up(off + 4 * npix, 256);
    L.a_rgb = off;
    off = round_up(off + 12 * npix, 256);
    L.a_normals = off;
    off = round_up(off + 12 * npix, 256);
    L.a_mask = off;
    off = round_up(off + npix, 256);
    L.a_nmask = off;
    off = round_up(off + npix, 256);
    L.partials = off;
    off = round_up(off + reduce_bytes(cc, 1), 256);
    L.rel = off;
    off = round_up(off + sizeof(Rel32), 256);
    L.desc = off;
    off = round_up(off + sizeof(AgentDesc), 256);
    L.total = off;
    return L;
}

prism_status check_cfg(const prism_filter_cfg* cfg) {
    REQUIRE(cfg, "cfg is NULL");
    prism_status s;
    if ((s = check_grid(&cfg->grid))) return s;
    if ((s = check_cam(&cfg->cam))) return s;
    if ((s = check_weights(&cfg->w))) return s;
    REQUIRE(isfinite(cfg->dt) && cfg->dt > 0, "dt must be > 0");
    REQUIRE(cfg->sigma_vel_t >= 0 && cfg->sigma_vel_r >= 0 && cfg->sigma_pose_t >= 0 && cfg->sigma_pose_r >= 0,
            "transition scales must be >= 0");
    REQUIRE(cfg->ema >= 0 && cfg->ema <= 1, "ema must be in [0, 1]");
    REQUIRE(cfg->n_gn >= 0 && cfg->n_gn <= 64, "n_gn must be in [0, 64]");
    REQUIRE(cfg->objective == PRISM_OBJ_P2 || cfg->objective == PRISM_OBJ_P1, "objective must be P2 or P1");
    REQUIRE(cfg->map.trunc > 0 && cfg->map.lam_update > 0, "map trunc and lam_update must be > 0");
    REQUIRE(!isnan(cfg->normal_disc), "normal_disc is NaN");
    REQUIRE(cfg->min_inlier_frac >= 0 && cfg->min_inlier_frac <= 1, "min_inlier_frac must be in [0, 1]");
    REQUIRE((cfg->modes & ~(PRISM_MODE_TRANSITION_DT2 | PRISM_MODE_LAPLACE_FACTOR1 | PRISM_MODE_IRLS_L1 |
                            PRISM_MODE_ACCEL_BIAS)) == 0,
            "unknown bits in modes (0x%x)", (unsigned)cfg->modes);
    REQUIRE(!(cfg->modes & PRISM_MODE_ACCEL_BIAS) ||
                (isfinite(cfg->sigma_bias) && cfg->sigma_bias >= 0 && isfinite(cfg->gravity[0]) &&
                 isfinite(cfg->gravity[1]) && isfinite(cfg->gravity[2])),
            "PRISM_MODE_ACCEL_BIAS needs a finite sigma_bias >= 0 and a finite gravity");
    REQUIRE(!(cfg->modes & PRISM_MODE_IRLS_L1) || (isfinite(cfg->irls_floor) && cfg->irls_floor > 0),
            "PRISM_MODE_IRLS_L1 needs a finite irls_floor > 0");
    return PRISM_OK;
}

prism_status check_frame(const prism_frame* fr, bool need_u) {
    REQUIRE(fr, "frame is NULL");
    REQUIRE(fr->depth && fr->rgb, "frame depth/rgb must be non-NULL");
    REQUIRE(aligned(fr->depth, 4) && aligned(fr->rgb, 4), "frame buffers must be 4-byte aligned");
    REQUIRE(!need_u || (fr->u && aligned(fr->u, 8)), "frame control u must be non-NULL and 8-byte aligned");
    return PRISM_OK;
}

// objective at S->iter into the handle's partials; returns the block count.
// rel_current: the handle's relative pose was formed from the current
// iterate (after predict or a Gauss-Newton step), so tracking reads it.
// gn: the rows of a Gauss-Newton iteration (reweighted under the L1 mode);
// else the rows of the Laplace covariance
prism_status eval_objective(prism_filter* f, const prism_frame* fr, int* nb, hipStream_t st,
                            bool rel_current = true, bool gn = false) {
    const WeightsC& w = gn ? f->w_gn : f->w;
    if (f->cfg.objective == PRISM_OBJ_P1) {
        HIP_TRY(launch_render_jac(f->g, f->c, f->gd, f->cd, f->cfg.grid.dtype, f->map,
                                  skip_table(&f->cfg.grid, &f->cfg.cam, f->map), &f->S->iter, 1, fr->depth,
                                  fr->rgb, w,
                                  nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, f->partials, st));
        *nb = render_blocks(f->c);
    } else {
        HIP_TRY(launch_track_p2(f->c, f->cd, &f->S->iter, &f->S->anchor, fr->depth, fr->rgb, f->a_depth, f->a_rgb,
                                f->a_mask, f->a_normals, f->a_nmask, w, nullptr, nullptr, nullptr, f->partials,
                                rel_current ? f->rel : nullptr, st));
        *nb = track_blocks(f->c);
    }
    return PRISM_OK;
}

prism_status pose_update_impl(prism_filter* f, const prism_frame* fr, hipStream_t st) {
    HIP_TRY(launch_predict(f->S, f->X, fr->u, f->tc, f->rel, st));
    int nb = 0;
    prism_status s;
    for (int i = 0; i < f->cfg.n_gn; ++i) {
        if ((s = eval_objective(f, fr, &nb, st, true, true))) return s;
        HIP_TRY(launch_gn_step(f->S, f->partials, nb, f->rel, st));
    }
    if ((s = eval_objective(f, fr, &nb, st))) return s;
    HIP_TRY(launch_laplace_combine(f->S, f->X, f->partials, nb, f->cfg.ema, f->min_inliers, f->lap_h, st));
    return PRISM_OK;
}

prism_status check_adam(const prism_filter* f, const prism_adam_params* p, const int32_t* pixels) {
    if (f->cfg.objective != PRISM_OBJ_P2)
        return fail(PRISM_UNSUPPORTED, "the Adam pose optimiser runs on the P2 objective only");
    if (f->cfg.modes & PRISM_MODE_IRLS_L1)
        return fail(PRISM_UNSUPPORTED, "the Adam pose optimiser does not run the IRLS-L1 objective");
    REQUIRE(p, "adam params are NULL");
    REQUIRE(p->n_steps >= 1 && p->n_steps <= 1000000, "adam n_steps must be in [1, 1000000]");
    REQUIRE(p->n_pixels >= 1 && p->n_pixels <= 65536, "adam n_pixels must be in [1, 65536]");
    REQUIRE(isfinite(p->lr_t) && p->lr_t >= 0 && isfinite(p->lr_r) && p->lr_r >= 0,
            "adam step sizes must be finite and >= 0");
    REQUIRE(p->beta2 >= 0 && p->beta2 < 1, "adam beta2 must be in [0, 1)");
    REQUIRE(isfinite(p->eps) && p->eps > 0, "adam eps must be finite and > 0");
    REQUIRE(pixels && aligned(pixels, 4), "pixels must be non-NULL and 4-byte aligned");
    return PRISM_OK;
}

prism_status pose_update_adam_impl(prism_filter* f, const prism_frame* fr, const prism_adam_params* p,
                                   const int32_t* pixels, hipStream_t st) {
    HIP_TRY(launch_predict(f->S, f->X, fr->u, f->tc, f->rel, st));
    AdamC ad;
    for (int i = 0; i < 3; ++i) {
        ad.lr[i] = p->lr_t;
        ad.lr[3 + i] = p->lr_r;
    }
    ad.beta2 = p->beta2;
    ad.eps = p->eps;
    ad.scale = (double)f->c.W * (double)f->c.H / (double)p->n_pixels;
    ad.n_steps = p->n_steps;
    ad.n_pix = p->n_pixels;
    HIP_TRY(launch_pose_adam(f->S, f->c, f->cd, fr->depth, fr->rgb, f->a_depth, f->a_rgb, f->a_mask, f->a_normals,
                             f->a_nmask, f->w, pixels, ad, st));
    int nb = 0;
    prism_status s;
    // the optimiser moved the iterate: the objective forms its own relative pose
    if ((s = eval_objective(f, fr, &nb, st, false))) return s;
    HIP_TRY(launch_laplace_combine(f->S, f->X, f->partials, nb, f->cfg.ema, f->min_inliers, f->lap_h, st));
    return PRISM_OK;
}

prism_status map_and_anchor(prism_filter* f, const prism_frame* fr, hipStream_t st) {
    // the update's count of voxels is totalled by the normals kernel at the end
    MapAux aux = map_aux(&f->cfg.grid, f->map);
    hipEvent_t tb = nullptr, te = nullptr;
    if (!timer_pair(PRISM_STAGE_MAP_UPDATE, st, &tb, &te)) tb = te = nullptr;
    HIP_TRY(launch_map_update(f->g, f->c, f->gd, f->cfg.grid.dtype, f->map, &f->S->pose, fr->depth, fr->rgb,
                              f->cfg.map.trunc, f->cfg.map.lam_update, aux, nullptr, st, tb, te));
    HIP_TRY(launch_render(f->g, f->c, f->gd, f->cd, f->cfg.grid.dtype, f->map,
                          skip_table(&f->cfg.grid, &f->cfg.cam, f->map), &f->S->pose, 1, f->a_depth, f->a_rgb,
                          f->a_mask, nullptr, st));
    HIP_TRY(launch_normals(f->c, 1, f->a_depth, f->a_mask, (float)f->cfg.normal_disc, f->a_normals, f->a_nmask,
                           aux.counts, map_update_groups(f->g), &f->S->n_updated, &f->S->n_updated_total, st));
    return PRISM_OK;
}

}  // namespace

extern "C" {

const char* prism_last_error(void) { return g_err; }

const char* prism_version(void) { return "prism-mi355x 0.1 (gfx950)"; }

size_t prism_sizeof(const char* name) {
    if (!name) return 0;
    struct { const char* n; size_t s; } t[] = {
        {"prism_grid", sizeof(prism_grid)},         {"prism_camera", sizeof(prism_camera)},
        {"prism_pose", sizeof(prism_pose)},         {"prism_weights", sizeof(prism_weights)},
        {"prism_map_params", sizeof(prism_map_params)}, {"prism_filter_cfg", sizeof(prism_filter_cfg)},
        {"prism_filter_state", sizeof(prism_filter_state)},
        {"prism_filter_bias_state", sizeof(prism_filter_bias_state)}, {"prism_frame", sizeof(prism_frame)},
        {"prism_adam_params", sizeof(prism_adam_params)}};
    for (auto& e : t)
        if (!strcmp(e.n, name)) return e.s;
    return 0;
}

prism_status prism_map_bytes(const prism_grid* grid, size_t* bytes) {
    prism_status s = check_grid(grid);
    if (s) return s;
    REQUIRE(bytes, "bytes is NULL");
    *bytes = map_layout(grid).total;
    return PRISM_OK;
}

prism_status prism_map_init(const prism_grid* grid, void* map, float occ0, float rgb0, float var0,
                            hipStream_t stream) {
    prism_status s = check_grid(grid);
    if (s) return s;
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(grid->capacity == 0 || (occ0 == (float)grid->occ_out && rgb0 == (float)grid->rgb_out),
            "a brick-pool map must be initialised with occ0 == occ_out and rgb0 == rgb_out");
    HIP_TRY(launch_map_init(grid_cm(grid, map), grid->dtype, map, occ0, rgb0, var0, map_aux(grid, map), stream));
    return PRISM_OK;
}

prism_status prism_map_pool_usage(const prism_grid* grid, const void* map, int32_t* usage, hipStream_t stream) {
    prism_status s = check_grid(grid);
    if (s) return s;
    if (grid->capacity == 0) return fail(PRISM_UNSUPPORTED, "map_pool_usage needs a brick-pool map");
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(usage && aligned(usage, 4), "usage must be non-NULL and 4-byte aligned");
    HIP_TRY(hipMemcpyAsync(usage, map_aux(grid, map).pool, 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
    return PRISM_OK;
}

prism_status prism_map_from_dense(const prism_grid* grid, void* map, const float* mean4, const float* var4,
                                  hipStream_t stream) {
    prism_status s = check_grid(grid);
    if (s) return s;
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    if (grid->capacity > 0) return fail(PRISM_UNSUPPORTED, "map_from_dense needs a dense map");
    REQUIRE(!mean4 || aligned(mean4, 4), "mean4 misaligned");
    REQUIRE(!var4 || aligned(var4, 4), "var4 misaligned");
    if (!mean4 && !var4) return PRISM_OK;
    HIP_TRY(launch_from_dense(grid_cm(grid, map), grid->dtype, map, mean4, var4, map_aux(grid, map), stream));
    return PRISM_OK;
}

prism_status prism_map_refresh(const prism_grid* grid, void* map, hipStream_t stream) {
    prism_status s = check_grid(grid);
    if (s) return s;
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    HIP_TRY(launch_brick_max(grid_cm(grid, map), grid->dtype, map, map_aux(grid, map), stream));
    return PRISM_OK;
}

prism_status prism_map_to_dense(const prism_grid* grid, const void* map, float* mean4, float* var4,
                                hipStream_t stream) {
    prism_status s = check_grid(grid);
    if (s) return s;
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(!mean4 || aligned(mean4, 4), "mean4 misaligned");
    REQUIRE(!var4 || aligned(var4, 4), "var4 misaligned");
    if (!mean4 && !var4) return PRISM_OK;
    HIP_TRY(launch_to_dense(grid_cm(grid, map), grid->dtype, map, mean4, var4, map_aux(grid, map), stream));
    return PRISM_OK;
}

static prism_status planes(int32_t n, int32_t channels, const float* src, float* dst, int to_dense,
                           hipStream_t stream) {
    if (n < 8 || n > 1024 || n % 8) return fail(PRISM_UNSUPPORTED, "n=%d unsupported (multiple of 8 in [8, 1024])", n);
    REQUIRE(channels >= 1 && channels <= 8, "channels must be in [1, 8]");
    REQUIRE(src && dst && aligned(src, 4) && aligned(dst, 4), "src/dst must be non-NULL and 4-byte aligned");
    REQUIRE(src != dst, "src and dst must not alias");
    HIP_TRY(launch_planes(n, channels, src, dst, to_dense, stream));
    return PRISM_OK;
}

prism_status prism_bricks_to_dense(int32_t n, int32_t channels, const float* bricks, float* dense,
                                   hipStream_t stream) {
    return planes(n, channels, bricks, dense, 1, stream);
}

prism_status prism_dense_to_bricks(int32_t n, int32_t channels, const float* dense, float* bricks,
                                   hipStream_t stream) {
    return planes(n, channels, dense, bricks, 0, stream);
}

prism_status prism_camera_paper_sampling(prism_camera* cam, double voxel, double max_depth) {
    REQUIRE(cam, "camera is NULL");
    REQUIRE(isfinite(voxel) && voxel > 0 && isfinite(max_depth) && max_depth > 0,
            "voxel and max_depth must be finite and > 0");
    // App. B: offsets eps, 2 eps, ...; App. G: eps = 0.4 voxel, up to the maximum depth
    const double eps = 0.4 * voxel;
    const double k = floor(max_depth / eps);
    if (k < 2 || k > 4096)
        return fail(PRISM_UNSUPPORTED, "%.0f samples of %g m up to %g m (2..4096 supported)", k, eps, max_depth);
    cam->d_near = eps;
    cam->n_samples = (int32_t)k;
    cam->d_far = k * eps;
    return PRISM_OK;
}

prism_status prism_render(const prism_grid* grid, const void* map, const prism_camera* cam, const prism_pose* poses,
                          int32_t n_frames, float* depth, float* rgb, uint8_t* mask, int32_t* hit_k, float* normals,
                          uint8_t* nmask, double normal_disc, hipStream_t stream) {
    prism_status s;
    if ((s = check_grid(grid)) || (s = check_cam(cam))) return s;
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(poses && aligned(poses, 8), "poses must be non-NULL and 8-byte aligned");
    REQUIRE(n_frames >= 1 && n_frames <= 65535, "n_frames must be in [1, 65535]");
    REQUIRE(depth && rgb && mask, "depth, rgb, mask must be non-NULL");
    REQUIRE(aligned(depth, 4) && aligned(rgb, 4) && (!hit_k || aligned(hit_k, 4)), "outputs misaligned");
    REQUIRE(!normals || (nmask && aligned(normals, 4)), "normals needs nmask (and 4-byte alignment)");
    REQUIRE(!normals || !isnan(normal_disc), "normal_disc is NaN");
    CamC c = cam_c(cam);
    HIP_TRY(launch_render(grid_cm(grid, map), c, grid_d(grid), cam_d(cam), grid->dtype, map, skip_table(grid, cam, map),
                          poses, n_frames, depth, rgb, mask, hit_k, stream));
    if (normals)
        HIP_TRY(launch_normals(c, n_frames, depth, mask, (float)normal_disc, normals, nmask, nullptr, 0, nullptr,
                               nullptr, stream));
    return PRISM_OK;
}

prism_status prism_reduce_workspace_bytes(const prism_camera* cam, int32_t n_frames, size_t* bytes) {
    prism_status s = check_cam(cam);
    if (s) return s;
    REQUIRE(n_frames >= 1 && n_frames <= 65535, "n_frames must be in [1, 65535]");
    REQUIRE(bytes, "bytes is NULL");
    *bytes = reduce_bytes(cam_c(cam), n_frames);
    return PRISM_OK;
}

prism_status prism_render_jacobian(const prism_grid* grid, const void* map, const prism_camera* cam,
                                   const prism_pose* poses, int32_t n_frames, const float* obs_depth,
                                   const float* obs_rgb, const prism_weights* w, float* depth, float* rgb,
                                   uint8_t* mask, float* J, float* resid, uint8_t* rowmask, double* neq,
                                   void* workspace, size_t workspace_bytes, hipStream_t stream) {
    prism_status s;
    if ((s = check_grid(grid)) || (s = check_cam(cam)) || (s = check_weights(w))) return s;
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(poses && aligned(poses, 8), "poses must be non-NULL and 8-byte aligned");
    REQUIRE(n_frames >= 1 && n_frames <= 65535, "n_frames must be in [1, 65535]");
    REQUIRE(obs_depth && obs_rgb && aligned(obs_depth, 4) && aligned(obs_rgb, 4), "observations must be non-NULL, aligned");
    REQUIRE(neq && aligned(neq, 8), "neq must be non-NULL and 8-byte aligned");
    REQUIRE((!J || aligned(J, 16)) && (!resid || aligned(resid, 16)), "J and resid must be 16-byte aligned");
    REQUIRE((!depth || aligned(depth, 4)) && (!rgb || aligned(rgb, 4)), "outputs misaligned");
    CamC c = cam_c(cam);
    REQUIRE(workspace && aligned(workspace, 8) && workspace_bytes >= reduce_bytes(c, n_frames),
            "workspace too small: need %zu bytes", reduce_bytes(c, n_frames));
    double* part = (double*)workspace;
    HIP_TRY(launch_render_jac(grid_cm(grid, map), c, grid_d(grid), cam_d(cam), grid->dtype, map,
                              skip_table(grid, cam, map), poses, n_frames, obs_depth, obs_rgb, weights_c(w),
                              depth, rgb, mask, J, resid, rowmask, part, stream));
    HIP_TRY(launch_finalize(part, render_blocks(c), n_frames, PRISM_NEQ, neq, PRISM_NEQ, stream));
    return PRISM_OK;
}

}  // extern "C"

// ---- render Jacobian without a workspace argument --------------------------
// The per-workgroup partial sums of prism_render_jacobian_noalloc live in this
// file-scope device array (one copy per GPU, held until the process ends).  In
// host code its name is only a stand-in: the device address of each GPU's copy
// is looked up once per device with hipGetSymbolAddress and used from then on.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// device address of the current device's copy of `scratch`
prism_status scratch_address(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PRISM_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PRISM_HIP_ERROR, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return PRISM_OK;
}

}  // namespace

extern "C" {

size_t prism_render_jacobian_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

prism_status prism_render_jacobian_noalloc(const prism_grid* grid, const void* map, const prism_camera* cam,
                                           const prism_pose* poses, int32_t n_frames, const float* obs_depth,
                                           const float* obs_rgb, const prism_weights* w, float* depth, float* rgb,
                                           uint8_t* mask, float* J, float* resid, uint8_t* rowmask, double* neq,
                                           hipStream_t stream) {
    prism_status s;
    if ((s = check_grid(grid)) || (s = check_cam(cam)) || (s = check_weights(w))) return s;
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(poses && aligned(poses, 8), "poses must be non-NULL and 8-byte aligned");
    REQUIRE(n_frames >= 1 && n_frames <= 65535, "n_frames must be in [1, 65535]");
    REQUIRE(obs_depth && obs_rgb && aligned(obs_depth, 4) && aligned(obs_rgb, 4), "observations must be non-NULL, aligned");
    REQUIRE(neq && aligned(neq, 8), "neq must be non-NULL and 8-byte aligned");
    REQUIRE((!J || aligned(J, 16)) && (!resid || aligned(resid, 16)), "J and resid must be 16-byte aligned");
    REQUIRE((!depth || aligned(depth, 4)) && (!rgb || aligned(rgb, 4)), "outputs misaligned");
    CamC c = cam_c(cam);
    const size_t need = (size_t)render_blocks(c) * n_frames * PRISM_NEQ * sizeof(double);
    REQUIRE(need <= kNoAllocScratchBytes,
            "render_jacobian_noalloc: %d frames of %dx%d need %zu bytes of partial sums, more than the %zu-byte "
            "scratch array (use prism_render_jacobian with a workspace)",
            n_frames, cam->width, cam->height, need, kNoAllocScratchBytes);
    void* part = nullptr;
    if ((s = scratch_address(&part))) return s;
    // every workgroup writes its own row of partial sums: nothing to clear
    HIP_TRY(launch_render_jac(grid_cm(grid, map), c, grid_d(grid), cam_d(cam), grid->dtype, map,
                              skip_table(grid, cam, map), poses, n_frames, obs_depth, obs_rgb, weights_c(w),
                              depth, rgb, mask, J, resid, rowmask, (double*)part, stream));
    HIP_TRY(launch_finalize((const double*)part, render_blocks(c), n_frames, PRISM_NEQ, neq, PRISM_NEQ, stream));
    return PRISM_OK;
}

prism_status prism_track_p2(const prism_camera* cam, const prism_pose* pose, const prism_pose* pose_prev,
                            const float* obs_depth, const float* obs_rgb, const float* anchor_depth,
                            const float* anchor_rgb, const uint8_t* anchor_mask, const float* anchor_normals,
                            const uint8_t* anchor_nmask, const prism_weights* w, float* J, float* resid,
                            uint8_t* rowmask, double* neq, void* workspace, size_t workspace_bytes,
                            hipStream_t stream) {
    prism_status s;
    if ((s = check_cam(cam)) || (s = check_weights(w))) return s;
    REQUIRE(pose && pose_prev && aligned(pose, 8) && aligned(pose_prev, 8), "poses must be non-NULL and aligned");
    REQUIRE(obs_depth && obs_rgb && aligned(obs_depth, 4) && aligned(obs_rgb, 4), "observations must be non-NULL, aligned");
    REQUIRE(anchor_depth && anchor_rgb && anchor_mask && anchor_normals && anchor_nmask, "anchor buffers must be non-NULL");
    REQUIRE(aligned(anchor_depth, 4) && aligned(anchor_rgb, 4) && aligned(anchor_normals, 4), "anchor buffers misaligned");
    REQUIRE(neq && aligned(neq, 8), "neq must be non-NULL and 8-byte aligned");
    REQUIRE((!J || aligned(J, 16)) && (!resid || aligned(resid, 16)), "J and resid must be 16-byte aligned");
    CamC c = cam_c(cam);
    REQUIRE(workspace && aligned(workspace, 8) && workspace_bytes >= reduce_bytes(c, 1),
            "workspace too small: need %zu bytes", reduce_bytes(c, 1));
    double* part = (double*)workspace;
    HIP_TRY(launch_track_p2(c, cam_d(cam), pose, pose_prev, obs_depth, obs_rgb, anchor_depth, anchor_rgb, anchor_mask,
                            anchor_normals, anchor_nmask, weights_c(w), J, resid, rowmask, part, nullptr, stream));
    HIP_TRY(launch_finalize(part, track_blocks(c), 1, PRISM_NEQ, neq, PRISM_NEQ, stream));
    return PRISM_OK;
}

prism_status prism_render_vjp(const prism_grid* grid, const void* map, const prism_camera* cam,
                              const prism_pose* poses, int32_t n_frames, const int32_t* hit_k, const float* g_depth,
                              const float* g_rgb, float* grad_mean, double* grad_pose, void* workspace,
                              size_t workspace_bytes, hipStream_t stream) {
    prism_status s;
    if ((s = check_grid(grid)) || (s = check_cam(cam))) return s;
    if (grid->dtype != PRISM_F32 || grid->capacity > 0)
        return fail(PRISM_UNSUPPORTED, "render_vjp needs a dense FP32 map");
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(poses && aligned(poses, 8), "poses must be non-NULL and 8-byte aligned");
    REQUIRE(n_frames >= 1 && n_frames <= 65535, "n_frames must be in [1, 65535]");
    REQUIRE(hit_k && g_depth && g_rgb && grad_mean && grad_pose, "inputs and outputs must be non-NULL");
    REQUIRE(aligned(hit_k, 4) && aligned(g_depth, 4) && aligned(g_rgb, 4) && aligned(grad_mean, 4) &&
                aligned(grad_pose, 8),
            "buffers misaligned");
    CamC c = cam_c(cam);
    REQUIRE(workspace && aligned(workspace, 8) && workspace_bytes >= reduce_bytes(c, n_frames),
            "workspace too small: need %zu bytes", reduce_bytes(c, n_frames));
    double* part = (double*)workspace;
    HIP_TRY(launch_render_vjp(grid_c(grid), c, grid_d(grid), cam_d(cam), (const float*)map, poses, n_frames, hit_k, g_depth, g_rgb, grad_mean,
                              part, stream));
    HIP_TRY(launch_finalize(part, vjp_blocks(c), n_frames, 6, grad_pose, 6, stream));
    return PRISM_OK;
}

prism_status prism_map_update(const prism_grid* grid, void* map, const prism_camera* cam, const prism_pose* pose,
                              const float* obs_depth, const float* obs_rgb, const prism_map_params* p,
                              int64_t* n_updated, hipStream_t stream) {
    prism_status s;
    if ((s = check_grid(grid)) || (s = check_cam(cam))) return s;
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(pose && aligned(pose, 8), "pose must be non-NULL and 8-byte aligned");
    REQUIRE(obs_depth && obs_rgb && aligned(obs_depth, 4) && aligned(obs_rgb, 4), "observations must be non-NULL, aligned");
    REQUIRE(p && isfinite(p->trunc) && p->trunc > 0 && isfinite(p->lam_update) && p->lam_update > 0,
            "map params: trunc and lam_update must be finite and > 0");
    REQUIRE(!n_updated || aligned(n_updated, 8), "n_updated misaligned");
    hipEvent_t tb = nullptr, te = nullptr;
    if (!timer_pair(PRISM_STAGE_MAP_UPDATE, stream, &tb, &te)) tb = te = nullptr;
    HIP_TRY(launch_map_update(grid_cm(grid, map), cam_c(cam), grid_d(grid), grid->dtype, map, pose, obs_depth, obs_rgb,
                              p->trunc, p->lam_update, map_aux(grid, map), n_updated, stream, tb, te));
    return PRISM_OK;
}

// descent-mapping workspace: gradient accumulators (double), the means of
// every stepped brick before the run, brick marks, cost partials
struct GdLayout {
    size_t grad, save, marks, saved, list, pd, pp, total;
    int words;
};

GdLayout gd_layout(const prism_grid* g, const prism_camera* cam) {
    GdLayout L;
    size_t nvox = (size_t)g->n * g->n * g->n;
    size_t nb3 = nvox / 512;
    L.words = (int)((nb3 + 31) / 32);
    L.grad = 0;
    L.save = round_up(4 * nvox * sizeof(double), 256);
    L.marks = L.save + round_up(4 * nvox * sizeof(float), 256);
    L.saved = L.marks + round_up(4 * (size_t)L.words, 256);
    L.list = L.saved + round_up(4 * (size_t)L.words, 256);
    L.pd = L.list + round_up(4 * (nb3 + 1), 256);
    L.pp = L.pd + round_up(sizeof(double) * (size_t)render_blocks(cam_c(cam)), 256);
    L.total = L.pp + round_up(sizeof(double) * (size_t)gd_update_groups(grid_c(g)), 256);
    return L;
}

prism_status prism_map_gd_workspace_bytes(const prism_grid* grid, const prism_camera* cam, size_t* bytes) {
    prism_status s;
    if ((s = check_grid(grid)) || (s = check_cam(cam))) return s;
    REQUIRE(bytes, "bytes is NULL");
    *bytes = gd_layout(grid, cam).total;
    return PRISM_OK;
}

prism_status prism_map_gd(const prism_grid* grid, void* map, const prism_camera* cam, const prism_pose* pose,
                          const float* obs_depth, const float* obs_rgb, const prism_weights* w, double lr_occ,
                          double lr_rgb, int32_t n_iters, double* cost, void* workspace, size_t workspace_bytes,
                          hipStream_t stream) {
    prism_status s;
    if ((s = check_grid(grid)) || (s = check_cam(cam)) || (s = check_weights(w))) return s;
    if (grid->dtype != PRISM_F32 || grid->capacity > 0)
        return fail(PRISM_UNSUPPORTED, "map_gd needs a dense FP32 map");
    REQUIRE(map && aligned(map, 256), "map must be non-NULL and 256-byte aligned");
    REQUIRE(pose && aligned(pose, 8), "pose must be non-NULL and 8-byte aligned");
    REQUIRE(obs_depth && obs_rgb && aligned(obs_depth, 4) && aligned(obs_rgb, 4), "observations must be non-NULL, aligned");
    REQUIRE(isfinite(lr_occ) && lr_occ >= 0 && isfinite(lr_rgb) && lr_rgb >= 0, "step sizes must be finite and >= 0");
    REQUIRE(n_iters >= 0, "n_iters must be >= 0");
    REQUIRE(!cost || aligned(cost, 8), "cost misaligned");
    GdLayout L = gd_layout(grid, cam);
    REQUIRE(workspace && aligned(workspace, 256) && workspace_bytes >= L.total,
            "workspace must be 256-byte aligned and hold %zu bytes", L.total);
    if (n_iters == 0) return PRISM_OK;
    char* ws = (char*)workspace;
    double* grad = (double*)(ws + L.grad);
    float* save = (float*)(ws + L.save);
    unsigned* marks = (unsigned*)(ws + L.marks);
    unsigned* saved = (unsigned*)(ws + L.saved);
    int* list = (int*)(ws + L.list);
    double* pd = (double*)(ws + L.pd);
    double* pp = (double*)(ws + L.pp);
    GridC g = grid_c(grid);
    CamC c = cam_c(cam);
    GridD gd = grid_d(grid);
    CamD cd = cam_d(cam);
    WeightsC wc = weights_c(w);
    MapAux aux = map_aux(grid, map);
    const unsigned* bits = skip_table(grid, cam, map);
    HIP_TRY(launch_gd_clear(marks, L.words, stream));
    HIP_TRY(launch_gd_clear(saved, L.words, stream));
    HIP_TRY(launch_gd_clear((unsigned*)list, 1, stream));
    for (int it = 0; it < n_iters; ++it) {
        HIP_TRY(launch_gd_grad(g, c, gd, cd, (const float*)map, bits, pose, obs_depth, obs_rgb, wc, grad, marks, list,
                               pd, stream));
        HIP_TRY(launch_gd_update(g, (float*)map, aux, save, grad, list, saved, lr_occ, lr_rgb, pp, stream));
        if (cost)
            HIP_TRY(launch_gd_cost(pd, render_blocks(c), pp, gd_update_groups(g), cost + it, stream));
    }
    return PRISM_OK;
}

prism_status prism_filter_bytes(const prism_filter_cfg* cfg, size_t* bytes) {
    prism_status s = check_cfg(cfg);
    if (s) return s;
    REQUIRE(bytes, "bytes is NULL");
    *bytes = state_layout(&cfg->cam).total;
    return PRISM_OK;
}

prism_status prism_filter_create(const prism_filter_cfg* cfg, void* state_mem, void* map_mem, prism_filter** out) {
    prism_status s = check_cfg(cfg);
    if (s) return s;
    REQUIRE(state_mem && aligned(state_mem, 256), "state_mem must be non-NULL and 256-byte aligned");
    REQUIRE(map_mem && aligned(map_mem, 256), "map_mem must be non-NULL and 256-byte aligned");
    REQUIRE(out, "out is NULL");
    prism_filter* f = new (std::nothrow) prism_filter();
    if (!f) return fail(PRISM_INVALID_ARGUMENT, "out of host memory");
    f->cfg = *cfg;
    f->g = grid_cm(&cfg->grid, map_mem);
    f->c = cam_c(&cfg->cam);
    f->gd = grid_d(&cfg->grid);
    f->cd = cam_d(&cfg->cam);
    f->w = weights_c(&cfg->w);
    f->w_gn = (cfg->modes & PRISM_MODE_IRLS_L1) ? weights_irls(&cfg->w, cfg->irls_floor) : f->w;
    f->lap_h = (cfg->modes & PRISM_MODE_LAPLACE_FACTOR1) ? 1.0 : 2.0;
    f->tc.dt = cfg->dt;
    f->tc.du = (cfg->modes & PRISM_MODE_TRANSITION_DT2) ? cfg->dt * cfg->dt : cfg->dt;
    const bool bias = (cfg->modes & PRISM_MODE_ACCEL_BIAS) != 0;
    for (int i = 0; i < 3; ++i) {
        f->tc.q[i] = cfg->sigma_pose_t * cfg->sigma_pose_t;
        f->tc.q[3 + i] = cfg->sigma_pose_r * cfg->sigma_pose_r;
        f->tc.q[6 + i] = cfg->sigma_vel_t * cfg->sigma_vel_t;
        f->tc.q[9 + i] = cfg->sigma_vel_r * cfg->sigma_vel_r;
        f->tc.q[12 + i] = bias ? cfg->sigma_bias * cfg->sigma_bias : 0.0;
        f->tc.g[i] = bias ? cfg->gravity[i] : 0.0;
    }
    StateLayout L = state_layout(&cfg->cam);
    char* base = (char*)state_mem;
    f->S = (prism_filter_state*)(base + L.state);
    f->X = bias ? (prism_filter_bias_state*)(base + L.bias) : nullptr;
    f->a_depth = (float*)(base + L.a_depth);
    f->a_rgb = (float*)(base + L.a_rgb);
    f->a_normals = (float*)(base + L.a_normals);
    f->a_mask = (uint8_t*)(base + L.a_mask);
    f->a_nmask = (uint8_t*)(base + L.a_nmask);
    f->partials = (double*)(base + L.partials);
    f->rel = (Rel32*)(base + L.rel);
    f->map = map_mem;
    f->steps = 0;
    // batched-step descriptor (slots are filled in by prism_filter_set_slots)
    AgentDesc& D = f->desc;
    D.g = f->g;
    D.c = f->c;
    D.gd = f->gd;
    D.cd = f->cd;
    D.w = f->w;
    D.w_irls = f->w_gn;
    D.tc = f->tc;
    D.lap_h = f->lap_h;
    D.mp = MapUpdC{(float)cfg->map.trunc, cfg->map.trunc, cfg->map.lam_update};
    D.aux = map_aux(&cfg->grid, map_mem);
    D.ema = cfg->ema;
    f->min_inliers = ceil(cfg->min_inlier_frac * (double)cfg->cam.width * (double)cfg->cam.height);
    D.min_inliers = f->min_inliers;
    D.normal_disc = (float)cfg->normal_disc;
    D.dtype = cfg->grid.dtype;
    D.n_gn = cfg->n_gn;
    D.nseg = (f->g.nb * f->g.nb * f->g.nb + 255) / 256;
    D.upd_groups = map_update_groups_batch(f->g);
    D.obj_blocks = cfg->objective == PRISM_OBJ_P1 ? render_blocks(f->c) : track_blocks(f->c);
    D.map = map_mem;
    D.bits = skip_table(&cfg->grid, &cfg->cam, map_mem);
    D.S = f->S;
    D.X = f->X;
    D.a_depth = f->a_depth;
    D.a_rgb = f->a_rgb;
    D.a_normals = f->a_normals;
    D.a_mask = f->a_mask;
    D.a_nmask = f->a_nmask;
    D.partials = f->partials;
    D.rel = f->rel;
    f->desc_dev = (AgentDesc*)(base + L.desc);
    f->desc_dirty = true;
    *out = f;
    return PRISM_OK;
}

prism_status prism_filter_destroy(prism_filter* f) {
    if (!f) return PRISM_OK;
    hipError_t e = hipSuccess;
    for (int i = 0; i < f->n_slots; ++i) {
        hipError_t ei = hipEventSynchronize(f->slot_done[i]);
        if (e == hipSuccess) e = ei;
        (void)hipEventDestroy(f->slot_done[i]);
    }
    for (int i = 0; i < f->n_graphs; ++i) {
        hipError_t ei = release_graph(f->graphs[i]);
        if (e == hipSuccess) e = ei;
    }
    if (f->save_done) {
        hipError_t ei = hipEventSynchronize(f->save_done);
        if (e == hipSuccess) e = ei;
        (void)hipEventDestroy(f->save_done);
    }
    {
        hipError_t ei = release_batch_graphs_of(f);
        if (e == hipSuccess) e = ei;
    }
    delete f;
    if (e != hipSuccess) return fail(PRISM_HIP_ERROR, "releasing step graphs: %s", hipGetErrorString(e));
    return PRISM_OK;
}

prism_status prism_filter_reset(prism_filter* f, const double* x0, const double* P0, hipStream_t stream) {
    REQUIRE(f && x0 && P0, "filter, x0 and P0 must be non-NULL");
    if (f->X) return fail(PRISM_UNSUPPORTED, "the filter has the 15-D state: use prism_filter_reset_bias");
    for (int i = 0; i < 13; ++i) REQUIRE(isfinite(x0[i]), "x0 not finite");
    for (int i = 0; i < 144; ++i) REQUIRE(isfinite(P0[i]), "P0 not finite");
    prism_filter_state& h = f->host_state;
    memset(&h, 0, sizeof h);
    for (int i = 0; i < 3; ++i) h.pose.t[i] = x0[i];
    for (int i = 0; i < 4; ++i) h.pose.q[i] = x0[3 + i];
    for (int i = 0; i < 3; ++i) {
        h.v[i] = x0[7 + i];
        h.w[i] = x0[10 + i];
    }
    memcpy(h.P, P0, sizeof h.P);
    h.anchor = h.pose;
    h.prior = h.pose;
    h.iter = h.pose;
    HIP_TRY(hipMemcpyAsync(f->S, &h, sizeof h, hipMemcpyHostToDevice, stream));
    f->steps = 0;
    return PRISM_OK;
}

prism_status prism_filter_reset_bias(prism_filter* f, const double* x0, const double* P0, hipStream_t stream) {
    REQUIRE(f && x0 && P0, "filter, x0 and P0 must be non-NULL");
    if (!f->X) return fail(PRISM_UNSUPPORTED, "prism_filter_reset_bias needs PRISM_MODE_ACCEL_BIAS");
    for (int i = 0; i < 16; ++i) REQUIRE(isfinite(x0[i]), "x0 not finite");
    for (int i = 0; i < 225; ++i) REQUIRE(isfinite(P0[i]), "P0 not finite");
    prism_filter_state& h = f->host_state;
    memset(&h, 0, sizeof h);
    for (int i = 0; i < 3; ++i) h.pose.t[i] = x0[i];
    for (int i = 0; i < 4; ++i) h.pose.q[i] = x0[3 + i];
    for (int i = 0; i < 3; ++i) {
        h.v[i] = x0[7 + i];
        h.w[i] = x0[10 + i];
    }
    for (int i = 0; i < 144; ++i) h.P[i] = P0[(i / 12) * 15 + i % 12];
    h.anchor = h.pose;
    h.prior = h.pose;
    h.iter = h.pose;
    prism_filter_bias_state& hb = f->host_bias;
    memset(&hb, 0, sizeof hb);
    for (int i = 0; i < 3; ++i) hb.b[i] = x0[13 + i];
    memcpy(hb.P, P0, sizeof hb.P);
    HIP_TRY(hipMemcpyAsync(f->S, &h, sizeof h, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(f->X, &hb, sizeof hb, hipMemcpyHostToDevice, stream));
    f->steps = 0;
    return PRISM_OK;
}

prism_status prism_pose_update(prism_filter* f, const prism_frame* frame, hipStream_t stream) {
    REQUIRE(f, "filter is NULL");
    prism_status s = check_frame(frame, true);
    if (s) return s;
    REQUIRE(f->steps > 0, "pose_update needs a filter past its first frame");
    return pose_update_impl(f, frame, stream);
}

prism_status prism_pose_update_adam(prism_filter* f, const prism_frame* frame, const prism_adam_params* p,
                                    const int32_t* pixels, hipStream_t stream) {
    REQUIRE(f, "filter is NULL");
    prism_status s = check_frame(frame, true);
    if (s) return s;
    if ((s = check_adam(f, p, pixels))) return s;
    REQUIRE(f->steps > 0, "pose_update_adam needs a filter past its first frame");
    return pose_update_adam_impl(f, frame, p, pixels, stream);
}

prism_status prism_filter_step_adam(prism_filter* f, const prism_frame* frame, const prism_adam_params* p,
                                    const int32_t* pixels, hipStream_t stream) {
    REQUIRE(f, "filter is NULL");
    prism_status s = check_frame(frame, f->steps > 0);
    if (s) return s;
    if ((s = check_adam(f, p, pixels))) return s;
    if (f->steps == 0) {
        if ((s = map_and_anchor(f, frame, stream))) return s;
        HIP_TRY(launch_first_frame(f->S, stream));
    } else {
        if ((s = pose_update_adam_impl(f, frame, p, pixels, stream))) return s;
        if ((s = map_and_anchor(f, frame, stream))) return s;
    }
    f->steps += 1;
    return PRISM_OK;
}

prism_status prism_rollout(prism_filter* f, const double* u, int32_t k, int32_t n_samples, const double* noise,
                           prism_pose* poses, double* mean, double* cov, float* depth, float* rgb, uint8_t* mask,
                           int32_t* flags, hipStream_t stream) {
    REQUIRE(f, "filter is NULL");
    REQUIRE(k >= 1 && k <= 4096, "k must be in [1, 4096]");
    REQUIRE(n_samples >= 0 && n_samples <= 65535, "n_samples must be in [0, 65535]");
    REQUIRE(u && aligned(u, 8), "controls u must be non-NULL and 8-byte aligned");
    REQUIRE(n_samples == 0 || (noise && poses && aligned(noise, 8) && aligned(poses, 8)),
            "sampling needs noise and poses (8-byte aligned)");
    REQUIRE((!mean || aligned(mean, 8)) && (!cov || aligned(cov, 8)) && (!flags || aligned(flags, 4)),
            "outputs misaligned");
    const bool frames = depth || rgb || mask;
    REQUIRE(!frames || (depth && rgb && mask && aligned(depth, 4) && aligned(rgb, 4)),
            "depth, rgb and mask go together (4-byte aligned)");
    REQUIRE(!frames || (n_samples >= 1 && (long long)n_samples * k <= 65535),
            "rendering needs 1 <= n_samples * k <= 65535");
    HIP_TRY(launch_rollout(f->S, f->X, u, k, n_samples, noise, f->tc, poses, mean, cov, flags, stream));
    if (frames)
        HIP_TRY(launch_render(f->g, f->c, f->gd, f->cd, f->cfg.grid.dtype, f->map,
                              skip_table(&f->cfg.grid, &f->cfg.cam, f->map), poses, n_samples * k, depth, rgb, mask,
                              nullptr, stream));
    return PRISM_OK;
}

namespace {

prism_status step_one(prism_filter* f, const prism_frame* fr, hipStream_t stream) {
    prism_status s;
    if (f->steps == 0) {
        if ((s = map_and_anchor(f, fr, stream))) return s;
        HIP_TRY(launch_first_frame(f->S, stream));
    } else {
        if ((s = pose_update_impl(f, fr, stream))) return s;
        if ((s = map_and_anchor(f, fr, stream))) return s;
    }
    f->steps += 1;
    return PRISM_OK;
}

prism_status check_batch(prism_filter* const* fs, int32_t n, const prism_frame* frames) {
    REQUIRE(fs && frames && n >= 1, "need n >= 1 filters and frames");
    for (int i = 0; i < n; ++i) {
        REQUIRE(fs[i], "filter %d is NULL", i);
        prism_status s = check_frame(&frames[i], fs[i]->steps > 0);
        if (s) return s;
    }
    return PRISM_OK;
}

// Records the steady-state step (state filter, map update, anchor) of f for
// the buffers of fr into an executable graph.
prism_status capture_step(prism_filter* f, const prism_frame* fr, hipStream_t stream, hipGraphExec_t* out) {
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(PRISM_CAPTURE_ERROR, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    prism_status s = pose_update_impl(f, fr, stream);
    if (!s) s = map_and_anchor(f, fr, stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(stream, &g);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return fail(PRISM_CAPTURE_ERROR, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PRISM_CAPTURE_ERROR, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return PRISM_OK;
}

prism_status graph_for(prism_filter* f, const prism_frame* fr, hipStream_t stream, int* out) {
    f->graph_clock += 1;
    for (int i = 0; i < f->n_graphs; ++i) {
        prism_filter::StepGraph& G = f->graphs[i];
        if (G.depth == fr->depth && G.rgb == fr->rgb && G.u == fr->u) {
            G.last_use = f->graph_clock;
            *out = i;
            return PRISM_OK;
        }
    }
    hipEvent_t done = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    hipGraphExec_t ex = nullptr;
    prism_status s = capture_step(f, fr, stream, &ex);
    if (s) {
        (void)hipEventDestroy(done);
        return s;
    }
    int slot = f->n_graphs;
    if (slot == prism_filter::kMaxGraphs) {
        slot = 0;
        for (int i = 1; i < f->n_graphs; ++i)
            if (f->graphs[i].last_use < f->graphs[slot].last_use) slot = i;
        hipError_t e = release_graph(f->graphs[slot]);   // the evicted graph may still be running
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(ex);
            (void)hipEventDestroy(done);
            f->n_graphs -= 1;
            f->graphs[slot] = f->graphs[f->n_graphs];
            return fail(PRISM_HIP_ERROR, "releasing an evicted step graph: %s", hipGetErrorString(e));
        }
    } else {
        f->n_graphs += 1;
    }
    f->graphs[slot] = {fr->depth, fr->rgb, fr->u, ex, done, nullptr, f->graph_clock};
    *out = slot;
    return PRISM_OK;
}

}  // namespace

prism_status prism_filter_step(prism_filter* const* fs, int32_t n, const prism_frame* frames, hipStream_t stream) {
    prism_status s = check_batch(fs, n, frames);
    if (s) return s;
    for (int i = 0; i < n; ++i)
        if ((s = step_one(fs[i], &frames[i], stream))) return s;
    return PRISM_OK;
}

prism_status prism_filter_step_graph(prism_filter* const* fs, int32_t n, const prism_frame* frames,
                                     hipStream_t stream) {
    prism_status s = check_batch(fs, n, frames);
    if (s) return s;
    REQUIRE(stream != nullptr, "graph-replayed steps need a non-default stream");
    prism_status cst = not_capturing(stream, "prism_filter_step_graph (use prism_filter_step inside a capture)");
    if (cst) return cst;
    for (int i = 0; i < n; ++i) {
        prism_filter* f = fs[i];
        if (f->steps == 0) {
            if ((s = step_one(f, &frames[i], stream))) return s;
            continue;
        }
        int slot = -1;
        if ((s = graph_for(f, &frames[i], stream, &slot))) return s;
        prism_filter::StepGraph& G = f->graphs[slot];
        if (G.last_stream && G.last_stream != stream) HIP_TRY(hipEventSynchronize(G.done));
        HIP_TRY(hipGraphLaunch(G.exec, stream));
        HIP_TRY(hipEventRecord(G.done, stream));
        G.last_stream = stream;
        f->steps += 1;
    }
    return PRISM_OK;
}

prism_status prism_filter_set_slots(prism_filter* f, int32_t n_slots, const prism_frame* slots) {
    REQUIRE(f, "filter is NULL");
    REQUIRE(n_slots >= 1 && n_slots <= prism_filter::kMaxSlots, "n_slots must be in [1, %d]", prism_filter::kMaxSlots);
    REQUIRE(slots, "slots is NULL");
    for (int i = 0; i < n_slots; ++i)
        REQUIRE(slots[i].depth && slots[i].rgb && slots[i].u && aligned(slots[i].depth, 16) &&
                    aligned(slots[i].rgb, 16) && aligned(slots[i].u, 16),
                "slot %d: depth, rgb and u must be non-NULL and 16-byte aligned", i);
    for (int i = 0; i < f->n_slots; ++i) {
        HIP_TRY(hipEventSynchronize(f->slot_done[i]));
        HIP_TRY(hipEventDestroy(f->slot_done[i]));
    }
    f->n_slots = 0;
    for (int i = 0; i < n_slots; ++i) {
        f->slots[i] = slots[i];
        f->desc.slots[i] = slots[i];
        HIP_TRY(hipEventCreateWithFlags(&f->slot_done[i], hipEventDisableTiming));
        f->n_slots = i + 1;
    }
    f->desc_dirty = true;
    f->submitted = f->completed = 0;
    f->submit_stream = nullptr;
    return PRISM_OK;
}

namespace {

prism_status poll_impl(prism_filter* f) {
    while (f->completed < f->submitted) {
        hipError_t q = hipEventQuery(f->slot_done[f->completed % f->n_slots]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return fail(PRISM_HIP_ERROR, "hipEventQuery: %s", hipGetErrorString(q));
        f->completed += 1;
    }
    return PRISM_OK;
}

}  // namespace

prism_status prism_filter_submit(prism_filter* f, const prism_frame* src, int32_t flags, hipStream_t stream,
                                 int64_t* seq) {
    REQUIRE(f, "filter is NULL");
    REQUIRE(f->n_slots > 0, "no input slots: call prism_filter_set_slots first");
    REQUIRE(stream != nullptr, "submission needs a non-default stream");
    if (prism_status cst = not_capturing(stream, "prism_filter_submit")) return cst;
    REQUIRE(!f->submit_stream || f->completed == f->submitted || f->submit_stream == stream,
            "all in-flight submissions of a handle must use one stream");
    prism_status s = check_frame(src, f->steps > 0);
    if (s) return s;
    if ((s = poll_impl(f))) return s;
    if (f->submitted - f->completed >= f->n_slots) return fail(PRISM_BUSY, "every input slot is in flight");
    const int k = (int)(f->submitted % f->n_slots);
    const prism_frame& slot = f->slots[k];
    const size_t npix = (size_t)f->cfg.cam.width * f->cfg.cam.height;
    if (flags & PRISM_SUBMIT_FROM_HOST) {
        // slot buffers are caller-owned writable memory (prism_frame holds const pointers)
        HIP_TRY(hipMemcpyAsync((void*)slot.depth, src->depth, 4 * npix, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync((void*)slot.rgb, src->rgb, 12 * npix, hipMemcpyHostToDevice, stream));
        if (src->u) HIP_TRY(hipMemcpyAsync((void*)slot.u, src->u, 48, hipMemcpyHostToDevice, stream));
    } else {
        HIP_TRY(launch_stage(src->depth, src->rgb, src->u, (float*)slot.depth, (float*)slot.rgb, (double*)slot.u,
                             (long long)npix, stream));
    }
    prism_frame fr{slot.depth, slot.rgb, src->u ? slot.u : nullptr};
    if (f->steps == 0 || (flags & PRISM_SUBMIT_EAGER)) {
        if ((s = step_one(f, &fr, stream))) return s;
    } else {
        int g = -1;
        if ((s = graph_for(f, &fr, stream, &g))) return s;
        prism_filter::StepGraph& G = f->graphs[g];
        if (G.last_stream && G.last_stream != stream) HIP_TRY(hipEventSynchronize(G.done));
        HIP_TRY(hipGraphLaunch(G.exec, stream));
        HIP_TRY(hipEventRecord(G.done, stream));
        G.last_stream = stream;
        f->steps += 1;
    }
    HIP_TRY(hipEventRecord(f->slot_done[k], stream));
    f->submit_stream = stream;
    if (seq) *seq = f->submitted;
    f->submitted += 1;
    return PRISM_OK;
}

prism_status prism_stage_timer_arm(int32_t cap) {
    REQUIRE(cap >= 0 && cap <= 1 << 16, "cap must be in [0, 65536]");
    std::lock_guard<std::mutex> lk(g_timer.mu);
    for (int s = 0; s < PRISM_N_STAGES; ++s) {
        while ((int)g_timer.ev[s].size() < 2 * cap) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            g_timer.ev[s].push_back(e);
        }
        g_timer.used[s] = 0;
    }
    g_timer.cap = cap;
    g_timer.armed = cap > 0;
    return PRISM_OK;
}

prism_status prism_stage_timer_read(double* ms, int64_t* launches) {
    REQUIRE(ms && launches, "ms and launches must be non-NULL");
    std::lock_guard<std::mutex> lk(g_timer.mu);
    g_timer.armed = false;
    for (int s = 0; s < PRISM_N_STAGES; ++s) {
        double t = 0.0;
        for (int i = 0; i < g_timer.used[s]; ++i) {
            HIP_TRY(hipEventSynchronize(g_timer.ev[s][2 * i + 1]));
            float e = 0.0f;
            HIP_TRY(hipEventElapsedTime(&e, g_timer.ev[s][2 * i], g_timer.ev[s][2 * i + 1]));
            t += e;
        }
        ms[s] = t;
        launches[s] = g_timer.used[s];
        g_timer.used[s] = 0;
    }
    return PRISM_OK;
}

namespace {

// block counts of one filter for each batched stage
int blocks_of(const prism_filter* f, int stage) {
    const CamC& c = f->c;
    switch (stage) {
        case 0: return stage_blocks(c);
        case 1: return 1;                                    // predict, GN, Laplace, first frame
        case 2: return track_blocks(c);
        case 3: return f->desc.nseg;                         // cull
        case 4: return f->desc.upd_groups;                   // update
        case 5: return render_blocks(c);
        case 7: return (free_words(f->g.nb) + 255) / 256;   // dilated free-space bits
        case 8: return render_blocks(c);                     // render-through objective
        default: return (c.W * c.H + 255) / 256;             // normals
    }
}

// kernel argument for `stage` over the filters fs[i] (i in idx[0..m)) with
// the given slots
BatchArgs make_batch(prism_filter* const* fs, const int* idx, int m, const int* slot, int stage) {
    BatchArgs b;
    b.n = m;
    b.irls = 0;
    b.start[0] = 0;
    for (int j = 0; j < m; ++j) {
        const prism_filter* f = fs[idx[j]];
        b.d[j] = f->desc_dev;
        b.slot[j] = (unsigned char)slot[idx[j]];
        b.start[j + 1] = b.start[j] + blocks_of(f, stage);
    }
    for (int j = m; j < kMaxBatch; ++j) {
        b.d[j] = nullptr;
        b.slot[j] = 0;
        b.start[j + 1] = b.start[m];
    }
    return b;
}

// the objective of every filter fs[idx[j]] at its iterate: one tracking
// launch for the P2 filters, one render-through launch per map kind for the
// P1 filters; gn: the rows of a Gauss-Newton iteration (each filter's
// reweighted rows under the L1 mode), else those of the Laplace covariance
prism_status batch_objective(prism_filter* const* fs, const int* idx, int m, const int* slot, hipStream_t st,
                             bool gn = false) {
    int p2[kMaxBatch], n2 = 0;
    for (int j = 0; j < m; ++j)
        if (fs[idx[j]]->cfg.objective == PRISM_OBJ_P2) p2[n2++] = idx[j];
    if (n2) {
        StageScope t(PRISM_STAGE_TRACK, st);
        BatchArgs b = make_batch(fs, p2, n2, slot, 2);
        b.irls = gn ? 1 : 0;
        HIP_TRY(launch_track_p2_batch(b, st));
    }
    for (int kind = 0; kind < 4 && n2 < m; ++kind) {
        const int dt = kind & 1 ? PRISM_BF16 : PRISM_F32;
        const bool pool = kind >= 2;
        int p1[kMaxBatch], n1 = 0, max_lds = 0;
        for (int j = 0; j < m; ++j) {
            const prism_filter* f = fs[idx[j]];
            if (f->cfg.objective != PRISM_OBJ_P1 || f->cfg.grid.dtype != dt || (f->cfg.grid.capacity > 0) != pool)
                continue;
            p1[n1++] = idx[j];
            int words = f->desc.bits ? free_lds_words(free_words(f->g.nb)) : 0;
            if (words > max_lds) max_lds = words;
        }
        if (!n1) continue;
        StageScope t(PRISM_STAGE_TRACK, st);
        BatchArgs b = make_batch(fs, p1, n1, slot, 8);
        b.irls = gn ? 1 : 0;
        HIP_TRY(launch_render_jac_batch(b, dt, pool, max_lds, st));
    }
    return PRISM_OK;
}

// one batched step for up to kMaxBatch filters already staged into slot[i]
prism_status step_batch_chunk(prism_filter* const* fs, int n, const int* slot, hipStream_t st) {
    int all[kMaxBatch], pu[kMaxBatch], ff[kMaxBatch], sub[kMaxBatch];
    int n_all = 0, n_pu = 0, n_ff = 0, max_gn = 0;
    for (int i = 0; i < n; ++i) {
        all[n_all++] = i;
        if (fs[i]->steps == 0) {
            ff[n_ff++] = i;
        } else {
            pu[n_pu++] = i;
            if (fs[i]->cfg.n_gn > max_gn) max_gn = fs[i]->cfg.n_gn;
        }
    }
    if (n_pu) {
        {
            StageScope t(PRISM_STAGE_PREDICT, st);
            HIP_TRY(launch_predict_batch(make_batch(fs, pu, n_pu, slot, 1), st));
        }
        for (int it = 0; it < max_gn; ++it) {
            int m = 0;
            for (int j = 0; j < n_pu; ++j)
                if (fs[pu[j]]->cfg.n_gn > it) sub[m++] = pu[j];
            prism_status so = batch_objective(fs, sub, m, slot, st, true);
            if (so) return so;
            {
                StageScope t(PRISM_STAGE_GN, st);
                HIP_TRY(launch_gn_step_batch(make_batch(fs, sub, m, slot, 1), st));
            }
        }
        prism_status so = batch_objective(fs, pu, n_pu, slot, st);
        if (so) return so;
        {
            StageScope t(PRISM_STAGE_LAPLACE, st);
            HIP_TRY(launch_laplace_combine_batch(make_batch(fs, pu, n_pu, slot, 1), st));
        }
    }
    {
        StageScope t(PRISM_STAGE_CULL, st);
        HIP_TRY(launch_cull_batch(make_batch(fs, all, n_all, slot, 3), st));
    }
    for (int kind = 0; kind < 4; ++kind) {
        const int dt = kind & 1 ? PRISM_BF16 : PRISM_F32;
        const bool pool = kind >= 2;
        int m = 0, max_nseg = 0, max_lds = 0;
        for (int j = 0; j < n_all; ++j) {
            const prism_filter* f = fs[all[j]];
            if (f->cfg.grid.dtype != dt || (f->cfg.grid.capacity > 0) != pool) continue;
            sub[m++] = all[j];
            if (f->desc.nseg > max_nseg) max_nseg = f->desc.nseg;
            int words = f->desc.bits ? free_lds_words(free_words(f->g.nb)) : 0;
            if (words > max_lds) max_lds = words;
        }
        if (!m) continue;
        {
            StageScope t(PRISM_STAGE_MAP_UPDATE, st);
            HIP_TRY(launch_map_update_batch(make_batch(fs, sub, m, slot, 4), dt, pool, max_nseg, st));
            HIP_TRY(launch_dilate_batch(make_batch(fs, sub, m, slot, 7), st));
        }
        {
            StageScope t(PRISM_STAGE_RENDER, st);
            HIP_TRY(launch_render_batch(make_batch(fs, sub, m, slot, 5), dt, pool, max_lds, st));
        }
    }
    {
        StageScope t(PRISM_STAGE_NORMALS, st);
        HIP_TRY(launch_normals_batch(make_batch(fs, all, n_all, slot, 6), st));
    }
    if (n_ff) {
        StageScope t(PRISM_STAGE_FIRST_FRAME, st);
        HIP_TRY(launch_first_frame_batch(make_batch(fs, ff, n_ff, slot, 1), st));
    }
    return PRISM_OK;
}

// ---- batched steps replayed from HIP graphs ---------------------------------
// A batched step's launches depend only on its members (their descriptors,
// which the kernels read at run time, and their block ranges), each member's
// input slot and whether it is on its first frame: a graph recorded for that
// key replays the step for any later frames staged into the same slots.
struct BatchGraph {
    std::vector<const prism_filter*> fs;
    std::vector<int> slot;
    std::vector<char> first;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;          // recorded after each launch
    hipStream_t last_stream = nullptr;  // stream of the latest launch (NULL: never launched)
    uint64_t last_use = 0;
};

constexpr size_t kMaxBatchGraphs = 64;
std::mutex g_bg_mu;
std::vector<BatchGraph*> g_bg;
uint64_t g_bg_clock = 0;

hipError_t free_batch_graph(BatchGraph* G) {
    hipError_t e = G->done ? hipEventSynchronize(G->done) : hipSuccess;
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->done) (void)hipEventDestroy(G->done);
    delete G;
    return e;
}

hipError_t release_batch_graphs_of(const prism_filter* f) {
    std::lock_guard<std::mutex> lk(g_bg_mu);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < g_bg.size();) {
        BatchGraph* G = g_bg[i];
        bool has = false;
        for (const prism_filter* m : G->fs) has |= m == f;
        if (!has) {
            ++i;
            continue;
        }
        hipError_t ei = free_batch_graph(G);
        if (e == hipSuccess) e = ei;
        g_bg.erase(g_bg.begin() + i);
    }
    return e;
}

// records the batched step of fs[0..n) with these slots into a graph
prism_status capture_batch(prism_filter* const* fs, int n, const int* slot, hipStream_t st, hipGraphExec_t* out) {
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(PRISM_CAPTURE_ERROR, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    prism_status s = step_batch_chunk(fs, n, slot, st);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return fail(PRISM_CAPTURE_ERROR, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PRISM_CAPTURE_ERROR, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return PRISM_OK;
}

// the batched step of fs[0..n) launched from its graph (recorded on first use)
prism_status step_batch_graph(prism_filter* const* fs, int n, const int* slot, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_bg_mu);
    g_bg_clock += 1;
    BatchGraph* G = nullptr;
    for (BatchGraph* c : g_bg) {
        if ((int)c->fs.size() != n) continue;
        bool same = true;
        for (int i = 0; i < n && same; ++i)
            same = c->fs[i] == fs[i] && c->slot[i] == slot[i] && c->first[i] == (fs[i]->steps == 0);
        if (same) {
            G = c;
            break;
        }
    }
    if (!G) {
        if (g_bg.size() >= kMaxBatchGraphs) {
            size_t lru = 0;
            for (size_t i = 1; i < g_bg.size(); ++i)
                if (g_bg[i]->last_use < g_bg[lru]->last_use) lru = i;
            BatchGraph* old = g_bg[lru];
            g_bg.erase(g_bg.begin() + lru);
            hipError_t e = free_batch_graph(old);   // waits for its last launch
            if (e != hipSuccess) return fail(PRISM_HIP_ERROR, "releasing a batched-step graph: %s", hipGetErrorString(e));
        }
        G = new (std::nothrow) BatchGraph();
        if (!G) return fail(PRISM_INVALID_ARGUMENT, "out of host memory");
        for (int i = 0; i < n; ++i) {
            G->fs.push_back(fs[i]);
            G->slot.push_back(slot[i]);
            G->first.push_back(fs[i]->steps == 0);
        }
        hipError_t e = hipEventCreateWithFlags(&G->done, hipEventDisableTiming);
        prism_status s = e == hipSuccess ? capture_batch(fs, n, slot, st, &G->exec)
                                         : fail(PRISM_HIP_ERROR, "hipEventCreate: %s", hipGetErrorString(e));
        if (s) {
            (void)free_batch_graph(G);
            return s;
        }
        g_bg.push_back(G);
    }
    G->last_use = g_bg_clock;
    // a graph never runs concurrently with itself
    if (G->last_stream && G->last_stream != st) HIP_TRY(hipEventSynchronize(G->done));
    HIP_TRY(hipGraphLaunch(G->exec, st));
    HIP_TRY(hipEventRecord(G->done, st));
    G->last_stream = st;
    return PRISM_OK;
}

}  // namespace

prism_status prism_filter_step_batch(prism_filter* const* fs, int32_t n, const prism_frame* src, int32_t flags,
                                     hipStream_t stream) {
    REQUIRE(fs && src && n >= 1, "need n >= 1 filters and frames");
    REQUIRE(stream != nullptr, "batched steps need a non-default stream");
    if (prism_status cst = not_capturing(stream, "prism_filter_step_batch")) return cst;
    prism_status s;
    for (int i = 0; i < n; ++i) {
        prism_filter* f = fs[i];
        REQUIRE(f, "filter %d is NULL", i);
        REQUIRE(f->n_slots > 0, "filter %d has no input slots (prism_filter_set_slots)", i);
        REQUIRE(!f->submit_stream || f->completed == f->submitted || f->submit_stream == stream,
                "filter %d: all in-flight submissions of a handle must use one stream", i);
        for (int j = 0; j < i; ++j) REQUIRE(fs[j] != f, "filter %d appears twice in the batch", i);
        if ((s = check_frame(&src[i], f->steps > 0))) return s;
        if ((s = poll_impl(f))) return s;
        if (f->submitted - f->completed >= f->n_slots)
            return fail(PRISM_BUSY, "filter %d: every input slot is in flight", i);
    }
    int slot[kMaxBatch];
    for (int c0 = 0; c0 < n; c0 += kMaxBatch) {
        const int m = n - c0 < kMaxBatch ? n - c0 : kMaxBatch;
        prism_filter* const* fc = fs + c0;
        const prism_frame* sc = src + c0;
        StageSrc ss;
        int dev_idx[kMaxBatch], n_dev = 0;
        for (int i = 0; i < m; ++i) {
            prism_filter* f = fc[i];
            slot[i] = (int)(f->submitted % f->n_slots);
            if (f->desc_dirty) {
                HIP_TRY(hipMemcpyAsync(f->desc_dev, &f->desc, sizeof(AgentDesc), hipMemcpyHostToDevice, stream));
                f->desc_dirty = false;
            }
            const prism_frame& sl = f->slots[slot[i]];
            if (flags & PRISM_SUBMIT_FROM_HOST) {
                const size_t npix = (size_t)f->cfg.cam.width * f->cfg.cam.height;
                HIP_TRY(hipMemcpyAsync((void*)sl.depth, sc[i].depth, 4 * npix, hipMemcpyHostToDevice, stream));
                HIP_TRY(hipMemcpyAsync((void*)sl.rgb, sc[i].rgb, 12 * npix, hipMemcpyHostToDevice, stream));
                if (sc[i].u) HIP_TRY(hipMemcpyAsync((void*)sl.u, sc[i].u, 48, hipMemcpyHostToDevice, stream));
            } else {
                ss.depth[n_dev] = sc[i].depth;
                ss.rgb[n_dev] = sc[i].rgb;
                ss.u[n_dev] = sc[i].u;
                dev_idx[n_dev++] = i;
            }
        }
        if (n_dev) {
            for (int j = n_dev; j < kMaxBatch; ++j) ss.depth[j] = ss.rgb[j] = ss.u[j] = nullptr;
            StageScope t(PRISM_STAGE_STAGING, stream);
            HIP_TRY(launch_stage_batch(make_batch(fc, dev_idx, n_dev, slot, 0), ss, stream));
        }
        if ((s = (flags & PRISM_SUBMIT_GRAPH) ? step_batch_graph(fc, m, slot, stream)
                                              : step_batch_chunk(fc, m, slot, stream)))
            return s;
        for (int i = 0; i < m; ++i) {
            prism_filter* f = fc[i];
            HIP_TRY(hipEventRecord(f->slot_done[slot[i]], stream));
            f->steps += 1;
            f->submitted += 1;
            f->submit_stream = stream;
        }
    }
    return PRISM_OK;
}

prism_status prism_filter_poll_batch(prism_filter* const* fs, int32_t n, int64_t* completed) {
    REQUIRE(fs && completed && n >= 0, "filters and completed must be non-NULL");
    for (int i = 0; i < n; ++i) {
        REQUIRE(fs[i], "filter %d is NULL", i);
        prism_status s = poll_impl(fs[i]);
        if (s) return s;
        completed[i] = fs[i]->completed;
    }
    return PRISM_OK;
}

prism_status prism_filter_poll(prism_filter* f, int64_t* completed) {
    REQUIRE(f && completed, "filter and completed must be non-NULL");
    prism_status s = poll_impl(f);
    if (s) return s;
    *completed = f->completed;
    return PRISM_OK;
}

}  // extern "C"

// ---- checkpoints -------------------------------------------------------------
namespace {

// Checkpoint layout: this header (512 bytes), then the state buffer's bytes
// [0, partials) (state struct and anchor frame), then [rel, desc) (relative
// pose of the iterate), then the whole map buffer.  The reduction partials
// are scratch and the batched-step descriptor holds the handle's own device
// addresses, so neither is saved.
struct CkptHeader {
    char magic[8];
    uint32_t version, header_bytes;
    prism_grid grid;
    prism_camera cam;
    int64_t steps;
    uint64_t state_bytes, rel_bytes, map_bytes;
    int32_t state_dim;   // 12, or 15 with the accelerometer bias
};
static_assert(sizeof(CkptHeader) <= 512, "checkpoint header exceeds its 512 bytes");
constexpr char kCkptMagic[8] = {'P', 'R', 'I', 'S', 'M', 'C', 'K', '1'};
constexpr uint32_t kCkptVersion = 2;
constexpr size_t kCkptHeader = 512;

size_t ckpt_bytes(const prism_filter_cfg* cfg, StateLayout* Lout = nullptr) {
    StateLayout L = state_layout(&cfg->cam);
    if (Lout) *Lout = L;
    return kCkptHeader + L.partials + (L.desc - L.rel) + map_layout(&cfg->grid).total;
}

bool same_grid(const prism_grid& a, const prism_grid& b) {
    return a.n == b.n && a.dtype == b.dtype && a.voxel == b.voxel && a.origin[0] == b.origin[0] &&
           a.origin[1] == b.origin[1] && a.origin[2] == b.origin[2] && a.occ_out == b.occ_out &&
           a.rgb_out == b.rgb_out && a.capacity == b.capacity;
}

bool same_cam(const prism_camera& a, const prism_camera& b) {
    return a.width == b.width && a.height == b.height && a.fx == b.fx && a.fy == b.fy && a.cx == b.cx &&
           a.cy == b.cy && a.d_near == b.d_near && a.d_far == b.d_far && a.n_samples == b.n_samples &&
           a.tau == b.tau;
}

}  // namespace

extern "C" {

prism_status prism_filter_save_bytes(const prism_filter_cfg* cfg, size_t* bytes) {
    prism_status s = check_cfg(cfg);
    if (s) return s;
    REQUIRE(bytes, "bytes is NULL");
    *bytes = ckpt_bytes(cfg);
    return PRISM_OK;
}

prism_status prism_filter_save(prism_filter* f, void* dst, size_t dst_bytes, hipStream_t stream) {
    REQUIRE(f, "filter is NULL");
    StateLayout L;
    const size_t need = ckpt_bytes(&f->cfg, &L);
    REQUIRE(dst && aligned(dst, 16) && dst_bytes >= need, "dst must be 16-byte aligned and hold %zu bytes", need);
    const size_t mbytes = map_layout(&f->cfg.grid).total;
    // the staged header may still be the source of the previous save's copy
    if (f->save_done) {
        HIP_TRY(hipEventSynchronize(f->save_done));
    } else {
        HIP_TRY(hipEventCreateWithFlags(&f->save_done, hipEventDisableTiming));
    }
    CkptHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, kCkptMagic, 8);
    h.version = kCkptVersion;
    h.state_dim = f->X ? 15 : 12;
    h.header_bytes = (uint32_t)kCkptHeader;
    h.grid = f->cfg.grid;
    h.cam = f->cfg.cam;
    h.steps = f->steps;
    h.state_bytes = L.partials;
    h.rel_bytes = L.desc - L.rel;
    h.map_bytes = mbytes;
    memset(f->save_hdr, 0, sizeof f->save_hdr);
    memcpy(f->save_hdr, &h, sizeof h);
    char* d = (char*)dst;
    const char* st = (const char*)f->S;   // the state struct opens the state buffer
    HIP_TRY(hipMemcpyAsync(d, f->save_hdr, kCkptHeader, hipMemcpyDefault, stream));
    HIP_TRY(hipEventRecord(f->save_done, stream));
    HIP_TRY(hipMemcpyAsync(d + kCkptHeader, st, L.partials, hipMemcpyDefault, stream));
    HIP_TRY(hipMemcpyAsync(d + kCkptHeader + L.partials, st + L.rel, L.desc - L.rel, hipMemcpyDefault, stream));
    HIP_TRY(hipMemcpyAsync(d + kCkptHeader + L.partials + (L.desc - L.rel), f->map, mbytes, hipMemcpyDefault,
                           stream));
    return PRISM_OK;
}

prism_status prism_filter_load(prism_filter* f, const void* src, size_t src_bytes, hipStream_t stream) {
    REQUIRE(f, "filter is NULL");
    StateLayout L;
    const size_t need = ckpt_bytes(&f->cfg, &L);
    REQUIRE(src && aligned(src, 16) && src_bytes >= need, "src must be 16-byte aligned and hold %zu bytes", need);
    if (prism_status cst = not_capturing(stream, "prism_filter_load")) return cst;
    CkptHeader h;
    HIP_TRY(hipMemcpyAsync(&h, src, sizeof h, hipMemcpyDefault, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    REQUIRE(memcmp(h.magic, kCkptMagic, 8) == 0 && h.version == kCkptVersion && h.header_bytes == kCkptHeader,
            "not a checkpoint of this library (magic or version)");
    REQUIRE(h.state_dim == (f->X ? 15 : 12), "checkpoint state is %d-D, the filter's %d-D", (int)h.state_dim,
            f->X ? 15 : 12);
    REQUIRE(same_grid(h.grid, f->cfg.grid), "checkpoint grid differs from the filter's grid");
    REQUIRE(same_cam(h.cam, f->cfg.cam), "checkpoint camera differs from the filter's camera");
    const size_t mbytes = map_layout(&f->cfg.grid).total;
    REQUIRE(h.state_bytes == L.partials && h.rel_bytes == L.desc - L.rel && h.map_bytes == mbytes,
            "checkpoint sizes do not match the filter");
    REQUIRE(h.steps >= 0, "checkpoint step counter is negative");
    const char* sp = (const char*)src;
    char* st = (char*)f->S;
    HIP_TRY(hipMemcpyAsync(st, sp + kCkptHeader, L.partials, hipMemcpyDefault, stream));
    HIP_TRY(hipMemcpyAsync(st + L.rel, sp + kCkptHeader + L.partials, L.desc - L.rel, hipMemcpyDefault, stream));
    HIP_TRY(hipMemcpyAsync(f->map, sp + kCkptHeader + L.partials + (L.desc - L.rel), mbytes, hipMemcpyDefault,
                           stream));
    f->steps = h.steps;
    return PRISM_OK;
}

prism_status prism_pose_retract(const prism_pose* poses, const double* delta, int32_t n, prism_pose* out,
                                hipStream_t stream) {
    REQUIRE(n >= 0 && n <= (1 << 24), "n must be in [0, 2^24]");
    if (n == 0) return PRISM_OK;
    REQUIRE(poses && delta && out && aligned(poses, 8) && aligned(delta, 8) && aligned(out, 8),
            "poses, delta and out must be non-NULL and 8-byte aligned");
    HIP_TRY(launch_pose_retract(poses, delta, n, out, stream));
    return PRISM_OK;
}

prism_status prism_filter_state_ptr(const prism_filter* f, prism_filter_state** state) {
    REQUIRE(f && state, "filter and state must be non-NULL");
    *state = f->S;
    return PRISM_OK;
}

prism_status prism_filter_bias_state_ptr(const prism_filter* f, prism_filter_bias_state** out) {
    REQUIRE(f && out, "filter and out must be non-NULL");
    if (!f->X) return fail(PRISM_UNSUPPORTED, "the filter has no bias state (PRISM_MODE_ACCEL_BIAS)");
    *out = f->X;
    return PRISM_OK;
}

prism_status prism_filter_anchor(const prism_filter* f, float** depth, float** rgb, uint8_t** mask, float** normals,
                                 uint8_t** nmask) {
    REQUIRE(f, "filter is NULL");
    if (depth) *depth = f->a_depth;
    if (rgb) *rgb = f->a_rgb;
    if (mask) *mask = f->a_mask;
    if (normals) *normals = f->a_normals;
    if (nmask) *nmask = f->a_nmask;
    return PRISM_OK;
}

}  // extern "C"
