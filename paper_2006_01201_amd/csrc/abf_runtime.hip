// Host runtime and C ABI of libabf (declared in include/abf.h).
//
// A plan owns host state only: parameters, the bound workspace, a small
// ring of pinned host buffers for the batch descriptor tables, the launch
// table chosen by the autotuner and a cache of instantiated hipGraphs.
// Every call lays the batch out in the workspace (pyramids and integer
// flows of every level of every strip), writes the descriptor tables
// (strip buffers, per-level geometry, per-stage tile prefix sums) to the
// head of the workspace and enqueues one launch per stage and level for
// the whole batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/abf.h"
#include "abf_internal.h"

using namespace abf;

namespace {

constexpr size_t kAlign = 256;
constexpr int kSlots = 4;

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// flows are read and written as one 64-bit (x, y) pair per pixel
inline bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

struct Launch {
    int tile_h;
    int grid;  // persistent workgroups per CU; 0 = one workgroup per tile
};

// Byte layout of one batch in the workspace.
struct Layout {
    int n = 0, N = 0;
    std::vector<int> H, W;                // per strip
    std::vector<std::vector<int>> hk, wk;  // [strip][level]
    size_t hdr_io = 0, hdr_lv = 0, hdr_prefix = 0, hdr_bytes = 0;
    size_t data_bytes = 0;
};

}  // namespace

struct abf_plan {
    abf_params p{};
    int max_strips = 0;
    int64_t max_pixels = 0;
    int max_H = 0, max_W = 0;
    int device = 0, n_cu = 0;
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
    size_t hdr_cap = 0;  // bytes reserved at the head of the workspace for descriptor tables
    std::string err;
    Launch launch[kStages][kSizeClasses];
    // pinned staging for descriptor uploads
    uint8_t *pinned[kSlots] = {};
    hipEvent_t ev[kSlots] = {};
    bool ev_used[kSlots] = {};
    int slot = 0;
    std::vector<uint8_t> last_upload;
    // last batch, for workspace views
    std::vector<StripLv> lv_host;  // [level * n + strip]
    int last_n = 0;
    // graphs
    std::map<std::string, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;
    // device address of the static scratch array on the plan's device
    uint8_t *scratch = nullptr;
};

namespace {

// Logging to stderr by the ABF_LOG environment variable (read once):
// 0 (default) silent; 1 failures, plan and workspace set-up, graph
// captures, tuning choices and merge steps; 2 also every batched call.
int log_level()
{
    static const int level = [] {
        const char *v = getenv("ABF_LOG");
        return v ? atoi(v) : 0;
    }();
    return level;
}

void logf(int level, const char *fmt, ...)
{
    if (log_level() < level) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    fprintf(stderr, "[abf] %s\n", buf);
}

abf_status fail(abf_plan *pl, abf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (pl) pl->err = buf;
    logf(1, "error %d: %s", (int)st, buf);
    return st;
}

abf_status hip_fail(abf_plan *pl, hipError_t e, const char *what)
{
    return fail(pl, ABF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(pl, expr)                                   \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(pl, e_, #expr); \
    } while (0)

int size_class(int64_t px)
{
    if (px < (1 << 16)) return 0;
    if (px < (1 << 20)) return 1;
    if (px < (1 << 23)) return 2;
    return 3;
}

void default_launch(abf_plan *pl)
{
    for (int s = 0; s < kStages; s++)
        for (int c = 0; c < kSizeClasses; c++) pl->launch[s][c] = {4, 0};
    for (int c = 0; c < kSizeClasses; c++) {
        pl->launch[ST_PROP][c].tile_h = 16;
        pl->launch[ST_REFINE][c].tile_h = 4;
    }
}

bool valid_th(int stage, int th)
{
    switch (stage) {
    case ST_SEARCH: return th == 1 || th == 2 || th == 4 || th == 8;
    case ST_PROP: return th == 8 || th == 10 || th == 12 || th == 16 || th == 32;
    case ST_REFINE: return th == 2 || th == 4;
    case ST_BLEND: return th == 1 || th == 2 || th == 4;  // pixels per thread
    default: return th == 4;
    }
}

abf_status check_params(const abf_params *p)
{
    if (p->levels < 1 || p->levels > kMaxLevels) return ABF_E_INVALID;
    if (p->patch < 1 || p->radius < 1 || p->radius_coarse < 1 || p->prop_steps < 0 || p->median < 0 ||
        p->lk_patch < 1 || p->lk_iters < 0)
        return ABF_E_INVALID;
    if (!(p->lk_eps > 0.f) || !std::isfinite(p->lk_eps) || !std::isfinite(p->k_sharp) ||
        !std::isfinite(p->k_flowmag))
        return ABF_E_INVALID;
    if (p->blend_mode != 0 && p->blend_mode != 1) return ABF_E_INVALID;
    if (p->gain_comp != 0 && p->gain_comp != 1) return ABF_E_INVALID;
    if (p->flow_method != 0 && p->flow_method != 1) return ABF_E_INVALID;
    if (p->patch > 2 || p->radius > 4 || p->radius_coarse > 4 || p->prop_steps > 4 || p->median > 1 ||
        p->prop_steps + p->median > 5 || p->lk_patch > 3 || p->lk_iters > 8)
        return ABF_E_UNSUPPORTED;
    return ABF_OK;
}

// Padded luma planes: kPad replicated pixels on every side, 64-byte
// aligned rows, plus 64 bytes of slack before and after (the aligned
// row loads may read a few bytes past the last padded row).
inline int ypitch_of(int w) { return (int)align_up((size_t)w + 2 * kPad, 64); }
inline size_t plane_bytes(int H, int W)
{
    return align_up(kPlaneLead + (size_t)ypitch_of(W) * (H + 2 * kPad) + kPlaneLead, kAlign);
}
inline int fpitch_of(int w) { return (int)align_up((size_t)w, 16); }

size_t header_bytes(int n, int N)
{
    size_t b = align_up(sizeof(StripIO) * n, kAlign);
    b += align_up(sizeof(StripLv) * n * N, kAlign);
    b += align_up(sizeof(int32_t) * (n + 1) * (size_t)(kLists * N), kAlign);
    return b;
}

// Upper bound of the data bytes of any batch within the plan's limits.
size_t data_bound(const abf_plan *pl)
{
    const int N = pl->p.levels;
    // per level and strip: a padded plane <= (w + 2 kPad + 64)(h + 2 kPad)
    // + 384 with w <= W/2^k + 1, h <= H/2^k + 1; a flow buffer <= (4 w + 64)
    // h + 256. Summed over strips with sum(H W) <= max_pixels.
    double b = 0;
    const double mp = (double)pl->max_pixels, S = pl->max_strips, Hm = pl->max_H, Wm = pl->max_W;
    const double pd = 2 * kPad + 1;
    for (int k = 0; k < N; k++) {
        const double f = std::ldexp(1.0, -k);
        b += 2 * (mp * f * f + S * ((Wm * f) * pd + (64 + pd) * (Hm * f + pd) + 384));
        // per direction: 2 flow buffers (int16 pairs: search, final; or, for
        // flow method 1, the float64 x and y planes) and 1 cost buffer
        const double e = pl->p.flow_method == 1 ? 8 : 4;
        b += 2 * 2 * (e * mp * f * f + S * (e * Wm * f + 16 * e * Hm * f + 17 * e + 256));
        b += 2 * 1 * (2 * mp * f * f + S * (2 * Wm * f + 32 * Hm * f + 34 + 256));
    }
    b += S * align_up(kSumWords * sizeof(unsigned long long), kAlign);  // exposure sums
    return align_up((size_t)b + 4096, kAlign);
}

void level_sizes(int H, int W, int N, std::vector<int> &hs, std::vector<int> &ws)
{
    hs.resize(N);
    ws.resize(N);
    for (int k = 0; k < N; k++) {
        hs[k] = H;
        ws[k] = W;
        H = (H + 1) / 2;
        W = (W + 1) / 2;
    }
}

// Tiles of one strip at one level for a work list (a stage, or the
// refinement's border pixels).
int stage_tiles(const abf_plan *pl, int stage, int cls, int H, int W)
{
    const int th = stage < kStages ? pl->launch[stage][cls].tile_h : 1;
    switch (stage) {
    case ST_LUMA: return tiles_luma(H, W);
    case ST_PYR: return 2 * tiles_pyr(H, W);
    case ST_SEARCH: return tiles_search(H, W, th);
    case ST_PROP: return tiles_prop(H, W, th, pl->p.prop_steps + pl->p.median);
    case ST_REFINE: return tiles_refine(H, W, th, pl->p.lk_patch);
    case LIST_REFINE_BORDER: return tiles_refine_border(H, W, pl->p.lk_patch);
    default: return tiles_blend(H, W, th);
    }
}

struct Batch {
    Layout lay;
    std::vector<StripIO> io;
    std::vector<StripLv> lv;              // [k * n + s]
    std::vector<int32_t> prefix;          // [(list * N + k) * (n + 1) + s]
    std::vector<int> cls;                 // [k] size class of level k over the batch
    std::vector<int64_t> level_px;        // [k]
};

abf_status build_batch(abf_plan *pl, const abf_strip *st, int n, bool flows, bool blend, Batch &b)
{
    const int N = pl->p.levels;
    Layout &L = b.lay;
    L.n = n;
    L.N = N;
    L.H.resize(n);
    L.W.resize(n);
    L.hk.resize(n);
    L.wk.resize(n);
    int64_t px = 0;
    for (int s = 0; s < n; s++) {
        const abf_strip &x = st[s];
        if (!x.L || !x.R || (blend && !x.F) || !x.flow_LtoR || !x.flow_RtoL)
            return fail(pl, ABF_E_INVALID, "strip %d: null pointer", s);
        if (!aligned8(x.flow_LtoR) || !aligned8(x.flow_RtoL))
            return fail(pl, ABF_E_INVALID, "strip %d: flows must be 8-byte aligned", s);
        if (x.H < 1 || x.W < 1) return fail(pl, ABF_E_SHAPE, "strip %d: size %d x %d", s, x.H, x.W);
        if (x.H > pl->max_H || x.W > pl->max_W)
            return fail(pl, ABF_E_SHAPE, "strip %d: %d x %d exceeds the plan's %d x %d", s, x.H, x.W, pl->max_H,
                        pl->max_W);
        if (x.pitch_L < 3 * x.W || x.pitch_R < 3 * x.W || (blend && x.pitch_F < 3 * x.W))
            return fail(pl, ABF_E_SHAPE, "strip %d: pitch smaller than 3 W", s);
        if (x.axis != 0 && x.axis != 1) return fail(pl, ABF_E_INVALID, "strip %d: axis %d", s, x.axis);
        L.H[s] = x.H;
        L.W[s] = x.W;
        level_sizes(x.H, x.W, N, L.hk[s], L.wk[s]);
        px += (int64_t)x.H * x.W;
    }
    if (n > pl->max_strips) return fail(pl, ABF_E_SHAPE, "%d strips exceed the plan's %d", n, pl->max_strips);
    if (px > pl->max_pixels)
        return fail(pl, ABF_E_SHAPE, "%lld pixels exceed the plan's %lld", (long long)px, (long long)pl->max_pixels);
    if (!pl->ws) return fail(pl, ABF_E_WORKSPACE, "no workspace bound");

    // header: io, lv, prefix
    L.hdr_io = 0;
    L.hdr_lv = align_up(sizeof(StripIO) * n, kAlign);
    L.hdr_prefix = L.hdr_lv + align_up(sizeof(StripLv) * n * N, kAlign);
    L.hdr_bytes = L.hdr_prefix + align_up(sizeof(int32_t) * (n + 1) * (size_t)(kLists * N), kAlign);
    if (L.hdr_bytes > pl->hdr_cap) return fail(pl, ABF_E_WORKSPACE, "descriptor tables exceed the reserved head");

    b.io.resize(n);
    b.lv.assign((size_t)n * N, StripLv{});
    b.level_px.assign(N, 0);
    for (int s = 0; s < n; s++)
        for (int k = 0; k < N; k++) b.level_px[k] += (int64_t)L.hk[s][k] * L.wk[s][k];
    b.cls.resize(N);
    for (int k = 0; k < N; k++) b.cls[k] = size_class(b.level_px[k]);

    size_t off = pl->hdr_cap;
    for (int s = 0; s < n; s++) {
        const abf_strip &x = st[s];
        StripIO &io = b.io[s];
        io.L = x.L;
        io.R = x.R;
        io.blend = x.blend;
        io.flow[0] = x.flow_LtoR;
        io.flow[1] = x.flow_RtoL;
        io.F = x.F;
        io.Ff32 = x.F_f32;
        io.pitchL = x.pitch_L;
        io.pitchR = x.pitch_R;
        io.pitchF = x.pitch_F;
        io.H = x.H;
        io.W = x.W;
        io.axis = x.axis;
        {
            const int ext = x.axis == 0 ? x.W : x.H;
            io.inv_ext1 = 1.0 / (ext + 1.0);
            io.inv_ext = 1.0 / ext;
        }
        if (!flows) continue;
        io.sums = reinterpret_cast<unsigned long long *>(pl->ws + off);
        off += align_up(kSumWords * sizeof(unsigned long long), kAlign);
        for (int k = 0; k < N; k++) {
            StripLv &v = b.lv[(size_t)k * n + s];
            v.H = L.hk[s][k];
            v.W = L.wk[s][k];
            v.ypitch = ypitch_of(v.W);
            v.fpitch = fpitch_of(v.W);
            for (int d = 0; d < 2; d++) {
                v.y[d] = pl->ws + off + kPlaneLead + (size_t)v.ypitch * kPad + kPad;
                off += plane_bytes(v.H, v.W);
            }
            // flow entries: int16 pairs, or float64 components (flow method 1)
            const size_t fb = align_up((size_t)v.fpitch * (pl->p.flow_method == 1 ? 8 : 4) * v.H, kAlign);
            const size_t cb = align_up((size_t)v.fpitch * 2 * v.H, kAlign);
            for (int d = 0; d < 2; d++) {
                v.ds[d] = reinterpret_cast<uint32_t *>(pl->ws + off);
                off += fb;
                v.df[d] = reinterpret_cast<uint32_t *>(pl->ws + off);
                off += fb;
                v.cs[d] = reinterpret_cast<uint16_t *>(pl->ws + off);
                off += cb;
            }
            v.radius = k == N - 1 ? pl->p.radius_coarse : pl->p.radius;
        }
        for (int k = 0; k < N; k++) {
            StripLv &v = b.lv[(size_t)k * n + s];
            if (k + 1 < N) {
                const StripLv &c = b.lv[(size_t)(k + 1) * n + s];
                v.dc[0] = c.df[0];
                v.dc[1] = c.df[1];
                v.Hc = c.H;
                v.Wc = c.W;
                v.fpitch_c = c.fpitch;
            }
            if (k > 0) {
                const StripLv &f = b.lv[(size_t)(k - 1) * n + s];
                v.yfine[0] = f.y[0];
                v.yfine[1] = f.y[1];
                v.Hf = f.H;
                v.Wf = f.W;
                v.ypitch_f = f.ypitch;
            }
        }
    }
    L.data_bytes = off - pl->hdr_cap;
    if (off > pl->ws_bytes)
        return fail(pl, ABF_E_WORKSPACE, "batch needs %zu workspace bytes, %zu bound", off, pl->ws_bytes);

    // tile prefix sums per stage and level
    b.prefix.assign((size_t)(n + 1) * kLists * N, 0);
    for (int stg = 0; stg < kLists; stg++)
        for (int k = 0; k < N; k++) {
            int32_t *pre = &b.prefix[((size_t)stg * N + k) * (n + 1)];
            int64_t acc = 0;
            for (int s = 0; s < n; s++) {
                pre[s] = (int32_t)acc;
                acc += stage_tiles(pl, stg, b.cls[k], L.hk[s][k], L.wk[s][k]);
            }
            pre[n] = (int32_t)acc;
            if (acc > 0x7fffffff) return fail(pl, ABF_E_SHAPE, "too many tiles");
        }
    return ABF_OK;
}

// Copies descriptor bytes to the head of the workspace (stream ordered),
// through a pinned slot whose previous copy has completed; skipped when
// the head already holds exactly these bytes.
abf_status upload_bytes(abf_plan *pl, std::vector<uint8_t> &host, hipStream_t s)
{
    if (host.size() > pl->hdr_cap) return fail(pl, ABF_E_WORKSPACE, "descriptor tables exceed the reserved head");
    if (host == pl->last_upload) return ABF_OK;
    const int k = pl->slot;
    pl->slot = (pl->slot + 1) % kSlots;
    if (pl->ev_used[k]) HIP_TRY(pl, hipEventSynchronize(pl->ev[k]));
    memcpy(pl->pinned[k], host.data(), host.size());
    HIP_TRY(pl, hipMemcpyAsync(pl->ws, pl->pinned[k], host.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(pl, hipEventRecord(pl->ev[k], s));
    pl->ev_used[k] = true;
    pl->last_upload.swap(host);
    return ABF_OK;
}

abf_status upload(abf_plan *pl, const Batch &b, hipStream_t s)
{
    const Layout &L = b.lay;
    std::vector<uint8_t> host(L.hdr_bytes, 0);
    memcpy(host.data() + L.hdr_io, b.io.data(), sizeof(StripIO) * L.n);
    memcpy(host.data() + L.hdr_lv, b.lv.data(), sizeof(StripLv) * b.lv.size());
    memcpy(host.data() + L.hdr_prefix, b.prefix.data(), sizeof(int32_t) * b.prefix.size());
    return upload_bytes(pl, host, s);
}

int grid_of(const abf_plan *pl, int stage, int cls)
{
    const int g = pl->launch[stage][cls].grid;
    return g > 0 ? g * pl->n_cu : 0;
}

// Optional per-launch timing: when `prof` is set, an event pair brackets
// every launch and the elapsed times are added to prof->ms[stage][level].
struct Prof {
    std::vector<hipEvent_t> ev;
    std::vector<std::pair<int, int>> tag;  // (stage, level) per event pair
};

// Enqueues the launch sequence of a batch whose tables are in place.
abf_status enqueue(abf_plan *pl, const Batch &b, bool flows, bool blend, hipStream_t s, Prof *prof = nullptr)
{
    const Layout &L = b.lay;
    const int n = L.n, N = L.N;
    const StripIO *io = reinterpret_cast<const StripIO *>(pl->ws + L.hdr_io);
    const StripLv *lv = reinterpret_cast<const StripLv *>(pl->ws + L.hdr_lv);
    const int32_t *pre = reinterpret_cast<const int32_t *>(pl->ws + L.hdr_prefix);
    auto work = [&](int stg, int k) {
        Work w;
        const size_t o = ((size_t)stg * N + k) * (n + 1);
        w.prefix = pre + o;
        w.n = n;
        w.total = b.prefix[o + n];
        return w;
    };
    const abf_params &p = pl->p;
    auto mark = [&](int stg, int k) -> hipError_t {
        if (!prof) return hipSuccess;
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        prof->ev.push_back(e);
        if (prof->ev.size() % 2 == 1) prof->tag.emplace_back(stg, k);
        return hipEventRecord(e, s);
    };
#define TIMED(stg, k, call)              \
    do {                                 \
        HIP_TRY(pl, mark(stg, k));       \
        HIP_TRY(pl, call);               \
        HIP_TRY(pl, mark(stg, k));       \
    } while (0)
    if (flows) {
        if (p.gain_comp) HIP_TRY(pl, launch_zero_sums(io, n, s));  // the exposure step's sums
        TIMED(ST_LUMA, 0, launch_luma(io, lv, work(ST_LUMA, 0), grid_of(pl, ST_LUMA, b.cls[0]), p.gain_comp != 0, s));
        if (p.gain_comp)
            TIMED(ST_LUMA, 1, launch_gain(io, lv, work(ST_LUMA, 0), grid_of(pl, ST_LUMA, b.cls[0]), s));
        for (int k = 1; k < N; k++)
            TIMED(ST_PYR, k, launch_pyr(lv + (size_t)k * n, work(ST_PYR, k), grid_of(pl, ST_PYR, b.cls[k]), s));
        if (p.flow_method == 1) {
            // classic coarse-to-fine Lucas-Kanade: one launch per level,
            // timed in the search stage's slots
            // (interior pixels in the refinement's slots, whose launch
            // shapes they use and the tuner sets; border pixels in the
            // search slots)
            LkParams lk{p.lk_patch, p.lk_iters, p.lk_eps};
            for (int k = N - 1; k >= 0; k--) {
                const int c = b.cls[k];
                const StripLv *lvk = lv + (size_t)k * n, *lvc = k == N - 1 ? nullptr : lv + (size_t)(k + 1) * n;
                TIMED(ST_REFINE, k,
                      launch_lk_interior(lvk, lvc, io, work(ST_REFINE, k), lk, pl->launch[ST_REFINE][c].tile_h,
                                         grid_of(pl, ST_REFINE, c), k == 0, s));
                TIMED(ST_SEARCH, k, launch_lk_border(lvk, lvc, io, work(LIST_REFINE_BORDER, k), lk, k == 0, s));
            }
        }
        for (int k = N - 1; k >= 0 && p.flow_method == 0; k--) {
            const int c = b.cls[k];
            const int r = k == N - 1 ? p.radius_coarse : p.radius;
            TIMED(ST_SEARCH, k,
                  launch_search(lv + (size_t)k * n, work(ST_SEARCH, k), p.patch, r, pl->launch[ST_SEARCH][c].tile_h,
                                grid_of(pl, ST_SEARCH, c), s));
            TIMED(ST_PROP, k,
                  launch_prop(lv + (size_t)k * n, work(ST_PROP, k), p.patch, p.prop_steps, p.median,
                              pl->launch[ST_PROP][c].tile_h, grid_of(pl, ST_PROP, c), s));
        }
        if (p.flow_method == 0) {
            LkParams lk{p.lk_patch, p.lk_iters, p.lk_eps};
            // interior tiles, then the border pixels (a forked stream that ran the
            // border concurrently made the graph replay slower); the border launch
            // is timed in the level-1 slot of the stage (refinement runs at level 0)
            TIMED(ST_REFINE, 0,
                  launch_refine(lv, io, work(ST_REFINE, 0), lk, pl->launch[ST_REFINE][b.cls[0]].tile_h,
                                grid_of(pl, ST_REFINE, b.cls[0]), s));
            TIMED(ST_REFINE, 1, launch_refine_border(lv, io, work(LIST_REFINE_BORDER, 0), lk, s));
        }
    }
    if (blend) {
        BlendParams bp{p.k_sharp, p.k_flowmag, p.blend_mode};
        TIMED(ST_BLEND, 0,
              launch_blend(io, work(ST_BLEND, 0), bp, pl->launch[ST_BLEND][b.cls[0]].tile_h,
                           grid_of(pl, ST_BLEND, b.cls[0]), s));
    }
#undef TIMED
    return ABF_OK;
}

std::string graph_key(const abf_plan *pl, const Batch &b, bool flows, bool blend)
{
    std::string k;
    char buf[96];
    snprintf(buf, sizeof(buf), "%d:%d:%d|", b.lay.n, (int)flows, (int)blend);
    k += buf;
    for (int s = 0; s < b.lay.n; s++) {
        snprintf(buf, sizeof(buf), "%d,%d,%d,%d,%d;", b.lay.H[s], b.lay.W[s], b.io[s].axis, b.io[s].blend != nullptr,
                 b.io[s].Ff32 != nullptr);
        k += buf;
    }
    for (int s = 0; s < kStages; s++)
        for (int c = 0; c < kSizeClasses; c++) {
            snprintf(buf, sizeof(buf), "%d/%d,", pl->launch[s][c].tile_h, pl->launch[s][c].grid);
            k += buf;
        }
    return k;
}

void clear_graphs(abf_plan *pl)
{
    for (auto &kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
    pl->graphs.clear();
}

abf_status run(abf_plan *pl, const abf_strip *st, int n, bool flows, bool blend, bool use_graph, hipStream_t s)
{
    Batch b;
    abf_status rc = build_batch(pl, st, n, flows, blend, b);
    if (rc != ABF_OK) return rc;
    rc = upload(pl, b, s);
    if (rc != ABF_OK) return rc;
    if (flows) {
        pl->lv_host = b.lv;
        pl->last_n = n;
    }
    logf(2, "run: %d strip(s), flows %d, blend %d, graph %d", n, (int)flows, (int)blend, (int)use_graph);
    if (!use_graph) return enqueue(pl, b, flows, blend, s);

    const std::string key = graph_key(pl, b, flows, blend);
    auto it = pl->graphs.find(key);
    if (it == pl->graphs.end()) {
        logf(1, "capturing a graph for %d strip(s) (%zu cached)", n, pl->graphs.size());
        if (!pl->cap_stream) HIP_TRY(pl, hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
        // the tables were uploaded on `s`; the capture stream only records
        HIP_TRY(pl, hipStreamSynchronize(s));
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(pl, ABF_E_CAPTURE, "hipStreamBeginCapture failed");
        abf_status er = enqueue(pl, b, flows, blend, pl->cap_stream);
        hipError_t ee = hipStreamEndCapture(pl->cap_stream, &g);
        if (er != ABF_OK) {
            if (g) (void)hipGraphDestroy(g);
            return er;
        }
        if (ee != hipSuccess || !g) return fail(pl, ABF_E_CAPTURE, "hipStreamEndCapture: %s", hipGetErrorString(ee));
        hipGraphExec_t ex = nullptr;
        hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return fail(pl, ABF_E_CAPTURE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        it = pl->graphs.emplace(key, ex).first;
    }
    HIP_TRY(pl, hipGraphLaunch(it->second, s));
    return ABF_OK;
}

}  // namespace

// ---------------------------------------------------------------------
// Static scratch of the allocation-free flow entry point: a file-scope
// device array (one copy per device, held until the process ends). In
// host code its name is only a stand-in for the symbol; the device address
// of each device's copy is looked up once per device with
// hipGetSymbolAddress (at plan creation, with that device current) and
// only that address is used.
static __device__ __align__(256) uint8_t scratch[ABF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch[kMaxDevices] = {};

// Address of the current device's scratch (device `dev`), looked up once.
abf_status scratch_address(int dev, uint8_t **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return ABF_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return ABF_E_DEVICE;
        g_scratch[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch[dev];
    return ABF_OK;
}

}  // namespace

// =====================================================================
// C ABI

extern "C" {

void abf_default_params(abf_params *p)
{
    if (!p) return;
    p->levels = 6;
    p->patch = 2;
    p->radius = 2;
    p->radius_coarse = 4;
    p->prop_steps = 2;
    p->median = 1;
    p->lk_patch = 2;
    p->lk_iters = 2;
    p->lk_eps = 25.0f;
    p->k_sharp = 10.0f;
    p->k_flowmag = 20.0f;
    p->blend_mode = 0;
    p->gain_comp = 0;
    p->flow_method = 0;
}

const char *abf_status_string(abf_status s)
{
    switch (s) {
    case ABF_OK: return "ABF_OK";
    case ABF_E_INVALID: return "ABF_E_INVALID: invalid argument";
    case ABF_E_SHAPE: return "ABF_E_SHAPE: inconsistent or out-of-range sizes";
    case ABF_E_WORKSPACE: return "ABF_E_WORKSPACE: workspace missing or too small";
    case ABF_E_DEVICE: return "ABF_E_DEVICE: HIP runtime error";
    case ABF_E_UNSUPPORTED: return "ABF_E_UNSUPPORTED: no gfx950 device or unsupported parameter";
    case ABF_E_CAPTURE: return "ABF_E_CAPTURE: hipGraph capture failed";
    }
    return "unknown abf_status";
}

const char *abf_last_error(const abf_plan *plan) { return plan ? plan->err.c_str() : "null plan"; }

abf_status abf_create_plan(const abf_params *params, int32_t max_strips, int64_t max_pixels, int32_t max_H,
                           int32_t max_W, abf_plan **out)
{
    if (!params || !out) return ABF_E_INVALID;
    *out = nullptr;
    abf_status rc = check_params(params);
    if (rc != ABF_OK) return rc;
    if (max_strips < 1 || max_pixels < 1 || max_H < 1 || max_W < 1) return ABF_E_INVALID;
    if ((int64_t)max_H * max_W > max_pixels) max_pixels = (int64_t)max_H * max_W;
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(nullptr, ABF_E_UNSUPPORTED, "no device");
    if (hipGetDevice(&dev) != hipSuccess) return ABF_E_UNSUPPORTED;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return ABF_E_UNSUPPORTED;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, ABF_E_UNSUPPORTED, "device %d is %s, not gfx950", dev, prop.gcnArchName);

    uint8_t *scr = nullptr;
    if (scratch_address(dev, &scr) != ABF_OK)
        return fail(nullptr, ABF_E_DEVICE, "hipGetSymbolAddress of the static scratch failed on device %d", dev);

    abf_plan *pl = new abf_plan();
    pl->scratch = scr;
    pl->p = *params;
    pl->max_strips = max_strips;
    pl->max_pixels = max_pixels;
    pl->max_H = max_H;
    pl->max_W = max_W;
    pl->device = dev;
    pl->n_cu = prop.multiProcessorCount;
    pl->hdr_cap = header_bytes(max_strips, params->levels);
    default_launch(pl);
    for (int k = 0; k < kSlots; k++) {
        if (hipHostMalloc((void **)&pl->pinned[k], pl->hdr_cap, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&pl->ev[k], hipEventDisableTiming) != hipSuccess) {
            abf_destroy(pl);
            return ABF_E_DEVICE;
        }
    }

    const char *cache = getenv("ABF_TUNE_CACHE");
    if (cache) {
        FILE *f = fopen(cache, "r");
        if (f) {
            char arch[64] = {0};
            if (fscanf(f, " { \"arch\" : \"%63[^\"]\" , \"launch\" : [", arch) == 1 &&
                strncmp(arch, prop.gcnArchName, 6) == 0) {
                Launch tmp[kStages][kSizeClasses];
                bool ok = true;
                for (int s = 0; s < kStages && ok; s++)
                    for (int c = 0; c < kSizeClasses && ok; c++)
                        ok = fscanf(f, " [ %d , %d ]%*[, ]", &tmp[s][c].tile_h, &tmp[s][c].grid) == 2 &&
                             valid_th(s, tmp[s][c].tile_h) && tmp[s][c].grid >= 0 && tmp[s][c].grid <= 64;
                if (ok) memcpy(pl->launch, tmp, sizeof(tmp));
            }
            fclose(f);
        }
    }
    logf(1, "plan on device %d (%s): %d strips, %lld px, %d x %d, %d levels, flow method %d; workspace %zu bytes",
         dev, prop.gcnArchName, max_strips, (long long)max_pixels, max_H, max_W, params->levels,
         params->flow_method, abf_workspace_bytes(pl));
    *out = pl;
    return ABF_OK;
}

size_t abf_workspace_bytes(const abf_plan *plan)
{
    if (!plan) return 0;
    return plan->hdr_cap + data_bound(plan);
}

abf_status abf_bind_workspace(abf_plan *plan, void *dev_ptr, size_t bytes)
{
    if (!plan || !dev_ptr) return fail(plan, ABF_E_INVALID, "null workspace");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign != 0)
        return fail(plan, ABF_E_INVALID, "workspace not %zu-byte aligned", kAlign);
    if (bytes < abf_workspace_bytes(plan))
        return fail(plan, ABF_E_WORKSPACE, "workspace of %zu bytes, %zu needed", bytes, abf_workspace_bytes(plan));
    plan->ws = static_cast<uint8_t *>(dev_ptr);
    plan->ws_bytes = bytes;
    plan->last_upload.clear();
    clear_graphs(plan);
    return ABF_OK;
}

abf_status abf_flow_bidirectional(abf_plan *plan, const uint8_t *L, const uint8_t *R, int32_t H, int32_t W,
                                  int32_t pitch_L, int32_t pitch_R, float *flow_LtoR, float *flow_RtoL,
                                  void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    abf_strip st{};
    st.L = L;
    st.R = R;
    st.H = H;
    st.W = W;
    st.pitch_L = pitch_L;
    st.pitch_R = pitch_R;
    st.flow_LtoR = flow_LtoR;
    st.flow_RtoL = flow_RtoL;
    return run(plan, &st, 1, true, false, false, static_cast<hipStream_t>(hip_stream));
}

abf_status abf_flow_bidirectional_noalloc(abf_plan *plan, const uint8_t *L, const uint8_t *R, int32_t H, int32_t W,
                                          int32_t pitch_L, int32_t pitch_R, float *flow_LtoR, float *flow_RtoL,
                                          void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!plan->scratch) return fail(plan, ABF_E_UNSUPPORTED, "no static scratch on the plan's device");
    abf_strip st{};
    st.L = L;
    st.R = R;
    st.H = H;
    st.W = W;
    st.pitch_L = pitch_L;
    st.pitch_R = pitch_R;
    st.flow_LtoR = flow_LtoR;
    st.flow_RtoL = flow_RtoL;
    // the flow path lays the strip out from the head of the static scratch
    // instead of the bound workspace; the descriptor tables are always
    // uploaded (another call may have overwritten the array since)
    uint8_t *const ws = plan->ws;
    const size_t ws_bytes = plan->ws_bytes;
    plan->ws = plan->scratch;
    plan->ws_bytes = ABF_NOALLOC_SCRATCH_BYTES;
    plan->last_upload.clear();
    abf_status rc = run(plan, &st, 1, true, false, false, static_cast<hipStream_t>(hip_stream));
    plan->ws = ws;
    plan->ws_bytes = ws_bytes;
    plan->last_upload.clear();
    if (rc == ABF_E_WORKSPACE)
        rc = fail(plan, ABF_E_WORKSPACE, "a %d x %d strip needs more than the %zu bytes of static scratch", H, W,
                  (size_t)ABF_NOALLOC_SCRATCH_BYTES);
    return rc;
}

abf_status abf_blend_asymmetric(abf_plan *plan, const uint8_t *L, const uint8_t *R, const float *flow_LtoR,
                                const float *flow_RtoL, const float *blend, int32_t axis, int32_t H, int32_t W,
                                int32_t pitch_L, int32_t pitch_R, uint8_t *F, int32_t pitch_F, float *F_f32,
                                void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!flow_LtoR || !flow_RtoL) return fail(plan, ABF_E_INVALID, "null flow");
    abf_strip st{};
    st.L = L;
    st.R = R;
    st.H = H;
    st.W = W;
    st.pitch_L = pitch_L;
    st.pitch_R = pitch_R;
    st.axis = axis;
    st.blend = blend;
    st.flow_LtoR = const_cast<float *>(flow_LtoR);
    st.flow_RtoL = const_cast<float *>(flow_RtoL);
    st.F = F;
    st.pitch_F = pitch_F;
    st.F_f32 = F_f32;
    return run(plan, &st, 1, false, true, false, static_cast<hipStream_t>(hip_stream));
}

abf_status abf_stitch_strips(abf_plan *plan, const abf_strip *strips, int32_t n, int32_t use_graph,
                             void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!strips || n < 1) return fail(plan, ABF_E_INVALID, "no strips");
    return run(plan, strips, n, true, true, use_graph != 0, static_cast<hipStream_t>(hip_stream));
}

abf_status abf_destroy(abf_plan *plan)
{
    if (!plan) return ABF_E_INVALID;
    clear_graphs(plan);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);

    for (int k = 0; k < kSlots; k++) {
        if (plan->ev[k]) {
            if (plan->ev_used[k]) (void)hipEventSynchronize(plan->ev[k]);
            (void)hipEventDestroy(plan->ev[k]);
        }
        if (plan->pinned[k]) (void)hipHostFree(plan->pinned[k]);
    }
    delete plan;
    return ABF_OK;
}

abf_status abf_workspace_view(const abf_plan *plan, int32_t kind, int32_t strip, int32_t level, int32_t dir,
                              void **dev_ptr, int32_t *H, int32_t *W, int32_t *pitch)
{
    if (!plan || !dev_ptr || !H || !W || !pitch) return ABF_E_INVALID;
    if (strip < 0 || strip >= plan->last_n || level < 0 || level >= plan->p.levels || dir < 0 || dir > 1)
        return ABF_E_SHAPE;
    const StripLv &v = plan->lv_host[(size_t)level * plan->last_n + strip];
    *H = v.H;
    *W = v.W;
    switch (kind) {
    case 0:
        *dev_ptr = v.y[dir];
        *pitch = v.ypitch;
        return ABF_OK;
    case 1:
        *dev_ptr = v.ds[dir];
        *pitch = v.fpitch;
        return ABF_OK;
    case 2:
        *dev_ptr = v.df[dir];
        *pitch = v.fpitch;
        return ABF_OK;
    }
    return ABF_E_INVALID;
}

abf_status abf_get_launch(const abf_plan *plan, int32_t stage, int32_t size_class, int32_t *tile_h, int32_t *grid)
{
    if (!plan || !tile_h || !grid || stage < 0 || stage >= kStages || size_class < 0 || size_class >= kSizeClasses)
        return ABF_E_INVALID;
    *tile_h = plan->launch[stage][size_class].tile_h;
    *grid = plan->launch[stage][size_class].grid;
    return ABF_OK;
}

abf_status abf_set_launch(abf_plan *plan, int32_t stage, int32_t size_class, int32_t tile_h, int32_t grid)
{
    if (!plan || stage < 0 || stage >= kStages || size_class < 0 || size_class >= kSizeClasses)
        return ABF_E_INVALID;
    if (!valid_th(stage, tile_h) || grid < 0 || grid > 64)
        return fail(plan, ABF_E_INVALID, "tile height %d / grid %d not available for stage %d", tile_h, grid, stage);
    plan->launch[stage][size_class] = {tile_h, grid};
    return ABF_OK;
}

// Size class of the launch that an event pair of enqueue() times, or -1
// when that launch takes no shape from the launch table (the refinement's
// border launch, the classic Lucas-Kanade border launches in the search
// slots).
int slot_class(const abf_plan *pl, const Batch &b, int stage, int k)
{
    switch (stage) {
    case ST_LUMA:
    case ST_BLEND: return b.cls[0];
    case ST_REFINE: return pl->p.flow_method == 1 ? b.cls[k] : (k == 0 ? b.cls[0] : -1);
    case ST_SEARCH: return pl->p.flow_method == 1 ? -1 : b.cls[k];
    default: return b.cls[k];
    }
}

abf_status abf_tune(abf_plan *plan, const abf_strip *strips, int32_t n, void *hip_stream)
{
    if (!plan || !strips || n < 1) return ABF_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // One eager pass with an event pair around every launch; `ms` receives
    // the summed time of the launches of (stage, size class) `want`, or,
    // with want.first < 0, `seen` the (stage, class) pairs that occur.
    bool seen[kStages][kSizeClasses] = {};
    auto pass = [&](std::pair<int, int> want, float &ms) -> abf_status {
        Batch b;  // the tile lists depend on the launch table
        abf_status rc = build_batch(plan, strips, n, true, true, b);
        if (rc != ABF_OK) return rc;
        rc = upload(plan, b, s);
        if (rc != ABF_OK) return rc;
        Prof prof;
        rc = enqueue(plan, b, true, true, s, &prof);
        const hipError_t e = hipStreamSynchronize(s);
        ms = 0.f;
        for (size_t i = 0; i + 1 < prof.ev.size() && rc == ABF_OK && e == hipSuccess; i += 2) {
            const int stg = prof.tag[i / 2].first, c = slot_class(plan, b, stg, prof.tag[i / 2].second);
            if (c < 0) continue;
            if (want.first < 0) {
                seen[stg][c] = true;
                continue;
            }
            float t = 0.f;
            if (stg == want.first && c == want.second &&
                hipEventElapsedTime(&t, prof.ev[i], prof.ev[i + 1]) == hipSuccess)
                ms += t;
        }
        for (hipEvent_t ev : prof.ev) (void)hipEventDestroy(ev);
        if (rc != ABF_OK) return rc;
        if (e != hipSuccess) return hip_fail(plan, e, "hipStreamSynchronize");
        plan->lv_host = b.lv;
        plan->last_n = n;
        return ABF_OK;
    };
    float unused = 0.f;
    abf_status rc = pass({-1, -1}, unused);
    static const int grids[] = {0, 1, 2, 4, 5, 6, 8};  // 0: a workgroup per tile, else per CU
    for (int stage = 0; stage < kStages && rc == ABF_OK; stage++)
        for (int c = 0; c < kSizeClasses && rc == ABF_OK; c++) {
            if (!seen[stage][c]) continue;
            Launch best = plan->launch[stage][c];
            float best_ms = 1e30f;
            for (int th : {1, 2, 4, 8, 10, 12, 16, 32}) {
                if (!valid_th(stage, th)) continue;
                for (int g : grids) {
                    plan->launch[stage][c] = {th, g};
                    float ms = 1e30f;
                    for (int r = 0; r < 4 && rc == ABF_OK; r++) {  // the first pass warms up
                        float t = 0.f;
                        rc = pass({stage, c}, t);
                        if (r > 0) ms = std::min(ms, t);
                    }
                    if (rc != ABF_OK) break;
                    if (ms < best_ms * 0.99f) {
                        best_ms = ms;
                        best = plan->launch[stage][c];
                    }
                }
                if (rc != ABF_OK) break;
            }
            plan->launch[stage][c] = best;
            logf(1, "tune: stage %d, size class %d: tile height %d, grid %d (%.4f ms)", stage, c, best.tile_h,
                 best.grid, best_ms);
        }
    if (rc != ABF_OK) return rc;
    const char *cache = getenv("ABF_TUNE_CACHE");
    if (cache) {
        FILE *f = fopen(cache, "w");
        if (f) {
            hipDeviceProp_t prop;
            (void)hipGetDeviceProperties(&prop, plan->device);
            fprintf(f, "{\"arch\": \"%s\", \"launch\": [", prop.gcnArchName);
            for (int st = 0; st < kStages; st++)
                for (int c = 0; c < kSizeClasses; c++)
                    fprintf(f, "%s[%d, %d]", st + c ? ", " : "", plan->launch[st][c].tile_h,
                            plan->launch[st][c].grid);
            fprintf(f, "]}\n");
            fclose(f);
        }
    }
    return ABF_OK;
}

// ------------------------------------------------------------------
// differentiable path: scratch (energy partials, fixed-point scatter
// buffers, the other half of the descent ping-pong) comes from the
// workspace's data region.

static abf_status grad_scratch(abf_plan *plan, size_t need, uint8_t **out)
{
    if (!plan->ws) return fail(plan, ABF_E_WORKSPACE, "no workspace bound");
    if (plan->hdr_cap + need > plan->ws_bytes)
        return fail(plan, ABF_E_WORKSPACE, "needs %zu scratch bytes, workspace holds %zu", need,
                    plan->ws_bytes - plan->hdr_cap);
    *out = plan->ws + plan->hdr_cap;
    return ABF_OK;
}

// ------------------------------------------------------------ canvas
// Scratch of the canvas passes: the row-distance plane G, its block minima
// M and (when the caller gives no Blend array) a Blend map, in the
// workspace's data region.
static size_t canvas_scratch(int H, int W)
{
    const size_t gp = (size_t)canvas_gpitch(W);
    return 2 * align_up(sizeof(uint32_t) * gp * H, kAlign) +
           align_up(sizeof(uint32_t) * gp * (size_t)ceil_div(H, kCanvasBH), kAlign);
}

static abf_status canvas_setup(abf_plan *plan, const uint8_t *mL, const uint8_t *mR, int32_t H, int32_t W,
                               int32_t pitchM, bool periodic, CanvasGeom &g, float **bmap)
{
    if (!mL || !mR) return fail(plan, ABF_E_INVALID, "null mask");
    if (H < 1 || W < 1 || H > kCanvasMaxDim || W > kCanvasMaxDim)
        return fail(plan, ABF_E_SHAPE, "canvas %d x %d (1..%d per side)", H, W, kCanvasMaxDim);
    if (pitchM < W) return fail(plan, ABF_E_SHAPE, "mask pitch %d < W %d", pitchM, W);
    uint8_t *scr = nullptr;
    abf_status rc = grad_scratch(plan, canvas_scratch(H, W), &scr);
    if (rc != ABF_OK) return rc;
    const size_t gp = (size_t)canvas_gpitch(W);
    const size_t plane = align_up(sizeof(uint32_t) * gp * H, kAlign);
    g.mL = mL;
    g.mR = mR;
    g.G = reinterpret_cast<uint32_t *>(scr);
    g.M = reinterpret_cast<uint32_t *>(scr + plane);
    *bmap = reinterpret_cast<float *>(scr + plane + align_up(sizeof(uint32_t) * gp * (size_t)ceil_div(H, kCanvasBH), kAlign));
    g.pitchM = pitchM;
    g.H = H;
    g.W = W;
    g.gpitch = (int32_t)gp;
    g.periodic = periodic ? 1 : 0;
    g.gx0 = 0;
    g.gx1 = W;
    return ABF_OK;
}

size_t abf_canvas_workspace_bytes(const abf_plan *plan, int32_t H, int32_t W)
{
    if (!plan || H < 1 || W < 1 || H > kCanvasMaxDim || W > kCanvasMaxDim) return 0;
    const size_t need = plan->hdr_cap + canvas_scratch(H, W);
    const size_t base = abf_workspace_bytes(plan);
    return need > base ? need : base;
}

abf_status abf_overlap_box(abf_plan *plan, const uint8_t *mask_L, const uint8_t *mask_R, int32_t H, int32_t W,
                           int32_t pitch_mask, int32_t periodic, int32_t *box, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!mask_L || !mask_R || !box) return fail(plan, ABF_E_INVALID, "null pointer");
    if (H < 1 || W < 1 || H > kCanvasMaxDim || W > kCanvasMaxDim)
        return fail(plan, ABF_E_SHAPE, "canvas %d x %d (1..%d per side)", H, W, kCanvasMaxDim);
    if (pitch_mask < W) return fail(plan, ABF_E_SHAPE, "mask pitch %d < W %d", pitch_mask, W);
    uint8_t *scr = nullptr;
    abf_status rc = grad_scratch(plan, overlap_box_scratch(H, W), &scr);
    if (rc != ABF_OK) return rc;
    HIP_TRY(plan, launch_overlap_box(mask_L, mask_R, pitch_mask, H, W, periodic != 0, reinterpret_cast<int32_t *>(scr),
                                     box, static_cast<hipStream_t>(hip_stream)));
    return ABF_OK;
}

abf_status abf_canvas_blend(abf_plan *plan, const uint8_t *mask_L, const uint8_t *mask_R, int32_t H, int32_t W,
                            int32_t pitch_mask, int32_t periodic, float *blend, int32_t pitch_blend, int32_t *dist2_1,
                            int32_t *dist2_2, int32_t pitch_dist, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if ((dist2_1 == nullptr) != (dist2_2 == nullptr))
        return fail(plan, ABF_E_INVALID, "dist2_1 and dist2_2 go together");
    if (!blend && !dist2_1) return fail(plan, ABF_E_INVALID, "no output");
    if (blend && pitch_blend < W) return fail(plan, ABF_E_SHAPE, "blend pitch %d < W %d", pitch_blend, W);
    if (dist2_1 && pitch_dist < W) return fail(plan, ABF_E_SHAPE, "distance pitch %d < W %d", pitch_dist, W);
    CanvasGeom g{};
    float *bmap = nullptr;
    abf_status rc = canvas_setup(plan, mask_L, mask_R, H, W, pitch_mask, periodic != 0, g, &bmap);
    if (rc != ABF_OK) return rc;
    HIP_TRY(plan, launch_canvas_dist(g, blend, pitch_blend, dist2_1, dist2_2, pitch_dist, nullptr,
                                     static_cast<hipStream_t>(hip_stream)));
    return ABF_OK;
}

abf_status abf_composite_canvas(abf_plan *plan, const uint8_t *L, const uint8_t *R, const uint8_t *mask_L,
                                const uint8_t *mask_R, int32_t H, int32_t W, int32_t pitch_L, int32_t pitch_R,
                                int32_t pitch_mask, int32_t periodic, const float *flow_LtoR, const float *flow_RtoL,
                                const int32_t *box, int32_t axis, const float *blend, int32_t pitch_blend,
                                uint8_t *F, int32_t pitch_F, float *F_f32, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!L || !R || !F || !box) return fail(plan, ABF_E_INVALID, "null pointer");
    if (axis != 0 && axis != 1) return fail(plan, ABF_E_INVALID, "axis %d", axis);
    if (pitch_L < 3 * W || pitch_R < 3 * W || pitch_F < 3 * W)
        return fail(plan, ABF_E_SHAPE, "image pitch smaller than 3 W");
    const int bx = box[0], by = box[1], bw = box[2], bh = box[3];
    // on a periodic canvas the box's columns may wrap past W - 1
    if (bx < 0 || by < 0 || bw < 0 || bh < 0 || (periodic ? (bx >= W || bw > W) : bx + bw > W) || by + bh > H)
        return fail(plan, ABF_E_SHAPE, "box {%d, %d, %d, %d} outside the %d x %d canvas", bx, by, bw, bh, H, W);
    const bool any = bw > 0 && bh > 0;
    if (any && (!flow_LtoR || !flow_RtoL)) return fail(plan, ABF_E_INVALID, "null flow");
    if (any && (!aligned8(flow_LtoR) || !aligned8(flow_RtoL)))
        return fail(plan, ABF_E_INVALID, "flows must be 8-byte aligned");
    if (blend && pitch_blend < W) return fail(plan, ABF_E_SHAPE, "blend pitch %d < W %d", pitch_blend, W);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    CanvasGeom g{};
    float *bmap = nullptr;
    abf_status rc = canvas_setup(plan, mask_L, mask_R, H, W, pitch_mask, periodic != 0, g, &bmap);
    if (rc != ABF_OK) return rc;
    CompositeArgs o{};
    o.blend = blend;
    o.pitchB = pitch_blend;
    if (!blend && any) {
        HIP_TRY(plan, launch_canvas_dist(g, bmap, g.gpitch, nullptr, nullptr, 0, box, s));
        o.blend = bmap;
        o.pitchB = g.gpitch;
    }
    o.L = L;
    o.R = R;
    o.mL = mask_L;
    o.mR = mask_R;
    o.flr = flow_LtoR;
    o.frl = flow_RtoL;
    o.F = F;
    o.Ff32 = F_f32;
    o.pitchL = pitch_L;
    o.pitchR = pitch_R;
    o.pitchM = pitch_mask;
    o.pitchF = pitch_F;
    o.H = H;
    o.W = W;
    o.bx = any ? bx : 0;
    o.by = any ? by : 0;
    o.bw = any ? bw : 0;
    o.bh = any ? bh : 0;
    o.axis = axis;
    o.periodic = periodic ? 1 : 0;
    o.inv_ext = any ? 1.0 / (double)(axis == 0 ? bw : bh) : 0.0;
    BlendParams bp{plan->p.k_sharp, plan->p.k_flowmag, plan->p.blend_mode};
    HIP_TRY(plan, launch_composite(o, bp, s));
    return ABF_OK;
}

// ------------------------------------------------------ photo merging
// Workspace of a merge: [head][flow path's data region, or the canvas
// passes' scratch, whichever is larger][FlowLtoR][FlowRtoL][box + box
// scratch][L crop][R crop]. The flows of a step must survive the canvas
// passes that follow them; the crops (contiguous copies of a box that
// wraps past the last column of a periodic canvas) feed the flow path.
static size_t merge_tail(const abf_plan *plan, int H, int W)
{
    const size_t a = data_bound(plan), b = canvas_scratch(H, W);
    return plan->hdr_cap + align_up(a > b ? a : b, kAlign);
}
static size_t merge_flow_bytes(const abf_plan *plan)
{
    return align_up(2 * sizeof(float) * (size_t)plan->max_pixels, kAlign);
}

static size_t merge_box_bytes(int H, int W) { return align_up(4 * sizeof(int32_t) + overlap_box_scratch(H, W), kAlign); }
static size_t merge_crop_bytes(const abf_plan *plan) { return align_up(3 * (size_t)plan->max_pixels, kAlign); }

size_t abf_merge_workspace_bytes(const abf_plan *plan, int32_t H, int32_t W)
{
    if (!plan || H < 1 || W < 1 || H > kCanvasMaxDim || W > kCanvasMaxDim) return 0;
    return merge_tail(plan, H, W) + 2 * merge_flow_bytes(plan) + merge_box_bytes(H, W) + 2 * merge_crop_bytes(plan);
}

abf_status abf_merge_photos(abf_plan *plan, const abf_photo *photos, int32_t n, int32_t H, int32_t W,
                            int32_t pitch_mask, int32_t periodic, uint8_t *canvas, int32_t pitch_canvas,
                            uint8_t *spare, int32_t pitch_spare, uint8_t *coverage, int32_t *boxes, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!photos || n < 1 || !canvas || !spare || !coverage) return fail(plan, ABF_E_INVALID, "null pointer or no photo");
    if (H < 1 || W < 1 || H > kCanvasMaxDim || W > kCanvasMaxDim)
        return fail(plan, ABF_E_SHAPE, "canvas %d x %d (1..%d per side)", H, W, kCanvasMaxDim);
    if (pitch_mask < W || pitch_canvas < 3 * W || pitch_spare < 3 * W)
        return fail(plan, ABF_E_SHAPE, "pitch below the canvas width");
    for (int i = 0; i < n; i++) {
        const abf_photo &p = photos[i];
        if (!p.image || !p.mask) return fail(plan, ABF_E_INVALID, "photo %d: null pointer", i);
        if (p.pitch < 3 * W) return fail(plan, ABF_E_SHAPE, "photo %d: pitch smaller than 3 W", i);
        if ((p.axis != 0 && p.axis != 1) || (p.side != 0 && p.side != 1))
            return fail(plan, ABF_E_INVALID, "photo %d: axis %d, side %d", i, p.axis, p.side);
    }
    if (!plan->ws) return fail(plan, ABF_E_WORKSPACE, "no workspace bound");
    const size_t need = abf_merge_workspace_bytes(plan, H, W);
    if (plan->ws_bytes < need)
        return fail(plan, ABF_E_WORKSPACE, "a %d x %d merge needs %zu workspace bytes, %zu bound", H, W, need,
                    plan->ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    uint8_t *tail = plan->ws + merge_tail(plan, H, W);
    float *flr = reinterpret_cast<float *>(tail);
    float *frl = reinterpret_cast<float *>(tail + merge_flow_bytes(plan));
    int32_t *dbox = reinterpret_cast<int32_t *>(tail + 2 * merge_flow_bytes(plan));
    int32_t *bscr = dbox + 4;  // the box kernels' scratch
    uint8_t *crop[2] = {tail + 2 * merge_flow_bytes(plan) + merge_box_bytes(H, W),
                        tail + 2 * merge_flow_bytes(plan) + merge_box_bytes(H, W) + merge_crop_bytes(plan)};
    uint8_t *buf[2] = {canvas, spare};
    const int32_t pitch[2] = {pitch_canvas, pitch_spare};
    // the buffer that holds the canvas merged so far; chosen so that the
    // last step writes `canvas`
    int cur = (n - 1) % 2 == 0 ? 0 : 1;
    HIP_TRY(plan, launch_photo_init(photos[0].image, photos[0].pitch, photos[0].mask, pitch_mask, H, W, buf[cur],
                                    pitch[cur], coverage, pitch_mask, s));
    if (boxes) boxes[0] = boxes[1] = boxes[2] = boxes[3] = 0;
    BlendParams bp{plan->p.k_sharp, plan->p.k_flowmag, plan->p.blend_mode};
    for (int i = 1; i < n; i++) {
        const abf_photo &p = photos[i];
        // L / R of this pairwise blend: the merged canvas and the photo
        const uint8_t *L = p.side == 0 ? buf[cur] : p.image, *R = p.side == 0 ? p.image : buf[cur];
        const int32_t pL = p.side == 0 ? pitch[cur] : p.pitch, pR = p.side == 0 ? p.pitch : pitch[cur];
        const uint8_t *mL = p.side == 0 ? coverage : p.mask, *mR = p.side == 0 ? p.mask : coverage;
        // the overlap box decides the size of the flow computation: read back
        HIP_TRY(plan, launch_overlap_box(mL, mR, pitch_mask, H, W, periodic != 0, bscr, dbox, s));
        int32_t hb[4];
        HIP_TRY(plan, hipMemcpyAsync(hb, dbox, sizeof(hb), hipMemcpyDeviceToHost, s));
        HIP_TRY(plan, hipStreamSynchronize(s));
        if (boxes) memcpy(boxes + 4 * i, hb, sizeof(hb));
        logf(1, "merge photo %d (axis %d, side %d): overlap box %d %d %d x %d", i, p.axis, p.side, hb[0], hb[1],
             hb[2], hb[3]);
        const bool any = hb[2] > 0 && hb[3] > 0;
        if (any) {
            abf_strip st{};
            if (hb[0] + hb[2] <= W) {
                st.L = L + (size_t)hb[1] * pL + 3 * (size_t)hb[0];
                st.R = R + (size_t)hb[1] * pR + 3 * (size_t)hb[0];
                st.pitch_L = pL;
                st.pitch_R = pR;
            } else {
                // a box across the wrap of a periodic canvas: flows of its contiguous copies
                if ((int64_t)hb[2] * hb[3] > plan->max_pixels)
                    return fail(plan, ABF_E_SHAPE, "merge box %d x %d exceeds the plan", hb[3], hb[2]);
                HIP_TRY(plan, launch_gather_box(L, pL, W, hb[0], hb[1], hb[2], hb[3], crop[0], 3 * hb[2], s));
                HIP_TRY(plan, launch_gather_box(R, pR, W, hb[0], hb[1], hb[2], hb[3], crop[1], 3 * hb[2], s));
                st.L = crop[0];
                st.R = crop[1];
                st.pitch_L = st.pitch_R = 3 * hb[2];
            }
            st.H = hb[3];
            st.W = hb[2];
            st.axis = p.axis;
            st.flow_LtoR = flr;
            st.flow_RtoL = frl;
            abf_status rc = run(plan, &st, 1, true, false, false, s);
            if (rc != ABF_OK) return rc;
        }
        CanvasGeom g{};
        float *bmap = nullptr;
        abf_status rc = canvas_setup(plan, mL, mR, H, W, pitch_mask, periodic != 0, g, &bmap);
        if (rc != ABF_OK) return rc;
        if (any) HIP_TRY(plan, launch_canvas_dist(g, bmap, g.gpitch, nullptr, nullptr, 0, hb, s));
        CompositeArgs o{};
        o.L = L;
        o.R = R;
        o.mL = mL;
        o.mR = mR;
        o.blend = bmap;
        o.pitchB = g.gpitch;
        o.flr = flr;
        o.frl = frl;
        o.F = buf[cur ^ 1];
        o.pitchL = pL;
        o.pitchR = pR;
        o.pitchM = pitch_mask;
        o.pitchF = pitch[cur ^ 1];
        o.H = H;
        o.W = W;
        o.bx = any ? hb[0] : 0;
        o.by = any ? hb[1] : 0;
        o.bw = any ? hb[2] : 0;
        o.bh = any ? hb[3] : 0;
        o.axis = p.axis;
        o.periodic = periodic ? 1 : 0;
        o.inv_ext = any ? 1.0 / (double)(p.axis == 0 ? hb[2] : hb[3]) : 0.0;
        o.cov = coverage;  // coverage |= the photo's mask, in the same pass
        HIP_TRY(plan, launch_composite(o, bp, s));
        cur ^= 1;
    }
    return ABF_OK;
}

// float images of the descent and Code 1 extensions: 32-bit element offsets
static bool float_image_ok(int32_t H, int32_t W)
{
    return H >= 1 && W >= 1 && 3 * (uint64_t)H * (uint64_t)W <= (uint64_t)UINT32_MAX;
}

abf_status abf_energy(abf_plan *plan, const float *Ref, const float *Tgt, const float *u, int32_t H, int32_t W,
                      float lambda, float eps, float *E_dev, float *g_u, float *g_Ref, float *g_Tgt,
                      int32_t deterministic, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!Ref || !Tgt || !u || !E_dev) return fail(plan, ABF_E_INVALID, "null pointer");
    if (!float_image_ok(H, W)) return fail(plan, ABF_E_SHAPE, "size %d x %d (1 <= H, W; 3 H W < 2^32)", H, W);
    if (!(eps * eps >= FLT_MIN) || !(lambda >= 0.f))
        return fail(plan, ABF_E_INVALID, "eps^2 must be a normal float (eps >= 1.1e-19), lambda >= 0");
    const size_t npart = align_up(sizeof(double) * energy_blocks(H, W), kAlign);
    const size_t nfix = (deterministic && g_Tgt) ? align_up(sizeof(uint64_t) * 3 * (size_t)H * W, kAlign) : 0;
    uint8_t *scr = nullptr;
    abf_status rc = grad_scratch(plan, npart + nfix, &scr);
    if (rc != ABF_OK) return rc;
    HIP_TRY(plan, launch_energy_full(Ref, Tgt, u, H, W, lambda, eps, reinterpret_cast<double *>(scr), E_dev, g_u,
                                     g_Ref, g_Tgt, nfix ? reinterpret_cast<unsigned long long *>(scr + npart) : nullptr,
                                     static_cast<hipStream_t>(hip_stream)));
    return ABF_OK;
}

abf_status abf_refine_flow(abf_plan *plan, const float *Ref, const float *Tgt, float *u, int32_t H, int32_t W,
                           int32_t steps, float eta, float lambda, float eps, float clip_px, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!Ref || !Tgt || !u) return fail(plan, ABF_E_INVALID, "null pointer");
    if (!float_image_ok(H, W) || steps < 0)
        return fail(plan, ABF_E_SHAPE, "size %d x %d (1 <= H, W; 3 H W < 2^32), %d steps", H, W, steps);
    if (!(eps * eps >= FLT_MIN) || !(lambda >= 0.f) || !(clip_px >= 0.f))
        return fail(plan, ABF_E_INVALID, "bad parameter (eps^2 must be a normal float, lambda and clip >= 0)");
    if (!aligned8(u)) return fail(plan, ABF_E_INVALID, "u must be 8-byte aligned");
    uint8_t *scr = nullptr;
    abf_status rc = grad_scratch(plan, sizeof(float) * 2 * (size_t)H * W, &scr);
    if (rc != ABF_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    float *bufs[2] = {u, reinterpret_cast<float *>(scr)};
    for (int k = 0; k < steps; k++)
        HIP_TRY(plan, launch_energy_step(Ref, Tgt, bufs[k & 1], bufs[(k + 1) & 1], H, W, eta, lambda, eps, clip_px, s));
    if (steps & 1) HIP_TRY(plan, launch_copy_f32(bufs[1], u, 2 * (int64_t)H * W, s));
    return ABF_OK;
}

// ------------------------------------------------------ multi-level energy
// Scratch of abf_energy_ms (in the workspace's data region): per level
// k >= 1 the reduced Ref, Tgt (3 floats per pixel) and u (2) and, with
// gradients, their gradients (8 floats per pixel); the per-level energies;
// the energy partials; the fixed-point scatter of level 0's dE/dTgt.
extern "C++" {  // helpers with C++ types inside the C-ABI block
namespace {

struct MsLayout {
    int N = 0;
    int h[kMaxLevels] = {}, w[kMaxLevels] = {};
    size_t ref[kMaxLevels] = {}, tgt[kMaxLevels] = {}, u[kMaxLevels] = {};
    size_t gu[kMaxLevels] = {}, gref[kMaxLevels] = {}, gtgt[kMaxLevels] = {};
    size_t El = 0, partials = 0, fix = 0, gstep = 0, bytes = 0;
};

MsLayout ms_layout(int H, int W, int N, bool grads, bool fix, bool step)
{
    MsLayout L;
    L.N = N;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b, kAlign);
        return o;
    };
    for (int k = 0; k < N; k++) {
        L.h[k] = k == 0 ? H : (L.h[k - 1] + 1) / 2;
        L.w[k] = k == 0 ? W : (L.w[k - 1] + 1) / 2;
        if (k == 0) continue;
        const size_t px = (size_t)L.h[k] * L.w[k];
        L.ref[k] = take(sizeof(float) * 3 * px);
        L.tgt[k] = take(sizeof(float) * 3 * px);
        L.u[k] = take(sizeof(float) * 2 * px);
        if (grads) {
            L.gu[k] = take(sizeof(float) * 2 * px);
            L.gref[k] = take(sizeof(float) * 3 * px);
            L.gtgt[k] = take(sizeof(float) * 3 * px);
        }
    }
    L.El = take(sizeof(float) * (kMaxLevels + 1));  // per level, and the descent's energy
    L.partials = take(sizeof(double) * (size_t)energy_blocks(H, W));
    if (fix) L.fix = take(sizeof(unsigned long long) * 3 * (size_t)H * W);
    if (step) L.gstep = take(sizeof(float) * 2 * (size_t)H * W);
    L.bytes = off;
    return L;
}

// The multi-level energy and, where the gradient pointers are non-null, its
// gradients at level 0: the pyramids are built in the scratch, each level's
// energy and gradients computed, and the coarse levels' gradients carried
// to the finer ones through the pyramid's adjoint (1/2 for the flow),
// coarsest first.
// With images_ready the image pyramids are already in the scratch (a
// descent builds them once); with E null only the gradients are formed.
abf_status energy_ms_run(abf_plan *plan, const MsLayout &L, uint8_t *scr, const float *Ref, const float *Tgt,
                         const float *u, float lambda, float eps, float *E, float *g_u, float *g_ref, float *g_tgt,
                         bool det, hipStream_t s, bool images_ready = false)
{
    const int N = L.N;
    auto F = [&](size_t o) { return reinterpret_cast<float *>(scr + o); };
    const float *R[kMaxLevels], *T[kMaxLevels], *U[kMaxLevels];
    R[0] = Ref;
    T[0] = Tgt;
    U[0] = u;
    for (int k = 1; k < N; k++) {
        if (!images_ready) {
            HIP_TRY(plan, launch_pyr_down_f32(R[k - 1], 3, L.h[k - 1], L.w[k - 1], F(L.ref[k]), 1.f, s));
            HIP_TRY(plan, launch_pyr_down_f32(T[k - 1], 3, L.h[k - 1], L.w[k - 1], F(L.tgt[k]), 1.f, s));
        }
        HIP_TRY(plan, launch_pyr_down_f32(U[k - 1], 2, L.h[k - 1], L.w[k - 1], F(L.u[k]), 0.5f, s));
        R[k] = F(L.ref[k]);
        T[k] = F(L.tgt[k]);
        U[k] = F(L.u[k]);
    }
    double *partials = E ? reinterpret_cast<double *>(scr + L.partials) : nullptr;
    float *El = F(L.El);
    unsigned long long *fix = det && g_tgt ? reinterpret_cast<unsigned long long *>(scr + L.fix) : nullptr;
    for (int k = N - 1; k >= 0; k--) {
        float *gu = k == 0 ? g_u : (g_u ? F(L.gu[k]) : nullptr);
        float *gr = k == 0 ? g_ref : (g_ref ? F(L.gref[k]) : nullptr);
        float *gt = k == 0 ? g_tgt : (g_tgt ? F(L.gtgt[k]) : nullptr);
        HIP_TRY(plan, launch_energy_full(R[k], T[k], U[k], L.h[k], L.w[k], lambda, eps, partials, El + k, gu, gr, gt,
                                         gt ? fix : nullptr, s));
        if (k == N - 1) continue;
        if (gu) HIP_TRY(plan, launch_pyr_adj_add_f32(F(L.gu[k + 1]), 2, L.h[k], L.w[k], gu, 0.5f, s));
        if (gr) HIP_TRY(plan, launch_pyr_adj_add_f32(F(L.gref[k + 1]), 3, L.h[k], L.w[k], gr, 1.f, s));
        if (gt) HIP_TRY(plan, launch_pyr_adj_add_f32(F(L.gtgt[k + 1]), 3, L.h[k], L.w[k], gt, 1.f, s));
    }
    if (E) HIP_TRY(plan, launch_sum_levels(El, N, E, s));
    return ABF_OK;
}

}  // namespace
}  // extern "C++"

size_t abf_energy_ms_workspace_bytes(const abf_plan *plan, int32_t H, int32_t W, int32_t levels)
{
    if (!plan || H < 1 || W < 1 || levels < 1 || levels > kMaxLevels) return 0;
    // gradients, the deterministic scatter and the descent's gradient: the
    // most any call of the two entry points takes
    const size_t need = plan->hdr_cap + ms_layout(H, W, levels, true, true, true).bytes;
    const size_t base = abf_workspace_bytes(plan);
    return need > base ? need : base;
}

abf_status abf_energy_ms(abf_plan *plan, const float *Ref, const float *Tgt, const float *u, int32_t H, int32_t W,
                         int32_t levels, float lambda, float eps, float *E_dev, float *g_u, float *g_Ref, float *g_Tgt,
                         int32_t deterministic, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!Ref || !Tgt || !u || !E_dev) return fail(plan, ABF_E_INVALID, "null pointer");
    if (!float_image_ok(H, W)) return fail(plan, ABF_E_SHAPE, "size %d x %d (1 <= H, W; 3 H W < 2^32)", H, W);
    if (levels < 1 || levels > kMaxLevels) return fail(plan, ABF_E_INVALID, "levels %d (1..%d)", levels, kMaxLevels);
    if (!(eps * eps >= FLT_MIN) || !(lambda >= 0.f))
        return fail(plan, ABF_E_INVALID, "eps^2 must be a normal float (eps >= 1.1e-19), lambda >= 0");
    const bool grads = g_u || g_Ref || g_Tgt;
    const MsLayout L = ms_layout(H, W, levels, grads, deterministic && g_Tgt, false);
    uint8_t *scr = nullptr;
    abf_status rc = grad_scratch(plan, L.bytes, &scr);
    if (rc != ABF_OK) return rc;
    return energy_ms_run(plan, L, scr, Ref, Tgt, u, lambda, eps, E_dev, g_u, g_Ref, g_Tgt, deterministic != 0,
                         static_cast<hipStream_t>(hip_stream));
}

abf_status abf_refine_flow_ms(abf_plan *plan, const float *Ref, const float *Tgt, float *u, int32_t H, int32_t W,
                              int32_t levels, int32_t steps, float eta, float lambda, float eps, float clip_px,
                              void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!Ref || !Tgt || !u) return fail(plan, ABF_E_INVALID, "null pointer");
    if (!float_image_ok(H, W) || steps < 0)
        return fail(plan, ABF_E_SHAPE, "size %d x %d (1 <= H, W; 3 H W < 2^32), %d steps", H, W, steps);
    if (levels < 1 || levels > kMaxLevels) return fail(plan, ABF_E_INVALID, "levels %d (1..%d)", levels, kMaxLevels);
    if (!(eps * eps >= FLT_MIN) || !(lambda >= 0.f) || !(clip_px >= 0.f))
        return fail(plan, ABF_E_INVALID, "bad parameter (eps^2 must be a normal float, lambda and clip >= 0)");
    const MsLayout L = ms_layout(H, W, levels, true, false, true);
    uint8_t *scr = nullptr;
    abf_status rc = grad_scratch(plan, L.bytes, &scr);
    if (rc != ABF_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    float *g = reinterpret_cast<float *>(scr + L.gstep);
    for (int k = 0; k < steps; k++) {
        // gradients only; the image pyramids are built by the first step
        rc = energy_ms_run(plan, L, scr, Ref, Tgt, u, lambda, eps, nullptr, g, nullptr, nullptr, false, s, k > 0);
        if (rc != ABF_OK) return rc;
        HIP_TRY(plan, launch_clip_step(u, g, 2 * (int64_t)H * W, eta, clip_px, s));
    }
    return ABF_OK;
}

abf_status abf_blend_asymmetric_f32(abf_plan *plan, const float *L, const float *R, const float *flow_LtoR,
                                    const float *flow_RtoL, const float *blend, int32_t axis, int32_t H, int32_t W,
                                    float *F, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!L || !R || !flow_LtoR || !flow_RtoL || !F) return fail(plan, ABF_E_INVALID, "null pointer");
    if (!float_image_ok(H, W)) return fail(plan, ABF_E_SHAPE, "size %d x %d (1 <= H, W; 3 H W < 2^32)", H, W);
    if (axis != 0 && axis != 1) return fail(plan, ABF_E_INVALID, "axis %d", axis);
    BlendParams bp{plan->p.k_sharp, plan->p.k_flowmag, plan->p.blend_mode};
    HIP_TRY(plan, launch_blend_f32(L, R, flow_LtoR, flow_RtoL, blend, axis, H, W, bp, F,
                                   static_cast<hipStream_t>(hip_stream)));
    return ABF_OK;
}

abf_status abf_blend_backward(abf_plan *plan, const float *L, const float *R, const float *flow_LtoR,
                              const float *flow_RtoL, const float *blend, int32_t axis, int32_t H, int32_t W,
                              const float *g_F, float *g_flow_LtoR, float *g_flow_RtoL, float *g_L, float *g_R,
                              int32_t deterministic, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!L || !R || !flow_LtoR || !flow_RtoL || !g_F) return fail(plan, ABF_E_INVALID, "null pointer");
    if (!float_image_ok(H, W)) return fail(plan, ABF_E_SHAPE, "size %d x %d (1 <= H, W; 3 H W < 2^32)", H, W);
    if (axis != 0 && axis != 1) return fail(plan, ABF_E_INVALID, "axis %d", axis);
    if (!aligned8(flow_LtoR) || !aligned8(flow_RtoL)) return fail(plan, ABF_E_INVALID, "flows must be 8-byte aligned");
    const bool det = deterministic != 0 && (g_L || g_R);
    const size_t nfix = align_up(sizeof(uint64_t) * 3 * (size_t)H * W, kAlign);
    uint8_t *scr = nullptr;
    if (det) {
        abf_status rc = grad_scratch(plan, 2 * nfix + kAlign, &scr);
        if (rc != ABF_OK) return rc;
    }
    BlendParams bp{plan->p.k_sharp, plan->p.k_flowmag, plan->p.blend_mode};
    HIP_TRY(plan, launch_blend_bwd_full(L, R, flow_LtoR, flow_RtoL, blend, axis, H, W, bp, g_F, g_flow_LtoR,
                                        g_flow_RtoL, g_L, g_R,
                                        det ? reinterpret_cast<unsigned long long *>(scr) : nullptr,
                                        det ? reinterpret_cast<unsigned long long *>(scr + nfix) : nullptr,
                                        det ? reinterpret_cast<uint32_t *>(scr + 2 * nfix) : nullptr,
                                        static_cast<hipStream_t>(hip_stream)));
    return ABF_OK;
}

abf_status abf_profile(abf_plan *plan, const abf_strip *strips, int32_t n, int32_t reps, float *ms_out,
                       void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!strips || n < 1 || reps < 1 || !ms_out) return fail(plan, ABF_E_INVALID, "bad arguments");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Batch b;
    abf_status rc = build_batch(plan, strips, n, true, true, b);
    if (rc != ABF_OK) return rc;
    for (int i = 0; i < kStages * kMaxLevels; i++) ms_out[i] = 0.f;
    for (int r = 0; r < reps; r++) {
        rc = upload(plan, b, s);
        if (rc != ABF_OK) return rc;
        Prof prof;
        rc = enqueue(plan, b, true, true, s, &prof);
        hipError_t e = hipStreamSynchronize(s);
        for (size_t i = 0; i + 1 < prof.ev.size(); i += 2) {
            float t = 0.f;
            if (rc == ABF_OK && e == hipSuccess && hipEventElapsedTime(&t, prof.ev[i], prof.ev[i + 1]) == hipSuccess)
                ms_out[prof.tag[i / 2].first * kMaxLevels + prof.tag[i / 2].second] += t / reps;
        }
        for (hipEvent_t ev : prof.ev) (void)hipEventDestroy(ev);
        if (rc != ABF_OK) return rc;
        if (e != hipSuccess) return hip_fail(plan, e, "hipStreamSynchronize");
    }
    plan->lv_host = b.lv;
    plan->last_n = n;
    return ABF_OK;
}

abf_status abf_refine_strips(abf_plan *plan, const abf_refine_strip *strips, int32_t n, int32_t steps, float eta,
                             float lambda, float eps, float clip_px, void *hip_stream)
{
    if (!plan) return ABF_E_INVALID;
    if (!strips || n < 1 || steps < 0) return fail(plan, ABF_E_INVALID, "bad arguments");
    if (n > plan->max_strips) return fail(plan, ABF_E_SHAPE, "%d strips exceed the plan's %d", n, plan->max_strips);
    if (!(eps * eps >= FLT_MIN) || !(lambda >= 0.f) || !(clip_px >= 0.f))
        return fail(plan, ABF_E_INVALID, "bad parameter (eps^2 must be a normal float, lambda and clip >= 0)");
    if (!plan->ws) return fail(plan, ABF_E_WORKSPACE, "no workspace bound");
    std::vector<RefineDesc> d(n);
    std::vector<int32_t> prefix(n + 1);
    size_t off = plan->hdr_cap;
    int64_t acc = 0;
    for (int i = 0; i < n; i++) {
        const abf_refine_strip &x = strips[i];
        if (!x.Ref || !x.Tgt || !x.u) return fail(plan, ABF_E_INVALID, "strip %d: null pointer", i);
        if (!aligned8(x.u)) return fail(plan, ABF_E_INVALID, "strip %d: u must be 8-byte aligned", i);
        if (!float_image_ok(x.H, x.W))
            return fail(plan, ABF_E_SHAPE, "strip %d: size %d x %d (1 <= H, W; 3 H W < 2^32)", i, x.H, x.W);
        d[i].Ref = x.Ref;
        d[i].Tgt = x.Tgt;
        d[i].u[0] = x.u;
        d[i].u[1] = reinterpret_cast<float *>(plan->ws + off);
        d[i].H = x.H;
        d[i].W = x.W;
        off += align_up(sizeof(float) * 2 * (size_t)x.H * x.W, kAlign);
        prefix[i] = (int32_t)acc;
        acc += ceil_div(x.H * x.W, 256);
    }
    prefix[n] = (int32_t)acc;
    if (off > plan->ws_bytes)
        return fail(plan, ABF_E_WORKSPACE, "batch needs %zu workspace bytes, %zu bound", off, plan->ws_bytes);
    if (acc > 0x7fffffff) return fail(plan, ABF_E_SHAPE, "too many tiles");
    const size_t dbytes = align_up(sizeof(RefineDesc) * n, kAlign);
    std::vector<uint8_t> host(dbytes + sizeof(int32_t) * (n + 1), 0);
    memcpy(host.data(), d.data(), sizeof(RefineDesc) * n);
    memcpy(host.data() + dbytes, prefix.data(), sizeof(int32_t) * (n + 1));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    abf_status rc = upload_bytes(plan, host, s);
    if (rc != ABF_OK) return rc;
    HIP_TRY(plan, launch_refine_batch(reinterpret_cast<const RefineDesc *>(plan->ws),
                                      reinterpret_cast<const int32_t *>(plan->ws + dbytes), n, (int)acc, steps, eta,
                                      lambda, eps, clip_px, s));
    return ABF_OK;
}

}  // extern "C"
