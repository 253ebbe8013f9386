// Internal definitions shared by the HIP kernels and the host runtime of
// libabf. Nothing here is part of the public ABI (include/abf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace abf {

constexpr int kMaxLevels = 12;
// Luma planes carry a border of kPad replicated pixels on every side, so a
// window that leaves the image by up to kPad pixels reads exactly the
// clamp-to-edge values without per-access clamping.
constexpr int kPad = 64;
// bytes of slack before (and after) every padded plane: the aligned row
// loads may read up to 3 bytes outside the padded rows
constexpr int kPlaneLead = 64;
constexpr int kStages = 6;       // luma, pyramid, search, propagation, refine, blend
constexpr int kSizeClasses = 4;  // by pixel count of one level over the batch

enum Stage { ST_LUMA = 0, ST_PYR = 1, ST_SEARCH = 2, ST_PROP = 3, ST_REFINE = 4, ST_BLEND = 5 };
// work lists: one per stage plus the refinement's border pixels
constexpr int kLists = kStages + 1;
constexpr int LIST_REFINE_BORDER = kStages;

// One strip at one pyramid level, as the kernels see it. Direction d uses
// y[d] as Ref and y[1 - d] as Tgt (d = 0: LtoR, d = 1: RtoL). Integer
// flows are int16 pairs packed in one uint32 (x low, y high).
struct StripLv {
    uint8_t *y[2];          // luma of L and R at this level (pitch ypitch bytes)
    uint32_t *ds[2];        // raw search result per direction (pitch fpitch)
    uint16_t *cs[2];        // its patch cost
    uint32_t *df[2];        // final flow of the level per direction
    const uint32_t *dc[2];  // final flow of the next coarser level (null at the coarsest)
    const uint8_t *yfine[2];// luma of the next finer level (pyramid input; null at level 0)
    int32_t H, W, ypitch, fpitch;
    int32_t Hc, Wc, fpitch_c;
    int32_t Hf, Wf, ypitch_f;  // finer level geometry (pyramid input)
    int32_t radius;
    int32_t pad_;
};

// The caller's buffers of one strip.
// slots per exposure sum (spread of the luma kernel's atomics); after the
// two sums' slots: the gain a of the exposure step
constexpr int kSumSlots = 64;
constexpr int kSumGain = 2 * kSumSlots;
constexpr int kSumWords = 2 * kSumSlots + 1;

struct StripIO {
    const uint8_t *L, *R;
    unsigned long long *sums;  // device: intensity sums of L, R (kSumSlots slots each), then the gain
    const float *blend;
    float *flow[2];  // [0] = FlowLtoR, [1] = FlowRtoL
    uint8_t *F;
    float *Ff32;
    int32_t pitchL, pitchR, pitchF;
    int32_t H, W, axis;
    int32_t pad_;
    double inv_ext1;  // 1 / (extent + 1) across the seam (eq. (1) ramp)
    double inv_ext;   // 1 / extent across the seam (flow magnitude scale)
};

// Launch of one stage over a batch: the strip table, per-strip tile
// prefix sums (n + 1 entries, device) and the total tile count.
struct Work {
    const int32_t *prefix;  // device
    int32_t n;              // strips
    int32_t total;          // tiles over all strips
};

// Float parameters the kernels take by value.
struct LkParams {
    // (Lucas-Kanade refinement)
    int32_t patch, iters;
    float eps;
};

struct BlendParams {
    float k_sharp, k_flowmag;
    int32_t mode;
};

// Tile geometry per stage, shared by host and device (tiles per strip are
// computed identically on both sides).
__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// search tiles: 128 x TH pixels (64 threads per row, two pixels each);
// refine: 64 x TH; propagation: (64 - 2h) x TH outputs, TH = 8, 10, 16 or 32; luma, exposure step and blend:
// 256 pixels of one row; pyramid: 256 x 4 output pixels (4 per thread). Luma, exposure
// and pyramid tiles cover the padded planes.
constexpr int kSearchTW = 128;
constexpr int kRefineTW = 64;
constexpr int kRowTW = 256;
constexpr int kPyrTW = 256;
constexpr int kPyrTH = 8;  // a wave per two output rows

// ---------------------------------------------------------------------
// Kernel launchers (defined in abf_kernels.hip). Each returns the HIP
// error of the launch. `grid` = 0 launches one workgroup per tile;
// otherwise that many persistent workgroups loop over the tiles.
// sums: also the luma sums of the exposure step
hipError_t launch_luma(const StripIO *io, const StripLv *lv0, Work w, int grid, bool sums, hipStream_t s);
hipError_t launch_zero_sums(const StripIO *io, int n, hipStream_t s);
hipError_t launch_gain(const StripIO *io, const StripLv *lv0, Work w, int grid, hipStream_t s);
hipError_t launch_pyr(const StripLv *lv, Work w, int grid, hipStream_t s);
hipError_t launch_search(const StripLv *lv, Work w, int patch, int radius, int th, int grid, hipStream_t s);
// the T propagation steps and the median of one level (one launch)
hipError_t launch_prop(const StripLv *lv, Work w, int patch, int steps, int median, int th, int grid, hipStream_t s);
// refine: interior tiles and, separately, the border pixels
hipError_t launch_refine(const StripLv *lv0, const StripIO *io, Work w, LkParams lk, int th, int grid, hipStream_t s);
hipError_t launch_refine_border(const StripLv *lv0, const StripIO *io, Work w, LkParams lk, hipStream_t s);
// blend: px (1, 2 or 4) pixels per thread, px * kRowTW per tile
hipError_t launch_blend(const StripIO *io, Work w, BlendParams bp, int px, int grid, hipStream_t s);
// classic coarse-to-fine Lucas-Kanade, one level (flow method 1): the
// border pixels on the refinement's border list of the level and the
// interior pixels (exact pair sums) on its refinement tiles (th 2 or 4);
// lvc = the next coarser level's entries (null at the coarsest); level0
// writes the caller's flows
hipError_t launch_lk_border(const StripLv *lv, const StripLv *lvc, const StripIO *io, Work w, LkParams lk, bool level0,
                            hipStream_t s);
hipError_t launch_lk_interior(const StripLv *lv, const StripLv *lvc, const StripIO *io, Work w, LkParams lk, int th,
                              int grid, bool level0, hipStream_t s);

// One strip of a batched refinement: u[0] is the caller's flow, u[1] the
// other half of the descent ping-pong (workspace).
struct RefineDesc {
    const float *Ref, *Tgt;
    float *u[2];
    int32_t H, W;
};
hipError_t launch_refine_batch(const RefineDesc *d, const int32_t *prefix, int n, int total, int steps, float eta,
                               float lambda, float eps, float clip, hipStream_t s);

// differentiable path (float images); `fix` buffers (3 H W uint64) select
// the deterministic fixed-point scatter, null selects float atomics (for
// the Code 1 adjoint, `gmax` (one uint32) selects it)
int energy_blocks(int H, int W);
hipError_t launch_energy_full(const float *Ref, const float *Tgt, const float *u, int H, int W, float lambda,
                              float eps, double *partials, float *E, float *g_u, float *g_ref, float *g_tgt,
                              unsigned long long *fix, hipStream_t s);
hipError_t launch_energy_step(const float *Ref, const float *Tgt, const float *u_in, float *u_out, int H, int W,
                              float eta, float lambda, float eps, float clip, hipStream_t s);
hipError_t launch_copy_f32(const float *src, float *dst, int64_t n, hipStream_t s);
// multi-level energy: one level of the float pyramid of a C-channel (2 or 3)
// HWC array, times scale; g += scale * its adjoint applied to G (G holds the
// coarse level of an H x W array); the sum of per-level energies; the
// clipped descent update u -= clip(eta g)
hipError_t launch_pyr_down_f32(const float *x, int C, int H, int W, float *y, float scale, hipStream_t s);
hipError_t launch_pyr_adj_add_f32(const float *G, int C, int H, int W, float *g, float scale, hipStream_t s);
hipError_t launch_sum_levels(const float *El, int n, float *E, hipStream_t s);
hipError_t launch_clip_step(float *u, const float *g, int64_t n, float eta, float clip, hipStream_t s);
hipError_t launch_blend_f32(const float *L, const float *R, const float *flr, const float *frl, const float *blend,
                            int axis, int H, int W, BlendParams bp, float *F, hipStream_t s);
hipError_t launch_blend_bwd_full(const float *L, const float *R, const float *flr, const float *frl,
                                 const float *blend, int axis, int H, int W, BlendParams bp, const float *gF,
                                 float *g_flr, float *g_frl, float *g_L, float *g_R, unsigned long long *fixL,
                                 unsigned long long *fixR, uint32_t *gmax, hipStream_t s);

// ---------------------------------------------------------------------
// Canvas compositing (defined in abf_canvas.hip). Canvases are at most
// kCanvasMaxDim on a side, so squared distances fit in 31 bits and row
// distances in uint16 (0xffff = no pixel of the area in the row).
constexpr int kCanvasMaxDim = 32767;
constexpr int kCanvasChunk = 16;    // columns per thread in the row pass
constexpr int kCanvasThreads = 256;
constexpr int kCanvasMaxChunks = (kCanvasMaxDim + kCanvasChunk - 1) / kCanvasChunk;
constexpr int kCanvasBH = 16;       // rows per block minimum of the column search
static_assert(kCanvasMaxChunks <= 8 * kCanvasThreads, "row scan holds 8 chunks per thread");

// Coverage masks and the scratch planes of the distance passes: G holds
// the row distance to Area1 (low half) and Area2 (high half) of every
// pixel, M its minimum over each kCanvasBH-row block of a column; both
// have gpitch (a multiple of 64) entries per row.
struct CanvasGeom {
    const uint8_t *mL, *mR;
    uint32_t *G, *M;
    int32_t pitchM, H, W, gpitch;
    int32_t periodic;  // columns wrap (W - 1 neighbours 0): row distances the shorter way round
    int32_t gx0, gx1;  // columns [gx0, gx1) of G that are written (every row is scanned whole)
    int32_t pad_;
};
__host__ __device__ inline int canvas_gpitch(int W) { return (W + 63) / 64 * 64; }

struct CompositeArgs {
    const uint8_t *L, *R, *mL, *mR;
    const float *blend;       // canvas Blend map (pitchB floats per row)
    const float *flr, *frl;   // bh x bw x 2 over the overlap box
    uint8_t *F;
    float *Ff32;              // H x W x 3 contiguous, or null
    uint8_t *cov;             // union of the coverages (pitchM), or null
    int32_t pitchL, pitchR, pitchM, pitchB, pitchF;
    int32_t H, W, bx, by, bw, bh, axis;
    int32_t periodic;         // columns wrap: the box's columns are bx .. bx + bw - 1 modulo W
    double inv_ext;           // 1 / the box's extent across the seam
};

// part: scratch of 2 H int32 (row extents) + ceil(W / 32) uint32 (the
// column occupancy of a periodic canvas)
inline size_t overlap_box_scratch(int H, int W) { return sizeof(int32_t) * (2 * (size_t)H + (W + 31) / 32); }
hipError_t launch_overlap_box(const uint8_t *mL, const uint8_t *mR, int pitchM, int H, int W, bool periodic,
                              int32_t *part, int32_t *box, hipStream_t s);
// copy of a box of an RGB canvas image whose columns wrap modulo W into a
// contiguous bh x bw x 3 buffer (rows pitchD bytes apart)
hipError_t launch_gather_box(const uint8_t *img, int pitch, int W, int bx, int by, int bw, int bh, uint8_t *dst,
                             int pitchD, hipStream_t s);
// eq. (1) distances and Blend over the canvas, or (box = {x, y, w, h}, not
// null) over the 64 x 16 tiles that meet the box (all columns if the box
// crosses the wrap of a periodic canvas): the composite reads Blend only
// inside the box
hipError_t launch_canvas_dist(const CanvasGeom &a, float *blend, int pitchB, int32_t *d1, int32_t *d2, int pitchD,
                              const int32_t *box, hipStream_t s);
hipError_t launch_composite(const CompositeArgs &o, BlendParams bp, hipStream_t s);
hipError_t launch_photo_init(const uint8_t *img, int pitchI, const uint8_t *mask, int pitchM, int H, int W,
                             uint8_t *dst, int pitchD, uint8_t *cov, int pitchC, hipStream_t s);

// tiles of one strip for a stage (both directions where the stage has two)
// luma and exposure: 4 pixels per thread over the padded rows
constexpr int kLumaTW = 4 * kRowTW;
__host__ __device__ inline int tiles_luma(int H, int W) { return (H + 2 * kPad) * ceil_div(W + 2 * kPad, kLumaTW); }
__host__ __device__ inline int tiles_pyr(int H, int W)
{
    return ceil_div(H + 2 * kPad, kPyrTH) * ceil_div(W + 2 * kPad, kPyrTW);
}
__host__ __device__ inline int tiles_search(int H, int W, int th) { return 2 * ceil_div(H, th) * ceil_div(W, kSearchTW); }
// fused propagation (T steps + median, halo h = T + M <= kPropMaxHalo):
// one wave per tile of (kPropRW - 2h) x th outputs over a
// kPropRW x (th + 2h) region held in registers (th = 8, 10, 16 or 32)
constexpr int kPropRW = 64;
constexpr int kPropMaxHalo = 5;
__host__ __device__ inline int tiles_prop(int H, int W, int th, int h)
{
    return 2 * ceil_div(H, th) * ceil_div(W, kPropRW - 2 * h);
}
// refine: tiles of 64 x th pixels over the interior rectangle (window
// inside the image) per direction; the border band around it (per
// direction) in tiles of kRowTW pixels enumerated along the band
struct RefineSplit {
    int ylo, yhi, xlo, xhi;  // interior rows [ylo, yhi), columns [xlo, xhi)
    int nint, nbp;           // interior tiles, border pixels
};
__host__ __device__ inline RefineSplit refine_split(int H, int W, int th, int lp)
{
    RefineSplit r;
    r.ylo = H < lp ? H : lp;
    r.yhi = H - lp > r.ylo ? H - lp : r.ylo;
    r.xlo = W < lp ? W : lp;
    r.xhi = W - lp > r.xlo ? W - lp : r.xlo;
    r.nint = ceil_div(r.yhi - r.ylo, th) * ceil_div(r.xhi - r.xlo, kRefineTW);
    r.nbp = H * W - (r.yhi - r.ylo) * (r.xhi - r.xlo);
    return r;
}
__host__ __device__ inline int tiles_refine(int H, int W, int th, int lp) { return 2 * refine_split(H, W, th, lp).nint; }
__host__ __device__ inline int tiles_refine_border(int H, int W, int lp)
{
    return 2 * ceil_div(refine_split(H, W, 1, lp).nbp, kRowTW);
}
__host__ __device__ inline int tiles_blend(int H, int W, int px) { return H * ceil_div(W, px * kRowTW); }

}  // namespace abf
