/*
 * abf.h - C ABI of libabf: asymmetric bidirectional optical flow and
 * asymmetric blending of panorama overlap strips on AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Meng & Liu, "High-quality Panorama Stitching based on Asymmetric
 * Bidirectional Optical Flow" (arXiv 2006.01201), Section III.C:
 *   - III.C.1: two dense flows per overlap strip, FlowRtoL (OverlappedR
 *     relative to OverlappedL) and FlowLtoR, by a coarse-to-fine pyramid
 *     method;
 *   - III.C.2, eq. (1): the global blending coefficient Blend;
 *   - III.C.3, Code 1: per-pixel warp of L by FlowRtoL * Blend and of R by
 *     FlowLtoR * (1 - Blend), then a softmax composite into F.
 *
 * Conventions shared by every call:
 *   - A strip is H rows x W columns and is the whole of Area3 (the
 *     overlap); L and R are its two crops, OverlappedL and OverlappedR.
 *   - Images are RGB uint8, interleaved (HWC), rows `pitch` bytes apart
 *     (pitch >= 3 W). Flows are float32 H x W x 2, contiguous, (x, y) =
 *     (column, row) components, 8-byte aligned (each pixel's pair is one
 *     64-bit access; ABF_E_INVALID otherwise).
 *   - Flow sense: Ref(p) ~ Tgt(p + u(p)). FlowRtoL has Ref = R and Tgt = L
 *     (R(p) ~ L(p + FlowRtoL(p))); FlowLtoR has Ref = L and Tgt = R.
 *   - axis 0: Area1 (only L) lies left of the strip and Area2 right of it;
 *     axis 1: Area1 above, Area2 below.
 *   - All pointers named as device pointers point to device memory owned
 *     by the caller. The library never allocates device memory on the hot
 *     path: scratch comes from one caller-provided workspace.
 *   - Calls are asynchronous on the given HIP stream (NULL = the default
 *     stream); a kernel fault surfaces at the next synchronisation.
 *   - A plan is bound to the device current at creation, and is not
 *     thread-safe: use one plan per stream.
 *   - Errors are returned as abf_status; no C++ exception crosses the ABI.
 *     abf_last_error() gives the text of the last failure of a plan. The
 *     environment variable ABF_LOG (read once) writes a log to stderr:
 *     1 = failures, plan and graph set-up, tuning choices, merge steps;
 *     2 = also every batched call.
 */
#ifndef ABF_H
#define ABF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum abf_status {
    ABF_OK = 0,
    ABF_E_INVALID = 1,     /* null pointer, bad parameter value */
    ABF_E_SHAPE = 2,       /* sizes inconsistent or beyond the plan's limits */
    ABF_E_WORKSPACE = 3,   /* no workspace bound, or too small */
    ABF_E_DEVICE = 4,      /* a HIP runtime error (text in abf_last_error) */
    ABF_E_UNSUPPORTED = 5, /* no device, not gfx950, or a parameter value the kernels do not implement */
    ABF_E_CAPTURE = 6      /* hipGraph capture or instantiation failed */
} abf_status;

/* Parameters that change results. The paper publishes no values for its
 * flow method or for kSoftmaxSharpness / kFlowMagCoef (Section III.C.3);
 * abf_default_params() fills the adopted defaults. */
typedef struct abf_params {
    int32_t levels;        /* pyramid levels N, 1..12 */
    int32_t patch;         /* P: (2P+1)^2 patch for the integer search; 1 or 2 */
    int32_t radius;        /* R: search radius at every level but the coarsest; 1..4 */
    int32_t radius_coarse; /* search radius at the coarsest level; 1..4 */
    int32_t prop_steps;    /* T: Jacobi propagation steps per level; 0..4 */
    int32_t median;        /* M: (2M+1)^2 component-wise median per level; 0 or 1 */
    int32_t lk_patch;      /* (2P+1)^2 window of the level-0 Lucas-Kanade refinement; 1..3 */
    int32_t lk_iters;      /* Gauss-Newton iterations; 0..8 */
    float lk_eps;          /* Tikhonov term added to the window-summed normal matrix; > 0 */
    float k_sharp;         /* kSoftmaxSharpness of Code 1 */
    float k_flowmag;       /* kFlowMagCoef of Code 1 (flow magnitude is divided by the strip
                              extent across the seam: W for axis 0, H for axis 1) */
    int32_t blend_mode;    /* 0: softmax composite of Code 1; 1: linear weights (SoftmaxR = Blend) */
    int32_t gain_comp;     /* 1: before the pyramid, scale R's intensity by the ratio of the two
                              strips' intensity sums (16-bit fixed point: a = floor(2^16 sum(YL) /
                              sum(YR)), YR' = min(255, (YR a + 2^15) >> 16)) to remove a residual
                              exposure gain left by pre-processing (Section III.B); 0: off, the
                              default (colour correction is the caller's pre-processing, and with
                              the step off a pure integer shift gives exactly that flow) */
    int32_t flow_method;   /* 0: integer patch search, propagation and median per level, then the
                              level-0 Lucas-Kanade refinement (the default); 1: the classic
                              coarse-to-fine Lucas-Kanade of Section III.C.1: at every level a
                              float flow from twice the coarser level's flow at (x/2, y/2) takes
                              lk_iters unclamped Gauss-Newton steps over the lk_patch window
                              (patch, radius, radius_coarse, prop_steps and median unused) */
} abf_params;

typedef struct abf_plan abf_plan;

/* One strip of a batch for abf_stitch_strips. Inputs: L, R, blend
 * (nullable: eq. (1) ramp). Outputs: both flows and F; F_f32 (nullable)
 * receives the unrounded composite, float32 H x W x 3 contiguous. */
typedef struct abf_strip {
    const uint8_t *L;
    const uint8_t *R;
    int32_t H, W;
    int32_t pitch_L, pitch_R;
    int32_t axis;
    const float *blend;
    float *flow_LtoR;
    float *flow_RtoL;
    uint8_t *F;
    int32_t pitch_F;
    float *F_f32;
} abf_strip;

/* Fills the adopted defaults: N = 6, P = 2, R = 2, Rc = 4, T = 2, M = 1,
 * lk window 5 x 5, 2 iterations, eps 25, kSoftmaxSharpness 10,
 * kFlowMagCoef 20, softmax blend, exposure step off, flow method 0. */
void abf_default_params(abf_params *p);

/* Creates a plan for batches of at most max_strips strips whose level-0
 * pixel counts sum to at most max_pixels, each strip at most max_H x max_W.
 * Checks the parameters (ABF_E_INVALID / ABF_E_UNSUPPORTED) and the device
 * (ABF_E_UNSUPPORTED without a gfx950 device). *out receives the plan. */
abf_status abf_create_plan(const abf_params *params, int32_t max_strips, int64_t max_pixels,
                           int32_t max_H, int32_t max_W, abf_plan **out);

/* Device bytes the workspace must hold for the plan's limits. */
size_t abf_workspace_bytes(const abf_plan *plan);

/* Binds caller-owned device memory (at least abf_workspace_bytes, 256-byte
 * aligned) as the plan's workspace: image pyramids, integer flows of every
 * level and the batch descriptor tables. The memory must stay valid while
 * the plan uses it; rebinding replaces it. */
abf_status abf_bind_workspace(abf_plan *plan, void *dev_ptr, size_t bytes);

/* Section III.C.1: FlowLtoR and FlowRtoL of one strip. Device pointers:
 * L, R (inputs), flow_LtoR, flow_RtoL (outputs, float32 H x W x 2).
 * Pipeline: luma, binomial pyramid, per level from coarse to fine an
 * integer patch-cost search around the upsampled coarser flow, Jacobi
 * propagation and a median, then Lucas-Kanade refinement at level 0.
 * ABF_E_SHAPE if the coarsest level would be smaller than 1 x 1 or the
 * strip exceeds the plan. */
abf_status abf_flow_bidirectional(abf_plan *plan, const uint8_t *L, const uint8_t *R, int32_t H,
                                  int32_t W, int32_t pitch_L, int32_t pitch_R, float *flow_LtoR,
                                  float *flow_RtoL, void *hip_stream);

/* Allocation-free variant of abf_flow_bidirectional, for callers that
 * cannot allocate device memory (code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same arguments, kernels and
 * results; the flow path's scratch (pyramids, integer flows of every level,
 * descriptor tables) lives in a static device array of
 * ABF_NOALLOC_SCRATCH_BYTES per device, which the library holds from the
 * first plan on that device until the process ends, instead of the plan's
 * workspace (none need be bound). The call allocates no device memory
 * (no hipMalloc or hipFree; the descriptor tables go through the plan's
 * pinned staging, a host-to-device copy on hip_stream). ABF_E_WORKSPACE if
 * the strip's layout exceeds the array (at 6 levels, strips up to about
 * 2 Mpx fit). Every call on one device shares that device's array, which
 * keeps the last call's contents (everything the path reads is written
 * first in the same call): calls that overlap in time on one device (two
 * streams, plans or threads) race and give wrong results, so order them on
 * one stream. */
#define ABF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
abf_status abf_flow_bidirectional_noalloc(abf_plan *plan, const uint8_t *L, const uint8_t *R, int32_t H,
                                          int32_t W, int32_t pitch_L, int32_t pitch_R, float *flow_LtoR,
                                          float *flow_RtoL, void *hip_stream);

/* Code 1 with eq. (1) over one strip. Device pointers: L, R, flow_LtoR,
 * flow_RtoL, blend (nullable: eq. (1) for a rectangular strip,
 * Blend = (x+1)/(W+1) for axis 0, (y+1)/(H+1) for axis 1; otherwise a
 * float32 H x W array of Blend values); F (output, uint8 RGB with pitch_F,
 * round half up, clamped); F_f32 (nullable output, float32 H x W x 3). A
 * non-finite flow component is used as 0. */
abf_status abf_blend_asymmetric(abf_plan *plan, const uint8_t *L, const uint8_t *R,
                                const float *flow_LtoR, const float *flow_RtoL, const float *blend,
                                int32_t axis, int32_t H, int32_t W, int32_t pitch_L, int32_t pitch_R,
                                uint8_t *F, int32_t pitch_F, float *F_f32, void *hip_stream);

/* Both flows and the blend for a batch of n strips (host array of
 * descriptors; the pointers inside are device pointers), with one launch
 * per pyramid level and stage covering all strips. Results equal those of
 * per-strip abf_flow_bidirectional + abf_blend_asymmetric bit for bit.
 * use_graph != 0 captures the launch sequence in a hipGraph per batch
 * shape and replays it (ABF_E_CAPTURE if capture fails). */
abf_status abf_stitch_strips(abf_plan *plan, const abf_strip *strips, int32_t n, int32_t use_graph,
                             void *hip_stream);

/* Destroys a plan (host state only; the workspace stays the caller's). */
abf_status abf_destroy(abf_plan *plan);

const char *abf_status_string(abf_status s);
const char *abf_last_error(const abf_plan *plan);

/* ------------------------------------------------------------------ */
/* Introspection of the workspace after a call, for tests: a device
 * pointer to one intermediate of strip `strip` (0-based position in the
 * last call's batch; 0 for the single-strip calls), level `level`,
 * direction `dir` (0: LtoR, Ref = L; 1: RtoL, Ref = R).
 *   kind 0: luma of the Ref image of `dir` at `level`, uint8, row pitch *pitch bytes;
 *   kind 1: raw search result, int16 pairs (x, y), row pitch *pitch pairs;
 *   kind 2: final flow of the level (after propagation and median), same layout.
 * With flow_method 1, kinds 1 and 2 of a level >= 1 hold the x and y
 * components of the level's flow as float64 (*pitch entries per row).
 * *H and *W receive the level size. */
abf_status abf_workspace_view(const abf_plan *plan, int32_t kind, int32_t strip, int32_t level,
                              int32_t dir, void **dev_ptr, int32_t *H, int32_t *W, int32_t *pitch);

/* ------------------------------------------------------------------ */
/* Flow refinement by gradient descent (an extension; not in the paper).
 * Energy of a flow u (float32 H x W x 2) between float32 RGB images Ref
 * and Tgt (H x W x 3, contiguous):
 *   E = sum_p sum_c rho(Tgt~_c(p + u(p)) - Ref_c(p))
 *     + lambda * sum_p sum_m sqrt((dx u_m)^2 + (dy u_m)^2 + eps^2),
 * rho(r) = sqrt(r^2 + eps^2), Tgt~ bilinear with clamped indices, forward
 * differences that are 0 at the last column / row. Sizes: 1 <= H, W and
 * 3 H W < 2^32 for this and every float-image call below (ABF_E_SHAPE
 * otherwise).
 * abf_energy writes E (one float, device) and, where non-null, dE/du,
 * dE/dRef, dE/dTgt (device, same shapes as u, Ref, Tgt; overwritten). The
 * derivative at an integer sample position is the right-hand one.
 * dE/dTgt is a bilinear scatter: with deterministic != 0 it is summed with
 * 64-bit fixed-point integer atomics, so the result does not depend on the
 * order of the additions; otherwise with float atomics. The fixed-point
 * scale is a power of two, 2^(62 - e) with 3 H W < 2^e (|rho'| <= 1 bounds
 * every pixel's sum by 3 H W), so no sum can overflow. eps^2 must be a normal float (eps >=
 * 1.1e-19; ABF_E_INVALID otherwise). Scratch: 8 bytes per energy block
 * and, if deterministic, 24 bytes per pixel of the bound workspace
 * (ABF_E_WORKSPACE if short). */
abf_status abf_energy(abf_plan *plan, const float *Ref, const float *Tgt, const float *u, int32_t H,
                      int32_t W, float lambda, float eps, float *E_dev, float *g_u, float *g_Ref,
                      float *g_Tgt, int32_t deterministic, void *hip_stream);

/* steps times u <- u - clip(eta * dE/du, -clip_px, clip_px) in place. u
 * must be 8-byte aligned (each pixel's (x, y) is one 64-bit access) and
 * eps^2 a normal float; ABF_E_INVALID otherwise. */
abf_status abf_refine_flow(abf_plan *plan, const float *Ref, const float *Tgt, float *u, int32_t H,
                           int32_t W, int32_t steps, float eta, float lambda, float eps, float clip_px,
                           void *hip_stream);

/* Multi-level energy (an extension): E_ms = the sum over pyramid levels
 * k = 0 .. levels - 1 of the energy of abf_energy at level k, where Ref_k
 * and Tgt_k are the images reduced k times by the float pyramid (the 5 x 5
 * binomial filter of the luma pyramid, weights w_i w_j / 256 with w = 1 4 6
 * 4 1, clamped indices, no rounding, decimated to ceil(H / 2) x
 * ceil(W / 2)) and u_k the flow reduced likewise and halved at each level
 * (displacements in level-k pixels). Writes E_ms (one float, device) and,
 * where non-null, its gradients with respect to the level-0 u, Ref, Tgt,
 * carried from the coarse levels through the pyramid's adjoint (the
 * transpose of filter and decimation). The pyramid levels are built in
 * the workspace during the call and not kept: a later gradient call
 * recomputes them from the level-0 inputs. deterministic as in abf_energy
 * (the adjoint passes are gathers, order-independent). levels = 1 gives
 * abf_energy's results. Scratch: about 11 bytes per level-0 pixel
 * (22 with gradients), plus abf_energy's. levels 1..12, else
 * ABF_E_INVALID. */
abf_status abf_energy_ms(abf_plan *plan, const float *Ref, const float *Tgt, const float *u, int32_t H,
                         int32_t W, int32_t levels, float lambda, float eps, float *E_dev, float *g_u,
                         float *g_Ref, float *g_Tgt, int32_t deterministic, void *hip_stream);

/* Workspace bytes for abf_energy_ms and abf_refine_flow_ms on an H x W
 * image with `levels` levels (at least abf_workspace_bytes); 0 for bad
 * arguments. */
size_t abf_energy_ms_workspace_bytes(const abf_plan *plan, int32_t H, int32_t W, int32_t levels);

/* steps times u <- u - clip(eta * dE_ms/du, -clip_px, clip_px) in place
 * (abf_refine_flow on the multi-level energy). */
abf_status abf_refine_flow_ms(abf_plan *plan, const float *Ref, const float *Tgt, float *u, int32_t H,
                              int32_t W, int32_t levels, int32_t steps, float eta, float lambda, float eps,
                              float clip_px, void *hip_stream);

/* One strip of a batched refinement (device pointers): float32 RGB Ref and
 * Tgt (H x W x 3) and the flow u (H x W x 2), refined in place. */
typedef struct abf_refine_strip {
    const float *Ref;
    const float *Tgt;
    float *u;
    int32_t H, W;
} abf_refine_strip;

/* abf_refine_flow over n strips at once (host array of descriptors): one
 * launch per descent step covers every strip. Results equal per-strip
 * abf_refine_flow calls bit for bit (same argument rules). Scratch: 8
 * bytes per pixel of the workspace. */
abf_status abf_refine_strips(abf_plan *plan, const abf_refine_strip *strips, int32_t n, int32_t steps,
                             float eta, float lambda, float eps, float clip_px, void *hip_stream);

/* Adjoint of Code 1 over float32 RGB images L, R (H x W x 3, contiguous;
 * any value scale): given g_F (float32 H x W x 3), writes the gradients
 * with respect to flow_LtoR, flow_RtoL (H x W x 2, 8-byte aligned) and
 * L, R (H x W x 3), each nullable and overwritten. d|f|/df = f/|f| for
 * f != 0 and 0 at 0; a non-finite flow component is used as 0 and
 * receives gradient 0. The image gradients are bilinear scatters, summed
 * with float atomics, or, with deterministic != 0, with order-independent
 * 64-bit fixed-point atomics whose power-of-two scale, 2^(62 - e) with
 * max |g_F| * 3 H W < 2^e (a bound on every sum; max |g_F| is taken on the
 * device), cannot overflow at any value scale; g_F must then be finite.
 * Scratch (deterministic only): 48 bytes per pixel of the workspace. */
abf_status abf_blend_backward(abf_plan *plan, const float *L, const float *R, const float *flow_LtoR,
                              const float *flow_RtoL, const float *blend, int32_t axis, int32_t H,
                              int32_t W, const float *g_F, float *g_flow_LtoR, float *g_flow_RtoL,
                              float *g_L, float *g_R, int32_t deterministic, void *hip_stream);

/* Code 1 forward over float32 RGB images (the differentiable variant of
 * abf_blend_asymmetric): F (float32 H x W x 3). */
abf_status abf_blend_asymmetric_f32(abf_plan *plan, const float *L, const float *R,
                                    const float *flow_LtoR, const float *flow_RtoL, const float *blend,
                                    int32_t axis, int32_t H, int32_t W, float *F, void *hip_stream);

/* ------------------------------------------------------------------ */
/* Canvas compositing: eq. (1) (Section III.C.2) and Code 1 (Section
 * III.C.3) on a canvas H x W (1..32767 on each side) where the areas have
 * any shape. The areas come from two coverage masks (uint8 H x W, rows
 * pitch_mask bytes apart, nonzero = the image covers the pixel): Area1 =
 * covered by L only, Area2 = by R only, Area3 = by both. OverlappedL /
 * OverlappedR are the crops of L and R to the bounding box of Area3 (the
 * "overlap box" {x, y, w, h}); the flows of the pair are computed on those
 * crops (abf_flow_bidirectional with the crop's first pixel and the
 * canvas pitches). Scratch comes from the plan's workspace:
 * abf_canvas_workspace_bytes gives the size a plan needs bound to handle an
 * H x W canvas (ABF_E_WORKSPACE otherwise). */

/* Workspace bytes for canvases up to H x W (at least abf_workspace_bytes). */
size_t abf_canvas_workspace_bytes(const abf_plan *plan, int32_t H, int32_t W);

/* Bounding box of Area3, written as int32 {x, y, w, h} to `box` (device,
 * 4 entries); {0, 0, 0, 0} when no pixel is covered by both images.
 * periodic != 0: the canvas wraps in x (a 360-degree panorama, column
 * W - 1 next to column 0), and the box's columns are the shortest circular
 * run holding every Area3 column: it starts right after the longest run of
 * columns without an Area3 pixel (of several, the one that starts at the
 * smallest column) and has w = W minus that run's length, so x + w may
 * exceed W (columns x .. x + w - 1 modulo W); every column holding Area3
 * gives x = 0, w = W. Scratch: 8 bytes per canvas row (+ W / 8 bytes if
 * periodic). */
abf_status abf_overlap_box(abf_plan *plan, const uint8_t *mask_L, const uint8_t *mask_R, int32_t H, int32_t W,
                           int32_t pitch_mask, int32_t periodic, int32_t *box, void *hip_stream);

/* eq. (1) over the canvas: Blend (float32, rows pitch_blend floats apart)
 * is 0 on Area1, 1 on Area2, 0.5 outside both images, and on Area3
 * Lmin / (Lmin + Rmin), with Lmin / Rmin the Euclidean distances between
 * pixel centres to the nearest Area1 / Area2 pixel (exact: integer squared
 * distances, then the ratio in double, rounded to float; on a periodic
 * canvas the column offset is taken the shorter way round, min(|dx|,
 * W - |dx|)). An empty Area1 gives 1 on Area3, an empty Area2 gives 0,
 * both empty give 0.5.
 * If dist2_1 / dist2_2 are non-null (both or neither; int32, rows
 * pitch_dist apart), they receive the squared distances of every canvas
 * pixel to Area1 / Area2 (0 inside the area, -1 if the area is empty).
 * blend may be null when the distances are requested. */
abf_status abf_canvas_blend(abf_plan *plan, const uint8_t *mask_L, const uint8_t *mask_R, int32_t H, int32_t W,
                            int32_t pitch_mask, int32_t periodic, float *blend, int32_t pitch_blend,
                            int32_t *dist2_1, int32_t *dist2_2, int32_t pitch_dist, void *hip_stream);

/* Code 1 over the canvas: F (uint8 RGB, rows pitch_F bytes apart) = L on
 * Area1, R on Area2, 0 outside both images; an Area3 pixel inside the box
 * is warped and blended exactly as pixel (x - box x, y - box y) of the
 * strip OverlappedL / OverlappedR by abf_blend_asymmetric (flows box h x
 * box w x 2, samples clamped to the box, flow magnitude divided by the box
 * width for axis 0, height for axis 1) with Blend read from `blend`
 * (float32 canvas array, rows pitch_blend floats apart) or, if null,
 * computed by eq. (1) as in abf_canvas_blend. An Area3 pixel outside the
 * box has no flow and is written as 0. `box` is a host array {x, y, w, h}
 * inside the canvas (w or h 0: no Area3 pixel is blended); with periodic
 * != 0 its columns may wrap past W - 1 (x < W, w <= W: the strip's column
 * c is canvas column x + c modulo W) and eq. (1) is periodic. F_f32
 * (nullable, H x W x 3 contiguous) receives the unrounded composite. */
abf_status abf_composite_canvas(abf_plan *plan, const uint8_t *L, const uint8_t *R, const uint8_t *mask_L,
                                const uint8_t *mask_R, int32_t H, int32_t W, int32_t pitch_L, int32_t pitch_R,
                                int32_t pitch_mask, int32_t periodic, const float *flow_LtoR, const float *flow_RtoL,
                                const int32_t *box, int32_t axis, const float *blend, int32_t pitch_blend,
                                uint8_t *F, int32_t pitch_F, float *F_f32, void *hip_stream);

/* ------------------------------------------------------------------ */
/* Repeated pairwise merging (Sections I and III.A: the two-photo blend is
 * applied photo after photo until the set is merged; Fig. 1: a ring of
 * photos around a vertical axis and a top photo). Every photo is given
 * on the common canvas H x W: image (RGB uint8, `pitch` bytes per row) and
 * coverage mask (uint8, nonzero = covered, pitch_mask bytes per row, the
 * same pitch for every mask and for `coverage`). Photo 0 starts the merged
 * canvas; photo i (i >= 1) is blended into the canvas merged so far with
 * the canvas path: overlap box, abf_flow_bidirectional on the box crops,
 * eq. (1), Code 1. side 0: the merged canvas plays L (Area1, left for
 * axis 0 / above for axis 1) and the photo R; side 1: the photo plays L.
 * A ring of photos merged left to right takes axis 0, side 0; a top photo
 * merged last takes axis 1, side 1 (Area1 = the top photo, above).
 * Outputs: `canvas` (merged RGB), `coverage` (1 where any photo reached);
 * `spare` (a second canvas-sized buffer) holds intermediate results. If
 * `boxes` (host, 4 n int32) is non-null it receives each step's overlap box
 * (zeros for photo 0). Each box must fit the plan's strip limits
 * (ABF_E_SHAPE otherwise). Synchronises the stream once per photo (the box
 * sizes the flow computation); not for graph capture. */
typedef struct abf_photo {
    const uint8_t *image;
    const uint8_t *mask;
    int32_t pitch;
    int32_t axis;
    int32_t side;
} abf_photo;

/* Workspace bytes for merges on an H x W canvas (flows of the largest box
 * the plan admits kept beside the canvas passes' scratch, and two box
 * copies). */
size_t abf_merge_workspace_bytes(const abf_plan *plan, int32_t H, int32_t W);

/* periodic != 0: the canvas is a 360-degree panorama that wraps in x; the
 * boxes, eq. (1) and Code 1 of every step are periodic (as in
 * abf_overlap_box, abf_canvas_blend and abf_composite_canvas), so the last
 * ring photo, whose coverage reaches across column W - 1 to the first
 * photo, closes the ring in its step (its box then wraps, and its flows are
 * computed on contiguous copies of the box crops). */
abf_status abf_merge_photos(abf_plan *plan, const abf_photo *photos, int32_t n, int32_t H, int32_t W,
                            int32_t pitch_mask, int32_t periodic, uint8_t *canvas, int32_t pitch_canvas,
                            uint8_t *spare, int32_t pitch_spare, uint8_t *coverage, int32_t *boxes,
                            void *hip_stream);

/* ------------------------------------------------------------------ */
/* Autotuning of launch shapes (never of results): times the candidate
 * tile heights and persistent grid sizes of each stage on the batch
 * `strips` and keeps the fastest per (stage, level-size class). Each
 * candidate is timed by event pairs around the launches of that stage and
 * class alone (best of three eager passes after a warm-up pass); classes
 * with no launch in the batch keep their shapes. Writes the choice to the
 * JSON file named by the ABF_TUNE_CACHE environment variable if set. Runs
 * synchronously. */
abf_status abf_tune(abf_plan *plan, const abf_strip *strips, int32_t n, void *hip_stream);

/* Current launch choice, for tests: stage 0..5 (luma, pyramid, search,
 * propagation, refine, blend), level-size class 0..3; *tile_h and *grid
 * receive the tile height and persistent workgroups per CU (0 = one
 * workgroup per tile). abf_set_launch overrides it; valid tile heights:
 * search 1, 2, 4, 8; propagation 8, 10, 12, 16, 32; refine 2, 4; blend 1, 2, 4 (pixels per
 * thread); other stages 4
 * (ABF_E_INVALID otherwise). */
abf_status abf_get_launch(const abf_plan *plan, int32_t stage, int32_t size_class, int32_t *tile_h,
                          int32_t *grid);
abf_status abf_set_launch(abf_plan *plan, int32_t stage, int32_t size_class, int32_t tile_h, int32_t grid);

/* Timing of the batched launch sequence (for benchmarks and profiles):
 * runs abf_stitch_strips' launches `reps` times without a graph, with a
 * hipEvent pair around every launch on `hip_stream`, and writes the mean
 * milliseconds per launch to ms_out[stage * 12 + level] (stage numbering
 * of abf_get_launch; 6 * 12 floats, host memory); the refinement (level 0
 * only) reports its interior launch in the level-0 slot and its border-pixel
 * launch in the level-1 slot. With flow_method 1 the refinement slots hold
 * each level's interior launch (which uses the refinement's launch shapes)
 * and the search slots each level's border-pixel launch. Synchronous. */
abf_status abf_profile(abf_plan *plan, const abf_strip *strips, int32_t n, int32_t reps, float *ms_out,
                       void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ABF_H */
