// HIP kernels of libabf for gfx950 (MI355X): coarse-to-fine bidirectional
// flow (Section III.C.1 of Meng & Liu, arXiv 2006.01201) and the
// asymmetric warp + softmax blend (Code 1 with eq. (1)).
//
// Work decomposition: every kernel walks a flat list of tiles that covers
// all strips of a batch (per-strip prefix sums give the strip of a tile),
// either one workgroup per tile or a persistent grid that strides over
// the list. Workgroup indices are remapped so that the workgroups that
// land on one XCD (dispatch is round-robin over the 8 XCDs) take
// neighbouring tiles and share that XCD's L2.
//
// The integer stages are bit-exact by construction (integer arithmetic,
// fixed candidate order, Jacobi updates into separate buffers). The
// patch costs use v_sad_u8 on byte-packed dwords read from LDS tables in
// which entry (y, x) holds bytes x..x+3 of row y ("H") or rows y..y+3 of
// column x ("V"), so any 4-byte run of a row or column is one aligned
// 32-bit LDS read.
#include "abf_internal.h"

namespace abf {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int find_strip(const int32_t *__restrict__ prefix, int n, int t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Workgroups are dispatched round-robin over 8 XCDs; give the workgroups
// of one XCD a contiguous range of logical indices.
__device__ __forceinline__ int xcd_block(int b, int G)
{
    constexpr int X = 8;
    int per = G / X, rem = G % X;
    int x = b % X, i = b / X;
    return x * per + min(x, rem) + i;
}

__device__ __forceinline__ uint32_t pack16(int x, int y)
{
    return (uint32_t)(uint16_t)(int16_t)x | ((uint32_t)(uint16_t)(int16_t)y << 16);
}
__device__ __forceinline__ int unpack_x(uint32_t v) { return (int)(int16_t)(v & 0xffffu); }
__device__ __forceinline__ int unpack_y(uint32_t v) { return (int)(int16_t)(v >> 16); }

template <int NT>
__device__ __forceinline__ void wg_minmax4(int &a0, int &a1, int &a2, int &a3, int *red)
{
    // a0, a1 reduced with min; a2, a3 with max
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        a0 = min(a0, __shfl_xor(a0, m, 64));
        a1 = min(a1, __shfl_xor(a1, m, 64));
        a2 = max(a2, __shfl_xor(a2, m, 64));
        a3 = max(a3, __shfl_xor(a3, m, 64));
    }
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[4 * w + 0] = a0;
        red[4 * w + 1] = a1;
        red[4 * w + 2] = a2;
        red[4 * w + 3] = a3;
    }
    __syncthreads();
    a0 = red[0];
    a1 = red[1];
    a2 = red[2];
    a3 = red[3];
#pragma unroll
    for (int k = 1; k < NW; k++) {
        a0 = min(a0, red[4 * k + 0]);
        a1 = min(a1, red[4 * k + 1]);
        a2 = max(a2, red[4 * k + 2]);
        a3 = max(a3, red[4 * k + 3]);
    }
    __syncthreads();
}

// Stage the box [bx0, bx0 + bw) x [by0, by0 + bh) of a uint8 image
// (coordinates clamped to the image) as H and V tables of row stride
// STRIDE entries. `raw` holds (bh + 3) rows of RAWQ dwords. Ends with a
// barrier.
template <int STRIDE, int RAWQ, int NT>
__device__ void stage_tables(const uint8_t *__restrict__ img, int H, int W, int pitch, int bx0, int by0,
                             int bw, int bh, uint32_t *raw, uint32_t *tabH, uint32_t *tabV, bool needV)
{
    const int ax0 = bx0 & ~3;  // floor to a multiple of 4 (two's complement)
    const int sh = bx0 - ax0;
    const int nq = ((sh + bw + 2) >> 2) + 2;
    const int rows = bh + 3;
    for (int e = threadIdx.x; e < rows * nq; e += NT) {
        int r = e / nq, q = e - r * nq;
        int gy = clampi(by0 + r, 0, H - 1);
        int gx = ax0 + 4 * q;
        const uint8_t *row = img + (size_t)gy * pitch;
        uint32_t v;
        if (gx >= 0 && gx + 3 <= W - 1) {
            v = *reinterpret_cast<const uint32_t *>(row + gx);
        } else {
            v = (uint32_t)row[clampi(gx, 0, W - 1)] | ((uint32_t)row[clampi(gx + 1, 0, W - 1)] << 8) |
                ((uint32_t)row[clampi(gx + 2, 0, W - 1)] << 16) | ((uint32_t)row[clampi(gx + 3, 0, W - 1)] << 24);
        }
        raw[r * RAWQ + q] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < bh * bw; e += NT) {
        int r = e / bw, c = e - r * bw;
        int xo = c + sh, q = xo >> 2, b = xo & 3;
        uint32_t lo = raw[r * RAWQ + q], hi = raw[r * RAWQ + q + 1];
        tabH[r * STRIDE + c] = __builtin_amdgcn_alignbyte(hi, lo, b);
        if (needV) {
            int s = 8 * b;
            uint32_t b0 = (raw[r * RAWQ + q] >> s) & 0xffu;
            uint32_t b1 = (raw[(r + 1) * RAWQ + q] >> s) & 0xffu;
            uint32_t b2 = (raw[(r + 2) * RAWQ + q] >> s) & 0xffu;
            uint32_t b3 = (raw[(r + 3) * RAWQ + q] >> s) & 0xffu;
            tabV[r * STRIDE + c] = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
        }
    }
    __syncthreads();
}

// Patch cost from tables. Ref values of the pixel are preloaded: rr[r] =
// row r bytes 0..3 (P = 2) or 0..2 (P = 1, byte 3 zero), rv = column 4
// rows 0..3, rs = byte (4, 4). `th`, `tv` point at the window's top-left
// entry in the Tgt tables.
template <int P, int STRIDE>
__device__ __forceinline__ uint32_t sad_tab(const uint32_t (&rr)[2 * P + 1], uint32_t rv, uint32_t rs,
                                            const uint32_t *th, const uint32_t *tv)
{
    uint32_t s = 0;
    if constexpr (P == 2) {
#pragma unroll
        for (int r = 0; r < 5; r++) s = __builtin_amdgcn_sad_u8(rr[r], th[r * STRIDE], s);
        s = __builtin_amdgcn_sad_u8(rv, tv[4], s);
        s = __builtin_amdgcn_sad_u8(rs, tv[STRIDE + 4] >> 24, s);
    } else {
#pragma unroll
        for (int r = 0; r < 3; r++) s = __builtin_amdgcn_sad_u8(rr[r], th[r * STRIDE] & 0x00ffffffu, s);
    }
    return s;
}

template <int P, int STRIDE>
__device__ __forceinline__ void load_ref(const uint32_t *rh, const uint32_t *rvt, uint32_t (&rr)[2 * P + 1],
                                         uint32_t &rv, uint32_t &rs)
{
#pragma unroll
    for (int r = 0; r < 2 * P + 1; r++) rr[r] = rh[r * STRIDE];
    if constexpr (P == 2) {
        rv = rvt[4];
        rs = rvt[STRIDE + 4] >> 24;
    } else {
#pragma unroll
        for (int r = 0; r < 3; r++) rr[r] &= 0x00ffffffu;
        rv = rs = 0;
    }
}

// Patch cost straight from global memory (fallback when a tile's target
// footprint does not fit the LDS tables).
template <int P>
__device__ uint32_t sad_global(const uint8_t *__restrict__ ref, const uint8_t *__restrict__ tgt, int H, int W,
                               int pitch, int x, int y, int dx, int dy)
{
    uint32_t s = 0;
    for (int j = -P; j <= P; j++) {
        const uint8_t *rrow = ref + (size_t)clampi(y + j, 0, H - 1) * pitch;
        const uint8_t *trow = tgt + (size_t)clampi(y + j + dy, 0, H - 1) * pitch;
        for (int i = -P; i <= P; i++) {
            int a = rrow[clampi(x + i, 0, W - 1)], b = trow[clampi(x + i + dx, 0, W - 1)];
            s += (uint32_t)abs(a - b);
        }
    }
    return s;
}

#define TILE_LOOP(total, grid_is_persistent)                                           \
    for (int t = xcd_block(blockIdx.x, gridDim.x); t < (total); t += gridDim.x)

// ------------------------------------------------------------------ luma
// Y = (77 R + 150 G + 29 B + 128) >> 8 for both images of every strip.
__global__ __launch_bounds__(256) void k_luma(const StripIO *__restrict__ io, const StripLv *__restrict__ lv,
                                              const int32_t *__restrict__ prefix, int n, int total)
{
    TILE_LOOP(total, 0)
    {
        const int s = find_strip(prefix, n, t);
        const int local = t - prefix[s];
        const int W = lv[s].W;
        const int segs = ceil_div(W, kRowTW);
        const int y = local / segs;
        const int x = (local - y * segs) * kRowTW + threadIdx.x;
        if (x < W) {
            const uint8_t *pl = io[s].L + (size_t)y * io[s].pitchL + 3 * x;
            const uint8_t *pr = io[s].R + (size_t)y * io[s].pitchR + 3 * x;
            const int yp = lv[s].ypitch;
            lv[s].y[0][(size_t)y * yp + x] = (uint8_t)((77 * pl[0] + 150 * pl[1] + 29 * pl[2] + 128) >> 8);
            lv[s].y[1][(size_t)y * yp + x] = (uint8_t)((77 * pr[0] + 150 * pr[1] + 29 * pr[2] + 128) >> 8);
        }
    }
}

// --------------------------------------------------------------- pyramid
// One reduction, both images: 5x5 binomial (1 4 6 4 1)^2 / 256 sampled at
// even positions, clamped borders, rounding (s + 128) >> 8.
__global__ __launch_bounds__(256) void k_pyr(const StripLv *__restrict__ lv, const int32_t *__restrict__ prefix,
                                             int n, int total)
{
    constexpr int w5[5] = {1, 4, 6, 4, 1};
    TILE_LOOP(total, 0)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int per_img = tiles_pyr(L.H, L.W);
        const int img = local / per_img;
        local -= img * per_img;
        const int tx = ceil_div(L.W, kPyrTW);
        const int ty = local / tx;
        const int x = (local - ty * tx) * kPyrTW + (threadIdx.x & (kPyrTW - 1));
        const int y = ty * kPyrTH + (threadIdx.x / kPyrTW);
        if (x < L.W && y < L.H) {
            const uint8_t *src = L.yfine[img];
            const int Hf = L.Hf, Wf = L.Wf, pf = L.ypitch_f;
            int cx[5];
#pragma unroll
            for (int i = 0; i < 5; i++) cx[i] = clampi(2 * x + i - 2, 0, Wf - 1);
            int acc = 0;
#pragma unroll
            for (int j = 0; j < 5; j++) {
                const uint8_t *row = src + (size_t)clampi(2 * y + j - 2, 0, Hf - 1) * pf;
                int h = 0;
#pragma unroll
                for (int i = 0; i < 5; i++) h += w5[i] * row[cx[i]];
                acc += w5[j] * h;
            }
            L.y[img][(size_t)y * L.ypitch + x] = (uint8_t)((acc + 128) >> 8);
        }
    }
}

// ---------------------------------------------------------------- search
// Integer patch-cost search around the upsampled coarser flow, both
// directions. Tile: 64 x TH pixels, one pixel per thread. Key of a
// candidate: (cost << 11) | (L1 offset << 7) | enumeration index, so one
// unsigned min gives the lexicographic winner.
constexpr int kTgtBW = 128;  // Tgt table row stride (entries)

template <int P, int R, int TH>
__global__ __launch_bounds__(64 * TH) void k_search(const StripLv *__restrict__ lv,
                                                    const int32_t *__restrict__ prefix, int n, int total)
{
    constexpr int NT = 64 * TH;
    constexpr int TW = kSearchTW;
    constexpr int S = R + P;
    constexpr int RBW = TW + 2 * P, RBH = TH + 2 * P;
    constexpr int TBH = TH + 16;  // Tgt table rows: 2S + vertical centre spread must fit
    constexpr int RAWQ = (kTgtBW + 8) / 4 + 2;
    constexpr int NC = 2 * R + 1;
    __shared__ uint32_t raw[(TBH + 3) * RAWQ];
    __shared__ uint32_t refH[RBH * RBW], refV[RBH * RBW];
    __shared__ uint32_t tgtH[TBH * kTgtBW], tgtV[TBH * kTgtBW];
    __shared__ int red[4 * (NT / 64)];

    const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
    TILE_LOOP(total, 0)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const int ntx = ceil_div(W, TW), per_dir = ntx * ceil_div(H, TH);
        const int dir = local / per_dir;
        local -= dir * per_dir;
        const int tyi = local / ntx;
        const int x0 = (local - tyi * ntx) * TW, y0 = tyi * TH;
        const int x = x0 + lane, y = y0 + wrow;
        const uint8_t *ref = L.y[dir], *tgt = L.y[1 - dir];

        int cx = 0, cy = 0;
        if (L.dc[dir]) {
            const uint32_t v = L.dc[dir][(size_t)min(min(y, H - 1) >> 1, L.Hc - 1) * L.fpitch_c +
                                         min(min(x, W - 1) >> 1, L.Wc - 1)];
            cx = 2 * unpack_x(v);
            cy = 2 * unpack_y(v);
        }
        int cxmin = cx, cymin = cy, cxmax = cx, cymax = cy;
        wg_minmax4<NT>(cxmin, cymin, cxmax, cymax, red);
        const int tbw = TW + 2 * S + (cxmax - cxmin), tbh = TH + 2 * S + (cymax - cymin);
        const bool fast = tbw <= kTgtBW && tbh <= TBH;

        uint32_t best = 0xffffffffu;
        if (fast) {
            stage_tables<RBW, RAWQ, NT>(ref, H, W, yp, x0 - P, y0 - P, RBW, RBH, raw, refH, refV, P == 2);
            uint32_t rr[2 * P + 1], rv, rs;
            load_ref<P, RBW>(refH + wrow * RBW + lane, refV + wrow * RBW + lane, rr, rv, rs);
            stage_tables<kTgtBW, RAWQ, NT>(tgt, H, W, yp, x0 + cxmin - S, y0 + cymin - S, tbw, tbh, raw, tgtH,
                                           tgtV, P == 2);
            const int off = (wrow + cy - cymin) * kTgtBW + lane + (cx - cxmin);
            const uint32_t *th = tgtH + off, *tv = tgtV + off;
#pragma unroll
            for (int j = 0; j < NC; j++)
#pragma unroll
                for (int i = 0; i < NC; i++) {
                    const uint32_t c = sad_tab<P, kTgtBW>(rr, rv, rs, th + j * kTgtBW + i, tv + j * kTgtBW + i);
                    const uint32_t K = ((uint32_t)(abs(i - R) + abs(j - R)) << 7) | (uint32_t)(j * NC + i);
                    best = min(best, (c << 11) + K);
                }
        } else {
            for (int j = 0; j < NC; j++)
                for (int i = 0; i < NC; i++) {
                    const uint32_t c = sad_global<P>(ref, tgt, H, W, yp, x, y, cx + i - R, cy + j - R);
                    const uint32_t K = ((uint32_t)(abs(i - R) + abs(j - R)) << 7) | (uint32_t)(j * NC + i);
                    best = min(best, (c << 11) + K);
                }
        }
        if (x < W && y < H) {
            const int idx = (int)(best & 127u);
            const int j = idx / NC, i = idx - j * NC;
            L.ds[dir][(size_t)y * L.fpitch + x] = pack16(cx + i - R, cy + j - R);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------- propagation
// T Jacobi steps (candidates self, left, right, up, down of the previous
// iterate; lower cost wins, earlier candidate on ties; neighbours outside
// the image skipped) and a (2M+1)^2 component-wise median with clamped
// indices, fused per 32 x TH tile by recomputing a halo of T + M pixels.
constexpr int kHaloMax = 5;
constexpr int kPropTgtBW = 96;

__device__ __forceinline__ int med3i(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

template <int P, int TH>
__global__ __launch_bounds__(256) void k_prop(const StripLv *__restrict__ lv, const int32_t *__restrict__ prefix,
                                              int n, int total, int T, int M)
{
    constexpr int NT = 256;
    constexpr int TW = kPropTW;
    constexpr int DW = TW + 2 * kHaloMax, DH = TH + 2 * kHaloMax;
    constexpr int RBW = TW + 2 * (kHaloMax - 1) + 2 * P;  // ref tables cover step-1 region + P
    constexpr int RBH = TH + 2 * (kHaloMax - 1) + 2 * P;
    constexpr int TBH = RBH + 8;
    constexpr int RAWQ = (kPropTgtBW + 8) / 4 + 2;
    __shared__ uint32_t dbuf[2][DH * DW];
    __shared__ uint32_t raw[(TBH + 3) * RAWQ];
    __shared__ uint32_t refH[RBH * RBW], refV[RBH * RBW];
    __shared__ uint32_t tgtH[TBH * kPropTgtBW], tgtV[TBH * kPropTgtBW];
    __shared__ int red[16];

    const int h = T + M;
    TILE_LOOP(total, 0)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const int ntx = ceil_div(W, TW), per_dir = ntx * ceil_div(H, TH);
        const int dir = local / per_dir;
        local -= dir * per_dir;
        const int tyi = local / ntx;
        const int x0 = (local - tyi * ntx) * TW, y0 = tyi * TH;
        const uint8_t *ref = L.y[dir], *tgt = L.y[1 - dir];
        const uint32_t *dsrc = L.ds[dir];
        // frame of the D buffers: (x0 - kHaloMax, y0 - kHaloMax)
        const int fx0 = x0 - kHaloMax, fy0 = y0 - kHaloMax;

        int dxmin = 1 << 20, dymin = 1 << 20, dxmax = -(1 << 20), dymax = -(1 << 20);
        for (int e = threadIdx.x; e < DH * DW; e += NT) {
            const int ry = e / DW, rx = e - ry * DW;
            const int gx = fx0 + rx, gy = fy0 + ry;
            uint32_t v = 0;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H && gx >= x0 - h && gx < x0 + TW + h && gy >= y0 - h &&
                gy < y0 + TH + h) {
                v = dsrc[(size_t)gy * L.fpitch + gx];
                const int vx = unpack_x(v), vy = unpack_y(v);
                dxmin = min(dxmin, vx);
                dxmax = max(dxmax, vx);
                dymin = min(dymin, vy);
                dymax = max(dymax, vy);
            }
            dbuf[0][e] = v;
        }
        wg_minmax4<NT>(dxmin, dymin, dxmax, dymax, red);
        int cur = 0;
        if (T > 0) {
            // step-1 region: tile +- (h - 1); its patches and displaced patches
            const int g = h - 1;
            const int rbx0 = x0 - g - P, rby0 = y0 - g - P;
            const int tbx0 = rbx0 + dxmin, tby0 = rby0 + dymin;
            const int tbw = TW + 2 * g + 2 * P + (dxmax - dxmin), tbh = TH + 2 * g + 2 * P + (dymax - dymin);
            const bool fast = dxmin <= dxmax && tbw <= kPropTgtBW && tbh <= TBH;
            if (fast) {
                stage_tables<RBW, RAWQ, NT>(ref, H, W, yp, rbx0, rby0, TW + 2 * g + 2 * P, TH + 2 * g + 2 * P, raw,
                                            refH, refV, P == 2);
                stage_tables<kPropTgtBW, RAWQ, NT>(tgt, H, W, yp, tbx0, tby0, tbw, tbh, raw, tgtH, tgtV, P == 2);
            }
            for (int step = 1; step <= T; step++) {
                const int gg = h - step;  // region of this step: tile +- gg
                const int rw = TW + 2 * gg, rh = TH + 2 * gg;
                const uint32_t *prev = dbuf[cur];
                uint32_t *next = dbuf[cur ^ 1];
                for (int e = threadIdx.x; e < rw * rh; e += NT) {
                    const int ly = e / rw, lx = e - ly * rw;
                    const int px = x0 - gg + lx, py = y0 - gg + ly;
                    const int fi = (py - fy0) * DW + (px - fx0);
                    if (px < 0 || px >= W || py < 0 || py >= H) {
                        next[fi] = 0;
                        continue;
                    }
                    uint32_t cand[5];
                    bool ok[5];
                    cand[0] = prev[fi];
                    ok[0] = true;
                    cand[1] = prev[fi - 1];
                    ok[1] = px > 0;
                    cand[2] = prev[fi + 1];
                    ok[2] = px < W - 1;
                    cand[3] = prev[fi - DW];
                    ok[3] = py > 0;
                    cand[4] = prev[fi + DW];
                    ok[4] = py < H - 1;
                    uint32_t rr[2 * P + 1], rv = 0, rs = 0;
                    const int qx = px - rbx0 - P, qy = py - rby0 - P;  // window top-left in ref tables
                    if (fast) load_ref<P, RBW>(refH + qy * RBW + qx, refV + qy * RBW + qx, rr, rv, rs);
                    uint32_t bestc = 0xffffffffu, bestv = cand[0];
#pragma unroll
                    for (int k = 0; k < 5; k++) {
                        if (!ok[k]) continue;
                        bool dup = false;
#pragma unroll
                        for (int m = 0; m < k; m++) dup |= ok[m] && cand[m] == cand[k];
                        if (dup) continue;  // an earlier equal candidate already has this cost
                        const int dx = unpack_x(cand[k]), dy = unpack_y(cand[k]);
                        uint32_t c;
                        if (fast) {
                            const int o = (qy + dy - dymin) * kPropTgtBW + (qx + dx - dxmin);
                            c = sad_tab<P, kPropTgtBW>(rr, rv, rs, tgtH + o, tgtV + o);
                        } else {
                            c = sad_global<P>(ref, tgt, H, W, yp, px, py, dx, dy);
                        }
                        if (c < bestc) {
                            bestc = c;
                            bestv = cand[k];
                        }
                    }
                    next[fi] = bestv;
                }
                __syncthreads();
                cur ^= 1;
            }
        }
        // median (or copy) over the tile
        const uint32_t *fin = dbuf[cur];
        for (int e = threadIdx.x; e < TW * TH; e += NT) {
            const int ly = e / TW, lx = e - ly * TW;
            const int px = x0 + lx, py = y0 + ly;
            if (px >= W || py >= H) continue;
            uint32_t outv;
            if (M == 0) {
                outv = fin[(py - fy0) * DW + (px - fx0)];
            } else {
                int vx[9], vy[9];
#pragma unroll
                for (int j = 0; j < 3; j++)
#pragma unroll
                    for (int i = 0; i < 3; i++) {
                        const int qx = clampi(px + i - 1, 0, W - 1), qy = clampi(py + j - 1, 0, H - 1);
                        const uint32_t v = fin[(qy - fy0) * DW + (qx - fx0)];
                        vx[3 * j + i] = unpack_x(v);
                        vy[3 * j + i] = unpack_y(v);
                    }
                // median of 9 = med3(max of row minima, med3 of row medians, min of row maxima)
                int mx, my;
                {
                    int lo0 = min(min(vx[0], vx[1]), vx[2]), lo1 = min(min(vx[3], vx[4]), vx[5]),
                        lo2 = min(min(vx[6], vx[7]), vx[8]);
                    int hi0 = max(max(vx[0], vx[1]), vx[2]), hi1 = max(max(vx[3], vx[4]), vx[5]),
                        hi2 = max(max(vx[6], vx[7]), vx[8]);
                    int md0 = med3i(vx[0], vx[1], vx[2]), md1 = med3i(vx[3], vx[4], vx[5]),
                        md2 = med3i(vx[6], vx[7], vx[8]);
                    mx = med3i(max(max(lo0, lo1), lo2), med3i(md0, md1, md2), min(min(hi0, hi1), hi2));
                }
                {
                    int lo0 = min(min(vy[0], vy[1]), vy[2]), lo1 = min(min(vy[3], vy[4]), vy[5]),
                        lo2 = min(min(vy[6], vy[7]), vy[8]);
                    int hi0 = max(max(vy[0], vy[1]), vy[2]), hi1 = max(max(vy[3], vy[4]), vy[5]),
                        hi2 = max(max(vy[6], vy[7]), vy[8]);
                    int md0 = med3i(vy[0], vy[1], vy[2]), md1 = med3i(vy[3], vy[4], vy[5]),
                        md2 = med3i(vy[6], vy[7], vy[8]);
                    my = med3i(max(max(lo0, lo1), lo2), med3i(md0, md1, md2), min(min(hi0, hi1), hi2));
                }
                outv = pack16(mx, my);
            }
            L.df[dir][(size_t)py * L.fpitch + px] = outv;
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- refine
// Level-0 Lucas-Kanade: central-difference gradient of Ref, normal matrix
// summed over the window (exact in integers: 4H), plus eps I; `iters`
// Gauss-Newton steps from the integer flow with bilinear Tgt samples; each
// component clamped to within 1 px of the integer flow. The displacement
// is split into floor + fraction so no FP32 coordinate is ever formed.
constexpr int kRefTgtBW = 192;

template <int LP, int TH>
__global__ __launch_bounds__(64 * TH) void k_refine(const StripLv *__restrict__ lv, const StripIO *__restrict__ io,
                                                    const int32_t *__restrict__ prefix, int n, int total, int iters,
                                                    float eps)
{
    constexpr int NT = 64 * TH;
    constexpr int TW = kRefineTW;
    constexpr int AW = TW + 2 * LP + 2, AH = TH + 2 * LP + 2;  // Ref box: tile +- (LP + 1)
    constexpr int GW = TW + 2 * LP, GH = TH + 2 * LP;          // gradient box: tile +- LP
    constexpr int BBH = TH + 2 * LP + 2 + 24;                  // Tgt box rows (vertical spread <= 24)
    constexpr int WN = 2 * LP + 1;
    __shared__ uint8_t abox[AH * AW];
    __shared__ uint32_t gbox[GH * GW];
    __shared__ uint8_t bbox[BBH * kRefTgtBW];
    __shared__ int red[4 * (NT / 64)];

    const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
    TILE_LOOP(total, 0)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const int ntx = ceil_div(W, TW), per_dir = ntx * ceil_div(H, TH);
        const int dir = local / per_dir;
        local -= dir * per_dir;
        const int tyi = local / ntx;
        const int x0 = (local - tyi * ntx) * TW, y0 = tyi * TH;
        const int x = x0 + lane, y = y0 + wrow;
        const uint8_t *A = L.y[dir], *B = L.y[1 - dir];

        // Ref box and gradients
        const int ax0 = x0 - LP - 1, ay0 = y0 - LP - 1;
        for (int e = threadIdx.x; e < AW * AH; e += NT) {
            const int r = e / AW, c = e - r * AW;
            abox[e] = A[(size_t)clampi(ay0 + r, 0, H - 1) * yp + clampi(ax0 + c, 0, W - 1)];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < GW * GH; e += NT) {
            const int r = e / GW, c = e - r * GW;
            // gradient at image position q = (x0 - LP + c, y0 - LP + r), clamped to the image
            const int qx = clampi(x0 - LP + c, 0, W - 1), qy = clampi(y0 - LP + r, 0, H - 1);
            const int bx = qx - ax0, by = qy - ay0;
            const int xm = clampi(qx - 1, 0, W - 1) - ax0, xp = clampi(qx + 1, 0, W - 1) - ax0;
            const int ym = clampi(qy - 1, 0, H - 1) - ay0, yq = clampi(qy + 1, 0, H - 1) - ay0;
            const int gx2 = (int)abox[by * AW + xp] - (int)abox[by * AW + xm];
            const int gy2 = (int)abox[yq * AW + bx] - (int)abox[ym * AW + bx];
            gbox[e] = pack16(gx2, gy2);
        }
        // integer flow and Tgt footprint
        const bool inside = x < W && y < H;
        const uint32_t d0 = L.df[dir][(size_t)min(y, H - 1) * L.fpitch + min(x, W - 1)];
        const int d0x = unpack_x(d0), d0y = unpack_y(d0);
        int dxmin = d0x, dymin = d0y, dxmax = d0x, dymax = d0y;
        wg_minmax4<NT>(dxmin, dymin, dxmax, dymax, red);
        const int bx0 = x0 - LP + dxmin - 1, by0 = y0 - LP + dymin - 1;
        const int bw = TW + 2 * LP + (dxmax - dxmin) + 3, bh = TH + 2 * LP + (dymax - dymin) + 3;
        const bool fast = bw <= kRefTgtBW && bh <= BBH;
        if (fast) {
            for (int e = threadIdx.x; e < bw * bh; e += NT) {
                const int r = e / bw, c = e - r * bw;
                bbox[r * kRefTgtBW + c] = B[(size_t)clampi(by0 + r, 0, H - 1) * yp + clampi(bx0 + c, 0, W - 1)];
            }
        }
        __syncthreads();

        // normal matrix (times 4, exact)
        int hxx = 0, hxy = 0, hyy = 0;
        for (int j = -LP; j <= LP; j++)
            for (int i = -LP; i <= LP; i++) {
                const int qx = clampi(x + i, 0, W - 1), qy = clampi(y + j, 0, H - 1);
                const uint32_t g = gbox[(qy - (y0 - LP)) * GW + (qx - (x0 - LP))];
                const int gx = unpack_x(g), gy = unpack_y(g);
                hxx += gx * gx;
                hxy += gx * gy;
                hyy += gy * gy;
            }
        const double Hxx = 0.25 * hxx + eps, Hxy = 0.25 * hxy, Hyy = 0.25 * hyy + eps;
        const double det = Hxx * Hyy - Hxy * Hxy;
        float ux = (float)d0x, uy = (float)d0y;
        const bool interior = x - LP >= 0 && x + LP <= W - 1 && y - LP >= 0 && y + LP <= H - 1;
        for (int it = 0; it < iters; it++) {
            const float fux = floorf(ux), fuy = floorf(uy);
            const float fx = ux - fux, fy = uy - fuy;
            const int iux = (int)fux, iuy = (int)fuy;
            float bxs = 0.f, bys = 0.f;
            if (fast && interior) {
                // window of Tgt samples on a (WN+1)^2 block with shared weights
                const int ox = x - LP + iux - bx0, oy = y - LP + iuy - by0;
                float hrow[WN + 1][WN];
#pragma unroll
                for (int r = 0; r <= WN; r++) {
                    const uint8_t *br = bbox + (oy + r) * kRefTgtBW + ox;
                    float prev = (float)br[0];
#pragma unroll
                    for (int c = 0; c < WN; c++) {
                        const float nx = (float)br[c + 1];
                        hrow[r][c] = prev + fx * (nx - prev);
                        prev = nx;
                    }
                }
#pragma unroll
                for (int j = 0; j < WN; j++)
#pragma unroll
                    for (int i = 0; i < WN; i++) {
                        const float bs = hrow[j][i] + fy * (hrow[j + 1][i] - hrow[j][i]);
                        const int qx = x - LP + i, qy = y - LP + j;
                        const float e = bs - (float)abox[(qy - ay0) * AW + (qx - ax0)];
                        const uint32_t g = gbox[(qy - (y0 - LP)) * GW + (qx - (x0 - LP))];
                        bxs = fmaf(0.5f * (float)unpack_x(g), e, bxs);
                        bys = fmaf(0.5f * (float)unpack_y(g), e, bys);
                    }
            } else {
                for (int j = -LP; j <= LP; j++)
                    for (int i = -LP; i <= LP; i++) {
                        const int qx = clampi(x + i, 0, W - 1), qy = clampi(y + j, 0, H - 1);
                        const int sx = qx + iux, sy = qy + iuy;
                        float v00, v01, v10, v11;
                        if (fast) {
                            // the box holds B at clamped coordinates, indexed by the
                            // unclamped position (which always lies inside the box;
                            // the clamped one need not when the box starts beyond
                            // an image edge)
                            const int cxa = sx - bx0, cxb = cxa + 1;
                            const int cya = sy - by0, cyb = cya + 1;
                            v00 = bbox[cya * kRefTgtBW + cxa];
                            v01 = bbox[cya * kRefTgtBW + cxb];
                            v10 = bbox[cyb * kRefTgtBW + cxa];
                            v11 = bbox[cyb * kRefTgtBW + cxb];
                        } else {
                            const uint8_t *ra = B + (size_t)clampi(sy, 0, H - 1) * yp;
                            const uint8_t *rb = B + (size_t)clampi(sy + 1, 0, H - 1) * yp;
                            const int cxa = clampi(sx, 0, W - 1), cxb = clampi(sx + 1, 0, W - 1);
                            v00 = ra[cxa];
                            v01 = ra[cxb];
                            v10 = rb[cxa];
                            v11 = rb[cxb];
                        }
                        const float top = v00 + fx * (v01 - v00), bot = v10 + fx * (v11 - v10);
                        const float bs = top + fy * (bot - top);
                        const float e = bs - (float)abox[(qy - ay0) * AW + (qx - ax0)];
                        const uint32_t g = gbox[(qy - (y0 - LP)) * GW + (qx - (x0 - LP))];
                        bxs = fmaf(0.5f * (float)unpack_x(g), e, bxs);
                        bys = fmaf(0.5f * (float)unpack_y(g), e, bys);
                    }
            }
            const double dx = -(Hyy * (double)bxs - Hxy * (double)bys) / det;
            const double dy = -(Hxx * (double)bys - Hxy * (double)bxs) / det;
            ux = fminf(fmaxf((float)((double)ux + dx), (float)(d0x - 1)), (float)(d0x + 1));
            uy = fminf(fmaxf((float)((double)uy + dy), (float)(d0y - 1)), (float)(d0y + 1));
        }
        if (inside) {
            float2 *out = reinterpret_cast<float2 *>(io[s].flow[dir]);
            out[(size_t)y * W + x] = make_float2(ux, uy);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- blend
// Code 1 per pixel. The scalar chain (Blend, displacements, flow
// magnitudes, softmax exponent difference) is evaluated in double so that
// no FP32 coordinate or large exponent is formed; bilinear sampling and
// the composite are FP32.
struct PixBlend {
    int lx, ly, rx, ry;      // integer cell corners of the L and R samples
    float lfx, lfy, rfx, rfy;
    float sL;                // SoftmaxL (SoftmaxR = 1 - sL)
};

__device__ __forceinline__ float finite0(float v) { return isfinite(v) ? v : 0.f; }

__device__ __forceinline__ PixBlend blend_setup(int x, int y, int H, int W, int axis, const float *blend,
                                                const float *flr, const float *frl, BlendParams bp)
{
    const size_t p = (size_t)y * W + x;
    const double t = blend ? (double)blend[p] : (axis == 0 ? (x + 1.0) / (W + 1.0) : (y + 1.0) / (H + 1.0));
    const float2 vrl = reinterpret_cast<const float2 *>(frl)[p];
    const float2 vlr = reinterpret_cast<const float2 *>(flr)[p];
    const double rlx = finite0(vrl.x), rly = finite0(vrl.y), lrx = finite0(vlr.x), lry = finite0(vlr.y);
    const double ax = rlx * t, ay = rly * t, bx = lrx * (1.0 - t), by = lry * (1.0 - t);
    const double fax = floor(ax), fay = floor(ay), fbx = floor(bx), fby = floor(by);
    PixBlend r;
    r.lx = x + (int)fax;
    r.ly = y + (int)fay;
    r.rx = x + (int)fbx;
    r.ry = y + (int)fby;
    r.lfx = (float)(ax - fax);
    r.lfy = (float)(ay - fay);
    r.rfx = (float)(bx - fbx);
    r.rfy = (float)(by - fby);
    if (bp.mode == 1) {
        r.sL = (float)(1.0 - t);
    } else {
        const double S = axis == 0 ? (double)W : (double)H;
        const double mrl = sqrt(rlx * rlx + rly * rly) / S, mlr = sqrt(lrx * lrx + lry * lry) / S;
        const double zL = (double)bp.k_sharp * (1.0 - t) * (1.0 + (double)bp.k_flowmag * mrl);
        const double zR = (double)bp.k_sharp * t * (1.0 + (double)bp.k_flowmag * mlr);
        r.sL = 1.0f / (1.0f + expf((float)(zR - zL)));
    }
    return r;
}

__device__ __forceinline__ void sample_u8(const uint8_t *img, int pitch, int H, int W, int x0, int y0, float fx,
                                          float fy, float out[3])
{
    const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    const uint8_t *ra = img + (size_t)clampi(y0, 0, H - 1) * pitch;
    const uint8_t *rb = img + (size_t)clampi(y0 + 1, 0, H - 1) * pitch;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const float v00 = ra[3 * xa + c], v01 = ra[3 * xb + c], v10 = rb[3 * xa + c], v11 = rb[3 * xb + c];
        const float top = v00 + fx * (v01 - v00), bot = v10 + fx * (v11 - v10);
        out[c] = top + fy * (bot - top);
    }
}

__global__ __launch_bounds__(256) void k_blend(const StripIO *__restrict__ io, const int32_t *__restrict__ prefix,
                                               int n, int total, BlendParams bp)
{
    TILE_LOOP(total, 0)
    {
        const int s = find_strip(prefix, n, t);
        const int local = t - prefix[s];
        const StripIO &o = io[s];
        const int W = o.W, H = o.H;
        const int segs = ceil_div(W, kRowTW);
        const int y = local / segs;
        const int x = (local - y * segs) * kRowTW + threadIdx.x;
        if (x >= W) continue;
        const PixBlend pb = blend_setup(x, y, H, W, o.axis, o.blend, o.flow[0], o.flow[1], bp);
        float cl[3], cr[3];
        sample_u8(o.L, o.pitchL, H, W, pb.lx, pb.ly, pb.lfx, pb.lfy, cl);
        sample_u8(o.R, o.pitchR, H, W, pb.rx, pb.ry, pb.rfx, pb.rfy, cr);
        const float sR = 1.0f - pb.sL;
        uint8_t *fo = o.F + (size_t)y * o.pitchF + 3 * x;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const float f = pb.sL * cl[c] + sR * cr[c];
            const float r = floorf(f + 0.5f);
            fo[c] = (uint8_t)fminf(fmaxf(r, 0.f), 255.f);
            if (o.Ff32) o.Ff32[3 * ((size_t)y * W + x) + c] = f;
        }
    }
}

// ------------------------------------------------------------- launchers
static inline int grid_for(int total, int grid)
{
    if (grid > 0) return grid < total ? grid : (total > 0 ? total : 1);
    return total > 0 ? total : 1;
}

hipError_t launch_luma(const StripIO *io, const StripLv *lv0, Work w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_luma, dim3(grid_for(w.total, grid)), dim3(256), 0, s, io, lv0, w.prefix, w.n, w.total);
    return hipGetLastError();
}

hipError_t launch_pyr(const StripLv *lv, Work w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_pyr, dim3(grid_for(w.total, grid)), dim3(256), 0, s, lv, w.prefix, w.n, w.total);
    return hipGetLastError();
}

template <int P, int R>
static hipError_t search_th(const StripLv *lv, Work w, int th, int grid, hipStream_t s)
{
    const int g = grid_for(w.total, grid);
    switch (th) {
    case 2: hipLaunchKernelGGL((k_search<P, R, 2>), dim3(g), dim3(128), 0, s, lv, w.prefix, w.n, w.total); break;
    case 8: hipLaunchKernelGGL((k_search<P, R, 8>), dim3(g), dim3(512), 0, s, lv, w.prefix, w.n, w.total); break;
    default: hipLaunchKernelGGL((k_search<P, R, 4>), dim3(g), dim3(256), 0, s, lv, w.prefix, w.n, w.total); break;
    }
    return hipGetLastError();
}

template <int P>
static hipError_t search_r(const StripLv *lv, Work w, int radius, int th, int grid, hipStream_t s)
{
    switch (radius) {
    case 1: return search_th<P, 1>(lv, w, th, grid, s);
    case 2: return search_th<P, 2>(lv, w, th, grid, s);
    case 3: return search_th<P, 3>(lv, w, th, grid, s);
    case 4: return search_th<P, 4>(lv, w, th, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_search(const StripLv *lv, Work w, int patch, int radius, int th, int grid, hipStream_t s)
{
    if (patch == 1) return search_r<1>(lv, w, radius, th, grid, s);
    if (patch == 2) return search_r<2>(lv, w, radius, th, grid, s);
    return hipErrorInvalidValue;
}

template <int P>
static hipError_t prop_th(const StripLv *lv, Work w, int steps, int median, int th, int grid, hipStream_t s)
{
    const int g = grid_for(w.total, grid);
    if (th == 4)
        hipLaunchKernelGGL((k_prop<P, 4>), dim3(g), dim3(256), 0, s, lv, w.prefix, w.n, w.total, steps, median);
    else
        hipLaunchKernelGGL((k_prop<P, 8>), dim3(g), dim3(256), 0, s, lv, w.prefix, w.n, w.total, steps, median);
    return hipGetLastError();
}

hipError_t launch_prop(const StripLv *lv, Work w, int patch, int steps, int median, int th, int grid,
                       hipStream_t s)
{
    if (steps + median > kHaloMax) return hipErrorInvalidValue;
    if (patch == 1) return prop_th<1>(lv, w, steps, median, th, grid, s);
    if (patch == 2) return prop_th<2>(lv, w, steps, median, th, grid, s);
    return hipErrorInvalidValue;
}

template <int LP>
static hipError_t refine_th(const StripLv *lv0, const StripIO *io, Work w, LkParams lk, int th, int grid,
                            hipStream_t s)
{
    const int g = grid_for(w.total, grid);
    if (th == 2)
        hipLaunchKernelGGL((k_refine<LP, 2>), dim3(g), dim3(128), 0, s, lv0, io, w.prefix, w.n, w.total, lk.iters,
                           lk.eps);
    else
        hipLaunchKernelGGL((k_refine<LP, 4>), dim3(g), dim3(256), 0, s, lv0, io, w.prefix, w.n, w.total, lk.iters,
                           lk.eps);
    return hipGetLastError();
}

hipError_t launch_refine(const StripLv *lv0, const StripIO *io, Work w, LkParams lk, int th, int grid,
                         hipStream_t s)
{
    switch (lk.patch) {
    case 1: return refine_th<1>(lv0, io, w, lk, th, grid, s);
    case 2: return refine_th<2>(lv0, io, w, lk, th, grid, s);
    case 3: return refine_th<3>(lv0, io, w, lk, th, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_blend(const StripIO *io, Work w, BlendParams bp, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_blend, dim3(grid_for(w.total, grid)), dim3(256), 0, s, io, w.prefix, w.n, w.total, bp);
    return hipGetLastError();
}

}  // namespace abf
