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
// Memory: luma planes carry a kPad-pixel replicated border, so the
// windows of the search, the propagation and the refinement are read
// straight from global memory (L1/L2) with aligned dword loads and
// byte-alignment shifts; only a window that leaves the image by more than
// kPad pixels takes a per-byte clamped path. Nothing depends on how far
// the flows of neighbouring pixels differ.
//
// The integer stages are bit-exact by construction (integer arithmetic,
// fixed candidate order, Jacobi updates into separate buffers). Patch
// costs use v_sad_u8 on byte-packed dwords.
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

#define TILE_LOOP(total) for (int t = xcd_block(blockIdx.x, gridDim.x); t < (total); t += gridDim.x)

__device__ __forceinline__ uint32_t pack16(int x, int y)
{
    return (uint32_t)(uint16_t)(int16_t)x | ((uint32_t)(uint16_t)(int16_t)y << 16);
}
__device__ __forceinline__ int unpack_x(uint32_t v) { return (int)(int16_t)(v & 0xffffu); }
__device__ __forceinline__ int unpack_y(uint32_t v) { return (int)(int16_t)(v >> 16); }

// Bytes c .. c+NB-1 of a padded luma row, normalised so that out[k] holds
// bytes c+4k .. c+4k+3. The row must hold those bytes (|c| <= kPad away).
template <int NB>
__device__ __forceinline__ void load_row(const uint8_t *__restrict__ row, int c, uint32_t (&out)[(NB + 3) / 4])
{
    constexpr int NO = (NB + 3) / 4;
    constexpr int ND = (NB + 6) / 4;  // dwords covering NB bytes at any alignment
    const int a = c & ~3;             // floor to a multiple of 4 (two's complement)
    const int s = c - a;
    const uint32_t *p = reinterpret_cast<const uint32_t *>(row + a);
    uint32_t w[ND + 1];
#pragma unroll
    for (int k = 0; k < ND; k++) w[k] = p[k];
    w[ND] = 0;
#pragma unroll
    for (int k = 0; k < NO; k++) out[k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], s);
}

// The same bytes with every index clamped to the image (for windows that
// leave the padded border); `img` points at pixel (0, 0).
template <int NB>
__device__ void load_row_clamped(const uint8_t *__restrict__ img, int H, int W, int pitch, int r, int c,
                                 uint32_t (&out)[(NB + 3) / 4])
{
    const uint8_t *row = img + (ptrdiff_t)clampi(r, 0, H - 1) * pitch;
#pragma unroll
    for (int k = 0; k < (NB + 3) / 4; k++) {
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; b++)
            if (4 * k + b < NB) v |= (uint32_t)row[clampi(c + 4 * k + b, 0, W - 1)] << (8 * b);
        out[k] = v;
    }
}

// dword of bytes o .. o+3 and byte o of a normalised row (o compile-time)
template <int NO>
__device__ __forceinline__ uint32_t dword_at(const uint32_t (&t)[NO], int o)
{
    const int q = o >> 2, sh = o & 3;
    return sh == 0 ? t[q] : __builtin_amdgcn_alignbyte(t[q + 1], t[q], sh);
}
template <int NO>
__device__ __forceinline__ uint32_t byte_at(const uint32_t (&t)[NO], int o)
{
    return (t[o >> 2] >> (8 * (o & 3))) & 0xffu;
}

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

// ------------------------------------------------------------------ luma
// Y = (77 R + 150 G + 29 B + 128) >> 8 for both images of every strip,
// written over the padded planes (a border pixel takes the value of the
// nearest image pixel). The intensity sums over the image (for the
// exposure step) are accumulated with 64-bit integer atomics, so they do
// not depend on the order of the additions.
__global__ __launch_bounds__(256) void k_zero_sums(const StripIO *__restrict__ io, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < 2 * n) io[i >> 1].sums[i & 1] = 0ull;
}

__device__ __forceinline__ int luma_of(uint32_t r, uint32_t g, uint32_t b) { return (77 * r + 150 * g + 29 * b + 128) >> 8; }

__global__ __launch_bounds__(256) void k_luma(const StripIO *__restrict__ io, const StripLv *__restrict__ lv,
                                              const int32_t *__restrict__ prefix, int n, int total)
{
    __shared__ unsigned long long red[2][4];
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        const int local = t - prefix[s];
        const int W = lv[s].W, H = lv[s].H;
        const int segs = ceil_div(W + 2 * kPad, kLumaTW);
        const int py = local / segs;
        const int px = (local - py * segs) * kLumaTW + 4 * (int)threadIdx.x;  // first of 4 padded columns
        const int y = py - kPad, x = px - kPad;
        const int cy = clampi(y, 0, H - 1);
        unsigned long long sl = 0, sr = 0;
        if (px < W + 2 * kPad) {
            const uint8_t *rl = io[s].L + (size_t)cy * io[s].pitchL;
            const uint8_t *rr = io[s].R + (size_t)cy * io[s].pitchR;
            int yl[4], yr[4];
            // four image pixels from 12-byte aligned runs when possible
            if (x >= 0 && x + 3 <= W - 1 && ((reinterpret_cast<uintptr_t>(rl + 3 * x) | reinterpret_cast<uintptr_t>(rr + 3 * x)) & 3) == 0) {
                const uint32_t *ql = reinterpret_cast<const uint32_t *>(rl + 3 * x);
                const uint32_t *qr = reinterpret_cast<const uint32_t *>(rr + 3 * x);
                const uint32_t a0 = ql[0], a1 = ql[1], a2 = ql[2], b0 = qr[0], b1 = qr[1], b2 = qr[2];
                yl[0] = luma_of(a0 & 0xff, (a0 >> 8) & 0xff, (a0 >> 16) & 0xff);
                yl[1] = luma_of(a0 >> 24, a1 & 0xff, (a1 >> 8) & 0xff);
                yl[2] = luma_of((a1 >> 16) & 0xff, a1 >> 24, a2 & 0xff);
                yl[3] = luma_of((a2 >> 8) & 0xff, (a2 >> 16) & 0xff, a2 >> 24);
                yr[0] = luma_of(b0 & 0xff, (b0 >> 8) & 0xff, (b0 >> 16) & 0xff);
                yr[1] = luma_of(b0 >> 24, b1 & 0xff, (b1 >> 8) & 0xff);
                yr[2] = luma_of((b1 >> 16) & 0xff, b1 >> 24, b2 & 0xff);
                yr[3] = luma_of((b2 >> 8) & 0xff, (b2 >> 16) & 0xff, b2 >> 24);
            } else {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int cx = clampi(x + k, 0, W - 1);
                    yl[k] = luma_of(rl[3 * cx], rl[3 * cx + 1], rl[3 * cx + 2]);
                    yr[k] = luma_of(rr[3 * cx], rr[3 * cx + 1], rr[3 * cx + 2]);
                }
            }
            const ptrdiff_t o = (ptrdiff_t)y * lv[s].ypitch + x;  // 4-byte aligned (padded rows are)
            *reinterpret_cast<uint32_t *>(lv[s].y[0] + o) =
                (uint32_t)yl[0] | ((uint32_t)yl[1] << 8) | ((uint32_t)yl[2] << 16) | ((uint32_t)yl[3] << 24);
            *reinterpret_cast<uint32_t *>(lv[s].y[1] + o) =
                (uint32_t)yr[0] | ((uint32_t)yr[1] << 8) | ((uint32_t)yr[2] << 16) | ((uint32_t)yr[3] << 24);
            if (y == cy) {
#pragma unroll
                for (int k = 0; k < 4; k++)
                    if (x + k >= 0 && x + k < W) {
                        sl += (unsigned long long)yl[k];
                        sr += (unsigned long long)yr[k];
                    }
            }
        }
        // workgroup sum, one atomic per image
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            sl += __shfl_xor(sl, m, 64);
            sr += __shfl_xor(sr, m, 64);
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][w] = sl;
            red[1][w] = sr;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long a = red[0][0] + red[0][1] + red[0][2] + red[0][3];
            const unsigned long long b = red[1][0] + red[1][1] + red[1][2] + red[1][3];
            if (a) atomicAdd(&io[s].sums[0], a);
            if (b) atomicAdd(&io[s].sums[1], b);
        }
        __syncthreads();
    }
}

// Exposure step: R's padded luma plane scaled by a = floor(2^16 sum(YL) /
// sum(YR)): YR' = min(255, (YR a + 2^15) >> 16); all-zero YR is kept.
__global__ __launch_bounds__(256) void k_gain(const StripIO *__restrict__ io, const StripLv *__restrict__ lv,
                                              const int32_t *__restrict__ prefix, int n, int total)
{
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        const int local = t - prefix[s];
        const int W = lv[s].W;
        const int segs = ceil_div(W + 2 * kPad, kLumaTW);
        const int py = local / segs;
        const int px = (local - py * segs) * kLumaTW + 4 * (int)threadIdx.x;
        const unsigned long long sl = io[s].sums[0], sr = io[s].sums[1];
        if (sr == 0 || px >= W + 2 * kPad) continue;
        const unsigned long long a = (sl << 16) / sr;
        uint32_t *p = reinterpret_cast<uint32_t *>(lv[s].y[1] + (ptrdiff_t)(py - kPad) * lv[s].ypitch + (px - kPad));
        const uint32_t v = *p;
        uint32_t o = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const unsigned long long g = ((unsigned long long)((v >> (8 * k)) & 0xffu) * a + (1ull << 15)) >> 16;
            o |= (uint32_t)(g > 255ull ? 255ull : g) << (8 * k);
        }
        *p = o;
    }
}

// --------------------------------------------------------------- pyramid
// One reduction, both images: 5x5 binomial (1 4 6 4 1)^2 / 256 sampled at
// even positions, clamped borders, rounding (s + 128) >> 8. Outputs cover
// the padded plane (a border pixel takes the value at the nearest image
// pixel); the taps of an image pixel stay inside the finer plane's border.
__global__ __launch_bounds__(256) void k_pyr(const StripLv *__restrict__ lv, const int32_t *__restrict__ prefix,
                                             int n, int total)
{
    constexpr int w5[5] = {1, 4, 6, 4, 1};
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int per_img = tiles_pyr(L.H, L.W);
        const int img = local / per_img;
        local -= img * per_img;
        const int tx = ceil_div(L.W + 2 * kPad, kPyrTW);
        const int ty = local / tx;
        const int px = (local - ty * tx) * kPyrTW + (int)(threadIdx.x & (kPyrTW - 1));
        const int py = ty * kPyrTH + (int)(threadIdx.x / kPyrTW);
        if (px < L.W + 2 * kPad && py < L.H + 2 * kPad) {
            const int x = clampi(px - kPad, 0, L.W - 1), y = clampi(py - kPad, 0, L.H - 1);
            const uint8_t *src = L.yfine[img];
            const int pf = L.ypitch_f;
            int acc = 0;
#pragma unroll
            for (int j = 0; j < 5; j++) {
                const uint8_t *row = src + (ptrdiff_t)(2 * y + j - 2) * pf + (2 * x - 2);
                int h = 0;
#pragma unroll
                for (int i = 0; i < 5; i++) h += w5[i] * row[i];
                acc += w5[j] * h;
            }
            L.y[img][(ptrdiff_t)(py - kPad) * L.ypitch + (px - kPad)] = (uint8_t)((acc + 128) >> 8);
        }
    }
}

// ---------------------------------------------------------------- search
// Integer patch-cost search around the upsampled coarser flow, both
// directions. A thread takes two horizontally adjacent pixels (x even):
// they share the centre (the coarser flow is upsampled by replication),
// so one set of target rows serves both and, for P = 2, the middle four
// columns of every row cost are shared. Key of a candidate:
// (cost << 11) | (L1 offset << 7) | enumeration index, so one unsigned min
// gives the lexicographic winner.
template <int P, int R, int TH>
__global__ __launch_bounds__(64 * TH) void k_search(const StripLv *__restrict__ lv,
                                                    const int32_t *__restrict__ prefix, int n, int total)
{
    constexpr int NC = 2 * R + 1;          // candidates per axis
    constexpr int NR = 2 * R + 2 * P + 1;  // target rows
    constexpr int NB = 2 * R + 2 * P + 2;  // target bytes per row (both pixels)
    constexpr int NBO = (NB + 3) / 4;
    constexpr int RB = 2 * P + 2;          // reference bytes per row (both pixels)
    const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const int ntx = ceil_div(W, kSearchTW), per_dir = ntx * ceil_div(H, TH);
        const int dir = local / per_dir;
        local -= dir * per_dir;
        const int tyi = local / ntx;
        const int x = (local - tyi * ntx) * kSearchTW + 2 * lane, y = tyi * TH + wrow;
        if (x >= W || y >= H) continue;  // no barrier in this kernel
        const uint8_t *ref = L.y[dir], *tgt = L.y[1 - dir];
        int cx = 0, cy = 0;
        if (L.dc[dir]) {
            const uint32_t v = L.dc[dir][(size_t)min(y >> 1, L.Hc - 1) * L.fpitch_c + min(x >> 1, L.Wc - 1)];
            cx = 2 * unpack_x(v);
            cy = 2 * unpack_y(v);
        }
        // reference rows y-P .. y+P, columns x-P .. x+1+P
        uint32_t rr[2 * P + 1][(RB + 3) / 4];
#pragma unroll
        for (int r = 0; r < 2 * P + 1; r++) load_row<RB>(ref + (ptrdiff_t)(y - P + r) * yp, x - P, rr[r]);
        // target rows, columns x+cx-R-P .. x+cx+R+P+1
        const int c0 = x + cx - R - P, r0 = y + cy - R - P;
        const bool inpad = c0 >= -kPad && c0 + NB - 1 <= W - 1 + kPad && r0 >= -kPad && r0 + NR - 1 <= H - 1 + kPad;
        uint32_t tt[NR][NBO];
        if (inpad) {
#pragma unroll
            for (int k = 0; k < NR; k++) load_row<NB>(tgt + (ptrdiff_t)(r0 + k) * yp, c0, tt[k]);
        } else {
#pragma unroll
            for (int k = 0; k < NR; k++) load_row_clamped<NB>(tgt, H, W, yp, r0 + k, c0, tt[k]);
        }
        uint32_t best0 = 0xffffffffu, best1 = 0xffffffffu;
        if constexpr (P == 2) {
            uint32_t rm[5], rl[5], rh[5];
#pragma unroll
            for (int r = 0; r < 5; r++) {
                rm[r] = dword_at(rr[r], 1);
                rl[r] = byte_at(rr[r], 0);
                rh[r] = byte_at(rr[r], 5);
            }
#pragma unroll
            for (int j = 0; j < NC; j++)
#pragma unroll
                for (int i = 0; i < NC; i++) {
                    uint32_t m = 0;
#pragma unroll
                    for (int r = 0; r < 5; r++) m = __builtin_amdgcn_sad_u8(rm[r], dword_at(tt[j + r], i + 1), m);
                    uint32_t s0 = m, s1 = m;
#pragma unroll
                    for (int r = 0; r < 5; r++) {
                        s0 = __builtin_amdgcn_sad_u8(rl[r], byte_at(tt[j + r], i), s0);
                        s1 = __builtin_amdgcn_sad_u8(rh[r], byte_at(tt[j + r], i + 5), s1);
                    }
                    const uint32_t K = ((uint32_t)(abs(i - R) + abs(j - R)) << 7) | (uint32_t)(j * NC + i);
                    best0 = min(best0, (s0 << 11) + K);
                    best1 = min(best1, (s1 << 11) + K);
                }
        } else {
            uint32_t r0m[3], r1m[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
                r0m[r] = rr[r][0] & 0x00ffffffu;
                r1m[r] = rr[r][0] >> 8;
            }
#pragma unroll
            for (int j = 0; j < NC; j++)
#pragma unroll
                for (int i = 0; i < NC; i++) {
                    uint32_t s0 = 0, s1 = 0;
#pragma unroll
                    for (int r = 0; r < 3; r++) {
                        s0 = __builtin_amdgcn_sad_u8(r0m[r], dword_at(tt[j + r], i) & 0x00ffffffu, s0);
                        s1 = __builtin_amdgcn_sad_u8(r1m[r], dword_at(tt[j + r], i + 1) & 0x00ffffffu, s1);
                    }
                    const uint32_t K = ((uint32_t)(abs(i - R) + abs(j - R)) << 7) | (uint32_t)(j * NC + i);
                    best0 = min(best0, (s0 << 11) + K);
                    best1 = min(best1, (s1 << 11) + K);
                }
        }
        uint32_t *out = L.ds[dir] + (size_t)y * L.fpitch + x;
        uint16_t *cst = L.cs[dir] + (size_t)y * L.fpitch + x;
        {
            const int idx = (int)(best0 & 127u), j = idx / NC, i = idx - j * NC;
            out[0] = pack16(cx + i - R, cy + j - R);
            cst[0] = (uint16_t)(best0 >> 11);
        }
        if (x + 1 < W) {
            const int idx = (int)(best1 & 127u), j = idx / NC, i = idx - j * NC;
            out[1] = pack16(cx + i - R, cy + j - R);
            cst[1] = (uint16_t)(best1 >> 11);
        }
    }
}

// ----------------------------------------------------------- propagation
// One Jacobi step per launch: each pixel keeps the lowest-cost vector among
// its own and those of its left, right, upper and lower neighbours in the
// previous iterate (neighbours outside the image skipped; on equal cost
// the earlier candidate in that order wins). The cost of a pixel's own
// vector is carried from the search / previous step, and a neighbour whose
// vector equals an earlier candidate's is skipped (same cost, loses the
// tie), so a pixel in a region of uniform flow evaluates no patch at all.
// A separate launch applies the (2M+1)^2 component-wise median.
__device__ __forceinline__ int med3i(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

template <int P>
__device__ __forceinline__ uint32_t patch_cost(const uint32_t (&rr)[2 * P + 1][(2 * P + 4) / 4],
                                               const uint8_t *__restrict__ tgt, int H, int W, int yp, int px, int py,
                                               int dx, int dy)
{
    constexpr int NB = 2 * P + 1;
    const int c0 = px + dx - P, r0 = py + dy - P;
    const bool inpad = c0 >= -kPad && c0 + NB - 1 <= W - 1 + kPad && r0 >= -kPad && r0 + NB - 1 <= H - 1 + kPad;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < NB; r++) {
        uint32_t t[(NB + 3) / 4];
        if (inpad) load_row<NB>(tgt + (ptrdiff_t)(r0 + r) * yp, c0, t);
        else load_row_clamped<NB>(tgt, H, W, yp, r0 + r, c0, t);
        if constexpr (P == 2) {
            s = __builtin_amdgcn_sad_u8(rr[r][0], t[0], s);
            s = __builtin_amdgcn_sad_u8(rr[r][1], t[1] & 0xffu, s);
        } else {
            s = __builtin_amdgcn_sad_u8(rr[r][0], t[0] & 0x00ffffffu, s);
        }
    }
    return s;
}

// buffers of propagation step `step` (1-based) of T: input, output
__device__ __forceinline__ void prop_bufs(const StripLv &L, int dir, int step, int T, int M, const uint32_t *&din,
                                          const uint16_t *&cin, uint32_t *&dout, uint16_t *&cout)
{
    din = step == 1 ? L.ds[dir] : L.dt[dir][(step - 2) & 1];
    cin = step == 1 ? L.cs[dir] : L.ct[dir][(step - 2) & 1];
    dout = (step == T && M == 0) ? L.df[dir] : L.dt[dir][(step - 1) & 1];
    cout = L.ct[dir][(step - 1) & 1];
}

// Work per workgroup: every pixel lists the neighbour vectors it must
// cost (on average well under one per pixel), the lists are packed into
// one LDS job array, the threads share the jobs evenly, and each pixel
// then picks its winner from its own cost slots in the fixed candidate
// order, so the result does not depend on the packing order.
template <int P, int TH>
__global__ __launch_bounds__(64 * TH) void k_prop_step(const StripLv *__restrict__ lv,
                                                       const int32_t *__restrict__ prefix, int n, int total, int step,
                                                       int T, int M)
{
    constexpr int NT = 64 * TH;
    __shared__ uint32_t jvec[4 * NT];    // candidate vector of a job
    __shared__ uint16_t jslot[4 * NT];   // owner thread * 4 + candidate - 1
    __shared__ uint32_t jcost[4 * NT];   // cost, indexed by slot
    __shared__ int njobs;
    const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch, fp = L.fpitch;
        const int ntx = ceil_div(W, kPropTW), per_dir = ntx * ceil_div(H, TH);
        const int dir = local / per_dir;
        local -= dir * per_dir;
        const int tyi = local / ntx;
        const int x0 = (local - tyi * ntx) * kPropTW, y0 = tyi * TH;
        const int x = x0 + lane, y = y0 + wrow;
        const bool valid = x < W && y < H;
        const uint32_t *din;
        const uint16_t *cin;
        uint32_t *dout;
        uint16_t *cout;
        prop_bufs(L, dir, step, T, M, din, cin, dout, cout);
        if (threadIdx.x == 0) njobs = 0;
        __syncthreads();
        const size_t p = (size_t)y * fp + x;
        uint32_t cand[5];
        bool need[5];
        need[0] = false;
        if (valid) {
            bool ok[5];
            cand[0] = din[p];
            ok[0] = true;
            cand[1] = x > 0 ? din[p - 1] : 0u;
            ok[1] = x > 0;
            cand[2] = x < W - 1 ? din[p + 1] : 0u;
            ok[2] = x < W - 1;
            cand[3] = y > 0 ? din[p - fp] : 0u;
            ok[3] = y > 0;
            cand[4] = y < H - 1 ? din[p + fp] : 0u;
            ok[4] = y < H - 1;
#pragma unroll
            for (int k = 1; k < 5; k++) {
                bool dup = !ok[k];
#pragma unroll
                for (int m = 0; m < k; m++) dup |= ok[m] && cand[m] == cand[k];
                need[k] = !dup;
                if (need[k]) {
                    const int j = atomicAdd(&njobs, 1);
                    jvec[j] = cand[k];
                    jslot[j] = (uint16_t)(threadIdx.x * 4 + k - 1);
                }
            }
        } else {
#pragma unroll
            for (int k = 1; k < 5; k++) need[k] = false;
        }
        __syncthreads();
        const int nj = njobs;
        const uint8_t *ref = L.y[dir], *tgt = L.y[1 - dir];
        for (int j = threadIdx.x; j < nj; j += NT) {
            const int slot = jslot[j];
            const int owner = slot >> 2;
            const int px = x0 + (owner & 63), py = y0 + (owner >> 6);
            uint32_t rr[2 * P + 1][(2 * P + 4) / 4];
#pragma unroll
            for (int r = 0; r < 2 * P + 1; r++) {
                load_row<2 * P + 1>(ref + (ptrdiff_t)(py - P + r) * yp, px - P, rr[r]);
                if constexpr (P == 2) rr[r][1] &= 0xffu;
                else rr[r][0] &= 0x00ffffffu;
            }
            const uint32_t v = jvec[j];
            jcost[slot] = patch_cost<P>(rr, tgt, H, W, yp, px, py, unpack_x(v), unpack_y(v));
        }
        __syncthreads();
        if (valid) {
            uint32_t bestv = cand[0], bestc = cin[p];
#pragma unroll
            for (int k = 1; k < 5; k++) {
                if (!need[k]) continue;
                const uint32_t c = jcost[threadIdx.x * 4 + k - 1];
                if (c < bestc) {
                    bestc = c;
                    bestv = cand[k];
                }
            }
            dout[p] = bestv;
            cout[p] = (uint16_t)bestc;
        }
        __syncthreads();
    }
}

template <int TH>
__global__ __launch_bounds__(64 * TH) void k_median(const StripLv *__restrict__ lv, const int32_t *__restrict__ prefix,
                                                    int n, int total, int T, int M)
{
    const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, fp = L.fpitch;
        const int ntx = ceil_div(W, kPropTW), per_dir = ntx * ceil_div(H, TH);
        const int dir = local / per_dir;
        local -= dir * per_dir;
        const int tyi = local / ntx;
        const int x = (local - tyi * ntx) * kPropTW + lane, y = tyi * TH + wrow;
        if (x >= W || y >= H) continue;
        const uint32_t *fin = T == 0 ? L.ds[dir] : L.dt[dir][(T - 1) & 1];
        uint32_t outv;
        if (M == 0) {
            outv = fin[(size_t)y * fp + x];
        } else {
            int vx[9], vy[9];
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const uint32_t *row = fin + (size_t)clampi(y + j - 1, 0, H - 1) * fp;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    const uint32_t v = row[clampi(x + i - 1, 0, W - 1)];
                    vx[3 * j + i] = unpack_x(v);
                    vy[3 * j + i] = unpack_y(v);
                }
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
        L.df[dir][(size_t)y * fp + x] = outv;
    }
}

// --------------------------------------------------------------- refine
// Level-0 Lucas-Kanade: central-difference gradient of Ref, normal matrix
// summed over the window (exact in integers: 4H), plus eps I; `iters`
// Gauss-Newton steps from the integer flow with bilinear Tgt samples; each
// component clamped to within 1 px of the integer flow. The displacement
// is split into floor + fraction so no FP32 coordinate is ever formed.
// A pixel whose window lies inside the image reads its Ref rows and its
// (WN+1)^2 Tgt block straight from the padded planes; a pixel near the
// border (its window positions are clamped, so they repeat) evaluates
// every window position on its own.
template <int LP, int TH>
__global__ __launch_bounds__(64 * TH) void k_refine(const StripLv *__restrict__ lv, const StripIO *__restrict__ io,
                                                    const int32_t *__restrict__ prefix, int n, int total, int iters,
                                                    float eps)
{
    constexpr int TW = kRefineTW;
    constexpr int WN = 2 * LP + 1;
    constexpr int AB = WN + 2;  // Ref bytes per row (window + gradient taps)
    const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const RefineSplit sp = refine_split(H, W, TH, LP);
        const int per_dir = sp.nint + sp.nbord;
        const int dir = local / per_dir;
        local -= dir * per_dir;
        int x, y;
        bool interior;
        if (local < sp.nint) {  // a tile of the interior rectangle
            const int ntx = ceil_div(sp.xhi - sp.xlo, TW);
            const int tyi = local / ntx;
            x = sp.xlo + (local - tyi * ntx) * TW + lane;
            y = sp.ylo + tyi * TH + wrow;
            if (x >= sp.xhi || y >= sp.yhi) continue;  // no barrier in this kernel
            interior = true;
        } else {  // border band: rows above and below, then columns left and right
            int b = (local - sp.nint) * TW * TH + (int)threadIdx.x;
            if (b >= sp.nbp) continue;
            const int top = sp.ylo * W, bot = (H - sp.yhi) * W;
            if (b < top) {
                y = b / W;
                x = b - y * W;
            } else if (b < top + bot) {
                b -= top;
                y = sp.yhi + b / W;
                x = b - (b / W) * W;
            } else {
                b -= top + bot;
                const int k = sp.xlo + W - sp.xhi;
                y = sp.ylo + b / k;
                const int c = b - (b / k) * k;
                x = c < sp.xlo ? c : sp.xhi + (c - sp.xlo);
            }
            interior = false;
        }
        const uint8_t *A = L.y[dir], *B = L.y[1 - dir];
        const uint32_t d0 = L.df[dir][(size_t)y * L.fpitch + x];
        const int d0x = unpack_x(d0), d0y = unpack_y(d0);

        // window: Ref value and doubled gradient at each (clamped) position
        int av[WN][WN], gx[WN][WN], gy[WN][WN];
        if (interior) {
            uint32_t ar[WN + 2][(AB + 3) / 4];
#pragma unroll
            for (int r = 0; r < WN + 2; r++) load_row<AB>(A + (ptrdiff_t)(y - LP - 1 + r) * yp, x - LP - 1, ar[r]);
#pragma unroll
            for (int j = 0; j < WN; j++)
#pragma unroll
                for (int i = 0; i < WN; i++) {
                    av[j][i] = (int)byte_at(ar[j + 1], i + 1);
                    gx[j][i] = (int)byte_at(ar[j + 1], i + 2) - (int)byte_at(ar[j + 1], i);
                    gy[j][i] = (int)byte_at(ar[j + 2], i + 1) - (int)byte_at(ar[j], i + 1);
                }
        } else {
#pragma unroll
            for (int j = 0; j < WN; j++)
#pragma unroll
                for (int i = 0; i < WN; i++) {
                    const int qx = clampi(x + i - LP, 0, W - 1), qy = clampi(y + j - LP, 0, H - 1);
                    const uint8_t *rw = A + (ptrdiff_t)qy * yp;  // q +- 1 stays inside the border
                    av[j][i] = rw[qx];
                    gx[j][i] = (int)rw[qx + 1] - (int)rw[qx - 1];
                    gy[j][i] = (int)rw[qx + yp] - (int)rw[qx - yp];
                }
        }
        int hxx = 0, hxy = 0, hyy = 0;
#pragma unroll
        for (int j = 0; j < WN; j++)
#pragma unroll
            for (int i = 0; i < WN; i++) {
                hxx += gx[j][i] * gx[j][i];
                hxy += gx[j][i] * gy[j][i];
                hyy += gy[j][i] * gy[j][i];
            }
        const double Hxx = 0.25 * hxx + eps, Hxy = 0.25 * hxy, Hyy = 0.25 * hyy + eps;
        const double det = Hxx * Hyy - Hxy * Hxy;
        float ux = (float)d0x, uy = (float)d0y;
        for (int it = 0; it < iters; it++) {
            const float fux = floorf(ux), fuy = floorf(uy);
            const float fx = ux - fux, fy = uy - fuy;
            const int iux = (int)fux, iuy = (int)fuy;
            float bxs = 0.f, bys = 0.f;
            const int c0 = x - LP + iux, r0 = y - LP + iuy;
            if (it == 0 && interior && c0 >= -kPad && c0 + WN <= W - 1 + kPad && r0 >= -kPad && r0 + WN <= H - 1 + kPad) {
                // the first step starts from the integer flow: the samples are
                // pixels (zero fractions), no interpolation
#pragma unroll
                for (int j = 0; j < WN; j++) {
                    uint32_t br[(WN + 3) / 4];
                    load_row<WN>(B + (ptrdiff_t)(r0 + j) * yp, c0, br);
#pragma unroll
                    for (int i = 0; i < WN; i++) {
                        const float e = (float)byte_at(br, i) - (float)av[j][i];
                        bxs = fmaf(0.5f * (float)gx[j][i], e, bxs);
                        bys = fmaf(0.5f * (float)gy[j][i], e, bys);
                    }
                }
            } else if (interior && c0 >= -kPad && c0 + WN <= W - 1 + kPad && r0 >= -kPad && r0 + WN <= H - 1 + kPad) {
                // (WN+1)^2 block of Tgt with shared bilinear weights
                float hrow[WN + 1][WN];
#pragma unroll
                for (int r = 0; r <= WN; r++) {
                    uint32_t br[(WN + 1 + 3) / 4];
                    load_row<WN + 1>(B + (ptrdiff_t)(r0 + r) * yp, c0, br);
                    float prev = (float)byte_at(br, 0);
#pragma unroll
                    for (int c = 0; c < WN; c++) {
                        const float nx = (float)byte_at(br, c + 1);
                        hrow[r][c] = prev + fx * (nx - prev);
                        prev = nx;
                    }
                }
#pragma unroll
                for (int j = 0; j < WN; j++)
#pragma unroll
                    for (int i = 0; i < WN; i++) {
                        const float bs = hrow[j][i] + fy * (hrow[j + 1][i] - hrow[j][i]);
                        const float e = bs - (float)av[j][i];
                        bxs = fmaf(0.5f * (float)gx[j][i], e, bxs);
                        bys = fmaf(0.5f * (float)gy[j][i], e, bys);
                    }
            } else {
#pragma unroll
                for (int j = 0; j < WN; j++)
#pragma unroll
                    for (int i = 0; i < WN; i++) {
                        const int qx = clampi(x + i - LP, 0, W - 1), qy = clampi(y + j - LP, 0, H - 1);
                        const int sx = qx + iux, sy = qy + iuy;
                        const uint8_t *ra = B + (ptrdiff_t)clampi(sy, 0, H - 1) * yp;
                        const uint8_t *rb = B + (ptrdiff_t)clampi(sy + 1, 0, H - 1) * yp;
                        const int xa = clampi(sx, 0, W - 1), xb = clampi(sx + 1, 0, W - 1);
                        const float v00 = ra[xa], v01 = ra[xb], v10 = rb[xa], v11 = rb[xb];
                        const float top = v00 + fx * (v01 - v00), bot = v10 + fx * (v11 - v10);
                        const float e = top + fy * (bot - top) - (float)av[j][i];
                        bxs = fmaf(0.5f * (float)gx[j][i], e, bxs);
                        bys = fmaf(0.5f * (float)gy[j][i], e, bys);
                    }
            }
            const double dx = -(Hyy * (double)bxs - Hxy * (double)bys) / det;
            const double dy = -(Hxx * (double)bys - Hxy * (double)bxs) / det;
            ux = fminf(fmaxf((float)((double)ux + dx), (float)(d0x - 1)), (float)(d0x + 1));
            uy = fminf(fmaxf((float)((double)uy + dy), (float)(d0y - 1)), (float)(d0y + 1));
        }
        float2 *out = reinterpret_cast<float2 *>(io[s].flow[dir]);
        out[(size_t)y * W + x] = make_float2(ux, uy);
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
    TILE_LOOP(total)
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

hipError_t launch_zero_sums(const StripIO *io, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_sums, dim3(ceil_div(2 * n, 256)), dim3(256), 0, s, io, n);
    return hipGetLastError();
}

hipError_t launch_gain(const StripIO *io, const StripLv *lv0, Work w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gain, dim3(grid_for(w.total, grid)), dim3(256), 0, s, io, lv0, w.prefix, w.n, w.total);
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
    case 1: hipLaunchKernelGGL((k_search<P, R, 1>), dim3(g), dim3(64), 0, s, lv, w.prefix, w.n, w.total); break;
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
static hipError_t prop_th(const StripLv *lv, Work w, int step, int steps, int median, int th, int grid,
                          hipStream_t s)
{
    const int g = grid_for(w.total, grid);
    if (step == 0) {
        switch (th) {
        case 1: hipLaunchKernelGGL((k_median<1>), dim3(g), dim3(64), 0, s, lv, w.prefix, w.n, w.total, steps, median); break;
        case 2: hipLaunchKernelGGL((k_median<2>), dim3(g), dim3(128), 0, s, lv, w.prefix, w.n, w.total, steps, median); break;
        default: hipLaunchKernelGGL((k_median<4>), dim3(g), dim3(256), 0, s, lv, w.prefix, w.n, w.total, steps, median); break;
        }
        return hipGetLastError();
    }
    switch (th) {
    case 1:
        hipLaunchKernelGGL((k_prop_step<P, 1>), dim3(g), dim3(64), 0, s, lv, w.prefix, w.n, w.total, step, steps, median);
        break;
    case 2:
        hipLaunchKernelGGL((k_prop_step<P, 2>), dim3(g), dim3(128), 0, s, lv, w.prefix, w.n, w.total, step, steps, median);
        break;
    default:
        hipLaunchKernelGGL((k_prop_step<P, 4>), dim3(g), dim3(256), 0, s, lv, w.prefix, w.n, w.total, step, steps, median);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_prop(const StripLv *lv, Work w, int patch, int step, int steps, int median, int th, int grid,
                       hipStream_t s)
{
    if (patch == 1) return prop_th<1>(lv, w, step, steps, median, th, grid, s);
    if (patch == 2) return prop_th<2>(lv, w, step, steps, median, th, grid, s);
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
