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
// costs use the byte-SAD instructions on byte-packed dwords.
#include "abf_tiles.h"

namespace abf {

// ------------------------------------------------------------------ luma
// Y = (77 R + 150 G + 29 B + 128) >> 8 for both images of every strip,
// written over the padded planes (a border pixel takes the value of the
// nearest image pixel). The intensity sums over the image (for the
// exposure step) are accumulated with 64-bit integer atomics, so they do
// not depend on the order of the additions; each sum is spread over
// kSumSlots slots (by workgroup) so that the atomics of the many
// workgroups do not all queue on one address.
__global__ __launch_bounds__(256) void k_zero_sums(const StripIO *__restrict__ io, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kSumWords * n) gst(io[i / kSumWords].sums)[i % kSumWords] = 0ull;
}

__device__ __forceinline__ int luma_of(uint32_t r, uint32_t g, uint32_t b) { return (77 * r + 150 * g + 29 * b + 128) >> 8; }

// Four consecutive RGB pixels (12 bytes) of a row starting at p, from
// aligned dwords when those lie inside [lo, hi) (the image data), else
// byte by byte; luma of each.
__device__ __forceinline__ void luma4(const uint8_t *p, uintptr_t lo, uintptr_t hi, int (&yv)[4])
{
    const uintptr_t a = (uintptr_t)p & ~(uintptr_t)3;
    if (a >= lo && a + 16 <= hi) {
        const auto q = reinterpret_cast<const __attribute__((address_space(1))) uint32_t *>(a);
        const uint32_t w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3];
        const int sh = (int)((uintptr_t)p - a);
        const uint32_t a0 = __builtin_amdgcn_alignbyte(w1, w0, sh), a1 = __builtin_amdgcn_alignbyte(w2, w1, sh),
                       a2 = __builtin_amdgcn_alignbyte(w3, w2, sh);
        yv[0] = luma_of(a0 & 0xff, (a0 >> 8) & 0xff, (a0 >> 16) & 0xff);
        yv[1] = luma_of(a0 >> 24, a1 & 0xff, (a1 >> 8) & 0xff);
        yv[2] = luma_of((a1 >> 16) & 0xff, a1 >> 24, a2 & 0xff);
        yv[3] = luma_of((a2 >> 8) & 0xff, (a2 >> 16) & 0xff, a2 >> 24);
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++) yv[k] = luma_of(p[3 * k], p[3 * k + 1], p[3 * k + 2]);
    }
}

// Outputs of a padded row in groups of four; a group wholly in the left or
// right border repeats the edge pixel's luma. With SUMS (the exposure step
// on) it also adds the strip's luma sums.
template <bool SUMS>
__global__ __launch_bounds__(64) void k_luma(const StripIO *__restrict__ io, const StripLv *__restrict__ lv,
                                             const int32_t *__restrict__ prefix, int n, int total)
{
    // a wave per tile of kLumaTW padded columns of a row: lane l takes the
    // groups of four columns l, l + 64, l + 128, l + 192
    static_assert(kLumaTW == 4 * 64 * 4, "four groups per lane");
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        const int local = t - prefix[s];
        const int W = lv[s].W, H = lv[s].H;
        const int segs = ceil_div(W + 2 * kPad, kLumaTW);
        const int py = local / segs;
        const int px0 = (local - py * segs) * kLumaTW;
        const int y = py - kPad;
        const int cy = clampi(y, 0, H - 1);
        const StripIO &o = io[s];
        const uint8_t *rl = o.L + (size_t)cy * o.pitchL;
        const uint8_t *rr = o.R + (size_t)cy * o.pitchR;
        const uintptr_t endL = (uintptr_t)(o.L + (size_t)(H - 1) * o.pitchL + 3 * (size_t)W);
        const uintptr_t endR = (uintptr_t)(o.R + (size_t)(H - 1) * o.pitchR + 3 * (size_t)W);
        uint32_t sl = 0, sr = 0;  // at most 16 x 255 per lane, 261120 per wave
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int px = px0 + 4 * ((int)threadIdx.x + 64 * j);  // first of 4 padded columns
            if (px >= W + 2 * kPad) break;
            const int x = px - kPad;
            int yl[4], yr[4];
            if (x >= 0 && x + 3 <= W - 1) {
                luma4(rl + 3 * x, (uintptr_t)o.L, endL, yl);
                luma4(rr + 3 * x, (uintptr_t)o.R, endR, yr);
            } else if (x + 3 < 0 || x > W - 1) {
                const int cx = x < 0 ? 0 : W - 1;
                const int vl = luma_of(rl[3 * cx], rl[3 * cx + 1], rl[3 * cx + 2]);
                const int vr = luma_of(rr[3 * cx], rr[3 * cx + 1], rr[3 * cx + 2]);
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    yl[k] = vl;
                    yr[k] = vr;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int cx = clampi(x + k, 0, W - 1);
                    yl[k] = luma_of(rl[3 * cx], rl[3 * cx + 1], rl[3 * cx + 2]);
                    yr[k] = luma_of(rr[3 * cx], rr[3 * cx + 1], rr[3 * cx + 2]);
                }
            }
            const ptrdiff_t off = (ptrdiff_t)y * lv[s].ypitch + x;  // 4-byte aligned (padded rows are)
            gst(reinterpret_cast<uint32_t *>(lv[s].y[0] + off))[0] =
                (uint32_t)yl[0] | ((uint32_t)yl[1] << 8) | ((uint32_t)yl[2] << 16) | ((uint32_t)yl[3] << 24);
            gst(reinterpret_cast<uint32_t *>(lv[s].y[1] + off))[0] =
                (uint32_t)yr[0] | ((uint32_t)yr[1] << 8) | ((uint32_t)yr[2] << 16) | ((uint32_t)yr[3] << 24);
            if (SUMS && y == cy) {
#pragma unroll
                for (int k = 0; k < 4; k++)
                    if (x + k >= 0 && x + k < W) {
                        sl += (uint32_t)yl[k];
                        sr += (uint32_t)yr[k];
                    }
            }
        }
        if constexpr (SUMS) {
            // wave sum, one atomic per image into the tile's slot
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) {
                sl += (uint32_t)__shfl_xor((int)sl, m, 64);
                sr += (uint32_t)__shfl_xor((int)sr, m, 64);
            }
            if (threadIdx.x == 0) {
                const int slot = (int)(blockIdx.x % kSumSlots);
                if (sl) atomicAdd(&io[s].sums[slot], (unsigned long long)sl);
                if (sr) atomicAdd(&io[s].sums[kSumSlots + slot], (unsigned long long)sr);
            }
        }
    }
}

// The gain of every strip from its two exposure sums (one wave per strip):
// a = floor(2^16 sum(YL) / sum(YR)), held at 2^24 (every nonzero byte
// saturates from there on, so the exposure step's result is the same and
// its products fit 32 bits); all-zero YR: 2^16, the identity.
__global__ __launch_bounds__(64) void k_gain_prep(const StripIO *__restrict__ io)
{
    static_assert(kSumSlots == 64, "one slot per lane");
    unsigned long long *const sums = io[blockIdx.x].sums;
    unsigned long long l = gld(sums)[threadIdx.x], r = gld(sums)[kSumSlots + threadIdx.x];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        l += __shfl_xor(l, m, 64);
        r += __shfl_xor(r, m, 64);
    }
    if (threadIdx.x == 0) {
        const unsigned long long a = r ? (l << 16) / r : 65536ull;
        gst(sums)[kSumGain] = a > (1ull << 24) ? (1ull << 24) : a;
    }
}

// Exposure step: R's padded luma plane scaled by a = floor(2^16 sum(YL) /
// sum(YR)) (made by k_gain_prep): YR' = min(255, (YR a + 2^15) >> 16);
// all-zero YR is kept (a = 2^16).
__global__ __launch_bounds__(64) void k_gain(const StripIO *__restrict__ io, const StripLv *__restrict__ lv,
                                             const int32_t *__restrict__ prefix, int n, int total)
{
    // a wave per luma tile (kLumaTW padded columns of a row): four dwords
    // per lane, kLumaTW / 4 / 64 = 4 apart
    static_assert(kLumaTW == 4 * 64 * 4, "four dwords per lane");
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        const int local = t - prefix[s];
        const int W = lv[s].W;
        const int segs = ceil_div(W + 2 * kPad, kLumaTW);
        const int py = local / segs;
        const int px0 = (local - py * segs) * kLumaTW;
        const uint32_t a = (uint32_t)gld(io[s].sums)[kSumGain];
        const auto row = gst(reinterpret_cast<uint32_t *>(lv[s].y[1] + (ptrdiff_t)(py - kPad) * lv[s].ypitch +
                                                          (px0 - kPad)));
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int i = (int)threadIdx.x + 64 * j;  // dword of the tile
            if (px0 + 4 * i >= W + 2 * kPad) break;
            const uint32_t v = row[i];
            uint32_t o = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t g = (((v >> (8 * k)) & 0xffu) * a + (1u << 15)) >> 16;
                o |= (g > 255u ? 255u : g) << (8 * k);
            }
            row[i] = o;
        }
    }
}

// --------------------------------------------------------------- pyramid
// One reduction, both images: 5x5 binomial (1 4 6 4 1)^2 / 256 sampled at
// even positions, clamped borders, rounding (s + 128) >> 8. Outputs cover
// the padded plane (a border pixel takes the value at the nearest image
// pixel); the taps of an image pixel stay inside the finer plane's border.
// A thread makes four horizontally adjacent outputs in each of two
// consecutive rows: inside the image it reads the 11 input bytes of each of
// the 7 source rows of the pair (3 shared) as aligned dwords and forms the
// horizontal taps once per source row with byte dot products; a group
// wholly in the left or right border repeats the edge output.
__device__ __forceinline__ uint32_t pyr_one(const uint8_t *src, int pf, int x, int y)
{
    constexpr int w5[5] = {1, 4, 6, 4, 1};
    int acc = 0;
#pragma unroll
    for (int j = 0; j < 5; j++) {
        const uint8_t *row = src + (ptrdiff_t)(2 * y + j - 2) * pf + (2 * x - 2);
        int hs = 0;
#pragma unroll
        for (int i = 0; i < 5; i++) hs += w5[i] * row[i];
        acc += w5[j] * hs;
    }
    return (uint32_t)((acc + 128) >> 8);
}

__global__ __launch_bounds__(256) void k_pyr(const StripLv *__restrict__ lv, const int32_t *__restrict__ prefix,
                                             int n, int total)
{
    constexpr uint32_t W4 = 0x04060401u;  // taps 1 4 6 4 on bytes 0..3
    constexpr int w5[5] = {1, 4, 6, 4, 1};
    static_assert(kPyrTH == 8, "a wave takes two output rows");
    // horizontal taps of the four outputs of one source row (bytes 2k .. 2k+4)
    auto hsum = [&](const uint32_t (&r)[3], uint32_t (&hs)[4]) {
        const uint32_t d1 = __builtin_amdgcn_alignbyte(r[1], r[0], 2);
        const uint32_t d3 = __builtin_amdgcn_alignbyte(r[2], r[1], 2);
        hs[0] = __builtin_amdgcn_udot4(r[0], W4, (r[1] >> 0) & 0xffu, false);
        hs[1] = __builtin_amdgcn_udot4(d1, W4, (r[1] >> 16) & 0xffu, false);
        hs[2] = __builtin_amdgcn_udot4(r[1], W4, (r[2] >> 0) & 0xffu, false);
        hs[3] = __builtin_amdgcn_udot4(d3, W4, (r[2] >> 16) & 0xffu, false);
    };
    auto pack = [](const uint32_t (&acc)[4]) {
        return ((acc[0] + 128) >> 8) | (((acc[1] + 128) >> 8) << 8) | (((acc[2] + 128) >> 8) << 16) |
               (((acc[3] + 128) >> 8) << 24);
    };
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
        const int px = (local - ty * tx) * kPyrTW + 4 * (int)(threadIdx.x & 63);
        const int py = ty * kPyrTH + 2 * (int)(threadIdx.x >> 6);  // the first of two output rows
        const int Hp = L.H + 2 * kPad;
        if (px >= L.W + 2 * kPad || py >= Hp) continue;  // no barrier in this kernel
        const bool two = py + 1 < Hp;
        const int x0 = px - kPad, ya = clampi(py - kPad, 0, L.H - 1), yb = clampi(py + 1 - kPad, 0, L.H - 1);
        const uint8_t *src = L.yfine[img];
        const int pf = L.ypitch_f;
        uint32_t oa, ob;
        if (x0 >= 0 && x0 + 3 <= L.W - 1) {
            if (yb == ya + 1) {
                // source rows 2 ya - 2 .. 2 ya + 4: the two outputs share three
                uint32_t r[7][3];
                load_rows<11, 7>(plane_org(src, pf), pf, 2 * ya - 2, 2 * x0 - 2, r);
                uint32_t acc_a[4] = {0, 0, 0, 0}, acc_b[4] = {0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < 7; j++) {
                    uint32_t hs[4];
                    hsum(r[j], hs);
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        if (j < 5) acc_a[k] += w5[j] * hs[k];
                        if (j >= 2) acc_b[k] += w5[j - 2] * hs[k];
                    }
                }
                oa = pack(acc_a);
                ob = pack(acc_b);
            } else {
                uint32_t r[5][3];
                load_rows<11, 5>(plane_org(src, pf), pf, 2 * ya - 2, 2 * x0 - 2, r);
                uint32_t acc[4] = {0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < 5; j++) {
                    uint32_t hs[4];
                    hsum(r[j], hs);
#pragma unroll
                    for (int k = 0; k < 4; k++) acc[k] += w5[j] * hs[k];
                }
                oa = pack(acc);
                ob = oa;  // both rows clamp to the same image row
            }
        } else if (x0 + 3 < 0 || x0 > L.W - 1) {
            const int cx = x0 < 0 ? 0 : L.W - 1;
            oa = pyr_one(src, pf, cx, ya) * 0x01010101u;
            ob = yb == ya ? oa : pyr_one(src, pf, cx, yb) * 0x01010101u;
        } else {
            oa = ob = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int cx = clampi(x0 + k, 0, L.W - 1);
                oa |= pyr_one(src, pf, cx, ya) << (8 * k);
                ob |= pyr_one(src, pf, cx, yb) << (8 * k);
            }
        }
        // padded rows are 64-byte aligned and px is a multiple of 4
        uint8_t *const orow = L.y[img] + (ptrdiff_t)(py - kPad) * L.ypitch + x0;
        gst(reinterpret_cast<uint32_t *>(orow))[0] = oa;
        if (two) gst(reinterpret_cast<uint32_t *>(orow + L.ypitch))[0] = ob;
    }
}

// ---------------------------------------------------------------- search
// Integer patch-cost search around the upsampled coarser flow, both
// directions. A thread takes two horizontally adjacent pixels (x even):
// they share the centre (the coarser flow is upsampled by replication),
// so one set of target rows serves both and, for P = 2, the middle four
// columns of every row cost are shared. Key of a candidate:
// (cost << 16) | (L1 offset << 7) | enumeration index, so one unsigned min
// gives the lexicographic winner. The sums run in v_sad_hi_u8, which adds
// each |difference| at bit 16, with the chain started at the candidate's
// tie bits: the last SAD leaves the key itself.
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
            const uint32_t v = gld(L.dc[dir])[(size_t)min(y >> 1, L.Hc - 1) * L.fpitch_c + min(x >> 1, L.Wc - 1)];
            cx = 2 * unpack_x(v);
            cy = 2 * unpack_y(v);
        }
        // reference rows y-P .. y+P, columns x-P .. x+1+P
        uint32_t rr[2 * P + 1][(RB + 3) / 4];
        load_rows<RB, 2 * P + 1>(plane_org(ref, yp), yp, y - P, x - P, rr);
        // target rows, columns x+cx-R-P .. x+cx+R+P+1
        const int c0 = x + cx - R - P, r0 = y + cy - R - P;
        const bool inpad = c0 >= -kPad && c0 + NB - 1 <= W - 1 + kPad && r0 >= -kPad && r0 + NR - 1 <= H - 1 + kPad;
        uint32_t tt[NR][NBO];
        if (inpad) {
            load_rows<NB, NR>(plane_org(tgt, yp), yp, r0, c0, tt);
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
            // candidate columns outer: each column offset's target words are
            // formed once per row
#pragma unroll
            for (int i = 0; i < NC; i++) {
                uint32_t tm[NR], tl[NR], th[NR];
#pragma unroll
                for (int q = 0; q < NR; q++) {
                    tm[q] = dword_at(tt[q], i + 1);
                    tl[q] = byte_at(tt[q], i);
                    th[q] = byte_at(tt[q], i + 5);
                }
#pragma unroll
                for (int j = 0; j < NC; j++) {
                    const uint32_t K = ((uint32_t)(abs(i - R) + abs(j - R)) << 7) | (uint32_t)(j * NC + i);
                    uint32_t m = K;
#pragma unroll
                    for (int r = 0; r < 5; r++) m = __builtin_amdgcn_sad_hi_u8(rm[r], tm[j + r], m);
                    uint32_t s0 = m, s1 = m;
#pragma unroll
                    for (int r = 0; r < 5; r++) {
                        s0 = __builtin_amdgcn_sad_hi_u8(rl[r], tl[j + r], s0);
                        s1 = __builtin_amdgcn_sad_hi_u8(rh[r], th[j + r], s1);
                    }
                    best0 = min(best0, s0);
                    best1 = min(best1, s1);
                    asm volatile("" : "+v"(best0), "+v"(best1));  // min chains in candidate order
                }
            }
        } else {
            uint32_t r0m[3], r1m[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
                r0m[r] = rr[r][0] & 0x00ffffffu;
                r1m[r] = rr[r][0] >> 8;
            }
#pragma unroll
            for (int i = 0; i < NC; i++) {
                uint32_t t0[NR], t1[NR];
#pragma unroll
                for (int q = 0; q < NR; q++) {
                    t0[q] = dword_at(tt[q], i) & 0x00ffffffu;
                    t1[q] = dword_at(tt[q], i + 1) & 0x00ffffffu;
                }
#pragma unroll
                for (int j = 0; j < NC; j++) {
                    const uint32_t K = ((uint32_t)(abs(i - R) + abs(j - R)) << 7) | (uint32_t)(j * NC + i);
                    uint32_t s0 = K, s1 = K;
#pragma unroll
                    for (int r = 0; r < 3; r++) {
                        s0 = __builtin_amdgcn_sad_hi_u8(r0m[r], t0[j + r], s0);
                        s1 = __builtin_amdgcn_sad_hi_u8(r1m[r], t1[j + r], s1);
                    }
                    best0 = min(best0, s0);
                    best1 = min(best1, s1);
                    asm volatile("" : "+v"(best0), "+v"(best1));  // min chains in candidate order
                }
            }
        }
        auto out = gst(L.ds[dir] + (size_t)y * L.fpitch + x);
        auto cst = gst(L.cs[dir] + (size_t)y * L.fpitch + x);
        {
            const int idx = (int)(best0 & 127u), j = idx / NC, i = idx - j * NC;
            out[0] = pack16(cx + i - R, cy + j - R);
            cst[0] = (uint16_t)(best0 >> 16);
        }
        if (x + 1 < W) {
            const int idx = (int)(best1 & 127u), j = idx / NC, i = idx - j * NC;
            out[1] = pack16(cx + i - R, cy + j - R);
            cst[1] = (uint16_t)(best1 >> 16);
        }
    }
}

// The same search for 5x5 patches with a 2 x 2 quad of pixels per thread
// (x, x+1 at rows y, y+1 with y even): the four share the centre, one set
// of 2R+6 target rows serves them, and for each candidate the sums of
// rows y-1 .. y+2 (middle four columns, and the two outer columns on
// their own) are shared, so the row y-2 and y+3 terms are all that
// differ between the two rows of the quad: 18 byte SADs per candidate for
// four pixels instead of 30. A tile of TH rows (TH even) is TH/2 waves,
// each a row pair of 128 columns; results are those of k_search.
template <int R, int TH>
__global__ __launch_bounds__(32 * TH) void k_search_quad(const StripLv *__restrict__ lv,
                                                         const int32_t *__restrict__ prefix, int n, int total)
{
    constexpr int P = 2;
    constexpr int NC = 2 * R + 1;          // candidates per axis
    constexpr int NR = 2 * R + 2 * P + 2;  // target rows (both output rows)
    constexpr int NB = 2 * R + 2 * P + 2;  // target bytes per row (both pixels)
    constexpr int NBO = (NB + 3) / 4;
    constexpr int RB = 2 * P + 2;          // reference bytes per row (both pixels)
    static_assert(TH % 2 == 0, "row pairs");
    const int lane = threadIdx.x & 63, wpair = threadIdx.x >> 6;
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
        const int x = (local - tyi * ntx) * kSearchTW + 2 * lane, y = tyi * TH + 2 * wpair;
        if (x >= W || y >= H) continue;  // no barrier in this kernel
        const uint8_t *ref = L.y[dir], *tgt = L.y[1 - dir];
        int cx = 0, cy = 0;
        if (L.dc[dir]) {
            const uint32_t v = gld(L.dc[dir])[(size_t)min(y >> 1, L.Hc - 1) * L.fpitch_c + min(x >> 1, L.Wc - 1)];
            cx = 2 * unpack_x(v);
            cy = 2 * unpack_y(v);
        }
        // reference rows y-P .. y+1+P (row y+1 may be the first row past the
        // image: its rows lie in the padded border), columns x-P .. x+1+P
        uint32_t rr[2 * P + 2][(RB + 3) / 4];
        load_rows<RB, 2 * P + 2>(plane_org(ref, yp), yp, y - P, x - P, rr);
        const int c0 = x + cx - R - P, r0 = y + cy - R - P;
        const bool inpad = c0 >= -kPad && c0 + NB - 1 <= W - 1 + kPad && r0 >= -kPad && r0 + NR - 1 <= H - 1 + kPad;
        uint32_t tt[NR][NBO];
        if (inpad) {
            load_rows<NB, NR>(plane_org(tgt, yp), yp, r0, c0, tt);
        } else {
#pragma unroll
            for (int k = 0; k < NR; k++) load_row_clamped<NB>(tgt, H, W, yp, r0 + k, c0, tt[k]);
        }
        uint32_t rm[6], rl[6], rh[6];
#pragma unroll
        for (int r = 0; r < 6; r++) {
            rm[r] = dword_at(rr[r], 1);
            rl[r] = byte_at(rr[r], 0);
            rh[r] = byte_at(rr[r], 5);
        }
        uint32_t b00 = 0xffffffffu, b01 = 0xffffffffu, b10 = 0xffffffffu, b11 = 0xffffffffu;
        // candidate column i outer: the target words and bytes at column
        // offset i are formed once per row and serve all NC candidate rows
        // (the order of the candidates does not matter: ties are in the key)
#pragma unroll
        for (int i = 0; i < NC; i++) {
            uint32_t tm[NR], tl[NR], th[NR];
#pragma unroll
            for (int q = 0; q < NR; q++) {
                tm[q] = dword_at(tt[q], i + 1);
                tl[q] = byte_at(tt[q], i);
                th[q] = byte_at(tt[q], i + 5);
            }
#pragma unroll
            for (int j = 0; j < NC; j++) {
                // the sums accumulate in the upper 16 bits (v_sad_hi_u8), and the
                // outer-column chains start at the tie key, so that m + l is
                // already the candidate's key (cost << 16) | K
                const uint32_t K = ((uint32_t)(abs(i - R) + abs(j - R)) << 7) | (uint32_t)(j * NC + i);
                uint32_t m = 0, l = K, h = K;
#pragma unroll
                for (int r = 1; r < 5; r++) {
                    m = __builtin_amdgcn_sad_hi_u8(rm[r], tm[j + r], m);
                    l = __builtin_amdgcn_sad_hi_u8(rl[r], tl[j + r], l);
                    h = __builtin_amdgcn_sad_hi_u8(rh[r], th[j + r], h);
                }
                const uint32_t m0 = __builtin_amdgcn_sad_hi_u8(rm[0], tm[j], m);
                const uint32_t m5 = __builtin_amdgcn_sad_hi_u8(rm[5], tm[j + 5], m);
                const uint32_t l0 = __builtin_amdgcn_sad_hi_u8(rl[0], tl[j], l);
                const uint32_t l5 = __builtin_amdgcn_sad_hi_u8(rl[5], tl[j + 5], l);
                const uint32_t h0 = __builtin_amdgcn_sad_hi_u8(rh[0], th[j], h);
                const uint32_t h5 = __builtin_amdgcn_sad_hi_u8(rh[5], th[j + 5], h);
                b00 = min(b00, m0 + l0);
                b01 = min(b01, m0 + h0);
                b10 = min(b10, m5 + l5);
                b11 = min(b11, m5 + h5);
                // keep the min chains in candidate order (a reassociated
                // tree would hold every candidate's key at once)
                asm volatile("" : "+v"(b00), "+v"(b01), "+v"(b10), "+v"(b11));
            }
        }
        const uint32_t best[2][2] = {{b00, b01}, {b10, b11}};
#pragma unroll
        for (int dy = 0; dy < 2; dy++) {
            if (y + dy >= H) break;
            auto out = gst(L.ds[dir] + (size_t)(y + dy) * L.fpitch + x);
            auto cst = gst(L.cs[dir] + (size_t)(y + dy) * L.fpitch + x);
#pragma unroll
            for (int dx = 0; dx < 2; dx++) {
                if (x + dx >= W) break;
                const uint32_t b = best[dy][dx];
                const int idx = (int)(b & 127u), jj = idx / NC, ii = idx - jj * NC;
                out[dx] = pack16(cx + ii - R, cy + jj - R);
                cst[dx] = (uint16_t)(b >> 16);
            }
        }
    }
}

// --------------------------------------------------------------- refine
// Level-0 Lucas-Kanade (step 4 of the flow): central-difference gradient
// of Ref, normal matrix summed over the window plus eps I, `iters`
// Gauss-Newton steps from the integer flow with bilinear Tgt samples, each
// component clamped to within 1 px of the integer flow.
//
// Everything that depends only on bytes is an exact integer sum: with the
// doubled gradients g = 2 grad A (integers), the window sums 4H = sum g g^T,
// sum g A and, for an integer displacement d, the correlations
// S(d) = sum g Tgt(q + d) are dot products of 16-bit pairs (v_dot2_i32_i16).
// The bilinear sample is linear in its four corners, so the right-hand side
// sum g (Tgt(q + u) - A) of a fractional u is the bilinear combination of
// S(d) - sum g A over the corners d of the cell of u, formed in FP32 with
// the 2x2 solve (the sums convert exactly; the combination, the solve and
// the iterate round at 2^-24 relative, far below the flow tolerance: the
// flow is stored as FP32 anyway). Window rows are padded to an even width
// with a zero gradient, so the padding sample never contributes.
//
// A pixel whose window lies inside the image reads its Ref rows and its
// (WN+1)^2 Tgt block from the padded planes; a pixel near the border (its
// window positions are clamped and repeat), or whose Tgt block leaves the
// padded border, evaluates every window position on its own.
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int dot2(uint32_t a, uint32_t b, int c)
{
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, a), __builtin_bit_cast(s16x2, b), c, false);
}
__device__ __forceinline__ uint32_t sub2(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(s16x2, a) - __builtin_bit_cast(s16x2, b));
}
__device__ __forceinline__ int lo16(uint32_t v) { return (int)(int16_t)(v & 0xffffu); }
__device__ __forceinline__ int hi16(uint32_t v) { return (int)(int16_t)(v >> 16); }

// bytes B, B+1 of a normalised row as a pair of 16-bit values; with Z the
// second value is zero
template <int B, bool Z, int NO>
__device__ __forceinline__ uint32_t pair_at(const uint32_t (&t)[NO])
{
    constexpr int q = B >> 2, o = B & 3;
    constexpr uint32_t sel = (uint32_t)o | 0x0c00u | (Z ? 0x0c0000u : (uint32_t)(o + 1) << 16) | 0x0c000000u;
    static_assert(q < NO && (Z || o < 3 || q + 1 < NO), "pair outside the row");
    if constexpr (Z || o < 3) return __builtin_amdgcn_perm(0u, t[q], sel);
    else return __builtin_amdgcn_perm(t[q + 1], t[q], sel);
}

template <int NP, int K, int NO>
__device__ __forceinline__ void odd_pairs(const uint32_t (&t)[NO], uint32_t (&o)[NP])
{
    // pairs of bytes (2k+1, 2k+2), the last one half zero
    if constexpr (K < NP - 1) {
        o[K] = pair_at<2 * K + 1, false>(t);
        odd_pairs<NP, K + 1>(t, o);
    } else {
        o[K] = pair_at<2 * K + 1, true>(t);
    }
}
template <int NP, int K, int NO>
__device__ __forceinline__ void gx_pairs(const uint32_t (&t)[NO], uint32_t (&g)[NP])
{
    // byte 2k+2 minus byte 2k (and the next pair), the last one half zero
    if constexpr (K < NP - 1) {
        g[K] = sub2(pair_at<2 * K + 2, false>(t), pair_at<2 * K, false>(t));
        gx_pairs<NP, K + 1>(t, g);
    } else {
        g[K] = sub2(pair_at<2 * K + 2, true>(t), pair_at<2 * K, true>(t));
    }
}
template <int NP, int K, int NO>
__device__ __forceinline__ void even_pairs(const uint32_t (&t)[NO], uint32_t (&e)[NP])
{
    e[K] = pair_at<2 * K, false>(t);
    if constexpr (K + 1 < NP) even_pairs<NP, K + 1>(t, e);
}
template <int NP, int K, int NO>
__device__ __forceinline__ void tgt_pairs(const uint32_t (&t)[NO], uint32_t (&e)[NP], uint32_t (&o)[NP])
{
    // pairs (2k, 2k+1) and (2k+1, 2k+2) of a Tgt row
    e[K] = pair_at<2 * K, false>(t);
    o[K] = pair_at<2 * K + 1, false>(t);
    if constexpr (K + 1 < NP) tgt_pairs<NP, K + 1>(t, e, o);
}

// The 2x2 solve of a refinement step, in FP32. Its inputs are integer
// window sums (|g| <= 255, so below 2^23 in magnitude for every window up
// to 7x7: they convert exactly); the determinant is Kahan's compensated
// ad - bc, since it cancels where the window's gradients are nearly
// parallel. The entries kept are those of H^-1 / 2 (the step is
// -H^-1 (b / 2), g doubled).
struct RefineSolve {
    float ixx, ixy, iyy;
};
__device__ __forceinline__ RefineSolve refine_solve(int hxx, int hxy, int hyy, float eps)
{
    const float Hxx = 0.25f * (float)hxx + eps, Hxy = 0.25f * (float)hxy, Hyy = 0.25f * (float)hyy + eps;
    const float w = Hxy * Hxy;
    const float det = fmaf(Hxx, Hyy, -w) + fmaf(-Hxy, Hxy, w);
    const float hdet = 0.5f / det;
    return {Hyy * hdet, Hxy * hdet, Hxx * hdet};
}
// sum over the window of g (Tgt(q + u) - A) from the corner correlations
// S(d) of the cell of u (corner (a, b) at column offset a, row offset b)
// and sum g A, with the bilinear weights of u's fraction
__device__ __forceinline__ float corner_mix(int s00, int s01, int s10, int s11, int sa, float fx, float fy)
{
    const float t = fmaf(fx, (float)(s01 - s00), (float)(s00 - sa));
    const float b = fmaf(fx, (float)(s11 - s10), (float)(s10 - sa));
    return fmaf(fy, b - t, t);
}
// one Gauss-Newton update, each component clamped to within 1 px of the
// integer flow
__device__ __forceinline__ void refine_update(const RefineSolve &q, float bx, float by, int d0x, int d0y, float &ux,
                                              float &uy)
{
    const float dx = fmaf(q.ixy, by, -q.ixx * bx);
    const float dy = fmaf(q.ixy, bx, -q.iyy * by);
    ux = fminf(fmaxf(ux + dx, (float)(d0x - 1)), (float)(d0x + 1));
    uy = fminf(fmaxf(uy + dy, (float)(d0y - 1)), (float)(d0y + 1));
}

// Corner correlations of target rows R0 .. R0 + NR - 1 of a window (tb
// holds them): row r adds to S(0, 0), S(1, 0) against window row r and to
// S(0, 1), S(1, 1) against window row r - 1 (x, y components), in row order.
template <int LP, int OFF, int NRW, int R0, int NR, int NBT>
__device__ __forceinline__ void corner_rows(const uint32_t (&gxp)[NRW][LP + 1], const uint32_t (&gyp)[NRW][LP + 1],
                                            const uint32_t (&tb)[NR][NBT], int (&sc)[8])
{
    constexpr int WN = 2 * LP + 1, NP = LP + 1;
#pragma unroll
    for (int i = 0; i < NR; i++) {
        const int r = R0 + i;
        uint32_t te[NP], to[NP];
        tgt_pairs<NP, 0>(tb[i], te, to);
#pragma unroll
        for (int k = 0; k < NP; k++) {
            if (r < WN) {
                sc[0] = dot2(gxp[OFF + r][k], te[k], sc[0]);
                sc[1] = dot2(gxp[OFF + r][k], to[k], sc[1]);
                sc[4] = dot2(gyp[OFF + r][k], te[k], sc[4]);
                sc[5] = dot2(gyp[OFF + r][k], to[k], sc[5]);
            }
            if (r > 0) {
                sc[2] = dot2(gxp[OFF + r - 1][k], te[k], sc[2]);
                sc[3] = dot2(gxp[OFF + r - 1][k], to[k], sc[3]);
                sc[6] = dot2(gyp[OFF + r - 1][k], te[k], sc[6]);
                sc[7] = dot2(gyp[OFF + r - 1][k], to[k], sc[7]);
            }
        }
    }
}

// `iters` Gauss-Newton steps of one interior pixel (x, y) from its integer
// flow (d0x, d0y): its window rows are rows OFF .. OFF + WN - 1 of the
// doubled-gradient pair arrays, sax / say its sums of g A. Returns the
// refined flow as a packed float2.
template <int LP, int OFF, int NRW>
__device__ __forceinline__ uint64_t refine_steps(const uint32_t (&gxp)[NRW][LP + 1], const uint32_t (&gyp)[NRW][LP + 1],
                                                 const uint8_t *Bo, int yp, int H, int W, int x, int y, int d0x,
                                                 int d0y, int sax, int say, const RefineSolve &q, int iters)
{
    constexpr int WN = 2 * LP + 1, NP = LP + 1;
    float ux = (float)d0x, uy = (float)d0y;
    for (int it = 0; it < iters; it++) {
        const float fux = floorf(ux), fuy = floorf(uy);
        const float fx = ux - fux, fy = uy - fuy;
        // the (WN+1)^2 target block at the cell of u; a block beyond the
        // padded border lies wholly on one side of the image, where every
        // sample is the edge value, so its origin is clamped to the
        // padded range without changing any sample
        const int c0 = clampi(x - LP + (int)fux, -kPad, W - 1 + kPad - (WN + 1));
        const int r0 = clampi(y - LP + (int)fuy, -kPad, H - 1 + kPad - WN);
        float bx, by;  // sum over the window of g (Tgt - A), g doubled
        if (it == 0) {
            // the integer start: one corner
            int sx = 0, sy = 0;
            uint32_t tb[WN][(WN + 1 + 3) / 4];
            load_rows<WN + 1, WN>(Bo, yp, r0, c0, tb);
#pragma unroll
            for (int j = 0; j < WN; j++) {
                uint32_t te[NP];
                even_pairs<NP, 0>(tb[j], te);
#pragma unroll
                for (int k = 0; k < NP; k++) {
                    sx = dot2(gxp[OFF + j][k], te[k], sx);
                    sy = dot2(gyp[OFF + j][k], te[k], sy);
                }
            }
            bx = (float)(sx - sax);
            by = (float)(sy - say);
        } else {
            // the WN + 1 target rows in two halves, each loaded and used
            // before the next is issued (fewer live registers)
            int sc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // s00x s01x s10x s11x s00y s01y s10y s11y
            constexpr int H1 = (WN + 1) / 2, H2 = WN + 1 - H1, NBT = (WN + 2 + 3) / 4;
            {
                uint32_t tb[H1][NBT];
                load_rows<WN + 2, H1>(Bo, yp, r0, c0, tb);
                corner_rows<LP, OFF, NRW, 0, H1>(gxp, gyp, tb, sc);
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                uint32_t tb[H2][NBT];
                load_rows<WN + 2, H2>(Bo, yp, r0 + H1, c0, tb);
                corner_rows<LP, OFF, NRW, H1, H2>(gxp, gyp, tb, sc);
            }
            bx = corner_mix(sc[0], sc[1], sc[2], sc[3], sax, fx, fy);
            by = corner_mix(sc[4], sc[5], sc[6], sc[7], say, fx, fy);
        }
        refine_update(q, bx, by, d0x, d0y, ux, uy);
    }
    return (uint64_t)__float_as_uint(ux) | ((uint64_t)__float_as_uint(uy) << 32);
}

// One pixel per thread; used for the 7x7 window (windows up to 5x5 take
// k_refine_pair below).
template <int LP, int TH>
__global__ __launch_bounds__(64 * TH) void k_refine(const StripLv *__restrict__ lv, const StripIO *__restrict__ io,
                                                    const int32_t *__restrict__ prefix, int n, int total, int iters,
                                                    float eps)
{
    constexpr int TW = kRefineTW;
    constexpr int WN = 2 * LP + 1;  // window width
    constexpr int NP = LP + 1;      // 16-bit pairs per window row (the last one half padding)
    constexpr int AB = WN + 2;      // Ref bytes per row (window + gradient taps)
    const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const RefineSplit sp = refine_split(H, W, TH, LP);
        const int dir = local / sp.nint;
        local -= dir * sp.nint;
        const int ntx = ceil_div(sp.xhi - sp.xlo, TW);
        const int tyi = local / ntx;
        const int x = sp.xlo + (local - tyi * ntx) * TW + lane;
        const int y = sp.ylo + tyi * TH + wrow;
        if (x >= sp.xhi || y >= sp.yhi) continue;  // no barrier in this kernel
        const uint8_t *Ao = plane_org(L.y[dir], yp), *Bo = plane_org(L.y[1 - dir], yp);
        const uint32_t d0 = gld(L.df[dir])[(uint32_t)(y * L.fpitch + x)];
        const int d0x = unpack_x(d0), d0y = unpack_y(d0);

        // doubled gradients and Ref values of the window as 16-bit pairs
        // (the window and its gradient taps lie inside the padded plane)
        uint32_t gxp[WN][NP], gyp[WN][NP];
        int hxx = 0, hxy = 0, hyy = 0, sax = 0, say = 0;
        {
            uint32_t op[WN + 2][NP], ar[WN + 2][(AB + 3) / 4];
            load_rows<AB, WN + 2>(Ao, yp, y - LP - 1, x - LP - 1, ar);
#pragma unroll
            for (int r = 0; r < WN + 2; r++) {
                odd_pairs<NP, 0>(ar[r], op[r]);
                if (r >= 1 && r <= WN) gx_pairs<NP, 0>(ar[r], gxp[r - 1]);
            }
#pragma unroll
            for (int j = 0; j < WN; j++)
#pragma unroll
                for (int k = 0; k < NP; k++) {
                    gyp[j][k] = sub2(op[j + 2][k], op[j][k]);
                    hxx = dot2(gxp[j][k], gxp[j][k], hxx);
                    hxy = dot2(gxp[j][k], gyp[j][k], hxy);
                    hyy = dot2(gyp[j][k], gyp[j][k], hyy);
                    sax = dot2(gxp[j][k], op[j + 1][k], sax);
                    say = dot2(gyp[j][k], op[j + 1][k], say);
                }
        }
        const RefineSolve q = refine_solve(hxx, hxy, hyy, eps);
        const uint64_t packed = refine_steps<LP, 0, WN>(gxp, gyp, Bo, yp, H, W, x, y, d0x, d0y, sax, say, q, iters);
        gst(reinterpret_cast<uint64_t *>(io[s].flow[dir]))[(uint32_t)(y * W + x)] = packed;
    }
}

// The interior refinement for windows up to 5x5 with a vertical pair of
// pixels per thread ((x, y) and (x, y+1)): the two windows share WN - 1 of
// their rows, so the Ref rows are loaded, the doubled gradients formed and
// the row sums of 4 H and sum g A taken once for the shared rows (the
// sums are exact integers, so the order of addition does not matter), and
// each pixel adds its own first or last row. The Gauss-Newton steps are
// those of k_refine, pixel by pixel. A tile of TH rows (TH even) is TH/2
// waves, each a row pair; the results are those of k_refine. Register
// budget: 96 VGPRs (5 waves per SIMD, no spills, with the fractional
// step's target rows loaded in two halves); at 80 (6 waves) it spills.
template <int LP, int TH>
__global__ __launch_bounds__(32 * TH) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_refine_pair(
    const StripLv *__restrict__ lv, const StripIO *__restrict__ io, const int32_t *__restrict__ prefix, int n,
    int total, int iters, float eps)
{
    constexpr int TW = kRefineTW;
    constexpr int WN = 2 * LP + 1;  // window width
    constexpr int NP = LP + 1;      // 16-bit pairs per window row (the last one half padding)
    constexpr int AB = WN + 2;      // Ref bytes per row (window + gradient taps)
    static_assert(TH % 2 == 0 && LP <= 2, "row pairs, windows up to 5x5");
    const int lane = threadIdx.x & 63, wpair = threadIdx.x >> 6;
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const RefineSplit sp = refine_split(H, W, TH, LP);
        const int dir = local / sp.nint;
        local -= dir * sp.nint;
        const int ntx = ceil_div(sp.xhi - sp.xlo, TW);
        const int tyi = local / ntx;
        const int x = sp.xlo + (local - tyi * ntx) * TW + lane;
        const int y = sp.ylo + tyi * TH + 2 * wpair;
        if (x >= sp.xhi || y >= sp.yhi) continue;  // no barrier in this kernel
        const bool two = y + 1 < sp.yhi;           // else row y + 1 is only read, in the padded plane
        const uint8_t *Ao = plane_org(L.y[dir], yp), *Bo = plane_org(L.y[1 - dir], yp);
        const auto df = gld(L.df[dir]);
        const uint32_t dA = df[(uint32_t)(y * L.fpitch + x)];
        const uint32_t dB = two ? df[(uint32_t)((y + 1) * L.fpitch + x)] : dA;

        // doubled gradients of the WN + 1 window rows of the pair
        uint32_t gxp[WN + 1][NP], gyp[WN + 1][NP];
        int hA[5], hB[5];  // 4 Hxx, 4 Hxy, 4 Hyy, sum gx A, sum gy A of each pixel
        {
            uint32_t op[WN + 3][NP], ar[WN + 3][(AB + 3) / 4];
            load_rows<AB, WN + 3>(Ao, yp, y - LP - 1, x - LP - 1, ar);
#pragma unroll
            for (int r = 0; r < WN + 3; r++) {
                odd_pairs<NP, 0>(ar[r], op[r]);
                if (r >= 1 && r <= WN + 1) gx_pairs<NP, 0>(ar[r], gxp[r - 1]);
            }
            int sh[5] = {0, 0, 0, 0, 0};  // rows 1 .. WN - 1, shared
#pragma unroll
            for (int j = 0; j <= WN; j++)
#pragma unroll
                for (int k = 0; k < NP; k++) gyp[j][k] = sub2(op[j + 2][k], op[j][k]);
#pragma unroll
            for (int j = 1; j < WN; j++)
#pragma unroll
                for (int k = 0; k < NP; k++) {
                    sh[0] = dot2(gxp[j][k], gxp[j][k], sh[0]);
                    sh[1] = dot2(gxp[j][k], gyp[j][k], sh[1]);
                    sh[2] = dot2(gyp[j][k], gyp[j][k], sh[2]);
                    sh[3] = dot2(gxp[j][k], op[j + 1][k], sh[3]);
                    sh[4] = dot2(gyp[j][k], op[j + 1][k], sh[4]);
                }
#pragma unroll
            for (int m = 0; m < 5; m++) hA[m] = hB[m] = sh[m];
#pragma unroll
            for (int k = 0; k < NP; k++) {
                hA[0] = dot2(gxp[0][k], gxp[0][k], hA[0]);
                hA[1] = dot2(gxp[0][k], gyp[0][k], hA[1]);
                hA[2] = dot2(gyp[0][k], gyp[0][k], hA[2]);
                hA[3] = dot2(gxp[0][k], op[1][k], hA[3]);
                hA[4] = dot2(gyp[0][k], op[1][k], hA[4]);
                hB[0] = dot2(gxp[WN][k], gxp[WN][k], hB[0]);
                hB[1] = dot2(gxp[WN][k], gyp[WN][k], hB[1]);
                hB[2] = dot2(gyp[WN][k], gyp[WN][k], hB[2]);
                hB[3] = dot2(gxp[WN][k], op[WN + 1][k], hB[3]);
                hB[4] = dot2(gyp[WN][k], op[WN + 1][k], hB[4]);
            }
        }
        const auto out = gst(reinterpret_cast<uint64_t *>(io[s].flow[dir]));
        {
            const RefineSolve q = refine_solve(hA[0], hA[1], hA[2], eps);
            out[(uint32_t)(y * W + x)] = refine_steps<LP, 0, WN + 1>(gxp, gyp, Bo, yp, H, W, x, y, unpack_x(dA),
                                                                     unpack_y(dA), hA[3], hA[4], q, iters);
        }
        if (two) {
            const RefineSolve q = refine_solve(hB[0], hB[1], hB[2], eps);
            out[(uint32_t)((y + 1) * W + x)] = refine_steps<LP, 1, WN + 1>(gxp, gyp, Bo, yp, H, W, x, y + 1,
                                                                           unpack_x(dB), unpack_y(dB), hB[3], hB[4],
                                                                           q, iters);
        }
    }
}

// Border pixel b (0 .. nbp - 1) of a level split by refine_split: the rows
// above and below the interior band, then the columns left and right of it.
__device__ __forceinline__ void border_pixel(const RefineSplit &sp, int H, int W, int b, int &x, int &y)
{
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
}

// The pixels whose window leaves the image (within LP of the border): every
// window position is clamped to the image on its own, so positions repeat.
// The clamped positions never decrease and step by 0 or 1, so the bytes a
// pixel needs from a row still form one short run: each window row loads
// its own (clamped) Ref and Tgt rows of the padded planes, and the 16-bit
// pairs of the dot products are gathered from the normalised run with
// per-pixel v_perm_b32 selectors. The arithmetic is that of k_refine.
__device__ __forceinline__ uint32_t psel(int b0, int b1)
{
    // selector of bytes b0, b1 (0..7 of hi:lo) as a 16-bit pair; b1 < 0: zero
    return (uint32_t)b0 | 0x0c00u | (b1 < 0 ? 0x0c0000u : (uint32_t)b1 << 16) | 0x0c000000u;
}

// The window of a border pixel: its clamped positions, the selectors that
// gather them from row runs, and its doubled gradients as 16-bit pairs with
// the exact sums 4 H and sum g A.
template <int LP>
struct BorderWin {
    static constexpr int WN = 2 * LP + 1, NP = LP + 1;
    int qx[WN], qy[WN];
    uint32_t sE[NP], sO[NP];
    uint32_t gxp[WN][NP], gyp[WN][NP];
    int hxx, hxy, hyy, sax, say;
};

template <int LP>
__device__ __forceinline__ void border_setup(const uint8_t *Ao, int yp, int H, int W, int x, int y, BorderWin<LP> &bw)
{
    constexpr int WN = 2 * LP + 1, NP = LP + 1, AB = WN + 2;
#pragma unroll
    for (int i = 0; i < WN; i++) {
        bw.qx[i] = clampi(x + i - LP, 0, W - 1);
        bw.qy[i] = clampi(y + i - LP, 0, H - 1);
    }
    // selectors: the Ref run starts at column qx[0] - 1, the Tgt run at
    // the cell column of qx[0]
    uint32_t sA[NP], sL[NP], sR[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const int i0 = 2 * k, i1 = 2 * k + 1;
        const int c0 = bw.qx[i0] - bw.qx[0] + 1, c1 = i1 < WN ? bw.qx[i1] - bw.qx[0] + 1 : -1;
        sA[k] = psel(c0, c1);
        sL[k] = psel(c0 - 1, c1 < 0 ? -1 : c1 - 1);
        sR[k] = psel(c0 + 1, c1 < 0 ? -1 : c1 + 1);
        bw.sE[k] = psel(c0 - 1, c1 < 0 ? -1 : c1 - 1);
        bw.sO[k] = psel(c0, c1);
    }
    int hxx = 0, hxy = 0, hyy = 0, sax = 0, say = 0;
    // the 3 WN Ref rows (clamped rows - 1, 0, + 1 of each window row), all
    // loads issued before the first is used
    uint32_t rw[WN][3][1][RawRows<AB>::ND + 1];
    int rs = 0;
#pragma unroll
    for (int j = 0; j < WN; j++)
#pragma unroll
        for (int d = 0; d < 3; d++) rs = issue_rows<AB, 1>(Ao, yp, bw.qy[j] + d - 1, bw.qx[0] - 1, rw[j][d]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < WN; j++) {
        uint32_t r[3][(AB + 3) / 4];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            uint32_t rr[1][(AB + 3) / 4];
            align_rows<AB, 1>(rw[j][d], rs, rr);
#pragma unroll
            for (int k = 0; k < (AB + 3) / 4; k++) r[d][k] = rr[0][k];
        }
#pragma unroll
        for (int k = 0; k < NP; k++) {
            const uint32_t av = __builtin_amdgcn_perm(r[1][1], r[1][0], sA[k]);
            uint32_t right = __builtin_amdgcn_perm(r[1][1], r[1][0], sR[k]);
            if constexpr (AB > 8) {
                // 7x7 window: the right tap of the last (half) pair can be
                // byte 8 of the run, beyond the 8 bytes one v_perm_b32
                // reaches; it is byte 4 of the next dword pair
                if (k == NP - 1 && bw.qx[WN - 1] - bw.qx[0] + 2 == 8)
                    right = __builtin_amdgcn_perm(r[1][2], r[1][1], psel(4, -1));
            }
            bw.gxp[j][k] = sub2(right, __builtin_amdgcn_perm(r[1][1], r[1][0], sL[k]));
            bw.gyp[j][k] = sub2(__builtin_amdgcn_perm(r[2][1], r[2][0], sA[k]),
                                __builtin_amdgcn_perm(r[0][1], r[0][0], sA[k]));
            hxx = dot2(bw.gxp[j][k], bw.gxp[j][k], hxx);
            hxy = dot2(bw.gxp[j][k], bw.gyp[j][k], hxy);
            hyy = dot2(bw.gyp[j][k], bw.gyp[j][k], hyy);
            sax = dot2(bw.gxp[j][k], av, sax);
            say = dot2(bw.gyp[j][k], av, say);
        }
    }
    bw.hxx = hxx;
    bw.hxy = hxy;
    bw.hyy = hyy;
    bw.sax = sax;
    bw.say = say;
}

// The four corner correlations S(d) = sum g Tgt(q + d), d = (ix + a, iy + b),
// of a border window (S[c][b][a], c = 0 for g_x, 1 for g_y), target indices
// clamped to the image: the Tgt run of a row holds the samples at
// qx[i] + ix (+ 1); a run beyond the padded border lies wholly on one side
// of the image and is clamped to it unchanged.
template <int LP>
__device__ __forceinline__ void border_corners(const BorderWin<LP> &bw, const uint8_t *Bo, int yp, int H, int W, int ix,
                                               int iy, int (&S)[2][2][2])
{
    constexpr int WN = 2 * LP + 1, NP = LP + 1;
    const int c0 = clampi(bw.qx[0] + ix, -kPad, W - 1 + kPad - (WN + 1));
    int s00x = 0, s01x = 0, s10x = 0, s11x = 0, s00y = 0, s01y = 0, s10y = 0, s11y = 0;
    // the 2 WN Tgt rows of the cells, all loads issued first
    uint32_t tw[WN][2][1][RawRows<WN + 2>::ND + 1];
    int ts = 0;
#pragma unroll
    for (int j = 0; j < WN; j++)
#pragma unroll
        for (int d = 0; d < 2; d++)
            ts = issue_rows<WN + 2, 1>(Bo, yp, clampi(bw.qy[j] + iy + d, -kPad, H - 1 + kPad), c0, tw[j][d]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < WN; j++) {
        uint32_t ta[1][(WN + 2 + 3) / 4], tb[1][(WN + 2 + 3) / 4];
        align_rows<WN + 2, 1>(tw[j][0], ts, ta);
        align_rows<WN + 2, 1>(tw[j][1], ts, tb);
#pragma unroll
        for (int k = 0; k < NP; k++) {
            const uint32_t ea = __builtin_amdgcn_perm(ta[0][1], ta[0][0], bw.sE[k]);
            const uint32_t oa = __builtin_amdgcn_perm(ta[0][1], ta[0][0], bw.sO[k]);
            const uint32_t eb = __builtin_amdgcn_perm(tb[0][1], tb[0][0], bw.sE[k]);
            const uint32_t ob = __builtin_amdgcn_perm(tb[0][1], tb[0][0], bw.sO[k]);
            s00x = dot2(bw.gxp[j][k], ea, s00x);
            s01x = dot2(bw.gxp[j][k], oa, s01x);
            s10x = dot2(bw.gxp[j][k], eb, s10x);
            s11x = dot2(bw.gxp[j][k], ob, s11x);
            s00y = dot2(bw.gyp[j][k], ea, s00y);
            s01y = dot2(bw.gyp[j][k], oa, s01y);
            s10y = dot2(bw.gyp[j][k], eb, s10y);
            s11y = dot2(bw.gyp[j][k], ob, s11y);
        }
    }
    S[0][0][0] = s00x;
    S[0][0][1] = s01x;
    S[0][1][0] = s10x;
    S[0][1][1] = s11x;
    S[1][0][0] = s00y;
    S[1][0][1] = s01y;
    S[1][1][0] = s10y;
    S[1][1][1] = s11y;
}

template <int LP>
__global__ __launch_bounds__(kRowTW) void k_refine_border(const StripLv *__restrict__ lv,
                                                          const StripIO *__restrict__ io,
                                                          const int32_t *__restrict__ prefix, int n, int total,
                                                          int iters, float eps)
{
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const RefineSplit sp = refine_split(H, W, 1, LP);
        const int nbt = ceil_div(sp.nbp, kRowTW);
        const int dir = local / nbt;
        local -= dir * nbt;
        int b = local * kRowTW + (int)threadIdx.x;
        if (b >= sp.nbp) continue;
        int x, y;
        border_pixel(sp, H, W, b, x, y);
        const uint8_t *Ao = plane_org(L.y[dir], yp), *Bo = plane_org(L.y[1 - dir], yp);
        const uint32_t d0 = gld(L.df[dir])[(uint32_t)(y * L.fpitch + x)];
        const int d0x = unpack_x(d0), d0y = unpack_y(d0);
        BorderWin<LP> bw;
        border_setup<LP>(Ao, yp, H, W, x, y, bw);
        const RefineSolve q = refine_solve(bw.hxx, bw.hxy, bw.hyy, eps);
        float ux = (float)d0x, uy = (float)d0y;
        for (int it = 0; it < iters; it++) {
            const float fux = floorf(ux), fuy = floorf(uy);
            const float fx = ux - fux, fy = uy - fuy;
            int S[2][2][2];
            border_corners<LP>(bw, Bo, yp, H, W, (int)fux, (int)fuy, S);
            refine_update(q, corner_mix(S[0][0][0], S[0][0][1], S[0][1][0], S[0][1][1], bw.sax, fx, fy),
                          corner_mix(S[1][0][0], S[1][0][1], S[1][1][0], S[1][1][1], bw.say, fx, fy), d0x, d0y, ux,
                          uy);
        }
        const uint64_t packed = (uint64_t)__float_as_uint(ux) | ((uint64_t)__float_as_uint(uy) << 32);
        gst(reinterpret_cast<uint64_t *>(io[s].flow[dir]))[(uint32_t)(y * W + x)] = packed;
    }
}

// ------------------------------------------------ classic pyramid LK
// The classic coarse-to-fine Lucas-Kanade (flow method 1): at every level
// a float flow starts from twice the coarser level's flow at
// (floor(x/2), floor(y/2)) (0 at the coarsest) and takes K Gauss-Newton
// steps with the window's normal matrix + eps I, the central-difference
// gradient of Ref and a bilinear Tgt (clamped indices), unclamped. A
// bilinear sample is linear in its four corners and every sample of a
// pixel's window has the same fractions, so the residual sum is the
// bilinear combination of four exact integer correlations of the doubled
// gradient with the target at integer offsets, minus the exact sum of the
// gradient times Ref; the combination and the 2x2 solve are double, so
// levels feed each other the values of an FP64 reference up to rounding
// order. Levels above 0 keep their flow as float64 x / y planes in the
// level's ds / df buffers (allocated with 8-byte entries for this method);
// level 0 writes the caller's float32 flow. Interior pixels take
// k_lk_interior (16-bit pair sums, as k_refine); the pixels within P of
// the image edge, whose window positions repeat, take lk_border_pixel
// (the row runs and gathers of k_refine_border), one thread each.

// One border pixel of the classic method (its window positions repeat):
// the clamped window and its exact sums as in k_refine_border, then K
// Gauss-Newton steps from twice the coarser flow, with the corner
// correlations of the cell of u at clamped target indices, combined with
// the bilinear weights and solved in double.
template <int P>
__device__ __forceinline__ void lk_border_pixel(const StripLv &L, const StripLv *__restrict__ lvc,
                                                const StripIO *__restrict__ io, int s, int dir, int x, int y, int K,
                                                double eps, bool level0)
{
    const int H = L.H, W = L.W, yp = L.ypitch;
    double ux = 0.0, uy = 0.0;
    if (lvc) {
        const StripLv &C = lvc[s];
        const size_t q = (size_t)min(y >> 1, C.H - 1) * C.fpitch + min(x >> 1, C.W - 1);
        ux = 2.0 * gld(reinterpret_cast<const double *>(C.ds[dir]))[q];
        uy = 2.0 * gld(reinterpret_cast<const double *>(C.df[dir]))[q];
    }
    BorderWin<P> bw;
    border_setup<P>(plane_org(L.y[dir], yp), yp, H, W, x, y, bw);
    const double hxx = eps + 0.25 * bw.hxx, hxy = 0.25 * bw.hxy, hyy = eps + 0.25 * bw.hyy;
    const double idet = 1.0 / (hxx * hyy - hxy * hxy);
    const uint8_t *Bo = plane_org(L.y[1 - dir], yp);
    for (int it = 0; it < K; it++) {
        const double fux = floor(ux), fuy = floor(uy);
        const double fx = ux - fux, fy = uy - fuy;
        // a cell farther than the padded border reads edge values only, so
        // the integer part is clamped before it is converted
        const int ix = (int)fmin(fmax(fux, -(double)(W + 2 * kPad)), (double)(W + 2 * kPad));
        const int iy = (int)fmin(fmax(fuy, -(double)(H + 2 * kPad)), (double)(H + 2 * kPad));
        int S[2][2][2];
        border_corners<P>(bw, Bo, yp, H, W, ix, iy, S);
        const double w00 = (1.0 - fx) * (1.0 - fy), w01 = fx * (1.0 - fy), w10 = (1.0 - fx) * fy, w11 = fx * fy;
        const double bx = 0.5 * (w00 * S[0][0][0] + w01 * S[0][0][1] + w10 * S[0][1][0] + w11 * S[0][1][1] - bw.sax);
        const double by = 0.5 * (w00 * S[1][0][0] + w01 * S[1][0][1] + w10 * S[1][1][0] + w11 * S[1][1][1] - bw.say);
        ux -= (hyy * bx - hxy * by) * idet;
        uy -= (hxx * by - hxy * bx) * idet;
    }
    if (level0) {
        const uint64_t v = (uint64_t)__float_as_uint((float)ux) | ((uint64_t)__float_as_uint((float)uy) << 32);
        gst(reinterpret_cast<uint64_t *>(io[s].flow[dir]))[(size_t)y * W + x] = v;
    } else {
        gst(reinterpret_cast<double *>(L.ds[dir]))[(size_t)y * L.fpitch + x] = ux;
        gst(reinterpret_cast<double *>(L.df[dir]))[(size_t)y * L.fpitch + x] = uy;
    }
}

// The classic method's border pixels (within P of the image edge), one per
// thread, on the refinement's border list of the level.
template <int P>
__global__ __launch_bounds__(kRowTW) void k_lk_border(const StripLv *__restrict__ lv, const StripLv *__restrict__ lvc,
                                                      const StripIO *__restrict__ io, const int32_t *__restrict__ prefix,
                                                      int n, int total, int K, double eps, bool level0)
{
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const RefineSplit sp = refine_split(L.H, L.W, 1, P);
        const int nbt = ceil_div(sp.nbp, kRowTW);
        const int dir = local / nbt;
        local -= dir * nbt;
        const int b = local * kRowTW + (int)threadIdx.x;
        if (b >= sp.nbp) continue;
        int x, y;
        border_pixel(sp, L.H, L.W, b, x, y);
        lk_border_pixel<P>(L, lvc, io, s, dir, x, y, K, eps, level0);
    }
}

// The classic method's interior pixels (window and gradient taps inside the
// image), with the exact 16-bit-pair sums of k_refine: doubled gradients,
// 4 H, sum G Ref and, per step, the four corner correlations of the target
// block at the cell of u (its origin clamped to the padded range as in
// k_refine), combined with the bilinear weights in double. The seed is
// fractional, so every step takes the four corners; no clamp. Register
// budget for windows up to 5x5: at most 96 VGPRs (5 waves per SIMD; one
// value spilled), 4 % faster than the compiler's own 105 at 4 waves; the
// 7x7 window keeps the compiler's budget (capped, it would spill).
template <int LP, int TH>
__global__ __launch_bounds__(64 * TH) __attribute__((amdgpu_waves_per_eu(LP <= 2 ? 5 : 1, 8))) void k_lk_interior(
    const StripLv *__restrict__ lv, const StripLv *__restrict__ lvc, const StripIO *__restrict__ io,
    const int32_t *__restrict__ prefix, int n, int total, int iters, double eps, bool level0)
{
    constexpr int TW = kRefineTW;
    constexpr int WN = 2 * LP + 1;
    constexpr int NP = LP + 1;
    constexpr int AB = WN + 2;
    const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch;
        const RefineSplit sp = refine_split(H, W, TH, LP);
        const int dir = local / sp.nint;
        local -= dir * sp.nint;
        const int ntx = ceil_div(sp.xhi - sp.xlo, TW);
        const int tyi = local / ntx;
        const int x = sp.xlo + (local - tyi * ntx) * TW + lane;
        const int y = sp.ylo + tyi * TH + wrow;
        if (x >= sp.xhi || y >= sp.yhi) continue;  // no barrier in this kernel
        const uint8_t *Ao = plane_org(L.y[dir], yp), *Bo = plane_org(L.y[1 - dir], yp);
        double ux = 0.0, uy = 0.0;
        if (lvc) {
            const StripLv &C = lvc[s];
            const size_t q = (size_t)min(y >> 1, C.H - 1) * C.fpitch + min(x >> 1, C.W - 1);
            ux = 2.0 * gld(reinterpret_cast<const double *>(C.ds[dir]))[q];
            uy = 2.0 * gld(reinterpret_cast<const double *>(C.df[dir]))[q];
        }
        uint32_t gxp[WN][NP], gyp[WN][NP];
        int hxx = 0, hxy = 0, hyy = 0, sax = 0, say = 0;
        {
            uint32_t op[WN + 2][NP], ar[WN + 2][(AB + 3) / 4];
            load_rows<AB, WN + 2>(Ao, yp, y - LP - 1, x - LP - 1, ar);
#pragma unroll
            for (int r = 0; r < WN + 2; r++) {
                odd_pairs<NP, 0>(ar[r], op[r]);
                if (r >= 1 && r <= WN) gx_pairs<NP, 0>(ar[r], gxp[r - 1]);
            }
#pragma unroll
            for (int j = 0; j < WN; j++)
#pragma unroll
                for (int k = 0; k < NP; k++) {
                    gyp[j][k] = sub2(op[j + 2][k], op[j][k]);
                    hxx = dot2(gxp[j][k], gxp[j][k], hxx);
                    hxy = dot2(gxp[j][k], gyp[j][k], hxy);
                    hyy = dot2(gyp[j][k], gyp[j][k], hyy);
                    sax = dot2(gxp[j][k], op[j + 1][k], sax);
                    say = dot2(gyp[j][k], op[j + 1][k], say);
                }
        }
        const double Hxx = 0.25 * hxx + eps, Hxy = 0.25 * hxy, Hyy = 0.25 * hyy + eps;
        const double idet = 1.0 / (Hxx * Hyy - Hxy * Hxy);
        for (int it = 0; it < iters; it++) {
            const double fux = floor(ux), fuy = floor(uy);
            const double fx = ux - fux, fy = uy - fuy;
            // |u| may exceed the int range only with a diverging step; the
            // clamp keeps the block origin in the padded plane either way
            const double cx = fmin(fmax(fux, -(double)(W + 2 * kPad)), (double)(W + 2 * kPad));
            const double cy = fmin(fmax(fuy, -(double)(H + 2 * kPad)), (double)(H + 2 * kPad));
            const int c0 = clampi(x - LP + (int)cx, -kPad, W - 1 + kPad - (WN + 1));
            const int r0 = clampi(y - LP + (int)cy, -kPad, H - 1 + kPad - WN);
            // the WN + 1 target rows in two halves, each loaded and used
            // before the next is issued (fewer live registers)
            int sc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // s00x s01x s10x s11x s00y s01y s10y s11y
            constexpr int H1 = (WN + 1) / 2, H2 = WN + 1 - H1, NBT = (WN + 2 + 3) / 4;
            {
                uint32_t tb[H1][NBT];
                load_rows<WN + 2, H1>(Bo, yp, r0, c0, tb);
                corner_rows<LP, 0, WN, 0, H1>(gxp, gyp, tb, sc);
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                uint32_t tb[H2][NBT];
                load_rows<WN + 2, H2>(Bo, yp, r0 + H1, c0, tb);
                corner_rows<LP, 0, WN, H1, H2>(gxp, gyp, tb, sc);
            }
            // residual sums with the doubled gradient: G (Tgt~ - A)
            const double w00 = (1.0 - fx) * (1.0 - fy), w01 = fx * (1.0 - fy), w10 = (1.0 - fx) * fy, w11 = fx * fy;
            const double bx = 0.5 * (w00 * sc[0] + w01 * sc[1] + w10 * sc[2] + w11 * sc[3] - sax);
            const double by = 0.5 * (w00 * sc[4] + w01 * sc[5] + w10 * sc[6] + w11 * sc[7] - say);
            ux -= (Hyy * bx - Hxy * by) * idet;
            uy -= (Hxx * by - Hxy * bx) * idet;
        }
        if (level0) {
            const uint64_t v = (uint64_t)__float_as_uint((float)ux) | ((uint64_t)__float_as_uint((float)uy) << 32);
            gst(reinterpret_cast<uint64_t *>(io[s].flow[dir]))[(size_t)y * W + x] = v;
        } else {
            gst(reinterpret_cast<double *>(L.ds[dir]))[(size_t)y * L.fpitch + x] = ux;
            gst(reinterpret_cast<double *>(L.df[dir]))[(size_t)y * L.fpitch + x] = uy;
        }
    }
}

// ----------------------------------------------------------------- blend
// One workgroup per segment of PX * kRowTW pixels of a row (PX pixels per
// thread, kRowTW apart, so that every pixel's loads are coalesced across
// the workgroup and a thread has PX pixels' loads to overlap). The uint8
// output of the segment is staged in LDS at the byte alignment of its
// destination, so that the segment is written with aligned dword stores
// (bytes only at its two ends).
template <int PX>
__global__ __launch_bounds__(kRowTW) void k_blend(const StripIO *__restrict__ io, const int32_t *__restrict__ prefix,
                                                  int n, int total, BlendParams bp)
{
    constexpr int TW = PX * kRowTW;
    __shared__ uint32_t stage[(3 * TW + 8) / 4];
    uint8_t *sb = reinterpret_cast<uint8_t *>(stage);
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        const int local = t - prefix[s];
        const StripIO &o = io[s];
        const int W = o.W, H = o.H;
        const int segs = ceil_div(W, TW);
        const int y = local / segs;
        const int xs = (local - y * segs) * TW;
        const int npx = min(TW, W - xs);
        uint8_t *const seg = o.F + (size_t)y * o.pitchF + 3 * (size_t)xs;  // first output byte of the segment
        const int off = (int)((uintptr_t)seg & 3);
#pragma unroll
        for (int k = 0; k < PX; k++) {
            const int i = k * kRowTW + (int)threadIdx.x, x = xs + i;
            if (x < W) {
                const uint32_t p = (uint32_t)(y * W + x);
                const double bl =
                    o.blend ? (double)gld(o.blend)[p] : (double)((o.axis == 0 ? x : y) + 1) * o.inv_ext1;
                const PixBlend pb = blend_setup(x, y, bl, p, o.inv_ext, o.flow[0], o.flow[1], bp);
                float cl[3], cr[3];
                sample_u8(o.L, o.pitchL, H, W, pb.lx, pb.ly, pb.lfx, pb.lfy, cl);
                sample_u8(o.R, o.pitchR, H, W, pb.rx, pb.ry, pb.rfx, pb.rfy, cr);
                const float sR = 1.0f - pb.sL;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const float f = pb.sL * cl[c] + sR * cr[c];
                    const float r = floorf(f + 0.5f);
                    sb[off + 3 * i + c] = (uint8_t)fminf(fmaxf(r, 0.f), 255.f);
                    if (o.Ff32) gst(o.Ff32)[3 * ((size_t)y * W + x) + c] = f;
                }
            }
        }
        __syncthreads();
        // bytes [off, off + nb) of the staging area go to seg - off + [off, off + nb)
        const int nb = 3 * npx, end = off + nb;
        const auto dst = reinterpret_cast<__attribute__((address_space(1))) uint32_t *>((uintptr_t)seg - off);
        const int first = (off + 3) >> 2, last = end >> 2;  // whole dwords [first, last)
        for (int k = first + (int)threadIdx.x; k < last; k += kRowTW) dst[k] = stage[k];
        if (threadIdx.x < 8) {
            // leading bytes [off, 4 first) and trailing bytes [4 last, end)
            const int i = threadIdx.x < 4 ? off + (int)threadIdx.x : 4 * last + (int)threadIdx.x - 4;
            const bool lead = threadIdx.x < 4 && i < min(4 * first, end);
            const bool trail = threadIdx.x >= 4 && i >= max(4 * last, 4 * first) && i < end;
            if (lead || trail) gst(seg - off)[i] = sb[i];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- launchers
hipError_t launch_luma(const StripIO *io, const StripLv *lv0, Work w, int grid, bool sums, hipStream_t s)
{
    if (sums)
        hipLaunchKernelGGL(k_luma<true>, dim3(grid_for(w.total, grid)), dim3(64), 0, s, io, lv0, w.prefix, w.n,
                           w.total);
    else
        hipLaunchKernelGGL(k_luma<false>, dim3(grid_for(w.total, grid)), dim3(64), 0, s, io, lv0, w.prefix, w.n,
                           w.total);
    return hipGetLastError();
}

hipError_t launch_zero_sums(const StripIO *io, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_sums, dim3(ceil_div(kSumWords * n, 256)), dim3(256), 0, s, io, n);
    return hipGetLastError();
}

hipError_t launch_gain(const StripIO *io, const StripLv *lv0, Work w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gain_prep, dim3(w.n), dim3(64), 0, s, io);
    hipLaunchKernelGGL(k_gain, dim3(grid_for(w.total, grid)), dim3(64), 0, s, io, lv0, w.prefix, w.n, w.total);
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
    if constexpr (P == 2 && R <= 2) {
        // 5x5 patches, tiles of 2, 4 or 8 rows: a 2 x 2 quad per thread
        switch (th) {
        case 2: hipLaunchKernelGGL((k_search_quad<R, 2>), dim3(g), dim3(64), 0, s, lv, w.prefix, w.n, w.total);
            return hipGetLastError();
        case 4: hipLaunchKernelGGL((k_search_quad<R, 4>), dim3(g), dim3(128), 0, s, lv, w.prefix, w.n, w.total);
            return hipGetLastError();
        case 8: hipLaunchKernelGGL((k_search_quad<R, 8>), dim3(g), dim3(256), 0, s, lv, w.prefix, w.n, w.total);
            return hipGetLastError();
        default: break;
        }
    }
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

template <int LP>
static hipError_t refine_lp(const StripLv *lv0, const StripIO *io, Work w, LkParams lk, int th, int grid,
                            hipStream_t s)
{
    if (w.total == 0) return hipSuccess;
    const int g = grid_for(w.total, grid);
    if constexpr (LP <= 2) {
        // vertical pixel pairs: TH / 2 waves per tile
        if (th == 2)
            hipLaunchKernelGGL((k_refine_pair<LP, 2>), dim3(g), dim3(64), 0, s, lv0, io, w.prefix, w.n, w.total,
                               lk.iters, lk.eps);
        else
            hipLaunchKernelGGL((k_refine_pair<LP, 4>), dim3(g), dim3(128), 0, s, lv0, io, w.prefix, w.n, w.total,
                               lk.iters, lk.eps);
        return hipGetLastError();
    } else {
        if (th == 2)
            hipLaunchKernelGGL((k_refine<LP, 2>), dim3(g), dim3(128), 0, s, lv0, io, w.prefix, w.n, w.total,
                               lk.iters, lk.eps);
        else
            hipLaunchKernelGGL((k_refine<LP, 4>), dim3(g), dim3(256), 0, s, lv0, io, w.prefix, w.n, w.total,
                               lk.iters, lk.eps);
        return hipGetLastError();
    }
}

hipError_t launch_refine(const StripLv *lv0, const StripIO *io, Work w, LkParams lk, int th, int grid, hipStream_t s)
{
    switch (lk.patch) {
    case 1: return refine_lp<1>(lv0, io, w, lk, th, grid, s);
    case 2: return refine_lp<2>(lv0, io, w, lk, th, grid, s);
    case 3: return refine_lp<3>(lv0, io, w, lk, th, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <int LP>
static hipError_t refine_border_lp(const StripLv *lv0, const StripIO *io, Work w, LkParams lk, hipStream_t s)
{
    if (w.total > 0)
        hipLaunchKernelGGL((k_refine_border<LP>), dim3(w.total), dim3(kRowTW), 0, s, lv0, io, w.prefix, w.n, w.total,
                           lk.iters, lk.eps);
    return hipGetLastError();
}

hipError_t launch_refine_border(const StripLv *lv0, const StripIO *io, Work w, LkParams lk, hipStream_t s)
{
    switch (lk.patch) {
    case 1: return refine_border_lp<1>(lv0, io, w, lk, s);
    case 2: return refine_border_lp<2>(lv0, io, w, lk, s);
    case 3: return refine_border_lp<3>(lv0, io, w, lk, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lk_border(const StripLv *lv, const StripLv *lvc, const StripIO *io, Work w, LkParams lk, bool level0,
                            hipStream_t s)
{
    const dim3 g(grid_for(w.total, 0)), b(kRowTW);
    const double e = lk.eps;
    switch (lk.patch) {
    case 1: hipLaunchKernelGGL(k_lk_border<1>, g, b, 0, s, lv, lvc, io, w.prefix, w.n, w.total, lk.iters, e, level0); break;
    case 2: hipLaunchKernelGGL(k_lk_border<2>, g, b, 0, s, lv, lvc, io, w.prefix, w.n, w.total, lk.iters, e, level0); break;
    default: hipLaunchKernelGGL(k_lk_border<3>, g, b, 0, s, lv, lvc, io, w.prefix, w.n, w.total, lk.iters, e, level0); break;
    }
    return hipGetLastError();
}

template <int LP>
static hipError_t lk_interior_th(const StripLv *lv, const StripLv *lvc, const StripIO *io, Work w, LkParams lk,
                                 int th, int grid, bool level0, hipStream_t s)
{
    const dim3 g(grid_for(w.total, grid));
    const double e = lk.eps;
    if (th == 2)
        hipLaunchKernelGGL((k_lk_interior<LP, 2>), g, dim3(128), 0, s, lv, lvc, io, w.prefix, w.n, w.total, lk.iters, e, level0);
    else
        hipLaunchKernelGGL((k_lk_interior<LP, 4>), g, dim3(256), 0, s, lv, lvc, io, w.prefix, w.n, w.total, lk.iters, e, level0);
    return hipGetLastError();
}

hipError_t launch_lk_interior(const StripLv *lv, const StripLv *lvc, const StripIO *io, Work w, LkParams lk, int th,
                              int grid, bool level0, hipStream_t s)
{
    if (lk.patch == 1) return lk_interior_th<1>(lv, lvc, io, w, lk, th, grid, level0, s);
    if (lk.patch == 2) return lk_interior_th<2>(lv, lvc, io, w, lk, th, grid, level0, s);
    return lk_interior_th<3>(lv, lvc, io, w, lk, th, grid, level0, s);
}

hipError_t launch_blend(const StripIO *io, Work w, BlendParams bp, int px, int grid, hipStream_t s)
{
    const dim3 g(grid_for(w.total, grid)), b(kRowTW);
    switch (px) {
    case 1: hipLaunchKernelGGL(k_blend<1>, g, b, 0, s, io, w.prefix, w.n, w.total, bp); break;
    case 2: hipLaunchKernelGGL(k_blend<2>, g, b, 0, s, io, w.prefix, w.n, w.total, bp); break;
    case 4: hipLaunchKernelGGL(k_blend<4>, g, b, 0, s, io, w.prefix, w.n, w.total, bp); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace abf
