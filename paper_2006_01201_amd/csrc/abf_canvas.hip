// HIP kernels of libabf for canvas compositing (gfx950): eq. (1) of Meng &
// Liu (arXiv 2006.01201, Section III.C.2) on a canvas whose Area1 (only L),
// Area2 (only R) and Area3 (both) have any shape, and Code 1 (Section
// III.C.3) with its Area1 / Area2 / else branches.
//
// eq. (1) needs, for every Area3 pixel, the Euclidean distances Lmin /
// Rmin to the nearest Area1 / Area2 pixel. They are computed exactly, as
// integer squared distances, in two passes that both keep the 64 lanes of a
// wave on 64 consecutive columns of one row (coalesced):
//   1. rows: g(x, y) = distance along row y to the nearest pixel of the
//      area (one workgroup per row; 16-pixel chunks, a workgroup scan of
//      the chunks' first/last members carries the nearest one across
//      chunks). Both areas are kept as a uint16 pair per pixel, and a
//      second kernel stores the minimum of g over every 16-row block of a
//      column.
//   2. columns: D(x, y) = min over rows y' of (y - y')^2 + g(x, y')^2,
//      searched outward from y, a 16-row block at a time. A block whose
//      nearest row is k rows away and whose minimum g is m cannot beat
//      k^2 + m^2, so it is skipped when that bound reaches the best value
//      found, and the search ends in a direction once k^2 does.
#include "abf_device.h"
#include "abf_tiles.h"

namespace abf {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kInf16 = 0xffffu;
constexpr uint32_t kInf32 = 0xffffffffu;

// squared distance of a row candidate k rows away with row distance g
// (kInf32 if the row holds no pixel of the area)
__device__ __forceinline__ uint32_t cand(uint32_t k2, uint32_t g)
{
    return g == kInf16 ? kInf32 : k2 + g * g;
}

// Nonzero bytes of row[x0 .. x0 + n) (n <= 16) as a bit mask (bit k = byte
// x0 + k): four aligned dword loads when the 16 bytes are whole and
// 4-byte aligned, else byte by byte.
__device__ __forceinline__ uint32_t chunk_nz(const uint8_t *row, int x0, int n)
{
    const uint8_t *p = row + x0;
    if (n == kCanvasChunk && ((uintptr_t)p & 3) == 0) {
        const auto q = gld(reinterpret_cast<const uint32_t *>(p));
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t v = q[j];
            // high bit of each byte set iff the byte is nonzero
            const uint32_t h = (((v & 0x7f7f7f7fu) + 0x7f7f7f7fu) | v) & 0x80808080u;
            m |= (((h >> 7) & 1u) | ((h >> 14) & 2u) | ((h >> 21) & 4u) | ((h >> 28) & 8u)) << (4 * j);
        }
        return m;
    }
    uint32_t m = 0;
    for (int k = 0; k < n; k++) m |= (uint32_t)(gld(p)[k] != 0) << k;
    return m;
}

// ------------------------------------------------------------ row pass
// One workgroup per canvas row. Chunk c covers columns [16 c, 16 c + 16).
__global__ __launch_bounds__(kCanvasThreads) void k_canvas_rows(CanvasGeom a)
{
    __shared__ int32_t lastA[kCanvasMaxChunks], lastB[kCanvasMaxChunks];
    __shared__ int32_t firstA[kCanvasMaxChunks], firstB[kCanvasMaxChunks];
    __shared__ uint32_t bits[kCanvasMaxChunks];
    __shared__ int32_t tot[4][kCanvasThreads];
    const int y = blockIdx.x, t = threadIdx.x;
    const int W = a.W, nC = ceil_div(W, kCanvasChunk);
    const uint8_t *rl = a.mL + (size_t)y * a.pitchM;
    const uint8_t *rr = a.mR + (size_t)y * a.pitchM;
    constexpr int INF = 0x7fffffff;
    for (int c = t; c < nC; c += kCanvasThreads) {
        const int x0 = c * kCanvasChunk, n = min(kCanvasChunk, W - x0);
        const uint32_t ml = chunk_nz(rl, x0, n), mr = chunk_nz(rr, x0, n);
        const uint32_t b1 = ml & ~mr, b2 = mr & ~ml;
        bits[c] = b1 | (b2 << 16);
        lastA[c] = b1 ? x0 + 31 - __clz(b1) : -1;
        lastB[c] = b2 ? x0 + 31 - __clz(b2) : -1;
        firstA[c] = b1 ? x0 + __ffs(b1) - 1 : INF;
        firstB[c] = b2 ? x0 + __ffs(b2) - 1 : INF;
    }
    __syncthreads();
    // thread t owns chunks [per t, per t + per) for the scan
    const int per = ceil_div(nC, kCanvasThreads), c0 = t * per;
    int la = -1, lb = -1, fa = INF, fb = INF;
    for (int i = 0; i < per; i++) {
        const int c = c0 + i;
        if (c < nC) {
            la = max(la, lastA[c]);
            lb = max(lb, lastB[c]);
            fa = min(fa, firstA[c]);
            fb = min(fb, firstB[c]);
        }
    }
    tot[0][t] = la;
    tot[1][t] = lb;
    tot[2][t] = fa;
    tot[3][t] = fb;
    __syncthreads();
    // inclusive prefix max from the left (last members) and suffix min
    // from the right (first members) over the threads
    for (int d = 1; d < kCanvasThreads; d <<= 1) {
        int v0 = tot[0][t], v1 = tot[1][t], v2 = tot[2][t], v3 = tot[3][t];
        if (t >= d) {
            v0 = max(v0, tot[0][t - d]);
            v1 = max(v1, tot[1][t - d]);
        }
        if (t + d < kCanvasThreads) {
            v2 = min(v2, tot[2][t + d]);
            v3 = min(v3, tot[3][t + d]);
        }
        __syncthreads();
        tot[0][t] = v0;
        tot[1][t] = v1;
        tot[2][t] = v2;
        tot[3][t] = v3;
        __syncthreads();
    }
    // the row's last and first members of each area: on a periodic canvas a
    // pixel with no member on one side reaches the other end's across the
    // wrap
    const int endA = tot[0][kCanvasThreads - 1], endB = tot[1][kCanvasThreads - 1];
    const int begA = tot[2][0], begB = tot[3][0];
    const bool wrap = a.periodic != 0;
    // exclusive carries per owned chunk, in place (each entry is read and
    // written by its owner only)
    int ca = t > 0 ? tot[0][t - 1] : -1, cb = t > 0 ? tot[1][t - 1] : -1;
    for (int i = 0; i < per; i++) {
        const int c = c0 + i;
        if (c < nC) {
            const int va = lastA[c], vb = lastB[c];
            lastA[c] = ca;
            lastB[c] = cb;
            ca = max(ca, va);
            cb = max(cb, vb);
        }
    }
    int ra = t + 1 < kCanvasThreads ? tot[2][t + 1] : INF, rb = t + 1 < kCanvasThreads ? tot[3][t + 1] : INF;
    for (int i = per - 1; i >= 0; i--) {
        const int c = c0 + i;
        if (c < nC) {
            const int va = firstA[c], vb = firstB[c];
            firstA[c] = ra;
            firstB[c] = rb;
            ra = min(ra, va);
            rb = min(rb, vb);
        }
    }
    __syncthreads();
    uint32_t *const orow = a.G + (size_t)y * a.gpitch;
    const int cend = min(nC, ceil_div(a.gx1, kCanvasChunk));
    for (int c = a.gx0 / kCanvasChunk + t; c < cend; c += kCanvasThreads) {
        const uint32_t bb = bits[c];
        const int x0 = c * kCanvasChunk, n = min(kCanvasChunk, W - x0);
        int l1 = lastA[c], l2 = lastB[c], r1 = firstA[c], r2 = firstB[c];
        uint32_t d[kCanvasChunk];
#pragma unroll
        for (int k = 0; k < kCanvasChunk; k++) {
            const int x = x0 + k;
            if ((bb >> k) & 1u) l1 = x;
            if ((bb >> (16 + k)) & 1u) l2 = x;
            const uint32_t e1 = l1 >= 0 ? (uint32_t)(x - l1) : (wrap && endA >= 0 ? (uint32_t)(x + W - endA) : kInf16);
            const uint32_t e2 = l2 >= 0 ? (uint32_t)(x - l2) : (wrap && endB >= 0 ? (uint32_t)(x + W - endB) : kInf16);
            d[k] = e1 | (e2 << 16);
        }
#pragma unroll
        for (int k = kCanvasChunk - 1; k >= 0; k--) {
            const int x = x0 + k;
            if ((bb >> k) & 1u) r1 = x;
            if ((bb >> (16 + k)) & 1u) r2 = x;
            const uint32_t e1 = r1 != INF ? (uint32_t)(r1 - x) : (wrap && begA != INF ? (uint32_t)(W - x + begA) : kInf16);
            const uint32_t e2 = r2 != INF ? (uint32_t)(r2 - x) : (wrap && begB != INF ? (uint32_t)(W - x + begB) : kInf16);
            d[k] = min(d[k] & 0xffffu, e1) | (min(d[k] >> 16, e2) << 16);
        }
        if (n == kCanvasChunk) {
            auto q = gst(reinterpret_cast<u32x4 *>(orow + x0));
#pragma unroll
            for (int j = 0; j < kCanvasChunk / 4; j++) q[j] = u32x4{d[4 * j], d[4 * j + 1], d[4 * j + 2], d[4 * j + 3]};
        } else {
#pragma unroll
            for (int k = 0; k < kCanvasChunk; k++)
                if (k < n) gst(orow)[x0 + k] = d[k];
        }
    }
}

// Minimum of g over each block of kCanvasBH rows of a column, per area.
__global__ __launch_bounds__(kCanvasThreads) void k_canvas_colmin(CanvasGeom a, int x0)
{
    const int x = x0 + blockIdx.x * kCanvasThreads + threadIdx.x, b = blockIdx.y;
    if (x >= a.W) return;
    const int r0 = b * kCanvasBH, r1 = min(r0 + kCanvasBH, a.H);
    uint32_t m1 = kInf16, m2 = kInf16;
    for (int r = r0; r < r1; r++) {
        const uint32_t g = gld(a.G)[(size_t)r * a.gpitch + x];
        m1 = min(m1, g & 0xffffu);
        m2 = min(m2, g >> 16);
    }
    gst(a.M)[(size_t)b * a.gpitch + x] = m1 | (m2 << 16);
}

// ------------------------------------------------------- column search
// One workgroup per 64 columns of one kCanvasBH-row block (the tile; wave
// w holds tile rows w, w + 4, w + 8, w + 12). The tile's own rows, then
// the blocks above and below at increasing distance, are staged in LDS
// (one coalesced 4 KiB load each) and every pixel of the tile takes its
// candidates from there, so the rows that neighbouring pixels share are
// read from memory once per tile. Block minima are examined kWin blocks
// per direction at a time: a block j blocks away is at least 16 j - 15
// rows from every row of the tile, so it is staged only if, for some
// column and area, that distance squared plus the block minimum squared
// is below the largest best value of the column's tile pixels; a
// direction ends once that distance squared reaches the largest best value
// of the tile. Squared distances saturate at 0xffffffff (no pixel of the
// area seen yet); pixels whose distances are not needed start at 0.
constexpr int kTileQ = kCanvasBH / 4;  // pixels (rows) per lane
constexpr int kWin = 8;                // blocks examined per direction at a time

__device__ __forceinline__ uint32_t sqg(uint32_t g) { return g == kInf16 ? kInf32 : g * g; }
__device__ __forceinline__ uint32_t adds(uint32_t a, uint32_t b) { return __builtin_elementwise_add_sat(a, b); }

// candidates of the lane's tile pixels (rows yq[q]) from the staged rows
// r0 .. r0 + kCanvasBH - 1 of its column. With `m` (the block's minima of
// the column) a pixel skips the block when its nearest row (dk rows away)
// and those minima cannot beat its best values.
__device__ __forceinline__ void eval_rows(const uint32_t (*rows)[64], int lane, int r0, const int (&yq)[kTileQ],
                                          uint32_t (&b1)[kTileQ], uint32_t (&b2)[kTileQ], bool bounded = false,
                                          uint32_t m = 0)
{
    const uint32_t ms1 = sqg(m & 0xffffu), ms2 = sqg(m >> 16);
#pragma unroll
    for (int q = 0; q < kTileQ; q++) {
        if (bounded) {
            const int dk = yq[q] < r0 ? r0 - yq[q] : yq[q] - (r0 + kCanvasBH - 1);
            const uint32_t dk2 = (uint32_t)(dk * dk);
            if (!(adds(dk2, ms1) < b1[q] || adds(dk2, ms2) < b2[q])) continue;
        }
#pragma unroll
        for (int rr = 0; rr < kCanvasBH; rr++) {
            const uint32_t g = rows[rr][lane];
            const int k = yq[q] - (r0 + rr);
            const uint32_t k2 = (uint32_t)(k * k);
            b1[q] = min(b1[q], adds(k2, sqg(g & 0xffffu)));
            b2[q] = min(b2[q], adds(k2, sqg(g >> 16)));
        }
    }
}

__global__ __launch_bounds__(256) void k_canvas_dist(CanvasGeom a, float *blend, int pitchB, int32_t *d1, int32_t *d2,
                                                     int pitchD, int tx0, int tb0)
{
    __shared__ uint32_t own[kCanvasBH][64];
    __shared__ uint32_t nbr[2][kCanvasBH][64];  // staged block above / below
    __shared__ uint32_t nbm[2][64];             // and its block minima
    __shared__ uint32_t flags[2][4];            // by window parity: a window may end without a barrier
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = (tx0 + (int)blockIdx.x) * 64 + lane, b0 = tb0 + (int)blockIdx.y, y0 = b0 * kCanvasBH;
    const int H = a.H, nb = ceil_div(H, kCanvasBH);
    const bool inx = x < a.W;
    const bool all = d1 != nullptr;
    auto stage = [&](uint32_t (*dst)[64], int b) {
#pragma unroll
        for (int q = 0; q < kTileQ; q++) {
            const int i = w + 4 * q, r = b * kCanvasBH + i;
            dst[i][lane] = inx && r < H ? gld(a.G)[(size_t)r * a.gpitch + x] : kInf32;
        }
    };
    stage(own, b0);
    int area[kTileQ], yq[kTileQ];
    uint32_t best1[kTileQ], best2[kTileQ];
#pragma unroll
    for (int q = 0; q < kTileQ; q++) {
        const int y = y0 + w + 4 * q;
        const bool in = inx && y < H;
        yq[q] = y;
        area[q] = in ? (gld(a.mL)[(size_t)y * a.pitchM + x] != 0) + 2 * (gld(a.mR)[(size_t)y * a.pitchM + x] != 0) : 0;
        best1[q] = best2[q] = in && (all || area[q] == 3) ? kInf32 : 0u;
    }
    __syncthreads();
    eval_rows(own, lane, y0, yq, best1, best2);
    bool up = b0 > 0, down = b0 + 1 < nb;
    for (int j0 = 1; up || down; j0 += kWin) {
        uint32_t m1 = 0, m2 = 0;
#pragma unroll
        for (int q = 0; q < kTileQ; q++) {
            m1 = max(m1, best1[q]);
            m2 = max(m2, best2[q]);
        }
        const uint32_t mm = max(m1, m2);
        uint32_t f = 0;
#pragma unroll
        for (int t = 0; t < kWin; t++) {
            const int bu = b0 - j0 - t, bd = b0 + j0 + t;
            const uint32_t dk = (uint32_t)(16 * (j0 + t) - 15), dk2 = dk * dk;
            const uint32_t mu = up && inx && bu >= 0 ? gld(a.M)[(size_t)bu * a.gpitch + x] : kInf32;
            const uint32_t md = down && inx && bd < nb ? gld(a.M)[(size_t)bd * a.gpitch + x] : kInf32;
            f |= (adds(dk2, sqg(mu & 0xffffu)) < m1 || adds(dk2, sqg(mu >> 16)) < m2) ? 1u << t : 0u;
            f |= (adds(dk2, sqg(md & 0xffffu)) < m1 || adds(dk2, sqg(md >> 16)) < m2) ? 1u << (kWin + t) : 0u;
        }
        const uint32_t dn = (uint32_t)(16 * (j0 + kWin) - 15);
        f |= dn * dn < mm ? 3u << (2 * kWin) : 0u;
        // OR over the wave, then over the workgroup
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) f |= (uint32_t)__shfl_xor((int)f, o);
        const int par = (j0 / kWin) & 1;
        if (lane == 0) flags[par][w] = f;
        __syncthreads();
        const uint32_t F = flags[par][0] | flags[par][1] | flags[par][2] | flags[par][3];
        for (int t = 0; t < kWin; t++) {
            const bool su = up && ((F >> t) & 1u), sd = down && ((F >> (kWin + t)) & 1u);
            if (!su && !sd) continue;  // workgroup-uniform
            const int bu = b0 - j0 - t, bd = b0 + j0 + t;
            if (su) stage(nbr[0], bu);
            if (sd) stage(nbr[1], bd);
            if (w == 0 && su) nbm[0][lane] = inx ? gld(a.M)[(size_t)bu * a.gpitch + x] : kInf32;
            if (w == 1 && sd) nbm[1][lane] = inx ? gld(a.M)[(size_t)bd * a.gpitch + x] : kInf32;
            __syncthreads();
            if (su) eval_rows(nbr[0], lane, bu * kCanvasBH, yq, best1, best2, true, nbm[0][lane]);
            if (sd) eval_rows(nbr[1], lane, bd * kCanvasBH, yq, best1, best2, true, nbm[1][lane]);
            __syncthreads();
        }
        up = up && b0 - j0 - kWin >= 0 && ((F >> (2 * kWin)) & 1u);
        down = down && b0 + j0 + kWin < nb && ((F >> (2 * kWin)) & 1u);
    }
#pragma unroll
    for (int q = 0; q < kTileQ; q++) {
        const int y = yq[q];
        if (!inx || y >= H) continue;
        const uint32_t e1 = best1[q], e2 = best2[q];
        if (blend) {
            float t;
            if (area[q] == 1) t = 0.f;
            else if (area[q] == 2) t = 1.f;
            else if (area[q] == 0) t = 0.5f;
            else if (e1 == kInf32 && e2 == kInf32) t = 0.5f;
            else if (e1 == kInf32) t = 1.f;
            else if (e2 == kInf32) t = 0.f;
            else {
                const double l = sqrt((double)e1), r = sqrt((double)e2);
                t = (float)(l / (l + r));
            }
            gst(blend)[(size_t)y * pitchB + x] = t;
        }
        if (all) {
            gst(d1)[(size_t)y * pitchD + x] = e1 == kInf32 ? -1 : (int32_t)e1;
            gst(d2)[(size_t)y * pitchD + x] = e2 == kInf32 ? -1 : (int32_t)e2;
        }
    }
}

// ------------------------------------------------------------ overlap box
// One workgroup per row: the extent {x0, x1} of the row's Area3 pixels
// ({INT_MAX, -1} if none) into part[2 y], part[2 y + 1]. Each thread reads 16 consecutive
// columns of both masks with all loads in flight at once. With `occ` (a
// periodic canvas) the first workgroup also clears the nw column-occupancy
// words that k_box_cols then fills.
__global__ __launch_bounds__(kCanvasThreads) void k_box_rows(const uint8_t *mL, const uint8_t *mR, int pitchM, int W,
                                                             int32_t *part, uint32_t *occ, int nw)
{
    __shared__ int32_t s[2];
    const int y = blockIdx.x;
    if (occ && y == 0)
        for (int i = threadIdx.x; i < nw; i += kCanvasThreads) gst(occ)[i] = 0u;
    if (threadIdx.x == 0) {
        s[0] = 0x7fffffff;
        s[1] = -1;
    }
    __syncthreads();
    const uint8_t *rl = mL + (size_t)y * pitchM, *rr = mR + (size_t)y * pitchM;
    int lo = 0x7fffffff, hi = -1;
    for (int x0 = kCanvasChunk * (int)threadIdx.x; x0 < W; x0 += kCanvasChunk * kCanvasThreads) {
        const int n = min(kCanvasChunk, W - x0);
        const uint32_t m = chunk_nz(rl, x0, n) & chunk_nz(rr, x0, n);
        if (m) {
            lo = min(lo, x0 + __ffs(m) - 1);
            hi = max(hi, x0 + 31 - __clz(m));
        }
    }
    if (hi >= 0) {
        atomicMin(&s[0], lo);
        atomicMax(&s[1], hi);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        gst(part)[2 * y] = s[0];
        gst(part)[2 * y + 1] = s[1];
    }
}

// Column occupancy of a periodic canvas: bit x of occ is set iff column x
// holds an Area3 pixel. A thread takes one 16-column chunk over a band of
// kBoxBand rows (grid: chunks x bands) and ORs the chunk's Area3 bits of
// those rows into its occupancy word (cleared by k_box_rows).
constexpr int kBoxBand = 8;
__global__ __launch_bounds__(256) void k_box_cols(const uint8_t *mL, const uint8_t *mR, int pitchM, int H, int W,
                                                  uint32_t *occ)
{
    const int x0 = (blockIdx.x * 256 + (int)threadIdx.x) * kCanvasChunk;
    if (x0 >= W) return;
    const int n = min(kCanvasChunk, W - x0);
    const int y0 = blockIdx.y * kBoxBand, y1 = min(H, y0 + kBoxBand);
    uint32_t m = 0;
    for (int y = y0; y < y1; y++) {
        const size_t r = (size_t)y * pitchM;
        m |= chunk_nz(mL + r, x0, n) & chunk_nz(mR + r, x0, n);
    }
    static_assert(32 % kCanvasChunk == 0, "a chunk lies in one occupancy word");
    if (m) atomicOr(occ + (x0 >> 5), m << (x0 & 31));
}

// Zero runs of one occupancy word (bits [0, vb) valid, column base): the
// zeros before its first set bit (pz) and after its last (sz), and its
// longest run strictly between two set bits (length il, first column is; of
// equally long runs the first).
struct OccWord {
    int pz, sz, il, is;
};
__device__ __forceinline__ OccWord occ_word(uint32_t w, int vb, int base)
{
    OccWord r{vb, vb, 0, -1};
    if (w == 0) return r;
    r.pz = __builtin_ctz(w);
    r.sz = vb - 1 - (31 - __builtin_clz(w));
    int i = r.pz;
    uint32_t rest = w & (w - 1);
    while (rest) {
        const int j = __builtin_ctz(rest);
        if (j - i - 1 > r.il) {
            r.il = j - i - 1;
            r.is = base + i + 1;
        }
        i = j;
        rest &= rest - 1;
    }
    return r;
}

// Merge of the row extents into {x, y, w, h} (zeros when no row has an
// Area3 pixel); one workgroup. With `occ` (a periodic canvas) the columns
// are the shortest circular run that holds every Area3 column: it starts
// right after the longest run of columns without one (of several, the one
// that starts at the smallest column), and w = W minus that run's length.
__global__ __launch_bounds__(1024) void k_box_fin(const int32_t *part, int H, int W, const uint32_t *occ,
                                                  int32_t *box)
{
    __shared__ int32_t red[4 * 16];
    __shared__ OccWord ow[(kCanvasMaxDim + 31) / 32 + 1];
    int x0 = 0x7fffffff, y0 = 0x7fffffff, x1 = -1, y1 = -1;
    for (int y = threadIdx.x; y < H; y += blockDim.x) {
        const int32_t ex = gld(part)[2 * y], ey = gld(part)[2 * y + 1];
        if (ey >= 0) {
            x0 = min(x0, ex);
            x1 = max(x1, ey);
            y0 = min(y0, y);
            y1 = max(y1, y);
        }
    }
    wg_minmax4<1024>(x0, y0, x1, y1, red);  // over the workgroup (every thread gets the result)
    const int s[4] = {x0, y0, x1, y1};
    const int nw = (W + 31) >> 5;
    if (occ)
        for (int k = threadIdx.x; k < nw; k += blockDim.x)
            ow[k] = occ_word(gld(occ)[k], k + 1 < nw ? 32 : W - 32 * k, 32 * k);
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool e = s[2] < 0;
        int bx = s[0], bw = s[2] - s[0] + 1;
        if (occ && !e) {
            // s[0] and s[2] are the first and last Area3 columns; the run
            // that wraps past W - 1 is weighed first when it starts at
            // column 0 (it holds column 0 only), last otherwise
            const int first = s[0], last = s[2];
            int best_len = last == W - 1 ? first : 0, best_s = 0;
            int prev = -1;  // last Area3 column seen
            for (int k = 0; k < nw; k++) {
                const OccWord o = ow[k];
                const int vb = k + 1 < nw ? 32 : W - 32 * k;
                if (o.pz == vb) continue;  // no Area3 column in the word
                const int f = 32 * k + o.pz;
                if (prev >= 0 && f - prev - 1 > best_len) {
                    best_len = f - prev - 1;
                    best_s = prev + 1;
                }
                if (o.il > best_len) {
                    best_len = o.il;
                    best_s = o.is;
                }
                prev = 32 * k + vb - 1 - o.sz;
            }
            if (last < W - 1 && W - 1 - last + first > best_len) {
                best_len = W - 1 - last + first;
                best_s = last + 1;
            }
            bx = best_len == 0 ? 0 : (best_s + best_len) % W;
            bw = W - best_len;
        }
        gst(box)[0] = e ? 0 : bx;
        gst(box)[1] = e ? 0 : s[1];
        gst(box)[2] = e ? 0 : bw;
        gst(box)[3] = e ? 0 : s[3] - s[1] + 1;
    }
}

// ------------------------------------------------------------- composite
// Bilinear RGB sample at (x0 + fx, y0 + fy) of the box crop of a canvas
// image whose box wraps past column W - 1: crop coordinates are clamped to
// the crop, crop column c is canvas column bx + c modulo W. Byte loads.
__device__ __forceinline__ void sample_box_wrap(const uint8_t *img, int pitch, int W, int bx, int by, int bw, int bh,
                                                int x0, int y0, float fx, float fy, float out[3])
{
    int c0 = bx + clampi(x0, 0, bw - 1), c1 = bx + clampi(x0 + 1, 0, bw - 1);
    if (c0 >= W) c0 -= W;
    if (c1 >= W) c1 -= W;
    const uint8_t *ra = img + (size_t)(by + clampi(y0, 0, bh - 1)) * pitch;
    const uint8_t *rb = img + (size_t)(by + clampi(y0 + 1, 0, bh - 1)) * pitch;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const float a0 = gld(ra)[3 * c0 + c], a1 = gld(ra)[3 * c1 + c];
        const float b0 = gld(rb)[3 * c0 + c], b1 = gld(rb)[3 * c1 + c];
        const float top = a0 + fx * (a1 - a0);
        const float bot = b0 + fx * (b1 - b0);
        out[c] = top + fy * (bot - top);
    }
}

// Code 1 over the canvas, one workgroup per PX kRowTW pixels of a row: Area1
// copies L, Area2 copies R, Area3 inside the overlap box is warped and
// blended as a strip pixel of the box (images and flows cropped to the
// box), everything else is 0. With `cov` (a photo merge), the union of the
// two coverages is written there (pitch of the masks). The uint8 output is staged in LDS at the
// byte alignment of its destination and written with aligned dwords.
template <int PX>
__global__ __launch_bounds__(kRowTW) void k_composite(CompositeArgs o, BlendParams bp)
{
    constexpr int TW = PX * kRowTW;  // pixels of a row segment; a thread takes PX of them, kRowTW apart
    __shared__ uint32_t stage[(3 * TW + 8) / 4];
    uint8_t *sb = reinterpret_cast<uint8_t *>(stage);
    const int W = o.W, segs = ceil_div(W, TW);
    const int y = blockIdx.x / segs, xs = (blockIdx.x - y * segs) * TW;
    const int npx = min(TW, W - xs);
    uint8_t *const seg = o.F + (size_t)y * o.pitchF + 3 * (size_t)xs;
    const int off = (int)((uintptr_t)seg & 3);
    const int yb = y - o.by;
#pragma unroll
    for (int k = 0; k < PX; k++) {
        const int i = k * kRowTW + (int)threadIdx.x, x = xs + i;
        if (x >= W) break;
        const size_t pm = (size_t)y * o.pitchM + x;
        const int area = (gld(o.mL)[pm] != 0) + 2 * (gld(o.mR)[pm] != 0);
        if (o.cov) gst(o.cov)[pm] = area != 0;  // may be one of the masks: read above, by this thread only
        int xb = x - o.bx;
        if (o.periodic && xb < 0) xb += W;  // box columns wrap modulo W
        float f[3] = {0.f, 0.f, 0.f};
        if (area == 1 || area == 2) {
            const uint8_t *src = area == 1 ? o.L + (size_t)y * o.pitchL : o.R + (size_t)y * o.pitchR;
#pragma unroll
            for (int c = 0; c < 3; c++) f[c] = (float)gld(src)[3 * x + c];
        } else if (area == 3 && xb >= 0 && xb < o.bw && yb >= 0 && yb < o.bh) {
            const uint32_t p = (uint32_t)(yb * o.bw + xb);
            const double t = (double)gld(o.blend)[(size_t)y * o.pitchB + x];
            const PixBlend pb = blend_setup(xb, yb, t, p, o.inv_ext, o.flr, o.frl, bp);
            float cl[3], cr[3];
            if (o.bx + o.bw <= W) {
                const uint8_t *Lb = o.L + (size_t)o.by * o.pitchL + 3 * (size_t)o.bx;
                const uint8_t *Rb = o.R + (size_t)o.by * o.pitchR + 3 * (size_t)o.bx;
                sample_u8(Lb, o.pitchL, o.bh, o.bw, pb.lx, pb.ly, pb.lfx, pb.lfy, cl);
                sample_u8(Rb, o.pitchR, o.bh, o.bw, pb.rx, pb.ry, pb.rfx, pb.rfy, cr);
            } else {
                sample_box_wrap(o.L, o.pitchL, W, o.bx, o.by, o.bw, o.bh, pb.lx, pb.ly, pb.lfx, pb.lfy, cl);
                sample_box_wrap(o.R, o.pitchR, W, o.bx, o.by, o.bw, o.bh, pb.rx, pb.ry, pb.rfx, pb.rfy, cr);
            }
            const float sR = 1.0f - pb.sL;
#pragma unroll
            for (int c = 0; c < 3; c++) f[c] = pb.sL * cl[c] + sR * cr[c];
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const float r = floorf(f[c] + 0.5f);
            sb[off + 3 * i + c] = (uint8_t)fminf(fmaxf(r, 0.f), 255.f);
            if (o.Ff32) gst(o.Ff32)[3 * ((size_t)y * W + x) + c] = f[c];
        }
    }
    __syncthreads();
    const int nb = 3 * npx, end = off + nb;
    const auto dst = reinterpret_cast<__attribute__((address_space(1))) uint32_t *>((uintptr_t)seg - off);
    const int first = (off + 3) >> 2, last = end >> 2;
    for (int k = first + (int)threadIdx.x; k < last; k += kRowTW) dst[k] = stage[k];
    if (threadIdx.x < 8) {
        const int i = threadIdx.x < 4 ? off + (int)threadIdx.x : 4 * last + (int)threadIdx.x - 4;
        const bool lead = threadIdx.x < 4 && i < min(4 * first, end);
        const bool trail = threadIdx.x >= 4 && i >= max(4 * last, 4 * first) && i < end;
        if (lead || trail) gst(seg - off)[i] = sb[i];
    }
}

// ------------------------------------------------------- photo merging
// The first photo of a merge: dst = image on its coverage, 0 elsewhere;
// cov = 1 on the coverage, 0 elsewhere. One thread per pixel.
__global__ __launch_bounds__(256) void k_photo_init(const uint8_t *img, int pitchI, const uint8_t *mask, int pitchM,
                                                    int H, int W, uint8_t *dst, int pitchD, uint8_t *cov, int pitchC)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= W) return;
    const bool m = gld(mask)[(size_t)y * pitchM + x] != 0;
#pragma unroll
    for (int c = 0; c < 3; c++) gst(dst)[(size_t)y * pitchD + 3 * x + c] = m ? gld(img)[(size_t)y * pitchI + 3 * x + c] : 0;
    gst(cov)[(size_t)y * pitchC + x] = m ? 1 : 0;
}

// Box crop of an RGB canvas image whose columns wrap modulo W, into a
// contiguous buffer (the input of the flow path for a box that wraps).
__global__ __launch_bounds__(256) void k_gather_box(const uint8_t *img, int pitch, int W, int bx, int by, int bw,
                                                    uint8_t *dst, int pitchD)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= bw) return;
    int cx = bx + x;
    if (cx >= W) cx -= W;
    const uint8_t *src = img + (size_t)(by + y) * pitch + 3 * (size_t)cx;
    uint8_t *d = dst + (size_t)y * pitchD + 3 * (size_t)x;
#pragma unroll
    for (int c = 0; c < 3; c++) gst(d)[c] = gld(src)[c];
}

// ------------------------------------------------------------- launchers
hipError_t launch_overlap_box(const uint8_t *mL, const uint8_t *mR, int pitchM, int H, int W, bool periodic,
                              int32_t *part, int32_t *box, hipStream_t s)
{
    uint32_t *occ = periodic ? reinterpret_cast<uint32_t *>(part + 2 * (size_t)H) : nullptr;
    hipLaunchKernelGGL(k_box_rows, dim3(H), dim3(kCanvasThreads), 0, s, mL, mR, pitchM, W, part, occ,
                       ceil_div(W, 32));
    if (occ)
        hipLaunchKernelGGL(k_box_cols, dim3(ceil_div(W, 256 * kCanvasChunk), ceil_div(H, kBoxBand)), dim3(256), 0, s,
                           mL, mR, pitchM, H, W, occ);
    hipLaunchKernelGGL(k_box_fin, dim3(1), dim3(1024), 0, s, part, H, W, occ, box);
    return hipGetLastError();
}

hipError_t launch_gather_box(const uint8_t *img, int pitch, int W, int bx, int by, int bw, int bh, uint8_t *dst,
                             int pitchD, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_box, dim3(ceil_div(bw, 256), bh), dim3(256), 0, s, img, pitch, W, bx, by, bw, dst,
                       pitchD);
    return hipGetLastError();
}

hipError_t launch_canvas_dist(const CanvasGeom &a, float *blend, int pitchB, int32_t *d1, int32_t *d2, int pitchD,
                              const int32_t *box, hipStream_t s)
{
    // tiles of 64 columns x kCanvasBH rows: all of them, or those that meet
    // the box (every column of a box across the wrap of a periodic canvas)
    int tx0 = 0, ntx = ceil_div(a.W, 64), tb0 = 0, ntb = ceil_div(a.H, kCanvasBH);
    if (box && box[2] > 0 && box[3] > 0) {
        if (box[0] + box[2] <= a.W) {
            tx0 = box[0] / 64;
            ntx = ceil_div(box[0] + box[2], 64) - tx0;
        }
        tb0 = box[1] / kCanvasBH;
        ntb = ceil_div(box[1] + box[3], kCanvasBH) - tb0;
    }
    CanvasGeom r = a;  // G only in the columns that the tiles read
    r.gx0 = tx0 * 64;
    r.gx1 = min(a.W, (tx0 + ntx) * 64);
    hipLaunchKernelGGL(k_canvas_rows, dim3(a.H), dim3(kCanvasThreads), 0, s, r);
    hipLaunchKernelGGL(k_canvas_colmin, dim3(ceil_div(min(ntx * 64, a.W - tx0 * 64), kCanvasThreads),
                                             ceil_div(a.H, kCanvasBH)),
                       dim3(kCanvasThreads), 0, s, a, tx0 * 64);
    hipLaunchKernelGGL(k_canvas_dist, dim3(ntx, ntb), dim3(256), 0, s, a, blend, pitchB, d1, d2, pitchD, tx0, tb0);
    return hipGetLastError();
}

hipError_t launch_photo_init(const uint8_t *img, int pitchI, const uint8_t *mask, int pitchM, int H, int W,
                             uint8_t *dst, int pitchD, uint8_t *cov, int pitchC, hipStream_t s)
{
    hipLaunchKernelGGL(k_photo_init, dim3(ceil_div(W, 256), H), dim3(256), 0, s, img, pitchI, mask, pitchM, H, W, dst,
                       pitchD, cov, pitchC);
    return hipGetLastError();
}

hipError_t launch_composite(const CompositeArgs &o, BlendParams bp, hipStream_t s)
{
    constexpr int PX = 4;
    hipLaunchKernelGGL(k_composite<PX>, dim3(o.H * ceil_div(o.W, PX * kRowTW)), dim3(kRowTW), 0, s, o, bp);
    return hipGetLastError();
}

}  // namespace abf
