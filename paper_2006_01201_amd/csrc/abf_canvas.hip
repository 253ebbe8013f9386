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
//      second kernel stores the minimum of g over every 32-row block of a
//      column.
//   2. columns: D(x, y) = min over rows y' of (y - y')^2 + g(x, y')^2,
//      searched outward from y. A block of rows whose nearest row is k
//      rows away and whose minimum g is m cannot beat k^2 + m^2, so it is
//      skipped when that bound reaches the best value found, and the
//      search ends in a direction once k^2 does. The work per pixel
//      grows with the distance only through the number of 32-row blocks
//      passed over, not their rows.
#include "abf_device.h"

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
        uint32_t b1 = 0, b2 = 0;
        for (int k = 0; k < n; k++) {
            const bool l = gld(rl)[x0 + k] != 0, r = gld(rr)[x0 + k] != 0;
            b1 |= (uint32_t)(l && !r) << k;
            b2 |= (uint32_t)(r && !l) << k;
        }
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
    for (int c = t; c < nC; c += kCanvasThreads) {
        const uint32_t bb = bits[c];
        const int x0 = c * kCanvasChunk, n = min(kCanvasChunk, W - x0);
        int l1 = lastA[c], l2 = lastB[c], r1 = firstA[c], r2 = firstB[c];
        uint32_t d[kCanvasChunk];
#pragma unroll
        for (int k = 0; k < kCanvasChunk; k++) {
            const int x = x0 + k;
            if ((bb >> k) & 1u) l1 = x;
            if ((bb >> (16 + k)) & 1u) l2 = x;
            const uint32_t e1 = l1 >= 0 ? (uint32_t)(x - l1) : kInf16;
            const uint32_t e2 = l2 >= 0 ? (uint32_t)(x - l2) : kInf16;
            d[k] = e1 | (e2 << 16);
        }
#pragma unroll
        for (int k = kCanvasChunk - 1; k >= 0; k--) {
            const int x = x0 + k;
            if ((bb >> k) & 1u) r1 = x;
            if ((bb >> (16 + k)) & 1u) r2 = x;
            const uint32_t e1 = r1 != INF ? (uint32_t)(r1 - x) : kInf16;
            const uint32_t e2 = r2 != INF ? (uint32_t)(r2 - x) : kInf16;
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
__global__ __launch_bounds__(kCanvasThreads) void k_canvas_colmin(CanvasGeom a)
{
    const int x = blockIdx.x * kCanvasThreads + threadIdx.x, b = blockIdx.y;
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
// The two squared distances of the pixel of this lane. Every lane of a
// wave is on row y (wave-uniform loop bounds); `best1` / `best2` start at
// the row distance of the pixel itself squared, or 0 for an area whose
// distance is not needed (then nothing is searched for it).
__device__ __forceinline__ void col_search(const CanvasGeom &a, int x, int y, bool in, uint32_t &best1,
                                           uint32_t &best2)
{
    const int H = a.H, b0 = y / kCanvasBH;
    const uint32_t *G = a.G;
    auto row = [&](int r, bool act) {
        const uint32_t k = (uint32_t)abs(r - y), k2 = k * k;
        if (act && k2 < max(best1, best2)) {
            const uint32_t g = gld(G)[(size_t)r * a.gpitch + x];
            best1 = min(best1, cand(k2, g & 0xffffu));
            best2 = min(best2, cand(k2, g >> 16));
        }
    };
    auto live = [&](uint32_t k2, bool act) { return __ballot(act && in && k2 < max(best1, best2)) != 0; };
    // rows of the pixel's own block, nearest first
    const int lo = b0 * kCanvasBH, hi = min(lo + kCanvasBH, H) - 1;
    for (int k = 1; y - k >= lo || y + k <= hi; k++) {
        if (!live((uint32_t)(k * k), true)) break;
        if (y - k >= lo) row(y - k, in);
        if (y + k <= hi) row(y + k, in);
    }
    // blocks above, nearest first
    for (int b = b0 - 1; b >= 0; b--) {
        const uint32_t dk = (uint32_t)(y - (b * kCanvasBH + kCanvasBH - 1)), dk2 = dk * dk;
        if (!live(dk2, true)) break;
        bool scan = false;
        if (in) {
            const uint32_t m = gld(a.M)[(size_t)b * a.gpitch + x];
            scan = cand(dk2, m & 0xffffu) < best1 || cand(dk2, m >> 16) < best2;
        }
        for (int r = b * kCanvasBH + kCanvasBH - 1; r >= b * kCanvasBH; r--) {
            const uint32_t k = (uint32_t)(y - r);
            if (!live(k * k, scan)) break;
            row(r, scan);
        }
    }
    // blocks below, nearest first
    const int nb = ceil_div(H, kCanvasBH);
    for (int b = b0 + 1; b < nb; b++) {
        const uint32_t dk = (uint32_t)(b * kCanvasBH - y), dk2 = dk * dk;
        if (!live(dk2, true)) break;
        bool scan = false;
        if (in) {
            const uint32_t m = gld(a.M)[(size_t)b * a.gpitch + x];
            scan = cand(dk2, m & 0xffffu) < best1 || cand(dk2, m >> 16) < best2;
        }
        const int rend = min(b * kCanvasBH + kCanvasBH, H);
        for (int r = b * kCanvasBH; r < rend; r++) {
            const uint32_t k = (uint32_t)(r - y);
            if (!live(k * k, scan)) break;
            row(r, scan);
        }
    }
}

// One wave per 64 columns of a row (workgroup = 4 rows). Writes Blend
// (eq. (1)) and, if requested, both squared distances of every pixel
// (-1 where the area is empty).
__global__ __launch_bounds__(256) void k_canvas_dist(CanvasGeom a, float *blend, int pitchB, int32_t *d1, int32_t *d2,
                                                     int pitchD)
{
    const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
    if (y >= a.H) return;  // whole waves
    const bool in = x < a.W;
    int area = 0;
    uint32_t g0 = kInf32;
    if (in) {
        area = (gld(a.mL)[(size_t)y * a.pitchM + x] != 0) + 2 * (gld(a.mR)[(size_t)y * a.pitchM + x] != 0);
        g0 = gld(a.G)[(size_t)y * a.gpitch + x];
    }
    const bool all = d1 != nullptr;
    const bool need = in && (all || area == 3);
    uint32_t best1 = need ? cand(0, g0 & 0xffffu) : 0u;
    uint32_t best2 = need ? cand(0, g0 >> 16) : 0u;
    col_search(a, x, y, in, best1, best2);
    if (!in) return;
    if (blend) {
        float t;
        if (area == 1) t = 0.f;
        else if (area == 2) t = 1.f;
        else if (area == 0) t = 0.5f;
        else if (best1 == kInf32 && best2 == kInf32) t = 0.5f;
        else if (best1 == kInf32) t = 1.f;
        else if (best2 == kInf32) t = 0.f;
        else {
            const double l = sqrt((double)best1), r = sqrt((double)best2);
            t = (float)(l / (l + r));
        }
        gst(blend)[(size_t)y * pitchB + x] = t;
    }
    if (all) {
        gst(d1)[(size_t)y * pitchD + x] = best1 == kInf32 ? -1 : (int32_t)best1;
        gst(d2)[(size_t)y * pitchD + x] = best2 == kInf32 ? -1 : (int32_t)best2;
    }
}

// ------------------------------------------------------------ overlap box
__global__ void k_box_init(int32_t *box)
{
    if (threadIdx.x < 4) gst(box)[threadIdx.x] = threadIdx.x < 2 ? 0x7fffffff : -1;
}

// One workgroup per row: extent of the row's Area3 pixels, merged into
// {x0, y0, x1, y1} with atomics.
__global__ __launch_bounds__(kCanvasThreads) void k_box_rows(const uint8_t *mL, const uint8_t *mR, int pitchM, int W,
                                                             int32_t *box)
{
    __shared__ int32_t s[2];
    const int y = blockIdx.x;
    if (threadIdx.x == 0) {
        s[0] = 0x7fffffff;
        s[1] = -1;
    }
    __syncthreads();
    int lo = 0x7fffffff, hi = -1;
    for (int x = threadIdx.x; x < W; x += kCanvasThreads)
        if (gld(mL)[(size_t)y * pitchM + x] != 0 && gld(mR)[(size_t)y * pitchM + x] != 0) {
            lo = min(lo, x);
            hi = max(hi, x);
        }
    if (hi >= 0) {
        atomicMin(&s[0], lo);
        atomicMax(&s[1], hi);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s[1] >= 0) {
        atomicMin(&box[0], s[0]);
        atomicMin(&box[1], y);
        atomicMax(&box[2], s[1]);
        atomicMax(&box[3], y);
    }
}

// {x0, y0, x1, y1} -> {x, y, w, h}, zeros when there is no Area3 pixel
__global__ void k_box_fin(int32_t *box)
{
    if (threadIdx.x == 0) {
        const int x0 = box[0], y0 = box[1], x1 = box[2], y1 = box[3];
        const bool e = x1 < 0;
        gst(box)[0] = e ? 0 : x0;
        gst(box)[1] = e ? 0 : y0;
        gst(box)[2] = e ? 0 : x1 - x0 + 1;
        gst(box)[3] = e ? 0 : y1 - y0 + 1;
    }
}

// ------------------------------------------------------------- composite
// Code 1 over the canvas, one workgroup per kRowTW pixels of a row: Area1
// copies L, Area2 copies R, Area3 inside the overlap box is warped and
// blended as a strip pixel of the box (images and flows cropped to the
// box), everything else is 0. The uint8 output is staged in LDS at the
// byte alignment of its destination and written with aligned dwords.
__global__ __launch_bounds__(kRowTW) void k_composite(CompositeArgs o, BlendParams bp)
{
    __shared__ uint32_t stage[(3 * kRowTW + 8) / 4];
    uint8_t *sb = reinterpret_cast<uint8_t *>(stage);
    const int W = o.W, segs = ceil_div(W, kRowTW);
    const int y = blockIdx.x / segs, xs = (blockIdx.x - y * segs) * kRowTW;
    const int npx = min(kRowTW, W - xs), x = xs + (int)threadIdx.x;
    uint8_t *const seg = o.F + (size_t)y * o.pitchF + 3 * (size_t)xs;
    const int off = (int)((uintptr_t)seg & 3);
    if (x < W) {
        const size_t pm = (size_t)y * o.pitchM + x;
        const int area = (gld(o.mL)[pm] != 0) + 2 * (gld(o.mR)[pm] != 0);
        const int xb = x - o.bx, yb = y - o.by;
        float f[3] = {0.f, 0.f, 0.f};
        if (area == 1 || area == 2) {
            const uint8_t *src = area == 1 ? o.L + (size_t)y * o.pitchL : o.R + (size_t)y * o.pitchR;
#pragma unroll
            for (int c = 0; c < 3; c++) f[c] = (float)gld(src)[3 * x + c];
        } else if (area == 3 && xb >= 0 && xb < o.bw && yb >= 0 && yb < o.bh) {
            const uint32_t p = (uint32_t)(yb * o.bw + xb);
            const double t = (double)gld(o.blend)[(size_t)y * o.pitchB + x];
            const PixBlend pb = blend_setup(xb, yb, t, p, o.inv_ext, o.flr, o.frl, bp);
            const uint8_t *Lb = o.L + (size_t)o.by * o.pitchL + 3 * (size_t)o.bx;
            const uint8_t *Rb = o.R + (size_t)o.by * o.pitchR + 3 * (size_t)o.bx;
            float cl[3], cr[3];
            sample_u8(Lb, o.pitchL, o.bh, o.bw, pb.lx, pb.ly, pb.lfx, pb.lfy, cl);
            sample_u8(Rb, o.pitchR, o.bh, o.bw, pb.rx, pb.ry, pb.rfx, pb.rfy, cr);
            const float sR = 1.0f - pb.sL;
#pragma unroll
            for (int c = 0; c < 3; c++) f[c] = pb.sL * cl[c] + sR * cr[c];
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const float r = floorf(f[c] + 0.5f);
            sb[off + 3 * threadIdx.x + c] = (uint8_t)fminf(fmaxf(r, 0.f), 255.f);
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

// ------------------------------------------------------------- launchers
hipError_t launch_overlap_box(const uint8_t *mL, const uint8_t *mR, int pitchM, int H, int W, int32_t *box,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_box_init, dim3(1), dim3(64), 0, s, box);
    hipLaunchKernelGGL(k_box_rows, dim3(H), dim3(kCanvasThreads), 0, s, mL, mR, pitchM, W, box);
    hipLaunchKernelGGL(k_box_fin, dim3(1), dim3(64), 0, s, box);
    return hipGetLastError();
}

hipError_t launch_canvas_dist(const CanvasGeom &a, float *blend, int pitchB, int32_t *d1, int32_t *d2, int pitchD,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_canvas_rows, dim3(a.H), dim3(kCanvasThreads), 0, s, a);
    hipLaunchKernelGGL(k_canvas_colmin, dim3(ceil_div(a.W, kCanvasThreads), ceil_div(a.H, kCanvasBH)),
                       dim3(kCanvasThreads), 0, s, a);
    hipLaunchKernelGGL(k_canvas_dist, dim3(ceil_div(a.W, 64), ceil_div(a.H, 4)), dim3(64, 4), 0, s, a, blend, pitchB,
                       d1, d2, pitchD);
    return hipGetLastError();
}

hipError_t launch_composite(const CompositeArgs &o, BlendParams bp, hipStream_t s)
{
    hipLaunchKernelGGL(k_composite, dim3(o.H * ceil_div(o.W, kRowTW)), dim3(kRowTW), 0, s, o, bp);
    return hipGetLastError();
}

}  // namespace abf
