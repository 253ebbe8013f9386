// Propagation and median of the coarse-to-fine flow (libabf, gfx950):
// Section III.C.1 of Meng & Liu, arXiv 2006.01201, as read in this
// library (the paper names the flow method but gives no details).
#include <type_traits>

#include "abf_tiles.h"

namespace abf {

// ----------------------------------------------------------- propagation
// T Jacobi propagation steps and the 3x3 median of one level in one
// launch (steps 3 and 4 of the flow). In a step each pixel keeps the
// lowest-cost vector among its own and those of its left, right, upper
// and lower neighbours in the previous iterate (neighbours outside the
// image skipped; on equal cost the earlier candidate in that order wins);
// the median is component-wise with clamped indices.
//
// One wave per tile, everything in registers: a lane owns one column of a
// 64 x (TB + 2h) region around a (64 - 2h) x TB output tile (h = T + M) and
// holds the vectors and costs of all its region rows. Upper and lower
// neighbours are the lane's own registers, left and right ones come from
// DPP lane shifts; step t updates the region inset by t and reads only the
// previous iterate, so the output equals that of T full-image steps. No
// barrier is needed but around the job list below.
//
// A neighbour's vector replaces a pixel's only at a strictly lower patch
// cost, and the pixel's own cost is carried, so a candidate is costed only
// if it can win:
//  - step 1: not if it lies in the pixel's search window (the search took
//    the minimum over that window), so never the two neighbours in the
//    pixel's 2 x 2 cell of the coarser level, which share that window;
//  - step t > 1: not if that neighbour did not change in step t - 1 (the
//    pixel already weighed that vector and holds one at most as costly);
//  - never if it equals an earlier candidate (same cost, loses the tie).
// The rest (about 0.1 per pixel and step at level 0 of the panorama) are
// packed into an LDS job list (ballot prefix counts per row), costed one
// per lane, and read back by each pixel in candidate order, so the result
// does not depend on the packing; a list longer than the LDS ring is
// processed in passes.
template <int NBITS>
__device__ __forceinline__ int wave_prefix(uint32_t c, int &total)
{
    // exclusive prefix sum over the wave of c (below 2^NBITS) and the wave total
    int pre = 0;
    total = 0;
#pragma unroll
    for (int b = 0; b < NBITS; b++) {
        const uint64_t m = __ballot((c >> b) & 1u);
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
        pre += below << b;
        total += __popcll(m) << b;
    }
    return pre;
}

// Whole-wave lane shifts (DPP): lane i takes the value of lane i - 1
// (from_left) or lane i + 1 (from_right); the end lane takes `end`. The
// propagation passes a different `end` in each phase, so that the compiler
// recomputes a shift (one instruction) rather than keeping the shifted
// rows of one phase live in registers through the next.
__device__ __forceinline__ uint32_t from_left(uint32_t v, uint32_t end)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)end, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t from_right(uint32_t v, uint32_t end)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)end, (int)v, 0x130, 0xf, 0xf, false);
}

typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ i16x2 as_i16x2(uint32_t v) { return __builtin_bit_cast(i16x2, v); }
__device__ __forceinline__ i16x2 pmin(i16x2 a, i16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ i16x2 pmax(i16x2 a, i16x2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ i16x2 pmed3(i16x2 a, i16x2 b, i16x2 c) { return pmax(pmin(a, b), pmin(pmax(a, b), c)); }

// Patch cost C(p, d) of pixel (px, py) and vector (dx, dy): Ref rows from
// `refo`, Tgt rows from `tgto` (padded-plane origins); a Tgt window beyond
// the padded border takes the per-byte clamped path.
template <int P>
__device__ __forceinline__ uint32_t job_cost(const uint8_t *refo, const uint8_t *tgto, const uint8_t *tgt, int yp,
                                             int H, int W, int px, int py, int dx, int dy)
{
    constexpr int NB = 2 * P + 1, ND = RawRows<NB>::ND;
    const int c0 = px + dx - P, r0 = py + dy - P;
    uint32_t rr[NB][(NB + 3) / 4], tt[NB][(NB + 3) / 4];
    if (c0 >= -kPad && c0 + 2 * P <= W - 1 + kPad && r0 >= -kPad && r0 + 2 * P <= H - 1 + kPad) {
        uint32_t wr[NB][ND + 1], wt[NB][ND + 1];
        const int sr = issue_rows<NB, NB>(refo, yp, py - P, px - P, wr);
        const int st = issue_rows<NB, NB>(tgto, yp, r0, c0, wt);
        __builtin_amdgcn_sched_barrier(0);
        align_rows<NB, NB>(wr, sr, rr);
        align_rows<NB, NB>(wt, st, tt);
    } else {
        load_rows<NB, NB>(refo, yp, py - P, px - P, rr);
#pragma unroll
        for (int r = 0; r < NB; r++) load_row_clamped<NB>(tgt, H, W, yp, r0 + r, c0, tt[r]);
    }
    uint32_t cost = 0;
#pragma unroll
    for (int r = 0; r < NB; r++) {
        if constexpr (P == 2) {
            cost = __builtin_amdgcn_sad_u8(rr[r][0], tt[r][0], cost);
            cost = __builtin_amdgcn_sad_u8(rr[r][1] & 0xffu, tt[r][1] & 0xffu, cost);
        } else {
            cost = __builtin_amdgcn_sad_u8(rr[r][0] & 0x00ffffffu, tt[r][0] & 0x00ffffffu, cost);
        }
    }
    return cost;
}

// Per-pixel state word of the propagation: the cost of the current vector
// (13 bits: at most 25 * 255), whether the vector changed in the previous
// step, and, within a step, the candidates to cost (4 bits, left, right,
// up, down), the lane's first job within its row's jobs (8 bits) and the
// winning candidate so far (0 = own vector).
constexpr uint32_t kPmCost = 0x1fffu, kPmChg = 1u << 13;
constexpr int kPmNeed = 14, kPmPre = 18, kPmWin = 26;
constexpr int kPropCap = 512;  // job records in LDS per pass

// Regions of up to 18 rows are held to 128 VGPRs (4 waves per SIMD): the
// 12-row tile of 2 steps and the median needs 135 unconstrained and fits
// without spills under the cap (larger regions would spill).
template <int P, int TB, int HB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TB + 2 * HB <= 18 ? 4 : 1, 8))) void k_prop(
    const StripLv *__restrict__ lv, const int32_t *__restrict__ prefix, int n, int total, int T)
{
    constexpr int RB = TB + 2 * HB, OW = 64 - 2 * HB;
    static_assert(TB % 2 == 0, "even tile heights: a region row's parity of y is fixed");
    constexpr int NCEN = (RB + (HB & 1) + 1) / 2;  // coarse rows under the region
    __shared__ uint2 jobs[kPropCap];               // (candidate vector, row << 6 | lane), then its cost
    const int M = HB - T;
    const int rx = threadIdx.x;
    TILE_LOOP(total)
    {
        const int s = find_strip(prefix, n, t);
        int local = t - prefix[s];
        const StripLv &L = lv[s];
        const int H = L.H, W = L.W, yp = L.ypitch, fp = L.fpitch, R = L.radius;
        const int ntx = ceil_div(W, OW), per_dir = ntx * ceil_div(H, TB);
        const int dir = local / per_dir;
        local -= dir * per_dir;
        const int tyi = local / ntx;
        const int gx0 = (local - tyi * ntx) * OW - HB, gy0 = tyi * TB - HB;  // image position of region (0, 0)
        const int x = gx0 + rx;
        const bool xin = x >= 0 && x < W;
        const uint8_t *refo = plane_org(L.y[dir], yp), *tgto = plane_org(L.y[1 - dir], yp);
        uint32_t v[RB], m[RB];
        // search centres: row q of the region lies under coarse row (gy0 + q) >> 1,
        // which rows q and q + 1 share for q + HB odd (gy0 has HB's parity)
        uint32_t cen[NCEN];
        {
            const auto din = gld(L.ds[dir]);
            const auto cin = gld(L.cs[dir]);
            const uint32_t *dc = L.dc[dir];
#pragma unroll
            for (int q = 0; q < RB; q++) {
                const int y = gy0 + q;
                const bool in = xin && y >= 0 && y < H;
                const uint32_t o = in ? (uint32_t)(y * fp + x) : 0u;
                v[q] = in ? din[o] : 0u;
                m[q] = in ? (uint32_t)cin[o] : 0u;
            }
#pragma unroll
            for (int c = 0; c < NCEN; c++) {
                const int q = 2 * c - (HB & 1), y = gy0 + (q < 0 ? 0 : q);
                const bool in = xin && y >= 0 && y < H && dc;
                cen[c] = in ? gld(dc)[(uint32_t)(min(y >> 1, L.Hc - 1) * L.fpitch_c + min(x >> 1, L.Wc - 1))] : 0u;
            }
        }

        uint64_t chg = ~0ull;  // bit q: some pixel of region row q changed in the last step
        auto step = [&](int st, auto first) {
            constexpr bool FIRST = decltype(first)::value;
            const bool xact = xin && rx >= st && rx < 64 - st;
            const bool okl = xact && x > 0, okr = xact && x < W - 1;
            int rowbase[RB];
            int J = 0;
            // candidates to cost, per row
#pragma unroll
            for (int q = 1; q < RB - 1; q++) {
                rowbase[q] = J;
                const int y = gy0 + q;
                if (q < st || q >= RB - st || y < 0 || y >= H) continue;  // uniform
                if (!FIRST && ((chg >> (q - 1)) & 7ull) == 0) {
                    // no pixel of rows q - 1 .. q + 1 changed: no candidate can win
                    m[q] &= kPmCost | kPmChg;
                    continue;
                }
                // lane shifts outside any divergent code (a DPP read of an inactive
                // lane returns the fallback value)
                const uint32_t c0 = v[q], c1 = from_left(c0, 0u), c2 = from_right(c0, 0u);
                const bool oku = xact && y > 0, okd = xact && y < H - 1;
                uint32_t need;
                int wt, pre;
                if constexpr (FIRST) {
                    // A neighbour in the pixel's 2 x 2 cell of the coarser level has
                    // the pixel's search window, which holds its vector: only the
                    // neighbour across each edge of the cell can win, the left one at
                    // even x, the right one at odd x, the upper one at even y, the
                    // lower one at odd y (y's parity is fixed per region row: gy0 has
                    // HB's parity). An earlier candidate it duplicates is either that
                    // other horizontal neighbour (in the window, so this one is too)
                    // or the horizontal candidate. need: bit 0 horizontal, bit 1
                    // vertical.
                    const bool ev = (x & 1) == 0, yev = ((q + HB) & 1) == 0;
                    const uint32_t ch = ev ? c1 : c2;
                    const uint32_t cv = yev ? v[q - 1] : v[q + 1];
                    const bool okh = ev ? okl : okr, okv = yev ? oku : okd;
                    const uint32_t ce = cen[(q + (HB & 1)) >> 1];
                    const int cx = unpack_x(ce) * 2, cy = unpack_y(ce) * 2;
                    const uint32_t w = (uint32_t)(2 * R);
                    auto out = [&](uint32_t c) {
                        return ((uint32_t)(unpack_x(c) - cx + R) > w) || ((uint32_t)(unpack_y(c) - cy + R) > w);
                    };
                    const bool nh = okh & (ch != c0) & out(ch);
                    const bool nv = okv & (cv != c0) & !(okh & (cv == ch)) & out(cv);
                    need = (nh ? 1u : 0u) | (nv ? 2u : 0u);
                    pre = wave_prefix<2>(__popc(need), wt);
                } else {
                    const uint32_t c3 = v[q - 1], c4 = v[q + 1];
                    bool n1 = okl & (c1 != c0);
                    bool n2 = okr & (c2 != c0) & !(okl & (c2 == c1));
                    bool n3 = oku & (c3 != c0) & !(okl & (c3 == c1)) & !(okr & (c3 == c2));
                    bool n4 = okd & (c4 != c0) & !(okl & (c4 == c1)) & !(okr & (c4 == c2)) & !(oku & (c4 == c3));
                    n1 &= (from_left(m[q], 0u) & kPmChg) != 0;
                    n2 &= (from_right(m[q], 0u) & kPmChg) != 0;
                    n3 &= (m[q - 1] & kPmChg) != 0;
                    n4 &= (m[q + 1] & kPmChg) != 0;
                    need = (n1 ? 1u : 0u) | (n2 ? 2u : 0u) | (n3 ? 4u : 0u) | (n4 ? 8u : 0u);
                    pre = wave_prefix<3>(__popc(need), wt);
                }
                m[q] = (m[q] & (kPmCost | kPmChg)) | need << kPmNeed | (uint32_t)pre << kPmPre;
                J += wt;
            }
            // cost the jobs, kPropCap at a time
            for (int base = 0; base < J; base += kPropCap) {
#pragma unroll
                for (int q = 1; q < RB - 1; q++) {
                    const int y = gy0 + q;
                    if (q < st || q >= RB - st || y < 0 || y >= H) continue;  // uniform
                    const uint32_t cl = from_left(v[q], 1u), cr = from_right(v[q], 1u);
                    const uint32_t need = (m[q] >> kPmNeed) & (FIRST ? 3u : 15u);
                    if (need) {
                        int j = rowbase[q] + (int)((m[q] >> kPmPre) & 0xffu) - base;
                        const uint32_t pos = (uint32_t)(q << 6 | rx);
                        if constexpr (FIRST) {
                            const bool ev = (x & 1) == 0, yev = ((q + HB) & 1) == 0;
                            const uint32_t ch = ev ? cl : cr;
                            if (need & 1u) {
                                if (j >= 0 && j < kPropCap) jobs[j] = make_uint2(ch, pos);
                                j++;
                            }
                            if ((need & 2u) && j >= 0 && j < kPropCap) jobs[j] = make_uint2(yev ? v[q - 1] : v[q + 1], pos);
                        } else {
#pragma unroll
                            for (int k = 0; k < 4; k++)
                                if (need & (1u << k)) {
                                    if (j >= 0 && j < kPropCap)
                                        jobs[j] = make_uint2(k == 0 ? cl : k == 1 ? cr : k == 2 ? v[q - 1] : v[q + 1], pos);
                                    j++;
                                }
                        }
                    }
                }
                __syncthreads();
                const int nb = min(kPropCap, J - base);
                for (int j = rx; j < nb; j += 64) {
                    const uint2 e = jobs[j];
                    const int px = gx0 + (int)(e.y & 63u), py = gy0 + (int)(e.y >> 6);
                    jobs[j].x = job_cost<P>(refo, tgto, L.y[1 - dir], yp, H, W, px, py, unpack_x(e.x), unpack_y(e.x));
                }
                __syncthreads();
                // values derived from the state words are recomputed below rather than
                // kept live through the job loop (an empty asm hides that they are unchanged)
#pragma unroll
                for (int q = 0; q < RB; q++) asm volatile("" : "+v"(m[q]));
#pragma unroll
                for (int q = 1; q < RB - 1; q++) {
                    const int y = gy0 + q;
                    if (q < st || q >= RB - st || y < 0 || y >= H) continue;  // uniform
                    const uint32_t need = (m[q] >> kPmNeed) & (FIRST ? 3u : 15u);
                    if (need) {
                        int j = rowbase[q] + (int)((m[q] >> kPmPre) & 0xffu) - base;
                        uint32_t bc = m[q] & kPmCost, bk = (m[q] >> kPmWin) & 7u;
                        // winner codes: 1 left, 2 right, 3 up, 4 down
                        auto take = [&](uint32_t code) {
                            if (j >= 0 && j < kPropCap) {
                                const uint32_t c = jobs[j].x;
                                if (c < bc) {
                                    bc = c;
                                    bk = code;
                                }
                            }
                            j++;
                        };
                        if constexpr (FIRST) {
                            const bool ev = (x & 1) == 0, yev = ((q + HB) & 1) == 0;
                            if (need & 1u) take(ev ? 1u : 2u);
                            if (need & 2u) take(yev ? 3u : 4u);
                        } else {
#pragma unroll
                            for (int k = 0; k < 4; k++)
                                if (need & (1u << k)) take((uint32_t)(k + 1));
                        }
                        m[q] = (m[q] & ~(kPmCost | 7u << kPmWin)) | bc | bk << kPmWin;
                    }
                }
                __syncthreads();  // the next pass overwrites the records
            }
            // apply the winners (Jacobi: every row reads the previous iterate)
            uint32_t up = v[0];
            chg = 0;
#pragma unroll
            for (int q = 1; q < RB - 1; q++) {
                const uint32_t old = v[q];
                const int y = gy0 + q;
                if (q >= st && q < RB - st && y >= 0 && y < H) {  // uniform
                    const uint32_t cl = from_left(old, 2u), cr = from_right(old, 2u);
                    const uint32_t bk = (m[q] >> kPmWin) & 7u;
                    v[q] = bk == 0 ? old : bk == 1 ? cl : bk == 2 ? cr : bk == 3 ? up : v[q + 1];
                    m[q] = (m[q] & kPmCost) | (bk ? kPmChg : 0u);
                    if (__ballot(bk != 0)) chg |= 1ull << q;
                }
                up = old;
            }
        };
        if (T >= 1) step(1, std::true_type{});
        for (int st = 2; st <= T; st++) step(st, std::false_type{});

        // median (or copy) of the output tile, on packed int16 pairs
        const auto dst = gst(L.df[dir]);
        const bool xout = xin && rx >= HB && rx < HB + OW;
        if (HB == 0 || M == 0) {
#pragma unroll
            for (int q = HB; q < HB + TB; q++) {
                const int y = gy0 + q;
                if (y < H && xout) dst[(uint32_t)(y * fp + x)] = v[q];
            }
        } else if constexpr (HB > 0) {
            // sorted horizontal triples (clamped) of rows q - 1, q, q + 1
            auto triple = [&](int q, i16x2 &lo, i16x2 &md, i16x2 &hi) {
                const uint32_t c = v[q], l = from_left(c, c), r = from_right(c, c);
                const i16x2 a = as_i16x2(x > 0 ? l : c), b = as_i16x2(c), d = as_i16x2(x < W - 1 ? r : c);
                lo = pmin(pmin(a, b), d);
                hi = pmax(pmax(a, b), d);
                md = pmed3(a, b, d);
            };
            i16x2 lo0, md0, hi0, lo1, md1, hi1;
            triple(HB - 1, lo0, md0, hi0);
            triple(HB, lo1, md1, hi1);
#pragma unroll
            for (int q = HB; q < HB + TB; q++) {
                i16x2 lo2, md2, hi2;
                triple(q + 1, lo2, md2, hi2);
                const int y = gy0 + q;
                // clamp rows to the image (uniform selects)
                const i16x2 lu = y > 0 ? lo0 : lo1, mu = y > 0 ? md0 : md1, hu = y > 0 ? hi0 : hi1;
                const i16x2 ld = y < H - 1 ? lo2 : lo1, mdn = y < H - 1 ? md2 : md1, hd = y < H - 1 ? hi2 : hi1;
                // median of 9 = med3(max of row minima, med3 of row medians, min of row maxima)
                const i16x2 a = pmax(pmax(lu, lo1), ld), b = pmin(pmin(hu, hi1), hd), c = pmed3(mu, md1, mdn);
                if (y < H && xout) dst[(uint32_t)(y * fp + x)] = __builtin_bit_cast(uint32_t, pmed3(a, c, b));
                lo0 = lo1, md0 = md1, hi0 = hi1;
                lo1 = lo2, md1 = md2, hi1 = hi2;
            }
        }
    }
}

// ------------------------------------------------------------- launchers
template <int P, int TB, int HB>
static void prop_launch(const StripLv *lv, Work w, int steps, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_prop<P, TB, HB>), dim3(grid_for(w.total, grid)), dim3(64), 0, s, lv, w.prefix, w.n,
                       w.total, steps);
}

template <int P, int TB>
static hipError_t prop_h(const StripLv *lv, Work w, int steps, int median, int grid, hipStream_t s)
{
    switch (steps + median) {
    case 0: prop_launch<P, TB, 0>(lv, w, steps, grid, s); break;
    case 1: prop_launch<P, TB, 1>(lv, w, steps, grid, s); break;
    case 2: prop_launch<P, TB, 2>(lv, w, steps, grid, s); break;
    case 3: prop_launch<P, TB, 3>(lv, w, steps, grid, s); break;
    case 4: prop_launch<P, TB, 4>(lv, w, steps, grid, s); break;
    case 5: prop_launch<P, TB, 5>(lv, w, steps, grid, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int P>
static hipError_t prop_th(const StripLv *lv, Work w, int steps, int median, int th, int grid, hipStream_t s)
{
    if (th == 8) return prop_h<P, 8>(lv, w, steps, median, grid, s);
    if (th == 10) return prop_h<P, 10>(lv, w, steps, median, grid, s);
    if (th == 12) return prop_h<P, 12>(lv, w, steps, median, grid, s);
    if (th == 16) return prop_h<P, 16>(lv, w, steps, median, grid, s);
    if (th == 32) return prop_h<P, 32>(lv, w, steps, median, grid, s);
    return hipErrorInvalidValue;
}

hipError_t launch_prop(const StripLv *lv, Work w, int patch, int steps, int median, int th, int grid, hipStream_t s)
{
    if (patch == 1) return prop_th<1>(lv, w, steps, median, th, grid, s);
    if (patch == 2) return prop_th<2>(lv, w, steps, median, th, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace abf
