// Device helpers of the tiled kernels of libabf (not part of the public
// ABI): the flat tile walk over all strips of a batch, and row loads from
// the padded luma planes.
#pragma once

#include "abf_device.h"

namespace abf {

// ---------------------------------------------------------------- helpers

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

// Offset of pixel (r, c), r, c >= -kPad, of a padded plane from the
// plane's origin (its first allocated byte). Window loads address a plane
// as a uniform origin plus a 32-bit offset, which the global loads take
// as a scalar base and a 32-bit vector offset (no 64-bit address
// arithmetic per row).
__device__ __forceinline__ const uint8_t *plane_org(const uint8_t *y, int pitch)
{
    return y - (kPlaneLead + (ptrdiff_t)pitch * kPad + kPad);
}
__device__ __forceinline__ uint32_t pix_off(int pitch, int r, int c)
{
    return (uint32_t)(kPlaneLead + (r + kPad) * pitch + c + kPad);
}

// Bytes c .. c+NB-1 of NR consecutive rows r0 .. r0+NR-1 of a padded
// plane (origin org), normalised so that out[r][k] holds bytes c+4k ..
// c+4k+3 of row r0+r; the rows must hold those bytes (|c| <= kPad away
// from the image). Split into issuing the aligned dword loads and
// normalising them, so that several blocks can be in flight together;
// load_rows does both, with all loads issued before the first row is
// normalised.
template <int NB>
struct RawRows {
    static constexpr int ND = (NB + 6) / 4;  // dwords covering NB bytes at any alignment
};
template <int NB, int NR>
__device__ __forceinline__ int issue_rows(const uint8_t *__restrict__ org, int pitch, int r0, int c,
                                          uint32_t (&w)[NR][RawRows<NB>::ND + 1])
{
    constexpr int ND = RawRows<NB>::ND;
    const uint32_t off = pix_off(pitch, r0, c), a = off & ~3u;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const gu32 *p = (const gu32 *)(const void *)(org + (a + (uint32_t)(r * pitch)));
#pragma unroll
        for (int k = 0; k < ND; k++) w[r][k] = p[k];
        w[r][ND] = 0;
    }
    return (int)(off - a);
}
template <int NB, int NR>
__device__ __forceinline__ void align_rows(const uint32_t (&w)[NR][RawRows<NB>::ND + 1], int s,
                                           uint32_t (&out)[NR][(NB + 3) / 4])
{
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < (NB + 3) / 4; k++) out[r][k] = __builtin_amdgcn_alignbyte(w[r][k + 1], w[r][k], s);
}
template <int NB, int NR>
__device__ __forceinline__ void load_rows(const uint8_t *__restrict__ org, int pitch, int r0, int c,
                                          uint32_t (&out)[NR][(NB + 3) / 4])
{
    uint32_t w[NR][RawRows<NB>::ND + 1];
    const int s = issue_rows<NB, NR>(org, pitch, r0, c, w);
    __builtin_amdgcn_sched_barrier(0);
    align_rows<NB, NR>(w, s, out);
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

// Workgroups of a launch: one per tile (grid = 0), or a persistent grid.
static inline int grid_for(int total, int grid)
{
    if (grid > 0) return grid < total ? grid : (total > 0 ? total : 1);
    return total > 0 ? total : 1;
}

}  // namespace abf
