// Device helpers shared by the kernel files of libabf (not part of the
// public ABI).
#pragma once

#include "abf_internal.h"

namespace abf {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

typedef const __attribute__((address_space(1))) uint32_t gu32;

// The buffers are plain device memory: accessing them through global
// (rather than generic) pointers makes the loads count on vmcnt only, so
// waits for them do not also wait for LDS traffic and vice versa.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gld(const T *p)
{
    return (const __attribute__((address_space(1))) T *)(const void *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gst(T *p)
{
    return (__attribute__((address_space(1))) T *)(void *)p;
}

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

// (x, y): the pixel in the crop that the images and flows cover; t: its
// Blend; p: its index in the flow arrays; inv_ext: 1 / the crop's extent
// across the seam (flow magnitude scale).
__device__ __forceinline__ PixBlend blend_setup(int x, int y, double t, uint32_t p, double inv_ext, const float *flr,
                                                const float *frl, BlendParams bp)
{
    const uint64_t vrl = gld(reinterpret_cast<const uint64_t *>(frl))[p];
    const uint64_t vlr = gld(reinterpret_cast<const uint64_t *>(flr))[p];
    const float frx = finite0(__uint_as_float((uint32_t)vrl)), fry = finite0(__uint_as_float((uint32_t)(vrl >> 32)));
    const float flx = finite0(__uint_as_float((uint32_t)vlr)), fly = finite0(__uint_as_float((uint32_t)(vlr >> 32)));
    // displacements in double (split into cell and fraction exactly)
    const double ax = (double)frx * t, ay = (double)fry * t, bx = (double)flx * (1.0 - t), by = (double)fly * (1.0 - t);
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
        // the exponents in double: with large flows both can be in the
        // hundreds and nearly equal, where FP32 rounding would move F
        const double mrl = sqrt((double)frx * frx + (double)fry * fry) * inv_ext;
        const double mlr = sqrt((double)flx * flx + (double)fly * fly) * inv_ext;
        const double zL = (double)bp.k_sharp * (1.0 - t) * (1.0 + (double)bp.k_flowmag * mrl);
        const double zR = (double)bp.k_sharp * t * (1.0 + (double)bp.k_flowmag * mlr);
        r.sL = 1.0f / (1.0f + expf((float)(zR - zL)));
    }
    return r;
}

// Bilinear RGB sample of a uint8 HWC image at (x0 + fx, y0 + fy) with
// clamp-to-edge indices. When the two corner pixels of a row are distinct
// and the dwords around them lie inside the image data, each row's 6
// bytes come from one aligned dwordx3 load; otherwise byte by byte.
__device__ __forceinline__ void sample_u8(const uint8_t *img, int pitch, int H, int W, int x0, int y0, float fx,
                                          float fy, float out[3])
{
    const uint8_t *ra = img + (size_t)clampi(y0, 0, H - 1) * pitch;
    const uint8_t *rb = img + (size_t)clampi(y0 + 1, 0, H - 1) * pitch;
    float v[2][6];
    const uintptr_t lo = (uintptr_t)img, hi = (uintptr_t)(img + (size_t)(H - 1) * pitch + 3 * (size_t)W);
    const uintptr_t pa = (uintptr_t)(ra + 3 * x0), pb = (uintptr_t)(rb + 3 * x0);
    const uintptr_t aa = pa & ~(uintptr_t)3, ab = pb & ~(uintptr_t)3;
    if (x0 >= 0 && x0 + 1 <= W - 1 && aa >= lo && aa + 12 <= hi && ab >= lo && ab + 12 <= hi) {
        const int s = (int)(pa - aa), t = (int)(pb - ab);
        const auto qa = reinterpret_cast<const __attribute__((address_space(1))) uint32_t *>(aa);
        const auto qb = reinterpret_cast<const __attribute__((address_space(1))) uint32_t *>(ab);
        const uint32_t a0 = qa[0], a1 = qa[1], a2 = qa[2], b0 = qb[0], b1 = qb[1], b2 = qb[2];
        const uint32_t ua = __builtin_amdgcn_alignbyte(a1, a0, s), wa = __builtin_amdgcn_alignbyte(a2, a1, s);
        const uint32_t ub = __builtin_amdgcn_alignbyte(b1, b0, t), wb = __builtin_amdgcn_alignbyte(b2, b1, t);
#pragma unroll
        for (int c = 0; c < 4; c++) {
            v[0][c] = (float)((ua >> (8 * c)) & 0xffu);
            v[1][c] = (float)((ub >> (8 * c)) & 0xffu);
        }
#pragma unroll
        for (int c = 0; c < 2; c++) {
            v[0][4 + c] = (float)((wa >> (8 * c)) & 0xffu);
            v[1][4 + c] = (float)((wb >> (8 * c)) & 0xffu);
        }
    } else {
        const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            v[0][c] = ra[3 * xa + c];
            v[0][3 + c] = ra[3 * xb + c];
            v[1][c] = rb[3 * xa + c];
            v[1][3 + c] = rb[3 * xb + c];
        }
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const float top = v[0][c] + fx * (v[0][3 + c] - v[0][c]);
        const float bot = v[1][c] + fx * (v[1][3 + c] - v[1][c]);
        out[c] = top + fy * (bot - top);
    }
}

}  // namespace abf
