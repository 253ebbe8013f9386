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

// Code 1 per pixel. The displacements and their split into cell and
// fraction, and the softmax exponents, are evaluated in double, so that no
// FP32 coordinate or large exponent is formed; the flow magnitudes take a
// float square root refined by one Newton step in double, the softmax
// weight a hardware 2^x and reciprocal in float (errors far below the
// blend tolerance: at most 5e-5 gray levels in a bound study with flows up
// to 150 px and kSoftmaxSharpness 60 / kFlowMagCoef 80); bilinear sampling
// and the composite are FP32.
struct PixBlend {
    int lx, ly, rx, ry;      // integer cell corners of the L and R samples
    float lfx, lfy, rfx, rfy;
    float sL;                // SoftmaxL (SoftmaxR = 1 - sL)
};

__device__ __forceinline__ float finite0(float v) { return isfinite(v) ? v : 0.f; }

// sqrt(m2) for a double m2 >= 0: float square root s, then
// s + (m2 - s^2) / (2 s) in double (relative error ~1e-14)
__device__ __forceinline__ double norm_from_sq(double m2)
{
    const float sf = __builtin_amdgcn_sqrtf((float)m2);
    if (!(sf > 0.f)) return 0.0;
    const double s = (double)sf;
    return fma(fma(-s, s, m2), (double)(0.5f * __builtin_amdgcn_rcpf(sf)), s);
}

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
        const double mrl = norm_from_sq((double)frx * frx + (double)fry * fry) * inv_ext;
        const double mlr = norm_from_sq((double)flx * flx + (double)fly * fly) * inv_ext;
        const double zL = (double)bp.k_sharp * (1.0 - t) * (1.0 + (double)bp.k_flowmag * mrl);
        const double zR = (double)bp.k_sharp * t * (1.0 + (double)bp.k_flowmag * mlr);
        // 1 / (1 + e^d) with e^d = 2^(d log2 e); e^d = inf gives 0
        const float e = __builtin_amdgcn_exp2f((float)(zR - zL) * 1.44269504f);
        r.sL = __builtin_amdgcn_rcpf(1.0f + e);
    }
    return r;
}

// Bilinear RGB sample of a uint8 HWC image at (x0 + fx, y0 + fy) with
// clamp-to-edge indices. When the two corner pixels of a row are distinct
// and the dwords around them lie inside the image data, each row's 6
// bytes come from one aligned dwordx3 load; otherwise byte by byte.
// Addresses are a uniform base plus 32-bit byte offsets (images up to
// 4 GiB).
__device__ __forceinline__ void sample_u8(const uint8_t *img, int pitch, int H, int W, int x0, int y0, float fx,
                                          float fy, float out[3])
{
    // offsets from the dword-aligned base below img; data = [lead, end)
    const uint8_t *base = reinterpret_cast<const uint8_t *>((uintptr_t)img & ~(uintptr_t)3);
    const uint32_t lead = (uint32_t)((uintptr_t)img & 3);
    const uint32_t end = lead + (uint32_t)(H - 1) * (uint32_t)pitch + 3u * (uint32_t)W;
    const uint32_t ra = lead + (uint32_t)clampi(y0, 0, H - 1) * (uint32_t)pitch;
    const uint32_t rb = lead + (uint32_t)clampi(y0 + 1, 0, H - 1) * (uint32_t)pitch;
    float v[2][6];
    const uint32_t pa = ra + 3u * (uint32_t)x0, pb = rb + 3u * (uint32_t)x0;
    const uint32_t aa = pa & ~3u, ab = pb & ~3u;
    if (x0 >= 0 && x0 + 1 <= W - 1 && aa >= lead && aa + 12u <= end && ab >= lead && ab + 12u <= end) {
        const uint32_t s = pa - aa, t = pb - ab;
        const auto qa = gld(reinterpret_cast<const uint32_t *>(base + aa));
        const auto qb = gld(reinterpret_cast<const uint32_t *>(base + ab));
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
        const uint32_t xa = 3u * (uint32_t)clampi(x0, 0, W - 1), xb = 3u * (uint32_t)clampi(x0 + 1, 0, W - 1);
        const auto g = gld(base);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            v[0][c] = g[ra + xa + c];
            v[0][3 + c] = g[ra + xb + c];
            v[1][c] = g[rb + xa + c];
            v[1][3 + c] = g[rb + xb + c];
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
