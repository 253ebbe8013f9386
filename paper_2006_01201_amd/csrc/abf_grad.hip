// Differentiable path of libabf (an extension of the paper's method):
//   - the photometric Charbonnier + TV energy of a flow between two float
//     RGB images, with its gradients with respect to the flow and both
//     images, and a fused gradient-descent step on the flow;
//   - Code 1 over float RGB images and its adjoint with respect to both
//     flows and both images.
// One thread per pixel. Bilinear samples split the displacement into
// floor + fraction (the derivative at an integer position is the
// right-hand one). Scatters into image gradients use float atomics, or,
// in deterministic mode, 64-bit fixed-point integer atomics (exactly
// order-independent) converted to float afterwards.
#include <hip/hip_runtime.h>

#include "abf_device.h"

namespace abf {

namespace {

__device__ __forceinline__ int clampg(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Deterministic scatters add v * scale, rounded, into 64-bit integers. The
// scale is a power of two chosen per call from a bound B on the sum of the
// magnitudes that can reach one pixel (so on every partial sum): 2^(62 - e)
// with B < 2^e, so |sum| * scale < 2^62 never overflows, and each addend
// keeps 62 bits below B. (B is at least 3 times the smallest float, so the
// exponent stays far from the double range.)
__host__ __device__ inline double fix_scale_for(double bound)
{
    int e = 0;
    if (bound > 0.0) (void)frexp(bound, &e);  // bound < 2^e
    return ldexp(1.0, 62 - e);
}

__device__ __forceinline__ void scatter_add(float *g, unsigned long long *gfix, double scale, size_t i, float v)
{
    if (gfix)
        atomicAdd(gfix + i, (unsigned long long)(long long)llrint((double)v * scale));
    else
        atomicAdd(g + i, v);
}

struct Bil {
    int xa, xb, ya, yb;
    float fx, fy;
};

__device__ __forceinline__ Bil bil_at(int x, int y, float ux, float uy, int H, int W)
{
    const float fux = floorf(ux), fuy = floorf(uy);
    const int x0 = x + (int)fux, y0 = y + (int)fuy;
    Bil b;
    b.fx = ux - fux;
    b.fy = uy - fuy;
    b.xa = clampg(x0, 0, W - 1);
    b.xb = clampg(x0 + 1, 0, W - 1);
    b.ya = clampg(y0, 0, H - 1);
    b.yb = clampg(y0 + 1, 0, H - 1);
    return b;
}

// value and position derivatives of channel c of a float HWC image (32-bit
// element offsets: the entry points admit images of 3 H W < 2^32 floats)
__device__ __forceinline__ void bil_eval(const float *img, int W, const Bil &b, int c, float &v, float &dX, float &dY)
{
    const auto g = gld(img);
    const uint32_t ra = (uint32_t)b.ya * (uint32_t)W, rb = (uint32_t)b.yb * (uint32_t)W;
    const uint32_t xa = (uint32_t)b.xa, xb = (uint32_t)b.xb, cc = (uint32_t)c;
    const float v00 = g[3u * (ra + xa) + cc], v01 = g[3u * (ra + xb) + cc];
    const float v10 = g[3u * (rb + xa) + cc], v11 = g[3u * (rb + xb) + cc];
    const float top = v00 + b.fx * (v01 - v00), bot = v10 + b.fx * (v11 - v10);
    v = top + b.fy * (bot - top);
    dX = (1.f - b.fy) * (v01 - v00) + b.fy * (v11 - v10);
    dY = (1.f - b.fx) * (v10 - v00) + b.fx * (v11 - v01);
}

// bil_eval for all three channels: each corner's three floats from one
// base address (merged loads)
__device__ __forceinline__ void bil_eval3(const float *img, int W, const Bil &b, float (&v)[3], float (&dX)[3],
                                          float (&dY)[3])
{
    const auto g = gld(img);
    const uint32_t ra = (uint32_t)b.ya * (uint32_t)W, rb = (uint32_t)b.yb * (uint32_t)W;
    const auto p00 = g + 3u * (ra + (uint32_t)b.xa), p01 = g + 3u * (ra + (uint32_t)b.xb);
    const auto p10 = g + 3u * (rb + (uint32_t)b.xa), p11 = g + 3u * (rb + (uint32_t)b.xb);
    float c00[3], c01[3], c10[3], c11[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        c00[c] = p00[c];
        c01[c] = p01[c];
        c10[c] = p10[c];
        c11[c] = p11[c];
    }
    // d/dX = the row differences lerped by fy; d/dY = bot - top, which
    // equals (1 - fx)(v10 - v00) + fx (v11 - v01)
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const float d0 = c01[c] - c00[c], d1 = c11[c] - c10[c];
        const float top = fmaf(b.fx, d0, c00[c]), bot = fmaf(b.fx, d1, c10[c]);
        const float bt = bot - top;
        v[c] = fmaf(b.fy, bt, top);
        dX[c] = fmaf(b.fy, d1 - d0, d0);
        dY[c] = bt;
    }
}

__device__ __forceinline__ void bil_scatter(float *g, unsigned long long *gfix, double scale, int W, const Bil &b,
                                            int c, float w)
{
    scatter_add(g, gfix, scale, 3 * ((size_t)b.ya * W + b.xa) + c, w * (1.f - b.fy) * (1.f - b.fx));
    scatter_add(g, gfix, scale, 3 * ((size_t)b.ya * W + b.xb) + c, w * (1.f - b.fy) * b.fx);
    scatter_add(g, gfix, scale, 3 * ((size_t)b.yb * W + b.xa) + c, w * b.fy * (1.f - b.fx));
    scatter_add(g, gfix, scale, 3 * ((size_t)b.yb * W + b.xb) + c, w * b.fy * b.fx);
}

// 1 / sqrt(v) for v >= FLT_MIN (v_rsq_f32, within 1 ulp; the entry points
// reject an eps whose square is below FLT_MIN, so every argument is a
// normal number): the gradient's quotients r / rho and d / s; the energy
// keeps the rounded square roots
__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }

// rho'(r) = r / sqrt(r^2 + eps^2), the Charbonnier derivative (both the
// flow gradient and the image gradients use this one form)
__device__ __forceinline__ float charb_d(float r, float eps) { return r * rsq(r * r + eps * eps); }

// dE/du at p (photometric + lambda * TV); also returns the pixel's energy.
// The flow is read as float pairs at p and at its neighbours p +- 1,
// p +- W, p - 1 + W and p + 1 - W (32-bit element offsets: 3 H W < 2^32).
__device__ __forceinline__ void grad_u_at(const float *Ref, const float *Tgt, const float *u, int H, int W, int x,
                                          int y, float lambda, float eps, float &gx, float &gy, double &e)
{
    const uint32_t p = (uint32_t)y * (uint32_t)W + (uint32_t)x, w = (uint32_t)W;
    const auto gr = gld(Ref);
    const auto g2 = gld(reinterpret_cast<const uint64_t *>(u));
    auto pair = [&](uint32_t i) {
        const uint64_t v = g2[i];
        return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
    };
    const float2 c = pair(p);
    const Bil b = bil_at(x, y, c.x, c.y, H, W);
    gx = gy = 0.f;
    e = 0.0;
    float v[3], dX[3], dY[3];
    bil_eval3(Tgt, W, b, v, dX, dY);
    const auto rp = gr + 3u * p;
    const float rv[3] = {rp[0], rp[1], rp[2]};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const float r = v[k] - rv[k];
        const float d = charb_d(r, eps);
        e += sqrtf(r * r + eps * eps);
        gx = fmaf(d, dX[k], gx);
        gy = fmaf(d, dY[k], gy);
    }
    // TV: s(q)^2 = dx^2 + dy^2 + eps^2 with forward differences (0 past the
    // last column / row) at q = p, p - 1 and p - W
    const bool xr = x < W - 1, yd = y < H - 1, xl = x > 0, yu = y > 0;
    const float2 rt = xr ? pair(p + 1) : c, dn = yd ? pair(p + w) : c;
    const float2 lf = xl ? pair(p - 1) : c, ld = xl && yd ? pair(p - 1 + w) : c;
    const float2 up = yu ? pair(p - w) : c, ur = yu && xr ? pair(p + 1 - w) : c;
#pragma unroll
    for (int m = 0; m < 2; m++) {
        const float cm = m ? c.y : c.x;
        const float dx = xr ? (m ? rt.y : rt.x) - cm : 0.f, dy = yd ? (m ? dn.y : dn.x) - cm : 0.f;
        const float s2 = dx * dx + dy * dy + eps * eps;
        e += (double)lambda * sqrtf(s2);
        float g = -(dx + dy) * rsq(s2);
        if (xl) {
            const float lm = m ? lf.y : lf.x;
            const float ddx = cm - lm, ddy = yd ? (m ? ld.y : ld.x) - lm : 0.f;
            const float sl2 = ddx * ddx + ddy * ddy + eps * eps;
            g = fmaf(ddx, rsq(sl2), g);
        }
        if (yu) {
            const float um = m ? up.y : up.x;
            const float ddx = xr ? (m ? ur.y : ur.x) - um : 0.f, ddy = cm - um;
            const float su2 = ddx * ddx + ddy * ddy + eps * eps;
            g = fmaf(ddy, rsq(su2), g);
        }
        if (m == 0) gx = fmaf(lambda, g, gx);
        else gy = fmaf(lambda, g, gy);
    }
}

constexpr int kEB = 256;

__global__ __launch_bounds__(kEB) void k_energy(const float *__restrict__ Ref, const float *__restrict__ Tgt,
                                                const float *__restrict__ u, int H, int W, float lambda, float eps,
                                                double *__restrict__ partials, float *__restrict__ g_u,
                                                float *__restrict__ g_ref, float *g_tgt, unsigned long long *g_fix,
                                                double fix_scale)
{
    __shared__ double red[kEB];
    const uint32_t n = (uint32_t)H * (uint32_t)W;
    double acc = 0.0;
    for (uint32_t p = blockIdx.x * (uint32_t)kEB + threadIdx.x; p < n; p += gridDim.x * (uint32_t)kEB) {
        const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * (uint32_t)W);
        float gx, gy;
        double e;
        grad_u_at(Ref, Tgt, u, H, W, x, y, lambda, eps, gx, gy, e);
        acc += e;
        if (g_u) {
            g_u[2 * p] = gx;
            g_u[2 * p + 1] = gy;
        }
        if (g_ref || g_tgt || g_fix) {
            const Bil b = bil_at(x, y, u[2 * p], u[2 * p + 1], H, W);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                float v, dX, dY;
                bil_eval(Tgt, W, b, c, v, dX, dY);
                const float d = charb_d(v - Ref[3 * p + c], eps);
                if (g_ref) g_ref[3 * p + c] = -d;
                if (g_tgt || g_fix) bil_scatter(g_tgt, g_fix, fix_scale, W, b, c, d);
            }
        }
    }
    if (!partials) return;  // gradients only (uniform)
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kEB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kEB) void k_sum_partials(const double *__restrict__ partials, int n, float *E)
{
    __shared__ double red[kEB];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kEB) acc += partials[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kEB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *E = (float)red[0];
}

__global__ __launch_bounds__(64) void k_zero_u32(uint32_t *a)
{
    if (threadIdx.x == 0) *a = 0u;
}

__global__ __launch_bounds__(256) void k_fill_zero(float *a, unsigned long long *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (a) a[i] = 0.f;
        if (b) b[i] = 0ull;
    }
}

// scale: the fixed-point scale itself, or, with gmax, the scale for the
// bound (largest |g_F|, as float bits) * fan
__global__ __launch_bounds__(256) void k_fix_to_float(const unsigned long long *__restrict__ b, float *a, int64_t n,
                                                      double scale, const uint32_t *__restrict__ gmax, double fan)
{
    if (gmax) scale = fix_scale_for((double)__uint_as_float(*gmax) * fan);
    const double inv = 1.0 / scale;  // a power of two: exact
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        a[i] = (float)((double)(long long)b[i] * inv);
}

// largest |v| over n floats, as float bits (an unsigned max of the bits of
// non-negative floats orders them; the result does not depend on the
// order); *out must start at 0
__global__ __launch_bounds__(256) void k_absmax(const float *__restrict__ v, int64_t n, uint32_t *out)
{
    uint32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = max(m, __float_as_uint(v[i]) & 0x7fffffffu);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
    if ((threadIdx.x & 63) == 0 && m) atomicMax(out, m);
}

__global__ __launch_bounds__(256) void k_energy_step(const float *__restrict__ Ref, const float *__restrict__ Tgt,
                                                     const float *__restrict__ u_in, float *__restrict__ u_out, int H,
                                                     int W, float eta, float lambda, float eps, float clip)
{
    const uint32_t n = (uint32_t)H * (uint32_t)W;
    for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < n; p += gridDim.x * 256u) {
        const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * (uint32_t)W);
        float gx, gy;
        double e;
        grad_u_at(Ref, Tgt, u_in, H, W, x, y, lambda, eps, gx, gy, e);
        const float sx = fminf(fmaxf(eta * gx, -clip), clip), sy = fminf(fmaxf(eta * gy, -clip), clip);
        const uint64_t w = gld(reinterpret_cast<const uint64_t *>(u_in))[p];
        const float ax = __uint_as_float((uint32_t)w) - sx, ay = __uint_as_float((uint32_t)(w >> 32)) - sy;
        gst(reinterpret_cast<uint64_t *>(u_out))[p] =
            (uint64_t)__float_as_uint(ax) | ((uint64_t)__float_as_uint(ay) << 32);
    }
}

// --- Code 1 on float images ------------------------------------------
struct Setup {
    Bil bl, br;
    double t, nrl, nlr;
    float rl[2], lr[2];
    bool okrl[2], oklr[2];
    float sL;
};

__device__ __forceinline__ Setup code1_setup(int x, int y, int H, int W, int axis, const float *blend,
                                             const float *flr, const float *frl, BlendParams bp)
{
    Setup s;
    const size_t p = (size_t)y * W + x;
    s.t = blend ? (double)blend[p] : (axis == 0 ? (x + 1.0) / (W + 1.0) : (y + 1.0) / (H + 1.0));
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const float a = frl[2 * p + k], b = flr[2 * p + k];
        s.okrl[k] = isfinite(a);
        s.oklr[k] = isfinite(b);
        s.rl[k] = s.okrl[k] ? a : 0.f;
        s.lr[k] = s.oklr[k] ? b : 0.f;
    }
    const double ax = s.rl[0] * s.t, ay = s.rl[1] * s.t, bx = s.lr[0] * (1.0 - s.t), by = s.lr[1] * (1.0 - s.t);
    const double fax = floor(ax), fay = floor(ay), fbx = floor(bx), fby = floor(by);
    auto mk = [&](int x0, int y0, float fx, float fy) {
        Bil b;
        b.fx = fx;
        b.fy = fy;
        b.xa = clampg(x0, 0, W - 1);
        b.xb = clampg(x0 + 1, 0, W - 1);
        b.ya = clampg(y0, 0, H - 1);
        b.yb = clampg(y0 + 1, 0, H - 1);
        return b;
    };
    s.bl = mk(x + (int)fax, y + (int)fay, (float)(ax - fax), (float)(ay - fay));
    s.br = mk(x + (int)fbx, y + (int)fby, (float)(bx - fbx), (float)(by - fby));
    s.nrl = sqrt((double)s.rl[0] * s.rl[0] + (double)s.rl[1] * s.rl[1]);
    s.nlr = sqrt((double)s.lr[0] * s.lr[0] + (double)s.lr[1] * s.lr[1]);
    if (bp.mode == 1) {
        s.sL = (float)(1.0 - s.t);
    } else {
        const double S = axis == 0 ? (double)W : (double)H;
        const double zL = (double)bp.k_sharp * (1.0 - s.t) * (1.0 + (double)bp.k_flowmag * s.nrl / S);
        const double zR = (double)bp.k_sharp * s.t * (1.0 + (double)bp.k_flowmag * s.nlr / S);
        s.sL = 1.0f / (1.0f + expf((float)(zR - zL)));
    }
    return s;
}

__global__ __launch_bounds__(256) void k_blend_f32(const float *__restrict__ L, const float *__restrict__ R,
                                                   const float *__restrict__ flr, const float *__restrict__ frl,
                                                   const float *__restrict__ blend, int axis, int H, int W,
                                                   BlendParams bp, float *__restrict__ F)
{
    const int64_t n = (int64_t)H * W;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const Setup s = code1_setup(x, y, H, W, axis, blend, flr, frl, bp);
        const float sR = 1.f - s.sL;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            float cl, cr, d0, d1;
            bil_eval(L, W, s.bl, c, cl, d0, d1);
            bil_eval(R, W, s.br, c, cr, d0, d1);
            F[3 * p + c] = s.sL * cl + sR * cr;
        }
    }
}

__global__ __launch_bounds__(256) void k_blend_bwd(const float *__restrict__ L, const float *__restrict__ R,
                                                   const float *__restrict__ flr, const float *__restrict__ frl,
                                                   const float *__restrict__ blend, int axis, int H, int W,
                                                   BlendParams bp, const float *__restrict__ gF,
                                                   float *__restrict__ g_flr, float *__restrict__ g_frl, float *g_L,
                                                   float *g_R, unsigned long long *fixL, unsigned long long *fixR,
                                                   const uint32_t *__restrict__ gmax)
{
    const int64_t n = (int64_t)H * W;
    // every (pixel, channel) of g_F adds at most |g_F| (weights sL, sR and
    // the bilinear weights are <= 1 and sum to <= 1) into an image gradient
    const double scale = gmax ? fix_scale_for((double)__uint_as_float(*gmax) * 3.0 * (double)n) : 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const Setup s = code1_setup(x, y, H, W, axis, blend, flr, frl, bp);
        const float sL = s.sL, sR = 1.f - s.sL;
        float gs = 0.f, gLx = 0.f, gLy = 0.f, gRx = 0.f, gRy = 0.f;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            float cl, cr, lX, lY, rX, rY;
            bil_eval(L, W, s.bl, c, cl, lX, lY);
            bil_eval(R, W, s.br, c, cr, rX, rY);
            const float g = gF[3 * p + c];
            gs = fmaf(g, cl - cr, gs);
            gLx = fmaf(g * sL, lX, gLx);
            gLy = fmaf(g * sL, lY, gLy);
            gRx = fmaf(g * sR, rX, gRx);
            gRy = fmaf(g * sR, rY, gRy);
            if (g_L || fixL) bil_scatter(g_L, fixL, scale, W, s.bl, c, g * sL);
            if (g_R || fixR) bil_scatter(g_R, fixR, scale, W, s.br, c, g * sR);
        }
        const float t = (float)s.t;
        float grl_x = t * gLx, grl_y = t * gLy, glr_x = (1.f - t) * gRx, glr_y = (1.f - t) * gRy;
        if (bp.mode != 1) {
            const double S = axis == 0 ? (double)W : (double)H;
            const double dz = (double)gs * (double)sL * (double)sR;
            if (s.nrl > 0) {
                const double k = dz * bp.k_sharp * (1.0 - s.t) * bp.k_flowmag / S / s.nrl;
                grl_x += (float)(k * s.rl[0]);
                grl_y += (float)(k * s.rl[1]);
            }
            if (s.nlr > 0) {
                const double k = -dz * bp.k_sharp * s.t * bp.k_flowmag / S / s.nlr;
                glr_x += (float)(k * s.lr[0]);
                glr_y += (float)(k * s.lr[1]);
            }
        }
        if (g_frl) {
            g_frl[2 * p] = s.okrl[0] ? grl_x : 0.f;
            g_frl[2 * p + 1] = s.okrl[1] ? grl_y : 0.f;
        }
        if (g_flr) {
            g_flr[2 * p] = s.oklr[0] ? glr_x : 0.f;
            g_flr[2 * p + 1] = s.oklr[1] ? glr_y : 0.f;
        }
    }
}

// Batched descent step over many strips: one launch per step, a flat list
// of 256-pixel tiles over all strips (prefix sums per strip); u[in] is
// read, u[1 - in] written.
__global__ __launch_bounds__(256) void k_energy_step_batch(const RefineDesc *__restrict__ d,
                                                           const int32_t *__restrict__ prefix, int n, int total,
                                                           int in, float eta, float lambda, float eps, float clip)
{
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const RefineDesc &r = d[lo];
        const uint32_t p = (uint32_t)(t - prefix[lo]) * 256u + threadIdx.x;
        if (p >= (uint32_t)r.H * (uint32_t)r.W) continue;
        const int y = (int)(p / (uint32_t)r.W), x = (int)(p - (uint32_t)y * (uint32_t)r.W);
        const float *u_in = r.u[in];
        float *u_out = r.u[1 - in];
        float gx, gy;
        double e;
        grad_u_at(r.Ref, r.Tgt, u_in, r.H, r.W, x, y, lambda, eps, gx, gy, e);
        const float sx = fminf(fmaxf(eta * gx, -clip), clip), sy = fminf(fmaxf(eta * gy, -clip), clip);
        const uint64_t w = gld(reinterpret_cast<const uint64_t *>(u_in))[p];
        const float ax = __uint_as_float((uint32_t)w) - sx, ay = __uint_as_float((uint32_t)(w >> 32)) - sy;
        gst(reinterpret_cast<uint64_t *>(u_out))[p] =
            (uint64_t)__float_as_uint(ax) | ((uint64_t)__float_as_uint(ay) << 32);
    }
}

__global__ __launch_bounds__(256) void k_copy_back_batch(const RefineDesc *__restrict__ d,
                                                         const int32_t *__restrict__ prefix, int n, int total)
{
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const RefineDesc &r = d[lo];
        const int64_t p = (int64_t)(t - prefix[lo]) * 256 + threadIdx.x;
        if (p >= (int64_t)r.H * r.W) continue;
        r.u[0][2 * p] = r.u[1][2 * p];
        r.u[0][2 * p + 1] = r.u[1][2 * p + 1];
    }
}

// --- multi-level energy: float pyramid and its adjoint ----------------
// One level of the float pyramid of a C-channel HWC array: the 5 x 5
// binomial filter (w_i w_j / 256, w = 1 4 6 4 1) with clamped indices,
// decimated by 2, times `scale` (1 for images; 1/2 for a flow, whose
// displacements halve with the pixels). One thread per output pixel.
__device__ __forceinline__ float binom(int i) { return i == 2 ? 6.f : (i == 1 || i == 3) ? 4.f : 1.f; }

template <int C>
__global__ __launch_bounds__(256) void k_pyr_down_f32(const float *__restrict__ x, int H, int W, float *__restrict__ y,
                                                      int h, int w, float scale)
{
    const int64_t n = (int64_t)h * w;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int Y = (int)(p / w), X = (int)(p - (int64_t)Y * w);
        float acc[C] = {};
#pragma unroll
        for (int j = 0; j < 5; j++) {
            const int r = clampg(2 * Y + j - 2, 0, H - 1);
            float row[C] = {};
#pragma unroll
            for (int i = 0; i < 5; i++) {
                const int c0 = clampg(2 * X + i - 2, 0, W - 1);
                const float wi = binom(i);
#pragma unroll
                for (int c = 0; c < C; c++) row[c] = fmaf(wi, gld(x)[C * ((size_t)r * W + c0) + c], row[c]);
            }
#pragma unroll
            for (int c = 0; c < C; c++) acc[c] = fmaf(binom(j), row[c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < C; c++) gst(y)[C * p + c] = acc[c] * (scale / 256.f);
    }
}

// The coarse indices X of a fine index x that k_pyr_down_f32's taps reach,
// with the summed tap weights (clamped taps pile up on the border): at
// most three, from X in [floor((x - 2) / 2), floor((x + 2) / 2)].
struct Taps {
    int n, X[3];
    float w[3];
};
__device__ __forceinline__ Taps adj_taps(int x, int N, int n)
{
    Taps t;
    t.n = 0;
    const int lo = max(0, (x - 2) >> 1), hi = min(n - 1, (x + 2) >> 1);
    for (int X = lo; X <= hi; X++) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < 5; i++)
            if (clampg(2 * X + i - 2, 0, N - 1) == x) s += binom(i);
        if (s != 0.f) {
            t.X[t.n] = X;
            t.w[t.n] = s;
            t.n++;
        }
    }
    return t;
}

// g += scale * adjoint(k_pyr_down_f32)(G): every fine pixel gathers the
// coarse values its taps fed, with their weights (the transpose of the
// filter and decimation). G: h x w x C, g: H x W x C.
template <int C>
__global__ __launch_bounds__(256) void k_pyr_adj_add_f32(const float *__restrict__ G, int h, int w,
                                                         float *__restrict__ g, int H, int W, float scale)
{
    const int64_t n = (int64_t)H * W;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const Taps ty = adj_taps(y, H, h), tx = adj_taps(x, W, w);
        float acc[C] = {};
        for (int a = 0; a < ty.n; a++) {
            float row[C] = {};
            for (int b = 0; b < tx.n; b++) {
#pragma unroll
                for (int c = 0; c < C; c++)
                    row[c] = fmaf(tx.w[b], gld(G)[C * ((size_t)ty.X[a] * w + tx.X[b]) + c], row[c]);
            }
#pragma unroll
            for (int c = 0; c < C; c++) acc[c] = fmaf(ty.w[a], row[c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < C; c++) g[C * p + c] = fmaf(acc[c], scale / 256.f, g[C * p + c]);
    }
}

// E = the sum of the n per-level energies (in double)
__global__ __launch_bounds__(64) void k_sum_levels(const float *__restrict__ El, int n, float *E)
{
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < n; k++) s += (double)El[k];
        *E = (float)s;
    }
}

// u <- u - clip(eta g, -clip, clip), per component
__global__ __launch_bounds__(256) void k_clip_step(float *__restrict__ u, const float *__restrict__ g, int64_t n,
                                                   float eta, float clip)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        u[i] -= fminf(fmaxf(eta * g[i], -clip), clip);
}

inline int blocks_for(int64_t n, int per = 256, int cap = 65536)
{
    int64_t b = (n + per - 1) / per;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

int energy_blocks(int H, int W) { return blocks_for((int64_t)H * W, kEB, 4096); }

// partials: energy_blocks doubles; fix: 3 H W uint64 (deterministic only)
hipError_t launch_energy_full(const float *Ref, const float *Tgt, const float *u, int H, int W, float lambda,
                              float eps, double *partials, float *E, float *g_u, float *g_ref, float *g_tgt,
                              unsigned long long *fix, hipStream_t s)
{
    const int64_t n3 = (int64_t)H * W * 3;
    const int nb = energy_blocks(H, W);
    if (g_tgt) {
        hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(n3)), dim3(256), 0, s, fix ? nullptr : g_tgt, fix, n3);
    }
    // |rho'| <= 1 and the bilinear weights sum to 1: no pixel of dE/dTgt
    // exceeds 3 H W in magnitude
    const double scale = fix_scale_for((double)n3);
    hipLaunchKernelGGL(k_energy, dim3(nb), dim3(kEB), 0, s, Ref, Tgt, u, H, W, lambda, eps, partials, g_u, g_ref,
                       fix ? nullptr : g_tgt, g_tgt ? fix : nullptr, scale);
    if (partials) hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kEB), 0, s, partials, nb, E);
    if (g_tgt && fix)
        hipLaunchKernelGGL(k_fix_to_float, dim3(blocks_for(n3)), dim3(256), 0, s, fix, g_tgt, n3, scale,
                           (const uint32_t *)nullptr, 0.0);
    return hipGetLastError();
}

hipError_t launch_pyr_down_f32(const float *x, int C, int H, int W, float *y, float scale, hipStream_t s)
{
    const int h = (H + 1) / 2, w = (W + 1) / 2;
    const dim3 g(blocks_for((int64_t)h * w));
    if (C == 3) hipLaunchKernelGGL(k_pyr_down_f32<3>, g, dim3(256), 0, s, x, H, W, y, h, w, scale);
    else hipLaunchKernelGGL(k_pyr_down_f32<2>, g, dim3(256), 0, s, x, H, W, y, h, w, scale);
    return hipGetLastError();
}

hipError_t launch_pyr_adj_add_f32(const float *G, int C, int H, int W, float *g, float scale, hipStream_t s)
{
    const int h = (H + 1) / 2, w = (W + 1) / 2;
    const dim3 gr(blocks_for((int64_t)H * W));
    if (C == 3) hipLaunchKernelGGL(k_pyr_adj_add_f32<3>, gr, dim3(256), 0, s, G, h, w, g, H, W, scale);
    else hipLaunchKernelGGL(k_pyr_adj_add_f32<2>, gr, dim3(256), 0, s, G, h, w, g, H, W, scale);
    return hipGetLastError();
}

hipError_t launch_sum_levels(const float *El, int n, float *E, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_levels, dim3(1), dim3(64), 0, s, El, n, E);
    return hipGetLastError();
}

hipError_t launch_clip_step(float *u, const float *g, int64_t n, float eta, float clip, hipStream_t s)
{
    hipLaunchKernelGGL(k_clip_step, dim3(blocks_for(n)), dim3(256), 0, s, u, g, n, eta, clip);
    return hipGetLastError();
}

hipError_t launch_energy_step(const float *Ref, const float *Tgt, const float *u_in, float *u_out, int H, int W,
                              float eta, float lambda, float eps, float clip, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_step, dim3(blocks_for((int64_t)H * W)), dim3(256), 0, s, Ref, Tgt, u_in, u_out, H,
                       W, eta, lambda, eps, clip);
    return hipGetLastError();
}

hipError_t launch_refine_batch(const RefineDesc *d, const int32_t *prefix, int n, int total, int steps, float eta,
                               float lambda, float eps, float clip, hipStream_t s)
{
    const int g = total < 65536 ? (total > 0 ? total : 1) : 65536;
    for (int k = 0; k < steps; k++)
        hipLaunchKernelGGL(k_energy_step_batch, dim3(g), dim3(256), 0, s, d, prefix, n, total, k & 1, eta, lambda,
                           eps, clip);
    if (steps & 1) hipLaunchKernelGGL(k_copy_back_batch, dim3(g), dim3(256), 0, s, d, prefix, n, total);
    return hipGetLastError();
}

hipError_t launch_copy_f32(const float *src, float *dst, int64_t n, hipStream_t s)
{
    return hipMemcpyAsync(dst, src, sizeof(float) * n, hipMemcpyDeviceToDevice, s);
}

hipError_t launch_blend_f32(const float *L, const float *R, const float *flr, const float *frl, const float *blend,
                            int axis, int H, int W, BlendParams bp, float *F, hipStream_t s)
{
    hipLaunchKernelGGL(k_blend_f32, dim3(blocks_for((int64_t)H * W)), dim3(256), 0, s, L, R, flr, frl, blend, axis,
                       H, W, bp, F);
    return hipGetLastError();
}

hipError_t launch_blend_bwd_full(const float *L, const float *R, const float *flr, const float *frl,
                                 const float *blend, int axis, int H, int W, BlendParams bp, const float *gF,
                                 float *g_flr, float *g_frl, float *g_L, float *g_R, unsigned long long *fixL,
                                 unsigned long long *fixR, uint32_t *gmax, hipStream_t s)
{
    const int64_t n3 = (int64_t)H * W * 3;
    const bool det = gmax && (g_L || g_R);
    if (det) {
        // the fixed-point scale follows the largest |g_F|, found on the device
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, gmax);
        hipLaunchKernelGGL(k_absmax, dim3(blocks_for(n3, 256, 2048)), dim3(256), 0, s, gF, n3, gmax);
    }
    if (g_L) hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(n3)), dim3(256), 0, s, det ? nullptr : g_L,
                                det ? fixL : nullptr, n3);
    if (g_R) hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(n3)), dim3(256), 0, s, det ? nullptr : g_R,
                                det ? fixR : nullptr, n3);
    hipLaunchKernelGGL(k_blend_bwd, dim3(blocks_for((int64_t)H * W)), dim3(256), 0, s, L, R, flr, frl, blend, axis,
                       H, W, bp, gF, g_flr, g_frl, det ? nullptr : g_L, det ? nullptr : g_R,
                       (det && g_L) ? fixL : nullptr, (det && g_R) ? fixR : nullptr,
                       det ? (const uint32_t *)gmax : nullptr);
    const double fan = 3.0 * (double)H * W;
    if (det && g_L)
        hipLaunchKernelGGL(k_fix_to_float, dim3(blocks_for(n3)), dim3(256), 0, s, fixL, g_L, n3, 0.0,
                           (const uint32_t *)gmax, fan);
    if (det && g_R)
        hipLaunchKernelGGL(k_fix_to_float, dim3(blocks_for(n3)), dim3(256), 0, s, fixR, g_R, n3, 0.0,
                           (const uint32_t *)gmax, fan);
    return hipGetLastError();
}

}  // namespace abf
