"""Error bound of the refinement's FP32 solve (the device computes the
bilinear mix of the corner correlations, the 2x2 inverse with a
compensated determinant, and the step in FP32; the oracle in FP64).

The step is d = -H^-1 (b / 2) with H = sum g g^T / 4 + eps I: where the
window's gradients are nearly parallel one eigenvalue of H is close to
eps, and FP32 rounding of b and of the inverse is amplified by up to
|b| / eps. This test re-evaluates one step both ways (FP32 with every
rounding and fused multiply-add of the device arithmetic, FP64 as the
oracle) on adversarial windows: gradients of magnitude 50..255 along one
direction with 0..20 of noise across it, and residuals drawn at full scale
(+-255) at every sample, the largest |b| the 8-bit data allow. Every step
the +-1 px clamp keeps must agree within 1e-3 px, a tenth of the flow
tolerance (measured over 12 M such windows: 6.2e-4 px at most; on the
synthetic parity and full-size cases the GPU stays within 2.5e-5 px of
the oracle after both steps)."""
import numpy as np
import pytest

EPS = 25.0


def r32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def fma32(a, b, c):
    # a * b is exact in float64 for float32 a, b; one rounding to float32
    return r32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def step64(hxx, hxy, hyy, c, fx, fy):
    Hxx, Hxy, Hyy = 0.25 * hxx + EPS, 0.25 * hxy, 0.25 * hyy + EPS
    hdet = 0.5 / (Hxx * Hyy - Hxy * Hxy)

    def mix(v):
        t = v[:, 0] + fx * (v[:, 1] - v[:, 0])
        b = v[:, 2] + fx * (v[:, 3] - v[:, 2])
        return t + fy * (b - t)

    bx, by = mix(c[:, 0]), mix(c[:, 1])
    return Hxy * hdet * by - Hyy * hdet * bx, Hxy * hdet * bx - Hxx * hdet * by


def step32(hxx, hxy, hyy, c, fx, fy):
    Hxx = r32(r32(0.25 * r32(hxx)) + np.float32(EPS))
    Hxy = r32(0.25 * r32(hxy))
    Hyy = r32(r32(0.25 * r32(hyy)) + np.float32(EPS))
    w = r32(Hxy.astype(np.float64) * Hxy)
    det = r32(fma32(Hxx, Hyy, -w.astype(np.float64)).astype(np.float64) + fma32(-Hxy, Hxy, w))
    hd = r32(0.5 / det.astype(np.float64))
    ixx, ixy, iyy = (r32(v.astype(np.float64) * hd) for v in (Hyy, Hxy, Hxx))
    fx, fy = r32(fx), r32(fy)

    def mix(v):
        t = fma32(fx, r32(v[:, 1] - v[:, 0]), r32(v[:, 0]))
        b = fma32(fx, r32(v[:, 3] - v[:, 2]), r32(v[:, 2]))
        return fma32(fy, r32(b.astype(np.float64) - t), t)

    bx, by = mix(c[:, 0]), mix(c[:, 1])
    dx = fma32(ixy, by, -r32(ixx.astype(np.float64) * bx).astype(np.float64))
    dy = fma32(ixy, bx, -r32(iyy.astype(np.float64) * by).astype(np.float64))
    return dx, dy


@pytest.mark.parametrize("noise", [0.0, 0.5, 2.0, 5.0, 20.0])
def test_fp32_step_within_a_tenth_of_the_tolerance(noise):
    rng = np.random.default_rng(int(noise * 10) + 1)
    n = 200_000
    th = rng.uniform(0, 2 * np.pi, n)
    mag = rng.uniform(50, 255, (n, 25))
    gx = np.clip(np.rint(mag * np.cos(th)[:, None] + rng.uniform(0, noise, (n, 25)) if noise else
                         mag * np.cos(th)[:, None]), -255, 255)
    gy = np.clip(np.rint(mag * np.sin(th)[:, None] + rng.uniform(0, noise, (n, 25)) if noise else
                         mag * np.sin(th)[:, None]), -255, 255)
    r = np.rint(rng.uniform(-255, 255, (n, 25, 4)))
    c = np.stack([(gx[..., None] * r).sum(1), (gy[..., None] * r).sum(1)], 1)  # corner sums minus sum g A
    hxx, hxy, hyy = (gx * gx).sum(1), (gx * gy).sum(1), (gy * gy).sum(1)
    fx, fy = rng.uniform(0, 1, n), rng.uniform(0, 1, n)
    dx, dy = step64(hxx, hxy, hyy, c, fx, fy)
    ex, ey = step32(hxx, hxy, hyy, c, fx, fy)
    kept = (np.abs(dx) < 1) & (np.abs(dy) < 1)
    assert kept.sum() > 10_000
    err = np.maximum(np.abs(ex - dx), np.abs(ey - dy))[kept]
    assert err.max() <= 1e-3, err.max()
