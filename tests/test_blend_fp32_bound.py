"""Error bound of the blend kernel's short float paths (the oracle
evaluates Code 1 in FP64):
  - the flow magnitudes |f| = sqrt(f_x^2 + f_y^2): the square in double,
    a float square root, then one Newton step in double with a float
    reciprocal, s + (m2 - s^2) * (0.5 / s);
  - the softmax weight SoftmaxL = 1 / (1 + e^(zR - zL)): the exponent
    difference in double, rounded to float, then 2^(d log2 e) and a
    reciprocal in float (hardware exp2 and rcp, each within one ulp).
The displacements and their floor / fraction split stay in double. The
test re-evaluates both ways on adversarial inputs: flows up to 150 px,
strips as narrow as 32 px, sharp and flat softmax parameters (kS up to
60, kF up to 80), Blend across (0, 1), and colours 0 / 255 apart (the
largest |ColorL - ColorR| the 8-bit data allow, which multiplies every
weight error). Each float operation is rounded to float32 and then
perturbed by one ulp against the error (the worst case of the hardware's
one-ulp exp2 / rcp / sqrt); the composite must stay within a quarter of
the 0.5/255 bound."""
import numpy as np
import pytest

LOG2E = np.float32(1.4426950408889634)


def r32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def ulp_worse(x, sign):
    # x moved by one float32 ulp in the direction `sign` (a worst-case hardware rounding)
    x = r32(x)
    return np.nextafter(x, np.where(sign > 0, np.float32(np.inf), np.float32(-np.inf)))


def magnitude_model(fx, fy, sign):
    m2 = fx.astype(np.float64) ** 2 + fy.astype(np.float64) ** 2
    sf = ulp_worse(np.sqrt(r32(m2).astype(np.float64)), sign)  # float sqrt of the float-rounded square
    rc = ulp_worse(np.float32(0.5) / np.where(sf > 0, sf, np.float32(1)), sign)
    s = sf.astype(np.float64)
    out = s + (m2 - s * s) * rc.astype(np.float64)
    return np.where(sf > 0, out, 0.0)


def softmax_model(d, sign):
    # 2^x overflows to inf for large x, as on the device: the weight is then 0
    with np.errstate(over="ignore"):
        x = ulp_worse(r32(d) * LOG2E, sign)
        e = ulp_worse(np.exp2(x.astype(np.float64)), sign)
        one_e = r32(np.float32(1.0) + e)
    return ulp_worse(1.0 / one_e.astype(np.float64), -sign).astype(np.float64)


@pytest.mark.parametrize("kS,kF", [(10.0, 20.0), (60.0, 80.0), (0.5, 0.0), (30.0, 200.0)])
def test_blend_weight_error_bound(kS, kF):
    rng = np.random.default_rng(int(kS * 7 + kF))
    n = 2_000_000
    S = rng.choice([32.0, 64.0, 480.0, 960.0, 9000.0], n)
    t = rng.uniform(0.0, 1.0, n)
    f = [r32(rng.uniform(-150.0, 150.0, n)) for _ in range(4)]
    # many pixels near the softmax's switch, where its slope is largest
    mrl = np.hypot(f[0].astype(np.float64), f[1].astype(np.float64))
    mlr = np.hypot(f[2].astype(np.float64), f[3].astype(np.float64))
    zL = kS * (1.0 - t) * (1.0 + kF * mrl / S)
    zR = kS * t * (1.0 + kF * mlr / S)
    sL = 1.0 / (1.0 + np.exp(np.clip(zR - zL, -700, 700)))
    worst = 0.0
    for sign in (-1, 1):
        qrl = magnitude_model(f[0], f[1], sign)
        qlr = magnitude_model(f[2], f[3], sign)
        assert np.abs(qrl - mrl).max() <= 1e-12 * np.maximum(mrl, 1.0).max()
        zl = kS * (1.0 - t) * (1.0 + kF * qrl / S)
        zr = kS * t * (1.0 + kF * qlr / S)
        q = softmax_model(np.clip(zr - zl, -3e38, 3e38), sign)
        worst = max(worst, float(np.abs(q - sL).max()) * 255.0)
    assert worst <= 0.25 * 0.5 / 255.0, worst
