"""Pins of the oracle's multi-level energy (the energy summed over a float
pyramid of the images and the flow): the pyramid filter against scipy's
convolution, its adjoint by the dot-product identity, one level against
the single-level energy, and the gradients against FP64 central
differences along random directions (the energy is smooth in Ref and Tgt;
along a random flow direction no bilinear kink lies within the step)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2006_01201_amd import synth


@pytest.mark.parametrize("H,W,C", [(16, 12, 3), (17, 9, 2), (1, 7, 3), (5, 1, 2), (2, 2, 3)])
def test_pyr_down_float_equals_convolution_and_decimation(H, W, C):
    x = np.random.default_rng(H * W).normal(size=(H, W, C))
    k = np.outer([1, 4, 6, 4, 1], [1, 4, 6, 4, 1]) / 256.0
    want = np.stack([ndimage.convolve(x[..., c], k, mode="nearest")[::2, ::2] for c in range(C)], -1)
    assert np.allclose(oracle.pyr_down_float(x), want, rtol=0, atol=1e-12)
    assert oracle.pyr_down_float(x).shape == ((H + 1) // 2, (W + 1) // 2, C)


@pytest.mark.parametrize("H,W", [(16, 12), (17, 9), (1, 7), (5, 1), (3, 3), (33, 64)])
def test_pyr_adjoint_dot_product_identity(H, W):
    rng = np.random.default_rng(H + 100 * W)
    x = rng.normal(size=(H, W, 2))
    y = rng.normal(size=((H + 1) // 2, (W + 1) // 2, 2))
    lhs = np.sum(oracle.pyr_down_float(x) * y)
    rhs = np.sum(x * oracle.pyr_down_float_adjoint(y, x.shape))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # constant in, constant out: the weights sum to one
    assert np.allclose(oracle.pyr_down_float(np.ones((H, W))), 1.0, rtol=0, atol=1e-15)


def _crop():
    st = synth.make_config_strip(3, 0, 0)
    r0, c0 = 992, 240
    Ref, Tgt = st.R[r0:r0 + 48, c0:c0 + 40], st.L[r0:r0 + 48, c0:c0 + 40]
    u = np.random.default_rng(5).uniform(-1.5, 1.5, (48, 40, 2)) + st.flow_rl_gt[r0:r0 + 48, c0:c0 + 40]
    return Ref, Tgt, u


def test_one_level_is_the_energy():
    Ref, Tgt, u = _crop()
    E1, gu1, gr1, gt1 = oracle.energy_ms(Ref, Tgt, u, 1)
    E, gu, gr, gt = oracle.energy(Ref, Tgt, u)
    assert E1 == E and np.array_equal(gu1, gu) and np.array_equal(gr1, gr) and np.array_equal(gt1, gt)


@pytest.mark.parametrize("levels", [2, 4])
def test_multilevel_gradients_against_central_differences(levels):
    Ref, Tgt, u = _crop()
    E, gu, gr, gt = oracle.energy_ms(Ref, Tgt, u, levels)
    # the sum of the levels' energies
    R, T, U = Ref, Tgt, u
    parts = 0.0
    for _ in range(levels):
        parts += oracle.energy(R, T, U, grads=False)
        R, T, U = oracle.pyr_down_float(R), oracle.pyr_down_float(T), oracle.pyr_down_float(U) / 2
    assert abs(E - parts) <= 1e-12 * E
    rng = np.random.default_rng(levels)
    for name, x, g, h in (("u", u, gu, 1e-7), ("Ref", Ref, gr, 1e-6), ("Tgt", Tgt, gt, 1e-6)):
        for _ in range(3):
            v = rng.normal(size=x.shape)
            args = {"u": (Ref, Tgt, None), "Ref": (None, Tgt, u), "Tgt": (Ref, None, u)}[name]

            def f(t):
                xs = x + t * v
                a = [xs if a is None else a for a in args]
                return oracle.energy_ms(a[0], a[1], a[2], levels, grads=False)

            fd = (f(h) - f(-h)) / (2 * h)
            an = float(np.sum(g * v))
            assert abs(fd - an) <= 2e-5 * max(abs(an), 1.0), (name, fd, an)
