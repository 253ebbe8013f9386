"""Pins of the oracle's classic coarse-to-fine Lucas-Kanade (float flows
at every level): the closed-form contraction on an intensity ramp, the
special case that reduces to the (pinned) level-0 refinement, a large
shift recovered through the pyramid, the seed taken from the coarser
level, and the two directions of a pure shift."""
import numpy as np
import pytest

import oracle
from paper_2006_01201_amd import synth


def test_ramp_contracts_by_the_closed_form():
    # A = 2x (Ref), B(x) = A(x + 2.5) = 2x + 5 (Tgt): A(p) = B(p + u) at
    # u = -2.5, and bilinear samples of a ramp are exact, so from u = 0
    # every step multiplies u + 2.5 by eps / (25 a^2 + eps) = 1 / (a^2 + 1)
    # with a window of 25 and eps = 25
    H, W = 30, 110
    x = np.arange(W)
    A = np.tile(2 * x, (H, 1)).astype(np.uint8)
    B = np.tile(np.minimum(2 * x + 5, 255), (H, 1)).astype(np.uint8)
    for K in (1, 2, 3):
        u = oracle.lk_level(A, B, None, P=2, K=K, eps=25.0)
        inner = u[3:-3, 6:W - 8]  # every window sample stays inside the ramp
        want = -2.5 + 2.5 / 5.0 ** K
        assert np.allclose(inner[..., 0], want, rtol=0, atol=1e-9)
        assert np.allclose(inner[..., 1], 0.0, rtol=0, atol=1e-12)


def test_small_shift_from_zero_equals_the_refinement():
    # with seed 0 and steps that never reach the refinement's 1 px clamp,
    # one level of the classic method is the level-0 refinement from D0 = 0
    s = synth.make_random(21, 40, 60, max_ux=0.4, max_uy=0.3, noise=0.0)
    A = (s.R[..., 0] // 2 + s.R[..., 1] // 2).astype(np.uint8)
    B = (s.L[..., 0] // 2 + s.L[..., 1] // 2).astype(np.uint8)
    traj = [oracle.lk_level(A, B, None, P=2, K=k, eps=25.0) for k in (1, 2, 3)]
    r = oracle.refine(A, B, np.zeros((40, 60, 2), np.int32), oracle.Params(lk_patch=2, lk_iters=3, lk_eps=25.0))
    # pixels whose every iterate stays strictly inside the clamp
    ok = np.all([np.abs(t).max(axis=2) < 1.0 for t in traj], axis=0)
    assert ok.mean() > 0.9
    assert np.array_equal(traj[-1][ok], r[ok])


def _shift_pair(H, W, sx, sy, seed=11):
    big = synth.make_random(seed, H + 80, W + 80, max_ux=0.0, max_uy=0.0, noise=0.0).L
    L = big[40:40 + H, 40:40 + W]
    R = big[40 + sy:40 + sy + H, 40 + sx:40 + sx + W]  # R(p) = L(p + s)
    return np.ascontiguousarray(L), np.ascontiguousarray(R)


def test_large_shift_through_the_pyramid():
    L, R = _shift_pair(96, 128, 13, -6)
    p = oracle.Params(levels=4, lk_iters=6, gain_comp=0)
    lr, rl = oracle.flow_lk_bidirectional(L, R, p)
    m = 24
    inner_rl = rl[0][m:-m, m:-m]
    inner_lr = lr[0][m:-m, m:-m]
    # R(p) = L(p + s): FlowRtoL = s, FlowLtoR = -s
    assert np.median(np.abs(inner_rl - [13, -6])) < 0.02
    assert np.median(np.abs(inner_lr - [-13, 6])) < 0.02
    assert (np.hypot(*(inner_rl - [13, -6]).transpose(2, 0, 1)) < 0.1).mean() > 0.95


def test_each_level_starts_from_the_doubled_coarser_flow():
    L, R = _shift_pair(40, 52, 5, 3)
    yl, yr = (oracle.luma(x) for x in (L, R))
    lv = oracle.flow_lk(yr, yl, 3, P=2, K=2, eps=25.0)
    A1, B1 = oracle.pyramid(yr, 3)[1], oracle.pyramid(yl, 3)[1]
    h, w = A1.shape
    ys, xs = np.mgrid[0:h, 0:w]
    seed = 2.0 * lv[2][np.minimum(ys // 2, lv[2].shape[0] - 1), np.minimum(xs // 2, lv[2].shape[1] - 1)]
    assert np.array_equal(oracle.lk_level(A1, B1, seed, P=2, K=2, eps=25.0), lv[1])


@pytest.mark.parametrize("K", [0])
def test_no_iterations_keeps_zero(K):
    L, R = _shift_pair(24, 30, 2, 1)
    lr, rl = oracle.flow_lk_bidirectional(L, R, oracle.Params(levels=3), K=K)
    assert all((f == 0).all() for f in lr + rl)
