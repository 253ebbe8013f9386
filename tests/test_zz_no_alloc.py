"""Allocation-free flow entry point (abf_flow_bidirectional_noalloc): on a
plan with no workspace bound it gives the results of abf_flow_bidirectional
(the same kernels, with the library's static scratch in place of the
workspace), on two calls in a row, the second with a smaller strip; a strip
whose layout exceeds the static array is rejected before any launch."""
import numpy as np
import pytest
import torch

from paper_2006_01201_amd import _abi, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_01201_amd import api as _api

    return _api


def test_noalloc_equals_flow_bidirectional(api):
    st = synth.make_config_strip(1, 0, 0)  # 4000 x 768, 6 levels
    L = torch.from_numpy(st.L).cuda()
    R = torch.from_numpy(st.R).cuda()
    p = api.Params()
    ref_plan = api.Plan(p, max_strips=1, max_H=st.H, max_W=st.W)
    # crops: 1500 x 768 (several tiles, ragged tails at every level), then 256 x 200 at an offset
    crops = [(slice(0, 1500), slice(0, 768)), (slice(1000, 1256), slice(100, 300))]
    refs, outs = [], []
    for rs, cs in crops:
        refs.append(ref_plan.flow_bidirectional(L[rs, cs], R[rs, cs]))
    torch.cuda.synchronize()
    # a plan with no workspace bound: the entry point needs none
    status, h = _abi.create_plan(p.to_c(), 1, st.H * st.W, st.H, st.W)
    _abi.check(status, None, "abf_create_plan")
    try:
        stream = torch.cuda.current_stream().cuda_stream
        for k, (rs, cs) in enumerate(crops):
            l, r = L[rs, cs], R[rs, cs]
            H, W = l.shape[:2]
            print(f"[gpu] noalloc call {k}: {H} x {W}", flush=True)
            flr = torch.full((H, W, 2), float("nan"), device="cuda")
            frl = torch.full((H, W, 2), float("nan"), device="cuda")
            rc = _abi.flow_bidirectional_noalloc(h, l.data_ptr(), r.data_ptr(), H, W, l.stride(0), r.stride(0),
                                                 flr.data_ptr(), frl.data_ptr(), stream)
            _abi.check(rc, h, "abf_flow_bidirectional_noalloc")
            outs.append((flr, frl))
        torch.cuda.synchronize()
    finally:
        _abi.destroy(h)
    for (rs, cs), ref, out in zip(crops, refs, outs):
        for a, b in zip(ref, out):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.isfinite(b).all()
            # same kernels and launch shapes: identical bits (far inside the 1e-2 px bound)
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), np.abs(a - b).max()


def test_noalloc_rejects_strips_beyond_the_static_scratch(api):
    # 4000 x 768 at 6 levels needs about 85 MB of scratch, more than the 64 MiB array
    H, W = 4000, 768
    plan = api.Plan(api.Params(), max_strips=1, max_H=H, max_W=W)
    L = torch.zeros((H, W, 3), dtype=torch.uint8, device="cuda")
    R = torch.zeros((H, W, 3), dtype=torch.uint8, device="cuda")
    out = (torch.zeros((H, W, 2), device="cuda"), torch.zeros((H, W, 2), device="cuda"))
    print("[gpu] noalloc oversize strip", flush=True)
    with pytest.raises(_abi.AbfError) as e:
        plan.flow_bidirectional_noalloc(L, R, out)
    assert e.value.status == _abi.E_WORKSPACE
    assert "static scratch" in str(e.value)
    # nothing was launched: the outputs are untouched, and the plan still works
    torch.cuda.synchronize()
    assert not out[0].any() and not out[1].any()
    small = (torch.zeros((64, 64, 2), device="cuda"), torch.zeros((64, 64, 2), device="cuda"))
    plan.flow_bidirectional_noalloc(L[:64, :64], R[:64, :64], small)
    torch.cuda.synchronize()
    assert not small[0].any() and not small[1].any()  # zero images: zero flow
