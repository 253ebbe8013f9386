"""Host-only checks of the C ABI: the library loads, exports every function
include/abf.h declares, and rejects bad arguments without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2006_01201_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "abf.h")).read()
    return sorted(set(re.findall(r"\b(abf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libabf.so not built")
    return _abi.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.EXPORTS)


def test_status_strings(lib):
    for s in range(7):
        assert _abi.status_string(s).startswith("ABF_")
    assert "unknown" in _abi.status_string(99)


def test_default_params(lib):
    p = _abi.default_params()
    assert (p.levels, p.patch, p.radius, p.radius_coarse, p.prop_steps, p.median) == (6, 2, 2, 4, 2, 1)
    assert (p.lk_patch, p.lk_iters, p.lk_eps, p.k_sharp, p.k_flowmag, p.blend_mode) == (2, 2, 25.0, 10.0, 20.0, 0)
    assert p.gain_comp == 0 and p.flow_method == 0


def test_defaults_match_oracle_and_api():
    import oracle
    from paper_2006_01201_amd import api

    o, a = oracle.Params(), api.Params()
    for f in ("levels", "patch", "radius", "radius_coarse", "prop_steps", "median", "lk_patch", "lk_iters",
              "lk_eps", "k_sharp", "k_flowmag", "blend_mode", "gain_comp"):
        assert getattr(o, f) == getattr(a, f), f


@pytest.mark.parametrize("field,value,status", [
    ("levels", 0, _abi.E_INVALID), ("levels", 13, _abi.E_INVALID), ("patch", 0, _abi.E_INVALID),
    ("lk_eps", 0.0, _abi.E_INVALID), ("lk_eps", float("nan"), _abi.E_INVALID), ("blend_mode", 2, _abi.E_INVALID),
    ("gain_comp", 2, _abi.E_INVALID), ("flow_method", 2, _abi.E_INVALID), ("flow_method", -1, _abi.E_INVALID),
    ("patch", 3, _abi.E_UNSUPPORTED), ("radius", 5, _abi.E_UNSUPPORTED), ("median", 2, _abi.E_UNSUPPORTED),
])
def test_create_plan_rejects_parameters(lib, field, value, status):
    p = _abi.default_params()
    setattr(p, field, value)
    st, h = _abi.create_plan(p, 1, 100, 10, 10)
    assert st == status and h is None


def test_create_plan_rejects_limits(lib):
    p = _abi.default_params()
    for args in [(0, 100, 10, 10), (1, 0, 10, 10), (1, 100, 0, 10), (1, 100, 10, -1)]:
        st, h = _abi.create_plan(p, *args)
        assert st == _abi.E_INVALID and h is None


def test_null_arguments(lib):
    assert lib.abf_create_plan(None, 1, 1, 1, 1, None) == _abi.E_INVALID
    assert lib.abf_destroy(None) == _abi.E_INVALID
    assert lib.abf_workspace_bytes(None) == 0
    assert lib.abf_bind_workspace(None, None, 0) == _abi.E_INVALID
    assert lib.abf_flow_bidirectional(None, None, None, 1, 1, 3, 3, None, None, None) == _abi.E_INVALID
    assert lib.abf_stitch_strips(None, None, 0, 0, None) == _abi.E_INVALID
    assert lib.abf_last_error(None) == b"null plan"


def test_no_device_is_unsupported(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _abi.create_plan(_abi.default_params(), 1, 100, 10, 10)
    assert st == _abi.E_UNSUPPORTED and h is None


def test_strip_struct_layout():
    # field offsets must follow the C declaration order with natural alignment
    S = _abi.AbfStrip
    assert S.H.offset == 16 and S.pitch_L.offset == 24 and S.blend.offset == 40
    assert S.F_f32.offset == 80 and ctypes.sizeof(S) == 88
    assert ctypes.sizeof(_abi.AbfParams) == 56 and _abi.AbfParams.flow_method.offset == 52
    P = _abi.AbfPhoto
    assert P.mask.offset == 8 and P.pitch.offset == 16 and P.side.offset == 24 and ctypes.sizeof(P) == 32


def test_canvas_and_merge_reject_null_plans(lib):
    assert lib.abf_canvas_workspace_bytes(None, 10, 10) == 0
    assert lib.abf_merge_workspace_bytes(None, 10, 10) == 0
    for per in (0, 1):
        assert lib.abf_overlap_box(None, None, None, 4, 4, 4, per, None, None) == _abi.E_INVALID
        assert lib.abf_canvas_blend(None, None, None, 4, 4, 4, per, None, 4, None, None, 4, None) == _abi.E_INVALID
        box = (ctypes.c_int32 * 4)(0, 0, 0, 0)
        assert lib.abf_composite_canvas(None, None, None, None, None, 4, 4, 12, 12, 4, per, None, None, box, 0, None,
                                        4, None, 12, None, None) == _abi.E_INVALID
        assert lib.abf_merge_photos(None, None, 0, 4, 4, 4, per, None, 12, None, 12, None, None,
                                    None) == _abi.E_INVALID


def test_log_to_stderr_by_environment(lib):
    import subprocess
    import sys

    code = ("from paper_2006_01201_amd import _abi; "
            "print(_abi.create_plan(_abi.default_params(), 1, 100, 10, 10)[0])")
    env = dict(os.environ, ABF_LOG="1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    quiet = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           env={k: v for k, v in env.items() if k != "ABF_LOG"}, cwd=ROOT)
    import torch

    if torch.cuda.is_available():
        assert "[abf] plan on device" in r.stderr
    else:
        assert "[abf] error 5: no device" in r.stderr and r.stdout.strip() == "5"
    assert "[abf]" not in quiet.stderr
