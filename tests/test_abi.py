"""Host-side checks of the C ABI: every function declared in include/msk.h is
exported by libmsk.so and bound by the Python module (no GPU compute)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "msk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(msk_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["msk_build_bvh", "msk_estimate_dtn", "msk_estimate_dtn_batched", "msk_steklov_modes",
              "msk_closest_points"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2606_05581_amd import msk

    assert os.path.exists(msk.LIB_PATH), "libmsk.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", msk.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(msk.LIB_PATH)
    for n in _declared():
        assert hasattr(L, n)
    assert set(_declared()) == set(msk.SIGNATURES), "binding and header disagree"


def test_library_is_built_for_gfx950():
    """The embedded device code object targets gfx950 (target id in the bundle)."""
    from paper_2606_05581_amd import msk

    blob = open(msk.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_opts_defaults_and_errors_without_device():
    """Option defaults come from the library; calls with bad arguments fail
    cleanly before touching a device."""
    from paper_2606_05581_amd import msk

    o = msk.DtnOpts()
    msk.lib().msk_dtn_opts_default(ctypes.byref(o))
    assert o.kappa == 2.0 ** -20 and o.delta_rel == 2.0 ** -21 and o.chunk == 64 and o.form == msk.FORM_PERSISTENT
    h = ctypes.c_void_p()
    assert msk.lib().msk_create(0, None, None) == msk.ERR_INVALID_ARG
    assert msk.lib().msk_estimate_dtn(None, None, None, None, 16, 1e-3, 0.05, 0, None, ctypes.byref(h)) != msk.OK


def test_eps_floor_covers_the_step_guard_and_fp32_resolution():
    """The shell must be wider than the step guard delta_rel R / (1 - kappa)
    (else a walk inside the shell could take a step of negative length and
    cross the surface) and than the FP32 resolution 2^-18 R of the scene
    frame; the floor scales with the mesh radius."""
    from paper_2606_05581_amd import msk

    L = msk.lib()
    o = msk.DtnOpts()
    L.msk_dtn_opts_default(ctypes.byref(o))
    for R in [1.0, 2.5, 1e3]:
        f = L.msk_eps_floor(R, ctypes.byref(o))
        assert f == max(o.delta_rel * R / (1 - o.kappa), R * 2.0 ** -18)
        assert f == L.msk_eps_floor(R, None)
        # a walk just outside the floor takes a positive step
        d = f * (1 + 1e-9)
        assert d * (1 - o.kappa) - o.delta_rel * R > 0
    # the header's example: eps = 1e-6 is refused on a mesh of radius > 0.262
    assert L.msk_eps_floor(0.25, None) < 1e-6 < L.msk_eps_floor(0.3, None)
    o.delta_rel = 2.0 ** -12  # a larger guard dominates
    assert L.msk_eps_floor(1.0, ctypes.byref(o)) == pytest.approx(2.0 ** -12 / (1 - o.kappa), rel=1e-15)
    assert L.msk_eps_floor(0.0, None) != L.msk_eps_floor(0.0, None)  # NaN
    assert L.msk_eps_floor(float("inf"), None) != L.msk_eps_floor(float("inf"), None)
