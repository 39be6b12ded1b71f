"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects bad arguments with the documented
codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fewbody.h")


@pytest.fixture(scope="module")
def fbmod():
    from paper_1208_1157_amd import fewbody
    return fewbody


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(fbmod):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(fbmod.lib(), n), f"{n} declared in fewbody.h but not exported"


def test_opts_layout_and_defaults(fbmod):
    o = fbmod.FbOpts()
    fbmod.lib().fb_opts_default(ctypes.byref(o))
    assert (o.adaptive, o.eta, o.stop_rules, o.r_eject, o.max_steps) == (0, 0.01, 0, 100.0, 0)
    assert (o.schedule, o.steps_per_quantum, o.compact) == (0, 0, 0)
    assert ctypes.sizeof(fbmod.FbOpts) == 56


def test_version(fbmod):
    assert "gfx950" in fbmod.version()


def test_workspace_bytes(fbmod):
    assert fbmod.workspace_bytes([3, 3, 5]) > 0
    assert fbmod.workspace_bytes([]) > 0
    assert fbmod.workspace_bytes([1]) == 0          # n_body below 2
    assert fbmod.workspace_bytes([513]) == 0        # n_body above 512
    assert fbmod.workspace_bytes([17, 300]) > 0     # large-n systems
    a = fbmod.workspace_bytes([3] * 1000)
    b = fbmod.workspace_bytes([3] * 2000)
    assert b > a


def _create(fbmod, n_body, mass, pos, vel):
    h = ctypes.c_void_p()
    nb = np.ascontiguousarray(n_body, dtype=np.int32)
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in (mass, pos, vel)]
    rc = fbmod.lib().fb_ensemble_create(len(nb), nb.ctypes.data_as(ctypes.c_void_p),
                                        *[a.ctypes.data_as(ctypes.c_void_p) for a in args],
                                        None, None, ctypes.byref(h))
    return rc, h


def test_create_rejects_bad_input_before_device_work(fbmod):
    m = np.array([1.0, 1e-3, 1e-3])
    x = np.array([[0, 0, 0], [1.0, 0, 0], [2.0, 0, 0]])
    v = np.zeros((3, 3))
    rc, h = _create(fbmod, [3], -m, x, v)
    assert rc == fbmod.E_INVAL and not h.value
    assert b"mass" in fbmod.lib().fb_last_error()
    x2 = x.copy(); x2[1, 1] = np.nan
    rc, _ = _create(fbmod, [3], m, x2, v)
    assert rc == fbmod.E_INVAL and b"finite" in fbmod.lib().fb_last_error()
    rc, _ = _create(fbmod, [1, 2], m, x, v)
    assert rc == fbmod.E_INVAL
    rc, _ = _create(fbmod, [513], np.ones(513), np.zeros((513, 3)), np.zeros((513, 3)))
    assert rc == fbmod.E_INVAL


def test_null_handles(fbmod):
    L = fbmod.lib()
    assert L.fb_integrate_steps(None, 10, 0.1, None) == fbmod.E_INVAL
    assert L.fb_integrate(None, 1.0, 0.1, None) == fbmod.E_INVAL
    assert L.fb_get_state(None, None, None, None, None, None) == fbmod.E_INVAL
    assert L.fb_diagnostics(None, None, None) == fbmod.E_INVAL
    assert L.fb_ensemble_destroy(None) == fbmod.OK


def test_plan_table(fbmod):
    m0 = fbmod.get_plan(5)
    fbmod.set_plan(5, fbmod.MAP_SPL, 2, 0)
    assert fbmod.get_plan(5) == (fbmod.MAP_SPL, 2, 0)
    fbmod.set_plan(5, fbmod.MAP_AUTO, 2, 0)
    assert fbmod.get_plan(5) == (fbmod.MAP_AUTO, 2, 0)     # auto is a setting, not "keep"
    fbmod.set_plan(5, m0[0], m0[1], m0[2])
    with pytest.raises(fbmod.FewbodyError):
        fbmod.set_plan(12, fbmod.MAP_SPL, 1, 0)     # SPL built for n <= 10 only
    with pytest.raises(fbmod.FewbodyError):
        fbmod.set_plan(1, fbmod.MAP_BPL, 1, 0)
    with pytest.raises(fbmod.FewbodyError):
        fbmod.set_plan(4, fbmod.MAP_BPL, 0, 0)


def test_product_path_does_not_touch_the_oracle():
    """The HIP binding, runtime and kernels never import or link the oracle."""
    pkg = os.path.join(ROOT, "paper_1208_1157_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt and "hermite_oracle" not in txt, f


def test_server_request_bytes(fbmod):
    """Host-only accounting: a staging block plus whole pool chunks per body
    count; invalid counts or options give 0."""
    assert ctypes.sizeof(fbmod.FbServerOpts) == 40
    one = fbmod.server_request_bytes([5], chunk_slots=64)
    full = fbmod.server_request_bytes([5] * 64, chunk_slots=64)
    two_chunks = fbmod.server_request_bytes([5] * 65, chunk_slots=64)
    two_counts = fbmod.server_request_bytes([5, 6], chunk_slots=64)
    assert 0 < one < full < two_chunks
    assert two_counts > one
    assert fbmod.server_request_bytes([5] * 64) > full          # default chunks hold 512
    assert fbmod.server_request_bytes([1], chunk_slots=64) == 0
    assert fbmod.server_request_bytes([17]) == 0
    assert fbmod.server_request_bytes([5], chunk_slots=100) == 0  # not a multiple of 64
    assert fbmod.server_request_bytes([5], policy=7) == 0
    assert fbmod.server_request_bytes([5], long_steps=-1) == 0
    assert fbmod.server_request_bytes([5], idle_spread=2) == 0
    assert fbmod.server_request_bytes([5], chunk_slots=64, idle_spread=-1) == one
    assert fbmod.server_request_bytes([]) > 0


def test_fma_ceiling_rejects_null(fbmod):
    assert fbmod.lib().fb_fp64_fma_ceiling(None) == fbmod.E_INVAL


def test_lds_rates_rejects_null(fbmod):
    x = ctypes.c_double()
    assert fbmod.lib().fb_lds_rates(None, ctypes.byref(x)) == fbmod.E_INVAL
    assert fbmod.lib().fb_lds_rates(ctypes.byref(x), None) == fbmod.E_INVAL


def test_log_bytes(fbmod):
    """Log buffer sizes follow the documented layouts; invalid kinds, record
    counts and body counts give 0."""
    nb = [3, 5, 2]
    R = 7
    assert fbmod.log_bytes(nb, fbmod.LOG_RV, R) == 8 * R * 2 * 3
    assert fbmod.log_bytes(nb, fbmod.LOG_ENERGY, R) == 8 * R * 5 * 3
    assert fbmod.log_bytes(nb, fbmod.LOG_STATE, R) == 8 * R * sum(1 + 6 * n for n in nb)
    assert fbmod.log_bytes(nb, 3, R) == 0
    assert fbmod.log_bytes(nb, fbmod.LOG_RV, 0) == 0
    assert fbmod.log_bytes([3, 513], fbmod.LOG_RV, R) == 0
    assert fbmod.log_bytes([], fbmod.LOG_STATE, R) == 0


def test_logged_integration_rejects_null(fbmod):
    L = fbmod.lib()
    spec = fbmod.FbLogSpec()
    assert L.fb_integrate_steps_logged(None, 10, 0.01, None, ctypes.byref(spec), None) == fbmod.E_INVAL
    assert ctypes.sizeof(fbmod.FbLogSpec) == 56
