"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, its structs match the header, and arguments are validated before any
device call (with no device present, a valid create fails with BM_ERR_DEVICE)."""
from __future__ import annotations

import ctypes
import glob
import os
import re
import subprocess
import tempfile

import pytest

from paper_1409_4923_amd import bmotor as B
from paper_1409_4923_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w\s\*]*?\b(bm_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_headers_exist_and_declare_entry_points():
    names = declared_functions()
    for must in ("bm_ensemble_create", "bm_integrate", "bm_reduce", "bm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = B.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (bm_\w+)", out))
    assert set(declared_functions()) <= exported


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) == {s[0] for s in B.SIGNATURES}


def test_abi_version():
    assert B.bm_abi_version() == 2


_LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "bmotor.h"
#define F(T, m) printf(#T " " #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("bm_model size %zu\n", sizeof(bm_model));
  printf("bm_run size %zu\n", sizeof(bm_run));
  printf("bm_stats size %zu\n", sizeof(bm_stats));
  printf("bm_tune size %zu\n", sizeof(bm_tune));
  printf("bm_path size %zu\n", sizeof(bm_path));
  F(bm_path, x) F(bm_path, periods_window) F(bm_path, kick_frac) F(bm_path, noise) F(bm_path, steps_taken)
  F(bm_run, step_tol) F(bm_run, max_halvings)
  F(bm_model, gamma) F(bm_model, D) F(bm_model, dich_mub)
  F(bm_run, dt) F(bm_run, n_steps) F(bm_run, seed) F(bm_run, v0_hi)
  F(bm_stats, mean) F(bm_stats, t_window)
  F(bm_tune, block)
  return 0;
}
"""


def test_struct_layout_matches_header():
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "l.c")
        exe = os.path.join(td, "l")
        open(src, "w").write(_LAYOUT_C)
        subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    for line in out.strip().splitlines():
        struct, field, val = line.split()
        cls = getattr(B, struct)
        if field == "size":
            assert ctypes.sizeof(cls) == int(val), line
        else:
            assert getattr(cls, field).offset == int(val), line


def _ok_model_run(**kw):
    m, r = W.to_c(W.C1)
    for k, v in kw.items():
        setattr(m if hasattr(m, k) else r, k, v)
    return m, r


def _ws_rc(m, r):
    n = ctypes.c_size_t()
    return B.lib().bm_ensemble_workspace_size(ctypes.byref(m), ctypes.byref(r), ctypes.byref(n)), n.value


def test_workspace_size_valid_configs():
    for w in (W.C1, W.C2, W.C3):
        m, r = W.to_c(w)
        rc, n = _ws_rc(m, r)
        assert rc == B.BM_OK, B.last_error()
        assert n % 256 == 0
        assert n >= w.n_paths * (4 * 8 + 8)          # the SoA state of every path
    m, r = W.to_c(W.C2)
    small = _ws_rc(m, r)[1]
    r.n_paths *= 2
    assert _ws_rc(m, r)[1] > small


@pytest.mark.parametrize("field,value,code", [
    ("size", 0, B.BM_ERR_INVALID_ARG),
    ("dyn", 7, B.BM_ERR_INVALID_ARG),
    ("pot", 9, B.BM_ERR_INVALID_ARG),
    ("noise", 32, B.BM_ERR_INVALID_ARG),
    ("noise", 16, B.BM_ERR_INVALID_ARG),           # jump-adapted grid without Poisson noise
    ("noise", 9, B.BM_ERR_INVALID_ARG),            # three-point and normal increments together
    ("prec", 3, B.BM_ERR_INVALID_ARG),
    ("gamma", 0.0, B.BM_ERR_INVALID_ARG),
    ("gamma", float("nan"), B.BM_ERR_INVALID_ARG),
    ("drive_omega", 0.0, B.BM_ERR_INVALID_ARG),
    ("dt", 0.1, B.BM_ERR_INVALID_ARG),             # dt must be 0 when spp > 0
    ("D", -1.0, B.BM_ERR_INVALID_ARG),
    ("n_paths", 0, B.BM_ERR_INVALID_ARG),
    ("n_paths", 1 << 32, B.BM_ERR_INVALID_ARG),
    ("x0_lo", 2.0, B.BM_ERR_INVALID_ARG),
    ("force", float("inf"), B.BM_ERR_INVALID_ARG),
])
def test_invalid_arguments_rejected(field, value, code):
    m, r = _ok_model_run()
    setattr(m if field in dict(B.bm_model._fields_) and field != "size" else r, field, value)
    rc, _ = _ws_rc(m, r)
    assert rc == code, (field, value, rc, B.last_error())
    assert B.last_error() != ""


def test_normal_increments_accepted():
    for noise in (W.NORMAL, W.NORMAL | W.POISSON, W.NORMAL | W.DICH, W.NORMAL | W.POISSON | W.DICH):
        m, r = W.to_c(W.C3.with_(noise=noise, dyn=W.INERTIAL, gamma=0.9))
        rc, _ = _ws_rc(m, r)
        assert rc == B.BM_OK, (noise, B.last_error())


def test_jump_grid_accepted_and_limited():
    for noise in (W.POISSON | W.JUMP_GRID, W.GAUSS | W.POISSON | W.JUMP_GRID,
                  W.NORMAL | W.POISSON | W.DICH | W.JUMP_GRID):
        m, r = W.to_c(W.C2.with_(noise=noise))
        rc, n = _ws_rc(m, r)
        assert rc == B.BM_OK, (noise, B.last_error())
        m0, r0 = W.to_c(W.C2)
        assert n >= _ws_rc(m0, r0)[1] + 8 * W.C2.n_paths    # the FP64 kick phase per path
    m, r = W.to_c(W.C2.with_(noise=W.POISSON | W.JUMP_GRID, lam=1e4))
    assert _ws_rc(m, r)[0] == B.BM_ERR_UNSUPPORTED          # more than 16 kicks per step expected
    pts = W.c4_points(8)
    M, R = _scan_arrays([pts[0].with_(noise=W.GAUSS | W.POISSON | W.JUMP_GRID, lam=1.0, zeta=0.1)])
    n = ctypes.c_size_t()
    assert B.lib().bm_scan_workspace_size(M, R, 1, ctypes.byref(n)) == B.BM_ERR_UNSUPPORTED


def test_drive_needs_steps_per_period():
    m, r = _ok_model_run(steps_per_period=0, dt=0.01)
    assert _ws_rc(m, r)[0] == B.BM_ERR_INVALID_ARG       # a = 4.2 without a phase grid
    m.drive_amp = 0.0
    assert _ws_rc(m, r)[0] == B.BM_OK


def test_jump_rate_limits():
    m, r = W.to_c(W.C2)
    m.shot_rate = 0.0
    assert _ws_rc(m, r)[0] == B.BM_ERR_INVALID_ARG
    m.shot_rate = 1e-12                                   # waiting times overflow int32
    assert _ws_rc(m, r)[0] == B.BM_ERR_UNSUPPORTED
    m, r = W.to_c(W.C3)
    m.dich_mua = -1.0
    assert _ws_rc(m, r)[0] == B.BM_ERR_INVALID_ARG


def test_null_arguments():
    L = B.lib()
    assert L.bm_ensemble_workspace_size(None, None, None) == B.BM_ERR_INVALID_ARG
    assert L.bm_integrate(None, 10) == B.BM_ERR_INVALID_ARG
    assert L.bm_reduce(None, None) == B.BM_ERR_INVALID_ARG
    assert L.bm_ensemble_destroy(None) == B.BM_ERR_INVALID_ARG
    assert L.bm_read_paths(None, 0, 1, None, None, None, None, None) == B.BM_ERR_INVALID_ARG
    assert L.bm_write_paths(None, 0, 1, None) == B.BM_ERR_INVALID_ARG
    assert L.bm_ensemble_set_tune(None, None) == B.BM_ERR_INVALID_ARG


def test_create_checks_workspace_then_device():
    m, r = W.to_c(W.C1)
    L = B.lib()
    h = ctypes.c_void_p()
    need = B.bm_ensemble_workspace_size(m, r)
    # misaligned / too small workspace: rejected before touching the device
    assert L.bm_ensemble_create(ctypes.byref(m), ctypes.byref(r), 0x1001, need, None,
                                ctypes.byref(h)) == B.BM_ERR_WORKSPACE
    assert L.bm_ensemble_create(ctypes.byref(m), ctypes.byref(r), 0x10000, need - 256, None,
                                ctypes.byref(h)) == B.BM_ERR_WORKSPACE
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if not has_gpu:
        rc = L.bm_ensemble_create(ctypes.byref(m), ctypes.byref(r), 0x10000, need, None, ctypes.byref(h))
        assert rc == B.BM_ERR_DEVICE, B.last_error()
        assert h.value is None


def test_attach_checks_arguments_before_device():
    m, r = W.to_c(W.C2)
    L = B.lib()
    h = ctypes.c_void_p()
    need = B.bm_ensemble_workspace_size(m, r)
    assert L.bm_ensemble_attach(ctypes.byref(m), ctypes.byref(r), 0x10000, need, 1 << 32, None,
                                ctypes.byref(h)) == B.BM_ERR_UNSUPPORTED
    assert L.bm_ensemble_attach(ctypes.byref(m), ctypes.byref(r), 0x1001, need, 10, None,
                                ctypes.byref(h)) == B.BM_ERR_WORKSPACE
    assert L.bm_ensemble_attach(ctypes.byref(m), ctypes.byref(r), 0x10000, need - 256, 10, None,
                                ctypes.byref(h)) == B.BM_ERR_WORKSPACE
    assert L.bm_ensemble_attach(ctypes.byref(m), ctypes.byref(r), 0x10000, need, 10, None,
                                None) == B.BM_ERR_INVALID_ARG


# ---------------------------------------------------------------------------
# Scan entry points (no device calls)
# ---------------------------------------------------------------------------
def _scan_arrays(ws):
    mr = [W.to_c(w) for w in ws]
    M = (B.bm_model * len(ws))(*[m for m, _ in mr])
    R = (B.bm_run * len(ws))(*[r for _, r in mr])
    return M, R


def test_scan_workspace_and_validation():
    pts = W.c4_points(64)
    M, R = _scan_arrays(pts)
    n = ctypes.c_size_t()
    assert B.lib().bm_scan_workspace_size(M, R, len(pts), ctypes.byref(n)) == B.BM_OK
    assert n.value % 256 == 0
    assert n.value >= sum((w.n_paths + 63) // 64 for w in pts) * 48
    # empty scan, mixed models, empty window
    assert B.lib().bm_scan_workspace_size(M, R, 0, ctypes.byref(n)) == B.BM_ERR_INVALID_ARG
    M2, R2 = _scan_arrays([pts[0], pts[1].with_(pot=W.POT_RATCHET)])
    assert B.lib().bm_scan_workspace_size(M2, R2, 2, ctypes.byref(n)) == B.BM_ERR_UNSUPPORTED
    M4, R4 = _scan_arrays([pts[0].with_(noise=W.NORMAL)])
    assert B.lib().bm_scan_workspace_size(M4, R4, 1, ctypes.byref(n)) == B.BM_ERR_UNSUPPORTED
    M3, R3 = _scan_arrays([pts[0].with_(n_window=pts[0].n_steps)])
    assert B.lib().bm_scan_workspace_size(M3, R3, 1, ctypes.byref(n)) == B.BM_ERR_INVALID_ARG
    assert "point 0" in B.last_error()


def test_tune_defaults_roundtrip_and_checks():
    # built-in: two paths per lane for FP32 inertial models without jump processes
    t = B.bm_tune_get_default(W.INERTIAL, W.POT_SIN, W.GAUSS, W.F32)
    assert (t.paths_per_lane, t.block, t.groups_per_cu) == (2, 128, 0)
    for dyn, noise, prec in ((W.INERTIAL, W.GAUSS | W.POISSON, W.F32), (W.OVERDAMPED, W.GAUSS, W.F32),
                             (W.INERTIAL, W.GAUSS, W.F64), (W.OVERDAMPED, W.GAUSS | W.DICH, W.F32)):
        t = B.bm_tune_get_default(dyn, W.POT_SIN, noise, prec)
        assert (t.paths_per_lane, t.block, t.groups_per_cu) == (1, 256, 0)
    B.bm_tune_set_default(W.INERTIAL, W.POT_SIN, W.GAUSS, W.F32, B.make_tune(2, 128, 3))
    t = B.bm_tune_get_default(W.INERTIAL, W.POT_SIN, W.GAUSS, W.F32)
    assert (t.paths_per_lane, t.block, t.groups_per_cu) == (2, 128, 3)
    B.bm_tune_set_default(W.INERTIAL, W.POT_SIN, W.GAUSS, W.F32, B.make_tune())
    with pytest.raises(B.BMError) as ex:
        B.bm_tune_set_default(W.INERTIAL, W.POT_SIN, W.GAUSS, W.F64, B.make_tune(2, 256))
    assert ex.value.code == B.BM_ERR_UNSUPPORTED
    with pytest.raises(B.BMError) as ex:
        B.bm_tune_set_default(W.INERTIAL, W.POT_SIN, W.GAUSS, W.F32, B.make_tune(1, 100))
    assert ex.value.code == B.BM_ERR_INVALID_ARG
    with pytest.raises(B.BMError) as ex:      # FP64 Poisson + dichotomous queues of 512 lanes > 64 KiB
        B.bm_tune_set_default(W.INERTIAL, W.POT_SIN, 7, W.F64, B.make_tune(1, 512))
    assert ex.value.code == B.BM_ERR_UNSUPPORTED


def test_scan_plan_needs_device_and_workspace():
    pts = W.c4_points(4)
    M, R = _scan_arrays(pts)
    h = ctypes.c_void_p()
    need = ctypes.c_size_t()
    B.lib().bm_scan_workspace_size(M, R, 4, ctypes.byref(need))
    L = B.lib()
    assert L.bm_scan_plan_create(M, R, 4, None, 0x10000, need.value - 256, 0x20000, None,
                                 ctypes.byref(h)) == B.BM_ERR_WORKSPACE
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if not has_gpu:
        assert L.bm_scan_plan_create(M, R, 4, None, 0x10000, need.value, 0x20000, None,
                                     ctypes.byref(h)) == B.BM_ERR_DEVICE


def test_tune_lookup_reports_installed_shapes():
    key = (B.BM_INERTIAL, B.BM_POT_TENT, B.BM_NOISE_DICH, B.BM_F64)
    assert B.bm_tune_lookup(*key) is None                      # only the built-in default
    B.bm_tune_set_default(*key, B.make_tune(1, 128, 3))
    t = B.bm_tune_lookup(*key)
    assert (t.paths_per_lane, t.block, t.groups_per_cu) == (1, 128, 3)


def test_tune_cache_file_checks(tmp_path):
    L = B.lib()
    assert L.bm_tune_save(b"") == B.BM_ERR_INVALID_ARG
    assert L.bm_tune_load(b"", None) == B.BM_ERR_INVALID_ARG
    assert L.bm_tune_load(os.fsencode(str(tmp_path / "missing.json")), None) == B.BM_ERR_INVALID_ARG
    # shapes installed without a device carry no architecture: the file holds none of them
    B.bm_tune_set_default(B.BM_OVERDAMPED, B.BM_POT_SIN, B.BM_NOISE_GAUSS, B.BM_F32, B.make_tune(1, 64, 0))
    out = tmp_path / "tune.json"
    B.bm_tune_save(str(out))
    import json
    doc = json.loads(out.read_text())
    assert doc["format"] == "libbmotor-tune" and doc["version"] == 1 and doc["entries"] == []
    bad = ['', '{', '[]', '{"entries": {}}', '{"entries": [{"dyn": 1.5}]}', '{"entries": [}',
           '{"format": "x"}', '{"entries": []} trailing', '{"entries": [{"arch": "a\\"b"}]}']
    for i, text in enumerate(bad):
        f = tmp_path / ("bad%d.json" % i)
        f.write_text(text)
        assert L.bm_tune_load(os.fsencode(str(f)), None) == B.BM_ERR_INVALID_ARG, text
    good = tmp_path / "good.json"
    good.write_text('{"version": 1, "note": [1, {"a": null}, -2.5e3], "entries": '
                    '[{"arch": "gfx950", "cus": 256, "dyn": 1, "pot": 0, "noise": 1, "prec": 1, '
                    '"paths_per_lane": 2, "block": 128, "groups_per_cu": 0, "extra": true}]}')
    # a well-formed file gets as far as the device check
    assert L.bm_tune_load(os.fsencode(str(good)), None) == B.BM_ERR_DEVICE


def test_step_control_validation():
    ok_m, ok_r = _ok_model_run(step_tol=1e-6, max_halvings=4)
    assert _ws_rc(ok_m, ok_r)[0] == B.BM_OK
    n_plain = _ws_rc(*_ok_model_run())[1]
    assert _ws_rc(ok_m, ok_r)[1] > n_plain                   # control state and the finer table
    for kw in (dict(step_tol=-1.0), dict(step_tol=float("nan")), dict(step_tol=1e-6, max_halvings=0),
               dict(step_tol=1e-6, max_halvings=9), dict(max_halvings=2), dict(pad=1)):
        m, r = _ok_model_run(**kw)
        assert _ws_rc(m, r)[0] == B.BM_ERR_INVALID_ARG, kw
    m, r = _ok_model_run(step_tol=1e-6, max_halvings=2, noise=B.BM_NOISE_NORMAL)
    assert _ws_rc(m, r)[0] == B.BM_ERR_UNSUPPORTED
    m, r = W.to_c(W.C2.with_(noise=W.GAUSS | W.POISSON | W.JUMP_GRID, step_tol=1e-6, max_halvings=2))
    assert _ws_rc(m, r)[0] == B.BM_ERR_UNSUPPORTED
    m, r = _ok_model_run(step_tol=1e-6, max_halvings=2)
    n = ctypes.c_size_t()
    assert B.lib().bm_scan_workspace_size(ctypes.byref(m), ctypes.byref(r), 1, ctypes.byref(n)) == \
        B.BM_ERR_UNSUPPORTED
