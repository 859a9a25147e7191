"""ctypes binding of libbmotor (include/bmotor.h): argument marshalling only.

Every step of the Monte Carlo path runs in the HIP kernels of libbmotor.so; this
module mirrors the C structs, forwards calls under the same names, and (in
``Ensemble``) allocates the caller-owned workspace as a torch tensor on the
current device and passes torch's current stream.  If the in-tree library is
missing the import fails: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbmotor.so")

BM_OK = 0
BM_ERR_INVALID_ARG = -1
BM_ERR_UNSUPPORTED = -2
BM_ERR_WORKSPACE = -3
BM_ERR_DEVICE = -4
BM_ERR_STATE = -5

BM_OVERDAMPED, BM_INERTIAL = 0, 1
BM_POT_SIN, BM_POT_RATCHET, BM_POT_TENT, BM_POT_FREE = 0, 1, 2, 3
BM_NOISE_GAUSS, BM_NOISE_POISSON, BM_NOISE_DICH, BM_NOISE_NORMAL, BM_NOISE_JUMP_GRID = 1, 2, 4, 8, 16
BM_F64, BM_F32 = 0, 1


class bm_model(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("dyn", ctypes.c_uint32), ("pot", ctypes.c_uint32),
                ("noise", ctypes.c_uint32), ("gamma", ctypes.c_double), ("drive_amp", ctypes.c_double),
                ("drive_omega", ctypes.c_double), ("force", ctypes.c_double), ("D", ctypes.c_double),
                ("shot_rate", ctypes.c_double), ("shot_mean", ctypes.c_double),
                ("dich_Fa", ctypes.c_double), ("dich_Fb", ctypes.c_double),
                ("dich_mua", ctypes.c_double), ("dich_mub", ctypes.c_double)]


class bm_run(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("prec", ctypes.c_uint32),
                ("steps_per_period", ctypes.c_uint32), ("point_id", ctypes.c_uint32),
                ("dt", ctypes.c_double), ("n_steps", ctypes.c_uint64), ("window_start", ctypes.c_uint64),
                ("n_paths", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("x0_lo", ctypes.c_double), ("x0_hi", ctypes.c_double),
                ("v0_lo", ctypes.c_double), ("v0_hi", ctypes.c_double),
                ("step_tol", ctypes.c_double), ("max_halvings", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class bm_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("n_nonfinite", ctypes.c_uint64), ("mean", ctypes.c_double),
                ("var", ctypes.c_double), ("se", ctypes.c_double), ("t_window", ctypes.c_double)]


class bm_path(ctypes.Structure):
    _fields_ = [("periods", ctypes.c_int64), ("x", ctypes.c_double), ("v", ctypes.c_double),
                ("periods_window", ctypes.c_int64), ("x_window", ctypes.c_double),
                ("kick_frac", ctypes.c_double), ("noise", ctypes.c_int64 * 5),
                ("step_level", ctypes.c_int64), ("steps_taken", ctypes.c_int64)]


# numpy view of an array of bm_path records
PATH_RECORD_FIELDS = [("periods", "<i8"), ("x", "<f8"), ("v", "<f8"), ("periods_window", "<i8"),
                      ("x_window", "<f8"), ("kick_frac", "<f8"), ("noise", "<i8", (5,)),
                      ("step_level", "<i8"), ("steps_taken", "<i8")]
PATH_BYTES = ctypes.sizeof(bm_path)


class bm_tune(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("paths_per_lane", ctypes.c_uint32),
                ("block", ctypes.c_uint32), ("groups_per_cu", ctypes.c_uint32)]


STATS_BYTES = ctypes.sizeof(bm_stats)


class BMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libbmotor error %d: %s" % (code, msg))
        self.code = code


_lib = None

# (name, restype, argtypes) of every entry point declared in include/bmotor.h
_vp, _sz = ctypes.c_void_p, ctypes.c_size_t
_P = ctypes.POINTER
SIGNATURES = [
    ("bm_abi_version", ctypes.c_uint32, []),
    ("bm_last_error", ctypes.c_char_p, []),
    ("bm_ensemble_workspace_size", ctypes.c_int, [_P(bm_model), _P(bm_run), _P(_sz)]),
    ("bm_ensemble_create", ctypes.c_int, [_P(bm_model), _P(bm_run), _vp, _sz, _vp, _P(_vp)]),
    ("bm_ensemble_attach", ctypes.c_int, [_P(bm_model), _P(bm_run), _vp, _sz, ctypes.c_uint64, _vp, _P(_vp)]),
    ("bm_ensemble_destroy", ctypes.c_int, [_vp]),
    ("bm_ensemble_set_tune", ctypes.c_int, [_vp, _P(bm_tune)]),
    ("bm_integrate", ctypes.c_int, [_vp, ctypes.c_uint64]),
    ("bm_ensemble_steps", ctypes.c_int, [_vp, _P(ctypes.c_uint64)]),
    ("bm_reduce", ctypes.c_int, [_vp, _vp]),
    ("bm_read_paths", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint64, _vp, _vp, _vp, _vp, _vp]),
    ("bm_write_paths", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint64, _vp]),
    ("bm_density", ctypes.c_int, [_vp, ctypes.c_uint32, _vp]),
    ("bm_scan_workspace_size", ctypes.c_int, [_P(bm_model), _P(bm_run), _sz, _P(_sz)]),
    ("bm_scan_plan_create", ctypes.c_int, [_P(bm_model), _P(bm_run), _sz, _P(bm_tune), _vp, _sz, _vp, _vp,
                                           _P(_vp)]),
    ("bm_scan_plan_launch", ctypes.c_int, [_vp]),
    ("bm_scan_plan_destroy", ctypes.c_int, [_vp]),
    ("bm_scan", ctypes.c_int, [_P(bm_model), _P(bm_run), _sz, _P(bm_tune), _vp, _sz, _vp, _vp]),
    ("bm_scan_autotune", ctypes.c_int, [_P(bm_model), _P(bm_run), _sz, ctypes.c_uint64, _vp, _sz, _vp, _vp,
                                        _P(bm_tune), _P(ctypes.c_float)]),
    ("bm_tune_set_default", ctypes.c_int, [ctypes.c_uint32] * 4 + [_P(bm_tune)]),
    ("bm_tune_get_default", ctypes.c_int, [ctypes.c_uint32] * 4 + [_P(bm_tune)]),
    ("bm_tune_lookup", ctypes.c_int, [ctypes.c_uint32] * 4 + [_P(bm_tune)]),
    ("bm_tune_save", ctypes.c_int, [ctypes.c_char_p]),
    ("bm_tune_load", ctypes.c_int, [ctypes.c_char_p, _P(ctypes.c_uint32)]),
    ("bm_mlp_workspace_size", ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, _P(_sz)]),
    ("bm_mlp_init", ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint64, _vp, _vp]),
    ("bm_mlp_cast", ctypes.c_int, [ctypes.c_uint32, _vp, _vp, _vp]),
    ("bm_mlp_forward", ctypes.c_int, [ctypes.c_uint32, _vp, _vp, _vp, ctypes.c_uint64, _vp, _vp, _sz, _vp]),
    ("bm_mlp_backward", ctypes.c_int, [ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint64, _vp, _vp, _vp,
                                       _sz, _vp]),
    ("bm_mlp_adam_step", ctypes.c_int, [ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint32, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp]),
    ("bm_surrogate_query", ctypes.c_int, [ctypes.c_uint32, _vp, _vp, _vp, ctypes.c_uint64, ctypes.c_float, _vp,
                                          _vp, _vp, _vp, _vp, _sz, _vp]),
    ("bm_surrogate_query_noalloc", ctypes.c_int, [ctypes.c_uint32, _vp, _vp, _vp, ctypes.c_uint64, ctypes.c_float,
                                                  _vp, _vp, _vp, _vp, _vp]),
]

BM_MLP_INPUTS, BM_MLP_HIDDEN, BM_MLP_PARAMS, BM_MLP_BF16, BM_MLP_MAX_MEMBERS = 5, 256, 133377, 132608, 16
BM_QUERY_SCRATCH_BYTES = 33554432


def lib() -> ctypes.CDLL:
    """Load the in-tree libbmotor.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbmotor.so not built (run python -m paper_1409_4923_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().bm_last_error().decode()


def check(rc: int) -> None:
    if rc != BM_OK:
        raise BMError(rc, last_error())


def make_model(**kw) -> bm_model:
    m = bm_model()
    m.size = ctypes.sizeof(bm_model)
    m.gamma, m.drive_omega, m.dich_mua, m.dich_mub, m.shot_rate = 1.0, 1.0, 1.0, 1.0, 1.0
    for k, v in kw.items():
        setattr(m, k, v)
    return m


def make_run(**kw) -> bm_run:
    r = bm_run()
    r.size = ctypes.sizeof(bm_run)
    r.x0_hi = 1.0
    r.n_paths = 1
    for k, v in kw.items():
        setattr(r, k, v)
    return r


def make_tune(paths_per_lane: int = 1, block: int = 256, groups_per_cu: int = 0) -> bm_tune:
    t = bm_tune()
    t.size = ctypes.sizeof(bm_tune)
    t.paths_per_lane = paths_per_lane
    t.block = block
    t.groups_per_cu = groups_per_cu
    return t


# ---------------------------------------------------------------------------
# Same-name thin wrappers (raise BMError on failure)
# ---------------------------------------------------------------------------
def bm_abi_version() -> int:
    return int(lib().bm_abi_version())


def bm_ensemble_workspace_size(model: bm_model, run: bm_run) -> int:
    n = ctypes.c_size_t()
    check(lib().bm_ensemble_workspace_size(ctypes.byref(model), ctypes.byref(run), ctypes.byref(n)))
    return int(n.value)


def bm_ensemble_create(model: bm_model, run: bm_run, d_ws: int, ws_bytes: int, stream: int) -> int:
    h = ctypes.c_void_p()
    check(lib().bm_ensemble_create(ctypes.byref(model), ctypes.byref(run), d_ws, ws_bytes, stream,
                                   ctypes.byref(h)))
    return int(h.value)


def bm_ensemble_attach(model: bm_model, run: bm_run, d_ws: int, ws_bytes: int, steps_done: int,
                       stream: int) -> int:
    h = ctypes.c_void_p()
    check(lib().bm_ensemble_attach(ctypes.byref(model), ctypes.byref(run), d_ws, ws_bytes, steps_done, stream,
                                   ctypes.byref(h)))
    return int(h.value)


def bm_ensemble_destroy(h: int) -> None:
    check(lib().bm_ensemble_destroy(h))


def bm_ensemble_set_tune(h: int, tune: bm_tune | None) -> None:
    check(lib().bm_ensemble_set_tune(h, ctypes.byref(tune) if tune is not None else None))


def bm_integrate(h: int, n_steps: int) -> None:
    check(lib().bm_integrate(h, n_steps))


def bm_ensemble_steps(h: int) -> int:
    n = ctypes.c_uint64()
    check(lib().bm_ensemble_steps(h, ctypes.byref(n)))
    return int(n.value)


def bm_reduce(h: int, d_out: int) -> None:
    check(lib().bm_reduce(h, d_out))


def bm_density(h: int, n_bins: int, d_counts: int) -> None:
    check(lib().bm_density(h, n_bins, d_counts))


def bm_read_paths(h: int, first: int, count: int, d_x: int | None, d_v: int | None,
                  d_noise: int | None, d_vp: int | None, d_state: int | None = None) -> None:
    check(lib().bm_read_paths(h, first, count, d_x, d_v, d_noise, d_vp, d_state))


def bm_write_paths(h: int, first: int, count: int, d_state: int) -> None:
    check(lib().bm_write_paths(h, first, count, d_state))


# ---------------------------------------------------------------------------
# Convenience owner of a workspace (torch device memory + current stream)
# ---------------------------------------------------------------------------
@dataclass
class PathState:
    x: "object"       # unwrapped position, float64 tensor
    v: "object"       # velocity, float64 tensor
    noise: "object"   # int64 [count, 5]: sP, kP, sD, mD, d
    vp: "object"      # eq. (31) per-path velocity (NaN until the window is open)


class Ensemble:
    """An ensemble of paths living in a torch-allocated workspace on the current GPU."""

    def __init__(self, model: bm_model, run: bm_run, tune: bm_tune | None = None, device=None,
                 checkpoint=None):
        """checkpoint: (workspace bytes as a uint8 tensor, steps done) from `checkpoint()`;
        the ensemble then resumes from that state instead of drawing initial conditions."""
        import torch
        self.torch = torch
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.model, self.run = model, run
        self.ws_bytes = bm_ensemble_workspace_size(model, run)
        self.stream = torch.cuda.current_stream(self.device)
        if checkpoint is None:
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            self.h = bm_ensemble_create(model, run, self.ws.data_ptr(), self.ws_bytes, self.stream.cuda_stream)
        else:
            data, steps = checkpoint
            if data.dtype != torch.uint8 or data.numel() != self.ws_bytes:
                raise ValueError("checkpoint holds %d bytes, this ensemble needs %d" % (data.numel(), self.ws_bytes))
            self.ws = data.to(self.device).contiguous().clone()
            self.h = bm_ensemble_attach(model, run, self.ws.data_ptr(), self.ws_bytes, int(steps),
                                        self.stream.cuda_stream)
        if tune is not None:
            bm_ensemble_set_tune(self.h, tune)

    @classmethod
    def resume(cls, model: bm_model, run: bm_run, steps_done: int, tune: bm_tune | None = None, device=None):
        """An ensemble opened at `steps_done` on a fresh workspace whose paths hold no
        state yet: every path is to be written with write_state before integrating."""
        import torch
        self = cls.__new__(cls)
        self.torch = torch
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.model, self.run = model, run
        self.ws_bytes = bm_ensemble_workspace_size(model, run)
        self.stream = torch.cuda.current_stream(self.device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.h = bm_ensemble_attach(model, run, self.ws.data_ptr(), self.ws_bytes, int(steps_done),
                                    self.stream.cuda_stream)
        if tune is not None:
            bm_ensemble_set_tune(self.h, tune)
        return self

    def checkpoint(self, device="cpu"):
        """(copy of the workspace, steps done): the whole state of the ensemble."""
        self.stream.synchronize()
        return self.ws.to(device, copy=True), self.steps

    def close(self):
        if getattr(self, "h", None):
            bm_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tune(self, tune: bm_tune | None):
        bm_ensemble_set_tune(self.h, tune)

    def integrate(self, n_steps: int):
        bm_integrate(self.h, n_steps)

    @property
    def steps(self) -> int:
        return bm_ensemble_steps(self.h)

    def reduce(self, out=None):
        """Enqueue the reduction; returns the raw 48-byte device tensor holding bm_stats."""
        torch = self.torch
        if out is None:
            out = torch.empty(STATS_BYTES, dtype=torch.uint8, device=self.device)
        bm_reduce(self.h, out.data_ptr())
        return out

    def stats(self) -> bm_stats:
        raw = self.reduce()
        self.stream.synchronize()
        return stats_from_bytes(raw.cpu().numpy().tobytes())

    def density(self, counts):
        """Add the histogram of the folded positions to the int64 tensor `counts` (eq. 19)."""
        bm_density(self.h, counts.numel(), counts.data_ptr())
        return counts

    def read_state(self, first: int = 0, count: int | None = None):
        """bm_path records of paths [first, first + count) as a uint8 device tensor
        (count x PATH_BYTES); `records()` turns it into a numpy structured array."""
        torch = self.torch
        count = self.run.n_paths - first if count is None else count
        st = torch.empty(max(count, 1) * PATH_BYTES, dtype=torch.uint8, device=self.device)
        bm_read_paths(self.h, first, count, None, None, None, None, st.data_ptr())
        return st[: count * PATH_BYTES]

    def write_state(self, state, first: int = 0):
        """Write bm_path records (a uint8 device tensor from read_state, or a numpy
        structured array of PATH_RECORD_FIELDS) into paths first, first + 1, ..."""
        torch = self.torch
        if not isinstance(state, torch.Tensor):
            import numpy as np
            state = torch.from_numpy(np.ascontiguousarray(state).view(np.uint8).reshape(-1))
        state = state.to(self.device).contiguous()
        if state.numel() % PATH_BYTES:
            raise ValueError("state holds %d bytes, not a whole number of bm_path records" % state.numel())
        bm_write_paths(self.h, first, state.numel() // PATH_BYTES, state.data_ptr())
        self._keep = state          # the copy is enqueued on the stream: keep the source alive

    def read(self, first: int = 0, count: int | None = None) -> PathState:
        torch = self.torch
        count = self.run.n_paths - first if count is None else count
        x = torch.empty(count, dtype=torch.float64, device=self.device)
        v = torch.empty(count, dtype=torch.float64, device=self.device)
        nz = torch.empty((count, 5), dtype=torch.int64, device=self.device)
        vp = torch.full((count,), float("nan"), dtype=torch.float64, device=self.device)
        bm_read_paths(self.h, first, count, x.data_ptr(), v.data_ptr(), nz.data_ptr(), vp.data_ptr())
        self.stream.synchronize()
        return PathState(x.cpu(), v.cpu(), nz.cpu(), vp.cpu())


def records(state):
    """numpy structured array (PATH_RECORD_FIELDS) of a read_state tensor."""
    import numpy as np
    raw = state.cpu().numpy() if hasattr(state, "cpu") else np.asarray(state, dtype=np.uint8)
    return raw.view(np.dtype(PATH_RECORD_FIELDS))


def stats_from_bytes(b: bytes) -> bm_stats:
    s = bm_stats()
    ctypes.memmove(ctypes.byref(s), b, STATS_BYTES)
    return s


# ---------------------------------------------------------------------------
# Batched scan
# ---------------------------------------------------------------------------
def _arrays(models, runs):
    """ctypes arrays of the records: passed through when given as such (see
    record_arrays), else built from sequences of bm_model / bm_run."""
    n = len(models)
    assert n == len(runs) and n > 0
    if isinstance(models, ctypes.Array) and isinstance(runs, ctypes.Array):
        return models, runs, n
    M = (bm_model * n)(*models)
    R = (bm_run * n)(*runs)
    return M, R, n


def record_arrays(n: int):
    """Zeroed numpy record arrays of n bm_model and n bm_run records (the sizes and the
    defaults of make_model / make_run filled in), and ctypes arrays over the same memory
    for the scan calls: fill the numpy columns, then pass the ctypes arrays."""
    import numpy as np
    mo = np.zeros(n, dtype=np.dtype(bm_model))
    ru = np.zeros(n, dtype=np.dtype(bm_run))
    mo["size"] = ctypes.sizeof(bm_model)
    for f in ("gamma", "drive_omega", "dich_mua", "dich_mub", "shot_rate"):
        mo[f] = 1.0
    ru["size"] = ctypes.sizeof(bm_run)
    ru["x0_hi"] = 1.0
    ru["n_paths"] = 1
    return mo, ru, (bm_model * n).from_buffer(mo), (bm_run * n).from_buffer(ru)


def bm_scan_workspace_size(models, runs) -> int:
    M, R, n = _arrays(models, runs)
    b = ctypes.c_size_t()
    check(lib().bm_scan_workspace_size(M, R, n, ctypes.byref(b)))
    return int(b.value)


def bm_scan_plan_create(models, runs, tune, d_ws: int, ws_bytes: int, d_results: int, stream: int) -> int:
    M, R, n = _arrays(models, runs)
    h = ctypes.c_void_p()
    check(lib().bm_scan_plan_create(M, R, n, ctypes.byref(tune) if tune is not None else None, d_ws, ws_bytes,
                                    d_results, stream, ctypes.byref(h)))
    return int(h.value)


def bm_scan_plan_launch(h: int) -> None:
    check(lib().bm_scan_plan_launch(h))


def bm_scan_plan_destroy(h: int) -> None:
    check(lib().bm_scan_plan_destroy(h))


def bm_scan(models, runs, tune, d_ws: int, ws_bytes: int, d_results: int, stream: int) -> None:
    M, R, n = _arrays(models, runs)
    check(lib().bm_scan(M, R, n, ctypes.byref(tune) if tune is not None else None, d_ws, ws_bytes, d_results,
                        stream))


def bm_scan_autotune(models, runs, max_steps: int, d_ws: int, ws_bytes: int, d_results: int, stream: int):
    M, R, n = _arrays(models, runs)
    t = bm_tune()
    ms = ctypes.c_float()
    check(lib().bm_scan_autotune(M, R, n, max_steps, d_ws, ws_bytes, d_results, stream, ctypes.byref(t),
                                 ctypes.byref(ms)))
    return t, float(ms.value)


def bm_tune_set_default(dyn: int, pot: int, noise: int, prec: int, tune: bm_tune) -> None:
    check(lib().bm_tune_set_default(dyn, pot, noise, prec, ctypes.byref(tune)))


def bm_tune_get_default(dyn: int, pot: int, noise: int, prec: int) -> bm_tune:
    t = bm_tune()
    check(lib().bm_tune_get_default(dyn, pot, noise, prec, ctypes.byref(t)))
    return t


def bm_tune_lookup(dyn: int, pot: int, noise: int, prec: int):
    """The launch shape set, tuned or loaded for this key, or None if only the
    built-in default applies."""
    t = bm_tune()
    rc = lib().bm_tune_lookup(dyn, pot, noise, prec, ctypes.byref(t))
    if rc == BM_ERR_STATE:
        return None
    check(rc)
    return t


def bm_tune_save(path: str) -> None:
    check(lib().bm_tune_save(os.fsencode(path)))


def bm_tune_load(path: str) -> int:
    n = ctypes.c_uint32()
    check(lib().bm_tune_load(os.fsencode(path), ctypes.byref(n)))
    return int(n.value)


def autotune_cached(models, runs, max_steps: int, d_ws: int, ws_bytes: int, d_results: int, stream: int,
                    cache: str):
    """Launch shape for the scan of (models, runs): taken from the JSON cache file
    `cache` when it holds one for this model family and device (no timing), else
    found by bm_scan_autotune and added to the file.  Returns (bm_tune, ms or None)."""
    m0, r0 = models[0], runs[0]
    if os.path.exists(cache):
        bm_tune_load(cache)
        t = bm_tune_lookup(m0.dyn, m0.pot, m0.noise, r0.prec)
        if t is not None:
            return t, None
    t, ms = bm_scan_autotune(models, runs, max_steps, d_ws, ws_bytes, d_results, stream)
    d = os.path.dirname(os.path.abspath(cache))
    os.makedirs(d, exist_ok=True)
    bm_tune_save(cache)
    return t, ms


def stats_array_from_bytes(b: bytes, n: int):
    arr = (bm_stats * n)()
    ctypes.memmove(arr, b, STATS_BYTES * n)
    return list(arr)


class Scan:
    """A planned scan over (bm_model, bm_run) pairs; workspace and results are torch tensors."""

    def __init__(self, models, runs, tune: bm_tune | None = None, device=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.models = models if isinstance(models, ctypes.Array) else list(models)
        self.runs = runs if isinstance(runs, ctypes.Array) else list(runs)
        self.n = len(self.models)
        self.ws_bytes = bm_scan_workspace_size(self.models, self.runs)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.results = torch.empty(self.n * STATS_BYTES, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = bm_scan_plan_create(self.models, self.runs, tune, self.ws.data_ptr(), self.ws_bytes,
                                     self.results.data_ptr(), self.stream.cuda_stream)

    def launch(self):
        bm_scan_plan_launch(self.h)

    def stats(self):
        self.stream.synchronize()
        return stats_array_from_bytes(self.results.cpu().numpy().tobytes(), self.n)

    def stats_records(self):
        """The per-point bm_stats as a numpy record array (fields n, n_nonfinite, mean,
        var, se, t_window)."""
        import numpy as np
        self.stream.synchronize()
        return np.frombuffer(self.results.cpu().numpy().tobytes(), dtype=np.dtype(bm_stats), count=self.n)

    def close(self):
        if getattr(self, "h", None):
            bm_scan_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Surrogate
# ---------------------------------------------------------------------------
def bm_mlp_workspace_size(n_members: int, batch: int, training: bool) -> int:
    b = ctypes.c_size_t()
    check(lib().bm_mlp_workspace_size(n_members, batch, int(training), ctypes.byref(b)))
    return int(b.value)


def bm_mlp_init(n_members: int, seed: int, d_params: int, stream: int) -> None:
    check(lib().bm_mlp_init(n_members, seed, d_params, stream))


def bm_mlp_cast(n_members: int, d_params: int, d_wbf: int, stream: int) -> None:
    check(lib().bm_mlp_cast(n_members, d_params, d_wbf, stream))


def bm_mlp_forward(n_members, d_params, d_wbf, d_x, batch, d_y, d_ws, ws_bytes, stream) -> None:
    check(lib().bm_mlp_forward(n_members, d_params, d_wbf, d_x, batch, d_y, d_ws, ws_bytes, stream))


def bm_mlp_backward(n_members, d_params, d_wbf, d_x, d_t, d_idx, batch, d_grad, d_loss, d_ws, ws_bytes,
                    stream) -> None:
    check(lib().bm_mlp_backward(n_members, d_params, d_wbf, d_x, d_t, d_idx, batch, d_grad, d_loss, d_ws,
                                ws_bytes, stream))


def bm_mlp_adam_step(n_members, d_params, d_grad, d_m, d_v, d_wbf, step, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                stream=None) -> None:
    check(lib().bm_mlp_adam_step(n_members, d_params, d_grad, d_m, d_v, d_wbf, step, lr, beta1, beta2, eps, stream))


def bm_surrogate_query(n_members, d_params, d_wbf, d_x, batch, threshold, d_mean, d_std, d_fidx, d_fcount, d_ws,
                       ws_bytes, stream) -> None:
    check(lib().bm_surrogate_query(n_members, d_params, d_wbf, d_x, batch, threshold, d_mean, d_std, d_fidx,
                                   d_fcount, d_ws, ws_bytes, stream))


def bm_surrogate_query_noalloc(n_members, d_params, d_wbf, d_x, batch, threshold, d_mean, d_std, d_fidx, d_fcount,
                               stream) -> None:
    check(lib().bm_surrogate_query_noalloc(n_members, d_params, d_wbf, d_x, batch, threshold, d_mean, d_std, d_fidx,
                                           d_fcount, stream))


class Surrogate:
    """Ensemble MLP whose parameters, Adam moments and BF16 copies are torch tensors."""

    def __init__(self, n_members: int = 5, params=None, seed: int = 0, device=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.n = n_members
        self.stream = torch.cuda.current_stream(self.device)
        s = self.stream.cuda_stream
        self.params = torch.empty((n_members, BM_MLP_PARAMS), dtype=torch.float32, device=self.device)
        if params is None:
            bm_mlp_init(n_members, seed, self.params.data_ptr(), s)
        else:
            self.params.copy_(torch.as_tensor(params, dtype=torch.float32))
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.wbf = torch.empty((n_members, BM_MLP_BF16), dtype=torch.int16, device=self.device)
        self.step = 0
        self._ws = {}
        self.cast()

    def _workspace(self, batch: int, training: bool):
        key = (batch, training)
        if key not in self._ws:
            nb = bm_mlp_workspace_size(self.n, batch, training)
            self._ws = {key: self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)}
        w = self._ws[key]
        return w.data_ptr(), w.numel()

    def cast(self):
        bm_mlp_cast(self.n, self.params.data_ptr(), self.wbf.data_ptr(), self.stream.cuda_stream)

    def forward(self, x):
        x = x.contiguous()
        B = x.shape[0]
        y = self.torch.empty((self.n, B), dtype=self.torch.float32, device=self.device)
        ws, nb = self._workspace(B, False)
        bm_mlp_forward(self.n, self.params.data_ptr(), self.wbf.data_ptr(), x.data_ptr(), B, y.data_ptr(), ws, nb,
                       self.stream.cuda_stream)
        return y

    def backward(self, x, t, idx=None):
        if idx is not None and (not idx.is_contiguous() or idx.dtype != self.torch.int32
                                or idx.dim() != 2 or idx.shape[0] != self.n):
            raise ValueError("idx must be a contiguous int32 tensor [n_members, batch]")
        B = idx.shape[1] if idx is not None else x.shape[0]
        loss = self.torch.empty(self.n, dtype=self.torch.float32, device=self.device)
        ws, nb = self._workspace(B, True)
        bm_mlp_backward(self.n, self.params.data_ptr(), self.wbf.data_ptr(), x.data_ptr(), t.data_ptr(),
                        idx.data_ptr() if idx is not None else None, B, self.grad.data_ptr(), loss.data_ptr(),
                        ws, nb, self.stream.cuda_stream)
        return loss

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        bm_mlp_adam_step(self.n, self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                    self.wbf.data_ptr(), self.step, lr, beta1, beta2, eps, self.stream.cuda_stream)

    def query(self, x, threshold: float):
        """(mean, std, fallback indices) for rows x [B, 5]."""
        torch = self.torch
        x = x.contiguous()
        B = x.shape[0]
        mean = torch.empty(B, dtype=torch.float32, device=self.device)
        std = torch.empty(B, dtype=torch.float32, device=self.device)
        fidx = torch.empty(B, dtype=torch.int32, device=self.device)
        fcnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        ws, nb = self._workspace(B, False)
        bm_surrogate_query(self.n, self.params.data_ptr(), self.wbf.data_ptr(), x.data_ptr(), B, threshold,
                           mean.data_ptr(), std.data_ptr(), fidx.data_ptr(), fcnt.data_ptr(), ws, nb,
                           self.stream.cuda_stream)
        return mean, std, fidx, fcnt
