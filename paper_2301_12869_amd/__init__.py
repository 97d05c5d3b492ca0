"""Python binding of the MI355X thermal pseudopotential LBM library (libtplbm.so).

Argument marshalling only: every step of the lattice update runs in the HIP
kernels behind the C ABI of ``include/tplbm.h``.  PyTorch supplies device
memory (one workspace tensor per lattice) and the HIP stream.  There is no CPU
fallback: if the library is missing, importing works but every constructor
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtplbm.so")

OK, EINVAL, ESHAPE, EUNSUPPORTED, EHIP, EUNPHYSICAL, ENOTCONVERGED, ENOSOLUTION = range(8)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ESHAPE", 3: "EUNSUPPORTED", 4: "EHIP",
                5: "EUNPHYSICAL", 6: "ENOTCONVERGED", 7: "ENOSOLUTION"}
D1Q3, D2Q9, D3Q19 = 1, 2, 3
FP64, FP32_DEV = 0, 1
STATE_AUTO, STATE_POPULATIONS, STATE_MOMENTS = 0, 1, 2
FIELDS = {"rho": 0, "ux": 1, "uy": 2, "uz": 3, "T": 4, "p_eos": 5, "p_nn": 6}
FLAG_NAMES = {1: "nan", 2: "rho<=0", 4: "eta>=1", 8: "psi undefined"}

PAPER = dict(a=0.5, b=4.0, R=1.0, G=-1.0, sigma=1.385, tau=(1.0,) * 6, cv=5.0, kappa=0.02)


class TplbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("walls", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("eos", ctypes.c_int32), ("gravity_form", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
        ("G", ctypes.c_double), ("sigma", ctypes.c_double), ("tau", ctypes.c_double * 6),
        ("cv", ctypes.c_double), ("kappa", ctypes.c_double), ("g", ctypes.c_double),
        ("rho_ref", ctypes.c_double), ("state", ctypes.c_int32), ("ref_interval", ctypes.c_int32),
        ("rho_v", ctypes.c_double),
    ]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("first_bad_step", ctypes.c_int64),
                ("mass", ctypes.c_double), ("mean_rho", ctypes.c_double),
                ("max_u", ctypes.c_double), ("min_rho", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


_lib = None

# (name, argtypes, restype) of every entry point declared in include/tplbm.h
_VP, _DP, _SZ = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_size_t)
_PP = ctypes.POINTER(Params)
SIGNATURES = {
    "tplbm_workspace_bytes": ([_PP, _SZ], ctypes.c_int),
    "tplbm_create": ([_PP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)], ctypes.c_int),
    "tplbm_set_state": ([_VP, _DP, _DP], ctypes.c_int),
    "tplbm_step": ([_VP, ctypes.c_int64], ctypes.c_int),
    "tplbm_step_async": ([_VP, ctypes.c_int64], ctypes.c_int),
    "tplbm_read": ([_VP, ctypes.c_int, _DP], ctypes.c_int),
    "tplbm_read_device": ([_VP, ctypes.c_int, _VP], ctypes.c_int),
    "tplbm_diagnostics": ([_VP, ctypes.POINTER(Diag)], ctypes.c_int),
    "tplbm_state_bytes": ([_VP, _SZ], ctypes.c_int),
    "tplbm_save_state": ([_VP, _VP], ctypes.c_int),
    "tplbm_load_state": ([_VP, _VP, ctypes.c_size_t], ctypes.c_int),
    "tplbm_destroy": ([_VP], None),
    "tplbm_last_error": ([_VP], ctypes.c_char_p),
    "tplbm_stream_copy": ([_VP, _VP, ctypes.c_size_t, _VP], ctypes.c_int),
    "tplbm_eos_critical": ([ctypes.c_double] * 3 + [_DP], ctypes.c_int),
    "tplbm_eos_coexistence": ([ctypes.c_double] * 4 + [_DP], ctypes.c_int),
    "tplbm_eos_spinodal": ([ctypes.c_double] * 4 + [_DP], ctypes.c_int),
}


class Column(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("gravity_form", ctypes.c_int32), ("g", ctypes.c_double),
                ("rho_v", ctypes.c_double)]


class BatchParams(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
                ("G", ctypes.c_double), ("sigma", ctypes.c_double), ("cv", ctypes.c_double),
                ("kappa", ctypes.c_double), ("eos", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ColResult(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("mass", ctypes.c_double), ("max_u", ctypes.c_double)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("nodes_per_thread", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("node_steps_per_s", ctypes.c_double)]


_BP = ctypes.POINTER(BatchParams)
_CP = ctypes.POINTER(Column)
SIGNATURES.update({
    "tplbm_batch_workspace_bytes": ([_BP, ctypes.c_int32, _CP, _SZ], ctypes.c_int),
    "tplbm_batch_create": ([_BP, ctypes.c_int32, _CP, _VP, ctypes.c_size_t, _VP,
                            ctypes.POINTER(_VP)], ctypes.c_int),
    "tplbm_batch_set_state": ([_VP, _DP, _DP], ctypes.c_int),
    "tplbm_batch_run": ([_VP, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ColResult)],
                        ctypes.c_int),
    "tplbm_batch_read": ([_VP, ctypes.c_int, _DP], ctypes.c_int),
    "tplbm_batch_autotune": ([_VP, ctypes.c_double, ctypes.POINTER(BatchTuning)], ctypes.c_int),
    "tplbm_batch_set_tuning": ([_VP, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "tplbm_batch_resume": ([_VP, _DP, _DP], ctypes.c_int),
    "tplbm_batch_destroy": ([_VP], None),
    "tplbm_batch_last_error": ([_VP], ctypes.c_char_p),
    "tplbm_batch_run_noalloc": ([_BP, ctypes.c_int32, _CP, _VP, _VP, _VP, _VP, _VP, ctypes.c_double,
                                 ctypes.c_int64, ctypes.c_int32, _VP], ctypes.c_int),
})
COL_STATUS = {0: "converged", 1: "diverged", 2: "max_steps"}


def load_library():
    """Load libtplbm.so (built by paper_2301_12869_amd.build)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname as the one the
        # library links; loading torch first makes the process hold one
        # runtime (torch's), which the library then binds to.  Loaded the
        # other way round, the two runtimes meet and HIP finds no device.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2301_12869_amd.build` (no CPU fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _device(device=None):
    """torch device with its index (a bare "cuda" becomes the current device),
    so that it compares equal to the device of a tensor allocated on it."""
    import torch

    d = torch.device(device or "cuda")
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _check(rc: int, ctx=None):
    if rc != OK:
        msg = load_library().tplbm_last_error(ctx).decode()
        raise TplbmError(rc, msg)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_DP)


# ---------------------------------------------------------------------------
# host FP64 equation-of-state utilities
# ---------------------------------------------------------------------------
def eos_critical(a=0.5, b=4.0, R=1.0):
    out = np.zeros(3)
    _check(load_library().tplbm_eos_critical(a, b, R, _dp(out)))
    return tuple(float(v) for v in out)  # rho_c, T_c, p_c


def eos_coexistence(T, a=0.5, b=4.0, R=1.0):
    out = np.zeros(3)
    _check(load_library().tplbm_eos_coexistence(a, b, R, float(T), _dp(out)))
    return tuple(float(v) for v in out)  # rho_v, rho_l, p_sat


def eos_spinodal(T, a=0.5, b=4.0, R=1.0):
    out = np.zeros(2)
    _check(load_library().tplbm_eos_spinodal(a, b, R, float(T), _dp(out)))
    return tuple(float(v) for v in out)


# ---------------------------------------------------------------------------
# sharp-interface theory of a column (host, FP64)
# ---------------------------------------------------------------------------
THEORY_CONFIGS = {"L-V": 0, "V-L": 1, "V-L-V": 2}
THEORY_REASONS = {1: "liquid spinodal", 2: "vapour spinodal", 4: "zero pressure",
                  8: "interface above T_c", 16: "no second interface", 32: "no placement matches the mean",
                  64: "broken bracket", 128: "EOS solve failed"}


class TheoryColumn(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("gravity_form", ctypes.c_int32),
                ("config", ctypes.c_int32), ("substeps", ctypes.c_int32),
                ("T_bot", ctypes.c_double), ("T_top", ctypes.c_double),
                ("g", ctypes.c_double), ("mean_rho", ctypes.c_double), ("rho_v", ctypes.c_double)]


class TheoryResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_interfaces", ctypes.c_int32),
                ("reasons", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("interface", ctypes.c_double * 2), ("mean_rho", ctypes.c_double)]


SIGNATURES.update({
    "tplbm_theory_solve": ([ctypes.c_double] * 3 + [ctypes.c_int32, ctypes.POINTER(TheoryColumn), _DP, _DP,
                                                   ctypes.POINTER(TheoryResult), ctypes.c_int32], ctypes.c_int),
    "tplbm_theory_last_error": ([], ctypes.c_char_p),
})


def theory_solve(columns, substeps=8, nthreads=0, a=0.5, b=4.0, R=1.0):
    """Sharp-interface equilibria of columns given as tuples
    (height, T_bot, T_top, g, gravity_form, mean_rho, config[, rho_v]) with
    config one of "L-V", "V-L", "V-L-V" (rho_v: gravity form 3).  Returns one dict per column: rho, p (node
    arrays) and interfaces for a configuration that exists, else None for
    rho/p and the list of reasons."""
    n = len(columns)
    cols = (TheoryColumn * max(n, 1))()
    heights = []
    for k, col in enumerate(columns):
        h, tb, tt, g, form, mean, cfg = col[:7]
        rv = float(col[7]) if len(col) > 7 else 0.0
        cols[k] = TheoryColumn(int(h), int(form), THEORY_CONFIGS[cfg], int(substeps),
                               float(tb), float(tt), float(g), float(mean), rv)
        heights.append(int(h))
    total = sum(heights)
    rho, p = np.empty(max(total, 1)), np.empty(max(total, 1))
    res = (TheoryResult * max(n, 1))()
    rc = load_library().tplbm_theory_solve(a, b, R, n, cols, _dp(rho), _dp(p), res, int(nthreads))
    if rc != OK:
        raise TplbmError(rc, load_library().tplbm_theory_last_error().decode())
    out, off = [], 0
    for k, h in enumerate(heights):
        r = res[k]
        if r.status == OK:
            out.append(dict(rho=rho[off:off + h].copy(), p=p[off:off + h].copy(),
                            interfaces=list(r.interface[:r.n_interfaces]), mean=r.mean_rho, reasons=[]))
        else:
            out.append(dict(rho=None, p=None, interfaces=[], mean=None,
                            reasons=[v for bit, v in THEORY_REASONS.items() if r.reasons & bit]))
        off += h
    return out


def make_params(lattice=D2Q9, nx=1, ny=1, nz=1, walls=True, precision=FP64, eos="cs",
                gravity_form=1, g=0.0, rho_ref=0.0, state=STATE_AUTO, rho_v=0.0, ref_interval=0,
                **over) -> Params:
    """Lattice parameters (paper values unless overridden).  FP32_DEV storage
    keeps one reference density per wall-normal layer, re-centred every
    ref_interval steps (0: the library's default interval; < 0: rho_ref for
    every layer, never re-centred)."""
    d = dict(PAPER)
    d.update(over)
    p = Params()
    p.lattice = int(lattice)
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.walls = 1 if walls else 0
    p.precision = int(precision)
    p.eos = {"cs": 0, "ideal": 1}[eos]
    p.gravity_form = int(gravity_form)
    p.a, p.b, p.R, p.G, p.sigma = d["a"], d["b"], d["R"], d["G"], d["sigma"]
    for k in range(6):
        p.tau[k] = float(d["tau"][k])
    p.cv, p.kappa, p.g, p.rho_ref = d["cv"], d["kappa"], float(g), float(rho_ref)
    p.state, p.ref_interval = int(state), int(ref_interval)
    p.rho_v = float(rho_v)
    return p


class Lattice:
    """A D2Q9 (or D3Q19) lattice living in one device workspace."""

    def __init__(self, params: Params, device=None, stream=None):
        import torch

        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP lattice needs an MI355X")
        self.params = params
        nbytes = ctypes.c_size_t()
        _check(lib.tplbm_workspace_bytes(ctypes.byref(params), ctypes.byref(nbytes)))
        self.device = _device(device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = _VP()
        _check(lib.tplbm_create(ctypes.byref(params), self.workspace.data_ptr(), int(nbytes.value),
                                self.stream.cuda_stream, ctypes.byref(h)))
        self._h = h
        self.n = params.nx * params.ny * (params.nz if params.lattice == D3Q19 else 1)

    # -- state -------------------------------------------------------------
    def set_state(self, rho0, T0):
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64).ravel()
        T0 = np.ascontiguousarray(T0, dtype=np.float64).ravel()
        if rho0.size != self.n or T0.size != self.n:
            raise ValueError(f"expected {self.n} values, got {rho0.size} and {T0.size}")
        _check(load_library().tplbm_set_state(self._h, _dp(rho0), _dp(T0)), self._h)

    def step(self, n: int = 1):
        _check(load_library().tplbm_step(self._h, int(n)), self._h)

    def step_async(self, n: int = 1):
        _check(load_library().tplbm_step_async(self._h, int(n)), self._h)

    def read(self, field: str) -> np.ndarray:
        out = np.empty(self.n)
        _check(load_library().tplbm_read(self._h, FIELDS[field], _dp(out)), self._h)
        return out

    def read_device(self, field: str, out):
        """Enqueue a readout into a contiguous float64 tensor of n elements on
        this lattice's device."""
        import torch

        if not isinstance(out, torch.Tensor) or out.device != self.device:
            raise ValueError(f"out must be a tensor on {self.device}")
        if out.dtype != torch.float64 or out.numel() != self.n or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float64 tensor of {self.n} elements")
        _check(load_library().tplbm_read_device(self._h, FIELDS[field], out.data_ptr()), self._h)

    def diagnostics(self) -> dict:
        d = Diag()
        _check(load_library().tplbm_diagnostics(self._h, ctypes.byref(d)), self._h)
        return dict(step=d.step, first_bad_step=d.first_bad_step, mass=d.mass,
                    mean_rho=d.mean_rho, max_u=d.max_u, min_rho=d.min_rho, flags=d.flags)

    def save_state(self) -> bytes:
        nb = ctypes.c_size_t()
        _check(load_library().tplbm_state_bytes(self._h, ctypes.byref(nb)), self._h)
        buf = ctypes.create_string_buffer(int(nb.value))
        _check(load_library().tplbm_save_state(self._h, buf), self._h)
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(load_library().tplbm_load_state(self._h, buf, len(blob)), self._h)

    def close(self):
        if getattr(self, "_h", None):
            load_library().tplbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bcheck(rc: int, h=None):
    if rc != OK:
        raise TplbmError(rc, load_library().tplbm_batch_last_error(h).decode())


class Batch:
    """Many independent 1-D columns swept to steady state by one persistent
    launch.  columns: sequence of (height, gravity_form, g) or
    (height, gravity_form, g, rho_v) (rho_v: gravity form 3)."""

    def __init__(self, columns, eos="cs", device=None, stream=None, **over):
        import torch

        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the batched sweep needs an MI355X")
        d = dict(PAPER)
        d.update(over)
        p = BatchParams()
        p.a, p.b, p.R, p.G, p.sigma = d["a"], d["b"], d["R"], d["G"], d["sigma"]
        p.cv, p.kappa = d["cv"], d["kappa"]
        p.eos = {"cs": 0, "ideal": 1}[eos]
        self.params = p
        self.ncols = len(columns)
        self.cols = (Column * self.ncols)()
        for k, col in enumerate(columns):
            h, form, g = col[:3]
            self.cols[k].height, self.cols[k].gravity_form, self.cols[k].g = int(h), int(form), float(g)
            self.cols[k].rho_v = float(col[3]) if len(col) > 3 else 0.0
        self.heights = np.array([c[0] for c in columns], dtype=np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.heights)])
        nb = ctypes.c_size_t()
        _bcheck(lib.tplbm_batch_workspace_bytes(ctypes.byref(p), self.ncols, self.cols,
                                                ctypes.byref(nb)))
        self.device = _device(device)
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = _VP()
        _bcheck(lib.tplbm_batch_create(ctypes.byref(p), self.ncols, self.cols,
                                       self.workspace.data_ptr(), int(nb.value),
                                       self.stream.cuda_stream, ctypes.byref(h)))
        self._h = h

    def set_state(self, rho_concat, T_concat):
        r = np.ascontiguousarray(rho_concat, dtype=np.float64)
        t = np.ascontiguousarray(T_concat, dtype=np.float64)
        if r.size != self.offsets[-1] or t.size != self.offsets[-1]:
            raise ValueError("concatenated arrays must hold sum(heights) values")
        _bcheck(load_library().tplbm_batch_set_state(self._h, _dp(r), _dp(t)), self._h)

    def run(self, tol: float, max_steps: int) -> dict:
        res = (ColResult * self.ncols)()
        _bcheck(load_library().tplbm_batch_run(self._h, float(tol), int(max_steps), res), self._h)
        return dict(steps=np.array([r.steps for r in res]),
                    status=np.array([r.status for r in res]),
                    mass=np.array([r.mass for r in res]),
                    max_u=np.array([r.max_u for r in res]))

    def read(self, field: str) -> np.ndarray:
        out = np.empty(int(self.offsets[-1]))
        _bcheck(load_library().tplbm_batch_read(self._h, FIELDS[field], _dp(out)), self._h)
        return out

    def resume(self, T_bot=None, T_top=None):
        """Make the next run continue from where the last one ended, with new
        wall temperatures (per-column sequences; None keeps those walls)."""
        def arr(v):
            if v is None:
                return None
            a = np.ascontiguousarray(v, dtype=np.float64)
            if a.size != self.ncols:
                raise ValueError("one wall temperature per column")
            return a
        tb, tt = arr(T_bot), arr(T_top)
        _bcheck(load_library().tplbm_batch_resume(self._h, _dp(tb) if tb is not None else None,
                                                  _dp(tt) if tt is not None else None), self._h)

    def column(self, arr, k):
        return arr[self.offsets[k]:self.offsets[k + 1]]

    def autotune(self, budget_ms: float = 2000.0) -> dict:
        t = BatchTuning()
        _bcheck(load_library().tplbm_batch_autotune(self._h, float(budget_ms), ctypes.byref(t)),
                self._h)
        return dict(shape=t.shape, threads=t.threads, nodes_per_thread=t.nodes_per_thread,
                    check_every=t.check_every, grid=t.grid, node_steps_per_s=t.node_steps_per_s)

    def set_tuning(self, shape: int = -1, check_every: int = 0):
        _bcheck(load_library().tplbm_batch_set_tuning(self._h, int(shape), int(check_every)),
                self._h)

    def close(self):
        if getattr(self, "_h", None):
            load_library().tplbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_params(eos="cs", **over) -> BatchParams:
    d = dict(PAPER)
    d.update(over)
    p = BatchParams()
    p.a, p.b, p.R, p.G, p.sigma = d["a"], d["b"], d["R"], d["G"], d["sigma"]
    p.cv, p.kappa = d["cv"], d["kappa"]
    p.eos = {"cs": 0, "ideal": 1}[eos]
    return p


def batch_run_noalloc(columns, rho0, T0, rho_out, T_out, results, tol: float, max_steps: int,
                      check_every: int, params: BatchParams = None, stream=None):
    """tplbm_batch_run_noalloc on caller tensors: rho0, T0, rho_out, T_out
    are contiguous float64 device tensors of sum(heights) values; results a
    contiguous device tensor of 32 * ncols bytes (one tplbm_col_result per
    column, readable with ``col_results``).  columns as for Batch."""
    import torch

    n = len(columns)
    cols = (Column * n)()
    for k, col in enumerate(columns):
        h, form, g = col[:3]
        cols[k].height, cols[k].gravity_form, cols[k].g = int(h), int(form), float(g)
        cols[k].rho_v = float(col[3]) if len(col) > 3 else 0.0
    total = int(sum(int(c[0]) for c in columns))
    dev = rho0.device
    for t in (rho0, T0, rho_out, T_out):
        if t.device != dev or t.dtype != torch.float64 or t.numel() != total or not t.is_contiguous():
            raise ValueError(f"density and temperature tensors must be contiguous float64 on {dev} "
                             f"with {total} values")
    if results.device != dev or results.numel() * results.element_size() != 32 * n \
            or not results.is_contiguous():
        raise ValueError(f"results must be a contiguous tensor of {32 * n} bytes on {dev}")
    p = params or batch_params()
    s = stream or torch.cuda.current_stream(dev)
    _bcheck(load_library().tplbm_batch_run_noalloc(
        ctypes.byref(p), n, cols, rho0.data_ptr(), T0.data_ptr(), rho_out.data_ptr(),
        T_out.data_ptr(), results.data_ptr(), float(tol), int(max_steps), int(check_every),
        s.cuda_stream))


def col_results(results) -> dict:
    """Decode a device or host buffer of tplbm_col_result records."""
    raw = results.cpu().numpy().view(np.uint8).tobytes() if hasattr(results, "cpu") else bytes(results)
    rec = np.frombuffer(raw, dtype=np.dtype([("steps", "<i8"), ("status", "<i4"), ("pad", "<i4"),
                                             ("mass", "<f8"), ("max_u", "<f8")]))
    return dict(steps=rec["steps"].copy(), status=rec["status"].copy(), mass=rec["mass"].copy(),
                max_u=rec["max_u"].copy())


# ---- learned warm start ------------------------------------------------------

class NetColumn(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("gravity_form", ctypes.c_int32),
                ("t_reduced", ctypes.c_double), ("g", ctypes.c_double),
                ("mean_reduced", ctypes.c_double), ("lever_height", ctypes.c_double)]


class NetConfig(ctypes.Structure):
    _fields_ = [("rho_c", ctypes.c_double), ("T_c", ctypes.c_double),
                ("max_cols", ctypes.c_int32), ("dataset_cols", ctypes.c_int32),
                ("max_nodes", ctypes.c_int64), ("dataset_nodes", ctypes.c_int64)]


_NCP = ctypes.POINTER(NetColumn)
_FP = ctypes.POINTER(ctypes.c_float)
_IP = ctypes.POINTER(ctypes.c_int32)
_U16P = ctypes.POINTER(ctypes.c_uint16)
SIGNATURES.update({
    "tplbm_net_num_params": ([ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "tplbm_net_workspace_bytes": ([ctypes.POINTER(NetConfig), _SZ], ctypes.c_int),
    "tplbm_net_create": ([ctypes.POINTER(NetConfig), _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)],
                         ctypes.c_int),
    "tplbm_net_set_params": ([_VP, _FP], ctypes.c_int),
    "tplbm_net_get_params": ([_VP, _FP], ctypes.c_int),
    "tplbm_net_set_dataset": ([_VP, ctypes.c_int32, _NCP, _DP, _DP], ctypes.c_int),
    "tplbm_net_loss_grad": ([_VP, ctypes.c_int32, _IP, _DP, _FP], ctypes.c_int),
    "tplbm_net_train_step": ([_VP, ctypes.c_int32, _IP, ctypes.c_float, _DP], ctypes.c_int),
    "tplbm_net_forward": ([_VP, ctypes.c_int32, _NCP, _FP], ctypes.c_int),
    "tplbm_net_predict": ([_VP, ctypes.c_int32, _NCP, _DP, _DP], ctypes.c_int),
    "tplbm_net_predict_device": ([_VP, ctypes.c_int32, _NCP, _VP, _VP], ctypes.c_int),
    "tplbm_net_init": ([_VP, ctypes.c_uint64], ctypes.c_int),
    "tplbm_net_mfma_check": ([_VP, _U16P, _U16P, _FP], ctypes.c_int),
    "tplbm_net_destroy": ([_VP], None),
    "tplbm_net_last_error": ([_VP], ctypes.c_char_p),
})


def _ncheck(rc: int, h=None):
    if rc != OK:
        raise TplbmError(rc, load_library().tplbm_net_last_error(h).decode())


def _fp(a):
    return a.ctypes.data_as(_FP)


def net_columns(columns):
    """ctypes array of network column descriptions from (height, form,
    t_reduced, g, mean_reduced, lever_height) tuples."""
    arr = (NetColumn * len(columns))()
    for k, (h, form, t, g, m, hl) in enumerate(columns):
        arr[k].height, arr[k].gravity_form = int(h), int(form)
        arr[k].t_reduced, arr[k].g, arr[k].mean_reduced = float(t), float(g), float(m)
        arr[k].lever_height = float(hl)
    return arr


def net_num_params() -> int:
    n = ctypes.c_int64()
    _ncheck(load_library().tplbm_net_num_params(ctypes.byref(n)))
    return int(n.value)


class Net:
    """The warm-start network on one GPU: parameters, Adam state, an optional
    device-resident training set and the buffers of one call of up to
    max_cols columns / max_nodes nodes."""

    def __init__(self, rho_c, T_c, max_cols, max_nodes, dataset_cols=0, dataset_nodes=0,
                 device=None, stream=None):
        import torch

        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the network kernels need an MI355X")
        c = NetConfig()
        c.rho_c, c.T_c = float(rho_c), float(T_c)
        c.max_cols, c.dataset_cols = int(max_cols), int(dataset_cols)
        c.max_nodes, c.dataset_nodes = int(max_nodes), int(dataset_nodes)
        self.config = c
        self.n_params = net_num_params()
        nb = ctypes.c_size_t()
        _ncheck(lib.tplbm_net_workspace_bytes(ctypes.byref(c), ctypes.byref(nb)))
        self.device = _device(device)
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = _VP()
        _ncheck(lib.tplbm_net_create(ctypes.byref(c), self.workspace.data_ptr(), int(nb.value),
                                     self.stream.cuda_stream, ctypes.byref(h)))
        self._h = h
        self.data_heights = None

    def set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        if t.size != self.n_params:
            raise ValueError(f"need {self.n_params} parameters")
        _ncheck(load_library().tplbm_net_set_params(self._h, _fp(t)), self._h)

    def init(self, seed: int):
        """He-uniform initialisation from the seeded SplitMix64 stream (C side)."""
        _ncheck(load_library().tplbm_net_init(self._h, int(seed) % (1 << 64)), self._h)

    def get_params(self) -> np.ndarray:
        t = np.empty(self.n_params, dtype=np.float32)
        _ncheck(load_library().tplbm_net_get_params(self._h, _fp(t)), self._h)
        return t

    def set_dataset(self, columns, rho_concat, T_concat):
        cols = net_columns(columns)
        r = np.ascontiguousarray(rho_concat, dtype=np.float64)
        t = np.ascontiguousarray(T_concat, dtype=np.float64)
        n = sum(int(c[0]) for c in columns)
        if r.size != n or t.size != n:
            raise ValueError("concatenated profiles must hold sum(heights) values")
        _ncheck(load_library().tplbm_net_set_dataset(self._h, len(columns), cols, _dp(r), _dp(t)),
                self._h)
        self.data_heights = np.array([int(c[0]) for c in columns])

    def loss_grad(self, idx):
        i = np.ascontiguousarray(idx, dtype=np.int32)
        loss = ctypes.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        _ncheck(load_library().tplbm_net_loss_grad(self._h, i.size, i.ctypes.data_as(_IP),
                                                   ctypes.byref(loss), _fp(g)), self._h)
        return float(loss.value), g

    def train_step(self, idx, lr: float, want_loss: bool = True):
        i = np.ascontiguousarray(idx, dtype=np.int32)
        loss = ctypes.c_double()
        _ncheck(load_library().tplbm_net_train_step(self._h, i.size, i.ctypes.data_as(_IP),
                                                    float(lr),
                                                    ctypes.byref(loss) if want_loss else None),
                self._h)
        return float(loss.value) if want_loss else None

    def forward(self, columns) -> np.ndarray:
        cols = net_columns(columns)
        n = sum(int(c[0]) for c in columns)
        out = np.empty(2 * n, dtype=np.float32)
        _ncheck(load_library().tplbm_net_forward(self._h, len(columns), cols, _fp(out)), self._h)
        return out.reshape(n, 2)

    def predict(self, columns):
        cols = net_columns(columns)
        n = sum(int(c[0]) for c in columns)
        rho, T = np.empty(n), np.empty(n)
        _ncheck(load_library().tplbm_net_predict(self._h, len(columns), cols, _dp(rho), _dp(T)),
                self._h)
        return rho, T

    def predict_device(self, columns, rho_out, T_out):
        """Profiles into float64 device tensors of sum(heights) values each,
        enqueued on the network's stream."""
        import torch

        cols = net_columns(columns)
        n = sum(int(c[0]) for c in columns)
        for t in (rho_out, T_out):
            if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != torch.float64 \
                    or t.numel() != n or not t.is_contiguous():
                raise ValueError(f"outputs must be contiguous float64 tensors of {n} values on {self.device}")
        _ncheck(load_library().tplbm_net_predict_device(self._h, len(columns), cols, rho_out.data_ptr(),
                                                        T_out.data_ptr()), self._h)

    def mfma_check(self, a, b) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint16)
        b = np.ascontiguousarray(b, dtype=np.uint16)
        if a.size != 512 or b.size != 512:
            raise ValueError("a and b hold 64 lanes x 8 bf16 values")
        d = np.empty(1024, dtype=np.float32)
        _ncheck(load_library().tplbm_net_mfma_check(self._h, a.ctypes.data_as(_U16P),
                                                    b.ctypes.data_as(_U16P), _fp(d)), self._h)
        return d.reshape(64, 16)

    def close(self):
        if getattr(self, "_h", None):
            load_library().tplbm_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
