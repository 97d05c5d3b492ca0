"""FP64 CPU oracle of the thermal pseudopotential LBM update (arXiv 2301.12869).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The product library never imports,
links or executes anything in this directory, and this directory never imports
the product.  The C source ``tplbm_oracle.c`` holds the arithmetic; this module
only marshals arguments through ctypes and builds the shared object with gcc.

Every function cites the passage of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tplbm_oracle.c")
_LIB = os.path.join(_HERE, "liborc_tplbm.so")

LATTICE = {"D1Q3": 1, "D2Q9": 2, "D3Q19": 3}
STATUS = {0: "converged", 1: "diverged", 2: "max_steps"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no contraction, no fast-math."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("walls", ctypes.c_int32), ("eos", ctypes.c_int32),
        ("gravity_form", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
        ("G", ctypes.c_double), ("sigma", ctypes.c_double), ("tau", ctypes.c_double * 6),
        ("cv", ctypes.c_double), ("kappa", ctypes.c_double), ("g", ctypes.c_double),
        ("rho_v", ctypes.c_double),
    ]


class Diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("mean_rho", ctypes.c_double),
                ("max_u", ctypes.c_double), ("min_rho", ctypes.c_double),
                ("flags", ctypes.c_double)]


_lib = None


def _bind(L):
    """Declare the argument and result types of the exported functions."""
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(Params)
    for name, args in {
        "orc_eos_p": [pp, ctypes.c_double, ctypes.c_double],
        "orc_eos_dpdT": [pp, ctypes.c_double, ctypes.c_double],
        "orc_eos_dpdrho": [pp, ctypes.c_double, ctypes.c_double],
        "orc_eos_d2pdrho2": [pp, ctypes.c_double, ctypes.c_double],
    }.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_double
    L.orc_critical.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    L.orc_spinodal.argtypes = [pp, ctypes.c_double, dp]
    L.orc_coexistence.argtypes = [pp, ctypes.c_double, dp]
    L.orc_init_rest.argtypes = [pp, dp, dp]
    L.orc_step.argtypes = [pp, dp, dp, ctypes.c_int64, ctypes.POINTER(Diag)]
    L.orc_run_to_steady.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_int64,
                                    ctypes.c_int64, dp]
    L.orc_macro.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp]
    L.orc_collide.argtypes = [pp, dp, dp, dp]
    L.orc_d2q9_minv.argtypes = [dp]
    L.orc_d3q19_velocities.argtypes = [ctypes.POINTER(ctypes.c_int), dp]
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = ctypes.c_int
    for fn in ("orc_critical", "orc_spinodal", "orc_coexistence", "orc_init_rest",
               "orc_step", "orc_run_to_steady", "orc_macro", "orc_collide"):
        getattr(L, fn).restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def load_build(path: str):
    """Load another build of the oracle source (the tests plant mistakes in a
    copy of it to check that the pins catch them).  Returns the bound library;
    assign it to ``oracle._lib`` to route every call here through it."""
    return _bind(ctypes.CDLL(os.path.abspath(path)))


def set_threads(n: int) -> int:
    """Run the D2Q9 and D3Q19 node loops on n threads (1: the plain serial
    definition, the default).  Results are bit for bit the same for any n.
    Returns the previous setting."""
    return int(lib().orc_set_threads(int(n)))


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
PAPER_PARAMS = dict(a=0.5, b=4.0, R=1.0, G=-1.0, sigma=1.385, tau=(1.0,) * 6,
                    cv=5.0, kappa=0.02)


def make_params(lattice="D2Q9", nx=1, ny=1, nz=1, walls=True, eos="cs", gravity_form=1,
                g=0.0, rho_v=0.0, **over) -> Params:
    d = dict(PAPER_PARAMS)
    d.update(over)
    p = Params()
    p.lattice = LATTICE[lattice]
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.walls = 1 if walls else 0
    p.eos = {"cs": 0, "ideal": 1}[eos]
    p.gravity_form = int(gravity_form)
    p.a, p.b, p.R, p.G, p.sigma = d["a"], d["b"], d["R"], d["G"], d["sigma"]
    for k in range(6):
        p.tau[k] = float(d["tau"][k])
    p.cv, p.kappa, p.g = d["cv"], d["kappa"], float(g)
    p.rho_v = float(rho_v)
    return p


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def nq(p: Params) -> int:
    return {1: 3, 2: 9, 3: 19}[p.lattice]


def nnodes(p: Params) -> int:
    if p.lattice == 1:
        return p.ny
    if p.lattice == 2:
        return p.nx * p.ny
    return p.nx * p.ny * p.nz


# ---------------------------------------------------------------------------
# equation of state utilities
# ---------------------------------------------------------------------------
def eos_p(p: Params, rho: float, T: float) -> float:
    return lib().orc_eos_p(ctypes.byref(p), rho, T)


def eos_dpdT(p: Params, rho: float, T: float) -> float:
    return lib().orc_eos_dpdT(ctypes.byref(p), rho, T)


def eos_dpdrho(p: Params, rho: float, T: float) -> float:
    return lib().orc_eos_dpdrho(ctypes.byref(p), rho, T)


def eos_d2pdrho2(p: Params, rho: float, T: float) -> float:
    return lib().orc_eos_d2pdrho2(ctypes.byref(p), rho, T)


def critical(a=0.5, b=4.0, R=1.0):
    out = np.zeros(3)
    _check(lib().orc_critical(a, b, R, _dp(out)), "critical")
    return tuple(out)  # rho_c, T_c, p_c


def spinodal(p: Params, T: float):
    out = np.zeros(2)
    _check(lib().orc_spinodal(ctypes.byref(p), T, _dp(out)), "spinodal")
    return tuple(out)


def coexistence(p: Params, T: float):
    out = np.zeros(3)
    _check(lib().orc_coexistence(ctypes.byref(p), T, _dp(out)), "coexistence")
    return tuple(out)  # rho_v, rho_l, p_sat


# ---------------------------------------------------------------------------
# lattice runs
# ---------------------------------------------------------------------------
def init_rest(p: Params, rho0: np.ndarray) -> np.ndarray:
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64).ravel()
    assert rho0.size == nnodes(p)
    f = np.zeros(nq(p) * nnodes(p))
    _check(lib().orc_init_rest(ctypes.byref(p), _dp(rho0), _dp(f)), "init_rest")
    return f


def step(p: Params, f: np.ndarray, T: np.ndarray, nsteps: int) -> dict:
    """Advance f, T in place by nsteps; returns the last step's diagnostics."""
    d = Diag()
    _check(lib().orc_step(ctypes.byref(p), _dp(f), _dp(T), int(nsteps), ctypes.byref(d)),
           "step")
    return dict(mass=d.mass, mean_rho=d.mean_rho, max_u=d.max_u, min_rho=d.min_rho,
                flags=int(d.flags))


def run_to_steady(p: Params, f, T, tol: float, check_every: int, max_steps: int):
    out = np.zeros(3)
    _check(lib().orc_run_to_steady(ctypes.byref(p), _dp(f), _dp(T), tol, int(check_every),
                                   int(max_steps), _dp(out)), "run_to_steady")
    return int(out[0]), STATUS[int(out[1])]


def macro(p: Params, f: np.ndarray, T: np.ndarray) -> dict:
    N = nnodes(p)
    outs = {k: np.zeros(N) for k in ("rho", "ux", "uy", "uz", "p_eos", "p_nn")}
    _check(lib().orc_macro(ctypes.byref(p), _dp(f), _dp(T), *[_dp(outs[k]) for k in
                           ("rho", "ux", "uy", "uz", "p_eos", "p_nn")]), "macro")
    outs["T"] = T.copy()
    return outs


def collide(p: Params, f: np.ndarray, T: np.ndarray) -> np.ndarray:
    fs = np.zeros_like(f)
    _check(lib().orc_collide(ctypes.byref(p), _dp(f), _dp(T), _dp(fs)), "collide")
    return fs


def d2q9_minv() -> np.ndarray:
    out = np.zeros(81)
    lib().orc_d2q9_minv(_dp(out))
    return out.reshape(9, 9)


def d3q19_velocities():
    c = (ctypes.c_int * 57)()
    w = np.zeros(19)
    lib().orc_d3q19_velocities(c, _dp(w))
    return np.array(list(c)).reshape(19, 3), w
