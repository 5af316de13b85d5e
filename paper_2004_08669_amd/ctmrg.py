"""Python binding of the CTMRG library (libctmrg.so, C ABI in include/ctmrg.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  There is no fallback: if the library is missing or the device is
not a gfx950 GPU, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctmrg.so")

CTMRG_OK = 0
STATUS = {
    0: "CTMRG_OK",
    1: "CTMRG_E_INVALID_ARG",
    2: "CTMRG_E_OUT_OF_MEMORY",
    3: "CTMRG_E_HIP",
    4: "CTMRG_E_NOT_CONVERGED",
    5: "CTMRG_E_NUMERICAL",
    6: "CTMRG_E_STATE",
    7: "CTMRG_E_UNSUPPORTED",
}
BUF = {"P": 0, "omega": 1, "spectrum": 2, "U": 3, "cext": 4, "W": 5}
STAGES = ["extension", "wmix_C", "dense_to_band", "band_to_tridiag", "bisection", "select_cut_entropy",
          "inverse_iteration", "orthonormalize", "backtransform_band", "backtransform_dense", "halfrow",
          "wmix_Z", "projection", "normalize", "step", "warm_topk"]
EIG_SOLVERS = {"two_stage": 0, "warm": 1}
WARM_TAILS = {"exact": 0, "bound": 1, "auto": 2}


class CTMRGError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("bc", ctypes.c_int),
        ("boundary_spin", ctypes.c_int),
        ("band", ctypes.c_int),
        ("gap_tol", ctypes.c_double),
        ("rank_tol", ctypes.c_double),
        ("hip_stream", ctypes.c_void_p),
        ("eig_solver", ctypes.c_int),
        ("warm_guard", ctypes.c_int),
        ("warm_degree", ctypes.c_int),
        ("warm_tol", ctypes.c_double),
        ("warm_tail", ctypes.c_int),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class Observables(ctypes.Structure):
    _fields_ = [
        ("f", ctypes.c_double),
        ("E", ctypes.c_double),
        ("M", ctypes.c_double),
        ("S_E", ctypes.c_double),
        ("ln_kappa_W", ctypes.c_double),
        ("ln_kappa_ratio", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("c_paper", ctypes.c_double),
        ("m_eff", ctypes.c_int),
        ("steps", ctypes.c_int),
        ("xi_e", ctypes.c_double),
        ("tm_lambda1", ctypes.c_double),
        ("tm_lambda2", ctypes.c_double),
        ("tm_residual", ctypes.c_double),
        ("tm_iterations", ctypes.c_int),
        ("tm_converged", ctypes.c_int),
    ]


class Derivative(ctypes.Structure):
    _fields_ = [
        ("F", ctypes.c_double),
        ("dF_dK", ctypes.c_double),
        ("d2F_dK2", ctypes.c_double),
        ("gauge_residual", ctypes.c_double),
        ("tangent_change", ctypes.c_double),
        ("aligned_steps", ctypes.c_int),
        ("iterations", ctypes.c_int),
        ("n_eigen", ctypes.c_int),
        ("E", ctypes.c_double),
        ("M", ctypes.c_double),
        ("dE_dK", ctypes.c_double),
        ("dM_dK", ctypes.c_double),
        ("status", ctypes.c_int),
    ]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def library_path() -> str:
    return LIB_PATH


def load():
    """Load libctmrg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2004_08669_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "ctmrg_default_options": ([ctypes.POINTER(Options)], ctypes.c_int),
        "ctmrg_init": ([ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Options),
                        ctypes.POINTER(_vp)], ctypes.c_int),
        "ctmrg_set_K": ([_vp, ctypes.c_double], ctypes.c_int),
        "ctmrg_step": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
        "ctmrg_run_to_fixed_point": ([_vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp],
                                     ctypes.c_int),
        "ctmrg_observables": ([_vp, ctypes.POINTER(Observables), _dp], ctypes.c_int),
        "ctmrg_sweep": ([_vp, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                         ctypes.POINTER(Observables), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(Derivative)],
                        ctypes.c_int),
        "ctmrg_backward": ([_vp, _dp, _dp, _dp], ctypes.c_int),
        "ctmrg_fixed_point_derivative": ([_vp, ctypes.c_int, ctypes.POINTER(Derivative)], ctypes.c_int),
        "ctmrg_export_state": ([_vp, _vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ctmrg_import_state": ([_vp, _vp, ctypes.c_size_t], ctypes.c_int),
        "ctmrg_set_state": ([_vp, ctypes.c_int, _dp, _dp], ctypes.c_int),
        "ctmrg_workspace_size": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(Options),
                                  ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ctmrg_extra_workspace_size": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(Options),
                                        ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ctmrg_get_buffer": ([_vp, ctypes.c_int, _dp, ctypes.c_size_t], ctypes.c_int),
        "ctmrg_extend": ([_vp], ctypes.c_int),
        "ctmrg_eigh_topk": ([ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp], ctypes.c_int),
        "ctmrg_eigh_topk_noalloc": ([ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp], ctypes.c_int),
        "ctmrg_set_profiling": ([_vp, ctypes.c_int], ctypes.c_int),
        "ctmrg_get_stage_times": ([_vp, _dp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "ctmrg_get_eig_stats": ([_vp, _dp], ctypes.c_int),
        "ctmrg_last_error": ([_vp], ctypes.c_char_p),
        "ctmrg_destroy": ([_vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def default_options() -> Options:
    o = Options()
    load().ctmrg_default_options(ctypes.byref(o))
    return o


# ctmrg_precision: contractions in FP64, FP32, or FP32 operands as three split-bf16 products
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
GAP_TOL = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-4}


def workspace_size(q: int, m: int, band: int = 16, precision: str = "fp64", eig: str = "two_stage") -> int:
    """Device bytes a context allocates at init (what a caller-owned workspace needs)."""
    o = default_options()
    o.band = band
    o.precision = PRECISIONS[precision]
    o.eig_solver = EIG_SOLVERS[eig]
    n = ctypes.c_size_t(0)
    st = load().ctmrg_workspace_size(q, m, ctypes.byref(o), ctypes.byref(n))
    if st != CTMRG_OK:
        raise CTMRGError(st)
    return int(n.value)


def extra_workspace_size(q: int, m: int, band: int = 16):
    """Device bytes allocated on first use: (by ctmrg_observables, by the fixed-point derivative)."""
    o = default_options()
    o.band = band
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    st = load().ctmrg_extra_workspace_size(q, m, ctypes.byref(o), ctypes.byref(a), ctypes.byref(b))
    if st != CTMRG_OK:
        raise CTMRGError(st)
    return int(a.value), int(b.value)


def eigh_topk(A: np.ndarray, k: int, band: int = 0):
    """All eigenvalues (ascending) and the k eigenpairs of largest |lambda| of a symmetric matrix."""
    A = _f64(A)
    n = A.shape[0]
    ev = np.empty(n)
    kept = np.empty(k)
    vec = np.empty((n, k))
    st = load().ctmrg_eigh_topk(n, _p(A), k, band, _p(ev), _p(kept), _p(vec))
    if st != CTMRG_OK:
        raise CTMRGError(st, "ctmrg_eigh_topk")
    return ev, kept, vec


def eigh_topk_noalloc(A: np.ndarray, k: int, band: int = 0):
    """ctmrg_eigh_topk_noalloc: the same outputs as eigh_topk, computed without device allocation."""
    A = _f64(A)
    n = A.shape[0]
    ev = np.empty(n)
    kept = np.empty(k)
    vec = np.empty((n, k))
    st = load().ctmrg_eigh_topk_noalloc(n, _p(A), k, band, _p(ev), _p(kept), _p(vec))
    if st != CTMRG_OK:
        raise CTMRGError(st, "ctmrg_eigh_topk_noalloc")
    return ev, kept, vec


class CTMRG:
    """A CTMRG context on the current GPU (see include/ctmrg.h)."""

    def __init__(self, V, K: float, m: int, bc: str = "fixed", boundary_spin: int = 0, band: int = 16,
                 gap_tol: float | None = None, rank_tol: float = 1e-13, precision: str = "fp64", stream=None,
                 eig: str = "two_stage", warm_guard: int = 0, warm_degree: int = 0, warm_tol: float = 0.0,
                 warm_tail: str = "auto", workspace=None):
        lib = load()
        self._lib = lib
        self.V = _f64(V)
        self.q, self.dim = self.V.shape
        self.m = int(m)
        self.N = self.q * self.m
        o = default_options()
        o.bc = {"fixed": 0, "free": 1}[bc]
        o.boundary_spin = boundary_spin
        o.band = band
        # multiplets of C' are split by the contraction rounding: ~1e-16 (FP64), ~1e-7 (FP32),
        # ~1e-5 (split-bf16 products)
        o.gap_tol = gap_tol if gap_tol is not None else GAP_TOL[precision]
        o.rank_tol = rank_tol
        o.precision = PRECISIONS[precision]
        o.hip_stream = stream
        o.eig_solver = EIG_SOLVERS[eig]
        o.warm_guard = warm_guard
        o.warm_degree = warm_degree
        o.warm_tol = warm_tol
        o.warm_tail = WARM_TAILS[warm_tail]
        # workspace: a device tensor (or any object with data_ptr() and nbytes) the caller keeps alive
        self._workspace = workspace
        if workspace is not None:
            o.workspace = ctypes.c_void_p(int(workspace.data_ptr()))
            o.workspace_bytes = int(workspace.nbytes)
        h = _vp()
        st = lib.ctmrg_init(self.q, self.dim, _p(self.V), float(K), self.m, ctypes.byref(o), ctypes.byref(h))
        self._h = h
        if st != CTMRG_OK:
            msg = lib.ctmrg_last_error(h).decode() if h.value else ""
            if h.value:
                lib.ctmrg_destroy(h)
            self._h = _vp()
            raise CTMRGError(st, msg)

    def _check(self, st):
        if st != CTMRG_OK:
            raise CTMRGError(st, self._lib.ctmrg_last_error(self._h).decode())

    def close(self):
        if self._h and self._h.value:
            self._lib.ctmrg_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_K(self, K: float):
        self._check(self._lib.ctmrg_set_K(self._h, float(K)))

    def step(self, n: int = 1) -> float:
        d = ctypes.c_double(0.0)
        self._check(self._lib.ctmrg_step(self._h, n, ctypes.byref(d)))
        return d.value

    def run_to_fixed_point(self, tol: float, max_steps: int):
        k = ctypes.c_int(0)
        d = ctypes.c_double(0.0)
        st = self._lib.ctmrg_run_to_fixed_point(self._h, tol, max_steps, ctypes.byref(k), ctypes.byref(d))
        if st not in (CTMRG_OK, 4):
            self._check(st)
        return k.value, d.value, st == CTMRG_OK

    def observables(self) -> dict:
        o = Observables()
        spec = np.empty(self.m)
        self._check(self._lib.ctmrg_observables(self._h, ctypes.byref(o), _p(spec)))
        out = {name: getattr(o, name) for name, _ in Observables._fields_}
        out["kept_spectrum"] = spec
        return out

    def sweep(self, T, tol: float, max_steps: int, warm_start: bool = True, derivative: bool = False) -> list:
        """ctmrg_sweep over the temperatures T (one dict of observables per temperature, with
        "T", "steps" and "converged" added, and with derivative=True the fixed-point derivative
        of each converged temperature under "derivative")."""
        Ts = _f64(np.atleast_1d(T))
        n = int(Ts.size)
        obs = (Observables * max(n, 1))()
        steps = (ctypes.c_int * max(n, 1))()
        conv = (ctypes.c_int * max(n, 1))()
        der = (Derivative * max(n, 1))() if derivative else None
        self._check(self._lib.ctmrg_sweep(self._h, n, _p(Ts), float(tol), int(max_steps), 1 if warm_start else 0,
                                          obs, steps, conv, der))
        out = []
        for i in range(n):
            d = {name: getattr(obs[i], name) for name, _ in Observables._fields_}
            d.update({"T": float(Ts[i]), "steps": int(steps[i]), "converged": bool(conv[i])})
            if derivative:
                d["derivative"] = {name: getattr(der[i], name) for name, _ in Derivative._fields_}
            out.append(d)
        return out

    def fixed_point_derivative(self, second_order=False) -> dict:
        """dF/dK, dE/dK and dM/dK at the converged fixed point, and d2F/dK2 with second_order
        (True or 1: dE/dK; 2: the central difference of dF/dK; see include/ctmrg.h)."""
        d = Derivative()
        self._check(self._lib.ctmrg_fixed_point_derivative(self._h, int(second_order), ctypes.byref(d)))
        return {name: getattr(d, name) for name, _ in Derivative._fields_}

    def backward(self, obs_bar, want_d2: bool = False):
        """K_bar = obs_bar . d(f, E, M)/dK; also d2F/dK2 when requested."""
        ob = _f64(obs_bar)
        kb = ctypes.c_double(0.0)
        d2 = ctypes.c_double(0.0)
        self._check(self._lib.ctmrg_backward(self._h, _p(ob), ctypes.byref(kb),
                                             ctypes.byref(d2) if want_d2 else None))
        return kb.value, (d2.value if want_d2 else None)

    def export_state(self) -> bytes:
        n = ctypes.c_size_t(0)
        self._check(self._lib.ctmrg_export_state(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self._lib.ctmrg_export_state(self._h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def import_state(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        self._check(self._lib.ctmrg_import_state(self._h, buf, len(data)))

    def set_state(self, P: np.ndarray, omega: np.ndarray):
        P = _f64(P)
        omega = _f64(omega)
        d = P.shape[1]
        self._check(self._lib.ctmrg_set_state(self._h, d, _p(P), _p(omega)))

    def extend(self):
        self._check(self._lib.ctmrg_extend(self._h))

    def get(self, which: str) -> np.ndarray:
        shapes = {
            "P": (self.m, self.N),
            "omega": (self.m,),
            "spectrum": (self.N,),
            "U": (self.N, self.m),
            "cext": (self.N, self.N),
            "W": (self.q * self.q, self.q * self.q),
        }
        out = np.empty(shapes[which])
        self._check(self._lib.ctmrg_get_buffer(self._h, BUF[which], _p(out), out.size))
        return out

    def set_profiling(self, enable: bool = True):
        self._check(self._lib.ctmrg_set_profiling(self._h, 1 if enable else 0))

    def stage_times(self):
        """Accumulated device milliseconds per stage and the number of timed steps."""
        ms = np.zeros(len(STAGES))
        n = ctypes.c_int(0)
        self._check(self._lib.ctmrg_get_stage_times(self._h, _p(ms), ctypes.byref(n)))
        return dict(zip(STAGES, ms.tolist())), n.value

    def eig_stats(self) -> dict:
        """Counters of the warm eigensolver (see ctmrg_get_eig_stats)."""
        out = np.zeros(13)
        self._check(self._lib.ctmrg_get_eig_stats(self._h, _p(out)))
        return {"warm_steps": int(out[0]), "fallback_steps": int(out[1]), "passes": int(out[2]),
                "products": int(out[3]), "tail_bound_max": float(out[4]), "tail_bound_last": float(out[5]),
                "last_reason": int(out[6]), "last_residual": float(out[7]), "product_ms": float(out[8]),
                "product_flops": float(out[9]), "product_launches": int(out[10]), "last_step_S_E": float(out[11]),
                "exact_tails": int(out[12])}

    def P_slices(self) -> np.ndarray:
        """The current P as q slices P_s (m x m)."""
        A = self.get("P")
        return A.reshape(self.m, self.q, self.m).transpose(1, 0, 2).copy()
