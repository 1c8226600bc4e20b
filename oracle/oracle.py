"""ctypes marshalling for the C oracle in ``vfp_oracle.c``.

TEST INFRASTRUCTURE: see the package docstring.  Nothing here computes any
part of the method; each function forwards numpy arrays to the C routine of
the same name, which cites the passage of the paper it implements.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vfp_oracle.c")
_LIB = os.path.join(_HERE, "libvfp_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
            "-D_GNU_SOURCE", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


class _P(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("q_min", C.c_double), ("q_max", C.c_double),
        ("p_min", C.c_double), ("p_max", C.c_double),
        ("steps_per_period", C.c_int), ("beta", C.c_double), ("interp", C.c_int),
        ("clamp", C.c_int), ("renormalize", C.c_int), ("padding", C.c_int),
        ("z_scale", C.c_double), ("rotation", C.c_int),
    ]


@dataclasses.dataclass
class OracleParams:
    n: int
    q_min: float = -6.0
    q_max: float = 6.0
    p_min: float = -6.0
    p_max: float = 6.0
    steps_per_period: int = 500
    beta: float = 0.0
    interp: int = 4
    clamp: int = 0
    renormalize: int = 1
    padding: int = 2
    z_scale: float = 0.0
    rotation: int = 0          # 0 standard, 1 Manhattan

    @classmethod
    def from_recipe(cls, s) -> "OracleParams":
        """From any object with the recipe attributes (n, ranges, steps, ...)."""
        return cls(n=s.n, q_min=s.q_min, q_max=s.q_max, p_min=s.p_min, p_max=s.p_max,
                   steps_per_period=s.steps_per_period, beta=s.beta, interp=s.interp,
                   clamp=s.clamp, renormalize=s.renormalize, padding=s.padding,
                   z_scale=s.z_scale, rotation=s.rotation)

    def c(self) -> _P:
        return _P(self.n, self.q_min, self.q_max, self.p_min, self.p_max,
                  self.steps_per_period, self.beta, self.interp, self.clamp,
                  self.renormalize, self.padding, self.z_scale, self.rotation)


_lib = None
_dp = C.POINTER(C.c_double)


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER(_P)
        lib.vfo_threads.restype = C.c_int
        lib.vfo_set_threads.argtypes = [C.c_int]
        lib.vfo_lagrange_weights.argtypes = [C.c_int, C.c_double, _dp]
        lib.vfo_profile.argtypes = [P, _dp, _dp]
        lib.vfo_charge.argtypes = [P, _dp]
        lib.vfo_charge.restype = C.c_double
        lib.vfo_wake_kernel.argtypes = [C.c_int, _dp, _dp, _dp]
        lib.vfo_wake.argtypes = [P, _dp, _dp, _dp]
        lib.vfo_rotate.argtypes = [P, _dp, _dp]
        lib.vfo_rotate_manhattan.argtypes = [P, _dp, _dp, _dp]
        lib.vfo_kick.argtypes = [P, _dp, _dp, _dp]
        lib.vfo_fokker_planck.argtypes = [P, _dp, _dp]
        lib.vfo_moments.argtypes = [P, _dp, _dp]
        lib.vfo_csr_power.argtypes = [P, _dp, _dp, _dp, _dp]
        lib.vfo_csr_power.restype = C.c_double
        lib.vfo_csr_spectrum.argtypes = [P, _dp, _dp, _dp, _dp]
        lib.vfo_haissinski.argtypes = [P, _dp, C.c_int, C.c_double, C.c_double, _dp]
        lib.vfo_step.argtypes = [P, _dp, _dp, C.c_double, _dp]
        lib.vfo_run.argtypes = [P, _dp, _dp, C.c_long, C.c_double, C.c_int, _dp, C.c_long]
        lib.vfo_run.restype = C.c_long
        lib.vfo_run_many.argtypes = [C.c_int, P, C.POINTER(_dp), C.POINTER(_dp),
                                     C.POINTER(C.c_long), _dp]
        _ip = C.POINTER(C.c_longlong)
        lib.vfo_fix_quantize.argtypes = [C.c_int, _dp, _ip, C.c_long]
        lib.vfo_fix_charge.argtypes = [P, C.c_int, _ip]
        lib.vfo_fix_charge.restype = C.c_double
        lib.vfo_fix_step.argtypes = [P, C.c_int, _dp, _ip, C.c_double, _dp, _ip, _dp]
        lib.vfo_fix_run.argtypes = [P, C.c_int, _dp, _ip, C.c_long, C.c_double, _dp]
        lib.vfo_fix_run.restype = C.c_int
        _lib = lib
    return _lib


def _a(x, n=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if n is not None and x.size != n:
        raise ValueError(f"expected {n} values, got {x.size}")
    return x


def _ptr(x):
    return None if x is None else x.ctypes.data_as(_dp)


def threads() -> int:
    return int(load().vfo_threads())


def set_threads(t: int) -> None:
    """Thread count of the oracle's OpenMP loops (for 1-core vs all-core timing)."""
    load().vfo_set_threads(int(t))


def lagrange_weights(K: int, t: float) -> np.ndarray:
    out = np.zeros(4)
    load().vfo_lagrange_weights(K, float(t), _ptr(out))
    return out[:K]


def wake_kernel(z_re, z_im, M: int = None) -> np.ndarray:
    """w[0..M-1] from the floor(M/2)+1 impedance samples (M even by default)."""
    z_re, z_im = _a(z_re), _a(z_im)
    if M is None:
        M = 2 * (z_re.size - 1)
    if z_re.size != M // 2 + 1 or z_im.size != M // 2 + 1:
        raise ValueError("need floor(M/2)+1 impedance samples")
    w = np.zeros(M)
    load().vfo_wake_kernel(M, _ptr(z_re), _ptr(z_im), _ptr(w))
    return w


def profile(p: OracleParams, psi) -> np.ndarray:
    psi = _a(psi, p.n * p.n)
    rho = np.zeros(p.n)
    load().vfo_profile(C.byref(p.c()), _ptr(psi), _ptr(rho))
    return rho


def charge(p: OracleParams, psi) -> float:
    return load().vfo_charge(C.byref(p.c()), _ptr(_a(psi, p.n * p.n)))


def wake(p: OracleParams, w, rho) -> np.ndarray:
    V = np.zeros(p.n)
    load().vfo_wake(C.byref(p.c()), _ptr(_a(w, p.padding * p.n)), _ptr(_a(rho, p.n)), _ptr(V))
    return V


def _map(fn, p, psi, *extra):
    src = _a(psi, p.n * p.n)
    dst = np.zeros_like(src)
    fn(C.byref(p.c()), *extra, _ptr(src), _ptr(dst))
    return dst.reshape(p.n, p.n)


def rotate(p: OracleParams, psi) -> np.ndarray:
    return _map(load().vfo_rotate, p, psi)


def rotate_manhattan(p: OracleParams, psi) -> np.ndarray:
    src = _a(psi, p.n * p.n)
    dst, tmp = np.zeros_like(src), np.zeros_like(src)
    load().vfo_rotate_manhattan(C.byref(p.c()), _ptr(src), _ptr(dst), _ptr(tmp))
    return dst.reshape(p.n, p.n)


def kick(p: OracleParams, V, psi) -> np.ndarray:
    return _map(load().vfo_kick, p, psi, _ptr(_a(V, p.n)))


def fokker_planck(p: OracleParams, psi) -> np.ndarray:
    return _map(load().vfo_fokker_planck, p, psi)


def moments(p: OracleParams, psi) -> np.ndarray:
    out = np.zeros(5)
    load().vfo_moments(C.byref(p.c()), _ptr(_a(psi, p.n * p.n)), _ptr(out))
    return out


def csr_power(p: OracleParams, w, psi) -> float:
    rho, V = np.zeros(p.n), np.zeros(p.n)
    return load().vfo_csr_power(C.byref(p.c()), _ptr(_a(w, p.padding * p.n)),
                                _ptr(_a(psi, p.n * p.n)), _ptr(rho), _ptr(V))


def csr_spectrum(p: OracleParams, z_re, psi) -> np.ndarray:
    M = p.padding * p.n
    out, rho = np.zeros(M // 2 + 1), np.zeros(p.n)
    load().vfo_csr_spectrum(C.byref(p.c()), _ptr(_a(z_re, M // 2 + 1)), _ptr(_a(psi, p.n * p.n)),
                            _ptr(rho), _ptr(out))
    return out


def haissinski(p: OracleParams, w, iters: int = 200, alpha: float = 0.5, Q0: float = 1.0) -> np.ndarray:
    out = np.zeros(p.n * p.n)
    load().vfo_haissinski(C.byref(p.c()), _ptr(_a(w, p.padding * p.n)), int(iters), float(alpha), float(Q0),
                          _ptr(out))
    return out.reshape(p.n, p.n)


def step(p: OracleParams, w, psi, Q0: float) -> np.ndarray:
    out = _a(psi, p.n * p.n).copy()
    work = np.zeros(2 * p.n * p.n + 4 * p.n)
    wp = None if w is None else _a(w, p.padding * p.n)
    load().vfo_step(C.byref(p.c()), _ptr(wp), _ptr(out), float(Q0), _ptr(work))
    return out.reshape(p.n, p.n)


def run(p: OracleParams, w, psi, nsteps: int, Q0: float, every: int = 0):
    """Returns (psi_final, records[rows, 7])."""
    out = _a(psi, p.n * p.n).copy()
    cap = nsteps // every if every > 0 else 0
    rec = np.zeros((max(cap, 1), 7))
    wp = None if w is None else _a(w, p.padding * p.n)
    rows = load().vfo_run(C.byref(p.c()), _ptr(wp), _ptr(out), int(nsteps), float(Q0),
                          int(every), _ptr(rec), int(cap))
    if rows < 0:
        raise MemoryError("oracle run failed to allocate")
    return out.reshape(p.n, p.n), rec[:rows]


def run_many(params, ws, psis, nsteps, Q0s):
    """Independent simulations run in parallel over OpenMP threads, in place."""
    count = len(params)
    arr = (_P * count)(*[q.c() for q in params])
    wk = [None if w is None else _a(w) for w in ws]
    ps = [_a(x) for x in psis]
    for x, q in zip(ps, params):
        if x.size != q.n * q.n:
            raise ValueError("psi size mismatch")
    wptrs = (_dp * count)(*[_ptr(w) if w is not None else _dp() for w in wk])
    pptrs = (_dp * count)(*[_ptr(x) for x in ps])
    steps = (C.c_long * count)(*[int(s) for s in nsteps])
    q0 = _a(Q0s, count)
    load().vfo_run_many(count, arr, wptrs, pptrs, steps, _ptr(q0))
    return [x.reshape(q.n, q.n) for x, q in zip(ps, params)]


# ---------------------------------------------------------------- fixed point
def _i64(x, n=None):
    x = np.ascontiguousarray(x, dtype=np.int64)
    if n is not None and x.size != n:
        raise ValueError(f"expected {n} values, got {x.size}")
    return x


def _iptr(x):
    return x.ctypes.data_as(C.POINTER(C.c_longlong))


def fix_quantize(F: int, x) -> np.ndarray:
    """raw = round(x * 2^F), ties to even."""
    x = _a(x)
    raw = np.zeros(x.shape, dtype=np.int64)
    load().vfo_fix_quantize(int(F), _ptr(x), _iptr(raw), x.size)
    return raw


def fix_charge(p: OracleParams, F: int, raw) -> float:
    return load().vfo_fix_charge(C.byref(p.c()), int(F), _iptr(_i64(raw, p.n * p.n)))


def fix_step(p: OracleParams, F: int, w, raw, Q0: float):
    """One fixed-point step.  Returns (raw_next, s used by the step)."""
    out = _i64(raw, p.n * p.n).copy()
    work = np.zeros(2 * p.n * p.n, dtype=np.int64)
    dwork = np.zeros(4 * p.n)
    s = C.c_double()
    wp = None if w is None else _a(w, p.padding * p.n)
    load().vfo_fix_step(C.byref(p.c()), int(F), _ptr(wp), _iptr(out), float(Q0), C.byref(s), _iptr(work),
                        _ptr(dwork))
    return out.reshape(p.n, p.n), s.value


def fix_run(p: OracleParams, F: int, w, raw, nsteps: int, Q0: float):
    """Returns (raw_final, s_final); the physical density is s_final * raw * 2^-F."""
    out = _i64(raw, p.n * p.n).copy()
    s = C.c_double()
    wp = None if w is None else _a(w, p.padding * p.n)
    if load().vfo_fix_run(C.byref(p.c()), int(F), _ptr(wp), _iptr(out), int(nsteps), float(Q0), C.byref(s)):
        raise MemoryError("oracle run failed to allocate")
    return out.reshape(p.n, p.n), s.value
