"""Thin ctypes binding of libvfp.so (see include/vfp.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch is optional and only supplies device memory (a
workspace tensor) and the stream.  Importing this module does not load the
library; the first handle does, and raises if ``libvfp.so`` is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvfp.so")

VFP_OK, VFP_EINVAL, VFP_ENOMEM, VFP_EDEVICE, VFP_ESTATE, VFP_EUNSTABLE = 0, -1, -2, -3, -4, -5
FP64, FP32, MIXED_BF16, MIXED_FP16, FIXED = 0, 1, 2, 3, 4
ROT_STANDARD, ROT_MANHATTAN = 0, 1
Z_SAMPLES, Z_PARALLEL_PLATES, Z_FREE_SPACE = 0, 1, 2
Z_MODELS = {"samples": Z_SAMPLES, "parallel_plate": Z_PARALLEL_PLATES, "free_space": Z_FREE_SPACE}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": MIXED_BF16, "fp16": MIXED_FP16, "fixed": FIXED}

_dp = C.POINTER(C.c_double)


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("q_min", C.c_double), ("q_max", C.c_double),
        ("p_min", C.c_double), ("p_max", C.c_double), ("steps_per_period", C.c_int32),
        ("beta", C.c_double), ("interp", C.c_int32), ("clamp", C.c_int32),
        ("renormalize", C.c_int32), ("precision", C.c_int32), ("padding", C.c_int32),
        ("rotation", C.c_int32), ("z_re", _dp), ("z_im", _dp), ("z_scale", C.c_double),
        ("psi0", _dp), ("max_steps", C.c_int64), ("z_model", C.c_int32), ("z_shield", C.c_double),
        ("fix_bits", C.c_int32),
    ]


class VfpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vfp error {code}: {msg}")
        self.code = code


_lib = None


def _share_torch_hip_runtime():
    """PyTorch ships its own HIP runtime (same soname) and loads it by path.
    Loading that file first makes libvfp.so bind to it, so one process never
    holds two HIP runtimes whichever of the two is imported first."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return
    path = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
    if os.path.exists(path):
        C.CDLL(path, mode=C.RTLD_GLOBAL)


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        _share_torch_hip_runtime()
        lib = C.CDLL(LIB_PATH)
        P = C.POINTER(Params)
        h = C.c_void_p
        sig = {
            "vfp_params_init": (None, [P]),
            "vfp_params_sizeof": (C.c_size_t, []),
            "vfp_impedance_samples": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                                C.c_double, _dp, _dp]),
            "vfp_impedance_samples_noalloc": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                                        C.c_double, _dp, _dp]),
            "vfp_workspace_size": (C.c_int, [P, C.c_int32, C.POINTER(C.c_size_t)]),
            "vfp_create": (C.c_int, [P, h, h, C.c_size_t, C.POINTER(h)]),
            "vfp_step": (C.c_int, [h, C.c_int64]),
            "vfp_profile": (C.c_int, [h, _dp]),
            "vfp_csr_power": (C.c_int, [h, _dp]),
            "vfp_moments": (C.c_int, [h, _dp]),
            "vfp_get_psi": (C.c_int, [h, _dp]),
            "vfp_set_psi": (C.c_int, [h, _dp]),
            "vfp_record": (C.c_int, [h, C.c_int32, C.c_int64]),
            "vfp_read_record": (C.c_int, [h, _dp, C.POINTER(C.c_int64)]),
            "vfp_steps_done": (C.c_int, [h, C.POINTER(C.c_int64)]),
            "vfp_destroy": (None, [h]),
            "vfp_last_error": (C.c_char_p, []),
            "vfp_batch_create": (C.c_int, [P, C.c_int32, h, h, C.c_size_t, C.POINTER(h)]),
            "vfp_batch_step": (C.c_int, [h, C.c_int64]),
            "vfp_batch_profile": (C.c_int, [h, C.c_int32, _dp]),
            "vfp_batch_csr_power": (C.c_int, [h, _dp]),
            "vfp_batch_moments": (C.c_int, [h, _dp]),
            "vfp_batch_get_psi": (C.c_int, [h, C.c_int32, _dp]),
            "vfp_batch_get_raw": (C.c_int, [h, C.c_int32, C.c_void_p, _dp]),
            "vfp_batch_set_psi": (C.c_int, [h, C.c_int32, _dp]),
            "vfp_batch_record": (C.c_int, [h, C.c_int32, C.c_int64]),
            "vfp_batch_read_record": (C.c_int, [h, C.c_int32, _dp, C.POINTER(C.c_int64)]),
            "vfp_batch_steps_done": (C.c_int, [h, C.c_int32, C.POINTER(C.c_int64)]),
            "vfp_batch_destroy": (None, [h]),
            "vfp_batch_set_tuning": (C.c_int, [h, C.c_int32, C.c_int32, C.c_int32]),
            "vfp_batch_set_streams": (C.c_int, [h, C.c_int32]),
            "vfp_batch_get_tuning": (C.c_int, [h, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "vfp_batch_autotune": (C.c_int, [h, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "vfp_device_arch": (C.c_int, [C.c_char_p, C.c_int32]),
            "vfp_batch_kernel_timing": (C.c_int, [h, C.c_int32]),
            "vfp_batch_last_wake": (C.c_int, [h, C.c_int32, _dp]),
            "vfp_batch_csr_spectrum": (C.c_int, [h, C.c_int32, _dp]),
            "vfp_csr_spectrum": (C.c_int, [h, _dp]),
            "vfp_batch_seed": (C.c_int, [h, C.c_int32, C.c_int32]),
            "vfp_batch_haissinski": (C.c_int, [h, C.c_int32, C.c_int32, C.c_double]),
            "vfp_haissinski": (C.c_int, [h, C.c_int32, C.c_double]),
            "vfp_batch_kernel_times": (C.c_int, [h, _dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.vfp_params_sizeof() != C.sizeof(Params):
            raise ImportError("vfp_params layout mismatch between libvfp.so and the binding")
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != VFP_OK:
        raise VfpError(rc, load().vfp_last_error().decode(errors="replace"))


def _f64(x, n=None):
    if x is None:
        return None
    a = np.ascontiguousarray(x, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def make_params(n=256, q_range=(-8.0, 8.0), p_range=None, steps_per_period=1000, beta=1e-3,
                interp=4, clamp=0, renormalize=1, precision="fp32", padding=2,
                rotation=ROT_STANDARD, z_re=None, z_im=None, z_scale=0.0, psi0=None,
                max_steps=0, z_model="samples", z_shield=1.0, fix_bits=44):
    """Returns (Params, keepalive) -- keepalive holds the numpy arrays the
    struct points to until the create call has copied them."""
    p = Params()
    load().vfp_params_init(C.byref(p))
    p_range = q_range if p_range is None else p_range
    p.n = int(n)
    p.q_min, p.q_max = map(float, q_range)
    p.p_min, p.p_max = map(float, p_range)
    p.steps_per_period = int(steps_per_period)
    p.beta = float(beta)
    p.interp = int(interp)
    p.clamp = int(clamp)
    p.renormalize = int(renormalize)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.padding = int(padding)
    p.rotation = int(rotation)
    M = p.padding * p.n
    zr = _f64(z_re, None if z_re is None else M // 2 + 1)
    zi = _f64(z_im, None if z_im is None else M // 2 + 1)
    p.z_re, p.z_im = _ptr(zr), _ptr(zi)
    p.z_scale = float(z_scale)
    ps = _f64(psi0, None if psi0 is None else p.n * p.n)
    p.psi0 = _ptr(ps)
    p.max_steps = int(max_steps)
    p.z_model = Z_MODELS[z_model] if isinstance(z_model, str) else int(z_model)
    p.z_shield = float(z_shield)
    p.fix_bits = int(fix_bits)
    return p, (zr, zi, ps)


def impedance_samples(n, padding, q_min, q_max, model="parallel_plate", Pi=1.0, noalloc=False):
    """Z_k at kappa_k = 2 pi k / (M dq), k = 0..M/2, evaluated on the device
    (the samples a simulation created with z_model=model uses).  Returns
    (z_re, z_im) as float64 arrays.  noalloc=True calls the entry point that
    uses the library's static device scratch instead of allocating."""
    M = int(padding) * int(n)
    zr = np.empty(M // 2 + 1, dtype=np.float64)
    zi = np.empty(M // 2 + 1, dtype=np.float64)
    m = Z_MODELS[model] if isinstance(model, str) else int(model)
    fn = load().vfp_impedance_samples_noalloc if noalloc else load().vfp_impedance_samples
    _check(fn(m, int(n), int(padding), float(q_min), float(q_max), float(Pi), _ptr(zr), _ptr(zi)))
    return zr, zi


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(int(stream.cuda_stream))      # torch.cuda.Stream


def _torch_workspace(nbytes: int):
    import torch  # device memory only
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


class Batch:
    """A set of independent simulations advanced together (vfp_batch_*)."""

    def __init__(self, params: Sequence[dict], stream=None, torch_workspace: bool = False):
        lib = load()
        ps, keep = [], []
        for d in params:
            p, k = make_params(**d)
            ps.append(p)
            keep.append(k)
        arr = (Params * len(ps))(*ps)
        self.count = len(ps)
        self.n = [p.n for p in ps]
        self._key = (ps[0].interp, ps[0].precision, ps[0].rotation, ps[0].clamp)
        self.M = [p.n * p.padding for p in ps]
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if torch_workspace:
            nbytes = C.c_size_t()
            _check(lib.vfp_workspace_size(arr, self.count, C.byref(nbytes)))
            self._ws = _torch_workspace(nbytes.value)
            ws_ptr, ws_bytes = C.c_void_p(self._ws.data_ptr()), nbytes.value
        self._h = C.c_void_p()
        _check(lib.vfp_batch_create(arr, self.count, _stream_handle(stream), ws_ptr, ws_bytes,
                                    C.byref(self._h)))

    def step(self, nticks: int):
        _check(load().vfp_batch_step(self._h, int(nticks)))

    def profile(self, i: int) -> np.ndarray:
        out = np.zeros(self.n[i])
        _check(load().vfp_batch_profile(self._h, i, _ptr(out)))
        return out

    def csr_power(self) -> np.ndarray:
        out = np.zeros(self.count)
        _check(load().vfp_batch_csr_power(self._h, _ptr(out)))
        return out

    def moments(self) -> np.ndarray:
        out = np.zeros((self.count, 5))
        _check(load().vfp_batch_moments(self._h, _ptr(out)))
        return out

    def get_psi(self, i: int) -> np.ndarray:
        out = np.zeros((self.n[i], self.n[i]))
        _check(load().vfp_batch_get_psi(self._h, i, _ptr(out)))
        return out

    def set_psi(self, i: int, psi):
        a = _f64(psi, self.n[i] ** 2)
        _check(load().vfp_batch_set_psi(self._h, i, _ptr(a)))

    def get_raw(self, i: int):
        """(stored density as held on the device, s): float64, int64 raw
        fixed-point values or float32 by precision; physical = s * stored
        (times 2^-fix_bits for the fixed-point storage)."""
        dt = {FP64: np.float64, FIXED: np.int64}.get(self._key[1], np.float32)
        out = np.zeros((self.n[i], self.n[i]), dtype=dt)
        s = C.c_double()
        _check(load().vfp_batch_get_raw(self._h, i, out.ctypes.data_as(C.c_void_p), C.byref(s)))
        return out, s.value

    def record(self, every: int, cap: int):
        _check(load().vfp_batch_record(self._h, int(every), int(cap)))

    def read_record(self, i: int) -> np.ndarray:
        rows = C.c_int64()
        _check(load().vfp_batch_read_record(self._h, i, None, C.byref(rows)))
        out = np.zeros((rows.value, 7))
        if rows.value:
            _check(load().vfp_batch_read_record(self._h, i, _ptr(out), C.byref(rows)))
        return out

    def steps_done(self, i: int) -> int:
        v = C.c_int64()
        _check(load().vfp_batch_steps_done(self._h, i, C.byref(v)))
        return v.value

    def set_tuning(self, cells_per_unit: int = 0, use_graph: bool = True, staged: int | None = None):
        """staged: 0 the generic kernel, 1 the LDS-staged kernel with a wake
        launch per tick (split), 2 the LDS-staged kernel with the one-launch tick
        (fused); None keeps the current form."""
        if staged is None:
            staged = self.get_tuning()[2]
        _check(load().vfp_batch_set_tuning(self._h, int(cells_per_unit), int(bool(use_graph)), int(staged)))

    def set_streams(self, groups: int):
        """1: every simulation on the batch's stream; 2-4: that many parts of
        about equal cell count, each on its own stream."""
        _check(load().vfp_batch_set_streams(self._h, int(groups)))

    def get_tuning(self) -> tuple:
        """(cells per unit, graph replay, kernel layout) in force."""
        c, g, l = C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().vfp_batch_get_tuning(self._h, C.byref(c), C.byref(g), C.byref(l)))
        return c.value, bool(g.value), l.value

    def autotune(self, ticks: int = 20, cache: Optional[str] = None) -> tuple:
        """Pick cells per unit and kernel layout by timing (vfp_batch_autotune).
        With `cache` (a JSON file), a previous choice for the same device,
        grid-size mix, interpolation, precision and rotation is reused and new
        choices are stored.  Returns (cells, layout)."""
        key = None
        if cache:
            import json
            buf = C.create_string_buffer(128)
            _check(load().vfp_device_arch(buf, 128))
            key = "|".join([buf.value.decode(), ",".join(f"{n}x{k}" for n, k in sorted(
                {n: self.n.count(n) for n in self.n}.items())), str(self._key)])
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            if key in table:
                cells, layout = table[key]
                self.set_tuning(cells, True, layout)
                return int(cells), int(layout)
        c, l = C.c_int32(), C.c_int32()
        _check(load().vfp_batch_autotune(self._h, int(ticks), C.byref(c), C.byref(l)))
        if cache:
            import json
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            table[key] = [c.value, l.value]
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return c.value, l.value

    def csr_spectrum(self, i: int) -> np.ndarray:
        out = np.zeros(self.M[i] // 2 + 1)
        _check(load().vfp_batch_csr_spectrum(self._h, i, _ptr(out)))
        return out

    def haissinski(self, i: int, iters: int = 200, alpha: float = 0.5):
        _check(load().vfp_batch_haissinski(self._h, int(i), int(iters), float(alpha)))

    def seed(self, dst: int, src: int):
        _check(load().vfp_batch_seed(self._h, int(dst), int(src)))

    def last_wake(self, i: int) -> np.ndarray:
        out = np.zeros(self.n[i])
        _check(load().vfp_batch_last_wake(self._h, i, _ptr(out)))
        return out

    def kernel_timing(self, enable: bool = True):
        _check(load().vfp_batch_kernel_timing(self._h, int(bool(enable))))

    def kernel_times(self) -> dict:
        out = np.zeros(4)
        _check(load().vfp_batch_kernel_times(self._h, _ptr(out)))
        return {"step_ms": out[0], "step_launches": int(out[1]), "wake_ms": out[2], "wake_launches": int(out[3])}

    def close(self):
        if getattr(self, "_h", None):
            load().vfp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sim:
    """One simulation in the plain per-simulation form (vfp_*)."""

    def __init__(self, stream=None, torch_workspace: bool = False, **params):
        lib = load()
        p, keep = make_params(**params)
        self.n = p.n
        self.M = p.n * p.padding
        self._precision = p.precision
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if torch_workspace:
            nbytes = C.c_size_t()
            _check(lib.vfp_workspace_size(C.byref(p), 1, C.byref(nbytes)))
            self._ws = _torch_workspace(nbytes.value)
            ws_ptr, ws_bytes = C.c_void_p(self._ws.data_ptr()), nbytes.value
        self._h = C.c_void_p()
        _check(lib.vfp_create(C.byref(p), _stream_handle(stream), ws_ptr, ws_bytes, C.byref(self._h)))
        del keep

    def step(self, nsteps: int):
        _check(load().vfp_step(self._h, int(nsteps)))

    def profile(self) -> np.ndarray:
        out = np.zeros(self.n)
        _check(load().vfp_profile(self._h, _ptr(out)))
        return out

    def csr_power(self) -> float:
        out = np.zeros(1)
        _check(load().vfp_csr_power(self._h, _ptr(out)))
        return float(out[0])

    def moments(self) -> np.ndarray:
        out = np.zeros(5)
        _check(load().vfp_moments(self._h, _ptr(out)))
        return out

    def csr_spectrum(self) -> np.ndarray:
        out = np.zeros(self.M // 2 + 1)
        _check(load().vfp_csr_spectrum(self._h, _ptr(out)))
        return out

    def haissinski(self, iters: int = 200, alpha: float = 0.5):
        _check(load().vfp_haissinski(self._h, int(iters), float(alpha)))

    def get_psi(self) -> np.ndarray:
        out = np.zeros((self.n, self.n))
        _check(load().vfp_get_psi(self._h, _ptr(out)))
        return out

    def set_psi(self, psi):
        a = _f64(psi, self.n * self.n)
        _check(load().vfp_set_psi(self._h, _ptr(a)))

    def get_raw(self):
        """(stored density, s) as Batch.get_raw."""
        dt = {FP64: np.float64, FIXED: np.int64}.get(self._precision, np.float32)
        out = np.zeros((self.n, self.n), dtype=dt)
        s = C.c_double()
        _check(load().vfp_batch_get_raw(self._h, 0, out.ctypes.data_as(C.c_void_p), C.byref(s)))
        return out, s.value

    def record(self, every: int, cap: int):
        _check(load().vfp_record(self._h, int(every), int(cap)))

    def read_record(self) -> np.ndarray:
        rows = C.c_int64()
        _check(load().vfp_read_record(self._h, None, C.byref(rows)))
        out = np.zeros((rows.value, 7))
        if rows.value:
            _check(load().vfp_read_record(self._h, _ptr(out), C.byref(rows)))
        return out

    def steps_done(self) -> int:
        v = C.c_int64()
        _check(load().vfp_steps_done(self._h, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            load().vfp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sim_kwargs(sim, precision="fp32", device_impedance=False, **over) -> dict:
    """Keyword arguments for Sim/Batch from an ``inputs.Sim`` recipe.  With
    device_impedance the impedance of the recipe's model is evaluated by the
    library on the device instead of being passed as host samples."""
    has_z = sim.Pi is not None and sim.z_scale != 0.0
    d = dict(n=sim.n, q_range=(sim.q_min, sim.q_max), p_range=(sim.p_min, sim.p_max),
             steps_per_period=sim.steps_per_period, beta=sim.beta, interp=sim.interp,
             clamp=sim.clamp, renormalize=sim.renormalize, precision=precision,
             padding=sim.padding, rotation=sim.rotation,
             z_scale=sim.z_scale if has_z else 0.0, psi0=sim.psi0())
    if has_z and device_impedance:
        d.update(z_model=sim.model, z_shield=sim.Pi)
    else:
        d["z_re"], d["z_im"] = sim.impedance()
    d.update(over)
    return d
