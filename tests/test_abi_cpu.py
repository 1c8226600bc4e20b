"""The C-ABI library builds, loads and exports every symbol its header
declares; parameter validation runs on the host without a GPU."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1611_05293_amd import vfp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vfp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vfp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(vfp.LIB_PATH), "libvfp.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", vfp.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(vfp_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    assert len(declared_functions()) >= 28


def test_loads_and_layout_matches():
    lib = vfp.load()
    assert lib.vfp_params_sizeof() == C.sizeof(vfp.Params)


def test_params_defaults():
    p = vfp.Params()
    vfp.load().vfp_params_init(C.byref(p))
    assert (p.n, p.steps_per_period, p.interp, p.precision, p.padding, p.renormalize) == (256, 1000, 4, 1, 2, 1)
    assert p.q_min == -8.0 and p.p_max == 8.0 and p.beta == 1e-3 and not p.z_re
    assert p.z_model == vfp.Z_SAMPLES and p.z_shield == 1.0


def test_densities_the_storage_holds_are_accepted():
    assert _ws(n=16, psi0=np.full(256, 1e39), precision="fp64")[0] == 0
    assert _ws(n=16, psi0=np.full(256, 3e38), precision="fp32")[0] == 0
    assert _ws(n=16, psi0=np.full(256, 3.9), precision="fixed", fix_bits=59)[0] == 0


def test_fixed_point_storage_is_eight_bytes():
    rc1, b64, _ = _ws(n=64, precision="fp64")
    rc2, bfx, _ = _ws(n=64, precision="fixed")
    assert rc1 == rc2 == 0 and bfx >= 2 * 64 * 64 * 8 and bfx >= b64


def test_device_impedance_models_validate_on_the_host():
    assert _ws(z_model="free_space", z_scale=1.0)[0] == 0
    assert _ws(z_model="parallel_plate", z_shield=0.4, z_scale=1.0)[0] == 0


@pytest.mark.parametrize("args,msg", [
    ((0, 64, 2, -8.0, 8.0, 1.0), "model"),
    ((1, 8, 2, -8.0, 8.0, 1.0), "n in"),
    ((1, 64, 1, -8.0, 8.0, 1.0), "padding"),
    ((1, 64, 2, 8.0, -8.0, 1.0), "q_min"),
    ((1, 64, 2, -8.0, 8.0, -1.0), "Pi"),
])
def test_impedance_samples_rejects_bad_arguments_on_the_host(args, msg):
    with pytest.raises(vfp.VfpError, match=msg):
        vfp.impedance_samples(*args[1:3], *args[3:5], model=args[0], Pi=args[5])


def _ws(**kw):
    p, keep = vfp.make_params(**kw)
    nb = C.c_size_t()
    rc = vfp.load().vfp_workspace_size(C.byref(p), 1, C.byref(nb))
    return rc, nb.value, vfp.load().vfp_last_error().decode()


def test_workspace_size_scales_with_grid_and_precision():
    rc1, b64, _ = _ws(n=64, precision="fp64")
    rc2, b32, _ = _ws(n=64, precision="fp32")
    rc3, b256, _ = _ws(n=256, precision="fp32")
    assert rc1 == rc2 == rc3 == 0
    assert b64 >= 2 * 64 * 64 * 8 and b32 >= 2 * 64 * 64 * 4 and b256 > 10 * b32


@pytest.mark.parametrize("kw,code,msg", [
    (dict(n=8), vfp.VFP_EINVAL, "n must be"),
    (dict(interp=5), vfp.VFP_EINVAL, "interp"),
    (dict(steps_per_period=0), vfp.VFP_EINVAL, "steps_per_period"),
    (dict(beta=-1.0), vfp.VFP_EINVAL, "beta"),
    (dict(padding=1), vfp.VFP_EINVAL, "padding"),
    (dict(q_range=(1.0, -1.0)), vfp.VFP_EINVAL, "q_min"),
    (dict(precision=9), vfp.VFP_EINVAL, "precision"),
    (dict(beta=50.0, steps_per_period=10), vfp.VFP_EUNSTABLE, "unstable"),
    (dict(n=16, psi0=np.full(256, 1e39)), vfp.VFP_EINVAL, "binary32"),
    (dict(n=16, psi0=np.full(256, 1e39), precision="fp16"), vfp.VFP_EINVAL, "binary32"),
    (dict(n=16, psi0=np.zeros(256)), vfp.VFP_EINVAL, "positive, finite charge"),
    (dict(n=16, psi0=np.zeros(256), renormalize=0), vfp.VFP_EINVAL, "positive, finite charge"),
    (dict(n=16, psi0=-np.ones(256), precision="fp64"), vfp.VFP_EINVAL, "positive, finite charge"),
    (dict(n=16, psi0=np.full(256, 1e307), precision="fp64"), vfp.VFP_EINVAL, "positive, finite charge"),
    (dict(precision="fixed", fix_bits=15), vfp.VFP_EINVAL, "fix_bits"),
    (dict(precision="fixed", fix_bits=60), vfp.VFP_EINVAL, "fix_bits"),
    (dict(n=16, precision="fixed", fix_bits=59, psi0=np.full(256, 4.0)), vfp.VFP_EINVAL, "2^(61-fix_bits)"),
    (dict(precision=5), vfp.VFP_EINVAL, "precision"),
    (dict(z_model=3), vfp.VFP_EINVAL, "z_model"),
    (dict(z_model="parallel_plate", z_shield=0.0), vfp.VFP_EINVAL, "z_shield"),
    (dict(z_model="parallel_plate", z_shield=float("inf")), vfp.VFP_EINVAL, "z_shield"),
    (dict(z_model="free_space", z_re=np.zeros(257), z_im=np.zeros(257)), vfp.VFP_EINVAL, "NULL"),
])
def test_validation_errors(kw, code, msg):
    rc, _, err = _ws(**kw)
    assert rc == code and msg in err


def test_create_rejects_bad_input_before_touching_the_device():
    p, keep = vfp.make_params(n=32, psi0=np.full(32 * 32, np.nan))
    h = C.c_void_p()
    rc = vfp.load().vfp_create(C.byref(p), None, None, 0, C.byref(h))
    assert rc == vfp.VFP_EINVAL and "finite" in vfp.load().vfp_last_error().decode()
    p2, keep2 = vfp.make_params(n=32, interp=3)
    arr = (vfp.Params * 2)(p, p2)
    p.psi0 = None
    arr = (vfp.Params * 2)(p, p2)
    rc = vfp.load().vfp_batch_create(arr, 2, None, None, 0, C.byref(h))
    assert rc == vfp.VFP_EINVAL and "agree" in vfp.load().vfp_last_error().decode()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(vfp, "_lib", None)
    monkeypatch.setattr(vfp, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        vfp.load()
