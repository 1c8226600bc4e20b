"""GPU parity of the plain per-simulation form against the FP64 oracle.

Bars: FP64 rel-L1(psi) <= 1e-12; FP32 and the mixed-precision wakes
rel-L1 <= 1e-5 at 100 steps of the single-simulation workload; diagnostics
(rho, moments, CSR power) against the oracle's definitions."""
import math

import numpy as np
import pytest

import oracle
from paper_1611_05293_amd import inputs, vfp
from gpu_common import oracle_run, rel_l1, small_sim

pytestmark = pytest.mark.gpu


def gpu_run(sim, nsteps, precision, psi0=None, **over):
    kw = vfp.sim_kwargs(sim, precision=precision, **over)
    if psi0 is not None:
        kw["psi0"] = psi0
    s = vfp.Sim(**kw)
    s.step(nsteps)
    return s


def test_cfg1_fp64_equilibrium_full_period():
    sim = inputs.config(1)[0]
    ref, _, _, _ = oracle_run(sim, 500)
    g = gpu_run(sim, 500, "fp64")
    out = g.get_psi()
    assert rel_l1(out, ref) <= 1e-12
    m = g.moments()
    assert abs(m[0] - 1.0) < 1e-12
    # the equilibrium drifts only by the method's own discretisation error
    # (K = 3 on 64 points), the same on both sides
    dev_gpu, dev_or = rel_l1(out, sim.psi0()), rel_l1(ref, sim.psi0())
    print(f"cfg1 deviation from equilibrium after 1 period: gpu {dev_gpu:.4e} oracle {dev_or:.4e}")
    assert abs(dev_gpu - dev_or) < 1e-10 and dev_gpu < 0.02


def test_cfg2_fp64_1000_steps():
    sim = inputs.config(2)[0]
    ref, _, _, _ = oracle_run(sim, 1000)
    out = gpu_run(sim, 1000, "fp64").get_psi()
    err = rel_l1(out, ref)
    print(f"cfg2 fp64 1000 steps rel-L1 {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
def test_cfg2_reduced_precision_100_steps(precision):
    sim = inputs.config(2)[0]
    ref, _, _, _ = oracle_run(sim, 100)
    out = gpu_run(sim, 100, precision).get_psi()
    err = rel_l1(out, ref)
    print(f"cfg2 {precision} 100 steps rel-L1 {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("K", [3, 4])
@pytest.mark.parametrize("clamp", [0, 1])
@pytest.mark.parametrize("rotation", [0, 1])
@pytest.mark.parametrize("n", [16, 37, 48])
def test_step_variants_fp64(K, clamp, rotation, n):
    sim = small_sim(n=n, K=K, clamp=clamp, rotation=rotation, steps=53 + n)
    ref, _, _, _ = oracle_run(sim, 30)
    out = gpu_run(sim, 30, "fp64").get_psi()
    assert rel_l1(out, ref) <= 1e-12


@pytest.mark.parametrize("K", [3, 4])
@pytest.mark.parametrize("clamp", [0, 1])
@pytest.mark.parametrize("rotation", [0, 1])
def test_step_variants_fp32(K, clamp, rotation):
    sim = small_sim(n=72, K=K, clamp=clamp, rotation=rotation, steps=120)
    ref, _, _, _ = oracle_run(sim, 20)
    out = gpu_run(sim, 20, "fp32").get_psi()
    assert rel_l1(out, ref) <= 1e-5


def test_raw_map_without_renormalisation_fp64():
    sim = small_sim(n=40, renormalize=0, lo=-4.0, hi=4.0, sigma0=1.3)
    ref, _, _, _ = oracle_run(sim, 25)
    g = gpu_run(sim, 25, "fp64")
    assert rel_l1(g.get_psi(), ref) <= 1e-12
    d = (8.0 / 39) ** 2
    assert abs(g.moments()[0] - d * ref.sum()) < 1e-12
    assert abs(d * ref.sum() - 1.0) > 1e-6          # charge did leave the grid


def test_quarter_turn_is_a_permutation():
    """steps_per_period = 4, no damping, no current: one step is the
    clockwise quarter turn numpy.rot90(psi, -1) on the symmetric lattice."""
    n = 33
    rng = np.random.default_rng(5)
    psi = rng.random((n, n)) + 0.5
    g = vfp.Sim(n=n, q_range=(-5, 5), steps_per_period=4, beta=0.0, interp=4, precision="fp64",
                renormalize=0, psi0=psi)
    g.step(1)
    assert np.max(np.abs(g.get_psi() - np.rot90(psi, -1))) < 1e-13


def test_diagnostics_match_oracle():
    sim = small_sim(n=64, S=1.5, Pi=0.5)
    ref, _, w, p = oracle_run(sim, 40)
    g = gpu_run(sim, 40, "fp64")
    assert rel_l1(g.profile(), oracle.profile(p, ref)) < 1e-12
    m, mo = g.moments(), oracle.moments(p, ref)
    assert np.allclose(m, mo, rtol=1e-11, atol=1e-13)
    P, Po = g.csr_power(), oracle.csr_power(p, w, ref)
    assert abs(P - Po) <= 1e-11 * abs(Po) and abs(Po) > 0


def test_record_ring_matches_oracle_series():
    sim = small_sim(n=48)
    _, rec, _, _ = oracle_run(sim, 60, every=10)
    kw = vfp.sim_kwargs(sim, precision="fp64")
    g = vfp.Sim(**kw)
    g.record(10, 100)
    g.step(60)
    r = g.read_record()
    assert r.shape == rec.shape == (6, 7)
    assert np.array_equal(r[:, 0], rec[:, 0])
    assert np.allclose(r[:, 1:], rec[:, 1:], rtol=1e-10, atol=1e-13)


def test_set_get_roundtrip_and_resume():
    sim = small_sim(n=40)
    kw = vfp.sim_kwargs(sim, precision="fp64")
    a = vfp.Sim(**kw)
    a.step(15)
    mid = a.get_psi()
    assert a.steps_done() == 15
    b = vfp.Sim(**kw)
    b.set_psi(mid)
    assert b.steps_done() == 0
    a.step(10)
    b.step(10)
    # b's Q0 is the charge of mid, which equals a's Q0 after renormalisation
    assert rel_l1(b.get_psi(), a.get_psi()) < 1e-13


def test_bitwise_determinism_fp32():
    sim = small_sim(n=96, S=2.0)
    a = gpu_run(sim, 50, "fp32").get_psi()
    b = gpu_run(sim, 50, "fp32").get_psi()
    assert np.array_equal(a, b)


def test_set_psi_rejects_non_finite():
    g = vfp.Sim(n=32, q_range=(-5, 5), precision="fp32")
    bad = np.ones((32, 32))
    bad[3, 4] = np.inf
    with pytest.raises(vfp.VfpError) as e:
        g.set_psi(bad)
    assert e.value.code == vfp.VFP_EINVAL


def test_torch_workspace_and_stream():
    torch = pytest.importorskip("torch")
    sim = small_sim(n=48)
    ref, _, _, _ = oracle_run(sim, 12)
    st = torch.cuda.Stream()
    g = vfp.Sim(stream=st, torch_workspace=True, **vfp.sim_kwargs(sim, precision="fp64"))
    g.step(12)
    assert rel_l1(g.get_psi(), ref) <= 1e-12


@pytest.mark.parametrize("precision,v_tol", [("fp32", 1e-4), ("fp16", 1e-4), ("bf16", 1e-3)])
def test_per_output_errors_vs_oracle(precision, v_tol):
    """Error of every output of the reduced-precision forms against the FP64
    oracle after 100 steps of the single-simulation workload: psi (rel-L1),
    the wake the last step used (max error / max |V|), rho, Q, sigma_q,
    sigma_p and the CSR power."""
    sim = inputs.config(2)[0]
    ref99, _, w, p = oracle_run(sim, 99)
    ref = oracle.step(p, w, ref99, 1.0)
    V99 = oracle.wake(p, w, oracle.profile(p, ref99))
    b = vfp.Batch([vfp.sim_kwargs(sim, precision=precision)])
    b.step(100)
    errs = {
        "psi": rel_l1(b.get_psi(0), ref),
        "V": float(np.abs(b.last_wake(0) - V99).max() / np.abs(V99).max()),
        "rho": rel_l1(b.profile(0), oracle.profile(p, ref)),
    }
    m, mo = b.moments()[0], oracle.moments(p, ref)
    errs.update({"Q": abs(m[0] - mo[0]), "sigma_q": abs(m[2] / mo[2] - 1), "sigma_p": abs(m[4] / mo[4] - 1)})
    P, Po = b.csr_power()[0], oracle.csr_power(p, w, ref)
    errs["P"] = abs(P / Po - 1)
    print(f"{precision} errors after 100 steps: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert errs["psi"] <= 1e-5 and errs["V"] <= v_tol and errs["rho"] <= 1e-5
    assert errs["Q"] <= 1e-12 and errs["sigma_q"] <= 1e-6 and errs["sigma_p"] <= 1e-6 and errs["P"] <= 1e-5


def test_fp32_error_growth_to_one_period():
    """rel-L1 of FP32 against FP64 on the GPU over one synchrotron period of
    the single-simulation workload (the FP64 path equals the oracle to 1e-12):
    the error must stay small and grow no faster than linearly."""
    sim = inputs.config(2)[0]
    a = vfp.Sim(**vfp.sim_kwargs(sim, precision="fp64"))
    b = vfp.Sim(**vfp.sim_kwargs(sim, precision="fp32"))
    done, curve = 0, []
    for t in (10, 100, 1000):
        a.step(t - done)
        b.step(t - done)
        done = t
        curve.append((t, rel_l1(b.get_psi(), a.get_psi())))
    print("fp32 rel-L1 growth: " + ", ".join(f"{t}: {e:.2e}" for t, e in curve))
    assert curve[1][1] <= 1e-5 and curve[2][1] <= 1e-4
    assert curve[2][1] <= 30 * curve[1][1]


def test_binary32_binary64_converged_bunch_length():
    """Sec. IV.A, Tab. datatype offset: a 16-bit quantised Gaussian with
    sigma = 2.8 damped with tau = 5 synchrotron periods converges to the same
    bunch length in binary32 and binary64.  The paper finds the two within
    1e-6 on its (unstated) grid; on this coarse grid (dq = 0.25) the
    converged value is sensitive to the storage rounding of psi itself (an
    FP64 run whose psi is rounded to binary32 after every step moves by
    ~3e-5), so the bound here is 2e-5 after 80 periods."""
    n, lo, hi, steps = 128, -16.0, 16.0, 500
    beta = 1.0 / (2 * math.pi * 5.0)
    psi0 = inputs.quantize16(inputs.gaussian_psi(n, lo, hi, lo, hi, 2.8, 2.8))
    kw = dict(n=n, q_range=(lo, hi), steps_per_period=steps, beta=beta, interp=4, psi0=psi0)
    s64 = vfp.Sim(precision="fp64", **kw)
    s32 = vfp.Sim(precision="fp32", **kw)
    s64.step(steps * 80)
    s32.step(steps * 80)
    m64, m32 = s64.moments(), s32.moments()
    print(f"converged sigma_q: fp64 {m64[2]:.10f} fp32 {m32[2]:.10f}; relative difference "
          f"{m32[2] / m64[2] - 1:.3e}")
    assert abs(m32[2] / m64[2] - 1) < 2e-5
    assert abs(m64[2] - 1.0) < 1e-5          # damped to the equilibrium length


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_long_run_statistics_match_oracle_ensemble(precision):
    """12,000 steps (40 periods) with current: time averages over the second
    half of sigma_q, sigma_p and of the CSR power P (mean, spread, dominant
    frequency) from the GPU agree with the oracle for every seed, within twice
    the oracle's seed-to-seed spread or the paper's data-type bound.  (At this
    grid size the runs settle instead of bursting, so the seed spread is tiny
    and the floor decides.)"""
    n, lo, hi, steps, periods = 96, -8.0, 8.0, 300, 40
    seeds = (1, 2, 3)
    stats = {"oracle": [], "gpu": []}
    for seed in seeds:
        sim = inputs.Sim(n, lo, hi, lo, hi, steps, 0.01, 4, z_scale=4.0, Pi=0.5, noise=1e-4, seed=seed)
        _, rec, _, _ = oracle_run(sim, steps * periods, every=10)
        g = vfp.Sim(**vfp.sim_kwargs(sim, precision=precision))
        g.record(10, steps * periods // 10)
        g.step(steps * periods)
        rg = g.read_record()
        for key, r in (("oracle", rec), ("gpu", rg)):
            h = r[len(r) // 2:]
            spec = np.abs(np.fft.rfft(h[:, 6] - h[:, 6].mean()))
            stats[key].append([h[:, 3].mean(), h[:, 5].mean(), h[:, 6].mean(), h[:, 6].std(), float(np.argmax(spec))])
    o, gpu = np.array(stats["oracle"]), np.array(stats["gpu"])
    spread = o.std(axis=0)
    # floor: the paper's bound for switching data types, < 0.1 % (Tab. maximum errors);
    # the spread of P around its mean within 5 %, the spectral peak within one bin
    floor = np.array([1e-3 * o[:, 0].mean(), 1e-3 * o[:, 1].mean(), 1e-3 * o[:, 2].mean(),
                      0.05 * o[:, 3].mean(), 1.0])
    tol = np.maximum(2 * spread, floor)
    print(f"{precision} long-run stats (sigma_q, sigma_p, <P>, std P, peak bin)\n oracle {o.mean(0)}\n gpu    {gpu.mean(0)}\n tol {tol}")
    assert np.all(np.abs(gpu - o) <= tol[None, :])
