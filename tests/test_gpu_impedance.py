"""Impedance samples computed on the device (Sec. II.B models) against the
host samples of the input generator, and simulations that take their
impedance from the device against the same simulations given host samples
and against the FP64 oracle."""
import numpy as np
import pytest

from paper_1611_05293_amd import inputs, vfp
from gpu_common import oracle_run, rel_l1, small_sim

pytestmark = pytest.mark.gpu

# The host samples come from scipy's scaled Airy functions, the device's from
# Taylor stepping and the asymptotic expansions; near u = 100 both lose about
# log10(zeta^2) digits to the cancellation inside Ai'Bi' + u Ai Bi, so samples
# are compared on the scale of the largest |Z_k| (what the wake sums over).
TOL = 1e-11


@pytest.mark.parametrize("n,pad,Pi", [(32, 2, 0.5), (64, 2, 1.0), (256, 3, 0.3), (1024, 2, 3.0),
                                      (512, 2, 0.05), (256, 2, 20.0), (4096, 2, 1.0)])
def test_parallel_plate_samples_match_host(n, pad, Pi):
    zr, zi = vfp.impedance_samples(n, pad, -8.0, 8.0, "parallel_plate", Pi)
    hr, hi = inputs.impedance_samples(n, pad, -8.0, 8.0, "parallel_plate", Pi)
    z, h = zr + 1j * zi, hr + 1j * hi
    assert z.shape == (n * pad // 2 + 1,)
    assert z[0] == 0.0
    err = np.abs(z - h).max() / np.abs(h).max()
    print(f"n={n} pad={pad} Pi={Pi}: max |dZ| / max |Z| = {err:.2e}")
    assert err <= TOL
    # Re Z >= 0 (a passive impedance) to rounding
    assert zr.min() >= -1e-14 * np.abs(h).max()


@pytest.mark.parametrize("n,pad", [(16, 2), (100, 3), (1024, 2)])
def test_free_space_samples_match_host(n, pad):
    zr, zi = vfp.impedance_samples(n, pad, -6.0, 7.0, "free_space")
    hr, hi = inputs.impedance_samples(n, pad, -6.0, 7.0, "free_space")
    assert zr[0] == zi[0] == 0.0
    np.testing.assert_allclose(zr[1:], hr[1:], rtol=1e-15, atol=0)
    np.testing.assert_allclose(zi[1:], hi[1:], rtol=1e-15, atol=0)


def test_weak_shielding_approaches_free_space():
    """Plates far away (small Pi) leave the free-space impedance at high
    frequency: the two device models agree there."""
    n, pad = 256, 2
    pr, pi = vfp.impedance_samples(n, pad, -8.0, 8.0, "parallel_plate", 0.05)
    fr, fi = vfp.impedance_samples(n, pad, -8.0, 8.0, "free_space")
    k = np.arange(n // 2, n + 1)
    d = np.abs((pr[k] + 1j * pi[k]) - (fr[k] + 1j * fi[k])) / np.abs(fr[k] + 1j * fi[k])
    assert d.max() < 1e-8


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp16", 1e-5)])
def test_batch_with_device_impedance_matches_host_samples(precision, tol):
    sims = [small_sim(n=32, steps=80, S=0.4, Pi=0.5, seed=1),
            small_sim(n=64, steps=160, S=2.0, Pi=2.0, seed=3, lo=-7.0, hi=7.0),
            small_sim(n=100, steps=250, S=0.9, Pi=0.8, seed=4, lo=-8.0, hi=8.0)]
    a = vfp.Batch([vfp.sim_kwargs(s, precision=precision, device_impedance=True) for s in sims])
    b = vfp.Batch([vfp.sim_kwargs(s, precision=precision) for s in sims])
    nt = 25
    a.step(nt)
    b.step(nt)
    for i, s in enumerate(sims):
        d = rel_l1(a.get_psi(i), b.get_psi(i))
        ref, _, _, _ = oracle_run(s, nt)
        e = rel_l1(a.get_psi(i), ref)
        print(f"{precision} sim {i}: device vs host Z {d:.2e}, vs oracle {e:.2e}")
        assert d <= tol and e <= tol
    # the samples agree to ~1e-12 of max |Z|, not of each Re Z_k: a strongly
    # shielded bunch radiates little, so its power is compared on the scale
    # of the batch's largest power
    pa, pb = a.csr_power(), b.csr_power()
    assert np.allclose(pa, pb, rtol=10 * tol, atol=10 * tol * np.abs(pb).max())


def test_free_space_model_simulation_matches_oracle():
    s = small_sim(n=64, steps=160, S=0.8, Pi=1.0, seed=7)
    s.model = "free_space"
    a = vfp.Batch([vfp.sim_kwargs(s, precision="fp64", device_impedance=True)])
    a.step(20)
    ref, _, _, _ = oracle_run(s, 20)
    assert rel_l1(a.get_psi(0), ref) <= 1e-12
