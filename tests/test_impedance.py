"""Pins of the impedance sampler (Sec. II.B) against the limits the paper
states: parallel plates tend to free space as the gap grows and at high
frequency, and both impedances vanish at zero frequency."""
import os

import numpy as np

from paper_1611_05293_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    vals = {}
    for line in open(os.path.join(GOLDEN, "free_space_impedance.txt")):
        if line.startswith("#"):
            continue
        k, v = line.split()
        vals[k] = float(v)
    return vals["re"] + 1j * vals["im"]


def test_free_space_constant():
    z = inputs.free_space_impedance(np.array([1.0, 8.0, 27.0]))
    assert np.allclose(z / np.array([1.0, 2.0, 3.0]), _golden(), rtol=1e-10)


def test_parallel_plate_tends_to_free_space_for_wide_gap():
    kap = np.array([1.0, 4.0])
    z = inputs.parallel_plate_impedance(kap, 0.1)
    assert np.allclose(z / np.cbrt(kap), _golden(), rtol=3e-4)
    # at fixed kappa the shielding correction shrinks as the gap widens
    errs = [abs(inputs.parallel_plate_impedance([0.5], P)[0] / np.cbrt(0.5) - _golden())
            for P in (0.5, 0.2, 0.1, 0.05)]
    assert all(a > b for a, b in zip(errs, errs[1:])) and errs[-1] < 2e-3


def test_parallel_plate_tends_to_free_space_at_high_frequency():
    kap = np.array([64.0, 200.0])
    z = inputs.parallel_plate_impedance(kap, 1.0)
    assert np.allclose(z / np.cbrt(kap), _golden(), rtol=2e-4)


def test_parallel_plate_vanishes_at_low_frequency():
    z = inputs.parallel_plate_impedance(np.array([0.5, 0.1, 0.01]), 1.0)
    assert abs(z[0]) < 5e-3 and abs(z[1]) < abs(z[0]) and abs(z[2]) < abs(z[1])
    assert abs(z[0].real) < 1e-20                    # real part exponentially small
    zs = inputs.impedance_samples(64, 2, -8, 8)
    assert zs[0][0] == 0.0 and zs[1][0] == 0.0


def test_airy_tail_continuity():
    """Near the switch from explicit Airy terms to the asymptotic tail the
    sampled impedance is smooth in kappa."""
    kap = np.linspace(0.2, 3.0, 400)
    z = inputs.parallel_plate_impedance(kap, 1.0)
    d2 = np.abs(np.diff(z, 2))
    assert d2.max() < 50 * np.median(d2) + 1e-12


def test_inputs_seeded_and_normalised():
    a = inputs.gaussian_psi(64, -8, 8, -8, 8, noise=1e-4, seed=4)
    b = inputs.gaussian_psi(64, -8, 8, -8, 8, noise=1e-4, seed=4)
    c = inputs.gaussian_psi(64, -8, 8, -8, 8, noise=1e-4, seed=5)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    d = 16 / 63
    assert abs(d * d * a.sum() - 1.0) < 1e-14
    cfg5 = inputs.config(5)
    assert len(cfg5) == 200 and sum(s.n ** 2 for s in cfg5) == 80 * 128 ** 2 + 60 * 256 ** 2 + 40 * 512 ** 2 + 20 * 1024 ** 2
