import numpy as np

from paper_1611_05293_amd import analysis


def test_bursting_spectrum_finds_the_oscillation():
    steps_per_period, every = 500, 10
    t = np.arange(2000) * every / steps_per_period          # in synchrotron periods
    P = 1.0 + 0.01 * np.sin(2 * np.pi * 2.0 * t)             # oscillation at 2 f_s
    rec = np.zeros((len(t), 7))
    rec[:, 6] = P
    f, s = analysis.bursting_spectrum(rec, every, steps_per_period)
    assert abs(f[np.argmax(s)] - 2.0) < f[1] - f[0]
    f2, m = analysis.spectrogram([rec, rec], every, steps_per_period)
    assert m.shape == (2, len(f)) and np.array_equal(f, f2)
