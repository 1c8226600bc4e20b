"""Post-processing of recorded time series (not part of the step).

The paper Fourier-transforms the CSR power P(t) of each run to obtain the
'bursting' spectrum and stacks the spectra of a current scan into a
spectrogram (Sec. IV.C, Fig. spectrogram)."""
from __future__ import annotations

from typing import Sequence

import numpy as np


def bursting_spectrum(records: np.ndarray, every: int, steps_per_period: int, first: float = 0.5):
    """Magnitude spectrum of P(t) from the record rows {step, Q, <q>, sq, <p>,
    sp, P} taken every `every` steps; the first fraction `first` of the series
    is dropped (transient).  Returns (frequencies in units of f_s, |FFT|)."""
    P = np.asarray(records)[:, 6]
    P = P[int(first * len(P)):]
    dt = every / steps_per_period                 # sampling interval in synchrotron periods
    spec = np.abs(np.fft.rfft(P - P.mean()))
    return np.fft.rfftfreq(len(P), dt), spec


def spectrogram(records: Sequence[np.ndarray], every: int, steps_per_period: int, first: float = 0.5):
    """Stack the bursting spectra of several runs (e.g. a current scan) into a
    matrix [run, frequency]; all runs must share the sampling."""
    rows = [bursting_spectrum(r, every, steps_per_period, first) for r in records]
    f = rows[0][0]
    return f, np.stack([s for _, s in rows])
