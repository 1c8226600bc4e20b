"""Seeded synthetic inputs for the VFP split step.

This module is shared by the GPU path and by the tests that drive the oracle,
so it holds none of the step's arithmetic: it only builds the arrays both
sides receive (initial densities, impedance samples) and the workload
recipes.  It imports nothing else from this package.

Impedance models (Sec. II.B of arXiv:1611.05293), in normalised form with
kappa = k * sigma_z0 and every physical prefactor absorbed into the
caller's current scale S:

* free space:  Z(kappa) = Gamma(2/3)/3^(1/3) * (sqrt(3)/2 + i/2) * kappa^(1/3)
* parallel plates (full gap g, bending radius R):
      Z(kappa; P) = 4 pi^2 2^(1/3) P kappa^(-1/3)
                    * sum_p [Ai'(u_p) Ci'(u_p) + u_p Ai(u_p) Ci(u_p)],
      Ci = Ai - i Bi,  u_p = pi^2 (2p+1)^2 2^(-2/3) P^2 kappa^(-4/3),
  with P = R^(1/3) sigma_z0^(2/3) / g.  A shielding parameter
  Pi = sigma_z0 R^(1/2) / g^(3/2) maps to P = Pi^(2/3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy import special

# Gamma(2/3)/3^(1/3): free-space CSR constant
_FS = special.gamma(2.0 / 3.0) / 3.0 ** (1.0 / 3.0)
_U_ASYM = 100.0   # beyond this Airy argument the parallel-plate term uses its asymptote


def free_space_impedance(kappa) -> np.ndarray:
    kappa = np.asarray(kappa, dtype=np.float64)
    mag = _FS * np.cbrt(np.maximum(kappa, 0.0))
    return mag * (math.sqrt(3.0) / 2.0) + 1j * mag * 0.5


def _pp_terms(u: np.ndarray) -> np.ndarray:
    """Ai'(u)Ci'(u) + u Ai(u)Ci(u) for u > 0, from exponentially scaled Airy
    functions so that the products Ai*Bi neither overflow nor cancel."""
    eai, eaip, ebi, ebip = special.airye(u)
    zeta2 = np.exp(-(4.0 / 3.0) * u ** 1.5)         # e^{-2 zeta}
    re = (eaip * eaip + u * eai * eai) * zeta2
    im = -(eaip * ebip + u * eai * ebi)
    return re + 1j * im


def parallel_plate_impedance(kappa, P: float) -> np.ndarray:
    """Normalised parallel-plate CSR impedance at wavenumbers kappa >= 0."""
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    out = np.zeros(kappa.shape, dtype=np.complex128)
    for idx, kap in np.ndenumerate(kappa):
        if kap <= 0.0:
            continue
        A = math.pi ** 2 * 2.0 ** (-2.0 / 3.0) * P * P * kap ** (-4.0 / 3.0)
        # u_p = A (2p+1)^2; explicit terms while u_p <= _U_ASYM
        p_star = 0
        if A <= _U_ASYM:
            p_star = int(math.floor((math.sqrt(_U_ASYM / A) - 1.0) / 2.0)) + 1
        s = 0.0 + 0.0j
        if p_star > 0:
            u = A * (2.0 * np.arange(p_star) + 1.0) ** 2
            s = np.sum(_pp_terms(u))
        # tail: Im term -> -(3/(16 pi)) u^{-5/2}; Re is exponentially small.
        # sum_{p>=p*} (2p+1)^{-5} = 2^{-5} zeta(5, p* + 1/2)
        tail = -(3.0 / (16.0 * math.pi)) * A ** (-2.5) * special.zeta(5.0, p_star + 0.5) / 32.0
        s = s + 1j * tail
        out[idx] = 4.0 * math.pi ** 2 * 2.0 ** (1.0 / 3.0) * P * kap ** (-1.0 / 3.0) * s
    return out


def impedance_samples(n: int, padding: int, q_min: float, q_max: float,
                      model: str = "parallel_plate", Pi: float = 1.0):
    """Z_k at kappa_k = 2 pi k / (M dq), k = 0..M/2, M = padding * n.
    Returns (z_re, z_im) as float64 arrays of M/2 + 1 values; Z_0 = 0."""
    M = padding * n
    dq = (q_max - q_min) / (n - 1)
    kappa = 2.0 * math.pi * np.arange(M // 2 + 1) / (M * dq)
    if model == "parallel_plate":
        z = parallel_plate_impedance(kappa, Pi ** (2.0 / 3.0))
    elif model == "free_space":
        z = free_space_impedance(kappa)
    else:
        raise ValueError(f"unknown impedance model {model!r}")
    z[0] = 0.0
    return np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)


def gaussian_psi(n: int, q_min: float, q_max: float, p_min: float, p_max: float,
                 sigma_q: float = 1.0, sigma_p: float = 1.0, noise: float = 0.0,
                 seed: Optional[int] = None, q0: float = 0.0, p0: float = 0.0) -> np.ndarray:
    """Gaussian density on the node grid, plus additive uniform noise
    noise * max(G) * U[0,1) from numpy's PCG64 stream ``seed``, scaled so
    that dq*dp*sum(psi) = 1.  Shape (n, n), index [i (q), j (p)]."""
    q = np.linspace(q_min, q_max, n)
    p = np.linspace(p_min, p_max, n)
    g = np.exp(-0.5 * ((q[:, None] - q0) / sigma_q) ** 2 - 0.5 * ((p[None, :] - p0) / sigma_p) ** 2)
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        g = g + noise * g.max() * rng.random((n, n))
    dq = (q_max - q_min) / (n - 1)
    dp = (p_max - p_min) / (n - 1)
    return np.ascontiguousarray(g / (dq * dp * g.sum()))


def quantize16(psi: np.ndarray) -> np.ndarray:
    """Round a density to 16-bit grey levels of its maximum (emulates a start
    pattern read from a 16-bit image)."""
    m = psi.max()
    return np.round(psi / m * 65535.0) / 65535.0 * m


# ---------------------------------------------------------------------------
# Workload recipes.  Sizes follow the paper's studied ranges: grids around
# 256 points per axis, 500-4000 steps per synchrotron period, Gaussian
# starts, and a current scan over many simulations.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Sim:
    n: int
    q_min: float
    q_max: float
    p_min: float
    p_max: float
    steps_per_period: int
    beta: float
    interp: int
    z_scale: float = 0.0
    Pi: Optional[float] = None          # None: zero current
    model: str = "parallel_plate"
    padding: int = 2
    noise: float = 0.0
    seed: Optional[int] = None
    sigma0: float = 1.0
    periods: float = 1.0
    clamp: int = 0
    renormalize: int = 1
    rotation: int = 0                   # 0 standard, 1 Manhattan

    @property
    def nsteps(self) -> int:
        return int(round(self.periods * self.steps_per_period))

    def psi0(self) -> np.ndarray:
        return gaussian_psi(self.n, self.q_min, self.q_max, self.p_min, self.p_max,
                            self.sigma0, self.sigma0, self.noise, self.seed)

    def impedance(self):
        if self.Pi is None or self.z_scale == 0.0:
            return None, None
        return impedance_samples(self.n, self.padding, self.q_min, self.q_max,
                                 self.model, self.Pi)


def config(k: int) -> List[Sim]:
    """The five synthetic workloads (1: equilibrium parity case, 2: single
    simulation below threshold, 3: long unstable run, 4: 64-simulation scan,
    5: uneven 200-simulation scan)."""
    if k == 1:
        return [Sim(64, -6, 6, -6, 6, 500, 1e-3, 3, periods=1.0)]
    if k == 2:
        return [Sim(256, -8, 8, -8, 8, 1000, 1e-3, 4, z_scale=0.3, Pi=1.0,
                    noise=1e-4, seed=2, periods=20.0)]
    if k == 3:
        return [Sim(512, -8, 8, -8, 8, 2000, 5e-4, 4, z_scale=1.5, Pi=0.5,
                    noise=1e-4, seed=3, periods=200.0)]
    if k == 4:
        sims = []
        for i in range(64):
            sims.append(Sim(256, -8, 8, -8, 8, 1000, 1e-3, 4,
                            z_scale=0.1 * 20.0 ** (i / 63.0), Pi=(0.5, 1.0, 2.0)[i % 3],
                            noise=1e-4, seed=4000 + i, periods=50.0))
        return sims
    if k == 5:
        rng = np.random.default_rng(5)
        sizes = [128] * 80 + [256] * 60 + [512] * 40 + [1024] * 20
        S = rng.uniform(0.1, 2.5, len(sizes))
        Pi = rng.uniform(0.3, 3.0, len(sizes))
        sims = []
        for i, n in enumerate(sizes):
            sims.append(Sim(n, -8, 8, -8, 8, 500 * n // 128, 1e-3, 4,
                            z_scale=float(S[i]), Pi=float(Pi[i]), noise=1e-4,
                            seed=5000 + i, periods=10.0))
        return sims
    raise ValueError(f"no workload {k}")
