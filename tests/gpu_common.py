"""Shared helpers of the GPU parity tests: run the same seeded inputs through
the oracle and through the library, and compare."""
import numpy as np

import oracle
from oracle import OracleParams
from paper_1611_05293_amd import inputs


def rel_l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum() / np.abs(np.asarray(b)).sum())


def oracle_params(sim: inputs.Sim) -> OracleParams:
    return OracleParams.from_recipe(sim)


def oracle_run(sim: inputs.Sim, nsteps: int, psi0=None, every: int = 0):
    """Final density, records and the wake table of the oracle for a recipe."""
    p = oracle_params(sim)
    zr, zi = sim.impedance()
    w = None if zr is None else oracle.wake_kernel(zr, zi, sim.padding * sim.n)
    psi = sim.psi0() if psi0 is None else psi0
    d = (sim.q_max - sim.q_min) / (sim.n - 1) * (sim.p_max - sim.p_min) / (sim.n - 1)
    Q0 = d * psi.sum()
    out, rec = oracle.run(p, w, psi, nsteps, Q0, every)
    return out, rec, w, p


def small_sim(n=48, K=4, steps=97, beta=2e-3, S=0.8, Pi=0.7, clamp=0, rotation=0, seed=7,
              lo=-6.0, hi=6.0, noise=1e-3, sigma0=1.2, model="parallel_plate", renormalize=1):
    return inputs.Sim(n, lo, hi, lo, hi, steps, beta, K, z_scale=S, Pi=Pi, model=model, noise=noise,
                      seed=seed, sigma0=sigma0, clamp=clamp, rotation=rotation, renormalize=renormalize)
