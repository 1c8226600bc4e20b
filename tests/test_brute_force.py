"""Brute force on tiny grids: the whole step assembled as explicit matrices
from the definitions, computed by a different route than the oracle.

* interpolation weights: solved from the Vandermonde system that defines
  Lagrange interpolation (reproduce 1, t, ..., t^(K-1) on the stencil),
  not from the product formula;
* damping/diffusion: the first-derivative stencil is obtained by
  differentiating the cubic through the four nodes, the second derivative
  by differentiating the quadratic through three;
* wake: Eq. "wakepotential" as an O(n*M) discrete Fourier sum of the
  profile spectrum times Z (no wake table, no Toeplitz sum).
The composed operator is applied to random inputs and compared with the
oracle's step to 1e-13.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleParams


def weights(K, t):
    offs = np.arange(K) - (K - 1) // 2
    A = np.vander(offs.astype(float), K, increasing=True).T     # A[d, k] = o_k^d
    return np.linalg.solve(A, t ** np.arange(K))


def interp_matrix_1d(n, K, r):
    """row vector mapping a length-n signal to its value at coordinate r"""
    row = np.zeros(n)
    m = math.floor(r)
    l = weights(K, r - m)
    for k, o in enumerate(np.arange(K) - (K - 1) // 2):
        if 0 <= m + o < n:
            row[m + o] += l[k]
    return row


def rotation_matrix(n, lo, hi, steps, K):
    d = (hi - lo) / (n - 1)
    th = 2 * math.pi / steps
    c, s = math.cos(th), math.sin(th)
    R = np.zeros((n * n, n * n))
    for i in range(n):
        for j in range(n):
            q, p = lo + i * d, lo + j * d
            rx = (q * c - p * s - lo) / d
            ry = (q * s + p * c - lo) / d
            R[i * n + j] = np.outer(interp_matrix_1d(n, K, rx), interp_matrix_1d(n, K, ry)).ravel()
    return R


def kick_matrix(n, K, shifts):
    Km = np.zeros((n * n, n * n))
    for i in range(n):
        for j in range(n):
            Km[i * n + j, i * n:(i + 1) * n] = interp_matrix_1d(n, K, j + shifts[i])
    return Km


def fp_matrix(n, lo, hi, bt):
    d = (hi - lo) / (n - 1)
    pj = lo + d * np.arange(n)
    offs4 = np.array([-1, 0, 1, 2], float)
    d1 = [np.polyval(np.polyder(np.polyfit(offs4, np.eye(4)[k], 3)), 0.0) for k in range(4)]
    offs3 = np.array([-1, 0, 1], float)
    d2 = [np.polyval(np.polyder(np.polyfit(offs3, np.eye(3)[k], 2), 2), 0.0) for k in range(3)]
    F1 = np.eye(n)
    for j in range(n):
        for k, o in enumerate((-1, 0, 1, 2)):
            if 0 <= j + o < n:
                F1[j, j + o] += bt * d1[k] * pj[j + o] / d
        for k, o in enumerate((-1, 0, 1)):
            if 0 <= j + o < n:
                F1[j, j + o] += bt * d2[k] / d ** 2
    return np.kron(np.eye(n), F1)


def wake_dft(rho, zr, zi, S):
    n = rho.size
    M = 2 * (zr.size - 1)
    zc = np.concatenate([zr + 1j * zi, (zr - 1j * zi)[1:-1][::-1]])
    zc[0] = zr[0]
    zc[M // 2] = zr[M // 2]
    k = np.arange(M)
    rt = np.array([np.sum(rho * np.exp(-2j * math.pi * kk * np.arange(n) / M)) for kk in k])
    V = np.array([np.sum(zc * rt * np.exp(2j * math.pi * k * i / M)) / M for i in range(n)])
    assert np.max(np.abs(V.imag)) < 1e-12
    return S * V.real


@pytest.mark.parametrize("K", [3, 4])
@pytest.mark.parametrize("current", [False, True])
def test_step_operator_16x16(K, current):
    n, lo, hi, steps, beta, S, pad = 16, -4.0, 4.0, 37, 0.03, 0.8, 2
    rng = np.random.default_rng(100 + K + 2 * current)
    psi = rng.random((n, n)) + 0.1
    d = (hi - lo) / (n - 1)
    Q0 = 1.7
    th = 2 * math.pi / steps
    zr = rng.normal(size=pad * n // 2 + 1) if current else np.zeros(pad * n // 2 + 1)
    zi = rng.normal(size=pad * n // 2 + 1) if current else np.zeros(pad * n // 2 + 1)
    rho = d * psi.sum(axis=1)
    V = wake_dft(rho, zr, zi, S) if current else np.zeros(n)
    R = rotation_matrix(n, lo, hi, steps, K)
    Km = kick_matrix(n, K, V * th / d)
    F = fp_matrix(n, lo, hi, beta * th)
    out = (F @ Km @ R @ psi.ravel()).reshape(n, n)
    out *= Q0 / (d * d * out.sum())
    p = OracleParams(n=n, q_min=lo, q_max=hi, p_min=lo, p_max=hi, steps_per_period=steps,
                     beta=beta, interp=K, padding=pad, z_scale=S)
    w = oracle.wake_kernel(zr, zi) if current else None
    got = oracle.step(p, w, psi, Q0)
    assert np.max(np.abs(got - out)) < 1e-13 * np.abs(out).max()
    if current:
        assert np.max(np.abs(V)) * th / d > 0.05          # the kick moved something


def test_manhattan_rotation_16x16():
    """Manhattan rotation: a drift pulled along q from q - dtheta*p, then an
    RF kick pulled along p from p + dtheta*q (two 1-D interpolations)."""
    n, lo, hi, steps, K = 16, -4.0, 4.0, 23, 4
    d = (hi - lo) / (n - 1)
    th = 2 * math.pi / steps
    rng = np.random.default_rng(7)
    psi = rng.random((n, n))
    Dm = np.zeros((n * n, n * n))
    for i in range(n):
        for j in range(n):
            row = interp_matrix_1d(n, K, (lo + i * d - th * (lo + j * d) - lo) / d)
            for a in range(n):
                Dm[i * n + j, a * n + j] = row[a]
    Km = np.zeros((n * n, n * n))
    for i in range(n):
        for j in range(n):
            Km[i * n + j, i * n:(i + 1) * n] = interp_matrix_1d(n, K, (lo + j * d + th * (lo + i * d) - lo) / d)
    exp = (Km @ Dm @ psi.ravel()).reshape(n, n)
    p = OracleParams(n=n, q_min=lo, q_max=hi, p_min=lo, p_max=hi, steps_per_period=steps, interp=K,
                     rotation=1)
    got = oracle.rotate_manhattan(p, psi)
    assert np.max(np.abs(got - exp)) < 1e-13
