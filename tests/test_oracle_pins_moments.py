"""Pins of the oracle's Manhattan rotation and of its moments against closed
forms that do not depend on the oracle's code.

Manhattan rotation (Sec. III.B): a drift that pulls along q from q - dtheta*p
followed by an RF kick that pulls along p from p + dtheta*q.  Each pass is a
1-D interpolation by a shift that is constant along the interpolated line.
Lagrange interpolation with K >= 3 nodes reproduces polynomials of degree
<= 2, so on a density that vanishes near the edges such a shift moves the
line's mean by exactly the shift and keeps its mass and its variance.  The
first and second moments of the whole density therefore follow the forward
map (q, p) -> (q + dtheta p, p - dtheta (q + dtheta p)) exactly (to
rounding): the centroid as x -> M x and the covariance as C -> M C M^T with
M = [[1, h], [-h, 1 - h^2]], h = dtheta.  A drift or kick of the wrong sign,
or the two passes in the other order, gives a different M.

Moments (Sec. IV.A reports bunch length and energy spread): for a sampled
Gaussian whose tails vanish inside the grid, the discrete sums equal the
integrals up to terms of order exp(-2 pi^2 sigma^2 / h^2) (Poisson summation),
far below rounding here, so <q>, <p>, sigma_q, sigma_p and the charge of an
off-centre, correlated Gaussian equal their closed forms."""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleParams


def correlated_gauss(n, lo, hi, q0, p0, sq, sp, r, amp=1.0):
    """amp * exp(-x^T C^-1 x / 2), C = [[sq^2, r sq sp], [r sq sp, sp^2]]."""
    q = np.linspace(lo, hi, n)[:, None] - q0
    p = np.linspace(lo, hi, n)[None, :] - p0
    C = np.array([[sq * sq, r * sq * sp], [r * sq * sp, sp * sp]])
    Ci = np.linalg.inv(C)
    return amp * np.exp(-0.5 * (Ci[0, 0] * q * q + 2 * Ci[0, 1] * q * p + Ci[1, 1] * p * p)), C


def raw_moments(n, lo, hi, psi):
    """Mass, centroid and covariance of a density on the node grid, summed
    directly in numpy (independent of the oracle)."""
    x = np.linspace(lo, hi, n)
    q, p = x[:, None], x[None, :]
    m = psi.sum()
    mq, mp = (q * psi).sum() / m, (p * psi).sum() / m
    cqq = ((q - mq) ** 2 * psi).sum() / m
    cpp = ((p - mp) ** 2 * psi).sum() / m
    cqp = ((q - mq) * (p - mp) * psi).sum() / m
    return m, np.array([mq, mp]), np.array([[cqq, cqp], [cqp, cpp]])


@pytest.mark.parametrize("K", [3, 4])
def test_manhattan_moves_moments_by_the_symplectic_euler_map(K):
    n, lo, hi, steps = 96, -8.0, 8.0, 60
    h = 2 * math.pi / steps
    psi, _ = correlated_gauss(n, lo, hi, 0.7, -0.4, 0.9, 0.8, 0.3)
    p = OracleParams(n=n, q_min=lo, q_max=hi, p_min=lo, p_max=hi, steps_per_period=steps, interp=K,
                     rotation=1)
    M = np.array([[1.0, h], [-h, 1.0 - h * h]])
    m0, c, C = raw_moments(n, lo, hi, psi)
    for _ in range(12):
        psi = oracle.rotate_manhattan(p, psi)
        m, c_got, C_got = raw_moments(n, lo, hi, psi)
        c, C = M @ c, M @ C @ M.T
        assert abs(m - m0) < 1e-12 * m0
        assert np.max(np.abs(c_got - c)) < 1e-12
        assert np.max(np.abs(C_got - C)) < 1e-11
    # the centroid has turned by 12 steps of ~h: far from where it started
    assert np.linalg.norm(c - np.array([0.7, -0.4])) > 0.5


def test_manhattan_sense_and_order_are_distinguished():
    """The maps a flipped drift, a flipped kick or the swapped order would
    produce differ from the oracle's result by far more than rounding."""
    n, lo, hi, steps, K = 96, -8.0, 8.0, 60, 4
    h = 2 * math.pi / steps
    psi, _ = correlated_gauss(n, lo, hi, 0.7, -0.4, 0.9, 0.8, 0.3)
    p = OracleParams(n=n, q_min=lo, q_max=hi, p_min=lo, p_max=hi, steps_per_period=steps, interp=K,
                     rotation=1)
    _, c0, _ = raw_moments(n, lo, hi, psi)
    _, c1, _ = raw_moments(n, lo, hi, oracle.rotate_manhattan(p, psi))
    wrong = {
        "drift sign": np.array([[1.0, -h], [-h, 1.0 + h * h]]),
        "kick sign": np.array([[1.0, h], [h, 1.0 + h * h]]),
        "kick first": np.array([[1.0 - h * h, h], [-h, 1.0]]),
    }
    for name, W in wrong.items():
        assert np.max(np.abs(W @ c0 - c1)) > 1e-3, name


def test_manhattan_invariant_ellipse_is_tilted():
    """The one-step map preserves q^2 + p^2 + h q p (up to the factor of the
    exact discrete invariant), so a full period of Manhattan steps returns a
    centred Gaussian elongated along the line q = -p by a relative amount of
    order h/2: the tilt the paper describes as a jitter of the bunch length."""
    steps = 40
    h = 2 * math.pi / steps
    M = np.array([[1.0, h], [-h, 1.0 - h * h]])
    A = np.array([[1.0, h / 2], [h / 2, 1.0]])
    # M^T A M = A: the quadratic form of A is invariant
    assert np.max(np.abs(M.T @ A @ M - A)) < 1e-14
    n, lo, hi, K = 96, -8.0, 8.0, 4
    psi, _ = correlated_gauss(n, lo, hi, 0.0, 0.0, 1.0, 1.0, 0.0)
    p = OracleParams(n=n, q_min=lo, q_max=hi, p_min=lo, p_max=hi, steps_per_period=steps, interp=K,
                     rotation=1)
    for _ in range(steps // 4):
        psi = oracle.rotate_manhattan(p, psi)
    _, _, C = raw_moments(n, lo, hi, psi)
    # after a quarter period the round Gaussian has been sheared: its
    # correlation is of order h/2, negative (elongated along q = -p)
    corr = C[0, 1] / math.sqrt(C[0, 0] * C[1, 1])
    assert -h < corr < -h / 8


@pytest.mark.parametrize("q0,p0,sq,sp,r", [(0.7, -0.4, 0.9, 0.8, 0.3), (-1.3, 0.9, 0.6, 0.8, -0.55),
                                           (0.0, 0.0, 1.0, 1.0, 0.0)])
def test_moments_of_an_offcentre_correlated_gaussian(q0, p0, sq, sp, r):
    n, lo, hi = 128, -8.0, 8.0
    amp = 2.5
    psi, C = correlated_gauss(n, lo, hi, q0, p0, sq, sp, r, amp)
    p = OracleParams(n=n, q_min=lo, q_max=hi, p_min=lo, p_max=hi)
    Q, mq, sgq, mp, sgp = oracle.moments(p, psi)
    # charge: integral of amp*exp(...) = amp * 2 pi sqrt(det C)
    assert abs(Q - amp * 2 * math.pi * math.sqrt(np.linalg.det(C))) < 1e-12 * Q
    assert abs(mq - q0) < 1e-12
    assert abs(mp - p0) < 1e-12
    assert abs(sgq - sq) < 1e-12
    assert abs(sgp - sp) < 1e-12


def test_moments_do_not_mix_the_axes():
    """A density narrow in q and wide in p (and off-centre in opposite
    directions) reports each axis's own values."""
    n, lo, hi = 128, -8.0, 8.0
    psi, _ = correlated_gauss(n, lo, hi, 1.5, -2.0, 0.5, 0.7, 0.0)
    p = OracleParams(n=n, q_min=lo, q_max=hi, p_min=lo, p_max=hi)
    _, mq, sgq, mp, sgp = oracle.moments(p, psi)
    assert (round(mq, 9), round(sgq, 9), round(mp, 9), round(sgp, 9)) == (1.5, 0.5, -2.0, 0.7)
