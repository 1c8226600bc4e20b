"""Each precision form's wake on its own (Sec. II.B, Eq. "wakepotential"):
the stored state is read back, the library takes one step, and the wake that
step used (vfp_batch_last_wake) is compared element by element with the
oracle's FP64 Toeplitz sum of that same state, against a bound derived from
the form's arithmetic.

With u the unit roundoff of the 16-bit type (2^-11 FP16, 2^-8 BF16), a hi/lo
pair represents x to |x - hi - lo| <= u^2 |x|, and dropping lo*lo costs
another u^2 |w||rho|: 3 u^2 per term.  The matrix cores add m terms per
accumulator in FP32 (m = 16 * ceil((2*nb - 1) / 4) for nb = ceil(n/16)
block diagonals dealt to four waves), plus the FP32 roundings of w and rho
before the split: (m + 2) 2^-24.  The vector-ALU FP32 wake rounds w and rho
to FP32 and adds blocks of 32 fused products: (32 + 2) 2^-24.  Each bound
is relative to sum_j |w_(i-j)| |rho_j|, which the CSR wake's oscillating
kernel makes much larger than |V_i|; the final cast of V to FP32 adds
2^-24 |V_i|, and FP16 subnormal lo parts an absolute n 2^-37 max|w| max|rho|.
"""
import numpy as np
import pytest

import oracle
from paper_1611_05293_amd import inputs, vfp
from gpu_common import oracle_params

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def coeff(precision, n):
    nb = (n + 15) // 16
    m = 16 * -(-(2 * nb - 1) // 4)
    if precision == "fp32":
        return (32 + 2) * U32
    u = 2.0 ** -11 if precision == "fp16" else 2.0 ** -8
    return 3 * u * u + (m + 2) * U32


def wake_sims():
    return [inputs.Sim(256, -8, 8, -8, 8, 1000, 1e-3, 4, z_scale=0.3, Pi=1.0, noise=1e-4, seed=2),
            inputs.Sim(1024, -8, 8, -8, 8, 4000, 1e-3, 4, z_scale=2.0, Pi=0.4, noise=1e-4, seed=9),
            inputs.Sim(128, -8, 8, -8, 8, 500, 1e-3, 4, z_scale=2.4, Pi=2.5, noise=1e-4, seed=7)]


@pytest.mark.parametrize("staged", [1, 2])
@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
def test_wake_of_each_form_within_its_bound(precision, staged):
    sims = wake_sims()
    b = vfp.Batch([vfp.sim_kwargs(s, precision=precision) for s in sims])
    b.set_tuning(0, True, staged)
    for step in (1, 2):      # fused tick: step 1 takes the first wake launch, step 2 the tick's own wake tiles
        states = [b.get_raw(i) for i in range(len(sims))]
        b.step(1)
        for i, s in enumerate(sims):
            raw, sfac = states[i]
            p = oracle_params(s)
            zr, zi = s.impedance()
            M = s.padding * s.n
            w = oracle.wake_kernel(zr, zi, M)
            rho = oracle.profile(p, sfac * raw.astype(np.float64))
            Vo = oracle.wake(p, w, rho)
            Vg = b.last_wake(i)
            idx = (np.arange(s.n)[:, None] - np.arange(s.n)[None, :]) % M
            absconv = s.z_scale * (np.abs(w[idx]) * np.abs(rho)[None, :]).sum(axis=1)
            bound = coeff(precision, s.n) * absconv + U32 * np.abs(Vo)
            if precision == "fp16":
                bound += s.z_scale * s.n * 2.0 ** -37 * np.abs(w).max() * np.abs(rho).max()
            err = np.abs(Vg - Vo)
            ratio = (err / bound).max()
            print(f"{precision} staged {staged} step {step} n={s.n}: max|dV|/max|V| {err.max() / np.abs(Vo).max():.2e}, "
                  f"max err/bound {ratio:.3f}, cancellation sum|w||rho|/|V| {absconv.max() / np.abs(Vo).max():.1f}")
            assert ratio <= 1.0
    b.close()
