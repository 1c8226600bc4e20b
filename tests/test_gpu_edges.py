"""Edge cases of the GPU path against the oracle: the largest grid the
boundary accepts (4096^2, every arithmetic form), the smallest and ragged
grids in the FP32-storage forms, zero-step calls, a batch whose every
simulation has retired, and densities the storage type cannot hold."""
import numpy as np
import pytest

from paper_1611_05293_amd import inputs, vfp
from gpu_common import oracle_run, rel_l1, small_sim

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-5, "fp16": 1e-5}


@pytest.fixture(scope="module")
def max_grid():
    # 4096^2 on [-8, 8]^2: 16000 steps per period keeps the corner displacement
    # at 1.1 cells, as in the scan recipes
    sim = inputs.Sim(4096, -8, 8, -8, 8, 16000, 1e-3, 4, z_scale=1.0, Pi=1.0, noise=1e-4, seed=41)
    ref, _, _, _ = oracle_run(sim, 2)
    return sim, ref


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_max_grid_4096(max_grid, precision):
    sim, ref = max_grid
    b = vfp.Batch([vfp.sim_kwargs(sim, precision=precision, device_impedance=True)])
    b.step(2)
    err = rel_l1(b.get_psi(0), ref)
    print(f"4096^2 {precision} 2 steps rel-L1 {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
@pytest.mark.parametrize("n", [16, 17, 37, 130])
def test_small_and_ragged_grids(n, precision):
    """n = 16 (smallest), odd n and n not a multiple of 4 (the generic FP32
    kernel), n = 130 (two 64-column units with a ragged second)."""
    sim = small_sim(n=n, steps=40 + 2 * n, S=1.0, Pi=0.8, seed=n)
    ref, _, _, _ = oracle_run(sim, 15)
    b = vfp.Batch([vfp.sim_kwargs(sim, precision=precision)])
    b.step(15)
    assert rel_l1(b.get_psi(0), ref) <= TOL[precision]


def test_zero_steps_change_nothing():
    sims = [small_sim(n=32, seed=1), small_sim(n=48, seed=2)]
    b = vfp.Batch([vfp.sim_kwargs(s, precision="fp32") for s in sims])
    before = [b.get_psi(i) for i in range(2)]
    b.step(0)
    assert [b.steps_done(i) for i in range(2)] == [0, 0]
    for i in range(2):
        assert np.array_equal(b.get_psi(i), before[i])


def test_fully_retired_batch_is_frozen():
    sims = [small_sim(n=32, seed=1), small_sim(n=48, seed=2)]
    b = vfp.Batch([vfp.sim_kwargs(s, precision="fp64", max_steps=c) for s, c in zip(sims, (3, 5))])
    b.step(5)
    frozen = [b.get_psi(i) for i in range(2)]
    b.step(7)
    assert [b.steps_done(i) for i in range(2)] == [3, 5]
    for i, s in enumerate(sims):
        assert np.array_equal(b.get_psi(i), frozen[i])
        ref, _, _, _ = oracle_run(s, (3, 5)[i])
        assert rel_l1(frozen[i], ref) <= 1e-12


@pytest.mark.parametrize("precision,ok", [("fp64", True), ("fp32", False), ("fp16", False)])
def test_density_beyond_binary32(precision, ok):
    g = vfp.Sim(n=32, q_range=(-5, 5), precision=precision)
    big = np.ones((32, 32))
    big[3, 4] = 1e39
    if ok:
        g.set_psi(big)
        assert np.array_equal(g.get_psi(), big)
    else:
        with pytest.raises(vfp.VfpError, match="binary32") as e:
            g.set_psi(big)
        assert e.value.code == vfp.VFP_EINVAL


@pytest.mark.parametrize("renormalize", [0, 1])
def test_zero_charge_is_rejected(renormalize):
    """The moments are charge-weighted and the renormalisation divides by
    the charge: a density without positive charge is refused, and the state
    it would have replaced is kept."""
    g = vfp.Sim(n=32, q_range=(-5, 5), precision="fp32", renormalize=renormalize)
    g.step(2)
    before = g.get_psi()
    for bad in (np.zeros((32, 32)), -np.ones((32, 32))):
        with pytest.raises(vfp.VfpError, match="positive, finite charge"):
            g.set_psi(bad)
    assert np.array_equal(g.get_psi(), before) and g.steps_done() == 2
