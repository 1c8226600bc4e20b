"""The allocation-free impedance sampler: the same samples as the allocating
entry point, bit for bit, through the C ABI; calls that follow each other
share the static scratch (the second call here is smaller than the first, so
stale entries of the first would show)."""
import numpy as np
import pytest

from paper_1611_05293_amd import vfp


@pytest.mark.gpu
def test_noalloc_samples_equal_the_allocating_entry_point():
    cases = [(1024, 8, -8.0, 8.0, "parallel_plate", 0.5),     # 4097 samples
             (64, 2, -6.0, 7.0, "parallel_plate", 1.7),       # 65 samples, after the larger call
             (200, 3, -5.0, 5.0, "free_space", 1.0)]
    for n, pad, lo, hi, model, Pi in cases:
        print(f"noalloc impedance: n={n} padding={pad} model={model} Pi={Pi}", flush=True)
        ar, ai = vfp.impedance_samples(n, pad, lo, hi, model, Pi)
        br, bi = vfp.impedance_samples(n, pad, lo, hi, model, Pi, noalloc=True)
        assert br.shape == ar.shape == (pad * n // 2 + 1,)
        assert np.array_equal(br, ar) and np.array_equal(bi, ai)
        assert np.abs(ai).max() > 0


def test_noalloc_rejects_sizes_beyond_the_scratch():
    # validated on the host before any device call
    assert vfp.load().vfp_impedance_samples_noalloc  # exported
    with pytest.raises(vfp.VfpError, match="static scratch"):
        vfp.impedance_samples(4096, 10, -8.0, 8.0, "parallel_plate", 1.0, noalloc=True)
    with pytest.raises(vfp.VfpError, match="padding"):
        vfp.impedance_samples(64, 1, -8.0, 8.0, "parallel_plate", 1.0, noalloc=True)
