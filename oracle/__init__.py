"""Plain FP64 CPU oracle for the VFP split step (arXiv:1611.05293).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1611_05293_amd``) and never imports it.

The arithmetic lives in ``vfp_oracle.c`` (plain loops, FP64, and 128-bit
integer sums for the fixed-point form; ``-O2 -ffp-contract=off``); this
module only builds and marshals.
"""
from .oracle import (  # noqa: F401
    OracleParams, build, load, threads, set_threads, lagrange_weights, wake_kernel, profile, charge,
    wake, rotate, rotate_manhattan, kick, fokker_planck, moments, csr_power, csr_spectrum,
    step, run, run_many, haissinski, fix_quantize, fix_charge, fix_step, fix_run,
)
