#!/usr/bin/env python3
"""Benchmark of the batched VFP step on one MI355X.

Workload (default): the uneven 200-simulation parameter scan -- 80 x 128^2,
60 x 256^2, 40 x 512^2 and 20 x 1024^2 grids, cubic interpolation, steps per
period 500..4000 (scaled with the grid), parallel-plate CSR impedance with
random current and shielding, FP32 density with the FP16 hi/lo matrix-core
wake and FP64 renormalisation.  One "step" is one tick: every simulation
advances by one of its own time steps.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "phase-space cell-updates/s (N²·steps·sims/s), batched vs plain, at stated L1 err"
HBM_PEAK_GBS = 8000.0
# the step kernel of each tick form: 0 the generic kernel (also FP64 and fixed
# point), 1 the LDS-staged step after its own wake launch (split tick), 2 the
# one-launch tick (the wake tiles of the current state, then the LDS-staged
# step units, in the same launch)
STEP_KERNEL = {0: "vfp::step_kernel", 1: "vfp::step32c_kernel", 2: "vfp::tick32_kernel"}
TICK_FORM = {0: "a wake launch (FP32 storage) and a step launch of the generic kernel per group",
             1: "a wake launch then one fused step launch per stream group (split tick)",
             2: "one launch per stream group: the wake tiles, then the fused step units (one-launch tick)"}
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "step_kernel_hbm_traffic_scan200_fp16.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    from paper_1611_05293_amd import inputs
    if name == "scan200":
        return inputs.config(5), "fp16", (
            "uneven scan: 200 sims (80x128^2, 60x256^2, 40x512^2, 20x1024^2), K=4, "
            "steps/period 500-4000, parallel-plate CSR, S~U[0.1,2.5], Pi~U[0.3,3]")
    if name == "scan64":
        return inputs.config(4), "bf16", (
            "scan: 64 sims at 256^2, K=4, 1000 steps/period, S log-spaced 0.1-2.0, Pi in {0.5,1,2}")
    if name == "single256":
        return inputs.config(2), "fp32", (
            "single simulation 256^2, K=4, 1000 steps/period, parallel-plate CSR Pi=1, S=0.3")
    if name == "run512":
        return inputs.config(3), "fp32", (
            "single simulation 512^2, K=4, 2000 steps/period, parallel-plate CSR Pi=0.5, S=1.5")
    if name == "equilibrium64":
        return inputs.config(1), "fp64", (
            "single simulation 64^2, K=3, 500 steps/period, zero current, FP64")
    raise SystemExit(f"unknown workload {name}")


def _cpu_model():
    """Model name with family/model/stepping from /proc/cpuinfo (first CPU)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (x.strip() for x in line.split(":", 1))
                info.setdefault(k, v)
            elif info:
                break
    except OSError:
        return "host CPU"
    name = info.get("model name", "host CPU")
    return (f"{name} (family {info.get('cpu family', '?')}, model {info.get('model', '?')}, "
            f"stepping {info.get('stepping', '?')}, {info.get('cpu MHz', '?')} MHz)")


def cpu_baseline(sims, seconds):
    """The FP64 oracle on this host's cores over a bounded sample of the same
    workload: one simulation per 20 of each grid size (the workload's size
    ratio), advanced over a prefix of ticks one simulation after another with
    the oracle's OpenMP loops over columns.  Timed twice: with all the
    threads OpenMP gives the process and with one thread."""
    import oracle
    by_n = {}
    for i, s in enumerate(sims):
        by_n.setdefault(s.n, []).append(i)
    ns = sorted(by_n)
    counts = {n: max(1, len(by_n[n]) // 20) for n in ns}       # 4:3:2:1 for the scan
    pick = [i for n in ns for i in by_n[n][:counts[n]]]
    prep = []
    for i in pick:
        s = sims[i]
        p = oracle.OracleParams.from_recipe(s)
        zr, zi = s.impedance()
        w = None if zr is None else oracle.wake_kernel(zr, zi, s.padding * s.n)
        psi = s.psi0()
        d = (s.q_max - s.q_min) / (s.n - 1) * (s.p_max - s.p_min) / (s.n - 1)
        prep.append((p, w, psi, d * psi.sum(), s.n))
    cells_tick = sum(x[4] ** 2 for x in prep)

    def rate(budget):
        t0 = time.perf_counter()
        for p, w, psi, Q0, _ in prep:
            oracle.run(p, w, psi, 1, Q0)
        one = time.perf_counter() - t0
        ticks = max(1, int(budget / max(one, 1e-6)))
        t0 = time.perf_counter()
        for p, w, psi, Q0, _ in prep:
            oracle.run(p, w, psi, ticks, Q0)
        dt = time.perf_counter() - t0
        return cells_tick * ticks / dt, ticks, dt

    def rate_many(budget):
        """The same simulations advanced together by the oracle's OpenMP loop
        over simulations (one thread per simulation)."""
        t0 = time.perf_counter()
        oracle.run_many([x[0] for x in prep], [x[1] for x in prep], [x[2].copy() for x in prep],
                        [1] * len(prep), [x[3] for x in prep])
        one = time.perf_counter() - t0
        ticks = max(1, int(budget / max(one, 1e-6)))
        t0 = time.perf_counter()
        oracle.run_many([x[0] for x in prep], [x[1] for x in prep], [x[2].copy() for x in prep],
                        [ticks] * len(prep), [x[3] for x in prep])
        dt = time.perf_counter() - t0
        return cells_tick * ticks / dt, ticks, dt

    threads = oracle.threads()
    v_all, t_all, dt_all = rate(0.4 * seconds)
    v_sims, t_sims, dt_sims = rate_many(0.3 * seconds)
    oracle.set_threads(1)
    try:
        v_one, t_one, dt_one = rate(0.3 * seconds)
    finally:
        oracle.set_threads(threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count()
    best, how = (v_all, "over columns") if v_all >= v_sims else (v_sims, "over simulations")
    return {
        "value": best, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
        "value_columns": v_all, "value_simulations": v_sims, "value_1core": v_one,
        "nproc": os.cpu_count(), "cpus_allowed": affinity, "cpu_model": _cpu_model(),
        "sample": f"{len(pick)} sims ({'+'.join(f'{counts[n]}x{n}^2' for n in ns)}), FP64; all {threads} OpenMP "
                  f"threads: a prefix of {t_all} ticks ({dt_all:.1f} s) with the loops over columns and {t_sims} "
                  f"ticks ({dt_sims:.1f} s) with the loop over simulations (value: the faster, {how}); "
                  f"1 thread: {t_one} ticks ({dt_one:.1f} s)",
    }


def parity(states, sims, nsteps):
    """Largest rel-L1 of the device states {i: psi} against the oracle after nsteps."""
    import oracle
    worst = 0.0
    for i, g in states.items():
        s = sims[i]
        p = oracle.OracleParams.from_recipe(s)
        zr, zi = s.impedance()
        w = None if zr is None else oracle.wake_kernel(zr, zi, s.padding * s.n)
        psi = s.psi0()
        d = (s.q_max - s.q_min) / (s.n - 1) * (s.p_max - s.p_min) / (s.n - 1)
        ref, _ = oracle.run(p, w, psi, nsteps, d * psi.sum())
        worst = max(worst, float(np.abs(g - ref).sum() / np.abs(ref).sum()))
    return worst


def timed(b, stream, cells_tick, es, steps):
    """K ticks between events on the batch's stream (graph replays prepared at
    create, single launches for a remainder shorter than a graph), then the
    per-kernel averages from a pass with events around every launch."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # untimed settling: the first few hundred ticks after the batch is made run
    # up to a quarter slower (clocks and caches still ramping), so the GPU runs
    # ticks for a quarter of a second first, whatever the warm-up count
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < 0.25:
        b.step(64)
        torch.cuda.synchronize()
    # untimed re-warm of two graph lengths right before the timed region, not
    # waited for: the GPU is still busy with it when the start event is
    # reached, so the host's launch latency of the timed ticks does not enter
    # the timed region
    b.step(32)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kt_ticks = 300
    b.kernel_timing(True)
    b.step(kt_ticks)
    kt = b.kernel_times()
    b.kernel_timing(False)
    step_ms = kt["step_ms"] / max(kt["step_launches"], 1)
    wake_ms = kt["wake_ms"] / max(kt["wake_launches"], 1) if kt["wake_launches"] else 0.0
    nbytes = cells_tick * 2 * es
    return {"ms": ms, "value": cells_tick * steps / (ms / 1e3), "step_us": step_ms * 1e3, "wake_us": wake_ms * 1e3,
            "bytes": nbytes, "achieved": nbytes / (step_ms / 1e3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="scan200",
                    choices=["scan200", "scan64", "single256", "run512", "equilibrium64"])
    ap.add_argument("--precision", default=None,
                    help="fp32 | bf16 | fp16 | fp64 | fixed (44 fractional bits) (default: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-aux", action="store_true", help="skip the timings of the device-side analysis calls")
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32 and Manhattan forms")
    ap.add_argument("--staged", type=int, default=None,
                    help="FP32-storage kernel and tick form: 0 generic, 1 staged split tick, 2 staged one-launch tick")
    ap.add_argument("--streams", type=int, default=3, choices=[1, 2, 3, 4], help="stream groups of the batch")
    ap.add_argument("--cells", type=int, default=0, help="cells per work unit (0: built-in)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy 5 times (scale of the HBM byte counters)")
    ap.add_argument("--counter-summary", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the step kernel's HBM bytes per launch from four rocprofv3 --pmc output "
                         "folders (no GPU needed) and exit")
    ap.add_argument("--layout-for-summary", type=int, default=1)
    args = ap.parse_args()
    if args.counter_summary:
        from paper_1611_05293_amd import inputs, profiles
        sims = inputs.config(5)
        alg = 8 * sum(s_.n * s_.n for s_ in sims)
        d = profiles.summarize(*args.counter_summary, kernel_prefix=STEP_KERNEL[args.layout_for_summary],
                               copy_bytes=512 << 20, algorithmic_bytes=alg)
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (a batch's simulations "
                                   "are independent and shard across GPUs by simulation, with no exchange per tick)"}))
        sys.exit(2)

    import torch                          # device memory and the stream only
    from paper_1611_05293_amd import vfp

    if args.copy_calibration:
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        c = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 512 << 20, "launches": 5}), flush=True)
        return

    sims, prec, desc = workload(args.workload)
    prec = args.precision or prec
    cells_tick = sum(s.n * s.n for s in sims)
    es = 8 if prec in ("fp64", "fixed") else 4     # bytes per stored cell (fixed point: int64)
    log(f"workload {args.workload}: {len(sims)} sims, {cells_tick} cells per tick, precision {prec}")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = vfp.Batch([vfp.sim_kwargs(s, precision=prec) for s in sims], stream=stream, torch_workspace=True)
    log("created batch")
    if args.staged is not None or args.cells:
        b.set_tuning(args.cells, True, b.get_tuning()[2] if args.staged is None else args.staged)
    tuned = None
    if args.autotune:
        tuned, layout = b.autotune(ticks=10)
        log(f"autotuned: {tuned} cells per unit, kernel layout {layout}")
    b.set_streams(args.streams)
    cells_unit, _, args.staged = b.get_tuning()
    b.step(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} ticks done")
    # states of one simulation per grid size after the warm-up, compared with the
    # oracle after the timed passes (the GPU does not idle during the comparison)
    states = {}
    if not args.no_parity and args.warmup > 0:
        for i, s in enumerate(sims):
            if all(sims[j].n != s.n for j in states):
                states[i] = b.get_psi(i)

    # timed region: K ticks (graph replays prepared at create; a remainder of
    # single ticks when K is not a multiple of the graph length)
    r = timed(b, stream, cells_tick, es, args.steps)
    value, ms = r["value"], r["ms"]
    log(f"timed {args.steps} ticks: {ms:.2f} ms -> {value:.4e} cell-updates/s; step kernel "
        f"{r['step_us']:.1f} us, wake kernel {r['wake_us']:.1f} us -> {r['achieved']:.0f} GB/s algorithmic")
    achieved, step_avg_ms, wake_avg_ms, bytes_launch = r["achieved"], r["step_us"] / 1e3, r["wake_us"] / 1e3, r["bytes"]
    err = None
    if states:
        err = parity(states, sims, args.warmup)
        log(f"parity after {args.warmup} ticks, one sim per grid size: max rel-L1 {err:.3e}")

    # the same workload in the other forms (same steps; no parity pass)
    forms = {}
    if not args.no_forms:
        # the 8-byte forms (FP64, 44-bit fixed point) run the generic kernel and fewer ticks
        other = 2 if args.staged == 1 else 1
        for name, fprec, rot, extra, stg in (
                ("one_launch_tick" if other == 2 else "split_tick", prec, 0, {}, other),
                ("fp32", "fp32", 0, {}, args.staged), ("manhattan_" + prec, prec, 1, {}, args.staged),
                ("fp64", "fp64", 0, {}, 0), ("fixed44", "fixed", 0, {"fix_bits": 44}, 0)):
            if (name.startswith("fp32") and prec == "fp32") or (name == "fp64" and prec == "fp64"):
                continue
            if prec in ("fp64", "fixed") and name in ("one_launch_tick", "split_tick"):
                continue
            wide = fprec in ("fp64", "fixed")
            fsteps = min(args.steps, 50) if wide else args.steps
            fb = vfp.Batch([vfp.sim_kwargs(s_, precision=fprec, rotation=rot, **extra) for s_ in sims],
                           stream=stream, torch_workspace=True)
            fb.set_tuning(0 if wide else cells_unit, True, stg)
            fb.set_streams(args.streams)
            fb.step(min(args.warmup, 5 if wide else 20))
            fr = timed(fb, stream, cells_tick, 8 if wide else 4, fsteps)
            forms[name] = {"value": fr["value"], "ms_per_step": fr["ms"] / fsteps, "steps": fsteps,
                           "tick": TICK_FORM[stg], "step_kernel": STEP_KERNEL[stg],
                           "step_kernel_us": fr["step_us"], "wake_kernel_us": fr["wake_us"],
                           "hbm_frac": fr["achieved"] / HBM_PEAK_GBS}
            log(f"form {name}: {fr['value']:.4e} cell-updates/s, step kernel {fr['step_us']:.1f} us "
                f"({fr['achieved']:.0f} GB/s)")
            fb.close()
            del fb
            torch.cuda.empty_cache()

    plain = None
    if not args.no_plain:
        # the plain per-simulation FP32 form: the same simulations one after another
        ps = args.plain_steps
        t_ms = 0.0
        for i, s in enumerate(sims):
            g = vfp.Sim(stream=stream, **vfp.sim_kwargs(s, precision="fp32"))
            torch.cuda.synchronize()
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            g.step(ps)
            a1.record(stream)
            torch.cuda.synchronize()
            t_ms += a0.elapsed_time(a1)
            g.close()
        pv = cells_tick * ps / (t_ms / 1e3)
        plain = {"value": pv, "unit": "cell-updates/s", "form": "plain per-simulation FP32, sims back-to-back",
                 "steps_per_sim": ps}
        log(f"plain form: {pv:.4e} cell-updates/s; batched speed-up {value / pv:.1f}x")

    # the device-side analysis and set-up calls of a scan, timed per call on the
    # host clock (synchronous calls: launch, device work and the copy of the result)
    aux = None
    with_z = [s_ for s_ in sims if s_.Pi is not None and s_.z_scale != 0.0]
    if not args.no_aux and with_z:
        import time as _time
        nmax = max(s_.n for s_ in with_z)
        big = [s_ for s_ in with_z if s_.n == nmax][:2]
        if len(big) == 1:
            big = big * 2
        ab = vfp.Batch([vfp.sim_kwargs(s_, precision=prec) for s_ in big], stream=stream, torch_workspace=True)
        ab.step(5)
        torch.cuda.synchronize()

        def per_call(fn, reps):
            fn()
            t0 = _time.perf_counter()
            for _ in range(reps):
                fn()
            return (_time.perf_counter() - t0) / reps * 1e6

        n1 = big[0]
        aux = {
            "unit": "us per call (host clock, synchronous)",
            "grid": f"{nmax}^2, padding {big[0].padding}",
            "impedance_samples_parallel_plates": per_call(
                lambda: vfp.impedance_samples(n1.n, n1.padding, n1.q_min, n1.q_max, "parallel_plate", n1.Pi), 5),
            "csr_spectrum": per_call(lambda: ab.csr_spectrum(0), 10),
            "haissinski_200_iterations": per_call(lambda: ab.haissinski(1, 200, 0.5), 3),
            "seed_from_other_simulation": per_call(lambda: ab.seed(1, 0), 10),
        }
        ab.close()
        del ab
        torch.cuda.empty_cache()
        log("aux calls (us): " + ", ".join(f"{k} {v:.0f}" for k, v in aux.items() if isinstance(v, float)))

    cpu = None
    if not args.no_cpu:
        log("timing the oracle on the host")
        cpu = cpu_baseline(sims, args.cpu_seconds)
        log(f"oracle: {cpu['value']:.3e} cell-updates/s on {cpu['cores']} threads (columns {cpu['value_columns']:.3e}, "
            f"simulations {cpu['value_simulations']:.3e}), {cpu['value_1core']:.3e} on 1 "
            f"({cpu['cpu_model']}, nproc {cpu['nproc']})")

    # HBM bytes per launch from the stored counter summary, only while it was
    # taken on the current kernel sources (and only for the workload it covers)
    kname = STEP_KERNEL[args.staged if prec not in ("fp64", "fixed") else 0]
    traffic = None
    if args.workload == "scan200" and prec == "fp16":
        from paper_1611_05293_amd import profiles
        traffic = profiles.traffic_for_current_sources(TRAFFIC_FILE, kname)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fixed": "int64"}.get(prec, "f32"),
        "data": "synthetic",
        "config": {"workload": desc,
                   "form": ("batched; a tick is, in each stream group, one step launch with the wake slice inside"
                            if prec in ("fp64", "fixed") else f"batched; a tick is {TICK_FORM[args.staged]}")
                           + "; ticks replayed from one hipGraph of 16 ticks per stream group, prepared at create",
                   "wake": {"fp16": "FP16 hi/lo MFMA", "bf16": "BF16 hi/lo MFMA",
                            "fp32": "FP32 VALU", "fp64": "FP64 VALU", "fixed": "FP64 VALU"}[prec],
                   "sims": len(sims), "cells_per_tick": cells_tick,
                   "cells_per_unit": cells_unit, "kernel_layout": args.staged, "stream_groups": args.streams},
        "parity": None if err is None else {"max_rel_l1_vs_fp64_oracle": err, "after_steps": args.warmup,
                                            "sims_checked": "one per grid size"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "avg_launch_us": step_avg_ms * 1e3,
                     "bytes_per_launch": bytes_launch, "wake_kernel_avg_us": wake_avg_ms * 1e3},
        "forms": forms,
        "plain": plain,
        "batched_speedup": None if plain is None else value / plain["value"],
        "aux": aux,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
