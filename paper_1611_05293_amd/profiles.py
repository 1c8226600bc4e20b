"""HBM byte counters of the step kernel, from rocprofv3 counter runs.

`summarize` reads the counter_collection CSVs of four runs (FETCH_SIZE and
WRITE_SIZE over the benchmark, the same two over a plain device copy of known
size) and returns the per-launch HBM bytes of one kernel, each counter scaled
by the factor that makes it read the copy's true size.  The result records a
hash of the kernel sources it was taken on; `traffic_for_current_sources`
returns it only while the sources are unchanged, so a stale figure is never
reported for a changed kernel.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("vfp_kernels.hpp", "vfp_step32c.hpp", "vfp.hip")]


def sources_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_means(run_dir: str, counter: str) -> dict:
    """Mean counter value (KiB) per dispatch, by kernel name."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    acc = {}
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, kernel_prefix, copy_bytes,
              algorithmic_bytes=None) -> dict:
    def pick(d, prefix):
        keys = [k for k in d if prefix in k]
        if not keys:
            raise KeyError(f"no kernel matching {prefix!r}: {sorted(d)}")
        return keys[0], d[keys[0]]

    name, fetch = pick(_counter_means(fetch_dir, "FETCH_SIZE"), kernel_prefix)
    _, write = pick(_counter_means(write_dir, "WRITE_SIZE"), kernel_prefix)
    _, cf = pick(_counter_means(copy_fetch_dir, "FETCH_SIZE"), "copyBuffer")
    _, cw = pick(_counter_means(copy_write_dir, "WRITE_SIZE"), "copyBuffer")
    ff, fw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    out = {
        "kernel": name,
        "fetch_kib_raw": fetch, "write_kib_raw": write,
        "copy_bytes": copy_bytes, "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
        "fetch_scale": ff, "write_scale": fw,
        "hbm_bytes_per_launch": fetch * 1024.0 * ff + write * 1024.0 * fw,
        "sources_sha256": sources_hash(),
    }
    if algorithmic_bytes:
        out["algorithmic_bytes_per_launch"] = algorithmic_bytes
        out["ratio_to_algorithmic"] = out["hbm_bytes_per_launch"] / algorithmic_bytes
    return out


def traffic_for_current_sources(path: str, kernel_prefix: str):
    """HBM bytes per launch from a stored summary, or None when the summary is
    missing, is for another kernel, or was taken on other sources."""
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if kernel_prefix not in d.get("kernel", "") or d.get("sources_sha256") != sources_hash():
        return None
    return d.get("hbm_bytes_per_launch")
