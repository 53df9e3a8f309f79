"""Autotuner for the schedule knobs of libfock (fock_tuning).

It times one fock_apply per candidate on the device with the library's own
per-kernel events and keeps the fastest, searching one knob at a time:

  whole-pair path   fused_split in {1, 2, 3, 4}       (partner slices per output)
  three-pass path   acc_workgroups in {512 .. 8192}    (output block size)
                    tbuf_mb in {1024, 4096, 16384}     (pairs per batch)

Only knobs of the paths the plan actually uses are searched (read from the
kernels a default apply launches).  Results are cached as JSON keyed by the
device name, precision and the instance shapes, in $FOCK_TUNE_CACHE or
~/.cache/fock_tune.json.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import fock

KNOBS = ("acc_workgroups", "tbuf_mb", "fused_split", "no_fused")
FUSED_SPLITS = (1, 2, 3, 4)
ACC_WORKGROUPS = (512, 1024, 2048, 4096, 8192)
TBUF_MB = (1024, 4096, 16384)


def cache_path():
    return os.environ.get("FOCK_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "fock_tune.json"))


def shape_key(instances, precision, device_name):
    shapes = []
    for inst in instances:
        g = tuple(int(x) for x in fock._get(inst, "grid"))
        nk = int(np.asarray(fock._get(inst, "kfrac")).reshape(-1, 3).shape[0])
        shapes.append((g, nk, int(fock._get(inst, "nbands"))))
    return json.dumps({"device": device_name, "precision": precision, "shapes": sorted(shapes)}, sort_keys=True)


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(entries, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_apply(instances, precision, device, tuning, psi, occ):
    """(apply ms, kernel kinds launched) for one tuned plan: one warm-up apply,
    then one apply timed by the library's per-kernel events."""
    import torch

    plan = fock.Plan(instances, precision=precision, device=device, tuning=tuning)
    try:
        out = [torch.empty_like(p) for p in psi]
        plan.fock_apply(psi, occ, out=out)
        torch.cuda.synchronize()
        plan.profile(True)
        plan.fock_apply(psi, occ, out=out)
        torch.cuda.synchronize()
        kern = plan.profile_read()
        plan.profile(False)
    finally:
        plan.close()
    ms = sum(v[0] for v in kern.values())
    kinds = {k for k, v in kern.items() if v[1] > 0}
    return ms, kinds


def autotune(instances, psi, occ, precision="c64", device=None, use_cache=True, log=None):
    """Pick fock_tuning knobs for these instances by measurement.

    psi, occ: lists of device tensors (the real inputs, or any data of the
    same shapes).  Returns (tuning dict, record dict)."""
    import torch

    device = torch.device(device or "cuda:0")
    dev_name = torch.cuda.get_device_name(device)
    key = shape_key(instances, precision, dev_name)
    entries = load_cache() if use_cache else {}
    if key in entries:
        return dict(entries[key]["tuning"]), entries[key]
    trials = []

    def run(t):
        ms, kinds = _time_apply(instances, precision, device, t, psi, occ)
        trials.append({"tuning": dict(t), "ms": ms})
        if log:
            log(f"autotune {t}: {ms:.3f} ms")
        return ms, kinds

    best = {}
    best_ms, kinds = run(best)
    if "fused" in kinds:
        for sp in FUSED_SPLITS:
            t = dict(best, fused_split=sp)
            ms, _ = run(t)
            if ms < best_ms:
                best_ms, best = ms, t
    if kinds & {"plane", "pencil", "accumulate"}:
        for aw in ACC_WORKGROUPS:
            t = dict(best, acc_workgroups=aw)
            ms, _ = run(t)
            if ms < best_ms:
                best_ms, best = ms, t
        for tb in TBUF_MB:
            t = dict(best, tbuf_mb=tb)
            ms, _ = run(t)
            if ms < best_ms:
                best_ms, best = ms, t
    record = {"tuning": best, "ms": best_ms, "trials": trials}
    if use_cache:
        entries = load_cache()
        entries[key] = record
        save_cache(entries)
    return dict(best), record
