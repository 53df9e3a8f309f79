"""Autotuner for the schedule knobs of libfock (fock_tuning).

It times one fock_apply per candidate schedule on the device with the
library's own per-kernel events and keeps the fastest.  Candidates, for the
paths the plan uses (read from the kernels a default apply launches):

  whole-pair path   one workgroup per output with fused_split in {1, 2, 3, 4}
                    partner slices, and unordered-pair rounds (fused_rounds)
  three-pass path   pair symmetry with the pair-buffer budget tbuf_mb in
                    {128 .. 16384} MiB (which sets the block size; 128 and
                    256 MiB keep a batch's pair buffer within the 256 MB
                    Infinity Cache), and the ordered schedule over the joint
                    grid tbuf_mb x acc_workgroups (output block size)

Candidates whose plans come out identical (same counters and workspace on
the host) are timed once.  Results are cached as JSON keyed by the device
name, precision and the instance shapes, in $FOCK_TUNE_CACHE or
~/.cache/fock_tune.json.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import fock

KNOBS = ("acc_workgroups", "tbuf_mb", "fused_split", "no_fused", "no_pair_symmetry", "fused_rounds")
FUSED_SPLITS = (1, 2, 3, 4)
SYM_TBUF_MB = (128, 256, 512, 1024, 4096, 16384)
ORDERED_TBUF_MB = (256, 1024, 4096, 16384)
ORDERED_ACC_WORKGROUPS = (512, 2048, 8192)


def candidates(kinds):
    """Candidate knob sets for the kernel kinds a default apply launched."""
    out = [{}]
    if "fused" in kinds:
        out += [{"fused_split": sp} for sp in FUSED_SPLITS] + [{"fused_rounds": 1}]
    if kinds & {"plane", "pencil", "accumulate"}:
        out += [{"tbuf_mb": tb} for tb in SYM_TBUF_MB]
        out += [{"no_pair_symmetry": 1, "tbuf_mb": tb, "acc_workgroups": aw}
                for tb in ORDERED_TBUF_MB for aw in ORDERED_ACC_WORKGROUPS]
    return out


def plan_signature(instances, precision, tuning):
    """Counters and workspace size of the plan these knobs give (host only):
    equal signatures mean the same schedule."""
    import ctypes

    keep = []
    descs = (fock.FockDesc * len(instances))()
    for i, inst in enumerate(instances):
        descs[i] = fock.make_desc(fock._get(inst, "lattice"), fock._get(inst, "grid"), fock._get(inst, "kfrac"),
                                  fock._get(inst, "kweight", None), fock._get(inst, "nbands"), None,
                                  fock._get(inst, "mu", 0.106), fock._get(inst, "kpairs", None), keep)
    L = fock.lib()
    h = ctypes.c_void_p()
    tn = fock.FockTuning(**{k: int(v) for k, v in tuning.items()})
    fock.check(L.fock_plan_tuned(descs, len(instances), fock.PRECISIONS[precision], None, ctypes.byref(tn),
                                 ctypes.byref(h)))
    try:
        size = ctypes.c_size_t()
        a, b, c, e = (ctypes.c_int64() for _ in range(4))
        fock.check(L.fock_workspace_size(h, ctypes.byref(size)))
        fock.check(L.fock_plan_stats(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(e)))
        return (a.value, b.value, e.value, size.value)
    finally:
        L.fock_destroy(h)


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
    seen = {plan_signature(instances, precision, best)}
    for t in candidates(kinds)[1:]:
        sig = plan_signature(instances, precision, t)
        if sig in seen:
            continue
        seen.add(sig)
        ms, _ = run(t)
        if ms < best_ms:
            best_ms, best = ms, t
    record = {"tuning": best, "ms": best_ms, "trials": trials}
    if use_cache:
        entries = load_cache()
        entries[key] = record
        save_cache(entries)
    return dict(best), record
