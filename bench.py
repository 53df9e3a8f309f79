"""Benchmark of the exchange hot path on one MI355X.

Workload: the alpha-boron-shaped cell (rhombohedral a = 9.56 bohr, 58.0 deg),
32^3 grid, uniform 4x4x4 k-mesh with all 64 k' per k (343 distinct
transfers), 18 bands, screened kernel mu = 0.106 bohr^-1; seeded random
orthonormal orbitals (12 Ha cutoff).  1,327,104 ordered band pairs.

A step is one pass of the whole path over that input: fock_apply_energy
(co-density, FFTs, kernel multiply, accumulate, the band overlap M, and E_x
from the per-pair energies of the same transforms) and fock_energy_backward
(dE_x/dpsi*, co-densities recomputed).  `value` counts ordered band pairs
per step divided by the step time; the FP32 (complex64) path is the
headline, the FP64 path is reported beside it.

Per-kernel times come from HIP events the library records on its own
stream around every launch, through the timed steps.  The roofline entry
rates the unit that dominates the step (the whole-pair kernel, or the three
passes of a three-pass batch together) by the compulsory 4 s N bytes per
ordered pair, and quotes a measured device-to-device copy rate beside the
8 TB/s peak.  The default run also times the largest workload, the
beta-boron-shaped 72^3 cell (1 warm-up + 3 steps, `beta_boron_fp32`).  The
CPU baseline is the FP64 oracle timed on a bounded sample of pairs of the
same workload on this host, with one thread and with one single-threaded
process per usable core; `host` records the machine.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--beta-steps B]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# copy-calibrated HBM traffic of the dominant FP32 kernel, written by
# paper_1111_0716_amd.profile_summary from rocprofv3 counter runs of this script
TRAFFIC_FILES = {"alpha": "profiles/{kind}_alpha_boron_32cubed_fp32_traffic.md",
                 "beta": "profiles/{kind}_beta_boron_72cubed_fp32_traffic.md",
                 "diff": "profiles/{kind}_diff_64cubed_fp32_traffic.md"}
WORKLOADS = {
    "2": "alpha-boron-shaped rhombohedral cell a=9.56 bohr alpha=58.0 deg, 32^3 grid, 4x4x4 k-mesh "
         "(all 64 k' per k), 18 bands f=1, mu=0.106",
    "3": "beta-boron-shaped rhombohedral cell a=19.16 bohr alpha=65.2 deg, 72^3 grid, 2x2x2 k-mesh, "
         "160 bands (8 fractional), mu=0.106",
    "5": "beta-boron-shaped cell a=19.16 bohr alpha=65.2 deg, 64^3 grid, Gamma, 128 bands, mu=0.106",
}
# Vector ALU peak without packed FP32 math: 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz.
VALU_PEAK_TFLOPS = {"c64": 78.6, "c128": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


THREE_PASS = ("plane", "pencil", "accumulate")
THREE_PASS_UNIT = "three-pass apply (plane + pencil + accumulate of one batch)"


def kernel_model(grid, s):
    """Algorithmic flops and bytes per band pair.

    apply (whole-pair kernel, or the three passes of a batch together):
        F = 10 N log2 N + 16 N,  B = 4 s N  (read u_m and u_n, read and write
        the output once per ordered pair: the compulsory operand traffic)
    energy (whole-pair energy kernel):
        F = 5 N log2 N + 9 N,    B = 2 s N  (read u_m and u_n)
    The passes of the three-pass path split the apply's flops
        plane       F = 5 N log2(N2 N3) + 6 N
        pencil      F = 10 N log2 N1 + 2 N
        accumulate  F = 5 N log2(N2 N3) + 8 N
    but carry no byte model of their own: what one pass moves depends on how
    much of its operands the caches serve, so per-pass bytes are only quoted
    from the hardware counters.  s is the complex size."""
    n1, n2, n3 = grid
    n = n1 * n2 * n3
    l23 = math.log2(n2 * n3)
    l1 = math.log2(n1)
    return {
        "fused": dict(flops=10 * n * math.log2(n) + 16 * n, bytes=4 * s * n),
        "energy_fused": dict(flops=5 * n * math.log2(n) + 9 * n, bytes=2 * s * n),
        "plane": dict(flops=5 * n * l23 + 6 * n),
        "pencil": dict(flops=10 * n * l1 + 2 * n),
        "accumulate": dict(flops=5 * n * l23 + 8 * n),
        "energy_plane": dict(flops=5 * n * l23 + 6 * n),
        "energy_pencil": dict(flops=5 * n * l1 + 3 * n),
    }


def _units(stats):
    """Band pairs a profiled step runs through each kernel kind (the bench
    step is one apply with energy and one backward: apply kinds run twice).
    An apply serves every ordered pair (the whole-pair kernel and the three
    passes taken together are rated per ordered pair); with pair symmetry the
    plane and pencil passes transform each unordered pair once
    (apply_fft_pairs), while the accumulate and mirror passes still do one
    inverse transform and accumulate per ordered pair."""
    u = {k: 2 * stats["ordered_pairs"] for k in ("fused", "accumulate")}
    u.update({k: 2 * stats["apply_fft_pairs"] for k in ("plane", "pencil")})
    u.update({k: stats["energy_fft_pairs"] for k in ("energy_fused", "energy_plane", "energy_pencil")})
    return u


def dominant_apply(kern):
    """(name, total ms, launches) of what dominates the step: the whole-pair
    kernel, the three passes of the three-pass path taken together (one
    launch of each per batch), or the whole-pair energy kernel."""
    cands = []
    for k in ("fused", "energy_fused"):
        if kern.get(k, (0, 0))[1] > 0:
            cands.append((k, kern[k][0], kern[k][1]))
    if all(kern.get(k, (0, 0))[1] > 0 for k in THREE_PASS):
        cands.append((THREE_PASS_UNIT, sum(kern[k][0] for k in THREE_PASS), kern["plane"][1]))
    return max(cands, key=lambda c: c[1])


def roofline(kern, stats, grid, s, peak_tflops, traffic=None, workload=None):
    """Roofline entry of the unit with the largest share of the profiled step.
    ``traffic``: counter bytes per launch of that unit (None if not measured
    for the current sources); with ``workload`` it is read from that
    workload's committed traffic summaries instead."""
    model = kernel_model(grid, s)
    units = _units(stats)
    dom, tot_ms, launches = dominant_apply(kern)
    mk = "energy_fused" if dom == "energy_fused" else "fused"  # the three passes are one apply
    nunits = units["fused"] if dom == THREE_PASS_UNIT else units[dom]
    if workload is not None:
        traffic = unit_traffic(workload, dom, kern, nunits / launches)
    per_launch_ms = tot_ms / launches
    flops = model[mk]["flops"] * nunits / launches
    byts = model[mk]["bytes"] * nunits / launches
    tflops = flops / (per_launch_ms * 1e-3) / 1e12
    gbs = byts / (per_launch_ms * 1e-3) / 1e9
    alu_frac = tflops / peak_tflops
    hbm_frac = gbs / HBM_PEAK_GBS
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": peak_tflops, "unit": "TFLOP/s",
                "frac": round(alu_frac, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    if traffic:
        roof["traffic_gbs"] = round(traffic / (per_launch_ms * 1e-3) / 1e9, 1)
        roof["traffic_over_algorithmic"] = round(traffic / byts, 4)
    roof.update({"traffic": traffic, "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                 "copy-calibrated)", "algorithmic_bytes_per_launch": byts, "kernel": dom, "launches": launches,
                 "launch_ms": round(per_launch_ms, 4), "units_per_launch": round(nunits / launches, 1),
                 "alt": {"hbm_gbs": round(gbs, 1), "hbm_frac": round(hbm_frac, 4), "alu_tflops": round(tflops, 3),
                         "alu_frac": round(alu_frac, 4)}})
    return roof


def unit_traffic(workload, dom, kern=None, units_per_launch=None):
    """Counter bytes per launch of the dominant unit from the committed
    traffic summaries, or None.  Each summary gives bytes per unit of work
    (per ordered pair: bytes per dispatch over the ordered pairs per batch of
    the counted run), so a run whose batches are larger or smaller than the
    counted one's is scaled by its own units per launch."""
    pattern = TRAFFIC_FILES.get(workload)
    if not pattern:
        return None
    from paper_1111_0716_amd.profile_summary import read_traffic
    kinds = THREE_PASS if dom == THREE_PASS_UNIT else (dom,)
    vals = [read_traffic(os.path.join(ROOT, pattern.format(kind=k)), k, per_unit=True) for k in kinds]
    if any(v is None for v in vals) or not units_per_launch:
        return None
    return sum(vals) * units_per_launch


def kernel_rates(kern, stats, grid, s):
    """Per kernel kind of a step: time, launches and achieved algorithmic
    TFLOP/s; GB/s of the 4 s N (apply) or 2 s N (energy) model only for the
    units that do a whole apply or energy: the whole-pair kernels and the
    three passes together."""
    model = kernel_model(grid, s)
    units = _units(stats)
    out = {}
    for k, (ms, n) in kern.items():
        if n == 0 or k not in model or ms <= 0:
            continue
        sec = ms * 1e-3
        out[k] = {"ms": round(ms, 3), "launches": n, "tflops": round(model[k]["flops"] * units[k] / sec / 1e12, 3)}
        if "bytes" in model[k]:
            out[k]["gbs"] = round(model[k]["bytes"] * units[k] / sec / 1e9, 1)
    if all(kern.get(k, (0, 0))[1] > 0 for k in THREE_PASS):
        ms = sum(kern[k][0] for k in THREE_PASS)
        sec = ms * 1e-3
        out["three_pass"] = {"ms": round(ms, 3), "launches": kern["plane"][1],
                             "gbs": round(model["fused"]["bytes"] * units["fused"] / sec / 1e9, 1),
                             "tflops": round(model["fused"]["flops"] * units["fused"] / sec / 1e12, 3)}
    return out


def launch_gaps(r):
    """Device time per step outside the library's kernels: the step time
    (events around each step on the stream) minus the summed per-launch
    event spans, with the launches per step."""
    kern = r["kernels"]
    busy = sum(v[0] for v in kern.values())
    n = sum(v[1] for v in kern.values())
    idle = r["ms_per_step"] - busy
    return {"launches_per_step": n, "kernel_ms_per_step": round(busy, 3), "idle_ms_per_step": round(idle, 3),
            "idle_frac": round(idle / r["ms_per_step"], 4), "idle_us_per_launch": round(1e3 * idle / max(n, 1), 2)}


def copy_bandwidth(device, mib=1024, reps=5):
    """Device-to-device copy rate (bytes read + written per second) of `mib` MiB."""
    import torch

    src = torch.ones(mib << 20, dtype=torch.uint8, device=device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * (mib << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def run_path(inst, prec, steps, warmup, device, profile=True, breakdown=True):
    import torch

    from paper_1111_0716_amd import fock

    dt = np.complex64 if prec == "c64" else np.complex128
    psi = torch.from_numpy(np.ascontiguousarray(inst.psi.astype(dt))).to(device)
    occ = torch.from_numpy(np.ascontiguousarray(inst.occ)).to(device)
    plan = fock.Plan([inst], precision=prec, device=device)
    st = plan.stats()
    out = torch.empty_like(psi)
    grad = torch.empty_like(psi)
    m = plan.meta[0]
    gex = torch.ones(1, dtype=torch.float64, device=device)
    exbuf = torch.empty(1, dtype=torch.float64, device=device)
    scale = 2.0 * m["omega"] / m["npts"]

    def step():
        _, _, ex = plan.fock_apply_energy([psi], [occ], out=[out], vmat=True, ex=exbuf)
        plan.fock_energy_backward([psi], [occ], gex, scale, out=[grad])
        return ex

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"  warm-up step {i + 1}/{warmup} done")
    stream = torch.cuda.current_stream(device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the library's per-kernel HIP events stay on through the timed steps:
    # they are recorded on the stream the kernels run on
    plan.profile_read()
    plan.profile(profile)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    marks = [e0]
    for i in range(steps):
        ex = step()
        if i + 1 < steps:
            mk = torch.cuda.Event(enable_timing=True)
            mk.record(stream)
            marks.append(mk)
            # one host sync per step keeps progress visible; it adds only a
            # launch latency between steps
            torch.cuda.synchronize()
            if (i + 1) % 5 == 0:
                log(f"  timed step {i + 1}/{steps} done")
    e1.record(stream)
    marks.append(e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    per = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(steps))
    res = dict(ms_per_step=ms, ms_median=per[steps // 2] if steps % 2 else 0.5 * (per[steps // 2 - 1] + per[steps // 2]),
               wall_s=wall, stats=st, ex=float(ex.item()))
    if profile:
        res["kernels"] = {k: (v[0] / steps, v[1] // steps) for k, v in plan.profile_read().items()}
        plan.profile(False)
    if profile and breakdown:
        # apply-only timing (one call) for the breakdown
        plan.profile_read()  # reset
        plan.profile(True)
        plan.fock_apply([psi], [occ], out=[out], vmat=False)
        torch.cuda.synchronize()
        res["apply_kernels"] = plan.profile_read()
        plan.profile(False)
    plan.close()
    del psi, occ, out, grad
    torch.cuda.empty_cache()
    return res


def _oracle_sample(inst, seconds, outputs=None):
    """(pairs, seconds): every partner (k', m) of each output (k, n) in
    ``outputs`` (default: k = 0, all n), in order, until ``seconds`` have
    passed (checked after each partner k-point)."""
    from oracle.fock_oracle import Oracle

    psi = inst.psi.astype(np.complex128)
    o = Oracle.from_instance(inst)
    outputs = [(0, n) for n in range(inst.nbands)] if outputs is None else outputs
    npairs = 0
    t0 = time.perf_counter()
    for (k, n) in outputs:
        for kp in range(inst.nk):
            v = o.v(k, kp)
            for m in range(inst.nbands):
                o.pair(psi[k, n], psi[kp, m], v)
                npairs += 1
            if time.perf_counter() - t0 > seconds:
                return npairs, time.perf_counter() - t0
    return npairs, time.perf_counter() - t0


_SAMPLE = {}


def _oracle_worker(args):
    """One process of the all-core sample: outputs (k, n) with
    (k N_b + n) mod workers == rank, one BLAS thread."""
    rank, workers, seconds = args
    from threadpoolctl import threadpool_limits

    inst = _SAMPLE["inst"]
    outs = [(k, n) for k in range(inst.nk) for n in range(inst.nbands) if (k * inst.nbands + n) % workers == rank]
    with threadpool_limits(limits=1):
        return _oracle_sample(inst, seconds, outs)


def cpu_baseline(inst, seconds, seconds_1t=5.0, max_workers=16):
    """The FP64 oracle on a bounded sample of the workload: one process with
    one thread, then one single-threaded process per usable core (at most
    ``max_workers``), each on its own output bands, for about ``seconds``.
    Band pairs are independent and of equal cost, so the all-core rate is
    the pairs of all processes over the slowest one's time.  Runs before the
    GPU is touched (the pool forks this process)."""
    import multiprocessing

    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        p1, t1 = _oracle_sample(inst, seconds_1t)
    single = {"value": round(p1 / t1, 2), "cores": 1, "sample": f"{p1} ordered pairs (outputs k=0) in {t1:.1f} s"}
    workers = max(1, min(len(os.sched_getaffinity(0)), max_workers))
    _SAMPLE["inst"] = inst
    ctx = multiprocessing.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, [(r, workers, seconds) for r in range(workers)])
    wall = time.perf_counter() - t0
    _SAMPLE.clear()
    pairs = sum(r[0] for r in res)
    slowest = max(r[1] for r in res)
    return dict(value=round(pairs / slowest, 2), unit="ordered band pairs/s (apply + energy per pair, FP64 oracle)",
                cores=workers, kind="oracle",
                sample=f"{pairs} ordered pairs over {workers} single-threaded processes, each on its own output bands "
                       f"(every k', m per output), {slowest:.1f} s each ({wall:.1f} s wall with start-up)",
                single_thread=single)


def host_info():
    """What the numbers were measured on."""
    info = {"nproc": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            names = [l.split(":", 1)[1].strip() for l in f if l.startswith("model name")]
        info["cpu_model"] = names[0] if names else None
    except OSError:
        info["cpu_model"] = None
    try:
        with open("/opt/rocm/.info/version") as f:
            info["rocm"] = f.read().strip()
    except OSError:
        info["rocm"] = None
    try:
        import torch

        info["torch"] = torch.__version__
        info["torch_hip"] = torch.version.hip
        if torch.cuda.is_available():
            info["gpu"] = torch.cuda.get_device_name(0)
            props = torch.cuda.get_device_properties(0)
            info["gpu_arch"] = getattr(props, "gcnArchName", None)
            info["gpu_cus"] = props.multi_processor_count
            info["gpu_mem_gib"] = round(props.total_memory / 2**30, 1)
    except ImportError:
        pass
    return info


def ragged(args):
    """Uneven batch: 48 independent instances (grids 24^3-64^3, 8-96 bands,
    Gamma or 2x2x2) in one plan with autotuned schedule knobs, replayed as one
    HIP graph per call (FP32), beside one-at-a-time FP64 plans."""
    import torch

    from paper_1111_0716_amd import autotune, fock, inputs

    device = torch.device("cuda:0")
    log("generating the 48-instance uneven batch")
    insts = inputs.uneven_batch(dtype=np.complex128, workers=16)
    pairs = sum(i.ordered_pairs() for i in insts)
    stream = torch.cuda.Stream(device)
    with torch.cuda.stream(stream):
        psi = [torch.from_numpy(i.psi.astype(np.complex64)).to(device) for i in insts]
        occ = [torch.from_numpy(i.occ).to(device) for i in insts]
        tuning, rec = autotune.autotune(insts, psi, occ, precision="c64", device=device, log=log)
        plan = fock.Plan(insts, precision="c64", device=device, stream=stream, tuning=tuning)
        plan.set_graph(True)
        out = [torch.empty_like(p) for p in psi]
        ex = torch.empty(len(insts), dtype=torch.float64, device=device)

        def step():
            plan.fock_apply_energy(psi, occ, out=out, ex=ex)

        for _ in range(args.warmup):
            step()
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        plan.close()
        del psi, out
        torch.cuda.empty_cache()
    def one_at_a_time(prec):
        """Sum over instances of one apply + energy on a plan of its own (after
        one untimed call); also the energy FFT pairs of each instance."""
        dt = np.complex64 if prec == "c64" else np.complex128
        total, epairs = 0.0, []
        for inst in insts:
            p1 = fock.Plan([inst], precision=prec, device=device)
            epairs.append(p1.stats()["energy_fft_pairs"])
            ps = torch.from_numpy(inst.psi.astype(dt)).to(device)
            oc = torch.from_numpy(inst.occ).to(device)
            o = torch.empty_like(ps)
            p1.fock_apply_energy([ps], [oc], out=[o])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p1.fock_apply_energy([ps], [oc], out=[o])
            torch.cuda.synchronize()
            total += (time.perf_counter() - t0) * 1e3
            p1.close()
            del ps, o
        return total, epairs

    log("one-at-a-time FP32 plans")
    ms32, _ = one_at_a_time("c64")
    log("one-at-a-time FP64 plans")
    ms64, _ = one_at_a_time("c128")
    # algorithmic bytes of a step: 4 s N per ordered pair of the apply (the
    # FP32 plan takes E_x from the apply's own transforms in
    # fock_apply_energy, so the energy adds no bytes)
    alg = sum(8 * int(np.prod(i.grid)) * 4 * i.ordered_pairs() for i in insts)
    gbs = alg / (ms / 1e3) / 1e9
    line = {"metric": "band-pair Fock applications/s, uneven batch (48 instances), FP32 one graph vs FP64 one-at-a-time",
            "value": round(pairs / (ms / 1e3), 1), "unit": "ordered band pairs/s (apply + energy per step)",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64 (fp32 complex)",
            "data": "synthetic", "config": {"workload": "48 uneven instances", "ordered_pairs_per_step": pairs,
                                            "tuning": tuning},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "whole step (all instances, graph replay)",
                         "algorithmic_bytes_per_step": alg},
            "fp32_one_at_a_time": {"ms_per_step": round(ms32, 3), "pairs_per_s": round(pairs / (ms32 / 1e3), 1),
                                   "batched_speedup": round(ms32 / ms, 3)},
            "fp64_one_at_a_time": {"ms_per_step": round(ms64, 3), "pairs_per_s": round(pairs / (ms64 / 1e3), 1)}}
    print(json.dumps(line), flush=True)


def fft3d(args):
    """Batched 3-D DFT (fock_dft3, forward, in place) per cubic size: GPU rate
    with the data resident in HBM, beside scipy's FFT on every host core; one
    grid and a batch of about 1 GiB per size (four times the 256 MB Infinity
    Cache, so the passes stream from HBM)."""
    import scipy.fft
    import torch

    from paper_1111_0716_amd import fock, inputs

    device = torch.device("cuda:0")
    cores = os.cpu_count() or 1
    rows = []
    for L in (16, 24, 32, 48, 64, 72):
        n = L ** 3
        inst = inputs.small_instance(grid=(L, L, L), kmesh=(1, 1, 1), nbands=1, seed=(400, L))
        plan = fock.Plan([inst], precision="c64", device=device)
        batch = max(1, (1024 << 20) // (8 * n))
        x = torch.randn(batch, n, dtype=torch.complex64, device=device)
        plan.dft3(x, -1)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            plan.dft3(x, -1)
        e1.record()
        torch.cuda.synchronize()
        gpu_us = e0.elapsed_time(e1) * 1e3 / (reps * batch)
        one = x[:1].clone()
        plan.dft3(one, -1)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            plan.dft3(one, -1)
        e1.record()
        torch.cuda.synchronize()
        gpu1_us = e0.elapsed_time(e1) * 1e3 / reps
        plan.close()
        del x, one
        torch.cuda.empty_cache()
        hb = min(batch, 32)
        h = (np.random.default_rng(L).standard_normal((hb, L, L, L)) + 0j).astype(np.complex64)
        scipy.fft.fftn(h[:1], axes=(1, 2, 3), workers=cores)
        t0 = time.perf_counter()
        scipy.fft.fftn(h, axes=(1, 2, 3), workers=cores)
        cpu_us = (time.perf_counter() - t0) * 1e6 / hb
        t0 = time.perf_counter()
        scipy.fft.fftn(h[:1], axes=(1, 2, 3), workers=cores)
        cpu1_us = (time.perf_counter() - t0) * 1e6
        flops = 5.0 * n * math.log2(n)
        byts = 4.0 * 8 * n  # two passes, each reads and writes the grid
        rows.append({"grid": L, "batch": batch, "gpu_us_per_grid": round(gpu_us, 3), "gpu_us_one_grid": round(gpu1_us, 2),
                     "cpu_us_per_grid": round(cpu_us, 2), "cpu_us_one_grid": round(cpu1_us, 2),
                     "gbs": round(byts / (gpu_us * 1e-6) / 1e9, 1), "tflops": round(flops / (gpu_us * 1e-6) / 1e12, 3)})
        log(f"  {L}^3: GPU {gpu_us:.2f} us/grid (one grid {gpu1_us:.1f} us), CPU {cpu_us:.1f} us/grid")
    top = rows[-1]
    cross = next((r["grid"] for r in rows if r["gpu_us_one_grid"] < r["cpu_us_one_grid"]), None)
    line = {"metric": "batched 3-D DFT rate (complex64, forward, in place)", "value": round(1e6 / top["gpu_us_per_grid"], 1),
            "unit": f"grids/s at {top['grid']}^3", "n_gpus": 1, "steps": 5, "warmup": 1,
            "ms_per_step": round(top["gpu_us_per_grid"] * top["batch"] / 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "c64 (fp32 complex)", "data": "synthetic (normal)",
            "config": {"workload": "batched cubic 3-D DFT, 16^3-72^3, ~1 GiB per batch"},
            "roofline": {"bound": "hbm", "achieved": top["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(top["gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "dft (plane + pencil passes)", "bytes_per_grid": 4 * 8 * top["grid"] ** 3},
            "cpu_baseline": {"value": round(1e6 / top["cpu_us_per_grid"], 1), "unit": f"grids/s at {top['grid']}^3",
                             "cores": cores, "kind": "scipy.fft.fftn", "sample": "batch of up to 32 grids"},
            "sizes": rows, "single_grid_gpu_faster_from": cross}
    print(json.dumps(line), flush=True)


def pw(args):
    """V_x psi on the plane-wave sphere (fock_apply_pw) against the grid
    apply, FP32, alpha-boron workload: the cost of the sphere boundary."""
    import torch

    from paper_1111_0716_amd import fock, inputs

    device = torch.device("cuda:0")
    inst = inputs.config("2", dtype=np.complex128, workers=16).astype(np.complex64)
    g = [inputs.sphere_indices(inst.lattice, inst.kfrac[k], inst.ecut, inst.grid) for k in range(inst.nk)]
    npw = np.array([len(x) for x in g], dtype=np.int32)
    npw_max = int(npw.max())
    gidx = np.full((inst.nk, npw_max), -1, dtype=np.int32)
    n1, n2, n3 = inst.grid
    for k, x in enumerate(g):
        gidx[k, : len(x)] = ((x[:, 0] % n1) * n2 + (x[:, 1] % n2)) * n3 + (x[:, 2] % n3)
    plan = fock.Plan([inst], precision="c64", device=device)
    psi = torch.from_numpy(inst.psi).to(device)
    occ = torch.from_numpy(inst.occ).to(device)
    g_d, n_d = torch.from_numpy(gidx).to(device), torch.from_numpy(npw).to(device)
    (coef,) = plan.grid_to_pw([psi.clone()], [g_d], [n_d])
    work_u, work_v = torch.empty_like(psi), torch.empty_like(psi)
    out = torch.empty_like(coef)
    vx = torch.empty_like(psi)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms_grid = timed(lambda: plan.fock_apply([psi], [occ], out=[vx]))
    ms_pw = timed(lambda: plan.fock_apply_pw([coef], [g_d], [n_d], [occ], psi_work=[work_u], vx_work=[work_v],
                                             out=[out]))
    plan.profile(True)
    plan.fock_apply_pw([coef], [g_d], [n_d], [occ], psi_work=[work_u], vx_work=[work_v], out=[out])
    torch.cuda.synchronize()
    kern = {k: round(v[0], 3) for k, v in plan.profile_read().items() if v[1]}
    plan.profile(False)
    pairs = plan.stats()["ordered_pairs"]
    line = {"metric": "band-pair Fock applications/s on the plane-wave sphere (FP32)",
            "value": round(pairs / (ms_pw / 1e3), 1), "unit": "ordered band pairs/s (fock_apply_pw)", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": round(ms_pw, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "c64 (fp32 complex)", "data": "synthetic",
            "config": {"workload": WORKLOADS["2"] + ", coefficients on the 12 Ha sphere",
                       "npw": [int(npw.min()), int(npw.max())]},
            "grid_apply_ms": round(ms_grid, 3), "boundary_overhead": round(ms_pw / ms_grid - 1.0, 4),
            "kernels_ms": kern}
    plan.close()
    print(json.dumps(line), flush=True)


def precision(args):
    """Precision policies on the alpha-boron workload: which calls of a step
    (apply, energy, backward) run on the FP32, FP64 or mixed path, with the
    step time and the error of each result against the FP64 path (itself
    held to 1e-12 of the oracle by the parity tests)."""
    import torch

    from paper_1111_0716_amd import fock, inputs

    device = torch.device("cuda:0")
    inst = inputs.config("2", dtype=np.complex128, workers=16)
    occ = torch.from_numpy(inst.occ).to(device)
    psi = {"c64": torch.from_numpy(inst.psi.astype(np.complex64)).to(device),
           "c128": torch.from_numpy(inst.psi).to(device)}
    psi["mixed"] = psi["mixed_inv"] = psi["c128"]
    plans = {pr: fock.Plan([inst], precision=pr, device=device) for pr in ("c64", "c128", "mixed", "mixed_inv")}
    m = plans["c128"].meta[0]
    scale = 2.0 * m["omega"] / m["npts"]
    gex = torch.ones(1, dtype=torch.float64, device=device)
    policies = {"all FP64": ("c128", "c128", "c128"), "all FP32": ("c64", "c64", "c64"),
                "FP32 apply and backward, FP64 energy": ("c64", "c128", "c64"),
                "mixed in every call (FP32 co-density and forward, FP64 multiply, inverse, accumulate)":
                    ("mixed", "mixed", "mixed"),
                "the other mixed policy in every call (FP64 co-density, forward, multiply and energy; FP32 "
                "inverse and accumulate)": ("mixed_inv", "mixed_inv", "mixed_inv")}
    rows, ref = {}, None
    for name, (pa, pe, pb) in list(policies.items()):
        def step():
            (vx,), _ = plans[pa].fock_apply([psi[pa]], [occ])
            ex = plans[pe].fock_energy([psi[pe]], [occ])
            (g,) = plans[pb].fock_energy_backward([psi[pb]], [occ], gex, scale)
            return vx, ex, g
        step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            vx, ex, g = step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        vx = vx.to(torch.complex128).cpu().numpy()
        g = g.to(torch.complex128).cpu().numpy()
        ex = float(ex.item())
        if ref is None:
            ref = (vx, ex, g)
        rows[name] = {"calls": {"apply": pa, "energy": pe, "backward": pb}, "ms_per_step": round(ms, 3),
                      "ex_rel_err": abs(ex - ref[1]) / abs(ref[1]),
                      "vx_rel_err": float(np.linalg.norm(vx - ref[0]) / np.linalg.norm(ref[0])),
                      "grad_rel_err": float(np.linalg.norm(g - ref[2]) / np.linalg.norm(ref[2]))}
        log(f"  {name}: {ms:.1f} ms/step, E_x err {rows[name]['ex_rel_err']:.2e}, V_x err {rows[name]['vx_rel_err']:.2e}")
    pairs = plans["c64"].stats()["ordered_pairs"]
    best = rows["all FP32"]
    line = {"metric": "precision policies: band-pair Fock applications/s and error vs the FP64 path",
            "value": round(pairs / (best["ms_per_step"] / 1e3), 1),
            "unit": "ordered band pairs/s (all-FP32 policy; apply + energy + backward)", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "c64 / c128 per call", "data": "synthetic",
            "config": {"workload": WORKLOADS["2"]}, "policies": rows}
    for p in plans.values():
        p.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--beta-steps", type=int, default=3,
                    help="timed steps of the beta-boron 72^3 leg of the default run (0: skip it)")
    ap.add_argument("--workload", choices=["alpha", "beta", "diff", "ragged", "fft3d", "pw", "precision", "membw"],
                    default="alpha")
    ap.add_argument("--bands", type=int, default=0,
                    help="--workload beta|diff: keep only the first N bands of every k (a smaller run of the same "
                         "kernels, e.g. for counter collection); 0: all")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (the reference dispatch "
                         "that scales rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the exchange path of this library runs on a single device).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "ragged":
        return ragged(args)
    if args.workload == "fft3d":
        return fft3d(args)
    if args.workload == "pw":
        return pw(args)
    if args.workload == "precision":
        return precision(args)
    if args.workload == "membw":
        return membw(args)

    import torch

    from paper_1111_0716_amd import inputs

    device = torch.device("cuda:0")
    cfg = {"alpha": "2", "beta": "3", "diff": "5"}[args.workload]
    log(f"generating inputs: preset {cfg} ({WORKLOADS[cfg]})")
    inst = inputs.config(cfg, dtype=np.complex128, workers=16)
    if args.bands and args.workload != "alpha":
        inst = inputs.band_subset(inst, args.bands)
        log(f"  first {inst.nbands} bands of every k")
    inst32 = inst.astype(np.complex64)
    cb = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the sample's process pool forks this process
        log(f"CPU baseline: FP64 oracle, one thread for ~5 s, then every usable core for ~{args.cpu_seconds:.0f} s")
        cb = cpu_baseline(inst, args.cpu_seconds)
        log(f"  {cb['value']} pairs/s on {cb['cores']} cores ({cb['single_thread']['value']} on one)")
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device=device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes device to device")
        del src, dst
        torch.cuda.empty_cache()

    log(f"FP32 path: {args.warmup} warm-up + {args.steps} timed steps")
    r32 = run_path(inst32, "c64", args.steps, args.warmup, device)
    log(f"  {r32['ms_per_step']:.2f} ms/step")
    r64 = None
    if not args.no_fp64:
        k64 = max(1, min(args.fp64_steps, args.steps))
        w64 = min(1, args.warmup)
        log(f"FP64 path: {w64} warm-up + {k64} timed steps")
        r64 = run_path(inst, "c128", k64, w64, device)
        log(f"  {r64['ms_per_step']:.2f} ms/step")

    pairs = r32["stats"]["ordered_pairs"]
    value = pairs / (r32["ms_per_step"] / 1e3)
    dom = dominant_apply(r32["kernels"])[0]
    roof = roofline(r32["kernels"], r32["stats"], inst.grid, 8, VALU_PEAK_TFLOPS["c64"],
                    workload=args.workload if not args.bands else None)
    copy_gbs = copy_bandwidth(device)
    roof["copy_gbs"] = round(copy_gbs, 1)
    roof["hbm_frac_vs_copy"] = round(roof["alt"]["hbm_gbs"] / copy_gbs, 4)

    line = {
        "metric": "band-pair Fock applications/s, FP32 vs FP64 path, + % of HBM roofline",
        "value": round(value, 1),
        "unit": "ordered band pairs/s (apply + overlap + energy + backward per step)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 complex)",
        "data": "synthetic (seeded random orthonormal orbitals, 12 Ha cutoff)",
        "config": {"workload": WORKLOADS[cfg],
                   "ordered_pairs_per_step": pairs, "grid": list(inst.grid), "nk": inst.nk, "nbands": inst.nbands},
        "roofline": roof,
        "ms_per_step_median": round(r32["ms_median"], 3),
        "launch_gaps": launch_gaps(r32),
        "fp32": {"ms_per_step": round(r32["ms_per_step"], 3), "pairs_per_s": round(value, 1),
                 "kernels_ms": {k: round(v[0], 3) for k, v in r32["kernels"].items() if v[1]},
                 "kernel_rates": kernel_rates(r32["kernels"], r32["stats"], inst.grid, 8),
                 "apply_ms": round(sum(v[0] for v in r32["apply_kernels"].values()), 3)},
    }
    if r64:
        v64 = pairs / (r64["ms_per_step"] / 1e3)
        line["fp64"] = {"ms_per_step": round(r64["ms_per_step"], 3), "pairs_per_s": round(v64, 1),
                        "kernels_ms": {k: round(v[0], 3) for k, v in r64["kernels"].items() if v[1]},
                        "kernel_rates": kernel_rates(r64["kernels"], r64["stats"], inst.grid, 16),
                        "apply_ms": round(sum(v[0] for v in r64["apply_kernels"].values()), 3)}
        line["fp32_speedup_over_fp64"] = round(r64["ms_per_step"] / r32["ms_per_step"], 3)
        line["ex_fp32_vs_fp64_rel"] = abs(r32["ex"] - r64["ex"]) / abs(r64["ex"])
    del inst, inst32
    if args.workload == "alpha" and args.beta_steps > 0:
        line["beta_boron_fp32"] = beta_leg(args, device)
    if cb:
        line["cpu_baseline"] = cb
    line["host"] = host_info()
    print(json.dumps(line), flush=True)


def membw(args):
    """Device memory bandwidth against working-set size: a full read (sum of
    a float32 buffer) and a copy (half the set read, half written), each
    repeated; sets that fit the 256 MB Infinity Cache are served from it on
    repeats, larger ones stream from HBM.  One JSON line per size."""
    import torch

    device = torch.device("cuda:0")
    buf = torch.zeros(2048 << 18, dtype=torch.float32, device=device)  # 2 GiB
    dst = torch.empty(1024 << 18, dtype=torch.float32, device=device)
    out = []
    for mib in (32, 64, 128, 192, 256, 384, 512, 1024, 2048):
        n = mib << 18  # float32 elements
        reps = 50 if mib <= 256 else 10
        x, h = buf[:n], n // 2
        for kind in ("read", "copy"):
            def op():
                if kind == "read":
                    return x.sum()
                return dst[:h].copy_(x[:h])
            op()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                op()
            e1.record()
            torch.cuda.synchronize()
            gbs = (mib << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
            out.append({"working_set_mib": mib, "kind": kind, "gbs": round(gbs, 1)})
            log(f"  {mib:5d} MiB {kind}: {gbs:8.1f} GB/s")
    print(json.dumps({"metric": "device memory bandwidth vs working set", "unit": "GB/s (bytes read + written)",
                      "results": out, "host": host_info()}), flush=True)


def beta_leg(args, device):
    """The largest workload (beta-boron-shaped 72^3, 2x2x2 k-mesh, 160 bands)
    on the FP32 path, timed like the headline: fock_apply_energy + backward
    per step, the three-pass apply rated on the 4 s N model."""
    from paper_1111_0716_amd import inputs

    log(f"beta-boron leg: generating inputs ({WORKLOADS['3']})")
    inst = inputs.config("3", dtype=np.complex64, workers=16)
    w = min(1, args.warmup)
    log(f"beta-boron FP32 path: {w} warm-up + {args.beta_steps} timed steps")
    r = run_path(inst, "c64", args.beta_steps, w, device, breakdown=False)
    log(f"  {r['ms_per_step']:.1f} ms/step")
    pairs = r["stats"]["ordered_pairs"]
    dom = dominant_apply(r["kernels"])[0]
    roof = roofline(r["kernels"], r["stats"], inst.grid, 8, VALU_PEAK_TFLOPS["c64"], workload="beta")
    return {"workload": WORKLOADS["3"], "ordered_pairs_per_step": pairs, "steps": args.beta_steps, "warmup": w,
            "ms_per_step": round(r["ms_per_step"], 3), "pairs_per_s": round(pairs / (r["ms_per_step"] / 1e3), 1),
            "roofline": roof, "launch_gaps": launch_gaps(r),
            "kernels_ms": {k: round(v[0], 3) for k, v in r["kernels"].items() if v[1]},
            "kernel_rates": kernel_rates(r["kernels"], r["stats"], inst.grid, 8)}


if __name__ == "__main__":
    main()
