"""Autotuner host logic (no GPU): cache keys, cache round trip, and that the
library accepts and validates the tuning knobs."""
import ctypes
import json

import numpy as np

from paper_1111_0716_amd import autotune, fock, inputs


def test_shape_key_is_order_independent_and_precision_specific():
    a = dict(grid=(24, 24, 24), kfrac=np.zeros((1, 3)), nbands=8)
    b = dict(grid=(32, 32, 32), kfrac=np.zeros((8, 3)), nbands=12)
    k1 = autotune.shape_key([a, b], "c64", "gfx950")
    k2 = autotune.shape_key([b, a], "c64", "gfx950")
    assert k1 == k2
    assert autotune.shape_key([a, b], "c128", "gfx950") != k1
    assert json.loads(k1)["shapes"][0][0] == [24, 24, 24]


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("FOCK_TUNE_CACHE", str(tmp_path / "tune.json"))
    assert autotune.load_cache() == {}
    autotune.save_cache({"k": {"tuning": {"fused_split": 2}, "ms": 1.0}})
    assert autotune.load_cache()["k"]["tuning"]["fused_split"] == 2


def _plan_with(tuning, grid=(32, 32, 32), nb=4, prec=fock.FOCK_C64):
    keep = []
    d = fock.make_desc(inputs.cubic_lattice(10.0), grid, inputs.gamma_mesh(2, 1, 1), nbands=nb, keep=keep)
    arr = (fock.FockDesc * 1)(d)
    h = ctypes.c_void_p()
    tn = fock.FockTuning(**tuning)
    st = fock.lib().fock_plan_tuned(arr, 1, prec, None, ctypes.byref(tn), ctypes.byref(h))
    return st, h


def test_tuning_knobs_change_the_schedule():
    st0, h0 = _plan_with({"no_pair_symmetry": 1})  # the whole-pair kernel, one workgroup per output
    st1, h1 = _plan_with({"no_fused": 1, "acc_workgroups": 64, "no_pair_symmetry": 1})
    assert st0 == fock.FOCK_OK and st1 == fock.FOCK_OK
    a0, a1 = ctypes.c_int64(), ctypes.c_int64()
    L = fock.lib()
    L.fock_plan_stats(h0, None, None, None, ctypes.byref(a0))
    L.fock_plan_stats(h1, None, None, None, ctypes.byref(a1))
    assert a0.value <= 2            # one whole-pair launch (plus a partial sum)
    assert a1.value >= 3            # three kernels per three-pass batch
    L.fock_destroy(h0)
    L.fock_destroy(h1)


def test_tuning_knob_validation():
    st, _ = _plan_with({"fused_split": 9})
    assert st == fock.FOCK_ERR_ARG
    st, _ = _plan_with({"fused_rounds": 2})
    assert st == fock.FOCK_ERR_ARG
    st, _ = _plan_with({"tbuf_mb": -1})
    assert st == fock.FOCK_ERR_ARG


def test_candidates_cover_the_joint_grid_and_collapse_equal_schedules():
    c = autotune.candidates({"plane", "pencil", "accumulate"})
    assert {} in c
    assert any(t.get("tbuf_mb") == 256 and "no_pair_symmetry" not in t for t in c)  # Infinity-Cache-sized batches
    ordered = {(t["tbuf_mb"], t["acc_workgroups"]) for t in c if t.get("no_pair_symmetry")}
    assert ordered == {(tb, aw) for tb in autotune.ORDERED_TBUF_MB for aw in autotune.ORDERED_ACC_WORKGROUPS}
    f = autotune.candidates({"fused"})
    assert {t.get("fused_split") for t in f if "fused_split" in t} == {1, 2, 3, 4}
    assert {"fused_rounds": 1} in f
    # a tiny three-pass instance: every pair-buffer budget gives the same plan
    inst = dict(lattice=inputs.cubic_lattice(10.0), grid=(24, 32, 32), kfrac=np.zeros((1, 3)), nbands=2)
    sigs = {autotune.plan_signature([inst], "c64", t) for t in c}
    assert len(sigs) < len(c)
    assert autotune.plan_signature([inst], "c64", {}) == autotune.plan_signature([inst], "c64", {"tbuf_mb": 128})
