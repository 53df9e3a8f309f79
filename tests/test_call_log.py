"""FOCK_LOG call records: one JSON line per API call of a plan created while
FOCK_LOG names a file, and a per-call summary at fock_destroy.  The CPU test
uses calls that fail before any device work (no workspace attached); the GPU
test checks device times of real calls, eager and under graph replay."""
import ctypes
import json

import numpy as np
import pytest

from paper_1111_0716_amd import fock, inputs


def _read(path):
    return [json.loads(line) for line in open(path) if line.strip()]


def test_records_and_summary_without_device_work(tmp_path, monkeypatch):
    path = tmp_path / "calls.jsonl"
    monkeypatch.setenv("FOCK_LOG", str(path))
    L = fock.lib()
    keep = []
    d = fock.make_desc(inputs.cubic_lattice(10.0), (8, 8, 8), np.zeros((1, 3)), nbands=2, keep=keep)
    h = ctypes.c_void_p()
    assert L.fock_plan((fock.FockDesc * 1)(d), 1, fock.FOCK_C64, None, ctypes.byref(h)) == fock.FOCK_OK
    one, two = fock._ptrs([1]), fock._ptrs([2])
    assert L.fock_apply(h, one, one, two, None) == fock.FOCK_ERR_STATE
    assert L.fock_energy(h, one, one, ctypes.c_void_p(1)) == fock.FOCK_ERR_STATE
    assert L.fock_apply(h, one, one, two, None) == fock.FOCK_ERR_STATE
    assert not path.exists() or not _read(path)  # written at fock_destroy
    L.fock_destroy(h)
    recs = _read(path)
    calls = [r for r in recs if "call" in r]
    summ = {r["summary"]: r for r in recs if "summary" in r}
    assert [r["call"] for r in calls] == ["fock_apply", "fock_energy", "fock_apply"]
    assert all(r["status"] == fock.FOCK_ERR_STATE and r["device_ms"] == -1 for r in calls)
    assert calls[0]["ordered_pairs"] == 4 and calls[0]["instances"] == 1
    assert len({r["plan"] for r in recs}) == 1
    assert summ["fock_apply"]["calls"] == 2 and summ["fock_energy"]["calls"] == 1


def test_no_records_without_the_variable(tmp_path, monkeypatch):
    monkeypatch.delenv("FOCK_LOG", raising=False)
    monkeypatch.chdir(tmp_path)
    L = fock.lib()
    keep = []
    d = fock.make_desc(inputs.cubic_lattice(10.0), (8, 8, 8), np.zeros((1, 3)), nbands=2, keep=keep)
    h = ctypes.c_void_p()
    assert L.fock_plan((fock.FockDesc * 1)(d), 1, fock.FOCK_C64, None, ctypes.byref(h)) == fock.FOCK_OK
    L.fock_destroy(h)
    assert list(tmp_path.iterdir()) == []


@pytest.mark.gpu
def test_device_times_are_recorded(tmp_path, monkeypatch, device):
    import torch

    path = tmp_path / "calls.jsonl"
    monkeypatch.setenv("FOCK_LOG", str(path))
    inst = inputs.small_instance(grid=(12, 10, 9), kmesh=(2, 1, 1), nbands=3, seed=(320, 0))
    stream = torch.cuda.Stream(device=device)
    plan = fock.Plan([inst], precision="c128", device=device, stream=stream)
    psi = torch.from_numpy(inst.psi).to(device)
    occ = torch.from_numpy(np.ascontiguousarray(inst.occ)).to(device)
    with torch.cuda.stream(stream):
        plan.fock_apply([psi], [occ])
        plan.set_graph(True)
        plan.fock_apply_energy([psi], [occ])
        plan.fock_apply_energy([psi], [occ])
    stream.synchronize()
    plan.close()
    recs = _read(path)
    calls = [r for r in recs if "call" in r]
    assert [r["call"] for r in calls] == ["fock_apply", "fock_apply_energy", "fock_apply_energy"]
    assert all(r["status"] == 0 and r["device_ms"] > 0 for r in calls)
    assert [r["graph"] for r in calls] == [0, 1, 1]
    summ = {r["summary"]: r for r in recs if "summary" in r}
    assert summ["fock_apply_energy"]["calls"] == 2 and summ["fock_apply_energy"]["ordered_pairs_per_s"] > 0
