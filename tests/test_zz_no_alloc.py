"""fock_apply_energy_static (the entry point that allocates nothing) against
fock_apply_energy on the same inputs, through the C ABI.

Three calls in a row on one device share the library's static workspace:
a register-line three-pass plan, then a smaller whole-pair plan, then the
first plan again (its tables must be uploaded again).  Each must give the
outputs of fock_apply_energy on a plan with its own workspace: V_x psi and
the overlaps bitwise equal (same kernels, same order), E_x equal, and both
within the oracle tolerances of the parity tests.
"""
import sys

import numpy as np
import pytest

from oracle.fock_oracle import Oracle
from paper_1111_0716_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"c128": dict(e=1e-12, v=1e-12), "c64": dict(e=1e-6, v=1e-5)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _case(grid, kmesh, nbands, prec, seed, device):
    import torch

    from paper_1111_0716_amd import fock

    inst = inputs.small_instance(grid=grid, kmesh=kmesh, nbands=nbands, seed=seed)
    dt = np.complex64 if prec == "c64" else np.complex128
    psi_np = np.ascontiguousarray(inst.psi.astype(dt))
    psi = torch.from_numpy(psi_np).to(device)
    occ = torch.from_numpy(np.ascontiguousarray(inst.occ)).to(device)
    static_plan = fock.Plan([inst], precision=prec, device=device, attach_workspace=False)
    ref_plan = fock.Plan([inst], precision=prec, device=device)
    assert static_plan.workspace_bytes <= fock.STATIC_WORKSPACE_BYTES
    return inst, psi_np, psi, occ, static_plan, ref_plan


def _check(inst, psi_np, psi, occ, static_plan, ref_plan, prec, tag):
    import torch

    nk, nb = inst.psi.shape[:2]
    cdt = static_plan.cdtype
    # outputs pre-filled with garbage: the call must write every element
    out = torch.full_like(psi, complex(7.0, -3.0))
    vmat = torch.full((nk, nb, nb), complex(5.0, 1.0), dtype=cdt, device=psi.device)
    ex = torch.full((1,), 11.0, dtype=torch.float64, device=psi.device)
    log(f"no-alloc {tag}: grid {inst.grid} nk {nk} nb {nb} {prec} static workspace "
        f"{static_plan.workspace_bytes} B")
    static_plan.fock_apply_energy_static([psi], [occ], out=[out], vmat=[vmat], ex=ex)
    (vref,), (mref,), eref = ref_plan.fock_apply_energy([psi], [occ], vmat=True)
    torch.cuda.synchronize()
    assert torch.equal(out, vref), f"{tag}: V_x psi differs from fock_apply_energy"
    assert torch.equal(vmat, mref), f"{tag}: overlap differs from fock_apply_energy"
    assert torch.equal(ex, eref), f"{tag}: E_x differs from fock_apply_energy"
    o = Oracle.from_instance(inst)
    v_or, e_or = o.apply(psi_np.astype(np.complex128), inst.occ)
    got = out.cpu().numpy().astype(np.complex128)
    verr = max(np.linalg.norm(got[k, n] - v_or[k, n]) / np.linalg.norm(v_or[k, n])
               for k in range(nk) for n in range(nb))
    eerr = abs(float(ex.item()) - e_or) / abs(e_or)
    log(f"no-alloc {tag}: |dVx|/|Vx| {verr:.2e} |dE|/|E| {eerr:.2e}")
    assert verr <= TOL[prec]["v"] and eerr <= TOL[prec]["e"]


def test_static_workspace_calls_match_apply_energy(device):
    from paper_1111_0716_amd import fock

    big = _case((24, 32, 32), (2, 1, 1), 3, "c64", (2101, 0), device)
    small = _case((16, 16, 16), (1, 1, 1), 2, "c128", (2102, 0), device)
    assert small[4].workspace_bytes < big[4].workspace_bytes
    _check(*big, "c64", "first (three-pass, 24x32x32)")
    _check(*small, "c128", "second (whole-pair, 16^3, smaller)")
    _check(*big, "c64", "third (first plan again)")
    for c in (big, small):
        c[4].close()
        c[5].close()
    assert fock.STATIC_WORKSPACE_BYTES == 64 << 20


def test_static_workspace_rejects_large_plans(device):
    from paper_1111_0716_amd import fock

    inst = inputs.small_instance(grid=(32, 32, 32), kmesh=(4, 4, 1), nbands=4, seed=(2103, 0))
    plan = fock.Plan([inst], precision="c128", device=device, attach_workspace=False)
    assert plan.workspace_bytes > fock.STATIC_WORKSPACE_BYTES
    import torch

    psi = torch.zeros(inst.psi.shape, dtype=torch.complex128, device=device)
    occ = torch.from_numpy(np.ascontiguousarray(inst.occ)).to(device)
    with pytest.raises(fock.FockError) as e:
        plan.fock_apply_energy_static([psi], [occ])
    assert e.value.status == fock.FOCK_ERR_NOMEM
    plan.close()
