"""Plane-wave boundary (sphere <-> grid) and batched 3-D DFT of the HIP
library, through the C ABI, against the FP64 oracle (oracle/pw_oracle.py,
oracle/fock_oracle.py).

Tolerances: relative 2-norm per grid or per band, FP64 <= 1e-12,
FP32 <= 1e-5 (the oracle runs on the complex64 values upcast)."""
import sys

import numpy as np
import pytest

from oracle import pw_oracle as pw
from oracle.fock_oracle import Oracle
from paper_1111_0716_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rel(a, b):
    a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def sphere(inst, ecut, pad=3, junk=False):
    """Slots per k (padded by `pad`); padding slots hold out-of-grid classes
    when `junk` (the library must skip them)."""
    g = [inputs.sphere_indices(inst.lattice, inst.kfrac[k], ecut, inst.grid) for k in range(inst.nk)]
    npw = np.array([len(x) for x in g], dtype=np.int32)
    npw_max = int(npw.max()) + pad
    gidx = np.full((inst.nk, npw_max), -1, dtype=np.int32)
    n = int(np.prod(inst.grid))
    for k, x in enumerate(g):
        gidx[k, : len(x)] = pw.grid_classes(x, inst.grid)
        if junk:
            gidx[k, len(x):] = np.arange(npw_max - len(x)) % 2 * (n + 7) - 1  # -1 and n + 6
    return gidx, npw, npw_max


def dev(a, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


@pytest.mark.parametrize("grid,prec", [((12, 10, 9), "c128"), ((16, 16, 16), "c64"), ((32, 32, 32), "c128"),
                                       ((5, 72, 6), "c64"), ((24, 20, 18), "c128"), ((72, 72, 72), "c64"),
                                       ((48, 64, 64), "c64"), ((72, 40, 40), "c64"), ((24, 16, 16), "c128"),
                                       ((16, 32, 32), "c128"), ((60, 60, 60), "c64"), ((50, 54, 54), "c64"),
                                       ((36, 36, 36), "c128")])
def test_dft3_matches_oracle(grid, prec, device):
    from paper_1111_0716_amd import fock

    log(f"dft3 grid={grid} prec={prec}")
    inst = inputs.small_instance(grid=grid, kmesh=(1, 1, 1), nbands=1, seed=(300, sum(grid)))
    plan = fock.Plan([inst], precision=prec, device=device)
    rng = np.random.default_rng(sum(grid))
    n = int(np.prod(grid))
    count = 1 if n > 200_000 else 3
    x = rng.standard_normal((count, n)) + 1j * rng.standard_normal((count, n))
    dt = np.complex64 if prec == "c64" else np.complex128
    x = x.astype(dt)
    for sign in (-1, +1):
        d = dev(x, device)
        plan.dft3(d, sign)
        got = d.cpu().numpy()
        for b in range(count):
            ref = pw.dft3(x[b].astype(np.complex128), grid, sign)
            err = rel(got[b], ref)
            assert err <= TOL[prec], (sign, b, err)
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_sphere_to_grid_and_back_match_oracle(prec, device):
    """Scatter + inverse DFT and forward DFT + gather against the oracle;
    padding slots carry out-of-grid classes and non-zero coefficients."""
    from paper_1111_0716_amd import fock

    inst = inputs.small_instance(grid=(12, 10, 9), kmesh=(2, 1, 1), nbands=3, seed=(301, 0))
    gidx, npw, npw_max = sphere(inst, inst.ecut, pad=3, junk=True)
    rng = np.random.default_rng(7)
    coef = rng.standard_normal((inst.nk, inst.nbands, npw_max)) + 1j * rng.standard_normal((inst.nk, inst.nbands, npw_max))
    dt = np.complex64 if prec == "c64" else np.complex128
    coef = coef.astype(dt)
    plan = fock.Plan([inst], precision=prec, device=device)
    g_d, n_d = dev(gidx, device), dev(npw, device)
    (u,) = plan.pw_to_grid([dev(coef, device)], [g_d], [n_d])
    u = u.cpu().numpy()
    uref = pw.pw_to_grid(inst.lattice, inst.grid, gidx, npw, coef.astype(np.complex128))
    assert rel(u, uref) <= TOL[prec]
    f = rng.standard_normal(uref.shape) + 1j * rng.standard_normal(uref.shape)
    f = f.astype(dt)
    (d,) = plan.grid_to_pw([dev(f, device)], [g_d], [n_d])
    d = d.cpu().numpy()
    dref = pw.grid_to_pw(inst.lattice, inst.grid, gidx, npw, npw_max, f.astype(np.complex128))
    assert rel(d, dref) <= TOL[prec]
    for k in range(inst.nk):
        assert np.all(d[k, :, npw[k]:] == 0)
    plan.close()


@pytest.mark.parametrize("grid,kmesh,prec", [((12, 10, 9), (2, 1, 1), "c128"), ((16, 16, 16), (1, 2, 1), "c64"),
                                             ((24, 24, 24), (2, 1, 1), "c64"), ((32, 32, 32), (1, 1, 1), "c128")])
def test_apply_on_the_sphere_matches_oracle(grid, kmesh, prec, device):
    """V_x psi on the sphere from sphere coefficients, against the oracle's
    operator on the grid projected to the sphere, and the band overlap."""
    from paper_1111_0716_amd import fock

    log(f"apply_pw grid={grid} kmesh={kmesh} prec={prec}")
    inst = inputs.small_instance(grid=grid, kmesh=kmesh, nbands=3, seed=(302, grid[0]))
    gidx, npw, npw_max = sphere(inst, inst.ecut, pad=1)
    coef = pw.grid_to_pw(inst.lattice, inst.grid, gidx, npw, npw_max, inst.psi)  # the generated orbitals
    dt = np.complex64 if prec == "c64" else np.complex128
    coef = coef.astype(dt)
    u = pw.pw_to_grid(inst.lattice, inst.grid, gidx, npw, coef.astype(np.complex128))
    o = Oracle.from_instance(inst)
    vx, _ = o.apply(u, inst.occ)
    dref = pw.grid_to_pw(inst.lattice, inst.grid, gidx, npw, npw_max, vx)
    plan = fock.Plan([inst], precision=prec, device=device)
    (d,), (psi_w,), (vx_w,) = plan.fock_apply_pw([dev(coef, device)], [dev(gidx, device)], [dev(npw, device)],
                                                 [dev(inst.occ, device)])
    d = d.cpu().numpy()
    err = max(rel(d[k, b], dref[k, b]) for k in range(inst.nk) for b in range(inst.nbands))
    log(f"  per-band err {err:.2e}")
    assert err <= TOL[prec]
    assert rel(psi_w.cpu().numpy(), u) <= TOL[prec]
    m_pw = np.einsum("kip,kjp->kij", coef.astype(np.complex128).conj(), d)
    m_ref = o.overlap(u, vx)
    assert rel(m_pw, m_ref) <= TOL[prec]
    plan.close()


def test_alpha_boron_sphere_round_trip_and_apply(device):
    """Full-size alpha-boron workload (32^3, 4x4x4, 18 bands) on the FP32 path:
    the sphere round trip is the identity, and V_x psi on the sphere equals
    the grid apply followed by the gather."""
    import torch

    from paper_1111_0716_amd import fock

    inst = inputs.config("2", dtype=np.complex128, workers=8)
    gidx, npw, npw_max = sphere(inst, inst.ecut, pad=0)
    coef = pw.grid_to_pw(inst.lattice, inst.grid, gidx, npw, npw_max, inst.psi[:, :2])
    log(f"config 2 sphere: npw {npw.min()}..{npw.max()}")
    plan = fock.Plan([inst.astype(np.complex64)], precision="c64", device=device)
    g_d, n_d = dev(gidx, device), dev(npw, device)
    psi = dev(inst.psi.astype(np.complex64), device)
    occ = dev(inst.occ, device)
    # coefficients of every band from the library's own gather, then back
    (c_all,) = plan.grid_to_pw([psi.clone()], [g_d], [n_d])
    assert rel(c_all[:, :2].cpu().numpy(), coef) <= 1e-5
    (u,) = plan.pw_to_grid([c_all], [g_d], [n_d])
    assert rel(u.cpu().numpy(), inst.psi) <= 1e-5
    (d,), _, _ = plan.fock_apply_pw([c_all], [g_d], [n_d], [occ])
    (vx,), _ = plan.fock_apply([u], [occ])
    (dref,) = plan.grid_to_pw([vx], [g_d], [n_d])
    torch.cuda.synchronize()
    assert rel(d.cpu().numpy(), dref.cpu().numpy()) <= 1e-6
    plan.close()
