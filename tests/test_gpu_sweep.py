"""Seeded sweep over the supported problem space, through the C ABI, against
the FP64 oracle: grid shapes of every path ({2,3,5}-smooth axes on the LDS
three-pass path, N1 x L x L register-line shapes, whole-pair cubes), skewed
cells, k-meshes, band counts, occupations (some zero), padded band strides,
explicit k-pair lists and all three precisions.

Each case checks V_x u (max over bands of the relative 2-norm error), E_x
(relative; from fock_energy and from fock_apply_energy, whose V_x u and M
must equal fock_apply's bitwise) and the overlap M (max-norm relative): FP64 path <= 1e-12,
FP32 and mixed paths <= 1e-5 on V_x u and M, <= 1e-6 on E_x, with the oracle
run on the exact complex64 values upcast for the FP32 path."""
import sys

import numpy as np
import pytest

from oracle.fock_oracle import Oracle
from paper_1111_0716_amd import inputs

pytestmark = pytest.mark.gpu

SMOOTH = [5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32, 36, 40, 45]
REG = [24, 32, 36, 40, 48, 50, 54, 60, 64, 72]
KMESHES = [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 2, 1)]
TOL = {"c128": dict(e=1e-12, v=1e-12), "c64": dict(e=1e-6, v=1e-5), "mixed": dict(e=1e-6, v=1e-5),
       "mixed_inv": dict(e=1e-6, v=1e-5)}
# oracle budget per case: ordered pairs x N x (N1 + N2 + N3), the direct DFT's work
BUDGET = 2e10
NCASES = 64


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def draw(i):
    """Case i of the sweep: grid, k-mesh, bands, precision, padding, k pairs."""
    rng = np.random.default_rng([11110716, 900, i])
    kind = i % 4
    if kind == 0:    # any smooth shape: LDS three-pass
        grid = tuple(int(x) for x in rng.choice(SMOOTH, 3))
    elif kind == 1:  # register-line N1 x L x L
        l = int(rng.choice(REG))
        grid = (int(rng.choice(REG)), l, l)
    elif kind == 2:  # whole-pair cubes (FP32), register-line or whole-pair (FP64)
        l = int(rng.choice([16, 24, 32]))
        grid = (l, l, l)
    else:            # larger smooth shapes
        grid = tuple(int(x) for x in rng.choice(SMOOTH[8:], 3))
    reg = grid[1] == grid[2] and grid[0] in REG and grid[1] in REG
    precs = ["c64", "c128"] + (["mixed", "mixed_inv"] if reg else [])
    prec = precs[int(rng.integers(len(precs)))]
    n = int(np.prod(grid))
    kmesh = KMESHES[int(rng.integers(len(KMESHES)))]
    nk = int(np.prod(kmesh))
    nb = int(rng.integers(1, 5))
    while nb > 1 and (nk * nb) ** 2 * n * sum(grid) > BUDGET:
        nb -= 1
    while nk > 1 and (nk * nb) ** 2 * n * sum(grid) > BUDGET:
        kmesh, nk = (1, 1, 1), 1
    pad = int(rng.choice([0, 0, 1, 37, 64]))
    kpairs = None
    if nk > 1 and rng.random() < 0.3:
        allp = [(a, b) for a in range(nk) for b in range(nk)]
        keep = rng.random(len(allp)) < 0.6
        kpairs = np.array([p for p, k in zip(allp, keep) if k] or [(0, 0)], dtype=np.int32)
    zero_band = nb > 1 and rng.random() < 0.3
    full = bool(rng.random() < 0.3)
    angle = float(rng.uniform(55.0, 75.0))
    edge = float(rng.uniform(6.0, 12.0))
    return dict(grid=grid, kmesh=kmesh, nb=nb, prec=prec, pad=pad, kpairs=kpairs, zero_band=zero_band,
                full=full, angle=angle, edge=edge, seed=i)


def band_err(got, ref):
    err = 0.0
    for k in range(ref.shape[0]):
        for b in range(ref.shape[1]):
            den = np.linalg.norm(ref[k, b])
            num = np.linalg.norm(got[k, b] - ref[k, b])
            err = max(err, num if den == 0 else num / den)
    return err


@pytest.mark.parametrize("i", range(NCASES))
def test_sweep_case_matches_oracle(i, device):
    import torch

    from paper_1111_0716_amd import fock

    c = draw(i)
    log(f"sweep case {i}: grid={c['grid']} kmesh={c['kmesh']} nb={c['nb']} prec={c['prec']} pad={c['pad']} "
        f"kpairs={None if c['kpairs'] is None else c['kpairs'].tolist()} zero_band={c['zero_band']} full={c['full']}")
    lat = inputs.rhombohedral_lattice(c["edge"], c["angle"])
    inst = inputs.small_instance(grid=c["grid"], kmesh=c["kmesh"], nbands=c["nb"], seed=(900, i), lattice=lat,
                                 full_grid=c["full"])
    if c["zero_band"]:
        inst.occ[:, -1] = 0.0
    dt = np.complex64 if c["prec"] == "c64" else np.complex128
    psi_h = inst.psi.astype(dt)
    n = inst.npoints
    bs = n + c["pad"]
    plan = fock.Plan([inst], precision=c["prec"], device=device, band_stride=[bs] if c["pad"] else None,
                     kpairs=[c["kpairs"]] if c["kpairs"] is not None else None)
    psi = torch.zeros((inst.nk, inst.nbands, bs), dtype=torch.complex64 if dt == np.complex64 else torch.complex128,
                      device=device)
    psi[:, :, :n] = torch.from_numpy(np.ascontiguousarray(psi_h)).to(device)
    occ = torch.from_numpy(np.ascontiguousarray(inst.occ)).to(device)
    (vx,), (m,) = plan.fock_apply([psi], [occ], vmat=True)
    ex = plan.fock_energy([psi], [occ]).item()
    (vx2,), (m2,), ex2 = plan.fock_apply_energy([psi], [occ], vmat=True)
    torch.cuda.synchronize()
    assert torch.equal(vx2[:, :, :n], vx[:, :, :n]) and torch.equal(m2, m)  # padding is never written
    ex2 = ex2.item()
    vx = vx[:, :, :n].cpu().numpy()
    m = m.cpu().numpy()
    plan.close()

    o = Oracle.from_instance(inst, kpairs=c["kpairs"])
    u = psi_h.astype(np.complex128)
    vref, eref = o.apply(u, inst.occ)
    mref = o.overlap(u, vref)
    tol = TOL[c["prec"]]
    ev = band_err(vx, vref)
    ee = abs(ex - eref) / abs(eref) if eref != 0 else abs(ex)
    em = np.max(np.abs(m - mref)) / max(np.max(np.abs(mref)), 1e-300)
    log(f"  V_x {ev:.2e}  E_x {ee:.2e}  M {em:.2e}")
    ee2 = abs(ex2 - eref) / abs(eref) if eref != 0 else abs(ex2)
    assert ev <= tol["v"]
    assert ee <= tol["e"] and ee2 <= tol["e"]
    assert em <= tol["v"]


@pytest.mark.parametrize("i", range(16))
def test_sweep_backward_matches_oracle_gradient(i, device):
    """dE_x/du* from fock_energy_backward (co-densities recomputed) against
    the oracle gradient, on the sweep's cases 64 + i."""
    import torch

    from paper_1111_0716_amd import fock

    c = draw(NCASES + i)
    log(f"backward case {i}: grid={c['grid']} kmesh={c['kmesh']} nb={c['nb']} prec={c['prec']} pad={c['pad']}")
    lat = inputs.rhombohedral_lattice(c["edge"], c["angle"])
    inst = inputs.small_instance(grid=c["grid"], kmesh=c["kmesh"], nbands=c["nb"], seed=(901, i), lattice=lat,
                                 full_grid=c["full"])
    dt = np.complex64 if c["prec"] == "c64" else np.complex128
    psi_h = inst.psi.astype(dt)
    n = inst.npoints
    bs = n + c["pad"]
    plan = fock.Plan([inst], precision=c["prec"], device=device, band_stride=[bs] if c["pad"] else None)
    psi = torch.zeros((inst.nk, inst.nbands, bs), dtype=torch.complex64 if dt == np.complex64 else torch.complex128,
                      device=device)
    psi[:, :, :n] = torch.from_numpy(np.ascontiguousarray(psi_h)).to(device)
    occ = torch.from_numpy(np.ascontiguousarray(inst.occ)).to(device)
    o = Oracle.from_instance(inst)
    gex = torch.full((1,), 0.75, dtype=torch.float64, device=device)
    (g,) = plan.fock_energy_backward([psi], [occ], gex, 2.0 * o.dv)
    torch.cuda.synchronize()
    g = g[:, :, :n].cpu().numpy()
    plan.close()
    gref = 0.75 * o.gradient(psi_h.astype(np.complex128), inst.occ)
    err = band_err(g, gref)
    log(f"  grad err {err:.2e}")
    assert err <= TOL[c["prec"]]["v"]


@pytest.mark.parametrize("i", range(24))
def test_sweep_dft3_matches_oracle(i, device):
    """Batched 3-D DFT (both signs, unnormalised) on random grid shapes,
    register-line N1 x L x L shapes included, against the oracle's DFT."""
    import torch

    from oracle import pw_oracle as pw
    from paper_1111_0716_amd import fock

    rng = np.random.default_rng([11110716, 902, i])
    if i % 3 == 0:
        l = int(rng.choice([16] + REG))
        grid = (int(rng.choice([16] + REG)), l, l)
    else:
        grid = tuple(int(x) for x in rng.choice(SMOOTH + [48, 50, 54, 60, 64, 72], 3))
    prec = "c64" if rng.random() < 0.5 else "c128"
    n = int(np.prod(grid))
    count = int(rng.integers(1, 4)) if n < 200_000 else 1
    log(f"dft3 case {i}: grid={grid} prec={prec} count={count}")
    inst = inputs.small_instance(grid=grid, kmesh=(1, 1, 1), nbands=1, seed=(902, i), full_grid=True)
    plan = fock.Plan([inst], precision=prec, device=device)
    x = rng.standard_normal((count, n)) + 1j * rng.standard_normal((count, n))
    x = x.astype(np.complex64 if prec == "c64" else np.complex128)
    tol = 1e-5 if prec == "c64" else 1e-12
    for sign in (-1, +1):
        d = torch.from_numpy(np.ascontiguousarray(x)).to(device)
        plan.dft3(d, sign)
        got = d.cpu().numpy()
        for b in range(count):
            ref = pw.dft3(x[b].astype(np.complex128), grid, sign)
            err = np.linalg.norm(got[b] - ref) / np.linalg.norm(ref)
            assert err <= tol, (sign, b, err)
    plan.close()
