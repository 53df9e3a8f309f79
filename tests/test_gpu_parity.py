"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (relative):  FP64 path  E_x and V_x psi <= 1e-12;
                        FP32 path  E_x <= 1e-6, V_x psi <= 1e-5 per band,
with the oracle run on the exact complex64 values upcast to complex128.
V_x psi error per band: ||delta||_2 / ||V_x psi||_2, max over (k, n).
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


def band_err(got, ref, bands=None):
    got = got.reshape(ref.shape)
    err = 0.0
    nk, nb = ref.shape[:2]
    for k in range(nk):
        for n in range(nb):
            if bands is not None and (k, n) not in bands:
                continue
            den = np.linalg.norm(ref[k, n])
            if den == 0:
                err = max(err, np.linalg.norm(got[k, n]))
            else:
                err = max(err, np.linalg.norm(got[k, n] - ref[k, n]) / den)
    return err


def run_gpu(inst, prec, device, kpairs=None, vmat=False):
    import torch

    from paper_1111_0716_amd import fock

    plan = fock.Plan([inst], precision=prec, device=device, kpairs=[kpairs] if kpairs is not None else None)
    dt = np.complex64 if prec == "c64" else np.complex128
    psi = torch.from_numpy(np.ascontiguousarray(inst.psi.astype(dt))).to(device)
    occ = torch.from_numpy(np.ascontiguousarray(inst.occ)).to(device)
    (vx,), mats = plan.fock_apply([psi], [occ], vmat=vmat)
    ex = plan.fock_energy([psi], [occ])
    torch.cuda.synchronize()
    out = dict(vx=vx.cpu().numpy(), ex=float(ex.item()), plan=plan, psi=psi, occ=occ)
    if vmat:
        out["vmat"] = mats[0].cpu().numpy()
    return out


CASES = [
    # grid, k-mesh, bands, full-grid orbitals, precision
    ((16, 16, 16), (1, 1, 1), 8, False, "c128"),
    ((12, 10, 9), (2, 1, 1), 3, False, "c128"),
    ((24, 20, 18), (2, 1, 1), 5, False, "c128"),
    ((8, 6, 10), (2, 2, 1), 3, True, "c128"),
    ((72, 6, 8), (1, 1, 1), 2, True, "c128"),
    ((6, 72, 5), (1, 1, 1), 2, True, "c128"),
    ((5, 6, 72), (1, 2, 1), 2, True, "c128"),
    ((48, 40, 36), (1, 1, 1), 2, False, "c128"),
    ((27, 25, 32), (1, 1, 2), 3, False, "c128"),
    ((24, 20, 18), (2, 1, 1), 5, False, "c64"),
    ((16, 30, 15), (1, 2, 1), 4, False, "c64"),
    ((8, 6, 10), (2, 2, 1), 3, True, "c64"),
    ((64, 64, 64), (1, 1, 1), 2, False, "c64"),
    ((72, 72, 72), (1, 1, 1), 1, False, "c64"),
    # register-line three-pass path (cubic grids)
    ((24, 24, 24), (2, 1, 1), 3, False, "c128"),
    ((32, 32, 32), (1, 2, 1), 2, True, "c128"),
    ((40, 40, 40), (1, 1, 1), 2, False, "c64"),
    ((48, 48, 48), (2, 1, 1), 2, True, "c64"),
    # lines shared by a lane pair (FP64 40^3 and up, FP32 64^3 and up)
    ((40, 40, 40), (1, 2, 1), 2, False, "c128"),
    ((48, 48, 48), (1, 1, 1), 2, True, "c128"),
    ((64, 64, 64), (1, 1, 1), 1, False, "c128"),
    ((72, 72, 72), (1, 1, 1), 1, True, "c128"),
    ((64, 64, 64), (2, 1, 1), 1, True, "c64"),
    # register-line path on grids N1 x L x L: plane and accumulate passes of
    # side L over N1 planes (a partial last plane group where N1 is not a
    # multiple of the planes per workgroup), pencil pass of length N1
    ((48, 64, 64), (1, 1, 1), 1, False, "c64"),
    ((72, 48, 48), (1, 1, 1), 1, True, "c64"),
    ((32, 24, 24), (2, 1, 1), 2, False, "c64"),
    ((24, 32, 32), (2, 1, 1), 2, False, "c128"),
    ((64, 40, 40), (1, 1, 1), 1, False, "c128"),
    ((24, 72, 72), (1, 1, 1), 1, False, "c128"),
    # lengths 36, 50, 54, 60 (one lane FP32; two lanes FP64)
    ((60, 60, 60), (1, 1, 1), 1, False, "c64"),
    ((36, 36, 36), (2, 1, 1), 2, True, "c128"),
    ((50, 54, 54), (1, 1, 1), 1, False, "c64"),
    ((36, 60, 60), (1, 1, 1), 1, False, "c128"),
    ((54, 36, 36), (1, 2, 1), 2, False, "c64"),
    # whole-pair path (cubic grids that fit one compute unit)
    ((32, 32, 32), (1, 1, 1), 3, False, "c64"),
    ((32, 32, 32), (2, 1, 1), 2, True, "c64"),
    ((24, 24, 24), (2, 1, 1), 3, False, "c64"),
    ((16, 16, 16), (1, 2, 1), 3, True, "c64"),
    ((16, 16, 16), (2, 1, 1), 3, True, "c128"),
]


@pytest.mark.parametrize("grid,kmesh,nb,full,prec", CASES)
def test_apply_and_energy_match_oracle(grid, kmesh, nb, full, prec, device):
    log(f"case grid={grid} kmesh={kmesh} nb={nb} full={full} prec={prec}")
    inst = inputs.small_instance(grid=grid, kmesh=kmesh, nbands=nb, seed=(200, sum(grid)), full_grid=full)
    if prec == "c64":
        inst = inst.astype(np.complex64)
    g = run_gpu(inst, prec, device, vmat=True)
    o = Oracle.from_instance(inst)
    vref, eref = o.apply(inst.psi.astype(np.complex128), inst.occ)
    ev = band_err(g["vx"], vref)
    ee = abs(g["ex"] - eref) / abs(eref)
    log(f"  V_x err {ev:.3e}  E_x err {ee:.3e}")
    assert ev <= TOL[prec]["v"]
    assert ee <= TOL[prec]["e"]
    mref = o.overlap(inst.psi.astype(np.complex128), vref)
    em = np.max(np.abs(g["vmat"] - mref)) / np.max(np.abs(mref))
    assert em <= TOL[prec]["v"]


def test_plane_wave_closed_form_on_gpu(device):
    """Golden closed form (one band at G=0, cubic 10 bohr, Gamma): E_x = -v(0)/(2 Omega)."""
    lat = inputs.cubic_lattice(10.0)
    grid = (16, 16, 16)
    psi = np.full((1, 1, 4096), 1.0 / np.sqrt(1000.0), dtype=np.complex128)
    inst = inputs.Instance(lat, grid, np.zeros((1, 3)), np.ones(1), np.ones((1, 1)), psi)
    g = run_gpu(inst, "c128", device)
    assert g["ex"] == pytest.approx(-0.13980031388349026, rel=1e-13)


def test_explicit_k_pairs_and_empty_partner_lists(device):
    inst = inputs.small_instance(grid=(12, 10, 9), kmesh=(2, 2, 1), nbands=3, seed=(201, 0))
    kp = np.array([[0, 0], [0, 1], [1, 3], [2, 2], [2, 0]], dtype=np.int32)  # k=3 has no partner
    g = run_gpu(inst, "c128", device, kpairs=kp)
    o = Oracle.from_instance(inst, kpairs=kp)
    vref, eref = o.apply(inst.psi, inst.occ)
    assert band_err(g["vx"], vref) <= 1e-12
    assert np.all(g["vx"].reshape(vref.shape)[3] == 0)
    assert abs(g["ex"] - eref) <= 1e-12 * abs(eref)


def test_fp64_results_are_bitwise_reproducible(device):
    import torch

    inst = inputs.small_instance(grid=(12, 10, 9), kmesh=(2, 1, 1), nbands=3, seed=(202, 0))
    g = run_gpu(inst, "c128", device)
    plan, psi, occ = g["plan"], g["psi"], g["occ"]
    (vx2,), _ = plan.fock_apply([psi], [occ])
    ex2 = plan.fock_energy([psi], [occ])
    torch.cuda.synchronize()
    assert np.array_equal(vx2.cpu().numpy(), g["vx"])
    assert ex2.item() == g["ex"]


@pytest.mark.parametrize("grid,prec", [((10, 12, 9), "c128"), ((10, 12, 9), "c64"), ((16, 16, 16), "c64"),
                                       ((24, 24, 24), "c64"), ((16, 16, 16), "c128"), ((32, 32, 32), "c128"),
                                       ((64, 64, 64), "c64"), ((40, 40, 40), "c128")])
def test_backward_matches_oracle_gradient(grid, prec, device):
    import torch

    log(f"backward grid={grid} prec={prec}")
    inst = inputs.small_instance(grid=grid, kmesh=(2, 1, 1), nbands=3, seed=(203, grid[0]), full_grid=True)
    if prec == "c64":
        inst = inst.astype(np.complex64)
    g = run_gpu(inst, prec, device)
    plan, psi, occ = g["plan"], g["psi"], g["occ"]
    o = Oracle.from_instance(inst)
    gref = o.gradient(inst.psi.astype(np.complex128), inst.occ)  # torch convention
    scale = 2.0 * o.dv
    gex = torch.full((1,), 0.75, dtype=torch.float64, device=device)
    (gg,) = plan.fock_energy_backward([psi], [occ], gex, scale)
    torch.cuda.synchronize()
    err = band_err(gg.cpu().numpy(), 0.75 * gref)
    assert err <= TOL[prec]["v"]


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_config_1_exact_inputs(prec, device):
    """The tiny preset as specified (cubic 10 bohr, 16^3, Gamma, 8 bands f=1,
    4 Ha sphere, seeded QR orbitals; its co-density span of 17 reaches the
    Nyquist classes): V_x psi, the overlap, E_x from both energy routes and
    the gradient against the oracle, FP64 and complex64 copies."""
    import torch

    from paper_1111_0716_amd import fock

    inst = inputs.config("1")
    if prec == "c64":
        inst = inst.astype(np.complex64)
    g = run_gpu(inst, prec, device, vmat=True)
    plan, psi, occ = g["plan"], g["psi"], g["occ"]
    (v2,), _, ex2 = plan.fock_apply_energy([psi], [occ])
    o = Oracle.from_instance(inst)
    u = inst.psi.astype(np.complex128)
    vref, eref = o.apply(u, inst.occ)
    gref = o.gradient(u, inst.occ, vref)
    gex = torch.full((1,), 1.25, dtype=torch.float64, device=device)
    (gg,) = plan.fock_energy_backward([psi], [occ], gex, 2.0 * o.dv)
    torch.cuda.synchronize()
    ev = band_err(g["vx"], vref)
    ee = max(abs(g["ex"] - eref), abs(ex2.item() - eref)) / abs(eref)
    em = np.max(np.abs(g["vmat"] - o.overlap(u, vref))) / np.max(np.abs(vref))
    eg = band_err(gg.cpu().numpy(), 1.25 * gref)
    log(f"config 1 {prec}: V_x {ev:.2e}  E_x {ee:.2e}  M {em:.2e}  grad {eg:.2e}")
    assert ev <= TOL[prec]["v"] and ee <= TOL[prec]["e"]
    assert em <= TOL[prec]["v"] and eg <= TOL[prec]["v"]
    assert torch.equal(v2.cpu(), torch.from_numpy(g["vx"]))
    plan.close()


def test_autograd_function_and_finite_differences(device):
    """FockEnergy forward = E_x, backward = the library gradient; FP64 central
    differences (h = 1e-6) along random directions."""
    import torch

    from paper_1111_0716_amd import fock

    inst = inputs.small_instance(grid=(12, 10, 9), kmesh=(1, 1, 1), nbands=4, seed=(204, 0))
    plan = fock.Plan([inst], precision="c128", device=device)
    FockEnergy = fock.fock_energy_autograd()
    psi = torch.from_numpy(inst.psi).to(device).requires_grad_(True)
    occ = torch.from_numpy(inst.occ).to(device)
    e = FockEnergy.apply(plan, [occ], psi)
    e.sum().backward()
    grad = psi.grad.detach()
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(4):
        d = rng.standard_normal(inst.psi.shape) + 1j * rng.standard_normal(inst.psi.shape)
        d = torch.from_numpy(d / np.linalg.norm(d)).to(device)
        with torch.no_grad():
            ep = plan.fock_energy([psi.detach() + h * d], [occ]).item()
            em = plan.fock_energy([psi.detach() - h * d], [occ]).item()
        fd = (ep - em) / (2 * h)
        an = torch.real(torch.vdot(grad.reshape(-1), d.reshape(-1))).item()
        assert abs(fd - an) <= 1e-8 * torch.linalg.norm(grad).item()


def test_autograd_function_over_instances_of_different_cells(device):
    """One plan over two instances of different cells and grids: the autograd
    Function returns both energies and gives each orbital set torch's
    gradient 2 dV_i g_i w f V_x u with its own dV_i, against the oracle."""
    import torch

    from paper_1111_0716_amd import fock

    insts = [inputs.small_instance(grid=(12, 10, 9), kmesh=(2, 1, 1), nbands=3, seed=(215, 0)),
             inputs.small_instance(grid=(16, 16, 16), kmesh=(1, 1, 1), nbands=2, seed=(215, 1),
                                   lattice=inputs.cubic_lattice(8.5))]
    plan = fock.Plan(insts, precision="c128", device=device)
    FockEnergy = fock.fock_energy_autograd()
    psi = [torch.from_numpy(i.psi).to(device).requires_grad_(True) for i in insts]
    occ = [torch.from_numpy(i.occ).to(device) for i in insts]
    e = FockEnergy.apply(plan, occ, *psi)
    w = torch.tensor([0.7, -1.3], dtype=torch.float64, device=device)
    (w * e).sum().backward()
    for i, inst in enumerate(insts):
        o = Oracle.from_instance(inst)
        vref, eref = o.apply(inst.psi, inst.occ)
        assert abs(e[i].item() - eref) <= 1e-12 * abs(eref)
        err = band_err(psi[i].grad.detach().cpu().numpy(), w[i].item() * o.gradient(inst.psi, inst.occ, vref))
        log(f"  instance {i}: gradient err {err:.2e}")
        assert err <= 1e-12
    plan.close()


@pytest.mark.parametrize("grid,prec", [((32, 32, 32), "c64"), ((24, 24, 24), "c64"), ((16, 16, 16), "c128")])
def test_whole_pair_path_matches_three_pass_path(grid, prec, device, monkeypatch):
    """The whole-pair kernels and the three-pass kernels compute the same
    operator: compare them directly (and both against the oracle above)."""
    inst = inputs.small_instance(grid=grid, kmesh=(2, 1, 1), nbands=3, seed=(205, grid[0]))
    if prec == "c64":
        inst = inst.astype(np.complex64)
    fused = run_gpu(inst, prec, device)
    monkeypatch.setenv("FOCK_NO_FUSED", "1")
    three = run_gpu(inst, prec, device)
    assert band_err(fused["vx"], three["vx"].reshape(fused["vx"].shape)) <= 2 * TOL[prec]["v"]
    assert abs(fused["ex"] - three["ex"]) <= 2 * TOL[prec]["e"] * abs(three["ex"])


def test_alpha_boron_config_sampled_outputs(device):
    """Full-size alpha-boron workload (32^3, 4x4x4 k-mesh, 18 bands) on the FP32
    path as the benchmark runs it: sampled outputs against the oracle (every
    partner of the sampled band), E_x against 1/2 sum w f <u|V_x u> from the
    GPU's own apply, and E_x against the FP64 path."""
    import torch

    from paper_1111_0716_amd import fock

    inst = inputs.config("2", dtype=np.complex128, workers=8)
    inst32 = inst.astype(np.complex64)
    log("config 2 FP32 full apply")
    g = run_gpu(inst32, "c64", device, vmat=True)
    o = Oracle.from_instance(inst32)
    for (k, n) in [(0, 0), (37, 11), (63, 17)]:
        vref, _ = o.apply(inst32.psi.astype(np.complex128), inst32.occ, outputs=[(k, n)])
        err = band_err(g["vx"], vref, bands={(k, n)})
        log(f"  output ({k},{n}) err {err:.2e}")
        assert err <= 1e-5
    m = g["vmat"]
    ex_apply = 0.5 * np.sum(inst.kweight[:, None] * inst.occ * np.real(np.einsum("kii->ki", m)))
    assert abs(ex_apply - g["ex"]) <= 1e-5 * abs(g["ex"])
    log("config 2 FP64 energy")
    plan64 = fock.Plan([inst], precision="c128", device=device)
    psi64 = torch.from_numpy(inst.psi).to(device)
    occ64 = torch.from_numpy(inst.occ).to(device)
    ex64 = plan64.fock_energy([psi64], [occ64]).item()
    log(f"  E32 {g['ex']:.12f}  E64 {ex64:.12f}")
    assert abs(g["ex"] - ex64) <= 1e-6 * abs(ex64)


@pytest.mark.parametrize("kp", [[[0, 0], [0, 1], [1, 0], [1, 1]], [[0, 0], [1, 1]], [[0, 1], [1, 0], [1, 1]]])
def test_whole_pair_explicit_k_pairs(kp, device):
    """Explicit k-pair lists on a whole-pair grid: the full set listed
    explicitly, a diagonal-only set, and a set without (0, 0)."""
    inst = inputs.small_instance(grid=(16, 16, 16), kmesh=(2, 1, 1), nbands=3, seed=(207, len(kp))).astype(np.complex64)
    kp = np.array(kp, dtype=np.int32)
    g = run_gpu(inst, "c64", device, kpairs=kp)
    o = Oracle.from_instance(inst, kpairs=kp)
    vref, eref = o.apply(inst.psi.astype(np.complex128), inst.occ)
    assert band_err(g["vx"], vref) <= 1e-5
    assert abs(g["ex"] - eref) <= 1e-6 * abs(eref)


@pytest.mark.parametrize("grid,prec", [((32, 32, 32), "c128"), ((24, 24, 24), "c128"), ((48, 48, 48), "c64"),
                                       ((64, 64, 64), "c64"), ((72, 72, 72), "c64"), ((40, 40, 40), "c128"),
                                       ((64, 64, 64), "c128"), ((48, 64, 64), "c64"), ((64, 40, 40), "c128"),
                                       ((32, 24, 24), "c64"), ((60, 60, 60), "c64"), ((36, 36, 36), "c128"),
                                       ((54, 50, 50), "c128")])
def test_register_line_path_matches_lds_path(grid, prec, device, monkeypatch):
    """The register-line three-pass kernels and the LDS-Stockham three-pass
    kernels compute the same operator and energy (FP64: to rounding)."""
    log(f"register-line vs LDS grid={grid} prec={prec}")
    inst = inputs.small_instance(grid=grid, kmesh=(2, 1, 1), nbands=2, seed=(208, grid[0]))
    if prec == "c64":
        inst = inst.astype(np.complex64)
    reg = run_gpu(inst, prec, device)
    monkeypatch.setenv("FOCK_NO_REG", "1")
    lds = run_gpu(inst, prec, device)
    tol = 1e-13 if prec == "c128" else 2e-6
    ev = band_err(reg["vx"], lds["vx"].reshape(reg["vx"].shape))
    ee = abs(reg["ex"] - lds["ex"]) / abs(lds["ex"])
    log(f"  V_x {ev:.2e}  E_x {ee:.2e}")
    assert ev <= tol and ee <= tol


@pytest.mark.parametrize("grid,kmesh,nb", [((24, 24, 24), (2, 1, 1), 3), ((32, 32, 32), (1, 2, 1), 2),
                                           ((48, 48, 48), (1, 1, 1), 2), ((64, 64, 64), (1, 1, 1), 1),
                                           ((72, 72, 72), (1, 1, 1), 1), ((32, 72, 72), (1, 1, 1), 1),
                                           ((72, 24, 24), (2, 1, 1), 2), ((60, 36, 36), (1, 1, 1), 2),
                                           ((50, 50, 50), (1, 1, 1), 1)])
def test_mixed_precision_matches_oracle(grid, kmesh, nb, device):
    """FP32 co-densities and forward transforms, FP64 multiply, inverse and
    accumulate: complex128 in and out, held to the FP32 tolerances."""
    log(f"mixed grid={grid} kmesh={kmesh} nb={nb}")
    inst = inputs.small_instance(grid=grid, kmesh=kmesh, nbands=nb, seed=(209, grid[0]), full_grid=grid[0] == 32)
    g = run_gpu(inst, "mixed", device, vmat=True)
    o = Oracle.from_instance(inst)
    vref, eref = o.apply(inst.psi, inst.occ)
    ev = band_err(g["vx"], vref)
    ee = abs(g["ex"] - eref) / abs(eref)
    log(f"  V_x err {ev:.3e}  E_x err {ee:.3e}")
    assert ev <= TOL["c64"]["v"] and ee <= TOL["c64"]["e"]
    mref = o.overlap(inst.psi, vref)
    assert np.max(np.abs(g["vmat"] - mref)) <= TOL["c64"]["v"] * np.max(np.abs(mref))


@pytest.mark.parametrize("grid,kmesh,nb", [((24, 24, 24), (2, 1, 1), 3), ((32, 32, 32), (1, 2, 1), 2),
                                           ((40, 40, 40), (1, 1, 1), 2), ((64, 64, 64), (1, 1, 1), 1),
                                           ((72, 72, 72), (1, 1, 1), 1), ((32, 72, 72), (1, 1, 1), 1),
                                           ((72, 24, 24), (2, 1, 1), 2), ((60, 36, 36), (1, 1, 1), 2),
                                           ((50, 54, 54), (1, 1, 1), 1)])
def test_mixed_inv_precision_matches_oracle(grid, kmesh, nb, device):
    """The other mixed policy: FP64 co-densities, forward transforms, kernel
    multiply and energies, FP32 inverse transforms and accumulate into FP64
    outputs; complex128 in and out, held to the FP32 tolerances, with E_x
    from the FP64 spectrum."""
    log(f"mixed_inv grid={grid} kmesh={kmesh} nb={nb}")
    inst = inputs.small_instance(grid=grid, kmesh=kmesh, nbands=nb, seed=(214, grid[0]), full_grid=grid[0] == 32)
    g = run_gpu(inst, "mixed_inv", device, vmat=True)
    o = Oracle.from_instance(inst)
    vref, eref = o.apply(inst.psi, inst.occ)
    ev = band_err(g["vx"], vref)
    ee = abs(g["ex"] - eref) / abs(eref)
    log(f"  V_x err {ev:.3e}  E_x err {ee:.3e}")
    assert ev <= TOL["c64"]["v"]
    assert ee <= 1e-12  # fock_energy runs on the FP64 transforms
    mref = o.overlap(inst.psi, vref)
    assert np.max(np.abs(g["vmat"] - mref)) <= TOL["c64"]["v"] * np.max(np.abs(mref))
    plan, psi, occ = g["plan"], g["psi"], g["occ"]
    (v2,), _, ex2 = plan.fock_apply_energy([psi], [occ])
    import torch

    torch.cuda.synchronize()
    assert np.array_equal(v2.cpu().numpy(), g["vx"])
    assert abs(float(ex2.item()) - eref) <= 1e-12 * abs(eref)  # pair energies in FP64 in the apply too


def test_mixed_inv_precision_backward(device):
    import torch

    inst = inputs.small_instance(grid=(24, 32, 32), kmesh=(2, 1, 1), nbands=3, seed=(215, 0), full_grid=True)
    g = run_gpu(inst, "mixed_inv", device)
    plan, psi, occ = g["plan"], g["psi"], g["occ"]
    o = Oracle.from_instance(inst)
    gref = o.gradient(inst.psi, inst.occ)
    gex = torch.full((1,), 0.5, dtype=torch.float64, device=device)
    (gg,) = plan.fock_energy_backward([psi], [occ], gex, 2.0 * o.dv)
    torch.cuda.synchronize()
    assert band_err(gg.cpu().numpy(), 0.5 * gref) <= TOL["c64"]["v"]


def test_mixed_precision_backward(device):
    import torch

    inst = inputs.small_instance(grid=(24, 24, 24), kmesh=(2, 1, 1), nbands=3, seed=(210, 0), full_grid=True)
    g = run_gpu(inst, "mixed", device)
    plan, psi, occ = g["plan"], g["psi"], g["occ"]
    o = Oracle.from_instance(inst)
    gref = o.gradient(inst.psi, inst.occ)
    gex = torch.full((1,), 0.5, dtype=torch.float64, device=device)
    (gg,) = plan.fock_energy_backward([psi], [occ], gex, 2.0 * o.dv)
    torch.cuda.synchronize()
    assert band_err(gg.cpu().numpy(), 0.5 * gref) <= TOL["c64"]["v"]


@pytest.mark.parametrize("grid,prec", [((16, 16, 16), "c64"), ((32, 32, 32), "c64"), ((16, 16, 16), "c128"),
                                       ((48, 48, 48), "c64"), ((32, 32, 32), "c128"), ((40, 40, 40), "c128"),
                                       ((12, 10, 9), "c128"), ((24, 24, 24), "mixed"), ((48, 64, 64), "c64"),
                                       ((24, 40, 40), "c128")])
def test_padded_band_stride_gives_identical_results(grid, prec, device):
    """Bands stored band_stride = N + 37 elements apart (odd padding) give
    bitwise the same V_x u, overlap and E_x as the packed layout, and the
    padding is never written."""
    import torch

    from paper_1111_0716_amd import fock

    inst = inputs.small_instance(grid=grid, kmesh=(2, 1, 1), nbands=2, seed=(211, grid[0]))
    dt = np.complex64 if prec == "c64" else np.complex128
    n = inst.npoints
    bs = n + 37
    psi = torch.from_numpy(np.ascontiguousarray(inst.psi.astype(dt))).to(device)
    occ = torch.from_numpy(inst.occ).to(device)
    packed = fock.Plan([inst], precision=prec, device=device)
    (vx0,), (m0,) = packed.fock_apply([psi], [occ], vmat=True)
    ex0 = packed.fock_energy([psi], [occ]).item()
    padded = fock.Plan([inst], precision=prec, device=device, band_stride=[bs])
    pp = torch.full((inst.nk, inst.nbands, bs), 7.0, dtype=psi.dtype, device=device)
    pp[:, :, :n] = psi
    out = torch.full_like(pp, 3.0)
    (vx1,), (m1,) = padded.fock_apply([pp], [occ], out=[out], vmat=True)
    ex1 = padded.fock_energy([pp], [occ]).item()
    torch.cuda.synchronize()
    assert torch.equal(vx1[:, :, :n], vx0)
    assert torch.all(vx1[:, :, n:] == 3.0)
    assert torch.equal(m1, m0)
    assert ex1 == ex0
    packed.close()
    padded.close()


@pytest.mark.parametrize("grid,prec", [((32, 32, 32), "c64"), ((12, 10, 9), "c128"), ((48, 48, 48), "c64")])
def test_zero_occupations_give_zero_exchange(grid, prec, device):
    inst = inputs.small_instance(grid=grid, kmesh=(2, 1, 1), nbands=2, seed=(212, grid[0]))
    inst.occ[:] = 0.0
    if prec == "c64":
        inst = inst.astype(np.complex64)
    g = run_gpu(inst, prec, device, vmat=True)
    assert np.all(g["vx"] == 0) and g["ex"] == 0.0 and np.all(g["vmat"] == 0)


@pytest.mark.parametrize("grid,kmesh,nb,prec", [((32, 32, 32), (2, 1, 1), 3, "c64"), ((24, 24, 24), (1, 2, 1), 3, "c64"),
                                                ((16, 16, 16), (2, 1, 1), 3, "c128"), ((16, 16, 16), (1, 1, 1), 4, "c64"),
                                                ((24, 24, 24), (2, 1, 1), 2, "c128"), ((12, 10, 9), (2, 1, 1), 3, "c128"),
                                                ((48, 40, 40), (1, 1, 1), 2, "mixed"), ((48, 48, 48), (1, 1, 1), 2, "c64"),
                                                ((40, 40, 40), (1, 2, 1), 2, "c128"), ((48, 64, 64), (1, 1, 1), 1, "c64"),
                                                ((72, 72, 72), (1, 1, 1), 1, "c64"), ((36, 60, 60), (1, 1, 1), 1, "c128"),
                                                ((20, 18, 24), (1, 2, 1), 2, "c64")])
def test_apply_energy_matches_apply_and_energy(grid, kmesh, nb, prec, device):
    """fock_apply_energy: V_x u and the overlap bitwise equal to fock_apply's,
    E_x equal to fock_energy's to rounding and to the oracle within the
    path's tolerance."""
    import torch

    from paper_1111_0716_amd import fock

    log(f"apply+energy grid={grid} kmesh={kmesh} nb={nb} prec={prec}")
    inst = inputs.small_instance(grid=grid, kmesh=kmesh, nbands=nb, seed=(213, grid[0]), full_grid=grid[0] == 16)
    dt = np.complex64 if prec == "c64" else np.complex128
    psi = torch.from_numpy(np.ascontiguousarray(inst.psi.astype(dt))).to(device)
    occ = torch.from_numpy(inst.occ).to(device)
    plan = fock.Plan([inst], precision=prec, device=device)
    (v0,), (m0,) = plan.fock_apply([psi], [occ], vmat=True)
    e0 = plan.fock_energy([psi], [occ]).item()
    (v1,), (m1,), ex = plan.fock_apply_energy([psi], [occ], vmat=True)
    e1 = ex.item()
    (v2,), (m2,), ex2 = plan.fock_apply_energy([psi], [occ], vmat=True)
    torch.cuda.synchronize()
    assert torch.equal(v1, v0) and torch.equal(m1, m0)
    assert torch.equal(v2, v1) and torch.equal(m2, m1) and ex2.item() == e1
    assert abs(e1 - e0) <= (1e-13 if prec == "c128" else 1e-7) * abs(e0)
    o = Oracle.from_instance(inst)
    _, eref = o.apply(inst.psi.astype(dt).astype(np.complex128), inst.occ)
    tol = TOL["c128"]["e"] if prec == "c128" else TOL["c64"]["e"]
    log(f"  E_x {e1:.12e} (energy call {e0:.12e}, oracle {eref:.12e})")
    assert abs(e1 - eref) <= tol * abs(eref)
    plan.close()


def test_apply_energy_mixed_plan_and_empty_partner_lists(device):
    """One plan with a whole-pair instance (explicit k pairs, one k without
    partners) and a register-line instance: E_x of each against the oracle."""
    import torch

    from paper_1111_0716_amd import fock

    a = inputs.small_instance(grid=(32, 32, 32), kmesh=(2, 2, 1), nbands=2, seed=(214, 0))
    b = inputs.small_instance(grid=(40, 40, 40), kmesh=(2, 1, 1), nbands=2, seed=(214, 1))
    kp = np.array([[0, 0], [0, 1], [1, 3], [2, 2], [2, 0]], dtype=np.int32)  # k = 3 has no partner
    insts = [a.astype(np.complex64), b.astype(np.complex64)]
    plan = fock.Plan(insts, precision="c64", device=device, kpairs=[kp, None])
    psi = [torch.from_numpy(np.ascontiguousarray(i.psi)).to(device) for i in insts]
    occ = [torch.from_numpy(i.occ).to(device) for i in insts]
    vx, _, ex = plan.fock_apply_energy(psi, occ)
    e0 = plan.fock_energy(psi, occ)
    torch.cuda.synchronize()
    for i, (inst, k) in enumerate(zip(insts, [kp, None])):
        o = Oracle.from_instance(inst, kpairs=k)
        vref, eref = o.apply(inst.psi.astype(np.complex128), inst.occ)
        assert band_err(vx[i].cpu().numpy(), vref) <= TOL["c64"]["v"]
        assert abs(ex[i].item() - eref) <= TOL["c64"]["e"] * abs(eref)
        assert abs(ex[i].item() - e0[i].item()) <= 1e-7 * abs(eref)
    assert np.all(vx[0].cpu().numpy()[3] == 0)
    plan.close()
