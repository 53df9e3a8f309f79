"""Seeded synthetic inputs for the screened exact-exchange path.

This module builds what a plane-wave code would hand to the Fock operator:
a cell, a Gamma-centred k-mesh with weights, occupations, and orthonormal
orbitals stored as their periodic parts on the FFT grid.  It holds none of
the exchange arithmetic (no co-density, no kernel, no FFT round trip); the
CPU oracle and the HIP library both receive its arrays as plain inputs.

Workload shapes follow the paper's boron runs (section "Setup of DFT
calculations", Table "tests": k-mesh 4x4x4 with NGX 24 for alpha-boron,
2x2x2 with NGX 48 for the larger cells) scaled to the synthetic presets
below.  Coefficients are i.i.d. complex normal on the plane-wave sphere
|k+G|^2/2 < E_cut, orthonormalised per k by an FP64 QR, and mapped to the
grid as u = (N/sqrt(Omega)) * IDFT(c placed on the grid), so that
dV * sum_j |u_j|^2 = 1 with dV = Omega/N.

Seeds: numpy.random.default_rng([11110716, config_id, instance_id, k_index]).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.fft

SEED_BASE = 11110716
MU_HSE = 0.106  # screening parameter of HSE06 in bohr^-1 (0.2 A^-1)


# ----------------------------------------------------------------------------
# cells and meshes
# ----------------------------------------------------------------------------
def cubic_lattice(a: float) -> np.ndarray:
    """Rows a1, a2, a3 of a simple cubic cell with edge ``a`` (bohr)."""
    return np.eye(3) * float(a)


def rhombohedral_lattice(a: float, alpha_deg: float) -> np.ndarray:
    """Rows of a rhombohedral cell: three edges of length ``a`` with the
    same angle ``alpha`` between every pair (the alpha/beta boron cells)."""
    al = np.deg2rad(alpha_deg)
    ca, sa = np.cos(al), np.sin(al)
    cy = (ca - ca * ca) / sa
    cz = np.sqrt(max(1.0 - ca * ca - cy * cy, 0.0))
    return float(a) * np.array([[1.0, 0.0, 0.0], [ca, sa, 0.0], [ca, cy, cz]])


def reciprocal_rows(lattice: np.ndarray) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T


def gamma_mesh(n1: int, n2: int, n3: int) -> np.ndarray:
    """Gamma-centred uniform mesh, fractional coordinates (i/n1, j/n2, l/n3)."""
    pts = [(i / n1, j / n2, l / n3) for i in range(n1) for j in range(n2) for l in range(n3)]
    return np.array(pts, dtype=np.float64)


def sphere_indices(lattice, kfrac, ecut, grid):
    """Integer G vectors with |k+G|^2/2 < ecut.  Raises if the sphere does not
    fit strictly inside the grid (|g_i| < N_i/2), since the orbital itself
    would then alias."""
    lattice = np.asarray(lattice, dtype=np.float64)
    b = reciprocal_rows(lattice)
    kc = np.asarray(kfrac, dtype=np.float64) @ b
    gmax_r = np.sqrt(2.0 * ecut) + np.linalg.norm(kc)
    lim = [int(np.ceil(gmax_r * np.linalg.norm(lattice[i]) / (2.0 * np.pi))) + 1 for i in range(3)]
    rng = [np.arange(-l, l + 1) for l in lim]
    g = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    kg = kc[None, :] + g @ b
    keep = 0.5 * np.einsum("ij,ij->i", kg, kg) < ecut
    g = g[keep]
    for i in range(3):
        if g.size and np.max(np.abs(g[:, i])) * 2 >= grid[i]:
            raise ValueError(f"cutoff sphere does not fit grid axis {i}: |g|max={np.max(np.abs(g[:, i]))}, N={grid[i]}")
    # deterministic order (lexicographic) so seeds map to the same coefficients
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0]))
    return g[order]


def orthonormal_coefficients(npw: int, nbands: int, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. complex normal (Re, Im ~ N(0, 1/2)) columns, orthonormalised by FP64 QR."""
    if npw < nbands:
        raise ValueError(f"{npw} plane waves cannot hold {nbands} orthonormal bands")
    c = (rng.standard_normal((npw, nbands)) + 1j * rng.standard_normal((npw, nbands))) * np.sqrt(0.5)
    q, r = np.linalg.qr(c)
    # fix the phase ambiguity of QR so the result is a function of the draw only
    d = np.diag(r)
    q = q * (d / np.abs(d))[None, :]
    return q


def coefficients_to_grid(lattice, grid, g, coef, workers=None) -> np.ndarray:
    """u = (N/sqrt(Omega)) * IDFT(coefficients placed at classes g mod N).
    coef: [npw, nb] -> returns complex128 [nb, N1*N2*N3]."""
    n1, n2, n3 = grid
    n = n1 * n2 * n3
    omega = abs(np.linalg.det(lattice))
    nb = coef.shape[1]
    box = np.zeros((nb, n1, n2, n3), dtype=np.complex128)
    c1, c2, c3 = (g[:, 0] % n1), (g[:, 1] % n2), (g[:, 2] % n3)
    box[:, c1, c2, c3] = coef.T
    u = scipy.fft.ifftn(box, axes=(1, 2, 3), workers=workers) * (n / np.sqrt(omega))
    return u.reshape(nb, n)


def random_grid_orbitals(grid, nk, nbands, rng, lattice) -> np.ndarray:
    """Full-grid random orbitals (every frequency class populated, including
    Nyquist), normalised per band: dV * sum |u|^2 = 1.  Used to exercise the
    kernel's alias convention; not orthonormalised."""
    n = int(np.prod(grid))
    omega = abs(np.linalg.det(lattice))
    u = rng.standard_normal((nk, nbands, n)) + 1j * rng.standard_normal((nk, nbands, n))
    nrm = np.sqrt((omega / n) * np.sum(np.abs(u) ** 2, axis=-1, keepdims=True))
    return u / nrm


# ----------------------------------------------------------------------------
# instances and presets
# ----------------------------------------------------------------------------
@dataclass
class Instance:
    """One exchange problem.  psi: complex [nk, nbands, N1*N2*N3] periodic parts."""

    lattice: np.ndarray
    grid: tuple
    kfrac: np.ndarray
    kweight: np.ndarray
    occ: np.ndarray
    psi: np.ndarray
    mu: float = MU_HSE
    ecut: float | None = None
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def nk(self):
        return self.kfrac.shape[0]

    @property
    def nbands(self):
        return self.psi.shape[1]

    @property
    def npoints(self):
        return int(np.prod(self.grid))

    def ordered_pairs(self):
        return self.nk * self.nk * self.nbands * self.nbands

    def astype(self, dtype):
        return Instance(self.lattice, self.grid, self.kfrac, self.kweight, self.occ,
                        self.psi.astype(dtype), self.mu, self.ecut, self.name, dict(self.extra))


def make_instance(lattice, grid, kmesh, nbands, ecut, seed, occ=None, mu=MU_HSE,
                  dtype=np.complex128, name="", kshift=(0.0, 0.0, 0.0), workers=None) -> Instance:
    """Orthonormal plane-wave orbitals for every k of a Gamma-centred mesh.
    ``seed`` is the tuple (config_id, instance_id); k index is appended."""
    lattice = np.asarray(lattice, dtype=np.float64)
    kfrac = gamma_mesh(*kmesh) + np.asarray(kshift, dtype=np.float64)[None, :]
    nk = kfrac.shape[0]
    n = int(np.prod(grid))
    psi = np.empty((nk, nbands, n), dtype=dtype)
    for ik in range(nk):
        rng = np.random.default_rng([SEED_BASE, *seed, ik])
        g = sphere_indices(lattice, kfrac[ik], ecut, grid)
        coef = orthonormal_coefficients(len(g), nbands, rng)
        psi[ik] = coefficients_to_grid(lattice, grid, g, coef, workers=workers)
    if occ is None:
        occ = np.ones((nk, nbands))
    occ = np.broadcast_to(np.asarray(occ, dtype=np.float64), (nk, nbands)).copy()
    kweight = np.full(nk, 1.0 / nk)
    return Instance(lattice, tuple(int(x) for x in grid), kfrac, kweight, occ, psi, mu, ecut, name)


BETA_A, BETA_ALPHA = 19.16, 65.2
ALPHA_A, ALPHA_ALPHA = 9.56, 58.0


def config(cfg_id, dtype=None, workers=None):
    """Preset workloads (boron-shaped synthetic cells).

    1  tiny: cubic 10 bohr, 16^3, Gamma, 8 bands f=1, E_cut 4 Ha, complex128
    2  alpha-boron-shaped: rhombohedral a=9.56, 58.0 deg, 32^3, 4x4x4, 18 bands, 12 Ha
    3  beta-boron-shaped: rhombohedral a=19.16, 65.2 deg, 72^3, 2x2x2, 160 bands
       (152 with f=1, 8 with f ~ U[0.05, 0.95] shared by all k), 12 Ha, complex64
    5  differentiation: a=19.16, 65.2 deg, 64^3, Gamma, 128 bands, 12 Ha, complex64
    "5s" the 24^3 / 16-band subset of 5, E_cut 1.5 Ha
    Config 4 (48 ragged instances) is built by ``uneven_batch``.
    """
    cid = str(cfg_id)
    if cid == "1":
        inst = make_instance(cubic_lattice(10.0), (16, 16, 16), (1, 1, 1), 8, 4.0, (1, 0),
                             dtype=dtype or np.complex128, name="tiny-16^3", workers=workers)
    elif cid == "2":
        inst = make_instance(rhombohedral_lattice(ALPHA_A, ALPHA_ALPHA), (32, 32, 32), (4, 4, 4), 18, 12.0,
                             (2, 0), dtype=dtype or np.complex64, name="alpha-boron-32^3-k444", workers=workers)
    elif cid == "3":
        rng = np.random.default_rng([SEED_BASE, 3, 0, 1_000_000])
        occ = np.ones(160)
        occ[152:] = rng.uniform(0.05, 0.95, size=8)
        inst = make_instance(rhombohedral_lattice(BETA_A, BETA_ALPHA), (72, 72, 72), (2, 2, 2), 160, 12.0,
                             (3, 0), occ=occ, dtype=dtype or np.complex64, name="beta-boron-72^3-k222",
                             workers=workers)
    elif cid == "5":
        inst = make_instance(rhombohedral_lattice(BETA_A, BETA_ALPHA), (64, 64, 64), (1, 1, 1), 128, 12.0,
                             (5, 0), dtype=dtype or np.complex64, name="beta-boron-64^3-gamma", workers=workers)
    elif cid == "5s":
        inst = make_instance(rhombohedral_lattice(BETA_A, BETA_ALPHA), (24, 24, 24), (1, 1, 1), 16, 1.5,
                             (5, 1), dtype=dtype or np.complex128, name="beta-boron-24^3-subset", workers=workers)
    else:
        raise ValueError(f"unknown config {cfg_id!r}")
    return inst


def band_subset(inst, nbands):
    """The instance restricted to the first `nbands` bands of every k."""
    nb = max(1, min(int(nbands), inst.nbands))
    return Instance(inst.lattice, inst.grid, inst.kfrac, inst.kweight, np.ascontiguousarray(inst.occ[:, :nb]),
                    np.ascontiguousarray(inst.psi[:, :nb]), inst.mu, inst.ecut, f"{inst.name}-first{nb}",
                    dict(inst.extra))


def uneven_batch_params(n_inst=48, seed=4):
    """Shapes of the ragged batch: per instance (cell, grid, k-mesh, bands, E_cut)."""
    rng = np.random.default_rng([SEED_BASE, seed, 999_999])
    grids = [24, 32, 40, 48, 64]
    out = []
    for i in range(n_inst):
        edge = float(rng.uniform(9.0, 20.0))
        if rng.uniform() < 0.5:
            lat = cubic_lattice(edge)
        else:
            lat = rhombohedral_lattice(edge, float(rng.uniform(55.0, 70.0)))
        ng = int(grids[rng.integers(0, len(grids))])
        kmesh = (1, 1, 1) if rng.uniform() < 0.5 else (2, 2, 2)
        nb = int(rng.integers(8, 97))
        amax = float(np.max(np.linalg.norm(lat, axis=1)))
        ecut = min(12.0, 0.5 * (2.0 * np.pi * ((ng - 1) // 4) / amax) ** 2)
        out.append(dict(lattice=lat, grid=(ng, ng, ng), kmesh=kmesh, nbands=nb, ecut=ecut))
    return out


def uneven_batch(n_inst=48, dtype=np.complex64, seed=4, workers=None, params=None):
    """Config 4: independent instances of uneven band count, grid and k-mesh."""
    params = params if params is not None else uneven_batch_params(n_inst, seed)
    insts = []
    for i, p in enumerate(params):
        insts.append(make_instance(p["lattice"], p["grid"], p["kmesh"], p["nbands"], p["ecut"], (seed, i),
                                   dtype=dtype, name=f"uneven-{i}", workers=workers))
    return insts


def small_instance(grid=(12, 10, 9), kmesh=(2, 1, 1), nbands=3, seed=(100, 0), lattice=None,
                   full_grid=False, dtype=np.complex128, occ=None, ecut=None):
    """Tiny instances for tests: by default a skewed cell, a non-cubic grid
    and fractional occupations."""
    lattice = rhombohedral_lattice(7.0, 63.0) if lattice is None else np.asarray(lattice, dtype=np.float64)
    kfrac = gamma_mesh(*kmesh)
    nk = kfrac.shape[0]
    rng = np.random.default_rng([SEED_BASE, *seed, 10_000])
    if occ is None:
        occ = rng.uniform(0.2, 1.0, size=(nk, nbands))
    occ = np.broadcast_to(np.asarray(occ, dtype=np.float64), (nk, nbands)).copy()
    if full_grid:
        psi = random_grid_orbitals(grid, nk, nbands, rng, lattice).astype(dtype)
        return Instance(lattice, tuple(grid), kfrac, np.full(nk, 1.0 / nk), occ, psi, MU_HSE, None, "small-full")
    if ecut is None:
        # a sphere that fits every axis of this grid (|g_i| < N_i/2)
        amax = np.max(np.linalg.norm(lattice, axis=1))
        ecut = 0.5 * (2.0 * np.pi * (((min(grid) - 1) // 2) - 0.5) / amax) ** 2
    inst = make_instance(lattice, grid, kmesh, nbands, ecut, seed, occ=occ, dtype=dtype, name="small")
    return inst
