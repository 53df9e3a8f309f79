"""Pins for the CPU FP64 oracle against what mathematics fixes independently
of its code: closed forms, brute force on tiny grids, the real-space form of
the kernel, invariances and finite differences.  A final group plants
plausible mistakes in a copy of the oracle and checks that a pin catches each.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

from oracle import fock_oracle as fo
from paper_1111_0716_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MU = 0.106


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                out[k.strip()] = float(v)
    return out


def cartesian_wavevector(lattice, x):
    """The Cartesian K of the plane wave exp(i K.r) whose phase advances by
    2 pi x_i along lattice vector a_i: the solution of a_i . K = 2 pi x_i.
    Solved directly from the lattice rows, so it does not go through the
    oracle's reciprocal basis."""
    return np.linalg.solve(np.asarray(lattice, dtype=np.float64), 2.0 * np.pi * np.asarray(x, dtype=np.float64))


def triclinic_lattice():
    """A cell with three different edges and angles: A A^T and A^T A differ,
    so the orientation of the reciprocal basis changes every |K|."""
    return np.array([[6.1, 0.3, -0.4], [1.2, 5.7, 0.5], [-0.8, 1.9, 6.6]])


def plane_wave(grid, g, omega):
    j = np.indices(grid).reshape(3, -1)
    ph = sum(2.0 * np.pi * g[i] * j[i] / grid[i] for i in range(3))
    return np.exp(1j * ph) / math.sqrt(omega)


# ----------------------------------------------------------------------------
# kernel
# ----------------------------------------------------------------------------
def test_kernel_golden_values():
    gold = read_golden("screened_kernel.txt")
    v = fo.screened_kernel(np.array([0.0, (2 * np.pi / 10) ** 2]), gold["mu"])
    assert v[0] == pytest.approx(gold["v_at_0"], rel=1e-15)
    assert v[1] == pytest.approx(gold["v_at_2pi_over_10"], rel=1e-14)


@pytest.mark.parametrize("r", [0.3, 1.0, 4.0, 12.0])
def test_kernel_is_fourier_transform_of_erfc_over_r(r):
    """4 pi/K^2 is the transform of 1/r, so 4 pi/K^2 - v(K) must be the
    transform of erf(mu r)/r, i.e. v is the transform of erfc(mu r)/r.
    Radial inverse transform: f(r) = 1/(2 pi^2 r) int_0^inf F(K) K sin(K r) dK."""
    def integrand(k):
        lr = 4 * np.pi / (k * k) - fo.screened_kernel(np.array([k * k]), MU)[0]
        return lr * k * math.sin(k * r)
    kmax = 2 * MU * 9.0  # exp(-81) tail
    val, err = integrate.quad(integrand, 1e-11, kmax, limit=400, epsabs=1e-13, epsrel=1e-12)
    f = val / (2 * np.pi ** 2 * r)
    assert f == pytest.approx(special.erf(MU * r) / r, rel=1e-10)


def test_kernel_small_and_large_k_limits():
    k2 = np.array([1e-12, 1e-8, 400.0])
    v = fo.screened_kernel(k2, MU)
    assert v[0] == pytest.approx(np.pi / MU ** 2, rel=1e-10)
    assert v[1] == pytest.approx(np.pi / MU ** 2, rel=1e-6)
    assert v[2] == pytest.approx(4 * np.pi / 400.0, rel=1e-14)


def test_kernel_table_alias_average_and_inversion_symmetry():
    """Slow per-class table equals the vectorised one, and the alias average
    makes v_{-q}(-c) = v_q(c) hold on even grids (it fails one-sided)."""
    lat = inputs.rhombohedral_lattice(7.0, 63.0)
    grid = (4, 6, 5)
    q = np.array([0.5, -0.25, 0.0])
    a = fo.kernel_table(lat, grid, q, MU)
    b = fo.kernel_table_fast(lat, grid, q, MU)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(a)
    bm = fo.kernel_table_fast(lat, grid, -q, MU)
    neg = bm[(-np.arange(4)) % 4][:, (-np.arange(6)) % 6][:, :, (-np.arange(5)) % 5]
    assert np.max(np.abs(neg - b)) <= 1e-13 * np.max(b)


# ----------------------------------------------------------------------------
# DFT
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("grid", [(4, 6, 5), (6, 4, 8), (3, 5, 2)])
def test_separable_dft_matches_full_dft(grid):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(grid) + 1j * rng.standard_normal(grid)
    j = np.indices(grid).reshape(3, -1)
    ph = sum(np.outer(j[i], j[i]) / grid[i] for i in range(3))
    full = np.exp(-2j * np.pi * ph)  # [c, j], non-separable O(N^2) matrix
    d = fo.DFT3(grid)
    assert np.allclose(d.forward(x).reshape(-1), full @ x.reshape(-1), rtol=0, atol=1e-12)
    assert np.allclose(d.inverse(d.forward(x)), x, rtol=0, atol=1e-13)
    # Parseval: sum |P|^2 = N sum |x|^2
    p = d.forward(x)
    assert np.sum(np.abs(p) ** 2) == pytest.approx(x.size * np.sum(np.abs(x) ** 2), rel=1e-13)
    # numpy's FFT uses the same sign and scaling conventions
    assert np.allclose(d.forward(x), np.fft.fftn(x), atol=1e-12)


# ----------------------------------------------------------------------------
# the operator: brute force through a dense real-space kernel
# ----------------------------------------------------------------------------
def dense_reference(inst):
    """V_x u and E_x with an explicit N x N real-space kernel per transfer q,
    K_q(a, b) = (1/N) sum_c v_q(c) exp(2 pi i c.(j_a - j_b)/N)."""
    grid = inst.grid
    n = int(np.prod(grid))
    omega = abs(np.linalg.det(inst.lattice))
    dv = omega / n
    j = np.indices(grid).reshape(3, -1)
    ph = sum(np.outer(j[i], j[i]) / grid[i] for i in range(3))
    f = np.exp(-2j * np.pi * ph)  # f[c, a]
    nk, nb, _ = inst.psi.shape
    vx = np.zeros((nk, nb, n), complex)
    ex = 0.0
    for ik in range(nk):
        for jk in range(nk):
            v = fo.kernel_table(inst.lattice, grid, inst.kfrac[ik] - inst.kfrac[jk], inst.mu).reshape(-1)
            kmat = (f.conj().T * v[None, :]) @ f / n
            for ib in range(nb):
                for jb in range(nb):
                    rho = np.conj(inst.psi[jk, jb]) * inst.psi[ik, ib]
                    krho = kmat @ rho
                    cf = inst.kweight[jk] * inst.occ[jk, jb]
                    vx[ik, ib] -= cf * inst.psi[jk, jb] * krho
                    ex -= 0.5 * inst.kweight[ik] * inst.occ[ik, ib] * cf * dv * np.vdot(rho, krho).real
    return vx, ex


@pytest.mark.parametrize("grid,kmesh,full", [((4, 6, 5), (2, 1, 1), True), ((6, 4, 4), (1, 2, 2), True),
                                              ((5, 5, 6), (1, 1, 1), False)])
def test_oracle_matches_dense_real_space_kernel(grid, kmesh, full):
    inst = inputs.small_instance(grid=grid, kmesh=kmesh, nbands=2, seed=(101, grid[0]), full_grid=full)
    o = fo.Oracle.from_instance(inst)
    vx, ex = o.apply(inst.psi, inst.occ)
    vref, eref = dense_reference(inst)
    assert np.max(np.abs(vx - vref)) <= 1e-12 * np.max(np.abs(vref))
    assert ex == pytest.approx(eref, rel=1e-12)


# ----------------------------------------------------------------------------
# closed forms
# ----------------------------------------------------------------------------
def test_plane_wave_gamma_golden():
    gold = read_golden("plane_wave_closed_form.txt")
    lat = inputs.cubic_lattice(10.0)
    grid = (16, 16, 16)
    o = fo.Oracle(lat, grid, np.zeros((1, 3)), None, MU)
    u1 = plane_wave(grid, (0, 0, 0), 1000.0)[None, None]
    assert o.energy(u1, np.ones((1, 1))) == pytest.approx(gold["one_band_gamma_Ex"], rel=1e-14)
    u2 = np.stack([plane_wave(grid, (0, 0, 0), 1000.0), plane_wave(grid, (1, 0, 0), 1000.0)])[None]
    vx, ex = o.apply(u2, np.ones((1, 2)))
    assert ex == pytest.approx(gold["two_band_gamma_Ex"], rel=1e-14)
    assert o.energy(u2, np.ones((1, 2))) == pytest.approx(gold["two_band_gamma_Ex"], rel=1e-14)


def test_plane_wave_eigenvalues_on_k_mesh():
    """Skewed cell, non-cubic grid, 2x2x1 mesh, fractional f, weights: each
    plane wave is an eigenvector of V_x with
    eps_kn = -(1/Omega) sum_k' w_k' sum_m f_k'm v(G_n - G_m + k - k')."""
    lat = inputs.rhombohedral_lattice(6.5, 61.0)
    grid = (8, 6, 10)
    kfrac = inputs.gamma_mesh(2, 2, 1) + np.array([0.125, 0.0, 0.05])
    kw = np.array([0.1, 0.2, 0.3, 0.4])
    nk, nb = 4, 3
    rng = np.random.default_rng(7)
    gs = rng.integers(-1, 2, size=(nk, nb, 3))
    gs[:, 1] += np.array([1, 0, 0])
    gs[:, 2] += np.array([0, 0, 2])
    occ = rng.uniform(0.1, 1.0, size=(nk, nb))
    omega = abs(np.linalg.det(lat))
    psi = np.stack([np.stack([plane_wave(grid, gs[k, n], omega) for n in range(nb)]) for k in range(nk)])
    o = fo.Oracle(lat, grid, kfrac, kw, MU)
    vx, ex = o.apply(psi, occ)
    eps = np.zeros((nk, nb))
    for k in range(nk):
        for n in range(nb):
            s = 0.0
            for kp in range(nk):
                for m in range(nb):
                    d = gs[k, n] - gs[kp, m]
                    assert np.all(2 * np.abs(d) < np.array(grid))  # no class reduction needed
                    kc = cartesian_wavevector(lat, d + kfrac[k] - kfrac[kp])
                    s += kw[kp] * occ[kp, m] * fo.screened_kernel(np.array([kc @ kc]), MU)[0]
            eps[k, n] = -s / omega
    for k in range(nk):
        for n in range(nb):
            assert np.allclose(vx[k, n], eps[k, n] * psi[k, n], rtol=0, atol=1e-13 * abs(eps[k, n]) / math.sqrt(omega))
    ex_cf = 0.5 * np.sum(kw[:, None] * occ * eps)
    assert ex == pytest.approx(ex_cf, rel=1e-13)


def test_constant_kernel_special_case():
    """v == c turns the FFT round trip into the identity:
    V_x u_n = -c sum w f |u_m|^2 u_n,  E_x = -(c/2) dV sum_j (sum w f |u|^2)^2."""
    inst = inputs.small_instance(grid=(6, 5, 4), kmesh=(2, 1, 1), nbands=3, seed=(102, 0), full_grid=True)
    c = 2.75
    o = fo.Oracle.from_instance(inst, kernel=c)
    vx, ex = o.apply(inst.psi, inst.occ)
    dens = np.sum(inst.kweight[:, None, None] * inst.occ[:, :, None] * np.abs(inst.psi) ** 2, axis=(0, 1))
    assert np.allclose(vx, -c * dens[None, None, :] * inst.psi, rtol=0, atol=1e-13 * np.max(np.abs(vx)))
    dv = abs(np.linalg.det(inst.lattice)) / inst.npoints
    assert ex == pytest.approx(-0.5 * c * dv * np.sum(dens ** 2), rel=1e-13)


# ----------------------------------------------------------------------------
# cell geometry: the reciprocal basis and rigid rotations of the cell
# ----------------------------------------------------------------------------
def test_reciprocal_rows_are_dual_to_the_lattice():
    """a_i . b_j = 2 pi delta_ij, and row i of the basis is the wave vector
    whose phase advances by 2 pi along a_i only (solved from the lattice)."""
    lat = triclinic_lattice()
    b = fo.reciprocal_rows(lat)
    assert np.allclose(lat @ b.T, 2.0 * np.pi * np.eye(3), rtol=0, atol=1e-13)
    for i in range(3):
        assert np.allclose(b[i], cartesian_wavevector(lat, np.eye(3)[i]), rtol=0, atol=1e-13)


def _kernel_table_cartesian_error():
    """Largest relative gap between the oracle's table and v(|K|) with K
    solved from the lattice, on every class of an odd grid (one
    representative per class) of a triclinic cell at a fractional transfer."""
    lat = triclinic_lattice()
    grid = (5, 3, 7)
    q = np.array([0.25, -0.5, 0.125])
    tab = fo.kernel_table_fast(lat, grid, q, MU)
    ref = np.empty(grid)
    for c in np.ndindex(*grid):
        g = np.array([ci if 2 * ci < n else ci - n for ci, n in zip(c, grid)], dtype=np.float64)
        kc = cartesian_wavevector(lat, g + q)
        ref[c] = fo.screened_kernel(np.array([kc @ kc]), MU)[0]
    return float(np.max(np.abs(tab - ref)) / np.max(ref))


def test_kernel_table_matches_cartesian_wave_vectors():
    assert _kernel_table_cartesian_error() <= 1e-14


def rotation_matrix(seed):
    """A proper rotation (det +1) drawn from a seeded normal matrix."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _rotation_error(inst):
    """Relative change of E_x and V_x u when every lattice vector is turned
    by the same rotation R (a_i -> R a_i) while the grid values of the
    orbitals, the fractional k-points and the weights stay as they are: a
    rigid rotation of the whole crystal, which changes no physical result."""
    o = fo.Oracle.from_instance(inst)
    vx, ex = o.apply(inst.psi, inst.occ)
    r = rotation_matrix(11)
    rot = fo.Oracle(inst.lattice @ r.T, inst.grid, inst.kfrac, inst.kweight, inst.mu)
    vr, er = rot.apply(inst.psi, inst.occ)
    return max(abs(er - ex) / abs(ex), float(np.max(np.abs(vr - vx)) / np.max(np.abs(vx))))


@pytest.fixture(scope="module")
def triclinic_instance():
    return inputs.small_instance(grid=(6, 4, 5), kmesh=(2, 2, 1), nbands=2, seed=(104, 0),
                                 lattice=triclinic_lattice(), full_grid=True)


def test_rigid_rotation_of_the_cell_changes_nothing(triclinic_instance):
    assert _rotation_error(triclinic_instance) <= 1e-13


# ----------------------------------------------------------------------------
# identities and invariants
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def skewed():
    inst = inputs.small_instance(grid=(6, 4, 5), kmesh=(2, 2, 1), nbands=3, seed=(103, 0), full_grid=True)
    o = fo.Oracle.from_instance(inst)
    vx, ex = o.apply(inst.psi, inst.occ)
    return inst, o, vx, ex


def test_energy_routes_agree_and_sign(skewed):
    inst, o, vx, ex = skewed
    assert ex < 0
    assert o.energy(inst.psi, inst.occ) == pytest.approx(ex, rel=1e-13)
    assert o.energy_from_apply(inst.psi, inst.occ, vx) == pytest.approx(ex, rel=1e-13)


def test_overlap_hermitian_negative_semidefinite(skewed):
    inst, o, vx, ex = skewed
    m = o.overlap(inst.psi, vx)
    for k in range(m.shape[0]):
        assert np.max(np.abs(m[k] - m[k].conj().T)) <= 1e-14 * np.max(np.abs(m[k]))
        assert np.max(np.linalg.eigvalsh(m[k])) <= 1e-14 * np.max(np.abs(m[k]))
    tr = 0.5 * np.sum(inst.kweight[:, None] * inst.occ * np.real(np.einsum("kii->ki", m)))
    assert tr == pytest.approx(ex, rel=1e-13)


def test_pair_energy_swap_symmetry(skewed):
    inst, o, vx, ex = skewed
    rng = np.random.default_rng(3)
    for _ in range(6):
        ik, jk = rng.integers(0, inst.nk, 2)
        ib, jb = rng.integers(0, inst.nbands, 2)
        e1, e2 = o.pair_energies(inst.psi, [(ik, ib, jk, jb), (jk, jb, ik, ib)])
        assert e1 == pytest.approx(e2, rel=1e-13)


def test_finite_difference_gradient(skewed):
    inst, o, vx, ex = skewed
    g = o.gradient(inst.psi, inst.occ, vx)  # torch convention
    rng = np.random.default_rng(4)
    h = 1e-5
    for _ in range(3):
        d = rng.standard_normal(inst.psi.shape) + 1j * rng.standard_normal(inst.psi.shape)
        d /= np.linalg.norm(d)
        fd = (o.energy(inst.psi + h * d, inst.occ) - o.energy(inst.psi - h * d, inst.occ)) / (2 * h)
        an = np.real(np.vdot(g, d))
        assert abs(fd - an) <= 1e-8 * np.linalg.norm(g)


def test_band_rotation_and_phase_invariance(skewed):
    inst, o, vx, ex = skewed
    occ = np.ones_like(inst.occ)
    vx0, e0 = o.apply(inst.psi, occ)
    rng = np.random.default_rng(5)
    psi2 = np.empty_like(inst.psi)
    us = []
    for k in range(inst.nk):
        a = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        u, _ = np.linalg.qr(a)
        us.append(u)
        psi2[k] = u.T @ inst.psi[k]
    vx2, e2 = o.apply(psi2, occ)
    assert e2 == pytest.approx(e0, rel=1e-13)
    for k in range(inst.nk):
        assert np.allclose(vx2[k], us[k].T @ vx0[k], atol=1e-13 * np.max(np.abs(vx0)))
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, size=(inst.nk, 3)))
    vx3, e3 = o.apply(inst.psi * ph[:, :, None], occ)
    assert e3 == pytest.approx(e0, rel=1e-13)
    assert np.allclose(vx3, vx0 * ph[:, :, None], atol=1e-13 * np.max(np.abs(vx0)))


def test_translation_and_mesh_shift_invariance(skewed):
    inst, o, vx, ex = skewed
    g = inst.grid
    sh = (1, 3, 2)
    roll = lambda a: np.roll(a.reshape(a.shape[:-1] + g), sh, axis=(-3, -2, -1)).reshape(a.shape)
    vxr, exr = o.apply(roll(inst.psi), inst.occ)
    assert exr == pytest.approx(ex, rel=1e-13)
    assert np.allclose(vxr, roll(vx), atol=1e-13 * np.max(np.abs(vx)))
    o2 = fo.Oracle(inst.lattice, g, inst.kfrac + np.array([0.25, 0.25, 0.25]), inst.kweight, inst.mu)
    vxs, exs = o2.apply(inst.psi, inst.occ)
    assert exs == pytest.approx(ex, rel=1e-13)
    assert np.allclose(vxs, vx, atol=1e-13 * np.max(np.abs(vx)))


# ----------------------------------------------------------------------------
# planted mistakes: each must be caught by one of the pins above
# ----------------------------------------------------------------------------
class _OneSidedNyquist(fo.Oracle):
    def v(self, ik, jk):
        q = self.kfrac[ik] - self.kfrac[jk]
        b = fo.reciprocal_rows(self.lattice)
        fr = [np.fft.fftfreq(n, 1.0 / n) + qi for n, qi in zip(self.grid, q)]
        x1, x2, x3 = np.meshgrid(*fr, indexing="ij")
        kc = np.stack([x1, x2, x3], -1) @ b
        return fo.screened_kernel(np.sum(kc * kc, -1), self.mu)


class _FlippedSign(fo.Oracle):
    def pair(self, u_n, u_m, v):
        rho = np.conj(u_m) * u_n
        p = self.dft.inverse(rho) * self.n
        w = self.dft.forward(v * p) / self.n
        return float(np.sum(v * np.abs(p) ** 2)), w.reshape(-1)


class _WrongConj(fo.Oracle):
    def pair(self, u_n, u_m, v):
        return super().pair(np.conj(u_n), np.conj(u_m), v)


class _FoldedQ(fo.Oracle):
    def v(self, ik, jk):
        q = self.kfrac[jk] - self.kfrac[ik]  # transfer taken the wrong way round
        return fo.kernel_table_fast(self.lattice, self.grid, q, self.mu)


def _closed_form_error(cls):
    lat = inputs.rhombohedral_lattice(6.5, 61.0)
    grid = (8, 6, 10)
    kfrac = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0]])
    omega = abs(np.linalg.det(lat))
    gs = [[(1, 0, 0), (0, 1, -1)], [(0, 0, 1), (-1, 0, 0)]]
    psi = np.array([[plane_wave(grid, g, omega) for g in row] for row in gs])
    good = fo.Oracle(lat, grid, kfrac, None, MU).apply(psi, np.ones((2, 2)))[0]
    bad = cls(lat, grid, kfrac, None, MU).apply(psi, np.ones((2, 2)))[0]
    return np.max(np.abs(bad - good)) / np.max(np.abs(good))


@pytest.mark.parametrize("cls", [_FlippedSign, _WrongConj, _FoldedQ])
def test_planted_mistakes_break_closed_form(cls):
    assert _closed_form_error(cls) > 1e-3


def test_planted_one_sided_nyquist_breaks_gradient(skewed):
    inst, _, _, _ = skewed
    o = _OneSidedNyquist.from_instance(inst)
    vx, _ = o.apply(inst.psi, inst.occ)
    g = o.gradient(inst.psi, inst.occ, vx)
    rng = np.random.default_rng(4)
    d = rng.standard_normal(inst.psi.shape) + 1j * rng.standard_normal(inst.psi.shape)
    d /= np.linalg.norm(d)
    h = 1e-5
    fd = (o.energy(inst.psi + h * d, inst.occ) - o.energy(inst.psi - h * d, inst.occ)) / (2 * h)
    assert abs(fd - np.real(np.vdot(g, d))) > 1e-6 * np.linalg.norm(g)


def test_planted_transposed_reciprocal_basis_is_caught(triclinic_instance, monkeypatch):
    """b taken as the rows of 2 pi A^-1 instead of 2 pi A^-T: the Cartesian
    wave-vector pin and the rigid-rotation pin both reject it."""
    monkeypatch.setattr(fo, "reciprocal_rows",
                        lambda lat: 2.0 * np.pi * np.linalg.inv(np.asarray(lat, dtype=np.float64)))
    assert _kernel_table_cartesian_error() > 1e-3
    assert _rotation_error(triclinic_instance) > 1e-3


# ----------------------------------------------------------------------------
# the gradient formula and the k-pair list
# ----------------------------------------------------------------------------
def test_gradient_formula_needs_a_symmetric_k_pair_list():
    """dE_x/du* = dV w f V_x u needs every listed (k, k') to have its swap
    (k', k) listed too.  For a list that is not closed under swapping, the
    derivative of Eq. (2)'s double sum takes each pair once as output and
    once as partner: it is the mean of the operator over the list and over
    its transpose.  The oracle refuses the short formula there; finite
    differences confirm the mean and reject the short formula."""
    inst = inputs.small_instance(grid=(6, 4, 5), kmesh=(2, 1, 1), nbands=2, seed=(105, 0), full_grid=True)
    kp = np.array([[0, 0], [0, 1], [1, 1]])
    o = fo.Oracle.from_instance(inst, kpairs=kp)
    with pytest.raises(ValueError):
        o.gradient(inst.psi, inst.occ)
    vl, _ = o.apply(inst.psi, inst.occ)
    vt, _ = fo.Oracle.from_instance(inst, kpairs=kp[:, ::-1]).apply(inst.psi, inst.occ)
    wf = inst.kweight[:, None, None] * inst.occ[:, :, None]
    g_mean = o.dv * wf * (vl + vt)       # torch convention: 2 dV w f (V^L + V^T)/2
    g_short = 2.0 * o.dv * wf * vl
    rng = np.random.default_rng(6)
    h = 1e-5
    for _ in range(3):
        d = rng.standard_normal(inst.psi.shape) + 1j * rng.standard_normal(inst.psi.shape)
        d /= np.linalg.norm(d)
        fd = (o.energy(inst.psi + h * d, inst.occ) - o.energy(inst.psi - h * d, inst.occ)) / (2 * h)
        assert abs(fd - np.real(np.vdot(g_mean, d))) <= 1e-8 * np.linalg.norm(g_mean)
        assert abs(fd - np.real(np.vdot(g_short, d))) > 1e-4 * np.linalg.norm(g_mean)
    # a symmetric explicit list is accepted and equals the full set
    full = np.array([[0, 0], [0, 1], [1, 0], [1, 1]])
    o2 = fo.Oracle.from_instance(inst, kpairs=full)
    g2 = o2.gradient(inst.psi, inst.occ)
    g3 = fo.Oracle.from_instance(inst).gradient(inst.psi, inst.occ)
    assert np.allclose(g2, g3, rtol=0, atol=1e-15 * np.max(np.abs(g3)))
