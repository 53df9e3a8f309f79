"""Seeded input generator: orthonormality, reproducibility, cutoff sphere and
the shapes of the boron-like presets."""
import numpy as np
import pytest

from paper_1111_0716_amd import inputs


def test_rhombohedral_cell_volume_and_angles():
    lat = inputs.rhombohedral_lattice(9.56, 58.0)
    vol = abs(np.linalg.det(lat))
    ca = np.cos(np.deg2rad(58.0))
    assert vol == pytest.approx(9.56 ** 3 * np.sqrt(1 - 3 * ca ** 2 + 2 * ca ** 3), rel=1e-13)
    for i in range(3):
        assert np.linalg.norm(lat[i]) == pytest.approx(9.56, rel=1e-14)
        for j in range(i + 1, 3):
            assert lat[i] @ lat[j] == pytest.approx(9.56 ** 2 * ca, rel=1e-13)
    b = inputs.reciprocal_rows(lat)
    assert np.allclose(lat @ b.T, 2 * np.pi * np.eye(3), atol=1e-13)


def test_config1_orthonormal_and_reproducible():
    a = inputs.config(1)
    b = inputs.config(1)
    assert a.psi.shape == (1, 8, 4096) and a.psi.dtype == np.complex128
    assert np.array_equal(a.psi, b.psi)
    dv = abs(np.linalg.det(a.lattice)) / a.npoints
    s = dv * a.psi[0].conj() @ a.psi[0].T
    assert np.allclose(s, np.eye(8), atol=1e-13)


def test_orbitals_live_on_the_cutoff_sphere():
    inst = inputs.small_instance(grid=(12, 10, 9), kmesh=(2, 1, 1), nbands=3, seed=(104, 0))
    for ik in range(inst.nk):
        g = inputs.sphere_indices(inst.lattice, inst.kfrac[ik], inst.ecut, inst.grid)
        mask = np.zeros(inst.grid, bool)
        mask[g[:, 0] % 12, g[:, 1] % 10, g[:, 2] % 9] = True
        c = np.fft.fftn(inst.psi[ik].reshape((3,) + inst.grid), axes=(1, 2, 3))
        assert np.max(np.abs(c[:, ~mask])) <= 1e-12 * np.max(np.abs(c))


def test_config3_occupations_and_shapes_without_orbitals(monkeypatch):
    # The 72^3 orbitals are large; check the occupation recipe and the sphere size only.
    lat = inputs.rhombohedral_lattice(inputs.BETA_A, inputs.BETA_ALPHA)
    g = inputs.sphere_indices(lat, np.zeros(3), 12.0, (72, 72, 72))
    assert len(g) >= 160
    span = 2 * np.max(np.abs(g), axis=0) + 1
    assert np.all(span <= 72)
    rng = np.random.default_rng([inputs.SEED_BASE, 3, 0, 1_000_000])
    f = rng.uniform(0.05, 0.95, size=8)
    assert np.all((f > 0.05) & (f < 0.95))


def test_uneven_batch_params_reproducible():
    p1 = inputs.uneven_batch_params()
    p2 = inputs.uneven_batch_params()
    assert len(p1) == 48
    for a, b in zip(p1, p2):
        assert a["grid"] == b["grid"] and a["nbands"] == b["nbands"] and a["kmesh"] == b["kmesh"]
        assert 8 <= a["nbands"] <= 96 and a["grid"][0] in (24, 32, 40, 48, 64)


def test_band_subset_keeps_the_first_bands():
    inst = inputs.small_instance(grid=(8, 6, 10), kmesh=(2, 1, 1), nbands=5, seed=(330, 0))
    sub = inputs.band_subset(inst, 3)
    assert sub.nbands == 3 and sub.nk == inst.nk
    assert np.array_equal(sub.psi, inst.psi[:, :3]) and np.array_equal(sub.occ, inst.occ[:, :3])
    assert sub.psi.flags["C_CONTIGUOUS"]
