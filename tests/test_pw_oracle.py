"""Pins of the plane-wave boundary oracle (oracle/pw_oracle.py) against what
the mathematics fixes: the closed form of one plane wave, the library FFT
(numpy), the input generator's own placement, Parseval, the round trip,
exact projection identities, and planted mistakes that the pins must catch."""
import numpy as np
import pytest

from oracle import pw_oracle as pw
from oracle.fock_oracle import Oracle
from paper_1111_0716_amd import inputs


def sphere(inst, ecut):
    g = [inputs.sphere_indices(inst.lattice, inst.kfrac[k], ecut, inst.grid) for k in range(inst.nk)]
    npw = [len(x) for x in g]
    npw_max = max(npw)
    gidx = np.zeros((inst.nk, npw_max), dtype=np.int64)
    for k, x in enumerate(g):
        gidx[k, : len(x)] = pw.grid_classes(x, inst.grid)
    return g, gidx, np.array(npw), npw_max


def test_single_plane_wave_closed_form():
    lat = inputs.rhombohedral_lattice(7.0, 63.0)
    grid = (6, 5, 8)
    omega = abs(np.linalg.det(lat))
    g0 = np.array([[1, -2, 3]])
    gidx = [pw.grid_classes(g0, grid)]
    u = pw.pw_to_grid(lat, grid, gidx, [1], np.ones((1, 1, 1)))[0, 0].reshape(grid)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), axis=-1)
    want = np.exp(2j * np.pi * (j[..., 0] * 1 / 6 + j[..., 1] * (-2) / 5 + j[..., 2] * 3 / 8)) / np.sqrt(omega)
    assert np.max(np.abs(u - want)) < 1e-14
    # and back: the coefficient of that plane wave is 1
    d = pw.grid_to_pw(lat, grid, gidx, [1], 1, u.reshape(1, 1, -1))
    assert abs(d[0, 0, 0] - 1.0) < 1e-13


@pytest.mark.parametrize("grid", [(4, 6, 5), (8, 8, 8), (9, 10, 12)])
def test_dft3_is_the_library_fft(grid):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(int(np.prod(grid))) + 1j * rng.standard_normal(int(np.prod(grid)))
    f = pw.dft3(x, grid, -1).reshape(grid)
    assert np.allclose(f, np.fft.fftn(x.reshape(grid)), rtol=0, atol=1e-11)
    b = pw.dft3(x, grid, +1).reshape(grid)
    assert np.allclose(b, np.fft.ifftn(x.reshape(grid)) * np.prod(grid), rtol=0, atol=1e-11)


def test_grid_placement_matches_input_generator_and_round_trip():
    inst = inputs.small_instance(grid=(12, 10, 9), kmesh=(2, 1, 1), nbands=3, seed=(40, 1))
    ecut = inst.ecut
    g, gidx, npw, npw_max = sphere(inst, ecut)
    rng = np.random.default_rng(4)
    coef = np.zeros((inst.nk, inst.nbands, npw_max), dtype=np.complex128)
    for k in range(inst.nk):
        coef[k, :, : npw[k]] = rng.standard_normal((inst.nbands, npw[k])) + 1j * rng.standard_normal((inst.nbands, npw[k]))
    u = pw.pw_to_grid(inst.lattice, inst.grid, gidx, npw, coef)
    for k in range(inst.nk):
        ref = inputs.coefficients_to_grid(inst.lattice, inst.grid, g[k], coef[k, :, : npw[k]].T)
        assert np.max(np.abs(u[k] - ref)) < 1e-13 * np.max(np.abs(ref))
    back = pw.grid_to_pw(inst.lattice, inst.grid, gidx, npw, npw_max, u)
    assert np.max(np.abs(back - coef)) < 1e-12
    # Parseval: sum |c|^2 = dV sum |u|^2
    dv = abs(np.linalg.det(inst.lattice)) / np.prod(inst.grid)
    assert np.allclose(np.sum(np.abs(coef) ** 2, axis=-1), dv * np.sum(np.abs(u) ** 2, axis=-1), rtol=1e-12)


def test_projection_identity_and_exchange_on_the_sphere():
    """For band-limited u_m and any grid f: sum_G conj(c_m) d_f(G) = dV sum conj(u_m) f.
    With f = V_x u_n this is the band overlap M of the grid oracle."""
    inst = inputs.small_instance(grid=(10, 12, 9), kmesh=(2, 1, 1), nbands=3, seed=(41, 2))
    g, gidx, npw, npw_max = sphere(inst, inst.ecut)
    coef = pw.grid_to_pw(inst.lattice, inst.grid, gidx, npw, npw_max, inst.psi)
    # the generated orbitals live on the sphere: they come back exactly
    assert np.max(np.abs(pw.pw_to_grid(inst.lattice, inst.grid, gidx, npw, coef) - inst.psi)) < 1e-12
    o = Oracle.from_instance(inst)
    vx, _ = o.apply(inst.psi, inst.occ)
    d = pw.grid_to_pw(inst.lattice, inst.grid, gidx, npw, npw_max, vx)
    m_grid = o.overlap(inst.psi, vx)
    m_pw = np.einsum("kip,kjp->kij", coef.conj(), d)
    assert np.max(np.abs(m_pw - m_grid)) < 1e-12 * np.max(np.abs(m_grid))


def test_planted_mistakes_are_caught():
    """Each variant below breaks one convention; a pin above must reject it."""
    lat = inputs.cubic_lattice(6.0)
    grid = (6, 6, 6)
    omega = abs(np.linalg.det(lat))
    g0 = np.array([[1, 0, 2]])
    gidx = [pw.grid_classes(g0, grid)]
    good = pw.pw_to_grid(lat, grid, gidx, [1], np.ones((1, 1, 1)))[0, 0]
    # wrong sign of the exponent: conjugated plane wave
    wrong_sign = np.conj(good)
    # missing 1/sqrt(Omega)
    wrong_scale = good * np.sqrt(omega)
    # class taken as -g mod N (a transposed index convention)
    wrong_class = pw.pw_to_grid(lat, grid, [pw.grid_classes(-g0, grid)], [1], np.ones((1, 1, 1)))[0, 0]
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), axis=-1).reshape(-1, 3)
    want = np.exp(2j * np.pi * (j @ np.array([1, 0, 2])) / 6) / np.sqrt(omega)
    assert np.max(np.abs(good - want)) < 1e-14
    for bad in (wrong_sign, wrong_scale, wrong_class):
        assert np.max(np.abs(bad - want)) > 1e-3
