"""Host-side checks of the Python binding and of the C ABI's k-pair rule
that need no GPU: every per-instance list must have one entry per instance
(the library reads that many pointers), descriptors are checked for their
k-weight count, and the gradient of a plan whose k-pair list is not closed
under swapping is refused."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1111_0716_amd import fock, inputs


def host_plan(n_inst=2, nk=1, nb=2, grid=(8, 8, 8), prec="c64"):
    """A Plan object with the instance metadata of the real constructor but
    no library handle and no workspace (enough to reach the argument checks,
    which run before any library call)."""
    p = fock.Plan.__new__(fock.Plan)
    p.torch = torch
    p.precision = prec
    p.prec = fock.PRECISIONS[prec]
    p.cdtype = torch.complex64 if prec == "c64" else torch.complex128
    p.device = torch.device("cuda", 0)
    p.stream = None
    p.handle = None
    n = int(np.prod(grid))
    p.meta = [dict(nk=nk, nbands=nb, npts=n, omega=1000.0, band_stride=n) for _ in range(n_inst)]
    return p


def grids(p, count):
    m = p.meta[0]
    return [torch.zeros((m["nk"], m["nbands"], m["npts"]), dtype=p.cdtype) for _ in range(count)]


def occs(p, count):
    m = p.meta[0]
    return [torch.ones((m["nk"], m["nbands"]), dtype=torch.float64) for _ in range(count)]


@pytest.mark.parametrize("method", ["fock_apply", "fock_apply_energy", "fock_energy"])
def test_short_orbital_or_occupation_lists_raise(method):
    p = host_plan(n_inst=2)
    with pytest.raises(ValueError, match="entries"):
        getattr(p, method)(grids(p, 1), occs(p, 1))
    with pytest.raises(ValueError, match="entries"):
        getattr(p, method)(grids(p, 2), occs(p, 1))
    with pytest.raises(ValueError, match="entries"):
        getattr(p, method)(grids(p, 3), occs(p, 3))


def test_short_output_and_gradient_lists_raise():
    p = host_plan(n_inst=3)
    with pytest.raises(ValueError, match="entries"):
        p.fock_energy_backward(grids(p, 2), occs(p, 2), torch.ones(3), 1.0)
    with pytest.raises(ValueError, match="entries"):
        p.pw_to_grid(grids(p, 2), [torch.zeros((1, 4), dtype=torch.int32)] * 3, [torch.zeros(1, dtype=torch.int32)] * 3)
    with pytest.raises(ValueError, match="entries"):
        p.grid_to_pw(grids(p, 3), [torch.zeros((1, 4), dtype=torch.int32)] * 2, [torch.zeros(1, dtype=torch.int32)] * 3)
    with pytest.raises(ValueError, match="entries"):
        p.fock_apply_pw(grids(p, 3), [torch.zeros((1, 4), dtype=torch.int32)] * 3,
                        [torch.zeros(1, dtype=torch.int32)] * 3, occs(p, 2))


def test_host_tensors_are_refused():
    """CPU tensors never reach the library (it would read them as device pointers)."""
    p = host_plan(n_inst=1)
    with pytest.raises(ValueError, match="tensor on cuda"):
        p.fock_apply(grids(p, 1), occs(p, 1))


def test_kweight_count_must_match_k_points():
    with pytest.raises(ValueError, match="kweight"):
        fock.make_desc(inputs.cubic_lattice(10.0), (8, 8, 8), inputs.gamma_mesh(2, 1, 1), kweight=[1.0], nbands=2)
    d = fock.make_desc(inputs.cubic_lattice(10.0), (8, 8, 8), inputs.gamma_mesh(2, 1, 1), kweight=[0.3, 0.7],
                       nbands=2)
    assert d.nk == 2


def plan_handle(kpairs, nk=2):
    keep = []
    d = fock.make_desc(inputs.cubic_lattice(10.0), (8, 8, 8), inputs.gamma_mesh(nk, 1, 1), nbands=2,
                       kpairs=kpairs, keep=keep)
    arr = (fock.FockDesc * 1)(d)
    h = ctypes.c_void_p()
    assert fock.lib().fock_plan(arr, 1, fock.FOCK_C128, None, ctypes.byref(h)) == fock.FOCK_OK
    return h


def test_backward_refuses_k_pair_lists_not_closed_under_swapping():
    L = fock.lib()
    one = fock._ptrs([1])
    h = plan_handle([[0, 0], [0, 1], [1, 1]])
    assert L.fock_energy_backward(h, one, one, ctypes.c_void_p(1), 1.0, fock._ptrs([2])) == fock.FOCK_ERR_UNSUPPORTED
    assert b"swapping" in L.fock_last_error()
    L.fock_destroy(h)
    # a swap-closed explicit list passes this check (and stops at the missing workspace)
    h = plan_handle([[0, 0], [0, 1], [1, 0], [1, 1]])
    assert L.fock_energy_backward(h, one, one, ctypes.c_void_p(1), 1.0, fock._ptrs([2])) == fock.FOCK_ERR_STATE
    L.fock_destroy(h)
