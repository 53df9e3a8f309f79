"""CPU FP64 oracle for the plane-wave boundary of the exchange path and for
the plain 3-D DFT.

TEST INFRASTRUCTURE ONLY.  Only the test suite may import or run this module;
the library path never calls it.  It shares no code with the HIP library
(it uses the direct DFT of fock_oracle, which is part of the same oracle).

A plane-wave code stores each orbital as coefficients c(G) on the cutoff
sphere |k+G|^2/2 < E_cut; the band-pair loop works on the FFT grid, and the
results go back to the sphere (paper, "CPU Performance Analysis": the
scatter/gather between cutoff sphere and grid around the FFTs of FOCK_ACC).
With psi(r) = Omega^-1/2 sum_G c(G) exp(i (k+G).r) and u = psi exp(-i k.r):

  to the grid    u[j] = Omega^-1/2 sum_G c(G) exp(+2 pi i sum_i c_i j_i / N_i)
  to the sphere  d(G) = <exp(i(k+G).r) Omega^-1/2 | f> = (Omega^1/2 / N) sum_j f[j] exp(-2 pi i sum_i c_i j_i / N_i)

for the grid class c_i = g_i mod N_i of G.  The second is the exact
coefficient of f on the sphere, so for band-limited orbitals
sum_G conj(c_m(G)) d_n(G) = dV sum_j conj(u_m[j]) f_n[j].

Sphere layout (as the library takes it): for each k, gidx[k][p] is the flat
grid class (c1 N2 + c2) N3 + c3 of slot p < npw[k]; coefficients are
[nk][nbands][npw_max] and slots p >= npw[k] are zero.
"""
from __future__ import annotations

import numpy as np

from oracle.fock_oracle import DFT3


def grid_classes(g, grid):
    """Flat grid class (c1 N2 + c2) N3 + c3, c_i = g_i mod N_i, of integer G rows."""
    g = np.asarray(g, dtype=np.int64)
    n1, n2, n3 = grid
    return ((g[:, 0] % n1) * n2 + (g[:, 1] % n2)) * n3 + (g[:, 2] % n3)


def dft3(x, grid, sign):
    """Unnormalised 3-D DFT with exp(sign 2 pi i c.j/N) of one grid (flat)."""
    d = DFT3(grid)
    out = d.forward(x) if sign < 0 else d.inverse(x) * d.n
    return out.reshape(-1)


def pw_to_grid(lattice, grid, gidx, npw, coef):
    """u[k][n] from sphere coefficients coef[k][n][p] (p < npw[k])."""
    omega = abs(np.linalg.det(np.asarray(lattice, dtype=np.float64)))
    coef = np.asarray(coef)
    nk, nb = coef.shape[:2]
    n = int(np.prod(grid))
    u = np.zeros((nk, nb, n), dtype=np.complex128)
    for k in range(nk):
        idx = np.asarray(gidx[k][: npw[k]], dtype=np.int64)
        for b in range(nb):
            box = np.zeros(n, dtype=np.complex128)
            box[idx] = coef[k, b, : npw[k]]
            u[k, b] = dft3(box, grid, +1) / np.sqrt(omega)
    return u


def grid_to_pw(lattice, grid, gidx, npw, npw_max, f):
    """Sphere coefficients d[k][n][p] of grid functions f[k][n] (zero past npw[k])."""
    omega = abs(np.linalg.det(np.asarray(lattice, dtype=np.float64)))
    f = np.asarray(f)
    nk, nb = f.shape[:2]
    n = int(np.prod(grid))
    d = np.zeros((nk, nb, npw_max), dtype=np.complex128)
    for k in range(nk):
        idx = np.asarray(gidx[k][: npw[k]], dtype=np.int64)
        for b in range(nb):
            d[k, b, : npw[k]] = dft3(f[k, b], grid, -1)[idx] * (np.sqrt(omega) / n)
    return d
