"""CPU FP64 oracle for the screened exact-exchange (Fock) operator.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the CPU-baseline leg of the benchmark may import or run this module; the
library path never calls it.  It shares no code with the HIP library.

What it computes (paper, section "Our Implementation", Eq. (2): the exchange
energy as a double sum over k-point pairs and band pairs of the Coulomb
interaction of band co-densities, here with the screened kernel), recast on
the FFT grid:

  cell      A (rows a_i, bohr), Omega = |det A|, B = 2 pi A^-T (rows b_i),
            N = N1 N2 N3 grid points, dV = Omega / N
  orbitals  u[k][n][j]: periodic part of the Bloch orbital on grid point
            j = (j1*N2 + j2)*N3 + j3 at r = sum_i (j_i/N_i) a_i
  pair      rho = conj(u[k'][m]) * u[k][n]
            P   = DFT(rho),  P(c) = sum_j rho_j exp(-2 pi i sum_i c_i j_i / N_i)
            e   = sum_c v_q(c) |P(c)|^2
            W   = IDFT(v_q * P)  (inverse carries 1/N)
            (V_x u)[k][n] += -w_k' f[k'][m] u[k'][m] * W
  energy    E_x = -1/2 sum w_k f[k][n] w_k' f[k'][m] (Omega/N^2) e
  overlap   M[k][i][j] = dV sum_j conj(u[k][i]) (V_x u)[k][j]
  gradient  dE_x / d conj(u[k][n]) = dV w_k f[k][n] (V_x u)[k][n]
            (torch's complex gradient convention is twice that)

Kernel: v(K) = 4 pi / |K|^2 * (1 - exp(-|K|^2 / (4 mu^2))) with the K -> 0
limit pi / mu^2 (the short-range screened Coulomb kernel of HSE06, the
hybrid the paper picks in its Introduction).  For transfer q = k - k' (fractional, never folded back into the
zone) and frequency class c, K = sum_i (g_i + q_i) b_i where g_i is the
integer representative of c_i in (-N_i/2, N_i/2); for even N_i the Nyquist
class c_i = N_i/2 has two representatives +-N_i/2 and v is averaged over all
of them (2^d aliases when d axes sit at Nyquist).

The DFTs are direct: one N_i x N_i matrix per axis, every angle formed as
2 pi ((c_i j_i) mod N_i) / N_i in FP64.  Nothing is blocked, fused or
reordered beyond that.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


# ----------------------------------------------------------------------------
# cell geometry
# ----------------------------------------------------------------------------
def reciprocal_rows(lattice):
    """b_i with a_i . b_j = 2 pi delta_ij."""
    return TWO_PI * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T


def cell_volume(lattice):
    return abs(float(np.linalg.det(np.asarray(lattice, dtype=np.float64))))


# ----------------------------------------------------------------------------
# kernel (HSE06 screened exchange, paper Introduction; Eq. (2) interaction)
# ----------------------------------------------------------------------------
def screened_kernel(k2, mu):
    """v(K) = 4 pi/|K|^2 (1 - exp(-|K|^2/(4 mu^2))), v(0) = pi/mu^2.
    ``k2`` is |K|^2 (array), evaluated in FP64 with expm1."""
    k2 = np.asarray(k2, dtype=np.float64)
    out = np.empty_like(k2)
    zero = k2 == 0.0
    nz = ~zero
    out[nz] = -4.0 * np.pi / k2[nz] * np.expm1(-k2[nz] / (4.0 * mu * mu))
    out[zero] = np.pi / (mu * mu)
    return out


def class_representatives(c, n):
    """Integer representatives of frequency class c on an axis of n points:
    c for c < n/2, c - n for c > n/2, and both +-n/2 for the Nyquist class."""
    if 2 * c == n:
        return (c, c - n)
    if 2 * c < n:
        return (c,)
    return (c - n,)


def kernel_table(lattice, grid, q, mu):
    """v_q on every class c of the grid, shape (N1, N2, N3), Nyquist classes
    averaged over their aliases.  q: fractional transfer k - k'."""
    b = reciprocal_rows(lattice)
    q = np.asarray(q, dtype=np.float64)
    n1, n2, n3 = grid
    # representative lists per axis, as (values, weights) over aliases
    axes = []
    for n, qi in zip(grid, q):
        reps = []
        for c in range(n):
            reps.append([g + qi for g in class_representatives(c, n)])
        axes.append(reps)
    out = np.zeros((n1, n2, n3))
    # enumerate classes and their aliases; the number of aliases is 1, 2, 4 or 8
    for c1 in range(n1):
        for c2 in range(n2):
            g12 = [(x1, x2) for x1 in axes[0][c1] for x2 in axes[1][c2]]
            for c3 in range(n3):
                combos = [(x1, x2, x3) for (x1, x2) in g12 for x3 in axes[2][c3]]
                kc = np.array(combos) @ b
                k2 = np.einsum("ij,ij->i", kc, kc)
                out[c1, c2, c3] = np.mean(screened_kernel(k2, mu))
    return out


def kernel_table_fast(lattice, grid, q, mu):
    """Same table as ``kernel_table``, vectorised over classes (the alias
    average is written as a mean over the 2^3 sign choices of the Nyquist
    components, which are identical unless that axis is at Nyquist)."""
    b = reciprocal_rows(lattice)
    q = np.asarray(q, dtype=np.float64)
    per_axis = []
    for n, qi in zip(grid, q):
        c = np.arange(n)
        lo = np.where(2 * c <= n, c, c - n).astype(np.float64)  # c - n for c > n/2; Nyquist keeps +n/2
        hi = np.where(2 * c == n, c - n, lo).astype(np.float64)  # Nyquist alias -n/2
        per_axis.append((lo + qi, hi + qi))
    acc = np.zeros(tuple(grid))
    for s1 in range(2):
        for s2 in range(2):
            for s3 in range(2):
                x1 = per_axis[0][s1][:, None, None]
                x2 = per_axis[1][s2][None, :, None]
                x3 = per_axis[2][s3][None, None, :]
                kx = x1 * b[0, 0] + x2 * b[1, 0] + x3 * b[2, 0]
                ky = x1 * b[0, 1] + x2 * b[1, 1] + x3 * b[2, 1]
                kz = x1 * b[0, 2] + x2 * b[1, 2] + x3 * b[2, 2]
                acc += screened_kernel(kx * kx + ky * ky + kz * kz, mu)
    return acc / 8.0


# ----------------------------------------------------------------------------
# direct DFT (separable, one matrix per axis)
# ----------------------------------------------------------------------------
def dft_matrix(n, sign):
    """D[c, j] = exp(sign * 2 pi i ((c j) mod n) / n)."""
    c = np.arange(n)
    ang = TWO_PI * ((np.outer(c, c) % n).astype(np.float64)) / n
    return np.cos(ang) + 1j * sign * np.sin(ang)


class DFT3:
    """Unnormalised forward (sign -1) and 1/N-normalised inverse DFT on a grid."""

    def __init__(self, grid):
        self.grid = tuple(int(x) for x in grid)
        self.f = [dft_matrix(n, -1) for n in self.grid]
        self.b = [dft_matrix(n, +1) for n in self.grid]
        self.n = int(np.prod(self.grid))

    def _apply(self, mats, x):
        n1, n2, n3 = self.grid
        x = np.asarray(x, dtype=np.complex128).reshape(n1, n2, n3)
        x = x @ mats[2].T                                   # axis 3
        x = np.matmul(mats[1], x)                           # axis 2 (per j1 slab)
        x = (mats[0] @ x.reshape(n1, n2 * n3)).reshape(n1, n2, n3)  # axis 1
        return x

    def forward(self, x):
        return self._apply(self.f, x)

    def inverse(self, x):
        return self._apply(self.b, x) / self.n


# ----------------------------------------------------------------------------
# the operator
# ----------------------------------------------------------------------------
def _pairs(nk, kpairs):
    if kpairs is None:
        return [(ik, jk) for ik in range(nk) for jk in range(nk)]
    return [tuple(int(x) for x in p) for p in kpairs]


class Oracle:
    """Exchange problem on one instance.

    psi: complex [nk, nb, N]; occ: [nk, nb]; kweight: [nk].  ``kernel`` may
    replace v_q by a constant (test-only special case)."""

    def __init__(self, lattice, grid, kfrac, kweight, mu, kpairs=None, kernel=None):
        self.lattice = np.asarray(lattice, dtype=np.float64)
        self.grid = tuple(int(x) for x in grid)
        self.kfrac = np.asarray(kfrac, dtype=np.float64).reshape(-1, 3)
        self.nk = self.kfrac.shape[0]
        self.kweight = (np.full(self.nk, 1.0 / self.nk) if kweight is None
                        else np.asarray(kweight, dtype=np.float64))
        self.mu = float(mu)
        self.omega = cell_volume(self.lattice)
        self.n = int(np.prod(self.grid))
        self.dv = self.omega / self.n
        self.kpairs = _pairs(self.nk, kpairs)
        self.dft = DFT3(self.grid)
        self.kernel = kernel
        self._vcache = {}

    @classmethod
    def from_instance(cls, inst, kernel=None, kpairs=None):
        return cls(inst.lattice, inst.grid, inst.kfrac, inst.kweight, inst.mu, kpairs=kpairs, kernel=kernel)

    # v_q for the pair (k, k'), q = k - k' unfolded
    def v(self, ik, jk):
        if self.kernel is not None:
            return np.full(self.grid, float(self.kernel))
        key = (ik, jk)
        if key not in self._vcache:
            q = self.kfrac[ik] - self.kfrac[jk]
            self._vcache[key] = kernel_table_fast(self.lattice, self.grid, q, self.mu)
        return self._vcache[key]

    def pair(self, u_n, u_m, v):
        """One band pair: returns (e, W) with rho = conj(u_m) u_n."""
        rho = np.conj(u_m) * u_n
        p = self.dft.forward(rho)
        e = float(np.sum(v * (p.real ** 2 + p.imag ** 2)))
        w = self.dft.inverse(v * p)
        return e, w.reshape(-1)

    def pair_energy(self, u_n, u_m, v):
        rho = np.conj(u_m) * u_n
        p = self.dft.forward(rho)
        return float(np.sum(v * (p.real ** 2 + p.imag ** 2)))

    def apply(self, psi, occ, outputs=None):
        """V_x u for every (k, n) (or the listed outputs) and E_x.

        Returns (vx, ex, e) where vx is complex [nk, nb, N] (zero where not
        requested), ex the exchange energy (only when all outputs are
        requested) and e the per-pair energies e[(ik, n, jk, m)]."""
        psi = np.asarray(psi)
        occ = np.asarray(occ, dtype=np.float64)
        nk, nb, n = psi.shape
        want = None if outputs is None else set((int(a), int(b)) for a, b in outputs)
        vx = np.zeros((nk, nb, n), dtype=np.complex128)
        esum = 0.0
        for (ik, jk) in self.kpairs:
            v = self.v(ik, jk)
            for ib in range(nb):
                if want is not None and (ik, ib) not in want:
                    continue
                u_n = psi[ik, ib].astype(np.complex128)
                for jb in range(nb):
                    u_m = psi[jk, jb].astype(np.complex128)
                    e, w = self.pair(u_n, u_m, v)
                    coef = self.kweight[jk] * occ[jk, jb]
                    vx[ik, ib] += -coef * u_m * w
                    esum += self.kweight[ik] * occ[ik, ib] * coef * e
        ex = -0.5 * (self.omega / (self.n * self.n)) * esum if want is None else None
        return vx, ex

    def energy(self, psi, occ):
        """E_x by the Fourier-sum route (no inverse transform)."""
        psi = np.asarray(psi)
        occ = np.asarray(occ, dtype=np.float64)
        nk, nb, n = psi.shape
        esum = 0.0
        for (ik, jk) in self.kpairs:
            v = self.v(ik, jk)
            for ib in range(nb):
                u_n = psi[ik, ib].astype(np.complex128)
                for jb in range(nb):
                    u_m = psi[jk, jb].astype(np.complex128)
                    e = self.pair_energy(u_n, u_m, v)
                    esum += self.kweight[ik] * occ[ik, ib] * self.kweight[jk] * occ[jk, jb] * e
        return -0.5 * (self.omega / (self.n * self.n)) * esum

    def pair_energies(self, psi, pairs):
        """e for listed ordered pairs (ik, n, jk, m)."""
        out = []
        for (ik, ib, jk, jb) in pairs:
            v = self.v(ik, jk)
            out.append(self.pair_energy(psi[ik, ib].astype(np.complex128), psi[jk, jb].astype(np.complex128), v))
        return np.array(out)

    def energy_from_apply(self, psi, occ, vx):
        """1/2 sum_k,n w_k f_kn <u_kn | V_x u_kn>, <a|b> = dV sum conj(a) b."""
        psi = np.asarray(psi).astype(np.complex128)
        tot = 0.0
        for ik in range(psi.shape[0]):
            for ib in range(psi.shape[1]):
                tot += self.kweight[ik] * occ[ik, ib] * self.dv * np.vdot(psi[ik, ib], vx[ik, ib]).real
        return 0.5 * tot

    def overlap(self, psi, vx):
        """M[k][i][j] = dV sum conj(u_ki) (V_x u)_kj."""
        psi = np.asarray(psi).astype(np.complex128)
        return self.dv * np.einsum("kin,kjn->kij", np.conj(psi), vx)

    def pairs_symmetric(self):
        """True when every listed (k, k') has its swap (k', k) listed."""
        s = set(self.kpairs)
        return all((b, a) in s for (a, b) in s)

    def gradient(self, psi, occ, vx=None, torch_convention=True):
        """dE_x/d conj(u) = dV w f V_x u; torch's convention doubles it.

        The formula differentiates Eq. (2)'s double sum only when the k-pair
        list is closed under swapping (k, k') -> (k', k): each pair then
        appears once with (k, n) as output and once with it as partner, and
        both give the same term.  Other lists raise ValueError."""
        if not self.pairs_symmetric():
            raise ValueError("dE_x/du* = dV w f V_x u needs a k-pair list closed under swapping")
        if vx is None:
            vx, _ = self.apply(psi, occ)
        g = self.dv * self.kweight[:, None, None] * np.asarray(occ)[:, :, None] * vx
        return 2.0 * g if torch_convention else g
