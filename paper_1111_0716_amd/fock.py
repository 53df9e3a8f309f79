"""Python binding of libfock.so: argument marshalling only.

Every step of the exchange path runs in the library's HIP kernels; this
module turns torch tensors into device pointers, keeps the workspace alive
and exposes the C ABI under the same names (fock_plan, fock_apply,
fock_energy, fock_energy_backward).  PyTorch supplies device memory and the
stream.  If the library is not built the calls raise: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FOCK_LIBRARY selects another build of the library (the host-code sanitizer
# variant of build.build_host_sanitized); default: the in-tree libfock.so
LIB_PATH = os.environ.get("FOCK_LIBRARY") or os.path.join(HERE, "libfock.so")

FOCK_OK, FOCK_ERR_ARG, FOCK_ERR_UNSUPPORTED, FOCK_ERR_NOMEM, FOCK_ERR_DEVICE, FOCK_ERR_STATE = range(6)
FOCK_C128, FOCK_C64, FOCK_MIXED, FOCK_MIXED_INV = 0, 1, 2, 3
PRECISIONS = {"c128": FOCK_C128, "c64": FOCK_C64, "mixed": FOCK_MIXED, "mixed_inv": FOCK_MIXED_INV}
STATIC_WORKSPACE_BYTES = 64 << 20  # FOCK_STATIC_WORKSPACE_BYTES of fock.h

EXPORTED = ["fock_plan", "fock_plan_tuned", "fock_workspace_size", "fock_set_workspace", "fock_set_stream", "fock_apply",
            "fock_apply_energy", "fock_apply_energy_static", "fock_energy", "fock_energy_backward", "fock_pw_to_grid", "fock_grid_to_pw", "fock_apply_pw", "fock_dft3",
            "fock_plan_stats", "fock_profile_enable", "fock_profile_read", "fock_set_graph", "fock_destroy",
            "fock_status_string", "fock_last_error"]
KERNEL_KINDS = ["plane", "pencil", "accumulate", "energy_plane", "energy_pencil", "energy_reduce", "overlap",
                "other", "fused", "energy_fused", "dft", "pw"]


class FockError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class FockTuning(ctypes.Structure):
    _fields_ = [("acc_workgroups", c_int32), ("tbuf_mb", c_int32), ("fused_split", c_int32), ("no_fused", c_int32),
                ("no_pair_symmetry", c_int32), ("fused_rounds", c_int32)]


class FockDesc(ctypes.Structure):
    _fields_ = [
        ("lattice", c_double * 9),
        ("grid", c_int32 * 3),
        ("nk", c_int32),
        ("kfrac", POINTER(c_double)),
        ("kweight", POINTER(c_double)),
        ("npairs", c_int32),
        ("kpairs", POINTER(c_int32)),
        ("nbands", c_int32),
        ("band_stride", c_int64),
        ("mu", c_double),
    ]


_lib = None


def lib():
    """Load libfock.so (raises if it has not been built).

    torch is imported first: libfock.so needs libamdhip64.so.7, and torch
    ships its own HIP runtime under that soname.  Loaded after torch, the
    library binds to torch's runtime, the one that owns the device memory
    and streams it is handed; loaded before, the dynamic loader would bring
    in the system runtime and torch a second copy, and the library's HIP
    calls would go to a runtime torch never initialised."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see above: one HIP runtime per process)

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.fock_plan.argtypes = [POINTER(FockDesc), c_int32, c_int, c_void_p, POINTER(c_void_p)]
        L.fock_plan_tuned.argtypes = [POINTER(FockDesc), c_int32, c_int, c_void_p, POINTER(FockTuning),
                                      POINTER(c_void_p)]
        L.fock_workspace_size.argtypes = [c_void_p, POINTER(c_size_t)]
        L.fock_set_workspace.argtypes = [c_void_p, c_void_p, c_size_t]
        L.fock_set_stream.argtypes = [c_void_p, c_void_p]
        L.fock_apply.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p)]
        L.fock_energy.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), c_void_p]
        L.fock_apply_energy.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                        POINTER(c_void_p), c_void_p]
        L.fock_apply_energy_static.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                               POINTER(c_void_p), c_void_p]
        L.fock_energy_backward.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), c_void_p, c_double,
                                           POINTER(c_void_p)]
        L.fock_pw_to_grid.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                       POINTER(c_int32), POINTER(c_void_p)]
        L.fock_grid_to_pw.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                       POINTER(c_int32), POINTER(c_void_p)]
        L.fock_apply_pw.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p), POINTER(c_int32),
                                     POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p)]
        L.fock_dft3.argtypes = [c_void_p, c_int32, c_int32, c_int64, c_void_p, c_int64]
        L.fock_plan_stats.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64),
                                      POINTER(c_int64)]
        L.fock_profile_enable.argtypes = [c_void_p, c_int]
        L.fock_profile_read.argtypes = [c_void_p, c_int, POINTER(c_double), POINTER(c_int64)]
        L.fock_set_graph.argtypes = [c_void_p, c_int]
        L.fock_destroy.argtypes = [c_void_p]
        L.fock_status_string.argtypes = [c_int]
        L.fock_status_string.restype = c_char_p
        L.fock_last_error.argtypes = []
        L.fock_last_error.restype = c_char_p
        for name in EXPORTED:
            if name not in ("fock_status_string", "fock_last_error"):
                getattr(L, name).restype = c_int
        _lib = L
    return _lib


def check(status):
    if status != FOCK_OK:
        L = lib()
        detail = L.fock_last_error().decode()
        raise FockError(status, f"{L.fock_status_string(status).decode()}: {detail}")


def _ptrs(values):
    arr = (c_void_p * len(values))()
    for i, v in enumerate(values):
        arr[i] = v
    return arr


def make_desc(lattice, grid, kfrac, kweight=None, nbands=1, band_stride=None, mu=0.106, kpairs=None, keep=None):
    """Fill a FockDesc; host arrays are appended to ``keep`` so they outlive fock_plan."""
    keep = keep if keep is not None else []
    d = FockDesc()
    lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
    for i in range(9):
        d.lattice[i] = float(lat[i])
    for i in range(3):
        d.grid[i] = int(grid[i])
    kf = np.ascontiguousarray(np.asarray(kfrac, dtype=np.float64).reshape(-1, 3))
    keep.append(kf)
    d.nk = kf.shape[0]
    d.kfrac = kf.ctypes.data_as(POINTER(c_double))
    if kweight is not None:
        kw = np.ascontiguousarray(np.asarray(kweight, dtype=np.float64).reshape(-1))
        if kw.shape[0] != kf.shape[0]:
            raise ValueError(f"kweight has {kw.shape[0]} entries for {kf.shape[0]} k-points")
        keep.append(kw)
        d.kweight = kw.ctypes.data_as(POINTER(c_double))
    if kpairs is not None:
        kp = np.ascontiguousarray(np.asarray(kpairs, dtype=np.int32).reshape(-1, 2))
        keep.append(kp)
        d.npairs = kp.shape[0]
        d.kpairs = kp.ctypes.data_as(POINTER(c_int32))
    d.nbands = int(nbands)
    n = int(grid[0]) * int(grid[1]) * int(grid[2])
    d.band_stride = int(band_stride if band_stride is not None else n)
    d.mu = float(mu)
    return d


class Plan:
    """A plan over one or more instances, its workspace and its stream.

    ``instances``: objects with lattice, grid, kfrac, kweight, nbands, mu
    (e.g. paper_1111_0716_amd.inputs.Instance) or dicts with those keys.
    ``band_stride``: per instance, elements between bands (default N): grid
    tensors are then [nk, nbands, band_stride] with the grid in the first N.
    ``attach_workspace``: False leaves the plan without a workspace (only
    fock_apply_energy_static, which brings its own, can then run).
    ``precision``: "c64" (FP32 path), "c128" (FP64 path) or "mixed" (complex128
    orbitals and outputs, FP32 co-densities and forward transforms, FP64 kernel
    multiply, inverse transforms and accumulate; grids N1 x L x L, N1 and L in
    24, 32, 36, 40, 48, 50, 54, 60, 64, 72)."""

    def __init__(self, instances, precision="c64", device=None, stream=None, kpairs=None, tuning=None,
                 band_stride=None, attach_workspace=True):
        import torch

        self.torch = torch
        if not isinstance(instances, (list, tuple)):
            instances = [instances]
        self.precision = precision
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self.prec = PRECISIONS[precision]
        self.cdtype = torch.complex64 if precision == "c64" else torch.complex128
        self.device = torch.device(device or "cuda:0")
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream
        keep = []
        descs = (FockDesc * len(instances))()
        self.meta = []
        for i, inst in enumerate(instances):
            g = _get(inst, "grid")
            nb = _get(inst, "nbands")
            kp = kpairs[i] if kpairs is not None else _get(inst, "kpairs", None)
            bstride = band_stride[i] if band_stride is not None else None
            descs[i] = make_desc(_get(inst, "lattice"), g, _get(inst, "kfrac"), _get(inst, "kweight", None), nb,
                                 bstride, _get(inst, "mu", 0.106), kp, keep)
            lat = np.asarray(_get(inst, "lattice"), dtype=np.float64).reshape(3, 3)
            n = int(np.prod(g))
            self.meta.append(dict(nk=descs[i].nk, nbands=nb, npts=n, omega=abs(float(np.linalg.det(lat))),
                                  band_stride=int(descs[i].band_stride)))
        handle = c_void_p()
        self.tuning = dict(tuning) if tuning else {}
        tn = FockTuning(**{k: int(v) for k, v in self.tuning.items()}) if tuning else None
        check(lib().fock_plan_tuned(descs, len(instances), self.prec, c_void_p(self._stream_ptr()),
                                    ctypes.byref(tn) if tn is not None else None, ctypes.byref(handle)))
        self.handle = handle
        size = c_size_t()
        check(lib().fock_workspace_size(self.handle, ctypes.byref(size)))
        self.workspace_bytes = size.value
        self.workspace = None
        if attach_workspace:
            self.set_workspace(torch.empty(max(size.value, 256), dtype=torch.uint8, device=self.device))

    def set_workspace(self, buf):
        """Attach a device buffer of at least ``workspace_bytes`` bytes (uint8,
        256-byte aligned) as the plan's workspace; the plan keeps a reference.
        Graphs recorded with the previous workspace are dropped."""
        t = self.torch
        if not (buf.is_cuda and buf.dtype == t.uint8 and buf.is_contiguous() and buf.device == self.device):
            raise ValueError(f"workspace must be a contiguous uint8 tensor on {self.device}")
        if buf.numel() < self.workspace_bytes or buf.data_ptr() % 256:
            raise ValueError(f"workspace needs {self.workspace_bytes} bytes at a 256-byte aligned address")
        check(lib().fock_set_workspace(self.handle, c_void_p(buf.data_ptr()), self.workspace_bytes))
        self.workspace = buf

    def _stream_ptr(self):
        if self.stream is not None:
            return int(self.stream.cuda_stream)
        return int(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_stream(self):
        check(lib().fock_set_stream(self.handle, c_void_p(self._stream_ptr())))

    def _check_count(self, name, seq):
        """One entry per instance of the plan (the library reads that many pointers)."""
        if len(seq) != len(self.meta):
            raise ValueError(f"{name} has {len(seq)} entries; the plan has {len(self.meta)} instances")

    def _check_ex(self, ex, name="ex"):
        t = self.torch
        if not (ex.is_cuda and ex.dtype == t.float64 and ex.is_contiguous() and ex.device == self.device and
                ex.numel() == len(self.meta)):
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device} with "
                             f"{len(self.meta)} entries (one per instance)")

    def _check_psi(self, psi, i, name="psi"):
        m = self.meta[i]
        if not (psi.is_cuda and psi.dtype == self.cdtype and psi.is_contiguous() and psi.device == self.device):
            raise ValueError(f"{name}[{i}] must be a contiguous {self.cdtype} tensor on {self.device}")
        if psi.dim() < 3 or tuple(psi.shape[:2]) != (m["nk"], m["nbands"]) or psi[0, 0].numel() != m["band_stride"]:
            raise ValueError(f"{name}[{i}] has shape {tuple(psi.shape)}, expected "
                             f"({m['nk']}, {m['nbands']}, {m['band_stride']})")

    def _check_occ(self, occ, i):
        m = self.meta[i]
        if not (occ.is_cuda and occ.dtype == self.torch.float64 and occ.is_contiguous() and
                occ.device == self.device and tuple(occ.shape) == (m["nk"], m["nbands"])):
            raise ValueError(f"occ[{i}] must be a contiguous float64 tensor on {self.device} of shape "
                             f"({m['nk']}, {m['nbands']})")

    def _inputs(self, psi, occ):
        """Validated per-instance lists of orbitals and occupations."""
        psi, occ = _aslist(psi), _aslist(occ)
        self._check_count("psi", psi)
        self._check_count("occ", occ)
        for i, (p, o) in enumerate(zip(psi, occ)):
            self._check_psi(p, i)
            self._check_occ(o, i)
        return psi, occ

    def _outputs(self, out, like, name="out"):
        """Per-instance output grids: new tensors, or the caller's, validated
        (distinct from the inputs, which the library rejects as aliases)."""
        if out is None:
            return [self.torch.empty_like(p) for p in like]
        out = _aslist(out)
        self._check_count(name, out)
        for i, o in enumerate(out):
            self._check_psi(o, i, name)
        return out

    def fock_apply(self, psi, occ, out=None, vmat=False):
        """V_x psi for every instance; returns (outputs, overlaps or None)."""
        psi, occ = self._inputs(psi, occ)
        out = self._outputs(out, psi)
        mats = None
        if vmat:
            mats = [self.torch.empty((m["nk"], m["nbands"], m["nbands"]), dtype=self.cdtype, device=self.device)
                    for m in self.meta]
        self._sync_stream()
        check(lib().fock_apply(self.handle, _ptrs([p.data_ptr() for p in psi]), _ptrs([o.data_ptr() for o in occ]),
                               _ptrs([x.data_ptr() for x in out]),
                               _ptrs([x.data_ptr() for x in mats]) if mats else None))
        return out, mats

    def fock_apply_energy(self, psi, occ, out=None, vmat=False, ex=None):
        """fock_apply and fock_energy in one call; returns (outputs, overlaps
        or None, E_x as a float64 tensor [n_inst])."""
        psi, occ = self._inputs(psi, occ)
        out = self._outputs(out, psi)
        mats = None
        if vmat:
            mats = [self.torch.empty((m["nk"], m["nbands"], m["nbands"]), dtype=self.cdtype, device=self.device)
                    for m in self.meta]
        if ex is None:
            ex = self.torch.empty(len(psi), dtype=self.torch.float64, device=self.device)
        self._check_ex(ex)
        self._sync_stream()
        check(lib().fock_apply_energy(self.handle, _ptrs([p.data_ptr() for p in psi]),
                                      _ptrs([o.data_ptr() for o in occ]), _ptrs([x.data_ptr() for x in out]),
                                      _ptrs([x.data_ptr() for x in mats]) if mats else None, c_void_p(ex.data_ptr())))
        return out, mats, ex

    def fock_apply_energy_static(self, psi, occ, out=None, vmat=None, ex=None):
        """fock_apply_energy on the library's static device workspace (the
        library allocates nothing; outputs are the caller's tensors, or new
        ones made here when not given).  ``vmat``: None, or a list of overlap
        tensors [nk, nbands, nbands].  Returns (outputs, vmat, E_x)."""
        psi, occ = self._inputs(psi, occ)
        out = self._outputs(out, psi)
        if vmat is not None:
            vmat = _aslist(vmat)
            self._check_count("vmat", vmat)
            for i, (x, m) in enumerate(zip(vmat, self.meta)):
                if not (x.is_cuda and x.dtype == self.cdtype and x.is_contiguous() and x.device == self.device and
                        tuple(x.shape) == (m["nk"], m["nbands"], m["nbands"])):
                    raise ValueError(f"vmat[{i}] must be a contiguous {self.cdtype} tensor "
                                     f"({m['nk']}, {m['nbands']}, {m['nbands']}) on {self.device}")
        if ex is None:
            ex = self.torch.empty(len(psi), dtype=self.torch.float64, device=self.device)
        self._check_ex(ex)
        self._sync_stream()
        with self.torch.cuda.device(self.device):
            check(lib().fock_apply_energy_static(self.handle, _ptrs([p.data_ptr() for p in psi]),
                                                 _ptrs([o.data_ptr() for o in occ]), _ptrs([x.data_ptr() for x in out]),
                                                 _ptrs([x.data_ptr() for x in vmat]) if vmat else None,
                                                 c_void_p(ex.data_ptr())))
        return out, vmat, ex

    def fock_energy(self, psi, occ, ex=None):
        """E_x of every instance as a float64 tensor [n_inst]."""
        psi, occ = self._inputs(psi, occ)
        if ex is None:
            ex = self.torch.empty(len(psi), dtype=self.torch.float64, device=self.device)
        self._check_ex(ex)
        self._sync_stream()
        check(lib().fock_energy(self.handle, _ptrs([p.data_ptr() for p in psi]), _ptrs([o.data_ptr() for o in occ]),
                                c_void_p(ex.data_ptr())))
        return ex

    def fock_energy_backward(self, psi, occ, grad_ex, scale, out=None):
        """grad_ex[i] * scale * w_k f_kn V_x u for every instance (grad_ex: one
        entry per instance)."""
        psi, occ = self._inputs(psi, occ)
        g = grad_ex.to(device=self.device, dtype=self.torch.float64).contiguous().reshape(-1)
        self._check_ex(g, "grad_ex")
        out = self._outputs(out, psi)
        self._sync_stream()
        check(lib().fock_energy_backward(self.handle, _ptrs([p.data_ptr() for p in psi]),
                                         _ptrs([o.data_ptr() for o in occ]), c_void_p(g.data_ptr()),
                                         float(scale), _ptrs([x.data_ptr() for x in out])))
        return out

    # ---- plane-wave boundary and batched 3-D DFT -------------------------
    def _sphere(self, gidx, npw):
        """Validate the per-instance sphere tensors; returns (gidx, npw, npw_max array)."""
        gidx, npw = _aslist(gidx), _aslist(npw)
        self._check_count("gidx", gidx)
        self._check_count("npw", npw)
        t = self.torch
        for i, (g, n) in enumerate(zip(gidx, npw)):
            m = self.meta[i]
            if not (g.is_cuda and g.dtype == t.int32 and g.is_contiguous() and g.dim() == 2 and g.shape[0] == m["nk"]
                    and g.shape[1] >= 1 and g.device == self.device):
                raise ValueError(f"gidx[{i}] must be a contiguous int32 CUDA tensor [nk, npw_max]")
            if not (n.is_cuda and n.dtype == t.int32 and n.is_contiguous() and tuple(n.shape) == (m["nk"],) and
                    n.device == self.device):
                raise ValueError(f"npw[{i}] must be a contiguous int32 CUDA tensor [nk]")
        npw_max = (c_int32 * len(gidx))(*[int(g.shape[1]) for g in gidx])
        return gidx, npw, npw_max

    def _check_coef(self, c, i, npw_max):
        m = self.meta[i]
        if not (c.is_cuda and c.dtype == self.cdtype and c.is_contiguous() and c.device == self.device and
                tuple(c.shape) == (m["nk"], m["nbands"], npw_max)):
            raise ValueError(f"coefficients[{i}] must be a contiguous {self.cdtype} CUDA tensor "
                             f"({m['nk']}, {m['nbands']}, {npw_max})")

    def pw_to_grid(self, coef, gidx, npw, out=None):
        """Orbitals on the grid from sphere coefficients (see fock_pw_to_grid)."""
        coef = _aslist(coef)
        self._check_count("coef", coef)
        gidx, npw, npw_max = self._sphere(gidx, npw)
        for i, c in enumerate(coef):
            self._check_coef(c, i, npw_max[i])
        if out is None:
            out = [self.torch.zeros((m["nk"], m["nbands"], m["band_stride"]), dtype=self.cdtype, device=self.device)
                   for m in self.meta]
        out = _aslist(out)
        self._check_count("out", out)
        for i, o in enumerate(out):
            self._check_psi(o, i, "out")
        self._sync_stream()
        check(lib().fock_pw_to_grid(self.handle, _ptrs([c.data_ptr() for c in coef]), _ptrs([g.data_ptr() for g in gidx]),
                                    _ptrs([n.data_ptr() for n in npw]), npw_max, _ptrs([o.data_ptr() for o in out])))
        return out

    def grid_to_pw(self, f, gidx, npw, out=None):
        """Sphere coefficients of grid functions f (f is transformed in place)."""
        f = _aslist(f)
        self._check_count("f", f)
        gidx, npw, npw_max = self._sphere(gidx, npw)
        for i, x in enumerate(f):
            self._check_psi(x, i, "f")
        out = [self.torch.empty((m["nk"], m["nbands"], npw_max[i]), dtype=self.cdtype, device=self.device)
               for i, m in enumerate(self.meta)] if out is None else _aslist(out)
        self._check_count("out", out)
        for i, c in enumerate(out):
            self._check_coef(c, i, npw_max[i])
        self._sync_stream()
        check(lib().fock_grid_to_pw(self.handle, _ptrs([x.data_ptr() for x in f]), _ptrs([g.data_ptr() for g in gidx]),
                                    _ptrs([n.data_ptr() for n in npw]), npw_max, _ptrs([c.data_ptr() for c in out])))
        return out

    def fock_apply_pw(self, coef, gidx, npw, occ, psi_work=None, vx_work=None, out=None):
        """V_x psi on the sphere; returns (coefficients, psi_work, vx_work)."""
        coef, occ = _aslist(coef), _aslist(occ)
        self._check_count("coef", coef)
        self._check_count("occ", occ)
        gidx, npw, npw_max = self._sphere(gidx, npw)
        t = self.torch
        for i, (c, o) in enumerate(zip(coef, occ)):
            self._check_coef(c, i, npw_max[i])
            self._check_occ(o, i)

        def grids():
            return [t.zeros((m["nk"], m["nbands"], m["band_stride"]), dtype=self.cdtype, device=self.device)
                    for m in self.meta]

        psi_work = grids() if psi_work is None else _aslist(psi_work)
        vx_work = grids() if vx_work is None else _aslist(vx_work)
        out = [t.empty_like(c) for c in coef] if out is None else _aslist(out)
        for name, seq in (("psi_work", psi_work), ("vx_work", vx_work), ("out", out)):
            self._check_count(name, seq)
        for i in range(len(coef)):
            self._check_psi(psi_work[i], i, "psi_work")
            self._check_psi(vx_work[i], i, "vx_work")
            self._check_coef(out[i], i, npw_max[i])
        self._sync_stream()
        check(lib().fock_apply_pw(self.handle, _ptrs([c.data_ptr() for c in coef]), _ptrs([g.data_ptr() for g in gidx]),
                                  _ptrs([n.data_ptr() for n in npw]), npw_max, _ptrs([o.data_ptr() for o in occ]),
                                  _ptrs([x.data_ptr() for x in psi_work]), _ptrs([x.data_ptr() for x in vx_work]),
                                  _ptrs([x.data_ptr() for x in out])))
        return out, psi_work, vx_work

    def dft3(self, data, sign, inst=0):
        """In-place unnormalised 3-D DFT of every grid in ``data`` (a contiguous
        complex tensor [..., N] of the plan precision on the instance's grid)."""
        if not 0 <= int(inst) < len(self.meta):
            raise ValueError(f"instance {inst} out of range (plan has {len(self.meta)})")
        m = self.meta[inst]
        if not (data.is_cuda and data.dtype == self.cdtype and data.is_contiguous() and data.device == self.device and
                data.numel() % m["npts"] == 0):
            raise ValueError(f"data must be a contiguous {self.cdtype} CUDA tensor of whole grids of {m['npts']} points")
        self._sync_stream()
        check(lib().fock_dft3(self.handle, int(inst), int(sign), data.numel() // m["npts"], c_void_p(data.data_ptr()),
                              m["npts"]))
        return data

    def stats(self):
        a, b, c, d = c_int64(), c_int64(), c_int64(), c_int64()
        check(lib().fock_plan_stats(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return dict(ordered_pairs=a.value, apply_fft_pairs=b.value, energy_fft_pairs=c.value, apply_launches=d.value)

    def set_graph(self, enable=True):
        """Record each call's launch sequence into one HIP graph and replay it
        (needs a non-default stream: pass ``stream=torch.cuda.Stream()``)."""
        self._sync_stream()
        check(lib().fock_set_graph(self.handle, 1 if enable else 0))

    def profile(self, enable=True):
        """Bracket every library launch with HIP events on the plan stream."""
        check(lib().fock_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self):
        """{kind: (total_ms, launches)} since the last read; waits for the events."""
        out = {}
        for k, name in enumerate(KERNEL_KINDS):
            ms, n = c_double(), c_int64()
            check(lib().fock_profile_read(self.handle, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().fock_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _get(obj, key, default=KeyError):
    if isinstance(obj, dict):
        if key in obj:
            return obj[key]
    elif hasattr(obj, key):
        return getattr(obj, key)
    if default is KeyError:
        raise KeyError(key)
    return default


def _aslist(x):
    return list(x) if isinstance(x, (list, tuple)) else [x]


def fock_energy_autograd():
    """torch.autograd.Function whose forward is E_x of every instance of a
    plan (library fock_energy, a float64 tensor [n_inst]) and whose backward
    is the library's hand-written gradient path (fock_energy_backward), with
    co-densities recomputed.

    Call as ``FockEnergy.apply(plan, occ, *psi)`` with one orbital tensor per
    instance and ``occ`` a list of occupation tensors.  Each psi[i] receives
    torch's complex gradient 2 dV_i grad_i w f V_x u (dV_i = Omega_i/N_i).
    Plans whose k-pair list is not closed under swapping raise (the library
    returns FOCK_ERR_UNSUPPORTED for their gradient)."""
    import torch

    class FockEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, occ, *psi):
            occ = _aslist(occ)
            ex = plan.fock_energy(list(psi), occ)
            ctx.save_for_backward(*psi)
            ctx.plan = plan
            ctx.occ = occ
            return ex

        @staticmethod
        def backward(ctx, grad):
            psi = list(ctx.saved_tensors)
            plan = ctx.plan
            # torch's complex gradient is 2 dE/d conj(psi), dE/d conj(psi) = dV w f V_x psi;
            # the per-instance factor 2 dV_i rides on grad_ex so that scale = 1
            dv2 = torch.tensor([2.0 * m["omega"] / m["npts"] for m in plan.meta], dtype=torch.float64,
                               device=plan.device)
            g = plan.fock_energy_backward(psi, ctx.occ, grad.reshape(-1).to(torch.float64) * dv2, 1.0)
            return (None, None, *g)

    return FockEnergy
