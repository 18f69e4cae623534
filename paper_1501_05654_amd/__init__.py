"""MI355X real-space Kohn-Sham H*psi library: thin Python binding.

Argument marshalling only.  Every numeric step runs in the HIP kernels of
``librsg.so`` (built from ``csrc/`` by ``build.py``); PyTorch supplies device
memory and the current stream.  Importing this package fails if the library
has not been built: there is no CPU fallback.

Orbital batches are orbital-major ``torch.complex128`` CUDA tensors of shape
[nst, ldp] with ``ldp >= np``: row n is orbital n over the compact points
(z-major, y, x); the first ``nst`` rows (default: all) are used and entries
np..ldp-1 of each row are never touched.  See ``include/rsg.h`` for the
definition of every entry point.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

__all__ = [
    "RSGError", "Grid", "Hamiltonian", "hpsi", "propagate_step", "propagate", "dot", "norm2",
    "energy", "dipole_expectation", "adjoint_step", "laser_field", "laser_grad",
    "control_forward", "control_backward", "OptimalControlJ", "copy", "kernel_timing",
    "C128", "MIXED", "LIB_PATH", "autotune", "set_tile", "get_tile", "tile_candidates", "Batch",
    "GridMap", "MAP_STANDARD", "MAP_BRICKS", "MAP_HILBERT", "shifted_solve", "bilinear", "cs_eigs",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librsg.so")

C128, MIXED = 0, 1
MAP_STANDARD, MAP_BRICKS, MAP_HILBERT = 0, 1, 2
_OP = {"hpsi": 0, "step": 1, "reduce": 2, "energy": 3, "adjoint": 4}


class RSGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rsg error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_1501_05654_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    i32, i64, dbl, vp, sz = C.c_int32, C.c_int64, C.c_double, C.c_void_p, C.c_size_t
    sig = {
        "rsg_grid_create": (C.c_int, [vp, vp, vp]),
        "rsg_grid_create_aligned": (C.c_int, [vp, i32, vp, vp]),
        "rsg_grid_create_box": (C.c_int, [i32, i32, i32, dbl, i32, vp, vp]),
        "rsg_grid_points": (C.c_int, [vp, vp, vp]),
        "rsg_grid_info": (C.c_int, [vp, vp, vp, vp]),
        "rsg_grid_coords": (C.c_int, [vp, vp]),
        "rsg_grid_positions": (C.c_int, [vp, vp]),
        "rsg_grid_destroy": (C.c_int, [vp]),
        "rsg_ham_create": (C.c_int, [vp, vp, dbl, i32, i32, vp, vp]),
        "rsg_ham_destroy": (C.c_int, [vp]),
        "rsg_ham_set_mask": (C.c_int, [vp, vp]),
        "rsg_workspace_bytes": (sz, [vp, i32, i64, i64, i32]),
        "rsg_hpsi": (C.c_int, [vp, vp, vp, i64, i64, i32, dbl, vp, sz, vp]),
        "rsg_propagate_step": (C.c_int, [vp, vp, i64, i64, i32, dbl, dbl, vp, sz, vp]),
        "rsg_propagate": (C.c_int, [vp, vp, i64, i64, i32, dbl, i64, vp, i32, vp, sz, vp]),
        "rsg_dot": (C.c_int, [vp, vp, vp, i64, i64, vp, vp, sz, vp]),
        "rsg_dot_noalloc": (C.c_int, [vp, vp, vp, i64, i64, vp, vp]),
        "rsg_dot_noalloc_max_bytes": (sz, []),
        "rsg_norm2": (C.c_int, [vp, vp, i64, i64, vp, vp, sz, vp]),
        "rsg_energy": (C.c_int, [vp, vp, i64, i64, i32, dbl, vp, vp, sz, vp]),
        "rsg_dipole_expectation": (C.c_int, [vp, vp, i64, i64, vp, vp, sz, vp]),
        "rsg_laser_field": (C.c_int, [vp, i32, dbl, dbl, i64, i64, vp, vp]),
        "rsg_laser_grad": (C.c_int, [vp, i64, dbl, dbl, i32, vp, vp]),
        "rsg_adjoint_step": (C.c_int, [vp, vp, vp, i64, i64, dbl, dbl, vp, vp, sz, vp]),
        "rsg_control_workspace_bytes": (sz, [vp, i64, i64, i64, i64]),
        "rsg_control_workspace_bytes_min": (sz, [vp, i64, i64, i64, i64]),
        "rsg_reduce_workspace_bytes": (sz, [vp, i64]),
        "rsg_control_forward": (C.c_int, [vp, vp, i64, i64, dbl, i64, vp, i32, i64, vp, vp, vp,
                                          sz, vp]),
        "rsg_control_backward": (C.c_int, [vp, vp, i64, i64, dbl, i64, vp, i32, i64, vp, vp, vp,
                                           vp, sz, vp]),
        "rsg_last_error": (C.c_char_p, []),
        "rsg_version": (C.c_char_p, []),
        "rsg_copy": (C.c_int, [vp, vp, sz, vp]),
        "rsg_timing_enable": (C.c_int, [i32]),
        "rsg_timing_query": (C.c_int, [vp, vp, vp]),
        "rsg_tile_candidates": (C.c_int, [i32, vp, i32, vp]),
        "rsg_set_tile": (C.c_int, [vp, i64, i32, vp]),
        "rsg_get_tile": (C.c_int, [vp, i64, i32, vp]),
        "rsg_autotune": (C.c_int, [vp, vp, i64, i64, i32, vp, sz, i32, vp, vp, vp]),
        "rsg_autotune_cache": (C.c_int, [vp, vp, i64, i64, i32, vp, sz, i32, C.c_char_p, vp, vp, vp, vp]),
        "rsg_batch_workspace_bytes": (sz, [i32, vp]),
        "rsg_batch_create": (C.c_int, [i32, vp, vp, sz, vp, vp]),
        "rsg_batch_destroy": (C.c_int, [vp]),
        "rsg_batch_set_tile": (C.c_int, [vp, vp, vp]),
        "rsg_batch_get_tile": (C.c_int, [vp, vp]),
        "rsg_batch_autotune": (C.c_int, [vp, i32, vp, vp, vp]),
        "rsg_batch_propagate": (C.c_int, [vp, dbl, i64, i32, vp]),
        "rsg_batch_plan_create": (C.c_int, [i32, vp, vp, sz, vp, vp]),
        "rsg_batch_run": (C.c_int, [vp, i64, dbl, vp]),
        "rsg_batch_classes": (C.c_int, [vp, vp, vp]),
        "rsg_batch_set_classes": (C.c_int, [vp, vp, vp]),
        "rsg_batch_set_class_tile": (C.c_int, [vp, i32, vp, vp]),
        "rsg_batch_get_class_tile": (C.c_int, [vp, i32, vp]),
        "rsg_batch_set_grid": (C.c_int, [vp, i32]),
        "rsg_batch_class_info": (C.c_int, [vp, i32, vp, vp, vp]),
        "rsg_ham_set_complex_scaling": (C.c_int, [vp, dbl, vp]),
        "rsg_bilinear": (C.c_int, [vp, vp, vp, i64, i64, vp, vp, sz, vp]),
        "rsg_cs_eigs_workspace_bytes": (sz, [vp, i64, i64]),
        "rsg_cs_eigs": (C.c_int, [vp, vp, vp, i64, i64, i32, dbl, i32, dbl, vp, vp, vp, sz, vp]),
        "rsg_solve_workspace_bytes": (sz, [vp, i32, i64, i64]),
        "rsg_shifted_solve": (C.c_int, [vp, vp, vp, vp, i64, i64, i32, dbl, i32, i32, vp, vp, vp, vp, sz,
                                        vp]),
        "rsg_map_create": (C.c_int, [vp, i32, i32, vp]),
        "rsg_map_destroy": (C.c_int, [vp]),
        "rsg_map_order": (C.c_int, [vp, vp]),
        "rsg_map_laplacian": (C.c_int, [vp, vp, vp, i64, i64, dbl, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = _load()


def _check(rc: int):
    if rc != 0:
        raise RSGError(rc, _lib.rsg_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _batch(t: torch.Tensor, name: str, np_: int, dtype=torch.complex128) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == dtype and t.dim() == 2 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor [nst, ldp]")
    if t.shape[1] < np_:
        raise ValueError(f"{name} rows hold {t.shape[1]} points, grid has {np_}")
    return t


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class _ProjDesc(C.Structure):
    _fields_ = [("n_support", C.c_int64), ("idx", C.c_void_p), ("p", C.c_void_p),
                ("E", C.c_double * 4)]


class _GridDesc(C.Structure):
    _fields_ = [("shape", C.c_int32), ("n", C.c_int32), ("radius", C.c_double), ("h", C.c_double)]


class Grid:
    """Uniform grid restricted to a sphere (radius R) or a cube (n per axis).

    align > 1 (a power of two) gives row-aligned storage: fields have
    ``np`` slots, of which ``npoints`` hold box points in the same order;
    the others are dead slots (coordinates -1) that inputs keep at zero.
    ``live()`` lists the slots of the box points."""

    def __init__(self, h: float, *, R: float | None = None, n: int | None = None, box=None,
                 align: int = 1):
        if sum(v is not None for v in (R, n, box)) != 1:
            raise ValueError("give exactly one of R (sphere), n (cube) or box=(nx, ny, nz)")
        self._h = C.c_void_p()
        if box is not None:
            nx, ny, nz = (int(v) for v in box)
            _check(_lib.rsg_grid_create_box(nx, ny, nz, float(h), int(align), _stream(), C.byref(self._h)))
        else:
            d = _GridDesc(1 if R is not None else 0, int(n or 0), float(R or 0.0), float(h))
            _check(_lib.rsg_grid_create_aligned(C.byref(d), int(align), _stream(), C.byref(self._h)))
        np_ = C.c_int64()
        dims = (C.c_int32 * 3)()
        hh = C.c_double()
        _check(_lib.rsg_grid_info(self._h, C.byref(np_), dims, C.byref(hh)))
        npts = C.c_int64()
        al = C.c_int32()
        _check(_lib.rsg_grid_points(self._h, C.byref(npts), C.byref(al)))
        self.np = int(np_.value)
        self.npoints = int(npts.value)
        self.align = int(al.value)
        self.dims = tuple(int(x) for x in dims)
        self.h = float(hh.value)
        self.R, self.n = R, n

    def live(self) -> np.ndarray:
        """Slot of every box point, ascending (all slots when align is 1)."""
        if self.npoints == self.np:
            return np.arange(self.np, dtype=np.int64)
        return np.nonzero(self.coords()[:, 0] >= 0)[0]

    def coords(self) -> np.ndarray:
        out = np.empty((self.np, 3), dtype=np.int32)
        _check(_lib.rsg_grid_coords(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def positions(self) -> np.ndarray:
        out = np.empty((self.np, 3), dtype=np.float64)
        _check(_lib.rsg_grid_positions(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rsg_grid_destroy(h)
            self._h = None


class Hamiltonian:
    """H = kin*Lap_h + V + field*x_axis + separable projectors.

    V: CUDA float64 [np] or None.  projectors: list of (idx int32 CUDA [n],
    p float64 CUDA [n, 4], E sequence of 4 floats).  The library copies
    every table."""

    def __init__(self, grid: Grid, V: torch.Tensor | None = None, kin: float = -0.5,
                 dipole_axis: int = -1, projectors=None):
        self.grid = grid
        self.axis = int(dipole_axis)
        projectors = list(projectors or [])
        descs = (_ProjDesc * max(1, len(projectors)))()
        keep = []
        for k, (idx, p, E) in enumerate(projectors):
            idx = idx.to(torch.int32).contiguous()
            p = p.to(torch.float64).contiguous()
            if not (idx.is_cuda and p.is_cuda and p.shape == (idx.shape[0], 4)):
                raise ValueError("projector tables must be CUDA tensors idx[n], p[n,4]")
            keep += [idx, p]
            descs[k] = _ProjDesc(idx.shape[0], idx.data_ptr(), p.data_ptr(),
                                 (C.c_double * 4)(*[float(e) for e in E]))
        if V is not None:
            V = V.to(torch.float64).contiguous()
            if not V.is_cuda or V.numel() != grid.np:
                raise ValueError("V must be a CUDA float64 tensor with np entries")
        self._h = C.c_void_p()
        torch.cuda.synchronize()  # tables written on any stream are complete
        _check(_lib.rsg_ham_create(grid._h, _ptr(V), float(kin), self.axis, len(projectors),
                                   descs, C.byref(self._h)))
        torch.cuda.synchronize()
        self.natoms = len(projectors)

    def set_mask(self, mask: torch.Tensor | None):
        """Absorber mask M(r) (CUDA float64 [np]) applied after every Taylor
        step, psi <- M psi; None removes it.  The library copies it."""
        if mask is not None:
            mask = mask.to(torch.float64).contiguous()
            if not mask.is_cuda or mask.numel() != self.grid.np:
                raise ValueError("mask must be a CUDA float64 tensor with np entries")
            torch.cuda.synchronize()
        _check(_lib.rsg_ham_set_mask(self._h, _ptr(mask)))

    def set_complex_scaling(self, theta: float, V_im: torch.Tensor | None = None):
        """Complex scaling r -> r e^{i theta}: kinetic prefactor kin
        e^{-2 i theta} and imaginary potential V_im (CUDA float64 [np], the
        imaginary part of the continued potential; the real part is the V
        given at creation).  theta = 0 and V_im = None undo it."""
        if V_im is not None:
            V_im = V_im.to(torch.float64).contiguous()
            if not V_im.is_cuda or V_im.numel() != self.grid.np:
                raise ValueError("V_im must be a CUDA float64 tensor with np entries")
            torch.cuda.synchronize()
        _check(_lib.rsg_ham_set_complex_scaling(self._h, float(theta), _ptr(V_im)))

    def workspace_bytes(self, op: str, nst: int, ldp: int, dtype: int = C128) -> int:
        return int(_lib.rsg_workspace_bytes(self._h, _OP[op], nst, ldp, dtype))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rsg_ham_destroy(h)
            self._h = None


def bilinear(grid: Grid | Hamiltonian, a: torch.Tensor, b: torch.Tensor,
             nst: int | None = None) -> torch.Tensor:
    """h^3 sum a_n b_n per orbital, no conjugation -> complex128 CUDA [nst]."""
    grid = _grid_of(grid)
    _batch(a, "a", grid.np)
    _batch(b, "b", grid.np)
    if a.shape != b.shape:
        raise ValueError("a and b must have the same shape")
    n = _nst(a, nst)
    out = torch.empty(2 * n, dtype=torch.float64, device=a.device)
    ws = _reduce_ws(grid, n, a.device)
    _check(_lib.rsg_bilinear(grid._h, _ptr(a), _ptr(b), n, a.shape[1], _ptr(out), _ptr(ws),
                             ws.numel(), _stream()))
    return torch.view_as_complex(out.view(n, 2))


def cs_eigs(ham: Hamiltonian, psi: torch.Tensor, targets, max_outer: int = 50, tol: float = 1e-12,
            qmr_maxiter: int = 5000, qmr_tol: float = 1e-12, nst: int | None = None):
    """Eigenvalues nearest targets[n] by shifted inverse iteration (QMR
    inner solves); psi (start vectors, orbital-major) is overwritten with
    the eigenvectors, normalised to h^3 psi^T psi = 1.  Returns (lambda
    complex numpy [nst], outer iterations)."""
    _batch(psi, "psi", ham.grid.np)
    n = _nst(psi, nst)
    z = np.asarray(targets, dtype=np.complex128).reshape(-1)
    if z.size == 1:
        z = np.full(n, z[0])
    if z.size < n:
        raise ValueError(f"need {n} targets")
    zt = np.ascontiguousarray(np.stack([z[:n].real, z[:n].imag], axis=1).reshape(-1))
    lam = np.zeros(2 * n)
    its = np.zeros(n, dtype=np.int32)
    ws = _ws(_lib.rsg_cs_eigs_workspace_bytes(ham._h, n, psi.shape[1]), psi.device)
    vp = C.c_void_p
    _check(_lib.rsg_cs_eigs(ham._h, zt.ctypes.data_as(vp), _ptr(psi), n, psi.shape[1], int(max_outer), float(tol),
                            int(qmr_maxiter), float(qmr_tol), lam.ctypes.data_as(vp), its.ctypes.data_as(vp),
                            _ptr(ws), ws.numel(), _stream()))
    return lam[0::2] + 1j * lam[1::2], its


def shifted_solve(ham: Hamiltonian, b: torch.Tensor, shift, x: torch.Tensor | None = None,
                  method: str = "qmr", tol: float = 1e-10, maxiter: int = 1000, check_every: int = 10,
                  nst: int | None = None, ws: torch.Tensor | None = None):
    """Solve (H + shift[n]) x_n = b_n for each orbital (orbital-major
    [nst, ldp] complex128).  method "qmr" (complex shifts) or "cg" (real
    shifts).  x (initial guess, default zeros) is updated in place and
    returned with per-orbital iterations, relative residuals and status
    (0 converged, 1 iteration limit, 2 breakdown)."""
    _batch(b, "b", ham.grid.np)
    x = torch.zeros_like(b) if x is None else _batch(x, "x", ham.grid.np)
    if x.shape != b.shape:
        raise ValueError("x must have the shape of b")
    n = _nst(b, nst)
    sh = np.asarray(shift, dtype=np.complex128).reshape(-1)
    if sh.size == 1:
        sh = np.full(n, sh[0])
    if sh.size < n:
        raise ValueError(f"need {n} shifts, got {sh.size}")
    host = np.ascontiguousarray(np.stack([sh[:n].real, sh[:n].imag], axis=1).reshape(-1))
    m = {"cg": 0, "qmr": 1}[method]
    need = int(_lib.rsg_solve_workspace_bytes(ham._h, m, n, b.shape[1]))
    if ws is None or ws.numel() < need:
        ws = _ws(need, b.device)
    iters = np.zeros(n, dtype=np.int32)
    res = np.zeros(n, dtype=np.float64)
    status = np.zeros(n, dtype=np.int32)
    vp = C.c_void_p
    _check(_lib.rsg_shifted_solve(ham._h, host.ctypes.data_as(vp), _ptr(b), _ptr(x), n, b.shape[1], m,
                                  float(tol), int(maxiter), int(check_every), iters.ctypes.data_as(vp),
                                  res.ctypes.data_as(vp), status.ctypes.data_as(vp), _ptr(ws), ws.numel(),
                                  _stream()))
    return x, {"iters": iters, "rel_res": res, "status": status}


class GridMap:
    """An order of the grid's points in memory (standard rows, param^3
    bricks or the 3D Hilbert curve) with the neighbour table of the 25-point
    stencil in that order.  Batches here are point-major [np, ld]
    complex128 (orbital fastest), in map order."""

    def __init__(self, grid: Grid, kind: int = MAP_STANDARD, param: int = 0):
        self.grid, self.kind, self.param = grid, int(kind), int(param)
        self._h = C.c_void_p()
        _check(_lib.rsg_map_create(grid._h, self.kind, self.param, C.byref(self._h)))

    def order(self) -> np.ndarray:
        """order[i] = compact index of the i-th point in map order."""
        out = np.empty(self.grid.np, dtype=np.int32)
        _check(_lib.rsg_map_order(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def laplacian(self, psi: torch.Tensor, out: torch.Tensor | None = None, nst: int | None = None,
                  scale: float = 1.0) -> torch.Tensor:
        """out[:, :nst] = scale * (8th-order star stencil sum) of psi[:, :nst]."""
        if not (psi.is_cuda and psi.dtype == torch.complex128 and psi.dim() == 2 and psi.is_contiguous()
                and psi.shape[0] == self.grid.np):
            raise ValueError("psi must be a contiguous CUDA complex128 tensor [np, ld]")
        out = torch.zeros_like(psi) if out is None else out
        if not (out.is_cuda and out.dtype == psi.dtype and out.shape == psi.shape and out.is_contiguous()):
            raise ValueError("out must match psi")
        n = psi.shape[1] if nst is None else int(nst)
        _check(_lib.rsg_map_laplacian(self._h, _ptr(psi), _ptr(out), n, psi.shape[1], float(scale),
                                      _stream()))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rsg_map_destroy(h)
            self._h = None


def _nst(t, nst):
    n = t.shape[0] if nst is None else int(nst)
    if not 0 <= n <= t.shape[0]:
        raise ValueError(f"nst = {n} outside 0..{t.shape[0]}")
    return n


def hpsi(ham: Hamiltonian, psi: torch.Tensor, field: float = 0.0, out: torch.Tensor | None = None,
         nst: int | None = None) -> torch.Tensor:
    _batch(psi, "psi", ham.grid.np)
    out = torch.zeros_like(psi) if out is None else _batch(out, "out", ham.grid.np)
    n = _nst(psi, nst)
    ws = _ws(ham.workspace_bytes("hpsi", n, psi.shape[1]), psi.device)
    _check(_lib.rsg_hpsi(ham._h, _ptr(psi), _ptr(out), n, psi.shape[1], C128, float(field),
                         _ptr(ws), ws.numel(), _stream()))
    return out


def _dt(dtype) -> int:
    return {"c128": C128, "mixed": MIXED, C128: C128, MIXED: MIXED}[dtype]


def propagate_step(ham: Hamiltonian, psi: torch.Tensor, dt: float, field: float = 0.0,
                   dtype="c128", nst: int | None = None, ws: torch.Tensor | None = None):
    """One Taylor(4) step in place."""
    _batch(psi, "psi", ham.grid.np)
    n = _nst(psi, nst)
    need = ham.workspace_bytes("step", n, psi.shape[1], _dt(dtype))
    ws = _ws(need, psi.device) if ws is None or ws.numel() < need else ws
    _check(_lib.rsg_propagate_step(ham._h, _ptr(psi), n, psi.shape[1], _dt(dtype), float(dt),
                                   float(field), _ptr(ws), ws.numel(), _stream()))
    return psi


def propagate(ham: Hamiltonian, psi: torch.Tensor, dt: float, nsteps: int,
              fields: torch.Tensor | None = None, graph: bool = False, dtype="c128",
              nst: int | None = None, ws: torch.Tensor | None = None):
    """nsteps Taylor(4) steps in place; fields: CUDA float64 [nsteps] or None."""
    _batch(psi, "psi", ham.grid.np)
    n = _nst(psi, nst)
    if fields is not None and (not fields.is_cuda or fields.dtype != torch.float64
                               or fields.numel() < nsteps):
        raise ValueError("fields must be a CUDA float64 tensor with nsteps entries")
    need = ham.workspace_bytes("step", n, psi.shape[1], _dt(dtype))
    ws = _ws(need, psi.device) if ws is None or ws.numel() < need else ws
    _check(_lib.rsg_propagate(ham._h, _ptr(psi), n, psi.shape[1], _dt(dtype), float(dt),
                              int(nsteps), _ptr(fields), 1 if graph else 0, _ptr(ws), ws.numel(),
                              _stream()))
    return psi


def _grid_of(g):
    return g.grid if isinstance(g, Hamiltonian) else g


def _reduce_ws(grid: Grid, n, device):
    return _ws(int(_lib.rsg_reduce_workspace_bytes(grid._h, n)), device)


def dot(grid: Grid | Hamiltonian, a: torch.Tensor, b: torch.Tensor,
        nst: int | None = None) -> torch.Tensor:
    """<a_n|b_n> = h^3 sum conj(a) b per orbital -> complex128 CUDA [nst]."""
    grid = _grid_of(grid)
    _batch(a, "a", grid.np)
    _batch(b, "b", grid.np)
    if a.shape != b.shape:
        raise ValueError("a and b must have the same shape")
    n = _nst(a, nst)
    out = torch.empty(2 * n, dtype=torch.float64, device=a.device)
    ws = _reduce_ws(grid, n, a.device)
    _check(_lib.rsg_dot(grid._h, _ptr(a), _ptr(b), n, a.shape[1], _ptr(out), _ptr(ws),
                        ws.numel(), _stream()))
    return torch.view_as_complex(out.view(n, 2))


def norm2(grid: Grid | Hamiltonian, a: torch.Tensor, nst: int | None = None) -> torch.Tensor:
    """h^3 sum |a_n|^2 per orbital -> float64 CUDA [nst]."""
    grid = _grid_of(grid)
    _batch(a, "a", grid.np)
    n = _nst(a, nst)
    out = torch.empty(n, dtype=torch.float64, device=a.device)
    ws = _reduce_ws(grid, n, a.device)
    _check(_lib.rsg_norm2(grid._h, _ptr(a), n, a.shape[1], _ptr(out), _ptr(ws), ws.numel(),
                          _stream()))
    return out


def energy(ham: Hamiltonian, psi: torch.Tensor, field: float = 0.0,
           nst: int | None = None) -> torch.Tensor:
    """<psi_n|H psi_n> per orbital -> complex128 CUDA [nst]."""
    _batch(psi, "psi", ham.grid.np)
    n = _nst(psi, nst)
    out = torch.empty(2 * n, dtype=torch.float64, device=psi.device)
    ws = _ws(ham.workspace_bytes("energy", n, psi.shape[1]), psi.device)
    _check(_lib.rsg_energy(ham._h, _ptr(psi), n, psi.shape[1], C128, float(field), _ptr(out),
                           _ptr(ws), ws.numel(), _stream()))
    return torch.view_as_complex(out.view(n, 2))


def dipole_expectation(ham: Hamiltonian, a: torch.Tensor, nst: int | None = None) -> torch.Tensor:
    _batch(a, "a", ham.grid.np)
    n = _nst(a, nst)
    out = torch.empty(n, dtype=torch.float64, device=a.device)
    ws = _reduce_ws(ham.grid, n, a.device)
    _check(_lib.rsg_dipole_expectation(ham._h, _ptr(a), n, a.shape[1], _ptr(out), _ptr(ws),
                                       ws.numel(), _stream()))
    return out


def adjoint_step(ham: Hamiltonian, psi_n: torch.Tensor, lam: torch.Tensor, dt: float,
                 field: float, nst: int | None = None) -> torch.Tensor:
    """lam <- T4(+i dt H) lam in place; returns g_n = dJ/dE_n (CUDA float64 [1])."""
    _batch(psi_n, "psi_n", ham.grid.np)
    _batch(lam, "lambda", ham.grid.np)
    n = _nst(psi_n, nst)
    g = torch.zeros(1, dtype=torch.float64, device=psi_n.device)
    ws = _ws(ham.workspace_bytes("adjoint", n, psi_n.shape[1]), psi_n.device)
    _check(_lib.rsg_adjoint_step(ham._h, _ptr(psi_n), _ptr(lam), n, psi_n.shape[1], float(dt),
                                 float(field), _ptr(g), _ptr(ws), ws.numel(), _stream()))
    return g


def laser_field(coef: torch.Tensor, T: float, dt: float, nsteps: int, step0: int = 0) -> torch.Tensor:
    out = torch.empty(int(nsteps), dtype=torch.float64, device=coef.device)
    c = coef.to(torch.float64).contiguous()
    _check(_lib.rsg_laser_field(_ptr(c), c.numel(), float(T), float(dt), int(step0), int(nsteps),
                                _ptr(out), _stream()))
    return out


def laser_grad(g: torch.Tensor, T: float, dt: float, ncoef: int) -> torch.Tensor:
    out = torch.empty(int(ncoef), dtype=torch.float64, device=g.device)
    gg = g.to(torch.float64).contiguous()
    _check(_lib.rsg_laser_grad(_ptr(gg), gg.numel(), float(T), float(dt), int(ncoef), _ptr(out),
                               _stream()))
    return out


def _control_ws(ham, n, ldp, nsteps, ckpt, device, workspace="full"):
    if workspace not in ("full", "min"):
        raise ValueError("workspace must be 'full' or 'min'")
    fn = _lib.rsg_control_workspace_bytes if workspace == "full" else _lib.rsg_control_workspace_bytes_min
    return _ws(int(fn(ham._h, n, ldp, nsteps, ckpt)), device)


def control_forward(ham: Hamiltonian, psi: torch.Tensor, dt: float, nsteps: int,
                    coef: torch.Tensor, ckpt_every: int, keep_checkpoints: bool = True,
                    workspace: str = "full"):
    """Propagate psi in place to T = nsteps*dt under the sine-series field.
    Returns (J as CUDA float64 [1], checkpoint store or None).  workspace:
    "full" or "min" scratch size (the forward pass needs only the minimum)."""
    _batch(psi, "psi", ham.grid.np)
    n, ldp = psi.shape[0], psi.shape[1]
    c = coef.to(torch.float64).contiguous()
    nck = nsteps // ckpt_every + 1
    ck = (torch.empty((nck, n, ldp), dtype=torch.complex128, device=psi.device)
          if keep_checkpoints else None)
    J = torch.zeros(1, dtype=torch.float64, device=psi.device)
    ws = _control_ws(ham, n, ldp, nsteps, ckpt_every, psi.device, workspace)
    _check(_lib.rsg_control_forward(ham._h, _ptr(psi), n, ldp, float(dt), int(nsteps), _ptr(c),
                                    c.numel(), int(ckpt_every), _ptr(ck), _ptr(J), _ptr(ws),
                                    ws.numel(), _stream()))
    return J, ck


def control_backward(ham: Hamiltonian, psi_T: torch.Tensor, dt: float, nsteps: int,
                     coef: torch.Tensor, ckpt_every: int, ckpt: torch.Tensor, workspace: str = "full"):
    """(dJ/dc [ncoef], dJ/dE_n [nsteps]) by checkpointed discrete adjoint.
    workspace "full" keeps every step's stage outputs of a segment (4 orbital
    batches per step); "min" keeps the states only and recomputes the stage
    outputs in each adjoint step (same results, more stencil work)."""
    _batch(psi_T, "psi_T", ham.grid.np)
    n, ldp = psi_T.shape[0], psi_T.shape[1]
    if ckpt is None or tuple(ckpt.shape) != (nsteps // ckpt_every + 1, n, ldp):
        raise ValueError("checkpoint store does not match psi_T and the step count")
    c = coef.to(torch.float64).contiguous()
    grad = torch.zeros(c.numel(), dtype=torch.float64, device=psi_T.device)
    gs = torch.zeros(int(nsteps), dtype=torch.float64, device=psi_T.device)
    ws = _control_ws(ham, n, ldp, nsteps, ckpt_every, psi_T.device, workspace)
    _check(_lib.rsg_control_backward(ham._h, _ptr(psi_T), n, ldp, float(dt), int(nsteps), _ptr(c),
                                     c.numel(), int(ckpt_every), _ptr(ckpt), _ptr(grad), _ptr(gs),
                                     _ptr(ws), ws.numel(), _stream()))
    return grad, gs


class OptimalControlJ(torch.autograd.Function):
    """J(c) = sum_n <psi_n(T)| x_axis |psi_n(T)> for the field
    E(t) = sum_k c_k sin(k pi t / T); backward gives dJ/dc by the
    checkpointed discrete adjoint (section "Quantum optimal control",
    eq. (qoctgradient))."""

    @staticmethod
    def forward(ctx, coef, ham, psi0, dt, nsteps, ckpt_every):
        psi = psi0.detach().clone()
        J, ck = control_forward(ham, psi, dt, nsteps, coef.detach(), ckpt_every)
        ctx.ham, ctx.dt, ctx.nsteps, ctx.ckpt_every = ham, dt, nsteps, ckpt_every
        ctx.save_for_backward(coef.detach(), psi, ck)
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        coef, psiT, ck = ctx.saved_tensors
        grad, _ = control_backward(ctx.ham, psiT, ctx.dt, ctx.nsteps, coef, ctx.ckpt_every, ck)
        return gJ * grad, None, None, None, None, None


def copy(src: torch.Tensor, dst: torch.Tensor):
    nb = src.numel() * src.element_size()
    _check(_lib.rsg_copy(_ptr(src), _ptr(dst), nb, _stream()))


class kernel_timing:
    """Context manager: HIP-event timing of every stencil-kernel launch.
    After exit, ``.count`` launches and ``.mean_ms`` average duration."""

    def __enter__(self):
        _check(_lib.rsg_timing_query(None, None, None))  # drop stale events
        _check(_lib.rsg_timing_enable(1))
        return self

    def __exit__(self, *exc):
        _check(_lib.rsg_timing_enable(0))
        n, m, t = C.c_int64(), C.c_double(), C.c_double()
        _check(_lib.rsg_timing_query(C.byref(n), C.byref(m), C.byref(t)))
        self.count, self.mean_ms, self.total_ms = int(n.value), float(m.value), float(t.value)
        return False


class _Tile(C.Structure):
    _fields_ = [("B", C.c_int32), ("TX", C.c_int32), ("TY", C.c_int32), ("ZC", C.c_int32),
                ("PD", C.c_int32), ("PT", C.c_int32), ("BO", C.c_int32), ("ZM", C.c_int32)]


def _tile_dict(t: _Tile) -> dict:
    return {"B": t.B, "TX": t.TX, "TY": t.TY, "ZC": t.ZC, "PD": t.PD, "PT": t.PT, "BO": t.BO,
            "ZM": t.ZM}


def tile_candidates(dtype="c128") -> list:
    n = C.c_int32()
    _check(_lib.rsg_tile_candidates(_dt(dtype), None, 0, C.byref(n)))
    arr = (_Tile * n.value)()
    _check(_lib.rsg_tile_candidates(_dt(dtype), arr, n.value, C.byref(n)))
    return [_tile_dict(t) for t in arr]


def set_tile(ham: Hamiltonian, nst: int, B: int, TX: int, TY: int, ZC: int = 0, PD: int = 1,
             PT: int = 0, BO: int = 0, ZM: int = 0, dtype="c128"):
    t = _Tile(B, TX, TY, ZC, PD, PT, BO, ZM)
    _check(_lib.rsg_set_tile(ham._h, int(nst), _dt(dtype), C.byref(t)))


def get_tile(ham: Hamiltonian, nst: int, dtype="c128") -> dict:
    t = _Tile()
    _check(_lib.rsg_get_tile(ham._h, int(nst), _dt(dtype), C.byref(t)))
    return _tile_dict(t)


def autotune(ham: Hamiltonian, psi: torch.Tensor, dtype="c128", reps: int = 3,
             nst: int | None = None):
    """Time the compiled tile shapes on a later Taylor stage of psi, re-time
    the six fastest on a whole step's stencil work (first stage + three
    later ones) and keep the fastest for this (nst, dtype); returns (tile,
    milliseconds of stencil work per step)."""
    _batch(psi, "psi", ham.grid.np)
    n = _nst(psi, nst)
    ws = _ws(ham.workspace_bytes("step", n, psi.shape[1], _dt(dtype)), psi.device)
    t = _Tile()
    ms = C.c_double()
    _check(_lib.rsg_autotune(ham._h, _ptr(psi), n, psi.shape[1], _dt(dtype), _ptr(ws), ws.numel(),
                             int(reps), C.byref(t), C.byref(ms), _stream()))
    return _tile_dict(t), float(ms.value)


def autotune_cached(ham: Hamiltonian, psi: torch.Tensor, cache_path: str, dtype="c128", reps: int = 3,
                    nst: int | None = None):
    """autotune through the tile cache file cache_path: returns (tile,
    milliseconds, cached) with cached True when the tile came from the file
    (no kernel was launched)."""
    _batch(psi, "psi", ham.grid.np)
    n = _nst(psi, nst)
    ws = _ws(ham.workspace_bytes("step", n, psi.shape[1], _dt(dtype)), psi.device)
    t = _Tile()
    ms = C.c_double()
    hit = C.c_int32()
    _check(_lib.rsg_autotune_cache(ham._h, _ptr(psi), n, psi.shape[1], _dt(dtype), _ptr(ws), ws.numel(),
                                   int(reps), os.fsencode(cache_path), C.byref(t), C.byref(ms), C.byref(hit),
                                   _stream()))
    return _tile_dict(t), float(ms.value), bool(hit.value)


class _SysDesc(C.Structure):
    _fields_ = [("ham", C.c_void_p), ("psi", C.c_void_p), ("nst", C.c_int64), ("ldp", C.c_int64)]


class Batch:
    """Many independent systems propagated together: each stage of a
    Taylor(4) step of all systems is one persistent stencil launch.

    systems: list of (Hamiltonian, psi, nst) with psi a CUDA complex128
    [>= nst, ldp] orbital-major tensor propagated in place.  The Hamiltonians and tensors must
    stay alive while the batch is used."""

    def __init__(self, systems):
        self.systems = list(systems)
        n = len(self.systems)
        descs = (_SysDesc * n)()
        for k, (ham, psi, nst) in enumerate(self.systems):
            _batch(psi, "psi", ham.grid.np)
            if not 1 <= int(nst) <= psi.shape[0]:
                raise ValueError(f"system {k}: nst = {nst} outside 1..{psi.shape[0]}")
            descs[k] = _SysDesc(ham._h.value, psi.data_ptr(), int(nst), psi.shape[1])
        self._descs = descs
        nbytes = int(_lib.rsg_batch_workspace_bytes(n, descs))
        if nbytes == 0:
            raise ValueError("invalid system list")
        self.ws = _ws(nbytes, self.systems[0][1].device)
        self._h = C.c_void_p()
        torch.cuda.synchronize()
        _check(_lib.rsg_batch_create(n, descs, _ptr(self.ws), self.ws.numel(), _stream(),
                                     C.byref(self._h)))

    def set_tile(self, B: int, TX: int, TY: int, ZC: int = 0, PD: int = 1, ZM: int = 0,
                 cls: int | None = None):
        """Tile of every size class (cls = None) or of class cls."""
        t = _Tile(B, TX, TY, ZC, PD, 0, 0, ZM)
        if cls is None:
            _check(_lib.rsg_batch_set_tile(self._h, C.byref(t), _stream()))
        else:
            _check(_lib.rsg_batch_set_class_tile(self._h, int(cls), C.byref(t), _stream()))

    def get_tile(self, cls: int | None = None) -> dict:
        t = _Tile()
        if cls is None:
            _check(_lib.rsg_batch_get_tile(self._h, C.byref(t)))
        else:
            _check(_lib.rsg_batch_get_class_tile(self._h, int(cls), C.byref(t)))
        return _tile_dict(t)

    def classes(self) -> np.ndarray:
        """Size class of every system."""
        n = C.c_int32()
        out = np.zeros(len(self.systems), dtype=np.int32)
        _check(_lib.rsg_batch_classes(self._h, C.byref(n), out.ctypes.data_as(C.c_void_p)))
        return out

    def set_classes(self, class_of_sys):
        c = np.ascontiguousarray(class_of_sys, dtype=np.int32)
        if c.shape != (len(self.systems),):
            raise ValueError("one class per system")
        _check(_lib.rsg_batch_set_classes(self._h, c.ctypes.data_as(C.c_void_p), _stream()))

    def class_info(self, cls: int) -> dict:
        """{nsys, nitems, grid} of size class cls: systems, stencil work items
        per stage, persistent workgroups per launch."""
        ns, ni, gr = C.c_int32(), C.c_int64(), C.c_int32()
        _check(_lib.rsg_batch_class_info(self._h, int(cls), C.byref(ns), C.byref(ni), C.byref(gr)))
        return {"nsys": ns.value, "nitems": ni.value, "grid": gr.value}

    def set_grid(self, max_workgroups: int):
        """Cap the persistent grid of every stencil launch (0: no cap)."""
        _check(_lib.rsg_batch_set_grid(self._h, int(max_workgroups)))

    def autotune(self, reps: int = 2):
        t = _Tile()
        ms = C.c_double()
        _check(_lib.rsg_batch_autotune(self._h, int(reps), C.byref(t), C.byref(ms), _stream()))
        return _tile_dict(t), float(ms.value)

    def propagate(self, dt: float, nsteps: int, graph: bool = False):
        _check(_lib.rsg_batch_propagate(self._h, float(dt), int(nsteps), 1 if graph else 0,
                                        _stream()))

    def run(self, nsteps: int, dt: float):
        """rsg_batch_run: graph-captured steps (needs a non-default stream)."""
        _check(_lib.rsg_batch_run(self._h, int(nsteps), float(dt), _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rsg_batch_destroy(h)
            self._h = None
