"""Plain FP64 CPU oracle for the real-space Kohn-Sham H*psi path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1501_05654_amd``) and never imports it.

The arithmetic lives in ``rsg_oracle.c`` (plain loops, double precision);
this module only marshals numpy arrays into it.  Each function names the
definition it computes; the file header of ``rsg_oracle.c`` lists where each
one comes from in the paper and which readings were taken where the paper is
silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsg_oracle.c")
_LIB = os.path.join(_HERE, "librsg_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE arithmetic: no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        i32, i64, dbl, vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
        L.or_sphere_points.restype = i64
        L.or_sphere_points.argtypes = [dbl, dbl, vp, vp]
        L.or_cube_points.restype = i64
        L.or_cube_points.argtypes = [i32, vp, vp]
        L.or_box_points.restype = i64
        L.or_box_points.argtypes = [i32, i32, i32, vp, vp]
        L.or_index_map.argtypes = [vp, i64, vp, vp]
        L.or_positions.argtypes = [vp, vp]
        L.or_hpsi.argtypes = [vp, vp, dbl, vp, i64, i64, vp]
        L.or_dot.argtypes = [vp, vp, vp, i64, i64, vp]
        L.or_norm2.argtypes = [vp, vp, i64, i64, vp]
        L.or_energy.restype = dbl
        L.or_energy.argtypes = [vp, vp, dbl, vp, i64, i64, vp]
        L.or_taylor_step.argtypes = [vp, vp, dbl, dbl, vp, i64, i64]
        L.or_propagate.argtypes = [vp, vp, dbl, i64, vp, vp, i64, i64]
        L.or_propagate_masked.argtypes = [vp, vp, dbl, i64, vp, vp, vp, i64, i64, vp]
        L.or_laser_field.restype = dbl
        L.or_laser_field.argtypes = [vp, i32, dbl, dbl]
        L.or_dipole_target.restype = dbl
        L.or_dipole_target.argtypes = [vp, vp, vp, i64, i64]
        L.or_control_forward.restype = dbl
        L.or_control_forward.argtypes = [vp, vp, dbl, i64, vp, i32, vp, i64, i64]
        L.or_adjoint_step.argtypes = [vp, vp, dbl, dbl, vp, vp, i64, i64, vp]
        L.or_control_gradient.argtypes = [vp, vp, dbl, i64, vp, i32, vp, i64, i64, vp, vp, vp]
        L.or_max_threads.restype = i32
        L.or_set_threads.argtypes = [i32]
        _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().or_max_threads())


def set_threads(n: int):
    """OpenMP thread count of the oracle's loops (timing only)."""
    lib().or_set_threads(int(n))


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _GridS(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("np", C.c_int64), ("h", C.c_double),
                ("ijk", C.c_void_p), ("map", C.c_void_p)]


class _HamS(C.Structure):
    _fields_ = [("V", C.c_void_p), ("kin", C.c_double), ("dipole_axis", C.c_int32),
                ("natoms", C.c_int32), ("kb_off", C.c_void_p), ("kb_idx", C.c_void_p),
                ("kb_p", C.c_void_p), ("kb_E", C.c_void_p), ("kin_im", C.c_double),
                ("V_im", C.c_void_p)]


class Grid:
    """Uniform grid restricted to a sphere (radius R), a cube (n per axis) or
    a rectangular box (box = (nx, ny, nz)), compact order z-major, then y,
    then x."""

    def __init__(self, h: float, *, R: float | None = None, n: int | None = None, box=None):
        L = lib()
        dims = np.zeros(3, dtype=np.int32)
        if box is not None:
            nx, ny, nz = (int(v) for v in box)
            npts = L.or_box_points(nx, ny, nz, _p(dims), None)
            ijk = np.zeros((npts, 3), dtype=np.int32)
            L.or_box_points(nx, ny, nz, _p(dims), _p(ijk))
            self.kind = "box"
        elif R is not None:
            npts = L.or_sphere_points(float(R), float(h), _p(dims), None)
            ijk = np.zeros((npts, 3), dtype=np.int32)
            L.or_sphere_points(float(R), float(h), _p(dims), _p(ijk))
            self.kind = "sphere"
        else:
            npts = L.or_cube_points(int(n), _p(dims), None)
            ijk = np.zeros((npts, 3), dtype=np.int32)
            L.or_cube_points(int(n), _p(dims), _p(ijk))
            self.kind = "cube"
        self.R, self.n, self.box, self.h = R, n, box, float(h)
        self.dims = dims
        self.ijk = ijk
        self.np = int(npts)
        self.map = np.empty(int(dims[0]) * int(dims[1]) * int(dims[2]), dtype=np.int64)
        L.or_index_map(_p(dims), self.np, _p(ijk), _p(self.map))
        self._s = _GridS((C.c_int32 * 3)(*dims.tolist()), self.np, self.h,
                         ijk.ctypes.data, self.map.ctypes.data)

    def positions(self) -> np.ndarray:
        xyz = np.empty((self.np, 3))
        lib().or_positions(C.byref(self._s), _p(xyz))
        return xyz


class Ham:
    """H = kin * Laplacian + V + field * x_axis + separable projectors.

    Complex scaling (section "Complex scaling and resonances"): theta != 0
    makes the kinetic prefactor kin e^{-2 i theta}; V_im is the imaginary
    part of the continued local potential v(r e^{i theta}) (V its real
    part)."""

    def __init__(self, grid: Grid, V=None, kin: float = -0.5, dipole_axis: int = -1,
                 projectors=None, theta: float = 0.0, V_im=None):
        self.grid = grid
        self.V = None if V is None else np.ascontiguousarray(V, dtype=np.float64)
        self.V_im = None if V_im is None else np.ascontiguousarray(V_im, dtype=np.float64)
        self.theta = float(theta)
        kc = complex(kin) * np.exp(-2j * self.theta) if self.theta != 0.0 else complex(kin)
        self.kin = float(kc.real)
        self.kin_im = float(kc.imag)
        self.dipole_axis = int(dipole_axis)
        na = 0 if projectors is None else projectors.natoms
        if na:
            sizes = [len(i) for i in projectors.idx]
            self.kb_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
            self.kb_idx = np.ascontiguousarray(np.concatenate(projectors.idx).astype(np.int32))
            self.kb_p = np.ascontiguousarray(np.concatenate(projectors.p, axis=0))
            self.kb_E = np.ascontiguousarray(np.stack(projectors.E).astype(np.float64))
        else:
            self.kb_off = np.zeros(1, dtype=np.int64)
            self.kb_idx = np.zeros(1, dtype=np.int32)
            self.kb_p = np.zeros(4)
            self.kb_E = np.zeros(4)
        self._s = _HamS(None if self.V is None else self.V.ctypes.data, self.kin,
                        self.dipole_axis, na, self.kb_off.ctypes.data, self.kb_idx.ctypes.data,
                        self.kb_p.ctypes.data, self.kb_E.ctypes.data, self.kin_im,
                        None if self.V_im is None else self.V_im.ctypes.data)


def _c(psi):
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    if a.ndim != 2:
        raise ValueError("orbitals must be [np][ld]")
    return a


def hpsi(ham: Ham, psi, field: float = 0.0, nst: int | None = None) -> np.ndarray:
    """H psi for the first nst columns (default: all)."""
    psi = _c(psi)
    nst = psi.shape[1] if nst is None else nst
    out = np.zeros_like(psi)
    lib().or_hpsi(C.byref(ham.grid._s), C.byref(ham._s), float(field), _p(psi), nst,
                  psi.shape[1], _p(out))
    return out


def dot(grid: Grid, a, b, nst: int | None = None) -> np.ndarray:
    a, b = _c(a), _c(b)
    nst = a.shape[1] if nst is None else nst
    out = np.zeros(nst, dtype=np.complex128)
    lib().or_dot(C.byref(grid._s), _p(a), _p(b), nst, a.shape[1], _p(out))
    return out


def norm2(grid: Grid, a, nst: int | None = None) -> np.ndarray:
    a = _c(a)
    nst = a.shape[1] if nst is None else nst
    out = np.zeros(nst)
    lib().or_norm2(C.byref(grid._s), _p(a), nst, a.shape[1], _p(out))
    return out


def energy(ham: Ham, psi, field: float = 0.0, nst: int | None = None):
    """(total, per-orbital <psi_n|H psi_n>)."""
    psi = _c(psi)
    nst = psi.shape[1] if nst is None else nst
    per = np.zeros(nst, dtype=np.complex128)
    e = lib().or_energy(C.byref(ham.grid._s), C.byref(ham._s), float(field), _p(psi), nst,
                        psi.shape[1], _p(per))
    return e, per


def taylor_step(ham: Ham, psi, dt: float, field: float = 0.0, nst: int | None = None):
    psi = _c(psi).copy()
    nst = psi.shape[1] if nst is None else nst
    lib().or_taylor_step(C.byref(ham.grid._s), C.byref(ham._s), float(dt), float(field),
                         _p(psi), nst, psi.shape[1])
    return psi


def propagate(ham: Ham, psi, dt: float, nsteps: int, fields=None, nst: int | None = None):
    psi = _c(psi).copy()
    nst = psi.shape[1] if nst is None else nst
    f = None if fields is None else np.ascontiguousarray(fields, dtype=np.float64)
    lib().or_propagate(C.byref(ham.grid._s), C.byref(ham._s), float(dt), int(nsteps), _p(f),
                       _p(psi), nst, psi.shape[1])
    return psi


def propagate_masked(ham: Ham, psi, dt: float, nsteps: int, mask, fields=None,
                     nst: int | None = None):
    """nsteps steps of psi <- M U(dt) psi (mask boundary absorber, section
    "Photoemission", eq. (mask_split)).  Returns (psi, removed) with removed[n]
    the charge orbital n lost through the mask over all steps."""
    psi = _c(psi).copy()
    nst = psi.shape[1] if nst is None else nst
    f = None if fields is None else np.ascontiguousarray(fields, dtype=np.float64)
    m = np.ascontiguousarray(mask, dtype=np.float64)
    if m.shape != (ham.grid.np,):
        raise ValueError("mask must have one value per grid point")
    removed = np.zeros(nst)
    lib().or_propagate_masked(C.byref(ham.grid._s), C.byref(ham._s), float(dt), int(nsteps), _p(f),
                              _p(m), _p(psi), nst, psi.shape[1], _p(removed))
    return psi, removed


def laser_field(coef, T: float, t: float) -> float:
    c = np.ascontiguousarray(coef, dtype=np.float64)
    return float(lib().or_laser_field(_p(c), c.size, float(T), float(t)))


def dipole_target(ham: Ham, psi, nst: int | None = None) -> float:
    psi = _c(psi)
    nst = psi.shape[1] if nst is None else nst
    return float(lib().or_dipole_target(C.byref(ham.grid._s), C.byref(ham._s), _p(psi), nst,
                                        psi.shape[1]))


def control_forward(ham: Ham, psi0, dt: float, nsteps: int, coef, nst: int | None = None):
    """(J, psi(T)) for the sine-series field built from coef."""
    psi = _c(psi0).copy()
    nst = psi.shape[1] if nst is None else nst
    c = np.ascontiguousarray(coef, dtype=np.float64)
    J = lib().or_control_forward(C.byref(ham.grid._s), C.byref(ham._s), float(dt), int(nsteps),
                                 _p(c), c.size, _p(psi), nst, psi.shape[1])
    return float(J), psi


def adjoint_step(ham: Ham, psi_n, lam, dt: float, field: float, nst: int | None = None):
    """(lambda_n, g_n) from (psi_n, lambda_{n+1})."""
    psi_n = _c(psi_n)
    lam = _c(lam).copy()
    nst = psi_n.shape[1] if nst is None else nst
    g = np.zeros(1)
    lib().or_adjoint_step(C.byref(ham.grid._s), C.byref(ham._s), float(dt), float(field),
                          _p(psi_n), _p(lam), nst, psi_n.shape[1], _p(g))
    return lam, float(g[0])


def control_gradient(ham: Ham, psi0, dt: float, nsteps: int, coef, nst: int | None = None):
    """(J, dJ/dc[ncoef], g_n[nsteps]) by the discrete adjoint."""
    psi0 = _c(psi0)
    nst = psi0.shape[1] if nst is None else nst
    c = np.ascontiguousarray(coef, dtype=np.float64)
    J = np.zeros(1)
    grad = np.zeros(c.size)
    gs = np.zeros(int(nsteps))
    lib().or_control_gradient(C.byref(ham.grid._s), C.byref(ham._s), float(dt), int(nsteps),
                              _p(c), c.size, _p(psi0), nst, psi0.shape[1], _p(J), _p(grad),
                              _p(gs))
    return float(J[0]), grad, gs
