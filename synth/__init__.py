"""Seeded synthetic inputs for the real-space Kohn-Sham H*psi path.

This module is shared by the FP64 oracle tests, the GPU parity tests and the
benchmark.  It holds none of the method's arithmetic: it draws seeded random
numbers and evaluates the synthetic *input* functions (potential wells,
projector functions, initial orbitals, laser coefficients) at grid positions
that the caller supplies.  The grid itself (box membership, compact order,
positions) is built separately by each side.

The paper's own workloads are real molecules described by pseudopotentials
(e.g. an N2 molecule in a sphere of radius 7.4 Angstrom at spacing 0.16
Angstrom, and the 500,000-point spherical grid of the GPU Laplacian figure in
the section "Parallelization, optimizations and graphics processing units").
Neither the pseudopotentials nor the geometries are available, so these
inputs stand in for them with the same shapes: spheres of 10^4..10^6 points,
tens of orbitals, a handful of atoms with separable projectors.

Every array is built from ``numpy.random.Generator(PCG64)`` streams keyed by
(seed, purpose), so each input can be regenerated independently.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Workload descriptions.  Sizes follow the five configurations the project is
# measured on; the names are what the tests and the benchmark refer to.
# ---------------------------------------------------------------------------

WORKLOADS = {
    # 32^3 cube, harmonic potential, 4 white-noise orbitals, no projectors:
    # 10 H*psi applications + 10 Taylor(4) steps.
    # Shifted solves (Sternheimer step): sphere R = 9.85 bohr at h = 0.2
    # (500,199 points), 16 white-noise right-hand sides, 4 wells with
    # projectors, shifts sigma_n = -eps_n + omega + i eta with eps_n ~
    # U(-0.6, -0.1) Ha, omega = 0.3 Ha, eta = 0.1 Ha; QMR to 1e-8.
    "sphere500k_qmr": dict(shape="sphere", R=9.85, h=0.2, nst=16, natoms=4, well_ball=4.0,
                           omega=0.3, eta=0.1, eps_lo=-0.6, eps_hi=-0.1, tol=1e-8,
                           maxiter=4000, seed=7),
    # Mixed precision at the benchmark scale: the sphere18_wells system
    # propagated with FP32 Hamiltonian arithmetic and complex64 work buffers.
    "sphere18_mixed": dict(base="sphere18_wells", steps=20),
    # Complex scaling: H_theta applications on the sphere18 grid (64
    # orbitals, its 16 wells continued to r e^{i theta}, no projectors), and
    # the levels of the harmonic oscillator continued to e^{2 i theta} r^2/2
    # on a 48^3 cube at h = 0.3 by inverse iteration from 4 targets.
    "sphere18_cs": dict(R=18.0, h=0.2, nst=64, natoms=16, well_ball=12.0, seed=2, theta=0.3,
                        cube_n=48, cube_h=0.3, targets=(1.45, 2.45, 3.45, 4.45)),
    # Grid-to-memory map study: spheres of 5.0e5 points (R = 9.85, h = 0.2)
    # and 3.05e6 points (R = 18, h = 0.2), point-major batches of 1..64
    # white-noise orbitals; standard, 4^3 / 8^3 brick and Hilbert orders.
    "sphere500k_gridmap": dict(shape="sphere", spheres=((9.85, 0.2), (18.0, 0.2)),
                               nst_list=(1, 4, 16, 64), seed=6,
                               maps=(("standard", 0, 0), ("bricks4", 1, 4), ("bricks8", 1, 8),
                                     ("hilbert", 2, 0))),
    "cube32_ho": dict(shape="cube", n=32, h=0.3, nst=4, potential="harmonic",
                      natoms=0, kb=False, steps=10, hpsi_calls=10, dt=0.01,
                      seed=1, orbitals="white"),
    # Sphere R=18 bohr at h=0.2 (3,053,617 points), 64 white-noise orbitals,
    # 16 Gaussian wells with 4 projectors each, 100 Taylor(4) steps.
    "sphere18_wells": dict(shape="sphere", R=18.0, h=0.2, nst=64,
                           potential="wells", natoms=16, well_ball=12.0,
                           kb=True, steps=100, dt=0.005, seed=2,
                           orbitals="white"),
    # 256 independent spheres, R ~ U(4,12) at h=0.25, nst ~ U{1..32},
    # 1..8 wells each with projectors, 50 Taylor(4) steps.
    "batch256": dict(shape="batch", nsys=256, Rmin=4.0, Rmax=12.0, h=0.25,
                     nst_max=32, atoms_max=8, kb=True, steps=50, dt=0.005,
                     seed=3),
    # The cube32 system with FP32 Hamiltonian arithmetic, 1000 steps.
    "cube32_mixed": dict(shape="cube", n=32, h=0.3, nst=4, potential="harmonic",
                         natoms=0, kb=False, steps=1000, dt=0.01, seed=4,
                         orbitals="white"),
    # Optimal control: 96^3 cube at h=0.3, 8 orthonormal packets, 4 wells,
    # E(t) = sum_k c_k sin(k pi t / T), 64 coefficients, 2000 steps dt=0.01.
    "cube96_control": dict(shape="cube", n=96, h=0.3, nst=8,
                           potential="wells", natoms=4, well_box=6.0,
                           kb=False, steps=2000, dt=0.01, ncoef=64,
                           checkpoint=50, seed=5, orbitals="packets"),
}


def rng(seed: int, purpose: int) -> np.random.Generator:
    """Independent PCG64 stream for (seed, purpose)."""
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence(entropy=seed, spawn_key=(purpose,))))


# purposes (stream keys)
_P_ORB, _P_WELLS, _P_KB_E, _P_LASER, _P_BATCH, _P_PACKETS, _P_MISC = range(7)


# ---------------------------------------------------------------------------
# Orbitals
# ---------------------------------------------------------------------------

def white_noise(seed: int, npts: int, nst: int, h: float, ld: int | None = None,
                purpose: int = _P_ORB) -> np.ndarray:
    """(N(0,1) + i N(0,1))/sqrt(2) per point and orbital, each orbital scaled
    to h^3 sum |psi|^2 = 1.  Layout [npts][ld], orbital index fastest; the
    padding columns nst..ld-1 are zero."""
    ld = nst if ld is None else ld
    g = rng(seed, purpose)
    out = np.zeros((npts, ld), dtype=np.complex128)
    re = g.standard_normal((npts, nst))
    out.real[:, :nst] = re
    del re
    im = g.standard_normal((npts, nst))
    out.imag[:, :nst] = im
    del im
    nrm = np.sqrt((np.abs(out[:, :nst]) ** 2).sum(axis=0) * h ** 3)
    out[:, :nst] /= nrm
    return out


def ho_ground_state(pos: np.ndarray) -> np.ndarray:
    """Continuum-normalised ground state of V = r^2/2: pi^(-3/4) exp(-r^2/2)."""
    r2 = (pos ** 2).sum(axis=1)
    return (math.pi ** -0.75) * np.exp(-0.5 * r2)


def ho_low_states(pos: np.ndarray, nst: int) -> np.ndarray:
    """Ground state and first excited states (x, y, z times the ground state)
    of the 3D harmonic oscillator, continuum-normalised, layout [npts][nst]."""
    g = ho_ground_state(pos)
    cols = [g, math.sqrt(2.0) * pos[:, 0] * g, math.sqrt(2.0) * pos[:, 1] * g,
            math.sqrt(2.0) * pos[:, 2] * g]
    while len(cols) < nst:
        cols.append(cols[len(cols) % 4])
    return np.stack(cols[:nst], axis=1).astype(np.complex128)


def gaussian_packets(seed: int, pos: np.ndarray, nst: int, h: float,
                     width: float = 1.0, centre_box: float = 5.0) -> np.ndarray:
    """nst Gaussian packets (width 1 bohr, seeded centres in [-5,5]^3, seeded
    small momenta and phases), Loewdin-orthonormalised in FP64 with respect
    to h^3 sum conj(a) b.  Layout [npts][nst]."""
    g = rng(seed, _P_PACKETS)
    centres = g.uniform(-centre_box, centre_box, size=(nst, 3))
    kvec = g.uniform(-0.5, 0.5, size=(nst, 3))
    phase = g.uniform(0.0, 2.0 * math.pi, size=nst)
    psi = np.empty((pos.shape[0], nst), dtype=np.complex128)
    for n in range(nst):
        d = pos - centres[n]
        env = np.exp(-(d ** 2).sum(axis=1) / (2.0 * width ** 2))
        psi[:, n] = env * np.exp(1j * (pos @ kvec[n] + phase[n]))
    s = (psi.conj().T @ psi) * h ** 3
    w, u = np.linalg.eigh(s)
    s_inv_half = (u * (1.0 / np.sqrt(w))) @ u.conj().T
    return psi @ s_inv_half


# ---------------------------------------------------------------------------
# Potentials and projectors
# ---------------------------------------------------------------------------

def harmonic_potential(pos: np.ndarray) -> np.ndarray:
    return 0.5 * (pos ** 2).sum(axis=1)


@dataclass
class Wells:
    centres: np.ndarray   # [natoms][3]
    depth: np.ndarray     # [natoms], Hartree
    width: np.ndarray     # [natoms], bohr


def gaussian_wells(seed: int, natoms: int, ball: float | None = None,
                   box: float | None = None, purpose: int = _P_WELLS) -> Wells:
    """natoms wells with depth ~ U(2,6) Ha and width ~ U(0.8,1.5) bohr.
    Centres uniform in a ball of radius ``ball`` or a cube [-box, box]^3."""
    g = rng(seed, purpose)
    if ball is not None:
        dirs = g.standard_normal((natoms, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        radii = ball * g.uniform(0.0, 1.0, size=natoms) ** (1.0 / 3.0)
        centres = dirs * radii[:, None]
    else:
        centres = g.uniform(-box, box, size=(natoms, 3))
    depth = g.uniform(2.0, 6.0, size=natoms)
    width = g.uniform(0.8, 1.5, size=natoms)
    return Wells(centres, depth, width)


def well_potential(pos: np.ndarray, wells: Wells) -> np.ndarray:
    """V(r) = -sum_a D_a exp(-|r - R_a|^2 / (2 w_a^2))."""
    v = np.zeros(pos.shape[0])
    for c, d, w in zip(wells.centres, wells.depth, wells.width):
        v -= d * np.exp(-((pos - c) ** 2).sum(axis=1) / (2.0 * w * w))
    return v


@dataclass
class Projectors:
    """Separable projectors, 4 per atom (s, p_x, p_y, p_z).

    idx[a]   int32 [n_a]      compact indices of the support S_a
    p[a]     float64 [n_a][4] projector values on S_a
    E[a]     float64 [4]      projector energies (Hartree)
    """
    idx: list = field(default_factory=list)
    p: list = field(default_factory=list)
    E: list = field(default_factory=list)

    @property
    def natoms(self) -> int:
        return len(self.idx)


def kb_projectors(seed: int, pos: np.ndarray, centres: np.ndarray,
                  rc: float = 0.6, rcut: float = 2.0,
                  purpose: int = _P_KB_E) -> Projectors:
    """p_s = exp(-d^2/(2 rc^2)), p_a = (d_a/rc) exp(-d^2/(2 rc^2)) for the
    points with |d| <= rcut; energies E ~ U(0.5, 2.0) Ha per projector."""
    g = rng(seed, purpose)
    out = Projectors()
    for c in centres:
        lo = c - rcut - 1e-9
        hi = c + rcut + 1e-9
        box = np.nonzero(np.all((pos >= lo) & (pos <= hi), axis=1))[0]
        d = pos[box] - c
        d2 = (d ** 2).sum(axis=1)
        keep = d2 <= rcut * rcut
        sel = box[keep]
        d = d[keep]
        env = np.exp(-d2[keep] / (2.0 * rc * rc))
        pv = np.empty((sel.size, 4))
        pv[:, 0] = env
        pv[:, 1:] = d / rc * env[:, None]
        out.idx.append(sel.astype(np.int32))
        out.p.append(np.ascontiguousarray(pv))
        out.E.append(g.uniform(0.5, 2.0, size=4))
    return out


def well_potential_scaled(pos: np.ndarray, wells: Wells, theta: float) -> np.ndarray:
    """The wells' potential continued to r e^{i theta} (complex scaling about
    the origin): -sum_a D_a exp(-sum_k (x_k e^{i theta} - R_ak)^2 / (2 w_a^2))."""
    z = pos * np.exp(1j * theta)
    v = np.zeros(pos.shape[0], dtype=np.complex128)
    for c, d, w in zip(wells.centres, wells.depth, wells.width):
        v -= d * np.exp(-((z - c) ** 2).sum(axis=1) / (2.0 * w * w))
    return v


def resonance_potential_1d(x: np.ndarray, theta: float) -> np.ndarray:
    """The one-dimensional well with barriers of the complex-scaling
    section's spectrum figure, v(x) = 3 (x^2 - 2) exp(-x^2 / 4), continued
    to x e^{i theta} (theta = 0 gives the real potential)."""
    z = np.asarray(x, dtype=np.float64) * np.exp(1j * theta)
    return 3.0 * (z * z - 2.0) * np.exp(-z * z / 4.0)


def radial_mask(pos: np.ndarray, R: float, width: float) -> np.ndarray:
    """Real mask M(r) for the boundary absorber: 1 inside |r| <= R - width,
    cos^2 ramp to 0 at |r| = R, 0 beyond.  The paper leaves the mask's form
    open; this smooth radial ramp is the input used here."""
    r = np.linalg.norm(pos, axis=1)
    t = np.clip((r - (R - width)) / width, 0.0, 1.0)
    return np.where(t >= 1.0, 0.0, np.cos(0.5 * np.pi * t) ** 2)


def laser_coefficients(seed: int, ncoef: int, sigma: float = 0.005) -> np.ndarray:
    """Sine-series coefficients c_k ~ N(0, sigma^2) of the control field."""
    return rng(seed, _P_LASER).normal(0.0, sigma, size=ncoef)


# ---------------------------------------------------------------------------
# Batched workload: many independent spheres
# ---------------------------------------------------------------------------

@dataclass
class SystemSpec:
    R: float
    h: float
    nst: int
    wells: Wells
    seed: int


def batch_specs(seed: int, nsys: int, Rmin: float = 4.0, Rmax: float = 12.0,
                h: float = 0.25, nst_max: int = 32, atoms_max: int = 8) -> list:
    g = rng(seed, _P_BATCH)
    specs = []
    for s in range(nsys):
        R = float(g.uniform(Rmin, Rmax))
        nst = int(g.integers(1, nst_max + 1))
        na = int(g.integers(1, atoms_max + 1))
        wells = gaussian_wells(seed * 100003 + s, na, ball=max(R - 3.0, 0.5))
        specs.append(SystemSpec(R=R, h=h, nst=nst, wells=wells,
                                seed=seed * 100003 + s))
    return specs


def random_unit(seed: int, n: int, purpose: int = _P_MISC) -> np.ndarray:
    """A seeded random direction (unit 2-norm) of length n."""
    v = rng(seed, purpose).standard_normal(n)
    return v / np.linalg.norm(v)
