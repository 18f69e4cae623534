"""Shared helpers of the GPU parity tests: build one system on both sides
from the same seeded inputs and compare results to the stated tolerance.

The oracle works on point-major arrays [np, ld]; the library takes
orbital-major tensors [nst, ldp].  to_om / from_om convert between the two
(a transpose plus optional padding points), nothing else."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def rsg():
    import paper_1501_05654_amd as m
    return m


# Value written into the padding points (np..ldp-1) of every orbital-major
# tensor the tests build, so that tests can check they stay untouched.
PAD = 7.0 - 3.0j


def to_om(a: np.ndarray, pad: int = 0) -> torch.Tensor:
    """Point-major [np, ld] array (the oracle's layout) -> orbital-major CUDA
    tensor [ld, np + pad], padding points set to PAD."""
    npts, ld = a.shape
    t = np.full((ld, npts + pad), PAD, dtype=np.complex128)
    t[:, :npts] = a.T
    return torch.from_numpy(t).to("cuda")


def from_om(t: torch.Tensor, npts: int) -> np.ndarray:
    """Orbital-major tensor [ld, ldp] -> point-major [np, ld] numpy array."""
    return np.ascontiguousarray(t.detach().cpu().numpy()[:, :npts].T)


def pad_untouched(t: torch.Tensor, npts: int) -> bool:
    return bool(np.all(t.detach().cpu().numpy()[:, npts:] == PAD))


class System:
    """One grid + Hamiltonian on the oracle and on the GPU, built from the
    same synth inputs evaluated at the oracle's grid positions.  The GPU
    grid is required to match the oracle grid point for point: slot for
    point with align 1, and on its live slots (in the same order) for a
    row-aligned grid, whose dead slots the tests fill with zero."""

    def __init__(self, h, *, R=None, n=None, box=None, potential="wells", natoms=0, nst=4, ld=None,
                 seed=0, dipole_axis=-1, kin=-0.5, well_ball=None, well_box=None, rcut=2.0,
                 orbitals="white", packet_box=5.0, pad=0, align=1):
        R_ = rsg()
        if box is not None:
            self.og = oracle.Grid(h, box=box)
            self.gg = R_.Grid(h, box=box, align=align)
        else:
            self.og = oracle.Grid(h, R=R, n=n)
            self.gg = R_.Grid(h, R=R, n=n, align=align)
        self.live = self.gg.live()
        assert self.gg.npoints == self.og.np and self.gg.dims == tuple(self.og.dims)
        assert align > 1 or self.gg.np == self.og.np
        np.testing.assert_array_equal(self.gg.coords()[self.live], self.og.ijk)
        pos = self.og.positions()
        self.pos = pos
        self.nst = nst
        self.ld = nst if ld is None else ld
        self.pad = pad  # padding points per orbital on the GPU side
        if potential == "harmonic":
            V = synth.harmonic_potential(pos)
            centres = np.zeros((0, 3))
        elif potential == "wells":
            if well_ball is None and well_box is None:
                well_ball = 0.4 * float(np.abs(pos).max())
            wells = synth.gaussian_wells(seed, max(natoms, 1), ball=well_ball, box=well_box)
            V = synth.well_potential(pos, wells)
            centres = wells.centres[:natoms]
        else:
            V = None
            centres = np.zeros((0, 3))
        self.V = V
        self.proj = synth.kb_projectors(seed, pos, centres, rcut=rcut) if natoms else None
        self.oh = oracle.Ham(self.og, V=V, kin=kin, dipole_axis=dipole_axis, projectors=self.proj)
        dev = torch.device("cuda")
        projs = []
        if self.proj is not None:
            for idx, p, E in zip(self.proj.idx, self.proj.p, self.proj.E):
                sidx = self.live[idx].astype(np.int32)
                projs.append((torch.from_numpy(sidx).to(dev), torch.from_numpy(p).to(dev), E))
        Vt = None if V is None else torch.from_numpy(self.slots(V)).to(dev)
        self.gh = R_.Hamiltonian(self.gg, V=Vt, kin=kin, dipole_axis=dipole_axis, projectors=projs)
        if orbitals == "white":
            self.psi = synth.white_noise(seed + 1000, self.og.np, nst, h, ld=self.ld)
        elif orbitals == "packets":
            p = synth.gaussian_packets(seed, pos, nst, h, centre_box=packet_box)
            self.psi = np.zeros((self.og.np, self.ld), dtype=np.complex128)
            self.psi[:, :nst] = p
        else:
            raise ValueError(orbitals)

    def slots(self, v: np.ndarray) -> np.ndarray:
        """Per-point array [npoints, ...] -> per-slot array, zero in dead slots."""
        if self.gg.np == self.og.np:
            return v
        out = np.zeros((self.gg.np,) + v.shape[1:], dtype=v.dtype)
        out[self.live] = v
        return out

    def to_gpu(self, a: np.ndarray) -> torch.Tensor:
        """Oracle-layout [np, ld] -> orbital-major GPU tensor [ld, slots + pad]
        (dead slots zero)."""
        return to_om(self.slots(a), self.pad)

    def from_gpu(self, t: torch.Tensor) -> np.ndarray:
        """Orbital-major GPU tensor -> oracle layout [np, ld] (live slots)."""
        if self.gg.np == self.og.np:
            return from_om(t, self.og.np)
        return np.ascontiguousarray(t.detach().cpu().numpy()[:, self.live].T)

    def dead_values(self, t: torch.Tensor) -> np.ndarray:
        """Values in the dead slots, [ld, ndead]."""
        a = t.detach().cpu().numpy()[:, :self.gg.np]
        mask = np.ones(self.gg.np, dtype=bool)
        mask[self.live] = False
        return a[:, mask]

    def pad_untouched(self, t: torch.Tensor) -> bool:
        return pad_untouched(t, self.gg.np)


def orbital_rel_err(got: np.ndarray, ref: np.ndarray, nst: int) -> float:
    """max over orbitals of ||got_n - ref_n||_2 / ||ref_n||_2."""
    g = got[:, :nst]
    r = ref[:, :nst]
    num = np.linalg.norm(g - r, axis=0)
    den = np.linalg.norm(r, axis=0)
    den = np.where(den == 0, 1.0, den)
    return float((num / den).max())
