"""Degenerate requests through the C ABI: zero orbitals and zero steps are
valid and leave every buffer as it was; the first orbitals of a wider batch
are the only ones touched (the rest, and the padding, keep their values)."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import System, orbital_rel_err, rsg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sys_():
    return System(0.3, R=3.1, potential="wells", natoms=2, nst=3, ld=5, seed=41, dipole_axis=1,
                  well_ball=1.0, pad=3)


def test_zero_orbitals_touch_nothing(sys_):
    s, R = sys_, rsg()
    psi = s.to_gpu(s.psi)
    before = psi.clone()
    out = torch.full_like(psi, 7.0 - 2.0j)
    R.hpsi(s.gh, psi, field=0.3, out=out, nst=0)
    assert torch.all(out == 7.0 - 2.0j)
    R.propagate_step(s.gh, psi, 0.01, field=0.3, nst=0)
    R.propagate(s.gh, psi, 0.01, 3, nst=0)
    assert torch.equal(psi, before)
    assert R.norm2(s.gg, psi, nst=0).numel() == 0


def test_zero_steps_touch_nothing(sys_):
    s, R = sys_, rsg()
    psi = s.to_gpu(s.psi)
    before = psi.clone()
    R.propagate(s.gh, psi, 0.01, 0)
    R.propagate(s.gh, psi, 0.01, 0, graph=True)
    assert torch.equal(psi, before)


def test_leading_orbitals_only(sys_):
    """nst = 2 of a 5-wide batch: orbitals 0, 1 step as the oracle's, orbitals
    2..4 and the padding points keep their bits."""
    s, R = sys_, rsg()
    psi = s.to_gpu(s.psi)
    before = psi.clone()
    R.propagate_step(s.gh, psi, 0.01, field=0.3, nst=2)
    ref = oracle.taylor_step(s.oh, s.psi, 0.01, field=0.3, nst=2)
    assert orbital_rel_err(s.from_gpu(psi), ref, 2) <= 1e-12
    assert torch.equal(psi[2:], before[2:])
    assert s.pad_untouched(psi)
