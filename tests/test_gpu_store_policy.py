"""The stencil's store policy does not change results.  A stage whose output
is 256 MiB or more runs the kernel set with non-temporal output stores, a
smaller one the set with default stores; the values written must be the
same.  On a 1.05 M-point sphere (row-aligned storage, 4 atoms with
projectors, dipole field) one launch over 17 orbitals (FP64, above the
threshold) is compared bit for bit with the same orbitals in two launches
of 8 and 9 (below it), for H psi and for a Taylor(4) step; the mixed step
likewise with 34 orbitals against 17 + 17 (its complex64 stage outputs
cross the threshold at 34).  The tile is fixed for every orbital count so
that only the store policy differs.  Orbital 0 of each one-launch result is
held to the oracle."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import System, orbital_rel_err, rsg

pytestmark = pytest.mark.gpu

NT_BYTES = 256 * 1024 * 1024  # stage outputs of at least this size stream past L2
DT, FIELD = 0.005, 0.2


@pytest.fixture(scope="module")
def big():
    return System(0.2, R=12.6, potential="wells", natoms=4, nst=34, seed=77, dipole_axis=2, align=16)


def _fix_tiles(s, counts, dtype, TX, TY, PD):
    for n in counts:
        rsg().set_tile(s.gh, n, 1, TX, TY, 0, PD, 0, 2, 0, dtype=dtype)


def test_fp64_store_policy_bitwise(big):
    s, R = big, rsg()
    slot = s.gg.np
    assert 17 * slot * 16 >= NT_BYTES > 9 * slot * 16
    print(f"[store-policy] fp64 np={slot} nst=17 vs 8+9", flush=True)
    _fix_tiles(s, (17, 8, 9), "c128", 32, 16, 2)
    psi = s.to_gpu(s.psi)[:17].contiguous()
    one = R.hpsi(s.gh, psi, field=FIELD)
    two = torch.cat([R.hpsi(s.gh, psi[:8].contiguous(), field=FIELD),
                     R.hpsi(s.gh, psi[8:].contiguous(), field=FIELD)])
    assert torch.equal(one, two)
    ref = oracle.hpsi(s.oh, s.psi, field=FIELD, nst=1)
    assert orbital_rel_err(s.from_gpu(one), ref, 1) <= 1e-12

    step_one = psi.clone()
    R.propagate_step(s.gh, step_one, DT, field=FIELD)
    a, b = psi[:8].clone(), psi[8:].clone()
    R.propagate_step(s.gh, a, DT, field=FIELD)
    R.propagate_step(s.gh, b, DT, field=FIELD)
    assert torch.equal(step_one, torch.cat([a, b]))
    ref = oracle.taylor_step(s.oh, s.psi, DT, field=FIELD, nst=1)
    assert orbital_rel_err(s.from_gpu(step_one), ref, 1) <= 1e-12
    assert np.all(s.dead_values(step_one) == 0)


def test_mixed_store_policy_bitwise(big):
    s, R = big, rsg()
    slot = s.gg.np
    assert 34 * slot * 8 >= NT_BYTES > 17 * slot * 8
    print(f"[store-policy] mixed np={slot} nst=34 vs 17+17", flush=True)
    _fix_tiles(s, (34, 17), "mixed", 32, 16, 1)
    psi = s.to_gpu(s.psi)
    one = psi.clone()
    R.propagate_step(s.gh, one, DT, field=FIELD, dtype="mixed")
    a, b = psi[:17].clone(), psi[17:].clone()
    R.propagate_step(s.gh, a, DT, field=FIELD, dtype="mixed")
    R.propagate_step(s.gh, b, DT, field=FIELD, dtype="mixed")
    assert torch.equal(one, torch.cat([a, b]))
    ref = oracle.taylor_step(s.oh, s.psi, DT, field=FIELD, nst=1)
    assert orbital_rel_err(s.from_gpu(one), ref, 1) <= 1e-5
