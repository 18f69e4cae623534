"""The optimal-control gradient at the size of its workload (section "Quantum
optimal control"): the 96^3 cube at h = 0.3 with 8 orthonormal packets, 4
wells, the field along z as a sine series of 64 coefficients, 400 steps with
checkpoints every 50.  The adjoint gradient along a random direction equals
the central finite difference of the forward target (1e-6 relative), with
the full workspace (stage outputs kept) and the minimum one (recomputed)
giving the same bits."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_common import rsg

pytestmark = pytest.mark.gpu


def test_cube96_control_gradient_against_central_difference():
    R = rsg()
    cfg = synth.WORKLOADS["cube96_control"]
    n, h, nst, dt, ck = cfg["n"], cfg["h"], cfg["nst"], cfg["dt"], cfg["checkpoint"]
    nsteps = 400
    gg = R.Grid(h, n=n)
    pos = gg.positions()
    wells = synth.gaussian_wells(cfg["seed"], cfg["natoms"], box=cfg["well_box"])
    gh = R.Hamiltonian(gg, V=torch.from_numpy(synth.well_potential(pos, wells)).cuda(), kin=-0.5,
                       dipole_axis=2)
    psi0 = torch.from_numpy(synth.gaussian_packets(cfg["seed"], pos, nst, h)).cuda().t().contiguous()
    coef = torch.from_numpy(synth.laser_coefficients(cfg["seed"], cfg["ncoef"])).cuda()
    assert coef.numel() == 64
    psi = psi0.clone()
    J, store = R.control_forward(gh, psi, dt, nsteps, coef, ck)
    grad, gs = R.control_backward(gh, psi, dt, nsteps, coef, ck, store)
    psi_m = psi0.clone()
    J_m, store_m = R.control_forward(gh, psi_m, dt, nsteps, coef, ck, workspace="min")
    grad_m, _ = R.control_backward(gh, psi_m, dt, nsteps, coef, ck, store_m, workspace="min")
    assert J.item() == J_m.item()
    np.testing.assert_array_equal(grad.cpu().numpy(), grad_m.cpu().numpy())
    d = torch.from_numpy(synth.random_unit(cfg["seed"], cfg["ncoef"])).cuda()
    ad = float((grad * d).sum())
    fd = {}
    for rel in (1e-3, 1e-4):
        eps = rel * float(coef.abs().max())
        jp, _ = R.control_forward(gh, psi0.clone(), dt, nsteps, coef + eps * d, ck, keep_checkpoints=False)
        jm, _ = R.control_forward(gh, psi0.clone(), dt, nsteps, coef - eps * d, ck, keep_checkpoints=False)
        fd[rel] = (jp.item() - jm.item()) / (2 * eps)
    assert abs(ad) > 1e-6
    assert abs(fd[1e-4] - ad) <= 1e-6 * abs(ad), (ad, fd)
    # the difference converges at second order in eps (Richardson check)
    assert abs(fd[1e-4] - ad) <= 0.05 * abs(fd[1e-3] - ad) + 1e-9 * abs(ad)
