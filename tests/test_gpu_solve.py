"""Shifted-Hamiltonian solves on the GPU (section "The Sternheimer
formulation of linear-response", eq. (sternheimer)).

- QMR with a different complex shift per orbital and CG with real shifts, on
  a small sphere with wells and projectors, 5 of 6 orbitals in use and
  padding points: the solutions match the dense direct solve of the oracle's
  H, the iterates after a fixed number of iterations match the oracle's
  QMR / CG to 1e-10, the spare orbital and the padding stay untouched.
- An eigenvector right-hand side stops after one iteration with b / (lambda
  + sigma); b = 0 and an exact initial guess stop before the first one.
- On the 5.0e5-point sphere with 16 orbitals the converged solution's true
  residual, recomputed with rsg.hpsi, meets the tolerance.
- Bad arguments are rejected before anything is launched."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from oracle import shifted as sv
from tests.gpu_common import System, rsg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sys_():
    s = System(0.5, R=2.9, potential="wells", natoms=2, nst=5, ld=6, seed=41, rcut=1.2, well_ball=1.0,
               pad=3)
    Hd = oracle.hpsi(s.oh, np.eye(s.og.np, dtype=np.complex128))
    return s, Hd


QSHIFTS = np.array([0.3 + 0.1j, -0.2 + 0.05j, 1.0 + 0.5j, 0.05 + 0.02j, 2.0 - 0.3j])


def _rhs(s, seed):
    rng = np.random.default_rng(seed)
    b = np.zeros((s.og.np, s.ld), dtype=np.complex128)
    b[:, :s.nst] = rng.standard_normal((s.og.np, s.nst)) + 1j * rng.standard_normal((s.og.np, s.nst))
    b[:, s.nst:] = 3.0 - 1.0j  # spare orbital: must stay as x's spare column
    return b


@pytest.mark.parametrize("method", ["qmr", "cg"])
def test_solution_matches_direct_solve(sys_, method):
    R = rsg()
    s, Hd = sys_
    if method == "qmr":
        shifts = QSHIFTS
    else:
        lam0 = np.linalg.eigvalsh(Hd.real)[0]
        shifts = -lam0 + np.array([0.5, 1.0, 2.0, 0.7, 3.0])
    b = _rhs(s, 7)
    x0 = np.zeros_like(b)
    x0[:, s.nst:] = -5.0 + 2.0j
    bg, xg = s.to_gpu(b), s.to_gpu(x0)
    xg, info = R.shifted_solve(s.gh, bg, shifts, x=xg, method=method, tol=1e-12, maxiter=3000,
                               check_every=7, nst=s.nst)
    assert np.all(info["status"] == 0), info
    x = s.from_gpu(xg)
    for n in range(s.nst):
        ref = np.linalg.solve(Hd + shifts[n] * np.eye(s.og.np), b[:, n])
        assert np.linalg.norm(x[:, n] - ref) <= 1e-9 * np.linalg.norm(ref), (method, n)
    assert np.all(info["rel_res"] <= 1e-12)
    np.testing.assert_array_equal(x[:, s.nst:], x0[:, s.nst:])
    assert s.pad_untouched(xg)
    # iteration counts close to the oracle's, which runs the same recurrences.
    # The iterates themselves are compared to rounding in
    # test_iterates_match_oracle; where a 1e-12 tolerance is crossed after a
    # few hundred steps is set by how fast rounding erodes the Lanczos
    # vectors' (bi)orthogonality, which differs between any two evaluation
    # orders (two GPU builds differing only in multiply-add fusion crossed
    # it 15 steps apart on 255).  The check catches a solver that needs
    # markedly more work than the recurrences do, not the rounding.
    _, its, _, st = sv.solve_batch(s.oh, b, shifts, method, tol=1e-12, maxiter=3000, nst=s.nst)
    assert np.all(st == 0)
    assert np.all(np.abs(info["iters"] - its) <= np.maximum(2, 0.15 * its)), (info["iters"], its)


@pytest.mark.parametrize("method", ["qmr", "cg"])
def test_iterates_match_oracle(sys_, method):
    R = rsg()
    s, Hd = sys_
    shifts = QSHIFTS if method == "qmr" else np.array([4.0, 5.0, 6.0, 7.0, 8.0])
    b = _rhs(s, 8)
    for k in (1, 2, 6):
        xg, info = R.shifted_solve(s.gh, s.to_gpu(b), shifts, method=method, tol=0.0, maxiter=k, nst=s.nst)
        assert np.all(info["iters"] == k) and np.all(info["status"] == 1)
        ref, its, _, _ = sv.solve_batch(s.oh, b, shifts, method, tol=0.0, maxiter=k, nst=s.nst)
        x = s.from_gpu(xg)
        for n in range(s.nst):
            e = np.linalg.norm(x[:, n] - ref[:, n]) / np.linalg.norm(ref[:, n])
            assert e <= 1e-10, (method, k, n, e)


def test_eigenvector_and_trivial_starts(sys_):
    R = rsg()
    s, Hd = sys_
    lam, U = np.linalg.eigh(Hd.real)
    b = np.zeros((s.og.np, s.ld), dtype=np.complex128)
    for n in range(s.nst):
        b[:, n] = U[:, 2 * n + 1] * (1.0 + 0.5j * n)
    for method, shifts in (("qmr", QSHIFTS), ("cg", np.full(s.nst, 3.0))):
        xg, info = R.shifted_solve(s.gh, s.to_gpu(b), shifts, method=method, tol=1e-12, maxiter=10,
                                   nst=s.nst)
        assert np.all(info["iters"] == 1) and np.all(info["status"] == 0), (method, info)
        x = s.from_gpu(xg)
        for n in range(s.nst):
            ref = b[:, n] / (lam[2 * n + 1] + shifts[n])
            np.testing.assert_allclose(x[:, n], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # b = 0: nothing to do; x = exact solution: nothing to do
    z = np.zeros((s.og.np, s.ld), dtype=np.complex128)
    xg, info = R.shifted_solve(s.gh, s.to_gpu(z), 1.0 + 0.1j, nst=s.nst)
    assert np.all(info["iters"] == 0) and np.all(info["status"] == 0)
    assert not np.any(s.from_gpu(xg)[:, :s.nst])
    xe = _rhs(s, 9)
    be = np.zeros_like(xe)
    for n in range(s.nst):
        be[:, n] = (Hd + QSHIFTS[n] * np.eye(s.og.np)) @ xe[:, n]
    xg, info = R.shifted_solve(s.gh, s.to_gpu(be), QSHIFTS, x=s.to_gpu(xe), tol=1e-10, nst=s.nst)
    assert np.all(info["iters"] == 0) and np.all(info["status"] == 0)


def test_isotropic_rhs_breaks_down_alone(sys_):
    """One orbital with b^T b = 0 (b = u + i w, u orthogonal to w, equal
    norms): QMR stops it at once with status 2 and leaves its x untouched,
    while the other orbitals converge as before."""
    R = rsg()
    s, Hd = sys_
    b = _rhs(s, 12)
    rng = np.random.default_rng(13)
    u = rng.standard_normal(s.og.np)
    w = rng.standard_normal(s.og.np)
    w -= (w @ u) / (u @ u) * u
    w *= np.linalg.norm(u) / np.linalg.norm(w)
    b[:, 2] = u + 1j * w
    x0 = np.zeros_like(b)
    x0[:, 2] = 0.25 - 0.5j
    xg, info = R.shifted_solve(s.gh, s.to_gpu(b), QSHIFTS, x=s.to_gpu(x0), method="qmr", tol=1e-12,
                               maxiter=3000, nst=s.nst)
    # the guess for orbital 2 leaves r = b - A x0 not isotropic: clear it
    xg2, info2 = R.shifted_solve(s.gh, s.to_gpu(b), QSHIFTS, method="qmr", tol=1e-12, maxiter=3000,
                                 nst=s.nst)
    assert info2["status"][2] == 2 and info2["iters"][2] == 0
    x = s.from_gpu(xg2)
    assert not np.any(x[:, 2])
    for n in (0, 1, 3, 4):
        assert info2["status"][n] == 0
        ref = np.linalg.solve(Hd + QSHIFTS[n] * np.eye(s.og.np), b[:, n])
        assert np.linalg.norm(x[:, n] - ref) <= 1e-9 * np.linalg.norm(ref)
    # with a nonzero guess the start residual is not isotropic and QMR runs
    assert info["status"][2] == 0


def test_large_sphere_true_residual():
    """R = 9.85 bohr, h = 0.2 (5.0e5 points), 16 orbitals, 2 wells with
    projectors; complex shifts -eps + omega + i eta: the converged x gives
    ||b - (H + sigma) x|| <= 10 tol ||b|| recomputed from scratch."""
    R = rsg()
    s = System(0.2, R=9.85, potential="wells", natoms=2, nst=16, seed=43, well_ball=3.0)
    rng = np.random.default_rng(44)
    shifts = -rng.uniform(-0.6, -0.1, 16) + 0.3 + 0.1j
    b = s.to_gpu(s.psi)
    tol = 1e-8
    x, info = R.shifted_solve(s.gh, b, shifts, method="qmr", tol=tol, maxiter=4000)
    assert np.all(info["status"] == 0), info
    hx = R.hpsi(s.gh, x)
    sig = torch.from_numpy(shifts).to("cuda")[:, None]
    r = b - hx - sig * x
    rel = (r.abs().pow(2).sum(1).sqrt() / b.abs().pow(2).sum(1).sqrt()).cpu().numpy()
    assert np.all(rel <= 10 * tol), rel


def test_solve_errors(sys_):
    R = rsg()
    s, Hd = sys_
    b = s.to_gpu(_rhs(s, 10))
    x = torch.zeros_like(b)
    L = R._lib
    need = L.rsg_solve_workspace_bytes(s.gh._h, 1, s.nst, b.shape[1])
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    sh = np.zeros(2 * s.nst)
    sh[1] = 0.1  # a complex shift
    it = np.zeros(s.nst, dtype=np.int32)
    vp = C.c_void_p
    args = lambda m, shp, bb, xx, nst, wsb: L.rsg_shifted_solve(
        s.gh._h, shp.ctypes.data_as(vp), vp(bb.data_ptr()), vp(xx.data_ptr()), nst, b.shape[1], m, 1e-8,
        10, 1, it.ctypes.data_as(vp), None, None, vp(ws.data_ptr()), wsb, None)
    assert args(0, sh, b, x, s.nst, need) == -1       # CG with a complex shift
    assert args(2, sh, b, x, s.nst, need) == -1       # unknown method
    assert args(1, sh, b, b, s.nst, need) == -1       # b and x overlap
    assert args(1, sh, b, x, 0, need) == -2           # no orbital
    assert args(1, sh, b, x, s.nst, need - 4096) == -5  # workspace too small
    bad = sh.copy()
    bad[0] = np.nan
    assert args(1, bad, b, x, s.nst, need) == -1
