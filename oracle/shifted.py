"""Shifted-Hamiltonian linear solves: plain numpy definitions.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it, and it never imports the GPU library.

Section "The Sternheimer formulation of linear-response", eq.
(sternheimer): each orbital's response solves (H - eps_n +- omega + i eta) x
= b.  Here sigma stands for the whole shift.  The paper uses conjugate
gradients for a real shift and QMR (Freund and Nachtigal 1991) for a complex
one.  H is the oracle's Hamiltonian (``hpsi``) without field: real
symmetric, so A = H + sigma is complex symmetric (A^T = A).

QMR follows the coupled two-term recurrences of Freund and Nachtigal
without look-ahead and without preconditioning, with the left Lanczos
vectors equal to the right ones (possible because A^T = A) and the bilinear
form u^T v.  Per iteration i: v_i = v~_i / rho_i, delta_i = v_i^T v_i; p_i =
v_i - (rho_i delta_i / eps_{i-1}) p_{i-1}; eps_i = p_i^T A p_i; beta_i =
eps_i / delta_i; v~_{i+1} = A p_i - beta_i v_i; rho_{i+1} = ||v~_{i+1}||;
theta_i = rho_{i+1} / (gamma_{i-1} |beta_i|); gamma_i = 1 / sqrt(1 +
theta_i^2); eta_i = -eta_{i-1} rho_i gamma_i^2 / (beta_i gamma_{i-1}^2); d_i
= eta_i p_i + (theta_{i-1} gamma_i)^2 d_{i-1}; s_i = eta_i A p_i + (theta_{i-1}
gamma_i)^2 s_{i-1}; x_i = x_{i-1} + d_i; r_i = r_{i-1} - s_i.  Start: r_0 = b
- A x_0, v~_1 = r_0, gamma_0 = 1, eta_0 = -1, d_0 = s_0 = 0.

CG is the textbook Hermitian method: alpha = r^H r / p^H A p, x += alpha p,
r -= alpha A p, beta = r'^H r' / r^H r, p = r' + beta p.

Both stop when ||r|| <= tol ||b|| (||b|| = 0 counts as 1), at a breakdown
(|v^T v| < 1e-13 for the unit-norm Lanczos vector v, any other divisor of
modulus below 1e-290, or rho_{i+1} = 0 without convergence) or after maxiter
iterations.  Status: 0 converged, 1 iteration limit, 2
breakdown.
"""
from __future__ import annotations

import numpy as np

from . import Ham, hpsi

TINY = 1e-290
DELTA_MIN = 1e-13  # |v^T v| of a unit-norm Lanczos vector below this: breakdown


def apply_shifted(ham: Ham, x: np.ndarray, sigma: complex) -> np.ndarray:
    """(H + sigma) x for one orbital column x [np]."""
    return hpsi(ham, x.reshape(-1, 1))[:, 0] + sigma * x


def qmr(ham: Ham, b: np.ndarray, sigma: complex, x0=None, tol: float = 1e-10, maxiter: int = 1000):
    """QMR for (H + sigma) x = b, one orbital (column vectors [np])."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - apply_shifted(ham, x, sigma)
    bnorm = np.linalg.norm(b)
    target = tol * (bnorm if bnorm > 0 else 1.0)
    rnorm = np.linalg.norm(r)
    if rnorm <= target or maxiter <= 0:
        return x, 0, rnorm / (bnorm if bnorm > 0 else 1.0), 0 if rnorm <= target else 1
    rho = rnorm
    vt = r.copy()
    gamma, eta, theta = 1.0, -1.0 + 0j, 0.0
    eps = None
    p = d = s = None
    it, status = 0, 1
    while it < maxiter:
        v = vt / rho
        delta = v @ v
        if abs(delta) < DELTA_MIN:
            status = 2
            break
        p = v.copy() if p is None else v - (rho * delta / eps) * p
        Ap = apply_shifted(ham, p, sigma)
        eps = p @ Ap
        if abs(eps) < TINY:
            status = 2
            break
        beta = eps / delta
        vt = Ap - beta * v
        rho_next = np.linalg.norm(vt)
        theta_new = rho_next / (gamma * abs(beta))
        gamma_new = 1.0 / np.sqrt(1.0 + theta_new ** 2)
        eta = -eta * rho * gamma_new ** 2 / (beta * gamma ** 2)
        c = (theta * gamma_new) ** 2
        d = eta * p if d is None else eta * p + c * d
        s = eta * Ap if s is None else eta * Ap + c * s
        x = x + d
        r = r - s
        theta, gamma, rho = theta_new, gamma_new, rho_next
        it += 1
        rnorm = np.linalg.norm(r)
        if rnorm <= target:
            status = 0
            break
        if rho <= 0:
            status = 2
            break
    return x, it, rnorm / (bnorm if bnorm > 0 else 1.0), status


def cg(ham: Ham, b: np.ndarray, sigma: float, x0=None, tol: float = 1e-10, maxiter: int = 1000):
    """Conjugate gradients for (H + sigma) x = b with a real shift."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - apply_shifted(ham, x, sigma)
    bnorm = np.linalg.norm(b)
    target = tol * (bnorm if bnorm > 0 else 1.0)
    rr = float(np.vdot(r, r).real)
    if np.sqrt(rr) <= target or maxiter <= 0:
        return x, 0, np.sqrt(rr) / (bnorm if bnorm > 0 else 1.0), 0 if np.sqrt(rr) <= target else 1
    p = r.copy()
    it, status = 0, 1
    while it < maxiter:
        Ap = apply_shifted(ham, p, sigma)
        pap = float(np.vdot(p, Ap).real)
        if abs(pap) < TINY:
            status = 2
            break
        alpha = rr / pap
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(np.vdot(r, r).real)
        it += 1
        if np.sqrt(rr_new) <= target:
            rr = rr_new
            status = 0
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it, np.sqrt(rr) / (bnorm if bnorm > 0 else 1.0), status


def solve_batch(ham: Ham, b: np.ndarray, shifts, method: str = "qmr", x0=None, tol: float = 1e-10,
                maxiter: int = 1000, nst: int | None = None):
    """Column by column over a point-major batch [np, ld]: returns x (spare
    columns copied from x0, or zero), iterations, relative residuals and
    status per orbital."""
    b = np.asarray(b, dtype=np.complex128)
    nst = b.shape[1] if nst is None else nst
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    shifts = np.broadcast_to(np.asarray(shifts, dtype=np.complex128), (nst,))
    its = np.zeros(nst, dtype=np.int64)
    res = np.zeros(nst)
    st = np.zeros(nst, dtype=np.int64)
    for n in range(nst):
        if method == "qmr":
            x[:, n], its[n], res[n], st[n] = qmr(ham, b[:, n], complex(shifts[n]), x[:, n], tol, maxiter)
        else:
            x[:, n], its[n], res[n], st[n] = cg(ham, b[:, n], float(shifts[n].real), x[:, n], tol, maxiter)
    return x, its, res, st
