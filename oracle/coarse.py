"""A cheaper coarse propagator (oracle, FP64, CPU): the backward-Euler coarse
step solved inexactly, by a fixed number of Jacobi-preconditioned conjugate
gradient iterations from the step's input state.

TEST INFRASTRUCTURE: used only by tests, the smoke check and the bench's CPU
baseline.

The paper finds the coarse propagators to be the bottleneck of the one-shot
method, and suggests making them cheaper (Sec. 7.3, Sec. 8). Here G_pri and
G_adj keep their definitions (Alg. 1 and Alg. 2 with dtau, coarse load time,
the same objective and sensitivity updates), except that the linear solve
  (C/dtau + K) x = b
becomes nu iterations of PCG with the diagonal of C/dtau + K as preconditioner,
started from x0 = the step's input state (T for G_pri, lambda for G_adj), on
the free nodes. It is a fixed function of the input, so every Parareal
invariant that holds for any G still holds; in particular N_tau iterations
reproduce the sequential method.

PCG in the textbook (Hestenes-Stiefel) form: r = b - A x, z = D^{-1} r, p = z;
then alpha = (r, z) / (p, A p), x += alpha p, r -= alpha A p, z = D^{-1} r,
beta = (r_new, z_new) / (r, z), p = z + beta p. It stops early only if r = 0.
"""
from __future__ import annotations

import numpy as np

from .fem import Discretisation
from .timestepping import pnorm_p


def pcg_fixed(A, b: np.ndarray, x0: np.ndarray, nu: int) -> np.ndarray:
    """nu iterations of Jacobi-preconditioned CG on A x = b from x0."""
    dinv = 1.0 / A.diagonal()
    x = np.array(x0, dtype=np.float64)
    r = b - A @ x
    if not np.any(r):
        return x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    for _ in range(nu):
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        if not np.any(r):
            break
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


def _coarse_solve(d: Discretisation, rhs: np.ndarray, x0: np.ndarray, nu: int) -> np.ndarray:
    P = d.prob
    A = d.restrict(d.C / P.dtau + d.K).tocsr()
    x = np.zeros(P.n_nodes)
    if d.free.size:
        x[d.free] = pcg_fixed(A, rhs[d.free], x0[d.free], nu)
    return x


def make_G_pri(nu: int):
    """G_pri with the truncated solve (load at tau_{n+1}, 1/N_tau in theta)."""
    def G(d: Discretisation, T: np.ndarray, theta: float, n: int):
        P = d.prob
        rhs = d.C @ T / P.dtau + d.load(P.M * (n + 1))
        Tn = _coarse_solve(d, rhs, T, nu)
        th = (theta ** P.p + pnorm_p(Tn, P.p) / (P.n_slices * P.n_elem)) ** (1.0 / P.p)
        return Tn, th
    return G


def make_G_adj(nu: int):
    """G_adj with the truncated solve: from lambda_{Mn+1} to lambda_m,
    m = M(n-1)+1, source and T at m, T_{m-M} in the capacity term (clamped
    to T_0 = 0)."""
    def G(d: Discretisation, S: np.ndarray, Theta: float, lam: np.ndarray, g: np.ndarray,
          n: int):
        P = d.prob
        m = P.M * (n - 1) + 1
        Tm = S[m - 1]
        Tprev = S[m - P.M - 1] if m - P.M >= 1 else np.zeros(P.n_nodes)
        src = Theta ** (1 - P.p) / P.n_elem * Tm ** (P.p - 1)
        rhs = d.C @ lam / P.dtau + src
        lam_n = _coarse_solve(d, rhs, lam, nu)
        g_n = g - d.element_term(lam_n, Tm, Tprev, P.dtau) / P.n_slices
        return lam_n, g_n
    return G
