"""Single-step propagators and the sequential reference method (oracle).

TEST INFRASTRUCTURE: used only by tests, the smoke check and the bench's CPU
baseline.

* ``h_pri``: Algorithm 1 -- one backward-Euler step (Eq. 2.7b) followed by the
  cumulative power-mean update theta_n = (theta_{n-1}^p + ||T_n||_p^p/(N N_e))^{1/p}
  (Sec. 4.4). With (step, N) = (dt, N_t) it is the fine step; with
  (dtau, N_tau) it is the coarse propagator G_pri.
* ``h_adj``: Algorithm 2 -- one backward-Euler step of the adjoint terminal
  value problem (Eq. 4.5b with the source of Eq. 4.6) followed by the
  cumulative sensitivity update (Eq. 4.16). With (dtau, N_tau) and indices
  shifted by M it is G_adj.
* ``forward_sequential`` / ``adjoint_sequential``: the reference method of
  Sec. 5.2 (H applied sequentially over all N_t steps), which Alg. 3 also uses
  in its first cycle.
"""
from __future__ import annotations

import numpy as np

from .fem import Discretisation


def pnorm_p(T: np.ndarray, p: int) -> float:
    """||T||_p^p = sum_i T_i^p for even p (Eq. 2.11), over every node."""
    return float(np.sum(T ** p))


def h_pri(d: Discretisation, T_prev: np.ndarray, theta_prev: float, step: float,
          q_index: int, n_norm: int):
    """Algorithm 1: solve C (T - T_prev)/step + K T = q_{q_index}, then update theta."""
    P = d.prob
    T = d.solve(step, d.C @ T_prev / step + d.load(q_index))
    theta = (theta_prev ** P.p + pnorm_p(T, P.p) / (n_norm * P.n_elem)) ** (1.0 / P.p)
    return T, theta


def adjoint_source(d: Discretisation, T: np.ndarray, Theta: float) -> np.ndarray:
    """N_t (dTheta/dT_n)^T = Theta^{1-p}/N_e T_n^{o(p-1)} (Eq. 4.6)."""
    P = d.prob
    return Theta ** (1 - P.p) / P.n_elem * T ** (P.p - 1)


def h_adj(d: Discretisation, lam_next: np.ndarray, g_next: np.ndarray, T: np.ndarray,
          T_prev: np.ndarray, Theta: float, step: float, n_norm: int):
    """Algorithm 2: solve C (lam - lam_next)/step + K lam = source(T), then
    g = g_next - (1/n_norm) lam^T (dC (T - T_prev)/step + dK T)."""
    lam = d.solve(step, d.C @ lam_next / step + adjoint_source(d, T, Theta))
    g = g_next - d.element_term(lam, T, T_prev, step) / n_norm
    return lam, g


def forward_sequential(d: Discretisation):
    """Reference forward method: S (N_t, N_n) holding T_1..T_{N_t}, and theta_0..theta_{N_t}."""
    P = d.prob
    T = np.zeros(P.n_nodes)
    theta = 0.0
    S = np.zeros((P.n_steps, P.n_nodes))
    thetas = [0.0]
    for n in range(1, P.n_steps + 1):
        T, theta = h_pri(d, T, theta, P.dt, n, P.n_steps)
        S[n - 1] = T
        thetas.append(theta)
    return S, np.array(thetas)


def adjoint_sequential(d: Discretisation, S: np.ndarray, Theta: float):
    """Reference adjoint method: returns (lam (N_t+2, N_n) with lam[n] = lambda_n,
    lambda_{N_t+1} = 0 and lam[0] unused, grad = g_1)."""
    P = d.prob
    lam = np.zeros((P.n_steps + 2, P.n_nodes))
    g = np.zeros(P.n_elem)
    for n in range(P.n_steps, 0, -1):
        T = S[n - 1]
        T_prev = S[n - 2] if n >= 2 else np.zeros(P.n_nodes)
        lam[n], g = h_adj(d, lam[n + 1], g, T, T_prev, Theta, P.dt, P.n_steps)
    return lam, g
