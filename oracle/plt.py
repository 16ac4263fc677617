"""One-shot Parareal with zero coarse propagators: the Parallel Local-in-Time
form of Sec. 7 (oracle, FP64, CPU).

TEST INFRASTRUCTURE: used only by tests, the smoke check and the bench's CPU
baseline.

With G_pri = G_adj = 0 (Eq. 7.1) the corrections of Eq. 4.10 and Eq. 4.14
reduce to (Eq. 7.2)
    u^{k+1}_{n+1} = F_pri(u^k_n),      v^{k+1}_{n-1} = F_adj(v^k_n),
with u^{k+1}_0 = 0 and v^{k+1}_{N_tau} = 0. As in the PLT method, u and v hold
only the states T_{Mn} and lambda_{Mn+1}. The objective is the modified one of
Eq. 7.4,
    Theta~ = Theta^p = sum_{j=1}^{N_t} ||T_j||_p^p / (N_t N_e),
evaluated from the fine trajectories after the pass. Its adjoint source is
p/N_e T_j^{o(p-1)} (Eq. 7.5) and its sensitivity sum is that of Eq. 4.16 with
this source. Theta and grad Theta follow from Eq. 7.6-7.7:
    Theta = Theta~^{1/p},      grad Theta = Theta^{1-p}/p grad Theta~.

Cold start: the coarse sweep u^0_{n+1} = G(u^0_n) of Sec. 5.2 gives u^0 = 0
and v^0 = 0 when G = 0.

Reading (the paper does not say): the capacity term of the first fine adjoint
step of slice n takes T_{M(n-1)} from S, i.e. the end state of slice n-1's
fine trajectory, as the Parareal adjoint takes it from the assembled S. It
matters only when c depends on rho; at convergence both choices coincide.
"""
from __future__ import annotations

import numpy as np

from .fem import Discretisation
from .parareal import F_pri
from .timestepping import pnorm_p


def plt_objective(d: Discretisation, S: np.ndarray) -> float:
    """Theta~ of Eq. 7.4 from the fine states T_1..T_{N_t} (rows of S)."""
    P = d.prob
    return sum(pnorm_p(S[j], P.p) for j in range(P.n_steps)) / (P.n_steps * P.n_elem)


def plt_forward(d: Discretisation, iterations: int = 1, guess_T=None):
    """Primal pass with G_pri = 0.

    Returns dict with S (N_t, N_n) = the last iteration's fine trajectories,
    uT (N_tau+1, N_n) = u^{K}, utheta (N_tau+1,) = the running objective
    (sum of the slices' Theta~ parts before tau_n)^{1/p}, Theta_tilde, Theta.
    """
    P = d.prob
    Nt, M = P.n_slices, P.M
    zero = np.zeros(P.n_nodes)
    if guess_T is None:
        uT = [zero] * (Nt + 1)
    else:
        uT = [np.array(g, dtype=np.float64) for g in guess_T]
        uT[0] = zero
    trajs = None
    for _ in range(iterations):
        trajs = []
        new = [zero]
        for n in range(Nt):
            T, _, tr = F_pri(d, uT[n], 0.0, n)
            trajs.append(tr)
            new.append(T)
        uT = new
    S = np.zeros((P.n_steps, P.n_nodes))
    for n in range(Nt):
        for i in range(M):
            S[M * n + i] = trajs[n][i]
    part = [sum(pnorm_p(T, P.p) for T in trajs[n]) / (P.n_steps * P.n_elem) for n in range(Nt)]
    run = np.concatenate([[0.0], np.cumsum(part)])
    Th_t = plt_objective(d, S)
    return dict(S=S, uT=np.array(uT), utheta=run ** (1.0 / P.p), Theta_tilde=Th_t,
                Theta=Th_t ** (1.0 / P.p))


def h_adj_tilde(d: Discretisation, lam_next: np.ndarray, g_next: np.ndarray, T: np.ndarray,
                T_prev: np.ndarray, step: float, n_norm: int):
    """Alg. 2 for Theta~: the source is p/N_e T^{o(p-1)} (Eq. 7.5)."""
    P = d.prob
    src = P.p / P.n_elem * T ** (P.p - 1)
    lam = d.solve(step, d.C @ lam_next / step + src)
    g = g_next - d.element_term(lam, T, T_prev, step) / n_norm
    return lam, g


def F_adj_tilde(d: Discretisation, S: np.ndarray, lam: np.ndarray, n: int):
    """Fine adjoint propagator of slice n for Theta~: j = Mn, ..., M(n-1)+1.
    Returns lambda_{M(n-1)+1} and the slice's sensitivity sum."""
    P = d.prob
    g = np.zeros(P.n_elem)
    for j in range(P.M * n, P.M * (n - 1), -1):
        T_prev = S[j - 2] if j >= 2 else np.zeros(P.n_nodes)
        lam, g = h_adj_tilde(d, lam, g, S[j - 1], T_prev, P.dt, P.n_steps)
    return lam, g


def plt_adjoint(d: Discretisation, S: np.ndarray, Theta: float, iterations: int = 1,
                guess_lambda=None):
    """Adjoint pass with G_adj = 0 for Theta~, then the back-transform.

    Returns dict with lam (N_tau+1, N_n) = v^{K} (lam[n] estimates
    lambda~_{Mn+1} of Theta~, lam[N_tau] = 0), grad_tilde = the sum of the last
    iteration's slice sensitivities, and grad = Theta^{1-p}/p grad_tilde.
    """
    P = d.prob
    Nt = P.n_slices
    zl = np.zeros(P.n_nodes)
    if guess_lambda is None:
        vl = [zl] * (Nt + 1)
    else:
        vl = [np.array(x, dtype=np.float64) for x in guess_lambda]
        vl[Nt] = zl
    gsum = None
    for _ in range(iterations):
        new = [None] * (Nt + 1)
        new[Nt] = zl
        gsum = np.zeros(P.n_elem)
        for n in range(Nt, 0, -1):
            lam, g = F_adj_tilde(d, S, vl[n], n)
            new[n - 1] = lam
            gsum = gsum + g
        vl = new
    grad = Theta ** (1 - P.p) / P.p * gsum
    return dict(lam=np.array(vl), grad_tilde=gsum, grad=grad)
