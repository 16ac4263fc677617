"""Modified Parareal for the primal problem and time-reversed vanilla Parareal for
the adjoint problem (oracle, FP64, CPU).

TEST INFRASTRUCTURE: used only by tests, the smoke check and the bench's CPU
baseline.

Primal (Sec. 4.2-4.4): u_n = (T_{Mn}, theta_{Mn}), u_0 = 0.
  F_pri(u_n) applies Alg. 1 M times with dt and N_t, keeping every
  intermediate state (the modification of Sec. 4.3).
  G_pri(u_n) is Alg. 1 once with dtau, N_tau and index n-1 replaced by n-M,
  so its load is q at tau_{n+1}.
  Correction (Eq. 4.10): u^{k+1}_{n+1} = G(u^{k+1}_n) + F(u^k_n) - G(u^k_n),
  applied to T and to theta alike.
  The result S keeps the fine intermediate states of the last F sweep (from
  the uncorrected u^k_n) and puts the corrected T at the coarse points;
  Theta = theta-part of u_{N_tau} (Sec. 4.4, steps 1-2).

Adjoint (Sec. 4.4): v_n = (lambda_{Mn+1}, g_{Mn+1}), v_{N_tau} = 0.
  F_adj(v_n) applies Alg. 2 M times (lambda_{Mn} ... lambda_{M(n-1)+1}).
  G_adj(v_n) is Alg. 2 once with dtau, N_tau, and n +- 1 replaced by n +- M:
  starting from lambda_{Mn+1} it produces lambda_m with m = M(n-1)+1, with
  source and T taken at fine index m and T_{m-M} in the capacity term
  (clamped to T_0 = 0 when m - M < 0).
  Reversed correction (Eq. 4.14): v^{k+1}_{n-1} = G(v^{k+1}_n) + F(v^k_n) - G(v^k_n).
  grad Theta = g-part of v_0 (Sec. 4.4, step 4).

Initial guesses: either given arrays (a warm restart, Alg. 3) or the coarse
sweeps u^0_{n+1} = G_pri(u^0_n), v^0_{n-1} = G_adj(v^0_n) (Sec. 5.2). The g part
of an adjoint guess cancels in the correction, so only lambda guesses are taken.
"""
from __future__ import annotations

import numpy as np

from .fem import Discretisation
from .timestepping import h_adj, h_pri


def G_pri(d: Discretisation, T: np.ndarray, theta: float, n: int):
    """Coarse primal propagator from tau_n to tau_{n+1}."""
    P = d.prob
    return h_pri(d, T, theta, P.dtau, P.M * (n + 1), P.n_slices)


def F_pri(d: Discretisation, T: np.ndarray, theta: float, n: int):
    """Fine primal propagator from tau_n to tau_{n+1}; returns (T, theta, traj)
    where traj[i] = T_{Mn+i+1} for i = 0..M-1."""
    P = d.prob
    traj = []
    for i in range(1, P.M + 1):
        T, theta = h_pri(d, T, theta, P.dt, P.M * n + i, P.n_steps)
        traj.append(T)
    return T, theta, traj


def parareal_forward(d: Discretisation, iterations: int = 1, guess_T=None,
                     guess_theta=None, G=None, fmap=None):
    """Modified Parareal for (T, theta).

    G: the coarse propagator (default G_pri; any function of (d, T, theta, n)).
    fmap: evaluates the fine propagators of one sweep, a function of the list
    [(n, T, theta)] returning [F_pri(d, T, theta, n)] in the same order. The
    slices are independent (Sec. 4.2), so a parallel map gives the same
    numbers; by default they run here one after another.
    Returns dict with S (N_t, N_n), uT (N_tau+1, N_n), utheta (N_tau+1,),
    Theta, and the initial guess that was used.
    """
    G_pri_ = G_pri if G is None else G
    P = d.prob
    Nt, M = P.n_slices, P.M
    zero = np.zeros(P.n_nodes)
    if guess_T is None:
        # cold start: coarse sweep from u_0 = 0; G(u^0_n) = u^0_{n+1} is reused
        uT = [zero]
        uth = [0.0]
        for n in range(Nt):
            T, th = G_pri_(d, uT[n], uth[n], n)
            uT.append(T)
            uth.append(th)
        GkT = [uT[n + 1] for n in range(Nt)]
        Gkth = [uth[n + 1] for n in range(Nt)]
    else:
        uT = [np.array(g, dtype=np.float64) for g in guess_T]
        uth = [float(t) for t in guess_theta]
        uT[0] = zero
        uth[0] = 0.0
        GkT = None
        Gkth = None
    guess = (np.array(uT), np.array(uth))
    # the intermediate slots of S take each F sweep's fine states as they are
    # computed; only the last iteration's survive (Sec. 4.3)
    S = np.zeros((P.n_steps, P.n_nodes))
    for _ in range(iterations):
        FT, Fth = [], []
        if fmap is None:
            outs = (F_pri(d, uT[n], uth[n], n) for n in range(Nt))
        else:
            outs = iter(fmap([(n, uT[n], uth[n]) for n in range(Nt)]))
        for n in range(Nt):
            T, th, tr = next(outs)
            FT.append(T)
            Fth.append(th)
            for i in range(1, M):
                S[M * n + i - 1] = tr[i - 1]
            del tr
        if GkT is None:
            GkT, Gkth = [], []
            for n in range(Nt):
                T, th = G_pri_(d, uT[n], uth[n], n)
                GkT.append(T)
                Gkth.append(th)
        newT, newth = [zero], [0.0]
        GnT, Gnth = [], []
        for n in range(Nt):
            gT, gth = G_pri_(d, newT[n], newth[n], n)
            GnT.append(gT)
            Gnth.append(gth)
            newT.append(gT + FT[n] - GkT[n])
            newth.append(gth + Fth[n] - Gkth[n])
        uT, uth = newT, newth
        GkT, Gkth = GnT, Gnth
    for n in range(Nt):
        S[M * (n + 1) - 1] = uT[n + 1]
    return dict(S=S, uT=np.array(uT), utheta=np.array(uth), Theta=uth[Nt],
                guess=guess)


def _T(S: np.ndarray, j: int) -> np.ndarray:
    """T_j from S, with T_j = T_0 = 0 for j <= 0."""
    if j <= 0:
        return np.zeros(S.shape[1])
    return S[j - 1]


def G_adj(d: Discretisation, S: np.ndarray, Theta: float, lam: np.ndarray,
          g: np.ndarray, n: int):
    """Coarse adjoint propagator from v_n (lambda_{Mn+1}) to v_{n-1} (lambda_{M(n-1)+1})."""
    P = d.prob
    m = P.M * (n - 1) + 1
    return h_adj(d, lam, g, _T(S, m), _T(S, m - P.M), Theta, P.dtau, P.n_slices)


def F_adj(d: Discretisation, S: np.ndarray, Theta: float, lam: np.ndarray,
          g: np.ndarray, n: int):
    """Fine adjoint propagator: Alg. 2 for j = Mn, Mn-1, ..., M(n-1)+1."""
    P = d.prob
    for j in range(P.M * n, P.M * (n - 1), -1):
        lam, g = h_adj(d, lam, g, _T(S, j), _T(S, j - 1), Theta, P.dt, P.n_steps)
    return lam, g


def parareal_adjoint(d: Discretisation, S: np.ndarray, Theta: float,
                     iterations: int = 1, guess_lambda=None, G=None, fmap=None):
    """Time-reversed vanilla Parareal for (lambda, g).

    G: the coarse propagator (default G_adj; any function of
    (d, S, Theta, lam, g, n)).
    fmap: evaluates the fine adjoint propagators of one sweep, a function of
    the list [(n, lam, g)] returning [F_adj(d, S, Theta, lam, g, n)] in the
    same order (by default one after another here).
    Returns dict with lam (N_tau+1, N_n) where lam[n] estimates lambda_{Mn+1}
    (lam[N_tau] = 0), grad = g-part of v_0, and the guess that was used.
    """
    G_adj_ = G_adj if G is None else G
    P = d.prob
    Nt = P.n_slices
    zl = np.zeros(P.n_nodes)
    zg = np.zeros(P.n_elem)
    if guess_lambda is None:
        vl = [None] * (Nt + 1)
        vg = [None] * (Nt + 1)
        vl[Nt], vg[Nt] = zl, zg
        for n in range(Nt, 0, -1):
            vl[n - 1], vg[n - 1] = G_adj_(d, S, Theta, vl[n], vg[n], n)
        Gkl = {n: vl[n - 1] for n in range(1, Nt + 1)}
        Gkg = {n: vg[n - 1] for n in range(1, Nt + 1)}
    else:
        vl = [np.array(x, dtype=np.float64) for x in guess_lambda]
        vg = [zg.copy() for _ in range(Nt + 1)]
        vl[Nt] = zl
        Gkl = Gkg = None
    guess = np.array(vl)
    for _ in range(iterations):
        Fl, Fg = {}, {}
        if fmap is None:
            for n in range(1, Nt + 1):
                Fl[n], Fg[n] = F_adj(d, S, Theta, vl[n], vg[n], n)
        else:
            outs = fmap([(n, vl[n], vg[n]) for n in range(1, Nt + 1)])
            for n, (lam, g) in zip(range(1, Nt + 1), outs):
                Fl[n], Fg[n] = lam, g
        if Gkl is None:
            Gkl, Gkg = {}, {}
            for n in range(1, Nt + 1):
                Gkl[n], Gkg[n] = G_adj_(d, S, Theta, vl[n], vg[n], n)
        nl = [None] * (Nt + 1)
        ng = [None] * (Nt + 1)
        nl[Nt], ng[Nt] = zl, zg
        Gnl, Gng = {}, {}
        for n in range(Nt, 0, -1):
            gl, gg = G_adj_(d, S, Theta, nl[n], ng[n], n)
            Gnl[n], Gng[n] = gl, gg
            nl[n - 1] = gl + Fl[n] - Gkl[n]
            ng[n - 1] = gg + Fg[n] - Gkg[n]
        vl, vg = nl, ng
        Gkl, Gkg = Gnl, Gng
    return dict(lam=np.array(vl), grad=vg[0], guess=guess)


def one_cycle(d: Discretisation, iterations: int = 1, guess_T=None, guess_theta=None,
              guess_lambda=None):
    """Steps 1-4 of Sec. 4.4: primal Parareal, Theta, adjoint Parareal, grad."""
    fw = parareal_forward(d, iterations, guess_T, guess_theta)
    ad = parareal_adjoint(d, fw["S"], fw["Theta"], iterations, guess_lambda)
    return fw, ad
