"""Pins of the oracle's time stepping, objective, adjoint, sensitivities and
Parareal passes against closed forms, invariants and finite differences.

Pin map (oracle function -> tests):
* h_pri / forward_sequential: uniform closed form (P1), modal closed form (P2),
  1-element objective; Eq. 2.7b, Eq. 2.11, Alg. 1.
* h_adj / adjoint_sequential: all-at-once transpose solve with an autograd
  objective gradient (P5), one-element closed form (P1), finite differences (P6).
* element_term: finite differences with c-SIMP active (P6), one-element
  capacity-term closed form.
* parareal_forward / parareal_adjoint: scalar recurrences on the uniform
  solution (theta correction, G load time, G_adj index m = M(n-1)+1 with the
  T_{m-M} clamp), Fig. 1 index example with a source spike (intermediate slots
  from the uncorrected guess), invariants K = N_tau, exact slices, M = 1,
  N_tau = 1 (P4), mirror symmetry (P7), homogeneity in q (P8).
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from workloads import density_uniform_noise

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- closed forms
def _uniform_T(q, dt, c, n):
    """T_n on a domain without Dirichlet nodes: K 1 = 0 and C 1 is the load
    pattern of a uniform source, so T_n = sum_{j<=n} q_j dt / c."""
    return sum(q(j) for j in range(1, n + 1)) * dt / c


@pytest.mark.parametrize("timevar", [False, True])
def test_uniform_closed_form_sequential(timevar):
    nx, ny, Nt, p = 5, 4, 12, 8
    qf = (lambda j: 0.5 * (1 - j / Nt) * (1 + np.cos(50 * j / Nt))) if timevar else (lambda j: 1.7)
    q = np.array([qf(j) for j in range(Nt + 1)]) if timevar else 1.7
    P = O.Problem(nx=nx, ny=ny, n_steps=Nt, n_slices=3, p=p, q=q, bc="none",
                  c0=1.3, cmin=1.3)
    rho = density_uniform_noise(nx, ny, 7)
    d = O.Discretisation(P, rho)
    S, th = O.forward_sequential(d)
    for n in range(1, Nt + 1):
        assert np.allclose(S[n - 1], _uniform_T(qf, P.dt, 1.3, n), rtol=1e-12, atol=1e-15)
    # Theta from Eq. 2.11: (1/(N_t N_e) sum_j N_n T_j^p)^(1/p)
    tp = sum(P.n_nodes * _uniform_T(qf, P.dt, 1.3, j) ** p for j in range(1, Nt + 1))
    assert th[-1] == pytest.approx((tp / (Nt * P.n_elem)) ** (1 / p), rel=1e-13)


def _scalar_parareal(Nt, Ntau, p, nn, ne, qf, c, iters=1):
    """Parareal on a Dirichlet-free domain as a scalar recurrence.

    K 1 = 0 and C 1 is the pattern of a uniform load, so every propagator maps
    a uniform field to a uniform one: a fine step adds q(t_j) dt / c, the coarse
    step to tau_{n+1} adds q(tau_{n+1}) dtau / c. theta gets N_n T^p/(N N_e)
    per step with N = N_t (fine) or N_tau (coarse). Returns the coarse
    (T, theta) of the last iterate and the modified-Parareal S (intermediate
    slots from F of the uncorrected guess, coarse slots corrected).
    """
    M = Nt // Ntau
    dt, dtau = 1.0 / Nt, 1.0 / Ntau

    def G(T, th, n):
        T = T + qf(M * (n + 1)) * dtau / c
        return T, (th ** p + nn * T ** p / (Ntau * ne)) ** (1 / p)

    def F(T, th, n):
        traj = []
        for j in range(M * n + 1, M * (n + 1) + 1):
            T = T + qf(j) * dt / c
            th = (th ** p + nn * T ** p / (Nt * ne)) ** (1 / p)
            traj.append(T)
        return T, th, traj

    u = [(0.0, 0.0)]
    for n in range(Ntau):
        u.append(G(*u[n], n))
    for _ in range(iters):
        Fs = [F(*u[n], n) for n in range(Ntau)]
        new = [(0.0, 0.0)]
        for n in range(Ntau):
            gn, gk = G(*new[n], n), G(*u[n], n)
            new.append((gn[0] + Fs[n][0] - gk[0], gn[1] + Fs[n][1] - gk[1]))
        u = new
    S = []
    for n in range(Ntau):
        S += Fs[n][2][:-1] + [u[n + 1][0]]
    return [x[0] for x in u], [x[1] for x in u], S


@pytest.mark.parametrize("Nt,Ntau,iters,timevar", [(12, 3, 1, False), (16, 4, 1, True),
                                                   (16, 4, 2, True), (15, 5, 5, False),
                                                   (15, 3, 1, True)])
def test_uniform_parareal_scalar_recurrence(Nt, Ntau, iters, timevar):
    """Pins the primal Parareal bookkeeping: the theta correction (Q9), the
    coarse load time tau_{n+1} and weight 1/N_tau (Q11), and the intermediate
    slots taken from F of the uncorrected guess (Q10)."""
    nx, ny, p, c = 3, 2, 8, 0.9
    if timevar:
        qf = lambda j: 0.5 * (1 - j / Nt) * (1 + np.cos(50 * j / Nt))
        q = np.array([qf(j) for j in range(Nt + 1)])
    else:
        qf = lambda j: 1.1
        q = 1.1
    P = O.Problem(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau, p=p, q=q, bc="none",
                  c0=c, cmin=c)
    d = O.Discretisation(P, density_uniform_noise(nx, ny, 2))
    fw = O.parareal_forward(d, iterations=iters)
    uT, uth, S = _scalar_parareal(Nt, Ntau, p, P.n_nodes, P.n_elem, qf, c, iters=iters)
    assert np.allclose(fw["utheta"], uth, rtol=1e-12, atol=0)
    assert fw["Theta"] == pytest.approx(uth[-1], rel=1e-12)
    for n in range(Ntau + 1):
        assert np.allclose(fw["uT"][n], uT[n], rtol=1e-12, atol=1e-15)
    for j in range(1, Nt + 1):
        assert np.allclose(fw["S"][j - 1], S[j - 1], rtol=1e-12, atol=1e-15)


def _one_element_adjoint(Nt, Ntau, p, q, c, dc, Theta, T):
    """One element, no Dirichlet node: C 1 = c/4 (1,1,1,1) and K 1 = 0, so lambda
    stays uniform: beta_j = beta_{j+1} + 4 dt s_j / c with s_j = Theta^{1-p} T_j^{p-1}.
    The conductivity term of the sensitivity vanishes (K0 1 = 0); the capacity
    term is dc * beta_j * 1^T C0 1 * (T_j - T_{j-1})/dt with 1^T C0 1 = 1."""
    s = lambda j: Theta ** (1 - p) * T(j) ** (p - 1)
    dt, dtau, M = 1.0 / Nt, 1.0 / Ntau, Nt // Ntau
    Tc = lambda j: T(max(j, 0))

    def F(beta, g, n):
        for j in range(M * n, M * (n - 1), -1):
            beta = beta + 4 * dt * s(j) / c
            g = g - dc * beta * (Tc(j) - Tc(j - 1)) / dt / Nt
        return beta, g

    def G(beta, g, n):
        m = M * (n - 1) + 1
        beta = beta + 4 * dtau * s(m) / c
        g = g - dc * beta * (Tc(m) - Tc(m - M)) / dtau / Ntau
        return beta, g

    seq_beta, seq_g = F(0.0, 0.0, 1) if Ntau == 1 else (None, None)
    # sequential over all steps
    beta, g = 0.0, 0.0
    for j in range(Nt, 0, -1):
        beta = beta + 4 * dt * s(j) / c
        g = g - dc * beta * (Tc(j) - Tc(j - 1)) / dt / Nt
    seq = (beta, g)
    # parareal, cold, one iteration
    v = {Ntau: (0.0, 0.0)}
    for n in range(Ntau, 0, -1):
        v[n - 1] = G(*v[n], n)
    new = {Ntau: (0.0, 0.0)}
    for n in range(Ntau, 0, -1):
        gn, gk, fk = G(*new[n], n), G(*v[n], n), F(*v[n], n)
        new[n - 1] = tuple(gn[i] + fk[i] - gk[i] for i in range(2))
    return seq, new


def test_one_element_closed_form():
    """nx = ny = 1, no Dirichlet node, capacity SIMP active (dC/drho != 0)."""
    Nt, Ntau, p, q = 12, 3, 8, 1.0
    P = O.Problem(nx=1, ny=1, n_steps=Nt, n_slices=Ntau, p=p, q=q, bc="none",
                  c0=1.0, cmin=0.5, pc=2.0)
    rho = np.array([0.6])
    d = O.Discretisation(P, rho)
    c = 0.5 + 0.5 * 0.6 ** 2
    dc = 2 * 0.5 * 0.6
    T = lambda j: q * j / Nt / c
    S, th = O.forward_sequential(d)
    Theta = th[-1]
    assert Theta == pytest.approx((sum(4 * T(j) ** p for j in range(1, Nt + 1)) / Nt) ** (1 / p),
                                  rel=1e-13)
    lam, g = O.adjoint_sequential(d, S, Theta)
    seq, par = _one_element_adjoint(Nt, Ntau, p, q, c, dc, Theta, T)
    assert np.allclose(lam[1], seq[0], rtol=1e-12)
    assert g[0] == pytest.approx(seq[1], rel=1e-12)
    # Parareal (cold, one iteration) on the sequential S: pins the G_adj index
    # m = M(n-1)+1 and the clamp T_{m-M} -> T_0 for n = 1.
    ad = O.parareal_adjoint(d, S, Theta, iterations=1)
    for n in range(Ntau + 1):
        assert np.allclose(ad["lam"][n], par[n][0], rtol=1e-12, atol=0)
    assert ad["grad"][0] == pytest.approx(par[0][1], rel=1e-12)


def test_modal_closed_form_one_dirichlet_corner():
    """One element with node 0 held at T = 0 (P2): three free DOFs; with
    generalised eigenpairs K phi = mu C phi, phi^T C phi = 1, backward Euler
    gives T_n = sum_i phi_i (phi_i^T f / mu_i) (1 - (1 + mu_i dt)^-n)."""
    Nt = 9
    P = O.Problem(nx=1, ny=1, n_steps=Nt, n_slices=3, bc=np.array([1, 0, 0, 0], bool),
                  k0=1.0, kmin=1.0, pk=1.0)
    d = O.Discretisation(P, np.array([0.5]))
    Kf = d.restrict(d.K).toarray()
    Cf = d.restrict(d.C).toarray()
    mu, phi = sla.eigh(Kf, Cf)
    f = d.f_unit[d.free]
    S, th = O.forward_sequential(d)
    for n in range(1, Nt + 1):
        Tn = sum(phi[:, i] * (phi[:, i] @ f / mu[i]) * (1 - (1 + mu[i] * P.dt) ** -n)
                 for i in range(3))
        assert np.allclose(S[n - 1][d.free], Tn, rtol=1e-12)
        assert S[n - 1][0] == 0.0
    # adjoint: modal backward recursion with the exact source
    lam, g = O.adjoint_sequential(d, S, th[-1])
    beta = np.zeros(3)
    for n in range(Nt, 0, -1):
        s = th[-1] ** (1 - P.p) * S[n - 1][d.free] ** (P.p - 1)
        beta = (beta / P.dt + phi.T @ s) / (1 / P.dt + mu)
        assert np.allclose(lam[n][d.free], phi @ beta, rtol=1e-11)


# ------------------------------------------------------- adjoint transposition
def test_adjoint_is_transpose_of_all_at_once_system():
    """P5: lambda from the oracle's backward recursion equals M^{-T} N_t (dTheta/dS)^T
    with M the all-at-once block matrix (Eq. 2.8) and dTheta/dS from autograd."""
    torch = pytest.importorskip("torch")
    P = O.Problem(nx=4, ny=3, n_steps=6, n_slices=2, bc="left_centre")
    P.bc = O.dirichlet_mask(4, 3, "left_edge")
    d = O.Discretisation(P, density_uniform_noise(4, 3, 9))
    S, th = O.forward_sequential(d)
    lam, _ = O.adjoint_sequential(d, S, th[-1])
    A = d.restrict(d.C / P.dt + d.K)
    B = -d.restrict(d.C / P.dt)
    nf = A.shape[0]
    Nt = P.n_steps
    blocks = [[None] * Nt for _ in range(Nt)]
    for n in range(Nt):
        blocks[n][n] = A
        if n > 0:
            blocks[n][n - 1] = B
    Mbig = sp.bmat(blocks).tocsc()
    St = torch.tensor(S, requires_grad=True, dtype=torch.float64)
    Theta = ((St ** P.p).sum() / (Nt * P.n_elem)) ** (1.0 / P.p)
    Theta.backward()
    rhs = Nt * St.grad.numpy()[:, d.free].reshape(-1)
    Lam = spla.spsolve(Mbig.T.tocsc(), rhs).reshape(Nt, nf)
    for n in range(1, Nt + 1):
        assert np.allclose(lam[n][d.free], Lam[n - 1], rtol=1e-10, atol=1e-14)
    # and the forward recursion solves M S = Q
    Q = np.concatenate([d.load(n)[d.free] for n in range(1, Nt + 1)])
    Sref = spla.spsolve(Mbig, Q).reshape(Nt, nf)
    assert np.allclose(S[:, d.free], Sref, rtol=1e-11)


# ------------------------------------------------------- finite differences
def _theta_seq(P, rho):
    d = O.Discretisation(P, rho)
    _, th = O.forward_sequential(d)
    return th[-1]


@pytest.mark.parametrize("n,csimp", [(2, False), (3, True), (6, True), (8, False)])
def test_finite_difference_sequential(n, csimp):
    """P6: central differences (h = 1e-6) along seeded unit directions agree
    with grad = g_1 from the adjoint. Round-off in Theta (~1e-16 Theta) divided
    by 2h and the O(h^2) truncation give a relative error far below 1e-6."""
    kw = dict(c0=1.0, cmin=0.5, pc=2.0) if csimp else {}
    P = O.Problem(nx=n, ny=n, n_steps=10, n_slices=2, p=8, **kw)
    rho = density_uniform_noise(n, n, 40 + n)
    d = O.Discretisation(P, rho)
    S, th = O.forward_sequential(d)
    _, grad = O.adjoint_sequential(d, S, th[-1])
    rng = np.random.default_rng(2002 + n)
    h = 1e-6
    for _ in range(4 if n > 4 else 8):
        dvec = rng.standard_normal(P.n_elem)
        dvec /= np.linalg.norm(dvec)
        fd = (_theta_seq(P, rho + h * dvec) - _theta_seq(P, rho - h * dvec)) / (2 * h)
        an = grad @ dvec
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9 * th[-1]


def test_finite_difference_parareal_exact_iterations():
    """With K = N_tau iterations Parareal is exact (P4), so its gradient is the
    derivative of its objective; FD checks the whole Parareal adjoint chain."""
    P = O.Problem(nx=4, ny=6, n_steps=8, n_slices=4, p=8, c0=1.0, cmin=0.5, pc=2.0)
    rho = density_uniform_noise(4, 6, 77)

    def theta(r):
        return O.parareal_forward(O.Discretisation(P, r), iterations=4)["Theta"]

    d = O.Discretisation(P, rho)
    fw, ad = O.one_cycle(d, iterations=4)
    rng = np.random.default_rng(5)
    for _ in range(4):
        dv = rng.standard_normal(P.n_elem)
        dv /= np.linalg.norm(dv)
        fd = (theta(rho + 1e-6 * dv) - theta(rho - 1e-6 * dv)) / 2e-6
        assert abs(fd - ad["grad"] @ dv) <= 1e-6 * abs(ad["grad"] @ dv) + 1e-9


# ------------------------------------------------------- Parareal invariants
def _seq(d):
    S, th = O.forward_sequential(d)
    lam, g = O.adjoint_sequential(d, S, th[-1])
    return S, th, lam, g


@pytest.mark.parametrize("Nt,Ntau", [(12, 4), (16, 8), (10, 5)])
def test_parareal_exact_after_ntau_iterations(Nt, Ntau):
    """P4(i): K = N_tau iterations reproduce the sequential solution (Sec. 4.2)."""
    P = O.Problem(nx=6, ny=6, n_steps=Nt, n_slices=Ntau, c0=1.0, cmin=0.5, pc=2.0)
    d = O.Discretisation(P, density_uniform_noise(6, 6, Nt))
    S, th, lam, g = _seq(d)
    fw, ad = O.one_cycle(d, iterations=Ntau)
    sc = np.abs(S).max()
    assert np.abs(fw["S"] - S).max() < 1e-13 * sc
    assert fw["Theta"] == pytest.approx(th[-1], rel=1e-13)
    assert np.allclose(fw["utheta"], th[::P.M], rtol=1e-13, atol=0)
    for n in range(Ntau + 1):
        ref = lam[P.M * n + 1] if P.M * n + 1 <= Nt else 0 * lam[0]
        assert np.abs(ad["lam"][n] - ref).max() < 1e-12 * np.abs(lam).max()
    assert np.linalg.norm(ad["grad"] - g) < 1e-12 * np.linalg.norm(g)


def test_parareal_exact_slices_after_k_iterations():
    """P4(ii): after k iterations u_n is exact for n <= k, and the stored fine
    states of slices 0..k-1 are exact."""
    P = O.Problem(nx=6, ny=6, n_steps=18, n_slices=6)
    d = O.Discretisation(P, density_uniform_noise(6, 6, 18))
    S, th, lam, g = _seq(d)
    for k in (1, 2, 3):
        fw = O.parareal_forward(d, iterations=k)
        for n in range(k + 1):
            assert np.abs(fw["uT"][n] - (S[P.M * n - 1] if n else 0)).max() < 1e-13
            assert fw["utheta"][n] == pytest.approx(th[P.M * n], rel=1e-13, abs=1e-300)
        assert np.abs(fw["S"][: P.M * k] - S[: P.M * k]).max() < 1e-13
        assert np.abs(fw["uT"][k + 1] - S[P.M * (k + 1) - 1]).max() > 1e-8


@pytest.mark.parametrize("Nt,Ntau", [(6, 6), (7, 1)])
def test_parareal_one_iteration_exact_when_G_is_F(Nt, Ntau):
    """P4(iii) M = 1 (G = F) and P4(iv) N_tau = 1: one iteration is exact."""
    P = O.Problem(nx=4, ny=6, n_steps=Nt, n_slices=Ntau)
    d = O.Discretisation(P, density_uniform_noise(4, 6, 4))
    S, th, lam, g = _seq(d)
    fw, ad = O.one_cycle(d, iterations=1)
    assert np.abs(fw["S"] - S).max() < 1e-13 * np.abs(S).max()
    assert fw["Theta"] == pytest.approx(th[-1], rel=1e-13)
    assert np.linalg.norm(ad["grad"] - g) < 1e-12 * np.linalg.norm(g)


def test_fig1_index_example_with_source_spike():
    """Fig. 1: N_t = 15, N_tau = 3, M = 5. A source only at t_7 (inside slice 1)
    on a Dirichlet-free domain: T_j = dt/c for j >= 7 in the sequential method.
    After one cold iteration the modified Parareal S holds F(u^0_n) at the
    intermediate slots, i.e. the uncorrected guess (Fig. 3 caption): slice 2's
    intermediate states stay 0 while its end point is corrected to dt/c."""
    vals = {}
    with open(os.path.join(GOLDEN, "fig1_index_example.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                vals[k] = [int(x) for x in v]
    Nt, Ntau, M = vals["N_t"][0], vals["N_tau"][0], vals["M"][0]
    q = np.zeros(Nt + 1)
    q[7] = 1.0
    P = O.Problem(nx=2, ny=2, n_steps=Nt, n_slices=Ntau, q=q, bc="none")
    assert P.M == M
    assert [P.M * n for n in range(Ntau + 1)] == vals["coarse_fine_indices"]
    d = O.Discretisation(P, np.full(4, 0.4))
    fw = O.parareal_forward(d, iterations=1)
    v = P.dt
    expect = [0] * 6 + [v] * 4 + [0] * 4 + [v]   # T_1..T_15
    got = [fw["S"][j - 1].mean() for j in range(1, Nt + 1)]
    assert np.allclose(got, expect, atol=1e-15)
    assert np.allclose([fw["uT"][n].mean() for n in range(Ntau + 1)], [0, 0, v, v], atol=1e-15)


# ------------------------------------------------------- symmetry, homogeneity
def test_mirror_symmetry():
    """P7: a design symmetric under y -> 1-y with the symmetric left-centre
    Dirichlet patch gives symmetric T, lambda and grad."""
    nx = ny = 10
    P = O.Problem(nx=nx, ny=ny, n_steps=12, n_slices=4)
    r = density_uniform_noise(nx, ny, 8).reshape(ny, nx)
    r = 0.5 * (r + r[::-1])
    d = O.Discretisation(P, r.reshape(-1))
    fw, ad = O.one_cycle(d, iterations=1)
    S = fw["S"].reshape(P.n_steps, ny + 1, nx + 1)
    assert np.abs(S - S[:, ::-1]).max() < 1e-13 * np.abs(S).max()
    g = ad["grad"].reshape(ny, nx)
    assert np.abs(g - g[::-1]).max() < 1e-12 * np.abs(g).max()


@pytest.mark.parametrize("iters", [1, 2])
def test_homogeneity_in_source(iters):
    """P8: q -> a q scales T, theta, Theta and grad by a and leaves lambda
    unchanged, for every Parareal iterate."""
    a = 3.7
    P1 = O.Problem(nx=6, ny=6, n_steps=12, n_slices=4, q=1.0)
    P2 = O.Problem(nx=6, ny=6, n_steps=12, n_slices=4, q=a)
    rho = density_uniform_noise(6, 6, 12)
    f1, a1 = O.one_cycle(O.Discretisation(P1, rho), iterations=iters)
    f2, a2 = O.one_cycle(O.Discretisation(P2, rho), iterations=iters)
    assert np.allclose(f2["S"], a * f1["S"], rtol=1e-12, atol=1e-15)
    assert f2["Theta"] == pytest.approx(a * f1["Theta"], rel=1e-12)
    assert np.allclose(a2["lam"], a1["lam"], rtol=1e-10, atol=1e-13 * np.abs(a1["lam"]).max())
    assert np.allclose(a2["grad"], a * a1["grad"], rtol=1e-10,
                       atol=1e-12 * np.abs(a1["grad"]).max())


def test_warm_restart_with_exact_guess_is_fixed_point():
    """A guess equal to the sequential solution at the coarse points is a fixed
    point of the correction (F(u) = G-consistent), so one warm iteration
    returns the sequential S, Theta and grad."""
    P = O.Problem(nx=5, ny=6, n_steps=12, n_slices=4)
    d = O.Discretisation(P, density_uniform_noise(5, 6, 21))
    S, th, lam, g = _seq(d)
    gT = np.array([np.zeros(P.n_nodes)] + [S[P.M * n - 1] for n in range(1, 5)])
    gth = th[::P.M]
    gl = np.array([lam[P.M * n + 1] if P.M * n + 1 <= P.n_steps else np.zeros(P.n_nodes)
                   for n in range(5)])
    fw = O.parareal_forward(d, 1, gT, gth)
    ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], 1, gl)
    assert np.abs(fw["S"] - S).max() < 1e-13 * np.abs(S).max()
    assert np.linalg.norm(ad["grad"] - g) < 1e-12 * np.linalg.norm(g)


def test_table1_golden_loads():
    """The paper's material table parses and gives a positive SIMP range."""
    vals = {}
    with open(os.path.join(GOLDEN, "table1_materials.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    k = O.simp(np.array([0.0, 1.0]), vals["k0"], vals["kmin"], vals["pk"])
    c = O.simp(np.array([0.0, 1.0]), vals["c0"], vals["cmin"], vals["pc"])
    assert list(k) == [0.03, 3.0] and list(c) == [0.5, 1.0]


def test_fine_sweeps_through_a_parallel_map_give_identical_results():
    """The fine propagators of a sweep are independent (Sec. 4.2): evaluating
    them through a thread pool, as the slice-parallel CPU baseline does with
    processes, returns the same numbers bit for bit."""
    from concurrent.futures import ThreadPoolExecutor
    P = O.Problem(nx=6, ny=5, n_steps=12, n_slices=4)
    rho = np.random.default_rng(3).uniform(0.2, 0.9, 30)
    d = O.Discretisation(P, rho)
    fw0 = O.parareal_forward(d, 2)
    ad0 = O.parareal_adjoint(d, fw0["S"], fw0["Theta"], 2)
    with ThreadPoolExecutor(3) as ex:
        def fmap(items):
            return list(ex.map(lambda a: O.F_pri(d, a[1], a[2], a[0]), items))

        def amap(items):
            return list(ex.map(lambda a: O.F_adj(d, fw0["S"], fw0["Theta"], a[1], a[2], a[0]),
                               items))
        fw1 = O.parareal_forward(d, 2, fmap=fmap)
        ad1 = O.parareal_adjoint(d, fw1["S"], fw1["Theta"], 2, fmap=amap)
    assert np.array_equal(fw0["S"], fw1["S"]) and fw0["Theta"] == fw1["Theta"]
    assert np.array_equal(ad0["lam"], ad1["lam"]) and np.array_equal(ad0["grad"], ad1["grad"])
