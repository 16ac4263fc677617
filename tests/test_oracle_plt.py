"""Pins of the oracle's zero-coarse-propagator (PLT) passes, Sec. 7.

Pin map (oracle function -> tests):
* plt_forward: scalar recurrence on the uniform solution of a Dirichlet-free
  domain (cold start u^0 = 0, u^{k+1}_{n+1} = F(u^k_n), Theta~ of Eq. 7.4 and
  the running objective), exactness after N_tau iterations and of slices
  0..k-1 after k iterations (P4(v)), fixed point at the exact guess.
* plt_adjoint / h_adj_tilde / F_adj_tilde: one-element closed form with c-SIMP
  (the source p/N_e T^{p-1} of Eq. 7.5, the slice-boundary T_{j-1} reading,
  the back-transform of Eq. 7.7), exactness after N_tau iterations against
  the sequential adjoint (lambda~ = p Theta^{p-1} lambda), finite differences
  of the N_tau-iteration PLT objective, homogeneity in q (P8).
"""
import numpy as np
import pytest

import oracle as O
from workloads import density_uniform_noise


def _scalar_plt(Nt, Ntau, iters, qf, c, nn, ne, p):
    """PLT on a Dirichlet-free domain, where every state is uniform: a fine step
    adds q(t_j) dt / c. Returns the coarse states u^K, the fine states of the
    last iteration and Theta~."""
    M, dt = Nt // Ntau, 1.0 / Nt
    u = [0.0] * (Ntau + 1)
    traj = None
    for _ in range(iters):
        traj = []
        new = [0.0]
        for n in range(Ntau):
            T = u[n]
            for j in range(M * n + 1, M * (n + 1) + 1):
                T = T + qf(j) * dt / c
                traj.append(T)
            new.append(T)
        u = new
    Th_t = sum(nn * T ** p for T in traj) / (Nt * ne)
    return u, traj, Th_t


@pytest.mark.parametrize("Nt,Ntau,iters", [(12, 3, 1), (16, 4, 2), (15, 5, 5), (12, 4, 6)])
def test_plt_uniform_scalar_recurrence(Nt, Ntau, iters):
    """Cold start from u^0 = 0; slice n restarts from u^k_n. With iters >= N_tau
    the states are the sequential ones."""
    nx, ny, p, c = 3, 2, 8, 0.9
    qf = lambda j: 0.5 * (1 - j / Nt) * (1 + np.cos(50 * j / Nt))
    q = np.array([qf(j) for j in range(Nt + 1)])
    P = O.Problem(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau, p=p, q=q, bc="none", c0=c, cmin=c)
    d = O.Discretisation(P, density_uniform_noise(nx, ny, 3))
    fw = O.plt_forward(d, iterations=iters)
    u, traj, Th_t = _scalar_plt(Nt, Ntau, iters, qf, c, P.n_nodes, P.n_elem, p)
    for j in range(Nt):
        assert np.allclose(fw["S"][j], traj[j], rtol=1e-12, atol=1e-15)
    for n in range(Ntau + 1):
        assert np.allclose(fw["uT"][n], u[n], rtol=1e-12, atol=1e-15)
    assert fw["Theta_tilde"] == pytest.approx(Th_t, rel=1e-12)
    assert fw["Theta"] == pytest.approx(Th_t ** (1 / p), rel=1e-12)
    M = P.M
    run = [sum(P.n_nodes * T ** p for T in traj[:M * n]) / (Nt * P.n_elem) for n in range(Ntau + 1)]
    assert np.allclose(fw["utheta"], np.array(run) ** (1 / p), rtol=1e-12, atol=0)
    if iters == 1 and Ntau > 1:
        # every slice restarted from 0: not the sequential solution
        assert abs(fw["uT"][Ntau].mean() - u[Ntau]) < 1e-15
        seq_end = sum(qf(j) for j in range(1, Nt + 1)) / Nt / c
        assert abs(u[Ntau] - seq_end) > 1e-3 * seq_end


@pytest.mark.parametrize("iters", [1, 2])
def test_plt_one_element_adjoint_closed_form(iters):
    """nx = ny = 1 without Dirichlet nodes and with c-SIMP: lambda~ stays uniform,
    beta_j = beta_{j+1} + 4 dt s_j / c with s_j = p T_j^{p-1} (N_e = 1); the
    conductivity term vanishes (K0 1 = 0) and the capacity term is
    dc beta_j (T_j - T_{j-1}) / dt with T_{j-1} from S, also across a slice
    boundary. grad = Theta^{1-p}/p grad~."""
    Nt, Ntau, p, q = 12, 3, 8, 1.0
    P = O.Problem(nx=1, ny=1, n_steps=Nt, n_slices=Ntau, p=p, q=q, bc="none",
                  c0=1.0, cmin=0.5, pc=2.0)
    d = O.Discretisation(P, np.array([0.6]))
    c = 0.5 + 0.5 * 0.6 ** 2
    dc = 2 * 0.5 * 0.6
    M, dt = P.M, 1.0 / Nt
    fw = O.plt_forward(d, iterations=iters)
    Tj = [0.0] + [fw["S"][j].mean() for j in range(Nt)]   # T_0 .. T_{N_t}
    Theta = fw["Theta"]
    assert Theta == pytest.approx((sum(4 * T ** p for T in Tj[1:]) / Nt) ** (1 / p), rel=1e-13)
    # scalar PLT adjoint
    v = [0.0] * (Ntau + 1)
    gsum = 0.0
    for _ in range(iters):
        new = [0.0] * (Ntau + 1)
        gsum = 0.0
        for n in range(Ntau, 0, -1):
            beta = v[n]
            for j in range(M * n, M * (n - 1), -1):
                beta = beta + 4 * dt * p * Tj[j] ** (p - 1) / c
                gsum -= dc * beta * (Tj[j] - Tj[j - 1]) / dt / Nt
            new[n - 1] = beta
        v = new
    ad = O.plt_adjoint(d, fw["S"], Theta, iterations=iters)
    for n in range(Ntau + 1):
        assert np.allclose(ad["lam"][n], v[n], rtol=1e-12, atol=0)
    assert ad["grad_tilde"][0] == pytest.approx(gsum, rel=1e-12)
    assert ad["grad"][0] == pytest.approx(Theta ** (1 - p) / p * gsum, rel=1e-12)


def _seq(d):
    S, th = O.forward_sequential(d)
    lam, g = O.adjoint_sequential(d, S, th[-1])
    return S, th, lam, g


@pytest.mark.parametrize("Nt,Ntau", [(12, 4), (16, 8), (10, 5), (9, 1)])
def test_plt_exact_after_ntau_iterations(Nt, Ntau):
    """P4(v): with G = 0, N_tau iterations reproduce the sequential solution.
    The adjoint of Theta~ is p Theta^{p-1} times the adjoint of Theta."""
    P = O.Problem(nx=6, ny=5, n_steps=Nt, n_slices=Ntau, c0=1.0, cmin=0.5, pc=2.0)
    d = O.Discretisation(P, density_uniform_noise(6, 5, Nt + Ntau))
    S, th, lam, g = _seq(d)
    fw = O.plt_forward(d, iterations=Ntau)
    ad = O.plt_adjoint(d, fw["S"], fw["Theta"], iterations=Ntau)
    assert np.abs(fw["S"] - S).max() < 1e-13 * np.abs(S).max()
    assert fw["Theta"] == pytest.approx(th[-1], rel=1e-13)
    assert np.allclose(fw["utheta"], th[::P.M], rtol=1e-13, atol=0)
    scale = P.p * th[-1] ** (P.p - 1)
    for n in range(Ntau + 1):
        ref = lam[P.M * n + 1] if P.M * n + 1 <= Nt else 0 * lam[0]
        assert np.abs(ad["lam"][n] - scale * ref).max() < 1e-12 * scale * np.abs(lam).max()
    assert np.linalg.norm(ad["grad"] - g) < 1e-12 * np.linalg.norm(g)


def test_plt_exact_slices_after_k_iterations():
    """P4(v): after k iterations u_n is exact for n <= k and the fine states of
    slices 0..k-1 are exact; slice k is not."""
    P = O.Problem(nx=6, ny=6, n_steps=18, n_slices=6)
    d = O.Discretisation(P, density_uniform_noise(6, 6, 19))
    S, th, lam, g = _seq(d)
    for k in (1, 2, 3):
        fw = O.plt_forward(d, iterations=k)
        for n in range(k + 1):
            assert np.abs(fw["uT"][n] - (S[P.M * n - 1] if n else 0)).max() < 1e-13
        assert np.abs(fw["S"][: P.M * k] - S[: P.M * k]).max() < 1e-13
        assert np.abs(fw["S"][P.M * k: P.M * (k + 1)] - S[P.M * k: P.M * (k + 1)]).max() > 1e-8


def test_plt_exact_guess_is_fixed_point():
    """Guesses equal to the sequential states and adjoint states of Theta~ are
    a fixed point: one warm iteration returns the sequential S, Theta and grad."""
    P = O.Problem(nx=5, ny=6, n_steps=12, n_slices=4, c0=1.0, cmin=0.5, pc=2.0)
    d = O.Discretisation(P, density_uniform_noise(5, 6, 23))
    S, th, lam, g = _seq(d)
    gT = np.array([np.zeros(P.n_nodes)] + [S[P.M * n - 1] for n in range(1, 5)])
    scale = P.p * th[-1] ** (P.p - 1)
    gl = np.array([scale * lam[P.M * n + 1] if P.M * n + 1 <= P.n_steps else np.zeros(P.n_nodes)
                   for n in range(5)])
    fw = O.plt_forward(d, 1, gT)
    ad = O.plt_adjoint(d, fw["S"], fw["Theta"], 1, gl)
    assert np.abs(fw["S"] - S).max() < 1e-13 * np.abs(S).max()
    assert fw["Theta"] == pytest.approx(th[-1], rel=1e-13)
    assert np.linalg.norm(ad["grad"] - g) < 1e-12 * np.linalg.norm(g)


def test_plt_finite_difference_exact_iterations():
    """With N_tau iterations the PLT objective is exact, so its back-transformed
    gradient is the derivative of Theta: central differences (h = 1e-6) along
    seeded unit directions, with c-SIMP active."""
    P = O.Problem(nx=4, ny=5, n_steps=8, n_slices=4, c0=1.0, cmin=0.5, pc=2.0)
    rho = density_uniform_noise(4, 5, 78)

    def theta(r):
        return O.plt_forward(O.Discretisation(P, r), iterations=4)["Theta"]

    d = O.Discretisation(P, rho)
    fw = O.plt_forward(d, iterations=4)
    ad = O.plt_adjoint(d, fw["S"], fw["Theta"], iterations=4)
    rng = np.random.default_rng(6)
    for _ in range(4):
        dv = rng.standard_normal(P.n_elem)
        dv /= np.linalg.norm(dv)
        fd = (theta(rho + 1e-6 * dv) - theta(rho - 1e-6 * dv)) / 2e-6
        assert abs(fd - ad["grad"] @ dv) <= 1e-6 * abs(ad["grad"] @ dv) + 1e-9


@pytest.mark.parametrize("iters", [1, 2])
def test_plt_homogeneity_in_source(iters):
    """P8: q -> a q scales T and Theta by a, lambda~ by a^{p-1} (its source is
    p/N_e T^{p-1}) and grad by a, for every iterate."""
    a = 1.9
    P1 = O.Problem(nx=6, ny=6, n_steps=12, n_slices=4, q=1.0)
    P2 = O.Problem(nx=6, ny=6, n_steps=12, n_slices=4, q=a)
    rho = density_uniform_noise(6, 6, 13)
    out = []
    for P in (P1, P2):
        d = O.Discretisation(P, rho)
        fw = O.plt_forward(d, iterations=iters)
        out.append((fw, O.plt_adjoint(d, fw["S"], fw["Theta"], iterations=iters)))
    (f1, a1), (f2, a2) = out
    p = P1.p
    assert np.allclose(f2["S"], a * f1["S"], rtol=1e-12, atol=1e-15)
    assert f2["Theta"] == pytest.approx(a * f1["Theta"], rel=1e-12)
    assert np.allclose(a2["lam"], a ** (p - 1) * a1["lam"], rtol=1e-10,
                       atol=1e-13 * a ** (p - 1) * np.abs(a1["lam"]).max())
    assert np.allclose(a2["grad"], a * a1["grad"], rtol=1e-10,
                       atol=1e-12 * np.abs(a1["grad"]).max())
