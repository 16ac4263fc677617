"""Pins of the oracle's cheaper coarse propagator (oracle/coarse.py): the
coarse solve truncated to a fixed number of Jacobi-PCG iterations.

* pcg_fixed: the same iterate as scipy's preconditioned CG run for exactly nu
  iterations (rtol = atol = 0, M = the inverse diagonal).
* make_G_pri / make_G_adj: nu = 0 returns the input state (the start is the
  input); with 40 iterations (converged to round-off on this grid, short of
  the Krylov space's exhaustion) they reproduce the exact G_pri and G_adj
  (load time, source and T indices, the clamp, the sensitivity increment).
* Parareal with the truncated G: N_tau iterations still give the sequential
  method (P4), in both passes.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from workloads import density_uniform_noise


def _disc(nx=7, ny=6, Nt=12, Ntau=4, seed=3, **kw):
    """c-SIMP and a time-varying load, so load times and capacity terms show."""
    t = np.arange(Nt + 1) / Nt
    q = 0.5 * (1 - t) * (1 + np.cos(50 * t)) + 0.1
    P = O.Problem(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau, c0=1.0, cmin=0.5, pc=2.0, q=q, **kw)
    return O.Discretisation(P, density_uniform_noise(nx, ny, seed))


@pytest.mark.parametrize("nu", [1, 3, 8])
def test_pcg_fixed_matches_scipy_cg(nu):
    d = _disc()
    P = d.prob
    A = d.restrict(d.C / P.dtau + d.K).tocsr()
    rng = np.random.default_rng(nu)
    b = rng.standard_normal(A.shape[0])
    x0 = rng.standard_normal(A.shape[0])
    M = sp.diags(1.0 / A.diagonal())
    ref, _ = spla.cg(A, b, x0=x0, rtol=0.0, atol=0.0, maxiter=nu, M=M)
    got = O.pcg_fixed(A, b, x0, nu)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_zero_iterations_return_the_input():
    d = _disc()
    P = d.prob
    T = np.zeros(P.n_nodes)
    T[d.free] = np.random.default_rng(1).uniform(0.1, 0.5, d.free.size)
    Tn, th = O.make_G_pri(0)(d, T, 0.2, 1)
    assert np.array_equal(Tn, T)
    assert th == pytest.approx((0.2 ** P.p + np.sum(T ** P.p) / (P.n_slices * P.n_elem))
                               ** (1 / P.p), rel=1e-14)
    lam = np.zeros(P.n_nodes)
    lam[d.free] = np.random.default_rng(2).standard_normal(d.free.size)
    S, th_s = O.forward_sequential(d)
    ln, _ = O.make_G_adj(0)(d, S, th_s[-1], lam, np.zeros(P.n_elem), 2)
    assert np.array_equal(ln, lam)


def test_many_iterations_give_the_exact_coarse_steps():
    d = _disc()
    P = d.prob
    S, th = O.forward_sequential(d)
    Theta = th[-1]
    rng = np.random.default_rng(5)
    for n in range(P.n_slices):
        T = S[P.M * n - 1] if n else np.zeros(P.n_nodes)
        a = O.G_pri(d, T, th[P.M * n], n)
        b = O.make_G_pri(40)(d, T, th[P.M * n], n)
        assert np.abs(a[0] - b[0]).max() <= 1e-12 * np.abs(a[0]).max()
        assert a[1] == pytest.approx(b[1], rel=1e-12)
    for n in range(1, P.n_slices + 1):
        lam = np.zeros(P.n_nodes)
        lam[d.free] = rng.standard_normal(d.free.size)
        g = rng.standard_normal(P.n_elem)
        a = O.G_adj(d, S, Theta, lam, g, n)
        b = O.make_G_adj(40)(d, S, Theta, lam, g, n)
        assert np.abs(a[0] - b[0]).max() <= 1e-11 * np.abs(a[0]).max()
        assert np.abs(a[1] - b[1]).max() <= 1e-11 * np.abs(a[1]).max()


@pytest.mark.parametrize("nu", [2, 6])
def test_parareal_with_truncated_G_is_exact_after_ntau_iterations(nu):
    d = _disc(Nt=12, Ntau=4, seed=9)
    P = d.prob
    S, th = O.forward_sequential(d)
    lam, g = O.adjoint_sequential(d, S, th[-1])
    fw = O.parareal_forward(d, P.n_slices, G=O.make_G_pri(nu))
    ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], P.n_slices, G=O.make_G_adj(nu))
    assert np.abs(fw["S"] - S).max() < 1e-12 * np.abs(S).max()
    assert fw["Theta"] == pytest.approx(th[-1], rel=1e-12)
    assert np.linalg.norm(ad["grad"] - g) < 1e-11 * np.linalg.norm(g)
    # one iteration is not exact, and differs from the exact-G estimate
    f1 = O.parareal_forward(d, 1, G=O.make_G_pri(nu))
    f1x = O.parareal_forward(d, 1)
    assert abs(f1["Theta"] - th[-1]) > 1e-9 and abs(f1["Theta"] - f1x["Theta"]) > 1e-12
