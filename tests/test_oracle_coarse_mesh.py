"""Pins of the oracle's coarse-spatial-mesh propagator (oracle/coarse_mesh.py).

* Factor 1: G_pri^c and G_adj^c are the paper's G_pri and G_adj (load time,
  theta normalisation, source scale, T indices, the clamp, the sensitivity
  increment), to round-off.
* P is the bilinear interpolant: it equals scipy's linear grid interpolation
  at the fine nodes, and R P is the identity.
* For a design constant on the f x f blocks of the coarse elements, the coarse
  matrices are the Galerkin projections P^T K P, P^T C P and P^T f of the fine
  ones (nested Q1 spaces with the same coefficients).
* For any design, the coarse energy of a linear field and the total heat
  capacity equal the fine ones: the coefficients are arithmetic means.
* Dirichlet nodes: the coarse mask is the injected fine mask, and outputs
  vanish at every fine Dirichlet node.
* P^T is the transpose of P (as a matrix, with the fine Dirichlet rows zero).
* A spatially uniform state with uniform capacity and no Dirichlet node
  advances by dtau q(tau_{n+1}) / c in closed form, with the closed-form theta.
* On a smooth problem the coarse steps stay within 1% of the fine-mesh ones
  (a source or theta evaluated on the coarse nodes would miss by 7-17%).
* Parareal with G^c: N_tau iterations give the sequential method (P4), in
  both passes; one iteration differs from the exact-G estimate.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle as O
from workloads import density_uniform_noise


def _disc(nx=8, ny=6, Nt=12, Ntau=4, seed=3, **kw):
    """c-SIMP and a time-varying load, so load times and capacity terms show."""
    t = np.arange(Nt + 1) / Nt
    q = 0.5 * (1 - t) * (1 + np.cos(50 * t)) + 0.1
    kw.setdefault("c0", 1.0)
    kw.setdefault("cmin", 0.5)
    kw.setdefault("pc", 2.0)
    kw.setdefault("bc", "left_edge")
    P = O.Problem(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau, q=q, **kw)
    return O.Discretisation(P, density_uniform_noise(nx, ny, seed))


def _rand_state(d, seed):
    T = np.zeros(d.prob.n_nodes)
    T[d.free] = np.random.default_rng(seed).uniform(0.1, 0.6, d.free.size)
    return T


def test_factor_one_is_the_paper_G():
    d = _disc()
    P = d.prob
    Gp, Ga = O.make_G_pri_mesh(d, 1), O.make_G_adj_mesh(d, 1)
    S, th = O.forward_sequential(d)
    rng = np.random.default_rng(4)
    for n in range(P.n_slices):
        T = _rand_state(d, n)
        a, b = O.G_pri(d, T, 0.3, n), Gp(d, T, 0.3, n)
        assert np.abs(a[0] - b[0]).max() <= 1e-13 * np.abs(a[0]).max()
        assert a[1] == pytest.approx(b[1], rel=1e-14)
    for n in range(1, P.n_slices + 1):
        lam = np.zeros(P.n_nodes)
        lam[d.free] = rng.standard_normal(d.free.size)
        g = rng.standard_normal(P.n_elem)
        a, b = O.G_adj(d, S, th[-1], lam, g, n), Ga(d, S, th[-1], lam, g, n)
        assert np.abs(a[0] - b[0]).max() <= 1e-12 * np.abs(a[0]).max()
        assert np.abs(a[1] - b[1]).max() <= 1e-12 * np.abs(a[1]).max()


@pytest.mark.parametrize("f", [2, 3])
def test_prolongation_is_bilinear_interpolation(f):
    nx, ny = 4 * f, 3 * f
    nxc, nyc = nx // f, ny // f
    Tc = np.random.default_rng(f).standard_normal((nxc + 1) * (nyc + 1))
    interp = RegularGridInterpolator((np.linspace(0, 1, nyc + 1), np.linspace(0, 1, nxc + 1)),
                                     Tc.reshape(nyc + 1, nxc + 1), method="linear")
    yy, xx = np.meshgrid(np.linspace(0, 1, ny + 1), np.linspace(0, 1, nx + 1), indexing="ij")
    ref = interp(np.stack([yy.reshape(-1), xx.reshape(-1)], axis=1))
    got = O.prolong_unmasked(Tc, nx, ny, f)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.array_equal(O.restrict(got, nx, ny, f), Tc)


def test_PT_is_the_transpose_of_P():
    mask = np.zeros(9 * 7, dtype=bool)
    mask[[0, 3, 9, 31]] = True
    d = _disc(nx=8, ny=6, bc=mask)
    cm = O.CoarseMesh(d, 2)
    Pm = np.stack([cm.P(np.eye(cm.n_nodes)[i]) for i in range(cm.n_nodes)], axis=1)
    v = np.random.default_rng(3).standard_normal(d.prob.n_nodes)
    assert np.abs(cm.PT(v) - Pm.T @ v).max() <= 1e-14 * np.abs(v).max()


def _P_matrix(nx, ny, f):
    nc = (nx // f + 1) * (ny // f + 1)
    return np.stack([O.prolong_unmasked(np.eye(nc)[i], nx, ny, f) for i in range(nc)], axis=1)


@pytest.mark.parametrize("f", [2, 3])
def test_coarse_operators_are_galerkin_for_blockwise_designs(f):
    nx, ny = 4 * f, 2 * f
    nxc, nyc = nx // f, ny // f
    blocks = np.random.default_rng(7).uniform(0.05, 1.0, (nyc, nxc))
    rho = np.kron(blocks, np.ones((f, f))).reshape(-1)
    P = O.Problem(nx=nx, ny=ny, n_steps=4, n_slices=2, c0=1.0, cmin=0.4, pc=2.0, bc="none")
    d = O.Discretisation(P, rho)
    cm = O.CoarseMesh(d, f)
    Pm = _P_matrix(nx, ny, f)
    Kg = Pm.T @ d.K.toarray() @ Pm
    Cg = Pm.T @ d.C.toarray() @ Pm
    assert np.abs(cm.K.toarray() - Kg).max() <= 1e-13 * np.abs(Kg).max()
    assert np.abs(cm.C.toarray() - Cg).max() <= 1e-13 * np.abs(Cg).max()
    assert np.abs(cm.f_unit - Pm.T @ d.f_unit).max() <= 1e-15


def test_coefficients_are_arithmetic_means():
    d = _disc(nx=8, ny=6, seed=11)
    P = d.prob
    cm = O.CoarseMesh(d, 2)
    # a linear field is exact on both meshes: energy = sum of k * area * |grad|^2
    for a, b in [(1.0, 0.0), (0.0, 1.0), (0.7, -0.4)]:
        xf = np.array([a * i / P.nx + b * j / P.ny for j in range(P.ny + 1)
                       for i in range(P.nx + 1)])
        xc = cm.R(xf)
        ef, ec = xf @ (d.K @ xf), xc @ (cm.K @ xc)
        assert ec == pytest.approx(ef, rel=1e-13)
    # total heat capacity
    assert cm.C.sum() == pytest.approx(d.C.sum(), rel=1e-13)
    # the load is that of the same uniform source
    assert cm.f_unit.sum() == pytest.approx(1.0, rel=1e-14)


def test_dirichlet_nodes():
    mask = np.zeros(9 * 9, dtype=bool)
    mask[[0, 1, 2, 9, 40, 41, 71]] = True
    d = _disc(nx=8, ny=8, bc=mask)
    cm = O.CoarseMesh(d, 2)
    assert np.array_equal(cm.dmask, O.restrict(mask, 8, 8, 2).astype(bool))
    Gp, Ga = O.make_G_pri_mesh(d), O.make_G_adj_mesh(d)
    T, th = Gp(d, _rand_state(d, 1), 0.2, 1)
    assert np.all(T[mask] == 0.0) and np.all(T[~mask] > 0.0)
    S, ths = O.forward_sequential(d)
    lam, _ = Ga(d, S, ths[-1], _rand_state(d, 2), np.zeros(d.prob.n_elem), 2)
    assert np.all(lam[mask] == 0.0)


@pytest.mark.parametrize("n", [0, 2, 3])
def test_uniform_state_closed_form(n):
    nx, ny, Nt, Ntau = 8, 6, 12, 4
    t = np.arange(Nt + 1) / Nt
    q = 1.0 + np.sin(7 * t)
    P = O.Problem(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau, c0=2.5, cmin=2.5, q=q, bc="none")
    d = O.Discretisation(P, density_uniform_noise(nx, ny, 5))
    u0, th0 = 0.4, 0.3
    T, th = O.make_G_pri_mesh(d)(d, np.full(P.n_nodes, u0), th0, n)
    v = u0 + P.dtau * q[P.M * (n + 1)] / 2.5
    assert np.abs(T - v).max() <= 1e-12
    assert th == pytest.approx(
        (th0 ** P.p + (nx + 1) * (ny + 1) * v ** P.p / (Ntau * nx * ny)) ** (1 / P.p), rel=1e-13)


def test_close_to_the_fine_steps_on_a_smooth_problem():
    nx = ny = 32
    Nt, Ntau = 16, 4
    P = O.Problem(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau, c0=1.0, cmin=1.0, q=1.0,
                  bc="left_edge")
    d = O.Discretisation(P, np.full(nx * ny, 0.6))
    S, th = O.forward_sequential(d)
    Gp, Ga = O.make_G_pri_mesh(d), O.make_G_adj_mesh(d)
    for n in range(1, Ntau):
        T = S[P.M * n - 1]
        a, b = O.G_pri(d, T, th[P.M * n], n), Gp(d, T, th[P.M * n], n)
        assert np.abs(a[0] - b[0]).max() <= 0.01 * np.abs(a[0]).max()
        inc_a, inc_b = a[1] ** P.p - th[P.M * n] ** P.p, b[1] ** P.p - th[P.M * n] ** P.p
        assert inc_b == pytest.approx(inc_a, rel=0.01)
    lam, _ = O.adjoint_sequential(d, S, th[-1])
    for n in range(2, Ntau + 1):
        v = lam[P.M * n + 1]
        a = O.G_adj(d, S, th[-1], v, np.zeros(P.n_elem), n)[0]
        b = Ga(d, S, th[-1], v, np.zeros(P.n_elem), n)[0]
        assert np.abs(a - b).max() <= 0.01 * np.abs(a).max()


@pytest.mark.parametrize("f", [2])
def test_parareal_with_the_coarse_mesh_is_exact_after_ntau_iterations(f):
    d = _disc(nx=8, ny=6, Nt=12, Ntau=4, seed=9)
    P = d.prob
    S, th = O.forward_sequential(d)
    lam, g = O.adjoint_sequential(d, S, th[-1])
    fw = O.parareal_forward(d, P.n_slices, G=O.make_G_pri_mesh(d, f))
    ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], P.n_slices, G=O.make_G_adj_mesh(d, f))
    assert np.abs(fw["S"] - S).max() < 1e-12 * np.abs(S).max()
    assert fw["Theta"] == pytest.approx(th[-1], rel=1e-12)
    assert np.linalg.norm(ad["grad"] - g) < 1e-11 * np.linalg.norm(g)
    f1 = O.parareal_forward(d, 1, G=O.make_G_pri_mesh(d, f))
    f1x = O.parareal_forward(d, 1)
    assert abs(f1["Theta"] - th[-1]) > 1e-9 and abs(f1["Theta"] - f1x["Theta"]) > 1e-9
