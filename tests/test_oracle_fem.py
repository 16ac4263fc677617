"""Pins of the oracle's discretisation (Sec. 2.2) against facts fixed by the
mathematics, not by the oracle's own formulas.

* energy identities: u^T K u = sum_e k_e int |grad u_h|^2 and
  u^T C u = sum_e c_e int u_h^2, with u_h written in the monomial basis
  a + b x + c y + d x y and integrated in closed form (pins the element
  matrices and the element-to-node connectivity);
* the load vector integrates the source: sum f = q * area;
* 1-D exactness: with T = 0 on the whole left edge and uniform k, the Q1
  stationary solution is nodally exact for -k T'' = q, T = q/k (x - x^2/2)
  (pins K's x part); the same with the bottom edge pins the y part;
* the steady-state limit of one huge backward-Euler step equals a stationary
  sparse solve (P3);
* Dirichlet index rules on the left / bottom edge centre.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from workloads import density_uniform_noise


def _bilinear_coeffs(vals, x0, y0, hx, hy):
    """Monomial coefficients (a, b, c, d) of the bilinear interpolant of 4
    corner values in the element's local node order."""
    pts = [(x0, y0), (x0 + hx, y0), (x0 + hx, y0 + hy), (x0, y0 + hy)]
    V = np.array([[1, x, y, x * y] for x, y in pts])
    return np.linalg.solve(V, vals)


def _int_grad2(a, b, c, d, x0, y0, hx, hy):
    """int over the rectangle of (b + d y)^2 + (c + d x)^2, in closed form."""
    x1, y1 = x0 + hx, y0 + hy

    def iy(f0, f1, f2):  # int_y0^y1 (f0 + f1 y + f2 y^2) dy
        return f0 * (y1 - y0) + f1 * (y1**2 - y0**2) / 2 + f2 * (y1**3 - y0**3) / 3

    def ix(f0, f1, f2):
        return f0 * (x1 - x0) + f1 * (x1**2 - x0**2) / 2 + f2 * (x1**3 - x0**3) / 3

    return iy(b * b, 2 * b * d, d * d) * hx + ix(c * c, 2 * c * d, d * d) * hy


def _int_sq(a, b, c, d, x0, y0, hx, hy):
    """int over the rectangle of (a + b x + c y + d x y)^2 via tensor 1-D moments."""
    x1, y1 = x0 + hx, y0 + hy
    mx = [(x1 ** (k + 1) - x0 ** (k + 1)) / (k + 1) for k in range(3)]
    my = [(y1 ** (k + 1) - y0 ** (k + 1)) / (k + 1) for k in range(3)]
    # (a + c y) + x (b + d y)
    A = np.array([a, c])
    B = np.array([b, d])
    tot = 0.0
    for px, coef in ((0, np.convolve(A, A)), (1, 2 * np.convolve(A, B)),
                     (2, np.convolve(B, B))):
        tot += mx[px] * sum(coef[k] * my[k] for k in range(len(coef)))
    return tot


@pytest.mark.parametrize("nx,ny", [(1, 1), (3, 2), (4, 5)])
def test_energy_identities(nx, ny):
    rng = np.random.default_rng(11)
    P = O.Problem(nx=nx, ny=ny, n_steps=1, n_slices=1, c0=2.0, cmin=0.5, pc=2.0,
                  bc="none")
    rho = rng.uniform(0.05, 1.0, nx * ny)
    d = O.Discretisation(P, rho)
    u = rng.standard_normal(P.n_nodes)
    hx, hy = 1.0 / nx, 1.0 / ny
    eK = eC = 0.0
    for ey in range(ny):
        for ex in range(nx):
            e = ey * nx + ex
            n0 = ey * (nx + 1) + ex
            ids = [n0, n0 + 1, n0 + nx + 2, n0 + nx + 1]
            x0, y0 = ex * hx, ey * hy
            a, b, c, dd = _bilinear_coeffs(u[ids], x0, y0, hx, hy)
            eK += d.k[e] * _int_grad2(a, b, c, dd, x0, y0, hx, hy)
            eC += d.c[e] * _int_sq(a, b, c, dd, x0, y0, hx, hy)
    assert u @ (d.K @ u) == pytest.approx(eK, rel=1e-12)
    assert u @ (d.C @ u) == pytest.approx(eC, rel=1e-12)
    # symmetric, and K annihilates constants
    assert abs(d.K - d.K.T).max() < 1e-15
    assert abs(d.C - d.C.T).max() < 1e-15
    assert np.abs(d.K @ np.ones(P.n_nodes)).max() < 1e-14
    # load integrates the source over the unit square
    assert d.f_unit.sum() == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("n,edge", [(8, "x"), (12, "x"), (8, "y")])
def test_1d_stationary_exactness(n, edge):
    """Uniform k, T = 0 on a whole edge, insulated elsewhere: nodal values of
    the Q1 solution equal q/k (s - s^2/2), s the distance from that edge."""
    P = O.Problem(nx=n, ny=n + 3, n_steps=1, n_slices=1, k0=2.5, kmin=2.5, pk=1.0)
    nn = P.n_nodes
    mask = np.zeros(nn, dtype=bool)
    for j in range(P.ny + 1):
        for i in range(P.nx + 1):
            if (edge == "x" and i == 0) or (edge == "y" and j == 0):
                mask[j * (P.nx + 1) + i] = True
    P.bc = mask
    d = O.Discretisation(P, np.full(P.n_elem, 0.5))
    A = d.restrict(d.K).tocsc()
    T = np.zeros(nn)
    T[d.free] = spla.spsolve(A, d.f_unit[d.free])
    jj, ii = np.divmod(np.arange(nn), P.nx + 1)
    s = ii / P.nx if edge == "x" else jj / P.ny
    exact = (1.0 / 2.5) * (s - s * s / 2)
    assert np.abs(T - exact).max() < 1e-12


def test_steady_state_limit():
    """One backward-Euler step with a huge dt reaches the stationary solution (P3)."""
    P = O.Problem(nx=10, ny=10, n_steps=1, n_slices=1, t_final=1e12)
    rho = density_uniform_noise(10, 10, 5)
    d = O.Discretisation(P, rho)
    S, _ = O.forward_sequential(d)
    Tst = np.zeros(P.n_nodes)
    Tst[d.free] = spla.spsolve(d.restrict(d.K).tocsc(), d.f_unit[d.free])
    assert np.abs(S[0] - Tst).max() / np.abs(Tst).max() < 1e-9


def test_solver_cross_check():
    """The cached factorisation agrees with a plain sparse solve (P10)."""
    P = O.Problem(nx=9, ny=8, n_steps=4, n_slices=2)
    d = O.Discretisation(P, density_uniform_noise(9, 8, 3))
    rhs = np.random.default_rng(1).standard_normal(P.n_nodes)
    x = d.solve(P.dt, rhs)
    A = d.restrict(d.C / P.dt + d.K).tocsc()
    ref = spla.spsolve(A, rhs[d.free])
    assert np.abs(x[d.free] - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.all(x[~np.isin(np.arange(P.n_nodes), d.free)] == 0)


@pytest.mark.parametrize("ny,expect", [(32, [15, 16, 17]), (256, list(range(116, 141))),
                                       (20, [9, 10, 11]), (100, list(range(45, 56))),
                                       (1, [])])
def test_dirichlet_left_centre(ny, expect):
    """Centre tenth of the left edge: y in [0.45, 0.55], closed interval."""
    m = O.dirichlet_mask(ny, ny, "left_centre")
    js = [j for j in range(ny + 1) if m[j * (ny + 1)]]
    assert js == expect
    assert m.sum() == len(expect)


def test_dirichlet_bottom_centre_paper_mesh():
    """The paper's 100x100 mesh with T = 0 on the bottom over width L/10 (Fig. 4)."""
    m = O.dirichlet_mask(100, 100, "bottom_centre")
    assert list(np.flatnonzero(m)) == list(range(45, 56))
