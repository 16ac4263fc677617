"""Design filter and projection (pt_filter_projection / _backward, Sec. 2.1)
against the oracle (oracle/design.py), and the front end in the differentiable
chain chi -> rho = P(H chi) -> Theta(rho).

Bar: 1e-13 relative to the field's maximum. Both sides form the same weighted
sums of at most a few thousand terms in FP64; only the summation order differs.
Cases:
- the paper's parameters on its 100 x 100 grid (r = 0.03: three elements);
- rectangular grids and elements, and a radius beyond the grid;
- a radius below one element (the identity filter), no projection (beta = 0);
- eta at 0 and at 1;
- one element;
- a 2048 x 2048 grid at r = 0.005 (ten elements), checked at seeded elements
  against the definition.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

CASES = [(100, 100, 0.03, 32.0, 0.5), (37, 23, 0.1, 8.0, 0.4), (16, 40, 0.2, 32.0, 0.5),
         (12, 9, 3.0, 4.0, 0.5), (20, 20, 0.04, 0.0, 0.5), (30, 10, 0.05, 16.0, 0.0),
         (30, 10, 0.05, 16.0, 1.0), (1, 1, 0.5, 32.0, 0.5)]


def _gpu(nx, ny, r, beta, eta, chi, grad):
    import torch

    from paper_2411_19030_amd import _pt
    f = _pt.make_filter(nx, ny, r, beta, eta)
    c = torch.tensor(chi, device="cuda")
    fil, phys = torch.empty_like(c), torch.empty_like(c)
    _pt.pt_filter_projection(f, c, fil, phys)
    g = torch.tensor(grad, device="cuda")
    work, gc = torch.empty_like(c), torch.empty_like(c)
    _pt.pt_filter_projection_backward(f, fil, g, work, gc)
    torch.cuda.synchronize()
    return fil.cpu().numpy(), phys.cpu().numpy(), gc.cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("nx,ny,r,beta,eta", CASES)
def test_filter_projection_against_oracle(gpu, nx, ny, r, beta, eta):
    rng = np.random.default_rng(nx * 1000 + ny)
    chi = rng.uniform(0.0, 1.0, nx * ny)
    grad = rng.standard_normal(nx * ny)
    fil, phys, gc = _gpu(nx, ny, r, beta, eta, chi, grad)
    o_fil, o_phys = O.filter_projection(chi, nx, ny, r, beta, eta)
    o_gc = O.filter_projection_backward(o_fil, grad, nx, ny, r, beta, eta)
    e = (_rel(fil, o_fil), _rel(phys, o_phys), _rel(gc, o_gc))
    print(nx, ny, r, beta, eta, e, flush=True)
    assert max(e) <= 1e-13


def test_identity_below_one_element(gpu):
    """Only the element itself has a positive weight: chi_fil = (r chi) / r,
    within one rounding of chi."""
    chi = np.random.default_rng(1).uniform(0, 1, 24 * 16)
    fil, phys, _ = _gpu(24, 16, 0.5 / 24, 0.0, 0.5, chi, chi)
    assert np.all(np.abs(fil - chi) <= np.spacing(chi))
    assert np.array_equal(phys, fil)


def test_large_grid_sampled(gpu):
    """2048 x 2048 at r = 0.005: forward at seeded elements from the definition,
    and the backward's adjoint identity <H x, y> = <x, H^T y> with beta = 0."""
    nx = ny = 2048
    r = 0.005
    rng = np.random.default_rng(2048)
    chi = rng.uniform(0.0, 1.0, nx * ny)
    y = rng.standard_normal(nx * ny)
    fil, phys, gc = _gpu(nx, ny, r, 0.0, 0.5, chi, y)
    R = int(np.floor(r * nx))
    di = np.arange(-R, R + 1)
    for e in rng.integers(0, nx * ny, 64):
        j, i = divmod(int(e), nx)
        ii, jj = np.meshgrid(i + di, j + di)
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        d = np.hypot((ii - i) / nx, (jj - j) / ny)
        w = np.where(ok, np.maximum(0.0, r - d), 0.0)
        ref = float((w * chi[np.where(ok, jj * nx + ii, 0)]).sum() / w.sum())
        assert abs(fil[e] - ref) <= 1e-13
    assert phys.tobytes() == fil.tobytes()
    lhs = float(fil @ y)
    rhs = float(chi @ gc)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(nx * ny) * np.abs(y).max()


def test_chain_through_filter_and_objective(gpu):
    """chi -> rho = P(H chi) -> Theta(rho) (one-slice exact mode): the gradient
    of the chain against the oracle's chain rule."""
    import torch

    from paper_2411_19030_amd import Problem
    from paper_2411_19030_amd.autograd import OneShotParareal
    from paper_2411_19030_amd.design import DesignFilter
    from tests.gpu_helpers import oracle_problem
    nx = ny = 24
    cfg = dict(nx=nx, ny=ny, n_steps=24, n_slices=1, pnorm=8)
    r, beta, eta = 0.1, 8.0, 0.5
    chi = np.random.default_rng(7).uniform(0.2, 0.6, nx * ny)
    flt = DesignFilter(nx, ny, r, beta, eta)
    obj = OneShotParareal(Problem(**cfg, cg_rtol=1e-13, max_iter=20000), "cuda", warm=False)
    x = torch.tensor(chi, device="cuda", requires_grad=True)
    theta = obj(flt(x))
    theta.backward()
    o_fil, o_rho = O.filter_projection(chi, nx, ny, r, beta, eta)
    d = O.Discretisation(oracle_problem(cfg), o_rho)
    S, th = O.forward_sequential(d)
    _, g_rho = O.adjoint_sequential(d, S, th[-1])
    g_chi = O.filter_projection_backward(o_fil, g_rho, nx, ny, r, beta, eta)
    et = abs(float(theta.detach()) - th[-1]) / th[-1]
    eg = float(np.linalg.norm(x.grad.cpu().numpy() - g_chi) / np.linalg.norm(g_chi))
    print(et, eg, flush=True)
    assert et <= 1e-10 and eg <= 1e-10
