"""The differentiable objective (torch.autograd.Function over the C ABI).

* parity of Theta and dTheta/drho with the oracle for a cold and a warm
  one-shot cycle (guesses: each side's own previous cycle);
* central finite differences of Theta against the adjoint gradient in the
  exact sequential mode (one slice: one Parareal iteration is the reference
  method, Sec. 4.2), on a small grid and on the 512 x 512, 1024-step workload.

Directions are per-element N(0,1) with h = 1e-6 as the step of every element.
The finite-difference error then has three parts:
- truncation, h^2 d^T H d, ~1e-12;
- round-off of Theta, ~1e-13 Theta / h;
- the CG tolerance, rtol 1e-13.

All three are far below 1e-3 of the directional derivative (~1e-3 here).
Directions of unit 2-norm would shrink the signal by sqrt(N_e) and drown it in
round-off at 262144 elements.
"""
import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import oracle_problem
from workloads import density_uniform_noise, workload

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def test_autograd_matches_oracle_cold_then_warm(gpu):
    torch = _torch()
    from paper_2411_19030_amd import Problem
    from paper_2411_19030_amd.autograd import OneShotParareal
    cfg = dict(nx=32, ny=32, n_steps=64, n_slices=8, pnorm=8)
    prob = Problem(**cfg, cg_rtol=1e-13, max_iter=20000)
    obj = OneShotParareal(prob, gpu, warm=True)
    rho0 = density_uniform_noise(32, 32, 0)
    rho1 = np.clip(rho0 + 0.01 * density_uniform_noise(32, 32, 5, 0.0, 1.0), 0, 1)
    d0 = O.Discretisation(oracle_problem(cfg), rho0)
    f0, a0 = O.one_cycle(d0, 1)
    d1 = O.Discretisation(oracle_problem(cfg), rho1)
    f1 = O.parareal_forward(d1, 1, f0["uT"], f0["utheta"])
    a1 = O.parareal_adjoint(d1, f1["S"], f1["Theta"], 1, a0["lam"])
    for rho, fo, go in ((rho0, f0["Theta"], a0["grad"]), (rho1, f1["Theta"], a1["grad"])):
        r = torch.tensor(rho, dtype=torch.float64, device=gpu, requires_grad=True)
        th = obj(r)
        th.backward()
        assert abs(float(th.detach()) - fo) <= 1e-10 * abs(fo)
        g = r.grad.cpu().numpy()
        assert np.linalg.norm(g - go) <= 1e-10 * np.linalg.norm(go)


def _fd_check(gpu, nx, n_steps, seed, ndir, tol):
    torch = _torch()
    from paper_2411_19030_amd import Problem
    from paper_2411_19030_amd.autograd import OneShotParareal
    from workloads import directions
    prob = Problem(nx=nx, ny=nx, n_steps=n_steps, n_slices=1, pnorm=8, cg_rtol=1e-13,
                   max_iter=50000)
    obj = OneShotParareal(prob, gpu, warm=False)
    rho = torch.tensor(density_uniform_noise(nx, nx, seed), dtype=torch.float64, device=gpu,
                       requires_grad=True)
    th = obj(rho)
    th.backward()
    g = rho.grad.detach()
    dirs = directions(nx * nx, seed + 2000, ndir) * np.sqrt(nx * nx)  # per-element N(0,1)
    h = 1e-6
    worst = 0.0
    for d in dirs:
        dt = torch.tensor(d, dtype=torch.float64, device=gpu)
        fp = obj.objective(rho.detach() + h * dt)
        fm = obj.objective(rho.detach() - h * dt)
        fd = (fp - fm) / (2 * h)
        an = float(torch.dot(g, dt))
        err = abs(fd - an) / abs(an)
        worst = max(worst, err)
        print(f"fd {fd:.12e} adjoint {an:.12e} rel {err:.2e}", flush=True)
        assert err <= tol
    return worst


def test_finite_differences_small_sequential(gpu):
    _fd_check(gpu, nx=12, n_steps=20, seed=31, ndir=8, tol=1e-5)


def test_finite_differences_diff_fp64_512(gpu):
    """The 512 x 512, 1024-step workload, exact sequential mode, 16 directions.
    The worst relative error measured is 6.3e-6; the bar 1e-4 leaves a factor
    of 16 for the solves' residual carried into the difference quotient."""
    w = workload("diff_fp64_512")
    _fd_check(gpu, nx=w["nx"], n_steps=w["n_steps"], seed=w["seed"], ndir=16, tol=1e-4)
