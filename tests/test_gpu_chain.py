"""Multi-cycle one-shot chains (Alg. 3) with the design filter in front,
against the same chain run by the oracle.

Each side runs three cycles over a seeded design schedule. It starts from an
exact cycle (N_tau iterations), then runs two one-iteration cycles, each warm
from that side's own previous outputs (u_n, theta_n, lambda_{Mn+1}). Every
cycle passes chi through the filter and projection and returns Theta and
dTheta/dchi. This covers the warm-restart data path across cycles, where a
cycle's guesses are the previous GPU outputs rather than oracle arrays.
Parareal and the PLT form are both covered, and c-SIMP is active.
Bar: 1e-10 at cg_rtol 1e-13.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from tests.gpu_helpers import oracle_problem
from workloads import density_branches, design_schedule

pytestmark = pytest.mark.gpu

NX = NY = 20
CFG = dict(nx=NX, ny=NY, n_steps=24, n_slices=4, pnorm=8, k0=3.0, kmin=0.03, pk=3.0, c0=1.0,
           cmin=0.5, pc=2.0, bc="bottom_centre")
FILTER = (0.1, 8.0, 0.5)


def _oracle_chain(designs, plt):
    out = []
    guess = None
    Ntau = CFG["n_slices"]
    for i, chi in enumerate(designs):
        fil, rho = O.filter_projection(chi, NX, NY, *FILTER)
        d = O.Discretisation(oracle_problem(CFG), rho)
        it = Ntau if i == 0 else 1
        if plt:
            fw = O.plt_forward(d, it, None if guess is None else guess[0])
            ad = O.plt_adjoint(d, fw["S"], fw["Theta"], it, None if guess is None else guess[2])
        elif guess is None:
            fw = O.parareal_forward(d, it)
            ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], it)
        else:
            fw = O.parareal_forward(d, it, guess[0], guess[1])
            ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], it, guess[2])
        guess = (fw["uT"], fw["utheta"], ad["lam"])
        g_chi = O.filter_projection_backward(fil, ad["grad"], NX, NY, *FILTER)
        out.append((fw["Theta"], g_chi))
    return out


@pytest.mark.parametrize("plt", [False, True])
def test_one_shot_chain_against_oracle(gpu, plt):
    import torch

    from paper_2411_19030_amd import Problem
    from paper_2411_19030_amd.autograd import OneShotParareal
    from paper_2411_19030_amd.design import DesignFilter
    designs = design_schedule(NX, NY, 11, 3, start=density_branches(NX, NY, 5))
    ref = _oracle_chain(designs, plt)
    prob = Problem(**CFG, cg_rtol=1e-13, max_iter=20000, propagator=1 if plt else 0)
    flt = DesignFilter(NX, NY, *FILTER)
    exact = OneShotParareal(dataclasses.replace(prob, iterations=CFG["n_slices"]), gpu, warm=True)
    obj = OneShotParareal(prob, gpu, warm=True)
    for i, chi in enumerate(designs):
        x = torch.tensor(chi, device=gpu, requires_grad=True)
        th = (exact if i == 0 else obj)(flt(x))
        th.backward()
        if i == 0:
            obj.guess_T, obj.guess_theta = exact.guess_T, exact.guess_theta
            obj.guess_lambda = exact.guess_lambda
        et = abs(float(th.detach()) - ref[i][0]) / ref[i][0]
        g = x.grad.cpu().numpy()
        eg = float(np.linalg.norm(g - ref[i][1]) / np.linalg.norm(ref[i][1]))
        print("cycle", i, "plt" if plt else "parareal", et, eg, flush=True)
        assert et <= 1e-10 and eg <= 1e-10
