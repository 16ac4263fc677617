"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

import oracle as O


def oracle_problem(cfg: dict) -> O.Problem:
    kw = {k: cfg[k] for k in ("nx", "ny", "n_steps", "n_slices")}
    for k in ("k0", "kmin", "pk", "c0", "cmin", "pc", "q", "t_final"):
        if k in cfg:
            kw[k] = cfg[k]
    kw["p"] = cfg.get("pnorm", 8)
    kw["bc"] = cfg.get("bc", "left_centre")
    return O.Problem(**kw)


def gpu_problem(cfg: dict):
    from paper_2411_19030_amd import Problem
    kw = {k: cfg[k] for k in ("nx", "ny", "n_steps", "n_slices")}
    for k in ("k0", "kmin", "pk", "c0", "cmin", "pc", "q", "t_final", "pnorm", "iterations",
              "cg_rtol", "max_iter", "bc", "precision", "precond", "storage", "propagator",
              "coarse_iters", "tuning"):
        if k in cfg:
            kw[k] = cfg[k]
    return Problem(**kw)


def run_oracle(cfg: dict, rho: np.ndarray, guess=None):
    """Oracle cycle; guess = (uT, utheta, lam) or None for the cold start."""
    d = O.Discretisation(oracle_problem(cfg), rho)
    it = cfg.get("iterations", 1)
    if cfg.get("propagator", 0) == 1:   # zero coarse propagators (PLT form)
        fw = O.plt_forward(d, it, None if guess is None else guess[0])
        ad = O.plt_adjoint(d, fw["S"], fw["Theta"], it, None if guess is None else guess[2])
        return dict(S=fw["S"], uT=fw["uT"], utheta=fw["utheta"], Theta=fw["Theta"],
                    lam=ad["lam"], grad=ad["grad"])
    nu = cfg.get("coarse_iters", 0)
    Gp = O.make_G_pri(nu) if nu > 0 else None
    Ga = O.make_G_adj(nu) if nu > 0 else None
    if cfg.get("propagator", 0) == 2:   # coarse propagators on the coarse spatial mesh
        Gp, Ga = O.make_G_pri_mesh(d), O.make_G_adj_mesh(d)
    if guess is None:
        fw = O.parareal_forward(d, it, G=Gp)
        ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], it, G=Ga)
    else:
        fw = O.parareal_forward(d, it, guess[0], guess[1], G=Gp)
        ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], it, guess[2], G=Ga)
    return dict(S=fw["S"], uT=fw["uT"], utheta=fw["utheta"], Theta=fw["Theta"],
                lam=ad["lam"], grad=ad["grad"])


def run_gpu(cfg: dict, rho: np.ndarray, guess=None, device="cuda", with_status=False,
            with_trace=False):
    import torch

    from paper_2411_19030_amd.cycle import Cycle
    prob = gpu_problem(cfg)
    cyc = Cycle(prob, device)
    r = torch.tensor(rho, dtype=torch.float64, device=device)
    if guess is None:
        res = cyc.run(r)
    else:
        g = [torch.tensor(np.asarray(x), dtype=torch.float64, device=device) for x in guess]
        res = cyc.run(r, g[0], g[1], g[2])
    torch.cuda.synchronize()
    out = dict(S=res.S.cpu().numpy(), uT=res.uT.cpu().numpy(), utheta=res.utheta.cpu().numpy(),
               Theta=float(res.Theta.cpu()), lam=res.lam.cpu().numpy(),
               grad=res.grad.cpu().numpy())
    if with_status:
        out["status"] = cyc.status()
    if with_trace:
        from paper_2411_19030_amd._pt import pt_query_trace
        out["trace"] = pt_query_trace(prob, cyc.ws)  # lanes of the last (adjoint) launch
    return out


def rel_max(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.abs(b).max()
    if scale == 0:
        return float(np.abs(a).max())
    return float(np.abs(a - b).max() / scale)


def grad_scale(theta: float, grad: np.ndarray) -> float:
    """Norm the gradient error is measured against.

    Each element moves Theta by about Theta/N_e, so a non-degenerate gradient
    has a norm of the order Theta/sqrt(N_e); the workloads here have norms of
    0.5-1 times that scale. Where the gradient vanishes analytically (no
    Dirichlet node: a uniform temperature field, and K0 1 = 0 kills every
    sensitivity term of Eq. 4.7) both sides return round-off of the solves, so
    the floor 1e-2 Theta/sqrt(N_e) turns the test into an absolute one on that
    natural scale."""
    n = float(np.linalg.norm(grad))
    floor = 1e-2 * abs(theta) / np.sqrt(grad.size)
    return max(n, floor)


def _grad_scale(o: dict) -> float:
    return grad_scale(o["Theta"], o["grad"])


def compare(g: dict, o: dict) -> dict:
    """Relative errors: the paper's objective / sensitivity forms (Sec. 5.2)
    plus max-norm relative errors of the stored fields."""
    gs = _grad_scale(o)
    gmax = max(float(np.abs(o["grad"]).max()), gs / np.sqrt(o["grad"].size))
    return dict(
        Theta=abs(g["Theta"] - o["Theta"]) / abs(o["Theta"]),
        grad=float(np.linalg.norm(g["grad"] - o["grad"]) / gs),
        grad_max=float(np.abs(g["grad"] - o["grad"]).max() / gmax),
        S=rel_max(g["S"], o["S"]),
        uT=rel_max(g["uT"], o["uT"]),
        utheta=rel_max(g["utheta"], o["utheta"]),
        lam=rel_max(g["lam"], o["lam"]),
    )
