"""Multigrid-preconditioned CG (precond = PT_GMG) against the FP64 oracle.

The preconditioner changes only how each backward-Euler system is solved, not
what is solved, so every output must match the oracle's direct solves at the
FP64 bar (1e-10 at cg_rtol 1e-13). The FP32 inner solve with FP64 refinement
must meet 1e-5, and 1e-6 on Theta. The tests cover:
- the default split (levels above 4096 nodes smoothed by the whole group, the
  rest by one workgroup);
- every level by the group (tuning gmg_tail = 0);
- every level by one workgroup (a large gmg_tail);
- grids that stop coarsening early or do not coarsen at all (odd sides).

Also checked: the multigrid solves need far fewer CG iterations than Jacobi
on the same problem.
"""
import pytest

from tests.gpu_helpers import compare, run_gpu, run_oracle
from workloads import density_gaussians, density_uniform_noise

pytestmark = pytest.mark.gpu


def _cfg(**kw):
    c = dict(nx=64, ny=64, n_steps=64, n_slices=8, pnorm=8, cg_rtol=1e-13, max_iter=20000,
             precond=1)
    c.update(kw)
    return c


def _check(cfg, rho, bar, theta_bar=None):
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho, with_status=True)
    e = compare(g, o)
    print(cfg["nx"], cfg["ny"], e, g["status"], flush=True)
    assert g["status"]["status"] == 0
    assert max(e.values()) <= bar
    if theta_bar is not None:
        assert e["Theta"] <= theta_bar
    return g["status"]


@pytest.mark.parametrize("tail", [None, 0, 100000])
def test_gmg_fp64_64(gpu, tail):
    # every level on the whole group (0), the default split, every level on one workgroup
    cfg = _cfg() if tail is None else dict(_cfg(), tuning=dict(gmg_tail=tail))
    _check(cfg, density_uniform_noise(64, 64, 11), 1e-10)


@pytest.mark.parametrize("nx,ny,Nt,Ntau", [(48, 40, 30, 5), (37, 23, 24, 6), (128, 32, 32, 4)])
def test_gmg_fp64_other_grids(gpu, nx, ny, Nt, Ntau):
    _check(_cfg(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau), density_uniform_noise(nx, ny, nx + ny),
           1e-10)


def test_gmg_fp64_smooth_high_contrast_field(gpu):
    """The large-design density law (Gaussian bumps, k from 1e-3 to 1).

    Here the true FP64 residual of a solve cannot be pushed below about 1.5e-13
    of ||b||: k spans three decades and k dt/h^2 reaches 256. The solves
    therefore stop at 5e-13. The solution error is then at most
    kappa(A) * 5e-13 with kappa(A) <~ 4e3 (1 + 8 k dt/h^2 over the contrast),
    which gives the bar of 2e-9."""
    _check(_cfg(nx=128, ny=128, n_steps=64, n_slices=8, cg_rtol=5e-13),
           density_gaussians(128, 128, 4), 2e-9)


def test_gmg_fp32_refine(gpu):
    _check(_cfg(precision=1, cg_rtol=1e-12), density_uniform_noise(64, 64, 12), 1e-5, 1e-6)


def test_gmg_needs_fewer_iterations_than_jacobi(gpu):
    cfg = _cfg(nx=128, ny=128, n_steps=64, n_slices=8, cg_rtol=1e-10)
    rho = density_gaussians(128, 128, 4)
    gm = run_gpu(cfg, rho, with_status=True)["status"]
    ja = run_gpu(dict(cfg, precond=0), rho, with_status=True)["status"]
    print("gmg", gm, "jacobi", ja, flush=True)
    assert gm["status"] == 0 and ja["status"] == 0
    assert 3 * gm["cg_iters_coarse"] < ja["cg_iters_coarse"]
    assert gm["cg_iters_fine"] < ja["cg_iters_fine"]


def test_gmg_batched(gpu):
    """Multigrid designs inside one multi-design launch."""
    import numpy as np
    import torch

    import oracle as O
    from paper_2411_19030_amd import Problem
    from paper_2411_19030_amd.batched import BatchedCycle
    from tests.gpu_helpers import grad_scale, oracle_problem
    shapes = [(64, 64, 32, 4), (48, 40, 30, 5), (16, 16, 32, 8)]
    probs = [Problem(nx=a, ny=b, n_steps=c, n_slices=d, pnorm=8, cg_rtol=1e-13, max_iter=20000,
                     precond=1) for a, b, c, d in shapes]
    rhos = [density_uniform_noise(a, b, 40 + k) for k, (a, b, _, _) in enumerate(shapes)]
    cyc = BatchedCycle(probs, gpu)
    th, gr = cyc.run([torch.tensor(r, device=gpu) for r in rhos], warm=False)
    torch.cuda.synchronize()
    assert all(s["status"] == 0 for s in cyc.status())
    for k, (a, b, c, d) in enumerate(shapes):
        dd = O.Discretisation(oracle_problem(dict(nx=a, ny=b, n_steps=c, n_slices=d, pnorm=8)),
                              rhos[k])
        fw = O.parareal_forward(dd, 1)
        ad = O.parareal_adjoint(dd, fw["S"], fw["Theta"], 1)
        et = abs(float(th[k]) - fw["Theta"]) / fw["Theta"]
        eg = np.linalg.norm(gr[k].cpu().numpy() - ad["grad"]) / grad_scale(fw["Theta"], ad["grad"])
        print(shapes[k], et, eg, flush=True)
        assert et <= 1e-10 and eg <= 1e-10


@pytest.mark.parametrize("nx,ny", [(64, 64), (48, 40)])
def test_gmg_bitwise_deterministic(gpu, nx, ny):
    """Two runs agree bit for bit (fixed-order reductions; the single-workgroup
    levels drain their stores before each intra-workgroup barrier)."""
    import numpy as np
    cfg = _cfg(nx=nx, ny=ny, n_steps=32, n_slices=4, cg_rtol=1e-10)
    rho = density_uniform_noise(nx, ny, 77)
    a = run_gpu(cfg, rho)
    b = run_gpu(cfg, rho)
    for key in ("Theta", "grad", "lam", "S", "uT"):
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key
