"""Zero coarse propagators (propagator = PT_PLT, Sec. 7) against the oracle's
PLT passes (oracle/plt.py).

The GPU runs only the fine lanes of each pass, starting from the guesses (or
from zero when cold), and forms Theta~, Theta and the back-transformed
gradient after the lanes. Every output must match the oracle at the FP64 bar
(1e-10 at cg_rtol 1e-13), and at 1e-5 (1e-6 on Theta) with the FP32 inner
solve. Cases: several grids and slice counts including N_tau = 1 and
M = 1, cold and warm starts, K_it = 2 and K_it = N_tau, the paper's own test
case (c-SIMP, time-varying q, bottom-edge Dirichlet patch, p = 20), multigrid,
checkpoints, and FP32 with refinement.
"""
import numpy as np
import pytest

from tests.gpu_helpers import compare, run_gpu, run_oracle
from workloads import density_uniform_noise

pytestmark = pytest.mark.gpu


def _cfg(**kw):
    c = dict(nx=32, ny=32, n_steps=64, n_slices=8, pnorm=8, cg_rtol=1e-13, max_iter=20000,
             propagator=1)
    c.update(kw)
    return c


def _check(cfg, rho, guess=None, bar=1e-10, theta_bar=None):
    o = run_oracle(cfg, rho, guess)
    g = run_gpu(cfg, rho, guess, with_status=True)
    e = compare(g, o)
    print(cfg["nx"], cfg["ny"], cfg["n_steps"], cfg["n_slices"], e, g["status"], flush=True)
    assert g["status"]["status"] == 0
    assert max(e.values()) <= bar
    if theta_bar is not None:
        assert e["Theta"] <= theta_bar
    return o, g


@pytest.mark.parametrize("nx,ny,Nt,Ntau", [(32, 32, 64, 8), (20, 12, 24, 8), (16, 16, 32, 16),
                                           (24, 20, 30, 10), (9, 14, 40, 4), (16, 16, 16, 1),
                                           (12, 12, 6, 6)])
def test_plt_cold_against_oracle(gpu, nx, ny, Nt, Ntau):
    _check(_cfg(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau), density_uniform_noise(nx, ny, nx * ny))


def test_plt_single_lane_on_a_wide_group(gpu):
    """One slice at 256 x 256: the planner spreads the single lane over more
    than 170 workgroups, so a round's partial sums (three per workgroup)
    outnumber the 512 threads that add them and some threads load two. At
    k dt / h^2 of about 4e3, FP64 Jacobi-PCG cannot certify a true residual
    of 1e-13 (one solve ended at 1.1e-13), so the solves run to 1e-12 and the
    bar is 1e-9."""
    cfg = _cfg(nx=256, ny=256, n_steps=16, n_slices=1, cg_rtol=1e-12)
    rho = density_uniform_noise(256, 256, 31)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho, with_status=True, with_trace=True)
    nwg = max(r["nwg"] for r in g["trace"])
    e = compare(g, o)
    print(nwg, e, g["status"], flush=True)
    assert nwg * 3 > 512
    assert g["status"]["status"] == 0
    assert max(e.values()) <= 1e-9


def test_plt_warm_and_two_iterations(gpu):
    """Warm restart from the oracle's cold outputs on a perturbed design, with
    one and with two iterations per pass."""
    cfg = _cfg()
    rho = density_uniform_noise(32, 32, 5)
    cold = run_oracle(cfg, rho)
    rho2 = np.clip(rho + 0.01 * density_uniform_noise(32, 32, 6, 0.0, 1.0), 0, 1)
    guess = (cold["uT"], cold["utheta"], cold["lam"])
    _check(cfg, rho2, guess)
    _check(dict(cfg, iterations=2), rho2, guess)


def test_plt_ntau_iterations_is_sequential(gpu):
    """K_it = N_tau: the PLT passes reproduce the sequential method."""
    import oracle as O
    from tests.gpu_helpers import oracle_problem
    cfg = _cfg(nx=16, ny=12, n_steps=24, n_slices=4, iterations=4)
    rho = density_uniform_noise(16, 12, 9)
    _, g = _check(cfg, rho)
    d = O.Discretisation(oracle_problem(cfg), rho)
    S, th = O.forward_sequential(d)
    _, grad = O.adjoint_sequential(d, S, th[-1])
    assert abs(g["Theta"] - th[-1]) <= 1e-10 * th[-1]
    assert np.linalg.norm(g["grad"] - grad) <= 1e-9 * np.linalg.norm(grad)


def test_plt_paper_test_case(gpu):
    """Sec. 5.1 materials law with c-SIMP (dC/drho != 0), q(t) = (1-t)(1+cos 50t)/2,
    the bottom-edge Dirichlet patch and p = 20, on a reduced grid."""
    Nt = 48
    t = np.arange(Nt + 1) / Nt
    q = 0.5 * (1 - t) * (1 + np.cos(50 * t))
    cfg = _cfg(nx=20, ny=20, n_steps=Nt, n_slices=8, pnorm=20, bc="bottom_centre", q=q,
               k0=1.0, kmin=1e-3, pk=3.0, c0=1.0, cmin=0.3, pc=2.0, iterations=2)
    _check(cfg, density_uniform_noise(20, 20, 31, 0.5, 0.4))


def test_plt_gmg_and_checkpoints(gpu):
    cfg = _cfg(nx=48, ny=40, n_steps=60, n_slices=6, precond=1)
    rho = density_uniform_noise(48, 40, 33)
    _check(cfg, rho)
    o = run_oracle(cfg, rho)
    g = run_gpu(dict(cfg, storage=1), rho, with_status=True)
    assert g["status"]["status"] == 0
    M, Ntau = 10, 6
    ref = dict(o, S=np.concatenate([o["S"][M - 1::M], o["S"][0::M]]))
    e = compare(g, ref)
    print("ckpt", e, flush=True)
    assert max(e.values()) <= 1e-10
    assert g["S"].shape[0] == 2 * Ntau


def test_plt_fp32_refine(gpu):
    _check(_cfg(nx=64, ny=64, precision=1, cg_rtol=1e-12), density_uniform_noise(64, 64, 35),
           bar=1e-5, theta_bar=1e-6)
