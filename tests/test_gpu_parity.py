"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerance: 1e-10 relative in FP64. The GPU solves each backward-Euler system
by Jacobi-PCG to ||b - A x|| <= rtol ||b||; the solution error is then at most
kappa(A) * rtol relative, with kappa <= ~1e3 for these grids and steps, so the
parity runs use rtol = 1e-13 (error <~ 1e-10) while the oracle solves
directly. Outputs compared element by element: S, the corrected coarse states
and thetas, Theta, lambda at the coarse points, and dTheta/drho.
"""
import numpy as np
import pytest

from tests.gpu_helpers import compare, run_gpu, run_oracle
from workloads import density_uniform_noise, workload

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _cfg(**kw):
    c = dict(nx=32, ny=32, n_steps=64, n_slices=8, pnorm=8, cg_rtol=1e-13, max_iter=20000)
    c.update(kw)
    return c


def _check(errs, tol=TOL):
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    assert not bad, f"parity failures {bad} (all: {errs})"


def test_plain_fp64_32_cold(gpu):
    """The 32x32 workload (64 steps, 8 slices, p = 8), cold start, one iteration."""
    w = workload("plain_fp64_32")
    cfg = _cfg(nx=w["nx"], ny=w["ny"], n_steps=w["n_steps"], n_slices=w["n_slices"])
    rho = density_uniform_noise(w["nx"], w["ny"], w["seed"])
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho, with_status=True)
    print("status", g["status"])
    _check(compare(g, o))


def test_plain_fp64_32_warm(gpu):
    """Warm restart (Alg. 3): guesses from the oracle's cold cycle on a
    perturbed design, fed identically to both sides."""
    w = workload("plain_fp64_32")
    cfg = _cfg(nx=w["nx"], ny=w["ny"], n_steps=w["n_steps"], n_slices=w["n_slices"])
    rho = density_uniform_noise(w["nx"], w["ny"], w["seed"])
    rho_prev = np.clip(rho + 0.02 * density_uniform_noise(w["nx"], w["ny"], 99, 0.0, 1.0), 0, 1)
    prev = run_oracle(cfg, rho_prev)
    guess = (prev["uT"], prev["utheta"], prev["lam"])
    o = run_oracle(cfg, rho, guess)
    g = run_gpu(cfg, rho, guess)
    _check(compare(g, o))


@pytest.mark.parametrize("nx,ny,Nt,Ntau", [(37, 23, 30, 5), (1, 1, 6, 3), (5, 2, 8, 8),
                                           (64, 20, 24, 6)])
def test_ragged_and_degenerate_grids(gpu, nx, ny, Nt, Ntau):
    """Odd node counts (ragged last tile), one element, M = 1, wide grids."""
    cfg = _cfg(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau)
    rho = density_uniform_noise(nx, ny, nx * 100 + ny)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho)
    _check(compare(g, o))


def test_sequential_mode_one_slice(gpu):
    """N_tau = 1: one iteration is the sequential reference method."""
    cfg = _cfg(nx=24, ny=24, n_steps=20, n_slices=1)
    rho = density_uniform_noise(24, 24, 5)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho)
    _check(compare(g, o))


def test_multiple_iterations_reach_sequential(gpu):
    """K = N_tau Parareal iterations reproduce the sequential method (Sec. 4.2)."""
    cfg = _cfg(nx=16, ny=16, n_steps=24, n_slices=4, iterations=4)
    rho = density_uniform_noise(16, 16, 6)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho)
    _check(compare(g, o))


def test_paper_physics_csimp_timevarying_source(gpu):
    """Table 1 materials with the capacity SIMP active, q(t) of Eq. 5.1, the
    bottom-centre Dirichlet patch of Fig. 4, p = 20."""
    Nt = 48
    t = np.arange(Nt + 1) / Nt
    q = 0.5 * (1 - t) * (1 + np.cos(50 * t))
    cfg = _cfg(nx=20, ny=20, n_steps=Nt, n_slices=6, pnorm=20, k0=3.0, kmin=0.03, pk=3.0,
               c0=1.0, cmin=0.5, pc=2.0, q=q, bc="bottom_centre")
    rho = density_uniform_noise(20, 20, 7, base=0.5, amp=0.4)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho)
    _check(compare(g, o))


def test_explicit_mask(gpu):
    """Dirichlet set given as a node mask (whole left edge)."""
    nx = ny = 12
    m = np.zeros((ny + 1) * (nx + 1), dtype=bool)
    m[:: nx + 1] = True
    cfg = _cfg(nx=nx, ny=ny, n_steps=12, n_slices=3, bc=m)
    rho = density_uniform_noise(nx, ny, 8)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho)
    _check(compare(g, o))


def test_no_dirichlet_node(gpu):
    """No Dirichlet node (PT_BC_NONE): C/dt + K stays SPD through its mass
    term, and the body heats up under the uniform source."""
    cfg = _cfg(nx=20, ny=14, n_steps=24, n_slices=6, bc="none")
    rho = density_uniform_noise(20, 14, 12)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho)
    _check(compare(g, o))


def test_queue_order_does_not_change_results(gpu):
    """The shared queue's lag of the batched coarse steps behind the fine lanes
    (gk_lag, warm cycles only: a cold cycle has no batched steps) changes only
    which group takes a lane when. Every group of the queue has one shape, so
    the outputs are bitwise the same, and they match the oracle."""
    cfg = _cfg(nx=40, ny=40, n_steps=48, n_slices=12)
    rho = density_uniform_noise(40, 40, 19)
    cold = run_gpu(cfg, rho)
    guess = (cold["uT"], cold["utheta"], cold["lam"])
    runs = [run_gpu(dict(cfg, tuning=dict(gk_lag=lag)), rho, guess, with_trace=True)
            for lag in (0, 3, 11)]
    order = [[r["kind"] for r in run["trace"] if r["kind"] in ("F_ADJ", "GK_ADJ")]
             for run in runs]
    assert "GK_ADJ" in order[0] and order[0] != order[1] != order[2]
    for r in runs[1:]:
        for k in ("S", "uT", "lam", "grad"):
            assert np.array_equal(r[k], runs[0][k]), k
        assert r["Theta"] == runs[0]["Theta"]
    _check(compare(runs[1], run_oracle(cfg, rho, guess)))


def test_bitwise_deterministic(gpu):
    """Two runs give bitwise-equal outputs (fixed-order reductions, no races)."""
    cfg = _cfg(nx=40, ny=40, n_steps=32, n_slices=8, cg_rtol=1e-10)
    rho = density_uniform_noise(40, 40, 9)
    a = run_gpu(cfg, rho)
    b = run_gpu(cfg, rho)
    for k in ("S", "uT", "lam", "grad"):
        assert np.array_equal(a[k], b[k]), k
    assert a["Theta"] == b["Theta"]
