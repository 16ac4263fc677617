"""Cheaper coarse propagator (coarse_iters = nu > 0): every coarse step is
exactly nu Jacobi-PCG iterations from its input state, against the oracle's
truncated propagators (oracle/coarse.py).

The truncated CG of the engine (single-reduction form) and the oracle's
textbook PCG produce the same iterates up to round-off, so with the fine
solves at cg_rtol 1e-13 every output must agree to 1e-10. Cases: cold and warm
starts, several nu, two iterations per pass (the truncated G of the sweep is
then used again as G(u^k_n)), c-SIMP with a time-varying load, and the
resident and streaming engines. (The multigrid preconditioner is rejected with
truncated coarse solves: the propagator is defined with Jacobi-PCG.)
"""
import numpy as np
import pytest

from tests.gpu_helpers import compare, run_gpu, run_oracle
from workloads import density_uniform_noise

pytestmark = pytest.mark.gpu


def _cfg(**kw):
    c = dict(nx=32, ny=32, n_steps=64, n_slices=8, pnorm=8, cg_rtol=1e-13, max_iter=20000,
             coarse_iters=6)
    c.update(kw)
    return c


def _check(cfg, rho, guess=None):
    o = run_oracle(cfg, rho, guess)
    g = run_gpu(cfg, rho, guess, with_status=True)
    e = compare(g, o)
    print(cfg.get("coarse_iters"), cfg["nx"], cfg["ny"], e, g["status"], flush=True)
    assert g["status"]["status"] == 0
    assert max(e.values()) <= 1e-10
    return o, g


@pytest.mark.parametrize("nu,nx,ny,Nt,Ntau", [(1, 32, 32, 64, 8), (6, 32, 32, 64, 8),
                                              (15, 24, 20, 30, 10), (4, 9, 14, 40, 4)])
def test_truncated_coarse_cold(gpu, nu, nx, ny, Nt, Ntau):
    _check(_cfg(coarse_iters=nu, nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau),
           density_uniform_noise(nx, ny, nx + nu))


def test_truncated_coarse_warm_and_two_iterations(gpu):
    cfg = _cfg()
    rho = density_uniform_noise(32, 32, 5)
    cold = run_oracle(cfg, rho)
    rho2 = np.clip(rho + 0.01 * density_uniform_noise(32, 32, 6, 0.0, 1.0), 0, 1)
    guess = (cold["uT"], cold["utheta"], cold["lam"])
    _check(cfg, rho2, guess)
    _check(dict(cfg, iterations=2), rho2, guess)


def test_truncated_coarse_csimp_timevarying(gpu):
    Nt = 48
    t = np.arange(Nt + 1) / Nt
    q = 0.5 * (1 - t) * (1 + np.cos(50 * t))
    _check(_cfg(nx=20, ny=20, n_steps=Nt, n_slices=8, pnorm=20, bc="bottom_centre", q=q,
                k0=3.0, kmin=0.03, c0=1.0, cmin=0.5, pc=2.0, coarse_iters=8),
           density_uniform_noise(20, 20, 31, 0.5, 0.4))


def test_truncated_coarse_streaming_engine(gpu, monkeypatch):
    monkeypatch.setenv("PT_RESIDENT", "0")
    _check(_cfg(nx=48, ny=40, n_steps=60, n_slices=6, coarse_iters=10),
           density_uniform_noise(48, 40, 33))
