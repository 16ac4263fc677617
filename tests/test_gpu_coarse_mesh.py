"""Coarse propagators on the coarse spatial mesh (propagator PT_COARSE_MESH)
against the oracle's (oracle/coarse_mesh.py), through the C ABI.

Both sides solve the same coarse systems: the oracle directly, the library by
Jacobi PCG to cg_rtol in the engine's coarse-mesh lanes (the batched steps,
the cold sweep and the correction sweep, on groups of workgroups). With
cg_rtol 1e-13 for every solve each output must agree to 1e-10 (relative to the
field's maximum), the bar of the other parity tests. Cases: cold starts on
several grids (ragged tiles, N_tau = 1, an odd-index Dirichlet mask), warm
starts and two iterations (the sweep's outputs then serve as G(u^k_n)),
c-SIMP with the paper's time-varying load and p = 20, sweep groups of one and
of many workgroups, bitwise reproducibility, the status counters, N_tau
iterations giving the sequential method, and the full 256 x 256 workload in
the launch configuration the benchmark times (cold and warm cycles at its own
cg_rtol 1e-10, bar 1e-8 as in the other full-size tests).
"""
import numpy as np
import pytest

from tests.gpu_helpers import compare, run_gpu, run_oracle
from workloads import density_uniform_noise, workload, workload_density

pytestmark = pytest.mark.gpu

CM = 2  # PT_COARSE_MESH


def _cfg(**kw):
    c = dict(nx=32, ny=32, n_steps=64, n_slices=8, pnorm=8, cg_rtol=1e-13, max_iter=20000,
             propagator=CM)
    c.update(kw)
    return c


def _check(cfg, rho, guess=None, bar=1e-10):
    print("case", {k: v for k, v in cfg.items() if k != "q"}, flush=True)
    o = run_oracle(cfg, rho, guess)
    g = run_gpu(cfg, rho, guess, with_status=True)
    e = compare(g, o)
    print(e, g["status"], flush=True)
    assert g["status"]["status"] == 0
    assert max(e.values()) <= bar
    return o, g


@pytest.mark.parametrize("nx,ny,Nt,Ntau", [(32, 32, 64, 8), (24, 20, 30, 10), (10, 14, 40, 4),
                                           (40, 6, 24, 3), (20, 20, 16, 1)])
def test_coarse_mesh_cold(gpu, nx, ny, Nt, Ntau):
    _check(_cfg(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau), density_uniform_noise(nx, ny, nx + ny))


def test_coarse_mesh_warm_and_two_iterations(gpu):
    cfg = _cfg()
    rho = density_uniform_noise(32, 32, 5)
    cold = run_oracle(cfg, rho)
    rho2 = np.clip(rho + 0.01 * density_uniform_noise(32, 32, 6, 0.0, 1.0), 0, 1)
    guess = (cold["uT"], cold["utheta"], cold["lam"])
    _check(cfg, rho2, guess)
    _check(dict(cfg, iterations=2), rho2, guess)
    _check(dict(cfg, iterations=3), rho2)


def test_coarse_mesh_paper_settings(gpu):
    Nt = 48
    t = np.arange(Nt + 1) / Nt
    q = 0.5 * (1 - t) * (1 + np.cos(50 * t))
    _check(_cfg(nx=20, ny=20, n_steps=Nt, n_slices=8, pnorm=20, bc="bottom_centre", q=q,
                k0=3.0, kmin=0.03, c0=1.0, cmin=0.5, pc=2.0),
           density_uniform_noise(20, 20, 31, 0.5, 0.4))


def test_coarse_mesh_caller_mask(gpu):
    nx, ny = 16, 12
    mask = np.zeros((nx + 1) * (ny + 1), dtype=bool)
    # fine Dirichlet nodes on and off the coarse nodes, interior and boundary
    mask[[0, 1, 2, 3, 17, 35, 100, 101, 117, 220]] = True
    _check(_cfg(nx=nx, ny=ny, n_steps=24, n_slices=6, bc=mask),
           density_uniform_noise(nx, ny, 8))


def test_coarse_mesh_reproducible_and_counted(gpu):
    cfg = _cfg(nx=24, ny=24, n_steps=32, n_slices=8)
    rho = density_uniform_noise(24, 24, 12)
    a = run_gpu(cfg, rho, with_status=True)
    b = run_gpu(cfg, rho, with_status=True)
    for k in ("S", "uT", "utheta", "lam", "grad"):
        assert np.array_equal(a[k], b[k]), k
    assert a["Theta"] == b["Theta"]
    st = a["status"]
    print(st, flush=True)
    # the adjoint call's counters: cold sweep (N_tau steps) + correction sweep (N_tau - 1)
    assert st["solves_coarse"] == 8 + 7
    assert st["solves_fine"] == 32
    assert st["max_rel_residual"] <= 1e-13


def test_coarse_mesh_ntau_iterations_is_sequential(gpu):
    cfg = _cfg(nx=24, ny=16, n_steps=24, n_slices=6)
    rho = density_uniform_noise(24, 16, 3)
    seq = run_gpu(dict(cfg, n_slices=1, propagator=0), rho)
    g = run_gpu(dict(cfg, iterations=6), rho)
    assert abs(g["Theta"] - seq["Theta"]) <= 1e-11 * seq["Theta"]
    assert np.abs(g["S"] - seq["S"]).max() <= 1e-10 * np.abs(seq["S"]).max()
    assert np.linalg.norm(g["grad"] - seq["grad"]) <= 1e-9 * np.linalg.norm(seq["grad"])


def test_coarse_mesh_full_size_256(gpu):
    w = workload("plain_fp64_256")
    cfg = dict(nx=w["nx"], ny=w["ny"], n_steps=w["n_steps"], n_slices=w["n_slices"],
               pnorm=w["p"], max_iter=20000, propagator=CM, cg_rtol=1e-10)
    rho = workload_density("plain_fp64_256")
    cold, _ = _check(cfg, rho, bar=1e-8)
    rho2 = np.clip(rho + 0.005 * np.cos(np.arange(rho.size) * 0.37), 0, 1)
    _check(cfg, rho2, (cold["uT"], cold["utheta"], cold["lam"]), bar=1e-8)


@pytest.mark.parametrize("wgs", [1, 7, 64])
def test_coarse_mesh_sweep_group_sizes(gpu, wgs):
    # the coarse-mesh sweep lanes (cold and correction) on one workgroup, on a
    # ragged split of the 143 coarse nodes, and on the most workgroups the
    # planner gives a group of this grid (tiles of a few coarse nodes)
    cfg = _cfg(nx=24, ny=20, n_steps=30, n_slices=10, tuning=dict(cm_sweep_wgs=wgs))
    rho = density_uniform_noise(24, 20, 44)
    _check(cfg, rho)
    _check(dict(cfg, iterations=2), rho)


@pytest.mark.parametrize("precision,precond,rtol,bar", [(1, 0, 1e-12, 1e-9), (0, 1, 1e-13, 1e-10),
                                                        (1, 1, 1e-12, 1e-9)])
def test_coarse_mesh_with_fp32_refine_and_multigrid_fine_lanes(gpu, precision, precond, rtol,
                                                               bar):
    # the fine lanes in FP32 with FP64 refinement and/or multigrid-preconditioned;
    # the coarse-mesh solves stay FP64 Jacobi PCG
    _check(_cfg(nx=48, ny=40, n_steps=60, n_slices=6, precision=precision, precond=precond,
                cg_rtol=rtol), density_uniform_noise(48, 40, 52), bar=bar)


def test_coarse_mesh_with_checkpoints(gpu):
    # S holds T_{Mn} and T_{Mn+1} only; the fine adjoint lanes recompute the rest
    cfg = _cfg(nx=48, ny=40, n_steps=60, n_slices=6)
    rho = density_uniform_noise(48, 40, 61)
    o = run_oracle(cfg, rho)
    g = run_gpu(dict(cfg, storage=1), rho, with_status=True)
    assert g["status"]["status"] == 0
    M, Ntau = 10, 6
    assert g["S"].shape[0] == 2 * Ntau
    ref = dict(o, S=np.concatenate([o["S"][M - 1::M], o["S"][0::M]]))
    e = compare(g, ref)
    print("ckpt", e, g["status"], flush=True)
    assert max(e.values()) <= 1e-10
    # two iterations: the sweep's outputs serve as G(u^k_n) again
    cfg2 = dict(cfg, iterations=2)
    o2 = run_oracle(cfg2, rho)
    g2 = run_gpu(dict(cfg2, storage=1), rho, with_status=True)
    e2 = compare(g2, dict(o2, S=np.concatenate([o2["S"][M - 1::M], o2["S"][0::M]])))
    print("ckpt 2 it", e2, flush=True)
    assert g2["status"]["status"] == 0 and max(e2.values()) <= 1e-10
