"""Parity at the full workload sizes, in the launch configuration the benchmark
times (default plan, resident engine).

* 256 x 256, 512 steps in 32 slices: the oracle runs in the test. Two cycles
  are checked element by element: a cold cycle, then a warm cycle on a
  perturbed design with the oracle's cold outputs as the guesses of both
  sides. The benchmark times this warm cycle.
* 512 x 512, 1024 steps in 64 slices: the oracle's cold cycle takes minutes,
  so its values at seeded sample indices are stored in
  tests/golden/oracle_diff_fp64_512.txt (written by
  tests/golden/make_oracle_samples.py, which calls only the oracle).

Bars: at cg_rtol 1e-13 every output is within 1e-10 (relative to the field's
maximum). At the benchmark's own cg_rtol 1e-10 the bar is 1e-8: a relative
residual of 1e-10 per solve, amplified by at most the operator's condition
growth over one pass, stays below 1e-8 (measured: ~2e-10 on Theta).
"""
import os

import numpy as np
import pytest

import oracle as O
from tests.golden.make_oracle_samples import load
from tests.gpu_helpers import compare, oracle_problem, run_gpu
from workloads import workload, workload_density

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _cfg(name, **kw):
    w = workload(name)
    c = dict(nx=w["nx"], ny=w["ny"], n_steps=w["n_steps"], n_slices=w["n_slices"], pnorm=w["p"],
             max_iter=20000)
    c.update(kw)
    return c


def _oracle_cycle(cfg, rho, guess=None):
    d = O.Discretisation(oracle_problem(cfg), rho)
    if guess is None:
        fw = O.parareal_forward(d, 1)
        ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], 1)
    else:
        fw = O.parareal_forward(d, 1, guess[0], guess[1])
        ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], 1, guess[2])
    return dict(S=fw["S"], uT=fw["uT"], utheta=fw["utheta"], Theta=fw["Theta"],
                lam=ad["lam"], grad=ad["grad"])


@pytest.fixture(scope="module")
def oracle_256():
    cfg = _cfg("plain_fp64_256")
    rho = workload_density("plain_fp64_256")
    cold = _oracle_cycle(cfg, rho)
    rho2 = np.clip(rho + 0.005 * np.cos(np.arange(rho.size) * 0.37), 0, 1)
    warm = _oracle_cycle(cfg, rho2, (cold["uT"], cold["utheta"], cold["lam"]))
    return cfg, rho, rho2, cold, warm


@pytest.mark.parametrize("rtol,bar", [(1e-13, 1e-10), (1e-10, 1e-8)])
def test_plain_fp64_256_cold_and_warm(gpu, oracle_256, rtol, bar):
    cfg, rho, rho2, cold, warm = oracle_256
    cfg = dict(cfg, cg_rtol=rtol)
    g = run_gpu(cfg, rho, device=gpu, with_status=True)
    assert g["status"]["status"] == 0
    e = compare(g, cold)
    print("cold", rtol, e, flush=True)
    assert max(e.values()) <= bar
    guess = (cold["uT"], cold["utheta"], cold["lam"])
    g2 = run_gpu(cfg, rho2, guess, device=gpu, with_status=True)
    assert g2["status"]["status"] == 0
    e2 = compare(g2, warm)
    print("warm", rtol, e2, flush=True)
    assert max(e2.values()) <= bar


def test_diff_fp64_512_cold_against_stored_oracle_samples(gpu):
    gold = load(os.path.join(HERE, "golden", "oracle_diff_fp64_512.txt"))
    cfg = _cfg("diff_fp64_512", cg_rtol=1e-13, max_iter=50000)
    g = run_gpu(cfg, workload_density("diff_fp64_512"), device=gpu, with_status=True)
    assert g["status"]["status"] == 0
    errs = {"Theta": abs(g["Theta"] - gold["Theta"]) / gold["Theta"],
            "utheta": float(np.abs(g["utheta"] - gold["utheta"]).max() / gold["Theta"]),
            "grad_norm": abs(np.linalg.norm(g["grad"]) - gold["grad_norm"]) / gold["grad_norm"],
            # the sum of N_e entries is at most sqrt(N_e) times their 2-norm
            "grad_sum": abs(float(np.sum(g["grad"])) - gold["grad_sum"]) /
            (np.sqrt(g["grad"].size) * gold["grad_norm"])}
    for key in ("S", "uT", "lam", "grad"):
        vals = np.asarray(g[key], dtype=np.float64).reshape(-1)[gold[key + "_idx"]]
        errs[key] = float(np.abs(vals - gold[key + "_val"]).max() / gold[key + "_absmax"])
        errs[key + "_absmax"] = abs(float(np.abs(g[key]).max()) - gold[key + "_absmax"]) / \
            gold[key + "_absmax"]
    print(errs, flush=True)
    assert max(errs.values()) <= 1e-10
