"""Checkpointed storage (storage = PT_CHECKPOINT) against the oracle and
against the store-all path.

With checkpoints, the forward pass keeps only the corrected coarse states
T_{Mn} and each slice's first fine state T_{Mn+1}. The adjoint pass recomputes
the other M-2 states of a slice inside the fine adjoint lane, then runs the
slice's adjoint steps. The recompute repeats the forward arithmetic exactly:
the fine lanes of both passes run on groups of the same fixed shape. Hence:
- the results match the oracle at the FP64 bar (1e-10);
- with the store-all path forced to the same fine-lane shape, every output is
  bit for bit equal to the store-all run;
- the stored rows are the oracle's T_{Mn} and T_{Mn+1}.

The large-design configuration (smooth Gaussian density, multigrid, FP32 inner
CG with FP64 refinement, checkpoints) is checked against stored oracle samples
(written by tests/golden/make_oracle_samples.py from the oracle only) at
512 x 512 (tests/golden/oracle_large_law_512.txt) and on the full 2048 x 2048
grid with 512 steps in 32 slices (tests/golden/oracle_large_2048_512.txt: the
large design's M = 16 and two waves of 16 recomputing slices). The bar is
1e-5, and 1e-6 on Theta. At 2048 x 2048 the same cycle is also compared with
the FP64 multigrid cycle that stores every state (see that test for its bar).
"""
import os

import numpy as np
import pytest

from tests.gpu_helpers import compare, run_gpu, run_oracle
from workloads import density_uniform_noise, workload, workload_density

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _cfg(**kw):
    c = dict(nx=32, ny=32, n_steps=64, n_slices=8, pnorm=8, cg_rtol=1e-13, max_iter=20000,
             storage=1)
    c.update(kw)
    return c


def _ck_compare(g, o, M, Ntau):
    """Errors of a checkpointed GPU run: S rows are T_{Mn} then T_{Mn+1}."""
    S_o = np.asarray(o["S"])
    coarse = S_o[M - 1::M]            # T_M, T_2M, ..., T_{N_t}
    first = S_o[0::M]                 # T_1, T_{M+1}, ...
    ref = dict(o)
    ref["S"] = np.concatenate([coarse, first])
    return compare(g, ref)


@pytest.mark.parametrize("nx,ny,Nt,Ntau", [(32, 32, 64, 8), (20, 12, 24, 8), (16, 16, 32, 16),
                                           (24, 20, 30, 10), (9, 14, 40, 4)])
def test_checkpoint_fp64_against_oracle(gpu, nx, ny, Nt, Ntau):
    """M = 8, 3, 2, 3 and 10 (recomputing 6, 1, 0, 1 and 8 states per slice)."""
    cfg = _cfg(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau)
    rho = density_uniform_noise(nx, ny, 7 * nx + ny)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho, with_status=True)
    assert g["status"]["status"] == 0
    e = _ck_compare(g, o, Nt // Ntau, Ntau)
    print((nx, ny, Nt, Ntau), e, flush=True)
    assert max(e.values()) <= 1e-10


def test_checkpoint_warm_and_few_slots(gpu):
    """Warm restart (guesses from the oracle's cold cycle), with fewer scratch
    slots than slices so that groups run several fine adjoint lanes each."""
    cfg = dict(_cfg(), tuning=dict(ck_slots=3))
    rho = density_uniform_noise(32, 32, 3)
    cold = run_oracle(cfg, rho)
    rho2 = np.clip(rho + 0.01 * density_uniform_noise(32, 32, 8, 0.0, 1.0), 0, 1)
    guess = (cold["uT"], cold["utheta"], cold["lam"])
    o = run_oracle(cfg, rho2, guess)
    g = run_gpu(cfg, rho2, guess, with_status=True)
    assert g["status"]["status"] == 0
    e = _ck_compare(g, o, 8, 8)
    print(e, flush=True)
    assert max(e.values()) <= 1e-10


@pytest.mark.parametrize("precond", [0, 1])
def test_checkpoint_bitwise_equals_store_all(gpu, precond):
    """Same fine-lane shape in both runs: the recomputed states are the stored
    ones, so lambda and dTheta/drho agree bit for bit."""
    cfg = _cfg(nx=48, ny=40, n_steps=60, n_slices=6, cg_rtol=1e-10, precond=precond,
               tuning=dict(fine_wgs=4, resident=0))
    rho = density_uniform_noise(48, 40, 21)
    ck = run_gpu(cfg, rho, with_status=True)
    sa = run_gpu(dict(cfg, storage=0), rho, with_status=True)
    assert ck["status"]["status"] == 0 and sa["status"]["status"] == 0
    assert ck["Theta"] == sa["Theta"]
    for key in ("grad", "lam", "uT", "utheta"):
        assert np.array_equal(ck[key], sa[key]), key
    M = 10
    assert np.array_equal(ck["S"][:6], sa["S"][M - 1::M])
    assert np.array_equal(ck["S"][6:], sa["S"][0::M])


def test_checkpoint_gmg_fp32_refine(gpu):
    """The large-design solver settings on a small grid."""
    cfg = _cfg(nx=64, ny=64, n_steps=64, n_slices=8, cg_rtol=1e-12, precond=1, precision=1)
    rho = density_uniform_noise(64, 64, 5)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho, with_status=True)
    assert g["status"]["status"] == 0
    e = _ck_compare(g, o, 8, 8)
    print(e, flush=True)
    assert e["Theta"] <= 1e-6 and max(e.values()) <= 1e-5


def test_large_law_512_against_stored_oracle_samples(gpu):
    """Gaussian-bump density, multigrid, FP32 + refinement, checkpoints at 512 x 512
    (N_t = 512 in 32 slices), cold cycle, against the stored oracle samples."""
    from tests.golden.make_oracle_samples import load
    path = os.path.join(HERE, "golden", "oracle_large_law_512.txt")
    gold = load(path)
    w = workload("large_law_512")
    cfg = dict(nx=w["nx"], ny=w["ny"], n_steps=w["n_steps"], n_slices=w["n_slices"], pnorm=8,
               cg_rtol=1e-10, max_iter=20000, precond=1, precision=1, storage=1)
    g = run_gpu(cfg, workload_density("large_law_512"), with_status=True)
    assert g["status"]["status"] == 0
    M, Ntau, Nn = 16, 32, 513 * 513
    errs = {"Theta": abs(g["Theta"] - gold["Theta"]) / gold["Theta"],
            "utheta": float(np.abs(g["utheta"] - gold["utheta"]).max() / gold["Theta"])}
    # S samples: only the checkpointed rows are on the GPU
    idx = gold["S_idx"]
    rows, cols = idx // Nn, idx % Nn
    sel_c = (rows + 1) % M == 0
    gv = g["S"][(rows[sel_c] + 1) // M - 1, cols[sel_c]]
    errs["S_coarse"] = float(np.abs(gv - gold["S_val"][sel_c]).max() / gold["S_absmax"])
    sel_f = rows % M == 0
    gv = g["S"][Ntau + rows[sel_f] // M, cols[sel_f]]
    errs["S_first"] = float(np.abs(gv - gold["S_val"][sel_f]).max() / gold["S_absmax"])
    for key in ("uT", "lam", "grad"):
        vals = np.asarray(g[key], dtype=np.float64).reshape(-1)[gold[key + "_idx"]]
        errs[key] = float(np.abs(vals - gold[key + "_val"]).max() / gold[key + "_absmax"])
    errs["grad_norm"] = abs(np.linalg.norm(g["grad"]) - gold["grad_norm"]) / gold["grad_norm"]
    print(errs, flush=True)
    assert errs["Theta"] <= 1e-6 and max(errs.values()) <= 1e-5


def _sampled_errors(g, gold, M, Ntau, Nn):
    """Errors of GPU outputs (torch tensors on the device, S checkpointed)
    at the fixture's sample indices, relative to the fixture's maxima."""
    import torch
    dev = g["grad"].device
    errs = {"Theta": abs(float(g["Theta"]) - gold["Theta"]) / gold["Theta"],
            "utheta": float(np.abs(g["utheta"].cpu().numpy() - gold["utheta"]).max() /
                            gold["Theta"])}
    idx = gold["S_idx"]
    rows, cols = idx // Nn, idx % Nn
    assert np.all(((rows + 1) % M == 0) | (rows % M == 0))
    ckrow = np.where((rows + 1) % M == 0, (rows + 1) // M - 1, Ntau + rows // M)
    flat = torch.tensor(ckrow * Nn + cols, device=dev)
    vals = g["S"].reshape(-1)[flat].cpu().numpy()
    errs["S"] = float(np.abs(vals - gold["S_val"]).max() / gold["S_absmax"])
    for key in ("uT", "lam", "grad"):
        vals = g[key].reshape(-1)[torch.tensor(gold[key + "_idx"], device=dev)].cpu().numpy()
        errs[key] = float(np.abs(vals - gold[key + "_val"]).max() / gold[key + "_absmax"])
    gn = float(torch.linalg.norm(g["grad"]))
    errs["grad_norm"] = abs(gn - gold["grad_norm"]) / gold["grad_norm"]
    return errs


def _large_cycle(gpu, precision, storage, rtol=1e-10):
    """One cold cycle of the large design at 2048 x 2048 (N_t = 512 in 32
    slices, multigrid); the outputs stay on the device."""
    import torch

    from paper_2411_19030_amd import Problem
    from paper_2411_19030_amd.cycle import Cycle
    w = workload("large_2048_512")
    prob = Problem(nx=w["nx"], ny=w["ny"], n_steps=w["n_steps"], n_slices=w["n_slices"],
                   pnorm=8, cg_rtol=rtol, max_iter=20000, precond=1, precision=precision,
                   storage=storage)
    cyc = Cycle(prob, gpu)
    rho = torch.tensor(workload_density("large_2048_512"), dtype=torch.float64, device=gpu)
    cyc.run(rho)
    torch.cuda.synchronize()
    st = cyc.status()
    out = dict(S=cyc.S, uT=cyc.uT, utheta=cyc.utheta, lam=cyc.lam, Theta=cyc.Theta,
               grad=cyc.grad, status=st)
    del cyc.ws
    torch.cuda.empty_cache()
    return out


def test_large_2048_against_stored_oracle_samples(gpu):
    """The large design's solver settings (multigrid, FP32 + refinement,
    checkpoints) on the full 2048 x 2048 grid, cold cycle, against the oracle."""
    from tests.golden.make_oracle_samples import load
    gold = load(os.path.join(HERE, "golden", "oracle_large_2048_512.txt"))
    print("2048 x 2048, 512 steps in 32 slices: multigrid, FP32 + refinement, checkpoints",
          flush=True)
    g = _large_cycle(gpu, precision=1, storage=1)
    assert g["status"]["status"] == 0, g["status"]
    errs = _sampled_errors(g, gold, 16, 32, 2049 * 2049)
    print(errs, g["status"], flush=True)
    assert errs["Theta"] <= 1e-6 and max(errs.values()) <= 1e-5


def test_large_2048_fp32_checkpoint_matches_fp64_store_all(gpu):
    """FP32 inner CG with FP64 refinement and checkpoints against the FP64
    multigrid cycle storing every state, both on the GPU at 2048 x 2048. Each
    solves every system to the same FP64 true-residual tolerance (1e-10), so
    the states differ by what that tolerance leaves, about 100 cg_rtol each
    against the exact solution (see the full-size FP64 tests): bar 1e-7 on
    every stored state (relative to its maximum, S on the checkpointed rows)
    and 1e-8 on Theta. The gradient sums lambda^T dK/drho T over all 512 fine
    steps, so it gathers the differences of every step (measured 2.5e-7
    against 1.9e-9 on the slice-end lambda): bar 1e-6 on its 2-norm."""
    import torch
    print("2048 x 2048: FP32 + refinement with checkpoints", flush=True)
    ck = _large_cycle(gpu, precision=1, storage=1)
    print("2048 x 2048: FP64 storing every state", flush=True)
    sa = _large_cycle(gpu, precision=0, storage=0)
    assert ck["status"]["status"] == 0 and sa["status"]["status"] == 0
    M, Ntau = 16, 32

    def rel(a, b):
        return float((a - b).abs().max() / b.abs().max())

    errs = {"Theta": abs(float(ck["Theta"]) - float(sa["Theta"])) / float(sa["Theta"]),
            "utheta": rel(ck["utheta"], sa["utheta"]),
            "S_coarse": rel(ck["S"][:Ntau], sa["S"][M - 1::M]),
            "S_first": rel(ck["S"][Ntau:], sa["S"][0::M]),
            "uT": rel(ck["uT"], sa["uT"]), "lam": rel(ck["lam"], sa["lam"]),
            "grad": float(torch.linalg.norm(ck["grad"] - sa["grad"]) /
                          torch.linalg.norm(sa["grad"]))}
    print(errs, flush=True)
    assert errs["Theta"] <= 1e-8 and errs["grad"] <= 1e-6
    assert max(v for k, v in errs.items() if k != "grad") <= 1e-7
