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
CG with FP64 refinement, checkpoints) is checked at 512 x 512 against stored
oracle samples (tests/golden/oracle_large_law_512.txt, written by
tests/golden/make_oracle_samples.py from the oracle only). The bar is 1e-5,
and 1e-6 on Theta.
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


def test_checkpoint_warm_and_few_slots(gpu, monkeypatch):
    """Warm restart (guesses from the oracle's cold cycle), with fewer scratch
    slots than slices so that groups run several fine adjoint lanes each."""
    monkeypatch.setenv("PT_CK_SLOTS", "3")
    cfg = _cfg()
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
def test_checkpoint_bitwise_equals_store_all(gpu, monkeypatch, precond):
    """Same fine-lane shape in both runs: the recomputed states are the stored
    ones, so lambda and dTheta/drho agree bit for bit."""
    monkeypatch.setenv("PT_FINE_WGS", "4")
    monkeypatch.setenv("PT_RESIDENT", "0")
    cfg = _cfg(nx=48, ny=40, n_steps=60, n_slices=6, cg_rtol=1e-10, precond=precond)
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
