"""pt_cycle_noalloc (the whole cycle on the library's static workspace) against
the three-call form with a caller-owned workspace, through the C ABI.

Two calls in a row on the static array, the second with a smaller problem:
each must reproduce the caller-workspace cycle on the same inputs. Both forms
run the same kernels with the same launch shapes and the engine's reductions
have a fixed order, so the outputs agree bit for bit; the stats written to
device memory match pt_query_status of the three-call form.
"""
import numpy as np
import pytest
import torch

from paper_2411_19030_amd import _pt
from paper_2411_19030_amd.cycle import Cycle
from tests.gpu_helpers import gpu_problem
from workloads import density_uniform_noise

pytestmark = pytest.mark.gpu

F64 = torch.float64


def _outputs(prob, dev):
    Nn, Nt1 = prob.n_nodes, prob.n_slices + 1
    rows = _pt.pt_state_bytes(prob) // (8 * Nn)
    return dict(S=torch.full((rows, Nn), float("nan"), dtype=F64, device=dev),
                uT=torch.full((Nt1, Nn), float("nan"), dtype=F64, device=dev),
                utheta=torch.full((Nt1,), float("nan"), dtype=F64, device=dev),
                lam=torch.full((Nt1, Nn), float("nan"), dtype=F64, device=dev),
                Theta=torch.full((), float("nan"), dtype=F64, device=dev),
                grad=torch.full((prob.n_elem,), float("nan"), dtype=F64, device=dev))


def _noalloc(prob, rho, guess, dev):
    out = _outputs(prob, dev)
    stats = torch.zeros(64, dtype=torch.uint8, device=dev)
    g = guess if guess is not None else (None, None, None)
    _pt.pt_cycle_noalloc(prob, rho, g[0], g[1], g[2], out["S"], out["uT"], out["utheta"],
                         out["lam"], out["Theta"], out["grad"], stats)
    torch.cuda.synchronize()
    st = _pt.stats_from_bytes(bytes(stats.cpu().numpy()))
    return {k: v.cpu().numpy() for k, v in out.items()}, st


def _reference(prob, rho, guess, dev):
    cyc = Cycle(prob, dev)
    if guess is None:
        cyc.forward(rho)
        cyc.adjoint(rho)
    else:
        cyc.forward(rho, guess[0], guess[1])
        cyc.adjoint(rho, guess[2])
    cyc.sensitivities(rho)
    torch.cuda.synchronize()
    st = cyc.status()
    out = dict(S=cyc.S, uT=cyc.uT, utheta=cyc.utheta, lam=cyc.lam, Theta=cyc.Theta, grad=cyc.grad)
    return {k: v.cpu().numpy() for k, v in out.items()}, st


def _check(a, b, sa, sb, tag):
    print(tag, "status", sa["status"], sb["status"], "iters", sa["cg_iters_fine"],
          sb["cg_iters_fine"], flush=True)
    for k in b:
        assert np.array_equal(a[k], b[k]), (tag, k, float(np.nanmax(np.abs(a[k] - b[k]))))
    assert sa == sb, (sa, sb)
    assert sa["status"] == 0


def test_noalloc_matches_caller_workspace_twice_second_smaller(gpu):
    dev = gpu
    # first call: 32 x 32, 64 steps in 8 slices, cold start
    p1 = gpu_problem(dict(nx=32, ny=32, n_steps=64, n_slices=8, cg_rtol=1e-12, max_iter=20000))
    assert _pt.pt_workspace_bytes(p1) <= _pt.PT_NOALLOC_WS_BYTES
    r1 = torch.tensor(density_uniform_noise(32, 32, 41), dtype=F64, device=dev)
    print("case 1: 32x32, 64/8, cold", flush=True)
    a1, sa1 = _noalloc(p1, r1, None, dev)
    b1, sb1 = _reference(p1, r1, None, dev)
    _check(a1, b1, sa1, sb1, "32x32 cold")
    # second call: a smaller problem (24 x 20, 36 steps in 6 slices) with a
    # warm start, on the array the first call left behind
    p2 = gpu_problem(dict(nx=24, ny=20, n_steps=36, n_slices=6, cg_rtol=1e-12, max_iter=20000))
    assert _pt.pt_workspace_bytes(p2) < _pt.pt_workspace_bytes(p1)
    r2 = torch.tensor(density_uniform_noise(24, 20, 42), dtype=F64, device=dev)
    print("case 2: 24x20, 36/6, cold then warm", flush=True)
    c2, _ = _noalloc(p2, r2, None, dev)
    guess = (torch.tensor(c2["uT"], device=dev), torch.tensor(c2["utheta"], device=dev),
             torch.tensor(c2["lam"], device=dev))
    a2, sa2 = _noalloc(p2, r2, guess, dev)
    b2, sb2 = _reference(p2, r2, guess, dev)
    _check(a2, b2, sa2, sb2, "24x20 warm")


def test_noalloc_rejects_a_problem_beyond_the_static_workspace(gpu):
    p = gpu_problem(dict(nx=256, ny=256, n_steps=512, n_slices=32))
    assert _pt.pt_workspace_bytes(p) > _pt.PT_NOALLOC_WS_BYTES
    out = _outputs(p, gpu)
    rho = torch.full((p.n_elem,), 0.3, dtype=F64, device=gpu)
    rc = _pt.pt_cycle_noalloc(p, rho, None, None, None, out["S"], None, None, None,
                              out["Theta"], out["grad"], check=False)
    assert rc == _pt.PT_ESIZE
