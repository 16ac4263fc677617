"""FP32 CG inside FP64 iterative refinement (precision = PT_FP32_REFINE) against
the FP64 oracle.

The inner Chronopoulos-Gear CG runs in FP32: stencil, vectors, halo exchange.
Its dot products, x and every refinement residual r = b - A x are FP64, so
each solve converges to the same FP64 tolerance as the FP64 path. The stated
bar for this precision is 1e-5 relative on every output and 1e-6 on Theta. The
tests also check that refinement reaches the FP64 bar (1e-9) on the 32x32
workload.
"""
import numpy as np
import pytest

from tests.gpu_helpers import compare, run_gpu, run_oracle
from workloads import density_uniform_noise

pytestmark = pytest.mark.gpu

PT_FP32_REFINE = 1


def _cfg(**kw):
    c = dict(nx=32, ny=32, n_steps=64, n_slices=8, pnorm=8, cg_rtol=1e-12, max_iter=20000,
             precision=PT_FP32_REFINE)
    c.update(kw)
    return c


def test_fp32_refine_plain_32_cold_and_warm(gpu):
    cfg = _cfg()
    rho = density_uniform_noise(32, 32, 0)
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho, with_status=True)
    e = compare(g, o)
    print("cold", e, g["status"])
    assert g["status"]["status"] == 0
    assert e["Theta"] <= 1e-6 and max(e.values()) <= 1e-5
    assert max(e.values()) <= 1e-9
    guess = (o["uT"], o["utheta"], o["lam"])
    rho2 = np.clip(rho + 0.01 * density_uniform_noise(32, 32, 4, 0.0, 1.0), 0, 1)
    o2 = run_oracle(cfg, rho2, guess)
    g2 = run_gpu(cfg, rho2, guess)
    e2 = compare(g2, o2)
    print("warm", e2)
    assert max(e2.values()) <= 1e-9


@pytest.mark.parametrize("nx,ny,Nt,Ntau", [(37, 23, 30, 5), (64, 20, 24, 6)])
def test_fp32_refine_ragged(gpu, nx, ny, Nt, Ntau):
    cfg = _cfg(nx=nx, ny=ny, n_steps=Nt, n_slices=Ntau)
    rho = density_uniform_noise(nx, ny, 3 * nx + ny)
    e = compare(run_gpu(cfg, rho), run_oracle(cfg, rho))
    assert e["Theta"] <= 1e-6 and max(e.values()) <= 1e-5


def test_fp32_refine_streaming_mode(gpu):
    """The streaming engine (vectors through HBM, FP32 storage) on the same problem."""
    cfg = _cfg(nx=40, ny=40, n_steps=32, n_slices=8, tuning=dict(resident=0))
    rho = density_uniform_noise(40, 40, 17)
    e = compare(run_gpu(cfg, rho), run_oracle(cfg, rho))
    assert e["Theta"] <= 1e-6 and max(e.values()) <= 1e-5


def test_fp64_streaming_mode(gpu):
    """The FP64 streaming engine meets the FP64 bar too."""
    cfg = _cfg(nx=40, ny=40, n_steps=32, n_slices=8, precision=0, cg_rtol=1e-13,
               tuning=dict(resident=0))
    rho = density_uniform_noise(40, 40, 17)
    e = compare(run_gpu(cfg, rho), run_oracle(cfg, rho))
    assert max(e.values()) <= 1e-10
