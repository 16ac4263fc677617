"""The paper's own test case (Sec. 5.1) at its full size against the oracle.

100 x 100 elements and N_t = 480. The Table 1 materials include c-SIMP, so
the capacity term of every sensitivity is live. The load q(t) follows
Eq. 5.1, the Dirichlet patch is the centre tenth of the bottom edge, and
p = 20. The seeded branched design stands in for the paper's optimised
design. Starts are cold: the guesses come from the coarse propagators
(Sec. 5.2), or are zero for the PLT form of Sec. 7. The coarse-spatial-mesh
propagators (Sec. 7.3) run here on their 51 x 51-node mesh, whose coarse
solves keep their vectors in LDS.

Solves run to rtol 1e-13. The bar is 1e-9: the coarse operator here reaches
k dtau / h^2 = 3000 at N_tau = 10, ten times the workloads' largest, and
the solution error of a solve grows with the condition number times the
residual.
"""
import pytest

from tests.gpu_helpers import compare, run_gpu, run_oracle
from workloads import workload, workload_density

pytestmark = pytest.mark.gpu


def _cfg(**kw):
    w = workload("paper_100")
    c = dict(nx=w["nx"], ny=w["ny"], n_steps=w["n_steps"], n_slices=w["n_slices"],
             pnorm=w["p"], k0=w["k0"], kmin=w["kmin"], pk=w["pk"], c0=w["c0"], cmin=w["cmin"],
             pc=w["pc"], q=w["q"], t_final=w["t_final"], bc=w["bc"], cg_rtol=1e-13,
             max_iter=50000)
    c.update(kw)
    return c


@pytest.mark.parametrize("Ntau,iters,prop", [(10, 2, 0), (30, 1, 0), (30, 3, 1), (5, 1, 1),
                                             (30, 1, 2), (10, 2, 2)])
def test_paper_test_case_against_oracle(gpu, Ntau, iters, prop):
    cfg = _cfg(n_slices=Ntau, iterations=iters, propagator=prop)
    rho = workload_density("paper_100")
    o = run_oracle(cfg, rho)
    g = run_gpu(cfg, rho, with_status=True)
    e = compare(g, o)
    print(Ntau, iters, prop, e, g["status"], flush=True)
    assert g["status"]["status"] == 0
    assert max(e.values()) <= 1e-9
