"""FP64 CPU oracle of one-shot Parareal topology optimisation for transient heat flow.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The HIP library never
calls it and shares no code with it; the only thing both sides consume in
common are the seeded arrays from ``workloads``.

It is a plain, slow implementation written from the paper: assembled sparse
Q1 matrices, a sparse direct solve per backward-Euler step, the sequential
reference method, the modified / time-reversed Parareal passes step by step
in the paper's order, the zero-coarse-propagator (PLT) form of Sec. 7, two
cheaper coarse propagators (a truncated solve, a coarse spatial mesh), and
the design filter and projection of Sec. 2.1.
Pins against closed forms, invariants and finite differences live in
``tests/test_oracle_*.py``.

Every function is pinned; see the tests' docstrings for which property pins
which part.
"""
from .coarse import make_G_adj, make_G_pri, pcg_fixed
from .coarse_mesh import CoarseMesh, prolong_unmasked, restrict
from .coarse_mesh import make_G_adj as make_G_adj_mesh
from .coarse_mesh import make_G_pri as make_G_pri_mesh
from .design import (filter_matrix, filter_projection, filter_projection_backward,
                     projection, projection_deriv)
from .fem import (Discretisation, Problem, dirichlet_mask, element_matrices,
                  element_nodes, simp, simp_deriv)
from .parareal import (F_adj, F_pri, G_adj, G_pri, one_cycle, parareal_adjoint,
                       parareal_forward)
from .plt import F_adj_tilde, h_adj_tilde, plt_adjoint, plt_forward, plt_objective
from .timestepping import (adjoint_sequential, adjoint_source, forward_sequential,
                           h_adj, h_pri, pnorm_p)

__all__ = [
    "Discretisation", "Problem", "dirichlet_mask", "element_matrices",
    "element_nodes", "simp", "simp_deriv", "F_adj", "F_pri", "G_adj", "G_pri",
    "one_cycle", "parareal_adjoint", "parareal_forward", "adjoint_sequential",
    "adjoint_source", "forward_sequential", "h_adj", "h_pri", "pnorm_p",
    "F_adj_tilde", "h_adj_tilde", "plt_adjoint", "plt_forward", "plt_objective",
    "filter_matrix", "filter_projection", "filter_projection_backward", "projection",
    "projection_deriv", "make_G_adj", "make_G_pri", "pcg_fixed",
    "CoarseMesh", "prolong_unmasked", "restrict", "make_G_adj_mesh", "make_G_pri_mesh",
]
