"""Q1 Galerkin discretisation of transient heat conduction (oracle, FP64, CPU).

TEST INFRASTRUCTURE: only the tests, the smoke check and the bench's CPU
baseline use this package. It shares no code with the HIP path.

Follows the paper's Sec. 2 (Eq. 2.1 PDE and boundary conditions; Sec. 2.1
SIMP interpolation Eq. 2.5-2.6; Sec. 2.2 "simple Galerkin" discretisation with
rectangular bilinear elements, element-wise constant k, c and q, Eq. 2.7).

Element matrices are derived here by 2x2 Gauss quadrature of the bilinear
shape functions rather than typed in, so that they are the Galerkin
definition written out. Local node order of an element (ex, ey):
(ex, ey), (ex+1, ey), (ex+1, ey+1), (ex, ey+1). Node (i, j) has id
j*(nx+1)+i; element (ex, ey) has id ey*nx+ex. The domain is the unit square
(L = 1, Sec. 5.1), so hx = 1/nx and hy = 1/ny; the out-of-plane depth is L = 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


def _shape(xi: float, eta: float):
    """Bilinear shape functions on the reference square [0,1]^2 and their
    derivatives with respect to xi and eta, in the local node order."""
    N = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta])
    dxi = np.array([-(1 - eta), (1 - eta), eta, -eta])
    deta = np.array([-(1 - xi), -xi, xi, (1 - xi)])
    return N, dxi, deta


def element_matrices(hx: float, hy: float):
    """Unit-coefficient element matrices of one hx x hy rectangle.

    Returns (K0, C0, f0): K0[a,b] = int grad N_a . grad N_b,
    C0[a,b] = int N_a N_b, f0[a] = int N_a (2x2 Gauss, exact for these
    polynomial degrees).
    """
    g, w = np.polynomial.legendre.leggauss(2)
    pts = (g + 1.0) / 2.0
    wts = w / 2.0
    K0 = np.zeros((4, 4))
    C0 = np.zeros((4, 4))
    f0 = np.zeros(4)
    for a, xi in enumerate(pts):
        for b, eta in enumerate(pts):
            N, dxi, deta = _shape(xi, eta)
            gx = dxi / hx
            gy = deta / hy
            wq = wts[a] * wts[b] * hx * hy
            K0 += wq * (np.outer(gx, gx) + np.outer(gy, gy))
            C0 += wq * np.outer(N, N)
            f0 += wq * N
    return K0, C0, f0


def element_nodes(nx: int, ny: int) -> np.ndarray:
    """Connectivity (N_e, 4): global node ids of each element in local order."""
    ex, ey = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    n0 = (ey * (nx + 1) + ex).reshape(-1)
    return np.stack([n0, n0 + 1, n0 + nx + 2, n0 + nx + 1], axis=1)


def simp(rho, v0: float, vmin: float, pen: float):
    """SIMP interpolation v(rho) = vmin + (v0 - vmin) rho^pen (Eq. 2.5-2.6)."""
    return vmin + (v0 - vmin) * np.power(rho, pen)


def simp_deriv(rho, v0: float, vmin: float, pen: float):
    """d v / d rho of the SIMP interpolation."""
    return pen * (v0 - vmin) * np.power(rho, pen - 1.0)


def dirichlet_mask(nx: int, ny: int, rule) -> np.ndarray:
    """Boolean node mask of T = 0 nodes.

    'left_centre'   : x = 0, 0.45 <= y <= 0.55 (the workloads' boundary);
                      node (0, j) iff 9*ny <= 20*j <= 11*ny.
    'bottom_centre' : y = 0, 0.45 <= x <= 0.55 (the paper's Fig. 4);
                      node (i, 0) iff 9*nx <= 20*i <= 11*nx.
    'left_edge'     : every node with x = 0.
    'none'          : no Dirichlet node.
    An explicit boolean array of length (nx+1)(ny+1) is returned as is.
    """
    nn = (nx + 1) * (ny + 1)
    if not isinstance(rule, str):
        m = np.asarray(rule, dtype=bool).reshape(-1)
        assert m.shape == (nn,)
        return m.copy()
    m = np.zeros(nn, dtype=bool)
    if rule == "left_centre":
        for j in range(ny + 1):
            if 9 * ny <= 20 * j <= 11 * ny:
                m[j * (nx + 1) + 0] = True
    elif rule == "bottom_centre":
        for i in range(nx + 1):
            if 9 * nx <= 20 * i <= 11 * nx:
                m[i] = True
    elif rule == "left_edge":
        for j in range(ny + 1):
            m[j * (nx + 1)] = True
    elif rule == "none":
        pass
    else:
        raise ValueError(f"unknown Dirichlet rule {rule!r}")
    return m


@dataclass
class Problem:
    """Everything the discretised primal/adjoint problems depend on, except rho.

    q is either a constant (uniform in space and time) or an array of length
    n_steps+1 holding q(t_n) (uniform in space), as in Eq. 5.1.
    """
    nx: int
    ny: int
    n_steps: int
    n_slices: int
    p: int = 8
    k0: float = 1.0
    kmin: float = 1e-3
    pk: float = 3.0
    c0: float = 1.0
    cmin: float = 1.0
    pc: float = 1.0
    q: object = 1.0
    t_final: float = 1.0
    bc: object = "left_centre"

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny

    @property
    def M(self) -> int:
        """Coarsening factor M = N_t / N_tau (Sec. 4.2); must be an integer."""
        if self.n_steps % self.n_slices:
            raise ValueError("N_tau must divide N_t")
        return self.n_steps // self.n_slices

    @property
    def dt(self) -> float:
        return self.t_final / self.n_steps

    @property
    def dtau(self) -> float:
        return self.t_final / self.n_slices

    def q_at(self, n: int) -> float:
        """Source at fine time t_n = n dt."""
        if np.isscalar(self.q):
            return float(self.q)
        return float(np.asarray(self.q)[n])


@dataclass
class Discretisation:
    """Assembled FP64 matrices for one design rho, with Dirichlet elimination."""
    prob: Problem
    rho: np.ndarray
    K: sp.csr_matrix = field(init=False)
    C: sp.csr_matrix = field(init=False)
    f_unit: np.ndarray = field(init=False)
    free: np.ndarray = field(init=False)

    def __post_init__(self):
        P = self.prob
        rho = np.asarray(self.rho, dtype=np.float64)
        assert rho.shape == (P.n_elem,)
        hx, hy = 1.0 / P.nx, 1.0 / P.ny
        self.K0, self.C0, self.f0 = element_matrices(hx, hy)
        self.conn = element_nodes(P.nx, P.ny)
        self.k = simp(rho, P.k0, P.kmin, P.pk)
        self.c = simp(rho, P.c0, P.cmin, P.pc)
        self.dk = simp_deriv(rho, P.k0, P.kmin, P.pk)
        self.dc = simp_deriv(rho, P.c0, P.cmin, P.pc)
        nn = P.n_nodes
        rows = np.repeat(self.conn, 4, axis=1).reshape(-1)
        cols = np.tile(self.conn, (1, 4)).reshape(-1)
        kv = (self.k[:, None] * self.K0.reshape(1, 16)).reshape(-1)
        cv = (self.c[:, None] * self.C0.reshape(1, 16)).reshape(-1)
        self.K = sp.coo_matrix((kv, (rows, cols)), shape=(nn, nn)).tocsr()
        self.C = sp.coo_matrix((cv, (rows, cols)), shape=(nn, nn)).tocsr()
        self.f_unit = np.zeros(nn)
        np.add.at(self.f_unit, self.conn.reshape(-1),
                  np.tile(self.f0, P.n_elem))
        self.dmask = dirichlet_mask(P.nx, P.ny, P.bc)
        self.free = np.flatnonzero(~self.dmask)
        self._factors = {}

    def restrict(self, A):
        return A[self.free][:, self.free]

    def _factor(self, step: float):
        """Sparse factorisation of C/step + K on the free nodes (cached).

        SuperLU with a symmetric minimum-degree ordering and no pivoting, which
        on this SPD matrix is an LDL^T factorisation stored as LU.
        """
        key = float(step)
        if key not in self._factors:
            A = self.restrict(self.C / step + self.K).tocsc()
            if A.shape[0] == 0:
                self._factors[key] = None
            else:
                from scipy.sparse.linalg import splu
                self._factors[key] = splu(
                    A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                    options=dict(SymmetricMode=True))
        return self._factors[key]

    def solve(self, step: float, rhs: np.ndarray) -> np.ndarray:
        """x with (C/step + K) x = rhs on the free nodes, x = 0 on Dirichlet nodes."""
        lu = self._factor(step)
        x = np.zeros(self.prob.n_nodes)
        if lu is not None:
            x[self.free] = lu.solve(rhs[self.free])
        return x

    def load(self, n: int) -> np.ndarray:
        """Nodal heat load q_n = q(t_n) * int N_a (element-constant q)."""
        return self.prob.q_at(n) * self.f_unit

    def element_term(self, lam: np.ndarray, T: np.ndarray, T_prev: np.ndarray,
                     step: float) -> np.ndarray:
        """Per-element lambda^T (dC/drho_e (T - T_prev)/step + dK/drho_e T) (Eq. 4.7)."""
        le = lam[self.conn]
        te = T[self.conn]
        de = (T - T_prev)[self.conn] / step
        kterm = np.einsum("ea,ab,eb->e", le, self.K0, te)
        cterm = np.einsum("ea,ab,eb->e", le, self.C0, de)
        return self.dc * cterm + self.dk * kterm
