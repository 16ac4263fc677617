"""A coarse propagator on a coarser spatial mesh (oracle, FP64, CPU).

TEST INFRASTRUCTURE: used only by tests, the smoke check and the bench's CPU
baseline.

The paper finds the sequential coarse propagators to be the bottleneck of the
one-shot method and proposes evaluating them on a coarse spatial mesh
(Sec. 7.3, Sec. 8). It does not define that propagator; this module is the
reading used here. With a coarsening factor f (nx and ny divisible by f):

* the coarse mesh has nx/f x ny/f elements of the same domain; coarse node
  (I, J) coincides with fine node (f I, f J);
* a coarse element's conductivity and capacity are the arithmetic means of
  the SIMP values (Eq. 2.5-2.6) of the f x f fine elements it covers;
* a coarse node is a Dirichlet node iff its fine node is one;
* R (fine to coarse) is injection at the coinciding nodes;
* P (coarse to fine) is the bilinear (Q1) interpolant of the coarse field,
  evaluated at the fine nodes and then set to 0 at the fine Dirichlet nodes;
* G_pri^c(T, theta, n): one backward-Euler step of size dtau (Alg. 1) on the
  coarse mesh from R T, with the load at tau_{n+1}; the state returned is
  T' = P T_c', and theta is updated from it as in Alg. 1,
  theta' = (theta^p + ||T'||_p^p / (N_tau N_e))^{1/p};
* G_adj^c(lambda, g, n): one backward-Euler step of the adjoint problem
  (Alg. 2) on the coarse mesh from R lambda, whose source is the fine source
  of Eq. 4.6 at T_m (m = M(n-1)+1 as in G_adj) carried to the coarse mesh by
  P^T, the transfer that also gives the coarse load (P^T f); then
  lambda' = P lambda_c' and g' = g - (1/N_tau) lambda'^T (dC (T_m - T_{m-M})/dtau
  + dK T_m) on the fine elements (Eq. 4.16 with the coarse step's output).

The objective and the adjoint source are nodal sums over the fine nodes, so
they are evaluated on the fine field (the coarse nodes with their own count
would weight the boundary differently and miss the fine step by up to ~17% in
the adjoint).
With f = 1 both reduce to the paper's G_pri and G_adj exactly. Every Parareal
property that holds for any G (exactness after N_tau iterations) holds here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from .fem import Discretisation, element_matrices, element_nodes, simp
from .timestepping import pnorm_p


def restrict(T: np.ndarray, nx: int, ny: int, f: int) -> np.ndarray:
    """Injection: the fine values at the nodes (f I, f J)."""
    return np.asarray(T).reshape(ny + 1, nx + 1)[::f, ::f].reshape(-1).copy()


def _weights(n: int, f: int):
    """For fine index k = 0..n: the coarse indices K, K1 of its coarse interval
    and the bilinear weight w of K1 (1 - w of K)."""
    k = np.arange(n + 1)
    K, a = np.divmod(k, f)
    return K, np.minimum(K + 1, n // f), a / f


def prolong_unmasked(Tc: np.ndarray, nx: int, ny: int, f: int) -> np.ndarray:
    """Bilinear interpolant of the coarse nodal field at every fine node."""
    G = np.asarray(Tc).reshape(ny // f + 1, nx // f + 1)
    I, I1, wx = _weights(nx, f)
    J, J1, wy = _weights(ny, f)
    wx, wy = wx[None, :], wy[:, None]
    out = ((1 - wx) * (1 - wy) * G[np.ix_(J, I)] + wx * (1 - wy) * G[np.ix_(J, I1)]
           + (1 - wx) * wy * G[np.ix_(J1, I)] + wx * wy * G[np.ix_(J1, I1)])
    return out.reshape(-1)


class CoarseMesh:
    """The coarse-mesh operators of one fine discretisation."""

    def __init__(self, d: Discretisation, f: int = 2):
        P = d.prob
        if P.nx % f or P.ny % f:
            raise ValueError("nx and ny must be divisible by the coarsening factor")
        self.d, self.f = d, f
        self.nx, self.ny = P.nx // f, P.ny // f
        nxc, nyc = self.nx, self.ny
        self.n_nodes = (nxc + 1) * (nyc + 1)
        self.n_elem = nxc * nyc
        # coefficient means over the f x f fine elements of each coarse element
        k = simp(d.rho, P.k0, P.kmin, P.pk).reshape(P.ny, P.nx)
        c = simp(d.rho, P.c0, P.cmin, P.pc).reshape(P.ny, P.nx)
        self.k = k.reshape(nyc, f, nxc, f).mean(axis=(1, 3)).reshape(-1)
        self.c = c.reshape(nyc, f, nxc, f).mean(axis=(1, 3)).reshape(-1)
        K0, C0, f0 = element_matrices(1.0 / nxc, 1.0 / nyc)
        conn = element_nodes(nxc, nyc)
        rows = np.repeat(conn, 4, axis=1).reshape(-1)
        cols = np.tile(conn, (1, 4)).reshape(-1)
        nn = self.n_nodes
        self.K = sp.coo_matrix(((self.k[:, None] * K0.reshape(1, 16)).reshape(-1), (rows, cols)),
                               shape=(nn, nn)).tocsr()
        self.C = sp.coo_matrix(((self.c[:, None] * C0.reshape(1, 16)).reshape(-1), (rows, cols)),
                               shape=(nn, nn)).tocsr()
        self.f_unit = np.zeros(nn)
        np.add.at(self.f_unit, conn.reshape(-1), np.tile(f0, self.n_elem))
        self.dmask = restrict(d.dmask, P.nx, P.ny, f).astype(bool)
        self.free = np.flatnonzero(~self.dmask)
        A = (self.C / P.dtau + self.K).tocsr()[self.free][:, self.free].tocsc()
        self._lu = splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                        options=dict(SymmetricMode=True)) if self.free.size else None

    def R(self, T: np.ndarray) -> np.ndarray:
        P = self.d.prob
        return restrict(T, P.nx, P.ny, self.f)

    def P(self, Tc: np.ndarray) -> np.ndarray:
        P = self.d.prob
        out = prolong_unmasked(Tc, P.nx, P.ny, self.f)
        out[self.d.dmask] = 0.0
        return out

    def PT(self, v: np.ndarray) -> np.ndarray:
        """The transpose of P: each fine value goes to the coarse nodes of its
        element with the bilinear weights (fine Dirichlet nodes contribute 0)."""
        Pd = self.d.prob
        w = np.where(self.d.dmask, 0.0, np.asarray(v, dtype=np.float64)).reshape(Pd.ny + 1,
                                                                              Pd.nx + 1)
        I, I1, wx = _weights(Pd.nx, self.f)
        J, J1, wy = _weights(Pd.ny, self.f)
        wx, wy = wx[None, :], wy[:, None]
        out = np.zeros((self.ny + 1, self.nx + 1))
        for rows, cols, wgt in ((J, I, (1 - wx) * (1 - wy)), (J, I1, wx * (1 - wy)),
                                (J1, I, (1 - wx) * wy), (J1, I1, wx * wy)):
            np.add.at(out, (rows[:, None], cols[None, :]), wgt * w)
        return out.reshape(-1)

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        """x with (C_c/dtau + K_c) x = rhs on the coarse free nodes, 0 elsewhere."""
        x = np.zeros(self.n_nodes)
        if self._lu is not None:
            x[self.free] = self._lu.solve(rhs[self.free])
        return x


def make_G_pri(d: Discretisation, f: int = 2):
    """G_pri^c as a function (d, T, theta, n) -> (T', theta') for the
    Parareal passes."""
    cm = CoarseMesh(d, f)

    def G(d_: Discretisation, T: np.ndarray, theta: float, n: int):
        P = d_.prob
        rhs = cm.C @ cm.R(T) / P.dtau + P.q_at(P.M * (n + 1)) * cm.f_unit
        Tn = cm.P(cm.solve(rhs))
        th = (theta ** P.p + pnorm_p(Tn, P.p) / (P.n_slices * P.n_elem)) ** (1.0 / P.p)
        return Tn, th

    G.mesh = cm
    return G


def make_G_adj(d: Discretisation, f: int = 2):
    """G_adj^c as a function (d, S, Theta, lam, g, n) -> (lam', g')."""
    cm = CoarseMesh(d, f)

    def G(d_: Discretisation, S: np.ndarray, Theta: float, lam: np.ndarray, g: np.ndarray,
          n: int):
        P = d_.prob
        m = P.M * (n - 1) + 1
        Tm = S[m - 1]
        Tprev = S[m - P.M - 1] if m - P.M >= 1 else np.zeros(P.n_nodes)
        src = cm.PT(Theta ** (1 - P.p) / P.n_elem * Tm ** (P.p - 1))
        lc = cm.solve(cm.C @ cm.R(lam) / P.dtau + src)
        lam_n = cm.P(lc)
        g_n = g - d_.element_term(lam_n, Tm, Tprev, P.dtau) / P.n_slices
        return lam_n, g_n

    G.mesh = cm
    return G
