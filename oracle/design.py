"""Design-field front end (oracle, FP64, CPU): the linear density filter and
the threshold projection of Sec. 2.1, and the chain rule through both.

TEST INFRASTRUCTURE: used only by tests, the smoke check and the bench's CPU
baseline.

  chi_fil = H chi,   H_ei = w_ei / sum_i w_ei,   w_ei = max(0, r_fil - |x_e - x_i|),
  chi_phys = P(chi_fil) = (tanh(beta (chi_fil - eta)) + tanh(beta eta))
                          / (tanh(beta (1 - eta)) + tanh(beta eta)),
with x_e the element centroids ((i+1/2)/nx, (j+1/2)/ny) of the unit square and
elements off the grid left out. The gradient of a function J(chi_phys) with
respect to chi is H^T (P'(chi_fil) o dJ/dchi_phys). beta <= 0 stands for no
projection (P the identity).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def filter_matrix(nx: int, ny: int, r: float) -> sp.csr_matrix:
    """H as a sparse matrix, row e = element (i, j) at j nx + i, built pair by pair
    from the definition (every element within distance r of element e)."""
    rows, cols, vals = [], [], []
    Rx = int(np.floor(r * nx))
    Ry = int(np.floor(r * ny))
    for j in range(ny):
        for i in range(nx):
            e = j * nx + i
            ws = []
            for j2 in range(max(0, j - Ry), min(ny, j + Ry + 1)):
                for i2 in range(max(0, i - Rx), min(nx, i + Rx + 1)):
                    d = np.hypot((i2 - i) / nx, (j2 - j) / ny)
                    w = max(0.0, r - d)
                    if w > 0.0:
                        ws.append((j2 * nx + i2, w))
            W = sum(w for _, w in ws)
            for k, w in ws:
                rows.append(e)
                cols.append(k)
                vals.append(w / W)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nx * ny, nx * ny))


def projection(x: np.ndarray, beta: float, eta: float) -> np.ndarray:
    if beta <= 0.0:
        return np.array(x, dtype=np.float64)
    den = np.tanh(beta * (1.0 - eta)) + np.tanh(beta * eta)
    return (np.tanh(beta * (x - eta)) + np.tanh(beta * eta)) / den


def projection_deriv(x: np.ndarray, beta: float, eta: float) -> np.ndarray:
    if beta <= 0.0:
        return np.ones_like(np.asarray(x, dtype=np.float64))
    den = np.tanh(beta * (1.0 - eta)) + np.tanh(beta * eta)
    return beta * (1.0 - np.tanh(beta * (x - eta)) ** 2) / den


def filter_projection(chi: np.ndarray, nx: int, ny: int, r: float, beta: float, eta: float):
    """Returns (chi_fil, chi_phys)."""
    H = filter_matrix(nx, ny, r)
    fil = H @ chi
    return fil, projection(fil, beta, eta)


def filter_projection_backward(chi_fil: np.ndarray, grad_phys: np.ndarray, nx: int, ny: int,
                               r: float, beta: float, eta: float) -> np.ndarray:
    """dJ/dchi = H^T (P'(chi_fil) o dJ/dchi_phys)."""
    H = filter_matrix(nx, ny, r)
    return H.T @ (projection_deriv(chi_fil, beta, eta) * grad_phys)
