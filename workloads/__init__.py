"""Seeded synthetic inputs shared by the oracle-side and GPU-side tests and the bench.

This module holds no arithmetic of the method itself: it only draws design
fields from seeded generators and lists the workload sizes. Both the oracle
(in tests) and the HIP path receive the arrays it returns, so no random number
has to be reproduced on two sides.

Workloads (the paper's test case is a transient heat problem on the unit square
with element-wise SIMP conductivity, Sec. 2 and Sec. 5.1; the paper's own
optimised design field is not given, so seeded densities stand in for it):

* ``plain_fp64_32``     32x32 Q1 elements, N_t=64 in N_tau=8 slices, p=8
* ``plain_fp64_256``    256x256, N_t=512 in 32 slices, Jacobi-PCG rtol 1e-10
* ``diff_fp64_512``     512x512, N_t=1024 in 64 slices
* ``batch_fp32``        64 designs of seeded side and slice count, M=16
* ``large_2048``        2048x2048, N_t=2048 in 128 slices, smooth field
* ``large_law_512``     the large design's density law and solver at 512x512,
                        N_t=512 in 32 slices (small enough for the oracle)
* ``large_2048_512``    the large design at 2048x2048 with N_t=512 in 32 slices
                        (M=16 as in ``large_2048``; one oracle cycle fits the
                        host's memory)
* ``paper_100``         the paper's own test case (Sec. 5.1): 100x100 elements,
                        N_t=480, Table 1 materials (c-SIMP), q(t) of Eq. 5.1,
                        the Dirichlet patch at the centre tenth of the bottom
                        edge, p = 20; a seeded branched design stands in for
                        the paper's optimised design
"""
from __future__ import annotations

import numpy as np

# Physical parameters shared by every workload: SIMP conductivity
# k = kmin + (k0-kmin) rho^pk with (k0, kmin, pk) = (1, 1e-3, 3), uniform
# volumetric heat capacity c = 1, uniform source q = 1, t in [0, 1], T0 = 0,
# T = 0 on the centre tenth of the left edge, insulated elsewhere.
PHYSICS = dict(k0=1.0, kmin=1e-3, pk=3.0, c0=1.0, cmin=1.0, pc=1.0, q=1.0,
               t_final=1.0, p=8, bc="left_centre")

WORKLOADS = {
    "plain_fp64_32": dict(nx=32, ny=32, n_steps=64, n_slices=8, seed=0,
                          rtol=1e-10, precision="fp64"),
    "plain_fp64_256": dict(nx=256, ny=256, n_steps=512, n_slices=32, seed=1,
                           rtol=1e-10, precision="fp64"),
    "diff_fp64_512": dict(nx=512, ny=512, n_steps=1024, n_slices=64, seed=2,
                          rtol=1e-10, precision="fp64"),
    "large_2048": dict(nx=2048, ny=2048, n_steps=2048, n_slices=128, seed=4,
                       rtol=1e-10, precision="fp32_refine"),
    "large_law_512": dict(nx=512, ny=512, n_steps=512, n_slices=32, seed=4,
                          rtol=1e-10, precision="fp32_refine"),
    # the large design at its full grid with a quarter of its steps (same
    # M = 16): small enough for one oracle cycle in the test fixtures
    "large_2048_512": dict(nx=2048, ny=2048, n_steps=512, n_slices=32, seed=4,
                           rtol=1e-10, precision="fp32_refine"),
    # Table 1: k0 = 3, kmin = 0.03, c0 = 1, cmin = 0.5, pk = 3, pc = 2; p = 20
    "paper_100": dict(nx=100, ny=100, n_steps=480, n_slices=10, seed=5, rtol=1e-12,
                      precision="fp64", k0=3.0, kmin=0.03, pk=3.0, c0=1.0, cmin=0.5,
                      pc=2.0, p=20, bc="bottom_centre", q="paper"),
}


def heat_load_paper(n_steps: int, t_final: float = 1.0) -> np.ndarray:
    """q(t_n) = (1 - t)(1 + cos 50 t)/2 at t_n = n t_T / N_t, n = 0..N_t (Eq. 5.1)."""
    t = np.arange(n_steps + 1) * (t_final / n_steps)
    return 0.5 * (1.0 - t) * (1.0 + np.cos(50.0 * t))


def density_branches(nx: int, ny: int, seed: int, n_arms: int = 7) -> np.ndarray:
    """A branched conductor grown from the centre of the bottom edge, standing in
    for an optimised heat-conduction design: seeded straight arms from (0.5, 0)
    at angles spread over (10, 170) degrees, lengths U[0.45, 0.9], half-widths
    U[0.015, 0.04]; rho = 0.1 + 0.9 max_arms exp(-d^2 / (2 w^2)) at element
    centroids, d the distance to the arm."""
    rng = np.random.default_rng(seed)
    base = np.linspace(10.0, 170.0, n_arms)
    ang = np.deg2rad(base + rng.uniform(-8.0, 8.0, n_arms))
    length = rng.uniform(0.45, 0.9, n_arms)
    width = rng.uniform(0.015, 0.04, n_arms)
    xc = (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xc, yc)
    field = np.zeros((ny, nx))
    for k in range(n_arms):
        ux, uy = np.cos(ang[k]), np.sin(ang[k])
        s = np.clip((X - 0.5) * ux + Y * uy, 0.0, length[k])
        d2 = (X - 0.5 - s * ux) ** 2 + (Y - s * uy) ** 2
        field = np.maximum(field, np.exp(-d2 / (2 * width[k] ** 2)))
    return np.clip(0.1 + 0.9 * field, 0.0, 1.0).reshape(-1).astype(np.float64)


def density_uniform_noise(nx: int, ny: int, seed: int, base: float = 0.3,
                          amp: float = 0.1) -> np.ndarray:
    """rho = clip(base + U(-amp, amp), 0, 1) per element, element id ey*nx+ex."""
    rng = np.random.default_rng(seed)
    rho = base + rng.uniform(-amp, amp, size=nx * ny)
    return np.clip(rho, 0.0, 1.0).astype(np.float64)


def density_gaussians(nx: int, ny: int, seed: int, n_blobs: int = 32) -> np.ndarray:
    """Sum of seeded Gaussian bumps at element centroids, clipped to [0, 1].

    Centres U[0,1]^2, widths U[0.02, 0.08], amplitudes U[0.25, 1.0].
    """
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.0, 1.0, n_blobs)
    cy = rng.uniform(0.0, 1.0, n_blobs)
    sig = rng.uniform(0.02, 0.08, n_blobs)
    amp = rng.uniform(0.25, 1.0, n_blobs)
    xc = (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) / ny
    field = np.zeros((ny, nx))
    for b in range(n_blobs):
        gx = np.exp(-((xc - cx[b]) ** 2) / (2 * sig[b] ** 2))
        gy = np.exp(-((yc - cy[b]) ** 2) / (2 * sig[b] ** 2))
        field += amp[b] * np.outer(gy, gx)
    return np.clip(field, 0.0, 1.0).reshape(-1).astype(np.float64)


def design_schedule(nx: int, ny: int, seed: int, n_cycles: int, start=0.3,
                    step: float = 0.08, decay: float = 0.9, n_blobs: int = 12):
    """A seeded sequence of design fields chi_0 .. chi_{n-1} standing in for the
    iterates of an optimiser: chi_0 = start (a value everywhere, or an [N_e]
    field), chi_{i+1} = clip(chi_i + step decay^i b_i, 0, 1) with b_i a sum of
    seeded signed Gaussian bumps scaled to max |b_i| = 1."""
    rng = np.random.default_rng(seed)
    xc = (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) / ny
    chi = np.broadcast_to(np.asarray(start, dtype=np.float64), (nx * ny,)).copy()
    out = [chi.copy()]
    for i in range(n_cycles - 1):
        b = np.zeros((ny, nx))
        for _ in range(n_blobs):
            cx, cy = rng.uniform(0, 1, 2)
            sig = rng.uniform(0.05, 0.2)
            sgn = rng.choice([-1.0, 1.0])
            b += sgn * np.outer(np.exp(-(yc - cy) ** 2 / (2 * sig ** 2)),
                                np.exp(-(xc - cx) ** 2 / (2 * sig ** 2)))
        b /= np.abs(b).max()
        chi = np.clip(chi + step * decay ** i * b.reshape(-1), 0.0, 1.0)
        out.append(chi.copy())
    return out


def batch_designs(seed: int = 3, n_designs: int = 64):
    """The multi-design batch: per design a side, a slice count and a density."""
    ss = np.random.SeedSequence(seed)
    out = []
    for child in ss.spawn(n_designs):
        rng = np.random.default_rng(child)
        side = int(rng.choice([64, 128, 192, 256, 384, 512]))
        n_slices = int(rng.choice([16, 32, 64]))
        dseed = int(rng.integers(0, 2**31 - 1))
        out.append(dict(nx=side, ny=side, n_slices=n_slices,
                        n_steps=16 * n_slices,
                        rho=density_uniform_noise(side, side, dseed)))
    return out


def directions(n_elem: int, seed: int, count: int = 16) -> np.ndarray:
    """Unit random directions for finite-difference checks, shape (count, n_elem)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count, n_elem))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def workload(name: str) -> dict:
    """Full parameter dict of a named workload, physics included."""
    w = dict(PHYSICS)
    w.update(WORKLOADS[name])
    if isinstance(w["q"], str):
        w["q"] = heat_load_paper(w["n_steps"], w["t_final"])
    w["name"] = name
    return w


def workload_density(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    if name in ("large_2048", "large_law_512", "large_2048_512"):
        return density_gaussians(w["nx"], w["ny"], w["seed"])
    if name == "paper_100":
        return density_branches(w["nx"], w["ny"], w["seed"])
    return density_uniform_noise(w["nx"], w["ny"], w["seed"])
