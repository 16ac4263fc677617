"""Write sampled oracle outputs of a full-size workload to a text fixture.

Run from the repository root:

    python tests/golden/make_oracle_samples.py diff_fp64_512

It calls only the oracle (``oracle/``) on the seeded density of ``workloads``:
one cold cycle with one Parareal iteration (coarse sweeps as the guess,
Sec. 5.2; the modified primal and reversed adjoint passes of Sec. 4.4). The
fixture keeps Theta, every theta_{Mn}, the 2-norm and sum of dTheta/drho, and
the values of S, u_T, lambda and dTheta/drho at seeded sample indices. The
GPU parity test at full size compares the HIP path against these samples.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from workloads import PHYSICS, workload, workload_density  # noqa: E402

N_SAMPLES = 1024


def sample_indices(seed: int, shape: tuple, count: int) -> np.ndarray:
    """Seeded flat indices into an array of the given shape (with repetition removed)."""
    rng = np.random.default_rng(seed)
    size = int(np.prod(shape))
    idx = np.unique(rng.integers(0, size, count))
    return idx


def checkpoint_rows(n_steps: int, n_slices: int) -> np.ndarray:
    """Rows of S[N_t][N_n] holding T_{Mn} (n = 1..N_tau) and T_{Mn+1} (n = 0..N_tau-1):
    the states that checkpointed storage keeps."""
    M = n_steps // n_slices
    return np.concatenate([np.arange(M - 1, n_steps, M), np.arange(0, n_steps, M)])


def sample_rows(seed: int, rows: np.ndarray, n_cols: int, count: int) -> np.ndarray:
    """Seeded flat indices into S[N_t][n_cols] restricted to the given rows."""
    rng = np.random.default_rng(seed)
    r = rows[rng.integers(0, rows.size, count)]
    c = rng.integers(0, n_cols, count)
    return np.unique(r.astype(np.int64) * n_cols + c)


# Workloads whose GPU runs keep only the checkpointed states: their S samples
# are drawn from those rows.
CHECKPOINTED = ("large_2048_512",)


def main(name: str) -> str:
    w = workload(name)
    rho = workload_density(name)
    prob = O.Problem(nx=w["nx"], ny=w["ny"], n_steps=w["n_steps"], n_slices=w["n_slices"],
                     p=PHYSICS["p"], k0=w["k0"], kmin=w["kmin"], pk=w["pk"], c0=w["c0"],
                     cmin=w["cmin"], pc=w["pc"], q=w["q"], t_final=w["t_final"], bc=w["bc"])
    t0 = time.time()
    d = O.Discretisation(prob, rho)
    fw = O.parareal_forward(d, 1)
    ad = O.parareal_adjoint(d, fw["S"], fw["Theta"], 1)
    elapsed = time.time() - t0
    S, uT, lam, grad = fw["S"], fw["uT"], ad["lam"], ad["grad"]
    lines = [
        f"# Oracle samples of workload {name}: cold cycle, one Parareal iteration,",
        f"# nx={w['nx']} ny={w['ny']} N_t={w['n_steps']} N_tau={w['n_slices']} p={PHYSICS['p']},",
        f"# density workloads.workload_density('{name}'). Written by",
        "# tests/golden/make_oracle_samples.py (oracle only, FP64 direct solves);",
        f"# oracle time {elapsed:.1f} s. Index lines give flat indices into the",
        "# row-major arrays S[N_t][N_n], uT[N_tau+1][N_n], lam[N_tau+1][N_n], grad[N_e].",
        f"Theta {fw['Theta']!r}",
        "utheta " + " ".join(repr(float(x)) for x in fw["utheta"]),
        f"grad_norm {float(np.linalg.norm(grad))!r}",
        f"grad_sum {float(np.sum(grad))!r}",
    ]
    for key, arr, seed in (("S", S, 11), ("uT", uT, 12), ("lam", lam, 13), ("grad", grad, 14)):
        a = np.asarray(arr, dtype=np.float64)
        if key == "S" and name in CHECKPOINTED:
            idx = sample_rows(seed, checkpoint_rows(w["n_steps"], w["n_slices"]), a.shape[1],
                              N_SAMPLES)
        else:
            idx = sample_indices(seed, a.shape, N_SAMPLES)
        flat = a.reshape(-1)
        lines.append(f"{key}_idx " + " ".join(str(int(i)) for i in idx))
        lines.append(f"{key}_val " + " ".join(repr(float(flat[i])) for i in idx))
        lines.append(f"{key}_absmax {float(np.abs(a).max())!r}")
    path = os.path.join(HERE, f"oracle_{name}.txt")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path


def load(path: str) -> dict:
    """Parse a fixture written by main()."""
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            if key.endswith("_idx"):
                out[key] = np.array([int(v) for v in vals], dtype=np.int64)
            elif len(vals) == 1 and key not in ("utheta",):
                out[key] = float(vals[0])
            else:
                out[key] = np.array([float(v) for v in vals], dtype=np.float64)
    return out


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["diff_fp64_512"]:
        print(main(nm), flush=True)
