"""ctypes binding of libpt (include/pt.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; this module converts
torch device tensors to pointers and a Python problem description to the C
struct. It raises if the library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpt.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EHIP, PT_ENOCONV, PT_EDOMAIN, PT_ESTATE, PT_ESIZE = (
    0, -1, -2, -3, -4, -5, -6, -7)
# bytes of the static per-GPU workspace of pt_cycle_noalloc (PT_NOALLOC_WS_BYTES)
PT_NOALLOC_WS_BYTES = 64 << 20
PT_BC = {"left_centre": 0, "bottom_centre": 1, "none": 2, "mask": 3}
PT_FP64, PT_FP32_REFINE = 0, 1
PT_JACOBI, PT_GMG = 0, 1
PT_STORE_ALL, PT_CHECKPOINT = 0, 1
PT_PARAREAL, PT_PLT, PT_COARSE_MESH = 0, 1, 2

EXPORTS = ["pt_workspace_bytes", "pt_state_bytes", "pt_validate", "pt_default_tuning",
           "pt_parareal_forward", "pt_parareal_adjoint",
           "pt_sensitivities", "pt_query_status", "pt_query_trace", "pt_strerror",
           "pt_batched_workspace_bytes", "pt_batch_default_tuning", "pt_parareal_batched",
           "pt_batched_status", "pt_autotune_batched", "pt_filter_validate",
           "pt_filter_projection", "pt_filter_projection_backward", "pt_cycle_noalloc"]


class PtTuning(ctypes.Structure):
    """Mirror of pt_tuning (execution settings; defaults from pt_default_tuning)."""
    _fields_ = [
        ("wg_per_cu", ctypes.c_int32), ("resident", ctypes.c_int32),
        ("resident_npt_max", ctypes.c_int32), ("sweep_wgs", ctypes.c_int32),
        ("cm_sweep_wgs", ctypes.c_int32), ("fine_wgs", ctypes.c_int32),
        ("fine_groups", ctypes.c_int32), ("gk_groups", ctypes.c_int32),
        ("gk_weight", ctypes.c_double), ("lead_fine", ctypes.c_int32),
        ("shared_queue", ctypes.c_int32), ("tile_max", ctypes.c_int32),
        ("ck_slots", ctypes.c_int32), ("extrap", ctypes.c_int32),
        ("sweep_x0", ctypes.c_int32), ("verify", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double), ("gmg_tail", ctypes.c_int32),
        ("gmg_sweeps", ctypes.c_int32), ("gmg_omega", ctypes.c_double),
        ("phase_timers", ctypes.c_int32),
        ("wait_timeout_s", ctypes.c_double), ("gk_lag", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def default_tuning() -> dict:
    """The library's default execution settings as a dict."""
    t = PtTuning()
    _check(load_library().pt_default_tuning(ctypes.byref(t)), "pt_default_tuning")
    return t.as_dict()


class PtProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("k0", ctypes.c_double), ("kmin", ctypes.c_double), ("pk", ctypes.c_double),
        ("c0", ctypes.c_double), ("cmin", ctypes.c_double), ("pc", ctypes.c_double),
        ("q", ctypes.c_double), ("q_t", ctypes.POINTER(ctypes.c_double)),
        ("t_final", ctypes.c_double),
        ("n_steps", ctypes.c_int32), ("n_slices", ctypes.c_int32),
        ("pnorm", ctypes.c_int32), ("iterations", ctypes.c_int32),
        ("cg_rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("precond", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("dirichlet_mask", ctypes.POINTER(ctypes.c_uint8)),
        ("propagator", ctypes.c_int32), ("coarse_iters", ctypes.c_int32),
        ("tuning", ctypes.POINTER(PtTuning)),
    ]


class PtStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("max_cg_iters", ctypes.c_int32),
        ("cg_iters_fine", ctypes.c_int64), ("cg_iters_coarse", ctypes.c_int64),
        ("solves_fine", ctypes.c_int64), ("solves_coarse", ctypes.c_int64),
        ("max_rel_residual", ctypes.c_double),
    ]


class PtBatchTuning(ctypes.Structure):
    _fields_ = [
        ("fine_wgs", ctypes.c_int32), ("sweep_wgs", ctypes.c_int32),
        ("sweep_groups", ctypes.c_int32), ("resident", ctypes.c_int32),
        ("grid", ctypes.c_int32), ("tile_max", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]
    KEYS = ("fine_wgs", "sweep_wgs", "sweep_groups", "resident", "grid", "tile_max")

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in self.KEYS}

    @staticmethod
    def from_dict(d: dict) -> "PtBatchTuning":
        t = PtBatchTuning()
        for k in PtBatchTuning.KEYS:
            setattr(t, k, int(d.get(k, 0)))
        return t


class PtFilter(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("r_fil", ctypes.c_double),
                ("beta", ctypes.c_double), ("eta", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpt.so; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpt.so not found at {path}: build it with "
                           "`python -m paper_2411_19030_amd.build`")
    # torch first: libpt.so then binds to the HIP runtime torch has loaded, the
    # one that owns the tensors and streams passed in. Opened before torch, it
    # would pull in the system runtime beside torch's bundled one, and its
    # launches would fail on torch's pointers and streams.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(PtProblem)
    vp = ctypes.c_void_p
    lib.pt_workspace_bytes.argtypes = [P]
    lib.pt_workspace_bytes.restype = ctypes.c_size_t
    lib.pt_validate.argtypes = [P]
    lib.pt_validate.restype = ctypes.c_int
    lib.pt_state_bytes.argtypes = [P]
    lib.pt_state_bytes.restype = ctypes.c_size_t
    lib.pt_default_tuning.argtypes = [ctypes.POINTER(PtTuning)]
    lib.pt_default_tuning.restype = ctypes.c_int
    lib.pt_parareal_forward.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pt_parareal_forward.restype = ctypes.c_int
    lib.pt_parareal_adjoint.argtypes = [P, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pt_parareal_adjoint.restype = ctypes.c_int
    lib.pt_sensitivities.argtypes = [P, vp, vp, ctypes.c_size_t, vp, vp]
    lib.pt_sensitivities.restype = ctypes.c_int
    lib.pt_query_status.argtypes = [vp, vp, ctypes.POINTER(PtStats)]
    lib.pt_query_status.restype = ctypes.c_int
    lib.pt_query_trace.argtypes = [P, vp, vp, ctypes.POINTER(ctypes.c_ulonglong), ctypes.c_size_t,
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.pt_query_trace.restype = ctypes.c_int
    lib.pt_strerror.argtypes = [ctypes.c_int]
    lib.pt_strerror.restype = ctypes.c_char_p
    TP = ctypes.POINTER(PtBatchTuning)
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.pt_batched_workspace_bytes.argtypes = [ctypes.c_int, P]
    lib.pt_batched_workspace_bytes.restype = ctypes.c_size_t
    lib.pt_batch_default_tuning.argtypes = [ctypes.c_int, TP]
    lib.pt_batch_default_tuning.restype = ctypes.c_int
    lib.pt_parareal_batched.argtypes = [ctypes.c_int, P, pp, ctypes.c_int, TP, vp, pp, vp,
                                        ctypes.c_size_t, vp]
    lib.pt_parareal_batched.restype = ctypes.c_int
    lib.pt_batched_status.argtypes = [ctypes.c_int, P, vp, vp, ctypes.POINTER(PtStats)]
    lib.pt_batched_status.restype = ctypes.c_int
    lib.pt_autotune_batched.argtypes = [ctypes.c_int, P, pp, vp, pp, vp, ctypes.c_size_t, vp, TP,
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), AUTOTUNE_PROGRESS, vp]
    lib.pt_autotune_batched.restype = ctypes.c_int
    FP = ctypes.POINTER(PtFilter)
    lib.pt_filter_validate.argtypes = [FP]
    lib.pt_filter_validate.restype = ctypes.c_int
    lib.pt_filter_projection.argtypes = [FP, vp, vp, vp, vp]
    lib.pt_filter_projection.restype = ctypes.c_int
    lib.pt_filter_projection_backward.argtypes = [FP, vp, vp, vp, vp, vp]
    lib.pt_filter_projection_backward.restype = ctypes.c_int
    lib.pt_cycle_noalloc.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pt_cycle_noalloc.restype = ctypes.c_int
    _lib = lib
    return lib


class PtError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load_library().pt_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


@dataclass
class Problem:
    """Python mirror of pt_problem (field meanings in include/pt.h)."""
    nx: int
    ny: int
    n_steps: int
    n_slices: int
    pnorm: int = 8
    k0: float = 1.0
    kmin: float = 1e-3
    pk: float = 3.0
    c0: float = 1.0
    cmin: float = 1.0
    pc: float = 1.0
    q: object = 1.0           # float, or array of q(t_n), n = 0..n_steps
    t_final: float = 1.0
    iterations: int = 1
    cg_rtol: float = 1e-10
    max_iter: int = 10000
    precision: int = PT_FP64
    precond: int = PT_JACOBI
    storage: int = PT_STORE_ALL
    bc: object = "left_centre"  # name or boolean/uint8 node mask
    propagator: int = PT_PARAREAL  # PT_PARAREAL, PT_PLT or PT_COARSE_MESH
    coarse_iters: int = 0       # > 0: coarse steps are this many CG iterations
    tuning: Optional[dict] = None  # execution settings over the defaults (pt_tuning fields)
    _keep: list = field(default_factory=list, repr=False, compare=False)

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny

    def to_c(self) -> PtProblem:
        c = PtProblem()
        c.nx, c.ny = int(self.nx), int(self.ny)
        c.k0, c.kmin, c.pk = float(self.k0), float(self.kmin), float(self.pk)
        c.c0, c.cmin, c.pc = float(self.c0), float(self.cmin), float(self.pc)
        self._keep.clear()
        if np.isscalar(self.q):
            c.q = float(self.q)
            c.q_t = ctypes.POINTER(ctypes.c_double)()
        else:
            qa = np.ascontiguousarray(self.q, dtype=np.float64)
            self._keep.append(qa)
            c.q = float("nan")
            c.q_t = qa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        c.t_final = float(self.t_final)
        c.n_steps, c.n_slices = int(self.n_steps), int(self.n_slices)
        c.pnorm, c.iterations = int(self.pnorm), int(self.iterations)
        c.cg_rtol, c.max_iter = float(self.cg_rtol), int(self.max_iter)
        c.precision, c.precond, c.storage = int(self.precision), int(self.precond), int(self.storage)
        if isinstance(self.bc, str):
            c.bc = PT_BC[self.bc]
            c.dirichlet_mask = ctypes.POINTER(ctypes.c_uint8)()
        else:
            m = np.ascontiguousarray(np.asarray(self.bc).astype(np.uint8))
            self._keep.append(m)
            c.bc = PT_BC["mask"]
            c.dirichlet_mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        c.propagator = int(self.propagator)
        c.coarse_iters = int(self.coarse_iters)
        if self.tuning:
            t = PtTuning()
            _check(load_library().pt_default_tuning(ctypes.byref(t)), "pt_default_tuning")
            names = {k for k, _ in PtTuning._fields_}
            for k, v in self.tuning.items():
                if k not in names:
                    raise ValueError(f"unknown tuning field {k!r}")
                setattr(t, k, v)
            self._keep.append(t)
            c.tuning = ctypes.pointer(t)
        else:
            c.tuning = ctypes.POINTER(PtTuning)()
        return c


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream)


def _check(rc: int, where: str):
    if rc != PT_OK:
        raise PtError(rc, where)


def _check_tensors(where: str, specs, raw=()):
    """Raise ValueError unless every given tensor can be handed to the library.

    specs: (tensor or None, name, numel) with numel None for "any size";
    None tensors (optional arguments) are skipped. Each tensor must be a
    contiguous torch.float64 tensor of exactly numel elements; `raw` lists
    (tensor or None, name) byte buffers such as the workspace, of any dtype
    and contiguous. All of them must live on one GPU. Dtype, layout and size
    are checked for every argument before devices."""
    import torch
    present = []
    for t, name, numel in specs:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{where}: {name} must be a torch tensor, got {type(t).__name__}")
        if t.dtype != torch.float64:
            raise ValueError(f"{where}: {name} has dtype {t.dtype}, expected torch.float64")
        if not t.is_contiguous():
            raise ValueError(f"{where}: {name} is not contiguous")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"{where}: {name} has {t.numel()} elements, expected {numel}")
        present.append((t, name))
    for t, name in raw:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or not t.is_contiguous():
            raise ValueError(f"{where}: {name} must be a contiguous torch tensor")
        present.append((t, name))
    dev = None
    for t, name in present:
        if not t.is_cuda:
            raise ValueError(f"{where}: {name} is on {t.device}, expected a GPU tensor")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{where}: {name} is on {t.device}, the other arguments on {dev}")


def _sizes(prob: "Problem") -> dict:
    """Element counts of the arrays of one problem (include/pt.h)."""
    Nn, Nt1 = prob.n_nodes, prob.n_slices + 1
    return dict(Ne=prob.n_elem, U=Nt1 * Nn, th=Nt1, S=pt_state_bytes(prob) // 8)


def pt_validate(prob: Problem) -> int:
    return load_library().pt_validate(ctypes.byref(prob.to_c()))


def pt_workspace_bytes(prob: Problem) -> int:
    return int(load_library().pt_workspace_bytes(ctypes.byref(prob.to_c())))


def pt_state_bytes(prob: Problem) -> int:
    return int(load_library().pt_state_bytes(ctypes.byref(prob.to_c())))


def pt_parareal_forward(prob: Problem, rho, guess_T, guess_theta, S, uT_out, utheta_out,
                        Theta_out, ws, stream=None, check: bool = True) -> int:
    z = _sizes(prob)
    _check_tensors("pt_parareal_forward", [
        (rho, "rho", z["Ne"]), (guess_T, "guess_T", z["U"]), (guess_theta, "guess_theta", z["th"]),
        (S, "S", z["S"]), (uT_out, "uT_out", z["U"]), (utheta_out, "utheta_out", z["th"]),
        (Theta_out, "Theta_out", 1)], [(ws, "ws")])
    c = prob.to_c()
    rc = load_library().pt_parareal_forward(
        ctypes.byref(c), _ptr(rho), _ptr(guess_T), _ptr(guess_theta), _ptr(S), _ptr(uT_out),
        _ptr(utheta_out), _ptr(Theta_out), _ptr(ws), ws.numel() * ws.element_size(),
        _stream(stream))
    if check:
        _check(rc, "pt_parareal_forward")
    return rc


def pt_parareal_adjoint(prob: Problem, rho, S, Theta, guess_lambda, lambda_out, ws,
                        stream=None, check: bool = True) -> int:
    z = _sizes(prob)
    _check_tensors("pt_parareal_adjoint", [
        (rho, "rho", z["Ne"]), (S, "S", z["S"]), (Theta, "Theta", 1),
        (guess_lambda, "guess_lambda", z["U"]), (lambda_out, "lambda_out", z["U"])],
                   [(ws, "ws")])
    c = prob.to_c()
    rc = load_library().pt_parareal_adjoint(
        ctypes.byref(c), _ptr(rho), _ptr(S), _ptr(Theta), _ptr(guess_lambda), _ptr(lambda_out),
        _ptr(ws), ws.numel() * ws.element_size(), _stream(stream))
    if check:
        _check(rc, "pt_parareal_adjoint")
    return rc


def pt_sensitivities(prob: Problem, rho, ws, dTheta_drho, stream=None, check: bool = True) -> int:
    z = _sizes(prob)
    _check_tensors("pt_sensitivities", [(rho, "rho", z["Ne"]),
                                        (dTheta_drho, "dTheta_drho", z["Ne"])],
                   [(ws, "ws")])
    c = prob.to_c()
    rc = load_library().pt_sensitivities(
        ctypes.byref(c), _ptr(rho), _ptr(ws), ws.numel() * ws.element_size(), _ptr(dTheta_drho),
        _stream(stream))
    if check:
        _check(rc, "pt_sensitivities")
    return rc


def pt_cycle_noalloc(prob: Problem, rho, guess_T, guess_theta, guess_lambda, S, uT_out,
                     utheta_out, lambda_out, Theta_out, dTheta_drho, stats_out=None,
                     stream=None, check: bool = True) -> int:
    """One whole cycle on the library's static workspace (no allocation);
    stats_out: optional device tensor of at least sizeof(pt_stats) bytes."""
    z = _sizes(prob)
    _check_tensors("pt_cycle_noalloc", [
        (rho, "rho", z["Ne"]), (guess_T, "guess_T", z["U"]), (guess_theta, "guess_theta", z["th"]),
        (guess_lambda, "guess_lambda", z["U"]), (S, "S", z["S"]), (uT_out, "uT_out", z["U"]),
        (utheta_out, "utheta_out", z["th"]), (lambda_out, "lambda_out", z["U"]),
        (Theta_out, "Theta_out", 1), (dTheta_drho, "dTheta_drho", z["Ne"])],
                   [(stats_out, "stats_out")])
    if stats_out is not None and stats_out.numel() * stats_out.element_size() < ctypes.sizeof(PtStats):
        raise ValueError("pt_cycle_noalloc: stats_out is smaller than pt_stats")
    c = prob.to_c()
    rc = load_library().pt_cycle_noalloc(
        ctypes.byref(c), _ptr(rho), _ptr(guess_T), _ptr(guess_theta), _ptr(guess_lambda),
        _ptr(S), _ptr(uT_out), _ptr(utheta_out), _ptr(lambda_out), _ptr(Theta_out),
        _ptr(dTheta_drho), _ptr(stats_out), _stream(stream))
    if check:
        _check(rc, "pt_cycle_noalloc")
    return rc


def stats_from_bytes(raw: bytes) -> dict:
    """A pt_stats read back from device memory (e.g. stats_out of pt_cycle_noalloc)."""
    st = PtStats.from_buffer_copy(raw[:ctypes.sizeof(PtStats)])
    return {k: getattr(st, k) for k, _ in PtStats._fields_}


LANE_KINDS = ["F_PRI", "GK_PRI", "SWEEP_PRI", "COLD_PRI", "F_ADJ", "GK_ADJ", "SWEEP_ADJ",
              "COLD_ADJ", "CM_GK_PRI", "CM_SWEEP_PRI", "CM_GK_ADJ", "CM_SWEEP_ADJ"]


def pt_query_trace(prob: Problem, ws, stream=None) -> list:
    """Per-lane records of the last engine launch: dicts with kind, slice,
    nwg, tile, rounds, iters and step end times in microseconds from the
    earliest lane start."""
    c = prob.to_c()
    words = 1 << 22
    buf = (ctypes.c_ulonglong * words)()
    nl, st = ctypes.c_int(), ctypes.c_int()
    _check(load_library().pt_query_trace(ctypes.byref(c), _ptr(ws), _stream(stream), buf, words,
                                         ctypes.byref(nl), ctypes.byref(st)), "pt_query_trace")
    arr = np.frombuffer(buf, dtype=np.uint64, count=nl.value * st.value).reshape(nl.value,
                                                                                 st.value)
    recs = [r for r in arr if r[6] != 0]
    hdr = 12
    if not recs:
        return []
    t0 = min(int(r[6]) for r in recs)
    out = []
    for r in recs:
        steps = [(int(x) - t0) / 100.0 for x in r[hdr:] if x != 0]
        out.append(dict(kind=LANE_KINDS[int(r[0])], slice=int(r[1]), nwg=int(r[2]),
                        tile=int(r[3]), rounds=int(r[4]), iters=int(r[5]),
                        start_us=(int(r[6]) - t0) / 100.0, step_end_us=steps,
                        work_us=int(r[7]) / 100.0, barrier_us=int(r[8]) / 100.0,
                        reduce_us=int(r[9]) / 100.0, flag_us=int(r[10]) / 100.0))
    return out


def pt_query_status(ws, stream=None) -> dict:
    st = PtStats()
    _check(load_library().pt_query_status(_ptr(ws), _stream(stream), ctypes.byref(st)),
           "pt_query_status")
    return {k: getattr(st, k) for k, _ in PtStats._fields_}


# ---------------------------------------------------------------------------
# Multi-design cycles
# ---------------------------------------------------------------------------

def _probs_array(probs):
    arr = (PtProblem * len(probs))()
    for k, p in enumerate(probs):
        arr[k] = p.to_c()
    return arr


def _ptr_array(tensors):
    return (ctypes.c_void_p * len(tensors))(*[_ptr(t) for t in tensors])


def _check_batch(where, probs, rhos, Theta_out, grads, ws):
    """grads None: a forward-only call (no gradient outputs)."""
    n = len(probs)
    if len(rhos) != n or (grads is not None and len(grads) != n):
        raise ValueError(f"{where}: {n} problems, {len(rhos)} densities, "
                         f"{None if grads is None else len(grads)} gradients")
    specs = [(Theta_out, "Theta_out", n)]
    for k, p in enumerate(probs):
        specs += [(rhos[k], f"rho[{k}]", p.n_elem)]
        if grads is not None:
            specs += [(grads[k], f"dTheta_drho[{k}]", p.n_elem)]
    _check_tensors(where, specs, [(ws, "ws")])


def pt_batched_workspace_bytes(probs) -> int:
    arr = _probs_array(probs)
    return int(load_library().pt_batched_workspace_bytes(len(probs), arr))


def pt_batch_default_tuning(n: int) -> dict:
    t = PtBatchTuning()
    _check(load_library().pt_batch_default_tuning(n, ctypes.byref(t)), "pt_batch_default_tuning")
    return t.as_dict()


def pt_parareal_batched(probs, rhos, warm: bool, tuning: Optional[dict], Theta_out, grads, ws,
                        stream=None, check: bool = True) -> int:
    """grads None: the primal pass only (Theta_out)."""
    _check_batch("pt_parareal_batched", probs, rhos, Theta_out, grads, ws)
    arr = _probs_array(probs)
    t = PtBatchTuning.from_dict(tuning) if tuning is not None else None
    rc = load_library().pt_parareal_batched(
        len(probs), arr, _ptr_array(rhos), 1 if warm else 0,
        ctypes.byref(t) if t is not None else None, _ptr(Theta_out),
        _ptr_array(grads) if grads is not None else None,
        _ptr(ws), ws.numel() * ws.element_size(), _stream(stream))
    if check:
        _check(rc, "pt_parareal_batched")
    return rc


def pt_batched_status(probs, ws, stream=None) -> list:
    arr = _probs_array(probs)
    st = (PtStats * len(probs))()
    _check(load_library().pt_batched_status(len(probs), arr, _ptr(ws), _stream(stream), st),
           "pt_batched_status")
    return [{k: getattr(s, k) for k, _ in PtStats._fields_} for s in st]


AUTOTUNE_PROGRESS = ctypes.CFUNCTYPE(None, ctypes.POINTER(PtBatchTuning), ctypes.c_double,
                                     ctypes.c_void_p)


def pt_autotune_batched(probs, rhos, Theta_out, grads, ws, stream=None, progress=None) -> tuple:
    """(best shape, its ms, the built-in shape's ms), timed from one state.
    progress(shape dict, ms) is called after each shape is timed."""
    _check_batch("pt_autotune_batched", probs, rhos, Theta_out, grads, ws)
    arr = _probs_array(probs)
    t = PtBatchTuning()
    ms, ms0 = ctypes.c_double(), ctypes.c_double()
    cb = AUTOTUNE_PROGRESS(lambda shape, v, _: progress(shape.contents.as_dict(), v)) \
        if progress is not None else AUTOTUNE_PROGRESS()
    _check(load_library().pt_autotune_batched(
        len(probs), arr, _ptr_array(rhos), _ptr(Theta_out), _ptr_array(grads), _ptr(ws),
        ws.numel() * ws.element_size(), _stream(stream), ctypes.byref(t), ctypes.byref(ms),
        ctypes.byref(ms0), cb, None), "pt_autotune_batched")
    return t.as_dict(), ms.value, ms0.value


# ---------------------------------------------------------------------------
# Design-field front end (filter and projection)
# ---------------------------------------------------------------------------

def make_filter(nx: int, ny: int, r_fil: float, beta: float, eta: float) -> PtFilter:
    f = PtFilter()
    f.nx, f.ny = int(nx), int(ny)
    f.r_fil, f.beta, f.eta = float(r_fil), float(beta), float(eta)
    return f


def pt_filter_validate(f: PtFilter) -> int:
    return load_library().pt_filter_validate(ctypes.byref(f))


def pt_filter_projection(f: PtFilter, chi, chi_fil, chi_phys, stream=None):
    ne = f.nx * f.ny
    _check_tensors("pt_filter_projection", [(chi, "chi", ne), (chi_fil, "chi_fil", ne),
                                            (chi_phys, "chi_phys", ne)])
    _check(load_library().pt_filter_projection(ctypes.byref(f), _ptr(chi), _ptr(chi_fil),
                                               _ptr(chi_phys), _stream(stream)),
           "pt_filter_projection")


def pt_filter_projection_backward(f: PtFilter, chi_fil, grad_phys, work, grad_chi, stream=None):
    ne = f.nx * f.ny
    _check_tensors("pt_filter_projection_backward", [
        (chi_fil, "chi_fil", ne), (grad_phys, "grad_phys", ne), (work, "work", ne),
        (grad_chi, "grad_chi", ne)])
    _check(load_library().pt_filter_projection_backward(
        ctypes.byref(f), _ptr(chi_fil), _ptr(grad_phys), _ptr(work), _ptr(grad_chi),
        _stream(stream)), "pt_filter_projection_backward")
