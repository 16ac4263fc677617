"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/pt.h declares, and rejects invalid arguments before
anything is enqueued."""
import ctypes
import os
import re

import pytest

from paper_2411_19030_amd import _pt
from paper_2411_19030_amd._pt import Problem, PtProblem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_pt.LIB_PATH):
        pytest.fail("libpt.so is not built (run __graft_entry__.build())")
    return _pt.load_library()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(names) >= set(_pt.EXPORTS) - set()
    for n in names:
        assert hasattr(lib, n), n
        assert getattr(lib, n) is not None


def base(**kw):
    p = dict(nx=8, ny=8, n_steps=16, n_slices=4)
    p.update(kw)
    return Problem(**p)


@pytest.mark.parametrize("kw", [
    dict(pnorm=7), dict(pnorm=0), dict(n_slices=5), dict(nx=0), dict(ny=-1),
    dict(cg_rtol=0.0), dict(cg_rtol=float("nan")), dict(max_iter=0), dict(iterations=0),
    dict(t_final=0.0), dict(kmin=0.0), dict(pk=0.5), dict(precision=7), dict(precond=9),
    dict(storage=4), dict(n_steps=0), dict(q=float("inf")), dict(propagator=3),
    dict(propagator=-1), dict(coarse_iters=-1), dict(coarse_iters=5, precision=1),
    dict(coarse_iters=5, propagator=1), dict(coarse_iters=5, precond=1),
    # the coarse spatial mesh halves even grids
    dict(propagator=2, nx=9), dict(propagator=2, ny=7), dict(propagator=2, coarse_iters=5),
    # size limits: 16384 elements per side, 4000 slices
    dict(nx=16385), dict(ny=16385), dict(n_steps=8002, n_slices=4001), dict(pnorm=-2),
])
def test_validate_rejects(lib, kw):
    p = base(**kw)
    assert _pt.pt_validate(p) == _pt.PT_EINVAL
    assert _pt.pt_workspace_bytes(p) == 0


def test_validate_accepts_and_sizes(lib):
    p = base()
    assert _pt.pt_validate(p) == _pt.PT_OK
    assert _pt.pt_validate(base(propagator=_pt.PT_PLT)) == _pt.PT_OK
    assert _pt.pt_validate(base(propagator=_pt.PT_COARSE_MESH)) == _pt.PT_OK
    for kw in (dict(precision=1), dict(precond=1), dict(precision=1, precond=1), dict(storage=1)):
        assert _pt.pt_validate(base(propagator=_pt.PT_COARSE_MESH, **kw)) == _pt.PT_OK
    # the coarse mesh's arrays are part of the workspace
    assert (_pt.pt_workspace_bytes(base(propagator=_pt.PT_COARSE_MESH))
            > _pt.pt_workspace_bytes(base()))
    small = _pt.pt_workspace_bytes(p)
    big = _pt.pt_workspace_bytes(base(nx=64, ny=64))
    assert 0 < small < big
    # the largest accepted grid and slice count size without overflow
    edge = base(nx=16384, ny=16384, n_steps=8000, n_slices=4000)
    assert _pt.pt_validate(edge) == _pt.PT_OK
    nn = 16385 * 16385
    # at least the slice-boundary states of the previous and the corrected
    # iterate (two FP64 arrays of N_tau + 1 rows)
    assert _pt.pt_workspace_bytes(edge) > 2 * 8 * nn * 4001


def test_time_dependent_source_must_be_finite(lib):
    import numpy as np
    q = np.ones(17)
    assert _pt.pt_validate(base(q=q)) == _pt.PT_OK
    q[3] = np.nan
    assert _pt.pt_validate(base(q=q)) == _pt.PT_EINVAL


def _fwd(lib, p, rho=0x1000, gT=None, gth=None, S=0x2000, uT=None, uth=None, Th=0x3000,
         ws=0x10000000, nbytes=None):
    c = p.to_c()
    if nbytes is None:
        nbytes = lib.pt_workspace_bytes(ctypes.byref(c))
    return lib.pt_parareal_forward(ctypes.byref(c), rho, gT, gth, S, uT, uth, Th, ws, nbytes,
                                   None)


def test_forward_argument_errors_before_any_device_work(lib):
    p = base()
    assert _fwd(lib, p, rho=None) == _pt.PT_EINVAL
    assert _fwd(lib, p, S=None) == _pt.PT_EINVAL
    assert _fwd(lib, p, Th=None) == _pt.PT_EINVAL
    assert _fwd(lib, p, ws=None) == _pt.PT_EINVAL
    assert _fwd(lib, p, gT=0x5000, gth=None) == _pt.PT_EINVAL
    assert _fwd(lib, p, nbytes=16) == _pt.PT_ENOMEM
    # a guess that overlaps the S output is rejected
    assert _fwd(lib, p, gT=0x2000, gth=0x9000000) == _pt.PT_EINVAL
    assert _fwd(lib, base(pnorm=3)) == _pt.PT_EINVAL


def test_adjoint_and_sensitivity_argument_errors(lib):
    p = base()
    c = p.to_c()
    nb = lib.pt_workspace_bytes(ctypes.byref(c))
    assert lib.pt_parareal_adjoint(ctypes.byref(c), None, 0x2000, 0x3000, None, None,
                                   0x10000000, nb, None) == _pt.PT_EINVAL
    assert lib.pt_parareal_adjoint(ctypes.byref(c), 0x1000, 0x2000, 0x3000, None, None,
                                   0x10000000, 8, None) == _pt.PT_ENOMEM
    assert lib.pt_sensitivities(ctypes.byref(c), 0x1000, 0x10000000, nb, None,
                                None) == _pt.PT_EINVAL
    assert lib.pt_sensitivities(ctypes.byref(c), 0x1000, 0x10000000, 8, 0x4000,
                                None) == _pt.PT_ENOMEM


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert isinstance(lib.pt_strerror(code), bytes)


def test_struct_layout_matches_header():
    """Field order and offsets of the ctypes mirror follow pt.h (natural alignment)."""
    offs = {name: getattr(PtProblem, name).offset for name, _ in PtProblem._fields_}
    assert offs["nx"] == 0 and offs["ny"] == 4 and offs["k0"] == 8
    assert offs["q_t"] == 64 and offs["t_final"] == 72 and offs["n_steps"] == 80
    assert offs["cg_rtol"] == 96 and offs["max_iter"] == 104
    assert offs["dirichlet_mask"] == 128 and offs["propagator"] == 136
    assert offs["coarse_iters"] == 140 and offs["tuning"] == 144
    assert ctypes.sizeof(PtProblem) == 152


def test_tuning_layout_matches_header():
    """pt_tuning: natural alignment, doubles at 8-byte offsets."""
    T = _pt.PtTuning
    offs = {name: getattr(T, name).offset for name, _ in T._fields_}
    assert offs["wg_per_cu"] == 0 and offs["gk_weight"] == 32 and offs["lead_fine"] == 40
    assert offs["verify"] == 64 and offs["inner_rtol"] == 72 and offs["gmg_tail"] == 80
    assert offs["gmg_omega"] == 88 and offs["phase_timers"] == 96
    assert offs["wait_timeout_s"] == 104 and offs["gk_lag"] == 112 and ctypes.sizeof(T) == 120


def test_default_tuning_and_its_validation(lib):
    d = _pt.default_tuning()
    assert d["wg_per_cu"] == 1 and d["resident"] == -1 and d["verify"] == 1
    assert d["phase_timers"] == 0 and d["tile_max"] == 4096 and d["gk_weight"] == 4.0
    assert d["gk_lag"] == -1
    assert lib.pt_default_tuning(None) == _pt.PT_EINVAL
    assert lib.pt_validate(ctypes.byref(base(tuning=dict(resident=0)).to_c())) == _pt.PT_OK
    assert lib.pt_validate(ctypes.byref(base(tuning=dict(phase_timers=1)).to_c())) == _pt.PT_OK
    for bad in (dict(wg_per_cu=0), dict(resident=2), dict(resident_npt_max=9),
                dict(gk_weight=0.0), dict(tile_max=128), dict(ck_slots=0), dict(verify=2),
                dict(inner_rtol=1.0), dict(gmg_omega=float("nan")), dict(phase_timers=-1),
                dict(wait_timeout_s=-1.0), dict(cm_sweep_wgs=0), dict(gk_lag=-2)):
        c = base(tuning=bad).to_c()
        assert lib.pt_validate(ctypes.byref(c)) == _pt.PT_EINVAL, bad
        assert lib.pt_workspace_bytes(ctypes.byref(c)) == 0, bad
    with pytest.raises(ValueError):
        base(tuning=dict(no_such_field=1)).to_c()


def _batch(lib, probs, rho=None, grads=None, theta=0x3000, ws=0x10000000, nbytes=None,
           warm=0, tuning=None):
    arr = (PtProblem * len(probs))(*[p.to_c() for p in probs])
    n = len(probs)
    rho = rho if rho is not None else [0x1000 + 0x100 * k for k in range(n)]
    grads = grads if grads is not None else [0x8000 + 0x100 * k for k in range(n)]
    rp = (ctypes.c_void_p * n)(*rho)
    gp = (ctypes.c_void_p * n)(*grads)
    if nbytes is None:
        nbytes = lib.pt_batched_workspace_bytes(n, arr)
    t = ctypes.byref(tuning) if tuning is not None else None
    return lib.pt_parareal_batched(n, arr, rp, warm, t, theta, gp, ws, nbytes, None)


def _batch_fwd(lib, probs, ws=0x10000000, nbytes=None):
    arr = (PtProblem * len(probs))(*[p.to_c() for p in probs])
    n = len(probs)
    rp = (ctypes.c_void_p * n)(*[0x1000 + 0x100 * k for k in range(n)])
    if nbytes is None:
        nbytes = lib.pt_batched_workspace_bytes(n, arr)
    return lib.pt_parareal_batched(n, arr, rp, 0, None, 0x3000, None, ws, nbytes, None)


def test_batched_workspace_and_validation(lib):
    a, b = base(), base(nx=12, ny=6, n_steps=30, n_slices=5)
    arr = (PtProblem * 2)(a.to_c(), b.to_c())
    one = (PtProblem * 1)(a.to_c())
    nb2 = lib.pt_batched_workspace_bytes(2, arr)
    nb1 = lib.pt_batched_workspace_bytes(1, one)
    assert nb2 > nb1 > 0
    # mixed precision, several Parareal iterations, zero or coarse-mesh coarse
    # propagators, invalid members: no workspace
    for bad in (base(precision=1), base(iterations=2), base(pnorm=3), base(propagator=1),
                base(propagator=2), base(coarse_iters=4)):
        arr_bad = (PtProblem * 2)(a.to_c(), bad.to_c())
        assert lib.pt_batched_workspace_bytes(2, arr_bad) == 0
    assert lib.pt_batched_workspace_bytes(0, arr) == 0


def test_batched_argument_errors_before_any_device_work(lib):
    a, b = base(), base(nx=12, ny=6, n_steps=30, n_slices=5)
    assert _batch(lib, [a, b], rho=[0x1000, None]) == _pt.PT_EINVAL
    assert _batch(lib, [a, b], grads=[None, 0x9000]) == _pt.PT_EINVAL
    # no gradient array at all: a forward-only call (still checked on the host)
    assert _batch_fwd(lib, [a, b], ws=None) == _pt.PT_EINVAL
    assert _batch_fwd(lib, [a, b], nbytes=64) == _pt.PT_ENOMEM
    assert _batch(lib, [a, b], theta=None) == _pt.PT_EINVAL
    assert _batch(lib, [a, b], ws=None) == _pt.PT_EINVAL
    assert _batch(lib, [a, b], warm=2) == _pt.PT_EINVAL
    assert _batch(lib, [a, b], nbytes=64) == _pt.PT_ENOMEM
    assert _batch(lib, [a, base(iterations=3)]) == _pt.PT_EINVAL
    # Theta output inside the workspace
    assert _batch(lib, [a, b], theta=0x10000000 + 256) == _pt.PT_EINVAL
    bad = _pt.PtBatchTuning.from_dict(dict(fine_wgs=0, sweep_wgs=16, sweep_groups=2))
    assert _batch(lib, [a, b], tuning=bad) == _pt.PT_EINVAL
    bad = _pt.PtBatchTuning.from_dict(dict(fine_wgs=2, sweep_wgs=16, sweep_groups=1,
                                           resident=3))
    assert _batch(lib, [a, b], tuning=bad) == _pt.PT_EINVAL


def test_batch_default_tuning(lib):
    t = _pt.PtBatchTuning()
    assert lib.pt_batch_default_tuning(64, ctypes.byref(t)) == _pt.PT_OK
    assert t.fine_wgs >= 1 and t.sweep_wgs >= 1 and 1 <= t.sweep_groups <= 64
    assert lib.pt_batch_default_tuning(0, ctypes.byref(t)) == _pt.PT_EINVAL


def test_batch_tuning_layout():
    assert ctypes.sizeof(_pt.PtBatchTuning) == 32


def test_state_bytes_store_all_and_checkpoint(lib):
    p = base(nx=8, ny=6, n_steps=24, n_slices=4)
    nn = 9 * 7
    assert _pt.pt_state_bytes(p) == 24 * nn * 8
    assert _pt.pt_state_bytes(base(nx=8, ny=6, n_steps=24, n_slices=4, storage=1)) == 8 * nn * 8
    assert _pt.pt_state_bytes(base(pnorm=3)) == 0
    # multigrid and checkpoint settings are valid single-design problems
    assert _pt.pt_validate(base(precond=1, storage=1)) == _pt.PT_OK
    # a batch accepts only store-all designs
    arr = (PtProblem * 2)(base().to_c(), base(storage=1).to_c())
    assert lib.pt_batched_workspace_bytes(2, arr) == 0


@pytest.mark.parametrize("kw", [dict(nx=0), dict(ny=-3), dict(r_fil=0.0), dict(r_fil=float("nan")),
                                dict(eta=1.5), dict(eta=-0.1), dict(beta=float("inf")),
                                dict(nx=4096, ny=4096, r_fil=0.1)])
def test_filter_validate_rejects(lib, kw):
    a = dict(nx=16, ny=16, r_fil=0.1, beta=8.0, eta=0.5)
    a.update(kw)
    f = _pt.make_filter(**a)
    assert _pt.pt_filter_validate(f) == _pt.PT_EINVAL
    assert lib.pt_filter_projection(ctypes.byref(f), 0x1000, None, 0x2000000, None) == _pt.PT_EINVAL


def test_filter_argument_errors_before_any_device_work(lib):
    f = _pt.make_filter(16, 16, 0.1, 8.0, 0.5)
    assert _pt.pt_filter_validate(f) == _pt.PT_OK
    n = 16 * 16 * 8
    # missing arrays, overlapping arrays
    assert lib.pt_filter_projection(ctypes.byref(f), None, None, 0x100000, None) == _pt.PT_EINVAL
    assert lib.pt_filter_projection(ctypes.byref(f), 0x100000, None, 0x100000 + n // 2,
                                    None) == _pt.PT_EINVAL
    assert lib.pt_filter_projection_backward(ctypes.byref(f), 0x100000, 0x200000, None, 0x300000,
                                             None) == _pt.PT_EINVAL
    assert lib.pt_filter_projection_backward(ctypes.byref(f), 0x100000, 0x200000, 0x300000,
                                             0x300000 + 8, None) == _pt.PT_EINVAL



def test_cycle_noalloc_host_errors(lib):
    """pt_cycle_noalloc rejects an invalid problem and one whose workspace
    exceeds the static array before touching the device."""
    fake = ctypes.c_void_p(16)
    args = [fake, None, None, None, fake, None, None, None, fake, fake, None, None]
    bad = base(pnorm=7).to_c()
    assert lib.pt_cycle_noalloc(ctypes.byref(bad), *args) == _pt.PT_EINVAL
    big = base(nx=256, ny=256, n_steps=512, n_slices=32)
    assert _pt.pt_workspace_bytes(big) > _pt.PT_NOALLOC_WS_BYTES
    c = big.to_c()
    assert lib.pt_cycle_noalloc(ctypes.byref(c), *args) == _pt.PT_ESIZE
    assert b"static" in lib.pt_strerror(_pt.PT_ESIZE)


def test_binding_rejects_unusable_tensors(lib):
    """The Python binding refuses tensors the kernels would misread (a float32
    density, a CPU pointer, a wrong size, a strided view) with ValueError,
    before anything reaches the library."""
    import torch
    f64 = torch.float64
    p = base()
    Ne, Nn, Nt1 = p.n_elem, p.n_nodes, p.n_slices + 1
    rows = _pt.pt_state_bytes(p) // (8 * Nn)
    rho = torch.full((Ne,), 0.3, dtype=f64)
    S = torch.zeros(rows, Nn, dtype=f64)
    U = torch.zeros(Nt1, Nn, dtype=f64)
    th = torch.zeros(Nt1, dtype=f64)
    Th = torch.zeros((), dtype=f64)
    g = torch.zeros(Ne, dtype=f64)
    ws = torch.zeros(64, dtype=torch.uint8)

    def fwd(r=rho, gT=None, gth=None, S_=S):
        _pt.pt_parareal_forward(p, r, gT, gth, S_, U, th, Th, ws)

    with pytest.raises(ValueError, match="dtype torch.float32"):
        fwd(r=rho.float())
    with pytest.raises(ValueError, match="elements"):
        fwd(r=torch.zeros(Ne + 1, dtype=f64))
    with pytest.raises(ValueError, match="elements"):
        fwd(gT=torch.zeros(Nt1 - 1, Nn, dtype=f64), gth=th)
    with pytest.raises(ValueError, match="contiguous"):
        fwd(r=torch.zeros(2 * Ne, dtype=f64)[::2])
    with pytest.raises(ValueError, match="elements"):
        fwd(S_=torch.zeros(rows - 1, Nn, dtype=f64))
    # right dtype, layout and sizes, but host memory
    with pytest.raises(ValueError, match="GPU tensor"):
        fwd()
    with pytest.raises(ValueError, match="elements"):
        _pt.pt_parareal_adjoint(p, rho, S, Th, torch.zeros(Nn, dtype=f64), U, ws)
    with pytest.raises(ValueError, match="float32"):
        _pt.pt_sensitivities(p, rho, ws, g.float())
    with pytest.raises(ValueError, match="GPU tensor"):
        _pt.pt_sensitivities(p, rho, ws, g)
    with pytest.raises(ValueError, match="elements"):
        _pt.pt_cycle_noalloc(p, rho, None, None, None, S, U, th, U, Th, torch.zeros(3, dtype=f64))
    with pytest.raises(ValueError, match="densities"):
        _pt.pt_parareal_batched([p, p], [rho], False, None, torch.zeros(2, dtype=f64), [g, g], ws)
    with pytest.raises(ValueError, match="dTheta_drho\\[1\\]"):
        _pt.pt_parareal_batched([p, p], [rho, rho], False, None, torch.zeros(2, dtype=f64),
                                [g, g.float()], ws)
    flt = _pt.make_filter(8, 8, 0.2, 8.0, 0.5)
    with pytest.raises(ValueError, match="elements"):
        _pt.pt_filter_projection(flt, rho, None, torch.zeros(Ne - 1, dtype=f64))
