// Host side of libpt: argument checks, workspace layout, lane planning and the
// stream-ordered launches of the single-design calls (forward / adjoint /
// sensitivities) and of the multi-design cycle.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/pt.h"
#include "pt_engine.hip"

using namespace pt;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxGrid = 1024;         // workgroups of one engine launch
constexpr int kMaxBatchGroups = 512;   // worker groups of a multi-design launch
constexpr long long kGmgLdsBytes = 158 * 1024;  // dynamic LDS of the multigrid lanes

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

pt_tuning default_settings() {
    pt_tuning t;
    memset(&t, 0, sizeof(t));
    t.wg_per_cu = 1;
    t.resident = -1;
    t.resident_npt_max = 8;
    t.sweep_wgs = 0;
    t.cm_sweep_wgs = 24;
    t.fine_wgs = 0;
    t.fine_groups = 0;
    t.gk_groups = 0;
    t.gk_weight = 4.0;
    t.lead_fine = 1;
    t.shared_queue = 1;
    t.tile_max = 4096;
    t.ck_slots = 24;
    t.extrap = 0;
    t.sweep_x0 = 1;
    t.verify = 1;
    t.inner_rtol = 1e-5;
    t.gmg_tail = 4096;
    t.gmg_sweeps = 16;
    t.gmg_omega = 1.3;
    t.phase_timers = 0;
    t.wait_timeout_s = 0.0;
    t.gk_lag = -1;
    return t;
}

// The problem's execution settings (its own, or the defaults).
pt_tuning tuning_of(const pt_problem *p) { return p->tuning ? *p->tuning : default_settings(); }

bool bool01(int v) { return v == 0 || v == 1; }

bool valid_settings(const pt_tuning &t) {
    return t.wg_per_cu >= 1 && t.wg_per_cu <= 4 && t.resident >= -1 && t.resident <= 1 &&
           t.resident_npt_max >= 1 && t.resident_npt_max <= 8 && t.sweep_wgs >= 0 &&
           t.sweep_wgs <= kMaxGroup && t.cm_sweep_wgs >= 1 && t.cm_sweep_wgs <= kMaxGroup &&
           t.fine_wgs >= 0 && t.fine_wgs <= kMaxGroup && t.fine_groups >= 0 &&
           t.gk_groups >= 0 && t.gk_weight > 0.0 && isfinite(t.gk_weight) &&
           bool01(t.lead_fine) && bool01(t.shared_queue) && t.tile_max >= 256 &&
           t.ck_slots >= 1 && bool01(t.extrap) && bool01(t.sweep_x0) && bool01(t.verify) &&
           t.inner_rtol > 0.0 && t.inner_rtol < 1.0 && t.gmg_tail >= 0 && t.gmg_sweeps >= 1 &&
           t.gmg_sweeps <= 1000 && t.gmg_omega > 0.0 && isfinite(t.gmg_omega) &&
           bool01(t.phase_timers) && t.wait_timeout_s >= 0.0 &&
           isfinite(t.wait_timeout_s) && t.gk_lag >= -1 && t.gk_lag <= 4096;
}


struct Carver {
    size_t o = 0;
    size_t take(size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    }
};

bool valid_problem(const pt_problem *p) {
    if (!p) return false;
    if (p->nx < 1 || p->ny < 1 || p->nx > 16384 || p->ny > 16384) return false;
    if ((long long)(p->nx + 1) * (p->ny + 1) > (1ll << 30)) return false;
    if (p->n_steps < 1 || p->n_slices < 1 || p->n_steps % p->n_slices) return false;
    if (p->n_slices > 4000) return false;
    if (p->pnorm < 2 || (p->pnorm % 2)) return false;
    if (p->iterations < 1) return false;
    if (!(p->cg_rtol > 0.0) || !isfinite(p->cg_rtol)) return false;
    if (p->max_iter < 1) return false;
    if (!(p->t_final > 0.0) || !isfinite(p->t_final)) return false;
    if (!isfinite(p->k0) || !isfinite(p->kmin) || !isfinite(p->pk)) return false;
    if (!isfinite(p->c0) || !isfinite(p->cmin) || !isfinite(p->pc)) return false;
    if (!(p->kmin > 0.0) || !(p->k0 > 0.0) || !(p->cmin > 0.0) || !(p->c0 > 0.0)) return false;
    if (p->pk < 1.0 || p->pc < 1.0) return false;
    if (!p->q_t && !isfinite(p->q)) return false;
    if ((p->precision != PT_FP64 && p->precision != PT_FP32_REFINE) ||
        (p->precond != PT_JACOBI && p->precond != PT_GMG) ||
        (p->storage != PT_STORE_ALL && p->storage != PT_CHECKPOINT))
        return false;
    if (p->bc < 0 || p->bc > 3) return false;
    if (p->bc == PT_BC_MASK && !p->dirichlet_mask) return false;
    if (p->propagator != PT_PARAREAL && p->propagator != PT_PLT &&
        p->propagator != PT_COARSE_MESH)
        return false;
    // the fine lanes may use any precision, preconditioner and storage (the
    // coarse solves are FP64 Jacobi PCG on the nx/2 x ny/2 mesh)
    if (p->propagator == PT_COARSE_MESH && ((p->nx % 2) || (p->ny % 2) || p->coarse_iters != 0))
        return false;
    if (p->coarse_iters < 0 || p->coarse_iters > 100000) return false;
    if (p->tuning && !valid_settings(*p->tuning)) return false;
    if (p->coarse_iters > 0 &&
        (p->precision != PT_FP64 || p->propagator != PT_PARAREAL || p->precond != PT_JACOBI))
        return false;
    if (p->q_t)
        for (int n = 0; n <= p->n_steps; ++n)
            if (!isfinite(p->q_t[n])) return false;
    return true;
}

// ---------------------------------------------------------------------------
// Multigrid hierarchy
// ---------------------------------------------------------------------------

// Levels of the vertex-centred hierarchy: halve both sides while they stay
// even and the coarse grid keeps at least 2 elements per side.
struct Hierarchy {
    int L = 1;
    long long off[kMaxLevels] = {0};
    long long nodes = 0;  // nodes of levels 1..L-1
};

Hierarchy hierarchy(const pt_problem *p) {
    Hierarchy h;
    if (p->precond != PT_GMG) return h;
    int nx = p->nx, ny = p->ny;
    while (h.L < kMaxLevels && nx % 2 == 0 && ny % 2 == 0 && nx >= 4 && ny >= 4) {
        nx /= 2;
        ny /= 2;
        h.off[h.L] = h.nodes;
        h.nodes += (long long)(nx + 1) * (ny + 1);
        ++h.L;
    }
    return h;
}

// Checkpointed storage: fine adjoint lanes run on at most ck_slots groups,
// each with scratch for the M-2 states its slice recomputes.
int ck_slots(const pt_problem *p) {
    return std::max(1, std::min(p->n_slices, tuning_of(p).ck_slots));
}

size_t state_rows(const pt_problem *p) {
    return p->storage == PT_CHECKPOINT ? 2 * (size_t)p->n_slices : (size_t)p->n_steps;
}

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------

// Arrays of one design.
struct DesignLayout {
    size_t ctl, FL, kq, cm, dk, dc, dinv_f, dinv_c, mask, qt, zero;
    size_t gA64, gA, gA0, gmg_g, gmg_w, ck;
    size_t ck_stride;
    size_t Gk, Gn, Gk_th, Gn_th, F_th, Uprev, Uprev_th, Ubuf, Ubuf_th, acc, accG;
    // coarse-mesh propagators (PT_COARSE_MESH)
    size_t cm_kE, cm_cE, cm_A9, cm_C9, cm_dinv, cm_fc, cm_Gk, cm_Gn;
    // multi-design cycles keep the cycle's state here
    size_t S, uT, uth, lam, gT, gth, gL;
};

void carve_design(Carver &c, const pt_problem *p, DesignLayout &L, bool batched) {
    const size_t Nn = (size_t)(p->nx + 1) * (p->ny + 1);
    const size_t Ne = (size_t)p->nx * p->ny;
    const size_t EP = (size_t)(p->nx + 2) * (p->ny + 2);
    const size_t Nt1 = (size_t)p->n_slices + 1;
    const size_t d = sizeof(double);
    L.ctl = c.take(sizeof(Control));
    L.FL = c.take(d * Nt1 * Nn);
    L.kq = c.take(d * EP);
    L.cm = c.take(d * EP);
    L.dk = c.take(d * Ne);
    L.dc = c.take(d * Ne);
    L.dinv_f = c.take(d * Nn);
    L.dinv_c = c.take(d * Nn);
    L.mask = c.take(Nn);
    L.qt = c.take(d * (p->n_steps + 1));
    L.zero = c.take(d * Nn);
    L.Gk = c.take(d * Nt1 * Nn);
    L.Gn = c.take(d * Nt1 * Nn);
    L.Gk_th = c.take(d * Nt1);
    L.Gn_th = c.take(d * Nt1);
    L.F_th = c.take(d * Nt1);
    L.acc = c.take(d * (size_t)p->n_slices * Ne);
    L.accG = c.take(d * Ne);
    const Hierarchy h = hierarchy(p);
    L.gA64 = c.take(d * 2 * 9 * (size_t)h.nodes + d);
    L.gA = c.take(d * 2 * 9 * (size_t)h.nodes + d);
    L.gA0 = c.take(p->precond == PT_GMG ? d * 2 * 9 * Nn : d);
    L.gmg_g = c.take(d * 2 * kMaxLevels);
    L.gmg_w = c.take(d * 2 * kMaxLevels);
    const int M = p->n_steps / p->n_slices;
    L.ck_stride = p->storage == PT_CHECKPOINT ? (size_t)std::max(M - 2, 0) * Nn : 0;
    L.ck = c.take(d * (size_t)ck_slots(p) * L.ck_stride + d);
    if (p->propagator == PT_COARSE_MESH) {
        const size_t Nc = (size_t)(p->nx / 2 + 1) * (p->ny / 2 + 1);
        const size_t Nec = (size_t)(p->nx / 2) * (p->ny / 2);
        L.cm_kE = c.take(d * Nec);
        L.cm_cE = c.take(d * Nec);
        L.cm_A9 = c.take(d * 9 * Nc);
        L.cm_C9 = c.take(d * 9 * Nc);
        L.cm_dinv = c.take(d * Nc);
        L.cm_fc = c.take(d * Nc);
        L.cm_Gk = c.take(d * Nt1 * Nc);
        L.cm_Gn = c.take(d * Nt1 * Nc);
    }
    if (!batched) {
        L.Uprev = c.take(d * Nt1 * Nn);
        L.Uprev_th = c.take(d * Nt1);
        L.Ubuf = c.take(d * Nt1 * Nn);
        L.Ubuf_th = c.take(d * Nt1);
    } else {
        L.S = c.take(d * (size_t)p->n_steps * Nn);
        L.uT = c.take(d * Nt1 * Nn);
        L.uth = c.take(d * Nt1);
        L.lam = c.take(d * Nt1 * Nn);
        L.gT = c.take(d * Nt1 * Nn);
        L.gth = c.take(d * Nt1);
        L.gL = c.take(d * Nt1 * Nn);
    }
}

// Launch-wide arrays of an engine launch.
struct SharedLayout {
    size_t desc, bar, flags, partials, wg_group, groups, lanes, qhead, qslot, pool, trace, xch;
    size_t gvec, gvec_stride;
    int max_lanes, max_groups, trace_stride, xch_stride;
    size_t pool_stride;
};

void carve_shared(Carver &c, SharedLayout &S, int n_designs, int max_lanes, int max_groups,
                  size_t pool_stride, int trace_stride, int xch_stride, size_t gmg_nodes) {
    S.max_lanes = max_lanes;
    S.max_groups = max_groups;
    S.trace_stride = trace_stride;
    S.xch_stride = xch_stride;
    S.pool_stride = pool_stride;
    S.desc = c.take(sizeof(EngineDesc) * n_designs);
    S.bar = c.take(sizeof(unsigned) * kMaxGroups * kBarStride);
    S.flags = c.take(sizeof(unsigned) * kMaxFlags * (size_t)n_designs);
    S.partials = c.take(sizeof(double) * (size_t)max_groups * 2 * kMaxGroup * 4);
    S.wg_group = c.take(sizeof(int) * kMaxGrid);
    S.groups = c.take(sizeof(Group) * kMaxGroups);
    S.lanes = c.take(sizeof(Lane) * (size_t)max_lanes);
    S.qhead = c.take(sizeof(unsigned) * 2);
    S.qslot = c.take(sizeof(int) * kMaxGroups);
    S.pool = c.take(sizeof(double) * (size_t)max_groups * kVecsPerLane * pool_stride);
    S.trace = c.take(sizeof(unsigned long long) * (size_t)max_lanes * trace_stride);
    S.xch = c.take(sizeof(double) * (size_t)kMaxGrid * 12 * xch_stride);
    // multigrid level vectors r, u_a, u_b of levels >= 1 per group
    S.gvec_stride = 3 * gmg_nodes;
    S.gvec = c.take(sizeof(double) * (size_t)max_groups * S.gvec_stride + sizeof(double));
}

// Groups a single-design launch may use: one per lane at most, and no more
// than keep the per-group CG vectors within about 16 GB.
int max_groups_of(const pt_problem *p) {
    const double nn = (double)(p->nx + 1) * (p->ny + 1);
    const int by_memory = (int)std::max(32.0, 16e9 / (kVecsPerLane * 8.0 * nn));
    return std::min(2 * p->n_slices + 2, std::min(by_memory, kMaxGroups));
}

int trace_stride_of(const pt_problem *p) {
    return TR_HDR + std::max(p->n_steps / p->n_slices, p->n_slices);
}

// Single-design workspace: the design's status block comes first (offset 0).
struct Layout {
    DesignLayout d;
    SharedLayout s;
    size_t total;
};

Layout layout(const pt_problem *p) {
    Layout L{};
    Carver c;
    carve_design(c, p, L.d, false);
    const int max_lanes = 2 * p->n_slices + 2;
    carve_shared(c, L.s, 1, max_lanes, max_groups_of(p), (size_t)(p->nx + 1) * (p->ny + 1),
                 trace_stride_of(p), p->nx + 2, (size_t)hierarchy(p).nodes);
    L.total = c.o;
    return L;
}

// Multi-design workspace.
struct BatchLayout {
    std::vector<DesignLayout> d;
    SharedLayout s;
    size_t total;
    size_t max_nn;
};

BatchLayout batch_layout(int n, const pt_problem *probs) {
    BatchLayout L{};
    L.d.resize(n);
    Carver c;
    int lanes = 0, tstride = TR_HDR, xs = 2;
    size_t max_nn = 1, max_gn = 0;
    for (int k = 0; k < n; ++k) {
        carve_design(c, &probs[k], L.d[k], true);
        max_gn = std::max(max_gn, (size_t)hierarchy(&probs[k]).nodes);
        lanes += 2 * probs[k].n_slices + 2;
        tstride = std::max(tstride, trace_stride_of(&probs[k]));
        xs = std::max(xs, probs[k].nx + 2);
        max_nn = std::max(max_nn, (size_t)(probs[k].nx + 1) * (probs[k].ny + 1));
    }
    carve_shared(c, L.s, n, lanes, kMaxBatchGroups, max_nn, tstride, xs, max_gn);
    L.max_nn = max_nn;
    L.total = c.o;
    return L;
}

Consts make_consts(const pt_problem *p) {
    Consts C{};
    C.nx = p->nx;
    C.ny = p->ny;
    C.W = p->nx + 1;
    C.Nn = (p->nx + 1) * (p->ny + 1);
    C.Ne = p->nx * p->ny;
    C.EW = p->nx + 2;
    C.Nt = p->n_steps;
    C.Ntau = p->n_slices;
    C.M = p->n_steps / p->n_slices;
    C.p = p->pnorm;
    C.max_iter = p->max_iter;
    const pt_tuning T = tuning_of(p);
    C.verify = T.verify;
    C.extrap = T.extrap;
    C.fp32 = p->precision == PT_FP32_REFINE ? 1 : 0;
    C.max_restarts = 40;
    C.inner_rtol = T.inner_rtol;
    C.hx = 1.0 / p->nx;
    C.hy = 1.0 / p->ny;
    const double rx = C.hy / C.hx, ry = C.hx / C.hy;
    C.e_self = 2.0 * (rx + ry);
    C.e_x = ry - 2.0 * rx;
    C.e_y = rx - 2.0 * ry;
    C.e_d = -(rx + ry);
    C.cm_unit = C.hx * C.hy / 36.0;
    C.quarter_area = C.hx * C.hy / 4.0;
    C.dt = p->t_final / p->n_steps;
    C.dtau = p->t_final / p->n_slices;
    C.inv_dt = 1.0 / C.dt;
    C.inv_dtau = 1.0 / C.dtau;
    C.rtol = p->cg_rtol;
    C.inv_NtNe = 1.0 / ((double)p->n_steps * (double)C.Ne);
    C.inv_NtauNe = 1.0 / ((double)p->n_slices * (double)C.Ne);
    C.inv_p = 1.0 / p->pnorm;
    // a device wait gives up after this many seconds (100 MHz realtime clock)
    const double tmo = T.wait_timeout_s > 0.0 ? T.wait_timeout_s : 20.0;
    C.timeout_ticks = (long long)(tmo * 1e8);
    C.k0 = p->k0;
    C.kmin = p->kmin;
    C.pk = p->pk;
    C.c0 = p->c0;
    C.cmin = p->cmin;
    C.pc = p->pc;
    C.q = p->q;
    C.bc_rule = p->bc;
    C.has_qt = p->q_t ? 1 : 0;
    const Hierarchy h = hierarchy(p);
    C.gmg = p->precond == PT_GMG ? 1 : 0;
    C.gmg_L = h.L;
    for (int l = 0; l < kMaxLevels; ++l) C.gmg_off[l] = h.off[l];
    C.gmg_nodes = h.nodes;
    // levels with more nodes than this are smoothed by the whole group
    const long long tail = T.gmg_tail;
    C.gmg_Lg = 0;
    for (int l = 0; l < h.L; ++l)
        if ((long long)((p->nx >> l) + 1) * ((p->ny >> l) + 1) > tail) C.gmg_Lg = l + 1;
    // an odd count leaves the coarsest solution in the second buffer
    C.gmg_tail_sweeps = 2 * T.gmg_sweeps + 1;
    C.gmg_omega = T.gmg_omega;
    C.ckpt = p->storage == PT_CHECKPOINT ? 1 : 0;
    C.sweep_x0 = T.sweep_x0;
    C.plt = p->propagator == PT_PLT ? 1 : 0;
    C.coarse_iters = p->coarse_iters;
    if (C.gmg || C.ckpt) C.extrap = 0;
    // LDS-staged chunks of the multigrid rounds (one operand window in the CG
    // precision) and of the FP64 set-up of a solve (two windows), within the
    // 160 KB of LDS less the engine's static share
    {
        const long long avail = kGmgLdsBytes;
        const long long halo = 2ll * (C.W + 1);
        const long long rsz = C.fp32 ? 4 : 8;
        long long ch = std::min(16384ll, avail / rsz - halo);
        long long chi = std::min(8192ll, (avail / 8 - 2 * halo) / 2);
        C.gmg_chunk = (int)std::max(0ll, ch / 256 * 256);
        C.gmg_chunk_init = (int)std::max(0ll, chi / 256 * 256);
    }
    return C;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

Bufs make_bufs(void *ws, const DesignLayout &L, const SharedLayout &S, int design) {
    Bufs B{};
    B.ctl = at<Control>(ws, L.ctl);
    B.flags = at<unsigned>(ws, S.flags) + (size_t)design * kMaxFlags;
    B.pool = at<double>(ws, S.pool);
    B.pool_stride = S.pool_stride;
    B.FL = at<double>(ws, L.FL);
    B.kq = at<double>(ws, L.kq);
    B.cm = at<double>(ws, L.cm);
    B.dk = at<double>(ws, L.dk);
    B.dc = at<double>(ws, L.dc);
    B.dinv_f = at<double>(ws, L.dinv_f);
    B.dinv_c = at<double>(ws, L.dinv_c);
    B.mask = at<unsigned char>(ws, L.mask);
    B.qt = at<double>(ws, L.qt);
    B.zero = at<double>(ws, L.zero);
    B.Gk = at<double>(ws, L.Gk);
    B.Gn = at<double>(ws, L.Gn);
    B.Gk_th = at<double>(ws, L.Gk_th);
    B.Gn_th = at<double>(ws, L.Gn_th);
    B.F_th = at<double>(ws, L.F_th);
    B.acc = at<double>(ws, L.acc);
    B.accG = at<double>(ws, L.accG);
    B.gA64 = at<double>(ws, L.gA64);
    B.gA = at<void>(ws, L.gA);
    B.gA0 = at<void>(ws, L.gA0);
    B.gmg_g = at<double>(ws, L.gmg_g);
    B.gmg_w = at<double>(ws, L.gmg_w);
    B.gvec = at<void>(ws, S.gvec);
    B.gvec_stride = S.gvec_stride;
    B.ck = at<double>(ws, L.ck);
    B.ck_stride = L.ck_stride;
    return B;
}

CoarseMesh make_coarse_mesh(void *ws, const DesignLayout &L, const pt_problem *p) {
    CoarseMesh M{};
    M.nxc = p->nx / 2;
    M.nyc = p->ny / 2;
    M.Wc = M.nxc + 1;
    M.Nc = M.Wc * (M.nyc + 1);
    M.Nec = M.nxc * M.nyc;
    M.kE = at<double>(ws, L.cm_kE);
    M.cE = at<double>(ws, L.cm_cE);
    M.A9 = at<double>(ws, L.cm_A9);
    M.C9 = at<double>(ws, L.cm_C9);
    M.dinv = at<double>(ws, L.cm_dinv);
    M.fc = at<double>(ws, L.cm_fc);
    M.Gk = at<double>(ws, L.cm_Gk);
    M.Gn = at<double>(ws, L.cm_Gn);
    return M;
}

Launch make_launch(void *ws, const SharedLayout &S, Control *ctl0, long long timeout_ticks) {
    Launch X{};
    X.wg_group = at<int>(ws, S.wg_group);
    X.groups = at<Group>(ws, S.groups);
    X.lanes = at<Lane>(ws, S.lanes);
    X.bar = at<unsigned>(ws, S.bar);
    X.partials = at<double>(ws, S.partials);
    X.xch = at<double>(ws, S.xch);
    X.xch_stride = S.xch_stride;
    X.qhead = at<unsigned>(ws, S.qhead);
    X.qslot = at<int>(ws, S.qslot);
    X.trace = at<unsigned long long>(ws, S.trace);
    X.trace_stride = S.trace_stride;
    X.ctl0 = ctl0;
    X.timeout_ticks = timeout_ticks;
    return X;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? PT_OK : PT_EHIP; }

#define PT_TRY(expr)                         \
    do {                                     \
        int _rc = (expr);                    \
        if (_rc != PT_OK) return _rc;        \
    } while (0)

int launch_check() { return hip_ok(hipGetLastError()); }

bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

// Writes host descriptors to device memory with by-value kernel arguments (so
// the upload is stream-ordered and can be captured in a graph).
int upload_descs(const std::vector<EngineDesc> &hd, EngineDesc *dst, hipStream_t stream) {
    for (size_t k = 0; k < hd.size(); k += kDescPerCopy) {
        DescChunk ch;
        memset(&ch, 0, sizeof(ch));
        const int m = (int)std::min<size_t>(kDescPerCopy, hd.size() - k);
        for (int q = 0; q < m; ++q) ch.d[q] = hd[k + q];
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(256), 0, stream, ch, m, dst + k);
        PT_TRY(launch_check());
    }
    return PT_OK;
}

// Per-design host copies (caller mask, q(t)), then material and diagonals of
// every design of D. Host copies cannot be captured in a graph.
int setup_designs(int n, const pt_problem *probs, const std::vector<EngineDesc> &hd,
                  EngineDesc *D, int keep_markers, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset_ctl, dim3(n), dim3(64), 0, stream, D, keep_markers);
    PT_TRY(launch_check());
    bool copied = false;
    for (int k = 0; k < n; ++k) {
        const pt_problem *p = &probs[k];
        if (p->bc == PT_BC_MASK || p->q_t) {
            if (capturing(stream)) return PT_EINVAL;
            copied = true;
        }
        if (p->bc == PT_BC_MASK)
            PT_TRY(hip_ok(hipMemcpyAsync(hd[k].B.mask, p->dirichlet_mask, (size_t)hd[k].C.Nn,
                                         hipMemcpyHostToDevice, stream)));
        if (p->q_t)
            PT_TRY(hip_ok(hipMemcpyAsync(hd[k].B.qt, p->q_t, sizeof(double) * (p->n_steps + 1),
                                         hipMemcpyHostToDevice, stream)));
    }
    // the caller's host arrays may be released once the call returns
    if (copied) PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    hipLaunchKernelGGL(k_setup_design, dim3(256, n), dim3(256), 0, stream, D);
    hipLaunchKernelGGL(k_diag, dim3(256, n), dim3(256), 0, stream, D);
    int maxL = 1;
    for (const auto &E : hd)
        if (E.C.gmg) maxL = std::max(maxL, E.C.gmg_L);
    if (maxL > 1 || std::any_of(hd.begin(), hd.end(), [](const EngineDesc &E) { return E.C.gmg; })) {
        hipLaunchKernelGGL(k_gmg_reset, dim3(n), dim3(64), 0, stream, D);
        hipLaunchKernelGGL(k_gmg_level0, dim3(256, n), dim3(256), 0, stream, D);
        for (int l = 0; l + 1 < maxL; ++l)
            hipLaunchKernelGGL(k_gmg_rap, dim3(256, n), dim3(128), 0, stream, D, l);
        hipLaunchKernelGGL(k_gmg_omega, dim3(n), dim3(64), 0, stream, D);
    }
    return launch_check();
}

struct Device {
    int cus = 0;
    int lds_max = 0;
};

int device_info(Device &d) {
    int dev = 0;
    PT_TRY(hip_ok(hipGetDevice(&dev)));
    PT_TRY(hip_ok(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev)));
    PT_TRY(hip_ok(hipDeviceGetAttribute(&d.lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)));
    return PT_OK;
}


// LDS doubles of the engine for tile size ts: two node windows (ts + 2H) and
// two element windows ((ts-1)/W + 3 rows of nx+2 elements).
size_t engine_lds_doubles(int ts, int W) {
    const size_t H = W + 1;
    return 2 * ((size_t)ts + 2 * H) + 2 * ((size_t)(ts - 1) / W + 3) * (W + 1);
}

// LDS of a multigrid lane: the larger of the round window and the two set-up windows.
size_t gmg_lds_bytes(const Consts &C) {
    const size_t halo = 2 * (size_t)(C.W + 1);
    const size_t rsz = C.fp32 ? 4 : 8;
    return std::max((C.gmg_chunk + halo) * rsz, 2 * (C.gmg_chunk_init + halo) * 8);
}

int lds_cap_doubles(const Device &dev) {
    return (std::min(dev.lds_max, 160 * 1024) - 1024) / 8;
}

// Streaming-mode tile: the group's share of the nodes, cut to what fits LDS
// and to tile_max (0: the built-in 4096).
int tile_for(int Nn, int nwg, int H, int cap_doubles, int tile_max) {
    int ts = (Nn + nwg - 1) / nwg;
    ts = (ts + 255) / 256 * 256;
    while (ts > 256 && engine_lds_doubles(ts, H - 1) > (size_t)cap_doubles) ts -= 256;
    ts = std::min(ts, std::max(256, tile_max > 0 ? tile_max : 4096));
    ts = std::max(ts, 256);
    return ts;
}

const void *engine_kernel(bool fp32, int npt, bool multi, bool cmesh = false, bool timed = false) {
    if (timed)  // FP64 single-design launches without coarse-mesh lanes; resident: 8 nodes
        return npt == 0 ? (const void *)k_engine<0, double, false, false, true>
                        : (const void *)k_engine<8, double, false, false, true>;
    if (cmesh) {
        // coarse-mesh launches: resident lanes always take the 8-node form
        if (fp32) return npt == 0 ? (const void *)k_engine<0, float, false, true>
                                  : (const void *)k_engine<8, float, false, true>;
        return npt == 0 ? (const void *)k_engine<0, double, false, true>
                        : (const void *)k_engine<8, double, false, true>;
    }
    if (multi) {
        if (fp32) return npt == 0 ? (const void *)k_engine<0, float, true>
                                  : (const void *)k_engine<8, float, true>;
        return npt == 0 ? (const void *)k_engine<0, double, true>
                        : (const void *)k_engine<8, double, true>;
    }
    if (fp32)
        return npt == 0   ? (const void *)k_engine<0, float, false>
               : npt == 1 ? (const void *)k_engine<1, float, false>
               : npt == 2 ? (const void *)k_engine<2, float, false>
               : npt == 4 ? (const void *)k_engine<4, float, false>
                          : (const void *)k_engine<8, float, false>;
    return npt == 0   ? (const void *)k_engine<0, double, false>
           : npt == 1 ? (const void *)k_engine<1, double, false>
           : npt == 2 ? (const void *)k_engine<2, double, false>
           : npt == 4 ? (const void *)k_engine<4, double, false>
                      : (const void *)k_engine<8, double, false>;
}

// Workgroups of the engine that fit on the device at once.
int engine_capacity(bool fp32, int npt, bool multi, size_t lds_bytes, const Device &dev,
                    int &cap, bool cmesh = false, bool timed = false) {
    const void *kern = engine_kernel(fp32, npt, multi, cmesh, timed);
    PT_TRY(hip_ok(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds_bytes)));
    int occ = 0;
    PT_TRY(hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kThreads, lds_bytes)));
    cap = occ * dev.cus;
    return PT_OK;
}

// One persistent launch of the engine. Every workgroup must be resident at
// once (groups spin on each other): the grid is checked against the
// occupancy bound, and the launch is cooperative unless the stream is being
// captured into a graph, where a plain launch of the same checked grid is used.
static_assert(sizeof(EngineDesc) + sizeof(Launch) + sizeof(void *) <= 4096,
              "engine kernel arguments exceed the kernel argument segment");

// single: the descriptor of a single-design launch (passed by value), or
// nullptr for a multi-design launch that reads D.
int launch_engine(bool fp32, int npt, const EngineDesc *D, const EngineDesc *single,
                  const Launch &X, int grid, size_t lds_bytes, const Device &dev,
                  hipStream_t stream, bool cmesh = false, bool timed = false) {
    const bool multi = single == nullptr;
    int cap = 0;
    PT_TRY(engine_capacity(fp32, npt, multi, lds_bytes, dev, cap, cmesh, timed));
    if (cap < grid || grid > kMaxGrid) return PT_ESIZE;
    const void *kern = engine_kernel(fp32, npt, multi, cmesh, timed);
    Launch Xv = X;
    const EngineDesc *Dv = D;
    EngineDesc E1;
    if (single) E1 = *single;
    else memset(&E1, 0, sizeof(E1));
    void *args[] = {(void *)&Dv, (void *)&Xv, (void *)&E1};
    if (capturing(stream))
        PT_TRY(hip_ok(hipLaunchKernel(kern, dim3(grid), dim3(kThreads), args, (unsigned)lds_bytes,
                                      stream)));
    else
        PT_TRY(hip_ok(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kThreads), args,
                                                 (unsigned)lds_bytes, stream)));
    return launch_check();
}

int reset_launch_state(void *ws, const SharedLayout &S, int n_designs, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, stream, at<unsigned>(ws, S.bar),
                       (size_t)kMaxGroups * kBarStride, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, stream, at<unsigned>(ws, S.flags),
                       (size_t)kMaxFlags * n_designs, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, at<unsigned>(ws, S.qhead),
                       (size_t)2, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, stream,
                       at<unsigned>(ws, S.trace), (size_t)S.max_lanes * S.trace_stride * 2, 0u);
    return launch_check();
}

// ---------------------------------------------------------------------------
// Single-design plan: groups with private lane lists
// ---------------------------------------------------------------------------

// Groups come in runs of identical shape: group r of a run gets the lanes
// with slices s0 + r*gstride + k*lstride, k = 0..nlanes-1, kept if within
// [smin, smax]. Built on the device from this kernel argument, so no host
// buffer must outlive the call.
struct Run {
    int kind, ngroups, nwg, tile, s0, gstride, lstride, nlanes, smin, smax;
    int lead_kind, lead_slice;  // a lane run first by every group of the run (kind < 0: none)
};

// Groups of one shape taking two kinds of lanes from shared queue 0, in the
// order the correction sweep consumes them: slice by slice along dirA, lane
// kind A before kind B of the same slice.
struct QueueArgs {
    int ngroups, nwg, tile;
    int kindA, nA, sA0, dirA;
    int kindB, nB, sB0, dirB;
    int lagB;  // B's slice n goes after A's slice n + lagB along the sweep
};

struct PlanArgs {
    int grid;
    int nruns;
    Run run[6];
    QueueArgs Q;
};

__global__ void k_build_plan(PlanArgs P, Group *groups, Lane *lanes, int *wg_group) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int gidx = 0, lidx = 0, w = 0;
    for (int r = 0; r < P.nruns; ++r) {
        const Run R = P.run[r];
        for (int q = 0; q < R.ngroups; ++q) {
            Group G;
            G.wg0 = w;
            G.nwg = R.nwg;
            G.vec = gidx;
            G.queue = -1;
            G.lane0 = lidx;
            int n = 0;
            if (R.lead_kind >= 0) {
                lanes[lidx].kind = R.lead_kind;
                lanes[lidx].slice = R.lead_slice;
                lanes[lidx].design = 0;
                lanes[lidx].tile = R.tile;
                ++n;
            }
            for (int k = 0; k < R.nlanes; ++k) {
                const int sl = R.s0 + q * R.gstride + k * R.lstride;
                if (sl < R.smin || sl > R.smax) continue;
                lanes[lidx + n].kind = R.kind;
                lanes[lidx + n].slice = sl;
                lanes[lidx + n].design = 0;
                lanes[lidx + n].tile = R.tile;
                ++n;
            }
            G.nlanes = n;
            lidx += n;
            groups[gidx] = G;
            for (int k = 0; k < R.nwg; ++k) wg_group[w++] = gidx;
            ++gidx;
        }
    }
    const QueueArgs &Q = P.Q;
    if (Q.ngroups > 0) {
        const int lane0 = lidx;
        // merge the two slice sequences by position along the sweep, B lagging
        // lagB slices behind A (both run in the same direction)
        int ia = 0, ib = 0;
        while (ia < Q.nA || ib < Q.nB) {
            const int sa = Q.sA0 + Q.dirA * ia, sb = Q.sB0 + Q.dirB * ib;
            const bool takeA =
                ib >= Q.nB || (ia < Q.nA && Q.dirA * sa <= Q.dirA * sb + Q.lagB);
            lanes[lidx].kind = takeA ? Q.kindA : Q.kindB;
            lanes[lidx].slice = takeA ? sa : sb;
            lanes[lidx].design = 0;
            lanes[lidx].tile = Q.tile;
            ++lidx;
            if (takeA) ++ia;
            else ++ib;
        }
        for (int q = 0; q < Q.ngroups; ++q) {
            Group G;
            G.wg0 = w;
            G.nwg = Q.nwg;
            G.vec = gidx;
            G.queue = 0;
            G.lane0 = lane0;
            G.nlanes = lidx - lane0;
            groups[gidx] = G;
            for (int k = 0; k < Q.nwg; ++k) wg_group[w++] = gidx;
            ++gidx;
        }
    }
    for (; w < P.grid; ++w) wg_group[w] = -1;
}

// One kind of lane and how its lanes are queued on groups.
struct LanePlan {
    int kind;
    int count;        // lanes
    int slice0;       // first slice in queue order
    int dir;          // +1 ascending, -1 descending slices
    double weight;    // work per lane (relative)
    bool latency;     // sweep-like: fixed group size
    int queues = 0;   // groups (0: one lane per group)
    int fixed_nwg = 0;  // workgroups per group if > 0 (same fine shape in both passes)
    int lead_kind = -1, lead_slice = 0;  // a lane the group runs first (one group only)
};

// Runs one single-design engine launch with descriptor D (already uploaded).
// cm: the coarse mesh of a launch with coarse-mesh lanes (else nullptr).
int run_engine(const EngineDesc &E, const EngineDesc *D, std::vector<LanePlan> &plans, void *ws,
               const Layout &Lay, const pt_tuning &T, hipStream_t stream,
               const CoarseMesh *cm = nullptr) {
    const Consts &C = E.C;
    Control *ctl = E.B.ctl;
    Device dev;
    PT_TRY(device_info(dev));
    const int H = C.W + 1;
    const int lds_cap_d = lds_cap_doubles(dev);
    int grid = dev.cus * T.wg_per_cu;
    // per-round phase times: FP64 launches without coarse-mesh lanes only
    const bool timed = T.phase_timers != 0 && !C.fp32 && !cm;
    // sweep group: 40 workgroups. A resident sweep of full solves to a tight
    // tolerance is the longest lane of the pass: it gets about 1000 nodes per
    // workgroup within 40..64 (a quarter of the grid; measured best at 256^2
    // and 100^2 with rtol 1e-10, the fine lanes queued ahead of the batched
    // coarse steps); shorter sweeps (truncated or loose solves) leave the fine
    // lanes critical, and there more sweep workgroups only slow the fine lanes
    const int sweep_wgs = T.sweep_wgs > 0 ? T.sweep_wgs : 40;
    const bool long_sweep = C.coarse_iters == 0 && C.rtol < 1e-9;
    const int sweep_wgs_res =
        T.sweep_wgs > 0 ? T.sweep_wgs : long_sweep ? std::min(64, std::max(40, C.Nn / 1000)) : 40;

    const int NT = kThreads;
    const int res_npt_max = T.resident_npt_max;
    const int g_min = (C.Nn + NT * res_npt_max - 1) / (NT * res_npt_max);
    bool resident = T.resident != 0 && g_min <= grid / 4 &&
                    (C.Nn + g_min - 1) / g_min >= H && !C.gmg && !C.ckpt;
    // a tile must be at least one halo (H nodes) long
    const int max_wg_per_lane = std::max(1, C.Nn / H);

    std::vector<int> ngroups(plans.size()), per_group(plans.size()), nwg(plans.size()),
        tile(plans.size());
    if (resident) {
        // one tile of <= NT*npt nodes per workgroup; every group holds a whole lane
        int lat_wgs = 0;
        int nq = 0;
        for (size_t k = 0; k < plans.size(); ++k) {
            auto &p = plans[k];
            if (p.latency) {
                nwg[k] = p.fixed_nwg > 0 ? std::max(g_min, p.fixed_nwg)
                                         : std::max(g_min, std::min(sweep_wgs_res, grid / 4));
                nwg[k] = std::max(1, std::min(nwg[k], max_wg_per_lane));
                ngroups[k] = p.count;
                lat_wgs += nwg[k] * p.count;
            } else {
                nwg[k] = g_min;
                ++nq;
            }
        }
        const int avail = (grid - lat_wgs) / g_min;  // groups left for batched lanes
        if (avail < nq) resident = false;
        // without a sequential sweep (G = 0) the lanes are the whole pass:
        // resident groups that cannot hold every lane at once leave the
        // streaming form (all lanes at once, HBM-bound) ahead
        int lanes = 0;
        for (const auto &p : plans) lanes += p.latency ? 0 : p.count;
        if (lat_wgs == 0 && avail < lanes && T.resident != 1) resident = false;
    }
    if (resident) {
        int nq = 0;
        double wF = 0.0;
        int lat_wgs = 0;
        for (size_t k = 0; k < plans.size(); ++k) {
            if (plans[k].latency) lat_wgs += nwg[k] * plans[k].count;
            else {
                wF += plans[k].weight * plans[k].count;
                ++nq;
            }
        }
        const int avail = (grid - lat_wgs) / g_min;
        int left = avail;
        for (size_t k = 0; k < plans.size(); ++k) {
            auto &p = plans[k];
            if (p.latency) continue;
            --nq;
            int q = p.queues > 0 ? p.queues : (int)floor(avail * p.weight * p.count / wF);
            q = std::max(1, std::min(q, std::min(p.count, left - nq)));
            ngroups[k] = q;
            left -= q;
        }
        // few batched lanes (e.g. one slice): spread each over more workgroups
        int used_b = 0;
        for (size_t k = 0; k < plans.size(); ++k)
            if (!plans[k].latency) used_b += ngroups[k] * g_min;
        const int spread = std::max(1, (grid - lat_wgs) / std::max(used_b, 1));
        for (size_t k = 0; k < plans.size(); ++k)
            if (!plans[k].latency)
                nwg[k] = std::max(g_min, std::min(g_min * spread, max_wg_per_lane));
        for (size_t k = 0; k < plans.size(); ++k) {
            per_group[k] = (plans[k].count + ngroups[k] - 1) / ngroups[k];
            const int ts = (C.Nn + nwg[k] - 1) / nwg[k];
            nwg[k] = (C.Nn + ts - 1) / ts;  // every workgroup owns a non-empty tile
            if (ts < H || ts > NT * res_npt_max) return PT_EINVAL;
            tile[k] = ts;
        }
    }
    if (!resident) {
        // streaming: explicit shapes first (sweeps, fixed fine lanes), then the
        // other lanes share the rest of the grid by weight, with at least
        // kMinStreamWgs workgroups per group and within the group budget
        constexpr int kMinStreamWgs = 4;
        int fixed = 0, groups = 0;
        double wsum = 0.0;
        for (size_t k = 0; k < plans.size(); ++k) {
            auto &p = plans[k];
            if (p.latency) {
                ngroups[k] = p.count;
                nwg[k] = p.fixed_nwg > 0 ? p.fixed_nwg : std::max(1, std::min(sweep_wgs, grid / 2));
            } else if (p.fixed_nwg > 0) {
                ngroups[k] = (p.queues <= 0 || p.queues > p.count) ? p.count : p.queues;
                nwg[k] = p.fixed_nwg;
            } else {
                wsum += p.weight * p.count;
                continue;
            }
            fixed += nwg[k] * ngroups[k];
            groups += ngroups[k];
        }
        if (C.ckpt) {
            // checkpointed fine lanes: as many of their fixed groups (at most
            // the recompute slots) as the grid holds beside the sweep groups,
            // leaving the batched coarse steps, if any, a sweep group's worth
            // of workgroups; fewer groups change no result (one group shape)
            int nshare = 0;
            for (const auto &p : plans)
                if (!p.latency && p.fixed_nwg <= 0 && p.count > 0) ++nshare;
            const int reserve = nshare > 0 ? std::max(nshare * kMinStreamWgs, sweep_wgs) : 0;
            for (size_t k = 0; k < plans.size(); ++k) {
                const auto &p = plans[k];
                if (p.latency || p.fixed_nwg <= 0 || (p.kind != F_PRI && p.kind != F_ADJ))
                    continue;
                const int other = fixed - nwg[k] * ngroups[k];
                const int fit = (grid - other - reserve) / nwg[k];
                if (fit >= 1 && fit < ngroups[k]) {
                    fixed -= nwg[k] * (ngroups[k] - fit);
                    groups -= ngroups[k] - fit;
                    ngroups[k] = fit;
                }
            }
        }
        const int rest = std::max(grid - fixed, 0);
        int budget = Lay.s.max_groups - groups;
        bool has_sweep = false;
        for (const auto &p : plans)
            if (p.latency && p.count > 0) has_sweep = true;
        for (size_t k = 0; k < plans.size(); ++k) {
            auto &p = plans[k];
            if (p.latency || p.fixed_nwg > 0) continue;
            const double share = wsum > 0.0 ? rest * p.weight * p.count / wsum : 0.0;
            int q = p.queues > 0 ? std::min(p.queues, p.count)
                                 : std::min(p.count, std::max(1, (int)(share / kMinStreamWgs)));
            if (p.queues <= 0 && has_sweep && p.count > 0) {
                // a sweep consumes these lanes' results slice by slice: run them
                // in balanced waves on groups of about three tiles per
                // workgroup, so results arrive in sweep order and a round
                // streams few tiles (at 512^2: 7 fine groups in 9 waves and
                // one coarse-step group, 37% faster than all lanes at once on
                // groups of 4 workgroups; checkpointed fine lanes keep their
                // fixed groups, their batched coarse steps take one group)
                const long long tile = std::max(256, std::min(T.tile_max, 4096));
                const int target =
                    std::max(kMinStreamWgs, (int)((C.Nn + 3 * tile - 1) / (3 * tile)));
                q = std::max(1, std::min(p.count, (int)(share / target)));
                const int waves = (p.count + q - 1) / q;
                q = (p.count + waves - 1) / waves;
            }
            q = std::max(1, std::min(q, budget));
            budget -= q;
            ngroups[k] = q;
            nwg[k] = std::max(1, (int)floor(share / q));
        }
        for (size_t k = 0; k < plans.size(); ++k) {
            per_group[k] = (plans[k].count + ngroups[k] - 1) / ngroups[k];
            tile[k] = tile_for(C.Nn, nwg[k], H, lds_cap_d, T.tile_max);
        }
    }
    int used = 0, max_tile = 256, total_groups = 0;
    for (size_t k = 0; k < plans.size(); ++k) {
        if (nwg[k] > kMaxGroup) return PT_EINVAL;
        used += nwg[k] * ngroups[k];
        total_groups += ngroups[k];
        max_tile = std::max(max_tile, tile[k]);
    }
    if (total_groups > Lay.s.max_groups) return PT_EINVAL;
    if (used > grid) grid = used;
    if (grid > kMaxGrid) return PT_EINVAL;
    int npt = 0;
    if (resident) {
        npt = 1;
        while (npt * NT < max_tile) npt *= 2;
        if (cm || timed) npt = 8;  // the one resident form of these launches
    }
    if (C.gmg && (C.gmg_chunk < 256 || C.gmg_chunk_init < 256)) return PT_EINVAL;
    size_t lds_bytes =
        C.gmg ? gmg_lds_bytes(C) : engine_lds_doubles(max_tile, C.W) * sizeof(double);
    if (cm) {
        // a coarse-mesh lane stages two windows of its coarse tile and halo
        for (size_t k = 0; k < plans.size(); ++k)
            if (is_cm_kind(plans[k].kind) && plans[k].count > 0) {
                const size_t tc = ((size_t)cm->Nc + nwg[k] - 1) / nwg[k];
                lds_bytes = std::max(lds_bytes, 2 * (tc + 2 * ((size_t)cm->Wc + 1)) * sizeof(double));
            }
    }
    if (lds_bytes > (size_t)dev.lds_max) return PT_EINVAL;

    PlanArgs P{};
    P.grid = grid;
    P.nruns = 0;
    // resident fine and batched coarse lanes of one shape: one shared queue in
    // sweep order instead of private lists (balances lanes of unequal length)
    int qa = -1, qb = -1;
    if (resident && T.shared_queue != 0) {
        for (size_t k = 0; k < plans.size(); ++k) {
            if (plans[k].latency || plans[k].count == 0) continue;
            if (qa < 0) qa = (int)k;
            else if (qb < 0) qb = (int)k;
            else qa = qb = -2;
        }
        if (qa >= 0 && qb >= 0 &&
            (nwg[qa] != nwg[qb] || tile[qa] != tile[qb] || plans[qa].dir != plans[qb].dir))
            qa = qb = -1;
        if (qb < 0) qa = qb = -1;
    }
    if (qa >= 0) {
        QueueArgs &Q = P.Q;
        Q.ngroups = ngroups[qa] + ngroups[qb];
        Q.nwg = nwg[qa];
        Q.tile = tile[qa];
        Q.kindA = plans[qa].kind;
        Q.nA = plans[qa].count;
        Q.sA0 = plans[qa].slice0;
        Q.dirA = plans[qa].dir;
        Q.kindB = plans[qb].kind;
        Q.nB = plans[qb].count;
        Q.sB0 = plans[qb].slice0;
        Q.dirB = plans[qb].dir;
        // a fine lane takes about as long as the sweep's next several steps:
        // queued a few slices ahead of the batched coarse steps, the last fine
        // lanes no longer hold up the sweep's last steps
        Q.lagB = T.gk_lag >= 0 ? T.gk_lag : std::min(6, C.Ntau / 5);
    }
    for (size_t k = 0; k < plans.size(); ++k) {
        const auto &p = plans[k];
        if (p.count == 0 || (int)k == qa || (int)k == qb) continue;
        if (P.nruns >= 6) return PT_EINVAL;
        Run &R = P.run[P.nruns++];
        R.kind = p.kind;
        R.ngroups = ngroups[k];
        R.nwg = nwg[k];
        R.tile = tile[k];
        R.s0 = p.slice0;
        R.gstride = p.dir;                 // neighbouring groups take consecutive slices
        R.lstride = p.dir * ngroups[k];    // a group's queue advances by the group count
        R.nlanes = per_group[k];
        R.smin = std::min(p.slice0, p.slice0 + p.dir * (p.count - 1));
        R.smax = std::max(p.slice0, p.slice0 + p.dir * (p.count - 1));
        R.lead_kind = p.lead_kind;
        R.lead_slice = p.lead_slice;
    }
    hipLaunchKernelGGL(k_build_plan, dim3(1), dim3(64), 0, stream, P, at<Group>(ws, Lay.s.groups),
                       at<Lane>(ws, Lay.s.lanes), at<int>(ws, Lay.s.wg_group));
    PT_TRY(launch_check());
    PT_TRY(reset_launch_state(ws, Lay.s, 1, stream));
    const Launch X = make_launch(ws, Lay.s, ctl, C.timeout_ticks);
    return launch_engine(C.fp32 != 0, npt, D, &E, X, grid, lds_bytes, dev, stream, cm != nullptr,
                         timed);
}

// Fine lanes of a single-design pass. With checkpoints (or PT_FINE_WGS set)
// they run on a fixed number of groups of a fixed size in both passes, so a
// fine adjoint lane recomputes its slice's states with exactly the forward
// pass's arithmetic, and its scratch slot (the group index) stays below
// ck_slots.
LanePlan fine_plan(int kind, int count, int slice0, int dir, const Consts &C,
                   const pt_problem *p) {
    const pt_tuning T = tuning_of(p);
    LanePlan lp{kind, count, slice0, dir, (double)C.M, false, T.fine_groups};
    const int fixed = T.fine_wgs;
    if (C.ckpt || fixed > 0) {
        lp.queues = ck_slots(p);
        lp.fixed_nwg = fixed > 0 ? fixed : 8;
    }
    return lp;
}

// The correction sweep's first step needs the first fine slice of its pass
// (F_0, or the last slice in the adjoint); its group runs that slice itself
// rather than waiting for a fine group. Not with a fixed fine-lane shape
// (checkpoints), where both passes must run every fine slice alike.
bool lead_fine(const Consts &C, int Ntau, bool plt, const pt_tuning &T) {
    if (plt || Ntau < 2 || C.ckpt || T.fine_wgs > 0) return false;
    return T.lead_fine != 0;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b) return false;
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

// ---------------------------------------------------------------------------
// Multi-design plan: worker groups sharing two lane queues
// ---------------------------------------------------------------------------

// Lanes of every design (blockIdx.x = design) in queue order. Queue 0 holds
// the fine lanes F_n interleaved with the batched coarse lanes G(u^k_n) in the
// order the design's sweep consumes them; queue 1 holds the cold sweeps of all
// designs, then their correction sweeps. With designs in the order the host
// chose, the lanes have a global order (all cold sweeps; then per design its
// fine lanes and its correction sweep) that both queues follow and in which
// every lane waits only on earlier lanes; as each queue hands out lanes in
// that order, a waiting lane's producers have all been taken by running
// groups, so the launch cannot deadlock.
__global__ void k_build_lanes(const EngineDesc *__restrict__ D, Lane *lanes) {
    if (threadIdx.x != 0) return;
    const int d = blockIdx.x;
    const EngineDesc &E = D[d];
    const DesignPlan &P = E.plan;
    const int Ntau = E.C.Ntau;
    const bool gk = E.I.gk_lanes != 0;
    int k = P.q0_lane0;
    auto put = [&](int pos, int kind, int slice, int tile) {
        lanes[pos].kind = kind;
        lanes[pos].slice = slice;
        lanes[pos].design = d;
        lanes[pos].tile = tile;
    };
    if (!P.adjoint) {
        for (int n = 0; n < Ntau; ++n) {
            put(k++, F_PRI, n, P.tile0);
            if (gk && n >= 1) put(k++, GK_PRI, n, P.tile0);
        }
    } else {
        for (int n = Ntau; n >= 1; --n) {
            put(k++, F_ADJ, n, P.tile0);
            if (gk && n <= Ntau - 1) put(k++, GK_ADJ, n, P.tile0);
        }
    }
    if (P.q1_cold >= 0) put(P.q1_cold, P.adjoint ? COLD_ADJ : COLD_PRI, 0, P.tile1);
    if (P.q1_sweep >= 0) put(P.q1_sweep, P.adjoint ? SWEEP_ADJ : SWEEP_PRI, 0, P.tile1);
}

struct GroupArgs {
    int grid;
    int n0, wgs0, lane0_0, nlanes0;  // queue 0 workers
    int n1, wgs1, lane0_1, nlanes1;  // queue 1 workers
};

__global__ void k_build_groups(GroupArgs A, Group *groups, int *wg_group) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int w = 0, gidx = 0;
    // sweep workers first: their lanes are the longest sequential chains
    for (int q = 0; q < A.n1; ++q, ++gidx) {
        Group G;
        G.wg0 = w;
        G.nwg = A.wgs1;
        G.lane0 = A.lane0_1;
        G.nlanes = A.nlanes1;
        G.vec = gidx;
        G.queue = 1;
        groups[gidx] = G;
        for (int k = 0; k < A.wgs1; ++k) wg_group[w++] = gidx;
    }
    for (int q = 0; q < A.n0; ++q, ++gidx) {
        Group G;
        G.wg0 = w;
        G.nwg = A.wgs0;
        G.lane0 = A.lane0_0;
        G.nlanes = A.nlanes0;
        G.vec = gidx;
        G.queue = 0;
        groups[gidx] = G;
        for (int k = 0; k < A.wgs0; ++k) wg_group[w++] = gidx;
    }
    for (; w < A.grid; ++w) wg_group[w] = -1;
}

pt_batch_tuning default_tuning(int n) {
    pt_batch_tuning t{};
    t.fine_wgs = 2;
    t.sweep_wgs = 16;
    t.sweep_groups = std::max(1, std::min(n, 8));
    t.resident = 0;
    t.grid = 0;
    t.tile_max = 0;
    return t;
}

bool valid_tuning(const pt_batch_tuning *t) {
    return t->fine_wgs >= 1 && t->fine_wgs <= kMaxGroup && t->sweep_wgs >= 1 &&
           t->sweep_wgs <= kMaxGroup && t->sweep_groups >= 1 &&
           t->sweep_groups < kMaxBatchGroups && (t->resident == 0 || t->resident == 1) &&
           t->grid >= 0 && t->grid <= kMaxGrid &&
           (t->tile_max == 0 || (t->tile_max >= 256 && t->tile_max <= 16384));
}

// Plans and runs one multi-design engine launch. `hd` holds the designs'
// descriptors (C, B, I set); their DesignPlan is filled here and the
// descriptors are uploaded.
int run_batched_engine(std::vector<EngineDesc> &hd, const pt_batch_tuning &T, bool adjoint,
                       void *ws, const BatchLayout &Lay, hipStream_t stream) {
    const int n = (int)hd.size();
    Device dev;
    PT_TRY(device_info(dev));
    const bool fp32 = hd[0].C.fp32 != 0;
    const int npt = T.resident ? 8 : 0;
    const int cap_d = lds_cap_doubles(dev);
    // tiles and LDS of every design on both kinds of worker
    size_t lds_d = 0;
    for (auto &E : hd) {
        const Consts &C = E.C;
        const int H = C.W + 1;
        int t0, t1;
        if (T.resident && C.gmg) return PT_EINVAL;
        if (T.resident) {
            t0 = (C.Nn + T.fine_wgs - 1) / T.fine_wgs;
            t1 = (C.Nn + T.sweep_wgs - 1) / T.sweep_wgs;
            if (t0 < H || t1 < H || t0 > kThreads * npt || t1 > kThreads * npt) return PT_EINVAL;
            // every workgroup of a resident group owns a non-empty tile
            if ((C.Nn + t0 - 1) / t0 != T.fine_wgs || (C.Nn + t1 - 1) / t1 != T.sweep_wgs)
                return PT_EINVAL;
        } else {
            t0 = tile_for(C.Nn, T.fine_wgs, H, cap_d, T.tile_max);
            t1 = tile_for(C.Nn, T.sweep_wgs, H, cap_d, T.tile_max);
        }
        E.plan.tile0 = t0;
        E.plan.tile1 = t1;
        E.plan.adjoint = adjoint ? 1 : 0;
        if (C.gmg && (C.gmg_chunk < 256 || C.gmg_chunk_init < 256)) return PT_EINVAL;
        lds_d = std::max(lds_d, C.gmg ? (gmg_lds_bytes(C) + 7) / 8
                                      : engine_lds_doubles(std::max(t0, t1), C.W));
    }
    const size_t lds_bytes = lds_d * sizeof(double);
    if (lds_bytes > (size_t)dev.lds_max) return PT_EINVAL;
    // designs with the longest sweeps first (N_tau solves of N_n nodes)
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (double)hd[a].C.Ntau * hd[a].C.Nn > (double)hd[b].C.Ntau * hd[b].C.Nn;
    });
    int q0 = 0, q1 = 0;
    for (int d : order) {
        auto &E = hd[d];
        const int Ntau = E.C.Ntau;
        E.plan.q0_lane0 = q0;
        E.plan.q0_count = Ntau + (E.I.gk_lanes ? Ntau - 1 : 0);
        q0 += E.plan.q0_count;
    }
    for (int d : order) {
        auto &E = hd[d];
        E.plan.q1_cold = E.I.cold ? q0 + q1++ : -1;
    }
    for (int d : order) {
        auto &E = hd[d];
        E.plan.q1_sweep = E.C.Ntau > 1 ? q0 + q1++ : -1;
    }
    if (q0 + q1 > Lay.s.max_lanes) return PT_EINVAL;
    int cap = 0;
    PT_TRY(engine_capacity(fp32, npt, true, lds_bytes, dev, cap));
    int grid = std::min(cap, kMaxGrid);
    if (T.grid > 0) grid = std::min(grid, T.grid);
    GroupArgs A{};
    A.n1 = q1 > 0 ? std::min(T.sweep_groups, q1) : 0;
    A.wgs1 = T.sweep_wgs;
    A.lane0_1 = q0;
    A.nlanes1 = q1;
    A.wgs0 = T.fine_wgs;
    A.lane0_0 = 0;
    A.nlanes0 = q0;
    const int left = grid - A.n1 * A.wgs1;
    if (left < A.wgs0) return PT_EINVAL;
    A.n0 = std::min(std::min(left / A.wgs0, q0), kMaxBatchGroups - A.n1);
    if (A.n0 < 1) return PT_EINVAL;
    A.grid = A.n1 * A.wgs1 + A.n0 * A.wgs0;
    EngineDesc *D = at<EngineDesc>(ws, Lay.s.desc);
    PT_TRY(upload_descs(hd, D, stream));
    hipLaunchKernelGGL(k_build_lanes, dim3(n), dim3(64), 0, stream, D, at<Lane>(ws, Lay.s.lanes));
    hipLaunchKernelGGL(k_build_groups, dim3(1), dim3(64), 0, stream, A,
                       at<Group>(ws, Lay.s.groups), at<int>(ws, Lay.s.wg_group));
    PT_TRY(launch_check());
    PT_TRY(reset_launch_state(ws, Lay.s, n, stream));
    const Launch X = make_launch(ws, Lay.s, hd[0].B.ctl, hd[0].C.timeout_ticks);
    return launch_engine(fp32, npt, D, nullptr, X, A.grid, lds_bytes, dev, stream);
}

bool valid_batch(int n, const pt_problem *probs) {
    if (n < 1 || n > 4096 || !probs) return false;
    for (int k = 0; k < n; ++k) {
        if (!valid_problem(&probs[k])) return false;
        if (probs[k].storage != PT_STORE_ALL) return false;
        if (probs[k].iterations != 1) return false;
        if (probs[k].propagator != PT_PARAREAL || probs[k].coarse_iters != 0) return false;
        if (probs[k].precision != probs[0].precision) return false;
    }
    return true;
}

// Passes with coarse propagators on the coarse spatial mesh (PT_COARSE_MESH).
// Per iteration one engine launch runs every slice's fine propagator from the
// guesses u^k_n, the batched coarse-mesh steps G(R u^k_n) (first warm
// iteration, queued with the fine lanes; later iterations reuse the previous
// sweep's outputs, a cold start the cold sweep's) and the coarse-mesh
// correction sweep on a group of its own, which follows the slices' flags;
// the corrected fine states (and the adjoint's coarse-correction
// sensitivities) follow the launch. A cold start first runs the coarse cold
// sweep and prolongs it into the fine guesses.
int coarse_mesh_pass(const pt_problem *prob, std::vector<EngineDesc> &hd, EngineDesc *D,
                     const Layout &Lay, void *ws, const double *guess, const double *guess_theta,
                     bool adjoint, hipStream_t stream) {
    EngineDesc &E = hd[0];
    const Consts &C = E.C;
    Bufs &B = E.B;
    const int Ntau = C.Ntau;
    const size_t Nt1 = (size_t)Ntau + 1, Nn = C.Nn;
    CoarseMesh &M = E.cm;
    M = make_coarse_mesh(ws, Lay.d, prob);
    double *Uprev = at<double>(ws, Lay.d.Uprev), *Uprev_th = at<double>(ws, Lay.d.Uprev_th);
    double *Ga_th = at<double>(ws, Lay.d.Gk_th), *Gb_th = at<double>(ws, Lay.d.Gn_th);
    if (Ntau > 1) {
        PT_TRY(upload_descs(hd, D, stream));
        PT_TRY(cm_setup(D, M, stream));
    }
    const pt_tuning T = tuning_of(prob);
    const bool lead = lead_fine(C, Ntau, false, T);
    for (int it = 0; it < prob->iterations; ++it) {
        LaunchInfo &I = E.I;
        I = LaunchInfo{};
        I.has_dc = (prob->c0 != prob->cmin) ? 1 : 0;
        I.epoch = 1;
        if (!adjoint) {
            B.Gk_th = Ga_th;
            B.Gn_th = Gb_th;
        }
        const bool cold0 = guess == nullptr && it == 0 && Ntau > 1;
        const double *in = it == 0 ? guess : Uprev;
        const double *in_th = it == 0 ? guess_theta : Uprev_th;
        if (cold0) {
            // the cold coarse sweep: the sweep lane alone in a cold launch
            B.in_L = nullptr;
            B.in_T = nullptr;
            B.in_th = nullptr;
            I.cold = 1;
            PT_TRY(upload_descs(hd, D, stream));
            std::vector<LanePlan> cp;
            cp.push_back({adjoint ? CM_SWEEP_ADJ : CM_SWEEP_PRI, 1, 0, +1, 0.0, true, 0});
            cp.back().fixed_nwg = T.cm_sweep_wgs;
            PT_TRY(run_engine(E, D, cp, ws, Lay, T, stream, &M));
            PT_TRY(cm_guess(D, M, C.Nn, Ntau, adjoint, Uprev, adjoint ? nullptr : Uprev_th,
                            stream));
            I.cold = 0;
            in = Uprev;
            in_th = Uprev_th;
        }
        if (adjoint) {
            B.in_L = in;
        } else {
            B.in_T = in;
            B.in_th = in_th;
        }
        I.gk_lanes = (it == 0 && !cold0 && Ntau > 1) ? 1 : 0;
        PT_TRY(upload_descs(hd, D, stream));
        std::vector<LanePlan> plans;
        const int fk = adjoint ? F_ADJ : F_PRI;
        if (adjoint)
            plans.push_back(lead ? fine_plan(fk, Ntau - 1, Ntau - 1, -1, C, prob)
                                 : fine_plan(fk, Ntau, Ntau, -1, C, prob));
        else
            plans.push_back(lead ? fine_plan(fk, Ntau - 1, 1, +1, C, prob)
                                 : fine_plan(fk, Ntau, 0, +1, C, prob));
        if (I.gk_lanes)
            plans.push_back({adjoint ? CM_GK_ADJ : CM_GK_PRI, Ntau - 1, adjoint ? Ntau - 1 : 1,
                             adjoint ? -1 : +1, T.gk_weight, false, T.gk_groups});
        if (Ntau > 1) {
            plans.push_back({adjoint ? CM_SWEEP_ADJ : CM_SWEEP_PRI, 1, 0, +1, 0.0, true, 0});
            plans.back().fixed_nwg = T.cm_sweep_wgs;
            if (lead) {
                plans.back().lead_kind = fk;
                plans.back().lead_slice = adjoint ? Ntau : 0;
            }
        }
        PT_TRY(run_engine(E, D, plans, ws, Lay, T, stream, Ntau > 1 ? &M : nullptr));
        if (Ntau > 1) PT_TRY(cm_correct(D, M, C.Nn, Ntau, adjoint, C.Ne, stream));
        if (it + 1 < prob->iterations) {
            double *out = adjoint ? B.out_L : B.out_T;
            hipLaunchKernelGGL(k_copy_f64, dim3(1024), dim3(256), 0, stream, Uprev, out, Nt1 * Nn);
            if (!adjoint)
                hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(256), 0, stream, Uprev_th, B.out_th,
                                   Nt1);
            PT_TRY(launch_check());
            std::swap(M.Gk, M.Gn);
            std::swap(Ga_th, Gb_th);
        }
    }
    if (adjoint) hipLaunchKernelGGL(k_finalize_adj, dim3(256, 1), dim3(256), 0, stream, D);
    else hipLaunchKernelGGL(k_finalize_fwd, dim3(256, 1), dim3(256), 0, stream, D);
    return launch_check();
}

// Status and counters of a single-design workspace as a pt_stats (device).
__global__ void k_write_stats(const Control *ctl, pt_stats *out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    out->status = ctl->status;
    out->max_cg_iters = ctl->max_iters;
    out->cg_iters_fine = (int64_t)ctl->iters_fine;
    out->cg_iters_coarse = (int64_t)ctl->iters_coarse;
    out->solves_fine = (int64_t)ctl->solves_fine;
    out->solves_coarse = (int64_t)ctl->solves_coarse;
    out->max_rel_residual = __longlong_as_double((long long)ctl->max_relres_bits);
}

// The workspace of pt_cycle_noalloc: one copy per GPU, held until the process
// ends. In host code `scratch` is only a host-side stand-in for the device
// array; kernels receive the device address hipGetSymbolAddress returns for
// the current device, taken once per device and kept below.
static __device__ __align__(256) unsigned char scratch[PT_NOALLOC_WS_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int noalloc_workspace(void **out) {
    int dev = 0;
    PT_TRY(hip_ok(hipGetDevice(&dev)));
    if (dev < 0 || dev >= kMaxDevices) return PT_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        PT_TRY(hip_ok(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch))));
        if (!ptr) return PT_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PT_OK;
}

int batched_cycle(int n, const pt_problem *probs, const double *const *rho, int warm,
                  const pt_batch_tuning *tuning, double *Theta_out, double *const *dTheta_drho,
                  void *ws, size_t ws_bytes, hipStream_t stream, bool save_guess);

}  // namespace

extern "C" {

int pt_validate(const pt_problem *prob) { return valid_problem(prob) ? PT_OK : PT_EINVAL; }

int pt_default_tuning(pt_tuning *out) {
    if (!out) return PT_EINVAL;
    *out = default_settings();
    return PT_OK;
}

size_t pt_workspace_bytes(const pt_problem *prob) {
    if (!valid_problem(prob)) return 0;
    return layout(prob).total;
}

size_t pt_state_bytes(const pt_problem *prob) {
    if (!valid_problem(prob)) return 0;
    return state_rows(prob) * (size_t)(prob->nx + 1) * (prob->ny + 1) * sizeof(double);
}

const char *pt_strerror(int code) {
    switch (code) {
        case PT_OK: return "ok";
        case PT_EINVAL: return "invalid argument";
        case PT_ENOMEM: return "workspace too small";
        case PT_EHIP: return "HIP runtime error or device wait timeout";
        case PT_ENOCONV: return "a CG solve reached max_iter";
        case PT_EDOMAIN: return "non-finite input or result, or Theta <= 0";
        case PT_ESTATE: return "call order violated";
        case PT_ESIZE:
            return "problem too large: more workspace than the static array of "
                   "pt_cycle_noalloc, or a launch the device cannot hold co-resident";
        default: return "unknown error";
    }
}

int pt_parareal_forward(const pt_problem *prob, const double *rho, const double *guess_T,
                        const double *guess_theta, double *S, double *uT_out, double *utheta_out,
                        double *Theta_out, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!valid_problem(prob)) return PT_EINVAL;
    if (!rho || !S || !Theta_out || !ws) return PT_EINVAL;
    const bool plt = prob->propagator == PT_PLT;
    if (plt) guess_theta = nullptr;  // u holds T only (Sec. 7)
    else if ((guess_T == nullptr) != (guess_theta == nullptr)) return PT_EINVAL;
    const Layout Lay = layout(prob);
    if (ws_bytes < Lay.total) return PT_ENOMEM;
    const Consts C = make_consts(prob);
    const pt_tuning T = tuning_of(prob);
    const size_t Nn = C.Nn, Nt1 = C.Ntau + 1;
    const size_t sz_U = Nt1 * Nn * sizeof(double), sz_S = state_rows(prob) * Nn * sizeof(double);
    if (guess_T) {
        const void *outs[] = {S, uT_out, utheta_out, Theta_out, ws};
        const size_t lens[] = {sz_S, sz_U, Nt1 * sizeof(double), sizeof(double), ws_bytes};
        for (int k = 0; k < 5; ++k)
            if (overlaps(guess_T, sz_U, outs[k], lens[k]) ||
                overlaps(guess_theta, Nt1 * sizeof(double), outs[k], lens[k]))
                return PT_EINVAL;
    }
    if (overlaps(S, sz_S, ws, ws_bytes) || overlaps(uT_out, sz_U, ws, ws_bytes)) return PT_EINVAL;

    std::vector<EngineDesc> hd(1);
    memset(hd.data(), 0, sizeof(EngineDesc));
    EngineDesc &E = hd[0];
    E.C = C;
    E.B = make_bufs(ws, Lay.d, Lay.s, 0);
    E.B.rho = rho;
    EngineDesc *D = at<EngineDesc>(ws, Lay.s.desc);
    PT_TRY(upload_descs(hd, D, stream));
    PT_TRY(setup_designs(1, prob, hd, D, 0, stream));

    double *outT = uT_out ? uT_out : at<double>(ws, Lay.d.Ubuf);
    double *outth = utheta_out ? utheta_out : at<double>(ws, Lay.d.Ubuf_th);
    double *Uprev = at<double>(ws, Lay.d.Uprev);
    double *Uprev_th = at<double>(ws, Lay.d.Uprev_th);
    double *Ga = at<double>(ws, Lay.d.Gk), *Gb = at<double>(ws, Lay.d.Gn);
    double *Ga_th = at<double>(ws, Lay.d.Gk_th), *Gb_th = at<double>(ws, Lay.d.Gn_th);
    const bool cold = guess_T == nullptr;
    const int Ntau = C.Ntau;
    Bufs &B = E.B;
    if (prob->propagator == PT_COARSE_MESH) {
        B.S = S;
        B.out_T = outT;
        B.out_th = outth;
        B.Theta_out = Theta_out;
        return coarse_mesh_pass(prob, hd, D, Lay, ws, guess_T, guess_theta, false, stream);
    }
    for (int it = 0; it < prob->iterations; ++it) {
        LaunchInfo &I = E.I;
        I = LaunchInfo{};
        // with G = 0 there are no coarse lanes: a cold pass has in_T == NULL
        I.cold = (cold && it == 0 && !plt) ? 1 : 0;
        I.gk_lanes = (!cold && it == 0 && Ntau > 1 && !plt) ? 1 : 0;
        I.has_dc = (prob->c0 != prob->cmin) ? 1 : 0;
        I.epoch = 1;
        B.in_T = it == 0 ? guess_T : Uprev;
        B.in_th = it == 0 ? guess_theta : Uprev_th;
        B.S = S;
        B.out_T = outT;
        B.out_th = outth;
        B.Gk = Ga;
        B.Gk_th = Ga_th;
        B.Gn = Gb;
        B.Gn_th = Gb_th;
        B.Theta_out = Theta_out;
        PT_TRY(upload_descs(hd, D, stream));
        std::vector<LanePlan> plans;
        // the sweep cannot start before F_0: its group runs F_0 itself
        const bool lead = lead_fine(C, Ntau, plt, T);
        plans.push_back(lead ? fine_plan(F_PRI, Ntau - 1, 1, +1, C, prob)
                             : fine_plan(F_PRI, Ntau, 0, +1, C, prob));
        if (I.gk_lanes)
            plans.push_back({GK_PRI, Ntau - 1, 1, +1, T.gk_weight, false, T.gk_groups});
        if (I.cold) plans.push_back({COLD_PRI, 1, 0, +1, 0.0, true, 0});
        if (Ntau > 1 && !plt) {
            plans.push_back({SWEEP_PRI, 1, 0, +1, 0.0, true, 0});
            if (lead) {
                plans.back().lead_kind = F_PRI;
                plans.back().lead_slice = 0;
            }
        }
        PT_TRY(run_engine(E, D, plans, ws, Lay, T, stream));
        if (it + 1 < prob->iterations) {
            hipLaunchKernelGGL(k_copy_f64, dim3(1024), dim3(256), 0, stream, Uprev, outT, Nt1 * Nn);
            if (!plt)
                hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(256), 0, stream, Uprev_th, outth, Nt1);
            PT_TRY(launch_check());
            std::swap(Ga, Gb);
            std::swap(Ga_th, Gb_th);
        }
    }
    hipLaunchKernelGGL(k_finalize_fwd, dim3(256, 1), dim3(256), 0, stream, D);
    return launch_check();
}

int pt_parareal_adjoint(const pt_problem *prob, const double *rho, const double *S,
                        const double *Theta, const double *guess_lambda, double *lambda_out,
                        void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!valid_problem(prob)) return PT_EINVAL;
    if (!rho || !S || !Theta || !ws) return PT_EINVAL;
    const Layout Lay = layout(prob);
    if (ws_bytes < Lay.total) return PT_ENOMEM;
    const Consts C = make_consts(prob);
    const pt_tuning T = tuning_of(prob);
    const size_t Nn = C.Nn, Nt1 = C.Ntau + 1;
    const size_t sz_U = Nt1 * Nn * sizeof(double);
    if (guess_lambda) {
        if (overlaps(guess_lambda, sz_U, lambda_out, sz_U) ||
            overlaps(guess_lambda, sz_U, ws, ws_bytes))
            return PT_EINVAL;
    }
    if (overlaps(lambda_out, sz_U, ws, ws_bytes)) return PT_EINVAL;
    const bool plt = prob->propagator == PT_PLT;
    std::vector<EngineDesc> hd(1);
    memset(hd.data(), 0, sizeof(EngineDesc));
    EngineDesc &E = hd[0];
    E.C = C;
    E.B = make_bufs(ws, Lay.d, Lay.s, 0);
    E.B.rho = rho;
    EngineDesc *D = at<EngineDesc>(ws, Lay.s.desc);
    PT_TRY(upload_descs(hd, D, stream));
    PT_TRY(setup_designs(1, prob, hd, D, 1, stream));

    double *outL = lambda_out ? lambda_out : at<double>(ws, Lay.d.Ubuf);
    double *Lprev = at<double>(ws, Lay.d.Uprev);
    double *Ga = at<double>(ws, Lay.d.Gk), *Gb = at<double>(ws, Lay.d.Gn);
    const bool cold = guess_lambda == nullptr;
    const int Ntau = C.Ntau;
    Bufs &B = E.B;
    if (prob->propagator == PT_COARSE_MESH) {
        B.S = const_cast<double *>(S);
        B.Theta = Theta;
        B.out_L = outL;
        return coarse_mesh_pass(prob, hd, D, Lay, ws, guess_lambda, nullptr, true, stream);
    }
    for (int it = 0; it < prob->iterations; ++it) {
        LaunchInfo &I = E.I;
        I = LaunchInfo{};
        I.cold = (cold && it == 0 && !plt) ? 1 : 0;
        I.gk_lanes = (!cold && it == 0 && Ntau > 1 && !plt) ? 1 : 0;
        I.has_dc = (prob->c0 != prob->cmin) ? 1 : 0;
        I.epoch = 1;
        B.S = const_cast<double *>(S);
        B.Theta = Theta;
        B.in_L = it == 0 ? guess_lambda : Lprev;
        B.out_L = outL;
        B.Gk = Ga;
        B.Gn = Gb;
        PT_TRY(upload_descs(hd, D, stream));
        std::vector<LanePlan> plans;
        // the reversed sweep consumes slices from N_tau downwards
        const bool lead = lead_fine(C, Ntau, plt, T);
        plans.push_back(lead ? fine_plan(F_ADJ, Ntau - 1, Ntau - 1, -1, C, prob)
                             : fine_plan(F_ADJ, Ntau, Ntau, -1, C, prob));
        if (I.gk_lanes)
            plans.push_back({GK_ADJ, Ntau - 1, Ntau - 1, -1, T.gk_weight, false, T.gk_groups});
        if (I.cold) plans.push_back({COLD_ADJ, 1, 0, +1, 0.0, true, 0});
        if (Ntau > 1 && !plt) {
            plans.push_back({SWEEP_ADJ, 1, 0, +1, 0.0, true, 0});
            if (lead) {
                plans.back().lead_kind = F_ADJ;
                plans.back().lead_slice = Ntau;
            }
        }
        PT_TRY(run_engine(E, D, plans, ws, Lay, T, stream));
        if (it + 1 < prob->iterations) {
            hipLaunchKernelGGL(k_copy_f64, dim3(1024), dim3(256), 0, stream, Lprev, outL, Nt1 * Nn);
            PT_TRY(launch_check());
            std::swap(Ga, Gb);
        }
    }
    hipLaunchKernelGGL(k_finalize_adj, dim3(256, 1), dim3(256), 0, stream, D);
    return launch_check();
}

int pt_sensitivities(const pt_problem *prob, const double *rho, const void *ws, size_t ws_bytes,
                     double *dTheta_drho, hipStream_t stream) {
    if (!valid_problem(prob)) return PT_EINVAL;
    if (!rho || !ws || !dTheta_drho) return PT_EINVAL;
    const Layout Lay = layout(prob);
    if (ws_bytes < Lay.total) return PT_ENOMEM;
    void *w = const_cast<void *>(ws);
    std::vector<EngineDesc> hd(1);
    memset(hd.data(), 0, sizeof(EngineDesc));
    hd[0].C = make_consts(prob);
    hd[0].B = make_bufs(w, Lay.d, Lay.s, 0);
    hd[0].B.rho = rho;
    hd[0].B.grad = dTheta_drho;
    EngineDesc *D = at<EngineDesc>(w, Lay.s.desc);
    PT_TRY(upload_descs(hd, D, stream));
    hipLaunchKernelGGL(k_sensitivities, dim3(512, 1), dim3(256), 0, stream, D);
    return launch_check();
}

int pt_query_trace(const pt_problem *prob, const void *ws, hipStream_t stream,
                   unsigned long long *out, size_t out_words, int *n_lanes, int *stride) {
    if (!valid_problem(prob) || !ws || !out || !n_lanes || !stride) return PT_EINVAL;
    const Layout Lay = layout(prob);
    PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    const size_t words = (size_t)Lay.s.max_lanes * Lay.s.trace_stride;
    const size_t n = std::min(words, out_words);
    PT_TRY(hip_ok(hipMemcpy(out, static_cast<const char *>(ws) + Lay.s.trace,
                            n * sizeof(unsigned long long), hipMemcpyDeviceToHost)));
    *n_lanes = Lay.s.max_lanes;
    *stride = Lay.s.trace_stride;
    return PT_OK;
}

static int read_status(const void *ctl_dev, pt_stats *out) {
    Control c;
    PT_TRY(hip_ok(hipMemcpy(&c, ctl_dev, sizeof(Control), hipMemcpyDeviceToHost)));
    memset(out, 0, sizeof(*out));
    out->status = c.status;
    out->max_cg_iters = c.max_iters;
    out->cg_iters_fine = (int64_t)c.iters_fine;
    out->cg_iters_coarse = (int64_t)c.iters_coarse;
    out->solves_fine = (int64_t)c.solves_fine;
    out->solves_coarse = (int64_t)c.solves_coarse;
    double r;
    memcpy(&r, &c.max_relres_bits, sizeof(double));
    out->max_rel_residual = r;
    return PT_OK;
}

int pt_query_status(const void *ws, hipStream_t stream, pt_stats *out) {
    if (!ws || !out) return PT_EINVAL;
    PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    return read_status(ws, out);
}

size_t pt_batched_workspace_bytes(int n, const pt_problem *probs) {
    if (!valid_batch(n, probs)) return 0;
    return batch_layout(n, probs).total;
}

int pt_batch_default_tuning(int n, pt_batch_tuning *out) {
    if (n < 1 || !out) return PT_EINVAL;
    *out = default_tuning(n);
    return PT_OK;
}

int pt_parareal_batched(int n, const pt_problem *probs, const double *const *rho, int warm,
                        const pt_batch_tuning *tuning, double *Theta_out,
                        double *const *dTheta_drho, void *ws, size_t ws_bytes,
                        hipStream_t stream) {
    return batched_cycle(n, probs, rho, warm, tuning, Theta_out, dTheta_drho, ws, ws_bytes,
                         stream, true);
}

int pt_batched_status(int n, const pt_problem *probs, const void *ws, hipStream_t stream,
                      pt_stats *out) {
    if (!valid_batch(n, probs) || !ws || !out) return PT_EINVAL;
    const BatchLayout Lay = batch_layout(n, probs);
    PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    for (int k = 0; k < n; ++k)
        PT_TRY(read_status(static_cast<const char *>(ws) + Lay.d[k].ctl, &out[k]));
    return PT_OK;
}

}  // extern "C"

namespace {

// One optimisation cycle of every design of a batch. With save_guess the
// corrected u and lambda become the next warm cycle's guesses (Alg. 3);
// without, the guesses in ws stay as they are (the autotuner's timed cycles
// all restart from one state).
int batched_cycle(int n, const pt_problem *probs, const double *const *rho, int warm,
                  const pt_batch_tuning *tuning, double *Theta_out, double *const *dTheta_drho,
                  void *ws, size_t ws_bytes, hipStream_t stream, bool save_guess) {
    if (!valid_batch(n, probs)) return PT_EINVAL;
    if (!rho || !Theta_out || !ws || (warm != 0 && warm != 1)) return PT_EINVAL;
    const bool fwd_only = dTheta_drho == nullptr;  // primal pass only
    for (int k = 0; k < n; ++k)
        if (!rho[k] || (!fwd_only && !dTheta_drho[k])) return PT_EINVAL;
    const pt_batch_tuning T = tuning ? *tuning : default_tuning(n);
    if (!valid_tuning(&T)) return PT_EINVAL;
    const BatchLayout Lay = batch_layout(n, probs);
    if (ws_bytes < Lay.total) return PT_ENOMEM;
    if (overlaps(Theta_out, sizeof(double) * n, ws, ws_bytes)) return PT_EINVAL;
    for (int k = 0; k < n && !fwd_only; ++k)
        if (overlaps(dTheta_drho[k], sizeof(double) * probs[k].nx * probs[k].ny, ws, ws_bytes))
            return PT_EINVAL;

    std::vector<EngineDesc> hd(n);
    memset(hd.data(), 0, sizeof(EngineDesc) * n);
    for (int k = 0; k < n; ++k) {
        EngineDesc &E = hd[k];
        const DesignLayout &L = Lay.d[k];
        E.C = make_consts(&probs[k]);
        // lanes of later designs may wait seconds for the shared sweep workers
        if (!(tuning_of(&probs[k]).wait_timeout_s > 0.0))
            E.C.timeout_ticks = (long long)(60.0 * 1e8);
        E.B = make_bufs(ws, L, Lay.s, k);
        E.B.rho = rho[k];
        E.B.S = at<double>(ws, L.S);
        E.B.out_T = at<double>(ws, L.uT);
        E.B.out_th = at<double>(ws, L.uth);
        E.B.out_L = at<double>(ws, L.lam);
        E.B.Theta_out = Theta_out + k;
        E.B.Theta = Theta_out + k;
        E.B.grad = fwd_only ? nullptr : dTheta_drho[k];
        E.B.save_T = at<double>(ws, L.gT);
        E.B.save_th = at<double>(ws, L.gth);
        E.B.save_L = at<double>(ws, L.gL);
        E.I.cold = warm ? 0 : 1;
        E.I.gk_lanes = (warm && E.C.Ntau > 1) ? 1 : 0;
        E.I.has_dc = (probs[k].c0 != probs[k].cmin) ? 1 : 0;
        E.I.epoch = 1;
    }
    EngineDesc *D = at<EngineDesc>(ws, Lay.s.desc);
    PT_TRY(upload_descs(hd, D, stream));
    PT_TRY(setup_designs(n, probs, hd, D, 0, stream));
    // primal pass of every design in one launch
    for (int k = 0; k < n; ++k) {
        Bufs &B = hd[k].B;
        B.in_T = warm ? at<double>(ws, Lay.d[k].gT) : nullptr;
        B.in_th = warm ? at<double>(ws, Lay.d[k].gth) : nullptr;
        B.Gk = at<double>(ws, Lay.d[k].Gk);
        B.Gk_th = at<double>(ws, Lay.d[k].Gk_th);
        B.Gn = at<double>(ws, Lay.d[k].Gn);
        B.Gn_th = at<double>(ws, Lay.d[k].Gn_th);
    }
    PT_TRY(run_batched_engine(hd, T, false, ws, Lay, stream));
    hipLaunchKernelGGL(k_finalize_fwd, dim3(64, n), dim3(256), 0, stream, D);
    PT_TRY(launch_check());
    if (fwd_only) {
        if (save_guess)
            hipLaunchKernelGGL(k_save_guess, dim3(128, n), dim3(256), 0, stream, D, 1,
                               warm ? 0 : 1);
        return launch_check();
    }
    // adjoint pass of every design in one launch
    for (int k = 0; k < n; ++k) {
        Bufs &B = hd[k].B;
        B.in_L = warm ? at<double>(ws, Lay.d[k].gL) : nullptr;
    }
    PT_TRY(run_batched_engine(hd, T, true, ws, Lay, stream));
    hipLaunchKernelGGL(k_finalize_adj, dim3(64, n), dim3(256), 0, stream, D);
    hipLaunchKernelGGL(k_sensitivities, dim3(128, n), dim3(256), 0, stream, D);
    if (save_guess) hipLaunchKernelGGL(k_save_guess, dim3(128, n), dim3(256), 0, stream, D, 0, 0);
    return launch_check();
}

}  // namespace

extern "C" {

int pt_autotune_batched(int n, const pt_problem *probs, const double *const *rho,
                        double *Theta_out, double *const *dTheta_drho, void *ws,
                        size_t ws_bytes, hipStream_t stream, pt_batch_tuning *best,
                        double *best_ms, double *default_ms, pt_autotune_progress progress,
                        void *user) {
    if (!valid_batch(n, probs) || !best) return PT_EINVAL;
    if (capturing(stream)) return PT_EINVAL;
    const pt_batch_tuning dflt = default_tuning(n);
    // the state every timed cycle restarts from
    PT_TRY(batched_cycle(n, probs, rho, 0, &dflt, Theta_out, dTheta_drho, ws, ws_bytes, stream,
                         true));
    PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    std::vector<pt_stats> st(n);
    PT_TRY(pt_batched_status(n, probs, ws, stream, st.data()));
    for (const auto &x : st)
        if (x.status != PT_OK) return x.status;
    hipEvent_t e0, e1;
    PT_TRY(hip_ok(hipEventCreate(&e0)));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PT_EHIP;
    }
    constexpr int kRepeats = 3;
    // median of kRepeats warm cycles; a shape the batch cannot use, or any
    // device-side problem of a design, makes the shape unusable (ms = +inf)
    auto time_raw = [&](const pt_batch_tuning &t, double &ms) -> int {
        ms = INFINITY;
        if (!valid_tuning(&t)) return PT_OK;
        double ts[kRepeats];
        for (int r = 0; r < kRepeats; ++r) {
            PT_TRY(hip_ok(hipEventRecord(e0, stream)));
            const int rc = batched_cycle(n, probs, rho, 1, &t, Theta_out, dTheta_drho, ws,
                                         ws_bytes, stream, false);
            if (rc == PT_EINVAL || rc == PT_ESIZE) return PT_OK;
            PT_TRY(rc);
            PT_TRY(hip_ok(hipEventRecord(e1, stream)));
            PT_TRY(hip_ok(hipEventSynchronize(e1)));
            float f = 0.0f;
            PT_TRY(hip_ok(hipEventElapsedTime(&f, e0, e1)));
            PT_TRY(pt_batched_status(n, probs, ws, stream, st.data()));
            for (const auto &x : st)
                if (x.status != PT_OK) return PT_OK;
            ts[r] = f;
        }
        std::sort(ts, ts + kRepeats);
        ms = ts[kRepeats / 2];
        return PT_OK;
    };
    auto time_shape = [&](const pt_batch_tuning &t, double &ms) -> int {
        const int rc = time_raw(t, ms);
        if (rc == PT_OK && progress) progress(&t, ms, user);
        return rc;
    };
    pt_batch_tuning cur = dflt;
    double best_t = INFINITY, t_dflt = INFINITY;
    int rc = time_shape(dflt, t_dflt);
    best_t = t_dflt;
    auto consider = [&](pt_batch_tuning t) -> int {
        if (memcmp(&t, &cur, sizeof(t)) == 0) return PT_OK;
        double ms = INFINITY;
        PT_TRY(time_shape(t, ms));
        if (ms < best_t) {
            best_t = ms;
            cur = t;
        }
        return PT_OK;
    };
    const int fine_opts[] = {1, 2, 4, 8, 16};
    const int sweep_opts[] = {4, 8, 16, 32};
    const int group_opts[] = {std::max(1, n / 8), std::max(1, n / 4), std::max(1, n / 2), n};
    const int tile_opts[] = {0, 2048, 1024};
    for (int pass = 0; pass < 2 && rc == PT_OK; ++pass) {
        for (int r = 0; r <= 1 && rc == PT_OK; ++r) {
            pt_batch_tuning t = cur;
            t.resident = r;
            rc = consider(t);
        }
        for (int f : fine_opts) {
            pt_batch_tuning t = cur;
            t.fine_wgs = f;
            if (rc == PT_OK) rc = consider(t);
        }
        for (int w : sweep_opts) {
            pt_batch_tuning t = cur;
            t.sweep_wgs = w;
            if (rc == PT_OK) rc = consider(t);
        }
        for (int g : group_opts) {
            pt_batch_tuning t = cur;
            t.sweep_groups = std::min(g, kMaxBatchGroups - 1);
            if (rc == PT_OK) rc = consider(t);
        }
        for (int tm : tile_opts) {
            pt_batch_tuning t = cur;
            if (t.resident) break;
            t.tile_max = tm;
            if (rc == PT_OK) rc = consider(t);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PT_OK) return rc;
    if (!(best_t < INFINITY)) return PT_ENOCONV;  // no shape ran the batch cleanly
    *best = cur;
    if (best_ms) *best_ms = best_t;
    if (default_ms) *default_ms = t_dflt;
    return PT_OK;
}

int pt_cycle_noalloc(const pt_problem *prob, const double *rho, const double *guess_T,
                     const double *guess_theta, const double *guess_lambda, double *S,
                     double *uT_out, double *utheta_out, double *lambda_out, double *Theta_out,
                     double *dTheta_drho, pt_stats *stats_out, hipStream_t stream) {
    if (!valid_problem(prob)) return PT_EINVAL;
    if (!rho || !S || !Theta_out || !dTheta_drho) return PT_EINVAL;
    if (layout(prob).total > PT_NOALLOC_WS_BYTES) return PT_ESIZE;
    void *ws = nullptr;
    PT_TRY(noalloc_workspace(&ws));
    const size_t bytes = PT_NOALLOC_WS_BYTES;
    PT_TRY(pt_parareal_forward(prob, rho, guess_T, guess_theta, S, uT_out, utheta_out, Theta_out,
                               ws, bytes, stream));
    PT_TRY(pt_parareal_adjoint(prob, rho, S, Theta_out, guess_lambda, lambda_out, ws, bytes,
                               stream));
    PT_TRY(pt_sensitivities(prob, rho, ws, bytes, dTheta_drho, stream));
    if (stats_out) {
        // the status block sits at offset 0 of a single-design workspace
        hipLaunchKernelGGL(k_write_stats, dim3(1), dim3(64), 0, stream,
                           static_cast<const Control *>(ws), stats_out);
        PT_TRY(launch_check());
    }
    return PT_OK;
}

}  // extern "C"
