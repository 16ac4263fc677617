// Host side of libpt: argument checks, workspace layout, lane planning and the
// stream-ordered launches of one forward / adjoint / sensitivity call.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/pt.h"
#include "pt_engine.hip"

using namespace pt;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t ctl, bar, flags, partials, wg_group, groups, lanes, FL;
    size_t kq, cm, dk, dc, dinv_f, dinv_c, mask, qt, zero;
    size_t Gk, Gn, Gk_th, Gn_th, F_th, Uprev, Uprev_th, Ubuf, Ubuf_th, Lprev, Lbuf;
    size_t acc, accG, pool, trace, xch;
    size_t total;
    int trace_stride;
    int max_lanes, max_grid;
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
    if ((p->precision != PT_FP64 && p->precision != PT_FP32_REFINE) || p->precond != PT_JACOBI ||
        p->storage != PT_STORE_ALL)
        return false;
    if (p->bc < 0 || p->bc > 3) return false;
    if (p->bc == PT_BC_MASK && !p->dirichlet_mask) return false;
    if (p->q_t)
        for (int n = 0; n <= p->n_steps; ++n)
            if (!isfinite(p->q_t[n])) return false;
    return true;
}

Layout layout(const pt_problem *p) {
    Layout L{};
    const size_t Nn = (size_t)(p->nx + 1) * (p->ny + 1);
    const size_t Ne = (size_t)p->nx * p->ny;
    const size_t EP = (size_t)(p->nx + 2) * (p->ny + 2);
    const size_t Nt1 = (size_t)p->n_slices + 1;
    L.max_lanes = 2 * p->n_slices + 2;
    L.max_grid = 1024;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.ctl = take(sizeof(Control));
    L.bar = take(sizeof(unsigned) * kMaxLanes);
    L.flags = take(sizeof(unsigned) * kMaxFlags);
    L.partials = take(sizeof(double) * (size_t)L.max_lanes * 2 * kMaxGroup * 4);
    L.wg_group = take(sizeof(int) * L.max_grid);
    L.groups = take(sizeof(Group) * kMaxLanes);
    L.lanes = take(sizeof(Lane) * L.max_lanes);
    L.FL = take(sizeof(double) * Nt1 * Nn);
    L.kq = take(sizeof(double) * EP);
    L.cm = take(sizeof(double) * EP);
    L.dk = take(sizeof(double) * Ne);
    L.dc = take(sizeof(double) * Ne);
    L.dinv_f = take(sizeof(double) * Nn);
    L.dinv_c = take(sizeof(double) * Nn);
    L.mask = take(Nn);
    L.qt = take(sizeof(double) * (p->n_steps + 1));
    L.zero = take(sizeof(double) * Nn);
    L.Gk = take(sizeof(double) * Nt1 * Nn);
    L.Gn = take(sizeof(double) * Nt1 * Nn);
    L.Gk_th = take(sizeof(double) * Nt1);
    L.Gn_th = take(sizeof(double) * Nt1);
    L.F_th = take(sizeof(double) * Nt1);
    L.Uprev = take(sizeof(double) * Nt1 * Nn);
    L.Uprev_th = take(sizeof(double) * Nt1);
    L.Ubuf = take(sizeof(double) * Nt1 * Nn);
    L.Ubuf_th = take(sizeof(double) * Nt1);
    L.Lprev = L.Uprev;  // adjoint reuses the primal scratch
    L.Lbuf = L.Ubuf;
    L.acc = take(sizeof(double) * (size_t)p->n_slices * Ne);
    L.accG = take(sizeof(double) * Ne);
    L.pool = take(sizeof(double) * (size_t)L.max_lanes * kVecsPerLane * Nn);
    L.trace_stride = TR_HDR + std::max(p->n_steps / p->n_slices, p->n_slices);
    L.trace = take(sizeof(unsigned long long) * (size_t)L.max_lanes * L.trace_stride);
    L.xch = take(sizeof(double) * (size_t)L.max_grid * 12 * (p->nx + 2));
    L.total = o;
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
    C.verify = getenv("PT_VERIFY") ? atoi(getenv("PT_VERIFY")) : 1;
    C.extrap = getenv("PT_EXTRAP") ? atoi(getenv("PT_EXTRAP")) : 0;
    C.fp32 = p->precision == PT_FP32_REFINE ? 1 : 0;
    C.max_restarts = 40;
    C.inner_rtol = getenv("PT_INNER_RTOL") ? atof(getenv("PT_INNER_RTOL")) : 1e-5;
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
    double tmo = 20.0;
    if (const char *e = getenv("PT_WAIT_TIMEOUT_S")) tmo = atof(e);
    if (!(tmo > 0.0)) tmo = 20.0;
    C.timeout_ticks = (long long)(tmo * 1e8);
    return C;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

Bufs make_bufs(void *ws, const Layout &L) {
    Bufs B{};
    B.ctl = at<Control>(ws, L.ctl);
    B.bar = at<unsigned>(ws, L.bar);
    B.flags = at<unsigned>(ws, L.flags);
    B.partials = at<double>(ws, L.partials);
    B.wg_group = at<int>(ws, L.wg_group);
    B.groups = at<Group>(ws, L.groups);
    B.lanes = at<Lane>(ws, L.lanes);
    B.FL = at<double>(ws, L.FL);
    B.pool = at<double>(ws, L.pool);
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
    B.trace = at<unsigned long long>(ws, L.trace);
    B.xch = at<double>(ws, L.xch);
    B.trace_stride = L.trace_stride;
    return B;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? PT_OK : PT_EHIP; }

#define PT_TRY(expr)                         \
    do {                                     \
        int _rc = (expr);                    \
        if (_rc != PT_OK) return _rc;        \
    } while (0)

int launch_check() { return hip_ok(hipGetLastError()); }

// Plan of one engine launch, built on the host and passed as a kernel
// argument (so no host buffer must outlive the call). Groups come in runs of
// identical shape: group r of a run gets the lanes with slices
// s0 + r*gstride + k*lstride, k = 0..nlanes-1, kept if within [smin, smax].
struct Run {
    int kind, ngroups, nwg, tile, s0, gstride, lstride, nlanes, smin, smax;
};

struct PlanArgs {
    int grid;
    int nruns;
    Run run[6];
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
            G.tile = R.tile;
            G.vec = gidx;
            G.lane0 = lidx;
            int n = 0;
            for (int k = 0; k < R.nlanes; ++k) {
                const int sl = R.s0 + q * R.gstride + k * R.lstride;
                if (sl < R.smin || sl > R.smax) continue;
                lanes[lidx + n].kind = R.kind;
                lanes[lidx + n].slice = sl;
                ++n;
            }
            G.nlanes = n;
            lidx += n;
            groups[gidx] = G;
            for (int k = 0; k < R.nwg; ++k) wg_group[w++] = gidx;
            ++gidx;
        }
    }
    for (; w < P.grid; ++w) wg_group[w] = -1;
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

int env_int(const char *name, int dflt) {
    const char *e = getenv(name);
    return e ? atoi(e) : dflt;
}

double env_double(const char *name, double dflt) {
    const char *e = getenv(name);
    return e ? atof(e) : dflt;
}

// LDS doubles of the engine for tile size ts: two node windows (ts + 2H) and
// two element windows ((ts-1)/W + 3 rows of nx+2 elements).
size_t engine_lds_doubles(int ts, int W) {
    const size_t H = W + 1;
    return 2 * ((size_t)ts + 2 * H) + 2 * ((size_t)(ts - 1) / W + 3) * (W + 1);
}

int tile_for(int Nn, int nwg, int H, int lds_cap_doubles) {
    int ts = (Nn + nwg - 1) / nwg;
    ts = (ts + 255) / 256 * 256;
    while (ts > 256 && engine_lds_doubles(ts, H - 1) > (size_t)lds_cap_doubles) ts -= 256;
    ts = std::min(ts, std::max(256, env_int("PT_TILE_MAX", 4096)));
    ts = std::max(ts, 256);
    return ts;
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
};

// Runs one engine launch.
int run_engine(const Consts &C, Bufs B, const LaunchInfo &I, std::vector<LanePlan> &plans,
               void *ws, const Layout &Lay, hipStream_t stream) {
    Device dev;
    PT_TRY(device_info(dev));
    const int H = C.W + 1;
    const int lds_cap = std::min(dev.lds_max, 160 * 1024) - 1024;
    const int lds_cap_d = lds_cap / 8;
    int grid = dev.cus * std::max(1, env_int("PT_WG_PER_CU", 1));
    const int sweep_wgs = env_int("PT_SWEEP_WGS", 32);

    const int NT = kThreads;
    const int res_npt_max = std::max(1, std::min(8, env_int("PT_RES_NPT", 8)));
    const int g_min = (C.Nn + NT * res_npt_max - 1) / (NT * res_npt_max);
    bool resident = env_int("PT_RESIDENT", 1) != 0 && g_min <= grid / 4 &&
                    (C.Nn + g_min - 1) / g_min >= H;
    // a tile must be at least one halo (H nodes) long
    const int max_wg_per_lane = std::max(1, C.Nn / H);

    std::vector<int> ngroups(plans.size()), per_group(plans.size()), nwg(plans.size()),
        tile(plans.size());
    if (resident) {
        // one tile of <= NT*npt nodes per workgroup; every group holds a whole lane
        int lat_wgs = 0;
        double wF = 0.0;
        int nq = 0;
        for (size_t k = 0; k < plans.size(); ++k) {
            auto &p = plans[k];
            if (p.latency) {
                nwg[k] = std::max(g_min, std::min(sweep_wgs, grid / 4));
                nwg[k] = std::max(1, std::min(nwg[k], max_wg_per_lane));
                ngroups[k] = p.count;
                lat_wgs += nwg[k] * p.count;
            } else {
                nwg[k] = g_min;
                wF += p.weight * p.count;
                ++nq;
            }
        }
        const int avail = (grid - lat_wgs) / g_min;  // groups left for batched lanes
        if (avail < nq) resident = false;
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
        int total_groups = 0, fixed = 0;
        double wsum = 0.0;
        for (size_t k = 0; k < plans.size(); ++k) {
            auto &p = plans[k];
            const int q = (p.queues <= 0 || p.queues > p.count) ? p.count : p.queues;
            ngroups[k] = q;
            per_group[k] = (p.count + q - 1) / q;
            total_groups += q;
            if (p.latency) fixed += std::max(1, std::min(sweep_wgs, grid / 2)) * q;
            else wsum += p.weight * per_group[k] * q;
        }
        if (total_groups > kMaxLanes) return PT_EINVAL;
        if (total_groups > grid) grid = total_groups;
        const int rest = std::max(grid - fixed, 0);
        for (size_t k = 0; k < plans.size(); ++k) {
            auto &p = plans[k];
            if (p.latency) nwg[k] = std::max(1, std::min(sweep_wgs, grid / 2));
            else nwg[k] = std::max(1, (int)floor(rest * p.weight * per_group[k] / wsum));
            tile[k] = tile_for(C.Nn, nwg[k], H, lds_cap_d);
        }
    }
    int used = 0, max_tile = 256, total_groups = 0;
    for (size_t k = 0; k < plans.size(); ++k) {
        if (nwg[k] > kMaxGroup) return PT_EINVAL;
        used += nwg[k] * ngroups[k];
        total_groups += ngroups[k];
        max_tile = std::max(max_tile, tile[k]);
    }
    if (total_groups > kMaxLanes) return PT_EINVAL;
    if (used > grid) grid = used;
    if (grid > Lay.max_grid) return PT_EINVAL;
    int npt = 0;
    if (resident) {
        npt = 1;
        while (npt * NT < max_tile) npt *= 2;
    }
    const size_t lds_bytes = engine_lds_doubles(max_tile, C.W) * sizeof(double);
    if (lds_bytes > (size_t)dev.lds_max) return PT_EINVAL;

    PlanArgs P{};
    P.grid = grid;
    P.nruns = 0;
    for (size_t k = 0; k < plans.size(); ++k) {
        const auto &p = plans[k];
        if (p.count == 0) continue;
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
    }
    hipLaunchKernelGGL(k_build_plan, dim3(1), dim3(64), 0, stream, P, at<Group>(ws, Lay.groups),
                       at<Lane>(ws, Lay.lanes), at<int>(ws, Lay.wg_group));
    PT_TRY(launch_check());
    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, stream, B.bar, (size_t)kMaxLanes, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, stream, B.flags, (size_t)kMaxFlags, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, stream, (unsigned *)B.trace,
                       (size_t)Lay.max_lanes * Lay.trace_stride * 2, 0u);
    PT_TRY(launch_check());

    const void *kern;
    if (C.fp32)
        kern = npt == 0   ? (const void *)k_engine<0, float>
               : npt == 1 ? (const void *)k_engine<1, float>
               : npt == 2 ? (const void *)k_engine<2, float>
               : npt == 4 ? (const void *)k_engine<4, float>
                          : (const void *)k_engine<8, float>;
    else
        kern = npt == 0   ? (const void *)k_engine<0, double>
               : npt == 1 ? (const void *)k_engine<1, double>
               : npt == 2 ? (const void *)k_engine<2, double>
               : npt == 4 ? (const void *)k_engine<4, double>
                          : (const void *)k_engine<8, double>;
    PT_TRY(hip_ok(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds_bytes)));
    int occ = 0;
    PT_TRY(hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kThreads, lds_bytes)));
    if ((long long)occ * dev.cus < grid) return PT_EHIP;
    void *args[] = {(void *)&C, (void *)&B, (void *)&I};
    PT_TRY(hip_ok(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kThreads), args,
                                             (unsigned)lds_bytes, stream)));
    return launch_check();
}

int setup_design(const pt_problem *p, const Consts &C, const Bufs &B, const double *rho,
                 void *ws, const Layout &Lay, hipStream_t stream) {
    const int blocks = 512;
    // Dirichlet mask
    if (p->bc == PT_BC_MASK) {
        PT_TRY(hip_ok(hipMemcpyAsync(at<unsigned char>(ws, Lay.mask), p->dirichlet_mask,
                                     (size_t)C.Nn, hipMemcpyHostToDevice, stream)));
        PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    } else {
        const int rule = p->bc == PT_BC_LEFT_CENTRE ? 0 : (p->bc == PT_BC_BOTTOM_CENTRE ? 1 : 2);
        hipLaunchKernelGGL(k_mask_rule, dim3(blocks), dim3(256), 0, stream, C, rule,
                           at<unsigned char>(ws, Lay.mask));
    }
    // source history
    if (p->q_t) {
        PT_TRY(hip_ok(hipMemcpyAsync(at<double>(ws, Lay.qt), p->q_t,
                                     sizeof(double) * (p->n_steps + 1), hipMemcpyHostToDevice,
                                     stream)));
        PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    } else {
        hipLaunchKernelGGL(k_fill_f64, dim3(8), dim3(256), 0, stream, at<double>(ws, Lay.qt),
                           (size_t)(p->n_steps + 1), p->q);
    }
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks), dim3(256), 0, stream, at<double>(ws, Lay.zero),
                       (size_t)C.Nn, 0.0);
    hipLaunchKernelGGL(k_material, dim3(blocks), dim3(256), 0, stream, C, rho,
                       at<double>(ws, Lay.kq), at<double>(ws, Lay.cm), at<double>(ws, Lay.dk),
                       at<double>(ws, Lay.dc), p->k0, p->kmin, p->pk, p->c0, p->cmin, p->pc,
                       B.ctl);
    hipLaunchKernelGGL(k_diag, dim3(blocks), dim3(256), 0, stream, C, B.kq, B.cm, B.mask,
                       at<double>(ws, Lay.dinv_f), at<double>(ws, Lay.dinv_c));
    return launch_check();
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b) return false;
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

__global__ void k_reset_ctl(Control *ctl, int keep_markers) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int f = ctl->fwd_done, a = ctl->adj_done;
        ctl->status = 0;
        ctl->abort = 0;
        ctl->max_iters = 0;
        ctl->iters_fine = ctl->iters_coarse = ctl->solves_fine = ctl->solves_coarse = 0;
        ctl->max_relres_bits = 0;
        ctl->fwd_done = keep_markers ? f : 0;
        ctl->adj_done = 0;
        (void)a;
    }
}

}  // namespace

extern "C" {

int pt_validate(const pt_problem *prob) { return valid_problem(prob) ? PT_OK : PT_EINVAL; }

size_t pt_workspace_bytes(const pt_problem *prob) {
    if (!valid_problem(prob)) return 0;
    return layout(prob).total;
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
        default: return "unknown error";
    }
}

int pt_parareal_forward(const pt_problem *prob, const double *rho, const double *guess_T,
                        const double *guess_theta, double *S, double *uT_out, double *utheta_out,
                        double *Theta_out, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!valid_problem(prob)) return PT_EINVAL;
    if (!rho || !S || !Theta_out || !ws) return PT_EINVAL;
    if ((guess_T == nullptr) != (guess_theta == nullptr)) return PT_EINVAL;
    const Layout Lay = layout(prob);
    if (ws_bytes < Lay.total) return PT_ENOMEM;
    const Consts C = make_consts(prob);
    const size_t Nn = C.Nn, Nt1 = C.Ntau + 1;
    const size_t sz_U = Nt1 * Nn * sizeof(double), sz_S = (size_t)C.Nt * Nn * sizeof(double);
    if (guess_T) {
        const void *outs[] = {S, uT_out, utheta_out, Theta_out, ws};
        const size_t lens[] = {sz_S, sz_U, Nt1 * sizeof(double), sizeof(double), ws_bytes};
        for (int k = 0; k < 5; ++k)
            if (overlaps(guess_T, sz_U, outs[k], lens[k]) ||
                overlaps(guess_theta, Nt1 * sizeof(double), outs[k], lens[k]))
                return PT_EINVAL;
    }
    if (overlaps(S, sz_S, ws, ws_bytes) || overlaps(uT_out, sz_U, ws, ws_bytes)) return PT_EINVAL;

    Bufs B = make_bufs(ws, Lay);
    hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, stream, B.ctl, 0);
    PT_TRY(setup_design(prob, C, B, rho, ws, Lay, stream));

    double *outT = uT_out ? uT_out : at<double>(ws, Lay.Ubuf);
    double *outth = utheta_out ? utheta_out : at<double>(ws, Lay.Ubuf_th);
    double *Uprev = at<double>(ws, Lay.Uprev);
    double *Uprev_th = at<double>(ws, Lay.Uprev_th);
    double *Ga = at<double>(ws, Lay.Gk), *Gb = at<double>(ws, Lay.Gn);
    double *Ga_th = at<double>(ws, Lay.Gk_th), *Gb_th = at<double>(ws, Lay.Gn_th);
    const bool cold = guess_T == nullptr;
    const int Ntau = C.Ntau;
    for (int it = 0; it < prob->iterations; ++it) {
        LaunchInfo I{};
        I.cold = (cold && it == 0) ? 1 : 0;
        I.gk_lanes = (!cold && it == 0 && Ntau > 1) ? 1 : 0;
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
        std::vector<LanePlan> plans;
        plans.push_back({F_PRI, Ntau, 0, +1, (double)C.M, false, env_int("PT_FQUEUES", 0)});
        if (I.gk_lanes)
            plans.push_back({GK_PRI, Ntau - 1, 1, +1, env_double("PT_GK_WEIGHT", 4.0), false,
                             env_int("PT_GQUEUES", 0)});
        if (I.cold) plans.push_back({COLD_PRI, 1, 0, +1, 0.0, true, 0});
        if (Ntau > 1) plans.push_back({SWEEP_PRI, 1, 0, +1, 0.0, true, 0});
        PT_TRY(run_engine(C, B, I, plans, ws, Lay, stream));
        if (it + 1 < prob->iterations) {
            hipLaunchKernelGGL(k_copy_f64, dim3(1024), dim3(256), 0, stream, Uprev, outT, Nt1 * Nn);
            hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(256), 0, stream, Uprev_th, outth, Nt1);
            PT_TRY(launch_check());
            std::swap(Ga, Gb);
            std::swap(Ga_th, Gb_th);
        }
    }
    B.out_T = outT;
    B.out_th = outth;
    hipLaunchKernelGGL(k_finalize_fwd, dim3(256), dim3(256), 0, stream, C, B, Theta_out);
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
    const size_t Nn = C.Nn, Nt1 = C.Ntau + 1;
    const size_t sz_U = Nt1 * Nn * sizeof(double);
    if (guess_lambda) {
        if (overlaps(guess_lambda, sz_U, lambda_out, sz_U) ||
            overlaps(guess_lambda, sz_U, ws, ws_bytes))
            return PT_EINVAL;
    }
    if (overlaps(lambda_out, sz_U, ws, ws_bytes)) return PT_EINVAL;
    Bufs B = make_bufs(ws, Lay);
    hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, stream, B.ctl, 1);
    PT_TRY(setup_design(prob, C, B, rho, ws, Lay, stream));

    double *outL = lambda_out ? lambda_out : at<double>(ws, Lay.Lbuf);
    double *Lprev = at<double>(ws, Lay.Lprev);
    double *Ga = at<double>(ws, Lay.Gk), *Gb = at<double>(ws, Lay.Gn);
    const bool cold = guess_lambda == nullptr;
    const int Ntau = C.Ntau;
    for (int it = 0; it < prob->iterations; ++it) {
        LaunchInfo I{};
        I.cold = (cold && it == 0) ? 1 : 0;
        I.gk_lanes = (!cold && it == 0 && Ntau > 1) ? 1 : 0;
        I.has_dc = (prob->c0 != prob->cmin) ? 1 : 0;
        I.epoch = 1;
        B.S = const_cast<double *>(S);
        B.Theta = Theta;
        B.in_L = it == 0 ? guess_lambda : Lprev;
        B.out_L = outL;
        B.Gk = Ga;
        B.Gn = Gb;
        std::vector<LanePlan> plans;
        // the reversed sweep consumes slices from N_tau downwards
        plans.push_back({F_ADJ, Ntau, Ntau, -1, (double)C.M, false, env_int("PT_FQUEUES", 0)});
        if (I.gk_lanes)
            plans.push_back({GK_ADJ, Ntau - 1, Ntau - 1, -1, env_double("PT_GK_WEIGHT", 4.0),
                             false, env_int("PT_GQUEUES", 0)});
        if (I.cold) plans.push_back({COLD_ADJ, 1, 0, +1, 0.0, true, 0});
        if (Ntau > 1) plans.push_back({SWEEP_ADJ, 1, 0, +1, 0.0, true, 0});
        PT_TRY(run_engine(C, B, I, plans, ws, Lay, stream));
        if (it + 1 < prob->iterations) {
            hipLaunchKernelGGL(k_copy_f64, dim3(1024), dim3(256), 0, stream, Lprev, outL, Nt1 * Nn);
            PT_TRY(launch_check());
            std::swap(Ga, Gb);
        }
    }
    B.out_L = outL;
    hipLaunchKernelGGL(k_finalize_adj, dim3(256), dim3(256), 0, stream, C, B);
    return launch_check();
}

int pt_sensitivities(const pt_problem *prob, const double *rho, const void *ws, size_t ws_bytes,
                     double *dTheta_drho, hipStream_t stream) {
    if (!valid_problem(prob)) return PT_EINVAL;
    if (!rho || !ws || !dTheta_drho) return PT_EINVAL;
    const Layout Lay = layout(prob);
    if (ws_bytes < Lay.total) return PT_ENOMEM;
    const Consts C = make_consts(prob);
    void *w = const_cast<void *>(ws);
    hipLaunchKernelGGL(k_sensitivities, dim3(512), dim3(256), 0, stream, C, at<double>(w, Lay.acc),
                       at<double>(w, Lay.accG), dTheta_drho);
    return launch_check();
}

int pt_query_trace(const pt_problem *prob, const void *ws, hipStream_t stream,
                   unsigned long long *out, size_t out_words, int *n_lanes, int *stride) {
    if (!valid_problem(prob) || !ws || !out || !n_lanes || !stride) return PT_EINVAL;
    const Layout Lay = layout(prob);
    PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    const size_t words = (size_t)Lay.max_lanes * Lay.trace_stride;
    const size_t n = std::min(words, out_words);
    PT_TRY(hip_ok(hipMemcpy(out, static_cast<const char *>(ws) + Lay.trace,
                            n * sizeof(unsigned long long), hipMemcpyDeviceToHost)));
    *n_lanes = Lay.max_lanes;
    *stride = Lay.trace_stride;
    return PT_OK;
}

int pt_query_status(const void *ws, hipStream_t stream, pt_stats *out) {
    if (!ws || !out) return PT_EINVAL;
    PT_TRY(hip_ok(hipStreamSynchronize(stream)));
    Control c;
    PT_TRY(hip_ok(hipMemcpy(&c, ws, sizeof(Control), hipMemcpyDeviceToHost)));
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

}  // extern "C"
