// Internal layout shared by the host driver and the HIP kernels of libpt.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace pt {

constexpr int kThreads = 512;       // threads per workgroup of the lane engine
constexpr int kMaxLanes = 512;      // lanes per engine launch
constexpr int kMaxGroup = 1024;     // workgroups per lane group (partials slots)
constexpr int kVecsPerLane = 10;    // x, p, r[2], w[2], s[2], tp, tq
constexpr int kMaxFlags = 4 * 4096; // dependency flags per launch

// Lane kinds: a lane is a sequence of linear solves executed by one group of
// workgroups; lanes of one launch run concurrently and meet only through flags.
enum LaneKind : int {
    F_PRI = 0,      // fine primal propagator of slice n: M backward-Euler steps (Alg. 1, dt)
    GK_PRI = 1,     // coarse primal step from the guess u^k_n (batched G(u^k_n))
    SWEEP_PRI = 2,  // sequential correction sweep u^{k+1}_{n+1} = G(u^{k+1}_n) + F_n - G(u^k_n)
    COLD_PRI = 3,   // cold coarse sweep u^0_{n+1} = G(u^0_n)
    F_ADJ = 4,      // fine adjoint propagator of slice n: M steps (Alg. 2, dt)
    GK_ADJ = 5,     // coarse adjoint step from the guess v^k_n
    SWEEP_ADJ = 6,  // reversed correction sweep
    COLD_ADJ = 7    // cold coarse sweep v^0_{n-1} = G(v^0_n)
};

// Flag slots (one per slice index per producer kind)
enum FlagKind : int { FL_F = 0, FL_GK = 1, FL_COLD = 2, FL_SWEEP = 3 };

struct Lane {
    int kind;
    int slice;      // n for F/GK lanes; unused for sweeps
};

// A group of workgroups runs a queue of lanes one after another; its
// workgroups share one barrier counter, one partial-sum slot and one vector set.
struct Group {
    int wg0, nwg;     // workgroup range
    int lane0, nlanes;  // lanes [lane0, lane0 + nlanes) in queue order
    int tile;         // nodes per tile
    int vec;          // vector set index in the pool
};

// Device-side control/status block at the start of the workspace.
struct Control {
    int status;            // first device-side error (PT_* code), 0 if none
    int abort;             // set when a wait times out; every wait then gives up
    int max_iters;         // largest CG count of a solve
    int pad0;
    unsigned long long iters_fine, iters_coarse, solves_fine, solves_coarse;
    unsigned long long max_relres_bits;  // max final ||r||/||b|| as double bits
    int fwd_done, adj_done;              // call-order markers (written by finalize kernels)
    int epoch;
    int pad1;
};

struct Consts {
    int nx, ny, W, Nn, Ne, EW;  // W = nx+1 nodes per row, EW = nx+2 padded elements per row
    int Nt, Ntau, M, p;
    int max_iter, verify;
    int extrap;  // fine steps start from the linear extrapolation 2 T_{j-1} - T_{j-2}
    int fp32;          // CG in FP32 inside FP64 iterative refinement
    int max_restarts;  // FP64 refinement steps per solve (FP32 mode)
    double inner_rtol; // relative residual reduction of one FP32 inner solve
    double hx, hy;
    double e_self, e_x, e_y, e_d;   // stiffness stencil factors (times k/6)
    double cm_unit;                  // hx*hy/36
    double quarter_area;             // hx*hy/4
    double dt, dtau, inv_dt, inv_dtau;
    double rtol;
    double inv_NtNe, inv_NtauNe, inv_p;
    long long timeout_ticks;         // s_memrealtime ticks before a wait gives up
};

// Pointers into the workspace and the caller's arrays for one engine launch.
struct Bufs {
    Control *ctl;
    unsigned *bar;         // [kMaxLanes] group barrier counters (one per group)
    unsigned *flags;       // [kMaxFlags]
    double *partials;      // [kMaxLanes][2][kMaxGroup][4] (one block per group)
    const int *wg_group;   // [grid] group of each workgroup (-1: idle)
    const Group *groups;   // [n_groups]
    const Lane *lanes;     // [n_lanes]
    double *pool;          // group vectors [n_groups][kVecsPerLane][Nn]
    double *FL;            // fine adjoint outputs F_adj(v^k_n), lambda part [Ntau+1][Nn]
    const double *kq;      // padded k/6   [(ny+2)(nx+2)]
    const double *cm;      // padded c*hx*hy/36
    const double *dk;      // k'(rho) per element [Ne]
    const double *dc;      // c'(rho) per element [Ne]
    const double *dinv_f;  // 1/diag of C/dt + K (0 on Dirichlet nodes) [Nn]
    const double *dinv_c;  // 1/diag of C/dtau + K
    const unsigned char *mask;  // Dirichlet mask [Nn]
    const double *qt;      // q(t_n), n = 0..Nt
    // primal
    const double *in_T;    // guess u^k (warm) [Ntau+1][Nn]
    const double *in_th;   // [Ntau+1]
    double *S;             // [Nt][Nn]
    double *out_T;         // corrected u^{k+1} [Ntau+1][Nn]
    double *out_th;        // [Ntau+1]
    double *Gk;            // G(u^k_n) [Ntau+1][Nn]   (read)
    double *Gk_th;         // [Ntau+1]
    double *Gn;            // G(u^{k+1}_n) written by the sweep [Ntau+1][Nn]
    double *Gn_th;
    double *F_th;          // theta part of F(u^k_n) [Ntau]
    // adjoint
    const double *Theta;   // device scalar
    const double *in_L;    // guess lambda [Ntau+1][Nn]
    double *out_L;         // [Ntau+1][Nn]
    double *acc;           // per fine adjoint slice sensitivity sums [Ntau][Ne]
    double *accG;          // coarse correction sensitivity sums [Ne]
    const double *zero;    // Nn zeros
    double *xch;           // resident-mode halo exchange [grid][2 parities][2 sides][3][W+2]
    unsigned long long *trace;  // per-lane record [n_lanes][trace_stride]
    int trace_stride;           // 8 header words + one timestamp per step
};

// Trace record of one lane (written by its leader): kind, slice, nwg, tile,
// rounds (group barriers), CG iterations, start tick, then the end tick of
// every step. Ticks are the 100 MHz s_memrealtime clock.
enum {
    TR_KIND = 0, TR_SLICE, TR_NWG, TR_TILE, TR_ROUNDS, TR_ITERS, TR_START,
    TR_T_WORK,    // ticks between the end of one barrier and the arrival at the next
    TR_T_BAR,     // ticks inside group barriers (drain + arrival + wait)
    TR_T_RED,     // ticks reading partial sums after barriers
    TR_T_FLAG,    // ticks waiting on other lanes' flags
    TR_HDR = 12
};

struct LaunchInfo {
    int cold;        // inputs of this iteration come from the cold sweep lane
    int gk_lanes;    // batched G(u^k_n) lanes are present (warm first iteration)
    int has_dc;      // dC/drho is not identically zero
    unsigned epoch;  // value a set flag holds in this launch
};

}  // namespace pt
