// Internal layout shared by the host driver and the HIP kernels of libpt.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace pt {

constexpr int kThreads = 512;       // threads per workgroup of the lane engine
constexpr int kMaxLanes = 512;      // lanes per single-design engine launch
constexpr int kMaxGroups = 1024;    // groups per engine launch
constexpr int kMaxGroup = 1024;     // workgroups per lane group (partials slots)
constexpr int kVecsPerLane = 10;    // x, p, r[2], w[2], s[2], tp, tq
constexpr int kMaxFlags = 4 * 4096; // dependency flags per launch
constexpr int kMaxLevels = 16;      // multigrid levels (level 0 = the element grid)
constexpr int kBarLine = 64;        // words per barrier counter (one 256-B line each)
constexpr int kBarParts = 8;        // counters per group barrier (workgroup b arrives at b % 8)
constexpr int kBarStride = kBarLine * kBarParts;  // words per group's barrier

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
    COLD_ADJ = 7,   // cold coarse sweep v^0_{n-1} = G(v^0_n)
    // coarse propagators on the coarse spatial mesh (propagator PT_COARSE_MESH)
    CM_GK_PRI = 8,     // batched coarse-mesh step G(R u^k_n)
    CM_SWEEP_PRI = 9,  // correction sweep on the coarse mesh
    CM_GK_ADJ = 10,    // batched coarse-mesh adjoint step G(R v^k_n)
    CM_SWEEP_ADJ = 11  // reversed correction sweep on the coarse mesh
};

__host__ __device__ inline bool is_cm_kind(int kind) { return kind >= CM_GK_PRI; }
// lanes of the adjoint pass
__host__ __device__ inline bool is_adjoint_kind(int kind) {
    return (kind >= F_ADJ && kind <= COLD_ADJ) || kind == CM_GK_ADJ || kind == CM_SWEEP_ADJ;
}

// Flag slots (one per slice index per producer kind)
enum FlagKind : int { FL_F = 0, FL_GK = 1, FL_COLD = 2, FL_SWEEP = 3 };

struct Lane {
    int kind;
    int slice;      // n for F/GK lanes; unused for sweeps
    int design;     // index into the launch's design descriptors
    int tile;       // nodes per workgroup tile for this lane on its group
};

// A group of workgroups runs a queue of lanes one after another; its
// workgroups share one barrier counter, one partial-sum slot and one vector set.
// queue < 0: the group owns lanes [lane0, lane0 + nlanes) in order.
// queue >= 0: the group shares queue `queue` (lanes [lane0, lane0 + nlanes))
// with other groups and takes the next untaken lane whenever it is free.
struct Group {
    int wg0, nwg;       // workgroup range
    int lane0, nlanes;  // lane range of the group's (or its queue's) list
    int vec;            // vector set index in the pool
    int queue;          // shared queue index, -1 for a private list
};

// Call-order markers of a single-design workspace: a complete forward pass
// leaves fwd_done = kFwdDone, a complete adjoint pass adj_done = kAdjDone. An
// adjoint without a forward, or sensitivities without an adjoint, report
// kStatusOrder (PT_ESTATE) and write NaN outputs instead of running.
constexpr int kFwdDone = 0x46574431;
constexpr int kAdjDone = 0x41444A31;
constexpr int kStatusOrder = -6;

// Device-side control/status block at the start of the workspace.
struct Control {
    int status;            // first device-side error (PT_* code), 0 if none
    int abort;             // set when a wait times out; every wait then gives up
    int max_iters;         // largest CG count of a solve
    int pad0;
    unsigned long long iters_fine, iters_coarse, solves_fine, solves_coarse;
    unsigned long long max_relres_bits;  // max final ||r||/||b|| as double bits
    int fwd_done, adj_done;              // call-order markers: kFwdDone / kAdjDone once the
                                         // pass finished (finalize kernels), else anything
    int epoch;
    int pad1;
    double grad_scale;  // factor of the summed sensitivities: Theta^{1-p}/p with G = 0, else 1
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
    // material law and source of the setup kernels (Eq. 2.5-2.6)
    double k0, kmin, pk, c0, cmin, pc, q;
    int bc_rule;  // 0 centre of left edge, 1 centre of bottom edge, 2 none, 3 caller mask
    int has_qt;   // q(t) was copied in by the host
    // geometric multigrid preconditioner (gmg != 0): levels l = 0..gmg_L-1 with
    // nx >> l by ny >> l elements; levels < gmg_Lg are smoothed by the whole
    // group, the rest (and the coarsest solve) by one workgroup
    int gmg, gmg_L, gmg_Lg, gmg_tail_sweeps;
    int gmg_chunk, gmg_chunk_init;    // nodes per LDS-staged chunk (rounds / FP64 set-up of a solve)
    // checkpointed storage: S keeps the corrected coarse states T_{Mn} and
    // every slice's first fine state T_{Mn+1}; fine adjoint lanes recompute
    // the other states of their slice
    int ckpt;
    int sweep_x0;  // correction sweeps start from G(u^k_n) + (u^{k+1}_n - u^k_n)
    int plt;       // zero coarse propagators (Sec. 7): fine lanes only, objective Theta^p
    int coarse_iters;  // > 0: coarse propagators are this many CG iterations from their input
    double gmg_omega;                 // smoother damping times the Gershgorin bound
    long long gmg_off[kMaxLevels];    // node offset of level l >= 1 in the level arrays
    long long gmg_nodes;              // sum of the nodes of levels 1..L-1
};

// Pointers of one design: its workspace arrays and the caller's arrays.
struct Bufs {
    Control *ctl;
    unsigned *flags;       // [kMaxFlags] dependency flags of this design
    double *pool;          // group vectors, slot (vec * kVecsPerLane + which) * pool_stride
    size_t pool_stride;    // >= Nn of every design sharing the pool
    double *FL;            // fine adjoint outputs F_adj(v^k_n), lambda part [Ntau+1][Nn]
    const double *rho;     // design densities [Ne]
    double *kq;            // padded k/6   [(ny+2)(nx+2)]
    double *cm;            // padded c*hx*hy/36
    double *dk;            // k'(rho) per element [Ne]
    double *dc;            // c'(rho) per element [Ne]
    double *dinv_f;        // 1/diag of C/dt + K (0 on Dirichlet nodes) [Nn]
    double *dinv_c;        // 1/diag of C/dtau + K
    unsigned char *mask;   // Dirichlet mask [Nn]
    double *qt;            // q(t_n), n = 0..Nt
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
    double *Theta_out;     // device scalar written by the forward finalize
    // adjoint
    const double *Theta;   // device scalar
    const double *in_L;    // guess lambda [Ntau+1][Nn]
    double *out_L;         // [Ntau+1][Nn]
    double *acc;           // per fine adjoint slice sensitivity sums [Ntau][Ne]
    double *accG;          // coarse correction sensitivity sums [Ne]
    double *grad;          // dTheta/drho [Ne] (sensitivity kernel output)
    double *zero;          // Nn zeros
    // multi-design cycles: where the corrected u and lambda are kept as the
    // next cycle's guesses
    double *save_T, *save_th, *save_L;
    // multigrid: Galerkin stencils of levels >= 1 for the fine (dt) and coarse
    // (dtau) operators, [2][9][gmg_nodes] in FP64 and in the CG precision;
    // per operator and level the Gershgorin bound of D^{-1} A and the damping
    double *gA64;
    void *gA;
    void *gA0;             // level-0 stencil rows [2][9][Nn] in the CG precision
    double *gmg_g;         // [2][kMaxLevels]
    double *gmg_w;         // [2][kMaxLevels]
    void *gvec;            // group level vectors [groups][3][gmg_nodes] (CG precision)
    size_t gvec_stride;    // elements per group
    double *ck;            // recomputed fine states per fine adjoint group [slots][M-2][Nn]
    size_t ck_stride;      // elements per slot
};

struct LaunchInfo {
    int cold;        // inputs of this iteration come from the cold sweep lane
    int gk_lanes;    // batched G(u^k_n) lanes are present (warm first iteration)
    int has_dc;      // dC/drho is not identically zero
    unsigned epoch;  // value a set flag holds in this launch
};

// Lane runs of one design in a multi-design launch: the fine lanes (F and, if
// present, G(u^k_n)) go to queue 0, the cold and correction sweeps to queue 1
// (the cold sweeps of all designs ahead of every correction sweep).
struct DesignPlan {
    int q0_lane0, q0_count;  // first lane index and count in the fine queue
    int q1_cold, q1_sweep;   // lane index of the cold / correction sweep (-1: none)
    int tile0, tile1;        // tile of this design's lanes on queue 0 / queue 1 groups
    int adjoint;             // lane kinds of the adjoint pass
};

// Coarse-spatial-mesh propagators (propagator PT_COARSE_MESH): the coarse
// mesh has nx/2 x ny/2 elements; coarse node (I, J) is fine node (2I, 2J).

struct CoarseMesh {
    int nxc, nyc, Wc, Nc, Nec;  // elements per side, nodes per row, nodes, elements
    double *kE, *cE;            // coarse element k and c (means of the fine SIMP values)
    double *A9;                 // [9][Nc] rows of C_c/dtau + K_c without Dirichlet rows/columns
    double *C9;                 // [9][Nc] rows of C_c/dtau (Dirichlet rows zero)
    double *dinv;               // [Nc] 1/diag of A (0 on Dirichlet nodes)
    double *fc;                 // [Nc] int N_I (0 on Dirichlet nodes)
    double *Gk, *Gn;            // [Ntau+1][Nc] coarse outputs G(R u^k_n), G(u^{k+1}_n)
};

// Everything a workgroup needs about one design, read from device memory.
struct EngineDesc {
    Consts C;
    Bufs B;
    LaunchInfo I;
    DesignPlan plan;
    CoarseMesh cm;  // coarse spatial mesh (propagator PT_COARSE_MESH), else unused
};

// Launch-wide arrays shared by every design of one engine launch.
struct Launch {
    const int *wg_group;   // [grid] group of each workgroup (-1: idle)
    const Group *groups;   // [n_groups]
    const Lane *lanes;     // [n_lanes]
    unsigned *bar;         // [kMaxGroups][kBarParts][kBarLine] group barrier counters
    double *partials;      // [kMaxGroups][2][kMaxGroup][4]
    double *xch;           // resident-mode halo exchange [grid][2][2][3][xch_stride]
    int xch_stride;        // >= W + 1 of every design
    unsigned *qhead;       // [2] next untaken position of each shared queue
    int *qslot;            // [kMaxGroups] lane position a group leader took
    unsigned long long *trace;  // per-lane record [n_lanes][trace_stride]
    int trace_stride;           // TR_HDR words + one timestamp per step
    Control *ctl0;         // status block for failures outside any lane
    long long timeout_ticks;
};

// Trace record of one lane (written by its leader): kind, slice, nwg, tile,
// rounds (group barriers), CG iterations, start tick, then the end tick of
// every step. Ticks are the 100 MHz s_memrealtime clock.
enum {
    TR_KIND = 0, TR_SLICE, TR_NWG, TR_TILE, TR_ROUNDS, TR_ITERS, TR_START,
    // phase times (launches with phase timers, else 0):
    TR_T_WORK,    // ticks between the end of one barrier and the arrival at the next
    TR_T_BAR,     // ticks inside group barriers (drain + arrival + wait)
    TR_T_RED,     // ticks reading partial sums after barriers
    TR_T_FLAG,    // ticks waiting on other lanes' flags
    TR_HDR = 12
};

// Host entry points of the coarse-mesh kernels (pt_cmesh.hip); D is the
// uploaded single-design descriptor. Each returns PT_OK or PT_EHIP.
int cm_setup(const EngineDesc *D, const CoarseMesh &M, hipStream_t stream);
// fine guesses of a cold start from the cold sweep's outputs in M.Gk
int cm_guess(const EngineDesc *D, const CoarseMesh &M, int Nn, int Ntau, bool adjoint,
             double *rows, double *th, hipStream_t stream);
int cm_correct(const EngineDesc *D, const CoarseMesh &M, int Nn, int Ntau, bool adjoint, int Ne,
               hipStream_t stream);

}  // namespace pt
