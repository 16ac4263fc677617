/*
 * pt.h -- C ABI of the MI355X (gfx950) hot path of one-shot Parareal topology
 * optimisation for transient heat conduction (Appel & Alexandersen).
 *
 * One optimisation cycle is three calls on one HIP stream:
 *   pt_parareal_forward   modified Parareal for (T, theta)            Sec. 4.3-4.4, Alg. 1
 *   pt_parareal_adjoint   time-reversed vanilla Parareal for lambda   Sec. 4.4, Alg. 2, Eq. 4.14
 *   pt_sensitivities      grad Theta = g_1                            Eq. 4.7, Eq. 4.16
 *
 * Discretisation (Sec. 2.2): unit square, nx x ny rectangular bilinear (Q1)
 * elements, hx = 1/nx, hy = 1/ny, out-of-plane depth 1, element-wise constant
 * k(rho), c(rho) by SIMP (Eq. 2.5-2.6) and uniform source q(t); consistent
 * (Galerkin) capacity matrix; backward Euler with dt = t_final/n_steps
 * (Eq. 2.7); T = 0 on a set of Dirichlet nodes (rows and columns eliminated),
 * insulated elsewhere, T_0 = 0.
 *
 * Layouts: node (i, j) has index j*(nx+1)+i, element (ex, ey) index ey*nx+ex,
 * both row-major with x fastest. All arrays are contiguous FP64.
 *
 * Ownership: every array argument is a DEVICE pointer owned by the caller,
 * except the fields of pt_problem marked HOST. The library allocates no
 * device memory: all scratch lives in the caller's workspace `ws`
 * (pt_workspace_bytes), or, for pt_cycle_noalloc only, in one static device
 * array per GPU. Apart from that array it keeps no global state between
 * calls; state that flows from one call to the next of the same cycle lives
 * in `ws`. Calls are
 * stream-ordered and asynchronous, except where noted; calls that overlap on
 * the same `ws` race.
 *
 * Errors: every entry point returns PT_OK (0) or a negative code. Argument
 * checks run on the host before anything is enqueued. Solver and domain
 * problems found on the device (a CG solve reaching max_iter, Theta <= 0,
 * non-finite values) are recorded in `ws` and reported by pt_query_status.
 */
#ifndef PT_H
#define PT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PT_OK = 0,
    PT_EINVAL = -1,   /* invalid argument (sizes, N_tau not dividing N_t, odd p, NULL, aliasing) */
    PT_ENOMEM = -2,   /* workspace smaller than pt_workspace_bytes()                              */
    PT_EHIP = -3,     /* HIP runtime error (launch, copy) or a device wait that timed out         */
    PT_ENOCONV = -4,  /* some CG solve stopped at max_iter; outputs were still written            */
    PT_EDOMAIN = -5,  /* non-finite input/result or Theta <= 0                                    */
    PT_ESTATE = -6,   /* call order violated (adjoint before forward, sensitivities before adjoint) */
    PT_ESIZE = -7     /* the problem does not fit: it needs more workspace than the static array   */
                      /* of pt_cycle_noalloc, or a launch shape the device cannot hold co-resident */
};

/* Dirichlet node sets */
enum {
    PT_BC_LEFT_CENTRE = 0,   /* x = 0, 0.45 <= y <= 0.55: node (0,j) with 9 ny <= 20 j <= 11 ny */
    PT_BC_BOTTOM_CENTRE = 1, /* y = 0, 0.45 <= x <= 0.55 (the paper's Fig. 4 test case)         */
    PT_BC_NONE = 2,          /* no Dirichlet node (then C/dt + K is still SPD)                  */
    PT_BC_MASK = 3           /* explicit HOST mask, one byte per node, non-zero = T fixed at 0  */
};

enum { PT_FP64 = 0, PT_FP32_REFINE = 1 };
enum { PT_JACOBI = 0, PT_GMG = 1 };
enum { PT_STORE_ALL = 0, PT_CHECKPOINT = 1 };
/* Coarse propagators: the method's G (Alg. 1-2 with dtau); G = 0, the
 * Parallel Local-in-Time form of Sec. 7; or G on a coarser spatial mesh, the
 * cheaper coarse propagator that Sec. 7.3 and Sec. 8 propose (see
 * pt_parareal_forward). */
enum { PT_PARAREAL = 0, PT_PLT = 1, PT_COARSE_MESH = 2 };

/* Execution settings of the calls: launch shapes, lane scheduling, solver
 * details and diagnostics. None of them changes the method; the solver
 * details change CG paths (results within cg_rtol), the others results at
 * most by rounding. pt_default_tuning fills the defaults (in brackets below);
 * pt_problem.tuning == NULL means the defaults. The library reads no
 * environment variables. */
typedef struct pt_tuning {
    int32_t wg_per_cu;         /* engine workgroups per compute unit                        (1)  */
    int32_t resident;          /* -1: resident groups (vectors in registers) where they pay;    */
                               /*  0: streaming groups only; 1: resident wherever they fit  (-1) */
    int32_t resident_npt_max;  /* nodes per thread of a resident tile, 1..8                 (8)  */
    int32_t sweep_wgs;         /* workgroups of a correction-sweep group; 0: by problem size (0) */
    int32_t cm_sweep_wgs;      /* workgroups of a coarse-mesh correction-sweep group        (24) */
    int32_t fine_wgs;          /* > 0: fine lanes on groups of this many workgroups, alike  */
                               /* in both passes; 0: by problem size                         (0) */
    int32_t fine_groups;       /* > 0: groups for the fine lanes; 0: by their work share    (0)  */
    int32_t gk_groups;         /* > 0: groups for the batched coarse steps; 0: by share     (0)  */
    double gk_weight;          /* work of a batched coarse step relative to a fine step     (4)  */
    int32_t lead_fine;         /* 1: a sweep's group first runs the slice the sweep starts  */
                               /* from                                                       (1) */
    int32_t shared_queue;      /* 1: resident fine and batched coarse lanes share a queue   (1)  */
    int32_t tile_max;          /* largest streaming tile in nodes, >= 256                   (4096) */
    int32_t ck_slots;          /* PT_CHECKPOINT: fine-lane groups (recompute slots), >= 1;  */
                               /* fewer if the grid cannot hold them beside the sweeps  (24) */
    int32_t extrap;            /* 1: fine steps start from 2 T_{j-1} - T_{j-2}               (0) */
    int32_t sweep_x0;          /* 1: a sweep step starts from G(u^k_n) + (u^{k+1}_n - u^k_n),  */
                               /* 0: from u^{k+1}_n                                          (1) */
    int32_t verify;            /* 1: the true residual decides a solve's convergence       (1)  */
    double inner_rtol;         /* PT_FP32_REFINE: residual reduction of one FP32 solve     (1e-5) */
    int32_t gmg_tail;          /* PT_GMG: levels of at most this many nodes run on one     */
                               /* workgroup                                                (4096) */
    int32_t gmg_sweeps;        /* PT_GMG: smoothing pairs on the coarsest level            (16)  */
    double gmg_omega;          /* PT_GMG: smoother damping times 1/(Gershgorin bound)      (1.3) */
    int32_t phase_timers;      /* 1: per-round phase times in the lane trace of FP64 launches */
                               /* without coarse-mesh lanes (slows the rounds)              (0) */
    double wait_timeout_s;     /* a device wait gives up after this long (PT_EHIP);        */
                               /* 0: 20 s (60 s in batched launches)                         (0) */
    int32_t gk_lag;            /* shared queue: the batched coarse step of slice n follows  */
                               /* the fine lane of slice n + gk_lag along the sweep, so the */
                               /* long fine lanes start earlier; -1: min(6, N_tau / 5)     (-1) */
} pt_tuning;

typedef struct pt_problem {
    int32_t nx, ny;            /* elements along x and y, >= 1                                   */
    double k0, kmin, pk;       /* k(rho) = kmin + (k0 - kmin) rho^pk            (Eq. 2.6)         */
    double c0, cmin, pc;       /* c(rho) = cmin + (c0 - cmin) rho^pc            (Eq. 2.5)         */
    double q;                  /* uniform source, used when q_t == NULL                           */
    const double *q_t;         /* HOST, optional: q(t_n) for n = 0..n_steps (uniform in space)    */
    double t_final;            /* t_T > 0; dt = t_T / n_steps, dtau = t_T / n_slices              */
    int32_t n_steps;           /* N_t >= 1                                                        */
    int32_t n_slices;          /* N_tau >= 1, must divide N_t; M = N_t / N_tau      (Sec. 4.2)    */
    int32_t pnorm;             /* p, even >= 2                                      (Eq. 2.11)     */
    int32_t iterations;        /* Parareal iterations per pass, >= 1 (1 = one-shot, Alg. 3)       */
    double cg_rtol;            /* stop when ||b - A x||_2 <= cg_rtol ||b||_2, per system, > 0     */
    int32_t max_iter;          /* CG iteration cap per solve, >= 1                                */
    int32_t precision;         /* PT_FP64, or PT_FP32_REFINE: FP32 CG (stencil, vectors, halo)    */
                               /* with FP64 dot products, FP64 x and FP64 residual refinement     */
    int32_t precond;           /* PT_JACOBI, or PT_GMG: geometric multigrid V(1,1) cycle (Galerkin */
                               /* coarse operators, bilinear transfer, damped Jacobi smoothing)   */
    int32_t storage;           /* PT_STORE_ALL: S holds every fine state T_1..T_{N_t}; or          */
                               /* PT_CHECKPOINT: S holds T_{Mn} (rows 0..N_tau-1, n = row+1) and  */
                               /* T_{Mn+1} (rows N_tau..2N_tau-1, n = row-N_tau) and the adjoint  */
                               /* pass recomputes the other fine states of each slice             */
    int32_t bc;                /* PT_BC_*                                                         */
    const uint8_t *dirichlet_mask; /* HOST, (nx+1)(ny+1) bytes, read when bc == PT_BC_MASK        */
    int32_t propagator;        /* PT_PARAREAL (0); PT_PLT: zero coarse propagators (Sec. 7);      */
                               /* PT_COARSE_MESH: coarse propagators on an nx/2 x ny/2 mesh      */
                               /* (nx, ny even; its coarse solves are FP64 Jacobi PCG)         */
    int32_t coarse_iters;      /* 0: coarse steps solved to cg_rtol; k > 0: a cheaper coarse     */
                               /* propagator, exactly k Jacobi-PCG iterations from the step's    */
                               /* input state (PT_FP64, PT_JACOBI and PT_PARAREAL only)         */
    const pt_tuning *tuning;   /* HOST, optional execution settings; NULL: pt_default_tuning    */
} pt_problem;

typedef struct pt_stats {
    int32_t status;            /* PT_OK, PT_ENOCONV or PT_EDOMAIN: first device-side problem     */
    int32_t max_cg_iters;      /* largest CG iteration count of any solve of the last pass       */
    int64_t cg_iters_fine;     /* total CG iterations of fine solves (forward + adjoint)          */
    int64_t cg_iters_coarse;   /* total CG iterations of coarse solves (cold, batched, sweep)    */
    int64_t solves_fine;
    int64_t solves_coarse;
    double max_rel_residual;   /* largest final ||r|| / ||b|| (recursive residual) of any solve  */
} pt_stats;

/* Bytes of device workspace the three calls need for this problem; 0 if the
 * problem is invalid (pt_validate gives the reason). */
size_t pt_workspace_bytes(const pt_problem *prob);

/* Host-side argument check only; returns PT_OK or PT_EINVAL. */
int pt_validate(const pt_problem *prob);

/* The default execution settings (see pt_tuning). PT_EINVAL if out is NULL. */
int pt_default_tuning(pt_tuning *out);

/* Bytes of the state array S: N_t rows of N_n doubles (PT_STORE_ALL) or 2 N_tau
 * rows (PT_CHECKPOINT); 0 if the problem is invalid. */
size_t pt_state_bytes(const pt_problem *prob);

/*
 * Primal pass: Parareal for u_n = (T_{Mn}, theta_{Mn}), n = 0..N_tau (Sec. 4.4,
 * Eq. 4.10 correction applied to T and theta; G_pri = Alg. 1 with dt -> dtau,
 * N_t -> N_tau, load at tau_{n+1}).
 *   rho          [N_e]              design, finite, >= 0 (rho^p with non-integer p needs rho >= 0)
 *   guess_T      [N_tau+1][N_n]     warm-restart guess u^k (Alg. 3), or NULL: cold start from the
 *                                   coarse sweep u^0_{n+1} = G(u^0_n) (Sec. 5.2)
 *   guess_theta  [N_tau+1]          theta part of the guess; NULL iff guess_T is NULL
 *   S            [N_t][N_n]         out: T_1..T_{N_t}; coarse slots T_{Mn} corrected, the other
 *                                   slots the fine states of the last F sweep (Sec. 4.3);
 *                                   with PT_CHECKPOINT [2 N_tau][N_n] as described at `storage`
 *   uT_out       [N_tau+1][N_n]     out: corrected T_{Mn} (the next cycle's guess); may be NULL
 *   utheta_out   [N_tau+1]          out: corrected theta_{Mn}; may be NULL
 *   Theta_out    [1]                out: Theta = theta_{N_t} estimate (device scalar)
 * guess arrays must not overlap any output. Returns PT_OK once enqueued.
 *
 * With propagator == PT_PLT (Sec. 7, Eq. 7.1-7.2) the coarse propagators are
 * zero: each iteration is u^{k+1}_{n+1} = F_pri(u^k_n), u^{k+1}_0 = 0, with u
 * holding T only, and the cold guess is u^0 = 0. No sequential sweep runs.
 * S holds the last iteration's fine trajectories (T_{M(n+1)} = F of u^k_n),
 * uT_out = u^{K}; the objective is the modified Theta~ = Theta^p of Eq. 7.4,
 * summed over those trajectories, and Theta_out = Theta~^{1/p} (Eq. 7.6);
 * utheta_out[n] = (the part of Theta~ before tau_n)^{1/p}. guess_theta is
 * ignored and may be NULL.
 *
 * With propagator == PT_COARSE_MESH the coarse propagators act on a mesh of
 * nx/2 x ny/2 elements whose node (I, J) is fine node (2I, 2J): k and c of a
 * coarse element are the means of its four fine elements' SIMP values, a
 * coarse node is fixed where its fine node is, R is injection and P bilinear
 * interpolation set to 0 at fine Dirichlet nodes. G_pri(T, theta, n) =
 * (P x, theta'), x the coarse backward-Euler step of size dtau from R T with
 * the load at tau_{n+1}, theta' = (theta^p + ||P x||_p^p/(N_tau N_e))^{1/p}.
 * Everything else is as with PT_PARAREAL; the coarse steps are solved to
 * cg_rtol by Jacobi PCG on one workgroup each.
 */
int pt_parareal_forward(const pt_problem *prob, const double *rho, const double *guess_T,
                        const double *guess_theta, double *S, double *uT_out,
                        double *utheta_out, double *Theta_out, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/*
 * Adjoint pass: reversed Parareal for v_n = (lambda_{Mn+1}, g_{Mn+1}), v_{N_tau} = 0
 * (Sec. 4.4, Eq. 4.14; H_adj = Alg. 2 with source Theta^{1-p}/N_e T_n^{o(p-1)}, Eq. 4.6;
 * G_adj = Alg. 2 with dt -> dtau, N_t -> N_tau, n+-1 -> n+-M, so the coarse step from
 * v_n uses source and T at fine index m = M(n-1)+1 and T_{m-M} (T_0 = 0 if m-M < 0)).
 *   S, Theta       from pt_parareal_forward of the same cycle (unchanged since)
 *   guess_lambda   [N_tau+1][N_n]  lambda_{Mn+1} guesses (previous cycle's lambda_out), or NULL
 *                                  for the cold sweep v^0_{n-1} = G(v^0_n); row N_tau is ignored
 *   lambda_out     [N_tau+1][N_n]  out: corrected lambda_{Mn+1}, row N_tau = 0; may be NULL
 * The g part of a guess cancels in the correction, so only lambda is taken.
 * Leaves the per-element sensitivity sums in ws for pt_sensitivities.
 *
 * With propagator == PT_PLT: v^{k+1}_{n-1} = F_adj(v^k_n), v_{N_tau} = 0, cold
 * guess v^0 = 0, for the adjoint of Theta~: source p/N_e T^{o(p-1)} (Eq. 7.5),
 * so lambda_out holds lambda~ = p Theta^{p-1} lambda. The first fine step of
 * slice n takes T_{M(n-1)} from S (the end of slice n-1's trajectory). Theta
 * (the forward's Theta_out) is kept for the back-transform of pt_sensitivities.
 *
 * With propagator == PT_COARSE_MESH: G_adj(lambda, n) = P x, x the coarse
 * adjoint step from R lambda whose source is P^T of the fine source of Eq. 4.6
 * at T_m (m = M(n-1)+1); the sensitivity increment of Eq. 4.16 uses P x on
 * the fine elements.
 */
int pt_parareal_adjoint(const pt_problem *prob, const double *rho, const double *S,
                        const double *Theta, const double *guess_lambda, double *lambda_out,
                        void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * grad Theta = g-part of v_0 (Sec. 4.4 step 4); with PT_PLT the fine terms
 * of Theta~ are summed and scaled by Theta^{1-p}/p (Eq. 7.7):
 *   dTheta_drho[e] = -(1/N_t) sum_fine lambda_j,e^T (dC/drho_e (T_j - T_{j-1})/dt + dK/drho_e T_j)
 *                    - (1/N_tau) (coarse-correction terms)          (Eq. 4.7, Eq. 4.16)
 *   dTheta_drho    [N_e] out
 */
int pt_sensitivities(const pt_problem *prob, const double *rho, const void *ws,
                     size_t ws_bytes, double *dTheta_drho, hipStream_t stream);

/*
 * Lane trace of the last engine launch (profiling aid). Synchronises `stream`
 * and copies up to out_words 64-bit words: n_lanes records of `stride` words,
 * each [kind, slice, workgroups, tile, group barriers, CG iterations,
 * start tick, ticks working, ticks in barriers, ticks reducing, ticks waiting
 * on other lanes, unused, end tick of step 0, 1, ...], ticks of the device's
 * 100 MHz real-time clock; unused records are zero. Lane kinds: 0 fine primal,
 * 1 batched coarse primal, 2 primal sweep, 3 cold primal sweep, 4-7 the adjoint
 * counterparts.
 */
int pt_query_trace(const pt_problem *prob, const void *ws, hipStream_t stream,
                   unsigned long long *out, size_t out_words, int *n_lanes, int *stride);

/* Synchronises `stream`, then reads the device status and counters in ws. */
int pt_query_status(const void *ws, hipStream_t stream, pt_stats *out);

/* Static string for a return code. */
const char *pt_strerror(int code);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * optimisation cycle -- pt_parareal_forward, pt_parareal_adjoint and
 * pt_sensitivities with the arguments of those calls -- whose workspace is a
 * static device array of PT_NOALLOC_WS_BYTES inside the library instead of a
 * caller-owned one. The array exists once per GPU the library runs on and is
 * held until the process ends; the call allocates and frees nothing.
 *   guess_T, guess_theta, guess_lambda  as for the three calls (NULL = cold start)
 *   S, uT_out, utheta_out, lambda_out,  outputs as for the three calls (uT_out,
 *   Theta_out, dTheta_drho              utheta_out, lambda_out may be NULL)
 *   stats_out   [1] DEVICE pt_stats, or NULL: the cycle's status and counters,
 *               written stream-ordered at the end (what pt_query_status reports
 *               after the adjoint and sensitivities of the three-call form)
 * Returns PT_ESIZE when pt_workspace_bytes(prob) > PT_NOALLOC_WS_BYTES, other
 * argument errors as the three calls do, all before anything is enqueued.
 * Every call on one GPU shares that GPU's array and leaves its contents there;
 * each call clears what must start at zero. Calls that overlap on one GPU
 * (other streams, other host threads) race on the array.
 * ------------------------------------------------------------------------ */
#define PT_NOALLOC_WS_BYTES ((size_t)64 << 20)

int pt_cycle_noalloc(const pt_problem *prob, const double *rho, const double *guess_T,
                     const double *guess_theta, const double *guess_lambda, double *S,
                     double *uT_out, double *utheta_out, double *lambda_out, double *Theta_out,
                     double *dTheta_drho, pt_stats *stats_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Design-field front end (Sec. 2.1): chi -> chi_fil = H chi -> chi_phys = P(chi_fil),
 * the input rho of the calls above, and the adjoint of that map.
 *   H: chi_fil_e = sum_i w_ei chi_i / W_e, w_ei = max(0, r_fil - |x_e - x_i|),
 *      W_e = sum_i w_ei, over element centroids x_e = ((i+1/2)/nx, (j+1/2)/ny)
 *      (elements off the grid are left out of both sums);
 *   P: (tanh(beta (x - eta)) + tanh(beta eta)) / (tanh(beta (1 - eta)) + tanh(beta eta))
 *      (the identity when beta <= 0).
 * Element arrays are [N_e] FP64 device arrays, element (i, j) at j nx + i.
 * ------------------------------------------------------------------------ */
typedef struct pt_filter {
    int32_t nx, ny;            /* elements along x and y, 1..16384                               */
    double r_fil;              /* filter radius > 0 in unit-square coordinates; a radius of      */
                               /* more than 255 elements (either direction) is rejected          */
    double beta;               /* projection sharpness; <= 0: no projection                      */
    double eta;                /* projection threshold in [0, 1]                                  */
} pt_filter;

/* Host-side check of a filter description: PT_OK or PT_EINVAL. */
int pt_filter_validate(const pt_filter *f);

/* chi_fil (may be NULL) and chi_phys from chi. No array may overlap another.
 * Returns PT_OK once enqueued. */
int pt_filter_projection(const pt_filter *f, const double *chi, double *chi_fil, double *chi_phys,
                         hipStream_t stream);

/* grad_chi = H^T (P'(chi_fil) o grad_phys): the gradient with respect to chi of a
 * function whose gradient with respect to chi_phys is grad_phys. chi_fil is the
 * forward's output; work is caller-owned [N_e] scratch, overwritten. No array
 * may overlap another. Returns PT_OK once enqueued. */
int pt_filter_projection_backward(const pt_filter *f, const double *chi_fil,
                                  const double *grad_phys, double *work, double *grad_chi,
                                  hipStream_t stream);

/* ------------------------------------------------------------------------
 * Many designs in one cycle (one persistent launch per pass for all designs).
 *
 * Each design is an independent problem of its own grid and slice count; all
 * designs of a batch share `precision` and take one Parareal iteration
 * (iterations == 1). One call runs a whole optimisation cycle of every design
 * (Sec. 4.4 steps 1-4): the primal passes of all designs in one engine launch,
 * the adjoint passes of all designs in a second launch, then the sensitivities.
 * The workspace keeps each design's S, its corrected coarse states u_n and
 * adjoint states v_n; with warm = 1 the next call restarts every design from
 * them (the one-shot warm restart of Alg. 3), so consecutive warm calls must
 * pass the same `probs` and the same workspace. Apart from caller masks and
 * q(t) (host copies), a call enqueues kernels only and can be captured in a
 * graph; the engine launch is then a plain launch of a grid that the
 * occupancy check has shown to be co-resident.
 * ------------------------------------------------------------------------ */

/* Worker shapes of a multi-design launch. Lanes (a slice's fine propagator or
 * a batched coarse step; a design's coarse sweep) are taken from two queues by
 * groups of workgroups: `sweep_groups` groups of `sweep_wgs` workgroups run
 * the sequential coarse sweeps, the rest of the grid is cut into groups of
 * `fine_wgs` workgroups for the fine and batched coarse lanes. */
typedef struct pt_batch_tuning {
    int32_t fine_wgs;      /* workgroups per fine-lane group, 1..1024                         */
    int32_t sweep_wgs;     /* workgroups per sweep group, 1..1024                             */
    int32_t sweep_groups;  /* sweep groups, >= 1                                              */
    int32_t resident;      /* 1: vectors held in registers (every design's tile must fit)   */
    int32_t grid;          /* workgroups of the launch, 0 = as many as are co-resident        */
    int32_t tile_max;      /* streaming (resident = 0): largest node tile a workgroup stages  */
                           /* per pass, 256..16384, or 0 for the built-in 4096               */
    int32_t reserved[2];
} pt_batch_tuning;

/* Workspace bytes of a batch of n designs; 0 if any problem is invalid, the
 * precisions differ, or a design has iterations != 1, storage != PT_STORE_ALL,
 * propagator != PT_PARAREAL (PT_PLT, PT_COARSE_MESH) or coarse_iters != 0. */
size_t pt_batched_workspace_bytes(int n, const pt_problem *probs);

/* The built-in worker shapes for n designs. */
int pt_batch_default_tuning(int n, pt_batch_tuning *out);

/*
 * One optimisation cycle of n designs.
 *   probs        [n] HOST problem descriptions (as for the single-design calls)
 *   rho          [n] HOST array of device pointers, rho[k] has probs[k].nx*ny elements
 *   warm         0: cold start from the coarse sweeps; 1: restart from the previous call's
 *                solution kept in ws
 *   tuning       worker shapes, or NULL for pt_batch_default_tuning
 *   Theta_out    [n] device array: Theta of every design
 *   dTheta_drho  [n] HOST array of device pointers to [N_e] outputs, or NULL: the primal
 *                pass only (Theta_out); the next warm call then restarts the adjoint
 *                from the last full cycle's lambda, or from lambda = 0 after a cold
 *                forward-only call
 * Outputs must not overlap ws. Device-side problems are reported per design
 * by pt_batched_status.
 */
int pt_parareal_batched(int n, const pt_problem *probs, const double *const *rho, int warm,
                        const pt_batch_tuning *tuning, double *Theta_out,
                        double *const *dTheta_drho, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* Synchronises `stream` and reads the status and counters of every design. */
int pt_batched_status(int n, const pt_problem *probs, const void *ws, hipStream_t stream,
                      pt_stats *out /* [n] */);

/* Picks the launch shape of this batch by timing whole warm cycles: a
 * coordinate descent, two passes from the defaults, over resident vs
 * streaming vectors, fine_wgs, sweep_wgs, sweep_groups and the streaming
 * tile_max. Synchronous. It runs one cold cycle first; every timed cycle then
 * restarts from that cycle's solution, which stays in ws as the warm state
 * (the timed cycles do not replace it). A shape's time is the median of three
 * cycles; shapes the batch cannot use, or whose cycle reports any device-side
 * problem (PT_ENOCONV included), are skipped. Leaves the outputs of the last
 * timed cycle.
 *   best, best_ms   the fastest shape and its time
 *   default_ms      may be NULL: the time of the built-in shape, from the same
 *                   state (so best_ms <= default_ms)
 *   progress, user  may be NULL: called on the host after each shape is timed,
 *                   with the shape, its time in ms (+inf if unusable) and user */
typedef void (*pt_autotune_progress)(const pt_batch_tuning *shape, double ms, void *user);
int pt_autotune_batched(int n, const pt_problem *probs, const double *const *rho,
                        double *Theta_out, double *const *dTheta_drho, void *ws,
                        size_t ws_bytes, hipStream_t stream, pt_batch_tuning *best,
                        double *best_ms, double *default_ms, pt_autotune_progress progress,
                        void *user);

#ifdef __cplusplus
}
#endif

#endif /* PT_H */
