// Lane engine: one persistent cooperative launch runs every propagator of one
// Parareal pass (Sec. 4.2-4.4) on gfx950.
//
// A *lane* is a sequence of backward-Euler solves (C/delta + K) x = b: the
// fine propagator of one time slice (M steps of Alg. 1 or Alg. 2 with dt), one
// batched coarse step G(u^k_n), the cold coarse sweep, or the sequential
// correction sweep (Eq. 4.10 / Eq. 4.14). A *group* of workgroups runs a queue of
// lanes one after another. All groups of a pass run concurrently; a lane waits
// on a device flag only where the method has a true data dependence (the
// sweep step n needs F_n and G(u^k_n); a cold-started slice needs its coarse
// guess). Fine slices are queued in the order the sweep consumes them, so the
// latency-bound sequential sweep overlaps the bandwidth-bound fine slices.
//
// Each solve is a Jacobi-preconditioned conjugate gradient in the single-
// reduction form of Chronopoulos and Gear: one group barrier per iteration,
// which both publishes the halo values of the iteration's vectors and combines
// the dot products (r,z), (z,Az), (r,r). The workgroups of a group own
// contiguous node ranges ("tiles"); every tile is staged in LDS with a halo of
// one grid row plus one node on each side, so the 9-point Q1 stencil reads LDS
// only. The halo values of z = D^{-1} r_{i+1} are recomputed locally from
// r_i, w_i, s_{i-1} (pointwise), which is why one barrier per iteration
// suffices; vectors that neighbours read in the same round are double-buffered
// by iteration parity.
//
// Round data shared between workgroups (lane vectors, partial sums) is moved
// with device-coherent (agent-scope) loads and stores, and a barrier drains
// the workgroup's memory counters before its relaxed arrival increment; this
// avoids the cache-wide write-back / invalidate of agent-scope fences, which
// dominate a round on a multi-XCD part. Full release/acquire fences are kept
// where a lane hands results to another lane (flags) and where a lane's plain
// stores must become visible to other groups.
//
// Control state (step, phase, alpha, beta, theta ...) is replicated: every
// workgroup of a group reduces the same partial sums in the same order and
// takes the same decisions. Reductions are deterministic (fixed order).
#include "pt_internal.h"

namespace pt {

namespace {

enum Phase : int { PH_INIT = 0, PH_FIRST = 1, PH_ITER = 2, PH_POST = 3, PH_DONE = 4 };

constexpr int kWaves = kThreads / 64;
constexpr int kU = 4;  // independent loads in flight per thread in streaming loops

__device__ __forceinline__ double ipow(double x, int n) {
    double r = 1.0, b = x;
    while (n) {
        if (n & 1) r *= b;
        b *= b;
        n >>= 1;
    }
    return r;
}

// pow through a call of its own: inlined, the library routine's registers
// raise the engine's peak pressure and push round values into scratch
__device__ __noinline__ double pow_call(double x, double y) { return pow(x, y); }

__device__ __forceinline__ long long now_ticks() {
    return (long long)__builtin_amdgcn_s_memrealtime();
}

// device-coherent accesses for data exchanged between workgroups within a launch
__device__ __forceinline__ double ldc(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ldc(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Marker of a Dirichlet node in an own-node residual slot of the streaming
// rounds' LDS (D^{-1} is exactly 0 there, and the residual is 0): a NaN bit
// pattern that is only ever stored and compared, never used in arithmetic.
__device__ __forceinline__ double dir_tag(double) {
    return __longlong_as_double(0x7FF8D1D1D1D1D1D1LL);
}
__device__ __forceinline__ float dir_tag(float) { return __int_as_float(0x7FC5D1D1); }
__device__ __forceinline__ bool is_dir_tag(double v) {
    return __double_as_longlong(v) == 0x7FF8D1D1D1D1D1D1LL;
}
__device__ __forceinline__ bool is_dir_tag(float v) { return __float_as_int(v) == 0x7FC5D1D1; }
__device__ __forceinline__ int ldc(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_status(Control *ctl, int code) {
    atomicCAS(&ctl->status, 0, code);
}

__device__ __forceinline__ bool aborted(Control *ctl) {
    return __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Workgroup barrier for LDS only: waits for this wave's LDS operations and
// synchronises the waves, but leaves global loads and stores in flight
// (__syncthreads also drains the vector memory counter, which would expose a
// memory round trip at every intra-workgroup sync). Global data is never
// exchanged between threads of a workgroup within a round.
__device__ __forceinline__ void lds_sync() {
    asm volatile("" ::: "memory");
    // lgkmcnt(0); vmcnt and expcnt left at their maxima (no wait)
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Group barrier of g workgroups. Every wave first waits for its own memory
// operations (the device-coherent stores of this round) to complete; thread 0
// then increments one of the group's counters, and the first wave spins until
// the counters sum to all g workgroups' arrivals, reading them in one load of
// up to eight lanes. Groups of kBarSplit or more workgroups spread their
// arrivals over kBarParts counters (workgroup b on counter b % 8): device-scope
// atomics on one address are performed one after another, which queued a large
// group's arrivals on the round's critical path; smaller groups keep one
// counter, where polling eight lines cost more than it saved. With `release`,
// thread 0 also issues an agent-scope release fence first, which publishes
// this workgroup's plain stores to other XCDs.
// Returns false on timeout or when another workgroup aborted. Each counter has
// a cache line of its own, and the spin reads the shared abort flag only every
// 64th turn: the groups' polls then do not contend for one line.
// SPLIT = false: always one counter. Every barrier of one group must count
// its arrivals the same way: the engine instance with coarse-mesh lanes uses
// one counter for all its groups (its registers are scarcer), the others
// split by group size.
constexpr int kBarSplit = 20;

template <bool SPLIT = true>
__device__ bool group_barrier(unsigned *cnt, unsigned g, unsigned target, Control *ctl,
                              long long timeout, bool release) {
    __shared__ int s_ok;
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if constexpr (!SPLIT) {
        // one counter: thread 0 arrives and spins
        if (threadIdx.x == 0) {
            if (release) __threadfence();
            __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int ok = 1;
            long long t0 = now_ticks();
            unsigned spins = 0;
            while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if ((++spins & 63u) == 0 && (aborted(ctl) || now_ticks() - t0 > timeout)) {
                    ok = 0;
                    break;
                }
            }
            s_ok = ok;
        }
    } else if (threadIdx.x < 64) {
        // thread 0 arrives at counter b % parts; the first wave reads the
        // counters in one load and sums them in scalar registers
        const int lane = threadIdx.x;
        const int parts = g >= (unsigned)kBarSplit ? kBarParts : 1;
        if (lane == 0) {
            if (release) __threadfence();
            __hip_atomic_fetch_add(cnt + (blockIdx.x % parts) * kBarLine, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        int ok = 1;
        long long t0 = now_ticks();
        unsigned spins = 0;
        for (;;) {
            const unsigned v = lane < parts ? __hip_atomic_load(cnt + lane * kBarLine,
                                                                __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT)
                                            : 0u;
            unsigned sum = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
            if (parts > 1) {
#pragma unroll
                for (int k = 1; k < kBarParts; ++k)
                    sum += (unsigned)__builtin_amdgcn_readlane((int)v, k);
            }
            if (sum >= target) break;
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 63u) == 0 && (aborted(ctl) || now_ticks() - t0 > timeout)) {
                ok = 0;
                break;
            }
        }
        if (lane == 0) s_ok = ok;
    }
    __syncthreads();
    asm volatile("" ::: "memory");
    return s_ok != 0;
}

// Wait until flags[idx] == epoch (set by a producer group's leader), then
// acquire at agent scope so the producer's plain stores are visible.
__device__ bool wait_flag(unsigned *flags, int idx, unsigned epoch, Control *ctl,
                          long long timeout) {
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        int ok = 1;
        long long t0 = now_ticks();
        while (__hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
               epoch) {
            __builtin_amdgcn_s_sleep(2);
            if (aborted(ctl) || now_ticks() - t0 > timeout) {
                ok = 0;
                break;
            }
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Called by thread 0 of the group leader after a release barrier.
__device__ void set_flag(unsigned *flags, int idx, unsigned epoch) {
    __threadfence();
    __hip_atomic_store(&flags[idx], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int flag_index(int kind, int n) { return kind * 4096 + n; }

// Deterministic block sum of Q values; every thread receives the totals.
template <int Q>
__device__ __forceinline__ void block_sum(double (&v)[Q], double *red) {
    for (int q = 0; q < Q; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[q] = x;
    }
    // per-call address math: a hoisted LDS address is held in a spilled
    // register, and its reload waits for every store still in flight
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int wave = tid >> 6;
    if ((tid & 63) == 0)
        for (int q = 0; q < Q; ++q) red[wave * Q + q] = v[q];
    lds_sync();
    for (int q = 0; q < Q; ++q) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += red[w * Q + q];
        v[q] = t;
    }
    lds_sync();
}

// Sum partials[0..g)[0..Q) in a fixed order (identical in every workgroup).
// Each thread loads one value (entry e: workgroup e / Q, component e % Q), so
// the loads of a round are all in flight at once; loading a workgroup's Q
// values in one thread made the compiler reuse one register pair and wait
// for each load in turn.
template <int Q>
__device__ void group_sum(const double *part, int g, double (&out)[Q], double *red) {
    double v[Q];
    for (int q = 0; q < Q; ++q) v[q] = 0.0;
    // per-call index math (a hoisted, spilled address would be reloaded
    // behind a wait for every load in flight)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    for (int e = tid; e < g * Q; e += kThreads) {
        const int r = e / Q, q = e - r * Q;
        const double x = ldc(part + r * 4 + q);
#pragma unroll
        for (int k = 0; k < Q; ++k) v[k] += (k == q) ? x : 0.0;
    }
    block_sum<Q>(v, red);
    for (int q = 0; q < Q; ++q) out[q] = v[q];
}

// Nine stencil coefficients of node (i, j): mass part scaled by ms (= 1/delta
// or 0), conductivity part scaled by ks (1 or 0). Element contributions follow
// the bilinear element matrices of an hx x hy rectangle: per element with
// m = c hx hy/(36 delta) and kap = k/6, self 4m + kap e_self, x-neighbour
// 2m + kap e_x, y-neighbour 2m + kap e_y, diagonal m + kap e_d.
struct Coef {
    double c, e, w, n, s, ne, nw, se, sw;
};

__device__ __forceinline__ Coef node_coef(const Consts &C, const double *kq, const double *cm,
                                          int i, int j, double ms, double ks) {
    const int eSW = j * C.EW + i, eSE = eSW + 1, eNW = eSW + C.EW, eNE = eNW + 1;
    const double mSW = cm[eSW] * ms, mSE = cm[eSE] * ms, mNW = cm[eNW] * ms, mNE = cm[eNE] * ms;
    const double kSW = kq[eSW] * ks, kSE = kq[eSE] * ks, kNW = kq[eNW] * ks, kNE = kq[eNE] * ks;
    Coef a;
    a.c = 4.0 * (mSW + mSE + mNW + mNE) + C.e_self * (kSW + kSE + kNW + kNE);
    a.e = 2.0 * (mSE + mNE) + C.e_x * (kSE + kNE);
    a.w = 2.0 * (mSW + mNW) + C.e_x * (kSW + kNW);
    a.n = 2.0 * (mNW + mNE) + C.e_y * (kNW + kNE);
    a.s = 2.0 * (mSW + mSE) + C.e_y * (kSW + kSE);
    a.ne = mNE + C.e_d * kNE;
    a.nw = mNW + C.e_d * kNW;
    a.se = mSE + C.e_d * kSE;
    a.sw = mSW + C.e_d * kSW;
    return a;
}

// Same, with k/6 and c hx hy/36 read from LDS element windows that start at
// padded element index ea.
__device__ __forceinline__ Coef node_coef_l(const Consts &C, const double *LK, const double *LC,
                                            int ea, int i, int j, double ms, double ks) {
    const int eSW = j * C.EW + i - ea, eSE = eSW + 1, eNW = eSW + C.EW, eNE = eNW + 1;
    const double mSW = LC[eSW] * ms, mSE = LC[eSE] * ms, mNW = LC[eNW] * ms, mNE = LC[eNE] * ms;
    const double kSW = LK[eSW] * ks, kSE = LK[eSE] * ks, kNW = LK[eNW] * ks, kNE = LK[eNE] * ks;
    Coef a;
    a.c = 4.0 * (mSW + mSE + mNW + mNE) + C.e_self * (kSW + kSE + kNW + kNE);
    a.e = 2.0 * (mSE + mNE) + C.e_x * (kSE + kNE);
    a.w = 2.0 * (mSW + mNW) + C.e_x * (kSW + kNW);
    a.n = 2.0 * (mNW + mNE) + C.e_y * (kNW + kNE);
    a.s = 2.0 * (mSW + mSE) + C.e_y * (kSW + kSE);
    a.ne = mNE + C.e_d * kNE;
    a.nw = mNW + C.e_d * kNW;
    a.se = mSE + C.e_d * kSE;
    a.sw = mSW + C.e_d * kSW;
    return a;
}

// Element rows a node tile [a, b) touches: padded rows a/W .. (b-1)/W + 1.
__device__ __forceinline__ void elem_window(const Consts &C, int a, int b, int &ea, int &elen) {
    const int ja = a / C.W, jb = (b - 1) / C.W;
    ea = ja * C.EW;
    elen = (jb - ja + 2) * C.EW;
}

// Stage kq, cm of the element window into LDS (coalesced, several loads in flight).
__device__ __forceinline__ void stage_elems(const Bufs &B, int ea, int elen, double *LK,
                                            double *LC) {
    for (int q0 = threadIdx.x; q0 < elen; q0 += kThreads * 4) {
        double kv[4], cv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * kThreads;
            kv[u] = q < elen ? B.kq[ea + q] : 0.0;
            cv[u] = q < elen ? B.cm[ea + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * kThreads;
            if (q < elen) {
                LK[q] = kv[u];
                LC[q] = cv[u];
            }
        }
    }
}

__device__ __forceinline__ double apply(const Coef &a, const double *L, int li, int W) {
    return a.c * L[li] + a.e * L[li + 1] + a.w * L[li - 1] + a.n * L[li + W] + a.s * L[li - W] +
           a.ne * L[li + W + 1] + a.nw * L[li + W - 1] + a.se * L[li - W + 1] +
           a.sw * L[li - W - 1];
}

// The CG working precision (FP64, or FP32 inside FP64 refinement): the same
// coefficients rounded to Real and the stencil evaluated in Real.
template <typename Real>
struct CoefT {
    Real c, e, w, n, s, ne, nw, se, sw;
};

template <typename Real>
__device__ __forceinline__ CoefT<Real> node_coef_t(const Consts &C, const double *LK,
                                                   const double *LC, int ea, int i, int j,
                                                   double ms, double ks) {
    const Coef a = node_coef_l(C, LK, LC, ea, i, j, ms, ks);
    CoefT<Real> r;
    r.c = (Real)a.c;
    r.e = (Real)a.e;
    r.w = (Real)a.w;
    r.n = (Real)a.n;
    r.s = (Real)a.s;
    r.ne = (Real)a.ne;
    r.nw = (Real)a.nw;
    r.se = (Real)a.se;
    r.sw = (Real)a.sw;
    return r;
}

template <typename Real>
__device__ __forceinline__ Real apply_t(const CoefT<Real> &a, const Real *L, int li, int W) {
    return a.c * L[li] + a.e * L[li + 1] + a.w * L[li - 1] + a.n * L[li + W] + a.s * L[li - W] +
           a.ne * L[li + W + 1] + a.nw * L[li + W - 1] + a.se * L[li - W + 1] +
           a.sw * L[li - W - 1];
}


// lambda^T K0 T and lambda^T C0 D of one element (unit k and c), local node
// order (ex,ey), (ex+1,ey), (ex+1,ey+1), (ex,ey+1).
__device__ __forceinline__ double elem_k(const Consts &C, double l0, double l1, double l2,
                                         double l3, double t0, double t1, double t2, double t3) {
    const double self = l0 * t0 + l1 * t1 + l2 * t2 + l3 * t3;
    const double xa = l0 * t1 + l1 * t0 + l2 * t3 + l3 * t2;
    const double ya = l0 * t3 + l3 * t0 + l1 * t2 + l2 * t1;
    const double dg = l0 * t2 + l2 * t0 + l1 * t3 + l3 * t1;
    return (C.e_self * self + C.e_x * xa + C.e_y * ya + C.e_d * dg) * (1.0 / 6.0);
}

__device__ __forceinline__ double elem_c(const Consts &C, double l0, double l1, double l2,
                                         double l3, double d0, double d1, double d2, double d3) {
    const double self = l0 * d0 + l1 * d1 + l2 * d2 + l3 * d3;
    const double adj = l0 * d1 + l1 * d0 + l2 * d3 + l3 * d2 + l0 * d3 + l3 * d0 + l1 * d2 +
                       l2 * d1;
    const double dg = l0 * d2 + l2 * d0 + l1 * d3 + l3 * d1;
    return C.cm_unit * (4.0 * self + 2.0 * adj + dg);
}

// Primal steps a fine adjoint lane recomputes before its adjoint steps when
// only checkpoints are stored: T_{M(n-1)+2} .. T_{Mn-1} of its slice.
__device__ __forceinline__ int ck_recompute(const Consts &C) {
    return C.ckpt ? max(C.M - 2, 0) : 0;
}

// The stored state T_j (1 <= j <= N_t). With checkpoints, T_{Mn} lives in row
// n-1 and T_{Mn+1} in row N_tau+n of S; the other states of a slice exist only
// in the recomputing lane's scratch (nullptr elsewhere).
__device__ __forceinline__ double *srow(const Consts &C, const Bufs &B, int j, double *scratch) {
    if (!C.ckpt) return B.S + (size_t)(j - 1) * C.Nn;
    if (j % C.M == 0) return B.S + (size_t)(j / C.M - 1) * C.Nn;
    if ((j - 1) % C.M == 0) return B.S + (size_t)(C.Ntau + (j - 1) / C.M) * C.Nn;
    return scratch ? scratch + (size_t)((j - 1) % C.M - 1) * C.Nn : nullptr;
}

// Per-lane, per-step description derived identically in every workgroup.
struct StepInfo {
    bool fine;        // delta = dt (else dtau)
    bool adjoint;
    int n;            // coarse index of coarse kinds / slice of fine kinds
    int j;            // fine time index: load index (primal) or source index (adjoint)
    int jprev;        // adjoint: index of T_{j-1} or T_{m-M} (<= 0 means T_0 = 0)
    const double *tp_src;  // vector for C/delta * tp (RHS); coherent loads
    const double *x0_src;  // initial guess; nullptr means "x already holds it"
    bool wait;        // a flag must be awaited before INIT
    int wait_idx;
    bool extrap;      // x0 = 2 x - tq (two previous states of a fine lane)
    bool recompute;   // a primal step recomputed inside a fine adjoint lane
    int s_adj;        // adjoint step index of a fine adjoint lane (step - recomputed steps)
    // x0 = x0_src + (d1 - d0) when d1 != nullptr: a correction sweep step starts
    // from G(u^k_n) plus the correction u^{k+1}_n - u^k_n of its input
    const double *d1, *d0;
};

__device__ __forceinline__ int lane_steps(const Consts &C, int kind) {
    switch (kind) {
        case F_PRI: return C.M;
        case F_ADJ: return C.M + ck_recompute(C);
        case GK_PRI:
        case GK_ADJ: return 1;
        case SWEEP_PRI:
        case SWEEP_ADJ: return C.Ntau - 1;
        default: return C.Ntau;  // cold sweeps
    }
}

enum { V_X = 0, V_P = 1, V_R0 = 2, V_R1 = 3, V_W0 = 4, V_W1 = 5, V_S0 = 6, V_S1 = 7, V_TP = 8, V_TQ = 9 };

__device__ __forceinline__ double *group_vec(const Bufs &B, int vec, int which) {
    return B.pool + ((size_t)vec * kVecsPerLane + which) * B.pool_stride;
}

__device__ StepInfo step_info(const Consts &C, const Bufs &B, const LaunchInfo &I, const Lane &L,
                              int s, const double *tpbuf) {
    StepInfo st;
    const size_t Nn = C.Nn;
    st.wait = false;
    st.wait_idx = 0;
    st.jprev = 0;
    st.extrap = C.extrap && (L.kind == F_PRI || L.kind == F_ADJ) && s >= 2;
    st.recompute = false;
    st.s_adj = 0;
    st.d1 = st.d0 = nullptr;
    switch (L.kind) {
        case F_PRI: {
            const int n = L.slice;
            st.fine = true;
            st.adjoint = false;
            st.n = n;
            st.j = C.M * n + s + 1;
            if (s == 0) {
                const double *src;
                if (I.cold) {
                    src = (n == 0) ? B.zero : B.Gk + (size_t)(n - 1) * Nn;
                    if (n > 0) {
                        st.wait = true;
                        st.wait_idx = flag_index(FL_COLD, n - 1);
                    }
                } else {
                    // with G = 0 a cold pass starts every slice from u^0_n = 0
                    src = (n == 0 || B.in_T == nullptr) ? B.zero : B.in_T + (size_t)n * Nn;
                }
                st.tp_src = src;
                st.x0_src = src;
            } else {
                st.tp_src = tpbuf;
                st.x0_src = nullptr;
            }
            break;
        }
        case GK_PRI: {
            const int n = L.slice;
            st.fine = false;
            st.adjoint = false;
            st.n = n;
            st.j = C.M * (n + 1);
            st.tp_src = B.in_T + (size_t)n * Nn;
            st.x0_src = B.in_T + (size_t)(n + 1) * Nn;
            break;
        }
        case COLD_PRI: {
            const int n = s;
            st.fine = false;
            st.adjoint = false;
            st.n = n;
            st.j = C.M * (n + 1);
            if (n == 0) {
                st.tp_src = B.zero;
                st.x0_src = B.zero;
            } else {
                st.tp_src = tpbuf;
                st.x0_src = nullptr;
            }
            break;
        }
        case SWEEP_PRI: {
            const int n = s + 1;
            st.fine = false;
            st.adjoint = false;
            st.n = n;
            st.j = C.M * (n + 1);
            st.tp_src = (n == 1) ? srow(C, B, C.M, nullptr) : tpbuf;
            st.x0_src = B.Gk + (size_t)n * Nn;
            if (C.sweep_x0 && I.gk_lanes) {
                st.d1 = st.tp_src;
                st.d0 = B.in_T + (size_t)n * Nn;
            }
            break;
        }
        case F_ADJ: {
            const int n = L.slice;
            const int rc = ck_recompute(C);
            if (s < rc) {
                // recompute T_{M(n-1)+s+2} from the stored first state of the slice
                st.fine = true;
                st.adjoint = false;
                st.recompute = true;
                st.n = n;
                st.j = C.M * (n - 1) + s + 2;
                if (s == 0) {
                    const double *src = srow(C, B, st.j - 1, nullptr);
                    st.tp_src = src;
                    st.x0_src = src;
                } else {
                    st.tp_src = tpbuf;
                    st.x0_src = nullptr;
                }
                break;
            }
            s -= rc;
            st.s_adj = s;
            st.fine = true;
            st.adjoint = true;
            st.n = n;
            st.j = C.M * n - s;
            st.jprev = st.j - 1;
            if (s == 0) {
                const double *src;
                if (n == C.Ntau) {
                    src = B.zero;
                } else if (I.cold) {
                    src = B.Gk + (size_t)(n + 1) * Nn;
                    st.wait = true;
                    st.wait_idx = flag_index(FL_COLD, n + 1);
                } else {
                    src = B.in_L == nullptr ? B.zero : B.in_L + (size_t)n * Nn;
                }
                st.tp_src = src;
                st.x0_src = src;
            } else {
                st.tp_src = tpbuf;
                st.x0_src = nullptr;
            }
            break;
        }
        case GK_ADJ: {
            const int n = L.slice;
            st.fine = false;
            st.adjoint = true;
            st.n = n;
            st.j = C.M * (n - 1) + 1;
            st.jprev = st.j - C.M;
            st.tp_src = B.in_L + (size_t)n * Nn;
            st.x0_src = B.in_L + (size_t)(n - 1) * Nn;
            break;
        }
        case COLD_ADJ: {
            const int n = C.Ntau - s;
            st.fine = false;
            st.adjoint = true;
            st.n = n;
            st.j = C.M * (n - 1) + 1;
            st.jprev = st.j - C.M;
            if (n == C.Ntau) {
                st.tp_src = B.zero;
                st.x0_src = B.zero;
            } else {
                st.tp_src = tpbuf;
                st.x0_src = nullptr;
            }
            break;
        }
        default: {  // SWEEP_ADJ
            const int n = C.Ntau - 1 - s;
            st.fine = false;
            st.adjoint = true;
            st.n = n;
            st.j = C.M * (n - 1) + 1;
            st.jprev = st.j - C.M;
            st.tp_src = (n == C.Ntau - 1) ? B.FL + (size_t)C.Ntau * Nn : tpbuf;
            st.x0_src = B.Gk + (size_t)n * Nn;
            if (C.sweep_x0 && I.gk_lanes) {
                st.d1 = st.tp_src;
                st.d0 = B.in_L + (size_t)n * Nn;
            }
            break;
        }
    }
    // truncated coarse solves: the coarse propagator is a fixed number of CG
    // iterations from its input state, so its start may depend on nothing else
    if (C.coarse_iters > 0 && !st.fine) {
        st.x0_src = st.tp_src;
        st.d1 = st.d0 = nullptr;
    }
    return st;
}

struct Ctl {
    int step, nsteps, phase, iter, it_local, restarts;
    bool verifying, zero_x;
    double alpha, beta, gamma;
    double bnorm, relres;
    double r0n;        // ||r|| at the last (re)start of CG
    double theta;      // primal: theta carried by the lane
    double src_scale;  // adjoint: Theta^{1-p} / N_e
};

// Per-element sensitivity term lambda^T (dk K0 T + dc C0 (T - Tp)/delta) of the
// element whose lower-left node is id (Eq. 4.7 summand for one element).
// States written earlier in the same launch by other workgroups (recomputed
// checkpoint states, coh = true) are read with device-coherent loads.
__device__ __forceinline__ double ld_state(const double *row, int q, bool coh) {
    return coh ? ldc(row + q) : row[q];
}

__device__ __forceinline__ double sens_term(const Consts &C, const Bufs &B, const LaunchInfo &I,
                                            int id, int e, double l0, double l1, double l2,
                                            double l3, const double *Tr, const double *Tp,
                                            double inv_delta, bool coh) {
    const double t0 = ld_state(Tr, id, coh), t1 = ld_state(Tr, id + 1, coh),
                 t2 = ld_state(Tr, id + C.W + 1, coh), t3 = ld_state(Tr, id + C.W, coh);
    double term = B.dk[e] * elem_k(C, l0, l1, l2, l3, t0, t1, t2, t3);
    if (I.has_dc) {
        double p0 = 0, p1 = 0, p2 = 0, p3 = 0;
        if (Tp) {
            p0 = ld_state(Tp, id, coh);
            p1 = ld_state(Tp, id + 1, coh);
            p2 = ld_state(Tp, id + C.W + 1, coh);
            p3 = ld_state(Tp, id + C.W, coh);
        }
        term += B.dc[e] * inv_delta *
                elem_c(C, l0, l1, l2, l3, t0 - p0, t1 - p1, t2 - p2, t3 - p3);
    }
    return term;
}

}  // namespace

#include "pt_gmg.hip"
#include "pt_cm_lane.hip"

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------

// Material (Eq. 2.5-2.6): padded k/6 and c hx hy/36, derivatives k', c'.
// Setup of every design of a launch (blockIdx.y = design): Dirichlet mask of
// the standard rules (PT_BC_*), the source history q(t_n) when it is constant,
// the zero vector, and the SIMP material of Eq. 2.5-2.6 per element:
// kq = k(rho)/6 and cm = c(rho) hx hy / 36 on a zero-padded element grid,
// dk = k'(rho), dc = c'(rho). Negative or non-finite densities set PT_EDOMAIN.
__global__ void k_setup_design(const EngineDesc *__restrict__ D) {
    const EngineDesc &E = D[blockIdx.y];
    const Consts &C = E.C;
    const Bufs &B = E.B;
    const int stride = gridDim.x * blockDim.x;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (C.bc_rule != 3) {
        for (int id = t0; id < C.Nn; id += stride) {
            const int j = id / C.W, i = id - j * C.W;
            unsigned char m = 0;
            if (C.bc_rule == 0) m = (i == 0 && 9 * C.ny <= 20 * j && 20 * j <= 11 * C.ny) ? 1 : 0;
            if (C.bc_rule == 1) m = (j == 0 && 9 * C.nx <= 20 * i && 20 * i <= 11 * C.nx) ? 1 : 0;
            B.mask[id] = m;
        }
    }
    if (!C.has_qt)
        for (int n = t0; n <= C.Nt; n += stride) B.qt[n] = C.q;
    for (int id = t0; id < C.Nn; id += stride) B.zero[id] = 0.0;
    const int EH = C.ny + 2;
    const int total = EH * C.EW;
    for (int t = t0; t < total; t += stride) {
        const int py = t / C.EW, px = t - py * C.EW;
        const int ex = px - 1, ey = py - 1;
        double kv = 0.0, cv = 0.0;
        if (ex >= 0 && ex < C.nx && ey >= 0 && ey < C.ny) {
            const int e = ey * C.nx + ex;
            const double r = B.rho[e];
            if (!(r >= 0.0) || !isfinite(r)) set_status(B.ctl, -5);
            const double rr = r > 0.0 ? r : 0.0;
            const double kk = C.kmin + (C.k0 - C.kmin) * pow(rr, C.pk);
            const double cc = C.cmin + (C.c0 - C.cmin) * pow(rr, C.pc);
            B.dk[e] = C.pk * (C.k0 - C.kmin) * pow(rr, C.pk - 1.0);
            B.dc[e] = C.pc * (C.c0 - C.cmin) * pow(rr, C.pc - 1.0);
            kv = kk * (1.0 / 6.0);
            cv = cc * C.cm_unit;
        }
        B.kq[t] = kv;
        B.cm[t] = cv;
    }
}

// Jacobi inverse diagonals of C/dt + K and C/dtau + K (0 on Dirichlet nodes),
// blockIdx.y = design.
__global__ void k_diag(const EngineDesc *__restrict__ D) {
    const EngineDesc &E = D[blockIdx.y];
    const Consts &C = E.C;
    const Bufs &B = E.B;
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < C.Nn; id += gridDim.x * blockDim.x) {
        const int j = id / C.W, i = id - j * C.W;
        const Coef af = node_coef(C, B.kq, B.cm, i, j, C.inv_dt, 1.0);
        const Coef ac = node_coef(C, B.kq, B.cm, i, j, C.inv_dtau, 1.0);
        const bool d = B.mask[id] != 0;
        B.dinv_f[id] = d ? 0.0 : 1.0 / af.c;
        B.dinv_c[id] = d ? 0.0 : 1.0 / ac.c;
    }
}

// Reset of each design's status block (blockIdx.x = design). An adjoint call
// (keep_markers = 1) keeps the forward-done marker and starts in the call-order
// error state if no complete forward pass left it.
__global__ void k_reset_ctl(const EngineDesc *__restrict__ D, int keep_markers) {
    if (threadIdx.x == 0) {
        Control *ctl = D[blockIdx.x].B.ctl;
        const int f = ctl->fwd_done;
        ctl->status = (keep_markers && f != kFwdDone) ? kStatusOrder : 0;
        ctl->abort = 0;
        ctl->max_iters = 0;
        ctl->iters_fine = ctl->iters_coarse = ctl->solves_fine = ctl->solves_coarse = 0;
        ctl->max_relres_bits = 0;
        ctl->fwd_done = keep_markers ? f : 0;
        ctl->adj_done = 0;
        ctl->grad_scale = 1.0;
    }
}

__global__ void k_fill_u32(unsigned *p, size_t n, unsigned v) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        p[t] = v;
}

__global__ void k_fill_f64(double *p, size_t n, double v) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        p[t] = v;
}

__global__ void k_copy_f64(double *dst, const double *src, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

// ---------------------------------------------------------------------------
// The engine
// ---------------------------------------------------------------------------
// MULTI: lanes of several designs read their descriptor from D; otherwise the
// single design's descriptor E1 is a kernel argument (cheaper scalar access).
// CMESH: the launch holds coarse-mesh lanes (single design only); they run
// from the uploaded descriptor D. TIMED: per-round phase times go to the lane
// trace (a separate instance: reading the clock is a scalar memory access, and
// the waits for it and the timers' registers cost a round about a microsecond).
template <int NPT, typename Real, bool MULTI, bool CMESH = false, bool TIMED = false>
__global__ void __launch_bounds__(kThreads) k_engine(const EngineDesc *__restrict__ D, Launch S,
                                                     EngineDesc E1) {
    static_assert(!(MULTI && CMESH), "coarse-mesh lanes run in single-design launches");
    static_assert(!(TIMED && (MULTI || CMESH)), "phase timers in plain single-design launches");
    extern __shared__ double lds[];
    __shared__ double red[kWaves * 4];

    const int gid = S.wg_group[blockIdx.x];
    if (gid < 0) return;
    // an adjoint pass with no forward pass before it does not run (every
    // workgroup reads the same status, written before the launch)
    if constexpr (!MULTI) {
        if (E1.B.ctl->status == kStatusOrder) return;
    }
    const Group G = S.groups[gid];
    const int rank = blockIdx.x - G.wg0;
    const int g = G.nwg;
    unsigned *bar = S.bar + (size_t)gid * kBarStride;
    double *part = S.partials + (size_t)gid * 2 * kMaxGroup * 4;
    unsigned nbar = 0;
    const int XS = S.xch_stride;  // launch-wide halo slot length (>= H of every design)

    // resident mode (NPT > 0): this workgroup's tile values of p, r, w, s live
    // in registers across rounds, D^{-1} of the tile in LDS, x in global memory
    // (updated in place each round); the tile's element window is staged once
    // per lane.
    constexpr int NR = NPT > 0 ? NPT : 1;
    Real rp[NR], rr[NR], rw[NR], rs[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) rp[k] = rr[k] = rw[k] = rs[k] = 0;
    Real *XCH = reinterpret_cast<Real *>(S.xch);

    // phase timers of the current lane (kept by thread 0 of rank 0, written to
    // the trace) in the TIMED instance
    constexpr bool timers = TIMED;
    unsigned long long t_work = 0, t_bar = 0, t_red = 0, t_flag = 0;
    long long t_mark = 0;
    if constexpr (timers) t_mark = now_ticks();
    const bool timer = timers && (rank == 0 && threadIdx.x == 0);
    auto my_part = [&](int parity) { return part + ((size_t)parity * kMaxGroup + rank) * 4; };
    auto all_part = [&](int parity) { return part + (size_t)parity * kMaxGroup * 4; };

    Control *ctl = S.ctl0;  // status block of the lane being run
    bool ok = true;
    for (int li = 0; ok; ++li) {
        int lane_id;
        if (G.queue < 0) {
            if (li >= G.nlanes) break;
            lane_id = G.lane0 + li;
        } else {
            // shared queue: the group leader takes the next position and the
            // barrier hands it to the group's other workgroups
            if (rank == 0 && threadIdx.x == 0)
                stc(S.qslot + gid, (int)__hip_atomic_fetch_add(S.qhead + G.queue, 1u,
                                                               __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT));
            ++nbar;
            ok = group_barrier<!CMESH>(bar, (unsigned)g, nbar * (unsigned)g, ctl,
                                       S.timeout_ticks, false);
            if (!ok) break;
            const int pos = ldc(S.qslot + gid);
            if (pos >= G.nlanes) break;
            lane_id = G.lane0 + pos;
        }
        const Lane L = S.lanes[lane_id];
        if constexpr (CMESH) {
            if (is_cm_kind(L.kind)) {
                ctl = E1.B.ctl;
                const long long r =
                    cm_lane(D, L.kind, L.slice, rank, g, G.vec, bar, part, nbar,
                            S.trace + (size_t)lane_id * S.trace_stride, S.trace_stride - TR_HDR);
                if (r < 0) {
                    ok = false;
                    break;
                }
                nbar = (unsigned)r;
                continue;
            }
            // no register value of a resident lane outlives its lane: with
            // them dead at the coarse-mesh call, the call saves none of them
#pragma unroll
            for (int k = 0; k < NR; ++k) rp[k] = rr[k] = rw[k] = rs[k] = 0;
        }
        const EngineDesc &E = [&]() -> const EngineDesc & {
            if constexpr (MULTI) return D[L.design];
            else return E1;
        }();
        const Consts &C = E.C;
        const Bufs &B = E.B;
        const LaunchInfo &I = E.I;
        ctl = B.ctl;
        const long long tmo = C.timeout_ticks;
        const int H = C.W + 1;  // halo on each side of a tile window
        const int TS = L.tile;
        const int win = TS + 2 * H;
        const int ewin = ((TS - 1) / C.W + 3) * C.EW;  // element window bound
        double *LA = lds;        // window A (halo'd)
        double *LB = lds + win;  // window B (INIT) / own residuals (ITER)
        double *LK = lds + 2 * win;          // k/6 of the tile's elements
        double *LC = lds + 2 * win + ewin;   // c hx hy/36 of the tile's elements
        const int ntiles = (C.Nn + TS - 1) / TS;

        double *X = group_vec(B, G.vec, V_X);
        // recomputed fine states of a checkpointed fine adjoint lane
        double *LSc = (C.ckpt && L.kind == F_ADJ) ? B.ck + (size_t)G.vec * B.ck_stride : nullptr;
        Real *P = reinterpret_cast<Real *>(group_vec(B, G.vec, V_P));
        double *TP = group_vec(B, G.vec, V_TP);
        double *TQ = group_vec(B, G.vec, V_TQ);
        auto rv_ = [&](int which) { return reinterpret_cast<Real *>(group_vec(B, G.vec, which)); };
        Real *Rb[2] = {rv_(V_R0), rv_(V_R1)};
        Real *Wb[2] = {rv_(V_W0), rv_(V_W1)};
        Real *Sb[2] = {rv_(V_S0), rv_(V_S1)};
        Real *LZ = reinterpret_cast<Real *>(LA);  // z window of the CG rounds
        Real *LR = reinterpret_cast<Real *>(LB);  // own residuals of the CG rounds
        Real *LD = LR;  // resident: D^{-1} of the tile (the INIT window is free after FIRST)
        int ea_res = 0;
        // resident: bit k set if this thread's k-th tile node is a Dirichlet node
        // (read once per lane; a per-round byte load per node would serialise a
        // cache round trip per node behind the unrolled stencil)
        unsigned dmask = 0;
        if constexpr (NPT > 0) {
            const int a = min(rank * TS, C.Nn);
            const int b = min(a + TS, C.Nn);
            int elen = 0;
            lds_sync();
            if (a < b) {
                elem_window(C, a, b, ea_res, elen);
                stage_elems(B, ea_res, elen, LK, LC);
            }
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int id = a + (int)threadIdx.x + k * kThreads;
                if (id < b && B.mask[id]) dmask |= 1u << k;
            }
            lds_sync();
        }
        // boundary values of r, w, s for the neighbours' halos: the first H nodes
        // of the tile go to side 0 (read by rank-1), the last H to side 1 (rank+1)
        auto publish = [&](int id, int a, int b, Real r, Real w, Real sv, int par) {
            const int off = id - a;
            if (off < H && rank > 0) {
                Real *base = XCH + (((size_t)blockIdx.x * 2 + par) * 2 + 0) * 3 * XS;
                stc(base + off, r);
                stc(base + XS + off, w);
                stc(base + 2 * XS + off, sv);
            }
            const int o2 = off - ((b - a) - H);
            if (o2 >= 0 && rank < g - 1) {
                Real *base = XCH + (((size_t)blockIdx.x * 2 + par) * 2 + 1) * 3 * XS;
                stc(base + o2, r);
                stc(base + XS + o2, w);
                stc(base + 2 * XS + o2, sv);
            }
        };
        (void)publish;
        auto barrier = [&](bool release) -> bool {
            ++nbar;
            if constexpr (!timers) {
                return group_barrier<!CMESH>(bar, (unsigned)g, nbar * (unsigned)g, ctl, tmo,
                                             release);
            } else {
                const long long t0 = now_ticks();
                const bool r = group_barrier<!CMESH>(bar, (unsigned)g, nbar * (unsigned)g, ctl,
                                                     tmo, release);
                const long long t1 = now_ticks();
                if (timer) {
                    t_work += t0 - t_mark;
                    t_bar += t1 - t0;
                    t_mark = t1;
                }
                return r;
            }
        };
        auto mark_red = [&]() {
            if constexpr (timers) {
                const long long t = now_ticks();
                if (timer) {
                    t_red += t - t_mark;
                    t_mark = t;
                }
            }
        };
        auto waitf = [&](int idx) -> bool {
            if constexpr (!timers) {
                return wait_flag(B.flags, idx, I.epoch, ctl, tmo);
            } else {
                const long long t0 = now_ticks();
                const bool r = wait_flag(B.flags, idx, I.epoch, ctl, tmo);
                const long long t1 = now_ticks();
                if (timer) {
                    t_work += t0 - t_mark;
                    t_flag += t1 - t0;
                    t_mark = t1;
                }
                return r;
            }
        };

        // One preconditioned round of CG with the multigrid preconditioner B
        // (streaming engine): with `update`, first the pointwise CG update
        // s = w + be s, p = u + be p, x += al p, r -= al s; then u = B r by a
        // V(1,1) cycle over the levels (group passes with a barrier between
        // dependent passes, the small levels by workgroup 0 alone), then
        // w = A u and the partial dot products (r,u), (u,w)[, (r,r)].
        auto gmg_round = [&](const StepInfo &st, bool update, bool first, double al, double be,
                             double *loc, int nloc) -> bool {
            const int op = st.fine ? 0 : 1;
            const double *dinv0 = st.fine ? B.dinv_f : B.dinv_c;
            // level 0: r = R, pre-smoothed u1 = U, the round's result u = UB0;
            // levels >= 1 in the group slot of the level arrays
            Real *R = Rb[0], *Wv = Wb[0], *Sv = Sb[0], *U = Rb[1], *UB0 = Wb[1];
            Real *GV = reinterpret_cast<Real *>(B.gvec) + (size_t)G.vec * B.gvec_stride;
            const size_t gn = (size_t)C.gmg_nodes;
            auto lr = [&](int l) -> Real * { return l == 0 ? R : GV + C.gmg_off[l]; };
            auto la = [&](int l) -> Real * { return l == 0 ? U : GV + gn + C.gmg_off[l]; };
            auto lb = [&](int l) -> Real * { return l == 0 ? UB0 : GV + 2 * gn + C.gmg_off[l]; };
            auto omega = [&](int l) -> Real { return (Real)B.gmg_w[op * kMaxLevels + l]; };
            Real *LV = reinterpret_cast<Real *>(lds);  // staged operand window
            // assembled stencil row of level l (CG precision, zero rows on
            // Dirichlet nodes of level 0)
            auto row = [&](int l, int id, Real(&a)[9]) {
                const Real *A = l == 0 ? reinterpret_cast<const Real *>(B.gA0) +
                                             (size_t)op * 9 * C.Nn + id
                                       : reinterpret_cast<const Real *>(B.gA) +
                                             (size_t)op * 9 * gn + C.gmg_off[l] + id;
                const size_t st9 = l == 0 ? (size_t)C.Nn : gn;
#pragma unroll
                for (int k = 0; k < 9; ++k) a[k] = A[(size_t)k * st9];
            };
            auto apply_lds = [&](const Real(&a)[9], int li, int W) -> Real {
                return a[0] * LV[li] + a[1] * LV[li + 1] + a[2] * LV[li - 1] + a[3] * LV[li + W] +
                       a[4] * LV[li - W] + a[5] * LV[li + W + 1] + a[6] * LV[li + W - 1] +
                       a[7] * LV[li - W + 1] + a[8] * LV[li - W - 1];
            };
            auto dinv_row = [&](int l, int id, const Real(&a)[9]) -> Real {
                if (l == 0) return (Real)dinv0[id];
                return a[0] != (Real)0 ? (Real)1 / a[0] : (Real)0;
            };
            // Nodes [a, b) of level l in LDS-sized chunks. The chunk's operand
            // window (one grid row and one node of halo on each side) is staged
            // with coalesced device-coherent loads: value(id) = v[id], plus the
            // bilinear prolongation of e when e is given (0 on Dirichlet nodes
            // of level 0). Then, kU nodes per thread at a time, ld(id) issues a
            // node's loads and op(id, li, W, vals) computes and stores.
            auto staged = [&](int l, const Real *v, const Real *e, int a, int b, auto &&ld,
                              auto &&opf) {
                const Lvl Lv = gmg_level(C, l);
                const int Hl = Lv.W + 1;
                for (int c0 = a; c0 < b; c0 += C.gmg_chunk) {
                    const int c1 = min(c0 + C.gmg_chunk, b);
                    const int lo = c0 - Hl, len = (c1 - c0) + 2 * Hl;
                    lds_sync();
                    for (int q0 = threadIdx.x; q0 < len; q0 += kThreads * kU) {
                        Real vv[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            Real x = 0;
                            if (q < len && id >= 0 && id < Lv.Nn) {
                                x = ldc(v + id);
                                if (e) x += gmg_prolong<Real>(C, l, id, e);
                                if (l == 0 && B.mask[id]) x = 0;
                            }
                            vv[u] = x;
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int q = q0 + u * kThreads;
                            if (q < len) LV[q] = vv[u];
                        }
                    }
                    lds_sync();
                    for (int id0 = c0 + threadIdx.x; id0 < c1; id0 += kThreads * kU) {
                        decltype(ld(0)) vals[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int id = id0 + u * kThreads;
                            if (id < c1) vals[u] = ld(id);
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int id = id0 + u * kThreads;
                            if (id < c1) opf(id, id - lo, Lv.W, vals[u]);
                        }
                    }
                }
            };
            auto own_range = [&](int l, int &a, int &b) {
                const int Nl = gmg_level(C, l).Nn;
                const int ts = (Nl + g - 1) / g;
                a = min(rank * ts, Nl);
                b = min(a + ts, Nl);
            };
            auto own = [&](int l, auto &&f) {
                int a, b;
                own_range(l, a, b);
                for (int id = a + threadIdx.x; id < b; id += kThreads) f(id);
            };
            auto whole = [&](int l, auto &&f) {
                const int Nl = gmg_level(C, l).Nn;
                for (int id = threadIdx.x; id < Nl; id += kThreads) f(id);
            };
            // between passes of the single-workgroup levels: every wave's
            // device-coherent stores must have landed before another wave of
            // the workgroup reads them back from L2
            auto wg_sync = [&]() {
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                asm volatile("" ::: "memory");
            };
            struct RowR {
                Real a[9];
                Real r;
            };
            // lb_l = r_l - A_l la_l on nodes [a, b)
            auto resid_pass = [&](int l, int a, int b) {
                staged(l, la(l), nullptr, a, b,
                       [&](int id) {
                           RowR x;
                           row(l, id, x.a);
                           x.r = ldc(lr(l) + id);
                           return x;
                       },
                       [&](int id, int li, int W, const RowR &x) {
                           stc(lb(l) + id, x.r - apply_lds(x.a, li, W));
                       });
            };
            // dst = v + omega D^{-1} (r - A v), v = src (+ P e) staged
            auto smooth_pass = [&](int l, const Real *src, const Real *e, Real *dst, int a, int b) {
                staged(l, src, e, a, b,
                       [&](int id) {
                           RowR x;
                           row(l, id, x.a);
                           x.r = ldc(lr(l) + id);
                           return x;
                       },
                       [&](int id, int li, int W, const RowR &x) {
                           stc(dst + id, LV[li] + omega(l) * dinv_row(l, id, x.a) *
                                                      (x.r - apply_lds(x.a, li, W)));
                       });
            };
            auto restr = [&](int l, int I) {  // r_{l+1} = P^T lb_l, la_{l+1} = omega D^{-1} r_{l+1}
                const Real rc = gmg_restrict<Real>(C, l, I, lb(l));
                stc(lr(l + 1) + I, rc);
                const Real c = reinterpret_cast<const Real *>(B.gA)[(size_t)op * 9 * gn +
                                                                     C.gmg_off[l + 1] + I];
                stc(la(l + 1) + I, c != (Real)0 ? omega(l + 1) * rc / c : (Real)0);
            };

            // pointwise CG update (u of the previous round is in UB0) and the
            // first smoothing step u1 = omega D^{-1} r
            own(0, [&](int id) {
                Real r = ldc(R + id);
                if (update) {
                    const Real w = ldc(Wv + id), u = ldc(UB0 + id);
                    const Real sn = first ? w : w + (Real)be * ldc(Sv + id);
                    const Real pn = first ? u : u + (Real)be * ldc(P + id);
                    stc(Sv + id, sn);
                    stc(P + id, pn);
                    stc(X + id, ldc(X + id) + al * (double)pn);
                    r = r - (Real)al * sn;
                    stc(R + id, r);
                }
                stc(U + id, omega(0) * (Real)dinv0[id] * r);
            });
            const int Lv = C.gmg_L, Lg = C.gmg_Lg;
            for (int l = 0; l < Lg; ++l) {
                if (!barrier(false)) return false;
                {
                    int a, b;
                    own_range(l, a, b);
                    resid_pass(l, a, b);
                }
                if (l + 1 < Lv) {
                    if (!barrier(false)) return false;
                    own(l + 1, [&](int I) { restr(l, I); });
                }
            }
            if (Lg < Lv) {
                if (!barrier(false)) return false;
                if (rank == 0) {
                    for (int l = Lg; l < Lv - 1; ++l) {
                        resid_pass(l, 0, gmg_level(C, l).Nn);
                        wg_sync();
                        whole(l + 1, [&](int I) { restr(l, I); });
                        wg_sync();
                    }
                    // coarsest level: an odd number of damped Jacobi sweeps, the
                    // result ends in lb
                    const int lc = Lv - 1;
                    for (int k = 0; k < C.gmg_tail_sweeps; ++k) {
                        const Real *src = (k & 1) ? lb(lc) : la(lc);
                        Real *dst = (k & 1) ? la(lc) : lb(lc);
                        smooth_pass(lc, src, nullptr, dst, 0, gmg_level(C, lc).Nn);
                        wg_sync();
                    }
                    for (int l = Lv - 2; l >= Lg; --l) {
                        smooth_pass(l, la(l), lb(l + 1), lb(l), 0, gmg_level(C, l).Nn);
                        wg_sync();
                    }
                }
            }
            // up: lb_l = v + omega D^{-1}(r - A v) with v = la_l + P lb_{l+1}
            for (int l = min(Lg, Lv) - 1; l >= 0; --l) {
                if (!barrier(false)) return false;
                int a, b;
                own_range(l, a, b);
                smooth_pass(l, la(l), l + 1 < Lv ? lb(l + 1) : nullptr, lb(l), a, b);
            }
            // w = A u and the dot products
            if (!barrier(false)) return false;
            {
                int a, b;
                own_range(0, a, b);
                staged(0, UB0, nullptr, a, b,
                       [&](int id) {
                           RowR x;
                           row(0, id, x.a);
                           x.r = ldc(R + id);
                           return x;
                       },
                       [&](int id, int li, int W, const RowR &x) {
                           const Real w = apply_lds(x.a, li, W);
                           stc(Wv + id, w);
                           const double u = LV[li], r = x.r;
                           loc[0] += r * u;
                           loc[1] += u * (double)w;
                           if (nloc > 2) loc[2] += r * r;
                       });
            }
            return true;
        };
        (void)gmg_round;

        // Resident rounds: the raw halo values (r, w, s of the neighbours'
        // boundary nodes) for the next round are loaded right after the
        // barrier, together with the partial sums, so both round trips overlap;
        // the halo z is formed once alpha and beta are known, with D^{-1} of the
        // halo nodes staged in LDS once per solve (FIRST).
        constexpr int kHP = 2;
        Real hpr[kHP], hpw[kHP], hps[kHP];
        bool hp_ok = false;
        auto halo_prefetch = [&](const StepInfo &st, bool need_s) {
            if constexpr (NPT > 0) {
                const int a = min(rank * TS, C.Nn);
                const int b = min(a + TS, C.Nn);
                const int ppar = (nbar - 1) & 1;  // parity of the round just published
                hp_ok = 2 * H <= kThreads * kHP;
                // per-call index math: hoisted out of the lane loop it would be
                // held in spilled registers, and each reload would wait for the
                // halo loads already in flight
                int tid = threadIdx.x;
                asm volatile("" : "+v"(tid));
#pragma unroll
                for (int u = 0; u < kHP; ++u) {
                    const int q = tid + u * kThreads;
                    hpr[u] = hpw[u] = hps[u] = (Real)0;
                    if (hp_ok && q < 2 * H) {
                        const bool left = q < H;
                        const int id = left ? a - H + q : b + (q - H);
                        if (id >= 0 && id < C.Nn) {
                            const int nb = left ? blockIdx.x - 1 : blockIdx.x + 1;
                            const int k = left ? q : q - H;
                            const Real *base =
                                XCH + (((size_t)nb * 2 + ppar) * 2 + (left ? 1 : 0)) * 3 * XS;
                            hpr[u] = ldc(base + k);
                            hpw[u] = ldc(base + XS + k);
                            if (need_s) hps[u] = ldc(base + 2 * XS + k);
                        }
                    }
                }
            } else {
                (void)st;
                (void)need_s;
            }
        };
        (void)halo_prefetch;

        const bool is_adj = is_adjoint_kind(L.kind);
        const bool tracer = (rank == 0 && threadIdx.x == 0);
        unsigned long long *trec = S.trace + (size_t)lane_id * S.trace_stride;
        unsigned long long iters_all = 0;
        const unsigned nbar0 = nbar;
        if (tracer) {
            trec[TR_KIND] = L.kind;
            trec[TR_SLICE] = L.slice;
            trec[TR_NWG] = g;
            trec[TR_TILE] = TS;
            trec[TR_START] = (unsigned long long)now_ticks();
            if constexpr (timers) t_mark = now_ticks();
        }

        Ctl c;
        c.step = 0;
        c.nsteps = lane_steps(C, L.kind);
        c.phase = c.nsteps > 0 ? PH_INIT : PH_DONE;
        c.iter = 0;
        c.it_local = 0;
        c.restarts = 0;
        c.verifying = false;
        c.zero_x = false;
        c.alpha = c.beta = c.gamma = 0.0;
        c.bnorm = c.relres = 0.0;
        c.r0n = 0.0;
        c.theta = 0.0;
        c.src_scale = 0.0;
        if (is_adj) {
            const double Th = *B.Theta;
            // the source of Theta (Eq. 4.6), or of Theta~ = Theta^p (Eq. 7.5)
            c.src_scale = C.plt ? (double)C.p / (double)C.Ne : pow_call(Th, 1.0 - C.p) / (double)C.Ne;
            if (!(Th > 0.0) || !isfinite(Th)) set_status(ctl, -5);
        }
        if (L.kind == F_PRI) {
            // a cold-started slice reads its theta after its flag wait (INIT)
            if (L.slice > 0 && !I.cold && !C.plt) c.theta = B.in_th[L.slice];
        } else if (L.kind == GK_PRI) {
            c.theta = B.in_th[L.slice];
        }

        StepInfo st{};
        while (c.phase != PH_DONE && ok) {
            if (c.phase == PH_INIT) {
                const bool first_entry = !c.verifying;
                st = step_info(C, B, I, L, c.step, TP);
                if (first_entry && st.wait) {
                    ok = waitf(st.wait_idx);
                    if (!ok) break;
                    if (L.kind == F_PRI && I.cold && L.slice > 0) c.theta = B.Gk_th[L.slice - 1];
                }
                if (first_entry && c.step == 0) {
                    if (L.kind == SWEEP_PRI) {
                        ok = waitf(flag_index(FL_F, 0));
                        if (!ok) break;
                        c.theta = B.F_th[0];
                    } else if (L.kind == SWEEP_ADJ) {
                        ok = waitf(flag_index(FL_F, C.Ntau));
                        if (!ok) break;
                    }
                }
                if (first_entry && (L.kind == SWEEP_PRI || L.kind == SWEEP_ADJ)) {
                    // G(u^k_n) must exist before it serves as the initial guess
                    if (I.cold) {
                        ok = waitf(flag_index(FL_COLD, st.n));
                    } else if (I.gk_lanes) {
                        ok = waitf(flag_index(FL_GK, st.n));
                    }
                    if (!ok) break;
                }
                const double ms = st.fine ? C.inv_dt : C.inv_dtau;
                const bool ext = first_entry && st.extrap;
                const bool x0copy = first_entry && (st.x0_src != nullptr || ext);
                const double *xs = (first_entry && st.x0_src != nullptr) ? st.x0_src : X;
                const double *ts = st.tp_src;
                // first solve of the lane's own kind (a fine adjoint lane's first
                // adjoint step follows its recomputed primal steps)
                const bool lane_start =
                    first_entry && (L.kind == F_ADJ ? (!st.recompute && st.s_adj == 0)
                                                    : c.step == 0);
                double loc[2] = {0.0, 0.0};  // ||b||^2, ||r0||^2
                // first step of a lane: zero sensitivity sums, publish copies
                // (tpv: the node's value of the C/delta operand, 0 on Dirichlet nodes)
                auto lane_start_work = [&](int id, int i, int j, double tpv) {
                    if (L.kind == F_ADJ) {
                        if (i < C.nx && j < C.ny)
                            B.acc[(size_t)(L.slice - 1) * C.Ne + j * C.nx + i] = 0.0;
                    } else if (L.kind == SWEEP_ADJ) {
                        if (i < C.nx && j < C.ny) B.accG[j * C.nx + i] = 0.0;
                        B.out_L[(size_t)C.Ntau * C.Nn + id] = 0.0;
                        B.out_L[(size_t)(C.Ntau - 1) * C.Nn + id] = tpv;
                    } else if (L.kind == SWEEP_PRI) {
                        B.out_T[(size_t)C.Nn + id] = tpv;
                    }
                };
                if (NPT == 0 && C.gmg) {
                    // multigrid lanes: the node ranges the multigrid rounds own, in
                    // chunks whose operand windows (C/delta operand and x0, one
                    // grid row of halo) are staged in LDS; rows of very wide
                    // grids do not fit the LDS tiles of the Jacobi path
                    const int ts0 = (C.Nn + g - 1) / g;
                    const int a0 = min(rank * ts0, C.Nn), b0 = min(a0 + ts0, C.Nn);
                    auto ldm = [&](const double *v, int q) -> double {
                        return (q >= 0 && q < C.Nn && !B.mask[q]) ? ldc(v + q) : 0.0;
                    };
                    const int CHI = C.gmg_chunk_init;
                    double *WT = lds;                       // C/delta operand window
                    double *WX = lds + CHI + 2 * H;         // x0 window
                    for (int c0 = a0; c0 < b0; c0 += CHI) {
                        const int c1 = min(c0 + CHI, b0);
                        const int lo = c0 - H, len = (c1 - c0) + 2 * H;
                        lds_sync();
                        for (int q0 = threadIdx.x; q0 < len; q0 += kThreads * kU) {
                            double vt[kU], vx[kU];
#pragma unroll
                            for (int u = 0; u < kU; ++u) {
                                const int q = q0 + u * kThreads;
                                vt[u] = q < len ? ldm(ts, lo + q) : 0.0;
                                vx[u] = q < len ? ldm(xs, lo + q) : 0.0;
                                if (q < len && first_entry && st.d1)
                                    vx[u] += ldm(st.d1, lo + q) - ldm(st.d0, lo + q);
                            }
#pragma unroll
                            for (int u = 0; u < kU; ++u) {
                                const int q = q0 + u * kThreads;
                                if (q < len) {
                                    WT[q] = vt[u];
                                    WX[q] = vx[u];
                                }
                            }
                        }
                        lds_sync();
                        for (int id = c0 + threadIdx.x; id < c1; id += kThreads) {
                            const int li2 = id - lo;
                            const int j = id / C.W, i = id - j * C.W;
                            double bval = 0.0, r0 = 0.0;
                            const double x0 = WX[li2];
                            if (!B.mask[id]) {
                                const Coef am = node_coef(C, B.kq, B.cm, i, j, ms, 0.0);
                                const Coef ak = node_coef(C, B.kq, B.cm, i, j, 0.0, 1.0);
                                double src;
                                if (!st.adjoint) {
                                    const int nex = (i > 0) + (i < C.nx), ney = (j > 0) + (j < C.ny);
                                    src = B.qt[st.j] * C.quarter_area * (double)(nex * ney);
                                } else {
                                    const double T = ld_state(srow(C, B, st.j, LSc), id, C.ckpt != 0);
                                    src = c.src_scale * ipow(T, C.p - 1);
                                }
                                bval = apply(am, WT, li2, C.W) + src;
                                r0 = bval - (apply(am, WX, li2, C.W) + apply(ak, WX, li2, C.W));
                            }
                            if (x0copy) stc(X + id, x0);
                            stc(Rb[0] + id, (Real)r0);
                            loc[0] += bval * bval;
                            loc[1] += r0 * r0;
                        }
                    }
                    // the lane's sums are zeroed by the very threads that
                    // accumulate them in the post-solve phase (same tiles, same
                    // node-to-thread map): plain stores are only ordered within
                    // a thread, and the L2 of another XCD may hold stale lines
                    if (lane_start)
                        for (int t = rank; t < ntiles; t += g) {
                            const int a = t * TS, b = min(a + TS, C.Nn);
                            for (int id = a + threadIdx.x; id < b; id += kThreads) {
                                const int j = id / C.W, i = id - j * C.W;
                                lane_start_work(id, i, j, ldm(ts, id));
                            }
                        }
                } else
                for (int t = rank; t < ntiles; t += g) {
                    const int a = t * TS;
                    const int b = min(a + TS, C.Nn);
                    const int lo = a - H;
                    const int len = (b - a) + 2 * H;
                    int ea, elen;
                    elem_window(C, a, b, ea, elen);
                    lds_sync();
                    stage_elems(B, ea, elen, LK, LC);
                    for (int q0 = threadIdx.x; q0 < len; q0 += kThreads * kU) {
                        double va[kU], vb[kU], vq[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            const bool in = q < len && id >= 0 && id < C.Nn;
                            va[u] = in ? ldc(xs + id) : 0.0;
                            if (in && first_entry && st.d1)
                                va[u] += ldc(st.d1 + id) - ldc(st.d0 + id);
                            vb[u] = in ? ldc(ts + id) : 0.0;
                            vq[u] = (in && ext) ? ldc(TQ + id) : 0.0;
                        }
                        if (ext) {
#pragma unroll
                            for (int u = 0; u < kU; ++u) va[u] = 2.0 * va[u] - vq[u];
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            if (q < len) {
                                const bool d = id >= 0 && id < C.Nn && B.mask[id];
                                LA[q] = d ? 0.0 : va[u];
                                LB[q] = d ? 0.0 : vb[u];
                            }
                        }
                    }
                    lds_sync();
                    for (int id = a + threadIdx.x; id < b; id += kThreads) {
                        const int li2 = id - lo;
                        const int j = id / C.W, i = id - j * C.W;
                        double bval = 0.0, r0 = 0.0;
                        const double x0 = LA[li2];
                        if (!B.mask[id]) {
                            const Coef am = node_coef_l(C, LK, LC, ea, i, j, ms, 0.0);
                            const Coef ak = node_coef_l(C, LK, LC, ea, i, j, 0.0, 1.0);
                            double src;
                            if (!st.adjoint) {
                                const int nex = (i > 0) + (i < C.nx), ney = (j > 0) + (j < C.ny);
                                src = B.qt[st.j] * C.quarter_area * (double)(nex * ney);
                            } else {
                                const double T = ld_state(srow(C, B, st.j, LSc), id, C.ckpt != 0);
                                src = c.src_scale * ipow(T, C.p - 1);
                            }
                            bval = apply(am, LB, li2, C.W) + src;
                            const double ax = apply(am, LA, li2, C.W) + apply(ak, LA, li2, C.W);
                            r0 = bval - ax;
                        }
                        if (x0copy) stc(X + id, x0);
                        stc(Rb[0] + id, (Real)r0);
                        loc[0] += bval * bval;
                        loc[1] += r0 * r0;
                        if (lane_start) lane_start_work(id, i, j, LB[li2]);
                    }
                }
                block_sum<2>(loc, red);
                const int par = nbar & 1;
                if (threadIdx.x == 0) {
                    stc(my_part(par) + 0, loc[0]);
                    stc(my_part(par) + 1, loc[1]);
                }
                ok = barrier(false);
                if (!ok) break;
                double tot[2];
                group_sum<2>(all_part(par), g, tot, red);
                mark_red();
                c.bnorm = sqrt(tot[0]);
                const double rn = sqrt(tot[1]);
                if (rank == 0 && threadIdx.x == 0 && c.step == 0 && first_entry) {
                    if (L.kind == SWEEP_PRI) B.out_th[1] = B.F_th[0];
                }
                if (first_entry) {
                    c.iter = 0;
                    c.restarts = 0;
                    c.zero_x = false;
                }
                c.it_local = 0;
                const int restart_cap = C.fp32 ? C.max_restarts : 3;
                if (C.coarse_iters > 0 && !st.fine) {
                    // truncated coarse solve: exactly coarse_iters CG iterations
                    // (fewer only if the residual vanishes)
                    c.relres = c.bnorm > 0.0 ? rn / c.bnorm : 0.0;
                    if (rn == 0.0) {
                        c.phase = PH_POST;
                    } else {
                        c.r0n = rn;
                        c.phase = PH_FIRST;
                    }
                } else if (c.bnorm == 0.0) {
                    c.zero_x = true;
                    c.relres = 0.0;
                    c.phase = PH_POST;
                } else if (rn <= C.rtol * c.bnorm) {
                    c.relres = rn / c.bnorm;
                    c.phase = PH_POST;
                } else if (!first_entry && (c.restarts >= restart_cap || c.iter >= C.max_iter)) {
                    // refinement / verification exhausted: keep x, report
                    c.relres = rn / c.bnorm;
                    c.phase = PH_POST;
                    if (rank == 0 && threadIdx.x == 0) set_status(ctl, -4);
                } else {
                    c.r0n = rn;
                    c.phase = PH_FIRST;
                }
                c.verifying = false;
            } else if (c.phase == PH_FIRST) {
                // w0 = A z0, z0 = D^{-1} r0; gamma0 = (r0, z0), delta0 = (z0, w0)
                const double ms = st.fine ? C.inv_dt : C.inv_dtau;
                const double *dinv = st.fine ? B.dinv_f : B.dinv_c;
                double loc[2] = {0.0, 0.0};
                if constexpr (NPT > 0) {
                // resident: one tile per workgroup; r0, w0, x, dinv stay in registers
                {
                    const int a = min(rank * TS, C.Nn);
                    const int b = min(a + TS, C.Nn);
                    const int lo = a - H;
                    const int len = (b - a) + 2 * H;
                    lds_sync();
                    for (int q0 = threadIdx.x; q0 < len; q0 += kThreads * kU) {
                        Real rv[kU], dv[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            const bool in = q < len && id >= 0 && id < C.Nn;
                            rv[u] = in ? ldc(Rb[0] + id) : (Real)0;
                            dv[u] = in ? (Real)dinv[id] : (Real)0;
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            if (q < len) {
                                LZ[q] = dv[u] * rv[u];
                                if (id >= a && id < b) LR[id - a] = rv[u];
                                // D^{-1} of the halo nodes, behind the tile's own
                                // (left halo first): fixed for the whole solve
                                else LR[TS + (q < H ? q : q - (b - a))] = dv[u];
                            }
                        }
                    }
                    lds_sync();
                    const int par = nbar & 1;
                    int tid = threadIdx.x;
                    asm volatile("" : "+v"(tid));  // per-round index math (not hoisted)
#pragma unroll
                    for (int k = 0; k < NPT; ++k) {
                        const int id = a + tid + k * kThreads;
                        rp[k] = rs[k] = 0.0;
                        if (id < b) {
                            const int li2 = id - lo;
                            Real w = 0;
                            if (!((dmask >> k) & 1u)) {
                                const int j = id / C.W, i = id - j * C.W;
                                const CoefT<Real> aa = node_coef_t<Real>(C, LK, LC, ea_res, i, j, ms, 1.0);
                                w = apply_t<Real>(aa, LZ, li2, C.W);
                            }
                            rr[k] = LR[id - a];
                            LD[id - a] = (Real)dinv[id];
                            rw[k] = w;
                            const Real z = LZ[li2];
                            loc[0] += (double)rr[k] * (double)z;
                            loc[1] += (double)z * (double)w;
                            publish(id, a, b, rr[k], rw[k], (Real)0, par);
                        } else {
                            rr[k] = rw[k] = 0.0;
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                } else if (C.gmg) {
                    ok = gmg_round(st, false, true, 0.0, 0.0, loc, 2);
                    if (!ok) break;
                } else {
                for (int t = rank; t < ntiles; t += g) {
                    const int a = t * TS;
                    const int b = min(a + TS, C.Nn);
                    const int lo = a - H;
                    const int len = (b - a) + 2 * H;
                    int ea, elen;
                    elem_window(C, a, b, ea, elen);
                    lds_sync();
                    stage_elems(B, ea, elen, LK, LC);
                    for (int q0 = threadIdx.x; q0 < len; q0 += kThreads * kU) {
                        Real rv[kU], dv[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            const bool in = q < len && id >= 0 && id < C.Nn;
                            rv[u] = in ? ldc(Rb[0] + id) : (Real)0;
                            dv[u] = in ? (Real)dinv[id] : (Real)0;
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            if (q < len) {
                                LZ[q] = dv[u] * rv[u];
                                if (id >= a && id < b) LR[id - a] = rv[u];
                            }
                        }
                    }
                    lds_sync();
                    for (int id = a + threadIdx.x; id < b; id += kThreads) {
                        const int li2 = id - lo;
                        Real w = 0;
                        const Real z = LZ[li2];
                        if (!B.mask[id]) {
                            const int j = id / C.W, i = id - j * C.W;
                            const CoefT<Real> aa = node_coef_t<Real>(C, LK, LC, ea, i, j, ms, 1.0);
                            w = apply_t<Real>(aa, LZ, li2, C.W);
                        }
                        stc(Wb[0] + id, w);
                        loc[0] += (double)LR[id - a] * (double)z;
                        loc[1] += (double)z * (double)w;
                    }
                }
                }
                block_sum<2>(loc, red);
                const int par = nbar & 1;
                if (threadIdx.x == 0) {
                    stc(my_part(par) + 0, loc[0]);
                    stc(my_part(par) + 1, loc[1]);
                }
                ok = barrier(false);
                if (!ok) break;
                if constexpr (NPT > 0) halo_prefetch(st, false);
                double tot[2];
                group_sum<2>(all_part(par), g, tot, red);
                mark_red();
                c.gamma = tot[0];
                c.alpha = tot[0] / tot[1];
                c.beta = 0.0;
                c.phase = PH_ITER;
            } else if (c.phase == PH_ITER) {
                const double ms = st.fine ? C.inv_dt : C.inv_dtau;
                const double *dinv = st.fine ? B.dinv_f : B.dinv_c;
                const int i0 = c.it_local;  // iteration since the last (re)start
                const bool first = (i0 == 0);
                const double al = c.alpha, be = c.beta;
                double loc[3] = {0.0, 0.0, 0.0};
                if constexpr (NPT > 0) {
                // resident: halo of z_{i+1} rebuilt from the neighbours' published
                // r_i, w_i, s_{i-1}; own values updated in registers
                {
                    const int a = min(rank * TS, C.Nn);
                    const int b = min(a + TS, C.Nn);
                    const int lo = a - H;
                    const int ppar = (nbar - 1) & 1;  // parity of the previous round
                    int tid = threadIdx.x;
                    asm volatile("" : "+v"(tid));  // per-round index math (not hoisted)
                    // x of the tile is read only by its owning thread during
                    // the rounds (plain loads of its own device-coherent stores)
                    double xo[NR];
#pragma unroll
                    for (int k = 0; k < NPT; ++k) {
                        const int id = a + tid + k * kThreads;
                        xo[k] = id < b ? X[id] : 0.0;
                    }
                    lds_sync();
                    if (hp_ok) {
#pragma unroll
                        for (int u = 0; u < kHP; ++u) {
                            const int q = tid + u * kThreads;
                            if (q < 2 * H) {
                                const Real sv = first ? hpw[u] : hpw[u] + (Real)be * hps[u];
                                const Real z = LD[TS + q] * (hpr[u] - (Real)al * sv);
                                LZ[q < H ? q : (b - lo) + (q - H)] = z;
                            }
                        }
                    } else
                    for (int q = threadIdx.x; q < 2 * H; q += kThreads) {
                        const bool left = q < H;
                        const int id = left ? a - H + q : b + (q - H);
                        Real z = 0;
                        if (id >= 0 && id < C.Nn) {
                            const int nb = left ? blockIdx.x - 1 : blockIdx.x + 1;
                            const int k = left ? q : q - H;
                            const Real *base =
                                XCH + (((size_t)nb * 2 + ppar) * 2 + (left ? 1 : 0)) * 3 * XS;
                            const Real rh = ldc(base + k);
                            const Real wh = ldc(base + XS + k);
                            const Real sh = first ? (Real)0 : ldc(base + 2 * XS + k);
                            const Real sv = first ? wh : wh + (Real)be * sh;
                            z = LD[TS + q] * (rh - (Real)al * sv);
                        }
                        LZ[left ? q : (b - lo) + (q - H)] = z;
                    }
                    // all x loads done before the first x store: with stores in
                    // flight the compiler can only wait for a load by draining
                    // the stores too (loads and stores share one counter), i.e.
                    // one store round trip per node
                    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
#pragma unroll
                    for (int k = 0; k < NPT; ++k) {
                        const int id = a + tid + k * kThreads;
                        if (id < b) {
                            const Real dk = LD[id - a];
                            const Real zi = dk * rr[k];
                            const Real pn = first ? zi : zi + (Real)be * rp[k];
                            const Real sn = first ? rw[k] : rw[k] + (Real)be * rs[k];
                            stc(X + id, xo[k] + al * (double)pn);
                            rr[k] -= (Real)al * sn;
                            rp[k] = pn;
                            rs[k] = sn;
                            LZ[id - lo] = dk * rr[k];
                        }
                    }
                    lds_sync();
                    const int par = nbar & 1;
#pragma unroll
                    for (int k = 0; k < NPT; ++k) {
                        const int id = a + tid + k * kThreads;
                        if (id < b) {
                            const int li2 = id - lo;
                            Real w = 0;
                            if (!((dmask >> k) & 1u)) {
                                const int j = id / C.W, i = id - j * C.W;
                                const CoefT<Real> aa = node_coef_t<Real>(C, LK, LC, ea_res, i, j, ms, 1.0);
                                w = apply_t<Real>(aa, LZ, li2, C.W);
                            }
                            rw[k] = w;
                            const Real z = LZ[li2];
                            loc[0] += (double)rr[k] * (double)z;
                            loc[1] += (double)z * (double)w;
                            loc[2] += (double)rr[k] * (double)rr[k];
                            publish(id, a, b, rr[k], rw[k], rs[k], par);
                        }
                        // keep the unrolled node iterations from being interleaved
                        // (register pressure)
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                } else if (C.gmg) {
                    // its own array: passing loc's address keeps loc in scratch
                    // memory in every round form, stored on every node
                    double gl[3] = {0.0, 0.0, 0.0};
                    ok = gmg_round(st, true, first, al, be, gl, 3);
                    if (!ok) break;
                    loc[0] = gl[0];
                    loc[1] = gl[1];
                    loc[2] = gl[2];
                } else {
                const int cur = i0 & 1, nxt = cur ^ 1;
                Real *Rc = Rb[cur], *Rn = Rb[nxt], *Wc = Wb[cur], *Wn = Wb[nxt];
                Real *Sc = Sb[cur], *Sn = Sb[nxt];
                for (int t = rank; t < ntiles; t += g) {
                    const int a = t * TS;
                    const int b = min(a + TS, C.Nn);
                    const int lo = a - H;
                    const int len = (b - a) + 2 * H;
                    int ea, elen;
                    elem_window(C, a, b, ea, elen);
                    lds_sync();
                    stage_elems(B, ea, elen, LK, LC);
                    constexpr int kUW = 6;  // window nodes per thread and iteration
                    for (int q0 = threadIdx.x; q0 < len; q0 += kThreads * kUW) {
                        Real rv[kUW], wv[kUW], sv[kUW], dv[kUW], pv[kUW];
                        double xv[kUW];
                        // D^{-1} is read unmasked at a clamped (always valid)
                        // index and zeroed afterwards: a masked load needs a zero
                        // default in its destination, so its address sits in
                        // another register, and reusing that register for the
                        // next node's address waited for every load in flight
#pragma unroll
                        for (int u = 0; u < kUW; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            const bool in = q < len && id >= 0 && id < C.Nn;
                            const double d = dinv[min(max(id, 0), C.Nn - 1)];
                            dv[u] = in ? (Real)d : (Real)0;
                        }
#pragma unroll
                        for (int u = 0; u < kUW; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            const bool in = q < len && id >= 0 && id < C.Nn;
                            const bool own = in && id >= a && id < b;
                            rv[u] = in ? ldc(Rc + id) : 0.0;
                            wv[u] = in ? ldc(Wc + id) : 0.0;
                            sv[u] = (in && !first) ? ldc(Sc + id) : 0.0;
                            pv[u] = (own && !first) ? ldc(P + id) : 0.0;
                            xv[u] = own ? ldc(X + id) : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < kUW; ++u) {
                            const int q = q0 + u * kThreads;
                            const int id = lo + q;
                            if (q < len) {
                                const Real s_new = first ? wv[u] : wv[u] + (Real)be * sv[u];
                                const Real r_new = rv[u] - (Real)al * s_new;
                                LZ[q] = dv[u] * r_new;
                                if (id >= a && id < b) {
                                    const Real zi = dv[u] * rv[u];
                                    const Real pn = first ? zi : zi + (Real)be * pv[u];
                                    stc(P + id, pn);
                                    stc(Sn + id, s_new);
                                    stc(X + id, xv[u] + al * (double)pn);
                                    stc(Rn + id, r_new);
                                    // Dirichlet nodes (D^{-1} = 0) carry the marker, so
                                    // the stencil loop below needs no flag load: a load
                                    // there would wait for the node stores in flight
                                    LR[id - a] = dv[u] == (Real)0 ? dir_tag(r_new) : r_new;
                                }
                            }
                        }
                    }
                    lds_sync();
                    for (int id = a + threadIdx.x; id < b; id += kThreads) {
                        const int li2 = id - lo;
                        Real w = 0;
                        const Real rraw = LR[id - a];
                        const bool dir = is_dir_tag(rraw);
                        if (!dir) {
                            const int j = id / C.W, i = id - j * C.W;
                            const CoefT<Real> aa = node_coef_t<Real>(C, LK, LC, ea, i, j, ms, 1.0);
                            w = apply_t<Real>(aa, LZ, li2, C.W);
                        }
                        stc(Wn + id, w);
                        const Real z = LZ[li2];
                        const double rn = dir ? 0.0 : (double)rraw;
                        loc[0] += rn * z;
                        loc[1] += (double)z * (double)w;
                        loc[2] += rn * rn;
                    }
                }
                }
                block_sum<3>(loc, red);
                const int par = nbar & 1;
                // one partial per thread: one thread storing all three reused a
                // register that an earlier store still read, and waited for it
                int tid3 = threadIdx.x;
                asm volatile("" : "+v"(tid3));  // per-round address (see block_sum)
                if (tid3 < 3) {
                    const double v = tid3 == 0 ? loc[0] : (tid3 == 1 ? loc[1] : loc[2]);
                    stc(my_part(par) + tid3, v);
                }
                ok = barrier(false);
                if (!ok) break;
                if constexpr (NPT > 0) halo_prefetch(st, true);
                double tot[3];
                group_sum<3>(all_part(par), g, tot, red);
                mark_red();
                c.it_local = i0 + 1;
                c.iter += 1;
                const double rn = sqrt(tot[2]);
                // FP32 inner solves stop at a relative reduction inner_rtol of the
                // residual they started from; the FP64 residual of the refinement
                // step (INIT) decides convergence
                const double target =
                    C.fp32 ? fmax(C.rtol * c.bnorm, C.inner_rtol * c.r0n) : C.rtol * c.bnorm;
                const bool trunc = C.coarse_iters > 0 && !st.fine;
                if (trunc ? (c.iter >= C.coarse_iters || rn == 0.0)
                          : (rn <= target || c.iter >= C.max_iter)) {
                    c.relres = c.bnorm > 0.0 ? rn / c.bnorm : 0.0;
                    const bool check =
                        !trunc && (C.fp32 ? (c.iter < C.max_iter)
                                          : (C.verify && rn <= C.rtol * c.bnorm && c.restarts < 3));
                    // (the rounds store x device-coherently, and the round's
                    // barrier has drained those stores: the residual and the
                    // adjoint post-solve phase read the neighbours' x at once)
                    if (check) {
                        // recompute r = b - A x in FP64, restart CG if needed
                        c.verifying = true;
                        c.restarts += 1;
                        c.phase = PH_INIT;
                    } else {
                        c.phase = PH_POST;
                        if (!trunc && rn > C.rtol * c.bnorm && rank == 0 && threadIdx.x == 0)
                            set_status(ctl, -4);
                    }
                } else {
                    const double gnew = tot[0];
                    const double bnew = gnew / c.gamma;
                    const double anew = gnew / (tot[1] - bnew * gnew / al);
                    c.beta = bnew;
                    c.alpha = anew;
                    c.gamma = gnew;
                }
            } else {  // PH_POST: lane-specific use of the converged solution x
                const bool last = (c.step == c.nsteps - 1);
                if (L.kind == SWEEP_PRI || L.kind == SWEEP_ADJ) {
                    ok = waitf(flag_index(FL_F, st.n));
                    if (!ok) break;
                }
                double loc[1] = {0.0};
                const bool zx = c.zero_x;
                for (int t = rank; t < ntiles; t += g) {
                    const int a = t * TS;
                    const int b = min(a + TS, C.Nn);
                    for (int id = a + threadIdx.x; id < b; id += kThreads) {
                        // resident: the owning thread of the rounds reads its own x
                        const double x = zx ? 0.0 : (NPT > 0 ? X[id] : ldc(X + id));
                        switch (L.kind) {
                            case F_PRI: {
                                if (double *Sj = srow(C, B, st.j, nullptr)) Sj[id] = x;
                                if (C.plt && last) B.out_T[(size_t)(L.slice + 1) * C.Nn + id] = x;
                                if (C.extrap) stc(TQ + id, ldc(TP + id));
                                stc(TP + id, x);
                                loc[0] += ipow(x, C.p);
                                break;
                            }
                            case GK_PRI:
                            case COLD_PRI: {
                                B.Gk[(size_t)st.n * C.Nn + id] = x;
                                stc(TP + id, x);
                                loc[0] += ipow(x, C.p);
                                break;
                            }
                            case SWEEP_PRI: {
                                const int n = st.n;
                                double *Sj = srow(C, B, C.M * (n + 1), nullptr);
                                const double u = x + Sj[id] - B.Gk[(size_t)n * C.Nn + id];
                                Sj[id] = u;
                                B.out_T[(size_t)(n + 1) * C.Nn + id] = u;
                                B.Gn[(size_t)n * C.Nn + id] = x;
                                stc(TP + id, u);
                                loc[0] += ipow(x, C.p);
                                break;
                            }
                            case F_ADJ: {
                                if (st.recompute) {
                                    stc(srow(C, B, st.j, LSc) + id, x);
                                    stc(TP + id, x);
                                    break;
                                }
                                if (C.extrap) stc(TQ + id, ldc(TP + id));
                                stc(TP + id, x);
                                if (last) B.FL[(size_t)L.slice * C.Nn + id] = x;
                                if (C.plt && last) B.out_L[(size_t)(L.slice - 1) * C.Nn + id] = x;
                                const int j2 = id / C.W, i2 = id - j2 * C.W;
                                if (i2 < C.nx && j2 < C.ny) {
                                    const int e = j2 * C.nx + i2;
                                    const double l1 = zx ? 0.0 : ldc(X + id + 1);
                                    const double l2 = zx ? 0.0 : ldc(X + id + C.W + 1);
                                    const double l3 = zx ? 0.0 : ldc(X + id + C.W);
                                    const double *Tr = srow(C, B, st.j, LSc);
                                    const double *Tp =
                                        st.jprev > 0 ? srow(C, B, st.jprev, LSc) : nullptr;
                                    B.acc[(size_t)(L.slice - 1) * C.Ne + e] +=
                                        sens_term(C, B, I, id, e, x, l1, l2, l3, Tr, Tp, C.inv_dt,
                                                  C.ckpt != 0);
                                }
                                break;
                            }
                            case GK_ADJ:
                            case COLD_ADJ: {
                                B.Gk[(size_t)st.n * C.Nn + id] = x;
                                stc(TP + id, x);
                                break;
                            }
                            default: {  // SWEEP_ADJ
                                const int n = st.n;
                                const double *FLn = B.FL + (size_t)n * C.Nn;
                                const double *Gkn = B.Gk + (size_t)n * C.Nn;
                                const double lam = x + FLn[id] - Gkn[id];
                                B.out_L[(size_t)(n - 1) * C.Nn + id] = lam;
                                B.Gn[(size_t)n * C.Nn + id] = x;
                                stc(TP + id, lam);
                                const int j2 = id / C.W, i2 = id - j2 * C.W;
                                if (i2 < C.nx && j2 < C.ny) {
                                    const int e = j2 * C.nx + i2;
                                    auto dl = [&](int k) { return (zx ? 0.0 : ldc(X + k)) - Gkn[k]; };
                                    const double *Tr = srow(C, B, st.j, nullptr);
                                    const double *Tp =
                                        st.jprev > 0 ? srow(C, B, st.jprev, nullptr) : nullptr;
                                    B.accG[e] += sens_term(C, B, I, id, e, dl(id), dl(id + 1),
                                                           dl(id + C.W + 1), dl(id + C.W), Tr, Tp,
                                                           C.inv_dtau, false);
                                }
                                break;
                            }
                        }
                    }
                }
                block_sum<1>(loc, red);
                const int par = nbar & 1;
                if (threadIdx.x == 0) stc(my_part(par), loc[0]);
                // release: plain stores of this step (S, Gk, FL, outputs) become visible
                ok = barrier(true);
                if (!ok) break;
                double tot[1];
                group_sum<1>(all_part(par), g, tot, red);
                mark_red();
                const bool leader = (rank == 0 && threadIdx.x == 0);
                // theta updates (Alg. 1, step 2) and lane outputs
                if (!is_adj) {
                    const double inv = st.fine ? C.inv_NtNe : C.inv_NtauNe;
                    // with G = 0 a fine lane keeps its slice's part of Theta~ instead
                    const double thG = C.plt ? c.theta + tot[0] * inv
                                             : pow_call(ipow(c.theta, C.p) + tot[0] * inv, C.inv_p);
                    if (L.kind == SWEEP_PRI) {
                        const int n = st.n;
                        const double thu = thG + B.F_th[n] - B.Gk_th[n];
                        if (leader) {
                            B.out_th[n + 1] = thu;
                            B.Gn_th[n] = thG;
                        }
                        c.theta = thu;
                    } else {
                        c.theta = thG;
                        if (leader && (L.kind == GK_PRI || L.kind == COLD_PRI)) B.Gk_th[st.n] = thG;
                        if (leader && L.kind == F_PRI && last) B.F_th[L.slice] = thG;
                    }
                }
                if (leader) {
                    const int it = c.iter;
                    if (st.fine) {
                        atomicAdd(&ctl->iters_fine, (unsigned long long)it);
                        atomicAdd(&ctl->solves_fine, 1ull);
                    } else {
                        atomicAdd(&ctl->iters_coarse, (unsigned long long)it);
                        atomicAdd(&ctl->solves_coarse, 1ull);
                    }
                    atomicMax(&ctl->max_iters, it);
                    atomicMax(&ctl->max_relres_bits,
                              (unsigned long long)__double_as_longlong(c.relres));
                    if (L.kind == GK_PRI || L.kind == GK_ADJ)
                        set_flag(B.flags, flag_index(FL_GK, st.n), I.epoch);
                    if (L.kind == COLD_PRI || L.kind == COLD_ADJ)
                        set_flag(B.flags, flag_index(FL_COLD, st.n), I.epoch);
                    if ((L.kind == F_PRI || L.kind == F_ADJ) && last)
                        set_flag(B.flags, flag_index(FL_F, L.slice), I.epoch);
                }
                iters_all += c.iter;
                if (tracer && c.step < S.trace_stride - TR_HDR)
                    trec[TR_HDR + c.step] = (unsigned long long)now_ticks();
                c.step += 1;
                c.phase = (c.step < c.nsteps) ? PH_INIT : PH_DONE;
                c.iter = 0;
                c.verifying = false;
            }
        }
        if (tracer) {
            trec[TR_ROUNDS] = nbar - nbar0;
            trec[TR_ITERS] = iters_all;
            trec[TR_T_WORK] = t_work;
            trec[TR_T_BAR] = t_bar;
            trec[TR_T_RED] = t_red;
            trec[TR_T_FLAG] = t_flag;
            t_work = t_bar = t_red = t_flag = 0;
        }
    }
    if (!ok && threadIdx.x == 0) {
        atomicExch(&ctl->abort, 1);
        set_status(ctl, -3);
    }
}

// After the primal engine (blockIdx.y = design): u_0 = 0, Theta, and the
// N_tau = 1 case. With G = 0, Theta~ is the sum of the slices' parts in slice
// order (Eq. 7.4) and Theta = Theta~^{1/p} (Eq. 7.6).
__global__ void k_finalize_fwd(const EngineDesc *__restrict__ D) {
    const EngineDesc &E = D[blockIdx.y];
    const Consts &C = E.C;
    const Bufs &B = E.B;
    const size_t Nn = C.Nn;
    for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < Nn;
         id += (size_t)gridDim.x * blockDim.x) {
        B.out_T[id] = 0.0;
        if (C.Ntau == 1 && !C.plt) B.out_T[Nn + id] = srow(C, B, C.Nt, nullptr)[id];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        B.out_th[0] = 0.0;
        if (C.plt) {
            double run = 0.0;
            for (int n = 0; n < C.Ntau; ++n) {
                run += B.F_th[n];
                B.out_th[n + 1] = pow(run, C.inv_p);
            }
        } else if (C.Ntau == 1) {
            B.out_th[1] = B.F_th[0];
        }
        const double Th = B.out_th[C.Ntau];
        *B.Theta_out = Th;
        if (!(Th > 0.0) || !isfinite(Th)) atomicCAS(&B.ctl->status, 0, -5);
        B.ctl->fwd_done = kFwdDone;
    }
}

// After the adjoint engine (blockIdx.y = design): lambda for N_tau = 1, the
// last row and coarse sums with G = 0, and the back-transform factor of the
// sensitivities (Eq. 7.7).
__global__ void k_finalize_adj(const EngineDesc *__restrict__ D) {
    const EngineDesc &E = D[blockIdx.y];
    const Consts &C = E.C;
    const Bufs &B = E.B;
    const size_t Nn = C.Nn;
    if (B.ctl->status == kStatusOrder) {
        // no forward pass preceded this adjoint: nothing ran, lambda is undefined
        const size_t n = (size_t)(C.Ntau + 1) * Nn;
        for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < n;
             id += (size_t)gridDim.x * blockDim.x)
            B.out_L[id] = __longlong_as_double(0x7FF8000000000000LL);
        return;
    }
    if (C.Ntau == 1 || C.plt) {
        for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < Nn;
             id += (size_t)gridDim.x * blockDim.x) {
            if (!C.plt) B.out_L[id] = B.FL[Nn + id];
            B.out_L[(size_t)C.Ntau * Nn + id] = 0.0;
        }
        for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)C.Ne;
             e += (size_t)gridDim.x * blockDim.x)
            B.accG[e] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        B.ctl->grad_scale = C.plt ? pow(*B.Theta, 1.0 - C.p) / (double)C.p : 1.0;
        B.ctl->adj_done = kAdjDone;
    }
}

// grad_e = -(1/N_t) sum_n acc[n][e] - (1/N_tau) accG[e]  (Eq. 4.16 summed,
// Sec. 4.4 step 4), times Theta^{1-p}/p with G = 0 (Eq. 7.7); blockIdx.y = design.
__global__ void k_sensitivities(const EngineDesc *__restrict__ D) {
    const EngineDesc &E = D[blockIdx.y];
    const Consts &C = E.C;
    const Bufs &B = E.B;
    if (B.ctl->adj_done != kAdjDone) {
        // no complete adjoint pass: the sensitivity sums are not this cycle's
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(&B.ctl->status, 0, kStatusOrder);
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < C.Ne; e += gridDim.x * blockDim.x)
            B.grad[e] = __longlong_as_double(0x7FF8000000000000LL);
        return;
    }
    const double scale = B.ctl->grad_scale;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < C.Ne; e += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int n = 0; n < C.Ntau; ++n) s += B.acc[(size_t)n * C.Ne + e];
        B.grad[e] = (-s / (double)C.Nt - B.accG[e] / (double)C.Ntau) * scale;
    }
}

// Keeps a design's corrected u^{k+1} and lambda^{k+1} as its next guesses
// (warm restart of Alg. 3); blockIdx.y = design.
// primal_only: a forward-only cycle keeps the lambda guess of the last full
// cycle, or (zero_lambda, a cold forward-only cycle) sets it to 0.
__global__ void k_save_guess(const EngineDesc *__restrict__ D, int primal_only, int zero_lambda) {
    const EngineDesc &E = D[blockIdx.y];
    const Consts &C = E.C;
    const Bufs &B = E.B;
    const size_t n = (size_t)(C.Ntau + 1) * C.Nn;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x) {
        B.save_T[t] = B.out_T[t];
        if (!primal_only) B.save_L[t] = B.out_L[t];
        else if (zero_lambda) B.save_L[t] = 0.0;
    }
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k <= C.Ntau; k += blockDim.x) B.save_th[k] = B.out_th[k];
}

// Copies n descriptors given by value into device memory (n <= kDescPerCopy).
constexpr int kDescPerCopy = 3;
struct DescChunk {
    EngineDesc d[kDescPerCopy];
};
static_assert(sizeof(DescChunk) + 16 <= 4096, "kernel argument limit");
__global__ void k_put_desc(DescChunk chunk, int n, EngineDesc *dst) {
    const int words = (int)(sizeof(EngineDesc) / sizeof(unsigned));
    for (int k = 0; k < n; ++k) {
        const unsigned *src = reinterpret_cast<const unsigned *>(&chunk.d[k]);
        unsigned *out = reinterpret_cast<unsigned *>(dst + k);
        for (int w = threadIdx.x; w < words; w += blockDim.x) out[w] = src[w];
    }
}

}  // namespace pt
