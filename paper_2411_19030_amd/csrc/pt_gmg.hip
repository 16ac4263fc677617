// Geometric multigrid preconditioner for the backward-Euler operator
// A = C/delta + K of the Q1 grid (the linear systems of Eq. 2.7b), used inside
// the lane engine's conjugate gradient.
//
// Hierarchy: level l has (nx >> l) x (ny >> l) elements; its nodes are the
// even-indexed nodes of level l-1 (vertex-centred coarsening, kept while both
// sides stay even and at least 2 coarse elements wide). Prolongation P is
// bilinear interpolation, restriction is P^T, and the coarse operators are the
// Galerkin products A_{l+1} = P^T A_l P, stored as 9-point stencils. Level 0
// is applied matrix-free from the element coefficients; Dirichlet nodes carry
// zero rows and zero prolongation weights, so every coarse operator stays SPD
// (the capacity term alone makes it definite).
//
// One application u = B r is a V(1,1) cycle with damped Jacobi smoothing,
// omega_l = gmg_omega / g_l with g_l the Gershgorin bound of D_l^{-1} A_l:
//   u1 = omega D^{-1} r;  r_{l+1} = P^T (r - A u1);  e = B_{l+1} r_{l+1};
//   u2 = u1 + P e;        u = u2 + omega D^{-1} (r - A u2)
// and on the coarsest level a fixed number of damped Jacobi sweeps from zero.
// Every step is a fixed linear map and the smoothing is symmetric, so B is
// symmetric positive definite and CG stays valid.
//
// Included by pt_engine.hip inside namespace pt, after the stencil helpers.

namespace {

struct Lvl {
    int nx, ny, W, Nn;
    long long off;
};

__device__ __forceinline__ Lvl gmg_level(const Consts &C, int l) {
    Lvl v;
    v.nx = C.nx >> l;
    v.ny = C.ny >> l;
    v.W = v.nx + 1;
    v.Nn = v.W * (v.ny + 1);
    v.off = l > 0 ? C.gmg_off[l] : 0;
    return v;
}

// neighbour offsets in the order c, e, w, n, s, ne, nw, se, sw
__device__ __forceinline__ int nb_off(int k, int W) {
    switch (k) {
        case 0: return 0;
        case 1: return 1;
        case 2: return -1;
        case 3: return W;
        case 4: return -W;
        case 5: return W + 1;
        case 6: return W - 1;
        case 7: return -W + 1;
        default: return -W - 1;
    }
}
__device__ __forceinline__ int nb_dx(int k) {
    return (k == 1 || k == 5 || k == 7) ? 1 : ((k == 2 || k == 6 || k == 8) ? -1 : 0);
}
__device__ __forceinline__ int nb_dy(int k) {
    return (k == 3 || k == 5 || k == 6) ? 1 : ((k == 4 || k == 7 || k == 8) ? -1 : 0);
}

// FP64 stencil row of level l at node id of operator op (0: dt, 1: dtau).
// Level 0 rows come from the element coefficients; Dirichlet nodes return a
// zero row.
__device__ __forceinline__ void gmg_row64(const Consts &C, const Bufs &B, int op, int l, int id,
                                          double (&a)[9]) {
    if (l == 0) {
        if (B.mask[id]) {
#pragma unroll
            for (int k = 0; k < 9; ++k) a[k] = 0.0;
            return;
        }
        const int j = id / C.W, i = id - j * C.W;
        const Coef c = node_coef(C, B.kq, B.cm, i, j, op ? C.inv_dtau : C.inv_dt, 1.0);
        a[0] = c.c;
        a[1] = c.e;
        a[2] = c.w;
        a[3] = c.n;
        a[4] = c.s;
        a[5] = c.ne;
        a[6] = c.nw;
        a[7] = c.se;
        a[8] = c.sw;
        return;
    }
    const size_t base = (size_t)op * 9 * C.gmg_nodes + C.gmg_off[l] + id;
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = B.gA64[base + (size_t)k * C.gmg_nodes];
}

// (A_l v)(id) in the CG precision; v is read with device-coherent loads (other
// workgroups of the group wrote it before the last barrier). diag returns the
// stencil centre (0 on Dirichlet nodes of level 0).
template <typename Real>
__device__ __forceinline__ Real gmg_apply(const Consts &C, const Bufs &B, int op, int l, int id,
                                          const Real *v, Real &diag) {
    const Lvl L = gmg_level(C, l);
    Real a[9];
    if (l == 0) {
        if (B.mask[id]) {
            diag = 0;
            return 0;
        }
        double a64[9];
        gmg_row64(C, B, op, 0, id, a64);
#pragma unroll
        for (int k = 0; k < 9; ++k) a[k] = (Real)a64[k];
    } else {
        const Real *A = reinterpret_cast<const Real *>(B.gA) + (size_t)op * 9 * C.gmg_nodes +
                        L.off + id;
#pragma unroll
        for (int k = 0; k < 9; ++k) a[k] = A[(size_t)k * C.gmg_nodes];
    }
    diag = a[0];
    Real s = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int q = id + nb_off(k, L.W);
        if (q >= 0 && q < L.Nn) s += a[k] * ldc(v + q);
    }
    return s;
}

// Restriction P^T of level-l values to coarse node I of level l+1.
template <typename Real>
__device__ __forceinline__ Real gmg_restrict(const Consts &C, int l, int I, const Real *v) {
    const Lvl F = gmg_level(C, l);
    const Lvl G = gmg_level(C, l + 1);
    const int Iy = I / G.W, Ix = I - Iy * G.W;
    Real s = 0;
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
        const int fy = 2 * Iy + b;
        if (fy < 0 || fy > F.ny) continue;
        const Real wy = b == 0 ? (Real)1 : (Real)0.5;
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
            const int fx = 2 * Ix + a;
            if (fx < 0 || fx > F.nx) continue;
            const Real wx = a == 0 ? (Real)1 : (Real)0.5;
            s += wx * wy * ldc(v + fy * F.W + fx);
        }
    }
    return s;
}

// Bilinear prolongation of level-(l+1) values to fine node id of level l.
template <typename Real>
__device__ __forceinline__ Real gmg_prolong(const Consts &C, int l, int id, const Real *e) {
    const Lvl F = gmg_level(C, l);
    const Lvl G = gmg_level(C, l + 1);
    const int fy = id / F.W, fx = id - fy * F.W;
    const int x0 = fx >> 1, y0 = fy >> 1;
    const bool ox = fx & 1, oy = fy & 1;
    if (!ox && !oy) return ldc(e + y0 * G.W + x0);
    if (ox && !oy) return (Real)0.5 * (ldc(e + y0 * G.W + x0) + ldc(e + y0 * G.W + x0 + 1));
    if (!ox && oy) return (Real)0.5 * (ldc(e + y0 * G.W + x0) + ldc(e + (y0 + 1) * G.W + x0));
    return (Real)0.25 * (ldc(e + y0 * G.W + x0) + ldc(e + y0 * G.W + x0 + 1) +
                         ldc(e + (y0 + 1) * G.W + x0) + ldc(e + (y0 + 1) * G.W + x0 + 1));
}

}  // namespace

// ---------------------------------------------------------------------------
// Setup (per design, blockIdx.y = design; designs without multigrid return)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void atomic_max_pos(double *p, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

// Level 0: the assembled stencil rows in the CG precision (zero rows on
// Dirichlet nodes) and the Gershgorin bounds of both operators.
template <typename Real>
__device__ void gmg_level0_node(const Consts &C, const Bufs &B, int id, double (&g)[2]) {
    for (int op = 0; op < 2; ++op) {
        double a[9];
        gmg_row64(C, B, op, 0, id, a);
        Real *A = reinterpret_cast<Real *>(B.gA0) + (size_t)op * 9 * C.Nn + id;
        double s = 0.0;
        for (int k = 0; k < 9; ++k) {
            A[(size_t)k * C.Nn] = (Real)a[k];
            s += fabs(a[k]);
        }
        if (!B.mask[id]) g[op] = fmax(g[op], s / a[0]);
    }
}

__global__ void k_gmg_level0(const EngineDesc *__restrict__ D) {
    const EngineDesc &E = D[blockIdx.y];
    const Consts &C = E.C;
    const Bufs &B = E.B;
    if (!C.gmg) return;
    double g[2] = {0.0, 0.0};
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < C.Nn; id += gridDim.x * blockDim.x) {
        if (C.fp32) gmg_level0_node<float>(C, B, id, g);
        else gmg_level0_node<double>(C, B, id, g);
    }
    for (int op = 0; op < 2; ++op)
        if (g[op] > 0.0) atomic_max_pos(&B.gmg_g[op * kMaxLevels + 0], g[op]);
}

// Galerkin product A_{l+1} = P^T A_l P for both operators, one coarse node per
// thread: the 9 fine nodes under coarse node I (weights of P), their stencil
// rows, and for every fine neighbour j the coarse nodes whose basis covers j.
template <typename Real>
__device__ void gmg_rap_node(const Consts &C, const Bufs &B, int l, int I) {
    const Lvl F = gmg_level(C, l);
    const Lvl G = gmg_level(C, l + 1);
    const int Iy = I / G.W, Ix = I - Iy * G.W;
    for (int op = 0; op < 2; ++op) {
        double acc[9];
        for (int k = 0; k < 9; ++k) acc[k] = 0.0;
        for (int b = -1; b <= 1; ++b) {
            const int fy = 2 * Iy + b;
            if (fy < 0 || fy > F.ny) continue;
            for (int a = -1; a <= 1; ++a) {
                const int fx = 2 * Ix + a;
                if (fx < 0 || fx > F.nx) continue;
                const double wi = (a == 0 ? 1.0 : 0.5) * (b == 0 ? 1.0 : 0.5);
                const int fi = fy * F.W + fx;
                if (l == 0 && B.mask[fi]) continue;
                double row[9];
                gmg_row64(C, B, op, l, fi, row);
                for (int k = 0; k < 9; ++k) {
                    if (row[k] == 0.0) continue;
                    const int jx = fx + nb_dx(k), jy = fy + nb_dy(k);
                    if (jx < 0 || jx > F.nx || jy < 0 || jy > F.ny) continue;
                    if (l == 0 && B.mask[jy * F.W + jx]) continue;
                    const double v = wi * row[k];
                    const int kx0 = jx >> 1, ky0 = jy >> 1;
                    const int kx1 = (jx & 1) ? kx0 + 1 : kx0, ky1 = (jy & 1) ? ky0 + 1 : ky0;
                    const double wkx = (jx & 1) ? 0.5 : 1.0, wky = (jy & 1) ? 0.5 : 1.0;
                    for (int ky = ky0; ky <= ky1; ++ky)
                        for (int kx = kx0; kx <= kx1; ++kx)
                            acc[(kx - Ix + 1) + 3 * (ky - Iy + 1)] += v * wkx * wky;
                }
            }
        }
        // 3x3 block (dx + 1) + 3 (dy + 1) to the order c, e, w, n, s, ne, nw, se, sw
        const double st[9] = {acc[4], acc[5], acc[3], acc[7], acc[1], acc[8], acc[6], acc[2], acc[0]};
        const size_t base = (size_t)op * 9 * C.gmg_nodes + C.gmg_off[l + 1] + I;
        double s = 0.0;
        for (int k = 0; k < 9; ++k) {
            B.gA64[base + (size_t)k * C.gmg_nodes] = st[k];
            reinterpret_cast<Real *>(B.gA)[base + (size_t)k * C.gmg_nodes] = (Real)st[k];
            s += fabs(st[k]);
        }
        if (st[0] > 0.0) atomic_max_pos(&B.gmg_g[op * kMaxLevels + l + 1], s / st[0]);
    }
}

__global__ void k_gmg_rap(const EngineDesc *__restrict__ D, int l) {
    const EngineDesc &E = D[blockIdx.y];
    const Consts &C = E.C;
    const Bufs &B = E.B;
    if (!C.gmg || l + 1 >= C.gmg_L) return;
    const Lvl G = gmg_level(C, l + 1);
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < G.Nn; I += gridDim.x * blockDim.x) {
        if (C.fp32) gmg_rap_node<float>(C, B, l, I);
        else gmg_rap_node<double>(C, B, l, I);
    }
}

// Zeroes the bounds (blockIdx.x = design) before the level kernels run.
__global__ void k_gmg_reset(const EngineDesc *__restrict__ D) {
    const EngineDesc &E = D[blockIdx.x];
    if (!E.C.gmg) return;
    for (int k = threadIdx.x; k < 2 * kMaxLevels; k += blockDim.x) E.B.gmg_g[k] = 0.0;
}

// Damping per operator and level from its Gershgorin bound.
__global__ void k_gmg_omega(const EngineDesc *__restrict__ D) {
    const EngineDesc &E = D[blockIdx.x];
    if (!E.C.gmg) return;
    for (int k = threadIdx.x; k < 2 * kMaxLevels; k += blockDim.x) {
        const double g = E.B.gmg_g[k];
        E.B.gmg_w[k] = g > 0.0 ? E.C.gmg_omega / g : 0.0;
    }
}
