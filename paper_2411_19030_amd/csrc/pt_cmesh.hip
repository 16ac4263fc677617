// Coarse propagators on a coarser spatial mesh (Sec. 7.3 and Sec. 8 name this
// as the way to cheapen the sequential coarse propagators; the construction
// below is this library's reading of it).
//
// The coarse mesh halves the element grid: coarse node (I, J) is fine node
// (2I, 2J). A coarse element's k and c are the means of the SIMP values of its
// four fine elements; a coarse node is fixed (T = 0) iff its fine node is.
// R is injection, P the bilinear interpolant set to 0 at fine Dirichlet nodes.
//   G_pri^c(T, theta, n): (C_c/dtau + K_c) x = C_c/dtau R T + q(tau_{n+1}) f_c,
//     output P x, theta' = (theta^p + ||P x||_p^p / (N_tau N_e))^{1/p} (Alg. 1);
//   G_adj^c(lambda, n): (C_c/dtau + K_c) x = C_c/dtau R lambda + P^T s(T_m),
//     s the fine source of Eq. 4.6 at m = M(n-1)+1, output P x (Alg. 2).
// The batched steps G(R u^k_n) and the sequential correction sweep run as
// lanes of the engine launch that runs the fine propagators (the coarse-mesh
// lanes of the engine). This file holds the coarse-mesh set-up (coefficients
// and assembled stencils), the cold sweep u^0_{n+1} = G(u^0_n) that gives a
// cold start its guesses, and the kernels after the launch: the corrected fine
// states F_n + P(G(u^{k+1}_n) - G(u^k_n)) (Eq. 4.10 / Eq. 4.14 with both coarse
// outputs prolonged by the same linear P) and the sensitivity part of the
// reversed correction, linear in the coarse output difference and summed per
// fine element (Eq. 4.16).
//
// The cold sweep's solves are Jacobi-preconditioned CG (Hestenes-Stiefel form)
// run by one workgroup of 1024 threads, with the true residual checked at the
// end; reductions are in a fixed order. The solve's vectors sit in LDS when
// they fit (about 3400 coarse nodes, e.g. the 51^2 mesh of a 100^2 design),
// else in global memory, with the same arithmetic. It runs once, before the
// first cycle of a cold start.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "pt.h"
#include "pt_internal.h"

namespace pt {

namespace {

constexpr int kCT = kCoarseMeshThreads;
constexpr int kCW = kCT / 64;

__device__ __forceinline__ double cm_ipow(double x, int n) {
    double r = 1.0, b = x;
    while (n) {
        if (n & 1) r *= b;
        b *= b;
        n >>= 1;
    }
    return r;
}

// Q1 rectangle element matrices, local nodes (0,0), (1,0), (1,1), (0,1):
// K = (1/6)(hy/hx Kx + hx/hy Ky), C = hx hy/36 Cm with the integer patterns
// below (derived from the tensor-product shape functions).
__device__ __forceinline__ int ox(int a) { return (a == 1 || a == 2) ? 1 : 0; }
__device__ __forceinline__ int oy(int a) { return a >= 2 ? 1 : 0; }
__device__ __forceinline__ double kx_pat(int a, int b) {
    return (ox(a) == ox(b) ? 1.0 : -1.0) * (oy(a) == oy(b) ? 2.0 : 1.0);
}
__device__ __forceinline__ double ky_pat(int a, int b) {
    return (oy(a) == oy(b) ? 1.0 : -1.0) * (ox(a) == ox(b) ? 2.0 : 1.0);
}
__device__ __forceinline__ double cm_pat(int a, int b) {
    return (ox(a) == ox(b) ? 2.0 : 1.0) * (oy(a) == oy(b) ? 2.0 : 1.0);
}

__device__ __forceinline__ int fine_of(const Consts &C, const CoarseMesh &M, int I) {
    const int J = I / M.Wc, i = I - J * M.Wc;
    return 2 * J * C.W + 2 * i;
}

// Row of S holding the fine state T_j (j >= 1). Store-all keeps every state;
// checkpoints keep the slice ends T_{Mn} (rows n - 1) and the slice starts
// T_{Mn+1} (rows N_tau + n), which are the only states the coarse-mesh
// kernels read (coarse points, and the adjoint's T_m and T_{m-M} with
// m = M(n-1)+1).
__device__ __forceinline__ double *cm_srow(const Consts &C, const Bufs &B, int j) {
    if (!C.ckpt) return B.S + (size_t)(j - 1) * C.Nn;
    if (j % C.M == 0) return B.S + (size_t)(j / C.M - 1) * C.Nn;
    return B.S + (size_t)(C.Ntau + (j - 1) / C.M) * C.Nn;
}

// Coarse element coefficients: means of the fine SIMP values (Eq. 2.5-2.6).
__global__ void k_cm_coef(const EngineDesc *__restrict__ D, CoarseMesh M) {
    const Consts &C = D->C;
    const Bufs &B = D->B;
    for (int E = blockIdx.x * blockDim.x + threadIdx.x; E < M.Nec; E += gridDim.x * blockDim.x) {
        const int EJ = E / M.nxc, EI = E - EJ * M.nxc;
        double ks = 0.0, cs = 0.0;
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double r = B.rho[(2 * EJ + b) * C.nx + 2 * EI + a];
                const double rr = r > 0.0 ? r : 0.0;
                ks += C.kmin + (C.k0 - C.kmin) * pow(rr, C.pk);
                cs += C.cmin + (C.c0 - C.cmin) * pow(rr, C.pc);
            }
        M.kE[E] = 0.25 * ks;
        M.cE[E] = 0.25 * cs;
    }
}

// 9-point rows of A = C_c/dtau + K_c (Dirichlet rows and columns removed),
// of C_c/dtau (Dirichlet rows removed), 1/diag(A), and the unit load
// f_c = int N_I (0 on Dirichlet nodes). Entry k = (dj+1)*3 + (di+1).
__global__ void k_cm_stencil(const EngineDesc *__restrict__ D, CoarseMesh M) {
    const Consts &C = D->C;
    const Bufs &B = D->B;
    const double Hx = 2.0 * C.hx, Hy = 2.0 * C.hy;
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < M.Nc; I += gridDim.x * blockDim.x) {
        const int J = I / M.Wc, i = I - J * M.Wc;
        const bool dir = B.mask[fine_of(C, M, I)] != 0;
        double a9[9], c9[9];
        for (int k = 0; k < 9; ++k) a9[k] = c9[k] = 0.0;
        double f = 0.0;
        // the (up to) four coarse elements around the node, and the node's
        // local index a in each
        for (int e = 0; e < 4; ++e) {
            const int EI = i - ox(e), EJ = J - oy(e);
            if (EI < 0 || EJ < 0 || EI >= M.nxc || EJ >= M.nyc) continue;
            const int a = e;
            const double kv = M.kE[EJ * M.nxc + EI], cv = M.cE[EJ * M.nxc + EI];
            f += 0.25 * Hx * Hy;
            for (int b = 0; b < 4; ++b) {
                const int di = ox(b) - ox(a), dj = oy(b) - oy(a);
                const int k = (dj + 1) * 3 + (di + 1);
                const double kab = kv * (Hy / Hx * kx_pat(a, b) + Hx / Hy * ky_pat(a, b)) / 6.0;
                const double cab = cv * Hx * Hy / 36.0 * cm_pat(a, b) * C.inv_dtau;
                c9[k] += cab;
                const int nb = (J + dj) * M.Wc + (i + di);
                const bool nb_dir = B.mask[fine_of(C, M, nb)] != 0;
                if (!nb_dir) a9[k] += kab + cab;
            }
        }
        for (int k = 0; k < 9; ++k) {
            M.A9[(size_t)k * M.Nc + I] = dir ? 0.0 : a9[k];
            M.C9[(size_t)k * M.Nc + I] = dir ? 0.0 : c9[k];
        }
        M.dinv[I] = dir ? 0.0 : 1.0 / a9[4];
        M.fc[I] = dir ? 0.0 : f;
    }
}

// 9-point row I of a stencil array applied to a coarse vector.
__device__ __forceinline__ double cm_row(const CoarseMesh &M, const double *S9, const double *x,
                                         int I) {
    const int J = I / M.Wc, i = I - J * M.Wc;
    double s = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int jj = J + dj;
        if (jj < 0 || jj > M.nyc) continue;
        for (int di = -1; di <= 1; ++di) {
            const int ii = i + di;
            if (ii < 0 || ii > M.nxc) continue;
            s += S9[(size_t)((dj + 1) * 3 + di + 1) * M.Nc + I] * x[jj * M.Wc + ii];
        }
    }
    return s;
}

// P x at fine node id (0 on fine Dirichlet nodes).
__device__ __forceinline__ double cm_prolong(const Consts &C, const CoarseMesh &M,
                                             const unsigned char *mask, const double *x, int id) {
    if (mask[id]) return 0.0;
    const int j = id / C.W, i = id - j * C.W;
    const int I = i >> 1, J = j >> 1;
    const double *r0 = x + (size_t)J * M.Wc + I;
    if (!(i & 1) && !(j & 1)) return r0[0];
    if (!(j & 1)) return 0.5 * r0[0] + 0.5 * r0[1];
    if (!(i & 1)) return 0.5 * r0[0] + 0.5 * r0[M.Wc];
    return 0.25 * r0[0] + 0.25 * r0[1] + 0.25 * r0[M.Wc] + 0.25 * r0[M.Wc + 1];
}

// P x - P y at fine node id.
__device__ __forceinline__ double cm_prolong_diff(const Consts &C, const CoarseMesh &M,
                                                  const unsigned char *mask, const double *x,
                                                  const double *y, int id) {
    return cm_prolong(C, M, mask, x, id) - cm_prolong(C, M, mask, y, id);
}

// (P^T s)_I for the fine adjoint source s_j = scale T_j^{p-1} (Eq. 4.6), with
// the bilinear weights 1, 1/2, 1/4 of the fine nodes around coarse node I.
__device__ __forceinline__ double cm_source(const Consts &C, const CoarseMesh &M,
                                            const unsigned char *mask, const double *Tm,
                                            double scale, int I) {
    const int J = I / M.Wc, i = I - J * M.Wc;
    double s = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int fj = 2 * J + dj;
        if (fj < 0 || fj > C.ny) continue;
        for (int di = -1; di <= 1; ++di) {
            const int fi = 2 * i + di;
            if (fi < 0 || fi > C.nx) continue;
            const int id = fj * C.W + fi;
            if (mask[id]) continue;
            const double w = (di == 0 ? 1.0 : 0.5) * (dj == 0 ? 1.0 : 0.5);
            s += w * (scale * cm_ipow(Tm[id], C.p - 1));
        }
    }
    return s;
}

// Sum of Q values over the workgroup in a fixed order (wave butterflies, then
// the wave totals in wave order); every thread returns the same totals.
// `red` holds 2 * Q * kCW doubles used alternately.
template <int Q>
__device__ void cm_reduce(double (&v)[Q], double *red, int &par) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double *buf = red + par * Q * kCW;
    if (l == 0)
#pragma unroll
        for (int q = 0; q < Q; ++q) buf[q * kCW + w] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double s = 0.0;
        for (int k = 0; k < kCW; ++k) s += buf[q * kCW + k];
        v[q] = s;
    }
    par ^= 1;
}

struct CmVecs {
    double *r, *z, *p, *q, *b, *u;
};

__device__ __forceinline__ CmVecs cm_vecs(const CoarseMesh &M, int slot) {
    double *base = M.vec + (size_t)slot * kCoarseMeshVecs * M.Nc;
    CmVecs V;
    V.r = base;
    V.z = base + M.Nc;
    V.p = base + 2 * (size_t)M.Nc;
    V.q = base + 3 * (size_t)M.Nc;
    V.b = base + 4 * (size_t)M.Nc;
    V.u = base + 5 * (size_t)M.Nc;
    return V;
}

// Solves (C_c/dtau + K_c) x = b on the coarse free nodes by Jacobi PCG from
// x0, to ||b - A x|| <= rtol ||b|| checked on the true residual (at most three
// restarts from it), x = 0 on Dirichlet nodes. rhs(I) and x0(I) are read once
// per node before any write to x. Records the solve in the status block.
template <typename Rhs, typename X0>
__device__ void cm_pcg(const Consts &C, const CoarseMesh &M, Control *ctl, const CmVecs &V,
                       double *x, Rhs rhs, X0 x0, double *red, int &par) {
    const int Nc = M.Nc;
    double bb[1] = {0.0};
    for (int I = threadIdx.x; I < Nc; I += kCT) {
        const bool d = M.dinv[I] == 0.0;
        const double b = d ? 0.0 : rhs(I);
        const double xv = d ? 0.0 : x0(I);
        V.b[I] = b;
        bb[0] += b * b;
        V.q[I] = xv;  // staged: x may alias the inputs rhs/x0 read
    }
    __syncthreads();
    for (int I = threadIdx.x; I < Nc; I += kCT) x[I] = V.q[I];
    cm_reduce<1>(bb, red, par);  // its barrier also completes x
    const double bnorm = sqrt(bb[0]);
    int it = 0;
    double rn = 0.0;
    if (bnorm == 0.0) {
        for (int I = threadIdx.x; I < Nc; I += kCT) x[I] = 0.0;
        __syncthreads();
    } else {
        const double tol = C.rtol * bnorm;
        for (int pass = 0;; ++pass) {
            // true residual r = b - A x, z = D^{-1} r, p = z
            double v[2] = {0.0, 0.0};
            for (int I = threadIdx.x; I < Nc; I += kCT) {
                const double r = V.b[I] - cm_row(M, M.A9, x, I);
                const double z = M.dinv[I] * r;
                V.r[I] = r;
                V.p[I] = z;
                v[0] += r * z;
                v[1] += r * r;
            }
            cm_reduce<2>(v, red, par);
            double rz = v[0];
            rn = sqrt(v[1]);
            if (rn <= tol || it >= C.max_iter || pass == 3) break;
            for (;;) {
                double w[1] = {0.0};
                for (int I = threadIdx.x; I < Nc; I += kCT) {
                    const double q = cm_row(M, M.A9, V.p, I);
                    V.q[I] = q;
                    w[0] += V.p[I] * q;
                }
                cm_reduce<1>(w, red, par);
                const double alpha = rz / w[0];
                double v2[2] = {0.0, 0.0};
                for (int I = threadIdx.x; I < Nc; I += kCT) {
                    x[I] += alpha * V.p[I];
                    const double r = V.r[I] - alpha * V.q[I];
                    const double z = M.dinv[I] * r;
                    V.r[I] = r;
                    V.z[I] = z;
                    v2[0] += r * z;
                    v2[1] += r * r;
                }
                cm_reduce<2>(v2, red, par);
                const double beta = v2[0] / rz;
                rz = v2[0];
                ++it;
                if (sqrt(v2[1]) <= tol || it >= C.max_iter) break;
                for (int I = threadIdx.x; I < Nc; I += kCT) V.p[I] = V.z[I] + beta * V.p[I];
                __syncthreads();
            }
        }
    }
    if (threadIdx.x == 0) {
        const double relres = bnorm > 0.0 ? rn / bnorm : 0.0;
        const bool conv = bnorm == 0.0 || rn <= C.rtol * bnorm;
        atomicAdd(&ctl->iters_coarse, (unsigned long long)it);
        atomicAdd(&ctl->solves_coarse, 1ull);
        atomicMax(&ctl->max_iters, it);
        atomicMax(&ctl->max_relres_bits, (unsigned long long)__double_as_longlong(relres));
        if (!conv) atomicCAS(&ctl->status, 0, PT_ENOCONV);
        if (!isfinite(relres)) atomicExch(&ctl->status, PT_EDOMAIN);
    }
    __syncthreads();
}

extern __shared__ double cm_lds[];

// The solve slot's vectors in LDS (6 Nc doubles of dynamic LDS) instead of
// global memory, for coarse meshes that fit: the same arithmetic, with the
// per-iteration vector traffic off the CU's cache path.
__device__ __forceinline__ CmVecs cm_vecs_lds(const CoarseMesh &M) {
    CmVecs V;
    V.r = cm_lds;
    V.z = cm_lds + M.Nc;
    V.p = cm_lds + 2 * (size_t)M.Nc;
    V.q = cm_lds + 3 * (size_t)M.Nc;
    V.b = cm_lds + 4 * (size_t)M.Nc;
    V.u = cm_lds + 5 * (size_t)M.Nc;
    return V;
}

// theta' = (theta^p + ||P x||_p^p / (N_tau N_e))^{1/p} (Alg. 1 with dtau, N_tau)
__device__ double cm_theta(const Consts &C, const CoarseMesh &M, const Bufs &B, const double *x,
                           double theta, double *red, int &par) {
    double s[1] = {0.0};
    for (int id = threadIdx.x; id < C.Nn; id += kCT)
        s[0] += cm_ipow(cm_prolong(C, M, B.mask, x, id), C.p);
    cm_reduce<1>(s, red, par);
    return pow(cm_ipow(theta, C.p) + s[0] * C.inv_NtauNe, C.inv_p);
}

__device__ __forceinline__ double *crow(double *base, const CoarseMesh &M, int n) {
    return base + (size_t)n * M.Nc;
}

// The cold coarse sweep on one workgroup (vectors in LDS, else slot 0):
// u^0_{n+1} = G(u^0_n) from u_0 = 0 (primal, with the theta chain into Gk_th)
// or v^0_{n-1} = G(v^0_n) from v_{N_tau} = 0 (adjoint), outputs into Gk. Each
// solve starts from its input.
template <bool LDS>
__global__ void __launch_bounds__(kCT) k_cm_cold(const EngineDesc *__restrict__ D, CoarseMesh M,
                                                 int adjoint) {
    __shared__ double red[2 * 2 * kCW];
    int par = 0;
    const Consts &C = D->C;
    const Bufs &B = D->B;
    if (B.ctl->status == kStatusOrder) return;  // adjoint with no forward before it
    const CmVecs V = LDS ? cm_vecs_lds(M) : cm_vecs(M, 0);
    const int Nt = C.Ntau;
    double *u = V.u;
    for (int I = threadIdx.x; I < M.Nc; I += kCT) u[I] = 0.0;
    __syncthreads();
    if (!adjoint) {
        double th = 0.0;
        for (int n = 0; n < Nt; ++n) {
            const double qn = B.qt[C.M * (n + 1)];
            double *x = crow(M.Gk, M, n);
            cm_pcg(
                C, M, B.ctl, V, x, [&](int I) { return cm_row(M, M.C9, u, I) + qn * M.fc[I]; },
                [&](int I) { return u[I]; }, red, par);
            th = cm_theta(C, M, B, x, th, red, par);
            if (threadIdx.x == 0) B.Gk_th[n] = th;
            for (int I = threadIdx.x; I < M.Nc; I += kCT) u[I] = x[I];
            __syncthreads();
        }
    } else {
        const double scale = pow(*B.Theta, 1.0 - C.p) / (double)C.Ne;
        for (int n = Nt; n >= 1; --n) {
            const double *Tm = cm_srow(C, B, C.M * (n - 1) + 1);
            double *x = crow(M.Gk, M, n);
            cm_pcg(
                C, M, B.ctl, V, x,
                [&](int I) {
                    return cm_row(M, M.C9, u, I) + cm_source(C, M, B.mask, Tm, scale, I);
                },
                [&](int I) { return u[I]; }, red, par);
            for (int I = threadIdx.x; I < M.Nc; I += kCT) u[I] = x[I];
            __syncthreads();
        }
    }
}

// Fine guesses from the cold sweep: primal T[n] = P Gk[n-1], th[n] = Gk_th[n-1]
// (T[0] = 0, th[0] = 0); adjoint L[n] = P Gk[n+1] (L[N_tau] = 0).
// blockIdx.y = row.
__global__ void k_cm_guess(const EngineDesc *__restrict__ D, CoarseMesh M, int adjoint,
                           double *rows, double *th) {
    const Consts &C = D->C;
    const Bufs &B = D->B;
    const int n = blockIdx.y;
    double *out = rows + (size_t)n * C.Nn;
    const int src = adjoint ? n + 1 : n - 1;
    const bool zero = adjoint ? n == C.Ntau : n == 0;
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < C.Nn; id += gridDim.x * blockDim.x)
        out[id] = zero ? 0.0 : cm_prolong(C, M, B.mask, crow(M.Gk, M, src), id);
    if (!adjoint && blockIdx.x == 0 && threadIdx.x == 0) th[n] = zero ? 0.0 : B.Gk_th[n - 1];
}

// Corrected fine states (blockIdx.y = n):
// primal u^{k+1}_{n+1} = F_n + P(Gn[n] - Gk[n]) into S row M(n+1) and out_T[n+1]
// (n = 0: F_0); adjoint lambda^{k+1}_{n-1} = F_n + P(Gn[n] - Gk[n]) into
// out_L[n-1] (n = N_tau: F_{N_tau}), and out_L[N_tau] = 0.
__global__ void k_cm_correct(const EngineDesc *__restrict__ D, CoarseMesh M, int adjoint) {
    const Consts &C = D->C;
    const Bufs &B = D->B;
    const int n = blockIdx.y + (adjoint ? 1 : 0);
    const bool corr = adjoint ? n < C.Ntau : n > 0;
    const double *gn = crow(M.Gn, M, n), *gk = crow(M.Gk, M, n);
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < C.Nn;
         id += gridDim.x * blockDim.x) {
        const double d = corr ? cm_prolong_diff(C, M, B.mask, gn, gk, id) : 0.0;
        if (!adjoint) {
            double *row = cm_srow(C, B, C.M * (n + 1));
            const double v = row[id] + d;
            row[id] = v;
            B.out_T[(size_t)(n + 1) * C.Nn + id] = v;
        } else {
            B.out_L[(size_t)(n - 1) * C.Nn + id] = B.FL[(size_t)n * C.Nn + id] + d;
            if (n == C.Ntau) B.out_L[(size_t)C.Ntau * C.Nn + id] = 0.0;
        }
    }
}

// accG_e = sum_{n=1}^{N_tau-1} lambda_n^T (dC (T_m - T_{m-M})/dtau + dK T_m) on
// fine element e, lambda_n = P(Gn[n] - Gk[n]), m = M(n-1)+1 (T_{m-M} = 0 when
// m - M < 1): the coarse-correction part of the summed Eq. 4.16.
__global__ void k_cm_sens(const EngineDesc *__restrict__ D, CoarseMesh M) {
    const Consts &C = D->C;
    const Bufs &B = D->B;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < C.Ne; e += gridDim.x * blockDim.x) {
        const int ey = e / C.nx, ex = e - ey * C.nx;
        int id[4];
        for (int a = 0; a < 4; ++a) id[a] = (ey + oy(a)) * C.W + ex + ox(a);
        double sk = 0.0, sc = 0.0;
        for (int n = 1; n < C.Ntau; ++n) {
            const double *gn = crow(M.Gn, M, n), *gk = crow(M.Gk, M, n);
            const int m = C.M * (n - 1) + 1;
            const double *Tm = cm_srow(C, B, m);
            const double *Tp = m - C.M >= 1 ? cm_srow(C, B, m - C.M) : nullptr;
            double l[4], t[4], dt[4];
            for (int a = 0; a < 4; ++a) {
                l[a] = cm_prolong_diff(C, M, B.mask, gn, gk, id[a]);
                t[a] = Tm[id[a]];
                dt[a] = t[a] - (Tp ? Tp[id[a]] : 0.0);
            }
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    sk += l[a] * (C.hy / C.hx * kx_pat(a, b) + C.hx / C.hy * ky_pat(a, b)) * t[b];
                    sc += l[a] * cm_pat(a, b) * dt[b];
                }
        }
        B.accG[e] = B.dk[e] * sk / 6.0 + B.dc[e] * C.inv_dtau * C.hx * C.hy / 36.0 * sc;
    }
}

int cm_check() { return hipGetLastError() == hipSuccess ? PT_OK : PT_EHIP; }

// LDS-resident solve vectors when allowed and they fit the workgroup's LDS.
size_t cm_lds_bytes(const CoarseMesh &M, bool use_lds) {
    if (!use_lds) return 0;
    int dev = 0, cap = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    const size_t need = sizeof(double) * kCoarseMeshVecs * (size_t)M.Nc;
    const size_t fixed = sizeof(double) * 2 * 2 * kCW;  // the reduction buffer
    return need + fixed <= (size_t)cap ? need : 0;
}

// Launches kernel K<true> with the vectors in LDS when they fit, else K<false>.
template <template <bool> class K, typename... Args>
int cm_launch(const CoarseMesh &M, bool use_lds, dim3 grid, hipStream_t stream, Args... args) {
    const size_t lds = cm_lds_bytes(M, use_lds);
    if (lds > 0) {
        auto kern = K<true>::kernel();
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return PT_EHIP;
        hipLaunchKernelGGL(kern, grid, dim3(kCT), (unsigned)lds, stream, args...);
    } else {
        hipLaunchKernelGGL(K<false>::kernel(), grid, dim3(kCT), 0, stream, args...);
    }
    return cm_check();
}

template <bool LDS>
struct ColdK {
    static auto kernel() { return &k_cm_cold<LDS>; }
};

}  // namespace

int cm_setup(const EngineDesc *D, const CoarseMesh &M, hipStream_t stream) {
    hipLaunchKernelGGL(k_cm_coef, dim3((M.Nec + 255) / 256), dim3(256), 0, stream, D, M);
    hipLaunchKernelGGL(k_cm_stencil, dim3((M.Nc + 255) / 256), dim3(256), 0, stream, D, M);
    return cm_check();
}

int cm_cold(const EngineDesc *D, const CoarseMesh &M, int Nn, int Ntau, bool adjoint,
            double *rows, double *th, bool use_lds, hipStream_t stream) {
    const int rc = cm_launch<ColdK>(M, use_lds, dim3(1), stream, D, M, adjoint ? 1 : 0);
    if (rc != PT_OK) return rc;
    hipLaunchKernelGGL(k_cm_guess, dim3(std::min((Nn + 255) / 256, 1024), Ntau + 1), dim3(256),
                       0, stream, D, M, adjoint ? 1 : 0, rows, th);
    return cm_check();
}

int cm_correct(const EngineDesc *D, const CoarseMesh &M, int Nn, int Ntau, bool adjoint, int Ne,
               hipStream_t stream) {
    hipLaunchKernelGGL(k_cm_correct, dim3(std::min((Nn + 255) / 256, 1024), Ntau), dim3(256), 0,
                       stream, D, M, adjoint ? 1 : 0);
    if (adjoint)
        hipLaunchKernelGGL(k_cm_sens, dim3(std::min((Ne + 255) / 256, 4096)), dim3(256), 0,
                           stream, D, M);
    return cm_check();
}

}  // namespace pt
