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
// The batched steps G(R u^k_n), the cold sweep and the sequential correction
// sweep run as lanes of the engine (the coarse-mesh lanes). This file holds
// the coarse-mesh set-up (coefficients and assembled stencils) and the
// kernels around the engine launches: the fine guesses of a cold start
// (the cold sweep prolonged), the corrected fine states
// F_n + P(G(u^{k+1}_n) - G(u^k_n)) (Eq. 4.10 / Eq. 4.14 with both coarse
// outputs prolonged by the same linear P) and the sensitivity part of the
// reversed correction, linear in the coarse output difference and summed per
// fine element (Eq. 4.16).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "pt.h"
#include "pt_internal.h"

namespace pt {

namespace {

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

__device__ __forceinline__ double *crow(double *base, const CoarseMesh &M, int n) {
    return base + (size_t)n * M.Nc;
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

}  // namespace

int cm_setup(const EngineDesc *D, const CoarseMesh &M, hipStream_t stream) {
    hipLaunchKernelGGL(k_cm_coef, dim3((M.Nec + 255) / 256), dim3(256), 0, stream, D, M);
    hipLaunchKernelGGL(k_cm_stencil, dim3((M.Nc + 255) / 256), dim3(256), 0, stream, D, M);
    return cm_check();
}

int cm_guess(const EngineDesc *D, const CoarseMesh &M, int Nn, int Ntau, bool adjoint,
             double *rows, double *th, hipStream_t stream) {
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
