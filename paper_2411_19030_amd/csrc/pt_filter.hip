// Design-field front end (Sec. 2.1): the linear density filter
//   chi_fil_e = sum_i w_ei chi_i / sum_i w_ei,   w_ei = max(0, r_fil - |x_e - x_i|)
// over element centroids x_e = ((i + 1/2)/nx, (j + 1/2)/ny), followed by the
// threshold projection
//   chi_phys = (tanh(beta (chi_fil - eta)) + tanh(beta eta))
//              / (tanh(beta (1 - eta)) + tanh(beta eta)),
// and its adjoint: grad_chi = H^T (P'(chi_fil) o grad_phys). The weights are
// symmetric in (e, i), so H^T y at i is sum_e w_ei y_e / W_e over the same
// neighbourhood. Each thread owns one element; the neighbourhood is read
// through the caches (this runs once per optimisation cycle on N_e values).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "pt.h"

namespace {

struct Geom {
    int nx, ny, Rx, Ry;
    double r;
};

constexpr int kBX = 16, kBY = 16;
constexpr long long kMaxWindow = 1ll << 18;  // neighbourhood cells per element

__device__ __forceinline__ double cone(const Geom &g, int di, int dj) {
    const double dx = (double)di / g.nx, dy = (double)dj / g.ny;
    return fmax(0.0, g.r - sqrt(dx * dx + dy * dy));
}

__device__ __forceinline__ double weight_sum(const Geom &g, int i, int j) {
    double W = 0.0;
    for (int dj = max(-g.Ry, -j); dj <= min(g.Ry, g.ny - 1 - j); ++dj)
        for (int di = max(-g.Rx, -i); di <= min(g.Rx, g.nx - 1 - i); ++di) W += cone(g, di, dj);
    return W;
}

__device__ __forceinline__ double proj(double f, double beta, double eta) {
    if (!(beta > 0.0)) return f;
    const double den = tanh(beta * (1.0 - eta)) + tanh(beta * eta);
    return (tanh(beta * (f - eta)) + tanh(beta * eta)) / den;
}

__device__ __forceinline__ double proj_deriv(double f, double beta, double eta) {
    if (!(beta > 0.0)) return 1.0;
    const double den = tanh(beta * (1.0 - eta)) + tanh(beta * eta);
    const double t = tanh(beta * (f - eta));
    return beta * (1.0 - t * t) / den;
}

__global__ void k_filter_forward(Geom g, double beta, double eta, const double *__restrict__ chi,
                                 double *__restrict__ fil, double *__restrict__ phys) {
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    double s = 0.0, W = 0.0;
    for (int dj = max(-g.Ry, -j); dj <= min(g.Ry, g.ny - 1 - j); ++dj) {
        const double *row = chi + (size_t)(j + dj) * g.nx + i;
        for (int di = max(-g.Rx, -i); di <= min(g.Rx, g.nx - 1 - i); ++di) {
            const double w = cone(g, di, dj);
            s += w * row[di];
            W += w;
        }
    }
    const double f = s / W;
    const size_t e = (size_t)j * g.nx + i;
    if (fil) fil[e] = f;
    phys[e] = proj(f, beta, eta);
}

// work_e = P'(chi_fil_e) grad_phys_e / W_e
__global__ void k_filter_scale(Geom g, double beta, double eta, const double *__restrict__ fil,
                               const double *__restrict__ grad_phys, double *__restrict__ work) {
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const size_t e = (size_t)j * g.nx + i;
    work[e] = proj_deriv(fil[e], beta, eta) * grad_phys[e] / weight_sum(g, i, j);
}

// grad_chi_i = sum_e w_ei work_e
__global__ void k_filter_adjoint(Geom g, const double *__restrict__ work,
                                 double *__restrict__ grad_chi) {
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    double s = 0.0;
    for (int dj = max(-g.Ry, -j); dj <= min(g.Ry, g.ny - 1 - j); ++dj) {
        const double *row = work + (size_t)(j + dj) * g.nx + i;
        for (int di = max(-g.Rx, -i); di <= min(g.Rx, g.nx - 1 - i); ++di)
            s += cone(g, di, dj) * row[di];
    }
    grad_chi[(size_t)j * g.nx + i] = s;
}

bool make_geom(const pt_filter *f, Geom &g) {
    if (!f) return false;
    if (f->nx < 1 || f->ny < 1 || f->nx > 16384 || f->ny > 16384) return false;
    if (!(f->r_fil > 0.0) || !std::isfinite(f->r_fil)) return false;
    if (!std::isfinite(f->beta) || !std::isfinite(f->eta) || f->eta < 0.0 || f->eta > 1.0)
        return false;
    g.nx = f->nx;
    g.ny = f->ny;
    g.r = f->r_fil;
    // |di|/nx < r for a positive weight; beyond the grid nothing is read
    const double rx = std::floor(f->r_fil * f->nx), ry = std::floor(f->r_fil * f->ny);
    g.Rx = (int)std::fmin(rx, (double)(f->nx - 1));
    g.Ry = (int)std::fmin(ry, (double)(f->ny - 1));
    if ((long long)(2 * g.Rx + 1) * (2 * g.Ry + 1) > kMaxWindow) return false;
    return true;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b) return false;
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

int launched() { return hipGetLastError() == hipSuccess ? PT_OK : PT_EHIP; }

}  // namespace

extern "C" int pt_filter_validate(const pt_filter *f) {
    Geom g;
    return make_geom(f, g) ? PT_OK : PT_EINVAL;
}

extern "C" int pt_filter_projection(const pt_filter *f, const double *chi, double *chi_fil,
                                    double *chi_phys, hipStream_t stream) {
    Geom g;
    if (!make_geom(f, g) || !chi || !chi_phys) return PT_EINVAL;
    const size_t n = (size_t)g.nx * g.ny * sizeof(double);
    if (overlap(chi, n, chi_phys, n) || overlap(chi, n, chi_fil, n) ||
        overlap(chi_fil, n, chi_phys, n))
        return PT_EINVAL;
    const dim3 grid((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY), block(kBX, kBY);
    hipLaunchKernelGGL(k_filter_forward, grid, block, 0, stream, g, f->beta, f->eta, chi, chi_fil,
                       chi_phys);
    return launched();
}

extern "C" int pt_filter_projection_backward(const pt_filter *f, const double *chi_fil,
                                             const double *grad_phys, double *work,
                                             double *grad_chi, hipStream_t stream) {
    Geom g;
    if (!make_geom(f, g) || !chi_fil || !grad_phys || !work || !grad_chi) return PT_EINVAL;
    const size_t n = (size_t)g.nx * g.ny * sizeof(double);
    if (overlap(work, n, grad_chi, n) || overlap(work, n, chi_fil, n) ||
        overlap(work, n, grad_phys, n) || overlap(grad_chi, n, chi_fil, n) ||
        overlap(grad_chi, n, grad_phys, n))
        return PT_EINVAL;
    const dim3 grid((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY), block(kBX, kBY);
    hipLaunchKernelGGL(k_filter_scale, grid, block, 0, stream, g, f->beta, f->eta, chi_fil,
                       grad_phys, work);
    hipLaunchKernelGGL(k_filter_adjoint, grid, block, 0, stream, g, work, grad_chi);
    return launched();
}
