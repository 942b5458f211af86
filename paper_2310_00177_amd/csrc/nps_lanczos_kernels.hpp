// Kernels of the Ritz-vector right-hand-side generator (training data of
// Sec. "Training"): Lanczos on the system matrix with full
// reorthogonalisation (the Gram-Schmidt products run on rocBLAS), then
// normalised combinations of Ritz vectors.  Every scalar of the recurrence
// (alpha_j, beta_j) lives in device memory, so no step waits for the host.
#pragma once

#include "nps_kernels.hpp"

namespace nps {

constexpr int kLzBlocks = 1024;   // grid of the Lanczos reductions and vector updates

// out = in on fluid cells, 0 elsewhere.
__global__ __launch_bounds__(kBlock) void k_lz_mask(size_t n, const uint8_t* __restrict__ lab,
                                                    const double* __restrict__ in, double* __restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        out[i] = lab[i] == kFluid ? in[i] : 0.0;
}

// Per-block partial of a . b (value 0 of the partials).
__global__ __launch_bounds__(kBlock) void k_lz_dot(size_t n, const double* __restrict__ a, const double* __restrict__ b,
                                                   double* partials) {
    double v[kRedWidth] = {0.0, 0.0, 0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) v[0] += a[i] * b[i];
    block_partials<kBlock>(v, partials);
}

// *out = sum of the nparts partials of value 0 (block order); SQRT: its root.
template <bool SQRT>
__global__ __launch_bounds__(kBlock) void k_lz_reduce(const double* __restrict__ partials, int nparts,
                                                      double* __restrict__ out) {
    double v[1];
    sum_partials<1, kBlock>(partials, nparts, 1, v);
    if (threadIdx.x == 0) *out = SQRT ? sqrt(v[0]) : v[0];
}

// w -= alpha_j v_j + beta_(j-1) v_(j-1)   (beta_prev null on the first step).
__global__ __launch_bounds__(kBlock) void k_lz_update(size_t n, double* __restrict__ w, const double* __restrict__ vj,
                                                      const double* __restrict__ vprev, const double* __restrict__ alpha_j,
                                                      const double* __restrict__ beta_prev) {
    const double a = *alpha_j, bp = beta_prev ? *beta_prev : 0.0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        double t = w[i] - a * vj[i];
        if (beta_prev) t -= bp * vprev[i];
        w[i] = t;
    }
}

// v_(j+1) = w / beta_j, or zero once beta_j falls below 1e-12 max(|alpha_1|, 1)
// (an invariant subspace: the steps from there on produce zeros; the host
// finds the step count from the betas).
__global__ __launch_bounds__(kBlock) void k_lz_next(size_t n, const double* __restrict__ w,
                                                    const double* __restrict__ beta_j, const double* __restrict__ alpha_1,
                                                    double* __restrict__ vnext) {
    const double b = *beta_j;
    const double thr = 1e-12 * fmax(fabs(*alpha_1), 1.0);
    const double inv = b >= thr ? 1.0 / b : 0.0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        vnext[i] = w[i] * inv;
}

// v = w / ||w|| with the norm already in *nrm.
__global__ __launch_bounds__(kBlock) void k_lz_scale(size_t n, const double* __restrict__ w,
                                                     const double* __restrict__ nrm, double* __restrict__ v) {
    const double inv = *nrm > 0.0 ? 1.0 / *nrm : 0.0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) v[i] = w[i] * inv;
}

// y = the m x m identity (column-major).
__global__ __launch_bounds__(kBlock) void k_identity(int m, double* __restrict__ y) {
    const size_t mm = (size_t)m * m;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < mm; i += (size_t)gridDim.x * kBlock)
        y[i] = (i % (size_t)(m + 1)) == 0 ? 1.0 : 0.0;
}

// Column c of r (n rows, column-major) scaled to unit 2-norm; one block per column.
__global__ __launch_bounds__(1024) void k_unit_columns(size_t n, double* __restrict__ r) {
    double* col = r + (size_t)blockIdx.x * n;
    double s = 0.0;
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) s += col[i] * col[i];
    __shared__ double sh[1024 / 64];
    __shared__ double inv;
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) t += sh[i];
        inv = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
    }
    __syncthreads();
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) col[i] *= inv;
}

}  // namespace nps
