// Exact coarsest-level solve by the discrete sine transform, shared by the coarsest-level
// kernel and the one-workgroup bottom of the 2D V-cycle (same arithmetic in both).
//
// K is the Kronecker sum of the 1D matrix tridiag(-1,2,-1) (times h in 3D), diagonalised by
// the discrete sine transform S_ab = sin(pi a b / n):
//   x = (2/n)^D (S x..x S) diag(1 / (h^(D-2) sum_k mu_k)) (S x..x S) f,
//   mu_a = 4 sin^2(pi a / (2n)).
// One workgroup; the m^D values (m = n-1) live in `sm` (m^2 + m + 2 m^D doubles of LDS).
// FP64 internally.  f and x are level arrays with the given pitch and plane stride (global
// memory or LDS).
#pragma once

#include "common.h"

namespace fmg {

__device__ inline void dst_axis(const double* __restrict__ src, double* __restrict__ dst, const double* __restrict__ S,
                                int m, int D, int axis) {
    int total = (D == 2) ? m * m : m * m * m;
    int st = (axis == 0) ? 1 : (axis == 1 ? m : m * m);
    for (int o = threadIdx.x; o < total; o += blockDim.x) {
        int q = (o / st) % m;
        int base = o - q * st;
        double acc = 0.0;
        for (int a = 0; a < m; ++a) acc += src[base + a * st] * S[a * m + q];
        dst[o] = acc;
    }
}

template <typename T>
__device__ inline void coarse_dst_solve(const T* f, T* x, int64_t pitch, int64_t plane, int n, int D, const double* aw,
                                        double* sm) {
    const int m = n - 1;
    const int total = (D == 2) ? m * m : m * m * m;
    double* S = sm;
    double* mu = S + m * m;
    double* A = mu + m;
    double* B = A + total;
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
        int a = t / m + 1, b = t % m + 1;
        S[t] = sinpi((double)((a * b) % (2 * n)) / n);
    }
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        double s = sinpi((double)(t + 1) / (2.0 * n));
        mu[t] = 4.0 * s * s;
    }
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        int i = t % m + 1, r = t / m;
        int64_t p = (D == 2) ? i + pitch * (r + 1) : i + pitch * (r % m + 1) + plane * (r / m + 1);
        A[t] = (double)f[p];
    }
    __syncthreads();
    dst_axis(A, B, S, m, D, 0);
    __syncthreads();
    dst_axis(B, A, S, m, D, 1);
    __syncthreads();
    double* cur = A;
    double* oth = B;
    if (D == 3) {
        dst_axis(A, B, S, m, D, 2);
        __syncthreads();
        cur = B;
        oth = A;
    }
    const double scale = (D == 2) ? (2.0 / n) * (2.0 / n) : (2.0 / n) * (2.0 / n) * (2.0 / n) * n;  // 1/h in 3D
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        int a = t % m, r = t / m;
        // eigenvalues of K = sum_d a_d K_d: weighted sums of the 1D eigenvalues (fused
        // multiply-adds written out, so every caller rounds alike)
        double lam = (D == 2) ? fma(aw[1], mu[r], aw[0] * mu[a])
                              : fma(aw[2], mu[r / m], fma(aw[1], mu[r % m], aw[0] * mu[a]));
        cur[t] = cur[t] * scale / lam;
    }
    __syncthreads();
    dst_axis(cur, oth, S, m, D, 0);
    __syncthreads();
    dst_axis(oth, cur, S, m, D, 1);
    __syncthreads();
    double* res = cur;
    if (D == 3) {
        dst_axis(cur, oth, S, m, D, 2);
        __syncthreads();
        res = oth;
    }
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        int i = t % m + 1, r = t / m;
        int64_t p = (D == 2) ? i + pitch * (r + 1) : i + pitch * (r % m + 1) + plane * (r / m + 1);
        x[p] = (T)res[t];
    }
}

}  // namespace fmg
