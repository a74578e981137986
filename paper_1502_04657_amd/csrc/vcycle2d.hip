// Fused, temporally blocked V-cycle level kernels for the 2D mesh family.
//
// A V(nu,nu) level is two passes over the fine arrays instead of ~14:
//   pre : y <- NH red-black half sweeps on x, then r_c = P^T (f - K y)   (read x, f; write y, r_c)
//   post: x <- y + P x_c, then NH red-black half sweeps                   (read y, f, x_c; write x)
// Each pass reads one array and writes another (y is a scratch level array): a workgroup
// reads a halo around its tile, so an in-place pass would let it read nodes that a
// neighbouring workgroup has already overwritten.
// with NH = 2 nu + 1 (the symmetric sweeps R,B,B,R,... collapse to R,B,R,... because a
// repeated half sweep of the same colour changes nothing).  Each workgroup owns a TX x TY
// tile, loads it with a halo of HALO nodes into LDS, and runs the half sweeps on shrinking
// regions (the dependency cone of the tile), so only the tile is written back.  Every node
// update, residual and restriction uses exactly the expression of the unfused kernels in
// grid.hip, so the fused and unfused paths produce identical bits.
#include <hip/hip_ext.h>

#include <utility>

#include "kernels.h"

namespace fmg {

namespace {

constexpr int THREADS = 256;

template <typename T>
__device__ inline T gs2f(T f, T w, T e, T s, T n) {
    return (f + ((w + e) + (s + n))) * T(0.25);
}

// Red-black half sweeps on the LDS region.  Region coordinates: column c in [0, RW),
// row r in [0, RH); global node (gi, gj) = (i0 - HALO + c, j0 - HALO + r).  Half sweep S
// updates the colour-`col` interior nodes within distance ext = R + NH - 1 - S of the tile:
// a (TX + 2 ext) x (TY + 2 ext) rectangle holding (TX/2 + ext) nodes of each colour per row.
// The nodes of one colour are independent, so the workgroup takes them as one flat list
// (compile-time sizes, no partly idle row passes); nodes outside the domain are skipped.
template <typename T, int TX, int TY, int HALO, int NH, int R, int S>
__device__ inline void half_sweep(T* xs, const T* fs, int i0, int j0, int n, int col) {
    constexpr int RW = TX + 2 * HALO;
    constexpr int ext = R + NH - 1 - S;
    constexpr int HW = TX / 2 + ext, NI = (TY + 2 * ext) * HW;
    const int ia = i0 - ext, ja = j0 - ext;
    for (int k = threadIdx.x; k < NI; k += THREADS) {
        const int r = k / HW, m = k - r * HW;
        const int gj = ja + r;
        const int gi = ia + 2 * m + ((col - gj - ia) & 1);   // nodes with (gi + gj) % 2 == col
        if (gi >= 1 && gi <= n - 1 && gj >= 1 && gj <= n - 1) {
            const int p = (gi - (i0 - HALO)) + RW * (r + HALO - ext);
            xs[p] = gs2f<T>(fs[p], xs[p - 1], xs[p + 1], xs[p - RW], xs[p + RW]);
        }
    }
    __syncthreads();
}

template <typename T, int TX, int TY, int HALO, int NH, int R, int... S>
__device__ inline void half_sweeps_seq(T* xs, const T* fs, int i0, int j0, int n, int first,
                                       std::integer_sequence<int, S...>) {
    (half_sweep<T, TX, TY, HALO, NH, R, S>(xs, fs, i0, j0, n, first ^ (S & 1)), ...);
}

template <typename T, int TX, int TY, int HALO, int NH, int R>
__device__ inline void half_sweeps(T* xs, const T* fs, int i0, int j0, int n, int first) {
    half_sweeps_seq<T, TX, TY, HALO, NH, R>(xs, fs, i0, j0, n, first, std::make_integer_sequence<int, NH>{});
}

// Loads the tile plus HALO rings of x (zero when zero_x) and f into LDS.  PROLONG adds the
// coarse correction P x_c on the interior nodes of the region (the expression of k_prolong).
// Every thread issues the loads of all its region nodes before the first LDS write, so a
// workgroup waits for memory once instead of once per node it loads.
template <typename T, int TX, int TY, int HALO, bool PROLONG>
__device__ inline void load_region(T* xs, T* fs, const T* __restrict__ x, const T* __restrict__ f,
                                   const T* __restrict__ xc, const Grid& g, const Grid& gc, int i0, int j0,
                                   int zero_x) {
    constexpr int RW = TX + 2 * HALO, RH = TY + 2 * HALO, NR = RW * RH;
    constexpr int NT = (NR + THREADS - 1) / THREADS;
    const int n = g.n;
    T xv[NT], fv[NT], c0[NT], c1[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        xv[k] = T(0); fv[k] = T(0); c0[k] = T(0); c1[k] = T(0);
        const int t = threadIdx.x + k * THREADS;
        if (t < NR) {
            const int r = t / RW, c = t - r * RW;
            const int gi = i0 - HALO + c, gj = j0 - HALO + r;
            if (gi >= 0 && gi <= n && gj >= 0 && gj <= n) {
                const int64_t q = gi + g.pitch * gj;
                if (!zero_x) xv[k] = x[q];
                fv[k] = f[q];
            }
            if (PROLONG && gi >= 1 && gi <= n - 1 && gj >= 1 && gj <= n - 1) {
                const int di = gi & 1, dj = gj & 1;
                const int64_t q0 = (gi >> 1) + gc.pitch * (gj >> 1);
                c0[k] = xc[q0];
                if (di | dj) c1[k] = xc[q0 + di + gc.pitch * dj];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int t = threadIdx.x + k * THREADS;
        if (t < NR) {
            T v = xv[k];
            if (PROLONG) {
                const int r = t / RW, c = t - r * RW;
                const int gi = i0 - HALO + c, gj = j0 - HALO + r;
                if (gi >= 1 && gi <= n - 1 && gj >= 1 && gj <= n - 1) {
                    T p = c0[k];
                    if ((gi & 1) | (gj & 1)) p = T(0.5) * (p + c1[k]);
                    v += p;
                }
            }
            xs[t] = v;
            fs[t] = fv[k];
        }
    }
}

template <typename T, int TX, int TY, int HALO>
__device__ inline void store_tile(const T* xs, T* __restrict__ x, const Grid& g, int i0, int j0) {
    constexpr int RW = TX + 2 * HALO;
    const int n = g.n;
    for (int t = threadIdx.x; t < TX * TY; t += THREADS) {
        const int r = t / TX, c = t - r * TX;
        const int gi = i0 + c, gj = j0 + r;
        if (gi <= n - 1 && gj <= n - 1) x[gi + g.pitch * gj] = xs[(c + HALO) + RW * (r + HALO)];
    }
}

// pre-smoothing + residual + restriction
template <typename T, int NH, int TX, int TY>
__global__ __launch_bounds__(THREADS) void k_vpre2d(const T* __restrict__ x, T* __restrict__ y,
                                                    const T* __restrict__ f, T* __restrict__ rc, Grid g, Grid gc,
                                                    int zero_x) {
    constexpr int R = 2;                 // x must be final within 2 rings for the residual ring
    constexpr int HALO = NH + R;
    constexpr int RW = TX + 2 * HALO, RH = TY + 2 * HALO;
    __shared__ T xs[RW * RH];
    __shared__ T fs[RW * RH];
    const int i0 = 1 + blockIdx.x * TX, j0 = 1 + blockIdx.y * TY;
    const int n = g.n;
    load_region<T, TX, TY, HALO, false>(xs, fs, x, f, nullptr, g, gc, i0, j0, zero_x);
    __syncthreads();
    half_sweeps<T, TX, TY, HALO, NH, R>(xs, fs, i0, j0, n, 0);
    // residual r = f - K x on the tile and one ring, stored over f
    {
        constexpr int W1 = TX + 2, H1 = TY + 2;
        for (int t = threadIdx.x; t < W1 * H1; t += THREADS) {
            const int r = t / W1, c = t - r * W1;
            const int gi = i0 - 1 + c, gj = j0 - 1 + r;
            if (gi < 1 || gi > n - 1 || gj < 1 || gj > n - 1) continue;
            const int p = (c - 1 + HALO) + RW * (r - 1 + HALO);
            fs[p] = fs[p] - (T(4) * xs[p] - ((xs[p - 1] + xs[p + 1]) + (xs[p - RW] + xs[p + RW])));
        }
    }
    __syncthreads();
    store_tile<T, TX, TY, HALO>(xs, y, g, i0, j0);
    // restriction for the coarse nodes whose centre 2I, 2J lies in this tile
    {
        constexpr int CW = TX / 2, CH = TY / 2;
        const int nc = gc.n;
        for (int t = threadIdx.x; t < CW * CH; t += THREADS) {
            const int r = t / CW, c = t - r * CW;
            const int I = (i0 + 1) / 2 + c, J = (j0 + 1) / 2 + r;
            if (I > nc - 1 || J > nc - 1) continue;
            const int p = (2 * I - i0 + HALO) + RW * (2 * J - j0 + HALO);
            const T e = (fs[p - 1] + fs[p + 1]) + (fs[p - RW] + fs[p + RW]) + (fs[p - 1 - RW] + fs[p + 1 + RW]);
            rc[I + gc.pitch * J] = fs[p] + T(0.5) * e;
        }
    }
}

// prolongation + correction + post-smoothing
template <typename T, int NH, int TX, int TY>
__global__ __launch_bounds__(THREADS) void k_vpost2d(const T* __restrict__ y, T* __restrict__ x,
                                                     const T* __restrict__ f, const T* __restrict__ xc, Grid g,
                                                     Grid gc) {
    constexpr int R = 0;
    constexpr int HALO = NH > 0 ? NH + R : 1;
    constexpr int RW = TX + 2 * HALO, RH = TY + 2 * HALO;
    __shared__ T xs[RW * RH];
    __shared__ T fs[RW * RH];
    const int i0 = 1 + blockIdx.x * TX, j0 = 1 + blockIdx.y * TY;
    const int n = g.n;
    // x = y + P x_c on every interior node of the region
    load_region<T, TX, TY, HALO, true>(xs, fs, y, f, xc, g, gc, i0, j0, 0);
    __syncthreads();
    half_sweeps<T, TX, TY, HALO, NH, R>(xs, fs, i0, j0, n, 0);
    store_tile<T, TX, TY, HALO>(xs, x, g, i0, j0);
}

// Tile shape by level: 64 x 32 where the level has many tiles, 16 x 16 on coarse levels
// (more workgroups, shorter sweeps; the halo overhead is irrelevant there).
constexpr int kSmallLevel = 256;


template <typename T, int NH>
void pre_launch(const Grid& g, const Grid& gc, const T* x, T* y, const T* f, T* rc, int zero_x, hipStream_t s) {
    if (g.n <= kSmallLevel) {
        dim3 grd(cdiv(g.n - 1, 16), cdiv(g.n - 1, 16));
        hipLaunchKernelGGL((k_vpre2d<T, NH, 16, 16>), grd, dim3(THREADS), 0, s, x, y, f, rc, g, gc, zero_x);
    } else {
        dim3 grd(cdiv(g.n - 1, 64), cdiv(g.n - 1, 32));
        hipLaunchKernelGGL((k_vpre2d<T, NH, 64, 32>), grd, dim3(THREADS), 0, s, x, y, f, rc, g, gc, zero_x);
    }
}
template <typename T, int NH>
void post_launch(const Grid& g, const Grid& gc, const T* y, T* x, const T* f, const T* xc, hipStream_t s,
                 hipEvent_t ev0, hipEvent_t ev1) {
    if (g.n <= kSmallLevel) {
        dim3 grd(cdiv(g.n - 1, 16), cdiv(g.n - 1, 16));
        hipExtLaunchKernelGGL((k_vpost2d<T, NH, 16, 16>), grd, dim3(THREADS), 0, s, ev0, ev1, 0, y, x, f, xc, g, gc);
    } else {
        dim3 grd(cdiv(g.n - 1, 64), cdiv(g.n - 1, 32));
        hipExtLaunchKernelGGL((k_vpost2d<T, NH, 64, 32>), grd, dim3(THREADS), 0, s, ev0, ev1, 0, y, x, f, xc, g, gc);
    }
}

}  // namespace

bool vpass2d_wide_tiles(const Grid& g) { return g.n > kSmallLevel; }

template <typename T>
bool launch_vpre2d(const Grid& g, const Grid& gc, const T* x, T* y, const T* f, T* rc, int nu, int zero_x,
                   hipStream_t s) {
    switch (nu) {
        case 0: pre_launch<T, 0>(g, gc, x, y, f, rc, zero_x, s); return true;
        case 1: pre_launch<T, 3>(g, gc, x, y, f, rc, zero_x, s); return true;
        case 2: pre_launch<T, 5>(g, gc, x, y, f, rc, zero_x, s); return true;
        default: return false;
    }
}
template <typename T>
bool launch_vpost2d(const Grid& g, const Grid& gc, const T* y, T* x, const T* f, const T* xc, int nu,
                    hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    switch (nu) {
        case 0: post_launch<T, 0>(g, gc, y, x, f, xc, s, ev0, ev1); return true;
        case 1: post_launch<T, 3>(g, gc, y, x, f, xc, s, ev0, ev1); return true;
        case 2: post_launch<T, 5>(g, gc, y, x, f, xc, s, ev0, ev1); return true;
        default: return false;
    }
}
template bool launch_vpre2d<double>(const Grid&, const Grid&, const double*, double*, const double*, double*, int,
                                    int, hipStream_t);
template bool launch_vpre2d<float>(const Grid&, const Grid&, const float*, float*, const float*, float*, int, int,
                                   hipStream_t);
template bool launch_vpost2d<double>(const Grid&, const Grid&, const double*, double*, const double*,
                                     const double*, int, hipStream_t, hipEvent_t, hipEvent_t);
template bool launch_vpost2d<float>(const Grid&, const Grid&, const float*, float*, const float*, const float*, int,
                                    hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace fmg
