// Fused, temporally blocked V-cycle level kernels for the 2D mesh family.
//
// A V(nu,nu) level is two passes over the fine arrays instead of ~14:
//   pre : y <- NH red-black half sweeps on x, then r_c = P^T (f - K y)   (read x, f; write y, r_c)
//   post: x <- y + P x_c, then NH red-black half sweeps                   (read y, f, x_c; write x)
// Each pass reads one array and writes another (y is a scratch level array): a workgroup
// reads a halo around its tile, so an in-place pass would let it read nodes that a
// neighbouring workgroup has already overwritten.
// NH = 2 nu + 1 (the symmetric sweeps R,B,B,R,... collapse to R,B,R,... because a repeated
// half sweep of the same colour changes nothing).  Each workgroup owns a TX x TY tile, reads
// it with a halo of HALO nodes, and runs the half sweeps on shrinking regions (the
// dependency cone of the tile), so only the tile is written back.  Each thread keeps f of
// the nodes it owns in registers; LDS holds x only.  Every node update, residual and
// restriction uses exactly the expression of the unfused kernels in grid.hip, so the fused
// and unfused paths produce identical bits.
#include <hip/hip_ext.h>

#include <algorithm>
#include <utility>

#include "dst.h"
#include "kernels.h"

namespace fmg {

namespace {

template <typename T>
__device__ inline T gs2f(const Stencil<T>& k, T f, T w, T e, T s, T n) {
    return gsu2(k, f, w, e, s, n);
}

// The LDS region of a workgroup: its TX x TY tile plus HALO rings, RW x RH nodes, region
// column c / row r <-> global node (i0 - HALO + c, j0 - HALO + r).  The region is cut into
// horizontal node pairs (columns 2p, 2p+1 of a row; RW is even); thread t owns pairs
// t, t + NT, ... for the whole pass and keeps their f in registers.  LDS holds
// only x, for the neighbour reads of the sweeps.  Each half sweep updates, in every owned
// pair, the node of the sweep's colour, so all owners of pairs inside the sweep's
// rectangle work in every half sweep.
template <int TX, int TY, int HALO, int NT>
struct Region {
    static constexpr int RW = TX + 2 * HALO, RH = TY + 2 * HALO;
    static constexpr int HP = RW / 2;                         // pairs per row
    static constexpr int NP = HP * RH;                        // pairs
    static constexpr int K = (NP + NT - 1) / NT;              // pairs per thread
    static_assert(RW % 2 == 0, "region rows hold whole pairs");
};

// per-thread values of the owned pairs
template <typename T, int TX, int TY, int HALO, int NT>
using PairVals = T[Region<TX, TY, HALO, NT>::K];

// The region's x in LDS as two colour planes (red nodes, black nodes), each RH rows of HP
// values: node (c, r) of colour k = (c + r + base) & 1 sits at plane k, row r, slot c / 2.
// The nodes a half sweep updates, and the neighbours it reads, are then consecutive in LDS
// across the lanes (no bank conflicts from the every-other-node pattern of one colour).
template <typename T, int TX, int TY, int HALO, int NT>
struct Planes {
    using Rg = Region<TX, TY, HALO, NT>;
    static constexpr int PL = Rg::RH * Rg::HP;
    T* x;
    int base;   // colour of region node (0, 0)
    Stencil<T> k;   // the level's stiffness stencil
    __device__ T& at(int c, int r) const { return x[((c + r + base) & 1) * PL + r * Rg::HP + (c >> 1)]; }
    __device__ T& plane(int k, int r, int slot) const { return x[k * PL + r * Rg::HP + slot]; }
};

template <int TX, int TY, int HALO, int NT>
__device__ inline void pair_coords(int k, int i0, int j0, int& c, int& r, int& gi, int& gj, bool& valid) {
    using Rg = Region<TX, TY, HALO, NT>;
    const int P = threadIdx.x + k * NT;
    valid = P < Rg::NP;
    r = P / Rg::HP;
    c = 2 * (P - r * Rg::HP);
    gi = i0 - HALO + c;
    gj = j0 - HALO + r;
}

__device__ inline bool interior(int gi, int gj, int n) { return gi >= 1 && gi <= n - 1 && gj >= 1 && gj <= n - 1; }

// Half sweep S of NH (colour col) on the owned pairs: the colour-col node of each pair
// within distance ext = R + NH - 1 - S of the tile, clipped to the domain interior.
template <typename T, int TX, int TY, int HALO, int NT, int NH, int R, int S>
__device__ inline void half_sweep(const Planes<T, TX, TY, HALO, NT>& X, const PairVals<T, TX, TY, HALO, NT>& fa,
                                  const PairVals<T, TX, TY, HALO, NT>& fb, int i0, int j0, int n, int col) {
    using Rg = Region<TX, TY, HALO, NT>;
    constexpr int ext = R + NH - 1 - S;
    const int ia = max(1, i0 - ext), ib = min(n - 1, i0 + TX - 1 + ext);
    const int ja = max(1, j0 - ext), jb = min(n - 1, j0 + TY - 1 + ext);
#pragma unroll
    for (int k = 0; k < Rg::K; ++k) {
        int c, r, gi, gj;
        bool valid;
        pair_coords<TX, TY, HALO, NT>(k, i0, j0, c, r, gi, gj, valid);
        const int sel = ((gi + gj) & 1) ^ col;   // 0: the even-column node has colour col
        const int g = gi + sel;
        if (valid && g >= ia && g <= ib && gj >= ja && gj <= jb) {
            // node (c + sel, r) has colour col; its four neighbours have the other colour:
            // W, E in this row at slots pc - 1 + sel, pc + sel; S, N at slot pc of rows r -+ 1
            const int o = col ^ 1, pc = c >> 1;
            X.plane(col, r, pc) = gs2f<T>(X.k, sel ? fb[k] : fa[k], X.plane(o, r, pc - 1 + sel),
                                          X.plane(o, r, pc + sel), X.plane(o, r - 1, pc), X.plane(o, r + 1, pc));
        }
    }
    __syncthreads();
}

template <typename T, int TX, int TY, int HALO, int NT, int NH, int R, int... S>
__device__ inline void half_sweeps_seq(const Planes<T, TX, TY, HALO, NT>& X, const PairVals<T, TX, TY, HALO, NT>& fa,
                                       const PairVals<T, TX, TY, HALO, NT>& fb, int i0, int j0, int n,
                                       std::integer_sequence<int, S...>) {
    (half_sweep<T, TX, TY, HALO, NT, NH, R, S>(X, fa, fb, i0, j0, n, S & 1), ...);
}

// x and f of the owned pairs (zero outside the domain; x zero when zero_x).  Every load of
// the thread is issued before the first use.
template <typename T, int TX, int TY, int HALO, int NT>
__device__ inline void load_pairs(PairVals<T, TX, TY, HALO, NT>& xa, PairVals<T, TX, TY, HALO, NT>& xb,
                                  PairVals<T, TX, TY, HALO, NT>& fa, PairVals<T, TX, TY, HALO, NT>& fb,
                                  const T* __restrict__ x, const T* __restrict__ f, const Grid& g, int i0, int j0,
                                  int zero_x) {
    using Rg = Region<TX, TY, HALO, NT>;
    const int n = g.n;
#pragma unroll
    for (int k = 0; k < Rg::K; ++k) {
        int c, r, gi, gj;
        bool valid;
        pair_coords<TX, TY, HALO, NT>(k, i0, j0, c, r, gi, gj, valid);
        xa[k] = T(0); xb[k] = T(0); fa[k] = T(0); fb[k] = T(0);
        const bool row = valid && gj >= 0 && gj <= n;
        const int q = gi + (int)g.pitch * gj;   // level arrays hold < 2^31 elements
        if (row && gi >= 0 && gi <= n) {
            if (!zero_x) xa[k] = x[q];
            fa[k] = f[q];
        }
        if (row && gi + 1 >= 0 && gi + 1 <= n) {
            if (!zero_x) xb[k] = x[q + 1];
            fb[k] = f[q + 1];
        }
    }
}

// owned x into the LDS region
template <typename T, int TX, int TY, int HALO, int NT>
__device__ inline void put_pairs(const Planes<T, TX, TY, HALO, NT>& X, const PairVals<T, TX, TY, HALO, NT>& xa,
                                 const PairVals<T, TX, TY, HALO, NT>& xb, int i0, int j0) {
    using Rg = Region<TX, TY, HALO, NT>;
#pragma unroll
    for (int k = 0; k < Rg::K; ++k) {
        int c, r, gi, gj;
        bool valid;
        pair_coords<TX, TY, HALO, NT>(k, i0, j0, c, r, gi, gj, valid);
        if (valid) {
            X.at(c, r) = xa[k];
            X.at(c + 1, r) = xb[k];
        }
    }
}

// the tile nodes of the owned pairs, from the LDS region, to the level array
template <typename T, int TX, int TY, int HALO, int NT>
__device__ inline void store_pairs(T* __restrict__ out, const Planes<T, TX, TY, HALO, NT>& X, const Grid& g, int i0,
                                   int j0) {
    using Rg = Region<TX, TY, HALO, NT>;
    const int n = g.n;
#pragma unroll
    for (int k = 0; k < Rg::K; ++k) {
        int c, r, gi, gj;
        bool valid;
        pair_coords<TX, TY, HALO, NT>(k, i0, j0, c, r, gi, gj, valid);
        if (!valid || gj < j0 || gj > min(n - 1, j0 + TY - 1)) continue;
        const int q = gi + (int)g.pitch * gj;
        if (gi >= i0 && gi <= min(n - 1, i0 + TX - 1)) out[q] = X.at(c, r);
        if (gi + 1 >= i0 && gi + 1 <= min(n - 1, i0 + TX - 1)) out[q + 1] = X.at(c + 1, r);
    }
}

// pre-smoothing + residual + restriction
template <typename T, int NH, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_vpre2d(const T* __restrict__ x, T* __restrict__ y,
                                                    const T* __restrict__ f, T* __restrict__ rc, Grid g, Grid gc,
                                                    int zero_x) {
    constexpr int R = 2;                 // x must be final within 2 rings for the residual ring
    constexpr int HALO = NH + R;
    using Rg = Region<TX, TY, HALO, NT>;
    __shared__ T xs[2 * Rg::RH * Rg::HP];
    const int i0 = 1 + blockIdx.x * TX, j0 = 1 + blockIdx.y * TY;
    const int n = g.n;
    const Planes<T, TX, TY, HALO, NT> X{xs, (i0 + j0) & 1, stencil_of<T>(g)};
    T xa[Rg::K], xb[Rg::K], fa[Rg::K], fb[Rg::K];
    load_pairs<T, TX, TY, HALO, NT>(xa, xb, fa, fb, x, f, g, i0, j0, zero_x);
    put_pairs<T, TX, TY, HALO, NT>(X, xa, xb, i0, j0);
    __syncthreads();
    half_sweeps_seq<T, TX, TY, HALO, NT, NH, R>(X, fa, fb, i0, j0, n, std::make_integer_sequence<int, NH>{});
    store_pairs<T, TX, TY, HALO, NT>(y, X, g, i0, j0);
    // residual r = f - K x on the tile and one ring (kept in fa/fb; f elsewhere)
    const int ia = i0 - 1, ib = i0 + TX, ja = j0 - 1, jb = j0 + TY;
#pragma unroll
    for (int k = 0; k < Rg::K; ++k) {
        int c, r, gi, gj;
        bool valid;
        pair_coords<TX, TY, HALO, NT>(k, i0, j0, c, r, gi, gj, valid);
        if (!valid || gj < ja || gj > jb) continue;
        if (gi >= ia && gi <= ib && interior(gi, gj, n))
            fa[k] = kres2(X.k, fa[k], X.at(c, r), X.at(c - 1, r), X.at(c + 1, r), X.at(c, r - 1), X.at(c, r + 1));
        if (gi + 1 >= ia && gi + 1 <= ib && interior(gi + 1, gj, n))
            fb[k] = kres2(X.k, fb[k], X.at(c + 1, r), X.at(c, r), X.at(c + 2, r), X.at(c + 1, r - 1),
                          X.at(c + 1, r + 1));
    }
    __syncthreads();
    put_pairs<T, TX, TY, HALO, NT>(X, fa, fb, i0, j0);   // the residuals replace x in LDS
    __syncthreads();
    // restriction for the coarse nodes whose centre 2I, 2J lies in this tile
    {
        constexpr int CW = TX / 2, CH = TY / 2;
        const int nc = gc.n;
        for (int t = threadIdx.x; t < CW * CH; t += NT) {
            const int r = t / CW, c = t - r * CW;
            const int I = (i0 + 1) / 2 + c, J = (j0 + 1) / 2 + r;
            if (I > nc - 1 || J > nc - 1) continue;
            const int cc = 2 * I - i0 + HALO, rr = 2 * J - j0 + HALO;
            const T e = (X.at(cc - 1, rr) + X.at(cc + 1, rr)) + (X.at(cc, rr - 1) + X.at(cc, rr + 1)) +
                        (X.at(cc - 1, rr - 1) + X.at(cc + 1, rr + 1));
            rc[I + gc.pitch * J] = X.at(cc, rr) + T(0.5) * e;
        }
    }
}

// prolongation + correction + post-smoothing
template <typename T, int NH, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_vpost2d(const T* __restrict__ y, T* __restrict__ x,
                                                     const T* __restrict__ f, const T* __restrict__ xc, Grid g,
                                                     Grid gc) {
    constexpr int R = 0;
    constexpr int HALO = NH > 0 ? NH + R : 1;
    using Rg = Region<TX, TY, HALO, NT>;
    // coarse values under the region: coarse node (I, J) for I in [(i0 - HALO) >> 1, ...]
    constexpr int CRW = Rg::RW / 2 + 2, CRH = Rg::RH / 2 + 2;
    __shared__ T xs[2 * Rg::RH * Rg::HP];
    __shared__ T cs[CRW * CRH];
    const int i0 = 1 + blockIdx.x * TX, j0 = 1 + blockIdx.y * TY;
    const int n = g.n, nc = gc.n;
    const int I0 = (i0 - HALO) >> 1, J0 = (j0 - HALO) >> 1;
    T xa[Rg::K], xb[Rg::K], fa[Rg::K], fb[Rg::K];
    constexpr int KC = (CRW * CRH + NT - 1) / NT;
    T cv[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int t = threadIdx.x + k * NT;
        const int r = t / CRW, c = t - r * CRW;
        const int I = I0 + c, J = J0 + r;
        cv[k] = (t < CRW * CRH && I >= 0 && I <= nc && J >= 0 && J <= nc) ? xc[I + (int)gc.pitch * J] : T(0);
    }
    load_pairs<T, TX, TY, HALO, NT>(xa, xb, fa, fb, y, f, g, i0, j0, 0);
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int t = threadIdx.x + k * NT;
        if (t < CRW * CRH) cs[t] = cv[k];
    }
    __syncthreads();
    // x = y + P x_c on the interior nodes of the region (the expression of k_prolong)
#pragma unroll
    for (int k = 0; k < Rg::K; ++k) {
        int c, r, gi, gj;
        bool valid;
        pair_coords<TX, TY, HALO, NT>(k, i0, j0, c, r, gi, gj, valid);
        if (!valid) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int gg = gi + h;
            if (!interior(gg, gj, n)) continue;
            const int di = gg & 1, dj = gj & 1;
            const int q0 = ((gg >> 1) - I0) + CRW * ((gj >> 1) - J0);
            T v = cs[q0];
            if (di | dj) v = T(0.5) * (v + cs[q0 + di + CRW * dj]);
            if (h) xb[k] += v;
            else xa[k] += v;
        }
    }
    const Planes<T, TX, TY, HALO, NT> X{xs, (i0 + j0) & 1, stencil_of<T>(g)};
    put_pairs<T, TX, TY, HALO, NT>(X, xa, xb, i0, j0);
    __syncthreads();
    half_sweeps_seq<T, TX, TY, HALO, NT, NH, R>(X, fa, fb, i0, j0, n, std::make_integer_sequence<int, NH>{});
    store_pairs<T, TX, TY, HALO, NT>(x, X, g, i0, j0);
}

// Tile shape by level: 16 x 16 on coarse levels (more workgroups, short sweeps; the halo
// overhead is irrelevant there); on finer levels the tiles whose padded region is a whole
// number of 256-pair rounds: post (5 halo rings) 54 x 22 -> 64 x 32 region, 4 pairs per
// thread; pre (7 rings) 50 x 34 -> 64 x 48 region, 6 pairs per thread.  The level size
// from which the wide tiles are used, and the largest level of the one-workgroup bottom
// below, are run-time choices (set_vpass2d_tuning; the autotuner times them).
constexpr int kWideMinDefault = 256, kBottomMaxDefault = 32;
static int g_wide_min = kWideMinDefault;       // levels with n > this use the wide tiles
static int g_bottom_max = kBottomMaxDefault;   // bottom kernel for levels with n <= this (0: off)
#ifndef FMG_VC_PRE_TILE
#define FMG_VC_PRE_TILE 50, 34, 256
#define FMG_VC_POST_TILE 54, 22, 256
#endif

template <int TX, int TY, int NT>
struct Tile {
    static constexpr int tx = TX, ty = TY, nt = NT;
};
using PreWide = Tile<FMG_VC_PRE_TILE>;
using PostWide = Tile<FMG_VC_POST_TILE>;

template <typename T, int NH>
void pre_launch(const Grid& g, const Grid& gc, const T* x, T* y, const T* f, T* rc, int zero_x, hipStream_t s) {
    if (g.n <= g_wide_min) {
        dim3 grd(cdiv(g.n - 1, 16), cdiv(g.n - 1, 16));
        hipLaunchKernelGGL((k_vpre2d<T, NH, 16, 16, 256>), grd, dim3(256), 0, s, x, y, f, rc, g, gc, zero_x);
    } else {
        using W = PreWide;
        dim3 grd(cdiv(g.n - 1, W::tx), cdiv(g.n - 1, W::ty));
        hipLaunchKernelGGL((k_vpre2d<T, NH, W::tx, W::ty, W::nt>), grd, dim3(W::nt), 0, s, x, y, f, rc, g, gc, zero_x);
    }
}
template <typename T, int NH>
void post_launch(const Grid& g, const Grid& gc, const T* y, T* x, const T* f, const T* xc, hipStream_t s,
                 hipEvent_t ev0, hipEvent_t ev1) {
    if (g.n <= g_wide_min) {
        dim3 grd(cdiv(g.n - 1, 16), cdiv(g.n - 1, 16));
        hipExtLaunchKernelGGL((k_vpost2d<T, NH, 16, 16, 256>), grd, dim3(256), 0, s, ev0, ev1, 0, y, x, f, xc, g, gc);
    } else {
        using W = PostWide;
        dim3 grd(cdiv(g.n - 1, W::tx), cdiv(g.n - 1, W::ty));
        hipExtLaunchKernelGGL((k_vpost2d<T, NH, W::tx, W::ty, W::nt>), grd, dim3(W::nt), 0, s, ev0, ev1, 0, y, x, f,
                              xc, g, gc);
    }
}

// ---- the bottom of a V-cycle in one workgroup ------------------------------------------
// Levels l, l-1, ..., 0 of a V-cycle whose level-l mesh is small: every level's x and f
// stay in LDS for the whole cycle, so the 2 l + 1 launches of the level passes and of the
// coarsest solve become one.  Measured on the 2D n = 2048 solve, this pays for the level
// n = 32 only: from n = 64 on, one workgroup takes longer than the level passes spread over
// the chip.  The steps are those of the unfused kernel sequence of grid.hip
// (half sweeps R, B, R, ..., residual and P^T, exact coarsest solve, P x_c added, the post
// sweeps) with the same expression at every node, so the result has the same bits.
// Level q (mesh n_q = n_0 2^q) is a dense (n_q + 1)^2 array with its zero ring; the
// coarsest-solve scratch follows the level arrays.
#ifndef FMG_BOTTOM_THREADS
#define FMG_BOTTOM_THREADS 512
#endif
#ifndef FMG_BOTTOM_MAX_N
#define FMG_BOTTOM_MAX_N 64
#endif
constexpr int kBottomThreads = FMG_BOTTOM_THREADS;
constexpr int kBottomMaxN = FMG_BOTTOM_MAX_N;
constexpr int kBottomMaxLevels = 8;

template <typename T>
__host__ __device__ inline size_t bottom_level_elems(int n0, int l) {
    size_t e = 0;
    for (int q = 0; q <= l; ++q) {
        const size_t p = (size_t)(n0 << q) + 1;
        e += 2 * p * p;
    }
    return e;
}
// elements of the level arrays below level q (each level: x, then f)
__device__ inline int bottom_off(int n0, int q) {
    int e = 0;
    for (int r = 0; r < q; ++r) e += 2 * ((n0 << r) + 1) * ((n0 << r) + 1);
    return e;
}
template <typename T>
inline size_t bottom_bytes(int n0, int l) {
    const size_t m = (size_t)n0 - 1;
    const size_t lv = (bottom_level_elems<T>(n0, l) * sizeof(T) + 7) / 8 * 8;
    return lv + sizeof(double) * (m * m + m + 2 * m * m);
}

// nh alternating half sweeps, colour 0 first, of x <- (f + sum of the 4 neighbours) / 4
template <typename T>
__device__ inline void bottom_sweeps(const Stencil<T>& k, T* X, const T* F, int n, int nh) {
    const int P = n + 1, half = n / 2;
    for (int h = 0; h < nh; ++h) {
        const int c = h & 1;
        for (int t = threadIdx.x; t < (n - 1) * half; t += blockDim.x) {
            const int j = 1 + t / half, slot = t - (j - 1) * half;
            const int i = (((1 + j) & 1) == c ? 1 : 2) + 2 * slot;
            if (i > n - 1) continue;
            const int p = i + P * j;
            X[p] = gs2f<T>(k, F[p], X[p - 1], X[p + 1], X[p - P], X[p + P]);
        }
        __syncthreads();
    }
}

template <typename T>
__device__ inline T bottom_resid(const Stencil<T>& k, const T* X, const T* F, int p, int P) {
    return kres2(k, F[p], X[p], X[p - 1], X[p + 1], X[p - P], X[p + P]);
}

template <typename T>
__global__ __launch_bounds__(kBottomThreads) void k_vbottom2d(T* __restrict__ x, const T* __restrict__ f, Grid g,
                                                              int n0, int l, int nh_pre, int nh_post, int zero_x) {
    extern __shared__ double smem[];
    const Stencil<T> kst = stencil_of<T>(g);   // the coefficient is the same on every level
    // level arrays addressed as offsets from the LDS base (so every access stays an LDS access)
    T* const base = reinterpret_cast<T*>(smem);
    auto X = [&](int q) { return base + bottom_off(n0, q); };
    auto F = [&](int q) { return base + bottom_off(n0, q) + ((n0 << q) + 1) * ((n0 << q) + 1); };
    double* dsm = smem + (bottom_level_elems<T>(n0, l) * sizeof(T) + 7) / 8;
    // lower levels start at zero (their rings stay zero); level l from global memory
    for (int t = threadIdx.x; t < bottom_off(n0, l); t += blockDim.x) base[t] = T(0);
    const int n = n0 << l, P = n + 1;
    for (int t = threadIdx.x; t < P * P; t += blockDim.x) {
        const int i = t % P, j = t / P;
        const bool in = i >= 1 && i <= n - 1 && j >= 1 && j <= n - 1;
        X(l)[t] = (in && !zero_x) ? x[i + g.pitch * j] : T(0);
        F(l)[t] = in ? f[i + g.pitch * j] : T(0);
    }
    __syncthreads();
    // down: pre sweeps, then f_{q-1} = P^T (f_q - K x_q)
    for (int q = l; q >= 1; --q) {
        const int nq = n0 << q, Pq = nq + 1, nc = nq / 2, Pc = nc + 1;
        bottom_sweeps<T>(kst, X(q), F(q), nq, nh_pre);
        const T* Xq = X(q);
        const T* Fq = F(q);
        T* Fc = F(q - 1);
        for (int t = threadIdx.x; t < (nc - 1) * (nc - 1); t += blockDim.x) {
            const int I = 1 + t % (nc - 1), J = 1 + t / (nc - 1);
            const int p = 2 * I + Pq * 2 * J;
            T c = bottom_resid<T>(kst, Xq, Fq, p, Pq);
            T e = (bottom_resid<T>(kst, Xq, Fq, p - 1, Pq) + bottom_resid<T>(kst, Xq, Fq, p + 1, Pq)) +
                  (bottom_resid<T>(kst, Xq, Fq, p - Pq, Pq) + bottom_resid<T>(kst, Xq, Fq, p + Pq, Pq)) +
                  (bottom_resid<T>(kst, Xq, Fq, p - 1 - Pq, Pq) + bottom_resid<T>(kst, Xq, Fq, p + 1 + Pq, Pq));
            Fc[I + Pc * J] = c + T(0.5) * e;
        }
        __syncthreads();
    }
    coarse_dst_solve<T>(F(0), X(0), n0 + 1, 0, n0, 2, g.a, dsm);
    __syncthreads();
    // up: x_q += P x_{q-1}, then the post sweeps
    for (int q = 1; q <= l; ++q) {
        const int nq = n0 << q, Pq = nq + 1, Pc = nq / 2 + 1;
        const T* xc = X(q - 1);
        T* Xq = X(q);
        for (int t = threadIdx.x; t < (nq - 1) * (nq - 1); t += blockDim.x) {
            const int i = 1 + t % (nq - 1), j = 1 + t / (nq - 1);
            const int di = i & 1, dj = j & 1;
            const int q0 = (i >> 1) + Pc * (j >> 1);
            T v = xc[q0];
            if (di | dj) v = T(0.5) * (v + xc[q0 + di + Pc * dj]);
            Xq[i + Pq * j] += v;
        }
        __syncthreads();
        bottom_sweeps<T>(kst, Xq, F(q), nq, nh_post);
    }
    for (int t = threadIdx.x; t < (n - 1) * (n - 1); t += blockDim.x) {
        const int i = 1 + t % (n - 1), j = 1 + t / (n - 1);
        x[i + g.pitch * j] = X(l)[i + P * j];
    }
}

}  // namespace

bool vpass2d_wide_tiles(const Grid& g) { return g.n > g_wide_min; }

void set_vpass2d_tuning(int wide_min, int bottom_max) {
    g_wide_min = wide_min > 0 ? wide_min : kWideMinDefault;
    g_bottom_max = bottom_max > 0 ? std::min(bottom_max, kBottomMaxN) : (bottom_max < 0 ? 0 : kBottomMaxDefault);
}
void get_vpass2d_tuning(int* wide_min, int* bottom_max) {
    *wide_min = g_wide_min;
    *bottom_max = g_bottom_max > 0 ? g_bottom_max : -1;
}

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


template <typename T>
bool launch_vbottom2d(const Grid* levels, int l, T* x, const T* f, int nu_pre, int nu_post, int zero_x,
                      hipStream_t s) {
    const int n0 = levels[0].n;
    if (l < 1 || l >= kBottomMaxLevels || levels[l].n > std::min(kBottomMaxN, g_bottom_max) || levels[l].dim != 2 ||
        nu_pre > 2 || nu_post > 2)
        return false;
    const size_t bytes = bottom_bytes<T>(n0, l);
    if (bytes > 150 * 1024) return false;
    // once per instantiation (thread-safe static initialisation)
    static const bool attr = [] {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vbottom2d<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024) == hipSuccess)
            return true;
        (void)hipGetLastError();
        return false;
    }();
    if (!attr) return false;
    const int nh_pre = nu_pre > 0 ? 2 * nu_pre + 1 : 0, nh_post = nu_post > 0 ? 2 * nu_post + 1 : 0;
    hipLaunchKernelGGL(k_vbottom2d<T>, dim3(1), dim3(kBottomThreads), bytes, s, x, f, levels[l], n0, l, nh_pre,
                       nh_post, zero_x);
    return true;
}
template bool launch_vbottom2d<double>(const Grid*, int, double*, const double*, int, int, int, hipStream_t);
template bool launch_vbottom2d<float>(const Grid*, int, float*, const float*, int, int, int, hipStream_t);

}  // namespace fmg
