// Shared definitions of the HIP library: level layout, launch helpers, small math.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/fmgeig.h"
#include "tables.h"

namespace fmg {

int set_error(int code, const char* fmt, ...);

// One level of a nested uniform mesh of [0,1]^D in the padded layout: (n+1)^D nodes
// including the Dirichlet ring, x fastest, rows padded to `pitch` elements, the
// (n+1) rows of each z-plane contiguous.  Node (i,j,k) -> i + pitch*(j + (n+1)*k).
struct Grid {
    int dim;
    int n;            // cells per side
    int64_t pitch;    // elements per row
    int64_t plane;    // elements per z-plane: (n+1)*pitch
    int64_t elems;    // total elements
    double h;         // 1/n
    // Diagonal SPD coefficient A = diag(a) of a-hat (2.5).  On these meshes the stiffness
    // couples axis neighbours only: K = [diag; -a_d on +-e_d] (times h in 3D) with
    // diag = 2 sum a_d; inv_diag = 1 / diag.  A = I: a = 1, diag = 2 D.
    double a[3];
    double diag, inv_diag;
};

inline int64_t pitch_for(int n) { return ((int64_t)(n + 1) + 15) / 16 * 16; }

inline Grid make_grid(int dim, int n) {
    Grid g;
    g.dim = dim;
    g.n = n;
    g.pitch = pitch_for(n);
    g.plane = (int64_t)(n + 1) * g.pitch;
    g.elems = dim == 2 ? g.plane : g.plane * (n + 1);
    g.h = 1.0 / n;
    g.a[0] = g.a[1] = g.a[2] = 1.0;
    g.diag = 2.0 * dim;
    g.inv_diag = 1.0 / g.diag;
    return g;
}

// the same level with the diagonal coefficient a (a[d] > 0 for d < dim)
inline Grid with_diffusion(Grid g, const double* a) {
    g.diag = 0.0;
    for (int d = 0; d < 3; ++d) {
        g.a[d] = d < g.dim ? a[d] : 1.0;
        if (d < g.dim) g.diag += 2.0 * g.a[d];
    }
    g.inv_diag = 1.0 / g.diag;
    return g;
}

__host__ __device__ inline int64_t at2(const Grid& g, int i, int j) { return i + g.pitch * j; }
__host__ __device__ inline int64_t at3(const Grid& g, int i, int j, int k) {
    return i + g.pitch * j + g.plane * k;
}

// Problem parameters as the kernels see them.
struct Phys {
    double w[3];      // W = sum w[k] x_k^2 + wc
    double wc;
    double zeta;
    double a[3];      // diagonal of the coefficient A of a-hat (2.5)
};

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// The stiffness stencil of a level in the working precision.  Every kernel forms the
// weighted neighbour sums, the row K x and the residual through the helpers below, whose
// fused multiply-adds are written out, so that all implementations of a sweep or residual
// round alike and give the same bits (with A = I the products by 1 are exact and the sums
// are those of the unweighted stencil).
template <typename T>
struct Stencil {
    T ax, ay, az, dg, inv;   // a_x, a_y, a_z, diag = 2 sum a_d, 1 / diag
};
template <typename T>
__host__ __device__ inline Stencil<T> stencil_of(const Grid& g) {
    return {T(g.a[0]), T(g.a[1]), T(g.a[2]), T(g.diag), T(g.inv_diag)};
}
// a_x (w + e) + a_y (s + n) [+ a_z (b + t)]
template <typename T>
__device__ inline T nsum2(const Stencil<T>& k, T w, T e, T s, T n) {
    return fma(k.ay, s + n, k.ax * (w + e));
}
template <typename T>
__device__ inline T nsum3(const Stencil<T>& k, T w, T e, T s, T n, T b, T t) {
    return fma(k.az, b + t, fma(k.ay, s + n, k.ax * (w + e)));
}
// diag x - (neighbour sum): the row of K x (times h in 3D)
template <typename T>
__device__ inline T kdiff(const Stencil<T>& k, T x, T ns) {
    return fma(k.dg, x, -ns);
}
// f - K x at a node: 2D f - kdiff, 3D f - h kdiff
template <typename T>
__device__ inline T kres2(const Stencil<T>& k, T f, T x, T w, T e, T s, T n) {
    return f - kdiff(k, x, nsum2(k, w, e, s, n));
}
template <typename T>
__device__ inline T kres3(const Stencil<T>& k, T f, T h, T x, T w, T e, T s, T n, T b, T t) {
    return fma(-h, kdiff(k, x, nsum3(k, w, e, s, n, b, t)), f);
}
// Gauss-Seidel update of a node: (f + sum) / diag in 2D, (f / h + sum) / diag in 3D
template <typename T>
__device__ inline T gsu2(const Stencil<T>& k, T f, T w, T e, T s, T n) {
    return (f + nsum2(k, w, e, s, n)) * k.inv;
}
template <typename T>
__device__ inline T gsu3(const Stencil<T>& k, T f, T inv_h, T w, T e, T s, T n, T b, T t) {
    return fma(f, inv_h, nsum3(k, w, e, s, n, b, t)) * k.inv;
}

// Warp (wavefront = 64 lanes) reduction of doubles.
// ---- cross-lane sums without the LDS crossbar: DPP moves inside each row of 16 lanes,
// the gfx950 permlane swaps across rows.  Each step adds two values that every lane of
// the pair combines in the same order, so all lanes end with the same bits.
__device__ inline double dbl_from(unsigned lo, unsigned hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return dbl_from(lo, hi);
}
// v(row 2r) + v(row 2r+1) at the same position of the row (rows of 16 lanes)
__device__ inline double xsum16(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return dbl_from(lo[0], hi[0]) + dbl_from(lo[1], hi[1]);
}
// v(lane l mod 32) + v(32 + l mod 32)
__device__ inline double xsum32(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return dbl_from(lo[0], hi[0]) + dbl_from(lo[1], hi[1]);
}
// sum over the 64 lanes of a full wavefront (all lanes active)
__device__ inline double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_f64<0x141>(v);   // row_half_mirror: the other quad of each half row
    v += dpp_f64<0x140>(v);   // row_mirror: the other half of each row
    return xsum32(xsum16(v));
}

}  // namespace fmg

#define FMG_HIP_CHECK(expr)                                                               \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return ::fmg::set_error(FMG_EHIP, "%s: %s", #expr,          \
                                                      hipGetErrorString(e_));             \
    } while (0)
