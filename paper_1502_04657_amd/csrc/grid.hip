// Grid kernels of the multigrid hot path: red-black Gauss-Seidel smoothing, residual and
// restriction, prolongation, exact coarsest solve, the right-hand side of the auxiliary
// problem (3.4), mixed-precision refinement helpers and the Rayleigh-quotient reductions.
//
// Operators (P1 elements, (2.3)-(2.5); mesh families of the paper's regular refinement):
//   2D  K = [4; -1 on E,W,N,S]                 (h-independent)
//   3D  K = h [6; -1 on +-x,+-y,+-z]
// Both are 2-colourable by the parity of i+j(+k), so a red-black half sweep updates all
// nodes of one colour at once and equals a Gauss-Seidel pass in red-black order.
// P is P1 interpolation: a fine node at a coarse node takes its value; any other fine node
// is the midpoint of one coarse edge (2D: x, y or (1,1) direction; 3D: the 7 Kuhn edge
// directions, which are exactly the nonzero parity patterns (i&1, j&1, k&1)).
#include <hip/hip_ext.h>

#include <cstddef>
#include <utility>

#include "dst.h"
#include "kernels.h"

namespace fmg {

// ------------------------------------------------------------------------------------------
// elementwise helpers
template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t count, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

template <typename T>
void launch_fill(T* p, int64_t count, T v, hipStream_t s) {
    if (count <= 0) return;
    unsigned blocks = (unsigned)std::min<int64_t>(cdiv(count, 256), 8192);
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, s, p, count, v);
}
template void launch_fill<double>(double*, int64_t, double, hipStream_t);
template void launch_fill<float>(float*, int64_t, float, hipStream_t);

// every 32-bit word of the state zero except the two of tol_lambda, which take its bits
__global__ void k_init_state(SmallState* st, double tol) {
    uint32_t* w = reinterpret_cast<uint32_t*>(st);
    constexpr int nw = (int)(sizeof(SmallState) / 4), t0 = (int)(offsetof(SmallState, tol_lambda) / 4);
    const unsigned long long b = (unsigned long long)__double_as_longlong(tol);
    for (int i = threadIdx.x; i < nw; i += blockDim.x)
        w[i] = i == t0 ? (uint32_t)b : (i == t0 + 1 ? (uint32_t)(b >> 32) : 0u);
}
void launch_init_state(SmallState* st, double tol_lambda, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(256), 0, s, st, tol_lambda);
}

__device__ inline int64_t compact_to_level(const Grid& g, int64_t c) {
    const int64_t m = g.n - 1;
    int64_t i = c % m + 1, r = c / m;
    if (g.dim == 2) return i + g.pitch * (r + 1);
    int64_t j = r % m + 1, k = r / m + 1;
    return i + g.pitch * j + g.plane * k;
}

__global__ void k_pack(Grid g, const double* __restrict__ c, double* __restrict__ lv, int64_t total) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total) lv[compact_to_level(g, t)] = c[t];
}
__global__ void k_unpack(Grid g, const double* __restrict__ lv, double* __restrict__ c, int64_t total) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total) c[t] = lv[compact_to_level(g, t)];
}

static int64_t interior_count(const Grid& g) {
    int64_t m = g.n - 1;
    return g.dim == 2 ? m * m : m * m * m;
}

void launch_pack(const Grid& g, const double* compact, double* level, hipStream_t s) {
    int64_t tot = interior_count(g);
    if (tot > 0) hipLaunchKernelGGL(k_pack, dim3(cdiv(tot, 256)), dim3(256), 0, s, g, compact, level, tot);
}
void launch_unpack(const Grid& g, const double* level, double* compact, hipStream_t s) {
    int64_t tot = interior_count(g);
    if (tot > 0) hipLaunchKernelGGL(k_unpack, dim3(cdiv(tot, 256)), dim3(256), 0, s, g, level, compact, tot);
}

// ------------------------------------------------------------------------------------------
// red-black Gauss-Seidel half sweep.  Thread (t, j[, k]) updates the t-th node of colour
// `color` ((i+j+k) % 2 == color) in row j.  The update expression is fixed so that every
// implementation of the sweep produces identical bits.
template <typename T>
__device__ inline T gs2(const Stencil<T>& k, T f, T w, T e, T s, T n) {
    return gsu2(k, f, w, e, s, n);
}
template <typename T>
__device__ inline T gs3(const Stencil<T>& k, T f, T inv_h, T w, T e, T s, T n, T b, T t) {
    return gsu3(k, f, inv_h, w, e, s, n, b, t);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_smooth_half(T* __restrict__ x, const T* __restrict__ f, Grid g,
                                                     int color) {
    const int n = g.n;
    const int j = 1 + blockIdx.y * 4 + threadIdx.y;
    const int k = (D == 3) ? 1 + (int)blockIdx.z : 0;
    if (j > n - 1) return;
    const int i0 = (((1 + j + k) & 1) == color) ? 1 : 2;
    const int i = i0 + 2 * (int)(blockIdx.x * 64 + threadIdx.x);
    if (i > n - 1) return;
    const int64_t P = g.pitch;
    if (D == 2) {
        const int64_t p = i + P * j;
        x[p] = gs2<T>(stencil_of<T>(g), f[p], x[p - 1], x[p + 1], x[p - P], x[p + P]);
    } else {
        const int64_t S = g.plane;
        const int64_t p = i + P * j + S * k;
        x[p] = gs3<T>(stencil_of<T>(g), f[p], T(n), x[p - 1], x[p + 1], x[p - P], x[p + P], x[p - S], x[p + S]);
    }
}

template <typename T>
void launch_smooth_half(const Grid& g, T* x, const T* f, int color, hipStream_t s) {
    const int n = g.n;
    if (n < 2) return;
    dim3 blk(64, 4, 1);
    dim3 grd(cdiv(n / 2 + 1, 64), cdiv(n - 1, 4), g.dim == 3 ? n - 1 : 1);
    if (g.dim == 2)
        hipLaunchKernelGGL((k_smooth_half<2, T>), grd, blk, 0, s, x, f, g, color);
    else
        hipLaunchKernelGGL((k_smooth_half<3, T>), grd, blk, 0, s, x, f, g, color);
}

template <typename T>
void launch_smooth(const Grid& g, T* x, const T* f, int half_sweeps, int first, hipStream_t s) {
    int c = first;
    for (int h = 0; h < half_sweeps; ++h, c ^= 1) launch_smooth_half<T>(g, x, f, c, s);
}
template void launch_smooth_half<double>(const Grid&, double*, const double*, int, hipStream_t);
template void launch_smooth_half<float>(const Grid&, float*, const float*, int, hipStream_t);
template void launch_smooth<double>(const Grid&, double*, const double*, int, int, hipStream_t);
template void launch_smooth<float>(const Grid&, float*, const float*, int, int, hipStream_t);

// ------------------------------------------------------------------------------------------
// residual r = f - K x on the fine level, restricted by P^T to the coarse level:
//   r_c(I) = r(2I) + 1/2 sum over the P1 edge neighbours d of r(2I +- d).
template <int D, typename T>
__device__ inline T resid_at(const Stencil<T>& k, const T* __restrict__ x, const T* __restrict__ f, int64_t q,
                             int64_t P, int64_t S, T h) {
    if (D == 2) return kres2(k, f[q], x[q], x[q - 1], x[q + 1], x[q - P], x[q + P]);
    return kres3(k, f[q], h, x[q], x[q - 1], x[q + 1], x[q - P], x[q + P], x[q - S], x[q + S]);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_resid_restrict(const T* __restrict__ x, const T* __restrict__ f,
                                                        T* __restrict__ rc, Grid gf, Grid gc) {
    const int I = 1 + blockIdx.x * 64 + threadIdx.x;
    const int J = 1 + blockIdx.y * 4 + threadIdx.y;
    const int Kz = (D == 3) ? 1 + (int)blockIdx.z : 0;
    const int nc = gc.n;
    if (I > nc - 1 || J > nc - 1) return;
    const int64_t P = gf.pitch, S = gf.plane;
    const T h = T(gf.h);
    const Stencil<T> kst = stencil_of<T>(gf);
    if (D == 2) {
        const int64_t p = 2 * I + P * 2 * J;
        T c = resid_at<2, T>(kst, x, f, p, P, S, h);
        T e = (resid_at<2, T>(kst, x, f, p - 1, P, S, h) + resid_at<2, T>(kst, x, f, p + 1, P, S, h)) +
              (resid_at<2, T>(kst, x, f, p - P, P, S, h) + resid_at<2, T>(kst, x, f, p + P, P, S, h)) +
              (resid_at<2, T>(kst, x, f, p - 1 - P, P, S, h) + resid_at<2, T>(kst, x, f, p + 1 + P, P, S, h));
        rc[I + gc.pitch * J] = c + T(0.5) * e;
    } else {
        const int64_t p = 2 * I + P * 2 * J + S * 2 * Kz;
        const int64_t d[7] = {1, P, S, 1 + P, P + S, 1 + S, 1 + P + S};
        T c = resid_at<3, T>(kst, x, f, p, P, S, h);
        T e = T(0);
#pragma unroll
        for (int q = 0; q < 7; ++q)
            e += resid_at<3, T>(kst, x, f, p - d[q], P, S, h) + resid_at<3, T>(kst, x, f, p + d[q], P, S, h);
        rc[I + gc.pitch * J + gc.plane * Kz] = c + T(0.5) * e;
    }
}

template <typename T>
void launch_resid_restrict(const Grid& gf, const Grid& gc, const T* x, const T* f, T* rc, hipStream_t s) {
    const int nc = gc.n;
    if (nc < 2) return;
    dim3 blk(64, 4, 1);
    dim3 grd(cdiv(nc - 1, 64), cdiv(nc - 1, 4), gf.dim == 3 ? nc - 1 : 1);
    if (gf.dim == 2)
        hipLaunchKernelGGL((k_resid_restrict<2, T>), grd, blk, 0, s, x, f, rc, gf, gc);
    else
        hipLaunchKernelGGL((k_resid_restrict<3, T>), grd, blk, 0, s, x, f, rc, gf, gc);
}
template void launch_resid_restrict<double>(const Grid&, const Grid&, const double*, const double*, double*,
                                            hipStream_t);
template void launch_resid_restrict<float>(const Grid&, const Grid&, const float*, const float*, float*,
                                           hipStream_t);

// ------------------------------------------------------------------------------------------
// prolongation x_f (+)= P x_c
template <int D, typename T>
__global__ __launch_bounds__(256) void k_prolong(const T* __restrict__ xc, T* __restrict__ xf, Grid gc, Grid gf,
                                                 int accumulate) {
    const int i = 1 + blockIdx.x * 64 + threadIdx.x;
    const int j = 1 + blockIdx.y * 4 + threadIdx.y;
    const int k = (D == 3) ? 1 + (int)blockIdx.z : 0;
    const int n = gf.n;
    if (i > n - 1 || j > n - 1) return;
    const int di = i & 1, dj = j & 1, dk = k & 1;
    const int64_t q0 = (i >> 1) + gc.pitch * (j >> 1) + gc.plane * (k >> 1);
    T v = xc[q0];
    if (di | dj | dk) v = T(0.5) * (v + xc[q0 + di + gc.pitch * dj + gc.plane * dk]);
    const int64_t p = i + gf.pitch * j + gf.plane * k;
    if (accumulate)
        xf[p] += v;
    else
        xf[p] = v;
}

template <typename T>
void launch_prolong(const Grid& gc, const Grid& gf, const T* xc, T* xf, int accumulate, hipStream_t s) {
    const int n = gf.n;
    dim3 blk(64, 4, 1);
    dim3 grd(cdiv(n - 1, 64), cdiv(n - 1, 4), gf.dim == 3 ? n - 1 : 1);
    if (gf.dim == 2)
        hipLaunchKernelGGL((k_prolong<2, T>), grd, blk, 0, s, xc, xf, gc, gf, accumulate);
    else
        hipLaunchKernelGGL((k_prolong<3, T>), grd, blk, 0, s, xc, xf, gc, gf, accumulate);
}
template void launch_prolong<double>(const Grid&, const Grid&, const double*, double*, int, hipStream_t);
template void launch_prolong<float>(const Grid&, const Grid&, const float*, float*, int, hipStream_t);

// ------------------------------------------------------------------------------------------
// Exact coarsest-level solve by the discrete sine transform (dst.h), one workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(const T* __restrict__ f, T* __restrict__ x, Grid g) {
    extern __shared__ double sm[];
    coarse_dst_solve<T>(f, x, g.pitch, g.plane, g.n, g.dim, g.a, sm);
}

template <typename T>
void launch_coarse_solve(const Grid& g, const T* f, T* x, hipStream_t s) {
    const int m = g.n - 1;
    const int total = g.dim == 2 ? m * m : m * m * m;
    size_t shm = sizeof(double) * ((size_t)m * m + m + 2 * (size_t)total);
    hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(256), shm, s, f, x, g);
}
template void launch_coarse_solve<double>(const Grid&, const double*, double*, hipStream_t);
template void launch_coarse_solve<float>(const Grid&, const float*, float*, hipStream_t);

// ------------------------------------------------------------------------------------------
// Right-hand side of the auxiliary problem (3.4): b = lambda M u - M_W u - zeta N(u).
// M and M_W rows come from the exact star moments (tables.h): with the node at X,
//   (M_W)_{i,i+o} = h^D [ sum_k w_k (X_k^2 m0[o] + 2 X_k h m1[k][o] + h^2 m2[k][o]) + wc m0[o] ].
// N(u)_i = int u_h^3 phi_i sums, over the elements e around node i, the exact value
//   |e| D! 3! / (D+4)! (h_3 + u_i h_2 + u_i^2 h_1 + u_i^3),
// h_k the complete homogeneous symmetric polynomials of the vertex values of e.

// interior node t (lexicographic, i fastest) -> (i, j, k); t < (n - 1)^D < 2^32 for every
// admissible mesh, so 32-bit division (64-bit division is a long software sequence)
__device__ inline void interior_ijk(int n, int D, int64_t t, int& i, int& j, int& k) {
    const unsigned m = (unsigned)(n - 1), tt = (unsigned)t;
    const unsigned r = tt / m, kk = (D == 3) ? r / m : 0u;
    i = (int)(tt - r * m) + 1;
    j = (int)(r - kk * m) + 1;
    k = (D == 3) ? (int)kk + 1 : 0;
}

// The per-node terms (M u)_i, (M_W u)_i, (N(u) u)_i and (K u)_i of a 2D level array (the 3D
// terms come from row segments: rhs3_node).
template <int D>
__device__ inline void node_forms(const double* __restrict__ u, const Grid& g, const Phys& ph, int i, int j, int k,
                                  double& Mu, double& MWu, double& Nu, double& Ku) {
    static_assert(D == 2, "3D levels use the row kernels");
    const int64_t P = g.pitch, S = g.plane;
    const int64_t p = i + P * j + S * k;
    const double h = g.h;
    const double X[3] = {i * h, j * h, k * h};
    constexpr int NS = (D == 2) ? kStencil2D : kStencil3D;
    // (M_W u)_i = sum_o (sum_a w_a (X_a^2 m0_o + 2 X_a h M1_ao + h^2 M2_ao) + wc m0_o) u_o:
    // the stencil sums of u against the constant tables m0, M1_a, M2_a first, then the
    // position-dependent weights once per node
    double mu = 0.0, s1[3] = {0.0, 0.0, 0.0}, s2[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int o = 0; o < NS; ++o) {
        const int64_t q = (D == 2) ? p + kOff2D[o][0] + P * kOff2D[o][1]
                                   : p + kOff3D[o][0] + P * kOff3D[o][1] + S * kOff3D[o][2];
        const double uq = u[q];
        mu += ((D == 2) ? kM0_2D[o] : kM0_3D[o]) * uq;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            s1[a] += ((D == 2) ? kM1_2D[a][o] : kM1_3D[a][o]) * uq;
            s2[a] += ((D == 2) ? kM2_2D[a][o] : kM2_3D[a][o]) * uq;
        }
    }
    double mw = ph.wc * mu;
#pragma unroll
    for (int a = 0; a < D; ++a) mw += ph.w[a] * (X[a] * X[a] * mu + 2.0 * X[a] * h * s1[a] + h * h * s2[a]);
    const double hd = (D == 2) ? h * h : h * h * h;
    Mu = hd * mu;
    MWu = hd * mw;
    const double u0 = u[p];
    double nl = 0.0;
    if (D == 2) {
        // the element term of (u0, a, b) expanded in u0: 4 u0^3 + 3 u0^2 (a + b) + 2 u0 (a^2 + ab + b^2)
        // + (a^3 + a^2 b + a b^2 + b^3); with s = a + b, q = ab the last two are s^2 - q and
        // s (s^2 - 2q), summed over the star before the powers of u0 are applied
        double t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
        for (int e = 0; e < kStarElems2D; ++e) {
            const double a = u[p + kStarElem2D[e][0][0] + P * kStarElem2D[e][0][1]];
            const double b = u[p + kStarElem2D[e][1][0] + P * kStarElem2D[e][1][1]];
            const double sab = a + b, q = a * b, s2 = sab * sab;
            t1 += sab;
            t2 += s2 - q;
            t3 += sab * (s2 - 2.0 * q);
        }
        nl = u0 * (u0 * (4.0 * kStarElems2D * u0 + 3.0 * t1) + 2.0 * t2) + t3;
        Nu = nl * (h * h / 120.0);
        const Stencil<double> ks = stencil_of<double>(g);
        Ku = kdiff(ks, u0, nsum2(ks, u[p - 1], u[p + 1], u[p - P], u[p + P]));
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_rhs(const double* __restrict__ u, double* __restrict__ b, Grid g, Phys ph,
                                             const double* __restrict__ lam_dev, double lam_host) {
    const int i = 1 + blockIdx.x * 64 + threadIdx.x;
    const int j = 1 + blockIdx.y * 4 + threadIdx.y;
    const int k = (D == 3) ? 1 + (int)blockIdx.z : 0;
    const int n = g.n;
    if (i > n - 1 || j > n - 1) return;
    const double lam = lam_dev ? *lam_dev : lam_host;
    double Mu, MWu, Nu, Ku;
    node_forms<D>(u, g, ph, i, j, k, Mu, MWu, Nu, Ku);
    b[i + g.pitch * j + g.plane * k] = lam * Mu - MWu - ph.zeta * Nu;
}

// The 3D right-hand side with kRhsNX consecutive nodes along x per thread.  The 15-point
// star of a node spans seven grid rows (dy, dz); a thread loads the segments of those rows
// covering its nodes and their x-neighbours once (7 (kRhsNX + 2) values instead of 15 per
// node) and evaluates each node from registers (rhs3_node): the mass moments over the sums
// and differences of opposite neighbours, the nonlinear term from the star's vertices,
// edges and triangles.
constexpr int kRhsNX = 4;
static constexpr int kRhsRows3D[7][2] = {{0, 0}, {-1, 0}, {0, -1}, {1, 0}, {0, 1}, {-1, -1}, {1, 1}};
__host__ __device__ constexpr int rhs_row3(int dy, int dz) {
    for (int r = 0; r < 7; ++r)
        if (kRhsRows3D[r][0] == dy && kRhsRows3D[r][1] == dz) return r;
    return -1;
}
__host__ __device__ constexpr int star_slot3(int dx, int dy, int dz) {
    for (int s = 0; s < kStencil3D; ++s)
        if (kOff3D[s][0] == dx && kOff3D[s][1] == dy && kOff3D[s][2] == dz) return s;
    return -1;
}
template <typename F, int... I>
__device__ __forceinline__ void rhs_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void rhs_for(F&& f) {
    rhs_for_impl(f, std::make_integer_sequence<int, N>{});
}
static_assert(rhs_row3(0, 0) == 0, "row table");

// The star of a node as a surface: its 14 outer vertices (stencil slots 1..14), each in
// deg[s] of the 24 tetrahedra, the 36 edges (ea, eb) between them, each shared by em
// tetrahedra, and the 24 triangles (edge tri_e, third vertex tri_c).  Summed over the star,
// the complete homogeneous sums of a tetrahedron's outer vertex values (a, b, c) are
//   sum h1 = sum_s deg_s u_s,   sum h2 = sum_s deg_s u_s^2 + sum_e em_e u_a u_b,
//   sum h3 = sum_s deg_s u_s^3 + sum_e em_e u_a u_b (u_a + u_b) + sum_t u_a u_b u_c.
struct StarLinks3 {
    int ne = 0;
    int ea[48] = {}, eb[48] = {}, em[48] = {};
    int deg[kStencil3D] = {};
    int tri_e[kStarElems3D] = {}, tri_c[kStarElems3D] = {};
};
__host__ __device__ constexpr StarLinks3 make_star_links3() {
    StarLinks3 L{};
    for (int e = 0; e < kStarElems3D; ++e) {
        int v[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k) v[k] = star_slot3(kStarElem3D[e][k][0], kStarElem3D[e][k][1], kStarElem3D[e][k][2]);
        for (int k = 0; k < 3; ++k) L.deg[v[k]] += 1;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const int a = v[p] < v[q] ? v[p] : v[q], b = v[p] < v[q] ? v[q] : v[p];
                int f = -1;
                for (int x = 0; x < L.ne; ++x)
                    if (L.ea[x] == a && L.eb[x] == b) f = x;
                if (f < 0) {
                    f = L.ne++;
                    L.ea[f] = a;
                    L.eb[f] = b;
                }
                L.em[f] += 1;
                if (p == 0 && q == 1) L.tri_e[e] = f;
            }
        L.tri_c[e] = v[2];
    }
    return L;
}
static constexpr StarLinks3 kStarLinks3 = make_star_links3();
static_assert(kStarLinks3.ne == 36 && kStarLinks3.deg[0] == 0, "star of a Kuhn vertex: 36 outer edges");

// the stencil slot of the offset opposite to slot s (the star is centrally symmetric)
__host__ __device__ constexpr int opposite3(int s) { return star_slot3(-kOff3D[s][0], -kOff3D[s][1], -kOff3D[s][2]); }
// the pairs (p, opposite) with p the member whose first nonzero offset is negative
__host__ __device__ constexpr bool neg_member3(int s) {
    return kOff3D[s][0] != 0 ? kOff3D[s][0] < 0 : (kOff3D[s][1] != 0 ? kOff3D[s][1] < 0 : kOff3D[s][2] < 0);
}
__host__ __device__ constexpr bool mass_moments_symmetric3() {
    for (int s = 1; s < kStencil3D; ++s) {
        const int t = opposite3(s);
        if (t < 0 || kM0_3D[s] != kM0_3D[t]) return false;
        for (int a = 0; a < 3; ++a)
            if (kM2_3D[a][s] != kM2_3D[a][t] || kM1_3D[a][s] != -kM1_3D[a][t]) return false;
    }
    return true;
}
static_assert(mass_moments_symmetric3(), "m0, M2 even and M1 odd under the point reflection of the star");

// Rows of the 3D right-hand-side and forms passes: seg[r][c] is row r (offsets
// kRhsRows3D[r]) at x = i0 - 1 + c, clamped to the boundary node n (values past it are
// loaded but belong to no node of the thread).
template <int NX>
__device__ __forceinline__ void rhs3_rows_load(const double* __restrict__ u, const Grid& g, int i0, int j, int k,
                                               double (&seg)[7][NX + 2]) {
    const int n = g.n;
    const int64_t P = g.pitch, S = g.plane;
    rhs_for<7>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const double* row = u + P * (j + kRhsRows3D[r][0]) + S * (k + kRhsRows3D[r][1]);
        rhs_for<NX + 2>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            seg[r][c] = row[min(i0 - 1 + c, n)];
        });
    });
}

// (M u)_i, (M_W u)_i and (N(u) u)_i of node i = i0 + q (position X) from the rows
template <int NX, int q>
__device__ __forceinline__ void rhs3_node(const double (&seg)[7][NX + 2], const Phys& ph, double h, double hd,
                                          const double (&X)[3], double& Mu, double& MWu, double& Nu) {
    // value at stencil offset (dx, dy, dz) of node i0 + q
    auto U = [&](auto sc) -> double {
        constexpr int s = decltype(sc)::value;
        return seg[rhs_row3(kOff3D[s][1], kOff3D[s][2])][q + 1 + kOff3D[s][0]];
    };
    const double u0 = U(std::integral_constant<int, 0>{});
    // the stencil sums of u against m0 and M2 (even) over the sums of opposite values,
    // against M1 (odd) over their differences
    double mu = kM0_3D[0] * u0, s1[3] = {0.0, 0.0, 0.0}, s2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) s2[a] = kM2_3D[a][0] * u0;
    rhs_for<kStencil3D>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        if constexpr (p > 0 && neg_member3(p)) {
            constexpr int t = opposite3(p);
            const double up = U(pc), ut = U(std::integral_constant<int, t>{});
            const double sp = up + ut, dp = ut - up;
            mu += kM0_3D[p] * sp;
            rhs_for<3>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                if constexpr (kM1_3D[a][t] != 0.0) s1[a] += kM1_3D[a][t] * dp;
                s2[a] += kM2_3D[a][p] * sp;
            });
        }
    });
    double mw = ph.wc * mu;
#pragma unroll
    for (int a = 0; a < 3; ++a) mw += ph.w[a] * (X[a] * X[a] * mu + 2.0 * X[a] * h * s1[a] + h * h * s2[a]);
    Mu = hd * mu;
    MWu = hd * mw;
    // sums over the star of the complete homogeneous polynomials h1, h2, h3 of each
    // tetrahedron's outer vertex values, from its vertices, edges and triangles
    double t1 = 0.0, t2 = 0.0, t3 = 0.0;
    rhs_for<kStencil3D>([&](auto sc) {
        constexpr int sl = decltype(sc)::value;
        if constexpr (kStarLinks3.deg[sl] > 0) {
            constexpr double dg = kStarLinks3.deg[sl];
            const double us = U(sc), u2 = us * us;
            t1 += dg * us;
            t2 += dg * u2;
            t3 += dg * (u2 * us);
        }
    });
    // every outer edge lies in two tetrahedra (the star's boundary is a closed surface)
    double ep[kStarLinks3.ne], e2 = 0.0, e3 = 0.0;
    rhs_for<kStarLinks3.ne>([&](auto ec) {
        constexpr int x = decltype(ec)::value;
        static_assert(kStarLinks3.em[x] == 2, "edge multiplicity");
        const double ua = U(std::integral_constant<int, kStarLinks3.ea[x]>{});
        const double ub = U(std::integral_constant<int, kStarLinks3.eb[x]>{});
        ep[x] = ua * ub;
        e2 += ep[x];
        e3 += ep[x] * (ua + ub);
    });
    t2 += 2.0 * e2;
    t3 += 2.0 * e3;
    rhs_for<kStarElems3D>([&](auto tc) {
        constexpr int e = decltype(tc)::value;
        t3 += ep[kStarLinks3.tri_e[e]] * U(std::integral_constant<int, kStarLinks3.tri_c[e]>{});
    });
    const double nl = t3 + u0 * (2.0 * t2 + u0 * (3.0 * t1 + (4.0 * kStarElems3D) * u0));
    Nu = nl * (h * h * h / 840.0);
}

__global__ __launch_bounds__(256) void k_rhs3_rows(const double* __restrict__ u, double* __restrict__ b, Grid g,
                                                   Phys ph, const double* __restrict__ lam_dev, double lam_host) {
    constexpr int NX = kRhsNX;
    const int i0 = 1 + (int)(blockIdx.x * 64 + threadIdx.x) * NX;
    const int j = 1 + (int)blockIdx.y * 4 + (int)threadIdx.y;
    const int k = 1 + (int)blockIdx.z;
    const int n = g.n;
    if (i0 > n - 1 || j > n - 1) return;
    const double lam = lam_dev ? *lam_dev : lam_host;
    const int64_t P = g.pitch, S = g.plane;
    double seg[7][NX + 2];
    rhs3_rows_load<NX>(u, g, i0, j, k, seg);
    const double h = g.h;
    const double hd = h * h * h;
    const double X1 = j * h, X2 = k * h;
    rhs_for<NX>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if (i0 + q > n - 1) return;
        const double X[3] = {(i0 + q) * h, X1, X2};
        double Mu, MWu, Nu;
        rhs3_node<NX, q>(seg, ph, h, hd, X, Mu, MWu, Nu);
        b[(i0 + q) + P * j + S * k] = lam * Mu - MWu - ph.zeta * Nu;
    });
}

// The forms of a 3D level array from the same rows: u.Ku, u.M_W u, u.Mu, u.N(u)u and, with
// lam, |Ku + M_W u + zeta N(u)u - lam Mu|^2 and |lam Mu|^2, per workgroup into partial.
// kReduceBlocks workgroups (64 x 4 threads; two per CU at this kernel's register count)
// stride over the row groups of the rhs grid.
template <int NQ>
__global__ __launch_bounds__(256) void k_forms3_rows(const double* __restrict__ u, Grid g, Phys ph,
                                                     const double* __restrict__ lam, double* __restrict__ partial) {
    constexpr int NX = kRhsNX;
    const int n = g.n, m = n - 1;
    const int gx = (m + 64 * NX - 1) / (64 * NX), gy = (m + 3) / 4;
    const int groups = gx * gy * m;
    const double lv = (NQ > 4) ? *lam : 0.0;
    const double h = g.h;
    const double hd = h * h * h;
    const Stencil<double> ks = stencil_of<double>(g);
    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = 0.0;
    for (int grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        const int bx = grp % gx, rest = grp / gx, by = rest % gy, bz = rest / gy;
        const int i0 = 1 + (bx * 64 + (int)threadIdx.x) * NX;
        const int j = 1 + by * 4 + (int)threadIdx.y;
        const int k = 1 + bz;
        if (i0 > n - 1 || j > n - 1) continue;
        double seg[7][NX + 2];
        rhs3_rows_load<NX>(u, g, i0, j, k, seg);
        const double X1 = j * h, X2 = k * h;
        rhs_for<NX>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if (i0 + q > n - 1) return;
            const double X[3] = {(i0 + q) * h, X1, X2};
            double Mu, MWu, Nu;
            rhs3_node<NX, q>(seg, ph, h, hd, X, Mu, MWu, Nu);
            // the stiffness couples the axis neighbours only
            constexpr int r0 = rhs_row3(0, 0), ym = rhs_row3(-1, 0), yp = rhs_row3(1, 0), zm = rhs_row3(0, -1),
                          zp = rhs_row3(0, 1);
            const double u0 = seg[r0][q + 1];
            const double Ku = h * kdiff(ks, u0, nsum3(ks, seg[r0][q], seg[r0][q + 2], seg[ym][q + 1], seg[yp][q + 1],
                                                      seg[zm][q + 1], seg[zp][q + 1]));
            a[0] += u0 * Ku;
            a[1] += u0 * MWu;
            a[2] += u0 * Mu;
            a[3] += u0 * Nu;
            if constexpr (NQ > 4) {
                const double lm = lv * Mu, r = (Ku + MWu + ph.zeta * Nu) - lm;
                a[4] += r * r;
                a[5] += lm * lm;
            }
        });
    }
    // blockDim (64, 4): wavefront threadIdx.y, lane threadIdx.x
    __shared__ double red[4][NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double v = wave_sum(a[q]);
        if (threadIdx.x == 0) red[threadIdx.y][q] = v;
    }
    __syncthreads();
    const int t = (int)threadIdx.x + 64 * (int)threadIdx.y;
    if (t < NQ) {
        double v = 0.0;
        for (int w = 0; w < 4; ++w) v += red[w][t];
        partial[blockIdx.x * NQ + t] = v;
    }
}

void launch_rhs(const Grid& g, const Phys& ph, const double* u, double* b, const double* lam_dev, double lam_host,
                hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const int n = g.n;
    dim3 blk(64, 4, 1);
    if (g.dim == 2) {
        dim3 grd(cdiv(n - 1, 64), cdiv(n - 1, 4), 1);
        hipExtLaunchKernelGGL(k_rhs<2>, grd, blk, 0, s, ev0, ev1, 0, u, b, g, ph, lam_dev, lam_host);
    } else {
        dim3 grd(cdiv(n - 1, 64 * kRhsNX), cdiv(n - 1, 4), n - 1);
        hipExtLaunchKernelGGL(k_rhs3_rows, grd, blk, 0, s, ev0, ev1, 0, u, b, g, ph, lam_dev, lam_host);
    }
}

// ------------------------------------------------------------------------------------------
// mixed precision helpers
template <int D>
__global__ __launch_bounds__(256) void k_residual_demote(const double* __restrict__ u, const double* __restrict__ b,
                                                         float* __restrict__ r, Grid g) {
    const int i = 1 + blockIdx.x * 64 + threadIdx.x;
    const int j = 1 + blockIdx.y * 4 + threadIdx.y;
    const int k = (D == 3) ? 1 + (int)blockIdx.z : 0;
    const int n = g.n;
    if (i > n - 1 || j > n - 1) return;
    const int64_t P = g.pitch, S = g.plane;
    const int64_t p = i + P * j + S * k;
    const Stencil<double> ks = stencil_of<double>(g);
    double ku;
    if (D == 2)
        ku = kdiff(ks, u[p], nsum2(ks, u[p - 1], u[p + 1], u[p - P], u[p + P]));
    else
        ku = g.h * kdiff(ks, u[p], nsum3(ks, u[p - 1], u[p + 1], u[p - P], u[p + P], u[p - S], u[p + S]));
    r[p] = (float)(b[p] - ku);
}

template <int D>
__global__ __launch_bounds__(256) void k_add_promote(double* __restrict__ u, const float* __restrict__ e, Grid g) {
    const int i = 1 + blockIdx.x * 64 + threadIdx.x;
    const int j = 1 + blockIdx.y * 4 + threadIdx.y;
    const int k = (D == 3) ? 1 + (int)blockIdx.z : 0;
    const int n = g.n;
    if (i > n - 1 || j > n - 1) return;
    const int64_t p = i + g.pitch * j + g.plane * k;
    u[p] += (double)e[p];
}

// The 3D form: each thread walks a column of up to kDemoteZ nodes along z and keeps u at
// k - 1, k and k + 1 in registers, so only the in-plane neighbours come through the caches;
// the node expression is that of k_residual_demote (same bits).
constexpr int kDemoteZ = 16;
__global__ __launch_bounds__(256) void k_residual_demote3_z(const double* __restrict__ u,
                                                            const double* __restrict__ b, float* __restrict__ r,
                                                            Grid g) {
    const int i = 1 + blockIdx.x * 64 + threadIdx.x;
    const int j = 1 + blockIdx.y * 4 + threadIdx.y;
    const int k0 = 1 + (int)blockIdx.z * kDemoteZ;
    const int n = g.n;
    if (i > n - 1 || j > n - 1) return;
    const int k1 = min(k0 + kDemoteZ, n);   // exclusive; k0 <= n - 1 by the grid
    const int64_t P = g.pitch, S = g.plane;
    const Stencil<double> ks = stencil_of<double>(g);
    int64_t p = i + P * j + S * k0;
    double um = u[p - S], uc = u[p];
#pragma unroll 4
    for (int k = k0; k < k1; ++k, p += S) {
        const double up = u[p + S];
        const double ku = g.h * kdiff(ks, uc, nsum3(ks, u[p - 1], u[p + 1], u[p - P], u[p + P], um, up));
        r[p] = (float)(b[p] - ku);
        um = uc;
        uc = up;
    }
}

void launch_residual_demote(const Grid& g, const double* u, const double* b, float* r, hipStream_t s) {
    const int n = g.n;
    dim3 blk(64, 4, 1);
    if (g.dim == 2) {
        dim3 grd(cdiv(n - 1, 64), cdiv(n - 1, 4), 1);
        hipLaunchKernelGGL(k_residual_demote<2>, grd, blk, 0, s, u, b, r, g);
    } else {
        dim3 grd(cdiv(n - 1, 64), cdiv(n - 1, 4), cdiv(n - 1, kDemoteZ));
        hipLaunchKernelGGL(k_residual_demote3_z, grd, blk, 0, s, u, b, r, g);
    }
}
void launch_add_promote(const Grid& g, double* u, const float* e, hipStream_t s) {
    const int n = g.n;
    dim3 blk(64, 4, 1);
    dim3 grd(cdiv(n - 1, 64), cdiv(n - 1, 4), g.dim == 3 ? n - 1 : 1);
    if (g.dim == 2)
        hipLaunchKernelGGL(k_add_promote<2>, grd, blk, 0, s, u, e, g);
    else
        hipLaunchKernelGGL(k_add_promote<3>, grd, blk, 0, s, u, e, g);
}

// ------------------------------------------------------------------------------------------
// u <- c u~ + Pi x_H.  Pi x_H at a fine node is the coarsest-level P1 function evaluated
// there: the coarse cell and the simplex inside it follow from the coarse-local
// coordinates (2D: lower triangle when X >= Y; 3D: the Kuhn simplex of the ordering of
// X, Y, Z), and the barycentric weights from the sorted coordinates.
template <int D>
__global__ __launch_bounds__(256) void k_form_u(double* __restrict__ u, const double* __restrict__ xc, Grid gf,
                                                Grid gc, const double* __restrict__ coef, int ls) {
    const int i = 1 + blockIdx.x * 64 + threadIdx.x;
    const int j = 1 + blockIdx.y * 4 + threadIdx.y;
    const int k = (D == 3) ? 1 + (int)blockIdx.z : 0;
    const int n = gf.n, nc = gc.n;
    if (i > n - 1 || j > n - 1) return;
    // fine cells per coarse cell edge: s = n / nc = 2^ls (nested refinements)
    const double inv_s = 1.0 / (double)(1 << ls);
    int c0[3] = {min(i >> ls, nc - 1), min(j >> ls, nc - 1), D == 3 ? min(k >> ls, nc - 1) : 0};
    double t[3] = {(i - (c0[0] << ls)) * inv_s, (j - (c0[1] << ls)) * inv_s, D == 3 ? (k - (c0[2] << ls)) * inv_s : 0.0};
    // sort axes by coordinate, descending (ties: lower axis first)
    int ax[3] = {0, 1, 2};
    if (D == 2) {
        if (t[1] > t[0]) { ax[0] = 1; ax[1] = 0; }
    } else {
        if (t[ax[1]] > t[ax[0]]) { int q = ax[0]; ax[0] = ax[1]; ax[1] = q; }
        if (t[ax[2]] > t[ax[1]]) { int q = ax[1]; ax[1] = ax[2]; ax[2] = q; }
        if (t[ax[1]] > t[ax[0]]) { int q = ax[0]; ax[0] = ax[1]; ax[1] = q; }
    }
    const int64_t Pc = gc.pitch, Sc = gc.plane;
    int64_t q = c0[0] + Pc * c0[1] + Sc * c0[2];
    double val = (1.0 - t[ax[0]]) * xc[q];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        q += (ax[r] == 0) ? 1 : (ax[r] == 1 ? Pc : Sc);
        double wgt = (r + 1 < D) ? t[ax[r]] - t[ax[r + 1]] : t[ax[r]];
        val += wgt * xc[q];
    }
    const int64_t p = i + gf.pitch * j + gf.plane * k;
    u[p] = coef[0] * u[p] + val;
}

void launch_form_u(const Grid& gf, const Grid& gc, double* u, const double* xc_level, const double* coef,
                   hipStream_t s) {
    const int n = gf.n;
    int ls = 0;
    while ((gc.n << ls) < n) ++ls;   // n = gc.n 2^ls on every level of the hierarchy
    dim3 blk(64, 4, 1);
    dim3 grd(cdiv(n - 1, 64), cdiv(n - 1, 4), gf.dim == 3 ? n - 1 : 1);
    if (gf.dim == 2)
        hipLaunchKernelGGL(k_form_u<2>, grd, blk, 0, s, u, xc_level, gf, gc, coef, ls);
    else
        hipLaunchKernelGGL(k_form_u<3>, grd, blk, 0, s, u, xc_level, gf, gc, coef, ls);
}

// ------------------------------------------------------------------------------------------
// Rayleigh-quotient pieces of a 2D level (3D: k_forms3_rows): (u^T K u, u^T M_W u, u^T M u,
// int u^4 = u^T N(u)), block sums in a fixed grid, then one block adds the partials in index
// order (deterministic).  With
// lam set, two more sums: |r|^2 and |lam M u|^2 of the nodal residual of the discrete
// problem (2.4), r = K u + M_W u + zeta N(u) - lam M u.
template <int D, int NQ>
__global__ __launch_bounds__(256) void k_forms(const double* __restrict__ u, Grid g, Phys ph,
                                               const double* __restrict__ lam, double* __restrict__ partial) {
    const int n = g.n, m = n - 1;
    const int64_t total = (D == 2) ? (int64_t)m * m : (int64_t)m * m * m;
    const double lv = (NQ > 4) ? *lam : 0.0;
    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        interior_ijk(n, D, t, i, j, k);
        double Mu, MWu, Nu, Ku;
        node_forms<D>(u, g, ph, i, j, k, Mu, MWu, Nu, Ku);
        double u0 = u[i + g.pitch * j + g.plane * k];
        a[0] += u0 * Ku;
        a[1] += u0 * MWu;
        a[2] += u0 * Mu;
        a[3] += u0 * Nu;
        if (NQ > 4) {
            const double lm = lv * Mu, r = (Ku + MWu + ph.zeta * Nu) - lm;
            a[4] += r * r;
            a[5] += lm * lm;
        }
    }
    __shared__ double red[4][NQ];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = wave_sum(a[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double v = 0.0;
        for (int w = 0; w < 4; ++w) v += red[w][threadIdx.x];
        partial[blockIdx.x * NQ + threadIdx.x] = v;
    }
}

// fixed-order sum of nblk partials (stride width, column q) by one 256-thread block:
// thread t adds rows t, t + 256, ...; then the wavefront tree and the 4 wavefronts in order
__device__ double block_sum_partials(const double* __restrict__ partial, int nblk, int width, int q) {
    __shared__ double red[4];
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) v += partial[b * width + q];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double tot = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int nblk, int width,
                                                      double* __restrict__ out) {
    for (int q = 0; q < width; ++q) {
        const double v = block_sum_partials(partial, nblk, width, q);
        if (threadIdx.x == 0) out[q] = v;
    }
}

void launch_forms(const Grid& g, const Phys& ph, const double* u, double* partial, double* out, hipStream_t s,
                  const double* lam) {
    const dim3 blk3(64, 4, 1);
    if (g.dim == 2 && lam)
        hipLaunchKernelGGL((k_forms<2, 6>), dim3(kReduceBlocks), dim3(256), 0, s, u, g, ph, lam, partial);
    else if (g.dim == 2)
        hipLaunchKernelGGL((k_forms<2, 4>), dim3(kReduceBlocks), dim3(256), 0, s, u, g, ph, lam, partial);
    else if (lam)
        hipLaunchKernelGGL((k_forms3_rows<6>), dim3(kReduceBlocks), blk3, 0, s, u, g, ph, lam, partial);
    else
        hipLaunchKernelGGL((k_forms3_rows<4>), dim3(kReduceBlocks), blk3, 0, s, u, g, ph, lam, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partial, kReduceBlocks, lam ? 6 : 4, out);
}

// ------------------------------------------------------------------------------------------
// Conjugate-gradient smoothing (the smoother of the paper's experiments): `steps`
// iterations of CG on K x = f from the current x.  r, p, q are level arrays with zero
// rings; sc holds (r.r, p.q, alpha, beta) in FP64.  Dot products are block partials in a
// fixed grid added in a fixed order (deterministic); alpha and beta are formed on the
// device, so the host only enqueues.  rr = 0 makes alpha = beta = 0 (x stays put, as an
// exact solve would leave it).
template <int D, typename T>
__device__ inline T apply_K(const Stencil<T>& k, const T* __restrict__ x, int64_t q, int64_t P, int64_t S, T h) {
    if (D == 2) return kdiff(k, x[q], nsum2(k, x[q - 1], x[q + 1], x[q - P], x[q + P]));
    return h * kdiff(k, x[q], nsum3(k, x[q - 1], x[q + 1], x[q - P], x[q + P], x[q - S], x[q + S]));
}

template <int D>
__device__ inline int64_t interior_node(const Grid& g, int64_t t) {
    int i, j, k;
    interior_ijk(g.n, D, t, i, j, k);
    return i + g.pitch * j + g.plane * k;
}

__device__ inline void block_partial(double v, double* __restrict__ partial) {
    __shared__ double red[4];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

#define CG_NODES(D, g)                                                                                   \
    const int64_t total_ = (D == 2) ? (int64_t)((g).n - 1) * ((g).n - 1)                                 \
                                    : (int64_t)((g).n - 1) * ((g).n - 1) * ((g).n - 1);                  \
    for (int64_t t_ = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t_ < total_;                       \
         t_ += (int64_t)gridDim.x * blockDim.x)

// zero the Dirichlet ring of a level array (the CG scratch arrays serve several levels, so
// their ring positions for this level may hold values of another level's layout)
template <int D, typename T>
__global__ __launch_bounds__(256) void k_zero_ring(T* __restrict__ a, Grid g) {
    const int n = g.n, w = n + 1;
    const int64_t per = (D == 2) ? (int64_t)w : (int64_t)w * w;
    const int64_t total = per * (2 * D);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int face = (int)(t / per);
        const int64_t rem = t - face * per;
        const int u = (int)(rem % w), v = (D == 3) ? (int)(rem / w) : 0;
        const int side = (face & 1) ? n : 0, axis = face >> 1;
        int c[3] = {u, v, 0};
        if (D == 2) {
            c[0] = axis == 0 ? side : u;
            c[1] = axis == 0 ? u : side;
        } else {
            c[0] = axis == 0 ? side : u;
            c[1] = axis == 1 ? side : (axis == 0 ? u : v);
            c[2] = axis == 2 ? side : v;
        }
        a[c[0] + g.pitch * c[1] + g.plane * c[2]] = T(0);
    }
}

// r = f - K x, p = r; partial r.r
template <int D, typename T>
__global__ __launch_bounds__(256) void k_cg_start(const T* __restrict__ x, const T* __restrict__ f, T* __restrict__ r,
                                                  T* __restrict__ p, Grid g, double* __restrict__ partial) {
    double acc = 0.0;
    CG_NODES(D, g) {
        const int64_t q = interior_node<D>(g, t_);
        const T v = resid_at<D, T>(stencil_of<T>(g), x, f, q, g.pitch, g.plane, T(g.h));
        r[q] = v;
        p[q] = v;
        acc += (double)v * (double)v;
    }
    block_partial(acc, partial);
}

// q = K p; partial p.q
template <int D, typename T>
__global__ __launch_bounds__(256) void k_cg_apply(const T* __restrict__ p, T* __restrict__ qv, Grid g,
                                                  double* __restrict__ partial) {
    double acc = 0.0;
    CG_NODES(D, g) {
        const int64_t q = interior_node<D>(g, t_);
        const T v = apply_K<D, T>(stencil_of<T>(g), p, q, g.pitch, g.plane, T(g.h));
        qv[q] = v;
        acc += (double)p[q] * (double)v;
    }
    block_partial(acc, partial);
}

// x += alpha p, r -= alpha q; partial r.r
template <int D, typename T>
__global__ __launch_bounds__(256) void k_cg_update(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                                   const T* __restrict__ qv, Grid g, const double* __restrict__ sc,
                                                   double* __restrict__ partial) {
    const T alpha = T(sc[2]);
    double acc = 0.0;
    CG_NODES(D, g) {
        const int64_t q = interior_node<D>(g, t_);
        x[q] += alpha * p[q];
        const T v = r[q] - alpha * qv[q];
        r[q] = v;
        acc += (double)v * (double)v;
    }
    block_partial(acc, partial);
}

// p = r + beta p
template <int D, typename T>
__global__ __launch_bounds__(256) void k_cg_direction(const T* __restrict__ r, T* __restrict__ p, Grid g,
                                                      const double* __restrict__ sc) {
    const T beta = T(sc[3]);
    CG_NODES(D, g) {
        const int64_t q = interior_node<D>(g, t_);
        p[q] = r[q] + beta * p[q];
    }
}
#undef CG_NODES

// stage 0: sc[0] = r.r; 1: sc[1] = p.q, alpha = r.r / p.q; 2: beta = r'.r' / r.r, sc[0] = r'.r'
__global__ __launch_bounds__(256) void k_cg_scalars(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ sc, int stage) {
    const double v = block_sum_partials(partial, nblk, 1, 0);
    if (threadIdx.x != 0) return;
    if (stage == 0) {
        sc[0] = v;
    } else if (stage == 1) {
        sc[1] = v;
        sc[2] = (sc[0] == 0.0) ? 0.0 : sc[0] / v;
    } else {
        sc[3] = (sc[0] == 0.0) ? 0.0 : v / sc[0];
        sc[0] = v;
    }
}

template <typename T>
void launch_cg_smooth(const Grid& g, T* x, const T* f, int steps, T* r, T* p, T* q, double* partial, double* sc,
                      hipStream_t s) {
    if (steps <= 0 || g.n < 2) return;
    const dim3 grd(kReduceBlocks), blk(256);
    if (g.dim == 2) {
        hipLaunchKernelGGL((k_zero_ring<2, T>), dim3(cdiv(4 * (int64_t)(g.n + 1), 256)), blk, 0, s, p, g);
        hipLaunchKernelGGL((k_cg_start<2, T>), grd, blk, 0, s, x, f, r, p, g, partial);
    } else {
        hipLaunchKernelGGL((k_zero_ring<3, T>), dim3(cdiv(6 * (int64_t)(g.n + 1) * (g.n + 1), 256)), blk, 0, s, p, g);
        hipLaunchKernelGGL((k_cg_start<3, T>), grd, blk, 0, s, x, f, r, p, g, partial);
    }
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), blk, 0, s, partial, kReduceBlocks, sc, 0);
    for (int it = 0; it < steps; ++it) {
        if (g.dim == 2) hipLaunchKernelGGL((k_cg_apply<2, T>), grd, blk, 0, s, p, q, g, partial);
        else hipLaunchKernelGGL((k_cg_apply<3, T>), grd, blk, 0, s, p, q, g, partial);
        hipLaunchKernelGGL(k_cg_scalars, dim3(1), blk, 0, s, partial, kReduceBlocks, sc, 1);
        if (g.dim == 2) hipLaunchKernelGGL((k_cg_update<2, T>), grd, blk, 0, s, x, r, p, q, g, sc, partial);
        else hipLaunchKernelGGL((k_cg_update<3, T>), grd, blk, 0, s, x, r, p, q, g, sc, partial);
        if (it + 1 == steps) break;   // the last direction is never used
        hipLaunchKernelGGL(k_cg_scalars, dim3(1), blk, 0, s, partial, kReduceBlocks, sc, 2);
        if (g.dim == 2) hipLaunchKernelGGL((k_cg_direction<2, T>), grd, blk, 0, s, r, p, g, sc);
        else hipLaunchKernelGGL((k_cg_direction<3, T>), grd, blk, 0, s, r, p, g, sc);
    }
}
template void launch_cg_smooth<double>(const Grid&, double*, const double*, int, double*, double*, double*, double*,
                                       double*, hipStream_t);
template void launch_cg_smooth<float>(const Grid&, float*, const float*, int, float*, float*, float*, double*, double*,
                                      hipStream_t);

}  // namespace fmg
