// Fine-grid quadratures for the augmented problem (3.6) on V_H + span{u~}.
//
// The nonlinear part of the augmented matrices is S(x) = Z^T M_{(Zx)^2} Z with
// Z = [coarse hats, u~] and u = u_H + c u~.  Expanding (u_H + c u~)^2 shows that every
// entry of S(x), for every x, is a combination of a fixed set of integrals of powers of u~
// against polynomials of the coarse barycentric coordinates on each coarse simplex
// (layout.h).  They are computed here in one pass over the fine mesh per correction step,
// so the Newton iterations of the small solve never touch the fine grid again.  (The paper
// re-assembles on the fine grid in every nonlinear iteration; the result is the same.)
//
// Pass 1 (k_moments_raw): block (coarse cell, chunk, coarse simplex type) integrates
// u~^a X^b over the fine simplices of that coarse simplex with an exact degree-4 rule
// (tables.h) and writes one partial sum per block.  A block walks only the fine cells that
// meet its coarse simplex: in 2D the cells (a0, a1) on one side of the diagonal (a
// triangular index set, folded into full rows), in 3D the cells whose coordinates are
// ordered as the coarse tetrahedron's axis permutation orders them (sorted triples).  Pass 2 (k_moments_final): one thread
// per coarse simplex adds the partials in chunk order and converts the X-monomial moments
// to the barycentric form.  Both passes are deterministic.
#include <utility>

#include "kernels.h"
#include "layout.h"

namespace fmg {

int moments_per_element(int dim) { return dim == 2 ? MomLayout<2>::SIZE : MomLayout<3>::SIZE; }

static constexpr int kChunkCells = 2048;

static int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    while (e--) r *= b;
    return r;
}

// cells_per: fine cells one block list covers.  2D: the fine cells (a0, a1) of one coarse
// triangle, a0 >= a1 or a0 <= a1 (diagonal cells included, s (s + 1) / 2 of them), as s / 2
// rows of s + 1 cells (s = n / nc is even on every level that has moments).  3D: the cells
// with a_p0 >= a_p1 >= a_p2 for the coarse tetrahedron's axis order (p0, p1, p2),
// s (s + 1) (s + 2) / 6 of them.
static void chunk_shape(int dim, int nc, int n, int64_t& ncell, int64_t& cells_per, int64_t& nchunk) {
    const int s = n / nc;
    ncell = ipow(nc, dim);
    cells_per = dim == 2 ? (int64_t)(s / 2) * (s + 1) : (int64_t)s * (s + 1) * (s + 2) / 6;
    nchunk = (cells_per + kChunkCells - 1) / kChunkCells;
}

size_t moments_scratch_bytes(int dim, int nc, int n) {
    int64_t ncell, cells_per, nchunk;
    chunk_shape(dim, nc, n, ncell, cells_per, nchunk);
    const int raw = dim == 2 ? RawLayout<2>::SIZE : RawLayout<3>::SIZE;
    const int ne = dim == 2 ? 2 : 6;
    return sizeof(double) * (size_t)(ncell * ne * nchunk * raw);
}

// coarse simplex type of a fine simplex of fine type tf in the fine cell at coarse-local
// offset a[]: order the axes by (a desc, position in the fine path asc)
template <int D>
__device__ inline int coarse_type(const int* a, int tf) {
    if (D == 2) {
        if (a[0] != a[1]) return a[0] > a[1] ? 0 : 1;
        return tf;
    } else {
        int pos[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) pos[kPerm3[tf][r]] = r;
        int ax[3] = {0, 1, 2};
        auto before = [&](int p, int q) { return a[p] != a[q] ? a[p] > a[q] : pos[p] < pos[q]; };
        if (before(ax[1], ax[0])) { int t = ax[0]; ax[0] = ax[1]; ax[1] = t; }
        if (before(ax[2], ax[1])) { int t = ax[1]; ax[1] = ax[2]; ax[2] = t; }
        if (before(ax[1], ax[0])) { int t = ax[0]; ax[0] = ax[1]; ax[1] = t; }
        return 2 * ax[0] + (ax[1] > ax[2] ? 1 : 0);
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_moments_raw(const double* __restrict__ ut, Grid g, int nc,
                                                     int64_t cells_per, int s, double* __restrict__ partial) {
    using R = RawLayout<D>;
    constexpr int V = D + 1;
    constexpr int NF = (D == 2) ? 2 : 6;   // fine simplices per fine cell
    const int64_t cell = blockIdx.x;
    const int64_t chunk = blockIdx.y;
    const int type = blockIdx.z;
    const int64_t nchunk = gridDim.y;
    int C[3] = {(int)(cell % nc), (int)((cell / nc) % nc), D == 3 ? (int)(cell / ((int64_t)nc * nc)) : 0};
    const int64_t start = chunk * kChunkCells;
    const int64_t end = min(cells_per, start + (int64_t)kChunkCells);
    const double inv_s = 1.0 / s;
    const double h = g.h;
    const double vol = (D == 2) ? 0.5 * h * h : h * h * h / 6.0;
    const int64_t P = g.pitch, S = g.plane;
    double acc[R::SIZE];
#pragma unroll
    for (int q = 0; q < R::SIZE; ++q) acc[q] = 0.0;

    for (int64_t idx = start + threadIdx.x; idx < end; idx += blockDim.x) {
        int a[3];
        if (D == 2) {
            // row pair (r, s-1-r) of the triangular set: s - r cells of row r, then r + 1 of
            // row s-1-r; (lo, hi) = (row, column) with hi >= lo
            const int t = (int)idx, r = t / (s + 1), x = t - r * (s + 1);
            int lo, hi;
            if (x < s - r) {
                lo = r;
                hi = r + x;
            } else {
                lo = s - 1 - r;
                hi = lo + (x - (s - r));
            }
            a[0] = type == 0 ? hi : lo;
            a[1] = type == 0 ? lo : hi;
            a[2] = 0;
        } else {
            // idx -> sorted triple i >= j >= k: i from the tetrahedral numbers i(i+1)(i+2)/6,
            // then (j, k) from the triangular numbers j(j+1)/2
            const int64_t t = idx;
            int i = (int)cbrt(6.0 * (double)t);
            while ((int64_t)i * (i + 1) * (i + 2) / 6 > t) --i;
            while ((int64_t)(i + 1) * (i + 2) * (i + 3) / 6 <= t) ++i;
            const int r = (int)(t - (int64_t)i * (i + 1) * (i + 2) / 6);
            int j = (int)((sqrt(8.0 * r + 1.0) - 1.0) * 0.5);
            while (j * (j + 1) / 2 > r) --j;
            while ((j + 1) * (j + 2) / 2 <= r) ++j;
            const int k = r - j * (j + 1) / 2;
            // type 2 p0 + q: largest axis p0; q = 1 puts the larger remaining axis second
            const int p0 = type >> 1, o1 = p0 == 0 ? 1 : 0, o2 = p0 == 2 ? 1 : 2;
            const int p1 = (type & 1) ? o2 : o1, p2 = (type & 1) ? o1 : o2;
            a[p0] = i;
            a[p1] = j;
            a[p2] = k;
        }
        const int i = C[0] * s + a[0], j = C[1] * s + a[1], k = D == 3 ? C[2] * s + a[2] : 0;
        const int64_t base = i + P * j + S * k;
#pragma unroll
        for (int tf = 0; tf < NF; ++tf) {
            if (coarse_type<D>(a, tf) != type) continue;
            double uv[V], X[V][3];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                int o[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) o[d] = (d < D) ? (D == 2 ? kCellElemVert2D[tf][v][d] : kCellElemVert3D[tf][v][d]) : 0;
                uv[v] = ut[base + o[0] + P * o[1] + S * o[2]];
#pragma unroll
                for (int d = 0; d < D; ++d) X[v][d] = (a[d] + o[d]) * inv_s;
            }
            // gradient moments
            double gr[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int d = 0; d < D; ++d)
                    gr[d] += uv[v] * (D == 2 ? kCellElemBary2D[tf][v][1 + d] : kCellElemBary3D[tf][v][1 + d]);
            double g2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                acc[R::G + d] += vol * gr[d] / h;
                g2 += gr[d] * gr[d];
            }
            acc[R::Q] += vol * g2 / (h * h);
            // exact degree-4 rule
            constexpr int NQ = (D == 2) ? kQuad2D : kQuad3D;
#pragma unroll
            for (int qp = 0; qp < NQ; ++qp) {
                double w = vol * (D == 2 ? kQuadW2D[qp] : kQuadW3D[qp]);
                double uq = 0.0, x[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    double b = (D == 2) ? kQuadPt2D[qp][v] : kQuadPt3D[qp][v];
                    uq += b * uv[v];
                    if (D == 3) {
#pragma unroll
                        for (int d = 0; d < D; ++d) x[d] += b * X[v][d];
                    }
                }
                if (D == 2) {
                    // the point's offset in the fine cell is a constant of (tf, qp): one
                    // multiply-add per coordinate instead of the vertex sum
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        double cd = 0.0;
#pragma unroll
                        for (int v = 0; v < V; ++v) cd += kQuadPt2D[qp][v] * kCellElemVert2D[tf][v][d];
                        x[d] = (a[d] + cd) * inv_s;
                    }
                }
                const double wu = w * uq, wu2 = wu * uq, wu3 = wu2 * uq, wu4 = wu3 * uq;
                if (D == 2) {
                    const double X1 = x[0], Y1 = x[1];
                    const double X2 = X1 * X1, XY = X1 * Y1, Y2 = Y1 * Y1;
                    const double m[10] = {1.0, X1, Y1, X2, XY, Y2, X2 * X1, X2 * Y1, X1 * Y2, Y2 * Y1};
#pragma unroll
                    for (int q = 0; q < 10; ++q) acc[R::P1 + q] += wu * m[q];
#pragma unroll
                    for (int q = 0; q < 6; ++q) acc[R::P2 + q] += wu2 * m[q];
#pragma unroll
                    for (int q = 0; q < 3; ++q) acc[R::P3 + q] += wu3 * m[q];
                } else {
                    double m[20];
#pragma unroll
                    for (int q = 0; q < 20; ++q) {
                        double t = 1.0;
#pragma unroll
                        for (int d = 0; d < 3; ++d)
#pragma unroll
                            for (int e = 0; e < kMon3[q][d]; ++e) t *= x[d];
                        m[q] = t;
                    }
#pragma unroll
                    for (int q = 0; q < 20; ++q) acc[R::P1 + q] += wu * m[q];
#pragma unroll
                    for (int q = 0; q < 10; ++q) acc[R::P2 + q] += wu2 * m[q];
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[R::P3 + q] += wu3 * m[q];
                }
                acc[R::P4] += wu4;
            }
        }
    }
    // block reduction (fixed order)
    __shared__ double red[4][R::SIZE];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < R::SIZE; ++q) {
        double v = wave_sum(acc[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    const int64_t ncell = gridDim.x;
    for (int q = threadIdx.x; q < R::SIZE; q += blockDim.x) {
        double v = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
        partial[(((int64_t)type * ncell + cell) * nchunk + chunk) * R::SIZE + q] = v;
    }
}

// ---- pass 2 ------------------------------------------------------------------------------
// Polynomials of the coarse-local coordinates are coefficient arrays over the graded
// monomial lists of layout.h (degree <= 3).  All loops below have compile-time bounds and
// indices, so the products are straight-line register code.
template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

template <int D>
struct Mono {
    static constexpr int NM = (D == 2) ? 10 : 20;        // degree <= 3
    static constexpr int N2 = (D == 2) ? 6 : 10;         // degree <= 2
    static constexpr int exp(int q, int k) { return D == 2 ? kMon2[q][k] : kMon3[q][k]; }
    // index of monomial q times x_d, -1 above degree 3
    static constexpr int times_x(int q, int d) {
        for (int r = 0; r < NM; ++r) {
            bool ok = true;
            for (int k = 0; k < D; ++k) ok = ok && exp(r, k) == exp(q, k) + (k == d ? 1 : 0);
            if (ok) return r;
        }
        return -1;
    }
    static constexpr int square(int d) { return times_x(times_x(0, d), d); }   // x_d^2
};

// out = A * (l[0] + sum_d l[1+d] x_d) for A of degree <= 2 (its first N2 coefficients)
template <int D>
__device__ __forceinline__ void mul_affine(const double* A, const double* l, double* out) {
    using M = Mono<D>;
    static_for<M::NM>([&](auto q) { out[q] = 0.0; });
    static_for<M::N2>([&](auto q_) {
        constexpr int q = decltype(q_)::value;
        out[q] += A[q] * l[0];
        static_for<D>([&](auto d_) {
            constexpr int d = decltype(d_)::value;
            constexpr int j = M::times_x(q, d);
            if constexpr (j >= 0) out[j] += A[q] * l[1 + d];
        });
    });
}

template <int D>
__global__ __launch_bounds__(64) void k_moments_final(const double* __restrict__ partial, int nc, int64_t nchunk, Phys ph,
                                double* __restrict__ out) {
    using R = RawLayout<D>;
    using L = MomLayout<D>;
    using M = Mono<D>;
    constexpr int V = D + 1;
    constexpr int NM = M::NM;
    const int64_t ncell = (D == 2) ? (int64_t)nc * nc : (int64_t)nc * nc * nc;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ncell * L::NE) return;
    const int64_t cell = e / L::NE;
    const int type = (int)(e % L::NE);
    double raw[R::SIZE];
    static_for<R::SIZE>([&](auto q) { raw[q] = 0.0; });
    for (int64_t c = 0; c < nchunk; ++c) {
        const double* pp = partial + (((int64_t)type * ncell + cell) * nchunk + c) * R::SIZE;
        static_for<R::SIZE>([&](auto q) { raw[q] += pp[q]; });
    }

    // barycentric coordinates of the coarse simplex as affine functions of X
    double lam[V][4], lamp[V][NM];
    static_for<V>([&](auto p) {
        static_for<D + 1>([&](auto k) {
            lam[p][k] = (D == 2) ? kCellElemBary2D[type][p][k] : kCellElemBary3D[type][p][k];
        });
        static_for<NM>([&](auto q) { lamp[p][q] = 0.0; });
        static_for<D + 1>([&](auto k) { lamp[p][k] = lam[p][k]; });   // 1, x_0, .. are monomials 0..D
    });
    // W in coarse-local coordinates: x_k = (C_k + X_k) H
    const double H = 1.0 / nc;
    const int C[3] = {(int)(cell % nc), (int)((cell / nc) % nc), D == 3 ? (int)(cell / ((int64_t)nc * nc)) : 0};
    double Wp[NM];
    static_for<NM>([&](auto q) { Wp[q] = 0.0; });
    Wp[0] = ph.wc;
    static_for<D>([&](auto d_) {
        constexpr int d = decltype(d_)::value;
        const double wk = ph.w[d] * H * H;
        Wp[0] += wk * C[d] * C[d];
        Wp[1 + d] += 2.0 * wk * C[d];
        Wp[M::square(d)] += wk;
    });
    double* o = out + e * L::SIZE;
    double t1[NM], t2[NM];
    static_for<V>([&](auto p_) {
        constexpr int p = decltype(p_)::value;
        static_for<V - p>([&](auto qq) {
            constexpr int q = p + decltype(qq)::value;
            mul_affine<D>(lamp[p], lam[q], t1);
            double s2 = 0.0;
            static_for<R::M2>([&](auto m) { s2 += t1[m] * raw[R::P2 + m]; });
            o[L::T2 + sym2(p, q, D + 1)] = s2;
            static_for<V - q>([&](auto rr) {
                constexpr int r = q + decltype(rr)::value;
                mul_affine<D>(t1, lam[r], t2);
                double s3 = 0.0;
                static_for<NM>([&](auto m) { s3 += t2[m] * raw[R::P1 + m]; });
                o[L::T3 + sym3(p, q, r, D + 1)] = s3;
            });
        });
    });
    static_for<V>([&](auto p) {
        double s1 = 0.0, sb = 0.0;
        static_for<R::M1>([&](auto m) {
            s1 += lamp[p][m] * raw[R::P3 + m];
            sb += lamp[p][m] * raw[R::P1 + m];
        });
        o[L::T1 + p] = s1;
        o[L::B1 + p] = sb;
        mul_affine<D>(Wp, lam[p], t1);
        double sw = 0.0;
        static_for<NM>([&](auto m) { sw += t1[m] * raw[R::P1 + m]; });
        o[L::AW1 + p] = sw;
        double kg = 0.0;
        static_for<D>([&](auto d) { kg += lam[p][1 + d] / H * raw[R::G + d]; });
        o[L::KG + p] = kg;
    });
    o[L::T0] = raw[R::P4];
    o[L::B2] = raw[R::P2];
    double aw2 = 0.0;
    static_for<R::M2>([&](auto m) { aw2 += Wp[m] * raw[R::P2 + m]; });
    o[L::AW2] = aw2;
    o[L::Q] = raw[R::Q];
}

void launch_moments(int dim, int nc, const Grid& g, const Phys& ph, const double* ut, double* scratch, double* out,
                    hipStream_t s) {
    int64_t ncell, cells_per, nchunk;
    chunk_shape(dim, nc, g.n, ncell, cells_per, nchunk);
    const int sc = g.n / nc;
    if (dim == 2) {
        hipLaunchKernelGGL(k_moments_raw<2>, dim3((unsigned)ncell, (unsigned)nchunk, 2), dim3(256), 0, s, ut, g, nc,
                           cells_per, sc, scratch);
        hipLaunchKernelGGL(k_moments_final<2>, dim3(cdiv(ncell * 2, 64)), dim3(64), 0, s, scratch, nc, nchunk, ph, out);
    } else {
        hipLaunchKernelGGL(k_moments_raw<3>, dim3((unsigned)ncell, (unsigned)nchunk, 6), dim3(256), 0, s, ut, g, nc,
                           cells_per, sc, scratch);
        hipLaunchKernelGGL(k_moments_final<3>, dim3(cdiv(ncell * 6, 64)), dim3(64), 0, s, scratch, nc, nchunk, ph, out);
    }
}

}  // namespace fmg
