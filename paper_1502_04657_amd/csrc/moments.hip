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
// u~^k X^b (X: coarse-local coordinates) over the fine cells of that coarse simplex and
// writes one partial sum per block.  Integration is exact and needs no quadrature points:
// on a fine cell with corner A (in fine-cell units of the coarse cell) and cell coordinates
// Y, X = (A + Y) / s, and every local moment int u~^k Y^b is a fixed rational combination
// of products of the cell's corner values (moment_tables.h, derived in
// gen_moment_tables.py) for u~ and u~^2, and of the power sums of each fine simplex's vertex
// values for u~^3 and u~^4; the local moments are then shifted to (A + Y)^b one coordinate
// at a time (binomial expansion), and the powers of s and h are applied once per block.
// A block walks only the fine cells that meet its coarse simplex, in two groups:
//   * interior cells, whose coordinates are strictly ordered as the coarse simplex's axis
//     permutation orders them (all fine simplices of the cell lie in the coarse simplex):
//     the whole-cell tables, grouped by corner products;
//   * cells on the coarse simplex's internal faces (ties among the coordinates): the
//     per-simplex tables for the fine simplices that belong to this coarse simplex.
// Blocks hold one group each, so a wavefront never mixes the two.  Pass 2
// (k_moments_final): one thread per coarse simplex adds the partials in chunk order and
// converts the X-monomial moments to the barycentric form.  Both passes are deterministic.
#include <hip/hip_ext.h>

#include <utility>

#include "kernels.h"
#include "layout.h"
#include "moment_tables.h"

namespace fmg {

int moments_per_element(int dim) { return dim == 2 ? MomLayout<2>::SIZE : MomLayout<3>::SIZE; }

// cells per chunk: at most kChunkCells, the cells of a group split into equal chunks (a
// block's fixed cost, the reduction of its partial sums, is then spread over as many cells as
// possible without a short last chunk)
static constexpr int kChunkCells = 8192;

static int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    while (e--) r *= b;
    return r;
}

// Cells one coarse simplex holds, s = n / nc fine cells per coarse edge:
//   interior: 2D the cells (a0, a1) with a0 > a1 (type 0; a0 < a1 for type 1), s (s - 1) / 2;
//             3D the cells with a_p0 > a_p1 > a_p2 for the type's axis order, s (s-1) (s-2) / 6;
//   ties:     2D the s diagonal cells; 3D the s^2 cells with a_p0 = a_p1 >= a_p2 or
//             a_p0 >= a_p1 = a_p2.
// Chunks of k_int (interior) and k_tie (tie) cells: the interior chunks first, then the tie
// chunks.
struct ChunkShape {
    int64_t ncell, n_int, n_tie, c_int, c_tie, k_int, k_tie;
};
static ChunkShape chunk_shape(int dim, int nc, int n, int target) {
    const int64_t kChunk = target > 0 ? target : kChunkCells;
    const int64_t s = n / nc;
    ChunkShape c;
    c.ncell = ipow(nc, dim);
    c.n_int = dim == 2 ? s * (s - 1) / 2 : s * (s - 1) * (s - 2) / 6;
    c.n_tie = dim == 2 ? s : s * s;
    c.c_int = (c.n_int + kChunk - 1) / kChunk;
    c.c_tie = (c.n_tie + kChunk - 1) / kChunk;
    c.k_int = c.c_int > 0 ? (c.n_int + c.c_int - 1) / c.c_int : 1;
    c.k_tie = c.c_tie > 0 ? (c.n_tie + c.c_tie - 1) / c.c_tie : 1;
    return c;
}

size_t moments_scratch_bytes(int dim, int nc, int n, int chunk_cells) {
    const ChunkShape c = chunk_shape(dim, nc, n, chunk_cells);
    const int raw = dim == 2 ? RawLayout<2>::SIZE : RawLayout<3>::SIZE;
    const int ne = dim == 2 ? 2 : 6;
    return sizeof(double) * (size_t)(c.ncell * ne * (c.c_int + c.c_tie) * raw);
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
    static constexpr int N1 = D + 1;                     // degree <= 1
    static constexpr int exp(int q, int k) { return D == 2 ? kMon2[q][k] : kMon3[q][k]; }
    static constexpr int deg(int q) {
        int t = 0;
        for (int k = 0; k < D; ++k) t += exp(q, k);
        return t;
    }
    // index of the monomial equal to q with the exponent of x_d replaced by e
    static constexpr int with_exp(int q, int d, int e) {
        for (int r = 0; r < NM; ++r) {
            bool ok = true;
            for (int k = 0; k < D; ++k) ok = ok && exp(r, k) == (k == d ? e : exp(q, k));
            if (ok) return r;
        }
        return -1;
    }
    // index of monomial q times x_d, -1 above degree 3
    static constexpr int times_x(int q, int d) { return with_exp(q, d, exp(q, d) + 1); }
    static constexpr int square(int d) { return times_x(times_x(0, d), d); }   // x_d^2
};

// Replace local moments L[q] = int f Y^{m_q} (monomials q < NQ of degree <= 3) by
// int f (A + Y)^{m_q}, one coordinate at a time: along d,
//   (A_d + Y_d)^e = sum_j C(e, j) A_d^(e-j) Y_d^j.
// Entries with a larger exponent of x_d are updated first, so every update reads
// unshifted values of the lower exponents.
template <int D, int NQ>
__device__ __forceinline__ void shift_moments(double* L, const double* A) {
    using M = Mono<D>;
    static_for<D>([&](auto d_) {
        constexpr int d = decltype(d_)::value;
        const double a1 = A[d], a2 = a1 * a1, a3 = a2 * a1;
        static_for<NQ>([&](auto qq) {
            constexpr int q = NQ - 1 - decltype(qq)::value;   // descending: higher degrees first
            constexpr int e = M::exp(q, d);
            if constexpr (e == 1) {
                L[q] += a1 * L[M::with_exp(q, d, 0)];
            } else if constexpr (e == 2) {
                L[q] += 2.0 * a1 * L[M::with_exp(q, d, 1)] + a2 * L[M::with_exp(q, d, 0)];
            } else if constexpr (e == 3) {
                L[q] += 3.0 * a1 * L[M::with_exp(q, d, 2)] + 3.0 * a2 * L[M::with_exp(q, d, 1)] +
                        a3 * L[M::with_exp(q, d, 0)];
            }
        });
    });
}

// table accessors by dimension (the other dimension's table is never indexed)
template <int D> __host__ __device__ constexpr double tC1(int c, int q) { if constexpr (D == 2) return kC1_2D[c][q]; else return kC1_3D[c][q]; }
template <int D> __host__ __device__ constexpr double tC2(int p, int q) { if constexpr (D == 2) return kC2_2D[p][q]; else return kC2_3D[p][q]; }
template <int D> __host__ __device__ constexpr double tCG(int c, int d) { if constexpr (D == 2) return kCG2D[c][d]; else return kCG3D[c][d]; }
template <int D> __host__ __device__ constexpr double tE1(int f, int v, int q) { if constexpr (D == 2) return kE1_2D[f][v][q]; else return kE1_3D[f][v][q]; }
template <int D> __host__ __device__ constexpr double tE2(int f, int p, int q) { if constexpr (D == 2) return kE2_2D[f][p][q]; else return kE2_3D[f][p][q]; }
template <int D> __host__ __device__ constexpr int tPair(int p, int k) { if constexpr (D == 2) return kPair2D[p][k]; else return kPair3D[p][k]; }
template <int D> __host__ __device__ constexpr int tCorner(int f, int v) { if constexpr (D == 2) return kCorner2D[f][v]; else return kCorner3D[f][v]; }
template <int D> __host__ __device__ constexpr double tBary(int f, int v, int k) { if constexpr (D == 2) return kCellElemBary2D[f][v][k]; else return kCellElemBary3D[f][v][k]; }

// Cubic and quartic moments of one fine simplex f of the cell (unit cell, |t| D! = 1), from
// the power sums p_k of its vertex values (u2, u3, u4: the corner values' powers) and the
// complete homogeneous symmetric polynomials h_k they give:
//   int u~^3 = 3!/(D+3)! h3,   int u~^3 l_w = 3!/(D+4)! (h3 + u_w h2 + u_w^2 h1 + u_w^3),
//   int u~^4 = 4!/(D+4)! h4,   Y_d = sum of the l_v of the vertices with y_vd = 1.
// Adds h3 to s3, h4 to s4 and sum over those vertices of the l_w bracket to sy[d]; the
// constants are applied by the caller.
template <int D, int f>
__device__ __forceinline__ void simplex_cubic_quartic(const double* uc, const double* u2, const double* u3,
                                                      const double* u4, double& s3, double& s4, double* sy) {
    constexpr int V = D + 1;
    double p1 = 0.0, p2 = 0.0, p3 = 0.0, p4 = 0.0;
    static_for<V>([&](auto v_) {
        constexpr int c = tCorner<D>(f, decltype(v_)::value);
        p1 += uc[c];
        p2 += u2[c];
        p3 += u3[c];
        p4 += u4[c];
    });
    const double p11 = p1 * p1;
    const double h2 = 0.5 * (p11 + p2);
    const double h3 = (p1 * (p11 + 3.0 * p2) + 2.0 * p3) * (1.0 / 6.0);
    s3 += h3;
    s4 += (p11 * (p11 + 6.0 * p2) + 3.0 * p2 * p2 + 8.0 * p1 * p3 + 6.0 * p4) * (1.0 / 24.0);
    double g[V];
    static_for<V>([&](auto v_) {
        constexpr int c = tCorner<D>(f, decltype(v_)::value);
        g[decltype(v_)::value] = h3 + uc[c] * (h2 + uc[c] * (p1 + uc[c]));
    });
    static_for<D>([&](auto d_) {
        constexpr int d = decltype(d_)::value;
        static_for<V>([&](auto v_) {
            constexpr int v = decltype(v_)::value;
            if constexpr (((tCorner<D>(f, v) >> d) & 1) != 0) sy[d] += g[v];
        });
    });
}

// Local moments of the cell with corner values uc[] (unit cell), accumulated into L1 (deg
// <= 3), L2 (deg <= 2), L3 (deg <= 1), L4 and the gradient sums G (int d u~/dY_d), Q
// (int grad_Y u~ . A grad_Y u~, A = diag(aw)).  WHOLE: all fine simplices of the cell; otherwise the fine simplices
// of the cell at coarse-local offset a[] that belong to coarse simplex `type`.
template <int D, bool WHOLE>
__device__ __forceinline__ void cell_moments(const double* uc, const int* a, int type, const double* aw, double* L1,
                                             double* L2, double* L3, double& L4, double* G, double& Q) {
    using M = Mono<D>;
    constexpr int V = D + 1;
    constexpr int NF = (D == 2) ? 2 : 6;
    constexpr double k4 = (D == 2) ? 1.0 / 30.0 : 1.0 / 210.0;    // 4! / (D + 4)!
    constexpr double k3 = (D == 2) ? 1.0 / 20.0 : 1.0 / 120.0;    // 3! / (D + 3)!
    constexpr double k3w = (D == 2) ? 1.0 / 120.0 : 1.0 / 840.0;  // 3! / (D + 4)!
    constexpr double vs = (D == 2) ? 0.5 : 1.0 / 6.0;             // simplex measure in the unit cell
    if constexpr (WHOLE) {
        constexpr int NC = 1 << D;
        constexpr int NP = (D == 2) ? kPairs2D : kPairs3D;
        static_for<NC>([&](auto c_) {
            constexpr int c = decltype(c_)::value;
            static_for<M::NM>([&](auto q) { L1[q] += uc[c] * tC1<D>(c, q); });
            static_for<D>([&](auto d) { G[d] += uc[c] * tCG<D>(c, d); });
        });
        double pr[NP];
        static_for<NP>([&](auto p_) {
            constexpr int p = decltype(p_)::value;
            constexpr int a = tPair<D>(p, 0);
            constexpr int b = tPair<D>(p, 1);
            pr[p] = uc[a] * uc[b];
            static_for<M::N2>([&](auto q) { L2[q] += pr[p] * tC2<D>(p, q); });
        });
        double u2[NC], u3[NC], u4[NC], s3 = 0.0, s4 = 0.0, sy[D];
        static_for<NC>([&](auto c) {
            u2[c] = uc[c] * uc[c];
            u3[c] = u2[c] * uc[c];
            u4[c] = u2[c] * u2[c];
        });
        static_for<D>([&](auto d) { sy[d] = 0.0; });
        static_for<NF>([&](auto f_) {
            constexpr int f = decltype(f_)::value;
            simplex_cubic_quartic<D, f>(uc, u2, u3, u4, s3, s4, sy);
            double uv[V], g[D];
            static_for<V>([&](auto v) { uv[v] = uc[tCorner<D>(f, v)]; });
            static_for<D>([&](auto d_) {
                constexpr int d = decltype(d_)::value;
                g[d] = 0.0;
                static_for<V>([&](auto v_) {
                    constexpr int v = decltype(v_)::value;
                    constexpr double gb = tBary<D>(f, v, 1 + d);
                    if constexpr (gb != 0.0) g[d] += gb * uv[v];
                });
            });
            double g2 = 0.0;
            static_for<D>([&](auto d) { g2 += aw[d] * g[d] * g[d]; });
            Q += vs * g2;
        });
        L3[0] += k3 * s3;
        static_for<D>([&](auto d) { L3[1 + d] += k3w * sy[d]; });
        L4 += k4 * s4;
    } else {
        constexpr int NC = 1 << D;
        double u2[NC], u3[NC], u4[NC], s3 = 0.0, s4 = 0.0, sy[D];
        static_for<NC>([&](auto c) {
            u2[c] = uc[c] * uc[c];
            u3[c] = u2[c] * uc[c];
            u4[c] = u2[c] * u2[c];
        });
        static_for<D>([&](auto d) { sy[d] = 0.0; });
        static_for<NF>([&](auto f_) {
            constexpr int f = decltype(f_)::value;
            if (coarse_type<D>(a, f) != type) return;
            double uv[V], g[D];
            static_for<V>([&](auto v) { uv[v] = uc[tCorner<D>(f, v)]; });
            static_for<V>([&](auto v) {
                static_for<M::NM>([&](auto q) { L1[q] += uv[v] * tE1<D>(f, v, q); });
            });
            // vertex pairs v <= w in lexicographic order
            int pi = 0;
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int w = v; w < V; ++w) {
                    const double pw = uv[v] * uv[w];
#pragma unroll
                    for (int q = 0; q < M::N2; ++q) L2[q] += pw * tE2<D>(f, pi, q);
                    ++pi;
                }
            simplex_cubic_quartic<D, f>(uc, u2, u3, u4, s3, s4, sy);
            static_for<D>([&](auto d_) {
                constexpr int d = decltype(d_)::value;
                g[d] = 0.0;
                static_for<V>([&](auto v_) {
                    constexpr int v = decltype(v_)::value;
                    constexpr double gb = tBary<D>(f, v, 1 + d);
                    if constexpr (gb != 0.0) g[d] += gb * uv[v];
                });
                G[d] += vs * g[d];
            });
            double g2 = 0.0;
            static_for<D>([&](auto d) { g2 += aw[d] * g[d] * g[d]; });
            Q += vs * g2;
        });
        L3[0] += k3 * s3;
        static_for<D>([&](auto d) { L3[1 + d] += k3w * sy[d]; });
        L4 += k4 * s4;
    }
}

// Inverses of the triangular numbers i (i + 1) / 2 and the tetrahedral numbers
// i (i + 1) (i + 2) / 6, in 32-bit integers (cell ids and edge counts stay below 2^31 and
// 1625 for every admissible mesh): a single-precision estimate from the hardware square root
// or logarithm and exponential, then exact integer corrections.
__device__ inline unsigned tri_num(unsigned i) { return i * (i + 1) / 2; }
__device__ inline unsigned tet_num(unsigned i) { return i * (i + 1) * (i + 2) / 6; }
// largest i with tri_num(i) <= t: (sqrt(8 t + 1) - 1) / 2 truncated is i up to the rounding
// of the estimate, which one step down and one step up absorb
__device__ inline unsigned tri_root(unsigned t) {
    const float e = (__builtin_amdgcn_sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f;
    unsigned i = e > 0.0f ? (unsigned)e : 0u;
    i -= (i > 0 && tri_num(i) > t) ? 1u : 0u;
    i += tri_num(i + 1) <= t ? 1u : 0u;
    return i;
}
// largest i with tet_num(i) <= t: for tet_num(i) <= t < tet_num(i + 1), (6 t + 1)^(1/3) lies
// in [i + 1 - 1/(3 (i + 1)), i + 2), so its truncation is i or i + 1 (up to the rounding of
// the estimate): one step down and one step up
__device__ inline unsigned tet_root(unsigned t) {
    const float e = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(6.0f * (float)t + 1.0f) * (1.0f / 3.0f));
    unsigned i = e > 0.0f ? (unsigned)e : 0u;
    i -= (i > 0 && tet_num(i) > t) ? 1u : 0u;
    i -= (i > 0 && tet_num(i) > t) ? 1u : 0u;
    i += tet_num(i + 1) <= t ? 1u : 0u;
    return i;
}

// axes of coarse simplex type `type` (3D): type 2 p0 + q, p0 the largest coordinate's axis,
// q = 1 puts the larger remaining axis second
__device__ inline void type_axes(int type, int& p0, int& p1, int& p2) {
    p0 = type >> 1;
    const int o1 = p0 == 0 ? 1 : 0, o2 = p0 == 2 ? 1 : 2;
    p1 = (type & 1) ? o2 : o1;
    p2 = (type & 1) ? o1 : o2;
}

// coarse-local cell offset of interior cell t (strictly ordered coordinates)
template <int D>
__device__ inline void interior_cell(unsigned t, int type, int* a) {
    if (D == 2) {
        // t -> (i', j'), i' >= j' >= 0 (triangular numbers); (hi, lo) = (i' + 1, j')
        const unsigned i = tri_root(t);
        const int hi = (int)i + 1, lo = (int)(t - tri_num(i));
        a[0] = type == 0 ? hi : lo;
        a[1] = type == 0 ? lo : hi;
        a[2] = 0;
    } else {
        // t -> sorted triple i' >= j' >= k' (tetrahedral, then triangular numbers);
        // (i, j, k) = (i' + 2, j' + 1, k') is strictly decreasing
        const unsigned i = tet_root(t);
        const unsigned r = t - tet_num(i);
        const unsigned j = tri_root(r);
        const int k = (int)(r - tri_num(j));
        int p0, p1, p2;
        type_axes(type, p0, p1, p2);
        a[p0] = (int)i + 2;
        a[p1] = (int)j + 1;
        a[p2] = k;
    }
}

// coarse-local cell offset of tie cell t (s: fine cells per coarse edge)
template <int D>
__device__ inline void tie_cell(unsigned t, int type, int s, int* a) {
    if (D == 2) {
        a[0] = a[1] = (int)t;
        a[2] = 0;
    } else {
        // three groups: i = j > k (s (s - 1) / 2 cells), i > j = k (as many), i = j = k (s)
        const unsigned half = tri_num((unsigned)s - 1);
        int i, j, k;
        if (t < 2 * half) {
            const unsigned r = t < half ? t : t - half;
            const unsigned p = tri_root(r);   // p >= q >= 0 over s - 1
            const int q = (int)(r - tri_num(p));
            if (t < half) { i = j = (int)p + 1; k = q; }
            else { i = (int)p + 1; j = k = q; }
        } else {
            i = j = k = (int)(t - 2 * half);
        }
        int p0, p1, p2;
        type_axes(type, p0, p1, p2);
        a[p0] = i;
        a[p1] = j;
        a[p2] = k;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_moments_raw(const double* __restrict__ ut, Grid g, int nc, int64_t n_int,
                                                     int64_t n_tie, int c_int, int64_t k_int, int64_t k_tie, int s,
                                                     double* __restrict__ partial) {
    using R = RawLayout<D>;
    using M = Mono<D>;
    constexpr int NC = 1 << D;
    const int64_t cell = blockIdx.x;
    const int chunk = blockIdx.y;
    const int type = blockIdx.z;
    const int64_t nchunk = gridDim.y;
    const bool ties = chunk >= c_int;
    const int64_t kc = ties ? k_tie : k_int;
    const int64_t start = (int64_t)(ties ? chunk - c_int : chunk) * kc;
    const int64_t end = min(ties ? n_tie : n_int, start + kc);
    const int C[3] = {(int)(cell % nc), (int)((cell / nc) % nc), D == 3 ? (int)(cell / ((int64_t)nc * nc)) : 0};
    const int64_t P = g.pitch, S = g.plane;
    double acc[R::SIZE];
#pragma unroll
    for (int q = 0; q < R::SIZE; ++q) acc[q] = 0.0;

    // decode cell id of this block's group and load its corner values
    auto fetch = [&](int64_t id, int* aa, double* u) {
        if (ties) tie_cell<D>((unsigned)id, type, s, aa);
        else interior_cell<D>((unsigned)id, type, aa);
        // 32 x 32 -> 64-bit products (row and plane indices and strides are below 2^32)
        const int64_t base = (int64_t)(C[0] * s + aa[0]) + (int64_t)(uint32_t)(C[1] * s + aa[1]) * (uint32_t)P +
                             (D == 3 ? (int64_t)(uint32_t)(C[2] * s + aa[2]) * (uint32_t)S : 0);
#pragma unroll
        for (int c = 0; c < NC; ++c) u[c] = ut[base + (c & 1) + P * ((c >> 1) & 1) + S * ((c >> 2) & 1)];
    };
    auto process = [&](const int* a, const double* uc) {
        double L1[M::NM], L2[M::N2], L3[M::N1], L4 = 0.0, G[D], Q = 0.0;
        static_for<M::NM>([&](auto q) { L1[q] = 0.0; });
        static_for<M::N2>([&](auto q) { L2[q] = 0.0; });
        static_for<M::N1>([&](auto q) { L3[q] = 0.0; });
        static_for<D>([&](auto d) { G[d] = 0.0; });
        if (!ties)
            cell_moments<D, true>(uc, a, type, g.a, L1, L2, L3, L4, G, Q);
        else
            cell_moments<D, false>(uc, a, type, g.a, L1, L2, L3, L4, G, Q);
        const double A[3] = {(double)a[0], (double)a[1], (double)a[2]};
        shift_moments<D, M::NM>(L1, A);
        shift_moments<D, M::N2>(L2, A);
        shift_moments<D, M::N1>(L3, A);
        static_for<M::NM>([&](auto q) { acc[R::P1 + q] += L1[q]; });
        static_for<M::N2>([&](auto q) { acc[R::P2 + q] += L2[q]; });
        static_for<M::N1>([&](auto q) { acc[R::P3 + q] += L3[q]; });
        acc[R::P4] += L4;
        static_for<D>([&](auto d) { acc[R::G + d] += G[d]; });
        acc[R::Q] += Q;
    };
    for (int64_t idx = start + threadIdx.x; idx < end; idx += blockDim.x) {
        int a[3];
        double uc[NC];
        fetch(idx, a, uc);
        process(a, uc);
    }
    // block reduction (fixed order), then the scales: unit cells -> h^D, (A + Y)^b -> X^b = s^-|b|,
    // d/dY -> h d/dx
    __shared__ double red[4][R::SIZE];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < R::SIZE; ++q) {
        double v = wave_sum(acc[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    const int64_t ncell = gridDim.x;
    const double h = g.h, hd = (D == 2) ? h * h : h * h * h, inv_s = 1.0 / s;
    for (int q = threadIdx.x; q < R::SIZE; q += blockDim.x) {
        double v = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
        double sc = hd;
        int deg = 0;
        if (q < R::P2) deg = M::deg(q);
        else if (q < R::P3) deg = M::deg(q - R::P2);
        else if (q < R::P4) deg = M::deg(q - R::P3);
        for (int e = 0; e < deg; ++e) sc *= inv_s;
        if (q >= R::G && q < R::Q) sc = hd / h;
        if (q == R::Q) sc = hd / (h * h);
        partial[(((int64_t)type * ncell + cell) * nchunk + chunk) * R::SIZE + q] = v * sc;
    }
}

// ---- pass 2 ------------------------------------------------------------------------------
// Polynomials of the coarse-local coordinates are coefficient arrays over the graded
// monomial lists of layout.h (degree <= 3).  All loops below have compile-time bounds and
// indices, so the products are straight-line register code.
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
        static_for<D>([&](auto d) { kg += ph.a[d] * (lam[p][1 + d] / H) * raw[R::G + d]; });
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
                    hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int chunk_cells) {
    const ChunkShape c = chunk_shape(dim, nc, g.n, chunk_cells);
    const int sc = g.n / nc;
    const unsigned nchunk = (unsigned)(c.c_int + c.c_tie);
    if (dim == 2) {
        hipExtLaunchKernelGGL(k_moments_raw<2>, dim3((unsigned)c.ncell, nchunk, 2), dim3(256), 0, s, ev0, ev1, 0, ut, g,
                              nc, c.n_int, c.n_tie, (int)c.c_int, c.k_int, c.k_tie, sc, scratch);
        hipLaunchKernelGGL(k_moments_final<2>, dim3(cdiv(c.ncell * 2, 64)), dim3(64), 0, s, scratch, nc,
                           (int64_t)nchunk, ph, out);
    } else {
        hipExtLaunchKernelGGL(k_moments_raw<3>, dim3((unsigned)c.ncell, nchunk, 6), dim3(256), 0, s, ev0, ev1, 0, ut, g,
                              nc, c.n_int, c.n_tie, (int)c.c_int, c.k_int, c.k_tie, sc, scratch);
        hipLaunchKernelGGL(k_moments_final<3>, dim3(cdiv(c.ncell * 6, 64)), dim3(64), 0, s, scratch, nc,
                           (int64_t)nchunk, ph, out);
    }
}

}  // namespace fmg
