// The small nonlinear eigenproblems of the method, solved on the device by one wavefront:
//   * Algorithm 3.2 step 1: the ground state on the coarsest space V_{h_1};
//   * Algorithm 3.1 step 2: the augmented problem (3.6) on V_H + span{u~}.
// With u = Z x, Z = [coarse hats, u~] (or the coarse hats alone),
//     F(x, mu) = [ (A + zeta S(x)) x - mu B x ; (1 - x^T B x)/2 ] = 0,
// A = Z^T (K + M_W) Z, B = Z^T M Z, S(x) = Z^T M_{(Zx)^2} Z, is solved by Newton's method
// (the paper allows a self-consistent or a Newton-type iteration) with the Jacobian
//     [ A + 3 zeta S(x) - mu B , -B x ; -(B x)^T , 0 ].
// The coarse block of the Jacobian is banded (coarse stencils, lexicographic order); it is
// factored by a banded LDL^T without pivoting and the one or two border rows are
// eliminated through a small Schur complement.  The coarse-coarse blocks of A and B are
// the coarse stencils themselves (Galerkin identities of nested P1 spaces); everything
// involving u~ comes from the fine-grid moments (layout.h).
//
// The factorisation is the sequential part, so it is reused: a factor is kept in device
// memory between calls and Newton steps use the latest factor (chord steps) for as long as
// the residual contracts by at least a factor 4 per step; otherwise the iterate goes back
// one step and the Jacobian is refactored there.  The fixed point is unchanged.
//
// On the coarsest space the iteration starts from the discrete sine mode and raises zeta in
// geometric stages (factor 8 from a first stage <= 1, the step halved on failure).  When
// requested, the final state is checked to be the ground state by the inertia of
// A + zeta S(x) - (mu - eps) B (no negative pivot).
#include "kernels.h"
#include "layout.h"

namespace fmg {

namespace {

constexpr int kThreads = 64;   // one wavefront: barriers are cheap, reductions are shuffles

template <int D>
struct Geo {
    static constexpr int V = D + 1;
    static constexpr int NE = (D == 2) ? 2 : 6;
    static constexpr int NS = (D == 2) ? kStencil2D : kStencil3D;
    static constexpr int NSTAR = (D == 2) ? 6 : 24;
};

template <int D>
__device__ inline int slot_of(const int* o) {
    for (int s = 0; s < Geo<D>::NS; ++s) {
        bool eq = true;
        for (int d = 0; d < D; ++d) eq = eq && ((D == 2 ? kOff2D[s][d] : kOff3D[s][d]) == o[d]);
        if (eq) return s;
    }
    return -1;
}

template <int D>
__device__ inline int cell_vert(int t, int v, int d) {
    return D == 2 ? kCellElemVert2D[t][v][d] : kCellElemVert3D[t][v][d];
}

struct Args {
    int nc;
    Phys ph;
    int max_iter;
    double tol;
    const double* mom;
    double* arena;       // global arena (used when the problem does not fit in LDS)
    int use_lds;
    double* xc;          // coarsest padded level array receiving x_H
    Grid gc;
    SmallState* st;
    int final_level;     // tolerance checks enabled for this step
    int certify;         // run the ground-state inertia check
    double* fac;         // persistent band factor (N*(w+1) doubles), may be null
    int reuse;           // start from the stored factor when it exists
    // dump mode
    const double* xin;
    double* Aout;
    double* Bout;
    double* Sout;
};

struct Sizes {
    int m, N, w, N1, np, nel;
};

template <int D, bool AUG>
__host__ __device__ inline Sizes sizes(int nc) {
    Sizes z;
    z.m = nc - 1;
    z.N = (D == 2) ? z.m * z.m : z.m * z.m * z.m;
    z.w = (D == 2) ? z.m + 1 : z.m * z.m + z.m + 1;
    if (z.w > z.N - 1) z.w = z.N > 1 ? z.N - 1 : 1;
    z.N1 = AUG ? z.N + 1 : z.N;
    z.np = z.w * (z.w + 1) / 2;
    z.nel = ((D == 2) ? nc * nc : nc * nc * nc) * Geo<D>::NE;
    return z;
}

template <int D, bool AUG>
struct Arena {
    Sizes z;
    double* Ast; double* Bst; double* Sst; double* band;
    double* x; double* xs; double* xk; double* y; double* z2; double* F; double* rhs;
    double* aH; double* bH; double* sH; double* sc; double* I4t;
    int* nb; int* star; int* enode; int* qslot; int* pairs;

    __device__ void carve(double* base, int nc) {
        z = sizes<D, AUG>(nc);
        constexpr int NS = Geo<D>::NS;
        constexpr int V = D + 1;
        const int N = z.N;
        double* p = base;
        Ast = p; p += (size_t)N * NS;
        Bst = p; p += (size_t)N * NS;
        Sst = p; p += (size_t)N * NS;
        band = p; p += (size_t)N * (z.w + 1);
        x = p; p += N + 2;
        xs = p; p += N + 2;
        xk = p; p += N + 2;
        y = p; p += N + 2;
        z2 = p; p += N + 2;
        F = p; p += N + 2;
        rhs = p; p += 3 * (size_t)N;
        aH = p; p += N;
        bH = p; p += N;
        sH = p; p += N;
        sc = p; p += 32;
        I4t = p; p += V * V * V * V;
        int* q = reinterpret_cast<int*>(p);
        nb = q; q += N * NS;
        star = q; q += N * Geo<D>::NSTAR;
        enode = q; q += z.nel * V;
        qslot = q; q += Geo<D>::NE * V * V;
        pairs = q;
    }
};

template <int D, bool AUG>
__host__ __device__ inline size_t arena_bytes_t(int nc) {
    Sizes z = sizes<D, AUG>(nc);
    constexpr int NS = Geo<D>::NS;
    constexpr int V = D + 1;
    size_t N = z.N;
    size_t dbl = 3 * N * NS + N * (z.w + 1) + 6 * (N + 2) + 3 * N + 3 * N + 32 + V * V * V * V;
    size_t ints = N * NS + N * Geo<D>::NSTAR + (size_t)z.nel * V + Geo<D>::NE * V * V + z.np;
    return dbl * sizeof(double) + ints * sizeof(int) + 64;
}

__device__ inline double wsum(double v) { return wave_sum(v); }

template <int D>
__device__ inline void node_pos(int a, int m, int* P) {
    P[0] = a % m + 1;
    P[1] = (a / m) % m + 1;
    P[2] = (D == 3) ? a / (m * m) + 1 : 0;
}

template <int D>
__device__ inline int node_id(const int* P, int m) {
    for (int d = 0; d < D; ++d)
        if (P[d] < 1 || P[d] > m) return -1;
    return (D == 2) ? (P[0] - 1) + m * (P[1] - 1) : (P[0] - 1) + m * ((P[1] - 1) + m * (P[2] - 1));
}

// ---------------------------------------------------------------------------------------
// setup: tables, coarse stencils of K + M_W and M, and the u~ border
template <int D, bool AUG>
__device__ void setup(Arena<D, AUG>& ar, const Args& a) {
    constexpr int NS = Geo<D>::NS;
    constexpr int NE = Geo<D>::NE;
    constexpr int V = D + 1;
    constexpr int NSTAR = Geo<D>::NSTAR;
    using L = MomLayout<D>;
    const int N = ar.z.N, m = ar.z.m, nc = a.nc;
    const double H = 1.0 / nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
    const int lane = threadIdx.x;
    // element vertex -> node table
    for (int e = lane; e < ar.z.nel; e += kThreads) {
        const int cl = e / NE, t = e % NE;
        int C[3] = {cl % nc, (cl / nc) % nc, D == 3 ? cl / (nc * nc) : 0};
        for (int v = 0; v < V; ++v) {
            int Q[3] = {0, 0, 0};
            for (int d = 0; d < D; ++d) Q[d] = C[d] + cell_vert<D>(t, v, d);
            ar.enode[e * V + v] = node_id<D>(Q, m);
        }
    }
    // stencil slot of vertex q seen from vertex va of a simplex of type t
    for (int k = lane; k < NE * V * V; k += kThreads) {
        const int t = k / (V * V), va = (k / V) % V, q = k % V;
        int o[3] = {0, 0, 0};
        for (int d = 0; d < D; ++d) o[d] = cell_vert<D>(t, q, d) - cell_vert<D>(t, va, d);
        ar.qslot[k] = slot_of<D>(o);
    }
    // LDL^T update pairs (ii >= jj) of the trailing window, ordered by ii
    for (int p = lane; p < ar.z.np; p += kThreads) {
        int ii = 0;
        while ((ii + 1) * (ii + 2) / 2 <= p) ++ii;
        const int jj = p - ii * (ii + 1) / 2;
        ar.pairs[p] = (ii << 16) | jj;
    }
    for (int i = lane; i < N; i += kThreads) {
        int P[3];
        node_pos<D>(i, m, P);
        double X[3] = {P[0] * H, P[1] * H, P[2] * H};
        for (int s = 0; s < NS; ++s) {
            int Q[3], o1 = 0;
            for (int d = 0; d < 3; ++d) Q[d] = P[d];
            for (int d = 0; d < D; ++d) {
                int od = (D == 2 ? kOff2D[s][d] : kOff3D[s][d]);
                Q[d] += od;
                o1 += od < 0 ? -od : od;
            }
            int j = node_id<D>(Q, m);
            ar.nb[i * NS + s] = j;
            double m0 = (D == 2) ? kM0_2D[s] : kM0_3D[s];
            double cw = a.ph.wc * m0;
            for (int k = 0; k < D; ++k) {
                double m1 = (D == 2) ? kM1_2D[k][s] : kM1_3D[k][s];
                double m2 = (D == 2) ? kM2_2D[k][s] : kM2_3D[k][s];
                cw += a.ph.w[k] * (X[k] * X[k] * m0 + 2.0 * X[k] * H * m1 + H * H * m2);
            }
            double kk;
            if (D == 2)
                kk = (o1 == 0) ? 4.0 : (o1 == 1 ? -1.0 : 0.0);
            else
                kk = (o1 == 0) ? 6.0 * H : (o1 == 1 ? -H : 0.0);
            ar.Ast[i * NS + s] = (j >= 0) ? kk + Hd * cw : 0.0;
            ar.Bst[i * NS + s] = (j >= 0) ? Hd * m0 : 0.0;
        }
        // the simplices around node i
        int cnt = 0;
        for (int cc = 0; cc < (1 << D); ++cc) {
            int C[3] = {P[0] - ((cc >> 0) & 1), P[1] - ((cc >> 1) & 1), D == 3 ? P[2] - ((cc >> 2) & 1) : 0};
            int cl = (D == 2) ? C[0] + nc * C[1] : C[0] + nc * (C[1] + nc * C[2]);
            for (int t = 0; t < NE; ++t)
                for (int v = 0; v < V; ++v) {
                    bool hit = true;
                    for (int d = 0; d < D; ++d) hit = hit && (C[d] + cell_vert<D>(t, v, d) == P[d]);
                    if (hit && cnt < NSTAR) ar.star[i * NSTAR + cnt++] = (cl * NE + t) * V + v;
                }
        }
        if (AUG) {
            double ah = 0.0, bh = 0.0;
            for (int s = 0; s < NSTAR; ++s) {
                const int pk = ar.star[i * NSTAR + s];
                const int e = pk / V, va = pk % V;
                const double* mo = a.mom + (size_t)e * L::SIZE;
                ah += mo[L::KG + va] + mo[L::AW1 + va];
                bh += mo[L::B1 + va];
            }
            ar.aH[i] = ah;
            ar.bH[i] = bh;
        }
    }
    if (AUG) {
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
        for (int e = lane; e < ar.z.nel; e += kThreads) {
            const double* mo = a.mom + (size_t)e * L::SIZE;
            v0 += mo[L::Q] + mo[L::AW2];
            v1 += mo[L::B2];
            double s = 0.0;
            for (int p = 0; p < V; ++p) s += mo[L::B1 + p];
            v2 += s;
        }
        v0 = wsum(v0); v1 = wsum(v1); v2 = wsum(v2);
        if (lane == 0) {
            ar.sc[0] = v0;  // aU
            ar.sc[1] = v1;  // bU
            ar.sc[2] = v2;  // int u~
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------------
// int l_p l_r l_a l_b / |E| = D! alpha! / (D+4)!  (compile-time for constant arguments)
__host__ __device__ constexpr double i4e(int p, int r, int a, int b, int D) {
    int v[4] = {p, r, a, b};
    double num = (D == 2) ? 2.0 : 6.0;
    for (int val = 0; val < 4; ++val) {
        int c = 0;
        for (int y = 0; y < 4; ++y) c += (v[y] == val) ? 1 : 0;
        for (int f = 2; f <= c; ++f) num *= f;
    }
    return num / ((D == 2) ? 720.0 : 5040.0);
}

// contributions of one simplex to row `va` of S(x) and to the border entry
template <int D, bool AUG, int VA>
__device__ inline void elem_row(const double* U, const double* mo, double c, double vol, const int* qs, double* srow,
                                double& sh) {
    constexpr int V = D + 1;
    using L = MomLayout<D>;
#pragma unroll
    for (int q = 0; q < V; ++q) {
        double val = 0.0;
#pragma unroll
        for (int p = 0; p < V; ++p)
#pragma unroll
            for (int r = 0; r < V; ++r) val += U[p] * U[r] * i4e(p, r, VA, q, D);
        val *= vol;
        if (AUG) {
            double t3 = 0.0;
#pragma unroll
            for (int p = 0; p < V; ++p) t3 += U[p] * mo[L::T3 + sym3(p, VA, q, V)];
            val += 2.0 * c * t3 + c * c * mo[L::T2 + sym2(VA, q, V)];
        }
        srow[qs[q]] += val;
    }
    if (AUG) {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int p = 0; p < V; ++p) {
#pragma unroll
            for (int r = 0; r < V; ++r) s1 += U[p] * U[r] * mo[L::T3 + sym3(p, r, VA, V)];
            s2 += U[p] * mo[L::T2 + sym2(p, VA, V)];
        }
        sh += s1 + 2.0 * c * s2 + c * c * mo[L::T1 + VA];
    }
}

// S(x): coarse stencil Sst, border sH, corner sc[3]
template <int D, bool AUG>
__device__ void assemble_S(Arena<D, AUG>& ar, const Args& a, const double* x) {
    constexpr int NS = Geo<D>::NS;
    constexpr int NE = Geo<D>::NE;
    constexpr int V = D + 1;
    constexpr int NSTAR = Geo<D>::NSTAR;
    using L = MomLayout<D>;
    const int N = ar.z.N, nc = a.nc;
    const double H = 1.0 / nc;
    const double vol = (D == 2) ? 0.5 * H * H : H * H * H / 6.0;
    const double c = AUG ? x[N] : 0.0;
    const int lane = threadIdx.x;
    for (int i = lane; i < N; i += kThreads) {
        double srow[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) srow[s] = 0.0;
        double sh = 0.0;
        for (int s = 0; s < NSTAR; ++s) {
            const int pk = ar.star[i * NSTAR + s];
            const int e = pk / V, va = pk % V, t = e % NE;
            double U[V];
            int qs[V];
#pragma unroll
            for (int p = 0; p < V; ++p) {
                const int j = ar.enode[e * V + p];
                U[p] = (j >= 0) ? x[j] : 0.0;
                qs[p] = ar.qslot[(t * V + va) * V + p];
            }
            const double* mo = AUG ? a.mom + (size_t)e * L::SIZE : nullptr;
            switch (va) {
                case 0: elem_row<D, AUG, 0>(U, mo, c, vol, qs, srow, sh); break;
                case 1: elem_row<D, AUG, 1>(U, mo, c, vol, qs, srow, sh); break;
                case 2: elem_row<D, AUG, 2>(U, mo, c, vol, qs, srow, sh); break;
                default: if (D == 3) elem_row<D, AUG, (D == 3 ? 3 : 2)>(U, mo, c, vol, qs, srow, sh); break;
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) ar.Sst[(size_t)i * NS + s] = (ar.nb[i * NS + s] >= 0) ? srow[s] : 0.0;
        if (AUG) ar.sH[i] = sh;
    }
    if (AUG) {
        double v = 0.0;
        for (int e = lane; e < ar.z.nel; e += kThreads) {
            double U[V];
#pragma unroll
            for (int p = 0; p < V; ++p) {
                const int j = ar.enode[e * V + p];
                U[p] = (j >= 0) ? x[j] : 0.0;
            }
            const double* mo = a.mom + (size_t)e * L::SIZE;
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int p = 0; p < V; ++p) {
#pragma unroll
                for (int r = 0; r < V; ++r) s1 += U[p] * U[r] * mo[L::T2 + sym2(p, r, V)];
                s2 += U[p] * mo[L::T1 + p];
            }
            v += s1 + 2.0 * c * s2 + c * c * mo[L::T0];
        }
        v = wsum(v);
        if (lane == 0) ar.sc[3] = v;  // sU
    }
    __syncthreads();
}

// y = (A + zs S) x, z = B x (with borders); sc[4] = x^T y, sc[5] = x^T z
template <int D, bool AUG>
__device__ void apply(Arena<D, AUG>& ar, double zs, const double* x, double* y, double* z) {
    constexpr int NS = Geo<D>::NS;
    const int N = ar.z.N;
    const double c = AUG ? x[N] : 0.0;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    for (int i = threadIdx.x; i < N; i += kThreads) {
        double yi = 0.0, zi = 0.0;
        for (int s = 0; s < NS; ++s) {
            int j = ar.nb[i * NS + s];
            if (j < 0) continue;
            yi += (ar.Ast[i * NS + s] + zs * ar.Sst[i * NS + s]) * x[j];
            zi += ar.Bst[i * NS + s] * x[j];
        }
        if (AUG) {
            const double g = ar.aH[i] + zs * ar.sH[i];
            yi += g * c;
            zi += ar.bH[i] * c;
            v2 += g * x[i];
            v3 += ar.bH[i] * x[i];
        }
        y[i] = yi;
        z[i] = zi;
        v0 += x[i] * yi;
        v1 += x[i] * zi;
    }
    v0 = wsum(v0); v1 = wsum(v1);
    if (AUG) { v2 = wsum(v2); v3 = wsum(v3); }
    if (threadIdx.x == 0) {
        if (AUG) {
            const double yU = v2 + (ar.sc[0] + zs * ar.sc[3]) * c;
            const double zU = v3 + ar.sc[1] * c;
            y[N] = yU;
            z[N] = zU;
            v0 += c * yU;
            v1 += c * zU;
        }
        ar.sc[4] = v0;
        ar.sc[5] = v1;
    }
    __syncthreads();
}

// band <- Ast + alpha Sst - sigma Bst   (lower band, row-major, band[i*(w+1)+k] = J(i,i-k))
template <int D, bool AUG>
__device__ void fill_band(Arena<D, AUG>& ar, double alpha, double sigma) {
    constexpr int NS = Geo<D>::NS;
    const int N = ar.z.N, W1 = ar.z.w + 1;
    for (int t = threadIdx.x; t < N * W1; t += kThreads) ar.band[t] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += kThreads)
        for (int s = 0; s < NS; ++s) {
            int j = ar.nb[i * NS + s];
            if (j < 0 || j > i) continue;
            ar.band[(size_t)i * W1 + (i - j)] =
                ar.Ast[i * NS + s] + alpha * ar.Sst[i * NS + s] - sigma * ar.Bst[i * NS + s];
        }
    __syncthreads();
}

// In-place banded LDL^T without pivoting; afterwards band[i][0] = d_i and band[i][t] =
// l_{i,i-t}.  Returns the number of negative pivots, or -1 for a (numerically) zero pivot.
template <int D, bool AUG>
__device__ int ldlt(Arena<D, AUG>& ar) {
    const int N = ar.z.N, w = ar.z.w, W1 = w + 1;
    double* b = ar.band;
    double scale = 0.0;
    for (int i = threadIdx.x; i < N; i += kThreads) scale = fmax(scale, fabs(b[(size_t)i * W1]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) scale = fmax(scale, __shfl_xor(scale, off, 64));
    int neg = 0;
    for (int k = 0; k < N; ++k) {
        const double d = b[(size_t)k * W1];
        if (!(fabs(d) > 1e-15 * scale)) return -1;
        if (d < 0.0) ++neg;
        const double inv = 1.0 / d;
        const int r = min(w, N - 1 - k);
        const int np = r * (r + 1) / 2;   // the pairs with ii < r come first
        for (int p = threadIdx.x; p < np; p += kThreads) {
            const int pk = ar.pairs[p];
            const int ii = pk >> 16, jj = pk & 0xffff;
            const int i = k + 1 + ii, j = k + 1 + jj;
            b[(size_t)i * W1 + (ii - jj)] -= b[(size_t)i * W1 + (ii + 1)] * b[(size_t)j * W1 + (jj + 1)] * inv;
        }
        __syncthreads();
    }
    // scale the columns: l_{i,k} = a_{i,k} / d_k
    for (int t = threadIdx.x; t < N * W1; t += kThreads) {
        const int i = t / W1, q = t - i * W1;
        if (q > 0 && i - q >= 0) b[t] /= b[(size_t)(i - q) * W1];
    }
    __syncthreads();
    return neg;
}

__device__ inline double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Solve (L D L^T) X = R for R right-hand sides stored as rhs[q*N + i].  Row i lives in
// lane i % 64, register slot i / 64; the value of the eliminated row is broadcast with
// readlane, so the dependency chain never goes through memory.  Needs N <= 64*SMAX and a
// band half-width w <= 128 (otherwise the LDS variant below is used).
constexpr int SMAX = 16;

template <int R>
__device__ void band_solve_reg(const double* __restrict__ b, int N, int w, double* rhs) {
    const int W1 = w + 1;
    const int lane = threadIdx.x;
    const int S = (N + 63) >> 6;
    double y[R][SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        const int i = 64 * s + lane;
#pragma unroll
        for (int q = 0; q < R; ++q) y[q][s] = (s < S && i < N) ? rhs[q * N + i] : 0.0;
    }
    // forward: unit lower L
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        if (s < S) {
            for (int kk = 0; kk < 64; ++kk) {
                const int k = 64 * s + kk;
                if (k >= N) break;
                double yk[R];
#pragma unroll
                for (int q = 0; q < R; ++q) yk[q] = readlane_d(y[q][s], kk);
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    if (s + o < SMAX) {
                        const int i = 64 * (s + o) + lane;
                        if (i > k && i <= k + w && i < N) {
                            const double l = b[(size_t)i * W1 + (i - k)];
#pragma unroll
                            for (int q = 0; q < R; ++q) y[q][s + o] -= l * yk[q];
                        }
                    }
                }
            }
        }
    }
    // diagonal
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        const int i = 64 * s + lane;
        if (s < S && i < N) {
            const double inv = 1.0 / b[(size_t)i * W1];
#pragma unroll
            for (int q = 0; q < R; ++q) y[q][s] *= inv;
        }
    }
    // backward: unit upper L^T
#pragma unroll
    for (int s = SMAX - 1; s >= 0; --s) {
        if (s < S) {
            for (int kk = 63; kk >= 0; --kk) {
                const int k = 64 * s + kk;
                if (k >= N) continue;
                double xk[R];
#pragma unroll
                for (int q = 0; q < R; ++q) xk[q] = readlane_d(y[q][s], kk);
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    if (s - o >= 0) {
                        const int j = 64 * (s - o) + lane;
                        if (j < k && j >= k - w) {
                            const double l = b[(size_t)k * W1 + (k - j)];
#pragma unroll
                            for (int q = 0; q < R; ++q) y[q][s - o] -= l * xk[q];
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        const int i = 64 * s + lane;
        if (s < S && i < N) {
#pragma unroll
            for (int q = 0; q < R; ++q) rhs[q * N + i] = y[q][s];
        }
    }
    __syncthreads();
}

// LDS variant for large problems (one barrier per elimination step)
template <int D, bool AUG>
__device__ void ldlt_solve_lds(Arena<D, AUG>& ar, double* rhs, int R) {
    const int N = ar.z.N, w = ar.z.w, W1 = w + 1;
    const double* b = ar.band;
    for (int k = 0; k < N; ++k) {
        const int r = min(w, N - 1 - k);
        for (int t = threadIdx.x; t < r * R; t += kThreads) {
            const int q = t / r, ii = t - q * r;
            const int i = k + 1 + ii;
            rhs[q * N + i] -= b[(size_t)i * W1 + (ii + 1)] * rhs[q * N + k];
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < N * R; t += kThreads) {
        const int i = t % N;
        rhs[t] /= b[(size_t)i * W1];
    }
    __syncthreads();
    for (int k = N - 1; k >= 0; --k) {
        const int r = min(w, k);
        for (int t = threadIdx.x; t < r * R; t += kThreads) {
            const int q = t / r, ii = t - q * r;
            const int i = k - 1 - ii;
            rhs[q * N + i] -= b[(size_t)k * W1 + (ii + 1)] * rhs[q * N + k];
        }
        __syncthreads();
    }
}

template <int D, bool AUG>
__device__ void ldlt_solve(Arena<D, AUG>& ar, double* rhs, int R) {
    const int N = ar.z.N, w = ar.z.w;
    __syncthreads();
    if (N <= 64 * SMAX && w <= 128) {
        if (R == 1) band_solve_reg<1>(ar.band, N, w, rhs);
        else if (R == 2) band_solve_reg<2>(ar.band, N, w, rhs);
        else band_solve_reg<3>(ar.band, N, w, rhs);
    } else {
        ldlt_solve_lds<D, AUG>(ar, rhs, R);
    }
}

// One Newton solve at coupling zs from the iterate in ar.x, using (and refreshing) the
// factor in ar.band.  `have` says whether band already holds a usable factor.  Returns
// iterations >= 0 on convergence, or -reason.  mu in sc[6], factorisations added to sc[8].
template <int D, bool AUG>
__device__ int newton(Arena<D, AUG>& ar, const Args& a, double zs, bool& have) {
    const int N = ar.z.N, N1 = ar.z.N1;
    const int lane = threadIdx.x;
    {
        // x <- x / ||x||_B  (B needs no assembly)
        constexpr int NS = Geo<D>::NS;
        double v = 0.0, vb = 0.0;
        const double c = AUG ? ar.x[N] : 0.0;
        for (int i = lane; i < N; i += kThreads) {
            double zi = 0.0;
            for (int s = 0; s < NS; ++s) {
                const int j = ar.nb[i * NS + s];
                if (j >= 0) zi += ar.Bst[i * NS + s] * ar.x[j];
            }
            v += ar.x[i] * zi;
            if (AUG) vb += ar.bH[i] * ar.x[i];
        }
        v = wsum(v);
        if (AUG) vb = wsum(vb);
        const double xbx = v + (AUG ? c * (2.0 * vb + ar.sc[1] * c) : 0.0);
        const double sN = 1.0 / sqrt(xbx);
        __syncthreads();
        for (int i = lane; i < N1; i += kThreads) ar.x[i] *= sN;
        __syncthreads();
    }
    double mu = 0.0, mus = 0.0, res_prev = 1e300;
    bool last_fresh = false, need_fresh = !have;
    for (int it = 0; it <= a.max_iter; ++it) {
        assemble_S<D, AUG>(ar, a, ar.x);
        apply<D, AUG>(ar, zs, ar.x, ar.y, ar.z2);
        if (it == 0) mu = ar.sc[4] / ar.sc[5];
        const double F2 = 0.5 * (1.0 - ar.sc[5]);
        double f2 = 0.0, zz = 0.0;
        for (int i = lane; i < N1; i += kThreads) {
            const double f = ar.y[i] - mu * ar.z2[i];
            ar.F[i] = f;
            f2 += f * f;
            zz += ar.z2[i] * ar.z2[i];
        }
        f2 = wsum(f2);
        zz = wsum(zz);
        const double res = sqrt(f2) / (fabs(mu) * sqrt(zz));
        if (lane == 0) ar.sc[7] = res;
        if (!(res == res) || !(mu == mu)) return -3;
        // x^T B x = 1 up to the rounding of an N-term dot product
        if (res <= a.tol && fabs(F2) <= 4.0 * N1 * 1.1e-16) {
            const double sN = 1.0 / sqrt(ar.sc[5]);
            for (int i = lane; i < N1; i += kThreads) ar.x[i] *= sN;
            if (lane == 0) ar.sc[6] = mu;
            __syncthreads();
            return it;
        }
        if (it == a.max_iter) return -2;
        if (it > 0 && !last_fresh && res > 0.25 * res_prev) {
            // the stale Jacobian stopped contracting: back to the previous iterate, refactor
            for (int i = lane; i < N1; i += kThreads) ar.x[i] = ar.xs[i];
            mu = mus;
            need_fresh = true;
            res_prev = 1e300;
            __syncthreads();
            continue;
        }
        if (need_fresh) {
            fill_band<D, AUG>(ar, 3.0 * zs, mu);
            if (ldlt<D, AUG>(ar) < 0) return -1;
            need_fresh = false;
            last_fresh = true;
            have = true;
            if (lane == 0) ar.sc[8] += 1.0;
        } else {
            last_fresh = false;
        }
        for (int i = lane; i < N1; i += kThreads) ar.xs[i] = ar.x[i];
        mus = mu;
        res_prev = res;
        const int R = AUG ? 3 : 2;
        for (int i = lane; i < N; i += kThreads) {
            ar.rhs[i] = -ar.F[i];
            if (AUG) {
                ar.rhs[N + i] = ar.aH[i] + 3.0 * zs * ar.sH[i] - mu * ar.bH[i];
                ar.rhs[2 * N + i] = -ar.z2[i];
            } else {
                ar.rhs[N + i] = -ar.z2[i];
            }
        }
        __syncthreads();
        ldlt_solve<D, AUG>(ar, ar.rhs, R);
        double dmu, dc = 0.0;
        if (AUG) {
            double s[6] = {0, 0, 0, 0, 0, 0};
            for (int i = lane; i < N; i += kThreads) {
                const double jh = ar.aH[i] + 3.0 * zs * ar.sH[i] - mu * ar.bH[i];
                const double zh = ar.z2[i];
                s[0] += jh * ar.rhs[i];
                s[1] += jh * ar.rhs[N + i];
                s[2] += jh * ar.rhs[2 * N + i];
                s[3] += zh * ar.rhs[i];
                s[4] += zh * ar.rhs[N + i];
                s[5] += zh * ar.rhs[2 * N + i];
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) s[q] = wsum(s[q]);
            const double jU = ar.sc[0] + 3.0 * zs * ar.sc[3] - mu * ar.sc[1];
            const double zU = ar.z2[N];
            const double a11 = jU - s[1], a12 = -s[2] - zU, r1 = -ar.F[N] - s[0];
            const double a21 = s[4] - zU, a22 = s[5], r2 = -F2 + s[3];
            const double det = a11 * a22 - a12 * a21;
            if (!(fabs(det) > 0.0)) return -4;
            dc = (r1 * a22 - a12 * r2) / det;
            dmu = (a11 * r2 - a21 * r1) / det;
            for (int i = lane; i < N; i += kThreads)
                ar.x[i] += ar.rhs[i] - ar.rhs[N + i] * dc - ar.rhs[2 * N + i] * dmu;
            if (lane == 0) ar.x[N] += dc;
        } else {
            double s0 = 0.0, s1 = 0.0;
            for (int i = lane; i < N; i += kThreads) {
                s0 += ar.z2[i] * ar.rhs[i];
                s1 += ar.z2[i] * ar.rhs[N + i];
            }
            s0 = wsum(s0);
            s1 = wsum(s1);
            if (!(fabs(s1) > 0.0)) return -4;
            dmu = (-F2 + s0) / s1;
            for (int i = lane; i < N; i += kThreads) ar.x[i] += ar.rhs[i] - ar.rhs[N + i] * dmu;
        }
        mu += dmu;
        __syncthreads();
    }
    return -2;
}

// inertia check: number of eigenvalues of (A + zs S(x), B) below sigma (0: ground state)
template <int D, bool AUG>
__device__ int count_below(Arena<D, AUG>& ar, double zs, double sigma) {
    const int N = ar.z.N;
    fill_band<D, AUG>(ar, zs, sigma);
    int neg = ldlt<D, AUG>(ar);
    if (neg < 0) return 1;
    if (AUG) {
        for (int i = threadIdx.x; i < N; i += kThreads) ar.rhs[i] = ar.aH[i] + zs * ar.sH[i] - sigma * ar.bH[i];
        __syncthreads();
        ldlt_solve<D, AUG>(ar, ar.rhs, 1);
        double s = 0.0;
        for (int i = threadIdx.x; i < N; i += kThreads) s += (ar.aH[i] + zs * ar.sH[i] - sigma * ar.bH[i]) * ar.rhs[i];
        s = wsum(s);
        const double schur = (ar.sc[0] + zs * ar.sc[3] - sigma * ar.sc[1]) - s;
        if (!(schur > 0.0)) ++neg;
    }
    return neg;
}

template <int D, bool AUG>
__device__ void store_factor(Arena<D, AUG>& ar, const Args& a) {
    if (!a.fac) return;
    const int n = ar.z.N * (ar.z.w + 1);
    for (int t = threadIdx.x; t < n; t += kThreads) a.fac[t] = ar.band[t];
    if (threadIdx.x == 0) a.st->fac_valid = 1;
}

template <int D, bool AUG>
__device__ void finish(Arena<D, AUG>& ar, const Args& a, int iters, bool ok, int reason) {
    const int N = ar.z.N, m = ar.z.m;
    const double H = 1.0 / a.nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
    if (ok) {
        const double mu = ar.sc[6];
        int below = 0;
        if (a.certify) below = count_below<D, AUG>(ar, a.ph.zeta, mu - 1e-9 * fabs(mu));
        // sign: int u_h > 0
        double v = 0.0;
        for (int i = threadIdx.x; i < N; i += kThreads) v += ar.x[i];
        v = wsum(v);
        const double integ = Hd * v + (AUG ? ar.x[N] * ar.sc[2] : 0.0);
        const double sgn = integ < 0.0 ? -1.0 : 1.0;
        for (int i = threadIdx.x; i < N; i += kThreads) {
            int P[3];
            node_pos<D>(i, m, P);
            a.xc[P[0] + a.gc.pitch * P[1] + a.gc.plane * P[2]] = sgn * ar.x[i];
        }
        if (threadIdx.x == 0) {
            SmallState* st = a.st;
            const double prev = st->lambda;
            st->lambda_prev = prev;
            st->lambda = mu;
            st->dlambda = fabs(mu - prev) / fabs(mu);
            st->c = AUG ? sgn * ar.x[N] : 0.0;
            st->newton_total += iters;
            st->fact_total += (int)ar.sc[8] + (a.certify ? 1 : 0);
            if (st->hist_len < 512) st->hist[st->hist_len] = mu;
            st->hist_len += 1;
            st->steps += AUG ? 1 : 0;
            if (below != 0) {
                st->certify_fail += 1;
                if (!st->fail_reason) {
                    st->fail_reason = 5;
                    st->fail_step = st->hist_len - 1;
                    st->fail_residual = ar.sc[7];
                }
            }
            if (AUG && a.final_level && st->tol_lambda > 0.0 && st->dlambda <= st->tol_lambda) st->done = 1;
        }
    } else {
        // keep u = u~ (c = 1, x_H = 0) so later kernels stay finite; report the failure
        for (int i = threadIdx.x; i < N; i += kThreads) {
            int P[3];
            node_pos<D>(i, m, P);
            a.xc[P[0] + a.gc.pitch * P[1] + a.gc.plane * P[2]] = 0.0;
        }
        if (threadIdx.x == 0) {
            a.st->c = 1.0;
            a.st->fac_valid = 0;
            if (a.st->status == 0) {
                a.st->status = (reason == 3) ? FMG_ENONFINITE : FMG_ENOCONV;
                a.st->fail_reason = reason;
                a.st->fail_step = a.st->hist_len;
                a.st->fail_residual = ar.sc[7];
            }
        }
    }
}

template <int D, bool AUG>
__global__ __launch_bounds__(kThreads) void k_newton(Args a) {
    extern __shared__ double lds[];
    Arena<D, AUG> ar;
    ar.carve(a.use_lds ? lds : a.arena, a.nc);
    if (AUG && a.st->done) return;   // tolerance loop already satisfied
    setup<D, AUG>(ar, a);
    const int N = ar.z.N, m = ar.z.m;
    const int lane = threadIdx.x;
    if (lane == 0) ar.sc[8] = 0.0;
    // a stored factor of the coarse Jacobian block (previous call) seeds chord steps
    bool have = false;
    if (a.reuse && a.fac && a.st->fac_valid) {
        const int n = N * (ar.z.w + 1);
        for (int t = lane; t < n; t += kThreads) ar.band[t] = a.fac[t];
        have = true;
    }
    __syncthreads();
    int iters = 0;
    bool ok = true;
    int reason = 0;
    if (AUG) {
        // start from u = u~ / ||u~||_M
        for (int i = lane; i < N; i += kThreads) ar.x[i] = 0.0;
        if (lane == 0) ar.x[N] = 1.0;
        __syncthreads();
        int r = newton<D, AUG>(ar, a, a.ph.zeta, have);
        ok = r >= 0;
        iters = ok ? r : 0;
        reason = ok ? 0 : -r;
    } else {
        // discrete sine mode, then zeta stages (first stage <= 1, factor 8)
        const double H = 1.0 / a.nc;
        for (int i = lane; i < N; i += kThreads) {
            int P[3];
            node_pos<D>(i, m, P);
            double v = sinpi(P[0] * H) * sinpi(P[1] * H);
            if (D == 3) v *= sinpi(P[2] * H);
            ar.x[i] = v;
        }
        __syncthreads();
        const double zeta = a.ph.zeta;
        if (zeta <= 1.0) {
            int r = newton<D, AUG>(ar, a, zeta, have);
            ok = r >= 0;
            iters = ok ? r : 0;
            reason = ok ? 0 : -r;
        } else {
            const double lf = log(8.0);
            const double lt = log(zeta);
            int J = (int)ceil(lt / lf - 1e-12);
            double lnext = lt - J * lf, step = lf, lcur = 0.0;
            bool have_cur = false;
            int first_tries = 0;
            for (int guard = 0; guard < 200; ++guard) {
                const bool last = !(lnext < lt);
                const double z = last ? zeta : exp(lnext);
                for (int i = lane; i < N; i += kThreads) ar.xk[i] = ar.x[i];   // committed iterate
                __syncthreads();
                int rr = newton<D, AUG>(ar, a, z, have);
                if (rr < 0) {
                    for (int i = lane; i < N; i += kThreads) ar.x[i] = ar.xk[i];
                    have = false;
                    __syncthreads();
                    if (!have_cur) {
                        // first stage failed from the sine mode: start lower
                        if (++first_tries > 4) { ok = false; reason = -rr; break; }
                        lnext -= lf;
                        continue;
                    }
                    step *= 0.5;
                    if (step < 1e-3) { ok = false; reason = -rr; break; }
                    lnext = lcur + step;
                    continue;
                }
                iters += rr;
                if (last) break;
                lcur = lnext;
                have_cur = true;
                lnext = fmin(lt, lcur + step);
            }
        }
    }
    __syncthreads();
    if (ok && ar.sc[8] > 0.0) store_factor<D, AUG>(ar, a);
    __syncthreads();
    finish<D, AUG>(ar, a, iters, ok, reason);
}

// dense A, B, S(x) of the augmented problem (tests)
template <int D>
__global__ __launch_bounds__(kThreads) void k_aug_dump(Args a) {
    extern __shared__ double lds[];
    Arena<D, true> ar;
    ar.carve(a.use_lds ? lds : a.arena, a.nc);
    setup<D, true>(ar, a);
    constexpr int NS = Geo<D>::NS;
    const int N = ar.z.N, N1 = N + 1;
    for (int i = threadIdx.x; i < N1; i += kThreads) ar.x[i] = a.xin[i];
    __syncthreads();
    assemble_S<D, true>(ar, a, ar.x);
    for (int t = threadIdx.x; t < N1 * N1; t += kThreads) {
        a.Aout[t] = 0.0;
        a.Bout[t] = 0.0;
        a.Sout[t] = 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += kThreads) {
        for (int s = 0; s < NS; ++s) {
            int j = ar.nb[i * NS + s];
            if (j < 0) continue;
            a.Aout[(size_t)i * N1 + j] = ar.Ast[i * NS + s];
            a.Bout[(size_t)i * N1 + j] = ar.Bst[i * NS + s];
            a.Sout[(size_t)i * N1 + j] = ar.Sst[i * NS + s];
        }
        a.Aout[(size_t)i * N1 + N] = a.Aout[(size_t)N * N1 + i] = ar.aH[i];
        a.Bout[(size_t)i * N1 + N] = a.Bout[(size_t)N * N1 + i] = ar.bH[i];
        a.Sout[(size_t)i * N1 + N] = a.Sout[(size_t)N * N1 + i] = ar.sH[i];
    }
    if (threadIdx.x == 0) {
        a.Aout[(size_t)N * N1 + N] = ar.sc[0];
        a.Bout[(size_t)N * N1 + N] = ar.sc[1];
        a.Sout[(size_t)N * N1 + N] = ar.sc[3];
    }
}

constexpr size_t kLdsLimit = 150 * 1024;

template <typename K>
int launch_small(K kern, size_t bytes, Args& a, hipStream_t s) {
    a.use_lds = bytes <= kLdsLimit;
    size_t shm = a.use_lds ? bytes : 0;
    if (shm > 64 * 1024) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm) != hipSuccess)
            return FMG_EHIP;
    }
    hipLaunchKernelGGL(kern, dim3(1), dim3(kThreads), shm, s, a);
    return hipGetLastError() == hipSuccess ? 0 : FMG_EHIP;
}

}  // namespace

size_t small_arena_bytes(int dim, int nc) {
    size_t a = dim == 2 ? std::max(arena_bytes_t<2, true>(nc), arena_bytes_t<2, false>(nc))
                        : std::max(arena_bytes_t<3, true>(nc), arena_bytes_t<3, false>(nc));
    return (a + 255) / 256 * 256;
}

size_t small_factor_bytes(int dim, int nc) {
    Sizes z = dim == 2 ? sizes<2, true>(nc) : sizes<3, true>(nc);
    return ((size_t)z.N * (z.w + 1) * sizeof(double) + 255) / 256 * 256;
}

int launch_coarse_newton(int dim, int nc, const Phys& ph, int max_iter, double tol, double* arena, double* fac,
                         double* xc_level, SmallState* state, hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.max_iter = max_iter; a.tol = tol; a.mom = nullptr; a.arena = arena;
    a.xc = xc_level; a.gc = make_grid(dim, nc); a.st = state; a.final_level = 0; a.certify = 1;
    a.fac = fac; a.reuse = 0;
    return dim == 2 ? launch_small(k_newton<2, false>, arena_bytes_t<2, false>(nc), a, s)
                    : launch_small(k_newton<3, false>, arena_bytes_t<3, false>(nc), a, s);
}

int launch_aug_newton(int dim, int nc, const Phys& ph, int max_iter, double tol, const double* moments, double* arena,
                      double* fac, double* xc_level, SmallState* state, int final_level, int certify, int reuse,
                      hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.max_iter = max_iter; a.tol = tol; a.mom = moments; a.arena = arena;
    a.xc = xc_level; a.gc = make_grid(dim, nc); a.st = state; a.final_level = final_level;
    a.certify = certify; a.fac = fac; a.reuse = reuse;
    return dim == 2 ? launch_small(k_newton<2, true>, arena_bytes_t<2, true>(nc), a, s)
                    : launch_small(k_newton<3, true>, arena_bytes_t<3, true>(nc), a, s);
}

int launch_aug_dump(int dim, int nc, const Phys& ph, const double* moments, const double* x, double* arena, double* A,
                    double* B, double* S, hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.mom = moments; a.arena = arena; a.xin = x; a.Aout = A; a.Bout = B; a.Sout = S;
    a.gc = make_grid(dim, nc);
    return dim == 2 ? launch_small(k_aug_dump<2>, arena_bytes_t<2, true>(nc), a, s)
                    : launch_small(k_aug_dump<3>, arena_bytes_t<3, true>(nc), a, s);
}

}  // namespace fmg
