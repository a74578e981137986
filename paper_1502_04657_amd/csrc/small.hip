// The small nonlinear eigenproblems of the method, solved on the device in one workgroup:
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
// involving u~ comes from the fine-grid moments (layout.h).  On the coarsest space the
// iteration starts from the discrete sine mode, solves the linear problem (zeta = 0)
// first and raises zeta in geometric stages (factor 4, halved on failure).  The final
// state is checked to be the ground state by the inertia of A + zeta S - (mu - eps) B.
#include "kernels.h"
#include "layout.h"

namespace fmg {

namespace {

constexpr int kThreads = 256;

template <int D>
struct Geo {
    static constexpr int V = D + 1;
    static constexpr int NE = (D == 2) ? 2 : 6;
    static constexpr int NS = (D == 2) ? kStencil2D : kStencil3D;
    static constexpr int NSTAR = (D == 2) ? 6 : 24;
};

// stencil slot of a neighbour offset (each component in -1..1), -1 if absent
template <int D>
__device__ inline int slot_of(const int* o) {
    for (int s = 0; s < Geo<D>::NS; ++s) {
        bool eq = true;
        for (int d = 0; d < D; ++d) eq = eq && ((D == 2 ? kOff2D[s][d] : kOff3D[s][d]) == o[d]);
        if (eq) return s;
    }
    return -1;
}

// int lambda_a lambda_b lambda_c lambda_d / |E| = D! alpha! / (D+4)!
template <int D>
__device__ inline double i4(int a, int b, int c, int d) {
    int cnt[4] = {0, 0, 0, 0};
    cnt[a]++; cnt[b]++; cnt[c]++; cnt[d]++;
    const double f[5] = {1.0, 1.0, 2.0, 6.0, 24.0};
    double num = (D == 2) ? 2.0 : 6.0;
    for (int v = 0; v < 4; ++v) num *= f[cnt[v]];
    return num / ((D == 2) ? 720.0 : 5040.0);
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
    // dump mode
    const double* xin;
    double* Aout;
    double* Bout;
    double* Sout;
};

template <int D, bool AUG>
struct Arena {
    int N, m, w, N1;
    double* Ast;
    double* Bst;
    double* Sst;
    double* band;
    double* x;
    double* xs;
    double* y;
    double* z;
    double* F;
    double* rhs;   // 3N
    double* aH;
    double* bH;
    double* sH;
    double* red;   // 4*16 reduction scratch
    double* sc;    // 32 shared scalars
    int* nb;       // N*NS neighbour index, -1 outside

    __device__ void carve(double* base, int nc) {
        m = nc - 1;
        N = (D == 2) ? m * m : m * m * m;
        w = (D == 2) ? m + 1 : m * m + m + 1;
        N1 = AUG ? N + 1 : N;
        constexpr int NS = Geo<D>::NS;
        double* p = base;
        Ast = p; p += (size_t)N * NS;
        Bst = p; p += (size_t)N * NS;
        Sst = p; p += (size_t)N * NS;
        band = p; p += (size_t)N * (w + 1);
        x = p; p += N + 2;
        xs = p; p += N + 2;
        y = p; p += N + 2;
        z = p; p += N + 2;
        F = p; p += N + 2;
        rhs = p; p += 3 * (size_t)N;
        aH = p; p += N;
        bH = p; p += N;
        sH = p; p += N;
        red = p; p += 64;
        sc = p; p += 32;
        nb = reinterpret_cast<int*>(p);
    }
};

__host__ __device__ inline size_t arena_doubles(int D, int nc) {
    int m = nc - 1;
    size_t N = (D == 2) ? (size_t)m * m : (size_t)m * m * m;
    size_t w = (D == 2) ? m + 1 : (size_t)m * m + m + 1;
    size_t NS = (D == 2) ? 7 : 15;
    size_t dbl = 3 * N * NS + N * (w + 1) + 5 * (N + 2) + 3 * N + 3 * N + 64 + 32;
    size_t ints = N * NS;
    return dbl + (ints + 1) / 2 + 8;
}

// block-wide sum of up to 8 values per thread; result broadcast to every thread
template <int K>
__device__ inline void block_sum(double (&v)[K], double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) red[wv * 16 + q] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = (red[q] + red[16 + q]) + (red[32 + q] + red[48 + q]);
    __syncthreads();
}

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

template <int D>
__device__ inline int cell_vert(int t, int v, int d) {
    return D == 2 ? kCellElemVert2D[t][v][d] : kCellElemVert3D[t][v][d];
}

// ---------------------------------------------------------------------------------------
// setup: neighbour table, coarse stencils of K + M_W and M, and the u~ border
template <int D, bool AUG>
__device__ void setup(Arena<D, AUG>& ar, const Args& a) {
    constexpr int NS = Geo<D>::NS;
    constexpr int NE = Geo<D>::NE;
    using L = MomLayout<D>;
    const int N = ar.N, m = ar.m, nc = a.nc;
    const double H = 1.0 / nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
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
        if (AUG) {
            // border: sum over the simplices around node i
            double ah = 0.0, bh = 0.0;
            for (int cc = 0; cc < (1 << D); ++cc) {
                int C[3] = {P[0] - ((cc >> 0) & 1), P[1] - ((cc >> 1) & 1), D == 3 ? P[2] - ((cc >> 2) & 1) : 0};
                int cl = (D == 2) ? C[0] + nc * C[1] : C[0] + nc * (C[1] + nc * C[2]);
                for (int t = 0; t < NE; ++t)
                    for (int v = 0; v < D + 1; ++v) {
                        bool hit = true;
                        for (int d = 0; d < D; ++d) hit = hit && (C[d] + cell_vert<D>(t, v, d) == P[d]);
                        if (!hit) continue;
                        const double* mo = a.mom + ((size_t)cl * NE + t) * L::SIZE;
                        ah += mo[L::KG + v] + mo[L::AW1 + v];
                        bh += mo[L::B1 + v];
                    }
            }
            ar.aH[i] = ah;
            ar.bH[i] = bh;
        }
    }
    if (AUG) {
        // scalars a_UU, b_UU and int u~ over all simplices
        const int nel = ((D == 2) ? nc * nc : nc * nc * nc) * NE;
        double v[3] = {0.0, 0.0, 0.0};
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
            const double* mo = a.mom + (size_t)e * L::SIZE;
            v[0] += mo[L::Q] + mo[L::AW2];
            v[1] += mo[L::B2];
            double s = 0.0;
            for (int p = 0; p < D + 1; ++p) s += mo[L::B1 + p];
            v[2] += s;
        }
        block_sum<3>(v, ar.red);
        if (threadIdx.x == 0) {
            ar.sc[0] = v[0];  // aU
            ar.sc[1] = v[1];  // bU
            ar.sc[2] = v[2];  // int u~
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------------
// S(x): coarse stencil Sst, border sH, corner sc[3]
template <int D, bool AUG>
__device__ void assemble_S(Arena<D, AUG>& ar, const Args& a, const double* x) {
    constexpr int NS = Geo<D>::NS;
    constexpr int NE = Geo<D>::NE;
    constexpr int V = D + 1;
    using L = MomLayout<D>;
    const int N = ar.N, m = ar.m, nc = a.nc;
    const double H = 1.0 / nc;
    const double vol = (D == 2) ? 0.5 * H * H : H * H * H / 6.0;
    const double c = AUG ? x[N] : 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        int P[3];
        node_pos<D>(i, m, P);
        double srow[NS];
        for (int s = 0; s < NS; ++s) srow[s] = 0.0;
        double sh = 0.0;
        for (int cc = 0; cc < (1 << D); ++cc) {
            int C[3] = {P[0] - ((cc >> 0) & 1), P[1] - ((cc >> 1) & 1), D == 3 ? P[2] - ((cc >> 2) & 1) : 0};
            int cl = (D == 2) ? C[0] + nc * C[1] : C[0] + nc * (C[1] + nc * C[2]);
            for (int t = 0; t < NE; ++t) {
                int va = -1;
                for (int v = 0; v < V; ++v) {
                    bool hit = true;
                    for (int d = 0; d < D; ++d) hit = hit && (C[d] + cell_vert<D>(t, v, d) == P[d]);
                    if (hit) va = v;
                }
                if (va < 0) continue;
                double U[V];
                int vs[V];
                for (int v = 0; v < V; ++v) {
                    int Q[3] = {0, 0, 0}, o[3] = {0, 0, 0};
                    for (int d = 0; d < D; ++d) {
                        Q[d] = C[d] + cell_vert<D>(t, v, d);
                        o[d] = Q[d] - P[d];
                    }
                    int j = node_id<D>(Q, m);
                    U[v] = (j >= 0) ? x[j] : 0.0;
                    vs[v] = slot_of<D>(o);
                }
                const double* mo = AUG ? a.mom + ((size_t)cl * NE + t) * L::SIZE : nullptr;
                for (int q = 0; q < V; ++q) {
                    double val = 0.0;
                    for (int p = 0; p < V; ++p)
                        for (int r = 0; r < V; ++r) val += U[p] * U[r] * i4<D>(p, r, va, q);
                    val *= vol;
                    if (AUG) {
                        double t3 = 0.0;
                        for (int p = 0; p < V; ++p)
                            t3 += U[p] * mo[L::T3 + sym3(p, va, q, D + 1)];
                        val += 2.0 * c * t3 + c * c * mo[L::T2 + sym2(va, q, D + 1)];
                    }
                    srow[vs[q]] += val;
                }
                if (AUG) {
                    double s1 = 0.0, s2 = 0.0;
                    for (int p = 0; p < V; ++p) {
                        for (int r = 0; r < V; ++r)
                            s1 += U[p] * U[r] * mo[L::T3 + sym3(p, r, va, D + 1)];
                        s2 += U[p] * mo[L::T2 + sym2(p, va, D + 1)];
                    }
                    sh += s1 + 2.0 * c * s2 + c * c * mo[L::T1 + va];
                }
            }
        }
        for (int s = 0; s < NS; ++s) ar.Sst[i * NS + s] = (ar.nb[i * NS + s] >= 0) ? srow[s] : 0.0;
        if (AUG) ar.sH[i] = sh;
    }
    if (AUG) {
        const int nel = ((D == 2) ? nc * nc : nc * nc * nc) * NE;
        double v[1] = {0.0};
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
            const int cl = e / NE, t = e % NE;
            int C[3] = {cl % nc, (cl / nc) % nc, D == 3 ? cl / (nc * nc) : 0};
            double U[V];
            for (int p = 0; p < V; ++p) {
                int Q[3] = {0, 0, 0};
                for (int d = 0; d < D; ++d) Q[d] = C[d] + cell_vert<D>(t, p, d);
                int j = node_id<D>(Q, m);
                U[p] = (j >= 0) ? x[j] : 0.0;
            }
            const double* mo = a.mom + (size_t)e * L::SIZE;
            double s1 = 0.0, s2 = 0.0;
            for (int p = 0; p < V; ++p) {
                for (int r = 0; r < V; ++r) s1 += U[p] * U[r] * mo[L::T2 + sym2(p, r, D + 1)];
                s2 += U[p] * mo[L::T1 + p];
            }
            v[0] += s1 + 2.0 * c * s2 + c * c * mo[L::T0];
        }
        block_sum<1>(v, ar.red);
        if (threadIdx.x == 0) ar.sc[3] = v[0];  // sU
    }
    __syncthreads();
}

// y = (A + zs S) x, z = B x (with borders); returns xTy, xTz via sc[4], sc[5]
template <int D, bool AUG>
__device__ void apply(Arena<D, AUG>& ar, double zs, const double* x, double* y, double* z) {
    constexpr int NS = Geo<D>::NS;
    const int N = ar.N;
    const double c = AUG ? x[N] : 0.0;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
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
            v[2] += g * x[i];
            v[3] += ar.bH[i] * x[i];
        }
        y[i] = yi;
        z[i] = zi;
        v[0] += x[i] * yi;
        v[1] += x[i] * zi;
    }
    block_sum<4>(v, ar.red);
    if (AUG && threadIdx.x == 0) {
        const double yU = v[2] + (ar.sc[0] + zs * ar.sc[3]) * c;
        const double zU = v[3] + ar.sc[1] * c;
        y[N] = yU;
        z[N] = zU;
        v[0] += c * yU;
        v[1] += c * zU;
    }
    if (threadIdx.x == 0) {
        ar.sc[4] = v[0];
        ar.sc[5] = v[1];
    }
    __syncthreads();
}

// band <- Ast + alpha Sst - sigma Bst   (lower band, row-major, band[i*(w+1)+k] = J(i,i-k))
template <int D, bool AUG>
__device__ void fill_band(Arena<D, AUG>& ar, double alpha, double sigma) {
    constexpr int NS = Geo<D>::NS;
    const int N = ar.N, w = ar.w;
    for (int t = threadIdx.x; t < N * (w + 1); t += blockDim.x) ar.band[t] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        for (int s = 0; s < NS; ++s) {
            int j = ar.nb[i * NS + s];
            if (j < 0 || j > i) continue;
            ar.band[(size_t)i * (w + 1) + (i - j)] = ar.Ast[i * NS + s] + alpha * ar.Sst[i * NS + s] - sigma * ar.Bst[i * NS + s];
        }
    __syncthreads();
}

// in-place banded LDL^T without pivoting; returns the number of negative pivots, or -1
// when a pivot is (numerically) zero or not finite.
template <int D, bool AUG>
__device__ int ldlt(Arena<D, AUG>& ar) {
    const int N = ar.N, w = ar.w, W1 = w + 1;
    double* b = ar.band;
    double scale = 0.0;
    for (int i = 0; i < N; ++i) scale = fmax(scale, fabs(b[(size_t)i * W1]));  // uniform loop (all threads)
    int neg = 0;
    for (int k = 0; k < N; ++k) {
        const double d = b[(size_t)k * W1];
        if (!(fabs(d) > 1e-14 * scale)) return -1;
        if (d < 0.0) ++neg;
        const int r = min(w, N - 1 - k);
        const int np = r * (r + 1) / 2;
        const double inv = 1.0 / d;
        for (int t = threadIdx.x; t < np; t += blockDim.x) {
            int ii = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
            if ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
            if (ii * (ii + 1) / 2 > t) --ii;
            const int jj = t - ii * (ii + 1) / 2;
            const int i = k + 1 + ii, j = k + 1 + jj;
            b[(size_t)i * W1 + (i - j)] -= b[(size_t)i * W1 + (i - k)] * b[(size_t)j * W1 + (j - k)] * inv;
        }
        __syncthreads();
    }
    return neg;
}

// solve (L D L^T) X = R for R rhs stored as rhs[r*N + i]
template <int D, bool AUG>
__device__ void ldlt_solve(Arena<D, AUG>& ar, double* rhs, int R) {
    const int N = ar.N, w = ar.w, W1 = w + 1;
    const double* b = ar.band;
    for (int k = 0; k < N; ++k) {
        const int r = min(w, N - 1 - k);
        for (int t = threadIdx.x; t < r * R; t += blockDim.x) {
            const int ii = t % r, q = t / r;
            const int i = k + 1 + ii;
            rhs[q * N + i] -= b[(size_t)i * W1 + (i - k)] / b[(size_t)k * W1] * rhs[q * N + k];
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < N * R; t += blockDim.x) {
        const int i = t % N;
        rhs[t] /= b[(size_t)i * W1];
    }
    __syncthreads();
    for (int k = N - 1; k >= 0; --k) {
        const int r = min(w, k);
        for (int t = threadIdx.x; t < r * R; t += blockDim.x) {
            const int ii = t % r, q = t / r;
            const int i = k - 1 - ii;
            rhs[q * N + i] -= b[(size_t)k * W1 + (k - i)] / b[(size_t)i * W1] * rhs[q * N + k];
        }
        __syncthreads();
    }
}

// One Newton solve at coupling zs from the iterate in ar.x.  Returns iterations >= 0 on
// convergence, -1 on failure.  mu in sc[6].
template <int D, bool AUG>
__device__ int newton(Arena<D, AUG>& ar, const Args& a, double zs) {
    const int N = ar.N, N1 = ar.N1;
    // normalise x^T B x = 1
    assemble_S<D, AUG>(ar, a, ar.x);
    apply<D, AUG>(ar, zs, ar.x, ar.y, ar.z);
    {
        const double s = 1.0 / sqrt(ar.sc[5]);
        for (int i = threadIdx.x; i < N1; i += blockDim.x) ar.x[i] *= s;
        __syncthreads();
    }
    double mu = 0.0;
    for (int it = 0; it <= a.max_iter; ++it) {
        assemble_S<D, AUG>(ar, a, ar.x);
        apply<D, AUG>(ar, zs, ar.x, ar.y, ar.z);
        if (it == 0) mu = ar.sc[4] / ar.sc[5];
        const double F2 = 0.5 * (1.0 - ar.sc[5]);
        double v[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < N1; i += blockDim.x) {
            const double f = ar.y[i] - mu * ar.z[i];
            ar.F[i] = f;
            v[0] += f * f;
            v[1] += ar.z[i] * ar.z[i];
        }
        block_sum<2>(v, ar.red);
        const double res = sqrt(v[0]) / (fabs(mu) * sqrt(v[1]));
        if (threadIdx.x == 0) ar.sc[7] = res;
        if (!(v[0] == v[0]) || !(mu == mu)) return -3;
        // x^T B x = 1 up to the rounding of an N-term dot product
        if (res <= a.tol && fabs(F2) <= 4.0 * N1 * 1.1e-16) {
            const double sN = 1.0 / sqrt(ar.sc[5]);
            for (int i = threadIdx.x; i < N1; i += blockDim.x) ar.x[i] *= sN;
            if (threadIdx.x == 0) ar.sc[6] = mu;
            __syncthreads();
            return it;
        }
        if (it == a.max_iter) return -2;
        // Jacobian blocks
        fill_band<D, AUG>(ar, 3.0 * zs, mu);
        if (ldlt<D, AUG>(ar) < 0) return -1;
        const int R = AUG ? 3 : 2;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            ar.rhs[i] = -ar.F[i];
            if (AUG) {
                ar.rhs[N + i] = ar.aH[i] + 3.0 * zs * ar.sH[i] - mu * ar.bH[i];
                ar.rhs[2 * N + i] = -ar.z[i];
            } else {
                ar.rhs[N + i] = -ar.z[i];
            }
        }
        __syncthreads();
        ldlt_solve<D, AUG>(ar, ar.rhs, R);
        double dmu, dc = 0.0;
        if (AUG) {
            // 2x2 Schur complement for (dc, dmu)
            double s[6] = {0, 0, 0, 0, 0, 0};
            for (int i = threadIdx.x; i < N; i += blockDim.x) {
                const double jh = ar.aH[i] + 3.0 * zs * ar.sH[i] - mu * ar.bH[i];
                const double zh = ar.z[i];
                s[0] += jh * ar.rhs[i];
                s[1] += jh * ar.rhs[N + i];
                s[2] += jh * ar.rhs[2 * N + i];
                s[3] += zh * ar.rhs[i];
                s[4] += zh * ar.rhs[N + i];
                s[5] += zh * ar.rhs[2 * N + i];
            }
            block_sum<6>(s, ar.red);
            const double jU = ar.sc[0] + 3.0 * zs * ar.sc[3] - mu * ar.sc[1];
            const double zU = ar.z[N];
            const double a11 = jU - s[1], a12 = -s[2] - zU, r1 = -ar.F[N] - s[0];
            const double a21 = s[4] - zU, a22 = s[5], r2 = -F2 + s[3];
            const double det = a11 * a22 - a12 * a21;
            if (!(fabs(det) > 0.0)) return -4;
            dc = (r1 * a22 - a12 * r2) / det;
            dmu = (a11 * r2 - a21 * r1) / det;
            for (int i = threadIdx.x; i < N; i += blockDim.x)
                ar.x[i] += ar.rhs[i] - ar.rhs[N + i] * dc - ar.rhs[2 * N + i] * dmu;
            if (threadIdx.x == 0) ar.x[N] += dc;
        } else {
            double s[2] = {0, 0};
            for (int i = threadIdx.x; i < N; i += blockDim.x) {
                s[0] += ar.z[i] * ar.rhs[i];
                s[1] += ar.z[i] * ar.rhs[N + i];
            }
            block_sum<2>(s, ar.red);
            if (!(fabs(s[1]) > 0.0)) return -4;
            dmu = (-F2 + s[0]) / s[1];
            for (int i = threadIdx.x; i < N; i += blockDim.x) ar.x[i] += ar.rhs[i] - ar.rhs[N + i] * dmu;
        }
        mu += dmu;
        __syncthreads();
    }
    return -2;
}

// inertia check: number of eigenvalues of (A + zs S(x), B) below sigma (0: ground state)
template <int D, bool AUG>
__device__ int count_below(Arena<D, AUG>& ar, const Args& a, double zs, double sigma) {
    const int N = ar.N;
    fill_band<D, AUG>(ar, zs, sigma);
    int neg = ldlt<D, AUG>(ar);
    if (neg < 0) return 1;
    if (AUG) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) ar.rhs[i] = ar.aH[i] + zs * ar.sH[i] - sigma * ar.bH[i];
        __syncthreads();
        ldlt_solve<D, AUG>(ar, ar.rhs, 1);
        double s[1] = {0.0};
        for (int i = threadIdx.x; i < N; i += blockDim.x) s[0] += (ar.aH[i] + zs * ar.sH[i] - sigma * ar.bH[i]) * ar.rhs[i];
        block_sum<1>(s, ar.red);
        const double schur = (ar.sc[0] + zs * ar.sc[3] - sigma * ar.sc[1]) - s[0];
        if (!(schur > 0.0)) ++neg;
    }
    return neg;
}

template <int D, bool AUG>
__device__ void finish(Arena<D, AUG>& ar, const Args& a, int iters, bool ok, int reason) {
    const int N = ar.N, m = ar.m;
    const double H = 1.0 / a.nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
    if (ok) {
        // ground-state check on the final iterate (S is current from the last Newton pass)
        const double mu = ar.sc[6];
        const int below = count_below<D, AUG>(ar, a, a.ph.zeta, mu - 1e-9 * fabs(mu));
        // sign: int u_h > 0
        double v[1] = {0.0};
        for (int i = threadIdx.x; i < N; i += blockDim.x) v[0] += ar.x[i];
        block_sum<1>(v, ar.red);
        double integ = Hd * v[0] + (AUG ? ar.x[N] * ar.sc[2] : 0.0);
        const double sgn = integ < 0.0 ? -1.0 : 1.0;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
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
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            int P[3];
            node_pos<D>(i, m, P);
            a.xc[P[0] + a.gc.pitch * P[1] + a.gc.plane * P[2]] = 0.0;
        }
        if (threadIdx.x == 0) {
            a.st->c = 1.0;
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
    const int N = ar.N, m = ar.m;
    int iters = 0;
    bool ok = true;
    int reason = 0;
    if (AUG) {
        // start from u = u~ / ||u~||_M
        for (int i = threadIdx.x; i < N; i += blockDim.x) ar.x[i] = 0.0;
        if (threadIdx.x == 0) ar.x[N] = 1.0;
        __syncthreads();
        int r = newton<D, AUG>(ar, a, a.ph.zeta);
        ok = r >= 0;
        iters = ok ? r : 0;
        reason = ok ? 0 : -r;
    } else {
        // discrete sine mode, linear ground state, then zeta stages
        const double H = 1.0 / a.nc;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            int P[3];
            node_pos<D>(i, m, P);
            double v = sinpi(P[0] * H) * sinpi(P[1] * H);
            if (D == 3) v *= sinpi(P[2] * H);
            ar.x[i] = v;
        }
        __syncthreads();
        int r = newton<D, AUG>(ar, a, 0.0);
        ok = r >= 0;
        iters = ok ? r : 0;
        reason = ok ? 0 : -r;
        const double zeta = a.ph.zeta;
        if (ok && zeta > 0.0) {
            const double lf = log(4.0);
            const double lt = log(zeta);
            int J = zeta > 1.0 ? (int)ceil(lt / lf - 1e-12) : 0;
            double lnext = lt - J * lf, step = lf, lcur = 0.0;
            bool have_cur = false;
            for (int guard = 0; guard < 200; ++guard) {
                const bool last = !(lnext < lt);
                const double z = last ? zeta : exp(lnext);
                for (int i = threadIdx.x; i < N; i += blockDim.x) ar.xs[i] = ar.x[i];
                __syncthreads();
                int rr = newton<D, AUG>(ar, a, z);
                if (rr < 0) {
                    for (int i = threadIdx.x; i < N; i += blockDim.x) ar.x[i] = ar.xs[i];
                    __syncthreads();
                    if (!have_cur) { ok = false; reason = -rr; break; }
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
    const int N = ar.N, N1 = N + 1;
    for (int i = threadIdx.x; i < N1; i += blockDim.x) ar.x[i] = a.xin[i];
    __syncthreads();
    assemble_S<D, true>(ar, a, ar.x);
    for (int t = threadIdx.x; t < N1 * N1; t += blockDim.x) {
        a.Aout[t] = 0.0;
        a.Bout[t] = 0.0;
        a.Sout[t] = 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
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
int launch_small(K kern, int dim, int nc, Args& a, hipStream_t s) {
    const size_t bytes = arena_doubles(dim, nc) * sizeof(double);
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

size_t small_arena_bytes(int dim, int nc) { return arena_doubles(dim, nc) * sizeof(double); }

int launch_coarse_newton(int dim, int nc, const Phys& ph, int max_iter, double tol, double* arena, double* xc_level,
                         SmallState* state, hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.max_iter = max_iter; a.tol = tol; a.mom = nullptr; a.arena = arena;
    a.xc = xc_level; a.gc = make_grid(dim, nc); a.st = state; a.final_level = 0;
    return dim == 2 ? launch_small(k_newton<2, false>, dim, nc, a, s) : launch_small(k_newton<3, false>, dim, nc, a, s);
}

int launch_aug_newton(int dim, int nc, const Phys& ph, int max_iter, double tol, const double* moments, double* arena,
                      double* xc_level, SmallState* state, int final_level, hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.max_iter = max_iter; a.tol = tol; a.mom = moments; a.arena = arena;
    a.xc = xc_level; a.gc = make_grid(dim, nc); a.st = state; a.final_level = final_level;
    return dim == 2 ? launch_small(k_newton<2, true>, dim, nc, a, s) : launch_small(k_newton<3, true>, dim, nc, a, s);
}

int launch_aug_dump(int dim, int nc, const Phys& ph, const double* moments, const double* x, double* arena, double* A,
                    double* B, double* S, hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.mom = moments; a.arena = arena; a.xin = x; a.Aout = A; a.Bout = B; a.Sout = S;
    a.gc = make_grid(dim, nc);
    return dim == 2 ? launch_small(k_aug_dump<2>, dim, nc, a, s) : launch_small(k_aug_dump<3>, dim, nc, a, s);
}

}  // namespace fmg
