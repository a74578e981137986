// The small nonlinear eigenproblems of the method, solved on the device by one workgroup:
//   * Algorithm 3.2 step 1: the ground state on the coarsest space V_{h_1};
//   * Algorithm 3.1 step 2: the augmented problem (3.6) on V_H + span{u~}.
// With u = Z x, Z = [coarse hats, u~] (or the coarse hats alone),
//     F(x, mu) = [ (A + zeta S(x)) x - mu B x ; (1 - x^T B x)/2 ] = 0,
// A = Z^T (K + M_W) Z, B = Z^T M Z, S(x) = Z^T M_{(Zx)^2} Z, is solved by Newton's method
// (the paper allows a self-consistent or a Newton-type iteration) with the Jacobian
//     [ A + 3 zeta S(x) - mu B , -B x ; -(B x)^T , 0 ].
// The coarse-coarse blocks of A and B are the coarse stencils themselves (Galerkin
// identities of nested P1 spaces), evaluated on the fly; everything involving u~ comes
// from the fine-grid moments (layout.h).
//
// Linear algebra.  In lexicographic order the coarse block J of the Jacobian is block
// tridiagonal: blocks are grid rows (2D) or grid planes (3D).  It is factored by block
// cyclic reduction: at each level the odd blocks of the remaining chain are eliminated in
// parallel (explicit inverse of each pivot block, Schur updates of the neighbours), so the
// dependency chain has log2(rows) levels of dense block products instead of one step per
// unknown.  A solve is one sweep down and one sweep up the levels.  The border rows of the
// Newton system are eliminated through a 2x2 (or 1x1) Schur complement.  The numbers of
// negative pivots of the block inverses give the inertia of J (Sylvester), which is the
// ground-state check.
//
// The factorisation is reused: it is kept in device memory between calls, and Newton
// steps use the latest factor and the border columns frozen with it (chord steps) for as
// long as the residual contracts by at least a factor 4 per step; otherwise the iterate
// goes back one step and the Jacobian is refactored there.  The fixed point is unchanged.
//
// On the coarsest space the iteration starts from the discrete sine mode and raises zeta in
// geometric stages (factor 8 from a first stage <= 16, the step halved on failure); stages
// before the last stop at a relative residual of 1e-3.
#include <utility>

#include "kernels.h"
#include "layout.h"

namespace fmg {

namespace {

constexpr int kThreads = 256;               // four wavefronts
#ifndef FMG_SMALL_STAGE_TOL
#define FMG_SMALL_STAGE_TOL 1e-3
#endif
constexpr double kStageTol = FMG_SMALL_STAGE_TOL;   // residual for intermediate continuation stages
#ifndef FMG_SMALL_FIRST_STAGE
#define FMG_SMALL_FIRST_STAGE 16.0
#endif
constexpr double kFirstStage = FMG_SMALL_FIRST_STAGE;   // largest coupling of the first stage
constexpr int kWaves = kThreads / 64;

template <int D>
struct Geo {
    static constexpr int V = D + 1;
    static constexpr int NE = (D == 2) ? 2 : 6;
    static constexpr int NS = (D == 2) ? kStencil2D : kStencil3D;
};

// stencil slot of vertex b seen from vertex a in simplex t of a cell (compile time)
template <int D>
__host__ __device__ constexpr int qslot_ce(int t, int a, int b) {
    for (int s = 0; s < Geo<D>::NS; ++s) {
        bool eq = true;
        for (int d = 0; d < D; ++d) {
            const int o = (D == 2) ? kCellElemVert2D[t % 2][b][d] - kCellElemVert2D[t % 2][a][d]
                                   : kCellElemVert3D[t][b][d] - kCellElemVert3D[t][a][d];
            eq = eq && (o == ((D == 2) ? kOff2D[s][d] : kOff3D[s][d]));
        }
        if (eq) return s;
    }
    return -1;
}
// local index in simplex t of the vertex in stencil slot s seen from vertex a, or -1
template <int D>
__host__ __device__ constexpr int slot_vert_ce(int t, int a, int s) {
    for (int b = 0; b < D + 1; ++b)
        if (qslot_ce<D>(t, a, b) == s) return b;
    return -1;
}
template <int D, int T, int A, int B>
struct QSlot {
    static constexpr int value = qslot_ce<D>(T, A, B);
    static_assert(value >= 0, "simplex edge outside the stencil");
};
template <int D, int T, int V, int Dim>
struct CellVert {
    static constexpr int value = (D == 2) ? kCellElemVert2D[T % 2][V % 3][Dim % 2] : kCellElemVert3D[T][V][Dim];
};
// local index in simplex T of the cell vertex with offsets (CV & 1, CV >> 1 & 1, CV >> 2 & 1),
// or -1 if T does not contain it
template <int D>
__host__ __device__ constexpr int vert_of(int t, int cv) {
    for (int v = 0; v < D + 1; ++v) {
        bool eq = true;
        for (int d = 0; d < D; ++d) {
            const int o = (D == 2) ? kCellElemVert2D[t % 2][v % 3][d % 2] : kCellElemVert3D[t][v][d];
            eq = eq && (o == ((cv >> d) & 1));
        }
        if (eq) return v;
    }
    return -1;
}
template <int D, int T, int CV>
struct VertOf {
    static constexpr int value = vert_of<D>(T, CV);
};
template <int D, int S, int Dim>
struct Off {
    static constexpr int value = (D == 2) ? kOff2D[S % 7][Dim % 2] : kOff3D[S][Dim];
};

// f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>), unrolled at compile time
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}
// f(integral_constant<int, t>) for t = 0 .. N-1 in a loop that is not unrolled (one
// instance of f per t, selected at run time), which keeps register pressure to one body
template <int N, typename F>
__device__ __forceinline__ void rolled_for(F&& f) {
#pragma unroll 1
    for (int t = 0; t < N; ++t) {
        static_for<N>([&](auto tc) {
            if (decltype(tc)::value == t) f(tc);
        });
    }
}
// simplices of a cell: unrolled in 2D, rolled in 3D
template <int D, typename F>
__device__ __forceinline__ void for_simplices(F&& f) {
    if constexpr (D == 2) static_for<Geo<D>::NE>(f);
    else rolled_for<Geo<D>::NE>(f);
}
// stencil slots of a node: unrolled in 2D (7), rolled in 3D (15)
template <int D, typename F>
__device__ __forceinline__ void for_slots(F&& f) {
    if constexpr (D == 2) static_for<Geo<D>::NS>(f);
    else rolled_for<Geo<D>::NS>(f);
}
// f(integral_constant<int, v>) for the run-time value v in [0, N) (uniform per wavefront)
template <int N, typename F>
__device__ __forceinline__ void dispatch(int v, F&& f) {
    static_for<N>([&](auto vc) {
        if (decltype(vc)::value == v) f(vc);
    });
}

struct Args {
    int nc;
    Phys ph;
    int max_iter;
    int fixed_iters;     // augmented solve: > 0 accepts the iterate after that many iterations
    double tol;
    const double* mom;
    double* arena;       // global arena (used when the problem does not fit in LDS)
    int use_lds;
    int stage_blocks;    // global-arena kernels: blocks inverted at a time in dynamic LDS
    double* xc;          // coarsest padded level array receiving x_H
    Grid gc;
    SmallState* st;
    int final_level;     // tolerance checks enabled for this step
    int certify;         // ground-state inertia check: 0 never, 1 always, 2 when the step meets tol_lambda
    double* fac;         // persistent block factor, may be null
    int reuse;           // start from the stored factor when it exists
    double* esc;         // global scratch: per-simplex values of the 3D assembly (kEsc each)
    int mstage;          // 3D bordered solves: per-simplex moments staged in LDS after the arena
    // dump mode
    const double* xin;
    double* Aout;
    double* Bout;
    double* Sout;
};

// Optional phase timers of the small solves (wall clock, 100 MHz ticks); compiled only
// with -DFMG_SMALL_TIMING, read back with fmg_debug_small_timers().
#if defined(FMG_SMALL_TIMING) || defined(FMG_SMALL_MICRO)
__device__ unsigned long long g_small_t[32];
#endif
#ifdef FMG_SMALL_TIMING
#define FMG_T0(v) const unsigned long long v = wall_clock64()
#define FMG_TACC(k, v) do { if (threadIdx.x == 0) atomicAdd(&g_small_t[(AUG ? 0 : 16) + (k)], wall_clock64() - (v)); } while (0)
#define FMG_TCNT(k) do { if (threadIdx.x == 0) atomicAdd(&g_small_t[(AUG ? 0 : 16) + (k)], 1ull); } while (0)
#else
#define FMG_T0(v) do { } while (0)
#define FMG_TACC(k, v) do { } while (0)
#define FMG_TCNT(k) do { } while (0)
#endif

struct Sizes {
    int m, N, N1, nel;
    int nb, bs, B2;   // block rows, block size, bs^2
    int h;            // most blocks eliminated on one level
    int sz1;          // scratch doubles (products, solve temporaries)
};

template <int D, bool AUG>
__host__ __device__ inline Sizes sizes(int nc) {
    Sizes z;
    z.m = nc - 1;
    z.N = (D == 2) ? z.m * z.m : z.m * z.m * z.m;
    z.N1 = AUG ? z.N + 1 : z.N;
    z.nel = ((D == 2) ? nc * nc : nc * nc * nc) * Geo<D>::NE;
    z.nb = z.m;
    z.bs = (D == 2) ? z.m : z.m * z.m;
    z.B2 = z.bs * z.bs;
    z.h = z.nb / 2 > 0 ? z.nb / 2 : 1;
    z.sz1 = z.h * z.B2 > 3 * z.N ? z.h * z.B2 : 3 * z.N;
    return z;
}

template <int D, bool AUG>
struct Arena {
    Sizes z;
    double* Sst;                                   // S(x) stencil, N x NS
    double* x; double* xs; double* xk; double* y; double* z2; double* F; double* rhs;
    double* xp; double* fp;                        // previous iterate and chord step (acceleration)
    double* stage = nullptr;                       // LDS staging of block inversions (global arena)
    int stage_blocks = 0;
    double* aH; double* bH; double* sH; double* sc; double* red;
    double* Dm; double* Fm; double* Rm;            // block factor (nb blocks each)
    double* S1; double* S2;                        // scratch
    bool s_stale = false;                          // Sst, sH, sc[3] not at the current x
    // moments T3..T0 of simplex e at mo + e * mstride (the global moments, or their LDS
    // copy) and the per-simplex values of the direct residual (3D)
    const double* mo = nullptr;
    int mstride = 0;
    double* tvs = nullptr;

    __device__ void carve(double* base, int nc) {
        z = sizes<D, AUG>(nc);
        constexpr int NS = Geo<D>::NS;
        const int N = z.N;
        double* p = base;
        Dm = p; p += (size_t)z.nb * z.B2;
        Fm = p; p += (size_t)z.nb * z.B2;
        Rm = p; p += (size_t)z.nb * z.B2;
        S1 = p; p += z.sz1;
        S2 = p; p += (size_t)z.h * z.B2;
        Sst = p; p += (size_t)N * NS;
        x = p; p += N + 2;
        xs = p; p += N + 2;
        xk = p; p += N + 2;
        y = p; p += N + 2;
        z2 = p; p += N + 2;
        F = p; p += N + 2;
        xp = p; p += N + 2;
        fp = p; p += N + 2;
        rhs = p; p += 3 * (size_t)N;
        aH = p; p += N;
        bH = p; p += N;
        sH = p; p += N;
        sc = p; p += 32;
        red = p;
    }
};

template <int D, bool AUG>
__host__ __device__ inline size_t arena_bytes_t(int nc) {
    Sizes z = sizes<D, AUG>(nc);
    constexpr int NS = Geo<D>::NS;
    size_t N = z.N;
    size_t dbl = 3 * (size_t)z.nb * z.B2 + z.sz1 + (size_t)z.h * z.B2 + N * NS + 8 * (N + 2) + 3 * N + 3 * N + 32 +
                 8 * kWaves;
    return dbl * sizeof(double) + 64;
}

// LDS stage of the 3D bordered solves, after the arena: the moments T3..T0 of every simplex
// (the part of the moment layout the Newton iterations read) and the per-simplex values of
// the direct residual
template <int D>
__host__ __device__ inline size_t mstage_doubles(int nc) {
    const size_t nel = (D == 2) ? (size_t)nc * nc * 2 : (size_t)nc * nc * nc * 6;
    return nel * (MomLayout<D>::T0 + 1 + (D + 1));
}

// factor = Dm, Fm, Rm (contiguous at the start of the arena)
template <int D>
__host__ __device__ inline size_t factor_doubles(int nc) {
    Sizes z = sizes<D, true>(nc);
    return 3 * (size_t)z.nb * z.B2;
}

// ---- workgroup reductions (fixed order: every thread gets the same bits) ------------------
template <int K>
__device__ __forceinline__ void bsum(double* red, double (&v)[K]) {
    static_assert(K <= 8, "at most 8 values per reduction");
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[wid * 8 + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = red[k];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s += red[w * 8 + k];
        v[k] = s;
    }
}
__device__ __forceinline__ double bsum1(double* red, double v) {
    double a[1] = {v};
    bsum<1>(red, a);
    return a[0];
}
__device__ __forceinline__ double bmax1(double* red, double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wid * 8] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s = fmax(s, red[w * 8]);
    return s;
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

// neighbour of node P in stencil slot S, or -1 on the boundary
template <int D, int S>
__device__ __forceinline__ int nbr(const int* P, int m) {
    int Q[3] = {P[0] + Off<D, S, 0>::value, P[1] + Off<D, S, 1>::value, (D == 3) ? P[2] + Off<D, S, 2>::value : 0};
    return node_id<D>(Q, m);
}

// x[j] for a neighbour index j, and 0 where there is none (j < 0): loaded from a clamped
// address, so the loads of a node's slots do not sit under branches and can be in flight
// together (adding the zero products leaves every sum unchanged)
__device__ __forceinline__ double nbr_val(const double* x, int j) {
    const double v = x[j < 0 ? 0 : j];
    return j < 0 ? 0.0 : v;
}

// coarse stencils at node X (coordinates), slot S: a = (K + M_W)_S, b = M_S
template <int D, int S>
__device__ __forceinline__ void stencil_ab(const double* X, double H, double Hd, const Phys& ph, double& a, double& b) {
    constexpr double m0 = (D == 2) ? kM0_2D[S % 7] : kM0_3D[S];
    double cw = ph.wc * m0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double m1 = (D == 2) ? kM1_2D[k % 2][S % 7] : kM1_3D[k][S];
        const double m2 = (D == 2) ? kM2_2D[k % 2][S % 7] : kM2_3D[k][S];
        cw += ph.w[k] * (X[k] * X[k] * m0 + 2.0 * X[k] * H * m1 + H * H * m2);
    }
    constexpr int o1 = (Off<D, S, 0>::value < 0 ? -Off<D, S, 0>::value : Off<D, S, 0>::value) +
                       (Off<D, S, 1>::value < 0 ? -Off<D, S, 1>::value : Off<D, S, 1>::value) +
                       (D == 3 ? (Off<D, S, 2>::value < 0 ? -Off<D, S, 2>::value : Off<D, S, 2>::value) : 0);
    // the stiffness couples axis neighbours only: diag = 2 sum a_d, -a_d along axis d
    constexpr int ax1 = Off<D, S, 0>::value != 0 ? 0 : (Off<D, S, 1>::value != 0 ? 1 : 2);
    const double dg = (D == 2) ? 2.0 * (ph.a[0] + ph.a[1]) : 2.0 * ((ph.a[0] + ph.a[1]) + ph.a[2]);
    double kk;
    if (D == 2)
        kk = (o1 == 0) ? dg : (o1 == 1 ? -ph.a[ax1] : 0.0);
    else
        kk = (o1 == 0) ? dg * H : (o1 == 1 ? -ph.a[ax1] * H : 0.0);
    a = kk + Hd * cw;
    b = Hd * m0;
}

// Cells of the coarse mesh in 2^D colour classes (parity of the cell index in every
// direction): cells of one class share no vertex, so one thread per cell and vertex may
// scatter into the vertex rows without atomics, and the summation order is fixed.
struct ColorClass {
    int px, py, pz, hx, hy, hz, ncol, ncolp;
};
template <int D>
__device__ __forceinline__ ColorClass color_class(int nc, int color) {
    ColorClass c;
    c.px = color & 1;
    c.py = (color >> 1) & 1;
    c.pz = (color >> 2) & 1;
    c.hx = (nc - c.px + 1) >> 1;
    c.hy = (nc - c.py + 1) >> 1;
    c.hz = (D == 3) ? (nc - c.pz + 1) >> 1 : 1;
    c.ncol = c.hx * c.hy * c.hz;
    c.ncolp = (c.ncol + 63) & ~63;   // a multiple of the wavefront: vertex index uniform per wave
    return c;
}
template <int D>
__device__ __forceinline__ void cell_of(const ColorClass& c, int q, int nc, int& C0, int& C1, int& C2, int& cl) {
    C0 = c.px + 2 * (q % c.hx);
    C1 = c.py + 2 * ((q / c.hx) % c.hy);
    C2 = (D == 3) ? c.pz + 2 * (q / (c.hx * c.hy)) : 0;
    cl = (D == 2) ? C0 + nc * C1 : C0 + nc * (C1 + nc * C2);
}

// interior node index of vertex V of simplex T in cell (C0, C1, C2), or -1 on the boundary
template <int D, int T, int V>
__device__ __forceinline__ int vert_node(int C0, int C1, int C2, int m) {
    int P[3] = {C0 + CellVert<D, T, V, 0>::value, C1 + CellVert<D, T, V, 1>::value,
                (D == 3) ? C2 + CellVert<D, T, V, 2>::value : 0};
    return node_id<D>(P, m);
}

// Where the Newton iterations find the moments: staged, they are copied once per call from
// the global moment array into LDS after the arena (lds_base: the arena's start) and the
// direct residual keeps its per-simplex values there too; otherwise both stay in global
// memory.
template <int D, bool AUG>
__device__ __forceinline__ void bind_moments(Arena<D, AUG>& ar, const Args& a, double* lds_base, bool staged) {
    using L = MomLayout<D>;
    constexpr int NM = L::T0 + 1;
    static_assert(L::T3 == 0 && L::T2 < L::T1 && L::T1 < L::T0, "leading moment block");
    if (staged) {
        double* st = lds_base + arena_bytes_t<D, AUG>(a.nc) / sizeof(double);
        // kB loads in flight per thread before their stores (clamped addresses stay in bounds;
        // 28 takes the 384 x 35 moments of the 4^3 mesh in two rounds)
        constexpr int kB = 28;
        const int total = ar.z.nel * NM;
        for (int k0 = threadIdx.x; k0 < total; k0 += kThreads * kB) {
            double v[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int k = min(k0 + u * kThreads, total - 1);
                const int e = k / NM, q = k - e * NM;
                v[u] = a.mom[(size_t)e * L::SIZE + q];
            }
#pragma unroll
            for (int u = 0; u < kB; ++u)
                if (k0 + u * kThreads < total) st[k0 + u * kThreads] = v[u];
        }
        ar.mo = st;
        ar.mstride = NM;
        ar.tvs = st + (size_t)total;
        __syncthreads();
    } else {
        ar.mo = a.mom;
        ar.mstride = L::SIZE;
        ar.tvs = a.esc;
    }
}

// ---------------------------------------------------------------------------------------
// setup: the u~ border a(u~, phi_i), b(u~, phi_i) and the scalars a(u~,u~), b(u~,u~), int u~
template <int D, bool AUG>
__device__ __forceinline__ void setup(Arena<D, AUG>& ar, const Args& a) {
    constexpr int NE = Geo<D>::NE;
    constexpr int V = D + 1;
    using L = MomLayout<D>;
    const int N = ar.z.N, m = ar.z.m, nc = a.nc;
    if (!AUG) return;
    double v3[3] = {0.0, 0.0, 0.0};
    // one pass: each node gathers its border entries from the simplices around it in a fixed
    // order (from clamped addresses with a 0/1 factor, so that all loads are in flight
    // together); the scalars are summed over the simplices by a second loop
    for (int i = threadIdx.x; i < N; i += kThreads) {
        int P[3];
        node_pos<D>(i, m, P);
        double sa = 0.0, sb = 0.0;
        static_for<(1 << D)>([&](auto cvc) {
            constexpr int cv = decltype(cvc)::value;
            const int C0 = P[0] - (cv & 1), C1 = P[1] - ((cv >> 1) & 1), C2 = (D == 3) ? P[2] - ((cv >> 2) & 1) : 0;
            const bool cin = !(C0 < 0 || C0 >= nc || C1 < 0 || C1 >= nc || (D == 3 && (C2 < 0 || C2 >= nc)));
            const int cl = cin ? ((D == 2) ? C0 + nc * C1 : C0 + nc * (C1 + nc * C2)) : 0;
            const double w = cin ? 1.0 : 0.0;
            static_for<Geo<D>::NE>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                constexpr int v = VertOf<D, t, cv>::value;
                if constexpr (v >= 0) {
                    const double* mo = a.mom + (size_t)(cl * NE + t) * L::SIZE;
                    sa += w * (mo[L::KG + v] + mo[L::AW1 + v]);
                    sb += w * mo[L::B1 + v];
                }
            });
        });
        ar.aH[i] = sa;
        ar.bH[i] = sb;
    }
    const int nsimp = ((D == 2) ? nc * nc : nc * nc * nc) * NE;
    for (int e = threadIdx.x; e < nsimp; e += kThreads) {
        const double* mo = a.mom + (size_t)e * L::SIZE;
        static_for<V>([&](auto vc) { v3[2] += mo[L::B1 + decltype(vc)::value]; });
        v3[0] += mo[L::Q] + mo[L::AW2];
        v3[1] += mo[L::B2];
    }
    bsum<3>(ar.red, v3);
    if (threadIdx.x == 0) {
        ar.sc[0] = v3[0];  // aU
        ar.sc[1] = v3[1];  // bU
        ar.sc[2] = v3[2];  // int u~
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

// S(x) on one simplex, row AA: Sr[b] = int u^2 l_AA l_b (u = sum_p U_p l_p + c u~) and,
// with AUG, the border entry sh = int u^2 u~ l_AA.  UU[sym2(p,r)] = U_p U_r (doubled off
// the diagonal).
template <int D, bool AUG, int AA>
__device__ __forceinline__ void elem_row(const double* U, const double* UU, const double* mo, double c, double vol,
                                         double* Sr, double& sh) {
    constexpr int V = D + 1;
    using L = MomLayout<D>;
#pragma unroll
    for (int bb = 0; bb < V; ++bb) {
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < V; ++p)
#pragma unroll
            for (int r = p; r < V; ++r) v += UU[sym2(p, r, V)] * i4e(p, r, AA, bb, D);
        v *= vol;
        if (AUG) {
            double t3 = 0.0;
#pragma unroll
            for (int p = 0; p < V; ++p) t3 += U[p] * mo[L::T3 + sym3(p, AA, bb, V)];
            v += 2.0 * c * t3 + c * c * mo[L::T2 + sym2(AA, bb, V)];
        }
        Sr[bb] = v;
    }
    if (AUG) {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int p = 0; p < V; ++p) {
#pragma unroll
            for (int r = p; r < V; ++r) s1 += UU[sym2(p, r, V)] * mo[L::T3 + sym3(p, r, AA, V)];
            s2 += U[p] * mo[L::T2 + sym2(p, AA, V)];
        }
        sh = s1 + 2.0 * c * s2 + c * c * mo[L::T1 + AA];
    }
}

// int u^2 u~^2 on one simplex (the corner of S with AUG)
template <int D>
__device__ __forceinline__ double elem_corner(const double* U, const double* UU, const double* mo, double c) {
    constexpr int V = D + 1;
    using L = MomLayout<D>;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int p = 0; p < V; ++p) {
#pragma unroll
        for (int r = p; r < V; ++r) s1 += UU[sym2(p, r, V)] * mo[L::T2 + sym2(p, r, V)];
        s2 += U[p] * mo[L::T1 + p];
    }
    return s1 + 2.0 * c * s2 + c * c * mo[L::T0];
}

// S(x) on one simplex of a 3D mesh: the upper triangle Se[sym2(a, b)] = int w^2 l_a l_b of
// the element matrix (w = u_H + c u~, u_H = sum_p U_p l_p) and, with AUG, the border entries
// sh[a] = int w^2 u~ l_a and the corner int w^2 u~^2 (returned).  The u_H^2 part is the
// closed form
//   int u_H^2 l_a l_b = |e| D! / (D+4)! (1 + delta_ab) (p1^2 + p2 + 2 p1 (U_a + U_b) + 2 (U_a^2 + U_a U_b + U_b^2)),
// p_k = sum_p U_p^k; the parts with u~ are sums of the moments, e.g.
// int u_H^2 u~ l_a = sum_{p <= r} UU[p, r] T3[p, r, a] (UU: U_p U_r, doubled off the diagonal).
template <bool AUG>
__device__ __forceinline__ double simplex_S3(const double* U, const double* UU, const double* mo, double c, double vol,
                                             double* Se, double* sh) {
    constexpr int V = 4;
    using L = MomLayout<3>;
    double p1 = 0.0, p2 = 0.0;
#pragma unroll
    for (int p = 0; p < V; ++p) {
        p1 += U[p];
        p2 += U[p] * U[p];
    }
    const double kv = vol * (6.0 / 5040.0);
    const double base = p1 * p1 + p2;
    static_for<V>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        static_for<V - a>([&](auto bc) {
            constexpr int b = a + decltype(bc)::value;
            const double uh = base + 2.0 * p1 * (U[a] + U[b]) + 2.0 * (U[a] * U[a] + U[a] * U[b] + U[b] * U[b]);
            double v = (a == b ? 2.0 : 1.0) * kv * uh;
            if (AUG) {
                double t = 0.0;
#pragma unroll
                for (int p = 0; p < V; ++p) t += U[p] * mo[L::T3 + sym3(p, a, b, V)];
                v += c * (2.0 * t + c * mo[L::T2 + sym2(a, b, V)]);
            }
            Se[sym2(a, b, V)] = v;
        });
    });
    double corner = 0.0;
    if (AUG) {
        double ct = 0.0, c1 = 0.0;
        static_for<V>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            double qa = 0.0, ta = 0.0;
#pragma unroll
            for (int p = 0; p < V; ++p) {
#pragma unroll
                for (int r = p; r < V; ++r) qa += UU[sym2(p, r, V)] * mo[L::T3 + sym3(p, r, a, V)];
                ta += U[p] * mo[L::T2 + sym2(p, a, V)];
            }
            const double t1 = mo[L::T1 + a];
            sh[a] = qa + c * (2.0 * ta + c * t1);
            ct += U[a] * ta;
            c1 += U[a] * t1;
        });
        corner = ct + c * (2.0 * c1 + c * mo[L::T0]);
    }
    return corner;
}

// S(x): coarse stencil Sst, border sH, corner sc[3], in one pass.  One thread per coarse
// node builds its own row: for every cell around the node and every simplex of that cell
// containing it, the simplex's row of that vertex, in a fixed order (no other thread writes
// the row, so no colouring and no atomics).  The corner term is summed over the simplices
// by a second loop of the same pass.
template <int D, bool AUG>
__device__ __forceinline__ void assemble_S_nodes(Arena<D, AUG>& ar, const Args& a, const double* x) {
    constexpr int NS = Geo<D>::NS;
    constexpr int NE = Geo<D>::NE;
    constexpr int V = D + 1;
    constexpr int NCV = 1 << D;
    using L = MomLayout<D>;
    const int N = ar.z.N, nc = a.nc, m = ar.z.m;
    const double H = 1.0 / nc;
    const double vol = (D == 2) ? 0.5 * H * H : H * H * H / 6.0;
    const double c = AUG ? x[N] : 0.0;
    for (int i = threadIdx.x; i < N; i += kThreads) {
        int P[3];
        node_pos<D>(i, m, P);
        double row[NS];
        static_for<NS>([&](auto sc_) { row[decltype(sc_)::value] = 0.0; });
        double shs = 0.0;
        auto corner = [&](auto cvc) {
            constexpr int cv = decltype(cvc)::value;
            // the node is cell vertex cv of the cell with origin P - (cv bits)
            const int C0 = P[0] - (cv & 1), C1 = P[1] - ((cv >> 1) & 1), C2 = (D == 3) ? P[2] - ((cv >> 2) & 1) : 0;
            if (C0 < 0 || C0 >= nc || C1 < 0 || C1 >= nc || (D == 3 && (C2 < 0 || C2 >= nc))) return;
            const int cl = (D == 2) ? C0 + nc * C1 : C0 + nc * (C1 + nc * C2);
            for_simplices<D>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                constexpr int aa = VertOf<D, t, cv>::value;
                if constexpr (aa >= 0) {
                    int nd[V];
                    double U[V];
                    static_for<V>([&](auto vc) {
                        constexpr int v = decltype(vc)::value;
                        nd[v] = vert_node<D, t, v>(C0, C1, C2, m);
                        U[v] = nd[v] >= 0 ? x[nd[v]] : 0.0;
                    });
                    double UU[V * (V + 1) / 2];
#pragma unroll
                    for (int p = 0; p < V; ++p)
#pragma unroll
                        for (int r = p; r < V; ++r) UU[sym2(p, r, V)] = (p == r ? 1.0 : 2.0) * U[p] * U[r];
                    const double* mo = AUG ? a.mom + (size_t)(cl * NE + t) * L::SIZE : nullptr;
                    double Sr[V], sh = 0.0;
                    elem_row<D, AUG, aa>(U, UU, mo, c, vol, Sr, sh);
                    static_for<V>([&](auto bc) {
                        constexpr int bb = decltype(bc)::value;
                        if (nd[bb] >= 0) row[QSlot<D, t, aa, bb>::value] += Sr[bb];
                    });
                    shs += sh;
                }
            });
        };
        if constexpr (D == 2) static_for<NCV>(corner);
        else rolled_for<NCV>(corner);
        double* out = ar.Sst + (size_t)i * NS;
        static_for<NS>([&](auto sc_) { out[decltype(sc_)::value] = row[decltype(sc_)::value]; });
        if (AUG) ar.sH[i] = shs;
    }
    if (AUG) {
        double sU = 0.0;
        const int nsimp = ((D == 2) ? nc * nc : nc * nc * nc) * NE;
        for (int e = threadIdx.x; e < nsimp; e += kThreads) {
            const int cl = e / NE, te = e - cl * NE;
            const int C0 = cl % nc, C1 = (cl / nc) % nc, C2 = (D == 3) ? cl / (nc * nc) : 0;
            dispatch<NE>(te, [&](auto tc) {
                constexpr int t = decltype(tc)::value;
                double U[V];
                static_for<V>([&](auto vc) {
                    constexpr int v = decltype(vc)::value;
                    const int nd = vert_node<D, t, v>(C0, C1, C2, m);
                    U[v] = nd >= 0 ? x[nd] : 0.0;
                });
                double UU[V * (V + 1) / 2];
#pragma unroll
                for (int p = 0; p < V; ++p)
#pragma unroll
                    for (int r = p; r < V; ++r) UU[sym2(p, r, V)] = (p == r ? 1.0 : 2.0) * U[p] * U[r];
                sU += elem_corner<D>(U, UU, a.mom + (size_t)(cl * NE + t) * L::SIZE, c);
            });
        }
        sU = bsum1(ar.red, sU);
        if (threadIdx.x == 0) ar.sc[3] = sU;
    }
    __syncthreads();
}

// S(x) in two passes (3D, where one thread per node would leave most lanes idle on small
// coarse spaces and the per-node version of 2D spills registers):
//   1. one thread per simplex computes its element matrix of S (the rows of elem_row; 10
//      unique entries), its border entries (4) and its corner term into the global scratch;
//   2. one thread per (stencil slot, node) adds, in a fixed order, the entries of the
//      simplices around the node that couple it to that neighbour, so no colouring and no
//      atomics.
constexpr int kEsc = 16;   // per-simplex scratch: 10 matrix entries, 4 border entries, corner
template <int D, bool AUG>
__device__ __forceinline__ void assemble_S_simplices(Arena<D, AUG>& ar, const Args& a, const double* x) {
    constexpr int NS = Geo<D>::NS;
    constexpr int NE = Geo<D>::NE;
    constexpr int V = D + 1;
    constexpr int NCV = 1 << D;
    constexpr int NSYM = V * (V + 1) / 2;
    static_assert(NSYM + V + 1 <= kEsc, "per-simplex scratch");
    static_assert(D == 3, "the 3D assembly");
    const int N = ar.z.N, nc = a.nc, m = ar.z.m;
    const double H = 1.0 / nc;
    const double vol = (D == 2) ? 0.5 * H * H : H * H * H / 6.0;
    const double c = AUG ? x[N] : 0.0;
    double* es = a.esc;
    const int ncell = (D == 2) ? nc * nc : nc * nc * nc;
    const int nsimp = ncell * NE;
    double sU = 0.0;
    // simplices in type-major order, so that the simplex type (a compile-time branch) is
    // uniform across a wavefront except where two types meet
    for (int f = threadIdx.x; f < nsimp; f += kThreads) {
        const int te = f / ncell, cl = f - te * ncell;
        const int e = cl * NE + te;
        const int C0 = cl % nc, C1 = (cl / nc) % nc, C2 = (D == 3) ? cl / (nc * nc) : 0;
        dispatch<NE>(te, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
            double U[V];
            static_for<V>([&](auto vc) {
                constexpr int v = decltype(vc)::value;
                const int nd = vert_node<D, t, v>(C0, C1, C2, m);
                U[v] = nd >= 0 ? x[nd] : 0.0;
            });
            double UU[NSYM];
#pragma unroll
            for (int p = 0; p < V; ++p)
#pragma unroll
                for (int r = p; r < V; ++r) UU[sym2(p, r, V)] = (p == r ? 1.0 : 2.0) * U[p] * U[r];
            constexpr int NM = MomLayout<D>::T0 + 1;
            double mo[NM];
            if (AUG) {
                const double* src = ar.mo + (size_t)e * ar.mstride;
#pragma unroll
                for (int q = 0; q < NM; ++q) mo[q] = src[q];
            }
            double* out = es + (size_t)e * kEsc;
            double Se[NSYM], sh[V];
            const double corner = simplex_S3<AUG>(U, UU, mo, c, vol, Se, sh);
#pragma unroll
            for (int q = 0; q < NSYM; ++q) out[q] = Se[q];
            if (AUG) {
#pragma unroll
                for (int q = 0; q < V; ++q) out[NSYM + q] = sh[q];
                sU += corner;
            }
        });
    }
    __syncthreads();
    // one item per (slot, node), slot-major (s = k / N), so a wavefront covers few slots and
    // every item's loads are independent; item (s, i) adds, over the cells around node i and
    // their simplices in a fixed order, the entry coupling node i to its neighbour in slot s
    // (s = NS: the border entry).  Every entry is loaded (from a clamped simplex where the
    // cell is off the mesh) and added with a 0/1 factor; adding a zero leaves the sum unchanged.
    for (int k = threadIdx.x; k < (AUG ? NS + 1 : NS) * N; k += kThreads) {
        const int s = k / N, i = k - s * N;
        int P[3];
        node_pos<D>(i, m, P);
        dispatch<NS + 1>(s, [&](auto sc_) {
            constexpr int S = decltype(sc_)::value;
            double acc = 0.0;
            static_for<NCV>([&](auto cvc) {
                constexpr int cv = decltype(cvc)::value;
                // the node is cell vertex cv of the cell with origin P - (cv bits)
                const int C0 = P[0] - (cv & 1), C1 = P[1] - ((cv >> 1) & 1), C2 = P[2] - ((cv >> 2) & 1);
                const bool cin = !(C0 < 0 || C0 >= nc || C1 < 0 || C1 >= nc || C2 < 0 || C2 >= nc);
                const int cl = cin ? C0 + nc * (C1 + nc * C2) : 0;
                const double w = cin ? 1.0 : 0.0;
                static_for<NE>([&](auto tc) {
                    constexpr int t = decltype(tc)::value;
                    constexpr int aa = VertOf<D, t, cv>::value;
                    if constexpr (aa >= 0) {
                        const double* in = es + (size_t)(cl * NE + t) * kEsc;
                        if constexpr (S == NS) {
                            acc += w * in[NSYM + aa];
                        } else {
                            constexpr int bb = slot_vert_ce<D>(t, aa, S);
                            if constexpr (bb >= 0) acc += w * in[sym2(aa, bb, V)];
                        }
                    }
                });
            });
            if constexpr (S < NS) ar.Sst[(size_t)i * NS + S] = nbr<D, S>(P, m) >= 0 ? acc : 0.0;
            else ar.sH[i] = acc;
        });
    }
    if (AUG) {
        sU = bsum1(ar.red, sU);
        if (threadIdx.x == 0) ar.sc[3] = sU;
    }
    __syncthreads();
}

template <int D, bool AUG>
__device__ __forceinline__ void assemble_S(Arena<D, AUG>& ar, const Args& a, const double* x) {
    if constexpr (D == 2) assemble_S_nodes<D, AUG>(ar, a, x);
    else assemble_S_simplices<D, AUG>(ar, a, x);
}

// y = (A + zs S) x, z = B x (with borders); sc[4] = x^T y, sc[5] = x^T z
template <int D, bool AUG>
__device__ __forceinline__ void apply(Arena<D, AUG>& ar, const Args& a, double zs, const double* x, double* y,
                                      double* z) {
    constexpr int NS = Geo<D>::NS;
    const int N = ar.z.N, m = ar.z.m;
    const double H = 1.0 / a.nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
    const double c = AUG ? x[N] : 0.0;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < N; i += kThreads) {
        int P[3];
        node_pos<D>(i, m, P);
        const double X[3] = {P[0] * H, P[1] * H, P[2] * H};
        double yi = 0.0, zi = 0.0;
        static_for<Geo<D>::NS>([&](auto sc_) {
            constexpr int s = decltype(sc_)::value;
            const int j = nbr<D, s>(P, m);
            double as, bs;
            stencil_ab<D, s>(X, H, Hd, a.ph, as, bs);
            const double xj = nbr_val(x, j);
            yi += (as + zs * ar.Sst[(size_t)i * NS + s]) * xj;
            zi += bs * xj;
        });
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
    bsum<4>(ar.red, v);
    if (threadIdx.x == 0) {
        if (AUG) {
            const double yU = v[2] + (ar.sc[0] + zs * ar.sc[3]) * c;
            const double zU = v[3] + ar.sc[1] * c;
            y[N] = yU;
            z[N] = zU;
            v[0] += c * yU;
            v[1] += c * zU;
        }
        ar.sc[4] = v[0];
        ar.sc[5] = v[1];
    }
    __syncthreads();
}

// Whether apply_direct can run: bordered solves; in 2D the per-simplex values must fit the
// scratch S1, S2 (contiguous; free between factorisations and block solves), in 3D they go
// to the global per-simplex scratch (kEsc >= D + 1 values per simplex).
template <int D, bool AUG>
__device__ __forceinline__ bool direct_ok(const Arena<D, AUG>& ar) {
    if constexpr (D == 3) return AUG;
    return AUG && (size_t)ar.z.nel * (D + 1) <= (size_t)ar.z.sz1 + (size_t)ar.z.h * ar.z.B2;
}

// y = (A + zs S) x and z = B x (with borders) as apply() gives them, without the stencil of
// S(x).  With w = c u~ + u_H, row i of S(x) x plus c times the border column is the integral
// of w^3 phi_i, and the border row's share is the integral of w^3 u~.  One pass over the
// simplices evaluates the first for each vertex and sums the second; a pass over the nodes
// then adds the values of the simplices around each node in a fixed order.  The chord steps
// need this residual but not the Jacobian, so S(x) is assembled only when the Jacobian is
// refactored or its border columns are frozen again.
//
// The simplices run in type-major order (the simplex type is a compile-time branch, uniform
// across a wavefront except where two types meet).  Their D + 1 vertex values go to the LDS
// scratch S1, S2 in 2D and to the per-simplex scratch (LDS or global) in 3D.  In 2D the
// moments come from global memory and each thread loads those of its two simplices before it
// uses either.  The node pass loads the values of the simplices around a node from clamped
// addresses and adds them with a 0/1 factor, so all its loads are independent of branches
// (adding a zero leaves every sum unchanged).
template <int D, bool AUG>
__device__ __forceinline__ void apply_direct(Arena<D, AUG>& ar, const Args& a, double zs, const double* x, double* y,
                                             double* z) {
    static_assert(AUG, "bordered solves only");
    constexpr int NE = Geo<D>::NE;
    constexpr int V = D + 1;
    constexpr int NCV = 1 << D;
    static_assert(D == 2 || V <= kEsc, "per-simplex scratch");
    using L = MomLayout<D>;
    constexpr int NM = L::T0 + 1;   // the moments used here: T3, T2, T1, T0 (leading entries)
    static_assert(L::T3 == 0 && L::T2 < L::T1 && L::T1 < L::T0, "leading moment block");
    // simplices per thread and round whose moments are loaded together
    constexpr int KS = (D == 2) ? 2 : 1;
    const int N = ar.z.N, nc = a.nc, m = ar.z.m;
    const double H = 1.0 / nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
    const double vol = (D == 2) ? 0.5 * H * H : H * H * H / 6.0;
    // int lambda^alpha over a simplex, |alpha| = 4: |e| D! alpha! / (D + 4)!
    const double kv = vol * ((D == 2) ? 12.0 / 720.0 : 36.0 / 5040.0);
    const double c = x[N];
    double* tv = (D == 2) ? ar.S1 : ar.tvs;   // nel x V
    const int ncell = (D == 2) ? nc * nc : nc * nc * nc;
    const int nsimp = ncell * NE;
    double sb = 0.0;
    auto simplex = [&](int f, const double* mo) {
        const int te = f / ncell, cl = f - te * ncell;
        const int e = cl * NE + te;
        const int C0 = cl % nc, C1 = (D == 2) ? cl / nc : (cl / nc) % nc, C2 = (D == 2) ? 0 : cl / (nc * nc);
        dispatch<NE>(te, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
            double U[V];
            static_for<V>([&](auto vc) {
                constexpr int v = decltype(vc)::value;
                const int nd = vert_node<D, t, v>(C0, C1, C2, m);
                U[v] = nd >= 0 ? x[nd] : 0.0;
            });
            double UU[V * (V + 1) / 2];
#pragma unroll
            for (int p = 0; p < V; ++p)
#pragma unroll
                for (int r = p; r < V; ++r) UU[sym2(p, r, V)] = (p == r ? 1.0 : 2.0) * U[p] * U[r];
            // int u_H^3 l_a = |e| D! 3! / (D+4)! (h3 + U_a h2 + U_a^2 h1 + U_a^3), h_k the
            // complete homogeneous symmetric polynomials of the vertex values U
            double p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
            for (int p = 0; p < V; ++p) {
                const double u2 = U[p] * U[p];
                p1 += U[p];
                p2 += u2;
                p3 += u2 * U[p];
            }
            const double h2 = 0.5 * (p1 * p1 + p2);
            const double h3 = (p1 * (p1 * p1 + 3.0 * p2) + 2.0 * p3) * (1.0 / 6.0);
            double su = 0.0, ra[V];
            static_for<V>([&](auto ac) {
                constexpr int aa = decltype(ac)::value;
                // qa = int u_H^2 u~ l_a, ta = int u_H u~^2 l_a
                double qa = 0.0, ta = 0.0;
#pragma unroll
                for (int p = 0; p < V; ++p) {
#pragma unroll
                    for (int r = p; r < V; ++r) qa += UU[sym2(p, r, V)] * mo[L::T3 + sym3(p, r, aa, V)];
                    ta += U[p] * mo[L::T2 + sym2(p, aa, V)];
                }
                const double t1 = mo[L::T1 + aa];
                const double cub = kv * (h3 + U[aa] * (h2 + U[aa] * (p1 + U[aa])));
                // int w^3 l_a, w = u_H + c u~
                ra[aa] = cub + c * (3.0 * qa + c * (3.0 * ta + c * t1));
                // int w^3 u~ = sum_a U_a (qa + 3 c ta + 3 c^2 t1_a) + c^3 int u~^4
                su += U[aa] * (qa + c * (3.0 * ta + c * (3.0 * t1)));
            });
            sb += su + c * c * c * mo[L::T0];
#pragma unroll
            for (int q = 0; q < V; ++q) tv[(size_t)e * V + q] = ra[q];
        });
    };
#ifdef FMG_SMALL_MICRO
    const unsigned long long tq0 = wall_clock64();
#endif
    for (int f0 = threadIdx.x; f0 < nsimp; f0 += KS * kThreads) {
        // the moments of the simplices in registers before any store (a store to the
        // per-simplex values could alias them, which would reload them after it)
        double mo[KS][NM];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int f = min(f0 + k * kThreads, nsimp - 1);
            const int te = f / ncell, cl = f - te * ncell;
            const double* src = ar.mo + (size_t)(cl * NE + te) * ar.mstride;
#pragma unroll
            for (int q = 0; q < NM; ++q) mo[k][q] = src[q];
        }
#pragma unroll
        for (int k = 0; k < KS; ++k)
            if (f0 + k * kThreads < nsimp) simplex(f0 + k * kThreads, mo[k]);
    }
    __syncthreads();
#ifdef FMG_SMALL_MICRO
    const unsigned long long tq1 = wall_clock64();
#endif
    double v[5] = {0.0, 0.0, 0.0, 0.0, sb};
    for (int i = threadIdx.x; i < N; i += kThreads) {
        int P[3];
        node_pos<D>(i, m, P);
        const double X[3] = {P[0] * H, P[1] * H, (D == 2) ? 0.0 : P[2] * H};
        double yi = 0.0, zi = 0.0, gi = 0.0;
        static_for<NCV>([&](auto cvc) {
            constexpr int cv = decltype(cvc)::value;
            const int C0 = P[0] - (cv & 1), C1 = P[1] - ((cv >> 1) & 1), C2 = (D == 2) ? 0 : P[2] - ((cv >> 2) & 1);
            const bool cin = !(C0 < 0 || C0 >= nc || C1 < 0 || C1 >= nc || C2 < 0 || C2 >= nc);
            const int cl = cin ? C0 + nc * (C1 + nc * C2) : 0;
            const double w = cin ? 1.0 : 0.0;
            static_for<Geo<D>::NE>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                constexpr int aa = VertOf<D, t, cv>::value;
                if constexpr (aa >= 0) gi += w * tv[(size_t)(cl * NE + t) * V + aa];
            });
        });
        static_for<Geo<D>::NS>([&](auto sc_) {
            constexpr int s = decltype(sc_)::value;
            const int j = nbr<D, s>(P, m);
            double as, bs;
            stencil_ab<D, s>(X, H, Hd, a.ph, as, bs);
            const double xj = nbr_val(x, j);
            yi += as * xj;
            zi += bs * xj;
        });
        yi += zs * gi + ar.aH[i] * c;
        zi += ar.bH[i] * c;
        v[2] += ar.aH[i] * x[i];
        v[3] += ar.bH[i] * x[i];
        y[i] = yi;
        z[i] = zi;
        v[0] += x[i] * yi;
        v[1] += x[i] * zi;
    }
#ifdef FMG_SMALL_MICRO
    __syncthreads();
    const unsigned long long tq2 = wall_clock64();
#endif
    bsum<5>(ar.red, v);
    if (threadIdx.x == 0) {
        const double yU = v[2] + ar.sc[0] * c + zs * v[4];
        const double zU = v[3] + ar.sc[1] * c;
        y[N] = yU;
        z[N] = zU;
        ar.sc[4] = v[0] + c * yU;
        ar.sc[5] = v[1] + c * zU;
    }
    __syncthreads();
#ifdef FMG_SMALL_MICRO
    if (threadIdx.x == 0) {
        atomicAdd(&g_small_t[13], tq1 - tq0);
        atomicAdd(&g_small_t[14], tq2 - tq1);
        atomicAdd(&g_small_t[15], wall_clock64() - tq2);
    }
#endif
}

// ---------------------------------------------------------------------------------------
// Block cyclic reduction of J = A + alpha S - sigma B (coarse block).  Blocks j = 0..nb-1
// hold rows j*bs .. j*bs+bs-1.  At level st (1, 2, 4, ...) the blocks e = st*(2i+1) are
// eliminated; their neighbours are l = e - st and r = e + st.  Afterwards
//     Dm[e] = P_e = (pivot block)^{-1},  Fm[e] = G_l = P_e J_{e,l},  Rm[e] = G_r = P_e J_{r,e}^T,
// and Dm[0] is the inverse of the last pivot block.  Fm[j] holds the coupling J_{j, left}
// of block j while j is still in the chain.

// Thread layout for block-vector work: this thread serves rows p = p0, p0 + pstep, ... of
// the blocks g, g + G, ... (one division per thread, none in the loops).
struct VecMap {
    int p0, pstep, g, G;
};
__device__ __forceinline__ VecMap vec_map(int bs) {
    VecMap v;
    if (bs <= kThreads) {
        v.G = kThreads / bs;
        v.g = threadIdx.x / bs;
        v.p0 = threadIdx.x - v.g * bs;
        v.pstep = bs;
        if (v.g >= v.G) v.g = 1 << 30;   // idle thread
    } else {
        v.G = 1;
        v.g = 0;
        v.p0 = threadIdx.x;
        v.pstep = kThreads;
    }
    return v;
}

// sum_k a[k*sa] * b[k*sb] for k = 0..n-1 in order; the loads of 8 terms are issued
// together (indices clamped in bounds)
__device__ __forceinline__ double dotn(const double* a, int sa, const double* b, int sb, int n) {
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += 8) {
        double x[8], y[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = min(k0 + j, n - 1);
            x[j] = a[k * sa];
            y[j] = b[k * sb];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (k0 + j < n) acc = fma(x[j], y[j], acc);
    }
    return acc;
}

// ---- blocks of at most 16 x 16: one wavefront per block product on the FP64 matrix
// cores (v_mfma_f64_16x16x4).  Lane l supplies A[l % 16][k0 + l / 16] and
// B[k0 + l / 16][l % 16]; the 16 x 16 result sits in lane l, register r at
// (row l / 16 + 4 r, column l % 16).  Blocks are stored row-major with leading dimension
// bs and padded with zeros to 16 inside the product.
typedef double d4_t __attribute__((ext_vector_type(4)));

struct Tile {
    int i;    // lane % 16: row of A, column of B and of the result
    int kq;   // lane / 16: k within a chunk of 4, row group of the result
};
__device__ __forceinline__ Tile tile_lane() {
    const int l = threadIdx.x & 63;
    return Tile{l & 15, l >> 4};
}

// Operands of one 16 x 16 x 16 product in this lane: av[j] = s * op(A)[i][4j + kq],
// bv[j] = op(B)[4j + kq][i] (zero outside the bs x bs block).  All loads are issued before
// the matrix instructions that consume them.
struct Ops16 {
    double av[4], bv[4];
};
__device__ __forceinline__ Ops16 ops_mm(const Tile& t, const double* A, bool ta, const double* B, bool tb, int bs,
                                        double s) {
    // fixed offsets from one base per operand (entries outside the block are read, the
    // arena continues past every block, and zeroed)
    Ops16 o;
    const double* a0 = A + (ta ? t.kq * bs + t.i : t.i * bs + t.kq);
    const double* b0 = B + (tb ? t.i * bs + t.kq : t.kq * bs + t.i);
    const int da = ta ? 4 * bs : 4, db = tb ? 4 : 4 * bs;
    double a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a[j] = a0[j * da];
        b[j] = b0[j * db];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * j + t.kq;
        const bool ok = t.i < bs && k < bs;
        o.av[j] = ok ? s * a[j] : 0.0;
        o.bv[j] = ok ? b[j] : 0.0;
    }
    return o;
}
__device__ __forceinline__ d4_t mfma16(const Ops16& o, d4_t c) {
#pragma unroll
    for (int j = 0; j < 4; ++j) c = __builtin_amdgcn_mfma_f64_16x16x4f64(o.av[j], o.bv[j], c, 0, 0, 0);
    return c;
}
// c += s * op(A) op(B) for bs x bs blocks (op = transpose when the flag is set)
__device__ __forceinline__ d4_t mm16(const Tile& t, const double* A, bool ta, const double* B, bool tb, int bs,
                                     double s, d4_t c) {
    return mfma16(ops_mm(t, A, ta, B, tb, bs, s), c);
}
__device__ __forceinline__ d4_t load16(const Tile& t, const double* M, int bs) {
    d4_t c;
    double v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = M[(t.kq + 4 * r) * bs + t.i];   // read past the block, zeroed
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = t.kq + 4 * r;
        c[r] = (row < bs && t.i < bs) ? v[r] : 0.0;
    }
    return c;
}
__device__ __forceinline__ void store16(const Tile& t, double* M, int bs, d4_t c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = t.kq + 4 * r;
        if (row < bs && t.i < bs) M[row * bs + t.i] = c[r];
    }
}

// 1/p: hardware estimate refined by two Newton-Raphson steps (r <- r + r (1 - p r))
__device__ __forceinline__ double recip(double p) {
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}

// row group G (lanes 16 G .. 16 G + 15) of v copied to all four row groups
template <int G>
__device__ __forceinline__ double rowgroup_bcast(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    // permlane16_swap: [0] holds row groups (0, 0, 2, 2), [1] holds (1, 1, 3, 3)
    const auto lo16 = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi16 = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const unsigned lo = (G & 1) ? lo16[1] : lo16[0], hi = (G & 1) ? hi16[1] : hi16[0];
    // permlane32_swap: [0] repeats lanes 0..31, [1] repeats lanes 32..63
    const auto lo32 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto hi32 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return (G & 2) ? dbl_from(lo32[1], hi32[1]) : dbl_from(lo32[0], hi32[0]);
}

// value of v in lane `lane` (uniform across the wavefront), through scalar registers
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}


// Gauss-Jordan inversion of the pivot blocks Dm[first + step*i], i < cnt, one wavefront per
// block with the block in registers (result layout of mm16); pivot rows and columns move
// between lanes with shuffles.  Returns the number of negative pivots (LDL^T pivots of the
// blocks), or -1 if one is zero relative to `scale`.
template <int D, bool AUG>
__device__ __forceinline__ int block_invert16(Arena<D, AUG>& ar, int first, int step, int cnt, double scale) {
    const int bs = ar.z.bs, B2 = ar.z.B2;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const Tile t = tile_lane();
    int neg = 0, bad = 0;
    #pragma unroll 1
    for (int task = wid; task < cnt; task += kWaves) {
        double* M = ar.Dm + (size_t)(first + step * task) * B2;
        d4_t m = load16(t, M, bs);
        // step k (unrolled: the lane moves take k as an immediate).  Row k of the block sits
        // in row group k % 4 of the lanes, register k / 4; column k in lane k of each row.
        static_for<16>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if (k >= bs) return;
            constexpr int kr = k >> 2, g = k & 3;
            const double rk = m[kr];
            // A[k][col]: row group g copied to every row group (lane swaps across rows)
            const double pr = rowgroup_bcast<g>(rk);
            // A[row][k] of my rows: lane k of each row of 16
            d4_t pc;
#pragma unroll
            for (int r = 0; r < 4; ++r) pc[r] = dpp_f64<0x150 + k>(m[r]);   // row_newbcast:k
            const double piv = readlane_f64(rk, g * 16 + k);         // A[k][k], uniform
            if (!(fabs(piv) > 1e-15 * scale)) bad = 1;
            if (piv < 0.0) ++neg;
            const double inv = recip(piv);
            const double prinv = pr * inv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = t.kq + 4 * r;
                const double off = (t.i == k) ? -pc[r] * inv : fma(-pc[r], prinv, m[r]);
                const double on = (t.i == k) ? inv : prinv;
                m[r] = (row == k) ? on : off;
            }
        });
        store16(t, M, bs, m);
    }
    // combine the per-wavefront counts
    __syncthreads();
    if (lane == 0) {
        ar.red[wid * 8 + 6] = (double)neg;
        ar.red[wid * 8 + 7] = (double)bad;
    }
    __syncthreads();
    int tn = 0, tb = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        tn += (int)ar.red[w * 8 + 6];
        tb += (int)ar.red[w * 8 + 7];
    }
    __syncthreads();
    return tb ? -1 : tn;
}

// the levels of the block cyclic reduction for bs <= 16 (blocks already built)
template <int D, bool AUG>
__device__ __forceinline__ int bcr_levels16(Arena<D, AUG>& ar, double scale) {
    const int nb = ar.z.nb, bs = ar.z.bs, B2 = ar.z.B2;
    const int wid = threadIdx.x >> 6;
    const Tile t = tile_lane();
    int neg = 0;
    for (int st = 1; st < nb; st *= 2) {
        int ne = 0;
        while (st * (2 * ne + 1) < nb) ++ne;
        const int r0 = block_invert16<D, AUG>(ar, st, 2 * st, ne, scale);
        if (r0 < 0) return -1;
        neg += r0;
        // G_l = P_e J_{e,l} -> S1[i],  G_r = P_e J_{r,e}^T -> Rm[e]
        #pragma unroll 1
        for (int task = wid; task < 2 * ne; task += kWaves) {
            const int i = task >> 1, e = st * (2 * i + 1), rr = e + st;
            const double* P = ar.Dm + (size_t)e * B2;
            d4_t c = {0.0, 0.0, 0.0, 0.0};
            if ((task & 1) == 0) {
                c = mm16(t, P, false, ar.Fm + (size_t)e * B2, false, bs, 1.0, c);
                store16(t, ar.S1 + (size_t)i * B2, bs, c);
            } else {
                if (rr < nb) c = mm16(t, P, false, ar.Fm + (size_t)rr * B2, true, bs, 1.0, c);
                store16(t, ar.Rm + (size_t)e * B2, bs, c);
            }
        }
        __syncthreads();
        // Schur updates of the blocks that stay, and the new couplings r <- l
        const int na = (nb - 1) / (2 * st) + 1;
        #pragma unroll 1
        for (int task = wid; task < na + ne; task += kWaves) {
            if (task < na) {
                const int aa = 2 * st * task, e1 = aa + st, e0 = aa - st;
                // D_a -= J_{e1,a}^T G_l(e1) + J_{a,e0} G_r(e0)  (missing neighbours: zero operands)
                const Ops16 o1 = ops_mm(t, ar.Fm + (size_t)(e1 < nb ? e1 : aa) * B2, true,
                                        ar.S1 + (size_t)(e1 < nb ? task : 0) * B2, false, bs, e1 < nb ? -1.0 : 0.0);
                const Ops16 o0 = ops_mm(t, ar.Fm + (size_t)aa * B2, false, ar.Rm + (size_t)(e0 >= 0 ? e0 : aa) * B2,
                                        false, bs, e0 >= 0 ? -1.0 : 0.0);
                d4_t c = load16(t, ar.Dm + (size_t)aa * B2, bs);
                c = mfma16(o1, c);
                c = mfma16(o0, c);
                store16(t, ar.Dm + (size_t)aa * B2, bs, c);
            } else {
                const int i = task - na, e = st * (2 * i + 1), rr = e + st;
                if (rr < nb) {   // J_{r,l} = -J_{r,e} G_l(e)
                    d4_t c = {0.0, 0.0, 0.0, 0.0};
                    c = mm16(t, ar.Fm + (size_t)rr * B2, false, ar.S1 + (size_t)i * B2, false, bs, -1.0, c);
                    store16(t, ar.S2 + (size_t)i * B2, bs, c);
                }
            }
        }
        __syncthreads();
        for (int e2 = threadIdx.x; e2 < B2; e2 += kThreads) {
            for (int i = 0; i < ne; ++i) {
                const int e = st * (2 * i + 1), rr = e + st;
                ar.Fm[(size_t)e * B2 + e2] = ar.S1[(size_t)i * B2 + e2];
                if (rr < nb) ar.Fm[(size_t)rr * B2 + e2] = ar.S2[(size_t)i * B2 + e2];
            }
        }
        __syncthreads();
    }
    const int r0 = block_invert16<D, AUG>(ar, 0, 1, 1, scale);
    if (r0 < 0) return -1;
    return neg + r0;
}

// Block-vector products for bs <= 16 on the vector ALU.  With one to three right-hand sides
// a 16 x 16 x 4 FP64 matrix instruction would leave most of its columns empty, and on this
// chip FP64 matrix and vector throughput are equal, so a wavefront splits each row's dot
// product over four lanes instead: lane (i = l % 16, kq = l / 16) takes the columns
// k = 4 j + kq, and two cross-row additions (lane swaps across rows of 16) give every lane
// the sum of row i.  All four lanes of a row then hold the same value, so lane kq stores column kq.
template <int R>
struct MvqOps {
    double av[4], xv[R][4];
};
// operands of one product, loaded at fixed offsets from one base: entries outside the block
// are read (the arena continues past every block and right-hand side) and zeroed in mvq_fma
template <int R>
__device__ __forceinline__ MvqOps<R> mvq_load(const Tile& t, const double* A, bool ta, const double* x, int N,
                                              int bs) {
    MvqOps<R> o;
    const double* a0 = A + (ta ? t.kq * bs + t.i : t.i * bs + t.kq);
    const int da = ta ? 4 * bs : 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) o.av[j] = a0[j * da];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) o.xv[q][j] = x[(size_t)q * N + 4 * j + t.kq];
    return o;
}
// acc += s op(A) X over this lane's columns (s = 0 drops a missing neighbour)
template <int R>
__device__ __forceinline__ void mvq_fma(const Tile& t, const MvqOps<R>& o, int bs, double s, double (&acc)[R]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * j + t.kq;
        const double a = (t.i < bs && k < bs) ? s * o.av[j] : 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = fma(a, k < bs ? o.xv[q][j] : 0.0, acc[q]);
    }
}
template <int R>
__device__ __forceinline__ void mvq_reduce(double (&acc)[R]) {
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = xsum32(xsum16(acc[q]));
}
// block solve for bs <= 16: one wavefront per block, all R (<= 4) right-hand sides at once
template <int D, bool AUG, int R>
__device__ __forceinline__ void bcr_solve16(Arena<D, AUG>& ar, double* rhs) {
    static_assert(R >= 1 && R <= 4, "one lane quarter stores each right-hand side");
    const int N = ar.z.N, nb = ar.z.nb, bs = ar.z.bs, B2 = ar.z.B2;
    const int wid = threadIdx.x >> 6;
    const Tile t = tile_lane();
    const bool writer = t.i < bs;
    __syncthreads();
    int top = 1;
    while (2 * top < nb) top *= 2;
    // down: b_a -= G_l(e1)^T b_e1 + G_r(e0)^T b_e0
    for (int st = 1; st < nb; st *= 2) {
        const int na = (nb - 1) / (2 * st) + 1;
        #pragma unroll 1
        for (int ka = wid; ka < na; ka += kWaves) {
            const int aa = 2 * st * ka, e1 = aa + st, e0 = aa - st;
            double acc[R];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = 0.0;
            // (a missing neighbour reads block aa and is scaled by zero)
            const int b1 = e1 < nb ? e1 : aa, b0 = e0 >= 0 ? e0 : aa;
            const MvqOps<R> o1 = mvq_load<R>(t, ar.Fm + (size_t)b1 * B2, true, rhs + b1 * bs, N, bs);
            const MvqOps<R> o0 = mvq_load<R>(t, ar.Rm + (size_t)b0 * B2, true, rhs + b0 * bs, N, bs);
            mvq_fma<R>(t, o1, bs, e1 < nb ? 1.0 : 0.0, acc);
            mvq_fma<R>(t, o0, bs, e0 >= 0 ? 1.0 : 0.0, acc);
            mvq_reduce<R>(acc);
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (writer && t.kq == q) rhs[(size_t)q * N + aa * bs + t.i] -= acc[q];
        }
        __syncthreads();
    }
    // last block, then up: x_e = P_e b_e - G_l(e) x_l - G_r(e) x_r (in place: only this
    // wavefront reads b_e, and every lane has read it before the reduction)
    if (wid == 0) {
        double acc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = 0.0;
        mvq_fma<R>(t, mvq_load<R>(t, ar.Dm, false, rhs, N, bs), bs, 1.0, acc);
        mvq_reduce<R>(acc);
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (writer && t.kq == q) rhs[(size_t)q * N + t.i] = acc[q];
    }
    __syncthreads();
    if (nb > 1) {
        for (int st = top; st >= 1; st /= 2) {
            int ne = 0;
            while (st * (2 * ne + 1) < nb) ++ne;
            #pragma unroll 1
            for (int i = wid; i < ne; i += kWaves) {
                const int e = st * (2 * i + 1), l = e - st, rr = e + st;
                double acc[R];
#pragma unroll
                for (int q = 0; q < R; ++q) acc[q] = 0.0;
                const MvqOps<R> op = mvq_load<R>(t, ar.Dm + (size_t)e * B2, false, rhs + e * bs, N, bs);
                const MvqOps<R> ol = mvq_load<R>(t, ar.Fm + (size_t)e * B2, false, rhs + l * bs, N, bs);
                const MvqOps<R> orr = mvq_load<R>(t, ar.Rm + (size_t)e * B2, false, rhs + (rr < nb ? rr : l) * bs, N, bs);
                mvq_fma<R>(t, op, bs, 1.0, acc);
                mvq_fma<R>(t, ol, bs, -1.0, acc);
                mvq_fma<R>(t, orr, bs, rr < nb ? -1.0 : 0.0, acc);
                mvq_reduce<R>(acc);
#pragma unroll
                for (int q = 0; q < R; ++q)
                    if (writer && t.kq == q) rhs[(size_t)q * N + e * bs + t.i] = acc[q];
            }
            __syncthreads();
        }
    }
}

// Batched Gauss-Jordan inversion of the pivot blocks Dm[first + step*i], i < cnt, in place.
// Steps alternate between the blocks and the scratch S1 (one barrier per step).  Pivots
// are those of an LDL^T of each block; returns the number of negative pivots, or -1 if one
// is zero relative to `scale`.
// Gauss-Jordan inversion of cnt blocks of size bs, in place in bufA (block stride strideA),
// alternating with bufB (stride strideB) at every step (one barrier per step).  Pivots are
// those of an LDL^T of each block; returns the number of negative pivots, or -1 if one is
// zero relative to `scale`.
__device__ __forceinline__ int gj_invert(double* bufA, size_t strideA, double* bufB, size_t strideB, int bs, int cnt,
                                         double scale) {
    const int B2 = bs * bs;
    int neg = 0;
    for (int k = 0; k < bs; ++k) {
        const bool fromA = (k & 1) == 0;
        const double* src = fromA ? bufA : bufB;
        double* dst = fromA ? bufB : bufA;
        const size_t ss = fromA ? strideA : strideB, ds = fromA ? strideB : strideA;
        for (int i0 = 0; i0 < cnt; i0 += 8) {
            double inv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = min(i0 + j, cnt - 1);
                const double piv = src[(size_t)i * ss + k * bs + k];
                if (i0 + j < cnt) {
                    if (!(fabs(piv) > 1e-15 * scale)) return -1;
                    if (piv < 0.0) ++neg;
                }
                inv[j] = 1.0 / piv;
            }
            for (int e2 = threadIdx.x; e2 < B2; e2 += kThreads) {
                const int r = e2 / bs, c = e2 - r * bs;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (i0 + j < cnt) {
                        const double* M = src + (size_t)(i0 + j) * ss;
                        const double mkc = M[k * bs + c], mrk = M[r * bs + k], mrc = M[r * bs + c];
                        double v;
                        if (r == k) v = (c == k) ? inv[j] : mkc * inv[j];
                        else v = (c == k) ? -mrk * inv[j] : mrc - mrk * (mkc * inv[j]);
                        dst[(size_t)(i0 + j) * ds + e2] = v;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (bs & 1) {   // the result sits in the scratch after an odd number of steps
        for (int e2 = threadIdx.x; e2 < B2; e2 += kThreads)
            for (int i = 0; i < cnt; ++i) bufA[(size_t)i * strideA + e2] = bufB[(size_t)i * strideB + e2];
        __syncthreads();
    }
    return neg;
}

// Inversion of the pivot blocks Dm[first + step*i], i < cnt, in place.  With a global-memory
// arena the blocks go through LDS in groups of stage_blocks (the Gauss-Jordan steps then
// touch LDS only); otherwise in place with the scratch S1.
template <int D, bool AUG>
__device__ __forceinline__ int block_invert(Arena<D, AUG>& ar, int first, int step, int cnt, double scale) {
    const int bs = ar.z.bs, B2 = ar.z.B2;
    if (ar.stage_blocks <= 0)
        return gj_invert(ar.Dm + (size_t)first * B2, (size_t)step * B2, ar.S1, B2, bs, cnt, scale);
    int neg = 0;
    for (int g0 = 0; g0 < cnt; g0 += ar.stage_blocks) {
        const int gc = min(ar.stage_blocks, cnt - g0);
        double* A = ar.stage;
        double* Bb = ar.stage + (size_t)gc * B2;
        for (int i = 0; i < gc; ++i) {
            const double* src = ar.Dm + (size_t)(first + step * (g0 + i)) * B2;
            for (int e2 = threadIdx.x; e2 < B2; e2 += kThreads) A[(size_t)i * B2 + e2] = src[e2];
        }
        __syncthreads();
        const int r = gj_invert(A, B2, Bb, B2, bs, gc, scale);
        if (r < 0) return -1;
        neg += r;
        for (int i = 0; i < gc; ++i) {
            double* dst = ar.Dm + (size_t)(first + step * (g0 + i)) * B2;
            for (int e2 = threadIdx.x; e2 < B2; e2 += kThreads) dst[e2] = A[(size_t)i * B2 + e2];
        }
        __syncthreads();
    }
    return neg;
}

template <int D, bool AUG, bool MF>
__device__ __forceinline__ int bcr_factor(Arena<D, AUG>& ar, const Args& a, double alpha, double sigma) {
    constexpr int NS = Geo<D>::NS;
    const int N = ar.z.N, m = ar.z.m, nb = ar.z.nb, bs = ar.z.bs, B2 = ar.z.B2;
    const double H = 1.0 / a.nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
    for (int t = threadIdx.x; t < nb * B2; t += kThreads) {
        ar.Dm[t] = 0.0;
        ar.Fm[t] = 0.0;
    }
    __syncthreads();
    double dmax = 0.0;
    for (int i = threadIdx.x; i < N; i += kThreads) {
        int P[3];
        node_pos<D>(i, m, P);
        const double X[3] = {P[0] * H, P[1] * H, P[2] * H};
        const int blk = i / bs, r = i - blk * bs;
        static_for<Geo<D>::NS>([&](auto sc_) {
            constexpr int s = decltype(sc_)::value;
            const int j = nbr<D, s>(P, m);
            if (j >= 0) {
                double as, bs_;
                stencil_ab<D, s>(X, H, Hd, a.ph, as, bs_);
                const double v = as + alpha * ar.Sst[(size_t)i * NS + s] - sigma * bs_;
                // neighbours lie in the same block row, the previous one or the next one
                const int jb = j < blk * bs ? blk - 1 : (j >= (blk + 1) * bs ? blk + 1 : blk);
                if (jb == blk) ar.Dm[(size_t)blk * B2 + r * bs + (j - jb * bs)] = v;
                else if (jb == blk - 1) ar.Fm[(size_t)blk * B2 + r * bs + (j - jb * bs)] = v;
                if (s == 0) dmax = fmax(dmax, fabs(v));
            }
        });
    }
    const double scale = bmax1(ar.red, dmax);   // (its barriers also publish the blocks)
    if constexpr (MF) return bcr_levels16<D, AUG>(ar, scale);
    int neg = 0;
    for (int st = 1; st < nb; st *= 2) {
        int ne = 0;
        while (st * (2 * ne + 1) < nb) ++ne;
        FMG_T0(t_inv);
        const int r0 = block_invert<D, AUG>(ar, st, 2 * st, ne, scale);
        FMG_TACC(15, t_inv);
        if (r0 < 0) return -1;
        neg += r0;
        // G_l = P_e J_{e,l} -> S1,  G_r = P_e J_{r,e}^T -> Rm[e]
        for (int e2 = threadIdx.x; e2 < B2; e2 += kThreads) {
            const int p = e2 / bs, q = e2 - p * bs;
            for (int i = 0; i < ne; ++i) {
                const int e = st * (2 * i + 1), rr = e + st;
                const double* P = ar.Dm + (size_t)e * B2 + p * bs;
                const double vl = dotn(P, 1, ar.Fm + (size_t)e * B2 + q, bs, bs);
                const double vr = rr < nb ? dotn(P, 1, ar.Fm + (size_t)rr * B2 + q * bs, 1, bs) : 0.0;
                ar.S1[(size_t)i * B2 + e2] = vl;
                ar.Rm[(size_t)e * B2 + e2] = vr;
            }
        }
        __syncthreads();
        // Schur updates of the blocks that stay (a = 2k st), and the new couplings r <- l
        const int na = (nb - 1) / (2 * st) + 1;
        for (int e2 = threadIdx.x; e2 < B2; e2 += kThreads) {
            const int p = e2 / bs, q = e2 - p * bs;
            for (int ka = 0; ka < na; ++ka) {
                const int aa = 2 * st * ka;
                const int e1 = aa + st, e0 = aa - st;
                double v = 0.0;
                if (e1 < nb)   // D_a -= J_{e1,a}^T G_l(e1), e1 = st (2 ka + 1)
                    v += dotn(ar.Fm + (size_t)e1 * B2 + p, bs, ar.S1 + (size_t)ka * B2 + q, bs, bs);
                if (e0 >= 0)   // D_a -= J_{a,e0} G_r(e0)
                    v += dotn(ar.Fm + (size_t)aa * B2 + p * bs, 1, ar.Rm + (size_t)e0 * B2 + q, bs, bs);
                ar.Dm[(size_t)aa * B2 + e2] -= v;
            }
            for (int i = 0; i < ne; ++i) {
                const int e = st * (2 * i + 1), rr = e + st;
                if (rr < nb)   // J_{r,l} = -J_{r,e} G_l(e)
                    ar.S2[(size_t)i * B2 + e2] =
                        -dotn(ar.Fm + (size_t)rr * B2 + p * bs, 1, ar.S1 + (size_t)i * B2 + q, bs, bs);
            }
        }
        __syncthreads();
        for (int e2 = threadIdx.x; e2 < B2; e2 += kThreads) {
            for (int i = 0; i < ne; ++i) {
                const int e = st * (2 * i + 1), rr = e + st;
                ar.Fm[(size_t)e * B2 + e2] = ar.S1[(size_t)i * B2 + e2];
                if (rr < nb) ar.Fm[(size_t)rr * B2 + e2] = ar.S2[(size_t)i * B2 + e2];
            }
        }
        __syncthreads();
    }
    const int r0 = block_invert<D, AUG>(ar, 0, 1, 1, scale);
    if (r0 < 0) return -1;
    return neg + r0;
}

// Solve J X = R for R right-hand sides stored as rhs[q*N + i] with the factor of bcr_factor.
template <int D, bool AUG, int R, bool MF>
__device__ __forceinline__ void bcr_solve(Arena<D, AUG>& ar, double* rhs) {
    if constexpr (MF) {
        bcr_solve16<D, AUG, R>(ar, rhs);
        return;
    }
    const int N = ar.z.N, nb = ar.z.nb, bs = ar.z.bs, B2 = ar.z.B2;
    double* tmp = ar.S1;
    const VecMap vm = vec_map(bs);
    __syncthreads();
    int top = 1;
    while (2 * top < nb) top *= 2;
    FMG_T0(t_dn);
    // down: b_l -= G_l(e)^T b_e, b_r -= G_r(e)^T b_e
    for (int st = 1; st < nb; st *= 2) {
        const int na = (nb - 1) / (2 * st) + 1;
        for (int ka = vm.g; ka < na; ka += vm.G) {
            const int aa = 2 * st * ka, e1 = aa + st, e0 = aa - st;
            for (int p = vm.p0; p < bs; p += vm.pstep) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const double* b = rhs + (size_t)q * N;
                    double v = 0.0;
                    if (e1 < nb) v += dotn(ar.Fm + (size_t)e1 * B2 + p, bs, b + e1 * bs, 1, bs);
                    if (e0 >= 0) v += dotn(ar.Rm + (size_t)e0 * B2 + p, bs, b + e0 * bs, 1, bs);
                    rhs[(size_t)q * N + aa * bs + p] -= v;
                }
            }
        }
        __syncthreads();
    }
    FMG_TACC(12, t_dn);
    FMG_T0(t_tp);
    // last block
    if (vm.g == 0) {
        for (int p = vm.p0; p < bs; p += vm.pstep) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                tmp[q * bs + p] = dotn(ar.Dm + p * bs, 1, rhs + (size_t)q * N, 1, bs);
            }
        }
    }
    __syncthreads();
    if (vm.g == 0) {
        for (int p = vm.p0; p < bs; p += vm.pstep) {
#pragma unroll
            for (int q = 0; q < R; ++q) rhs[(size_t)q * N + p] = tmp[q * bs + p];
        }
    }
    __syncthreads();
    FMG_TACC(13, t_tp);
    FMG_T0(t_upp);
    // up: x_e = P_e b_e - G_l(e) x_l - G_r(e) x_r
    if (nb > 1) {
        for (int st = top; st >= 1; st /= 2) {
            int ne = 0;
            while (st * (2 * ne + 1) < nb) ++ne;
            for (int i = vm.g; i < ne; i += vm.G) {
                const int e = st * (2 * i + 1), l = e - st, rr = e + st;
                for (int p = vm.p0; p < bs; p += vm.pstep) {
                    const double* P = ar.Dm + (size_t)e * B2 + p * bs;
                    const double* Gl = ar.Fm + (size_t)e * B2 + p * bs;
                    const double* Gr = ar.Rm + (size_t)e * B2 + p * bs;
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const double* b = rhs + (size_t)q * N;
                        double v = dotn(P, 1, b + e * bs, 1, bs) - dotn(Gl, 1, b + l * bs, 1, bs);
                        if (rr < nb) v -= dotn(Gr, 1, b + rr * bs, 1, bs);
                        tmp[((size_t)q * ne + i) * bs + p] = v;
                    }
                }
            }
            __syncthreads();
            for (int i = vm.g; i < ne; i += vm.G) {
                const int e = st * (2 * i + 1);
                for (int p = vm.p0; p < bs; p += vm.pstep) {
#pragma unroll
                    for (int q = 0; q < R; ++q) rhs[(size_t)q * N + e * bs + p] = tmp[((size_t)q * ne + i) * bs + p];
                }
            }
            __syncthreads();
        }
    }
    FMG_TACC(14, t_upp);
}

// One Newton solve at coupling zs from the iterate in ar.x, using (and refreshing) the
// factor.  `have` says whether the arena already holds a usable factor.  Returns
// iterations >= 0 on convergence, or -reason.  mu in sc[6], factorisations added to sc[8].
//
// Steps are chord steps with a frozen bordered Jacobian
//     M = [ J   C ]     J = A + 3 zs S - mu B (coarse block, factored),
//         [ C^T E ]     C = border columns (d/dc and d/dmu), E = 2x2 (or 1x1) corner,
// all taken at the last refresh.  With V = J^{-1} C (kept in rhs[N..]) and the Schur
// complement G = E - C^T V, a step is
//     y0 = J^{-1}(-F_H),  G dbeta = r_beta - C^T y0,  dx_H = y0 - V dbeta,
// and because J is symmetric C^T y0 = -V^T F_H, so one right-hand side per step suffices.
// A refresh (new factor, or first step of a call with a stored factor) freezes the
// current border columns again.
template <int D, bool AUG, bool MF>
__device__ __forceinline__ int newton(Arena<D, AUG>& ar, const Args& a, double zs, double tol, bool& have) {
    const int N = ar.z.N, N1 = ar.z.N1, m = ar.z.m;
    const int tid = threadIdx.x;
    FMG_TCNT(9);
    if constexpr (AUG) {
        // the bordered solve starts from u = c u~ (x_H = 0): ||x||_B^2 = c^2 b(u~, u~)
        const double c = ar.x[N];
        const double sN = 1.0 / sqrt(c * (ar.sc[1] * c));
        for (int i = tid; i < N1; i += kThreads) ar.x[i] *= sN;
        __syncthreads();
    } else {
        // x <- x / ||x||_B  (B needs no assembly)
        const double H = 1.0 / a.nc;
        const double Hd = (D == 2) ? H * H : H * H * H;
        double v[2] = {0.0, 0.0};
        const double c = AUG ? ar.x[N] : 0.0;
        for (int i = tid; i < N; i += kThreads) {
            int P[3];
            node_pos<D>(i, m, P);
            const double X[3] = {P[0] * H, P[1] * H, P[2] * H};
            double zi = 0.0;
            static_for<Geo<D>::NS>([&](auto sc_) {
                constexpr int s = decltype(sc_)::value;
                const int j = nbr<D, s>(P, m);
                double as, bs;
                stencil_ab<D, s>(X, H, Hd, a.ph, as, bs);
                zi += bs * nbr_val(ar.x, j);
            });
            v[0] += ar.x[i] * zi;
            if (AUG) v[1] += ar.bH[i] * ar.x[i];
        }
        bsum<2>(ar.red, v);
        const double xbx = v[0] + (AUG ? c * (2.0 * v[1] + ar.sc[1] * c) : 0.0);
        const double sN = 1.0 / sqrt(xbx);
        for (int i = tid; i < N1; i += kThreads) ar.x[i] *= sN;
        __syncthreads();
    }
    double mu = 0.0, mus = 0.0, res_prev = 1e300;
    double mu_prev = 0.0, fmu_prev = 0.0;   // acceleration history (mu part)
    bool aa_have = false;
    bool last_fresh = false, need_fresh = !have, frozen = false;
    double g11 = 0.0, g12 = 0.0, g21 = 0.0, g22 = 1.0;   // frozen Schur complement G
    for (int it = 0; it <= a.max_iter; ++it) {
        FMG_TCNT(8);
        FMG_T0(t_as);
        // a chord step reuses the frozen Jacobian and border columns: residual only
        const bool direct = frozen && !need_fresh && direct_ok<D, AUG>(ar);
        if (!direct) assemble_S<D, AUG>(ar, a, ar.x);
        ar.s_stale = direct;
        FMG_TACC(1, t_as);
        FMG_T0(t_ap);
        if constexpr (AUG) {
            if (direct) apply_direct<D, AUG>(ar, a, zs, ar.x, ar.y, ar.z2);
            else apply<D, AUG>(ar, a, zs, ar.x, ar.y, ar.z2);
        } else {
            apply<D, AUG>(ar, a, zs, ar.x, ar.y, ar.z2);
        }
        if (it == 0) mu = ar.sc[4] / ar.sc[5];
        const double F2 = 0.5 * (1.0 - ar.sc[5]);
        double fz[2] = {0.0, 0.0};
        for (int i = tid; i < N1; i += kThreads) {
            const double f = ar.y[i] - mu * ar.z2[i];
            ar.F[i] = f;
            fz[0] += f * f;
            fz[1] += ar.z2[i] * ar.z2[i];
        }
        bsum<2>(ar.red, fz);
        const double res = sqrt(fz[0]) / (fabs(mu) * sqrt(fz[1]));
        if (tid == 0) ar.sc[7] = res;
        if (!(res == res) || !(mu == mu)) return -3;
        // x^T B x = 1 up to the rounding of an N-term dot product; an intermediate stage of
        // the coarse continuation (tol above the requested one) only needs tol
        const double f2_tol = tol > a.tol ? tol : 4.0 * N1 * 1.1e-16;
        if ((res <= tol && fabs(F2) <= f2_tol) || (AUG && a.fixed_iters > 0 && it == a.fixed_iters)) {
            const double sN = 1.0 / sqrt(ar.sc[5]);
            for (int i = tid; i < N1; i += kThreads) ar.x[i] *= sN;
            if (tid == 0) ar.sc[6] = mu;
            __syncthreads();
            return it;
        }
        FMG_TACC(2, t_ap);
        if (it == a.max_iter) return -2;
        if (it > 0 && !last_fresh && res > 0.25 * res_prev) {
            // the frozen Jacobian stopped contracting: back to the previous iterate, refactor
            for (int i = tid; i < N1; i += kThreads) ar.x[i] = ar.xs[i];
            mu = mus;
            need_fresh = true;
            res_prev = 1e300;
            aa_have = false;
            __syncthreads();
            continue;
        }
        if (need_fresh) {
            FMG_T0(t_f);
            if (bcr_factor<D, AUG, MF>(ar, a, 3.0 * zs, mu) < 0) return -1;
            FMG_TACC(3, t_f);
            FMG_TCNT(12);
            need_fresh = false;
            last_fresh = true;
            frozen = false;
            have = true;
            aa_have = false;
            if (tid == 0) ar.sc[8] += 1.0;
        } else {
            last_fresh = false;
        }
        for (int i = tid; i < N1; i += kThreads) ar.xs[i] = ar.x[i];
        mus = mu;
        res_prev = res;
        FMG_T0(t_s);
        if (!frozen) {
            // freeze the border columns at this iterate: V = J^{-1} C
            for (int i = tid; i < N; i += kThreads) {
                ar.rhs[i] = -ar.F[i];
                if (AUG) {
                    ar.rhs[N + i] = ar.aH[i] + 3.0 * zs * ar.sH[i] - mu * ar.bH[i];
                    ar.rhs[2 * N + i] = -ar.z2[i];
                } else {
                    ar.rhs[N + i] = -ar.z2[i];
                }
            }
            bcr_solve<D, AUG, AUG ? 3 : 2, MF>(ar, ar.rhs);
            if (AUG) {
                double s[4] = {0.0, 0.0, 0.0, 0.0};
                for (int i = tid; i < N; i += kThreads) {
                    const double jh = ar.aH[i] + 3.0 * zs * ar.sH[i] - mu * ar.bH[i];
                    const double zh = ar.z2[i];
                    s[0] += jh * ar.rhs[N + i];
                    s[1] += jh * ar.rhs[2 * N + i];
                    s[2] += zh * ar.rhs[N + i];
                    s[3] += zh * ar.rhs[2 * N + i];
                }
                bsum<4>(ar.red, s);
                const double jU = ar.sc[0] + 3.0 * zs * ar.sc[3] - mu * ar.sc[1];
                const double zU = ar.z2[N];
                g11 = jU - s[0];
                g12 = -s[1] - zU;
                g21 = s[2] - zU;
                g22 = s[3];
            } else {
                double s1 = 0.0;
                for (int i = tid; i < N; i += kThreads) s1 += ar.z2[i] * ar.rhs[N + i];
                g22 = bsum1(ar.red, s1);
            }
            frozen = true;
        } else {
            for (int i = tid; i < N; i += kThreads) ar.rhs[i] = -ar.F[i];
            bcr_solve<D, AUG, 1, MF>(ar, ar.rhs);
        }
        FMG_TACC(4, t_s);
        FMG_T0(t_u);
        // C^T y0 = -V^T F_H; the chord step (dx, dmu) goes to y (free until the next apply)
        double dmu, dc = 0.0;
        double* dx = ar.y;
        if (AUG) {
            double p[2] = {0.0, 0.0};
            for (int i = tid; i < N; i += kThreads) {
                p[0] += ar.rhs[N + i] * ar.F[i];
                p[1] += ar.rhs[2 * N + i] * ar.F[i];
            }
            bsum<2>(ar.red, p);
            // C = [j_H, -z_H]: C^T y0 = -V^T F_H = (-p1, -p2), so j_H.y0 = -p1, z_H.y0 = p2
            const double r1 = -ar.F[N] + p[0], r2 = -F2 + p[1];
            const double det = g11 * g22 - g12 * g21;
            if (!(fabs(det) > 0.0)) return -4;
            dc = (r1 * g22 - g12 * r2) / det;
            dmu = (g11 * r2 - g21 * r1) / det;
            for (int i = tid; i < N; i += kThreads) dx[i] = ar.rhs[i] - ar.rhs[N + i] * dc - ar.rhs[2 * N + i] * dmu;
            if (tid == 0) dx[N] = dc;
        } else {
            double p1 = 0.0;
            for (int i = tid; i < N; i += kThreads) p1 += ar.rhs[N + i] * ar.F[i];
            p1 = bsum1(ar.red, p1);
            if (!(fabs(g22) > 0.0)) return -4;
            dmu = (-F2 + p1) / g22;   // z.y0 = p1 with V = J^{-1}(-z)
            for (int i = tid; i < N; i += kThreads) dx[i] = ar.rhs[i] - ar.rhs[N + i] * dmu;
        }
        __syncthreads();
        // Anderson acceleration (one previous pair) of the chord map z -> z + dz, z = (x, mu):
        // gamma minimises |dz - gamma (dz - dz_prev)|, z <- z + dz - gamma (z - z_prev + dz - dz_prev).
        // The history restarts whenever the frozen Jacobian changes.
        double gamma = 0.0;
        if (aa_have) {
            double v[2] = {0.0, 0.0};
            for (int i = tid; i < N1; i += kThreads) {
                const double df = dx[i] - ar.fp[i];
                v[0] += df * dx[i];
                v[1] += df * df;
            }
            if (tid == 0) {
                const double dfm = dmu - fmu_prev;
                v[0] += dfm * dmu;
                v[1] += dfm * dfm;
            }
            bsum<2>(ar.red, v);
            gamma = v[1] > 0.0 ? v[0] / v[1] : 0.0;
        }
        for (int i = tid; i < N1; i += kThreads) {
            const double xi = ar.x[i], di = dx[i];
            ar.x[i] = xi + di - gamma * ((xi - ar.xp[i]) + (di - ar.fp[i]));
            ar.xp[i] = xi;
            ar.fp[i] = di;
        }
        {
            const double mnew = mu + dmu - gamma * ((mu - mu_prev) + (dmu - fmu_prev));
            mu_prev = mu;
            fmu_prev = dmu;
            mu = mnew;
        }
        aa_have = true;
        __syncthreads();
        FMG_TACC(5, t_u);
    }
    return -2;
}

// inertia check: number of eigenvalues of (A + zs S(x), B) below sigma (0: ground state)
template <int D, bool AUG, bool MF>
__device__ __forceinline__ int count_below(Arena<D, AUG>& ar, const Args& a, double zs, double sigma) {
    const int N = ar.z.N;
    if (ar.s_stale) {   // the last steps evaluated the residual only
        assemble_S<D, AUG>(ar, a, ar.x);
        ar.s_stale = false;
    }
    int neg = bcr_factor<D, AUG, MF>(ar, a, zs, sigma);
    if (neg < 0) return 1;
    if (AUG) {
        for (int i = threadIdx.x; i < N; i += kThreads) ar.rhs[i] = ar.aH[i] + zs * ar.sH[i] - sigma * ar.bH[i];
        bcr_solve<D, AUG, 1, MF>(ar, ar.rhs);
        double s = 0.0;
        for (int i = threadIdx.x; i < N; i += kThreads)
            s += (ar.aH[i] + zs * ar.sH[i] - sigma * ar.bH[i]) * ar.rhs[i];
        s = bsum1(ar.red, s);
        const double schur = (ar.sc[0] + zs * ar.sc[3] - sigma * ar.sc[1]) - s;
        if (!(schur > 0.0)) ++neg;
    }
    return neg;
}

template <int D, bool AUG>
__device__ __forceinline__ void store_factor(Arena<D, AUG>& ar, const Args& a) {
    if (!a.fac) return;
    const int n = 3 * ar.z.nb * ar.z.B2;
    for (int t = threadIdx.x; t < n; t += kThreads) a.fac[t] = ar.Dm[t];
    if (threadIdx.x == 0) a.st->fac_valid = 1;
}

template <int D, bool AUG, bool MF>
__device__ __forceinline__ void finish(Arena<D, AUG>& ar, const Args& a, int iters, bool ok, int reason) {
    const int N = ar.z.N, m = ar.z.m;
    const double H = 1.0 / a.nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
    if (ok) {
        const double mu = ar.sc[6];
        // certify 1: always; 2: only when this step meets the lambda tolerance
        const double prev = a.st->lambda;
        const bool meets = AUG && a.final_level && a.st->tol_lambda > 0.0 &&
                           fabs(mu - prev) / fabs(mu) <= a.st->tol_lambda;
        const bool cert = a.certify == 1 || (a.certify == 2 && meets);
        int below = 0;
        FMG_T0(t_cb);
        if (cert) below = count_below<D, AUG, MF>(ar, a, a.ph.zeta, mu - 1e-9 * fabs(mu));
        FMG_TACC(7, t_cb);
        // sign: int u_h > 0
        double v = 0.0;
        for (int i = threadIdx.x; i < N; i += kThreads) v += ar.x[i];
        v = bsum1(ar.red, v);
        const double integ = Hd * v + (AUG ? ar.x[N] * ar.sc[2] : 0.0);
        const double sgn = integ < 0.0 ? -1.0 : 1.0;
        for (int i = threadIdx.x; i < N; i += kThreads) {
            int P[3];
            node_pos<D>(i, m, P);
            a.xc[P[0] + a.gc.pitch * P[1] + a.gc.plane * P[2]] = sgn * ar.x[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            SmallState* st = a.st;
            st->lambda_prev = prev;
            st->lambda = mu;
            st->dlambda = fabs(mu - prev) / fabs(mu);
            st->c = AUG ? sgn * ar.x[N] : 0.0;
            st->newton_total += iters;
            st->fact_total += (int)ar.sc[8] + (cert ? 1 : 0);
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
            if (meets) st->done = 1;
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

template <int D, bool AUG, bool LDS, bool MF>
__global__ __launch_bounds__(kThreads) void k_newton(Args a) {
    extern __shared__ double lds[];
    Arena<D, AUG> ar;
    if constexpr (LDS) {
        ar.carve(lds, a.nc);
    } else {
        ar.carve(a.arena, a.nc);
        ar.stage = lds;
        ar.stage_blocks = a.stage_blocks;
    }
    if (AUG && a.st->done) return;   // tolerance loop already satisfied
    FMG_T0(t_all);
    FMG_T0(t_setup);
    if (AUG) bind_moments<D, AUG>(ar, a, lds, LDS && a.mstage);
    setup<D, AUG>(ar, a);
    FMG_TACC(0, t_setup);
    const int N = ar.z.N, m = ar.z.m;
    const int tid = threadIdx.x;
    if (tid == 0) ar.sc[8] = 0.0;
    // a stored factor of the coarse Jacobian block (previous call) seeds chord steps
    bool have = false;
    if (a.reuse && a.fac && a.st->fac_valid) {
        // kB loads in flight per thread before their stores (clamped addresses stay in bounds)
        constexpr int kB = 16;
        const int n = 3 * ar.z.nb * ar.z.B2;
        for (int t0 = tid; t0 < n; t0 += kThreads * kB) {
            double v[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) v[u] = a.fac[min(t0 + u * kThreads, n - 1)];
#pragma unroll
            for (int u = 0; u < kB; ++u)
                if (t0 + u * kThreads < n) ar.Dm[t0 + u * kThreads] = v[u];
        }
        have = true;
    }
    __syncthreads();
    int iters = 0;
    bool ok = true;
    int reason = 0;
    if (AUG) {
        // start from u = u~ / ||u~||_M
        for (int i = tid; i < N; i += kThreads) ar.x[i] = 0.0;
        if (tid == 0) ar.x[N] = 1.0;
        __syncthreads();
        int r = newton<D, AUG, MF>(ar, a, a.ph.zeta, a.tol, have);
        ok = r >= 0;
        iters = ok ? r : 0;
        reason = ok ? 0 : -r;
    } else {
        // discrete sine mode, then zeta stages (first stage <= 16, factor 8); a failed stage
        // goes back to the last converged iterate and retries with half the step
        const double H = 1.0 / a.nc;
        for (int i = tid; i < N; i += kThreads) {
            int P[3];
            node_pos<D>(i, m, P);
            double v = sinpi(P[0] * H) * sinpi(P[1] * H);
            if (D == 3) v *= sinpi(P[2] * H);
            ar.x[i] = v;
        }
        __syncthreads();
        const double zeta = a.ph.zeta;
        const bool direct = !(zeta > kFirstStage);
        const double lf = log(8.0);
        const double lt = direct ? 0.0 : log(zeta);
        const int J = direct ? 0 : (int)ceil((lt - log(kFirstStage)) / lf - 1e-12);
        double lnext = lt - J * lf, step = lf, lcur = 0.0;
        bool have_cur = false;
        int first_tries = 0;
        for (int guard = 0; guard < 200; ++guard) {
            const bool last = direct || !(lnext < lt);
            const double z = last ? zeta : exp(lnext);
            for (int i = tid; i < N; i += kThreads) ar.xk[i] = ar.x[i];   // committed iterate
            __syncthreads();
            // a new coupling changes the 3 zeta S term of the Jacobian by up to a factor 8:
            // factor afresh; intermediate stages only seed the next one (looser residual)
            have = false;
            const int rr = newton<D, AUG, MF>(ar, a, z, last ? a.tol : fmax(a.tol, kStageTol), have);
            if (rr < 0) {
                for (int i = tid; i < N; i += kThreads) ar.x[i] = ar.xk[i];
                have = false;
                __syncthreads();
                if (direct) { ok = false; reason = -rr; break; }
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
    __syncthreads();
#ifdef FMG_SMALL_MICRO
    // measurement build only: repeat phases on the converged state (results are discarded)
    if (AUG && ok) {
        unsigned long long tt[8];
        const int reps = 50;
        __syncthreads();
        tt[0] = wall_clock64();
        for (int r = 0; r < reps; ++r) assemble_S<D, AUG>(ar, a, ar.x);
        __syncthreads();
        tt[1] = wall_clock64();
        for (int r = 0; r < reps; ++r) apply<D, AUG>(ar, a, a.ph.zeta, ar.x, ar.y, ar.z2);
        __syncthreads();
        tt[2] = wall_clock64();
        for (int r = 0; r < reps; ++r) bcr_solve<D, AUG, 1, MF>(ar, ar.rhs);
        __syncthreads();
        tt[3] = wall_clock64();
        for (int r = 0; r < reps; ++r) bcr_solve<D, AUG, 3, MF>(ar, ar.rhs);
        __syncthreads();
        tt[4] = wall_clock64();
        for (int r = 0; r < 10; ++r) bcr_factor<D, AUG, MF>(ar, a, 3.0 * a.ph.zeta, ar.sc[6]);
        __syncthreads();
        tt[5] = wall_clock64();
        double acc = 0.0;
        for (int r = 0; r < reps; ++r) acc += bsum1(ar.red, (double)r);
        __syncthreads();
        tt[6] = wall_clock64();
        for (int r = 0; r < reps; ++r) __syncthreads();
        tt[7] = wall_clock64();
        unsigned long long tu[4];
        tu[0] = wall_clock64();
        if constexpr (MF) {
            int sink = 0;
            for (int r = 0; r < 10; ++r) sink += block_invert16<D, AUG>(ar, 1, 2, (ar.z.nb - 1) / 2, 1e-300);
            __syncthreads();
            tu[1] = wall_clock64();
            for (int r = 0; r < 10; ++r) sink += block_invert16<D, AUG>(ar, 0, 1, 1, 1e-300);
            __syncthreads();
            tu[2] = wall_clock64();
            for (int r = 0; r < 10; ++r) sink += bcr_levels16<D, AUG>(ar, 1e-300);
            __syncthreads();
            tu[3] = wall_clock64();
            if (threadIdx.x == 0 && sink == 12345) g_small_t[31] = 1;
        } else {
            tu[1] = tu[2] = tu[3] = tu[0];
        }
        unsigned long long td0 = wall_clock64(), td1 = td0;
        if constexpr (D == 3 && AUG) {
            for (int r = 0; r < reps; ++r) apply_direct<D, AUG>(ar, a, a.ph.zeta, ar.x, ar.y, ar.z2);
            __syncthreads();
            td1 = wall_clock64();
        }
        unsigned long long te[5];
        te[0] = wall_clock64();
        if constexpr (D == 2 && AUG) {
            if (direct_ok<D, AUG>(ar))
                for (int r = 0; r < reps; ++r) apply_direct<D, AUG>(ar, a, a.ph.zeta, ar.x, ar.y, ar.z2);
        }
        __syncthreads();
        te[1] = wall_clock64();
        if (a.fac) {
            const int nf = 3 * ar.z.nb * ar.z.B2;
            for (int r = 0; r < 10; ++r) {
                constexpr int kB = 16;
                for (int t0 = threadIdx.x; t0 < nf; t0 += kThreads * kB) {
                    double vv[kB];
#pragma unroll
                    for (int u = 0; u < kB; ++u) vv[u] = a.fac[min(t0 + u * kThreads, nf - 1)];
#pragma unroll
                    for (int u = 0; u < kB; ++u)
                        if (t0 + u * kThreads < nf) ar.Dm[t0 + u * kThreads] = vv[u];
                }
                __syncthreads();
            }
        }
        te[2] = wall_clock64();
        for (int r = 0; r < 10; ++r) setup<D, AUG>(ar, a);
        __syncthreads();
        te[3] = wall_clock64();
        for (int r = 0; r < reps; ++r) {
            double fz[2] = {0.0, 0.0};
            for (int i = threadIdx.x; i < ar.z.N1; i += kThreads) {
                const double f = ar.y[i] - 1.5 * ar.z2[i];
                ar.F[i] = f;
                fz[0] += f * f;
                fz[1] += ar.z2[i] * ar.z2[i];
            }
            bsum<2>(ar.red, fz);
            acc += fz[0] * 1e-300;
        }
        __syncthreads();
        te[4] = wall_clock64();
        if (threadIdx.x == 0) {
            for (int k = 0; k < 4; ++k) atomicAdd(&g_small_t[16 + k], te[k + 1] - te[k]);
            atomicAdd(&g_small_t[12], td1 - td0);
            for (int k = 0; k < 3; ++k) atomicAdd(&g_small_t[9 + k], tu[k + 1] - tu[k]);
            for (int k = 0; k < 7; ++k) atomicAdd(&g_small_t[k], tt[k + 1] - tt[k]);
            atomicAdd(&g_small_t[7], 1ull);
            atomicAdd(&g_small_t[8], acc < 0.0 ? 1ull : 0ull);
        }
    }
#endif
    FMG_T0(t_fin);
    if (ok && ar.sc[8] > 0.0) store_factor<D, AUG>(ar, a);
    __syncthreads();
    finish<D, AUG, MF>(ar, a, iters, ok, reason);
    FMG_TACC(6, t_fin);
    FMG_TACC(10, t_all);
    FMG_TCNT(11);
}

// dense A, B, S(x) of the augmented problem (tests)
template <int D, bool LDS>
__global__ __launch_bounds__(kThreads) void k_aug_dump(Args a) {
    extern __shared__ double lds[];
    Arena<D, true> ar;
    if constexpr (LDS) ar.carve(lds, a.nc);
    else ar.carve(a.arena, a.nc);
    bind_moments<D, true>(ar, a, lds, false);
    setup<D, true>(ar, a);
    constexpr int NS = Geo<D>::NS;
    const int N = ar.z.N, N1 = N + 1, m = ar.z.m;
    const double H = 1.0 / a.nc;
    const double Hd = (D == 2) ? H * H : H * H * H;
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
        int P[3];
        node_pos<D>(i, m, P);
        const double X[3] = {P[0] * H, P[1] * H, P[2] * H};
        for_slots<D>([&](auto sc_) {
            constexpr int s = decltype(sc_)::value;
            const int j = nbr<D, s>(P, m);
            if (j >= 0) {
                double as, bs;
                stencil_ab<D, s>(X, H, Hd, a.ph, as, bs);
                a.Aout[(size_t)i * N1 + j] = as;
                a.Bout[(size_t)i * N1 + j] = bs;
                a.Sout[(size_t)i * N1 + j] = ar.Sst[(size_t)i * NS + s];
            }
        });
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

// the whole arena in LDS when it fits (gfx950: 160 KiB per workgroup); a build may lower the
// limit (FMG_SMALL_LDS_LIMIT) to exercise the global-memory arena on small problems
#ifndef FMG_SMALL_LDS_LIMIT
#define FMG_SMALL_LDS_LIMIT (156 * 1024)
#endif
constexpr size_t kLdsLimit = FMG_SMALL_LDS_LIMIT;

// blocks of the coarse Jacobian: grid rows (2D) or planes (3D); up to 16 x 16, with the arena
// in LDS, they go to the matrix cores (the global-arena build of that path would spill)
inline bool small_blocks(int dim, int nc, size_t bytes) {
    const int m = nc - 1;
    return (dim == 2 ? m : m * m) <= 16 && bytes <= kLdsLimit;
}

// blocks a global-arena kernel inverts at a time in LDS (two buffers of B2 doubles each)
inline int stage_blocks_for(int dim, int nc) {
    const int m = nc - 1, bs = dim == 2 ? m : m * m, nb = m;
    const size_t pair = 2 * sizeof(double) * (size_t)bs * bs;
    const int most = (nb + 1) / 2;   // pivot blocks inverted together at the first level
    return (int)std::min<size_t>(most, kLdsLimit / pair);
}

template <typename K>
int launch_small(K kern_lds, K kern_glb, size_t bytes, Args& a, hipStream_t s) {
    a.use_lds = bytes <= kLdsLimit;
    const int dim = a.gc.dim;
    a.stage_blocks = a.use_lds ? 0 : stage_blocks_for(dim, a.nc);
    const int m = a.nc - 1, bs = dim == 2 ? m : m * m;
    size_t shm = a.use_lds ? bytes : 2 * sizeof(double) * (size_t)bs * bs * a.stage_blocks;
    K kern = a.use_lds ? kern_lds : kern_glb;
    if (shm > 64 * 1024) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm) != hipSuccess)
            return FMG_EHIP;
    }
    hipLaunchKernelGGL(kern, dim3(1), dim3(kThreads), shm, s, a);
    return hipGetLastError() == hipSuccess ? 0 : FMG_EHIP;
}

}  // namespace

#if defined(FMG_SMALL_TIMING) || defined(FMG_SMALL_MICRO)
extern "C" int fmg_debug_small_timers(double* out, int reset) {
    unsigned long long h[32];
    if (hipMemcpyFromSymbol(h, HIP_SYMBOL(g_small_t), sizeof(h)) != hipSuccess) return -5;
    for (int k = 0; k < 32; ++k) out[k] = (double)h[k];
    if (reset) {
        unsigned long long z[32] = {};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_small_t), z, sizeof(z)) != hipSuccess) return -5;
    }
    return 0;
}
#endif

// the global arena of a solve: the arena itself (used when it does not fit in LDS), then the
// per-simplex scratch of the 3D assembly (always in global memory)
static size_t arena_part(int dim, int nc) {
    size_t a = dim == 2 ? std::max(arena_bytes_t<2, true>(nc), arena_bytes_t<2, false>(nc))
                        : std::max(arena_bytes_t<3, true>(nc), arena_bytes_t<3, false>(nc));
    return (a + 255) / 256 * 256;
}
static size_t esc_bytes(int dim, int nc) {
    const size_t nel = (dim == 2 ? (size_t)nc * nc * 2 : (size_t)nc * nc * nc * 6);
    return (nel * kEsc * sizeof(double) + 255) / 256 * 256;
}
static double* esc_of(double* arena, int dim, int nc) { return arena + arena_part(dim, nc) / sizeof(double); }

size_t small_arena_bytes(int dim, int nc) { return arena_part(dim, nc) + esc_bytes(dim, nc); }

size_t small_factor_bytes(int dim, int nc) {
    const size_t n = dim == 2 ? factor_doubles<2>(nc) : factor_doubles<3>(nc);
    return (n * sizeof(double) + 255) / 256 * 256;
}

int launch_coarse_newton(int dim, int nc, const Phys& ph, int max_iter, double tol, double* arena, double* fac,
                         double* xc_level, SmallState* state, hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.max_iter = max_iter; a.tol = tol; a.mom = nullptr; a.arena = arena;
    a.xc = xc_level; a.gc = make_grid(dim, nc); a.st = state; a.final_level = 0; a.certify = 1;
    a.fac = fac; a.reuse = 0; a.esc = esc_of(arena, dim, nc);
    if (dim == 2) {
        const size_t b = arena_bytes_t<2, false>(nc);
        return small_blocks(2, nc, b) ? launch_small(k_newton<2, false, true, true>, k_newton<2, false, true, true>, b, a, s)
                                      : launch_small(k_newton<2, false, true, false>, k_newton<2, false, false, false>, b, a, s);
    }
    const size_t b = arena_bytes_t<3, false>(nc);
    return small_blocks(3, nc, b) ? launch_small(k_newton<3, false, true, true>, k_newton<3, false, true, true>, b, a, s)
                                  : launch_small(k_newton<3, false, true, false>, k_newton<3, false, false, false>, b, a, s);
}

int launch_aug_newton(int dim, int nc, const Phys& ph, int max_iter, int fixed_iters, double tol, const double* moments,
                      double* arena,
                      double* fac, double* xc_level, SmallState* state, int final_level, int certify, int reuse,
                      hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.max_iter = max_iter; a.fixed_iters = fixed_iters; a.tol = tol; a.mom = moments;
    a.arena = arena;
    a.xc = xc_level; a.gc = make_grid(dim, nc); a.st = state; a.final_level = final_level;
    a.certify = certify; a.fac = fac; a.reuse = reuse; a.esc = esc_of(arena, dim, nc);
    if (dim == 2) {
        const size_t b = arena_bytes_t<2, true>(nc);
        return small_blocks(2, nc, b) ? launch_small(k_newton<2, true, true, true>, k_newton<2, true, true, true>, b, a, s)
                                      : launch_small(k_newton<2, true, true, false>, k_newton<2, true, false, false>, b, a, s);
    }
    // the moments go to LDS after the arena when both fit
    const size_t b0 = arena_bytes_t<3, true>(nc);
    const size_t bst = b0 + mstage_doubles<3>(nc) * sizeof(double);
    a.mstage = bst <= kLdsLimit ? 1 : 0;
    const size_t b = a.mstage ? bst : b0;
    return small_blocks(3, nc, b) ? launch_small(k_newton<3, true, true, true>, k_newton<3, true, true, true>, b, a, s)
                                  : launch_small(k_newton<3, true, true, false>, k_newton<3, true, false, false>, b, a, s);
}

int launch_aug_dump(int dim, int nc, const Phys& ph, const double* moments, const double* x, double* arena, double* A,
                    double* B, double* S, hipStream_t s) {
    Args a{};
    a.nc = nc; a.ph = ph; a.mom = moments; a.arena = arena; a.xin = x; a.Aout = A; a.Bout = B; a.Sout = S;
    a.esc = esc_of(arena, dim, nc);
    a.gc = make_grid(dim, nc);
    return dim == 2 ? launch_small(k_aug_dump<2, true>, k_aug_dump<2, false>, arena_bytes_t<2, true>(nc), a, s)
                    : launch_small(k_aug_dump<3, true>, k_aug_dump<3, false>, arena_bytes_t<3, true>(nc), a, s);
}

}  // namespace fmg
