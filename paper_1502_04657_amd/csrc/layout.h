// Per-coarse-element moment layout shared by the moment kernels and the small solves.
//
// For a coarse simplex E with barycentric coordinates lambda_0..lambda_D and the fine
// function u~ (P1 on the fine mesh), the moment kernels deliver
//   T3[pqr] = int_E u~ l_p l_q l_r     (p<=q<=r)      T2[pq] = int_E u~^2 l_p l_q  (p<=q)
//   T1[p]   = int_E u~^3 l_p                           T0     = int_E u~^4
//   B1[p]   = int_E u~ l_p                             B2     = int_E u~^2
//   AW1[p]  = int_E W u~ l_p                           AW2    = int_E W u~^2
//   KG[p]   = int_E A grad u~ . grad l_p               Q      = int_E A grad u~ . grad u~
// which is everything the augmented matrices of (3.6) need beyond the coarse matrices.
#pragma once

namespace fmg {

template <int D>
struct MomLayout {
    static constexpr int V = D + 1;
    static constexpr int NT3 = (D == 2) ? 10 : 20;
    static constexpr int NT2 = (D == 2) ? 6 : 10;
    static constexpr int T3 = 0;
    static constexpr int T2 = T3 + NT3;
    static constexpr int T1 = T2 + NT2;
    static constexpr int T0 = T1 + V;
    static constexpr int B1 = T0 + 1;
    static constexpr int B2 = B1 + V;
    static constexpr int AW1 = B2 + 1;
    static constexpr int AW2 = AW1 + V;
    static constexpr int KG = AW2 + 1;
    static constexpr int Q = KG + V;
    static constexpr int SIZE = Q + 1;  // 32 (2D) / 50 (3D)
    static constexpr int NE = (D == 2) ? 2 : 6;  // simplices per cell
};

// index of a multiset {p,q[,r]} (entries in [0,V)) among the sorted tuples in
// lexicographic order: closed form, so no lookup table is indexed at run time
__host__ __device__ constexpr int sym2(int p, int q, int V) {
    const int a = p < q ? p : q, b = p < q ? q : p;
    return a * V - a * (a - 1) / 2 + (b - a);
}
__host__ __device__ constexpr int sym3(int p, int q, int r, int V) {
    int a = p, b = q, c = r, t = 0;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    int idx = 0;
    for (int k = 0; k < a; ++k) idx += (V - k) * (V - k + 1) / 2;   // tuples starting below a
    return idx + sym2(b - a, c - a, V - a);
}
static_assert(sym2(1, 1, 3) == 3 && sym2(2, 0, 3) == 2 && sym2(2, 2, 3) == 5, "sym2");
static_assert(sym3(0, 1, 1, 3) == 3 && sym3(1, 1, 1, 3) == 6 && sym3(2, 1, 2, 3) == 8 && sym3(2, 2, 2, 3) == 9,
              "sym3");
static_assert(sym3(3, 3, 3, 4) == 19 && sym3(1, 1, 1, 4) == 10 && sym2(3, 3, 4) == 9, "sym3 (4)");

// monomials X^a (|a| <= 3) of the coarse-local coordinates, ordered by degree
static constexpr int kMon2[10][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {1, 1}, {0, 2}, {3, 0}, {2, 1}, {1, 2}, {0, 3}};
static constexpr int kMon3[20][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {1, 1, 0}, {1, 0, 1},
                                     {0, 2, 0}, {0, 1, 1}, {0, 0, 2}, {3, 0, 0}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0},
                                     {1, 1, 1}, {1, 0, 2}, {0, 3, 0}, {0, 2, 1}, {0, 1, 2}, {0, 0, 3}};

// path order (axis permutation) of the cell simplices of tables.h; the simplex of
// permutation s holds the points with X_s0 >= X_s1 (>= X_s2)
static constexpr int kPerm2[2][2] = {{0, 1}, {1, 0}};
static constexpr int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// raw moment accumulators: int u~ X^a (|a|<=3), int u~^2 X^a (|a|<=2), int u~^3 X^a
// (|a|<=1), int u~^4, int grad u~ (D), int |grad u~|^2
template <int D>
struct RawLayout {
    static constexpr int M3 = (D == 2) ? 10 : 20;
    static constexpr int M2 = (D == 2) ? 6 : 10;
    static constexpr int M1 = D + 1;
    static constexpr int P1 = 0;
    static constexpr int P2 = M3;
    static constexpr int P3 = P2 + M2;
    static constexpr int P4 = P3 + M1;
    static constexpr int G = P4 + 1;
    static constexpr int Q = G + D;
    static constexpr int SIZE = Q + 1;  // 23 (2D) / 39 (3D)
};

}  // namespace fmg
