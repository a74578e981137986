// Per-coarse-element moment layout shared by the moment kernels and the small solves.
//
// For a coarse simplex E with barycentric coordinates lambda_0..lambda_D and the fine
// function u~ (P1 on the fine mesh), the moment kernels deliver
//   T3[pqr] = int_E u~ l_p l_q l_r     (p<=q<=r)      T2[pq] = int_E u~^2 l_p l_q  (p<=q)
//   T1[p]   = int_E u~^3 l_p                           T0     = int_E u~^4
//   B1[p]   = int_E u~ l_p                             B2     = int_E u~^2
//   AW1[p]  = int_E W u~ l_p                           AW2    = int_E W u~^2
//   KG[p]   = int_E grad u~ . grad l_p                 Q      = int_E |grad u~|^2
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

// index of a multiset {p,q[,r]} among the sorted tuples in lexicographic order
template <int V>
struct SymIdx {
    int i2[V][V];
    int i3[V][V][V];
    constexpr SymIdx() : i2{}, i3{} {
        int c = 0;
        for (int p = 0; p < V; ++p)
            for (int q = p; q < V; ++q) {
                i2[p][q] = c;
                i2[q][p] = c;
                ++c;
            }
        c = 0;
        for (int p = 0; p < V; ++p)
            for (int q = p; q < V; ++q)
                for (int r = q; r < V; ++r) {
                    i3[p][q][r] = c; i3[p][r][q] = c; i3[q][p][r] = c;
                    i3[q][r][p] = c; i3[r][p][q] = c; i3[r][q][p] = c;
                    ++c;
                }
    }
};
static constexpr SymIdx<3> kSym2{};
static constexpr SymIdx<4> kSym3{};

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
