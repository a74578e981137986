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
};

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Warp (wavefront = 64 lanes) reduction of doubles.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace fmg

#define FMG_HIP_CHECK(expr)                                                               \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return ::fmg::set_error(FMG_EHIP, "%s: %s", #expr,          \
                                                      hipGetErrorString(e_));             \
    } while (0)
