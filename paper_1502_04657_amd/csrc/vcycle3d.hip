// Fused V-cycle level passes for the 3D mesh family (Kuhn tetrahedra, K = h [6; -1 on +-e]).
//
// A pass applies NS red-black Gauss-Seidel half sweeps to a level array in one read and
// one write of the array, optionally preceded by the prolongation x = y + P x_c (POST) or
// followed by the residual r = f - K x and its restriction r_c = P^T r (PRE):
//   PLAIN: xout <- NS half sweeps of xin                         (read xin, f; write xout)
//   PRE  : xout <- NS half sweeps of xin, rc <- P^T (f - K xout)  (also write rc)
//   POST : xout <- NS half sweeps of (xin + P xc)                 (also read xc)
// The passes are out of place because a workgroup reads a halo that its neighbours write.
//
// Each workgroup owns a TX x TY tile of one z-chunk and marches along z.  With halo
// G = NS (+ 2 for PRE: the residual ring and the restriction ring) it keeps a window of
// planes of the (TX + 2G) x (TY + 2G) region in LDS and pipelines the half sweeps over the
// planes: at step t it loads plane t and applies half sweep s to plane t - s, so half sweep
// s reads half sweep s-1 on planes t-s-1 .. t-s+1.  Updates are in place in the window:
// half sweep s changes only nodes of its colour and reads only nodes of the other colour,
// which no other half sweep touches in the same step.  Every thread keeps the same region
// columns through all stages, so the z-neighbours it reads were written by itself; the
// xy-neighbours were written in an earlier step, so one barrier per step suffices.  Each
// plane of the window is stored as two colour halves (node (c, r) of colour k at half k,
// row r, slot c / 2), so the nodes a half sweep updates and the neighbours it reads are
// consecutive across the lanes (no LDS bank conflicts).
//
// Every node update, residual, restriction and prolongation uses the expression of the
// unfused kernels in grid.hip, so the passes give identical bits.
#include <hip/hip_ext.h>

#include <utility>

#include "dst.h"
#include "kernels.h"

#ifndef FMG_VPASS3D_PREFETCH
#define FMG_VPASS3D_PREFETCH 4
#endif

namespace fmg {

namespace {

enum { kPlain = 0, kPre = 1, kPost = 2 };

template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// Workgroup barrier for LDS only: waits for this wavefront's LDS operations, not for its
// global loads, so loads issued for later steps stay in flight across the barrier (the
// plain __syncthreads waits for every outstanding memory operation).  The march shares data
// between wavefronts through LDS alone.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Stores that a lane may have to skip go through a buffer resource: a lane that must not
// write gets an offset beyond the resource's size and the hardware drops its store.  Every
// store is then issued unconditionally, so the compiler can count the memory operations in
// flight (a store under a branch makes it wait for all of them).
constexpr unsigned kNoStore = 0xFFFFFFFFu;
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(T* base, int64_t elems) {
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)(elems * (int64_t)sizeof(T)), 0x00020000);
}
template <typename T>
__device__ __forceinline__ void masked_store(T v, __amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        __attribute__((ext_vector_type(2))) unsigned int w;
        w.x = (unsigned)b;
        w.y = (unsigned)(b >> 32);
        __builtin_amdgcn_raw_buffer_store_b64(w, r, byte_off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, byte_off, 0, 0);
    }
}

template <typename T>
__device__ inline T gs3f(const Stencil<T>& k, T f, T inv_h, T w, T e, T s, T n, T b, T t) {
    return gsu3(k, f, inv_h, w, e, s, n, b, t);
}

template <int NS, int MODE, int TX, int TY>
struct Geo3 {
    static constexpr int R = (MODE == kPre) ? 2 : 0;
    static constexpr int G = NS + R;                 // halo rings and z cone
    static constexpr int RX = TX + 2 * G, RY = TY + 2 * G;
    static constexpr int HP = RX / 2;                // pairs per region row
    static constexpr int NP = HP * RY;               // pairs per plane
    static constexpr int W = NS + 2 + (MODE == kPre ? 1 : 0);   // planes in the LDS x window
    static constexpr int D = FMG_VPASS3D_PREFETCH;   // planes loaded ahead of their step
    static constexpr int U = W + D;                  // period of the register windows
    static constexpr int HALF = RY * HP;             // nodes of one colour half
    static_assert(RX % 2 == 0, "region rows hold whole pairs");
};

// XCD-aware block order: consecutive block indices go to different XCDs, so block b runs
// tile xcd * per + b / 8 of the x-fastest (tile x, tile y, z chunk) order: each XCD walks a
// contiguous range of neighbouring tiles and their shared halos meet in its L2.
__device__ inline int tile_of_block(int b, int nblocks) {
    const int per = (nblocks + 7) >> 3;
    const int xcd = b & 7, r = b >> 3;
    const int full = nblocks - 8 * (per - 1);   // XCDs that get `per` blocks (the others per - 1)
    return xcd < full ? xcd * per + r : full * per + (xcd - full) * (per - 1) + r;
}

// Per-block context of a pass (everything the steps need besides the window and registers).
struct Ctx {
    int n, i0, j0, z0, z1, base, zero_x, tfirst;
    int64_t P, S;
};

template <typename T, int NS, int MODE, int C1, int TX, int TY, int NT>
struct Pass3 {
    using Ge = Geo3<NS, MODE, TX, TY>;
    static constexpr int G = Ge::G, RX = Ge::RX, RY = Ge::RY, HP = Ge::HP, NP = Ge::NP, W = Ge::W, HALF = Ge::HALF;
    static constexpr int D = Ge::D, U = Ge::U;
    static constexpr int KP = (NP + NT - 1) / NT;   // pairs per thread
    static constexpr int RRX = TX + 2, RRY = TY + 2;   // residual region: tile + 1 ring
    static constexpr int RSN = (MODE == kPre) ? RRX * RRY : 1, RSW = (MODE == kPre) ? 4 : 1;   // residual window

    __device__ static unsigned long long bits(T v) {
        if constexpr (sizeof(T) == 8) return (unsigned long long)__double_as_longlong(v);
        else return (unsigned long long)(unsigned)__float_as_uint(v);
    }
    template <typename U>
    __device__ static U from_bits(unsigned long long b) {
        if constexpr (sizeof(U) == 8) return __longlong_as_double((long long)b);
        else return __uint_as_float((unsigned)b);
    }

    // Raw global loads of plane t for the owned pair (k) into the register slots of plane t:
    // x (or y), f, and for POST the coarse values of the prolongation (zero where a node is
    // off the interior).  Nothing here uses a loaded value, so no load is waited for until
    // the plane's step (D steps later).
    static constexpr int NCV = (MODE == kPost) ? 4 : 1;   // coarse values per pair
    static_assert(NP == KP * NT, "one region pair per thread and round");
    __device__ static void load(const Ctx& cx, const T* __restrict__ xin, const T* __restrict__ f,
                                const T* __restrict__ xc, const Grid& gc, int t, T (&xr)[KP][2], T (&fr)[KP][2],
                                T (&cr)[KP][NCV]) {
        const int n = cx.n;
        // every load is issued unconditionally at an address clamped into the array (values
        // off the interior are replaced by zero where they are used), so the compiler can
        // count the loads in flight and wait for exactly the ones a step needs
        const int tc = min(max(t, 0), n);
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int q = threadIdx.x + k * NT;
            const int r = q / HP, m = q - r * HP;
            const int gi = min(max(cx.i0 - G + 2 * m, 0), n - 1), gj = min(max(cx.j0 - G + r, 0), n);
            const int64_t a0 = gi + cx.P * gj + cx.S * tc;
            xr[k][0] = xin[a0];
            xr[k][1] = xin[a0 + 1];
            fr[k][0] = f[a0];
            fr[k][1] = f[a0 + 1];
            if constexpr (MODE == kPost) {
                // the coarse values of k_prolong: x_c at (i/2, j/2, k/2) and at the other end of
                // the coarse edge (the same node for nodes on coarse nodes)
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int ii = min(max(cx.i0 - G + 2 * m + hh, 0), n), jj = gj;
                    const int di = ii & 1, dj = jj & 1, dk = tc & 1;
                    const int64_t q0 = (ii >> 1) + gc.pitch * (jj >> 1) + gc.plane * (tc >> 1);
                    const int64_t q1 = q0 + min(di + gc.pitch * dj + gc.plane * dk, (int64_t)(ii < n && jj < n && tc < n) *
                                                                                     (di + gc.pitch * dj + gc.plane * dk));
                    cr[k][2 * hh] = xc[q0];
                    cr[k][2 * hh + 1] = xc[q1];
                }
            }
        }
    }

    // value of a register pair at position sel (0 or 1) without indexing a register array at
    // run time (integer masks)
    __device__ static T pick(T a, T b, int sel) {
        const unsigned long long msk = 0ull - (unsigned long long)sel;
        return from_bits<T>((bits(a) & ~msk) | (bits(b) & msk));
    }

    // one step of the march; SL = t mod U (compile time): the register slots of plane t.
    // The LDS window slot of plane p is p mod W (run time).
    template <int SL>
    __device__ static void step(const Ctx& cx, int t, T (*xs)[2 * HALF], T (*rs)[RSN], T (&xw)[U][KP][2],
                                T (&fw)[U][KP][2], T (&cw)[U][KP][NCV], const T* __restrict__ xin, T* __restrict__ xout,
                                const T* __restrict__ f, T* __restrict__ rc, const T* __restrict__ xc,
                                const Grid& g, const Grid& gc) {
        const int n = cx.n, i0 = cx.i0, j0 = cx.j0, z0 = cx.z0, z1 = cx.z1, base = cx.base;
        const T inv_h = T(n), h = T(g.h);
        const Stencil<T> kst = stencil_of<T>(g);
        auto lslot = [](int p) { return ((p % W) + W) % W; };
        // ---- plane t (loaded D steps earlier) into the window
        if (t >= cx.tfirst && t <= z1 - 1 + G) {
            T* X = xs[lslot(t)];
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int q = threadIdx.x + k * NT;
                if (q >= NP) continue;
                const int r = q / HP, m = q - r * HP;
                const int k0 = (base + r + t) & 1;          // colour of column 2m
                const int gi = i0 - G + 2 * m, gj = j0 - G + r;
                const bool rowin = gj >= 1 && gj <= n - 1 && t >= 1 && t <= n - 1;
                const bool in0 = rowin && gi >= 1 && gi <= n - 1, in1 = rowin && gi + 1 >= 1 && gi + 1 <= n - 1;
                T v0 = (in0 && !cx.zero_x) ? xw[SL][k][0] : T(0), v1 = (in1 && !cx.zero_x) ? xw[SL][k][1] : T(0);
                if constexpr (MODE == kPost) {
                    // x = y + P x_c (the expression of k_prolong, accumulate)
                    const bool odd0 = ((gi & 1) | (gj & 1) | (t & 1)) != 0, odd1 = (((gi + 1) & 1) | (gj & 1) | (t & 1)) != 0;
                    T p0 = cw[SL][k][0], p1 = cw[SL][k][2];
                    if (odd0) p0 = T(0.5) * (p0 + cw[SL][k][1]);
                    if (odd1) p1 = T(0.5) * (p1 + cw[SL][k][3]);
                    if (in0) v0 += p0;
                    if (in1) v1 += p1;
                }
                X[k0 * HALF + r * HP + m] = v0;
                X[(k0 ^ 1) * HALF + r * HP + m] = v1;
            }
        }
        // ---- prefetch plane t + D
        load(cx, xin, f, xc, gc, t + D, xw[(SL + D) % U], fw[(SL + D) % U], cw[(SL + D) % U]);
        // ---- half sweeps: stage s on plane t - s, colour c1 ^ (s - 1)
        static_for<NS>([&](auto s_) {
            constexpr int s = decltype(s_)::value + 1;
            constexpr int fs = (SL - s + U) % U;   // f registers of plane t - s
            const int p = t - s;
            if (p < z0 - G + s || p > z1 - 1 + G - s || p < 1 || p > n - 1) return;
            constexpr int col = (C1 + s - 1) & 1, o = col ^ 1;
            const int ca = max(s, 1 - (i0 - G)), cb = min(RX - 1 - s, n - 1 - (i0 - G));
            const int ra = max(s, 1 - (j0 - G)), rb = min(RY - 1 - s, n - 1 - (j0 - G));
            const int sl = lslot(p), su = lslot(p + 1), sd = lslot(p - 1);
            const T* Xo = xs[sl] + o * HALF;
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int q = threadIdx.x + k * NT;
                if (q >= NP) continue;
                const int r = q / HP, m = q - r * HP;
                const int sel = ((base + r + p) & 1) ^ col;     // 0: column 2m has the colour, 1: 2m + 1
                const int c = 2 * m + sel;
                if (c < ca || c > cb || r < ra || r > rb) continue;
                const T wv = Xo[r * HP + m - 1 + sel], ev = Xo[r * HP + m + sel];
                const T sv = Xo[(r - 1) * HP + m], nv = Xo[(r + 1) * HP + m];
                const T bv = xs[sd][o * HALF + r * HP + m], tv = xs[su][o * HALF + r * HP + m];
                const T fv = pick(fw[fs][k][0], fw[fs][k][1], sel);
                xs[sl][col * HALF + r * HP + m] = gs3f<T>(kst, fv, inv_h, wv, ev, sv, nv, bv, tv);
            }
        });
        // ---- output: plane t - NS of the tile (lanes off the tile or steps off the chunk
        // store nothing)
        {
            const int p = t - NS;
            const bool pok = p >= z0 && p <= z1 - 1;
            const int pc = min(max(p, 0), n);
            const __amdgpu_buffer_rsrc_t rx = plane_rsrc(xout + cx.S * pc, cx.S);
            const int sl = lslot(pc);
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int q = threadIdx.x + k * NT;
                const int r = q / HP, m = q - r * HP;
                const int gi = i0 - G + 2 * m, gj = j0 - G + r;
                const bool rok = pok && gj >= j0 && gj <= min(n - 1, j0 + TY - 1);
                const int k0 = (base + r + pc) & 1;
                const unsigned o0 = (unsigned)(gi + cx.P * gj) * (unsigned)sizeof(T);
                const bool ok0 = rok && gi >= max(i0, 1) && gi <= min(n - 1, i0 + TX - 1);
                const bool ok1 = rok && gi + 1 >= max(i0, 1) && gi + 1 <= min(n - 1, i0 + TX - 1);
                masked_store(xs[sl][k0 * HALF + r * HP + m], rx, ok0 ? o0 : kNoStore);
                masked_store(xs[sl][(k0 ^ 1) * HALF + r * HP + m], rx, ok1 ? o0 + (unsigned)sizeof(T) : kNoStore);
            }
        }
        if constexpr (MODE == kPre) {
            // ---- residual on plane t - NS - 1, tile + 1 ring (zero off the interior)
            {
                constexpr int fs = (SL - NS - 1 + 2 * U) % U;
                const int p = t - NS - 1;
                if (p >= z0 - 1 && p <= z1 && p >= 1 && p <= n - 1) {
                    const int sl = lslot(p), su = lslot(p + 1), sd = lslot(p - 1);
                    T* R = rs[((p % 4) + 4) % 4];
                    auto X = [&](int slot, int c, int r, int pp) -> T {
                        return xs[slot][((base + c + r + pp) & 1) * HALF + r * HP + (c >> 1)];
                    };
#pragma unroll
                    for (int k = 0; k < KP; ++k) {
                        const int q = threadIdx.x + k * NT;
                        if (q >= NP) continue;
                        const int r = q / HP, m = q - r * HP;
                        const int k0 = (base + r + p) & 1;
                        static_for<2>([&](auto cc_) {
                            constexpr int cc = decltype(cc_)::value;      // colour of the node
                            const int c = 2 * m + (k0 ^ cc);
                            const int gi = i0 - G + c, gj = j0 - G + r;
                            if (c < G - 1 || c > RX - G || r < G - 1 || r > RY - G) return;
                            T v = T(0);
                            if (gi >= 1 && gi <= n - 1 && gj >= 1 && gj <= n - 1) {
                                const T fv = pick(fw[fs][k][0], fw[fs][k][1], k0 ^ cc);
                                v = kres3(kst, fv, h, X(sl, c, r, p), X(sl, c - 1, r, p), X(sl, c + 1, r, p),
                                          X(sl, c, r - 1, p), X(sl, c, r + 1, p), X(sd, c, r, p - 1),
                                          X(su, c, r, p + 1));
                            }
                            R[(r - (G - 1)) * RRX + (c - (G - 1))] = v;
                        });
                    }
                }
            }
            // ---- restriction for the coarse nodes whose centre plane is t - NS - 3 (every
            // step runs it; steps without such a plane store nothing)
            {
                const int pc0 = t - NS - 3;
                const int nc = gc.n;
                const bool ok = pc0 >= z0 && pc0 <= z1 - 1 && (pc0 & 1) == 0 && pc0 / 2 >= 1 && pc0 / 2 <= nc - 1;
                const int pc = ok ? pc0 : 2;
                const int K = pc / 2;
                const __amdgpu_buffer_rsrc_t rr = plane_rsrc(rc + gc.plane * K, gc.plane);
                const T* Rm = rs[(((pc - 1) % 4) + 4) % 4];
                const T* R0 = rs[(pc % 4 + 4) % 4];
                const T* Rp = rs[((pc + 1) % 4 + 4) % 4];
                constexpr int CW = TX / 2, CH = TY / 2;
                static_assert(CW * CH <= NT, "one coarse node per thread");
                const int q = threadIdx.x;
                const int cr = q / CW, cc = q - cr * CW;
                const int I = (i0 + 1) / 2 + cc, J = (j0 + 1) / 2 + cr;   // 2I: the even columns of the tile
                const bool mine = ok && q < CW * CH && I >= 1 && I <= nc - 1 && J <= nc - 1;
                const int c = min(2 * I - i0 + 1, RRX - 2), r = min(2 * J - j0 + 1, RRY - 2);   // residual-region coords
                const int o = r * RRX + c;
                // the order of k_resid_restrict: d = 1, P, S, 1+P, P+S, 1+S, 1+P+S
                T e = T(0);
                e += R0[o - 1] + R0[o + 1];
                e += R0[o - RRX] + R0[o + RRX];
                e += Rm[o] + Rp[o];
                e += R0[o - 1 - RRX] + R0[o + 1 + RRX];
                e += Rm[o - RRX] + Rp[o + RRX];
                e += Rm[o - 1] + Rp[o + 1];
                e += Rm[o - 1 - RRX] + Rp[o + 1 + RRX];
                masked_store(R0[o] + T(0.5) * e, rr,
                             mine ? (unsigned)(I + gc.pitch * J) * (unsigned)sizeof(T) : kNoStore);
            }
        }
        lds_barrier();
    }
};

template <typename T, int NS, int MODE, int C1, int TX, int TY, int NT, int... SL>
__device__ __forceinline__ void steps_block(const Ctx& cx, int t, int tlast, T (*xs)[2 * Pass3<T, NS, MODE, C1, TX, TY, NT>::HALF],
                                            T (*rs)[Pass3<T, NS, MODE, C1, TX, TY, NT>::RSN],
                                            T (&xw)[Pass3<T, NS, MODE, C1, TX, TY, NT>::U][Pass3<T, NS, MODE, C1, TX, TY, NT>::KP][2],
                                            T (&fw)[Pass3<T, NS, MODE, C1, TX, TY, NT>::U][Pass3<T, NS, MODE, C1, TX, TY, NT>::KP][2],
                                            T (&cw)[Pass3<T, NS, MODE, C1, TX, TY, NT>::U][Pass3<T, NS, MODE, C1, TX, TY, NT>::KP][Pass3<T, NS, MODE, C1, TX, TY, NT>::NCV],
                                            const T* xin, T* xout, const T* f, T* rc, const T* xc, const Grid& g,
                                            const Grid& gc, std::integer_sequence<int, SL...>) {
    using PS = Pass3<T, NS, MODE, C1, TX, TY, NT>;
    // every step of the block runs: steps before the first plane or after the last one
    // only load clamped addresses and store nothing (their LDS work is out of its plane
    // range), and without a branch around the steps the compiler counts the loads in flight
    (PS::template step<SL>(cx, t + SL, xs, rs, xw, fw, cw, xin, xout, f, rc, xc, g, gc), ...);
}

template <typename T, int NS, int MODE, int C1, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_vpass3d(const T* __restrict__ xin, T* __restrict__ xout,
                                                const T* __restrict__ f, T* __restrict__ rc,
                                                const T* __restrict__ xc, Grid g, Grid gc, int zero_x, int zc,
                                                int tiles_x, int tiles_y) {
    using PS = Pass3<T, NS, MODE, C1, TX, TY, NT>;
    constexpr int G = PS::G, W = PS::W, KP = PS::KP;
    __shared__ T xs[W][2 * PS::HALF];
    __shared__ T rs[PS::RSW][PS::RSN];
    Ctx cx;
    cx.n = g.n;
    cx.P = g.pitch;
    cx.S = g.plane;
    const int tile = tile_of_block(blockIdx.x, gridDim.x);
    const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, tz = tile / (tiles_x * tiles_y);
    // x origin of the tile: the region (tile + G columns each side) starts at an even column,
    // so the pair loads are 16-byte aligned (rows are padded to 16 elements); for even G the
    // first tile starts at the boundary column 0, which is never written
    cx.i0 = (G & 1) ? 1 + tx * TX : tx * TX;
    cx.j0 = 1 + ty * TY;
    cx.z0 = 1 + tz * zc;
    cx.z1 = min(g.n, cx.z0 + zc);              // output planes [z0, z1)
    cx.base = (cx.i0 + cx.j0 - 2 * G) & 1;     // colour parity of region node (0, 0) at plane 0
    cx.zero_x = zero_x;
    cx.tfirst = cx.z0 - G;
    const int tlast = cx.z1 - 1 + NS + (MODE == kPre ? 3 : 0);
    constexpr int U = PS::U;
    T xw[U][KP][2];
    T fw[U][KP][2];
    T cw[U][KP][PS::NCV];
    // The register slots of plane t are t mod U: the march goes in unrolled blocks of U
    // steps from a multiple of U, so every step knows its register slots at compile time.
    // Steps tfirst - D .. tfirst - 1 only prefetch the first planes.
    const int t_pre = cx.tfirst - PS::D;
    for (int t = t_pre - ((t_pre % U) + U) % U; t <= tlast; t += U)
        steps_block<T, NS, MODE, C1, TX, TY, NT>(cx, t, tlast, xs, rs, xw, fw, cw, xin, xout, f, rc, xc, g, gc,
                                                 std::make_integer_sequence<int, U>{});
}


// ---- small levels: the whole V-cycle below a level in one workgroup ----------------------
// A level with at most kBottom3MaxN cells per side and every level below it run in one
// workgroup, with each level's x and f as a dense (n_q + 1)^3 array (zero ring) in LDS:
// the pre half sweeps, the residual and its restriction, the exact coarsest solve, the
// prolongation and the post half sweeps of the unfused kernel sequence (grid.hip), node by
// node with the same expressions, so the result has the same bits, in one launch instead of
// about a dozen per level.  The coarsest-solve scratch follows the level arrays.
// 16 wavefronts (100 VGPRs each fit four per SIMD): the n = 16 half sweeps take two items per
// thread instead of four
constexpr int kBottom3Threads = 1024;
constexpr int kBottom3MaxN = 16;
constexpr size_t kBottom3MaxBytes = 150 * 1024;

__host__ __device__ inline int b3_elems(int n0, int q) {
    const int p = (n0 << q) + 1;
    return p * p * p;
}
// elements of the level arrays below level q (each level: x, then f)
__host__ __device__ inline int b3_off(int n0, int q) {
    int e = 0;
    for (int r = 0; r < q; ++r) e += 2 * b3_elems(n0, r);
    return e;
}
template <typename T>
size_t b3_bytes(int n0, int l) {
    const size_t m = (size_t)n0 - 1;
    return ((size_t)b3_off(n0, l + 1) * sizeof(T) + 7) / 8 * 8 + sizeof(double) * (m * m + m + 2 * m * m * m);
}

// nh alternating half sweeps, colour 0 first
template <typename T>
__device__ void b3_sweeps(const Stencil<T>& kst, T* X, const T* F, int n, int nh) {
    const int P = n + 1, S = P * P, half = n / 2, m = n - 1;
    const T inv_h = T(n);
    for (int hs = 0; hs < nh; ++hs) {
        const int c = hs & 1;
        for (int t = threadIdx.x; t < m * m * half; t += blockDim.x) {
            const int row = t / half, slot = t - row * half;
            const int j = 1 + row % m, k = 1 + row / m;
            const int i = (((1 + j + k) & 1) == c ? 1 : 2) + 2 * slot;
            if (i > m) continue;
            const int p = i + P * j + S * k;
            X[p] = gs3f<T>(kst, F[p], inv_h, X[p - 1], X[p + 1], X[p - P], X[p + P], X[p - S], X[p + S]);
        }
        __syncthreads();
    }
}

template <typename T>
__device__ inline T b3_resid(const Stencil<T>& kst, const T* X, const T* F, int q, int P, int S, T h) {
    return kres3(kst, F[q], h, X[q], X[q - 1], X[q + 1], X[q - P], X[q + P], X[q - S], X[q + S]);
}

template <typename T>
__global__ __launch_bounds__(kBottom3Threads) void k_vbottom3d(T* __restrict__ x, const T* __restrict__ f, Grid g,
                                                               int n0, int l, int nh_pre, int nh_post, int zero_x) {
    extern __shared__ double smem[];
    const Stencil<T> kst = stencil_of<T>(g);   // the coefficient is the same on every level
    T* const base = reinterpret_cast<T*>(smem);
    auto X = [&](int q) { return base + b3_off(n0, q); };
    auto F = [&](int q) { return base + b3_off(n0, q) + b3_elems(n0, q); };
    double* dsm = smem + ((size_t)b3_off(n0, l + 1) * sizeof(T) + 7) / 8;
    // lower levels start at zero (their rings stay zero); level l from global memory
    for (int t = threadIdx.x; t < b3_off(n0, l); t += blockDim.x) base[t] = T(0);
    const int n = n0 << l, P = n + 1, S = P * P;
    for (int t = threadIdx.x; t < P * S; t += blockDim.x) {
        const int i = t % P, j = (t / P) % P, k = t / S;
        const bool in = i >= 1 && i < n && j >= 1 && j < n && k >= 1 && k < n;
        const int64_t gp = i + g.pitch * j + g.plane * k;
        X(l)[t] = (in && !zero_x) ? x[gp] : T(0);
        F(l)[t] = in ? f[gp] : T(0);
    }
    __syncthreads();
    // down: pre sweeps, then f_{q-1} = P^T (f_q - K x_q)
    for (int q = l; q >= 1; --q) {
        const int nq = n0 << q, Pq = nq + 1, Sq = Pq * Pq, nc = nq / 2, Pc = nc + 1, mc = nc - 1;
        const T hq = T(1.0 / nq);
        b3_sweeps<T>(kst, X(q), F(q), nq, nh_pre);
        const T* Xq = X(q);
        const T* Fq = F(q);
        T* Fc = F(q - 1);
        const int d[7] = {1, Pq, Sq, 1 + Pq, Pq + Sq, 1 + Sq, 1 + Pq + Sq};
        for (int t = threadIdx.x; t < mc * mc * mc; t += blockDim.x) {
            const int I = 1 + t % mc, J = 1 + (t / mc) % mc, K = 1 + t / (mc * mc);
            const int p = 2 * I + Pq * 2 * J + Sq * 2 * K;
            const T c = b3_resid<T>(kst, Xq, Fq, p, Pq, Sq, hq);
            T e = T(0);
#pragma unroll
            for (int r = 0; r < 7; ++r)
                e += b3_resid<T>(kst, Xq, Fq, p - d[r], Pq, Sq, hq) + b3_resid<T>(kst, Xq, Fq, p + d[r], Pq, Sq, hq);
            Fc[I + Pc * J + Pc * Pc * K] = c + T(0.5) * e;
        }
        __syncthreads();
    }
    coarse_dst_solve<T>(F(0), X(0), n0 + 1, (int64_t)(n0 + 1) * (n0 + 1), n0, 3, g.a, dsm);
    __syncthreads();
    // up: x_q += P x_{q-1}, then the post sweeps
    for (int q = 1; q <= l; ++q) {
        const int nq = n0 << q, Pq = nq + 1, Sq = Pq * Pq, Pc = nq / 2 + 1, Sc = Pc * Pc, m = nq - 1;
        const T* xc = X(q - 1);
        T* Xq = X(q);
        for (int t = threadIdx.x; t < m * m * m; t += blockDim.x) {
            const int i = 1 + t % m, j = 1 + (t / m) % m, k = 1 + t / (m * m);
            const int di = i & 1, dj = j & 1, dk = k & 1;
            const int q0 = (i >> 1) + Pc * (j >> 1) + Sc * (k >> 1);
            T v = xc[q0];
            if (di | dj | dk) v = T(0.5) * (v + xc[q0 + di + Pc * dj + Sc * dk]);
            Xq[i + Pq * j + Sq * k] += v;
        }
        __syncthreads();
        b3_sweeps<T>(kst, Xq, F(q), nq, nh_post);
    }
    const int m = n - 1;
    for (int t = threadIdx.x; t < m * m * m; t += blockDim.x) {
        const int i = 1 + t % m, j = 1 + (t / m) % m, k = 1 + t / (m * m);
        x[i + g.pitch * j + g.plane * k] = X(l)[i + P * j + S * k];
    }
}


// ---- small levels: red-black half sweeps in LDS tiles ---------------------------------------
// Levels between the one-workgroup bottom and the z-pipelined passes have too few planes for
// the march along z to pay.  There a workgroup owns a cube of kTile^3 interior nodes and
// loads it with NS rings of halo (x and f) into LDS; half sweep s updates the nodes of its
// colour that lie at least s + 1 rings inside the region, so after NS half sweeps the cube
// holds the values of the unfused sequence (the halo is recomputed by every workgroup that
// needs it) and is written out of place.  NS half sweeps in one launch instead of NS, with
// the node expression of the unfused kernel (same bits).
constexpr int kTile = 8;
constexpr int kTileThreads = 256;

template <typename T, int NS>
__global__ __launch_bounds__(kTileThreads) void k_vtile3d(const T* __restrict__ xin, T* __restrict__ xout,
                                                          const T* __restrict__ f, Grid g, int first, int zero_x) {
    constexpr int R = kTile + 2 * NS, RR = R * R, RV = RR * R;
    constexpr int NL = (RV + kTileThreads - 1) / kTileThreads;
    __shared__ T xs[RV];
    __shared__ T fs[RV];
    const int n = g.n;
    const int i0 = 1 + (int)blockIdx.x * kTile - NS, j0 = 1 + (int)blockIdx.y * kTile - NS,
              k0 = 1 + (int)blockIdx.z * kTile - NS;   // node of region cell (0, 0, 0)
    const int64_t P = g.pitch, S = g.plane;
    // every load of the region in flight before the stores to LDS (nodes off the mesh: 0)
    T vx[NL], vf[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int t = (int)threadIdx.x + u * kTileThreads;
        const int a = t % R, b = (t / R) % R, c = t / RR;
        const int i = i0 + a, j = j0 + b, k = k0 + c;
        const bool in = t < RV && i >= 0 && i <= n && j >= 0 && j <= n && k >= 0 && k <= n;
        const int64_t p = in ? i + P * j + S * k : 0;
        const T x0 = xin[zero_x ? 0 : p], f0 = f[p];
        vx[u] = (in && !zero_x) ? x0 : T(0);
        vf[u] = in ? f0 : T(0);
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int t = (int)threadIdx.x + u * kTileThreads;
        if (t < RV) {
            xs[t] = vx[u];
            fs[t] = vf[u];
        }
    }
    __syncthreads();
    const Stencil<T> kst = stencil_of<T>(g);
    const T inv_h = T(n);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        // nodes of colour c ((i + j + k) & 1 == c) with region coordinates in [s + 1, R - 2 - s]
        const int c = (first + s) & 1;
        const int lo = s + 1, w = R - 2 * (s + 1), hw = (w + 1) / 2;
        for (int t = threadIdx.x; t < hw * w * w; t += kTileThreads) {
            const int m = t % hw, b = lo + (t / hw) % w, cz = lo + t / (hw * w);
            const int j = j0 + b, k = k0 + cz;
            // first region column of the colour in this row
            const int a = lo + ((i0 + lo + j + k + c) & 1) + 2 * m;
            const int i = i0 + a;
            if (a > R - 2 - s || i < 1 || i > n - 1 || j < 1 || j > n - 1 || k < 1 || k > n - 1) continue;
            const int q = a + R * b + RR * cz;
            xs[q] = gs3f<T>(kst, fs[q], inv_h, xs[q - 1], xs[q + 1], xs[q - R], xs[q + R], xs[q - RR], xs[q + RR]);
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < kTile * kTile * kTile; t += kTileThreads) {
        const int a = NS + t % kTile, b = NS + (t / kTile) % kTile, cz = NS + t / (kTile * kTile);
        const int i = i0 + a, j = j0 + b, k = k0 + cz;
        if (i > n - 1 || j > n - 1 || k > n - 1) continue;
        xout[i + P * j + S * k] = xs[a + R * b + RR * cz];
    }
}

}  // namespace

// ---- launch --------------------------------------------------------------------------------
// Tile shapes: one region pair per thread ((TX + 2G) / 2 * (TY + 2G) = NT) in variant 0:
// 256 threads, 32 x 16 region; variant 1: 512 threads, 32 x 32; variant 2: 512 threads,
// 64 x 16 (longer contiguous rows per plane); and two pairs per thread in variant 3: 512
// threads, 64 x 32 (less halo per tile; the register windows double).
template <int G, int V>
struct Shape3 {
    static constexpr int NT = V ? 512 : 256;
    // RX / 2 pairs per region row; variant 3 holds two pairs per thread
    static constexpr int RX = (V == 2 || V == 3) ? 64 : 32, RY = V == 3 ? 32 : 2 * NT / RX;
    static constexpr int TX = RX - 2 * G, TY = RY - 2 * G;
    static_assert(TX > 0 && TY > 0 && TX % 2 == 0, "tile shape");
};

static int g_var3 = 1;        // tile variant of the fused 3D passes
static int g_min_n3 = 128;    // smallest level that takes the fused passes
static int g_one3 = 0;        // nu = 2: one pass of 5 half sweeps per side (1) or 3 + 2 (0)
static int g_cus = 0;         // compute units of the device (queried once)

// z planes per chunk: all blocks of a pass resident at once (no tail wave of blocks), and
// at least 8 planes per chunk
template <typename K>
static int z_chunk(K kern, int nt, int n, int tiles_xy) {
    static thread_local int cached_dev = -1;
    if (g_cus == 0 || cached_dev < 0) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) == hipSuccess) g_cus = pr.multiProcessorCount;
        if (g_cus <= 0) g_cus = 256;
        cached_dev = dev;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), nt, 0) !=
            hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    // enough chunks for every CU, no more than fit at once
    const int cap = per_cu * g_cus;
    const int chunks = std::max(cdiv(g_cus, std::max(1, tiles_xy)), (unsigned)std::max(1, cap / std::max(1, tiles_xy)));
    return std::min(n - 1, std::max(8, (int)cdiv(n - 1, chunks)));
}

template <typename T, int NS, int MODE, int C1, int V>
static void pass3d_v(const Grid& g, const Grid& gc, const T* xin, T* xout, const T* f, T* rc, const T* xc,
                     int zero_x, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    constexpr int G = Geo3<NS, MODE, 2, 2>::G;
    using Sh = Shape3<G, V>;
    auto kern = k_vpass3d<T, NS, MODE, C1, Sh::TX, Sh::TY, Sh::NT>;
    // columns 1 .. n-1 (odd G: tiles from column 1; even G: from column 0)
    const int tiles_x = (int)cdiv(g.n - 1 + ((G & 1) ? 0 : 1), Sh::TX), tiles_y = (int)cdiv(g.n - 1, Sh::TY);
    static thread_local int zc_n = -1, zc_v = 0;   // chunk of the last level size
    if (zc_n != g.n) {
        zc_v = z_chunk(kern, Sh::NT, g.n, tiles_x * tiles_y);
        zc_n = g.n;
    }
    const int zc = zc_v;
    const int tiles_z = (int)cdiv(g.n - 1, zc);
    const int nb = tiles_x * tiles_y * tiles_z;
    hipExtLaunchKernelGGL(kern, dim3(nb), dim3(Sh::NT), 0, s, ev0, ev1, 0, xin, xout, f, rc, xc, g, gc, zero_x, zc,
                          tiles_x, tiles_y);
}

template <typename T, int NS, int MODE, int C1>
static void pass3d(const Grid& g, const Grid& gc, const T* xin, T* xout, const T* f, T* rc, const T* xc,
                   int zero_x, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (g_var3 == 3)
        pass3d_v<T, NS, MODE, C1, 3>(g, gc, xin, xout, f, rc, xc, zero_x, s, ev0, ev1);
    else if (g_var3 == 2)
        pass3d_v<T, NS, MODE, C1, 2>(g, gc, xin, xout, f, rc, xc, zero_x, s, ev0, ev1);
    else if (g_var3 == 1)
        pass3d_v<T, NS, MODE, C1, 1>(g, gc, xin, xout, f, rc, xc, zero_x, s, ev0, ev1);
    else
        pass3d_v<T, NS, MODE, C1, 0>(g, gc, xin, xout, f, rc, xc, zero_x, s, ev0, ev1);
}

void set_vpass3d_tuning(int variant, int min_n, int one_pass) {
    if (variant >= 0) g_var3 = variant > 3 ? 3 : variant;
    if (min_n > 0) g_min_n3 = min_n;
    if (one_pass >= 0) g_one3 = one_pass ? 1 : 0;
}
void get_vpass3d_tuning(int* variant, int* min_n, int* one_pass) {
    *variant = g_var3;
    *min_n = g_min_n3;
    *one_pass = g_one3;
}

bool vpass3d_applies(const Grid& g, int nu_pre, int nu_post) {
    return g.dim == 3 && g.n >= g_min_n3 && nu_pre == nu_post && (nu_pre == 1 || nu_pre == 2);
}

// pre smoothing (2 nu + 1 half sweeps) + residual + restriction: x -> y (result in x for the
// two-pass split, in y for the one-pass one); returns the array that holds the smoothed x
template <typename T>
T* launch_vpre3d(const Grid& g, const Grid& gc, T* x, T* y, const T* f, T* rc, int nu, int zero_x, hipStream_t s,
                 hipEvent_t ev0, hipEvent_t ev1) {
    if (nu == 2 && g_one3) {
        // five half sweeps in one pass (5-ring halo), then the residual and its restriction
        pass3d<T, 5, kPlain, 0>(g, gc, x, y, f, nullptr, nullptr, zero_x, s, ev0, ev1);
        launch_resid_restrict<T>(g, gc, y, f, rc, s);
        return y;
    }
    if (nu == 2) {
        // five half sweeps in two passes; the residual and its restriction then as their own
        // streaming kernel (a pass that also restricts needs a 4-ring halo, which costs more
        // than reading x and f once more)
        pass3d<T, 3, kPlain, 0>(g, gc, x, y, f, nullptr, nullptr, zero_x, s, ev0, ev1);
        pass3d<T, 2, kPlain, 1>(g, gc, y, x, f, nullptr, nullptr, 0, s, nullptr, nullptr);
        launch_resid_restrict<T>(g, gc, x, f, rc, s);
        return x;
    }
    pass3d<T, 3, kPre, 0>(g, gc, x, y, f, rc, nullptr, zero_x, s, ev0, ev1);
    return y;
}

// x_out = post smoothing of (xs + P xc); xs is the array launch_vpre3d returned, x_out the
// V-cycle's x (the other array is scratch)
template <typename T>
void launch_vpost3d(const Grid& g, const Grid& gc, T* xs, T* scratch, T* x_out, const T* f, const T* xc, int nu,
                    hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (nu == 2 && g_one3) {
        // xs is the scratch array here (the one-pass pre ends in y): y -> x
        pass3d<T, 5, kPost, 0>(g, gc, xs, x_out, f, nullptr, xc, 0, s, ev0, ev1);
        return;
    }
    if (nu == 2) {
        // xs == x_out here (the pre split ends in x): x -> scratch -> x
        pass3d<T, 3, kPost, 0>(g, gc, xs, scratch, f, nullptr, xc, 0, s, ev0, ev1);
        pass3d<T, 2, kPlain, 1>(g, gc, scratch, x_out, f, nullptr, nullptr, 0, s, nullptr, nullptr);
        return;
    }
    // xs is the scratch array here: y -> x
    pass3d<T, 3, kPost, 0>(g, gc, xs, x_out, f, nullptr, xc, 0, s, ev0, ev1);
}

template double* launch_vpre3d<double>(const Grid&, const Grid&, double*, double*, const double*, double*, int, int,
                                       hipStream_t, hipEvent_t, hipEvent_t);
template float* launch_vpre3d<float>(const Grid&, const Grid&, float*, float*, const float*, float*, int, int,
                                     hipStream_t, hipEvent_t, hipEvent_t);
template void launch_vpost3d<double>(const Grid&, const Grid&, double*, double*, double*, const double*,
                                     const double*, int, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_vpost3d<float>(const Grid&, const Grid&, float*, float*, float*, const float*, const float*, int,
                                    hipStream_t, hipEvent_t, hipEvent_t);

template <typename T>
bool launch_vbottom3d(const Grid* levels, int l, T* x, const T* f, int nu_pre, int nu_post, int zero_x,
                      hipStream_t s) {
    if (l < 1 || levels[l].dim != 3 || levels[l].n > kBottom3MaxN || nu_pre > 2 || nu_post > 2) return false;
    const int n0 = levels[0].n;
    const size_t bytes = b3_bytes<T>(n0, l);
    if (bytes > kBottom3MaxBytes) return false;
    // once per instantiation (thread-safe static initialisation)
    static const bool attr = [] {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vbottom3d<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBottom3MaxBytes) == hipSuccess)
            return true;
        (void)hipGetLastError();
        return false;
    }();
    if (!attr) return false;
    const int nh_pre = nu_pre > 0 ? 2 * nu_pre + 1 : 0, nh_post = nu_post > 0 ? 2 * nu_post + 1 : 0;
    hipLaunchKernelGGL(k_vbottom3d<T>, dim3(1), dim3(kBottom3Threads), bytes, s, x, f, levels[l], n0, l, nh_pre,
                       nh_post, zero_x);
    return true;
}
template bool launch_vbottom3d<double>(const Grid*, int, double*, const double*, int, int, int, hipStream_t);
template bool launch_vbottom3d<float>(const Grid*, int, float*, const float*, int, int, int, hipStream_t);

static int g_tile3 = 1;   // levels below the z-pipelined passes: LDS tiles (1) or one launch per half sweep (0)

void set_vtile3d_tuning(int enable) { g_tile3 = enable ? 1 : 0; }
int get_vtile3d_tuning() { return g_tile3; }

bool vtile3d_applies(const Grid& g, int nu_pre, int nu_post) {
    return g_tile3 && g.dim == 3 && g.n > kBottom3MaxN && g.n < g_min_n3 && nu_pre == nu_post &&
           (nu_pre == 1 || nu_pre == 2);
}

template <typename T>
void launch_vtile3d(const Grid& g, const T* xin, T* xout, const T* f, int half_sweeps, int first, int zero_x,
                    hipStream_t s) {
    const int nt = (int)cdiv(g.n - 1, kTile);
    const dim3 grd(nt, nt, nt);
    if (half_sweeps == 3)
        hipLaunchKernelGGL((k_vtile3d<T, 3>), grd, dim3(kTileThreads), 0, s, xin, xout, f, g, first, zero_x);
    else
        hipLaunchKernelGGL((k_vtile3d<T, 2>), grd, dim3(kTileThreads), 0, s, xin, xout, f, g, first, zero_x);
}
template void launch_vtile3d<double>(const Grid&, const double*, double*, const double*, int, int, int, hipStream_t);
template void launch_vtile3d<float>(const Grid&, const float*, float*, const float*, int, int, int, hipStream_t);

}  // namespace fmg
