// Host-side launchers of the HIP kernels (one translation unit per kernel family).
#pragma once

#include "common.h"

namespace fmg {

// ---- grid.hip ---------------------------------------------------------------------------
template <typename T> void launch_fill(T* p, int64_t count, T v, hipStream_t s);
void launch_pack(const Grid& g, const double* compact, double* level, hipStream_t s);
void launch_unpack(const Grid& g, const double* level, double* compact, hipStream_t s);
// one red-black half sweep of Gauss-Seidel on K x = f for the nodes of `color`
template <typename T> void launch_smooth_half(const Grid& g, T* x, const T* f, int color, hipStream_t s);
// `half_sweeps` alternating half sweeps starting with colour `first` (temporal blocking
// inside one kernel where the level is small enough; identical arithmetic)
template <typename T> void launch_smooth(const Grid& g, T* x, const T* f, int half_sweeps, int first,
                                         hipStream_t s);
template <typename T> void launch_resid_restrict(const Grid& gf, const Grid& gc, const T* x, const T* f,
                                                 T* rc, hipStream_t s);
template <typename T> void launch_prolong(const Grid& gc, const Grid& gf, const T* xc, T* xf, int accumulate,
                                          hipStream_t s);
template <typename T> void launch_coarse_solve(const Grid& g, const T* f, T* x, hipStream_t s);
// `steps` conjugate-gradient iterations on K x = f from x; r, p, q: level arrays of g with
// zero rings; partial: kReduceBlocks doubles; sc: 4 doubles
template <typename T> void launch_cg_smooth(const Grid& g, T* x, const T* f, int steps, T* r, T* p, T* q,
                                            double* partial, double* sc, hipStream_t s);
// b = lambda M u - M_W u - zeta N(u); lambda = *lam_dev if lam_dev else lam_host
void launch_rhs(const Grid& g, const Phys& ph, const double* u, double* b, const double* lam_dev,
                double lam_host, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// mixed precision: r32 = (float)(b - K u); u += (double)e32
void launch_residual_demote(const Grid& g, const double* u, const double* b, float* r, hipStream_t s);
void launch_add_promote(const Grid& g, double* u, const float* e, hipStream_t s);
// u <- c * ut + Pi x_H   (Pi: P1 interpolation from the coarsest level); c = coef[0]
void launch_form_u(const Grid& gf, const Grid& gc, double* u, const double* xc_level, const double* coef,
                   hipStream_t s);
// out[0..3] = (u^T K u, u^T M_W u, u^T M u, int u^4): two-stage fixed-order reduction,
// partial must hold kReduceBlocks*4 doubles.  With lam (device scalar): also out[4..5] =
// (|r|^2, |lam M u|^2) of the nodal residual r = K u + M_W u + zeta N(u) - lam M u, and
// partial must hold kReduceBlocks*6 doubles.
constexpr int kReduceBlocks = 512;
void launch_forms(const Grid& g, const Phys& ph, const double* u, double* partial, double* out, hipStream_t s,
                  const double* lam = nullptr);

// ---- vcycle2d.hip ----------------------------------------------------------------------
// fused 2D V-cycle level passes (nu symmetric sweeps = 2 nu + 1 half sweeps, nu <= 2);
// return false when nu is not supported (the caller then uses the unfused kernels).
// zero_x: treat the incoming x as zero (coarse-level corrections) without reading it.
// pre reads x and writes the smoothed values to y; post reads y and writes x (out of place:
// the passes read halos across tiles).  Boundary rings of x and y must be zero.
// ev0/ev1 (optional): events stamped by the dispatch itself at the start and end of the
// post kernel (per-launch timing without the launch gaps of stream-recorded events).
template <typename T> bool launch_vpre2d(const Grid& g, const Grid& gc, const T* x, T* y, const T* f, T* rc,
                                         int nu, int zero_x, hipStream_t s);
// levels above 256 cells per side use the wide tiles, smaller ones 16 x 16
bool vpass2d_wide_tiles(const Grid& g);
// levels l..0 of a 2D V-cycle in one workgroup (level-l mesh n <= 32, nu <= 2): x_l (+)= the
// V-cycle's correction, bit-identical to the level-by-level passes; false if it does not apply
template <typename T> bool launch_vbottom2d(const Grid* levels, int l, T* x, const T* f, int nu_pre, int nu_post,
                                            int zero_x, hipStream_t s);
// the same for 3D (level-l mesh n <= 16, all levels' x and f in LDS)
template <typename T> bool launch_vbottom3d(const Grid* levels, int l, T* x, const T* f, int nu_pre, int nu_post,
                                            int zero_x, hipStream_t s);
template <typename T> bool launch_vpost2d(const Grid& g, const Grid& gc, const T* y, T* x, const T* f, const T* xc,
                                          int nu, hipStream_t s, hipEvent_t ev0 = nullptr,
                                          hipEvent_t ev1 = nullptr);

// ---- vcycle3d.hip ----------------------------------------------------------------------
// fused 3D V-cycle level passes (z-pipelined red-black half sweeps): applies to levels with
// n >= 16 and nu_pre = nu_post in {1, 2}.  pre: x (zero_x: taken as zero) -> smoothed, and
// rc = P^T (f - K x_smoothed); returns the array (x or y) that holds the smoothed values.
// post: x = post smoothing of (that array + P xc); the other array is scratch.
bool vpass3d_applies(const Grid& g, int nu_pre, int nu_post);
// tile variant (0: 256 threads, 1: 512 threads) and the smallest level that takes the
// fused passes (negative / 0: keep the current value)
// 3D: tile variant, smallest fused level, and for V(2,2) one pass of 5 half sweeps per
// side (1) or two of 3 + 2 (0); negative values leave a choice as it is
void set_vpass3d_tuning(int variant, int min_n, int one_pass);
void get_vpass3d_tuning(int* variant, int* min_n, int* one_pass);
// 2D: levels with n > wide_min use the wide tiles (0: the default 256); levels with
// n <= bottom_max run the one-workgroup bottom (0: the default 32, -1: never)
void set_vpass2d_tuning(int wide_min, int bottom_max);
void get_vpass2d_tuning(int* wide_min, int* bottom_max);
// levels between the bottom and the z-pipelined passes: half_sweeps (2 or 3) red-black half
// sweeps from colour `first` in LDS tiles, xin (zero_x: taken as zero) -> xout
bool vtile3d_applies(const Grid& g, int nu_pre, int nu_post);
void set_vtile3d_tuning(int enable);
int get_vtile3d_tuning();
template <typename T> void launch_vtile3d(const Grid& g, const T* xin, T* xout, const T* f, int half_sweeps,
                                          int first, int zero_x, hipStream_t s);
template <typename T> T* launch_vpre3d(const Grid& g, const Grid& gc, T* x, T* y, const T* f, T* rc, int nu,
                                       int zero_x, hipStream_t s, hipEvent_t ev0 = nullptr,
                                       hipEvent_t ev1 = nullptr);
template <typename T> void launch_vpost3d(const Grid& g, const Grid& gc, T* xs, T* scratch, T* x_out, const T* f,
                                          const T* xc, int nu, hipStream_t s, hipEvent_t ev0 = nullptr,
                                          hipEvent_t ev1 = nullptr);

// ---- moments.hip ------------------------------------------------------------------------
int moments_per_element(int dim);            // doubles per coarse element in the output
// chunk_cells: most fine cells one block integrates (0: the default, 8192)
size_t moments_scratch_bytes(int dim, int nc, int n, int chunk_cells = 0);
void launch_moments(int dim, int nc, const Grid& g, const Phys& ph, const double* ut, double* scratch,
                    double* out, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int chunk_cells = 0);

// ---- small.hip --------------------------------------------------------------------------
struct SmallState {
    double lambda;        // current eigenvalue estimate
    double lambda_prev;
    double dlambda;       // |lambda - lambda_prev| / lambda of the last augmented solve
    double c;             // coefficient of u~ of the last augmented solve
    double tol_lambda;    // tolerance-loop threshold (0: inactive)
    int32_t status;       // 0, or FMG_E* of the first failure
    int32_t newton_total;
    int32_t hist_len;
    int32_t done;         // tolerance loop satisfied: later steps become no-ops
    int32_t steps;
    int32_t certify_fail;
    int32_t fail_reason;  // first failure: 1 zero pivot, 2 no convergence, 3 non-finite,
                          // 4 singular border system, 5 not the ground state
    int32_t fail_step;    // history index of the first failure
    double fail_residual; // relative Newton residual at the first failure
    int32_t fac_valid;    // the persistent Jacobian factor holds a usable factor
    int32_t fact_total;   // LDL^T factorisations (Newton, chord refreshes, inertia checks)
    double hist[512];
};
// zero the state and set its tolerance (a kernel, so that a captured graph can replay it)
void launch_init_state(SmallState* st, double tol_lambda, hipStream_t s);
size_t small_arena_bytes(int dim, int nc);
size_t small_factor_bytes(int dim, int nc);   // persistent Jacobian factor
// Coarse nonlinear eigenproblem (Algorithm 3.2 step 1) -> x_H written into the coarsest
// padded level array xc_level, lambda into state.  Ground-state check always on.
int launch_coarse_newton(int dim, int nc, const Phys& ph, int max_iter, double tol, double* arena, double* fac,
                         double* xc_level, SmallState* state, hipStream_t s);
// Augmented nonlinear eigenproblem (3.6) from the moments of u~ -> x_H into xc_level,
// c into state->c, lambda into state (history appended, tolerance flag updated).
// certify: ground-state inertia check (0 never, 1 always, 2 only when the step meets the
// lambda tolerance); reuse: start from the stored factor.
// fixed_iters > 0: accept the iterate after exactly that many iterations (no residual test)
int launch_aug_newton(int dim, int nc, const Phys& ph, int max_iter, int fixed_iters, double tol, const double* moments,
                      double* arena, double* fac, double* xc_level, SmallState* state, int final_level,
                      int certify, int reuse, hipStream_t s);
// Dense augmented matrices A, B, S(x) (row-major (N+1)^2 each) for tests.
int launch_aug_dump(int dim, int nc, const Phys& ph, const double* moments, const double* x, double* arena,
                    double* A, double* B, double* S, hipStream_t s);

}  // namespace fmg
