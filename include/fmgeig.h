/*
 * fmgeig.h -- C ABI of libfmgeig.so, an MI355X (gfx950) implementation of the full
 * multigrid method for nonlinear eigenvalue problems of Jia, Xie, Xie and Xu
 * ("A Full Multigrid Method for Nonlinear Eigenvalue Problems", arXiv:1502.04657).
 *
 * Problem (Section 2, (2.1) with the Gross-Pitaevskii nonlinearity of Example 4.1):
 *     -Laplace(u) + W u + zeta u^3 = lambda u  in [0,1]^dim,  u = 0 on the boundary,
 *     int u^2 = 1,   W(x) = sum_k w_quad[k] x_k^2 + w_const,
 * discretised by P1 elements on nested uniform meshes (2D: cells cut along the
 * (i,j)-(i+1,j+1) diagonal; 3D: cubes cut into 6 Kuhn tetrahedra), level l having
 * n_l = n_coarse * 2^(l-1) cells per side (regular refinement, (3.1)-(3.2)).
 *
 * Conventions for every entry point
 *   - All functions are extern "C" and never throw.  Return 0 on success or a negative
 *     FMG_E* code; fmg_last_error() then returns a thread-local message.
 *   - Pointers named d_* are DEVICE pointers (hipMalloc'd or torch CUDA tensors) on the
 *     current HIP device.  The caller owns every buffer it passes in.  The library
 *     allocates no device memory: fmg_solve works inside the caller's workspace.
 *   - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on it;
 *     fmg_solve returns after its result is complete, the fmg_op_* calls return
 *     after enqueueing (they are asynchronous).
 *   - "Compact" vectors hold the interior nodal values of one level, length (n-1)^dim,
 *     node (i,j[,k]) (1 <= i,j,k <= n-1) at index (i-1) + (n-1)((j-1) + (n-1)(k-1)).
 *   - "Level" arrays use the library's padded layout: (n+1)^dim nodes including the
 *     Dirichlet ring, x fastest, rows padded to fmg_level_pitch(dim, n) elements; node
 *     (i,j[,k]) sits at i + pitch*(j + (n+1)*k).  The ring must hold zeros; kernels
 *     never write it.  fmg_pack / fmg_unpack convert between the two layouts.
 */
#ifndef FMGEIG_H
#define FMGEIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FMG_OK = 0,
    FMG_PENDING = 1,
    FMG_EINVAL = -1,      /* invalid argument (sizes, non-finite inputs, layout)          */
    FMG_ENOMEM = -2,      /* workspace smaller than fmg_workspace_bytes()                 */
    FMG_ENOCONV = -3,     /* a nonlinear solve or the tolerance loop did not converge;    */
                          /* u_out still holds the last iterate                           */
    FMG_ENONFINITE = -4,  /* NaN/Inf appeared in lambda or in the small systems           */
    FMG_EHIP = -5         /* a HIP runtime call failed                                    */
};

enum { FMG_FP64 = 0, FMG_MIXED = 1 };
enum { FMG_SMOOTH_SGS = 0, FMG_SMOOTH_CG = 1 };

/* The problem of Example 4.1 generalised to dim = 2, 3, an anisotropic harmonic W and a
 * constant diagonal SPD coefficient A in a-hat(w, v) = int A grad w . grad v ((2.1),
 * (2.5), (4.1)); the mesh sequence of (3.1)-(3.2).                                     */
typedef struct {
    int32_t dim;          /* 2 or 3; Omega = [0,1]^dim                                    */
    int32_t n_coarse;     /* cells per side of the coarsest mesh T_{h_1} (= T_H), >= 2    */
    int32_t n_refine;     /* regular refinements; finest n = n_coarse * 2^n_refine        */
    int32_t reserved;
    double  w_quad[3];    /* W(x) = sum_k w_quad[k] x_k^2 + w_const                        */
    double  w_const;
    double  zeta;         /* >= 0, coefficient of u^3                                     */
    double  diffusion[3]; /* A = diag(diffusion[0..dim-1]), each > 0; all zero: A = I     */
} fmg_problem;

/* Algorithm 3.1 / 3.2 parameters.                                                        */
typedef struct {
    double  tol_lambda;   /* > 0: after the p steps of the finest level, continue          */
                          /* correction steps until |dlambda| <= tol_lambda * lambda;     */
                          /* 0: fixed schedule                                            */
    int32_t m;            /* V-cycles per correction step, MG(.,.,.,m) of (3.5), >= 1      */
    int32_t p;            /* correction steps per level (Algorithm 3.2), >= 1              */
    int32_t nu_pre;       /* symmetric Gauss-Seidel sweeps before / after the coarse       */
    int32_t nu_post;      /* correction of each V-cycle level                             */
    int32_t max_final_steps; /* cap on the tolerance loop                                   */
    int32_t newton_max_iter; /* cap per nonlinear solve (Newton iterations)                 */
    double  newton_tol;   /* relative residual at which a Newton solve stops (e.g. 1e-13)  */
    int32_t precision;    /* FMG_FP64, or FMG_MIXED: FP32 V-cycles inside an FP64          */
                          /* iterative-refinement loop (residual, quadratures, Rayleigh   */
                          /* quotient and the small eigensolves stay FP64)                */
    int32_t newton_fixed_iters; /* 0: every augmented problem (3.6) is solved to          */
                          /* newton_tol; k > 0: exactly k nonlinear iterations per        */
                          /* augmented problem, accepted without a residual test (the     */
                          /* fixed-iteration-count variant of Section 3.3; the coarse     */
                          /* problem of Algorithm 3.2 step 1 is still solved to newton_tol)*/
    int32_t smoother;     /* FMG_SMOOTH_SGS: nu red-black symmetric Gauss-Seidel sweeps;   */
                          /* FMG_SMOOTH_CG: nu conjugate-gradient steps on K x = f (the     */
                          /* smoother of the paper's experiments, Section 4)              */
    int32_t reserved;
} fmg_options;

#define FMG_HISTORY_MAX 512

typedef struct {
    double  lambda;       /* final eigenvalue: the augmented-problem eigenvalue of (3.6)  */
    double  lambda_rq;    /* a(u,u)/b(u,u) of (2.2) evaluated on the finest level         */
    double  norm;         /* b(u,u) of the returned u (1 up to rounding)                  */
    double  dlambda;      /* |lambda_last - lambda_previous| / lambda of the last step     */
    int32_t status;       /* 0 or FMG_E*                                                   */
    int32_t levels;
    int32_t steps_total;  /* correction steps executed (all levels)                       */
    int32_t newton_total; /* Newton iterations (coarse step + every augmented solve)      */
    double  seconds;      /* host wall time: of the call (fmg_solve); from the batch call  */
                          /* or the submission to completion (batch, server)              */
    double  wait_seconds; /* batch / server: time queued before admission (0 otherwise)   */
    int32_t history_len;  /* entries in history[]                                         */
    int32_t factor_total; /* banded LDL^T factorisations of the small solves (incl. checks)  */
    double  residual;     /* |K u + M_W u + zeta N(u) - lambda M u|_2 / |lambda M u|_2 on the  */
                          /* finest level: nodal residual of the discrete problem (2.4)    */
    double  gamma_est;    /* contraction estimate of the finest-level correction steps     */
                          /* (Theorem 3.1): |dlambda_last| / |dlambda_previous|; -1 when    */
                          /* fewer than three finest-level steps ran                      */
    double  history[FMG_HISTORY_MAX]; /* lambda after the coarse step and after every      */
                                      /* correction step, in execution order              */
} fmg_result;

const char* fmg_last_error(void);
const char* fmg_version(void);

/* Select the V-cycle implementation for later calls in this process: 1 (default) fused
 * temporally blocked level passes (2D; 3D levels with n >= 16 and nu_pre = nu_post in
 * {1, 2}), 0 the unfused kernel sequence.  Both execute the same floating-point operations
 * and give identical results.  Not thread-safe.                                          */
int fmg_set_fused_vcycle(int32_t enable);

/* ---- kernel tuning ------------------------------------------------------------------------ */
/* Launch choices of the fused V-cycle passes, process-wide (not thread-safe; set them before
 * solves start).  They change speed only: every choice gives the same bits.  The values come
 * from fmg_autotune_vcycle or a cache of its results.                                    */
typedef struct {
    int32_t vpass3d_variant;  /* 3D pass tiles (region columns x rows, threads): 0 = 32 x 16,  */
                              /* 256; 1 = 32 x 32, 512; 2 = 64 x 16, 512; 3 = 64 x 32, 512   */
                              /* (two region pairs per thread)                                */
    int32_t vpass3d_min_n;    /* smallest 3D level (cells per side) on the fused passes      */
    int32_t vpass2d_wide_min_n; /* 2D levels with more cells per side use the wide tiles    */
                                /* (0 in fmg_set_tuning: the default 256)                    */
    int32_t vbottom2d_max_n;  /* 2D levels with at most this many cells per side run the    */
                              /* one-workgroup V-cycle bottom (0: the default 32; -1: never; */
                              /* at most 64)                                                 */
    int32_t vpass3d_one_pass; /* 3D V(2,2): 1 = one pass of 5 half sweeps per side (5-ring  */
                              /* halo), 0 = two passes of 3 + 2                              */
    int32_t vtile3d;          /* 3D levels between the one-workgroup bottom (n <= 16) and    */
                              /* vpass3d_min_n: 1 (or 0: the default) = the half sweeps of a */
                              /* side in LDS tiles of 8^3 nodes, 3 + 2 per launch; -1 = one  */
                              /* launch per half sweep                                       */
    int32_t reserved[2];
} fmg_tuning;
int fmg_get_tuning(fmg_tuning* out);
int fmg_set_tuning(const fmg_tuning* in);   /* FMG_EINVAL for values out of range            */
/* Tile autotuner: times whole V(2,2) cycles (every level down to the exact coarsest solve)
 * of a level with n cells per side, in FP64 (precision FMG_FP64) or FP32 (FMG_MIXED), on a
 * scratch hierarchy it allocates and frees, and returns the fastest choice in *out: in 3D
 * over every pass variant, smallest fused level (16, 32, ... up to "none") and the small
 * levels' LDS tiles or per-half-sweep launches, in 2D over
 * the level from which the wide tiles are used (64 .. n, or none) and the largest level of
 * the one-workgroup bottom (none, 16, 32, 64).  The other dimension's fields keep their
 * current values.  The current tuning is left as it was; apply the result with
 * fmg_set_tuning.  n must be n_c 2^k with 2 <= n_c <= 7 (3D, 16 <= n <= 1024) or
 * 8 <= n_c <= 31 (2D, 64 <= n <= 32768).  Synchronises `stream`; not to be called while
 * solves run.                                                                            */
int fmg_autotune_vcycle(int32_t dim, int32_t n, int32_t precision, void* stream, fmg_tuning* out);

/* ---- measurement hooks ------------------------------------------------------------------ */
/* Per-launch timing of one kernel inside later solves: a pair of HIP events is stamped by
 * each launch's own dispatch on its stream (hipExtLaunchKernel start/stop events, so the
 * interval is the kernel's execution without launch gaps; up to max_launches), with the
 * algorithmic bytes and the units of work of each launch.  Only launches on the finest level
 * of each solve are recorded (N_l: interior nodes of that level, N_{l-1} of the next coarser):
 *   FMG_PROF_VPOST2D_F64  fused 2D FP64 post-smoothing level pass (prolongation-add plus the
 *                         post half sweeps) when the level has more than 256 cells per side;
 *                         bytes 8 (3 N_l + N_{l-1}) (read x, f, the coarse correction; write x);
 *                         units N_l.
 *   FMG_PROF_VPOST3D_F64  fused 3D FP64 pass of prolongation-add plus three post half sweeps;
 *                         bytes 8 (3 N_l + N_{l-1}); units N_l.
 *   FMG_PROF_VPRE3D_F64   fused 3D FP64 pass of the first three pre half sweeps (out of place);
 *                         bytes 8 * 3 N_l (read x, f; write the new iterate); units N_l.
 *   FMG_PROF_MOMENTS3D    3D fine-grid moment pass (the per-block partial integrals of the
 *                         augmented problem); bytes 8 N_l (read u~; the partials are small);
 *                         units: fine cells n^3.
 *   FMG_PROF_RHS3D        3D right-hand side (3.4); bytes 16 N_l (read u, write b); units N_l.
 * Not thread-safe; one profile at a time.  The events are created without a system-scope
 * fence (timing only); fmg_profile_end synchronises the device and fills *out.             */
enum {
    FMG_PROF_VPOST2D_F64 = 1,
    FMG_PROF_VPOST3D_F64 = 2,
    FMG_PROF_VPRE3D_F64 = 3,
    FMG_PROF_MOMENTS3D = 4,
    FMG_PROF_RHS3D = 5
};
typedef struct {
    int64_t launches;   /* launches recorded                                               */
    double seconds;     /* sum of the per-launch event intervals                           */
    double bytes;       /* sum of the algorithmic bytes of those launches                  */
    double units;       /* sum of the units of work (nodes or cells) of those launches     */
} fmg_kernel_profile;
int fmg_profile_begin(int32_t kernel, int32_t max_launches);
int fmg_profile_end(fmg_kernel_profile* out);

/* ---- whole solve (Algorithm 3.2) ---------------------------------------------------- */

/* Bytes of device workspace fmg_solve needs for this problem and options.  Pure function.
 * Returns FMG_EINVAL for invalid problems/options.                                       */
int fmg_workspace_bytes(const fmg_problem* prob, const fmg_options* opt, size_t* bytes);

/* Full multigrid eigensolve: coarse nonlinear solve (Algorithm 3.2 step 1), then on every
 * finer level FMG prolongation and p correction steps (Algorithm 3.1: right-hand side of
 * (3.4), m V-cycles (3.5), augmented nonlinear eigenproblem (3.6) on V_H + span{u~}),
 * plus the tolerance loop on the finest level when opt->tol_lambda > 0.
 *   d_workspace : device memory of at least fmg_workspace_bytes() bytes, 256-B aligned;
 *                 contents on entry are ignored (the call initialises what it uses).
 *   d_u_out     : compact layout, u_len = (n-1)^dim, device or host memory (told apart with
 *                 hipPointerGetAttributes; a host target is written by a device-to-host
 *                 copy before the call returns); receives u_h with
 *                 b(u,u) = 1 and int u_h > 0.
 *   out         : host struct, filled on return (also on FMG_ENOCONV).
 * The coarsest solution and the returned state (last step of a fixed schedule, or the step
 * that meets tol_lambda) are checked to be the ground state by an inertia count; a failed
 * check returns FMG_ENOCONV.
 * Errors: FMG_EINVAL (dim not 2/3, n_coarse < 2, n_refine < 0 or > 12, zeta < 0 or
 * non-finite inputs, m/p < 1, nu_pre + nu_post < 1, u_len mismatch), FMG_ENOMEM
 * (workspace too small), FMG_ENOCONV, FMG_ENONFINITE, FMG_EHIP.                            */
int fmg_solve(const fmg_problem* prob, const fmg_options* opt, void* d_workspace,
              size_t workspace_bytes, void* stream, double* d_u_out, int64_t u_len,
              fmg_result* out);

/* fmg_solve for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the workspace is a static device array of
 * FMG_STATIC_WORKSPACE_BYTES bytes that the library holds on every GPU it runs on until the
 * process ends, and the call allocates no device memory and no pinned host memory (the
 * host mirror of the device state lives on the caller's stack).  Same problem, options,
 * output and errors as fmg_solve; FMG_ENOMEM, before any device work, when the problem's
 * workspace (fmg_workspace_bytes) exceeds FMG_STATIC_WORKSPACE_BYTES (e.g. 2D up to
 * n = 1024, 3D up to n = 64 in FP64).  Every call on one GPU uses that GPU's one array,
 * whose contents the call initialises itself: calls that overlap on the same GPU (other
 * threads or streams) race and must be serialised by the caller.                       */
#define FMG_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int fmg_solve_static(const fmg_problem* prob, const fmg_options* opt, void* stream, double* u_out, int64_t u_len,
                     fmg_result* out);

/* ---- many solves: footprint, allocator, batch, serving -------------------------------- */
/* Every instance below is the problem and method of fmg_solve (Section 2 problem, the
 * mesh sequence of (3.1)-(3.2), Algorithm 3.2 with the tolerance loop); results are bitwise
 * those of fmg_solve on the same problem and options, alone or in any mix.               */

/* Device bytes one solve holds while it runs (its workspace, rounded to 256 B): the
 * admission footprint of the batch and serving calls.  Pure; 0 for an invalid problem
 * or options.                                                                            */
size_t fmg_footprint_bytes(const fmg_problem* prob, const fmg_options* opt);

/* Device allocator for the memory pools of fmg_batch_solve and fmg_server_create (e.g.
 * torch's caching allocator).  alloc(bytes, ctx) must return 256-B aligned device memory
 * or NULL; free(ptr, ctx) releases it.  Both NULL restores hipMalloc / hipFree.  A pool
 * is freed with the allocator that created it.  Applies to pools created afterwards.      */
int fmg_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_fn)(void* ptr, void* ctx),
                      void* ctx);

/* fmg_solve with the workspace allocated for the call (through the allocator registered
 * with fmg_set_allocator, else hipMalloc) and released before it returns: the problem
 * statement alone in, (lambda, u_h) out.  Same arguments and errors as fmg_solve, plus
 * FMG_ENOMEM when the allocation fails.                                                  */
int fmg_solve_alloc(const fmg_problem* prob, const fmg_options* opt, void* stream, double* u_out, int64_t u_len,
                    fmg_result* out);

/* Solve `count` independent instances (probs[i], opts[i]) together: one pool holding every
 * workspace is allocated for the call, up to 8 instances run at once on streams of their
 * own (their kernels overlap on the device), and each u is written to d_u_out[i] (device,
 * compact layout, u_len[i] = (n_i - 1)^dim_i).  Work already enqueued on `stream` runs
 * first.  Returns after every instance is done; out[i] is filled for each (seconds: from
 * the call to that instance's completion, wait_seconds: until its admission).  Returns 0,
 * or the status of the first failed instance (the others still complete), or FMG_EINVAL /
 * FMG_ENOMEM before any work for bad arguments or a failed pool allocation.              */
int fmg_batch_solve(int32_t count, const fmg_problem* probs, const fmg_options* opts, void* stream,
                    double* const* d_u_out, const int64_t* u_len, fmg_result* out);

/* A batch plan: the instances of a batch set up once (one pool for all their workspaces,
 * through the allocator of fmg_set_allocator else hipMalloc) and each instance's kernel
 * sequence captured into HIP graphs: the first chunk of its solve (state initialisation,
 * Algorithm 3.2 step 1 and every level's p correction steps), one more finest-level
 * correction step (replayed while the lambda tolerance is not met) and the final chunk
 * (Rayleigh quotient and residual).  fmg_batch_plan_run replays them for every instance,
 * the instances spread over up to 16 streams of the plan (their graphs overlap on the
 * device), one host thread deciding between the chunks from the copied-back state, and
 * writes each u into d_u_out[i] (device, compact, u_len[i] = (n_i - 1)^dim_i).  Results
 * are bitwise those of fmg_solve.  Work already enqueued on `stream` runs before a run's
 * first graph; run returns after every instance is done, out[i] as for fmg_batch_solve.
 * A plan runs any number of times; runs of one plan must not overlap.  create returns
 * NULL on failure (fmg_last_error says why): invalid instances, FMG_ENOMEM, or a capture
 * failure.                                                                               */
typedef struct fmg_batch_plan fmg_batch_plan;
fmg_batch_plan* fmg_batch_plan_create(int32_t count, const fmg_problem* probs, const fmg_options* opts,
                                      void* stream);
int fmg_batch_plan_run(fmg_batch_plan* plan, double* const* d_u_out, const int64_t* u_len, fmg_result* out);
void fmg_batch_plan_destroy(fmg_batch_plan* plan);

/* Serving: continuous batching of requests of different sizes.  The server owns a pool of
 * hbm_budget bytes (0: half of the free device memory) and up to max_slots (1..64)
 * streams, and a worker thread that admits queued requests in FIFO order whenever a
 * stream and fmg_footprint_bytes() of pool memory are free, and advances running ones.
 * A finished request keeps its workspace until it is polled.  Work of the caller on
 * `stream` before a request's admission runs first; poll copies u on `stream`.
 * create returns NULL on failure (fmg_last_error says why).                              */
typedef struct fmg_server fmg_server;
fmg_server* fmg_server_create(size_t hbm_budget, int32_t max_slots, void* stream);
/* Queue one request.  FMG_EINVAL for invalid problems/options, FMG_ENOMEM when its
 * footprint exceeds the whole budget (it could never be admitted).  Thread-safe.         */
int fmg_server_submit(fmg_server* server, const fmg_problem* prob, const fmg_options* opt,
                      uint64_t* ticket);
/* FMG_PENDING (1) while the request is queued or running.  Once done: fills *out (seconds:
 * submission to completion, wait_seconds: submission to admission), copies u into d_u_out
 * (device, compact, u_len = (n-1)^dim; NULL to skip) and synchronises `stream`, releases
 * the request's memory and forgets the ticket; returns the solve's status.  FMG_EINVAL for
 * an unknown ticket or a wrong u_len (the request stays pollable).  Thread-safe.          */
int fmg_server_poll(fmg_server* server, uint64_t ticket, fmg_result* out, double* d_u_out, int64_t u_len);
/* Stops admissions, waits for running requests to finish, frees everything (requests not
 * yet polled are dropped).                                                               */
void fmg_server_destroy(fmg_server* server);

/* ---- level layout -------------------------------------------------------------------- */
int64_t fmg_level_pitch(int32_t dim, int32_t n);   /* row pitch in elements, or -1          */
int64_t fmg_level_elems(int32_t dim, int32_t n);   /* elements of one level array, or -1    */

/* compact <-> level layout (FP64).  pack writes the interior only; the caller zeroes the
 * ring of d_level once (e.g. at allocation).                                              */
int fmg_pack(int32_t dim, int32_t n, const double* d_compact, double* d_level, void* stream);
int fmg_unpack(int32_t dim, int32_t n, const double* d_level, double* d_compact, void* stream);

/* ---- single steps of the method (level layout; for tests and custom schedules) -------- */

/* Right-hand side of the auxiliary problem (3.4) with f(x,u) = W u + zeta u^3:
 *   b_i = lambda (M u)_i - int W u_h phi_i - zeta int u_h^3 phi_i   (exact P1 integration)
 * on the level with n cells per side.  FP64.                                             */
int fmg_op_rhs(const fmg_problem* prob, int32_t n, double lambda, const double* d_u,
               double* d_b, void* stream);

/* Red-black symmetric Gauss-Seidel on K x = f (K: P1 stiffness matrix of a-hat, (2.5)):
 * `sweeps` symmetric sweeps (forward red,black then backward black,red).  precision:
 * FMG_FP64 (double*) or FMG_MIXED meaning FP32 (float* passed as void*).                 */
int fmg_op_smooth(int32_t dim, int32_t n, int32_t precision, void* d_x, const void* d_f,
                  int32_t sweeps, void* stream);

/* `steps` iterations of the conjugate gradient method on K x = f started from x (the
 * smoother of the paper's experiments, Section 4): r = f - K x, p = r; per step q = K p,
 * alpha = r.r / p.q, x += alpha p, r -= alpha q, p = r + (r'.r' / r.r) p.  Dot products in
 * FP64 with a fixed summation order.  d_scratch: device, 256-B aligned, at least
 * 3 * round256(s * fmg_level_elems(dim, n)) + 8 * (512 + 8) bytes, s = 8 (FMG_FP64) or 4. */
int fmg_op_cg_smooth(int32_t dim, int32_t n, int32_t precision, void* d_x, const void* d_f,
                     int32_t steps, void* d_scratch, size_t scratch_bytes, void* stream);

/* r_c = P^T (f - K x): residual of the fine level (n cells) restricted to level n/2.      */
int fmg_op_residual_restrict(int32_t dim, int32_t n, int32_t precision, const void* d_x,
                             const void* d_f, void* d_rc, void* stream);

/* x_f (+)= P x_c, P = P1 interpolation from level n/2 to level n; accumulate 0: overwrite */
int fmg_op_prolong(int32_t dim, int32_t n, int32_t precision, const void* d_xc, void* d_xf,
                   int32_t accumulate, void* stream);

/* Exact solve K x = f on a coarsest level with n cells per side (n <= 64).               */
int fmg_op_coarse_solve(int32_t dim, int32_t n, int32_t precision, const void* d_f, void* d_x,
                        void* stream);

/* One V(nu_pre, nu_post)-cycle for K x = f on level n = n_coarse * 2^(levels-1), using the
 * library's level hierarchy in d_workspace (bytes from fmg_workspace_bytes of a problem with
 * the same dim, n_coarse and n_refine = levels-1).  FP64.                                */
int fmg_op_vcycle(int32_t dim, int32_t n_coarse, int32_t levels, int32_t nu_pre, int32_t nu_post,
                  double* d_x, const double* d_f, void* d_workspace, size_t workspace_bytes,
                  void* stream);

/* Fine-grid quadratures that build the augmented problem (3.6) for V_H + span{u~}:
 * for every coarse simplex E (index (cell * S + type), cell = I + nc*(J + nc*K), S = 2 (2D)
 * or 6 (3D) simplices per cell in the order of the mesh description above), d_out receives
 * fmg_moments_layout().per_element doubles:
 *   int_E u~ l_p l_q l_r (p<=q<=r), int_E u~^2 l_p l_q (p<=q), int_E u~^3 l_p, int_E u~^4,
 *   int_E u~ l_p, int_E u~^2, int_E W u~ l_p, int_E W u~^2, int_E grad u~ . grad l_p,
 *   int_E |grad u~|^2
 * (l_p: barycentric coordinates of E; multisets in lexicographic order).  d_ut is a level
 * array with n cells per side; d_scratch holds scratch_bytes of fmg_moments_layout.      */
int fmg_moments_layout(int32_t dim, int32_t n_coarse, int32_t n, int32_t* per_element,
                       size_t* scratch_bytes);
int fmg_op_moments(const fmg_problem* prob, int32_t n, const double* d_ut, double* d_out,
                   void* d_scratch, size_t scratch_bytes, void* stream);
/* The same with the fine cells of each coarse simplex split into blocks of at most
 * chunk_cells cells (0: the default of fmg_op_moments and fmg_solve, 8192), for tests of the
 * block decomposition: the partial sums are added in another order, so results agree to
 * rounding, not bit for bit.  With s = n / n_c, a coarse simplex has s (s-1) / 2 (2D) or
 * s (s-1) (s-2) / 6 (3D) interior cells and s (2D) or s^2 (3D) cells on its internal faces,
 * each group split into ceil(cells / chunk_cells) blocks; every block writes 23 (2D) or 39
 * (3D) doubles of scratch.  FMG_EINVAL for chunk_cells outside [0, 2^20], FMG_ENOMEM when
 * scratch_bytes is smaller than that.                                                      */
int fmg_op_moments_chunked(const fmg_problem* prob, int32_t n, const double* d_ut, double* d_out,
                           void* d_scratch, size_t scratch_bytes, int32_t chunk_cells, void* stream);

/* Device scratch (bytes) of the small nonlinear solves on the coarsest space.             */
int fmg_small_scratch_bytes(int32_t dim, int32_t n_coarse, size_t* bytes);

/* Dense augmented matrices of (3.6) in the basis [coarse hats (compact order), u~]:
 * A = Z^T (K + M_W) Z, B = Z^T M Z, S = Z^T M_{(Zx)^2} Z, each (N+1)x(N+1) row-major,
 * N = (n_coarse-1)^dim, from the moments of u~ and the coefficient vector d_x (N+1).     */
int fmg_op_augmented_matrices(const fmg_problem* prob, const double* d_moments, const double* d_x,
                              double* d_A, double* d_B, double* d_S, void* d_scratch,
                              size_t scratch_bytes, void* stream);

/* Ground state of the augmented problem (3.6) from the moments of u~ (Newton on the
 * bordered system).  d_xc_level: coarsest level array (ring zero) receiving x_H; returns
 * lambda, the u~ coefficient c (u = Pi x_H + c u~), the Newton iteration count and
 * whether the ground-state inertia check passed.  Synchronises the stream.               */
int fmg_op_augmented_solve(const fmg_problem* prob, const fmg_options* opt, const double* d_moments,
                           double* d_xc_level, void* d_scratch, size_t scratch_bytes, void* stream,
                           double* lambda, double* c, int32_t* newton_iters, int32_t* ground_state);

/* Ground state on the coarsest space (Algorithm 3.2 step 1): x written into d_xc_level,
 * lambda returned.  Synchronises the stream.                                             */
int fmg_op_coarse_nonlinear(const fmg_problem* prob, const fmg_options* opt, double* d_xc_level,
                            void* d_scratch, size_t scratch_bytes, void* stream, double* lambda,
                            int32_t* newton_iters, int32_t* ground_state);

/* u <- c u + Pi x_H on level n (Pi: P1 interpolation from the coarsest level). FP64.
 * n = n_coarse 2^k (a level of the hierarchy), else FMG_EINVAL.                          */
int fmg_op_form_u(int32_t dim, int32_t n_coarse, int32_t n, double c, const double* d_xc_level,
                  double* d_u, void* d_scratch, void* stream);

/* (u^T K u, u^T M_W u, u^T M u, int u_h^4) of a level array; d_scratch >= 4200 doubles.  */
int fmg_op_forms(const fmg_problem* prob, int32_t n, const double* d_u, double* out4,
                 void* d_scratch, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FMGEIG_H */
