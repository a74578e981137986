// C ABI and host schedule of the full multigrid eigensolver (Algorithm 3.2 driving
// Algorithm 3.1).  Every arithmetic step runs in the HIP kernels; the host only carves the
// caller's workspace, enqueues kernels on the caller's stream and, in tolerance mode,
// reads the device-side convergence flag between finest-level correction steps.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/fmgeig.h"
#include "job.h"

namespace fmg {

constexpr int kMaxDevices = 64;
static thread_local char g_err[512] = "";
// fused 2D V-cycle passes (1) or the unfused kernel sequence (0); both give identical bits
static int g_fused = 1;

// Optional per-launch timing of one kernel (instrumentation for measurements): HIP events
// recorded around each launch on the stream it runs on, plus the algorithmic bytes and the
// units of work of each launch.  Not thread-safe.
struct KernelProfiler {
    int kernel = 0;                  // FMG_PROF_* being recorded, 0: off
    int cap = 0, used = 0;
    std::vector<hipEvent_t> ev;      // 2 per launch
    double bytes = 0.0, units = 0.0;
};
static KernelProfiler g_prof;

// is the next launch of `kind` to be recorded
static bool prof_on(int kind) { return g_prof.kernel == kind && g_prof.used < g_prof.cap; }
// start (k = 0) or stop (k = 1) event of the next recorded launch, or none
static hipEvent_t prof_ev(bool on, int k) { return on ? g_prof.ev[2 * (size_t)g_prof.used + k] : nullptr; }
static void prof_add(double bytes, double units) {
    g_prof.bytes += bytes;
    g_prof.units += units;
    ++g_prof.used;
}
static double interior_nodes(const Grid& g) { return std::pow((double)(g.n - 1), (double)g.dim); }

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

bool is_device_pointer(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // unregistered host memory
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// the diagonal of A (all zero in the problem: the identity)
static void diffusion_of(const fmg_problem* p, double* a) {
    const bool id = p->diffusion[0] == 0.0 && p->diffusion[1] == 0.0 && p->diffusion[2] == 0.0;
    for (int k = 0; k < 3; ++k) a[k] = (id || k >= p->dim) ? 1.0 : p->diffusion[k];
}

static Phys make_phys(const fmg_problem* p) {
    Phys ph;
    for (int k = 0; k < 3; ++k) ph.w[k] = (k < p->dim) ? p->w_quad[k] : 0.0;
    ph.wc = p->w_const;
    ph.zeta = p->zeta;
    diffusion_of(p, ph.a);
    return ph;
}

// a level of the problem's mesh sequence, with its coefficient
static Grid problem_grid(const fmg_problem* p, int n) {
    double a[3];
    diffusion_of(p, a);
    return with_diffusion(make_grid(p->dim, n), a);
}

int check_problem(const fmg_problem* p) {
    if (!p) return set_error(FMG_EINVAL, "problem is NULL");
    if (p->dim != 2 && p->dim != 3) return set_error(FMG_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->n_coarse < 2) return set_error(FMG_EINVAL, "n_coarse must be >= 2 (got %d)", p->n_coarse);
    if (p->n_refine < 0 || p->n_refine > 12) return set_error(FMG_EINVAL, "n_refine out of range (got %d)", p->n_refine);
    if (p->dim == 2 && p->n_coarse > 32) return set_error(FMG_EINVAL, "2D n_coarse must be <= 32");
    if (p->dim == 3 && p->n_coarse > 16) return set_error(FMG_EINVAL, "3D n_coarse must be <= 16");
    int64_t n = (int64_t)p->n_coarse << p->n_refine;
    if (p->dim == 2 && n > 32768) return set_error(FMG_EINVAL, "finest 2D n too large");
    if (p->dim == 3 && n > 1024) return set_error(FMG_EINVAL, "finest 3D n too large");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->w_quad[k])) return set_error(FMG_EINVAL, "w_quad[%d] is not finite", k);
    if (!std::isfinite(p->w_const)) return set_error(FMG_EINVAL, "w_const is not finite");
    if (!std::isfinite(p->zeta) || p->zeta < 0.0) return set_error(FMG_EINVAL, "zeta must be finite and >= 0");
    const bool id = p->diffusion[0] == 0.0 && p->diffusion[1] == 0.0 && p->diffusion[2] == 0.0;
    for (int k = 0; k < p->dim && !id; ++k)
        if (!std::isfinite(p->diffusion[k]) || !(p->diffusion[k] > 0.0))
            return set_error(FMG_EINVAL, "diffusion[%d] must be finite and > 0 (or all zero: A = I)", k);
    return 0;
}

int check_options(const fmg_options* o) {
    if (!o) return set_error(FMG_EINVAL, "options is NULL");
    if (o->m < 1 || o->p < 1) return set_error(FMG_EINVAL, "m and p must be >= 1");
    if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_pre + o->nu_post < 1)
        return set_error(FMG_EINVAL, "nu_pre, nu_post >= 0 with nu_pre + nu_post >= 1");
    if (!(o->tol_lambda >= 0.0) || !std::isfinite(o->tol_lambda)) return set_error(FMG_EINVAL, "tol_lambda invalid");
    if (o->max_final_steps < 0) return set_error(FMG_EINVAL, "max_final_steps must be >= 0");
    if (o->newton_max_iter < 1) return set_error(FMG_EINVAL, "newton_max_iter must be >= 1");
    if (!(o->newton_tol > 0.0)) return set_error(FMG_EINVAL, "newton_tol must be > 0");
    if (o->newton_fixed_iters < 0 || o->newton_fixed_iters > o->newton_max_iter)
        return set_error(FMG_EINVAL, "newton_fixed_iters must be in [0, newton_max_iter]");
    if (o->precision != FMG_FP64 && o->precision != FMG_MIXED) return set_error(FMG_EINVAL, "precision invalid");
    if (o->smoother != FMG_SMOOTH_SGS && o->smoother != FMG_SMOOTH_CG) return set_error(FMG_EINVAL, "smoother invalid");
    return 0;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

Layout make_layout(int dim, int nc, int levels, int mixed, int cg) {
    Layout lo;
    lo.dim = dim; lo.nc = nc; lo.L = levels; lo.mixed = mixed; lo.cg = cg;
    for (int l = 0; l < levels; ++l) lo.g.push_back(make_grid(dim, nc << l));
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    lo.state = take(sizeof(SmallState));
    lo.xc = take(sizeof(double) * lo.g[0].elems);
    const size_t ts = mixed ? sizeof(float) : sizeof(double);
    lo.u.resize(levels); lo.b.resize(levels); lo.xv.resize(levels); lo.fv.resize(levels); lo.tv.resize(levels);
    for (int l = 0; l < levels; ++l) {
        lo.u[l] = (l == 0) ? lo.xc : take(sizeof(double) * lo.g[l].elems);
        lo.b[l] = take(sizeof(double) * lo.g[l].elems);
        // V-cycle work arrays; in FP64 mode the top level uses u/b directly
        bool top_only = !mixed && l == levels - 1;
        lo.xv[l] = top_only ? 0 : take(ts * lo.g[l].elems);
        lo.fv[l] = top_only ? 0 : take(ts * lo.g[l].elems);
        // the fused passes run in the V-cycle precision; the coarsest level needs none
        lo.tv[l] = l > 0 ? take(ts * lo.g[l].elems) : 0;
    }
    if (cg) {
        // CG smoothing: r, p, q sized for the finest level (zero rings: inside the zeroed range)
        const size_t e = ts * lo.g[levels - 1].elems;
        lo.cgr = take(e);
        lo.cgp = take(e);
        lo.cgq = take(e);
    }
    const int64_t ncell = dim == 2 ? (int64_t)nc * nc : (int64_t)nc * nc * nc;
    const int ne = dim == 2 ? 2 : 6;
    lo.mom = take(sizeof(double) * ncell * ne * moments_per_element(dim));
    size_t ms = 0;
    for (int l = 1; l < levels; ++l) ms = std::max(ms, moments_scratch_bytes(dim, nc, nc << l));
    lo.momscr = take(std::max<size_t>(ms, 256));
    lo.arena = take(small_arena_bytes(dim, nc));
    lo.fac = take(small_factor_bytes(dim, nc));
    lo.forms = take(sizeof(double) * (kReduceBlocks * 6 + 8));
    if (cg) lo.cgsc = take(sizeof(double) * (kReduceBlocks + 8));   // partials, then 4 scalars
    lo.total = off;
    return lo;
}

Layout layout_for(const fmg_problem* p, const fmg_options* o) {
    Layout lo = make_layout(p->dim, p->n_coarse, p->n_refine + 1, o->precision == FMG_MIXED,
                            o->smoother == FMG_SMOOTH_CG);
    double a[3];
    diffusion_of(p, a);
    for (auto& g : lo.g) g = with_diffusion(g, a);
    return lo;
}

template <typename T>
static T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

// ----------------------------------------------------------------------------------------
// V-cycle: x_l (+)= MG step for K_l x = f_l; levels below l use the workspace arrays.
// zero_x: x enters as zero (it is not read).  2D uses the fused level passes.
template <typename T>
static void vcycle(const Layout& lo, void* ws, int l, T* x, const T* f, int nu_pre, int nu_post, hipStream_t s,
                   bool zero_x = false) {
    const Grid& g = lo.g[l];
    if (l == 0) {
        launch_coarse_solve<T>(g, f, x, s);
        return;
    }
    T* xc = at<T>(ws, lo.xv[l - 1]);
    T* fc = at<T>(ws, lo.fv[l - 1]);
    if (lo.dim == 2 && nu_pre <= 2 && nu_post <= 2 && g_fused && !lo.cg) {
        // a small level and everything below it: one workgroup, all levels in LDS
        if (launch_vbottom2d<T>(lo.g.data(), l, x, f, nu_pre, nu_post, zero_x ? 1 : 0, s)) return;
        T* y = at<T>(ws, lo.tv[l]);
        launch_vpre2d<T>(g, lo.g[l - 1], x, y, f, fc, nu_pre, zero_x ? 1 : 0, s);
        vcycle<T>(lo, ws, l - 1, xc, fc, nu_pre, nu_post, s, true);
        const bool rec = sizeof(T) == 8 && l == lo.L - 1 && vpass2d_wide_tiles(g) && prof_on(FMG_PROF_VPOST2D_F64);
        launch_vpost2d<T>(g, lo.g[l - 1], y, x, f, xc, nu_post, s, prof_ev(rec, 0), prof_ev(rec, 1));
        // read x, f and the coarse correction, write x (interior values)
        if (rec) prof_add((3.0 * interior_nodes(g) + interior_nodes(lo.g[l - 1])) * sizeof(double), interior_nodes(g));
        return;
    }
    if (lo.dim == 3 && g_fused && !lo.cg &&
        launch_vbottom3d<T>(lo.g.data(), l, x, f, nu_pre, nu_post, zero_x ? 1 : 0, s))
        return;
    if (lo.dim == 3 && g_fused && !lo.cg && vpass3d_applies(g, nu_pre, nu_post)) {
        T* y = at<T>(ws, lo.tv[l]);
        const bool top = sizeof(T) == 8 && l == lo.L - 1;
        const double nf = interior_nodes(g), ncs = interior_nodes(lo.g[l - 1]);
        const bool rpre = top && prof_on(FMG_PROF_VPRE3D_F64);
        T* xs = launch_vpre3d<T>(g, lo.g[l - 1], x, y, f, fc, nu_pre, zero_x ? 1 : 0, s, prof_ev(rpre, 0),
                                 prof_ev(rpre, 1));
        // first pre pass: read x (unless it enters as zero) and f, write the new iterate (and,
        // for one sweep, the restricted residual)
        if (rpre) prof_add(((zero_x ? 2.0 : 3.0) * nf + (nu_pre == 1 ? ncs : 0.0)) * sizeof(double), nf);
        vcycle<T>(lo, ws, l - 1, xc, fc, nu_pre, nu_post, s, true);
        const bool rpost = top && prof_on(FMG_PROF_VPOST3D_F64);
        launch_vpost3d<T>(g, lo.g[l - 1], xs, xs == x ? y : x, x, f, xc, nu_post, s, prof_ev(rpost, 0),
                          prof_ev(rpost, 1));
        if (rpost) prof_add((3.0 * nf + ncs) * sizeof(double), nf);
        return;
    }
    if (lo.dim == 3 && g_fused && !lo.cg && vtile3d_applies(g, nu_pre, nu_post)) {
        // levels below the z-pipelined passes: the 2 nu + 1 half sweeps of a side in LDS
        // tiles, out of place (V(2,2): 3 + 2, x -> y -> x; V(1,1): 3, x -> y, then y -> x)
        T* y = at<T>(ws, lo.tv[l]);
        T* xs = nu_pre == 2 ? x : y;
        launch_vtile3d<T>(g, x, y, f, 3, 0, zero_x ? 1 : 0, s);
        if (nu_pre == 2) launch_vtile3d<T>(g, y, x, f, 2, 1, 0, s);
        launch_resid_restrict<T>(g, lo.g[l - 1], xs, f, fc, s);
        vcycle<T>(lo, ws, l - 1, xc, fc, nu_pre, nu_post, s, true);
        launch_prolong<T>(lo.g[l - 1], g, xc, xs, 1, s);
        if (nu_post == 2) {
            launch_vtile3d<T>(g, x, y, f, 3, 0, 0, s);
            launch_vtile3d<T>(g, y, x, f, 2, 1, 0, s);
        } else {
            launch_vtile3d<T>(g, y, x, f, 3, 0, 0, s);
        }
        return;
    }
    // unfused: red-black SGS (nu sweeps = 2 nu + 1 half sweeps) or nu CG steps
    auto smooth = [&](int nu) {
        if (nu <= 0) return;
        if (lo.cg) {
            double* part = at<double>(ws, lo.cgsc);
            launch_cg_smooth<T>(g, x, f, nu, at<T>(ws, lo.cgr), at<T>(ws, lo.cgp), at<T>(ws, lo.cgq), part,
                                part + kReduceBlocks, s);
        } else {
            launch_smooth<T>(g, x, f, 2 * nu + 1, 0, s);
        }
    };
    if (zero_x) launch_fill<T>(x, g.elems, T(0), s);
    smooth(nu_pre);
    launch_resid_restrict<T>(g, lo.g[l - 1], x, f, fc, s);
    launch_fill<T>(xc, lo.g[l - 1].elems, T(0), s);
    vcycle<T>(lo, ws, l - 1, xc, fc, nu_pre, nu_post, s);
    launch_prolong<T>(lo.g[l - 1], g, xc, x, 1, s);
    smooth(nu_post);
}

// one correction step (Algorithm 3.1) on level k
static int correction_step(const Layout& lo, void* ws, const fmg_problem* prob, const fmg_options* opt, int k,
                           int final_flag, int certify, hipStream_t s) {
    const Grid& g = lo.g[k];
    const Phys ph = make_phys(prob);
    SmallState* st = at<SmallState>(ws, lo.state);
    double* u = at<double>(ws, lo.u[k]);
    double* b = at<double>(ws, lo.b[k]);
    const bool fin3 = lo.dim == 3 && k == lo.L - 1;
    // (3.4): right-hand side lambda u - f(x, u) in the weak form
    const bool rr = fin3 && prof_on(FMG_PROF_RHS3D);
    launch_rhs(g, ph, u, b, &st->lambda, 0.0, s, prof_ev(rr, 0), prof_ev(rr, 1));
    if (rr) prof_add(2.0 * interior_nodes(g) * sizeof(double), interior_nodes(g));
    // (3.5): m multigrid iterations started from u
    for (int j = 0; j < opt->m; ++j) {
        if (opt->precision == FMG_MIXED) {
            float* r = at<float>(ws, lo.fv[k]);
            float* e = at<float>(ws, lo.xv[k]);
            launch_residual_demote(g, u, b, r, s);
            vcycle<float>(lo, ws, k, e, r, opt->nu_pre, opt->nu_post, s, true);
            launch_add_promote(g, u, e, s);
        } else {
            vcycle<double>(lo, ws, k, u, b, opt->nu_pre, opt->nu_post, s);
        }
    }
    // (3.6): augmented nonlinear eigenproblem on V_H + span{u~}
    double* mom = at<double>(ws, lo.mom);
    const bool rm = fin3 && prof_on(FMG_PROF_MOMENTS3D);
    launch_moments(lo.dim, lo.nc, g, ph, u, at<double>(ws, lo.momscr), mom, s, prof_ev(rm, 0), prof_ev(rm, 1));
    if (rm) prof_add(interior_nodes(g) * sizeof(double), std::pow((double)g.n, 3.0));
    int rc = launch_aug_newton(lo.dim, lo.nc, ph, opt->newton_max_iter, opt->newton_fixed_iters, opt->newton_tol, mom,
                               at<double>(ws, lo.arena),
                               at<double>(ws, lo.fac), at<double>(ws, lo.xc), st, final_flag, certify, 1, s);
    if (rc) return set_error(rc, "augmented solve launch failed");
    launch_form_u(g, lo.g[0], u, at<double>(ws, lo.xc), &st->c, s);
    return 0;
}

// ---- whole solve as a resumable schedule --------------------------------------------------
int64_t compact_len(const fmg_problem* p) {
    const int64_t n = (int64_t)p->n_coarse << p->n_refine;
    return p->dim == 2 ? (n - 1) * (n - 1) : (n - 1) * (n - 1) * (n - 1);
}

static bool tol_mode(const SolveJob& j) { return j.opt.tol_lambda > 0.0 && j.lo.L > 1; }

// Each chunk is a body (kernels and the copies of the device state into the host mirror:
// what a captured graph of the chunk holds), then the outputs of the final chunk and the
// chunk's event, which depend on the call.

// device state (and the Rayleigh-quotient forms after the final chunk) into the host mirror
static int copy_state(SolveJob& j, bool final_chunk) {
    SmallState* st = at<SmallState>(j.ws, j.lo.state);
    // a tolerance check needs only the scalars in front of the lambda history
    const size_t bytes = final_chunk ? sizeof(SmallState) : offsetof(SmallState, hist);
    FMG_HIP_CHECK(hipMemcpyAsync(&j.host->st, st, bytes, hipMemcpyDeviceToHost, j.s));
    if (final_chunk)
        FMG_HIP_CHECK(hipMemcpyAsync(j.host->forms, at<double>(j.ws, j.lo.forms), sizeof(j.host->forms),
                                     hipMemcpyDeviceToHost, j.s));
    return 0;
}

// Rayleigh quotient and residual of the finest u
static int body_final(SolveJob& j) {
    const Layout& lo = j.lo;
    const Grid& gf = lo.g[lo.L - 1];
    double* forms = at<double>(j.ws, lo.forms);
    const double* u = at<double>(j.ws, lo.u[lo.L - 1]);
    launch_forms(gf, make_phys(&j.prob), u, forms + 8, forms, j.s, &at<SmallState>(j.ws, lo.state)->lambda);
    return copy_state(j, true);
}

// state initialisation, Algorithm 3.2 step 1 and every level's p correction steps (and,
// without a lambda tolerance, the final body)
static int body_first(SolveJob& j) {
    const Layout& lo = j.lo;
    const fmg_problem* prob = &j.prob;
    const fmg_options* opt = &j.opt;
    hipStream_t s = j.s;
    void* ws = j.ws;
    const Phys ph = make_phys(prob);
    const int L = lo.L;
    // initial state and zeroed level arrays (the Dirichlet rings must be zero)
    SmallState* st = at<SmallState>(ws, lo.state);
    launch_init_state(st, opt->tol_lambda, s);
    launch_fill<double>(at<double>(ws, lo.xc), (int64_t)((lo.mom - lo.xc) / sizeof(double)), 0.0, s);
    // Algorithm 3.2 step 1
    int rc = launch_coarse_newton(prob->dim, prob->n_coarse, ph, opt->newton_max_iter, opt->newton_tol,
                                  at<double>(ws, lo.arena), at<double>(ws, lo.fac), at<double>(ws, lo.xc), st, s);
    if (rc) return set_error(rc, "coarse solve launch failed");
    // Algorithm 3.2 step 2
    for (int k = 1; k < L; ++k) {
        launch_prolong<double>(lo.g[k - 1], lo.g[k], at<double>(ws, lo.u[k - 1]), at<double>(ws, lo.u[k]), 0, s);
        const bool finest = (k == L - 1);
        const bool tm = finest && tol_mode(j);
        for (int step = 0; step < opt->p; ++step) {
            int flag = tm && step >= std::max(1, opt->p - 1);
            // ground-state check of the returned state only: the last step of a fixed
            // schedule, or the step that meets the lambda tolerance
            int cert = !finest ? 0 : (tm ? (flag ? 2 : 0) : (step == opt->p - 1 ? 1 : 0));
            if ((rc = correction_step(lo, ws, prob, opt, k, flag, cert, s))) return rc;
        }
    }
    return tol_mode(j) ? copy_state(j, false) : body_final(j);
}

// one more finest-level correction step (Algorithm 3.1)
static int body_step(SolveJob& j) {
    if (int rc = correction_step(j.lo, j.ws, &j.prob, &j.opt, j.lo.L - 1, 1, 2, j.s)) return rc;
    return copy_state(j, false);
}

static int run_body(SolveJob& j, int which) {
    if (j.gx[which]) {
        FMG_HIP_CHECK(hipGraphLaunch(j.gx[which], j.s));
        return 0;
    }
    return which == 0 ? body_first(j) : (which == 1 ? body_step(j) : body_final(j));
}

// the outputs of the final chunk: u into the caller's device or host target
static int outputs(SolveJob& j) {
    const Layout& lo = j.lo;
    const Grid& gf = lo.g[lo.L - 1];
    const double* u = at<double>(j.ws, lo.u[lo.L - 1]);
    if (j.u_out) launch_unpack(gf, u, j.u_out, j.s);
    if (j.u_host) {
        // host target: compact copy in the finest right-hand-side array (not needed any
        // more), then one device-to-host copy
        double* stage = at<double>(j.ws, lo.b[lo.L - 1]);
        launch_unpack(gf, u, stage, j.s);
        FMG_HIP_CHECK(hipMemcpyAsync(j.u_host, stage, sizeof(double) * compact_len(&j.prob), hipMemcpyDeviceToHost,
                                     j.s));
    }
    return 0;
}

static int end_chunk(SolveJob& j) {
    if (j.ev) FMG_HIP_CHECK(hipEventRecord(j.ev, j.s));
    return 0;
}

int job_start(SolveJob& j) {
    j.phase = 0;
    j.extra = 0;
    std::memset(&j.host->st, 0, sizeof(SmallState));
    j.host->st.tol_lambda = j.opt.tol_lambda;
    if (int rc = run_body(j, 0)) return rc;
    if (tol_mode(j)) {
        j.phase = 1;
    } else {
        if (int rc = outputs(j)) return rc;
        j.phase = 2;
    }
    return end_chunk(j);
}

int job_step(SolveJob& j) {
    if (j.phase == 1) {
        const SmallState& h = j.host->st;
        if (h.done || h.status != 0 || j.extra >= j.opt.max_final_steps) {
            if (int rc = run_body(j, 2)) return rc;
            if (int rc = outputs(j)) return rc;
            j.phase = 2;
            return end_chunk(j);
        }
        if (int rc = run_body(j, 1)) return rc;
        ++j.extra;
        return end_chunk(j);
    }
    if (j.phase == 2) j.phase = 3;
    return 0;
}

int job_capture(SolveJob& j, hipStream_t cs) {
    job_release(j);
    const hipStream_t saved = j.s;
    j.s = cs;
    int rc = 0;
    for (int w = 0; w < 3 && !rc; ++w) {
        if (w > 0 && !tol_mode(j)) break;   // without a tolerance the first body is the whole solve
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
            rc = set_error(FMG_EHIP, "hipStreamBeginCapture failed");
            break;
        }
        rc = w == 0 ? body_first(j) : (w == 1 ? body_step(j) : body_final(j));
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (!rc && (e != hipSuccess || !g)) rc = set_error(FMG_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        if (!rc && hipGraphInstantiate(&j.gx[w], g, nullptr, nullptr, 0) != hipSuccess) {
            j.gx[w] = nullptr;
            rc = set_error(FMG_EHIP, "hipGraphInstantiate failed");
        }
        if (g) (void)hipGraphDestroy(g);
    }
    (void)hipGetLastError();
    j.s = saved;
    if (rc) job_release(j);
    return rc;
}

void job_release(SolveJob& j) {
    for (auto& g : j.gx) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

int job_result(const SolveJob& j, fmg_result* out) {
    const SmallState& h = j.host->st;
    const double* f4 = j.host->forms;
    out->lambda = h.lambda;
    out->norm = f4[2];
    out->lambda_rq = (f4[0] + f4[1] + j.prob.zeta * f4[3]) / f4[2];
    out->residual = f4[5] > 0.0 ? std::sqrt(f4[4] / f4[5]) : 0.0;
    out->dlambda = h.dlambda;
    // contraction of the finest-level correction steps (Theorem 3.1): the ratio of the last
    // two eigenvalue changes; the finest level starts from the previous level's eigenvalue
    {
        const int nh = std::min(h.hist_len, FMG_HISTORY_MAX);
        const int fine = j.lo.L > 1 ? h.steps - (j.lo.L - 2) * j.opt.p : 0;   // steps on the finest level
        out->gamma_est = -1.0;
        if (fine >= 3 && nh >= 3 && nh == h.hist_len) {
            const double d1 = std::fabs(h.hist[nh - 1] - h.hist[nh - 2]), d0 = std::fabs(h.hist[nh - 2] - h.hist[nh - 3]);
            if (d0 > 0.0) out->gamma_est = d1 / d0;
        }
    }
    out->levels = j.lo.L;
    out->steps_total = h.steps;
    out->newton_total = h.newton_total;
    out->factor_total = h.fact_total;
    out->history_len = std::min(h.hist_len, FMG_HISTORY_MAX);
    for (int i = 0; i < out->history_len; ++i) out->history[i] = h.hist[i];
    int status = h.status;
    if (!status && !std::isfinite(h.lambda)) status = FMG_ENONFINITE;
    if (!status && h.certify_fail) status = FMG_ENOCONV;
    if (!status && j.opt.tol_lambda > 0.0 && !h.done) status = FMG_ENOCONV;
    out->status = status;
    if (status) {
        static const char* why[] = {"", "zero pivot", "Newton did not converge", "non-finite value",
                                    "singular border system", "not the ground state"};
        if (h.fail_reason)
            return set_error(status, "status %d: %s in the nonlinear solve after history entry %d (residual %.3e)",
                             status, why[h.fail_reason > 5 ? 0 : h.fail_reason], h.fail_step, h.fail_residual);
        return set_error(status, "status %d: tolerance %.3e not reached in %d final steps (last dlambda %.3e)",
                         status, j.opt.tol_lambda, j.opt.max_final_steps, h.dlambda);
    }
    return 0;
}

// fmg_solve inside a given workspace.  pinned_mirror: keep a pinned host mirror of the
// device state per calling thread (allocated once with hipHostMalloc); otherwise the
// chunk-end copies go to a pageable mirror on the stack and nothing is allocated.
static int solve_in(const fmg_problem* prob, const fmg_options* opt, void* ws, size_t ws_bytes, void* stream,
                    double* u_out, int64_t u_len, fmg_result* out, bool pinned_mirror) {
    auto t0 = std::chrono::steady_clock::now();
    if (int rc = check_problem(prob)) return rc;
    if (int rc = check_options(opt)) return rc;
    if (!out) return set_error(FMG_EINVAL, "result is NULL");
    std::memset(out, 0, sizeof(*out));
    if (u_len != compact_len(prob))
        return set_error(FMG_EINVAL, "u_len %lld != (n-1)^dim = %lld", (long long)u_len, (long long)compact_len(prob));
    if (!ws || !u_out) return set_error(FMG_EINVAL, "workspace and u_out must not be NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return set_error(FMG_EINVAL, "workspace must be 256-byte aligned");
    SolveJob j;
    j.prob = *prob;
    j.opt = *opt;
    j.lo = layout_for(prob, opt);
    if (ws_bytes < j.lo.total) return set_error(FMG_ENOMEM, "workspace %zu < required %zu bytes", ws_bytes, j.lo.total);
    // host mirror in pinned memory (one per calling thread, kept for the process): the
    // chunk-end copies are then direct DMA instead of staged pageable copies
    static thread_local JobHost* pinned = nullptr;
    if (pinned_mirror && !pinned &&
        hipHostMalloc(reinterpret_cast<void**>(&pinned), sizeof(JobHost), hipHostMallocDefault) != hipSuccess) {
        pinned = nullptr;
        (void)hipGetLastError();
    }
    JobHost local;
    j.ws = ws;
    j.s = static_cast<hipStream_t>(stream);
    if (is_device_pointer(u_out))
        j.u_out = u_out;
    else
        j.u_host = u_out;
    j.host = (pinned_mirror && pinned) ? pinned : &local;
    // each chunk ends with the device state copied into `host`; wait for it, then continue
    int rc = job_start(j);
    while (!rc && j.phase != 3) {
        FMG_HIP_CHECK(hipStreamSynchronize(j.s));
        rc = job_step(j);
    }
    if (rc) return rc;
    FMG_HIP_CHECK(hipGetLastError());
    const int status = job_result(j, out);
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

// Workspace of fmg_solve_static: a file-scope device array, one copy per GPU the library
// runs on, held until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in for the symbol); it uses the device
// address that hipGetSymbolAddress returns, looked up once per device with that device
// current.
constexpr size_t kStaticWorkspaceBytes = FMG_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

static std::mutex g_static_mu;
static void* g_static_ptr[kMaxDevices] = {};

static int static_workspace(void** out) {
    int dev = 0;
    FMG_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(FMG_EINVAL, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(FMG_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return 0;
}

}  // namespace fmg

using namespace fmg;

extern "C" {

const char* fmg_last_error(void) { return g_err; }

int fmg_set_fused_vcycle(int32_t enable) {
    g_fused = enable ? 1 : 0;
    return 0;
}
int fmg_get_tuning(fmg_tuning* out) {
    if (!out) return set_error(FMG_EINVAL, "tuning is NULL");
    std::memset(out, 0, sizeof(*out));
    int v = 0, mn = 0, w2 = 0, b2 = 0, one = 0;
    get_vpass3d_tuning(&v, &mn, &one);
    get_vpass2d_tuning(&w2, &b2);
    out->vpass3d_variant = v;
    out->vpass3d_min_n = mn;
    out->vpass3d_one_pass = one;
    out->vpass2d_wide_min_n = w2;
    out->vbottom2d_max_n = b2;
    out->vtile3d = get_vtile3d_tuning() ? 1 : -1;
    return 0;
}

int fmg_set_tuning(const fmg_tuning* in) {
    if (!in) return set_error(FMG_EINVAL, "tuning is NULL");
    if (in->vpass3d_variant < 0 || in->vpass3d_variant > 3)
        return set_error(FMG_EINVAL, "vpass3d_variant must be 0, 1, 2 or 3");
    if (in->vpass3d_min_n < 16) return set_error(FMG_EINVAL, "vpass3d_min_n must be >= 16");
    if (in->vpass2d_wide_min_n != 0 && in->vpass2d_wide_min_n < 16)
        return set_error(FMG_EINVAL, "vpass2d_wide_min_n must be 0 or >= 16");
    if (in->vbottom2d_max_n < -1 || in->vbottom2d_max_n > 64)
        return set_error(FMG_EINVAL, "vbottom2d_max_n must be in [-1, 64]");
    if (in->vpass3d_one_pass != 0 && in->vpass3d_one_pass != 1)
        return set_error(FMG_EINVAL, "vpass3d_one_pass must be 0 or 1");
    if (in->vtile3d < -1 || in->vtile3d > 1) return set_error(FMG_EINVAL, "vtile3d must be -1, 0 or 1");
    set_vpass3d_tuning(in->vpass3d_variant, in->vpass3d_min_n, in->vpass3d_one_pass);
    set_vpass2d_tuning(in->vpass2d_wide_min_n, in->vbottom2d_max_n);
    set_vtile3d_tuning(in->vtile3d >= 0 ? 1 : 0);
    return 0;
}

int fmg_autotune_vcycle(int32_t dim, int32_t n, int32_t precision, void* stream, fmg_tuning* out) {
    if (!out) return set_error(FMG_EINVAL, "tuning is NULL");
    if (dim != 2 && dim != 3) return set_error(FMG_EINVAL, "dim must be 2 or 3");
    if (precision != FMG_FP64 && precision != FMG_MIXED) return set_error(FMG_EINVAL, "precision invalid");
    fmg_tuning cur;
    fmg_get_tuning(&cur);
    *out = cur;
    const int nc_max = dim == 2 ? 31 : 7;
    int nc = n, levels = 1;
    while (nc > nc_max && nc % 2 == 0) {
        nc /= 2;
        ++levels;
    }
    if (dim == 3 && (n < 16 || n > 1024 || nc < 2 || levels < 2))
        return set_error(FMG_EINVAL, "3D n must be n_c 2^k with 2 <= n_c <= 7 and 16 <= n <= 1024 (got %d)", n);
    if (dim == 2 && (n < 64 || n > 32768 || nc < 8 || levels < 2))
        return set_error(FMG_EINVAL, "2D n must be n_c 2^k with 8 <= n_c <= 31 and 64 <= n <= 32768 (got %d)", n);
    const Layout lo = make_layout(dim, nc, levels, precision == FMG_MIXED, 0);
    void* ws = nullptr;
    if (hipMalloc(&ws, lo.total) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FMG_ENOMEM, "hipMalloc of %zu bytes failed", lo.total);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = set_error(FMG_EHIP, "events");
    const int top = levels - 1, reps = dim == 2 ? 10 : 5;
    // every array zero (the Dirichlet rings), then the top right-hand side one
    if (!rc) launch_fill<double>(static_cast<double*>(ws), (int64_t)(lo.total / sizeof(double)), 0.0, s);
    auto time_cycles = [&](auto zero) -> float {
        using T = decltype(zero);
        T* x = sizeof(T) == 8 ? at<T>(ws, lo.u[top]) : at<T>(ws, lo.xv[top]);
        T* f = sizeof(T) == 8 ? at<T>(ws, lo.b[top]) : at<T>(ws, lo.fv[top]);
        launch_fill<T>(f, lo.g[top].elems, T(1), s);
        vcycle<T>(lo, ws, top, x, f, 2, 2, s);   // first launches of this choice
        float ms = -1.f;
        if (hipEventRecord(e0, s) != hipSuccess) return ms;
        for (int r = 0; r < reps; ++r) vcycle<T>(lo, ws, top, x, f, 2, 2, s);
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            ms = -1.f;
        return ms;
    };
    float best = -1.f;
    auto consider = [&](int a, int b, int c, int tl) {
        if (dim == 3) {
            set_vpass3d_tuning(a, b, c);
            set_vtile3d_tuning(tl > 0 ? 1 : 0);
        } else {
            set_vpass2d_tuning(a, b);
        }
        const float ms = precision == FMG_MIXED ? time_cycles(0.0f) : time_cycles(0.0);
        if (ms < 0.f) {
            rc = set_error(FMG_EHIP, "timing failed");
            return;
        }
        if (best < 0.f || ms < best) {
            best = ms;
            if (dim == 3) {
                out->vpass3d_variant = a;
                out->vpass3d_min_n = b;
                out->vpass3d_one_pass = c;
                out->vtile3d = tl;
            } else {
                out->vpass2d_wide_min_n = a;
                out->vbottom2d_max_n = b;
            }
        }
    };
    if (dim == 3) {
        for (int mn = 16; !rc && mn <= 2 * n; mn *= 2)
            // mn > n: no level on the fused passes (the variant and pass split do not matter);
            // the LDS tiles apply to the levels between the bottom (16) and mn
            for (int v = 0; v < 4 && !rc; ++v)
                for (int one = 0; one < 2 && !rc; ++one)
                    for (int tl : {1, -1})
                        if (!rc && (mn <= n || (v == cur.vpass3d_variant && one == cur.vpass3d_one_pass)) &&
                            (mn > 32 || tl == cur.vtile3d))
                            consider(v, mn, one, tl);
    } else {
        for (int wm = 64; !rc && wm <= n; wm *= 2)   // wm = n: no level on the wide tiles
            for (int bm : {-1, 16, 32, 64})
                if (!rc) consider(wm, bm, 0, 0);
    }
    set_vtile3d_tuning(cur.vtile3d >= 0 ? 1 : 0);
    set_vpass3d_tuning(cur.vpass3d_variant, cur.vpass3d_min_n, cur.vpass3d_one_pass);
    set_vpass2d_tuning(cur.vpass2d_wide_min_n, cur.vbottom2d_max_n);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = set_error(FMG_EHIP, "autotune failed");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(ws);
    if (rc) *out = cur;
    return rc;
}

int fmg_profile_begin(int32_t kernel, int32_t max_launches) {
    if (kernel < FMG_PROF_VPOST2D_F64 || kernel > FMG_PROF_RHS3D || max_launches < 1 || max_launches > (1 << 20))
        return set_error(FMG_EINVAL, "bad profile request");
    if (g_prof.kernel) return set_error(FMG_EINVAL, "a profile is already running");
    g_prof.ev.resize(2 * (size_t)max_launches);
    // timing-only events: no system-scope fence (cache writeback) when they are stamped
    for (auto& e : g_prof.ev) FMG_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    g_prof.cap = max_launches;
    g_prof.used = 0;
    g_prof.bytes = 0.0;
    g_prof.units = 0.0;
    g_prof.kernel = kernel;
    return 0;
}

int fmg_profile_end(fmg_kernel_profile* out) {
    if (!g_prof.kernel) return set_error(FMG_EINVAL, "no profile is running");
    g_prof.kernel = 0;
    double ms_total = 0.0;
    int rc = 0;
    // the events carry no fence, so wait for the device rather than for the last event
    if (hipDeviceSynchronize() != hipSuccess) rc = FMG_EHIP;
    for (int i = 0; i < g_prof.used && !rc; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) != hipSuccess) rc = FMG_EHIP;
        ms_total += ms;
    }
    for (auto& e : g_prof.ev) (void)hipEventDestroy(e);
    g_prof.ev.clear();
    if (rc) return set_error(rc, "profile events failed");
    if (out) {
        out->launches = g_prof.used;
        out->seconds = ms_total * 1e-3;
        out->bytes = g_prof.bytes;
        out->units = g_prof.units;
    }
    return 0;
}

const char* fmg_version(void) { return "fmgeig 0.1 (gfx950)"; }

int64_t fmg_level_pitch(int32_t dim, int32_t n) {
    if ((dim != 2 && dim != 3) || n < 1) return -1;
    return make_grid(dim, n).pitch;
}
int64_t fmg_level_elems(int32_t dim, int32_t n) {
    if ((dim != 2 && dim != 3) || n < 1) return -1;
    return make_grid(dim, n).elems;
}

int fmg_workspace_bytes(const fmg_problem* prob, const fmg_options* opt, size_t* bytes) {
    if (int rc = check_problem(prob)) return rc;
    if (int rc = check_options(opt)) return rc;
    if (!bytes) return set_error(FMG_EINVAL, "bytes is NULL");
    Layout lo = layout_for(prob, opt);
    *bytes = lo.total;
    return 0;
}

int fmg_solve(const fmg_problem* prob, const fmg_options* opt, void* ws, size_t ws_bytes, void* stream, double* u_out,
              int64_t u_len, fmg_result* out) {
    return solve_in(prob, opt, ws, ws_bytes, stream, u_out, u_len, out, true);
}

int fmg_solve_static(const fmg_problem* prob, const fmg_options* opt, void* stream, double* u_out, int64_t u_len,
                     fmg_result* out) {
    if (int rc = check_problem(prob)) return rc;
    if (int rc = check_options(opt)) return rc;
    const size_t need = layout_for(prob, opt).total;
    if (need > kStaticWorkspaceBytes)
        return set_error(FMG_ENOMEM, "fmg_solve_static: this problem needs %zu bytes of workspace, more than the "
                                     "%zu bytes of the library's static workspace; use fmg_solve",
                         need, kStaticWorkspaceBytes);
    void* ws = nullptr;
    if (int rc = static_workspace(&ws)) return rc;
    return solve_in(prob, opt, ws, kStaticWorkspaceBytes, stream, u_out, u_len, out, false);
}

// ---- single steps ----------------------------------------------------------------------
int fmg_pack(int32_t dim, int32_t n, const double* c, double* lv, void* stream) {
    if ((dim != 2 && dim != 3) || n < 2 || !c || !lv) return set_error(FMG_EINVAL, "bad pack arguments");
    launch_pack(make_grid(dim, n), c, lv, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "pack launch failed");
}
int fmg_unpack(int32_t dim, int32_t n, const double* lv, double* c, void* stream) {
    if ((dim != 2 && dim != 3) || n < 2 || !c || !lv) return set_error(FMG_EINVAL, "bad unpack arguments");
    launch_unpack(make_grid(dim, n), lv, c, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "unpack launch failed");
}

int fmg_op_rhs(const fmg_problem* prob, int32_t n, double lambda, const double* u, double* b, void* stream) {
    if (int rc = check_problem(prob)) return rc;
    if (n < 2 || !u || !b) return set_error(FMG_EINVAL, "bad rhs arguments");
    launch_rhs(problem_grid(prob, n), make_phys(prob), u, b, nullptr, lambda, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "rhs launch failed");
}

int fmg_op_smooth(int32_t dim, int32_t n, int32_t precision, void* x, const void* f, int32_t sweeps, void* stream) {
    if ((dim != 2 && dim != 3) || n < 2 || sweeps < 0 || !x || !f) return set_error(FMG_EINVAL, "bad smooth arguments");
    Grid g = make_grid(dim, n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int hs = sweeps > 0 ? 2 * sweeps + 1 : 0;
    if (precision == FMG_MIXED)
        launch_smooth<float>(g, static_cast<float*>(x), static_cast<const float*>(f), hs, 0, s);
    else
        launch_smooth<double>(g, static_cast<double*>(x), static_cast<const double*>(f), hs, 0, s);
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "smooth launch failed");
}

int fmg_op_cg_smooth(int32_t dim, int32_t n, int32_t precision, void* x, const void* f, int32_t steps, void* scratch,
                     size_t scratch_bytes, void* stream) {
    if ((dim != 2 && dim != 3) || n < 2 || steps < 0 || !x || !f || !scratch)
        return set_error(FMG_EINVAL, "bad CG smoothing arguments");
    if (reinterpret_cast<uintptr_t>(scratch) % 256) return set_error(FMG_EINVAL, "scratch must be 256-byte aligned");
    Grid g = make_grid(dim, n);
    const size_t ts = precision == FMG_MIXED ? sizeof(float) : sizeof(double);
    const size_t e = align256(ts * g.elems);
    if (scratch_bytes < 3 * e + sizeof(double) * (kReduceBlocks + 8))
        return set_error(FMG_ENOMEM, "scratch %zu < %zu bytes", scratch_bytes, 3 * e + sizeof(double) * (kReduceBlocks + 8));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* b = static_cast<char*>(scratch);
    double* part = reinterpret_cast<double*>(b + 3 * e);
    if (precision == FMG_MIXED)
        launch_cg_smooth<float>(g, static_cast<float*>(x), static_cast<const float*>(f), steps, reinterpret_cast<float*>(b),
                                reinterpret_cast<float*>(b + e), reinterpret_cast<float*>(b + 2 * e), part,
                                part + kReduceBlocks, s);
    else
        launch_cg_smooth<double>(g, static_cast<double*>(x), static_cast<const double*>(f), steps,
                                 reinterpret_cast<double*>(b), reinterpret_cast<double*>(b + e),
                                 reinterpret_cast<double*>(b + 2 * e), part, part + kReduceBlocks, s);
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "CG smoothing launch failed");
}

int fmg_op_residual_restrict(int32_t dim, int32_t n, int32_t precision, const void* x, const void* f, void* rc,
                             void* stream) {
    if ((dim != 2 && dim != 3) || n < 4 || (n & 1) || !x || !f || !rc) return set_error(FMG_EINVAL, "bad restrict arguments");
    Grid gf = make_grid(dim, n), gc = make_grid(dim, n / 2);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == FMG_MIXED)
        launch_resid_restrict<float>(gf, gc, static_cast<const float*>(x), static_cast<const float*>(f),
                                     static_cast<float*>(rc), s);
    else
        launch_resid_restrict<double>(gf, gc, static_cast<const double*>(x), static_cast<const double*>(f),
                                      static_cast<double*>(rc), s);
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "restrict launch failed");
}

int fmg_op_prolong(int32_t dim, int32_t n, int32_t precision, const void* xc, void* xf, int32_t accumulate,
                   void* stream) {
    if ((dim != 2 && dim != 3) || n < 4 || (n & 1) || !xc || !xf) return set_error(FMG_EINVAL, "bad prolong arguments");
    Grid gf = make_grid(dim, n), gc = make_grid(dim, n / 2);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == FMG_MIXED)
        launch_prolong<float>(gc, gf, static_cast<const float*>(xc), static_cast<float*>(xf), accumulate, s);
    else
        launch_prolong<double>(gc, gf, static_cast<const double*>(xc), static_cast<double*>(xf), accumulate, s);
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "prolong launch failed");
}

int fmg_op_coarse_solve(int32_t dim, int32_t n, int32_t precision, const void* f, void* x, void* stream) {
    if ((dim != 2 && dim != 3) || n < 2 || (dim == 2 && n > 32) || (dim == 3 && n > 16) || !f || !x)
        return set_error(FMG_EINVAL, "bad coarse solve arguments");
    Grid g = make_grid(dim, n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == FMG_MIXED)
        launch_coarse_solve<float>(g, static_cast<const float*>(f), static_cast<float*>(x), s);
    else
        launch_coarse_solve<double>(g, static_cast<const double*>(f), static_cast<double*>(x), s);
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "coarse solve launch failed");
}

int fmg_op_vcycle(int32_t dim, int32_t n_coarse, int32_t levels, int32_t nu_pre, int32_t nu_post, double* x,
                  const double* f, void* ws, size_t ws_bytes, void* stream) {
    fmg_problem p{};
    p.dim = dim; p.n_coarse = n_coarse; p.n_refine = levels - 1;
    if (int rc = check_problem(&p)) return rc;
    if (nu_pre < 0 || nu_post < 0 || !x || !f || !ws) return set_error(FMG_EINVAL, "bad vcycle arguments");
    Layout lo = make_layout(dim, n_coarse, levels, 0, 0);
    if (ws_bytes < lo.total) return set_error(FMG_ENOMEM, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int l = 0; l < levels; ++l) {
        if (l + 1 < levels) {
            launch_fill<double>(at<double>(ws, lo.xv[l]), lo.g[l].elems, 0.0, s);
            launch_fill<double>(at<double>(ws, lo.fv[l]), lo.g[l].elems, 0.0, s);
        }
        if (lo.tv[l]) launch_fill<double>(at<double>(ws, lo.tv[l]), lo.g[l].elems, 0.0, s);
    }
    vcycle<double>(lo, ws, levels - 1, x, f, nu_pre, nu_post, s);
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "vcycle launch failed");
}

int fmg_moments_layout(int32_t dim, int32_t n_coarse, int32_t n, int32_t* per_element, size_t* scratch_bytes) {
    if ((dim != 2 && dim != 3) || n_coarse < 2 || n < n_coarse || n % n_coarse) return set_error(FMG_EINVAL, "bad layout args");
    if (per_element) *per_element = moments_per_element(dim);
    if (scratch_bytes) *scratch_bytes = std::max<size_t>(moments_scratch_bytes(dim, n_coarse, n), 256);
    return 0;
}

int fmg_op_moments_chunked(const fmg_problem* prob, int32_t n, const double* ut, double* out, void* scratch,
                           size_t scratch_bytes, int32_t chunk_cells, void* stream) {
    if (int rc = check_problem(prob)) return rc;
    const int nc = prob->n_coarse;
    if (n < nc || n % nc || ((n / nc) & (n / nc - 1)) || !ut || !out || !scratch)
        return set_error(FMG_EINVAL, "bad moments arguments");
    if (chunk_cells < 0 || chunk_cells > (1 << 20)) return set_error(FMG_EINVAL, "chunk_cells must be in [0, 2^20]");
    if (scratch_bytes < moments_scratch_bytes(prob->dim, nc, n, chunk_cells))
        return set_error(FMG_ENOMEM, "moments scratch too small");
    launch_moments(prob->dim, nc, problem_grid(prob, n), make_phys(prob), ut, static_cast<double*>(scratch), out,
                   static_cast<hipStream_t>(stream), nullptr, nullptr, chunk_cells);
    return hipGetLastError() == hipSuccess ? 0 : set_error(FMG_EHIP, "moments launch failed");
}

int fmg_op_moments(const fmg_problem* prob, int32_t n, const double* ut, double* out, void* scratch,
                   size_t scratch_bytes, void* stream) {
    return fmg_op_moments_chunked(prob, n, ut, out, scratch, scratch_bytes, 0, stream);
}

static size_t small_scratch(int dim, int nc) {
    return align256(sizeof(SmallState)) + align256(small_arena_bytes(dim, nc)) + small_factor_bytes(dim, nc);
}

int fmg_small_scratch_bytes(int32_t dim, int32_t n_coarse, size_t* bytes) {
    if ((dim != 2 && dim != 3) || n_coarse < 2 || !bytes) return set_error(FMG_EINVAL, "bad arguments");
    *bytes = small_scratch(dim, n_coarse);
    return 0;
}

int fmg_op_augmented_matrices(const fmg_problem* prob, const double* mom, const double* x, double* A, double* B,
                              double* S, void* scratch, size_t scratch_bytes, void* stream) {
    if (int rc = check_problem(prob)) return rc;
    if (!mom || !x || !A || !B || !S || !scratch) return set_error(FMG_EINVAL, "bad arguments");
    if (scratch_bytes < small_scratch(prob->dim, prob->n_coarse)) return set_error(FMG_ENOMEM, "scratch too small");
    double* arena = at<double>(scratch, align256(sizeof(SmallState)));
    int rc = launch_aug_dump(prob->dim, prob->n_coarse, make_phys(prob), mom, x, arena, A, B, S,
                             static_cast<hipStream_t>(stream));
    return rc ? set_error(rc, "augmented dump launch failed") : 0;
}

static int small_common(const fmg_problem* prob, const fmg_options* opt, double* xc, void* scratch, size_t bytes,
                        hipStream_t s, bool aug, const double* mom, double* lambda, double* c, int32_t* iters,
                        int32_t* ground) {
    if (int rc = check_problem(prob)) return rc;
    if (int rc = check_options(opt)) return rc;
    if (!xc || !scratch || (aug && !mom)) return set_error(FMG_EINVAL, "bad arguments");
    if (bytes < small_scratch(prob->dim, prob->n_coarse)) return set_error(FMG_ENOMEM, "scratch too small");
    SmallState init;
    std::memset(&init, 0, sizeof(init));
    SmallState* st = at<SmallState>(scratch, 0);
    double* arena = at<double>(scratch, align256(sizeof(SmallState)));
    double* fac = at<double>(scratch, align256(sizeof(SmallState)) + align256(small_arena_bytes(prob->dim, prob->n_coarse)));
    FMG_HIP_CHECK(hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, s));
    int rc = aug ? launch_aug_newton(prob->dim, prob->n_coarse, make_phys(prob), opt->newton_max_iter,
                                     opt->newton_fixed_iters, opt->newton_tol,
                                     mom, arena, fac, xc, st, 0, 1, 0, s)
                 : launch_coarse_newton(prob->dim, prob->n_coarse, make_phys(prob), opt->newton_max_iter,
                                        opt->newton_tol, arena, fac, xc, st, s);
    if (rc) return set_error(rc, "small solve launch failed");
    SmallState h;
    FMG_HIP_CHECK(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
    FMG_HIP_CHECK(hipStreamSynchronize(s));
    if (lambda) *lambda = h.lambda;
    if (c) *c = h.c;
    if (iters) *iters = h.newton_total;
    if (ground) *ground = h.certify_fail == 0;
    if (h.status)
        return set_error(h.status, "nonlinear solve failed (reason %d, residual %.3e)", h.fail_reason, h.fail_residual);
    return 0;
}

int fmg_op_augmented_solve(const fmg_problem* prob, const fmg_options* opt, const double* mom, double* xc,
                           void* scratch, size_t bytes, void* stream, double* lambda, double* c, int32_t* iters,
                           int32_t* ground) {
    return small_common(prob, opt, xc, scratch, bytes, static_cast<hipStream_t>(stream), true, mom, lambda, c, iters,
                        ground);
}

int fmg_op_coarse_nonlinear(const fmg_problem* prob, const fmg_options* opt, double* xc, void* scratch, size_t bytes,
                            void* stream, double* lambda, int32_t* iters, int32_t* ground) {
    return small_common(prob, opt, xc, scratch, bytes, static_cast<hipStream_t>(stream), false, nullptr, lambda,
                        nullptr, iters, ground);
}

int fmg_op_form_u(int32_t dim, int32_t n_coarse, int32_t n, double c, const double* xc, double* u, void* scratch,
                  void* stream) {
    if ((dim != 2 && dim != 3) || n_coarse < 2 || n < n_coarse || n % n_coarse || !xc || !u || !scratch)
        return set_error(FMG_EINVAL, "bad form_u arguments");
    if ((n / n_coarse) & (n / n_coarse - 1))
        return set_error(FMG_EINVAL, "form_u: n / n_coarse = %d is not a power of two", n / n_coarse);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* cd = static_cast<double*>(scratch);
    FMG_HIP_CHECK(hipMemcpyAsync(cd, &c, sizeof(double), hipMemcpyHostToDevice, s));
    launch_form_u(make_grid(dim, n), make_grid(dim, n_coarse), u, xc, cd, s);
    FMG_HIP_CHECK(hipStreamSynchronize(s));
    return 0;
}

int fmg_op_forms(const fmg_problem* prob, int32_t n, const double* u, double* out4, void* scratch, void* stream) {
    if (int rc = check_problem(prob)) return rc;
    if (n < 2 || !u || !out4 || !scratch) return set_error(FMG_EINVAL, "bad forms arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* f = static_cast<double*>(scratch);
    launch_forms(problem_grid(prob, n), make_phys(prob), u, f + 8, f, s);
    FMG_HIP_CHECK(hipMemcpyAsync(out4, f, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    FMG_HIP_CHECK(hipStreamSynchronize(s));
    return 0;
}

}  // extern "C"
