// Workspace layout of one solve and the solve itself (Algorithm 3.2 with the tolerance
// loop) as a resumable schedule: a sequence of chunks enqueued on one stream, each ending
// with the device state copied into a host mirror.  fmg_solve drives it synchronously; the
// batch and serving runtime drive many of them at once on several streams.
#pragma once

#include <vector>

#include "kernels.h"

namespace fmg {

int check_problem(const fmg_problem* p);
int check_options(const fmg_options* o);
int64_t compact_len(const fmg_problem* p);   // (n - 1)^dim on the finest level
bool is_device_pointer(const void* p);       // device (or managed) memory of the HIP runtime

// Byte offsets into the caller's workspace (each region 256-B aligned).
struct Layout {
    int dim, nc, L, mixed;
    std::vector<Grid> g;
    size_t state, xc, mom, momscr, arena, fac, forms;
    std::vector<size_t> u, b, xv, fv;   // per level (u[0] = xc)
    std::vector<size_t> tv;             // per level: target of the fused 2D pre pass
    int cg = 0;                         // CG smoothing: r, p, q arrays and reduction scratch
    size_t cgr = 0, cgp = 0, cgq = 0, cgsc = 0;
    size_t total;
};
Layout make_layout(int dim, int nc, int levels, int mixed, int cg);
Layout layout_for(const fmg_problem* p, const fmg_options* o);

// What the host reads back between chunks.
struct JobHost {
    SmallState st;
    double forms[6];   // u^T K u, u^T M_W u, u^T M u, int u^4 of the finest u; |r|^2, |lam M u|^2
};

struct SolveJob {
    fmg_problem prob{};
    fmg_options opt{};
    Layout lo;
    void* ws = nullptr;          // device workspace of at least lo.total bytes, 256-B aligned
    hipStream_t s = nullptr;
    double* u_out = nullptr;     // device, compact: the final chunk unpacks u into it when set
    double* u_host = nullptr;    // host, compact: the final chunk copies u into it when set
    JobHost* host = nullptr;     // pinned memory when the driver does not synchronise per chunk
    hipEvent_t ev = nullptr;     // when set, recorded at the end of every chunk
    int phase = 0;               // 1: tolerance check pending, 2: final chunk pending, 3: done
    int extra = 0;               // finest-level correction steps beyond p
    // captured chunk bodies (job_capture): first chunk, one more finest step, final chunk;
    // when set they are replayed instead of enqueued kernel by kernel
    hipGraphExec_t gx[3] = {nullptr, nullptr, nullptr};
};

// Enqueue the first chunk: state initialisation, the coarse solve and every level's p
// correction steps (and, without a lambda tolerance, the final chunk).
int job_start(SolveJob& j);
// Called once the last enqueued chunk has completed (its copies into `host` are done):
// enqueue the next chunk (one more finest-level step, or the final chunk) or mark the
// job done (phase 3).
int job_step(SolveJob& j);
// Fill *out from the host mirror of a finished job; returns its status (and sets the
// thread's error message when it is not 0).  seconds is left to the driver.
int job_result(const SolveJob& j, fmg_result* out);
// Capture the job's chunk bodies on stream cs (relaxed capture mode) into executable graphs
// that job_start / job_step then launch on the job's stream.  Needs ws and a pinned host
// mirror (the graphs copy into them); the outputs (u_out, u_host) and the chunk events stay
// outside the graphs.  Nothing runs during the capture.
int job_capture(SolveJob& j, hipStream_t cs);
void job_release(SolveJob& j);   // destroy the captured graphs

}  // namespace fmg
