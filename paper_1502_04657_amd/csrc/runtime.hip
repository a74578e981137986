// Batched and serving runtime: many independent eigensolves in flight on one GPU.
//
// Each solve is a resumable schedule (job.h) on a stream of its own; a scheduler pass
// admits queued solves while a stream slot and workspace memory are free, and advances
// every running solve whose last chunk has completed (a HIP event query, no blocking).
// Solves on different streams overlap on the device: the single-workgroup small solves of
// one instance run beside the bandwidth-bound V-cycles of others.
//
// Workspace memory comes from a pool: one device block (the HBM budget) carved first-fit
// into 256-B aligned regions, so admission by footprint is exact and no allocation happens
// while solves are running.  The pool block comes from the caller's allocator when one is
// registered (fmg_set_allocator), else from hipMalloc.
//
// fmg_batch_solve runs the scheduler in the calling thread until every solve of the batch
// is done.  A server runs it in a worker thread: submit queues a request (FIFO admission),
// poll returns FMG_PENDING until the request is done and then copies its u out and
// releases its workspace.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "job.h"

namespace fmg {

namespace {

// ---- device allocator hooks ----------------------------------------------------------------
struct Allocator {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*free)(void*, void*) = nullptr;
    void* ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

struct DeviceBlock {
    void* p = nullptr;
    Allocator a;   // the allocator that produced p (frees go back to it)
    int get(size_t bytes) {
        {
            std::lock_guard<std::mutex> lk(g_alloc_mu);
            a = g_alloc;
        }
        if (a.alloc) {
            p = a.alloc(bytes, a.ctx);
            if (!p) return set_error(FMG_ENOMEM, "caller allocator returned NULL for %zu bytes", bytes);
            if (reinterpret_cast<uintptr_t>(p) % 256)
                return set_error(FMG_EINVAL, "caller allocator returned a pointer that is not 256-B aligned");
            return 0;
        }
        if (hipMalloc(&p, bytes) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return set_error(FMG_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
        }
        return 0;
    }
    void put() {
        if (!p) return;
        if (a.free) a.free(p, a.ctx);
        else (void)hipFree(p);
        p = nullptr;
    }
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// First-fit sub-allocator over one device block.
class Pool {
  public:
    int init(size_t bytes) {
        size_ = align256(bytes);
        if (int rc = blk_.get(size_)) return rc;
        free_.clear();
        free_[0] = size_;
        return 0;
    }
    void destroy() { blk_.put(); }
    size_t size() const { return size_; }
    char* base() const { return static_cast<char*>(blk_.p); }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    DeviceBlock blk_;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
};

// One solve as the scheduler sees it.
struct Task {
    uint64_t ticket = 0;
    SolveJob job;
    size_t bytes = 0, off = 0;
    int slot = -1;
    enum { QUEUED, RUNNING, DONE } state = QUEUED;
    int rc = 0;                       // status of the solve (0 or FMG_E*)
    std::string msg;
    fmg_result res{};
    std::chrono::steady_clock::time_point t_submit, t_admit, t_done;
    bool keep_ws = false;             // server: workspace held until poll copies u out
};

// Streams, events and pinned host mirrors of the slots, and the scheduling pass.  Several
// host threads pump at once (kernel launches cost microseconds of host time each, so one
// thread enqueueing for many solves would limit the device): worker w of nw owns slots
// w, w + nw, ...; the queue, the pool, the finished list and the slot table are shared and
// guarded by one mutex, held only around their updates, never across HIP launches.
class Scheduler {
  public:
    int init(int slots, hipStream_t user) {
        user_ = user;
        slots_ = slots;
        str_.assign(slots, nullptr);
        ev_.assign(slots, nullptr);
        uev_.assign(slots, nullptr);
        busy_.assign(slots, nullptr);
        for (int i = 0; i < slots; ++i) {
            FMG_HIP_CHECK(hipStreamCreateWithFlags(&str_[i], hipStreamNonBlocking));
            FMG_HIP_CHECK(hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming));
            FMG_HIP_CHECK(hipEventCreateWithFlags(&uev_[i], hipEventDisableTiming));
        }
        FMG_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&host_), sizeof(JobHost) * slots, hipHostMallocDefault));
        return 0;
    }
    void destroy() {
        for (auto s : str_)
            if (s) (void)hipStreamDestroy(s);
        for (auto e : ev_)
            if (e) (void)hipEventDestroy(e);
        for (auto e : uev_)
            if (e) (void)hipEventDestroy(e);
        if (host_) (void)hipHostFree(host_);
        str_.clear();
        ev_.clear();
        uev_.clear();
        host_ = nullptr;
    }
    int slots() const { return slots_; }
    // with mu held
    bool idle(int w, int nw) const {
        for (int i = w; i < slots_; i += nw)
            if (busy_[i]) return false;
        return true;
    }
    // One pass over the slots of worker w: advance running tasks whose last chunk has
    // completed, then fill free slots from the queue (FIFO; the head blocks the queue until
    // its footprint fits the pool).  Returns the number of tasks that changed state;
    // finished tasks are appended to `done`.  Launch failures end the task with that status.
    int pump(int w, int nw, std::mutex& mu, std::deque<Task*>& queue, Pool& pool, std::vector<Task*>& done,
             bool admit = true) {
        int changes = 0;
        for (int i = w; i < slots_; i += nw) {
            Task* t = busy_[i];   // written only by this worker (under mu)
            if (t) {
                const hipError_t q = hipEventQuery(ev_[i]);
                if (q == hipErrorNotReady) continue;
                const int rc = (q == hipSuccess) ? job_step(t->job) : set_error(FMG_EHIP, "event query failed");
                if (!rc && t->job.phase != 3) continue;   // next chunk enqueued
                finish(i, rc, mu, pool, done);
                ++changes;
            }
            if (!admit) continue;
            Task* nt = nullptr;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (!queue.empty() && pool.alloc(queue.front()->bytes, &queue.front()->off)) {
                    nt = queue.front();
                    queue.pop_front();
                    nt->state = Task::RUNNING;
                    busy_[i] = nt;
                }
            }
            if (nt) {
                start(i, nt, mu, pool, done);
                ++changes;
            }
        }
        return changes;
    }

  private:
    void start(int i, Task* t, std::mutex& mu, Pool& pool, std::vector<Task*>& done) {
        t->slot = i;
        t->t_admit = std::chrono::steady_clock::now();
        SolveJob& j = t->job;
        j.ws = pool.base() + t->off;
        j.s = str_[i];
        j.ev = ev_[i];
        j.host = host_ + i;
        // work the caller enqueued on its stream before the admission comes first
        int rc = 0;
        if (hipEventRecord(uev_[i], user_) != hipSuccess || hipStreamWaitEvent(str_[i], uev_[i], 0) != hipSuccess)
            rc = set_error(FMG_EHIP, "ordering after the caller's stream failed");
        if (!rc) rc = job_start(j);
        if (rc) finish(i, rc, mu, pool, done);
    }
    void finish(int i, int rc, std::mutex& mu, Pool& pool, std::vector<Task*>& done) {
        Task* t = busy_[i];
        int status;
        std::string msg;
        if (rc) {
            // a launch failed: let what was enqueued drain before the memory is reused
            (void)hipStreamSynchronize(str_[i]);
            status = rc;
            msg = fmg_last_error();
            t->res.status = rc;
        } else {
            status = job_result(t->job, &t->res);
            if (status) msg = fmg_last_error();
        }
        std::lock_guard<std::mutex> lk(mu);
        t->rc = status;
        t->msg = msg;
        t->t_done = std::chrono::steady_clock::now();
        t->state = Task::DONE;
        t->job.host = nullptr;
        t->job.ev = nullptr;
        if (!t->keep_ws || rc) {
            pool.release(t->off, t->bytes);
            t->bytes = 0;
        }
        busy_[i] = nullptr;
        done.push_back(t);
    }

    hipStream_t user_ = nullptr;
    int slots_ = 0;
    std::vector<hipStream_t> str_;
    std::vector<hipEvent_t> ev_, uev_;
    std::vector<Task*> busy_;
    JobHost* host_ = nullptr;
};

// host threads that enqueue for a scheduler
constexpr int kHostThreads = 8;

int validate(const fmg_problem* p, const fmg_options* o, size_t* bytes) {
    if (int rc = check_problem(p)) return rc;
    if (int rc = check_options(o)) return rc;
    *bytes = layout_for(p, o).total;
    return 0;
}

constexpr int kMaxSlots = 64;     // streams of a server
constexpr int kBatchSlots = 8;    // streams of a batch call
constexpr int kPlanStreams = 16;  // streams of a batch plan
constexpr int kMaxPlanInstances = 4096;

}  // namespace

}  // namespace fmg

// ---- serving ------------------------------------------------------------------------------
struct fmg_server {
    fmg::Pool pool;
    fmg::Scheduler sched;
    hipStream_t user = nullptr;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<fmg::Task*> queue;
    std::map<uint64_t, std::unique_ptr<fmg::Task>> tasks;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;

    // worker w of nw: pumps its slots until the server stops and its slots are idle
    void run(int w, int nw) {
        (void)hipSetDevice(device);
        std::vector<fmg::Task*> done;
        for (;;) {
            bool stopping;
            {
                std::lock_guard<std::mutex> lk(mu);
                stopping = stop;
                if (stopping) {
                    queue.clear();   // not admitted yet: dropped with the server
                    if (sched.idle(w, nw)) break;
                }
            }
            const int changes = sched.pump(w, nw, mu, queue, pool, done, !stopping);
            done.clear();
            if (changes) {
                cv.notify_all();
            } else {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait_for(lk, std::chrono::microseconds(20));
            }
        }
        cv.notify_all();
    }
};

// ---- batch plans ---------------------------------------------------------------------------
struct fmg_batch_plan {
    fmg::Pool pool;
    std::vector<fmg::SolveJob> jobs;
    std::vector<hipStream_t> str;
    std::vector<hipEvent_t> ev;
    hipStream_t user = nullptr, cap = nullptr;
    hipEvent_t uev = nullptr;
    fmg::JobHost* host = nullptr;

    int init(int count) {
        jobs.resize(count);
        str.assign(std::min(count, fmg::kPlanStreams), nullptr);
        ev.assign(count, nullptr);
        for (auto& s : str) FMG_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        for (auto& e : ev) FMG_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        FMG_HIP_CHECK(hipEventCreateWithFlags(&uev, hipEventDisableTiming));
        FMG_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        FMG_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&host), sizeof(fmg::JobHost) * count,
                                    hipHostMallocDefault));
        return 0;
    }
    void destroy() {
        for (auto& s : str)
            if (s) (void)hipStreamSynchronize(s);
        for (auto& j : jobs) fmg::job_release(j);
        for (auto& s : str)
            if (s) (void)hipStreamDestroy(s);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (uev) (void)hipEventDestroy(uev);
        if (cap) (void)hipStreamDestroy(cap);
        if (host) (void)hipHostFree(host);
        str.clear();
        ev.clear();
        jobs.clear();
        uev = nullptr;
        cap = nullptr;
        host = nullptr;
        pool.destroy();
    }
};

using namespace fmg;

extern "C" {

int fmg_set_allocator(void* (*alloc)(size_t, void*), void (*free_fn)(void*, void*), void* ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return set_error(FMG_EINVAL, "alloc and free must both be set or both be NULL");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free = free_fn;
    g_alloc.ctx = ctx;
    return 0;
}

size_t fmg_footprint_bytes(const fmg_problem* prob, const fmg_options* opt) {
    size_t bytes = 0;
    if (validate(prob, opt, &bytes)) return 0;
    return align256(bytes);
}

int fmg_solve_alloc(const fmg_problem* prob, const fmg_options* opt, void* stream, double* u_out, int64_t u_len,
                    fmg_result* out) {
    size_t bytes = 0;
    if (int rc = validate(prob, opt, &bytes)) return rc;
    DeviceBlock blk;
    if (int rc = blk.get(align256(bytes))) return rc;
    const int rc = fmg_solve(prob, opt, blk.p, align256(bytes), stream, u_out, u_len, out);
    // fmg_solve has synchronised the stream, so the workspace is free to go
    blk.put();
    return rc;
}

int fmg_batch_solve(int32_t count, const fmg_problem* probs, const fmg_options* opts, void* stream,
                    double* const* u_out, const int64_t* u_len, fmg_result* out) {
    auto t0 = std::chrono::steady_clock::now();
    if (count < 0) return set_error(FMG_EINVAL, "count must be >= 0");
    if (count == 0) return 0;
    if (!probs || !opts || !u_out || !u_len || !out) return set_error(FMG_EINVAL, "NULL array argument");
    std::vector<std::unique_ptr<Task>> tasks(count);
    size_t total = 0;
    for (int i = 0; i < count; ++i) {
        auto t = std::make_unique<Task>();
        if (int rc = validate(&probs[i], &opts[i], &t->bytes))
            return set_error(rc, "instance %d: %s", i, std::string(fmg_last_error()).c_str());
        if (u_len[i] != compact_len(&probs[i]))
            return set_error(FMG_EINVAL, "instance %d: u_len %lld != (n-1)^dim = %lld", i, (long long)u_len[i],
                             (long long)compact_len(&probs[i]));
        if (!u_out[i]) return set_error(FMG_EINVAL, "instance %d: u_out is NULL", i);
        t->ticket = i;
        t->job.prob = probs[i];
        t->job.opt = opts[i];
        t->job.lo = layout_for(&probs[i], &opts[i]);
        t->job.u_out = u_out[i];
        total += align256(t->bytes);
        tasks[i] = std::move(t);
    }
    Pool pool;
    if (int rc = pool.init(total)) return rc;
    Scheduler sched;
    int rc = sched.init(std::min(count, kBatchSlots), static_cast<hipStream_t>(stream));
    if (rc) {
        sched.destroy();
        pool.destroy();
        return rc;
    }
    std::deque<Task*> queue;
    for (auto& t : tasks) {
        t->t_submit = t0;
        queue.push_back(t.get());
    }
    std::vector<Task*> done;
    std::mutex mu;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const int nw = std::min(sched.slots(), kHostThreads);
    auto work = [&](int w) {
        if (w) (void)hipSetDevice(dev);
        for (;;) {
            {
                std::lock_guard<std::mutex> lk(mu);
                if (done.size() == (size_t)count) return;
            }
            if (!sched.pump(w, nw, mu, queue, pool, done)) std::this_thread::sleep_for(std::chrono::microseconds(10));
        }
    };
    std::vector<std::thread> helpers;
    for (int w = 1; w < nw; ++w) helpers.emplace_back(work, w);
    work(0);
    for (auto& th : helpers) th.join();
    sched.destroy();
    pool.destroy();
    int first = 0;
    for (int i = 0; i < count; ++i) {
        Task& t = *tasks[i];
        out[i] = t.res;
        out[i].status = t.rc;
        out[i].seconds = std::chrono::duration<double>(t.t_done - t0).count();
        out[i].wait_seconds = std::chrono::duration<double>(t.t_admit - t0).count();
        if (t.rc && !first) {
            first = t.rc;
            set_error(t.rc, "instance %d: %s", i, t.msg.c_str());
        }
    }
    return first;
}

fmg_batch_plan* fmg_batch_plan_create(int32_t count, const fmg_problem* probs, const fmg_options* opts,
                                      void* stream) {
    if (count < 1 || count > kMaxPlanInstances) {
        set_error(FMG_EINVAL, "count must be in [1, %d]", kMaxPlanInstances);
        return nullptr;
    }
    if (!probs || !opts) {
        set_error(FMG_EINVAL, "NULL array argument");
        return nullptr;
    }
    auto plan = std::make_unique<fmg_batch_plan>();
    plan->user = static_cast<hipStream_t>(stream);
    std::vector<size_t> bytes(count), off(count);
    size_t total = 0;
    for (int i = 0; i < count; ++i) {
        if (int rc = validate(&probs[i], &opts[i], &bytes[i])) {
            set_error(rc, "instance %d: %s", i, std::string(fmg_last_error()).c_str());
            return nullptr;
        }
        off[i] = total;
        total += align256(bytes[i]);
    }
    if (plan->pool.init(total)) return nullptr;
    if (plan->init(count) != 0) {
        plan->destroy();
        return nullptr;
    }
    for (int i = 0; i < count; ++i) {
        SolveJob& j = plan->jobs[i];
        j.prob = probs[i];
        j.opt = opts[i];
        j.lo = layout_for(&probs[i], &opts[i]);
        j.ws = plan->pool.base() + off[i];
        j.host = plan->host + i;
        j.s = plan->str[i % plan->str.size()];
        j.ev = plan->ev[i];
        if (int rc = job_capture(j, plan->cap)) {
            set_error(rc, "instance %d: %s", i, std::string(fmg_last_error()).c_str());
            plan->destroy();
            return nullptr;
        }
    }
    return plan.release();
}

int fmg_batch_plan_run(fmg_batch_plan* plan, double* const* u_out, const int64_t* u_len, fmg_result* out) {
    auto t0 = std::chrono::steady_clock::now();
    if (!plan || !u_out || !u_len || !out) return set_error(FMG_EINVAL, "NULL argument");
    const int count = (int)plan->jobs.size();
    for (int i = 0; i < count; ++i) {
        if (u_len[i] != compact_len(&plan->jobs[i].prob))
            return set_error(FMG_EINVAL, "instance %d: u_len %lld != (n-1)^dim = %lld", i, (long long)u_len[i],
                             (long long)compact_len(&plan->jobs[i].prob));
        if (!u_out[i] || !is_device_pointer(u_out[i]))
            return set_error(FMG_EINVAL, "instance %d: u_out must be device memory", i);
    }
    // work the caller enqueued on its stream comes first
    FMG_HIP_CHECK(hipEventRecord(plan->uev, plan->user));
    for (hipStream_t st : plan->str) FMG_HIP_CHECK(hipStreamWaitEvent(st, plan->uev, 0));
    std::vector<int> rc(count, 0);
    std::vector<char> fin(count, 0);
    std::vector<std::chrono::steady_clock::time_point> t_done(count);
    int left = count;
    for (int i = 0; i < count; ++i) {
        SolveJob& j = plan->jobs[i];
        j.u_out = u_out[i];
        j.u_host = nullptr;
        if ((rc[i] = job_start(j))) {
            fin[i] = 1;
            --left;
            t_done[i] = std::chrono::steady_clock::now();
        }
    }
    while (left > 0) {
        bool moved = false;
        for (int i = 0; i < count; ++i) {
            if (fin[i]) continue;
            SolveJob& j = plan->jobs[i];
            const hipError_t q = hipEventQuery(j.ev);
            if (q == hipErrorNotReady) continue;
            moved = true;
            rc[i] = (q == hipSuccess) ? job_step(j) : set_error(FMG_EHIP, "event query failed");
            if (rc[i] || j.phase == 3) {
                fin[i] = 1;
                --left;
                t_done[i] = std::chrono::steady_clock::now();
            }
        }
        if (!moved) std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
    for (hipStream_t st : plan->str) FMG_HIP_CHECK(hipStreamSynchronize(st));
    int first = 0;
    for (int i = 0; i < count; ++i) {
        std::memset(&out[i], 0, sizeof(out[i]));
        int status = rc[i];
        if (!status) status = job_result(plan->jobs[i], &out[i]);
        out[i].status = status;
        out[i].seconds = std::chrono::duration<double>(t_done[i] - t0).count();
        out[i].wait_seconds = 0.0;
        if (status && !first) {
            first = status;
            set_error(status, "instance %d: %s", i, std::string(fmg_last_error()).c_str());
        }
    }
    return first;
}

void fmg_batch_plan_destroy(fmg_batch_plan* plan) {
    if (!plan) return;
    plan->destroy();
    delete plan;
}

fmg_server* fmg_server_create(size_t hbm_budget, int32_t max_slots, void* stream) {
    if (max_slots < 1 || max_slots > kMaxSlots) {
        set_error(FMG_EINVAL, "max_slots must be in [1, %d]", kMaxSlots);
        return nullptr;
    }
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            set_error(FMG_EHIP, "hipMemGetInfo failed");
            return nullptr;
        }
        hbm_budget = fr / 2;
    }
    auto* sv = new fmg_server();
    sv->user = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&sv->device) != hipSuccess) {
        set_error(FMG_EHIP, "hipGetDevice failed");
        delete sv;
        return nullptr;
    }
    if (sv->pool.init(hbm_budget) || sv->sched.init(max_slots, sv->user)) {
        const std::string m = fmg_last_error();
        sv->sched.destroy();
        sv->pool.destroy();
        delete sv;
        set_error(FMG_ENOMEM, "%s", m.c_str());
        return nullptr;
    }
    const int nw = std::min<int>(max_slots, kHostThreads);
    for (int w = 0; w < nw; ++w) sv->workers.emplace_back([sv, w, nw] { sv->run(w, nw); });
    return sv;
}

int fmg_server_submit(fmg_server* sv, const fmg_problem* prob, const fmg_options* opt, uint64_t* ticket) {
    if (!sv || !ticket) return set_error(FMG_EINVAL, "server and ticket must not be NULL");
    auto t = std::make_unique<Task>();
    if (int rc = validate(prob, opt, &t->bytes)) return rc;
    if (align256(t->bytes) > sv->pool.size())
        return set_error(FMG_ENOMEM, "footprint %zu bytes exceeds the server budget %zu", align256(t->bytes),
                         sv->pool.size());
    t->job.prob = *prob;
    t->job.opt = *opt;
    t->job.lo = layout_for(prob, opt);
    t->keep_ws = true;
    t->t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return set_error(FMG_EINVAL, "server is shutting down");
    t->ticket = sv->next_ticket++;
    *ticket = t->ticket;
    sv->queue.push_back(t.get());
    sv->tasks.emplace(t->ticket, std::move(t));
    sv->cv.notify_all();
    return 0;
}

int fmg_server_poll(fmg_server* sv, uint64_t ticket, fmg_result* out, double* u_out, int64_t u_len) {
    if (!sv) return set_error(FMG_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tasks.find(ticket);
    if (it == sv->tasks.end()) return set_error(FMG_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Task& t = *it->second;
    if (t.state != Task::DONE) return FMG_PENDING;
    if (u_out && u_len != compact_len(&t.job.prob)) {
        return set_error(FMG_EINVAL, "u_len %lld != (n-1)^dim = %lld", (long long)u_len,
                         (long long)compact_len(&t.job.prob));
    }
    int rc = t.rc;
    if (u_out && t.bytes) {
        // the solve's chunks have completed; copy u on the caller's stream, then release
        const Layout& lo = t.job.lo;
        launch_unpack(lo.g[lo.L - 1], reinterpret_cast<const double*>(sv->pool.base() + t.off + lo.u[lo.L - 1]), u_out,
                      sv->user);
        if (hipStreamSynchronize(sv->user) != hipSuccess) rc = set_error(FMG_EHIP, "copy of u failed");
    }
    if (out) {
        *out = t.res;
        out->status = t.rc;
        out->seconds = std::chrono::duration<double>(t.t_done - t.t_submit).count();
        out->wait_seconds = std::chrono::duration<double>(t.t_admit - t.t_submit).count();
    }
    if (t.bytes) sv->pool.release(t.off, t.bytes);
    const std::string msg = t.msg;
    const int solve_rc = t.rc;
    sv->tasks.erase(it);   // t is gone from here on
    sv->cv.notify_all();
    if (rc && rc == solve_rc && !msg.empty()) return set_error(rc, "%s", msg.c_str());
    return rc;
}

void fmg_server_destroy(fmg_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    for (auto& th : sv->workers)
        if (th.joinable()) th.join();
    sv->sched.destroy();
    sv->pool.destroy();
    delete sv;
}

}  // extern "C"
