// Continuous-batching (T) server (bqc_server_* / bqc_t_submit / bqc_t_poll).
//
// Each request is one independent (T) solve of an embedding fragment (the
// fragments of the paper's embedding layer are independent problems).  The
// server owns:
//   * one device arena of mem_budget_bytes, allocated once at creation and
//     carved first-fit per request (inputs + workspace), so the serving loop
//     never calls hipMalloc/hipFree;
//   * max_inflight slot threads, each with its own HIP stream.  An idle slot
//     admits the oldest queued request whose footprint fits into the arena
//     (a request may be overtaken by smaller ones at most kMaxBypass times,
//     after which admission waits for it), uploads it, enqueues its whole
//     solve on its stream and waits for it, so that admitted requests run
//     concurrently on the device while new ones keep arriving.  By default
//     the request's triple-batch launch sequence is built as one hipGraph
//     (kernel nodes with the pipeline's dependencies, no stream capture) and
//     launched as a unit.
// A request's launch sequence is the one bqc_t_energy_ex uses, so its result
// is bitwise identical alone and in the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bqc.h"
#include "bqc_internal.h"

namespace bqc {

int fail(int code, const std::string& msg);
int validate(int32_t nocc, int32_t nvir, const double* eps_o, const double* eps_v, const double* t1,
             const double* t2, const double* ovvv, const double* ooov, const double* ovov,
             bool host_eps);

namespace {

using clk = std::chrono::steady_clock;
constexpr int kMaxBypass = 32;
inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
  public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t n, size_t* off) {
        n = a256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = a256(n);
        auto it = free_.emplace(off, n).first;
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
    std::map<size_t, size_t> free_;
};

enum class St { Queued, Running, Done };

struct Request {
    uint64_t ticket = 0;
    int o = 0, v = 0;
    const double* src[7] = {};
    St state = St::Queued;
    int rc = BQC_PENDING;
    std::string err;
    double energy = 0.0;
    bqc_t_stats stats{};
    clk::time_point t_submit, t_admit;
    size_t bytes = 0, off = 0;
    size_t held = 0;  // bytes of the arena range this request holds from `off` (a group's range: its first member)
    int bypassed = 0;
    bool dev_in = false;  // inputs are device pointers read in place
    int fault_stage = 0, fault_code = 0;  // injected failure (host-side tests)
};

// Stages at which a host-side test can make one request fail.
constexpr int FAULT_AT_ADMISSION = 1;  // right after its memory is carved out, before any upload
constexpr int FAULT_AFTER_SOLVE = 2;   // after its kernels have run, before its result is read

}  // namespace
}  // namespace bqc

struct bqc_server {
    int device = 0, precision = 0, max_inflight = 4;
    bool graphs = true;  // run each request's launch sequence as one hipGraph
    bool group = true;   // admit queued small requests together and run them as one batch
    uint64_t budget = 0;
    void* arena_base = nullptr;
    bqc::Arena* arena = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<bqc::Request*> queue;
    std::unordered_map<uint64_t, bqc::Request*> reqs;
    std::vector<std::thread> slots;
    std::vector<hipStream_t> streams;
    std::vector<hipStream_t> sides;  // epilogue stream of each slot
    std::vector<double*> pinned;
    bool stop = false;
    int callers = 0;                 // threads inside submit/poll/wait (destroy waits for them)
    std::map<uint64_t, std::pair<int, int>> faults;  // host-side tests: ticket -> (stage, code)
    bool hold = false;               // host-side tests: admit nothing until released (or stopping)
    std::condition_variable cv_idle;
    uint64_t next_ticket = 1;
    hipStream_t check_stream = nullptr;  // reads device orbital energies at submit
    std::mutex check_mu;
};

namespace bqc {
namespace {

size_t request_bytes(int o, int v, int precision, bool dev_in) {
    return (dev_in ? 0 : a256((size_t)input_bytes(o, v))) + a256((size_t)workspace_bytes(o, v, precision));
}

// Runs one admitted request on the slot's stream; returns the BQC code.
int run_request(bqc_server* s, Request* r, hipStream_t st, hipStream_t side, double* pinned) {
    const int o = r->o, v = r->v;
    char* base = (char*)s->arena_base + r->off;
    const size_t sizes[7] = {(size_t)o, (size_t)v, (size_t)o * v, (size_t)o * o * v * v,
                             (size_t)o * v * v * v, (size_t)o * o * o * v, (size_t)o * v * o * v};
    const double* dst[7];
    double upload_s = 0.0;
    void* ws = base;
    if (r->dev_in) {
        for (int a = 0; a < 7; ++a) dst[a] = r->src[a];
    } else {
        char* p = base;
        const auto u0 = clk::now();
        for (int a = 0; a < 7; ++a) {
            BQC_HIP(hipMemcpyAsync(p, r->src[a], sizes[a] * sizeof(double), hipMemcpyHostToDevice, st));
            dst[a] = (const double*)p;
            p += a256(sizes[a] * sizeof(double));
        }
        BQC_HIP(hipStreamSynchronize(st));
        upload_s = std::chrono::duration<double>(clk::now() - u0).count();
        ws = base + a256((size_t)input_bytes(o, v));
    }
    DevInputs in;
    in.o = o; in.v = v;
    in.eps_o = dst[0]; in.eps_v = dst[1]; in.t1 = dst[2]; in.t2 = dst[3];
    in.ovvv = dst[4]; in.ooov = dst[5]; in.ovov = dst[6];
    const Plan plan = make_plan(o, v, s->precision);
    SolveStats ss;
    enqueue_solve(plan, in, ws, nullptr, st, side, false, &ss, s->graphs);
    if (r->fault_stage == FAULT_AFTER_SOLVE) throw Error(r->fault_code, "injected failure after the solve");
    BQC_HIP(hipMemcpyAsync(pinned, workspace_energy(ws, o, v, s->precision), sizeof(double),
                           hipMemcpyDeviceToHost, st));
    BQC_HIP(hipStreamSynchronize(st));
    if (!std::isfinite(*pinned)) throw Error(BQC_EDEVICE, "non-finite energy");
    r->energy = *pinned;
    r->stats.upload_s = upload_s;
    r->stats.prepare_s = ss.prepare_s;
    r->stats.gpu_s = ss.gpu_s;
    r->stats.footprint_bytes = r->bytes;
    r->stats.flops = 12.0 * (double)num_triples(o) * (double)v * v * v * (double)(v + o);
    r->stats.precision = s->precision;
    r->stats.n_triples = (int32_t)num_triples(o);
    return BQC_OK;
}

// Small requests may be admitted together and run as one batch (grouped
// launches, batch.hip): requests of at most kGroupFlops algorithmic flops
// (a few milliseconds of contraction, where launch overhead is a large
// share), at most kGroupMax of them.  Each result is bitwise the one the
// request has alone.
constexpr double kGroupFlops = 5e11;
constexpr int kGroupMax = 32;

// Device bytes a group needs: the host-input members' inputs and the batch
// workspace.
size_t group_bytes(bqc_server* s, const std::vector<Request*>& g) {
    std::vector<int> o, v;
    size_t in = 0;
    for (Request* r : g) {
        o.push_back(r->o);
        v.push_back(r->v);
        if (!r->dev_in) in += a256((size_t)input_bytes(r->o, r->v));
    }
    return in + a256(plan_batch((int)g.size(), o.data(), v.data(), s->precision).total);
}

// Runs an admitted group of requests as one batch on the slot's stream.
void run_group(bqc_server* s, const std::vector<Request*>& g, hipStream_t st) {
    const int n = (int)g.size();
    char* p = (char*)s->arena_base + g[0]->off;
    std::vector<DevInputs> ins(n);
    std::vector<int> o(n), v(n);
    const auto u0 = clk::now();
    bool uploaded = false;
    for (int f = 0; f < n; ++f) {
        Request* r = g[f];
        o[f] = r->o;
        v[f] = r->v;
        const double* dst[7];
        if (r->dev_in) {
            for (int a = 0; a < 7; ++a) dst[a] = r->src[a];
        } else {
            const size_t sizes[7] = {(size_t)r->o, (size_t)r->v, (size_t)r->o * r->v, (size_t)r->o * r->o * r->v * r->v,
                                     (size_t)r->o * r->v * r->v * r->v, (size_t)r->o * r->o * r->o * r->v,
                                     (size_t)r->o * r->v * r->o * r->v};
            char* q = p;
            for (int a = 0; a < 7; ++a) {
                BQC_HIP(hipMemcpyAsync(q, r->src[a], sizes[a] * sizeof(double), hipMemcpyHostToDevice, st));
                dst[a] = (const double*)q;
                q += a256(sizes[a] * sizeof(double));
            }
            p += a256((size_t)input_bytes(r->o, r->v));
            uploaded = true;
        }
        DevInputs& in = ins[f];
        in.o = r->o; in.v = r->v;
        in.eps_o = dst[0]; in.eps_v = dst[1]; in.t1 = dst[2]; in.t2 = dst[3];
        in.ovvv = dst[4]; in.ooov = dst[5]; in.ovov = dst[6];
    }
    if (uploaded) BQC_HIP(hipStreamSynchronize(st));
    const double upload_s = std::chrono::duration<double>(clk::now() - u0).count();
    const BatchPlan bp = plan_batch(n, o.data(), v.data(), s->precision);
    std::vector<double> e(n);
    SolveStats ss;
    enqueue_batch(bp, s->precision, n, ins.data(), p, st, e.data(), &ss);
    for (int f = 0; f < n; ++f) {
        Request* r = g[f];
        if (!std::isfinite(e[f])) throw Error(BQC_EDEVICE, "non-finite energy");
        r->energy = e[f];
        r->stats.upload_s = upload_s;
        r->stats.gpu_s = ss.gpu_s;
        r->stats.footprint_bytes = g[0]->held;
        r->stats.flops = 12.0 * (double)num_triples(r->o) * (double)r->v * r->v * r->v * (double)(r->v + r->o);
        r->stats.precision = s->precision;
        r->stats.n_triples = (int32_t)num_triples(r->o);
        r->stats.gemm_launches = ss.gemm_launches;
        r->stats.epilogue_launches = ss.epi_launches;
    }
}

// Picks the request to admit (caller holds s->mu); nullptr if none fits.
Request* admit_locked(bqc_server* s) {
    for (size_t q = 0; q < s->queue.size(); ++q) {
        Request* r = s->queue[q];
        size_t off = 0;
        if (s->arena->alloc(r->bytes, &off)) {
            r->off = off;
            r->held = r->bytes;
            auto f = s->faults.find(r->ticket);
            if (f != s->faults.end()) {
                r->fault_stage = f->second.first;
                r->fault_code = f->second.second;
                s->faults.erase(f);
            }
            for (size_t b = 0; b < q; ++b) s->queue[b]->bypassed++;
            s->queue.erase(s->queue.begin() + q);
            return r;
        }
        if (r->bypassed >= kMaxBypass) return nullptr;  // no overtaking a starved request
    }
    return nullptr;
}

// The request to admit and, if it is small, the queued small requests that
// join it (caller holds s->mu).  The group holds one arena range (its first
// member's `off` / `held`); empty if nothing fits.
std::vector<Request*> admit_group_locked(bqc_server* s) {
    Request* r = admit_locked(s);
    if (!r) return {};
    auto small = [&](Request* q) {
        const double fl = 12.0 * (double)num_triples(q->o) * (double)q->v * q->v * q->v * (double)(q->v + q->o);
        return fl <= kGroupFlops && q->fault_stage == 0 && s->faults.find(q->ticket) == s->faults.end();
    };
    if (!s->group || !small(r)) return {r};
    std::vector<Request*> cand{r};
    for (Request* q : s->queue) {
        if ((int)cand.size() >= kGroupMax) break;
        if (small(q)) cand.push_back(q);
        else if (q->bypassed >= kMaxBypass) break;  // take no memory a starved request waits for
    }
    if (cand.size() == 1) return {r};
    // the largest prefix of the candidates whose batch fits the arena
    s->arena->release(r->off, r->held);
    for (size_t k = cand.size(); k >= 2; --k) {
        std::vector<Request*> g(cand.begin(), cand.begin() + k);
        const size_t bytes = group_bytes(s, g);
        size_t off = 0;
        if (s->arena->alloc(bytes, &off)) {
            for (size_t m = 1; m < k; ++m) {
                auto it = std::find(s->queue.begin(), s->queue.end(), g[m]);
                s->queue.erase(it);
                g[m]->off = 0;
                g[m]->held = 0;
            }
            r->off = off;
            r->held = bytes;
            return g;
        }
    }
    size_t off = 0;  // alone after all (the range it held is free again)
    if (!s->arena->alloc(r->bytes, &off)) throw Error(BQC_ENOMEM, "arena state changed during admission");
    r->off = off;
    r->held = r->bytes;
    return {r};
}

void slot_main(bqc_server* s, int idx) {
    (void)hipSetDevice(s->device);
    hipStream_t st = s->streams[idx];
    hipStream_t side = s->sides[idx];
    double* pinned = s->pinned[idx];
    for (;;) {
        std::vector<Request*> grp;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stop && s->queue.empty()) return;
                if (!s->hold || s->stop) grp = admit_group_locked(s);
                if (!grp.empty()) break;
                s->cv_work.wait(lk);
            }
            const auto now = clk::now();
            for (Request* q : grp) {
                q->state = St::Running;
                q->t_admit = now;
            }
        }
        Request* r = grp[0];
        int rc;
        std::string err;
        try {
            if (r->fault_stage == FAULT_AT_ADMISSION) throw Error(r->fault_code, "injected failure at admission");
            if (grp.size() > 1) {
                run_group(s, grp, st);
                rc = BQC_OK;
            } else {
                rc = run_request(s, r, st, side, pinned);
            }
        } catch (const Error& e) {
            rc = e.code;
            err = e.what();
        } catch (const std::bad_alloc&) {
            rc = BQC_ENOMEM;
            err = "host allocation failed";
        } catch (const std::exception& e) {
            rc = BQC_EDEVICE;
            err = e.what();
        }
        // a failed request may still have work in flight on either stream:
        // its memory goes back to the arena only once both have drained
        if (rc != BQC_OK) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamSynchronize(side);
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->arena->release(r->off, r->held);
            const auto now = clk::now();
            for (Request* q : grp) {  // a group shares its outcome
                q->stats.queue_s = std::chrono::duration<double>(q->t_admit - q->t_submit).count();
                q->stats.total_s = std::chrono::duration<double>(now - q->t_submit).count();
                q->rc = rc;
                q->err = err;
                q->state = St::Done;
            }
        }
        s->cv_work.notify_all();  // freed memory may admit queued requests
        s->cv_done.notify_all();
    }
}

int create_impl(const bqc_server_cfg* cfg, bqc_server** out) {
    if (!cfg || !out) return fail(BQC_EINVAL, "null argument");
    if (cfg->precision < 0 || cfg->precision > 3) return fail(BQC_EINVAL, "unknown precision");
    if (cfg->max_inflight < 0 || cfg->max_inflight > 64) return fail(BQC_EINVAL, "max_inflight out of range");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BQC_EDEVICE, "no HIP device");
    if (cfg->device < 0 || cfg->device >= ndev) return fail(BQC_EINVAL, "device ordinal out of range");
    int prev = 0;
    BQC_HIP(hipGetDevice(&prev));
    BQC_HIP(hipSetDevice(cfg->device));
    auto* s = new bqc_server();
    s->device = cfg->device;
    s->precision = cfg->precision;
    s->max_inflight = cfg->max_inflight > 0 ? cfg->max_inflight : 4;
    s->graphs = cfg->direct_launch == 0;
    s->group = cfg->no_grouping == 0;
    try {
        size_t fr = 0, tot = 0;
        BQC_HIP(hipMemGetInfo(&fr, &tot));
        s->budget = cfg->mem_budget_bytes ? cfg->mem_budget_bytes : (uint64_t)(0.85 * (double)fr);
        s->budget &= ~(uint64_t)255;
        BQC_HIP(hipMalloc(&s->arena_base, s->budget));
        BQC_HIP(hipStreamCreateWithFlags(&s->check_stream, hipStreamNonBlocking));
        s->arena = new Arena(s->budget);
        for (int k = 0; k < s->max_inflight; ++k) {
            hipStream_t st;
            BQC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            s->streams.push_back(st);
            hipStream_t sd;
            BQC_HIP(hipStreamCreateWithFlags(&sd, hipStreamNonBlocking));
            s->sides.push_back(sd);
            double* p = nullptr;
            BQC_HIP(hipHostMalloc((void**)&p, 256, hipHostMallocDefault));
            s->pinned.push_back(p);
        }
    } catch (...) {
        (void)hipSetDevice(prev);
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        for (hipStream_t st : s->sides) (void)hipStreamDestroy(st);
        if (s->check_stream) (void)hipStreamDestroy(s->check_stream);
        for (double* p : s->pinned) (void)hipHostFree(p);
        if (s->arena_base) (void)hipFree(s->arena_base);
        delete s->arena;
        delete s;
        throw;
    }
    for (int k = 0; k < s->max_inflight; ++k) s->slots.emplace_back(slot_main, s, k);
    (void)hipSetDevice(prev);
    *out = s;
    return BQC_OK;
}

}  // namespace

// Threads inside submit/poll/wait of the server (host-side tests use it to
// destroy a server while waiters are known to be blocked).
int server_callers(bqc_server* s) {
    std::lock_guard<std::mutex> lk(s->mu);
    return s->callers;
}

// Host-side tests: the request with this ticket (submitted already or in
// the future; tickets count up from 1) fails with `code` at `stage`
// (FAULT_AT_ADMISSION or FAULT_AFTER_SOLVE) instead of completing.
void server_inject_fault(bqc_server* s, uint64_t ticket, int stage, int code) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->faults[ticket] = {stage, code};
}

// Host-side tests: while `on`, the slots admit no request (submitted ones
// stay queued, so that a cancel meets them there); off lets them run.
void server_hold_admission(bqc_server* s, bool on) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->hold = on;
    if (!on) s->cv_work.notify_all();
}

namespace {

int destroy_impl(bqc_server* s) {
    if (!s) return fail(BQC_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Request* r : s->queue) {
            r->rc = BQC_ESHUTDOWN;
            r->state = St::Done;
        }
        s->queue.clear();
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& th : s->slots) th.join();
    {
        // every request is Done now: wake the waiters and let every thread
        // still inside an entry point of this server leave before freeing it
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.notify_all();
        s->cv_idle.wait(lk, [&] { return s->callers == 0; });
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    for (hipStream_t st : s->sides) (void)hipStreamDestroy(st);
    (void)hipStreamDestroy(s->check_stream);
    for (double* p : s->pinned) (void)hipHostFree(p);
    (void)hipFree(s->arena_base);
    (void)hipSetDevice(prev);
    for (auto& kv : s->reqs) delete kv.second;
    delete s->arena;
    delete s;
    return BQC_OK;
}

// Counts a thread inside an entry point of the server (destroy waits until
// none is left).  Constructed and destroyed without s->mu held.
struct Caller {
    bqc_server* s;
    explicit Caller(bqc_server* srv) : s(srv) {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->callers;
    }
    ~Caller() {
        std::lock_guard<std::mutex> lk(s->mu);
        if (--s->callers == 0) s->cv_idle.notify_all();
    }
};

int submit_impl(bqc_server* s, int32_t o, int32_t v, const double* const src[7], bool dev_in,
                uint64_t* ticket) {
    if (!s || !ticket) return fail(BQC_EINVAL, "null argument");
    Caller in_call(s);
    int rc = validate(o, v, src[0], src[1], src[2], src[3], src[4], src[5], src[6], !dev_in);
    if (rc != BQC_OK) return rc;
    if (dev_in) {  // orbital energies are checked from a host copy, read on the server's own stream
        std::vector<double> eo(o), ev(v);
        hipError_t err = hipSuccess;
        {
            std::lock_guard<std::mutex> lk(s->check_mu);
            int prev = 0;
            BQC_HIP(hipGetDevice(&prev));
            BQC_HIP(hipSetDevice(s->device));
            err = hipMemcpyAsync(eo.data(), src[0], o * sizeof(double), hipMemcpyDeviceToHost, s->check_stream);
            if (err == hipSuccess)
                err = hipMemcpyAsync(ev.data(), src[1], v * sizeof(double), hipMemcpyDeviceToHost, s->check_stream);
            if (err == hipSuccess) err = hipStreamSynchronize(s->check_stream);
            (void)hipSetDevice(prev);
        }
        if (err != hipSuccess)
            return fail(BQC_EINVAL, std::string("orbital energies are not readable device memory: ") +
                                        hipGetErrorString(err));
        rc = validate(o, v, eo.data(), ev.data(), src[2], src[3], src[4], src[5], src[6], true);
        if (rc != BQC_OK) return rc;
    }
    const size_t bytes = request_bytes(o, v, s->precision, dev_in);
    if (bytes > s->budget)
        return fail(BQC_ENOMEM, "request footprint " + std::to_string(bytes) + " B exceeds the budget " +
                                    std::to_string(s->budget) + " B");
    auto* r = new Request();
    r->o = o;
    r->v = v;
    r->dev_in = dev_in;
    for (int a = 0; a < 7; ++a) r->src[a] = src[a];
    r->bytes = bytes;
    r->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return fail(BQC_ESHUTDOWN, "server is shutting down");
        }
        r->ticket = s->next_ticket++;
        s->reqs[r->ticket] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_all();
    *ticket = r->ticket;
    return BQC_OK;
}

// Cancels a queued request: it leaves the queue, never runs, and its
// terminal status is BQC_ECANCELED.  A running request is not interrupted.
int cancel_impl(bqc_server* s, uint64_t ticket) {
    if (!s) return fail(BQC_EINVAL, "null server");
    Caller in_call(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(BQC_ENOTFOUND, "unknown or consumed ticket");
        Request* r = it->second;
        if (r->state == St::Running) return BQC_PENDING;
        if (r->state == St::Done) return BQC_OK;  // finished (or failed) already: the poll tells which
        auto q = std::find(s->queue.begin(), s->queue.end(), r);
        if (q != s->queue.end()) s->queue.erase(q);
        r->rc = BQC_ECANCELED;
        r->err = "request cancelled before admission";
        r->stats.queue_s = std::chrono::duration<double>(clk::now() - r->t_submit).count();
        r->state = St::Done;
    }
    s->cv_work.notify_all();  // the head of the queue may have changed
    s->cv_done.notify_all();
    return BQC_OK;
}

int poll_impl(bqc_server* s, uint64_t ticket, double* E_T, bqc_t_stats* stats, bool wait) {
    if (!s) return fail(BQC_EINVAL, "null server");
    Caller in_call(s);
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(BQC_ENOTFOUND, "unknown or consumed ticket");
    if (wait) {
        // the ticket is looked up again on every wake-up: another thread may
        // have consumed it (and freed its request) meanwhile
        s->cv_done.wait(lk, [&] {
            auto f = s->reqs.find(ticket);
            return f == s->reqs.end() || f->second->state == St::Done;
        });
        it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(BQC_ENOTFOUND, "ticket consumed by another thread");
    }
    Request* r = it->second;
    if (r->state != St::Done) return BQC_PENDING;
    const int rc = r->rc;
    if (rc == BQC_OK) {
        if (E_T) *E_T = r->energy;
        if (stats) *stats = r->stats;
    } else {
        fail(rc, r->err.empty() ? "request failed" : r->err);
    }
    s->reqs.erase(it);
    delete r;
    return rc;
}

template <typename F>
int guarded_srv(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(BQC_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(BQC_EDEVICE, e.what());
    } catch (...) {
        return fail(BQC_EDEVICE, "unknown failure");
    }
}

}  // namespace
}  // namespace bqc

using namespace bqc;

extern "C" {

int bqc_server_create(const bqc_server_cfg* cfg, bqc_server** out) {
    return guarded_srv([&] { return create_impl(cfg, out); });
}

int bqc_server_destroy(bqc_server* s) {
    return guarded_srv([&] { return destroy_impl(s); });
}

int bqc_t_submit(bqc_server* s, int32_t nocc, int32_t nvir, const double* eps_o, const double* eps_v,
                 const double* t1, const double* t2, const double* ovvv, const double* ooov,
                 const double* ovov, uint64_t* ticket) {
    const double* src[7] = {eps_o, eps_v, t1, t2, ovvv, ooov, ovov};
    return guarded_srv([&] { return submit_impl(s, nocc, nvir, src, false, ticket); });
}

int bqc_t_submit_ex(bqc_server* s, int32_t nocc, int32_t nvir, const double* eps_o, const double* eps_v,
                    const double* t1, const double* t2, const double* ovvv, const double* ooov,
                    const double* ovov, int32_t inputs_on_device, uint64_t* ticket) {
    const double* src[7] = {eps_o, eps_v, t1, t2, ovvv, ooov, ovov};
    return guarded_srv([&] { return submit_impl(s, nocc, nvir, src, inputs_on_device != 0, ticket); });
}

int bqc_t_poll(bqc_server* s, uint64_t ticket, double* E_T, bqc_t_stats* stats) {
    return guarded_srv([&] { return poll_impl(s, ticket, E_T, stats, false); });
}

int bqc_t_wait(bqc_server* s, uint64_t ticket, double* E_T, bqc_t_stats* stats) {
    return guarded_srv([&] { return poll_impl(s, ticket, E_T, stats, true); });
}

int bqc_t_cancel(bqc_server* s, uint64_t ticket) {
    return guarded_srv([&] { return cancel_impl(s, ticket); });
}

}  // extern "C"
