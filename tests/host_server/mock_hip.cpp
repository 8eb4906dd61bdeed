// Test infrastructure (see mock_hip.h): the stand-in HIP runtime.
#include "mock_hip.h"

#include <sys/mman.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

using clk = std::chrono::steady_clock;

[[noreturn]] void die(const char* fmt, const char* what, const void* p, size_t n) {
    std::fprintf(stderr, "MOCK-HIP FAULT: ");
    std::fprintf(stderr, fmt, what, p, n);
    std::fprintf(stderr, "\n");
    std::fflush(stderr);
    std::abort();
}

// ------------------------------------------------------------------ device memory
struct Alloc {
    size_t size;
    bool live;
};
std::mutex g_mem_mu;
std::map<uintptr_t, Alloc> g_allocs;  // base -> allocation (dead ones kept to name use-after-free)
std::atomic<uint64_t> g_nalloc{0}, g_nfree{0}, g_nlaunch{0}, g_ngraph{0}, g_nnodes{0};
constexpr size_t kDevFree = (size_t)256 << 30;

bool is_device(const void* p) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_allocs.upper_bound((uintptr_t)p);
    if (it == g_allocs.begin()) return false;
    --it;
    return (uintptr_t)p < it->first + it->second.size;
}

// ------------------------------------------------------------------ streams
struct Task {
    std::function<void()> fn;
};

}  // namespace

struct ihipStream_t {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Task> q;
    uint64_t submitted = 0, completed = 0;
    bool stop = false;
    std::thread worker;
    void run() {
        for (;;) {
            Task t;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !q.empty(); });
                if (q.empty()) return;
                t = std::move(q.front());
                q.pop_front();
            }
            t.fn();
            {
                std::lock_guard<std::mutex> lk(mu);
                ++completed;
            }
            cv.notify_all();
        }
    }
    void push(std::function<void()> fn) {
        {
            std::lock_guard<std::mutex> lk(mu);
            q.push_back(Task{std::move(fn)});
            ++submitted;
        }
        cv.notify_all();
    }
    void sync() {
        std::unique_lock<std::mutex> lk(mu);
        const uint64_t target = submitted;
        cv.wait(lk, [&] { return completed >= target; });
    }
};

struct ihipEvent_t {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t recorded = 0, done = 0;
    clk::time_point t;
};

namespace {

// ------------------------------------------------------------------ kernels
struct KernelInfo {
    std::vector<size_t> sizes;
    std::function<void(void**)> emu;
};
std::mutex g_k_mu;
std::unordered_map<const void*, KernelInfo> g_kernels;

struct BoundCall {  // a launch with copies of its argument values
    const KernelInfo* k = nullptr;
    std::vector<std::vector<char>> args;
    void run() const {
        std::vector<void*> p(args.size());
        for (size_t a = 0; a < args.size(); ++a) p[a] = (void*)args[a].data();
        k->emu(p.data());
    }
};

BoundCall bind(const void* fn, void** args) {
    std::lock_guard<std::mutex> lk(g_k_mu);
    auto it = g_kernels.find(fn);
    if (it == g_kernels.end()) die("%s %p (%zu)", "launch of an unregistered kernel", fn, 0);
    BoundCall c;
    c.k = &it->second;
    for (size_t a = 0; a < it->second.sizes.size(); ++a) {
        std::vector<char> b(it->second.sizes[a]);
        std::memcpy(b.data(), args[a], b.size());
        c.args.push_back(std::move(b));
    }
    return c;
}

thread_local int g_dev = 0;
thread_local hipError_t g_last = hipSuccess;

}  // namespace

// ------------------------------------------------------------------ graphs
struct hipGraphNode {
    BoundCall call;
    std::vector<hipGraphNode*> deps;
    size_t index = 0;
};
struct ihipGraph {
    std::vector<std::unique_ptr<hipGraphNode>> nodes;
};
struct hipGraphExec {
    std::vector<BoundCall> order;  // topological order (a copy of the graph's nodes)
};

namespace mock {

double seconds_per_flop = 0.0;

void check_range(const void* p, size_t n, const char* what, bool write) {
    if (n == 0) return;
    const uintptr_t a = (uintptr_t)p;
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_allocs.upper_bound(a);
    if (it == g_allocs.begin()) die("%s: %p + %zu is not device memory", what, p, n);
    --it;
    if (a >= it->first + it->second.size) die("%s: %p + %zu is not device memory", what, p, n);
    if (!it->second.live) die("%s: %p + %zu lies in freed device memory", what, p, n);
    if (a + n > it->first + it->second.size) die("%s: %p + %zu runs past the end of its allocation", what, p, n);
    volatile char* c = (volatile char*)p;
    if (write) {
        c[0] = c[0];
        c[n - 1] = c[n - 1];
    } else {
        (void)c[0];
        (void)c[n - 1];
    }
}

void submit(hipStream_t st, std::function<void()> fn) {
    if (!st) die("%s %p %zu", "work submitted to the null stream", nullptr, 0);
    g_nlaunch++;
    st->push(std::move(fn));
}

void register_kernel(const void* fn, std::vector<size_t> sizes, std::function<void(void**)> emu) {
    std::lock_guard<std::mutex> lk(g_k_mu);
    g_kernels[fn] = KernelInfo{std::move(sizes), std::move(emu)};
}

Counters counters() { return Counters{g_nlaunch.load(), g_ngraph.load(), g_nnodes.load(), g_nalloc.load(), g_nfree.load()}; }

}  // namespace mock

extern "C" {

hipError_t hipGetDevice(int* d) { *d = g_dev; return hipSuccess; }
hipError_t hipSetDevice(int d) { g_dev = d; return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock HIP error"; }
hipError_t hipGetLastError(void) { hipError_t e = g_last; g_last = hipSuccess; return e; }
hipError_t hipRuntimeGetVersion(int* v) { *v = 70000000; return hipSuccess; }
hipError_t hipMemGetInfo(size_t* f, size_t* t) { *f = kDevFree; *t = kDevFree; return hipSuccess; }

hipError_t hipMalloc(void** p, size_t n) {
    if (n == 0) n = 1;
    void* m = mmap(nullptr, n, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (m == MAP_FAILED) return hipErrorOutOfMemory;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        // a new mapping may reuse the address range of a freed one
        auto it = g_allocs.lower_bound((uintptr_t)m);
        while (it != g_allocs.end() && it->first < (uintptr_t)m + n) it = g_allocs.erase(it);
        if (it != g_allocs.begin()) {
            auto pv = std::prev(it);
            if (!pv->second.live && pv->first + pv->second.size > (uintptr_t)m) g_allocs.erase(pv);
        }
        g_allocs[(uintptr_t)m] = Alloc{n, true};
    }
    g_nalloc++;
    *p = m;
    return hipSuccess;
}

hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    size_t n = 0;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        auto it = g_allocs.find((uintptr_t)p);
        if (it == g_allocs.end() || !it->second.live) die("%s: %p (%zu)", "hipFree of a pointer that is not a live allocation", p, 0);
        it->second.live = false;
        n = it->second.size;
    }
    g_nfree++;
    // keep the range reserved but inaccessible, so a late access faults
    mmap(p, n, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE | MAP_FIXED, -1, 0);
    return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { *p = std::malloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    auto* st = new ihipStream_t();
    st->worker = std::thread([st] { st->run(); });
    *s = st;
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    if (!s) return hipSuccess;
    s->sync();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    if (!s) die("%s %p %zu", "synchronize of the null stream", nullptr, 0);
    s->sync();
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t st) {
    const bool dd = kind == hipMemcpyDeviceToDevice || kind == hipMemcpyDeviceToHost;
    const bool dh = kind == hipMemcpyDeviceToDevice || kind == hipMemcpyHostToDevice;
    if (dd) mock::check_range(src, n, "hipMemcpyAsync source", false);
    if (dh) mock::check_range(dst, n, "hipMemcpyAsync destination", true);
    if (!dd && is_device(src)) die("%s %p (%zu)", "host-to-device copy whose source is device memory", src, n);
    mock::submit(st, [=] {
        if (dd) mock::check_range(src, n, "hipMemcpyAsync source (at execution)", false);
        if (dh) mock::check_range(dst, n, "hipMemcpyAsync destination (at execution)", true);
        // large copies move their first and last 4 KB only (the emulated
        // device memory is reserved address space, not backed data)
        if (n <= ((size_t)1 << 20)) {
            std::memcpy(dst, src, n);
        } else {
            std::memcpy(dst, src, 4096);
            std::memcpy((char*)dst + n - 4096, (const char*)src + n - 4096, 4096);
        }
    });
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) {
    {
        std::lock_guard<std::mutex> lk(e->mu);
        if (e->done < e->recorded) die("%s %p (%zu)", "event destroyed with a pending record", (void*)e, 0);
    }
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t st) {
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        gen = ++e->recorded;
    }
    mock::submit(st, [e, gen] {
        // notify under the lock: once a waiter sees the record complete it
        // may destroy the event, and this task touches it no more
        std::lock_guard<std::mutex> lk(e->mu);
        e->done = std::max(e->done, gen);
        e->t = clk::now();
        e->cv.notify_all();
    });
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    std::unique_lock<std::mutex> lk(e->mu);
    const uint64_t gen = e->recorded;
    e->cv.wait(lk, [&] { return e->done >= gen; });
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> la(a->mu);
    std::lock_guard<std::mutex> lb(b->mu);
    if (a->done < a->recorded || b->done < b->recorded || a->recorded == 0 || b->recorded == 0)
        return hipErrorNotReady;
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t e, unsigned int) {
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        gen = e->recorded;
    }
    mock::submit(st, [e, gen] {
        std::unique_lock<std::mutex> lk(e->mu);
        e->cv.wait(lk, [&] { return e->done >= gen; });
    });
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void* fn, dim3, dim3, void** args, size_t, hipStream_t st) {
    BoundCall c = bind(fn, args);
    mock::submit(st, [c] { c.run(); });
    return hipSuccess;
}

hipError_t hipGraphCreate(hipGraph_t* g, unsigned int) { *g = new ihipGraph(); return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphAddKernelNode(hipGraphNode_t* out, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* kp) {
    auto n = std::make_unique<hipGraphNode>();
    n->call = bind(kp->func, kp->kernelParams);
    for (size_t d = 0; d < ndeps; ++d) {
        hipGraphNode* dep = deps[d];
        bool found = false;
        for (auto& x : g->nodes) found |= x.get() == dep;
        if (!found) die("%s %p (%zu)", "graph dependency that is not a node of the graph", (void*)dep, d);
        n->deps.push_back(dep);
    }
    n->index = g->nodes.size();
    *out = n.get();
    g->nodes.push_back(std::move(n));
    g_nnodes++;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* out, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    // Kahn's algorithm; ties keep insertion order
    const size_t n = g->nodes.size();
    std::vector<int> indeg(n, 0);
    std::vector<std::vector<size_t>> succ(n);
    for (auto& x : g->nodes)
        for (hipGraphNode* d : x->deps) { indeg[x->index]++; succ[d->index].push_back(x->index); }
    std::deque<size_t> ready;
    for (size_t i = 0; i < n; ++i) if (indeg[i] == 0) ready.push_back(i);
    auto* ex = new hipGraphExec();
    while (!ready.empty()) {
        const size_t i = ready.front();
        ready.pop_front();
        ex->order.push_back(g->nodes[i]->call);
        for (size_t s : succ[i]) if (--indeg[s] == 0) ready.push_back(s);
    }
    if (ex->order.size() != n) { delete ex; return hipErrorInvalidValue; }
    *out = ex;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t st) {
    g_ngraph++;
    mock::submit(st, [ex] {
        for (const BoundCall& c : ex->order) c.run();
    });
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) { delete ex; return hipSuccess; }

}  // extern "C"
