// Test infrastructure: drivers of the real server (server.cpp), C ABI
// (abi.cpp) and solve driver (solve.hip) on the stand-in runtime
// (mock_hip.cpp, mock_kernels.cpp), for AddressSanitizer,
// UndefinedBehaviorSanitizer and ThreadSanitizer runs on the CPU.
//
//   serving_stress threads
//       six client threads submit small requests (host or device inputs),
//       consume them with poll or wait, and check every energy; a small
//       arena makes admission wait for memory.
//   serving_stress stream <shapes file> <direct_launch 0|1> [max_requests]
//       the serving benchmark's pattern at its real shapes: one thread
//       allocates each fragment's device inputs through a caching allocator
//       when the outstanding input bytes allow, fills them on its own
//       stream, synchronises that stream and submits; it polls every
//       pending ticket, releases the inputs of finished ones and empties the
//       allocator's cache after every completion (device frees while the
//       server's slots run); at the end three fragments are solved alone
//       with bqc_t_energy_ex and compared with their served energies.
//   serving_stress faults <direct_launch 0|1>
//       failure isolation: some requests fail at admission (BQC_ENOMEM) or
//       after their solve (BQC_EDEVICE) by injection, others are cancelled
//       while queued; every other request's energy is unchanged.
//   serving_stress batch
//       bqc_t_energy_batch over fragments of mixed sizes (several rounds of
//       triple batches, host and device inputs): every energy as predicted
//       and equal to the fragment's bqc_t_energy_ex alone.
//   serving_stress consumers
//       two threads consume the same ticket at once (wait and poll); one
//       gets the result, the other BQC_ENOTFOUND; then the server is
//       destroyed while a waiter is blocked on a ticket that never
//       finishes before the destroy.
// The emulated solve's energy is sum over triples of (m/3)(1 + e_i + e_j +
// e_k) (mock_kernels.cpp), which the drivers recompute on the host.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "bqc.h"
#include "mock_hip.h"

namespace bqc {
int server_callers(bqc_server* s);  // server.cpp: threads inside an entry point
void server_inject_fault(bqc_server* s, uint64_t ticket, int stage, int code);  // server.cpp
void server_hold_admission(bqc_server* s, bool on);                               // server.cpp
}

namespace {

double expected_energy(int o, const std::vector<double>& eo) {
    double s = 0;
    for (int i = 0; i < o; ++i)
        for (int j = i; j < o; ++j)
            for (int k = j; k < o; ++k) {
                if (i == j && j == k) continue;
                const int m = (i < j && j < k) ? 6 : 3;
                s += m / 3.0 * (1.0 + eo[i] + eo[j] + eo[k]);
            }
    return s;
}

std::vector<double> occ_energies(int o, int tag) {
    std::vector<double> eo(o);
    for (int i = 0; i < o; ++i) eo[i] = -2.0 + 0.03 * i - 0.001 * (tag % 97);
    return eo;
}

int fails = 0;
std::mutex fail_mu;
void report(const char* what, int tag, double got, double want) {
    std::lock_guard<std::mutex> lk(fail_mu);
    ++fails;
    std::fprintf(stderr, "MISMATCH %s request %d: got %.17g want %.17g\n", what, tag, got, want);
}

// --------------------------------------------------------------- threads
int run_threads() {
    bqc_server_cfg cfg{};
    cfg.mem_budget_bytes = (uint64_t)256 << 20;  // admission waits for memory
    cfg.max_inflight = 4;
    cfg.precision = BQC_PREC_BF16X3;
    bqc_server* s = nullptr;
    if (bqc_server_create(&cfg, &s) != 0) { std::printf("create failed: %s\n", bqc_last_error()); return 1; }
    std::atomic<int> done{0};
    auto worker = [&](int id) {
        std::mt19937 rng(id);
        for (int it = 0; it < 60; ++it) {
            const int o = 2 + rng() % 7, v = o + 3 + rng() % 30;
            const int tag = id * 1000 + it;
            std::vector<double> eo = occ_energies(o, tag), ev(v), t1((size_t)o * v);
            for (int a = 0; a < v; ++a) ev[a] = 0.5 + 0.01 * a;
            const bool dev = rng() % 2;
            const size_t sz[7] = {(size_t)o, (size_t)v, (size_t)o * v, (size_t)o * o * v * v,
                                  (size_t)o * v * v * v, (size_t)o * o * o * v, (size_t)o * v * o * v};
            std::vector<std::vector<double>> host(7);
            const double* ptr[7];
            void* dptr[7] = {};
            for (int a = 0; a < 7; ++a) {
                if (dev) {
                    (void)hipMalloc(&dptr[a], sz[a] * 8);
                    ptr[a] = (const double*)dptr[a];
                } else {
                    host[a].assign(sz[a], 0.0);
                    ptr[a] = host[a].data();
                }
            }
            if (dev) {
                std::memcpy(dptr[0], eo.data(), o * 8);
                std::memcpy(dptr[1], ev.data(), v * 8);
            } else {
                host[0] = eo;
                host[1] = ev;
                ptr[0] = host[0].data();
                ptr[1] = host[1].data();
            }
            uint64_t t = 0;
            int rc = bqc_t_submit_ex(s, o, v, ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6], dev, &t);
            if (rc != 0) { report("submit", tag, rc, 0); continue; }
            double e = 0;
            bqc_t_stats st{};
            if (rng() % 2) {
                rc = bqc_t_wait(s, t, &e, &st);
            } else {
                while ((rc = bqc_t_poll(s, t, &e, &st)) == BQC_PENDING) std::this_thread::yield();
            }
            const double want = expected_energy(o, eo);
            if (rc != 0 || e != want) report("energy", tag, rc != 0 ? rc : e, want);
            for (int a = 0; a < 7; ++a) if (dptr[a]) (void)hipFree(dptr[a]);
            done++;
        }
    };
    std::vector<std::thread> th;
    for (int k = 0; k < 6; ++k) th.emplace_back(worker, k);
    for (auto& x : th) x.join();
    bqc_server_destroy(s);
    std::printf("threads: done %d bad %d\n", done.load(), fails);
    std::fflush(stdout);
    return fails != 0;
}

// --------------------------------------------------------------- stream
// A caching allocator in the manner of a framework's: freed blocks are kept
// for reuse by size until empty_cache() returns them to the runtime.
struct Cache {
    std::multimap<size_t, void*> free_blocks;
    void* get(size_t n) {
        auto it = free_blocks.find(n);
        if (it != free_blocks.end()) {
            void* p = it->second;
            free_blocks.erase(it);
            return p;
        }
        void* p = nullptr;
        if (hipMalloc(&p, n) != hipSuccess) { std::fprintf(stderr, "allocation failed\n"); std::abort(); }
        return p;
    }
    void put(size_t n, void* p) { free_blocks.emplace(n, p); }
    void empty() {
        for (auto& kv : free_blocks) (void)hipFree(kv.second);
        free_blocks.clear();
    }
};

struct Frag {
    int o, v, tag;
    void* in[7];
    size_t sz[7];
    std::vector<double> eo;
    double served = NAN;
};

int run_stream(const char* path, int direct, int max_req) {
    std::vector<std::pair<int, int>> shapes;
    {
        std::ifstream f(path);
        int o, v;
        while (f >> o >> v) shapes.emplace_back(o, v);
    }
    if (max_req > 0 && (int)shapes.size() > max_req) shapes.resize(max_req);
    mock::seconds_per_flop = 2e-16;  // the stream's ~8e16 flops take ~16 s of emulated device time
    bqc_server_cfg cfg{};
    cfg.mem_budget_bytes = (uint64_t)100e9;
    cfg.max_inflight = 4;
    cfg.precision = BQC_PREC_BF16X3;
    cfg.direct_launch = direct;
    bqc_server* s = nullptr;
    if (bqc_server_create(&cfg, &s) != 0) { std::printf("create failed: %s\n", bqc_last_error()); return 1; }
    hipStream_t gen;
    (void)hipStreamCreateWithFlags(&gen, 0);
    Cache cache;
    const double cap = 80e9;
    double outstanding = 0;
    std::map<uint64_t, Frag*> pending;
    std::vector<Frag*> all;
    size_t next = 0, finished = 0;
    const auto t0 = std::chrono::steady_clock::now();
    while (finished < shapes.size()) {
        while (next < shapes.size()) {
            const int o = shapes[next].first, v = shapes[next].second;
            const size_t sz[7] = {(size_t)o, (size_t)v, (size_t)o * v, (size_t)o * o * v * v,
                                  (size_t)o * v * v * v, (size_t)o * o * o * v, (size_t)o * v * o * v};
            double bytes = 0;
            for (size_t x : sz) bytes += 8.0 * x;
            if (!pending.empty() && outstanding + bytes > cap) break;
            auto* f = new Frag();
            f->o = o; f->v = v; f->tag = (int)next;
            f->eo = occ_energies(o, f->tag);
            for (int a = 0; a < 7; ++a) { f->sz[a] = sz[a] * 8; f->in[a] = cache.get(f->sz[a]); }
            // the framework fills the inputs on its own stream; the binding
            // synchronises it before submitting
            std::vector<double> ev(v);
            for (int a = 0; a < v; ++a) ev[a] = 0.5 + 0.01 * a;
            (void)hipMemcpyAsync(f->in[0], f->eo.data(), o * 8, hipMemcpyHostToDevice, gen);
            (void)hipMemcpyAsync(f->in[1], ev.data(), v * 8, hipMemcpyHostToDevice, gen);
            (void)hipStreamSynchronize(gen);
            uint64_t t = 0;
            const double* p[7];
            for (int a = 0; a < 7; ++a) p[a] = (const double*)f->in[a];
            const int rc = bqc_t_submit_ex(s, o, v, p[0], p[1], p[2], p[3], p[4], p[5], p[6], 1, &t);
            if (rc != 0) { std::printf("submit failed %d: %s\n", rc, bqc_last_error()); return 1; }
            pending[t] = f;
            all.push_back(f);
            outstanding += bytes;
            ++next;
        }
        std::vector<uint64_t> done;
        for (auto& kv : pending) {
            double e = 0;
            bqc_t_stats st{};
            const int rc = bqc_t_poll(s, kv.first, &e, &st);
            if (rc == BQC_PENDING) continue;
            Frag* f = kv.second;
            const double want = expected_energy(f->o, f->eo);
            if (rc != 0 || e != want) report("served energy", f->tag, rc != 0 ? rc : e, want);
            f->served = e;
            done.push_back(kv.first);
        }
        for (uint64_t t : done) {
            Frag* f = pending[t];
            pending.erase(t);
            double bytes = 0;
            for (int a = 0; a < 7; ++a) { bytes += f->sz[a]; }
            outstanding -= bytes;
            ++finished;
            if (f->o > 12 || finished > 8) {  // keep a few small ones for the alone check
                for (int a = 0; a < 7; ++a) { cache.put(f->sz[a], f->in[a]); f->in[a] = nullptr; }
            }
        }
        if (!done.empty()) {
            cache.empty();
            if (finished % 32 == 0) {
                std::printf("stream: %zu/%zu done at %.1f s\n", finished, shapes.size(),
                            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
                std::fflush(stdout);
            }
        } else {
            std::this_thread::sleep_for(std::chrono::microseconds(500));
        }
    }
    // alone = served, for fragments whose inputs were kept
    int alone = 0;
    for (Frag* f : all) {
        if (!f->in[0] || alone >= 3) continue;
        bqc_t_opts op{};
        op.precision = BQC_PREC_BF16X3;
        op.inputs_on_device = 1;
        double e = 0;
        const double* p[7];
        for (int a = 0; a < 7; ++a) p[a] = (const double*)f->in[a];
        const int rc = bqc_t_energy_ex(f->o, f->v, p[0], p[1], p[2], p[3], p[4], p[5], p[6], &op, &e, nullptr);
        if (rc != 0 || e != f->served) report("alone vs served", f->tag, rc != 0 ? rc : e, f->served);
        ++alone;
    }
    bqc_server_destroy(s);
    for (Frag* f : all) {
        for (int a = 0; a < 7; ++a) if (f->in[a]) (void)hipFree(f->in[a]);
        delete f;
    }
    cache.empty();
    (void)hipStreamDestroy(gen);
    const mock::Counters c = mock::counters();
    std::printf("stream: done %zu bad %d alone-checked %d; launches %llu graph launches %llu graph nodes %llu\n",
                finished, fails, alone, (unsigned long long)c.launches, (unsigned long long)c.graph_launches,
                (unsigned long long)c.graph_nodes);
    std::fflush(stdout);
    return fails != 0;
}

// --------------------------------------------------------------- faults
int run_faults(int direct) {
    bqc_server_cfg cfg{};
    cfg.mem_budget_bytes = (uint64_t)6 << 30;  // a few requests at a time: the others queue
    cfg.max_inflight = 3;
    cfg.precision = BQC_PREC_BF16X3;
    cfg.direct_launch = direct;
    bqc_server* s = nullptr;
    if (bqc_server_create(&cfg, &s) != 0) { std::printf("create failed: %s\n", bqc_last_error()); return 1; }
    constexpr int N = 90;
    // tickets count up from 1: inject before submitting
    for (int n = 0; n < N; ++n) {
        const uint64_t t = (uint64_t)n + 1;
        if (n % 7 == 3) bqc::server_inject_fault(s, t, 1, BQC_ENOMEM);
        if (n % 7 == 5) bqc::server_inject_fault(s, t, 2, BQC_EDEVICE);
    }
    struct Job { int o, v; std::vector<double> eo, ev, z; uint64_t t; int cancel_rc; };
    std::vector<Job> jobs(N);
    // nothing is admitted until every request is submitted and the chosen
    // ones are cancelled: those cancels meet queued requests
    bqc::server_hold_admission(s, true);
    for (int n = 0; n < N; ++n) {
        Job& j = jobs[n];
        j.o = 4 + n % 9;
        j.v = 40 + 7 * (n % 5);
        j.eo = occ_energies(j.o, n);
        j.ev.assign(j.v, 0.6);
        j.z.assign((size_t)j.o * j.v * j.v * j.v + (size_t)j.o * j.o * j.v * j.v, 0.0);
        const double* z = j.z.data();
        if (bqc_t_submit(s, j.o, j.v, j.eo.data(), j.ev.data(), z, z, z, z, z, &j.t) != 0 ||
            j.t != (uint64_t)n + 1) {
            std::printf("submit %d failed: %s\n", n, bqc_last_error());
            return 1;
        }
        j.cancel_rc = n % 11 == 4 ? bqc_t_cancel(s, j.t) : 99;
    }
    bqc::server_hold_admission(s, false);
    int bad = 0, cancelled = 0, enomem = 0, edevice = 0, ok = 0;
    for (int n = N - 1; n >= 0; --n) {  // consume in reverse order
        Job& j = jobs[n];
        double e = 0;
        const int rc = bqc_t_wait(s, j.t, &e, nullptr);
        int want = BQC_OK;  // the outcome had the request run
        if (n % 7 == 3) want = BQC_ENOMEM;
        else if (n % 7 == 5) want = BQC_EDEVICE;
        // every cancel met its request queued: it ends with BQC_ECANCELED
        const bool good = j.cancel_rc == 99
                              ? rc == want && (rc != BQC_OK || e == expected_energy(j.o, j.eo))
                              : j.cancel_rc == BQC_OK && rc == BQC_ECANCELED;
        if (!good) {
            std::printf("faults: request %d rc %d (want %d) energy %.17g (want %.17g) cancel %d\n", n, rc, want, e,
                        expected_energy(j.o, j.eo), j.cancel_rc);
            ++bad;
        }
        cancelled += rc == BQC_ECANCELED;
        enomem += rc == BQC_ENOMEM;
        edevice += rc == BQC_EDEVICE;
        ok += rc == BQC_OK;
        double e2 = 0;
        if (bqc_t_poll(s, j.t, &e2, nullptr) != BQC_ENOTFOUND) ++bad;  // consumed
    }
    if (bqc_t_cancel(s, 12345) != BQC_ENOTFOUND) ++bad;
    bqc_server_destroy(s);
    std::printf("faults: ok %d cancelled %d enomem %d edevice %d bad %d\n", ok, cancelled, enomem, edevice, bad);
    std::fflush(stdout);
    return bad != 0 || cancelled == 0 || enomem == 0 || edevice == 0;
}

// --------------------------------------------------------------- batch
int run_batch() {
    int bad = 0;
    const int shapes[][2] = {{12, 120}, {3, 20}, {1, 9}, {12, 118}, {6, 30}, {11, 120}, {8, 60}, {2, 17}};
    const int n = (int)(sizeof(shapes) / sizeof(shapes[0]));
    for (int dev = 0; dev < 2; ++dev) {
        std::vector<std::vector<double>> eo(n), ev(n), big(n);
        std::vector<void*> dmem;
        std::vector<bqc_t_fragment> fr(n);
        for (int f = 0; f < n; ++f) {
            const int o = shapes[f][0], v = shapes[f][1];
            eo[f] = occ_energies(o, 700 + f);
            ev[f].assign(v, 0.4 + 0.001 * f);
            const size_t nbig = (size_t)o * v * v * v + (size_t)o * o * v * v + (size_t)o * o * o * v;
            const double *pe = eo[f].data(), *pv = ev[f].data(), *pz;
            if (dev) {
                void* a = nullptr;
                void* b = nullptr;
                void* c = nullptr;
                (void)hipMalloc(&a, o * 8);
                (void)hipMalloc(&b, v * 8);
                (void)hipMalloc(&c, nbig * 8);
                std::memcpy(a, pe, o * 8);
                std::memcpy(b, pv, v * 8);
                dmem.push_back(a); dmem.push_back(b); dmem.push_back(c);
                pe = (const double*)a; pv = (const double*)b; pz = (const double*)c;
            } else {
                big[f].assign(nbig, 0.0);
                pz = big[f].data();
            }
            fr[f] = bqc_t_fragment{o, v, pe, pv, pz, pz, pz, pz, pz};
        }
        bqc_t_opts op{};
        op.precision = BQC_PREC_BF16X3;
        op.inputs_on_device = dev;
        std::vector<double> e(n, -1.0);
        bqc_t_stats st{};
        const int rc = bqc_t_energy_batch(n, fr.data(), &op, e.data(), &st);
        if (rc != 0) { std::printf("batch failed %d: %s\n", rc, bqc_last_error()); return 1; }
        for (int f = 0; f < n; ++f) {
            const double want = expected_energy(shapes[f][0], eo[f]);
            double alone = 0;
            const bqc_t_fragment& x = fr[f];
            const int rc2 = bqc_t_energy_ex(x.nocc, x.nvir, x.eps_o, x.eps_v, x.t1, x.t2, x.ovvv, x.ooov, x.ovov, &op,
                                            &alone, nullptr);
            if (e[f] != want || rc2 != 0 || alone != e[f]) {
                std::printf("batch fragment %d (%d, %d): %.17g, alone %.17g, want %.17g\n", f, x.nocc, x.nvir, e[f],
                            alone, want);
                ++bad;
            }
        }
        if (st.epilogue_launches < 2) { std::printf("batch ran in one round\n"); ++bad; }
        for (void* p : dmem) (void)hipFree(p);
    }
    std::printf("batch: bad %d\n", bad);
    std::fflush(stdout);
    return bad != 0;
}

// --------------------------------------------------------------- consumers
int run_consumers() {
    bqc_server_cfg cfg{};
    cfg.mem_budget_bytes = (uint64_t)4 << 30;  // two of the (8, 60) requests at a time
    cfg.max_inflight = 2;
    bqc_server* s = nullptr;
    if (bqc_server_create(&cfg, &s) != 0) { std::printf("create failed: %s\n", bqc_last_error()); return 1; }
    int bad = 0;
    for (int round = 0; round < 50; ++round) {
        const int o = 3 + round % 4, v = 12 + round % 9;
        std::vector<double> eo = occ_energies(o, round), ev(v, 0.7), z((size_t)o * v * v * v + o * o * v * v, 0.0);
        uint64_t t = 0;
        if (bqc_t_submit(s, o, v, eo.data(), ev.data(), z.data(), z.data(), z.data(), z.data(), z.data(), &t) != 0) {
            std::printf("submit failed: %s\n", bqc_last_error());
            return 1;
        }
        std::atomic<int> ok{0}, nf{0}, other{0};
        auto consume = [&](bool wait) {
            double e = 0;
            int rc;
            if (wait) rc = bqc_t_wait(s, t, &e, nullptr);
            else while ((rc = bqc_t_poll(s, t, &e, nullptr)) == BQC_PENDING) std::this_thread::yield();
            if (rc == BQC_OK) ok++;
            else if (rc == BQC_ENOTFOUND) nf++;
            else other++;
        };
        std::thread a(consume, true), b(consume, round % 2 == 0), c(consume, false);
        a.join(); b.join(); c.join();
        if (ok.load() != 1 || nf.load() != 2 || other.load() != 0) {
            std::printf("consumers round %d: ok %d notfound %d other %d\n", round, ok.load(), nf.load(), other.load());
            ++bad;
        }
    }
    // destroy while a waiter is blocked on a queued request: the waiter ends
    // with BQC_ESHUTDOWN (or OK if the request ran first), never reads freed state
    {
        std::vector<double> eo = occ_energies(8, 1), ev(60, 0.9), z((size_t)8 * 60 * 60 * 60 + 8 * 8 * 60 * 60, 0.0);
        std::vector<uint64_t> ts(12);
        for (auto& t : ts)
            if (bqc_t_submit(s, 8, 60, eo.data(), ev.data(), z.data(), z.data(), z.data(), z.data(), z.data(), &t) != 0) {
                std::printf("submit failed: %s\n", bqc_last_error());
                return 1;
            }
        std::atomic<int> started{0};
        std::vector<std::thread> ws;
        std::atomic<int> wrong{0}, done_waiting{0};
        for (uint64_t t : ts)
            ws.emplace_back([&, t] {
                started++;
                double e = 0;
                const int rc = bqc_t_wait(s, t, &e, nullptr);
                done_waiting++;
                if (rc != BQC_OK && rc != BQC_ESHUTDOWN && rc != BQC_ENOTFOUND) wrong++;
            });
        while (started.load() < (int)ts.size()) std::this_thread::yield();
        // every waiter is inside bqc_t_wait (or already returned) before the destroy
        while (bqc::server_callers(s) + done_waiting.load() < (int)ts.size()) std::this_thread::yield();
        bqc_server_destroy(s);
        for (auto& w : ws) w.join();
        if (wrong.load()) { std::printf("destroy with waiters: %d unexpected codes\n", wrong.load()); ++bad; }
    }
    std::printf("consumers: bad %d\n", bad);
    std::fflush(stdout);
    return bad != 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) { std::printf("usage: serving_stress threads|stream|consumers ...\n"); return 2; }
    const std::string mode = argv[1];
    if (mode == "threads") return run_threads();
    if (mode == "consumers") return run_consumers();
    if (mode == "batch") return run_batch();
    if (mode == "faults" && argc >= 3) return run_faults(std::atoi(argv[2]));
    if (mode == "stream" && argc >= 4) return run_stream(argv[2], std::atoi(argv[3]), argc > 4 ? std::atoi(argv[4]) : 0);
    std::printf("bad arguments\n");
    return 2;
}
