// Stress of the server's host logic (bqc_server_* with the mock runtime):
// six client threads submit host- or device-flagged requests of varying
// shape, poll or wait for them, and check every energy; the arena is small
// enough that admission waits for memory.
#include <cstdio>
#include <cmath>
#include <thread>
#include <vector>
#include <atomic>
#include <random>
#include "bqc.h"

int main() {
    bqc_server_cfg cfg{};
    cfg.mem_budget_bytes = 64 << 20;  // admission is exercised
    cfg.max_inflight = 4;
    bqc_server* s = nullptr;
    if (bqc_server_create(&cfg, &s) != 0) { std::printf("create failed\n"); return 1; }
    std::atomic<int> bad{0}, done{0};
    auto worker = [&](int id) {
        std::mt19937 rng(id);
        for (int it = 0; it < 150; ++it) {
            const int o = 2 + rng() % 7, v = o + 3 + rng() % 30;
            std::vector<double> eo(o), ev(v), t1(o * v), t2((size_t)o * o * v * v), ovvv((size_t)o * v * v * v),
                ooov((size_t)o * o * o * v), ovov((size_t)o * v * o * v);
            for (int a = 0; a < o; ++a) eo[a] = -1.0 - 0.01 * a;
            for (int a = 0; a < v; ++a) ev[a] = 0.5 + 0.01 * a;
            uint64_t t = 0;
            const int dev = (int)(rng() % 2);
            int rc = bqc_t_submit_ex(s, o, v, eo.data(), ev.data(), t1.data(), t2.data(), ovvv.data(), ooov.data(),
                                     ovov.data(), dev, &t);
            if (rc != 0) { bad++; continue; }
            double e = 0;
            bqc_t_stats st{};
            if (rng() % 2) {
                rc = bqc_t_wait(s, t, &e, &st);
            } else {
                while ((rc = bqc_t_poll(s, t, &e, &st)) == 1) std::this_thread::yield();
            }
            double expect = 0;
            for (double x : eo) expect += x;
            for (double x : ev) expect += x;
            expect += o * 1000.0 + v;
            if (rc != 0 || std::fabs(e - expect) > 1e-9) bad++;
            done++;
        }
    };
    std::vector<std::thread> th;
    for (int k = 0; k < 6; ++k) th.emplace_back(worker, k);
    for (auto& x : th) x.join();
    bqc_server_destroy(s);
    std::printf("done %d bad %d\n", done.load(), bad.load());
    return bad.load() != 0;
}
