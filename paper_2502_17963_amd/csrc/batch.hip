// Batched solve of several independent fragments (each its own (T) energy,
// paper section 2.4.2; the fragments of the paper's embedding layer are
// independent problems, section 2.5).  Small fragments leave the device idle
// between the launches of their own solves; here every step of the path is
// one grouped launch over all fragments:
//   operand conversion (one launch per factor, all fragments),
//   then R rounds of [contraction, epilogue, per-triple sums], each a
//   grouped launch over the current triple batch of every fragment that has
//   one left (one contraction launch per wave-tile size in use),
//   then the fixed-order total of every fragment in one launch.
// Fragment f runs its unique triples in batches of nb_f = ceil(ntrip_f / R)
// through its own H buffer, with R the smallest number of rounds whose H
// buffers fit the batch's H budget.  A triple's energy and the order of every
// sum do not depend on the batching, so each fragment's energy is bitwise the
// one bqc_t_energy_ex returns for it alone.
#include <algorithm>
#include <vector>

#include "bqc_internal.h"

namespace bqc {

namespace {

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device memory the H buffers of a batch may take together.
constexpr int64_t kBatchHBudget = (int64_t)8 << 30;

int64_t h_per_triple(int v, int precision) { return 3 * hpair_elems(v) * hbuf_bytes(precision); }

}  // namespace

BatchPlan plan_batch(int n, const int* nocc, const int* nvir, int precision) {
    BatchPlan bp;
    bp.frag.resize(n);
    int64_t max_trip = 0;
    for (int f = 0; f < n; ++f) {
        BatchFrag& x = bp.frag[f];
        x.o = nocc[f];
        x.v = nvir[f];
        x.ntrip = num_triples(x.o);
        x.norbit = (int)num_tile_orbits(ceil_div(x.v, EPI_T));
        max_trip = std::max(max_trip, x.ntrip);
    }
    // fewest rounds whose H buffers fit the budget (at least one triple per round)
    auto h_need = [&](int64_t R) {
        int64_t s = 0;
        for (const BatchFrag& x : bp.frag)
            if (x.ntrip > 0) s += (x.ntrip + R - 1) / R * h_per_triple(x.v, precision);
        return s;
    };
    int64_t lo = 1, hi = std::max<int64_t>(max_trip, 1);
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (h_need(mid) <= kBatchHBudget) hi = mid;
        else lo = mid + 1;
    }
    bp.rounds = max_trip > 0 ? (int)lo : 0;
    size_t off = 0;
    for (BatchFrag& x : bp.frag) {
        x.nb = bp.rounds > 0 ? (int)((x.ntrip + bp.rounds - 1) / bp.rounds) : 0;
        x.ops = off; off += a256((size_t)prepare_bytes(precision, x.o, x.v));
        x.hbuf = off; off += a256((size_t)x.nb * h_per_triple(x.v, precision));
        x.partial = off; off += a256((size_t)x.nb * x.norbit * sizeof(double));
        x.etrip = off; off += a256((size_t)std::max<int64_t>(x.ntrip, 1) * sizeof(double));
    }
    // triple and tile-orbit tables of every fragment, contiguous (one copy)
    bp.tabs = off;
    size_t tab = 0;
    for (BatchFrag& x : bp.frag) {
        x.trip = tab; tab += (size_t)x.ntrip * sizeof(int4);
        x.orbits = tab; tab += (size_t)x.norbit * sizeof(int4);
    }
    bp.tabs_bytes = tab;
    off += a256(tab);
    // grouped-launch tables: factors (4 n), per round n entries of each
    // kind, totals (n), and the energies (n)
    bp.factor_tab = off; off += a256((size_t)4 * n * sizeof(FactorGroupEntry));
    bp.entries = off;
    bp.entries_bytes = (size_t)bp.rounds * n * (sizeof(GemmGroupEntry) + sizeof(EpiGroupEntry) + sizeof(RedGroupEntry)) +
                       (size_t)n * sizeof(TotalGroupEntry);
    off += a256(bp.entries_bytes);
    bp.energies = off; off += a256((size_t)std::max(n, 1) * sizeof(double));
    bp.total = off;
    return bp;
}

void enqueue_batch(const BatchPlan& bp, int precision, int n, const DevInputs* ins, void* ws, hipStream_t st,
                   double* energies_host, SolveStats* stats) {
    char* base = (char*)ws;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Ev { hipEvent_t* a; hipEvent_t* b; ~Ev() { if (*a) (void)hipEventDestroy(*a); if (*b) (void)hipEventDestroy(*b); } } evg{&e0, &e1};
    if (stats) {
        BQC_HIP(hipEventCreate(&e0));
        BQC_HIP(hipEventCreate(&e1));
        BQC_HIP(hipEventRecord(e0, st));
    }
    // tables of triples and tile orbits
    std::vector<char> tabs(std::max<size_t>(bp.tabs_bytes, 1));
    for (int f = 0; f < n; ++f) {
        const BatchFrag& x = bp.frag[f];
        const Plan p = make_plan(x.o, x.v, precision);
        if (x.ntrip > 0) std::memcpy(tabs.data() + x.trip, p.trip.data(), x.ntrip * sizeof(int4));
        std::memcpy(tabs.data() + x.orbits, p.orbits.data(), x.norbit * sizeof(int4));
    }
    if (bp.tabs_bytes) BQC_HIP(hipMemcpyAsync(base + bp.tabs, tabs.data(), bp.tabs_bytes, hipMemcpyHostToDevice, st));

    // operand conversion, one launch per factor
    std::vector<void*> ws_ops(n);
    std::vector<Operands> ops(n);
    for (int f = 0; f < n; ++f) ws_ops[f] = base + bp.frag[f].ops;
    std::vector<FactorGroupEntry> ftab;
    launch_prepare_group(precision, n, ins, ws_ops.data(), ops.data(), (FactorGroupEntry*)(base + bp.factor_tab), ftab,
                         st);

    // grouped-launch entries of every round, built on the host, one copy
    const int R = bp.rounds;
    std::vector<char> ent(std::max<size_t>(bp.entries_bytes, 1));
    GemmGroupEntry* g_h = (GemmGroupEntry*)ent.data();
    EpiGroupEntry* e_h = (EpiGroupEntry*)(g_h + (size_t)R * n);
    RedGroupEntry* r_h = (RedGroupEntry*)(e_h + (size_t)R * n);
    TotalGroupEntry* t_h = (TotalGroupEntry*)(r_h + (size_t)R * n);
    GemmGroupEntry* g_d = (GemmGroupEntry*)(base + bp.entries);
    EpiGroupEntry* e_d = (EpiGroupEntry*)(g_d + (size_t)R * n);
    RedGroupEntry* r_d = (RedGroupEntry*)(e_d + (size_t)R * n);
    TotalGroupEntry* t_d = (TotalGroupEntry*)(r_d + (size_t)R * n);
    double* d_energies = (double*)(base + bp.energies);

    struct GemmLaunchSet { int wb, first, count; int64_t n_wg; };
    struct RoundLaunches {
        std::vector<GemmLaunchSet> gemm;
        int epi_first = 0, epi_count = 0, red_first = 0, red_count = 0;
        int64_t epi_wg = 0;
        int red_blocks = 0;
    };
    std::vector<RoundLaunches> rounds(R);
    for (int r = 0; r < R; ++r) {
        RoundLaunches& rl = rounds[r];
        // contraction entries grouped by wave tile, each group contiguous
        int gi = r * n;
        for (int wb = 2; wb <= 5; ++wb) {
            GemmLaunchSet set{wb, gi, 0, 0};
            for (int f = 0; f < n; ++f) {
                const BatchFrag& x = bp.frag[f];
                const int64_t b0 = (int64_t)r * x.nb;
                if (b0 >= x.ntrip || wave_blocks(x.v) != wb) continue;
                const int nbt = (int)std::min<int64_t>(x.nb, x.ntrip - b0);
                GemmGroupEntry& y = g_h[gi++];
                y.g.o = x.o; y.g.v = x.v; y.g.ntrip = nbt;
                y.g.trip = (const int4*)(base + bp.tabs + x.trip) + b0;
                y.g.ops = ops[f];
                y.g.hbuf = base + x.hbuf;
                const Tiling tl = contraction_tiling(x.v, wb, nbt);
                y.nblk = tl.nblk; y.ntile_u = tl.ntile_u; y.ntile_w = tl.ntile_w;
                y.wg0 = (int)set.n_wg;
                set.n_wg += tl.n_wg;
                if (set.n_wg > ((int64_t)1 << 31) - 8) throw Error(-1, "batch contraction grid too large");
                ++set.count;
            }
            if (set.count) rl.gemm.push_back(set);
        }
        rl.epi_first = rl.red_first = r * n;
        for (int f = 0; f < n; ++f) {
            const BatchFrag& x = bp.frag[f];
            const int64_t b0 = (int64_t)r * x.nb;
            if (b0 >= x.ntrip) continue;
            const int nbt = (int)std::min<int64_t>(x.nb, x.ntrip - b0);
            const int4* trip = (const int4*)(base + bp.tabs + x.trip) + b0;
            EpiGroupEntry& y = e_h[r * n + rl.epi_count++];
            y.e.o = x.o; y.e.v = x.v; y.e.ntrip = nbt; y.e.trip = trip; y.e.hbuf = base + x.hbuf;
            y.e.eps_o = ins[f].eps_o; y.e.eps_v = ins[f].eps_v; y.e.t1 = ins[f].t1; y.e.ovov = ins[f].ovov;
            y.e.ovov_sp = (int64_t)x.v * x.o * x.v; y.e.ovov_sx = (int64_t)x.o * x.v; y.e.ovov_sq = x.v;
            y.e.t2 = ins[f].t2; y.e.fock_ov = nullptr;
            y.e.orbits = (const int4*)(base + bp.tabs + x.orbits);
            y.e.norbit = x.norbit;
            y.e.partial = (double*)(base + x.partial);
            y.wg0 = (int)rl.epi_wg;
            rl.epi_wg += (int64_t)nbt * x.norbit;
            if (rl.epi_wg > ((int64_t)1 << 31) - 1) throw Error(-1, "batch epilogue grid too large");
            RedGroupEntry& z = r_h[r * n + rl.red_count++];
            z.partial = (const double*)(base + x.partial);
            z.norbit = x.norbit;
            z.trip = trip;
            z.e_trip = (double*)(base + x.etrip) + b0;
            z.b0 = rl.red_blocks;
            rl.red_blocks += nbt;
        }
    }
    for (int f = 0; f < n; ++f) {
        const BatchFrag& x = bp.frag[f];
        t_h[f].e_trip = (const double*)(base + x.etrip);
        t_h[f].n = x.ntrip;
        t_h[f].out = d_energies + f;
    }
    BQC_HIP(hipMemcpyAsync(g_d, ent.data(), bp.entries_bytes, hipMemcpyHostToDevice, st));

    int gemm_launches = 0, epi_launches = 0;
    for (int r = 0; r < R; ++r) {
        const RoundLaunches& rl = rounds[r];
        for (const GemmLaunchSet& set : rl.gemm) {
            gemm_group_call(precision, set.wb, g_d + set.first, set.count, set.n_wg).launch(st);
            ++gemm_launches;
        }
        if (rl.epi_count) {
            epilogue_group_call(precision, e_d + rl.epi_first, rl.epi_count, rl.epi_wg).launch(st);
            reduce_triples_group_call(r_d + rl.red_first, rl.red_count, rl.red_blocks).launch(st);
            ++epi_launches;
        }
    }
    if (n > 0) reduce_total_group_call(t_d, n).launch(st);
    if (stats) BQC_HIP(hipEventRecord(e1, st));
    if (n > 0) BQC_HIP(hipMemcpyAsync(energies_host, d_energies, n * sizeof(double), hipMemcpyDeviceToHost, st));
    BQC_HIP(hipStreamSynchronize(st));
    if (stats) {
        float ms = 0;
        BQC_HIP(hipEventElapsedTime(&ms, e0, e1));
        stats->gpu_s = ms * 1e-3;
        stats->gemm_launches = gemm_launches;
        stats->epi_launches = epi_launches;
        stats->footprint = bp.total;
    }
}

}  // namespace bqc
