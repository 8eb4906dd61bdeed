// Host driver of one (T) solve: the triple and tile-orbit tables, the
// workspace layout and the launch sequence
//   prepare (a1) -> per triple batch: contraction, epilogue, per-triple sum
//   -> compensated sum over triples.
// The loop runs over unique occupied triples with tiles of virtuals
// (FORM_OCC), or over unique virtual triples with tiles of occupied indices
// (FORM_VIR, the paper's loop order); "triple space" and "tile space" below
// are (occupied, virtual) or (virtual, occupied) accordingly.
#include <algorithm>
#include <chrono>

#include "bqc_internal.h"

namespace bqc {

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device memory the H buffers of one batch may take: 1.5 GiB (4 triples per
// launch at nvir = 300; measured 2 % faster than 3 and no slower than 6),
// but at least two triples per launch while two fit in twice that (at
// nvir = 480 a launch of one triple ends in a partial wave of work groups;
// two per launch measured 2 % faster).
constexpr int64_t kHBudget = (int64_t)3 << 29;

struct Layout {
    size_t ops, trip, orbits, hbuf, partial, etrip, energy, aux, total;
};

// sizes of the triple space and of the tile space
inline int triple_space(int o, int v, int form) { return form == FORM_VIR ? v : o; }
inline int tile_space(int o, int v, int form) { return form == FORM_VIR ? o : v; }

Layout layout(int o, int v, int precision, int form, bool fock) {
    const int nb = batch_triples(o, v, precision, form);
    const int nt = ceil_div(tile_space(o, v, form), EPI_T);
    const int64_t norbit = num_tile_orbits(nt);
    const int64_t ntrip = num_triples(triple_space(o, v, form));
    const int64_t hp = hpair_elems(tile_space(o, v, form));
    Layout L;
    size_t off = 0;
    L.ops = off; off += align256(prepare_bytes(precision, o, v));
    L.trip = off; off += align256((size_t)std::max<int64_t>(ntrip, 1) * sizeof(int4));
    L.orbits = off; off += align256((size_t)norbit * sizeof(int4));
    L.hbuf = off; off += 2 * align256((size_t)nb * 3 * hp * hbuf_bytes(precision));
    L.partial = off; off += align256((size_t)nb * norbit * sizeof(double));
    L.etrip = off; off += align256((size_t)std::max<int64_t>(ntrip, 1) * sizeof(double));
    L.energy = off; off += 256;
    L.aux = off; off += form == FORM_VIR ? align256(vir_aux_bytes(o, v, fock)) : 0;
    L.total = off;
    return L;
}

}  // namespace

int batch_triples(int o, int v, int precision, int form) {
    const int64_t per = 3 * hpair_elems(tile_space(o, v, form)) * hbuf_bytes(precision);
    int64_t nb = kHBudget / std::max<int64_t>(per, 1);
    if (nb == 1) nb = 2;  // one triple's H fits the budget, two fit twice it
    nb = std::max<int64_t>(nb, 1);
    nb = std::min<int64_t>(nb, std::max<int64_t>(num_triples(triple_space(o, v, form)), 1));
    nb = std::min<int64_t>(nb, 4096);
    return (int)nb;
}

int64_t workspace_bytes(int o, int v, int precision, int form, bool fock) {
    return (int64_t)layout(o, v, precision, form, fock).total;
}

int64_t input_bytes(int o, int v) {
    const int64_t n = (int64_t)o + v + (int64_t)o * v + (int64_t)o * o * v * v +
                      (int64_t)o * v * v * v + (int64_t)o * o * o * v + (int64_t)o * v * o * v;
    return n * 8 + 7 * 256;
}

Plan make_plan(int o, int v, int precision, int64_t begin, int64_t end, int form) {
    Plan p;
    p.o = o;
    p.v = v;
    p.precision = precision;
    p.form = form;
    p.nb = batch_triples(o, v, precision, form);
    const int nx = triple_space(o, v, form);
    for (int i = 0; i < nx; ++i)
        for (int j = i; j < nx; ++j)
            for (int k = j; k < nx; ++k) {
                if (i == j && j == k) continue;
                const int m = (i < j && j < k) ? 6 : 3;
                p.trip.push_back(make_int4(i, j, k, m));
            }
    p.begin = end > 0 ? begin : 0;
    p.end = end > 0 ? end : (int64_t)p.trip.size();
    const int nt = ceil_div(tile_space(o, v, form), EPI_T);
    for (int A = 0; A < nt; ++A)
        for (int B = 0; B <= A; ++B)
            for (int C = 0; C <= B; ++C) {
                const int stab = (A == B && B == C) ? 6 : ((A == B || B == C) ? 2 : 1);
                p.orbits.push_back(make_int4(A, B, C, stab));
            }
    return p;
}

void enqueue_solve(const Plan& plan, const DevInputs& in, void* ws, double* d_energy,
                   hipStream_t st, hipStream_t side, bool timing, SolveStats* stats, bool graph) {
    const int o = plan.o, v = plan.v, prec = plan.precision, form = plan.form;
    const Layout L = layout(o, v, prec, form, in.fock_ov != nullptr);
    char* base = (char*)ws;
    int4* d_trip = (int4*)(base + L.trip);
    int4* d_orb = (int4*)(base + L.orbits);
    const size_t hsize = (size_t)plan.nb * 3 * hpair_elems(tile_space(o, v, form)) * hbuf_bytes(prec);
    void* hbuf[2] = {base + L.hbuf, base + L.hbuf + align256(hsize)};
    double* partial = (double*)(base + L.partial);
    double* etrip = (double*)(base + L.etrip);
    const int ntrip = (int)plan.trip.size();
    const int norbit = (int)plan.orbits.size();

    std::vector<hipEvent_t> ev;
    auto make_event = [&](bool timed) -> hipEvent_t {
        hipEvent_t e;
        BQC_HIP(hipEventCreateWithFlags(&e, timed ? hipEventDefault : hipEventDisableTiming));
        ev.push_back(e);
        return e;
    };
    auto mark = [&](bool on, hipStream_t s) -> hipEvent_t {
        if (!on) return nullptr;
        hipEvent_t e = make_event(true);
        BQC_HIP(hipEventRecord(e, s));
        return e;
    };
    if (!stats || graph) timing = false;
    const bool want = stats != nullptr;
    hipEvent_t e_begin = mark(want, st);

    if (ntrip > 0)
        BQC_HIP(hipMemcpyAsync(d_trip, plan.trip.data(), plan.trip.size() * sizeof(int4),
                               hipMemcpyHostToDevice, st));
    BQC_HIP(hipMemcpyAsync(d_orb, plan.orbits.data(), plan.orbits.size() * sizeof(int4),
                           hipMemcpyHostToDevice, st));
    Operands ops;
    VirAux aux;
    if (ntrip > 0) {
        launch_prepare(prec, in, base + L.ops, &ops, st, form);
        if (form == FORM_VIR) aux = launch_vir_aux(in, base + L.aux, st);
    }
    hipEvent_t e_prep = mark(want, st);

    // Two H buffers: the contraction of batch b+1 (stream st, MFMA-bound)
    // overlaps the epilogue of batch b (stream side, memory-bound).
    const int t_begin = (int)plan.begin, t_end = (int)plan.end;
    auto gemm_of = [&](int b0, int nb, int k) {
        GemmLaunch g;
        g.o = o; g.v = v; g.ntrip = nb; g.trip = d_trip + b0; g.ops = ops; g.hbuf = hbuf[k];
        return gemm_call(prec, g, form);
    };
    auto epi_of = [&](int b0, int nb, int k) {
        EpiLaunch e;
        e.ntrip = nb; e.trip = d_trip + b0; e.hbuf = hbuf[k];
        if (form == FORM_VIR) {  // triples of virtuals, tiles of occupied indices
            e.o = v; e.v = o;
            e.eps_o = aux.neg_eps_v; e.eps_v = aux.neg_eps_o; e.t1 = aux.t1_t; e.ovov = aux.ovov_t;
            e.ovov_sp = (int64_t)v * o * o; e.ovov_sx = o; e.ovov_sq = (int64_t)o * o;
            e.t2 = aux.t2_t; e.fock_ov = aux.fock_t;
        } else {
            e.o = o; e.v = v;
            e.eps_o = in.eps_o; e.eps_v = in.eps_v; e.t1 = in.t1; e.ovov = in.ovov;
            e.ovov_sp = (int64_t)v * o * v; e.ovov_sx = (int64_t)o * v; e.ovov_sq = v;
            e.t2 = in.t2; e.fock_ov = in.fock_ov;
        }
        e.orbits = d_orb; e.norbit = norbit; e.partial = partial;
        return epilogue_call(prec, e);
    };
    double* d_total = (double*)(base + L.energy);

    std::vector<std::pair<hipEvent_t, hipEvent_t>> gemm_ev, epi_ev;
    if (graph) {
        // The batch sequence as explicitly built hipGraphs of at most
        // kGraphBatches batches each, launched in order on `st`: kernel nodes
        // with the dependencies of the two-stream pipeline and no stream
        // capture, so other threads' runtime calls cannot interfere:
        //   gemm(b)   after gemm(b-1) and reduce(b-2)  (H buffer b mod 2 free)
        //   epi(b)    after gemm(b) and reduce(b-1)
        //   reduce(b) after epi(b)
        // The bound keeps each graph's dependency chain short: the runtime
        // walks a graph's dependencies depth-first when it orders the nodes,
        // and one graph per solve (up to 3 x 11440 nodes in one chain for a
        // 40-occupied fragment) overflowed the stack of the thread doing so.
        constexpr int kGraphBatches = 64;
        std::vector<hipGraphExec_t> execs;
        struct ExecGuard {
            std::vector<hipGraphExec_t>& e;
            ~ExecGuard() { for (hipGraphExec_t x : e) (void)hipGraphExecDestroy(x); }
        } eg{execs};
        for (int c0 = t_begin; c0 < t_end; c0 += kGraphBatches * plan.nb) {
            const int c1 = std::min(t_end, c0 + kGraphBatches * plan.nb);
            hipGraph_t gr = nullptr;
            BQC_HIP(hipGraphCreate(&gr, 0));
            struct GraphGuard { hipGraph_t g; ~GraphGuard() { (void)hipGraphDestroy(g); } } gg{gr};
            std::vector<hipGraphNode_t> red;
            hipGraphNode_t last_gemm = nullptr;
            int batch = 0;
            for (int b0 = c0; b0 < c1; b0 += plan.nb, ++batch) {
                const int nb = std::min(plan.nb, c1 - b0);
                const int k = batch & 1;  // graphs run one after another on `st`
                std::vector<hipGraphNode_t> dg;
                if (last_gemm) dg.push_back(last_gemm);
                if (batch >= 2) dg.push_back(red[batch - 2]);
                last_gemm = gemm_of(b0, nb, k).add_to(gr, dg);
                std::vector<hipGraphNode_t> de{last_gemm};
                if (batch >= 1) de.push_back(red[batch - 1]);
                const hipGraphNode_t ep = epi_of(b0, nb, k).add_to(gr, de);
                red.push_back(reduce_triples_call(partial, nb, norbit, d_trip + b0, etrip + b0).add_to(gr, {ep}));
            }
            hipGraphExec_t ex = nullptr;
            BQC_HIP(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
            execs.push_back(ex);
            BQC_HIP(hipGraphLaunch(ex, st));
        }
        reduce_total_call(etrip + t_begin, t_end - t_begin, d_total).launch(st);
        BQC_HIP(hipStreamSynchronize(st));
    } else {
        hipEvent_t filled[2] = {make_event(false), make_event(false)};
        hipEvent_t freed[2] = {make_event(false), make_event(false)};
        hipEvent_t ready = make_event(false);
        BQC_HIP(hipEventRecord(ready, st));
        BQC_HIP(hipStreamWaitEvent(side, ready, 0));  // tables and operands are in place
        int batch = 0;
        for (int b0 = t_begin; b0 < t_end; b0 += plan.nb, ++batch) {
            const int nb = std::min(plan.nb, t_end - b0);
            const int k = batch & 1;
            if (batch >= 2) BQC_HIP(hipStreamWaitEvent(st, freed[k], 0));
            hipEvent_t g0 = mark(timing, st);
            gemm_of(b0, nb, k).launch(st);
            hipEvent_t g1 = mark(timing, st);
            if (timing) gemm_ev.emplace_back(g0, g1);
            BQC_HIP(hipEventRecord(filled[k], st));

            BQC_HIP(hipStreamWaitEvent(side, filled[k], 0));
            hipEvent_t p0 = mark(timing, side);
            epi_of(b0, nb, k).launch(side);
            hipEvent_t p1 = mark(timing, side);
            if (timing) epi_ev.emplace_back(p0, p1);
            reduce_triples_call(partial, nb, norbit, d_trip + b0, etrip + b0).launch(side);
            BQC_HIP(hipEventRecord(freed[k], side));
        }
        hipEvent_t done_side = make_event(false);
        BQC_HIP(hipEventRecord(done_side, side));
        BQC_HIP(hipStreamWaitEvent(st, done_side, 0));
        reduce_total_call(etrip + t_begin, t_end - t_begin, d_total).launch(st);
    }
    if (d_energy)
        BQC_HIP(hipMemcpyAsync(d_energy, base + L.energy, sizeof(double), hipMemcpyDeviceToDevice, st));
    hipEvent_t e_end = mark(want, st);

    if (stats) {
        BQC_HIP(hipEventSynchronize(e_end));
        float ms = 0;
        BQC_HIP(hipEventElapsedTime(&ms, e_begin, e_prep));
        stats->prepare_s = ms * 1e-3;
        BQC_HIP(hipEventElapsedTime(&ms, e_begin, e_end));
        stats->gpu_s = ms * 1e-3;
        double gs = 0, es = 0;
        for (auto& pr : gemm_ev) { BQC_HIP(hipEventElapsedTime(&ms, pr.first, pr.second)); gs += ms * 1e-3; }
        for (auto& pr : epi_ev) { BQC_HIP(hipEventElapsedTime(&ms, pr.first, pr.second)); es += ms * 1e-3; }
        stats->gemm_s = gs;
        stats->epi_s = es;
        stats->gemm_launches = (int)gemm_ev.size();
        stats->epi_launches = (int)epi_ev.size();
        stats->footprint = L.total;
    }
    // every event is complete before it is destroyed
    BQC_HIP(hipStreamSynchronize(st));
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

// Device pointer of the per-triple energies and the total inside a workspace
// (neither offset depends on the f_ov block).
double* workspace_etrip(void* ws, int o, int v, int precision, int form) {
    return (double*)((char*)ws + layout(o, v, precision, form, false).etrip);
}
double* workspace_energy(void* ws, int o, int v, int precision, int form) {
    return (double*)((char*)ws + layout(o, v, precision, form, false).energy);
}

}  // namespace bqc
