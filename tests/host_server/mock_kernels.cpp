// Test infrastructure: host stand-ins for the library's kernel launchers
// (the functions the solve driver calls from kernels_*.hip), so that the
// real solve driver (solve.hip), C ABI (abi.cpp) and server (server.cpp)
// run against the stand-in runtime of mock_hip.cpp.
//
// Each emulated kernel checks every device range the real kernel reads or
// writes (sizes from the real host layout functions in sizes.cpp) and passes
// a value along the real data path, so that a driver can predict each
// solve's energy exactly:
//   contraction: writes a signature of (triple, pair) into element 0 of each
//     H pair of its batch;
//   epilogue: checks the signatures of its batch and writes the triple's
//     partial (m / 3) (1 + e_i + e_j + e_k), with e the orbital energies of
//     the triple space it is given, to orbit 0 (the other orbits 0);
//   per-triple sum: sums each triple's orbit partials in order;
//   total: sums the per-triple energies in order.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>

#include "bqc_internal.h"
#include "mock_hip.h"

namespace bqc {
namespace {

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

char k_gemm, k_epi, k_red_trip, k_red_total;  // addresses that stand for the kernels
char k_gemm_group, k_epi_group, k_red_trip_group, k_red_total_group;

float sig(int4 t, int h) { return (float)(h * 1000000 + t.x * 10000 + t.y * 100 + t.z); }

void check_triples(const int4* trip, int n, int nspace, const char* what) {
    mock::check_range(trip, (size_t)n * sizeof(int4), what, false);
    for (int t = 0; t < n; ++t) {
        const int4 x = trip[t];
        const bool ok = 0 <= x.x && x.x <= x.y && x.y <= x.z && x.z < nspace && !(x.x == x.y && x.y == x.z) &&
                        x.w == ((x.x < x.y && x.y < x.z) ? 6 : 3);
        if (!ok) {
            std::fprintf(stderr, "MOCK-HIP FAULT: %s: invalid triple (%d,%d,%d,%d) at %d\n", what, x.x, x.y, x.z, x.w, t);
            std::abort();
        }
    }
}

void emu_gemm(void** a) {
    const GemmLaunch g = *(const GemmLaunch*)a[0];
    const int prec = *(const int*)a[1], form = *(const int*)a[2];
    const int n = form == FORM_VIR ? g.o : g.v, ns = form == FORM_VIR ? g.v : g.o;
    check_triples(g.trip, g.ntrip, ns, "contraction triple table");
    const Sizes z = factor_sizes(g.o, g.v, prec);
    const int eb = operand_bytes(prec);
    mock::check_range(g.ops.ovvv, (size_t)z.m_ovvv * n * z.Kv * eb, "contraction (ov|vv) operand", false);
    mock::check_range(g.ops.t2, (size_t)z.m_t2 * n * z.Kv * eb, "contraction t2 operand", false);
    mock::check_range(g.ops.t2l, (size_t)z.m_t2l * n * z.Ko * eb, "contraction t2 hole operand", false);
    mock::check_range(g.ops.hoo, (size_t)z.m_hoo * n * z.Ko * eb, "contraction (ov|oo) operand", false);
    const int hb = hbuf_bytes(prec);
    const int64_t hp = hpair_elems(n);
    mock::check_range(g.hbuf, (size_t)g.ntrip * 3 * hp * hb, "contraction H store", true);
    for (int t = 0; t < g.ntrip; ++t)
        for (int h = 0; h < 3; ++h) {
            char* p = (char*)g.hbuf + ((int64_t)t * 3 + h) * hp * hb;
            if (hb == 8) *(double*)p = sig(g.trip[t], h);
            else *(float*)p = sig(g.trip[t], h);
        }
    const double fl = 12.0 * g.ntrip * (double)n * n * n * (g.o + g.v);
    if (mock::seconds_per_flop > 0)
        std::this_thread::sleep_for(std::chrono::duration<double>(fl * mock::seconds_per_flop));
}

void emu_epi(void** a) {
    const EpiLaunch e = *(const EpiLaunch*)a[0];
    const int prec = *(const int*)a[1];
    check_triples(e.trip, e.ntrip, e.o, "epilogue triple table");
    mock::check_range(e.orbits, (size_t)e.norbit * sizeof(int4), "epilogue orbit table", false);
    mock::check_range(e.partial, (size_t)e.ntrip * e.norbit * 8, "epilogue partials", true);
    mock::check_range(e.eps_o, (size_t)e.o * 8, "epilogue orbital energies (triples)", false);
    mock::check_range(e.eps_v, (size_t)e.v * 8, "epilogue orbital energies (tiles)", false);
    mock::check_range(e.t1, (size_t)e.o * e.v * 8, "epilogue t1", false);
    const int64_t last = (e.o - 1) * e.ovov_sp + (e.v - 1) * e.ovov_sx + (e.o - 1) * e.ovov_sq + (e.v - 1);
    mock::check_range(e.ovov, (size_t)(last + 1) * 8, "epilogue (ov|ov)", false);
    if (e.fock_ov) {
        mock::check_range(e.fock_ov, (size_t)e.o * e.v * 8, "epilogue f_ov", false);
        mock::check_range(e.t2, (size_t)e.o * e.o * e.v * e.v * 8, "epilogue t2", false);
    }
    const int hb = hbuf_bytes(prec);
    const int64_t hp = hpair_elems(e.v);
    mock::check_range(e.hbuf, (size_t)e.ntrip * 3 * hp * hb, "epilogue H read", false);
    for (int t = 0; t < e.ntrip; ++t) {
        const int4 tr = e.trip[t];
        for (int h = 0; h < 3; ++h) {
            const char* p = (const char*)e.hbuf + ((int64_t)t * 3 + h) * hp * hb;
            const float got = hb == 8 ? (float)*(const double*)p : *(const float*)p;
            if (got != sig(tr, h)) {
                std::fprintf(stderr, "MOCK-HIP FAULT: epilogue reads H of another triple or a stale batch: "
                             "triple (%d,%d,%d) pair %d holds %g\n", tr.x, tr.y, tr.z, h, (double)got);
                std::abort();
            }
        }
        const double val = tr.w / 3.0 * (1.0 + e.eps_o[tr.x] + e.eps_o[tr.y] + e.eps_o[tr.z]);
        for (int b = 0; b < e.norbit; ++b) e.partial[(int64_t)t * e.norbit + b] = b == 0 ? val : 0.0;
    }
}

void emu_red_trip(void** a) {
    const double* partial = *(const double* const*)a[0];
    const int ntrip = *(const int*)a[1], norbit = *(const int*)a[2];
    double* out = *(double* const*)a[4];
    mock::check_range(partial, (size_t)ntrip * norbit * 8, "per-triple sum partials", false);
    mock::check_range(out, (size_t)ntrip * 8, "per-triple sum output", true);
    for (int t = 0; t < ntrip; ++t) {
        double s = 0;
        for (int b = 0; b < norbit; ++b) s += partial[(int64_t)t * norbit + b];
        out[t] = s;
    }
}

void emu_red_total(void** a) {
    const double* e = *(const double* const*)a[0];
    const int64_t n = *(const int64_t*)a[1];
    double* out = *(double* const*)a[2];
    mock::check_range(e, (size_t)n * 8, "total sum input", false);
    mock::check_range(out, 8, "total sum output", true);
    double s = 0;
    for (int64_t t = 0; t < n; ++t) s += e[t];
    *out = s;
}

// Grouped launches: each entry is emulated as the single launch it stands for.
void emu_gemm_group(void** a) {
    const GemmGroupEntry* ent = *(const GemmGroupEntry* const*)a[0];
    const int nent = *(const int*)a[1], prec = *(const int*)a[2];
    mock::check_range(ent, (size_t)nent * sizeof(GemmGroupEntry), "grouped contraction entries", false);
    int64_t wg = 0;
    for (int e = 0; e < nent; ++e) {
        if (ent[e].wg0 != wg) {
            std::fprintf(stderr, "MOCK-HIP FAULT: grouped contraction entry %d starts at %d, not %lld\n", e,
                         ent[e].wg0, (long long)wg);
            std::abort();
        }
        wg += (int64_t)ent[e].g.ntrip * 3 * ent[e].g.v * ent[e].ntile_u * ent[e].ntile_w;
        GemmLaunch g = ent[e].g;
        int form = FORM_OCC;
        void* args[3] = {&g, (void*)&prec, &form};
        emu_gemm(args);
    }
}

void emu_epi_group(void** a) {
    const EpiGroupEntry* ent = *(const EpiGroupEntry* const*)a[0];
    const int nent = *(const int*)a[1], prec = *(const int*)a[2];
    mock::check_range(ent, (size_t)nent * sizeof(EpiGroupEntry), "grouped epilogue entries", false);
    for (int e = 0; e < nent; ++e) {
        EpiLaunch x = ent[e].e;
        int p = prec;
        void* args[2] = {&x, &p};
        emu_epi(args);
    }
}

void emu_red_trip_group(void** a) {
    const RedGroupEntry* ent = *(const RedGroupEntry* const*)a[0];
    const int nent = *(const int*)a[1];
    mock::check_range(ent, (size_t)nent * sizeof(RedGroupEntry), "grouped per-triple sum entries", false);
    for (int e = 0; e < nent; ++e) {
        const int ntrip = (e + 1 < nent ? ent[e + 1].b0 : *(const int*)a[2]) - ent[e].b0;
        const double* partial = ent[e].partial;
        int nt = ntrip, nb = ent[e].norbit;
        const int4* trip = ent[e].trip;
        double* out = ent[e].e_trip;
        void* args[5] = {&partial, &nt, &nb, &trip, &out};
        emu_red_trip(args);
    }
}

void emu_red_total_group(void** a) {
    const TotalGroupEntry* ent = *(const TotalGroupEntry* const*)a[0];
    const int nent = *(const int*)a[1];
    mock::check_range(ent, (size_t)nent * sizeof(TotalGroupEntry), "grouped total entries", false);
    for (int e = 0; e < nent; ++e) {
        const double* x = ent[e].e_trip;
        int64_t n = ent[e].n;
        double* out = ent[e].out;
        void* args[3] = {&x, &n, &out};
        emu_red_total(args);
    }
}

struct Registrar {
    Registrar() {
        mock::register_kernel(&k_gemm_group, {sizeof(void*), sizeof(int), sizeof(int)}, emu_gemm_group);
        mock::register_kernel(&k_epi_group, {sizeof(void*), sizeof(int), sizeof(int)}, emu_epi_group);
        mock::register_kernel(&k_red_trip_group, {sizeof(void*), sizeof(int), sizeof(int)}, emu_red_trip_group);
        mock::register_kernel(&k_red_total_group, {sizeof(void*), sizeof(int)}, emu_red_total_group);
        mock::register_kernel(&k_gemm, {sizeof(GemmLaunch), sizeof(int), sizeof(int)}, emu_gemm);
        mock::register_kernel(&k_epi, {sizeof(EpiLaunch), sizeof(int)}, emu_epi);
        mock::register_kernel(&k_red_trip, {sizeof(void*), sizeof(int), sizeof(int), sizeof(void*), sizeof(void*)},
                              emu_red_trip);
        mock::register_kernel(&k_red_total, {sizeof(void*), sizeof(int64_t), sizeof(void*)}, emu_red_total);
    }
} g_registrar;

}  // namespace

void launch_prepare(int precision, const DevInputs& in, void* ws, Operands* ops, hipStream_t st, int form) {
    const int o = in.o, v = in.v;
    const int n = form == FORM_VIR ? o : v;
    const Sizes z = factor_sizes(o, v, precision);
    const int eb = operand_bytes(precision);
    char* p = (char*)ws;
    ops->ovvv = p; p += a256((size_t)z.m_ovvv * n * z.Kv * eb);
    ops->t2 = p;   p += a256((size_t)z.m_t2 * n * z.Kv * eb);
    ops->t2l = p;  p += a256((size_t)z.m_t2l * n * z.Ko * eb);
    ops->hoo = p;
    ops->Kv = z.Kv;
    ops->Ko = z.Ko;
    const size_t bytes = (size_t)prepare_bytes(precision, o, v);
    mock::submit(st, [=] {
        mock::check_range(ws, bytes, "precision conversion output", true);
        mock::check_range(in.eps_o, (size_t)o * 8, "conversion eps_o", false);
        mock::check_range(in.t2, (size_t)o * o * v * v * 8, "conversion t2", false);
        mock::check_range(in.ooov, (size_t)o * o * o * v * 8, "conversion (oo|ov)", false);
        if (in.ovvv) mock::check_range(in.ovvv, (size_t)o * v * v * v * 8, "conversion (ov|vv)", false);
    });
}

VirAux launch_vir_aux(const DevInputs& in, void* aux, hipStream_t st) {
    const int o = in.o, v = in.v;
    const int64_t ov = (int64_t)o * v;
    char* p = (char*)aux;
    VirAux x;
    x.neg_eps_v = (double*)p; p += a256(v * 8);
    x.neg_eps_o = (double*)p; p += a256(o * 8);
    x.t1_t = (double*)p;      p += a256(ov * 8);
    x.ovov_t = (double*)p;    p += a256(ov * ov * 8);
    if (in.fock_ov) {
        x.t2_t = (double*)p;   p += a256(ov * ov * 8);
        x.fock_t = (double*)p;
    }
    const size_t bytes = (size_t)vir_aux_bytes(o, v, in.fock_ov != nullptr);
    mock::submit(st, [=] {
        mock::check_range(aux, bytes, "virtual-loop transposes", true);
        mock::check_range(in.eps_v, (size_t)v * 8, "transpose eps_v", false);
        mock::check_range(in.eps_o, (size_t)o * 8, "transpose eps_o", false);
        for (int a = 0; a < v; ++a) x.neg_eps_v[a] = -in.eps_v[a];
        for (int i = 0; i < o; ++i) x.neg_eps_o[i] = -in.eps_o[i];
    });
    return x;
}

KernelCall gemm_call(int precision, const GemmLaunch& g, int form) {
    KernelCall k;
    k.fn = &k_gemm;
    k.arg(g).arg(precision).arg(form);
    return k;
}

KernelCall epilogue_call(int precision, const EpiLaunch& e) {
    KernelCall k;
    k.fn = &k_epi;
    k.arg(e).arg(precision);
    return k;
}

KernelCall reduce_triples_call(const double* partial, int ntrip, int norbit, const int4* trip, double* e_trip) {
    KernelCall k;
    k.fn = &k_red_trip;
    k.arg(partial).arg(ntrip).arg(norbit).arg(trip).arg(e_trip);
    return k;
}

KernelCall reduce_total_call(const double* e_trip, int64_t n, double* out) {
    KernelCall k;
    k.fn = &k_red_total;
    k.arg(e_trip).arg(n).arg(out);
    return k;
}

int wave_blocks(int, int) { return 5; }

void launch_prepare_group(int precision, int n, const DevInputs* ins, void* const* ws, Operands* ops,
                          FactorGroupEntry* d_tables, std::vector<FactorGroupEntry>& tables, hipStream_t st) {
    tables.assign((size_t)4 * n, FactorGroupEntry{});
    for (int f = 0; f < n; ++f) launch_prepare(precision, ins[f], ws[f], &ops[f], st, FORM_OCC);
    mock::submit(st, [=] { mock::check_range(d_tables, (size_t)4 * n * sizeof(FactorGroupEntry), "factor tables", true); });
}

KernelCall gemm_group_call(int precision, int wb, const GemmGroupEntry* d_ent, int nent, int64_t n_wg) {
    (void)wb;
    (void)n_wg;
    KernelCall k;
    k.fn = &k_gemm_group;
    k.arg(d_ent).arg(nent).arg(precision);
    return k;
}

KernelCall epilogue_group_call(int precision, const EpiGroupEntry* d_ent, int nent, int64_t n_wg) {
    (void)n_wg;
    KernelCall k;
    k.fn = &k_epi_group;
    k.arg(d_ent).arg(nent).arg(precision);
    return k;
}

KernelCall reduce_triples_group_call(const RedGroupEntry* d_ent, int nent, int nblocks) {
    KernelCall k;
    k.fn = &k_red_trip_group;
    k.arg(d_ent).arg(nent).arg(nblocks);
    return k;
}

KernelCall reduce_total_group_call(const TotalGroupEntry* d_ent, int nent) {
    KernelCall k;
    k.fn = &k_red_total_group;
    k.arg(d_ent).arg(nent);
    return k;
}

// MP2 is not exercised by these drivers.
int64_t mp2_workspace_bytes(int, int) { return 256; }
double* enqueue_mp2(int, int, int, const double*, const double*, const double*, void*, hipStream_t, double**) {
    std::fprintf(stderr, "MOCK-HIP FAULT: MP2 is not emulated\n");
    std::abort();
}

}  // namespace bqc
