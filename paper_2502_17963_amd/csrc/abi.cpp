// extern "C" entry points of include/bqc.h: argument validation, device
// context pool, host<->device copies and error translation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bqc.h"
#include "bqc_internal.h"

namespace bqc {


thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

// Validates sizes, pointers, finiteness of the orbital energies and the gap.
int validate(int32_t nocc, int32_t nvir, const double* eps_o, const double* eps_v, const double* t1,
             const double* t2, const double* ovvv, const double* ooov, const double* ovov,
             bool host_eps) {
    if (nocc < 1 || nvir < 1) return fail(BQC_EINVAL, "nocc and nvir must be >= 1");
    if (nocc > 4096 || nvir > 8192) return fail(BQC_EINVAL, "nocc or nvir beyond the supported range");
    if (!eps_o || !eps_v || !t1 || !t2 || !ovvv || !ooov || !ovov)
        return fail(BQC_EINVAL, "null input pointer");
    if (!host_eps) return BQC_OK;
    double omax = -INFINITY, vmin = INFINITY;
    for (int i = 0; i < nocc; ++i) {
        if (!std::isfinite(eps_o[i])) return fail(BQC_EINVAL, "non-finite occupied orbital energy");
        omax = std::max(omax, eps_o[i]);
    }
    for (int a = 0; a < nvir; ++a) {
        if (!std::isfinite(eps_v[a])) return fail(BQC_EINVAL, "non-finite virtual orbital energy");
        vmin = std::min(vmin, eps_v[a]);
    }
    if (!(omax < vmin)) return fail(BQC_EINVAL, "gap condition max(eps_o) < min(eps_v) violated");
    return BQC_OK;
}

// ------------------------------------------------------------------ context pool
struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;  // epilogue stream of the two-stream pipeline
    void* ws = nullptr;
    size_t ws_size = 0;
    void* in = nullptr;
    size_t in_size = 0;
    double* host_energy = nullptr;  // pinned 8 bytes
    void* df_tmp = nullptr;         // FP64 scratch of the density-fitting product
    size_t df_tmp_size = 0;
    bool busy = false;
};

std::mutex g_pool_mu;
std::vector<Ctx*> g_pool;

Ctx* acquire_ctx(int device) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (Ctx* c : g_pool)
        if (!c->busy && c->device == device) { c->busy = true; return c; }
    Ctx* c = new Ctx();
    c->device = device;
    c->busy = true;
    g_pool.push_back(c);
    return c;
}
void release_ctx(Ctx* c) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    c->busy = false;
}

void ensure(void*& p, size_t& have, size_t need) {
    if (have >= need && p) return;
    if (p) { BQC_HIP(hipFree(p)); p = nullptr; have = 0; }
    BQC_HIP(hipMalloc(&p, std::max<size_t>(need, 256)));
    have = std::max<size_t>(need, 256);
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        BQC_HIP(hipGetDevice(&prev));
        if (prev != dev) BQC_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// One solve.  df = false: (ia|bc) is the input ovvv; df = true: it is formed
// on the device from the density-fitting factors b_ov, b_vv (naux of them).
int solve_impl(int32_t o, int32_t v, const double* eps_o, const double* eps_v, const double* t1,
               const double* t2, const double* ovvv, const double* ooov, const double* ovov,
               const bqc_t_opts* opts, double* E_T, bqc_t_stats* stats, bool df = false,
               int32_t naux = 0, const double* b_ov = nullptr, const double* b_vv = nullptr) {
    bqc_t_opts op;
    std::memset(&op, 0, sizeof(op));
    if (opts) op = *opts;
    if (!E_T) return fail(BQC_EINVAL, "E_T is null");
    if (op.precision < 0 || op.precision > 3) return fail(BQC_EINVAL, "unknown precision");
    if (op.formulation != BQC_FORM_OCCUPIED && op.formulation != BQC_FORM_VIRTUAL)
        return fail(BQC_EINVAL, "unknown formulation");
    const int form = op.formulation == BQC_FORM_VIRTUAL ? FORM_VIR : FORM_OCC;
    if (form == FORM_VIR && op.precision == BQC_PREC_FP8)
        return fail(BQC_EINVAL, "the virtual-triple formulation runs in FP64, FP32 or split-BF16x3");
    const bool dev_in = op.inputs_on_device != 0;
    if (df && (naux < 1 || !b_ov || !b_vv))
        return fail(BQC_EINVAL, "density fitting needs naux >= 1 and non-null b_ov, b_vv");
    int rc = validate(o, v, eps_o, eps_v, t1, t2, df ? b_ov : ovvv, ooov, ovov, !dev_in);
    if (rc != BQC_OK) return rc;
    if (op.fock_ov && !dev_in)
        for (int64_t a = 0; a < (int64_t)o * v; ++a)
            if (!std::isfinite(op.fock_ov[a])) return fail(BQC_EINVAL, "non-finite fock_ov element");
    const int64_t ntrip_all = num_triples(form == FORM_VIR ? v : o);
    if (ntrip_all > (int64_t)INT32_MAX)
        return fail(BQC_EINVAL, "more unique triples than one solve supports (2^31 - 1)");
    if (op.triple_end == 0 ? op.triple_begin != 0
                           : (op.triple_begin < 0 || op.triple_begin >= op.triple_end || op.triple_end > ntrip_all))
        return fail(BQC_EINVAL, "triple range outside [0, number of unique triples] or empty");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BQC_EDEVICE, "no HIP device");
    if (op.device < 0 || op.device >= ndev) return fail(BQC_EINVAL, "device ordinal out of range");

    auto wall0 = std::chrono::steady_clock::now();
    DeviceGuard dg(op.device);
    Ctx* ctx = acquire_ctx(op.device);
    struct Rel { Ctx* c; ~Rel() { release_ctx(c); } } rel{ctx};
    if (!ctx->stream) BQC_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    if (!ctx->side) BQC_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    if (!ctx->host_energy) BQC_HIP(hipHostMalloc((void**)&ctx->host_energy, 256, hipHostMallocDefault));
    hipStream_t st = op.stream ? (hipStream_t)op.stream : ctx->stream;

    if (dev_in) {  // check the orbital energies from a host copy
        std::vector<double> eo(o), evv(v);
        BQC_HIP(hipMemcpyAsync(eo.data(), eps_o, o * sizeof(double), hipMemcpyDeviceToHost, st));
        BQC_HIP(hipMemcpyAsync(evv.data(), eps_v, v * sizeof(double), hipMemcpyDeviceToHost, st));
        BQC_HIP(hipStreamSynchronize(st));
        rc = validate(o, v, eo.data(), evv.data(), t1, t2, df ? b_ov : ovvv, ooov, ovov, true);
        if (rc != BQC_OK) return rc;
    }

    // inputs: eps_o, eps_v, t1, t2, [ovvv | b_ov, b_vv], ooov, ovov
    std::vector<const double*> src = {eps_o, eps_v, t1, t2};
    std::vector<size_t> sizes = {(size_t)o, (size_t)v, (size_t)o * v, (size_t)o * o * v * v};
    if (df) {
        src.push_back(b_ov); sizes.push_back((size_t)naux * o * v);
        src.push_back(b_vv); sizes.push_back((size_t)naux * v * v);
    } else {
        src.push_back(ovvv); sizes.push_back((size_t)o * v * v * v);
    }
    src.push_back(ooov); sizes.push_back((size_t)o * o * o * v);
    src.push_back(ovov); sizes.push_back((size_t)o * v * o * v);
    if (op.fock_ov) { src.push_back(op.fock_ov); sizes.push_back((size_t)o * v); }
    std::vector<const double*> dst(src.size());
    double upload_s = 0.0;
    size_t in_bytes = 0;
    if (dev_in) {
        dst = src;
    } else {
        for (size_t s : sizes) in_bytes += a256(s * sizeof(double));
        ensure(ctx->in, ctx->in_size, in_bytes);
        char* p = (char*)ctx->in;
        auto u0 = std::chrono::steady_clock::now();
        for (size_t a = 0; a < src.size(); ++a) {
            BQC_HIP(hipMemcpyAsync(p, src[a], sizes[a] * sizeof(double), hipMemcpyHostToDevice, st));
            dst[a] = (const double*)p;
            p += a256(sizes[a] * sizeof(double));
        }
        BQC_HIP(hipStreamSynchronize(st));
        upload_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - u0).count();
    }
    DevInputs in;
    in.o = o;
    in.v = v;
    in.eps_o = dst[0]; in.eps_v = dst[1]; in.t1 = dst[2]; in.t2 = dst[3];
    if (df) {
        in.b_ov = dst[4]; in.b_vv = dst[5]; in.naux = naux;
        in.ooov = dst[6]; in.ovov = dst[7];
        ensure(ctx->df_tmp, ctx->df_tmp_size, (size_t)df_scratch_elems(o, v) * sizeof(double));
        in.df_tmp = (double*)ctx->df_tmp;
        in.df_block = df_block_planes(o, v);
    } else {
        in.ovvv = dst[4]; in.ooov = dst[5]; in.ovov = dst[6];
    }
    if (op.fock_ov) in.fock_ov = dst.back();

    const Plan plan = make_plan(o, v, op.precision, op.triple_begin, op.triple_end, form);
    const int64_t nshare = plan.end - plan.begin;
    ensure(ctx->ws, ctx->ws_size, (size_t)workspace_bytes(o, v, op.precision, form, op.fock_ov != nullptr));
    SolveStats ss;
    enqueue_solve(plan, in, ctx->ws, nullptr, st, ctx->side, op.timing != 0, stats ? &ss : nullptr);
    BQC_HIP(hipMemcpyAsync(ctx->host_energy, workspace_energy(ctx->ws, o, v, op.precision, form), sizeof(double),
                           hipMemcpyDeviceToHost, st));
    std::vector<double> etrip;
    if (op.triple_energies && nshare > 0) {
        etrip.resize(nshare);
        BQC_HIP(hipMemcpyAsync(etrip.data(), workspace_etrip(ctx->ws, o, v, op.precision, form) + plan.begin,
                               nshare * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    BQC_HIP(hipStreamSynchronize(st));
    const double e = *ctx->host_energy;
    if (!std::isfinite(e)) return fail(BQC_EDEVICE, "non-finite energy (device arithmetic failed)");
    *E_T = e;
    if (op.triple_energies && nshare > 0)
        std::memcpy(op.triple_energies + plan.begin, etrip.data(), nshare * sizeof(double));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->upload_s = upload_s;
        stats->prepare_s = ss.prepare_s;
        stats->gpu_s = ss.gpu_s;
        stats->gemm_s = ss.gemm_s;
        stats->epilogue_s = ss.epi_s;
        stats->gemm_launches = ss.gemm_launches;
        stats->epilogue_launches = ss.epi_launches;
        stats->footprint_bytes = ss.footprint + in_bytes +
                                 (df ? (uint64_t)df_scratch_elems(o, v) * sizeof(double) : 0);
        // per unique triple: 3 pairs x n planes x n^2 outputs x 2 (2v + 2o), n = tile space
        const double nt = form == FORM_VIR ? o : v;
        stats->flops = 12.0 * (double)nshare * nt * nt * nt * (double)(v + o);
        stats->precision = op.precision;
        stats->n_triples = (int32_t)nshare;
        stats->total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
    }
    return BQC_OK;
}

// Several fragments in one batched solve (batch.hip).
int batch_impl(int32_t nfrag, const bqc_t_fragment* frags, const bqc_t_opts* opts, double* E_T, bqc_t_stats* stats) {
    bqc_t_opts op;
    std::memset(&op, 0, sizeof(op));
    if (opts) op = *opts;
    if (nfrag < 0 || (nfrag > 0 && (!frags || !E_T))) return fail(BQC_EINVAL, "nfrag < 0, or null frags / E_T");
    if (nfrag > (1 << 20)) return fail(BQC_EINVAL, "more fragments than one batch supports (2^20)");
    if (op.precision < 0 || op.precision > 3) return fail(BQC_EINVAL, "unknown precision");
    if (op.formulation != BQC_FORM_OCCUPIED)
        return fail(BQC_EINVAL, "a batch runs the loop over occupied triples");
    if (op.triple_begin != 0 || op.triple_end != 0 || op.fock_ov || op.triple_energies)
        return fail(BQC_EINVAL, "a batch takes no triple range, f_ov block or per-triple output");
    const bool dev_in = op.inputs_on_device != 0;
    for (int32_t f = 0; f < nfrag; ++f) {
        const bqc_t_fragment& x = frags[f];
        const int rc = validate(x.nocc, x.nvir, x.eps_o, x.eps_v, x.t1, x.t2, x.ovvv, x.ooov, x.ovov, !dev_in);
        if (rc != BQC_OK) return fail(rc, "fragment " + std::to_string(f) + ": " + g_last_error);
    }
    if (nfrag == 0) return BQC_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BQC_EDEVICE, "no HIP device");
    if (op.device < 0 || op.device >= ndev) return fail(BQC_EINVAL, "device ordinal out of range");
    auto wall0 = std::chrono::steady_clock::now();
    DeviceGuard dg(op.device);
    Ctx* ctx = acquire_ctx(op.device);
    struct Rel { Ctx* c; ~Rel() { release_ctx(c); } } rel{ctx};
    if (!ctx->stream) BQC_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    hipStream_t st = op.stream ? (hipStream_t)op.stream : ctx->stream;
    std::vector<const double*> src((size_t)7 * nfrag);
    for (int32_t f = 0; f < nfrag; ++f) {
        const bqc_t_fragment& x = frags[f];
        const double* a[7] = {x.eps_o, x.eps_v, x.t1, x.t2, x.ovvv, x.ooov, x.ovov};
        for (int k = 0; k < 7; ++k) src[(size_t)7 * f + k] = a[k];
    }
    if (dev_in) {  // check the orbital energies from host copies
        for (int32_t f = 0; f < nfrag; ++f) {
            const bqc_t_fragment& x = frags[f];
            std::vector<double> eo(x.nocc), ev(x.nvir);
            BQC_HIP(hipMemcpyAsync(eo.data(), x.eps_o, x.nocc * sizeof(double), hipMemcpyDeviceToHost, st));
            BQC_HIP(hipMemcpyAsync(ev.data(), x.eps_v, x.nvir * sizeof(double), hipMemcpyDeviceToHost, st));
            BQC_HIP(hipStreamSynchronize(st));
            const int rc = validate(x.nocc, x.nvir, eo.data(), ev.data(), x.t1, x.t2, x.ovvv, x.ooov, x.ovov, true);
            if (rc != BQC_OK) return fail(rc, "fragment " + std::to_string(f) + ": " + g_last_error);
        }
    }
    // inputs: device pointers as given, or uploaded into one buffer
    std::vector<const double*> dst = src;
    double upload_s = 0.0;
    size_t in_bytes = 0;
    if (!dev_in) {
        for (int32_t f = 0; f < nfrag; ++f) in_bytes += a256((size_t)input_bytes(frags[f].nocc, frags[f].nvir));
        ensure(ctx->in, ctx->in_size, in_bytes);
        char* p = (char*)ctx->in;
        const auto u0 = std::chrono::steady_clock::now();
        for (int32_t f = 0; f < nfrag; ++f) {
            const int o = frags[f].nocc, v = frags[f].nvir;
            const size_t sizes[7] = {(size_t)o, (size_t)v, (size_t)o * v, (size_t)o * o * v * v,
                                     (size_t)o * v * v * v, (size_t)o * o * o * v, (size_t)o * v * o * v};
            char* q = p;
            for (int k = 0; k < 7; ++k) {
                BQC_HIP(hipMemcpyAsync(q, src[(size_t)7 * f + k], sizes[k] * sizeof(double), hipMemcpyHostToDevice,
                                       st));
                dst[(size_t)7 * f + k] = (const double*)q;
                q += a256(sizes[k] * sizeof(double));
            }
            p += a256((size_t)input_bytes(o, v));
        }
        BQC_HIP(hipStreamSynchronize(st));
        upload_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - u0).count();
    }
    std::vector<DevInputs> ins(nfrag);
    std::vector<int> no(nfrag), nv(nfrag);
    for (int32_t f = 0; f < nfrag; ++f) {
        DevInputs& in = ins[f];
        in.o = no[f] = frags[f].nocc;
        in.v = nv[f] = frags[f].nvir;
        in.eps_o = dst[(size_t)7 * f]; in.eps_v = dst[(size_t)7 * f + 1]; in.t1 = dst[(size_t)7 * f + 2];
        in.t2 = dst[(size_t)7 * f + 3]; in.ovvv = dst[(size_t)7 * f + 4]; in.ooov = dst[(size_t)7 * f + 5];
        in.ovov = dst[(size_t)7 * f + 6];
    }
    const BatchPlan bp = plan_batch(nfrag, no.data(), nv.data(), op.precision);
    ensure(ctx->ws, ctx->ws_size, bp.total);
    std::vector<double> e(nfrag);
    SolveStats ss;
    enqueue_batch(bp, op.precision, nfrag, ins.data(), ctx->ws, st, e.data(), stats ? &ss : nullptr);
    for (int32_t f = 0; f < nfrag; ++f)
        if (!std::isfinite(e[f])) return fail(BQC_EDEVICE, "non-finite energy of fragment " + std::to_string(f));
    std::memcpy(E_T, e.data(), nfrag * sizeof(double));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        double flops = 0;
        int64_t ntrip = 0;
        for (int32_t f = 0; f < nfrag; ++f) {
            const double v = frags[f].nvir;
            flops += 12.0 * (double)num_triples(frags[f].nocc) * v * v * v * (v + frags[f].nocc);
            ntrip += num_triples(frags[f].nocc);
        }
        stats->upload_s = upload_s;
        stats->gpu_s = ss.gpu_s;
        stats->flops = flops;
        stats->footprint_bytes = bp.total + in_bytes;
        stats->gemm_launches = ss.gemm_launches;
        stats->epilogue_launches = ss.epi_launches;
        stats->precision = op.precision;
        stats->n_triples = (int32_t)std::min<int64_t>(ntrip, INT32_MAX);
        stats->total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
    }
    return BQC_OK;
}

// MP2 energy (density-fitted): validation, residency, one enqueue_mp2.
int mp2_impl(int32_t o, int32_t v, int32_t naux, const double* eps_o, const double* eps_v, const double* b_ov,
             const bqc_t_opts* opts, double* E, bqc_t_stats* stats) {
    bqc_t_opts op;
    std::memset(&op, 0, sizeof(op));
    if (opts) op = *opts;
    if (!E) return fail(BQC_EINVAL, "E_MP2 is null");
    if (o < 1 || v < 1 || naux < 1) return fail(BQC_EINVAL, "nocc, nvir and naux must be >= 1");
    if (!eps_o || !eps_v || !b_ov) return fail(BQC_EINVAL, "null input pointer");
    if (op.precision != BQC_PREC_FP64) return fail(BQC_EINVAL, "MP2 runs in FP64 only");
    const bool dev_in = op.inputs_on_device != 0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BQC_EDEVICE, "no HIP device");
    if (op.device < 0 || op.device >= ndev) return fail(BQC_EINVAL, "device ordinal out of range");
    auto wall0 = std::chrono::steady_clock::now();
    DeviceGuard dg(op.device);
    Ctx* ctx = acquire_ctx(op.device);
    struct Rel { Ctx* c; ~Rel() { release_ctx(c); } } rel{ctx};
    if (!ctx->stream) BQC_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    if (!ctx->host_energy) BQC_HIP(hipHostMalloc((void**)&ctx->host_energy, 256, hipHostMallocDefault));
    hipStream_t st = op.stream ? (hipStream_t)op.stream : ctx->stream;
    std::vector<double> eo(o), ev(v);
    if (dev_in) {
        BQC_HIP(hipMemcpyAsync(eo.data(), eps_o, o * sizeof(double), hipMemcpyDeviceToHost, st));
        BQC_HIP(hipMemcpyAsync(ev.data(), eps_v, v * sizeof(double), hipMemcpyDeviceToHost, st));
        BQC_HIP(hipStreamSynchronize(st));
    } else {
        std::memcpy(eo.data(), eps_o, o * sizeof(double));
        std::memcpy(ev.data(), eps_v, v * sizeof(double));
    }
    double omax = -INFINITY, vmin = INFINITY;
    for (double x : eo) { if (!std::isfinite(x)) return fail(BQC_EINVAL, "non-finite occupied orbital energy"); omax = std::max(omax, x); }
    for (double x : ev) { if (!std::isfinite(x)) return fail(BQC_EINVAL, "non-finite virtual orbital energy"); vmin = std::min(vmin, x); }
    if (!(omax < vmin)) return fail(BQC_EINVAL, "no gap: max eps_o >= min eps_v");

    const double* d_eo = eps_o;
    const double* d_ev = eps_v;
    const double* d_b = b_ov;
    double upload_s = 0.0;
    size_t in_bytes = 0;
    if (!dev_in) {
        const size_t nb = (size_t)naux * o * v;
        in_bytes = a256(o * sizeof(double)) + a256(v * sizeof(double)) + a256(nb * sizeof(double));
        ensure(ctx->in, ctx->in_size, in_bytes);
        char* p = (char*)ctx->in;
        const auto u0 = std::chrono::steady_clock::now();
        BQC_HIP(hipMemcpyAsync(p, eps_o, o * sizeof(double), hipMemcpyHostToDevice, st));
        d_eo = (const double*)p; p += a256(o * sizeof(double));
        BQC_HIP(hipMemcpyAsync(p, eps_v, v * sizeof(double), hipMemcpyHostToDevice, st));
        d_ev = (const double*)p; p += a256(v * sizeof(double));
        BQC_HIP(hipMemcpyAsync(p, b_ov, nb * sizeof(double), hipMemcpyHostToDevice, st));
        d_b = (const double*)p;
        BQC_HIP(hipStreamSynchronize(st));
        upload_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - u0).count();
    }
    ensure(ctx->ws, ctx->ws_size, (size_t)mp2_workspace_bytes(o, v));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
        BQC_HIP(hipEventCreate(&e0));
        BQC_HIP(hipEventCreate(&e1));
        BQC_HIP(hipEventRecord(e0, st));
    }
    struct Ev { hipEvent_t a, b; ~Ev() { if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); } } evg{e0, e1};
    double* d_pair = nullptr;
    double* d_e = enqueue_mp2(o, v, naux, d_eo, d_ev, d_b, ctx->ws, st, &d_pair);
    if (stats) BQC_HIP(hipEventRecord(e1, st));
    BQC_HIP(hipMemcpyAsync(ctx->host_energy, d_e, sizeof(double), hipMemcpyDeviceToHost, st));
    const int64_t npair = (int64_t)o * (o + 1) / 2;
    std::vector<double> pairs;
    if (op.triple_energies) {
        pairs.resize(npair);
        BQC_HIP(hipMemcpyAsync(pairs.data(), d_pair, npair * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    BQC_HIP(hipStreamSynchronize(st));
    const double e = *ctx->host_energy;
    if (!std::isfinite(e)) return fail(BQC_EDEVICE, "non-finite energy (device arithmetic failed)");
    *E = e;
    if (op.triple_energies) std::memcpy(op.triple_energies, pairs.data(), npair * sizeof(double));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        float ms = 0;
        BQC_HIP(hipEventElapsedTime(&ms, e0, e1));
        stats->gpu_s = ms * 1e-3;
        stats->upload_s = upload_s;
        stats->flops = (double)o * (o + 1) / 2.0 * 2.0 * (double)v * v * naux;
        stats->footprint_bytes = (uint64_t)mp2_workspace_bytes(o, v) + in_bytes;
        stats->precision = BQC_PREC_FP64;
        stats->total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
    }
    return BQC_OK;
}

template <typename F>
int guarded(F&& f) {
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

}  // namespace bqc

using namespace bqc;

extern "C" {

int bqc_t_energy(int32_t nocc, int32_t nvir, const double* eps_o, const double* eps_v,
                 const double* t1, const double* t2, const double* ovvv, const double* ooov,
                 const double* ovov, double* E_T) {
    return guarded([&] {
        return solve_impl(nocc, nvir, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, nullptr, E_T, nullptr);
    });
}

int bqc_t_energy_ex(int32_t nocc, int32_t nvir, const double* eps_o, const double* eps_v,
                    const double* t1, const double* t2, const double* ovvv, const double* ooov,
                    const double* ovov, const bqc_t_opts* opts, double* E_T, bqc_t_stats* stats) {
    return guarded([&] {
        return solve_impl(nocc, nvir, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, opts, E_T, stats);
    });
}

int bqc_t_energy_df(int32_t nocc, int32_t nvir, int32_t naux, const double* eps_o, const double* eps_v,
                    const double* t1, const double* t2, const double* b_ov, const double* b_vv,
                    const double* ooov, const double* ovov, const bqc_t_opts* opts, double* E_T,
                    bqc_t_stats* stats) {
    return guarded([&] {
        if (!b_ov || !b_vv || naux < 1)
            return fail(BQC_EINVAL, "density fitting needs naux >= 1 and non-null b_ov, b_vv");
        return solve_impl(nocc, nvir, eps_o, eps_v, t1, t2, nullptr, ooov, ovov, opts, E_T, stats, true, naux,
                          b_ov, b_vv);
    });
}

int bqc_mp2_energy_df(int32_t nocc, int32_t nvir, int32_t naux, const double* eps_o, const double* eps_v,
                      const double* b_ov, const bqc_t_opts* opts, double* E_MP2, bqc_t_stats* stats) {
    return guarded([&] { return mp2_impl(nocc, nvir, naux, eps_o, eps_v, b_ov, opts, E_MP2, stats); });
}

int bqc_t_energy_batch(int32_t nfrag, const bqc_t_fragment* frags, const bqc_t_opts* opts, double* E_T,
                       bqc_t_stats* stats) {
    return guarded([&] { return batch_impl(nfrag, frags, opts, E_T, stats); });
}

int64_t bqc_t_batch_footprint(int32_t nfrag, const int32_t* nocc, const int32_t* nvir, int32_t precision) {
    if (nfrag < 0 || (nfrag > 0 && (!nocc || !nvir)) || precision < 0 || precision > 3) return -1;
    std::vector<int> o(nfrag), v(nfrag);
    int64_t in = 0;
    for (int32_t f = 0; f < nfrag; ++f) {
        if (nocc[f] < 1 || nvir[f] < 1) return -1;
        o[f] = nocc[f];
        v[f] = nvir[f];
        in += (int64_t)a256((size_t)input_bytes(o[f], v[f]));
    }
    return (int64_t)plan_batch(nfrag, o.data(), v.data(), precision).total + in;
}

int64_t bqc_t_num_triples(int32_t nocc) { return num_triples(nocc); }

int64_t bqc_t_footprint(int32_t nocc, int32_t nvir, int32_t precision) {
    if (nocc < 1 || nvir < 1 || precision < 0 || precision > 3) return -1;
    return workspace_bytes(nocc, nvir, precision) + input_bytes(nocc, nvir);
}

int64_t bqc_t_footprint_ex(int32_t nocc, int32_t nvir, int32_t precision, int32_t formulation, int32_t fock) {
    if (nocc < 1 || nvir < 1 || precision < 0 || precision > 3) return -1;
    if (formulation != BQC_FORM_OCCUPIED && formulation != BQC_FORM_VIRTUAL) return -1;
    const int form = formulation == BQC_FORM_VIRTUAL ? FORM_VIR : FORM_OCC;
    if (form == FORM_VIR && precision == BQC_PREC_FP8) return -1;
    int64_t in = input_bytes(nocc, nvir);
    if (fock) in += (int64_t)nocc * nvir * 8 + 256;
    return workspace_bytes(nocc, nvir, precision, form, fock != 0) + in;
}

const char* bqc_last_error(void) { return g_last_error.c_str(); }

int32_t bqc_version(void) { return 200; }

int bqc_hip_versions(int32_t* compiled, int32_t* runtime) {
    if (compiled) *compiled = HIP_VERSION;
    if (!runtime) return BQC_OK;
    int rv = 0;
    if (hipRuntimeGetVersion(&rv) != hipSuccess) return fail(BQC_EDEVICE, "hipRuntimeGetVersion failed");
    *runtime = rv;
    return BQC_OK;
}

}  // extern "C"
