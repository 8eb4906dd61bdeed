// bqc_t_energy_noalloc: the solve of bqc_t_energy_ex with device-resident
// inputs, for callers that cannot allocate device memory.  Its workspace is a
// file-scope device array (`scratch`, BQC_NOALLOC_SCRATCH_BYTES bytes per
// device, held by the library until the process ends); nothing here calls
// hipMalloc, hipFree, an event or stream constructor, or any other routine
// that allocates device memory.
//
// The launch sequence is the library's (precision conversion of the inputs,
// then per batch of triples: contraction, fused epilogue, per-triple
// fixed-order sum; then the fixed-order sum over triples), run in order on
// the caller's stream with one H buffer, and with the triple and tile-orbit
// tables written by a kernel instead of copied from the host.  A triple's
// energy and the order of every sum do not depend on the batch size, so the
// result equals bqc_t_energy_ex's bit for bit.
//
// Every call on a device shares that device's array: calls that overlap on
// one device race.  Nothing in the array needs to start at zero: every
// element a kernel reads was written earlier in the same call (the operand
// padding included), except H elements with an index past the tile space,
// which the epilogue masks.
#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/bqc.h"
#include "bqc_internal.h"

namespace bqc {

int fail(int code, const std::string& msg);
int validate(int32_t nocc, int32_t nvir, const double* eps_o, const double* eps_v, const double* t1,
             const double* t2, const double* ovvv, const double* ooov, const double* ovov, bool host_eps);

namespace {

static __device__ __align__(256) char scratch[BQC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).  The array's name is not a device
// address in host code: only this pointer is passed to kernels.
void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) throw Error(BQC_EINVAL, "device ordinal beyond the supported range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Error(BQC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int triple_space(int o, int v, int form) { return form == FORM_VIR ? v : o; }
inline int tile_space(int o, int v, int form) { return form == FORM_VIR ? o : v; }

// Workspace of a solve with nb triples per batch and ONE H buffer.
struct NLayout {
    size_t ops, trip, orbits, hbuf, partial, etrip, energy, check, aux, total;
};
NLayout nlayout(int o, int v, int prec, int form, bool fock, int64_t nb) {
    const int nt = ceil_div(tile_space(o, v, form), EPI_T);
    const int64_t norbit = num_tile_orbits(nt);
    const int64_t ntrip = num_triples(triple_space(o, v, form));
    NLayout L;
    size_t off = 0;
    L.ops = off; off += a256(prepare_bytes(prec, o, v));
    L.trip = off; off += a256((size_t)std::max<int64_t>(ntrip, 1) * sizeof(int4));
    L.orbits = off; off += a256((size_t)norbit * sizeof(int4));
    L.hbuf = off; off += a256((size_t)nb * 3 * hpair_elems(tile_space(o, v, form)) * hbuf_bytes(prec));
    L.partial = off; off += a256((size_t)nb * norbit * sizeof(double));
    L.etrip = off; off += a256((size_t)std::max<int64_t>(ntrip, 1) * sizeof(double));
    L.energy = off; off += 256;
    L.check = off; off += 256;
    L.aux = off; off += form == FORM_VIR ? a256(vir_aux_bytes(o, v, fock)) : 0;
    L.total = off;
    return L;
}

// Triples per batch: the library's batch size, reduced until the workspace
// fits the array; 0 if not even one triple per batch fits.
int64_t noalloc_batch(int o, int v, int prec, int form, bool fock) {
    int64_t nb = batch_triples(o, v, prec, form);
    while (nb >= 1 && nlayout(o, v, prec, form, fock, nb).total > (size_t)BQC_NOALLOC_SCRATCH_BYTES) {
        const int64_t fit = nb / 2;
        nb = fit;
    }
    return nb;
}

// Unique triples (x, y, z, m) of {0..n-1}, x <= y <= z, x = y = z skipped,
// in lexicographic order: thread x writes those whose first index is x.
__global__ void triple_table_kernel(int n, int4* out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int64_t at = 0;  // triples whose first index is below x: sum over x' < x of (n-x')(n-x'+1)/2 - 1
    for (int p = 0; p < x; ++p) at += (int64_t)(n - p) * (n - p + 1) / 2 - 1;
    for (int y = x; y < n; ++y)
        for (int z = y; z < n; ++z) {
            if (x == y && y == z) continue;
            out[at++] = make_int4(x, y, z, (x < y && y < z) ? 6 : 3);
        }
}

// Tile orbits (A, B, C, |stabiliser|), A >= B >= C, A outermost: thread A
// writes the orbits whose first tile is A (A (A+1)(A+2)/6 precede them).
__global__ void orbit_table_kernel(int nt, int4* out) {
    const int A = blockIdx.x * blockDim.x + threadIdx.x;
    if (A >= nt) return;
    int64_t at = (int64_t)A * (A + 1) * (A + 2) / 6;
    for (int B = 0; B <= A; ++B)
        for (int C = 0; C <= B; ++C)
            out[at++] = make_int4(A, B, C, (A == B && B == C) ? 6 : ((A == B || B == C) ? 2 : 1));
}

// max(eps_o), min(eps_v) and whether every orbital energy is finite, for the
// gap check on the host: out[0] = max eps_o, out[1] = min eps_v, out[2] = 1
// if all are finite (one work group, strided).
__global__ void gap_check_kernel(const double* eps_o, int o, const double* eps_v, int v, double* out) {
    __shared__ double smax[256], smin[256];
    __shared__ int sfin[256];
    double mx = -INFINITY, mn = INFINITY;
    int fin = 1;
    for (int i = threadIdx.x; i < o; i += blockDim.x) {
        mx = fmax(mx, eps_o[i]);
        fin &= isfinite(eps_o[i]) ? 1 : 0;
    }
    for (int a = threadIdx.x; a < v; a += blockDim.x) {
        mn = fmin(mn, eps_v[a]);
        fin &= isfinite(eps_v[a]) ? 1 : 0;
    }
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    sfin[threadIdx.x] = fin;
    __syncthreads();
    for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + h]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + h]);
            sfin[threadIdx.x] &= sfin[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smax[0];
        out[1] = smin[0];
        out[2] = sfin[0] ? 1.0 : 0.0;
    }
}

int noalloc_impl(int32_t o, int32_t v, const double* eps_o, const double* eps_v, const double* t1,
                 const double* t2, const double* ovvv, const double* ooov, const double* ovov,
                 const bqc_t_opts* opts, double* E_T, bqc_t_stats* stats) {
    if (!opts) return fail(BQC_EINVAL, "opts is required (inputs_on_device = 1)");
    const bqc_t_opts op = *opts;
    if (!E_T) return fail(BQC_EINVAL, "E_T is null");
    if (!op.inputs_on_device) return fail(BQC_EINVAL, "bqc_t_energy_noalloc takes device-resident inputs only");
    if (op.precision < 0 || op.precision > 3) return fail(BQC_EINVAL, "unknown precision");
    if (op.formulation != BQC_FORM_OCCUPIED && op.formulation != BQC_FORM_VIRTUAL)
        return fail(BQC_EINVAL, "unknown formulation");
    const int form = op.formulation == BQC_FORM_VIRTUAL ? FORM_VIR : FORM_OCC;
    if (form == FORM_VIR && op.precision == BQC_PREC_FP8)
        return fail(BQC_EINVAL, "the virtual-triple formulation runs in FP64, FP32 or split-BF16x3");
    int rc = validate(o, v, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, false);
    if (rc != BQC_OK) return rc;
    const int nx = triple_space(o, v, form);
    const int64_t ntrip = num_triples(nx);
    if (ntrip > (int64_t)INT32_MAX) return fail(BQC_EINVAL, "more unique triples than one solve supports");
    if (op.triple_end == 0 ? op.triple_begin != 0
                           : (op.triple_begin < 0 || op.triple_begin >= op.triple_end || op.triple_end > ntrip))
        return fail(BQC_EINVAL, "triple range outside [0, number of unique triples] or empty");
    const bool fock = op.fock_ov != nullptr;
    const int prec = op.precision;
    const int64_t nb = noalloc_batch(o, v, prec, form, fock);
    if (nb < 1)
        return fail(BQC_ENOMEM, "workspace of (nocc, nvir) = (" + std::to_string(o) + ", " + std::to_string(v) +
                                    ") in this precision exceeds the " + std::to_string(BQC_NOALLOC_SCRATCH_BYTES) +
                                    "-byte array of bqc_t_energy_noalloc");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(BQC_EDEVICE, "no HIP device");
    if (op.device < 0 || op.device >= ndev) return fail(BQC_EINVAL, "device ordinal out of range");
    int prev = 0;
    BQC_HIP(hipGetDevice(&prev));
    struct Restore { int d; ~Restore() { (void)hipSetDevice(d); } } restore{prev};
    BQC_HIP(hipSetDevice(op.device));
    char* base = (char*)scratch_ptr(op.device);
    hipStream_t st = (hipStream_t)op.stream;  // NULL: the device's null stream

    const NLayout L = nlayout(o, v, prec, form, fock, nb);
    double* chk = (double*)(base + L.check);
    gap_check_kernel<<<1, 256, 0, st>>>(eps_o, o, eps_v, v, chk);
    BQC_HIP(hipGetLastError());
    double gap[3] = {0, 0, 0};
    BQC_HIP(hipMemcpyAsync(gap, chk, sizeof(gap), hipMemcpyDeviceToHost, st));
    BQC_HIP(hipStreamSynchronize(st));
    if (gap[2] != 1.0) return fail(BQC_EINVAL, "non-finite orbital energy");
    if (!(gap[0] < gap[1])) return fail(BQC_EINVAL, "gap condition max(eps_o) < min(eps_v) violated");

    DevInputs in;
    in.o = o; in.v = v;
    in.eps_o = eps_o; in.eps_v = eps_v; in.t1 = t1; in.t2 = t2;
    in.ovvv = ovvv; in.ooov = ooov; in.ovov = ovov; in.fock_ov = op.fock_ov;

    int4* d_trip = (int4*)(base + L.trip);
    int4* d_orb = (int4*)(base + L.orbits);
    const int nt = ceil_div(tile_space(o, v, form), EPI_T);
    const int norbit = (int)num_tile_orbits(nt);
    void* hbuf = base + L.hbuf;
    double* partial = (double*)(base + L.partial);
    double* etrip = (double*)(base + L.etrip);
    double* d_total = (double*)(base + L.energy);
    const int t_begin = op.triple_end > 0 ? (int)op.triple_begin : 0;
    const int t_end = op.triple_end > 0 ? (int)op.triple_end : (int)ntrip;

    orbit_table_kernel<<<ceil_div(nt, 64), 64, 0, st>>>(nt, d_orb);
    BQC_HIP(hipGetLastError());
    if (ntrip > 0) {
        triple_table_kernel<<<ceil_div(nx, 64), 64, 0, st>>>(nx, d_trip);
        BQC_HIP(hipGetLastError());
        Operands ops;
        launch_prepare(prec, in, base + L.ops, &ops, st, form);
        VirAux aux;
        if (form == FORM_VIR) aux = launch_vir_aux(in, base + L.aux, st);
        for (int b0 = t_begin; b0 < t_end; b0 += (int)nb) {
            const int n = (int)std::min<int64_t>(nb, t_end - b0);
            GemmLaunch g;
            g.o = o; g.v = v; g.ntrip = n; g.trip = d_trip + b0; g.ops = ops; g.hbuf = hbuf;
            gemm_call(prec, g, form).launch(st);
            EpiLaunch e;
            e.ntrip = n; e.trip = d_trip + b0; e.hbuf = hbuf;
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
            epilogue_call(prec, e).launch(st);
            reduce_triples_call(partial, n, norbit, d_trip + b0, etrip + b0).launch(st);
        }
    }
    reduce_total_call(etrip + t_begin, t_end - t_begin, d_total).launch(st);
    double e = 0.0;
    BQC_HIP(hipMemcpyAsync(&e, d_total, sizeof(double), hipMemcpyDeviceToHost, st));
    const int64_t nshare = t_end - t_begin;
    if (op.triple_energies && nshare > 0)
        BQC_HIP(hipMemcpyAsync(op.triple_energies + t_begin, etrip + t_begin, nshare * sizeof(double),
                               hipMemcpyDeviceToHost, st));
    BQC_HIP(hipStreamSynchronize(st));
    if (!std::isfinite(e)) return fail(BQC_EDEVICE, "non-finite energy (device arithmetic failed)");
    *E_T = e;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->footprint_bytes = L.total;
        const double n = tile_space(o, v, form);
        stats->flops = 12.0 * (double)nshare * n * n * n * (double)(v + o);
        stats->precision = prec;
        stats->n_triples = (int32_t)nshare;
    }
    return BQC_OK;
}

}  // namespace
}  // namespace bqc

extern "C" {

int bqc_t_energy_noalloc(int32_t nocc, int32_t nvir, const double* eps_o, const double* eps_v,
                         const double* t1, const double* t2, const double* ovvv, const double* ooov,
                         const double* ovov, const bqc_t_opts* opts, double* E_T, bqc_t_stats* stats) {
    try {
        return bqc::noalloc_impl(nocc, nvir, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, opts, E_T, stats);
    } catch (const bqc::Error& e) {
        return bqc::fail(e.code, e.what());
    } catch (const std::exception& e) {
        return bqc::fail(BQC_EDEVICE, e.what());
    } catch (...) {
        return bqc::fail(BQC_EDEVICE, "unknown failure");
    }
}

int64_t bqc_t_noalloc_batch(int32_t nocc, int32_t nvir, int32_t precision, int32_t formulation, int32_t fock) {
    if (nocc < 1 || nvir < 1 || precision < 0 || precision > 3) return -1;
    if (formulation != BQC_FORM_OCCUPIED && formulation != BQC_FORM_VIRTUAL) return -1;
    const int form = formulation == BQC_FORM_VIRTUAL ? bqc::FORM_VIR : bqc::FORM_OCC;
    if (form == bqc::FORM_VIR && precision == BQC_PREC_FP8) return -1;
    return bqc::noalloc_batch(nocc, nvir, precision, form, fock != 0);
}

}  // extern "C"
