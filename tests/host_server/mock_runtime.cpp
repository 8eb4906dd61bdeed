// Test infrastructure, never linked into the library: host-only stand-ins
// for the HIP runtime calls and the solve entry points that csrc/server.cpp
// uses, so that the server's queueing, admission, arena and ticket logic can
// run on the CPU under ThreadSanitizer / AddressSanitizer.  The stand-in
// solve touches the whole workspace, reads the orbital energies and writes an
// energy that the stress driver can predict.
#include <hip/hip_runtime_api.h>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>
#include "bqc_internal.h"

static thread_local int g_dev = 0;
extern "C" {
hipError_t hipGetDevice(int* d) { *d = g_dev; return hipSuccess; }
hipError_t hipSetDevice(int d) { g_dev = d; return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock error"; }
hipError_t hipMalloc(void** p, size_t n) { *p = std::malloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { *p = std::malloc(n); return hipSuccess; }
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemGetInfo(size_t* f, size_t* t) { *f = (size_t)1 << 30; *t = (size_t)1 << 31; return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) { *s = (hipStream_t)std::malloc(16); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { std::free((void*)s); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
}

namespace bqc {
// the solve writes a value derived from (o, v) into the workspace energy slot
int64_t workspace_bytes(int o, int v, int, int, bool) { return (int64_t)(o * 7 + v) * 256 + 4096; }
int64_t input_bytes(int o, int v) {
    const int64_t n = (int64_t)o + v + (int64_t)o * v + (int64_t)o * o * v * v + (int64_t)o * v * v * v +
                      (int64_t)o * o * o * v + (int64_t)o * v * o * v;
    return n * 8 + 7 * 256;
}
double* workspace_energy(void* ws, int, int, int, int) { return (double*)ws; }
Plan make_plan(int o, int v, int precision, int64_t, int64_t, int) { Plan p; p.o = o; p.v = v; p.precision = precision; return p; }
void enqueue_solve(const Plan& plan, const DevInputs& in, void* ws, double*, hipStream_t, hipStream_t, bool,
                   SolveStats* st, bool) {
    // touch the whole workspace and read every input element, like the device would
    const size_t n = (size_t)workspace_bytes(plan.o, plan.v, plan.precision);
    std::memset(ws, 0x11, n);
    double acc = 0;
    for (int a = 0; a < plan.o; ++a) acc += in.eps_o[a];
    for (int a = 0; a < plan.v; ++a) acc += in.eps_v[a];
    std::this_thread::sleep_for(std::chrono::microseconds(200 + (plan.o * 37 + plan.v) % 500));
    *(double*)ws = acc + plan.o * 1000.0 + plan.v;
    if (st) st->gpu_s = 1e-4;
}
// Batches (small requests admitted together): the same energy per member as
// the stand-in solve, written by the stand-in batch.
BatchPlan plan_batch(int n, const int* nocc, const int* nvir, int precision) {
    BatchPlan bp;
    bp.frag.resize(n);
    size_t off = 0;
    for (int f = 0; f < n; ++f) {
        bp.frag[f].o = nocc[f];
        bp.frag[f].v = nvir[f];
        bp.frag[f].ops = off;
        off += (size_t)workspace_bytes(nocc[f], nvir[f], precision);
    }
    bp.total = off + 256;
    return bp;
}
void enqueue_batch(const BatchPlan& bp, int, int n, const DevInputs* ins, void* ws, hipStream_t, double* e,
                   SolveStats* st) {
    std::memset(ws, 0x22, bp.total);
    for (int f = 0; f < n; ++f) {
        double acc = 0;
        for (int a = 0; a < ins[f].o; ++a) acc += ins[f].eps_o[a];
        for (int a = 0; a < ins[f].v; ++a) acc += ins[f].eps_v[a];
        e[f] = acc + ins[f].o * 1000.0 + ins[f].v;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(300));
    if (st) { st->gpu_s = 1e-4; st->gemm_launches = 1; st->epi_launches = 1; }
}
}  // namespace bqc
namespace bqc {
thread_local std::string g_err;
int fail(int code, const std::string& msg) { g_err = msg; return code; }
int validate(int32_t o, int32_t v, const double* eo, const double* ev, const double* t1, const double* t2,
             const double* ovvv, const double* ooov, const double* ovov, bool host_eps) {
    if (o < 1 || v < 1 || !eo || !ev || !t1 || !t2 || !ovvv || !ooov || !ovov) return fail(-1, "bad");
    if (host_eps) { volatile double x = eo[o - 1] + ev[0]; (void)x; }
    return 0;
}
}  // namespace bqc
