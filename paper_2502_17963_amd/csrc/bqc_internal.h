// Internal declarations of the (T) library: kernel launchers, device
// layouts and the solve driver.  Not part of the public ABI (include/bqc.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace bqc {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define BQC_HIP(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            throw ::bqc::Error(e_ == hipErrorOutOfMemory ? -2 : -3,                \
                               std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                          \
    } while (0)

// ------------------------------------------------------------------ shapes
// Virtual-orbital tile of the epilogue: energies are reduced over orbits of
// EPI_T^3 tiles under the six permutations of (a, b, c).
constexpr int EPI_T = 8;

inline int64_t num_triples(int o) {
    return o < 1 ? 0 : (int64_t)o * (o + 1) * (o + 2) / 6 - o;
}
inline int64_t num_tile_orbits(int nt) { return (int64_t)nt * (nt + 1) * (nt + 2) / 6; }
__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Element size of the contraction operands per precision.
int operand_bytes(int precision);   // bytes per element of every operand copy
int hbuf_bytes(int precision);      // bytes per element of the H buffers

// ------------------------------------------------------------------ layouts
// Device-resident inputs of one solve.  FP64 arrays are the caller's layout.
struct DevInputs {
    int o = 0, v = 0;
    const double* eps_o = nullptr;
    const double* eps_v = nullptr;
    const double* t1 = nullptr;
    const double* t2 = nullptr;
    const double* ovvv = nullptr;
    const double* ooov = nullptr;
    const double* ovov = nullptr;
};

// Contraction operands in the contraction precision (a1):
//   ovvv_c [o][v][v][v]  = (ia|bc)
//   t2_c   [o][o][v][v]  = t_ij^ab
//   t2l_c  [o][v][v][o]  t2l[P][y][u][l] = t_lP^yu
//   hoo_c  [o][o][v][o]  hoo[q][P][u][l] = -(Pu|ql) = -ooov[q][l][P][u]
// For BF16X3 each array holds the hi part followed by the lo part.
// For FP8 each array holds e4m3 bytes; the scales sit in separate arrays
// with one power-of-two exponent per 32 consecutive contraction elements.
struct Operands {
    const void* ovvv = nullptr;
    const void* t2 = nullptr;
    const void* t2l = nullptr;
    const void* hoo = nullptr;
    // FP8 only: E8M0 exponents per 32-element block along the contraction
    const uint8_t* ovvv_s = nullptr;
    const uint8_t* t2_s = nullptr;
    const uint8_t* t2l_s = nullptr;
    const uint8_t* hoo_s = nullptr;
    int64_t lo_off_ovvv = 0, lo_off_t2 = 0, lo_off_t2l = 0, lo_off_hoo = 0;  // BF16X3 lo offsets (elements)
};

// One launch of the contraction kernel covers a batch of triples.
struct GemmLaunch {
    int o, v;
    int ntrip;             // triples in the batch
    const int4* trip;      // (i, j, k, m) per triple in the batch
    Operands ops;
    void* hbuf;            // [ntrip][3][v][v][v] in the H precision
};

struct EpiLaunch {
    int o, v;
    int ntrip;
    const int4* trip;
    const void* hbuf;
    const double* eps_o;
    const double* eps_v;
    const double* t1;
    const double* ovov;
    const int4* orbits;    // (A, B, C, |stabiliser|) with A >= B >= C
    int norbit;
    double* partial;       // [ntrip][norbit]
};

// ------------------------------------------------------------------ launchers
void launch_prepare(int precision, const DevInputs& in, void* ws_ops, Operands* ops,
                    hipStream_t st);
int64_t prepare_bytes(int precision, int o, int v);

void launch_gemm(int precision, const GemmLaunch& g, hipStream_t st);
void launch_epilogue(int precision, const EpiLaunch& e, hipStream_t st);
void launch_reduce_triples(const double* partial, int ntrip, int norbit, const int4* trip,
                           double* e_trip, hipStream_t st);
void launch_reduce_total(const double* e_trip, int64_t n, double* out, hipStream_t st);

// ------------------------------------------------------------------ solve
struct SolveStats {
    double upload_s = 0, prepare_s = 0, gpu_s = 0, gemm_s = 0, epi_s = 0;
    int gemm_launches = 0, epi_launches = 0;
    uint64_t footprint = 0;
};

// Triple-batch size of a solve: a function of (o, v, precision) only, so
// that a solve's decomposition never depends on what else runs.
int batch_triples(int o, int v, int precision);

// Device bytes a solve holds, excluding its FP64 inputs.
int64_t workspace_bytes(int o, int v, int precision);
int64_t input_bytes(int o, int v);

// Host-side plan of a solve: triple table and tile-orbit table.
struct Plan {
    int o = 0, v = 0, precision = 0, nb = 0;
    std::vector<int4> trip;    // unique triples (i, j, k, m)
    std::vector<int4> orbits;  // epilogue tile orbits
};
Plan make_plan(int o, int v, int precision);

// A solve whose inputs are resident on the device.  The caller owns `ws`
// (workspace_bytes(o, v, precision) bytes, 256-byte aligned) and the stream.
// Enqueues everything; the energy lands in *d_energy (device) and the
// per-triple energies in d_etrip (device, num_triples(o) doubles).
void enqueue_solve(const Plan& plan, const DevInputs& in, void* ws, double* d_energy,
                   hipStream_t st, bool timing, SolveStats* stats);

}  // namespace bqc
