// Internal declarations of the (T) library: kernel launchers, device
// layouts and the solve driver.  Not part of the public ABI (include/bqc.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
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
// Tile of the epilogue (of virtuals, or of occupied orbitals in the loop
// over virtual triples): energies are reduced over orbits of EPI_T^3 tiles
// under the six permutations of the three tile-space indices.
constexpr int EPI_T = 8;

// The H buffers are stored in EPI_T^3 blocks, so that the epilogue reads every
// block it needs as one contiguous run: with n the size of the tile space
// (nvir, or nocc in the loop over virtual triples) and nt = ceil(n / EPI_T),
// element (y, u, w) of one pair lies at
//   ((y / 8 * nt + u / 8) * nt + w / 8) * 512 + (y % 8 * 8 + u % 8) * 8 + w % 8.
// Elements with an index >= n are never written and never read.
__host__ __device__ inline int64_t hpair_elems(int v) {
    const int64_t nt = (v + EPI_T - 1) / EPI_T;
    return nt * nt * nt * EPI_T * EPI_T * EPI_T;
}

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
    const double* ovvv = nullptr;  // nullptr: formed from b_ov, b_vv (density fitting)
    const double* ooov = nullptr;
    const double* ovov = nullptr;
    // density-fitting factors b_ov[naux][o][v], b_vv[naux][v][v] and the FP64
    // scratch for df_block occupied planes (o-slices of (ov|vv)) at a time
    const double* b_ov = nullptr;
    const double* b_vv = nullptr;
    int naux = 0;
    double* df_tmp = nullptr;
    int df_block = 0;
    const double* fock_ov = nullptr;  // f_ia of a non-canonical reference, or nullptr
};

// Contraction operands in the contraction precision (a1), chunk-major: a
// factor is a set of matrices M of v rows; for each 128-byte chunk of the
// contraction index (KC elements: 16 FP64, 32 FP32, 32 bf16 hi + 32 lo for
// BF16X3) all v rows are contiguous:  byte offset of (M, row r, chunk c) =
// ((M * nchunk + c) * v + r) * 128.  Contraction lengths are zero-padded to
// Kv = roundup(v, KPAD) and Ko = roundup(o, KPAD).
//   ovvv  M = P*v + y, r = u, k = d:  (Pu|yd)
//   t2    M = P*o + q, r = u, k = d:  t_Pq^ud
//   t2l   M = P*v + y, r = u, k = l:  t_lP^yu
//   hoo   M = q*o + P, r = u, k = l:  -(Pu|ql)
// In the loop over virtual triples the matrices have o rows instead (same
// byte counts; the matrix maps are in kernels_prep.hip).
// FP8: KC = 128 e4m3 bytes per chunk and contraction lengths padded to 128;
// each row of each chunk also has a 4-byte word of E8M0 exponents, one per
// 32 elements (scale 2^(byte - 127)), at ((M * nchunk + c) * v + r) * 4.
constexpr int KPAD = 32;
int chunk_elems(int precision);
int kpad_of(int precision);
struct Operands {
    const void* ovvv = nullptr;
    const void* t2 = nullptr;
    const void* t2l = nullptr;
    const void* hoo = nullptr;
    const uint32_t* ovvv_s = nullptr;  // FP8 scale words
    const uint32_t* t2_s = nullptr;
    const uint32_t* t2l_s = nullptr;
    const uint32_t* hoo_s = nullptr;
    int Kv = 0, Ko = 0;
};

// Formulations of a solve.  FORM_OCC: the loop runs over unique occupied
// triples i <= j <= k and every launch works on tensors over the virtual
// indices.  FORM_VIR: the loop runs over unique virtual triples a <= b <= c
// (the paper's loop order) and the same kernels work on tensors over the
// occupied indices; the energy is the same sum taken in the other order.
constexpr int FORM_OCC = 0, FORM_VIR = 1;

// One launch of the contraction kernel covers a batch of triples.
struct GemmLaunch {
    int o, v;
    int ntrip;             // triples in the batch
    const int4* trip;      // (i, j, k, m) per triple in the batch
    Operands ops;
    void* hbuf;            // [ntrip][3] pairs of hpair_elems(n) blocked elements in the H precision
                           // (n = v, or o for FORM_VIR)
};

// Grouped launches: one launch covers the current triple batch of several
// solves (fragments).  Each entry describes one fragment's part and the first
// logical work group (or block) of that part; entries are in increasing
// order of it, and a work group finds its entry by binary search.
struct GemmGroupEntry {
    GemmLaunch g;
    int nblk, ntile_u, ntile_w;  // the fragment's tiling (contraction_tiling)
    int wg0;                     // first logical work group of this entry
};

// The epilogue is written for triples (i, j, k) of one orbital space and
// tiles of the other: o is the size of the triples' space and v that of the
// tiles' space, eps_o / eps_v their orbital energies, t1 [o][v], ovov
// [o][v][o][v], t2 [o][o][v][v] and fock_ov [o][v] in those roles.  The
// occupied-triple loop passes the inputs as they are; the virtual-triple loop
// passes o = nvir, v = nocc, -eps_v, -eps_o and the transposed arrays
// t1[a][i], (ia|jb) as [a][b][i][j], t2[a][b][i][j], f[a][i] (every term of V and of Z is
// symmetric in the two spaces, and the sign flip keeps D = sum over the
// triple's energies minus the tiles').
struct EpiLaunch {
    int o, v;
    int ntrip;
    const int4* trip;
    const void* hbuf;
    const double* eps_o;
    const double* eps_v;
    const double* t1;
    const double* ovov;    // (px|qy) at p * ovov_sp + x * ovov_sx + q * ovov_sq + y
    int64_t ovov_sp, ovov_sx, ovov_sq;
    const double* t2;      // t2[i][j][a][b] (used with fock_ov)
    const double* fock_ov; // nullptr: canonical reference; else f_ia [o][v]
    const int4* orbits;    // (A, B, C, |stabiliser|) with A >= B >= C
    int norbit;
    double* partial;       // [ntrip][norbit]
};

// Padded contraction lengths and matrix counts of the four factors (the
// counts of the virtual-triple layout differ, the sizes in bytes do not).
struct Sizes {
    int Kv, Ko;
    int64_t m_ovvv, m_t2, m_t2l, m_hoo;  // matrices per factor
};
Sizes factor_sizes(int o, int v, int precision);

// ------------------------------------------------------------------ launchers
// One kernel launch held as data (function, shape, argument values), so that
// it can be launched on a stream or added to a hipGraph as a kernel node.
struct KernelCall {
    const void* fn = nullptr;
    dim3 grid, block;
    unsigned shmem = 0;
    alignas(16) char buf[384];
    size_t at[8] = {};
    int nargs = 0;
    size_t used = 0;
    template <class T>
    KernelCall& arg(const T& x) {
        used = (used + alignof(T) - 1) / alignof(T) * alignof(T);
        if (nargs >= 8 || used + sizeof(T) > sizeof(buf)) throw Error(-1, "kernel argument buffer too small");
        std::memcpy(buf + used, &x, sizeof(T));
        at[nargs++] = used;
        used += sizeof(T);
        return *this;
    }
    // argument pointers into this object's buffer (valid while it lives)
    void pointers(void** p) const {
        for (int a = 0; a < nargs; ++a) p[a] = (void*)(buf + at[a]);
    }
    void launch(hipStream_t st) const {
        void* p[8];
        pointers(p);
        BQC_HIP(hipLaunchKernel(fn, grid, block, p, shmem, st));
    }
    // kernel node after `deps` (the node copies the argument values)
    hipGraphNode_t add_to(hipGraph_t gr, const std::vector<hipGraphNode_t>& deps) const {
        void* p[8];
        pointers(p);
        hipKernelNodeParams kp{};
        kp.func = const_cast<void*>(fn);
        kp.gridDim = grid;
        kp.blockDim = block;
        kp.sharedMemBytes = shmem;
        kp.kernelParams = p;
        kp.extra = nullptr;
        hipGraphNode_t n = nullptr;
        BQC_HIP(hipGraphAddKernelNode(&n, gr, deps.empty() ? nullptr : deps.data(), deps.size(), &kp));
        return n;
    }
};

void launch_prepare(int precision, const DevInputs& in, void* ws_ops, Operands* ops,
                    hipStream_t st, int form = FORM_OCC);

// The operand conversion of several solves (loop over occupied triples,
// (ia|bc) given) in one launch per factor: entry x converts its factor
// (`src` -> `dst`, nmat matrices of `rows` rows, contraction length len
// padded to kpad) with blocks [b0, b0 + nb).  ws[f] is solve f's operand
// area (prepare_bytes); `tables` (host) and d_tables (device, 4 n entries)
// must stay valid until the stream has passed the launches.
struct FactorGroupEntry {
    const double* src;
    void* dst;
    int64_t nmat;
    int rows, len, kpad, o, v;
    int b0, nb;
};
void launch_prepare_group(int precision, int n, const DevInputs* ins, void* const* ws, Operands* ops,
                          FactorGroupEntry* d_tables, std::vector<FactorGroupEntry>& tables, hipStream_t st);

// Transposed FP64 inputs of the virtual-triple loop's epilogue (see
// EpiLaunch), built once per solve: -eps_v, -eps_o, t1[a][i], (ia|jb) as
// ovov_t[a][b][i][j] (an o x o matrix per virtual pair, so that the
// epilogue's 8 x 8 blocks are compact), and with a non-canonical reference
// t2[a][b][i][j] and f[a][i].
struct VirAux {
    double *neg_eps_v = nullptr, *neg_eps_o = nullptr, *t1_t = nullptr, *ovov_t = nullptr;
    double *t2_t = nullptr, *fock_t = nullptr;
};
int64_t vir_aux_bytes(int o, int v, bool fock);
VirAux launch_vir_aux(const DevInputs& in, void* aux, hipStream_t st);
int64_t prepare_bytes(int precision, int o, int v);
// Occupied planes of (ov|vv) formed per pass of the density-fitting product,
// and the scratch (doubles) they need.
int df_block_planes(int o, int v);
int64_t df_scratch_elems(int o, int v);

// form = FORM_VIR: the triples of g are virtual and the planes, rows and
// columns of H run over the occupied indices.
KernelCall gemm_call(int precision, const GemmLaunch& g, int form = FORM_OCC);
// Contraction wave tile (16-blocks per side) for rows and columns of size n;
// tiles of min_wb .. 5 blocks are considered.
int wave_blocks(int n, int min_wb = 2);
KernelCall epilogue_call(int precision, const EpiLaunch& e);

// Tiling of one contraction launch with wave tiles of wb x wb blocks:
// 16-blocks of the tile space, tiles along rows and columns, and the work
// groups of a launch of ntrip triples (3 pairs x n planes x tiles).
struct Tiling {
    int nblk, ntile_u, ntile_w;
    int64_t n_wg;
};
Tiling contraction_tiling(int n, int wb, int ntrip);
struct EpiGroupEntry {
    EpiLaunch e;
    int wg0;  // first logical work group: ntrip x norbit groups per entry
};
struct RedGroupEntry {
    const double* partial;  // [ntrip][norbit]
    int norbit;
    const int4* trip;
    double* e_trip;         // per-triple energies of the entry's triples
    int b0;                 // first block: one block per triple
};
struct TotalGroupEntry {
    const double* e_trip;
    int64_t n;
    double* out;
};
// Grouped contraction (loop over occupied triples, wave tile wb x wb for
// every entry), epilogue, per-triple sums and totals (one block per entry).
KernelCall gemm_group_call(int precision, int wb, const GemmGroupEntry* d_ent, int nent, int64_t n_wg);
KernelCall epilogue_group_call(int precision, const EpiGroupEntry* d_ent, int nent, int64_t n_wg);
KernelCall reduce_triples_group_call(const RedGroupEntry* d_ent, int nent, int nblocks);
KernelCall reduce_total_group_call(const TotalGroupEntry* d_ent, int nent);
KernelCall reduce_triples_call(const double* partial, int ntrip, int norbit, const int4* trip,
                               double* e_trip);
KernelCall reduce_total_call(const double* e_trip, int64_t n, double* out);

// ------------------------------------------------------------------ MP2
int64_t mp2_workspace_bytes(int o, int v);
// Enqueues the density-fitted MP2 energy; returns after `st` has drained,
// with the energy (and the per-pair energies, if pair_e) in the workspace.
double* enqueue_mp2(int o, int v, int naux, const double* eps_o, const double* eps_v, const double* b_ov,
                    void* ws, hipStream_t st, double** pair_e);

// ------------------------------------------------------------------ solve
struct SolveStats {
    double upload_s = 0, prepare_s = 0, gpu_s = 0, gemm_s = 0, epi_s = 0;
    int gemm_launches = 0, epi_launches = 0;
    uint64_t footprint = 0;
};

// Triple-batch size of a solve: a function of (o, v, precision, form) only,
// so that a solve's decomposition never depends on what else runs.
int batch_triples(int o, int v, int precision, int form = FORM_OCC);

// Device bytes a solve holds, excluding its FP64 inputs (fock: the solve
// has an f_ov block, which the virtual-triple loop transposes).
int64_t workspace_bytes(int o, int v, int precision, int form = FORM_OCC, bool fock = false);
int64_t input_bytes(int o, int v);

// Host-side plan of a solve: triple table and tile-orbit table.
struct Plan {
    int o = 0, v = 0, precision = 0, nb = 0;
    int form = FORM_OCC;
    std::vector<int4> trip;    // unique triples (i, j, k, m) of the loop's orbital space
    std::vector<int4> orbits;  // epilogue tile orbits
    int64_t begin = 0, end = 0;  // the solved share [begin, end) of `trip`
};
// Plan of the share [begin, end) of the unique triples (end = 0: all).
Plan make_plan(int o, int v, int precision, int64_t begin = 0, int64_t end = 0, int form = FORM_OCC);

// A solve whose inputs are resident on the device.  The caller owns `ws`
// (workspace_bytes(o, v, precision) bytes, 256-byte aligned) and the stream.
// Enqueues everything; the energy and the per-triple energies stay in the
// workspace (workspace_energy / workspace_etrip).
// `side` is a second stream of the same device on which the epilogues run,
// overlapping the contractions on `st`; everything is ordered back onto `st`.
// Returns after `st` has drained (the solve is complete).  graph = true
// builds the batch sequence as one hipGraph (kernel nodes with the same
// dependencies; no stream capture, `side` unused) and launches it on `st` as
// one unit (no per-kernel timing then).
// Device pointers of the per-triple energies and of the total in a workspace.
double* workspace_etrip(void* ws, int o, int v, int precision, int form = FORM_OCC);
double* workspace_energy(void* ws, int o, int v, int precision, int form = FORM_OCC);

void enqueue_solve(const Plan& plan, const DevInputs& in, void* ws, double* d_energy,
                   hipStream_t st, hipStream_t side, bool timing, SolveStats* stats, bool graph = false);

// ------------------------------------------------------------------ batch
// Several fragments solved together with grouped launches (batch.hip), loop
// over occupied triples.  Workspace offsets (bytes) of one fragment's parts.
struct BatchFrag {
    int o = 0, v = 0;
    int64_t ntrip = 0;
    int norbit = 0;
    int nb = 0;                              // triples per round
    size_t ops = 0, hbuf = 0, partial = 0, etrip = 0;
    size_t trip = 0, orbits = 0;             // offsets inside the tables region
};
struct BatchPlan {
    int rounds = 0;
    std::vector<BatchFrag> frag;
    size_t tabs = 0, tabs_bytes = 0;         // triple and orbit tables of all fragments
    size_t factor_tab = 0;                   // operand-conversion entries
    size_t entries = 0, entries_bytes = 0;   // grouped-launch entries of every round
    size_t energies = 0;                     // the fragments' energies, contiguous
    size_t total = 0;                        // workspace bytes
};
BatchPlan plan_batch(int n, const int* nocc, const int* nvir, int precision);
// Enqueues the whole batch on st (inputs device resident), copies the n
// energies to energies_host and returns after st has drained.
void enqueue_batch(const BatchPlan& bp, int precision, int n, const DevInputs* ins, void* ws, hipStream_t st,
                   double* energies_host, SolveStats* stats);

}  // namespace bqc
