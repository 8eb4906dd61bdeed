// Closed-shell MP2 correlation energy with density-fitted integrals (the
// paper's MP2 equation; density fitting as in its section 2.2):
//   E = sum_{i,j} sum_{a,b} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b),
//   (ia|jb) = sum_Q B^Q_ia B^Q_jb.
// No four-index integral or denominator tensor is stored: one work group
// takes one occupied pair i <= j and one pair of 64-wide virtual tiles A <= B
// and forms on FP64 MFMA (16x16x4), contracting over Q in LDS-staged steps,
//   K1[a][b] = (ia|jb)   (a in A, b in B)   and   K2[b][a] = (ib|ja)   (b in B, a in A),
// then divides by the denominator in registers.  With x = K1[a][b] and
// y = K2[b][a] (read through LDS):
//   A < B:  the ordered pairs (a, b) and (b, a) together give (2x^2 + 2y^2 - 2xy) / D,
//   A = B:  each ordered pair gives x (2x - y) / D (K2 = K1 then),
// and i < j counts twice ((ia|jb) = (jb|ia)).  Each work group writes one
// FP64 partial; partials are summed per pair and then over pairs in a fixed
// order with Neumaier compensation (deterministic, no atomics).
#include "bqc_internal.h"

namespace bqc {
namespace {

constexpr int M_T = 64, M_K = 16, M_THREADS = 256;
typedef double d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(M_THREADS) void mp2_kernel(const double* __restrict__ b_ov,
                                                        const double* __restrict__ eps_o,
                                                        const double* __restrict__ eps_v, const int2* pairs,
                                                        const int2* tiles, int ntp, int o, int v, int naux,
                                                        double* partial) {
    const int64_t wg = blockIdx.x;
    const int2 ij = pairs[wg / ntp];
    const int2 tb = tiles[wg % ntp];
    const int i = ij.x, j = ij.y;
    const int A0 = tb.x * M_T, B0 = tb.y * M_T;

    // strips s: 0 = B^Q_{i, A}, 1 = B^Q_{i, B}, 2 = B^Q_{j, A}, 3 = B^Q_{j, B}; after the
    // contraction the same memory holds K2 for the exchange through LDS
    __shared__ double lds[4 * M_K * M_T];
    __shared__ double red[M_THREADS / 64];
    double (*S)[M_K][M_T] = (double (*)[M_K][M_T])lds;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;  // this wave's 32 x 32 block
    const int fr = lane & 15, fg = lane >> 4;

    d4 k1[2][2], k2[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) k1[x][y] = k2[x][y] = d4{0, 0, 0, 0};

    const int64_t ov = (int64_t)o * v;
    // the strips of step Q0 + M_K are loaded into registers while step Q0 is
    // contracted from LDS
    double r[16];
    auto load = [&](int Q0) {
#pragma unroll
        for (int n = 0; n < 16; ++n) {
            const int idx = tid + M_THREADS * n;  // < 4 * 16 * 64
            const int s = idx / (M_K * M_T), k = (idx / M_T) % M_K, m = idx % M_T;
            const int occ = s < 2 ? i : j, col = (s & 1 ? B0 : A0) + m, Q = Q0 + k;
            r[n] = (Q < naux && col < v) ? b_ov[(int64_t)Q * ov + (int64_t)occ * v + col] : 0.0;
        }
    };
    load(0);
    for (int Q0 = 0; Q0 < naux; Q0 += M_K) {
        __syncthreads();  // the previous step's fragment reads are done
#pragma unroll
        for (int n = 0; n < 16; ++n) lds[tid + M_THREADS * n] = r[n];
        __syncthreads();
        if (Q0 + M_K < naux) load(Q0 + M_K);
#pragma unroll
        for (int st = 0; st < M_K / 4; ++st) {
            const int k = 4 * st + fg;  // contraction index of this lane in the 16x16x4 step
            double a1[2], b1[2], a2[2], b2[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a1[x] = S[0][k][wr + 16 * x + fr];  // rows a of K1: B_{i,A}
                b1[x] = S[3][k][wc + 16 * x + fr];  // cols b of K1: B_{j,B}
                a2[x] = S[1][k][wr + 16 * x + fr];  // rows b of K2: B_{i,B}
                b2[x] = S[2][k][wc + 16 * x + fr];  // cols a of K2: B_{j,A}
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    k1[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[x], b1[y], k1[x][y], 0, 0, 0);
                    k2[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[x], b2[y], k2[x][y], 0, 0, 0);
                }
        }
    }
    __syncthreads();
    // K2 to LDS as K2s[b][a] (FP64 accumulator layout: register r of lane l
    // holds row (l / 16) + 4 r, column l % 16 of the 16x16 block)
    double* K2s = lds;  // 64 x 64 doubles
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                K2s[(wr + 16 * x + fg + 4 * q) * M_T + wc + 16 * y + fr] = k2[x][y][q];
    __syncthreads();

    const double eij = eps_o[i] + eps_o[j];
    const bool diag = tb.x == tb.y;
    double acc = 0.0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int al = wr + 16 * x + fg + 4 * q, bl = wc + 16 * y + fr;  // locals of a (in A), b (in B)
                const int a = A0 + al, b = B0 + bl;
                if (a < v && b < v) {
                    const double xk = k1[x][y][q], yk = K2s[bl * M_T + al];
                    const double d = eij - eps_v[a] - eps_v[b];
                    acc += diag ? xk * (2.0 * xk - yk) / d : (2.0 * (xk * xk + yk * yk) - 2.0 * xk * yk) / d;
                }
            }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < M_THREADS / 64; ++w) s += red[w];
        partial[wg] = (i < j ? 2.0 : 1.0) * s;
    }
}

// Neumaier compensated accumulation: (s, c) += x
__device__ __forceinline__ void neu(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

// out[g] = fixed-order compensated sum of x[g * n .. g * n + n) (one block per g)
__global__ __launch_bounds__(256) void segment_sum_kernel(const double* x, int64_t n, double* out) {
    __shared__ double ss[256], cs[256];
    const double* seg = x + (int64_t)blockIdx.x * n;
    double s = 0.0, c = 0.0;
    for (int64_t idx = threadIdx.x; idx < n; idx += 256) neu(s, c, seg[idx]);
    ss[threadIdx.x] = s;
    cs[threadIdx.x] = c;
    __syncthreads();
    for (int half = 128; half >= 1; half >>= 1) {
        if ((int)threadIdx.x < half) {
            double s1 = ss[threadIdx.x], c1 = cs[threadIdx.x];
            neu(s1, c1, ss[threadIdx.x + half]);
            ss[threadIdx.x] = s1;
            cs[threadIdx.x] = c1 + cs[threadIdx.x + half];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = ss[0] + cs[0];
}

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Mp2Layout {
    size_t pairs, tiles, partial, pair_e, energy, total;
    int64_t npair, ntp;
};

Mp2Layout mp2_layout(int o, int v) {
    Mp2Layout L;
    const int64_t nt = ceil_div(v, M_T);
    L.npair = (int64_t)o * (o + 1) / 2;
    L.ntp = nt * (nt + 1) / 2;
    size_t off = 0;
    L.pairs = off; off += a256((size_t)L.npair * sizeof(int2));
    L.tiles = off; off += a256((size_t)L.ntp * sizeof(int2));
    L.partial = off; off += a256((size_t)(L.npair * L.ntp) * sizeof(double));
    L.pair_e = off; off += a256((size_t)L.npair * sizeof(double));
    L.energy = off; off += 256;
    L.total = off;
    return L;
}

}  // namespace

int64_t mp2_workspace_bytes(int o, int v) { return (int64_t)mp2_layout(o, v).total; }

// Enqueues the MP2 energy on `st` into the workspace; returns the device
// address of the energy (and of the per-pair energies via pair_e).
double* enqueue_mp2(int o, int v, int naux, const double* eps_o, const double* eps_v, const double* b_ov,
                    void* ws, hipStream_t st, double** pair_e) {
    const Mp2Layout L = mp2_layout(o, v);
    if (L.npair * L.ntp > ((int64_t)1 << 31) - 1) throw Error(-1, "MP2 grid too large");
    char* base = (char*)ws;
    std::vector<int2> pairs, tiles;
    for (int i = 0; i < o; ++i)
        for (int j = i; j < o; ++j) pairs.push_back(make_int2(i, j));
    const int nt = ceil_div(v, M_T);
    for (int a = 0; a < nt; ++a)
        for (int b = a; b < nt; ++b) tiles.push_back(make_int2(a, b));
    BQC_HIP(hipMemcpyAsync(base + L.pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    BQC_HIP(hipMemcpyAsync(base + L.tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    double* partial = (double*)(base + L.partial);
    double* pe = (double*)(base + L.pair_e);
    double* e = (double*)(base + L.energy);
    hipLaunchKernelGGL(mp2_kernel, dim3((unsigned)(L.npair * L.ntp)), dim3(M_THREADS), 0, st, b_ov, eps_o, eps_v,
                       (const int2*)(base + L.pairs), (const int2*)(base + L.tiles), (int)L.ntp, o, v, naux,
                       partial);
    BQC_HIP(hipGetLastError());
    hipLaunchKernelGGL(segment_sum_kernel, dim3((unsigned)L.npair), dim3(256), 0, st, partial, L.ntp, pe);
    BQC_HIP(hipGetLastError());
    hipLaunchKernelGGL(segment_sum_kernel, dim3(1), dim3(256), 0, st, pe, L.npair, e);
    BQC_HIP(hipGetLastError());
    // the host tables are read by the copies above before this returns
    BQC_HIP(hipStreamSynchronize(st));
    if (pair_e) *pair_e = pe;
    return e;
}

}  // namespace bqc
