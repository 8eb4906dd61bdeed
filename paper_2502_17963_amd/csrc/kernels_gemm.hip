// Contraction kernels of the (T) energy (paper section 2.4.2, Eq. 2) for the
// FP64 and FP32 modes: MFMA 16x16x4 GEMMs on LDS-staged tiles.
//
// For an occupied triple (i, j, k) the six permuted terms of W are paired by
// the virtual index that neither factor of the particle product carries
// along a row of its GEMM.  With q the occupied index whose virtual y is held
// fixed and (P, u), (R, w) the other two pairs, each pair of terms is
//
//   H[y][u][w] = X_{PqR}(u, y, w) + X_{RqP}(w, y, u)
//              = sum_K Row[y][u][K] * Col[y][w][K],   K over 4 segments:
//     seg 0 (v): Row = (Pu|yd)          Col = t_{Rq}^{wd}
//     seg 1 (o): Row = -(Pu|ql)         Col = t_{lR}^{yw}
//     seg 2 (v): Row = t_{Pq}^{ud}      Col = (Rw|yd)
//     seg 3 (o): Row = t_{lP}^{yu}      Col = -(Rw|ql)
// (X_pqr(x,y,z) = sum_d (px|yd) t_rq^zd - sum_l (px|ql) t_lr^yz.)  The three
// pairs are H_a (q=i, P=j, R=k), H_b (q=j, P=i, R=k), H_c (q=k, P=i, R=j), so
//   W[a][b][c] = H_a[a][b][c] + H_b[b][a][c] + H_c[c][a][b].
// In every segment exactly one factor depends on the plane index y; a work
// group computes G_NW consecutive planes (one per wave) of a 64 x 64 (u, w)
// tile and stages the plane-independent factor once in LDS for all waves.
#include "bqc_internal.h"

namespace bqc {
namespace {

constexpr int G_NW = 4;            // waves = planes per work group
constexpr int G_BM = 64;           // u rows per wave tile
constexpr int G_BN = 64;           // w cols per wave tile
constexpr int G_KC = 16;           // contraction elements per LDS stage
constexpr int G_LD = G_KC + 1;     // LDS row stride (elements), odd to spread banks
constexpr int G_ROWS = G_BM * (1 + G_NW);  // shared rows + per-wave rows
constexpr int G_THREADS = 64 * G_NW;
constexpr int G_PER_THREAD = G_ROWS * G_KC / G_THREADS;
static_assert(G_BM == G_BN, "shared and dependent tiles have the same row count");
static_assert(G_ROWS * G_KC % G_THREADS == 0, "stage loads divide evenly");

template <typename T>
struct Mfma;
// Operand layout of both 16x16x4 instructions: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16].  The accumulator layouts differ: register r of lane l
// holds D[row(l, r)][l % 16] with row = (l / 16) + 4 r for FP64 and
// row = 4 (l / 16) + r for FP32.
template <>
struct Mfma<double> {
    typedef double acc4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc4 op(double a, double b, acc4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef float acc4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc4 op(float a, float b, acc4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T>
struct Seg {
    const T* sh;       // plane-independent factor
    int64_t sh_row;
    const T* dep;      // plane-dependent factor
    int64_t dep_row, dep_plane;
    int len;
    bool dep_is_row;   // true: the dependent factor indexes u (rows); false: w (cols)
};

template <typename T>
__device__ __forceinline__ Seg<T> make_seg(int s, int o, int v, int q, int P, int R,
                                           const T* ovvv, const T* t2, const T* t2l,
                                           const T* hoo) {
    const int64_t v2 = (int64_t)v * v, v3 = v2 * v, vo = (int64_t)v * o;
    Seg<T> g;
    switch (s) {
        case 0:  // Row (Pu|yd) = ovvv[P][u][y][d];  Col t_Rq^wd = t2[R][q][w][d]
            g.dep = ovvv + P * v3; g.dep_row = v2; g.dep_plane = v; g.dep_is_row = true;
            g.sh = t2 + ((int64_t)R * o + q) * v2; g.sh_row = v; g.len = v;
            break;
        case 1:  // Row -(Pu|ql) = hoo[q][P][u][l];  Col t_lR^yw = t2l[R][y][w][l]
            g.sh = hoo + ((int64_t)q * o + P) * vo; g.sh_row = o;
            g.dep = t2l + R * v2 * o; g.dep_row = o; g.dep_plane = vo; g.dep_is_row = false;
            g.len = o;
            break;
        case 2:  // Row t_Pq^ud = t2[P][q][u][d];  Col (Rw|yd) = ovvv[R][w][y][d]
            g.sh = t2 + ((int64_t)P * o + q) * v2; g.sh_row = v;
            g.dep = ovvv + R * v3; g.dep_row = v2; g.dep_plane = v; g.dep_is_row = false;
            g.len = v;
            break;
        default:  // Row t_lP^yu = t2l[P][y][u][l];  Col -(Rw|ql) = hoo[q][R][w][l]
            g.dep = t2l + P * v2 * o; g.dep_row = o; g.dep_plane = vo; g.dep_is_row = true;
            g.sh = hoo + ((int64_t)q * o + R) * vo; g.sh_row = o;
            g.len = o;
            break;
    }
    return g;
}

// Occupied roles of pair h for triple (i, j, k): (q, P, R).
__device__ __forceinline__ void roles(int h, int i, int j, int k, int& q, int& P, int& R) {
    if (h == 0) { q = i; P = j; R = k; }
    else if (h == 1) { q = j; P = i; R = k; }
    else { q = k; P = i; R = j; }
}

template <typename T, typename HT>
__global__ __launch_bounds__(G_THREADS) void h_gemm_kernel(GemmLaunch g, int n_tiles,
                                                             int n_ut, int n_yg, int per_xcd) {
    // XCD-aware order: hardware block n runs on XCD n % 8; give each XCD a
    // contiguous range of logical tiles so tiles sharing a factor share an L2.
    const int n = blockIdx.x;
    const int L = (n % 8) * per_xcd + n / 8;
    if (L >= n_tiles) return;
    const int o = g.o, v = g.v;
    int rem = L;
    const int wt = rem % n_ut; rem /= n_ut;
    const int ut = rem % n_ut; rem /= n_ut;
    const int yg = rem % n_yg; rem /= n_yg;
    const int h = rem % 3;
    const int t = rem / 3;
    const int4 tr = g.trip[t];
    int q, P, R;
    roles(h, tr.x, tr.y, tr.z, q, P, R);

    const T* ovvv = (const T*)g.ops.ovvv;
    const T* t2 = (const T*)g.ops.t2;
    const T* t2l = (const T*)g.ops.t2l;
    const T* hoo = (const T*)g.ops.hoo;

    const int u0 = ut * G_BM, w0 = wt * G_BN, y0 = yg * G_NW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    __shared__ T lds[2][G_ROWS * G_LD];

    typedef typename Mfma<T>::acc4 acc4;
    acc4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = acc4{0, 0, 0, 0};

    // chunk bookkeeping: segments of length v, o, v, o in chunks of G_KC
    const int nch_v = ceil_div(v, G_KC), nch_o = ceil_div(o, G_KC);
    const int nch = 2 * nch_v + 2 * nch_o;
    auto chunk_seg = [&](int c, int& s, int& k0) {
        if (c < nch_v) { s = 0; k0 = c * G_KC; }
        else if (c < nch_v + nch_o) { s = 1; k0 = (c - nch_v) * G_KC; }
        else if (c < 2 * nch_v + nch_o) { s = 2; k0 = (c - nch_v - nch_o) * G_KC; }
        else { s = 3; k0 = (c - 2 * nch_v - nch_o) * G_KC; }
    };

    T reg[G_PER_THREAD];
    auto load = [&](int c) {
        int s, k0;
        chunk_seg(c, s, k0);
        const Seg<T> sg = make_seg<T>(s, o, v, q, P, R, ovvv, t2, t2l, hoo);
        const int sh0 = sg.dep_is_row ? w0 : u0;
        const int dp0 = sg.dep_is_row ? u0 : w0;
#pragma unroll
        for (int e = 0; e < G_PER_THREAD; ++e) {
            const int idx = tid + e * G_THREADS;
            const int row = idx / G_KC, kk = idx % G_KC, k = k0 + kk;
            T val = T(0);
            if (row < G_BM) {
                const int gr = sh0 + row;
                if (gr < v && k < sg.len) val = sg.sh[(int64_t)gr * sg.sh_row + k];
            } else {
                const int wv = (row - G_BM) / G_BM, r = (row - G_BM) % G_BM;
                const int gr = dp0 + r, y = y0 + wv;
                if (gr < v && y < v && k < sg.len)
                    val = sg.dep[(int64_t)y * sg.dep_plane + (int64_t)gr * sg.dep_row + k];
            }
            reg[e] = val;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < G_PER_THREAD; ++e) {
            const int idx = tid + e * G_THREADS;
            const int row = idx / G_KC, kk = idx % G_KC;
            lds[buf][row * G_LD + kk] = reg[e];
        }
    };

    load(0);
    store(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        if (c + 1 < nch) load(c + 1);
        int s, k0;
        chunk_seg(c, s, k0);
        const bool dep_row = (s == 0 || s == 3);
        const T* shb = &lds[c & 1][0];
        const T* dpb = &lds[c & 1][(G_BM + wave * G_BM) * G_LD];
        const T* A = dep_row ? dpb : shb;
        const T* B = dep_row ? shb : dpb;
#pragma unroll
        for (int ks = 0; ks < G_KC / 4; ++ks) {
            T af[4], bf[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
                af[mb] = A[(mb * 16 + (lane & 15)) * G_LD + ks * 4 + (lane >> 4)];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                bf[nb] = B[(nb * 16 + (lane & 15)) * G_LD + ks * 4 + (lane >> 4)];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = Mfma<T>::op(af[mb], bf[nb], acc[mb][nb]);
        }
        if (c + 1 < nch) store((c + 1) & 1);
        __syncthreads();
    }

    const int y = y0 + wave;
    if (y >= v) return;
    const int64_t v2 = (int64_t)v * v;
    HT* out = (HT*)g.hbuf + ((int64_t)(t * 3 + h) * v + y) * v2;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = u0 + mb * 16 + Mfma<T>::row(lane, r);
                const int w = w0 + nb * 16 + (lane & 15);
                if (u < v && w < v) out[(int64_t)u * v + w] = (HT)acc[mb][nb][r];
            }
}

}  // namespace

void launch_gemm_fp(int precision, const GemmLaunch& g, hipStream_t st) {
    const int n_ut = ceil_div(g.v, G_BM);
    const int n_yg = ceil_div(g.v, G_NW);
    const int64_t n_tiles64 = (int64_t)g.ntrip * 3 * n_yg * n_ut * n_ut;
    if (n_tiles64 > (int64_t)1 << 30) throw Error(-1, "contraction grid too large");
    const int n_tiles = (int)n_tiles64;
    const int per_xcd = ceil_div(n_tiles, 8);
    dim3 grid(per_xcd * 8), block(G_THREADS);
    if (precision == 0)
        hipLaunchKernelGGL((h_gemm_kernel<double, double>), grid, block, 0, st, g, n_tiles, n_ut,
                           n_yg, per_xcd);
    else
        hipLaunchKernelGGL((h_gemm_kernel<float, float>), grid, block, 0, st, g, n_tiles, n_ut,
                           n_yg, per_xcd);
    BQC_HIP(hipGetLastError());
}

}  // namespace bqc
