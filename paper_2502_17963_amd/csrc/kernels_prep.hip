// Device residency and precision conversion of the (T) inputs.
//
// The contraction kernels stage every factor through LDS as row tiles of one
// 128-byte contraction chunk per row.  Each factor is therefore converted
// once per solve into a chunk-major layout: it is a set of matrices (M) of
// v rows (r), and for every 128-byte chunk (c) of the contraction index all
// rows are contiguous,
//     element (M, r, k) at  ((M * nchunk + k / KC) * v + r) * KC + k % KC,
// so that the operand tile of one stage (up to 160 consecutive rows) is one
// contiguous block.  The contraction index is zero-padded to Kv = roundup(v,
// KPAD) or Ko = roundup(o, KPAD).  The factors (matrix index -> rows, k):
//   ovvv_c  M = P*v + y:  r = u, k = d   (Pu|yd)
//   t2_c    M = P*o + q:  r = u, k = d   t_Pq^ud
//   t2l_c   M = P*v + y:  r = u, k = l   t_lP^yu = t2[l][P][y][u]
//   hoo_c   M = q*o + P:  r = u, k = l   -(Pu|ql) = -ooov[q][l][P][u]
// The loop over virtual triples uses the same four factors with the two
// orbital spaces exchanged: matrices of o rows (occupied u or w),
//   ovvv_c  M = A*v + B:  r = u, k = d   (uA|Bd)       = ovvv[u][A][B][d]
//   t2_c    M = y*v + A:  r = u, k = d   t_uy^Ad       = t2[u][y][A][d]
//   t2l_c   M = B*v + C:  r = w, k = l   t_lw^BC       = t2[l][w][B][C]
//   hoo_c   M = y*v + A:  r = u, k = l   -(uA|yl)      = -ooov[y][l][u][A]
// (the same element counts as the occupied-triple layout).
// KC = elements per 128-byte chunk: 16 (FP64), 32 (FP32), and for the
// split-BF16x3 mode a chunk holds 32 bf16 hi parts followed by their 32 lo
// parts (x_hi = bf16(x), x_lo = bf16(x - x_hi)).  The FP8 mode pads to 128
// and stores 128 e4m3 bytes per chunk row plus one E8M0 exponent per 32.
#include <algorithm>

#include "bqc_internal.h"

namespace bqc {

namespace {

constexpr int P_THREADS = 256;

inline dim3 grid_for(int64_t n) {
    int64_t b = (n + P_THREADS - 1) / P_THREADS;
    if (b > (int64_t)1 << 20) b = (int64_t)1 << 20;
    return dim3((unsigned)(b < 1 ? 1 : b));
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Round-to-nearest-even FP32 -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Source value of factor F at (matrix M, row r, contraction index k < len).
// F_V_*: the factors of the virtual-triple layout.
enum Factor { F_OVVV = 0, F_T2 = 1, F_T2L = 2, F_HOO = 3, F_V_OVVV = 4, F_V_T2 = 5, F_V_T2L = 6, F_V_HOO = 7 };

template <int F>
__device__ __forceinline__ double source(const double* __restrict__ src, int64_t M, int64_t r, int64_t k,
                                         int64_t o, int64_t v) {
    if constexpr (F == F_OVVV) {  // ovvv[P][u][y][d]
        const int64_t P = M / v, y = M % v;
        return src[((P * v + r) * v + y) * v + k];
    } else if constexpr (F == F_T2) {  // t2[P][q][u][d]
        return src[(M * v + r) * v + k];
    } else if constexpr (F == F_T2L) {  // t2[l][P][y][u]
        return src[k * o * v * v + M * v + r];
    } else if constexpr (F == F_HOO) {  // -ooov[q][l][P][u]
        const int64_t q = M / o, P = M % o;
        return -src[((q * o + k) * o + P) * v + r];
    } else if constexpr (F == F_V_OVVV) {  // ovvv[u][A][B][d], M = A v + B (src may start at a row block)
        return src[r * v * v * v + M * v + k];
    } else if constexpr (F == F_V_T2) {  // t2[u][y][A][d], M = y v + A
        return src[r * o * v * v + M * v + k];
    } else if constexpr (F == F_V_T2L) {  // t2[l][w][B][C], M = B v + C
        return src[(k * o + r) * v * v + M];
    } else {  // -ooov[y][l][u][A], M = y v + A
        const int64_t y = M / v, A = M % v;
        return -src[((y * o + k) * o + r) * v + A];
    }
}

// Rows of every matrix of factor F: v in the occupied-triple layout, o in
// the virtual-triple layout.
template <int F>
constexpr bool vir_factor() { return F >= F_V_OVVV; }

// One thread per destination element (chunk-major order) of the rows
// [row0, row0 + nrows) of every matrix (matrices of `rows` rows); the
// source is read at the row relative to row0.
template <int PREC, int F>
__device__ __forceinline__ void factor_elem(const double* __restrict__ src, void* dst, int64_t idx, int rows,
                                            int row0, int nrows, int nchunk, int len, int o, int v) {
    constexpr int KC = (PREC == 0) ? 16 : 32;
    {
        const int kk = (int)(idx % KC);
        int64_t rest = idx / KC;
        const int64_t r = rest % nrows; rest /= nrows;
        const int c = (int)(rest % nchunk);
        const int64_t M = rest / nchunk;
        const int k = c * KC + kk;
        const double x = k < len ? source<F>(src, M, r, k, o, v) : 0.0;
        const int64_t di = (((M * nchunk + c) * rows) + row0 + r) * KC + kk;  // destination element
        if constexpr (PREC == 0) {
            ((double*)dst)[di] = x;
        } else if constexpr (PREC == 1) {
            ((float*)dst)[di] = (float)x;
        } else {
            // chunk of 32 elements -> 32 hi parts then 32 lo parts
            uint16_t* d = (uint16_t*)dst + (di - kk) * 2;
            const uint16_t h = bf16_bits((float)x);
            d[kk] = h;
            d[32 + kk] = bf16_bits((float)(x - (double)bf16_value(h)));
        }
    }
}

template <int PREC, int F>
__global__ void make_factor(const double* __restrict__ src, void* dst, int64_t nmat, int rows, int row0,
                            int nrows, int len, int kpad, int o, int v) {
    constexpr int KC = (PREC == 0) ? 16 : 32;
    const int nchunk = kpad / KC;
    const int64_t n = nmat * nchunk * (int64_t)nrows * KC;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x)
        factor_elem<PREC, F>(src, dst, idx, rows, row0, nrows, nchunk, len, o, v);
}

// One factor of several solves in one launch: entry x covers blocks
// [x.b0, x.b0 + x.nb) and converts all rows of all its matrices.
template <int PREC, int F>
__global__ void make_factor_group(const FactorGroupEntry* __restrict__ ent, int nent) {
    constexpr int KC = (PREC == 0) ? 16 : 32;
    int lo = 0, hi = nent - 1;
    const int b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ent[mid].b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const FactorGroupEntry x = ent[lo];
    const int nchunk = x.kpad / KC;
    const int64_t n = x.nmat * nchunk * (int64_t)x.rows * KC;
    for (int64_t idx = (int64_t)(b - x.b0) * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)x.nb * blockDim.x)
        factor_elem<PREC, F>(x.src, x.dst, idx, x.rows, 0, x.rows, nchunk, x.len, x.o, x.v);
}

// OCP FP8 e4m3 (bias 7, max 448, no infinities) of y with round-to-nearest-
// even and saturation at 448.
__device__ __forceinline__ uint8_t e4m3_rne(double y) {
    const uint8_t sign = y < 0.0 ? 0x80 : 0;
    const double a = fabs(y);
    if (!(a < 464.0)) return sign | 0x7E;               // rounds above 448 (or NaN)
    if (a < 0.015625) {                                  // below 2^-6: subnormal, step 2^-9
        const int m = (int)rint(a * 512.0);              // 0..8 (8 is the smallest normal)
        return sign | (uint8_t)m;
    }
    int ex;
    const double f = frexp(a, &ex);                      // a = f 2^ex, f in [0.5, 1)
    int E = ex - 1;
    int m = (int)rint((2.0 * f - 1.0) * 8.0);            // 3-bit mantissa, may carry
    if (m == 8) { m = 0; E += 1; }
    if (E > 8 || (E == 8 && m == 7)) return sign | 0x7E;
    return sign | (uint8_t)(((E + 7) << 3) | m);
}

// FP8 factor: one thread per 32-element block of a (matrix, row, chunk):
// exponent e = ceil(log2(amax / 448)) (so every |x| 2^-e <= 448), stored as
// the E8M0 byte e + 127, and the 32 elements as e4m3(x 2^-e).
template <int F>
__global__ void make_factor_fp8(const double* __restrict__ src, uint8_t* dst, uint8_t* scl, int64_t nmat,
                                int len, int kpad, int o, int v) {
    const int nchunk = kpad / 128;
    const int64_t n = nmat * nchunk * (int64_t)v * 4;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx % 4);
        int64_t rest = idx / 4;
        const int64_t r = rest % v; rest /= v;
        const int c = (int)(rest % nchunk);
        const int64_t M = rest / nchunk;
        const int k0 = c * 128 + 32 * j;
        double amax = 0.0;
        for (int i = 0; i < 32; ++i)
            if (k0 + i < len) amax = fmax(amax, fabs(source<F>(src, M, r, k0 + i, o, v)));
        int e = -127;
        if (amax > 0.0) {
            int ex;
            const double fr = frexp(amax / 448.0, &ex);
            e = (fr == 0.5) ? ex - 1 : ex;
            e = e < -127 ? -127 : (e > 127 ? 127 : e);
        }
        const int64_t row = (M * nchunk + c) * (int64_t)v + r;
        scl[row * 4 + j] = (uint8_t)(e + 127);
        uint8_t* d = dst + row * 128 + 32 * j;
        for (int i = 0; i < 32; ++i) {
            const double x = k0 + i < len ? source<F>(src, M, r, k0 + i, o, v) : 0.0;
            d[i] = e4m3_rne(ldexp(x, -e));
        }
    }
}

template <int F>
void launch_factor_fp8(const double* src, void* dst, void* scl, int64_t nmat, int len, int kpad, int o,
                       int v, hipStream_t st) {
    const int64_t n = nmat * (int64_t)v * (kpad / 32);
    hipLaunchKernelGGL((make_factor_fp8<F>), grid_for(n), dim3(P_THREADS), 0, st, src, (uint8_t*)dst,
                       (uint8_t*)scl, nmat, len, kpad, o, v);
}

void prepare_fp8(const DevInputs& in, void* ws, Operands* ops, hipStream_t st);

// Density fitting of (ov|vv) (paper section 2.2) for the occupied indices
// P0 <= P < P0 + np:  out[P - P0][u][n] = sum_Q b_ov[Q][P][u] b_vv[Q][n],
// n = y v + d, i.e. out holds ovvv[P][u][y][d] for the block.  FP64 MFMA
// 16x16x4 on 64 x 64 (u, n) tiles, 16 values of Q staged through LDS per step.
constexpr int DF_T = 64, DF_K = 16;

__global__ __launch_bounds__(256) void df_ovvv_kernel(const double* __restrict__ b_ov,
                                                      const double* __restrict__ b_vv, double* __restrict__ out,
                                                      int o, int v, int naux, int P0) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    const int64_t v2 = (int64_t)v * v;
    const int64_t n0 = (int64_t)blockIdx.x * DF_T;
    const int u0 = blockIdx.y * DF_T, P = P0 + (int)blockIdx.z;
    __shared__ double As[DF_K][DF_T];  // As[k][u] = b_ov[Q0 + k][P][u0 + u]
    __shared__ double Bs[DF_K][DF_T];  // Bs[k][n] = b_vv[Q0 + k][n0 + n]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;  // this wave's 32 x 32 block
    const int fr = lane & 15, fg = lane >> 4;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
    for (int Q0 = 0; Q0 < naux; Q0 += DF_K) {
        double ra[4], rb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + 256 * i, k = idx / DF_T, m = idx % DF_T;
            const int Q = Q0 + k;
            ra[i] = (Q < naux && u0 + m < v) ? b_ov[((int64_t)Q * o + P) * v + u0 + m] : 0.0;
            rb[i] = (Q < naux && n0 + m < v2) ? b_vv[(int64_t)Q * v2 + n0 + m] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + 256 * i;
            As[idx / DF_T][idx % DF_T] = ra[i];
            Bs[idx / DF_T][idx % DF_T] = rb[i];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < DF_K / 4; ++s) {
            // operand of lane (fr, fg): row fr of the 16-block, contraction index 4 s + fg
            double a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = As[4 * s + fg][wm + 16 * x + fr];
                b[x] = Bs[4 * s + fg][wn + 16 * x + fr];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
    // FP64 accumulator layout: register r of lane l holds row (l / 16) + 4 r, column l % 16
    double* o_p = out + (int64_t)blockIdx.z * v * v2;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = u0 + wm + 16 * x + fg + 4 * r;
                const int64_t n = n0 + wn + 16 * y + fr;
                if (u < v && n < v2) o_p[(int64_t)u * v2 + n] = acc[x][y][r];
            }
}

void launch_df_ovvv(const DevInputs& in, int P0, int np, hipStream_t st) {
    const int64_t v2 = (int64_t)in.v * in.v;
    const dim3 grid((unsigned)((v2 + DF_T - 1) / DF_T), (unsigned)ceil_div(in.v, DF_T), (unsigned)np);
    hipLaunchKernelGGL(df_ovvv_kernel, grid, dim3(256), 0, st, in.b_ov, in.b_vv, in.df_tmp, in.o, in.v, in.naux,
                       P0);
    BQC_HIP(hipGetLastError());
}

}  // namespace


namespace {

template <int PREC, int F>
void launch_factor(const double* src, void* dst, int64_t nmat, int len, int kpad, int o, int v,
                   hipStream_t st, int row0 = 0, int nrows = -1) {
    const int rows = vir_factor<F>() ? o : v;
    if (nrows < 0) nrows = rows;
    const int64_t n = nmat * (int64_t)nrows * kpad;
    hipLaunchKernelGGL((make_factor<PREC, F>), grid_for(n), dim3(P_THREADS), 0, st, src, dst, nmat, rows, row0,
                       nrows, len, kpad, o, v);
}

// The factors of the virtual-triple layout (same byte sizes and order as
// those of prepare_t); with density fitting, (uA|Bd) is formed for a block
// of occupied u at a time and written to those rows of every matrix.
template <int PREC>
void prepare_vir(const DevInputs& in, void* ws, Operands* ops, hipStream_t st) {
    const int o = in.o, v = in.v;
    const Sizes z = factor_sizes(o, v, PREC);
    const int eb = operand_bytes(PREC);
    const int64_t vv = (int64_t)v * v, ov = (int64_t)o * v;
    char* p = (char*)ws;
    void* d_ovvv = p; p += align256((size_t)vv * o * z.Kv * eb);
    void* d_t2 = p;   p += align256((size_t)ov * o * z.Kv * eb);
    void* d_t2l = p;  p += align256((size_t)vv * o * z.Ko * eb);
    void* d_hoo = p;
    if (in.ovvv) {
        launch_factor<PREC, F_V_OVVV>(in.ovvv, d_ovvv, vv, v, z.Kv, o, v, st);
    } else {
        for (int P0 = 0; P0 < o; P0 += in.df_block) {
            const int np = std::min(in.df_block, o - P0);
            launch_df_ovvv(in, P0, np, st);
            launch_factor<PREC, F_V_OVVV>(in.df_tmp, d_ovvv, vv, v, z.Kv, o, v, st, P0, np);
        }
    }
    launch_factor<PREC, F_V_T2>(in.t2, d_t2, ov, v, z.Kv, o, v, st);
    launch_factor<PREC, F_V_T2L>(in.t2, d_t2l, vv, o, z.Ko, o, v, st);
    launch_factor<PREC, F_V_HOO>(in.ooov, d_hoo, ov, o, z.Ko, o, v, st);
    BQC_HIP(hipGetLastError());
    ops->ovvv = d_ovvv;
    ops->t2 = d_t2;
    ops->t2l = d_t2l;
    ops->hoo = d_hoo;
    ops->Kv = z.Kv;
    ops->Ko = z.Ko;
}

template <int PREC>
void prepare_t(const DevInputs& in, void* ws, Operands* ops, hipStream_t st) {
    const int o = in.o, v = in.v;
    const Sizes z = factor_sizes(o, v, PREC);
    const int eb = operand_bytes(PREC);
    char* p = (char*)ws;
    void* d_ovvv = p; p += align256((size_t)z.m_ovvv * v * z.Kv * eb);
    void* d_t2 = p;   p += align256((size_t)z.m_t2 * v * z.Kv * eb);
    void* d_t2l = p;  p += align256((size_t)z.m_t2l * v * z.Ko * eb);
    void* d_hoo = p;
    if (in.ovvv) {
        launch_factor<PREC, F_OVVV>(in.ovvv, d_ovvv, z.m_ovvv, v, z.Kv, o, v, st);
    } else {  // density fitting, df_block occupied planes at a time through the scratch
        for (int P0 = 0; P0 < o; P0 += in.df_block) {
            const int np = std::min(in.df_block, o - P0);
            launch_df_ovvv(in, P0, np, st);
            launch_factor<PREC, F_OVVV>(in.df_tmp, (char*)d_ovvv + (size_t)P0 * v * v * z.Kv * eb,
                                        (int64_t)np * v, v, z.Kv, o, v, st);
        }
    }
    launch_factor<PREC, F_T2>(in.t2, d_t2, z.m_t2, v, z.Kv, o, v, st);
    launch_factor<PREC, F_T2L>(in.t2, d_t2l, z.m_t2l, o, z.Ko, o, v, st);
    launch_factor<PREC, F_HOO>(in.ooov, d_hoo, z.m_hoo, o, z.Ko, o, v, st);
    BQC_HIP(hipGetLastError());
    ops->ovvv = d_ovvv;
    ops->t2 = d_t2;
    ops->t2l = d_t2l;
    ops->hoo = d_hoo;
    ops->Kv = z.Kv;
    ops->Ko = z.Ko;
}

void prepare_fp8(const DevInputs& in, void* ws, Operands* ops, hipStream_t st) {
    const int o = in.o, v = in.v;
    const Sizes z = factor_sizes(o, v, 3);
    char* p = (char*)ws;
    void* d_ovvv = p; p += align256((size_t)z.m_ovvv * v * z.Kv);
    void* d_t2 = p;   p += align256((size_t)z.m_t2 * v * z.Kv);
    void* d_t2l = p;  p += align256((size_t)z.m_t2l * v * z.Ko);
    void* d_hoo = p;  p += align256((size_t)z.m_hoo * v * z.Ko);
    void* s_ovvv = p; p += align256((size_t)z.m_ovvv * v * z.Kv / 32);
    void* s_t2 = p;   p += align256((size_t)z.m_t2 * v * z.Kv / 32);
    void* s_t2l = p;  p += align256((size_t)z.m_t2l * v * z.Ko / 32);
    void* s_hoo = p;
    if (in.ovvv) {
        launch_factor_fp8<F_OVVV>(in.ovvv, d_ovvv, s_ovvv, z.m_ovvv, v, z.Kv, o, v, st);
    } else {
        for (int P0 = 0; P0 < o; P0 += in.df_block) {
            const int np = std::min(in.df_block, o - P0);
            launch_df_ovvv(in, P0, np, st);
            launch_factor_fp8<F_OVVV>(in.df_tmp, (char*)d_ovvv + (size_t)P0 * v * v * z.Kv,
                                      (char*)s_ovvv + (size_t)P0 * v * v * z.Kv / 32, (int64_t)np * v, v, z.Kv,
                                      o, v, st);
        }
    }
    launch_factor_fp8<F_T2>(in.t2, d_t2, s_t2, z.m_t2, v, z.Kv, o, v, st);
    launch_factor_fp8<F_T2L>(in.t2, d_t2l, s_t2l, z.m_t2l, o, z.Ko, o, v, st);
    launch_factor_fp8<F_HOO>(in.ooov, d_hoo, s_hoo, z.m_hoo, o, z.Ko, o, v, st);
    BQC_HIP(hipGetLastError());
    ops->ovvv = d_ovvv; ops->t2 = d_t2; ops->t2l = d_t2l; ops->hoo = d_hoo;
    ops->ovvv_s = (const uint32_t*)s_ovvv; ops->t2_s = (const uint32_t*)s_t2;
    ops->t2l_s = (const uint32_t*)s_t2l; ops->hoo_s = (const uint32_t*)s_hoo;
    ops->Kv = z.Kv;
    ops->Ko = z.Ko;
}

}  // namespace

template <int PREC>
void prepare_group_t(int n, const DevInputs* ins, void* const* ws, Operands* ops, FactorGroupEntry* d_tables,
                     std::vector<FactorGroupEntry>& tables, hipStream_t st) {
    tables.assign((size_t)4 * n, FactorGroupEntry{});
    const int eb = operand_bytes(PREC);
    int nblocks[4] = {0, 0, 0, 0};
    for (int f = 0; f < n; ++f) {
        const DevInputs& in = ins[f];
        const int o = in.o, v = in.v;
        const Sizes z = factor_sizes(o, v, PREC);
        char* p = (char*)ws[f];
        void* dst[4];
        dst[0] = p; p += align256((size_t)z.m_ovvv * v * z.Kv * eb);
        dst[1] = p; p += align256((size_t)z.m_t2 * v * z.Kv * eb);
        dst[2] = p; p += align256((size_t)z.m_t2l * v * z.Ko * eb);
        dst[3] = p;
        const double* src[4] = {in.ovvv, in.t2, in.t2, in.ooov};
        const int64_t nmat[4] = {z.m_ovvv, z.m_t2, z.m_t2l, z.m_hoo};
        const int len[4] = {v, v, o, o}, kpad[4] = {z.Kv, z.Kv, z.Ko, z.Ko};
        for (int k = 0; k < 4; ++k) {
            FactorGroupEntry& x = tables[(size_t)k * n + f];
            x.src = src[k]; x.dst = dst[k]; x.nmat = nmat[k]; x.rows = v; x.len = len[k]; x.kpad = kpad[k];
            x.o = o; x.v = v;
            const int64_t elems = nmat[k] * (int64_t)v * kpad[k];
            x.nb = (int)std::max<int64_t>(1, std::min<int64_t>((elems + P_THREADS - 1) / P_THREADS, 4096));
            x.b0 = nblocks[k];
            nblocks[k] += x.nb;
        }
        ops[f].ovvv = dst[0]; ops[f].t2 = dst[1]; ops[f].t2l = dst[2]; ops[f].hoo = dst[3];
        ops[f].Kv = z.Kv; ops[f].Ko = z.Ko;
    }
    BQC_HIP(hipMemcpyAsync(d_tables, tables.data(), tables.size() * sizeof(FactorGroupEntry), hipMemcpyHostToDevice,
                           st));
    hipLaunchKernelGGL((make_factor_group<PREC, F_OVVV>), dim3(nblocks[0]), dim3(P_THREADS), 0, st, d_tables, n);
    hipLaunchKernelGGL((make_factor_group<PREC, F_T2>), dim3(nblocks[1]), dim3(P_THREADS), 0, st, d_tables + n, n);
    hipLaunchKernelGGL((make_factor_group<PREC, F_T2L>), dim3(nblocks[2]), dim3(P_THREADS), 0, st, d_tables + 2 * n, n);
    hipLaunchKernelGGL((make_factor_group<PREC, F_HOO>), dim3(nblocks[3]), dim3(P_THREADS), 0, st, d_tables + 3 * n, n);
    BQC_HIP(hipGetLastError());
}

void launch_prepare(int precision, const DevInputs& in, void* ws, Operands* ops, hipStream_t st, int form) {
    if (form == FORM_VIR) {
        switch (precision) {
            case 0: prepare_vir<0>(in, ws, ops, st); return;
            case 1: prepare_vir<1>(in, ws, ops, st); return;
            case 2: prepare_vir<2>(in, ws, ops, st); return;
            default: throw Error(-1, "the virtual-triple loop runs in FP64, FP32 or split-BF16x3");
        }
    }
    switch (precision) {
        case 0: prepare_t<0>(in, ws, ops, st); break;
        case 1: prepare_t<1>(in, ws, ops, st); break;
        case 2: prepare_t<2>(in, ws, ops, st); break;
        case 3: prepare_fp8(in, ws, ops, st); break;
        default: throw Error(-1, "unknown precision");
    }
}

// ------------------------------------------------------------------ virtual-triple epilogue inputs
namespace {

// dst[e] for e < n: the transposes of the epilogue's inputs (one thread per
// destination element).  kind 0: dst[a][i] = src[i][a] (t1, f_ov; o x v
// source); 1: dst[a][b][i][j] = src[i][a][j][b] ((ia|jb)); 2: dst[a][b][i][j]
// = src[i][j][a][b] (t2); 3: dst[x] = -src[x].
__global__ void vir_aux_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n, int kind,
                               int o, int v) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t si;
        if (kind == 0) {
            const int64_t a = e / o, i = e % o;
            si = i * v + a;
        } else if (kind == 1 || kind == 2) {  // destination [a][b][i][j]
            int64_t r = e;
            const int64_t j = r % o; r /= o;
            const int64_t i = r % o; r /= o;
            const int64_t b = r % v;
            const int64_t a = r / v;
            si = kind == 1 ? ((i * v + a) * o + j) * v + b : ((i * o + j) * v + a) * v + b;
        } else {
            dst[e] = -src[e];
            continue;
        }
        dst[e] = src[si];
    }
}

void launch_aux(const double* src, double* dst, int64_t n, int kind, int o, int v, hipStream_t st) {
    hipLaunchKernelGGL(vir_aux_kernel, grid_for(n), dim3(P_THREADS), 0, st, src, dst, n, kind, o, v);
    BQC_HIP(hipGetLastError());
}

}  // namespace

VirAux launch_vir_aux(const DevInputs& in, void* aux, hipStream_t st) {
    const int o = in.o, v = in.v;
    const int64_t ov = (int64_t)o * v;
    char* p = (char*)aux;
    VirAux x;
    x.neg_eps_v = (double*)p; p += align256(v * 8);
    x.neg_eps_o = (double*)p; p += align256(o * 8);
    x.t1_t = (double*)p;      p += align256(ov * 8);
    x.ovov_t = (double*)p;    p += align256(ov * ov * 8);
    launch_aux(in.eps_v, x.neg_eps_v, v, 3, o, v, st);
    launch_aux(in.eps_o, x.neg_eps_o, o, 3, o, v, st);
    launch_aux(in.t1, x.t1_t, ov, 0, o, v, st);
    launch_aux(in.ovov, x.ovov_t, ov * ov, 1, o, v, st);
    if (in.fock_ov) {
        x.t2_t = (double*)p;   p += align256(ov * ov * 8);
        x.fock_t = (double*)p;
        launch_aux(in.t2, x.t2_t, ov * ov, 2, o, v, st);
        launch_aux(in.fock_ov, x.fock_t, ov, 0, o, v, st);
    }
    return x;
}

void launch_prepare_group(int precision, int n, const DevInputs* ins, void* const* ws, Operands* ops,
                          FactorGroupEntry* d_tables, std::vector<FactorGroupEntry>& tables, hipStream_t st) {
    switch (precision) {
        case 0: prepare_group_t<0>(n, ins, ws, ops, d_tables, tables, st); return;
        case 1: prepare_group_t<1>(n, ins, ws, ops, d_tables, tables, st); return;
        case 2: prepare_group_t<2>(n, ins, ws, ops, d_tables, tables, st); return;
        default:  // FP8 factors have their own converter: one launch set per solve
            for (int f = 0; f < n; ++f) launch_prepare(precision, ins[f], ws[f], &ops[f], st);
            return;
    }
}

}  // namespace bqc
