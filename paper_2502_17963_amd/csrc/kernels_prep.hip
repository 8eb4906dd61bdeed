// Device residency and precision conversion of the (T) inputs.
//
// The contraction kernels read every factor as rows that are contiguous along
// the contraction index.  (ia|bc) and t_ij^ab already are; the hole factors
// are re-laid out once per solve:
//   t2l[P][y][u][l] = t_lP^yu = t2[l][P][y][u]
//   hoo[q][P][u][l] = -(Pu|ql) = -ooov[q][l][P][u]
// and every factor is converted to the contraction precision.
#include "bqc_internal.h"

namespace bqc {

int operand_bytes(int precision) {
    switch (precision) {
        case 0: return 8;
        case 1: return 4;
        case 2: return 4;  // hi + lo bf16
        case 3: return 1;
        default: throw Error(-1, "unknown precision");
    }
}
int hbuf_bytes(int precision) { return precision == 0 ? 8 : 4; }

namespace {

constexpr int P_THREADS = 256;

inline dim3 grid_for(int64_t n) {
    int64_t b = (n + P_THREADS - 1) / P_THREADS;
    if (b > (int64_t)1 << 20) b = (int64_t)1 << 20;
    return dim3((unsigned)(b < 1 ? 1 : b));
}

// t2l[P][y][u][l] = s * t2[l][P][y][u]; output index runs l fastest.
template <typename T>
__global__ void make_t2l(const double* __restrict__ t2, T* __restrict__ out, int o, int v) {
    const int64_t n = (int64_t)o * o * v * v;
    const int64_t v2 = (int64_t)v * v;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(idx % o);
        const int64_t pyu = idx / o;  // (P, y, u) flattened: P * v^2 + y * v + u
        out[idx] = (T)t2[(int64_t)l * o * v2 + pyu];
    }
}

// hoo[q][P][u][l] = -ooov[q][l][P][u]
template <typename T>
__global__ void make_hoo(const double* __restrict__ ooov, T* __restrict__ out, int o, int v) {
    const int64_t n = (int64_t)o * o * v * o;
    const int64_t ov = (int64_t)o * v;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(idx % o);
        const int64_t rest = idx / o;       // (q, P, u)
        const int64_t pu = rest % ov;       // P * v + u
        const int64_t q = rest / ov;
        out[idx] = (T)(-ooov[(q * o + l) * ov + pu]);
    }
}

template <typename T>
__global__ void convert(const double* __restrict__ in, T* __restrict__ out, int64_t n) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x)
        out[idx] = (T)in[idx];
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int64_t prepare_bytes(int precision, int o, int v) {
    const int64_t n_ovvv = (int64_t)o * v * v * v, n_t2 = (int64_t)o * o * v * v;
    const int64_t n_t2l = n_t2, n_hoo = (int64_t)o * o * v * o;
    const int eb = operand_bytes(precision);
    int64_t b = 0;
    if (precision != 0) b += align256(n_ovvv * eb) + align256(n_t2 * eb);
    b += align256(n_t2l * eb) + align256(n_hoo * eb);
    if (precision == 3) {  // one scale byte per 32 contraction elements (rows padded)
        b += align256(n_ovvv / v * ceil_div(v, 32)) + align256(n_t2 / v * ceil_div(v, 32));
        b += align256(n_t2l / o * ceil_div(o, 32)) + align256(n_hoo / o * ceil_div(o, 32));
    }
    return b;
}

void launch_prepare_lowp(int precision, const DevInputs& in, void* ws, Operands* ops,
                         hipStream_t st);

void launch_prepare(int precision, const DevInputs& in, void* ws, Operands* ops, hipStream_t st) {
    const int o = in.o, v = in.v;
    const int64_t n_ovvv = (int64_t)o * v * v * v, n_t2 = (int64_t)o * o * v * v;
    const int64_t n_hoo = (int64_t)o * o * v * o;
    char* p = (char*)ws;
    if (precision == 0) {
        ops->ovvv = in.ovvv;
        ops->t2 = in.t2;
        double* t2l = (double*)p; p += align256(n_t2 * 8);
        double* hoo = (double*)p;
        hipLaunchKernelGGL(make_t2l<double>, grid_for(n_t2), dim3(P_THREADS), 0, st, in.t2, t2l, o, v);
        hipLaunchKernelGGL(make_hoo<double>, grid_for(n_hoo), dim3(P_THREADS), 0, st, in.ooov, hoo, o, v);
        ops->t2l = t2l;
        ops->hoo = hoo;
    } else if (precision == 1) {
        float* ovvv = (float*)p; p += align256(n_ovvv * 4);
        float* t2 = (float*)p; p += align256(n_t2 * 4);
        float* t2l = (float*)p; p += align256(n_t2 * 4);
        float* hoo = (float*)p;
        hipLaunchKernelGGL(convert<float>, grid_for(n_ovvv), dim3(P_THREADS), 0, st, in.ovvv, ovvv, n_ovvv);
        hipLaunchKernelGGL(convert<float>, grid_for(n_t2), dim3(P_THREADS), 0, st, in.t2, t2, n_t2);
        hipLaunchKernelGGL(make_t2l<float>, grid_for(n_t2), dim3(P_THREADS), 0, st, in.t2, t2l, o, v);
        hipLaunchKernelGGL(make_hoo<float>, grid_for(n_hoo), dim3(P_THREADS), 0, st, in.ooov, hoo, o, v);
        ops->ovvv = ovvv;
        ops->t2 = t2;
        ops->t2l = t2l;
        ops->hoo = hoo;
    } else {
        launch_prepare_lowp(precision, in, ws, ops, st);
    }
    BQC_HIP(hipGetLastError());
}

}  // namespace bqc
