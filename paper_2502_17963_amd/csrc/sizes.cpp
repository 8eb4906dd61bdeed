// Host-side sizes of a solve's device buffers: operand element sizes and
// paddings, the contraction operands' bytes, the density-fitting scratch,
// the transposes of the loop over virtual triples and the contraction's
// tiling.  Host code only (no kernels), so the layout arithmetic is shared
// by the library and by the host-side tests that run the solve driver
// against a stand-in runtime.
#include <algorithm>

#include "bqc_internal.h"

namespace bqc {

namespace {
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

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
int chunk_elems(int precision) { return 128 / operand_bytes(precision); }
int kpad_of(int precision) { return precision == 3 ? 128 : KPAD; }

int df_block_planes(int o, int v) {
    const int64_t v3 = (int64_t)v * v * v;
    const int64_t cap = (int64_t)1 << 26;  // 512 MB of FP64 scratch
    int64_t b = cap / std::max<int64_t>(v3, 1);
    b = std::max<int64_t>(1, std::min<int64_t>(b, o));
    return (int)b;
}
int64_t df_scratch_elems(int o, int v) { return (int64_t)df_block_planes(o, v) * v * v * v; }


Sizes factor_sizes(int o, int v, int precision) {
    const int kp = kpad_of(precision);
    Sizes s;
    s.Kv = ceil_div(v, kp) * kp;
    s.Ko = ceil_div(o, kp) * kp;
    s.m_ovvv = (int64_t)o * v;
    s.m_t2 = (int64_t)o * o;
    s.m_t2l = (int64_t)o * v;
    s.m_hoo = (int64_t)o * o;
    return s;
}

int64_t prepare_bytes(int precision, int o, int v) {
    const Sizes z = factor_sizes(o, v, precision);
    const int eb = operand_bytes(precision);
    int64_t b = align256((size_t)z.m_ovvv * v * z.Kv * eb) + align256((size_t)z.m_t2 * v * z.Kv * eb) +
                align256((size_t)z.m_t2l * v * z.Ko * eb) + align256((size_t)z.m_hoo * v * z.Ko * eb);
    if (precision == 3) {  // one scale byte per 32 contraction elements
        b += align256((size_t)z.m_ovvv * v * z.Kv / 32) + align256((size_t)z.m_t2 * v * z.Kv / 32) +
             align256((size_t)z.m_t2l * v * z.Ko / 32) + align256((size_t)z.m_hoo * v * z.Ko / 32);
    }
    return b;
}

Tiling contraction_tiling(int n, int wb, int ntrip) {
    Tiling t;
    t.nblk = ceil_div(n, 16);
    t.ntile_u = ceil_div(t.nblk, 2 * wb);
    t.ntile_w = ceil_div(t.nblk, 2 * wb);
    t.n_wg = (int64_t)ntrip * 3 * n * t.ntile_u * t.ntile_w;
    return t;
}

int64_t vir_aux_bytes(int o, int v, bool fock) {
    const int64_t ov = (int64_t)o * v;
    int64_t b = align256(v * 8) + align256(o * 8) + align256(ov * 8) + align256(ov * ov * 8);
    if (fock) b += align256(ov * ov * 8) + align256(ov * 8);
    return b;
}

}  // namespace bqc
