// Contraction kernels of the (T) energy (paper section 2.4.2, Eq. 2):
// MFMA GEMMs on LDS-staged tiles in FP64, FP32, split-BF16x3 and FP8.
//
// For an occupied triple (i, j, k) the six permuted terms of W are paired so
// that both members of a pair hold the same virtual index y fixed.  With q
// the occupied index carrying y and (P, u), (R, w) the other two pairs,
//
//   H[y][u][w] = X_{PqR}(u, y, w) + X_{RqP}(w, y, u)
//              = sum_K Row[y][u][K] * Col[y][w][K],   K over four segments:
//     seg 0 (v): Row = (Pu|yd)          Col = t_{Rq}^{wd}
//     seg 1 (o): Row = -(Pu|ql)         Col = t_{lR}^{yw}
//     seg 2 (v): Row = t_{Pq}^{ud}      Col = (Rw|yd)
//     seg 3 (o): Row = t_{lP}^{yu}      Col = -(Rw|ql)
// where X_pqr(x,y,z) = sum_d (px|yd) t_rq^zd - sum_l (px|ql) t_lr^yz.  The
// three pairs are H_a (q=i, P=j, R=k), H_b (q=j, P=i, R=k) and
// H_c (q=k, P=i, R=j), so that W[a][b][c] = H_a[a][b][c] + H_b[b][a][c] +
// H_c[c][a][b].  Particle and hole terms therefore run on the same MFMA
// tiles (K = 2v + 2o per plane).
//
// The loop over virtual triples (a, b, c) is the same computation with the
// two orbital spaces exchanged: with X^{pqr}(x,y,z) = sum_d (xp|qd) t_zy^rd
// - sum_l (xp|yl) t_lz^qr over occupied x, y, z, the pair of the virtual
// roles (B middle, A, C) is
//   H[y][u][w] = X^{ABC}(u, y, w) + X^{CBA}(w, y, u)     (y, u, w occupied)
//     seg 0 (v): Row = (uA|Bd)        Col = t_{wy}^{Cd}
//     seg 1 (o): Row = -(uA|yl)       Col = t_{lw}^{BC}
//     seg 2 (v): Row = t_{uy}^{Ad}    Col = (wC|Bd)
//     seg 3 (o): Row = t_{lu}^{BA}    Col = -(wC|yl)
// with (B, A, C) = (a, b, c), (b, a, c), (c, a, b) for the three pairs, so
// that W^{ijk} = H_a[i][j][k] + H_b[j][i][k] + H_c[k][i][j]: the same
// kernel with planes, rows and columns over the occupied indices and the
// operand matrices of the virtual-triple layout (FORM = 1).
//
// Work decomposition: one work group = one plane y of one pair of one
// triple, and a tile of up to 160 x 160 (u, w).  The 16-row blocks of v are
// split evenly over the tiles (v = 300: 19 blocks -> 10 + 9), and each of the
// four waves owns up to 5 x 5 blocks.  A wave always runs all 25 block
// products (rows past the tile are zero in LDS and their results are not
// stored): a branch per MFMA would cost more than the idle blocks.  Operands are staged through LDS in
// stages of 128 bytes per row (8 16-byte vectors, swizzled so that the
// fragment reads are free of bank conflicts), double-buffered through
// registers.  Within a stage, MFMA lane group g (lanes 16g..16g+15) takes
// the 16-byte units g and 4+g of each staged row (two 16-byte LDS reads per
// fragment, free of bank conflicts); A and B use the same assignment, so
// every element of the stage is contracted exactly once.
#include "bqc_internal.h"

namespace bqc {
namespace {

constexpr int ROWB = 128;              // bytes per LDS row and stage

// Work-group geometry: WU x WW waves, each owning up to WB x WB 16x16 blocks,
// so a tile covers up to WU*WB*16 rows u and WW*WB*16 columns w.
template <int WU_, int WW_, int WB_>
struct Geo {
    static constexpr int WU = WU_, WW = WW_, WB = WB_;
    static constexpr int TILE_U = WU * WB * 16, TILE_W = WW * WB * 16;
    static constexpr int NROW = TILE_U + TILE_W;       // LDS rows: Row factor, then Col factor
    static constexpr int NTHR = 64 * WU * WW;
    static constexpr int NVEC = (NROW * 8 + NTHR - 1) / NTHR;  // 16-byte vectors per thread per stage
};

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// Mode traits.  E = element type in memory, KC = contraction elements per stage.
template <int PREC>
struct Mode;
template <>
struct Mode<0> {  // FP64 operands, FP64 MFMA 16x16x4
    typedef double E;
    typedef d4 Acc;
    typedef double HT;
    static constexpr int KC = 16;
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mode<1> {  // FP32 operands, FP32 MFMA 16x16x4
    typedef float E;
    typedef f4 Acc;
    typedef float HT;
    static constexpr int KC = 32;
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mode<2> {  // bf16 hi/lo operands, bf16 MFMA 16x16x32, three products
    typedef uint16_t E;
    typedef f4 Acc;
    typedef float HT;
    static constexpr int KC = 32;
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct Mode<3> {  // FP8 e4m3 operands, E8M0 scale per 32 elements, MX-scaled MFMA 16x16x128
    typedef uint8_t E;
    typedef f4 Acc;
    typedef float HT;
    static constexpr int KC = 128;
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

typedef int i8v __attribute__((ext_vector_type(8)));

// Byte offset of 16-byte vector q of LDS row r (XOR swizzle by row pair).
__device__ __forceinline__ int lds_off(int r, int q) { return r * ROWB + ((q ^ ((r >> 1) & 7)) << 4); }

// Balanced split of nblk 16-blocks into ntile parts.
__device__ __forceinline__ void tile_range(int t, int nblk, int ntile, int& start, int& count) {
    const int base = nblk / ntile, extra = nblk % ntile;
    start = t * base + min(t, extra);
    count = base + (t < extra ? 1 : 0);
}

// Matrices and chunk counts of the two factors of segment s (see the
// operand layout in bqc_internal.h).
struct SegGeom {
    int64_t row_mat, col_mat;
    int nchunk;           // contraction chunks of the segment
    int arr_row, arr_col; // 0 ovvv, 1 t2, 2 t2l, 3 hoo
};

__device__ __forceinline__ SegGeom seg_geom(int s, int o, int v, int nch_v, int nch_o, int q, int P, int R,
                                            int y) {
    SegGeom g;
    switch (s) {
        case 0:  // Row (Pu|yd): ovvv[P*v+y]   Col t_Rq^wd: t2[R*o+q]
            g.row_mat = (int64_t)P * v + y; g.arr_row = 0;
            g.col_mat = (int64_t)R * o + q; g.arr_col = 1;
            g.nchunk = nch_v;
            break;
        case 1:  // Row -(Pu|ql): hoo[q*o+P]   Col t_lR^yw: t2l[R*v+y]
            g.row_mat = (int64_t)q * o + P; g.arr_row = 3;
            g.col_mat = (int64_t)R * v + y; g.arr_col = 2;
            g.nchunk = nch_o;
            break;
        case 2:  // Row t_Pq^ud: t2[P*o+q]     Col (Rw|yd): ovvv[R*v+y]
            g.row_mat = (int64_t)P * o + q; g.arr_row = 1;
            g.col_mat = (int64_t)R * v + y; g.arr_col = 0;
            g.nchunk = nch_v;
            break;
        default:  // Row t_lP^yu: t2l[P*v+y]   Col -(Rw|ql): hoo[q*o+R]
            g.row_mat = (int64_t)P * v + y; g.arr_row = 2;
            g.col_mat = (int64_t)q * o + R; g.arr_col = 3;
            g.nchunk = nch_o;
            break;
    }
    return g;
}

// The same for the loop over virtual triples: q = B, P = A, R = C (virtual),
// y the occupied plane; matrices of the virtual-triple layout (bqc_internal.h).
__device__ __forceinline__ SegGeom seg_geom_vir(int s, int v, int nch_v, int nch_o, int B, int A, int C,
                                                int y) {
    SegGeom g;
    switch (s) {
        case 0:  // Row (uA|Bd): ovvv[A*v+B]     Col t_wy^Cd: t2[y*v+C]
            g.row_mat = (int64_t)A * v + B; g.arr_row = 0;
            g.col_mat = (int64_t)y * v + C; g.arr_col = 1;
            g.nchunk = nch_v;
            break;
        case 1:  // Row -(uA|yl): hoo[y*v+A]     Col t_lw^BC: t2l[B*v+C]
            g.row_mat = (int64_t)y * v + A; g.arr_row = 3;
            g.col_mat = (int64_t)B * v + C; g.arr_col = 2;
            g.nchunk = nch_o;
            break;
        case 2:  // Row t_uy^Ad: t2[y*v+A]       Col (wC|Bd): ovvv[C*v+B]
            g.row_mat = (int64_t)y * v + A; g.arr_row = 1;
            g.col_mat = (int64_t)C * v + B; g.arr_col = 0;
            g.nchunk = nch_v;
            break;
        default:  // Row t_lu^BA: t2l[B*v+A]     Col -(wC|yl): hoo[y*v+C]
            g.row_mat = (int64_t)B * v + A; g.arr_row = 2;
            g.col_mat = (int64_t)y * v + C; g.arr_col = 3;
            g.nchunk = nch_o;
            break;
    }
    return g;
}

__device__ __forceinline__ const char* arr_base(const Operands& ops, int a) {
    const void* p = a == 0 ? ops.ovvv : a == 1 ? ops.t2 : a == 2 ? ops.t2l : ops.hoo;
    return (const char*)p;
}
__device__ __forceinline__ const uint32_t* scale_base(const Operands& ops, int a) {
    return a == 0 ? ops.ovvv_s : a == 1 ? ops.t2_s : a == 2 ? ops.t2l_s : ops.hoo_s;
}

__device__ __forceinline__ void roles(int h, int i, int j, int k, int& q, int& P, int& R) {
    if (h == 0) { q = i; P = j; R = k; }
    else if (h == 1) { q = j; P = i; R = k; }
    else { q = k; P = i; R = j; }
}

// The fragments of one staged chunk for one wave (FP64, FP32, split-BF16x3):
// A fragments from LDS rows arow0 + 16 m + (lane % 16), B fragments from
// rows brow0 + 16 n + (lane % 16), read by read() and multiplied by mfma(),
// so that a caller can issue other work between the two.
template <int PREC, int WB>
struct StageFrags {
    typedef typename Mode<PREC>::E E;
    static constexpr int NS = (PREC == 0) ? 4 : 8;  // MFMA K-steps per stage
    E af[WB][NS], bfr[WB][NS];
    __device__ __forceinline__ void read(const char* L0, int arow0, int brow0, int fr, int fg) {
#pragma unroll
        for (int m = 0; m < WB; ++m) {
            const int ra = arow0 + m * 16 + fr, rb = brow0 + m * 16 + fr;
            const u4 a0 = *(const u4*)(L0 + lds_off(ra, fg));
            const u4 a1 = *(const u4*)(L0 + lds_off(ra, 4 + fg));
            const u4 b0 = *(const u4*)(L0 + lds_off(rb, fg));
            const u4 b1 = *(const u4*)(L0 + lds_off(rb, 4 + fg));
            const E* pa0 = (const E*)&a0; const E* pa1 = (const E*)&a1;
            const E* pb0 = (const E*)&b0; const E* pb1 = (const E*)&b1;
#pragma unroll
            for (int s = 0; s < NS / 2; ++s) {
                af[m][s] = pa0[s]; af[m][NS / 2 + s] = pa1[s];
                bfr[m][s] = pb0[s]; bfr[m][NS / 2 + s] = pb1[s];
            }
        }
    }
    __device__ __forceinline__ void mfma(typename Mode<PREC>::Acc (&acc)[WB][WB]) const {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int m = 0; m < WB; ++m)
#pragma unroll
                for (int nn = 0; nn < WB; ++nn) {
                    if constexpr (PREC == 0)
                        acc[m][nn] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[m][s], bfr[nn][s], acc[m][nn], 0, 0, 0);
                    else
                        acc[m][nn] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[m][s], bfr[nn][s], acc[m][nn], 0, 0, 0);
                }
    }
};
// split-BF16x3: per accumulator lo*hi, then hi*lo, then hi*hi
template <int WB>
struct StageFrags<2, WB> {
    bf8 ah[WB], al[WB], bh[WB], bl[WB];
    __device__ __forceinline__ void read(const char* L0, int arow0, int brow0, int fr, int fg) {
#pragma unroll
        for (int m = 0; m < WB; ++m) {
            const int ra = arow0 + m * 16 + fr, rb = brow0 + m * 16 + fr;
            ah[m] = *(const bf8*)(L0 + lds_off(ra, fg));
            al[m] = *(const bf8*)(L0 + lds_off(ra, 4 + fg));
            bh[m] = *(const bf8*)(L0 + lds_off(rb, fg));
            bl[m] = *(const bf8*)(L0 + lds_off(rb, 4 + fg));
        }
    }
    __device__ __forceinline__ void mfma(f4 (&acc)[WB][WB]) const {
#pragma unroll
        for (int m = 0; m < WB; ++m)
#pragma unroll
            for (int nn = 0; nn < WB; ++nn)
                acc[m][nn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[m], bh[nn], acc[m][nn], 0, 0, 0);
#pragma unroll
        for (int m = 0; m < WB; ++m)
#pragma unroll
            for (int nn = 0; nn < WB; ++nn)
                acc[m][nn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], bl[nn], acc[m][nn], 0, 0, 0);
#pragma unroll
        for (int m = 0; m < WB; ++m)
#pragma unroll
            for (int nn = 0; nn < WB; ++nn)
                acc[m][nn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], bh[nn], acc[m][nn], 0, 0, 0);
    }
};

// The MFMA products of one staged chunk for one wave: WB x WB 16 x 16
// blocks, A fragments from LDS rows arow0 + 16 m + (lane % 16), B fragments
// from rows brow0 + 16 n + (lane % 16) of the stage at L0 (FP8: exponent
// words of the staged rows at Ls).
template <int PREC, int WB>
__device__ __forceinline__ void stage_products(typename Mode<PREC>::Acc (&acc)[WB][WB], const char* L0,
                                               const uint32_t* Ls, int arow0, int brow0, int fr, int fg) {
    if constexpr (PREC == 3) {
        // The FP8 16x16x128 MFMA reads lane group g's 32 bytes as
        // contraction elements [16g, 16g+16) and [64+16g, 64+16g+16) and
        // takes from lane group g the exponent of elements [32g, 32g+32).
        // Feeding units g and 4+g of the staged row places every staged
        // 32-element block b (units 2b, 2b+1) exactly in the MFMA's block
        // b, whose exponent, byte b of the row's scale word, group b holds.
        i8v af[WB], bfr[WB];
        int sa[WB], sb[WB];
#pragma unroll
        for (int m = 0; m < WB; ++m) {
            const int ra = arow0 + m * 16 + fr, rb = brow0 + m * 16 + fr;
            const u4 a0 = *(const u4*)(L0 + lds_off(ra, fg));
            const u4 a1 = *(const u4*)(L0 + lds_off(ra, 4 + fg));
            const u4 b0 = *(const u4*)(L0 + lds_off(rb, fg));
            const u4 b1 = *(const u4*)(L0 + lds_off(rb, 4 + fg));
            af[m] = i8v{(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
            bfr[m] = i8v{(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
            sa[m] = (int)((Ls[ra] >> (8 * fg)) & 0xffu);
            sb[m] = (int)((Ls[rb] >> (8 * fg)) & 0xffu);
        }
#pragma unroll
        for (int m = 0; m < WB; ++m)
#pragma unroll
            for (int nn = 0; nn < WB; ++nn)
                acc[m][nn] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(af[m], bfr[nn], acc[m][nn], 0, 0,
                                                                              0, sa[m], 0, sb[nn]);
    } else {
        StageFrags<PREC, WB> f;
        f.read(L0, arow0, brow0, fr, fg);
        f.mfma(acc);
    }
}

// The work of logical work group L of one contraction launch of g (the
// launch's tiles are nblk 16-blocks split into ntile_u x ntile_w tiles).
// Store of a wave's WB x WB accumulator blocks into one plane of a blocked H
// buffer (element (u, w) of the plane at out + (u / 8) nt 512 + (u % 8) 8 +
// (w / 8) 512 + w % 8) when the whole wave tile lies inside the plane and
// the plane's offsets fit 32 bits: one byte offset per lane and row slot r,
// stepped by block (uniform strides), and no masks.  Returns false (nothing
// stored) otherwise; the caller then stores element by element.
template <class M, int WB, class Acc, class HT>
__device__ __forceinline__ bool store_tile_fast(const Acc (&acc)[WB][WB], HT* out, int n, int nt, int u00, int w00,
                                                int wun, int wwn, int lane) {
    const int64_t rowblk = (int64_t)nt * 512;  // elements from one 8-row group to the next
    const bool full = wun == WB && wwn == WB && u00 + 16 * WB <= n && w00 + 16 * WB <= n &&
                      (int64_t)nt * nt * 512 * (int64_t)sizeof(HT) < ((int64_t)1 << 31);
    if (!full) return false;
    const int fr = lane & 15;
    const int w = w00 + fr;
    const uint32_t wbyte = (uint32_t)(((w >> 3) * 512 + (w & 7)) * (int)sizeof(HT));
    uint32_t roff[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int u = u00 + M::row(lane, r);
        roff[r] = (uint32_t)(((u >> 3) * rowblk + (u & 7) * 8) * (int64_t)sizeof(HT)) + wbyte;
    }
    const uint32_t mstep = (uint32_t)(2 * rowblk * (int64_t)sizeof(HT));  // 16 rows
    constexpr uint32_t nstep = 2 * 512 * sizeof(HT);                      // 16 columns
    char* base = (char*)out;
#pragma unroll
    for (int m = 0; m < WB; ++m)
#pragma unroll
        for (int nn = 0; nn < WB; ++nn)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                *(HT*)(base + (roff[r] + m * mstep + nn * nstep)) = (HT)acc[m][nn][r];
    return true;
}

// The wave's tile of plane y of pair slot `pair` (triple t, pair h: 3 t + h)
// into its blocked H buffer (layout in bqc_internal.h): the unmasked store
// when the whole wave tile lies inside the plane, else element by element.
template <class M, int WB, class Acc>
__device__ __forceinline__ void store_plane_tile(const Acc (&acc)[WB][WB], void* hbuf, int n, int pair, int y,
                                                 int u00, int w00, int wun, int wwn, int lane) {
    typedef typename M::HT HT;
    const int nt = ceil_div(n, EPI_T);
    HT* out = (HT*)hbuf + (int64_t)pair * hpair_elems(n) + (int64_t)(y >> 3) * nt * nt * 512 + (y & 7) * 64;
    if (store_tile_fast<M, WB>(acc, out, n, nt, u00, w00, wun, wwn, lane)) return;
    const int fr = lane & 15;
#pragma unroll
    for (int m = 0; m < WB; ++m)
#pragma unroll
        for (int nn = 0; nn < WB; ++nn)
            if (m < wun && nn < wwn) {
                const int w = w00 + nn * 16 + fr;
                const int wo = (w >> 3) * 512 + (w & 7);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int u = u00 + m * 16 + M::row(lane, r);
                    if (u < n && w < n) out[(int64_t)(u >> 3) * nt * 512 + (u & 7) * 8 + wo] = (HT)acc[m][nn][r];
                }
            }
}


// The unmasked store of store_tile_fast through a wave-private LDS region of
// 4 WB 256-byte runs: block row m of the wave tile (16 x 16 WB elements) is
// 4 WB runs of 8 x 8 elements (two 8-row groups times 2 WB 8-column groups),
// each contiguous in the blocked H layout.  The lanes write their elements
// into the runs in LDS, read them back 16 bytes at a time and store each run
// with 16 lanes of 16-byte stores.  Word pos = 8 (u % 8) + w % 8 of run k
// sits at pos ^ 8 (k & 1) ^ 16 (pos / 32) ^ 32 (k >= 2 WB): every 16-byte
// group stays whole and in order, and the 64 lanes of one write meet 64
// different banks (each half wave 32).  Same values at the same places as
// store_tile_fast; false (nothing stored) when it would return false.  The
// wave's LDS accesses stay in issue order, so no waits are needed between
// the writes and the reads.  The stores are non-temporal: H is read once,
// by a later kernel, and the operand rows that the other work groups re-read
// keep the L2 to themselves.
template <int WB>
__device__ __forceinline__ bool store_tile_lds(const f4 (&acc)[WB][WB], float* out, int n, int nt, int u00, int w00,
                                               int wun, int wwn, int lane, float* region) {
    const int64_t rowblk = (int64_t)nt * 512;
    const bool full = wun == WB && wwn == WB && u00 + 16 * WB <= n && w00 + 16 * WB <= n &&
                      (int64_t)nt * nt * 512 * 4 < ((int64_t)1 << 31);
    if (!full) return false;
    const int fr = lane & 15, g = lane >> 4;
    // write side: lane holds rows 4 g + r, column fr of each 16 x 16 block
    const int wr_run = (g >> 1) * (2 * WB) + (fr >> 3);                 // run of block (m, 0)
    const int wr_pos = (4 * (g & 1)) * 8 + (fr & 7);                    // pos at r = 0
    const int wr_swz = 8 * (fr >> 3) + 16 * (g & 1) + 32 * (g >> 1);   // run parity follows fr / 8
    // read side: lane takes 16-byte group j of run 4 k + lane / 16
    const int j = lane & 15, rq = lane >> 4;
    char* base = (char*)out;
#pragma unroll
    for (int m = 0; m < WB; ++m) {
#pragma unroll
        for (int nn = 0; nn < WB; ++nn)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                region[(wr_run + 2 * nn) * 64 + ((wr_pos + 8 * r) ^ wr_swz)] = acc[m][nn][r];
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < WB; ++k) {
            const int run = 4 * k + rq;
            const int slot = (4 * j) ^ (8 * (run & 1)) ^ (16 * (j >> 3)) ^ (run >= 2 * WB ? 32 : 0);
            const f4 val = *(const f4*)&region[run * 64 + slot];
            const int u0 = u00 + 16 * m + 8 * (run / (2 * WB)), w0 = w00 + 8 * (run % (2 * WB));
            const uint32_t off = (uint32_t)(((int64_t)(u0 >> 3) * rowblk + (int64_t)(w0 >> 3) * 512) * 4) + 16 * j;
            __builtin_nontemporal_store(val, (f4*)(base + off));
        }
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
    }
    return true;
}

// s_waitcnt immediate: vmcnt = vm (6 bits, split over [3:0] and [15:14]),
// expcnt and lgkmcnt not waited on.
constexpr int waitcnt_vm(int vm) { return (vm & 15) | (((vm >> 4) & 3) << 14) | (7 << 4) | (15 << 8); }
// s_waitcnt immediate: lgkmcnt = lgkm ([11:8]), vmcnt and expcnt not waited on.
constexpr int waitcnt_lgkm(int lgkm) { return 15 | (3 << 14) | (7 << 4) | ((lgkm & 15) << 8); }

// The work of logical work group L as h_gemm_body does it (loop over
// occupied triples, split-BF16x3; measured slower than h_gemm_body for FP32,
// over the register budget of two waves per SIMD for FP64, and FP8 rows
// carry scale words), with the operands going from global memory straight into LDS
// (global_load_lds_dwordx4: lane L of a wave writes the 16 bytes it loads at
// the instruction's LDS base + 16 L, so each instruction fills eight
// swizzled 128-byte rows, and the lane loads the 16-byte unit that belongs
// at its LDS position).  Two LDS stages: after the barrier of chunk c every
// wave reads its fragments of chunk c, issues the loads of chunk c + 1 into
// the other stage (which every wave finished reading before that barrier)
// and runs the MFMAs of chunk c; the barrier is preceded by a wait for the
// wave's own loads only, without a memory fence.  Without staging registers
// the compiler reads all of a chunk's fragments at once instead of block row
// by block row.  Same operands, products, order and H as h_gemm_body; a
// wave tile that lies wholly inside the plane is stored through the freed
// stage (store_tile_lds).
template <int PREC, class G>
__device__ __forceinline__ void h_gemm_dma_body(const GemmLaunch& g, int L, int nblk, int ntile_u, int ntile_w) {
    static_assert(PREC == 1 || PREC == 2, "FP32 or split-BF16x3 rows (no scale words, four-byte elements)");
    constexpr int TILE_U = G::TILE_U, NROW = G::NROW, NTHR = G::NTHR, WB = G::WB;
    constexpr int NW = NTHR / 64;       // waves
    static_assert(TILE_U % 8 == 0 && NROW % (8 * NW) == 0, "whole eight-row pieces, evenly over the waves");
    constexpr int NPW = NROW / 8 / NW;  // eight-row (1 KB) pieces per wave and chunk
    static_assert(TILE_U % (NPW * 8) == 0, "a wave's pieces stay on one side");
    static_assert(NPW < 64, "vmcnt holds the loads of one chunk");
    typedef Mode<PREC> M;
    typedef typename M::Acc Acc;
    constexpr int KC = M::KC;

    const int o = g.o, v = g.v, Kv = g.ops.Kv, Ko = g.ops.Ko;
    const int n = v;
    // uniform indices in scalar registers, as in h_gemm_body
    int rem = L;
    const int tw = __builtin_amdgcn_readfirstlane(rem % ntile_w); rem /= ntile_w;
    const int tu = __builtin_amdgcn_readfirstlane(rem % ntile_u); rem /= ntile_u;
    const int h = __builtin_amdgcn_readfirstlane(rem % 3); rem /= 3;
    const int y = __builtin_amdgcn_readfirstlane(rem % n);
    const int t = __builtin_amdgcn_readfirstlane(rem / n);
    const int4 tr = g.trip[t];
    int q, P, R;
    roles(h, __builtin_amdgcn_readfirstlane(tr.x), __builtin_amdgcn_readfirstlane(tr.y),
          __builtin_amdgcn_readfirstlane(tr.z), q, P, R);
    int ub, un, wb, wn;
    tile_range(tu, nblk, ntile_u, ub, un);
    tile_range(tw, nblk, ntile_w, wb, wn);

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wu = wave % G::WU, ww = wave / G::WU;
    int wub, wun, wwb, wwn;
    tile_range(wu, un, G::WU, wub, wun);
    tile_range(ww, wn, G::WW, wwb, wwn);
    const int arow0 = wub * 16, brow0 = TILE_U + wwb * 16;

    __shared__ __attribute__((aligned(1024))) char lds[2][NROW * ROWB];

    // The lane's source in each of the wave's pieces: LDS row `row`, 16-byte
    // position `unit` holds unit unit ^ ((row >> 1) & 7) of the row (the
    // swizzle of lds_off).  Rows past the operand's last row, or past the
    // tile's blocks, read the operand's last row: their products land only
    // in rows or columns of H that are not stored.
    const bool srow = wave * NPW * 8 < TILE_U;  // the wave's pieces hold the Row factor
    uint32_t soff[NPW];
#pragma unroll
    for (int p = 0; p < NPW; ++p) {
        const int row = (wave * NPW + p) * 8 + (lane >> 3);
        const int unit = lane & 7;
        const int r = srow ? row : row - TILE_U;
        const int gr = min((srow ? ub : wb) * 16 + r, n - 1);
        soff[p] = (uint32_t)(gr * ROWB + ((unit ^ ((row >> 1) & 7)) << 4));
    }

    // the wave's factor at chunk 0 of the loop, per segment (chunk c of
    // segment s lies c - (first chunk of s) blocks after the segment's
    // first block)
    const int nch_v = Kv / KC, nch_o = Ko / KC;
    const int nch = 2 * nch_v + 2 * nch_o;
    const int64_t blk = (int64_t)n * ROWB;
    const int seg1 = nch_v, seg2 = nch_v + nch_o, seg3 = 2 * nch_v + nch_o;
    const char* base[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const SegGeom sg = seg_geom(s, o, v, nch_v, nch_o, q, P, R, y);
        const int first = s == 0 ? 0 : s == 1 ? seg1 : s == 2 ? seg2 : seg3;
        base[s] = srow ? arr_base(g.ops, sg.arr_row) + (sg.row_mat * sg.nchunk - first) * blk
                       : arr_base(g.ops, sg.arr_col) + (sg.col_mat * sg.nchunk - first) * blk;
    }
    const int64_t d1 = base[1] - base[0], d2 = base[2] - base[1], d3 = base[3] - base[2];
    auto issue = [&](int c) {
        const int64_t d = (c >= seg1 ? d1 : 0) + (c >= seg2 ? d2 : 0) + (c >= seg3 ? d3 : 0);
        const char* src = base[0] + d + c * blk;
        char* dst = lds[c & 1] + wave * NPW * 1024;
#pragma unroll
        for (int p = 0; p < NPW; ++p)
            __builtin_amdgcn_global_load_lds((const void*)(src + soff[p]), dst + p * 1024, 16, 0, 0);
    };
    auto meet = [&]() {
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };

    Acc acc[WB][WB];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    const int fr = lane & 15, fg = lane >> 4;
    issue(0);
    for (int c = 0; c < nch; ++c) {
        meet();
        // all fragment reads first: the loads into the other stage are
        // ordered after them (both touch LDS), and the MFMAs wait on the
        // reads one by one
        StageFrags<PREC, WB> f;
        f.read(lds[c & 1], arow0, brow0, fr, fg);
        if (c + 1 < nch) issue(c + 1);
        f.mfma(acc);
    }

    // the store goes through the stage of chunk nch - 2: after every wave's
    // own loads and fragment reads are done and this barrier, no load
    // targets it and no wave still reads it
    static_assert(NW * 4 * WB * 256 <= NROW * ROWB, "a store region per wave fits in one stage");
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0) & waitcnt_lgkm(0));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    {
        const int nt = ceil_div(n, EPI_T);
        float* out = (float*)g.hbuf + (int64_t)(t * 3 + h) * hpair_elems(n) + (int64_t)(y >> 3) * nt * nt * 512 +
                     (y & 7) * 64;
        float* region = (float*)(lds[nch & 1] + wave * (4 * WB * 256));
        if (store_tile_lds<WB>(acc, out, n, nt, (ub + wub) * 16, (wb + wwb) * 16, wun, wwn, lane, region)) return;
    }
    store_plane_tile<M, WB>(acc, g.hbuf, n, t * 3 + h, y, (ub + wub) * 16, (wb + wwb) * 16, wun, wwn, lane);
}

template <int PREC, class G, int FORM>
__device__ __forceinline__ void h_gemm_body(const GemmLaunch& g, int L, int nblk, int ntile_u, int ntile_w) {
    constexpr int TILE_U = G::TILE_U, NROW = G::NROW, NTHR = G::NTHR, NVEC = G::NVEC, WB = G::WB;
    typedef Mode<PREC> M;
    typedef typename M::Acc Acc;
    constexpr int KC = M::KC;

    const int o = g.o, v = g.v, Kv = g.ops.Kv, Ko = g.ops.Ko;
    // size of the space the planes, rows and columns of H run over
    const int n = FORM == FORM_VIR ? o : v;
    // The work-group indices are uniform; the integer divisions that decode
    // them leave their results in vector registers, so they are moved back to
    // scalar registers (then every operand address of the chunk loop is
    // scalar arithmetic plus one 32-bit lane offset).
    int rem = L;
    const int tw = __builtin_amdgcn_readfirstlane(rem % ntile_w); rem /= ntile_w;
    const int tu = __builtin_amdgcn_readfirstlane(rem % ntile_u); rem /= ntile_u;
    // the three pairs of a plane are neighbours: they share the plane's
    // (ov|vv) rows of i, j and k in L2 (half the HBM fetch of pair-major order)
    const int h = __builtin_amdgcn_readfirstlane(rem % 3); rem /= 3;
    const int y = __builtin_amdgcn_readfirstlane(rem % n);
    const int t = __builtin_amdgcn_readfirstlane(rem / n);
    const int4 tr = g.trip[t];
    int q, P, R;
    roles(h, __builtin_amdgcn_readfirstlane(tr.x), __builtin_amdgcn_readfirstlane(tr.y),
          __builtin_amdgcn_readfirstlane(tr.z), q, P, R);

    int ub, un, wb, wn;  // tile block start / count along u and w
    tile_range(tu, nblk, ntile_u, ub, un);
    tile_range(tw, nblk, ntile_w, wb, wn);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wu = wave % G::WU, ww = wave / G::WU;
    int wub, wun, wwb, wwn;  // this wave's blocks within the tile
    tile_range(wu, un, G::WU, wub, wun);
    tile_range(ww, wn, G::WW, wwb, wwn);
    const int arow0 = wub * 16;           // first LDS Row-factor row of this wave
    const int brow0 = TILE_U + wwb * 16;  // first LDS Col-factor row of this wave

    __shared__ __attribute__((aligned(16))) char lds[2][NROW * ROWB];
    // FP8 only: the E8M0 exponent word (4 x 32 elements) of every staged row
    __shared__ uint32_t lds_s[2][PREC == 3 ? NROW : 1];

    Acc acc[WB][WB];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    // This thread's 16-byte vector qv of each staged row, and its rows: vector
    // e covers LDS row (tid / 8) + e NTHR / 8; rows [0, TILE_U) hold the Row
    // factor (u), rows [TILE_U, NROW) the Col factor (w).  Byte offsets
    // within a chunk block are fixed for the work group, and vector e of
    // every thread lies on the same side (TILE_U is a multiple of NTHR / 8).
    // Rows past the operand's last row, or past the tile's blocks,
    // read the operand's last row: their products land only in rows or
    // columns of H that are not stored, so every load is unconditional.
    static_assert(TILE_U % (NTHR / 8) == 0, "each staging vector stays on one side");
    const int qv = tid & 7;
    uint32_t off[NVEC];
    constexpr auto isrow = [](int e) { return e * (NTHR / 8) < TILE_U; };
#pragma unroll
    for (int e = 0; e < NVEC; ++e) {
        const int row = (tid >> 3) + e * (NTHR / 8);
        const int r = isrow(e) ? row : row - TILE_U;
        const int gr = min((isrow(e) ? ub : wb) * 16 + r, n - 1);
        off[e] = (uint32_t)(gr * ROWB + qv * 16);
    }

    const int nch_v = Kv / KC, nch_o = Ko / KC;
    const int nch = 2 * nch_v + 2 * nch_o;
    const int64_t blk = (int64_t)n * ROWB;  // bytes of one chunk block (all n rows)

    // FP8 scale words: thread tid stages rows tid and tid + 256 (< NROW)
    constexpr int NSROW = (NROW + NTHR - 1) / NTHR;
    int srow_g[NSROW];
    bool srow_ok[NSROW];
    if constexpr (PREC == 3) {
#pragma unroll
        for (int e = 0; e < NSROW; ++e) {
            const int row = tid + e * NTHR;
            const bool isr = row < TILE_U;
            const int r = isr ? row : row - TILE_U;
            const int gr = (isr ? ub : wb) * 16 + r;
            srow_ok[e] = row < NROW && r < (isr ? un : wn) * 16 && gr < n;
            srow_g[e] = gr;
        }
    }

    // Chunk c of segment s lies (c - first chunk of s) blocks after the
    // segment's first block: per segment, the Row and Col addresses of chunk
    // 0 (of the whole loop) are formed once, so that a chunk's address is one
    // selection by segment and one multiply-add.
    const int seg1 = nch_v, seg2 = nch_v + nch_o, seg3 = 2 * nch_v + nch_o;
    const char* rseg[4];
    const char* cseg[4];
    const uint32_t* rsseg[4];
    const uint32_t* csseg[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const SegGeom sg = FORM == FORM_VIR ? seg_geom_vir(s, v, nch_v, nch_o, q, P, R, y)
                                            : seg_geom(s, o, v, nch_v, nch_o, q, P, R, y);
        const int first = s == 0 ? 0 : s == 1 ? seg1 : s == 2 ? seg2 : seg3;
        rseg[s] = arr_base(g.ops, sg.arr_row) + (sg.row_mat * sg.nchunk - first) * blk;
        cseg[s] = arr_base(g.ops, sg.arr_col) + (sg.col_mat * sg.nchunk - first) * blk;
        if constexpr (PREC == 3) {
            rsseg[s] = scale_base(g.ops, sg.arr_row) + (sg.row_mat * sg.nchunk - first) * (int64_t)n;
            csseg[s] = scale_base(g.ops, sg.arr_col) + (sg.col_mat * sg.nchunk - first) * (int64_t)n;
        }
    }
    // base of chunk c's segment as segment 0's base plus the steps between
    // segment bases that c has passed (branch-free scalar selects)
    auto pick = [&](int c, auto const (&a)[4]) {
        const int64_t d1 = (const char*)a[1] - (const char*)a[0], d2 = (const char*)a[2] - (const char*)a[1],
                      d3 = (const char*)a[3] - (const char*)a[2];
        const int64_t d = (c >= seg1 ? d1 : 0) + (c >= seg2 ? d2 : 0) + (c >= seg3 ? d3 : 0);
        return (std::remove_const_t<std::remove_reference_t<decltype(a[0])>>)((const char*)a[0] + d);
    };

    u4 reg[NVEC];
    uint32_t sreg[NSROW];
    auto load = [&](int c) {
        const char* rb = pick(c, rseg) + c * blk;
        const char* cb = pick(c, cseg) + c * blk;
#pragma unroll
        for (int e = 0; e < NVEC; ++e) reg[e] = *(const u4*)((isrow(e) ? rb : cb) + off[e]);
        if constexpr (PREC == 3) {
            const uint32_t* rs = pick(c, rsseg) + c * (int64_t)n;
            const uint32_t* cs = pick(c, csseg) + c * (int64_t)n;
#pragma unroll
            for (int e = 0; e < NSROW; ++e) {
                const int row = tid + e * NTHR;
                sreg[e] = srow_ok[e] ? (row < TILE_U ? rs : cs)[srow_g[e]] : 0u;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < NVEC; ++e) {
            const int row = (tid >> 3) + e * (NTHR / 8);
            if ((NVEC * NTHR == NROW * 8) || row < NROW) *(u4*)(&lds[buf][lds_off(row, qv)]) = reg[e];
        }
        if constexpr (PREC == 3) {
#pragma unroll
            for (int e = 0; e < NSROW; ++e) {
                const int row = tid + e * NTHR;
                if (row < NROW) lds_s[buf][row] = sreg[e];
            }
        }
    };

    const int fr = lane & 15, fg = lane >> 4;
    auto compute = [&](int buf) {
        stage_products<PREC, WB>(acc, lds[buf], lds_s[buf], arow0, brow0, fr, fg);
    };

    load(0);
    store(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        if (c + 1 < nch) load(c + 1);
        compute(c & 1);
        if (c + 1 < nch) store((c + 1) & 1);
        __syncthreads();
    }

    store_plane_tile<M, WB>(acc, g.hbuf, n, t * 3 + h, y, (ub + wub) * 16, (wb + wwb) * 16, wun, wwn, lane);
}

template <int PREC, class G, int FORM>
__global__ __launch_bounds__(G::NTHR, 1) void h_gemm_kernel(GemmLaunch g, int n_wg, int nblk, int ntile_u,
                                                              int ntile_w, int per_xcd) {
    // XCD-aware order: hardware block hw runs on XCD hw % 8; each XCD gets a
    // contiguous range of logical tiles (neighbours share operands in L2).
    const int hw = blockIdx.x;
    const int L = (hw % 8) * per_xcd + hw / 8;
    if (L >= n_wg) return;
    if constexpr (FORM == FORM_OCC && PREC == 2)
        h_gemm_dma_body<PREC, G>(g, L, nblk, ntile_u, ntile_w);
    else
        h_gemm_body<PREC, G, FORM>(g, L, nblk, ntile_u, ntile_w);
}

// One contraction launch over several solves (fragments) at once: entry e
// holds a launch of one fragment, its tiling and the first logical work
// group of the launch (entries in increasing order of wg0); logical work
// group L runs work group L - wg0 of the entry with the largest wg0 <= L.
template <int PREC, class G>
__global__ __launch_bounds__(G::NTHR, 1) void h_gemm_group_kernel(const GemmGroupEntry* __restrict__ ent, int nent,
                                                                    int n_wg, int per_xcd) {
    const int hw = blockIdx.x;
    const int L = (hw % 8) * per_xcd + hw / 8;
    if (L >= n_wg) return;
    int lo = 0, hi = nent - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ent[mid].wg0 <= L) lo = mid;
        else hi = mid - 1;
    }
    const GemmGroupEntry e = ent[lo];
    if constexpr (PREC == 2)
        h_gemm_dma_body<PREC, G>(e.g, L - e.wg0, e.nblk, e.ntile_u, e.ntile_w);
    else
        h_gemm_body<PREC, G, FORM_OCC>(e.g, L - e.wg0, e.nblk, e.ntile_u, e.ntile_w);
}

// The loop over virtual triples has small planes (n = nocc rows and
// columns), and in every segment one of the two factors does not depend on
// the plane y: the Row factor in segments 0 and 3 ((uA|Bd), t_lu^BA) and the
// Col factor in segments 1 and 2 (t_lw^BC, (wC|Bd)).  A work group of PL_NP
// waves therefore takes PL_NP consecutive planes of one pair of one triple,
// one plane per wave (all n x n of it, WB x WB 16-blocks), and stages the
// plane-independent factor once per chunk for all of them: LDS rows
// [0, 16 WB) hold it, rows [16 WB (1 + p), 16 WB (2 + p)) the factor of
// plane y0 + p.  Same chunk-major operands, staging, swizzle and MFMA
// products as h_gemm_kernel.
constexpr int PL_NP = 4;

template <int PREC, int WB>
__global__ __launch_bounds__(64 * PL_NP, 1) void h_gemm_planes_kernel(GemmLaunch g, int n_wg, int ngrp,
                                                                      int per_xcd) {
    constexpr int NTHR = 64 * PL_NP, NPAD = 16 * WB, NROW = (1 + PL_NP) * NPAD;
    constexpr int NVEC = (NROW * 8 + NTHR - 1) / NTHR;
    typedef Mode<PREC> M;
    typedef typename M::Acc Acc;
    typedef typename M::HT HT;
    constexpr int KC = M::KC;

    const int hw = blockIdx.x;
    const int L = (hw % 8) * per_xcd + hw / 8;  // XCD-aware order, as in h_gemm_kernel
    if (L >= n_wg) return;
    const int o = g.o, v = g.v, Kv = g.ops.Kv, Ko = g.ops.Ko;
    const int n = o;  // planes, rows and columns run over the occupied indices
    int rem = L;
    const int grp = rem % ngrp; rem /= ngrp;
    const int h = rem % 3;
    const int t = rem / 3;
    const int4 tr = g.trip[t];
    int B, A, C;  // middle virtual of the pair and the other two
    roles(h, tr.x, tr.y, tr.z, B, A, C);
    const int y0 = grp * PL_NP;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ __attribute__((aligned(16))) char lds[2][NROW * ROWB];

    Acc acc[WB][WB];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    // staged row of this thread's vector e: (tid / 8) + e NTHR / 8; block 0
    // is the plane-independent factor, block 1 + p the factor of plane y0 + p
    const int qv = tid & 7;
    int off[NVEC], plane[NVEC];
    bool ok[NVEC];
#pragma unroll
    for (int e = 0; e < NVEC; ++e) {
        const int row = (tid >> 3) + e * (NTHR / 8);
        const int blkrow = row / NPAD, r = row % NPAD;
        plane[e] = blkrow - 1;  // -1: plane-independent factor
        ok[e] = row < NROW && r < n && (blkrow == 0 || y0 + blkrow - 1 < n);
        off[e] = r * ROWB + qv * 16;
    }

    const int nch_v = Kv / KC, nch_o = Ko / KC;
    const int nch = 2 * nch_v + 2 * nch_o;
    auto chunk_seg = [&](int c, int& s, int& kb) {
        if (c < nch_v) { s = 0; kb = c; }
        else if (c < nch_v + nch_o) { s = 1; kb = c - nch_v; }
        else if (c < 2 * nch_v + nch_o) { s = 2; kb = c - nch_v - nch_o; }
        else { s = 3; kb = c - 2 * nch_v - nch_o; }
    };
    const int64_t blk = (int64_t)n * ROWB;  // bytes of one chunk block (all n rows)

    u4 reg[NVEC];
    auto load = [&](int c) {
        int s, kb;
        chunk_seg(c, s, kb);
        // plane-independent matrix and the plane-y matrix y * v + X of this segment
        // (the matrices of seg_geom_vir)
        int arr_s, arr_y, X;
        int64_t mat_s;
        switch (s) {
            case 0: arr_s = 0; mat_s = (int64_t)A * v + B; arr_y = 1; X = C; break;  // (uA|Bd) | t_wy^Cd
            case 1: arr_s = 2; mat_s = (int64_t)B * v + C; arr_y = 3; X = A; break;  // t_lw^BC | -(uA|yl)
            case 2: arr_s = 0; mat_s = (int64_t)C * v + B; arr_y = 1; X = A; break;  // (wC|Bd) | t_uy^Ad
            default: arr_s = 2; mat_s = (int64_t)B * v + A; arr_y = 3; X = C; break;  // t_lu^BA | -(wC|yl)
        }
        const int nchunk = (s == 0 || s == 2) ? nch_v : nch_o;
        const char* sb = arr_base(g.ops, arr_s) + (mat_s * nchunk + kb) * blk;
        const char* yb = arr_base(g.ops, arr_y) + ((int64_t)X * nchunk + kb) * blk;
        const int64_t ystep = (int64_t)v * nchunk * blk;  // next plane: matrix + v
#pragma unroll
        for (int e = 0; e < NVEC; ++e) {
            const char* base = plane[e] < 0 ? sb : yb + (int64_t)(y0 + plane[e]) * ystep;
            reg[e] = ok[e] ? *(const u4*)(base + off[e]) : u4{0, 0, 0, 0};
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < NVEC; ++e) {
            const int row = (tid >> 3) + e * (NTHR / 8);
            if ((NVEC * NTHR == NROW * 8) || row < NROW) *(u4*)(&lds[buf][lds_off(row, qv)]) = reg[e];
        }
    };

    const int fr = lane & 15, fg = lane >> 4;
    const int own = NPAD * (1 + wave);  // first LDS row of this wave's plane factor
    auto compute = [&](int buf, int c) {
        int s, kb;
        chunk_seg(c, s, kb);
        const bool shared_row = (s == 0 || s == 3);  // the Row factor is the shared one
        stage_products<PREC, WB>(acc, lds[buf], nullptr, shared_row ? 0 : own, shared_row ? own : 0, fr, fg);
    };

    load(0);
    store(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        if (c + 1 < nch) load(c + 1);
        compute(c & 1, c);
        if (c + 1 < nch) store((c + 1) & 1);
        __syncthreads();
    }

    const int y = y0 + wave;
    if (y >= n) return;
    const int nt = ceil_div(n, EPI_T);
    HT* out = (HT*)g.hbuf + (int64_t)(t * 3 + h) * hpair_elems(n) + (int64_t)(y >> 3) * nt * nt * 512 +
              (y & 7) * 64;
    if (store_tile_fast<M, WB>(acc, out, n, nt, 0, 0, WB, WB, lane)) return;
#pragma unroll
    for (int m = 0; m < WB; ++m)
#pragma unroll
        for (int nn = 0; nn < WB; ++nn) {
            const int w = nn * 16 + fr;
            const int wo = (w >> 3) * 512 + (w & 7);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = m * 16 + M::row(lane, r);
                if (u < n && w < n) out[(int64_t)(u >> 3) * nt * 512 + (u & 7) * 8 + wo] = (HT)acc[m][nn][r];
            }
        }
}

// The work of h_gemm_planes_kernel for split-BF16x3 with the operands going from global
// memory straight into two LDS stages, as h_gemm_dma_body does (the stage's
// 8-row pieces are spread over the waves; a piece holds rows of the
// plane-independent factor or of one plane's factor).  Rows past the
// occupied space read its last row and planes past it read its last plane:
// their products land only in rows, columns or planes of H that are not
// stored.  Same operands, products, order and H as h_gemm_planes_kernel.
template <int WB>
__device__ __forceinline__ void h_gemm_planes_dma_body(const GemmLaunch& g, int L, int ngrp) {
    constexpr int PREC = 2;
    constexpr int NPAD = 16 * WB, NROW = (1 + PL_NP) * NPAD;
    constexpr int NPIECE = NROW / 8;                       // eight-row (1 KB) pieces per stage
    constexpr int NPW = (NPIECE + PL_NP - 1) / PL_NP;      // pieces per wave (the last may be absent)
    static_assert(NPAD % 8 == 0, "a piece lies in one factor block");
    typedef Mode<PREC> M;
    constexpr int KC = M::KC;

    const int o = g.o, v = g.v, Kv = g.ops.Kv, Ko = g.ops.Ko;
    const int n = o;
    int rem = L;
    const int grp = __builtin_amdgcn_readfirstlane(rem % ngrp); rem /= ngrp;
    const int h = __builtin_amdgcn_readfirstlane(rem % 3);
    const int t = __builtin_amdgcn_readfirstlane(rem / 3);
    const int4 tr = g.trip[t];
    int B, A, C;  // middle virtual of the pair and the other two
    roles(h, __builtin_amdgcn_readfirstlane(tr.x), __builtin_amdgcn_readfirstlane(tr.y),
          __builtin_amdgcn_readfirstlane(tr.z), B, A, C);
    const int y0 = grp * PL_NP;

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    __shared__ __attribute__((aligned(1024))) char lds[2][NROW * ROWB];

    f4 acc[WB][WB];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) acc[a][b] = f4{0, 0, 0, 0};

    // piece k of this wave: piece wave + k PL_NP of the stage (uniform per wave)
    uint32_t soff[NPW];
    int pplane[NPW];  // -1: plane-independent factor, else the (clamped) plane
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
        const int pc = wave + k * PL_NP;
        const int row = 8 * pc + (lane >> 3);  // LDS row
        const int blkrow = (8 * pc) / NPAD;
        const int r = min(row % NPAD, n - 1);
        pplane[k] = blkrow == 0 ? -1 : min(y0 + blkrow - 1, n - 1);
        soff[k] = (uint32_t)(r * ROWB + (((lane & 7) ^ ((row >> 1) & 7)) << 4));
    }

    const int nch_v = Kv / KC, nch_o = Ko / KC;
    const int nch = 2 * nch_v + 2 * nch_o;
    const int64_t blk = (int64_t)n * ROWB;  // bytes of one chunk block (all n rows)
    auto seg_of = [&](int c) { return (c >= nch_v) + (c >= nch_v + nch_o) + (c >= 2 * nch_v + nch_o); };
    auto issue = [&](int c) {
        const int s = seg_of(c);
        const int kb = c - (s == 0 ? 0 : s == 1 ? nch_v : s == 2 ? nch_v + nch_o : 2 * nch_v + nch_o);
        // plane-independent matrix and the plane-y matrix y * v + X of this
        // segment (the matrices of seg_geom_vir)
        int arr_s, arr_y, X;
        int64_t mat_s;
        switch (s) {
            case 0: arr_s = 0; mat_s = (int64_t)A * v + B; arr_y = 1; X = C; break;  // (uA|Bd) | t_wy^Cd
            case 1: arr_s = 2; mat_s = (int64_t)B * v + C; arr_y = 3; X = A; break;  // t_lw^BC | -(uA|yl)
            case 2: arr_s = 0; mat_s = (int64_t)C * v + B; arr_y = 1; X = A; break;  // (wC|Bd) | t_uy^Ad
            default: arr_s = 2; mat_s = (int64_t)B * v + A; arr_y = 3; X = C; break;  // t_lu^BA | -(wC|yl)
        }
        const int nchunk = (s == 0 || s == 2) ? nch_v : nch_o;
        const char* sb = arr_base(g.ops, arr_s) + (mat_s * nchunk + kb) * blk;
        const char* yb = arr_base(g.ops, arr_y) + ((int64_t)X * nchunk + kb) * blk;
        const int64_t ystep = (int64_t)v * nchunk * blk;  // next plane: matrix + v
#pragma unroll
        for (int k = 0; k < NPW; ++k) {
            const int pc = wave + k * PL_NP;
            if (pc < NPIECE) {
                const char* src = (pplane[k] < 0 ? sb : yb + pplane[k] * ystep) + soff[k];
                __builtin_amdgcn_global_load_lds((const void*)src, lds[c & 1] + pc * 1024, 16, 0, 0);
            }
        }
    };
    auto meet = [&]() {
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };

    const int fr = lane & 15, fg = lane >> 4;
    const int own = NPAD * (1 + wave);  // first LDS row of this wave's plane factor
    issue(0);
    for (int c = 0; c < nch; ++c) {
        meet();
        const int s = seg_of(c);
        const bool shared_row = (s == 0 || s == 3);  // the Row factor is the shared one
        StageFrags<PREC, WB> f;
        f.read(lds[c & 1], shared_row ? 0 : own, shared_row ? own : 0, fr, fg);
        if (c + 1 < nch) issue(c + 1);
        f.mfma(acc);
    }

    const int y = y0 + wave;
    if (y >= n) return;
    store_plane_tile<M, WB>(acc, g.hbuf, n, t * 3 + h, y, 0, 0, WB, WB, lane);
}

template <int WB>
__global__ __launch_bounds__(64 * PL_NP, 1) void h_gemm_planes_dma_kernel(GemmLaunch g, int n_wg, int ngrp,
                                                                          int per_xcd) {
    const int hw = blockIdx.x;
    const int L = (hw % 8) * per_xcd + hw / 8;  // XCD-aware order, as in h_gemm_kernel
    if (L >= n_wg) return;
    h_gemm_planes_dma_body<WB>(g, L, ngrp);
}

}  // namespace

namespace {

template <int PREC, class G, int FORM>
KernelCall geo_call(const GemmLaunch& g) {
    const int n = FORM == FORM_VIR ? g.o : g.v;
    const int nblk = ceil_div(n, 16);
    const int ntile_u = ceil_div(nblk, G::WU * G::WB), ntile_w = ceil_div(nblk, G::WW * G::WB);
    const int64_t n64 = (int64_t)g.ntrip * 3 * n * ntile_u * ntile_w;
    if (n64 > ((int64_t)1 << 31) - 8) throw Error(-1, "contraction grid too large");
    const int n_wg = (int)n64;
    const int per_xcd = ceil_div(n_wg, 8);
    KernelCall k;
    k.fn = (const void*)&h_gemm_kernel<PREC, G, FORM>;
    k.grid = dim3(per_xcd * 8);
    k.block = dim3(G::NTHR);
    k.arg(g).arg(n_wg).arg(nblk).arg(ntile_u).arg(ntile_w).arg(per_xcd);
    return k;
}

// Share of the computed 16x16 block products that are useful when the nblk
// blocks of v are split over tiles of 2 x 2 waves of at most wb x wb blocks.
double block_use(int nblk, int wb) {
    const int ntile = ceil_div(nblk, 2 * wb);
    const double slots = (double)ntile * ntile * 4 * wb * wb;
    return (double)nblk * nblk / slots;
}

template <int PREC, int WB>
KernelCall planes_call(const GemmLaunch& g) {
    const int ngrp = ceil_div(g.o, PL_NP);
    const int64_t n64 = (int64_t)g.ntrip * 3 * ngrp;
    if (n64 > ((int64_t)1 << 31) - 8) throw Error(-1, "contraction grid too large");
    const int n_wg = (int)n64;
    const int per_xcd = ceil_div(n_wg, 8);
    KernelCall k;
    if constexpr (PREC == 2)
        k.fn = (const void*)&h_gemm_planes_dma_kernel<WB>;
    else
        k.fn = (const void*)&h_gemm_planes_kernel<PREC, WB>;
    k.grid = dim3(per_xcd * 8);
    k.block = dim3(64 * PL_NP);
    k.arg(g).arg(n_wg).arg(ngrp).arg(per_xcd);
    return k;
}

template <int PREC>
KernelCall mode_call(const GemmLaunch& g, int form) {
    if (form == FORM_VIR) {
        // occupied spaces are small: tiles down to one 16 x 16 block per wave
        if constexpr (PREC == 3) {
            throw Error(-1, "the virtual-triple loop has no FP8 contraction");
        } else {
            // up to 64 occupied orbitals: one plane per wave (h_gemm_planes_kernel)
            switch (ceil_div(g.o, 16)) {
                case 1: return planes_call<PREC, 1>(g);
                case 2: return planes_call<PREC, 2>(g);
                case 3: return planes_call<PREC, 3>(g);
                case 4: return planes_call<PREC, 4>(g);
                default: break;
            }
            switch (wave_blocks(g.o, 1)) {
                case 1: return geo_call<PREC, Geo<2, 2, 1>, FORM_VIR>(g);
                case 2: return geo_call<PREC, Geo<2, 2, 2>, FORM_VIR>(g);
                case 3: return geo_call<PREC, Geo<2, 2, 3>, FORM_VIR>(g);
                case 4: return geo_call<PREC, Geo<2, 2, 4>, FORM_VIR>(g);
                default: return geo_call<PREC, Geo<2, 2, 5>, FORM_VIR>(g);
            }
        }
    }
    switch (wave_blocks(g.v)) {
        case 2: return geo_call<PREC, Geo<2, 2, 2>, FORM_OCC>(g);
        case 3: return geo_call<PREC, Geo<2, 2, 3>, FORM_OCC>(g);
        case 4: return geo_call<PREC, Geo<2, 2, 4>, FORM_OCC>(g);
        default: return geo_call<PREC, Geo<2, 2, 5>, FORM_OCC>(g);
    }
}

}  // namespace

// Wave tile size (blocks per side) for rows and columns of size n: a smaller
// tile wastes fewer block products on partial tiles but loads more operand
// bytes per flop, so it is taken only when its useful share is at least 20%
// higher.
int wave_blocks(int n, int min_wb) {
    const int nblk = ceil_div(n, 16);
    int best = 5;
    double use = block_use(nblk, 5);
    for (int wb = 4; wb >= min_wb; --wb) {
        const double u = block_use(nblk, wb);
        if (u > 1.2 * use) { use = u; best = wb; }
    }
    return best;
}

namespace {
template <int PREC, int WB>
KernelCall group_call_wb(const GemmGroupEntry* d_ent, int nent, int64_t n_wg) {
    if (n_wg > ((int64_t)1 << 31) - 8) throw Error(-1, "grouped contraction grid too large");
    const int per_xcd = ceil_div((int)n_wg, 8);
    KernelCall k;
    k.fn = (const void*)&h_gemm_group_kernel<PREC, Geo<2, 2, WB>>;
    k.grid = dim3(per_xcd * 8);
    k.block = dim3(Geo<2, 2, WB>::NTHR);
    k.arg(d_ent).arg(nent).arg((int)n_wg).arg(per_xcd);
    return k;
}
template <int PREC>
KernelCall group_call_prec(int wb, const GemmGroupEntry* d_ent, int nent, int64_t n_wg) {
    switch (wb) {
        case 2: return group_call_wb<PREC, 2>(d_ent, nent, n_wg);
        case 3: return group_call_wb<PREC, 3>(d_ent, nent, n_wg);
        case 4: return group_call_wb<PREC, 4>(d_ent, nent, n_wg);
        case 5: return group_call_wb<PREC, 5>(d_ent, nent, n_wg);
        default: throw Error(-1, "unsupported wave tile");
    }
}
}  // namespace

KernelCall gemm_group_call(int precision, int wb, const GemmGroupEntry* d_ent, int nent, int64_t n_wg) {
    switch (precision) {
        case 0: return group_call_prec<0>(wb, d_ent, nent, n_wg);
        case 1: return group_call_prec<1>(wb, d_ent, nent, n_wg);
        case 2: return group_call_prec<2>(wb, d_ent, nent, n_wg);
        case 3: return group_call_prec<3>(wb, d_ent, nent, n_wg);
        default: throw Error(-1, "unsupported precision for the MFMA contraction");
    }
}

// Work groups of 2 x 2 waves; the wave tile is chosen per v (wave_blocks).
// A 320 x 160 tile with 8 waves loads a quarter fewer operand bytes per flop
// than 160 x 160 but measured slower (FP32 7.9 s vs 7.6 s, BF16x3 3.7 s vs
// 3.4 s per solve at o = 32, v = 300).
KernelCall gemm_call(int precision, const GemmLaunch& g, int form) {
    switch (precision) {
        case 0: return mode_call<0>(g, form);
        case 1: return mode_call<1>(g, form);
        case 2: return mode_call<2>(g, form);
        case 3: return mode_call<3>(g, form);
        default: throw Error(-1, "unsupported precision for the MFMA contraction");
    }
}

}  // namespace bqc
