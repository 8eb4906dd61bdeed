// Fused FP64 epilogue of the (T) energy and the deterministic reductions
// (paper section 2.4.2, Eqs. 3-4 and 6-7; the denominator is formed in
// registers from the orbital energies, as the paper's in-place denominator
// kernel does, and no rank-6 or rank-3 denominator tensor exists).
//
// For one occupied triple (i, j, k) of weight m and a tile orbit
// {A, B, C} (A >= B >= C, tiles of EPI_T virtuals), the work group builds in
// LDS, for the six tile permutations s(A, B, C),
//   W = H_a[a][b][c] + H_b[b][a][c] + H_c[c][a][b]            (six-fold P)
// together with the 8 x 8 blocks of (jb|kc), (ia|kc), (ia|jb) and the t1
// slices the orbit needs, and every thread takes one element (a, b, c) of the
// base tile with its six permutations p, forming
//   V = W + t_i^a (jb|kc) + t_j^b (ia|kc) + t_k^c (ia|jb)       (singles term)
// on the fly.  With D = e_i + e_j + e_k - e_a - e_b - e_c (the same
// for all six) the numerator operator 4 + cyclic - 2 transpositions acting on
// V gives, for even p:  3 V_p + S_e - 2 S_o  and for odd p:  3 V_p + S_o - 2 S_e
// (S_e, S_o = sums of V over even and odd permutations), so
//   sum_p W_p Z_p = [3 sum_p W_p V_p + (S_e - 2 S_o) W_e + (S_o - 2 S_e) W_o] / D.
// Summing this over the base tile counts every element of the orbit's tiles
// |stabiliser(A, B, C)| times, which the work group divides out.  Padding
// elements (index >= v) have W = 0 and contribute nothing.
//
// No floating-point atomics: each work group writes one FP64 partial; the
// partials are summed per triple and then over triples in a fixed order with
// Neumaier compensation.
//
// The loop over virtual triples runs this same kernel with the two orbital
// spaces exchanged (triples (a, b, c), tiles of occupied orbitals; the
// arguments are described with EpiLaunch).
#include "bqc_internal.h"

namespace bqc {
namespace {

constexpr int E_T3 = EPI_T * EPI_T * EPI_T;
constexpr int E_THREADS = 256;
static_assert(E_T3 % E_THREADS == 0, "tile elements divide over threads");

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// x if keep, else +0.  The mask is made opaque to the compiler so that the
// load producing x stays unconditional (a plain select would be turned into a
// branch around the load, which serialises the loads of a work group).
__device__ __forceinline__ double keep_if(double x, bool keep) {
    long long m = keep ? -1ll : 0ll;
    asm volatile("" : "+v"(m));
    return __longlong_as_double(__double_as_longlong(x) & m);
}

// FOCK: the reference is non-canonical (f_ov != 0) and V also holds
// f_ia t_jk^bc + f_jb t_ik^ac + f_kc t_ij^ab (paper Eqs. 5 and 7), staged
// exactly like the singles term (t2 blocks in place of (ov|ov) blocks, f_ov
// slices in place of t1 slices).
// Tile orbit `orb` of triple `t` of the launch e.
template <typename HT, bool FOCK>
__device__ __forceinline__ void epilogue_body(const EpiLaunch& e, int orb, int t) {
    const int4 ob = e.orbits[orb];
    const int4 tr = e.trip[t];
    const int i = tr.x, j = tr.y, k = tr.z;
    const int v = e.v;
    const int nt = ceil_div(v, EPI_T);
    const int64_t hp = hpair_elems(v);
    const HT* Ha = (const HT*)e.hbuf + (int64_t)(t * 3 + 0) * hp;
    const HT* Hb = Ha + hp;
    const HT* Hc = Hb + hp;
    // first element of block (X, Y, Z) of a blocked H buffer
    auto blk = [&](const HT* H, int X, int Y, int Z) { return H + (((int64_t)X * nt + Y) * nt + Z) * E_T3; };

    constexpr int T = EPI_T, T2 = EPI_T * EPI_T;
    // LDS layouts, XOR-swizzled so that the permuted reads of phase 3 meet
    // at most two addresses per bank (eight without): W element (x, y, z) of
    // a tile permutation at x T2 + (y ^ x) T + (z ^ y), and element (x, y) of
    // an 8 x 8 block of the singles (and f_ov) factors at x T + (y ^ x)
    auto widx = [](int x, int y, int z) { return x * T2 + ((y ^ x) * T) + (z ^ y); };
    auto gidx = [](int x, int y) { return x * T + (y ^ x); };
    __shared__ double Ws[6][E_T3];
    // singles-term factors of the orbit's tiles: G[m][X][Y][x][y] with
    // m = 0: (jb|kc), 1: (ia|kc), 2: (ia|jb), X, Y tile ids in {A, B, C};
    // t1s[n][X][x] = t_{i,j,k}^{tile X, x}
    __shared__ double Gs[3][3][3][T2];
    __shared__ double t1s[3][3][T];
    // f_ov term: Ts[m][X][Y][x][y] with m = 0: t_jk^{bc}, 1: t_ik^{ac}, 2: t_ij^{ab}
    // (first virtual in tile X, second in Y); fs[n][X][x] = f_{i,j,k}^{tile X, x}
    __shared__ double Ts[FOCK ? 3 : 1][3][3][FOCK ? T2 : 1];
    __shared__ double fs[FOCK ? 3 : 1][3][FOCK ? T : 1];
    __shared__ double red[E_THREADS / 64];

    const int TT[3] = {ob.x, ob.y, ob.z};  // tile ids 0, 1, 2 -> tiles A, B, C
    // tile permutations as tile ids: 0 (A,B,C) 1 (A,C,B) 2 (B,A,C) 3 (B,C,A) 4 (C,A,B) 5 (C,B,A)
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

    // Phases 0 and 1 issue every global load of the work group before the
    // first LDS store, so that the group waits for one memory latency, not
    // one per loop trip.
    // phase 0 loads: singles-term factors (27 8x8 blocks of (ov|ov)) and t1
    constexpr int NG = (27 * T2 + E_THREADS - 1) / E_THREADS;
    double gv[NG];
#pragma unroll
    for (int n = 0; n < NG; ++n) {
        const int el = threadIdx.x + n * E_THREADS;
        const int m = el / (9 * T2), rem = el % (9 * T2);
        const int X = rem / (3 * T2), Y = (rem / T2) % 3, xy = rem % T2;
        const int tx = X == 0 ? TT[0] : X == 1 ? TT[1] : TT[2];
        const int ty = Y == 0 ? TT[0] : Y == 1 ? TT[1] : TT[2];
        const int x = tx * T + xy / T, y = ty * T + xy % T;
        // m = 0: (jb|kc) with b in X, c in Y; 1: (ia|kc); 2: (ia|jb)
        const int p = m == 0 ? j : i, q = m == 2 ? j : k;
        // unconditional load at a clamped (valid) index, then masked: no branch
        const double g = e.ovov[p * e.ovov_sp + min(x, v - 1) * e.ovov_sx + q * e.ovov_sq + min(y, v - 1)];
        gv[n] = keep_if(g, el < 27 * T2 && x < v && y < v);
    }
    // f_ov term loads (same shapes as the singles term)
    double tv[FOCK ? NG : 1];
    double fv = 0.0;
    if constexpr (FOCK) {
        const int64_t vv = (int64_t)v * v;
#pragma unroll
        for (int n = 0; n < NG; ++n) {
            const int el = threadIdx.x + n * E_THREADS;
            const int m = el / (9 * T2), rem = el % (9 * T2);
            const int X = rem / (3 * T2), Y = (rem / T2) % 3, xy = rem % T2;
            const int tx = X == 0 ? TT[0] : X == 1 ? TT[1] : TT[2];
            const int ty = Y == 0 ? TT[0] : Y == 1 ? TT[1] : TT[2];
            const int x = tx * T + xy / T, y = ty * T + xy % T;
            // m = 0: t_jk^{bc}; 1: t_ik^{ac}; 2: t_ij^{ab}
            const int p = m == 0 ? j : i, q = m == 2 ? j : k;
            const double g = e.t2[((int64_t)p * e.o + q) * vv + (int64_t)min(x, v - 1) * v + min(y, v - 1)];
            tv[n] = keep_if(g, el < 27 * T2 && x < v && y < v);
        }
        if (threadIdx.x < 9 * T) {
            const int n = threadIdx.x / (3 * T), X = (threadIdx.x / T) % 3;
            const int tx = X == 0 ? TT[0] : X == 1 ? TT[1] : TT[2];
            const int x = tx * T + threadIdx.x % T;
            const int on = n == 0 ? i : n == 1 ? j : k;
            if (x < v) fv = e.fock_ov[(int64_t)on * v + x];
        }
    }
    double t1v = 0.0;
    if (threadIdx.x < 9 * T) {
        const int n = threadIdx.x / (3 * T), X = (threadIdx.x / T) % 3;
        const int tx = X == 0 ? TT[0] : X == 1 ? TT[1] : TT[2];
        const int x = tx * T + threadIdx.x % T;
        const int on = n == 0 ? i : n == 1 ? j : k;
        if (x < v) t1v = e.t1[(int64_t)on * v + x];
    }
    // phase 1 loads: the H_a, H_b and H_c blocks of the six tile permutations.
    // Each block is one contiguous run of 512 elements; a wave covers 64
    // consecutive elements of a block (one run, or eight 32-byte pieces).
    constexpr int NE = E_T3 / E_THREADS;
    double wv[6][NE];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int X = TT[perm[s][0]], Y = TT[perm[s][1]], Z = TT[perm[s][2]];
        const HT* ba = blk(Ha, X, Y, Z);
        const HT* bb = blk(Hb, Y, X, Z);
        const HT* bc = blk(Hc, Z, X, Y);
#pragma unroll
        for (int n = 0; n < NE; ++n) {
            const int el = threadIdx.x + n * E_THREADS;
            const int x = el / T2, y = (el / T) % T, z = el % T;
            // every element of a block is allocated; those with an index >= v
            // were never written and are masked after an unconditional load
            const double w = (double)ba[el] + (double)bb[(y * T + x) * T + z] + (double)bc[(z * T + x) * T + y];
            wv[s][n] = keep_if(w, X * T + x < v && Y * T + y < v && Z * T + z < v);
        }
    }
    // LDS stores
#pragma unroll
    for (int n = 0; n < NG; ++n) {
        const int el = threadIdx.x + n * E_THREADS;
        if (el < 27 * T2) (&Gs[0][0][0][0])[el - el % T2 + gidx(el % T2 / T, el % T)] = gv[n];
    }
    if (threadIdx.x < 9 * T) (&t1s[0][0][0])[threadIdx.x] = t1v;
    if constexpr (FOCK) {
#pragma unroll
        for (int n = 0; n < NG; ++n) {
            const int el = threadIdx.x + n * E_THREADS;
            if (el < 27 * T2) (&Ts[0][0][0][0])[el - el % T2 + gidx(el % T2 / T, el % T)] = tv[n];
        }
        if (threadIdx.x < 9 * T) (&fs[0][0][0])[threadIdx.x] = fv;
    }
#pragma unroll
    for (int s = 0; s < 6; ++s)
#pragma unroll
        for (int n = 0; n < NE; ++n) {
            const int el = threadIdx.x + n * E_THREADS;
            Ws[s][widx(el / T2, (el / T) % T, el % T)] = wv[s][n];
        }
    __syncthreads();

    // phase 3: one element (a, b, c) of the base tile and its six permutations
    const double eocc = e.eps_o[i] + e.eps_o[j] + e.eps_o[k];
    double acc = 0.0;
    for (int el = threadIdx.x; el < E_T3; el += E_THREADS) {
        const int l[3] = {el / T2, (el / T) % T, el % T};  // locals of a, b, c
        const int a = TT[0] * T + l[0], b = TT[1] * T + l[1], c = TT[2] * T + l[2];
        if (a >= v || b >= v || c >= v) continue;
        double W[6], V[6];
        // t_{i,j,k} at the element's three virtuals (tile id A, local l[A])
        double tv[3][3];
#pragma unroll
        for (int n = 0; n < 3; ++n)
#pragma unroll
            for (int A = 0; A < 3; ++A) tv[n][A] = t1s[n][A][l[A]];
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            // permutation p puts tile ids (X, Y, Z) on the virtual slots a, b, c
            const int X = perm[p][0], Y = perm[p][1], Z = perm[p][2];
            const int x = l[X], y = l[Y], z = l[Z];
            W[p] = Ws[p][widx(x, y, z)];
            V[p] = W[p] + tv[0][X] * Gs[0][Y][Z][gidx(y, z)] + tv[1][Y] * Gs[1][X][Z][gidx(x, z)] +
                   tv[2][Z] * Gs[2][X][Y][gidx(x, y)];
            if constexpr (FOCK)
                V[p] += fs[0][X][x] * Ts[0][Y][Z][gidx(y, z)] + fs[1][Y][y] * Ts[1][X][Z][gidx(x, z)] +
                        fs[2][Z][z] * Ts[2][X][Y][gidx(x, y)];
        }
        const double d = eocc - e.eps_v[a] - e.eps_v[b] - e.eps_v[c];
        const double se = V[0] + V[3] + V[4], so = V[1] + V[2] + V[5];
        const double we = W[0] + W[3] + W[4], wo = W[1] + W[2] + W[5];
        double wv = 0.0;
#pragma unroll
        for (int p = 0; p < 6; ++p) wv += W[p] * V[p];
        const double num = 3.0 * wv + (se - 2.0 * so) * we + (so - 2.0 * se) * wo;
        acc += num / d;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < E_THREADS / 64; ++w) s += red[w];
        e.partial[(int64_t)t * e.norbit + orb] = s / (double)ob.w;
    }
}

template <typename HT, bool FOCK>
__global__ __launch_bounds__(E_THREADS) void epilogue_kernel(EpiLaunch e) {
    epilogue_body<HT, FOCK>(e, blockIdx.x, blockIdx.y);
}

// Index of the entry with the largest first block <= b (entries ascending).
template <typename T>
__device__ __forceinline__ int group_entry(const T* __restrict__ ent, int nent, int b) {
    int lo = 0, hi = nent - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ent[mid].wg0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One epilogue launch over several solves: entry e has ntrip x norbit work
// groups from its wg0 on (orbit fastest).
template <typename HT>
__global__ __launch_bounds__(E_THREADS) void epilogue_group_kernel(const EpiGroupEntry* __restrict__ ent, int nent) {
    const int b = blockIdx.x;
    const EpiGroupEntry x = ent[group_entry(ent, nent, b)];
    const int l = b - x.wg0;
    epilogue_body<HT, false>(x.e, l % x.e.norbit, l / x.e.norbit);
}

// Neumaier compensated accumulation: (s, c) += x
__device__ __forceinline__ void neu_add(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

constexpr int R_THREADS = 256;

// Fixed-order compensated sum of n values at stride 1; block-wide result in thread 0.
__device__ double block_sum_fixed(const double* x, int64_t n) {
    __shared__ double ss[R_THREADS], cs[R_THREADS];
    double s = 0.0, c = 0.0;
    // thread t adds x[t], x[t + R], x[t + 2R], ... in this order; the loads of
    // RU consecutive terms are issued together (terms past n read x[n - 1]
    // and are masked to +0, which leaves (s, c) unchanged)
    constexpr int RU = 8;
    for (int64_t idx = threadIdx.x; idx < n; idx += RU * R_THREADS) {
        double xv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t q = idx + (int64_t)u * R_THREADS;
            xv[u] = keep_if(x[q < n ? q : n - 1], q < n);
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) neu_add(s, c, xv[u]);
    }
    ss[threadIdx.x] = s;
    cs[threadIdx.x] = c;
    __syncthreads();
    for (int half = R_THREADS / 2; half >= 1; half >>= 1) {
        if ((int)threadIdx.x < half) {
            double s1 = ss[threadIdx.x], c1 = cs[threadIdx.x];
            neu_add(s1, c1, ss[threadIdx.x + half]);
            c1 += cs[threadIdx.x + half];
            ss[threadIdx.x] = s1;
            cs[threadIdx.x] = c1;
        }
        __syncthreads();
    }
    return ss[0] + cs[0];
}

__global__ __launch_bounds__(R_THREADS) void reduce_triples_kernel(const double* partial, int norbit,
                                                                     const int4* trip, double* e_trip) {
    const int t = blockIdx.x;
    const double s = block_sum_fixed(partial + (int64_t)t * norbit, norbit);
    if (threadIdx.x == 0) e_trip[t] = s * (double)trip[t].w / 3.0;
}

__global__ __launch_bounds__(R_THREADS) void reduce_total_kernel(const double* e_trip, int64_t n,
                                                                   double* out) {
    const double s = block_sum_fixed(e_trip, n);
    if (threadIdx.x == 0) *out = s;
}

// Per-triple sums of several solves: one block per triple, entry by entry.
__global__ __launch_bounds__(R_THREADS) void reduce_triples_group_kernel(const RedGroupEntry* __restrict__ ent,
                                                                           int nent) {
    int lo = 0, hi = nent - 1;
    const int b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ent[mid].b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const RedGroupEntry x = ent[lo];
    const int t = b - x.b0;
    const double s = block_sum_fixed(x.partial + (int64_t)t * x.norbit, x.norbit);
    if (threadIdx.x == 0) x.e_trip[t] = s * (double)x.trip[t].w / 3.0;
}

// The totals of several solves: one block per entry.
__global__ __launch_bounds__(R_THREADS) void reduce_total_group_kernel(const TotalGroupEntry* __restrict__ ent) {
    const TotalGroupEntry x = ent[blockIdx.x];
    const double s = block_sum_fixed(x.e_trip, x.n);
    if (threadIdx.x == 0) *x.out = s;
}

}  // namespace

KernelCall epilogue_call(int precision, const EpiLaunch& e) {
    if (e.ntrip > 65535) throw Error(-1, "epilogue batch too large");
    KernelCall k;
    const bool f = e.fock_ov != nullptr;
    k.fn = precision == 0 ? (f ? (const void*)&epilogue_kernel<double, true> : (const void*)&epilogue_kernel<double, false>)
                          : (f ? (const void*)&epilogue_kernel<float, true> : (const void*)&epilogue_kernel<float, false>);
    k.grid = dim3(e.norbit, e.ntrip);
    k.block = dim3(E_THREADS);
    k.arg(e);
    return k;
}

KernelCall epilogue_group_call(int precision, const EpiGroupEntry* d_ent, int nent, int64_t n_wg) {
    if (n_wg > ((int64_t)1 << 31) - 1) throw Error(-1, "grouped epilogue grid too large");
    KernelCall k;
    k.fn = precision == 0 ? (const void*)&epilogue_group_kernel<double> : (const void*)&epilogue_group_kernel<float>;
    k.grid = dim3((unsigned)n_wg);
    k.block = dim3(E_THREADS);
    k.arg(d_ent).arg(nent);
    return k;
}

KernelCall reduce_triples_group_call(const RedGroupEntry* d_ent, int nent, int nblocks) {
    KernelCall k;
    k.fn = (const void*)&reduce_triples_group_kernel;
    k.grid = dim3(nblocks);
    k.block = dim3(R_THREADS);
    k.arg(d_ent).arg(nent);
    return k;
}

KernelCall reduce_total_group_call(const TotalGroupEntry* d_ent, int nent) {
    KernelCall k;
    k.fn = (const void*)&reduce_total_group_kernel;
    k.grid = dim3(nent);
    k.block = dim3(R_THREADS);
    k.arg(d_ent);
    return k;
}

KernelCall reduce_triples_call(const double* partial, int ntrip, int norbit, const int4* trip,
                               double* e_trip) {
    KernelCall k;
    k.fn = (const void*)&reduce_triples_kernel;
    k.grid = dim3(ntrip);
    k.block = dim3(R_THREADS);
    k.arg(partial).arg(norbit).arg(trip).arg(e_trip);
    return k;
}

KernelCall reduce_total_call(const double* e_trip, int64_t n, double* out) {
    KernelCall k;
    k.fn = (const void*)&reduce_total_kernel;
    k.grid = dim3(1);
    k.block = dim3(R_THREADS);
    k.arg(e_trip).arg(n).arg(out);
    return k;
}

}  // namespace bqc
