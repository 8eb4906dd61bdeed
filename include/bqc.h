/*
 * bqc.h - C ABI of the MI355X (gfx950) closed-shell (T) energy library.
 *
 * The library computes the perturbative-triples correction E_T of CCSD(T)
 * for a closed-shell canonical Hartree-Fock reference (paper section 2.4.2,
 * Eqs. 2-7): from the converged CCSD singles t1 and doubles t2, the orbital
 * energies and the MO integrals (ia|bc), (ia|jl), (ia|jb) it returns one
 * scalar.  Everything of the computation runs in HIP kernels on one GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * o = nocc >= 1 occupied, v = nvir >= 1 virtual spatial orbitals.  All arrays
 * are dense, row-major (last index fastest), IEEE FP64:
 *   eps_o [o]             occupied orbital energies e_i
 *   eps_v [v]             virtual orbital energies e_a
 *   t1    [o][v]          t_i^a
 *   t2    [o][o][v][v]    t_ij^ab  (the caller guarantees t_ij^ab = t_ji^ba)
 *   ovvv  [o][v][v][v]    (ia|bc)  chemists' notation, symmetric in b,c
 *   ooov  [o][o][o][v]    ooov[j][l][i][a] = (jl|ia) = (ia|jl)
 *   ovov  [o][v][o][v]    (ia|jb)
 * Symmetries of the inputs are not checked.  The gap condition
 * max(eps_o) < min(eps_v) is checked (it makes every energy denominator
 * e_i + e_j + e_k - e_a - e_b - e_c negative); a violated gap, a non-finite
 * orbital energy, a null pointer or a size below 1 returns BQC_EINVAL.
 *
 * Input buffers are borrowed, read-only and owned by the caller.  Outputs are
 * written only when the call returns BQC_OK; on any error nothing is written.
 * No C++ exception crosses this interface.  bqc_last_error() returns a
 * thread-local message for the last non-OK return of the calling thread.
 *
 * Unique occupied triples: i <= j <= k without i = j = k, in lexicographic
 * order of (i, j, k).  There are o(o+1)(o+2)/6 - o of them; their per-triple
 * energies sum to E_T.
 */
#ifndef BQC_H
#define BQC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BQC_OK         0
#define BQC_PENDING    1   /* bqc_t_poll only: the request has not finished */
#define BQC_EINVAL    -1   /* bad argument (see above) */
#define BQC_ENOMEM    -2   /* request larger than the memory budget, or a device allocation failed */
#define BQC_EDEVICE   -3   /* HIP runtime or kernel failure */
#define BQC_ENOTFOUND -4   /* unknown or already consumed ticket */
#define BQC_ESHUTDOWN -5   /* the server is shutting down */
#define BQC_ECANCELED -6   /* the request was cancelled before it ran (bqc_t_cancel) */

/* Arithmetic of the contractions (Eq. 2).  The energy denominator, the
 * per-triple energy and the sum over triples are FP64 in every mode. */
typedef enum {
    BQC_PREC_FP64   = 0,  /* FP64 MFMA, FP64 accumulation */
    BQC_PREC_FP32   = 1,  /* FP32 operands, FP32 MFMA accumulation */
    BQC_PREC_BF16X3 = 2,  /* split x = hi + lo in bf16, hi*hi + hi*lo + lo*hi, FP32 accumulation */
    BQC_PREC_FP8    = 3   /* FP8 e4m3 operands with a power-of-two scale per 32 contraction elements */
} bqc_precision;

/*
 * Synchronous single solve (paper Eqs. 2-7): host input pointers, FP64
 * contractions, device 0, the library's own stream.  Writes *E_T on success.
 */
int bqc_t_energy(int32_t nocc, int32_t nvir,
                 const double* eps_o, const double* eps_v,
                 const double* t1, const double* t2,
                 const double* ovvv, const double* ooov, const double* ovov,
                 double* E_T);

/* Options of bqc_t_energy_ex.  A zero-initialised struct means: FP64,
 * device 0, host inputs, library stream, no per-triple output.  The first
 * four fields are the boundary's base options (precision, device, input
 * residency, stream); the fields after them extend it, so a caller that
 * knows only the first four and zero-fills the rest gets the defaults. */
typedef struct {
    int32_t precision;        /* bqc_precision */
    int32_t device;           /* HIP device ordinal */
    int32_t inputs_on_device; /* 1: the seven input pointers are device pointers on `device`,
                                 readable in stream order on `stream` */
    void*   stream;           /* hipStream_t to run on, or NULL for the library's stream of `device` */
    /* ---- extensions (zero = default) ---- */
    int32_t timing;           /* 1: record per-kernel HIP events and fill the kernel fields of stats */
    int32_t formulation;      /* BQC_FORM_OCCUPIED (0, default): the loop runs over unique occupied
                                 triples i <= j <= k with tensors over the virtuals.  BQC_FORM_VIRTUAL:
                                 the loop runs over unique virtual triples a <= b <= c with tensors over
                                 the occupied indices (the loop order of paper section 2.4.2); E_T is the
                                 same sum taken in the other order.  With BQC_FORM_VIRTUAL "triple" in
                                 triple_energies, triple_begin and triple_end means a unique virtual
                                 triple (a <= b <= c, lexicographic, a = b = c skipped;
                                 bqc_t_num_triples(nvir) of them), stats->flops is 12 n_triples nocc^3
                                 (nocc + nvir), and BQC_PREC_FP8 is rejected with BQC_EINVAL.  Any
                                 other value: BQC_EINVAL.  A solve whose loop has more than 2^31 - 1
                                 unique triples (nvir > 2343 here) is rejected with BQC_EINVAL. */
    double* triple_energies;  /* NULL, or a HOST array of bqc_t_num_triples(nocc) doubles that receives
                                 the per-triple energies e_ijk in unique-triple order (with a triple
                                 range, only the entries of the range are written) */
    int64_t triple_begin;     /* first unique triple of the share (see triple_end) */
    int64_t triple_end;       /* Share of the solve: only the unique triples with index in
                                 [triple_begin, triple_end) of the unique-triple order (i <= j <= k,
                                 lexicographic, i = j = k skipped) are computed, and E_T is their
                                 fixed-order compensated sum.  triple_end = 0 means all triples
                                 (triple_begin must then be 0).  Otherwise 0 <= triple_begin <
                                 triple_end <= bqc_t_num_triples(nocc), else BQC_EINVAL.  Shares of
                                 one solve (one per GPU, or consecutive pieces of a long solve) add
                                 up to the whole: every triple's energy does not depend on the range. */
    const double* fock_ov;    /* NULL: canonical reference (f_ov = 0).  Else f_ia, [nocc][nvir] FP64, host
                                 or device memory like the other inputs: the occupied-virtual Fock block
                                 of a reference with diagonal occupied and virtual blocks (orbital
                                 energies eps); adds the f_ov t2 part of the disconnected triples (paper
                                 Eqs. 5 and 7: x_k F_ck), folded into V as f_ia t_jk^bc + f_jb t_ik^ac +
                                 f_kc t_ij^ab.  Must be finite (host) else BQC_EINVAL. */
} bqc_t_opts;

#define BQC_FORM_OCCUPIED 0
#define BQC_FORM_VIRTUAL  1

/* Per-solve measurements.  Times are seconds.  The first six fields are the
 * boundary's base statistics; the fields after them extend it. */
typedef struct {
    double   queue_s;      /* serving: submit -> admission */
    double   upload_s;     /* host -> device copies (0 for device inputs) */
    double   gpu_s;        /* first kernel start -> final reduction end (HIP events) */
    double   total_s;      /* wall time of the call (serving: submit -> completion) */
    double   flops;        /* algorithmic flops 12 * n_triples * v^3 * (v + o) */
    uint64_t footprint_bytes; /* device memory the solve held */
    /* ---- extensions ---- */
    double   prepare_s;    /* layout and precision conversion of the inputs (HIP events) */
    double   gemm_s;       /* timing=1: summed duration of the contraction kernel launches */
    double   epilogue_s;   /* timing=1: summed duration of the epilogue kernel launches */
    int32_t  gemm_launches;
    int32_t  epilogue_launches;
    int32_t  precision;
    int32_t  n_triples;
} bqc_t_stats;

/*
 * Single solve with options (see bqc_t_opts).  Returns when *E_T is known
 * (the stream is synchronised).  stats may be NULL.
 */
int bqc_t_energy_ex(int32_t nocc, int32_t nvir,
                    const double* eps_o, const double* eps_v,
                    const double* t1, const double* t2,
                    const double* ovvv, const double* ooov, const double* ovov,
                    const bqc_t_opts* opts, double* E_T, bqc_t_stats* stats);

/*
 * Single solve with (ia|bc) formed on the device from density-fitting
 * factors (paper section 2.2: (pq|rs) = sum_Q B^Q_pq B^Q_rs) instead of being
 * passed as the o*v^3 array:
 *   b_ov  [naux][nocc][nvir]  = B^Q_ia        (row-major, FP64)
 *   b_vv  [naux][nvir][nvir]  = B^Q_bc        (symmetric in b, c)
 * The other inputs, the options (inputs_on_device applies to b_ov and b_vv
 * too), the outputs and the error codes are those of bqc_t_energy_ex; naux
 * must be >= 1 and b_ov, b_vv non-NULL (else BQC_EINVAL).  The product over Q
 * runs in FP64 on the device for a few occupied indices at a time and goes
 * straight into the contraction operand of the chosen precision, so no
 * o*v^3 FP64 array is held (device memory for it: a bounded scratch of at
 * most max(v^3, 2^26) doubles).  E_T equals bqc_t_energy_ex's with
 * ovvv = sum_Q b_ov b_vv up to the rounding of that product.
 */
int bqc_t_energy_df(int32_t nocc, int32_t nvir, int32_t naux,
                    const double* eps_o, const double* eps_v,
                    const double* t1, const double* t2,
                    const double* b_ov, const double* b_vv,
                    const double* ooov, const double* ovov,
                    const bqc_t_opts* opts, double* E_T, bqc_t_stats* stats);

/*
 * Closed-shell MP2 correlation energy with density-fitted integrals (the
 * paper's MP2 equation; (ia|jb) = sum_Q B^Q_ia B^Q_jb):
 *   E_MP2 = sum_{ijab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b).
 * Inputs: eps_o[nocc], eps_v[nvir], b_ov[naux][nocc][nvir] (FP64, row-major),
 * borrowed.  Of the options only precision (must be BQC_PREC_FP64), device,
 * inputs_on_device, stream, timing and triple_energies are used (opts may be
 * NULL); here triple_energies is NULL or a HOST array of nocc(nocc+1)/2
 * doubles that receives the pair energies e_ij, i <= j in lexicographic
 * order (e_ij = sum_ab (ia|jb)[2(ia|jb) - (ib|ja)]/D_ij^ab, doubled for
 * i < j to count the pair (j, i)), of which E_MP2 is the sum.  The
 * integrals are contracted on FP64 MFMA per occupied pair and virtual tile
 * pair with the denominator applied in registers (no four-index tensor is
 * stored); the sum is fixed-order and compensated.  Errors: BQC_EINVAL for
 * sizes < 1, NULL pointers, a non-FP64 precision, non-finite orbital energies
 * or no gap (max eps_o >= min eps_v); BQC_ENOMEM, BQC_EDEVICE as elsewhere.
 * stats (may be NULL): gpu_s, total_s, upload_s, flops = nocc(nocc+1)/2 *
 * 2 nvir^2 naux, footprint_bytes.
 */
int bqc_mp2_energy_df(int32_t nocc, int32_t nvir, int32_t naux,
                      const double* eps_o, const double* eps_v, const double* b_ov,
                      const bqc_t_opts* opts, double* E_MP2, bqc_t_stats* stats);

/* ------------------------------------------------------------------ batch
 * Several independent fragments solved together (the fragments of the
 * paper's embedding layer, section 2.5, are independent (T) problems of
 * uneven size).  Small fragments are bound by launch overhead when solved
 * one by one (the batching argument of section 2.4.2); here each step of
 * the path is one grouped launch over all fragments (operand conversion, then
 * rounds of contraction / epilogue / per-triple sums over every fragment's
 * current triple batch, then the totals).  E_T[f] is bitwise the energy
 * bqc_t_energy_ex returns for fragment f alone with the same options.
 *
 * frags[f] holds fragment f's sizes and its seven inputs (layouts as for
 * bqc_t_energy); opts (may be NULL) applies to all of them: precision,
 * device, inputs_on_device (then every pointer of every fragment is a
 * device pointer) and stream are used; formulation must be
 * BQC_FORM_OCCUPIED and triple_begin / triple_end / fock_ov /
 * triple_energies must be zero (else BQC_EINVAL); timing is ignored.  E_T
 * is a HOST array of nfrag doubles, written only on BQC_OK.  nfrag = 0 is
 * BQC_OK with nothing written.  An invalid fragment fails the whole call
 * with BQC_EINVAL (the message names the fragment).  stats (may be NULL):
 * the batch's gpu_s, total_s, upload_s, summed flops and triples,
 * footprint_bytes (bqc_t_batch_footprint), gemm_launches (grouped
 * contraction launches) and epilogue_launches (grouped epilogue launches).
 * The H buffers of a batch take at most 8 GiB together (fragments then run
 * their triples in more rounds); the rest of the workspace grows with the
 * fragments' sizes.
 */
typedef struct {
    int32_t nocc, nvir;
    const double *eps_o, *eps_v, *t1, *t2, *ovvv, *ooov, *ovov;
} bqc_t_fragment;

int bqc_t_energy_batch(int32_t nfrag, const bqc_t_fragment* frags, const bqc_t_opts* opts,
                       double* E_T, bqc_t_stats* stats);

/* Device bytes a batch of these fragment shapes holds (inputs included, as
 * for host inputs), or -1 for invalid arguments. */
int64_t bqc_t_batch_footprint(int32_t nfrag, const int32_t* nocc, const int32_t* nvir, int32_t precision);

/* Number of unique triples p <= q <= r (p = q = r excluded) of an orbital
 * space of n orbitals: the occupied triples for n = nocc, the virtual
 * triples of BQC_FORM_VIRTUAL for n = nvir (0 for n < 1). */
int64_t bqc_t_num_triples(int32_t nocc);

/* Device bytes one solve of this shape and precision holds (its footprint,
 * inputs included) with the default formulation and a canonical reference,
 * or -1 for invalid arguments. */
int64_t bqc_t_footprint(int32_t nocc, int32_t nvir, int32_t precision);

/* bqc_t_footprint for a formulation (BQC_FORM_*) and a reference with
 * (fock != 0) or without an f_ov block: the loop over virtual triples also
 * holds transposed copies of t1, (ia|jb) and, with f_ov, t2 and f_ov.
 * -1 for invalid arguments (sizes < 1, unknown precision or formulation,
 * FP8 with BQC_FORM_VIRTUAL). */
int64_t bqc_t_footprint_ex(int32_t nocc, int32_t nvir, int32_t precision, int32_t formulation, int32_t fock);

/* ------------------------------------------------------- no device allocation
 * For callers that cannot allocate device memory (code running under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * solve of bqc_t_energy_ex with device-resident inputs whose workspace is a
 * fixed device array of the library, BQC_NOALLOC_SCRATCH_BYTES bytes on each
 * device the library runs on, held from its first use until the process
 * ends.  The call allocates no device memory and creates no stream or event.
 *
 * opts is required and must have inputs_on_device = 1 (else BQC_EINVAL); the
 * seven input pointers (and fock_ov, if set) are device pointers on
 * opts->device, read in stream order on opts->stream (NULL: the device's
 * null stream).  precision, formulation, triple_begin/triple_end, fock_ov
 * and triple_energies (a HOST array, as in bqc_t_energy_ex) work as in
 * bqc_t_energy_ex; timing is ignored.  Returns after the stream has drained,
 * with *E_T bitwise equal to bqc_t_energy_ex's for the same arguments (the
 * kernels and every summation order are the same; only the number of triples
 * per launch may be smaller).  stats (may be NULL): flops, footprint_bytes
 * (bytes of the array used), precision and n_triples; the time fields are 0.
 *
 * A shape whose workspace does not fit the array, even at one triple per
 * launch, is rejected with BQC_ENOMEM (bqc_t_noalloc_batch returns 0 for it);
 * other errors as bqc_t_energy_ex.  Every call on one device uses the same
 * array: calls that overlap in time on one device race and must be
 * serialised by the caller.
 */
#define BQC_NOALLOC_SCRATCH_BYTES (64u << 20)

int bqc_t_energy_noalloc(int32_t nocc, int32_t nvir,
                         const double* eps_o, const double* eps_v,
                         const double* t1, const double* t2,
                         const double* ovvv, const double* ooov, const double* ovov,
                         const bqc_t_opts* opts, double* E_T, bqc_t_stats* stats);

/* Triples per launch bqc_t_energy_noalloc uses for this shape (0: the shape
 * does not fit the array; -1: invalid arguments, as bqc_t_footprint_ex). */
int64_t bqc_t_noalloc_batch(int32_t nocc, int32_t nvir, int32_t precision, int32_t formulation, int32_t fock);

/* ---------------------------------------------------------------- serving
 * Continuous batching of independent (T) solves.  The paper's embedding
 * layer splits a system into fragments (clusters) whose correlated
 * calculations are independent problems of uneven size (section 2.5), and
 * the cost of the small ones is dominated by launch overhead unless their
 * work is batched (section 2.4.2); a server keeps many such solves in
 * flight on one device.
 *
 * A server owns one device, a device memory arena of mem_budget_bytes
 * (allocated once at creation; the serving loop itself never allocates) and
 * max_inflight slot threads, each with its own streams.  A request is one
 * solve; an idle slot admits the oldest queued request whose footprint
 * (workspace, plus the inputs when they are host arrays) fits the arena
 * (smaller requests may overtake a waiting one a bounded number of times),
 * uploads it and runs its launch sequence, so admitted requests run
 * concurrently on the device while new ones keep arriving.  A request's
 * result is bitwise identical to bqc_t_energy_ex at the same precision on
 * the same device: its decomposition and reduction order depend only on
 * (nocc, nvir, precision).  A failing request (device error, failed host
 * allocation) returns its error at its terminal poll; its memory returns to
 * the arena after its streams have drained, and other requests are not
 * affected.
 */
typedef struct bqc_server bqc_server;

typedef struct {
    int32_t  device;           /* HIP device ordinal */
    int32_t  precision;        /* bqc_precision for every request */
    uint64_t mem_budget_bytes; /* 0: 85% of the device's free memory at creation */
    int32_t  max_inflight;     /* 0: 4 */
    int32_t  direct_launch;    /* 0: each request's triple-batch launch sequence is built as one hipGraph
                                  (kernel nodes, no stream capture) and launched as a unit; 1: kernels
                                  are launched one by one on the slot's two streams */
    int32_t  no_grouping;      /* 0: a slot that admits a small request (at most 5e11 algorithmic flops,
                                  a few milliseconds of contraction) also admits up to 31 more queued
                                  small ones that fit the arena together and runs them as one batch
                                  (bqc_t_energy_batch's grouped launches; each result is bitwise the
                                  request's alone; a failure of the batch is every member's);
                                  1: one request per slot */
} bqc_server_cfg;

/* Creates a server; *out is written on BQC_OK. */
int bqc_server_create(const bqc_server_cfg* cfg, bqc_server** out);

/* Cancels queued requests (they never run), waits for admitted ones, frees
 * every device buffer, every ticket and the server.  No ticket of the server
 * may be polled afterwards. */
int bqc_server_destroy(bqc_server* s);

/*
 * Enqueues one solve with HOST input pointers.  The buffers are borrowed
 * until bqc_t_poll returns a terminal status for the ticket.  A request whose
 * footprint exceeds the budget is rejected here with BQC_ENOMEM and never
 * queued.  *ticket is written on BQC_OK.  Thread-safe.
 */
int bqc_t_submit(bqc_server* s, int32_t nocc, int32_t nvir,
                 const double* eps_o, const double* eps_v,
                 const double* t1, const double* t2,
                 const double* ovvv, const double* ooov, const double* ovov,
                 uint64_t* ticket);

/*
 * bqc_t_submit with a choice of input residency.  inputs_on_device = 1: the
 * seven pointers are device pointers on the server's device (they are read
 * in place, never copied, and must stay valid and unmodified until the
 * ticket's terminal poll; the request's footprint is then its workspace
 * only).  inputs_on_device = 0 is bqc_t_submit.  Thread-safe.
 */
int bqc_t_submit_ex(bqc_server* s, int32_t nocc, int32_t nvir,
                    const double* eps_o, const double* eps_v,
                    const double* t1, const double* t2,
                    const double* ovvv, const double* ooov, const double* ovov,
                    int32_t inputs_on_device, uint64_t* ticket);

/*
 * Non-blocking status of a ticket: BQC_PENDING while queued or running;
 * BQC_OK with *E_T (and *stats if non-NULL) written once it finished; a
 * negative code if the request failed.  A terminal return consumes the
 * ticket (a later poll returns BQC_ENOTFOUND).  Thread-safe.
 */
int bqc_t_poll(bqc_server* s, uint64_t ticket, double* E_T, bqc_t_stats* stats);

/* Blocking variant of bqc_t_poll (waits until the ticket is terminal).  If
 * another thread consumes the ticket meanwhile, returns BQC_ENOTFOUND. */
int bqc_t_wait(bqc_server* s, uint64_t ticket, double* E_T, bqc_t_stats* stats);

/* Cancels a queued request: it is removed from the queue and never runs; its
 * terminal poll returns BQC_ECANCELED.  Returns BQC_OK (cancelled, or the
 * request had already finished: its poll tells which), BQC_PENDING (it is
 * running and will complete normally), BQC_ENOTFOUND (unknown or consumed
 * ticket).  Thread-safe. */
int bqc_t_cancel(bqc_server* s, uint64_t ticket);

/* Thread-local message of the calling thread's last non-OK return. */
const char* bqc_last_error(void);

/* ABI version: major * 10000 + minor * 100 + patch. */
int32_t bqc_version(void);

/* HIP versions (major * 10000000 + minor * 100000 + patch): *compiled = the
 * HIP headers the library was built with, *runtime = hipRuntimeGetVersion()
 * of the HIP runtime the process has loaded (the library binds to the one
 * runtime of the process, e.g. the one a framework loaded first).  Either
 * pointer may be NULL.  Returns BQC_OK, or BQC_EDEVICE if the runtime cannot
 * report its version. */
int bqc_hip_versions(int32_t* compiled, int32_t* runtime);

#ifdef __cplusplus
}
#endif

#endif /* BQC_H */
