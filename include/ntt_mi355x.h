/*
 * ntt_mi355x.h -- C ABI of the batched negacyclic NTT library for MI355X (gfx950).
 *
 * Paper: Kim, Jung, Park, Ahn, "Accelerating Number Theoretic Transformations for
 * Bootstrappable Homomorphic Encryption on GPUs", arXiv 2012.01968.
 *
 * Problem statement (Section III-B; Algorithm 1, its REQUIRE and ENSURE clauses):
 * a polynomial of Z_Q[X]/(X^N+1) is held in RNS form as L residue vectors of length
 * N, vector l taken mod a prime q_l = 1 (mod 2N).  The library applies the merged-twist
 * NTT (Section III-A) to every vector of a batch, its inverse, the element-wise
 * product in the NTT domain, and the full negacyclic product.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Data layout   A batch is a device array of uint64_t laid out [n_polys][L][N]
 *               (limb-major, each limb vector contiguous).  Vector (p, l) starts at
 *               element (p*L + l)*N and is reduced mod q_l.
 * Values        Inputs must be canonical residues in [0, q_l); outputs are canonical.
 * Order         Forward output and inverse input are in bit-reversed order: slot i of
 *               the forward output holds A_{brv(i)} = sum_n a_n psi^{n(2 brv(i)+1)},
 *               exactly what Algorithm 1 leaves in place.  Inverse output and polymul
 *               inputs/outputs are coefficients in natural order.
 * Root          psi_l is the smallest primitive 2N-th root of unity mod q_l (the paper
 *               does not fix one; ntt_plan_get_roots reports the roots in use).
 * Streams       `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *               Calls enqueue work on it and return at once; results are ready when
 *               the stream reaches that point.
 * Memory        The caller owns every data buffer.  The plan owns its device tables.
 *               Device pointers must be 16-byte aligned.
 * Errors        Argument errors are reported synchronously and nothing is enqueued.
 *               A failed launch returns NTT_ERR_HIP; faults that happen on the device
 *               surface at the caller's next synchronisation with the stream.
 *               No C++ exception crosses this interface.
 * Threads       A plan is immutable after creation and may be used from any host
 *               thread and stream at once.  ntt_polymul_negacyclic keeps one scratch
 *               buffer per stream, so products on different streams never wait for each
 *               other.
 */
#ifndef NTT_MI355X_H
#define NTT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ntt_plan_s* ntt_plan_t;

typedef enum {
    NTT_OK = 0,
    NTT_ERR_ARG = -1,          /* null pointer, zero count, bad option value       */
    NTT_ERR_N = -2,            /* N not a power of two in [2, 2^17]                */
    NTT_ERR_PRIME = -3,        /* a modulus is not prime, not 1 mod 2N, not below  */
                               /* 2^62, or repeated                                */
    NTT_ERR_NOMEM = -4,        /* host or device allocation failed                 */
    NTT_ERR_HIP = -5,          /* a HIP runtime call or kernel launch failed       */
    NTT_ERR_UNSUPPORTED = -6   /* option combination not built into the library    */
} ntt_status;

/* Twiddle sources (Section VII).  TABLE reads every twiddle and its Shoup companion
 * from a precomputed table; OT ("on-the-fly twiddling") rebuilds the twiddles of the
 * last `ot_stages` forward stages (first inverse stages) from two small base tables by
 * multiplying the operand by both factors in turn. */
enum { NTT_TWIDDLE_AUTO = 0, NTT_TWIDDLE_TABLE = 1, NTT_TWIDDLE_OT = 2 };

/* Plan options.  A zero-filled struct (or NULL) asks for the defaults. */
typedef struct {
    int32_t twiddle_mode;   /* NTT_TWIDDLE_*; AUTO picks TABLE unless ot_stages > 0     */
    int32_t ot_stages;      /* 1 or 2: stages rebuilt on the fly (OT mode); 0 = 2       */
    int32_t ot_log2_base;   /* log2 of the OT digit base; 0 = 10 (base 1024)            */
    int32_t log2_n1;        /* size of the first (column) pass, N = N1 * N2; 0 = auto;  */
                            /* -1 forces the single-pass kernel where N allows it       */
    int32_t kernel_path;    /* NTT_PATH_*: how the two passes are launched               */
    int32_t use_autotune;   /* 1: fill the fields above that are zero from the tuner's   */
                            /* measured choice for this shape (see below); 0: do not    */
    int32_t tune_polys;     /* polynomials per call the plan is tuned for; 0 = 1         */
    int32_t order;          /* NTT_ORDER_*: slot order of the NTT domain (see below)     */
    int32_t log2_radix;     /* NTT_PATH_REGISTER: stages per launch, 2..5; 0 = 4         */
    int32_t word_bits;      /* residue word: 0 or 64 = uint64_t, 32 = uint32_t (below)   */
    int32_t r1;             /* row pass values per lane (per-thread NTT size): 0 = 8, 4, 8 */
    int32_t wg_size;        /* row pass workgroup lanes: 0 = 128, 64, 128, 256           */
    int32_t col_width;      /* column pass tile width in adjacent columns: 0 = automatic, */
                            /* 16 .. 256 (at most N2; longer columns take fewer)         */
    int32_t reserved;       /* must be zero                                             */
} ntt_plan_opts;
/* Tile options (r1, wg_size, col_width; Section VI-C's per-thread NTT size and thread-block
 * shape) apply to 64-bit plans on the split path; elsewhere they are refused with
 * NTT_ERR_UNSUPPORTED, as is r1 = 4 for rows of 8192 points (a row's lanes form one
 * workgroup of at most 1024) and a col_width wider than N2.  The shape applies to every row
 * pass of the plan, the key-product rows of ntt_polymul_negacyclic and NTT_OP_MULKEY batch
 * jobs included.  Every tile shape computes the same residues; only the speed differs. */

/* Slot order of the NTT domain (Section III-C).  BITREV (the default) is Algorithm 1's own
 * order: forward output slot i holds A_{brv(i)}, and the inverse takes that order.  NATURAL
 * puts A_i in slot i: the forward transform ends with an in-place bit-reversal permutation
 * of every vector and the inverse begins with one (one more read and write of the data per
 * transform, the cost for which the paper keeps HE in bit-reversed order).  The order
 * applies to ntt_forward / ntt_inverse (and their passes) and to the NTT-domain keys of
 * batch jobs; ntt_pointwise_mul works in either order and ntt_polymul_negacyclic does not
 * depend on it. */
enum { NTT_ORDER_BITREV = 0, NTT_ORDER_NATURAL = 1 };

/* Tuned plans (Section VI-C's choice of kernel sizes, Section VII's OT depth and base, made
 * by measurement).  The Python tuner (paper_2012_01968_amd/autotune.py) writes its choices to
 * a text file, one line per shape:
 *   <arch>:<CUs>CU <kernel source hash> <N> <L> <P> <prime bits> <log2_n1> <twiddle_mode>
 *   <ot_stages> <ot_log2_base> <kernel_path> [<r1> <wg_size> <col_width>]
 * With use_autotune = 1, ntt_plan_create reads $NTT_TUNE_FILE, else tune_cache.txt in the
 * library's directory, and takes the line for the current device, the kernels this library
 * was built from, N and the primes' width: the one with L and P = tune_polys if present, else
 * the one whose L*P is nearest.  No line (or no file) leaves the defaults; that is not an
 * error.  ntt_plan_tuned reports which happened.
 *
 * Debug modes.  When NTT_DEBUG is set at plan creation and holds "poison", the plan's column
 * and row passes fill their LDS with a poison pattern before use; with "reverse", their
 * workgroups take the tiles in reverse order.  Results must not change in either mode (no
 * exchange reads a slot it did not write; no tile depends on another).  Other paths ignore
 * NTT_DEBUG. */

/* Kernel paths for two-pass plans.  SPLIT launches the column pass and the row pass as
 * two kernels.  FUSED runs both in one persistent launch whose workgroups drain
 * per-XCD queues of tiles, so the pass-1 output of a limb is read back from that XCD's L2
 * (Section VI-C's two kernels, scheduled for gfx950's eight L2 slices); it needs every
 * prime below 2^60 and N1 x N2 one of 2^6 x 2^7, 2^7 x 2^7, 2^7 x 2^8, 2^8 x 2^8, 2^8 x 2^9.
 * AUTO takes SPLIT (measured faster on MI355X).  Launches of one FUSED plan share a small counter
 * block, so the library orders them across streams (a launch on another stream waits for
 * the previous one). */
enum { NTT_PATH_AUTO = 0, NTT_PATH_SPLIT = 1, NTT_PATH_FUSED = 2, NTT_PATH_RADIX2 = 3, NTT_PATH_REGISTER = 4 };

/* The two paths of the paper's ablation ladder (Section VI-A, VI-B; Table II), kept for
 * comparison with the split design: the data goes back to global memory after every group
 * of stages, and twiddles come from the table (no OT, no column/row split).
 *   RADIX2    one launch per stage of Algorithm 1, one butterfly per lane (log2 N launches);
 *   REGISTER  one launch per log2_radix consecutive stages, each lane holding the 2^log2_radix
 *             elements of one group of butterflies in registers (ceil(log2 N / log2_radix)
 *             launches; the last group may be shorter).
 * Both give the same results as every other path; ntt_forward_pass / ntt_inverse_pass run one
 * launch each (ntt_plan_num_passes of them). */

/* Create a plan for length-N transforms over L primes (Section III-B; Algorithm 1
 * REQUIRE: each q = 1 mod 2N).  `primes` is a host array of L distinct primes with
 * 2 < q < 2^62 and q = 1 (mod 2N).  The plan computes psi_l, the twiddle tables
 * Psi[i] = psi^{brv(i)} and Psi_inv[i] = psi^{-brv(i)} with their Shoup companions
 * floor(w * 2^64 / q) (Algorithm 4), N^{-1}, and the OT base tables, and uploads
 * them to the current HIP device.  On success *out holds the plan; on failure *out
 * is set to NULL.  Errors: NTT_ERR_ARG, NTT_ERR_N, NTT_ERR_PRIME, NTT_ERR_NOMEM,
 * NTT_ERR_HIP. */
ntt_status ntt_plan_create(ntt_plan_t* out, uint32_t N, const uint64_t* primes, uint32_t L,
                           const ntt_plan_opts* opts);

/* Drop the creator's reference to a plan.  A batch that names the plan holds a reference
 * of its own, so the plan stays usable by that batch (and only by it: every other call on
 * the handle returns NTT_ERR_ARG) until the last such batch is reassigned or destroyed.  The
 * call that drops the last reference frees the plan; the free first waits for all work queued
 * on the plan's device, so kernels already enqueued with the plan finish before its tables go.
 * NULL is accepted.  Errors: NTT_ERR_ARG when the plan was already destroyed and is still
 * held by a batch (a handle whose plan has been freed must not be passed at all). */
ntt_status ntt_plan_destroy(ntt_plan_t plan);

/* Copy the L roots psi_l in use into the host array psi_out (L entries). */
ntt_status ntt_plan_get_roots(ntt_plan_t plan, uint64_t* psi_out);

/* N, L, the pass split, twiddle mode, OT stages and kernel path (NTT_PATH_SPLIT, FUSED,
 * RADIX2 or REGISTER; single-pass plans report SPLIT) chosen by the plan.  Any pointer may be
 * NULL. */
ntt_status ntt_plan_get_info(ntt_plan_t plan, uint32_t* N, uint32_t* L, uint32_t* log2_n1,
                             int32_t* twiddle_mode, int32_t* ot_stages, int32_t* kernel_path);

/* The tile shape the plan was created with (r1, wg_size, col_width of ntt_plan_opts; 0 where
 * the built-in default applies: 8 values per lane, 128-lane row workgroups, and 64 columns
 * per column tile where N2 holds them, else 16).  Any pointer may be NULL. */
ntt_status ntt_plan_get_tiles(ntt_plan_t plan, int32_t* r1, int32_t* wg_size, int32_t* col_width);

/* In-place forward NTT of every vector of d_data ([n_polys][L][N] uint64, device).
 * Section III-A merged-twist transform computed as Algorithm 1 (Cooley-Tukey with the
 * butterfly of Algorithm 2 and Shoup's modmul of Algorithm 4) split into an LDS-staged
 * column pass and row pass (Section VI-C).  Output in bit-reversed order (natural order
 * for a NTT_ORDER_NATURAL plan). */
ntt_status ntt_forward(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, void* stream);

/* One kernel of the forward transform, for callers that schedule or time the passes
 * themselves (Section VI-C's Kernel-1 / Kernel-2).  pass 0 runs the column pass (the
 * first log2 N1 stages), pass 1 the row pass (the remaining stages, final reduction,
 * bit-reversed output).  A single-pass or fused plan has only pass 0.  A natural-order
 * plan adds the permutation as the last pass.  Running every pass in order equals
 * ntt_forward.  Errors: NTT_ERR_ARG for a pass index at or above ntt_plan_num_passes. */
ntt_status ntt_forward_pass(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, uint32_t pass, void* stream);

/* One kernel of the inverse transform: pass 0 runs the row pass (the first
 * Gentleman-Sande stages), pass 1 the column pass (the last stages with the 1/N scale).
 * A single-pass or fused plan has only pass 0.  A natural-order plan adds the permutation
 * as the first pass (the others move up by one).  Running every pass in order equals
 * ntt_inverse. */
ntt_status ntt_inverse_pass(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, uint32_t pass, void* stream);

/* Number of kernels per transform for this plan: 1 (single pass or fused) or 2, plus one
 * for the permutation of a natural-order plan; 0 for a NULL or destroyed plan. */
uint32_t ntt_plan_num_passes(ntt_plan_t plan);

/* The plan's NTT-domain slot order (NTT_ORDER_*), -1 for a NULL or destroyed plan. */
int32_t ntt_plan_order(ntt_plan_t plan);

/* Stages per launch of a RADIX2 (1) or REGISTER plan, 0 for the other paths, -1 for a NULL
 * or destroyed plan. */
int32_t ntt_plan_log2_radix(ntt_plan_t plan);

/* 1 when the plan's options came from the tuner's file (use_autotune found a line), 0 when
 * not, -1 for a NULL or destroyed plan. */
int32_t ntt_plan_tuned(ntt_plan_t plan);

/* In-place inverse: takes NTT-domain vectors in the plan's order (bit-reversed unless the
 * plan is NTT_ORDER_NATURAL) and returns natural-order coefficients, with the Psi^{-1}
 * twist and the 1/N scale merged in (Section III-A). */
ntt_status ntt_inverse(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, void* stream);

/* Element-wise product in the NTT domain (Section III-A, the Hadamard product):
 * d_c[k] = d_a[k] * d_b[k] mod q_l for every element of the [n_polys][L][N] batch.
 * d_c may alias d_a or d_b. */
ntt_status ntt_pointwise_mul(ntt_plan_t plan, const uint64_t* d_a, const uint64_t* d_b, uint64_t* d_c,
                             uint32_t n_polys, void* stream);

/* Negacyclic product in Z_q[X]/(X^N+1) per vector (Section III-A):
 * c = iNTT(NTT(a) * NTT(b)).  Inputs and output are natural-order coefficients;
 * d_a and d_b are left unchanged; d_c may alias d_a but not d_b.  NTT(b) goes to a
 * plan-owned scratch buffer of n_polys*L*N*8 bytes, one per stream, grown on demand (the
 * growth waits for the stream's previous product). */
ntt_status ntt_polymul_negacyclic(ntt_plan_t plan, const uint64_t* d_a, const uint64_t* d_b, uint64_t* d_c,
                                  uint32_t n_polys, void* stream);

/* The same product for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, hosts that forbid hipMalloc): identical arguments, result
 * and launches as ntt_polymul_negacyclic, but NTT(b) goes to one fixed 64 MiB device array
 * that the library holds on every device it runs on until the process ends, so the call
 * allocates nothing.  n_polys*L*N must not exceed ntt_polymul_noalloc_max_words() (2^23
 * residues), else NTT_ERR_ARG and nothing is enqueued; larger batches go in several calls.
 * Every call on one device shares that array: calls whose work overlaps on the device
 * (different streams, or different host threads without ordering) race and give wrong
 * results.  Calls on one stream are ordered and safe.  The array is fully written before it
 * is read, so no call depends on what an earlier one left there. */
ntt_status ntt_polymul_negacyclic_noalloc(ntt_plan_t plan, const uint64_t* d_a, const uint64_t* d_b, uint64_t* d_c,
                                          uint32_t n_polys, void* stream);
uint64_t ntt_polymul_noalloc_max_words(void);

/* ---------------------------------------------------------------- batches of uneven jobs
 *
 * Many polynomials of different N and limb counts (Section VI-A's batching, taken to
 * uneven sizes).  A job names a plan and a device array [n_polys][n_limbs][N] whose limb l
 * is reduced mod the plan's prime l: n_limbs may be any prefix 1..L of the plan's primes,
 * so one plan over a long prime chain serves every limb count.  A batch object validates
 * the jobs once and uploads per-vector descriptors; runs then enqueue the work:
 *
 *   NTT_BATCH_PLAIN    one call per step of each job (the baseline);
 *   NTT_BATCH_GROUPED  one launch per pass over every vector of every job sharing a plan
 *                      (vector-list launches: all forward work, then all key products, then
 *                      all inverse work);
 *   NTT_BATCH_GRAPH    the GROUPED launches captured once into a hipGraph (on a stream the
 *                      batch owns) and replayed on the caller's stream on every run;
 *   NTT_BATCH_GRAPH_BRANCHED  the same launches captured as up to four independent
 *                      branches of one graph (each plan's forward, key-product and inverse
 *                      launches in one branch, plans balanced over the branches by work),
 *                      so that on the device the launches of different sizes overlap.
 *
 * op is a set of steps run in the order forward, key product, inverse: NTT_OP_MULKEY
 * multiplies every polynomial of the job element-wise by the job's key, a device array
 * [n_limbs][N] already in the NTT domain, in the plan's slot order (the
 * ciphertext-times-plaintext step of Section III-A's polynomial product).  Results
 * are bit-identical across the three modes.  A batch holds a reference on each plan its
 * jobs name (see ntt_plan_destroy), so a plan may be destroyed before the batch; the data
 * arrays must stay valid and may not overlap between jobs. */
enum { NTT_OP_FORWARD = 1, NTT_OP_INVERSE = 2, NTT_OP_FORWARD_INVERSE = 3, NTT_OP_MULKEY = 4 };
enum { NTT_BATCH_PLAIN = 0, NTT_BATCH_GROUPED = 1, NTT_BATCH_GRAPH = 2, NTT_BATCH_GRAPH_BRANCHED = 3 };

typedef struct {
    ntt_plan_t plan;
    uint64_t* d_data;     /* [n_polys][n_limbs][N] uint64, device, 16-byte aligned    */
    uint32_t n_polys;     /* >= 1                                                     */
    uint32_t n_limbs;     /* 1..L: the plan's first n_limbs primes; 0 = all L          */
    uint32_t op;          /* NTT_OP_* bits (nonzero)                                   */
    uint32_t reserved;    /* must be zero                                             */
    const uint64_t* d_key;/* [n_limbs][N] key in the NTT domain when op has MULKEY      */
} ntt_job;

typedef struct ntt_batch_s* ntt_batch_t;

/* Validate `n_jobs` jobs (copied; the array may be freed afterwards) and upload their
 * vector descriptors to the device of the first job's plan.  Errors: NTT_ERR_ARG for a
 * null plan or buffer, a bad op, n_limbs above L, mixed devices; NTT_ERR_NOMEM; NTT_ERR_HIP. */
ntt_status ntt_batch_create(ntt_batch_t* out, const ntt_job* jobs, uint32_t n_jobs);

/* Replace the jobs of an existing batch (same rules as ntt_batch_create; the plans must
 * live on the batch's device).  The descriptors go through the batch's pinned staging
 * buffer and are copied asynchronously on `stream`, which first waits for the batch's last
 * run, into the batch's device storage; that storage grows only when the new job set needs
 * more (growth blocks the host until the earlier work is done).  A captured graph is
 * dropped and re-captured by the next NTT_BATCH_GRAPH run.  Runs of the batch must then be
 * enqueued on `stream` (or ordered after it).  Meant for request loops that reuse a few
 * batch objects instead of creating one per iteration.  On error the batch is left with
 * no jobs (its runs enqueue nothing) until the next successful assign. */
ntt_status ntt_batch_assign(ntt_batch_t batch, const ntt_job* jobs, uint32_t n_jobs, void* stream);

/* Enqueue one run of the batch on `stream` in the given NTT_BATCH_* mode. */
ntt_status ntt_batch_run(ntt_batch_t batch, int32_t mode, void* stream);

/* Release the batch (its descriptors, private stream and captured graph).  The caller
 * must make sure no run is still in flight.  NULL is accepted. */
ntt_status ntt_batch_destroy(ntt_batch_t batch);

/* ---------------------------------------------------------------- 32-bit words
 *
 * The word-size choice of Section IV taken the other way: a plan created with word_bits = 32
 * holds residues in uint32_t words, for primes below 2^30 (four times a prime fits a word,
 * so the lazy butterfly ranges hold), and Shoup products of one high and two low 32x32
 * multiplies.  The same modulus budget takes twice the limbs of 64-bit words.  Such a plan
 * takes table twiddles, the split (or single-pass) kernels and bit-reversed order; other
 * options return NTT_ERR_UNSUPPORTED and primes at or above 2^30 NTT_ERR_PRIME.  Its data
 * goes through the _u32 calls below ([n_polys][L][N] uint32_t, device, 16-byte aligned),
 * with the same meaning, order, streams and errors as their 64-bit counterparts; the other
 * data calls and batches refuse a 32-bit plan (NTT_ERR_ARG / NTT_ERR_UNSUPPORTED), and the
 * _u32 calls refuse a 64-bit one. */
ntt_status ntt_forward_u32(ntt_plan_t plan, uint32_t* d_data, uint32_t n_polys, void* stream);
ntt_status ntt_inverse_u32(ntt_plan_t plan, uint32_t* d_data, uint32_t n_polys, void* stream);
ntt_status ntt_pointwise_mul_u32(ntt_plan_t plan, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_c,
                                 uint32_t n_polys, void* stream);
ntt_status ntt_polymul_negacyclic_u32(ntt_plan_t plan, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_c,
                                      uint32_t n_polys, void* stream);

/* 32 or 64: the plan's residue word; -1 for a NULL or destroyed plan. */
int32_t ntt_plan_word_bits(ntt_plan_t plan);

/* ---------------------------------------------------------------- RNS <-> integers
 *
 * The conversions on either side of the transform (Section III-B): a coefficient of
 * Z_Q[X]/(X^N+1), Q = q_0 q_1 ... q_{L-1} (the plan's primes), is held in RNS form as its L
 * residues.  Integers are arrays of little-endian 64-bit words stored word-major:
 * [n_polys][W][N] uint64_t, word w of coefficient c of polynomial p at (p*W + w)*N + c.
 * The first call that needs them builds the conversion tables (Q / q_l, their inverses mod
 * q_l, 2^(64 w) mod q_l, the multiples of Q) and uploads them to the plan's device (a device
 * allocation).  64-bit plans only. */

/* Words of Q: the width W of a reconstructed integer.  0 for a NULL, destroyed or 32-bit plan
 * or when the tables cannot be built. */
uint32_t ntt_crt_words(ntt_plan_t plan);

/* d_res [n_polys][L][N] = the residues of the n_words-word integers in d_words (any values
 * below 2^(64 n_words), 1 <= n_words <= 64) modulo each prime, canonical. */
ntt_status ntt_rns_decompose(ntt_plan_t plan, const uint64_t* d_words, uint32_t n_words, uint64_t* d_res,
                             uint32_t n_polys, void* stream);

/* d_words [n_polys][W][N], W = ntt_crt_words(plan): the unique integer in [0, Q) with the
 * canonical residues d_res [n_polys][L][N] (Chinese remainder theorem).  L <= 64
 * (NTT_ERR_UNSUPPORTED above); d_words must not alias d_res. */
ntt_status ntt_crt_reconstruct(ntt_plan_t plan, const uint64_t* d_res, uint64_t* d_words, uint32_t n_polys,
                               void* stream);

/* ---------------------------------------------------------------- measurement yardstick
 *
 * Not part of the transform: a plain device-to-device copy of `bytes` bytes on the current
 * device, one 16-byte vector per lane in a single pass, which measurements use as the memory
 * rate a kernel on this GPU can reach to compare the passes with.  `bytes` must be a multiple
 * of 16 and below 2^35; both pointers 16-byte aligned device addresses of caller-owned,
 * non-overlapping buffers.  Enqueued on `stream`; NTT_ERR_ARG for null or misaligned pointers
 * and bad sizes (0 bytes is a no-op), NTT_ERR_HIP for a launch failure. */
ntt_status ntt_device_copy(void* d_dst, const void* d_src, size_t bytes, void* stream);

/* Human-readable name of a status code (static storage). */
const char* ntt_status_string(ntt_status s);

/* Message of the last failure on the calling thread (static per-thread storage). */
const char* ntt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NTT_MI355X_H */
