/*
 * slrng — bulk generation from the scrambled linear pseudorandom number
 * generators of D. Blackman and S. Vigna, "Scrambled Linear Pseudorandom
 * Number Generators" (ACM TOMS), on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  No C++ exceptions cross it.  Every function returns SLRNG_OK (0) on
 * success or a negative SLRNG_E* code; slrng_strerror() names the code and
 * slrng_last_hip_error() returns the HIP error behind SLRNG_EHIP (per thread).
 *
 * Conventions
 *  - A generator is a linear engine (Section "Linear engines": xoroshiro128,
 *    xoshiro256, xoshiro512, xoroshiro1024) combined with a scrambler
 *    (Section "Scramblers": +, ++, *, **), with the parameters of tables
 *    tab:par64 and tab:scr64 and the state words named in the code figures
 *    fig:xoroshiro128, fig:xoroshiro1024, fig:xoshiro256 and fig:xoshiro512.
 *  - A state is k 64-bit words (k = 2, 4, 8, 16) in logical order: the row
 *    vector that the transition matrix (X_kw of equation eq:M, S_4w, S_8w)
 *    multiplies from the right.  For xoroshiro128, xoshiro256 and xoshiro512
 *    this is the array s[] of the figures; for xoroshiro1024 logical word j is
 *    s[(p + 1 + j) & 15] of fig:xoroshiro1024.
 *  - Output t of a stream is the scrambler applied to the state after t steps
 *    (the figures compute the output before advancing the state).
 *  - Doubles are the upper 53 bits: (x >> 11) * 2^-53, exactly (Section
 *    "Choosing a generator").
 *  - Seeding: the state is filled with consecutive outputs of SplitMix64
 *    seeded with the 64-bit seed (Section "Choosing a generator").
 *  - 32-bit generators (ids 14 .. 18): states are k = 2 or 4 32-bit words,
 *    exchanged through the same uint64 host arrays (one word per element,
 *    upper half zero; set_state rejects larger values with SLRNG_EINVAL).
 *    Seeding fills the state array with the SplitMix64 output stream, each
 *    64-bit output giving two words, low half first (the paper only says a
 *    32-bit SplitMix is immediate to define).  Their outputs are 32-bit
 *    (SLRNG_U32, SLRNG_F32).  Batches and the server take the 64-bit
 *    generators only.
 *  - Jumps (Section "Combining linear engines and scramblers": every generator
 *    has jump functions): SLRNG_JUMP advances by 2^(n/2) steps and
 *    SLRNG_LONG_JUMP by 2^(3n/4) steps, n = 64k the state size in bits.
 *  - Functions taking a hipStream_t are asynchronous and ordered on that
 *    stream (0 = the null stream); the caller orders calls on one handle.
 *  - Device buffers are caller-owned unless stated; handles own their state
 *    memory.  Handles are not thread-safe.  Large outputs write fastest into
 *    memory from slrng_output_alloc (physical pages spread over the HBM).
 */
#ifndef SLRNG_H
#define SLRNG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SLRNG_ABI_VERSION 1

typedef enum slrng_variant {
  SLRNG_XOROSHIRO128_PLUS = 0,       /* fig:xoroshiro128, s0 + s1 */
  SLRNG_XOROSHIRO128_PLUSPLUS = 1,   /* rotl(s0 + s1, 17) + s0, engine 49/21/28 */
  SLRNG_XOROSHIRO128_STARSTAR = 2,   /* rotl(s0 * 5, 7) * 9 */
  SLRNG_XOSHIRO256_PLUS = 3,         /* fig:xoshiro256, s0 + s3 */
  SLRNG_XOSHIRO256_PLUSPLUS = 4,     /* rotl(s0 + s3, 23) + s0 */
  SLRNG_XOSHIRO256_STARSTAR = 5,     /* rotl(s1 * 5, 7) * 9 */
  SLRNG_XOSHIRO512_PLUS = 6,         /* fig:xoshiro512, s0 + s2 */
  SLRNG_XOSHIRO512_PLUSPLUS = 7,     /* rotl(s0 + s2, 17) + s2 */
  SLRNG_XOSHIRO512_STARSTAR = 8,     /* rotl(s1 * 5, 7) * 9 */
  SLRNG_XOROSHIRO1024_PLUS = 9,      /* fig:xoroshiro1024, s0 + s15 */
  SLRNG_XOROSHIRO1024_PLUSPLUS = 10, /* rotl(s0 + s15, 23) + s15 */
  SLRNG_XOROSHIRO1024_STARSTAR = 11, /* rotl(s0 * 5, 7) * 9 */
  SLRNG_XOROSHIRO128_STAR = 12,      /* s0 * 0x9e3779b97f4a7c13 */
  SLRNG_XOROSHIRO1024_STAR = 13,     /* s0 * 0x9e3779b97f4a7c13 */
  SLRNG_NUM_VARIANTS = 14,           /* the 64-bit generators are ids 0 .. 13 */
  /* 32-bit generators (Section "The 32-bit case", tables tab:par32 and
   * tab:scr32; words read as in fig:xoroshiro128 and fig:xoshiro256) */
  SLRNG_XOROSHIRO64_STAR = 14,       /* s0 * 0x9E3779BB, engine 26/9/13 */
  SLRNG_XOROSHIRO64_STARSTAR = 15,   /* rotl(s0 * 0x9E3779BB, 5) * 5 */
  SLRNG_XOSHIRO128_PLUS = 16,        /* s0 + s3, engine 9/11 */
  SLRNG_XOSHIRO128_PLUSPLUS = 17,    /* rotl(s0 + s3, 7) + s0 */
  SLRNG_XOSHIRO128_STARSTAR = 18,    /* rotl(s1 * 5, 7) * 9 */
  SLRNG_NUM_VARIANTS_ALL = 19
} slrng_variant;

typedef enum slrng_kind {
  SLRNG_U64 = 0, /* uint64 outputs (64-bit generators) */
  SLRNG_F64 = 1, /* doubles in [0, 1) from the upper 53 bits (64-bit generators) */
  SLRNG_U32 = 2, /* uint32 outputs (32-bit generators) */
  SLRNG_F32 = 3  /* floats in [0, 1) from the upper 24 bits, (x >> 8) * 2^-24,
                    exact (32-bit generators) */
} slrng_kind;

typedef enum slrng_jump_kind {
  SLRNG_JUMP = 0,     /* 2^(n/2) steps */
  SLRNG_LONG_JUMP = 1 /* 2^(3n/4) steps */
} slrng_jump_kind;

enum {
  SLRNG_OK = 0,
  SLRNG_EINVAL = -1,     /* bad argument (null pointer, unknown enum, ld < n) */
  SLRNG_ERANGE = -2,     /* a size overflows 64 bits or exceeds a limit */
  SLRNG_ENOMEM = -3,     /* device or host allocation failed */
  SLRNG_EZEROSTATE = -4, /* an all-zero state (a fixed point of every engine) */
  SLRNG_EAGAIN = -5,     /* resource temporarily unavailable (server budget) */
  SLRNG_EHIP = -6,       /* a HIP call failed; see slrng_last_hip_error() */
  SLRNG_ENOTIMPL = -7    /* not implemented */
};

typedef struct slrng_streams slrng_streams; /* opaque: S device-resident states */

/* Library version (SLRNG_ABI_VERSION). */
int slrng_version(void);

/* Error name of a return code; never NULL. */
const char *slrng_strerror(int err);

/* HIP error code of the last SLRNG_EHIP returned on this thread. */
int slrng_last_hip_error(void);

/* Words of state k (2, 4, 8 or 16) of a variant, or SLRNG_EINVAL. */
int slrng_state_words(int variant);

/* ---------------------------------------------------------------- host-side
 * polynomial tools (no GPU needed).  Polynomials over Z/2Z are arrays of
 * little-endian 64-bit words: bit i of word i/64 is the coefficient of x^i.
 *
 * slrng_charpoly: the characteristic polynomial p(x) = det(M - xI) of the
 * variant's engine (Section "Polynomials and full period"), degree n = 64k,
 * written to out[0 .. n/64] (n/64 + 1 words).  The library derives it with
 * Berlekamp-Massey on 2n values of one state bit.
 *
 * slrng_jump_poly: r(x) = x^J mod p(x) for J = sum_i J_words[i] 2^(64 i),
 * i < nj, written to out[0 .. n/64) (n/64 words).  By Cayley-Hamilton,
 * state * M^J = sum_i r_i (state * M^i): the jump of J steps. */
int slrng_charpoly(int variant, uint64_t *out, int out_words);
int slrng_jump_poly(int variant, const uint64_t *J_words, int nj, uint64_t *out, int out_words);

/* slrng_jump_poly_device: the same polynomials for many distances at once,
 * computed on the device.  dev_J (device memory, m x 2 words) holds the
 * 128-bit distances J_j = dev_J[2j] + 2^64 dev_J[2j+1]; word w of
 * x^(J_j) mod p(x) is written to dev_out[j n/64 + w] (device memory, m x n/64
 * words).  Each result is the product in Z/2Z[x]/p of the entries
 * x^(d 2^(10 l)) mod p selected by J_j's radix-1024 digits d (level l); those
 * tables are themselves computed on the device from p(x) alone, by repeated
 * squaring and multiplication, the first time an engine is used on a device
 * (jump functions, Section "Combining linear engines and scramblers").
 * Asynchronous on `stream`.  EINVAL for a bad variant or a null or unaligned
 * pointer, ERANGE for m > 2^32; m = 0 does nothing. */
int slrng_jump_poly_device(int variant, const uint64_t *dev_J, uint64_t m, uint64_t *dev_out,
                           hipStream_t stream);

/* ---------------------------------------------------------------- streams
 *
 * slrng_streams_create: S = n_streams streams on the current device.  The
 * base state is the SplitMix64 fill of `seed` and stream i is the base
 * jumped i times by SLRNG_JUMP, i.e. state_i = base * M^(i 2^(n/2)).
 * n_streams in [1, 2^31] (ERANGE otherwise).  The handle owns 2 S k words of
 * device memory.  EZEROSTATE if the seed gives the all-zero state (possible
 * only for xoroshiro64, whose state is a single SplitMix64 output).
 *
 * slrng_streams_create_from_states: S streams with the given logical-order
 * states, host_words[i*k + j] = word j of stream i.  EZEROSTATE if a state is
 * all zero.  Synchronous upload.
 *
 * slrng_streams_seed: re-seeds an existing handle in place, exactly as
 * slrng_streams_create would position it (no allocation; asynchronous).
 *
 * slrng_streams_count / slrng_streams_variant: S and the variant.
 *
 * slrng_streams_jump / slrng_streams_advance: every stream advances by the
 * jump (SLRNG_JUMP or SLRNG_LONG_JUMP) or by steps_hi 2^64 + steps_lo steps.
 *
 * slrng_generate: for every stream i, out[i*ld + t] = output t, t < n; the
 * stream then stands n steps further (generate(a); generate(b) produces the
 * same values as generate(a + b)).  dev_out: device memory aligned to the
 * element (8 bytes for SLRNG_U64 / SLRNG_F64, 4 for SLRNG_U32 / SLRNG_F32),
 * at least (S-1) ld + n elements; ld >= n (EINVAL otherwise), overflow of the
 * extent is ERANGE.  n = 0 is a successful no-op.  kind must match the
 * generator's word size (EINVAL otherwise); all kinds are bit-exact.
 *
 * slrng_get_state / slrng_set_state: copy the S x k logical-order states to or
 * from host memory (host_words[i*k + j]); synchronous on `stream`.  set_state
 * rejects an all-zero state with EZEROSTATE and leaves the handle unchanged.
 *
 * slrng_streams_advance_each: stream i advances by its own distance
 * J_i = dev_steps[2i] + 2^64 dev_steps[2i+1] (any 128-bit value; the jump
 * functions of Section "Combining linear engines and scramblers" with
 * per-stream distances).  Everything runs on the device: J_i is cut into 13
 * radix-1024 digits d_l and the stream is jumped by x^(d_l 2^(10 l)) mod p(x)
 * for each nonzero digit, from a per-engine table of those polynomials built
 * once per device (13 x 1024 entries of n bits; built on the first call).
 * dev_steps: device memory, 8-byte aligned, 2 S words, read by work queued on
 * `stream` (keep it alive until that work is done).  Asynchronous.
 * EINVAL for a null or misaligned dev_steps.
 *
 * slrng_streams_destroy: frees the handle (after the device is idle). */
int slrng_streams_create(int variant, uint64_t seed, uint64_t n_streams, hipStream_t stream,
                         slrng_streams **out);
int slrng_streams_create_from_states(int variant, const uint64_t *host_words, uint64_t n_streams,
                                     hipStream_t stream, slrng_streams **out);
int slrng_streams_seed(slrng_streams *h, uint64_t seed, hipStream_t stream);
int slrng_streams_count(const slrng_streams *h, uint64_t *n_streams);
int slrng_streams_variant(const slrng_streams *h, int *variant);
int slrng_streams_jump(slrng_streams *h, int jump_kind, hipStream_t stream);
int slrng_streams_advance(slrng_streams *h, uint64_t steps_hi, uint64_t steps_lo,
                          hipStream_t stream);
int slrng_streams_advance_each(slrng_streams *h, const uint64_t *dev_steps, hipStream_t stream);

/* slrng_linear_complexity: an on-device linearity check.  For every stream
 * i, dev_lc[i] = the linear complexity of bit `bit` of its next nbits outputs
 * (the integer outputs, before any conversion), computed with the
 * Berlekamp-Massey algorithm as in Section "A theoretical analysis of
 * scramblers" (e.g. bit 0 of the + and * scramblers has the engine's
 * complexity n, table tab:plusdeg; the result is the true complexity when
 * nbits >= 2 x complexity).  The streams are not advanced.  bit < 64 (< 32
 * for the 32-bit generators), nbits a multiple of 32 in [32, 2560]; dev_lc:
 * device memory, 4-byte aligned, S uint32.  Asynchronous.  EINVAL otherwise. */
int slrng_linear_complexity(const slrng_streams *h, int bit, uint32_t nbits, uint32_t *dev_lc,
                            hipStream_t stream);

/* slrng_equidistribution_rank: the test of Section "Equidistribution" for
 * one word of a linear engine, on the device.  For the engine of `variant`
 * (the scrambler plays no part; n = k w state bits), *dev_rank = the rank
 * over Z/2Z of the n x (dims w) matrix whose row i holds word `word` of
 * e_i M^0, e_i M^1, ..., e_i M^(dims-1), with e_i the state whose only set
 * bit is bit i (logical word order; the columns of M^t that belong to that
 * word, juxtaposed).  With dims = k the word is equidistributed in the
 * maximum dimension exactly when the rank is n (the matrix is invertible);
 * for dims < k, d-dimensionally equidistributed exactly when it is dims w.
 * word in [0, k), dims in [1, k]; dev_rank: device memory, 4-byte aligned,
 * one uint32.  One workgroup; asynchronous.  EINVAL otherwise.
 *
 * slrng_gf2_rank: the Gaussian elimination over Z/2Z behind it, on a
 * caller's matrix: nrows and ncols in [1, 1024]; dev_rows: device memory,
 * 8-byte aligned, row r in words r * ceil(ncols/64) .. + ceil(ncols/64) - 1,
 * bit b of word q = column 64 q + b (bits past ncols are ignored);
 * *dev_rank = the rank.  Asynchronous.  EINVAL otherwise. */
int slrng_equidistribution_rank(int variant, int word, int dims, uint32_t *dev_rank,
                                hipStream_t stream);
int slrng_gf2_rank(const uint64_t *dev_rows, uint32_t nrows, uint32_t ncols, uint32_t *dev_rank,
                   hipStream_t stream);
int slrng_generate(slrng_streams *h, int kind, uint64_t n, void *dev_out, uint64_t ld,
                   hipStream_t stream);
int slrng_get_state(const slrng_streams *h, uint64_t *host_words, hipStream_t stream);
int slrng_set_state(slrng_streams *h, const uint64_t *host_words, hipStream_t stream);
int slrng_streams_destroy(slrng_streams *h);

/* ---------------------------------------------------------------- output memory
 *
 * slrng_output_alloc: device memory for large outputs on the current device,
 * virtually contiguous, with its physical backing spread over the HBM.  Not
 * an operation of the generators: on MI355X the store bandwidth one buffer
 * sees depends on how widely its physical pages are spread, and a large
 * allocation that lands in one compact physical range caps streams of stores
 * near 5.5 TB/s where the same bytes spread over about four times the span
 * reach 6.5-6.9 TB/s.  From 1 GiB up the buffer is made of physical pieces of
 * P = 256 MiB .. 1 GiB (a power of two near bytes / 64): gap x M pieces are
 * created in order, every gap-th is kept and the others are returned at once
 * (gap = 16, lower when free memory is short: gap x M x P bytes are held
 * only during the call, so a 32 GiB buffer gets about 8 on an empty device);
 * the kept pieces are mapped into one virtual range aligned
 * to P in bit-reversed order of their creation, so that any contiguous part
 * of the buffer is spread over the whole span too (a few GB written into the
 * start of a buffer measured 6.1-6.5 TB/s this way, 5.3-5.5 in creation
 * order).  Below 1 GiB, and on a device without the HIP virtual memory API
 * or when the pieces cannot be mapped, it is a plain device allocation
 * (256-byte aligned); placement changes speed only, never values.
 * The memory is uninitialised and usable like any device pointer (kernels,
 * copies) on that device.  Synchronous.  EINVAL for bytes = 0 or a null
 * dev_ptr, ENOMEM if the device cannot supply it, EHIP for other HIP errors.
 * Thread-safe.
 *
 * slrng_output_free: frees memory from slrng_output_alloc.  It waits for the
 * device to be idle first (unmapping memory that queued work still writes
 * would fault).  NULL is a no-op; EINVAL for a pointer that
 * slrng_output_alloc did not return (or already freed).  Thread-safe. */
int slrng_output_alloc(uint64_t bytes, void **dev_ptr);
int slrng_output_free(void *dev_ptr);

/* ---------------------------------------------------------------- tuning
 *
 * Launch shape of slrng_generate per (variant, kind):
 *  tile          outputs per lane staged through LDS per round (16 or 32);
 *  target_waves  streams are split into chunks (each chunk starts from the
 *                stream jumped by a multiple of the chunk length) until about
 *                this many waves run, at most 16 chunks per stream;
 *  skew          1, 2, 4, 8 or 16 classes of staggered chunk boundaries
 *                (groups of 64 streams in different classes start their
 *                chunks at different offsets, which spreads concurrent stores
 *                over the memory channels when the row stride is a power of
 *                two); 1 = no stagger; applied only to chunks of at least
 *                8 x tile x skew outputs;
 *  min_chunk     no chunk shorter than this many outputs;
 *  store         0: plain (write-back) output stores; 1: nontemporal ones
 *                (on the 16-byte aligned path; for the 64-bit generators
 *                only when n >= 2048, shorter rows measuring faster with
 *                plain stores).  Which is faster depends on
 *                the physical placement of the output (compact memory:
 *                plain; slrng_output_alloc memory: nontemporal, as measured
 *                on MI355X).
 * The launch shape never changes the values produced.  Values outside the
 * accepted range give EINVAL. */
typedef struct slrng_tuning {
  int32_t tile;
  int32_t target_waves;
  int32_t skew;
  int32_t store;    /* output stores: 0 plain (write-back), 1 nontemporal */
  uint64_t min_chunk;
} slrng_tuning;

int slrng_get_tuning(int variant, int kind, slrng_tuning *out);
int slrng_set_tuning(int variant, int kind, const slrng_tuning *t);

/* ---------------------------------------------------------------- batches
 *
 * Many independent requests of uneven lengths and mixed generators in one
 * launch.  Request r asks for n outputs of generator `variant`, as `kind`,
 * starting `start` steps after the origin state (the SplitMix64 fill of
 * `seed`, as in slrng_streams_create): dev_out[t] = output (start + t) of
 * that stream, t < n.  dev_out: device memory, 8-byte aligned, n elements.
 * Requests are independent (they may overlap in stream and position, not in
 * output memory).  Every request's values are the same in any batch, alone or
 * in any mix, in every mode.
 *
 * slrng_batch_plan: plans a batch once (host descriptors, device descriptor
 * upload; with SLRNG_BATCH_GRAPH also captures and instantiates a hipGraph).
 * The request array is not kept.  Start states of requests with start > 0
 * are computed on the device from the digits of start (the engine's digit
 * matrices M^(d 2^(b l)), built on the device the first time the engine is
 * used in a batch or a server: 32 MiB for xoshiro256, 64 MiB for
 * xoroshiro1024); no polynomial is computed per request.
 * slrng_batch_launch: enqueues the planned work on `stream` (asynchronous;
 * replays the graph in SLRNG_BATCH_GRAPH mode).  Launches of one batch must
 * not overlap in time (they share a claim counter).
 * slrng_batch_run: plan + launch + synchronize + destroy.
 * slrng_batch_info: tiles, lane-chunks and outputs of a plan.
 * slrng_batch_latencies: a measurement aid.  Launches the planned batch once
 * with timing events (without the graph), waits for it, and writes for every
 * request the time in ms from the start of the launch until that request's
 * outputs were complete: one value for all requests in the batched modes,
 * each request's own launch end in the plain form (0 for empty requests).
 * done_ms has one entry per planned request.  Synchronous.
 * Errors: EINVAL for a bad variant, kind, mode, tile, null or misaligned
 * output; ERANGE for more than 2^24 requests or a request too long to chunk.
 *
 * Options (slrng_batch_default_opts fills the defaults):
 *  mode          SLRNG_BATCH_GRAPH: one persistent kernel over all tiles,
 *                captured into a hipGraph at plan time;
 *                SLRNG_BATCH_PERSISTENT: the same kernel launched directly;
 *                SLRNG_BATCH_PLAIN: one launch of the same kernel per request
 *                (the unbatched comparison form).
 *  tile          outputs per lane staged through LDS per round (16 or 32);
 *  waves_per_cu  persistent grid size (0 = default);
 *  chunk[v]      lane-chunk length for variant v (0 = default): a request is
 *                cut into chunks of this many outputs, each on one lane,
 *                started by a jump of j*chunk steps. */
typedef struct slrng_request {
  int32_t variant;
  int32_t kind;
  uint64_t seed;
  uint64_t start;
  uint64_t n;
  void *dev_out;
} slrng_request;

enum { SLRNG_BATCH_GRAPH = 0, SLRNG_BATCH_PERSISTENT = 1, SLRNG_BATCH_PLAIN = 2 };

typedef struct slrng_batch_opts {
  int32_t mode;
  int32_t tile;
  int32_t waves_per_cu;
  int32_t reserved;
  uint64_t chunk[SLRNG_NUM_VARIANTS];
} slrng_batch_opts;

typedef struct slrng_batch slrng_batch; /* opaque planned batch */

int slrng_batch_default_opts(slrng_batch_opts *opts);
int slrng_batch_plan(const slrng_request *reqs, size_t n_reqs, const slrng_batch_opts *opts,
                     slrng_batch **out);
int slrng_batch_launch(slrng_batch *b, hipStream_t stream);
int slrng_batch_info(const slrng_batch *b, uint64_t *n_tiles, uint64_t *n_lanes,
                     uint64_t *total_outputs);
int slrng_batch_latencies(slrng_batch *b, hipStream_t stream, double *done_ms);
int slrng_batch_destroy(slrng_batch *b);
int slrng_batch_run(const slrng_request *reqs, size_t n_reqs, const slrng_batch_opts *opts,
                    hipStream_t stream);

/* slrng_batch_run_static: slrng_batch_run for callers that cannot allocate
 * device memory (code that must not call hipMalloc, tight serving loops).
 * Same requests, options, values and errors as slrng_batch_run, with these
 * differences:
 *  - it calls no hipMalloc, hipFree or other allocating routine: the
 *    descriptors, claim counters, request start states and chunk tables go
 *    into a fixed device array of SLRNG_BATCH_STATIC_SCRATCH_BYTES (32 MiB)
 *    that the library holds on every device it runs on until the process
 *    ends (its device address is taken once per device, on the first call);
 *  - it runs the persistent form only: SLRNG_BATCH_GRAPH runs as
 *    SLRNG_BATCH_PERSISTENT (instantiating a graph allocates), and
 *    SLRNG_BATCH_PLAIN is EINVAL;
 *  - SLRNG_ERANGE when the plan needs more than the array holds (about
 *    32 bytes per 64-output lane-chunk plus 16 per tile, 128 per request that
 *    starts past its origin, and the chunk tables: n/8 bytes per chunk of the
 *    longest request of each generator);
 *  - every call on one device shares that device's array, which keeps the
 *    last call's contents.  Calls are synchronous (the work is finished when
 *    the call returns) and calls from several host threads on one device are
 *    serialised inside the library; the array is not meant to be touched by
 *    anything else.
 * The caller still provides the output buffers (request dev_out). */
#define SLRNG_BATCH_STATIC_SCRATCH_BYTES (32u << 20)
int slrng_batch_run_static(const slrng_request *reqs, size_t n_reqs, const slrng_batch_opts *opts,
                           hipStream_t stream);

/* ---------------------------------------------------------------- serving
 *
 * A request server with continuous batching over device-resident streams.
 * Stream j (j < n_streams) is positioned as by slrng_streams_create(variant,
 * seed, n_streams): the SplitMix64 base jumped j times.  Every request takes
 * the next positions of its stream in admission order, so request r on stream
 * j receives outputs pos_r .. pos_r + n_r - 1 of that stream, where pos_r is
 * the stream's head when r was admitted: the total length of the earlier
 * requests on j plus any slrng_server_advance of j (positions are 128-bit,
 * modulo 2^128).  Its values do not depend on what else is in flight (the
 * same request alone gives the same values).  The start state s_j M^pos_r is
 * computed on the device from the digits of pos_r (jump functions, Section
 * "Combining linear engines and scramblers"), with matrices M^(d 2^(b l))
 * built once per device and engine when the first server of that engine is
 * created (32 MiB for xoshiro256, 64 MiB for xoroshiro1024); no polynomial
 * arithmetic is done per request.
 *
 * Admission (slrng_server_submit) reserves 8 n bytes of the device output
 * arena (budget_bytes).  When the arena is full it blocks until space is
 * released, or returns SLRNG_EAGAIN with SLRNG_SUBMIT_NONBLOCK.  A worker
 * thread batches every pending request into one iteration (request-state
 * kernel + persistent generation kernel) and launches it on one of
 * `inflight` HIP streams while earlier iterations still run; one completion
 * thread per stream stamps latencies when its iteration completes, so
 * iterations complete in any order.  The generation kernel's last wave
 * signals completion through pinned host memory, once every output of the
 * iteration is visible device-wide; the completion thread polls that signal
 * (up to 2 ms, then it blocks on the stream's end event).  Latency runs from the request's arrival
 * (the submit call, before any wait for arena space; for slrng_server_replay
 * the scheduled arrival time) to the completion of its iteration.  Outputs are
 * read from the arena pointer that poll/wait return, then released
 * (slrng_server_release), or released automatically at completion with
 * SLRNG_SUBMIT_AUTORELEASE (throughput runs).
 *
 * slrng_server_poll: 1 when done, 0 while pending, SLRNG_EHIP if its iteration
 *   failed, SLRNG_EINVAL for an unknown or released ticket; fills the output
 *   pointer and the stream position (its low 64 bits).  slrng_server_wait:
 *   blocks until done.
 * slrng_server_advance: moves stream j's head by steps_hi 2^64 + steps_lo
 *   (requests admitted later start that much further; earlier ones keep their
 *   positions).  EINVAL for a bad stream id.
 * slrng_server_intervals: the generation kernels' device intervals, one per
 *   iteration in completion order: from the claim of the first tile to the
 *   end of the last wave, read from the device clock (wall_clock64) that the
 *   kernels stamp (ms from the server's creation),
 *   written up to `cap` entries; *count = the number recorded since creation
 *   or the last reset_stats.  Iterations on different HIP streams overlap on
 *   the device when one's interval starts before another's ends.
 * slrng_server_release: frees a completed request's arena range (EAGAIN while
 *   it is still pending or in flight).
 * slrng_server_drain: waits until every submitted request has completed.
 * slrng_server_get_stats / _reset_stats: counters; latency percentiles of the
 *   completed requests; busy_s is the union of the iterations' device time
 *   (from the start of the iteration's first kernel to the end of the generation
 *   kernel), kernel_s that of the generation kernels alone (the intervals
 *   above); both from the device clock stamps.
 * slrng_server_replay: submits count requests at the given arrival times
 *   (seconds from the call), with SLRNG_SUBMIT_AUTORELEASE, then drains (a
 *   load generator for benchmarks).
 * slrng_server_destroy: completes everything submitted, stops the threads and
 *   frees all memory.  submit/poll/wait/release/stats are thread-safe. */
typedef struct slrng_server slrng_server;

typedef struct slrng_server_opts {
  uint64_t budget_bytes; /* output arena (device memory) */
  uint64_t seed;         /* resident streams' seed */
  uint64_t chunk;        /* lane-chunk length (0 = default) */
  uint32_t n_streams;    /* resident streams */
  int32_t variant;
  int32_t max_batch;     /* requests per iteration (0 = default; 1 = the plain form) */
  int32_t inflight;      /* iterations in flight, 1..8 (0 = default) */
  int32_t tile;          /* 16 or 32 (0 = default) */
  int32_t waves_per_cu;  /* persistent grid (0 = default) */
  int32_t window_us;     /* batching window: an iteration waits until its oldest
                            request is this old (default 0: launch as soon as a
                            slot is free; requests arriving meanwhile wait for
                            the next iteration) ... */
  int32_t min_chunk;     /* smallest lane-chunk (outputs) when the chunk length is
                            fitted to an iteration (0 = default: the larger of
                            64 and n/2, n the state bits) */
  uint64_t window_bytes; /* ... or until this many bytes are pending */
  int32_t arena_plain;   /* 1: the arena is one plain device allocation; 0 (default):
                            memory from slrng_output_alloc (physical pages spread
                            over the HBM) */
  int32_t store;         /* output stores of the generation kernel: 0 (default)
                            write-through, 1 plain, 2 nontemporal (values never
                            change) */
} slrng_server_opts;

enum { SLRNG_SUBMIT_NONBLOCK = 1, SLRNG_SUBMIT_AUTORELEASE = 2 };

typedef struct slrng_server_stats {
  uint64_t submitted, completed, failed, rejected, outputs;
  uint64_t iterations, max_inflight, max_batch, peak_reserved_bytes, reserved_bytes;
  double wall_s, busy_s, mean_batch;
  double p50_us, p99_us, max_us;
  double kernel_s; /* union of the generation kernels' device time */
} slrng_server_stats;

int slrng_server_default_opts(slrng_server_opts *opts);
int slrng_server_create(const slrng_server_opts *opts, slrng_server **out);
int slrng_server_submit(slrng_server *sv, uint32_t stream_id, uint64_t n, int kind, int flags,
                        uint64_t *ticket);
int slrng_server_poll(slrng_server *sv, uint64_t ticket, void **dev_ptr, uint64_t *pos);
int slrng_server_wait(slrng_server *sv, uint64_t ticket, void **dev_ptr, uint64_t *pos);
int slrng_server_release(slrng_server *sv, uint64_t ticket);
int slrng_server_drain(slrng_server *sv);
int slrng_server_get_stats(slrng_server *sv, slrng_server_stats *out);
int slrng_server_reset_stats(slrng_server *sv);
int slrng_server_replay(slrng_server *sv, const double *t_arrival_s, const uint32_t *stream_ids,
                        const uint64_t *n, const int32_t *kinds, size_t count);
int slrng_server_advance(slrng_server *sv, uint32_t stream_id, uint64_t steps_hi, uint64_t steps_lo);
int slrng_server_intervals(slrng_server *sv, double *kernel_start_ms, double *kernel_end_ms, uint64_t cap,
                           uint64_t *count);
int slrng_server_destroy(slrng_server *sv);

#ifdef __cplusplus
}
#endif

#endif /* SLRNG_H */
