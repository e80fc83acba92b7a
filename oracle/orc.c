/*
 * CPU oracle for the scrambled linear generators of Blackman & Vigna,
 * "Scrambled Linear Pseudorandom Number Generators" (ACM TOMS).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, serial restatement
 * of what the paper defines.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library, and the GPU library never calls it.
 *
 * Everything is integer arithmetic, so the GPU result must match bit for bit.
 *
 * What follows which passage of the paper:
 *   - xoroshiro engine, two words:   Section "Linear engines", figure
 *     fig:xoroshiro128 and matrix X_2w.
 *   - xoroshiro engine, k > 2 words: figure fig:xoroshiro1024 (cyclic update
 *     with the index p) and the block matrix of equation eq:M.
 *   - xoshiro engines (4 and 8 words): figures fig:xoshiro256, fig:xoshiro512,
 *     matrices S_4w and S_8w.
 *   - scramblers +, *, ++, **: Section "Scramblers"; the words each scrambler
 *     reads are the ones named in the four code figures.
 *   - engine parameters: Table tab:par64 (64-bit) and the small-word instances
 *     quoted in Section "Equidistribution"; scrambler constants: tab:scr64.
 *   - characteristic polynomial by Berlekamp-Massey on one bit of the engine:
 *     Section "Polynomials and full period" and Section "The + scrambler".
 *   - jump functions: Section "Combining linear engines and scramblers" says
 *     every generator has jump functions; the method used here is the
 *     Cayley-Hamilton reading: s*M^J = sum_i r_i * s*M^i where
 *     r(x) = x^J mod p(x) and p is the characteristic polynomial.
 *   - SplitMix seeding: Section "Choosing a generator" (fill the state with the
 *     outputs of a SplitMix generator seeded with the 64-bit seed).  The paper
 *     prints no SplitMix constants.  The golden gamma is pinned by a test (the
 *     odd integer nearest 2^64/phi); the finalizer's shift amounts and
 *     multipliers are those of the SplitMix64 publication (Steele, Lea and
 *     Flood, OOPSLA 2014, mix64): parity unpinned against any external
 *     implementation, since no test vector is available.
 *   - 53-bit doubles: Section "Choosing a generator" (upper 53 bits); the
 *     value is (x >> 11) * 2^-53, exact.
 *   - 32-bit generators: Section "The 32-bit case", tables tab:par32 and
 *     tab:scr32; the paper says the word choices of the 64-bit two-word
 *     xoroshiro and of xoshiro256 carry over to xoroshiro64 and xoshiro128.
 *     Seeding them: the paper only remarks that a 32-bit SplitMix is
 *     immediate to define.  Reading taken here: the state array is filled
 *     with the output stream of SplitMix64, i.e. each 64-bit output gives two
 *     32-bit words, low half first (parity unpinned, like SplitMix itself).
 *
 * State convention.  A state is k words in the "logical order" of the block
 * matrices: word j of the row vector x = <x_0 .. x_{k-1}> with the next state
 * equal to x * M.  For the two-word xoroshiro and for xoshiro this is the array
 * s[] of the figures.  For xoroshiro with k > 2 words the figure keeps an array
 * s[] and an index p; the logical order is x_j = s[(p + 1 + j) mod k].
 *
 * Word size w may be anything from 1 to 64 bits so that the small instances
 * the paper uses as counterexamples run through exactly the same code.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef uint64_t u64;

enum { ORC_XOROSHIRO = 0, ORC_XOSHIRO = 1 };
enum { ORC_NONE = 0, ORC_PLUS = 1, ORC_PLUSPLUS = 2, ORC_STAR = 3, ORC_STARSTAR = 4 };

#define ORC_MAXK 16

/* One generator: engine family, word size, number of words, engine
 * parameters a, b, c, and scrambler kind with its rotation r and
 * multipliers ms (first) and mt (second).  Layout mirrored by ctypes. */
typedef struct {
    int32_t family;
    int32_t w;
    int32_t k;
    int32_t a, b, c;
    int32_t scr;
    int32_t r;
    u64 ms, mt;
} orc_gen;

/* ------------------------------------------------------------------ */
/* w-bit word arithmetic                                               */
/* ------------------------------------------------------------------ */

static u64 wmask(int w) { return w >= 64 ? ~(u64)0 : (((u64)1 << w) - 1); }

/* left shift of a w-bit word: the matrix S^b (ones on the subdiagonal) */
static u64 shl(u64 x, int b, int w) { return b >= w ? 0 : ((x << b) & wmask(w)); }

/* left rotation of a w-bit word: the matrix R^r */
static u64 rotl(u64 x, int r, int w)
{
    r %= w;
    if (r == 0) return x & wmask(w);
    return ((x << r) | (x >> (w - r))) & wmask(w);
}

static u64 addw(u64 x, u64 y, int w) { return (x + y) & wmask(w); }
static u64 mulw(u64 x, u64 y, int w) { return (x * y) & wmask(w); }

/* ------------------------------------------------------------------ */
/* Engine state in the layout of the figures                           */
/* ------------------------------------------------------------------ */

typedef struct {
    u64 s[ORC_MAXK];
    int p;           /* only for xoroshiro with k > 2 */
} orc_state;

static void load_logical(const orc_gen *g, const u64 *x, orc_state *st)
{
    for (int j = 0; j < g->k; j++) st->s[j] = x[j] & wmask(g->w);
    /* with p = k-1, s[(p+1+j) mod k] = s[j] = x_j */
    st->p = g->k - 1;
}

static void store_logical(const orc_gen *g, const orc_state *st, u64 *x)
{
    if (g->family == ORC_XOROSHIRO && g->k > 2) {
        for (int j = 0; j < g->k; j++) x[j] = st->s[(st->p + 1 + j) % g->k];
    } else {
        for (int j = 0; j < g->k; j++) x[j] = st->s[j];
    }
}

/* Scrambled output of the current state (outputs are computed before the
 * state is advanced, as in all four code figures). */
static u64 output(const orc_gen *g, const orc_state *st)
{
    const int w = g->w;
    if (g->family == ORC_XOROSHIRO) {
        u64 s0, sl;
        if (g->k == 2) { s0 = st->s[0]; sl = st->s[1]; }
        else { s0 = st->s[(st->p + 1) % g->k]; sl = st->s[st->p]; }
        switch (g->scr) {
        case ORC_NONE: return s0;
        case ORC_PLUS: return addw(s0, sl, w);
        case ORC_PLUSPLUS:
            /* fig:xoroshiro128 adds s0 after the rotation;
             * fig:xoroshiro1024 adds s15, the last word */
            if (g->k == 2) return addw(rotl(addw(s0, sl, w), g->r, w), s0, w);
            return addw(rotl(addw(s0, sl, w), g->r, w), sl, w);
        case ORC_STAR: return mulw(s0, g->ms, w);
        case ORC_STARSTAR: return mulw(rotl(mulw(s0, g->ms, w), g->r, w), g->mt, w);
        }
        return 0;
    }
    const u64 *s = st->s;
    if (g->k == 4) {
        /* fig:xoshiro256 */
        switch (g->scr) {
        case ORC_NONE: return s[0];
        case ORC_PLUS: return addw(s[0], s[3], w);
        case ORC_PLUSPLUS: return addw(rotl(addw(s[0], s[3], w), g->r, w), s[0], w);
        case ORC_STARSTAR: return mulw(rotl(mulw(s[1], g->ms, w), g->r, w), g->mt, w);
        }
        return 0;
    }
    /* fig:xoshiro512 */
    switch (g->scr) {
    case ORC_NONE: return s[0];
    case ORC_PLUS: return addw(s[0], s[2], w);
    case ORC_PLUSPLUS: return addw(rotl(addw(s[0], s[2], w), g->r, w), s[2], w);
    case ORC_STARSTAR: return mulw(rotl(mulw(s[1], g->ms, w), g->r, w), g->mt, w);
    }
    return 0;
}

/* One step of the linear engine, as the code figures write it. */
static void step(const orc_gen *g, orc_state *st)
{
    const int w = g->w;
    u64 *s = st->s;
    if (g->family == ORC_XOROSHIRO) {
        if (g->k == 2) {
            /* fig:xoroshiro128 */
            const u64 s0 = s[0];
            u64 s1 = s[1];
            s1 ^= s0;
            s[0] = rotl(s0, g->a, w) ^ s1 ^ shl(s1, g->b, w);
            s[1] = rotl(s1, g->c, w);
        } else {
            /* fig:xoroshiro1024, with 15 replaced by k-1 */
            const int q = st->p;
            st->p = (st->p + 1) % g->k;
            const u64 s0 = s[st->p];
            u64 sl = s[q];
            sl ^= s0;
            s[q] = rotl(s0, g->a, w) ^ sl ^ shl(sl, g->b, w);
            s[st->p] = rotl(sl, g->c, w);
        }
        return;
    }
    if (g->k == 4) {
        /* fig:xoshiro256 */
        const u64 t = shl(s[1], g->a, w);
        s[2] ^= s[0];
        s[3] ^= s[1];
        s[1] ^= s[2];
        s[0] ^= s[3];
        s[2] ^= t;
        s[3] = rotl(s[3], g->b, w);
    } else {
        /* fig:xoshiro512 */
        const u64 t = shl(s[1], g->a, w);
        s[2] ^= s[0];
        s[5] ^= s[1];
        s[1] ^= s[2];
        s[7] ^= s[3];
        s[3] ^= s[4];
        s[4] ^= s[5];
        s[0] ^= s[6];
        s[6] ^= s[7];
        s[6] ^= t;
        s[7] = rotl(s[7], g->b, w);
    }
}

/* ------------------------------------------------------------------ */
/* Public: stepping and generation                                     */
/* ------------------------------------------------------------------ */

int orc_valid(const orc_gen *g)
{
    if (g->w < 1 || g->w > 64) return 0;
    if (g->family == ORC_XOROSHIRO) {
        if (g->k < 2 || g->k > ORC_MAXK) return 0;
    } else if (g->family == ORC_XOSHIRO) {
        if (g->k != 4 && g->k != 8) return 0;   /* only S_4w and S_8w exist */
        if (g->scr == ORC_STAR) return 0;        /* no * variant of xoshiro */
    } else {
        return 0;
    }
    return g->scr >= ORC_NONE && g->scr <= ORC_STARSTAR;
}

/* x (k words, logical order) <- x * M^nsteps */
void orc_advance(const orc_gen *g, u64 *x, u64 nsteps)
{
    orc_state st;
    load_logical(g, x, &st);
    for (u64 i = 0; i < nsteps; i++) step(g, &st);
    store_logical(g, &st, x);
}

/* Scrambled output of one state (logical order). */
u64 orc_output(const orc_gen *g, const u64 *x)
{
    orc_state st;
    load_logical(g, x, &st);
    return output(g, &st);
}

/* Serial generation for one stream: out[t] = scramble(x * M^t), t < n;
 * x is advanced by n steps. */
void orc_generate1(const orc_gen *g, u64 *x, u64 n, u64 *out)
{
    orc_state st;
    load_logical(g, x, &st);
    for (u64 t = 0; t < n; t++) {
        out[t] = output(g, &st);
        step(g, &st);
    }
    store_logical(g, &st, x);
}

/* The same, but keep only outputs at times t_lo <= t < t_hi (the state is
 * still advanced through every step). */
void orc_generate_window(const orc_gen *g, u64 *x, u64 t_lo, u64 t_hi, u64 *out)
{
    orc_state st;
    load_logical(g, x, &st);
    for (u64 t = 0; t < t_hi; t++) {
        if (t >= t_lo) out[t - t_lo] = output(g, &st);
        step(g, &st);
    }
    store_logical(g, &st, x);
}

/* 53-bit double from the upper 53 bits (exact). */
double orc_to_double(u64 v) { return (double)(v >> 11) * 0x1.0p-53; }

void orc_to_double_array(const u64 *v, double *d, u64 n)
{
    for (u64 i = 0; i < n; i++) d[i] = orc_to_double(v[i]);
}

/* Many streams, stream-major: states is S x k (logical order, updated in
 * place), out is S x ld with n outputs per row.  Streams are independent;
 * the only parallelism is one thread per block of streams. */
typedef struct {
    const orc_gen *g;
    u64 *states;
    u64 S, n, ld;
    u64 *out;
    double *dout;
    int tid, nth;
} gen_job;

static void *gen_worker(void *arg)
{
    gen_job *j = (gen_job *)arg;
    const int k = j->g->k;
    for (u64 i = (u64)j->tid; i < j->S; i += (u64)j->nth) {
        u64 *x = j->states + i * k;
        if (j->out) {
            orc_generate1(j->g, x, j->n, j->out + i * j->ld);
            if (j->dout) orc_to_double_array(j->out + i * j->ld, j->dout + i * j->ld, j->n);
        } else {
            /* doubles only */
            orc_state st;
            load_logical(j->g, x, &st);
            double *d = j->dout + i * j->ld;
            for (u64 t = 0; t < j->n; t++) {
                d[t] = orc_to_double(output(j->g, &st));
                step(j->g, &st);
            }
            store_logical(j->g, &st, x);
        }
    }
    return NULL;
}

int orc_generate_many(const orc_gen *g, u64 *states, u64 S, u64 n, u64 *out,
                      double *dout, u64 ld, int nthreads)
{
    if (!orc_valid(g)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    gen_job jobs[256];
    for (int t = 0; t < nthreads; t++) {
        jobs[t] = (gen_job){g, states, S, n, ld, out, dout, t, nthreads};
        if (nthreads == 1) { gen_worker(&jobs[t]); return 0; }
        pthread_create(&th[t], NULL, gen_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    return 0;
}

/* ------------------------------------------------------------------ */
/* SplitMix seeding                                                    */
/* ------------------------------------------------------------------ */

/* The odd integer nearest 2^64/phi (pinned by a test). */
#define ORC_GOLDEN_GAMMA 0x9e3779b97f4a7c15ULL

u64 orc_splitmix_gamma(void) { return ORC_GOLDEN_GAMMA; }

/* SplitMix64 finalizer (mix64 of the SplitMix publication). */
u64 orc_splitmix_mix(u64 z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Fill k words: the generator's counter starts at the seed; each output
 * first adds the gamma to the counter, then returns the finalizer of it. */
void orc_splitmix_fill(u64 seed, u64 *x, int k)
{
    u64 ctr = seed;
    for (int j = 0; j < k; j++) {
        ctr += ORC_GOLDEN_GAMMA;
        x[j] = orc_splitmix_mix(ctr);
    }
}

/* ------------------------------------------------------------------ */
/* Berlekamp-Massey over Z/2Z                                          */
/* ------------------------------------------------------------------ */

/* Bit sequence s[0..N) (one byte per bit, 0 or 1).  Returns the linear
 * complexity L and, if conn != NULL, the connection polynomial
 * C(z) = 1 + c_1 z + ... + c_L z^L as bytes conn[0..L].  The sequence then
 * satisfies s_t + c_1 s_{t-1} + ... + c_L s_{t-L} = 0 for L <= t < N.
 *
 * The textbook algorithm (Massey 1969), with the polynomials kept as bit
 * arrays packed into 64-bit words so that long sequences stay tractable; the
 * discrepancy is the parity of C AND the reversed window of the sequence. */
long orc_berlekamp_massey(const uint8_t *s, long N, uint8_t *conn)
{
    const long W = N / 64 + 2;
    u64 *C = calloc((size_t)W, 8), *B = calloc((size_t)W, 8), *T = calloc((size_t)W, 8);
    u64 *rv = calloc((size_t)W + 1, 8);   /* rv bit j = s[N-1-j] */
    if (!C || !B || !T || !rv) { free(C); free(B); free(T); free(rv); return -1; }
    for (long j = 0; j < N; j++)
        if (s[N - 1 - j]) rv[j >> 6] |= (u64)1 << (j & 63);
    C[0] = 1;
    B[0] = 1;
    long L = 0, m = 1;
    for (long n = 0; n < N; n++) {
        /* discrepancy d = sum_{i=0..L} c_i s_{n-i}, and s_{n-i} is bit
         * (N-1-n+i) of rv: the parity of C AND rv shifted right by N-1-n */
        const long off = N - 1 - n;
        const long ow = off >> 6;
        const int ob = (int)(off & 63);
        const long nw = L / 64 + 1;
        u64 acc = 0;
        for (long i = 0; i < nw; i++) {
            u64 word = rv[ow + i] >> ob;
            if (ob) word |= rv[ow + i + 1] << (64 - ob);
            if (i == nw - 1) {
                const int top = (int)(L & 63);
                word &= top == 63 ? ~(u64)0 : (((u64)1 << (top + 1)) - 1);
            }
            acc ^= C[i] & word;
        }
        if (!__builtin_parityll(acc)) { m++; continue; }
        /* C <- C + z^m B (and B <- old C when the length changes) */
        const int lengthen = 2 * L <= n;
        if (lengthen) memcpy(T, C, (size_t)W * 8);
        const long sw = m >> 6;
        const int sb = (int)(m & 63);
        for (long i = W - 1; i >= sw; i--) {
            u64 v = B[i - sw] << sb;
            if (sb && i - sw - 1 >= 0) v |= B[i - sw - 1] >> (64 - sb);
            C[i] ^= v;
        }
        if (lengthen) {
            L = n + 1 - L;
            memcpy(B, T, (size_t)W * 8);
            m = 1;
        } else {
            m++;
        }
    }
    if (conn)
        for (long i = 0; i <= L; i++) conn[i] = (uint8_t)((C[i >> 6] >> (i & 63)) & 1);
    free(C); free(B); free(T); free(rv);
    return L;
}

/* ------------------------------------------------------------------ */
/* Polynomials over Z/2Z (bit i of word i/64 = coefficient of x^i)     */
/* ------------------------------------------------------------------ */

static int pbit(const u64 *a, long i) { return (int)((a[i >> 6] >> (i & 63)) & 1); }
static void pflip(u64 *a, long i) { a[i >> 6] ^= (u64)1 << (i & 63); }

/* out = a * b mod p; deg p = n; a, b of degree < n; all arrays n/64+1 words */
void orc_poly_mulmod(const u64 *a, const u64 *b, const u64 *p, int n, u64 *out)
{
    int W = n / 64 + 1;
    int W2 = 2 * W + 1;
    u64 *prod = calloc((size_t)W2, 8);
    /* schoolbook product */
    for (long i = 0; i < n; i++) {
        if (!pbit(a, i)) continue;
        for (long j = 0; j < n; j++)
            if (pbit(b, j)) pflip(prod, i + j);
    }
    /* reduce from the top: subtract x^(d-n) p whenever bit d is set */
    for (long d = 2L * n - 2; d >= n; d--) {
        if (!pbit(prod, d)) continue;
        for (long j = 0; j <= n; j++)
            if (pbit(p, j)) pflip(prod, d - n + j);
    }
    memset(out, 0, (size_t)W * 8);
    for (long i = 0; i < n; i++)
        if (pbit(prod, i)) pflip(out, i);
    free(prod);
}

/* out = x^J mod p, J given as little-endian 64-bit words jw[0..nj) */
void orc_poly_xpow(const u64 *jw, int nj, const u64 *p, int n, u64 *out)
{
    int W = n / 64 + 1;
    u64 *acc = calloc((size_t)W, 8), *xp = calloc((size_t)W, 8), *tmp = calloc((size_t)W, 8);
    acc[0] = 1;                 /* 1 */
    /* xp = x mod p (n >= 2 here) */
    pflip(xp, 1);
    /* right-to-left binary exponentiation: acc *= xp for set bits, xp squared */
    int top = nj * 64 - 1;
    while (top >= 0 && !((jw[top >> 6] >> (top & 63)) & 1)) top--;
    for (int i = 0; i <= top; i++) {
        if ((jw[i >> 6] >> (i & 63)) & 1) {
            orc_poly_mulmod(acc, xp, p, n, tmp);
            memcpy(acc, tmp, (size_t)W * 8);
        }
        if (i < top) {
            orc_poly_mulmod(xp, xp, p, n, tmp);
            memcpy(xp, tmp, (size_t)W * 8);
        }
    }
    memcpy(out, acc, (size_t)W * 8);
    free(acc); free(xp); free(tmp);
}

/* Characteristic polynomial of the engine (degree n = k*w): Berlekamp-Massey
 * on 2n consecutive values of bit 0 of word 0 starting from x0 (nonzero).
 * The connection polynomial C(z) of degree L gives p(x) = x^L C(1/x).
 * Returns L (equal to n when p is irreducible and x0 is nonzero). */
long orc_charpoly(const orc_gen *g, const u64 *x0, u64 *p_out)
{
    const long n = (long)g->k * g->w;
    const long N = 2 * n;
    uint8_t *bits = malloc((size_t)N), *conn = malloc((size_t)N + 1);
    orc_gen e = *g;
    e.scr = ORC_NONE;
    orc_state st;
    load_logical(&e, x0, &st);
    u64 x[ORC_MAXK];
    for (long t = 0; t < N; t++) {
        store_logical(&e, &st, x);
        bits[t] = (uint8_t)(x[0] & 1);
        step(&e, &st);
    }
    long L = orc_berlekamp_massey(bits, N, conn);
    memset(p_out, 0, (size_t)(n / 64 + 1) * 8);
    for (long i = 0; i <= L; i++)
        if (conn[i]) pflip(p_out, L - i);
    free(bits); free(conn);
    return L;
}

/* x <- x * M^J where r(x) = x^J mod p is given (degree < n):
 * acc = sum_i r_i * (x * M^i), accumulated while stepping. */
void orc_jump_poly(const orc_gen *g, u64 *x, const u64 *r)
{
    const long n = (long)g->k * g->w;
    u64 acc[ORC_MAXK] = {0}, cur[ORC_MAXK];
    orc_gen e = *g;
    orc_state st;
    load_logical(&e, x, &st);
    for (long i = 0; i < n; i++) {
        if (pbit(r, i)) {
            store_logical(&e, &st, cur);
            for (int j = 0; j < g->k; j++) acc[j] ^= cur[j];
        }
        step(&e, &st);
    }
    for (int j = 0; j < g->k; j++) x[j] = acc[j];
}

/* Seeded state of a generator.  64-bit words: consecutive SplitMix64
 * outputs.  32-bit words: the SplitMix64 output stream split into 32-bit
 * words, low half first (the reading stated at the top).  Any other word
 * size (the paper's small instances): one output per word, masked. */
void orc_seed_state(const orc_gen *g, u64 seed, u64 *x)
{
    const int k = g->k;
    if (g->w == 32) {
        u64 out[ORC_MAXK];
        orc_splitmix_fill(seed, out, (k + 1) / 2);
        for (int j = 0; j < k; j++)
            x[j] = (j & 1) ? (out[j / 2] >> 32) : (out[j / 2] & 0xffffffffULL);
        return;
    }
    orc_splitmix_fill(seed, x, k);
    for (int j = 0; j < k; j++) x[j] &= wmask(g->w);
}

/* Stream chain: base = seeded state; stream i = base * (M^J)^i.
 * p is the characteristic polynomial, r = x^J mod p.  states: S x k. */
void orc_stream_chain(const orc_gen *g, u64 seed, const u64 *r, u64 S, u64 *states)
{
    const int k = g->k;
    u64 x[ORC_MAXK];
    orc_seed_state(g, seed, x);
    for (u64 i = 0; i < S; i++) {
        memcpy(states + i * k, x, (size_t)k * 8);
        orc_jump_poly(g, x, r);
    }
}

/* Apply the jump polynomial r to every state of an array, in threads. */
typedef struct { const orc_gen *g; u64 *states; u64 S; const u64 *r; int tid, nth; } jmp_job;

static void *jmp_worker(void *arg)
{
    jmp_job *j = (jmp_job *)arg;
    for (u64 i = (u64)j->tid; i < j->S; i += (u64)j->nth)
        orc_jump_poly(j->g, j->states + i * j->g->k, j->r);
    return NULL;
}

void orc_jump_many(const orc_gen *g, u64 *states, u64 S, const u64 *r, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    jmp_job jobs[256];
    for (int t = 0; t < nthreads; t++) {
        jobs[t] = (jmp_job){g, states, S, r, t, nthreads};
        if (nthreads == 1) { jmp_worker(&jobs[t]); return; }
        pthread_create(&th[t], NULL, jmp_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------ */
/* Small-instance tools used by the pins                               */
/* ------------------------------------------------------------------ */

/* Period of the engine from a nonzero state, by brute force (stops at
 * limit and returns 0 if the start state has not come back by then). */
u64 orc_period(const orc_gen *g, const u64 *x0, u64 limit)
{
    orc_state st, st0;
    load_logical(g, x0, &st);
    st0 = st;
    u64 x[ORC_MAXK], y[ORC_MAXK];
    store_logical(g, &st0, y);
    for (u64 t = 1; t <= limit; t++) {
        step(g, &st);
        store_logical(g, &st, x);
        if (memcmp(x, y, (size_t)g->k * 8) == 0) return t;
    }
    return 0;
}

/* d-dimensional output histogram over every state of a small generator
 * (k*w <= 32): counts[v_0 + v_1 2^w + ... ] for the first d outputs from
 * each of the 2^(k w) states, the zero state included.  counts has 2^(d w)
 * entries. */
int orc_tuple_counts(const orc_gen *g, int d, uint32_t *counts)
{
    const int n = g->k * g->w;
    if (n > 32 || d * g->w > 32) return -1;
    const u64 nstates = (u64)1 << n;
    memset(counts, 0, ((size_t)1 << (d * g->w)) * sizeof(uint32_t));
    u64 x[ORC_MAXK];
    for (u64 v = 0; v < nstates; v++) {
        for (int j = 0; j < g->k; j++) x[j] = (v >> (j * g->w)) & wmask(g->w);
        orc_state st;
        load_logical(g, x, &st);
        u64 idx = 0;
        for (int t = 0; t < d; t++) {
            idx |= output(g, &st) << (t * g->w);
            step(g, &st);
        }
        counts[idx]++;
    }
    return 0;
}
