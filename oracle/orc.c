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
 *   - engine steps: Section "Linear engines".  The step is the product of the
 *     state row vector with the block matrix the paper prints (X_2w, X_kw of
 *     equation eq:M, S_4w, S_8w), expanded block by block into xors of
 *     shifted and rotated words; the code figures are not transcribed.
 *   - scramblers +, *, ++, **: Section "Scramblers" (the formulas), with the
 *     words each one reads taken from the code figures fig:xoroshiro128,
 *     fig:xoroshiro1024, fig:xoshiro256 and fig:xoshiro512.
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
 *     Flood, OOPSLA 2014, mix64), pinned only by a test that inverts the
 *     finalizer with its own statement of those constants.
 *   - 53-bit doubles: Section "Choosing a generator" (upper 53 bits); the
 *     value is (x >> 11) * 2^-53, exact.
 *   - 32-bit generators: Section "The 32-bit case", tables tab:par32 and
 *     tab:scr32; the paper says the word choices of the 64-bit two-word
 *     xoroshiro and of xoshiro256 carry over to xoroshiro64 and xoshiro128.
 *     Seeding them: the paper only remarks that a 32-bit SplitMix is
 *     immediate to define.  Reading taken here: the state array is filled
 *     with the output stream of SplitMix64, i.e. each 64-bit output gives two
 *     32-bit words, low half first.
 *
 * Parity unpinned (no fact of the paper fixes these; they follow the code
 * figures or the cited publication, and no external test vector exists here):
 *   - the SplitMix64 finalizer constants (shifts 30, 27, 31 and the two
 *     multipliers) against any external SplitMix64 implementation;
 *   - the word that ** scrambles: the first logical word of xoroshiro, word 1
 *     of xoshiro (the equidistribution results allow other words);
 *   - the word ++ adds back for the two-word xoroshiro (the first; both
 *     choices are 1-dimensionally equidistributed there);
 *   - the split of SplitMix64 outputs into the 32-bit generators' words.
 *
 * State convention.  A state is k words in the "logical order" of the block
 * matrices: word j of the row vector x = <x_0 .. x_{k-1}> with the next state
 * equal to x * M.  For the two-word xoroshiro and for xoshiro this is the array
 * s[] of the figures.  For xoroshiro with k > 2 words the figure keeps an array
 * s[] and a cyclic index p; its logical order is x_j = s[(p + 1 + j) mod k],
 * and the oracle stores the logical order directly.
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
/* Transition matrices of Section "Linear engines", block by block     */
/* ------------------------------------------------------------------ */

/* The step is the product x' = x M of the state row vector x (k words in
 * logical order) with the engine's kw x kw block matrix M.  Block (i, j) maps
 * word i of x to its contribution to word j of x'; every block is a sum of
 * identities I, shifts S^e and rotations R^e (e = a, b or c), so x'_j is the
 * xor over i of those operators applied to x_i.  The blocks are written below
 * as the paper prints them; the code figures play no part in the oracle's
 * step. */

/* S_4w and S_8w (xoshiro256 and xoshiro512), entry [i][j] as printed: "0" is
 * the zero block, "I" the identity, "Sa" = S^a, "Rb" = R^b; '+' separates the
 * terms of a sum. */
static const char *const S4W[4][4] = {
    {"I", "I", "I",  "0"},
    {"I", "I", "Sa", "Rb"},
    {"0", "I", "I",  "0"},
    {"I", "0", "0",  "Rb"},
};
static const char *const S8W[8][8] = {
    {"I", "I", "I", "0", "0", "0", "0",  "0"},
    {"0", "I", "0", "0", "I", "I", "Sa", "0"},
    {"0", "I", "I", "0", "0", "0", "0",  "0"},
    {"0", "0", "0", "I", "0", "0", "I",  "Rb"},
    {"0", "0", "0", "I", "I", "0", "0",  "0"},
    {"0", "0", "0", "0", "I", "I", "0",  "0"},
    {"I", "0", "0", "0", "0", "0", "I",  "0"},
    {"0", "0", "0", "0", "0", "0", "I",  "Rb"},
};

/* X_kw of equation eq:M (X_2w when k = 2): the first row holds R^a + S^b + I
 * and R^c in the last two columns, rows 1 .. k-2 hold one identity just left
 * of the diagonal (the words move down by one position), and the last row
 * holds S^b + I and R^c in the last two columns. */
static const char *xoroshiro_block(int k, int i, int j)
{
    if (i == 0 && j == k - 2) return "Ra+Sb+I";
    if (i == 0 && j == k - 1) return "Rc";
    if (i == k - 1 && j == k - 2) return "Sb+I";
    if (i == k - 1 && j == k - 1) return "Rc";
    if (i >= 1 && i <= k - 2 && j == i - 1) return "I";
    return "0";
}

enum { OP_I = 0, OP_S = 1, OP_R = 2 };

/* One term of a block: word src, operator op with amount e, xored into word
 * dst of the next state. */
typedef struct { uint8_t src, dst, op, e; } term;

#define ORC_MAXTERMS 64

typedef struct {
    orc_gen g;
    int nt;
    term t[ORC_MAXTERMS];
} engine;

static int param(const orc_gen *g, char name)
{
    return name == 'a' ? g->a : name == 'b' ? g->b : g->c;
}

/* Expand every block of the engine's matrix into its terms. */
static void engine_init(const orc_gen *g, engine *m)
{
    m->g = *g;
    m->nt = 0;
    for (int i = 0; i < g->k; i++)
        for (int j = 0; j < g->k; j++) {
            const char *blk = g->family == ORC_XOSHIRO
                                  ? (g->k == 4 ? S4W[i][j] : S8W[i][j])
                                  : xoroshiro_block(g->k, i, j);
            for (const char *c = blk; *c; c++) {
                term t = {(uint8_t)i, (uint8_t)j, OP_I, 0};
                if (*c == '0' || *c == '+') continue;
                if (*c == 'S' || *c == 'R') {
                    t.op = *c == 'S' ? OP_S : OP_R;
                    t.e = (uint8_t)param(g, c[1]);
                    c++;
                }
                if (m->nt < ORC_MAXTERMS) m->t[m->nt++] = t;
            }
        }
}

/* x <- x M (logical order). */
static void step(const engine *m, u64 *x)
{
    const int w = m->g.w;
    u64 y[ORC_MAXK] = {0};
    for (int q = 0; q < m->nt; q++) {
        const term *t = &m->t[q];
        const u64 v = x[t->src];
        y[t->dst] ^= t->op == OP_I ? v : t->op == OP_S ? shl(v, t->e, w) : rotl(v, t->e, w);
    }
    memcpy(x, y, (size_t)m->g.k * 8);
}

/* Scrambled output of a state in logical order (Section "Scramblers"); the
 * output is taken before the state is advanced.  The words each scrambler
 * reads follow the code figures: for xoroshiro the first and last logical
 * words (s0 and s1 of fig:xoroshiro128, s0 and s15 of fig:xoroshiro1024), for
 * xoshiro256 words 0 and 3, for xoshiro512 words 0 and 2; ** scrambles the
 * first word of xoroshiro and word 1 of xoshiro.  ++ adds back the first word
 * for the two-word xoroshiro and xoshiro256, the last word for the longer
 * xoroshiro, word 2 for xoshiro512. */
static u64 output(const orc_gen *g, const u64 *x)
{
    const int w = g->w;
    u64 first, second, added, starred;
    if (g->family == ORC_XOROSHIRO) {
        first = x[0];
        second = x[g->k - 1];
        added = g->k == 2 ? first : second;
        starred = x[0];
    } else {
        first = x[0];
        second = x[g->k == 4 ? 3 : 2];
        added = g->k == 4 ? first : second;
        starred = x[1];
    }
    switch (g->scr) {
    case ORC_NONE: return first;
    case ORC_PLUS: return addw(first, second, w);
    case ORC_PLUSPLUS: return addw(rotl(addw(first, second, w), g->r, w), added, w);
    case ORC_STAR: return mulw(starred, g->ms, w);
    case ORC_STARSTAR: return mulw(rotl(mulw(starred, g->ms, w), g->r, w), g->mt, w);
    }
    return 0;
}

static void load(const orc_gen *g, const u64 *src, u64 *x)
{
    for (int j = 0; j < g->k; j++) x[j] = src[j] & wmask(g->w);
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
    engine m;
    engine_init(g, &m);
    u64 s[ORC_MAXK];
    load(g, x, s);
    for (u64 i = 0; i < nsteps; i++) step(&m, s);
    memcpy(x, s, (size_t)g->k * 8);
}

/* Scrambled output of one state (logical order). */
u64 orc_output(const orc_gen *g, const u64 *x)
{
    u64 s[ORC_MAXK];
    load(g, x, s);
    return output(g, s);
}

/* Serial generation for one stream: out[t] = scramble(x * M^t), t < n;
 * x is advanced by n steps. */
void orc_generate1(const orc_gen *g, u64 *x, u64 n, u64 *out)
{
    engine m;
    engine_init(g, &m);
    u64 s[ORC_MAXK];
    load(g, x, s);
    for (u64 t = 0; t < n; t++) {
        out[t] = output(g, s);
        step(&m, s);
    }
    memcpy(x, s, (size_t)g->k * 8);
}

/* The same, but keep only outputs at times t_lo <= t < t_hi (the state is
 * still advanced through every step). */
void orc_generate_window(const orc_gen *g, u64 *x, u64 t_lo, u64 t_hi, u64 *out)
{
    engine m;
    engine_init(g, &m);
    u64 s[ORC_MAXK];
    load(g, x, s);
    for (u64 t = 0; t < t_hi; t++) {
        if (t >= t_lo) out[t - t_lo] = output(g, s);
        step(&m, s);
    }
    memcpy(x, s, (size_t)g->k * 8);
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
            engine m;
            engine_init(j->g, &m);
            u64 s[ORC_MAXK];
            load(j->g, x, s);
            double *d = j->dout + i * j->ld;
            for (u64 t = 0; t < j->n; t++) {
                d[t] = orc_to_double(output(j->g, s));
                step(&m, s);
            }
            memcpy(x, s, (size_t)j->g->k * 8);
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
    engine m;
    engine_init(g, &m);
    u64 x[ORC_MAXK];
    load(g, x0, x);
    for (long t = 0; t < N; t++) {
        bits[t] = (uint8_t)(x[0] & 1);
        step(&m, x);
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
    engine m;
    engine_init(g, &m);
    load(g, x, cur);
    for (long i = 0; i < n; i++) {
        if (pbit(r, i))
            for (int j = 0; j < g->k; j++) acc[j] ^= cur[j];
        step(&m, cur);
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
    engine m;
    engine_init(g, &m);
    u64 x[ORC_MAXK], y[ORC_MAXK];
    load(g, x0, x);
    memcpy(y, x, sizeof y);
    for (u64 t = 1; t <= limit; t++) {
        step(&m, x);
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
    engine m;
    engine_init(g, &m);
    u64 x[ORC_MAXK];
    for (u64 v = 0; v < nstates; v++) {
        for (int j = 0; j < g->k; j++) x[j] = (v >> (j * g->w)) & wmask(g->w);
        u64 idx = 0;
        for (int t = 0; t < d; t++) {
            idx |= output(g, x) << (t * g->w);
            step(&m, x);
        }
        counts[idx]++;
    }
    return 0;
}
