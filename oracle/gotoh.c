/*
 * CPU oracle for exact local alignment with affine gaps (Smith-Waterman with
 * Gotoh's three-state recurrence) -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file.  It shares nothing with the GPU library: no headers, no
 * tables, no helpers.  It is written to be read against the paper, not to be
 * fast: plain loops, 64-bit integers (so the "minus infinity" sentinel can be
 * decremented freely), one cell at a time.
 *
 * What it computes (SW# paper, Section 2, and the affine-gap model stated in
 * its abstract):
 *   gap of length k costs   open + (k-1)*extend           (both positive)
 *   s(x,y) = +match if x == y (case-insensitive) else -mismatch, or an entry of a
 *            substitution matrix over a given alphabet (protein scoring)
 *   E(i,j) = max(E(i,j-1) - extend, H(i,j-1) - open)     horizontal, consumes B  -> CIGAR 'I'
 *   F(i,j) = max(F(i-1,j) - extend, H(i-1,j) - open)     vertical,   consumes A  -> CIGAR 'D'
 *   H(i,j) = max(0, H(i-1,j-1) + s(A_i,B_j), E(i,j), F(i,j))
 *   H(0,.) = H(.,0) = 0,  E(.,0) = F(0,.) = -inf
 *
 *  - score + endpoint (Section 2, first phase): S = max H; the endpoint is the
 *    lexicographically smallest (i,j) -- A index first -- with H(i,j) = S.
 *  - start point (Section 2, second phase): the same recurrence without the
 *    zero and with minus-infinity borders except the anchor, run on the reversed
 *    prefixes that end at the endpoint; the start is the lexicographically
 *    smallest reversed cell whose value equals S.
 *  - the same two passes over row stripes on several threads (Section 2,
 *    linear memory), for inputs too large for one core: orc_sw_linear_mt and
 *    orc_sw_start_mt; cells are computed by the same formulas.
 *  - alignment (Section 2, reconstruction phase): Myers-Miller divide and
 *    conquer on the start..end rectangle with gap cost g + h*k, g = open -
 *    extend, h = extend; midline ties go to the smallest column, a plain
 *    crossing before a gap-spanning one; base cases as documented at mm_rec().
 *
 * Every function returns 0 on success, -1 on invalid arguments.
 */
#include <pthread.h>
#include <sched.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NEG (-((int64_t)1 << 40))

typedef struct {
    int32_t match;      /* > 0 */
    int32_t mismatch;   /* >= 0, subtracted on a mismatch */
    int32_t gap_open;   /* cost of the first gap position */
    int32_t gap_extend; /* cost of each further gap position */
    /* Substitution matrix (protein scoring): NULL for the match/mismatch scoring
     * above.  Otherwise letter_class maps every byte to its index in the alphabet
     * (-1: not a letter of it) and s(x, y) = matrix[class(x) * size + class(y)]. */
    const int8_t* matrix;
    const int8_t* letter_class;
    int32_t size;
    int32_t pad_;
} orc_scoring;

static int up(uint8_t c) { return (c >= 'a' && c <= 'z') ? c - 32 : c; }

static int64_t sub_score(uint8_t x, uint8_t y, const orc_scoring* sc) {
    if (sc->matrix) return sc->matrix[sc->letter_class[x] * sc->size + sc->letter_class[y]];
    return up(x) == up(y) ? (int64_t)sc->match : -(int64_t)sc->mismatch;
}

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

static int bad_letters(const uint8_t* s, int64_t n, const orc_scoring* sc) {
    if (!sc->matrix) return 0;
    for (int64_t i = 0; i < n; i++)
        if (sc->letter_class[s[i]] < 0) return 1;
    return 0;
}

static int bad_args(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const orc_scoring* sc) {
    if (m < 0 || n < 0 || !sc) return 1;
    if ((m > 0 && !a) || (n > 0 && !b)) return 1;
    if (sc->gap_extend <= 0 || sc->gap_open < sc->gap_extend) return 1;
    if (sc->matrix) {
        if (sc->size < 1 || sc->size > 32 || !sc->letter_class) return 1;
        if (bad_letters(a, m, sc) || bad_letters(b, n, sc)) return 1;
    } else if (sc->match <= 0 || sc->mismatch < 0) {
        return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ full matrix */

/* Full (M+1)x(N+1) matrices of H, E and F; for small inputs only. */
int orc_sw_full(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const orc_scoring* sc,
                int64_t* score, int64_t* end_a, int64_t* end_b) {
    if (bad_args(a, m, b, n, sc)) return -1;
    int64_t W = n + 1;
    int64_t* H = (int64_t*)calloc((size_t)((m + 1) * W), sizeof(int64_t));
    int64_t* E = (int64_t*)calloc((size_t)((m + 1) * W), sizeof(int64_t));
    int64_t* F = (int64_t*)calloc((size_t)((m + 1) * W), sizeof(int64_t));
    if (!H || !E || !F) { free(H); free(E); free(F); return -1; }
    for (int64_t j = 0; j <= n; j++) { H[j] = 0; E[j] = ORC_NEG; F[j] = ORC_NEG; }
    for (int64_t i = 1; i <= m; i++) {
        H[i * W] = 0; E[i * W] = ORC_NEG; F[i * W] = ORC_NEG;
        for (int64_t j = 1; j <= n; j++) {
            int64_t e = max2(E[i * W + j - 1] - sc->gap_extend, H[i * W + j - 1] - sc->gap_open);
            int64_t f = max2(F[(i - 1) * W + j] - sc->gap_extend, H[(i - 1) * W + j] - sc->gap_open);
            int64_t h = H[(i - 1) * W + j - 1] + sub_score(a[i - 1], b[j - 1], sc);
            h = max2(max2(h, 0), max2(e, f));
            E[i * W + j] = e; F[i * W + j] = f; H[i * W + j] = h;
        }
    }
    int64_t best = 0, bi = -1, bj = -1;
    for (int64_t i = 1; i <= m; i++)
        for (int64_t j = 1; j <= n; j++)
            if (H[i * W + j] > best) { best = H[i * W + j]; bi = i - 1; bj = j - 1; }
    *score = best; *end_a = bi; *end_b = bj;
    free(H); free(E); free(F);
    return 0;
}

/* Value of every cell, for property tests on small inputs (H only, row-major (M+1)x(N+1)). */
int orc_sw_matrix(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const orc_scoring* sc,
                  int64_t* H_out) {
    if (bad_args(a, m, b, n, sc) || !H_out) return -1;
    int64_t W = n + 1;
    int64_t* E = (int64_t*)malloc((size_t)W * sizeof(int64_t));
    int64_t* F = (int64_t*)malloc((size_t)W * sizeof(int64_t));
    if (!E || !F) { free(E); free(F); return -1; }
    for (int64_t j = 0; j <= n; j++) { H_out[j] = 0; F[j] = ORC_NEG; }
    for (int64_t i = 1; i <= m; i++) {
        int64_t e = ORC_NEG;
        H_out[i * W] = 0;
        for (int64_t j = 1; j <= n; j++) {
            e = max2(e - sc->gap_extend, H_out[i * W + j - 1] - sc->gap_open);
            F[j] = max2(F[j] - sc->gap_extend, H_out[(i - 1) * W + j] - sc->gap_open);
            int64_t h = H_out[(i - 1) * W + j - 1] + sub_score(a[i - 1], b[j - 1], sc);
            H_out[i * W + j] = max2(max2(h, 0), max2(e, F[j]));
        }
    }
    free(E); free(F);
    return 0;
}

/* ------------------------------------------------------------------ linear space */

/* Row by row: one row of H, one of F, one scalar E; first strict maximum in row-major order. */
int orc_sw_linear(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const orc_scoring* sc,
                  int64_t* score, int64_t* end_a, int64_t* end_b) {
    if (bad_args(a, m, b, n, sc)) return -1;
    int64_t* H = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    int64_t* F = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!H || !F) { free(H); free(F); return -1; }
    for (int64_t j = 0; j <= n; j++) { H[j] = 0; F[j] = ORC_NEG; }
    int64_t best = 0, bi = -1, bj = -1;
    for (int64_t i = 1; i <= m; i++) {
        int64_t diag = H[0];  /* H(i-1, 0) */
        int64_t e = ORC_NEG;
        H[0] = 0;
        for (int64_t j = 1; j <= n; j++) {
            e = max2(e - sc->gap_extend, H[j - 1] - sc->gap_open);          /* H[j-1] = H(i, j-1) */
            F[j] = max2(F[j] - sc->gap_extend, H[j] - sc->gap_open);        /* H[j]   = H(i-1, j) */
            int64_t h = max2(max2(diag + sub_score(a[i - 1], b[j - 1], sc), 0), max2(e, F[j]));
            diag = H[j];
            H[j] = h;
            if (h > best) { best = h; bi = i - 1; bj = j - 1; }
        }
    }
    *score = best; *end_a = bi; *end_b = bj;
    free(H); free(F);
    return 0;
}

/* ------------------------------------------------------------------ linear space, several threads */

/*
 * The row-by-row recurrence above, spread over threads as a pipeline of row
 * stripes (stripe s holds rows s*h+1 .. s*h+h).  Thread t runs stripes t,
 * t + T, t + 2T, ... in that order.  A stripe walks the columns in chunks; it
 * starts a chunk once the stripe above has published its bottom row (H and F)
 * up to the chunk's last column.  Bottom rows go to a ring of K row buffers;
 * before writing buffer s mod K a stripe waits until the stripe that read the
 * buffer's previous contents (stripe s - K + 1) has finished.  A stripe only
 * ever waits on older stripes, so the oldest unfinished one always runs.
 *
 * Every cell is computed by the formulas of orc_sw_linear (or, anchored, of
 * orc_sw_start); the order in which cells are visited changes, so the cell
 * holding the answer is chosen by comparing (row, column) explicitly.
 *
 *   local    (orc_sw_linear_mt): zero borders and floor; S = max H, the
 *            endpoint is the lexicographically smallest cell holding S.
 *   anchored (orc_sw_start_mt):  orc_sw_start's reverse pass on reversed
 *            copies of the prefixes; the start is the lexicographically
 *            smallest reversed cell holding S.
 */
typedef struct {
    const uint8_t *a, *b;
    int64_t m, n;
    const orc_scoring* sc;
    int anchored;          /* 0: local; 1: anchored global recurrence */
    int64_t target;        /* anchored: the value searched for */
    int64_t h, chunk;      /* rows per stripe, columns per chunk */
    int64_t nstripes, K;
    int T;
    int64_t* ringH;        /* K rows of n + 1 values each */
    int64_t* ringF;
    _Atomic int64_t* progress;  /* per stripe: last column of its bottom row published */
    int64_t *rbest, *ri, *rj;   /* per stripe: best value (local) and its cell; anchored: first hit */
    _Atomic int64_t hit_stripe; /* anchored: lowest stripe known to hold a cell equal to the target */
    int failed;
} mt_job;

typedef struct {
    mt_job* J;
    int t;
} mt_arg;

static void mt_wait(_Atomic int64_t* p, int64_t need) {
    while (atomic_load_explicit(p, memory_order_acquire) < need) sched_yield();
}

/* (i1, j1) before (i2, j2) in row-major order */
static int lex_less(int64_t i1, int64_t j1, int64_t i2, int64_t j2) {
    return i1 < i2 || (i1 == i2 && j1 < j2);
}

/* Row 0 of the matrix. */
static int64_t mt_top(const mt_job* J, int64_t j) {
    if (!J->anchored) return 0;
    return j == 0 ? 0 : ORC_NEG;
}

static void mt_stripe(mt_job* J, int64_t s, int64_t* Hc, int64_t* Fc, int64_t* Hl, int64_t* El) {
    const int64_t n = J->n, r0 = s * J->h;
    const int64_t r1 = r0 + J->h < J->m ? r0 + J->h : J->m;
    const orc_scoring* sc = J->sc;
    const int64_t ext = sc->gap_extend, open = sc->gap_open;
    const uint8_t *A = J->a, *B = J->b;
    const int anchored = J->anchored;
    const int64_t target = J->target;
    if (s >= J->K) mt_wait(&J->progress[s - J->K + 1], n);
    const int64_t* upH = s > 0 ? J->ringH + ((s - 1) % J->K) * (n + 1) : NULL;
    const int64_t* upF = s > 0 ? J->ringF + ((s - 1) % J->K) * (n + 1) : NULL;
    int64_t* outH = J->ringH + (s % J->K) * (n + 1);
    int64_t* outF = J->ringF + (s % J->K) * (n + 1);
    for (int64_t k = 0; k < r1 - r0; k++) {
        Hl[k] = J->anchored ? ORC_NEG : 0;  /* H(i, 0), i >= 1 */
        El[k] = ORC_NEG;                    /* E(i, 0) */
    }
    int64_t best = 0, bi = INT64_MAX, bj = INT64_MAX;
    for (int64_t c0 = 1; c0 <= n; c0 += J->chunk) {
        const int64_t c1 = c0 + J->chunk - 1 < n ? c0 + J->chunk - 1 : n;
        if (s > 0) mt_wait(&J->progress[s - 1], c1);
        if (anchored && atomic_load_explicit(&J->hit_stripe, memory_order_acquire) < s) {
            /* An earlier stripe holds a hit: every row here comes after it, so no cell of this
             * stripe can be the first one (the single-threaded pass stops at that row too).
             * Later stripes see the same hit and stop as well, so the partly written bottom
             * row is never read. */
            J->rbest[s] = 0; J->ri[s] = INT64_MAX; J->rj[s] = INT64_MAX;
            atomic_store_explicit(&J->progress[s], n, memory_order_release);
            return;
        }
        /* the row above the stripe over columns c0-1 .. c1, at index j - (c0 - 1) */
        for (int64_t j = c0 - 1; j <= c1; j++) {
            Hc[j - c0 + 1] = s > 0 ? upH[j] : mt_top(J, j);
            Fc[j - c0 + 1] = s > 0 ? upF[j] : ORC_NEG;
        }
        for (int64_t k = 0; k < r1 - r0; k++) {
            const int64_t i = r0 + k + 1;
            const uint8_t ai = A[i - 1];
            int64_t diag = Hc[0];  /* H(i-1, c0-1) */
            int64_t e = El[k];     /* E(i, c0-1) */
            Hc[0] = Hl[k];         /* H(i, c0-1) */
            for (int64_t j = c0; j <= c1; j++) {
                const int64_t x = j - c0 + 1;
                e = max2(e - ext, Hc[x - 1] - open);       /* Hc[x-1] = H(i, j-1) */
                Fc[x] = max2(Fc[x] - ext, Hc[x] - open);   /* Hc[x]   = H(i-1, j) */
                int64_t hv = max2(diag + sub_score(ai, B[j - 1], sc), max2(e, Fc[x]));
                if (!anchored) hv = max2(hv, 0);
                diag = Hc[x];
                Hc[x] = hv;
                if (anchored) {
                    if (hv == target && lex_less(i - 1, j - 1, bi, bj)) { bi = i - 1; bj = j - 1; }
                } else if (hv > 0 && (hv > best || (hv == best && lex_less(i - 1, j - 1, bi, bj)))) {
                    best = hv; bi = i - 1; bj = j - 1;
                }
            }
            Hl[k] = Hc[c1 - c0 + 1];
            El[k] = e;
        }
        /* Hc, Fc now hold the stripe's bottom row */
        if (c0 == 1) { outH[0] = J->anchored ? ORC_NEG : 0; outF[0] = ORC_NEG; }
        for (int64_t j = c0; j <= c1; j++) { outH[j] = Hc[j - c0 + 1]; outF[j] = Fc[j - c0 + 1]; }
        atomic_store_explicit(&J->progress[s], c1, memory_order_release);
    }
    J->rbest[s] = best;
    J->ri[s] = bi;
    J->rj[s] = bj;
    if (anchored && bi != INT64_MAX) {
        int64_t cur = atomic_load(&J->hit_stripe);
        while (s < cur && !atomic_compare_exchange_weak(&J->hit_stripe, &cur, s)) {
        }
    }
}

static void* mt_thread(void* p) {
    mt_arg* A = (mt_arg*)p;
    mt_job* J = A->J;
    int64_t* Hc = (int64_t*)malloc((size_t)(J->chunk + 1) * sizeof(int64_t));
    int64_t* Fc = (int64_t*)malloc((size_t)(J->chunk + 1) * sizeof(int64_t));
    int64_t* Hl = (int64_t*)malloc((size_t)J->h * sizeof(int64_t));
    int64_t* El = (int64_t*)malloc((size_t)J->h * sizeof(int64_t));
    if (!Hc || !Fc || !Hl || !El) {
        /* cannot run: abort the whole job (every waiter sees a finished stripe) */
        J->failed = 1;
        for (int64_t s = A->t; s < J->nstripes; s += J->T) atomic_store(&J->progress[s], J->n);
    } else {
        for (int64_t s = A->t; s < J->nstripes; s += J->T) mt_stripe(J, s, Hc, Fc, Hl, El);
    }
    free(Hc); free(Fc); free(Hl); free(El);
    return NULL;
}

/* Runs the job on J->T threads; per-stripe results in rbest / ri / rj. */
static int mt_run(mt_job* J) {
    J->nstripes = (J->m + J->h - 1) / J->h;
    J->K = 2 * (int64_t)J->T;
    if (J->K < 2) J->K = 2;
    J->failed = 0;
    const size_t row = (size_t)(J->n + 1);
    J->ringH = (int64_t*)malloc((size_t)J->K * row * sizeof(int64_t));
    J->ringF = (int64_t*)malloc((size_t)J->K * row * sizeof(int64_t));
    J->progress = (_Atomic int64_t*)malloc((size_t)J->nstripes * sizeof(_Atomic int64_t));
    J->rbest = (int64_t*)malloc((size_t)J->nstripes * sizeof(int64_t));
    J->ri = (int64_t*)malloc((size_t)J->nstripes * sizeof(int64_t));
    J->rj = (int64_t*)malloc((size_t)J->nstripes * sizeof(int64_t));
    pthread_t* th = (pthread_t*)malloc((size_t)J->T * sizeof(pthread_t));
    mt_arg* args = (mt_arg*)malloc((size_t)J->T * sizeof(mt_arg));
    int rc = -1;
    if (J->ringH && J->ringF && J->progress && J->rbest && J->ri && J->rj && th && args) {
        for (int64_t s = 0; s < J->nstripes; s++) atomic_init(&J->progress[s], 0);
        atomic_init(&J->hit_stripe, INT64_MAX);
        int started = 0;
        for (int t = 0; t < J->T; t++) {
            args[t].J = J;
            args[t].t = t;
            if (pthread_create(&th[t], NULL, mt_thread, &args[t]) != 0) break;
            started++;
        }
        if (started < J->T) {
            /* the stripes of threads that did not start are marked finished so that
             * no waiter blocks; the job reports failure */
            J->failed = 1;
            for (int t = started; t < J->T; t++)
                for (int64_t s = t; s < J->nstripes; s += J->T) atomic_store(&J->progress[s], J->n);
        }
        for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
        rc = J->failed ? -1 : 0;
    }
    free(J->ringH); free(J->ringF); free((void*)J->progress); free(th); free(args);
    if (rc) { free(J->rbest); free(J->ri); free(J->rj); }
    return rc;
}

/* orc_sw_linear on `threads` threads; stripe_rows / chunk_cols 0 = 512 / 16384. */
int orc_sw_linear_mt(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const orc_scoring* sc,
                     int threads, int64_t stripe_rows, int64_t chunk_cols,
                     int64_t* score, int64_t* end_a, int64_t* end_b) {
    if (bad_args(a, m, b, n, sc) || threads < 1 || stripe_rows < 0 || chunk_cols < 0) return -1;
    *score = 0; *end_a = -1; *end_b = -1;
    if (m == 0 || n == 0) return 0;
    mt_job J;
    memset(&J, 0, sizeof J);
    J.a = a; J.b = b; J.m = m; J.n = n; J.sc = sc;
    J.anchored = 0;
    J.h = stripe_rows ? stripe_rows : 512;
    J.chunk = chunk_cols ? chunk_cols : 16384;
    J.T = threads;
    if (mt_run(&J)) return -1;
    int64_t best = 0, bi = INT64_MAX, bj = INT64_MAX;
    for (int64_t s = 0; s < J.nstripes; s++)
        if (J.rbest[s] > 0 && (J.rbest[s] > best || (J.rbest[s] == best && lex_less(J.ri[s], J.rj[s], bi, bj)))) {
            best = J.rbest[s]; bi = J.ri[s]; bj = J.rj[s];
        }
    free(J.rbest); free(J.ri); free(J.rj);
    if (best > 0) { *score = best; *end_a = bi; *end_b = bj; }
    return 0;
}

/* ------------------------------------------------------------------ start point */

/*
 * Anchored reverse pass: R over A^r = reverse(A[0..end_a]) and B^r = reverse(B[0..end_b]),
 *   R_H(0,0) = 0, every other border value -inf, no zero floor;
 * start = lexicographically smallest reversed cell (i,j) with R_H(i,j) = S,
 * reported as (end_a - i + 1, end_b - j + 1).
 */
int orc_sw_start(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const orc_scoring* sc,
                 int64_t score, int64_t end_a, int64_t end_b, int64_t* start_a, int64_t* start_b) {
    if (bad_args(a, m, b, n, sc)) return -1;
    if (score <= 0) { *start_a = -1; *start_b = -1; return 0; }
    if (end_a < 0 || end_a >= m || end_b < 0 || end_b >= n) return -1;
    int64_t rm = end_a + 1, rn = end_b + 1;
    int64_t* H = (int64_t*)malloc((size_t)(rn + 1) * sizeof(int64_t));
    int64_t* F = (int64_t*)malloc((size_t)(rn + 1) * sizeof(int64_t));
    if (!H || !F) { free(H); free(F); return -1; }
    H[0] = 0;
    for (int64_t j = 1; j <= rn; j++) H[j] = ORC_NEG;
    for (int64_t j = 0; j <= rn; j++) F[j] = ORC_NEG;
    int found = 0;
    for (int64_t i = 1; i <= rm && !found; i++) {
        int64_t diag = H[0], e = ORC_NEG;
        H[0] = ORC_NEG;
        uint8_t ai = a[end_a - (i - 1)];
        for (int64_t j = 1; j <= rn; j++) {
            e = max2(e - sc->gap_extend, H[j - 1] - sc->gap_open);
            F[j] = max2(F[j] - sc->gap_extend, H[j] - sc->gap_open);
            int64_t h = max2(diag + sub_score(ai, b[end_b - (j - 1)], sc), max2(e, F[j]));
            diag = H[j];
            H[j] = h;
            if (h == score) {
                *start_a = end_a - i + 1; *start_b = end_b - j + 1;
                found = 1;
                break;
            }
        }
    }
    free(H); free(F);
    return found ? 0 : -1;
}

/* orc_sw_start on `threads` threads (same result; stripe_rows / chunk_cols as above). */
int orc_sw_start_mt(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const orc_scoring* sc,
                    int64_t score, int64_t end_a, int64_t end_b, int threads, int64_t stripe_rows,
                    int64_t chunk_cols, int64_t* start_a, int64_t* start_b) {
    if (bad_args(a, m, b, n, sc) || threads < 1 || stripe_rows < 0 || chunk_cols < 0) return -1;
    if (score <= 0) { *start_a = -1; *start_b = -1; return 0; }
    if (end_a < 0 || end_a >= m || end_b < 0 || end_b >= n) return -1;
    const int64_t rm = end_a + 1, rn = end_b + 1;
    uint8_t* ra = (uint8_t*)malloc((size_t)rm);
    uint8_t* rb = (uint8_t*)malloc((size_t)rn);
    if (!ra || !rb) { free(ra); free(rb); return -1; }
    for (int64_t i = 0; i < rm; i++) ra[i] = a[end_a - i];
    for (int64_t j = 0; j < rn; j++) rb[j] = b[end_b - j];
    mt_job J;
    memset(&J, 0, sizeof J);
    J.a = ra; J.b = rb; J.m = rm; J.n = rn; J.sc = sc;
    J.anchored = 1;
    J.target = score;
    J.h = stripe_rows ? stripe_rows : 512;
    J.chunk = chunk_cols ? chunk_cols : 16384;
    J.T = threads;
    int rc = mt_run(&J);
    free(ra); free(rb);
    if (rc) return -1;
    int64_t bi = INT64_MAX, bj = INT64_MAX;
    for (int64_t s = 0; s < J.nstripes; s++)
        if (lex_less(J.ri[s], J.rj[s], bi, bj)) { bi = J.ri[s]; bj = J.rj[s]; }
    free(J.rbest); free(J.ri); free(J.rj);
    if (bi == INT64_MAX) return -1;
    *start_a = end_a - bi;
    *start_b = end_b - bj;
    return 0;
}

/* ------------------------------------------------------------------ Myers-Miller */

typedef struct {
    char* ops;
    int64_t* lens;
    int64_t n, cap;
    int failed;
} orc_cigar;

static void cig_push(orc_cigar* c, char op, int64_t k) {
    if (k <= 0 || c->failed) return;
    if (c->n > 0 && c->ops[c->n - 1] == op) { c->lens[c->n - 1] += k; return; }
    if (c->n == c->cap) {
        int64_t nc = c->cap ? 2 * c->cap : 64;
        char* o = (char*)realloc(c->ops, (size_t)nc);
        int64_t* l = (int64_t*)realloc(c->lens, (size_t)nc * sizeof(int64_t));
        if (!o || !l) { c->failed = 1; if (o) c->ops = o; if (l) c->lens = l; return; }
        c->ops = o; c->lens = l; c->cap = nc;
    }
    c->ops[c->n] = op; c->lens[c->n] = k; c->n++;
}

typedef struct {
    const orc_scoring* sc;
    int64_t g, h;                 /* gap of length k costs g + h*k */
    int64_t *CC, *DD, *RR, *SS;   /* scratch rows, length >= N+1 */
    uint8_t *ra, *rb;             /* scratch for reversed copies */
} mm_ctx;

static int64_t gapc(const mm_ctx* x, int64_t k) { return k > 0 ? x->g + x->h * k : 0; }

/*
 * Forward half: C(i,j) best path (0,0)->(i,j), D(i,j) best such path whose last
 * edge is vertical (a deletion of A_i).  A vertical run leaving (0,0) opens at
 * cost tb instead of g.  Writes C(M,.) to CC and D(M,.) to DD.
 */
static void mm_forward(const mm_ctx* x, const uint8_t* A, int64_t M, const uint8_t* B, int64_t N,
                       int64_t tb, int64_t* CC, int64_t* DD) {
    CC[0] = 0;
    DD[0] = ORC_NEG;
    for (int64_t j = 1; j <= N; j++) { CC[j] = -gapc(x, j); DD[j] = ORC_NEG; }
    for (int64_t i = 1; i <= M; i++) {
        int64_t diag = CC[0];
        CC[0] = -(tb + x->h * i);
        DD[0] = CC[0];
        int64_t ins = ORC_NEG;
        for (int64_t j = 1; j <= N; j++) {
            ins = max2(ins - x->h, CC[j - 1] - x->g - x->h);
            DD[j] = max2(DD[j] - x->h, CC[j] - x->g - x->h);
            int64_t c = max2(diag + sub_score(A[i - 1], B[j - 1], x->sc), max2(DD[j], ins));
            diag = CC[j];
            CC[j] = c;
        }
    }
}

static void mm_rec(mm_ctx* x, const uint8_t* A, int64_t M, const uint8_t* B, int64_t N,
                   int64_t tb, int64_t te, orc_cigar* out) {
    if (N == 0) { cig_push(out, 'D', M); return; }
    if (M == 0) { cig_push(out, 'I', N); return; }
    if (M == 1) {
        /* (i) delete A_0 and insert all of B as one run; the deletion sits next
         *     to the cheaper open side (first unless te < tb);
         * (ii) align A_0 with B_k (smallest k among the best), insert the rest. */
        int64_t open_i = tb < te ? tb : te;
        int64_t v_i = -(open_i + x->h) - gapc(x, N);
        int64_t v_ii = ORC_NEG, k_ii = -1;
        for (int64_t k = 1; k <= N; k++) {
            int64_t v = -gapc(x, k - 1) + sub_score(A[0], B[k - 1], x->sc) - gapc(x, N - k);
            if (v > v_ii) { v_ii = v; k_ii = k; }
        }
        if (v_ii >= v_i) {
            cig_push(out, 'I', k_ii - 1);
            cig_push(out, up(A[0]) == up(B[k_ii - 1]) ? '=' : 'X', 1);
            cig_push(out, 'I', N - k_ii);
        } else if (te < tb) {
            cig_push(out, 'I', N);
            cig_push(out, 'D', 1);
        } else {
            cig_push(out, 'D', 1);
            cig_push(out, 'I', N);
        }
        return;
    }
    int64_t mid = M / 2;
    /* forward over A[0..mid), reverse over A[mid..M) */
    mm_forward(x, A, mid, B, N, tb, x->CC, x->DD);
    int64_t rm = M - mid;
    for (int64_t i = 0; i < rm; i++) x->ra[i] = A[M - 1 - i];
    for (int64_t j = 0; j < N; j++) x->rb[j] = B[N - 1 - j];
    mm_forward(x, x->ra, rm, x->rb, N, te, x->RR, x->SS);
    /* RR/SS are indexed by reversed column: suffix starting at column j is index N-j */
    int64_t best = ORC_NEG, bj = -1;
    int type = 0;
    for (int64_t j = 0; j <= N; j++) {
        int64_t v1 = x->CC[j] + x->RR[N - j];
        if (v1 > best) { best = v1; bj = j; type = 1; }
        int64_t v2 = x->DD[j] + x->SS[N - j] + x->g;
        if (v2 > best) { best = v2; bj = j; type = 2; }
    }
    if (type == 1) {
        mm_rec(x, A, mid, B, bj, tb, x->g, out);
        mm_rec(x, A + mid, M - mid, B + bj, N - bj, x->g, te, out);
    } else {
        mm_rec(x, A, mid - 1, B, bj, tb, 0, out);
        cig_push(out, 'D', 2);
        mm_rec(x, A + mid + 1, M - mid - 1, B + bj, N - bj, 0, te, out);
    }
}

/* Writes the run-length CIGAR of the canonical alignment of A[0..M) x B[0..N) into buf. */
int orc_mm_align(const uint8_t* A, int64_t M, const uint8_t* B, int64_t N, const orc_scoring* sc,
                 int64_t tb, int64_t te, char* buf, int64_t cap, int64_t* out_len) {
    if (bad_args(A, M, B, N, sc) || !buf || cap <= 0) return -1;
    mm_ctx x;
    x.sc = sc;
    x.g = (int64_t)sc->gap_open - sc->gap_extend;
    x.h = sc->gap_extend;
    int64_t W = N + 1;
    x.CC = (int64_t*)malloc((size_t)W * sizeof(int64_t));
    x.DD = (int64_t*)malloc((size_t)W * sizeof(int64_t));
    x.RR = (int64_t*)malloc((size_t)W * sizeof(int64_t));
    x.SS = (int64_t*)malloc((size_t)W * sizeof(int64_t));
    x.ra = (uint8_t*)malloc((size_t)(M + 1));
    x.rb = (uint8_t*)malloc((size_t)(N + 1));
    orc_cigar c = {0};
    int rc = -1;
    if (x.CC && x.DD && x.RR && x.SS && x.ra && x.rb) {
        if (tb < 0) tb = x.g;
        if (te < 0) te = x.g;
        mm_rec(&x, A, M, B, N, tb, te, &c);
        if (!c.failed) {
            int64_t pos = 0;
            rc = 0;
            for (int64_t k = 0; k < c.n; k++) {
                char tmp[32];
                int64_t v = c.lens[k];
                int t = 0;
                do { tmp[t++] = (char)('0' + v % 10); v /= 10; } while (v);
                if (pos + t + 1 >= cap) { rc = -2; break; }
                while (t) buf[pos++] = tmp[--t];
                buf[pos++] = c.ops[k];
            }
            buf[pos < cap ? pos : cap - 1] = 0;
            *out_len = pos;
        }
    }
    free(x.CC); free(x.DD); free(x.RR); free(x.SS); free(x.ra); free(x.rb);
    free(c.ops); free(c.lens);
    return rc;
}

/* Best global score of A x B with the tb/te convention above (for tests). */
int orc_global_score(const uint8_t* A, int64_t M, const uint8_t* B, int64_t N, const orc_scoring* sc,
                     int64_t tb, int64_t te, int64_t* out) {
    if (bad_args(A, M, B, N, sc)) return -1;
    mm_ctx x;
    x.sc = sc;
    x.g = (int64_t)sc->gap_open - sc->gap_extend;
    x.h = sc->gap_extend;
    if (N == 0) { *out = M ? -((tb < te ? tb : te) + x.h * M) : 0; return 0; }
    int64_t* CC = (int64_t*)malloc((size_t)(N + 1) * sizeof(int64_t));
    int64_t* DD = (int64_t*)malloc((size_t)(N + 1) * sizeof(int64_t));
    if (!CC || !DD) { free(CC); free(DD); return -1; }
    (void)te;
    mm_forward(&x, A, M, B, N, tb, CC, DD);
    /* a trailing deletion run ending at (M,N) opens at te instead of g */
    int64_t v = CC[N];
    if (M > 0) v = max2(v, DD[N] + x.g - te);
    *out = v;
    free(CC); free(DD);
    return 0;
}
