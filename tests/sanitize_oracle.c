/*
 * Drives every entry point of the C oracle (oracle/gotoh.c) on seeded random
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py compiles and runs it).  The point is memory
 * and arithmetic safety of the oracle; as a side check its modes must agree
 * with each other (full matrix, row by row, row stripes on threads, the
 * anchored start pass single- and multi-threaded, Myers-Miller against the
 * global score).  Exit status 0: clean; 1: a disagreement (a sanitizer report
 * ends the process with its own status).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t match, mismatch, gap_open, gap_extend;
    const int8_t* matrix;
    const int8_t* letter_class;
    int32_t size, pad_;
} orc_scoring;

int orc_sw_full(const uint8_t*, int64_t, const uint8_t*, int64_t, const orc_scoring*, int64_t*, int64_t*, int64_t*);
int orc_sw_linear(const uint8_t*, int64_t, const uint8_t*, int64_t, const orc_scoring*, int64_t*, int64_t*, int64_t*);
int orc_sw_linear_mt(const uint8_t*, int64_t, const uint8_t*, int64_t, const orc_scoring*, int, int64_t, int64_t,
                     int64_t*, int64_t*, int64_t*);
int orc_sw_matrix(const uint8_t*, int64_t, const uint8_t*, int64_t, const orc_scoring*, int64_t*);
int orc_sw_start(const uint8_t*, int64_t, const uint8_t*, int64_t, const orc_scoring*, int64_t, int64_t, int64_t,
                 int64_t*, int64_t*);
int orc_sw_start_mt(const uint8_t*, int64_t, const uint8_t*, int64_t, const orc_scoring*, int64_t, int64_t, int64_t,
                    int, int64_t, int64_t, int64_t*, int64_t*);
int orc_mm_align(const uint8_t*, int64_t, const uint8_t*, int64_t, const orc_scoring*, int64_t, int64_t, char*,
                 int64_t, int64_t*);
int orc_global_score(const uint8_t*, int64_t, const uint8_t*, int64_t, const orc_scoring*, int64_t, int64_t,
                     int64_t*);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint32_t next(void) {  /* xorshift64* */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (uint32_t)((state * 0x2545F4914F6CDD1Dull) >> 32);
}

static void letters(uint8_t* s, int64_t n, const char* alphabet, int k) {
    for (int64_t i = 0; i < n; i++) s[i] = (uint8_t)alphabet[next() % (uint32_t)k];
}

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "disagreement at line %d, case %d\n", __LINE__, t); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main(void) {
    static const char amino[] = "ARNDCQEGHILKMFPSTWYV";
    int8_t matrix[20 * 20], cls[256];
    memset(cls, -1, sizeof cls);
    for (int i = 0; i < 20; i++) {
        cls[(uint8_t)amino[i]] = (int8_t)i;
        cls[(uint8_t)amino[i] + 32] = (int8_t)i;
        for (int j = 0; j < 20; j++) matrix[i * 20 + j] = (int8_t)(i == j ? 4 + (int)(next() % 8) : (int)(next() % 7) - 4);
    }
    const orc_scoring dna = {1, 3, 5, 2, NULL, NULL, 0, 0};
    const orc_scoring prot = {0, 0, 11, 1, matrix, cls, 20, 0};
    for (int t = 0; t < 400; t++) {
        const int protein = t & 1;
        const orc_scoring* sc = protein ? &prot : &dna;
        const char* alphabet = protein ? amino : "ACGTacgt";
        const int k = protein ? 20 : 8;
        const int64_t m = next() % 90, n = next() % 90;
        uint8_t* a = (uint8_t*)malloc((size_t)m + 1);
        uint8_t* b = (uint8_t*)malloc((size_t)n + 1);
        letters(a, m, alphabet, k);
        letters(b, n, alphabet, k);
        int64_t s1, i1, j1, s2, i2, j2, s3, i3, j3;
        CHECK(orc_sw_full(a, m, b, n, sc, &s1, &i1, &j1) == 0);
        CHECK(orc_sw_linear(a, m, b, n, sc, &s2, &i2, &j2) == 0);
        CHECK(orc_sw_linear_mt(a, m, b, n, sc, 1 + t % 4, 1 + t % 7, 1 + t % 5, &s3, &i3, &j3) == 0);
        CHECK(s1 == s2 && i1 == i2 && j1 == j2 && s1 == s3 && i1 == i3 && j1 == j3);
        int64_t* H = (int64_t*)malloc((size_t)((m + 1) * (n + 1)) * sizeof(int64_t));
        CHECK(orc_sw_matrix(a, m, b, n, sc, H) == 0);
        free(H);
        if (s1 > 0) {
            int64_t sa, sb, sa2, sb2, g, len;
            CHECK(orc_sw_start(a, m, b, n, sc, s1, i1, j1, &sa, &sb) == 0);
            CHECK(orc_sw_start_mt(a, m, b, n, sc, s1, i1, j1, 1 + t % 3, 1 + t % 6, 1 + t % 4, &sa2, &sb2) == 0);
            CHECK(sa == sa2 && sb == sb2);
            const int64_t M = i1 - sa + 1, N = j1 - sb + 1;
            const int64_t gg = (int64_t)sc->gap_open - sc->gap_extend;
            CHECK(orc_global_score(a + sa, M, b + sb, N, sc, gg, gg, &g) == 0);
            CHECK(g == s1);
            char cigar[4096];
            CHECK(orc_mm_align(a + sa, M, b + sb, N, sc, -1, -1, cigar, sizeof cigar, &len) == 0);
            CHECK(len > 0 && (int64_t)strlen(cigar) == len);
        }
        /* tb/te variants of the reconstruction on the whole of a x b */
        {
            char cigar[4096];
            int64_t len;
            const int64_t gg = (int64_t)sc->gap_open - sc->gap_extend;
            CHECK(orc_mm_align(a, m, b, n, sc, t % 3 ? gg : 0, t % 5 ? gg : 0, cigar, sizeof cigar, &len) == 0);
        }
        free(a);
        free(b);
    }
    /* invalid arguments are refused, not read */
    int64_t s, i, j;
    const uint8_t bad[] = "ACGB";
    int t = -1;
    CHECK(orc_sw_linear(bad, 4, bad, 4, &prot, &s, &i, &j) == -1);
    CHECK(orc_sw_linear(NULL, 3, bad, 4, &dna, &s, &i, &j) == -1);
    puts("oracle sanitizer run: clean");
    return 0;
}
