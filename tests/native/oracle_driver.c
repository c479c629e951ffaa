/*
 * Host-only driver for running the oracle (oracle/sw_oracle.c) under the
 * address and undefined-behaviour sanitizers: random pairs of every small
 * length (empty included) under several schemes, through the batch entry
 * point on several threads, the single-pair entry point, the full score
 * matrix and the alignment paths.  Checks that the entry points agree with
 * each other and that every path consumes exactly its result box; prints
 * "oracle sanitize ok" on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { const int8_t* matrix; int32_t alphabet, gap_open, gap_extend; } oracle_scheme;
typedef struct { int32_t score, q_start, q_end, r_start, r_end; } oracle_result;

int oracle_align_pair(const uint8_t*, int64_t, const uint8_t*, int64_t, const oracle_scheme*, oracle_result*);
int oracle_align_batch(const uint8_t*, const int64_t*, const uint8_t*, const int64_t*, const uint8_t*, int64_t,
                       const oracle_scheme*, int, const int64_t*, int64_t, oracle_result*, int);
int oracle_score_matrix(const uint8_t*, int64_t, const uint8_t*, int64_t, const oracle_scheme*, int64_t*);
int oracle_cigar_pair(const uint8_t*, int64_t, const uint8_t*, int64_t, const oracle_scheme*,
                      const oracle_result*, uint32_t*, int64_t, int64_t*);
int oracle_cigar_batch(const uint8_t*, const int64_t*, const uint8_t*, const int64_t*, const uint8_t*, int64_t,
                       const oracle_scheme*, int, const int64_t*, int64_t, const oracle_result*, const int64_t*,
                       uint32_t*, int64_t*, int);

#define FAIL(...) do { printf("FAIL: " __VA_ARGS__); printf("\n"); return 1; } while (0)

static uint64_t rng_state = 2208123500ULL;
static uint32_t next_u32(void) {
    /* xorshift64* */
    rng_state ^= rng_state >> 12; rng_state ^= rng_state << 25; rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 2685821657736338717ULL) >> 32);
}
static int below(int n) { return (int)(next_u32() % (uint32_t)n); }

int main(void) {
    enum { P = 1500, NS = 3 };
    int8_t dna[16], prot[400], lin[9];
    for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) dna[a * 4 + b] = a == b ? 3 : -3;
    for (int a = 0; a < 20; ++a) for (int b = 0; b <= a; ++b) {
        const int v = a == b ? 4 + below(8) : -4 + below(8);
        prot[a * 20 + b] = prot[b * 20 + a] = (int8_t)v;
    }
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) lin[a * 3 + b] = (int8_t)(a == b ? 2 : -2 - a);
    oracle_scheme sc[NS] = {{dna, 4, 6, 1}, {prot, 20, 11, 1}, {lin, 3, 1, 1}};

    int64_t* q_off = calloc(P + 1, sizeof(int64_t));
    int64_t* r_off = calloc(P + 1, sizeof(int64_t));
    uint8_t* sid = malloc(P);
    for (int i = 0; i < P; ++i) {
        sid[i] = (uint8_t)below(NS);
        q_off[i + 1] = q_off[i] + (i % 97 == 0 ? 0 : below(40));
        r_off[i + 1] = r_off[i] + (i % 89 == 0 ? 0 : below(60));
    }
    uint8_t* q = malloc((size_t)q_off[P] + 1);
    uint8_t* r = malloc((size_t)r_off[P] + 1);
    for (int i = 0; i < P; ++i) {
        const int A = sc[sid[i]].alphabet;
        for (int64_t k = q_off[i]; k < q_off[i + 1]; ++k) q[k] = (uint8_t)below(A);
        for (int64_t k = r_off[i]; k < r_off[i + 1]; ++k) r[k] = (uint8_t)below(A);
        /* embed a copy of part of the query in the reference half of the time */
        const int64_t n = q_off[i + 1] - q_off[i], m = r_off[i + 1] - r_off[i];
        if (n > 0 && m >= n && below(2)) memcpy(r + r_off[i] + below((int)(m - n) + 1), q + q_off[i], (size_t)n);
    }
    oracle_result* res = malloc(P * sizeof(oracle_result));
    if (oracle_align_batch(q, q_off, r, r_off, sid, P, sc, NS, NULL, 0, res, 7) != 0) FAIL("align_batch");

    int64_t* run_off = calloc(P + 1, sizeof(int64_t));
    for (int i = 0; i < P; ++i) run_off[i + 1] = run_off[i] + (q_off[i + 1] - q_off[i]) + (r_off[i + 1] - r_off[i]);
    uint32_t* runs = malloc((size_t)(run_off[P] + 1) * sizeof(uint32_t));
    int64_t* n_runs = malloc(P * sizeof(int64_t));
    if (oracle_cigar_batch(q, q_off, r, r_off, sid, P, sc, NS, NULL, 0, res, run_off, runs, n_runs, 5) != 0)
        FAIL("cigar_batch");

    for (int i = 0; i < P; ++i) {
        const uint8_t* a = q + q_off[i];
        const uint8_t* b = r + r_off[i];
        const int64_t n = q_off[i + 1] - q_off[i], m = r_off[i + 1] - r_off[i];
        const oracle_scheme* s = &sc[sid[i]];
        oracle_result one;
        if (oracle_align_pair(a, n, b, m, s, &one) != 0) FAIL("align_pair %d", i);
        if (memcmp(&one, &res[i], sizeof(one)) != 0) FAIL("pair %d: batch and single-pair results differ", i);
        /* the score matrix's maximum is the score */
        int64_t* H = malloc(sizeof(int64_t) * (size_t)(n + 1) * (size_t)(m + 1));
        if (oracle_score_matrix(a, n, b, m, s, H) != 0) FAIL("score_matrix %d", i);
        int64_t mx = 0;
        for (int64_t k = 0; k < (n + 1) * (m + 1); ++k) mx = H[k] > mx ? H[k] : mx;
        free(H);
        if (mx != res[i].score) FAIL("pair %d: matrix maximum %lld, score %d", i, (long long)mx, res[i].score);
        /* the path (from the batch and from the single-pair call) covers the box exactly */
        uint32_t buf[128];
        int64_t k1 = -1;
        if (oracle_cigar_pair(a, n, b, m, s, &res[i], buf, 128, &k1) != 0) FAIL("cigar_pair %d", i);
        if (k1 != n_runs[i] || memcmp(buf, runs + run_off[i], (size_t)k1 * sizeof(uint32_t)) != 0)
            FAIL("pair %d: batch and single-pair paths differ", i);
        int64_t qa = 0, rb = 0;
        for (int64_t k = 0; k < k1; ++k) {
            const uint32_t op = buf[k] & 15u, len = buf[k] >> 4;
            if (op == 7 || op == 8) { qa += len; rb += len; }
            else if (op == 1) qa += len;
            else if (op == 2) rb += len;
            else FAIL("pair %d: op %u", i, op);
        }
        const int64_t bq = res[i].score > 0 ? res[i].q_end - res[i].q_start + 1 : 0;
        const int64_t br = res[i].score > 0 ? res[i].r_end - res[i].r_start + 1 : 0;
        if (qa != bq || rb != br) FAIL("pair %d: path spans %lldx%lld, box %lldx%lld", i, (long long)qa,
                                       (long long)rb, (long long)bq, (long long)br);
    }
    free(q); free(r); free(q_off); free(r_off); free(sid); free(res); free(run_off); free(runs); free(n_runs);
    printf("oracle sanitize ok\n");
    return 0;
}
