/*
 * sw_oracle.c -- scalar CPU oracle for batched affine-gap Smith-Waterman.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never calls it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * What it computes, for one pair a[0..n-1] (query, rows) and b[0..m-1]
 * (reference, columns), with substitution matrix M (row = query residue,
 * column = reference residue) and gap penalties o (open) and e (extend), a gap
 * of length k costing o + (k-1)e:
 *
 *   Forward pass (the scoring matrix of Section II-B-1 / Fig. 2(a), with the
 *   single linear gap penalty of the worked example generalised to an affine
 *   one, which is the E state that the ADEPT-V1 listing of Fig. 9 carries):
 *     H[i][0] = H[0][j] = 0,  E[i][0] = F[0][j] = -inf
 *     E[i][j] = max(E[i][j-1] - e, H[i][j-1] - o)      gap along the row
 *     F[i][j] = max(F[i-1][j] - e, H[i-1][j] - o)      gap down the column
 *     H[i][j] = max(0, H[i-1][j-1] + M[a_i][b_j], E[i][j], F[i][j])
 *   S = max H.  The end (q_end, r_end) is the first cell in row-major order
 *   that holds S (smallest row, then smallest column), 0-based.
 *
 *   Reverse pass (replaces the traceback of Fig. 2(c), which follows the
 *   highest scores back from the maximum until a zero): the same recurrence
 *   on a' = a[q_end], a[q_end-1], ..., a[0] and b' = b[r_end], ..., b[0].
 *   The first cell (p, q) in row-major order of that matrix holding S gives
 *   q_start = q_end - p, r_start = r_end - q (p, q 0-based).  This is the
 *   latest start of any S-scoring alignment that ends at (q_end, r_end),
 *   i.e. the one a traceback reaches when it stops at the first zero.
 *
 *   If S == 0 (including empty sequences) every coordinate is -1.
 *
 * The arithmetic is done in int64 so that no input within the documented
 * limits can overflow.  Memory is O(m) per pair (one previous row).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef struct {
    const int8_t* matrix;   /* alphabet x alphabet, row-major, row = query residue */
    int32_t alphabet;
    int32_t gap_open;       /* positive cost of a length-1 gap */
    int32_t gap_extend;     /* positive cost of each further gap position */
} oracle_scheme;

typedef struct {
    int32_t score, q_start, q_end, r_start, r_end;
} oracle_result;

#define ORACLE_NEG_INF (-((int64_t)1 << 50))

static int64_t max2(int64_t x, int64_t y) { return x > y ? x : y; }

/*
 * Fill the Gotoh matrices row by row.  If `target` < 0, return the maximum
 * over all cells and the first cell in row-major order that reaches it.  If
 * `target` >= 0, return the first cell in row-major order whose H equals
 * `target` (the maximum is still returned in *best).
 */
static void gotoh_scan(const uint8_t* a, int64_t n, const uint8_t* b, int64_t m,
                       const oracle_scheme* sc, int64_t target,
                       int64_t* best, int64_t* bi, int64_t* bj,
                       int64_t* Hprev, int64_t* Hcur, int64_t* F)
{
    const int64_t o = sc->gap_open, e = sc->gap_extend;
    const int A = sc->alphabet;
    int64_t j;
    *best = 0; *bi = -1; *bj = -1;
    int found = 0;
    for (j = 0; j <= m; ++j) { Hprev[j] = 0; F[j] = ORACLE_NEG_INF; }
    for (int64_t i = 1; i <= n; ++i) {
        int64_t E = ORACLE_NEG_INF;
        Hcur[0] = 0;
        for (j = 1; j <= m; ++j) {
            E = max2(E - e, Hcur[j - 1] - o);
            F[j] = max2(F[j] - e, Hprev[j] - o);
            int64_t h = Hprev[j - 1] + sc->matrix[a[i - 1] * A + b[j - 1]];
            h = max2(h, E);
            h = max2(h, F[j]);
            h = max2(h, 0);
            Hcur[j] = h;
            if (h > *best) {
                *best = h;
                if (target < 0) { *bi = i - 1; *bj = j - 1; }
            }
            if (target >= 0 && !found && h == target) {
                found = 1; *bi = i - 1; *bj = j - 1;
            }
        }
        int64_t* t = Hprev; Hprev = Hcur; Hcur = t;
    }
}

/* Align one pair.  Returns 0, or -1 on allocation failure / bad input. */
int oracle_align_pair(const uint8_t* a, int64_t n, const uint8_t* b, int64_t m,
                      const oracle_scheme* sc, oracle_result* out)
{
    out->score = 0; out->q_start = out->q_end = out->r_start = out->r_end = -1;
    if (n <= 0 || m <= 0) return 0;
    for (int64_t i = 0; i < n; ++i) if (a[i] >= sc->alphabet) return -1;
    for (int64_t j = 0; j < m; ++j) if (b[j] >= sc->alphabet) return -1;

    int64_t* buf = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)(m + 1));
    uint8_t* ra = (uint8_t*)malloc((size_t)n);
    uint8_t* rb = (uint8_t*)malloc((size_t)m);
    if (!buf || !ra || !rb) { free(buf); free(ra); free(rb); return -1; }
    int64_t* Hprev = buf;
    int64_t* Hcur = buf + (m + 1);
    int64_t* F = buf + 2 * (m + 1);

    int64_t S, qe, re;
    gotoh_scan(a, n, b, m, sc, -1, &S, &qe, &re, Hprev, Hcur, F);
    if (S > 0) {
        /* reversed prefixes a[0..qe], b[0..re] */
        for (int64_t p = 0; p <= qe; ++p) ra[p] = a[qe - p];
        for (int64_t q = 0; q <= re; ++q) rb[q] = b[re - q];
        int64_t S2, p, q;
        gotoh_scan(ra, qe + 1, rb, re + 1, sc, S, &S2, &p, &q, Hprev, Hcur, F);
        if (S2 != S || p < 0) { free(buf); free(ra); free(rb); return -1; }
        out->score = (int32_t)S;
        out->q_end = (int32_t)qe;
        out->r_end = (int32_t)re;
        out->q_start = (int32_t)(qe - p);
        out->r_start = (int32_t)(re - q);
    }
    free(buf); free(ra); free(rb);
    return 0;
}

typedef struct {
    const uint8_t* queries; const int64_t* q_off;
    const uint8_t* refs; const int64_t* r_off;
    const uint8_t* scheme_id; int64_t n_pairs;
    const oracle_scheme* schemes; int n_schemes;
    const int64_t* index;   /* optional subset of pairs to run (NULL = all) */
    int64_t n_index;
    oracle_result* out;
    int64_t next;           /* shared work counter */
    int error;
    pthread_mutex_t lock;
} oracle_job;

static void* oracle_worker(void* arg)
{
    oracle_job* J = (oracle_job*)arg;
    const int64_t total = J->index ? J->n_index : J->n_pairs;
    for (;;) {
        int64_t k;
        pthread_mutex_lock(&J->lock);
        k = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (k >= total) break;
        int64_t i = J->index ? J->index[k] : k;
        int sid = J->scheme_id ? J->scheme_id[i] : 0;
        if (i < 0 || i >= J->n_pairs || sid >= J->n_schemes) { J->error = 1; continue; }
        const int64_t qa = J->q_off[i], qb = J->q_off[i + 1];
        const int64_t ra = J->r_off[i], rb = J->r_off[i + 1];
        if (oracle_align_pair(J->queries + qa, qb - qa, J->refs + ra, rb - ra,
                              &J->schemes[sid], &J->out[k]) != 0)
            J->error = 1;
    }
    return NULL;
}

/*
 * Align pairs on `n_threads` host threads.  If `index` is non-NULL only the
 * pairs index[0..n_index-1] are aligned and out[k] receives pair index[k];
 * otherwise out[i] receives pair i.  Returns 0, or -1 if any pair failed.
 */
int oracle_align_batch(const uint8_t* queries, const int64_t* q_off,
                       const uint8_t* refs, const int64_t* r_off,
                       const uint8_t* scheme_id, int64_t n_pairs,
                       const oracle_scheme* schemes, int n_schemes,
                       const int64_t* index, int64_t n_index,
                       oracle_result* out, int n_threads)
{
    oracle_job J;
    J.queries = queries; J.q_off = q_off; J.refs = refs; J.r_off = r_off;
    J.scheme_id = scheme_id; J.n_pairs = n_pairs;
    J.schemes = schemes; J.n_schemes = n_schemes;
    J.index = index; J.n_index = n_index;
    J.out = out; J.next = 0; J.error = 0;
    pthread_mutex_init(&J.lock, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 0; t < n_threads; ++t) {
        if (pthread_create(&th[t], NULL, oracle_worker, &J) != 0) break;
        ++started;
    }
    if (started == 0) oracle_worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    return J.error ? -1 : 0;
}

/* Full score matrix H (n+1) x (m+1), row-major, for small-case tests. */
int oracle_score_matrix(const uint8_t* a, int64_t n, const uint8_t* b, int64_t m,
                        const oracle_scheme* sc, int64_t* H)
{
    const int64_t o = sc->gap_open, e = sc->gap_extend;
    const int A = sc->alphabet;
    int64_t* E = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1) * (size_t)(m + 1));
    int64_t* F = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1) * (size_t)(m + 1));
    if (!E || !F) { free(E); free(F); return -1; }
    const int64_t W = m + 1;
    for (int64_t i = 0; i <= n; ++i)
        for (int64_t j = 0; j <= m; ++j) {
            if (i == 0 || j == 0) {
                H[i * W + j] = 0; E[i * W + j] = ORACLE_NEG_INF; F[i * W + j] = ORACLE_NEG_INF;
                continue;
            }
            E[i * W + j] = max2(E[i * W + j - 1] - e, H[i * W + j - 1] - o);
            F[i * W + j] = max2(F[(i - 1) * W + j] - e, H[(i - 1) * W + j] - o);
            int64_t h = H[(i - 1) * W + j - 1] + sc->matrix[a[i - 1] * A + b[j - 1]];
            h = max2(h, E[i * W + j]);
            h = max2(h, F[i * W + j]);
            H[i * W + j] = max2(h, 0);
        }
    free(E); free(F);
    return 0;
}

/*
 * Alignment path (the traceback of Fig. 2(c)), as run-length columns.
 *
 * Given the result of oracle_align_pair, the path is recovered inside the
 * box a[q_start..q_end] x b[r_start..r_end]: the Gotoh matrices of the box
 * alone are filled (same recurrences, local, H = 0 / E = F = -inf on the
 * box's top row and left column) and followed back from the box's last cell,
 * whose H equals S, until H reaches 0.  Every S-scoring alignment that ends at
 * (q_end, r_end) and lies in the box starts at the box corner (a later start
 * would contradict the latest-start rule), so the walk must stop exactly
 * there; anything else is reported as an error.
 *
 * Among equally scoring paths the walk takes, at each cell, the first valid
 * choice of:
 *   in H:  the diagonal (H == H[i-1][j-1] + M), then F (a query residue over
 *          a gap), then E (a reference residue over a gap);
 *   in F:  opening the gap here (F == H[i-1][j] - o), then extending it;
 *   in E:  opening the gap here (E == H[i][j-1] - o), then extending it.
 * Read from the end, this is the smallest sequence of choices in that order.
 *
 * Columns are emitted as runs (length << 4) | op with the SAM/BAM operation
 * codes: 7 '=' (equal residue codes), 8 'X' (other substitution), 1 'I'
 * (query residue over a gap), 2 'D' (reference residue over a gap), from the
 * first column of the alignment to the last.  S == 0 gives no runs.
 * Returns 0, or -1 on inconsistent input, allocation failure or when more
 * than `cap` runs would be needed.
 */
enum { ORACLE_OP_I = 1, ORACLE_OP_D = 2, ORACLE_OP_EQ = 7, ORACLE_OP_X = 8 };

int oracle_cigar_pair(const uint8_t* a, int64_t n, const uint8_t* b, int64_t m,
                      const oracle_scheme* sc, const oracle_result* res,
                      uint32_t* runs, int64_t cap, int64_t* n_runs)
{
    *n_runs = 0;
    if (res->score == 0) return 0;
    const int64_t qs = res->q_start, qe = res->q_end, rs = res->r_start, re = res->r_end;
    if (res->score < 0 || qs < 0 || qs > qe || qe >= n || rs < 0 || rs > re || re >= m) return -1;
    const int64_t o = sc->gap_open, e = sc->gap_extend;
    const int A = sc->alphabet;
    const int64_t nb = qe - qs + 1, mb = re - rs + 1, W = mb + 1;
    const uint8_t* x = a + qs;
    const uint8_t* y = b + rs;
    for (int64_t i = 0; i < nb; ++i) if (x[i] >= A) return -1;
    for (int64_t j = 0; j < mb; ++j) if (y[j] >= A) return -1;
    const size_t cells = (size_t)(nb + 1) * (size_t)(mb + 1);
    int64_t* H = (int64_t*)malloc(sizeof(int64_t) * cells);
    int64_t* E = (int64_t*)malloc(sizeof(int64_t) * cells);
    int64_t* F = (int64_t*)malloc(sizeof(int64_t) * cells);
    char* ops = (char*)malloc((size_t)(nb + mb));
    int rc = -1;
    if (!H || !E || !F || !ops) goto done;
    for (int64_t i = 0; i <= nb; ++i)
        for (int64_t j = 0; j <= mb; ++j) {
            if (i == 0 || j == 0) {
                H[i * W + j] = 0; E[i * W + j] = ORACLE_NEG_INF; F[i * W + j] = ORACLE_NEG_INF;
                continue;
            }
            E[i * W + j] = max2(E[i * W + j - 1] - e, H[i * W + j - 1] - o);
            F[i * W + j] = max2(F[(i - 1) * W + j] - e, H[(i - 1) * W + j] - o);
            int64_t h = H[(i - 1) * W + j - 1] + sc->matrix[x[i - 1] * A + y[j - 1]];
            h = max2(h, E[i * W + j]);
            h = max2(h, F[i * W + j]);
            H[i * W + j] = max2(h, 0);
        }
    if (H[nb * W + mb] != res->score) goto done;
    {
        int64_t i = nb, j = mb, k = 0;
        char state = 'H';
        for (;;) {
            if (state == 'H') {
                const int64_t h = H[i * W + j];
                if (h == 0) break;
                if (h == H[(i - 1) * W + j - 1] + sc->matrix[x[i - 1] * A + y[j - 1]]) {
                    ops[k++] = x[i - 1] == y[j - 1] ? '=' : 'X';
                    --i; --j;
                } else if (h == F[i * W + j]) {
                    state = 'F';
                } else if (h == E[i * W + j]) {
                    state = 'E';
                } else {
                    goto done;
                }
            } else if (state == 'F') {
                ops[k++] = 'I';
                if (i < 2 && F[i * W + j] != H[(i - 1) * W + j] - o) goto done;
                state = F[i * W + j] == H[(i - 1) * W + j] - o ? 'H' : 'F';
                if (state == 'F' && F[i * W + j] != F[(i - 1) * W + j] - e) goto done;
                --i;
            } else {
                ops[k++] = 'D';
                if (j < 2 && E[i * W + j] != H[i * W + j - 1] - o) goto done;
                state = E[i * W + j] == H[i * W + j - 1] - o ? 'H' : 'E';
                if (state == 'E' && E[i * W + j] != E[i * W + j - 1] - e) goto done;
                --j;
            }
            if (k > nb + mb) goto done;
        }
        if (i != 0 || j != 0) goto done;
        /* ops[] runs from the last column back to the first */
        int64_t r = 0;
        for (int64_t p = k - 1; p >= 0;) {
            int64_t q = p;
            while (q > 0 && ops[q - 1] == ops[p]) --q;
            const uint32_t len = (uint32_t)(p - q + 1);
            const uint32_t code = ops[p] == '=' ? ORACLE_OP_EQ : ops[p] == 'X' ? ORACLE_OP_X
                                : ops[p] == 'I' ? ORACLE_OP_I : ORACLE_OP_D;
            if (r >= cap) goto done;
            runs[r++] = (len << 4) | code;
            p = q - 1;
        }
        *n_runs = r;
        rc = 0;
    }
done:
    free(H); free(E); free(F); free(ops);
    return rc;
}

typedef struct {
    const uint8_t* queries; const int64_t* q_off;
    const uint8_t* refs; const int64_t* r_off;
    const uint8_t* scheme_id; int64_t n_pairs;
    const oracle_scheme* schemes; int n_schemes;
    const int64_t* index; int64_t n_index;
    const oracle_result* res;     /* res[k]: result of the k-th pair run */
    const int64_t* run_off;       /* runs of the k-th pair go to runs[run_off[k] .. run_off[k+1]) */
    uint32_t* runs;
    int64_t* n_runs;
    int64_t next;
    int error;
    pthread_mutex_t lock;
} oracle_cigar_job;

static void* oracle_cigar_worker(void* arg)
{
    oracle_cigar_job* J = (oracle_cigar_job*)arg;
    const int64_t total = J->index ? J->n_index : J->n_pairs;
    for (;;) {
        int64_t k;
        pthread_mutex_lock(&J->lock);
        k = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (k >= total) break;
        int64_t i = J->index ? J->index[k] : k;
        int sid = J->scheme_id ? J->scheme_id[i] : 0;
        if (i < 0 || i >= J->n_pairs || sid >= J->n_schemes) { J->error = 1; continue; }
        const int64_t qa = J->q_off[i], qb = J->q_off[i + 1];
        const int64_t ra = J->r_off[i], rb = J->r_off[i + 1];
        if (oracle_cigar_pair(J->queries + qa, qb - qa, J->refs + ra, rb - ra, &J->schemes[sid],
                              &J->res[k], J->runs + J->run_off[k], J->run_off[k + 1] - J->run_off[k],
                              &J->n_runs[k]) != 0)
            J->error = 1;
    }
    return NULL;
}

/*
 * Alignment paths of a batch (or of the subset `index`, as in
 * oracle_align_batch), given the results `res` of those pairs in the same
 * order.  Returns 0, or -1 if any pair failed.
 */
int oracle_cigar_batch(const uint8_t* queries, const int64_t* q_off,
                       const uint8_t* refs, const int64_t* r_off,
                       const uint8_t* scheme_id, int64_t n_pairs,
                       const oracle_scheme* schemes, int n_schemes,
                       const int64_t* index, int64_t n_index,
                       const oracle_result* res, const int64_t* run_off,
                       uint32_t* runs, int64_t* n_runs, int n_threads)
{
    oracle_cigar_job J;
    J.queries = queries; J.q_off = q_off; J.refs = refs; J.r_off = r_off;
    J.scheme_id = scheme_id; J.n_pairs = n_pairs;
    J.schemes = schemes; J.n_schemes = n_schemes;
    J.index = index; J.n_index = n_index;
    J.res = res; J.run_off = run_off; J.runs = runs; J.n_runs = n_runs;
    J.next = 0; J.error = 0;
    pthread_mutex_init(&J.lock, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 0; t < n_threads; ++t) {
        if (pthread_create(&th[t], NULL, oracle_cigar_worker, &J) != 0) break;
        ++started;
    }
    if (started == 0) oracle_cigar_worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    return J.error ? -1 : 0;
}
