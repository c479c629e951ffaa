/*
 * swalign.h -- C ABI of the batched affine-gap Smith-Waterman library
 * (libswalign.so, built for AMD Instinct MI355X / gfx950).
 *
 * What is computed (Section II-B-1 and Fig. 2 of arXiv 2208.12350, with the
 * gap penalty generalised from the worked example's single linear cost to an
 * affine open/extend pair, i.e. the E state of the ADEPT-V1 listing in
 * Fig. 9):  for every pair (query a, reference b) the local-alignment score
 * matrix H of the Gotoh recurrences
 *
 *     E[i][j] = max(E[i][j-1] - e, H[i][j-1] - o)
 *     F[i][j] = max(F[i-1][j] - e, H[i-1][j] - o)
 *     H[i][j] = max(0, H[i-1][j-1] + M[a_i][b_j], E[i][j], F[i][j])
 *
 * with zero first row/column, is swept once forward; its maximum S and the
 * first cell holding S in row-major order give the end coordinates.  A second
 * sweep of the same recurrence over the reversed prefixes a[q_end..0],
 * b[r_end..0] stands in for the traceback of Fig. 2(c): its first cell
 * holding S gives the start, which is the latest start of any S-scoring
 * alignment that ends at (q_end, r_end).  A gap of length k costs
 * o + (k-1)e.  Coordinates are 0-based and inclusive; a pair whose best
 * score is 0 (including an empty query or reference) reports all -1.
 *
 * Threading: a handle may be used by one host thread at a time.
 * Streams: `stream` is a hipStream_t passed as void*; NULL means the
 * device's null stream.  All functions return one of the SW_* codes below
 * (never throw); sw_last_error() gives a human-readable reason.
 */
#ifndef SWALIGN_H
#define SWALIGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SW_OK          0
#define SW_PENDING     1    /* sw_poll: request not finished yet */
#define SW_EINVAL     -1    /* bad argument or invalid input data */
#define SW_ENOMEM     -2    /* device or host allocation failed / budget exceeded */
#define SW_ETOOLONG   -3    /* a sequence exceeds SW_MAX_QUERY / SW_MAX_REF */
#define SW_EDEVICE    -4    /* a HIP runtime call failed */
#define SW_EINTERNAL  -5    /* an internal consistency check failed */

/* ---- limits ------------------------------------------------------------ */
#define SW_MAX_QUERY     2048    /* query (row) length handled in one sweep */
#define SW_MAX_REF      60000    /* reference (column) length */
#define SW_MAX_ALPHABET    31    /* residue codes 0..alphabet-1 */
#define SW_MAX_SCHEMES      4
#define SW_NOALLOC_MAX_PAIRS (1 << 20)   /* batch limit of sw_align_batch_noalloc */

/* One result per pair, in the caller's pair order. */
typedef struct {
    int32_t score;
    int32_t q_start, q_end;     /* query (row) coordinates, 0-based inclusive */
    int32_t r_start, r_end;     /* reference (column) coordinates */
} sw_result;

/* A scoring scheme.  `matrix` is a HOST pointer to alphabet*alphabet int8
 * scores, row-major, row = query residue, column = reference residue.
 * Gap costs are positive integers with gap_open >= gap_extend >= 0 and
 * gap_open >= 1. */
typedef struct {
    const int8_t* matrix;
    int32_t alphabet;
    int32_t gap_open;
    int32_t gap_extend;
} sw_scheme;

/* A batch of pairs.  Every pointer is a DEVICE pointer on the handle's
 * device, owned by the caller and left unmodified:
 *   queries   uint8 residue codes of all queries, concatenated
 *   q_off     int64[n_pairs+1], query i is queries[q_off[i] .. q_off[i+1])
 *   refs      uint8 residue codes of all references, concatenated
 *   r_off     int64[n_pairs+1]
 *   scheme_id uint8[n_pairs] index into the scheme array, or NULL (all 0)
 * Offsets must be non-decreasing; lengths may be zero. */
typedef struct {
    const uint8_t* queries;
    const int64_t* q_off;
    const uint8_t* refs;
    const int64_t* r_off;
    const uint8_t* scheme_id;
    int64_t n_pairs;
} sw_batch;

typedef struct sw_handle sw_handle;

/* Create a handle bound to HIP device `device`.  `tuning` is NULL (built-in
 * defaults) or a string of `key=value` pairs separated by ';' or ',': the
 * keys of sw_set_option, plus "route16" / "route32" whose value is a
 * routing table "WxR@rows_max/WxR@rows_max/..." (see sw_set_routing).
 * Returns NULL on failure (including a malformed tuning string). */
sw_handle* sw_create(int device, const char* tuning);

/* Release the handle and every device buffer it owns.  Waits for its work. */
void sw_destroy(sw_handle* h);

/* Reason for the last non-OK status returned on this handle. */
const char* sw_last_error(sw_handle* h);

/* Set a tuning or behaviour option (integer valued):
 *   "mode"      0 = one plain launch per length bin, 1 = persistent launch
 *               over a device work queue (default 1)
 *   "graph"     1 = capture the call into a hipGraph and replay it while
 *               the buffers, schemes and options stay the same (the batch
 *               size may change up to the capacity); default 1
 *   "validate"  1 = check residue codes (default 1); invalid residues make
 *               the call return SW_EINVAL (results of those pairs undefined)
 *   "precision" 0 = automatic routing (default): a pair runs on the packed
 *               int16 path when min(n, m) * (largest matrix score) <= 30592
 *               and m <= 32000, which bounds every intermediate value;
 *               otherwise on int32.
 *               32 = force every pair onto the int32 path
 *   "timing"    1 = record HIP events around the phases of each call on the
 *               caller's stream (read back with sw_last_timing);
 *               2 = also around every sweep kernel launch, with the
 *               launches serialised on the caller's stream (read back with
 *               sw_last_bin_stats).  Timing turns graph replay off.
 *   "capacity"  reserve workspace for this many pairs now (it otherwise
 *               grows to the largest batch seen).  Launch grids and captured
 *               graphs are sized for the capacity and read the batch size
 *               from device memory, so one graph serves every batch with the
 *               same buffers and at most that many pairs
 *   "colpath"   1 = pairs whose scheme has at most 4 residues (and whose
 *               scores plus gap_open fit a byte) read their substitution
 *               scores from per-column words instead of table lookups
 *               (default 1; 0 = always table lookups)
 *   "pairtable" 1 = when exactly one scheme of a call takes table lookups
 *               (alphabet of at most 24 residues, scores plus gap_open a
 *               byte, gap_open <= 1024), its packed int16 pairs read two
 *               rows' scores per load from a pair table (default 1);
 *               0 = byte-table lookups.  Read-only "pairtable_used": whether
 *               the last finished call used it
 *   "qprofile"  1 = the forward pass of sw_search profiles the query in LDS
 *               (scores of each lane's rows against every residue) when the
 *               scheme qualifies for the pair table (default 1); 0 = pair
 *               table.  Read-only "qprofile_used" as for "pairtable_used"
 *   "chunk"     reference steps staged per LDS tile by the 16- and 32-lane
 *               packed int16 kernels: 128 (default) or 64 (fewer prefetch
 *               registers per lane, twice as many tile boundaries)
 *   "streams"   1..8: persistent mode spreads the bins' kernels over this
 *               many streams forked from (and joined back into) the
 *               caller's stream (default 4; more than the process's
 *               hardware queues, GPU_MAX_HW_QUEUES, 4 by default, share them)
 *   "families"  1 (default) = persistent mode with the default tile launches,
 *               per pass and score source, one kernel for each family of
 *               compiled shapes (a lane width and a run of rows per lane)
 *               that takes the items of all its routed bins (when it has at
 *               least two); 0 = one launch per bin
 *   "max_query" 0 (default) or 1..SW_MAX_QUERY: the caller's bound on
 *               query lengths.  Persistent mode then launches no bin that
 *               only longer queries route to (each launch costs its stream
 *               time even when its bin is empty), and sw_align_cigar no
 *               path-sweep bin for taller boxes, nor its int32 bins when
 *               the bound times the best substitution score fits the packed
 *               range; a pair with a longer query makes the call return
 *               SW_ETOOLONG
 *   "cigar_workspace"  device bytes for the path records of sw_align_cigar
 *               (default half the device's memory, at least 32 GiB; the
 *               smallest accepted value is about 123 MB)
 * Returns SW_OK or SW_EINVAL for an unknown key / bad value. */
int sw_set_option(sw_handle* h, const char* key, int64_t value);
/* Read an option, or the read-only "captures" (graphs captured so far) and
 * "capture_refusals" (captures the runtime refused; those calls ran their
 * kernels without a graph). */
int sw_get_option(sw_handle* h, const char* key, int64_t* value);

/* Align every pair of `batch` and write out[i] (a DEVICE pointer to
 * n_pairs sw_result records) for pair i.  Work is enqueued on `stream`; the
 * call returns after it has completed (it is sw_submit followed by
 * sw_poll with wait = 1).
 * `schemes` is a HOST array of n_schemes (1..SW_MAX_SCHEMES) schemes.
 * Errors: SW_EINVAL (null pointer with n_pairs > 0, bad scheme, decreasing
 * offsets, scheme id out of range, residue >= alphabet), SW_ETOOLONG (a
 * query longer than SW_MAX_QUERY or reference longer than SW_MAX_REF),
 * SW_ENOMEM, SW_EDEVICE.  On error the contents of `out` are undefined. */
int sw_align_batch(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes,
                   int n_schemes, sw_result* out, void* stream);

/* Asynchronous form of sw_align_batch (the same computation, Section II-B-1
 * with the affine gap reading above): enqueue the whole call on `stream`
 * and return at once with *ticket identifying it.  Planning happens on the
 * device, so nothing waits for the GPU: input checks that need the data
 * (offsets, scheme ids, lengths, residue codes) are reported by sw_poll.
 * The caller keeps `batch`'s device buffers and `out` alive and unmodified
 * until sw_poll reports the ticket finished; `schemes` (host) is read
 * before sw_submit returns.  Calls of one handle run one after another on
 * the device, in submission order, whatever their streams (a call on
 * another stream than the previous one waits for it on the device), and
 * each result is what sw_align_batch would give for that batch alone.  Up
 * to 8 calls are in flight per handle; a ninth submit first waits for the
 * oldest (whose status sw_poll still reports).  A submit may also wait for
 * the calls in flight when it must replace what they use: a larger
 * workspace, a new routing table, or a captured graph evicted from the
 * handle's cache of 4.  Errors returned by sw_submit itself (nothing is
 * then enqueued and no ticket issued): SW_EINVAL for bad arguments that
 * the host can see (null pointers, bad schemes, the "timing" option set),
 * SW_ENOMEM, SW_EDEVICE. */
int sw_submit(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes, int n_schemes,
              sw_result* out, void* stream, uint64_t* ticket);

/* Status of a submitted call: with wait == 0, SW_PENDING while it runs;
 * otherwise (or once it has finished) its final status, as sw_align_batch
 * would have returned it (SW_OK, SW_EINVAL for invalid input data,
 * SW_ETOOLONG, SW_EINTERNAL), with the reason in sw_last_error.  Polling a
 * finished ticket forgets it; an unknown or already collected ticket is
 * SW_EINVAL.  The statistics calls below describe the last call that
 * finished.  Poll every ticket: finished statuses are kept until then. */
int sw_poll(sw_handle* h, uint64_t ticket, int wait);

/* For callers that cannot allocate device memory (code inside a tight
 * serving loop, harnesses that forbid hipMalloc): the same call as
 * sw_align_batch, with the same arguments, results and errors, except that
 * it allocates and frees nothing.  Its planning workspace (sort keys, pair
 * order and work items; 16 bytes per pair) is one static device array of
 * 16 MiB that each GPU the library runs on holds until the process ends;
 * the handle (created beforehand with sw_create, which does allocate) gives
 * everything else.  The call never captures or replays a graph; its kernels
 * are launched on `stream` and it returns after they have completed.
 * Limits: at most SW_NOALLOC_MAX_PAIRS pairs (more is SW_EINVAL, checked
 * before anything is launched).  Every call on one GPU, from any handle,
 * shares that GPU's array: calls that overlap in time on one GPU (from two
 * host threads, or on two streams) race and give undefined results. */
int sw_align_batch_noalloc(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes,
                           int n_schemes, sw_result* out, void* stream);

/* Same as sw_align_batch for pairs given by explicit spans instead of
 * prefix offsets: query i is queries[q_beg[i] .. q_end[i]) and reference i is
 * refs[r_beg[i] .. r_end[i]); spans may overlap and appear in any order, so
 * pairs can be drawn from a resident pool of sequences.  All pointers are
 * DEVICE pointers except `schemes`; errors as for sw_align_batch (an end
 * before its begin is SW_EINVAL). */
int sw_align_spans(sw_handle* h, const uint8_t* queries, const int64_t* q_beg, const int64_t* q_end,
                   const uint8_t* refs, const int64_t* r_beg, const int64_t* r_end,
                   const uint8_t* scheme_id, int64_t n_pairs, const sw_scheme* schemes, int n_schemes,
                   sw_result* out, void* stream);

/* Database search: align one query against every reference of a set, as
 * sw_align_batch would align the pairs (query, reference i) -- the use that
 * Sections I and VII give alignment in assembly pipelines, one read against
 * many candidate sequences; out[i] is the
 * result of reference i.  `query` (q_len residues), `refs` and `r_off`
 * (int64[n_refs+1], non-decreasing; reference i is refs[r_off[i] ..
 * r_off[i+1])) are DEVICE pointers owned by the caller; `scheme` is one HOST
 * scheme.  The query is stored once and every pair's span points at it; the
 * spans are kept on the device between calls with the same query length, so
 * repeated searches replay one captured graph.  When the scheme takes table
 * lookups (a large alphabet) the forward pass reads its scores from a query
 * profile that each workgroup builds in LDS: for every residue b, the
 * scores M[a_i][b] of each lane's query rows, read as whole dwords (option
 * "qprofile").  Errors as for sw_align_batch
 * (SW_ETOOLONG for q_len > SW_MAX_QUERY). */
int sw_search(sw_handle* h, const uint8_t* query, int64_t q_len, const uint8_t* refs, const int64_t* r_off,
              int64_t n_refs, const sw_scheme* scheme, sw_result* out, void* stream);

/* Statistics of the last alignment call on this handle that finished: number of
 * forward cells (sum of n*m), reverse cells (sum of (q_end+1)*(r_end+1) over
 * pairs with a positive score) and the number of pairs routed to the int32
 * path.  Any pointer may be NULL. */
int sw_last_stats(sw_handle* h, int64_t* fwd_cells, int64_t* rev_cells, int64_t* int32_pairs);

/* Device time in milliseconds of the phases of the last sw_align_batch call,
 * measured with HIP events on the caller's stream; all zero unless the
 * "timing" option is set.  plan = classification + sort + histogram copy,
 * forward / reverse = the forward and reverse sweeps (every launch of each).
 * Any pointer may be NULL. */
int sw_last_timing(sw_handle* h, float* plan_ms, float* forward_ms, float* reverse_ms);

/* Host wall time in milliseconds of the last call: from entry until all its
 * work was enqueued (argument checks, planning launches, sweep launches or
 * graph launch), and the wait for the device after that.  Always recorded;
 * any pointer may be NULL. */
int sw_last_host_timing(sw_handle* h, double* enqueue_ms, double* wait_ms);

/* ---- alignment paths (the traceback of Fig. 2(c)) ----------------------
 *
 * The path of a pair is recovered inside its result box a[q_start..q_end] x
 * b[r_start..r_end]: every alignment of score S that ends at (q_end, r_end)
 * within the box starts at (q_start, r_start), so it is a traceback of the
 * box's own Gotoh matrices from the box's last cell.  Among equally scoring
 * paths the traceback takes, at each cell and read from the end backwards,
 * the first valid choice of: a substitution column, then a query residue
 * over a gap, then a reference residue over a gap; inside a gap, opening it
 * here before extending it further back.
 *
 * A path is written as runs, uint32 (length << 4) | op, from the first
 * column of the alignment to the last, with the SAM/BAM operation codes: */
#define SW_OP_I   1   /* query residue over a gap (insertion to the reference) */
#define SW_OP_D   2   /* reference residue over a gap (deletion from the reference) */
#define SW_OP_EQ  7   /* substitution column, equal residue codes */
#define SW_OP_X   8   /* substitution column, different residue codes */

/* Align every pair of `batch` as sw_align_batch does (out[i] as there) and
 * write its path: pair i's runs go to cigar[cigar_off[i] ..
 * cigar_off[i+1]) and their number to cigar_len[i] (0 when the score is 0).
 * cigar_off (int64[n_pairs+1], non-decreasing), cigar (uint32) and
 * cigar_len (int32[n_pairs]) are DEVICE pointers owned by the caller; a room
 * of q_len + r_len runs per pair always suffices.  The paths are found by a
 * sweep of each box that stores 4 bits per cell in a device workspace (option
 * "cigar_workspace", default half the device's memory; batches whose boxes
 * need more are done in chunks), then a walk back per pair.  The workspace is
 * allocated to what the batch needs, up to that bound, and kept.  Synchronises `stream`; not captured in
 * a graph.  Errors: those of sw_align_batch; SW_EINVAL when a pair's room
 * is too small (its cigar_len is -1, the other pairs' paths are written);
 * SW_ENOMEM when the workspace cannot be allocated. */
int sw_align_cigar(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes, int n_schemes,
                   sw_result* out, const int64_t* cigar_off, uint32_t* cigar, int32_t* cigar_len,
                   void* stream);

/* Statistics of the last sw_align_cigar call: cells of the path boxes (sum
 * of (q_end-q_start+1)*(r_end-r_start+1)), bytes of path records, chunks,
 * and with the "timing" option (which serialises the launches) the device
 * milliseconds of the box sweeps and of the walks; the box sweeps of each
 * shape are also the entries of sw_last_bin_stats with pass 2 (packed
 * int16 shapes have a column-word kernel, used when every scheme of the
 * call has at most four residues whose scores plus the gap open cost fit a
 * byte, beside the table-lookup one; both write the same records).  Any
 * pointer may be NULL. */
int sw_last_cigar_stats(sw_handle* h, int64_t* box_cells, int64_t* record_bytes, int32_t* chunks,
                        float* sweep_ms, float* walk_ms);

/* ---- routing: which sweep shape aligns which query length -------------
 *
 * A sweep shape is (lanes, rows): a group of `lanes` lanes (16, 32 or 64)
 * shares one pair (two pairs packed per register at 16-bit precision), and
 * each lane holds `rows` consecutive query rows, so a shape covers queries of
 * up to lanes * rows residues in one sweep of m + lanes - 1 steps.
 *
 * sw_shapes lists the compiled shapes into HOST arrays of `capacity`
 * entries (*n_out = the number of shapes; SW_EINVAL if capacity is short). */
int sw_shapes(sw_handle* h, int32_t* precision, int32_t* lanes, int32_t* rows, int capacity, int* n_out);

/* Route queries of one precision (16 or 32) by length: entry k sends the
 * queries of rows_max[k-1]+1 .. rows_max[k] residues (rows_max[-1] = 0) to
 * shape (lanes[k], rows[k]).  rows_max must increase in steps that are
 * multiples of 16 and end at SW_MAX_QUERY; each shape must be compiled and
 * cover its rows (lanes * rows >= rows_max).  n == 0 restores the built-in
 * routing.  HOST arrays; SW_EINVAL on a malformed table (the routing is then
 * unchanged).  Results never depend on the routing, only speed does. */
int sw_set_routing(sw_handle* h, int precision, const int32_t* rows_max, const int32_t* lanes, const int32_t* rows,
                   int n);
/* The current routing of one precision, in the same form (merged runs). */
int sw_get_routing(sw_handle* h, int precision, int32_t* rows_max, int32_t* lanes, int32_t* rows, int capacity,
                   int* n_out);

/* The pairs of one bin of the last call: the pairs of one shape
 * (precision, lanes per pair group, query rows per lane) in one pass, and of
 * one score source (column words for small alphabets, or table lookups),
 * with the kernel launch that swept them.  A family launch (option
 * "families") sweeps several bins of one lane width with one kernel: those
 * bins share `launch` and `ms`, so per-launch figures group the entries by
 * (pass, launch). */
typedef struct sw_bin_stat {
    int32_t pass;        /* 0 forward, 1 reverse, 2 path boxes (sw_align_cigar) */
    int32_t precision;   /* 16 (two pairs packed per register) or 32 */
    int32_t lanes;       /* lanes that share one pair */
    int32_t rows;        /* query rows held by each lane */
    int64_t pairs;       /* pairs the bin held in this pass */
    int64_t cells;       /* DP cells of those pairs in this pass */
    float ms;            /* time of the launch that swept the bin (HIP events) with
                            "timing" = 2, else 0 */
    int32_t column;      /* 1 = the column-word kernel, 0 = the table-lookup kernel,
                            2 = the pair-table kernel, 3 = the query-profile kernel */
    int32_t tile;        /* reference steps per LDS tile of the kernel (option "chunk") */
    int32_t launch;      /* index of that launch within its pass (the last enqueued
                            call's; a replayed graph repeats its capture's), -1 if none */
    int32_t family_hi;   /* family launch: the largest and smallest rows per lane of */
    int32_t family_lo;   /* the family's shapes; 0 for a launch of one shape */
    int32_t family_waves;/* family launch: wavefronts per SIMD its kernel is compiled for */
} sw_bin_stat;

/* Per-launch statistics of the last call on this handle: writes up to
 * `capacity` entries (every kernel of every bin of the forward pass, then
 * of the reverse pass) into the HOST array `out` and their number into
 * *n_out.  Returns
 * SW_EINVAL (with *n_out set to the number needed) if capacity is too small. */
int sw_last_bin_stats(sw_handle* h, sw_bin_stat* out, int capacity, int* n_out);

/* ---- serving: continuous batching over a device-resident pool ----------
 *
 * The paper's alignment workload (Section II-B) arrives as independent
 * batches of pairs; these calls serve such batches as requests that come
 * and go while others run, each aligned exactly as sw_align_batch would
 * align it alone.  Unlike sw_submit, requests are HOST arrays: the server
 * owns the device copies (its pool), so it can admit requests by device
 * memory and free them itself.
 *
 * A server owns a device memory pool of `pool_bytes` (the admission budget),
 * `slots` worker streams (1..16) and a copy of the schemes.  Requests are
 * batches of pairs given as HOST arrays (same layout as sw_batch); submit
 * checks them, stages a copy (the caller may free its arrays on return) and
 * queues them.  An admission thread moves queued requests, first in first
 * out, into the pool as soon as it has room; each free slot then takes every
 * admitted request that fits `max_batch_pairs`, aligns them as one batch on
 * its own stream, hands each request its results and releases its memory.
 * Requests that arrive while others run are admitted and merged into the
 * next batch of the first slot to free up, so work from different requests
 * overlaps on the device.  Results are identical to aligning each request
 * alone.  Each slot holds two handles: merged batches of up to 8192 pairs
 * run with a routing of few bins (16x16 up to 256 rows, 32x16 up to 512,
 * cooperative 256x8 above), which shortens the critical path of small
 * batches; larger ones use the routing of `tuning` (or the built-in one).
 * Each handle's call is captured into a graph once, when the server is
 * created, and replayed for every batch.  A server may be driven from
 * several host threads. */
typedef struct sw_server sw_server;

/* Returns NULL on failure (bad scheme, no such device, allocation failure).
 * `schemes` is a host array, copied. */
sw_server* sw_server_create(int device, const sw_scheme* schemes, int n_schemes, int64_t pool_bytes,
                            int slots, int64_t max_batch_pairs, const char* tuning);

/* Stops the workers (after the batches already running) and frees the pool;
 * requests not yet completed are dropped. */
void sw_server_destroy(sw_server* s);
const char* sw_server_last_error(sw_server* s);

/* Queue a request.  Errors (the request is then not queued): SW_EINVAL (bad
 * offsets, residue outside its scheme's alphabet, scheme id out of range,
 * more pairs than max_batch_pairs), SW_ETOOLONG, SW_ENOMEM (the request alone
 * needs more than the whole pool).  On success *ticket identifies it. */
int sw_server_submit(sw_server* s, const uint8_t* queries, const int64_t* q_off, const uint8_t* refs,
                     const int64_t* r_off, const uint8_t* scheme_id, int64_t n_pairs, uint64_t* ticket);

/* Collect a request: SW_PENDING if not finished (and wait == 0); otherwise
 * its status, with n_pairs results copied to the HOST array `out` and the
 * time from the submit call's entry (host checks and staging included) to
 * the results being on the host in *latency_ms.  A collected ticket is
 * forgotten. */
int sw_server_poll(sw_server* s, uint64_t ticket, sw_result* out, int wait, double* latency_ms);

/* Peak pool bytes in use so far, pool capacity, requests completed, batches
 * launched and pairs aligned.  Any pointer may be NULL. */
int sw_server_stats(sw_server* s, int64_t* pool_peak_bytes, int64_t* pool_capacity, int64_t* requests_done,
                    int64_t* batches, int64_t* pairs_done);

/* Cumulative wall time in milliseconds the server spent admitting requests
 * (staging and copying them into the pool), aligning merged batches, and
 * fetching their results to the host.  Any pointer may be NULL. */
int sw_server_timing(sw_server* s, double* admit_ms, double* align_ms, double* fetch_ms);

#ifdef __cplusplus
}
#endif

#endif /* SWALIGN_H */
