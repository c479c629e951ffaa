// sw_internal.h -- types shared by the host runtime and the gfx950 kernels
// of libswalign.  Not part of the public ABI (see include/swalign.h).
#pragma once

#include <stdint.h>
#include "swalign.h"

namespace sw {

// Residue code used for rows below the query end and columns past the
// reference end (and, before the sweep reaches them, columns left of 0).
// Its substitution score is -1 against everything, so a padded cell can
// never reach the best score of its pair (see sw_sweep.h).
constexpr int kPad = 31;
constexpr int kMatDim = 32;                    // LDS matrix is 32 x 32 int8
constexpr int kMatBytes = kMatDim * kMatDim;   // per scheme
// After the matrices, per scheme and reference residue b: the column word
// of the small-alphabet path, bytes M[a][b] + o for a = 0..3 (see sw_sweep.h).
constexpr int kColWordsBytes = SW_MAX_SCHEMES * kMatDim * 4;
// Then the pair table of one scheme (the "pair-table" sweep, sw_sweep.h):
// for residues x, y of two consecutive query rows and reference residue b,
// the 16-bit entry [(x * D + y) * D + b] holds the bytes M[x][b] + o (low)
// and M[y][b] + o (high), where D = alphabet + 1 and code D - 1 (= alphabet)
// pads rows past the query end and columns outside the reference: its
// bytes are 0, a score of -o.
constexpr int kPtabMaxDim = 25;                          // alphabets of up to 24 residues
constexpr int kPtabBytes = (kPtabMaxDim * kPtabMaxDim * kPtabMaxDim * 2 + 15) / 16 * 16;
constexpr int kPtabOffset = SW_MAX_SCHEMES * kMatBytes + kColWordsBytes;
constexpr int kSchemeBytes = kPtabOffset + kPtabBytes;
constexpr int kBlock = 256;                    // 4 wavefronts per workgroup
// Reference tile of the sweeps, in steps: kChunk by default; the 16- and
// 32-lane packed shapes are also compiled for kChunkNarrow (fewer prefetch
// registers per lane, more tile boundaries).
constexpr int kChunk = 128;
constexpr int kChunkNarrow = 64;
constexpr int kWavesPerBlock = kBlock / 64;

// ---- planning: bins, length buckets, work items ----------------------------
// A bin is one compiled sweep shape (precision, lanes per group W, rows per
// lane R).  Pairs are bucketed by (bin, reference length) with one integer
// key so a counting sort on the device groups pairs of one bin with the longest
// references first; consecutive pairs of a bin then form wave work items.
constexpr int kMaxBins = 80;
constexpr int kMBuckets = 1024;                        // length buckets per bin
constexpr int kTrivialKey = kMaxBins * kMBuckets;      // empty / invalid pairs
constexpr int kHistSize = kTrivialKey + 1;

// Reference length -> bucket within one half of a bin's key range,
// monotone: exact below 256, then 32 buckets per octave (width <= 1/32 of
// the length) up to 65535.
constexpr int kMHalf = kMBuckets / 2;
__host__ __device__ inline int m_bucket(int m) {
    if (m < 256) return m;
    const int lg = 31 - __builtin_clz((unsigned)m);          // 8..15
    const int frac = (m >> (lg - 5)) & 31;
    int b = 256 + (lg - 8) * 32 + frac;
    return b < kMHalf ? b : kMHalf - 1;
}

// Most shapes one family kernel serves (one lane width, a run of rows per
// lane).
constexpr int kFamilyMax = 12;

struct BinInfo {
    uint8_t prec;     // 16 = two pairs per lane group packed in int16 halves, 32 = int32
    uint8_t R;        // query rows per lane
    uint16_t W;       // lanes per group: 16, 32, 64, or 256 (a workgroup's four wavefronts)
    uint16_t ppw;     // pairs per work item
    uint8_t col;      // 1 = the shape has a column-word kernel (small alphabets)
    uint8_t ptab;     // 1 = the shape has a pair-table kernel
};

// Pairs per work item of a shape: a wavefront's groups (times two packed
// pairs at 16 bits), or for a cooperative group the two pairs of one
// workgroup.  Work items per workgroup: its four wavefronts, or one.
__host__ __device__ inline int pairs_per_item(int prec, int W) {
    return (W <= 64 ? 64 / W : 1) * (prec == 16 ? 2 : 1);
}
__host__ __device__ inline int items_per_block(int W) { return W <= 64 ? kWavesPerBlock : 1; }

// One work item: pairs order[first .. first+count) of one bin.
struct WorkItem {
    int32_t first;
    uint16_t count;
    uint8_t bin;
    uint8_t pad;
};

// Layout of the per-pass planning metadata array (int32).
// Within a bin, items [first, split) hold only pairs of column-path schemes
// and go to the shape's column-word kernel; [split, next bin's first) hold
// only the other pairs and go to its table-lookup (or pair-table) kernel
// (split == first for shapes without a column kernel).  Each of the two has
// its own queue head.
enum : int {
    kMetaBinFirst = 0,                                // [kMaxBins + 1] first sorted position of each bin
    kMetaItemFirst = kMetaBinFirst + kMaxBins + 1,    // [kMaxBins + 1] first item of each bin
    kMetaItemSplit = kMetaItemFirst + kMaxBins + 1,   // [kMaxBins] first table-lookup item of each bin
    kMetaHeads = kMetaItemSplit + kMaxBins,           // [kMaxBins] queue head of each bin's table-lookup items
    kMetaColHeads = kMetaHeads + kMaxBins,            // [kMaxBins] and of its column-word items
    kMetaBinCol = kMetaColHeads + kMaxBins,           // [kMaxBins] column-path pairs of each bin
    kMetaSize = kMetaBinCol + kMaxBins,
};

// Layout of the 64-bit statistics counters of a call (cleared at its start).
enum : int {
    kCtrFwdCells = 0,
    kCtrRevCells = 1,
    kCtrI32Pairs = 2,
    kCtrTraceCells = 3,                      // cells of the path boxes (alignment paths)
    kCtrBinCells = 4,                        // [2 * kMaxBins] cells per (pass, bin)
    kCtrBinPairs = kCtrBinCells + 2 * kMaxBins,   // [2 * kMaxBins] pairs per (pass, bin)
    kCtrBinColCells = kCtrBinPairs + 2 * kMaxBins,   // [2 * kMaxBins] cells of column-path pairs
    kCtrBinColPairs = kCtrBinColCells + 2 * kMaxBins,   // [2 * kMaxBins] column-path pairs
    kCtrTraceBinCells = kCtrBinColPairs + 2 * kMaxBins,   // [kMaxBins] box cells per path-sweep bin
    kCtrTraceBinPairs = kCtrTraceBinCells + kMaxBins,      // [kMaxBins] pairs per path-sweep bin
    kNumCounters = kCtrTraceBinPairs + kMaxBins,
};

// Arguments shared by every sweep launch.
struct KParams {
    const uint8_t* queries;
    const int64_t* q_beg;        // query i is queries[q_beg[i] .. q_end[i])
    const int64_t* q_end;
    const uint8_t* refs;
    const int64_t* r_beg;        // reference i is refs[r_beg[i] .. r_end[i])
    const int64_t* r_end;
    const uint8_t* scheme_id;    // nullable
    const int32_t* order;        // pair ids grouped by bin, longest references first
    const WorkItem* items;
    int32_t* meta;               // planning metadata (item ranges, queue heads)
    sw_result* out;
    int32_t* flags;              // kFlag* error flags
    const int8_t* mats;          // [SW_MAX_SCHEMES][32][32], [s][b][a] = M_s[a][b]
    int32_t alphabet[SW_MAX_SCHEMES];
    int32_t gap_open[SW_MAX_SCHEMES];
    int32_t gap_extend[SW_MAX_SCHEMES];
    int32_t col_ok[SW_MAX_SCHEMES];   // scheme can take the small-alphabet column path
    int32_t max_score[SW_MAX_SCHEMES];   // largest substitution score (at least 1)
    int32_t validate;
    int32_t reverse;             // 0 = forward sweep, 1 = reverse sweep
    int32_t lo_idx, hi_idx;      // meta[lo_idx] .. meta[hi_idx] is this launch's item range
    int32_t head_idx;            // meta[head_idx] is this launch's queue head
    const int32_t* n_dev;        // device copy of the number of pairs in the batch
    int32_t n_pairs;             // pair capacity the grids are sized for (>= *n_dev)
    int32_t max_items;           // capacity of the items array (bound for every item index)
    int32_t ptab_sid;            // scheme of the pair table (mats + kPtabOffset), or -1
    int32_t ptab_dim;            // its D = alphabet + 1
    int32_t qprof;               // 1: the forward pass may use the query profile of queries[0 .. qprof_n)
    int32_t qprof_n;
    int8_t fam_bins[kFamilyMax];   // family launch: member k's bin, or -1 (not launched)
};

enum : int32_t {
    kFlagBadResidue = 0,
    kFlagReverseMismatch = 1,
    kFlagBadOffsets = 2,
    kFlagBadScheme = 3,
    kFlagTooLong = 4,
    kFlagInternal = 5,           // a planning or work-item invariant did not hold
    kFlagPathRoom = 6,           // an alignment path needs more runs than its output room
    kNumFlags = 8,
};

// Packed int16 path: values are stored plus kI16Bias so that they are
// positive normal half-precision bit patterns (<= 0x7BFF); a pair takes the
// path when min(n, m) * max_score <= kI16Limit and m <= kI16MaxRef.
constexpr int kI16Bias = 1024;
constexpr int kI16Limit = 0x7BFF - kI16Bias - 127;
constexpr int kI16MaxRef = 32000;

// Classification inputs: lut[sel * kLutRows + (n-1)/16] gives the bin of a
// pair with query length n, where sel = 0 for the packed int16 path and 1
// for int32; a pair takes int16 when min(n, m) * max_score[s] <= i16_limit.
constexpr int kLutRows = SW_MAX_QUERY / 16;
struct ClassifyArgs {
    int32_t max_score[SW_MAX_SCHEMES];
    int32_t col_ok[SW_MAX_SCHEMES];
    int32_t i16_limit;      // negative disables the int16 path
    int32_t n_schemes;
    int32_t n_bins;
    int32_t max_query;      // 0, or the caller's bound on query lengths (longer: kFlagTooLong)
};

}  // namespace sw

#include <hip/hip_runtime_api.h>

namespace sw {

// A compiled queue kernel: it aligns the work items [meta[lo_idx],
// meta[hi_idx]) of one bin shape.
using QueueFn = void (*)(KParams);

struct ShapeDesc { int prec, W, R; };

// Score sources of a shape's kernels: table lookups (any scheme), column
// words (small alphabets), the pair table (one scheme per call) and the
// query profile (the forward pass of a database search).
enum : int { kVarTable = 0, kVarCol = 1, kVarPtab = 2, kVarQprof = 3, kNumVars = 4 };

// The kernel of a compiled shape for one score source, with the default or
// the narrow reference tile (nullptr when the shape has no such variant).
QueueFn shape_kernel(int prec, int W, int R, bool reverse, int var = kVarTable, bool narrow = false);
// The family that serves shape (prec, W, R) with the default tile, or null:
// `rows[0..n)` are its members' rows per lane, largest first (the order of
// KParams::fam_bins), and k[var][reverse] its kernels (kVarTable, kVarCol,
// kVarPtab; null where there is none).
struct FamilyEntry { int prec, W, n; int rows[kFamilyMax]; QueueFn k[3][2]; int waves[3]; int tile[3]; };
const FamilyEntry* shape_family(int prec, int W, int R);
const ShapeDesc* compiled_shapes(int* n);

hipError_t launch_reset(int32_t* p, int n, hipStream_t s);
// Start of an alignment call: small[0..n_small) = 0 (flags and counters) and
// *n_dev = n_pairs.
hipError_t launch_call_start(int32_t* small, int n_small, int32_t* n_dev, int32_t n_pairs, hipStream_t s);
// beg[0..n) = 0, end[0..n) = len (the query spans of a database search)
hipError_t launch_fill_span(int64_t* beg, int64_t* end, int64_t n, int64_t len, hipStream_t s);
// The planning launches are sized for `cap` pairs; the kernels take the
// batch size from device memory (P.n_dev / n_dev), so a captured graph can be
// replayed for any batch of at most `cap` pairs.
hipError_t launch_classify(const KParams& P, const ClassifyArgs& C, const int8_t* lut, const BinInfo* bins,
                           int64_t cap, int32_t* keys, int32_t* hist,
                           unsigned long long* counters, hipStream_t s);
hipError_t launch_plan(const BinInfo* bins, int n_bins, int32_t* hist, int32_t* meta,
                       hipStream_t s);
// The same plan for a score pass, one workgroup per bin, from the pass's
// per-bin pair counters that launch_classify accumulates.
hipError_t launch_plan_bins(const BinInfo* bins, int n_bins, int32_t* hist, int32_t* meta,
                            const unsigned long long* counters, int reverse, hipStream_t s);
hipError_t launch_scatter(const int32_t* keys, const int32_t* n_dev, int64_t cap, int32_t* hist,
                          int32_t* order, hipStream_t s);
hipError_t launch_items(const int32_t* meta, const BinInfo* bins, int n_bins, const int32_t* n_dev,
                        int64_t cap, WorkItem* items, hipStream_t s);

// ---- alignment paths (sw_trace.hip) ----------------------------------------
// The path of a pair is recovered in its result box a[q_start..q_end] x
// b[r_start..r_end]: a sweep of the box writes 4 bits per cell (the
// traceback choices) into a device record, and a walk from the box's last
// cell reads them back.  Records of a batch are laid out back to back in pair
// order (rec_off, an exclusive scan of their sizes) and produced in chunks:
// chunk c holds the pairs whose record starts in [c * chunk_bytes,
// (c + 1) * chunk_bytes), at offset rec_off - c * chunk_bytes of the workspace.
struct TraceArgs {
    uint8_t* ws;                 // workspace of the current chunk
    const int64_t* rec_off;      // [n_pairs + 1] record byte offsets (the last = total)
    int64_t chunk_bytes;
    int64_t ws_bytes;            // workspace capacity (>= chunk_bytes + the largest record)
    int32_t chunk;
    int32_t n_bins;
    int32_t i16_limit;           // pairs with S <= i16_limit take the packed int16 path sweep
    const int8_t* lut;           // [2 * kLutRows] path-sweep bin per (int16 / int32, 16-row bucket of box rows)
    const BinInfo* bins;         // path-sweep bins
};

// Path-sweep shapes (precision 16: two pairs per W-lane group; 32: one;
// R a multiple of 4).
using TraceFn = void (*)(KParams, TraceArgs);
const ShapeDesc* trace_shapes(int* n);
TraceFn trace_kernel(int prec, int W, int R, bool col = false);
// The box-sweep family of packed int16 shape (prec, W, R), or null: its
// members' rows per lane, largest first, and its kernels (table lookups,
// column words).
struct TraceFamily { int prec, W, n; int rows[kFamilyMax]; TraceFn fn, col; };
const TraceFamily* trace_family(int prec, int W, int R);
// Records are written in blocks of kStage sweep steps.
constexpr int kStage = 8;
// Record bytes of a box of m columns on shape (W, R): m + W - 1 sweep steps
// rounded up to whole blocks, each step W lanes x R rows x 4 bits.
__host__ __device__ inline int64_t trace_record_bytes(int W, int R, int64_t m) {
    const int64_t steps = (m + W - 1 + kStage - 1) / kStage * kStage;
    return steps * (int64_t)W * R / 2;
}
// The largest record any pair can need (64 lanes x 32 rows, the longest reference).
constexpr int64_t kMaxRecordBytes = (int64_t)(SW_MAX_REF + 63 + kStage - 1) / kStage * kStage * 64 * 32 / 2;

hipError_t launch_trace_sizes(const KParams& P, const TraceArgs& T, int64_t cap, int64_t* rec_off,
                              int64_t* block_sums, unsigned long long* counters, hipStream_t s);
// Planning of one chunk; in chunk 0 it also sets path_len = 0 for pairs
// without an alignment.
hipError_t launch_trace_classify(const KParams& P, const TraceArgs& T, int64_t cap, int32_t* keys,
                                 int32_t* hist, unsigned long long* counters, int32_t* path_len, hipStream_t s);
// Walks of the pairs of one path-sweep bin (after the bin's sweep).
hipError_t launch_trace_walk(const KParams& P, const TraceArgs& T, int bin, int blocks, int active,
                             const int64_t* path_off, uint32_t* path, int32_t* path_len, hipStream_t s);
// Blocks of the size scan for `cap` pairs (the length of block_sums minus one).
int64_t trace_scan_blocks(int64_t cap);

}  // namespace sw
