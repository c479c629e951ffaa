// sw_internal.h -- types shared by the host runtime and the gfx950 kernels
// of libswalign.  Not part of the public ABI (see include/swalign.h).
#pragma once

#include <stdint.h>
#include "swalign.h"

namespace sw {

// Residue code used for rows below the query end and columns past the
// reference end (and, before the sweep reaches them, columns left of 0).
// Its substitution score is -1 against everything, so a padded cell can
// never reach the best score of its pair (see the kernel header comment).
constexpr int kPad = 31;
constexpr int kMatDim = 32;                    // LDS matrix is 32 x 32 int8
constexpr int kMatBytes = kMatDim * kMatDim;   // per scheme
constexpr int kBlock = 256;                    // 4 wavefronts per workgroup
constexpr int kWavesPerBlock = kBlock / 64;

// Precision / geometry class of a length bin.
struct BinShape {
    int16_t prec;     // 32 = int32 lanes, 16 = two int16 pairs packed per lane
    int16_t W;        // lanes per pair group: 16 or 64
    int16_t R;        // query rows per lane
};

// Arguments shared by every alignment launch.
struct KParams {
    const uint8_t* queries;
    const int64_t* q_off;
    const uint8_t* refs;
    const int64_t* r_off;
    const uint8_t* scheme_id;    // nullable
    const int32_t* order;        // pair ids sorted by (bin, reference length desc)
    sw_result* out;
    int32_t* flags;              // [0] invalid residue, [1] reverse-pass mismatch
    const int8_t* mats;          // [SW_MAX_SCHEMES][32][32], [s][b][a] = M_s[a][b]
    int32_t alphabet[SW_MAX_SCHEMES];
    int32_t gap_open[SW_MAX_SCHEMES];
    int32_t gap_extend[SW_MAX_SCHEMES];
    int32_t validate;
};

// Per-pair classification written by the classify kernel.
enum : int32_t {
    kFlagBadResidue = 0,
    kFlagReverseMismatch = 1,
    kFlagBadOffsets = 2,
    kFlagBadScheme = 3,
    kFlagTooLong = 4,
    kNumFlags = 8,
};

}  // namespace sw

#include <hip/hip_runtime_api.h>

namespace sw {
using PassFn = void (*)(KParams, int, int, int);
// A compiled sweep kernel: precision (32 or 16), lanes per group W, rows per lane R.
struct ShapeEntry { int prec, W, R; PassFn fn; };
const ShapeEntry* shapes_i32(int* n);
const ShapeEntry* shapes_i16(int* n);
// Pairs one workgroup of the given shape aligns.
inline int pairs_per_block(const ShapeEntry& e) {
    return kWavesPerBlock * (64 / e.W) * (e.prec == 16 ? 2 : 1);
}
hipError_t launch_pass(const ShapeEntry& e, const KParams& P, int first, int count, int reverse,
                       hipStream_t stream);
// Classification inputs: bin_of_rows[sel * kLutRows + (n-1)/16] gives the bin
// of a pair with query length n, where sel = 0 for the packed int16 path and
// 1 for int32; a pair takes int16 when min(n, m) * max_score[s] <= i16_limit.
constexpr int kLutRows = SW_MAX_QUERY / 16;
struct ClassifyArgs {
    int32_t max_score[SW_MAX_SCHEMES];
    int32_t i16_limit;      // 0 disables the int16 path
    int32_t n_schemes;
    int32_t n_bins;
};
hipError_t launch_classify(const int64_t* q_off, const int64_t* r_off, const uint8_t* scheme_id,
                           int64_t n_pairs, const ClassifyArgs& C, const int8_t* bin_of_rows,
                           uint32_t* keys, int32_t* vals, sw_result* out, int32_t* flags,
                           int32_t* hist, int32_t* maxm, unsigned long long* fwd_cells,
                           hipStream_t stream);
hipError_t launch_reverse_cells(const sw_result* out, int64_t n, unsigned long long* acc,
                                hipStream_t stream);
}  // namespace sw
