// sw_kernels.hip -- gfx950 kernels of libswalign.
//
// Hot path: the forward and reverse sweeps of the affine-gap Smith-Waterman
// (Gotoh) recurrences of Section II-B-1 / Fig. 2, batched over many
// independent query/reference pairs.
//
// Mapping onto CDNA4 (one pair per lane group, anti-diagonal sweep):
//   * A wavefront (64 lanes) is split into 64/W groups of W lanes (W = 16 or
//     64).  Each group owns one pair.  Lane l of a group owns query rows
//     l*R .. l*R+R-1 in registers (H, E and the row's running best), so a
//     group covers W*R >= n rows in a single sweep.
//   * At step t lane l computes column j = t - l for its R rows, i.e. the
//     group sweeps anti-diagonals of lane-blocks.  The value a lane needs from
//     the row above its block (H and F of the last row of lane l-1 at
//     column j) was produced by lane l-1 one step earlier and arrives through
//     a DPP row/wave shift -- the same mechanism for every lane, with no
//     divergent first-lane path (the lesson of Section V-A).  Lane 0 of a
//     group receives zeros, the matrix's top boundary.
//   * The reference of each group is staged in LDS as pre-scaled row offsets
//     into the LDS substitution matrix, so one LDS byte read per cell gives
//     M[a_i][b_j].  Columns left of 0 (ramp-up) and right of m (ramp-down)
//     read a padding code whose score is -1.
//   * No per-step barrier or warp vote: a wavefront runs in lock-step
//     (Section V-B), and shared state is initialised once, by the lanes that
//     use it (Section V-C).
//
// Exactness of the padding: E and F are carried clamped at zero
// (E* = max(E, 0)), which leaves H unchanged because H takes a max with 0.  A
// padded cell (row >= n or column >= m or < 0) scores at most
// max(diag - 1, E, F) where diag <= S and E, F <= S - o, so with o >= 1 it is
// strictly below the pair's best S and never changes S or its first cell;
// real cells never depend on padded ones (they lie below or to the right).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

// One sweep (forward or reverse) of pairs order[first .. first+count), one
// pair per W-lane group, int32 arithmetic.
template <int W, int R>
__global__ __launch_bounds__(kBlock) void sw_pass_i32(KParams P, int first, int count,
                                                      int reverse) {
    constexpr int G = 64 / W;
    using Stager = RefStager<W>;
    __shared__ __attribute__((aligned(16))) SchemeLds S;
    __shared__ uint16_t refbuf[kWavesPerBlock * G * Stager::kBuf];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int g = lane / W;
    const int l = lane % W;

    load_schemes(S, P, tid);

    const int slot = (blockIdx.x * kWavesPerBlock + wave) * G + g;
    const int pair = slot < count ? P.order[first + slot] : -1;
    const PairJob J = load_job(P, pair, reverse);

    // wave-uniform step count: longest reference in the wavefront + ramp
    int mmax = J.m;
    for (int off = 32; off > 0; off >>= 1) mmax = imax(mmax, __shfl_xor(mmax, off));
    const int steps = __builtin_amdgcn_readfirstlane(mmax > 0 ? mmax + W - 1 : 0);

    uint16_t* buf = refbuf + (wave * G + g) * Stager::kBuf;
    Stager stage;
    stage.load(P.refs, J, P.order, 0, l);

    // query rows of this lane (padding code below the query end)
    int a[R];
    {
        int raw[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int i = l * R + r;
            i = i < J.n ? i : (J.n > 0 ? J.n - 1 : 0);
            const uint8_t* p = J.n > 0 ? P.queries + J.qbase + (int64_t)J.dir * i
                                       : reinterpret_cast<const uint8_t*>(P.order);
            raw[r] = *p;
        }
        __syncthreads();   // scheme tables
        const int A = S.alphabet[J.sid];
        bool bad = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool inside = l * R + r < J.n;
            bad |= inside && raw[r] >= A;
            a[r] = (inside && raw[r] < A) ? raw[r] : kPad;
        }
        stage.store(buf, J, A, 0, l, bad);
        if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);
    }
    const int A = S.alphabet[J.sid];
    const int go = S.gap_open[J.sid];
    const int ge = S.gap_extend[J.sid];
    wave_lds_sync();

    int H[R], E[R], Hm[R], best[R], bj[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = 0; E[r] = 0; Hm[r] = 0; best[r] = 0; bj[r] = -1; }
    int Hlast = 0, Flast = 0, Hup_prev = 0;
    const uint16_t* rbl = buf + W - l;   // rbl[tt] = column t0 + tt - l

    // software pipeline: scores of the current step and the matrix row of
    // the next step are read one step ahead
    int sc[R];
    int bb_next = rbl[1];
    {
        const int bb0 = rbl[0];
#pragma unroll
        for (int r = 0; r < R; ++r) sc[r] = S.mat[bb0 + a[r]];
    }
    bool bad = false;
    int j = -l;
    for (int t0 = 0; t0 < steps; t0 += kChunk) {
        const bool more = t0 + kChunk < steps;
        if (more) stage.load(P.refs, J, P.order, t0 + kChunk, l);
        const int tn = __builtin_amdgcn_readfirstlane(steps - t0 < kChunk ? steps - t0 : kChunk);
        for (int tt = 0; tt < tn; ++tt) {
            const int bb2 = rbl[tt + 2];
            int sn[R];
#pragma unroll
            for (int r = 0; r < R; ++r) sn[r] = S.mat[bb_next + a[r]];
            const int Hup = shift_in_group<W>(Hlast);
            const int Fup = shift_in_group<W>(Flast);
            int diag = Hup_prev;
            Hup_prev = Hup;
            int Hmu = sat_sub(Hup, go);
            int F = Fup;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int en = imax(E[r] - ge, Hm[r]);
                F = imax(F - ge, Hmu);
                const int h = imax(imax(diag + sc[r], en), F);
                diag = H[r];
                H[r] = h;
                E[r] = en;
                Hm[r] = sat_sub(h, go);
                Hmu = Hm[r];
                if (h > best[r]) { best[r] = h; bj[r] = j; }
            }
            Hlast = H[R - 1];
            Flast = F;
#pragma unroll
            for (int r = 0; r < R; ++r) sc[r] = sn[r];
            bb_next = bb2;
            ++j;
        }
        if (more) {
            wave_lds_sync();
            stage.store(buf, J, A, t0 + kChunk, l, bad);
            wave_lds_sync();
            // the two look-ahead reads of the next chunk's first steps were
            // taken from the old buffer; the new buffer holds the same
            // columns at entries W-l+0 and W-l+1, so re-read them
            bb_next = rbl[1];
            const int bb0 = rbl[0];
#pragma unroll
            for (int r = 0; r < R; ++r) sc[r] = S.mat[bb0 + a[r]];
        }
    }
    if (bad && P.validate) atomicOr(&P.flags[kFlagBadResidue], 1);

    // best of this lane in row-major order, then of the group
    int lb = 0, li = -1, lj = -1;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (best[r] > lb) { lb = best[r]; li = l * R + r; lj = bj[r]; }
    for (int off = 1; off < W; off <<= 1) {
        const int ob = __shfl_xor(lb, off);
        const int oi = __shfl_xor(li, off);
        const int oj = __shfl_xor(lj, off);
        if (ob > lb || (ob == lb && oi < li)) { lb = ob; li = oi; lj = oj; }
    }
    if (l == 0 && pair >= 0) {
        if (!reverse) {
            sw_result res;
            if (lb > 0) { res.score = lb; res.q_start = -1; res.q_end = li; res.r_start = -1; res.r_end = lj; }
            else { res.score = 0; res.q_start = res.q_end = res.r_start = res.r_end = -1; }
            P.out[pair] = res;
        } else if (J.fwd_score > 0) {
            if (lb != J.fwd_score) {
                atomicOr(&P.flags[kFlagReverseMismatch], 1);
            } else {
                P.out[pair].q_start = J.fwd_qe - li;
                P.out[pair].r_start = J.fwd_re - lj;
            }
        }
    }
}

// Classify every pair: validate offsets, lengths and scheme ids, route empty
// or invalid pairs to a trivial result, and emit a sort key
// (bin << 16 | (65535 - m)) so that a radix sort groups pairs by bin with
// the longest references first.
__global__ void sw_classify(const int64_t* q_off, const int64_t* r_off, const uint8_t* scheme_id,
                            int64_t n_pairs, ClassifyArgs C, const int8_t* bin_of_rows,
                            uint32_t* keys, int32_t* vals, sw_result* out,
                            int32_t* flags, int32_t* hist, int32_t* maxm,
                            unsigned long long* fwd_cells) {
    __shared__ int32_t s_hist[64];
    __shared__ int32_t s_maxm[64];
    __shared__ unsigned long long s_cells;
    const int n_bins = C.n_bins;
    for (int k = threadIdx.x; k < 64; k += blockDim.x) { s_hist[k] = 0; s_maxm[k] = 0; }
    if (threadIdx.x == 0) s_cells = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pairs) {
        const int64_t n = q_off[i + 1] - q_off[i];
        const int64_t m = r_off[i + 1] - r_off[i];
        const int s = scheme_id ? (int)scheme_id[i] : 0;
        int bin = n_bins;  // trivial
        if (n < 0 || m < 0) atomicOr(&flags[kFlagBadOffsets], 1);
        else if (s >= C.n_schemes) atomicOr(&flags[kFlagBadScheme], 1);
        else if (n > SW_MAX_QUERY || m > SW_MAX_REF) atomicOr(&flags[kFlagTooLong], 1);
        else if (n > 0 && m > 0) {
            const int64_t mn = n < m ? n : m;
            const int sel = mn * C.max_score[s] <= C.i16_limit ? 0 : 1;
            bin = bin_of_rows[sel * kLutRows + (n - 1) / 16];
        }
        if (bin >= n_bins) {
            sw_result z;
            z.score = 0; z.q_start = z.q_end = z.r_start = z.r_end = -1;
            out[i] = z;
            keys[i] = 0xFFFFFFFFu;
        } else {
            keys[i] = ((uint32_t)bin << 16) | (uint32_t)(65535 - (int)m);
            atomicAdd(&s_hist[bin], 1);
            atomicMax(&s_maxm[bin], (int)m);
            atomicAdd(&s_cells, (unsigned long long)(n * m));
        }
        vals[i] = (int32_t)i;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n_bins; k += blockDim.x) {
        if (s_hist[k]) { atomicAdd(&hist[k], s_hist[k]); atomicMax(&maxm[k], s_maxm[k]); }
    }
    if (threadIdx.x == 0 && s_cells) atomicAdd(fwd_cells, s_cells);
}

}  // namespace sw

// ---------------------------------------------------------------------------
// Launch table of the compiled int32 bin shapes.
// ---------------------------------------------------------------------------
namespace sw {

template <int W, int R>
static constexpr PassFn pass_i32() { return &sw_pass_i32<W, R>; }

static const ShapeEntry kShapesI32[] = {
    {32, 16, 2, pass_i32<16, 2>()},   {32, 16, 4, pass_i32<16, 4>()},
    {32, 16, 6, pass_i32<16, 6>()},   {32, 16, 8, pass_i32<16, 8>()},
    {32, 16, 10, pass_i32<16, 10>()}, {32, 16, 12, pass_i32<16, 12>()},
    {32, 16, 14, pass_i32<16, 14>()}, {32, 16, 16, pass_i32<16, 16>()},
    {32, 64, 6, pass_i32<64, 6>()},   {32, 64, 8, pass_i32<64, 8>()},
    {32, 64, 10, pass_i32<64, 10>()}, {32, 64, 12, pass_i32<64, 12>()},
    {32, 64, 14, pass_i32<64, 14>()}, {32, 64, 16, pass_i32<64, 16>()},
    {32, 64, 20, pass_i32<64, 20>()}, {32, 64, 24, pass_i32<64, 24>()},
    {32, 64, 28, pass_i32<64, 28>()}, {32, 64, 32, pass_i32<64, 32>()},
};

const ShapeEntry* shapes_i32(int* n) {
    *n = (int)(sizeof(kShapesI32) / sizeof(kShapesI32[0]));
    return kShapesI32;
}

hipError_t launch_pass(const ShapeEntry& e, const KParams& P, int first, int count, int reverse,
                       hipStream_t stream) {
    const int ppb = pairs_per_block(e);
    const int blocks = (count + ppb - 1) / ppb;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(e.fn, dim3(blocks), dim3(kBlock), 0, stream, P, first, count, reverse);
    return hipGetLastError();
}

hipError_t launch_classify(const int64_t* q_off, const int64_t* r_off, const uint8_t* scheme_id,
                           int64_t n_pairs, const ClassifyArgs& C, const int8_t* bin_of_rows,
                           uint32_t* keys, int32_t* vals, sw_result* out, int32_t* flags,
                           int32_t* hist, int32_t* maxm, unsigned long long* fwd_cells,
                           hipStream_t stream) {
    const int threads = 256;
    const int64_t blocks = (n_pairs + threads - 1) / threads;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(sw_classify, dim3((unsigned)blocks), dim3(threads), 0, stream, q_off, r_off,
                       scheme_id, n_pairs, C, bin_of_rows, keys, vals, out, flags, hist, maxm,
                       fwd_cells);
    return hipGetLastError();
}

// Reverse cells of a finished batch: sum over pairs with a positive score of
// (q_end+1)*(r_end+1).
__global__ void sw_reverse_cells(const sw_result* out, int64_t n, unsigned long long* acc) {
    __shared__ unsigned long long s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    unsigned long long v = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const sw_result r = out[i];
        if (r.score > 0) v += (unsigned long long)(r.q_end + 1) * (unsigned long long)(r.r_end + 1);
    }
    atomicAdd(&s, v);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(acc, s);
}

hipError_t launch_reverse_cells(const sw_result* out, int64_t n, unsigned long long* acc,
                                hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(sw_reverse_cells, dim3((unsigned)blocks), dim3(256), 0, stream, out, n, acc);
    return hipGetLastError();
}

}  // namespace sw
