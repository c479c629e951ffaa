// sw_plan.hip -- device-side planning of a sweep pass (gfx950).
//
// For each pass (forward, then reverse) the pairs are
//   1. classified: validated (forward), routed to int16 or int32 by their
//      score bound, given a bin from their (sub)query length and a 16-bit
//      key (bin, reference-length bucket, longest first);
//   2. counted into a histogram of keys, which one workgroup scans into
//      bucket offsets and per-bin pair and work-item ranges;
//   3. scattered into key order (order within a bucket is irrelevant: every
//      pair's result is independent of where it runs);
//   4. cut into wavefront work items of ppw consecutive pairs of one bin.
// The reverse pass re-bins pairs by the shape of their reverse sub-problem
// (q_end+1 rows, r_end+1 columns), which can differ a lot from the forward
// shape.  Nothing here synchronises with the host and nothing is cleared
// with a memset, so a whole call can be captured in a hipGraph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

__global__ void sw_reset_kernel(int32_t* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void sw_call_start_kernel(int32_t* small, int n_small, int32_t* n_dev, int32_t n_pairs) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_small; i += gridDim.x * blockDim.x) small[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_dev = n_pairs;
}

__global__ void sw_classify_kernel(KParams P, ClassifyArgs C, const int8_t* lut, const BinInfo* bins,
                                   int32_t* keys, int32_t* hist, unsigned long long* counters) {
    const int64_t n_pairs = *P.n_dev;
    // counters[0] / [1]: forward / reverse cells; counters[2]: int32 pairs
    // (forward); per bin of this pass: cells and pairs (kCtrBinCells,
    // kCtrBinPairs, indexed pass * kMaxBins + bin)
    __shared__ unsigned long long s_cells;
    __shared__ int32_t s_trivial, s_i32;
    __shared__ unsigned long long s_bin_cells[2][kMaxBins];   // [column path?][bin]
    __shared__ uint32_t s_bin_pairs[2][kMaxBins];
    if (threadIdx.x == 0) { s_cells = 0; s_trivial = 0; s_i32 = 0; }
    if (threadIdx.x < kMaxBins) {
        s_bin_cells[0][threadIdx.x] = s_bin_cells[1][threadIdx.x] = 0;
        s_bin_pairs[0][threadIdx.x] = s_bin_pairs[1][threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long my_cells = 0;
    if (i < n_pairs) {
        int64_t n = 0, m = 0;
        int s = 0;
        bool ok = false;
        if (!P.reverse) {
            n = P.q_end[i] - P.q_beg[i];
            m = P.r_end[i] - P.r_beg[i];
            s = P.scheme_id ? (int)P.scheme_id[i] : 0;
            if (n < 0 || m < 0) atomicOr(&P.flags[kFlagBadOffsets], 1);
            else if (s >= C.n_schemes) atomicOr(&P.flags[kFlagBadScheme], 1);
            else if (n > SW_MAX_QUERY || m > SW_MAX_REF || (C.max_query > 0 && n > C.max_query))
                atomicOr(&P.flags[kFlagTooLong], 1);
            else ok = n > 0 && m > 0;
            if (!ok) {
                sw_result z;
                z.score = 0; z.q_start = z.q_end = z.r_start = z.r_end = -1;
                P.out[i] = z;
            }
        } else {
            // the reverse sub-problem is the prefix box ending at the forward
            // end; an end outside the pair would be an internal error
            const sw_result r = P.out[i];
            if (r.score > 0) {
                const int64_t n0 = P.q_end[i] - P.q_beg[i];
                const int64_t m0 = P.r_end[i] - P.r_beg[i];
                n = (int64_t)r.q_end + 1;
                m = (int64_t)r.r_end + 1;
                s = P.scheme_id ? (int)P.scheme_id[i] : 0;
                ok = n >= 1 && n <= n0 && m >= 1 && m <= m0 && s < C.n_schemes;
                if (!ok) {
                    atomicOr(&P.flags[kFlagInternal], 1);
                } else {
                    // the part of the prefixes that can hold the start (the
                    // sweep cuts its job the same way)
                    int nn = (int)n, mm = (int)m;
                    reverse_extent(r.score, P.max_score[s], P.gap_open[s], P.gap_extend[s], nn, mm);
                    n = nn;
                    m = mm;
                }
            }
        }
        int key = kTrivialKey;
        if (ok) {
            const int64_t mn = n < m ? n : m;
            const int sel = (mn * C.max_score[s] <= C.i16_limit && m <= kI16MaxRef) ? 0 : 1;
            if (sel && !P.reverse) atomicAdd(&s_i32, 1);
            const int bin = lut[sel * kLutRows + (int)((n - 1) / 16)];
            // within a bin: pairs of column-path schemes first (the bin's
            // column-word kernel takes them), each part by decreasing
            // reference length; only packed-int16 pairs use column words
            const int col = (sel == 0 && C.col_ok[s] && bins[bin].col) ? 1 : 0;
            key = bin * kMBuckets + (col ? 0 : kMHalf) + (kMHalf - 1 - m_bucket((int)m));
            atomicAdd(&hist[key], 1);
            my_cells = (unsigned long long)(n * m);
            atomicAdd(&s_bin_cells[col][bin], my_cells);
            atomicAdd(&s_bin_pairs[col][bin], 1u);
        } else {
            atomicAdd(&s_trivial, 1);
        }
        keys[i] = key;
    }
    if (my_cells) atomicAdd(&s_cells, my_cells);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_cells) atomicAdd(&counters[P.reverse ? kCtrRevCells : kCtrFwdCells], s_cells);
        if (s_i32) atomicAdd(&counters[kCtrI32Pairs], (unsigned long long)s_i32);
        if (s_trivial) atomicAdd(&hist[kTrivialKey], s_trivial);
    }
    if (threadIdx.x < kMaxBins) {
        const int b = threadIdx.x;
        const int slot = (P.reverse ? kMaxBins : 0) + b;
        const unsigned long long pairs = s_bin_pairs[0][b] + s_bin_pairs[1][b];
        if (pairs) {
            atomicAdd(&counters[kCtrBinCells + slot], s_bin_cells[0][b] + s_bin_cells[1][b]);
            atomicAdd(&counters[kCtrBinPairs + slot], pairs);
        }
        if (s_bin_pairs[1][b]) {
            atomicAdd(&counters[kCtrBinColCells + slot], s_bin_cells[1][b]);
            atomicAdd(&counters[kCtrBinColPairs + slot], (unsigned long long)s_bin_pairs[1][b]);
        }
    }
}

// One workgroup of 1024 threads: exclusive scan of the key histogram in
// place, then the per-bin pair and work-item ranges.  The histogram is
// scanned in segments staged through LDS (coalesced loads and stores; each
// thread then sums a run of kRun consecutive entries, padded by one word per
// run against bank conflicts), with wave-level shuffle scans in between.
constexpr int kPlanThreads = 1024;
constexpr int kRun = 16;
constexpr int kSeg = kPlanThreads * kRun;

__device__ __forceinline__ int lds_slot(int e) { return e + e / kRun; }

// Inclusive scan within a wavefront.
__device__ __forceinline__ int32_t wave_scan(int32_t v, int lane) {
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    return v;
}

__global__ __launch_bounds__(kPlanThreads) void sw_plan_kernel(const BinInfo* bins, int n_bins,
                                                               int32_t* hist, int32_t* meta) {
    __shared__ int32_t seg[kSeg + kSeg / kRun];
    __shared__ int32_t wave_tot[kPlanThreads / 64];
    __shared__ int32_t bin_items[kMaxBins + 1];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    int32_t carry = 0;   // sum of all earlier segments (same value in every thread)
    for (int base = 0; base < kHistSize; base += kSeg) {
        const int n = kHistSize - base < kSeg ? kHistSize - base : kSeg;
        for (int e = t; e < kSeg; e += kPlanThreads) seg[lds_slot(e)] = e < n ? hist[base + e] : 0;
        __syncthreads();
        int32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kRun; ++k) sum += seg[lds_slot(t * kRun + k)];
        const int32_t incl = wave_scan(sum, lane);
        if (lane == 63) wave_tot[wave] = incl;
        __syncthreads();
        int32_t before = 0, total = 0;
        for (int w = 0; w < kPlanThreads / 64; ++w) {
            const int32_t x = wave_tot[w];
            before += w < wave ? x : 0;
            total += x;
        }
        int32_t run = carry + before + incl - sum;   // exclusive prefix of this thread's run
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const int slot = lds_slot(t * kRun + k);
            const int32_t c = seg[slot];
            seg[slot] = run;
            run += c;
        }
        __syncthreads();
        for (int e = t; e < n; e += kPlanThreads) hist[base + e] = seg[lds_slot(e)];
        carry += total;
        __syncthreads();
    }
    // per-bin ranges: the bin's first sorted position is the scanned count
    // of its first key; its items are its pairs in groups of ppw, the
    // column-path pairs (the first half of its keys) first
    int32_t my_col = 0;
    if (t <= kMaxBins) {
        const int32_t f = hist[t * kMBuckets];   // t == kMaxBins: the trivial key
        meta[kMetaBinFirst + t] = f;
        bin_items[t] = f;
        if (t < kMaxBins) my_col = hist[t * kMBuckets + kMHalf] - f;
    }
    if (t < kMaxBins) {
        meta[kMetaHeads + t] = 0;
        meta[kMetaColHeads + t] = 0;
    }
    __syncthreads();
    int32_t my_items = 0, my_col_items = 0;
    if (t < n_bins && t < kMaxBins) {
        const int32_t cnt = bin_items[t + 1] - bin_items[t];
        const int ppw = bins[t].ppw;
        // the column-path pairs (first in the bin) and the others are cut
        // into items separately, so no item mixes the two; a shape without
        // a column kernel sorts none of its pairs as column-path pairs
        if (!bins[t].col) my_col = 0;
        my_col_items = (my_col + ppw - 1) / ppw;
        my_items = my_col_items + (cnt - my_col + ppw - 1) / ppw;
    }
    if (t < kMaxBins) meta[kMetaBinCol + t] = t < n_bins ? my_col : 0;
    __syncthreads();
    if (t < kMaxBins) bin_items[t] = my_items;
    __syncthreads();
    if (t == 0) {
        int32_t items = 0;
        for (int b = 0; b < kMaxBins; ++b) {
            meta[kMetaItemFirst + b] = items;
            items += bin_items[b];
        }
        meta[kMetaItemFirst + kMaxBins] = items;
    }
    __syncthreads();
    if (t < kMaxBins) meta[kMetaItemSplit + t] = meta[kMetaItemFirst + t] + my_col_items;
}

// Parallel form of the plan for the score passes, whose classify kernel
// also counts every bin's pairs and column-path pairs (counters
// kCtrBinPairs / kCtrBinColPairs of the pass): those counts are the sums of
// the bin's histogram entries and of their first half, so every bin's
// first sorted position, column split and work items follow from them
// directly.  Workgroup b < kMaxBins scans bin b's kMBuckets entries in
// place, offset by the pairs of bins 0..b-1 (a bin without pairs is left
// as it is: no key of it occurs); workgroup kMaxBins writes the trivial
// key's position and the metadata.  The result equals sw_plan_kernel's.
constexpr int kBinScanThreads = 256;
constexpr int kBinScanRun = kMBuckets / kBinScanThreads;

__global__ __launch_bounds__(kBinScanThreads) void sw_plan_bins_kernel(const BinInfo* bins, int n_bins,
                                                                        int32_t* hist, int32_t* meta,
                                                                        const unsigned long long* counters,
                                                                        int reverse) {
    __shared__ int32_t s_pairs[kMaxBins], s_col[kMaxBins];
    __shared__ int32_t wave_tot[kBinScanThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int slot0 = reverse ? kMaxBins : 0;
    if (t < kMaxBins) {
        const bool real = t < n_bins;
        s_pairs[t] = real ? (int32_t)counters[kCtrBinPairs + slot0 + t] : 0;
        s_col[t] = real && bins[t].col ? (int32_t)counters[kCtrBinColPairs + slot0 + t] : 0;
    }
    __syncthreads();
    const int b = blockIdx.x;
    if (b < kMaxBins) {
        if (s_pairs[b] == 0) return;
        int32_t base = 0;
        for (int k = 0; k < b; ++k) base += s_pairs[k];
        int32_t* hb = hist + b * kMBuckets + t * kBinScanRun;
        int32_t v[kBinScanRun];
        int32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kBinScanRun; ++k) {
            v[k] = hb[k];
            sum += v[k];
        }
        const int32_t incl = wave_scan(sum, lane);
        if (lane == 63) wave_tot[wave] = incl;
        __syncthreads();
        int32_t run = base + incl - sum;
        for (int w = 0; w < wave; ++w) run += wave_tot[w];
#pragma unroll
        for (int k = 0; k < kBinScanRun; ++k) {
            hb[k] = run;
            run += v[k];
        }
        return;
    }
    // the metadata, as sw_plan_kernel writes it
    if (t == 0) {
        int32_t pos = 0, items = 0;
        for (int k = 0; k < kMaxBins; ++k) {
            meta[kMetaBinFirst + k] = pos;
            meta[kMetaItemFirst + k] = items;
            const int ppw = k < n_bins ? bins[k].ppw : 1;
            const int32_t col_items = (s_col[k] + ppw - 1) / ppw;
            meta[kMetaItemSplit + k] = items + col_items;
            items += col_items + (s_pairs[k] - s_col[k] + ppw - 1) / ppw;
            pos += s_pairs[k];
        }
        meta[kMetaBinFirst + kMaxBins] = pos;
        meta[kMetaItemFirst + kMaxBins] = items;
        hist[kTrivialKey] = pos;
    }
    if (t < kMaxBins) {
        meta[kMetaHeads + t] = 0;
        meta[kMetaColHeads + t] = 0;
        meta[kMetaBinCol + t] = s_col[t];
    }
}

// Pairs with the trivial key get no position: nothing reads the sorted order
// past the last bin (their results, if any, were written at
// classification).  Skipping them keeps one counter from taking an atomic
// per such pair, which serialised e.g. the pairs outside a path chunk.
__global__ void sw_scatter_kernel(const int32_t* keys, const int32_t* n_dev, int32_t* offs, int32_t* order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *n_dev) return;
    const int32_t key = keys[i];
    if (key == kTrivialKey) return;
    const int32_t pos = atomicAdd(&offs[key], 1);
    order[pos] = (int32_t)i;
}

__global__ void sw_items_kernel(const int32_t* meta, const BinInfo* bins, int n_bins, const int32_t* n_dev,
                                WorkItem* items) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *n_dev || i >= meta[kMetaBinFirst + n_bins]) return;
    // the bin holding sorted position i: the last bin whose first position
    // is at most i (empty bins share their successor's first position)
    int lo = 0, hi = n_bins - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (meta[kMetaBinFirst + mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const int b = lo;
    const int32_t f = meta[kMetaBinFirst + b];
    const int32_t cnt = meta[kMetaBinFirst + b + 1] - f;
    const int32_t ncol = meta[kMetaBinCol + b];
    const BinInfo bi = bins[b];
    // column-path pairs [0, ncol) of the bin, then the others, each cut
    // into items of ppw pairs
    int32_t k = (int32_t)i - f, end = ncol, item = meta[kMetaItemFirst + b];
    if (k >= ncol) {
        k -= ncol;
        end = cnt - ncol;
        item += (ncol + bi.ppw - 1) / bi.ppw;
    }
    if (k % bi.ppw != 0) return;
    WorkItem w;
    w.first = (int32_t)i;
    w.count = (uint16_t)(end - k < bi.ppw ? end - k : bi.ppw);
    w.bin = (uint8_t)b;
    w.pad = 0;
    items[item + k / bi.ppw] = w;
}

__global__ void sw_fill_span_kernel(int64_t* beg, int64_t* end, int64_t n, int64_t len) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        beg[i] = 0;
        end[i] = len;
    }
}

static unsigned grid_for(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
    return (unsigned)(b > 0 ? b : 1);
}

hipError_t launch_fill_span(int64_t* beg, int64_t* end, int64_t n, int64_t len, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    unsigned blocks = grid_for(n, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(sw_fill_span_kernel, dim3(blocks), dim3(256), 0, s, beg, end, n, len);
    return hipGetLastError();
}

hipError_t launch_reset(int32_t* p, int n, hipStream_t s) {
    unsigned blocks = grid_for(n, 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(sw_reset_kernel, dim3(blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_call_start(int32_t* small, int n_small, int32_t* n_dev, int32_t n_pairs, hipStream_t s) {
    unsigned blocks = grid_for(n_small, 256);
    if (blocks > 64) blocks = 64;
    hipLaunchKernelGGL(sw_call_start_kernel, dim3(blocks), dim3(256), 0, s, small, n_small, n_dev, n_pairs);
    return hipGetLastError();
}

hipError_t launch_classify(const KParams& P, const ClassifyArgs& C, const int8_t* lut, const BinInfo* bins,
                           int64_t cap, int32_t* keys, int32_t* hist,
                           unsigned long long* counters, hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(sw_classify_kernel, dim3(grid_for(cap, 256)), dim3(256), 0, s, P, C, lut, bins,
                       keys, hist, counters);
    return hipGetLastError();
}

hipError_t launch_plan(const BinInfo* bins, int n_bins, int32_t* hist, int32_t* meta, hipStream_t s) {
    hipLaunchKernelGGL(sw_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, bins, n_bins, hist, meta);
    return hipGetLastError();
}

hipError_t launch_plan_bins(const BinInfo* bins, int n_bins, int32_t* hist, int32_t* meta,
                            const unsigned long long* counters, int reverse, hipStream_t s) {
    hipLaunchKernelGGL(sw_plan_bins_kernel, dim3(kMaxBins + 1), dim3(kBinScanThreads), 0, s, bins, n_bins, hist,
                       meta, counters, reverse);
    return hipGetLastError();
}

hipError_t launch_scatter(const int32_t* keys, const int32_t* n_dev, int64_t cap, int32_t* hist,
                          int32_t* order, hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(sw_scatter_kernel, dim3(grid_for(cap, 256)), dim3(256), 0, s, keys, n_dev,
                       hist, order);
    return hipGetLastError();
}

hipError_t launch_items(const int32_t* meta, const BinInfo* bins, int n_bins, const int32_t* n_dev,
                        int64_t cap, WorkItem* items, hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(sw_items_kernel, dim3(grid_for(cap, 256)), dim3(256), 0, s, meta, bins, n_bins,
                       n_dev, items);
    return hipGetLastError();
}



}  // namespace sw
