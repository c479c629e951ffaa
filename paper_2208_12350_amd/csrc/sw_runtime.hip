// sw_runtime.hip -- host runtime of libswalign: argument checks, device-side
// classification and length binning, launch planning, error reporting.
//
// One sw_align_batch call:
//   1. host checks of the arguments and schemes; the schemes' matrices are
//      packed into a [scheme][ref residue][query residue] int8 table;
//   2. sw_classify (device): per pair length/offset/scheme checks, a bin
//      from the query length, and a sort key (bin, longest reference first);
//   3. hipcub radix sort of (key, pair id) on the device;
//   4. one small device->host copy of the per-bin histogram (the only
//      synchronisation before the sweeps);
//   5. the forward sweep of every bin, then the reverse sweep of every bin;
//   6. a device->host copy of the error flags.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "sw_internal.h"

using namespace sw;

namespace {

constexpr int kLutEntries = 2 * kLutRows;       // [int16 | int32] x 16-row buckets of query length
constexpr int kSmallInts = 256;                   // pinned host staging for hist/maxm/flags

struct DeviceBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct sw_handle {
    int device = 0;
    std::string err;
    int64_t opt_mode = 0;
    int64_t opt_graph = 0;
    int64_t opt_validate = 1;
    int64_t opt_precision = 0;
    int64_t opt_timing = 0;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float t_plan = 0.f, t_fwd = 0.f, t_rev = 0.f;

    std::vector<ShapeEntry> bins;        // the kernel shape of each bin
    std::vector<int8_t> lut;             // precision x (query length - 1) / 16 -> bin

    int8_t* d_mats = nullptr;
    int8_t* d_lut = nullptr;
    int32_t* d_small = nullptr;          // flags[8] | hist[64] | maxm[64]
    unsigned long long* d_cells = nullptr;  // [0] forward cells, [1] reverse cells
    uint32_t* d_keys = nullptr;
    uint32_t* d_keys2 = nullptr;
    int32_t* d_vals = nullptr;
    int32_t* d_vals2 = nullptr;
    int64_t cap_pairs = 0;
    void* d_temp = nullptr;
    size_t temp_bytes = 0;

    int8_t* h_mats = nullptr;            // pinned
    int32_t* h_small = nullptr;          // pinned
    unsigned long long* h_cells = nullptr;  // pinned

    int64_t last_fwd = 0;
    int64_t last_i32 = 0;
    const sw_result* last_out = nullptr;
    int64_t last_n = 0;
    hipStream_t last_stream = nullptr;
};

static int fail(sw_handle* h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    return code;
}

#define HIP_TRY(h, call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((h), SW_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

static void build_bins(sw_handle* h) {
    // Bins 0.. are the packed int16 shapes, then the int32 shapes.  Default
    // binning: queries up to 256 rows run on 16-lane groups, longer ones on
    // 64-lane groups; the rows per lane R is the smallest compiled value
    // covering the upper end of the query's 16-row bucket.
    h->bins.clear();
    int n16 = 0, n32 = 0;
    const ShapeEntry* s16 = shapes_i16(&n16);
    const ShapeEntry* s32 = shapes_i32(&n32);
    for (int k = 0; k < n16; ++k) h->bins.push_back(s16[k]);
    for (int k = 0; k < n32; ++k) h->bins.push_back(s32[k]);
    h->lut.assign(kLutEntries, -1);
    for (int sel = 0; sel < 2; ++sel) {
        const int prec = sel == 0 ? 16 : 32;
        for (int k = 0; k < kLutRows; ++k) {
            const int rows = 16 * (k + 1);
            const int W = rows <= 256 ? 16 : 64;
            int best = -1;
            for (int b = 0; b < (int)h->bins.size(); ++b) {
                const ShapeEntry& e = h->bins[b];
                if (e.prec != prec || e.W != W || e.W * e.R < rows) continue;
                if (best < 0 || e.R < h->bins[best].R) best = b;
            }
            h->lut[sel * kLutRows + k] = (int8_t)best;
        }
    }
}

static void free_dev(void* p) {
    if (p) (void)hipFree(p);
}

static int ensure_pairs(sw_handle* h, int64_t n) {
    if (n <= h->cap_pairs) return SW_OK;
    free_dev(h->d_keys); free_dev(h->d_keys2); free_dev(h->d_vals); free_dev(h->d_vals2);
    free_dev(h->d_temp);
    h->d_keys = h->d_keys2 = nullptr; h->d_vals = h->d_vals2 = nullptr; h->d_temp = nullptr;
    h->cap_pairs = 0;
    const int64_t cap = std::max<int64_t>(n, 1024);
    if (hipMalloc(&h->d_keys, cap * 4) != hipSuccess || hipMalloc(&h->d_keys2, cap * 4) != hipSuccess ||
        hipMalloc(&h->d_vals, cap * 4) != hipSuccess || hipMalloc(&h->d_vals2, cap * 4) != hipSuccess)
        return fail(h, SW_ENOMEM, "device allocation of %lld pair slots failed", (long long)cap);
    size_t tb = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tb, h->d_keys, h->d_keys2, h->d_vals, h->d_vals2,
                                           (int)cap, 0, 22) != hipSuccess)
        return fail(h, SW_EDEVICE, "radix sort sizing failed");
    if (hipMalloc(&h->d_temp, tb) != hipSuccess)
        return fail(h, SW_ENOMEM, "device allocation of sort scratch failed");
    h->temp_bytes = tb;
    h->cap_pairs = cap;
    return SW_OK;
}

extern "C" {

sw_handle* sw_create(int device, const char* tuning) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return nullptr;
    if (hipSetDevice(device) != hipSuccess) return nullptr;
    sw_handle* h = new sw_handle();
    h->device = device;
    build_bins(h);
    bool ok = hipMalloc(&h->d_mats, SW_MAX_SCHEMES * kMatBytes) == hipSuccess &&
              hipMalloc(&h->d_lut, kLutEntries) == hipSuccess &&
              hipMalloc(&h->d_small, kSmallInts * 4) == hipSuccess &&
              hipMalloc(&h->d_cells, 4 * sizeof(unsigned long long)) == hipSuccess &&
              hipHostMalloc(&h->h_mats, SW_MAX_SCHEMES * kMatBytes, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&h->h_small, kSmallInts * 4, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&h->h_cells, 4 * sizeof(unsigned long long), hipHostMallocDefault) == hipSuccess;
    for (int k = 0; ok && k < 5; ++k) ok = hipEventCreate(&h->ev[k]) == hipSuccess;
    if (ok) ok = hipMemcpy(h->d_lut, h->lut.data(), kLutEntries, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) { sw_destroy(h); return nullptr; }
    if (tuning) {
        std::string s(tuning);
        size_t pos = 0;
        while (pos < s.size()) {
            size_t end = s.find_first_of(";,", pos);
            if (end == std::string::npos) end = s.size();
            std::string kv = s.substr(pos, end - pos);
            size_t eq = kv.find('=');
            if (eq != std::string::npos) {
                if (sw_set_option(h, kv.substr(0, eq).c_str(), atoll(kv.substr(eq + 1).c_str())) != SW_OK) {
                    sw_destroy(h);
                    return nullptr;
                }
            }
            pos = end + 1;
        }
    }
    return h;
}

void sw_destroy(sw_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    free_dev(h->d_mats); free_dev(h->d_lut); free_dev(h->d_small); free_dev(h->d_cells);
    free_dev(h->d_keys); free_dev(h->d_keys2); free_dev(h->d_vals); free_dev(h->d_vals2);
    free_dev(h->d_temp);
    if (h->h_mats) (void)hipHostFree(h->h_mats);
    if (h->h_small) (void)hipHostFree(h->h_small);
    if (h->h_cells) (void)hipHostFree(h->h_cells);
    for (int k = 0; k < 5; ++k)
        if (h->ev[k]) (void)hipEventDestroy(h->ev[k]);
    delete h;
}

const char* sw_last_error(sw_handle* h) { return h ? h->err.c_str() : "null handle"; }

int sw_set_option(sw_handle* h, const char* key, int64_t value) {
    if (!h || !key) return SW_EINVAL;
    std::string k(key);
    if (k == "mode") {
        if (value != 0 && value != 1) return fail(h, SW_EINVAL, "mode must be 0 or 1");
        h->opt_mode = value;
    } else if (k == "graph") {
        h->opt_graph = value ? 1 : 0;
    } else if (k == "validate") {
        h->opt_validate = value ? 1 : 0;
    } else if (k == "timing") {
        h->opt_timing = value ? 1 : 0;
    } else if (k == "precision") {
        if (value != 0 && value != 32) return fail(h, SW_EINVAL, "precision must be 0 or 32");
        h->opt_precision = value;
    } else {
        return fail(h, SW_EINVAL, "unknown option '%s'", key);
    }
    return SW_OK;
}

int sw_get_option(sw_handle* h, const char* key, int64_t* value) {
    if (!h || !key || !value) return SW_EINVAL;
    std::string k(key);
    if (k == "mode") *value = h->opt_mode;
    else if (k == "graph") *value = h->opt_graph;
    else if (k == "validate") *value = h->opt_validate;
    else if (k == "precision") *value = h->opt_precision;
    else if (k == "timing") *value = h->opt_timing;
    else return fail(h, SW_EINVAL, "unknown option '%s'", key);
    return SW_OK;
}

int sw_align_batch(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes, int n_schemes,
                   sw_result* out, void* stream_ptr) {
    if (!h) return SW_EINVAL;
    h->err.clear();
    if (!batch || !schemes) return fail(h, SW_EINVAL, "null batch or schemes");
    if (n_schemes < 1 || n_schemes > SW_MAX_SCHEMES)
        return fail(h, SW_EINVAL, "n_schemes must be 1..%d", SW_MAX_SCHEMES);
    const int64_t P = batch->n_pairs;
    if (P < 0) return fail(h, SW_EINVAL, "negative n_pairs");
    if (P > (int64_t)0x7FFFFFFF) return fail(h, SW_EINVAL, "more than 2^31-1 pairs in one batch");
    for (int s = 0; s < n_schemes; ++s) {
        const sw_scheme& sc = schemes[s];
        if (!sc.matrix) return fail(h, SW_EINVAL, "scheme %d: null matrix", s);
        if (sc.alphabet < 1 || sc.alphabet > SW_MAX_ALPHABET)
            return fail(h, SW_EINVAL, "scheme %d: alphabet must be 1..%d", s, SW_MAX_ALPHABET);
        if (sc.gap_open < 1 || sc.gap_extend < 0 || sc.gap_extend > sc.gap_open || sc.gap_open > 1000000)
            return fail(h, SW_EINVAL, "scheme %d: need 1 <= gap_open <= 1e6 and 0 <= gap_extend <= gap_open", s);
    }
    h->last_fwd = 0; h->last_i32 = 0; h->last_out = out; h->last_n = P;
    h->t_plan = h->t_fwd = h->t_rev = 0.f;
    if (P == 0) return SW_OK;
    if (!batch->q_off || !batch->r_off || !out)
        return fail(h, SW_EINVAL, "null offsets or output with n_pairs > 0");
    hipStream_t stream = (hipStream_t)stream_ptr;
    h->last_stream = stream;
    HIP_TRY(h, hipSetDevice(h->device));
    int rc = ensure_pairs(h, P);
    if (rc != SW_OK) return rc;

    // substitution tables: [s][b][a] = M_s[a][b]; padding rows/columns score -1
    for (int s = 0; s < SW_MAX_SCHEMES; ++s) {
        int8_t* T = h->h_mats + s * kMatBytes;
        for (int b = 0; b < kMatDim; ++b)
            for (int a = 0; a < kMatDim; ++a) {
                int8_t v = -1;
                if (s < n_schemes && a < schemes[s].alphabet && b < schemes[s].alphabet)
                    v = schemes[s].matrix[a * schemes[s].alphabet + b];
                T[b * kMatDim + a] = v;
            }
    }
    HIP_TRY(h, hipMemcpyAsync(h->d_mats, h->h_mats, SW_MAX_SCHEMES * kMatBytes, hipMemcpyHostToDevice, stream));
    HIP_TRY(h, hipMemsetAsync(h->d_small, 0, kSmallInts * 4, stream));
    HIP_TRY(h, hipMemsetAsync(h->d_cells, 0, 4 * sizeof(unsigned long long), stream));

    const bool timing = h->opt_timing != 0;
    if (timing) HIP_TRY(h, hipEventRecord(h->ev[0], stream));
    int32_t* d_flags = h->d_small;
    int32_t* d_hist = h->d_small + kNumFlags;
    int32_t* d_maxm = h->d_small + kNumFlags + 64;
    const int n_bins = (int)h->bins.size();
    ClassifyArgs C;
    for (int s = 0; s < SW_MAX_SCHEMES; ++s) {
        int mx = 1;
        if (s < n_schemes)
            for (int k = 0; k < schemes[s].alphabet * schemes[s].alphabet; ++k)
                mx = std::max(mx, (int)schemes[s].matrix[k]);
        C.max_score[s] = mx;
    }
    // int16 holds every value of a pair when min(n, m) * max_score plus one
    // more substitution score stays below 2^15
    C.i16_limit = h->opt_precision == 32 ? -1 : 32767 - 127;
    C.n_schemes = n_schemes;
    C.n_bins = n_bins;
    HIP_TRY(h, launch_classify(batch->q_off, batch->r_off, batch->scheme_id, P, C, h->d_lut,
                               h->d_keys, h->d_vals, out, d_flags, d_hist, d_maxm, h->d_cells,
                               stream));
    size_t tb = h->temp_bytes;
    HIP_TRY(h, hipcub::DeviceRadixSort::SortPairs(h->d_temp, tb, h->d_keys, h->d_keys2, h->d_vals,
                                                  h->d_vals2, (int)P, 0, 22, stream));
    HIP_TRY(h, hipMemcpyAsync(h->h_small, h->d_small, kSmallInts * 4, hipMemcpyDeviceToHost, stream));
    if (timing) HIP_TRY(h, hipEventRecord(h->ev[1], stream));
    HIP_TRY(h, hipMemcpyAsync(h->h_cells, h->d_cells, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
    HIP_TRY(h, hipStreamSynchronize(stream));
    const int32_t* flags = h->h_small;
    if (flags[kFlagBadOffsets]) return fail(h, SW_EINVAL, "offsets decrease");
    if (flags[kFlagBadScheme]) return fail(h, SW_EINVAL, "scheme id out of range");
    if (flags[kFlagTooLong])
        return fail(h, SW_ETOOLONG, "a query exceeds %d or a reference exceeds %d residues", SW_MAX_QUERY, SW_MAX_REF);
    h->last_fwd = (int64_t)h->h_cells[0];
    if (!batch->queries || !batch->refs) {
        if (h->last_fwd > 0) return fail(h, SW_EINVAL, "null queries or refs with non-empty sequences");
    }

    KParams K;
    K.queries = batch->queries; K.q_off = batch->q_off; K.refs = batch->refs; K.r_off = batch->r_off;
    K.scheme_id = batch->scheme_id; K.order = h->d_vals2; K.out = out; K.flags = d_flags;
    K.mats = h->d_mats; K.validate = (int32_t)h->opt_validate;
    for (int s = 0; s < SW_MAX_SCHEMES; ++s) {
        const bool v = s < n_schemes;
        K.alphabet[s] = v ? schemes[s].alphabet : 1;
        K.gap_open[s] = v ? schemes[s].gap_open : 1;
        K.gap_extend[s] = v ? schemes[s].gap_extend : 0;
    }
    const int32_t* hist = h->h_small + kNumFlags;
    std::vector<int> first(n_bins + 1, 0);
    for (int b = 0; b < n_bins; ++b) first[b + 1] = first[b] + hist[b];
    if (timing) HIP_TRY(h, hipEventRecord(h->ev[2], stream));
    for (int pass = 0; pass < 2; ++pass) {
        for (int b = 0; b < n_bins; ++b) {
            if (hist[b] == 0) continue;
            HIP_TRY(h, launch_pass(h->bins[b], K, first[b], hist[b], pass, stream));
            if (pass == 0 && h->bins[b].prec == 32) h->last_i32 += hist[b];
        }
        if (timing) HIP_TRY(h, hipEventRecord(h->ev[3 + pass], stream));
    }
    HIP_TRY(h, hipMemcpyAsync(h->h_small, h->d_small, kNumFlags * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(h, hipStreamSynchronize(stream));
    if (timing) {
        HIP_TRY(h, hipEventElapsedTime(&h->t_plan, h->ev[0], h->ev[1]));
        HIP_TRY(h, hipEventElapsedTime(&h->t_fwd, h->ev[2], h->ev[3]));
        HIP_TRY(h, hipEventElapsedTime(&h->t_rev, h->ev[3], h->ev[4]));
    }
    if (flags[kFlagBadResidue]) return fail(h, SW_EINVAL, "residue code outside its scheme's alphabet");
    if (flags[kFlagReverseMismatch]) return fail(h, SW_EINTERNAL, "reverse sweep did not reproduce the forward score");
    return SW_OK;
}

int sw_last_stats(sw_handle* h, int64_t* fwd_cells, int64_t* rev_cells, int64_t* int32_pairs) {
    if (!h) return SW_EINVAL;
    if (fwd_cells) *fwd_cells = h->last_fwd;
    if (int32_pairs) *int32_pairs = h->last_i32;
    if (rev_cells) {
        *rev_cells = 0;
        if (h->last_out && h->last_n > 0) {
            HIP_TRY(h, hipSetDevice(h->device));
            HIP_TRY(h, hipMemsetAsync(h->d_cells + 1, 0, sizeof(unsigned long long), h->last_stream));
            HIP_TRY(h, launch_reverse_cells(h->last_out, h->last_n, h->d_cells + 1, h->last_stream));
            HIP_TRY(h, hipMemcpyAsync(h->h_cells, h->d_cells, 2 * sizeof(unsigned long long),
                                      hipMemcpyDeviceToHost, h->last_stream));
            HIP_TRY(h, hipStreamSynchronize(h->last_stream));
            *rev_cells = (int64_t)h->h_cells[1];
        }
    }
    return SW_OK;
}

int sw_last_timing(sw_handle* h, float* plan_ms, float* forward_ms, float* reverse_ms) {
    if (!h) return SW_EINVAL;
    if (plan_ms) *plan_ms = h->t_plan;
    if (forward_ms) *forward_ms = h->t_fwd;
    if (reverse_ms) *reverse_ms = h->t_rev;
    return SW_OK;
}

}  // extern "C"
