// sw_runtime.hip -- host runtime of libswalign: argument checks, launch
// sequencing of the planning and sweep kernels, hipGraph capture and replay,
// error reporting.
//
// One sw_align_batch call, for each of the two passes (forward, reverse):
//   classify -> plan (scan) -> scatter -> items   (sw_plan.hip)
//   sweeps over the work items                    (sw_queue*.hip)
// Persistent mode (default): one queue kernel per bin, longest bins first,
// each sized to the resident capacity of the device (capped by what the
// batch could need); nothing synchronises with the host until the end, and
// the whole sequence can be captured once into a hipGraph and replayed for
// later calls with the same arguments.
// Plain mode: after each pass is planned the host reads the per-bin item
// counts and launches one kernel per non-empty bin, sized to its items.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sw_internal.h"

using namespace sw;

namespace {

std::mutex g_capture_mu;   // one graph capture at a time in the process

// Workspace of sw_align_batch_noalloc: the sort keys, the pair order and the
// work items of up to SW_NOALLOC_MAX_PAIRS pairs, in one array that every
// GPU the library runs on holds from the library's load until the process
// ends.  Host code never names the array: it uses the address that
// hipGetSymbolAddress gives for the current device, looked up once per
// device when the first handle on that device is created.
constexpr int64_t kStaticPairs = SW_NOALLOC_MAX_PAIRS;
constexpr int64_t kStaticKeys = 0;
constexpr int64_t kStaticOrder = kStaticKeys + 4 * kStaticPairs;
constexpr int64_t kStaticItems = kStaticOrder + 4 * kStaticPairs;
constexpr int64_t kStaticBytes = kStaticItems + (kStaticPairs + kMaxBins) * (int64_t)sizeof(WorkItem);
static __device__ __align__(256) uint8_t scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_addr[kMaxDevices] = {};   // per device: the array's device address

// The array's address on `device`, which must be current; nullptr if the
// lookup fails.
static uint8_t* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
            g_scratch_addr[device] = static_cast<uint8_t*>(p);
        else
            (void)hipGetLastError();
    }
    return g_scratch_addr[device];
}

// Where one call's per-pair planning arrays live: the handle's own buffers,
// or the static array of sw_align_batch_noalloc.  Launch grids are sized for
// `cap` pairs.
struct Workspace {
    int32_t* keys;
    int32_t* order;
    WorkItem* items;
    int64_t cap;
};

constexpr int kLutEntries = 2 * kLutRows;
constexpr int kCtrBase = 16;     // int index of the first 64-bit counter
constexpr int kSmallInts = kCtrBase + 2 * kNumCounters;   // flags [0, kNumFlags) | counters

// Everything a captured graph depends on besides device memory contents.
struct GraphKey {
    const void* queries;
    const void* q_beg;
    const void* q_end;
    const void* refs;
    const void* r_beg;
    const void* r_end;
    const void* scheme_id;
    const void* out;
    int64_t cap_pairs;     // grids are sized for it; the batch size itself is read on the device
    int32_t alphabet[SW_MAX_SCHEMES];
    int32_t gap_open[SW_MAX_SCHEMES];
    int32_t gap_extend[SW_MAX_SCHEMES];
    int32_t max_score[SW_MAX_SCHEMES];
    int32_t col_ok[SW_MAX_SCHEMES];
    int32_t n_schemes;
    int32_t validate;
    int32_t precision;
    int32_t ptab_sid;
    int32_t qprof;
    int32_t qprof_n;       // a profile is built for this query length (a kernel argument)
    int32_t search_n;      // every pair's query length (a search: one forward bin), or -1
    int32_t max_query;     // the max_query option (bins above it are not launched)
};

}  // namespace

struct sw_handle {
    int device = 0;
    int n_cu = 0;
    std::string err;
    int64_t opt_mode = 1;
    int64_t opt_graph = 1;
    int64_t opt_validate = 1;
    int64_t opt_precision = 0;
    int64_t opt_timing = 0;
    int64_t opt_streams = 4;
    int64_t opt_max_query = 0;          // 0, or the caller's bound on query lengths
    std::vector<int> bin_min_query;     // per bin: the shortest query any route sends to it
    int64_t opt_colpath = 1;

    std::vector<BinInfo> bins;
    std::vector<int> route[2];          // per precision (int16, int32) and 16-row bucket: bin
    std::vector<int8_t> lut;            // device copy of route
    std::vector<char> bin_used;         // bins some route points at
    bool lut_dirty = true;
    std::vector<int> resident_blocks[2][2][kNumVars];   // per tile, pass, score source and bin: workgroups the device holds at once
    std::vector<std::pair<QueueFn, int>> fam_resident;  // per family kernel: workgroups the device holds at once
    int64_t opt_families = 1;
    int64_t opt_chunk = kChunk;         // reference tile of 16- and 32-lane packed shapes: kChunk or kChunkNarrow
    int64_t opt_ptab = 1;
    int64_t opt_qprof = 1;
    int32_t last_ptab = 0;              // the last call's table-range kernels used the pair table
    int32_t last_qprof = 0;             // the last call's forward pass used the query profile

    int8_t* d_mats = nullptr;
    int8_t* d_lut = nullptr;
    BinInfo* d_bins = nullptr;
    int32_t* d_small = nullptr;
    int32_t* d_n = nullptr;       // batch size, written by the call-start kernel of each call
    int32_t* d_hist = nullptr;
    int32_t* d_meta = nullptr;
    int32_t* d_keys = nullptr;
    int32_t* d_order = nullptr;
    WorkItem* d_items = nullptr;
    int64_t cap_pairs = 0;
    uint8_t* d_scratch = nullptr;     // this device's address of the static workspace (sw_align_batch_noalloc)

    int32_t* h_small = nullptr;   // pinned (alignment paths)
    int32_t* h_meta = nullptr;    // pinned
    std::vector<int8_t> dev_mats;       // what d_mats holds (or will, in stream order) after the last upload
    std::vector<int8_t> tables;         // the current call's tables, built on the host

    // Calls in flight (sw_submit): each holds one slot until it is polled,
    // or completed by a later submit that needs the slot.  A slot's pinned
    // buffers receive the call's scheme tables (when they must be uploaded)
    // and its flags and counters; its event marks the end of the call.
    struct CallSlot {
        uint64_t ticket = 0;           // 0 = free
        hipEvent_t done = nullptr;
        int32_t* h_small = nullptr;    // pinned: flags and counters of the call
        int8_t* h_mats = nullptr;      // pinned: staging of the scheme tables
        bool timing = false;
        bool ptab = false;             // its table-range kernels used the pair table
        bool qprof = false;            // its forward pass used the query profile
        int chunk = kChunk;            // its "chunk" option
        std::chrono::steady_clock::time_point t_entry;
    };
    static constexpr int kSlots = 8;
    CallSlot slots[kSlots];
    uint64_t next_ticket = 1;
    int next_slot = 0;
    int last_slot = -1;                 // slot of the last submitted call
    hipStream_t last_stream = nullptr;
    struct Finished { int status; std::string err; };
    std::map<uint64_t, Finished> finished;   // completed but not yet polled
    int8_t* h_lut = nullptr;      // pinned staging of the routing table (sw_align_batch_noalloc)

    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float t_plan = 0.f, t_fwd = 0.f, t_rev = 0.f;
    double t_enqueue = 0.0, t_wait = 0.0;   // host milliseconds of the last call
    // per (pass, bin) event pairs for "timing" = 2, created on first use
    std::vector<hipEvent_t> bin_ev;
    std::vector<char> bin_launched;     // per (pass, bin, variant) of the last call
    // per (pass, bin, variant) of the last enqueued call: the launch that
    // swept the bin (index within its pass, or -1), the family of a family
    // launch (rows per lane of its first and last shape, else 0) and its
    // event slot ("timing" = 2)
    static constexpr int kFamLaunches = 16;
    std::vector<int32_t> bin_launch, bin_fam_hi, bin_fam_lo, bin_fam_slot, bin_fam_waves, bin_fam_tile;
    std::vector<hipEvent_t> fam_ev;     // [pass][kFamLaunches][start, end]
    std::vector<sw_bin_stat> bin_stats;

    hipStream_t cap_stream = nullptr;   // private stream the graph is captured on
    static constexpr int kForks = 8;    // persistent mode spreads bins over up to this many streams
    hipStream_t fork[kForks] = {};
    hipEvent_t fork_ev[kForks + 1] = {};
    // captured calls, most recently used last (at most kGraphs)
    struct GraphEntry {
        GraphKey key;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    static constexpr int kGraphs = 4;
    std::vector<GraphEntry> graphs;
    int64_t n_captures = 0;
    int64_t n_capture_refusals = 0;

    int64_t last_fwd = 0, last_rev = 0, last_i32 = 0;

    // alignment paths (sw_align_cigar)
    std::vector<BinInfo> tbins;          // path-sweep shapes
    std::vector<int> tresident;          // workgroups the device holds at once, per path-sweep bin
    std::vector<int> tresident_col;      // and for its column-word kernel
    std::vector<int> tbin_min_rows;      // per path-sweep bin: the fewest box rows the routing sends to it
    std::vector<std::pair<TraceFn, int>> tfam_resident;   // per box-sweep family kernel
    std::vector<int> tfam_first;         // per path-sweep bin of the last chunk: first bin of its family launch, or -1
    static constexpr int kTraceFams = 8; // box-sweep family launches per chunk at most
    hipEvent_t tfam_ev[kTraceFams] = {}; // end of a box-sweep family launch, for its walks on other streams
    int32_t last_col_ok[SW_MAX_SCHEMES] = {0};   // column-word eligibility of the last score call's schemes
    BinInfo* d_tbins = nullptr;
    int8_t* d_tlut = nullptr;            // [2 * kLutRows] path-sweep bin per (precision, 16-row bucket of box rows)
    int64_t* d_rec_off = nullptr;        // [trace_cap + 1]
    int64_t* d_bsum = nullptr;           // [scan blocks + 1]
    int64_t trace_cap = 0;
    uint8_t* d_ws = nullptr;             // path records of one chunk
    int64_t ws_alloc = 0;
    int64_t opt_path_ws = (int64_t)32 << 30;   // set to half the device's memory at creation
    int64_t* h_i64 = nullptr;            // pinned
    std::vector<hipEvent_t> tbin_ev;     // per path-sweep bin: sweep start, sweep end, walk end ("timing")
    int64_t last_path_cells = 0, last_path_bytes = 0;
    int32_t last_path_chunks = 0;
    float t_path_sweep = 0.f, t_path_walk = 0.f;

    // database search (sw_search): the shared query's span for every pair
    int64_t* d_qspan = nullptr;          // [2 * search_cap]: begins, then ends
    int64_t search_cap = 0;
    int64_t search_len = -1;             // query length the spans hold
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

// 64-bit counters live in d_small from int index kCtrBase (layout kCtr*).
static unsigned long long* counters(int32_t* small) {
    return reinterpret_cast<unsigned long long*>(small + kCtrBase);
}

static void build_bins(sw_handle* h) {
    // Bins run longest work first: int16 before int32, then decreasing rows
    // per group (W * R), wider groups first at equal rows.
    int n = 0;
    const ShapeDesc* sh = compiled_shapes(&n);
    std::vector<ShapeDesc> v(sh, sh + n);
    std::stable_sort(v.begin(), v.end(), [](const ShapeDesc& a, const ShapeDesc& b) {
        if (a.prec != b.prec) return a.prec < b.prec;
        if (a.W * a.R != b.W * b.R) return a.W * a.R > b.W * b.R;
        return a.W > b.W;
    });
    h->bins.clear();
    for (const ShapeDesc& s : v) {
        BinInfo b;
        b.prec = (uint8_t)s.prec;
        b.W = (uint16_t)s.W;
        b.R = (uint8_t)s.R;
        b.ppw = (uint16_t)pairs_per_item(s.prec, s.W);
        b.col = shape_kernel(s.prec, s.W, s.R, false, kVarCol) != nullptr ? 1 : 0;
        b.ptab = shape_kernel(s.prec, s.W, s.R, false, kVarPtab) != nullptr ? 1 : 0;
        h->bins.push_back(b);
    }
}

static int find_bin(const sw_handle* h, int prec, int W, int R) {
    for (int b = 0; b < (int)h->bins.size(); ++b)
        if (h->bins[b].prec == prec && h->bins[b].W == W && h->bins[b].R == R) return b;
    return -1;
}

// Default routing of one precision: each 16-row bucket goes to the covering
// shape with the fewest lane-row slots per pair, W*R*(m + W - 1), for a
// reference of twice the query length plus 64 (the sweep of a W-lane group
// takes m + W - 1 steps).  Ties go to the narrower group.  Queries above 512
// rows go to cooperative 256-lane groups when they are compiled: their
// per-pair latency is about four times shorter than a 64-lane group's, and
// that latency bounds small batches and the tails of large ones.
// The int32 routing uses six shapes of 64 to 2048 rows (doubling): int32
// pairs are rare unless a call forces the precision (references above
// kI16MaxRef, or scores past the packed range), and every bin a route uses
// costs a launch per pass in every call, with work or without.
static bool coarse_i32_shape(const BinInfo& e) {
    const int rows = e.W * e.R;
    return (e.W == 16 && (rows == 64 || rows == 128 || rows == 256)) ||
           (e.W == 64 && (rows == 512 || rows == 1024 || rows == 2048));
}

static void default_routing(sw_handle* h, int sel) {
    const int prec = sel == 0 ? 16 : 32;
    for (int k = 0; k < kLutRows; ++k) {
        const int rows = 16 * (k + 1);
        const double m = 2.0 * rows + 64.0;
        int best = -1;
        double best_cost = 0;
        bool have_coop = false;
        for (const BinInfo& e : h->bins)
            have_coop |= e.prec == prec && e.W > 64 && e.W * e.R >= rows;
        const bool coop = have_coop && rows > 512;
        for (int b = 0; b < (int)h->bins.size(); ++b) {
            const BinInfo& e = h->bins[b];
            if (e.prec != prec || e.W * e.R < rows || (e.W > 64) != coop) continue;
            if (sel == 1 && !coarse_i32_shape(e)) continue;
            const double cost = (double)e.W * e.R * (m + e.W - 1);
            if (best < 0 || cost < best_cost || (cost == best_cost && e.W < h->bins[best].W)) {
                best = b;
                best_cost = cost;
            }
        }
        h->route[sel][k] = best;
    }
}

static void rebuild_lut(sw_handle* h) {
    h->lut.assign(kLutEntries, -1);
    h->bin_used.assign(h->bins.size(), 0);
    h->bin_min_query.assign(h->bins.size(), SW_MAX_QUERY + 1);
    for (int sel = 0; sel < 2; ++sel)
        for (int k = 0; k < kLutRows; ++k) {
            const int b = h->route[sel][k];
            h->lut[sel * kLutRows + k] = (int8_t)b;
            if (b >= 0) {
                h->bin_used[b] = 1;
                h->bin_min_query[b] = std::min(h->bin_min_query[b], 16 * k + 1);
            }
        }
    h->lut_dirty = true;
}

// Install a routing table for one precision (sel 0 = int16, 1 = int32):
// queries of rows_max[k-1]+1 .. rows_max[k] residues go to shape
// (lanes[k], rows[k]).  n == 0 restores the default.
static int set_routing(sw_handle* h, int sel, const int32_t* rows_max, const int32_t* lanes,
                       const int32_t* rows, int n) {
    const int prec = sel == 0 ? 16 : 32;
    if (n == 0) {
        default_routing(h, sel);
        rebuild_lut(h);
        return SW_OK;
    }
    if (n < 0 || n > kLutRows || !rows_max || !lanes || !rows)
        return fail(h, SW_EINVAL, "routing needs 1..%d entries", kLutRows);
    std::vector<int> r(kLutRows, -1);
    int prev = 0;
    for (int e = 0; e < n; ++e) {
        const int hi = rows_max[e];
        if (hi <= prev || hi % 16 != 0 || hi > SW_MAX_QUERY)
            return fail(h, SW_EINVAL, "routing entry %d: rows_max must increase in steps of 16 up to %d", e,
                        SW_MAX_QUERY);
        const int b = find_bin(h, prec, lanes[e], rows[e]);
        if (b < 0) return fail(h, SW_EINVAL, "routing entry %d: no compiled int%d shape %dx%d", e, prec, lanes[e], rows[e]);
        if (lanes[e] * rows[e] < hi)
            return fail(h, SW_EINVAL, "routing entry %d: shape %dx%d covers %d rows, fewer than %d", e, lanes[e],
                        rows[e], lanes[e] * rows[e], hi);
        for (int k = prev / 16; k < hi / 16; ++k) r[k] = b;
        prev = hi;
    }
    if (prev != SW_MAX_QUERY) return fail(h, SW_EINVAL, "routing must end at rows_max = %d", SW_MAX_QUERY);
    for (int k = 0; k < kLutRows; ++k) h->route[sel][k] = r[k];
    rebuild_lut(h);
    return SW_OK;
}

// "16x4@64/16x8@128/..." -> routing entries (shape W x R up to rows_max)
static int parse_routing(sw_handle* h, int sel, const std::string& v) {
    std::vector<int32_t> hi, W, R;
    size_t pos = 0;
    while (pos < v.size()) {
        size_t end = v.find('/', pos);
        if (end == std::string::npos) end = v.size();
        int a = 0, b = 0, c = 0;
        if (sscanf(v.substr(pos, end - pos).c_str(), "%dx%d@%d", &a, &b, &c) != 3)
            return fail(h, SW_EINVAL, "bad routing entry '%s'", v.substr(pos, end - pos).c_str());
        W.push_back(a); R.push_back(b); hi.push_back(c);
        pos = end + 1;
    }
    return set_routing(h, sel, hi.data(), W.data(), R.data(), (int)hi.size());
}

static void free_dev(void* p) {
    if (p) (void)hipFree(p);
}

static int complete_slot(sw_handle* h, int k);

// Wait for every call in flight on the handle; their statuses are kept
// for sw_poll.  Needed before anything they may still use is freed,
// replaced or rewritten from the host.
static void drain(sw_handle* h) {
    for (int k = 0; k < sw_handle::kSlots; ++k) {
        sw_handle::CallSlot& sl = h->slots[k];
        if (!sl.ticket) continue;
        const uint64_t t = sl.ticket;
        (void)hipEventSynchronize(sl.done);
        const int st = complete_slot(h, k);
        h->finished[t] = sw_handle::Finished{st, h->err};
    }
    h->err.clear();
}

static void drop_graph(sw_handle* h) {
    drain(h);
    for (sw_handle::GraphEntry& g : h->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    h->graphs.clear();
}

static int ensure_pairs(sw_handle* h, int64_t n) {
    if (n <= h->cap_pairs) return SW_OK;
    drop_graph(h);
    free_dev(h->d_keys); free_dev(h->d_order); free_dev(h->d_items);
    h->d_keys = h->d_order = nullptr; h->d_items = nullptr;
    h->cap_pairs = 0;
    const int64_t cap = std::max<int64_t>(n, 4096);
    if (hipMalloc(&h->d_keys, cap * 4) != hipSuccess || hipMalloc(&h->d_order, cap * 4) != hipSuccess ||
        hipMalloc(&h->d_items, (cap + kMaxBins) * sizeof(WorkItem)) != hipSuccess)
        return fail(h, SW_ENOMEM, "device allocation of %lld pair slots failed", (long long)cap);
    h->cap_pairs = cap;
    return SW_OK;
}

// Item range and queue head of bin b's column-word kernel (v = 1) or
// table-lookup kernel (v = 0).
static void set_range(KParams& K, int b, int v) {
    K.lo_idx = v ? kMetaItemFirst + b : kMetaItemSplit + b;
    K.hi_idx = v ? kMetaItemSplit + b : kMetaItemFirst + b + 1;
    K.head_idx = v ? kMetaColHeads + b : kMetaHeads + b;
}

// Workgroups the device holds at once of family kernel fn (0 if unknown).
static int family_resident(const sw_handle* h, QueueFn fn) {
    for (const auto& e : h->fam_resident)
        if (e.first == fn) return e.second;
    return 0;
}

static int bin_ev_index(int pass, int b, int v, int end) { return ((pass * kMaxBins + b) * 2 + v) * 2 + end; }

// Score source of bin e's kernel for its column-word range (v = 1) or its
// other range: the query profile in the forward pass of a search, else the
// pair table when the call has one, else table lookups.
static int table_var(const sw_handle* h, const BinInfo& e, const KParams& K, int v) {
    (void)h;
    if (v == 1) return kVarCol;
    if (K.qprof && !K.reverse && shape_kernel(e.prec, e.W, e.R, false, kVarQprof) != nullptr) return kVarQprof;
    return e.ptab && K.ptab_sid >= 0 ? kVarPtab : kVarTable;
}

// 1 when bin e's kernel of score source `var` runs with the narrow
// reference tile (the "chunk" option; only 16- and 32-lane packed shapes
// have it).
static int narrow_tile(const sw_handle* h, const BinInfo& e, int var) {
    return h->opt_chunk == kChunkNarrow && shape_kernel(e.prec, e.W, e.R, false, var, true) != nullptr ? 1 : 0;
}

// Enqueue one pass (planning + sweeps).  Plain mode synchronises `stream`
// once to read the per-bin item counts.
static int enqueue_pass(sw_handle* h, KParams K, const ClassifyArgs& C, const Workspace& ws, int pass,
                        hipStream_t stream, bool timing, int64_t search_n) {
    K.reverse = pass;
    const int64_t cap = ws.cap;
    const int n_bins = (int)h->bins.size();
    HIP_TRY(h, launch_reset(h->d_hist, kHistSize, stream));
    HIP_TRY(h, launch_classify(K, C, h->d_lut, h->d_bins, cap, ws.keys, h->d_hist, counters(h->d_small), stream));
    HIP_TRY(h, launch_plan_bins(h->d_bins, n_bins, h->d_hist, h->d_meta, counters(h->d_small), pass, stream));
    HIP_TRY(h, launch_scatter(ws.keys, h->d_n, cap, h->d_hist, ws.order, stream));
    HIP_TRY(h, launch_items(h->d_meta, h->d_bins, n_bins, h->d_n, cap, ws.items, stream));
    const bool per_bin = timing && h->opt_timing == 2;
    if (h->bin_launch.size() != (size_t)(2 * kMaxBins * 2)) {
        h->bin_launch.assign(2 * kMaxBins * 2, -1);
        h->bin_fam_hi.assign(2 * kMaxBins * 2, 0);
        h->bin_fam_lo.assign(2 * kMaxBins * 2, 0);
        h->bin_fam_slot.assign(2 * kMaxBins * 2, -1);
        h->bin_fam_waves.assign(2 * kMaxBins * 2, 0);
        h->bin_fam_tile.assign(2 * kMaxBins * 2, 0);
    }
    for (int i = pass * kMaxBins * 2; i < (pass + 1) * kMaxBins * 2; ++i) {
        h->bin_launch[i] = -1;
        h->bin_fam_hi[i] = h->bin_fam_lo[i] = h->bin_fam_waves[i] = h->bin_fam_tile[i] = 0;
        h->bin_fam_slot[i] = -1;
    }
    int n_launch = 0;   // launches of this pass
    if (timing && h->opt_mode == 1) HIP_TRY(h, hipEventRecord(h->ev[pass == 0 ? 1 : 3], stream));
    if (h->opt_mode == 1) {
        // Bins go round-robin, longest first, to the forked streams, which
        // are joined back into `stream`: the bins' launch tails, and the
        // launches of bins that turn out to be empty, overlap with the work
        // of the other streams.  Per-launch timing serialises them.
        const int forks = per_bin ? 0 : (int)h->opt_streams;
        int launched = 0;
        // A bin's column-word items exist only when some scheme of the call
        // takes column words, and its other items only when some scheme does
        // not: the launches that cannot have work are left out (each one is
        // a graph node, and every node delays the start of its branch).
        bool any_col = false, all_col = true;
        for (int s = 0; s < C.n_schemes; ++s) {
            any_col |= C.col_ok[s] != 0;
            all_col &= C.col_ok[s] != 0;
        }
        if (forks > 1) {
            HIP_TRY(h, hipEventRecord(h->fork_ev[sw_handle::kForks], stream));
            for (int f = 0; f < forks; ++f)
                HIP_TRY(h, hipStreamWaitEvent(h->fork[f], h->fork_ev[sw_handle::kForks], 0));
        }
        // In the forward pass of a search every pair has the query's length,
        // so its pairs are in that length's int16 or int32 bin: only those
        // two are launched.
        int only16 = -1, only32 = -1;
        const bool one_length = pass == 0 && search_n >= 1 && search_n <= SW_MAX_QUERY;
        if (one_length) {
            only16 = h->route[0][(search_n - 1) / 16];
            only32 = h->route[1][(search_n - 1) / 16];
        }
        std::vector<char> launchable(n_bins, 0);
        for (int b = 0; b < n_bins; ++b)
            launchable[b] = h->bin_used[b] && !(one_length && b != only16 && b != only32) &&
                            !(h->opt_max_query > 0 && h->bin_min_query[b] > h->opt_max_query);
        // Family launches (default tile): one kernel per family, score
        // source and pass takes the items of all its launchable member bins;
        // the bins it covers get no launch of their own below.
        std::vector<char> covered(2 * n_bins, 0);
        int fam_slot = 0;
        if (h->opt_families && h->opt_chunk == kChunk) {
            std::vector<const FamilyEntry*> seen;
            for (int b = 0; b < n_bins; ++b) {
                if (!launchable[b]) continue;
                const FamilyEntry* f = shape_family(h->bins[b].prec, h->bins[b].W, h->bins[b].R);
                if (!f || std::find(seen.begin(), seen.end(), f) != seen.end()) continue;
                seen.push_back(f);
                for (int v = 1; v >= 0; --v) {
                    int var = -1, members = 0;
                    for (int k = 0; k < kFamilyMax; ++k) K.fam_bins[k] = -1;
                    for (int k = 0; k < f->n; ++k) {
                        const int mb = find_bin(h, f->prec, f->W, f->rows[k]);
                        if (mb < 0 || !launchable[mb]) continue;
                        const BinInfo& m = h->bins[mb];
                        if (v == 1 ? !(any_col && m.col) : (m.col && all_col)) continue;
                        const int mv = table_var(h, m, K, v);
                        if (mv == kVarQprof || (var >= 0 && mv != var)) continue;
                        var = mv;
                        K.fam_bins[k] = (int8_t)mb;
                        ++members;
                    }
                    // a family of one routed bin gains nothing over that
                    // shape's own kernel (measured: small batches on three
                    // bins of different widths ran 15% slower)
                    if (members < 2 || !f->k[var][pass] || fam_slot >= sw_handle::kFamLaunches) continue;
                    for (int k = 0; k < f->n; ++k) {
                        const int mb = K.fam_bins[k];
                        if (mb < 0) continue;
                        covered[2 * mb + v] = 1;
                        const int i2 = bin_ev_index(pass, mb, v, 0) / 2;
                        h->bin_launch[i2] = n_launch;
                        h->bin_fam_hi[i2] = f->rows[0];
                        h->bin_fam_lo[i2] = f->rows[f->n - 1];
                        h->bin_fam_slot[i2] = fam_slot;
                        h->bin_fam_waves[i2] = f->waves[var];
                        h->bin_fam_tile[i2] = f->tile[var];
                    }
                    const QueueFn fn = f->k[var][pass];
                    const int ppw = pairs_per_item(f->prec, f->W), ipb = items_per_block(f->W);
                    const int64_t need = (cap / ppw + 1 + ipb - 1) / ipb;
                    const int blocks = (int)std::min<int64_t>(need, std::max(1, family_resident(h, fn)));
                    hipStream_t ls = forks > 1 ? h->fork[launched % forks] : stream;
                    hipEvent_t* fe = per_bin ? &h->fam_ev[(pass * sw_handle::kFamLaunches + fam_slot) * 2] : nullptr;
                    if (fe) HIP_TRY(h, hipEventRecord(fe[0], ls));
                    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), 0, ls, K);
                    HIP_TRY(h, hipGetLastError());
                    if (fe) HIP_TRY(h, hipEventRecord(fe[1], ls));
                    ++launched;
                    ++n_launch;
                    ++fam_slot;
                }
            }
        }
        for (int b = 0; b < n_bins; ++b) {
            if (!launchable[b]) continue;
            const BinInfo& e = h->bins[b];
            // no bin can hold more than cap / ppw items
            const int ipb = items_per_block(e.W);
            const int64_t need = (cap / e.ppw + 1 + ipb - 1) / ipb;
            bool any = false;
            for (int v = e.col ? 1 : 0; v >= 0; --v) {   // column-word kernel first
                if (v == 1 ? !any_col : (e.col && all_col)) continue;
                if (covered[2 * b + v]) continue;
                any = true;
                const int var = table_var(h, e, K, v);
                const int nw = narrow_tile(h, e, var);
                const int blocks = (int)std::min<int64_t>(need, h->resident_blocks[nw][pass][var][b]);
                set_range(K, b, v);
                h->bin_launch[bin_ev_index(pass, b, v, 0) / 2] = n_launch++;
                // a bin's kernels share a stream; bins go round-robin
                hipStream_t ls = forks > 1 ? h->fork[launched % forks] : stream;
                if (per_bin) HIP_TRY(h, hipEventRecord(h->bin_ev[bin_ev_index(pass, b, v, 0)], ls));
                hipLaunchKernelGGL(shape_kernel(e.prec, e.W, e.R, pass != 0, var, nw == 1), dim3(blocks), dim3(kBlock),
                                   0, ls, K);
                HIP_TRY(h, hipGetLastError());
                if (per_bin) HIP_TRY(h, hipEventRecord(h->bin_ev[bin_ev_index(pass, b, v, 1)], ls));
                if (per_bin) h->bin_launched[bin_ev_index(pass, b, v, 0) / 2] = 1;
            }
            if (any) ++launched;
        }
        for (int f = 0; forks > 1 && f < forks; ++f) {
            HIP_TRY(h, hipEventRecord(h->fork_ev[f], h->fork[f]));
            HIP_TRY(h, hipStreamWaitEvent(stream, h->fork_ev[f], 0));
        }
    } else {
        HIP_TRY(h, hipMemcpyAsync(h->h_meta, h->d_meta, kMetaSize * 4, hipMemcpyDeviceToHost, stream));
        HIP_TRY(h, hipStreamSynchronize(stream));
        if (timing) HIP_TRY(h, hipEventRecord(h->ev[pass == 0 ? 1 : 3], stream));
        for (int b = 0; b < n_bins; ++b) {
            const BinInfo& e = h->bins[b];
            for (int v = e.col ? 1 : 0; v >= 0; --v) {
                set_range(K, b, v);
                const int items = h->h_meta[K.hi_idx] - h->h_meta[K.lo_idx];
                if (items <= 0) continue;
                const int blocks = (items + items_per_block(e.W) - 1) / items_per_block(e.W);
                const int var = table_var(h, e, K, v);
                const int nw = narrow_tile(h, e, var);
                h->bin_launch[bin_ev_index(pass, b, v, 0) / 2] = n_launch++;
                if (per_bin) HIP_TRY(h, hipEventRecord(h->bin_ev[bin_ev_index(pass, b, v, 0)], stream));
                hipLaunchKernelGGL(shape_kernel(e.prec, e.W, e.R, pass != 0, var, nw == 1), dim3(blocks), dim3(kBlock),
                                   0, stream, K);
                HIP_TRY(h, hipGetLastError());
                if (per_bin) HIP_TRY(h, hipEventRecord(h->bin_ev[bin_ev_index(pass, b, v, 1)], stream));
                if (per_bin) h->bin_launched[bin_ev_index(pass, b, v, 0) / 2] = 1;
            }
        }
    }
    if (timing) HIP_TRY(h, hipEventRecord(h->ev[pass == 0 ? 2 : 4], stream));
    return SW_OK;
}

// Path-sweep bins and their routing: for each precision (packed int16,
// int32), each 16-row bucket of box rows goes to the covering shape with the
// fewest lane-row slots for a box of as many columns plus 32 (a result box
// is about as wide as it is tall).
static bool init_paths(sw_handle* h) {
    int n = 0;
    const ShapeDesc* sh = trace_shapes(&n);
    h->tbins.clear();
    for (int k = 0; k < n; ++k) {
        BinInfo b;
        b.prec = (uint8_t)sh[k].prec;
        b.W = (uint16_t)sh[k].W;
        b.R = (uint8_t)sh[k].R;
        b.ppw = (uint16_t)pairs_per_item(sh[k].prec, sh[k].W);
        b.col = trace_kernel(sh[k].prec, sh[k].W, sh[k].R, true) != nullptr ? 1 : 0;
        b.ptab = 0;
        h->tbins.push_back(b);
    }
    if (h->tbins.empty() || h->tbins.size() > (size_t)kMaxBins) return false;
    std::vector<int8_t> lut(2 * kLutRows, -1);
    for (int sel = 0; sel < 2; ++sel)
        for (int k = 0; k < kLutRows; ++k) {
            const int rows = 16 * (k + 1);
            const double m = rows + 32.0;
            int best = -1;
            double best_cost = 0;
            for (int b = 0; b < (int)h->tbins.size(); ++b) {
                const BinInfo& e = h->tbins[b];
                if (e.prec != (sel == 0 ? 16 : 32) || e.W * e.R < rows) continue;
                const double cost = (double)e.W * e.R * (m + e.W - 1);
                if (best < 0 || cost < best_cost) { best = b; best_cost = cost; }
            }
            if (best < 0) return false;
            lut[sel * kLutRows + k] = (int8_t)best;
        }
    h->tbin_min_rows.assign(h->tbins.size(), SW_MAX_QUERY + 1);
    for (int sel = 0; sel < 2; ++sel)
        for (int k = 0; k < kLutRows; ++k) {
            const int b = lut[sel * kLutRows + k];
            h->tbin_min_rows[b] = std::min(h->tbin_min_rows[b], 16 * k + 1);
        }
    h->tresident.assign(h->tbins.size(), 1);
    h->tresident_col.assign(h->tbins.size(), 1);
    for (size_t b = 0; b < h->tbins.size(); ++b) {
        for (int v = 0; v < 2; ++v) {
            if (v == 1 && !h->tbins[b].col) continue;
            int per_cu = 0;
            const TraceFn fn = trace_kernel(h->tbins[b].prec, h->tbins[b].W, h->tbins[b].R, v == 1);
            if (!fn ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kBlock, 0) != hipSuccess)
                return false;
            (v ? h->tresident_col : h->tresident)[b] = std::max(1, per_cu) * std::max(1, h->n_cu);
            const TraceFamily* f = trace_family(h->tbins[b].prec, h->tbins[b].W, h->tbins[b].R);
            const TraceFn ff = f ? (v ? f->col : f->fn) : nullptr;
            bool have = !ff;
            for (const auto& e : h->tfam_resident) have |= e.first == ff;
            if (!have) {
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)ff, kBlock, 0) != hipSuccess)
                    return false;
                h->tfam_resident.push_back({ff, std::max(1, per_cu) * std::max(1, h->n_cu)});
            }
        }
    }
    bool ok = hipMalloc(&h->d_tbins, kMaxBins * sizeof(BinInfo)) == hipSuccess &&
              hipMalloc(&h->d_tlut, 2 * kLutRows) == hipSuccess &&
              hipHostMalloc(&h->h_i64, 16, hipHostMallocDefault) == hipSuccess &&
              hipMemcpy(h->d_tbins, h->tbins.data(), h->tbins.size() * sizeof(BinInfo), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(h->d_tlut, lut.data(), 2 * kLutRows, hipMemcpyHostToDevice) == hipSuccess;
    return ok;
}

extern "C" {

sw_handle* sw_create(int device, const char* tuning) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return nullptr;
    if (hipSetDevice(device) != hipSuccess) return nullptr;
    sw_handle* h = new sw_handle();
    h->device = device;
    h->d_scratch = scratch_address(device);
    hipDeviceProp_t prop;
    bool ok = hipGetDeviceProperties(&prop, device) == hipSuccess;
    h->n_cu = ok ? prop.multiProcessorCount : 0;
    // path-record workspace: half the device's memory (144 GiB on a 288 GB
    // MI355X), so that a batch's records usually fit in one chunk; each
    // chunk costs its own planning and walk tails
    if (ok && prop.totalGlobalMem / 2 > (size_t)h->opt_path_ws) h->opt_path_ws = (int64_t)(prop.totalGlobalMem / 2);
    build_bins(h);
    for (int sel = 0; sel < 2; ++sel) {
        h->route[sel].assign(kLutRows, -1);
        default_routing(h, sel);
    }
    rebuild_lut(h);
    ok = ok && h->bins.size() <= (size_t)kMaxBins &&
         hipMalloc(&h->d_mats, kSchemeBytes) == hipSuccess &&
         hipMalloc(&h->d_lut, kLutEntries) == hipSuccess &&
         hipMalloc(&h->d_bins, kMaxBins * sizeof(BinInfo)) == hipSuccess &&
         hipMalloc(&h->d_small, kSmallInts * 4) == hipSuccess &&
         hipMalloc(&h->d_n, 16) == hipSuccess &&
         hipHostMalloc(&h->h_lut, kLutEntries, hipHostMallocDefault) == hipSuccess &&
         hipMalloc(&h->d_hist, kHistSize * 4) == hipSuccess &&
         hipMalloc(&h->d_meta, kMetaSize * 4) == hipSuccess &&
         hipHostMalloc(&h->h_small, kSmallInts * 4, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc(&h->h_meta, kMetaSize * 4, hipHostMallocDefault) == hipSuccess;
    for (int k = 0; ok && k < sw_handle::kSlots; ++k) {
        sw_handle::CallSlot& sl = h->slots[k];
        ok = hipHostMalloc(&sl.h_small, kSmallInts * 4, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc(&sl.h_mats, kSchemeBytes, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
    }
    for (int k = 0; ok && k < 5; ++k) ok = hipEventCreate(&h->ev[k]) == hipSuccess;
    for (int f = 0; ok && f < sw_handle::kForks; ++f)
        ok = hipStreamCreateWithFlags(&h->fork[f], hipStreamNonBlocking) == hipSuccess;
    for (int f = 0; ok && f <= sw_handle::kForks; ++f)
        ok = hipEventCreateWithFlags(&h->fork_ev[f], hipEventDisableTiming) == hipSuccess;
    for (int f = 0; ok && f < sw_handle::kTraceFams; ++f)
        ok = hipEventCreateWithFlags(&h->tfam_ev[f], hipEventDisableTiming) == hipSuccess;
    if (ok) ok = hipMemcpy(h->d_bins, h->bins.data(), h->bins.size() * sizeof(BinInfo),
                           hipMemcpyHostToDevice) == hipSuccess;
    for (int nw = 0; nw < 2; ++nw)
        for (int pass = 0; pass < 2; ++pass)
            for (int v = 0; v < kNumVars; ++v) {
                h->resident_blocks[nw][pass][v].assign(h->bins.size(), 1);
                for (size_t b = 0; ok && b < h->bins.size(); ++b) {
                    if ((v == kVarCol && !h->bins[b].col) || (v == kVarPtab && !h->bins[b].ptab)) continue;
                    const QueueFn fn = shape_kernel(h->bins[b].prec, h->bins[b].W, h->bins[b].R, pass != 0, v, nw == 1);
                    if (!fn) {
                        ok = nw == 1 || v == kVarQprof;   // only the narrow tile and reverse profiles may be missing
                        continue;
                    }
                    int per_cu = 0;
                    ok = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kBlock, 0) == hipSuccess;
                    h->resident_blocks[nw][pass][v][b] = std::max(1, per_cu) * std::max(1, h->n_cu);
                }
            }
    for (size_t b = 0; ok && b < h->bins.size(); ++b) {
        const FamilyEntry* f = shape_family(h->bins[b].prec, h->bins[b].W, h->bins[b].R);
        for (int var = 0; f && ok && var <= kVarPtab; ++var)
            for (int pass = 0; pass < 2; ++pass) {
                const QueueFn fn = f->k[var][pass];
                if (!fn || family_resident(h, fn) > 0) continue;
                int per_cu = 0;
                ok = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kBlock, 0) == hipSuccess;
                h->fam_resident.push_back({fn, std::max(1, per_cu) * std::max(1, h->n_cu)});
            }
    }
    if (ok) ok = init_paths(h);
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
                const std::string key = kv.substr(0, eq), val = kv.substr(eq + 1);
                int rc;
                if (key == "route16") rc = parse_routing(h, 0, val);
                else if (key == "route32") rc = parse_routing(h, 1, val);
                else rc = sw_set_option(h, key.c_str(), atoll(val.c_str()));
                if (rc != SW_OK) {
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
    drop_graph(h);
    free_dev(h->d_mats); free_dev(h->d_lut); free_dev(h->d_bins); free_dev(h->d_small); free_dev(h->d_n);
    if (h->h_lut) (void)hipHostFree(h->h_lut);
    for (int k = 0; k < sw_handle::kSlots; ++k) {
        sw_handle::CallSlot& sl = h->slots[k];
        if (sl.h_small) (void)hipHostFree(sl.h_small);
        if (sl.h_mats) (void)hipHostFree(sl.h_mats);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    free_dev(h->d_hist); free_dev(h->d_meta); free_dev(h->d_keys); free_dev(h->d_order);
    free_dev(h->d_items);
    free_dev(h->d_tbins); free_dev(h->d_tlut); free_dev(h->d_rec_off); free_dev(h->d_bsum); free_dev(h->d_ws);
    free_dev(h->d_qspan);
    if (h->h_i64) (void)hipHostFree(h->h_i64);
    for (hipEvent_t e : h->tbin_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->h_small) (void)hipHostFree(h->h_small);
    if (h->h_meta) (void)hipHostFree(h->h_meta);
    for (int k = 0; k < 5; ++k)
        if (h->ev[k]) (void)hipEventDestroy(h->ev[k]);
    for (hipEvent_t e : h->fam_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->tfam_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->bin_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (int f = 0; f < sw_handle::kForks; ++f)
        if (h->fork[f]) (void)hipStreamDestroy(h->fork[f]);
    for (int f = 0; f <= sw_handle::kForks; ++f)
        if (h->fork_ev[f]) (void)hipEventDestroy(h->fork_ev[f]);
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
        if (value < 0 || value > 2) return fail(h, SW_EINVAL, "timing must be 0, 1 or 2");
        if (value == 2 && h->bin_ev.empty()) {
            h->bin_ev.assign(2 * kMaxBins * 2 * 2, nullptr);
            for (hipEvent_t& e : h->bin_ev)
                if (hipEventCreate(&e) != hipSuccess) return fail(h, SW_EDEVICE, "event creation failed");
            h->fam_ev.assign(2 * sw_handle::kFamLaunches * 2, nullptr);
            for (hipEvent_t& e : h->fam_ev)
                if (hipEventCreate(&e) != hipSuccess) return fail(h, SW_EDEVICE, "event creation failed");
        }
        h->opt_timing = value;
    } else if (k == "colpath") {
        h->opt_colpath = value ? 1 : 0;
    } else if (k == "chunk") {
        if (value != kChunk && value != kChunkNarrow)
            return fail(h, SW_EINVAL, "chunk (reference tile steps) must be %d or %d", kChunk, kChunkNarrow);
        h->opt_chunk = value;
    } else if (k == "pairtable") {
        h->opt_ptab = value ? 1 : 0;
    } else if (k == "qprofile") {
        h->opt_qprof = value ? 1 : 0;
    } else if (k == "capacity") {
        // reserve workspace for this many pairs up front (grids and graphs are
        // sized for the capacity, so batches up to it reuse one graph)
        if (value < 0 || value > (int64_t)0x7FFFFFFF) return fail(h, SW_EINVAL, "capacity must be 0..2^31-1");
        (void)hipSetDevice(h->device);
        const int rc = ensure_pairs(h, value);
        if (rc != SW_OK) return rc;
        return SW_OK;
    } else if (k == "families") {
        h->opt_families = value ? 1 : 0;
    } else if (k == "max_query") {
        if (value < 0 || value > SW_MAX_QUERY) return fail(h, SW_EINVAL, "max_query must be 0..%d", SW_MAX_QUERY);
        h->opt_max_query = value;
    } else if (k == "streams") {
        if (value < 1 || value > sw_handle::kForks) return fail(h, SW_EINVAL, "streams must be 1..%d", sw_handle::kForks);
        h->opt_streams = value;
    } else if (k == "cigar_workspace") {
        // device bytes for path records; a batch whose records need more is
        // processed in chunks (each chunk needs room for the largest record)
        if (value < 2 * kMaxRecordBytes)
            return fail(h, SW_EINVAL, "cigar_workspace must be at least %lld bytes", (long long)(2 * kMaxRecordBytes));
        h->opt_path_ws = value;
        return SW_OK;
    } else if (k == "precision") {
        if (value != 0 && value != 32) return fail(h, SW_EINVAL, "precision must be 0 or 32");
        h->opt_precision = value;
    } else {
        return fail(h, SW_EINVAL, "unknown option '%s'", key);
    }
    drop_graph(h);
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
    else if (k == "streams") *value = h->opt_streams;
    else if (k == "max_query") *value = h->opt_max_query;
    else if (k == "families") *value = h->opt_families;
    else if (k == "capacity") *value = h->cap_pairs;
    else if (k == "colpath") *value = h->opt_colpath;
    else if (k == "chunk") *value = h->opt_chunk;
    else if (k == "pairtable") *value = h->opt_ptab;
    else if (k == "qprofile") *value = h->opt_qprof;
    else if (k == "qprofile_used") *value = h->last_qprof;
    else if (k == "pairtable_used") *value = h->last_ptab;
    else if (k == "cigar_workspace") *value = h->opt_path_ws;
    else if (k == "captures") *value = h->n_captures;
    else if (k == "capture_refusals") *value = h->n_capture_refusals;
    else return fail(h, SW_EINVAL, "unknown option '%s'", key);
    return SW_OK;
}

}  // extern "C"

// Status of a finished call from its flags and counters (in slot k's pinned
// buffer); frees the slot.  Sets the handle's statistics of the last call
// (and, for a timed call, its phase and per-launch times).
static int complete_slot(sw_handle* h, int k) {
    sw_handle::CallSlot& sl = h->slots[k];
    sl.ticket = 0;
    if (h->last_slot == k) h->last_slot = -1;
    h->err.clear();
    const int32_t* flags = sl.h_small;
    const unsigned long long* cnt = counters(sl.h_small);
    h->last_fwd = (int64_t)cnt[kCtrFwdCells];
    h->last_rev = (int64_t)cnt[kCtrRevCells];
    h->last_i32 = (int64_t)cnt[kCtrI32Pairs];
    h->bin_stats.clear();
    h->last_ptab = sl.ptab ? 1 : 0;
    h->last_qprof = sl.qprof ? 1 : 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int b = 0; b < (int)h->bins.size(); ++b)
            for (int v = h->bins[b].col ? 1 : 0; v >= 0; --v) {
                sw_bin_stat st;
                memset(&st, 0, sizeof(st));
                st.pass = pass;
                st.precision = h->bins[b].prec;
                st.lanes = h->bins[b].W;
                st.rows = h->bins[b].R;
                const bool qp = sl.qprof && pass == 0 && v == 0 &&
                                shape_kernel(st.precision, st.lanes, st.rows, false, kVarQprof) != nullptr;
                st.column = v == 1 ? 1 : (qp ? 3 : (sl.ptab && h->bins[b].ptab ? 2 : 0));
                st.tile = !qp && sl.chunk == kChunkNarrow &&
                                  shape_kernel(st.precision, st.lanes, st.rows, false, v == 1 ? kVarCol : kVarTable, true)
                              ? kChunkNarrow
                              : kChunk;
                const int i = pass * kMaxBins + b;
                const int64_t col_cells = (int64_t)cnt[kCtrBinColCells + i];
                const int64_t col_pairs = (int64_t)cnt[kCtrBinColPairs + i];
                st.cells = v ? col_cells : (int64_t)cnt[kCtrBinCells + i] - col_cells;
                st.pairs = v ? col_pairs : (int64_t)cnt[kCtrBinPairs + i] - col_pairs;
                const int i2 = bin_ev_index(pass, b, v, 0) / 2;
                const bool known = (size_t)i2 < h->bin_launch.size();
                st.launch = known ? h->bin_launch[i2] : -1;
                st.family_hi = known ? h->bin_fam_hi[i2] : 0;
                st.family_lo = known ? h->bin_fam_lo[i2] : 0;
                st.family_waves = known ? h->bin_fam_waves[i2] : 0;
                if (known && h->bin_fam_tile[i2] > 0) st.tile = h->bin_fam_tile[i2];
                h->bin_stats.push_back(st);
            }
    h->t_plan = h->t_fwd = h->t_rev = 0.f;
    if (sl.timing) {
        float a = 0, b = 0;
        HIP_TRY(h, hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
        HIP_TRY(h, hipEventElapsedTime(&h->t_fwd, h->ev[1], h->ev[2]));
        HIP_TRY(h, hipEventElapsedTime(&b, h->ev[2], h->ev[3]));
        HIP_TRY(h, hipEventElapsedTime(&h->t_rev, h->ev[3], h->ev[4]));
        h->t_plan = a + b;
        if (h->opt_timing == 2)
            for (sw_bin_stat& st : h->bin_stats) {
                // only launched kernels have events (plain mode skips empty
                // item ranges; no mode launches a bin no route points at)
                const int b = find_bin(h, st.precision, st.lanes, st.rows);
                const int i = bin_ev_index(st.pass, b, st.column == 1 ? 1 : 0, 0);
                const int slot = (size_t)(i / 2) < h->bin_fam_slot.size() ? h->bin_fam_slot[i / 2] : -1;
                if (slot >= 0) {
                    // a family launch: its time, shared by its bins
                    const hipEvent_t* fe = &h->fam_ev[(st.pass * sw_handle::kFamLaunches + slot) * 2];
                    HIP_TRY(h, hipEventElapsedTime(&st.ms, fe[0], fe[1]));
                    continue;
                }
                if (!h->bin_launched[i / 2]) continue;
                HIP_TRY(h, hipEventElapsedTime(&st.ms, h->bin_ev[i], h->bin_ev[i + 1]));
            }
    }
    if (flags[kFlagBadOffsets]) return fail(h, SW_EINVAL, "offsets decrease");
    if (flags[kFlagBadScheme]) return fail(h, SW_EINVAL, "scheme id out of range");
    if (flags[kFlagTooLong])
        return fail(h, SW_ETOOLONG, "a query exceeds %d or a reference exceeds %d residues",
                    h->opt_max_query > 0 ? (int)h->opt_max_query : SW_MAX_QUERY, SW_MAX_REF);
    if (flags[kFlagBadResidue]) return fail(h, SW_EINVAL, "residue code outside its scheme's alphabet");
    if (flags[kFlagInternal]) return fail(h, SW_EINTERNAL, "a planning invariant did not hold");
    if (flags[kFlagReverseMismatch]) return fail(h, SW_EINTERNAL, "reverse sweep did not reproduce the forward score");
    return SW_OK;
}

// A ticket whose call needed no device work (an empty batch).
static uint64_t finish_now(sw_handle* h) {
    const uint64_t t = h->next_ticket++;
    h->finished[t] = sw_handle::Finished{SW_OK, std::string()};
    h->last_fwd = h->last_rev = h->last_i32 = 0;
    h->bin_stats.clear();
    h->t_plan = h->t_fwd = h->t_rev = 0.f;
    return t;
}

// Enqueue the alignment of pairs given as spans (query i is queries[q_beg[i]
// .. q_end[i]), reference i is refs[r_beg[i] .. r_end[i])) on `stream`, and
// return a ticket for sw_poll.  Nothing waits for the device, except a
// submit that finds every slot in flight (it completes the oldest) or that
// must free or rewrite what calls in flight use (a larger workspace, a new
// routing table, a graph evicted from the cache).  Shared by sw_submit,
// sw_align_batch and sw_align_spans (a submit and a wait), and
// sw_align_batch_noalloc.
// With `no_alloc` the planning arrays live in the static workspace, grids
// are sized for the batch itself, nothing is captured into a graph and
// nothing is allocated or freed.  Timed calls (`allow_timing`) must be
// waited for before the next call: they share the handle's events.
static int submit_spans(sw_handle* h, const uint8_t* queries, const int64_t* q_beg, const int64_t* q_end,
                        const uint8_t* refs, const int64_t* r_beg, const int64_t* r_end,
                        const uint8_t* scheme_id, int64_t n_pairs, const sw_scheme* schemes,
                        int n_schemes, sw_result* out, void* stream_ptr, bool no_alloc, bool allow_timing,
                        uint64_t* ticket, int64_t search_n = -1) {
    if (!h) return SW_EINVAL;
    h->err.clear();
    const auto t_entry = std::chrono::steady_clock::now();
    h->t_enqueue = h->t_wait = 0.0;
    if (!ticket) return fail(h, SW_EINVAL, "null ticket");
    if (!schemes) return fail(h, SW_EINVAL, "null schemes");
    if (n_schemes < 1 || n_schemes > SW_MAX_SCHEMES)
        return fail(h, SW_EINVAL, "n_schemes must be 1..%d", SW_MAX_SCHEMES);
    const int64_t P = n_pairs;
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
    if (no_alloc && P > kStaticPairs)
        return fail(h, SW_EINVAL, "%lld pairs: the allocation-free call takes at most %lld", (long long)P,
                    (long long)kStaticPairs);
    const bool timing = h->opt_timing != 0;
    if (timing && !allow_timing)
        return fail(h, SW_EINVAL, "the \"timing\" option needs a synchronous call (sw_align_batch)");
    if (P == 0) {
        *ticket = finish_now(h);
        return SW_OK;
    }
    if (!q_beg || !q_end || !r_beg || !r_end || !queries || !refs || !out)
        return fail(h, SW_EINVAL, "null device pointer with n_pairs > 0");
    hipStream_t stream = (hipStream_t)stream_ptr;
    HIP_TRY(h, hipSetDevice(h->device));

    // a slot for this call: the oldest in flight is completed if need be
    const int k = h->next_slot;
    sw_handle::CallSlot& sl = h->slots[k];
    if (sl.ticket) {
        const uint64_t t = sl.ticket;
        HIP_TRY(h, hipEventSynchronize(sl.done));
        const int st = complete_slot(h, k);
        h->finished[t] = sw_handle::Finished{st, h->err};
        h->err.clear();
    }
    // calls of one handle share its workspace: one submitted on another
    // stream than the last waits for it on the device
    if (h->last_slot >= 0 && h->last_stream != stream)
        HIP_TRY(h, hipStreamWaitEvent(stream, h->slots[h->last_slot].done, 0));

    Workspace ws;
    if (no_alloc) {
        if (!h->d_scratch) return fail(h, SW_EDEVICE, "the static workspace has no address on device %d", h->device);
        ws.keys = reinterpret_cast<int32_t*>(h->d_scratch + kStaticKeys);
        ws.order = reinterpret_cast<int32_t*>(h->d_scratch + kStaticOrder);
        ws.items = reinterpret_cast<WorkItem*>(h->d_scratch + kStaticItems);
        ws.cap = P;
        // a changed routing table is uploaded in stream order, but stays
        // marked dirty: the next graph-capable call must still drop its
        // graphs (which launch the bins of the old table) and upload it again
        if (h->lut_dirty) {
            memcpy(h->h_lut, h->lut.data(), kLutEntries);
            HIP_TRY(h, hipMemcpyAsync(h->d_lut, h->h_lut, kLutEntries, hipMemcpyHostToDevice, stream));
        }
    } else {
        int rc = ensure_pairs(h, P);
        if (rc != SW_OK) return rc;
        if (h->lut_dirty) {
            drop_graph(h);
            HIP_TRY(h, hipMemcpy(h->d_lut, h->lut.data(), kLutEntries, hipMemcpyHostToDevice));
            h->lut_dirty = false;
        }
        ws.keys = h->d_keys;
        ws.order = h->d_order;
        ws.items = h->d_items;
        ws.cap = h->cap_pairs;
    }

    // substitution tables: [s][b][a] = M_s[a][b]; padding rows/columns score -1
    ClassifyArgs C;
    h->tables.assign(kSchemeBytes, 0);
    for (int s = 0; s < SW_MAX_SCHEMES; ++s) {
        int8_t* T = h->tables.data() + s * kMatBytes;
        int mx = 1;
        for (int b = 0; b < kMatDim; ++b)
            for (int a = 0; a < kMatDim; ++a) {
                int8_t v = -1;
                if (s < n_schemes && a < schemes[s].alphabet && b < schemes[s].alphabet) {
                    v = schemes[s].matrix[a * schemes[s].alphabet + b];
                    mx = std::max(mx, (int)v);
                }
                T[b * kMatDim + a] = v;
            }
        C.max_score[s] = mx;
        // small-alphabet column path: alphabet <= 4, 1 <= o <= kI16Bias and
        // every M[a][b] + o a byte; column word of residue b = bytes
        // M[a][b] + o, a = 0..3 (0 for residues outside the alphabet)
        uint32_t* cw = reinterpret_cast<uint32_t*>(h->tables.data() + SW_MAX_SCHEMES * kMatBytes) + s * kMatDim;
        bool ok = s < n_schemes && schemes[s].alphabet <= 4 && schemes[s].gap_open >= 1 &&
                  schemes[s].gap_open <= kI16Bias;
        for (int b = 0; b < kMatDim; ++b) {
            uint32_t w = 0;
            for (int a = 0; ok && a < 4; ++a) {
                if (a >= schemes[s].alphabet || b >= schemes[s].alphabet) continue;
                const int v = schemes[s].matrix[a * schemes[s].alphabet + b] + schemes[s].gap_open;
                if (v < 0 || v > 255) ok = false;
                w |= (uint32_t)(v & 0xFF) << (8 * a);
            }
            cw[b] = w;
        }
        C.col_ok[s] = ok ? 1 : 0;
    }
    // the packed path holds every value of a pair when its score bound
    // min(n, m) * max_score is at most kI16Limit
    C.i16_limit = h->opt_precision == 32 ? -1 : kI16Limit;
    C.n_schemes = n_schemes;
    C.n_bins = (int)h->bins.size();
    C.max_query = (int32_t)h->opt_max_query;

    // Pair table: when exactly one scheme of the call takes table lookups
    // (every other one takes column words), the packed int16 table-range
    // kernels read that scheme's scores from a pair table instead, provided
    // its alphabet has at most kPtabMaxDim - 1 residues, 1 <= o <= K and
    // every M[a][b] + o is a byte.
    int ptab_sid = -1, D = 0;
    if (h->opt_ptab) {
        int n_table = 0, cand = -1;
        for (int sidx = 0; sidx < n_schemes; ++sidx)
            if (!(C.col_ok[sidx] && h->opt_colpath)) { ++n_table; cand = sidx; }
        if (n_table == 1) {
            const sw_scheme& sc = schemes[cand];
            bool ok = sc.alphabet + 1 <= kPtabMaxDim && sc.gap_open >= 1 && sc.gap_open <= kI16Bias;
            for (int k2 = 0; ok && k2 < sc.alphabet * sc.alphabet; ++k2) {
                const int v = sc.matrix[k2] + sc.gap_open;
                ok = v >= 0 && v <= 255;
            }
            if (ok) { ptab_sid = cand; D = sc.alphabet + 1; }
        }
    }
    if (ptab_sid >= 0) {
        // entry [(x D + y) D + b] = bytes M[x][b] + o (low), M[y][b] + o
        // (high); code D - 1 pads rows and columns with 0
        const sw_scheme& sc = schemes[ptab_sid];
        const int A = sc.alphabet;
        uint16_t* T = reinterpret_cast<uint16_t*>(h->tables.data() + kPtabOffset);
        auto byte = [&](int a, int b) -> uint16_t {
            return (a < A && b < A) ? (uint16_t)(sc.matrix[a * A + b] + sc.gap_open) : (uint16_t)0;
        };
        for (int x = 0; x < D; ++x)
            for (int y = 0; y < D; ++y)
                for (int b = 0; b < D; ++b)
                    T[(x * D + y) * D + b] = (uint16_t)(byte(x, b) | (byte(y, b) << 8));
    }

    KParams K;
    memset(&K, 0, sizeof(K));
    K.queries = queries; K.q_beg = q_beg; K.q_end = q_end; K.refs = refs; K.r_beg = r_beg; K.r_end = r_end;
    K.scheme_id = scheme_id; K.order = ws.order; K.items = ws.items; K.meta = h->d_meta;
    K.out = out; K.flags = h->d_small; K.mats = h->d_mats; K.validate = (int32_t)h->opt_validate;
    K.n_dev = h->d_n;
    K.n_pairs = (int32_t)ws.cap;
    K.max_items = (int32_t)(ws.cap + kMaxBins);
    K.ptab_sid = ptab_sid;
    K.ptab_dim = D;
    // query profile: a search (every pair aligns queries[0 .. qprof_n)) with
    // the pair table's scheme profiles its query for the forward pass
    K.qprof = (search_n >= 1 && search_n <= SW_MAX_QUERY && ptab_sid >= 0 && h->opt_qprof) ? 1 : 0;
    K.qprof_n = K.qprof ? (int32_t)search_n : 0;
    for (int s = 0; s < SW_MAX_SCHEMES; ++s) {
        const bool v = s < n_schemes;
        K.alphabet[s] = v ? schemes[s].alphabet : 1;
        K.gap_open[s] = v ? schemes[s].gap_open : 1;
        K.gap_extend[s] = v ? schemes[s].gap_extend : 0;
        K.max_score[s] = C.max_score[s];
        K.col_ok[s] = C.col_ok[s] && h->opt_colpath;
        C.col_ok[s] = K.col_ok[s];
        h->last_col_ok[s] = K.col_ok[s];
    }

    const bool use_graph = h->opt_mode == 1 && h->opt_graph != 0 && !timing && !no_alloc;
    GraphKey key;
    memset(&key, 0, sizeof(key));
    key.queries = queries; key.q_beg = q_beg; key.q_end = q_end; key.refs = refs;
    key.r_beg = r_beg; key.r_end = r_end; key.scheme_id = scheme_id; key.out = out;
    key.cap_pairs = h->cap_pairs;
    memcpy(key.alphabet, K.alphabet, sizeof(key.alphabet));
    memcpy(key.gap_open, K.gap_open, sizeof(key.gap_open));
    memcpy(key.gap_extend, K.gap_extend, sizeof(key.gap_extend));
    memcpy(key.max_score, C.max_score, sizeof(key.max_score));
    memcpy(key.col_ok, C.col_ok, sizeof(key.col_ok));
    key.n_schemes = n_schemes; key.validate = (int32_t)h->opt_validate; key.precision = (int32_t)h->opt_precision;
    key.ptab_sid = ptab_sid;
    key.qprof = K.qprof;
    key.qprof_n = K.qprof_n;
    key.search_n = (int32_t)std::max<int64_t>(-1, std::min<int64_t>(search_n, SW_MAX_QUERY + 1));
    key.max_query = C.max_query;

    // Start of the call, in stream order and outside any graph: the scheme
    // tables when they differ from what the device holds (from this call's
    // own pinned staging, which no later call rewrites while it is in
    // flight), then one kernel that clears the flags and counters and
    // writes the batch size (a kernel argument, so nothing on the host
    // must outlive the submit).  A captured graph reads the batch size from
    // device memory, so it serves every batch of at most cap_pairs pairs.
    if (timing) HIP_TRY(h, hipEventRecord(h->ev[0], stream));
    if (h->dev_mats != h->tables) {
        memcpy(sl.h_mats, h->tables.data(), kSchemeBytes);
        HIP_TRY(h, hipMemcpyAsync(h->d_mats, sl.h_mats, kSchemeBytes, hipMemcpyHostToDevice, stream));
        h->dev_mats = h->tables;
    }
    HIP_TRY(h, launch_call_start(h->d_small, kSmallInts, h->d_n, (int32_t)P, stream));

    auto enqueue_all = [&](hipStream_t es) -> int {
        const int rc0 = enqueue_pass(h, K, C, ws, 0, es, timing, search_n);
        if (rc0 != SW_OK) return rc0;
        return enqueue_pass(h, K, C, ws, 1, es, timing, search_n);
    };
    if (timing) h->bin_launched.assign(2 * kMaxBins * 2, 0);
    int gi = -1;
    for (int g = 0; use_graph && g < (int)h->graphs.size(); ++g)
        if (memcmp(&key, &h->graphs[g].key, sizeof(key)) == 0) gi = g;
    if (gi >= 0) {
        // most recently used last
        std::rotate(h->graphs.begin() + gi, h->graphs.begin() + gi + 1, h->graphs.end());
        HIP_TRY(h, hipGraphLaunch(h->graphs.back().exec, stream));
    } else {
        // The graph is captured on the handle's private stream (the caller's
        // stream may be the null stream, which cannot be captured) and then
        // launched on the caller's stream.
        // Captures are serialised across the handles of the process (the
        // runtime has refused a capture begun while another thread was
        // capturing); if one is refused anyway, this call runs eagerly on the
        // caller's stream and a later call captures.
        std::unique_lock<std::mutex> capture_lock(g_capture_mu, std::defer_lock);
        bool capturing = false;
        if (use_graph) {
            if ((int)h->graphs.size() >= sw_handle::kGraphs) {
                // evict the least recently used graph once nothing in
                // flight can still be running it
                drain(h);
                (void)hipGraphExecDestroy(h->graphs.front().exec);
                (void)hipGraphDestroy(h->graphs.front().graph);
                h->graphs.erase(h->graphs.begin());
            }
            // created on first use, so that the fork streams, created with
            // the handle, take consecutive hardware queues
            if (!h->cap_stream) HIP_TRY(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
            capture_lock.lock();
            capturing = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (!capturing) {
                (void)hipGetLastError();
                capture_lock.unlock();
                ++h->n_capture_refusals;
            }
        }
        bool eager = !capturing;
        if (capturing) {
            const int erc = enqueue_all(h->cap_stream);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(h->cap_stream, &g);
            if (erc == SW_OK && ce == hipSuccess && g) {
                ++h->n_captures;
                hipGraphExec_t ge = nullptr;
                const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                capture_lock.unlock();
                if (ie != hipSuccess) {
                    (void)hipGraphDestroy(g);
                    return fail(h, SW_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
                }
                h->graphs.push_back(sw_handle::GraphEntry{key, g, ge});
                HIP_TRY(h, hipGraphLaunch(ge, stream));
            } else {
                // nothing captured has run: discard it and run the call eagerly
                if (g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
                capture_lock.unlock();
                ++h->n_capture_refusals;
                for (int f = 0; f < sw_handle::kForks; ++f) {
                    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
                    if (hipStreamIsCapturing(h->fork[f], &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
                        return fail(h, SW_EDEVICE, "a stream stayed in capture after a failed capture");
                }
                h->err.clear();
                eager = true;
            }
        }
        if (eager) {
            const int erc = enqueue_all(stream);
            if (erc != SW_OK) return erc;
        }
    }
    // end of the call: its flags and counters to the slot, then its event
    HIP_TRY(h, hipMemcpyAsync(sl.h_small, h->d_small, kSmallInts * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(h, hipEventRecord(sl.done, stream));
    sl.ticket = h->next_ticket++;
    sl.timing = timing;
    sl.ptab = ptab_sid >= 0;
    sl.qprof = K.qprof != 0;
    sl.chunk = (int)h->opt_chunk;
    sl.t_entry = t_entry;
    h->last_slot = k;
    h->last_stream = stream;
    h->next_slot = (k + 1) % sw_handle::kSlots;
    *ticket = sl.ticket;
    h->t_enqueue = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_entry).count();
    return SW_OK;
}

// Wait for (wait != 0) or test the call of `ticket`: SW_PENDING while it
// runs, else its status (the ticket is then forgotten).
static int poll_ticket(sw_handle* h, uint64_t ticket, int wait) {
    auto it = h->finished.find(ticket);
    if (it != h->finished.end()) {
        const sw_handle::Finished f = it->second;
        h->finished.erase(it);
        h->err = f.err;
        return f.status;
    }
    int k = -1;
    for (int j = 0; j < sw_handle::kSlots; ++j)
        if (ticket && h->slots[j].ticket == ticket) k = j;
    if (k < 0) return fail(h, SW_EINVAL, "unknown ticket %llu (never issued, or already polled)",
                           (unsigned long long)ticket);
    HIP_TRY(h, hipSetDevice(h->device));
    if (wait) {
        HIP_TRY(h, hipEventSynchronize(h->slots[k].done));
    } else {
        const hipError_t q = hipEventQuery(h->slots[k].done);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();
            return SW_PENDING;
        }
        if (q != hipSuccess) return fail(h, SW_EDEVICE, "hipEventQuery failed: %s", hipGetErrorString(q));
    }
    return complete_slot(h, k);
}

// The synchronous calls: a submit, then a wait for it.
static int align_spans(sw_handle* h, const uint8_t* queries, const int64_t* q_beg, const int64_t* q_end,
                       const uint8_t* refs, const int64_t* r_beg, const int64_t* r_end,
                       const uint8_t* scheme_id, int64_t n_pairs, const sw_scheme* schemes,
                       int n_schemes, sw_result* out, void* stream_ptr, bool no_alloc = false,
                       int64_t search_n = -1) {
    if (!h) return SW_EINVAL;
    uint64_t t = 0;
    const int rc = submit_spans(h, queries, q_beg, q_end, refs, r_beg, r_end, scheme_id, n_pairs, schemes,
                                n_schemes, out, stream_ptr, no_alloc, true, &t, search_n);
    if (rc != SW_OK) return rc;
    const double enq = h->t_enqueue;
    const auto t0 = std::chrono::steady_clock::now();
    const int st = poll_ticket(h, t, 1);
    h->t_enqueue = enq;
    h->t_wait = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

extern "C" {

int sw_align_batch(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes, int n_schemes,
                   sw_result* out, void* stream_ptr) {
    if (!h) return SW_EINVAL;
    if (!batch) return fail(h, SW_EINVAL, "null batch");
    const int64_t* qo = batch->q_off;
    const int64_t* ro = batch->r_off;
    return align_spans(h, batch->queries, qo, qo ? qo + 1 : nullptr, batch->refs, ro, ro ? ro + 1 : nullptr,
                       batch->scheme_id, batch->n_pairs, schemes, n_schemes, out, stream_ptr);
}

int sw_submit(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes, int n_schemes, sw_result* out,
              void* stream_ptr, uint64_t* ticket) {
    if (!h) return SW_EINVAL;
    if (!batch) return fail(h, SW_EINVAL, "null batch");
    const int64_t* qo = batch->q_off;
    const int64_t* ro = batch->r_off;
    return submit_spans(h, batch->queries, qo, qo ? qo + 1 : nullptr, batch->refs, ro, ro ? ro + 1 : nullptr,
                        batch->scheme_id, batch->n_pairs, schemes, n_schemes, out, stream_ptr, false, false, ticket);
}

int sw_poll(sw_handle* h, uint64_t ticket, int wait) {
    if (!h) return SW_EINVAL;
    return poll_ticket(h, ticket, wait);
}

int sw_align_batch_noalloc(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes, int n_schemes,
                           sw_result* out, void* stream_ptr) {
    if (!h) return SW_EINVAL;
    if (!batch) return fail(h, SW_EINVAL, "null batch");
    const int64_t* qo = batch->q_off;
    const int64_t* ro = batch->r_off;
    return align_spans(h, batch->queries, qo, qo ? qo + 1 : nullptr, batch->refs, ro, ro ? ro + 1 : nullptr,
                       batch->scheme_id, batch->n_pairs, schemes, n_schemes, out, stream_ptr, true);
}

int sw_align_spans(sw_handle* h, const uint8_t* queries, const int64_t* q_beg, const int64_t* q_end,
                   const uint8_t* refs, const int64_t* r_beg, const int64_t* r_end,
                   const uint8_t* scheme_id, int64_t n_pairs, const sw_scheme* schemes, int n_schemes,
                   sw_result* out, void* stream) {
    return align_spans(h, queries, q_beg, q_end, refs, r_beg, r_end, scheme_id, n_pairs, schemes, n_schemes,
                       out, stream);
}

int sw_last_stats(sw_handle* h, int64_t* fwd_cells, int64_t* rev_cells, int64_t* int32_pairs) {
    if (!h) return SW_EINVAL;
    if (fwd_cells) *fwd_cells = h->last_fwd;
    if (rev_cells) *rev_cells = h->last_rev;
    if (int32_pairs) *int32_pairs = h->last_i32;
    return SW_OK;
}

int sw_shapes(sw_handle* h, int32_t* precision, int32_t* lanes, int32_t* rows, int capacity, int* n_out) {
    if (!h) return SW_EINVAL;
    const int n = (int)h->bins.size();
    if (n_out) *n_out = n;
    if (!precision || !lanes || !rows || capacity < n) return fail(h, SW_EINVAL, "need room for %d shapes", n);
    for (int b = 0; b < n; ++b) {
        precision[b] = h->bins[b].prec;
        lanes[b] = h->bins[b].W;
        rows[b] = h->bins[b].R;
    }
    return SW_OK;
}

int sw_set_routing(sw_handle* h, int precision, const int32_t* rows_max, const int32_t* lanes, const int32_t* rows,
                   int n) {
    if (!h) return SW_EINVAL;
    if (precision != 16 && precision != 32) return fail(h, SW_EINVAL, "precision must be 16 or 32");
    return set_routing(h, precision == 16 ? 0 : 1, rows_max, lanes, rows, n);
}

int sw_get_routing(sw_handle* h, int precision, int32_t* rows_max, int32_t* lanes, int32_t* rows, int capacity,
                   int* n_out) {
    if (!h) return SW_EINVAL;
    if (precision != 16 && precision != 32) return fail(h, SW_EINVAL, "precision must be 16 or 32");
    const std::vector<int>& r = h->route[precision == 16 ? 0 : 1];
    std::vector<int32_t> hi, W, R;
    for (int k = 0; k < kLutRows; ++k) {
        const bool last = k + 1 == kLutRows || r[k + 1] != r[k];
        if (!last) continue;
        hi.push_back(16 * (k + 1));
        W.push_back(r[k] >= 0 ? h->bins[r[k]].W : 0);
        R.push_back(r[k] >= 0 ? h->bins[r[k]].R : 0);
    }
    const int n = (int)hi.size();
    if (n_out) *n_out = n;
    if (!rows_max || !lanes || !rows || capacity < n) return fail(h, SW_EINVAL, "need room for %d entries", n);
    for (int e = 0; e < n; ++e) {
        rows_max[e] = hi[e];
        lanes[e] = W[e];
        rows[e] = R[e];
    }
    return SW_OK;
}

int sw_last_bin_stats(sw_handle* h, sw_bin_stat* out, int capacity, int* n_out) {
    if (!h) return SW_EINVAL;
    const int n = (int)h->bin_stats.size();
    if (n_out) *n_out = n;
    if (n > 0 && (!out || capacity < n)) return fail(h, SW_EINVAL, "need room for %d entries", n);
    for (int k = 0; k < n; ++k) out[k] = h->bin_stats[k];
    return SW_OK;
}

int sw_last_host_timing(sw_handle* h, double* enqueue_ms, double* wait_ms) {
    if (!h) return SW_EINVAL;
    if (enqueue_ms) *enqueue_ms = h->t_enqueue;
    if (wait_ms) *wait_ms = h->t_wait;
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

// ---- alignment paths ---------------------------------------------------------

static int ensure_path_buffers(sw_handle* h, int64_t cap) {
    if (cap <= h->trace_cap) return SW_OK;
    free_dev(h->d_rec_off); free_dev(h->d_bsum);
    h->d_rec_off = nullptr; h->d_bsum = nullptr;
    h->trace_cap = 0;
    if (hipMalloc(&h->d_rec_off, (cap + 1) * 8) != hipSuccess ||
        hipMalloc(&h->d_bsum, (trace_scan_blocks(cap) + 1) * 8) != hipSuccess)
        return fail(h, SW_ENOMEM, "device allocation of path offsets for %lld pairs failed", (long long)cap);
    h->trace_cap = cap;
    return SW_OK;
}

// Paths of the pairs whose results are in `out` (written by the score passes
// of the same call): record layout, then per chunk planning, path sweeps and
// walks.  Synchronises `stream` once to read the records' total size (and
// once per chunk when timing).
static int trace_paths(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes, int n_schemes,
                       sw_result* out, const int64_t* path_off, uint32_t* path, int32_t* path_len,
                       hipStream_t stream) {
    const int64_t P = batch->n_pairs;
    const bool timing = h->opt_timing != 0;
    const int n_tb = (int)h->tbins.size();
    if (timing && h->tbin_ev.empty()) {
        h->tbin_ev.assign(3 * n_tb, nullptr);
        for (hipEvent_t& e : h->tbin_ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(h, SW_EDEVICE, "event creation failed");
    }
    const int64_t cap = h->cap_pairs;
    int rc = ensure_path_buffers(h, cap);
    if (rc != SW_OK) return rc;

    KParams K;
    memset(&K, 0, sizeof(K));
    K.queries = batch->queries; K.q_beg = batch->q_off; K.q_end = batch->q_off + 1;
    K.refs = batch->refs; K.r_beg = batch->r_off; K.r_end = batch->r_off + 1;
    K.scheme_id = batch->scheme_id; K.order = h->d_order; K.items = h->d_items; K.meta = h->d_meta;
    K.out = out; K.flags = h->d_small; K.mats = h->d_mats; K.validate = 0;
    K.n_dev = h->d_n;
    K.n_pairs = (int32_t)cap;
    K.max_items = (int32_t)(cap + kMaxBins);
    K.ptab_sid = -1;
    K.ptab_dim = 0;
    for (int s = 0; s < SW_MAX_SCHEMES; ++s) {
        const bool v = s < n_schemes;
        K.alphabet[s] = v ? schemes[s].alphabet : 1;
        K.gap_open[s] = v ? schemes[s].gap_open : 1;
        K.gap_extend[s] = v ? schemes[s].gap_extend : 0;
        int mx = 1;   // as the score passes set it (the path sweep itself does not read it)
        for (int k = 0; v && k < schemes[s].alphabet * schemes[s].alphabet; ++k)
            mx = std::max(mx, (int)schemes[s].matrix[k]);
        K.max_score[s] = mx;
    }
    // Pairs of schemes with column words (the score call just made uploaded
    // them) take the column-word path sweep, the others the byte-table one:
    // a packed bin's column-word pairs come first in its sorted order, and
    // each part has its own kernel (variant 1, variant 0).
    bool all_col = n_schemes > 0, any_col = false;
    for (int s = 0; s < n_schemes && s < SW_MAX_SCHEMES; ++s) {
        all_col = all_col && h->last_col_ok[s] != 0;
        any_col = any_col || h->last_col_ok[s] != 0;
    }
    for (int s = 0; s < SW_MAX_SCHEMES; ++s) K.col_ok[s] = s < n_schemes && h->last_col_ok[s] ? 1 : 0;
    // does bin e have pairs for variant v (1 column words, 0 byte table)?
    auto wants = [&](const BinInfo& e, int v) { return v == 1 ? (e.col && any_col) : !(e.col && all_col); };
    // Bins no pair can reach are not launched (a launch with no items still
    // costs its stream a few microseconds, and its walks as many): with the
    // caller's bound on query lengths ("max_query"), a box has at most that
    // many rows, and its score S is at most max_query times the best
    // substitution score, so no pair takes an int32 bin when that product
    // fits the packed range.  (A call with a longer query has already
    // failed with SW_ETOOLONG in the score passes.)
    int mx_all = 0;
    for (int s = 0; s < n_schemes && s < SW_MAX_SCHEMES; ++s) mx_all = std::max(mx_all, K.max_score[s]);
    const int64_t max_q = h->opt_max_query;
    const bool i16_only = h->opt_precision != 32 && max_q > 0 && max_q * mx_all <= kI16Limit;
    auto reachable = [&](int b) {
        const BinInfo& e = h->tbins[b];
        if (max_q > 0 && h->tbin_min_rows[b] > max_q) return false;
        if (e.prec == 16 && h->opt_precision == 32) return false;   // every pair takes int32
        return !(e.prec == 32 && i16_only);
    };
    TraceArgs T;
    memset(&T, 0, sizeof(T));
    T.rec_off = h->d_rec_off;
    T.lut = h->d_tlut;
    T.i16_limit = h->opt_precision == 32 ? -1 : kI16Limit;
    T.bins = h->d_tbins;
    T.n_bins = n_tb;
    T.chunk_bytes = 1;

    HIP_TRY(h, launch_reset(h->d_small, kSmallInts, stream));
    HIP_TRY(h, launch_trace_sizes(K, T, cap, h->d_rec_off, h->d_bsum, counters(h->d_small), stream));
    HIP_TRY(h, hipMemcpyAsync(h->h_i64, h->d_rec_off + P, 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(h, hipStreamSynchronize(stream));
    const int64_t total = h->h_i64[0];
    if (total < 0) return fail(h, SW_EINTERNAL, "negative path record size");

    // chunking: the workspace holds one chunk's records; records start in
    // [c * C, (c + 1) * C) and none is larger than kMaxRecordBytes
    int64_t C, ws;
    if (total + 256 <= h->opt_path_ws) {
        C = std::max<int64_t>(total, 1);
        ws = (total + 255) & ~(int64_t)255;
    } else {
        C = (h->opt_path_ws - kMaxRecordBytes) & ~(int64_t)255;
        ws = C + kMaxRecordBytes;
    }
    const int chunks = total > 0 ? (int)((total + C - 1) / C) : 1;
    ws = std::max<int64_t>(ws, 256);
    if (ws > h->ws_alloc) {
        free_dev(h->d_ws);
        h->d_ws = nullptr;
        h->ws_alloc = 0;
        if (hipMalloc(&h->d_ws, ws) != hipSuccess)
            return fail(h, SW_ENOMEM, "device allocation of %lld path record bytes failed", (long long)ws);
        h->ws_alloc = ws;
    }
    T.ws = h->d_ws;
    T.ws_bytes = h->ws_alloc;
    T.chunk_bytes = C;
    h->last_path_bytes = total;
    h->last_path_chunks = chunks;
    h->t_path_sweep = h->t_path_walk = 0.f;
    std::vector<float> bin_ms(n_tb, 0.f);

    for (int c = 0; c < chunks; ++c) {
        T.chunk = c;
        HIP_TRY(h, launch_reset(h->d_hist, kHistSize, stream));
        HIP_TRY(h, launch_trace_classify(K, T, cap, h->d_keys, h->d_hist, counters(h->d_small), path_len, stream));
        HIP_TRY(h, launch_plan(h->d_tbins, n_tb, h->d_hist, h->d_meta, stream));
        HIP_TRY(h, launch_scatter(h->d_keys, h->d_n, cap, h->d_hist, h->d_order, stream));
        HIP_TRY(h, launch_items(h->d_meta, h->d_tbins, n_tb, h->d_n, cap, h->d_items, stream));
        // longest boxes first: each bin's sweep (sized to fill the device),
        // then its walks, on one stream; bins go round-robin to the forked
        // streams (joined back at the end of the chunk), so that walks and
        // launch tails overlap other bins' sweeps.  Timing serialises
        // everything on the caller's stream.
        const int forks = timing ? 0 : (int)h->opt_streams;
        const int walk_blocks = (int)std::min<int64_t>((cap + 255) / 256, 4 * std::max(1, h->n_cu));
        if (forks > 1) {
            HIP_TRY(h, hipEventRecord(h->fork_ev[sw_handle::kForks], stream));
            for (int f = 0; f < forks; ++f)
                HIP_TRY(h, hipStreamWaitEvent(h->fork[f], h->fork_ev[sw_handle::kForks], 0));
        }
        int launched = 0;
        // walks per wavefront: fewer for longer boxes (a wavefront waits
        // for every miss of any of its walks)
        auto walk = [&](int b, hipStream_t ls) -> hipError_t {
            const int rows = h->tbins[b].W * h->tbins[b].R;
            const int active = rows >= 1024 ? 8 : rows >= 768 ? 16 : rows >= 96 ? 32 : 64;
            const int wblocks = active == 64 ? walk_blocks
                                             : (int)std::min<int64_t>((cap + 4 * active - 1) / (4 * active),
                                                                      4 * std::max(1, h->n_cu));
            return launch_trace_walk(K, T, b, wblocks, active, path_off, path, path_len, ls);
        };
        // Family launches (option "families"): per lane width and variant, one
        // box-sweep kernel takes the items of all its bins, largest rows
        // first.  The two variants of a width run on different streams; a
        // member's walks start once both have swept it.
        h->tfam_first.assign(n_tb, -1);
        int n_fam = 0;
        for (int b = n_tb - 1; h->opt_families && b >= 0; --b) {
            if (h->tfam_first[b] >= 0 || !reachable(b)) continue;
            const BinInfo& e = h->tbins[b];
            const TraceFamily* f = trace_family(e.prec, e.W, e.R);
            if (!f) continue;
            int members[kFamilyMax], nm = 0;
            int8_t fam_bins[kFamilyMax];
            for (int k = 0; k < kFamilyMax; ++k) fam_bins[k] = -1;
            for (int k = 0; k < f->n; ++k) {
                int mb = -1;
                for (int t = 0; t < n_tb; ++t)
                    if (h->tbins[t].prec == f->prec && h->tbins[t].W == f->W && h->tbins[t].R == f->rows[k]) mb = t;
                if (mb < 0 || h->tfam_first[mb] >= 0 || !reachable(mb)) continue;
                fam_bins[k] = (int8_t)mb;
                members[nm++] = mb;
            }
            // the variants its members need, each with its kernel and residency
            TraceFn fns[2] = {nullptr, nullptr};
            int res[2] = {0, 0}, n_var = 0;
            bool ok = nm >= 2;
            for (int v = 1; ok && v >= 0; --v) {
                bool need_v = false;
                for (int k = 0; k < nm; ++k) need_v = need_v || wants(h->tbins[members[k]], v);
                if (!need_v) continue;
                fns[v] = v ? f->col : f->fn;
                for (const auto& r : h->tfam_resident)
                    if (r.first == fns[v]) res[v] = r.second;
                ok = fns[v] && res[v] > 0;
                ++n_var;
            }
            if (!ok || n_var == 0 || n_fam + n_var > sw_handle::kTraceFams) continue;
            const int b0 = members[0];
            for (int k = 0; k < nm; ++k) h->tfam_first[members[k]] = b0;
            for (int k = 0; k < kFamilyMax; ++k) K.fam_bins[k] = fam_bins[k];
            const int64_t need = (cap / e.ppw + 1 + kWavesPerBlock - 1) / kWavesPerBlock;
            hipStream_t ls = forks > 1 ? h->fork[launched++ % forks] : stream;
            if (timing) HIP_TRY(h, hipEventRecord(h->tbin_ev[3 * b0], ls));
            hipEvent_t swept[2];
            int n_swept = 0;
            for (int v = 1; v >= 0; --v) {
                if (!fns[v]) continue;
                hipStream_t vs = n_swept == 0 || forks <= 1 ? ls : h->fork[launched++ % forks];
                hipLaunchKernelGGL(fns[v], dim3((int)std::min<int64_t>(need, res[v])), dim3(kBlock), 0, vs, K, T);
                HIP_TRY(h, hipGetLastError());
                swept[n_swept] = h->tfam_ev[n_fam++];
                if (forks > 1) HIP_TRY(h, hipEventRecord(swept[n_swept], vs));
                ++n_swept;
            }
            if (timing) HIP_TRY(h, hipEventRecord(h->tbin_ev[3 * b0 + 1], ls));
            // the members' walks, once the sweeps have written their records:
            // spread over the forked streams so that they overlap other
            // sweeps (timing keeps everything on the caller's stream)
            for (int k = 0; k < nm; ++k) {
                const int mb = members[k];
                hipStream_t ws = ls;
                if (forks > 1) {
                    if (k > 0) ws = h->fork[launched++ % forks];
                    for (int q = 0; q < n_swept; ++q) HIP_TRY(h, hipStreamWaitEvent(ws, swept[q], 0));
                }
                if (timing && mb != b0) HIP_TRY(h, hipEventRecord(h->tbin_ev[3 * mb + 1], ws));
                HIP_TRY(h, walk(mb, ws));
                if (timing) HIP_TRY(h, hipEventRecord(h->tbin_ev[3 * mb + 2], ws));
            }
        }
        for (int b = n_tb - 1; b >= 0; --b) {
            if (h->tfam_first[b] >= 0 || !reachable(b)) continue;
            const BinInfo& e = h->tbins[b];
            const int64_t need = (cap / e.ppw + 1 + kWavesPerBlock - 1) / kWavesPerBlock;
            hipStream_t ls = forks > 1 ? h->fork[launched++ % forks] : stream;
            if (timing) HIP_TRY(h, hipEventRecord(h->tbin_ev[3 * b], ls));
            // the column-word kernel takes the bin's small-alphabet items,
            // the table kernel the rest, one after the other on the bin's
            // stream; a kernel with no items returns at once
            for (int v = 1; v >= 0; --v) {
                if (!wants(e, v)) continue;
                const int blocks = (int)std::min<int64_t>(need, (v ? h->tresident_col : h->tresident)[b]);
                set_range(K, b, v);
                hipLaunchKernelGGL(trace_kernel(e.prec, e.W, e.R, v == 1), dim3(blocks), dim3(kBlock), 0, ls, K,
                                   T);
                HIP_TRY(h, hipGetLastError());
            }
            if (timing) HIP_TRY(h, hipEventRecord(h->tbin_ev[3 * b + 1], ls));
            HIP_TRY(h, walk(b, ls));
            if (timing) HIP_TRY(h, hipEventRecord(h->tbin_ev[3 * b + 2], ls));
        }
        for (int f = 0; forks > 1 && f < forks; ++f) {
            HIP_TRY(h, hipEventRecord(h->fork_ev[f], h->fork[f]));
            HIP_TRY(h, hipStreamWaitEvent(stream, h->fork_ev[f], 0));
        }
        if (timing) {
            HIP_TRY(h, hipStreamSynchronize(stream));
            for (int b = 0; b < n_tb; ++b) {
                if (!reachable(b)) continue;   // not launched
                // a family launch's sweep is timed once (at its first bin)
                // and shared by its bins; every bin has its own walk
                const int b0 = h->tfam_first[b] >= 0 ? h->tfam_first[b] : b;
                float a = 0, w = 0;
                HIP_TRY(h, hipEventElapsedTime(&a, h->tbin_ev[3 * b0], h->tbin_ev[3 * b0 + 1]));
                HIP_TRY(h, hipEventElapsedTime(&w, h->tbin_ev[3 * b + 1], h->tbin_ev[3 * b + 2]));
                if (b0 == b) h->t_path_sweep += a;
                h->t_path_walk += w;
                bin_ms[b] += a;
            }
        }
    }
    HIP_TRY(h, hipMemcpyAsync(h->h_small, h->d_small, kSmallInts * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(h, hipStreamSynchronize(stream));
    const int32_t* flags = h->h_small;
    const unsigned long long* cnt = counters(h->h_small);
    h->last_path_cells = (int64_t)cnt[kCtrTraceCells];
    for (int b = 0; b < n_tb; ++b) {
        sw_bin_stat st;
        memset(&st, 0, sizeof(st));
        st.pass = 2;
        st.precision = h->tbins[b].prec;
        st.lanes = h->tbins[b].W;
        st.rows = h->tbins[b].R;
        st.column = h->tbins[b].col && any_col ? 1 : 0;   // its column-word pairs took column words
        st.tile = kChunk;
        st.pairs = (int64_t)cnt[kCtrTraceBinPairs + b];
        st.cells = (int64_t)cnt[kCtrTraceBinCells + b];
        st.ms = bin_ms[b];
        // launch index: the family launch's first bin, or the bin itself
        // (box sweeps launch the largest shapes first)
        const int b0 = (size_t)b < h->tfam_first.size() && h->tfam_first[b] >= 0 ? h->tfam_first[b] : b;
        st.launch = n_tb - 1 - b0;
        if (b0 != b || ((size_t)b < h->tfam_first.size() && h->tfam_first[b] == b)) {
            const TraceFamily* f = trace_family(st.precision, st.lanes, st.rows);
            if (f) {
                st.family_hi = f->rows[0];
                st.family_lo = f->rows[f->n - 1];
            }
        }
        h->bin_stats.push_back(st);
    }
    for (int b = 0; b < n_tb; ++b)
        if (!reachable(b) && cnt[kCtrTraceBinPairs + b] != 0)
            return fail(h, SW_EINTERNAL, "a pair reached path-sweep bin %d, which was not launched", b);
    if (flags[kFlagInternal]) return fail(h, SW_EINTERNAL, "an alignment path could not be recovered");
    if (flags[kFlagPathRoom])
        return fail(h, SW_EINVAL, "the output room of a pair is too small for its path (cigar_len = -1)");
    return SW_OK;
}

extern "C" {

int sw_align_cigar(sw_handle* h, const sw_batch* batch, const sw_scheme* schemes, int n_schemes, sw_result* out,
                   const int64_t* cigar_off, uint32_t* cigar, int32_t* cigar_len, void* stream) {
    if (!h) return SW_EINVAL;
    if (!batch) return fail(h, SW_EINVAL, "null batch");
    h->last_path_cells = h->last_path_bytes = 0;
    h->last_path_chunks = 0;
    h->t_path_sweep = h->t_path_walk = 0.f;
    if (batch->n_pairs > 0 && (!cigar_off || !cigar || !cigar_len))
        return fail(h, SW_EINVAL, "null cigar buffer with n_pairs > 0");
    const int rc = sw_align_batch(h, batch, schemes, n_schemes, out, stream);
    if (rc != SW_OK || batch->n_pairs == 0) return rc;
    return trace_paths(h, batch, schemes, n_schemes, out, cigar_off, cigar, cigar_len, (hipStream_t)stream);
}

int sw_last_cigar_stats(sw_handle* h, int64_t* box_cells, int64_t* record_bytes, int32_t* chunks, float* sweep_ms,
                        float* walk_ms) {
    if (!h) return SW_EINVAL;
    if (box_cells) *box_cells = h->last_path_cells;
    if (record_bytes) *record_bytes = h->last_path_bytes;
    if (chunks) *chunks = h->last_path_chunks;
    if (sweep_ms) *sweep_ms = h->t_path_sweep;
    if (walk_ms) *walk_ms = h->t_path_walk;
    return SW_OK;
}

}  // extern "C"

// ---- database search ---------------------------------------------------------------

extern "C" int sw_search(sw_handle* h, const uint8_t* query, int64_t q_len, const uint8_t* refs,
                         const int64_t* r_off, int64_t n_refs, const sw_scheme* scheme, sw_result* out,
                         void* stream_ptr) {
    if (!h) return SW_EINVAL;
    h->err.clear();
    if (n_refs < 0 || n_refs > (int64_t)0x7FFFFFFF) return fail(h, SW_EINVAL, "n_refs must be 0..2^31-1");
    if (q_len < 0) return fail(h, SW_EINVAL, "negative query length");
    if (q_len > SW_MAX_QUERY)
        return fail(h, SW_ETOOLONG, "a query exceeds %d or a reference exceeds %d residues", SW_MAX_QUERY, SW_MAX_REF);
    if (!scheme) return fail(h, SW_EINVAL, "null scheme");
    if (n_refs == 0) return SW_OK;
    if (!refs || !r_off || !out || (q_len > 0 && !query))
        return fail(h, SW_EINVAL, "null device pointer with n_refs > 0");
    hipStream_t stream = (hipStream_t)stream_ptr;
    HIP_TRY(h, hipSetDevice(h->device));
    if (n_refs > h->search_cap) {
        drop_graph(h);
        free_dev(h->d_qspan);
        h->d_qspan = nullptr;
        h->search_cap = 0;
        h->search_len = -1;
        const int64_t cap = std::max<int64_t>(n_refs, 4096);
        if (hipMalloc(&h->d_qspan, 2 * cap * 8) != hipSuccess)
            return fail(h, SW_ENOMEM, "device allocation of %lld query spans failed", (long long)cap);
        h->search_cap = cap;
    }
    int64_t* beg = h->d_qspan;
    int64_t* end = h->d_qspan + h->search_cap;
    if (q_len != h->search_len) {
        // every pair reads the same query: spans [0, q_len) over `query`
        HIP_TRY(h, launch_fill_span(beg, end, h->search_cap, q_len, stream));
        h->search_len = q_len;
    }
    const uint8_t* qptr = query ? query : refs;   // an empty query is never read
    return align_spans(h, qptr, beg, end, refs, r_off, r_off + 1, nullptr, n_refs, scheme, 1, out, stream, false,
                       q_len);
}
