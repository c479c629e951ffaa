// sw_server.hip -- continuous-batching request loop over libswalign.
//
// Requests (batches of pairs, host arrays) are submitted at any time.  Each is
// checked and staged on the host, then admitted into a device-resident
// sequence pool when the pool has room (admission by memory budget, FIFO).
// K slot workers, each owning a handle and a stream, repeatedly take every
// admitted request that fits the slot's pair budget, merge them into one
// span-based batch (the sequences stay where admission put them; only the
// 8-byte spans are gathered), align it, hand each request its results and
// release its pool memory.  Requests arriving while others are on the GPU
// join the next batch of whichever slot frees first, so their work overlaps
// on the device with the batches already running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sw_internal.h"
#include "sw_pool.h"

using namespace sw;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int64_t n_pairs = 0;
    int64_t seq_bytes = 0;              // queries then references
    std::vector<uint8_t> data;          // staged residues
    std::vector<int64_t> spans;         // 4 x n_pairs, offsets within `data`
    std::vector<uint8_t> sid;
    int64_t pool_bytes = 0;
    int64_t pool_off = -1;
    std::vector<sw_result> results;
    Clock::time_point t_submit, t_done;
    int state = 0;                      // 0 waiting, 1 admitted, 2 running, 3 done
    int status = SW_OK;
};

// One gather segment: copy n spans/ids of a request's pool block into the
// merged batch at position dst.
struct Seg {
    int64_t src;      // pool offset of the request's span block
    int64_t n;
    int64_t dst;
};

__global__ void gather_spans_kernel(const Seg* segs, const uint8_t* pool, int64_t* qb, int64_t* qe,
                                    int64_t* rb, int64_t* re, uint8_t* sid) {
    const Seg s = segs[blockIdx.x];
    const int64_t* sp = reinterpret_cast<const int64_t*>(pool + s.src);
    const uint8_t* ids = pool + s.src + 32 * s.n;
    for (int64_t i = threadIdx.x; i < s.n; i += blockDim.x) {
        qb[s.dst + i] = sp[i];
        qe[s.dst + i] = sp[s.n + i];
        rb[s.dst + i] = sp[2 * s.n + i];
        re[s.dst + i] = sp[3 * s.n + i];
        sid[s.dst + i] = ids[i];
    }
}

// Batches of at most kLatencyPairs pairs (a request or a few, at low load)
// run on a slot's latency handle, whose routing has few bins: 16x16 up to
// 256 rows, 32x16 up to 512, and one cooperative 256-lane shape (8 rows per
// lane) above.  The sweeps of a pass run bin by bin on each of a handle's
// streams, so a small batch waits for the sum of its bins' longest pairs;
// with three bins that sum is about half of the default routing's (single
// mixed requests: 6.4 ms against 13 ms at the median).  Larger merged
// batches run on the throughput handle, with the routing of the server's
// tuning string (or the built-in one).
constexpr int64_t kLatencyPairs = 8192;
constexpr const char* kLatencyRoute = "route16=16x16@256/32x16@512/256x8@2048";

struct Slot {
    sw_handle* h = nullptr;       // throughput handle
    sw_handle* hl = nullptr;      // latency handle
    hipStream_t stream = nullptr;
    int64_t* d_spans = nullptr;   // 4 x max_pairs
    uint8_t* d_sid = nullptr;
    sw_result* d_out = nullptr;
    Seg* d_segs = nullptr;
    Seg* h_segs = nullptr;        // pinned
    sw_result* h_out = nullptr;   // pinned
    std::thread th;
};

}  // namespace

struct sw_server {
    int device = 0;
    std::string err;
    std::vector<std::vector<int8_t>> mats;
    std::vector<sw_scheme> schemes;
    int64_t max_pairs = 0;
    uint8_t* pool = nullptr;
    PoolAllocator alloc;
    std::vector<std::unique_ptr<Slot>> slots;
    hipStream_t admit_stream = nullptr;
    uint8_t* stage = nullptr;           // pinned host staging of the admission thread
    std::thread admit_th;

    std::mutex mu;
    std::condition_variable cv_admit, cv_ready, cv_done;
    std::deque<Request*> waiting, ready;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    int64_t n_done = 0, n_batches = 0, pairs_done = 0;
    double t_admit = 0, t_align = 0, t_fetch = 0;   // cumulative milliseconds
};

// Pageable host memory is copied to the device through this pinned staging
// buffer, in chunks of at most its size.
constexpr int64_t kStageBytes = 32 << 20;

static int sfail(sw_server* s, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (s) {
        std::lock_guard<std::mutex> g(s->mu);
        s->err = buf;
    }
    return code;
}

static int64_t span_block_bytes(int64_t n) { return PoolAllocator::round_up(32 * n + n); }

static void admission_loop(sw_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_admit.wait(lk, [&] { return S->stop || !S->waiting.empty(); });
        if (S->stop) return;
        Request* r = S->waiting.front();
        const int64_t off = S->alloc.alloc(r->pool_bytes);
        if (off < 0) {
            // wait until a batch releases memory (cv_admit is notified then)
            S->cv_admit.wait(lk);
            continue;
        }
        S->waiting.pop_front();
        r->pool_off = off;
        lk.unlock();
        const Clock::time_point t0 = Clock::now();
        // pool block: sequences, then the absolute spans and scheme ids of
        // the request; assembled in pinned memory chunk by chunk and copied
        const int64_t seq = PoolAllocator::round_up(r->seq_bytes);
        const int64_t total = seq + 33 * r->n_pairs;
        bool ok = true;
        for (int64_t c0 = 0; ok && c0 < total; c0 += kStageBytes) {
            const int64_t c1 = std::min(total, c0 + kStageBytes);
            for (int64_t x = c0; x < c1;) {
                if (x < r->seq_bytes) {
                    const int64_t e = std::min(c1, r->seq_bytes);
                    memcpy(S->stage + (x - c0), r->data.data() + x, e - x);
                    x = e;
                } else if (x < seq) {
                    const int64_t e = std::min(c1, seq);
                    memset(S->stage + (x - c0), 0, e - x);
                    x = e;
                } else if (x < seq + 32 * r->n_pairs) {
                    // spans are 8-byte values and seq is 256-aligned, so a
                    // chunk boundary (a multiple of kStageBytes) never splits one
                    const int64_t e = std::min(c1, seq + 32 * r->n_pairs);
                    int64_t* dst = reinterpret_cast<int64_t*>(S->stage + (x - c0));
                    for (int64_t k = (x - seq) / 8; k < (e - seq) / 8; ++k) *dst++ = r->spans[k] + off;
                    x = e;
                } else {
                    const int64_t b = x - seq - 32 * r->n_pairs;
                    memcpy(S->stage + (x - c0), r->sid.data() + b, c1 - x);
                    x = c1;
                }
            }
            ok = hipMemcpyAsync(S->pool + off + c0, S->stage, c1 - c0, hipMemcpyHostToDevice, S->admit_stream) ==
                     hipSuccess &&
                 hipStreamSynchronize(S->admit_stream) == hipSuccess;
        }
        const double ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        lk.lock();
        S->t_admit += ms;
        std::vector<uint8_t>().swap(r->data);
        if (!ok) {
            S->alloc.release(off);
            r->pool_off = -1;
            r->status = SW_EDEVICE;
            r->state = 3;
            r->t_done = Clock::now();
            S->cv_done.notify_all();
            continue;
        }
        r->state = 1;
        S->ready.push_back(r);
        S->cv_ready.notify_one();
    }
}

static void slot_loop(sw_server* S, Slot* slot) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_ready.wait(lk, [&] { return S->stop || !S->ready.empty(); });
        if (S->stop) return;
        std::vector<Request*> batch;
        int64_t total = 0;
        while (!S->ready.empty()) {
            Request* r = S->ready.front();
            if (!batch.empty() && total + r->n_pairs > S->max_pairs) break;
            S->ready.pop_front();
            r->state = 2;
            batch.push_back(r);
            total += r->n_pairs;
        }
        lk.unlock();
        int status = SW_OK;
        const int64_t P = total;
        const Clock::time_point t0 = Clock::now();
        for (size_t k = 0, at = 0; k < batch.size(); ++k) {
            const Request* r = batch[k];
            slot->h_segs[k].src = r->pool_off + PoolAllocator::round_up(r->seq_bytes);
            slot->h_segs[k].n = r->n_pairs;
            slot->h_segs[k].dst = (int64_t)at;
            at += r->n_pairs;
        }
        const int nseg = (int)batch.size();
        if (hipMemcpyAsync(slot->d_segs, slot->h_segs, nseg * sizeof(Seg), hipMemcpyHostToDevice, slot->stream) !=
            hipSuccess)
            status = SW_EDEVICE;
        if (status == SW_OK) {
            int64_t* qb = slot->d_spans;
            hipLaunchKernelGGL(gather_spans_kernel, dim3(nseg), dim3(256), 0, slot->stream, slot->d_segs, S->pool,
                               qb, qb + S->max_pairs, qb + 2 * S->max_pairs, qb + 3 * S->max_pairs, slot->d_sid);
            if (hipGetLastError() != hipSuccess) status = SW_EDEVICE;
        }
        sw_handle* hh = P <= kLatencyPairs ? slot->hl : slot->h;
        if (status == SW_OK) {
            int64_t* qb = slot->d_spans;
            status = sw_align_spans(hh, S->pool, qb, qb + S->max_pairs, S->pool, qb + 2 * S->max_pairs,
                                    qb + 3 * S->max_pairs, slot->d_sid, P, S->schemes.data(),
                                    (int)S->schemes.size(), slot->d_out, slot->stream);
        }
        const Clock::time_point t1 = Clock::now();
        if (status == SW_OK && P > 0) {
            if (hipMemcpyAsync(slot->h_out, slot->d_out, P * sizeof(sw_result), hipMemcpyDeviceToHost,
                               slot->stream) != hipSuccess ||
                hipStreamSynchronize(slot->stream) != hipSuccess)
                status = SW_EDEVICE;
        }
        std::string why = status == SW_OK ? std::string() : std::string(sw_last_error(hh));
        lk.lock();
        const Clock::time_point now = Clock::now();
        S->t_align += std::chrono::duration<double, std::milli>(t1 - t0).count();
        S->t_fetch += std::chrono::duration<double, std::milli>(now - t1).count();
        for (size_t k = 0, at = 0; k < batch.size(); ++k) {
            Request* r = batch[k];
            if (status == SW_OK) r->results.assign(slot->h_out + at, slot->h_out + at + r->n_pairs);
            at += r->n_pairs;
            r->status = status;
            r->state = 3;
            r->t_done = now;
            S->alloc.release(r->pool_off);
            r->pool_off = -1;
        }
        if (status != SW_OK) S->err = why;
        S->n_done += (int64_t)batch.size();
        S->pairs_done += P;
        S->n_batches += 1;
        S->cv_done.notify_all();
        S->cv_admit.notify_all();
    }
}

extern "C" {

sw_server* sw_server_create(int device, const sw_scheme* schemes, int n_schemes, int64_t pool_bytes, int n_slots,
                            int64_t max_batch_pairs, const char* tuning) {
    if (!schemes || n_schemes < 1 || n_schemes > SW_MAX_SCHEMES || pool_bytes <= 0 || n_slots < 1 ||
        n_slots > 16 || max_batch_pairs < 1)
        return nullptr;
    for (int k = 0; k < n_schemes; ++k) {
        const sw_scheme& sc = schemes[k];
        if (!sc.matrix || sc.alphabet < 1 || sc.alphabet > SW_MAX_ALPHABET || sc.gap_open < 1 ||
            sc.gap_extend < 0 || sc.gap_extend > sc.gap_open)
            return nullptr;
    }
    if (hipSetDevice(device) != hipSuccess) return nullptr;
    sw_server* S = new sw_server();
    S->device = device;
    S->max_pairs = max_batch_pairs;
    for (int k = 0; k < n_schemes; ++k) {
        S->mats.emplace_back(schemes[k].matrix, schemes[k].matrix + schemes[k].alphabet * schemes[k].alphabet);
        sw_scheme c = schemes[k];
        S->schemes.push_back(c);
    }
    for (int k = 0; k < n_schemes; ++k) S->schemes[k].matrix = S->mats[k].data();
    bool ok = hipMalloc(&S->pool, pool_bytes) == hipSuccess &&
              hipHostMalloc(&S->stage, kStageBytes, hipHostMallocDefault) == hipSuccess &&
              hipStreamCreateWithFlags(&S->admit_stream, hipStreamNonBlocking) == hipSuccess;
    if (ok) S->alloc.reset(pool_bytes);
    const std::string lat_tuning = std::string(tuning ? tuning : "") + ";" + kLatencyRoute;
    for (int k = 0; ok && k < n_slots; ++k) {
        std::unique_ptr<Slot> sl(new Slot());
        sl->h = sw_create(device, tuning);
        sl->hl = sw_create(device, lat_tuning.c_str());
        ok = sl->h && sl->hl && sw_set_option(sl->h, "capacity", max_batch_pairs) == SW_OK &&
             sw_set_option(sl->hl, "capacity", std::min<int64_t>(max_batch_pairs, kLatencyPairs)) == SW_OK &&
             hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) == hipSuccess &&
             hipMalloc(&sl->d_spans, 32 * max_batch_pairs) == hipSuccess &&
             hipMalloc(&sl->d_sid, max_batch_pairs) == hipSuccess &&
             hipMalloc(&sl->d_out, max_batch_pairs * sizeof(sw_result)) == hipSuccess &&
             hipMalloc(&sl->d_segs, max_batch_pairs * sizeof(Seg)) == hipSuccess &&
             hipHostMalloc(&sl->h_segs, max_batch_pairs * sizeof(Seg), hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc(&sl->h_out, max_batch_pairs * sizeof(sw_result), hipHostMallocDefault) == hipSuccess;
        S->slots.push_back(std::move(sl));
    }
    // Each slot's calls always use the same buffers, schemes and capacity,
    // so one captured graph serves all of them (the batch size is read on
    // the device).  It is captured here, on this thread, one slot after the
    // other, by aligning one pair of zero residues at the start of the
    // pool: captures running on several threads at once have been
    // invalidated by the runtime.  A slot whose capture is refused runs
    // its calls eagerly and never captures.
    if (ok) ok = hipMemset(S->pool, 0, 256) == hipSuccess;
    for (size_t k = 0; ok && k < S->slots.size(); ++k) {
        Slot* sl = S->slots[k].get();
        const int64_t one[4] = {0, 1, 0, 1};
        for (int f = 0; ok && f < 4; ++f)
            ok = hipMemcpy(sl->d_spans + f * max_batch_pairs, &one[f], 8, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemset(sl->d_sid, 0, 1) == hipSuccess;
        if (!ok) break;
        int64_t* qb = sl->d_spans;
        for (sw_handle* hh : {sl->h, sl->hl}) {
            ok = ok && sw_align_spans(hh, S->pool, qb, qb + max_batch_pairs, S->pool, qb + 2 * max_batch_pairs,
                                      qb + 3 * max_batch_pairs, sl->d_sid, 1, S->schemes.data(),
                                      (int)S->schemes.size(), sl->d_out, sl->stream) == SW_OK;
            int64_t captures = 0;
            if (ok && (sw_get_option(hh, "captures", &captures) != SW_OK || captures != 1))
                ok = sw_set_option(hh, "graph", 0) == SW_OK;
        }
    }
    if (!ok) {
        sw_server_destroy(S);
        return nullptr;
    }
    S->admit_th = std::thread(admission_loop, S);
    for (auto& sl : S->slots) sl->th = std::thread(slot_loop, S, sl.get());
    return S;
}

void sw_server_destroy(sw_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_admit.notify_all();
    S->cv_ready.notify_all();
    S->cv_done.notify_all();
    if (S->admit_th.joinable()) S->admit_th.join();
    for (auto& sl : S->slots)
        if (sl->th.joinable()) sl->th.join();
    (void)hipSetDevice(S->device);
    for (auto& sl : S->slots) {
        if (sl->stream) (void)hipStreamSynchronize(sl->stream);
        if (sl->h) sw_destroy(sl->h);
        if (sl->hl) sw_destroy(sl->hl);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
        if (sl->d_spans) (void)hipFree(sl->d_spans);
        if (sl->d_sid) (void)hipFree(sl->d_sid);
        if (sl->d_out) (void)hipFree(sl->d_out);
        if (sl->d_segs) (void)hipFree(sl->d_segs);
        if (sl->h_segs) (void)hipHostFree(sl->h_segs);
        if (sl->h_out) (void)hipHostFree(sl->h_out);
    }
    if (S->admit_stream) (void)hipStreamDestroy(S->admit_stream);
    if (S->stage) (void)hipHostFree(S->stage);
    if (S->pool) (void)hipFree(S->pool);
    delete S;
}

const char* sw_server_last_error(sw_server* S) {
    if (!S) return "null server";
    std::lock_guard<std::mutex> g(S->mu);
    static thread_local std::string copy;
    copy = S->err;
    return copy.c_str();
}

int sw_server_submit(sw_server* S, const uint8_t* queries, const int64_t* q_off, const uint8_t* refs,
                     const int64_t* r_off, const uint8_t* scheme_id, int64_t n_pairs, uint64_t* ticket) {
    if (!S || !ticket) return SW_EINVAL;
    if (n_pairs < 0) return sfail(S, SW_EINVAL, "negative n_pairs");
    if (n_pairs > S->max_pairs) return sfail(S, SW_EINVAL, "request larger than the slot pair budget");
    if (n_pairs > 0 && (!q_off || !r_off)) return sfail(S, SW_EINVAL, "null offsets");
    std::unique_ptr<Request> r(new Request());
    r->t_submit = Clock::now();   // latency includes the host checks and staging
    r->n_pairs = n_pairs;
    // host checks: the whole request is rejected here rather than failing a
    // merged batch later
    const int64_t qn = n_pairs > 0 ? q_off[n_pairs] - q_off[0] : 0;
    const int64_t rn = n_pairs > 0 ? r_off[n_pairs] - r_off[0] : 0;
    if (qn < 0 || rn < 0) return sfail(S, SW_EINVAL, "offsets decrease");
    if ((qn > 0 && !queries) || (rn > 0 && !refs)) return sfail(S, SW_EINVAL, "null sequences");
    r->spans.resize(4 * n_pairs);
    r->sid.resize(n_pairs);
    for (int64_t i = 0; i < n_pairs; ++i) {
        const int64_t n = q_off[i + 1] - q_off[i], m = r_off[i + 1] - r_off[i];
        if (n < 0 || m < 0) return sfail(S, SW_EINVAL, "offsets decrease");
        if (n > SW_MAX_QUERY || m > SW_MAX_REF)
            return sfail(S, SW_ETOOLONG, "a query exceeds %d or a reference exceeds %d residues", SW_MAX_QUERY,
                         SW_MAX_REF);
        const int s = scheme_id ? scheme_id[i] : 0;
        if (s >= (int)S->schemes.size()) return sfail(S, SW_EINVAL, "scheme id out of range");
        const int A = S->schemes[s].alphabet;
        for (int64_t k = q_off[i]; k < q_off[i + 1]; ++k)
            if (queries[k] >= A) return sfail(S, SW_EINVAL, "residue code outside its scheme's alphabet");
        for (int64_t k = r_off[i]; k < r_off[i + 1]; ++k)
            if (refs[k] >= A) return sfail(S, SW_EINVAL, "residue code outside its scheme's alphabet");
        r->spans[i] = q_off[i] - q_off[0];
        r->spans[n_pairs + i] = q_off[i + 1] - q_off[0];
        r->spans[2 * n_pairs + i] = qn + r_off[i] - r_off[0];
        r->spans[3 * n_pairs + i] = qn + r_off[i + 1] - r_off[0];
        r->sid[i] = (uint8_t)s;
    }
    r->seq_bytes = qn + rn;
    r->data.resize(r->seq_bytes);
    if (qn) memcpy(r->data.data(), queries + q_off[0], qn);
    if (rn) memcpy(r->data.data() + qn, refs + r_off[0], rn);
    r->pool_bytes = PoolAllocator::round_up(r->seq_bytes) + span_block_bytes(n_pairs);
    if (r->pool_bytes > S->alloc.capacity())
        return sfail(S, SW_ENOMEM, "request needs %lld bytes, more than the whole pool", (long long)r->pool_bytes);
    std::lock_guard<std::mutex> g(S->mu);
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    Request* raw = r.get();
    S->reqs[r->ticket] = std::move(r);
    if (n_pairs == 0) {
        raw->state = 3;
        raw->t_done = raw->t_submit;
        S->cv_done.notify_all();
    } else {
        S->waiting.push_back(raw);
        S->cv_admit.notify_one();
    }
    return SW_OK;
}

int sw_server_poll(sw_server* S, uint64_t ticket, sw_result* out, int wait, double* latency_ms) {
    if (!S) return SW_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        S->err = "unknown ticket";
        return SW_EINVAL;
    }
    Request* r = it->second.get();
    if (wait) S->cv_done.wait(lk, [&] { return r->state == 3 || S->stop; });
    if (r->state != 3) return SW_PENDING;
    const int status = r->status;
    if (status == SW_OK && out && r->n_pairs > 0) memcpy(out, r->results.data(), r->n_pairs * sizeof(sw_result));
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    S->reqs.erase(it);
    return status;
}

int sw_server_stats(sw_server* S, int64_t* pool_peak_bytes, int64_t* pool_capacity, int64_t* requests_done,
                    int64_t* batches, int64_t* pairs_done) {
    if (!S) return SW_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    if (pool_peak_bytes) *pool_peak_bytes = S->alloc.peak();
    if (pool_capacity) *pool_capacity = S->alloc.capacity();
    if (requests_done) *requests_done = S->n_done;
    if (batches) *batches = S->n_batches;
    if (pairs_done) *pairs_done = S->pairs_done;
    return SW_OK;
}

int sw_server_timing(sw_server* S, double* admit_ms, double* align_ms, double* fetch_ms) {
    if (!S) return SW_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    if (admit_ms) *admit_ms = S->t_admit;
    if (align_ms) *align_ms = S->t_align;
    if (fetch_ms) *fetch_ms = S->t_fetch;
    return SW_OK;
}

}  // extern "C"
