// foldin.cpp -- fold-in serving: resident posterior samples, a request queue
// and a continuous-batching scheduler thread.
//
// A fold-in request is a new user with n (movie, rating) pairs.  For each of
// the S stored samples (V^(s), mu_U^(s), Lambda_U^(s)) the user's factor is
// drawn from the same row conditional as Algorithm 1's user loop, the user
// scores every movie against V^(s), and the request returns the top-n
// unrated movies by predictive mean with their predictive variance.
//
// Scheduling: submissions (any thread) go to one FIFO per size class (by
// number of ratings).  kSlots staging slots, each with its own HIP stream,
// carry batches: whenever a slot is free the scheduler thread takes the size
// class whose oldest request is the oldest overall, packs that class's
// requests (oldest first) and then requests of smaller classes while they fit
// the slot's memory (rating and request capacity), and launches the batch's
// H2D copy, draw, score, top-n and D2H copy on the slot's stream.  A batch's
// time is set by its largest request, so a batch never takes a request of a
// larger class than the one it was opened for: small requests do not wait
// behind large ones, and the batches of several slots run on the device at
// the same time.  Requests are admitted as slots free up; a request larger
// than a slot's rating capacity is refused at submission.  Completions are
// found by polling each busy slot's event.  Every per-request result
// depends only on that request (each draw, score and selection is computed
// independently of the others in its batch), so a request's result is the
// same alone and in any mix.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bpmf.h"
#include "internal.h"

namespace bpmf {

size_t foldin_topk_lds(int N, int top_max);

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kTopMax = 1024;       // largest top_n (power of two for the sort)
constexpr int kBatchReq = 64;       // requests per batch
constexpr int kSlots = 4;           // staging slots, one stream each
constexpr int kClasses = 4;         // size classes of the request queue
constexpr size_t kMaxPending = 1u << 20;

// Size class of a request with n ratings: up to 32, 256, 2048, more.
int size_class(size_t n) { return n <= 32 ? 0 : (n <= 256 ? 1 : (n <= 2048 ? 2 : 3)); }

struct Request {
    uint64_t id = 0;
    std::vector<int32_t> movie;
    std::vector<float> rc;  // centred ratings
    int top_n = 0;
    Clock::time_point t_submit, t_done;
    bool done = false;
    std::vector<int32_t> ids;
    std::vector<float> mean, var;
};

struct Slot {
    // device
    int32_t *d_nbr = nullptr;
    float *d_rc = nullptr;
    FoldItem *d_items = nullptr;
    uint64_t *d_req = nullptr;
    int32_t *d_beg = nullptr;
    int32_t *d_topn = nullptr;
    float *d_U = nullptr, *d_mean = nullptr, *d_var = nullptr;
    int32_t *d_oid = nullptr;
    float *d_omean = nullptr, *d_ovar = nullptr;
    // pinned host staging
    int32_t *h_nbr = nullptr;
    float *h_rc = nullptr;
    FoldItem *h_items = nullptr;
    uint64_t *h_req = nullptr;
    int32_t *h_beg = nullptr, *h_topn = nullptr;
    int32_t *h_oid = nullptr;
    float *h_omean = nullptr, *h_ovar = nullptr;
    hipEvent_t done = nullptr;
    hipStream_t stream = nullptr;
    bool busy = false;
    std::vector<std::shared_ptr<Request>> reqs;
};

}  // namespace

struct FoldinState {
    int S_cap = 0;
    int n_stored = 0;
    int next_slot = 0;
    float *Vring = nullptr, *Lam_ring = nullptr, *Lmu_ring = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Request>> pending[kClasses];
    size_t n_pending = 0;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> table;
    uint64_t next_id = 1;
    std::thread th;
    bool stop = false;
    bool storing = false;
    int inflight = 0;
    Slot slots[kSlots];
    int64_t R_max = 0;  // ratings per batch
    std::string dev_err;
    // statistics
    int64_t n_batches = 0, n_launched = 0;
    int max_batch = 0, max_inflight = 0;
};

namespace {

template <typename T>
hipError_t dal(T **p, size_t n)
{
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

template <typename T>
hipError_t hal(T **p, size_t n)
{
    return hipHostMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault);
}

void free_slot(Slot &s)
{
    void *d[] = {s.d_nbr, s.d_rc, s.d_items, s.d_req, s.d_beg, s.d_topn, s.d_U,
                 s.d_mean, s.d_var, s.d_oid, s.d_omean, s.d_ovar};
    for (void *p : d) (void)hipFree(p);
    void *h[] = {s.h_nbr, s.h_rc, s.h_items, s.h_req, s.h_beg, s.h_topn, s.h_oid, s.h_omean, s.h_ovar};
    for (void *p : h)
        if (p) (void)hipHostFree(p);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
}

hipError_t alloc_slot(Slot &s, const bpmf_ctx *c, int S, int64_t R)
{
    hipError_t e;
    const size_t B = kBatchReq;
#define A(x)                              \
    if ((e = (x)) != hipSuccess) return e;
    A(dal(&s.d_nbr, R));
    A(dal(&s.d_rc, R));
    A(dal(&s.d_items, B * S));
    A(dal(&s.d_req, B));
    A(dal(&s.d_beg, B + 1));
    A(dal(&s.d_topn, B));
    A(dal(&s.d_U, B * S * (size_t)c->ld));
    A(dal(&s.d_mean, B * (size_t)c->N));
    A(dal(&s.d_var, B * (size_t)c->N));
    A(dal(&s.d_oid, B * kTopMax));
    A(dal(&s.d_omean, B * kTopMax));
    A(dal(&s.d_ovar, B * kTopMax));
    A(hal(&s.h_nbr, R));
    A(hal(&s.h_rc, R));
    A(hal(&s.h_items, B * S));
    A(hal(&s.h_req, B));
    A(hal(&s.h_beg, B + 1));
    A(hal(&s.h_topn, B));
    A(hal(&s.h_oid, B * kTopMax));
    A(hal(&s.h_omean, B * kTopMax));
    A(hal(&s.h_ovar, B * kTopMax));
    A(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
    A(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
#undef A
    return hipSuccess;
}

// Pack pending requests into slot `sl` and launch its work: the size class
// holding the oldest request opens the batch, then that class and the
// smaller ones fill it, oldest first within each class, while the slot's
// rating and request capacity allow.  Called with the lock held; releases it
// while staging and launching.
hipError_t launch_batch(bpmf_ctx *c, FoldinState &f, Slot &sl, std::unique_lock<std::mutex> &lk)
{
    sl.reqs.clear();
    int open = -1;
    for (int k = 0; k < kClasses; ++k)
        if (!f.pending[k].empty() && (open < 0 || f.pending[k].front()->id < f.pending[open].front()->id))
            open = k;
    int64_t R = 0;
    for (int k = open; k >= 0 && (int)sl.reqs.size() < kBatchReq; --k) {
        auto &q = f.pending[k];
        while (!q.empty() && (int)sl.reqs.size() < kBatchReq) {
            auto &r = q.front();
            if (R + (int64_t)r->movie.size() > f.R_max && !sl.reqs.empty()) break;
            R += (int64_t)r->movie.size();
            sl.reqs.push_back(r);
            q.pop_front();
        }
    }
    f.n_pending -= sl.reqs.size();
    const int S = f.n_stored;
    sl.busy = true;
    ++f.inflight;
    ++f.n_batches;
    f.n_launched += (int64_t)sl.reqs.size();
    f.max_batch = std::max(f.max_batch, (int)sl.reqs.size());
    f.max_inflight = std::max(f.max_inflight, f.inflight);
    lk.unlock();
    // largest requests first in the draw launch; outputs are indexed by
    // position in the batch
    const int nb = (int)sl.reqs.size();
    std::vector<int> order(nb);
    for (int i = 0; i < nb; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return sl.reqs[a]->movie.size() > sl.reqs[b]->movie.size();
    });
    int64_t off = 0;
    for (int i = 0; i < nb; ++i) {
        const Request &r = *sl.reqs[i];
        sl.h_beg[i] = (int32_t)off;
        sl.h_req[i] = r.id;
        sl.h_topn[i] = r.top_n;
        memcpy(sl.h_nbr + off, r.movie.data(), sizeof(int32_t) * r.movie.size());
        memcpy(sl.h_rc + off, r.rc.data(), sizeof(float) * r.rc.size());
        off += (int64_t)r.movie.size();
    }
    sl.h_beg[nb] = (int32_t)off;
    int64_t q = 0;
    for (int oi = 0; oi < nb; ++oi) {
        const int i = order[oi];
        for (int s = 0; s < S; ++s)
            sl.h_items[q++] = FoldItem{i, s, (int64_t)sl.h_beg[i], (int64_t)sl.h_beg[i + 1]};
    }
    hipStream_t st = sl.stream;
    hipError_t e;
#define A(x)                              \
    if ((e = (x)) != hipSuccess) return e;
    A(hipMemcpyAsync(sl.d_nbr, sl.h_nbr, sizeof(int32_t) * std::max<int64_t>(off, 1), hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(sl.d_rc, sl.h_rc, sizeof(float) * std::max<int64_t>(off, 1), hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(sl.d_items, sl.h_items, sizeof(FoldItem) * std::max<int64_t>(q, 1), hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(sl.d_req, sl.h_req, sizeof(uint64_t) * nb, hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(sl.d_beg, sl.h_beg, sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(sl.d_topn, sl.h_topn, sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
    A(launch_foldin_draw(c, sl.d_items, q, sl.d_nbr, sl.d_rc, f.Vring, f.Lam_ring, f.Lmu_ring,
                         sl.d_req, S, sl.d_U, st));
    A(launch_foldin_score(c, nb, S, f.Vring, sl.d_U, sl.d_mean, sl.d_var, st));
    A(launch_foldin_topk(c, nb, sl.d_mean, sl.d_var, sl.d_beg, sl.d_nbr, sl.d_topn, kTopMax,
                         sl.d_oid, sl.d_omean, sl.d_ovar, st));
    A(hipMemcpyAsync(sl.h_oid, sl.d_oid, sizeof(int32_t) * nb * kTopMax, hipMemcpyDeviceToHost, st));
    A(hipMemcpyAsync(sl.h_omean, sl.d_omean, sizeof(float) * nb * kTopMax, hipMemcpyDeviceToHost, st));
    A(hipMemcpyAsync(sl.h_ovar, sl.d_ovar, sizeof(float) * nb * kTopMax, hipMemcpyDeviceToHost, st));
    A(hipEventRecord(sl.done, st));
#undef A
    lk.lock();
    return hipSuccess;
}

// Copy a finished slot's results into its requests (lock held).
void complete_batch(FoldinState &f, Slot &sl, Clock::time_point now)
{
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        Request &r = *sl.reqs[i];
        const size_t o = i * kTopMax;
        r.ids.assign(sl.h_oid + o, sl.h_oid + o + r.top_n);
        r.mean.assign(sl.h_omean + o, sl.h_omean + o + r.top_n);
        r.var.assign(sl.h_ovar + o, sl.h_ovar + o + r.top_n);
        r.t_done = now;
        r.done = true;
    }
    sl.reqs.clear();
    sl.busy = false;
    --f.inflight;
}

void scheduler(bpmf_ctx *c)
{
    FoldinState &f = *c->foldin;
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(f.mu);
    for (;;) {
        if (f.stop && f.inflight == 0) break;
        bool progressed = false;
        // collect every finished batch
        for (auto &s : f.slots) {
            if (!s.busy) continue;
            hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) f.dev_err = hipGetErrorString(q);
            complete_batch(f, s, Clock::now());
            progressed = true;
        }
        if (progressed) f.cv.notify_all();
        // fill every free slot
        for (auto &s : f.slots) {
            if (f.stop || f.storing || f.n_pending == 0 || !f.dev_err.empty()) break;
            if (s.busy) continue;
            hipError_t e = launch_batch(c, f, s, lk);
            if (e != hipSuccess) {
                if (!lk.owns_lock()) lk.lock();
                f.dev_err = hipGetErrorString(e);
                complete_batch(f, s, Clock::now());  // its requests report the error on poll
            }
            progressed = true;
        }
        if (progressed) {
            f.cv.notify_all();
            continue;
        }
        if (f.inflight > 0) {
            f.cv.wait_for(lk, std::chrono::microseconds(20));
            continue;
        }
        f.cv.wait(lk, [&] { return f.stop || (f.n_pending > 0 && !f.storing); });
    }
}

int ffail(bpmf_ctx *c, int code, const char *msg)
{
    c->err = msg;
    return code;
}

}  // namespace

void foldin_destroy(bpmf_ctx *c)
{
    FoldinState *f = c->foldin;
    if (!f) return;
    {
        std::lock_guard<std::mutex> g(f->mu);
        f->stop = true;
        for (auto &q : f->pending) q.clear();
        f->n_pending = 0;
    }
    f->cv.notify_all();
    if (f->th.joinable()) f->th.join();
    for (auto &s : f->slots)
        if (s.stream) (void)hipStreamSynchronize(s.stream);
    for (auto &s : f->slots) free_slot(s);
    (void)hipFree(f->Vring);
    (void)hipFree(f->Lam_ring);
    (void)hipFree(f->Lmu_ring);
    delete f;
    c->foldin = nullptr;
}

}  // namespace bpmf

using namespace bpmf;

extern "C" {

int bpmf_store_sample(bpmf_ctx *c)
{
    if (!c) return BPMF_E_INVAL;
    if (c->sticky) return ffail(c, BPMF_E_DEVICE, "context unusable after a device error");
    if (!fast_path_available(c)) return ffail(c, BPMF_E_INVAL, "fold-in needs FP32 factors and K <= 64");
    if (foldin_topk_lds((int)c->N, kTopMax) > 65536)
        return ffail(c, BPMF_E_INVAL, "fold-in: N too large for one workgroup's LDS");
    hipError_t e;
    if (!c->foldin) {
        auto *f = new FoldinState();
        c->foldin = f;
        f->S_cap = c->foldin_S;
        const size_t vsz = (size_t)c->N * c->ld;
        // the pool holds the rated movies of the batches in flight (8 B per
        // rating, kSlots batches); score buffers and outputs are sized by the
        // batch limit
        const size_t pool = c->foldin_pool ? c->foldin_pool : (256ull << 20);
        f->R_max = (int64_t)std::min<size_t>(pool / (8 * kSlots), 1u << 28);
        if (f->R_max < 1) {
            foldin_destroy(c);
            return ffail(c, BPMF_E_INVAL, "fold-in pool too small");
        }
        e = dal(&f->Vring, vsz * f->S_cap);
        if (e == hipSuccess) e = dal(&f->Lam_ring, (size_t)f->S_cap * c->K * c->K);
        if (e == hipSuccess) e = dal(&f->Lmu_ring, (size_t)f->S_cap * c->K);
        for (int q = 0; q < kSlots && e == hipSuccess; ++q) e = alloc_slot(f->slots[q], c, f->S_cap, f->R_max);
        if (e != hipSuccess) {
            foldin_destroy(c);
            (void)hipGetLastError();
            return ffail(c, e == hipErrorOutOfMemory ? BPMF_E_NOMEM : BPMF_E_DEVICE, hipGetErrorString(e));
        }
        f->th = std::thread(scheduler, c);
    }
    FoldinState &f = *c->foldin;
    std::unique_lock<std::mutex> lk(f.mu);
    f.storing = true;  // no new batch reads the ring while it changes
    f.cv.wait(lk, [&] { return f.inflight == 0; });
    const int slot = f.next_slot;
    const size_t vsz = (size_t)c->N * c->ld;
    e = hipMemcpyAsync(f.Vring + slot * vsz, c->side[BPMF_SIDE_V].X, vsz * sizeof(float),
                       hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f.Lam_ring + (size_t)slot * c->K * c->K, c->side[BPMF_SIDE_U].Lam_w,
                           sizeof(float) * c->K * c->K, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f.Lmu_ring + (size_t)slot * c->K, c->side[BPMF_SIDE_U].Lmu_w,
                           sizeof(float) * c->K, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) {
        f.next_slot = (slot + 1) % f.S_cap;
        f.n_stored = std::min(f.n_stored + 1, f.S_cap);
    }
    f.storing = false;
    lk.unlock();
    f.cv.notify_all();
    if (e != hipSuccess) {
        c->sticky = true;
        return ffail(c, BPMF_E_DEVICE, hipGetErrorString(e));
    }
    return BPMF_OK;
}

int bpmf_foldin_submit(bpmf_ctx *c, int32_t n, const int32_t *movie, const float *rating,
                       int32_t top_n, uint64_t *req_id)
{
    if (!c || !req_id || n < 0 || (n > 0 && (!movie || !rating))) return BPMF_E_INVAL;
    if (top_n < 1 || top_n > kTopMax) return BPMF_E_INVAL;
    FoldinState *f = c->foldin;
    if (!f) return BPMF_E_NOSAMPLES;
    {
        std::lock_guard<std::mutex> g(f->mu);
        if (f->n_stored == 0) return BPMF_E_NOSAMPLES;
    }
    if (n > f->R_max) return BPMF_E_TOOBIG;
    auto r = std::make_shared<Request>();
    r->movie.assign(movie, movie + n);
    r->rc.resize(n);
    {
        // range and duplicate check in O(n): one bit per movie, per calling
        // thread, cleared again before returning
        thread_local std::vector<uint64_t> seen;
        if (seen.size() < (size_t)(c->N + 63) / 64) seen.assign((size_t)(c->N + 63) / 64, 0);
        int rc = BPMF_OK;
        int32_t i = 0;
        for (; i < n; ++i) {
            const int32_t m = movie[i];
            if (m < 0 || m >= c->N) {
                rc = BPMF_E_RANGE;
                break;
            }
            uint64_t &w = seen[(size_t)m >> 6];
            const uint64_t bit = 1ull << (m & 63);
            if (w & bit) {
                rc = BPMF_E_FORMAT;
                break;
            }
            w |= bit;
        }
        for (int32_t j = 0; j < i; ++j) seen[(size_t)movie[j] >> 6] &= ~(1ull << (movie[j] & 63));
        if (rc != BPMF_OK) return rc;
    }
    if (c->relabel)
        for (int32_t &m : r->movie) m = c->int_of[1][m];
    for (int32_t i = 0; i < n; ++i) {
        if (!(rating[i] == rating[i]) || rating[i] > 3.4e38f || rating[i] < -3.4e38f) return BPMF_E_FORMAT;
        r->rc[i] = (float)((double)rating[i] - c->rbar);
    }
    r->top_n = top_n;
    {
        std::lock_guard<std::mutex> g(f->mu);
        if (!f->dev_err.empty()) return BPMF_E_DEVICE;
        if (f->n_pending >= kMaxPending) return BPMF_E_BUSY;
        r->id = f->next_id++;
        r->t_submit = Clock::now();
        f->pending[size_class(r->movie.size())].push_back(r);
        ++f->n_pending;
        f->table.emplace(r->id, r);
        *req_id = r->id;
    }
    f->cv.notify_all();
    return BPMF_OK;
}

int bpmf_foldin_poll(bpmf_ctx *c, uint64_t req_id, int32_t *movie_out, float *mean_out,
                     float *var_out, double *latency_s)
{
    if (!c) return BPMF_E_INVAL;
    FoldinState *f = c->foldin;
    if (!f) return BPMF_E_NOTFOUND;
    std::lock_guard<std::mutex> g(f->mu);
    auto it = f->table.find(req_id);
    if (it == f->table.end()) return BPMF_E_NOTFOUND;
    Request &r = *it->second;
    if (!f->dev_err.empty()) return BPMF_E_DEVICE;
    if (!r.done) return BPMF_PENDING;
    if (movie_out) {
        for (size_t k = 0; k < r.ids.size(); ++k)
            movie_out[k] = (c->relabel && r.ids[k] >= 0) ? c->ext_of[1][r.ids[k]] : r.ids[k];
    }
    if (mean_out) memcpy(mean_out, r.mean.data(), sizeof(float) * r.mean.size());
    if (var_out) memcpy(var_out, r.var.data(), sizeof(float) * r.var.size());
    if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
    f->table.erase(it);
    return BPMF_OK;
}

int bpmf_foldin_drain(bpmf_ctx *c)
{
    if (!c) return BPMF_E_INVAL;
    FoldinState *f = c->foldin;
    if (!f) return BPMF_OK;
    std::unique_lock<std::mutex> lk(f->mu);
    f->cv.wait(lk, [&] { return (f->n_pending == 0 && f->inflight == 0) || !f->dev_err.empty(); });
    return f->dev_err.empty() ? BPMF_OK : BPMF_E_DEVICE;
}

int bpmf_foldin_stats(bpmf_ctx *c, int64_t *batches, int64_t *requests, int32_t *max_batch_requests,
                      int32_t *max_inflight_batches)
{
    if (!c) return BPMF_E_INVAL;
    FoldinState *f = c->foldin;
    std::unique_lock<std::mutex> lk;
    if (f) lk = std::unique_lock<std::mutex>(f->mu);
    if (batches) *batches = f ? f->n_batches : 0;
    if (requests) *requests = f ? f->n_launched : 0;
    if (max_batch_requests) *max_batch_requests = f ? f->max_batch : 0;
    if (max_inflight_batches) *max_inflight_batches = f ? f->max_inflight : 0;
    return BPMF_OK;
}

int bpmf_foldin_samples(const bpmf_ctx *c)
{
    if (!c || !c->foldin) return 0;
    return c->foldin->n_stored;
}

int64_t bpmf_foldin_capacity(const bpmf_ctx *c)
{
    if (!c || !c->foldin) return 0;
    return c->foldin->R_max;
}

}  // extern "C"
