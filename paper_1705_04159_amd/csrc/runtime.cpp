// runtime.cpp -- host side of the C ABI declared in include/bpmf.h:
// validation, the degree plan, device memory, the sweep graph and timing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/bpmf.h"
#include "internal.h"

namespace bpmf {
hipError_t launch_row_generic(bpmf_ctx *c, int side_id, hipStream_t s, int stage);
hipError_t launch_row_fast(bpmf_ctx *c, int side_id, hipStream_t s, int stage, bool *handled);
hipError_t launch_row_big(bpmf_ctx *c, int side_id, hipStream_t s, int stage, bool *handled);
hipError_t prepare_kernels(bpmf_ctx *c);
}  // namespace bpmf

using namespace bpmf;

namespace {

thread_local std::string g_create_err;

constexpr uint32_t kTimedSweeps = 1024;  // replays with their own timing events

int fail(bpmf_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (code == BPMF_E_DEVICE) c->sticky = true;
    } else {
        g_create_err = buf;
    }
    return code;
}

#define HIPCK(c, expr)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((c), e_ == hipErrorOutOfMemory ? BPMF_E_NOMEM : BPMF_E_DEVICE,     \
                        "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

#define STICKY(c)                                                                     \
    do {                                                                              \
        if (!(c)) return BPMF_E_INVAL;                                                \
        if ((c)->sticky) return fail((c), BPMF_E_DEVICE, "context unusable after a device error: %s", (c)->err.c_str()); \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

// Host Cholesky-based inverse of an SPD matrix (row-major), for W0^-1 at
// setup.  Returns false if A is not SPD.
bool spd_inverse_host(int K, const std::vector<double> &A, std::vector<double> &inv)
{
    std::vector<double> L(A);
    for (int j = 0; j < K; ++j) {
        double s = L[j * K + j];
        for (int k = 0; k < j; ++k) s -= L[j * K + k] * L[j * K + k];
        if (!(s > 0)) return false;
        double d = sqrt(s);
        L[j * K + j] = d;
        for (int i = j + 1; i < K; ++i) {
            double v = L[i * K + j];
            for (int k = 0; k < j; ++k) v -= L[i * K + k] * L[j * K + k];
            L[i * K + j] = v / d;
        }
    }
    inv.assign((size_t)K * K, 0.0);
    std::vector<double> col(K);
    for (int j = 0; j < K; ++j) {
        for (int i = 0; i < K; ++i) {
            double v = (i == j) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[i * K + k] * col[k];
            col[i] = v / L[i * K + i];
        }
        for (int i = K - 1; i >= 0; --i) {
            double v = col[i];
            for (int k = i + 1; k < K; ++k) v -= L[k * K + i] * col[k];
            col[i] = v / L[i * K + i];
        }
        for (int i = 0; i < K; ++i) inv[i * K + j] = col[i];
    }
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < i; ++j) {
            double s = 0.5 * (inv[i * K + j] + inv[j * K + i]);
            inv[i * K + j] = inv[j * K + i] = s;
        }
    return true;
}

// Degree plan of one side: rows in degree-descending order (ties by row id);
// rows with more than `split` ratings are cut into segments of at most
// `seg` ratings whose partial sums land in consecutive slots.
void plan_side(const std::vector<int64_t> &ptr, int64_t rows, int64_t split, int64_t seg,
               std::vector<int32_t> &perm, int64_t &n_split, std::vector<RowItem> &items,
               std::vector<FinishItem> &fin, int64_t &n_slots, int64_t low_dmax, int64_t &n_low,
               int64_t &n_low_small)
{
    perm.resize(rows);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
        return (ptr[a + 1] - ptr[a]) > (ptr[b + 1] - ptr[b]);
    });
    n_split = 0;
    while (n_split < rows && ptr[perm[n_split] + 1] - ptr[perm[n_split]] > split) ++n_split;
    items.clear();
    fin.clear();
    n_slots = 0;
    for (int64_t q = 0; q < n_split; ++q) {
        int32_t r = perm[q];
        int64_t beg = ptr[r], end = ptr[r + 1];
        FinishItem f{r, (int32_t)n_slots, 0, 0};
        for (int64_t s = beg; s < end; s += seg) {
            items.push_back(RowItem{r, (int32_t)n_slots, s, std::min(end, s + seg)});
            ++n_slots;
            ++f.count;
        }
        fin.push_back(f);
    }
    n_low = n_low_small = 0;
    for (int64_t q = n_split; q < rows; ++q) {
        int32_t r = perm[q];
        items.push_back(RowItem{r, -1, ptr[r], ptr[r + 1]});
        const int64_t d = ptr[r + 1] - ptr[r];
        if (d <= low_dmax) ++n_low;  // a suffix: degrees descend
        if (d <= std::min<int64_t>(low_dmax, 8)) ++n_low_small;
    }
}

// Whether a side's rows with at most low_dmax ratings take the rank-one path:
// worth it when the factorisations saved (K^3/3 each) outweigh transforming
// the gathered factor (K^2 per row of the other side) several times over.
int64_t low_rows_used(const bpmf_ctx *c, int64_t n_low, int64_t other_rows)
{
    if (c->low_dmax <= 0 || !lowrank_available(c)) return 0;
    const double K = (double)c->K;
    return (double)n_low * K * K * K / 3.0 > 4.0 * (double)other_rows * K * K ? n_low : 0;
}

// Device buffers of the rank-one path for a side that uses it.
hipError_t alloc_lowrank(bpmf_ctx *c, Side &sd, int64_t other_rows)
{
    hipError_t e = hipSuccess;
    if (!sd.Linv_w && (e = hipMalloc(&sd.Linv_w, sizeof(float) * c->K * c->K)) != hipSuccess) return e;
    if (!sd.Ltmu_w && (e = hipMalloc(&sd.Ltmu_w, sizeof(float) * c->K)) != hipSuccess) return e;
    if (!sd.Yt) e = hipMalloc(&sd.Yt, sizeof(float) * std::max<int64_t>(1, other_rows * c->ld));
    return e;
}

size_t elem_bytes(const bpmf_ctx *c) { return c->prec == 0 ? sizeof(double) : sizeof(float); }

// One stage of a side's row update (see UpdateStage), without the rank-one
// rows of the whole-rows stage.
static hipError_t enqueue_stage_kernels(bpmf_ctx *c, int side_id, hipStream_t s, int stage)
{
    bool handled = false;
    hipError_t e = launch_row_fast(c, side_id, s, stage, &handled);
    if (e != hipSuccess) return e;
    if (!handled) e = launch_row_big(c, side_id, s, stage, &handled);
    if (e != hipSuccess) return e;
    if (!handled) e = launch_row_generic(c, side_id, s, stage);
    return e;
}

// One stage of a side's row update (see UpdateStage).
hipError_t enqueue_update_stage(bpmf_ctx *c, int side_id, hipStream_t s, int stage)
{
    if (stage == kStageShadow) return c->prec == 2 ? launch_to_bf16(c, side_id, s) : hipSuccess;
    hipError_t e = enqueue_stage_kernels(c, side_id, s, stage);
    if (e != hipSuccess) return e;
    if (stage == kStageRows && c->side[side_id].n_low) e = launch_row_lowrank(c, side_id, s);
    return e;
}

hipError_t enqueue_update_stages(bpmf_ctx *c, int side_id, hipStream_t s, int first, int last)
{
    for (int st = first; st <= last; ++st)
        if (hipError_t e = enqueue_update_stage(c, side_id, s, st)) return e;
    return hipSuccess;
}

hipError_t enqueue_update(bpmf_ctx *c, int side_id, hipStream_t s)
{
    return enqueue_update_stages(c, side_id, s, kStagePrior, kStageShadow);
}

// Algorithm 1 once, eagerly, with an event after every phase:
// [hyper V][rows V][split V][hyper U][rows U][split U][predict] -> 7 intervals
// (rows: prior, segments and whole rows; split: finishing and BF16 shadow).
hipError_t enqueue_sweep_profiled(bpmf_ctx *c, hipStream_t s, hipEvent_t *ev)
{
    hipError_t e;
    if ((e = launch_advance_t(c->ctr, s)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    int q = 1;
    for (int side : {BPMF_SIDE_V, BPMF_SIDE_U}) {
        if ((e = launch_hyper(c, side, s)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev[q++], s)) != hipSuccess) return e;
        if ((e = enqueue_update_stages(c, side, s, kStagePrior, kStageRows)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev[q++], s)) != hipSuccess) return e;
        if ((e = enqueue_update_stages(c, side, s, kStageFinish, kStageShadow)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev[q++], s)) != hipSuccess) return e;
    }
    if ((e = launch_predict_test(c, s)) != hipSuccess) return e;
    return hipEventRecord(ev[7], s);
}

// One sweep of Algorithm 1 as captured into the graph, for t = ctr[0].  The
// V hyperparameters of sweep t were drawn before (by the prologue of
// bpmf_run_sweeps, or by the previous replay).  Dependencies allow two
// overlaps on a second stream: the U draw of sweep t needs only U of sweep
// t-1, so it runs beside the V update; the V draw of sweep t+1 needs only V
// of sweep t, so it runs beside the U update.  The sweep ends by advancing t.
// Row update of one side inside the captured sweep: the rank-one rows (or,
// without them, the factorisation kernels' whole rows) on a branch of their
// own beside the segments and finishing of the split rows, with external
// event records around the update (all but the BF16 shadow) for timing.
// Whether the whole-rows stage launches anything of its own (the rank-one
// path, or the blocked kernel's whole rows); without it the update stays on
// one branch (a fork and join cost more than they hide).
static bool rows_branch(const bpmf_ctx *c, const Side &sd)
{
    if (sd.n_low > 0) return true;
    const bool fast = fast_path_available(c) && c->K <= c->fast_kmax;
    return !fast && big_path_available(c) && sd.n_items - sd.n_slots - sd.n_low > 0;
}

hipError_t enqueue_update_timed(bpmf_ctx *c, int side_id, hipStream_t s, hipEvent_t a, hipEvent_t b)
{
    hipError_t e;
    hipStream_t s3 = c->stream3;
    if ((e = hipEventRecordWithFlags(a, s, hipEventRecordExternal)) != hipSuccess) return e;
    if (!rows_branch(c, c->side[side_id])) {
        if ((e = enqueue_update_stages(c, side_id, s, kStagePrior, kStageFinish)) != hipSuccess) return e;
        if ((e = hipEventRecordWithFlags(b, s, hipEventRecordExternal)) != hipSuccess) return e;
        return enqueue_update_stage(c, side_id, s, kStageShadow);
    }
    if ((e = enqueue_update_stage(c, side_id, s, kStagePrior)) != hipSuccess) return e;
    if ((e = hipEventRecord(c->stage_ev[0], s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s3, c->stage_ev[0], 0)) != hipSuccess) return e;
    // With rank-one rows the branch takes only those (the longest part), and
    // the factorisation kernels' whole rows follow the segments; otherwise
    // the branch takes the whole rows.
    const bool low = c->side[side_id].n_low > 0;
    if (low) {
        if ((e = launch_row_lowrank(c, side_id, s3)) != hipSuccess) return e;
    } else if ((e = enqueue_stage_kernels(c, side_id, s3, kStageRows)) != hipSuccess) {
        return e;
    }
    if ((e = hipEventRecord(c->stage_ev[1], s3)) != hipSuccess) return e;
    if ((e = enqueue_update_stages(c, side_id, s, kStageSegments, kStageSegments)) != hipSuccess) return e;
    if (low && (e = enqueue_stage_kernels(c, side_id, s, kStageRows)) != hipSuccess) return e;
    if ((e = enqueue_update_stage(c, side_id, s, kStageFinish)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, c->stage_ev[1], 0)) != hipSuccess) return e;
    if ((e = hipEventRecordWithFlags(b, s, hipEventRecordExternal)) != hipSuccess) return e;
    return enqueue_update_stage(c, side_id, s, kStageShadow);
}

hipError_t enqueue_sweep(bpmf_ctx *c, hipStream_t s)
{
    hipError_t e;
    hipStream_t s2 = c->stream2;
    if ((e = hipEventRecord(c->fork_ev[0], s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s2, c->fork_ev[0], 0)) != hipSuccess) return e;
    if ((e = launch_hyper(c, BPMF_SIDE_U, s2, 0)) != hipSuccess) return e;
    if ((e = hipEventRecord(c->fork_ev[1], s2)) != hipSuccess) return e;
    if ((e = enqueue_update_timed(c, BPMF_SIDE_V, s, c->tev[0], c->tev[1])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, c->fork_ev[1], 0)) != hipSuccess) return e;
    if ((e = hipEventRecord(c->fork_ev[2], s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s2, c->fork_ev[2], 0)) != hipSuccess) return e;
    if ((e = launch_hyper(c, BPMF_SIDE_V, s2, 1)) != hipSuccess) return e;
    if ((e = hipEventRecord(c->fork_ev[1], s2)) != hipSuccess) return e;
    if ((e = enqueue_update_timed(c, BPMF_SIDE_U, s, c->tev[2], c->tev[3])) != hipSuccess) return e;
    if ((e = launch_predict_test(c, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, c->fork_ev[1], 0)) != hipSuccess) return e;
    return launch_advance_t(c->ctr, s);
}

void free_side(Side &s)
{
    void *ps[] = {s.ptr, s.nbr, s.rc, s.X, s.Xbf, s.rc3, s.mu, s.Lam, s.Lam_w, s.Lmu_w, s.Lam_img, s.Lam_pk,
                  s.items, s.fin, s.Linv_w, s.Ltmu_w, s.Yt};
    for (void *p : ps) (void)hipFree(p);
}

}  // namespace

extern "C" {

void bpmf_default_params(bpmf_params *p, int32_t K)
{
    memset(p, 0, sizeof(*p));
    p->K = K;
    p->prec = BPMF_FP32;
    p->alpha = 2.0;
    p->beta0 = 2.0;
    p->nu0 = (double)K;
    p->mu0 = nullptr;
    p->W0 = nullptr;
    p->seed = 0;
    p->center = 1;
    p->burn_in = 0;
    p->foldin_S = 16;
    p->split_threshold = 0;
    p->foldin_pool_bytes = 0;
    p->stream = nullptr;
    p->reorder = 0;
}

const char *bpmf_last_error(const bpmf_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

}  // extern "C"

namespace {

// The reordering of R before partitioning (Sec. IV-B), used here for
// locality: users and movies are relabelled in descending order of their
// rating counts (ties by the caller's id), so the most-gathered rows of each
// factor sit together at the front of its array.  The relabelled matrix is
// built from the transposition (columns visited in their new order, so each
// new row's columns come out ascending) and handed to the ordinary create;
// the maps between the two labellings stay with the context, and every call
// that takes or returns user or movie ids translates them.  A relabelled
// context on R computes exactly what an ordinary one computes on the
// relabelled R.
int create_relabelled(int64_t M, int64_t N, const int64_t *csr_ptr, const std::vector<int64_t> &tptr,
                      const std::vector<int32_t> &trow, const std::vector<float> &tval, int64_t nnz,
                      const int32_t *test_row, const int32_t *test_col, const float *test_val,
                      int64_t n_test, const bpmf_params *p, bpmf_ctx **out)
{
    auto degree_order = [](int64_t rows, const int64_t *ptr, std::vector<int32_t> &ext,
                           std::vector<int32_t> &inv) {
        ext.resize(rows);
        inv.resize(rows);
        std::iota(ext.begin(), ext.end(), 0);
        std::stable_sort(ext.begin(), ext.end(), [ptr](int32_t a, int32_t b) {
            return ptr[a + 1] - ptr[a] > ptr[b + 1] - ptr[b];
        });
        for (int64_t r = 0; r < rows; ++r) inv[ext[r]] = (int32_t)r;
    };
    std::vector<int32_t> ext[2], inv[2];
    degree_order(M, csr_ptr, ext[0], inv[0]);
    degree_order(N, tptr.data(), ext[1], inv[1]);
    std::vector<int64_t> nptr(M + 1, 0);
    for (int64_t r = 0; r < M; ++r) nptr[r + 1] = nptr[r] + (csr_ptr[ext[0][r] + 1] - csr_ptr[ext[0][r]]);
    std::vector<int32_t> ncol(nnz);
    std::vector<float> nval(nnz);
    {
        std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
        for (int64_t jn = 0; jn < N; ++jn) {
            const int32_t j = ext[1][jn];
            for (int64_t e = tptr[j]; e < tptr[j + 1]; ++e) {
                const int64_t q = fill[inv[0][trow[e]]]++;
                ncol[q] = (int32_t)jn;
                nval[q] = tval[e];
            }
        }
    }
    std::vector<int32_t> ntr(n_test), ntc(n_test);
    for (int64_t e = 0; e < n_test; ++e) {
        ntr[e] = inv[0][test_row[e]];
        ntc[e] = inv[1][test_col[e]];
    }
    bpmf_params q = *p;
    q.reorder = 0;
    bpmf_ctx *c = nullptr;
    int rc = bpmf_create(M, N, nptr.data(), ncol.data(), nval.data(), nullptr, nullptr, nullptr, nnz,
                         ntr.data(), ntc.data(), test_val, n_test, &q, &c);
    if (rc != BPMF_OK) return rc;
    c->relabel = true;
    for (int sid = 0; sid < 2; ++sid) {
        const int64_t rows = sid == 0 ? M : N;
        hipError_t e = dalloc(&c->d_int_of[sid], rows);
        if (e == hipSuccess)
            e = hipMemcpy(c->d_int_of[sid], inv[sid].data(), sizeof(int32_t) * rows, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            bpmf_destroy(c);
            return fail(nullptr, e == hipErrorOutOfMemory ? BPMF_E_NOMEM : BPMF_E_DEVICE,
                        "relabelling maps: %s", hipGetErrorString(e));
        }
        c->ext_of[sid] = std::move(ext[sid]);
        c->int_of[sid] = std::move(inv[sid]);
    }
    *out = c;
    return BPMF_OK;
}

}  // namespace

extern "C" {

int bpmf_create(int64_t M, int64_t N, const int64_t *csr_ptr, const int32_t *csr_col,
                const float *csr_val, const int64_t *csc_ptr, const int32_t *csc_row,
                const float *csc_val, int64_t nnz, const int32_t *test_row,
                const int32_t *test_col, const float *test_val, int64_t n_test,
                const bpmf_params *p, bpmf_ctx **out)
{
    if (!out || !p) return fail(nullptr, BPMF_E_INVAL, "null output or params");
    *out = nullptr;
    const int K = p->K;
    if (K < 1 || K > 128) return fail(nullptr, BPMF_E_INVAL, "K=%d outside 1..128", K);
    if (p->prec < 0 || p->prec > 2) return fail(nullptr, BPMF_E_INVAL, "bad precision %d", p->prec);
    if (p->prec == BPMF_FP64 && K > 64) return fail(nullptr, BPMF_E_INVAL, "FP64 mode supports K <= 64");
    if (p->foldin_S < 0 || p->foldin_S > 64) return fail(nullptr, BPMF_E_INVAL, "foldin_S outside 0..64");
    if (p->split_threshold < 0 || p->split_threshold > (1 << 24))
        return fail(nullptr, BPMF_E_INVAL, "split_threshold outside 0..2^24");
    if (!(p->alpha > 0) || !(p->beta0 > 0) || !(p->nu0 > K - 1))
        return fail(nullptr, BPMF_E_INVAL, "need alpha > 0, beta0 > 0, nu0 > K - 1");
    if (M < 1 || N < 1 || M > INT32_MAX || N > INT32_MAX || nnz < 0)
        return fail(nullptr, BPMF_E_INVAL, "bad sizes M=%lld N=%lld nnz=%lld", (long long)M,
                    (long long)N, (long long)nnz);
    if (!csr_ptr || (nnz > 0 && (!csr_col || !csr_val)))
        return fail(nullptr, BPMF_E_INVAL, "missing CSR arrays");
    if (n_test < 0 || (n_test > 0 && (!test_row || !test_col || !test_val)))
        return fail(nullptr, BPMF_E_INVAL, "missing test arrays");
    // ---- validate CSR ----
    if (csr_ptr[0] != 0 || csr_ptr[M] != nnz)
        return fail(nullptr, BPMF_E_FORMAT, "csr_ptr must start at 0 and end at nnz");
    for (int64_t i = 0; i < M; ++i) {
        if (csr_ptr[i + 1] < csr_ptr[i])
            return fail(nullptr, BPMF_E_FORMAT, "csr_ptr decreases at row %lld", (long long)i);
        for (int64_t e = csr_ptr[i]; e < csr_ptr[i + 1]; ++e) {
            if (csr_col[e] < 0 || csr_col[e] >= N)
                return fail(nullptr, BPMF_E_RANGE, "column %d out of range at %lld", csr_col[e],
                            (long long)e);
            if (e > csr_ptr[i] && csr_col[e] <= csr_col[e - 1])
                return fail(nullptr, BPMF_E_FORMAT,
                            "columns not strictly increasing in row %lld", (long long)i);
            if (!isfinite(csr_val[e]))
                return fail(nullptr, BPMF_E_FORMAT, "non-finite rating at %lld", (long long)e);
        }
    }
    for (int64_t e = 0; e < n_test; ++e) {
        if (test_row[e] < 0 || test_row[e] >= M || test_col[e] < 0 || test_col[e] >= N)
            return fail(nullptr, BPMF_E_RANGE, "test pair %lld out of range", (long long)e);
        if (!isfinite(test_val[e])) return fail(nullptr, BPMF_E_FORMAT, "non-finite test value");
    }
    // ---- transpose (counting sort, rows ascending within a column) ----
    std::vector<int64_t> tptr(N + 1, 0);
    std::vector<int32_t> trow(nnz);
    std::vector<float> tval(nnz);
    for (int64_t e = 0; e < nnz; ++e) tptr[csr_col[e] + 1]++;
    for (int64_t j = 0; j < N; ++j) tptr[j + 1] += tptr[j];
    {
        std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
        for (int64_t i = 0; i < M; ++i)
            for (int64_t e = csr_ptr[i]; e < csr_ptr[i + 1]; ++e) {
                int64_t q = fill[csr_col[e]]++;
                trow[q] = (int32_t)i;
                tval[q] = csr_val[e];
            }
    }
    if (csc_ptr || csc_row || csc_val) {
        if (!csc_ptr || (nnz > 0 && (!csc_row || !csc_val)))
            return fail(nullptr, BPMF_E_INVAL, "incomplete CSC arrays");
        if (memcmp(csc_ptr, tptr.data(), sizeof(int64_t) * (N + 1)) ||
            (nnz && memcmp(csc_row, trow.data(), sizeof(int32_t) * nnz)) ||
            (nnz && memcmp(csc_val, tval.data(), sizeof(float) * nnz)))
            return fail(nullptr, BPMF_E_FORMAT, "CSC is not the exact transpose of the CSR");
    }
    std::vector<double> mu0(K, 0.0), W0((size_t)K * K, 0.0), W0inv;
    if (p->mu0)
        for (int k = 0; k < K; ++k) mu0[k] = p->mu0[k];
    for (int k = 0; k < K; ++k) W0[(size_t)k * K + k] = 1.0;
    if (p->W0)
        for (size_t q = 0; q < (size_t)K * K; ++q) W0[q] = p->W0[q];
    if (!spd_inverse_host(K, W0, W0inv)) return fail(nullptr, BPMF_E_INVAL, "W0 is not SPD");
    if (p->reorder < 0 || p->reorder > 1) return fail(nullptr, BPMF_E_INVAL, "reorder must be 0 or 1");
    if (p->reorder) return create_relabelled(M, N, csr_ptr, tptr, trow, tval, nnz, test_row, test_col,
                                             test_val, n_test, p, out);

    bpmf_ctx *c = new bpmf_ctx();
    c->M = M;
    c->N = N;
    c->nnz = nnz;
    c->n_test = n_test;
    c->K = K;
    c->prec = p->prec;
    c->ld = p->prec == BPMF_FP64 ? K : ((K + 3) / 4) * 4;
    c->alpha = p->alpha;
    c->beta0 = p->beta0;
    c->nu0 = p->nu0;
    c->seed = p->seed;
    c->burn_in = p->burn_in;
    c->side[0].rows = M;
    c->side[1].rows = N;
    // default: rows above 2048 ratings are split (above 8192 for K > 64, where
    // a segment's partial sums are large and its Gram long enough to keep
    // the waves busy)
    c->split_threshold = p->split_threshold > 0 ? p->split_threshold : (K > 64 ? 8192 : 2048);
    // rank-one path for rows with at most 8 ratings where it pays (FP32, K <= 64)
    c->low_dmax = lowrank_available(c) ? 8 : 0;
    c->foldin_S = p->foldin_S > 0 ? p->foldin_S : 16;
    c->foldin_pool = p->foldin_pool_bytes;
    double rbar = 0.0;
    if (p->center) {
        double s = 0.0;
        for (int64_t e = 0; e < nnz; ++e) s += (double)csr_val[e];
        rbar = nnz ? s / (double)nnz : 0.0;
    }
    c->rbar = rbar;
    int rc = BPMF_OK;
#define CK(expr)                         \
    do {                                 \
        hipError_t e_ = (expr);          \
        if (e_ != hipSuccess) {          \
            rc = fail(nullptr, e_ == hipErrorOutOfMemory ? BPMF_E_NOMEM : BPMF_E_DEVICE, \
                      "%s: %s", #expr, hipGetErrorString(e_)); \
            goto error;                  \
        }                                \
    } while (0)
    {
        CK(hipGetDevice(&c->device));
        if (p->stream) {
            c->stream = (hipStream_t)p->stream;
            c->own_stream = false;
        } else {
            CK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        }
        CK(hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
        CK(hipStreamCreateWithFlags(&c->stream3, hipStreamNonBlocking));
        for (auto &ev : c->fork_ev) CK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        for (auto &ev : c->stage_ev) CK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        CK(hipEventCreate(&c->ev0));
        CK(hipEventCreate(&c->ev1));
        for (auto &ev : c->tev) CK(hipEventCreate(&ev));
        const size_t es = elem_bytes(c);
        std::vector<int64_t> csr_ptr_v(csr_ptr, csr_ptr + M + 1);
        const std::vector<int64_t> *ptrs[2] = {&csr_ptr_v, &tptr};
        const int32_t *nbrs[2] = {csr_col, trow.data()};
        const float *vals[2] = {csr_val, tval.data()};
        for (int sid = 0; sid < 2; ++sid) {
            Side &sd = c->side[sid];
            sd.rows = sid == 0 ? M : N;
            sd.stream_row = sid == 0 ? 1u : 2u;
            sd.stream_hyp = sid == 0 ? 3u : 4u;
            sd.stream_init = sid == 0 ? 5u : 6u;
            CK(dalloc(&sd.ptr, sd.rows + 1));
            CK(dalloc(&sd.nbr, nnz));
            CK(hipMalloc(&sd.rc, std::max<size_t>(1, nnz) * es));
            CK(hipMalloc(&sd.X, std::max<size_t>(1, (size_t)sd.rows * c->ld) * es));
            if (c->prec == BPMF_BF16_GRAM) CK(dalloc(&sd.Xbf, (size_t)sd.rows * c->ld));
            // rating parts for the matrix-core rhs of the blocked kernel and of
            // the FP32 K <= 32 kernel's three-part Gram (read at byte offsets
            // below 2^30 across all three planes; beyond that the blocked
            // kernel sums the rhs on the vector units and the K <= 32 one
            // keeps its FP32 Gram)
            if ((c->prec == BPMF_BF16_GRAM || parts_gram_wanted(c)) && 6 * ((uint64_t)nnz + 32) < (1ull << 30))
                CK(dalloc(&sd.rc3, 3 * ((size_t)nnz + 32)));
            CK(dalloc(&sd.mu, K));
            CK(dalloc(&sd.Lam, (size_t)K * K));
            CK(hipMalloc(&sd.Lam_w, (size_t)K * K * es));
            CK(hipMalloc(&sd.Lmu_w, (size_t)K * es));
            if (K <= 128) {
                const size_t nb = (K + 15) / 16;
                CK(hipMalloc(&sd.Lam_img, sizeof(float) * nb * (nb + 1) / 2 * 256));
                const size_t kp = 16 * nb;
                if (K <= 64) CK(hipMalloc(&sd.Lam_pk, sizeof(float) * kp * (kp + 1) / 2));
            }
            CK(hipMemcpy(sd.ptr, ptrs[sid]->data(), sizeof(int64_t) * (sd.rows + 1),
                         hipMemcpyHostToDevice));
            if (nnz) CK(hipMemcpy(sd.nbr, nbrs[sid], sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
            if (nnz) {
                if (c->prec == BPMF_FP64) {
                    std::vector<double> r(nnz);
                    for (int64_t e = 0; e < nnz; ++e) r[e] = (double)vals[sid][e] - rbar;
                    CK(hipMemcpy(sd.rc, r.data(), sizeof(double) * nnz, hipMemcpyHostToDevice));
                } else {
                    std::vector<float> r(nnz);
                    for (int64_t e = 0; e < nnz; ++e) r[e] = (float)((double)vals[sid][e] - rbar);
                    CK(hipMemcpy(sd.rc, r.data(), sizeof(float) * nnz, hipMemcpyHostToDevice));
                }
            }
            sd.hptr = *ptrs[sid];
            std::vector<RowItem> items;
            std::vector<FinishItem> fin;
            int64_t n_low = 0, n_low_small = 0;
            plan_side(*ptrs[sid], sd.rows, c->split_threshold,
                      std::max<int64_t>(128, c->split_threshold / 2), sd.perm, sd.n_split, items,
                      fin, sd.n_slots, c->low_dmax, n_low, n_low_small);
            sd.n_low = low_rows_used(c, n_low, sid == 0 ? N : M);
            sd.n_low_small = sd.n_low ? n_low_small : 0;
            if (sd.n_low) CK(alloc_lowrank(c, sd, sid == 0 ? N : M));
            sd.n_items = (int64_t)items.size();
            sd.n_fin = (int64_t)fin.size();
            CK(dalloc(&sd.items, items.size()));
            CK(dalloc(&sd.fin, fin.size()));
            if (!items.empty())
                CK(hipMemcpy(sd.items, items.data(), sizeof(RowItem) * items.size(),
                             hipMemcpyHostToDevice));
            if (!fin.empty())
                CK(hipMemcpy(sd.fin, fin.data(), sizeof(FinishItem) * fin.size(),
                             hipMemcpyHostToDevice));
            // prior mean as the initial hyperparameters: mu0, nu0 W0
            std::vector<double> lam0((size_t)K * K);
            for (size_t q = 0; q < lam0.size(); ++q) lam0[q] = p->nu0 * W0[q];
            CK(hipMemcpy(sd.mu, mu0.data(), sizeof(double) * K, hipMemcpyHostToDevice));
            CK(hipMemcpy(sd.Lam, lam0.data(), sizeof(double) * K * K, hipMemcpyHostToDevice));
        }
        const int KK2 = K * (K + 1) / 2;
        c->part_slots = std::max(c->side[0].n_slots, c->side[1].n_slots);
        CK(hipMalloc(&c->part, std::max<size_t>(1, (size_t)c->part_slots *
                                                      std::max<int64_t>(KK2 + K, part_slot_elems(c))) * es));
        CK(dalloc(&c->d_mu0, K));
        CK(dalloc(&c->d_W0inv, (size_t)K * K));
        CK(hipMemcpy(c->d_mu0, mu0.data(), sizeof(double) * K, hipMemcpyHostToDevice));
        CK(hipMemcpy(c->d_W0inv, W0inv.data(), sizeof(double) * K * K, hipMemcpyHostToDevice));
        c->hyp_blocks = K <= 64 ? 2048 : 1024;  // row blocks of the moment sums (one wave each on the matrix-core path)
        for (int sid = 0; sid < 2; ++sid) {
            CK(dalloc(&c->hyp_part[sid], (size_t)c->hyp_blocks * (K + KK2)));
            CK(dalloc(&c->hyp_red[sid], (size_t)16 * (K + KK2)));
            CK(dalloc(&c->hyp_stats[sid], (size_t)(K + KK2)));
            CK(dalloc(&c->hyp_scratch[sid], (size_t)4 * K * K + 8 * K));
        }
        CK(dalloc(&c->hyp_status, 2));
        {
            const int ones[2] = {1, 1};
            CK(hipMemcpy(c->hyp_status, ones, sizeof(ones), hipMemcpyHostToDevice));
        }
        // test set
        CK(dalloc(&c->test_row, n_test));
        CK(dalloc(&c->test_col, n_test));
        CK(dalloc(&c->test_val, n_test));
        CK(dalloc(&c->pred_sum, n_test));
        if (n_test) {
            // held in user order (stable counting sort): the pairs of one user
            // are neighbours, so the prediction kernel reads each user's row
            // once per wave instead of once per pair; only the order of the
            // FP64 error sums depends on it
            std::vector<int64_t> start(M + 1, 0);
            for (int64_t e = 0; e < n_test; ++e) ++start[test_row[e] + 1];
            for (int64_t i = 0; i < M; ++i) start[i + 1] += start[i];
            std::vector<int32_t> tr(n_test), tc(n_test);
            std::vector<float> tv(n_test);
            c->test_src.resize(n_test);
            for (int64_t e = 0; e < n_test; ++e) {
                const int64_t q = start[test_row[e]]++;
                c->test_src[q] = e;
                tr[q] = test_row[e];
                tc[q] = test_col[e];
                tv[q] = test_val[e];
            }
            CK(hipMemcpy(c->test_row, tr.data(), sizeof(int32_t) * n_test, hipMemcpyHostToDevice));
            CK(hipMemcpy(c->test_col, tc.data(), sizeof(int32_t) * n_test, hipMemcpyHostToDevice));
            CK(hipMemcpy(c->test_val, tv.data(), sizeof(float) * n_test, hipMemcpyHostToDevice));
        }
        c->rmse_blocks = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (n_test + 127) / 128));
        CK(dalloc(&c->rmse_part, 2 * (size_t)c->rmse_blocks));
        c->hist_cap = 64;
        CK(dalloc(&c->rmse_hist, 2 * (size_t)c->hist_cap));
        CK(dalloc(&c->ctr, 4));
        CK(hipMemsetAsync(c->ctr, 0, 4 * sizeof(uint32_t), c->stream));
        CK(launch_fill_f64(c->pred_sum, n_test, 0.0, c->stream));
        CK(prepare_kernels(c));
        CK(predict_scratch_init(c));
        for (int sid = 0; sid < 2; ++sid) {
            CK(launch_init_factor(c, sid, c->stream));
            CK(launch_prior_to_working(c, sid, c->stream));
            if (c->prec == BPMF_BF16_GRAM) CK(launch_to_bf16(c, sid, c->stream));
            CK(launch_split_ratings(c, sid, c->stream));  // if the side has rating parts
        }
        CK(hipStreamSynchronize(c->stream));
    }
#undef CK
    *out = c;
    return BPMF_OK;
error:
    bpmf_destroy(c);
    return rc;
}

void bpmf_destroy(bpmf_ctx *c)
{
    if (!c) return;
    foldin_destroy(c);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_src) (void)hipGraphDestroy(c->graph_src);
    for (auto &ev : c->tev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &ev : c->tpool) (void)hipEventDestroy(ev);
    for (auto &s : c->side) free_side(s);
    void *ps[] = {c->d_mu0, c->d_W0inv, c->test_row, c->test_col, c->test_val, c->pred_sum,
                  c->rmse_part, c->rmse_hist, c->hyp_part[0], c->hyp_red[0], c->hyp_stats[0], c->hyp_scratch[0],
                  c->hyp_part[1], c->hyp_red[1], c->hyp_stats[1], c->hyp_scratch[1],
                  c->hyp_status, c->part, c->ctr, c->q_row, c->q_col, c->q_out,
                  c->d_int_of[0], c->d_int_of[1]};
    for (void *p : ps) (void)hipFree(p);
    for (auto &ev : c->fork_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &ev : c->stage_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->stream2) (void)hipStreamDestroy(c->stream2);
    if (c->stream3) (void)hipStreamDestroy(c->stream3);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->stream && c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

static int check_side(bpmf_ctx *c, int32_t side)
{
    if (side != BPMF_SIDE_U && side != BPMF_SIDE_V) return fail(c, BPMF_E_INVAL, "bad side %d", side);
    return BPMF_OK;
}

static int timed_end(bpmf_ctx *c)
{
    HIPCK(c, hipEventRecord(c->ev1, c->stream));
    HIPCK(c, hipEventSynchronize(c->ev1));
    float ms = 0;
    HIPCK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms = ms;
    return BPMF_OK;
}

// The device flags the kernels clear on a non-positive pivot (hyper draw,
// row draws); read and re-armed after every call that launches them.
static int check_status(bpmf_ctx *c)
{
    int st[2] = {1, 1};
    HIPCK(c, hipMemcpy(st, c->hyp_status, sizeof(st), hipMemcpyDeviceToHost));
    if (!st[0] || !st[1]) {
        const int ones[2] = {1, 1};
        HIPCK(c, hipMemcpy(c->hyp_status, ones, sizeof(ones), hipMemcpyHostToDevice));
        return fail(c, BPMF_E_NOTSPD, "%s",
                    !st[0] ? "hyperparameter draw hit a matrix that is not positive definite"
                           : "a row's precision matrix was not positive definite in working precision");
    }
    return BPMF_OK;
}

int bpmf_sample_hyper(bpmf_ctx *c, int32_t side, uint32_t t)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    HIPCK(c, hipEventRecord(c->ev0, c->stream));
    HIPCK(c, launch_set_counter(c->ctr, 0, t, c->stream));
    HIPCK(c, launch_hyper(c, side, c->stream));
    if (int r = timed_end(c)) return r;
    return check_status(c);
}

int bpmf_update_side(bpmf_ctx *c, int32_t side, uint32_t t)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    HIPCK(c, hipEventRecord(c->ev0, c->stream));
    HIPCK(c, launch_set_counter(c->ctr, 0, t, c->stream));
    HIPCK(c, enqueue_update(c, side, c->stream));
    if (int r = timed_end(c)) return r;
    return check_status(c);
}

// The external event-record nodes of the captured sweep (V start, V end,
// U start, U end), so that each replay can be pointed at its own events.
static int find_timing_nodes(bpmf_ctx *c)
{
    size_t nn = 0;
    HIPCK(c, hipGraphGetNodes(c->graph_src, nullptr, &nn));
    std::vector<hipGraphNode_t> nodes(nn);
    HIPCK(c, hipGraphGetNodes(c->graph_src, nodes.data(), &nn));
    for (auto &t : c->tnode) t = nullptr;
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        HIPCK(c, hipGraphNodeGetType(nd, &ty));
        if (ty != hipGraphNodeTypeEventRecord) continue;
        hipEvent_t ev = nullptr;
        HIPCK(c, hipGraphEventRecordNodeGetEvent(nd, &ev));
        for (int k = 0; k < 4; ++k)
            if (ev == c->tev[k]) c->tnode[k] = nd;
    }
    c->timing_nodes = true;
    for (auto t : c->tnode)
        if (!t) c->timing_nodes = false;  // sweeps still run, untimed
    return BPMF_OK;
}

// Re-plan both sides for a new split threshold / kernel family: work items,
// finishing items and the partial-sum workspace; the sweep graph is rebuilt
// on the next bpmf_run_sweeps.
static int ensure_graph(bpmf_ctx *c);

static int replan(bpmf_ctx *c, int split, int fast_kmax, int low_dmax, bool force_low = false)
{
    HIPCK(c, hipStreamSynchronize(c->stream));
    c->split_threshold = split;
    c->fast_kmax = fast_kmax;
    c->low_dmax = low_dmax;
    for (int sid = 0; sid < 2; ++sid) {
        Side &sd = c->side[sid];
        std::vector<RowItem> items;
        std::vector<FinishItem> fin;
        int64_t n_low = 0, n_low_small = 0;
        plan_side(sd.hptr, sd.rows, split, std::max<int64_t>(128, split / 2), sd.perm, sd.n_split,
                  items, fin, sd.n_slots, low_dmax, n_low, n_low_small);
        const int64_t other = c->side[1 - sid].rows;
        sd.n_low = force_low && lowrank_available(c) ? n_low : low_rows_used(c, n_low, other);
        sd.n_low_small = sd.n_low ? n_low_small : 0;
        if (sd.n_low) HIPCK(c, alloc_lowrank(c, sd, other));
        (void)hipFree(sd.items);
        (void)hipFree(sd.fin);
        sd.items = nullptr;
        sd.fin = nullptr;
        sd.n_items = (int64_t)items.size();
        sd.n_fin = (int64_t)fin.size();
        HIPCK(c, dalloc(&sd.items, items.size()));
        HIPCK(c, dalloc(&sd.fin, fin.size()));
        if (!items.empty())
            HIPCK(c, hipMemcpy(sd.items, items.data(), sizeof(RowItem) * items.size(), hipMemcpyHostToDevice));
        if (!fin.empty())
            HIPCK(c, hipMemcpy(sd.fin, fin.data(), sizeof(FinishItem) * fin.size(), hipMemcpyHostToDevice));
    }
    const int64_t KK2 = (int64_t)c->K * (c->K + 1) / 2;
    c->part_slots = std::max(c->side[0].n_slots, c->side[1].n_slots);
    (void)hipFree(c->part);
    c->part = nullptr;
    HIPCK(c, hipMalloc(&c->part, std::max<size_t>(1, (size_t)c->part_slots *
                                                        std::max<int64_t>(KK2 + c->K, part_slot_elems(c))) *
                                    elem_bytes(c)));
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_src) (void)hipGraphDestroy(c->graph_src);
    c->graph = nullptr;
    c->graph_src = nullptr;
    return BPMF_OK;
}

// Device copies of everything a sweep changes (factors, BF16 shadows,
// hyperparameters, running prediction sums, counters).
struct ChainSnapshot {
    std::vector<std::pair<void *, size_t>> regions;  // (live buffer, bytes)
    std::vector<void *> copies;
};

static int snapshot_take(bpmf_ctx *c, ChainSnapshot &sn)
{
    const size_t es = elem_bytes(c);
    const size_t K = (size_t)c->K;
    for (auto &sd : c->side) {
        sn.regions.push_back({sd.X, (size_t)sd.rows * c->ld * es});
        if (sd.Xbf) sn.regions.push_back({sd.Xbf, (size_t)sd.rows * c->ld * sizeof(uint16_t)});
        sn.regions.push_back({sd.mu, K * sizeof(double)});
        sn.regions.push_back({sd.Lam, K * K * sizeof(double)});
        sn.regions.push_back({sd.Lam_w, K * K * es});
        sn.regions.push_back({sd.Lmu_w, K * es});
    }
    sn.regions.push_back({c->pred_sum, (size_t)c->n_test * sizeof(double)});
    sn.regions.push_back({c->ctr, 4 * sizeof(uint32_t)});
    for (auto &rg : sn.regions) {
        void *p = nullptr;
        if (rg.second) HIPCK(c, hipMalloc(&p, rg.second));
        sn.copies.push_back(p);
        if (rg.second)
            HIPCK(c, hipMemcpyAsync(p, rg.first, rg.second, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCK(c, hipStreamSynchronize(c->stream));
    return BPMF_OK;
}

static int snapshot_restore(bpmf_ctx *c, const ChainSnapshot &sn)
{
    for (size_t q = 0; q < sn.regions.size(); ++q)
        if (sn.regions[q].second)
            HIPCK(c, hipMemcpyAsync(sn.regions[q].first, sn.copies[q], sn.regions[q].second,
                                    hipMemcpyDeviceToDevice, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    return BPMF_OK;
}

static void snapshot_free(ChainSnapshot &sn)
{
    for (void *p : sn.copies) (void)hipFree(p);
    sn.copies.clear();
}

int bpmf_run_sweeps(bpmf_ctx *c, uint32_t t0, uint32_t n, double *rmse_avg, double *rmse_last);

// Rank-one path inputs from the current (mu, Lambda) of each side using it.
static int refresh_lowrank(bpmf_ctx *c)
{
    for (int sid = 0; sid < 2; ++sid)
        if (c->side[sid].n_low) HIPCK(c, launch_prior_to_working(c, sid, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    return BPMF_OK;
}

// Split threshold from the workload model of Sec. IV-B (measured as Fig. 2
// on gfx950: a row costs a fixed amount plus an amount per rating, the
// fixed part worth about 3K ratings in the factorising kernels at K = 32 and
// K = 100).  With W = sum over a side's rows of (r + d_i), r = 3K, and P rows
// in flight on the GPU, a row of degree d alone on its wave takes the share
// (r + d) P / W of the side's stage; it does not prolong the stage while
// that share is at most one half, so d* = W / (2P) - r.  The smaller d* of the
// two sides (the threshold is shared).
static double model_split(const bpmf_ctx *c)
{
    const int K = c->K;
    const double r = 3.0 * K;
    double P;  // rows in flight: SIMDs x waves per SIMD x rows per wave of the kernel family
    if (c->prec == BPMF_FP64) P = 512.0;  // one 256-thread workgroup per row
    else if (K <= 16) P = 1024.0 * 8 * 4;
    else if (K <= 32) P = 1024.0 * 7 * 2;
    else if (K <= 48) P = 1024.0 * 4;
    else if (K <= 64) P = 1024.0 * 3;
    else P = 1024.0 * 2;
    double dstar = 1e300;
    for (auto &sd : c->side) {
        double W = 0.0;
        for (int64_t i = 0; i < sd.rows; ++i) W += r + (double)(sd.hptr[i + 1] - sd.hptr[i]);
        dstar = std::min(dstar, W / (2.0 * P) - r);
    }
    return std::max(1.0, dstar);
}

int bpmf_autotune(bpmf_ctx *c, uint32_t n_sweeps, int32_t *chosen_split, int32_t *chosen_kmax,
                  int32_t *chosen_low, int32_t *n_tried, int32_t *tried_split, int32_t *tried_kmax,
                  int32_t *tried_low, double *tried_ms)
{
    STICKY(c);
    if (n_sweeps == 0 || n_sweeps > 64) return fail(c, BPMF_E_INVAL, "n_sweeps must be 1..64");
    // candidate cut-offs: the powers of two from 512 up to the first at or
    // above the largest degree (no split) that lie within a factor of four
    // of the workload model's threshold (the one nearest it if none does),
    // plus the current one; and the kernel families for FP32 K in (32, 64]
    int64_t max_deg = 0;
    for (auto &sd : c->side)
        for (int64_t r = 0; r < sd.rows; ++r) max_deg = std::max(max_deg, sd.hptr[r + 1] - sd.hptr[r]);
    const double dstar = model_split(c);
    std::vector<int> all, splits;
    for (int64_t s = 512; s <= (1 << 24); s *= 2) {
        all.push_back((int)s);
        if (s >= max_deg) break;
    }
    for (int s : all)
        if (s >= dstar / 4 && s <= dstar * 4) splits.push_back(s);
    if (splits.empty()) {
        int near = all.front();
        for (int s : all)
            if (std::fabs(std::log((double)s / dstar)) < std::fabs(std::log((double)near / dstar))) near = s;
        splits.push_back(near);
    }
    if (std::find(splits.begin(), splits.end(), c->split_threshold) == splits.end())
        splits.push_back(c->split_threshold);
    std::vector<int> kmaxes = {c->fast_kmax};
    if (c->prec == BPMF_FP32 && c->K > 32 && c->K <= 64) kmaxes = {32, 64};
    std::vector<int> lows = {c->low_dmax};
    if (lowrank_available(c)) lows = {0, 8, 16};
    const int old_split = c->split_threshold, old_kmax = c->fast_kmax, old_low = c->low_dmax;
    ChainSnapshot sn;
    if (int r = snapshot_take(c, sn)) {
        snapshot_free(sn);
        return r;
    }
    int best_split = old_split, best_kmax = old_kmax, best_low = old_low, q = 0, rc = BPMF_OK;
    double best = 1e300, incumbent = 1e300;
    for (int ld : lows)
    for (int km : kmaxes)
        for (int sp : splits) {
            if ((rc = replan(c, sp, km, ld)) != BPMF_OK) break;
            if ((rc = snapshot_restore(c, sn)) != BPMF_OK) break;
            if ((rc = refresh_lowrank(c)) != BPMF_OK) break;
            // one untimed sweep builds the graph, then n_sweeps timed
            if ((rc = bpmf_run_sweeps(c, 1, 1, nullptr, nullptr)) != BPMF_OK) break;
            if ((rc = bpmf_run_sweeps(c, 2, n_sweeps, nullptr, nullptr)) != BPMF_OK) break;
            const double ms = c->last_ms / n_sweeps;
            if (q < 64) {
                if (tried_split) tried_split[q] = sp;
                if (tried_kmax) tried_kmax[q] = km;
                if (tried_low) tried_low[q] = ld;
                if (tried_ms) tried_ms[q] = ms;
            }
            ++q;
            if (sp == old_split && km == old_kmax && ld == old_low) incumbent = ms;
            if (ms < best) {
                best = ms;
                best_split = sp;
                best_kmax = km;
                best_low = ld;
            }
        }
    // keep the current plan unless a candidate is clearly faster (timing noise)
    if (best > 0.99 * incumbent) {
        best_split = old_split;
        best_kmax = old_kmax;
        best_low = old_low;
    }
    if (rc == BPMF_OK) rc = replan(c, best_split, best_kmax, best_low);
    if (rc == BPMF_OK) rc = snapshot_restore(c, sn);
    if (rc == BPMF_OK) rc = refresh_lowrank(c);
    if (rc == BPMF_OK) rc = ensure_graph(c);  // the chosen plan's graph, ready for timed sweeps
    snapshot_free(sn);
    if (rc != BPMF_OK) return rc;
    if (chosen_split) *chosen_split = best_split;
    if (chosen_kmax) *chosen_kmax = best_kmax;
    if (chosen_low) *chosen_low = best_low;
    if (n_tried) *n_tried = std::min(q, 64);
    return BPMF_OK;
}

// Capture and instantiate the sweep graph for the current plan if there is
// none (plan changes drop it), without launching it.
static int ensure_graph(bpmf_ctx *c)
{
    if (c->graph) return BPMF_OK;
    hipGraph_t g = nullptr;
    HIPCK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_sweep(c, c->stream);
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return fail(c, BPMF_E_DEVICE, "graph capture failed: %s / %s", hipGetErrorString(e),
                    hipGetErrorString(e2));
    }
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        c->graph = nullptr;
        return fail(c, BPMF_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    c->graph_src = g;
    return find_timing_nodes(c);
}

int bpmf_set_plan(bpmf_ctx *c, int32_t split_threshold, int32_t fast_kmax, int32_t lowrank_dmax)
{
    STICKY(c);
    if (split_threshold < 1 || split_threshold > (1 << 24))
        return fail(c, BPMF_E_INVAL, "split_threshold must be 1..2^24");
    if (fast_kmax < 0 || fast_kmax > 64) return fail(c, BPMF_E_INVAL, "fast_kmax must be 0..64");
    if (lowrank_dmax != 0 && lowrank_dmax != 4 && lowrank_dmax != 8 && lowrank_dmax != 16)
        return fail(c, BPMF_E_INVAL, "lowrank_dmax must be 0, 4, 8 or 16");
    if (lowrank_dmax && !lowrank_available(c))
        return fail(c, BPMF_E_INVAL, "the rank-one path needs FP32 factors and K <= 64");
    if (int rc = replan(c, split_threshold, fast_kmax, lowrank_dmax, true)) return rc;
    if (int rc = refresh_lowrank(c)) return rc;
    return ensure_graph(c);  // so that the next timed sweeps do not include the capture
}

int bpmf_run_sweeps(bpmf_ctx *c, uint32_t t0, uint32_t n, double *rmse_avg, double *rmse_last)
{
    STICKY(c);
    if (n == 0) return BPMF_OK;
    if (t0 == 0) return fail(c, BPMF_E_INVAL, "sweeps are numbered from 1 (t = 0 is the initialisation)");
    if ((int64_t)n > c->hist_cap) {
        HIPCK(c, hipStreamSynchronize(c->stream));
        hipFree(c->rmse_hist);
        c->rmse_hist = nullptr;
        int64_t cap = std::max<int64_t>(n, 2 * c->hist_cap);
        HIPCK(c, dalloc(&c->rmse_hist, 2 * (size_t)cap));
        c->hist_cap = cap;
        if (c->graph) {
            hipGraphExecDestroy(c->graph);
            c->graph = nullptr;
        }
        if (c->graph_src) {
            hipGraphDestroy(c->graph_src);
            c->graph_src = nullptr;
        }
    }
    if (int r = ensure_graph(c)) return r;
    // one set of four timing events per replay (replays past kTimedSweeps
    // share the last set, so the mean covers the first kTimedSweeps - 1 and
    // the final one)
    const uint32_t n_sets = c->timing_nodes ? std::min<uint32_t>(n, kTimedSweeps) : 0;
    if (c->tpool.size() < 4 * (size_t)n_sets) {
        // new events are recorded once before their first use in the graph:
        // an event's first record sets it up, which would otherwise happen
        // inside the timed replays
        while (c->tpool.size() < 4 * (size_t)n_sets) {
            hipEvent_t ev = nullptr;
            HIPCK(c, hipEventCreate(&ev));
            HIPCK(c, hipEventRecord(ev, c->stream));
            c->tpool.push_back(ev);
        }
        HIPCK(c, hipStreamSynchronize(c->stream));
    }
    c->row_ms[0] = c->row_ms[1] = -1.0;
    HIPCK(c, hipEventRecord(c->ev0, c->stream));
    HIPCK(c, launch_set_counter(c->ctr, 0, t0, c->stream));
    HIPCK(c, launch_set_counter(c->ctr, 1, t0, c->stream));
    HIPCK(c, launch_hyper(c, BPMF_SIDE_V, c->stream, 0));
    for (uint32_t i = 0; i < n; ++i) {
        if (n_sets) {
            const size_t set = std::min<uint32_t>(i, n_sets - 1);
            for (int k = 0; k < 4; ++k)
                HIPCK(c, hipGraphExecEventRecordNodeSetEvent(c->graph, c->tnode[k],
                                                             c->tpool[4 * set + k]));
        }
        HIPCK(c, hipGraphLaunch(c->graph, c->stream));
    }
    if (int r = timed_end(c)) return r;
    if (int r = check_status(c)) return r;
    double acc[2] = {0.0, 0.0};
    for (uint32_t q = 0; q < n_sets; ++q)
        for (int sd = 0; sd < 2; ++sd) {
            float ms = 0.f;
            HIPCK(c, hipEventElapsedTime(&ms, c->tpool[4 * q + 2 * sd], c->tpool[4 * q + 2 * sd + 1]));
            acc[sd] += ms;
        }
    if (n_sets) {
        c->row_ms[0] = acc[0] / n_sets;
        c->row_ms[1] = acc[1] / n_sets;
    }
    std::vector<double> h(2 * (size_t)n);
    HIPCK(c, hipMemcpy(h.data(), c->rmse_hist, sizeof(double) * 2 * n, hipMemcpyDeviceToHost));
    for (uint32_t i = 0; i < n; ++i) {
        if (rmse_avg) rmse_avg[i] = h[2 * i];
        if (rmse_last) rmse_last[i] = h[2 * i + 1];
    }
    return BPMF_OK;
}

int bpmf_profile_sweeps(bpmf_ctx *c, uint32_t t0, uint32_t n, double *phase_ms)
{
    STICKY(c);
    if (n == 0 || !phase_ms) return fail(c, BPMF_E_INVAL, "need n > 0 and an output array");
    if (t0 == 0) return fail(c, BPMF_E_INVAL, "sweeps are numbered from 1");
    if ((int64_t)n > c->hist_cap) return fail(c, BPMF_E_INVAL, "n exceeds the RMSE history (run bpmf_run_sweeps with n first)");
    hipEvent_t ev[8] = {};
    for (auto &e : ev) HIPCK(c, hipEventCreate(&e));
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    int rc = BPMF_OK;
    if (launch_set_counter(c->ctr, 0, t0 - 1, c->stream) != hipSuccess ||
        launch_set_counter(c->ctr, 1, t0, c->stream) != hipSuccess)
        rc = fail(c, BPMF_E_DEVICE, "counter launch failed");
    for (uint32_t i = 0; i < n && rc == BPMF_OK; ++i) {
        hipError_t e = enqueue_sweep_profiled(c, c->stream, ev);
        if (e == hipSuccess) e = hipEventSynchronize(ev[7]);
        for (int q = 0; q < 7 && e == hipSuccess; ++q) {
            float ms = 0;
            e = hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
            acc[q] += ms;
        }
        if (e != hipSuccess) rc = fail(c, BPMF_E_DEVICE, "profiled sweep: %s", hipGetErrorString(e));
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (rc != BPMF_OK) return rc;
    for (int q = 0; q < 7; ++q) phase_ms[q] = acc[q] / n;
    return check_status(c);
}

int bpmf_predict(bpmf_ctx *c, uint32_t t, int64_t n, const int32_t *row, const int32_t *col,
                 float *out, double *rmse_avg, double *rmse_last)
{
    STICKY(c);
    if (n < 0) return fail(c, BPMF_E_INVAL, "negative n");
    if (n == 0) {
        HIPCK(c, launch_set_counter(c->ctr, 0, t, c->stream));
        HIPCK(c, launch_set_counter(c->ctr, 1, t, c->stream));
        HIPCK(c, launch_predict_test(c, c->stream));
        double h[2];
        HIPCK(c, hipMemcpyAsync(h, c->rmse_hist, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIPCK(c, hipStreamSynchronize(c->stream));
        if (rmse_avg) *rmse_avg = h[0];
        if (rmse_last) *rmse_last = h[1];
        return BPMF_OK;
    }
    if (!row || !col || !out) return fail(c, BPMF_E_INVAL, "null pair arrays");
    for (int64_t e = 0; e < n; ++e)
        if (row[e] < 0 || row[e] >= c->M || col[e] < 0 || col[e] >= c->N)
            return fail(c, BPMF_E_RANGE, "pair %lld out of range", (long long)e);
    if (n > c->q_cap) {
        HIPCK(c, hipStreamSynchronize(c->stream));
        hipFree(c->q_row);
        hipFree(c->q_col);
        hipFree(c->q_out);
        c->q_row = c->q_col = nullptr;
        c->q_out = nullptr;
        c->q_cap = 0;
        HIPCK(c, dalloc(&c->q_row, n));
        HIPCK(c, dalloc(&c->q_col, n));
        HIPCK(c, dalloc(&c->q_out, n));
        c->q_cap = n;
    }
    HIPCK(c, hipMemcpyAsync(c->q_row, row, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
    HIPCK(c, hipMemcpyAsync(c->q_col, col, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
    HIPCK(c, launch_map_pairs(c, n, c->q_row, c->q_col, c->stream));
    HIPCK(c, launch_predict_pairs(c, n, c->q_row, c->q_col, c->q_out, c->stream));
    HIPCK(c, hipMemcpyAsync(out, c->q_out, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    return BPMF_OK;
}

static int copy_factor(bpmf_ctx *c, int32_t side, void *host, bool to_host)
{
    Side &sd = c->side[side];
    size_t es = elem_bytes(c);
    HIPCK(c, hipStreamSynchronize(c->stream));
    if (sd.rows == 0) return BPMF_OK;
    if (c->relabel) {
        // internal row r is the caller's row ext_of[side][r]
        const size_t rb = (size_t)c->K * es;
        const std::vector<int32_t> &ext = c->ext_of[side];
        std::vector<char> tmp((size_t)sd.rows * rb);
        char *h = (char *)host;
        if (to_host) {
            HIPCK(c, hipMemcpy2D(tmp.data(), rb, sd.X, c->ld * es, rb, sd.rows, hipMemcpyDeviceToHost));
            for (int64_t r = 0; r < sd.rows; ++r) memcpy(h + (size_t)ext[r] * rb, tmp.data() + (size_t)r * rb, rb);
        } else {
            for (int64_t r = 0; r < sd.rows; ++r) memcpy(tmp.data() + (size_t)r * rb, h + (size_t)ext[r] * rb, rb);
            HIPCK(c, hipMemcpy2D(sd.X, c->ld * es, tmp.data(), rb, rb, sd.rows, hipMemcpyHostToDevice));
        }
        return BPMF_OK;
    }
    if (to_host)
        HIPCK(c, hipMemcpy2D(host, c->K * es, sd.X, c->ld * es, c->K * es, sd.rows,
                             hipMemcpyDeviceToHost));
    else
        HIPCK(c, hipMemcpy2D(sd.X, c->ld * es, host, c->K * es, c->K * es, sd.rows,
                             hipMemcpyHostToDevice));
    return BPMF_OK;
}

int bpmf_get_factor(bpmf_ctx *c, int32_t side, void *host)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    if (!host) return fail(c, BPMF_E_INVAL, "null buffer");
    return copy_factor(c, side, host, true);
}

int bpmf_set_factor(bpmf_ctx *c, int32_t side, const void *host)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    if (!host) return fail(c, BPMF_E_INVAL, "null buffer");
    if (int r = copy_factor(c, side, const_cast<void *>(host), false)) return r;
    if (c->prec == BPMF_BF16_GRAM) {
        HIPCK(c, launch_to_bf16(c, side, c->stream));
        HIPCK(c, hipStreamSynchronize(c->stream));
    }
    return BPMF_OK;
}

int bpmf_get_factor_f64(bpmf_ctx *c, int32_t side, double *host)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    if (!host) return fail(c, BPMF_E_INVAL, "null buffer");
    if (c->prec == BPMF_FP64) return copy_factor(c, side, host, true);
    size_t n = (size_t)c->side[side].rows * c->K;
    std::vector<float> tmp(n);
    if (int r = copy_factor(c, side, tmp.data(), true)) return r;
    for (size_t q = 0; q < n; ++q) host[q] = tmp[q];
    return BPMF_OK;
}

int bpmf_set_factor_f64(bpmf_ctx *c, int32_t side, const double *host)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    if (!host) return fail(c, BPMF_E_INVAL, "null buffer");
    if (c->prec == BPMF_FP64) return copy_factor(c, side, const_cast<double *>(host), false);
    size_t n = (size_t)c->side[side].rows * c->K;
    std::vector<float> tmp(n);
    for (size_t q = 0; q < n; ++q) tmp[q] = (float)host[q];
    return bpmf_set_factor(c, side, tmp.data());
}

int bpmf_get_hyper(bpmf_ctx *c, int32_t side, double *mu, double *Lambda)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    HIPCK(c, hipStreamSynchronize(c->stream));
    if (mu) HIPCK(c, hipMemcpy(mu, c->side[side].mu, sizeof(double) * c->K, hipMemcpyDeviceToHost));
    if (Lambda)
        HIPCK(c, hipMemcpy(Lambda, c->side[side].Lam, sizeof(double) * c->K * c->K,
                           hipMemcpyDeviceToHost));
    return BPMF_OK;
}

int bpmf_set_hyper(bpmf_ctx *c, int32_t side, const double *mu, const double *Lambda)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    if (!mu || !Lambda) return fail(c, BPMF_E_INVAL, "null hyperparameters");
    HIPCK(c, hipStreamSynchronize(c->stream));
    HIPCK(c, hipMemcpy(c->side[side].mu, mu, sizeof(double) * c->K, hipMemcpyHostToDevice));
    HIPCK(c, hipMemcpy(c->side[side].Lam, Lambda, sizeof(double) * c->K * c->K,
                       hipMemcpyHostToDevice));
    HIPCK(c, launch_prior_to_working(c, side, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    return BPMF_OK;
}

int bpmf_get_chain_state(bpmf_ctx *c, double *pred_sum, uint32_t *n_avg)
{
    STICKY(c);
    HIPCK(c, hipStreamSynchronize(c->stream));
    if (n_avg) HIPCK(c, hipMemcpy(n_avg, c->ctr + 2, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (pred_sum && c->n_test) {
        std::vector<double> h(c->n_test);
        HIPCK(c, hipMemcpy(h.data(), c->pred_sum, sizeof(double) * c->n_test, hipMemcpyDeviceToHost));
        for (int64_t q = 0; q < c->n_test; ++q) pred_sum[c->test_src[q]] = h[q];
    }
    return BPMF_OK;
}

int bpmf_set_chain_state(bpmf_ctx *c, const double *pred_sum, uint32_t n_avg)
{
    STICKY(c);
    if (!pred_sum && c->n_test) return fail(c, BPMF_E_INVAL, "null prediction sums");
    for (int64_t e = 0; e < c->n_test; ++e)
        if (!isfinite(pred_sum[e])) return fail(c, BPMF_E_FORMAT, "non-finite prediction sum at %lld", (long long)e);
    HIPCK(c, hipStreamSynchronize(c->stream));
    if (c->n_test) {
        std::vector<double> h(c->n_test);
        for (int64_t q = 0; q < c->n_test; ++q) h[q] = pred_sum[c->test_src[q]];
        HIPCK(c, hipMemcpy(c->pred_sum, h.data(), sizeof(double) * c->n_test, hipMemcpyHostToDevice));
    }
    HIPCK(c, hipMemcpy(c->ctr + 2, &n_avg, sizeof(uint32_t), hipMemcpyHostToDevice));
    return BPMF_OK;
}

int bpmf_get_csc(bpmf_ctx *c, int64_t *ptr, int32_t *row, void *rc)
{
    STICKY(c);
    Side &sd = c->side[BPMF_SIDE_V];
    HIPCK(c, hipStreamSynchronize(c->stream));
    if (c->relabel) {
        // the stored CSC is that of the relabelled R: caller column j is internal
        // column int_of[1][j], whose rows map back through ext_of[0] and are
        // sorted again
        const size_t es = elem_bytes(c);
        std::vector<int64_t> iptr(c->N + 1);
        std::vector<int32_t> irow(c->nnz);
        std::vector<char> irc(c->nnz * es);
        HIPCK(c, hipMemcpy(iptr.data(), sd.ptr, sizeof(int64_t) * (c->N + 1), hipMemcpyDeviceToHost));
        if (c->nnz) {
            HIPCK(c, hipMemcpy(irow.data(), sd.nbr, sizeof(int32_t) * c->nnz, hipMemcpyDeviceToHost));
            HIPCK(c, hipMemcpy(irc.data(), sd.rc, es * c->nnz, hipMemcpyDeviceToHost));
        }
        std::vector<std::pair<int32_t, int64_t>> seg;
        int64_t q = 0;
        if (ptr) ptr[0] = 0;
        for (int64_t j = 0; j < c->N; ++j) {
            const int32_t jj = c->int_of[1][j];
            seg.clear();
            for (int64_t e = iptr[jj]; e < iptr[jj + 1]; ++e) seg.emplace_back(c->ext_of[0][irow[e]], e);
            std::sort(seg.begin(), seg.end());
            for (const auto &x : seg) {
                if (row) row[q] = x.first;
                if (rc) memcpy((char *)rc + q * es, irc.data() + x.second * es, es);
                ++q;
            }
            if (ptr) ptr[j + 1] = q;
        }
        return BPMF_OK;
    }
    if (ptr) HIPCK(c, hipMemcpy(ptr, sd.ptr, sizeof(int64_t) * (c->N + 1), hipMemcpyDeviceToHost));
    if (row && c->nnz)
        HIPCK(c, hipMemcpy(row, sd.nbr, sizeof(int32_t) * c->nnz, hipMemcpyDeviceToHost));
    if (rc && c->nnz)
        HIPCK(c, hipMemcpy(rc, sd.rc, elem_bytes(c) * c->nnz, hipMemcpyDeviceToHost));
    return BPMF_OK;
}

int bpmf_get_plan(bpmf_ctx *c, int32_t side, int32_t *perm, int64_t *n_split, int64_t *n_low)
{
    STICKY(c);
    if (int r = check_side(c, side)) return r;
    Side &sd = c->side[side];
    if (perm && c->relabel)
        for (int64_t k = 0; k < sd.rows; ++k) perm[k] = c->ext_of[side][sd.perm[k]];
    else if (perm)
        memcpy(perm, sd.perm.data(), sizeof(int32_t) * sd.rows);
    if (n_split) *n_split = sd.n_split;
    if (n_low) *n_low = sd.n_low;
    return BPMF_OK;
}

double bpmf_mean_rating(const bpmf_ctx *c) { return c ? c->rbar : 0.0; }

int bpmf_synchronize(bpmf_ctx *c)
{
    STICKY(c);
    HIPCK(c, hipStreamSynchronize(c->stream));
    return BPMF_OK;
}

int bpmf_last_time_ms(bpmf_ctx *c, double *ms)
{
    if (!c || !ms) return BPMF_E_INVAL;
    *ms = c->last_ms;
    return BPMF_OK;
}

int bpmf_row_kernel_ms(bpmf_ctx *c, double *ms)
{
    if (!c || !ms) return BPMF_E_INVAL;
    if (c->row_ms[0] < 0.0) return fail(c, BPMF_E_INVAL, "no timed sweeps (none run, or the graph has no timing nodes)");
    ms[0] = c->row_ms[0];
    ms[1] = c->row_ms[1];
    return BPMF_OK;
}

}  // extern "C"
