// internal.h -- library-private types shared by the host runtime and the
// kernel launchers.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace bpmf {

// One unit of row-update work.  slot < 0: the whole row [beg, end) of the
// neighbour list is processed and the row is redrawn.  slot >= 0: only the
// segment [beg, end) is accumulated and its partial Gram and rhs are written
// to partial slot `slot` (the row is finished later from its slots).
struct RowItem {
    int32_t row;
    int32_t slot;
    int64_t beg;
    int64_t end;
};

// A split row: its partials are slots [first, first + count), summed in
// slot order.
struct FinishItem {
    int32_t row;
    int32_t first;
    int32_t count;
    int32_t pad;
};

// One fold-in draw: request `req` (index into the batch) against stored
// sample `s`; its ratings are [beg, end) of the batch arrays.
struct FoldItem {
    int32_t req;
    int32_t s;
    int64_t beg;
    int64_t end;
};

struct FoldinState;  // fold-in server (foldin.cpp)

// Stages of one side's row update (the item loop of Algorithm 1), in an
// order that is also a valid serial order: the working copies of the prior
// the row kernels read; the segments of split rows (partial sums); the whole
// rows and the rank-one path; the finishing of split rows (needs the
// segments); the BF16 shadow of the factor (needs everything).  Whole rows
// depend only on the prior, so the sweep graph runs them beside the
// segments and the finishing.
enum UpdateStage { kStagePrior = 0, kStageSegments = 1, kStageRows = 2, kStageFinish = 3, kStageShadow = 4 };

struct Side {
    int64_t rows = 0;
    int64_t *ptr = nullptr;  // device [rows + 1] neighbour offsets
    int32_t *nbr = nullptr;  // device [nnz] neighbour ids (other side)
    void *rc = nullptr;      // device [nnz] centred ratings (float, or double in FP64 mode)
    void *X = nullptr;       // device [rows * ld] factor
    uint16_t *Xbf = nullptr; // device [rows * ld] BF16 copy of the factor (BF16 mode)
    uint16_t *rc3 = nullptr; // device [3 * (nnz + 32)] the centred ratings as three BF16 parts,
                             // hi, mid and lo, each a plane in rc's order ending in 32 zeros
                             // (BF16 mode, and FP32 with K <= 32; hi + mid + lo == rc exactly)
    double *mu = nullptr;    // device [K]
    double *Lam = nullptr;   // device [K * K]
    void *Lam_w = nullptr;   // device [K * K] Lambda in working precision
    void *Lmu_w = nullptr;   // device [K]     Lambda mu in working precision
    float *Lam_img = nullptr; // device [nb (nb + 1) / 2 * 256], nb = ceil(K / 16): Lambda in
                              // the blocked kernel's accumulator layout (K <= 128)
    float *Lam_pk = nullptr;  // device [KP (KP + 1) / 2], KP = 16 ceil(K / 16): Lambda packed
                              // lower-triangular for the K <= 64 matrix-core kernel
    RowItem *items = nullptr;
    int64_t n_items = 0;
    FinishItem *fin = nullptr;
    int64_t n_fin = 0;
    int64_t n_slots = 0;
    std::vector<int32_t> perm;  // host copy of the processing order
    std::vector<int64_t> hptr;  // host copy of the neighbour offsets (re-planning)
    // rows with few ratings on the rank-one-update path: the last n_low
    // work items; L_Lam^-1 and L_Lam^T mu from the hyper draw, and the
    // gathered factor premultiplied by L_Lam^-1
    int64_t n_low = 0;
    int64_t n_low_small = 0;  // the last of those with at most 8 ratings
    void *Linv_w = nullptr;   // device [K * K] FP32
    void *Ltmu_w = nullptr;   // device [K] FP32
    float *Yt = nullptr;      // device [other rows * ld]
    int64_t n_split = 0;
    uint32_t stream_row = 0, stream_hyp = 0, stream_init = 0;
};

}  // namespace bpmf

struct bpmf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;           // Gibbs calls (the caller's, or our own)
    bool own_stream = true;
    hipStream_t stream2 = nullptr;          // second stream for overlapped hyper draws
    hipStream_t stream3 = nullptr;          // whole rows beside the split rows in the graph
    hipEvent_t fork_ev[3] = {};             // fork/join events of the sweep graph
    hipEvent_t stage_ev[2] = {};            // fork/join of a side's whole-row branch
    int64_t M = 0, N = 0, nnz = 0, n_test = 0;
    int K = 0, ld = 0, prec = 1;
    double alpha = 2, beta0 = 2, nu0 = 0, rbar = 0;
    uint64_t seed = 0;
    int burn_in = 0;
    int split_threshold = 0;
    int fast_kmax = 32;  // FP32 rows up to this K take the column-per-lane kernel
    int low_dmax = 0;    // rows with at most this many ratings take the rank-one path (0: off)
    double *d_mu0 = nullptr, *d_W0inv = nullptr;
    bpmf::Side side[2];
    // test set
    int32_t *test_row = nullptr, *test_col = nullptr;
    float *test_val = nullptr;
    double *pred_sum = nullptr;
    std::vector<int64_t> test_src;  // test pair q (held in user order) is the caller's pair test_src[q]
    double *rmse_part = nullptr;  // per-block partial sums of squared errors
    int rmse_blocks = 0;
    double *rmse_hist = nullptr;  // [2 * hist_cap] (avg, last) per sweep of a run
    int64_t hist_cap = 0;
    // hyper workspace, one set per side so that the two draws may overlap
    double *hyp_part[2] = {};     // [hyp_blocks * (K + K(K+1)/2)]
    double *hyp_red[2] = {};      // [kHypRedGroups * (K + K(K+1)/2)] sums of the reduction's first pass
    int hyp_blocks = 0;
    double *hyp_stats[2] = {};    // [K + K(K+1)/2]
    double *hyp_scratch[2] = {};  // [4 * K * K + 8 * K]
    int *hyp_status = nullptr;    // device flags, 1 = ok: [0] hyper draw, [1] row draws (pivots)
    int hyp_lds_max = 65536;      // LDS bytes the draw kernel may use
    // split partials
    void *part = nullptr;
    int64_t part_slots = 0;
    // device counters: [0] = t, [1] = t0 of the running graph, [2] = running-mean count
    uint32_t *ctr = nullptr;
    // predict scratch for user-supplied pairs
    int32_t *q_row = nullptr, *q_col = nullptr;
    float *q_out = nullptr;
    int64_t q_cap = 0;
    void *scratch = nullptr;  // this device's staging area of bpmf_predict_noalloc
    // graph of one sweep
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_src = nullptr;          // kept: owns the event-record nodes below
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // row-kernel timing inside the graph: external event-record nodes before
    // and after the row kernel of each side (V start, V end, U start, U end),
    // re-pointed at a fresh set of events before every replay
    hipEvent_t tev[4] = {};
    hipGraphNode_t tnode[4] = {};
    bool timing_nodes = false;
    std::vector<hipEvent_t> tpool;           // 4 per sweep of the last run
    double row_ms[2] = {-1.0, -1.0};         // mean per launch, V and U
    double last_ms = 0;
    std::string err;
    bool sticky = false;
    int foldin_S = 16;
    uint64_t foldin_pool = 0;
    bpmf::FoldinState *foldin = nullptr;
    // degree-order relabelling (params.reorder): users and movies are held in
    // descending-degree order; ext_of[side][internal row] is the caller's id,
    // int_of[side][caller id] the internal row (host), d_int_of the device
    // copy of int_of used to map pair ids on the device
    bool relabel = false;
    std::vector<int32_t> ext_of[2], int_of[2];
    int32_t *d_int_of[2] = {};
};

namespace bpmf {

// ---- launchers (defined in the .hip files; all enqueue on `s`) ----
// Row update of one side: items, then split-row finishes.
hipError_t launch_row_update(bpmf_ctx *c, int side_id, hipStream_t s);
// Hyper draw of one side (statistics, reduction, single-workgroup draw) for
// sweep ctr[0] + t_off.
hipError_t launch_hyper(bpmf_ctx *c, int side_id, hipStream_t s, uint32_t t_off = 0);
// Predict the registered test set as sweep ctr[0]; writes rmse_hist[slot].
hipError_t launch_predict_test(bpmf_ctx *c, hipStream_t s);
hipError_t launch_predict_pairs(bpmf_ctx *c, int64_t n, const int32_t *row, const int32_t *col,
                                float *out, hipStream_t s);
// Caller ids to internal rows in place (relabelled contexts): row[e] and col[e]
// through d_int_of of the user and movie sides.
hipError_t launch_map_pairs(bpmf_ctx *c, int64_t n, int32_t *row, int32_t *col, hipStream_t s);
// Device address of the staging area of bpmf_predict_noalloc on c's device.
hipError_t predict_scratch_init(bpmf_ctx *c);
// Factor initialisation from Philox normals.
hipError_t launch_init_factor(bpmf_ctx *c, int side_id, hipStream_t s);
// Device counters.
hipError_t launch_set_counter(uint32_t *ctr, int idx, uint32_t value, hipStream_t s);
hipError_t launch_advance_t(uint32_t *ctr, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
// Working-precision prior (Lambda, Lambda mu) from the FP64 hyperparameters.
hipError_t launch_prior_to_working(bpmf_ctx *c, int side_id, hipStream_t s);
// BF16 copy of a factor.
hipError_t launch_to_bf16(bpmf_ctx *c, int side_id, hipStream_t s);
// The centred ratings of a side as three BF16 parts (rc3).
hipError_t launch_split_ratings(bpmf_ctx *c, int side_id, hipStream_t s);
// FP32 contexts whose matrix-core kernels take the rating planes rc3 for
// the rhs of their three-part BF16 Gram.
bool parts_gram_wanted(const bpmf_ctx *c);
// Largest dynamic LDS a generic row kernel needs for K (bytes).
size_t row_generic_lds_bytes(int K, int prec);
// Fold-in kernels (FP32 factors, K <= 64).
bool fast_path_available(const bpmf_ctx *c);
// Row kernel for FP32 with 32 < K <= 128 and BF16-Gram with K <= 128.
bool big_path_available(const bpmf_ctx *c);
// Rank-one-update path for rows with few ratings (FP32, K <= 64).
bool lowrank_available(const bpmf_ctx *c);
hipError_t launch_row_lowrank(bpmf_ctx *c, int side_id, hipStream_t s);
// Elements of one split-row partial slot: K(K+1)/2 + K packed for the
// column-per-lane and generic kernels, the accumulator image of the blocked
// kernel otherwise.
int64_t part_slot_elems(const bpmf_ctx *c);
// Sum each split row's partial slots (E elements each) into its first slot.
hipError_t launch_part_reduce(bpmf_ctx *c, Side &sd, hipStream_t s, int64_t E);
hipError_t launch_foldin_draw(const bpmf_ctx *c, const FoldItem *items, int64_t n_items,
                              const int32_t *nbr, const float *rc, const float *Vring,
                              const float *Lam_ring, const float *Lmu_ring, const uint64_t *req_ids,
                              int n_samples, float *U, hipStream_t s);
hipError_t launch_foldin_score(const bpmf_ctx *c, int n_req, int S, const float *Vring,
                               const float *U, float *mean, float *var, hipStream_t s);
hipError_t launch_foldin_topk(const bpmf_ctx *c, int n_req, const float *mean, const float *var,
                              const int32_t *req_beg, const int32_t *nbr, const int32_t *top_n,
                              int top_max, int32_t *out_ids, float *out_mean, float *out_var,
                              hipStream_t s);
void foldin_destroy(bpmf_ctx *c);

}  // namespace bpmf
