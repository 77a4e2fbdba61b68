// hm_internal.h -- internal types of libhm (host side and kernel interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hm.h"

namespace hm {

// Workspace buffers the block products read from and write to.  Each is
// row-major with leading dimension ldq (Q rounded up to a multiple of the
// column tile of the evaluation).
enum Buf : int32_t {
    BUF_WT = 0,    // N x Qp   W in tree order
    BUF_YT = 1,    // N x Qp   Y in tree order
    BUF_WHAT = 2,  // R x Qp   skeleton weights, node a at rows [wrow[a], wrow[a]+k_a)
    BUF_YHAT = 3,  // R x Qp   skeleton potentials, same rows
    BUF_COUNT = 4
};

// One operand pair of a block product: the A block (stored K-major: element
// (row i, contraction t) at a_off + t*lda + i, zero-padded to lda >= M rows
// and to Kpad = round_up(K, 16) contraction rows) times K rows of workspace
// buffer b_buf starting at row b_row.
struct Seg {
    int64_t a_off;  // element offset into the block store
    int64_t b_row;
    int32_t lda;    // padded row count of the A block (multiple of 16)
    int32_t K;      // contraction length (> 0)
    int32_t b_buf;
    int32_t Kpad;   // stored contraction rows (multiple of 16)
    int64_t a_off16; // element offset of the block in the split-BF16 store (see k_make_bf16x3)
    int64_t b_row16; // first row of the B operand's node in its split-BF16 workspace (see Split16)
    int32_t from_pts; // the A block can be computed from points, A[k][m] = K(x_m, y_k):
                      //   1: near block of the job's leaf a and the leaf b whose W rows start
                      //      at b_row (x: a's points, y: b's points, both tree order)
                      //   2: far block B_ab of the job's node a and node b whose Ŵ rows start
                      //      at b_row (x: a's skeleton points, y: b's, both in Ŵ row order)
                      //   0: stored only
    int32_t trans;    // 1: a mirror block of a symmetric store: element (row i, contraction t) at
                      //   a_off + i * tstride + t (the stored block of the partner pair, read
                      //   transposed); 0: K-major as above
    int32_t tstride;  // trans: distance between consecutive rows of this A block (elements)
    int32_t pad_;
};

// Largest point dimension of the near field computed from points (the tile's
// points sit in LDS beside the pipeline stages).
constexpr int kMaxPointDim = 15;
// Largest point dimension of blocks computed from points at all (above
// kMaxPointDim the lanes read the tile's points from global memory).
constexpr int kMaxPointDimAny = 64;

// Split-BF16 workspaces of the mixed-precision evaluation: W (tree order),
// Ŵ and the leaves' Ŷ, each value v stored as hi = bf16(v), lo = bf16(v - hi)
// (from the FP32 value).  Every node's rows start at a multiple of 32 (its
// padded row start, b_row16 / out16) and are cut into 32-row chunks; the
// chunk of rows [g, g + 32) holds, for each column n < ldq, the 32 hi values
// then the 32 lo values: element (row g + k, column n, part h) at
//     g * 2 * ldq + n * 64 + h * 32 + k      (bf16 elements, g % 32 == 0).
// A chunk of a column tile is then one contiguous run, copied as is into the
// LDS layout of the split-BF16 products.  Rows past a node's last row are zero.
struct Split16 {
    static constexpr int kRows = 32;
};

// One output block: rows [out_row, out_row + M) of buffer out_buf (M <= tile
// height) receive the sum over segments [seg_begin, seg_end) (overwritten).
// m0 is the first row of the A blocks this task covers (tasks taller than the
// tile are split).
struct Task {
    int64_t out_row;
    int32_t out_buf;
    int32_t M;
    int32_t m0;
    int32_t seg_begin;
    int32_t seg_end;
    int32_t pad_;
};

// A phase = one launch: a contiguous task range with a common tile height.
struct Phase {
    int32_t kind;         // 1 up, 2 down, 3 leaf
    int32_t level;
    int32_t task_begin;
    int32_t task_count;
    int32_t bm;           // tile height (64 or 128)
    int64_t seg_count;
    double flops_per_col; // algorithmic flops of this phase per column
};

// Validated host-side copy of the compressed representation.
struct HostRepr {
    int64_t N = 0, d = 0;
    int32_t n_nodes = 0, depth = 0;
    uint32_t flags = 0;
    int32_t kernel = 0, rmax = 0, m = 0;
    double h = 0, tol = 0, tau = 0;
    std::vector<int64_t> perm, start, size, basis_off, far_ptr, far_off, near_ptr, near_off;
    std::vector<int32_t> parent, left, right, level, rank, far_col, near_col;
    std::vector<double> basis, B, D;          // owned values (file loads)
    std::vector<int64_t> skel_ptr, skel;       // skeleton point indices per node (empty: not given)
    const double *basis_ext = nullptr;         // borrowed values (host-array loads)
    const double *B_ext = nullptr;
    const double *D_ext = nullptr;
    int64_t basis_len = 0, B_len = 0, D_len = 0;
    const double *basis_ptr() const { return basis_ext ? basis_ext : basis.data(); }
    const double *B_ptr() const { return B_ext ? B_ext : B.data(); }
    const double *D_ptr() const { return D_ext ? D_ext : D.data(); }
};

// One block copy of the device repack (see k_repack).
struct RepackJob {
    int64_t src_off;  // offset into the staged source chunk
    int64_t dst_off;  // offset into the block store
    int32_t rows, cols;
    int32_t mode;     // 0 transpose, 1 column slice
    int32_t c0, ncols;
    int32_t ld;       // padded length of a stored row
};

// One entry of the persistent task-graph launch (see k_persistent): a row
// tile of one output block for one column tile, with its dependencies.
struct PTask {
    int64_t out_row;
    int64_t out16;       // split-BF16 copy of the output: first row in the split workspace, or -1
    int32_t out_buf, M, m0, seg_begin, seg_end;
    int32_t bm;          // tile height: 32, 64, 96 or 128 (64 or 128 in a mixed-precision launch)
    int32_t accumulate;  // 1: out += product (a leaf's far part after its near part)
    int32_t n0;          // first column of the tile
    int32_t bn;          // tile width: the launch's column tile, or (a plan with narrow tiles) a
                         // narrower power of two for the last columns of a matrix
    int32_t mat;         // index into the MatDesc table
    int32_t ndeps;       // entries that must finish first
    int32_t succ_begin, succ_end;  // successor entries (queue positions) in the succ array
    int32_t mode;        // 0: products in the launch's type; 1: split BF16 (hi+lo) with FP32
                         // accumulation; 2: split BF16 for all segments but the last, FP64 for
                         // the last one, continuing from the FP32 partial sums
    int32_t out_split;   // with out16 >= 0: 1 = FP64 output and split copy, 2 = split copy only
};

// Device addresses of one matrix for the persistent launch.
struct MatDesc {
    const void *store;
    void *buf[4];
    int64_t ldq;
    const Seg *segs;
    const void *store16;  // split-BF16 store (mixed precision), or null
    void *buf16[4];       // split-BF16 workspaces (mixed precision): [BUF_WT] W, [BUF_WHAT] Ŵ, [BUF_YHAT] Ŷ
    const double *pts;    // FP64 launch: points in tree order (N x pts_d) to compute the near
                          // blocks from, or null to read them from the store
    const double *skel_pts;  // FP64 launch: skeleton points in Ŵ row order (skel_rows x pts_d) to
                             // compute the far blocks from, or null to read them from the store
    int32_t pts_d;
    int32_t kern;         // 0: exp(-r^2 kscale), 1: exp(-r kscale)
    double kscale;        // 1 / (2 h^2) or 1 / h
};

// One matrix's permutes in a batched launch.
struct PermDesc {
    const void *W;
    int64_t ldw;
    void *Y;
    int64_t ldy;
    void *Wt;
    const void *Yt;
    int64_t ldq;
    const int64_t *perm;
    int64_t N, Q;
};

// One request of a served sweep: its columns [col0, col0 + Q) of the sweep
// come from W (original order, leading dimension ldw) and go to Y.
struct ReqDesc {
    const void *W;
    int64_t ldw;
    void *Y;
    int64_t ldy;
    int64_t col0, Q;
};
// Widest served sweep (columns); a sweep's column -> request map is an int16
// table of this length.
constexpr int kServeMaxCols = 1024;

// A node-level job of the evaluation's dependency graph (host side).
struct GJob {
    int32_t kind;        // 1 up, 2 down, 3 near, 4 leaf far part
    int32_t node;
    int32_t out_buf;
    int64_t out_row;
    int32_t M;
    int32_t seg_begin, seg_end;  // into the matrix's segment table
    int32_t accumulate;
    int32_t mode;        // 0 native, 1 split BF16, 2 split BF16 then FP64 (see PTask)
    int64_t kpad;        // sum of Kpad over its segments (work model)
    int64_t kpad_split;  // the part of kpad computed in split BF16
    int64_t out16 = -1;  // split-BF16 copy of the output (see PTask)
    int32_t out_split = 0;
    std::vector<int32_t> preds;  // job indices
};

// Expanded, ordered graph of one matrix for one (column tile, Q) choice.
struct GraphPlan {
    int bn = 0;
    int64_t Q = -1;      // cache key: padded columns (padded_columns)
    int mode = 0;        // 0: native job graph, 1: mixed-precision job graph
    int n_tasks = 0;
    PTask *d_tasks = nullptr;
    int32_t *d_succ = nullptr;
    int32_t *d_counters = nullptr;
    double est_ms = 0;   // list-scheduling estimate (diagnostic)
    bool sym = false;    // some matrix of the plan has a symmetric store (mirror blocks)
    bool narrow = false; // some tile is narrower than bn (launched with the narrow-tile instantiation)
};

// Output of inspector-p1 (Section 5 "Reusing Inspection"): everything the
// compression needs that depends on the points and the admissibility only,
// not on the kernel function or the accuracy.  Built once on the host, reused
// by every inspector-p2 run.
struct Structure {
    HostRepr r;                        // tree, perm, geometry-derived far/near lists; no ranks or blocks
    std::vector<double> X;             // N x d points, original order (a copy)
    std::vector<int64_t> rows_ptr;     // row sample of node a: rows[rows_ptr[a] .. rows_ptr[a+1]),
    std::vector<int64_t> rows;         //   original point indices of the sampled far-field points
    int32_t leaf_size = 0, admissibility = 0;
    double tau = 0;
};

struct PrecStore {
    void *blocks = nullptr;   // device block store (FP64 or FP32 elements)
    size_t bytes = 0;
};

struct ProfileAcc {
    double ms[5] = {0, 0, 0, 0, 0};
    int64_t launches[5] = {0, 0, 0, 0, 0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[5];
};

}  // namespace hm

struct hm_matrix_s {
    int device = 0;
    int64_t N = 0;
    int32_t n_nodes = 0, depth = 0, max_rank = 0;
    int64_t n_far = 0, n_near = 0;
    int64_t E_V = 0, E_T = 0, E_B = 0, E_D = 0;
    int64_t skel_rows = 0;                 // rows of the What / Yhat buffers
    int64_t store_elems = 0;               // elements of the padded block store
    hm::PrecStore prec[2];                 // [HM_PREC_FP64], [HM_PREC_FP32]
    int64_t *d_perm = nullptr;             // tree position -> original index
    hm::Task *d_tasks = nullptr;
    hm::Seg *d_segs = nullptr;
    std::vector<hm::Phase> phases;
    std::vector<hm::GJob> gjobs;           // dependency graph of one evaluation (down jobs cut)
    std::vector<hm::GJob> gjobs_whole;     // same, every down job whole (launches of many graphs)
    std::vector<hm::GJob> gjobs_mixed;     // same, with split-BF16 and FP64 parts separated
    double task_k = 0;                     // job_task_k(gjobs)
    void *store16 = nullptr;               // split-BF16 block store (HM_PREC_BF16X3)
    size_t store16_bytes = 0;
    int64_t rows16_w = 0, rows16_h = 0;    // rows of the split W / Ŵ, Ŷ workspaces (see Split16)
    int64_t *d_wchunks = nullptr;          // W's 32-row chunks: (first tree row, rows, split row)
    int64_t n_wchunks = 0;
    void *ws16[hm::BUF_COUNT] = {nullptr};  // split workspaces, grown on demand ([BUF_WT], [BUF_WHAT], [BUF_YHAT])
    size_t ws16_bytes[hm::BUF_COUNT] = {0};
    std::vector<hm::GraphPlan> plans[2];   // per element size: one plan per (tile, tile count)
    hm::MatDesc *d_mat = nullptr;          // one descriptor (persistent launch)
    hm::MatDesc mat_cache[2] = {};         // last uploaded descriptor per element size
    int mat_slot = -1;                     // element-size slot of the uploaded descriptor
    int32_t *d_head = nullptr;             // queue head + error flag (2 ints)
    int n_cu = 0;                          // compute units of the device
    // workspaces (per element size), grown on demand
    void *ws[2][hm::BUF_COUNT] = {{nullptr}};
    size_t ws_bytes[2][hm::BUF_COUNT] = {{0}};
    hm::ProfileAcc prof;
    bool symmetric = false;                // loaded with HM_LOAD_SYMMETRIC (mirror blocks in the store)
    bool near_stored = true;               // false: loaded with HM_LOAD_NO_NEAR_BLOCKS
    bool far_stored = true;                // false: loaded with HM_LOAD_NO_FAR_BLOCKS
    std::vector<int64_t> skel_row_pt;      // original point index of each Ŵ row (empty: no skeletons)
    // points for the blocks computed on the fly (hm_set_points)
    double *d_pts = nullptr;               // N x pts_d, tree order
    double *d_skel_pts = nullptr;          // skel_rows x pts_d, Ŵ row order (with skeletons)
    int32_t pts_d = 0, pts_kern = 0;
    double pts_scale = 0;
    // what the representation was compressed with (its metadata; 0 = not stated)
    int64_t repr_d = 0;
    int32_t repr_kernel = 0;
    double repr_h = 0;
};

struct hm_repr_s {
    hm::HostRepr r;
    std::vector<int64_t> skel_ptr, skel;
};

struct hm_structure_s {
    hm::Structure s;
};

namespace hm {

// Thread-local error reporting.
hm_status fail(hm_status s, const std::string &msg);

// Parse an HMC1 file into a HostRepr (host only; no device work).
hm_status read_file(const char *path, HostRepr &out);
// Copy and validate host arrays.
hm_status from_view(const hm_host_repr &v, HostRepr &out);
// Structural validation shared by both loaders.
hm_status validate(const HostRepr &r);

// Where the far and near blocks of build_matrix come from when they are not
// in the representation's arrays: generated in the device store from the
// points (inspector-p2 builds a matrix this way without copying its blocks
// through the host).  All device pointers belong to the caller and stay
// valid during build_matrix.
struct BlockSource {
    const double *X = nullptr;       // device, N x d points in the caller's original order
    int32_t d = 0, kern = 0;         // kernel 0: exp(-r^2 kscale), 1: exp(-r kscale)
    double kscale = 0;
    const int64_t *idx = nullptr;    // device: [perm (N entries) | every node's skeleton, node order]
};
// One generated block: dst[t * ld + i] = K(X[idx[r_off + i]], X[idx[c_off + t]])
// for i < rows, t < cols, and zero for rows <= i < ld.
struct GenJob {
    int64_t dst_off, r_off, c_off;
    int32_t rows, cols, ld, pad_;
};
hipError_t launch_gen_store(const GenJob *jobs, int njobs, const BlockSource &src, double *store, hipStream_t s);

// Build the device store, tables and phases for a validated representation.
// gen (optional): generate the far and near blocks from the points instead
// of copying them from r.B and r.D (which may then be empty).
hm_status build_matrix(const HostRepr &r, int device, unsigned prec_mask, hm_matrix *out,
                       const BlockSource *gen = nullptr);

// Kernel launchers (hm_kernels.hip).
// Column tile for Q columns (16..256) in a phase of the given kind (1 up,
// 2 down, 3 leaf): the smallest tile that holds Q columns, at most 256.
int pick_bn(int64_t Q, int kind);
// Whether a persistent launch with column tile bn over elem_bytes elements
// also has 32- and 96-row tiles (besides 64 and 128).  Not in mixed-precision
// launches, nor for FP64 with 128-column tiles, which is held to 128 VGPRs
// (two workgroups per compute unit) and has no registers to spare.
constexpr bool fine_tiles(int elem_bytes, int bn, bool split) {
    return !split && !(elem_bytes == 8 && bn == 128);
}
// Whether it has 48-, 80- and 112-row tiles as well (row tiles in steps of 16):
// FP32 at 256 columns, where every such tile keeps all 8 waves busy (one
// wave per 32 columns, each over the tile's full height).
constexpr bool fine16_tiles(int elem_bytes, int bn, bool split) {
    return !split && elem_bytes == 4 && bn == 256;
}
// Column tile of the persistent task-graph launch for Q columns of elem_bytes
// (split: the launch runs split-BF16 tiles; task_k: the flop-weighted mean
// contraction length of the graph's jobs, see job_task_k).
int graph_bn(int64_t Q, int elem_bytes, bool split, double task_k);
// Flop-weighted mean contraction length of a job graph: sum M k^2 / sum M k.
double job_task_k(const std::vector<GJob> &jobs);
hipError_t launch_phase(const hm_matrix_s *h, const Phase &ph, int elem_bytes, int bn, int64_t ldq,
                        void *const bufs[BUF_COUNT], hipStream_t s);
hipError_t launch_permute_in(const void *W, int64_t ldw, void *Wt, int64_t Qp, const int64_t *perm,
                             int64_t N, int64_t Q, int elem_bytes, hipStream_t s);
hipError_t launch_permute_out(const void *Yt, int64_t Qp, void *Y, int64_t ldy, const int64_t *perm,
                              int64_t N, int64_t Q, int elem_bytes, hipStream_t s);
hipError_t launch_convert_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t s);
// Served sweep: Wt[t * ldt + c] = W_r[perm[t] * ldw_r + c - col0_r] for the
// request r = col2req[c] owning column c < cols, zero for cols <= c < width.
hipError_t launch_gather_in(const ReqDesc *reqs, const int16_t *col2req, int64_t cols, int64_t width,
                            void *Wt, int64_t ldt, const int64_t *perm, int64_t N, int elem_bytes, hipStream_t s);
// Served sweep: Y_r[perm[t] * ldy_r + c - col0_r] = Yt[t * ldt + c] for c < cols.
hipError_t launch_scatter_out(const ReqDesc *reqs, const int16_t *col2req, int64_t cols, const void *Yt,
                              int64_t ldt, const int64_t *perm, int64_t N, int elem_bytes, hipStream_t s);
// Split-BF16 copies of blocks (one per segment) of the FP64 store.
// W (original order, ldw, FP64) -> split-BF16 W in tree order (see Split16),
// one 32-row chunk per (chunks entry, column); columns >= Q and rows past a
// leaf are zero.  perm null: identity.
hipError_t launch_permute_in_split(const double *W, int64_t ldw, void *W16, int64_t ldq, const int64_t *perm,
                                   const int64_t *chunks, int64_t n_chunks, int64_t Q, hipStream_t s);
hipError_t launch_make_bf16x3(const double *store, const Seg *segs, int nsegs, void *store16,
                              hipStream_t s);
hipError_t launch_repack(const double *stage, const RepackJob *jobs, int njobs, double *store,
                         hipStream_t s);
// Batched row gather (in = true: W -> Wt) or scatter (Yt -> Y) for n matrices;
// max_elems bounds N * ldq over the batch.
hipError_t launch_permute_batched(const PermDesc *d, int n, int64_t max_elems, int elem_bytes,
                                  bool in, hipStream_t s);
// Where a single-matrix launch writes the leaf rows: the caller's Y (row
// perm[t] for tree row t, or t when perm is null; leading dimension ldy;
// first Q columns).  Y null: the tree-order workspace (then a permute-out
// follows).
struct OutScatter {
    void *Y = nullptr;
    int64_t ldy = 0, Q = 0;
    const int64_t *perm = nullptr;
    bool from_points = false;  // FP64: the launch that computes near and/or far blocks from points
};
// Validated arguments of one evaluation and the launch shape they imply.
struct EvalSetup {
    bool valid = false;   // false with HM_OK: Q = 0, nothing to do
    int es = 8, slot = 0; // element bytes of W and Y; workspace / plan slot (0 FP64, 1 FP32)
    bool mixed = false, level_sched = false, near_pts = false, far_pts = false, from_points = false;
    int bn_kind[4] = {0, 0, 0, 0};  // column tile per phase kind (1 up, 2 down, 3 leaf); one tile for the graph
    int64_t Qp = 0;                 // workspace leading dimension (padded_columns)
    bool narrow = false;            // the task graph may end a matrix's columns with a narrower tile
    const int64_t *perm = nullptr;  // tree position -> caller's row (null with HM_TREE_ORDER)
};
// Validate hm_eval's arguments against h (no device work, messages prefixed
// by `who`) and derive the tiles and the workspace leading dimension.
hm_status eval_setup(const char *who, hm_matrix h, const void *W, int64_t ldw, void *Y, int64_t ldy, int64_t Q,
                     hm_dtype dtype, hm_prec prec, unsigned flags, EvalSetup &out);
// Persistent launch of a plan (init + graph kernel) on stream s.  counters:
// the dependency counters to use (one per queue entry), or null for the
// plan's own (launches that may overlap on one plan need their own).
hipError_t launch_persistent(const GraphPlan &plan, int elem_bytes, const MatDesc *d_mat,
                             int32_t *d_head, int grid, hipStream_t s, const OutScatter &out = OutScatter{},
                             int32_t *counters = nullptr);
// Resident workgroups per CU of the persistent kernel for (elem_bytes, bn).
int persistent_occupancy(int elem_bytes, int bn, bool split = false, bool sym = false, bool narrow = false);
// Workspace columns for Q columns in tiles of bn: Q rounded up to bn, or with
// narrow_tail, the last partial tile only to the smallest power of two (at
// least 16) that holds it.  A plan's tiles are bn wide up to the last full
// tile of bn in Qp and the rest is that narrower tile.
int64_t padded_columns(int64_t Q, int bn, bool narrow_tail);

// Expand the job graph for Q columns with column tile bn, order it by list
// scheduling on `workers` simulated workgroups, and upload it (hm_sched.hip).
// The plan of h for (bn, ldq / bn column tiles), built and cached on first use.
// build = false: look the plan up only (HM_ERR_INVALID when it was never built).
hm_status get_plan(hm_matrix h, int slot, int bn, int64_t ldq, int workers, GraphPlan **out,
                   int mode = 0, bool build = true);
// Grow h's workspaces for element-size slot to a leading dimension of ldq.
hm_status reserve_ws(hm_matrix h, int slot, int64_t ldq);
// One matrix's share of a (possibly multi-matrix) plan.
struct PlanPart {
    hm_matrix h;
    int mat;  // index in the MatDesc table
    int64_t Qp;  // padded columns: tiles of bn, then at most one narrower tile (padded_columns)
    int mode = 0;  // which job graph of h: 0 native, 1 mixed precision
    bool cut_down = true;  // native graph: down jobs cut (one matrix alone) or whole (many graphs)
};
hm_status build_plan(const std::vector<PlanPart> &parts, int bn, int elem_bytes, int workers, GraphPlan &plan);
void free_plan(GraphPlan &p);

}  // namespace hm
