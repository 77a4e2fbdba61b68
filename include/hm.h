/*
 * hm.h -- C ABI of libhm: evaluation Y = K~ W of a compressed H^2 (HMatrix)
 * kernel matrix on an AMD Instinct MI355X (gfx950).
 *
 * The operation (MatRox, arXiv 1812.07152, Section 2.1 "Evaluation", with the
 * compressed representation of Section 3.1): K~ is the N x N matrix made of
 *   - near blocks  K~[I_a, I_b] = D_ab (dense, leaf pairs in the near lists),
 *   - far blocks   K~[I_a, I_b] = Pc_a^T B_ab Pc_b for the far pairs, where the
 *     nested basis Pc_a is the leaf interpolation matrix P_a for a leaf and
 *     T_a * blockdiag(Pc_left, Pc_right) for an internal node (the V/U
 *     generators; U = V for the symmetric kernels the paper targets).
 * Evaluation computes Y = K~ W without assembling K~: a bottom-up pass over
 * the cluster tree (skeleton weights), the far-field reduction over B, a
 * top-down pass, and the near-field reduction over D (the two loop types the
 * paper distinguishes: reduction loops and tree loops).
 *
 * Conventions for every entry point:
 *   - Every function returns hm_status (HM_OK = 0) and never throws; on a
 *     non-OK status hm_last_error() describes the failure (thread-local).
 *   - Arguments are validated before any device work; an invalid argument
 *     returns HM_ERR_INVALID and launches nothing.
 *   - W and Y are caller-owned DEVICE pointers (HIP global memory), row-major
 *     N x Q with leading dimensions ldw, ldy (in elements, >= Q), in the
 *     caller's original point order unless HM_TREE_ORDER is set.  Y is
 *     overwritten, never accumulated.  Both must stay alive until the work
 *     enqueued on the stream has completed.
 *   - hm_eval is asynchronous on the caller's hipStream_t (NULL = the null
 *     stream); W may be reused or freed only after the stream has completed.
 *   - The library owns the device copy of the compressed representation and
 *     all workspaces; they live until hm_free().
 */
#ifndef HM_H
#define HM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HM_OK = 0,
    HM_ERR_INVALID = -1,  /* bad argument (null pointer, Q < 0, ld < Q, precision not loaded, ...) */
    HM_ERR_FORMAT = -2,   /* malformed compressed representation (file or host arrays) */
    HM_ERR_NOMEM = -3,    /* device or host allocation failed */
    HM_ERR_DEVICE = -4,   /* a HIP call failed */
    HM_ERR_BUSY = -5,     /* admission refused (server): retry later */
    HM_ERR_PENDING = -6,  /* result not ready yet */
    HM_ERR_INTERNAL = -7
} hm_status;

/* Element type of W and Y. */
typedef enum { HM_F64 = 0, HM_F32 = 1 } hm_dtype;

/* Arithmetic used for the block products.
 *   HM_PREC_FP64: FP64 everywhere (W, Y in FP64).
 *   HM_PREC_FP32: FP32 blocks and FP32 accumulation (W, Y in FP32).
 *   HM_PREC_BF16X3: mixed precision (W, Y in FP64).  The near-field, far
 *     (coupling) and leaf-basis products split both operands into BF16
 *     hi + lo parts and sum hi*hi + hi*lo + lo*hi on MFMA with FP32
 *     accumulation (relative error of a product about 2^-16); the transfer
 *     products of the up and down passes and the final near + far sum stay in
 *     FP64.  Loading it keeps the FP64 store and adds a split-BF16 store. */
typedef enum { HM_PREC_FP64 = 0, HM_PREC_FP32 = 1, HM_PREC_BF16X3 = 2 } hm_prec;

/* Bit for hm_load_*'s prec_mask: which precisions to keep on the device. */
#define HM_PRECBIT(p) (1u << (unsigned)(p))
/* prec_mask bit: leave the near blocks out of the device store (their HBM is
 * not allocated).  FP64 only (HM_ERR_INVALID with the FP32 or BF16X3 bits);
 * every hm_eval on the matrix must then pass HM_NEAR_FROM_POINTS (points set
 * with hm_set_points), and hm_batch_create / hm_server_add reject it. */
#define HM_LOAD_NO_NEAR_BLOCKS (1u << 8)
/* prec_mask bit: leave the far (coupling) blocks B_ab out of the device store.
 * FP64 only, as HM_LOAD_NO_NEAR_BLOCKS, and the representation must carry its
 * skeletons (skel_ptr/skel; HM_ERR_INVALID otherwise); every hm_eval on the
 * matrix must then pass HM_FAR_FROM_POINTS. */
#define HM_LOAD_NO_FAR_BLOCKS (1u << 9)
/* prec_mask bit: symmetric storage.  The kernel matrix is symmetric
 * (Section 1), so B_ba = B_ab^T and D_ba = D_ab^T: each far and near block of
 * an unordered pair is stored once (for the lower node number) and the other
 * product reads it transposed; the FP64 and FP32 stores hold about half the
 * bytes (the split-BF16 store keeps both orientations).  The representation
 * must be symmetric bitwise (partner in the other node's list, transposed
 * values): HM_ERR_FORMAT otherwise.  Results equal those of the full store
 * bitwise. */
#define HM_LOAD_SYMMETRIC (1u << 10)

/* hm_eval flags */
#define HM_TREE_ORDER 1u  /* W and Y are already in tree order: skip both permutes */
#define HM_PROFILE 2u     /* record HIP events around each phase (see hm_profile_read) */
#define HM_NEAR_FROM_POINTS 4u /* FP64 only: compute the near blocks from the points set with
                                  hm_set_points instead of reading them from the device store */
#define HM_FAR_FROM_POINTS 8u  /* FP64 only: compute the far blocks B_ab = K(X[skel_a], X[skel_b])
                                  from the points and the skeletons instead of reading them */
#define HM_LEVEL_LAUNCHES 16u  /* FP64 / FP32 only: one launch per tree level (up levels, down
                                  levels, leaf pass, permute-out) instead of the persistent
                                  task-graph launch; same results to rounding */

typedef struct hm_matrix_s *hm_matrix;

/* Host view of a compressed representation (the HMC1 file's content).  All
 * pointers are borrowed and only read during hm_load_compressed_mem.  Arrays
 * are indexed by node 0..n_nodes-1 (node 0 is the root) or by pair.
 *   perm[t]       original index of the point at tree position t (N entries)
 *   start,size    each node owns tree positions [start, start+size)
 *   parent,left,right  tree links (-1 when absent); a node has 0 or 2 children
 *   level         depth from the root; rank = k_a (0 = no basis)
 *   basis_off     offset (in doubles) of the node's basis in basis[]: the
 *                 k_a x size_a matrix P_a (leaf) or k_a x (k_l + k_r) transfer
 *                 T_a (internal), row-major, columns [skeleton(l), skeleton(r)]
 *   far_ptr/far_col/far_off, B   far pairs, CSR by row node a: B_ab is
 *                 k_a x k_b row-major at B + far_off[e]
 *   near_ptr/near_col/near_off, D near pairs (leaves only): D_ab is
 *                 size_a x size_b row-major at D + near_off[e], rows and columns
 *                 in tree order
 *   skel_ptr/skel optional (may be NULL): skeleton point indices per node. */
typedef struct {
    int64_t N, d;
    int32_t n_nodes, depth;
    uint32_t flags;                 /* bit0: built with HSS admissibility (metadata) */
    int32_t kernel;                 /* metadata: 0 Gaussian, 1 Laplace-type */
    double h, tol, tau;             /* metadata */
    int32_t rmax, m;                /* metadata */
    int64_t n_far, n_near, basis_len, B_len, D_len, skel_len;
    const int64_t *perm, *start, *size;
    const int32_t *parent, *left, *right, *level, *rank;
    const int64_t *basis_off;
    const double *basis;
    const int64_t *far_ptr;
    const int32_t *far_col;
    const int64_t *far_off;
    const double *B;
    const int64_t *near_ptr;
    const int32_t *near_col;
    const int64_t *near_off;
    const double *D;
    const int64_t *skel_ptr, *skel;
} hm_host_repr;

typedef struct {
    int64_t N;
    int32_t n_nodes, depth, max_rank, device;
    int64_t n_far, n_near;
    int64_t E_V, E_T, E_B, E_D;     /* stored entries of leaf bases, transfers, B, D */
    double flops_per_col;           /* algorithmic flops per column of W: 2(2E_V+2E_T+E_B+E_D) */
    double bytes_fp64, bytes_fp32;  /* device bytes of the block store per precision (0 = not loaded) */
    double bytes_bf16x3;            /* device bytes of the split-BF16 store (0 = not loaded) */
    int32_t n_phases;               /* launches of one evaluation (excluding permutes) */
} hm_info_t;

/* Load the compressed representation (the output of the compression phase,
 * Section 3.1, stored in the order the evaluation visits it as the paper's
 * CDS format does, Section 3.2) from an HMC1 file (the inspector's
 * output: 128-byte little-endian header "HMC1", version 1, then the arrays of
 * hm_host_repr in its field order) onto HIP device `device`, keeping the
 * precisions in prec_mask (HM_PRECBIT(HM_PREC_FP64) | ...).  The file is
 * parsed and validated on the host first: HM_ERR_FORMAT for a bad magic,
 * version, size or inconsistent structure (nothing is allocated on the device
 * then).  On success *out owns the device copy. */
hm_status hm_load_compressed(const char *path, int device, unsigned prec_mask, hm_matrix *out);

/* Same, from host arrays (copied; the caller may free them on return). */
hm_status hm_load_compressed_mem(const hm_host_repr *repr, int device, unsigned prec_mask,
                                 hm_matrix *out);

/* Sizes and algorithmic cost of a loaded matrix. */
hm_status hm_info(hm_matrix h, hm_info_t *out);

/* Release the device copy and workspaces.  NULL is accepted.  The caller must
 * make sure no enqueued hm_eval on h is still running. */
hm_status hm_free(hm_matrix h);

/* The evaluation phase (Section 2.1 "Evaluation"): Y = K~ W for Q columns on
 * `stream` (a hipStream_t, NULL = null stream), by the tree loops (up pass
 * with the bases, down pass) and the reduction loops (far blocks B, near
 * blocks D) of the paper, as one persistent task-graph launch.
 * dtype must be HM_F64 with HM_PREC_FP64 or HM_PREC_BF16X3, HM_F32 with HM_PREC_FP32; the
 * precision must have been loaded.  flags: HM_TREE_ORDER, HM_PROFILE, and
 * HM_NEAR_FROM_POINTS and HM_FAR_FROM_POINTS (HM_PREC_FP64 with points set by
 * hm_set_points, in the task-graph launch; the far flag also needs the
 * skeletons loaded with the representation; HM_ERR_INVALID otherwise).  Q = 0 is a valid no-op.  Workspaces grow
 * on demand (the first call at a larger Q allocates).  Calls on the same h
 * must be serialized by the caller (they share workspaces). */
hm_status hm_eval(hm_matrix h, const void *W, int64_t ldw, void *Y, int64_t ldy, int64_t Q,
                  hm_dtype dtype, hm_prec prec, unsigned flags, void *stream);

/* Bytes of the fixed device array behind hm_eval_noalloc (64 MiB per device). */
#define HM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results (bitwise) and asynchrony as hm_eval, but the
 * per-call device memory (W in tree order, the skeleton weights and
 * potentials, their split-BF16 copies, the dependency counters and the
 * launch descriptor) comes from one fixed array of HM_NOALLOC_SCRATCH_BYTES
 * in device memory, which each device the library runs on holds until the
 * process ends.  The call makes no hipMalloc, hipFree or other allocating
 * call and no host-device copy: it enqueues kernels only.
 *   - Limit: an evaluation that needs more than HM_NOALLOC_SCRATCH_BYTES
 *     (about N*Q'*s + 2*R*Q'*s bytes, with Q' = Q rounded up to the column
 *     tile, s the element size and R the total skeleton rank; the split
 *     copies add 4 bytes a value) returns HM_ERR_INVALID and launches nothing.
 *   - The task graph of the evaluation (per column-tile count, element type
 *     and precision) must already exist: one hm_eval on h with the same
 *     dtype, precision and a Q in the same column-tile class builds it.
 *     HM_ERR_INVALID otherwise (and after it has been evicted: a matrix keeps
 *     the 16 most recent graphs per element type).
 *   - flags: HM_TREE_ORDER, HM_NEAR_FROM_POINTS, HM_FAR_FROM_POINTS as for
 *     hm_eval; HM_LEVEL_LAUNCHES and HM_PROFILE return HM_ERR_INVALID.
 *   - Every call on one device shares that device's array and leaves its
 *     contents behind (each call initialises what it reads).  Calls that
 *     overlap on one device race, whatever their matrices and streams: the
 *     caller serializes them (one stream, or events).  An expired dependency
 *     wait is reported by hm_check(h), as for hm_eval. */
hm_status hm_eval_noalloc(hm_matrix h, const void *W, int64_t ldw, void *Y, int64_t ldy, int64_t Q,
                          hm_dtype dtype, hm_prec prec, unsigned flags, void *stream);

/* Matrix-free blocks (Section 2.1: a near block is the kernel matrix of
 * two leaves, K(X[I_a], X[I_b])).  Copies the N points (row i at X + i*ldx,
 * d coordinates, FP64, the caller's original point order, host memory) to the
 * device in tree order, with the kernel that the representation was
 * compressed with: kernel 0 is exp(-|x-y|^2 / (2 h^2)), kernel 1 is
 * exp(-|x-y| / h).  An hm_eval with HM_NEAR_FROM_POINTS then evaluates every
 * near block from the points inside its product tiles instead of reading it
 * from the device store.  When the representation was loaded with its
 * skeletons, the skeleton points are copied too (in the order of the
 * skeleton rows), and HM_FAR_FROM_POINTS computes every far block B_ab =
 * K(X[skel_a], X[skel_b]) (Section 2.1: the coupling block of an ID-based H2
 * matrix is the kernel matrix of the two skeletons) the same way.  Requires 1 <= d <= 64
 * (up to 15 the product tiles keep their points in LDS, above they read them
 * from global memory), ldx >= d, h > 0 (HM_ERR_INVALID otherwise).  Calling it again replaces the
 * points; they are freed with the matrix.  The caller may free X on return.
 * d, kernel and h must equal the representation's metadata (d, kernel, h of
 * hm_host_repr or the HMC1 header) when it states them (d > 0, h > 0):
 * HM_ERR_INVALID otherwise, and the points are not replaced.  The point
 * coordinates themselves cannot be checked: other points of that shape give
 * the near field of other points.  On any error the previous points stay in
 * place. */
hm_status hm_set_points(hm_matrix h, const double *X, int64_t ldx, int64_t d, int kernel, double h_param);

/* Synchronize the device and report whether any evaluation on h since the
 * last check hit the bounded dependency wait of the persistent launch
 * (HM_ERR_INTERNAL: those results are invalid; the launch itself always
 * terminates).  HM_OK otherwise. */
hm_status hm_check(hm_matrix h);

/* Per-phase timings of evaluations run with HM_PROFILE since the last reset:
 * for phase i (0 permute-in, 1 up pass, 2 down pass (far reduction and
 * transfers), 3 leaf pass (near field and leaf basis), 4 permute-out) writes the
 * summed milliseconds to ms[i] and the number of launches to launches[i].
 * Synchronizes with the recorded events. */
hm_status hm_profile_read(hm_matrix h, double ms[5], int64_t launches[5]);
hm_status hm_profile_reset(hm_matrix h);

/* ---------------------------------------------------------------------------
 * Batched evaluation: many matrices of uneven size, rank and width evaluated
 * by one persistent task-graph launch.  Their dependency graphs are merged
 * into one queue, ordered together by list scheduling, so that the small
 * matrices' tree passes and the large ones' near fields share the machine.
 * A batch fixes its matrices, their widths Q[i], dtype and precision; it owns
 * its workspaces (so it never disturbs hm_eval on the same matrices), runs on
 * a private stream joined to the caller's stream by events, and replays one
 * captured HIP graph (batched permute-in, graph launch, batched permute-out)
 * per evaluation.  With HM_BATCH_AUTOTUNE the column tile is chosen by timing
 * every candidate (32, 64, 128, 256) on the batch itself at creation. */
typedef struct hm_batch_s *hm_batch;
#define HM_BATCH_AUTOTUNE 1u   /* time the candidate column tiles and keep the fastest */
#define HM_BATCH_NO_GRAPH 2u   /* enqueue the launches directly instead of a captured graph */
/* Fix the column tile (16, 32, 64, 128 or 256) instead of taking the default
 * or the autotuner's (not together with HM_BATCH_AUTOTUNE).  With 256, each
 * matrix's last columns run in a tile no wider than they need (the smallest
 * power of two, at least 16, that holds them); so does the default or tuned
 * tile when it is 256. */
#define HM_BATCH_TILE(bn) ((unsigned)(bn) << 8)

typedef struct {
    int32_t n, column_tile, n_tasks, workgroups;
    double flops;             /* algorithmic flops of one batched evaluation */
    double tuned_ms[5];       /* autotuner timing per tile 16, 32, 64, 128, 256 (0 = not tried) */
    double workspace_bytes;
} hm_batch_info_t;

/* Create a batch of n matrices (same device, precision loaded) with widths Q
 * (1 <= Q[i] <= 2^24).  Synchronizes the device while it builds the plan. */
hm_status hm_batch_create(int n, const hm_matrix *hs, const int64_t *Q, hm_dtype dtype,
                          hm_prec prec, unsigned flags, hm_batch *out);
/* Y[i] = K~_i W[i] for every matrix of the batch (device pointers, row-major,
 * leading dimensions ldw[i], ldy[i] >= Q[i]); asynchronous on `stream`.
 * Evaluations of one batch are serialized on its private stream. */
hm_status hm_batch_eval(hm_batch b, const void *const *W, const int64_t *ldw, void *const *Y,
                        const int64_t *ldy, void *stream);
hm_status hm_batch_info(hm_batch b, hm_batch_info_t *out);
/* Wait for the batch's stream; HM_ERR_INTERNAL if a bounded wait expired. */
hm_status hm_batch_check(hm_batch b);
hm_status hm_batch_free(hm_batch b);
/* One-shot form: create, evaluate, wait, free. */
hm_status hm_eval_batched(int n, const hm_matrix *hs, const void *const *W, const int64_t *ldw,
                          void *const *Y, const int64_t *ldy, const int64_t *Q, hm_dtype dtype,
                          hm_prec prec, void *stream);

/* ---------------------------------------------------------------------------
 * Serving (no section of the paper: the served form of the evaluation of
 * Section 2.1): several compressed matrices resident in HBM, requests of any
 * width Q in [1, 1024] submitted without blocking and served by continuous
 * batching.  A server thread owns max_slots slots; a slot is a stream with
 * its own workspaces, sized when matrices are added for the largest of them
 * at 1024 columns.  Whenever a slot is free and the HBM budget allows it, the
 * pending requests of the next matrix (round robin) are coalesced
 * column-wise into one sweep of up to 1024 columns: gathered from each
 * request's W, evaluated by one persistent task-graph launch, scattered into
 * each request's Y.  Requests that arrive while sweeps run join the next
 * sweep a free slot takes, also for a matrix that already has a sweep in
 * flight, so sweeps of one or several matrices overlap on the device.  A
 * result is bitwise the same alone and in the mix (column j of Y depends only
 * on column j of W).  Add every matrix before submitting work; the matrices
 * must outlive the server.  The server never touches a matrix's own
 * workspaces, but it shares its store: do not free it while the server runs.
 * Calls are thread-safe. */
typedef struct hm_server_s *hm_server;
typedef uint64_t hm_ticket;

typedef struct {
    int64_t completed, failed, sweeps, columns, pending;
    int32_t inflight, peak_inflight;   /* sweeps on the device now / at most at once */
    double peak_bytes;        /* largest sum of 2 N Q x element size over the sweeps in flight */
} hm_server_stats_t;

/* max_slots: sweeps in flight at once (1..16); hbm_budget: bound on the
 * working set of the sweeps in flight, counted as 2 N Q x element size per
 * sweep (its columns of W and Y); a sweep waits until it fits.  dtype/prec as
 * for hm_eval (FP64 or FP32).  Creates the slots' streams and a server
 * thread. */
hm_status hm_server_create(int device, size_t hbm_budget, int max_slots, hm_dtype dtype,
                           hm_prec prec, hm_server *out);
/* Make h resident: builds its launch plans for every sweep width and grows
 * the slots' workspaces and counters to fit it (so that sweeps never plan,
 * allocate or upload); *mat_id names it in hm_submit.  HM_ERR_BUSY while
 * sweeps are running. */
hm_status hm_server_add(hm_server s, hm_matrix h, int *mat_id);
/* Queue Y = K~ W for matrix mat_id (device pointers, N x Q row-major in the
 * caller's point order; they must stay valid until hm_poll reports done).
 * The request is ordered after the work enqueued on `stream` (a hipStream_t;
 * NULL = the null stream) before this call: an event recorded there is
 * waited for before the sweep reads W or writes Y.  Never blocks on the GPU;
 * HM_ERR_BUSY when the request alone exceeds the budget or too many requests
 * are queued. */
hm_status hm_submit(hm_server s, int mat_id, const void *W, int64_t ldw, void *Y, int64_t ldy,
                    int64_t Q, void *stream, hm_ticket *out);
/* *done = 1 once Y is written (then *latency_us = submit-to-completion time
 * and the ticket is retired); *done = 0 while pending.  HM_ERR_INVALID for an
 * unknown or retired ticket; HM_ERR_INTERNAL (ticket retired) when the
 * sweep's launch hit its bounded dependency wait, so Y is invalid;
 * HM_ERR_DEVICE when a HIP call of the sweep failed. */
hm_status hm_poll(hm_server s, hm_ticket t, int *done, double *latency_us);
hm_status hm_server_stats(hm_server s, hm_server_stats_t *out);
/* Stop the server thread and wait for the sweeps in flight; queued requests
 * that never started are dropped. */
hm_status hm_server_destroy(hm_server s);

/* ---------------------------------------------------------------------------
 * Inspector: host-side compression of a point set into the representation
 * above (the compression phase of the paper, Section 3.1: tree construction,
 * interaction computation, sampling, ID low-rank approximation).  Runs on the
 * host CPU threads; its output feeds hm_load_compressed_mem.  Readings of the
 * steps the paper leaves open: a perfect binary tree cut at the median of the
 * widest coordinate (or, with partitioner 1, along the direction between the
 * two means of Lloyd's 2-means of the node's points: Section 3.1 two-means
 * partitioning); far iff tau * centroid distance > diam(a) + diam(b)
 * (diam = twice the largest distance to the centroid), or every off-diagonal
 * pair for HSS, or the budget rule below (Section 4.1); ID rows = the whole far field when it has at most sample_rows
 * points, otherwise half from the nearest far clusters and half by a seeded
 * SplitMix64 key; pivoted-QR ID with rank = first j with |R_jj| <= tol |R_11|,
 * capped at max_rank. */
typedef struct {
    int32_t kernel;         /* 0: exp(-|x-y|^2 / (2 h^2)), 1: exp(-|x-y| / h) */
    double h;               /* bandwidth (> 0) */
    int32_t leaf_size;      /* m >= 2: leaves hold at most m points */
    double tol;             /* ID tolerance relative to |R_11| (>= 0) */
    int32_t max_rank;       /* rank cap */
    int32_t admissibility;  /* 0 distance (uses tau), 1 HSS, 2 budget (uses budget; H^2-b) */
    double tau;
    int64_t sample_rows;    /* row-sample cap S of each ID */
    uint64_t seed;          /* sample seed */
    int32_t threads;        /* host threads (0 = all hardware threads) */
    int32_t partitioner;    /* 0 median of the widest coordinate, 1 two-means direction (d > 3) */
    double budget;          /* admissibility 2: each leaf is near itself and its
                               floor(budget * #leaves) nearest leaves by centroid distance
                               (symmetrized); two nodes are far iff no leaf below one is near a
                               leaf below the other.  0.03 is the paper's H^2-b, 0 gives HSS */
} hm_compress_opts;

typedef struct hm_repr_s *hm_repr;  /* library-owned host representation */

/* Compress X (N x d, row-major FP64, host memory, read only during the call).
 * HM_ERR_INVALID for bad options or non-finite coordinates. */
hm_status hm_compress(const double *X, int64_t N, int64_t d, const hm_compress_opts *opts,
                      hm_repr *out);
/* Fill *view with pointers into r (valid until hm_repr_free(r)). */
hm_status hm_repr_view(hm_repr r, hm_host_repr *view);
/* Write r as an HMC1 file (the format hm_load_compressed reads). */
hm_status hm_repr_write(hm_repr r, const char *path);
/* Release r (NULL accepted). */
hm_status hm_repr_free(hm_repr r);

/* ---------------------------------------------------------------------------
 * Reusing inspection (Section 5 "Reusing Inspection"): the compression is
 * split in two phases.  inspector-p1 holds what depends on the points and
 * the admissibility condition only (tree, interaction lists, row sampling);
 * inspector-p2 holds what depends on the kernel function and the accuracy
 * (the low-rank approximation of every node and the blocks).  When the
 * kernel, its bandwidth or the accuracy change, only p2 runs again, on the
 * p1 output kept from before.  Here p1 runs on the host and p2 on the GPU. */
typedef struct hm_structure_s *hm_structure;  /* library-owned inspector-p1 output */

typedef struct {
    int64_t N, d;
    int32_t n_nodes, depth;
    int64_t n_far, n_near;
    int64_t rows_total;  /* row-sample entries over all nodes */
} hm_structure_info_t;

/* inspector-p1 on the host: the tree, the far and near lists and every
 * node's row sample, with the same readings as hm_compress (fields used:
 * leaf_size, admissibility, tau, sample_rows, seed, threads; the kernel,
 * h, tol and max_rank fields are ignored).  X is N x d row-major FP64 host
 * memory, copied (the caller may free it on return).  HM_ERR_INVALID for bad
 * options or non-finite coordinates. */
hm_status hm_inspect_p1(const double *X, int64_t N, int64_t d, const hm_compress_opts *opts,
                        hm_structure *out);
hm_status hm_structure_info(hm_structure s, hm_structure_info_t *out);
/* Row sample of one node: original point indices in tree order.  *count
 * receives its length; rows (may be NULL) receives the entries when
 * cap >= *count (HM_ERR_INVALID otherwise). */
hm_status hm_structure_rows(hm_structure s, int32_t node, int64_t *rows, int64_t cap, int64_t *count);
hm_status hm_structure_free(hm_structure s);

/* inspector-p2 on GPU `device` (Section 3.1 low-rank approximation by
 * interpolative decomposition, Section 5 reuse): for every node, deepest
 * level first, the kernel block A = K(X[rows], X[candidates]) of its row
 * sample and its candidate columns (a leaf's points, or its children's
 * skeletons) is formed on the device, its Gram matrix A^T A is taken on the
 * matrix cores, and a pivoted partial Cholesky of the Gram matrix gives the
 * pivots and the triangular factor of a column-pivoted QR of A (the same
 * pivots and |R_jj| in exact arithmetic).  The rank is the first j with
 * R_jj <= tol * R_11, capped at max_rank; the interpolation matrix is
 * [I, R11^-1 R12] in pivot order.  The far blocks B_ab = K(X[skel_a],
 * X[skel_b]) and the near blocks D_ab = K(X[I_a], X[I_b]) are generated on
 * the device.  The result is a host representation (with its skeletons) for
 * hm_load_compressed_mem or hm_repr_write.  kernel 0 is
 * exp(-|x-y|^2 / (2 h^2)), 1 is exp(-|x-y| / h); h > 0, tol >= 0,
 * 1 <= max_rank <= 1024 and leaves of at most 2048 points (HM_ERR_INVALID
 * otherwise).  Synchronous; the structure is only read and may be reused by
 * any number of p2 runs. */
hm_status hm_inspect_p2(hm_structure s, int device, int32_t kernel, double h, double tol, int32_t max_rank,
                        hm_repr *out);

/* inspector-p2 straight into a device matrix: the same IDs as hm_inspect_p2,
 * then the device store of hm_load_compressed_mem built on `device` with
 * prec_mask (same meaning and checks), its far and near blocks generated in
 * the store from the points instead of being copied through the host (the
 * data layout construction of Section 3.2 done on the device).  Results of
 * hm_eval on it equal those on hm_load_compressed_mem(hm_inspect_p2(...))
 * bitwise.  With HM_LOAD_NO_NEAR_BLOCKS / HM_LOAD_NO_FAR_BLOCKS the blocks
 * are not generated; hm_set_points with the same points, kernel and h then
 * enables HM_NEAR_FROM_POINTS / HM_FAR_FROM_POINTS. */
hm_status hm_inspect_p2_load(hm_structure s, int device, int32_t kernel, double h, double tol, int32_t max_rank,
                             unsigned prec_mask, hm_matrix *out);

/* Message for the last non-OK status returned on this thread. */
const char *hm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HM_H */
