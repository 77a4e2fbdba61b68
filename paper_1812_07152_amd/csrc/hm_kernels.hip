// hm_kernels.hip -- HIP kernels of the evaluation Y = K~ W for gfx950.
//
// Every step of the evaluation (Section 2.1 "Evaluation": the bottom-up V
// loop, the reduction over the far blocks B, the top-down U loop and the
// reduction over the near blocks D) is a set of small dense products
//     out_block (M x Q) = sum_s A_s (M x K_s) * B_s (K_s x Q)
// with A_s a stored block and B_s a row range of a workspace.  The persistent
// task-graph kernel k_persistent runs all of them in one launch (per-level
// launches of k_block_products remain as an alternative): one workgroup per
// (output block, column tile) accumulates all of its segments in registers
// and writes its block once (a single writer per output row block, as in the
// paper's blocking, Section 3.2, so no atomics are needed and results are
// deterministic).
//
// Tiling: a BM x BN output tile per workgroup, split over WAVES_M x WAVES_N
// wave64s, each wave owning (BM/WAVES_M) x (BN/WAVES_N) = FM x FN MFMA
// 16x16 fragments.  The contraction runs in chunks of BK = 16 rows (32 for
// split BF16).  FP64 and split-BF16 tiles of the persistent kernel load their
// chunks straight into LDS (global_load_lds_dwordx4) with up to three stages
// (product_loop_f64_dma, product_loop_bf16x3); FP32 tiles and the per-level
// kernel stage 16-byte loads through registers into one of two LDS buffers
// (product_loop).  One barrier per chunk.  Lane mapping of the 16x16x4
// MFMAs (checked on the device): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l holds D[4r + l/16][l%16]
// for FP64 and D[4(l/16) + r][l%16] for FP32.
#include <algorithm>

#include "hm_internal.h"

namespace hm {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
// 16-byte staging vectors as native clang vectors (the HIP double2/float4
// wrapper structs keep register arrays of them in scratch memory)
typedef double d2_t __attribute__((ext_vector_type(2)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef d4_t acc_t;
    typedef d2_t vec_t;  // 16 bytes
    static constexpr int kVec = 2;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

template <>
struct Mfma<float> {
    typedef f4_t acc_t;
    typedef f4_t vec_t;
    static constexpr int kVec = 4;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Loads of the block store and the workspaces go through global (address
// space 1) pointers.  The persistent launch reads its buffer addresses from a
// descriptor in memory, so the compiler cannot infer their address space and
// would emit flat loads; a flat load also counts against the LDS wait
// counter, so the wait for the LDS reads of the current chunk would wait for
// the global loads of the next one as well.
template <typename V>
__device__ __forceinline__ V load_global(const void *p) {
    return *(const __attribute__((address_space(1))) V *)p;
}

__device__ __forceinline__ Seg load_seg(const Seg *p) {
    const __attribute__((address_space(1))) Seg *g = (const __attribute__((address_space(1))) Seg *)p;
    Seg s;
    s.a_off = g->a_off;
    s.b_row = g->b_row;
    s.lda = g->lda;
    s.K = g->K;
    s.b_buf = g->b_buf;
    s.Kpad = g->Kpad;
    s.a_off16 = g->a_off16;
    s.b_row16 = g->b_row16;
    s.trans = g->trans;
    s.tstride = g->tstride;
    return s;
}

// One direct global-to-LDS load: the 64 lanes' 16-byte vectors at src land
// in 1 KB of LDS from the wave-uniform address lds_addr, lane l at
// lds_addr + 16 l.  Written as inline asm so that the compiler does not track
// these LDS writes: it would otherwise wait for every outstanding one before
// any LDS read, including the reads of the stage already complete; the
// chunk pipeline below waits for them itself (wait_vm_barrier).
__device__ __forceinline__ void load_lds16(const void *src, const char *lds_dst) {
    const uint32_t a = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char *)lds_dst;
    asm volatile("global_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(__builtin_amdgcn_readfirstlane(a))
                 : "memory");
}

// Segment descriptor through a scalar (constant address space) load: it
// counts against the scalar counter, so the compiler's wait for it never
// covers the chunk loads in flight.  The descriptors are read-only during a
// launch and the address is uniform.
__device__ __forceinline__ Seg load_seg_scalar(const Seg *p) {
    const __attribute__((address_space(4))) Seg *g = (const __attribute__((address_space(4))) Seg *)p;
    Seg s;
    s.a_off = g->a_off;
    s.b_row = g->b_row;
    s.lda = g->lda;
    s.K = g->K;
    s.b_buf = g->b_buf;
    s.Kpad = g->Kpad;
    s.a_off16 = g->a_off16;
    s.b_row16 = g->b_row16;
    s.from_pts = g->from_pts;
    s.trans = g->trans;
    s.tstride = g->tstride;
    s.pad_ = 0;
    return s;
}

// Waits until at most N of this wave's vector memory operations are
// outstanding, then joins the workgroup barrier.  No fence: the barrier of
// __syncthreads() also waits for every outstanding load, which would drain
// the loads that are meant to stay in flight across it.  The direct
// global-to-LDS writes of a chunk are complete once the counter covers them.
template <int N>
__device__ __forceinline__ void wait_vm_barrier() {
    static_assert(N >= 0 && N < 64, "vmcnt out of range");
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef short s16x8_t __attribute__((ext_vector_type(8)));

// v ~= hi + lo with hi = bf16(v) and lo = bf16(v - hi), from the FP32 value.
__device__ __forceinline__ void split_bf16(float f, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)f;
    lo = (__bf16)(f - (float)hi);
}

constexpr int kBK = 16;
// LDS rows are padded by 128 bytes so that the four 16-lane groups of a
// fragment read land on alternating bank halves.
template <typename T>
constexpr int lds_pad() { return 128 / (int)sizeof(T); }

// Invariants the host guarantees (so that no load needs a bounds check and
// the compiler never has to wait for a load before the MFMAs of the current
// chunk):
//   - every stored A block has Kpad = round_up(K, 16) rows (zero beyond K) and
//     the store has slack after its last block for the row over-read of a
//     tile taller than the block;
//   - workspaces have leading dimension ldq, a multiple of BN.

// One output block of a task as the tile code sees it.  With Y set, the
// block's rows are rows perm[out_row + row] (perm null: out_row + row) of the
// caller's Y (leading dimension ldy, first Q columns) instead of rows of the
// output workspace.
struct TileJob {
    int64_t out_row;
    int32_t out_buf, M, m0, seg_begin, seg_end, accumulate;
    void *Y = nullptr;
    int64_t ldy = 0, Q = 0;
    const int64_t *perm = nullptr;
    // split-BF16 copy of the block (mixed precision): rows out16 + r of the
    // split workspace Y16; out_split 2: the copy only (no FP64 output)
    void *Y16 = nullptr;
    int64_t out16 = -1;
    int32_t out_split = 0;
};

// Fragment grid of a BM x BN tile over WAVES_M x WAVES_N waves.
template <int BM, int BN, int WAVES_M, int WAVES_N>
struct Tile {
    static constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
    static constexpr int FM = WM / 16, FN = WN / 16;
};

// Row of accumulator register r of lane l within a 16 x 16 fragment:
// 4r + l/16 (FP64 MFMA) or 4(l/16) + r (FP32 accumulation, and FP64 with
// permuted A rows, see product_loop).
template <bool F32_ROWS>
__device__ __forceinline__ int frag_row(int lane, int r) {
    return F32_ROWS ? 4 * (lane >> 4) + r : 4 * r + (lane >> 4);
}

// Accumulates rows [m0, m0 + BM) x columns [n0, n0 + BN) of
//   sum over segments [sb, se) of A_s (K-major in the store) * B_s rows
// into acc.  NT threads take part in loads and barriers; the first
// WAVES_M * WAVES_N waves own FM x FN MFMA fragments each.  As/Bs are LDS
// buffers of 2 x kBK x (BM + pad) and 2 x kBK x (BN + pad) elements.
// ROWPERM (FP64 only): fragment row x reads A row 4(x % 4) + x / 4, which
// puts the FP64 accumulators in the FP32 register layout (frag_row<true>),
// so that a product can continue from FP32 partial sums.
// SYM: the loop may meet mirror blocks of a symmetric store (Seg::trans); a
// separate instantiation, so that the loops of full stores keep their
// registers and code.
template <typename T, int BM, int BN, int WAVES_M, int WAVES_N, int NT, bool ROWPERM = false, bool SYM = false>
__device__ __forceinline__ void product_loop(
    const Seg *__restrict__ segs, int sb, int se, int m0, const T *__restrict__ store, T *buf0, T *buf1,
    T *buf2, T *buf3, int64_t ldq, int64_t n0, T *As_, T *Bs_,
    typename Mfma<T>::acc_t (&acc)[Tile<BM, BN, WAVES_M, WAVES_N>::FM][Tile<BM, BN, WAVES_M, WAVES_N>::FN]) {
    using M_ = Mfma<T>;
    using vec_t = typename M_::vec_t;
    constexpr int WM = Tile<BM, BN, WAVES_M, WAVES_N>::WM, WN = Tile<BM, BN, WAVES_M, WAVES_N>::WN;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int VEC = M_::kVec;
    constexpr int A_ROWV = BM / VEC, B_ROWV = BN / VEC;        // vectors per chunk row
    constexpr int A_VECS = kBK * A_ROWV, B_VECS = kBK * B_ROWV;
    constexpr int A_PER = (A_VECS + NT - 1) / NT, B_PER = (B_VECS + NT - 1) / NT;
    constexpr int LA = BM + lds_pad<T>(), LB = BN + lds_pad<T>();
    static_assert(FM >= 1 && FN >= 1 && WM % 16 == 0 && WN % 16 == 0, "bad tile");
    static_assert(64 * WAVES_M * WAVES_N <= NT, "too few threads");
    T(*As)[kBK][LA] = reinterpret_cast<T(*)[kBK][LA]>(As_);
    T(*Bs)[kBK][LB] = reinterpret_cast<T(*)[kBK][LB]>(Bs_);

    // (the thread index is not made opaque here: hoisting this loop's
    // per-thread offsets out of the task loop pays for the FP32 tiles)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool computes = wave < WAVES_M * WAVES_N;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    const int arow = ROWPERM ? 4 * (lane & 3) + ((lane >> 2) & 3) : (lane & 15);
    // buffer select without a dynamically indexed private array
    auto bufp = [&](int b) { return b == 0 ? buf0 : b == 1 ? buf1 : b == 2 ? buf2 : buf3; };

    vec_t ra[A_PER], rb[B_PER];

    // Global -> registers for the chunk at contraction row kk of segment sg.
    // Unconditional loads: thread slots beyond the chunk re-load its last
    // vector, B rows beyond K re-load row K-1 (multiplied by zero rows of A).
    auto load = [&](const Seg &sg, int kk) {
        const T *Bp = bufp(sg.b_buf) + (sg.b_row) * ldq + n0;
        if (SYM && sg.trans) {  // mirror block: the VEC rows of a vector sit tstride apart
            const T *A = store + sg.a_off + (int64_t)m0 * sg.tstride + kk;
            int mt = tid;  // opaque: these offsets are not hoisted out of the task loop
            asm volatile("" : "+v"(mt));
#pragma unroll
            for (int u = 0; u < A_PER; u++) {
                const int idx = min(mt + u * NT, A_VECS - 1);
                const int kr = idx / A_ROWV, c = (idx % A_ROWV) * VEC;
#pragma unroll
                for (int v = 0; v < VEC; v++) ra[u][v] = load_global<T>(A + (int64_t)(c + v) * sg.tstride + kr);
            }
        } else {
            const T *A = store + sg.a_off + m0 + (int64_t)kk * sg.lda;
#pragma unroll
            for (int u = 0; u < A_PER; u++) {
                const int idx = min(tid + u * NT, A_VECS - 1);
                const int kr = idx / A_ROWV, c = (idx % A_ROWV) * VEC;
                ra[u] = load_global<vec_t>(A + (int64_t)kr * sg.lda + c);
            }
        }
#pragma unroll
        for (int u = 0; u < B_PER; u++) {
            const int idx = min(tid + u * NT, B_VECS - 1);
            const int kr = min(kk + idx / B_ROWV, sg.K - 1), c = (idx % B_ROWV) * VEC;
            rb[u] = load_global<vec_t>(Bp + (int64_t)kr * ldq + c);
        }
    };
    auto stash = [&](int b) {
#pragma unroll
        for (int u = 0; u < A_PER; u++) {
            const int idx = tid + u * NT;
            if (A_VECS % NT == 0 || idx < A_VECS)
                *reinterpret_cast<vec_t *>(&As[b][idx / A_ROWV][(idx % A_ROWV) * VEC]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < B_PER; u++) {
            const int idx = tid + u * NT;
            if (B_VECS % NT == 0 || idx < B_VECS)
                *reinterpret_cast<vec_t *>(&Bs[b][idx / B_ROWV][(idx % B_ROWV) * VEC]) = rb[u];
        }
    };
    auto compute = [&](int b) {
#pragma unroll
        for (int ks = 0; ks < kBK; ks += 4) {
            T af[FM], bf[FN];
            const int kr = ks + (lane >> 4);
#pragma unroll
            for (int i = 0; i < FM; i++) af[i] = As[b][kr][wm * WM + i * 16 + arow];
#pragma unroll
            for (int j = 0; j < FN; j++) bf[j] = Bs[b][kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < FM; i++)
#pragma unroll
                for (int j = 0; j < FN; j++) acc[i][j] = M_::mma(af[i], bf[j], acc[i][j]);
        }
    };

    if (sb < se) {
        int s = sb, kk = 0, b = 0;
        Seg sg = load_seg(segs + s);
        load(sg, 0);
        stash(0);
        __syncthreads();
        while (true) {
            int nkk = kk + kBK, ns = s;
            Seg nsg = sg;
            if (nkk >= sg.Kpad) {
                ns = s + 1;
                nkk = 0;
                if (ns < se) nsg = load_seg(segs + ns);
            }
            const bool more = ns < se;
            load(nsg, more ? nkk : kk);  // on the last chunk: a harmless re-load
            if (computes) compute(b);
            stash(b ^ 1);
            __syncthreads();
            if (!more) break;
            s = ns;
            kk = nkk;
            sg = nsg;
            b ^= 1;
        }
    }
}

// FP64 products in the persistent launch: the same loop as product_loop, fed
// by direct global-to-LDS loads (see product_loop_bf16x3 for the pipeline
// and its waits).  A stage holds the chunk's 16 contraction rows of A (BM
// values each) and then of B (BN values each), K-major and unpadded.  An
// MFMA operand read takes 16 consecutive values of one row per 16 lanes, and
// two 16-lane groups (rows kr and kr + 1) share an LDS cycle; where a row is
// an even number of 128-byte halves long, odd rows are stored with their
// 16-byte slots permuted by slot ^ 8 (their halves swapped within each
// 256 bytes), so the two groups fall on different bank halves.  STAGES 3
// keeps two chunks in flight; STAGES 2 (one) fits two workgroups per compute
// unit at 128 columns.
template <int BN, bool ROWPERM>
constexpr int f64_stages() {
    return (BN == 128 && !ROWPERM) ? 2 : 3;
}
template <int BM, int BN, bool ROWPERM>
constexpr int f64_lds_bytes() {
    return f64_stages<BN, ROWPERM>() * (BM + BN) * kBK * 8;
}
// The largest f64_lds_bytes<128, W, false> over the widths W = BN, BN / 2,
// ... 16 of a launch with narrow tiles (a narrower tile can take more stages:
// 64 columns three, 128 columns two).
template <int BN>
constexpr int f64_lds_bytes_narrow() {
    int most = 0;
    for (int w = BN; w >= 16; w /= 2) {
        const int b = ((w == 128) ? 2 : 3) * (128 + w) * kBK * 8;
        most = b > most ? b : most;
    }
    return most;
}

// Blocks computed from points (matrix-free near and far field): with pts
// set, a segment whose from_pts equals kind has the A block K(x_a, x_b): x_a
// the points of the tile's rows (pts rows a_row.., m_valid rows in this
// tile), x_b those of the B operand's rows (pts rows b_row..).  kind 1: a
// leaf tile's near blocks, pts the points in tree order; kind 2: a down-pass
// tile's far blocks, pts the skeleton points in Ŵ row order.  xa: LDS for
// the tile's points (d x 128, coordinate-major), used when d <= kMaxPointDim.
struct NearGen {
    const double *pts = nullptr;  // rows x d
    int kind = 0;
    int d = 0;
    int kern = 0;                 // 0: exp(-r^2 kscale), 1: exp(-r kscale)
    double kscale = 0;
    int64_t a_row = 0;
    int m_valid = 0;
    char *xa = nullptr;
};
constexpr int kPointLds = 128 * kMaxPointDim * 8;  // the tile's points, BM <= 128

template <int BM, int BN, int WAVES_M, int WAVES_N, int NT, bool ROWPERM, bool SYM = false>
__device__ __forceinline__ void product_loop_f64_dma(
    const Seg *__restrict__ segs, int sb, int se, int m0, const double *__restrict__ store, double *buf0,
    double *buf1, double *buf2, double *buf3, int64_t ldq, int64_t n0, char *lds,
    d4_t (&acc)[Tile<BM, BN, WAVES_M, WAVES_N>::FM][Tile<BM, BN, WAVES_M, WAVES_N>::FN],
    NearGen ng = NearGen()) {
    constexpr int WM = Tile<BM, BN, WAVES_M, WAVES_N>::WM, WN = Tile<BM, BN, WAVES_M, WAVES_N>::WN;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int STAGES = f64_stages<BN, ROWPERM>();
    constexpr int kStage = (BM + BN) * kBK * 8;
    constexpr int A_BLOCKS = BM / 8;             // 1 KB blocks (64 slots of 2 values) of A
    constexpr int BLOCKS = (BM + BN) / 8;        // A then B
    constexpr int PER_WAVE = (BLOCKS + 7) / 8;   // loads per wave and chunk
    // slot permutation of odd rows (see above), where a row is an even number
    // of 128-byte halves and a wave's fragments along it are an even number
    // (so that a fragment's half is known at compile time); else none
    constexpr int SWA = ((BM / 16) % 2 == 0 && FM % 2 == 0) ? 8 : 0;
    constexpr int SWB = ((BN / 16) % 2 == 0 && FN % 2 == 0) ? 8 : 0;
    static_assert(NT == 512, "8 waves fill a stage");
    static_assert(FM >= 1 && FN >= 1 && WM % 16 == 0 && WN % 16 == 0, "bad tile");
    static_assert(BLOCKS * 1024 == kStage, "stage size");

    int tid = threadIdx.x;  // opaque, see store_tile
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool computes = WAVES_M * WAVES_N == NT / 64 || wave < WAVES_M * WAVES_N;  // all waves: known at compile time
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    const int arow = ROWPERM ? 4 * (lane & 3) + ((lane >> 2) & 3) : (lane & 15);
    auto bufp = [&](int b) { return b == 0 ? buf0 : b == 1 ? buf1 : b == 2 ? buf2 : buf3; };

    // Chunk at contraction row kk of segment sg into stage st.  Slot t =
    // 64 q + lane of block q is (row kr, value pair p) of A or of B; B rows
    // past K re-load row K - 1 (multiplied by zero rows of A).
    const bool gen = ng.pts != nullptr;
    // A mirror block (sg.trans) holds a row's contraction values
    // contiguously, tstride apart from the next row's.  Its chunk goes into
    // the A part of the stage pair-major instead: 16-byte slot P = s BM + r
    // holds contraction values 2 s and 2 s + 1 of row r, one direct 16-byte
    // load per slot as for any other block, and compute() reads such a stage
    // with that layout (the 16 rows a 16-lane group reads at one contraction
    // index sit 16 bytes apart, its two halves 8: no bank conflicts).
    auto issue = [&](int st, const Seg &sg, int kk) -> bool {
        const double *A = store + sg.a_off + m0 + (int64_t)kk * sg.lda;
        const char *AT = reinterpret_cast<const char *>(store + sg.a_off + (int64_t)m0 * sg.tstride + kk);
        const double *Bp = bufp(sg.b_buf) + sg.b_row * ldq + n0;
        char *stage = lds + st * kStage;
        const bool make_a = gen && sg.from_pts == ng.kind;  // wave-uniform
        const bool mirror = SYM && sg.trans && !make_a;     // wave-uniform
#pragma unroll
        for (int u = 0; u < PER_WAVE; u++) {
            int q = min(u * 8 + wave, BLOCKS - 1);  // wave-uniform
            // an A block computed below: load a B block in its place (the
            // bytes its own load writes, to the same place), so that every
            // wave still issues PER_WAVE loads per chunk
            if (make_a && q < A_BLOCKS) q = A_BLOCKS + q % (BLOCKS - A_BLOCKS);
            if (mirror && q < A_BLOCKS) {
                // the lane index made opaque here: addresses computed per use,
                // not once per kernel and held through the task loop
                int ml = lane;
                asm volatile("" : "+v"(ml));
                const int t = q * 64 + ml, sp = t / BM, r = t % BM;
                load_lds16(AT + ((int64_t)r * sg.tstride + 2 * sp) * 8, stage + q * 1024);
                continue;
            }
            const double *src;
            if (q < A_BLOCKS) {
                const int t = q * 64 + lane, kr = t / (BM / 2), pr = (t % (BM / 2)) ^ ((kr & 1) ? SWA : 0);
                src = A + (int64_t)kr * sg.lda + 2 * pr;
            } else {
                const int t = (q - A_BLOCKS) * 64 + lane, kr = t / (BN / 2), pr = (t % (BN / 2)) ^ ((kr & 1) ? SWB : 0);
                src = Bp + (int64_t)min(kk + kr, sg.K - 1) * ldq + 2 * pr;
            }
            load_lds16(src, stage + q * 1024);
        }
        return mirror;
    };
    // The A block of a chunk of a segment made from points: A[k][m] =
    // K(x_a[m], x_b[kk + k]), zero past the segment's K rows and the tile's
    // rows.  Wave w takes rows w and w + 8 (x_b through scalar loads), lanes
    // take m: NV values a lane, value v is row kh = v / NJ, column block
    // j = v % NJ.  All NV values at once, coordinate by coordinate: the NV
    // distance sums, then the NV exponentials, are independent chains in one
    // basic block, so their latencies overlap (one value at a time, with a
    // branch per coordinate, ran about 20% slower).
    constexpr int NJ = (BM + 63) / 64, NV = 2 * NJ;
    auto make_dist = [&](const Seg &sg, int kk, double (&r2)[NV]) {
        const __attribute__((address_space(4))) double *P =
            (const __attribute__((address_space(4))) double *)ng.pts;
        const double *xa = reinterpret_cast<const double *>(ng.xa);
        const int kg0 = kk + wave, kg1 = kg0 + 8;
        const bool kv0 = kg0 < sg.K, kv1 = kg1 < sg.K;  // wave-uniform
        const int64_t r0 = (sg.b_row + kg0) * ng.d, r1 = (sg.b_row + kg1) * ng.d;
#pragma unroll
        for (int v = 0; v < NV; v++) r2[v] = 0.0;
        if (ng.d <= kMaxPointDim) {
#pragma unroll 4
            for (int t = 0; t < ng.d; t++) {
                const double xb0 = kv0 ? P[r0 + t] : 0.0, xb1 = kv1 ? P[r1 + t] : 0.0;
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const double df = xa[t * 128 + lane + 64 * (v % NJ)] - (v / NJ ? xb1 : xb0);
                    r2[v] = fma(df, df, r2[v]);
                }
            }
        } else {  // the tile's points from global memory (rows past m_valid read the last one)
            const double *xg = ng.pts + ng.a_row * ng.d;  // wave-uniform base
            int xo[NJ];
#pragma unroll
            for (int j = 0; j < NJ; j++) xo[j] = min(lane + 64 * j, ng.m_valid - 1) * ng.d;
#pragma unroll 1
            for (int t = 0; t < ng.d; t++) {
                const double xb0 = kv0 ? P[r0 + t] : 0.0, xb1 = kv1 ? P[r1 + t] : 0.0;
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const double df = xg[xo[v % NJ] + t] - (v / NJ ? xb1 : xb0);
                    r2[v] = fma(df, df, r2[v]);
                }
            }
        }
    };
    auto make_store = [&](int st, const Seg &sg, int kk, double (&r2)[NV]) {
        const int kg0 = kk + wave, kg1 = kg0 + 8;
        const bool kv0 = kg0 < sg.K, kv1 = kg1 < sg.K;  // wave-uniform
        if (ng.kern != 0) {
#pragma unroll
            for (int v = 0; v < NV; v++) r2[v] = sqrt(r2[v]);
        }
#pragma unroll
        for (int v = 0; v < NV; v++) r2[v] = exp(-r2[v] * ng.kscale);
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const int kh = v / NJ, k = wave + 8 * kh, m = lane + 64 * (v % NJ);
            if (BM % 64 == 0 || m < BM) {
                const bool ok = (kh ? kv1 : kv0) && m < ng.m_valid;
                *reinterpret_cast<double *>(lds + st * kStage + k * BM * 8 +
                                            ((((m >> 1) ^ ((k & 1) ? SWA : 0))) << 4) + ((m & 1) << 3)) =
                    ok ? r2[v] : 0.0;
            }
        }
    };
    auto make_all = [&](int st, const Seg &sg, int kk) {
        double r2[NV];
        make_dist(sg, kk, r2);
        make_store(st, sg, kk, r2);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // written before the barrier that publishes it
    };
    // A lane reads rows kr = ks + lane / 16 (ks % 4 == 0), so its row parity
    // is fixed.  Fragment i of the wave sits at byte (wm WM + i 16 + arow) 8 of
    // the row; on a permuted (odd) row its 128-byte half is swapped, which is
    // +128 bytes for even i and -128 for odd i (wm FM is even).  Two lane
    // bases, one per parity of i, leave only compile-time offsets.
    const int odd = (lane >> 4) & 1;
    const int a_lane = (lane >> 4) * BM * 8 + (wm * WM + arow) * 8, a_sw = (SWA && odd) ? 128 : 0;
    const int b_lane = (lane >> 4) * BN * 8 + (wn * WN + (lane & 15)) * 8, b_sw = (SWB && odd) ? 128 : 0;
    const int a_even = a_lane + a_sw, a_odd = a_lane - a_sw, b_even = b_lane + b_sw, b_odd = b_lane - b_sw;
    // a mirror chunk's A (pair-major, see issue): value k = ks + lane / 16 of
    // fragment i's row at ks BM 8 + a_mir + 256 i
    const int a_mir = SYM ? (lane >> 5) * BM * 16 + ((lane >> 4) & 1) * 8 + (wm * WM + arow) * 16 : 0;
    // g: also make the A block of the chunk in stage gst (segment gsg, row
    // gkk) between MFMA steps, so that its VALU work runs while the other
    // wave of the SIMD keeps the MFMA pipe busy: the distances after the
    // first step, the exponentials after the third (after the first, too,
    // at BN < 256, where carrying the distances over two steps spills)
    constexpr int kStoreStep = BN >= 256 ? 8 : 0;
    auto compute = [&](int st, bool mir, bool g, int gst, const Seg &gsg, int gkk) {
        const char *sa = lds + st * kStage;
        const char *sb_ = sa + BM * kBK * 8;
        double r2g[NV];
        int ai[FM];  // SYM: A fragment offsets within a k-step's rows, by the stage's layout
        if constexpr (SYM) {
#pragma unroll
            for (int i = 0; i < FM; i++) ai[i] = mir ? a_mir + i * 256 : ((i & 1) ? a_odd : a_even) + i * 128;
        }
        // 256-column tiles (registers to spare at two waves per SIMD): the
        // next k-step's operands are read from LDS before this k-step's
        // MFMAs, so that their latency hides behind them (128-column tiles,
        // at four waves per SIMD, gained nothing from it)
        constexpr bool kPipe = BN >= 256;
        double af[2][FM], bf[2][FN];
        auto frags = [&](int ks, double (&a)[FM], double (&b)[FN]) {
#pragma unroll
            for (int i = 0; i < FM; i++)
                a[i] = *reinterpret_cast<const double *>(
                    sa + ks * BM * 8 + (SYM ? ai[i] : ((i & 1) ? a_odd : a_even) + i * 128));
#pragma unroll
            for (int j = 0; j < FN; j++)
                b[j] = *reinterpret_cast<const double *>(sb_ + ks * BN * 8 + ((j & 1) ? b_odd : b_even) + j * 128);
        };
        if constexpr (kPipe) frags(0, af[0], bf[0]);
#pragma unroll
        for (int ks = 0; ks < kBK; ks += 4) {
            const int cb = kPipe ? (ks / 4) & 1 : 0;
            if constexpr (kPipe) {
                if (ks + 4 < kBK) frags(ks + 4, af[cb ^ 1], bf[cb ^ 1]);
            } else {
                frags(ks, af[0], bf[0]);
            }
#pragma unroll
            for (int i = 0; i < FM; i++)
#pragma unroll
                for (int j = 0; j < FN; j++) acc[i][j] = Mfma<double>::mma(af[cb][i], bf[cb][j], acc[i][j]);
            if (g && ks == 0) make_dist(gsg, gkk, r2g);
            if (g && ks == kStoreStep) make_store(gst, gsg, gkk, r2g);
        }
        if (g) asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // written before the next barrier
    };
    auto compute_and_make = [&](int st, bool mir, bool g, int gst, const Seg &gsg, int gkk) {
        if (computes)
            compute(st, mir, g, gst, gsg, gkk);
        else if (g)
            make_all(gst, gsg, gkk);
    };

    // next chunk to load (see product_loop_bf16x3): chunks of 16 rows over Kpad
    struct Cursor {
        int s, kk;
        Seg sg, nsg;
    };
    auto advance = [&](Cursor c) {
        if (c.s < se) {
            c.kk += kBK;
            if (c.kk >= c.sg.Kpad) {
                c.s++;
                c.kk = 0;
                if (c.s < se) {
                    c.sg = c.nsg;
                    if (c.s + 1 < se) c.nsg = load_seg_scalar(segs + c.s + 1);
                }
            }
        }
        c.s = __builtin_amdgcn_readfirstlane(c.s);
        c.kk = __builtin_amdgcn_readfirstlane(c.kk);
        return c;
    };

    if (sb < se) {
        if (gen && ng.d <= kMaxPointDim) {  // the tile's points (m_valid rows) into LDS before any chunk
                                           // is made, coordinate-major (xa[t][m]: the lanes of a wave
                                           // read consecutive m)
            double *xa = reinterpret_cast<double *>(ng.xa);
            for (int e = tid; e < ng.m_valid * ng.d; e += NT) xa[(e % ng.d) * 128 + e / ng.d] = ng.pts[ng.a_row * ng.d + e];
            __syncthreads();
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // only this loop's loads in flight
        Cursor cur;
        cur.s = sb;
        cur.kk = 0;
        cur.sg = load_seg_scalar(segs + sb);
        cur.nsg = sb + 1 < se ? load_seg_scalar(segs + sb + 1) : cur.sg;
        // bit st: the chunk in stage st was loaded as a mirror block
        int mbits = (SYM && issue(0, cur.sg, 0)) ? 1 : 0;  // chunk 0
        if (!SYM) issue(0, cur.sg, 0);
        if (gen && cur.sg.from_pts == ng.kind) make_all(0, cur.sg, 0);
        cur = advance(cur);   // chunk 1
        int st = 0;           // stage of chunk c
        // (the loop test sits at the bottom, after the accumulators' only
        // update: an exit between the MFMAs and the next iteration made the
        // register allocator copy every accumulator)
        if constexpr (STAGES == 3) {
            bool next_valid = cur.s < se;
            if (SYM && issue(1, cur.sg, cur.kk)) mbits |= 2;
            if (!SYM) issue(1, cur.sg, cur.kk);
            if (gen && cur.sg.from_pts == ng.kind) make_all(1, cur.sg, cur.kk);
            cur = advance(cur);  // chunk c + 2
            bool more = true;
            do {
                wait_vm_barrier<PER_WAVE>();  // chunk c landed; stage of c + 2 free
                const bool after_valid = cur.s < se;
                const int gst = st == 0 ? 2 : st - 1;
                const bool mir = SYM && ((mbits >> st) & 1);
                if constexpr (SYM)
                    mbits = __builtin_amdgcn_readfirstlane((mbits & ~(1 << gst)) | (issue(gst, cur.sg, cur.kk) ? 1 << gst : 0));
                else
                    issue(gst, cur.sg, cur.kk);
                compute_and_make(st, mir, gen && cur.sg.from_pts == ng.kind, gst, cur.sg, cur.kk);
                more = next_valid;
                next_valid = after_valid;
                cur = advance(cur);
                st = __builtin_amdgcn_readfirstlane(st == 2 ? 0 : st + 1);
            } while (more);
        } else {
            bool more = true;
            do {
                wait_vm_barrier<0>();  // chunk c landed; the other stage is free
                more = cur.s < se;     // chunk c + 1 exists
                const bool mir = SYM && ((mbits >> st) & 1);
                if constexpr (SYM)  // chunk c + 1 (or a repeat)
                    mbits = __builtin_amdgcn_readfirstlane((mbits & ~(1 << (st ^ 1))) | (issue(st ^ 1, cur.sg, cur.kk) ? 1 << (st ^ 1) : 0));
                else
                    issue(st ^ 1, cur.sg, cur.kk);
                compute_and_make(st, mir, gen && cur.sg.from_pts == ng.kind, st ^ 1, cur.sg, cur.kk);
                cur = advance(cur);
                st = __builtin_amdgcn_readfirstlane(st ^ 1);
            } while (more);
        }
        wait_vm_barrier<0>();  // no load may land in the LDS after the loop
    }
}

// LDS of the split-BF16 copy in store_tile: the tile as FP32, column-major
// with a pitch of BM + 4 values (16-byte accesses without bank conflicts).
template <int BM, int BN>
constexpr int split_copy_lds_bytes() {
    return BN * (BM + 4) * 4;
}

// Writes (or, with task.accumulate, adds) the tile's accumulators to rows
// [0, task.M) x columns [n0, n0 + BN) of the task's output block.  With
// task.Y set, row r goes to the caller's Y row perm[out_row + r] (first Q
// columns only); the destination rows are staged in LDS (free once the main
// loop has ended), so that no index stays live beside the accumulators.
// With task.out16 >= 0 (mixed precision; FP64 output in the FP32 register
// layout) the tile is also written to the split-BF16 workspace task.Y16 at
// rows out16.. (zero past row M); out_split 2 writes that copy only.  The
// copy goes through LDS (split_copy_lds_bytes), so that it runs after the
// accumulators are dead.  Y and out16 never come together (the caller's Y
// receives leaf outputs, the split copies are of Ŵ and Ŷ).
// Every thread of the workgroup calls it (it holds barriers).
template <typename OUT, typename ACC, int BM, int BN, int WAVES_M, int WAVES_N, bool F32_ROWS, bool BATCH_RMW = true>
__device__ __forceinline__ void store_tile(const TileJob &task, OUT *buf0, OUT *buf1, OUT *buf2, OUT *buf3,
                                           int64_t ldq, int64_t n0, void *lds,
                                           const ACC (&acc)[Tile<BM, BN, WAVES_M, WAVES_N>::FM]
                                                           [Tile<BM, BN, WAVES_M, WAVES_N>::FN]) {
    constexpr int WM = Tile<BM, BN, WAVES_M, WAVES_N>::WM, WN = Tile<BM, BN, WAVES_M, WAVES_N>::WN;
    constexpr int FM = WM / 16, FN = WN / 16;
    typedef __attribute__((address_space(1))) OUT gOUT;
    // thread index made opaque here, so that no address below is computed
    // once per kernel and held in registers through the product loops
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool computes = WAVES_M * WAVES_N == 8 || wave < WAVES_M * WAVES_N;  // 8: every wave of the largest workgroup
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    constexpr bool kSplitCopy = F32_ROWS && sizeof(OUT) == 8;
    constexpr int kPitch = BM + 4;
    const bool split_copy = kSplitCopy && task.out16 >= 0;  // uniform over the workgroup
    if constexpr (kSplitCopy) {
        if (split_copy && computes) {
            float *tile = reinterpret_cast<float *>(lds);
            // with task.accumulate, the copy is of the output's earlier value
            // plus this tile (a transfer added to far blocks written before)
            const OUT *prev = (task.out_buf == 0 ? buf0 : task.out_buf == 1 ? buf1 : task.out_buf == 2 ? buf2 : buf3) +
                              task.out_row * ldq + n0;
            // registers r = 0..3 of a lane are rows 4(l/16) + r of one column
#pragma unroll
            for (int i = 0; i < FM; i++)
#pragma unroll
                for (int j = 0; j < FN; j++) {
                    const int col = wn * WN + j * 16 + (lane & 15);
                    const int row = wm * WM + i * 16 + 4 * (lane >> 4);
                    f4_t v;
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        OUT x = (OUT)acc[i][j][u];
                        if (task.accumulate && row + u < task.M) x += prev[(int64_t)(row + u) * ldq + col];
                        v[u] = (float)x;
                    }
                    *reinterpret_cast<f4_t *>(tile + col * kPitch + row) = v;
                }
        }
    }
    int64_t *rows = reinterpret_cast<int64_t *>(lds);
    if (task.Y) {
        if (tid < task.M) {
            const int64_t t = task.out_row + tid;
            rows[tid] = task.perm ? *(const __attribute__((address_space(1))) int64_t *)(task.perm + t) : t;
        }
        __syncthreads();
    }
    if (computes && !(split_copy && task.out_split == 2)) {
        OUT *base = task.out_buf == 0 ? buf0 : task.out_buf == 1 ? buf1 : task.out_buf == 2 ? buf2 : buf3;
        OUT *out = base + task.out_row * ldq + n0;
        const int64_t lim = task.Y ? task.Q - n0 : BN;  // columns of this tile to store
        // BATCH_RMW: with task.accumulate, a row's earlier values are all
        // loaded before any of them is stored, so that those loads are in
        // flight together (a load after a store the compiler cannot tell
        // apart from it waits for the store's round trip)
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int row = wm * WM + i * 16 + frag_row<F32_ROWS>(lane, r);
                if (row >= task.M) continue;
                gOUT *o = task.Y ? (gOUT *)((OUT *)task.Y + rows[row] * task.ldy + n0)
                                 : (gOUT *)(out + (int64_t)row * ldq);
                if constexpr (BATCH_RMW) {
                    OUT prev[FN];
#pragma unroll
                    for (int j = 0; j < FN; j++) {
                        const int col = wn * WN + j * 16 + (lane & 15);
                        prev[j] = task.accumulate && col < lim ? o[col] : (OUT)0;
                    }
#pragma unroll
                    for (int j = 0; j < FN; j++) {
                        const int col = wn * WN + j * 16 + (lane & 15);
                        if (col < lim) o[col] = prev[j] + (OUT)acc[i][j][r];
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < FN; j++) {
                        const int col = wn * WN + j * 16 + (lane & 15);
                        if (col < lim) o[col] = task.accumulate ? o[col] + (OUT)acc[i][j][r] : (OUT)acc[i][j][r];
                    }
                }
            }
    }
    if constexpr (kSplitCopy) {
        if (split_copy) {
            __syncthreads();
            // one (32-row chunk, column) per step: 32 hi then 32 lo values,
            // 128 contiguous bytes of the workspace
            const float *tile = reinterpret_cast<const float *>(lds);
            __bf16 *Y16 = reinterpret_cast<__bf16 *>(task.Y16);
            constexpr int kChunks = BM / Split16::kRows;
            const int chunks = (task.M + Split16::kRows - 1) / Split16::kRows;
#pragma unroll 1
            for (int e = tid; e < kChunks * BN; e += blockDim.x) {
                const int c = e / BN, col = e % BN;
                if (c >= chunks) break;
                const float *src = tile + col * kPitch + c * 32;
                __bf16 *dst = Y16 + (task.out16 + c * 32) * 2 * ldq + (n0 + col) * 64;
#pragma unroll
                for (int v = 0; v < 4; v++) {  // rows 8v .. 8v + 7 of the chunk
                    const f4_t x0 = *reinterpret_cast<const f4_t *>(src + 8 * v);
                    const f4_t x1 = *reinterpret_cast<const f4_t *>(src + 8 * v + 4);
                    bf16x8_t hi, lo;
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        __bf16 h, l;
                        split_bf16(c * 32 + 8 * v + u < task.M ? (u < 4 ? x0[u] : x1[u - 4]) : 0.0f, h, l);
                        hi[u] = h;
                        lo[u] = l;
                    }
                    *(__attribute__((address_space(1))) bf16x8_t *)(dst + 8 * v) = hi;
                    *(__attribute__((address_space(1))) bf16x8_t *)(dst + 32 + 8 * v) = lo;
                }
            }
        }
    }
}

// One output tile: out (=|+=) sum over the task's segments of A_s * B_s.
// ROWPERM (FP64): accumulate in the FP32 register layout (see product_loop),
// as the mixed-precision launch does so that the split copy of the output
// can be written from consecutive rows.
// DMA (FP64, persistent launch): the direct global-to-LDS loop, with As_ the
// start of an LDS region of f64_lds_bytes<BM, BN, ROWPERM>() bytes.
template <typename T, int BM, int BN, int WAVES_M, int WAVES_N, int NT, bool ROWPERM = false, bool DMA = false,
          bool SYM = false>
__device__ __forceinline__ void block_product(const TileJob &task, const Seg *__restrict__ segs,
                                              const T *__restrict__ store, T *buf0, T *buf1,
                                              T *buf2, T *buf3, int64_t ldq, int64_t n0, T *As_,
                                              T *Bs_, NearGen ng = NearGen()) {
    typedef Tile<BM, BN, WAVES_M, WAVES_N> TL;
    typename Mfma<T>::acc_t acc[TL::FM][TL::FN];
#pragma unroll
    for (int i = 0; i < TL::FM; i++)
#pragma unroll
        for (int j = 0; j < TL::FN; j++) acc[i][j] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    if constexpr (DMA && sizeof(T) == 8) {
        ng.a_row = task.out_row;        // the tile's first row (task.m0 is its offset in the block)
        ng.m_valid = min(BM, task.M);   // the tile's rows
        product_loop_f64_dma<BM, BN, WAVES_M, WAVES_N, NT, ROWPERM, SYM>(segs, task.seg_begin, task.seg_end,
                                                                        task.m0, store, buf0, buf1, buf2, buf3,
                                                                        ldq, n0, reinterpret_cast<char *>(As_),
                                                                        acc, ng);
    }
    else
        product_loop<T, BM, BN, WAVES_M, WAVES_N, NT, ROWPERM, SYM>(segs, task.seg_begin, task.seg_end, task.m0,
                                                                    store, buf0, buf1, buf2, buf3, ldq, n0, As_,
                                                                    Bs_, acc);
    store_tile<T, typename Mfma<T>::acc_t, BM, BN, WAVES_M, WAVES_N, ROWPERM || sizeof(T) == 4, NT == 512>(
        task, buf0, buf1, buf2, buf3, ldq, n0, As_, acc);
}

// ---------------------------------------------------------------------------
// Split-BF16 products (mixed precision).  An FP64 value v is carried as
// v ~= hi + lo with hi = bf16(v), lo = bf16(v - hi), and a product as
// A B ~= A_hi B_hi + A_hi B_lo + A_lo B_hi, each term a
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (lane mapping checked on
// the device: lane l supplies A[l%16][8(l/16)..8(l/16)+7] and
// B[8(l/16)..8(l/16)+7][l%16]; accumulator register r of lane l holds
// D[4(l/16)+r][l%16]).  A blocks come from the split-BF16 store, where a
// block is a run of 32-wide contraction chunks, each chunk the hi part
// (lda rows x 32 contraction values, row-major) followed by the lo part.
// B rows come pre-split from the split-BF16 workspaces (see Split16).

constexpr int kKC = 32;     // contraction rows per chunk
constexpr int kStages = 3;  // LDS stages: one consumed, two being filled

// One LDS stage of a split-BF16 chunk, unpadded: A as [hi, lo][BM rows][32]
// (64 bytes a row), then B as [BN columns][hi 32, lo 32] (128 bytes a
// column), both in 16-byte slots.  The stage is filled by direct
// global-to-LDS loads (each wave instruction writes 64 consecutive slots), so
// bank conflicts of the MFMA operand reads are avoided by permuting the slots
// within a row (A) or column (B) instead of padding: logical 16-byte vector
// g of A row r sits in slot g ^ swz_a(r), logical vector j of B column n in
// slot j ^ swz_b(n).  For the 16 rows (columns) that one 16-lane group of a
// fragment read touches, and for any 8 consecutive of them, the slots then
// fall into distinct 16-byte bank groups.
template <int BM, int BN>
constexpr int bf16_stage_bytes() {
    return (BM + BN) * 128;
}
template <int BM, int BN>
constexpr int bf16_lds_bytes() {
    return kStages * bf16_stage_bytes<BM, BN>();
}
__device__ __forceinline__ int swz_a(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }
__device__ __forceinline__ int swz_b(int n) { return ((n >> 1) & 7) ^ ((n & 1) << 2); }

// LDS of a tile of the mixed-precision launch: the split-BF16 stages, the
// FP32 partial sums of the whole tile while they are handed over, or the
// split copy of the output, whichever is largest.
template <int BM, int BN>
constexpr int split_f64_lds_bytes() {
    constexpr int a = bf16_lds_bytes<BM, BN>() > BM * BN * 4 ? bf16_lds_bytes<BM, BN>() : BM * BN * 4;
    return a > split_copy_lds_bytes<BM, BN>() ? a : split_copy_lds_bytes<BM, BN>();
}

// Accumulates rows [m0, m0 + BM) x columns [n0, n0 + BN) of the split-BF16
// products of segments [sb, se) into FP32 accumulators (FP32 register
// layout, frag_row<true>).
//
// Pipeline: chunks of 32 contraction rows go straight from global memory
// into one of three LDS stages (global_load_lds_dwordx4, no staging
// registers).  While the MFMAs consume chunk c, the loads of chunks c + 1
// and c + 2 are in flight; one barrier per chunk.  Every wave issues the same
// number of loads per chunk (block indices past the stage re-load its last
// block, the same bytes to the same place), so a chunk is complete once the
// wave's counter is down to the one later chunk's loads.  Past the last chunk
// the loads repeat a valid chunk into a stage nobody reads, and the loop ends
// with every load drained, since the LDS is reused after it.
template <int BM, int BN, int WAVES_M, int WAVES_N, int NT>
__device__ __forceinline__ void product_loop_bf16x3(
    const Seg *__restrict__ segs, int sb, int se, int m0, const __bf16 *__restrict__ store16,
    const __bf16 *w16, const __bf16 *what16, const __bf16 *yhat16, int64_t ldq, int64_t n0, char *lds,
    f4_t (&acc)[Tile<BM, BN, WAVES_M, WAVES_N>::FM][Tile<BM, BN, WAVES_M, WAVES_N>::FN]) {
    constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
    constexpr int FM = WM / 16, FN = WN / 16;
    static_assert(FM >= 1 && FN >= 1, "bad tile");
    static_assert(NT == 512, "8 waves fill a stage");
    constexpr int kStage = bf16_stage_bytes<BM, BN>();
    constexpr int A_BLOCKS = BM / 8;                  // 1 KB blocks (64 slots) of A: 2 parts x BM rows x 4 slots
    constexpr int BLOCKS = (BM + BN) / 8;             // A then B (8 slots a column)
    constexpr int PER_WAVE = (BLOCKS + 7) / 8;        // loads per wave and chunk
    static_assert(BLOCKS * 1024 == kStage, "stage size");

    // thread index made opaque (as in store_tile): the per-thread load and
    // LDS offsets are computed per task, not once per kernel and held
    // through every other path of the persistent loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool computes = WAVES_M * WAVES_N == NT / 64 || wave < WAVES_M * WAVES_N;  // all waves: known at compile time
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    // the split workspace of a segment's B operand (by its FP64 buffer id)
    auto b16p = [&](int b) { return b == BUF_WT ? w16 : b == BUF_WHAT ? what16 : yhat16; };

    // Chunk kk / 32 of segment sg into LDS stage st.  Slot t = 64 q + lane of
    // block q: A slots are (part, row, slot), B slots are (column, slot).
    auto issue = [&](int st, const Seg &sg, int kk) {
        const __bf16 *A = store16 + sg.a_off16 + (int64_t)(kk / kKC) * 2 * sg.lda * kKC;
        const __bf16 *B = b16p(sg.b_buf) + (sg.b_row16 + kk) * 2 * ldq + n0 * 64;
        char *stage = lds + st * kStage;
#pragma unroll
        for (int u = 0; u < PER_WAVE; u++) {
            const int q = min(u * 8 + wave, BLOCKS - 1);  // wave-uniform
            const __bf16 *src;
            if (q < A_BLOCKS) {
                const int t = q * 64 + lane, part = t / (BM * 4), r = (t / 4) % BM, g = (t % 4) ^ swz_a(r);
                src = A + (int64_t)part * sg.lda * kKC + (int64_t)(m0 + r) * kKC + g * 8;
            } else {
                const int t = (q - A_BLOCKS) * 64 + lane, n = t / 8, j = (t % 8) ^ swz_b(n);
                src = B + n * 64 + j * 8;
            }
            load_lds16(src, stage + q * 1024);
        }
    };
    auto compute = [&](int st) {
        const char *stage = lds + st * kStage;
        const int kg = lane >> 4;
        bf16x8_t ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
        for (int i = 0; i < FM; i++) {
            const int r = wm * WM + i * 16 + (lane & 15);
            const int off = r * 64 + ((kg ^ swz_a(r)) * 16);
            ah[i] = *reinterpret_cast<const bf16x8_t *>(stage + off);
            al[i] = *reinterpret_cast<const bf16x8_t *>(stage + BM * 64 + off);
        }
#pragma unroll
        for (int j = 0; j < FN; j++) {
            const int n = wn * WN + j * 16 + (lane & 15);
            const char *col = stage + BM * 128 + n * 128;
            bh[j] = *reinterpret_cast<const bf16x8_t *>(col + ((kg ^ swz_b(n)) * 16));
            bl[j] = *reinterpret_cast<const bf16x8_t *>(col + (((4 + kg) ^ swz_b(n)) * 16));
        }
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int j = 0; j < FN; j++) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            }
    };

    // Position of the next chunk to load: chunk kk / 32 of segment s, with
    // the descriptor of segment s + 1 loaded one segment ahead (so that its
    // wait never covers the chunk loads issued after it).  Past the last
    // chunk (s == se) it keeps the last segment with kk = 0: loads issued for
    // it stay inside that segment's block and node rows.
    struct Cursor {
        int s, kk;
        Seg sg, nsg;
    };
    // (readfirstlane: the cursor is wave-uniform, and keeping it in scalar
    // registers keeps the loop's branches and descriptor loads scalar)
    auto advance = [&](Cursor c) {
        if (c.s < se) {
            c.kk += kKC;
            if (c.kk >= c.sg.K) {
                c.s++;
                c.kk = 0;
                if (c.s < se) {
                    c.sg = c.nsg;
                    if (c.s + 1 < se) c.nsg = load_seg_scalar(segs + c.s + 1);
                }
            }
        }
        c.s = __builtin_amdgcn_readfirstlane(c.s);
        c.kk = __builtin_amdgcn_readfirstlane(c.kk);
        return c;
    };

    if (sb < se) {
        // nothing older may be outstanding: the count-based waits below
        // assume that only this loop's loads are in flight
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        Cursor cur;
        cur.s = sb;
        cur.kk = 0;
        cur.sg = load_seg_scalar(segs + sb);
        cur.nsg = sb + 1 < se ? load_seg_scalar(segs + sb + 1) : cur.sg;
        issue(0, cur.sg, cur.kk);  // chunk 0
        cur = advance(cur);
        bool next_valid = cur.s < se;  // chunk c + 1 exists
        issue(1, cur.sg, cur.kk);      // chunk 1 (or a repeat)
        cur = advance(cur);            // chunk c + 2
        int st = 0;                    // stage of chunk c
        while (true) {
            wait_vm_barrier<PER_WAVE>();  // chunk c has landed in every wave's part; stage c + 2 is free
            const bool after_valid = cur.s < se;
            issue(st == 0 ? 2 : st - 1, cur.sg, cur.kk);  // chunk c + 2 (or a repeat)
            if (computes) compute(st);
            if (!next_valid) break;
            next_valid = after_valid;
            cur = advance(cur);
            st = __builtin_amdgcn_readfirstlane(st == 2 ? 0 : st + 1);
        }
        wait_vm_barrier<0>();  // no load may land in the LDS after the loop
    }
}

// One output tile in split BF16: out (=|+=) sum over the task's segments.
template <int BM, int BN, int WAVES_M, int WAVES_N, int NT>
__device__ __forceinline__ void block_product_bf16x3(const TileJob &task, const Seg *__restrict__ segs,
                                                     const __bf16 *__restrict__ store16, const __bf16 *w16,
                                                     const __bf16 *what16, const __bf16 *yhat16, double *buf0,
                                                     double *buf1, double *buf2, double *buf3,
                                                     int64_t ldq, int64_t n0, char *lds) {
    typedef Tile<BM, BN, WAVES_M, WAVES_N> TL;
    f4_t acc[TL::FM][TL::FN];
#pragma unroll
    for (int i = 0; i < TL::FM; i++)
#pragma unroll
        for (int j = 0; j < TL::FN; j++) acc[i][j] = f4_t{0, 0, 0, 0};
    product_loop_bf16x3<BM, BN, WAVES_M, WAVES_N, NT>(segs, task.seg_begin, task.seg_end, task.m0, store16,
                                                      w16, what16, yhat16, ldq, n0, lds, acc);
    store_tile<double, f4_t, BM, BN, WAVES_M, WAVES_N, true>(task, buf0, buf1, buf2, buf3, ldq, n0, lds, acc);
}

// A down-pass tile of the mixed-precision graph: the far blocks (all
// segments but the last) in split BF16 with FP32 accumulation, then the
// transfer from the parent (the last segment) in FP64 continuing from those
// partial sums (converted to FP64), written once.
template <int BM, int BN, int WAVES_M, int WAVES_N, int NT>
__device__ __forceinline__ void block_product_split_then_f64(const TileJob &task, const Seg *__restrict__ segs,
                                                             const double *__restrict__ store,
                                                             const __bf16 *__restrict__ store16, const __bf16 *w16,
                                                             const __bf16 *what16, const __bf16 *yhat16,
                                                             double *buf0, double *buf1, double *buf2, double *buf3,
                                                             int64_t ldq, int64_t n0, char *lds) {
    typedef Tile<BM, BN, WAVES_M, WAVES_N> TL;
    f4_t acc32[TL::FM][TL::FN];
#pragma unroll
    for (int i = 0; i < TL::FM; i++)
#pragma unroll
        for (int j = 0; j < TL::FN; j++) acc32[i][j] = f4_t{0, 0, 0, 0};
    product_loop_bf16x3<BM, BN, WAVES_M, WAVES_N, NT>(segs, task.seg_begin, task.seg_end - 1, task.m0, store16,
                                                      w16, what16, yhat16, ldq, n0, lds, acc32);
    // hand the partial sums over through LDS (free once the split loop has
    // ended), so that the FP32 and FP64 accumulators are never live together
    constexpr int kVals = TL::FM * TL::FN * 4;
    float *stage = reinterpret_cast<float *>(lds);
    int tid = threadIdx.x;  // opaque: the LDS addresses are not hoisted out of the task loop
    asm volatile("" : "+v"(tid));
    const bool computes = WAVES_M * WAVES_N == NT / 64 || __builtin_amdgcn_readfirstlane(tid >> 6) < WAVES_M * WAVES_N;
    if (computes) {
#pragma unroll
        for (int i = 0; i < TL::FM; i++)
#pragma unroll
            for (int j = 0; j < TL::FN; j++)
#pragma unroll
                for (int r = 0; r < 4; r++) stage[((i * TL::FN + j) * 4 + r) * NT + tid] = acc32[i][j][r];
    }
    __syncthreads();
    d4_t acc[TL::FM][TL::FN];
#pragma unroll
    for (int i = 0; i < TL::FM; i++)
#pragma unroll
        for (int j = 0; j < TL::FN; j++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                acc[i][j][r] = computes ? (double)stage[((i * TL::FN + j) * 4 + r) * NT + tid] : 0.0;
    static_assert(kVals * NT * 4 <= split_f64_lds_bytes<BM, BN>(), "LDS hand-over does not fit");
    __syncthreads();
    product_loop_f64_dma<BM, BN, WAVES_M, WAVES_N, NT, true>(segs, task.seg_end - 1, task.seg_end, task.m0, store,
                                                             buf0, buf1, buf2, buf3, ldq, n0, lds, acc);
    store_tile<double, d4_t, BM, BN, WAVES_M, WAVES_N, true>(task, buf0, buf1, buf2, buf3, ldq, n0, lds, acc);
}

// Split-BF16 copy of one block per workgroup: for chunk c, part h (0 hi,
// 1 lo), row i < lda, value k < 32: dst = split(src[(32c + k) * lda + i]),
// zero beyond the block's K contraction rows.
__global__ void k_make_bf16x3(const double *__restrict__ store, const Seg *__restrict__ segs,
                              __bf16 *__restrict__ store16) {
    const Seg sg = segs[blockIdx.x];
    const int nchunks = (sg.K + kKC - 1) / kKC;
    const int64_t per_chunk = (int64_t)sg.lda * kKC;
    for (int64_t e = threadIdx.x; e < nchunks * per_chunk; e += blockDim.x) {
        const int c = (int)(e / per_chunk), rem = (int)(e % per_chunk), i = rem / kKC, k = rem % kKC;
        const int kk = c * kKC + k;
        const float v = kk < sg.K ? (float)store[sg.trans ? sg.a_off + (int64_t)i * sg.tstride + kk
                                                          : sg.a_off + (int64_t)kk * sg.lda + i]
                                  : 0.0f;
        __bf16 hi, lo;
        split_bf16(v, hi, lo);
        __bf16 *dst = store16 + sg.a_off16 + (int64_t)c * 2 * per_chunk;
        dst[rem] = hi;
        dst[per_chunk + rem] = lo;
    }
}

// One launch = one phase: workgroup (x, y) computes task x, column tile y.
template <typename T, int BM, int BN, int WAVES_M, int WAVES_N, bool SYM>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void k_block_products(
    const Task *__restrict__ tasks, const Seg *__restrict__ segs, int task_begin,
    const T *__restrict__ store, T *buf0, T *buf1, T *buf2, T *buf3, int64_t ldq) {
    constexpr int NT = 64 * WAVES_M * WAVES_N;
    __shared__ __attribute__((aligned(16))) T As[2 * kBK * (BM + lds_pad<T>())];
    __shared__ __attribute__((aligned(16))) T Bs[2 * kBK * (BN + lds_pad<T>())];
    const Task t = tasks[task_begin + blockIdx.x];
    const TileJob job{t.out_row, t.out_buf, t.M, t.m0, t.seg_begin, t.seg_end, 0};  // workspace output
    block_product<T, BM, BN, WAVES_M, WAVES_N, NT, false, false, SYM>(job, segs, store, buf0, buf1, buf2, buf3,
                                                                      ldq, (int64_t)blockIdx.y * BN, As, Bs);
}

// Wave layouts of the persistent kernel (8 waves) per tile: {WAVES_M, WAVES_N}.
template <int BM, int BN>
struct PLayout {
    static constexpr int WN = BN >= 256 ? (BM == 128 ? 4 : 8) : BN == 128 ? (BM == 128 ? 2 : 4)
                            : BN == 64 ? (BM == 128 ? 1 : 2) : BN == 32 ? (BM == 128 ? 1 : 2) : 1;
    // waves along M: as many as fit beside WN, dividing the BM / 16 fragment
    // rows evenly (96 rows: 6 fragment rows over 1, 2, 3 or 6 waves)
    static constexpr int kMaxM = 8 / WN;
    static constexpr int WMv = BM == 96 ? (kMaxM >= 6 ? 6 : kMaxM >= 3 ? 3 : kMaxM >= 2 ? 2 : 1)
                                        : ((BM / 16 < kMaxM) ? BM / 16 : kMaxM);
};

// 8 waves per workgroup.  With column tiles up to 128 the kernel is held to
// 128 VGPRs (4 waves per SIMD), so that two workgroups share a compute unit.
constexpr int kPersistThreads = 512;
constexpr int kWaitLimit = 1 << 20;  // polls (each followed by a sleep) before giving up

// A tile of stored (or generated) blocks at column width W in the launch's
// type: the row-tile height bm picks the instantiation.  Where W lacks the
// height the plan made (a narrow tile in a launch whose own width has finer
// tiles, see fine_tiles and fine16_tiles), the next taller tile covers the
// rows.
template <typename T, int W, bool SPLIT, bool SYM, int LDS_BYTES>
__device__ __forceinline__ void native_tile(int bm, const TileJob &job, const Seg *__restrict__ segs,
                                            const T *__restrict__ store, const MatDesc &md, int64_t n0, T *As,
                                            T *Bs, const NearGen &ng) {
    if constexpr (fine16_tiles(sizeof(T), W, SPLIT)) {
        if (bm == 48 || bm == 80 || bm == 112) {
            if (bm == 48)
                block_product<T, 48, W, PLayout<48, W>::WMv, PLayout<48, W>::WN, kPersistThreads, false, false,
                              SYM>(job, segs, store, (T *)md.buf[0], (T *)md.buf[1], (T *)md.buf[2],
                                   (T *)md.buf[3], md.ldq, n0, As, Bs, ng);
            else if (bm == 80)
                block_product<T, 80, W, PLayout<80, W>::WMv, PLayout<80, W>::WN, kPersistThreads, false, false,
                              SYM>(job, segs, store, (T *)md.buf[0], (T *)md.buf[1], (T *)md.buf[2],
                                   (T *)md.buf[3], md.ldq, n0, As, Bs, ng);
            else
                block_product<T, 112, W, PLayout<112, W>::WMv, PLayout<112, W>::WN, kPersistThreads, false, false,
                              SYM>(job, segs, store, (T *)md.buf[0], (T *)md.buf[1], (T *)md.buf[2],
                                   (T *)md.buf[3], md.ldq, n0, As, Bs, ng);
            return;
        }
    }
    bm = bm <= 32 ? 32 : bm <= 64 ? 64 : bm <= 96 ? 96 : 128;
    constexpr bool kFine = fine_tiles(sizeof(T), W, SPLIT);
    // the tallest tile's stages fit the kernel's LDS (FP64: the direct-to-LDS
    // stages from As; FP32: the register-staged As and Bs)
    static_assert(sizeof(T) != 8 || f64_lds_bytes<128, W, SPLIT>() <= LDS_BYTES, "FP64 stages exceed the LDS");
    static_assert(sizeof(T) != 4 ||
                      (2 * kBK * (128 + lds_pad<T>()) + 2 * kBK * (W + lds_pad<T>())) * (int)sizeof(T) <= LDS_BYTES,
                  "FP32 stages exceed the LDS");
    if (bm == 128 || (!kFine && bm == 96)) {
        block_product<T, 128, W, PLayout<128, W>::WMv, PLayout<128, W>::WN, kPersistThreads,
                      SPLIT && sizeof(T) == 8, sizeof(T) == 8, SYM>(job, segs, store, (T *)md.buf[0], (T *)md.buf[1],
                                               (T *)md.buf[2], (T *)md.buf[3], md.ldq, n0, As, Bs, ng);
    } else if (!kFine || bm == 64) {
        block_product<T, 64, W, PLayout<64, W>::WMv, PLayout<64, W>::WN, kPersistThreads,
                      SPLIT && sizeof(T) == 8, sizeof(T) == 8, SYM>(job, segs, store, (T *)md.buf[0], (T *)md.buf[1],
                                               (T *)md.buf[2], (T *)md.buf[3], md.ldq, n0, As, Bs, ng);
    } else if constexpr (kFine) {
        // 32- and 96-row tiles, for output blocks whose row count would
        // waste most of a 64- or 128-row tile
        if (bm == 96)
            block_product<T, 96, W, PLayout<96, W>::WMv, PLayout<96, W>::WN, kPersistThreads, false,
                          sizeof(T) == 8, SYM>(job, segs, store, (T *)md.buf[0], (T *)md.buf[1], (T *)md.buf[2],
                                                  (T *)md.buf[3], md.ldq, n0, As, Bs, ng);
        else
            block_product<T, 32, W, PLayout<32, W>::WMv, PLayout<32, W>::WN, kPersistThreads, false,
                          sizeof(T) == 8, SYM>(job, segs, store, (T *)md.buf[0], (T *)md.buf[1], (T *)md.buf[2],
                                                  (T *)md.buf[3], md.ldq, n0, As, Bs, ng);
    }
}

// native_tile at the task's own width bn (a power of two, 16 <= bn <= W).
template <typename T, int W, bool SPLIT, bool SYM, int LDS_BYTES>
__device__ __forceinline__ void narrow_tile(int bn, int bm, const TileJob &job, const Seg *__restrict__ segs,
                                            const T *__restrict__ store, const MatDesc &md, int64_t n0, T *As,
                                            T *Bs, const NearGen &ng) {
    if constexpr (W > 16) {
        if (bn < W) {
            narrow_tile<T, W / 2, SPLIT, SYM, LDS_BYTES>(bn, bm, job, segs, store, md, n0, As, Bs, ng);
            return;
        }
    }
    native_tile<T, W, SPLIT, SYM, LDS_BYTES>(bm, job, segs, store, md, n0, As, Bs, ng);
}

// Persistent task-graph launch: workgroups take queue entries in order with
// an atomic head; an entry starts once its dependency counter is zero (a
// bounded wait, see kWaitLimit), then decrements its successors' counters
// after its output is written back (agent-scope release / acquire, which
// also makes results visible across the XCDs' separate L2 caches).  The
// queue order is topological, so every awaited entry was taken earlier by a
// running workgroup: the launch cannot deadlock and every workgroup exits
// when the queue is drained.
// NARROW: a 256-column launch whose plan has narrower tiles for the last
// columns of a matrix (GraphPlan::narrow): a task runs at its own width pt.bn
// (256, 128, ... 16); a separate instantiation, so that launches without such
// tiles keep their registers and code.
// GEN: the FP64 launch that computes the near blocks from the points (see
// NearGen); a separate instantiation, so that the stored-block launch keeps
// its registers and code.  With SYM as well for a symmetric store (its
// stored blocks may be mirrors): the mirror-capable loop costs the points
// launch about 5%, so it is not compiled into the plain one.
template <typename T, int BN, bool SPLIT, bool GEN = false, bool SYM = false, bool NARROW = false>
__global__ __launch_bounds__(kPersistThreads, (NARROW && sizeof(T) == 4) || BN <= 128 ? 4 : 1)
void k_persistent(
    const PTask *__restrict__ tasks, int n_tasks, const int32_t *__restrict__ succ,
    int32_t *counters, int32_t *head, int32_t *err, const MatDesc *__restrict__ mats, void *Y, int64_t ldy,
    int64_t Q, const int64_t *__restrict__ perm) {
    constexpr int kRegs = (2 * kBK * (128 + lds_pad<T>()) + 2 * kBK * (BN + lds_pad<T>())) * (int)sizeof(T);
    constexpr int kNative = sizeof(T) != 8 ? kRegs : NARROW ? f64_lds_bytes_narrow<BN>() : f64_lds_bytes<128, BN, SPLIT>();
    constexpr int kSplit = (SPLIT && sizeof(T) == 8) ? split_f64_lds_bytes<128, BN>() : 0;
    constexpr int kMain = kNative > kSplit ? kNative : kSplit;
    // (not at 64 columns, where the points' LDS would cost the second
    // workgroup per compute unit: hm_eval runs that mode at 128 columns)
    constexpr bool kGen = GEN;
    static_assert(!GEN || (sizeof(T) == 8 && !SPLIT && BN != 64), "near blocks from points: FP64 only");
    static_assert(!NARROW || (!SPLIT && !GEN && BN == 256), "narrow tiles: 256-column stored-block launches only");
    __shared__ __attribute__((aligned(16))) char lds[kMain + (kGen ? kPointLds : 0)];
    T *As = reinterpret_cast<T *>(lds);
    T *Bs = As + 2 * kBK * (128 + lds_pad<T>());
    __shared__ int s_t;
    while (true) {
        if (threadIdx.x == 0) s_t = __hip_atomic_fetch_add(head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_t);  // uniform: task fields load as scalars
        __syncthreads();
        if (t >= n_tasks) break;
        const PTask pt = tasks[t];
        if (threadIdx.x == 0 && pt.ndeps > 0) {
            int polls = 0;
            while (__hip_atomic_load(&counters[t], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) > 0) {
                if (++polls > kWaitLimit) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __syncthreads();
        const MatDesc &md = mats[pt.mat];  // fields read in place: a private copy would be indexed dynamically (buf16) and live in scratch
        TileJob job{pt.out_row, pt.out_buf, pt.M, pt.m0, pt.seg_begin, pt.seg_end, pt.accumulate};
        if (Y && pt.out_buf == BUF_YT) {  // leaf rows go straight to the caller's Y
            job.Y = Y;
            job.ldy = ldy;
            job.Q = Q;
            job.perm = perm;
        }
        if constexpr (SPLIT && sizeof(T) == 8) {
            if (pt.out16 >= 0) {  // split copy of Ŵ or of a leaf's Ŷ (mixed precision)
                job.Y16 = md.buf16[pt.out_buf];
                job.out16 = pt.out16;
                job.out_split = pt.out_split;
            }
        }
        const int64_t n0 = pt.n0;
        const T *store = (const T *)md.store;
        const Seg *segs = md.segs;
        NearGen ng;
        if constexpr (kGen) {
            // leaf tiles: near blocks (rows of Y in tree order = point rows);
            // down-pass tiles: far blocks (rows of Ŷ = skeleton point rows);
            // null: the blocks come from the store
            if (pt.out_buf == BUF_YT && md.pts) {
                ng.pts = md.pts;
                ng.kind = 1;
            } else if (pt.out_buf == BUF_YHAT && md.skel_pts) {
                ng.pts = md.skel_pts;
                ng.kind = 2;
            }
            ng.d = md.pts_d;
            ng.kern = md.kern;
            ng.kscale = md.kscale;
            ng.xa = lds + kMain;
        }
        int mode = 0;
        if constexpr (SPLIT && sizeof(T) == 8) mode = pt.mode;
        if (mode != 0) {
            if constexpr (SPLIT && sizeof(T) == 8) {
                const __bf16 *s16 = (const __bf16 *)md.store16;
                const __bf16 *w16 = (const __bf16 *)md.buf16[BUF_WT], *wh16 = (const __bf16 *)md.buf16[BUF_WHAT],
                             *yh16 = (const __bf16 *)md.buf16[BUF_YHAT];
                double *b0 = (double *)md.buf[0], *b1 = (double *)md.buf[1], *b2 = (double *)md.buf[2],
                       *b3 = (double *)md.buf[3];
                if (mode == 1 && pt.bm == 128)
                    block_product_bf16x3<128, BN, PLayout<128, BN>::WMv, PLayout<128, BN>::WN, kPersistThreads>(
                        job, segs, s16, w16, wh16, yh16, b0, b1, b2, b3, md.ldq, n0, lds);
                else if (mode == 1)
                    block_product_bf16x3<64, BN, PLayout<64, BN>::WMv, PLayout<64, BN>::WN, kPersistThreads>(
                        job, segs, s16, w16, wh16, yh16, b0, b1, b2, b3, md.ldq, n0, lds);
                else if (pt.bm == 128)
                    block_product_split_then_f64<128, BN, PLayout<128, BN>::WMv, PLayout<128, BN>::WN,
                                                 kPersistThreads>(job, segs, (const double *)store, s16, w16, wh16,
                                                                  yh16, b0, b1, b2, b3, md.ldq, n0, lds);
                else
                    block_product_split_then_f64<64, BN, PLayout<64, BN>::WMv, PLayout<64, BN>::WN,
                                                 kPersistThreads>(job, segs, (const double *)store, s16, w16, wh16,
                                                                  yh16, b0, b1, b2, b3, md.ldq, n0, lds);
            }
        } else if constexpr (NARROW) {
            narrow_tile<T, BN, SPLIT, SYM, kMain>(pt.bn, pt.bm, job, segs, store, md, n0, As, Bs, ng);
        } else {
            native_tile<T, BN, SPLIT, SYM, kMain>(pt.bm, job, segs, store, md, n0, As, Bs, ng);
        }
        __syncthreads();  // every wave's stores of this task are done
        if (threadIdx.x == 0 && pt.succ_end > pt.succ_begin) {
            __threadfence();  // release this task's output to every XCD
            for (int e = pt.succ_begin; e < pt.succ_end; e++)
                __hip_atomic_fetch_add(&counters[succ[e]], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// counters[i] = tasks[i].ndeps; head = 0 (run before each persistent launch).
__global__ void k_persistent_init(const PTask *__restrict__ tasks, int n_tasks, int32_t *counters,
                                  int32_t *head) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_tasks) counters[i] = tasks[i].ndeps;
    if (i == 0) *head = 0;
}

// Row gather W (original order, leading dimension ldw) -> Wt (tree order, Qp),
// zero-filling the padding columns; perm == nullptr means identity.
template <typename T>
__global__ void k_permute_in(const T *__restrict__ W, int64_t ldw, T *__restrict__ Wt, int64_t Qp,
                             const int64_t *__restrict__ perm, int64_t N, int64_t Q) {
    const int64_t total = N * Qp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / Qp, c = e % Qp;
        const int64_t src = perm ? perm[t] : t;
        Wt[e] = c < Q ? W[src * ldw + c] : T(0);
    }
}

// Split-BF16 W in tree order (see Split16): one thread per (32-row chunk,
// column); chunks[3c..3c+2] = (first tree row, rows, first split row).  Rows
// past the chunk's rows and columns >= Q are zero.
__global__ void k_permute_in_split(const double *__restrict__ W, int64_t ldw, __bf16 *__restrict__ W16,
                                   int64_t ldq, const int64_t *__restrict__ perm,
                                   const int64_t *__restrict__ chunks, int64_t n_chunks, int64_t Q) {
    const int64_t total = n_chunks * ldq;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / ldq, col = e % ldq;
        const int64_t t0 = chunks[3 * c], nr = chunks[3 * c + 1], g = chunks[3 * c + 2];
        bf16x8_t hi[4], lo[4];
#pragma unroll
        for (int k = 0; k < 32; k++) {
            double v = 0.0;
            if (k < nr && col < Q) {
                const int64_t t = t0 + k;
                v = W[(perm ? perm[t] : t) * ldw + col];
            }
            __bf16 h, l;
            split_bf16((float)v, h, l);
            hi[k / 8][k % 8] = h;
            lo[k / 8][k % 8] = l;
        }
        __bf16 *dst = W16 + g * 2 * ldq + col * 64;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            *reinterpret_cast<bf16x8_t *>(dst + v * 8) = hi[v];
            *reinterpret_cast<bf16x8_t *>(dst + 32 + v * 8) = lo[v];
        }
    }
}

// Row scatter Yt (tree order, Qp) -> Y (original order, ldy), first Q columns.
template <typename T>
__global__ void k_permute_out(const T *__restrict__ Yt, int64_t Qp, T *__restrict__ Y, int64_t ldy,
                              const int64_t *__restrict__ perm, int64_t N, int64_t Q) {
    const int64_t total = N * Q;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / Q, c = e % Q;
        const int64_t dst = perm ? perm[t] : t;
        Y[dst * ldy + c] = Yt[t * Qp + c];
    }
}

// Repack one source block per workgroup into the K-major padded store.
//   mode 0 (transpose): src is rows x cols row-major; dst row t (t < ncols)
//     holds src[:, c0 + t] in its first `rows` entries.
//   mode 1 (slice):     src is rows x cols row-major; dst row t (t < rows)
//     holds src[t, c0 : c0 + ncols].
// Entries [valid, ld) of every dst row are zero; rows beyond the ones written
// keep the zeros the store was cleared with.
__global__ void k_repack(const double *__restrict__ stage, const RepackJob *__restrict__ jobs,
                         double *__restrict__ store) {
    __shared__ double tile[32][33];
    const RepackJob j = jobs[blockIdx.x];
    const double *src = stage + j.src_off;
    double *dst = store + j.dst_off;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    if (j.mode == 0) {
        for (int i0 = 0; i0 < j.ld; i0 += 32)
            for (int t0 = 0; t0 < j.ncols; t0 += 32) {
                for (int y = ty; y < 32; y += 8) {
                    const int i = i0 + y, t = t0 + tx;
                    tile[y][tx] = (i < j.rows && t < j.ncols) ? src[(int64_t)i * j.cols + j.c0 + t] : 0.0;
                }
                __syncthreads();
                for (int y = ty; y < 32; y += 8) {
                    const int t = t0 + y, i = i0 + tx;
                    if (t < j.ncols && i < j.ld) dst[(int64_t)t * j.ld + i] = tile[tx][y];
                }
                __syncthreads();
            }
    } else {
        for (int t = ty; t < j.rows; t += 8)
            for (int i = tx; i < j.ld; i += 32)
                dst[(int64_t)t * j.ld + i] = i < j.ncols ? src[(int64_t)t * j.cols + j.c0 + i] : 0.0;
    }
}

// Batched permutes: blockIdx.y selects the matrix.
template <typename T>
__global__ void k_permute_in_batched(const PermDesc *__restrict__ d) {
    const PermDesc pd = d[blockIdx.y];
    const int64_t total = pd.N * pd.ldq;
    const T *W = (const T *)pd.W;
    T *Wt = (T *)pd.Wt;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / pd.ldq, c = e % pd.ldq;
        const int64_t src = pd.perm ? pd.perm[t] : t;
        Wt[e] = c < pd.Q ? W[src * pd.ldw + c] : T(0);
    }
}

template <typename T>
__global__ void k_permute_out_batched(const PermDesc *__restrict__ d) {
    const PermDesc pd = d[blockIdx.y];
    const int64_t total = pd.N * pd.Q;
    const T *Yt = (const T *)pd.Yt;
    T *Y = (T *)pd.Y;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / pd.Q, c = e % pd.Q;
        const int64_t dst = pd.perm ? pd.perm[t] : t;
        Y[dst * pd.ldy + c] = Yt[t * pd.ldq + c];
    }
}

// Served sweeps: the columns of a sweep belong to several requests (col2req
// maps a column to its request).  One thread per (tree row, column).
template <typename T>
__global__ void k_gather_in(const ReqDesc *__restrict__ reqs, const int16_t *__restrict__ col2req, int64_t cols,
                            int64_t width, T *__restrict__ Wt, int64_t ldt, const int64_t *__restrict__ perm,
                            int64_t N) {
    const int64_t total = N * width;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / width, c = e % width;
        T v = T(0);
        if (c < cols) {
            const ReqDesc &r = reqs[col2req[c]];
            v = ((const T *)r.W)[perm[t] * r.ldw + (c - r.col0)];
        }
        Wt[t * ldt + c] = v;
    }
}

template <typename T>
__global__ void k_scatter_out(const ReqDesc *__restrict__ reqs, const int16_t *__restrict__ col2req, int64_t cols,
                              const T *__restrict__ Yt, int64_t ldt, const int64_t *__restrict__ perm, int64_t N) {
    const int64_t total = N * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / cols, c = e % cols;
        const ReqDesc &r = reqs[col2req[c]];
        ((T *)r.Y)[perm[t] * r.ldy + (c - r.col0)] = Yt[t * ldt + c];
    }
}

__global__ void k_f64_to_f32(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        d[e] = (float)s[e];
}

int grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

template <typename T, int BM, int BN, int WM_, int WN_>
hipError_t run(const Phase &ph, const hm_matrix_s *h, const T *store, void *const bufs[4],
               int64_t ldq, hipStream_t s) {
    dim3 grid((unsigned)ph.task_count, (unsigned)(ldq / BN));
    if (h->symmetric)
        hipLaunchKernelGGL((k_block_products<T, BM, BN, WM_, WN_, true>), grid, dim3(64 * WM_ * WN_), 0, s,
                           h->d_tasks, h->d_segs, ph.task_begin, store, (T *)bufs[0], (T *)bufs[1],
                           (T *)bufs[2], (T *)bufs[3], ldq);
    else
        hipLaunchKernelGGL((k_block_products<T, BM, BN, WM_, WN_, false>), grid, dim3(64 * WM_ * WN_), 0, s,
                           h->d_tasks, h->d_segs, ph.task_begin, store, (T *)bufs[0], (T *)bufs[1],
                           (T *)bufs[2], (T *)bufs[3], ldq);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch(const hm_matrix_s *h, const Phase &ph, int bn, int64_t ldq,
                    void *const bufs[4], hipStream_t s) {
    const T *store = (const T *)h->prec[sizeof(T) == 8 ? HM_PREC_FP64 : HM_PREC_FP32].blocks;
    if (ph.bm == 128) {
        switch (bn) {
            case 16: return run<T, 128, 16, 4, 1>(ph, h, store, bufs, ldq, s);
            case 32: return run<T, 128, 32, 4, 1>(ph, h, store, bufs, ldq, s);
            case 64: return run<T, 128, 64, 2, 2>(ph, h, store, bufs, ldq, s);
            case 128: return run<T, 128, 128, 2, 2>(ph, h, store, bufs, ldq, s);
            default: return run<T, 128, 256, 2, 4>(ph, h, store, bufs, ldq, s);
        }
    }
    switch (bn) {
        case 16: return run<T, 64, 16, 4, 1>(ph, h, store, bufs, ldq, s);
        case 32: return run<T, 64, 32, 4, 1>(ph, h, store, bufs, ldq, s);
        case 64: return run<T, 64, 64, 2, 2>(ph, h, store, bufs, ldq, s);
        case 128: return run<T, 64, 128, 1, 4>(ph, h, store, bufs, ldq, s);
        default: return run<T, 64, 256, 1, 4>(ph, h, store, bufs, ldq, s);
    }
}

}  // namespace

int pick_bn(int64_t Q, int kind) {
    (void)kind;
    if (Q <= 16) return 16;
    if (Q <= 32) return 32;
    if (Q <= 64) return 64;
    if (Q <= 128) return 128;
    return 256;
}

int graph_bn(int64_t Q, int elem_bytes, bool split, double task_k) {
    const int bn = pick_bn(Q, 3);
    // Tiles up to 128 columns fit two workgroups per compute unit (at most
    // 128 VGPRs, see k_persistent), so one workgroup's task switches (fetch,
    // pipeline fill, epilogue) and barriers overlap the other's MFMAs.  That
    // pays when tasks are short.  An FP64 graph whose work sits in long
    // contractions (a flop's task has task_k > 8192 contraction rows) keeps
    // the 256-wide tile, which reads the block store half as often.  The
    // split-BF16 instantiation does not fit two workgroups and keeps it too.
    if (split || (elem_bytes == 8 && task_k > 8192.0)) return bn;
    return std::min(bn, 128);
}

hipError_t launch_phase(const hm_matrix_s *h, const Phase &ph, int elem_bytes, int bn, int64_t ldq,
                        void *const bufs[BUF_COUNT], hipStream_t s) {
    if (ph.task_count == 0) return hipSuccess;
    return elem_bytes == 8 ? dispatch<double>(h, ph, bn, ldq, bufs, s)
                           : dispatch<float>(h, ph, bn, ldq, bufs, s);
}

namespace {

template <typename T, int BN>
hipError_t run_persistent(const GraphPlan &plan, const MatDesc *mats, int32_t *head, int grid,
                          const OutScatter &out, int32_t *counters, hipStream_t s) {
    const int nt = plan.n_tasks;
    if (plan.narrow && (plan.sym || plan.mode == 1 || out.from_points || BN != 256)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_persistent_init, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s,
                       plan.d_tasks, nt, counters, head);
    if constexpr (sizeof(T) == 8 && BN != 64) {
        if (out.from_points) {
            if (plan.sym)  // stored blocks of a symmetric store may be mirrors
                hipLaunchKernelGGL((k_persistent<T, BN, false, true, true>), dim3((unsigned)grid),
                                   dim3(kPersistThreads), 0, s, plan.d_tasks, nt, plan.d_succ, counters, head,
                                   head + 1, mats, out.Y, out.ldy, out.Q, out.perm);
            else
                hipLaunchKernelGGL((k_persistent<T, BN, false, true>), dim3((unsigned)grid), dim3(kPersistThreads),
                                   0, s, plan.d_tasks, nt, plan.d_succ, counters, head, head + 1, mats, out.Y,
                                   out.ldy, out.Q, out.perm);
            return hipGetLastError();
        }
    }
    if (out.from_points) return hipErrorInvalidValue;
    if (sizeof(T) == 8 && plan.mode == 1)
        hipLaunchKernelGGL((k_persistent<T, BN, true>), dim3((unsigned)grid), dim3(kPersistThreads), 0,
                           s, plan.d_tasks, nt, plan.d_succ, counters, head, head + 1, mats, out.Y,
                           out.ldy, out.Q, out.perm);
    else if (plan.sym)
        hipLaunchKernelGGL((k_persistent<T, BN, false, false, true>), dim3((unsigned)grid), dim3(kPersistThreads),
                           0, s, plan.d_tasks, nt, plan.d_succ, counters, head, head + 1, mats, out.Y,
                           out.ldy, out.Q, out.perm);
    else if (plan.narrow) {
        if constexpr (BN == 256)
            hipLaunchKernelGGL((k_persistent<T, BN, false, false, false, true>), dim3((unsigned)grid),
                               dim3(kPersistThreads), 0, s, plan.d_tasks, nt, plan.d_succ, counters, head, head + 1,
                               mats, out.Y, out.ldy, out.Q, out.perm);
        else
            return hipErrorInvalidValue;
    }
    else
        hipLaunchKernelGGL((k_persistent<T, BN, false>), dim3((unsigned)grid), dim3(kPersistThreads), 0,
                           s, plan.d_tasks, nt, plan.d_succ, counters, head, head + 1, mats, out.Y,
                           out.ldy, out.Q, out.perm);
    return hipGetLastError();
}

template <typename T>
hipError_t persistent_bn(const GraphPlan &plan, const MatDesc *mats, int32_t *head, int grid,
                         const OutScatter &out, int32_t *counters, hipStream_t s) {
    switch (plan.bn) {
        case 16: return run_persistent<T, 16>(plan, mats, head, grid, out, counters, s);
        case 32: return run_persistent<T, 32>(plan, mats, head, grid, out, counters, s);
        case 64: return run_persistent<T, 64>(plan, mats, head, grid, out, counters, s);
        case 128: return run_persistent<T, 128>(plan, mats, head, grid, out, counters, s);
        default: return run_persistent<T, 256>(plan, mats, head, grid, out, counters, s);
    }
}

template <typename T, bool SPLIT, bool SYM = false, bool NARROW = false>
int occupancy_bn(int bn) {
    int n = 0;
    hipError_t e = hipSuccess;
    switch (bn) {
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, 16, SPLIT, false, SYM>, kPersistThreads, 0); break;
        case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, 32, SPLIT, false, SYM>, kPersistThreads, 0); break;
        case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, 64, SPLIT, false, SYM>, kPersistThreads, 0); break;
        case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, 128, SPLIT, false, SYM>, kPersistThreads, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, 256, SPLIT, false, SYM, NARROW>, kPersistThreads, 0); break;
    }
    return e == hipSuccess ? std::max(n, 1) : 1;
}

}  // namespace

hipError_t launch_persistent(const GraphPlan &plan, int elem_bytes, const MatDesc *d_mat,
                             int32_t *d_head, int grid, hipStream_t s, const OutScatter &out,
                             int32_t *counters) {
    if (plan.n_tasks == 0) return hipSuccess;
    int32_t *c = counters ? counters : plan.d_counters;
    return elem_bytes == 8 ? persistent_bn<double>(plan, d_mat, d_head, grid, out, c, s)
                           : persistent_bn<float>(plan, d_mat, d_head, grid, out, c, s);
}

int persistent_occupancy(int elem_bytes, int bn, bool split, bool sym, bool narrow) {
    narrow = narrow && !split && !sym && bn == 256;
    if (elem_bytes == 8)
        return split ? occupancy_bn<double, true>(bn) : sym ? occupancy_bn<double, false, true>(bn)
               : narrow ? occupancy_bn<double, false, false, true>(bn) : occupancy_bn<double, false>(bn);
    return sym ? occupancy_bn<float, false, true>(bn)
               : narrow ? occupancy_bn<float, false, false, true>(bn) : occupancy_bn<float, false>(bn);
}

hipError_t launch_permute_in(const void *W, int64_t ldw, void *Wt, int64_t Qp, const int64_t *perm,
                             int64_t N, int64_t Q, int elem_bytes, hipStream_t s) {
    const int g = grid_for(N * Qp, 256);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_permute_in<double>, dim3(g), dim3(256), 0, s, (const double *)W, ldw,
                           (double *)Wt, Qp, perm, N, Q);
    else
        hipLaunchKernelGGL(k_permute_in<float>, dim3(g), dim3(256), 0, s, (const float *)W, ldw,
                           (float *)Wt, Qp, perm, N, Q);
    return hipGetLastError();
}

hipError_t launch_permute_out(const void *Yt, int64_t Qp, void *Y, int64_t ldy, const int64_t *perm,
                              int64_t N, int64_t Q, int elem_bytes, hipStream_t s) {
    const int g = grid_for(N * Q, 256);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_permute_out<double>, dim3(g), dim3(256), 0, s, (const double *)Yt, Qp,
                           (double *)Y, ldy, perm, N, Q);
    else
        hipLaunchKernelGGL(k_permute_out<float>, dim3(g), dim3(256), 0, s, (const float *)Yt, Qp,
                           (float *)Y, ldy, perm, N, Q);
    return hipGetLastError();
}

hipError_t launch_permute_batched(const PermDesc *d, int n, int64_t max_elems, int elem_bytes,
                                  bool in, hipStream_t s) {
    const dim3 grid((unsigned)std::min<int64_t>(std::max<int64_t>((max_elems + 255) / 256, 1), 2048),
                    (unsigned)n);
    if (in) {
        if (elem_bytes == 8)
            hipLaunchKernelGGL(k_permute_in_batched<double>, grid, dim3(256), 0, s, d);
        else
            hipLaunchKernelGGL(k_permute_in_batched<float>, grid, dim3(256), 0, s, d);
    } else {
        if (elem_bytes == 8)
            hipLaunchKernelGGL(k_permute_out_batched<double>, grid, dim3(256), 0, s, d);
        else
            hipLaunchKernelGGL(k_permute_out_batched<float>, grid, dim3(256), 0, s, d);
    }
    return hipGetLastError();
}

hipError_t launch_repack(const double *stage, const RepackJob *jobs, int njobs, double *store,
                         hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_repack, dim3((unsigned)njobs), dim3(256), 0, s, stage, jobs, store);
    return hipGetLastError();
}

hipError_t launch_permute_in_split(const double *W, int64_t ldw, void *W16, int64_t ldq, const int64_t *perm,
                                   const int64_t *chunks, int64_t n_chunks, int64_t Q, hipStream_t s) {
    if (n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_in_split, dim3(grid_for(n_chunks * ldq, 256)), dim3(256), 0, s, W, ldw,
                       (__bf16 *)W16, ldq, perm, chunks, n_chunks, Q);
    return hipGetLastError();
}

hipError_t launch_make_bf16x3(const double *store, const Seg *segs, int nsegs, void *store16,
                              hipStream_t s) {
    if (nsegs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_bf16x3, dim3((unsigned)nsegs), dim3(256), 0, s, store, segs,
                       (__bf16 *)store16);
    return hipGetLastError();
}

hipError_t launch_gather_in(const ReqDesc *reqs, const int16_t *col2req, int64_t cols, int64_t width,
                            void *Wt, int64_t ldt, const int64_t *perm, int64_t N, int elem_bytes, hipStream_t s) {
    const int g = grid_for(N * width, 256);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_gather_in<double>, dim3(g), dim3(256), 0, s, reqs, col2req, cols, width, (double *)Wt,
                           ldt, perm, N);
    else
        hipLaunchKernelGGL(k_gather_in<float>, dim3(g), dim3(256), 0, s, reqs, col2req, cols, width, (float *)Wt,
                           ldt, perm, N);
    return hipGetLastError();
}

hipError_t launch_scatter_out(const ReqDesc *reqs, const int16_t *col2req, int64_t cols, const void *Yt,
                              int64_t ldt, const int64_t *perm, int64_t N, int elem_bytes, hipStream_t s) {
    const int g = grid_for(N * cols, 256);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_scatter_out<double>, dim3(g), dim3(256), 0, s, reqs, col2req, cols,
                           (const double *)Yt, ldt, perm, N);
    else
        hipLaunchKernelGGL(k_scatter_out<float>, dim3(g), dim3(256), 0, s, reqs, col2req, cols,
                           (const float *)Yt, ldt, perm, N);
    return hipGetLastError();
}

hipError_t launch_convert_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace hm
