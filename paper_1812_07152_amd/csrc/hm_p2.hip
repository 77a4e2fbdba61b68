// hm_p2.hip -- inspector-p2 on the GPU: the low-rank approximation of every
// node (interpolative decomposition, Section 3.1) and the near and far
// blocks, for a kernel function and an accuracy, on the inspector-p1
// structure (tree, interaction lists, row samples) kept from an earlier run
// (Section 5 "Reusing Inspection").
//
// Per tree level, deepest first, and per node a of the level:
//   1. A = K(X[rows(a)], X[cand(a)]) is formed on the device (k_gen_a), with
//      rows(a) the node's row sample and cand(a) its candidate columns: the
//      leaf's points, or the skeletons of its two children;
//   2. the Gram matrix G = A^T A on the FP64 matrix cores (k_gram);
//   3. a pivoted partial Cholesky of G (k_pchol).  Column-pivoted QR of A and
//      diagonally pivoted Cholesky of A^T A choose the same pivots and give
//      the same |R_jj| in exact arithmetic: the Schur complement's diagonal
//      entry of a column is the squared norm of that column's part orthogonal
//      to the chosen columns, the quantity the QR pivot maximises.  The rank
//      is the first j with R_jj <= tol R_11 (capped), and the interpolation
//      matrix [I, R11^-1 R12] in pivot order comes from a triangular solve on
//      the Cholesky factor.
// Numerics: the Gram form resolves R_jj down to about sqrt(c eps) R_11, far
// below the tolerances used (>= 1e-7 relative), and the residual of the
// resulting interpolation is within about cond(A_skel) eps |A| of the
// least-squares one.
// The blocks B_ab = K(X[skel_a], X[skel_b]) and D_ab = K(X[I_a], X[I_b]) are
// generated on the device as well: into host arrays (k_gen_blocks, for a
// representation on the host) or straight into the padded K-major device
// store of the evaluation (k_gen_store, for a matrix built on the device).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hm_internal.h"

namespace hm {
namespace {

constexpr int kP2Threads = 256;
constexpr int kP2MaxCols = 2048;   // candidate columns of one ID (leaf size, or twice the rank cap)
constexpr int kP2MaxRank = 1024;

typedef double d4_t __attribute__((ext_vector_type(4)));

// One node's ID inside a level batch; every offset is in elements.
struct P2Node {
    int64_t a_off;     // A: mrp x ncp, row-major, zero past (mr, nc)
    int64_t g_off;     // G: ncp x ncp, row-major
    int64_t l_off;     // Cholesky factor, step-major: L[t * nc + c] for step t < cap
    int64_t p_off;     // interpolation matrix, row-major cap x nc (first k rows valid)
    int64_t rows_off;  // row sample (original point indices) in the rows array
    int64_t cand_off;  // candidate columns (original point indices) in the candidate array
    int32_t mr, mrp, nc, ncp, cap, slot;  // slot: index of the node's rank and skeleton outputs
};

// One block to generate: rows x cols values K(x_r, x_c), row-major at out_off,
// rows and columns taken from the index array at r_off and c_off.
struct BlockJob {
    int64_t out_off, r_off, c_off;
    int32_t rows, cols;
};

__device__ __forceinline__ double kernel_value(const double *__restrict__ x, const double *__restrict__ y, int d,
                                               int kern, double kscale) {
    double r2 = 0.0;
    for (int t = 0; t < d; t++) {
        const double df = x[t] - y[t];
        r2 += df * df;
    }
    return kern == 0 ? exp(-r2 * kscale) : exp(-sqrt(r2) * kscale);
}

// A of each node, 16 rows per workgroup: chunk b covers rows [row0, row0 + 16)
// of node chunks[2b].
__global__ __launch_bounds__(kP2Threads) void k_gen_a(const P2Node *__restrict__ nodes,
                                                      const int32_t *__restrict__ chunks,
                                                      const double *__restrict__ X, int d, int kern, double kscale,
                                                      const int64_t *__restrict__ rows,
                                                      const int64_t *__restrict__ cand, double *__restrict__ A) {
    const P2Node nd = nodes[chunks[2 * blockIdx.x]];
    const int row0 = chunks[2 * blockIdx.x + 1];
    const int n = 16 * nd.ncp;
    for (int e = threadIdx.x; e < n; e += kP2Threads) {
        const int r = e / nd.ncp, c = e - r * nd.ncp, i = row0 + r;
        double v = 0.0;
        if (i < nd.mr && c < nd.nc)
            v = kernel_value(X + rows[nd.rows_off + i] * d, X + cand[nd.cand_off + c] * d, d, kern, kscale);
        A[nd.a_off + (int64_t)i * nd.ncp + c] = v;
    }
}

// G = A^T A, one 64 x 64 tile (ti <= tj) per workgroup; the tile is also
// written mirrored.  Four wave64s, each a 32 x 32 quarter of 2 x 2 MFMA
// fragments (v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l is D[4r + l/16][l%16]).
__global__ __launch_bounds__(kP2Threads) void k_gram(const P2Node *__restrict__ nodes,
                                                     const int32_t *__restrict__ tiles,
                                                     const double *__restrict__ A, double *__restrict__ G) {
    const P2Node nd = nodes[tiles[3 * blockIdx.x]];
    const int ti = tiles[3 * blockIdx.x + 1], tj = tiles[3 * blockIdx.x + 2];
    __shared__ double sa[16][64], sb[16][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    d4_t acc[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
    const double *An = A + nd.a_off;
    for (int i0 = 0; i0 < nd.mrp; i0 += 16) {
        for (int e = tid; e < 16 * 64; e += kP2Threads) {
            const int r = e >> 6, c = e & 63;
            const int64_t o = (int64_t)(i0 + r) * nd.ncp;
            sa[r][c] = An[o + ti * 64 + c];
            sb[r][c] = An[o + tj * 64 + c];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const int kr = kk + (lane >> 4);
            double a[2], b[2];
#pragma unroll
            for (int f = 0; f < 2; f++) {
                a[f] = sa[kr][wm * 32 + f * 16 + (lane & 15)];
                b[f] = sb[kr][wn * 32 + f * 16 + (lane & 15)];
            }
#pragma unroll
            for (int fm = 0; fm < 2; fm++)
#pragma unroll
                for (int fn = 0; fn < 2; fn++)
                    acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[fm], b[fn], acc[fm][fn], 0, 0, 0);
        }
        __syncthreads();
    }
    double *Gn = G + nd.g_off;
#pragma unroll
    for (int fm = 0; fm < 2; fm++)
#pragma unroll
        for (int fn = 0; fn < 2; fn++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int row = ti * 64 + wm * 32 + fm * 16 + 4 * r + (lane >> 4);
                const int col = tj * 64 + wn * 32 + fn * 16 + (lane & 15);
                Gn[(int64_t)row * nd.ncp + col] = acc[fm][fn][r];
                if (ti != tj) Gn[(int64_t)col * nd.ncp + row] = acc[fm][fn][r];
            }
}

// Pivoted partial Cholesky of G and the interpolation matrix, one node per
// workgroup.  Left-looking: step j takes the column p of largest remaining
// Schur diagonal (lowest position on ties, positions as reordered by the
// earlier swaps), forms L[j][c] = (G[c][p] - sum_{t<j} L[t][c] L[t][p]) / R_jj
// and downdates the diagonal.  With R = L^T in pivot order, R11 is k x k upper
// triangular and R12 its remaining columns; P[:, piv[i]] = e_i and
// P[:, piv[k+c]] = (R11^-1 R12)[:, c].
__global__ __launch_bounds__(kP2Threads) void k_pchol(const P2Node *__restrict__ nodes, const double *__restrict__ G,
                                                      double *__restrict__ L, double *__restrict__ P, double tol,
                                                      const int64_t *__restrict__ cand, int32_t *__restrict__ rank_out,
                                                      int64_t *__restrict__ skel_out, int skel_stride) {
    const P2Node nd = nodes[blockIdx.x];
    __shared__ double dg[kP2MaxCols];
    __shared__ int piv[kP2MaxCols];
    __shared__ unsigned char done[kP2MaxCols];
    __shared__ double lp[kP2MaxRank];
    __shared__ double red_v[kP2Threads / 64];
    __shared__ int red_q[kP2Threads / 64];
    __shared__ int s_k;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nc = nd.nc, ncp = nd.ncp;
    const double *Gn = G + nd.g_off;
    double *Ln = L + nd.l_off;
    double *Pn = P + nd.p_off;
    for (int c = tid; c < nc; c += kP2Threads) {
        dg[c] = Gn[(int64_t)c * ncp + c];
        piv[c] = c;
        done[c] = 0;
    }
    __syncthreads();
    double r11 = 0.0;
    int k = 0;
    for (int j = 0;; j++) {
        if (j >= nd.cap) {
            k = j;
            break;
        }
        // argmax of the remaining diagonal over positions [j, nc)
        double best = -1.0;
        int bq = nc;
        for (int q = j + tid; q < nc; q += kP2Threads) {
            const double v = dg[piv[q]];
            if (v > best) {
                best = v;
                bq = q;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(best, off);
            const int oq = __shfl_xor(bq, off);
            if (ov > best || (ov == best && oq < bq)) {
                best = ov;
                bq = oq;
            }
        }
        if (lane == 0) {
            red_v[wave] = best;
            red_q[wave] = bq;
        }
        __syncthreads();
        best = red_v[0];
        bq = red_q[0];
        for (int w = 1; w < kP2Threads / 64; w++)
            if (red_v[w] > best || (red_v[w] == best && red_q[w] < bq)) {
                best = red_v[w];
                bq = red_q[w];
            }
        const double rjj = sqrt(fmax(best, 0.0));
        if (j == 0) r11 = rjj;
        if (rjj == 0.0 || (j > 0 && rjj <= tol * r11)) {
            k = j;
            break;
        }
        __syncthreads();  // every thread has read red_v / red_q and piv
        if (tid == 0) {
            const int t = piv[j];
            piv[j] = piv[bq];
            piv[bq] = t;
        }
        __syncthreads();
        const int p = piv[j];
        for (int t = tid; t < j; t += kP2Threads) lp[t] = Ln[(int64_t)t * nc + p];
        __syncthreads();
        for (int c = tid; c < nc; c += kP2Threads) {
            double v;
            if (c == p) {
                v = rjj;
            } else if (done[c]) {
                v = 0.0;
            } else {
                double s = Gn[(int64_t)c * ncp + p];
                for (int t = 0; t < j; t++) s -= Ln[(int64_t)t * nc + c] * lp[t];
                v = s / rjj;
                dg[c] -= v * v;
            }
            Ln[(int64_t)j * nc + c] = v;
        }
        if (tid == 0) done[p] = 1;
        __syncthreads();
    }
    if (tid == 0) s_k = k;
    __syncthreads();
    k = s_k;
    __threadfence_block();
    // R11[i][t] = L[i][piv[t]], R12[i][c] = L[i][c]; T = R11^-1 R12 by back substitution,
    // one non-skeleton column per thread, written straight into P
    for (int q = k + tid; q < nc; q += kP2Threads) {
        const int c = piv[q];
        for (int i = k - 1; i >= 0; i--) {
            double s = Ln[(int64_t)i * nc + c];
            for (int t = i + 1; t < k; t++) s -= Ln[(int64_t)i * nc + piv[t]] * Pn[(int64_t)t * nc + c];
            Pn[(int64_t)i * nc + c] = s / Ln[(int64_t)i * nc + piv[i]];
        }
    }
    for (int e = tid; e < k * k; e += kP2Threads) {
        const int i = e / k, t = e - i * k;
        Pn[(int64_t)i * nc + piv[t]] = i == t ? 1.0 : 0.0;
    }
    for (int i = tid; i < k; i += kP2Threads) skel_out[(int64_t)nd.slot * skel_stride + i] = cand[nd.cand_off + piv[i]];
    if (tid == 0) rank_out[nd.slot] = k;
}

// Blocks of kernel values: job blockIdx.x, rows [16 blockIdx.y, +16).
__global__ __launch_bounds__(kP2Threads) void k_gen_blocks(const BlockJob *__restrict__ jobs,
                                                           const double *__restrict__ X, int d, int kern,
                                                           double kscale, const int64_t *__restrict__ idx,
                                                           double *__restrict__ out) {
    const BlockJob jb = jobs[blockIdx.x];
    const int r0 = 16 * blockIdx.y;
    if (r0 >= jb.rows) return;
    const int nr = min(16, jb.rows - r0);
    const int n = nr * jb.cols;
    for (int e = threadIdx.x; e < n; e += kP2Threads) {
        const int r = e / jb.cols, c = e - r * jb.cols;
        out[jb.out_off + (int64_t)(r0 + r) * jb.cols + c] =
            kernel_value(X + idx[jb.r_off + r0 + r] * d, X + idx[jb.c_off + c] * d, d, kern, kscale);
    }
}

// Far and near blocks generated in the device store (see GenJob): one block
// per workgroup, columns t of the block over the lanes' rows i, so that each
// contraction row of the K-major block is written with consecutive lanes.
__global__ __launch_bounds__(kP2Threads) void k_gen_store(const GenJob *__restrict__ jobs,
                                                          const double *__restrict__ X, int d, int kern,
                                                          double kscale, const int64_t *__restrict__ idx,
                                                          double *__restrict__ store) {
    const GenJob jb = jobs[blockIdx.x];
    double *dst = store + jb.dst_off;
    const int n = jb.cols * jb.ld;
    for (int e = threadIdx.x; e < n; e += kP2Threads) {
        const int t = e / jb.ld, i = e - t * jb.ld;
        dst[e] = i < jb.rows ? kernel_value(X + idx[jb.r_off + i] * d, X + idx[jb.c_off + t] * d, d, kern, kscale)
                             : 0.0;
    }
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t ensure(size_t b) {
        b = std::max<size_t>(b, 256);
        if (bytes >= b) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            bytes = 0;
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    template <typename T>
    T *as() const {
        return (T *)p;
    }
};

#define P2_HIP(call)                                                                                    \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return fail(e_ == hipErrorOutOfMemory ? HM_ERR_NOMEM : HM_ERR_DEVICE,                       \
                        std::string("hm_inspect_p2: " #call ": ") + hipGetErrorString(e_));            \
    } while (0)

struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

constexpr size_t kP2BatchBytes = (size_t)4 << 30;  // workspace of one level batch (A, G, L, P)

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace

hipError_t launch_gen_store(const GenJob *jobs, int njobs, const BlockSource &src, double *store, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_store, dim3((unsigned)njobs), dim3(kP2Threads), 0, s, jobs, src.X, src.d, src.kern,
                       src.kscale, src.idx, store);
    return hipGetLastError();
}

// mat == nullptr: the blocks are generated and copied into out's host arrays.
// Otherwise the matrix is built on the device (prec_mask as for
// hm_load_compressed_mem) with its blocks generated in the device store, and
// out receives the representation without block values.
hm_status p2_run(const Structure &S, int device, int kern, double h, double tol, int rmax, hm_repr_s &out,
                 unsigned prec_mask = 0, hm_matrix *mat = nullptr) {
    const HostRepr &T = S.r;
    const int n = T.n_nodes;
    const int64_t N = T.N, d = T.d;
    HostRepr R;  // the result: the structure's tree and lists, plus ranks, bases and blocks
    R.N = N;
    R.d = d;
    R.n_nodes = n;
    R.depth = T.depth;
    R.perm = T.perm;
    R.start = T.start;
    R.size = T.size;
    R.parent = T.parent;
    R.left = T.left;
    R.right = T.right;
    R.level = T.level;
    R.far_ptr = T.far_ptr;
    R.far_col = T.far_col;
    R.near_ptr = T.near_ptr;
    R.near_col = T.near_col;
    R.rank.assign(n, 0);
    const double kscale = kern == 0 ? 1.0 / (2.0 * h * h) : 1.0 / h;

    DeviceScope ds(device);
    if (ds.err != hipSuccess) return fail(HM_ERR_DEVICE, "hm_inspect_p2: cannot select the device");
    hipStream_t s = nullptr;
    DevBuf dX, dRows, dCand, dNodes, dChunks, dTiles, dA, dG, dL, dP, dRank, dSkel;
    P2_HIP(dX.ensure(sizeof(double) * (size_t)(N * d)));
    P2_HIP(hipMemcpy(dX.p, S.X.data(), sizeof(double) * (size_t)(N * d), hipMemcpyHostToDevice));
    P2_HIP(dRows.ensure(sizeof(int64_t) * std::max<size_t>(S.rows.size(), 1)));
    if (!S.rows.empty())
        P2_HIP(hipMemcpy(dRows.p, S.rows.data(), sizeof(int64_t) * S.rows.size(), hipMemcpyHostToDevice));

    std::vector<std::vector<int64_t>> skel((size_t)n);
    std::vector<std::vector<double>> basis((size_t)n);
    for (int lev = T.depth; lev >= 0; lev--) {
        std::vector<int> todo;
        for (int a = 0; a < n; a++) {
            if (T.level[a] != lev) continue;
            const int64_t mr = S.rows_ptr[(size_t)a + 1] - S.rows_ptr[(size_t)a];
            const int64_t nc = T.left[a] < 0 ? T.size[a]
                                             : (int64_t)(skel[(size_t)T.left[a]].size() + skel[(size_t)T.right[a]].size());
            if (mr > 0 && nc > 0) todo.push_back(a);
        }
        size_t next = 0;
        while (next < todo.size()) {
            // one batch: nodes in order while the workspaces stay under kP2BatchBytes
            std::vector<P2Node> nodes;
            std::vector<int64_t> cand;
            std::vector<int32_t> chunks, tiles;
            int64_t a_el = 0, g_el = 0, l_el = 0;
            std::vector<int> batch;
            while (next < todo.size()) {
                const int a = todo[next];
                std::vector<int64_t> c;
                if (T.left[a] < 0) {
                    for (int64_t t = 0; t < T.size[a]; t++) c.push_back(T.perm[(size_t)(T.start[a] + t)]);
                } else {
                    c = skel[(size_t)T.left[a]];
                    c.insert(c.end(), skel[(size_t)T.right[a]].begin(), skel[(size_t)T.right[a]].end());
                }
                P2Node nd{};
                nd.mr = (int32_t)(S.rows_ptr[(size_t)a + 1] - S.rows_ptr[(size_t)a]);
                nd.nc = (int32_t)c.size();
                nd.mrp = (int32_t)round_up(nd.mr, 16);
                nd.ncp = (int32_t)round_up(nd.nc, 64);
                nd.cap = std::min({rmax, nd.nc, nd.mr});
                const int64_t ab = (int64_t)nd.mrp * nd.ncp, gb = (int64_t)nd.ncp * nd.ncp,
                              lb = (int64_t)std::max(nd.cap, 1) * nd.nc;
                if (!nodes.empty() && (size_t)(a_el + ab + gb + g_el + 2 * (lb + l_el)) * 8 > kP2BatchBytes) break;
                nd.a_off = a_el;
                nd.g_off = g_el;
                nd.l_off = l_el;
                nd.p_off = l_el;
                nd.rows_off = S.rows_ptr[(size_t)a];
                nd.cand_off = (int64_t)cand.size();
                nd.slot = (int32_t)nodes.size();
                for (int r0 = 0; r0 < nd.mrp; r0 += 16) {
                    chunks.push_back(nd.slot);
                    chunks.push_back(r0);
                }
                const int nt = nd.ncp / 64;
                for (int ti = 0; ti < nt; ti++)
                    for (int tj = ti; tj < nt; tj++) {
                        tiles.push_back(nd.slot);
                        tiles.push_back(ti);
                        tiles.push_back(tj);
                    }
                a_el += ab;
                g_el += gb;
                l_el += lb;
                cand.insert(cand.end(), c.begin(), c.end());
                nodes.push_back(nd);
                batch.push_back(a);
                next++;
            }
            const int nb = (int)nodes.size();
            int skel_stride = 0;
            for (const P2Node &nd : nodes) skel_stride = std::max(skel_stride, nd.cap);
            skel_stride = std::max(skel_stride, 1);
            P2_HIP(dNodes.ensure(sizeof(P2Node) * nodes.size()));
            P2_HIP(dCand.ensure(sizeof(int64_t) * cand.size()));
            P2_HIP(dChunks.ensure(sizeof(int32_t) * chunks.size()));
            P2_HIP(dTiles.ensure(sizeof(int32_t) * tiles.size()));
            P2_HIP(dA.ensure(sizeof(double) * (size_t)a_el));
            P2_HIP(dG.ensure(sizeof(double) * (size_t)g_el));
            P2_HIP(dL.ensure(sizeof(double) * (size_t)l_el));
            P2_HIP(dP.ensure(sizeof(double) * (size_t)l_el));
            P2_HIP(dRank.ensure(sizeof(int32_t) * (size_t)nb));
            P2_HIP(dSkel.ensure(sizeof(int64_t) * (size_t)nb * skel_stride));
            P2_HIP(hipMemcpy(dNodes.p, nodes.data(), sizeof(P2Node) * nodes.size(), hipMemcpyHostToDevice));
            P2_HIP(hipMemcpy(dCand.p, cand.data(), sizeof(int64_t) * cand.size(), hipMemcpyHostToDevice));
            P2_HIP(hipMemcpy(dChunks.p, chunks.data(), sizeof(int32_t) * chunks.size(), hipMemcpyHostToDevice));
            P2_HIP(hipMemcpy(dTiles.p, tiles.data(), sizeof(int32_t) * tiles.size(), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(k_gen_a, dim3((unsigned)(chunks.size() / 2)), dim3(kP2Threads), 0, s,
                               dNodes.as<P2Node>(), dChunks.as<int32_t>(), dX.as<double>(), (int)d, kern, kscale,
                               dRows.as<int64_t>(), dCand.as<int64_t>(), dA.as<double>());
            P2_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_gram, dim3((unsigned)(tiles.size() / 3)), dim3(kP2Threads), 0, s,
                               dNodes.as<P2Node>(), dTiles.as<int32_t>(), dA.as<double>(), dG.as<double>());
            P2_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_pchol, dim3((unsigned)nb), dim3(kP2Threads), 0, s, dNodes.as<P2Node>(),
                               dG.as<double>(), dL.as<double>(), dP.as<double>(), tol, dCand.as<int64_t>(),
                               dRank.as<int32_t>(), dSkel.as<int64_t>(), skel_stride);
            P2_HIP(hipGetLastError());
            std::vector<int32_t> ranks((size_t)nb);
            std::vector<int64_t> sk((size_t)nb * skel_stride);
            std::vector<double> pv((size_t)l_el);
            P2_HIP(hipMemcpy(ranks.data(), dRank.p, sizeof(int32_t) * ranks.size(), hipMemcpyDeviceToHost));
            P2_HIP(hipMemcpy(sk.data(), dSkel.p, sizeof(int64_t) * sk.size(), hipMemcpyDeviceToHost));
            P2_HIP(hipMemcpy(pv.data(), dP.p, sizeof(double) * pv.size(), hipMemcpyDeviceToHost));
            for (int i = 0; i < nb; i++) {
                const int a = batch[(size_t)i];
                const int k = ranks[(size_t)i];
                if (k < 0 || k > nodes[(size_t)i].cap) return fail(HM_ERR_INTERNAL, "hm_inspect_p2: bad rank");
                R.rank[a] = k;
                skel[(size_t)a].assign(sk.begin() + (size_t)i * skel_stride, sk.begin() + (size_t)i * skel_stride + k);
                const size_t off = (size_t)nodes[(size_t)i].p_off, len = (size_t)k * nodes[(size_t)i].nc;
                basis[(size_t)a].assign(pv.begin() + off, pv.begin() + off + len);
            }
        }
    }
    // bases, in node order
    R.basis_off.assign(n, 0);
    int64_t off = 0;
    for (int a = 0; a < n; a++) {
        R.basis_off[a] = off;
        off += (int64_t)basis[(size_t)a].size();
    }
    R.basis.resize((size_t)off);
    for (int a = 0; a < n; a++) std::copy(basis[(size_t)a].begin(), basis[(size_t)a].end(), R.basis.begin() + R.basis_off[a]);
    R.basis_len = off;
    // block offsets (far: k_a x k_b, near: |I_a| x |I_b|, row-major, CSR order)
    R.far_off.resize(R.far_col.size());
    R.near_off.resize(R.near_col.size());
    int64_t bo = 0, dof = 0;
    for (int a = 0; a < n; a++) {
        for (int64_t e = R.far_ptr[a]; e < R.far_ptr[a + 1]; e++) {
            R.far_off[e] = bo;
            bo += (int64_t)R.rank[a] * R.rank[R.far_col[e]];
        }
        for (int64_t e = R.near_ptr[a]; e < R.near_ptr[a + 1]; e++) {
            R.near_off[e] = dof;
            dof += R.size[a] * R.size[R.near_col[e]];
        }
    }
    if (!mat) {
        R.B.assign((size_t)bo, 0.0);
        R.D.assign((size_t)dof, 0.0);
    }
    R.B_len = bo;
    R.D_len = dof;
    // skeletons (original indices) and the index array of the block generator:
    // [perm | skeletons]
    out.skel_ptr.assign((size_t)n + 1, 0);
    out.skel.clear();
    for (int a = 0; a < n; a++) {
        out.skel_ptr[(size_t)a + 1] = out.skel_ptr[(size_t)a] + (int64_t)skel[(size_t)a].size();
        out.skel.insert(out.skel.end(), skel[(size_t)a].begin(), skel[(size_t)a].end());
    }
    R.kernel = kern;
    R.h = h;
    R.tol = tol;
    R.tau = T.tau;
    R.rmax = rmax;
    R.m = T.m;
    R.flags = T.flags;
    R.skel_ptr = out.skel_ptr;
    R.skel = out.skel;
    std::vector<int64_t> idx(R.perm);
    idx.insert(idx.end(), out.skel.begin(), out.skel.end());
    DevBuf dIdx;
    P2_HIP(dIdx.ensure(sizeof(int64_t) * idx.size()));
    P2_HIP(hipMemcpy(dIdx.p, idx.data(), sizeof(int64_t) * idx.size(), hipMemcpyHostToDevice));
    if (mat) {
        hm_status st = validate(R);
        if (st != HM_OK) return st;
        BlockSource gen;
        gen.X = dX.as<double>();
        gen.d = (int32_t)d;
        gen.kern = kern;
        gen.kscale = kscale;
        gen.idx = dIdx.as<int64_t>();
        st = build_matrix(R, device, prec_mask, mat, &gen);
        if (st != HM_OK) return st;
        out.r = std::move(R);
        return HM_OK;
    }
    {
        DevBuf dJobs, dOut;
        // jobs in batches of at most kP2BatchBytes of output
        struct Pending {
            std::vector<BlockJob> jobs;
            std::vector<double> *dst = nullptr;
            int64_t dst_off = 0, elems = 0;
            int max_rows = 0;
        } pend;
        auto flush = [&]() -> hm_status {
            if (pend.jobs.empty()) return HM_OK;
            P2_HIP(dJobs.ensure(sizeof(BlockJob) * pend.jobs.size()));
            P2_HIP(dOut.ensure(sizeof(double) * (size_t)pend.elems));
            P2_HIP(hipMemcpy(dJobs.p, pend.jobs.data(), sizeof(BlockJob) * pend.jobs.size(), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(k_gen_blocks, dim3((unsigned)pend.jobs.size(), (unsigned)((pend.max_rows + 15) / 16)),
                               dim3(kP2Threads), 0, s, dJobs.as<BlockJob>(), dX.as<double>(), (int)d, kern, kscale,
                               dIdx.as<int64_t>(), dOut.as<double>());
            P2_HIP(hipGetLastError());
            P2_HIP(hipMemcpy(pend.dst->data() + pend.dst_off, dOut.p, sizeof(double) * (size_t)pend.elems,
                             hipMemcpyDeviceToHost));
            pend.jobs.clear();
            pend.elems = 0;
            pend.max_rows = 0;
            return HM_OK;
        };
        auto add = [&](std::vector<double> &dst, int64_t dst_off, int64_t r_off, int32_t rows, int64_t c_off,
                       int32_t cols) -> hm_status {
            const int64_t el = (int64_t)rows * cols;
            if (el == 0) return HM_OK;
            if (!pend.jobs.empty() &&
                (pend.dst != &dst || pend.dst_off + pend.elems != dst_off ||
                 (size_t)(pend.elems + el) * 8 > kP2BatchBytes || pend.jobs.size() >= (1u << 20))) {
                hm_status st = flush();
                if (st != HM_OK) return st;
            }
            if (pend.jobs.empty()) {
                pend.dst = &dst;
                pend.dst_off = dst_off;
            }
            pend.jobs.push_back(BlockJob{pend.elems, r_off, c_off, rows, cols});
            pend.elems += el;
            pend.max_rows = std::max(pend.max_rows, (int)rows);
            return HM_OK;
        };
        const int64_t sk0 = N;  // skeletons start after perm in idx
        for (int a = 0; a < n; a++)
            for (int64_t e = R.far_ptr[a]; e < R.far_ptr[a + 1]; e++) {
                const int b = R.far_col[e];
                hm_status st = add(R.B, R.far_off[e], sk0 + out.skel_ptr[(size_t)a], R.rank[a],
                                   sk0 + out.skel_ptr[(size_t)b], R.rank[b]);
                if (st != HM_OK) return st;
            }
        {
            hm_status st = flush();
            if (st != HM_OK) return st;
        }
        for (int a = 0; a < n; a++)
            for (int64_t e = R.near_ptr[a]; e < R.near_ptr[a + 1]; e++) {
                const int b = R.near_col[e];
                hm_status st = add(R.D, R.near_off[e], R.start[a], (int32_t)R.size[a], R.start[b], (int32_t)R.size[b]);
                if (st != HM_OK) return st;
            }
        hm_status st = flush();
        if (st != HM_OK) return st;
    }
    hm_status st = validate(R);
    if (st != HM_OK) return st;
    out.r = std::move(R);
    return HM_OK;
}

hm_status p2_check(hm_structure s, int device, int32_t kernel, double h, double tol, int32_t max_rank) {
    if (!s) return fail(HM_ERR_INVALID, "hm_inspect_p2: structure is NULL");
    if ((kernel != 0 && kernel != 1) || !(h > 0.0) || !std::isfinite(h) || !(tol >= 0.0) || max_rank < 1 ||
        max_rank > kP2MaxRank)
        return fail(HM_ERR_INVALID, "hm_inspect_p2: invalid kernel, h, tol or max_rank");
    const Structure &S = s->s;
    for (int a = 0; a < S.r.n_nodes; a++)
        if (S.r.left[a] < 0 && S.r.size[a] > kP2MaxCols)
            return fail(HM_ERR_INVALID, "hm_inspect_p2: leaves of more than 2048 points");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(HM_ERR_INVALID, "hm_inspect_p2: no such HIP device");
    return HM_OK;
}

}  // namespace hm

using namespace hm;

extern "C" {

hm_status hm_inspect_p2(hm_structure s, int device, int32_t kernel, double h, double tol, int32_t max_rank,
                        hm_repr *out) {
    if (!out) return fail(HM_ERR_INVALID, "hm_inspect_p2: out is NULL");
    *out = nullptr;
    {
        hm_status st = p2_check(s, device, kernel, h, tol, max_rank);
        if (st != HM_OK) return st;
    }
    hm_repr r = new (std::nothrow) hm_repr_s();
    if (!r) return fail(HM_ERR_NOMEM, "hm_inspect_p2: allocation failed");
    hm_status st = p2_run(s->s, device, kernel, h, tol, max_rank, *r);
    if (st != HM_OK) {
        delete r;
        return st;
    }
    *out = r;
    return HM_OK;
}

hm_status hm_inspect_p2_load(hm_structure s, int device, int32_t kernel, double h, double tol, int32_t max_rank,
                             unsigned prec_mask, hm_matrix *out) {
    if (!out) return fail(HM_ERR_INVALID, "hm_inspect_p2_load: out is NULL");
    *out = nullptr;
    if (!(prec_mask & (HM_PRECBIT(HM_PREC_FP64) | HM_PRECBIT(HM_PREC_FP32) | HM_PRECBIT(HM_PREC_BF16X3))))
        return fail(HM_ERR_INVALID, "hm_inspect_p2_load: prec_mask selects no precision");
    if ((prec_mask & (HM_LOAD_NO_NEAR_BLOCKS | HM_LOAD_NO_FAR_BLOCKS)) &&
        (!(prec_mask & HM_PRECBIT(HM_PREC_FP64)) ||
         (prec_mask & (HM_PRECBIT(HM_PREC_FP32) | HM_PRECBIT(HM_PREC_BF16X3)))))
        return fail(HM_ERR_INVALID, "hm_inspect_p2_load: HM_LOAD_NO_NEAR_BLOCKS and HM_LOAD_NO_FAR_BLOCKS are for "
                                    "the FP64 store alone");
    {
        hm_status st = p2_check(s, device, kernel, h, tol, max_rank);
        if (st != HM_OK) return st;
    }
    hm_repr_s r;
    return p2_run(s->s, device, kernel, h, tol, max_rank, r, prec_mask, out);
}

}  // extern "C"
