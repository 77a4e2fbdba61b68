// hm_build.hip -- turn a validated representation into the device block store
// and the per-phase task tables of the evaluation.
//
// Phases, in launch order (Section 2.1 "Evaluation"; the loop structure of
// the paper's executor, re-cut into one launch per tree level):
//   up(l), l = deepest..1   nodes at level l with k > 0:
//                           What_a = P_a Wt[I_a] (leaf) or T_a [What_l; What_r]
//   down(l), l = 1..deepest nodes at level l with k > 0:
//                           Yhat_a = sum_{b in Far(a)} B_ab What_b
//                                    + T_p[:, cols(a)]^T Yhat_p   (p = parent)
//                           (the far reduction fused with the top-down pass)
//   leaf                    every leaf a:
//                           Yt[I_a] = sum_{b in Near(a)} D_ab Wt[I_b] + P_a^T Yhat_a
//                           (near reduction fused with the leaf far part and
//                           the final sum)
// The root has no far pairs (it overlaps every node), so it is skipped.
#include <algorithm>
#include <cstring>
#include <map>

#include "hm_internal.h"

namespace hm {

namespace {

// A symmetric store needs B_ba = B_ab^T and D_ba = D_ab^T (the kernel
// matrix is symmetric, Section 1; the oracle and the inspectors produce them
// bitwise): every pair must have its partner in the other node's list and
// the transposed values.
hm_status check_symmetric(const HostRepr &r, bool near, bool far) {
    auto find = [](const std::vector<int64_t> &ptr, const std::vector<int32_t> &col, int a, int b) -> int64_t {
        auto first = col.begin() + ptr[(size_t)a], last = col.begin() + ptr[(size_t)a + 1];
        auto it = std::lower_bound(first, last, b);
        return (it != last && *it == b) ? (int64_t)(it - col.begin()) : -1;
    };
    for (int a = 0; a < r.n_nodes; a++) {
        if (far)
            for (int64_t e = r.far_ptr[(size_t)a]; e < r.far_ptr[(size_t)a + 1]; e++) {
                const int b = r.far_col[(size_t)e];
                if (b <= a) continue;
                const int64_t f = find(r.far_ptr, r.far_col, b, a);
                if (f < 0) return fail(HM_ERR_FORMAT, "HM_LOAD_SYMMETRIC: far lists are not symmetric");
                const int64_t ka = r.rank[(size_t)a], kb = r.rank[(size_t)b];
                const double *x = r.B_ptr() + r.far_off[(size_t)e], *y = r.B_ptr() + r.far_off[(size_t)f];
                for (int64_t i = 0; i < ka; i++)
                    for (int64_t j = 0; j < kb; j++)
                        if (x[i * kb + j] != y[j * ka + i])
                            return fail(HM_ERR_FORMAT, "HM_LOAD_SYMMETRIC: a far block is not the transpose of its mirror");
            }
        if (near)
            for (int64_t e = r.near_ptr[(size_t)a]; e < r.near_ptr[(size_t)a + 1]; e++) {
                const int b = r.near_col[(size_t)e];
                if (b < a) continue;
                const int64_t f = find(r.near_ptr, r.near_col, b, a);
                if (f < 0) return fail(HM_ERR_FORMAT, "HM_LOAD_SYMMETRIC: near lists are not symmetric");
                const int64_t ma = r.size[(size_t)a], mb = r.size[(size_t)b];
                const double *x = r.D_ptr() + r.near_off[(size_t)e], *y = r.D_ptr() + r.near_off[(size_t)f];
                for (int64_t i = 0; i < ma; i++)
                    for (int64_t j = 0; j < mb; j++)
                        if (x[i * mb + j] != y[j * ma + i])
                            return fail(HM_ERR_FORMAT, "HM_LOAD_SYMMETRIC: a near block is not the transpose of its mirror");
            }
    }
    return HM_OK;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// b_row16: the B operand node's first row in its split-BF16 workspace
Seg seg(int64_t a_off, int64_t b_row, int32_t lda, int32_t K, int32_t buf, int64_t b_row16) {
    return Seg{a_off, b_row, lda, K, buf, (int32_t)round_up(K, 16), 0, b_row16, 0, 0};
}

struct Block {            // one output block of a phase before tiling
    int32_t out_buf;
    int64_t out_row;
    int32_t M;
    std::vector<Seg> segs;
    int32_t node = -1;
    int64_t work() const {
        int64_t k = 0;
        for (const Seg &s : segs) k += s.K;
        return k;
    }
};

struct Planner {
    int64_t store_off = 0;
    std::vector<RepackJob> jobs[3];  // per source: 0 basis, 1 B, 2 D
    std::vector<Task> tasks;
    std::vector<Seg> segs;
    std::vector<Phase> phases;
    struct Placed {
        int32_t kind, node, out_buf, M, seg_begin, seg_end;
        int64_t out_row, kpad;
    };
    std::vector<Placed> placed;  // every block with its segment range

    // Reserve a K-major block of `krows` contraction rows (padded with zero
    // rows to a multiple of 16) of `ld` elements each.
    int64_t alloc(int64_t krows, int64_t ld) {
        int64_t off = store_off;
        store_off += round_up(round_up(krows, 16) * ld, 32);  // 256-byte aligned blocks
        return off;
    }

    void add_phase(int kind, int level, std::vector<Block> &blocks) {
        if (blocks.empty()) return;
        Phase ph{};
        ph.kind = kind;
        ph.level = level;
        int32_t maxM = 0;
        for (const Block &b : blocks) maxM = std::max(maxM, b.M);
        // tile height: the one with less padded work (ties go to 128)
        double w64 = 0, w128 = 0;
        for (const Block &b : blocks) {
            w64 += (double)((b.M + 63) / 64) * 64 * b.work();
            w128 += (double)((b.M + 127) / 128) * 128 * b.work();
        }
        ph.bm = (maxM <= 64 || w64 < w128) ? 64 : 128;
        // longest contraction first: the hardware dispatcher then fills the
        // machine greedily (longest-processing-time order)
        std::stable_sort(blocks.begin(), blocks.end(),
                         [](const Block &x, const Block &y) { return x.work() > y.work(); });
        ph.task_begin = (int32_t)tasks.size();
        double flops = 0;
        for (const Block &b : blocks) {
            int32_t sb = (int32_t)segs.size();
            for (const Seg &s : b.segs) {
                segs.push_back(s);
                flops += 2.0 * b.M * s.K;
            }
            int32_t se = (int32_t)segs.size();
            int64_t kp = 0;
            for (const Seg &sg : b.segs) kp += sg.Kpad;
            placed.push_back({kind, b.node, b.out_buf, b.M, sb, se, b.out_row, kp});
            for (int32_t m0 = 0; m0 < std::max(b.M, 1); m0 += ph.bm) {
                Task t{};
                t.out_row = b.out_row + m0;
                t.out_buf = b.out_buf;
                t.M = std::min(ph.bm, b.M - m0);
                t.m0 = m0;
                t.seg_begin = sb;
                t.seg_end = se;
                tasks.push_back(t);
            }
        }
        ph.task_count = (int32_t)tasks.size() - ph.task_begin;
        ph.seg_count = 0;
        ph.flops_per_col = flops;
        phases.push_back(ph);
    }
};

struct DevicePtrs {
    void *p[8] = {nullptr};
    int n = 0;
    void add(void *q) { p[n++] = q; }
    ~DevicePtrs() {
        for (int i = 0; i < n; i++)
            if (p[i]) (void)hipFree(p[i]);
    }
};

#define HM_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? HM_ERR_NOMEM : HM_ERR_DEVICE,     \
                        std::string(#call ": ") + hipGetErrorString(e_));            \
    } while (0)

// Stage one source array through device memory in chunks and repack its jobs.
hm_status repack_source(const double *host, std::vector<RepackJob> &jobs, double *store,
                        double *stage, int64_t stage_elems, RepackJob *d_jobs, int64_t max_jobs,
                        hipStream_t s) {
    std::sort(jobs.begin(), jobs.end(),
              [](const RepackJob &a, const RepackJob &b) { return a.src_off < b.src_off; });
    size_t i = 0;
    while (i < jobs.size()) {
        const int64_t c0 = jobs[i].src_off;
        int64_t c1 = c0;
        size_t j = i;
        while (j < jobs.size() && (int64_t)(j - i) < max_jobs) {
            int64_t end = jobs[j].src_off + (int64_t)jobs[j].rows * jobs[j].cols;
            if (end - c0 > stage_elems) break;
            c1 = std::max(c1, end);
            j++;
        }
        if (j == i) return fail(HM_ERR_INTERNAL, "repack: block larger than the staging buffer");
        std::vector<RepackJob> chunk(jobs.begin() + i, jobs.begin() + j);
        for (RepackJob &r : chunk) r.src_off -= c0;
        HM_HIP(hipMemcpyAsync(stage, host + c0, sizeof(double) * (size_t)(c1 - c0),
                              hipMemcpyHostToDevice, s));
        HM_HIP(hipMemcpyAsync(d_jobs, chunk.data(), sizeof(RepackJob) * chunk.size(),
                              hipMemcpyHostToDevice, s));
        HM_HIP(launch_repack(stage, d_jobs, (int)chunk.size(), store, s));
        HM_HIP(hipStreamSynchronize(s));
        i = j;
    }
    return HM_OK;
}

}  // namespace

hm_status build_matrix(const HostRepr &r, int device, unsigned prec_mask, hm_matrix *out,
                       const BlockSource *gen) {
    const int32_t n = r.n_nodes;
    const bool no_near = (prec_mask & HM_LOAD_NO_NEAR_BLOCKS) != 0;
    const bool no_far = (prec_mask & HM_LOAD_NO_FAR_BLOCKS) != 0;
    if (no_far && r.skel_ptr.empty())
        return fail(HM_ERR_INVALID, "HM_LOAD_NO_FAR_BLOCKS needs the skeletons in the representation");
    auto leaf = [&](int a) { return r.left[a] < 0; };
    std::vector<int64_t> wrow((size_t)n + 1, 0);
    for (int a = 0; a < n; a++) wrow[a + 1] = wrow[a] + r.rank[a];
    // padded row starts in the split-BF16 workspaces: leaves' point rows (W)
    // and nodes' skeleton rows (Ŵ, Ŷ), each node starting at a multiple of 32
    std::vector<int64_t> w16row((size_t)n, 0), h16row((size_t)n + 1, 0);
    std::vector<int32_t> leaves;
    for (int a = 0; a < n; a++)
        if (leaf(a)) leaves.push_back(a);
    std::sort(leaves.begin(), leaves.end(), [&](int x, int y) { return r.start[x] < r.start[y]; });
    int64_t rows16_w = 0;
    for (int a : leaves) {
        w16row[a] = rows16_w;
        rows16_w += round_up(r.size[a], Split16::kRows);
    }
    for (int a = 0; a < n; a++) h16row[a + 1] = h16row[a] + round_up(r.rank[a], Split16::kRows);

    if (gen && (r.skel_ptr.size() != (size_t)n + 1))
        return fail(HM_ERR_INVALID, "generated blocks need the skeletons in the representation");
    const bool sym = (prec_mask & HM_LOAD_SYMMETRIC) != 0;
    if (sym && !gen) {
        hm_status st = check_symmetric(r, !no_near, !no_far);
        if (st != HM_OK) return st;
    }
    // symmetric store: the block of an unordered pair {a, b} is stored once,
    // for the row node a <= b (visited first); the other job reads it as a
    // mirror (Seg::trans), its rows tstride apart
    std::map<std::pair<int, int>, std::pair<int64_t, int32_t>> stored;  // pair -> (offset, lda)
    int32_t max_tstride = 0;
    Planner P;
    std::vector<GenJob> gjobs;  // far and near blocks generated from the points (gen)
    std::vector<std::vector<int>> by_level((size_t)r.depth + 1);
    for (int a = 0; a < n; a++) by_level[(size_t)r.level[a]].push_back(a);

    int64_t E_V = 0, E_T = 0;
    // up pass
    for (int lvl = r.depth; lvl >= 1; lvl--) {
        std::vector<Block> blocks;
        for (int a : by_level[(size_t)lvl]) {
            const int32_t k = r.rank[a];
            if (k == 0) continue;
            const int32_t kp = (int32_t)round_up(k, 16);
            Block b{BUF_WHAT, wrow[a], k, {}, a};
            if (leaf(a)) {
                const int32_t m = (int32_t)r.size[a];
                int64_t off = P.alloc(m, kp);
                P.jobs[0].push_back({r.basis_off[a], off, k, m, 0, 0, m, kp});
                b.segs.push_back(seg(off, r.start[a], kp, m, BUF_WT, w16row[a]));
                E_V += (int64_t)k * m;
            } else {
                // T_a's column halves (left / right child skeletons) are stored
                // as two blocks so that each is zero-padded on its own
                const int32_t kl = r.rank[r.left[a]], kr = r.rank[r.right[a]];
                if (kl > 0) {
                    int64_t off = P.alloc(kl, kp);
                    P.jobs[0].push_back({r.basis_off[a], off, k, kl + kr, 0, 0, kl, kp});
                    b.segs.push_back(seg(off, wrow[r.left[a]], kp, kl, BUF_WHAT, h16row[r.left[a]]));
                }
                if (kr > 0) {
                    int64_t off = P.alloc(kr, kp);
                    P.jobs[0].push_back({r.basis_off[a], off, k, kl + kr, 0, kl, kr, kp});
                    b.segs.push_back(seg(off, wrow[r.right[a]], kp, kr, BUF_WHAT, h16row[r.right[a]]));
                }
                E_T += (int64_t)k * (kl + kr);
            }
            blocks.push_back(std::move(b));
        }
        P.add_phase(1, lvl, blocks);
    }
    // down pass (far reduction fused with the top-down transfers)
    int64_t E_B = 0;
    for (int lvl = 1; lvl <= r.depth; lvl++) {
        std::vector<Block> blocks;
        for (int a : by_level[(size_t)lvl]) {
            const int32_t ka = r.rank[a];
            if (ka == 0) continue;
            const int32_t kap = (int32_t)round_up(ka, 16);
            Block b{BUF_YHAT, wrow[a], ka, {}, a};
            for (int64_t e = r.far_ptr[a]; e < r.far_ptr[a + 1]; e++) {
                const int32_t bn = r.far_col[e], kb = r.rank[bn];
                if (kb == 0) continue;
                // left out of the store as the near blocks are (below)
                int64_t off = 0;
                int32_t tstride = 0;
                if (!no_far && sym && bn < a) {
                    auto it = stored.find({bn, a});
                    if (it == stored.end()) return fail(HM_ERR_INTERNAL, "symmetric store: far block not placed");
                    off = it->second.first;
                    tstride = it->second.second;
                    max_tstride = std::max(max_tstride, tstride);
                } else if (!no_far) {
                    off = P.alloc(kb, kap);
                    P.jobs[1].push_back({r.far_off[e], off, ka, kb, 0, 0, kb, kap});
                    if (gen)  // rows: a's skeleton, columns: bn's skeleton
                        gjobs.push_back({off, r.N + r.skel_ptr[a], r.N + r.skel_ptr[bn], ka, kb, kap, 0});
                    if (sym) stored[{a, bn}] = {off, kap};
                }
                b.segs.push_back(seg(off, wrow[bn], kap, kb, BUF_WHAT, h16row[bn]));
                b.segs.back().from_pts = 2;
                b.segs.back().trans = tstride > 0;
                b.segs.back().tstride = tstride;
                E_B += (int64_t)ka * kb;
            }
            const int32_t p = r.parent[a];
            if (p >= 0 && r.level[p] >= 1 && r.rank[p] > 0) {
                const int32_t kpar = r.rank[p], kl = r.rank[r.left[p]], kr = r.rank[r.right[p]];
                const int32_t c0 = (a == r.left[p]) ? 0 : kl;
                int64_t off = P.alloc(kpar, kap);
                P.jobs[0].push_back({r.basis_off[p], off, kpar, kl + kr, 1, c0, ka, kap});
                b.segs.push_back(seg(off, wrow[p], kap, kpar, BUF_YHAT, h16row[p]));
            }
            blocks.push_back(std::move(b));
        }
        P.add_phase(2, lvl, blocks);
    }
    // leaf pass (near reduction + leaf far part + final sum)
    int64_t E_D = 0;
    {
        std::vector<Block> blocks;
        for (int a = 0; a < n; a++) {
            if (!leaf(a)) continue;
            const int32_t ma = (int32_t)r.size[a], map = (int32_t)round_up(ma, 16);
            Block b{BUF_YT, r.start[a], ma, {}, a};
            for (int64_t e = r.near_ptr[a]; e < r.near_ptr[a + 1]; e++) {
                const int32_t bn = r.near_col[e];
                const int32_t mb = (int32_t)r.size[bn];
                // left out of the store: the segment's A offset is never read
                // (its evaluations compute the block from the points)
                int64_t off = 0;
                int32_t tstride = 0;
                if (!no_near && sym && bn < a) {
                    auto it = stored.find({bn, a});
                    if (it == stored.end()) return fail(HM_ERR_INTERNAL, "symmetric store: near block not placed");
                    off = it->second.first;
                    tstride = it->second.second;
                    max_tstride = std::max(max_tstride, tstride);
                } else if (!no_near) {
                    off = P.alloc(mb, map);
                    P.jobs[2].push_back({r.near_off[e], off, ma, mb, 0, 0, mb, map});
                    if (gen)  // rows: a's points, columns: bn's points (tree order)
                        gjobs.push_back({off, r.start[a], r.start[bn], ma, mb, map, 0});
                    if (sym) stored[{a, bn}] = {off, map};
                }
                b.segs.push_back(seg(off, r.start[bn], map, mb, BUF_WT, w16row[bn]));
                b.segs.back().from_pts = 1;
                b.segs.back().trans = tstride > 0;
                b.segs.back().tstride = tstride;
                E_D += (int64_t)ma * mb;
            }
            const int32_t k = r.rank[a];
            if (k > 0 && r.level[a] >= 1) {
                int64_t off = P.alloc(k, map);
                P.jobs[0].push_back({r.basis_off[a], off, k, ma, 1, 0, ma, map});
                b.segs.push_back(seg(off, wrow[a], map, k, BUF_YHAT, h16row[a]));
            }
            blocks.push_back(std::move(b));
        }
        P.add_phase(3, r.depth, blocks);
    }

    // ---- dependency graph for the persistent launch
    // A down job whose far blocks outweigh the transfer from its parent (at
    // least 4x the contraction rows) is cut in two: its far blocks (which
    // wait only for the partners' up jobs) and then the transfer, added to
    // them, which waits for the parent's Ŷ.  The chain down the tree then
    // holds the short transfers only, not every node's far field.  The cut
    // costs one more read and write of the output tile; it pays where one
    // matrix's graph has the launch to itself.  A launch of many graphs (a
    // batch, concurrent served sweeps) is not bound by any one chain and
    // takes the whole down jobs (the second native graph).
    auto split_down = [&](int64_t k_far, int64_t k_td, int64_t ratio) {
        return k_far > 0 && k_td > 0 && k_far >= ratio * k_td;
    };
    // The thresholds, in contraction rows: 4x for the native graph, 2x for the
    // mixed one, whose far blocks run in split BF16 and so cost less against
    // the FP64 transfer than their length says (measured on the two-means
    // budget structure: native 4x over 1x, 2x and 8x; mixed 2x over 4x and
    // 8x, with 1x cutting the HSS down jobs, far block and transfer of equal
    // length, to a loss).
    constexpr int64_t kCutRatio = 4, kCutRatioMixed = 2;
    auto native_graph = [&](bool cut, std::vector<GJob> &jobs) -> hm_status {
        std::vector<int32_t> up_job(n, -1), down_job(n, -1), near_job(n, -1);
        for (const Planner::Placed &pl : P.placed) {
            GJob j{};
            j.kind = pl.kind;
            j.node = pl.node;
            j.out_buf = pl.out_buf;
            j.out_row = pl.out_row;
            j.M = pl.M;
            j.seg_begin = pl.seg_begin;
            j.seg_end = pl.seg_end;
            j.accumulate = 0;
            j.kpad = pl.kpad;
            const int a = pl.node;
            if (pl.kind == 1) {
                if (!leaf(a)) {
                    if (r.rank[r.left[a]] > 0) j.preds.push_back(up_job[r.left[a]]);
                    if (r.rank[r.right[a]] > 0) j.preds.push_back(up_job[r.right[a]]);
                }
                up_job[a] = (int32_t)jobs.size();
                jobs.push_back(j);
            } else if (pl.kind == 2) {
                for (int64_t e = r.far_ptr[a]; e < r.far_ptr[a + 1]; e++)
                    if (r.rank[r.far_col[e]] > 0) j.preds.push_back(up_job[r.far_col[e]]);
                const int32_t p = r.parent[a];
                const bool has_td = p >= 0 && r.level[p] >= 1 && r.rank[p] > 0;
                // segments: the far blocks, then (with has_td) the transfer from the parent
                const int64_t k_td = has_td ? P.segs[pl.seg_end - 1].Kpad : 0;
                if (cut && has_td && split_down(pl.kpad - k_td, k_td, kCutRatio)) {
                    GJob fj = j;  // far blocks
                    fj.seg_end = pl.seg_end - 1;
                    fj.kpad = pl.kpad - k_td;
                    const int32_t far_job = (int32_t)jobs.size();
                    jobs.push_back(fj);
                    GJob tj = j;  // transfer from the parent, added
                    tj.seg_begin = pl.seg_end - 1;
                    tj.kpad = k_td;
                    tj.accumulate = 1;
                    tj.preds = {far_job, down_job[p]};
                    down_job[a] = (int32_t)jobs.size();
                    jobs.push_back(tj);
                } else {
                    if (has_td) j.preds.push_back(down_job[p]);
                    down_job[a] = (int32_t)jobs.size();
                    jobs.push_back(j);
                }
            } else {
                // the leaf block's segments are its near blocks followed by
                // the leaf far part (present when the leaf has a basis)
                const bool far_part = r.rank[a] > 0 && r.level[a] >= 1;
                GJob nj = j;
                nj.kind = 3;
                nj.seg_end = far_part ? pl.seg_end - 1 : pl.seg_end;
                nj.kpad = 0;
                for (int32_t q = nj.seg_begin; q < nj.seg_end; q++) nj.kpad += P.segs[q].Kpad;
                near_job[a] = (int32_t)jobs.size();
                jobs.push_back(nj);
                if (far_part) {
                    GJob fj = j;
                    fj.kind = 4;
                    fj.seg_begin = pl.seg_end - 1;
                    fj.accumulate = 1;
                    fj.kpad = P.segs[fj.seg_begin].Kpad;
                    fj.preds = {near_job[a], down_job[a]};
                    jobs.push_back(fj);
                }
            }
        }
        for (const GJob &j : jobs)
            for (int32_t q : j.preds)
                if (q < 0) return fail(HM_ERR_INTERNAL, "dependency graph: missing predecessor job");
        return HM_OK;
    };
    std::vector<GJob> jobs, jobs_whole;
    {
        hm_status gst = native_graph(true, jobs);
        if (gst == HM_OK) gst = native_graph(false, jobs_whole);
        if (gst != HM_OK) return gst;
    }
    // Mixed precision: the same jobs with the products of the leaf bases, far
    // blocks and near blocks in split BF16 and the transfers in FP64; a down
    // job runs its far blocks in split BF16 and continues in FP64 with the
    // transfer from its parent (mode 2).
    std::vector<GJob> mjobs;
    {
        std::vector<int32_t> up_job(n, -1), down_job(n, -1), near_job(n, -1);
        for (const Planner::Placed &pl : P.placed) {
            GJob j{};
            j.node = pl.node;
            j.out_buf = pl.out_buf;
            j.out_row = pl.out_row;
            j.M = pl.M;
            const int a = pl.node;
            auto kpad_of = [&](int32_t b, int32_t e) {
                int64_t k = 0;
                for (int32_t q = b; q < e; q++) k += P.segs[q].Kpad;
                return k;
            };
            if (pl.kind == 1) {
                j.kind = 1;
                j.seg_begin = pl.seg_begin;
                j.seg_end = pl.seg_end;
                j.mode = leaf(a) ? 1 : 0;
                j.kpad = pl.kpad;
                j.kpad_split = leaf(a) ? pl.kpad : 0;
                j.out16 = h16row[a];  // Ŵ: FP64 (parent's transfer) and split (far blocks)
                j.out_split = 1;
                if (!leaf(a)) {
                    if (r.rank[r.left[a]] > 0) j.preds.push_back(up_job[r.left[a]]);
                    if (r.rank[r.right[a]] > 0) j.preds.push_back(up_job[r.right[a]]);
                }
                up_job[a] = (int32_t)mjobs.size();
                mjobs.push_back(j);
            } else if (pl.kind == 2) {
                // segments: the far blocks, then (if the parent has a
                // basis) the transfer from the parent
                const int32_t p = r.parent[a];
                const bool has_td = p >= 0 && r.level[p] >= 1 && r.rank[p] > 0;
                const int32_t far_end = has_td ? pl.seg_end - 1 : pl.seg_end;
                GJob dj = j;
                dj.kind = 2;
                dj.seg_begin = pl.seg_begin;
                dj.seg_end = pl.seg_end;
                dj.kpad = kpad_of(pl.seg_begin, pl.seg_end);
                dj.kpad_split = kpad_of(pl.seg_begin, far_end);
                dj.mode = !has_td ? 1 : far_end > pl.seg_begin ? 2 : 0;
                if (dj.mode == 0) dj.kpad_split = 0;
                if (leaf(a)) {  // a leaf's Ŷ feeds only its leaf far part (split BF16)
                    dj.out16 = h16row[a];
                    dj.out_split = 2;
                }
                for (int64_t e = r.far_ptr[a]; e < r.far_ptr[a + 1]; e++)
                    if (r.rank[r.far_col[e]] > 0) dj.preds.push_back(up_job[r.far_col[e]]);
                const int64_t k_td = has_td ? P.segs[pl.seg_end - 1].Kpad : 0;
                if (dj.mode == 2 && split_down(dj.kpad_split, k_td, kCutRatioMixed)) {
                    // cut as in the native graph: the far blocks in split
                    // BF16 written as FP64, then the FP64 transfer added to
                    // them (a leaf's transfer job writes the split copy of the
                    // sum, the only form its leaf far part reads)
                    GJob fj = dj;
                    fj.mode = 1;
                    fj.seg_end = far_end;
                    fj.kpad = dj.kpad_split;
                    fj.out16 = -1;
                    fj.out_split = 0;
                    const int32_t far_job = (int32_t)mjobs.size();
                    mjobs.push_back(fj);
                    GJob tj = dj;
                    tj.mode = 0;
                    tj.seg_begin = far_end;
                    tj.kpad = k_td;
                    tj.kpad_split = 0;
                    tj.accumulate = 1;
                    tj.preds = {far_job, down_job[p]};
                    down_job[a] = (int32_t)mjobs.size();
                    mjobs.push_back(tj);
                } else {
                    if (has_td) dj.preds.push_back(down_job[p]);
                    down_job[a] = (int32_t)mjobs.size();
                    mjobs.push_back(dj);
                }
            } else {
                const bool far_part = r.rank[a] > 0 && r.level[a] >= 1;
                GJob nj = j;
                nj.kind = 3;
                nj.mode = 1;
                nj.seg_begin = pl.seg_begin;
                nj.seg_end = far_part ? pl.seg_end - 1 : pl.seg_end;
                nj.kpad = kpad_of(nj.seg_begin, nj.seg_end);
                nj.kpad_split = nj.kpad;
                near_job[a] = (int32_t)mjobs.size();
                mjobs.push_back(nj);
                if (far_part) {
                    GJob fj = j;
                    fj.kind = 4;
                    fj.mode = 1;
                    fj.accumulate = 1;
                    fj.seg_begin = pl.seg_end - 1;
                    fj.seg_end = pl.seg_end;
                    fj.kpad = kpad_of(fj.seg_begin, fj.seg_end);
                    fj.kpad_split = fj.kpad;
                    fj.preds = {near_job[a], down_job[a]};
                    mjobs.push_back(fj);
                }
            }
        }
        for (const GJob &j : mjobs)
            for (int32_t q : j.preds)
                if (q < 0) return fail(HM_ERR_INTERNAL, "mixed dependency graph: missing predecessor job");
    }
    // offsets of every block in the split-BF16 store (32-wide contraction
    // chunks, hi then lo part of lda x 32 values each)
    int64_t store16_elems = 0;
    for (Seg &sg : P.segs) {
        sg.a_off16 = store16_elems;
        store16_elems += (int64_t)((sg.K + 31) / 32) * 2 * sg.lda * 32;
    }
    store16_elems += 8192;  // slack for tiles taller than their block

    // ---- device side
    int prev = 0;
    HM_HIP(hipGetDevice(&prev));
    HM_HIP(hipSetDevice(device));
    struct Restore {
        int d;
        ~Restore() { (void)hipSetDevice(d); }
    } restore{prev};

    hm_matrix h = new (std::nothrow) hm_matrix_s();
    if (!h) return fail(HM_ERR_NOMEM, "hm_load: host allocation failed");
    struct Guard {
        hm_matrix h;
        bool keep = false;
        ~Guard() {
            if (!keep) hm_free(h);
        }
    } guard{h};
    h->device = device;
    h->symmetric = sym;
    h->near_stored = !no_near;
    h->far_stored = !no_far;
    if (!r.skel_ptr.empty()) {  // original point of each Ŵ row (node a's rows follow its skeleton)
        h->skel_row_pt.assign((size_t)wrow[n], 0);
        for (int a = 0; a < n; a++)
            for (int32_t i = 0; i < r.rank[a]; i++)
                h->skel_row_pt[(size_t)(wrow[a] + i)] = r.skel[(size_t)(r.skel_ptr[a] + i)];
    }
    h->N = r.N;
    h->repr_d = r.d;
    h->repr_kernel = r.kernel;
    h->repr_h = r.h;
    h->n_nodes = n;
    h->depth = r.depth;
    for (int a = 0; a < n; a++) h->max_rank = std::max(h->max_rank, r.rank[a]);
    h->n_far = (int64_t)r.far_col.size();
    h->n_near = (int64_t)r.near_col.size();
    h->E_V = E_V;
    h->E_T = E_T;
    h->E_B = E_B;
    h->E_D = E_D;
    h->skel_rows = wrow[n];
    // slack after the last block: a tile taller than its block reads past it
    // (a mirror block's rows are tstride apart: up to 128 rows of them)
    h->store_elems = P.store_off + 512 + (int64_t)128 * max_tstride;
    h->phases = P.phases;
    h->task_k = job_task_k(jobs);
    h->gjobs = std::move(jobs);
    h->gjobs_whole = std::move(jobs_whole);
    h->gjobs_mixed = std::move(mjobs);

    hipStream_t s = nullptr;
    HM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } sg{s};

    double *store64 = nullptr;
    HM_HIP(hipMalloc(&store64, sizeof(double) * (size_t)h->store_elems));
    h->prec[HM_PREC_FP64].blocks = store64;
    h->prec[HM_PREC_FP64].bytes = sizeof(double) * (size_t)h->store_elems;
    HM_HIP(hipMemsetAsync(store64, 0, sizeof(double) * (size_t)h->store_elems, s));
    {
        const int64_t max_src = gen ? std::max(r.basis_len, (int64_t)1)
                                    : std::max({r.basis_len, r.B_len, r.D_len, (int64_t)1});
        const int64_t stage_elems = std::min<int64_t>(max_src, (int64_t)64 << 20);  // <= 512 MiB
        const int64_t max_jobs = 1 << 16;
        DevicePtrs tmp;
        double *stage = nullptr;
        RepackJob *d_jobs = nullptr;
        HM_HIP(hipMalloc(&stage, sizeof(double) * (size_t)stage_elems));
        tmp.add(stage);
        HM_HIP(hipMalloc(&d_jobs, sizeof(RepackJob) * (size_t)max_jobs));
        tmp.add(d_jobs);
        const double *src[3] = {r.basis_ptr(), r.B_ptr(), r.D_ptr()};
        for (int k = 0; k < (gen ? 1 : 3); k++) {
            hm_status st = repack_source(src[k], P.jobs[k], store64, stage, stage_elems, d_jobs,
                                         max_jobs, s);
            if (st != HM_OK) return st;
        }
        if (gen) {
            const int64_t per = max_jobs * (int64_t)sizeof(RepackJob) / (int64_t)sizeof(GenJob);
            for (size_t i = 0; i < gjobs.size(); i += (size_t)per) {
                const int cnt = (int)std::min<size_t>((size_t)per, gjobs.size() - i);
                HM_HIP(hipMemcpyAsync(d_jobs, gjobs.data() + i, sizeof(GenJob) * (size_t)cnt,
                                      hipMemcpyHostToDevice, s));
                HM_HIP(launch_gen_store((const GenJob *)d_jobs, cnt, *gen, store64, s));
                HM_HIP(hipStreamSynchronize(s));
            }
        }
    }
    if (prec_mask & HM_PRECBIT(HM_PREC_BF16X3)) {
        HM_HIP(hipMalloc(&h->store16, 2 * (size_t)store16_elems));
        h->store16_bytes = 2 * (size_t)store16_elems;
        HM_HIP(hipMemsetAsync(h->store16, 0, h->store16_bytes, s));
    }
    if (prec_mask & HM_PRECBIT(HM_PREC_FP32)) {
        float *store32 = nullptr;
        HM_HIP(hipMalloc(&store32, sizeof(float) * (size_t)h->store_elems));
        h->prec[HM_PREC_FP32].blocks = store32;
        h->prec[HM_PREC_FP32].bytes = sizeof(float) * (size_t)h->store_elems;
        HM_HIP(launch_convert_f64_to_f32(store64, store32, h->store_elems, s));
    }
    HM_HIP(hipMalloc(&h->d_perm, sizeof(int64_t) * (size_t)r.N));
    HM_HIP(hipMemcpyAsync(h->d_perm, r.perm.data(), sizeof(int64_t) * (size_t)r.N,
                          hipMemcpyHostToDevice, s));
    HM_HIP(hipMalloc(&h->d_tasks, sizeof(Task) * std::max<size_t>(P.tasks.size(), 1)));
    HM_HIP(hipMalloc(&h->d_segs, sizeof(Seg) * std::max<size_t>(P.segs.size(), 1)));
    if (!P.tasks.empty())
        HM_HIP(hipMemcpyAsync(h->d_tasks, P.tasks.data(), sizeof(Task) * P.tasks.size(),
                              hipMemcpyHostToDevice, s));
    if (!P.segs.empty())
        HM_HIP(hipMemcpyAsync(h->d_segs, P.segs.data(), sizeof(Seg) * P.segs.size(),
                              hipMemcpyHostToDevice, s));
    h->rows16_w = rows16_w;
    h->rows16_h = h16row[n];
    if (prec_mask & HM_PRECBIT(HM_PREC_BF16X3)) {
        // W's 32-row chunks for the split permute-in
        std::vector<int64_t> ch;
        for (int a : leaves)
            for (int64_t c = 0; c < r.size[a]; c += Split16::kRows) {
                ch.push_back(r.start[a] + c);
                ch.push_back(std::min<int64_t>(Split16::kRows, r.size[a] - c));
                ch.push_back(w16row[a] + c);
            }
        h->n_wchunks = (int64_t)ch.size() / 3;
        HM_HIP(hipMalloc(&h->d_wchunks, sizeof(int64_t) * std::max<size_t>(ch.size(), 3)));
        if (!ch.empty()) HM_HIP(hipMemcpy(h->d_wchunks, ch.data(), sizeof(int64_t) * ch.size(), hipMemcpyHostToDevice));
    }
    HM_HIP(hipMalloc(&h->d_mat, sizeof(MatDesc)));
    HM_HIP(hipMalloc(&h->d_head, 2 * sizeof(int32_t)));
    HM_HIP(hipMemsetAsync(h->d_head, 0, 2 * sizeof(int32_t), s));
    {
        hipDeviceProp_t prop;
        HM_HIP(hipGetDeviceProperties(&prop, device));
        h->n_cu = prop.multiProcessorCount;
    }
    if (h->store16)
        HM_HIP(launch_make_bf16x3(store64, h->d_segs, (int)P.segs.size(), h->store16, s));
    HM_HIP(hipStreamSynchronize(s));
    if (!(prec_mask & (HM_PRECBIT(HM_PREC_FP64) | HM_PRECBIT(HM_PREC_BF16X3)))) {
        HM_HIP(hipFree(store64));
        h->prec[HM_PREC_FP64].blocks = nullptr;
        h->prec[HM_PREC_FP64].bytes = 0;
    }
    guard.keep = true;
    *out = h;
    return HM_OK;
}

}  // namespace hm
