// hm_sched.hip -- the persistent launch's queue: expand the evaluation's job
// graph into entries (one per row tile and column tile), give each entry a
// priority equal to its critical-path length to the end of the graph, and
// order the queue by a list-scheduling simulation of the workgroups.
//
// This takes the place of the paper's coarsening and blocking schedules
// (Algorithms 1 and 2, Section 3.2), which balance a multicore CPU by bin
// packing subtrees of a coarsened level: on the GPU the dependencies are
// tracked per entry on the device, so an entry may start as soon as its
// inputs exist, and near-field work (which depends on nothing) fills the
// machine while the tree passes run.
#include <algorithm>
#include <queue>

#include "hm_internal.h"

namespace hm {

double job_task_k(const std::vector<GJob> &jobs) {
    double num = 0, den = 0;
    for (const GJob &j : jobs) {
        num += (double)j.M * (double)j.kpad * (double)j.kpad;
        den += (double)j.M * (double)j.kpad;
    }
    return den > 0 ? num / den : 0.0;
}

void free_plan(GraphPlan &p) {
    if (p.d_tasks) (void)hipFree(p.d_tasks);
    if (p.d_succ) (void)hipFree(p.d_succ);
    if (p.d_counters) (void)hipFree(p.d_counters);
    p = GraphPlan{};
}

hm_status build_plan(const std::vector<PlanPart> &parts, int bn, int elem_bytes, int workers, GraphPlan &plan) {
    // per part: row tiles per job, entry offsets
    struct P {
        const std::vector<GJob> *jobs;
        int mat, nq, per_q;
        std::vector<std::pair<int32_t, int32_t>> cols;  // column tiles: (first column, width)
        int64_t base;
        std::vector<int32_t> rows, bm, first;  // bm: height of a job's row tiles (its last one: last_bm)
        std::vector<int32_t> last_bm;
        std::vector<std::vector<int32_t>> succ_jobs;
        std::vector<double> cost, blevel;  // per local entry (one column tile)
    };
    std::vector<P> ps(parts.size());
    int64_t total64 = 0;
    const double overhead = 2.0 * 128 * 64 * 256;  // fixed per-entry cost, in flops
    for (size_t i = 0; i < parts.size(); i++) {
        P &p = ps[i];
        p.jobs = parts[i].mode == 1 ? &parts[i].h->gjobs_mixed
                 : parts[i].cut_down ? &parts[i].h->gjobs
                                     : &parts[i].h->gjobs_whole;
        p.mat = parts[i].mat;
        for (int64_t n0 = 0; n0 < parts[i].Qp; n0 += bn) {
            const int64_t w = std::min<int64_t>(bn, parts[i].Qp - n0);
            if (w < 16 || (w & (w - 1)) != 0 || (w < bn && n0 + w != parts[i].Qp))
                return fail(HM_ERR_INTERNAL, "task graph: padded columns are not whole tiles");
            p.cols.push_back({(int32_t)n0, (int32_t)w});
        }
        p.nq = (int)p.cols.size();
        if (p.nq == 0) return fail(HM_ERR_INTERNAL, "task graph: no columns");
        const std::vector<GJob> &jobs = *p.jobs;
        const int nj = (int)jobs.size();
        p.rows.resize(nj);
        p.bm.resize(nj);
        p.last_bm.resize(nj);
        p.first.assign(nj + 1, 0);
        for (int j = 0; j < nj; j++) {
            // row tiles of 128 rows; a job's last (or only) tile takes the
            // smallest height that holds its remaining rows: a multiple of
            // 16 from 32 where the launch has those tiles (fine16_tiles), 32,
            // 64, 96 or 128 where it has the fine tiles (fine_tiles), else 64
            // or 128
            const int M = std::max(1, jobs[j].M);
            p.bm[j] = 128;
            p.rows[j] = (M + 127) / 128;
            const int rem = M - (p.rows[j] - 1) * 128;
            const bool split = parts[i].mode == 1;
            p.last_bm[j] = fine16_tiles(elem_bytes, bn, split) ? std::max(32, (rem + 15) / 16 * 16)
                           : !fine_tiles(elem_bytes, bn, split)
                               ? (rem <= 64 ? 64 : 128)
                               : rem <= 32 ? 32 : rem <= 64 ? 64 : rem <= 96 ? 96 : 128;
            p.first[j + 1] = p.first[j] + p.rows[j];
        }
        p.per_q = p.first[nj];
        p.base = total64;
        total64 += (int64_t)p.per_q * p.nq;
        p.succ_jobs.assign(nj, {});
        for (int j = 0; j < nj; j++)
            for (int32_t q : jobs[j].preds) p.succ_jobs[q].push_back(j);
        p.cost.resize(p.per_q);
        p.blevel.resize(p.per_q);
        // a split-BF16 contraction row is priced at a fifth of an FP64 one
        // (measured: 0.35 and 0.5 order the mixed launches worse)
        for (int j = 0; j < nj; j++)
            for (int r = 0; r < p.rows[j]; r++)
                p.cost[p.first[j] + r] = 2.0 * (r + 1 < p.rows[j] ? p.bm[j] : p.last_bm[j]) * bn *
                                             (jobs[j].kpad - 0.80 * jobs[j].kpad_split) + overhead;
        // critical path to the end of the graph (jobs are topologically ordered)
        std::vector<double> jbl(nj, 0.0);
        for (int j = nj - 1; j >= 0; j--) {
            double m = 0.0;
            for (int32_t s2 : p.succ_jobs[j]) m = std::max(m, jbl[s2]);
            jbl[j] = p.cost[p.first[j]] + m;
            for (int r = 0; r < p.rows[j]; r++) p.blevel[p.first[j] + r] = jbl[j];
        }
    }
    if (total64 > (int64_t)1 << 30) return fail(HM_ERR_INVALID, "task graph too large");
    const int total = (int)total64;
    // global entry -> (part, column tile, job, row)
    auto locate = [&](int e, int &pi, int &q, int &j, int &r) {
        pi = 0;
        while (pi + 1 < (int)ps.size() && ps[pi + 1].base <= e) pi++;
        const P &p = ps[pi];
        const int loc = (int)(e - p.base);
        q = loc / p.per_q;
        const int l = loc % p.per_q;
        j = (int)(std::upper_bound(p.first.begin(), p.first.end(), l) - p.first.begin()) - 1;
        r = l - p.first[j];
    };
    std::vector<int32_t> remaining(total);
    for (const P &p : ps)
        for (int q = 0; q < p.nq; q++)
            for (size_t j = 0; j < p.jobs->size(); j++) {
                int nd = 0;
                for (int32_t pr : (*p.jobs)[j].preds) nd += p.rows[pr];
                for (int r = 0; r < p.rows[j]; r++)
                    remaining[p.base + (int64_t)q * p.per_q + p.first[j] + r] = nd;
            }
    const std::vector<int32_t> ndeps = remaining;

    // tie-break key among entries of equal priority: the row and column
    // tiles of one job come one after another, so that they run at the same
    // time and share their operands in the caches
    std::vector<int64_t> ekey(total);
    {
        int64_t job_base = 0, max_nq = 1, max_rows = 1;
        for (const P &p : ps) {
            max_nq = std::max<int64_t>(max_nq, p.nq);
            for (int32_t rr : p.rows) max_rows = std::max<int64_t>(max_rows, rr);
        }
        for (const P &p : ps) {
            const std::vector<GJob> &jobs = *p.jobs;
            for (int q = 0; q < p.nq; q++)
                for (size_t j = 0; j < jobs.size(); j++)
                    for (int r = 0; r < p.rows[j]; r++)
                        ekey[p.base + (int64_t)q * p.per_q + p.first[j] + r] =
                            ((job_base + (int64_t)j) * max_nq + q) * max_rows + r;
            job_base += (int64_t)jobs.size();
        }
    }

    // list scheduling: the earliest-free simulated workgroup takes the
    // released entry with the longest critical path
    struct Avail {
        double bl;
        int64_t key;
        int e;
        bool operator<(const Avail &o) const { return bl < o.bl || (bl == o.bl && key > o.key); }
    };
    std::priority_queue<Avail> avail;
    typedef std::pair<double, int> Ev;  // (finish time, entry)
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> finishes;
    std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
    for (int w = 0; w < std::max(workers, 1); w++) free_at.push(0.0);
    auto blevel_of = [&](int e) {
        int pi, q, j, r;
        locate(e, pi, q, j, r);
        return ps[pi].blevel[ps[pi].first[j] + r];
    };
    auto cost_of = [&](int e) {  // the per-column part scales with the tile's width
        int pi, q, j, r;
        locate(e, pi, q, j, r);
        return (ps[pi].cost[ps[pi].first[j] + r] - overhead) * ps[pi].cols[q].second / bn + overhead;
    };
    for (int e = 0; e < total; e++)
        if (remaining[e] == 0) avail.push({blevel_of(e), ekey[e], e});
    auto release = [&](int e) {
        int pi, q, j, r;
        locate(e, pi, q, j, r);
        const P &p = ps[pi];
        for (int32_t s2 : p.succ_jobs[j])
            for (int rr = 0; rr < p.rows[s2]; rr++) {
                const int f = (int)(p.base + (int64_t)q * p.per_q + p.first[s2] + rr);
                if (--remaining[f] == 0) avail.push({p.blevel[p.first[s2] + rr], ekey[f], f});
            }
    };
    std::vector<int32_t> order;
    order.reserve(total);
    double makespan = 0.0;
    while ((int)order.size() < total) {
        double t = free_at.top();
        while (!finishes.empty() && finishes.top().first <= t) {
            release(finishes.top().second);
            finishes.pop();
        }
        if (avail.empty()) {
            if (finishes.empty()) return fail(HM_ERR_INTERNAL, "task graph has a cycle");
            t = finishes.top().first;
            while (!finishes.empty() && finishes.top().first <= t) {
                release(finishes.top().second);
                finishes.pop();
            }
            free_at.pop();
            free_at.push(t);
            continue;
        }
        const Avail a = avail.top();
        avail.pop();
        free_at.pop();
        const double fin = t + cost_of(a.e);
        free_at.push(fin);
        finishes.push({fin, a.e});
        makespan = std::max(makespan, fin);
        order.push_back(a.e);
    }

    // queue arrays in that order
    std::vector<int32_t> pos(total);
    for (int i = 0; i < total; i++) pos[order[i]] = i;
    std::vector<PTask> tasks(total);
    std::vector<int32_t> succ;
    for (int i = 0; i < total; i++) {
        const int e = order[i];
        int pi, q, j, r;
        locate(e, pi, q, j, r);
        const P &p = ps[pi];
        const GJob &g = (*p.jobs)[j];
        PTask t{};
        const int tile_bm = r + 1 < p.rows[j] ? p.bm[j] : p.last_bm[j];
        t.out_row = g.out_row + (int64_t)r * p.bm[j];
        t.out_buf = g.out_buf;
        t.M = std::min(p.bm[j], g.M - r * p.bm[j]);
        t.m0 = r * p.bm[j];
        t.seg_begin = g.seg_begin;
        t.seg_end = g.seg_end;
        t.bm = tile_bm;
        t.out16 = g.out16 >= 0 ? g.out16 + t.m0 : -1;
        t.out_split = g.out16 >= 0 ? g.out_split : 0;
        t.accumulate = g.accumulate;
        t.n0 = p.cols[q].first;
        t.bn = p.cols[q].second;
        t.mat = p.mat;
        t.mode = g.mode;
        t.ndeps = ndeps[e];
        t.succ_begin = (int32_t)succ.size();
        for (int32_t s2 : p.succ_jobs[j])
            for (int rr = 0; rr < p.rows[s2]; rr++)
                succ.push_back(pos[p.base + (int64_t)q * p.per_q + p.first[s2] + rr]);
        t.succ_end = (int32_t)succ.size();
        tasks[i] = t;
    }

    free_plan(plan);
    hipError_t err = hipMalloc(&plan.d_tasks, sizeof(PTask) * std::max(total, 1));
    if (err == hipSuccess) err = hipMalloc(&plan.d_succ, sizeof(int32_t) * std::max<size_t>(succ.size(), 1));
    if (err == hipSuccess) err = hipMalloc(&plan.d_counters, sizeof(int32_t) * std::max(total, 1));
    if (err == hipSuccess && total)
        err = hipMemcpy(plan.d_tasks, tasks.data(), sizeof(PTask) * total, hipMemcpyHostToDevice);
    if (err == hipSuccess && !succ.empty())
        err = hipMemcpy(plan.d_succ, succ.data(), sizeof(int32_t) * succ.size(), hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        free_plan(plan);
        return fail(err == hipErrorOutOfMemory ? HM_ERR_NOMEM : HM_ERR_DEVICE,
                    std::string("uploading the task graph: ") + hipGetErrorString(err));
    }
    plan.bn = bn;
    plan.narrow = false;
    for (const P &p : ps) plan.narrow = plan.narrow || p.cols.back().second < bn;
    plan.sym = false;
    for (const PlanPart &pp : parts) plan.sym = plan.sym || pp.h->symmetric;
    plan.n_tasks = total;
    plan.est_ms = makespan;
    return HM_OK;
}

int64_t padded_columns(int64_t Q, int bn, bool narrow_tail) {
    const int64_t full = Q / bn * bn, rest = Q - full;
    if (rest == 0) return std::max<int64_t>(full, bn);
    if (!narrow_tail) return full + bn;
    int64_t w = 16;
    while (w < rest) w *= 2;
    return full + std::min<int64_t>(w, bn);
}

hm_status get_plan(hm_matrix h, int slot, int bn, int64_t ldq, int workers, GraphPlan **out,
                   int mode, bool build) {
    for (GraphPlan &p : h->plans[slot])
        if (p.bn == bn && p.Q == ldq && p.mode == mode) {
            *out = &p;
            return HM_OK;
        }
    if (!build)
        return fail(HM_ERR_INVALID, "no task graph for this column-tile count, precision and element type yet: "
                                    "one hm_eval with the same Q class, dtype and precision builds it");
    if (h->plans[slot].size() >= 16) {  // bounded cache: drop the oldest plan
        free_plan(h->plans[slot].front());
        h->plans[slot].erase(h->plans[slot].begin());
    }
    GraphPlan p;
    std::vector<PlanPart> parts{{h, 0, ldq, mode}};
    hm_status st = build_plan(parts, bn, slot == 0 ? 8 : 4, workers, p);
    if (st != HM_OK) return st;
    p.Q = ldq;  // cache key: padded columns
    p.mode = mode;
    h->plans[slot].push_back(p);
    *out = &h->plans[slot].back();
    return HM_OK;
}

}  // namespace hm
