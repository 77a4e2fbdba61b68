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

void free_plan(GraphPlan &p) {
    if (p.d_tasks) (void)hipFree(p.d_tasks);
    if (p.d_succ) (void)hipFree(p.d_succ);
    if (p.d_counters) (void)hipFree(p.d_counters);
    p = GraphPlan{};
}

hm_status make_plan(hm_matrix h, int slot, int bn, int64_t Q, int64_t ldq, int workers) {
    GraphPlan &plan = h->plan[slot];
    const std::vector<GJob> &jobs = h->gjobs;
    const int nj = (int)jobs.size();
    const int nq = (int)(ldq / bn);
    // row tiles per job
    std::vector<int32_t> rows(nj), bm(nj), first(nj + 1, 0);
    for (int j = 0; j < nj; j++) {
        bm[j] = jobs[j].M <= 64 ? 64 : 128;
        rows[j] = std::max(1, (jobs[j].M + bm[j] - 1) / bm[j]);
        first[j + 1] = first[j] + rows[j];
    }
    const int per_q = first[nj];
    const int64_t total64 = (int64_t)per_q * nq;
    if (total64 > (int64_t)1 << 30) return fail(HM_ERR_INVALID, "hm_eval: task graph too large");
    const int total = (int)total64;
    std::vector<std::vector<int32_t>> succ_jobs(nj);
    for (int j = 0; j < nj; j++)
        for (int32_t p : jobs[j].preds) succ_jobs[p].push_back(j);

    // work model: padded flops plus a fixed per-entry overhead (in flops)
    const double overhead = 2.0 * 128 * 64 * 256;
    std::vector<double> cost(per_q), blevel(per_q);
    for (int j = 0; j < nj; j++)
        for (int r = 0; r < rows[j]; r++) cost[first[j] + r] = 2.0 * bm[j] * jobs[j].kpad * bn + overhead;
    // critical path to the end of the graph (jobs are topologically ordered)
    std::vector<double> job_bl(nj, 0.0);
    for (int j = nj - 1; j >= 0; j--) {
        double m = 0.0;
        for (int32_t s : succ_jobs[j]) m = std::max(m, job_bl[s]);
        job_bl[j] = cost[first[j]] + m;
        for (int r = 0; r < rows[j]; r++) blevel[first[j] + r] = job_bl[j];
    }

    // entry e = q * per_q + first[j] + r; dependencies per entry
    auto job_of = [&](int local) {
        return (int)(std::upper_bound(first.begin(), first.end(), local) - first.begin()) - 1;
    };
    std::vector<int32_t> remaining(total);
    for (int q = 0; q < nq; q++)
        for (int j = 0; j < nj; j++) {
            int nd = 0;
            for (int32_t p : jobs[j].preds) nd += rows[p];
            for (int r = 0; r < rows[j]; r++) remaining[q * per_q + first[j] + r] = nd;
        }
    std::vector<int32_t> ndeps = remaining;

    // list scheduling: earliest-free simulated workgroup takes the released
    // entry of largest critical path
    struct Avail {
        double bl;
        int e;
        bool operator<(const Avail &o) const { return bl < o.bl || (bl == o.bl && e > o.e); }
    };
    std::priority_queue<Avail> avail;
    typedef std::pair<double, int> Ev;  // (finish time, entry)
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> finishes;
    std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
    for (int w = 0; w < std::max(workers, 1); w++) free_at.push(0.0);
    for (int e = 0; e < total; e++)
        if (remaining[e] == 0) avail.push({blevel[e % per_q], e});
    std::vector<int32_t> order;
    order.reserve(total);
    double makespan = 0.0;
    auto release = [&](int e) {
        const int q = e / per_q, j = job_of(e % per_q);
        for (int32_t s : succ_jobs[j])
            for (int r = 0; r < rows[s]; r++) {
                const int f = q * per_q + first[s] + r;
                if (--remaining[f] == 0) avail.push({blevel[first[s] + r], f});
            }
    };
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
        const double fin = t + cost[a.e % per_q];
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
        const int e = order[i], q = e / per_q, loc = e % per_q, j = job_of(loc), r = loc - first[j];
        const GJob &g = jobs[j];
        PTask t{};
        t.out_row = g.out_row + (int64_t)r * bm[j];
        t.out_buf = g.out_buf;
        t.M = std::min(bm[j], g.M - r * bm[j]);
        t.m0 = r * bm[j];
        t.seg_begin = g.seg_begin;
        t.seg_end = g.seg_end;
        t.bm = bm[j];
        t.accumulate = g.accumulate;
        t.qtile = q;
        t.mat = 0;
        t.ndeps = ndeps[e];
        t.succ_begin = (int32_t)succ.size();
        for (int32_t s : succ_jobs[j])
            for (int rr = 0; rr < rows[s]; rr++) succ.push_back(pos[q * per_q + first[s] + rr]);
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
                    std::string("hm_eval: uploading the task graph: ") + hipGetErrorString(err));
    }
    plan.bn = bn;
    plan.Q = Q;
    plan.n_tasks = total;
    plan.est_ms = makespan;
    return HM_OK;
}

}  // namespace hm
