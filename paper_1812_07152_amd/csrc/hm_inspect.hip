// hm_inspect.hip -- host-side inspector: compress a point set into the H^2
// representation that hm_load_compressed_mem evaluates (the compression
// phase of the paper, Section 3.1: tree construction, interaction
// computation, sampling, low-rank approximation by interpolative
// decomposition).  Host C++ only; nodes of one tree level are processed in
// parallel threads.
//
// Readings (the paper leaves these open):
//   tree      perfect binary tree of the smallest depth L with leaves of at
//             most m points; a node is cut at the median of its widest
//             bounding-box coordinate (lowest coordinate on ties), points
//             ordered by (coordinate value, original index);
//   geometry  dist = centroid distance, diam = 2 * max distance to the
//             centroid; far iff tau * dist > diam(a) + diam(b) (Section 2.1),
//             or every off-diagonal pair for HSS (Section 4.1);
//   sampling  the rows of a node's ID are its whole far field F(a) (far
//             partners of a and of its ancestors) if |F(a)| <= S, otherwise
//             S/2 points from the nearest far clusters plus the remaining
//             far points with the smallest SplitMix64 keys;
//   ID        Householder QR with column pivoting on exactly recomputed
//             column norms; rank = first j with |R_jj| <= tol |R_11|, capped
//             at max_rank; the interpolation matrix is [I, R11^-1 R12] in the
//             pivoted column order.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <thread>

#include "hm_internal.h"


namespace hm {
namespace {

void parallel_for(int64_t n, int threads, const std::function<void(int64_t)> &fn) {
    if (n <= 0) return;
    const int t = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n));
    if (t == 1) {
        for (int64_t i = 0; i < n; i++) fn(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> pool;
    for (int w = 0; w < t; w++)
        pool.emplace_back([&] {
            for (int64_t i; (i = next.fetch_add(1)) < n;) fn(i);
        });
    for (auto &th : pool) th.join();
}

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014), used as a
// counter-based generator: key = f(f(f(seed) ^ node) ^ point).
uint64_t splitmix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Inspector {
    const double *X;
    int64_t N, d;
    hm_compress_opts o;
    int threads;
    HostRepr &R;
    std::vector<double> cen, rad;
    std::vector<std::vector<int64_t>> skel;  // per node, original indices

    double kval(int64_t i, int64_t j) const {
        const double *x = X + i * d, *y = X + j * d;
        double r2 = 0.0;
        for (int64_t t = 0; t < d; t++) {
            const double df = x[t] - y[t];
            r2 += df * df;
        }
        return o.kernel == 0 ? std::exp(-r2 / (2.0 * o.h * o.h)) : std::exp(-std::sqrt(r2) / o.h);
    }
    double cdist(int a, int b) const {
        double r2 = 0.0;
        for (int64_t t = 0; t < d; t++) {
            const double df = cen[a * d + t] - cen[b * d + t];
            r2 += df * df;
        }
        return std::sqrt(r2);
    }
    bool leaf(int a) const { return R.left[a] < 0; }

    void tree() {
        int L = 0;
        while (((N + ((int64_t)1 << L) - 1) >> L) > o.leaf_size) L++;
        const int n = (int)(((int64_t)2 << L) - 1);
        R.N = N;
        R.d = d;
        R.n_nodes = n;
        R.depth = L;
        R.perm.resize(N);
        for (int64_t t = 0; t < N; t++) R.perm[t] = t;
        R.start.assign(n, 0);
        R.size.assign(n, 0);
        R.parent.assign(n, -1);
        R.left.assign(n, -1);
        R.right.assign(n, -1);
        R.level.assign(n, 0);
        R.size[0] = N;
        for (int lev = 0; lev <= L; lev++) {
            const int first = (1 << lev) - 1, count = 1 << lev;
            parallel_for(count, threads, [&](int64_t q) {
                const int a = first + (int)q;
                R.level[a] = lev;
                if (lev == L) return;
                const int64_t s = R.start[a], sz = R.size[a];
                if (o.partitioner == 1) {
                    two_means_split(a, s, sz);
                    return;
                }
                int jstar = 0;
                double best = -1.0;
                for (int64_t t = 0; t < d; t++) {
                    double lo = INFINITY, hi = -INFINITY;
                    for (int64_t p = s; p < s + sz; p++) {
                        const double v = X[R.perm[p] * d + t];
                        lo = std::min(lo, v);
                        hi = std::max(hi, v);
                    }
                    if (hi - lo > best) {
                        best = hi - lo;
                        jstar = (int)t;
                    }
                }
                std::sort(R.perm.begin() + s, R.perm.begin() + s + sz, [&](int64_t x, int64_t y) {
                    const double vx = X[x * d + jstar], vy = X[y * d + jstar];
                    return vx < vy || (vx == vy && x < y);
                });
                const int l = 2 * a + 1, r = 2 * a + 2;
                R.left[a] = l;
                R.right[a] = r;
                R.parent[l] = R.parent[r] = a;
                R.start[l] = s;
                R.size[l] = sz / 2;
                R.start[r] = s + sz / 2;
                R.size[r] = sz - sz / 2;
            });
        }
    }

    static double dist2(const double *x, const double *y, int64_t d) {
        double r2 = 0.0;
        for (int64_t t = 0; t < d; t++) {
            const double df = x[t] - y[t];
            r2 += df * df;
        }
        return r2;
    }

    // Two-means split of node a over tree positions [s, s + sz): Lloyd's
    // 2-means from the point farthest from the centroid and the point
    // farthest from it (lowest index on ties; a point joins the second mean
    // only when strictly nearer), until the assignment repeats (at most 100
    // rounds, or until a group would be empty); then the median cut along the
    // direction between the two means, points ordered by (projection, index).
    void two_means_split(int a, int64_t s, int64_t sz) {
        std::vector<double> cen((size_t)d, 0.0), c1((size_t)d), c2((size_t)d), m1((size_t)d), m2((size_t)d);
        const int64_t *pp = R.perm.data() + s;
        for (int64_t p = 0; p < sz; p++)
            for (int64_t t = 0; t < d; t++) cen[(size_t)t] += X[pp[p] * d + t];
        for (int64_t t = 0; t < d; t++) cen[(size_t)t] /= (double)sz;
        int64_t i1 = -1, i2 = -1;
        double best = -1.0;
        for (int64_t p = 0; p < sz; p++) {
            const int64_t i = pp[p];
            const double r2 = dist2(X + i * d, cen.data(), d);
            if (r2 > best || (r2 == best && i < i1)) {
                best = r2;
                i1 = i;
            }
        }
        best = -1.0;
        for (int64_t p = 0; p < sz; p++) {
            const int64_t i = pp[p];
            const double r2 = dist2(X + i * d, X + i1 * d, d);
            if (r2 > best || (r2 == best && i < i2)) {
                best = r2;
                i2 = i;
            }
        }
        std::copy(X + i1 * d, X + i1 * d + d, c1.begin());
        std::copy(X + i2 * d, X + i2 * d + d, c2.begin());
        std::vector<unsigned char> grp((size_t)sz), prev((size_t)sz);
        for (int64_t p = 0; p < sz; p++) {
            const double *x = X + pp[p] * d;
            grp[(size_t)p] = dist2(x, c2.data(), d) < dist2(x, c1.data(), d);
        }
        for (int it = 0; it < 100; it++) {
            int64_t n1 = 0, n2 = 0;
            std::fill(m1.begin(), m1.end(), 0.0);
            std::fill(m2.begin(), m2.end(), 0.0);
            for (int64_t p = 0; p < sz; p++) {
                const double *x = X + pp[p] * d;
                std::vector<double> &m = grp[(size_t)p] ? m2 : m1;
                for (int64_t t = 0; t < d; t++) m[(size_t)t] += x[t];
                if (grp[(size_t)p])
                    n2++;
                else
                    n1++;
            }
            if (n1 == 0 || n2 == 0) break;
            for (int64_t t = 0; t < d; t++) {
                c1[(size_t)t] = m1[(size_t)t] / (double)n1;
                c2[(size_t)t] = m2[(size_t)t] / (double)n2;
            }
            prev = grp;
            bool changed = false;
            for (int64_t p = 0; p < sz; p++) {
                const double *x = X + pp[p] * d;
                grp[(size_t)p] = dist2(x, c2.data(), d) < dist2(x, c1.data(), d);
                changed |= grp[(size_t)p] != prev[(size_t)p];
            }
            if (!changed) break;
        }
        std::vector<std::pair<double, int64_t>> key((size_t)sz);
        for (int64_t p = 0; p < sz; p++) {
            const int64_t i = pp[p];
            double v = 0.0;
            for (int64_t t = 0; t < d; t++) v += X[i * d + t] * (c2[(size_t)t] - c1[(size_t)t]);
            key[(size_t)p] = {v, i};
        }
        std::sort(key.begin(), key.end());
        for (int64_t p = 0; p < sz; p++) R.perm[(size_t)(s + p)] = key[(size_t)p].second;
        const int l = 2 * a + 1, r = 2 * a + 2;
        R.left[a] = l;
        R.right[a] = r;
        R.parent[l] = R.parent[r] = a;
        R.start[l] = s;
        R.size[l] = sz / 2;
        R.start[r] = s + sz / 2;
        R.size[r] = sz - sz / 2;
    }

    void geometry() {
        const int n = R.n_nodes;
        cen.assign((size_t)n * d, 0.0);
        rad.assign(n, 0.0);
        parallel_for(n, threads, [&](int64_t a) {
            double *c = &cen[a * d];
            for (int64_t p = R.start[a]; p < R.start[a] + R.size[a]; p++)
                for (int64_t t = 0; t < d; t++) c[t] += X[R.perm[p] * d + t];
            for (int64_t t = 0; t < d; t++) c[t] /= (double)R.size[a];
            double m2 = 0.0;
            for (int64_t p = R.start[a]; p < R.start[a] + R.size[a]; p++) {
                double r2 = 0.0;
                for (int64_t t = 0; t < d; t++) {
                    const double df = X[R.perm[p] * d + t] - c[t];
                    r2 += df * df;
                }
                m2 = std::max(m2, r2);
            }
            rad[a] = std::sqrt(m2);
        });
    }

    // Budget admissibility: near leaves as a prefix-summed 0/1 matrix, so
    // that "some leaf below a is near some leaf below b" is one lookup.
    int nl_ = 0, first_leaf_ = 0;
    std::vector<int32_t> near_sum_;  // (nl+1) x (nl+1) inclusive prefix sums

    void budget_near() {
        const int L = R.depth;
        nl_ = 1 << L;
        first_leaf_ = nl_ - 1;
        int64_t kb = (int64_t)std::floor(o.budget * nl_);
        kb = std::min<int64_t>(kb, nl_ - 1);
        std::vector<unsigned char> nearm((size_t)nl_ * nl_, 0);
        std::vector<std::pair<double, int>> cl;
        for (int x = 0; x < nl_; x++) {
            nearm[(size_t)x * nl_ + x] = 1;
            cl.clear();
            for (int y = 0; y < nl_; y++)
                if (y != x) cl.push_back({cdist(first_leaf_ + x, first_leaf_ + y), first_leaf_ + y});
            std::partial_sort(cl.begin(), cl.begin() + kb, cl.end());
            for (int64_t j = 0; j < kb; j++) {
                const int y = cl[(size_t)j].second - first_leaf_;
                nearm[(size_t)x * nl_ + y] = nearm[(size_t)y * nl_ + x] = 1;
            }
        }
        near_sum_.assign((size_t)(nl_ + 1) * (nl_ + 1), 0);
        for (int x = 0; x < nl_; x++)
            for (int y = 0; y < nl_; y++)
                near_sum_[(size_t)(x + 1) * (nl_ + 1) + y + 1] = nearm[(size_t)x * nl_ + y] +
                                                                  near_sum_[(size_t)x * (nl_ + 1) + y + 1] +
                                                                  near_sum_[(size_t)(x + 1) * (nl_ + 1) + y] -
                                                                  near_sum_[(size_t)x * (nl_ + 1) + y];
    }

    bool admissible(int a, int b) const {
        if (a == b) return false;
        if (o.admissibility == 1) return true;
        if (o.admissibility == 2) {
            // leaves below a node of level l: 2^(L-l) consecutive ones from (a+1) 2^(L-l) - 1
            const int64_t ca = (int64_t)1 << (R.depth - R.level[a]), cb = (int64_t)1 << (R.depth - R.level[b]);
            const int64_t fa = (a + 1) * ca - 1 - first_leaf_, fb = (b + 1) * cb - 1 - first_leaf_;
            const int64_t w = nl_ + 1;
            const int32_t cnt = near_sum_[(size_t)((fa + ca) * w + fb + cb)] - near_sum_[(size_t)(fa * w + fb + cb)] -
                                near_sum_[(size_t)((fa + ca) * w + fb)] + near_sum_[(size_t)(fa * w + fb)];
            return cnt == 0;
        }
        return o.tau * cdist(a, b) > 2.0 * rad[a] + 2.0 * rad[b];
    }

    void interactions() {
        if (o.admissibility == 2) budget_near();
        std::vector<std::pair<int, int>> far, near;
        std::vector<std::pair<int, int>> stack{{0, 0}};
        while (!stack.empty()) {
            auto [a, b] = stack.back();
            stack.pop_back();
            const bool la = leaf(a), lb = leaf(b);
            std::vector<std::pair<int, int>> kids;
            if (a == b) {
                if (la) {
                    near.push_back({a, a});
                    continue;
                }
                const int l = R.left[a], r = R.right[a];
                kids = {{l, l}, {l, r}, {r, l}, {r, r}};
            } else if (admissible(a, b)) {
                far.push_back({a, b});
                continue;
            } else if (la && lb) {
                near.push_back({a, b});
                continue;
            } else if (la) {
                kids = {{a, R.left[b]}, {a, R.right[b]}};
            } else if (lb) {
                kids = {{R.left[a], b}, {R.right[a], b}};
            } else {
                kids = {{R.left[a], R.left[b]}, {R.left[a], R.right[b]},
                        {R.right[a], R.left[b]}, {R.right[a], R.right[b]}};
            }
            for (auto it = kids.rbegin(); it != kids.rend(); ++it) stack.push_back(*it);
        }
        auto csr = [&](std::vector<std::pair<int, int>> &pairs, std::vector<int64_t> &ptr,
                       std::vector<int32_t> &col) {
            std::sort(pairs.begin(), pairs.end());
            ptr.assign(R.n_nodes + 1, 0);
            col.resize(pairs.size());
            for (size_t e = 0; e < pairs.size(); e++) {
                ptr[pairs[e].first + 1]++;
                col[e] = pairs[e].second;
            }
            for (int a = 0; a < R.n_nodes; a++) ptr[a + 1] += ptr[a];
        };
        csr(far, R.far_ptr, R.far_col);
        csr(near, R.near_ptr, R.near_col);
    }

    // Tree positions of the ID rows of node a (ascending).
    std::vector<int64_t> sample_rows(int a) const {
        struct Cl {
            double dist;
            int node;
        };
        std::vector<Cl> cl;
        int64_t total = 0;
        for (int x = a; x >= 0; x = R.parent[x])
            for (int64_t e = R.far_ptr[x]; e < R.far_ptr[x + 1]; e++) {
                const int b = R.far_col[e];
                cl.push_back({cdist(a, b), b});
                total += R.size[b];
            }
        std::vector<int64_t> rows;
        if (total <= o.sample_rows) {
            for (const Cl &c : cl)
                for (int64_t p = 0; p < R.size[c.node]; p++) rows.push_back(R.start[c.node] + p);
        } else {
            std::sort(cl.begin(), cl.end(), [](const Cl &x, const Cl &y) {
                return x.dist < y.dist || (x.dist == y.dist && x.node < y.node);
            });
            const int64_t half = o.sample_rows / 2;
            size_t i = 0;
            int64_t part = 0;
            while ((int64_t)rows.size() < half) {
                rows.push_back(R.start[cl[i].node] + part);
                if (++part == R.size[cl[i].node]) {
                    i++;
                    part = 0;
                }
            }
            const uint64_t base = splitmix(splitmix(o.seed) ^ (uint64_t)a);
            std::vector<std::pair<uint64_t, int64_t>> keyed;
            for (size_t j = i; j < cl.size(); j++)
                for (int64_t p = (j == i ? part : 0); p < R.size[cl[j].node]; p++) {
                    const int64_t pos = R.start[cl[j].node] + p;
                    keyed.push_back({splitmix(base ^ (uint64_t)R.perm[pos]), pos});
                }
            const int64_t need = o.sample_rows - (int64_t)rows.size();
            std::partial_sort(keyed.begin(), keyed.begin() + need, keyed.end());
            for (int64_t j = 0; j < need; j++) rows.push_back(keyed[j].second);
        }
        std::sort(rows.begin(), rows.end());
        return rows;
    }

    // Pivoted-QR ID of the column-major mr x nc matrix A (overwritten).
    // Returns the rank; piv receives the column order, P (k x nc, row-major)
    // the interpolation matrix.
    int id(std::vector<double> &A, int64_t mr, int nc, std::vector<int> &piv,
           std::vector<double> &P) const {
        const int cap = (int)std::min<int64_t>({(int64_t)o.max_rank, (int64_t)nc, mr});
        piv.resize(nc);
        for (int j = 0; j < nc; j++) piv[j] = j;
        std::vector<double> v(mr);
        double r11 = 0.0;
        int k = 0;
        for (int j = 0;; j++) {
            if (j >= nc || j >= mr) {
                k = j;
                break;
            }
            int p = j;
            double best = -1.0;
            for (int c = j; c < nc; c++) {
                const double *col = &A[(size_t)c * mr];
                double s2 = 0.0;
                for (int64_t i = j; i < mr; i++) s2 += col[i] * col[i];
                if (s2 > best) {
                    best = s2;
                    p = c;
                }
            }
            const double rjj = std::sqrt(best);
            if (j == 0) r11 = rjj;
            if (rjj == 0.0 || (j > 0 && rjj <= o.tol * r11) || j == cap) {
                k = j;
                break;
            }
            if (p != j) {
                std::swap_ranges(A.begin() + (size_t)j * mr, A.begin() + (size_t)(j + 1) * mr,
                                 A.begin() + (size_t)p * mr);
                std::swap(piv[j], piv[p]);
            }
            double *aj = &A[(size_t)j * mr];
            const double alpha = aj[j] >= 0.0 ? -rjj : rjj;
            for (int64_t i = j; i < mr; i++) v[i] = aj[i];
            v[j] -= alpha;
            double vtv = 0.0;
            for (int64_t i = j; i < mr; i++) vtv += v[i] * v[i];
            aj[j] = alpha;
            for (int64_t i = j + 1; i < mr; i++) aj[i] = 0.0;
            if (vtv > 0.0)
                for (int c = j + 1; c < nc; c++) {
                    double *col = &A[(size_t)c * mr];
                    double s = 0.0;
                    for (int64_t i = j; i < mr; i++) s += v[i] * col[i];
                    const double f = 2.0 * s / vtv;
                    for (int64_t i = j; i < mr; i++) col[i] -= f * v[i];
                }
        }
        // T = R11^{-1} R12 by back substitution; P[:, piv[i]] = e_i, P[:, piv[k+c]] = T[:, c]
        const int nr = nc - k;
        std::vector<double> T((size_t)k * nr);
        for (int c = 0; c < nr; c++)
            for (int i = k - 1; i >= 0; i--) {
                double s = A[(size_t)(k + c) * mr + i];
                for (int t = i + 1; t < k; t++) s -= A[(size_t)t * mr + i] * T[(size_t)t * nr + c];
                T[(size_t)i * nr + c] = s / A[(size_t)i * mr + i];
            }
        P.assign((size_t)k * nc, 0.0);
        for (int i = 0; i < k; i++) {
            P[(size_t)i * nc + piv[i]] = 1.0;
            for (int c = 0; c < nr; c++) P[(size_t)i * nc + piv[k + c]] = T[(size_t)i * nr + c];
        }
        return k;
    }

    void compress() {
        const int n = R.n_nodes;
        R.rank.assign(n, 0);
        skel.assign(n, {});
        std::vector<std::vector<double>> bases(n);
        for (int lev = R.depth; lev >= 0; lev--) {
            const int first = (1 << lev) - 1, count = 1 << lev;
            parallel_for(count, threads, [&](int64_t q) {
                const int a = first + (int)q;
                std::vector<int64_t> cand;
                if (leaf(a)) {
                    for (int64_t p = 0; p < R.size[a]; p++) cand.push_back(R.perm[R.start[a] + p]);
                } else {
                    cand = skel[R.left[a]];
                    cand.insert(cand.end(), skel[R.right[a]].begin(), skel[R.right[a]].end());
                }
                const std::vector<int64_t> rows = sample_rows(a);
                const int64_t mr = (int64_t)rows.size();
                const int nc = (int)cand.size();
                if (mr == 0 || nc == 0) return;
                std::vector<double> A((size_t)mr * nc);
                for (int j = 0; j < nc; j++)
                    for (int64_t i = 0; i < mr; i++) A[(size_t)j * mr + i] = kval(R.perm[rows[i]], cand[j]);
                std::vector<int> piv;
                const int k = id(A, mr, nc, piv, bases[a]);
                R.rank[a] = k;
                for (int i = 0; i < k; i++) skel[a].push_back(cand[piv[i]]);
            });
        }
        R.basis_off.assign(n, 0);
        int64_t off = 0;
        for (int a = 0; a < n; a++) {
            R.basis_off[a] = off;
            off += (int64_t)bases[a].size();
        }
        R.basis.resize(off);
        for (int a = 0; a < n; a++) std::copy(bases[a].begin(), bases[a].end(), R.basis.begin() + R.basis_off[a]);
        R.basis_len = off;
    }

    void blocks() {
        const int n = R.n_nodes;
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
        R.B.resize(bo);
        R.D.resize(dof);
        R.B_len = bo;
        R.D_len = dof;
        parallel_for(n, threads, [&](int64_t a) {
            for (int64_t e = R.far_ptr[a]; e < R.far_ptr[a + 1]; e++) {
                const int b = R.far_col[e];
                double *blk = &R.B[R.far_off[e]];
                for (int i = 0; i < R.rank[a]; i++)
                    for (int j = 0; j < R.rank[b]; j++) blk[(size_t)i * R.rank[b] + j] = kval(skel[a][i], skel[b][j]);
            }
            for (int64_t e = R.near_ptr[a]; e < R.near_ptr[a + 1]; e++) {
                const int b = R.near_col[e];
                double *blk = &R.D[R.near_off[e]];
                for (int64_t i = 0; i < R.size[a]; i++)
                    for (int64_t j = 0; j < R.size[b]; j++)
                        blk[i * R.size[b] + j] = kval(R.perm[R.start[a] + i], R.perm[R.start[b] + j]);
            }
        });
    }
};

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" {

hm_status hm_compress(const double *X, int64_t N, int64_t d, const hm_compress_opts *opts,
                      hm_repr *out) {
    if (!out) return fail(HM_ERR_INVALID, "hm_compress: out is NULL");
    *out = nullptr;
    if (!X || !opts) return fail(HM_ERR_INVALID, "hm_compress: NULL argument");
    if (N < 1 || d < 1) return fail(HM_ERR_INVALID, "hm_compress: need N >= 1 and d >= 1");
    if (opts->leaf_size < 2 || opts->max_rank < 0 || opts->sample_rows < 1 || !(opts->h > 0.0) ||
        !(opts->tol >= 0.0) || (opts->kernel != 0 && opts->kernel != 1) ||
        opts->admissibility < 0 || opts->admissibility > 2 || opts->partitioner < 0 || opts->partitioner > 1 ||
        !(opts->budget >= 0.0 && opts->budget <= 1.0))
        return fail(HM_ERR_INVALID, "hm_compress: invalid options");
    for (int64_t i = 0; i < N * d; i++)
        if (!std::isfinite(X[i])) return fail(HM_ERR_INVALID, "hm_compress: non-finite point coordinate");
    hm_repr r = new (std::nothrow) hm_repr_s();
    if (!r) return fail(HM_ERR_NOMEM, "hm_compress: allocation failed");
    unsigned hw = std::thread::hardware_concurrency();
    Inspector I{X, N, d, *opts, opts->threads > 0 ? opts->threads : (int)std::max(1u, hw), r->r, {}, {}, {}};
    I.tree();
    I.geometry();
    I.interactions();
    I.compress();
    I.blocks();
    HostRepr &R = r->r;
    R.kernel = opts->kernel;
    R.h = opts->h;
    R.tol = opts->tol;
    R.tau = opts->tau;
    R.rmax = opts->max_rank;
    R.m = opts->leaf_size;
    R.flags = opts->admissibility == 1 ? 1u : opts->admissibility == 2 ? 2u : 0u;
    r->skel_ptr.assign(R.n_nodes + 1, 0);
    for (int a = 0; a < R.n_nodes; a++) {
        r->skel_ptr[a + 1] = r->skel_ptr[a] + (int64_t)I.skel[a].size();
        r->skel.insert(r->skel.end(), I.skel[a].begin(), I.skel[a].end());
    }
    hm_status st = validate(R);
    if (st != HM_OK) {
        delete r;
        return st;
    }
    *out = r;
    return HM_OK;
}

hm_status hm_inspect_p1(const double *X, int64_t N, int64_t d, const hm_compress_opts *opts,
                        hm_structure *out) {
    if (!out) return fail(HM_ERR_INVALID, "hm_inspect_p1: out is NULL");
    *out = nullptr;
    if (!X || !opts) return fail(HM_ERR_INVALID, "hm_inspect_p1: NULL argument");
    if (N < 1 || d < 1) return fail(HM_ERR_INVALID, "hm_inspect_p1: need N >= 1 and d >= 1");
    if (opts->leaf_size < 2 || opts->sample_rows < 1 || opts->admissibility < 0 || opts->admissibility > 2 ||
        !(opts->tau >= 0.0) || opts->partitioner < 0 || opts->partitioner > 1 ||
        !(opts->budget >= 0.0 && opts->budget <= 1.0))
        return fail(HM_ERR_INVALID, "hm_inspect_p1: invalid options");
    for (int64_t i = 0; i < N * d; i++)
        if (!std::isfinite(X[i])) return fail(HM_ERR_INVALID, "hm_inspect_p1: non-finite point coordinate");
    hm_structure st = new (std::nothrow) hm_structure_s();
    if (!st) return fail(HM_ERR_NOMEM, "hm_inspect_p1: allocation failed");
    unsigned hw = std::thread::hardware_concurrency();
    const int threads = opts->threads > 0 ? opts->threads : (int)std::max(1u, hw);
    Structure &S = st->s;
    Inspector I{X, N, d, *opts, threads, S.r, {}, {}, {}};
    I.tree();
    I.geometry();
    I.interactions();
    // the row sample of every node (original point indices), in tree-position order
    const int n = S.r.n_nodes;
    std::vector<std::vector<int64_t>> rows((size_t)n);
    parallel_for(n, threads, [&](int64_t a) {
        rows[(size_t)a] = I.sample_rows((int)a);
        for (int64_t &t : rows[(size_t)a]) t = S.r.perm[(size_t)t];
    });
    S.rows_ptr.assign((size_t)n + 1, 0);
    for (int a = 0; a < n; a++) S.rows_ptr[(size_t)a + 1] = S.rows_ptr[(size_t)a] + (int64_t)rows[(size_t)a].size();
    S.rows.resize((size_t)S.rows_ptr[(size_t)n]);
    for (int a = 0; a < n; a++) std::copy(rows[(size_t)a].begin(), rows[(size_t)a].end(), S.rows.begin() + S.rows_ptr[(size_t)a]);
    S.X.assign(X, X + N * d);
    S.leaf_size = opts->leaf_size;
    S.admissibility = opts->admissibility;
    S.tau = opts->tau;
    S.r.m = opts->leaf_size;
    S.r.tau = opts->tau;
    S.r.flags = opts->admissibility == 1 ? 1u : opts->admissibility == 2 ? 2u : 0u;
    *out = st;
    return HM_OK;
}

hm_status hm_structure_info(hm_structure s, hm_structure_info_t *o) {
    if (!s || !o) return fail(HM_ERR_INVALID, "hm_structure_info: NULL argument");
    const Structure &S = s->s;
    o->N = S.r.N;
    o->d = S.r.d;
    o->n_nodes = S.r.n_nodes;
    o->depth = S.r.depth;
    o->n_far = (int64_t)S.r.far_col.size();
    o->n_near = (int64_t)S.r.near_col.size();
    o->rows_total = (int64_t)S.rows.size();
    return HM_OK;
}

hm_status hm_structure_rows(hm_structure s, int32_t node, int64_t *rows, int64_t cap, int64_t *count) {
    if (!s || !count) return fail(HM_ERR_INVALID, "hm_structure_rows: NULL argument");
    const Structure &S = s->s;
    if (node < 0 || node >= S.r.n_nodes) return fail(HM_ERR_INVALID, "hm_structure_rows: no such node");
    const int64_t b = S.rows_ptr[(size_t)node], e = S.rows_ptr[(size_t)node + 1];
    *count = e - b;
    if (rows) {
        if (cap < e - b) return fail(HM_ERR_INVALID, "hm_structure_rows: cap too small");
        std::copy(S.rows.begin() + b, S.rows.begin() + e, rows);
    }
    return HM_OK;
}

hm_status hm_structure_free(hm_structure s) {
    delete s;
    return HM_OK;
}

hm_status hm_repr_view(hm_repr h, hm_host_repr *v) {
    if (!h || !v) return fail(HM_ERR_INVALID, "hm_repr_view: NULL argument");
    const HostRepr &R = h->r;
    v->N = R.N;
    v->d = R.d;
    v->n_nodes = R.n_nodes;
    v->depth = R.depth;
    v->flags = R.flags;
    v->kernel = R.kernel;
    v->h = R.h;
    v->tol = R.tol;
    v->tau = R.tau;
    v->rmax = R.rmax;
    v->m = R.m;
    v->n_far = (int64_t)R.far_col.size();
    v->n_near = (int64_t)R.near_col.size();
    v->basis_len = R.basis_len;
    v->B_len = R.B_len;
    v->D_len = R.D_len;
    v->skel_len = (int64_t)h->skel.size();
    v->perm = R.perm.data();
    v->start = R.start.data();
    v->size = R.size.data();
    v->parent = R.parent.data();
    v->left = R.left.data();
    v->right = R.right.data();
    v->level = R.level.data();
    v->rank = R.rank.data();
    v->basis_off = R.basis_off.data();
    v->basis = R.basis.data();
    v->far_ptr = R.far_ptr.data();
    v->far_col = R.far_col.data();
    v->far_off = R.far_off.data();
    v->B = R.B.data();
    v->near_ptr = R.near_ptr.data();
    v->near_col = R.near_col.data();
    v->near_off = R.near_off.data();
    v->D = R.D.data();
    v->skel_ptr = h->skel_ptr.data();
    v->skel = h->skel.data();
    return HM_OK;
}

hm_status hm_repr_write(hm_repr h, const char *path) {
    if (!h || !path) return fail(HM_ERR_INVALID, "hm_repr_write: NULL argument");
    const HostRepr &R = h->r;
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(HM_ERR_INVALID, std::string("hm_repr_write: cannot create ") + path);
    unsigned char hdr[128] = {0};
    auto put = [&](int off, const void *p, size_t n) { std::memcpy(hdr + off, p, n); };
    const uint32_t version = 1;
    const int64_t n_far = (int64_t)R.far_col.size(), n_near = (int64_t)R.near_col.size();
    const int64_t skel_len = (int64_t)h->skel.size();
    std::memcpy(hdr, "HMC1", 4);
    put(4, &version, 4);
    put(8, &R.N, 8);
    put(16, &R.d, 8);
    put(24, &R.n_nodes, 4);
    put(28, &R.depth, 4);
    put(32, &R.flags, 4);
    put(36, &R.kernel, 4);
    put(40, &R.h, 8);
    put(48, &R.tol, 8);
    put(56, &R.tau, 8);
    put(64, &R.rmax, 4);
    put(68, &R.m, 4);
    put(72, &n_far, 8);
    put(80, &n_near, 8);
    put(88, &R.basis_len, 8);
    put(96, &R.B_len, 8);
    put(104, &R.D_len, 8);
    put(112, &skel_len, 8);
    bool ok = std::fwrite(hdr, 1, 128, f) == 128;
    auto w = [&](const auto &vec) {
        const size_t bytes = vec.size() * sizeof(vec[0]);
        if (ok && bytes) ok = std::fwrite(vec.data(), 1, bytes, f) == bytes;
    };
    w(R.perm); w(R.start); w(R.size); w(R.parent); w(R.left); w(R.right); w(R.level); w(R.rank);
    w(R.basis_off); w(R.basis); w(R.far_ptr); w(R.far_col); w(R.far_off); w(R.B);
    w(R.near_ptr); w(R.near_col); w(R.near_off); w(R.D); w(h->skel_ptr); w(h->skel);
    if (std::fclose(f) != 0) ok = false;
    return ok ? HM_OK : fail(HM_ERR_INVALID, std::string("hm_repr_write: write failed for ") + path);
}

hm_status hm_repr_free(hm_repr h) {
    delete h;
    return HM_OK;
}

}  // extern "C"
