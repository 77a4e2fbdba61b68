// hm_store.hip -- loading, validation and the device-resident block store.
//
// Device layout (the GPU analogue of the paper's CDS format, Section 3.2
// "Data layout construction": submatrices are stored in the order the
// evaluation visits them, with offsets derived from the ranks):
//   up pass, levels deepest..1:   per node, its leaf basis P_a or transfer T_a
//   down pass, levels 1..deepest: per node, its coupling blocks B_ab (far list
//                                 order) and then its slice of the parent's
//                                 transfer
//   leaf pass:                    per leaf, its near blocks D_ab (near list
//                                 order) and then P_a for the leaf's far part
// Every block is stored K-major (the contraction index is the slow one) with
// its output-row count zero-padded to a multiple of 16, so one contraction
// step of a block is a contiguous, 16-byte aligned run of memory and the
// kernels load it with full-width vector loads.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <thread>

#include "hm_internal.h"

namespace hm {

namespace {

// ---------------------------------------------------------------------------
// HMC1 parsing

struct Reader {
    const unsigned char *p;
    size_t n, off = 0;
    bool take(void *dst, size_t bytes) {
        if (bytes > n - off) return false;
        if (bytes) std::memcpy(dst, p + off, bytes);
        off += bytes;
        return true;
    }
    template <class T>
    bool vec(std::vector<T> &v, int64_t count) {
        if (count < 0) return false;
        if ((size_t)count > (n - off) / sizeof(T)) return false;
        v.resize((size_t)count);
        return take(v.data(), sizeof(T) * (size_t)count);
    }
};

template <class T>
T field(const unsigned char *hdr, int off) {
    T v;
    std::memcpy(&v, hdr + off, sizeof(T));
    return v;
}

}  // namespace

hm_status read_file(const char *path, HostRepr &r) {
    if (!path) return fail(HM_ERR_INVALID, "hm_load_compressed: path is NULL");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(HM_ERR_INVALID, std::string("hm_load_compressed: cannot open ") + path);
    std::fseek(f, 0, SEEK_END);
    long long len = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    if (len < 128) {
        std::fclose(f);
        return fail(HM_ERR_FORMAT, "HMC1: file shorter than the 128-byte header");
    }
    std::vector<unsigned char> buf((size_t)len);
    size_t got = std::fread(buf.data(), 1, buf.size(), f);
    std::fclose(f);
    if (got != buf.size()) return fail(HM_ERR_FORMAT, "HMC1: short read");
    const unsigned char *h = buf.data();
    if (std::memcmp(h, "HMC1", 4) != 0) return fail(HM_ERR_FORMAT, "HMC1: bad magic");
    if (field<uint32_t>(h, 4) != 1u) return fail(HM_ERR_FORMAT, "HMC1: unsupported version");
    r.N = field<int64_t>(h, 8);
    r.d = field<int64_t>(h, 16);
    r.n_nodes = field<int32_t>(h, 24);
    r.depth = field<int32_t>(h, 28);
    r.flags = field<uint32_t>(h, 32);
    r.kernel = field<int32_t>(h, 36);
    r.h = field<double>(h, 40);
    r.tol = field<double>(h, 48);
    r.tau = field<double>(h, 56);
    r.rmax = field<int32_t>(h, 64);
    r.m = field<int32_t>(h, 68);
    int64_t n_far = field<int64_t>(h, 72), n_near = field<int64_t>(h, 80);
    int64_t basis_len = field<int64_t>(h, 88), B_len = field<int64_t>(h, 96);
    int64_t D_len = field<int64_t>(h, 104), skel_len = field<int64_t>(h, 112);
    if (r.N < 1 || r.n_nodes < 1 || n_far < 0 || n_near < 0 || basis_len < 0 || B_len < 0 ||
        D_len < 0 || skel_len < 0)
        return fail(HM_ERR_FORMAT, "HMC1: negative or empty sizes in header");
    Reader rd{h, buf.size(), 128};
    int64_t n = r.n_nodes;
    std::vector<int64_t> skel_ptr, skel;
    bool ok = rd.vec(r.perm, r.N) && rd.vec(r.start, n) && rd.vec(r.size, n) &&
              rd.vec(r.parent, n) && rd.vec(r.left, n) && rd.vec(r.right, n) &&
              rd.vec(r.level, n) && rd.vec(r.rank, n) && rd.vec(r.basis_off, n) &&
              rd.vec(r.basis, basis_len) && rd.vec(r.far_ptr, n + 1) && rd.vec(r.far_col, n_far) &&
              rd.vec(r.far_off, n_far) && rd.vec(r.B, B_len) && rd.vec(r.near_ptr, n + 1) &&
              rd.vec(r.near_col, n_near) && rd.vec(r.near_off, n_near) && rd.vec(r.D, D_len) &&
              rd.vec(skel_ptr, n + 1) && rd.vec(skel, skel_len);
    if (!ok) return fail(HM_ERR_FORMAT, "HMC1: file shorter than its header announces");
    if (rd.off != buf.size()) return fail(HM_ERR_FORMAT, "HMC1: trailing bytes after the arrays");
    r.basis_len = basis_len;
    r.B_len = B_len;
    r.D_len = D_len;
    if (skel_len > 0) {  // a file without skeletons stores skel_len 0
        r.skel_ptr = std::move(skel_ptr);
        r.skel = std::move(skel);
    }
    return validate(r);
}

hm_status from_view(const hm_host_repr &v, HostRepr &r) {
    if (v.N < 1 || v.n_nodes < 1 || v.n_far < 0 || v.n_near < 0 || v.basis_len < 0 ||
        v.B_len < 0 || v.D_len < 0)
        return fail(HM_ERR_FORMAT, "hm_host_repr: negative or empty sizes");
    const void *need[] = {v.perm, v.start, v.size, v.parent, v.left, v.right, v.level, v.rank,
                          v.basis_off, v.far_ptr, v.near_ptr};
    for (const void *p : need)
        if (!p) return fail(HM_ERR_INVALID, "hm_host_repr: required array pointer is NULL");
    if ((v.basis_len && !v.basis) || (v.n_far && (!v.far_col || !v.far_off)) ||
        (v.B_len && !v.B) || (v.n_near && (!v.near_col || !v.near_off)) || (v.D_len && !v.D))
        return fail(HM_ERR_INVALID, "hm_host_repr: array pointer is NULL");
    r.N = v.N; r.d = v.d; r.n_nodes = v.n_nodes; r.depth = v.depth; r.flags = v.flags;
    r.kernel = v.kernel; r.h = v.h; r.tol = v.tol; r.tau = v.tau; r.rmax = v.rmax; r.m = v.m;
    int64_t n = v.n_nodes;
    r.perm.assign(v.perm, v.perm + v.N);
    r.start.assign(v.start, v.start + n);
    r.size.assign(v.size, v.size + n);
    r.parent.assign(v.parent, v.parent + n);
    r.left.assign(v.left, v.left + n);
    r.right.assign(v.right, v.right + n);
    r.level.assign(v.level, v.level + n);
    r.rank.assign(v.rank, v.rank + n);
    r.basis_off.assign(v.basis_off, v.basis_off + n);
    r.far_ptr.assign(v.far_ptr, v.far_ptr + n + 1);
    r.near_ptr.assign(v.near_ptr, v.near_ptr + n + 1);
    r.far_col.assign(v.far_col, v.far_col + v.n_far);
    r.far_off.assign(v.far_off, v.far_off + v.n_far);
    r.near_col.assign(v.near_col, v.near_col + v.n_near);
    r.near_off.assign(v.near_off, v.near_off + v.n_near);
    // the large value arrays are borrowed, not copied (see build_matrix)
    r.basis_ext = v.basis; r.basis_len = v.basis_len;
    r.B_ext = v.B; r.B_len = v.B_len;
    r.D_ext = v.D; r.D_len = v.D_len;
    if (v.skel_ptr && v.skel && v.skel_len > 0) {  // optional
        r.skel_ptr.assign(v.skel_ptr, v.skel_ptr + n + 1);
        r.skel.assign(v.skel, v.skel + v.skel_len);
    }
    return validate(r);
}

// ---------------------------------------------------------------------------
// Validation: everything the kernels rely on for in-bounds access.

hm_status validate(const HostRepr &r) {
    const int64_t n = r.n_nodes, N = r.N;
    if ((int64_t)r.perm.size() != N) return fail(HM_ERR_FORMAT, "perm has the wrong length");
    {
        std::vector<char> seen((size_t)N, 0);
        for (int64_t t = 0; t < N; t++) {
            int64_t p = r.perm[t];
            if (p < 0 || p >= N || seen[(size_t)p]) return fail(HM_ERR_FORMAT, "perm is not a permutation");
            seen[(size_t)p] = 1;
        }
    }
    if (r.parent[0] != -1 || r.start[0] != 0 || r.size[0] != N || r.level[0] != 0)
        return fail(HM_ERR_FORMAT, "node 0 must be the root covering [0, N)");
    std::vector<int> child_of((size_t)n, 0);
    int32_t depth = 0;
    for (int64_t a = 0; a < n; a++) {
        if (r.size[a] < 1 || r.start[a] < 0 || r.start[a] > N || r.size[a] > N - r.start[a])
            return fail(HM_ERR_FORMAT, "node range out of bounds or empty");
        if (r.rank[a] < 0) return fail(HM_ERR_FORMAT, "negative rank");
        int32_t l = r.left[a], rr = r.right[a];
        if ((l < 0) != (rr < 0)) return fail(HM_ERR_FORMAT, "a node needs 0 or 2 children");
        if (l >= 0) {
            if (l >= n || rr >= n || l == 0 || rr == 0 || l == rr)
                return fail(HM_ERR_FORMAT, "child index out of range");
            child_of[(size_t)l]++;
            child_of[(size_t)rr]++;
            if (r.parent[l] != a || r.parent[rr] != a) return fail(HM_ERR_FORMAT, "parent link mismatch");
            if (r.level[l] != r.level[a] + 1 || r.level[rr] != r.level[a] + 1)
                return fail(HM_ERR_FORMAT, "child level is not parent level + 1");
            if (r.start[l] != r.start[a] || r.start[rr] != r.start[a] + r.size[l] ||
                r.size[l] + r.size[rr] != r.size[a])
                return fail(HM_ERR_FORMAT, "children do not partition the parent's range");
        }
        depth = std::max(depth, r.level[a]);
    }
    for (int64_t a = 1; a < n; a++)
        if (child_of[(size_t)a] != 1) return fail(HM_ERR_FORMAT, "node is not reachable from the root");
    if (depth != r.depth) return fail(HM_ERR_FORMAT, "depth does not match the node levels");
    // ranks and basis extents
    for (int64_t a = 0; a < n; a++) {
        int64_t nc = r.left[a] < 0 ? r.size[a] : (int64_t)r.rank[r.left[a]] + r.rank[r.right[a]];
        if (r.rank[a] > nc) return fail(HM_ERR_FORMAT, "rank exceeds the basis width");
        int64_t len = (int64_t)r.rank[a] * nc;
        if (len > 0 && (r.basis_off[a] < 0 || r.basis_off[a] > r.basis_len - len))
            return fail(HM_ERR_FORMAT, "basis offset out of range");
    }
    auto disjoint = [&](int64_t a, int64_t b) {
        return r.start[a] + r.size[a] <= r.start[b] || r.start[b] + r.size[b] <= r.start[a];
    };
    // CSR pointers: every one checked before any pair is read, so that a
    // damaged pointer cannot send the walk past the column array
    auto csr_ok = [&](const std::vector<int64_t> &ptr, size_t cols) {
        if ((int64_t)ptr.size() != n + 1 || ptr[0] != 0 || ptr[(size_t)n] != (int64_t)cols) return false;
        for (int64_t a = 0; a < n; a++)
            if (ptr[(size_t)a + 1] < ptr[(size_t)a]) return false;
        return true;
    };
    if (!csr_ok(r.far_ptr, r.far_col.size()) || r.far_off.size() != r.far_col.size())
        return fail(HM_ERR_FORMAT, "far CSR pointers are inconsistent");
    for (int64_t a = 0; a < n; a++) {
        for (int64_t e = r.far_ptr[a]; e < r.far_ptr[a + 1]; e++) {
            int64_t b = r.far_col[e];
            if (b < 0 || b >= n || !disjoint(a, b)) return fail(HM_ERR_FORMAT, "invalid far pair");
            int64_t len = (int64_t)r.rank[a] * r.rank[b];
            if (len > 0 && (r.far_off[e] < 0 || r.far_off[e] > r.B_len - len))
                return fail(HM_ERR_FORMAT, "B offset out of range");
        }
    }
    if (!csr_ok(r.near_ptr, r.near_col.size()) || r.near_off.size() != r.near_col.size())
        return fail(HM_ERR_FORMAT, "near CSR pointers are inconsistent");
    for (int64_t a = 0; a < n; a++) {
        for (int64_t e = r.near_ptr[a]; e < r.near_ptr[a + 1]; e++) {
            int64_t b = r.near_col[e];
            if (b < 0 || b >= n || r.left[a] >= 0 || r.left[b] >= 0)
                return fail(HM_ERR_FORMAT, "near pairs must join two leaves");
            if (a != b && !disjoint(a, b)) return fail(HM_ERR_FORMAT, "invalid near pair");
            if (r.size[b] > r.D_len / r.size[a]) return fail(HM_ERR_FORMAT, "D offset out of range");
            int64_t len = r.size[a] * r.size[b];
            if (r.near_off[e] < 0 || r.near_off[e] > r.D_len - len)
                return fail(HM_ERR_FORMAT, "D offset out of range");
        }
    }
    if (!r.skel_ptr.empty()) {  // optional skeletons: k_a original point indices per node
        if (!csr_ok(r.skel_ptr, r.skel.size())) return fail(HM_ERR_FORMAT, "skeleton pointers are inconsistent");
        for (int64_t a = 0; a < n; a++)
            if (r.skel_ptr[a + 1] - r.skel_ptr[a] != r.rank[a])
                return fail(HM_ERR_FORMAT, "a node's skeleton size differs from its rank");
        for (int64_t p : r.skel)
            if (p < 0 || p >= N) return fail(HM_ERR_FORMAT, "skeleton index out of range");
    }
    return HM_OK;
}

}  // namespace hm
