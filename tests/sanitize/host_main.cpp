// Drives the library's host-only code (the inspector: tree, interaction
// lists, sampling and ID of Section 3.1; inspector-p1 of Section 5; the
// representation reader and its validation) on small seeded point sets, for a
// build with AddressSanitizer and UndefinedBehaviorSanitizer.  Every file the
// reader is given here is either one the inspector wrote or a truncated or
// byte-damaged copy of one: a damaged file must be refused or accepted only
// after validation, and never read out of bounds.
// Test infrastructure: built and run by tests/test_sanitizers.py only.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "hm_internal.h"

namespace hm {
// the library's thread-local error text lives in its device-facing part
hm_status fail(hm_status s, const std::string &msg) {
    (void)msg;
    return s;
}
}  // namespace hm

static int fails = 0;
#define CHECK(c, ...)                     \
    do {                                  \
        if (!(c)) {                       \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fputc('\n', stderr);     \
            fails++;                      \
        }                                 \
    } while (0)

static uint64_t st = 0x243f6a8885a308d3ull;
static uint64_t next() {  // xorshift64*
    st ^= st >> 12;
    st ^= st << 25;
    st ^= st >> 27;
    return st * 0x2545f4914f6cdd1dull;
}
static double urand() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }

static std::vector<unsigned char> slurp(const std::string &p) {
    std::vector<unsigned char> b;
    FILE *f = std::fopen(p.c_str(), "rb");
    if (!f) return b;
    int c;
    while ((c = std::fgetc(f)) != EOF) b.push_back((unsigned char)c);
    std::fclose(f);
    return b;
}
static void spit(const std::string &p, const unsigned char *b, size_t n) {
    FILE *f = std::fopen(p.c_str(), "wb");
    if (n) std::fwrite(b, 1, n, f);
    std::fclose(f);
}

static void one(const char *name, int64_t N, int64_t d, hm_compress_opts o, const std::string &dir) {
    std::vector<double> X((size_t)(N * d));
    for (int64_t i = 0; i < N * d; i++) X[(size_t)i] = urand() * (i % d == 0 ? 4.0 : 1.0);
    hm_repr r = nullptr;
    CHECK(hm_compress(X.data(), N, d, &o, &r) == HM_OK && r, "%s: compress failed", name);
    if (!r) return;
    hm_host_repr v{};
    CHECK(hm_repr_view(r, &v) == HM_OK, "%s: view failed", name);
    CHECK(v.N == N && v.d == d && v.n_nodes >= 1, "%s: view sizes", name);
    const std::string path = dir + "/" + name + ".hmc";
    CHECK(hm_repr_write(r, path.c_str()) == HM_OK, "%s: write failed", name);
    hm::HostRepr back;
    CHECK(hm::read_file(path.c_str(), back) == HM_OK, "%s: reading its own file failed", name);
    CHECK(back.N == v.N && back.n_nodes == v.n_nodes && (int64_t)back.far_col.size() == v.n_far &&
              (int64_t)back.near_col.size() == v.n_near && back.B_len == v.B_len && back.D_len == v.D_len,
          "%s: file content differs from the view", name);
    hm::HostRepr fromv;
    CHECK(hm::from_view(v, fromv) == HM_OK, "%s: from_view failed", name);
    // damaged copies: truncations, then single-byte changes
    const std::vector<unsigned char> good = slurp(path);
    const std::string bad = dir + "/" + name + "_bad.hmc";
    const size_t cuts[] = {0, 3, 64, 127, 128, 129, good.size() / 2, good.size() - 8, good.size() - 1};
    for (size_t c : cuts) {
        spit(bad, good.data(), c);
        hm::HostRepr t;
        CHECK(hm::read_file(bad.c_str(), t) != HM_OK, "%s: truncation at %zu accepted", name, c);
    }
    std::vector<unsigned char> dmg = good;
    dmg.push_back(0);
    spit(bad, dmg.data(), dmg.size());
    {
        hm::HostRepr t;
        CHECK(hm::read_file(bad.c_str(), t) != HM_OK, "%s: trailing byte accepted", name);
    }
    for (int k = 0; k < 400; k++) {
        dmg = good;
        // half the damage in the header and the small tables, where sizes and links live
        const size_t pos = k % 2 ? (size_t)(next() % std::min<size_t>(good.size(), 4096))
                                 : (size_t)(next() % good.size());
        dmg[pos] ^= (unsigned char)(1 + next() % 255);
        spit(bad, dmg.data(), dmg.size());
        hm::HostRepr t;
        (void)hm::read_file(bad.c_str(), t);  // any status; the sanitizers judge the access
    }
    std::remove(bad.c_str());
    hm_structure s = nullptr;
    CHECK(hm_inspect_p1(X.data(), N, d, &o, &s) == HM_OK && s, "%s: inspect_p1 failed", name);
    if (s) {
        hm_structure_info_t si{};
        CHECK(hm_structure_info(s, &si) == HM_OK && si.n_nodes == v.n_nodes, "%s: structure info", name);
        std::vector<int64_t> rows;
        for (int32_t a = 0; a < si.n_nodes; a++) {
            int64_t cnt = -1;
            CHECK(hm_structure_rows(s, a, nullptr, 0, &cnt) == HM_OK && cnt >= 0, "%s: rows of %d", name, a);
            rows.resize((size_t)std::max<int64_t>(cnt, 1));
            CHECK(hm_structure_rows(s, a, rows.data(), cnt, &cnt) == HM_OK, "%s: rows of %d", name, a);
        }
        int64_t cnt = 0;
        CHECK(hm_structure_rows(s, si.n_nodes, nullptr, 0, &cnt) != HM_OK, "%s: missing node accepted", name);
        hm_structure_free(s);
    }
    hm_repr_free(r);
}

int main(int argc, char **argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    hm_compress_opts o{};
    o.kernel = 0;
    o.h = 0.8;
    o.leaf_size = 32;
    o.tol = 1e-7;
    o.max_rank = 40;
    o.admissibility = 0;
    o.tau = 2.0;
    o.sample_rows = 64;
    o.seed = 11;
    o.threads = 2;
    one("h2_gauss", 900, 3, o, dir);
    o.kernel = 1;
    o.h = 1.5;
    o.admissibility = 1;
    o.leaf_size = 24;
    one("hss_lap", 700, 2, o, dir);
    o.kernel = 0;
    o.h = 1.0;
    o.admissibility = 2;
    o.budget = 0.03;
    o.partitioner = 1;
    o.tol = 1e-5;
    o.max_rank = 64;
    one("h2b_twomeans", 800, 8, o, dir);
    o.admissibility = 0;
    o.partitioner = 0;
    o.tol = 0.0;
    o.max_rank = 4;
    o.leaf_size = 16;
    one("rank_cap", 600, 3, o, dir);
    o.leaf_size = 32;
    o.max_rank = 16;
    one("one_leaf", 20, 3, o, dir);
    // invalid input is refused before it is read
    double bad[6] = {0, 1, NAN, 3, 4, 5};
    hm_repr r = nullptr;
    CHECK(hm_compress(bad, 2, 3, &o, &r) != HM_OK && !r, "NaN accepted");
    CHECK(hm_compress(bad, 0, 3, &o, &r) != HM_OK && !r, "N = 0 accepted");
    o.leaf_size = 1;
    CHECK(hm_compress(bad, 1, 3, &o, &r) != HM_OK && !r, "leaf size 1 accepted");
    {
        hm::HostRepr t;
        CHECK(hm::read_file((dir + "/missing.hmc").c_str(), t) != HM_OK, "a missing file accepted");
    }
    if (fails) return 1;
    std::puts("host sanitizer run ok");
    return 0;
}
