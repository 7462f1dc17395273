// Randomised checks of the library's host-only logic (host.cpp), built by
// tests/test_host_sanitizers.py with AddressSanitizer and UBSan.  Exits 0 when
// every check holds; prints the failing case and exits 1 otherwise.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "host.hpp"

using lrr::host::check_partition;
using lrr::host::parse_tune;
using lrr::host::plan_rounds;
using lrr::host::TuneEntry;

static int fails = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            std::fprintf(stderr, "FAIL %s: ", #c);      \
            std::fprintf(stderr, __VA_ARGS__);          \
            std::fprintf(stderr, "\n");                 \
            ++fails;                                    \
        }                                               \
    } while (0)

static void partitions(std::mt19937& g) {
    for (int trial = 0; trial < 2000; ++trial) {
        const int n = 1 + (int)(g() % 300), t = 1 + (int)(g() % n);
        std::vector<int> perm(n), off(t + 1);
        for (int i = 0; i < n; ++i) perm[i] = i;
        std::shuffle(perm.begin(), perm.end(), g);
        std::vector<int> cuts;
        for (int i = 1; i < n; ++i) cuts.push_back(i);
        std::shuffle(cuts.begin(), cuts.end(), g);
        cuts.resize(t - 1);
        std::sort(cuts.begin(), cuts.end());
        off[0] = 0;
        for (int i = 0; i < t - 1; ++i) off[i + 1] = cuts[i];
        off[t] = n;
        std::string why;
        CHECK(check_partition(n, t, perm.data(), off.data(), why) == LRR_OK, "n=%d t=%d valid rejected: %s", n, t,
              why.c_str());
        // one corruption at a time must be rejected
        std::vector<int> p2 = perm, o2 = off;
        switch (g() % 5) {
            case 0: if (n > 1) p2[g() % n] = p2[g() % n]; else p2[0] = 1; break;   // a repeat (or no change)
            case 1: p2[g() % n] = (g() & 1) ? -1 - (int)(g() % 5) : n + (int)(g() % 5); break;
            case 2: o2[t] = n + 1 + (int)(g() % 3); break;
            case 3: if (t > 1) o2[1 + g() % (t - 1)] = o2[0]; else o2[0] = 1; break;
            default: o2[0] = -1; break;
        }
        const bool same = p2 == perm && o2 == off;
        if (!same)
            CHECK(check_partition(n, t, p2.data(), o2.data(), why) == LRR_EINVAL, "n=%d t=%d corrupted accepted", n, t);
    }
    std::string why;
    int one = 0;
    CHECK(check_partition(0, 1, &one, &one, why) == LRR_EINVAL, "n=0");
    CHECK(check_partition(3, 4, &one, &one, why) == LRR_EINVAL, "t>n");
    CHECK(check_partition(3, 1, nullptr, &one, why) == LRR_EINVAL, "null perm");
}

static void rounds(std::mt19937& g) {
    for (int trial = 0; trial < 3000; ++trial) {
        const int nb = 2 * (1 + (int)(g() % 32));
        const double dens = (g() % 100) / 100.0 * ((g() & 1) ? 1.0 : 0.1);
        std::vector<int> need((size_t)nb * nb, 0);
        std::uniform_real_distribution<double> u(0.0, 1.0);
        for (int p = 0; p < nb; ++p)
            for (int q = p; q < nb; ++q) need[(size_t)p * nb + q] = u(g) < dens;
        const int cap = (g() & 1) ? nb * nb : (int)(g() % nb);
        std::vector<int> out((size_t)std::max(cap, 1) * (nb / 2) + 1, -7);
        const int sentinel = out.back();
        const int r = plan_rounds(need.data(), nb, cap, out.data());
        CHECK(out.back() == sentinel, "nb=%d cap=%d wrote past cap rounds", nb, cap);
        CHECK(r == -1 || (r >= 0 && r <= cap), "nb=%d cap=%d returned %d", nb, cap, r);
        if (r < 0) continue;
        std::vector<char> pair_done((size_t)nb * nb, 0), inner_done(nb, 0);
        for (int k = 0; k < r; ++k) {
            std::vector<int> seen(nb, 0);
            for (int s = 0; s < nb / 2; ++s) {
                const int v = out[(size_t)k * (nb / 2) + s], p = v & 0xffff, q = v >> 16;
                CHECK(p >= 0 && p < q && q < nb, "nb=%d round %d slot %d = (%d, %d)", nb, k, s, p, q);
                if (!(p >= 0 && p < q && q < nb)) continue;
                seen[p]++;
                seen[q]++;
                pair_done[(size_t)p * nb + q] = 1;
                inner_done[p] = inner_done[q] = 1;
            }
            for (int b = 0; b < nb; ++b) CHECK(seen[b] == 1, "nb=%d round %d block %d used %d times", nb, k, b, seen[b]);
        }
        for (int p = 0; p < nb; ++p) {
            if (need[(size_t)p * nb + p]) CHECK(inner_done[p], "nb=%d inner block %d never swept", nb, p);
            for (int q = p + 1; q < nb; ++q)
                if (need[(size_t)p * nb + q]) CHECK(pair_done[(size_t)p * nb + q], "nb=%d pair (%d,%d) missed", nb, p, q);
        }
    }
}

static std::string write_file(const std::string& text, int k) {
    const char* dir = std::getenv("TMPDIR");
    std::string path = std::string(dir ? dir : "/tmp") + "/lrr_tune_check_" + std::to_string(k) + ".txt";
    FILE* f = std::fopen(path.c_str(), "w");
    std::fputs(text.c_str(), f);
    std::fclose(f);
    return path;
}

static void tune_tables(std::mt19937& g) {
    std::vector<TuneEntry> e;
    std::string why;
    // a valid table with comments and blank lines
    std::string ok = "# m n t maxl precision eig_block use_graph check_every coords\n\n"
                     "500 2000 4 500 0 16 0 4 2   # workload 2\n   \n2016 2432 16 200 1 32 3 1 0\n";
    CHECK(parse_tune(write_file(ok, 0).c_str(), e, why) && e.size() == 2 && e[1].eig_block == 32 && e[1].use_graph == 3,
          "valid table: %s", why.c_str());
    const char* bad[] = {"500 2000 4 500 0 16 0 4\n",        "500 2000 4 500 0 16 0 4 2 9\n",
                         "500 2000 4 500 0 24 0 4 2\n",      "500 2000 4 500 3 16 0 4 2\n",
                         "500 2000 4 500 0 16 4 4 2\n",      "500 2000 4 500 0 16 0 0 2\n",
                         "0 2000 4 500 0 16 0 4 2\n",        "a b c\n"};
    for (int i = 0; i < 8; ++i) {
        e.clear();
        CHECK(!parse_tune(write_file(bad[i], 1 + i).c_str(), e, why) && why.find("line 1") != std::string::npos,
              "malformed line %d accepted", i);
    }
    e.clear();
    CHECK(!parse_tune("/nonexistent/lrr_tune.txt", e, why), "missing file accepted");
    // random bytes and over-long lines never crash the parser
    for (int k = 0; k < 200; ++k) {
        std::string s;
        const int len = (int)(g() % 2000);
        for (int i = 0; i < len; ++i) {
            const int c = (int)(g() % 100);
            s.push_back(c < 10 ? '\n' : c < 25 ? ' ' : c < 70 ? (char)('0' + g() % 10) : (char)(32 + g() % 95));
        }
        e.clear();
        (void)parse_tune(write_file(s, 100).c_str(), e, why);
        for (const TuneEntry& t : e)
            CHECK((t.eig_block == 16 || t.eig_block == 32) && t.check_every >= 1, "accepted an invalid entry");
    }
}

int main() {
    std::mt19937 g(12345);
    partitions(g);
    rounds(g);
    tune_tables(g);
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
