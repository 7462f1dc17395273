// Host-only logic of the library; see host.hpp.
#include "host.hpp"

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstring>
#include <utility>

namespace lrr {
namespace host {

// Targeted Jacobi rounds.  need (nb x nb, p <= q at p * nb + q) marks the
// index-block pairs that still hold an entry needing a rotation (p == q: inside
// block p).  Greedy maximal matchings of the marked pairs, each completed to a
// perfect matching of the nb blocks (a block inside which something is marked
// goes with any free partner; the rest pair up in order), are written to out as
// p | q << 16 per slot, nb / 2 slots per round.  Returns the number of rounds,
// or -1 if more than cap would be needed.
int plan_rounds(const int* need, int nb, int cap, int* out) {
    std::vector<std::pair<int, int>> pend, keep;
    std::vector<char> inner(nb, 0), used(nb);
    for (int p = 0; p < nb; ++p)
        for (int q = p; q < nb; ++q)
            if (need[p * nb + q]) {
                if (p == q) inner[p] = 1;
                else pend.emplace_back(p, q);
            }
    int rounds = 0;
    for (;;) {
        bool left = !pend.empty();
        for (int p = 0; p < nb && !left; ++p) left = inner[p] != 0;
        if (!left) return rounds;
        if (rounds == cap) return -1;
        int* slot = out + (size_t)rounds * (nb / 2);
        int ns = 0;
        std::fill(used.begin(), used.end(), 0);
        auto put = [&](int p, int q) {
            slot[ns++] = std::min(p, q) | (std::max(p, q) << 16);
            used[p] = used[q] = 1;
            inner[p] = inner[q] = 0;   // a pair solve also sweeps inside both blocks
        };
        keep.clear();
        for (const auto& e : pend) {
            if (!used[e.first] && !used[e.second]) put(e.first, e.second);
            else keep.push_back(e);
        }
        pend.swap(keep);
        for (int p = 0; p < nb; ++p) {
            if (!inner[p] || used[p]) continue;
            int q = -1;
            for (int x = 0; x < nb; ++x)
                if (x != p && !used[x] && (q < 0 || (inner[x] && !inner[q]))) q = x;
            put(p, q);   // nb is even, so a free partner exists
        }
        int u = -1;
        for (int x = 0; x < nb; ++x) {
            if (used[x]) continue;
            if (u < 0) u = x;
            else { put(u, x); u = -1; }
        }
        ++rounds;
    }
}

// parse a schedule table; returns false with a message naming the line
bool parse_tune(const char* path, std::vector<TuneEntry>& out, std::string& why) {
    FILE* f = std::fopen(path, "r");
    if (!f) { why = std::string("cannot open ") + path; return false; }
    char line[512];
    int no = 0;
    bool ok = true;
    while (std::fgets(line, sizeof(line), f)) {
        ++no;
        if (char* c = std::strchr(line, '#')) *c = '\0';
        bool blank = true;
        for (const char* c = line; *c; ++c) if (!std::isspace((unsigned char)*c)) { blank = false; break; }
        if (blank) continue;
        TuneEntry e;
        char extra;
        const int k = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %c", &e.m, &e.n, &e.t, &e.maxl, &e.precision,
                                  &e.eig_block, &e.use_graph, &e.check_every, &e.coords, &extra);
        if (k != 9 || e.m < 1 || e.n < 1 || e.t < 1 || e.maxl < 1 || e.precision < 0 || e.precision > 2 ||
            (e.eig_block != 16 && e.eig_block != 32) || e.use_graph < 0 || e.use_graph > 3 ||
            e.check_every < 1 || e.coords < 0 || e.coords > 2) {
            why = std::string(path) + ": malformed entry on line " + std::to_string(no);
            ok = false;
            break;
        }
        out.push_back(e);
    }
    std::fclose(f);
    return ok;
}

lrr_status check_partition(int n, int t, const int* perm, const int* offsets, std::string& why) {
    if (n <= 0 || t <= 0 || t > n) { why = "need 0 < t <= n"; return LRR_EINVAL; }
    if (!perm || !offsets) { why = "perm and offsets must not be NULL"; return LRR_EINVAL; }
    if (offsets[0] != 0 || offsets[t] != n) { why = "offsets must start at 0 and end at n"; return LRR_EINVAL; }
    for (int i = 0; i < t; ++i)
        if (offsets[i + 1] <= offsets[i]) { why = "offsets must be strictly increasing"; return LRR_EINVAL; }
    std::vector<char> seen(n, 0);
    for (int j = 0; j < n; ++j) {
        const int v = perm[j];
        if (v < 0 || v >= n || seen[v]) { why = "perm is not a permutation of 0..n-1"; return LRR_EINVAL; }
        seen[v] = 1;
    }
    return LRR_OK;
}

}  // namespace host
}  // namespace lrr
