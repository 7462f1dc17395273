// Host-only logic of the library (no HIP): the schedule of targeted Jacobi
// rounds, the partition check of the D step, the autotuner's table parser.
// Built into the library and, with sanitizers, into a stand-alone CPU test.
#ifndef LRR_HOST_HPP
#define LRR_HOST_HPP

#include <string>
#include <vector>

#include "../../include/lrr.h"

namespace lrr {
namespace host {

// one line of the schedule table (lrr_tune_load)
struct TuneEntry {
    int m, n, t, maxl, precision;     // the problem shape the entry is for
    int eig_block, use_graph, check_every, coords;
};

// Targeted Jacobi rounds for nb index blocks (nb even): need (nb x nb, entry
// p * nb + q for p <= q) marks the pairs still holding a coupling (p == q:
// inside block p); out receives nb / 2 slots per round, each p | q << 16 with
// p < q.  Returns the number of rounds, or -1 if more than cap are needed (out
// then holds cap rounds: the caller sizes it for cap * nb / 2 ints).
int plan_rounds(const int* need, int nb, int cap, int* out);

// perm must be a permutation of 0..n-1 and offsets (t + 1 entries) strictly
// increasing from 0 to n; otherwise LRR_EINVAL with the reason in why
lrr_status check_partition(int n, int t, const int* perm, const int* offsets, std::string& why);

// parse a schedule table; false with a message naming the line on a malformed
// entry or an unreadable file (out then holds the entries before that line)
bool parse_tune(const char* path, std::vector<TuneEntry>& out, std::string& why);

}  // namespace host
}  // namespace lrr

#endif  // LRR_HOST_HPP
