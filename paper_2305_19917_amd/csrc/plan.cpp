// Schedules of the models of computation of the paper (Sec. V).
//
// All three produce the same mathematical result, the forward substitution
// of Sec. IV; they differ only in how the unknowns are grouped and in which
// order the products of already-solved blocks are subtracted.
#include "plan.h"

#include <algorithm>
#include <map>

namespace redsea {

namespace {

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Sec. V-A: a solve of order m is refined into the solve of the top half,
// the product update of the bottom half with the solved top half, and the
// solve of the bottom half (the three stages of Sec. IV), applied again to
// each half until the order is at most nb.  The split is placed on a leaf
// boundary (the first half receives the larger share of leaves) so every
// leaf below is a full nb block except possibly the last one.
void recurse(int64_t r0, int64_t m, int64_t nb, std::vector<Task>& out, int64_t& round) {
    if (m <= 0) return;
    if (m <= nb) {
        out.push_back({TASK_LEAF, r0, m, r0, m, round++});
        return;
    }
    int64_t nblk = ceil_div(m, nb);
    int64_t m1 = ceil_div(nblk, 2) * nb;
    recurse(r0, m1, nb, out, round);
    out.push_back({TASK_GEMM, r0 + m1, m - m1, r0, m1, round++});
    recurse(r0 + m1, m - m1, nb, out, round);
}

}  // namespace

std::vector<std::vector<std::pair<int64_t, int64_t>>> blocked_rounds(int64_t r) {
    // Sec. V-C prescribes r-1 rounds with r/2 blocks each, (r-1) r / 2 blocks
    // in total, but not which block goes to which round.  Reading used here:
    // earliest deadline first.  Block (p, q) becomes available once leaf q
    // is solved and must finish before leaf p; each round takes up to
    // ceil(r/2) available blocks in (p, q) order.  Should a deadline still be
    // open at the end of its round the remaining blocks of that row are added
    // to the round (never the case for the sizes the tests cover).
    std::vector<std::vector<std::pair<int64_t, int64_t>>> rounds;
    if (r < 2) return rounds;
    const int64_t cap = ceil_div(r, 2);
    // next_q[p] = first q of row p not yet scheduled (rows are taken in q order)
    std::vector<int64_t> next_q(r, 0);
    for (int64_t t = 1; t < r; ++t) {
        std::vector<std::pair<int64_t, int64_t>> cur;
        // available blocks: q <= t-1, q < p, not yet taken; visit by (p, q)
        for (int64_t p = 1; p < r && (int64_t)cur.size() < cap; ++p) {
            while (next_q[p] < p && next_q[p] <= t - 1 && (int64_t)cur.size() < cap) {
                cur.push_back({p, next_q[p]});
                ++next_q[p];
            }
        }
        // deadline of leaf t: every block (t, q), q < t, must be done now
        while (next_q[t] < t) {
            cur.push_back({t, next_q[t]});
            ++next_q[t];
        }
        rounds.push_back(cur);
    }
    return rounds;
}

std::vector<Task> build_schedule(int variant, int64_t m, int64_t nb) {
    std::vector<Task> out;
    if (m <= 0 || nb <= 0) return out;
    int64_t round = 0;
    const int64_t r = ceil_div(m, nb);
    auto leaf = [&](int64_t p) {
        int64_t r0 = p * nb, rows = std::min(nb, m - r0);
        out.push_back({TASK_LEAF, r0, rows, r0, rows, round++});
    };
    switch (variant) {
        case VAR_ITERATIVE:
            // Sec. V-B: r leaves of order nb; after leaf p one product updates
            // every row below it (r - 1 product panels in total).
            for (int64_t p = 0; p < r; ++p) {
                leaf(p);
                int64_t below = (p + 1) * nb;
                if (below < m) out.push_back({TASK_GEMM, below, m - below, p * nb, nb, round++});
            }
            break;
        case VAR_BLOCKED: {
            // Sec. V-C: r leaves and (r-1) r / 2 product blocks of order nb,
            // issued in r-1 rounds.  Blocks of one row in one round are
            // merged into a single product over their joint column range,
            // so one launch never has two writers of the same rows.
            auto rounds = blocked_rounds(r);
            leaf(0);
            for (int64_t t = 1; t < r; ++t) {
                std::map<int64_t, std::vector<int64_t>> rows;
                for (auto& pq : rounds[t - 1]) rows[pq.first].push_back(pq.second);
                // A row whose q values are not contiguous would need two
                // products on the same rows; split such runs over sub-rounds.
                std::vector<std::vector<Task>> sub;
                for (auto& kv : rows) {
                    auto qs = kv.second;
                    std::sort(qs.begin(), qs.end());
                    size_t run = 0;
                    for (size_t i = 0; i < qs.size();) {
                        size_t j = i;
                        while (j + 1 < qs.size() && qs[j + 1] == qs[j] + 1) ++j;
                        int64_t p = kv.first;
                        int64_t r0 = p * nb, rr = std::min(nb, m - r0);
                        int64_t c0 = qs[i] * nb, cc = (qs[j] - qs[i] + 1) * nb;
                        if (sub.size() <= run) sub.resize(run + 1);
                        sub[run].push_back({TASK_GEMM, r0, rr, c0, cc, 0});
                        ++run;
                        i = j + 1;
                    }
                }
                for (auto& s : sub) {
                    for (auto& tk : s) {
                        tk.round = round;
                        out.push_back(tk);
                    }
                    ++round;
                }
                leaf(t);
            }
            break;
        }
        case VAR_RECURSIVE:
        default:
            recurse(0, m, nb, out, round);
            break;
    }
    return out;
}

}  // namespace redsea
