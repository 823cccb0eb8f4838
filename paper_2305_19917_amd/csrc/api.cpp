// C interface of libredsea: argument checks, canonicalisation of the BLAS
// flags onto one forward-substitution family, schedule construction and
// execution on a HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/redsea.h"
#include "exec.h"
#include "kernels.h"
#include "mixed.h"
#include "ozaki.h"
#include "picker.h"
#include "plan.h"

namespace redsea {

// ------------------------------------------------------------------ workspace
// One buffer per (device, stream, slot).  Solves on different streams never
// share memory, and a buffer grows in stream order: the old one is released
// with hipFreeAsync and the new one taken with hipMallocAsync on the same
// stream, so work already queued there finishes with the old buffer first.
// A lease holds the entry's lock while its holder enqueues the work that
// uses the buffer, so a second host thread on the same stream cannot release
// it in between.  On a stream that is being captured into a graph a cached
// pointer would outlive its buffer (a later growth frees it), so the lease is
// refused there: graph capture goes through the entry point with static
// scratch memory, or the batched plan, which owns its memory.
namespace {

struct WsEntry {
    std::mutex mu;
    void* ptr = nullptr;
    size_t bytes = 0;
};

std::mutex g_ws_mu;
std::map<std::tuple<int, uintptr_t, int>, std::unique_ptr<WsEntry>> g_ws;

}  // namespace

int workspace(int slot, size_t bytes, hipStream_t s, WsLease& out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return REDSEA_ERR_HIP;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return REDSEA_ERR_HIP;
    if (cap != hipStreamCaptureStatusNone) return REDSEA_ERR_UNSUPPORTED;
    WsEntry* e = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_ws_mu);
        auto& slotp = g_ws[std::make_tuple(dev, (uintptr_t)s, slot)];
        if (!slotp) slotp.reset(new WsEntry);
        e = slotp.get();
    }
    std::unique_lock<std::mutex> lock(e->mu);
    if (e->bytes < bytes) {
        if (e->ptr) {
            if (hipFreeAsync(e->ptr, s) != hipSuccess) return REDSEA_ERR_HIP;
            e->ptr = nullptr;
            e->bytes = 0;
        }
        const size_t want = bytes + bytes / 4;
        if (hipMallocAsync(&e->ptr, want, s) != hipSuccess) {
            (void)hipGetLastError();
            e->ptr = nullptr;
            return REDSEA_ERR_ALLOC;
        }
        e->bytes = want;
    }
    out.lock = std::move(lock);
    out.ptr = e->ptr;
    return REDSEA_OK;
}

// ------------------------------------------------------------------ canonical form

Canon canonicalize(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                   const void* A, int64_t lda, void* B, int64_t ldb) {
    Canon c;
    c.dtype = dtype;
    c.unit = diag == REDSEA_UNIT;
    // Right side: X op(A) = alpha B  <=>  op(A)^T X^T = alpha B^T, a left
    // solve with the transpose flag flipped on the transposed right-hand side.
    const bool right = side == REDSEA_RIGHT;
    c.op_trans = right ? (trans == REDSEA_NOTRANS) : (trans != REDSEA_NOTRANS);
    c.rhs_trans = right;
    c.k = right ? n : m;
    c.nrhs = right ? m : n;
    // M = op_eff(A) is lower iff (A lower) xor transposed.
    const bool m_lower = (uplo == REDSEA_LOWER) != c.op_trans;
    c.reverse = !m_lower;
    c.A = A;
    c.lda = lda;
    c.B = B;
    c.ldb = ldb;
    const int64_t k = c.k;
    // Canonical T(i, j) = M(i, j), or M(k-1-i, k-1-j) when reversed.
    c.tri.base = A;
    if (!c.reverse) {
        c.tri.off = 0;
        c.tri.tr = c.op_trans ? lda : 1;
        c.tri.tc = c.op_trans ? 1 : lda;
    } else {
        c.tri.off = (k - 1) * (1 + lda);
        c.tri.tr = c.op_trans ? -lda : -1;
        c.tri.tc = c.op_trans ? -1 : -lda;
    }
    // Canonical right-hand sides: column j of the left problem.
    c.rhs.base = B;
    const int64_t s_row = right ? ldb : 1, s_col = right ? 1 : ldb;
    if (!c.reverse) {
        c.rhs.off = 0;
        c.rhs.br = s_row;
    } else {
        c.rhs.off = (k - 1) * s_row;
        c.rhs.br = -s_row;
    }
    c.rhs.bc = s_col;
    return c;
}

// Product task in storage coordinates: canonical rows [r0, r0+R) of C and
// canonical columns [c0, c0+K) of T become storage rows of M = op_eff(A).
GemmArgs gemm_args(const Canon& c, int64_t r0, int64_t R, int64_t c0, int64_t K) {
    const int64_t k = c.k;
    int64_t R0 = r0, K0 = c0;
    if (c.reverse) {
        R0 = k - r0 - R;
        K0 = k - c0 - K;
    }
    const size_t es = c.dtype == REDSEA_F64 ? 8 : 4;
    GemmArgs g;
    g.M = R;
    g.N = c.nrhs;
    g.K = K;
    const char* a = (const char*)c.A;
    // M(i, j) = A[i + j*lda] (not transposed) or A[j + i*lda] (transposed);
    // the BF16 copy holds M by rows
    if (c.gemm_bf16) {
        g.a = (const char*)c.A16 + 2 * (K0 + R0 * c.lda16);
        g.lda = c.lda16;
    } else {
        g.a = c.op_trans ? a + es * (K0 + R0 * c.lda) : a + es * (R0 + K0 * c.lda);
        g.lda = c.lda;
    }
    char* b = (char*)c.B;
    if (!c.rhs_trans) {
        g.x = b + es * K0;
        g.c = b + es * R0;
    } else {
        g.x = b + es * (K0 * c.ldb);
        g.c = b + es * (R0 * c.ldb);
    }
    g.ldx = c.ldb;
    g.ldc = c.ldb;
    return g;
}

// ------------------------------------------------------------------ plans

namespace {

std::mutex g_plan_mu;
std::map<std::tuple<int, int64_t, int64_t>, std::vector<Task>> g_plans;

// Leaves larger than the leaf kernel's register block are themselves solved
// by the recursive split (Sec. V-A) down to that block.
std::vector<Task> expand_leaves(const std::vector<Task>& in, int64_t kleaf) {
    std::vector<Task> out;
    int64_t round = 0, last = -1;
    for (const Task& t : in) {
        if (t.round != last) {
            last = t.round;
            ++round;
        }
        if (t.kind == TASK_LEAF && t.rows > kleaf) {
            std::vector<Task> sub = build_schedule(VAR_RECURSIVE, t.rows, kleaf);
            for (Task s : sub) {
                s.row0 += t.row0;
                s.col0 += t.row0;
                s.round = round++;
                out.push_back(s);
            }
        } else {
            Task s = t;
            s.round = round;
            out.push_back(s);
        }
    }
    return out;
}

}  // namespace

const std::vector<Task>& plan_for(int variant, int64_t k, int64_t nb, int64_t kleaf) {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    auto key = std::make_tuple(variant, k, nb * 1024 + kleaf);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return it->second;
    std::vector<Task> t = expand_leaves(build_schedule(variant, k, nb), kleaf);
    return g_plans.emplace(key, std::move(t)).first->second;
}

// ------------------------------------------------------------------ tracing
// When enabled, every kernel launch of the executor is bracketed by a pair of
// HIP events on its stream; redsea_trace_end() waits for them and returns the
// summed durations and algorithmic flops per kernel class.

namespace {

struct TraceRec {
    int kind;
    double flops;
    hipEvent_t e0, e1;
};

std::mutex g_tr_mu;
bool g_tr_on = false;
std::vector<TraceRec> g_tr;

}  // namespace

bool trace_on() { return g_tr_on; }

void trace_push(int kind, double flops, hipEvent_t e0, hipEvent_t e1) {
    std::lock_guard<std::mutex> lock(g_tr_mu);
    g_tr.push_back({kind, flops, e0, e1});
}

// ------------------------------------------------------------------ execution

namespace {

std::mutex g_st_mu;
std::map<int, std::vector<hipStream_t>> g_side;  // device -> helper streams

// Helper streams of the current device (default priority, non-blocking),
// created on first use and kept until the process ends.
int side_streams(int count, hipStream_t* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return REDSEA_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_st_mu);
    std::vector<hipStream_t>& v = g_side[dev];
    while ((int)v.size() < count) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return REDSEA_ERR_HIP;
        v.push_back(st);
    }
    for (int i = 0; i < count; ++i) out[i] = v[i];
    return REDSEA_OK;
}

// The same solve restricted to right-hand sides [c0, c0 + w).
Canon column_slice(const Canon& c, int64_t c0, int64_t w) {
    Canon sub = c;
    const size_t es = c.dtype == REDSEA_F64 ? 8 : 4;
    sub.nrhs = w;
    sub.rhs.off += c0 * c.rhs.bc;
    sub.B = (char*)c.B + es * (c.rhs_trans ? c0 : c0 * c.ldb);
    return sub;
}

// Helper stream and events of the look-ahead split, one set per (device,
// caller's stream) so that solves on different streams never wait on each
// other's events; created on first use and kept until the process ends.  An
// event is recorded again only after the waits on its previous record have
// been enqueued, and the caller holds the stream's workspace lease while it
// enqueues, so one set is never used by two solves at once.
constexpr int64_t kLookaheadMaxRhs = 2048;

struct Lookahead {
    hipStream_t helper = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};
std::mutex g_la_mu;
std::map<std::pair<int, uintptr_t>, Lookahead> g_la;

int lookahead_for(hipStream_t s, Lookahead* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return REDSEA_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_la_mu);
    Lookahead& la = g_la[{dev, (uintptr_t)s}];
    if (!la.helper) {
        Lookahead n;
        if (hipStreamCreateWithFlags(&n.helper, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&n.ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&n.ev[1], hipEventDisableTiming) != hipSuccess)
            return REDSEA_ERR_HIP;
        la = n;
    }
    *out = la;
    return REDSEA_OK;
}

// Look-ahead (the overlap of leaf solves with independent products, paper
// Sec. V-C): when a single product is followed by the leaf that solves its
// first rows, only those rows are updated on the stream s; the rest of the
// product runs on the helper stream `side`, concurrently with that leaf, and
// the next product (which writes the same rows as the rest) waits for it.
// A blocked round (several block products) followed by a leaf is split the
// same way: the blocks that write the leaf's rows run on s, the others on
// `side` while the leaf runs (they read only blocks solved before and write
// other rows).  Both parts keep the round's tile configuration, and every
// product tile runs the same MFMA sequence in the same k order, so the split
// changes no result bit.  Any later leaf or round waits for the helper first.
int run_tasks(const Canon& c, const std::vector<Task>& tasks, int64_t kleaf, const void* packed,
              hipStream_t s, const Lookahead* la = nullptr) {
    const size_t es = c.dtype == REDSEA_F64 ? 8 : 4;
    hipStream_t side = la ? la->helper : nullptr;
    const hipEvent_t ev[2] = {la ? la->ev[0] : nullptr, la ? la->ev[1] : nullptr};
    bool pending = false;  // a product tail is in flight on `side`
    int64_t overlap_row = -1;  // row0 of the one leaf that may run beside it
    auto join = [&]() -> bool {
        if (!pending) return true;
        pending = false;
        return hipStreamWaitEvent(s, ev[1], 0) == hipSuccess;
    };
    // block products as grouped launches of at most kMaxGroup, one tile
    // configuration for all of them
    auto launch_blocks = [&](const std::vector<GemmArgs>& blocks, int tile,
                             hipStream_t st) -> bool {
        GemmGroup grp;
        grp.count = 0;
        for (size_t q = 0; q < blocks.size(); ++q) {
            grp.g[grp.count++] = blocks[q];
            if (grp.count == kMaxGroup || q + 1 == blocks.size()) {
                double fl = 0.0;
                for (int u = 0; u < grp.count; ++u) fl += 2.0 * grp.g[u].M * grp.g[u].N * grp.g[u].K;
                if (traced(REDSEA_KERNEL_GEMM_GROUP, fl, st, [&] {
                        return launch_gemm_group(c.dtype, c.op_trans, c.rhs_trans, grp, st, tile);
                    }) != hipSuccess)
                    return false;
                grp.count = 0;
            }
        }
        return true;
    };
    size_t i = 0;
    while (i < tasks.size()) {
        const Task& t = tasks[i];
        if (t.kind == TASK_LEAF) {
            if (pending && t.row0 != overlap_row && !join()) return REDSEA_ERR_HIP;
            overlap_row = -1;
            const char* pb =
                (const char*)packed + (size_t)(t.row0 / kleaf) * leaf_block_elems((int)kleaf) * es;
            const double fl = (double)t.rows * t.rows * c.nrhs;
            if (traced(REDSEA_KERNEL_LEAF, fl, s, [&] {
                    return launch_leaf(c.dtype, (int)kleaf, pb, t.rows, c.rhs, t.row0, c.nrhs,
                                       c.unit, s);
                }) != hipSuccess)
                return REDSEA_ERR_HIP;
            ++i;
            continue;
        }
        // gather the products of this round
        size_t j = i;
        while (j < tasks.size() && tasks[j].kind == TASK_GEMM && tasks[j].round == t.round) ++j;
        if (!join()) return REDSEA_ERR_HIP;
        if (side && !c.gemm_bf16 && j - i == 1 && j < tasks.size() &&
            tasks[j].kind == TASK_LEAF && tasks[j].row0 == t.row0 && t.rows > tasks[j].rows) {
            const int64_t head = tasks[j].rows;
            GemmArgs gt = gemm_args(c, t.row0 + head, t.rows - head, t.col0, t.cols);
            GemmArgs gh = gemm_args(c, t.row0, head, t.col0, t.cols);
            if (hipEventRecord(ev[0], s) != hipSuccess || hipStreamWaitEvent(side, ev[0], 0) != hipSuccess)
                return REDSEA_ERR_HIP;
            if (traced(REDSEA_KERNEL_GEMM, 2.0 * gt.M * gt.N * gt.K, side, [&] {
                    return launch_gemm(c.dtype, c.op_trans, c.rhs_trans, gt, side);
                }) != hipSuccess ||
                hipEventRecord(ev[1], side) != hipSuccess)
                return REDSEA_ERR_HIP;
            pending = true;
            overlap_row = tasks[j].row0;
            if (traced(REDSEA_KERNEL_GEMM, 2.0 * gh.M * gh.N * gh.K, s, [&] {
                    return launch_gemm(c.dtype, c.op_trans, c.rhs_trans, gh, s);
                }) != hipSuccess)
                return REDSEA_ERR_HIP;
            i = j;
            continue;
        }
        if (side && !c.gemm_bf16 && j - i > 1 && j < tasks.size() && tasks[j].kind == TASK_LEAF) {
            const Task& lf = tasks[j];
            std::vector<GemmArgs> head, tail;
            for (size_t q = i; q < j; ++q) {
                const Task& b = tasks[q];
                const bool hits = b.row0 < lf.row0 + lf.rows && lf.row0 < b.row0 + b.rows;
                (hits ? head : tail).push_back(gemm_args(c, b.row0, b.rows, b.col0, b.cols));
            }
            if (!tail.empty()) {
                const GemmArgs f = gemm_args(c, t.row0, t.rows, t.col0, t.cols);
                const int tile = gemm_default_tile(c.dtype, f.M, f.N, f.K);
                if (hipEventRecord(ev[0], s) != hipSuccess ||
                    hipStreamWaitEvent(side, ev[0], 0) != hipSuccess || !launch_blocks(tail, tile, side) ||
                    hipEventRecord(ev[1], side) != hipSuccess)
                    return REDSEA_ERR_HIP;
                pending = true;
                overlap_row = lf.row0;
                if (!head.empty() && !launch_blocks(head, tile, s)) return REDSEA_ERR_HIP;
                i = j;
                continue;
            }
        }
        if (c.gemm_bf16) {
            for (size_t q = i; q < j; ++q) {
                GemmArgs g = gemm_args(c, tasks[q].row0, tasks[q].rows, tasks[q].col0,
                                       tasks[q].cols);
                const double fl = 2.0 * g.M * g.N * g.K;
                if (traced(REDSEA_KERNEL_GEMM, fl, s, [&] {
                        return launch_gemm_bf16(true, c.rhs_trans, g, s);
                    }) != hipSuccess)
                    return REDSEA_ERR_HIP;
            }
        } else if (j - i == 1) {
            GemmArgs g = gemm_args(c, t.row0, t.rows, t.col0, t.cols);
            const double fl = 2.0 * g.M * g.N * g.K;
            if (traced(REDSEA_KERNEL_GEMM, fl, s,
                       [&] { return launch_gemm(c.dtype, c.op_trans, c.rhs_trans, g, s); }) !=
                hipSuccess)
                return REDSEA_ERR_HIP;
        } else {
            GemmGroup grp;
            grp.count = 0;
            for (size_t q = i; q < j; ++q) {
                grp.g[grp.count++] = gemm_args(c, tasks[q].row0, tasks[q].rows, tasks[q].col0,
                                               tasks[q].cols);
                if (grp.count == kMaxGroup || q + 1 == j) {
                    double fl = 0.0;
                    for (int u = 0; u < grp.count; ++u)
                        fl += 2.0 * grp.g[u].M * grp.g[u].N * grp.g[u].K;
                    if (traced(REDSEA_KERNEL_GEMM_GROUP, fl, s, [&] {
                            return launch_gemm_group(c.dtype, c.op_trans, c.rhs_trans, grp, s);
                        }) != hipSuccess)
                        return REDSEA_ERR_HIP;
                    grp.count = 0;
                }
            }
        }
        i = j;
    }
    return join() ? REDSEA_OK : REDSEA_ERR_HIP;
}

}  // namespace

// Number of right-hand-side column groups solved concurrently on helper
// streams: the leaf chain of one group then overlaps the products of the
// others (the columns are independent systems).
int column_groups(const Canon& c) {
    const char* e = std::getenv("REDSEA_STREAMS");
    int g = e ? std::atoi(e) : 1;
    if (g < 1) g = 1;
    if (g > 4) g = 4;
    while (g > 1 && c.nrhs / g < 256) --g;
    return g;
}

// Rows of the leaf kernel's block for leaf size nb: up to 128 rows one wave
// per 16 columns holds the whole block; 256 rows are solved by two waves per
// 16 columns holding alternate 16-row blocks (leaf_ilv_kernel).  Larger
// leaves are split recursively down to 256 rows: more waves per column group
// put two waves on a SIMD, where the FP64 matrix work of one and the FP64
// substitution of the other contend, and measured slower.
static int64_t leaf_rows(int64_t nb) { return nb >= 256 ? 256 : std::min<int64_t>(nb, 128); }

size_t packed_bytes(const Canon& c, int64_t nb) {
    const int64_t kleaf = leaf_rows(nb);
    const int64_t nblk = (c.k + kleaf - 1) / kleaf;
    const size_t es = c.dtype == REDSEA_F64 ? 8 : 4;
    return (size_t)nblk * leaf_block_elems((int)kleaf) * es;
}

// Recursive solves with few right-hand sides run as one dataflow launch
// (k_thin.hip; groups of 16 right-hand sides solved side by side) when the
// library owns the memory.  Measured on MI355X (FP64, diagonally dominant
// lower triangle), the launch beats both the split recursive and the
// iterative schedules (nb 256) up to 256 right-hand sides at every order
// from 512 to 8192 (n = 8192: 0.47 / 0.77 / 1.22 ms for 1 / 64 / 256 right-
// hand sides against 1.47 / 1.66 / 1.82 ms iterative), and loses from 512 on.
// REDSEA_THIN=1 takes the launch for every width, REDSEA_THIN=0 never.
constexpr int64_t kThinMaxRhs = 256;

bool thin_pays(int64_t, int64_t nrhs) { return nrhs <= kThinMaxRhs; }

// Whether a recursive solve of this shape takes the one-launch solve.
bool thin_taken(int64_t n, int64_t nrhs) {
    const char* env = std::getenv("REDSEA_THIN");
    const int mode = env ? std::atoi(env) : -1;  // -1: by the measured crossover
    return mode == 1 || (mode != 0 && thin_pays(n, nrhs));
}

int execute(const Canon& c, int variant, int64_t nb, hipStream_t s, void* packed,
            int* thin_flags) {
    if (variant == VAR_RECURSIVE && (!packed || thin_flags) && !c.gemm_bf16) {
        if (thin_taken(c.k, c.nrhs)) {
            WsLease fl;
            if (!packed) {
                int rc = workspace(6, (size_t)thin_flag_count(c.k, c.nrhs) * sizeof(int), s, fl);
                if (rc) return rc;
                thin_flags = (int*)fl.ptr;
            }
            const hipError_t e = traced(REDSEA_KERNEL_THIN, (double)c.k * c.k * c.nrhs, s, [&] {
                return launch_thin(c.dtype, c.tri, c.rhs, c.k, c.nrhs, c.unit, thin_flags, s);
            });
            if (e == hipSuccess) return REDSEA_OK;
            if (e != hipErrorCooperativeLaunchTooLarge) return REDSEA_ERR_HIP;
            (void)hipGetLastError();  // a device that cannot hold one workgroup: the split below
        }
    }
    const int64_t kleaf = leaf_rows(nb);
    const std::vector<Task>& tasks = plan_for(variant, c.k, nb, kleaf);
    const int64_t nblk = (c.k + kleaf - 1) / kleaf;
    int rc = REDSEA_OK;
    WsLease lease;
    if (!packed) {
        if ((rc = workspace(0, packed_bytes(c, nb), s, lease))) return rc;
        packed = lease.ptr;
    }
    if (traced(REDSEA_KERNEL_PACK, 0.0, s, [&] {
            return launch_pack_diag(c.dtype, c.tri, c.k, (int)kleaf, 0, nblk, c.unit, packed, s);
        }) != hipSuccess)
        return REDSEA_ERR_HIP;
    // helper streams only when the library owns the memory: callers that
    // bring it (a batched plan, static scratch) may be capturing a graph
    const int groups = lease.ptr ? column_groups(c) : 1;
    if (groups == 1) {
        // look-ahead on a helper stream (library-owned memory only, as above)
        // for fewer than kLookaheadMaxRhs right-hand sides, where the products
        // leave CUs idle: at n = 8192 it cuts 7-12 % off nrhs = 1 .. 1024,
        // while at nrhs = 8192 the leaves, sharing CUs with the concurrent
        // product, take five times longer (9.41 -> 9.95 ms per solve).
        // REDSEA_LOOKAHEAD=0 / 1 turns it off / on for every width.
        const char* env = std::getenv("REDSEA_LOOKAHEAD");
        const bool want = env ? std::atoi(env) != 0 : c.nrhs < kLookaheadMaxRhs;
        if (!lease.ptr || !want) return run_tasks(c, tasks, kleaf, packed, s);
        Lookahead la;
        if ((rc = lookahead_for(s, &la))) return rc;
        return run_tasks(c, tasks, kleaf, packed, s, &la);
    }

    hipStream_t side[4];
    if ((rc = side_streams(groups, side))) return rc;
    hipEvent_t fork, join[4];
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return REDSEA_ERR_HIP;
    if (hipEventRecord(fork, s) != hipSuccess) return REDSEA_ERR_HIP;
    const int64_t w = (c.nrhs + groups - 1) / groups;
    int made = 0;
    for (int gi = 0; gi < groups && rc == REDSEA_OK; ++gi) {
        const int64_t c0 = gi * w, cw = std::min(w, c.nrhs - c0);
        if (cw <= 0) break;
        if (hipStreamWaitEvent(side[gi], fork, 0) != hipSuccess) { rc = REDSEA_ERR_HIP; break; }
        rc = run_tasks(column_slice(c, c0, cw), tasks, kleaf, packed, side[gi]);
        if (hipEventCreateWithFlags(&join[gi], hipEventDisableTiming) != hipSuccess) {
            rc = REDSEA_ERR_HIP;
            break;
        }
        ++made;
        if (hipEventRecord(join[gi], side[gi]) != hipSuccess ||
            hipStreamWaitEvent(s, join[gi], 0) != hipSuccess)
            rc = REDSEA_ERR_HIP;
    }
    for (int gi = 0; gi < made; ++gi) (void)hipEventDestroy(join[gi]);
    (void)hipEventDestroy(fork);
    return rc;
}

// Exhaustive tuning of one shape on generated data (only when the
// REDSEA_TUNE environment variable is 1), cached per process.
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int64_t, int>, int> g_tuned;
}  // namespace

int tuned_candidate(int dtype, int64_t k, int64_t nrhs, double kappa, hipStream_t s) {
    const char* e = std::getenv("REDSEA_TUNE");
    if (!e || std::atoi(e) != 1) return -1;
    const int kclass = (int)std::lround(std::log10(kappa > 1.0 ? kappa : 1.0));
    auto key = std::make_tuple(dtype, k, nrhs, kclass);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) return it->second;
    }
    std::vector<int> cand;
    for (int c = 0; c < REDSEA_CANDIDATES; ++c)
        if (dtype == REDSEA_F64 || c % 3 == 0) cand.push_back(c);
    std::vector<double> ms(cand.size(), -1.0);
    // the generator's constant diagonal reaches roughly this condition number
    const double cdiag = kappa >= 1e5 ? 0.004 : kappa >= 1e3 ? 0.012 : kappa >= 50 ? 0.1 : 0.0;
    if (redsea_tune_shape(dtype, k, nrhs, cdiag, 12345, 2, cand.data(), (int)cand.size(), ms.data(),
                          s) != REDSEA_OK)
        return -1;
    int best = -1;
    for (size_t i = 0; i < cand.size(); ++i)
        if (ms[i] > 0 && (best < 0 || ms[i] < ms[best])) best = (int)i;
    const int pick = best < 0 ? -1 : cand[best];
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[key] = pick;
    return pick;
}

// Condition estimate from the diagonal alone: for a triangular matrix the
// diagonal entries are the eigenvalues, so max|t_ii| / min|t_ii| is a lower
// bound on its condition number in any norm.  O(k) reads on the device and one
// wait for the two extremes; a unit diagonal gives 1, a zero or non-finite
// extreme an infinite estimate.
int diag_kappa(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
               const void* A, int64_t lda, hipStream_t s, double* kappa) {
    *kappa = 1.0;
    if (diag == REDSEA_UNIT) return REDSEA_OK;
    const Canon c = canonicalize(dtype, side, uplo, trans, diag, m, n, A, lda, nullptr, 1);
    WsLease lease;
    int rc = workspace(2, 2 * sizeof(double), s, lease);
    if (rc) return rc;
    double h[2] = {0.0, 0.0};
    if (launch_diag_extremes(dtype, c.tri, c.k, (double*)lease.ptr, s) != hipSuccess ||
        hipMemcpyAsync(h, lease.ptr, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return REDSEA_ERR_HIP;
    *kappa = (h[1] > 0.0 && std::isfinite(h[0])) ? h[0] / h[1] : INFINITY;
    return REDSEA_OK;
}

int check_args(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
               const void* A, int64_t lda, const void* B, int64_t ldb, bool need_a) {
    if (dtype != REDSEA_F64 && dtype != REDSEA_F32) return -1;
    if (side != REDSEA_LEFT && side != REDSEA_RIGHT) return -2;
    if (uplo != REDSEA_LOWER && uplo != REDSEA_UPPER) return -3;
    if (trans != REDSEA_NOTRANS && trans != REDSEA_TRANS && trans != REDSEA_CONJTRANS) return -4;
    if (diag != REDSEA_NONUNIT && diag != REDSEA_UNIT) return -5;
    if (m < 0) return -6;
    if (n < 0) return -7;
    const int64_t ka = side == REDSEA_LEFT ? m : n;
    if (lda < std::max<int64_t>(1, ka)) return -10;
    if (ldb < std::max<int64_t>(1, m)) return -12;
    if (m > 0 && n > 0) {
        if (need_a && A == nullptr) return -9;
        if (B == nullptr) return -11;
    }
    return 0;
}

// Leaf size when the caller fixes the variant but not nb: the 256-row leaf
// above order 128 (n = 8192: 56.7 TFLOP/s against 53.3 at nb 128; n = 512:
// 97.4 us against 132.6), else 128 (the 256-row kernel always runs its 16
// block steps).
int pick_nb(int requested, int64_t k) {
    if (requested > 0) return requested;
    return k > 128 ? 256 : 128;
}

}  // namespace redsea

using namespace redsea;

extern "C" {

#ifndef REDSEA_BUILD_ID
#define REDSEA_BUILD_ID "unknown"
#endif
const char* redsea_version(void) { return "0.2.0+" REDSEA_BUILD_ID; }

const char* redsea_status_string(int code) {
    if (code < 0) return "invalid argument";
    switch (code) {
        case REDSEA_OK: return "success";
        case REDSEA_ERR_HIP: return "HIP runtime error";
        case REDSEA_ERR_ALLOC: return "device memory allocation failed";
        case REDSEA_ERR_NOCONV: return "iterative refinement did not converge";
        case REDSEA_ERR_NONFINITE: return "non-finite value in result";
        case REDSEA_ERR_UNSUPPORTED: return "unsupported combination";
        case REDSEA_ERR_TOO_LARGE: return "problem exceeds the fixed scratch memory";
        default: return "unknown status";
    }
}

int64_t redsea_schedule(int variant, int64_t m, int nb, int64_t* tasks, int64_t max_tasks) {
    if (variant < 0 || variant > 3) return -1;
    if (m < 0) return -2;
    if (nb <= 0) return -3;
    if (max_tasks > 0 && tasks == nullptr) return -4;
    std::vector<Task> t = build_schedule(variant == 0 ? VAR_RECURSIVE : variant, m, nb);
    for (int64_t i = 0; i < (int64_t)t.size() && i < max_tasks; ++i) {
        tasks[6 * i + 0] = t[i].kind;
        tasks[6 * i + 1] = t[i].row0;
        tasks[6 * i + 2] = t[i].rows;
        tasks[6 * i + 3] = t[i].col0;
        tasks[6 * i + 4] = t[i].cols;
        tasks[6 * i + 5] = t[i].round;
    }
    return (int64_t)t.size();
}

int redsea_trsm(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                double alpha, const void* A, int64_t lda, void* B, int64_t ldb,
                const redsea_opts* opts, void* stream) {
    int rc = check_args(dtype, side, uplo, trans, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (rc) return rc;
    int variant = opts ? opts->variant : 0;
    int nb = opts ? opts->nb : 0;
    int precision = opts ? opts->precision : 0;
    if (variant < 0 || variant > 3) return -13;
    if (!(nb == 0 || nb == 16 || nb == 32 || nb == 64 || nb == 128 || nb == 256 || nb == 512))
        return -13;
    if (precision < 0 || precision > 3) return -13;
    if (m == 0 || n == 0) return REDSEA_OK;
    hipStream_t s = (hipStream_t)stream;
    redsea_opts chosen = opts ? *opts : redsea_opts{0, 0, 0, 0.0, 0};
    if (variant == 0 && nb == 0 && precision == 0 && alpha != 0.0) {
        // learned picker (falls back to the exhaustive tuner when asked to and
        // not confident); a condition estimate, when not given, is taken as
        // that of a diagonally dominant matrix of this order
        const int64_t k = side == REDSEA_LEFT ? m : n, nrhs = side == REDSEA_LEFT ? n : m;
        int confident = 0;
        int cand = -1;
        if (thin_taken(k, nrhs)) {
            // the one-launch solve, measured faster than every split schedule
            // at these widths (the picker's timings of the recursive
            // candidates there predate it)
            variant = VAR_RECURSIVE;
            precision = REDSEA_PREC_NATIVE;
        } else {
            double kap = chosen.kappa;
            if (!(kap > 0.0) &&
                (rc = diag_kappa(dtype, side, uplo, trans, diag, m, n, A, lda, s, &kap)))
                return rc;
            cand = pick_candidate(dtype, k, nrhs, kap, &confident);
            if (!confident) {
                int tuned = tuned_candidate(dtype, k, nrhs, kap, s);
                if (tuned >= 0) cand = tuned;
            }
        }
        if (cand >= 0) decode_candidate(cand, &variant, &nb, &precision);
        chosen.variant = variant;
        chosen.nb = nb;
        chosen.precision = precision;
        opts = &chosen;
    }
    if (alpha != 0.0 && (precision == REDSEA_PREC_FP32_IR || precision == REDSEA_PREC_BF16_IR)) {
        if (dtype != REDSEA_F64) return REDSEA_ERR_UNSUPPORTED;
        const int inner = precision == REDSEA_PREC_FP32_IR ? 1 : 2;
        return mixed_solve(side, uplo, trans, diag, m, n, alpha, (const double*)A, lda,
                           (double*)B, ldb, inner, 1e-12, inner == 1 ? 5 : 10, nullptr, 0,
                           nullptr, opts, s);
    }
    if (alpha == 0.0 || alpha != 1.0) {
        if (launch_scale(dtype, B, m, n, ldb, alpha, s) != hipSuccess) return REDSEA_ERR_HIP;
        if (alpha == 0.0) return REDSEA_OK;
    }
    Canon c = canonicalize(dtype, side, uplo, trans, diag, m, n, A, lda, B, ldb);
    if (variant == 0) variant = VAR_RECURSIVE;
    return execute(c, variant, pick_nb(nb, c.k), s);
}

int redsea_trmm(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                double beta, void* C, int64_t ldc, int method, void* stream) {
    if (dtype != REDSEA_F64 && dtype != REDSEA_F32) return -1;
    if (side != REDSEA_LEFT && side != REDSEA_RIGHT) return -2;
    if (uplo != REDSEA_LOWER && uplo != REDSEA_UPPER) return -3;
    if (trans != REDSEA_NOTRANS && trans != REDSEA_TRANS && trans != REDSEA_CONJTRANS) return -4;
    if (diag != REDSEA_NONUNIT && diag != REDSEA_UNIT) return -5;
    if (m < 0) return -6;
    if (n < 0) return -7;
    const int64_t ka = side == REDSEA_LEFT ? m : n;
    if (lda < std::max<int64_t>(1, ka)) return -10;
    if (ldb < std::max<int64_t>(1, m)) return -12;
    if (ldc < std::max<int64_t>(1, m)) return -15;
    if (method != REDSEA_TRMM_MFMA && method != REDSEA_TRMM_INT8) return -16;
    if (method == REDSEA_TRMM_INT8 && dtype != REDSEA_F64) return -16;
    if (m == 0 || n == 0) return REDSEA_OK;
    if (alpha != 0.0) {
        if (!A) return -9;
        if (!B) return -11;
    }
    if (!C) return -14;
    hipStream_t s = (hipStream_t)stream;
    if (alpha == 0.0)  // C := beta C (zeros without reading C when beta is 0)
        return beta == 1.0 || launch_scale(dtype, C, m, n, ldc, beta, s) == hipSuccess
                   ? REDSEA_OK
                   : REDSEA_ERR_HIP;
    // the product in storage coordinates: C (left) or C^T (right) += M X with
    // M = op(A) (left) or op(A)^T (right)
    const bool right = side == REDSEA_RIGHT;
    const bool a_trans = right ? trans == REDSEA_NOTRANS : trans != REDSEA_NOTRANS;
    const int tri = ((uplo == REDSEA_LOWER) != a_trans) ? 1 : 2;
    const bool unit = diag == REDSEA_UNIT;
    const int64_t k = ka, nrhs = right ? m : n;
    if (method == REDSEA_TRMM_INT8) {
        WsLease lease;
        const size_t mb = (ozaki_m_bytes(k) + 255) & ~(size_t)255;
        int rc = workspace(5, mb + ozaki_x_bytes(k, nrhs), s, lease);
        if (rc) return rc;
        char* ws = (char*)lease.ptr;
        if (ozaki_split_m((const double*)A, lda, k, uplo, a_trans, unit, ws, s) != hipSuccess ||
            ozaki_product(ws, tri, k, nrhs, right, beta, alpha, (const double*)B, ldb,
                          (const double*)C, ldc, (double*)C, ldc, ws + mb, s) != hipSuccess)
            return REDSEA_ERR_HIP;
        return REDSEA_OK;
    }
    GemmArgs g{k, nrhs, k, A, lda, B, ldb, C, ldc};
    return launch_trmm(dtype, a_trans, right, tri, unit, beta, alpha, g, s) == hipSuccess
               ? REDSEA_OK
               : REDSEA_ERR_HIP;
}

void redsea_trace_begin(void) {
    std::lock_guard<std::mutex> lock(g_tr_mu);
    for (auto& r : g_tr) {
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_tr.clear();
    g_tr_on = true;
}

int redsea_trace_end(int64_t* launches, double* ms, double* flops, int nkinds) {
    std::lock_guard<std::mutex> lock(g_tr_mu);
    g_tr_on = false;
    if (nkinds < 0 || (nkinds > 0 && (!launches || !ms || !flops))) return -4;
    for (int k = 0; k < nkinds; ++k) {
        launches[k] = 0;
        ms[k] = 0.0;
        flops[k] = 0.0;
    }
    int rc = REDSEA_OK;
    for (auto& r : g_tr) {
        float t = 0.f;
        if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&t, r.e0, r.e1) != hipSuccess)
            rc = REDSEA_ERR_HIP;
        if (r.kind >= 0 && r.kind < nkinds) {
            launches[r.kind] += 1;
            ms[r.kind] += t;
            flops[r.kind] += r.flops;
        }
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_tr.clear();
    return rc;
}

int redsea_gemm_update(int dtype, int transa, int transx, int64_t M, int64_t N, int64_t K,
                       const void* A, int64_t lda, const void* X, int64_t ldx, void* C,
                       int64_t ldc, int tile, void* stream) {
    if (dtype != REDSEA_F64 && dtype != REDSEA_F32 && dtype != REDSEA_BF16) return -1;
    if (transa != 0 && transa != 1) return -2;
    if (transx != 0 && transx != 1) return -3;
    if (M < 0) return -4;
    if (N < 0) return -5;
    if (K < 0) return -6;
    if (lda < std::max<int64_t>(1, transa ? K : M)) return -8;
    if (ldx < std::max<int64_t>(1, transx ? N : K)) return -10;
    if (ldc < std::max<int64_t>(1, transx ? N : M)) return -12;
    if (tile < -1 || tile >= gemm_tile_count() || (dtype == REDSEA_BF16 && tile != -1)) return -13;
    if (M == 0 || N == 0 || K == 0) return REDSEA_OK;
    if (!A) return -7;
    if (!X) return -9;
    if (!C) return -11;
    GemmArgs g{M, N, K, A, lda, X, ldx, C, ldc};
    const double fl = 2.0 * M * N * K;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == REDSEA_BF16)
        return traced(REDSEA_KERNEL_GEMM, fl, s, [&] {
                   return launch_gemm_bf16(transa != 0, transx != 0, g, s);
               }) == hipSuccess
                   ? REDSEA_OK
                   : REDSEA_ERR_HIP;
    return traced(REDSEA_KERNEL_GEMM, fl, s, [&] {
               return launch_gemm(dtype, transa != 0, transx != 0, g, s, tile);
           }) == hipSuccess
               ? REDSEA_OK
               : REDSEA_ERR_HIP;
}

}  // extern "C"
