// Schedules of the three models of computation (paper Sec. V) as task lists
// in canonical coordinates: the solve is always a forward substitution with
// a lower-triangular T of order m, rows split at multiples of the leaf size.
#pragma once
#include <cstdint>
#include <vector>

namespace redsea {

enum TaskKind : int { TASK_LEAF = 0, TASK_GEMM = 1 };

// kind LEAF: X[row0:row0+rows] = T[row0.., row0..]^{-1} B[row0:row0+rows]
// kind GEMM: B[row0:row0+rows] -= T[row0:row0+rows, col0:col0+cols] X[col0:col0+cols]
// Tasks with the same `round` are independent and are issued as one launch;
// rounds run in increasing order.
struct Task {
    int kind;
    int64_t row0, rows, col0, cols;
    int64_t round;
};

enum Variant : int { VAR_AUTO = 0, VAR_RECURSIVE = 1, VAR_ITERATIVE = 2, VAR_BLOCKED = 3 };

// Builds the task list; nb > 0, m >= 0.
std::vector<Task> build_schedule(int variant, int64_t m, int64_t nb);

// Blocked rounds only (Sec. V-C): for r leaves, the list of rounds, each a
// list of (p, q) blocks meaning "row block p -= T_pq X_q".  Round t (1-based)
// runs after leaf t-1 and before leaf t.
std::vector<std::vector<std::pair<int64_t, int64_t>>> blocked_rounds(int64_t r);

}  // namespace redsea
