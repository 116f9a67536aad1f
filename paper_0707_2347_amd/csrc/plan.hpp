// Planner: expands a memory schedule of Winograd's algorithm into a list of
// device operations on views of A, B, C and one workspace.
//
// Each table of the paper (Tables 1-9) and Algorithm 2 is a host function
// that emits, row by row, either an addition row (dst <- sum c_i * src_i mod p)
// or a product row (dst <- alpha*a*b + beta*e).  Recursion stops after
// `levels` Winograd levels; the remaining product rows are base products run
// on the matrix cores.  A fusion pass then merges consecutive rows into one
// launch when that cannot change any stored value (see Fuser).
#pragma once

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "wsmul.h"

namespace wsmul {

using View = ws_view;
using OpDesc = ws_op_desc;

// Which table runs (also reported in ws_stats.schedule).
enum Table : int {
    TAB_CLASSICAL = 0,
    TAB_T1 = 1,     // Table 1
    TAB_HL = 2,     // Table 2
    TAB_IP = 3,     // Table 3
    TAB_OVL = 4,    // Table 4
    TAB_OVR = 5,    // Table 5
    TAB_ACLR = 6,   // Table 6
    TAB_ACCR = 7,   // Table 7
    TAB_ACR = 8,    // Table 8
    TAB_ACC = 9,    // Table 9
    TAB_IP0VMM = 11,  // Algorithm 1
    TAB_IPMM = 12,  // Algorithm 2
    TAB_IPMM_ACC = 15,  // Algorithm 2 with Table 9 accumulations
    TAB_BLOCKED_HL = 13,   // Section 7.2, t x t blocks over Table 2
    TAB_BLOCKED_ACC = 14,  // Section 7.2, t x t blocks over Table 9
    TAB_ROWS = 16,         // a schedule given as rows (PlanKey::blocks holds its id)
};

struct PlanKey {
    int64_t m, k, n, p, lda, ldb, ldc, alpha, beta;
    int32_t dtype, table, levels, fuse;
    int32_t blocks;   // t of the blocked tables, 0 for the others
    bool operator==(const PlanKey &o) const;
};

struct Plan {
    PlanKey key{};
    std::vector<OpDesc> ops;
    int64_t ws_elems = 0;         // workspace elements (the schedule's extra memory)
    int64_t rows = 0;             // schedule rows emitted (before fusion)
    int64_t element_additions = 0;
    int64_t base_flops = 0;
    int64_t add_ops = 0, gemm_ops = 0;
    // Per-base execution lists derived from ops on first use (the digit
    // base's temporaries held as digit planes), kept with the plan.
    mutable std::mutex exec_mu;
    mutable std::shared_ptr<const void> exec_cache;
};

// Validation result for a (schedule, shape, beta) request.
struct Resolved {
    int status = WS_OK;
    std::string error;
    int table = TAB_CLASSICAL;
    int levels = 0;
};

// Map the public schedule selector and beta to a table, checking shapes.
// `blocks` is t of the blocked schedules (ignored by the others).
Resolved resolve_schedule(int schedule, int64_t m, int64_t k, int64_t n, bool beta_nonzero,
                          int levels, int blocks = 2);

// Do two views share no element?  Exact for views of one leading dimension,
// by the address spans they touch otherwise.
bool views_disjoint(const View &a, const View &b);

// Build the plan for an already resolved request.
void build_plan(const PlanKey &key, Plan &plan);

// Temporaries (elements) of a resolved table at this shape.
int64_t workspace_elems(int table, int64_t m, int64_t k, int64_t n, int levels, int blocks = 2);

// Lengths of the consecutive parts of one dimension of length d in the
// blocked accumulation with t blocks per dimension and depth L.
std::vector<int64_t> block_parts(int64_t d, int t, int L);

// Row schedules: validate and register one (returns an id >= 1, or 0 with
// *error set); ids of equal row lists are equal.
int register_rows(const ws_row *rows, int nrows, int ntemps, std::string *error);
bool rows_registered(int id);

bool ipmm_supported(int64_t m, int64_t k, int64_t n, int levels);
bool ip0vmm_supported(int64_t m, int64_t k, int64_t n, int levels);

}  // namespace wsmul
