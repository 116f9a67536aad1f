// Temporaries held as digit planes on the 8-bit digit base.
//
// A base product on the digit base first splits each operand into three
// planes of signed 8-bit digits (limbs.hip).  When a schedule's temporary is
// written by an addition group and then read only by base products (in one
// operand role) and by later addition groups, until something overwrites it,
// it can live in its block as those planes instead of as residues: the
// addition group writes the planes (3 bytes per entry instead of 8), the
// products read them without a split, and the later addition groups decode
// them.  The block holds the same value, in the form its readers use; its
// location is the one the schedule's table names.
//
// An epilogue row that does not read the product (Table 1 forms T4 in the
// epilogue of P1) is moved into an addition group of its own just before
// the product, so that the temporary it reads and the one it writes qualify
// too; heavy epilogues move into a group after the product.  When the plan
// never writes A (B), the whole input is split into planes once at the start
// of the call and the products and groups read its quadrants from there.
// The analysis runs once per plan and is kept with it; wsmul_plan_export
// shows the result as view forms.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "wsmul_internal.hpp"

namespace wsmul {

namespace {

constexpr int TILE_ROWS = 128, KSTEP_COLS = 64;   // the digit product's tiling

bool same_view(const View &a, const View &b) {
    return a.buf == b.buf && a.off == b.off && a.rows == b.rows && a.cols == b.cols &&
           a.ld == b.ld;
}

bool overlap(const View &a, const View &b) { return !views_disjoint(a, b); }

bool writes_overlap(const OpDesc &op, const View &v) {
    for (int o = 0; o < op.nout; ++o)
        if (overlap(op.out[o], v))
            return true;
    return false;
}

// Can the digit-plane addition kernel run this group?
bool lin_capable(const OpDesc &op) {
    if (op.kind != WS_OP_ADD || op.nin > LD_MAX || op.nout > LD_MAX || op.nout < 1)
        return false;
    const int64_t R = op.out[0].rows, C = op.out[0].cols;
    if (R % 64 || C % 64 || R == 0 || C == 0)
        return false;
    for (int i = 0; i < op.nin; ++i)
        if (op.in[i].rows != R || op.in[i].cols != C)
            return false;
    for (int o = 0; o < op.nout; ++o)
        if (op.out[o].rows != R || op.out[o].cols != C)
            return false;
    return true;
}

bool role_fits(const View &v, int role) {
    if (v.ld != v.cols || v.off % 2)      // dense, 16-byte aligned planes
        return false;
    if (role == 1)
        return v.rows % TILE_ROWS == 0 && v.cols % KSTEP_COLS == 0;
    return v.cols % TILE_ROWS == 0 && v.rows % KSTEP_COLS == 0;
}

// Move epilogue rows that do not read the product out of a product's
// epilogue into an addition group placed just before it, when nothing else
// in that operation touches the row's destination.
void extract_epilogue_rows(std::vector<ExecOp> &ops) {
    std::vector<ExecOp> out;
    out.reserve(ops.size() + 8);
    for (ExecOp &e : ops) {
        OpDesc &g = e.op;
        if (g.kind != WS_OP_GEMM) {
            out.push_back(e);
            continue;
        }
        for (int o = 0; o < g.nout;) {
            const View d = g.out[o];
            bool ok = g.coef[o][0] == 0 && d.buf == WS_BUF_W && !overlap(d, g.a) && !overlap(d, g.b);
            for (int o2 = 0; ok && o2 < g.nout; ++o2)
                if (o2 != o && overlap(d, g.out[o2]))
                    ok = false;
            for (int i = 1; ok && i < g.nin; ++i)
                if (overlap(d, g.in[i]))
                    for (int o2 = 0; o2 < g.nout; ++o2)
                        if (o2 != o && g.coef[o2][i] != 0)
                            ok = false;
            int used = 0;
            for (int i = 1; i < g.nin; ++i)
                used += g.coef[o][i] != 0;
            if (!ok || used == 0 || g.nout == 1) {
                ++o;
                continue;
            }
            ExecOp add{};
            add.op.kind = WS_OP_ADD;
            add.op.depth = g.depth;
            add.op.nout = 1;
            add.op.out[0] = d;
            for (int i = 1; i < g.nin; ++i)
                if (g.coef[o][i] != 0) {
                    add.op.in[add.op.nin] = g.in[i];
                    add.op.coef[0][add.op.nin] = g.coef[o][i];
                    ++add.op.nin;
                }
            out.push_back(add);
            // drop output o, then every epilogue input no output reads
            for (int o2 = o; o2 + 1 < g.nout; ++o2) {
                g.out[o2] = g.out[o2 + 1];
                std::memcpy(g.coef[o2], g.coef[o2 + 1], sizeof(g.coef[o2]));
            }
            --g.nout;
            for (int i = g.nin - 1; i >= 1; --i) {
                bool read = false;
                for (int o2 = 0; o2 < g.nout; ++o2)
                    read = read || g.coef[o2][i] != 0;
                if (read)
                    continue;
                for (int j = i; j + 1 < g.nin; ++j) {
                    g.in[j] = g.in[j + 1];
                    for (int o2 = 0; o2 < g.nout; ++o2)
                        g.coef[o2][j] = g.coef[o2][j + 1];
                }
                --g.nin;
            }
        }
        out.push_back(e);
    }
    ops.swap(out);
}

// A digit product runs its epilogue after its matrix-core work, every tile
// of a round at once, so each epilogue stream beyond the product's own store
// costs its bytes at about 3.2 TB/s, where an addition group moves them at
// about 5 TB/s.  A product with HEAVY_EPILOGUE or more such streams keeps
// only an output that is the product itself, and the other rows move to an
// addition group right after it that reads that output back.
constexpr int HEAVY_EPILOGUE = 4;

void split_heavy_epilogues(std::vector<ExecOp> &ops) {
    std::vector<ExecOp> out;
    out.reserve(ops.size() + 8);
    for (const ExecOp &e : ops) {
        const OpDesc &g = e.op;
        if (g.kind != WS_OP_GEMM || (g.nin - 1) + (g.nout - 1) < HEAVY_EPILOGUE) {
            out.push_back(e);
            continue;
        }
        int star = -1;
        for (int o = 0; o < g.nout && star < 0; ++o) {
            bool ok = g.coef[o][0] == 1;
            for (int i = 1; ok && i < g.nin; ++i)
                ok = g.coef[o][i] == 0 && !overlap(g.out[o], g.in[i]);
            for (int o2 = 0; ok && o2 < g.nout; ++o2)
                ok = o2 == o || !overlap(g.out[o], g.out[o2]);
            ok = ok && !overlap(g.out[o], g.a) && !overlap(g.out[o], g.b);
            if (ok)
                star = o;
        }
        if (star < 0) {
            out.push_back(e);
            continue;
        }
        ExecOp prod = e;
        prod.op.nin = 1;
        prod.op.nout = 1;
        prod.op.out[0] = g.out[star];
        std::memset(prod.op.coef, 0, sizeof(prod.op.coef));
        prod.op.coef[0][0] = 1;
        ExecOp add{};
        add.op.kind = WS_OP_ADD;
        add.op.depth = g.depth;
        add.op.nin = g.nin;
        add.op.in[0] = g.out[star];          // the product, read back
        for (int i = 1; i < g.nin; ++i)
            add.op.in[i] = g.in[i];
        for (int o = 0; o < g.nout; ++o) {
            if (o == star)
                continue;
            add.op.out[add.op.nout] = g.out[o];
            for (int i = 0; i < g.nin; ++i)
                add.op.coef[add.op.nout][i] = g.coef[o][i];
            ++add.op.nout;
        }
        out.push_back(prod);
        out.push_back(add);
    }
    ops.swap(out);
}

// Producer (op, output) pairs barred from holding digits.
using Banned = std::vector<std::pair<size_t, int>>;

bool banned(const Banned &b, size_t i, int o) {
    return std::find(b.begin(), b.end(), std::make_pair(i, o)) != b.end();
}

// Mark every temporary that qualifies (see the head of this file).  src[j][k]
// records which producer an addition input decodes, for conflict repair.
void mark_digit_temporaries(std::vector<ExecOp> &ops, const Banned &ban,
                            std::vector<std::array<std::pair<size_t, int>, WS_MAX_IN>> &src) {
    src.assign(ops.size(), {});
    for (size_t i = 0; i < ops.size(); ++i) {
        const OpDesc &prod = ops[i].op;
        if (!lin_capable(prod))
            continue;
        for (int o = 0; o < prod.nout; ++o) {
            const View v = prod.out[o];
            if (v.buf != WS_BUF_W || banned(ban, i, o))
                continue;
            int role = 0;
            bool ok = true, any_gemm = false;
            std::vector<std::pair<size_t, int>> adds;     // (op, input slot) decoding v
            std::vector<std::pair<size_t, int>> gemms;    // (op, 1 = a, 2 = b)
            for (size_t j = i + 1; j < ops.size() && ok; ++j) {
                const OpDesc &c = ops[j].op;
                if (c.kind == WS_OP_GEMM) {
                    for (int which = 1; which <= 2; ++which) {
                        const View &x = which == 1 ? c.a : c.b;
                        if (same_view(x, v)) {
                            if (role && role != which)
                                ok = false;
                            role = which;
                            any_gemm = true;
                            gemms.push_back({j, which});
                        } else if (overlap(x, v)) {
                            ok = false;
                        }
                    }
                    for (int k = 1; k < c.nin; ++k)
                        if (overlap(c.in[k], v))
                            ok = false;
                } else {
                    for (int k = 0; k < c.nin; ++k) {
                        if (same_view(c.in[k], v)) {
                            if (lin_capable(c))
                                adds.push_back({j, k});
                            else
                                ok = false;
                        } else if (overlap(c.in[k], v)) {
                            ok = false;
                        }
                    }
                }
                if (writes_overlap(c, v))
                    break;
            }
            if (!ok || !any_gemm || !role_fits(v, role))
                continue;
            ops[i].out_enc[o] = (int8_t)role;
            for (auto &g : gemms)
                (g.second == 1 ? ops[g.first].pre_a : ops[g.first].pre_b) = true;
            for (auto &a : adds) {
                ops[a.first].in_enc[a.second] = (int8_t)role;
                src[a.first][a.second] = {i, o};
            }
        }
    }
}

// An addition group that reads a view in one form and writes it back in
// another would have workgroups overwrite bytes that others still read (the
// two forms place a tile at different bytes).  Bar one side and mark again
// until no group does.
void assign_encodings(std::vector<ExecOp> &ops) {
    const std::vector<ExecOp> base = ops;
    Banned ban;
    std::vector<std::array<std::pair<size_t, int>, WS_MAX_IN>> src;
    for (;;) {
        ops = base;
        mark_digit_temporaries(ops, ban, src);
        const size_t before = ban.size();
        for (size_t j = 0; j < ops.size(); ++j) {
            const ExecOp &e = ops[j];
            if (e.op.kind != WS_OP_ADD)
                continue;
            for (int o = 0; o < e.op.nout; ++o)
                for (int k = 0; k < e.op.nin; ++k)
                    if (same_view(e.op.in[k], e.op.out[o]) && e.in_enc[k] != e.out_enc[o]) {
                        if (e.out_enc[o])
                            ban.push_back({j, o});
                        else
                            ban.push_back(src[j][k]);
                    }
        }
        if (ban.size() == before)
            return;
    }
}

// Inputs read as planes.  When the plan never writes A (B), every view of
// it that a product takes as its left (right) operand, or a digit addition
// group reads, and that covers whole tiles, can be read from digit planes of
// the whole input, split once at the start of the call: a product skips its
// split of that view and a group reads 3 bytes per entry instead of 8.  It
// is done for an input when the bytes it spares exceed the whole split's.
void mark_input_planes(DigitExec &x, const PlanKey &key) {
    constexpr int A_ROLE = 1, B_ROLE = 2;
    bool writes_a = false, writes_b = false;
    for (const ExecOp &e : x.ops)
        for (int o = 0; o < e.op.nout; ++o) {
            writes_a = writes_a || e.op.out[o].buf == WS_BUF_A;
            writes_b = writes_b || e.op.out[o].buf == WS_BUF_B;
        }
    auto aligned = [&](const View &v, int role) {
        const int64_t ld = role == A_ROLE ? key.lda : key.ldb;
        if (v.rows <= 0 || v.cols <= 0 || v.ld != ld || ld <= 0)
            return false;
        const int64_t r0 = v.off / ld, c0 = v.off % ld;
        if (role == A_ROLE)
            return r0 % TILE_ROWS == 0 && v.rows % TILE_ROWS == 0 && c0 % KSTEP_COLS == 0 &&
                   v.cols % KSTEP_COLS == 0;
        return c0 % TILE_ROWS == 0 && v.cols % TILE_ROWS == 0 && r0 % KSTEP_COLS == 0 &&
               v.rows % KSTEP_COLS == 0;
    };
    for (int role = A_ROLE; role <= B_ROLE; ++role) {
        const int buf = role == A_ROLE ? WS_BUF_A : WS_BUF_B;
        if (role == A_ROLE ? writes_a : writes_b)
            continue;
        double spared = 0.0;
        for (const ExecOp &e : x.ops) {
            const OpDesc &op = e.op;
            if (op.kind == WS_OP_GEMM) {
                const View &v = role == A_ROLE ? op.a : op.b;
                if (v.buf == buf && aligned(v, role))
                    spared += 11.0 * (double)v.rows * (double)v.cols;
            } else if (lin_capable(op)) {
                for (int i = 0; i < op.nin; ++i)
                    if (op.in[i].buf == buf && aligned(op.in[i], role))
                        spared += 5.0 * (double)op.in[i].rows * (double)op.in[i].cols;
            }
        }
        const double whole = 11.0 * (double)key.k * (double)(role == A_ROLE ? key.m : key.n);
        if (spared <= whole)
            continue;
        for (ExecOp &e : x.ops) {
            OpDesc &op = e.op;
            if (op.kind == WS_OP_GEMM) {
                const View &v = role == A_ROLE ? op.a : op.b;
                if (v.buf == buf && aligned(v, role))
                    (role == A_ROLE ? e.pre_a : e.pre_b) = true;
            } else if (lin_capable(op)) {
                for (int i = 0; i < op.nin; ++i)
                    if (op.in[i].buf == buf && aligned(op.in[i], role))
                        e.in_enc[i] = (int8_t)role;
            }
        }
        if (role == A_ROLE) {
            x.split_a = true;
            x.a_rows = (key.m + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
            x.a_kp = (std::max<int64_t>(key.k, 1) + KSTEP_COLS - 1) / KSTEP_COLS * KSTEP_COLS;
        } else {
            x.split_b = true;
            x.b_cols = (key.n + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS;
            x.b_kp = (std::max<int64_t>(key.k, 1) + KSTEP_COLS - 1) / KSTEP_COLS * KSTEP_COLS;
        }
    }
    x.input_bytes = (size_t)(3 * (x.a_rows * x.a_kp + x.b_cols * x.b_kp));
    x.split_bytes = 0;
    for (const ExecOp &e : x.ops)
        if (e.op.kind == WS_OP_GEMM) {
            const int64_t M = e.op.a.rows, K = std::max<int64_t>(e.op.a.cols, 1), N = e.op.b.cols;
            const int64_t Kp = (K + KSTEP_COLS - 1) / KSTEP_COLS * KSTEP_COLS;
            const size_t own =
                (e.pre_a ? 0 : (size_t)(3 * ((M + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS) * Kp)) +
                (e.pre_b ? 0 : (size_t)(3 * ((N + TILE_ROWS - 1) / TILE_ROWS * TILE_ROWS) * Kp));
            x.split_bytes = std::max(x.split_bytes, own);
        }
}

// Where a view with a form keeps its planes.
struct PlaneAt {
    const int8_t *ptr;
    int64_t ld, plane;      // inner length of the plane rows (K), bytes per plane
};

PlaneAt plane_at(const DigitExec &x, const View &v, int role, const DevBufs &bufs) {
    if (v.buf == WS_BUF_W) {
        const int8_t *p = static_cast<const int8_t *>(bufs.ptr[WS_BUF_W]) + v.off * 8;
        return {p, role == 1 ? v.cols : v.rows, v.rows * v.cols};
    }
    const int8_t *base = static_cast<const int8_t *>(bufs.scratch);
    constexpr int64_t BLOCK = TILE_ROWS * KSTEP_COLS;
    const int64_t r0 = v.off / v.ld, c0 = v.off % v.ld;
    if (v.buf == WS_BUF_A)      // rows r0.., inner c0..
        return {base + ((r0 / TILE_ROWS) * (x.a_kp / KSTEP_COLS) + c0 / KSTEP_COLS) * BLOCK,
                x.a_kp, x.a_rows * x.a_kp};
    const int8_t *bp = base + 3 * x.a_rows * x.a_kp;   // B: inner rows r0.., columns c0..
    return {bp + ((c0 / TILE_ROWS) * (x.b_kp / KSTEP_COLS) + r0 / KSTEP_COLS) * BLOCK, x.b_kp,
            x.b_cols * x.b_kp};
}

}  // namespace

std::shared_ptr<const DigitExec> digit_exec(const Plan &plan) {
    std::lock_guard<std::mutex> lock(plan.exec_mu);
    if (plan.exec_cache)
        return std::static_pointer_cast<const DigitExec>(plan.exec_cache);
    auto x = std::make_shared<DigitExec>();
    x->ops.reserve(plan.ops.size());
    for (const OpDesc &op : plan.ops) {
        ExecOp e{};
        e.op = op;
        x->ops.push_back(e);
    }
    extract_epilogue_rows(x->ops);
    split_heavy_epilogues(x->ops);
    assign_encodings(x->ops);
    mark_input_planes(*x, plan.key);
    plan.exec_cache = x;
    return x;
}

bool exec_uses_digits(const ExecOp &e) {
    for (int i = 0; i < e.op.nin; ++i)
        if (e.in_enc[i])
            return true;
    for (int o = 0; o < e.op.nout; ++o)
        if (e.out_enc[o])
            return true;
    return false;
}

hipError_t launch_input_splits(const DigitExec &x, const DevBufs &bufs, int64_t lda, int64_t ldb,
                               int64_t m, int64_t k, int64_t n, int dtype, int64_t p,
                               hipStream_t stream) {
    int8_t *base = static_cast<int8_t *>(bufs.scratch);
    if ((x.split_a || x.split_b) && (!base || bufs.scratch_bytes < x.input_bytes))
        return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    if (x.split_a)
        e = launch_split_rows(bufs.ptr[WS_BUF_A], lda, m, k, base, dtype, p, stream);
    if (e == hipSuccess && x.split_b)
        e = launch_split_cols(bufs.ptr[WS_BUF_B], ldb, k, n, base + 3 * x.a_rows * x.a_kp, dtype,
                              p, stream);
    return e;
}

hipError_t launch_exec_gemm(const DigitExec &x, const ExecOp &e, const DevBufs &bufs, int dtype,
                            int64_t p, hipStream_t stream) {
    const OpDesc &op = e.op;
    PlaneRef ra{}, rb{};
    if (e.pre_a) {
        const PlaneAt at = plane_at(x, op.a, 1, bufs);
        ra = {at.ptr, at.plane, at.ld / KSTEP_COLS};
    }
    if (e.pre_b) {
        const PlaneAt at = plane_at(x, op.b, 2, bufs);
        rb = {at.ptr, at.plane, at.ld / KSTEP_COLS};
    }
    DevBufs b = bufs;
    b.split_offset = x.input_bytes;
    return launch_gemm_limbs(op, b, dtype, p, stream, e.pre_a ? &ra : nullptr,
                             e.pre_b ? &rb : nullptr);
}

// One addition group with digit-plane inputs or outputs.  Its outputs fall
// into independent parts (outputs that share no input, as the S and T halves
// of a Table 1 pre-addition); each part is its own launch, so a workgroup
// holds only the part's inputs in LDS and more of them fit on a CU.
hipError_t launch_exec_add(const DigitExec &x, const ExecOp &e, const DevBufs &bufs, int dtype,
                           int64_t p, hipStream_t stream) {
    const OpDesc &op = e.op;
    int part[WS_MAX_OUT];
    for (int o = 0; o < op.nout; ++o)
        part[o] = o;
    auto root = [&](int o) {
        while (part[o] != o)
            o = part[o];
        return o;
    };
    for (int i = 0; i < op.nin; ++i) {
        int first = -1;
        for (int o = 0; o < op.nout; ++o)
            if (op.coef[o][i] != 0) {
                if (first < 0)
                    first = o;
                else
                    part[root(o)] = root(first);
            }
    }
    // an output that overwrites a view some part reads joins that part: the
    // kernel reads every input of a tile before it writes any output
    for (int i = 0; i < op.nin; ++i)
        for (int o = 0; o < op.nout; ++o)
            if (overlap(op.in[i], op.out[o]))
                for (int o2 = 0; o2 < op.nout; ++o2)
                    if (op.coef[o2][i] != 0)
                        part[root(o2)] = root(o);
    // an output that reads nothing is a part of its own (written as zero)
    auto io = [&](const View &v, int kind) {
        DigitIO d{};
        d.kind = kind;
        if (kind == 0) {
            d.ptr = static_cast<const char *>(bufs.ptr[v.buf]) + v.off * 8;
            d.ld = v.ld;
        } else {
            const PlaneAt at = plane_at(x, v, kind, bufs);
            d.ptr = at.ptr;
            d.ld = at.ld;
            d.plane = at.plane;
        }
        return d;
    };
    for (int r = 0; r < op.nout; ++r) {
        if (root(r) != r)
            continue;
        LinDigitsParams L{};
        L.R = op.out[0].rows;
        L.Cc = op.out[0].cols;
        L.p = (double)p;
        L.pinv = 1.0 / (double)p;
        L.half = digit_threshold(p);
        int in_of[WS_MAX_IN];
        for (int i = 0; i < op.nin; ++i) {
            in_of[i] = -1;
            bool used = false;
            for (int o = 0; o < op.nout; ++o)
                used = used || (root(o) == r && op.coef[o][i] != 0);
            if (used) {
                in_of[i] = L.nin;
                L.in[L.nin++] = io(op.in[i], e.in_enc[i]);
            }
        }
        if (L.nin == 0) {            // outputs with no inputs: read one as a dummy
            in_of[0] = 0;
            L.in[L.nin++] = io(op.in[0], e.in_enc[0]);
        }
        for (int o = 0; o < op.nout; ++o) {
            if (root(o) != r)
                continue;
            for (int i = 0; i < op.nin; ++i)
                if (in_of[i] >= 0)
                    L.coef[L.nout][in_of[i]] = (double)op.coef[o][i];
            L.out[L.nout++] = io(op.out[o], e.out_enc[o]);
        }
        const hipError_t err = launch_lin_digits(L, dtype, stream);
        if (err != hipSuccess)
            return err;
    }
    return hipSuccess;
}

}  // namespace wsmul
