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
// too; heavy epilogues move into a group after the product.  The analysis
// runs once per plan and is kept with it.
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

}  // namespace

std::shared_ptr<const std::vector<ExecOp>> digit_exec(const Plan &plan) {
    std::lock_guard<std::mutex> lock(plan.exec_mu);
    if (plan.exec_cache)
        return std::static_pointer_cast<const std::vector<ExecOp>>(plan.exec_cache);
    auto ops = std::make_shared<std::vector<ExecOp>>();
    ops->reserve(plan.ops.size());
    for (const OpDesc &op : plan.ops) {
        ExecOp e{};
        e.op = op;
        ops->push_back(e);
    }
    extract_epilogue_rows(*ops);
    split_heavy_epilogues(*ops);
    assign_encodings(*ops);
    plan.exec_cache = ops;
    return ops;
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

// One addition group with digit-plane inputs or outputs.  Its outputs fall
// into independent parts (outputs that share no input, as the S and T halves
// of a Table 1 pre-addition); each part is its own launch, so a workgroup
// holds only the part's inputs in LDS and more of them fit on a CU.
hipError_t launch_exec_add(const ExecOp &e, const DevBufs &bufs, int dtype, int64_t p,
                           hipStream_t stream) {
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
        d.ptr = static_cast<const char *>(bufs.ptr[v.buf]) + v.off * 8;
        d.ld = kind == 0 ? v.ld : (kind == 1 ? v.cols : v.rows);
        d.plane = v.rows * v.cols;
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
        L.half = std::floor((double)p / 2.0);
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
