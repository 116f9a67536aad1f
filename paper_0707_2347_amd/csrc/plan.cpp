// Schedule expansion and row fusion (host code, no GPU needed).
//
// Notation follows Section 2: A (m x k), B (k x n), C (m x n) split into
// quadrants; S1..S4 and T1..T4 are the pre-additions, P1..P7 the products,
// U1..U7 the post-additions.  Every row below writes the location of the
// table's "loc." column.  alpha is applied by the base products (linearity);
// beta where the rows say; "-beta" is the residue p - beta.  Where an
// "operation" entry names only the beta-free value (e.g. Table 9 row 10), the
// row is executed with the location semantics that yield alpha*A*B + beta*C.
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

namespace wsmul {

bool PlanKey::operator==(const PlanKey &o) const {
    return m == o.m && k == o.k && n == o.n && p == o.p && lda == o.lda && ldb == o.ldb &&
           ldc == o.ldc && alpha == o.alpha && beta == o.beta && dtype == o.dtype &&
           table == o.table && levels == o.levels && fuse == o.fuse && blocks == o.blocks;
}

namespace {

View mkview(int buf, int64_t off, int64_t rows, int64_t cols, int64_t ld) {
    View v;
    std::memset(&v, 0, sizeof(v));
    v.buf = buf;
    v.off = off;
    v.rows = rows;
    v.cols = cols;
    v.ld = ld;
    return v;
}

// Quadrant (i, j) of v: half the rows and half the columns (Section 2).
View quad(const View &v, int i, int j) {
    const int64_t r = v.rows / 2, c = v.cols / 2;
    return mkview(v.buf, v.off + i * r * v.ld + j * c, r, c, v.ld);
}

View block(const View &v, int64_t r0, int64_t c0, int64_t r, int64_t c) {
    return mkview(v.buf, v.off + r0 * v.ld + c0, r, c, v.ld);
}

bool same(const View &a, const View &b) {
    return a.buf == b.buf && a.off == b.off && a.rows == b.rows && a.cols == b.cols &&
           a.ld == b.ld;
}

// Exact disjointness of two strided views.  With equal leading dimensions
// both are rectangles of one row-major grid: place a's origin at (0, 0); b's
// origin is then (q, s) with 0 <= s < ld, and b covers columns [s, s+cols)
// of its rows, the part past ld wrapping to column 0 of the next row.
// Otherwise fall back to the address spans they touch.
bool disjoint(const View &a, const View &b) {
    if (a.buf != b.buf || a.rows == 0 || a.cols == 0 || b.rows == 0 || b.cols == 0)
        return true;
    if (a.ld == b.ld && a.ld > 0 && a.cols <= a.ld && b.cols <= b.ld) {
        const int64_t ld = a.ld, delta = b.off - a.off;
        int64_t q = delta / ld, s = delta % ld;
        if (s < 0) {
            s += ld;
            q -= 1;
        }
        auto hit = [&](int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
            // does [r0, r1) x [c0, c1) meet a's [0, rows) x [0, cols)?
            return r0 < a.rows && r1 > 0 && c0 < a.cols && c1 > 0 && r0 < r1 && c0 < c1;
        };
        const int64_t first = std::min(s + b.cols, ld);
        if (hit(q, q + b.rows, s, first))
            return false;
        if (s + b.cols > ld && hit(q + 1, q + 1 + b.rows, 0, s + b.cols - ld))
            return false;
        return true;
    }
    const int64_t a0 = a.off, a1 = a.off + (a.rows - 1) * a.ld + a.cols;
    const int64_t b0 = b.off, b1 = b.off + (b.rows - 1) * b.ld + b.cols;
    return a1 <= b0 || b1 <= a0;
}

}  // namespace

bool views_disjoint(const View &a, const View &b) { return disjoint(a, b); }

namespace {

struct Term {
    int64_t c;
    View v;
};

std::string describe(const View &v) {
    return "[buf " + std::to_string(v.buf) + " off " + std::to_string(v.off) + " " +
           std::to_string(v.rows) + "x" + std::to_string(v.cols) + " ld " + std::to_string(v.ld) + "]";
}

// ---------------------------------------------------------------- fusion
// Rows arrive in schedule order.  A group is a set of rows applied to every
// element position independently: the kernel loads each distinct input
// location once, forms every written location as a linear combination of
// those inputs, and stores each written location once.  That equals running
// the rows one after the other provided all views have one shape and any two
// distinct views are disjoint.  A product row opens a group whose input 0 is
// the product itself; following addition rows join it as its epilogue when,
// in addition, nothing they write overlaps the product's operands (other
// workgroups are still reading those).
class Fuser {
  public:
    Fuser(int64_t p, bool enabled, std::vector<OpDesc> &out) : p_(p), on_(enabled), out_(out) {}

    void row_add(const View &dst, const std::vector<Term> &terms, int depth) {
        if (open_ && on_ && append(dst, terms))
            return;
        flush();
        std::memset(&g_, 0, sizeof(g_));
        g_.kind = WS_OP_ADD;
        g_.depth = depth;
        open_ = true;
        if (!append(dst, terms)) {
            std::string msg = "addition row with overlapping views: dst " + describe(dst);
            for (const Term &t : terms)
                msg += " src " + describe(t.v);
            throw std::logic_error(msg);
        }
    }

    void row_gemm(const View &a, const View &b, const View &d, int64_t alpha, int64_t beta,
                  int depth) {
        if (!disjoint(d, a) || !disjoint(d, b))
            throw std::logic_error("product destination overlaps an operand");
        flush();
        std::memset(&g_, 0, sizeof(g_));
        g_.kind = WS_OP_GEMM;
        g_.depth = depth;
        g_.alpha = alpha;
        g_.a = a;
        g_.b = b;
        g_.nin = 1;  // in[0] is the product
        g_.in[0] = mkview(-1, 0, d.rows, d.cols, 0);
        g_.nout = 1;
        g_.out[0] = d;
        g_.coef[0][0] = 1;
        if (beta % p_) {
            g_.in[1] = d;
            g_.nin = 2;
            g_.coef[0][1] = beta % p_;
        }
        open_ = true;
    }

    void flush() {
        if (open_)
            out_.push_back(g_);
        open_ = false;
    }

  private:
    int find(const View *vs, int lo, int n, const View &v) const {
        for (int i = lo; i < n; ++i)
            if (same(vs[i], v))
                return i;
        return -1;
    }

    bool compatible(const View &v) const {
        const int lo = g_.kind == WS_OP_GEMM ? 1 : 0;
        for (int i = lo; i < g_.nin; ++i)
            if (!same(g_.in[i], v) && !disjoint(g_.in[i], v))
                return false;
        for (int o = 0; o < g_.nout; ++o)
            if (!same(g_.out[o], v) && !disjoint(g_.out[o], v))
                return false;
        return true;
    }

    bool append(const View &dst, const std::vector<Term> &terms) {
        const bool empty = g_.nout == 0 && g_.nin == 0;
        int64_t rows = empty ? dst.rows : g_.out[0].rows;
        int64_t cols = empty ? dst.cols : g_.out[0].cols;
        if (dst.rows != rows || dst.cols != cols)
            return false;
        for (const Term &t : terms) {
            if (t.v.rows != rows || t.v.cols != cols)
                return false;
            if (!same(t.v, dst) && !disjoint(t.v, dst))
                return false;
            for (const Term &u : terms)
                if (!same(t.v, u.v) && !disjoint(t.v, u.v))
                    return false;
        }
        if (!compatible(dst))
            return false;
        for (const Term &t : terms)
            if (!compatible(t.v))
                return false;
        if (g_.kind == WS_OP_GEMM && (!disjoint(dst, g_.a) || !disjoint(dst, g_.b)))
            return false;

        OpDesc t = g_;
        const int lo = t.kind == WS_OP_GEMM ? 1 : 0;
        int64_t comb[WS_MAX_IN] = {0};
        for (const Term &term : terms) {
            const int64_t c = ((term.c % p_) + p_) % p_;
            const int o = find(t.out, 0, t.nout, term.v);
            if (o >= 0) {
                for (int i = 0; i < WS_MAX_IN; ++i)
                    comb[i] = (comb[i] + c * t.coef[o][i]) % p_;
                continue;
            }
            int i = find(t.in, lo, t.nin, term.v);
            if (i < 0) {
                if (t.nin == WS_MAX_IN)
                    return false;
                i = t.nin++;
                t.in[i] = term.v;
            }
            comb[i] = (comb[i] + c) % p_;
        }
        int o = find(t.out, 0, t.nout, dst);
        if (o < 0) {
            if (t.nout == WS_MAX_OUT)
                return false;
            o = t.nout++;
            t.out[o] = dst;
        }
        for (int i = 0; i < WS_MAX_IN; ++i)
            t.coef[o][i] = comb[i];
        g_ = t;
        return true;
    }

    int64_t p_;
    bool on_;
    std::vector<OpDesc> &out_;
    OpDesc g_{};
    bool open_ = false;
};

// --------------------------------------------------------------- emitter
// Registered row schedules (index + 1 is the id); never removed.
struct RowSchedule {
    std::vector<ws_row> rows;
    int ntemps;
};
std::mutex g_rows_mu;
std::vector<RowSchedule> g_row_schedules;

bool row_schedule(int id, std::vector<ws_row> &rows, int &ntemps) {
    std::lock_guard<std::mutex> lock(g_rows_mu);
    if (id < 1 || id > (int)g_row_schedules.size())
        return false;
    rows = g_row_schedules[(size_t)id - 1].rows;
    ntemps = g_row_schedules[(size_t)id - 1].ntemps;
    return true;
}

class Emitter {
  public:
    Emitter(int64_t p, bool measure, bool fuse, std::vector<OpDesc> &ops)
        : p_(p), measure_(measure), fuser_(p, fuse, ops) {}

    std::vector<int64_t> need;      // per call depth: elements of temporaries
    std::vector<int64_t> base;      // per call depth: offset in the workspace
    int64_t rows = 0, element_additions = 0, base_flops = 0;

    int64_t neg(int64_t x) const { return (p_ - x % p_) % p_; }

    // ---- rows
    void lin(const View &d, std::vector<Term> terms) {
        ++rows;
        element_additions += d.rows * d.cols;
        if (!measure_)
            fuser_.row_add(d, terms, depth_);
    }
    void add(const View &d, const View &x, const View &y) { lin(d, {{1, x}, {1, y}}); }
    void sub(const View &d, const View &x, const View &y) { lin(d, {{1, x}, {p_ - 1, y}}); }
    // d <- alpha*a*b + beta*d; a base product (classical, on the matrix cores)
    void gemm(const View &a, const View &b, const View &d, int64_t alpha, int64_t beta) {
        ++rows;
        base_flops += 2 * a.rows * a.cols * b.cols;
        if (!measure_)
            fuser_.row_gemm(a, b, d, alpha % p_, beta % p_, depth_);
    }
    void finish() { fuser_.flush(); }

    // ---- temporaries
    struct Frame {
        View v[WS_ROW_MAX_TEMPS > 3 ? WS_ROW_MAX_TEMPS : 3];
        bool region = false;
    };
    // Temporaries of one call at call depth d.  Normally they are carved from
    // the workspace slot of that depth (calls at one depth never overlap in
    // time); inside Algorithms 1 and 2 they are quadrants of a lent region
    // (a free square of C or A): first in the top-left, second in the
    // bottom-left, third in the top-right, and the bottom-right is lent on to
    // the callees.
    Frame frame(int d, std::initializer_list<std::pair<int64_t, int64_t>> shapes) {
        return frame(d, std::vector<std::pair<int64_t, int64_t>>(shapes));
    }
    Frame frame(int d, const std::vector<std::pair<int64_t, int64_t>> &shapes) {
        Frame f;
        if (!regions_.empty()) {
            const View R = regions_.back();
            const View slot[3] = {quad(R, 0, 0), quad(R, 1, 0), quad(R, 0, 1)};
            if (shapes.size() > 3)
                throw std::logic_error("a lent region hosts at most three temporaries");
            int i = 0;
            for (auto &s : shapes) {
                if (s.first > slot[i].rows || s.second > slot[i].cols)
                    throw std::logic_error("temporary does not fit its quadrant");
                f.v[i] = block(slot[i], 0, 0, s.first, s.second);
                ++i;
            }
            regions_.push_back(quad(R, 1, 1));
            f.region = true;
            return f;
        }
        if ((int)need.size() <= d) {
            need.resize(d + 1, 0);
        }
        int64_t total = 0;
        int i = 0;
        for (auto &s : shapes) {
            const int64_t off = (!measure_ && d < (int)base.size()) ? base[d] + total : 0;
            f.v[i++] = mkview(WS_BUF_W, off, s.first, s.second, s.second);
            total += s.first * s.second;
        }
        need[d] = std::max(need[d], total);
        return f;
    }
    void release(const Frame &f) {
        if (f.region)
            regions_.pop_back();
    }

    // ---- Table 1: C <- a*A*B, temporaries X (m/2 x max(k/2,n/2)), Y (k/2 x n/2)
    void t1(View A, View B, View C, int64_t a, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, 0);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const int64_t h = A.rows / 2, kk = A.cols / 2, w = B.cols / 2;
        Frame f = frame(d, {{h, std::max(kk, w)}, {kk, w}});
        View X = f.v[0], Y = f.v[1];
        View XS = X, XP = X;       // X holding an S block, then a product
        XS.cols = kk;
        XP.cols = w;
        if (!f.region) {
            XS.ld = kk;
            XP.ld = w;
        }
        sub(XS, A11, A21);                    // 1  S3
        sub(Y, B22, B12);                     // 2  T3
        t1(XS, Y, C21, a, lev - 1, d + 1);    // 3  P7 = S3 T3
        depth_ = d;
        add(XS, A21, A22);                    // 4  S1
        sub(Y, B12, B11);                     // 5  T1
        t1(XS, Y, C22, a, lev - 1, d + 1);    // 6  P5 = S1 T1
        depth_ = d;
        sub(XS, XS, A11);                     // 7  S2
        sub(Y, B22, Y);                       // 8  T2
        t1(XS, Y, C12, a, lev - 1, d + 1);    // 9  P6 = S2 T2
        depth_ = d;
        sub(XS, A12, XS);                     // 10 S4
        t1(XS, B22, C11, a, lev - 1, d + 1);  // 11 P3 = S4 B22
        t1(A11, B11, XP, a, lev - 1, d + 1);  // 12 P1
        depth_ = d;
        add(C12, XP, C12);                    // 13 U2 = P1 + P6
        add(C21, C12, C21);                   // 14 U3 = U2 + P7
        add(C12, C12, C22);                   // 15 U4 = U2 + P5
        add(C22, C21, C22);                   // 16 U7 = U3 + P5
        add(C12, C12, C11);                   // 17 U5 = U4 + P3
        sub(Y, Y, B21);                       // 18 T4 = T2 - B21
        t1(A22, Y, C11, a, lev - 1, d + 1);   // 19 P4 = A22 T4
        depth_ = d;
        sub(C21, C21, C11);                   // 20 U6 = U3 - P4
        t1(A12, B21, C11, a, lev - 1, d + 1); // 21 P2
        depth_ = d;
        add(C11, XP, C11);                    // 22 U1 = P1 + P2
        release(f);
    }

    // ---- Table 2: C <- a*A*B + b*C, temporaries X (m/2 x k/2), Y (k/2 x n/2), Z (m/2 x n/2)
    void hl(View A, View B, View C, int64_t a, int64_t b, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, b);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const int64_t h = A.rows / 2, kk = A.cols / 2, w = B.cols / 2;
        Frame f = frame(d, {{h, kk}, {kk, w}, {h, w}});
        const View X = f.v[0], Y = f.v[1], Z = f.v[2];
        add(X, A21, A22);                       // 1  S1
        sub(Y, B12, B11);                       // 2  T1
        t1(X, Y, Z, a, lev - 1, d + 1);         // 3  P5 = a S1 T1
        depth_ = d;
        lin(C22, {{1, Z}, {b, C22}});           // 4  C22 = P5 + b C22
        lin(C12, {{1, Z}, {b, C12}});           // 5  C12 = P5 + b C12
        sub(X, X, A11);                         // 6  S2
        sub(Y, B22, Y);                         // 7  T2
        t1(A11, B11, Z, a, lev - 1, d + 1);     // 8  P1
        depth_ = d;
        lin(C11, {{1, Z}, {b, C11}});           // 9  C11 = P1 + b C11
        hl(X, Y, Z, a, 1, lev - 1, d + 1);      // 10 U2 = a S2 T2 + P1
        hl(A12, B21, C11, a, 1, lev - 1, d + 1);// 11 U1 = a A12 B21 + C11
        depth_ = d;
        sub(X, A12, X);                         // 12 S4
        sub(Y, Y, B21);                         // 13 T4
        hl(X, B22, C12, a, 1, lev - 1, d + 1);  // 14 C12 = a S4 B22 + C12
        depth_ = d;
        add(C12, Z, C12);                       // 15 U5 = U2 + C12
        hl(A22, Y, C21, a, neg(b), lev - 1, d + 1); // 16 C21 = a A22 T4 - b C21
        depth_ = d;
        sub(X, A11, A21);                       // 17 S3
        sub(Y, B22, B12);                       // 18 T3
        hl(X, Y, Z, a, 1, lev - 1, d + 1);      // 19 U3 = a S3 T3 + U2
        depth_ = d;
        add(C22, Z, C22);                       // 20 U7 = U3 + C22
        sub(C21, Z, C21);                       // 21 U6 = U3 - C21
        release(f);
    }

    // ---- Table 3: C <- a*A*B in place, no temporary; overwrites A and B
    void ip(View A, View B, View C, int64_t a, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, 0);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        sub(C11, A11, A21);                   // 1  S3
        add(A21, A21, A22);                   // 2  S1
        sub(C22, B12, B11);                   // 3  T1
        sub(B12, B22, B12);                   // 4  T3
        ip(C11, B12, C21, a, lev - 1, d + 1); // 5  P7 = S3 T3
        depth_ = d;
        sub(C12, A21, A11);                   // 6  S2
        ip(A11, B11, C11, a, lev - 1, d + 1); // 7  P1
        depth_ = d;
        sub(B11, B22, C22);                   // 8  T2
        ip(A21, C22, A11, a, lev - 1, d + 1); // 9  P5 = S1 T1
        depth_ = d;
        sub(C22, B11, B21);                   // 10 T4
        ip(A22, C22, A21, a, lev - 1, d + 1); // 11 P4 = A22 T4
        depth_ = d;
        sub(A22, A12, C12);                   // 12 S4
        ip(C12, B11, C22, a, lev - 1, d + 1); // 13 P6 = S2 T2
        depth_ = d;
        add(C22, C11, C22);                   // 14 U2 = P1 + P6
        ip(A12, B21, C12, a, lev - 1, d + 1); // 15 P2
        depth_ = d;
        add(C11, C11, C12);                   // 16 U1 = P1 + P2
        add(C12, C22, A11);                   // 17 U4 = U2 + P5
        add(C22, C22, C21);                   // 18 U3 = U2 + P7
        sub(C21, C22, A21);                   // 19 U6 = U3 - P4
        add(C22, C22, A11);                   // 20 U7 = U3 + P5
        ip(A22, B22, A12, a, lev - 1, d + 1); // 21 P3 = S4 B22
        depth_ = d;
        add(C12, C12, A12);                   // 22 U5 = U4 + P3
    }

    // ---- Table 4: C <- a*A*B, one temporary X ((n/2)^2); overwrites A
    void ovl(View A, View B, View C, int64_t a, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, 0);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const int64_t h = C.rows / 2;
        Frame f = frame(d, {{h, h}});
        const View X = f.v[0];
        sub(C22, A11, A21);                    // 1  S3
        add(A21, A21, A22);                    // 2  S1
        sub(C12, A21, A11);                    // 3  S2 = S1 - A11
        sub(C21, B12, B11);                    // 4  T1
        ovl(A11, B11, C11, a, lev - 1, d + 1); // 5  P1
        depth_ = d;
        sub(A11, B22, B12);                    // 6  T3
        ip(C22, A11, X, a, lev - 1, d + 1);    // 7  P7 = S3 T3
        depth_ = d;
        sub(A11, B22, C21);                    // 8  T2 = B22 - T1
        ip(A21, C21, C22, a, lev - 1, d + 1);  // 9  P5 = S1 T1
        depth_ = d;
        sub(C21, A12, C12);                    // 10 S4 = A12 - S2
        ovl(C21, B22, A21, a, lev - 1, d + 1); // 11 P3 = S4 B22
        ovl(C12, A11, C21, a, lev - 1, d + 1); // 12 P6 = S2 T2
        depth_ = d;
        sub(A11, A11, B21);                    // 13 T4 = T2 - B21
        add(C21, C11, C21);                    // 14 U2 = P1 + P6
        add(C12, C21, C22);                    // 15 U4 = U2 + P5
        add(C21, C21, X);                      // 16 U3 = U2 + P7
        add(C22, C21, C22);                    // 17 U7 = U3 + P5
        add(C12, C12, A21);                    // 18 U5 = U4 + P3
        ovl(A12, B21, X, a, lev - 1, d + 1);   // 19 P2
        depth_ = d;
        add(C11, C11, X);                      // 20 U1 = P1 + P2
        ip(A22, A11, A21, a, lev - 1, d + 1);  // 21 P4 = A22 T4
        depth_ = d;
        sub(C21, C21, A21);                    // 22 U6 = U3 - P4
        release(f);
    }

    // ---- Table 5: C <- a*A*B, one temporary X ((n/2)^2); overwrites B
    void ovr(View A, View B, View C, int64_t a, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, 0);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const int64_t h = C.rows / 2;
        Frame f = frame(d, {{h, h}});
        const View X = f.v[0];
        sub(C22, A11, A21);                    // 1  S3
        add(C21, A21, A22);                    // 2  S1
        sub(C12, B12, B11);                    // 3  T1
        ovr(A11, B11, C11, a, lev - 1, d + 1); // 4  P1
        depth_ = d;
        sub(B11, C21, A11);                    // 5  S2
        sub(B12, B22, B12);                    // 6  T3
        ip(C22, B12, X, a, lev - 1, d + 1);    // 7  P7 = S3 T3
        depth_ = d;
        sub(B12, B22, C12);                    // 8  T2
        ip(C21, C12, C22, a, lev - 1, d + 1);  // 9  P5 = S1 T1
        depth_ = d;
        sub(C12, B12, B21);                    // 10 T4
        ovr(B11, B12, C21, a, lev - 1, d + 1); // 11 P6 = S2 T2
        ovr(A22, C12, B12, a, lev - 1, d + 1); // 12 P4 = A22 T4
        depth_ = d;
        sub(B11, A12, B11);                    // 13 S4
        add(C21, C11, C21);                    // 14 U2 = P1 + P6
        add(C12, C21, C22);                    // 15 U4 = U2 + P5
        add(C21, C21, X);                      // 16 U3 = U2 + P7
        add(C22, C21, C22);                    // 17 U7 = U3 + P5
        sub(C21, C21, B12);                    // 18 U6 = U3 - P4
        ip(B11, B22, B12, a, lev - 1, d + 1);  // 19 P3 = S4 B22
        depth_ = d;
        add(C12, C12, B12);                    // 20 U5 = U4 + P3
        ovr(A12, B21, B12, a, lev - 1, d + 1); // 21 P2
        depth_ = d;
        add(C11, C11, B12);                    // 22 U1 = P1 + P2
        release(f);
    }

    // ---- Table 6: C <- a*A*B + b*C, two temporaries; overwrites A and B.
    // Rows in table order (left column 1-12, right column 13-24).
    void aclr(View A, View B, View C, int64_t a, int64_t b, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, b);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const int64_t h = C.rows / 2;
        Frame f = frame(d, {{h, h}, {h, h}});
        const View X = f.v[0], Y = f.v[1];
        sub(C22, C22, C12);                           // 1  Z1
        add(X, A21, A22);                             // 2  S1
        sub(Y, B12, B11);                             // 3  T1
        sub(C21, C21, C22);                           // 4  Z2 = C21 - Z1
        sub(B12, B22, B12);                           // 5  T3
        sub(A21, A11, A21);                           // 6  S3
        aclr(A21, B12, C22, a, b, lev - 1, d + 1);    // 7  P7 + b Z1
        depth_ = d;
        sub(A21, X, A11);                             // 8  S2 = S1 - A11
        sub(B12, B22, Y);                             // 9  T2 = B22 - T1
        aclr(X, Y, C12, a, b, lev - 1, d + 1);        // 10 P5 + b C12
        ip(A11, B11, Y, a, lev - 1, d + 1);           // 11 P1
        depth_ = d;
        sub(X, B12, B21);                             // 12 T4 = T2 - B21
        aclr(A22, X, C21, a, neg(b), lev - 1, d + 1); // 13 P4 - b Z2
        depth_ = d;
        sub(A22, A12, A21);                           // 14 S4 = A12 - S2
        ip(A21, B12, X, a, lev - 1, d + 1);           // 15 P6 = S2 T2
        aclr(A12, B21, C11, a, b, lev - 1, d + 1);    // 16 P2 + b C11
        depth_ = d;
        add(C11, Y, C11);                             // 17 U1 = P1 + P2
        add(X, Y, X);                                 // 18 U2 = P1 + P6
        add(C22, X, C22);                             // 19 U3 = U2 + P7
        add(X, X, C12);                               // 20 U4 = U2 + P5
        sub(C21, C22, C21);                           // 21 U6 = U3 - P4
        add(C22, C22, C12);                           // 22 U7 = U3 + P5
        ip(A22, B22, C12, a, lev - 1, d + 1);         // 23 P3 = S4 B22
        depth_ = d;
        add(C12, X, C12);                             // 24 U5 = U4 + P3
        release(f);
    }

    // ---- Table 7: C <- a*A*B + b*C, two temporaries; overwrites B only
    void accr(View A, View B, View C, int64_t a, int64_t b, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, b);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const int64_t h = C.rows / 2;
        Frame f = frame(d, {{h, h}, {h, h}});
        const View X = f.v[0], Y = f.v[1];
        sub(C22, C22, C12);                           // 1  Z1
        sub(X, B12, B11);                             // 2  T1
        sub(C21, C21, C22);                           // 3  Z2 = C21 - Z1
        sub(B12, B22, B12);                           // 4  T3
        sub(Y, A11, A21);                             // 5  S3
        accr(Y, B12, C22, a, b, lev - 1, d + 1);      // 6  P7 + b Z1
        depth_ = d;
        add(Y, A21, A22);                             // 7  S1
        sub(B12, B22, X);                             // 8  T2 = B22 - T1
        accr(Y, X, C12, a, b, lev - 1, d + 1);        // 9  P5 + b C12
        depth_ = d;
        sub(X, B12, B21);                             // 10 T4 = T2 - B21
        accr(A22, X, C21, a, neg(b), lev - 1, d + 1); // 11 P4 - b Z2
        ovr(A11, B11, X, a, lev - 1, d + 1);          // 12 P1
        accr(A12, B21, C11, a, b, lev - 1, d + 1);    // 13 P2 + b C11
        depth_ = d;
        sub(Y, Y, A11);                               // 14 S2 = S1 - A11
        ovr(Y, B12, B21, a, lev - 1, d + 1);          // 15 P6 = S2 T2
        depth_ = d;
        sub(Y, A12, Y);                               // 16 S4 = A12 - S2
        add(B21, X, B21);                             // 17 U2 = P1 + P6
        add(C22, B21, C22);                           // 18 U3 = U2 + P7
        add(B21, B21, C12);                           // 19 U4 = U2 + P5
        sub(C21, C22, C21);                           // 20 U6 = U3 - P4
        add(C11, X, C11);                             // 21 U1 = P1 + P2
        add(C22, C22, C12);                           // 22 U7 = U3 + P5
        ip(Y, B22, C12, a, lev - 1, d + 1);           // 23 P3 = S4 B22
        depth_ = d;
        add(C12, B21, C12);                           // 24 U5 = U4 + P3
        release(f);
    }

    // ---- Table 8: C <- a*A*B + b*C for any even shape, temporaries
    // X (max(m/2, k/2) x n/2: a T block, then products) and Y (m/2 x k/2: S
    // blocks); overwrites B only.  Rows 12 and 22 are Table 1 calls.
    void acr(View A, View B, View C, int64_t a, int64_t b, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, b);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const int64_t h = A.rows / 2, kk = A.cols / 2, w = B.cols / 2;
        Frame f = frame(d, {{std::max(h, kk), w}, {h, kk}});
        const View XT = block(f.v[0], 0, 0, kk, w), XP = block(f.v[0], 0, 0, h, w), Y = f.v[1];
        sub(C22, C22, C12);                           // 1  Z1
        sub(XT, B12, B11);                            // 2  T1
        sub(C21, C21, C22);                           // 3  Z2 = C21 - Z1
        sub(B12, B22, B12);                           // 4  T3
        sub(Y, A11, A21);                             // 5  S3
        acr(Y, B12, C22, a, b, lev - 1, d + 1);       // 6  P7 + b Z1
        depth_ = d;
        add(Y, A21, A22);                             // 7  S1
        sub(B12, B22, XT);                            // 8  T2 = B22 - T1
        acr(Y, XT, C12, a, b, lev - 1, d + 1);        // 9  P5 + b C12
        depth_ = d;
        sub(XT, B12, B21);                            // 10 T4 = T2 - B21
        acr(A22, XT, C21, a, neg(b), lev - 1, d + 1); // 11 P4 - b Z2
        t1(A11, B11, XP, a, lev - 1, d + 1);          // 12 P1
        acr(A12, B21, C11, a, b, lev - 1, d + 1);     // 13 P2 + b C11
        depth_ = d;
        add(C11, XP, C11);                            // 14 U1 = P1 + P2
        sub(Y, Y, A11);                               // 15 S2 = S1 - A11
        acr(Y, B12, XP, a, 1, lev - 1, d + 1);        // 16 U2 = a S2 T2 + P1
        depth_ = d;
        add(C22, XP, C22);                            // 17 U3 = U2 + P7
        sub(C21, C22, C21);                           // 18 U6 = U3 - P4
        add(C22, C22, C12);                           // 19 U7 = U3 + P5
        add(XP, XP, C12);                             // 20 U4 = U2 + P5
        sub(Y, A12, Y);                               // 21 S4 = A12 - S2
        t1(Y, B22, C12, a, lev - 1, d + 1);           // 22 P3 = S4 B22
        depth_ = d;
        add(C12, XP, C12);                            // 23 U5 = U4 + P3
        release(f);
    }

    // ---- Table 9: C <- a*A*B + b*C, two temporaries; A and B read only
    void acc(View A, View B, View C, int64_t a, int64_t b, int lev, int d) {
        if (lev == 0)
            return gemm(A, B, C, a, b);
        depth_ = d;
        const View A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
        const View B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const int64_t h = C.rows / 2;
        Frame f = frame(d, {{h, h}, {h, h}});
        const View X = f.v[0], Y = f.v[1];
        sub(C22, C22, C12);                           // 1  Z1
        sub(C12, C12, C21);                           // 2  Z3
        add(X, A21, A22);                             // 3  S1
        sub(Y, B12, B11);                             // 4  T1
        acc(X, Y, C12, a, b, lev - 1, d + 1);         // 5  P5 + b Z3
        depth_ = d;
        sub(X, X, A11);                               // 6  S2
        sub(Y, B22, Y);                               // 7  T2
        acc(X, Y, C21, a, b, lev - 1, d + 1);         // 8  P6 + b C21
        depth_ = d;
        sub(X, A12, X);                               // 9  S4
        lin(C22, {{1, C12}, {b, C22}});               // 10 W1 = P5 + b Z1
        acc(X, B22, C12, a, 1, lev - 1, d + 1);       // 11 P3 + P5
        t1(A11, B11, X, a, lev - 1, d + 1);           // 12 P1
        depth_ = d;
        add(C21, C21, X);                             // 13 U2 = P6 + P1
        acc(A12, B21, C11, a, b, lev - 1, d + 1);     // 14 P2 + b C11
        depth_ = d;
        add(C11, X, C11);                             // 15 U1 = P1 + P2
        add(C12, C21, C12);                           // 16 U5 = U2 + P3
        sub(X, A11, A21);                             // 17 S3
        sub(Y, B22, B12);                             // 18 T3
        aclr(X, Y, C21, a, 1, lev - 1, d + 1);        // 19 U3 = a S3 T3 + U2
        depth_ = d;
        add(C22, C21, C22);                           // 20 U7 = U3 + W1
        sub(Y, B12, B11);                             // 21 T1'
        sub(Y, B22, Y);                               // 22 T2'
        sub(Y, Y, B21);                               // 23 T4
        accr(A22, Y, C21, neg(a), 1, lev - 1, d + 1); // 24 U6 = U3 - a A22 T4
        release(f);
    }

    // ---- A schedule given as rows (one level; products recurse as Table 1,
    // accumulating products into this same schedule).
    void rowsched(View A, View B, View C, int64_t a, int64_t b, int lev, int d,
                  const std::vector<ws_row> &rows, int ntemps) {
        if (lev == 0)
            return gemm(A, B, C, a, b);
        depth_ = d;
        View blk[12 + WS_ROW_MAX_TEMPS];
        for (int q = 0; q < 4; ++q) {
            blk[q] = quad(C, q / 2, q % 2);
            blk[4 + q] = quad(A, q / 2, q % 2);
            blk[8 + q] = quad(B, q / 2, q % 2);
        }
        const int64_t h = C.rows / 2;
        Frame f = frame(d, std::vector<std::pair<int64_t, int64_t>>((size_t)ntemps, {h, h}));
        for (int i = 0; i < ntemps; ++i)
            blk[12 + i] = f.v[i];
        auto coef = [&](int c) -> int64_t {
            switch (c) {
            case WS_COEF_ONE: return 1;
            case WS_COEF_MINUS_ONE: return p_ - 1;
            case WS_COEF_BETA: return b % p_;
            default: return neg(b);
            }
        };
        for (const ws_row &r : rows) {
            const int64_t sa = r.sign > 0 ? a : neg(a);
            if (r.op == WS_ROW_ADD) {
                lin(blk[r.dst], {{coef(r.cx), blk[r.x]}, {coef(r.cy), blk[r.y]}});
            } else if (r.op == WS_ROW_MUL) {
                t1(blk[r.x], blk[r.y], blk[r.dst], sa, lev - 1, d + 1);
                depth_ = d;
            } else {
                rowsched(blk[r.x], blk[r.y], blk[r.dst], sa, coef(r.cs), lev - 1, d + 1, rows, ntemps);
                depth_ = d;
            }
        }
        release(f);
    }

    // ---- Algorithm 2: C <- a*A*B with no extra memory, A and B read only.
    // At depth dd < L the three quadrant products run as Table 1 (first
    // inner chunk) and Table 2 (the other chunks; Table 9 with acc_base, for
    // square chunks) of depth L - dd, with their temporaries in C22; C22 is
    // then computed the same way.  At depth L the
    // remaining corner is one classical product over the whole inner dimension.
    void ipmm(View A, View B, View C, int64_t a, int L, int dd, bool acc_base = false) {
        const int64_t s = C.rows, k = A.cols;
        if (dd == L || s < 2 || k == 0)
            return gemm(A, B, C, a, 0);
        const int64_t h = s / 2, K = std::min(h, k);
        const View C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
        const View A1 = block(A, 0, 0, h, k), A2 = block(A, h, 0, h, k);
        const View B1 = block(B, 0, 0, k, h), B2 = block(B, 0, h, k, h);
        const int lev = L - dd;
        regions_.push_back(C22);
        for (int64_t i = 0; i < k / K; ++i) {
            const View a1 = block(A1, 0, i * K, h, K), a2 = block(A2, 0, i * K, h, K);
            const View b1 = block(B1, i * K, 0, K, h), b2 = block(B2, i * K, 0, K, h);
            if (i == 0) {
                t1(a1, b1, C11, a, lev, 0);
                t1(a1, b2, C12, a, lev, 0);
                t1(a2, b1, C21, a, lev, 0);
            } else if (acc_base) {
                acc(a1, b1, C11, a, 1, lev, 0);
                acc(a1, b2, C12, a, 1, lev, 0);
                acc(a2, b1, C21, a, 1, lev, 0);
            } else {
                hl(a1, b1, C11, a, 1, lev, 0);
                hl(a1, b2, C12, a, 1, lev, 0);
                hl(a2, b1, C21, a, 1, lev, 0);
            }
        }
        regions_.pop_back();
        ipmm(A2, B2, C22, a, L, dd + 1, acc_base);
    }

    // ---- Algorithm 1, with the cutting into squares of its section:
    // C <- a*A*B with no extra memory, s = n = min(m, k, n) dividing m and k;
    // A, B, C cut into s x s squares A_ij, B_j, C_i.  With m/s >= 2: C_1 by
    // Table 1 with its temporaries in C_2, then A_11 is free space for the
    // Table 4 products C_i = A_i1 B_1 (i >= 2, overwriting A_i1) and the
    // Table 2 accumulations C_i += A_ij B_j (j >= 2).  With m = s: C by
    // Table 3 from A_1 and B_1, then C += A_j B_j by Table 6 with temporaries
    // in the freed A_1.  Temporaries in a free square are placed as in
    // Algorithm 2 (quadrants, callees in the bottom-right one).
    void ip0vmm(View A, View B, View C, int64_t a, int L) {
        const int64_t s = B.cols, m0 = A.rows / s, k0 = A.cols / s;
        auto Ab = [&](int64_t i, int64_t j) { return block(A, i * s, j * s, s, s); };
        auto Bb = [&](int64_t j) { return block(B, j * s, 0, s, s); };
        auto Cb = [&](int64_t i) { return block(C, i * s, 0, s, s); };
        if (m0 == 1) {
            ip(Ab(0, 0), Bb(0), Cb(0), a, L, 0);
            regions_.push_back(Ab(0, 0));
            for (int64_t j = 1; j < k0; ++j)
                aclr(Ab(0, j), Bb(j), Cb(0), a, 1, L, 0);
            regions_.pop_back();
            return;
        }
        regions_.push_back(Cb(1));
        t1(Ab(0, 0), Bb(0), Cb(0), a, L, 0);
        regions_.pop_back();
        regions_.push_back(Ab(0, 0));
        for (int64_t i = 1; i < m0; ++i)
            ovl(Ab(i, 0), Bb(0), Cb(i), a, L, 0);
        for (int64_t j = 1; j < k0; ++j)
            for (int64_t i = 0; i < m0; ++i)
                hl(Ab(i, j), Bb(j), Cb(i), a, 1, L, 0);
        regions_.pop_back();
    }

    // ---- Section 7.2: C <- a*A*B + b*C as a t x t grid of blocks.  Block
    // C_ij receives the t products A_il B_lj one after the other, each by one
    // accumulating call of Table 2 (or Table 9 for square blocks), the first
    // with b and the others with 1.  Every call sits at depth 0, so all of
    // them share the same workspace slots: the extra memory is that of one
    // call on an (n/t)-block.
    void blocked(bool acc_base, View A, View B, View C, int64_t a, int64_t b, int t, int L) {
        const std::vector<int64_t> rp = block_parts(A.rows, t, L), cp = block_parts(B.cols, t, L);
        std::vector<int64_t> kp = block_parts(A.cols, t, L);
        if (kp.empty())
            kp.push_back(0);   // k == 0: one empty product still scales C by b
        int64_t r0 = 0;
        for (int64_t rl : rp) {
            int64_t c0 = 0;
            for (int64_t cl : cp) {
                const View Cij = block(C, r0, c0, rl, cl);
                int64_t k0 = 0;
                for (size_t l = 0; l < kp.size(); ++l) {
                    const int64_t kl = kp[l], bl = l == 0 ? b : 1;
                    const View Ail = block(A, r0, k0, rl, kl), Blj = block(B, k0, c0, kl, cl);
                    if (acc_base)
                        peeled([&](View A0, View B0, View C0) { acc(A0, B0, C0, a, bl, L, 0); },
                               Ail, Blj, Cij, a, bl, L);
                    else
                        peeled([&](View A0, View B0, View C0) { hl(A0, B0, C0, a, bl, L, 0); },
                               Ail, Blj, Cij, a, bl, L);
                    k0 += kl;
                }
                c0 += cl;
            }
            r0 += rl;
        }
    }

    // ---- peeling: Winograd on the leading block whose dimensions are
    // multiples of 2^L, classical products for the thin remainders.
    template <typename Core>
    void peeled(Core core, View A, View B, View C, int64_t a, int64_t b, int L) {
        const int64_t m = A.rows, k = A.cols, n = B.cols, q = int64_t(1) << L;
        const int64_t m0 = m - m % q, k0 = k - k % q, n0 = n - n % q;
        if (m0 == 0 || k0 == 0 || n0 == 0)
            return gemm(A, B, C, a, b);
        core(block(A, 0, 0, m0, k0), block(B, 0, 0, k0, n0), block(C, 0, 0, m0, n0));
        depth_ = 0;
        if (k0 < k)
            gemm(block(A, 0, k0, m0, k - k0), block(B, k0, 0, k - k0, n0), block(C, 0, 0, m0, n0), a, 1);
        if (n0 < n)
            gemm(block(A, 0, 0, m0, k), block(B, 0, n0, k, n - n0), block(C, 0, n0, m0, n - n0), a, b);
        if (m0 < m)
            gemm(block(A, m0, 0, m - m0, k), B, block(C, m0, 0, m - m0, n), a, b);
    }

  private:
    int64_t p_;
    bool measure_;
    Fuser fuser_;
    std::vector<View> regions_;
    int depth_ = 0;
};

void run(Emitter &e, const PlanKey &key) {
    const View A = mkview(WS_BUF_A, 0, key.m, key.k, key.lda);
    const View B = mkview(WS_BUF_B, 0, key.k, key.n, key.ldb);
    const View C = mkview(WS_BUF_C, 0, key.m, key.n, key.ldc);
    const int64_t p = key.p;
    const int64_t a = ((key.alpha % p) + p) % p, b = ((key.beta % p) + p) % p;
    const int L = key.levels;
    if (key.m == 0 || key.n == 0)
        return;
    switch (key.table) {
    case TAB_CLASSICAL:
        e.gemm(A, B, C, a, b);
        break;
    case TAB_T1:
        e.peeled([&](View A0, View B0, View C0) { e.t1(A0, B0, C0, a, L, 0); }, A, B, C, a, 0, L);
        break;
    case TAB_HL:
        e.peeled([&](View A0, View B0, View C0) { e.hl(A0, B0, C0, a, b, L, 0); }, A, B, C, a, b, L);
        break;
    case TAB_ACC:
        e.peeled([&](View A0, View B0, View C0) { e.acc(A0, B0, C0, a, b, L, 0); }, A, B, C, a, b, L);
        break;
    case TAB_IP:
        e.ip(A, B, C, a, L, 0);
        break;
    case TAB_OVR:
        e.ovr(A, B, C, a, L, 0);
        break;
    case TAB_ACLR:
        e.aclr(A, B, C, a, b, L, 0);
        break;
    case TAB_ACCR:
        e.accr(A, B, C, a, b, L, 0);
        break;
    case TAB_OVL:
        e.ovl(A, B, C, a, L, 0);
        break;
    case TAB_ACR:
        e.acr(A, B, C, a, b, L, 0);
        break;
    case TAB_IP0VMM:
        e.ip0vmm(A, B, C, a, L);
        break;
    case TAB_IPMM:
        e.ipmm(A, B, C, a, L, 0);
        break;
    case TAB_IPMM_ACC:
        e.ipmm(A, B, C, a, L, 0, true);
        break;
    case TAB_BLOCKED_HL:
    case TAB_BLOCKED_ACC:
        e.blocked(key.table == TAB_BLOCKED_ACC, A, B, C, a, b, key.blocks, L);
        break;
    case TAB_ROWS: {
        std::vector<ws_row> rows;
        int ntemps = 0;
        if (!row_schedule(key.blocks, rows, ntemps))
            throw std::logic_error("unknown row schedule");
        e.rowsched(A, B, C, a, b, L, 0, rows, ntemps);
        break;
    }
    default:
        throw std::logic_error("unknown table");
    }
    e.finish();
}

}  // namespace

int register_rows(const ws_row *rows, int nrows, int ntemps, std::string *error) {
    auto bad = [&](const std::string &m) {
        if (error)
            *error = m;
        return 0;
    };
    if (!rows || nrows < 1 || nrows > WS_ROW_MAX_ROWS)
        return bad("a row schedule has 1 to WS_ROW_MAX_ROWS rows");
    if (ntemps < 0 || ntemps > WS_ROW_MAX_TEMPS)
        return bad("a row schedule has 0 to WS_ROW_MAX_TEMPS temporaries");
    const int nblk = 12 + ntemps;
    auto coef_ok = [](int c) { return c >= WS_COEF_ONE && c <= WS_COEF_MINUS_BETA; };
    for (int i = 0; i < nrows; ++i) {
        const ws_row &r = rows[i];
        const std::string at = " (row " + std::to_string(i) + ")";
        if (r.dst < 0 || r.dst >= nblk || r.x < 0 || r.x >= nblk || r.y < 0 || r.y >= nblk)
            return bad("block id out of range" + at);
        if (r.dst >= 4 && r.dst < 12)
            return bad("A and B are read only" + at);
        if (r.op == WS_ROW_ADD) {
            if (!coef_ok(r.cx) || !coef_ok(r.cy))
                return bad("unknown coefficient code" + at);
        } else if (r.op == WS_ROW_MUL || r.op == WS_ROW_ACC) {
            if (r.sign != 1 && r.sign != -1)
                return bad("a product's sign is +1 or -1" + at);
            if (r.dst == r.x || r.dst == r.y)
                return bad("a product cannot land on its own operand" + at);
            if (r.op == WS_ROW_ACC && !coef_ok(r.cs))
                return bad("unknown coefficient code" + at);
        } else {
            return bad("unknown row kind" + at);
        }
    }
    std::vector<ws_row> v(rows, rows + nrows);
    for (ws_row &r : v) {      // fields a row kind does not use compare equal
        if (r.op != WS_ROW_ADD)
            r.cx = r.cy = 0;
        if (r.op != WS_ROW_ACC)
            r.cs = 0;
        if (r.op == WS_ROW_ADD)
            r.sign = 0;
    }
    std::lock_guard<std::mutex> lock(g_rows_mu);
    for (size_t i = 0; i < g_row_schedules.size(); ++i) {
        const RowSchedule &s = g_row_schedules[i];
        if (s.ntemps == ntemps && s.rows.size() == v.size() &&
            std::memcmp(s.rows.data(), v.data(), v.size() * sizeof(ws_row)) == 0)
            return (int)i + 1;
    }
    if (g_row_schedules.size() >= 4096)
        return bad("too many distinct row schedules registered");
    g_row_schedules.push_back(RowSchedule{v, ntemps});
    return (int)g_row_schedules.size();
}

bool rows_registered(int id) {
    std::lock_guard<std::mutex> lock(g_rows_mu);
    return id >= 1 && id <= (int)g_row_schedules.size();
}

std::vector<int64_t> block_parts(int64_t d, int t, int L) {
    std::vector<int64_t> out;
    if (d <= 0 || t < 1)
        return out;
    if (d % t == 0)
        return std::vector<int64_t>((size_t)t, d / t);
    const int64_t q = int64_t(1) << L;
    int64_t s = (d + t - 1) / t;
    s = (s + q - 1) / q * q;
    for (int64_t r = d; r > 0; r -= s)
        out.push_back(std::min(s, r));
    return out;
}

bool ip0vmm_supported(int64_t m, int64_t k, int64_t n, int levels) {
    return n > 0 && levels >= 0 && levels < 62 && n <= m && n <= k && m % n == 0 && k % n == 0 &&
           n % (int64_t(1) << levels) == 0;
}

bool ipmm_supported(int64_t m, int64_t k, int64_t n, int levels) {
    if (m != n || levels < 0)
        return false;
    int64_t s = n;
    for (int d = 0; d < levels; ++d) {
        if (s % 2)
            return false;
        const int64_t h = s / 2, K = std::min(h, k), q = int64_t(1) << (levels - d);
        if (K == 0 || k % K || h % q || K % q)
            return false;
        s = h;
    }
    return true;
}

Resolved resolve_schedule(int schedule, int64_t m, int64_t k, int64_t n, bool beta_nonzero,
                          int levels, int blocks) {
    Resolved r;
    r.levels = levels;
    if (levels < 0 || levels > 24) {
        r.status = WS_EINVAL;
        r.error = "levels must lie in [0, 24]";
        return r;
    }
    const bool square = m == k && k == n;
    const bool divisible = levels < 62 && m % (int64_t(1) << levels) == 0;
    const bool all_divisible = divisible && k % (int64_t(1) << levels) == 0 &&
                               n % (int64_t(1) << levels) == 0;
    auto shape_error = [&](const char *what) {
        r.status = WS_ESHAPE;
        r.error = what;
    };
    switch (schedule) {
    case WS_CLASSICAL:
        r.table = TAB_CLASSICAL;
        r.levels = 0;
        break;
    case WS_TWO_TEMP:
        if (!beta_nonzero) {
            r.table = TAB_T1;
        } else {
            r.table = TAB_ACC;
            if (!square)
                shape_error("the two-temporary accumulating schedule (Table 9) needs m == k == n");
        }
        break;
    case WS_OVERWRITE:
        if (square) {
            r.table = beta_nonzero ? TAB_ACLR : TAB_IP;
            if (!divisible)
                shape_error("the square overwriting schedules (Tables 3 and 6) need n divisible by 2^levels");
        } else if (!beta_nonzero) {
            r.table = TAB_IP0VMM;
            if (!ip0vmm_supported(m, k, n, levels))
                shape_error("Algorithm 1 needs n = min(m, k, n) dividing m and k, and n divisible by 2^levels");
        } else {
            r.table = TAB_ACR;
            if (!all_divisible)
                shape_error("Table 8 needs m, k and n divisible by 2^levels");
        }
        break;
    case WS_IPMM_ACC:
        r.table = TAB_IPMM_ACC;
        if (beta_nonzero) {
            r.status = WS_ESCHEDULE;
            r.error = "Algorithm 2 computes C = alpha*A*B only (beta must be 0 mod p)";
        } else if (!ipmm_supported(m, k, n, levels) || 2 * k < n) {
            shape_error("Algorithm 2 with Table 9 needs the shapes of Algorithm 2 and k >= n/2 "
                        "(square chunks)");
        }
        break;
    case WS_ROWS:
        r.table = TAB_ROWS;
        if (!square || !divisible)
            shape_error("a row schedule needs m == k == n divisible by 2^levels");
        break;
    case WS_OVL:
        r.table = TAB_OVL;
        if (beta_nonzero) {
            r.status = WS_ESCHEDULE;
            r.error = "Table 4 computes C = alpha*A*B only (beta must be 0 mod p)";
        } else if (!square || !divisible) {
            shape_error("Table 4 needs m == k == n divisible by 2^levels");
        }
        break;
    case WS_ACR:
        r.table = TAB_ACR;
        if (!all_divisible)
            shape_error("Table 8 needs m, k and n divisible by 2^levels");
        break;
    case WS_READONLY_INPLACE:
        r.table = TAB_IPMM;
        if (beta_nonzero) {
            r.status = WS_ESCHEDULE;
            r.error = "Algorithm 2 computes C = alpha*A*B only (beta must be 0 mod p)";
        } else if (!ipmm_supported(m, k, n, levels)) {
            shape_error("Algorithm 2 needs m == n, n divisible by 2^(levels+1) and k a multiple of its chunks");
        }
        break;
    case WS_HL_THREE_TEMP:
        r.table = TAB_HL;
        break;
    case WS_OVR:
        r.table = TAB_OVR;
        if (beta_nonzero) {
            r.status = WS_ESCHEDULE;
            r.error = "Table 5 computes C = alpha*A*B only (beta must be 0 mod p)";
        } else if (!square || !divisible) {
            shape_error("Table 5 needs m == k == n divisible by 2^levels");
        }
        break;
    case WS_ACCR:
        r.table = TAB_ACCR;
        if (!square || !divisible)
            shape_error("Table 7 needs m == k == n divisible by 2^levels");
        break;
    case WS_BLOCKED:
    case WS_BLOCKED_ACC:
        r.table = schedule == WS_BLOCKED ? TAB_BLOCKED_HL : TAB_BLOCKED_ACC;
        if (blocks < 1 || blocks > 64) {
            r.status = WS_EINVAL;
            r.error = "the block count t of Section 7.2 must lie in [1, 64]";
        } else if (schedule == WS_BLOCKED_ACC && (!square || m % blocks)) {
            shape_error("blocked accumulation over Table 9 needs m == k == n divisible by t");
        }
        break;
    default:
        r.status = WS_ESCHEDULE;
        r.error = "unknown schedule";
    }
    // An empty product has nothing to schedule: m == 0 or n == 0 leaves C
    // alone and k == 0 gives C <- beta*C, which one classical base product
    // does for every schedule.
    if (r.status == WS_ESHAPE && (m == 0 || k == 0 || n == 0)) {
        r.status = WS_OK;
        r.error.clear();
        r.table = TAB_CLASSICAL;
        r.levels = 0;
    }
    return r;
}

void build_plan(const PlanKey &key, Plan &plan) {
    plan.key = key;
    plan.ops.clear();
    // Pass 1: shapes only, to size the workspace slot of every call depth.
    std::vector<OpDesc> none;
    Emitter measure(key.p, true, false, none);
    run(measure, key);
    // Pass 2: emit with final workspace offsets.
    Emitter e(key.p, false, key.fuse != 0, plan.ops);
    int64_t off = 0;
    for (int64_t need : measure.need) {
        e.base.push_back(off);
        off += need;
    }
    run(e, key);
    plan.ws_elems = off;
    plan.rows = e.rows;
    plan.element_additions = e.element_additions;
    plan.base_flops = e.base_flops;
    plan.add_ops = plan.gemm_ops = 0;
    for (const OpDesc &op : plan.ops)
        (op.kind == WS_OP_GEMM ? plan.gemm_ops : plan.add_ops) += 1;
}

int64_t workspace_elems(int table, int64_t m, int64_t k, int64_t n, int levels, int blocks) {
    PlanKey key{};
    key.m = m;
    key.k = k;
    key.n = n;
    key.p = 65521;
    key.lda = k;
    key.ldb = n;
    key.ldc = n;
    key.alpha = 1;
    key.beta = (table == TAB_HL || table == TAB_ACC || table == TAB_ACLR || table == TAB_ACCR ||
                table == TAB_ACR || table == TAB_BLOCKED_HL || table == TAB_BLOCKED_ACC)
                   ? 1
                   : 0;
    key.table = table;
    key.levels = levels;
    key.blocks = (table == TAB_BLOCKED_HL || table == TAB_BLOCKED_ACC) ? blocks : 0;
    std::vector<OpDesc> none;
    Emitter measure(key.p, true, false, none);
    run(measure, key);
    int64_t total = 0;
    for (int64_t x : measure.need)
        total += x;
    return total;
}

}  // namespace wsmul
