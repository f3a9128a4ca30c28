// Chain-order planner: the dynamic program of Sec. 3.1 (Eq. 1) over the
// sparse product cost of Sec. 3.2 (Eq. 2),
//     c(X*Y) = alpha*nnz(X) + beta*N_op + gamma*nnz(Z)  (+ delta per product),
// with two estimators for N_op and nnz(Z):
//   Uniform  the paper's average-case E_ac: nonzeros spread uniformly, so
//            N_op = nnz(X)*nnz(Y)/k and rho_Z = 1 - (1 - rho_X*rho_Y)^k;
//   Sketch   degree-aware: the columns of X follow the in-degree of the
//            junction type under the last relation of X, the rows of Y follow
//            the out-degree under the first relation of Y (joint log2 buckets
//            of both degrees), each capped by the other operand's extent.
//            The result's nonzeros are the distinct cells hit when each row's
//            products fall on columns with probability proportional to their
//            in-degree under Y's last relation (log2 buckets): a column of
//            weight w is hit with probability 1 - exp(-n w) by n products.
//            This is exact for N_op when X and Y are single relations and
//            catches the hub rows and hub columns that the uniform estimate
//            misses.
// The order never changes the result (associativity), only its cost.
#include "planner.hpp"

#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <map>

namespace atp {

double eac_density(double rx, double ry, double k) {
    double r = rx * ry;
    if (r <= 0 || k <= 0) return 0.0;
    if (r >= 1) return 1.0;
    double d = -std::expm1(k * std::log1p(-r));
    return d < 0 ? 0 : (d > 1 ? 1 : d);
}

static double sat_fill(double n_op, double cells) {
    // expected occupied cells after n_op uniform throws into `cells` cells
    if (cells <= 0 || n_op <= 0) return 0;
    return cells * -std::expm1(-n_op / cells);
}

// expected distinct columns hit by n products spread by column popularity
static double fill_columns(const ColumnHist &h, double sel, double n) {
    if (h.total <= 0 || n <= 0 || sel <= 0) return 0;
    double s = 0;
    for (const auto &b : h.buckets) s += b.n * sel * -std::expm1(-n * b.deg / (h.total * sel));
    return s;
}

ColumnHist make_column_hist(const int32_t *in_deg, int64_t n) {
    ColumnHist h;
    std::map<int, ColumnHist::Bucket> acc;
    for (int64_t b = 0; b < n; ++b) {
        const int64_t d = in_deg[b];
        if (d <= 0) continue;
        int lg = 0;
        while ((d >> lg) > 1) ++lg;
        auto &bk = acc[lg];
        bk.n += 1;
        bk.deg += (double)d;
        h.total += (double)d;
    }
    for (auto &kv : acc) h.buckets.push_back({kv.second.n, kv.second.deg / kv.second.n});
    return h;
}

ChainStats estimate_product(const ChainStats &x, const ChainStats &y, const JunctionSketch *j, double sel,
                            const ColumnHist *ycols, double ycol_sel, Estimator est, double *n_op_out) {
    ChainStats z;
    z.dim_r = x.dim_r;
    z.dim_c = y.dim_c;
    double n_op;
    const bool uniform = est == Estimator::Uniform || j == nullptr || j->sum_in <= 0 || j->sum_out <= 0;
    if (uniform) {
        const double k = x.dim_c;
        const double rx = (x.dim_r * k) > 0 ? x.nnz / (x.dim_r * k) : 0;
        const double ry = (k * y.dim_c) > 0 ? y.nnz / (k * y.dim_c) : 0;
        n_op = k > 0 ? x.nnz * y.nnz / k : 0;
        const double rz = eac_density(rx, ry, k);
        z.nnz = x.dim_r * y.dim_c * rz;
        z.rows = x.rows;
        z.cols = y.cols;
        if (n_op_out) *n_op_out = n_op;
        return z;
    }
    {
        const double sin = j->sum_in * sel, sout = j->sum_out * sel;
        const double ax = sin > 0 ? x.nnz / sin : 0;
        const double ay = sout > 0 ? y.nnz / sout : 0;
        double s = 0;
        for (const auto &b : j->buckets) {
            double cx = std::min(ax * b.in, x.rows);
            double ry = std::min(ay * b.out, y.cols);
            s += b.n * cx * ry;
        }
        n_op = s * sel;
        z.rows = x.rows * -std::expm1(-(x.rows > 0 ? n_op / x.rows : 0));
        if (ycols && ycols->total > 0) {
            const double per_row = z.rows > 0 ? n_op / z.rows : 0;
            z.nnz = std::min(n_op, z.rows * fill_columns(*ycols, ycol_sel, per_row));
            z.cols = std::min(y.cols, fill_columns(*ycols, ycol_sel, n_op));
        } else {
            z.cols = y.cols * -std::expm1(-(y.cols > 0 ? n_op / y.cols : 0));
            z.nnz = std::min(n_op, sat_fill(n_op, z.rows * z.cols));
        }
    }
    if (n_op_out) *n_op_out = n_op;
    return z;
}

PlanResult plan_chain(const std::vector<ChainStats> &leaves, const std::vector<JunctionSketch> &junctions,
                      const std::vector<double> &junction_sel, const std::vector<ColumnHist> &col_hists,
                      const std::vector<double> &col_sel, Estimator est, const CostCoeffs &cc,
                      const std::vector<std::vector<const ChainStats *>> *cached) {
    const int p = (int)leaves.size();
    PlanResult out;
    if (p == 0) return out;
    std::vector<std::vector<double>> C(p, std::vector<double>(p, 0.0));
    std::vector<std::vector<int>> S(p, std::vector<int>(p, -1));
    std::vector<std::vector<ChainStats>> D(p, std::vector<ChainStats>(p));
    for (int i = 0; i < p; ++i) D[i][i] = leaves[i];
    for (int len = 2; len <= p; ++len) {
        for (int i = 0; i + len - 1 < p; ++i) {
            const int j = i + len - 1;
            if (cached && (*cached)[i][j]) {  // retrieved, not computed
                C[i][j] = 0;
                S[i][j] = -2;
                D[i][j] = *(*cached)[i][j];
                continue;
            }
            double best = std::numeric_limits<double>::infinity();
            for (int k = i; k < j; ++k) {
                const JunctionSketch *js = k < (int)junctions.size() ? &junctions[k] : nullptr;
                const double sel = k < (int)junction_sel.size() ? junction_sel[k] : 1.0;
                double n_op = 0;
                const ColumnHist *yc = j < (int)col_hists.size() ? &col_hists[j] : nullptr;
                const double ycs = j < (int)col_sel.size() ? col_sel[j] : 1.0;
                ChainStats z = estimate_product(D[i][k], D[k + 1][j], js, sel, yc, ycs, est, &n_op);
                double c = C[i][k] + C[k + 1][j] + cc.alpha * D[i][k].nnz + cc.beta * n_op + cc.gamma * z.nnz +
                           cc.delta;
                if (c < best) {  // strict: ties keep the smallest split
                    best = c;
                    S[i][j] = k;
                    D[i][j] = z;
                }
            }
            C[i][j] = best;
        }
    }
    std::function<std::string(int, int)> str = [&](int i, int j) -> std::string {
        if (i == j) {
            out.node_stats.push_back(D[i][i]);
            return std::to_string(i);
        }
        const int k = S[i][j];
        if (k == -2) {
            out.node_stats.push_back(D[i][j]);
            return "[" + std::to_string(i) + "-" + std::to_string(j) + "]";
        }
        std::string l = str(i, k), r = str(k + 1, j);
        out.node_stats.push_back(D[i][j]);
        return "(" + l + "," + r + ")";
    };
    out.plan = str(0, p - 1);
    out.cost = C[0][p - 1];
    out.span_nnz.assign(p, std::vector<double>(p, 0.0));
    for (int i = 0; i < p; ++i)
        for (int j = i; j < p; ++j) out.span_nnz[i][j] = D[i][j].nnz;
    return out;
}

JunctionSketch make_sketch(const int32_t *in_deg, const int64_t *out_row_ptr, int64_t n) {
    JunctionSketch js;
    std::map<int, JunctionSketch::Bucket> acc;
    auto lg = [](int64_t d) {
        int b = 0;
        while ((d >> b) > 1) ++b;
        return d > 0 ? b + 1 : 0;
    };
    for (int64_t b = 0; b < n; ++b) {
        const int64_t di = in_deg[b];
        const int64_t dout = out_row_ptr[b + 1] - out_row_ptr[b];
        js.sum_in += (double)di;
        js.sum_out += (double)dout;
        if (di == 0 || dout == 0) continue;
        auto &bk = acc[lg(di) * 64 + lg(dout)];
        bk.n += 1;
        bk.in += (double)di;
        bk.out += (double)dout;
    }
    for (auto &kv : acc) {
        auto b = kv.second;
        b.in /= b.n;
        b.out /= b.n;
        js.buckets.push_back(b);
    }
    return js;
}

// ---- plan strings ----------------------------------------------------------

namespace {
struct Parser {
    const char *s;
    size_t pos = 0;
    int p;
    int next_leaf = 0;
    std::vector<PlanTree> &nodes;
    bool ok = true;
    Parser(const char *str, int p_, std::vector<PlanTree> &n) : s(str), p(p_), nodes(n) {}
    void ws() {
        while (s[pos] == ' ' || s[pos] == '\t' || s[pos] == '\n') ++pos;
    }
    long read_num() {
        if (!(s[pos] >= '0' && s[pos] <= '9')) {
            ok = false;
            return -1;
        }
        long v = 0;
        while (s[pos] >= '0' && s[pos] <= '9') {
            v = v * 10 + (s[pos] - '0');
            if (v > 1000000) {
                ok = false;
                return -1;
            }
            ++pos;
        }
        return v;
    }
    int node() {
        ws();
        if (s[pos] == '(') {
            ++pos;
            int l = node();
            ws();
            if (!ok || s[pos] != ',') {
                ok = false;
                return -1;
            }
            ++pos;
            int r = node();
            ws();
            if (!ok || s[pos] != ')') {
                ok = false;
                return -1;
            }
            ++pos;
            PlanTree t;
            t.left = l;
            t.right = r;
            nodes.push_back(t);
            return (int)nodes.size() - 1;
        }
        if (s[pos] == '[') {
            ++pos;
            long lo = read_num(), hi;
            if (!ok || s[pos] != '-') {
                ok = false;
                return -1;
            }
            ++pos;
            hi = read_num();
            if (!ok || s[pos] != ']' || lo != next_leaf || hi < lo || hi >= p) {
                ok = false;
                return -1;
            }
            ++pos;
            next_leaf = (int)hi + 1;
            PlanTree t;
            t.block_lo = (int)lo;
            t.block_hi = (int)hi;
            nodes.push_back(t);
            return (int)nodes.size() - 1;
        }
        if (s[pos] >= '0' && s[pos] <= '9') {
            long v = 0;
            while (s[pos] >= '0' && s[pos] <= '9') {
                v = v * 10 + (s[pos] - '0');
                if (v > 1000000) {
                    ok = false;
                    return -1;
                }
                ++pos;
            }
            if (v != next_leaf || v >= p) {  // leaves must appear once each, in chain order
                ok = false;
                return -1;
            }
            ++next_leaf;
            PlanTree t;
            t.leaf = (int)v;
            nodes.push_back(t);
            return (int)nodes.size() - 1;
        }
        ok = false;
        return -1;
    }
};
}  // namespace

bool parse_plan(const char *s, int p, std::vector<PlanTree> &nodes, int &root) {
    nodes.clear();
    if (!s) return false;
    Parser ps(s, p, nodes);
    root = ps.node();
    ps.ws();
    return ps.ok && s[ps.pos] == '\0' && ps.next_leaf == p;
}

double fit_cost(const std::vector<double> &nnz_x, const std::vector<double> &n_op, const std::vector<double> &nnz_z,
                const std::vector<double> &t, CostCoeffs &out) {
    const size_t n = t.size();
    constexpr int K = 4;
    bool active[K] = {true, true, true, true};
    double coef[K] = {0, 0, 0, 0};
    auto feat = [&](size_t i, int k) {
        return k == 0 ? nnz_x[i] : k == 1 ? n_op[i] : k == 2 ? nnz_z[i] : 1.0;
    };
    for (int round = 0; round < K; ++round) {
        std::vector<int> idx;
        for (int k = 0; k < K; ++k)
            if (active[k]) idx.push_back(k);
        const int m = (int)idx.size();
        if (m == 0 || n == 0) break;
        // normal equations over the active features, columns scaled to unit norm
        std::vector<double> scale(m, 0.0);
        for (int a = 0; a < m; ++a) {
            for (size_t i = 0; i < n; ++i) scale[a] += feat(i, idx[a]) * feat(i, idx[a]);
            scale[a] = scale[a] > 0 ? std::sqrt(scale[a]) : 1.0;
        }
        std::vector<double> A(m * (m + 1), 0.0);
        for (size_t i = 0; i < n; ++i)
            for (int a = 0; a < m; ++a) {
                const double fa = feat(i, idx[a]) / scale[a];
                for (int b = 0; b < m; ++b) A[a * (m + 1) + b] += fa * feat(i, idx[b]) / scale[b];
                A[a * (m + 1) + m] += fa * t[i];
            }
        for (int a = 0; a < m; ++a) A[a * (m + 1) + a] += 1e-12;  // keeps a rank-deficient system solvable
        for (int col = 0; col < m; ++col) {  // Gauss-Jordan with partial pivoting
            int piv = col;
            for (int r = col + 1; r < m; ++r)
                if (std::fabs(A[r * (m + 1) + col]) > std::fabs(A[piv * (m + 1) + col])) piv = r;
            for (int q = 0; q <= m; ++q) std::swap(A[col * (m + 1) + q], A[piv * (m + 1) + q]);
            const double d = A[col * (m + 1) + col];
            if (std::fabs(d) < 1e-300) continue;
            for (int q = 0; q <= m; ++q) A[col * (m + 1) + q] /= d;
            for (int r = 0; r < m; ++r) {
                if (r == col) continue;
                const double f = A[r * (m + 1) + col];
                for (int q = 0; q <= m; ++q) A[r * (m + 1) + q] -= f * A[col * (m + 1) + q];
            }
        }
        int worst = -1;
        double wv = 0;
        for (int k = 0; k < K; ++k) coef[k] = 0;
        for (int a = 0; a < m; ++a) {
            coef[idx[a]] = A[a * (m + 1) + m] / scale[a];
            if (coef[idx[a]] < wv) {
                wv = coef[idx[a]];
                worst = idx[a];
            }
        }
        if (worst < 0) break;
        active[worst] = false;
        coef[worst] = 0;
    }
    for (int k = 0; k < K; ++k)
        if (coef[k] < 0) coef[k] = 0;
    out.alpha = coef[0];
    out.beta = coef[1];
    out.gamma = coef[2];
    out.delta = coef[3];
    double mean = 0, ss_tot = 0, ss_res = 0;
    for (size_t i = 0; i < n; ++i) mean += t[i];
    mean = n ? mean / n : 0;
    for (size_t i = 0; i < n; ++i) {
        double pred = 0;
        for (int k = 0; k < K; ++k) pred += coef[k] * feat(i, k);
        ss_res += (t[i] - pred) * (t[i] - pred);
        ss_tot += (t[i] - mean) * (t[i] - mean);
    }
    return ss_tot > 0 ? 1.0 - ss_res / ss_tot : 1.0;
}

}  // namespace atp
