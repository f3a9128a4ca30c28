// Chain-order planner (host only).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace atp {

// Estimated shape of a (sub)chain product.
struct ChainStats {
    double rows = 0;   // non-empty rows
    double cols = 0;   // non-empty columns
    double nnz = 0;
    double dim_r = 0;  // full dimensions
    double dim_c = 0;
};

// Joint degree sketch of a junction node type between relation k (into the
// type) and relation k+1 (out of it): nodes grouped by (log2 in-degree,
// log2 out-degree) with their count and mean degrees.
struct JunctionSketch {
    struct Bucket {
        double n, in, out;
    };
    std::vector<Bucket> buckets;
    double sum_in = 0, sum_out = 0;  // over all nodes of the type
};

// Column popularity of a relation: its columns grouped by log2 in-degree.
struct ColumnHist {
    struct Bucket {
        double n, deg;
    };
    std::vector<Bucket> buckets;
    double total = 0;  // sum of in-degrees
};

// Default coefficients, in units of one product: a left-operand entry costs a
// segment set-up (its right row's bounds, a scan slot) worth about a dozen
// products, a product is mostly an L2-resident gather and one LDS add, a
// result entry is written and compacted.  Eq. 2 fitted on timed
// multiplications of random walks puts alpha / beta at about 15 on the
// scholarly network (beta near 0 on the news network).
struct CostCoeffs {
    double alpha = 12.0;   // per nonzero of the left operand
    double beta = 1.0;     // per product (N_op)
    double gamma = 2.0;    // per nonzero of the result
    double delta = 2.0e5;  // fixed cost of one product (launches and synchronisation)
};

enum class Estimator { Uniform, Sketch };

struct PlanResult {
    std::string plan;
    double cost = 0;
    std::vector<ChainStats> node_stats;  // estimate of the root and every product, post-order
    std::vector<std::vector<double>> span_nnz;  // [i][j]: estimated nnz of the product of leaves i..j
};

// Dynamic program of Eq. 1 over p = leaves.size() matrices.  junctions[k]
// (k < p-1) describes the node type between leaf k and k+1, and
// junction_sel[k] the fraction of its nodes kept by that position's mask.
// col_hists[i] / col_sel[i] describe the columns of leaf i (used by Sketch to
// estimate how many distinct cells the products of a product hit).
// cached[i][j] (optional, p x p): the product of leaves i..j is available at
// no cost with the given shape (Sec. 3.2: a cached result costs only its
// retrieval); such a block appears in the plan string as "[i-j]".
PlanResult plan_chain(const std::vector<ChainStats> &leaves, const std::vector<JunctionSketch> &junctions,
                      const std::vector<double> &junction_sel, const std::vector<ColumnHist> &col_hists,
                      const std::vector<double> &col_sel, Estimator est, const CostCoeffs &cc,
                      const std::vector<std::vector<const ChainStats *>> *cached = nullptr);

// Product estimate for X * Y meeting at a junction; ycols describes the
// columns of Y's last relation (exposed for tests).
ChainStats estimate_product(const ChainStats &x, const ChainStats &y, const JunctionSketch *junction, double sel,
                            const ColumnHist *ycols, double ycol_sel, Estimator est, double *n_op);

ColumnHist make_column_hist(const int32_t *in_deg, int64_t n);

// The paper's E_ac density estimate: 1 - (1 - rx*ry)^k, computed stably.
double eac_density(double rx, double ry, double k);

// Build a junction sketch from per-node in-degrees and out-degrees.
JunctionSketch make_sketch(const int32_t *in_deg, const int64_t *out_row_ptr, int64_t n);

// Plan strings: "3" for a single leaf, "(L,R)" for a product.
struct PlanTree {
    int leaf = -1;
    int left = -1, right = -1;  // node indices
    int block_lo = -1, block_hi = -1;  // a cached block of leaves (plan token "[lo-hi]")
};
bool parse_plan(const char *s, int p, std::vector<PlanTree> &nodes, int &root);

// Least-squares fit of Eq. 2's coefficients (plus the per-product constant
// delta) to measured multiplications: t ~ alpha*nnz(X) + beta*N_op +
// gamma*nnz(Z) + delta, every coefficient >= 0 (a coefficient that comes out
// negative is fixed at 0 and the rest refit).  Returns R^2 of the fit.
double fit_cost(const std::vector<double> &nnz_x, const std::vector<double> &n_op, const std::vector<double> &nnz_z,
                const std::vector<double> &t, CostCoeffs &out);

}  // namespace atp
