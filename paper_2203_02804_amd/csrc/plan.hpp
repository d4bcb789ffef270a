// Host-side problem setup: validation, per-asset term decomposition and grid choice.
#pragma once
#include <string>
#include <vector>

#include "ttfp.h"

namespace ttfp {

// KIND_STRIP: coordinate of the single-strip call on the minimum (factor 1/(i z_k), times the
// joint factor (-1)^(d+1) / (1 + i sum_k z_k) that every coordinate of that term shares);
// KIND_ONE: no payoff factor (the characteristic function's own train in the two-train variant)
enum FactorKind { KIND_CALL = 0, KIND_LT = 1, KIND_GT = 2, KIND_STRIP = 3, KIND_ONE = 4 };

// One separable term of an option: the Gaussian of w = P x and one payoff factor per
// coordinate, on the grid u_k(i) = -L_k + (i + 1/2) 2 L_k / N shifted by i alpha_k.
struct TermPlan {
    int d = 0, N = 0;
    std::vector<double> P;      // rotation, d x d row-major (w = P x)
    std::vector<double> m;      // mean of w
    std::vector<double> C;      // covariance of w, d x d row-major
    std::vector<double> L;      // half-widths
    std::vector<double> alpha;  // signed contour shifts
    std::vector<int> kind;      // payoff factor per coordinate
    std::vector<int> sign;      // +1 strip above the real axis, -1 below
    std::vector<double> mJ;     // Merton jumps: mean of the log-jump sizes in w coordinates
    std::vector<double> CJ;     // their covariance in w coordinates, d x d row-major
    double lamT = 0.0;          // jump rate times maturity (0: no jumps)
    double scale = 0.0;         // K e^{-rT} prod_k eta_k / (2 pi)
    double absmass = 0.0;       // estimate of scale * sum |integrand| over the grid
};

struct OptionPlan {
    int d = 0, payoff = 0;
    std::vector<double> S0, sigma, corr;
    double K = 0, T = 0, r = 0;
    std::vector<TermPlan> terms;
};

// Validates and builds the plan. Returns TTFP_OK or TTFP_EINVAL with a message.
int build_plan(const ttfp_option *opt, const ttfp_grid *grid, OptionPlan &out, std::string &err);

// Validates the TT-cross part of a grid (ranks, sweeps, tolerances).
int check_cross_settings(const ttfp_grid *grid, std::string &err);

}  // namespace ttfp
