// Host-side problem setup for the pricer.
//
// Model (Sec. II.A): x_j = ln(S_T^j / K) is Gaussian with mean
// m_j = ln(S0_j / K) + (r - sigma_j^2 / 2) T and covariance C = T diag(sigma) R diag(sigma);
// the characteristic function of Sec. III.C is written with the maturity in its
// quadratic term.
//
// Merton jumps (the extension named in Sec. VI): with a Poisson clock of rate lambda and normal
// log-jumps J ~ N(muJ, CJ), the mean carries the compensator -lambda T (e^{muJ_j + CJ_jj/2} - 1)
// and the characteristic function the factor exp(lambda T (E[e^{i z.J}] - 1)); in the coordinates
// w = P x of a term the jumps have mean P muJ and covariance P CJ P^T.
//
// Term decomposition: (max_j e^{x_j} - 1)^+ = sum_j (e^{x_j} - 1)^+ prod_{l != j} 1{x_l < x_j}.
// Term j uses w_0 = x_j, w_l = x_l - x_j (l != j in increasing order), so that its payoff
// is a product of one-dimensional factors whose transforms are
//   (e^w - 1)^+ and (1 - e^w)^+ : 1/(iz(1+iz))  (Im z > 1, resp. Im z < 0)
//   1{w < 0}                   : 1/(iz)        (Im z < 0)
//   1{w > 0}                   : -1/(iz)       (Im z > 0).
// Put-on-max swaps the call factor's strip; call-on-min uses 1{w > 0}.
// The single-strip call on the minimum (the paper's form) is one term with w = x and the
// joint transform (-1)^(d+1) / ((1 + i sum_k z_k) prod_k (i z_k)), Im z_k > 0, sum Im z_k > 1.
//
// Grid (Sec. III.D): N midpoint nodes on [-L_k, L_k] per coordinate. Automatic choice:
// L_k = sqrt(2 tau (C_w^{-1})_kk) -- the marginal of exp(-u^T C_w u / 2) along u_k has
// variance (C_w^{-1})_kk -- and a contour distance a_k to the factor's pole with
// exp(-a_k 2 pi / eta_k) = exp(-tau), eta_k = 2 L_k / N (the aliasing period in x is
// 2 pi / eta_k). tau = ln(100 / tol) clamped to [18, 34.5]: the damping e^{alpha.w} of a
// larger shift inflates the absolute size of the summand faster than it cuts aliasing. When
// the damping exponent Phi = ln E[e^{alpha.w}] = alpha.m + alpha^T C_w alpha / 2 (plus the jump
// part lambda T (E[e^{alpha.J_w}] - 1)) exceeds 12 (coarse grids), tau is lowered by bisection on
// [2, tau] (60 halvings) until Phi <= 12.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace ttfp {

static const double TWO_PI = 6.283185307179586476925286766559;

static bool finite(double x) { return std::isfinite(x); }

static double grid_tau(double tol) { return std::min(34.5, std::max(18.0, std::log(100.0 / tol))); }

static const double PHI_MAX = 12.0;

// ln E[e^{alpha.w}] of a term: the Gaussian part and, with jumps, lambda T (E[e^{alpha.J_w}] - 1)
static double damping_exponent(const TermPlan &tp, const std::vector<double> &alpha)
{
    const int d = tp.d;
    double phi = 0.0, pj = 0.0;
    for (int a = 0; a < d; ++a) {
        phi += alpha[a] * tp.m[a];
        for (int b = 0; b < d; ++b) phi += 0.5 * alpha[a] * tp.C[(size_t)a * d + b] * alpha[b];
        if (tp.lamT > 0.0) {
            pj += alpha[a] * tp.mJ[a];
            for (int b = 0; b < d; ++b) pj += 0.5 * alpha[a] * tp.CJ[(size_t)a * d + b] * alpha[b];
        }
    }
    if (tp.lamT > 0.0) phi += tp.lamT * std::expm1(pj);
    return phi;
}

// Automatic (L, alpha) of one term for exponent tau; returns the damping exponent Phi.
static double rule_at(const TermPlan &tp, int N, double tau, const std::vector<double> &prec,
                      std::vector<double> &L, std::vector<double> &alpha)
{
    const int d = tp.d;
    L.assign(d, 0.0);
    alpha.assign(d, 0.0);
    for (int k = 0; k < d; ++k) {
        L[k] = std::sqrt(2.0 * tau * prec[k]);
        const double dist = tau * (2.0 * L[k] / N) / TWO_PI;
        if (tp.kind[k] == KIND_STRIP) alpha[k] = dist + 1.0 / d;   // sum_k dist from the joint pole too
        else alpha[k] = (tp.kind[k] == KIND_CALL && tp.sign[k] > 0) ? 1.0 + dist : tp.sign[k] * dist;
    }
    return damping_exponent(tp, alpha);
}

// Cholesky of a symmetric positive definite n x n matrix (row-major). False if not SPD.
static bool cholesky(const std::vector<double> &A, int n, std::vector<double> &Lc)
{
    Lc.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= Lc[(size_t)j * n + k] * Lc[(size_t)j * n + k];
        if (!(s > 0.0)) return false;
        double ljj = std::sqrt(s);
        Lc[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= Lc[(size_t)i * n + k] * Lc[(size_t)j * n + k];
            Lc[(size_t)i * n + j] = t / ljj;
        }
    }
    return true;
}

// Diagonal of A^{-1} from the Cholesky factor (solve L y = e_k, then ||L^{-T}..||).
static std::vector<double> inverse_diagonal(const std::vector<double> &A, int n, bool &ok)
{
    std::vector<double> Lc;
    ok = cholesky(A, n, Lc);
    std::vector<double> out(n, 0.0);
    if (!ok) return out;
    // A^{-1} = L^{-T} L^{-1};  (A^{-1})_kk = sum_i (L^{-1})_{ik}^2
    std::vector<double> Linv((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= Lc[(size_t)i * n + k] * Linv[(size_t)k * n + c];
            Linv[(size_t)i * n + c] = s / Lc[(size_t)i * n + i];
        }
    }
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += Linv[(size_t)i * n + k] * Linv[(size_t)i * n + k];
        out[k] = s;
    }
    return out;
}

int check_cross_settings(const ttfp_grid *g, std::string &err)
{
    if (!g) { err = "grid is NULL"; return TTFP_EINVAL; }
    if (g->N < 2 || g->N > 1024) { err = "N must be in [2, 1024]"; return TTFP_EINVAL; }
    if (g->max_rank < 1 || g->max_rank > TTFP_MAX_RANK) { err = "max_rank must be in [1, 64]"; return TTFP_EINVAL; }
    if (g->n_enrich < 0 || g->max_rank + g->n_enrich > TTFP_MAX_RANK + 4) {
        err = "n_enrich must be >= 0 and max_rank + n_enrich <= 68";
        return TTFP_EINVAL;
    }
    if (!(g->tol > 0.0) || !finite(g->tol)) { err = "tol must be positive"; return TTFP_EINVAL; }
    if (!finite(g->rank_tol)) { err = "rank_tol must be finite"; return TTFP_EINVAL; }
    if (g->max_sweeps < 1 || g->max_sweeps > 64) { err = "max_sweeps must be in [1, 64]"; return TTFP_EINVAL; }
    if (g->n_err_samples > (1 << 24)) { err = "n_err_samples must be at most 2^24"; return TTFP_EINVAL; }
    if (g->certify != 0 && g->certify != 1) { err = "certify must be 0 or 1"; return TTFP_EINVAL; }
    if (g->certify && g->n_err_samples < 0) { err = "certify needs the sampled error estimate (n_err_samples >= 0)"; return TTFP_EINVAL; }
    return TTFP_OK;
}

int build_plan(const ttfp_option *o, const ttfp_grid *g, OptionPlan &out, std::string &err)
{
    if (!o) { err = "option is NULL"; return TTFP_EINVAL; }
    if (!g) { err = "grid is NULL"; return TTFP_EINVAL; }
    const int d = o->d;
    if (d < 1 || d > TTFP_MAX_D) { err = "d must be in [1, 32]"; return TTFP_EINVAL; }
    if (o->payoff < 0 || o->payoff > 3) { err = "unknown payoff"; return TTFP_EINVAL; }
    if (!o->S0 || !o->sigma || !o->corr) { err = "S0, sigma and corr must be non-NULL"; return TTFP_EINVAL; }
    if (!(o->K > 0) || !(o->T > 0) || !finite(o->K) || !finite(o->T) || !finite(o->r)) {
        err = "K and T must be positive and finite, r finite";
        return TTFP_EINVAL;
    }
    if (g->N < 2 || g->N > 1024) { err = "N must be in [2, 1024]"; return TTFP_EINVAL; }
    out = OptionPlan();
    out.d = d;
    out.payoff = o->payoff;
    out.K = o->K;
    out.T = o->T;
    out.r = o->r;
    out.S0.assign(o->S0, o->S0 + d);
    out.sigma.assign(o->sigma, o->sigma + d);
    out.corr.assign(o->corr, o->corr + (size_t)d * d);
    for (int j = 0; j < d; ++j) {
        if (!(out.S0[j] > 0) || !finite(out.S0[j])) { err = "S0 must be positive"; return TTFP_EINVAL; }
        if (!(out.sigma[j] > 0) || !finite(out.sigma[j])) { err = "sigma must be positive"; return TTFP_EINVAL; }
    }
    for (int i = 0; i < d; ++i) {
        if (std::fabs(out.corr[(size_t)i * d + i] - 1.0) > 1e-12) { err = "corr must have unit diagonal"; return TTFP_EINVAL; }
        for (int j = 0; j < d; ++j) {
            double a = out.corr[(size_t)i * d + j], b = out.corr[(size_t)j * d + i];
            if (!finite(a) || std::fabs(a - b) > 1e-12) { err = "corr must be symmetric and finite"; return TTFP_EINVAL; }
        }
    }
    std::vector<double> Lc;
    if (!cholesky(out.corr, d, Lc)) { err = "corr is not positive definite"; return TTFP_EINVAL; }
    // jumps
    const double lam = o->jump_rate;
    if (!finite(lam) || lam < 0.0) { err = "jump_rate must be finite and >= 0"; return TTFP_EINVAL; }
    std::vector<double> muJ(d, 0.0), CJx((size_t)d * d, 0.0);
    if (lam > 0.0) {
        if (!o->jump_mean || !o->jump_cov) { err = "jump_mean and jump_cov must be non-NULL when jump_rate > 0"; return TTFP_EINVAL; }
        double dmax = 0.0;
        for (int i = 0; i < d; ++i) {
            muJ[i] = o->jump_mean[i];
            if (!finite(muJ[i])) { err = "jump_mean must be finite"; return TTFP_EINVAL; }
            for (int j = 0; j < d; ++j) {
                const double a = o->jump_cov[(size_t)i * d + j], b = o->jump_cov[(size_t)j * d + i];
                if (!finite(a) || std::fabs(a - b) > 1e-12 * (1.0 + std::fabs(a))) { err = "jump_cov must be symmetric and finite"; return TTFP_EINVAL; }
                CJx[(size_t)i * d + j] = a;
            }
            if (CJx[(size_t)i * d + i] < 0.0) { err = "jump_cov must have a nonnegative diagonal"; return TTFP_EINVAL; }
            dmax = std::max(dmax, CJx[(size_t)i * d + i]);
        }
        // positive semidefinite: Cholesky of CJ + 1e-12 (1 + max diag) I
        std::vector<double> Cs = CJx, Ls;
        for (int i = 0; i < d; ++i) Cs[(size_t)i * d + i] += 1e-12 * (1.0 + dmax);
        if (!cholesky(Cs, d, Ls)) { err = "jump_cov is not positive semidefinite"; return TTFP_EINVAL; }
    }

    // log-moneyness moments
    std::vector<double> mx(d), Cx((size_t)d * d);
    for (int j = 0; j < d; ++j) {
        mx[j] = std::log(out.S0[j] / out.K) + (out.r - 0.5 * out.sigma[j] * out.sigma[j]) * out.T;
        if (lam > 0.0) mx[j] -= lam * out.T * std::expm1(muJ[j] + 0.5 * CJx[(size_t)j * d + j]);   // compensator
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            Cx[(size_t)i * d + j] = out.T * out.sigma[i] * out.sigma[j] * out.corr[(size_t)i * d + j];

    const bool strip = o->payoff == TTFP_CALL_MIN_STRIP;
    const int n_terms = strip ? 1 : d;   // d == 1 gives one term as well
    const int N = g->N;
    const double tau = grid_tau(g->tol > 0 ? g->tol : 1e-12);
    for (int t = 0; t < n_terms; ++t) {
        TermPlan tp;
        tp.d = d;
        tp.N = N;
        tp.P.assign((size_t)d * d, 0.0);
        if (strip) {
            for (int l = 0; l < d; ++l) tp.P[(size_t)l * d + l] = 1.0;
        } else {
            tp.P[(size_t)0 * d + t] = 1.0;
            int row = 1;
            for (int l = 0; l < d; ++l) {
                if (l == t) continue;
                tp.P[(size_t)row * d + l] = 1.0;
                tp.P[(size_t)row * d + t] = -1.0;
                ++row;
            }
        }
        tp.m.assign(d, 0.0);
        tp.C.assign((size_t)d * d, 0.0);
        for (int a = 0; a < d; ++a)
            for (int k = 0; k < d; ++k) tp.m[a] += tp.P[(size_t)a * d + k] * mx[k];
        std::vector<double> PC((size_t)d * d, 0.0);
        for (int a = 0; a < d; ++a)
            for (int k = 0; k < d; ++k) {
                double s = 0.0;
                for (int l = 0; l < d; ++l) s += tp.P[(size_t)a * d + l] * Cx[(size_t)l * d + k];
                PC[(size_t)a * d + k] = s;
            }
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                double s = 0.0;
                for (int k = 0; k < d; ++k) s += PC[(size_t)a * d + k] * tp.P[(size_t)b * d + k];
                tp.C[(size_t)a * d + b] = s;
            }
        // jumps in the term's coordinates
        tp.lamT = lam * out.T;
        tp.mJ.assign(d, 0.0);
        tp.CJ.assign((size_t)d * d, 0.0);
        if (lam > 0.0) {
            std::vector<double> PJ((size_t)d * d, 0.0);
            for (int a = 0; a < d; ++a)
                for (int k = 0; k < d; ++k) {
                    tp.mJ[a] += tp.P[(size_t)a * d + k] * muJ[k];
                    double s = 0.0;
                    for (int l = 0; l < d; ++l) s += tp.P[(size_t)a * d + l] * CJx[(size_t)l * d + k];
                    PJ[(size_t)a * d + k] = s;
                }
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    double s = 0.0;
                    for (int k = 0; k < d; ++k) s += PJ[(size_t)a * d + k] * tp.P[(size_t)b * d + k];
                    tp.CJ[(size_t)a * d + b] = s;
                }
        }
        tp.kind.assign(d, KIND_CALL);
        tp.sign.assign(d, 1);
        if (strip) {
            tp.kind.assign(d, KIND_STRIP);
        } else {
            tp.sign[0] = (o->payoff == TTFP_PUT_MAX) ? -1 : 1;
            for (int k = 1; k < d; ++k) {
                tp.kind[k] = (o->payoff == TTFP_CALL_MIN) ? KIND_GT : KIND_LT;
                tp.sign[k] = (o->payoff == TTFP_CALL_MIN) ? 1 : -1;
            }
        }
        // ---- grid
        bool ok = true;
        std::vector<double> prec = inverse_diagonal(tp.C, d, ok);
        if (!ok) { err = "term covariance is not positive definite"; return TTFP_EINVAL; }
        tp.L.assign(d, 0.0);
        tp.alpha.assign(d, 0.0);
        std::vector<double> Lauto, Aauto;
        if (!g->L_k && !(g->L > 0)) {
            double tu = tau;
            if (rule_at(tp, N, tu, prec, Lauto, Aauto) > PHI_MAX) {
                double lo = 2.0, hi = tau;
                for (int itb = 0; itb < 60; ++itb) {
                    const double mid = 0.5 * (lo + hi);
                    if (rule_at(tp, N, mid, prec, Lauto, Aauto) <= PHI_MAX) lo = mid;
                    else hi = mid;
                }
                tu = lo;
                rule_at(tp, N, tu, prec, Lauto, Aauto);
            }
        }
        for (int k = 0; k < d; ++k) {
            double L;
            if (g->L_k) L = g->L_k[(size_t)t * d + k];
            else if (g->L > 0) L = g->L;
            else L = Lauto[k];
            if (!(L > 0) || !finite(L)) { err = "L must be positive"; return TTFP_EINVAL; }
            tp.L[k] = L;
            double a;
            if (g->alpha_k) {
                a = g->alpha_k[(size_t)t * d + k];
            } else if (g->alpha > 0) {
                a = tp.sign[k] * g->alpha;
            } else if (!Aauto.empty()) {
                a = Aauto[k];
            } else {
                double eta = 2.0 * L / N;
                double dist = tau * eta / TWO_PI;
                if (tp.kind[k] == KIND_STRIP) a = dist + 1.0 / d;
                else a = (tp.kind[k] == KIND_CALL && tp.sign[k] > 0) ? 1.0 + dist : tp.sign[k] * dist;
            }
            // strip check
            bool inside;
            if (tp.kind[k] == KIND_CALL) inside = (tp.sign[k] > 0) ? (a > 1.0) : (a < 0.0);
            else inside = (tp.sign[k] > 0) ? (a > 0.0) : (a < 0.0);
            if (!inside || !finite(a)) {
                char buf[160];
                std::snprintf(buf, sizeof buf, "contour shift %g outside the strip of coordinate %d of term %d", a, k, t);
                err = buf;
                return TTFP_EINVAL;
            }
            tp.alpha[k] = a;
        }
        if (strip) {
            double sa = 0.0;
            for (int k = 0; k < d; ++k) sa += tp.alpha[k];
            if (!(sa > 1.0)) {
                char buf[160];
                std::snprintf(buf, sizeof buf, "contour shifts sum to %g: the single-strip transform needs more than 1", sa);
                err = buf;
                return TTFP_EINVAL;
            }
        }
        double sc = out.K * std::exp(-out.r * out.T);
        for (int k = 0; k < d; ++k) sc *= (2.0 * tp.L[k] / N) / TWO_PI;
        tp.scale = sc;
        // Absolute size of the sum, by the Gaussian peak approximation:
        // sum |integrand| ~ E[e^{alpha.w}] prod_k |h_k(i alpha_k)|
        //                  x (2 pi)^{d/2} det(C)^{-1/2} / prod_k eta_k;
        // divided by the price it estimates the cancellation factor of the quadrature.
        const double expo = damping_exponent(tp, tp.alpha);
        std::vector<double> Lw;
        cholesky(tp.C, d, Lw);
        double logdet = 0.0;
        for (int k = 0; k < d; ++k) logdet += 2.0 * std::log(Lw[(size_t)k * d + k]);
        double lmass = expo + 0.5 * d * std::log(TWO_PI) - 0.5 * logdet;
        double asum = 0.0;
        for (int k = 0; k < d; ++k) {
            const double v = tp.alpha[k];
            asum += v;
            double h = 1.0 / std::fabs(v);                       // |1/(i z)| at z = i v
            if (tp.kind[k] == KIND_CALL) h /= std::fabs(1.0 - v);   // |1/(1 + i z)|
            lmass += std::log(h) - std::log(2.0 * tp.L[k] / N);
        }
        if (strip) lmass -= std::log(std::fabs(1.0 - asum));      // |1/(1 + i sum z)| at z = i alpha
        double mass = std::exp(std::min(lmass, 700.0));
        tp.absmass = sc * mass;
        out.terms.push_back(std::move(tp));
    }
    return TTFP_OK;
}

}  // namespace ttfp
