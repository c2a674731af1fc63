// Host planner: Leja points of [-2, 2], scalar phi_l and Newton divided
// differences (Sec. 1 and Sec. 2.1 of arXiv 2310.08344).  Plain C++, no HIP.
#include "planner.h"

#include "dd_math.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <mutex>
#include <vector>

namespace lx {

// ---------------------------------------------------------------------------
// phi_l(z), z real (Sec. 1).  For |z| < max(1.5, l) the removable
// singularity of the recursion is avoided by the Taylor series
// sum_k z^k/(k+l)!, whose terms then decrease monotonically (40 terms,
// relative truncation < 1e-20); otherwise phi_0 = exp(z), phi_1 = expm1(z)/z
// and the recursion phi_{k+1} = (phi_k - 1/k!)/z.
// ---------------------------------------------------------------------------
double phi_scalar(int l, double z) {
    if (l < 0) return std::numeric_limits<double>::quiet_NaN();
    double fact_l = 1.0;
    for (int k = 2; k <= l; ++k) fact_l *= k;
    if (z == 0.0) return 1.0 / fact_l;
    if (std::fabs(z) < std::max(1.5, static_cast<double>(l))) {
        // coefficients 1/(k+l)! for k = 0..40, summed by Horner from the tail
        constexpr int kTerms = 40;
        double coef[kTerms + 1];
        double f = fact_l;
        for (int k = 0; k <= kTerms; ++k) {
            if (k > 0) f *= static_cast<double>(k + l);
            coef[k] = 1.0 / f;
        }
        double acc = 0.0;
        for (int k = kTerms; k >= 0; --k) acc = acc * z + coef[k];
        return acc;
    }
    if (l == 0) return std::exp(z);
    double val = std::expm1(z) / z;          // phi_1
    double inv_fact = 1.0;                   // 1/k! for k = 1
    for (int k = 1; k < l; ++k) {
        val = (val - inv_fact) / z;          // phi_{k+1}
        inv_fact /= static_cast<double>(k + 1);
    }
    return val;
}

// ---------------------------------------------------------------------------
// Leja points of [-2, 2] (Sec. 2.1).  The first point is +2 (maximal modulus;
// the tie with -2 goes to the larger point), the second -2.  Each further
// point maximises L(x) = sum_k log|x - x_k| over [-2, 2]; it lies inside a
// gap between neighbouring points, where L is concave, at the root of
// L'(x) = sum_k 1/(x - x_k) (bracketed Newton iteration).
//
// To avoid re-solving every gap for every new point, each gap keeps a
// point x_g with L(x_g) and L'(x_g) updated in O(1) when a point is added.
// L(x_g) bounds the gap maximum from below; concavity with
// L'' <= -8/w^2 (w the gap width) bounds it from above by
// L(x_g) + L'(x_g)^2 w^2 / 16.  Only gaps whose upper bound reaches the best
// lower bound are re-solved exactly, until the winner is certain.
// ---------------------------------------------------------------------------
namespace {

struct Gap {
    double a, b;      // neighbouring points, a < b
    double x;         // tracked point inside (a, b)
    double V;         // L(x) over all current points
    double G;         // L'(x) over all current points
    bool exact;       // x is the maximiser for the current point set
};

double log_prod(double x, const std::vector<double>& pts) {
    double s = 0.0;
    for (double p : pts) s += std::log(std::fabs(x - p));
    return s;
}

// root of L' in (a, b) by bracketed Newton from x0
double gap_max(double a, double b, double x0, const std::vector<double>& pts) {
    double lo = a, hi = b;
    double x = (x0 > lo && x0 < hi) ? x0 : 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double g = 0.0, gp = 0.0;
        for (double p : pts) {
            const double r = 1.0 / (x - p);
            g += r;
            gp -= r * r;
        }
        if (g == 0.0) return x;
        if (g > 0.0) lo = x; else hi = x;
        double xn = x - g / gp;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 2.0 * std::numeric_limits<double>::epsilon() * std::fabs(x) ||
            xn == lo || xn == hi) {
            return xn;
        }
        x = xn;
    }
    return x;
}

void solve_gap(Gap& g, const std::vector<double>& pts) {
    g.x = gap_max(g.a, g.b, g.x, pts);
    g.V = log_prod(g.x, pts);
    double d = 0.0;
    for (double p : pts) d += 1.0 / (g.x - p);
    g.G = d;
    g.exact = true;
}

std::mutex g_leja_mutex;
std::vector<double> g_leja;       // points generated so far (prefix-stable)
std::vector<Gap> g_gaps;          // gaps between the sorted points, in order

void extend_leja(int M) {
    if (static_cast<int>(g_leja.size()) >= M) return;
    if (g_leja.empty()) g_leja.push_back(2.0);
    if (static_cast<int>(g_leja.size()) >= M) return;
    if (g_leja.size() == 1) {
        g_leja.push_back(-2.0);
        Gap g{-2.0, 2.0, 0.0, 0.0, 0.0, false};
        solve_gap(g, g_leja);
        g_gaps.push_back(g);
    }
    while (static_cast<int>(g_leja.size()) < M) {
        // choose the gap whose maximum is largest
        size_t win = 0;
        for (;;) {
            double best = -std::numeric_limits<double>::infinity();
            for (const Gap& g : g_gaps) best = std::max(best, g.V);
            const double tie = 1e-12 * std::max(1.0, std::fabs(best));
            bool refined = false;
            for (Gap& g : g_gaps) {
                const double w = g.b - g.a;
                const double upper = g.V + g.G * g.G * w * w / 16.0;
                if (!g.exact && upper >= best - tie) {
                    solve_gap(g, g_leja);
                    refined = true;
                }
            }
            if (refined) continue;
            // every gap that can still win is exact: largest value, exact
            // (to rounding) ties to the larger point
            best = -std::numeric_limits<double>::infinity();
            for (const Gap& g : g_gaps) best = std::max(best, g.V);
            double bx = -std::numeric_limits<double>::infinity();
            for (size_t i = 0; i < g_gaps.size(); ++i) {
                const Gap& g = g_gaps[i];
                if (g.exact && best - g.V <= tie && g.x > bx) {
                    bx = g.x;
                    win = i;
                }
            }
            break;
        }
        const double p = g_gaps[win].x;
        g_leja.push_back(p);
        for (Gap& g : g_gaps) {
            g.V += std::log(std::fabs(g.x - p));
            g.G += 1.0 / (g.x - p);
            g.exact = false;
        }
        const Gap old = g_gaps[win];
        Gap left{old.a, p, 0.5 * (old.a + p), 0.0, 0.0, false};
        Gap right{p, old.b, 0.5 * (p + old.b), 0.0, 0.0, false};
        solve_gap(left, g_leja);
        solve_gap(right, g_leja);
        g_gaps[win] = left;
        g_gaps.insert(g_gaps.begin() + static_cast<long>(win) + 1, right);
    }
}

}  // namespace

bool leja_points(int M, double* out) {
    if (M < 1 || M > kMaxPoints || out == nullptr) return false;
    std::lock_guard<std::mutex> lock(g_leja_mutex);
    extend_leja(M);
    std::copy(g_leja.begin(), g_leja.begin() + M, out);
    return true;
}

// ---------------------------------------------------------------------------
// Newton coefficients (Sec. 2.1, Eq. (2)): the divided differences
// d_j = f[xi_0, ..., xi_j] of f(xi) = sigma * phi_l(alpha*h*(c + gamma*xi)).
// The Newton basis at Leja points can grow by many orders of magnitude while
// the high-order d_j become tiny, so every d_j needs a small *relative*
// error: values and differences are carried in double-double and rounded
// to FP64 once.  The last row T_i = f[xi_i, ..., xi_J] of the divided-
// difference table is kept, so the next coefficient costs O(J):
//     T'_J = f(xi_J),  T'_i = (T'_{i+1} - T_i) / (xi_J - xi_i),  d_J = T'_0.
// ---------------------------------------------------------------------------
struct NewtonSeries::Impl {
    std::vector<dd> row;
    double alpha = 1.0, h = 0.0, sigma = 1.0, c = 0.0, gamma = 0.0;
    int l = 0;
};

NewtonSeries::NewtonSeries() : impl_(new Impl()) {}
NewtonSeries::~NewtonSeries() { delete impl_; }

void NewtonSeries::reset(int l, double alpha, double sigma, double h, double c, double gamma, const double* xi) {
    impl_->row.clear();
    impl_->alpha = alpha;
    impl_->h = h;
    impl_->sigma = sigma;
    impl_->c = c;
    impl_->gamma = gamma;
    impl_->l = l;
    xi_ = xi;
    count_ = 0;
}

double NewtonSeries::next() {
    Impl& s = *impl_;
    const int J = count_;
    const double x = xi_[J];
    s.row.push_back(dd_phi_at(s.l, s.alpha, s.sigma, s.h, s.c, s.gamma, x));
    for (int i = J - 1; i >= 0; --i) {
        const dd diff = two_sum(x, -xi_[i]);   // exact
        s.row[i] = dd_div(dd_sub(s.row[i + 1], s.row[i]), diff);
    }
    ++count_;
    return s.row[0].hi + s.row[0].lo;
}

bool newton_coeffs(int l, double alpha, double sigma, double h, double c, double gamma,
                   int M, const double* xi, double* d) {
    if (M < 1 || l < 0 || xi == nullptr || d == nullptr) return false;
    NewtonSeries ns;
    ns.reset(l, alpha, sigma, h, c, gamma, xi);
    for (int j = 0; j < M; ++j) d[j] = ns.next();
    return true;
}

}  // namespace lx
