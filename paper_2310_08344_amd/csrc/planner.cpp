// Host planner: Leja points of [-2, 2], scalar phi_l and Newton divided
// differences (Sec. 1 and Sec. 2.1 of arXiv 2310.08344).  Plain C++, no HIP.
#include "planner.h"

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
// Double-double arithmetic (a value is hi + lo with |lo| <= ulp(hi)/2), from
// the error-free transformations of Knuth (TwoSum) and Dekker (TwoProduct,
// here with an FMA) and the double-double algorithms of Hida, Li and Bailey
// ("Algorithms for quad-double precision floating point arithmetic", 2001).
// About 32 significant digits.
// ---------------------------------------------------------------------------
namespace {

struct dd {
    double hi, lo;
};

inline dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

inline dd quick_two_sum(double a, double b) {
    const double s = a + b;
    return {s, b - (s - a)};
}

inline dd two_prod(double a, double b) {
    const double p = a * b;
    return {p, std::fma(a, b, -p)};
}

inline dd dd_add(dd x, dd y) {
    dd s = two_sum(x.hi, y.hi);
    dd t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

inline dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
inline dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }

inline dd dd_mul(dd x, dd y) {
    dd p = two_prod(x.hi, y.hi);
    p.lo += x.hi * y.lo + x.lo * y.hi;
    return quick_two_sum(p.hi, p.lo);
}

inline dd dd_mul_d(dd x, double b) {
    dd p = two_prod(x.hi, b);
    p.lo += x.lo * b;
    return quick_two_sum(p.hi, p.lo);
}

inline dd dd_div(dd x, dd y) {
    const double q1 = x.hi / y.hi;
    dd r = dd_sub(x, dd_mul_d(y, q1));
    const double q2 = r.hi / y.hi;
    r = dd_sub(r, dd_mul_d(y, q2));
    const double q3 = r.hi / y.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add(q, dd{q3, 0.0});
}

inline dd dd_div_d(dd x, double b) { return dd_div(x, dd{b, 0.0}); }
inline dd dd_ldexp(dd x, int e) { return {std::ldexp(x.hi, e), std::ldexp(x.lo, e)}; }

// ln 2 = kLn2Hi + kLn2Lo to double-double accuracy
constexpr double kLn2Hi = 6.931471805599452862e-01;
constexpr double kLn2Lo = 2.319046813846299558e-17;

// e^a - 1 and the power of two it was reduced by: with a = k ln2 + r,
// |r| <= ln2/2, returns s = e^r - 1 (r scaled by 2^-10, Taylor series to
// order 12, then ten doublings e^{2x} - 1 = 2(e^x - 1) + (e^x - 1)^2) and k.
dd expm1_reduced(dd a, int* k_out) {
    const double k = std::nearbyint(a.hi / kLn2Hi);
    dd r = dd_sub(a, dd_add(two_prod(k, kLn2Hi), two_prod(k, kLn2Lo)));
    r = dd_ldexp(r, -10);
    dd term = r, s = r;
    for (int n = 2; n <= 12; ++n) {
        term = dd_div_d(dd_mul(term, r), static_cast<double>(n));
        s = dd_add(s, term);
    }
    for (int i = 0; i < 10; ++i) s = dd_add(dd_mul_d(s, 2.0), dd_mul(s, s));
    *k_out = static_cast<int>(k);
    return s;
}

dd dd_exp(dd a) {
    if (a.hi < -1000.0) return {0.0, 0.0};
    int k = 0;
    const dd s = expm1_reduced(a, &k);
    return dd_ldexp(dd_add(s, dd{1.0, 0.0}), k);
}

dd dd_expm1(dd a) {
    if (a.hi < -1000.0) return {-1.0, 0.0};
    int k = 0;
    const dd s = expm1_reduced(a, &k);
    if (k == 0) return s;
    return dd_sub(dd_ldexp(dd_add(s, dd{1.0, 0.0}), k), dd{1.0, 0.0});
}

// phi_l(z) in double-double (Sec. 1): the Taylor series sum_k z^k/(k+l)!
// while its terms decrease monotonically (|z| < max(1.5, l)), otherwise
// phi_1 = expm1(z)/z and the recursion phi_{k+1} = (phi_k - 1/k!)/z.
dd dd_phi(int l, dd z) {
    dd inv_fact_l{1.0, 0.0};
    for (int k = 2; k <= l; ++k) inv_fact_l = dd_div_d(inv_fact_l, static_cast<double>(k));
    if (z.hi == 0.0) return inv_fact_l;
    if (std::fabs(z.hi) < std::max(1.5, static_cast<double>(l))) {
        constexpr int kTerms = 60;
        dd coef[kTerms + 1];
        coef[0] = inv_fact_l;
        for (int k = 1; k <= kTerms; ++k) coef[k] = dd_div_d(coef[k - 1], static_cast<double>(k + l));
        dd acc{0.0, 0.0};
        for (int k = kTerms; k >= 0; --k) acc = dd_add(dd_mul(acc, z), coef[k]);
        return acc;
    }
    if (l == 0) return dd_exp(z);
    dd val = dd_div(dd_expm1(z), z);          // phi_1
    dd inv_fact{1.0, 0.0};                    // 1/k! for k = 1
    for (int k = 1; k < l; ++k) {
        val = dd_div(dd_sub(val, inv_fact), z);
        inv_fact = dd_div_d(inv_fact, static_cast<double>(k + 1));
    }
    return val;
}

}  // namespace

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
    dd ah{0.0, 0.0};
    dd sigma{1.0, 0.0};
    double c = 0.0, gamma = 0.0;
    int l = 0;
};

NewtonSeries::NewtonSeries() : impl_(new Impl()) {}
NewtonSeries::~NewtonSeries() { delete impl_; }

void NewtonSeries::reset(int l, double alpha, double sigma, double h, double c, double gamma, const double* xi) {
    impl_->row.clear();
    impl_->ah = two_prod(alpha, h);
    impl_->sigma = dd{sigma, 0.0};
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
    // z = alpha h (c + gamma xi_J) in double-double
    const dd t = dd_add(dd{s.c, 0.0}, two_prod(s.gamma, x));
    const dd f = dd_mul(s.sigma, dd_phi(s.l, dd_mul(s.ah, t)));
    s.row.push_back(f);
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
