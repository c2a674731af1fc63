// Host planner of the Leja phi-action library (plain C++, no HIP).
#pragma once

namespace lx {

constexpr int kMaxPoints = 1008;   // LX_MAX_ITERS + 8: windows of D iterations read up to d_{max_iters+D}

// phi_l(z) for real z (Sec. 1 recursion; Taylor series near 0).
double phi_scalar(int l, double z);

// First M Leja points of [-2, 2] (Sec. 2.1), generated once per process and
// extended on demand; thread-safe.  Returns false for M outside 1..kMaxPoints.
bool leja_points(int M, double* out);

// Divided differences of f(xi) = sigma*phi_l(alpha*h*(c + gamma*xi)) at the
// points xi[0], xi[1], ... (Sec. 2.1, Eq. (2)), produced one at a time in
// double-double arithmetic and rounded to FP64: next() returns d_J and costs
// O(J).  xi must stay valid while the series is used.
class NewtonSeries {
public:
    NewtonSeries();
    ~NewtonSeries();
    NewtonSeries(const NewtonSeries&) = delete;
    NewtonSeries& operator=(const NewtonSeries&) = delete;
    void reset(int l, double alpha, double sigma, double h, double c, double gamma, const double* xi);
    double next();
    int count() const { return count_; }

private:
    struct Impl;
    Impl* impl_;
    const double* xi_ = nullptr;
    int count_ = 0;
};

// d_0..d_{M-1} of the series above at the points xi[0..M-1].
bool newton_coeffs(int l, double alpha, double sigma, double h, double c, double gamma,
                   int M, const double* xi, double* d);

}  // namespace lx
