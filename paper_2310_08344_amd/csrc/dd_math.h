// Double-double arithmetic and the phi functions in double-double, shared
// by the host planner (plain C++) and the device planner (HIP).
//
// A value is hi + lo with |lo| <= ulp(hi)/2.  The error-free
// transformations are Knuth's TwoSum and Dekker's TwoProduct (with an FMA);
// addition, multiplication and division follow Hida, Li and Bailey,
// "Algorithms for quad-double precision floating point arithmetic" (2001).
// About 32 significant digits.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define LX_HD __host__ __device__ inline
#else
#define LX_HD inline
#endif

// The error-free transformations need every product and sum rounded on its
// own: a multiply fused into a later add (which HIP device code allows by
// default, also across inlined calls) breaks them and leaves plain double
// precision.  Every function below switches contraction off for its body.
#if defined(__clang__)
#define LX_NO_CONTRACT _Pragma("clang fp contract(off)")
#else
#define LX_NO_CONTRACT
#endif

namespace lx {

struct dd {
    double hi, lo;
};

LX_HD dd two_sum(double a, double b) {
    LX_NO_CONTRACT
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

LX_HD dd quick_two_sum(double a, double b) {
    LX_NO_CONTRACT
    const double s = a + b;
    return {s, b - (s - a)};
}

LX_HD dd two_prod(double a, double b) {
    LX_NO_CONTRACT
    const double p = a * b;
    return {p, fma(a, b, -p)};
}

LX_HD dd dd_add(dd x, dd y) {
    LX_NO_CONTRACT
    dd s = two_sum(x.hi, y.hi);
    const dd t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

LX_HD dd dd_neg(dd x) {
    LX_NO_CONTRACT
    return {-x.hi, -x.lo};
}
LX_HD dd dd_sub(dd x, dd y) {
    LX_NO_CONTRACT
    return dd_add(x, dd_neg(y));
}

LX_HD dd dd_mul(dd x, dd y) {
    LX_NO_CONTRACT
    dd p = two_prod(x.hi, y.hi);
    p.lo += x.hi * y.lo + x.lo * y.hi;
    return quick_two_sum(p.hi, p.lo);
}

LX_HD dd dd_mul_d(dd x, double b) {
    LX_NO_CONTRACT
    dd p = two_prod(x.hi, b);
    p.lo += x.lo * b;
    return quick_two_sum(p.hi, p.lo);
}

LX_HD dd dd_div(dd x, dd y) {
    LX_NO_CONTRACT
    const double q1 = x.hi / y.hi;
    dd r = dd_sub(x, dd_mul_d(y, q1));
    const double q2 = r.hi / y.hi;
    r = dd_sub(r, dd_mul_d(y, q2));
    const double q3 = r.hi / y.hi;
    const dd q = quick_two_sum(q1, q2);
    return dd_add(q, dd{q3, 0.0});
}

LX_HD dd dd_div_d(dd x, double b) {
    LX_NO_CONTRACT
    return dd_div(x, dd{b, 0.0});
}
LX_HD dd dd_ldexp(dd x, int e) {
    LX_NO_CONTRACT
    return {ldexp(x.hi, e), ldexp(x.lo, e)};
}

// e^r - 1 for a = k ln2 + r, |r| <= ln2/2: r is scaled by 2^-10, the Taylor
// series to order 12 is summed, then ten doublings
// e^{2x} - 1 = 2(e^x - 1) + (e^x - 1)^2 undo the scaling.  Returns k too.
LX_HD dd expm1_reduced(dd a, int* k_out) {
    LX_NO_CONTRACT
    const double ln2_hi = 6.931471805599452862e-01;   // ln 2 = hi + lo
    const double ln2_lo = 2.319046813846299558e-17;
    const double k = rint(a.hi / ln2_hi);
    dd r = dd_sub(a, dd_add(two_prod(k, ln2_hi), two_prod(k, ln2_lo)));
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

LX_HD dd dd_exp(dd a) {
    LX_NO_CONTRACT
    if (a.hi < -1000.0) return {0.0, 0.0};
    int k = 0;
    const dd s = expm1_reduced(a, &k);
    return dd_ldexp(dd_add(s, dd{1.0, 0.0}), k);
}

LX_HD dd dd_expm1(dd a) {
    LX_NO_CONTRACT
    if (a.hi < -1000.0) return {-1.0, 0.0};
    int k = 0;
    const dd s = expm1_reduced(a, &k);
    if (k == 0) return s;
    return dd_sub(dd_ldexp(dd_add(s, dd{1.0, 0.0}), k), dd{1.0, 0.0});
}

// phi_l(z) in double-double (Sec. 1 of the paper): the Taylor series
// sum_k z^k/(k+l)! while its terms decrease monotonically (|z| < max(1.5, l),
// 60 terms), otherwise phi_1 = expm1(z)/z and the recursion
// phi_{k+1} = (phi_k - 1/k!)/z.
LX_HD dd dd_phi(int l, dd z) {
    LX_NO_CONTRACT
    dd inv_fact_l{1.0, 0.0};
    for (int k = 2; k <= l; ++k) inv_fact_l = dd_div_d(inv_fact_l, static_cast<double>(k));
    if (z.hi == 0.0) return inv_fact_l;
    const double lim = (static_cast<double>(l) > 1.5) ? static_cast<double>(l) : 1.5;
    if (fabs(z.hi) < lim) {
        // Horner from the tail; coefficient k is 1/(k+l)!
        dd coef_top = inv_fact_l;
        for (int k = 1; k <= 60; ++k) coef_top = dd_div_d(coef_top, static_cast<double>(k + l));
        dd acc{0.0, 0.0};
        dd c = coef_top;
        for (int k = 60; k >= 0; --k) {
            acc = dd_add(dd_mul(acc, z), c);
            if (k > 0) c = dd_mul_d(c, static_cast<double>(k + l));   // 1/(k-1+l)!
        }
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

// f(xi) = sigma * phi_l(alpha*h*(c + gamma*xi)) in double-double, from FP64
// inputs taken exactly
LX_HD dd dd_phi_at(int l, double alpha, double sigma, double h, double c, double gamma, double xi) {
    LX_NO_CONTRACT
    const dd ah = two_prod(alpha, h);
    const dd t = dd_add(dd{c, 0.0}, two_prod(gamma, xi));
    return dd_mul(dd{sigma, 0.0}, dd_phi(l, dd_mul(ah, t)));
}

}  // namespace lx
