// The Hankel function H0^(1)(x) = J0(x) + i Y0(x) for real x > 0, the 2D
// Helmholtz kernel G = (i/4) H0^(1)(kappa r) (section 2, the Helmholtz
// fundamental solution in the plane), in float64, for the host build and the
// device kernels alike.
//
//   x < kHankelSwitch: the power series
//       J0(x) = sum_k (-1)^k t_k,            t_k = (x^2/4)^k / (k!)^2,
//       Y0(x) = (2/pi) [ (log(x/2) + gamma) J0(x) + sum_{k>=1} (-1)^(k+1) H_k t_k ],
//     with H_k the harmonic numbers (Abramowitz & Stegun 9.1.12-13).  Its terms
//     grow to about 1e9 before they decay (x near 25), so they are summed in
//     double-double arithmetic (a float64 pair whose sum carries about 32
//     digits: error-free sums and products after Dekker and Knuth), which keeps
//     the cancellation below float64 rounding.
//   x >= kHankelSwitch: Hankel's asymptotic expansion
//       H0^(1)(x) = sqrt(2 / (pi x)) e^{i (x - pi/4)} sum_k i^k a_k / x^k,
//       a_k = (-1)^k (1 * 3 * ... * (2k-1))^2 / (k! 8^k)   (A&S 9.2.7 with nu = 0),
//     truncated at the first term below 1e-17 (the smallest term is about
//     e^{-2x}, far below that for x >= 25).
#pragma once

#include <cmath>

#if defined(__HIP__)
#define SKF_HD __host__ __device__
#else
#define SKF_HD
#endif
// The error-free transformations below need every sum and product rounded as
// written: no multiply-add contraction across statements (the device compiler
// contracts by default, which would fold a product into the sum whose rounding
// error the next statement recovers).
#if defined(__clang__)
#define SKF_EXACT_FP _Pragma("clang fp contract(off)")
#else
#define SKF_EXACT_FP
#endif

namespace skelfmm {
namespace hankel {

constexpr double kSwitch = 25.0;
constexpr double kEulerGamma = 0.57721566490153286060651209008240243;
constexpr double kTwoOverPi = 0.63661977236758134307553505349005745;
constexpr double kInvSqrt2 = 0.70710678118654752440084436210484904;

// double-double value hi + lo, |lo| <= ulp(hi) / 2
struct DD {
    double hi, lo;
};

SKF_HD inline DD two_sum(double a, double b) {
    SKF_EXACT_FP
    const double s = a + b;
    const double bb = s - a;
    return DD{s, (a - (s - bb)) + (b - bb)};
}
SKF_HD inline DD quick_two_sum(double a, double b) {
    SKF_EXACT_FP
    const double s = a + b;
    return DD{s, b - (s - a)};
}
SKF_HD inline DD dd_add(DD a, DD b) {
    SKF_EXACT_FP
    DD s = two_sum(a.hi, b.hi);
    const DD t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
SKF_HD inline DD dd_neg(DD a) { return DD{-a.hi, -a.lo}; }
SKF_HD inline DD dd_mul(DD a, DD b) {
    SKF_EXACT_FP
    const double p = a.hi * b.hi;
    const double e = std::fma(a.hi, b.hi, -p);
    return quick_two_sum(p, e + (a.hi * b.lo + a.lo * b.hi));
}
// a / d for a double d
SKF_HD inline DD dd_div(DD a, double d) {
    SKF_EXACT_FP
    const double q1 = a.hi / d;
    // remainder a - q1 d, exact in its leading part
    const double p = q1 * d;
    const double e = std::fma(q1, d, -p);
    const DD r = dd_add(a, DD{-p, -e});
    const double q2 = r.hi / d;
    return quick_two_sum(q1, q2);
}

// H0^(1)(x) for x > 0: *j0 = J0(x), *y0 = Y0(x).
SKF_HD inline void h0(double x, double* j0, double* y0) {
    SKF_EXACT_FP
    if (x < kSwitch) {
        // q = x^2 / 4 exactly as a double-double
        const double x2 = x * x;
        const DD q = DD{0.25 * x2, 0.25 * std::fma(x, x, -x2)};
        DD t{1.0, 0.0};          // t_k
        DD sj{1.0, 0.0};         // sum (-1)^k t_k
        DD sy{0.0, 0.0};         // sum (-1)^(k+1) H_k t_k
        DD hk{0.0, 0.0};         // H_k
        for (int k = 1; k < 120; ++k) {
            t = dd_div(dd_mul(t, q), static_cast<double>(k) * static_cast<double>(k));
            hk = dd_add(hk, dd_div(DD{1.0, 0.0}, static_cast<double>(k)));
            const DD th = dd_mul(t, hk);
            if (k & 1) {
                sj = dd_add(sj, dd_neg(t));
                sy = dd_add(sy, th);
            } else {
                sj = dd_add(sj, t);
                sy = dd_add(sy, dd_neg(th));
            }
            if (th.hi < 1e-18 && t.hi < 1e-18) break;
        }
        const double j = sj.hi + sj.lo;
        *j0 = j;
        *y0 = kTwoOverPi * ((std::log(0.5 * x) + kEulerGamma) * j + (sy.hi + sy.lo));
        return;
    }
    // asymptotic expansion: P = sum_even (-1)^(k/2) T_k, Q = sum_odd (-1)^((k-1)/2) T_k
    double tk = 1.0, P = 1.0, Q = 0.0, prev = 2.0;
    for (int k = 1; k < 80; ++k) {
        const double f = static_cast<double>(2 * k - 1);
        tk *= -(f * f) / (8.0 * k * x);
        const double at = std::fabs(tk);
        if (at > prev) break;   // the expansion has started to diverge
        prev = at;
        switch (k & 3) {
            case 0: P += tk; break;
            case 1: Q += tk; break;
            case 2: P -= tk; break;
            default: Q -= tk; break;
        }
        if (at < 1e-17) break;
    }
    // e^{i (x - pi/4)} = (cos x + sin x + i (sin x - cos x)) / sqrt 2
    double s, c;
#if defined(__HIP_DEVICE_COMPILE__)
    sincos(x, &s, &c);
#else
    s = std::sin(x);
    c = std::cos(x);
#endif
    const double cr = (c + s) * kInvSqrt2, ci = (s - c) * kInvSqrt2;
    const double amp = std::sqrt(kTwoOverPi / x);
    *j0 = amp * (cr * P - ci * Q);
    *y0 = amp * (ci * P + cr * Q);
}

}  // namespace hankel
}  // namespace skelfmm
