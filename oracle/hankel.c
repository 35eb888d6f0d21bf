/*
 * ORACLE -- test infrastructure only.  Nothing in the library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.
 *
 * H0^(1)(x) = J0(x) + i Y0(x), x > 0, for the 2D Helmholtz kernel
 * G = (i/4) H0^(1)(kappa r) (section 2, the Helmholtz fundamental solution in
 * the plane).  Plain float64, three ranges:
 *
 *   x < 4       the power series of J0 and Y0 (Abramowitz & Stegun 9.1.12-13);
 *               its terms stay below 4 in size, so float64 keeps ~15 digits.
 *   4 <= x < 25 Miller's backward recurrence J_{n-1} = (2n/x) J_n - J_{n+1}
 *               from an index N well above x, normalised by the identity
 *               J0 + 2 (J2 + J4 + ...) = 1 (A&S 9.1.46), and the Neumann series
 *               Y0 = (2/pi)(log(x/2) + gamma) J0 - (4/pi) sum_{k>=1} (-1)^k J_{2k} / k
 *               (A&S 9.1.88).
 *   x >= 25     Hankel's asymptotic expansion (A&S 9.2.5, 9.2.9-10 with nu = 0):
 *               J0 = sqrt(2/(pi x)) (P cos chi - Q sin chi),
 *               Y0 = sqrt(2/(pi x)) (P sin chi + Q cos chi),  chi = x - pi/4,
 *               P and Q summed until their terms fall below 1e-17.
 *
 * Pinned against scipy.special.hankel1 (tests/test_oracle_hankel.py).
 */
#include <math.h>
#include <stdint.h>

#define H_PI 3.14159265358979323846
#define H_GAMMA 0.57721566490153286061

static void h0_series(double x, double* j0, double* y0)
{
    const double z = 0.25 * x * x;
    double term = 1.0, sj = 1.0, sy = 0.0, hk = 0.0;
    for (int k = 1; k < 200; ++k) {
        term *= z / ((double)k * (double)k);
        hk += 1.0 / k;
        const double sgn = (k % 2) ? -1.0 : 1.0;
        sj += sgn * term;
        sy -= sgn * hk * term;
        if (hk * term < 1e-18) break;
    }
    *j0 = sj;
    *y0 = (2.0 / H_PI) * ((log(0.5 * x) + H_GAMMA) * sj + sy);
}

static void h0_miller(double x, double* j0, double* y0)
{
    int N = (int)(1.3 * x) + 34;
    if (N % 2) ++N;
    double jp = 0.0, jc = 1e-250;   /* J_{n+1}, J_n (unnormalised) */
    double even = 0.0;              /* J2 + J4 + ... */
    double alt = 0.0;               /* sum_{k>=1} (-1)^k J_{2k} / k */
    for (int n = N; n >= 1; --n) {
        const double jm = (2.0 * n / x) * jc - jp;   /* J_{n-1} */
        jp = jc;
        jc = jm;
        const int m = n - 1;
        if (m >= 2 && m % 2 == 0) {
            even += jc;
            const int k = m / 2;
            alt += ((k % 2) ? -1.0 : 1.0) * jc / k;
        }
    }
    const double norm = jc + 2.0 * even;
    const double J0 = jc / norm;
    *j0 = J0;
    *y0 = (2.0 / H_PI) * (log(0.5 * x) + H_GAMMA) * J0 - (4.0 / H_PI) * (alt / norm);
}

static void h0_asymptotic(double x, double* j0, double* y0)
{
    /* terms a_k / x^k with a_k = (-1)^k (1*3*...*(2k-1))^2 / (k! 8^k);
       P takes k = 0, 2, 4, ... with signs +, -, +, ...; Q takes k = 1, 3, ... with +, -, ... */
    double t = 1.0, P = 1.0, Q = 0.0, last = 2.0;
    for (int k = 1; k < 100; ++k) {
        t *= -((2.0 * k - 1) * (2.0 * k - 1)) / (8.0 * k * x);
        const double at = fabs(t);
        if (at > last) break;
        last = at;
        if (k % 2 == 0) P += ((k / 2) % 2 ? -1.0 : 1.0) * t;
        else Q += (((k - 1) / 2) % 2 ? -1.0 : 1.0) * t;
        if (at < 1e-17) break;
    }
    const double chi = x - 0.25 * H_PI;
    const double amp = sqrt(2.0 / (H_PI * x));
    *j0 = amp * (P * cos(chi) - Q * sin(chi));
    *y0 = amp * (P * sin(chi) + Q * cos(chi));
}

void oracle_h0(double x, double* j0, double* y0)
{
    if (x < 4.0) h0_series(x, j0, y0);
    else if (x < 25.0) h0_miller(x, j0, y0);
    else h0_asymptotic(x, j0, y0);
}

/* J0 and Y0 at n points (for the pins). */
void oracle_h0_many(int64_t n, const double* x, double* j0, double* y0)
{
    for (int64_t i = 0; i < n; ++i) oracle_h0(x[i], &j0[i], &y0[i]);
}
