/*
 * ORACLE -- test infrastructure only.  Nothing in the library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.
 *
 * O1: the dense direct sum that defines the problem (section 1, the sum
 * u_i = sum_{j != i} G(x_i, x_j) q_j, and its matrix form u = A q with a zero
 * diagonal).  Plain loops in float64 (complex128 for Helmholtz), OpenMP over
 * targets, Neumaier-compensated accumulation so the oracle's own rounding
 * stays near one unit in the last place of the result.
 *
 * Kernels (section 2, the Laplace and Helmholtz fundamental solutions):
 *   2D Laplace    G = -log(r) / (2 pi)
 *   3D Laplace    G = 1 / (4 pi r)
 *   2D Helmholtz  G = (i/4) H0^(1)(kappa r)   (H0^(1) from hankel.c)
 *   3D Helmholtz  G = exp(i kappa r) / (4 pi r)
 * A pair with the same index is the excluded diagonal.  A pair of distinct
 * points at distance zero contributes zero (the paper does not define it).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <omp.h>

#define O_PI 3.14159265358979323846

void oracle_h0(double x, double* j0, double* y0);   /* hankel.c */

typedef struct { double s, c; } neu_t;   /* Neumaier running sum + correction */

static inline void neu_add(neu_t* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static inline double dist(int dim, const double* a, const double* b) {
    double s = 0.0;
    for (int d = 0; d < dim; ++d) { double t = a[d] - b[d]; s += t * t; }
    return sqrt(s);
}

/*
 * oracle_direct: u[t, :] = sum_{j != targ[t]} G(x_targ[t], x_j) q[j, :]
 *   dim    2 or 3;  kind 0 = Laplace, 1 = Helmholtz
 *   pts    n x dim row-major
 *   q      n x nrhs row-major; complex values interleaved (re, im) when kind == 1
 *   targ   ntarg target indices into pts
 *   out    ntarg x nrhs (x2 interleaved when complex)
 * Returns 0, or -1 on an unsupported combination.
 */
int oracle_direct(int dim, int kind, double kappa, int64_t n, const double* pts,
                  int nrhs, const double* q, int64_t ntarg, const int64_t* targ,
                  double* out)
{
    if ((dim != 2 && dim != 3) || (kind != 0 && kind != 1))
        return -1;
    const int cplx = (kind == 1);
    const int w = cplx ? 2 * nrhs : nrhs;
    #pragma omp parallel
    {
        neu_t* acc = (neu_t*)__builtin_alloca(sizeof(neu_t) * (size_t)w);
        #pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < ntarg; ++t) {
            const int64_t i = targ[t];
            const double* xi = pts + i * dim;
            memset(acc, 0, sizeof(neu_t) * (size_t)w);
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                const double r = dist(dim, xi, pts + j * dim);
                if (r == 0.0) continue;
                const double* qj = q + j * w;
                if (!cplx) {
                    const double g = (dim == 2) ? -log(r) / (2.0 * O_PI) : 1.0 / (4.0 * O_PI * r);
                    for (int c = 0; c < nrhs; ++c) neu_add(&acc[c], g * qj[c]);
                } else {
                    double gr, gi;
                    if (dim == 3) {
                        gr = cos(kappa * r) / (4.0 * O_PI * r);
                        gi = sin(kappa * r) / (4.0 * O_PI * r);
                    } else {
                        /* (i/4)(J0 + i Y0) */
                        double j0, y0;
                        oracle_h0(kappa * r, &j0, &y0);
                        gr = -0.25 * y0;
                        gi = 0.25 * j0;
                    }
                    for (int c = 0; c < nrhs; ++c) {
                        const double a = qj[2 * c], b = qj[2 * c + 1];
                        neu_add(&acc[2 * c], gr * a);
                        neu_add(&acc[2 * c], -gi * b);
                        neu_add(&acc[2 * c + 1], gr * b);
                        neu_add(&acc[2 * c + 1], gi * a);
                    }
                }
            }
            for (int c = 0; c < w; ++c) out[t * w + c] = acc[c].s + acc[c].c;
        }
    }
    return 0;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }
