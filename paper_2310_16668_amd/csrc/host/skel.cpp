// Strong recursive skeletonization (section 3, "Build stage", Algorithm
// "Strong recursive skeletonization"), bottom-up, every box of a level in
// parallel.
//
// For a box B with index set I_B (a leaf: its points; a tree box: its
// children's skeletons concatenated in child order), the proxy matrix
// M = G(Y, X_B) stands in for the far field (section 2.1, the proxy surface):
//   3D: first-kind Chebyshev nodes on the six faces of a cube of side 2.95 a
//       centred on B (p x p per face);
//   2D: equispaced points on a circle of radius 1.475 a (or the square's four
//       edges).
// For a real symmetric kernel the concatenated matrix of equation (5) has two
// identical blocks, so M alone is compressed.  For the complex symmetric
// Helmholtz kernels (3D exp(i kappa r) / (4 pi r), 2D (i/4) H0^(1)(kappa r)),
// [M; conj M] is unitarily equivalent to sqrt2 [Re M; Im M], a real matrix, so
// the interpolation matrix comes out real.
// Column-pivoted Householder QR (pivot: largest remaining column norm, lowest
// index on ties) stops at the first pivot with |R_jj| <= tol |R_11|; the first
// k pivots are the skeleton, T = R11^{-1} R12.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <stdexcept>

#include "../hankel.h"
#include "parallel.h"
#include "plan.h"
#include "skel.h"

namespace skelfmm {

namespace {

constexpr double kPi = 3.14159265358979323846;

void proxy_points(const Plan& p, int lev, const int32_t* c, std::vector<double>& Y) {
    const double a = std::ldexp(p.root_side, -lev);
    double ctr[3] = {0, 0, 0};
    for (int d = 0; d < p.dim; ++d) ctr[d] = p.root_lo[d] + (c[d] + 0.5) * a;
    std::vector<double> U;
    const double h = proxy_pattern(p, U) * a;
    Y.resize(U.size());
    for (size_t i = 0; i < U.size(); ++i) Y[i] = ctr[i % p.dim] + h * U[i];
}

// Column-pivoted Householder QR of the column-major m x n matrix A (destroyed),
// truncated at |R_jj| <= tol |R_11|.  Returns k; perm receives the pivot order;
// T (k x (n-k), column-major) = R11^{-1} R12.
int cpqr_id(double* A, int m, int n, double tol, std::vector<int64_t>& perm, std::vector<double>& T) {
    perm.resize(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::vector<double> nrm(n), ref(n);
    for (int c = 0; c < n; ++c) {
        const double* col = A + static_cast<int64_t>(c) * m;
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += col[i] * col[i];
        nrm[c] = ref[c] = s;
    }
    const int kmax = std::min(m, n);
    const double tol_norm2 = std::sqrt(2.220446049250313e-16);
    double r11 = 0.0;
    int k = 0;
    std::vector<double> v(m);
    for (int j = 0; j < kmax; ++j) {
        int piv = j;
        for (int c = j + 1; c < n; ++c)
            if (nrm[c] > nrm[piv]) piv = c;
        if (piv != j) {
            std::swap_ranges(A + static_cast<int64_t>(j) * m, A + static_cast<int64_t>(j + 1) * m,
                             A + static_cast<int64_t>(piv) * m);
            std::swap(nrm[j], nrm[piv]);
            std::swap(ref[j], ref[piv]);
            std::swap(perm[j], perm[piv]);
        }
        double* cj = A + static_cast<int64_t>(j) * m;
        double s = 0.0;
        for (int i = j; i < m; ++i) s += cj[i] * cj[i];
        const double alpha = std::sqrt(s);
        if (j == 0) r11 = alpha;
        if (!(alpha > tol * r11) || alpha == 0.0) break;
        // Householder reflector H = I - beta v v^T with H x = rjj e1
        const double x0 = cj[j];
        const double rjj = x0 >= 0 ? -alpha : alpha;
        const double v0 = x0 - rjj;
        v[j] = 1.0;
        for (int i = j + 1; i < m; ++i) v[i] = cj[i] / v0;
        const double beta = -v0 / rjj;
        cj[j] = rjj;
        for (int i = j + 1; i < m; ++i) cj[i] = 0.0;
        for (int c = j + 1; c < n; ++c) {
            double* cc = A + static_cast<int64_t>(c) * m;
            double w = 0.0;
            for (int i = j; i < m; ++i) w += v[i] * cc[i];
            w *= beta;
            for (int i = j; i < m; ++i) cc[i] -= w * v[i];
            // downdate the remaining norm; recompute when cancellation looms
            double t = nrm[c] - cc[j] * cc[j];
            if (t <= tol_norm2 * ref[c]) {
                t = 0.0;
                for (int i = j + 1; i < m; ++i) t += cc[i] * cc[i];
                ref[c] = t;
            }
            nrm[c] = std::max(t, 0.0);
        }
        k = j + 1;
    }
    // T = R11^{-1} R12 by back substitution, column by column
    T.assign(static_cast<size_t>(k) * (n - k), 0.0);
    for (int c = 0; c < n - k; ++c) {
        const double* r12 = A + static_cast<int64_t>(k + c) * m;
        double* t = T.data() + static_cast<int64_t>(c) * k;
        for (int i = k - 1; i >= 0; --i) {
            double s = r12[i];
            for (int l = i + 1; l < k; ++l) s -= A[static_cast<int64_t>(l) * m + i] * t[l];
            t[i] = s / A[static_cast<int64_t>(i) * m + i];
        }
    }
    return k;
}

void skeletonize_box(const Plan& p, int b, BoxSkel& out) {
    const int n = static_cast<int>(out.idx.size());
    if (p.opt.no_compression || n == 0) {
        out.k = n;
        out.pos.resize(n);
        std::iota(out.pos.begin(), out.pos.end(), 0);
        out.T.clear();
        return;
    }
    std::vector<double> Y;
    proxy_points(p, p.level[b], &p.coord[3 * b], Y);
    const int np = static_cast<int>(Y.size()) / p.dim;
    const int m = p.kind == 1 ? 2 * np : np;
    std::vector<double> A(static_cast<size_t>(m) * n);
    for (int a = 0; a < n; ++a) {
        const double* x = &p.pts[out.idx[a] * p.dim];
        double* col = A.data() + static_cast<int64_t>(a) * m;
        for (int r = 0; r < np; ++r) {
            const double* y = &Y[static_cast<size_t>(r) * p.dim];
            double s = 0.0;
            for (int d = 0; d < p.dim; ++d) { const double t = x[d] - y[d]; s += t * t; }
            const double rr = std::sqrt(s);
            if (p.kind == 0) {
                col[r] = p.dim == 2 ? -std::log(rr) / (2 * kPi) : 1.0 / (4 * kPi * rr);
            } else if (p.dim == 3) {
                col[r] = std::cos(p.kappa * rr) / (4 * kPi * rr);
                col[np + r] = std::sin(p.kappa * rr) / (4 * kPi * rr);
            } else {
                // (i/4) H0^(1)(kappa r) = (-Y0 + i J0) / 4
                double j0, y0;
                hankel::h0(p.kappa * rr, &j0, &y0);
                col[r] = -0.25 * y0;
                col[np + r] = 0.25 * j0;
            }
        }
    }
    std::vector<int64_t> perm;
    out.k = cpqr_id(A.data(), m, n, p.tol, perm, out.T);
    out.pos = perm;
}

}  // namespace

double proxy_pattern(const Plan& p, std::vector<double>& U) {
    const double scale = p.opt.proxy_scale > 0 ? p.opt.proxy_scale : 2.95;
    U.clear();
    if (p.dim == 3) {
        const int q = p.opt.proxy_points > 0 ? p.opt.proxy_points : 10;
        std::vector<double> t(q);
        for (int i = 0; i < q; ++i) t[i] = std::cos((2.0 * i + 1.0) * kPi / (2.0 * q));
        for (int ax = 0; ax < 3; ++ax)
            for (int sgn = -1; sgn <= 1; sgn += 2)
                for (int i = 0; i < q; ++i)
                    for (int j = 0; j < q; ++j) {
                        double y[3];
                        y[ax] = sgn;
                        y[(ax + 1) % 3] = t[i];
                        y[(ax + 2) % 3] = t[j];
                        for (int d = 0; d < 3; ++d) U.push_back(y[d]);
                    }
    } else if (p.opt.proxy_shape != 1) {
        const int m = p.opt.proxy_points > 0 ? p.opt.proxy_points : 128;
        for (int j = 0; j < m; ++j) {
            const double th = 2.0 * kPi * j / m;
            U.push_back(std::cos(th));
            U.push_back(std::sin(th));
        }
    } else {
        const int q = p.opt.proxy_points > 0 ? p.opt.proxy_points : 32;
        for (int ax = 0; ax < 2; ++ax)
            for (int sgn = -1; sgn <= 1; sgn += 2)
                for (int i = 0; i < q; ++i) {
                    double y[2];
                    y[ax] = sgn;
                    y[1 - ax] = std::cos((2.0 * i + 1.0) * kPi / (2.0 * q));
                    U.push_back(y[0]);
                    U.push_back(y[1]);
                }
    }
    return 0.5 * scale;
}

double host_kernel_real(const Plan& p, const double* x, const double* y) {
    double s = 0.0;
    for (int d = 0; d < p.dim; ++d) { const double t = x[d] - y[d]; s += t * t; }
    const double r = std::sqrt(s);
    if (r == 0.0) return 0.0;
    return p.dim == 2 ? -std::log(r) / (2 * kPi) : 1.0 / (4 * kPi * r);
}

void skeletonize(Plan& p, const std::vector<int64_t>& order, const std::vector<int64_t>& leaf_range) {
    const int nb = p.n_boxes;
    const int threads = host_threads(p.opt.num_threads);
    std::vector<BoxSkel> S(nb);
    const int top = p.top_level;
    std::unique_ptr<LevelSkeletonizer> dev;
    if (p.opt.gpu_build && !p.opt.no_compression) dev = make_device_skeletonizer(p);
    // index sets and skeletons, deepest level first
    for (int l = p.max_level; l >= top; --l) {
        const int b0 = p.level_ptr[l], b1 = p.level_ptr[l + 1];
        const auto tl = std::chrono::steady_clock::now();
        parallel_for(b1 - b0, threads, [&](int64_t t) {
            const int b = b0 + static_cast<int>(t);
            BoxSkel& s = S[b];
            if (p.is_leaf[b]) {
                s.idx.assign(order.begin() + leaf_range[2 * b], order.begin() + leaf_range[2 * b + 1]);
            } else {
                for (int e = p.child_ptr[b]; e < p.child_ptr[b + 1]; ++e) {
                    const BoxSkel& c = S[p.child_idx[e]];
                    for (int i = 0; i < c.k; ++i) s.idx.push_back(c.idx[c.pos[i]]);
                }
            }
            if (l <= top) {
                s.k = -1;
                s.pos.resize(s.idx.size());
                std::iota(s.pos.begin(), s.pos.end(), 0);
            } else if (!dev) {
                skeletonize_box(p, b, s);
            }
        });
        if (!dev) {   // the host IDs ran inside the loop above, with the index sets
            p.t_skel_qr += std::chrono::duration<double>(std::chrono::steady_clock::now() - tl).count();
        } else if (l > top) {
            const auto tq = std::chrono::steady_clock::now();
            dev->level(p, b0, b1, S);
            p.t_skel_qr += std::chrono::duration<double>(std::chrono::steady_clock::now() - tq).count();
        }
    }
    // flatten into CSR arrays (boxes above the top level keep empty sets)
    p.idx_ptr.assign(nb + 1, 0);
    p.T_ptr.assign(nb + 1, 0);
    p.rank.assign(nb, -1);
    p.k_max = 0;
    for (int b = 0; b < nb; ++b) {
        p.idx_ptr[b + 1] = p.idx_ptr[b] + static_cast<int64_t>(S[b].idx.size());
        p.T_ptr[b + 1] = p.T_ptr[b] + S[b].t_size();
        if (p.level[b] > top) { p.rank[b] = S[b].k; p.k_max = std::max(p.k_max, S[b].k); }
    }
    p.idx.resize(p.idx_ptr[nb]);
    p.pos.resize(p.idx_ptr[nb]);
    p.T.resize(p.T_ptr[nb]);
    parallel_for(nb, threads, [&](int64_t b) {
        std::copy(S[b].idx.begin(), S[b].idx.end(), p.idx.begin() + p.idx_ptr[b]);
        std::copy(S[b].pos.begin(), S[b].pos.end(), p.pos.begin() + p.idx_ptr[b]);
        if (S[b].Tsrc) std::copy(S[b].Tsrc, S[b].Tsrc + S[b].Tn, p.T.begin() + p.T_ptr[b]);
        else std::copy(S[b].T.begin(), S[b].T.end(), p.T.begin() + p.T_ptr[b]);
    }, 64);
    {
        std::vector<double> Y;
        if (nb > 0) proxy_points(p, 0, &p.coord[0], Y);
        p.proxy_count = static_cast<int>(Y.size()) / p.dim;
    }
}

}  // namespace skelfmm
