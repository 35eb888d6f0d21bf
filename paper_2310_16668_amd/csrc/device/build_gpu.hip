// The interpolative decompositions of a tree level on the GPU (section 2.1,
// equation (5), the proxy-surface ID; section 3, "Build stage", Algorithm
// "Strong recursive skeletonization").  The host still builds the tree, the
// neighbor lists and every box's index set; per level, the device
//   1. evaluates the proxy matrices M = G(Y_B, X_B) of all boxes (m x n, stored
//      row by row; Helmholtz: m = 2 np rows, [Re M; Im M], which is unitarily
//      equivalent to the concatenation [M; conj M] of equation (5), so T is real),
//   2. runs column-pivoted Householder QR on each of them, one block per box
//      and one thread per column, so every step streams the trailing rows with
//      coalesced loads; it stops at the first pivot with |R_jj| <= tol |R_11|
//      (pivot: largest remaining column norm, lowest index on ties; norms
//      downdated and recomputed when cancellation looms, as the host build does),
//   3. solves T = R11^{-1} R12 by back substitution, one thread per column,
// and hands k, the pivot order and T back to the host.  The arithmetic is that
// of the host build in float64; only the summation order differs, so the
// skeletons agree except where rounding decides a near tie.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../hankel.h"
#include "../host/skel.h"
#include "device.h"

namespace skelfmm {

namespace {

#define SKF_BHIP(x)                                                                                \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) {                                                                    \
            if (e_ == hipErrorOutOfMemory) throw OutOfMemory(std::string(#x) + ": out of memory"); \
            throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_));                    \
        }                                                                                          \
    } while (0)

constexpr double kPiB = 3.14159265358979323846;
// Proxy matrix of box b (blockIdx.y), row-major: M[r n + a] = G(y_r, x_idx[a])
// (real kernels), rows np..2np-1 the imaginary parts (Helmholtz).  The proxy
// points are y_r = c_b + h_b U_r, as on the host; consecutive threads take
// consecutive points of one proxy row.
__global__ void __launch_bounds__(256) k_proxy_matrix(const double* __restrict__ pts, int dim, int kind,
                                                      double kappa, const int32_t* __restrict__ idx,
                                                      const int64_t* __restrict__ ioff,
                                                      const int32_t* __restrict__ nn,
                                                      const double* __restrict__ ctrh,
                                                      const double* __restrict__ U, int np,
                                                      const int64_t* __restrict__ moff, double* __restrict__ M) {
    const int b = blockIdx.y;
    const int n = nn[b];
    const int m = kind == 1 ? 2 * np : np;
    const double* ch = ctrh + 4 * b;
    const int64_t total = static_cast<int64_t>(np) * n;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int r = static_cast<int>(e / n), a = static_cast<int>(e - static_cast<int64_t>(r) * n);
        const int64_t pi = idx[ioff[b] + a];
        double s = 0.0;
        for (int d = 0; d < dim; ++d) {
            const double y = ch[d] + ch[3] * U[r * dim + d];
            const double t = pts[pi * dim + d] - y;
            s += t * t;
        }
        const double rr = sqrt(s);
        double* row = M + moff[b] + static_cast<int64_t>(r) * n + a;
        if (kind == 0) {
            row[0] = dim == 2 ? -log(rr) / (2 * kPiB) : 1.0 / (4 * kPiB * rr);
        } else if (dim == 3) {
            double sn, cs;
            sincos(kappa * rr, &sn, &cs);
            row[0] = cs / (4 * kPiB * rr);
            row[static_cast<int64_t>(np) * n] = sn / (4 * kPiB * rr);
        } else {
            double j0, y0;
            hankel::h0(kappa * rr, &j0, &y0);
            row[0] = -0.25 * y0;
            row[static_cast<int64_t>(np) * n] = 0.25 * j0;
        }
    }
}

// Column-pivoted Householder QR of box blockIdx.x's m x n matrix A (row-major,
// in place), truncated at |R_jj| <= tol |R_11|.  Thread t owns columns t,
// t + blockDim, ... (blockDim a power of two, for the tree reductions); perm
// receives the pivot order, kout k; nrm holds 2 n doubles of scratch per box
// (running and reference column norms).
__global__ void __launch_bounds__(1024) k_cpqr(double* __restrict__ M, const int64_t* __restrict__ moff,
                                               const int32_t* __restrict__ nn, int m, double tol,
                                               int32_t* __restrict__ kout, int32_t* __restrict__ perm,
                                               const int64_t* __restrict__ poff, double* __restrict__ nrmbuf) {
    extern __shared__ double v[];   // the Householder vector, m entries
    __shared__ double red_v[1024];
    __shared__ int red_i[1024];
    const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    double* __restrict__ A = M + moff[b];
    const int n = nn[b];
    int32_t* __restrict__ pm = perm + poff[b];
    double* __restrict__ nrm = nrmbuf + 2 * poff[b];
    double* __restrict__ ref = nrm + n;
    for (int c = tid; c < n; c += nt) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) {
            const double x = A[static_cast<int64_t>(i) * n + c];
            s += x * x;
        }
        nrm[c] = s;
        ref[c] = s;
        pm[c] = c;
    }
    __syncthreads();
    const double tol_norm2 = 1.4901161193847656e-08;   // sqrt(2^-52): recompute a norm below this fraction
    const int kmax = min(m, n);
    double r11 = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        // pivot: the largest remaining norm, the lowest index on ties
        double best = -1.0;
        int bi = n;
        for (int c = j + tid; c < n; c += nt) {
            const double x = nrm[c];
            if (x > best) { best = x; bi = c; }
        }
        red_v[tid] = best;
        red_i[tid] = bi;
        __syncthreads();
        for (int o = nt / 2; o > 0; o >>= 1) {
            if (tid < o) {
                const double x = red_v[tid + o];
                const int xi = red_i[tid + o];
                if (x > red_v[tid] || (x == red_v[tid] && xi < red_i[tid])) {
                    red_v[tid] = x;
                    red_i[tid] = xi;
                }
            }
            __syncthreads();
        }
        const int piv = red_i[0];
        __syncthreads();
        if (piv != j) {
            for (int i = tid; i < m; i += nt) {
                double* row = A + static_cast<int64_t>(i) * n;
                const double t = row[j];
                row[j] = row[piv];
                row[piv] = t;
            }
            if (tid == 0) {
                double t = nrm[j]; nrm[j] = nrm[piv]; nrm[piv] = t;
                t = ref[j]; ref[j] = ref[piv]; ref[piv] = t;
                const int32_t pt = pm[j]; pm[j] = pm[piv]; pm[piv] = pt;
            }
        }
        __syncthreads();
        // alpha = |A[j:, j]|: the column's rows, one per thread, then a tree sum
        double s = 0.0;
        for (int i = j + tid; i < m; i += nt) {
            const double x = A[static_cast<int64_t>(i) * n + j];
            v[i] = x;
            s += x * x;
        }
        red_v[tid] = s;
        __syncthreads();
        for (int o = nt / 2; o > 0; o >>= 1) {
            if (tid < o) red_v[tid] += red_v[tid + o];
            __syncthreads();
        }
        const double alpha = sqrt(red_v[0]);
        __syncthreads();
        if (j == 0) r11 = alpha;
        if (!(alpha > tol * r11) || alpha == 0.0) break;
        // Householder reflector H = I - beta v v^T with H x = rjj e1, v_j = 1
        const double x0 = v[j];
        const double rjj = x0 >= 0 ? -alpha : alpha;
        const double v0 = x0 - rjj;
        const double beta = -v0 / rjj;
        __syncthreads();
        for (int i = j + tid; i < m; i += nt) {
            v[i] = i == j ? 1.0 : v[i] / v0;
            A[static_cast<int64_t>(i) * n + j] = i == j ? rjj : 0.0;
        }
        __syncthreads();
        // the trailing columns, one per thread: w = beta v^T A[j:, c]; A[j:, c] -= w v
        for (int c = j + 1 + tid; c < n; c += nt) {
            double* col = A + c;
            double w = 0.0;
            for (int i = j; i < m; ++i) w += v[i] * col[static_cast<int64_t>(i) * n];
            w *= beta;
            double s2 = 0.0, cjn = 0.0;
            for (int i = j; i < m; ++i) {
                const double x = col[static_cast<int64_t>(i) * n] - w * v[i];
                col[static_cast<int64_t>(i) * n] = x;
                if (i > j) s2 += x * x;
                else cjn = x;
            }
            double t = nrm[c] - cjn * cjn;
            if (t <= tol_norm2 * ref[c]) {
                t = s2;
                ref[c] = t;
            }
            nrm[c] = t > 0.0 ? t : 0.0;
        }
        __syncthreads();
        k = j + 1;
    }
    if (tid == 0) kout[b] = k;
}

// T = R11^{-1} R12 of box blockIdx.y by back substitution, one thread per column
// of R12; T is written row-major (k x (n - k)) so the threads' accesses coalesce.
__global__ void __launch_bounds__(256) k_tsolve(const double* __restrict__ M, const int64_t* __restrict__ moff,
                                                const int32_t* __restrict__ nn, const int32_t* __restrict__ kk,
                                                const int64_t* __restrict__ toff, double* __restrict__ T) {
    const int b = blockIdx.y;
    const int n = nn[b], k = kk[b], w = n - k;
    const double* __restrict__ A = M + moff[b];
    double* __restrict__ Tb = T + toff[b];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < w; c += gridDim.x * blockDim.x) {
        for (int i = k - 1; i >= 0; --i) {
            const double* row = A + static_cast<int64_t>(i) * n;
            double s = row[k + c];
            for (int l = i + 1; l < k; ++l) s -= row[l] * Tb[static_cast<int64_t>(l) * w + c];
            Tb[static_cast<int64_t>(i) * w + c] = s / row[i];
        }
    }
}

template <class T>
struct DBuf {
    T* p = nullptr;
    size_t cap = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() {
        if (p) (void)hipFree(p);
    }
    T* need(size_t count) {
        if (count > cap) {
            if (p) SKF_BHIP(hipFree(p));
            p = nullptr;
            cap = 0;
            SKF_BHIP(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)));
            cap = std::max<size_t>(count, 1);
        }
        return p;
    }
    void put(const std::vector<T>& h) {
        need(h.size());
        if (!h.empty()) SKF_BHIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    void get(std::vector<T>& h, size_t count) const {
        h.resize(count);
        if (count) SKF_BHIP(hipMemcpy(h.data(), p, count * sizeof(T), hipMemcpyDeviceToHost));
    }
};

class DeviceSkeletonizer final : public LevelSkeletonizer {
public:
    explicit DeviceSkeletonizer(const Plan& p) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
            throw NotSupported("gpu_build needs a HIP device");
        pts_.put(p.pts);
        std::vector<double> U;
        half_ = proxy_pattern(p, U);
        np_ = static_cast<int>(U.size()) / p.dim;
        U_.put(U);
        m_ = p.kind == 1 ? 2 * np_ : np_;
    }

    void level(const Plan& p, int b0, int b1, std::vector<BoxSkel>& S) override {
        // boxes in batches whose proxy matrices fit the budget
        const size_t budget = size_t(1) << 29;   // doubles (4 GiB)
        int a = b0;
        while (a < b1) {
            size_t need = 0;
            int e = a;
            while (e < b1) {
                const size_t add = static_cast<size_t>(m_) * S[e].idx.size();
                if (e > a && need + add > budget) break;
                need += add;
                ++e;
            }
            batch(p, a, e, S);
            a = e;
        }
    }

private:
    void batch(const Plan& p, int a, int e, std::vector<BoxSkel>& S) {
        std::vector<int> boxes;
        for (int b = a; b < e; ++b) {
            if (S[b].idx.empty()) {
                S[b].k = 0;
                S[b].pos.clear();
                S[b].T.clear();
            } else {
                boxes.push_back(b);
            }
        }
        const int nbx = static_cast<int>(boxes.size());
        if (nbx == 0) return;
        std::vector<int32_t> nn(nbx), idx;
        std::vector<int64_t> ioff(nbx), moff(nbx), poff(nbx);
        std::vector<double> ctrh(4 * static_cast<size_t>(nbx), 0.0);
        int64_t io = 0, mo = 0, po = 0;
        int nmax = 0;
        for (int i = 0; i < nbx; ++i) {
            const int b = boxes[i];
            const int n = static_cast<int>(S[b].idx.size());
            nn[i] = n;
            nmax = std::max(nmax, n);
            ioff[i] = io;
            moff[i] = mo;
            poff[i] = po;
            for (int64_t x : S[b].idx) idx.push_back(static_cast<int32_t>(x));
            io += n;
            mo += static_cast<int64_t>(m_) * n;
            po += n;
            const double side = std::ldexp(p.root_side, -p.level[b]);
            for (int d = 0; d < p.dim; ++d) ctrh[4 * i + d] = p.root_lo[d] + (p.coord[3 * b + d] + 0.5) * side;
            ctrh[4 * i + 3] = half_ * side;
        }
        idx_.put(idx);
        ioff_.put(ioff);
        nn_.put(nn);
        ctrh_.put(ctrh);
        moff_.put(moff);
        poff_.put(poff);
        double* M = M_.need(static_cast<size_t>(mo));
        int32_t* perm = perm_.need(static_cast<size_t>(po));
        double* nrm = nrm_.need(2 * static_cast<size_t>(po));
        int32_t* kd = k_.need(nbx);
        const int gx = static_cast<int>(std::min<int64_t>(64, (static_cast<int64_t>(np_) * nmax + 255) / 256));
        hipLaunchKernelGGL(k_proxy_matrix, dim3(gx, nbx), dim3(256), 0, 0, pts_.p, p.dim, p.kind, p.kappa, idx_.p,
                           ioff_.p, nn_.p, ctrh_.p, U_.p, np_, moff_.p, M);
        SKF_BHIP(hipGetLastError());
        // one thread per column up to 1024; a power of two for the tree reductions
        int qt = 64;
        while (qt < nmax && qt < 1024) qt *= 2;
        hipLaunchKernelGGL(k_cpqr, dim3(nbx), dim3(qt), m_ * sizeof(double), 0, M, moff_.p, nn_.p, m_, p.tol, kd,
                           perm, poff_.p, nrm);
        SKF_BHIP(hipGetLastError());
        std::vector<int32_t> kk;
        k_.get(kk, nbx);
        std::vector<int64_t> toff(nbx);
        int64_t to = 0;
        int rmax = 0;
        for (int i = 0; i < nbx; ++i) {
            toff[i] = to;
            to += static_cast<int64_t>(kk[i]) * (nn[i] - kk[i]);
            rmax = std::max(rmax, nn[i] - kk[i]);
        }
        toff_.put(toff);
        double* T = T_.need(static_cast<size_t>(to));
        if (to > 0) {
            const int tx = std::min(16, (rmax + 255) / 256);
            hipLaunchKernelGGL(k_tsolve, dim3(tx, nbx), dim3(256), 0, 0, M, moff_.p, nn_.p, k_.p, toff_.p, T);
            SKF_BHIP(hipGetLastError());
        }
        std::vector<int32_t> ph;
        std::vector<double> Th;
        perm_.get(ph, static_cast<size_t>(po));
        T_.get(Th, static_cast<size_t>(to));
        for (int i = 0; i < nbx; ++i) {
            BoxSkel& s = S[boxes[i]];
            const int n = nn[i];
            s.k = kk[i];
            s.pos.assign(ph.begin() + poff[i], ph.begin() + poff[i] + n);
            // row-major k x (n - k) on the device, column-major in the plan
            const int64_t w = n - s.k;
            s.T.resize(static_cast<size_t>(s.k) * w);
            const double* src = Th.data() + toff[i];
            for (int64_t r = 0; r < s.k; ++r)
                for (int64_t c = 0; c < w; ++c) s.T[r + c * s.k] = src[r * w + c];
        }
    }

    int np_ = 0, m_ = 0;
    double half_ = 0.0;
    DBuf<double> pts_, U_, ctrh_, M_, nrm_, T_;
    DBuf<int32_t> idx_, nn_, perm_, k_;
    DBuf<int64_t> ioff_, moff_, poff_, toff_;
};

}  // namespace

std::unique_ptr<LevelSkeletonizer> make_device_skeletonizer(const Plan& p) {
    return std::make_unique<DeviceSkeletonizer>(p);
}

}  // namespace skelfmm
