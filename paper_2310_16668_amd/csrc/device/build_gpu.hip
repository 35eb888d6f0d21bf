// The interpolative decompositions of a tree level on the GPU (section 2.1,
// equation (5), the proxy-surface ID; section 3, "Build stage", Algorithm
// "Strong recursive skeletonization").  The host still builds the tree, the
// neighbor lists and every box's index set; per level, the device
//   1. evaluates the proxy matrices M = G(Y_B, X_B) of all boxes (m x n, stored
//      row by row; Helmholtz: m = 2 np rows, [Re M; Im M], which is unitarily
//      equivalent to the concatenation [M; conj M] of equation (5), so T is real),
//   2. runs column-pivoted Householder QR on each of them, one block per box
//      and one thread per column, so every step streams the trailing rows with
//      coalesced loads, in panels whose reflectors reach the trailing columns
//      once per panel; it stops at the first pivot with |R_jj| <= tol |R_11|
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
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "../hankel.h"
#include "../host/parallel.h"
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

// Sums over the block of cnt <= B per-thread values p[0 .. cnt): every
// thread receives them in out[0 .. cnt) (LDS).  wpart holds B x 16 doubles.
template <int B>
__device__ __forceinline__ void block_sums(const double (&p)[B], int cnt, double* wpart, double* out) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int l = 0; l < B; ++l) {
        if (l >= cnt) break;
        double v = p[l];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) wpart[l * 16 + wv] = v;
    }
    __syncthreads();
    if (tid < cnt) {
        double v = 0.0;
        for (int w = 0; w < nw; ++w) v += wpart[tid * 16 + w];
        out[tid] = v;
    }
    __syncthreads();
}

// Column-pivoted Householder QR of box blockIdx.x's m x n matrix A (row-major,
// in place), truncated at |R_jj| <= tol |R_11|, in panels of B pivots.  Within
// a panel the trailing columns are not updated: after reflectors 0 .. i - 1 of
// the panel the current matrix is A - sum_l v_l z_l^T, where z_l[c] = beta_l
// v_l^T (current column c) is kept per column (scratch), so pivot i needs one
// read of the trailing rows for z_i (corrected by the panel's Gram matrix
// v_i^T v_l) and the row j entries for the norm downdates; the panel's
// reflectors are applied to the trailing columns once, at its end.  Per pivot
// that reads the trailing matrix about (B + 2) / B times instead of three
// times; the pivots, the norm downdates and the stopping rule are those of the
// plain algorithm (in exact arithmetic the same factorization).  Thread t owns
// columns t, t + blockDim, ... (blockDim a power of two); perm receives the
// pivot order, kout k; scratch holds (2 + B) n doubles per box (running and
// reference column norms, z of the panel); V (dynamic LDS) B m doubles.
// rows per batch of a thread's column loops: their loads are issued together
constexpr int kRowBatch = 8;

template <int B>
__global__ void __launch_bounds__(1024) k_cpqr(double* __restrict__ M, const int64_t* __restrict__ moff,
                                               const int32_t* __restrict__ nn, int m, double tol,
                                               int32_t* __restrict__ kout, int32_t* __restrict__ perm,
                                               const int64_t* __restrict__ poff, double* __restrict__ scratch) {
    extern __shared__ double V[];   // the panel's Householder vectors, V[l m + r]
    __shared__ double wbest[16];
    __shared__ int wbi[16];
    __shared__ int piv_sh;
    __shared__ double wpart[B * 16];
    __shared__ double gsum[B];
    const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    double* __restrict__ A = M + moff[b];
    const int n = nn[b];
    int32_t* __restrict__ pm = perm + poff[b];
    double* __restrict__ nrm = scratch + (2 + B) * poff[b];
    double* __restrict__ ref = nrm + n;
    double* __restrict__ Z = ref + n;   // Z[l n + c]
    for (int c = tid; c < n; c += nt) {
        double s = 0.0;
        const double* __restrict__ col = A + c;
        int i = 0;
        for (; i + kRowBatch <= m; i += kRowBatch) {
            double a[kRowBatch];
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) a[u] = col[static_cast<int64_t>(i + u) * n];
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) s += a[u] * a[u];
        }
        for (; i < m; ++i) {
            const double x = col[static_cast<int64_t>(i) * n];
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
    int j = 0;
    bool stop = false;
    while (j < kmax && !stop) {
        const int j0 = j;
        const int jend = min(j0 + B, kmax);
        for (; j < jend; ++j) {
            const int i = j - j0;
            // pivot: the largest remaining norm, the lowest index on ties (a
            // total order on (norm, index): per thread, then across the wave
            // with shuffles, then across the waves)
            double best = -1.0;
            int bi = n;
            for (int c = j + tid; c < n; c += nt) {
                const double x = nrm[c];
                if (x > best) { best = x; bi = c; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double x = __shfl_xor(best, o);
                const int xi = __shfl_xor(bi, o);
                if (x > best || (x == best && xi < bi)) { best = x; bi = xi; }
            }
            if ((tid & 63) == 0) { wbest[tid >> 6] = best; wbi[tid >> 6] = bi; }
            __syncthreads();
            if (tid == 0) {
                for (int w = 1; w < (nt >> 6); ++w)
                    if (wbest[w] > best || (wbest[w] == best && wbi[w] < bi)) { best = wbest[w]; bi = wbi[w]; }
                piv_sh = bi;
            }
            __syncthreads();
            const int piv = piv_sh;
            if (piv != j) {
                for (int r = tid; r < m; r += nt) {
                    double* row = A + static_cast<int64_t>(r) * n;
                    const double t = row[j];
                    row[j] = row[piv];
                    row[piv] = t;
                }
                if (tid < i) {
                    const double t = Z[tid * n + j];
                    Z[tid * n + j] = Z[tid * n + piv];
                    Z[tid * n + piv] = t;
                }
                if (tid == 0) {
                    double t = nrm[j]; nrm[j] = nrm[piv]; nrm[piv] = t;
                    t = ref[j]; ref[j] = ref[piv]; ref[piv] = t;
                    const int32_t pt = pm[j]; pm[j] = pm[piv]; pm[piv] = pt;
                }
            }
            __syncthreads();
            // the current column j, rows j .. m - 1: the vector to reflect (into V
            // row i); its rows j0 .. j - 1 become R entries once the pivot is taken
            double zj[B];
#pragma unroll
            for (int l = 0; l < B; ++l) zj[l] = l < i ? Z[l * n + j] : 0.0;
            double sq[B];
#pragma unroll
            for (int l = 0; l < B; ++l) sq[l] = 0.0;
            for (int r = j + tid; r < m; r += nt) {
                double x = A[static_cast<int64_t>(r) * n + j];
#pragma unroll
                for (int l = 0; l < B; ++l)
                    if (l < i) x -= V[l * m + r] * zj[l];
                V[i * m + r] = x;
                sq[0] += x * x;
            }
            block_sums<B>(sq, 1, wpart, gsum);
            const double alpha = sqrt(gsum[0]);
            if (j == 0) r11 = alpha;
            if (!(alpha > tol * r11) || alpha == 0.0) {
                stop = true;
                break;
            }
            // Householder reflector H = I - beta v v^T with H x = rjj e1, v_j = 1
            const double x0 = V[i * m + j];
            const double rjj = x0 >= 0 ? -alpha : alpha;
            const double v0 = x0 - rjj;
            const double beta = -v0 / rjj;
            __syncthreads();
            for (int r = j0 + tid; r < m; r += nt) {
                if (r < j) {
                    // R entry: the column after the panel's reflectors so far (a stop
                    // leaves the column to the panel's end, which applies them)
                    double x = A[static_cast<int64_t>(r) * n + j];
#pragma unroll
                    for (int l = 0; l < B; ++l)
                        if (l < i) x -= V[l * m + r] * zj[l];
                    A[static_cast<int64_t>(r) * n + j] = x;
                    V[i * m + r] = 0.0;
                } else {
                    V[i * m + r] = r == j ? 1.0 : V[i * m + r] / v0;
                    A[static_cast<int64_t>(r) * n + j] = r == j ? rjj : 0.0;
                }
            }
            __syncthreads();
            // the panel's Gram row: g[l] = v_i^T v_l (rows >= j), l < i
#pragma unroll
            for (int l = 0; l < B; ++l) sq[l] = 0.0;
            for (int r = j + tid; r < m; r += nt) {
                const double vi = V[i * m + r];
#pragma unroll
                for (int l = 0; l < B; ++l)
                    if (l < i) sq[l] += vi * V[l * m + r];
            }
            block_sums<B>(sq, i, wpart, gsum);
            double g[B], vj[B];
#pragma unroll
            for (int l = 0; l < B; ++l) {
                g[l] = l < i ? gsum[l] : 0.0;
                vj[l] = l < i ? V[l * m + j] : 0.0;
            }
            // trailing columns: z_i[c] = beta v_i^T (A - sum_l v_l z_l^T)[:, c]
            // and the norm downdates with the updated row j
            for (int c = j + 1 + tid; c < n; c += nt) {
                const double* __restrict__ col = A + c;
                const double* __restrict__ vi = V + i * m;
                // four partial sums (rows r = 4 q + p go to partial p), added in order
                double dp[4] = {0.0, 0.0, 0.0, 0.0};
                int r = j;
                for (; r + kRowBatch <= m; r += kRowBatch) {
                    double a[kRowBatch];
#pragma unroll
                    for (int u = 0; u < kRowBatch; ++u) a[u] = col[static_cast<int64_t>(r + u) * n];
#pragma unroll
                    for (int u = 0; u < kRowBatch; ++u) dp[u & 3] += vi[r + u] * a[u];
                }
                for (; r < m; ++r) dp[(r - j) & 3] += vi[r] * col[static_cast<int64_t>(r) * n];
                double d = (dp[0] + dp[1]) + (dp[2] + dp[3]);
                double zc[B];
#pragma unroll
                for (int l = 0; l < B; ++l) zc[l] = l < i ? Z[l * n + c] : 0.0;
#pragma unroll
                for (int l = 0; l < B; ++l) d -= g[l] * zc[l];
                const double z = beta * d;
                Z[i * n + c] = z;
                double ajc = col[static_cast<int64_t>(j) * n] - z;
#pragma unroll
                for (int l = 0; l < B; ++l) ajc -= vj[l] * zc[l];
                double t = nrm[c] - ajc * ajc;
                if (t <= tol_norm2 * ref[c]) {
                    double s2 = 0.0;
                    for (int r = j + 1; r < m; ++r) {
                        double x = col[static_cast<int64_t>(r) * n] - V[i * m + r] * z;
#pragma unroll
                        for (int l = 0; l < B; ++l)
                            if (l < i) x -= V[l * m + r] * zc[l];
                        s2 += x * x;
                    }
                    t = s2;
                    ref[c] = t;
                }
                nrm[c] = t > 0.0 ? t : 0.0;
            }
            __syncthreads();
        }
        // the panel's reflectors on the trailing columns (from j: after a stop the
        // rejected column is trailing too), rows j0 .. m - 1
        const int nv = j - j0;
        if (nv > 0) {
            for (int c = j + tid; c < n; c += nt) {
                double zc[B];
#pragma unroll
                for (int l = 0; l < B; ++l) zc[l] = l < nv ? Z[l * n + c] : 0.0;
                double* __restrict__ col = A + c;
                int r = j0;
                for (; r + kRowBatch <= m; r += kRowBatch) {
                    double a[kRowBatch];
#pragma unroll
                    for (int u = 0; u < kRowBatch; ++u) a[u] = col[static_cast<int64_t>(r + u) * n];
#pragma unroll
                    for (int u = 0; u < kRowBatch; ++u) {
#pragma unroll
                        for (int l = 0; l < B; ++l)
                            if (l < nv) a[u] -= V[l * m + r + u] * zc[l];
                        col[static_cast<int64_t>(r + u) * n] = a[u];
                    }
                }
                for (; r < m; ++r) {
                    double x = col[static_cast<int64_t>(r) * n];
#pragma unroll
                    for (int l = 0; l < B; ++l)
                        if (l < nv) x -= V[l * m + r] * zc[l];
                    col[static_cast<int64_t>(r) * n] = x;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) kout[b] = j;
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
            int l = i + 1;
            for (; l + kRowBatch <= k; l += kRowBatch) {
                double t[kRowBatch];
#pragma unroll
                for (int u = 0; u < kRowBatch; ++u) t[u] = Tb[static_cast<int64_t>(l + u) * w + c];
#pragma unroll
                for (int u = 0; u < kRowBatch; ++u) s -= row[l + u] * t[u];
            }
            for (; l < k; ++l) s -= row[l] * Tb[static_cast<int64_t>(l) * w + c];
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
        // boxes in batches whose proxy matrices fit the budget, at most 65,535 per
        // batch (the grid's y extent of the per-box launches)
        const size_t budget = size_t(1) << 30;   // doubles (8 GiB): a level of the 1M cube in one launch
        const int max_boxes = 65535;
        int a = b0;
        while (a < b1) {
            size_t need = 0;
            int e = a;
            while (e < b1) {
                const size_t add = static_cast<size_t>(m_) * S[e].idx.size();
                if (e > a && (need + add > budget || e - a >= max_boxes)) break;
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
        // panels of up to 8 pivots: the panel's Householder vectors (panel x m
        // doubles) stay within 40 KiB of LDS; blocks of one wave (boxes of at most
        // 64 entries) take panels of 4 so that more of them share a CU
        int panel = m_ <= 640 ? 8 : (m_ <= 1280 ? 4 : (m_ <= 2560 ? 2 : 1));
        if (nmax <= 64) panel = std::min(panel, 4);
        if (m_ > 5120) throw NotSupported("gpu_build supports proxy matrices of at most 5120 rows");
        double* nrm = nrm_.need(static_cast<size_t>(2 + panel) * static_cast<size_t>(po));
        int32_t* kd = k_.need(nbx);
        const int gx = static_cast<int>(std::min<int64_t>(64, (static_cast<int64_t>(np_) * nmax + 255) / 256));
        hipLaunchKernelGGL(k_proxy_matrix, dim3(gx, nbx), dim3(256), 0, 0, pts_.p, p.dim, p.kind, p.kappa, idx_.p,
                           ioff_.p, nn_.p, ctrh_.p, U_.p, np_, moff_.p, M);
        SKF_BHIP(hipGetLastError());
        // one thread per column up to 1024; a power of two for the tree reductions
        int qt = 64;
        while (qt < nmax && qt < 1024) qt *= 2;
        const auto qr = [&](auto kern_fn) {
            hipLaunchKernelGGL(kern_fn, dim3(nbx), dim3(qt), static_cast<size_t>(panel) * m_ * sizeof(double), 0, M,
                               moff_.p, nn_.p, m_, p.tol, kd, perm, poff_.p, nrm);
        };
        if (panel == 8) qr(k_cpqr<8>);
        else if (panel == 4) qr(k_cpqr<4>);
        else if (panel == 2) qr(k_cpqr<2>);
        else qr(k_cpqr<1>);
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
        perm_.get(ph, static_cast<size_t>(po));
        // T comes back through a pinned staging buffer, a run of whole boxes at a
        // time (a pageable copy of the level's T ran at a fraction of the link)
        const int threads = host_threads(p.opt.num_threads);
        // the batch's T, column-major per box, stays here until the plan copies it
        blocks_.emplace_back(new double[static_cast<size_t>(std::max<int64_t>(to, 1))]);
        double* const blk = blocks_.back().get();
        const auto end_of = [&](int i) { return i + 1 < nbx ? toff[i + 1] : to; };   // end of box i's T
        for (int i0 = 0; i0 < nbx;) {
            // boxes i0 .. i1 - 1: as many as fit the staging buffer (at least one)
            int i1 = i0 + 1;
            while (i1 < nbx && end_of(i1) - toff[i0] <= static_cast<int64_t>(kStageDoubles)) ++i1;
            const int64_t t0 = toff[i0], t1 = end_of(i1 - 1);
            const double* src0 = nullptr;
            std::unique_ptr<double[]> big;
            if (t1 - t0 <= static_cast<int64_t>(kStageDoubles)) {
                double* st = stage();
                if (t1 > t0)
                    SKF_BHIP(hipMemcpy(st, T + t0, static_cast<size_t>(t1 - t0) * sizeof(double),
                                       hipMemcpyDeviceToHost));
                src0 = st;
            } else {   // one box larger than the staging buffer
                big.reset(new double[static_cast<size_t>(t1 - t0)]);
                SKF_BHIP(hipMemcpy(big.get(), T + t0, static_cast<size_t>(t1 - t0) * sizeof(double),
                                   hipMemcpyDeviceToHost));
                src0 = big.get();
            }
            parallel_for(i1 - i0, threads, [&](int64_t q) {
                const int i = i0 + static_cast<int>(q);
                BoxSkel& s = S[boxes[i]];
                const int n = nn[i];
                s.k = kk[i];
                s.pos.assign(ph.begin() + poff[i], ph.begin() + poff[i] + n);
                // row-major k x (n - k) on the device, column-major in the plan
                const int64_t w = n - s.k;
                const double* src = src0 + (toff[i] - t0);
                double* dst = blk + toff[i];
                for (int64_t r = 0; r < s.k; ++r)
                    for (int64_t c = 0; c < w; ++c) dst[r + c * s.k] = src[r * w + c];
                s.T.clear();
                s.Tsrc = dst;
                s.Tn = s.k * w;
            }, 16);
            i0 = i1;
        }
    }

    // the pinned staging buffer, allocated on first use and kept for the build
    static constexpr size_t kStageDoubles = size_t(1) << 25;   // 256 MiB
    double* stage() {
        if (!stage_) {
            void* h = nullptr;
            SKF_BHIP(hipHostMalloc(&h, kStageDoubles * sizeof(double), hipHostMallocDefault));
            stage_ = static_cast<double*>(h);
        }
        return stage_;
    }
    double* stage_ = nullptr;
    std::vector<std::unique_ptr<double[]>> blocks_;

public:
    ~DeviceSkeletonizer() override {
        if (stage_) (void)hipHostFree(stage_);
    }

private:

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
