// GPU sweep of the FMM apply (section 3, "FMM apply"; Algorithm "FMM apply").
//
// One sweep is: gather charges into leaf entries -> upward pass, one launch per
// level (qhat = q[0:k] + T q[k:n], written to the box's skeleton vector and,
// through pmap, into its parent's entries) -> one near-field launch over every
// level (ifo, ifs, tfo and the top-level direct sum) -> downward pass, one
// launch per level (uhat += parent's u at the box's slots; u[0:k] += uhat;
// u[k:n] += T^T uhat; leaves write the caller's output) -> output of the
// top-level leaves.
//
// The near field is the hot loop.  A work item is one wavefront: `TPL` targets
// per lane (64 TPL consecutive entries of one target box) against every source
// box on the target's segment list.  Source data is wave-uniform, so it is read
// with scalar loads into SGPRs and used directly as VALU operands: no LDS
// staging, no barriers; each lane keeps its targets and accumulators in VGPRs.
// The skeleton part of a source box comes first in its entries, so the uhat
// update (one extra FMA per skeleton pair, the sub-block reuse of section 4)
// runs over a prefix of the same loop.
//
// Precision policies:
//   F64   coordinates, kernel and accumulators in float64;
//   F32   coordinates and kernel in float32, accumulators in float64 (the
//         float64 FMA issues at the float32 rate on CDNA4, so the wider
//         accumulator costs one conversion per pair);
//   C128 / C64 the complex analogues; C64 with f64_leaf evaluates in float64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace skelfmm {
namespace kern {

constexpr double kInv4Pi = 0.079577471545947667884441881686257;  // 1 / (4 pi)

template <typename R>
struct alignas(4 * sizeof(R)) Rec4 { R x, y, z, w; };

// ---------------------------------------------------------------------------
// kernel values without the 1/(4 pi) factor; zero at r = 0 (the excluded
// diagonal and coincident points)
// ---------------------------------------------------------------------------

// 2/r in float64: hardware reciprocal square root y ~ 1/r refined by one
// Newton step for f(y) = 1/y^2 - r2, which gives y (3 - r2 y^2) / 2; the
// factor 1/2 is folded into the final scale, so this returns 2/r.  At r2 = 0
// the step yields NaN, and max(NaN, 0) = 0 (IEEE maxNum) removes the pair.
__device__ __forceinline__ double two_inv_r(double r2) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double t = r2 * y;
    const double e = fma(-t, y, 3.0);
    return fmax(y * e, 0.0);
}
__device__ __forceinline__ double inv_r(double r2) { return 0.5 * two_inv_r(r2); }
__device__ __forceinline__ float inv_r(float r2) {
    const float y = __builtin_amdgcn_rsqf(r2);
    return r2 > 0.0f ? y : 0.0f;
}

// -log(r2) (= -2 log r); zero at r2 = 0
__device__ __forceinline__ double neg_log_r2(double r2) { return r2 > 0.0 ? -log(r2) : 0.0; }
__device__ __forceinline__ float neg_log_r2(float r2) { return r2 > 0.0f ? -__logf(r2) : 0.0f; }

__device__ __forceinline__ void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }

template <typename R, typename A, typename V, int DIM, int KIND>
struct Pol {
    using Rt = R;   // coordinates / kernel evaluation
    using At = A;   // accumulators
    using Vt = V;   // stored vectors
    static constexpr int dim = DIM;
    static constexpr int kind = KIND;   // 0 Laplace, 1 Helmholtz
    static constexpr int nv = KIND == 1 ? 2 : 1;
    // 3D Laplace in float64 evaluates 2/r (see two_inv_r); the factor is undone in the scale
    static constexpr bool twice = DIM == 3 && KIND == 0 && sizeof(R) == 8;
    static constexpr double gscale = twice ? 0.5 : 1.0;
};

// G(x_t, x_s) (times 4 pi for 3D, times 4 pi / 2 for 2D: the common factor is
// applied once at the end).  Real kernels return gr only.
template <class P, bool CONJ>
__device__ __forceinline__ void green(typename P::Rt dx, typename P::Rt dy, typename P::Rt dz,
                                      typename P::Rt kappa, typename P::Rt& gr, typename P::Rt& gi) {
    using R = typename P::Rt;
    R r2 = dx * dx;
    r2 = fma(dy, dy, r2);
    if constexpr (P::dim == 3) r2 = fma(dz, dz, r2);
    if constexpr (P::kind == 0) {
        if constexpr (P::twice) gr = two_inv_r(r2);
        else if constexpr (P::dim == 3) gr = inv_r(r2);
        else gr = neg_log_r2(r2);
        gi = R(0);
    } else {
        const R ir = inv_r(r2);
        const R r = r2 * ir;
        R s, c;
        sin_cos(kappa * r, &s, &c);
        gr = c * ir;
        gi = CONJ ? -s * ir : s * ir;
    }
}

// ---------------------------------------------------------------------------
// gather / scatter of leaf entries
// ---------------------------------------------------------------------------
template <typename VI, typename VO>
__global__ void k_gather(const int32_t* __restrict__ dst_e, const int32_t* __restrict__ src_p, int64_t cnt,
                         int W, const VI* __restrict__ in, VO* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cnt * W) return;
    const int64_t r = i / W, c = i - r * W;
    out[static_cast<int64_t>(dst_e[r]) * W + c] = static_cast<VO>(in[static_cast<int64_t>(src_p[r]) * W + c]);
}

template <typename VI, typename VO>
__global__ void k_scatter(const int32_t* __restrict__ src_e, const int32_t* __restrict__ dst_p, int64_t cnt,
                          int W, const VI* __restrict__ in, VO* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cnt * W) return;
    const int64_t r = i / W, c = i - r * W;
    out[static_cast<int64_t>(dst_p[r]) * W + c] = static_cast<VO>(in[static_cast<int64_t>(src_e[r]) * W + c]);
}

// ---------------------------------------------------------------------------
// upward pass, one block per box of a level:
//   qhat[i] = q[i] + sum_j T[i + j k] q[k + j]     (i < k)
// lanes own rows i, the block's four waves split the columns j, LDS reduces.
// ---------------------------------------------------------------------------
struct BoxArgs {
    const int64_t* voff;
    const int64_t* hoff;
    const int64_t* toff;
    const int32_t* nb;
    const int32_t* kb;
    const int32_t* is_leaf;
    const int32_t* level;
    const int32_t* pmap;
    const int32_t* perm;
};

template <typename V, typename TT>
__global__ void __launch_bounds__(256) k_upward(BoxArgs a, int b0, int W, const TT* __restrict__ T,
                                               V* __restrict__ Q, V* __restrict__ Qh) {
    __shared__ double part[4][64];
    const int b = b0 + blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t voff = a.voff[b], hoff = a.hoff[b];
    const int n = a.nb[b], k = a.kb[b];
    const int m = n - k;
    const TT* Tb = T + a.toff[b];
    for (int c = 0; c < W; ++c) {
        for (int r0 = 0; r0 < k; r0 += 64) {
            const int i = r0 + lane;
            double acc = 0.0;
            if (i < k)
                for (int j = wave; j < m; j += 4)
                    acc = fma(static_cast<double>(Tb[i + static_cast<int64_t>(j) * k]),
                              static_cast<double>(Q[(voff + k + j) * W + c]), acc);
            part[wave][lane] = acc;
            __syncthreads();
            if (wave == 0 && i < k) {
                const double s = static_cast<double>(Q[(voff + i) * W + c]) + part[0][lane] + part[1][lane] +
                                 part[2][lane] + part[3][lane];
                const V v = static_cast<V>(s);
                Qh[(hoff + i) * W + c] = v;
                Q[static_cast<int64_t>(a.pmap[hoff + i]) * W + c] = v;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// downward pass, one block per box of a level:
//   uhat = Uh + U_parent[pmap]; u[i] += uhat[i] (i < k); u[k+j] += sum_i T[i + j k] uhat[i]
// a leaf writes its final potential to the caller's output instead of U.
// Columns of T are contiguous: a wave reads a column with consecutive lanes
// and reduces across the wave.
// ---------------------------------------------------------------------------
template <typename V, typename TT, typename VO>
__global__ void __launch_bounds__(256) k_downward(BoxArgs a, int b0, int W, const TT* __restrict__ T,
                                                 const V* __restrict__ Uh, V* __restrict__ U,
                                                 VO* __restrict__ out) {
    extern __shared__ double uh_s[];
    const int b = b0 + blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t voff = a.voff[b], hoff = a.hoff[b];
    const int n = a.nb[b], k = a.kb[b];
    const int m = n - k;
    const bool leaf = a.is_leaf[b] != 0;
    const TT* Tb = T + a.toff[b];
    for (int c = 0; c < W; ++c) {
        for (int i = threadIdx.x; i < k; i += blockDim.x) {
            const double uh = static_cast<double>(Uh[(hoff + i) * W + c]) +
                              static_cast<double>(U[static_cast<int64_t>(a.pmap[hoff + i]) * W + c]);
            uh_s[i] = uh;
            const double u = static_cast<double>(U[(voff + i) * W + c]) + uh;
            if (leaf) out[static_cast<int64_t>(a.perm[voff + i]) * W + c] = static_cast<VO>(u);
            else U[(voff + i) * W + c] = static_cast<V>(u);
        }
        __syncthreads();
        for (int j = wave; j < m; j += 4) {
            const TT* col = Tb + static_cast<int64_t>(j) * k;
            double acc = 0.0;
            for (int i = lane; i < k; i += 64) acc = fma(static_cast<double>(col[i]), uh_s[i], acc);
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) {
                const double u = static_cast<double>(U[(voff + k + j) * W + c]) + acc;
                if (leaf) out[static_cast<int64_t>(a.perm[voff + k + j]) * W + c] = static_cast<VO>(u);
                else U[(voff + k + j) * W + c] = static_cast<V>(u);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// near field: ifo, ifs, tfo and the top-level direct sum in one launch
// ---------------------------------------------------------------------------
// Per-box record read with one scalar load.
struct alignas(32) BoxRec {
    int64_t voff;     // first entry
    int64_t hoff;     // first skeleton entry
    int32_t n;        // entries
    int32_t k;        // skeleton entries (0 at and above the top level)
    int32_t level;
    int32_t leaf;
};

// MODE 0: u += G w ;  1: u += G w, uh -= G wh ;  2: u += G w, uh -= G w ;  3: u += G (w - wh)
template <class P, int TPL, bool CONJ, int MODE>
__device__ __forceinline__ void near_loop(const Rec4<typename P::Rt>* __restrict__ X,
                                          const typename P::Vt* __restrict__ Q,
                                          const typename P::Vt* __restrict__ Qh, int s0, int s1,
                                          typename P::Rt kappa,
                                          const typename P::Rt (&xt)[TPL], const typename P::Rt (&yt)[TPL],
                                          const typename P::Rt (&zt)[TPL],
                                          typename P::At (&acc)[TPL][P::nv], typename P::At (&acch)[TPL][P::nv]) {
    using R = typename P::Rt;
    using A = typename P::At;
    constexpr int nv = P::nv;
#pragma unroll 2
    for (int s = s0; s < s1; ++s) {
        const Rec4<R> xs = X[s];
        A w[nv], wh[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            w[v] = static_cast<A>(Q[s * nv + v]);
            if constexpr (MODE == 1 || MODE == 3) wh[v] = static_cast<A>(Qh[s * nv + v]);
            if constexpr (MODE == 3) w[v] -= wh[v];
        }
#pragma unroll
        for (int p = 0; p < TPL; ++p) {
            R gr, gi;
            green<P, CONJ>(xt[p] - xs.x, yt[p] - xs.y, zt[p] - xs.z, kappa, gr, gi);
            const A g = static_cast<A>(gr);
            if constexpr (nv == 1) {
                acc[p][0] = fma(g, w[0], acc[p][0]);
                if constexpr (MODE == 1) acch[p][0] = fma(-g, wh[0], acch[p][0]);
                if constexpr (MODE == 2) acch[p][0] = fma(-g, w[0], acch[p][0]);
            } else {
                const A h = static_cast<A>(gi);
                acc[p][0] = fma(g, w[0], fma(-h, w[1], acc[p][0]));
                acc[p][1] = fma(g, w[1], fma(h, w[0], acc[p][1]));
                if constexpr (MODE == 1) {
                    acch[p][0] = fma(-g, wh[0], fma(h, wh[1], acch[p][0]));
                    acch[p][1] = fma(-g, wh[1], fma(-h, wh[0], acch[p][1]));
                }
                if constexpr (MODE == 2) {
                    acch[p][0] = fma(-g, w[0], fma(h, w[1], acch[p][0]));
                    acch[p][1] = fma(-g, w[1], fma(-h, w[0], acch[p][1]));
                }
            }
        }
    }
}

// One wavefront per work item; every pointer is a separate restrict argument so
// the compiler can prove the source data is never written by this kernel and
// read it with scalar loads.
template <class P, int TPL, bool CONJ>
__global__ void __launch_bounds__(256) k_near(const Task* __restrict__ tasks, int ntasks, int top,
                                              const int32_t* __restrict__ seg_ptr, const int2* __restrict__ segs,
                                              const BoxRec* __restrict__ box,
                                              const Rec4<typename P::Rt>* __restrict__ X,
                                              const typename P::Vt* __restrict__ Q,
                                              const typename P::Vt* __restrict__ Qh,
                                              typename P::Vt* __restrict__ U, typename P::Vt* __restrict__ Uh,
                                              typename P::Rt kappa, double scale) {
    using R = typename P::Rt;
    using A = typename P::At;
    using V = typename P::Vt;
    constexpr int nv = P::nv;
    const int lane = threadIdx.x & 63;
    const int tid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tid >= ntasks) return;
    const Task tk = tasks[tid];
    const BoxRec tb = box[tk.box];
    const bool has_h = tb.level > top && tk.t0 < tb.k;

    R xt[TPL], yt[TPL], zt[TPL];
    A acc[TPL][nv], acch[TPL][nv];
#pragma unroll
    for (int p = 0; p < TPL; ++p) {
        const int t = min(tk.t0 + lane + 64 * p, tb.n - 1);
        const Rec4<R> x = X[tb.voff + t];
        xt[p] = x.x; yt[p] = x.y; zt[p] = x.z;
#pragma unroll
        for (int v = 0; v < nv; ++v) { acc[p][v] = A(0); acch[p][v] = A(0); }
    }
    const int e1 = seg_ptr[tk.box + 1];
    for (int e = seg_ptr[tk.box]; e < e1; ++e) {
        const int2 sg = segs[e];
        const BoxRec sb = box[sg.x];
        const Rec4<R>* Xs = X + sb.voff;
        const V* Qs = Q + sb.voff * nv;
        const V* Qhs = Qh + sb.hoff * nv;
        if (sg.y == SEG_IFO) {
            if (has_h) {
                near_loop<P, TPL, CONJ, 1>(Xs, Qs, Qhs, 0, sb.k, kappa, xt, yt, zt, acc, acch);
                near_loop<P, TPL, CONJ, 0>(Xs, Qs, Qhs, sb.k, sb.n, kappa, xt, yt, zt, acc, acch);
            } else {
                near_loop<P, TPL, CONJ, 0>(Xs, Qs, Qhs, 0, sb.n, kappa, xt, yt, zt, acc, acch);
            }
        } else if (sg.y == SEG_IFS) {
            if (has_h) near_loop<P, TPL, CONJ, 2>(Xs, Qs, Qhs, 0, sb.n, kappa, xt, yt, zt, acc, acch);
            else near_loop<P, TPL, CONJ, 0>(Xs, Qs, Qhs, 0, sb.n, kappa, xt, yt, zt, acc, acch);
        } else if (sg.y == SEG_TFO) {
            near_loop<P, TPL, CONJ, 3>(Xs, Qs, Qhs, 0, sb.k, kappa, xt, yt, zt, acc, acch);
            near_loop<P, TPL, CONJ, 0>(Xs, Qs, Qhs, sb.k, sb.n, kappa, xt, yt, zt, acc, acch);
        } else {
            near_loop<P, TPL, CONJ, 0>(Xs, Qs, Qhs, 0, sb.n, kappa, xt, yt, zt, acc, acch);
        }
    }
    const A sc = static_cast<A>(scale * P::gscale);
#pragma unroll
    for (int p = 0; p < TPL; ++p) {
        const int t = tk.t0 + lane + 64 * p;
        if (t < tb.n) {
#pragma unroll
            for (int v = 0; v < nv; ++v) U[(tb.voff + t) * nv + v] = static_cast<V>(acc[p][v] * sc);
            if (has_h && t < tb.k) {
#pragma unroll
                for (int v = 0; v < nv; ++v) Uh[(tb.hoff + t) * nv + v] = static_cast<V>(acch[p][v] * sc);
            }
        }
    }
}

}  // namespace kern
}  // namespace skelfmm
