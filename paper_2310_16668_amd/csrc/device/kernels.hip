// GPU sweep of the FMM apply (section 3, "FMM apply"; Algorithm "FMM apply").
//
// One sweep is: gather charges into leaf entries -> upward pass, one launch per
// level (qhat = q[0:k] + T q[k:n], written to the box's skeleton vector and,
// through pmap, into its parent's entries) -> one near-field launch over every
// level (ifo, ifs, tfo and the top-level direct sum) -> downward pass, one
// launch per level (uhat += parent's u at the box's slots; u[0:k] += uhat;
// u[k:n] += T^T uhat) -> scatter of the leaf entries to the caller's output.
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
// Precision.  Coordinates, their differences and |d|^2 are always float64:
// float32 differences of nearby points lose their relative precision whenever
// the points sit far from the coordinate origin (a clustered surface).  A
// float64 add or multiply-add issues in four cycles per wavefront against two
// for a float32 multiply-add, so |d|^2 costs about as much as the reciprocal
// square root; the pair kernel's expanded form keeps it to one add and three
// multiply-adds.  Policies:
//   F64   kernel value and accumulators in float64 (reciprocal square root
//         refined by one Newton step);
//   F32   |d|^2 rounded once to float32, kernel value (reciprocal square root,
//         log, sincos) in float32, accumulators in float64, stored vectors and
//         transfer matrices in float32;
//   C128 / C64 the complex analogues; C64 with f64_leaf evaluates in float64.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "../hankel.h"
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
// 1/r in float32.  A zero distance can only occur when a box is paired with
// itself (points at one position fall in one box at every level), so only
// those segments pay for the r = 0 test (MASK).
template <bool MASK>
__device__ __forceinline__ float inv_r_f(float r2) {
    const float y = __builtin_amdgcn_rsqf(r2);
    if constexpr (MASK) return r2 > 0.0f ? y : 0.0f;
    return y;
}

// -log(r2) (= -2 log r); zero at r2 = 0
__device__ __forceinline__ double neg_log_r2(double r2) { return r2 > 0.0 ? -log(r2) : 0.0; }
__device__ __forceinline__ float neg_log_r2(float r2) { return r2 > 0.0f ? -__logf(r2) : 0.0f; }

__device__ __forceinline__ void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }

template <typename R, typename A, typename V, int DIM, int KIND, bool COMP = false, int RHS = 1>
struct Pol {
    using Rt = R;   // kernel evaluation (coordinates are float64 in every policy)
    using At = A;   // accumulators
    using Vt = V;   // stored vectors
    static constexpr int dim = DIM;
    static constexpr int kind = KIND;   // 0 Laplace, 1 Helmholtz
    // float32 pair kernel: partial sums of at most four products before they
    // reach float64, column sums over the lanes in float64
    static constexpr bool comp = COMP;
    // values per entry: the real and imaginary parts of a complex kernel's
    // vector, or RHS interleaved columns of a real kernel (a forward apply and
    // an adjoint apply share one sweep: for a real symmetric kernel the
    // adjoint's kernel values are the forward's)
    static constexpr int rhs = RHS;
    static_assert(KIND == 0 || RHS == 1, "interleaved columns are for real kernels");
    static constexpr int nv = KIND == 1 ? 2 : RHS;
    // 3D Laplace in float64 evaluates 2/r (see two_inv_r); the factor is undone in the scale
    static constexpr bool twice = DIM == 3 && KIND == 0 && sizeof(R) == 8;
    static constexpr double gscale = twice ? 0.5 : 1.0;
};
// The same policy with the pair kernel's compensated leaf sums.
template <class P>
using WithComp = Pol<typename P::Rt, typename P::At, typename P::Vt, P::dim, P::kind, true, P::rhs>;

// G(x_t, x_s) without the common factor kscale (for 2D Laplace: -log r^2, the
// kernel times 4 pi; for 2D Helmholtz: i H0^(1)(kappa r), the kernel times 4),
// applied once at the end.  MASK: zero the pair at r = 0
// (only needed where a box meets itself).  Real kernels return gr only.
// The common factor applied once at the end: 1 / (4 pi) for the 3D kernels and
// for 2D Laplace (evaluated as -log r^2), 1/4 for 2D Helmholtz (evaluated as
// i H0^(1)).
template <class P>
constexpr double kscale() { return (P::dim == 2 && P::kind == 1) ? 0.25 : kInv4Pi; }

template <class P, bool CONJ, bool MASK>
__device__ __forceinline__ void green_r2(double r2d, typename P::Rt kappa, typename P::Rt& gr,
                                         typename P::Rt& gi) {
    using R = typename P::Rt;
    if constexpr (P::dim == 2 && P::kind == 1) {
        // i H0^(1)(kappa r) = -Y0 + i J0, evaluated in float64 in every policy
        double j0 = 0.0, y0 = 0.0;
        if (r2d > 0.0) hankel::h0(static_cast<double>(kappa) * sqrt(r2d), &j0, &y0);
        gr = static_cast<R>(-y0);
        gi = static_cast<R>(CONJ ? -j0 : j0);
        return;
    }
    const R r2 = static_cast<R>(r2d);
    R ir;
    if constexpr (sizeof(R) == 8) ir = (P::twice) ? two_inv_r(r2) : inv_r(r2);
    else ir = inv_r_f<MASK>(r2);
    if constexpr (P::kind == 0) {
        if constexpr (P::dim == 3) gr = ir;
        else gr = (sizeof(R) == 8 || MASK) ? neg_log_r2(r2) : -__logf(r2);
        gi = R(0);
    } else {
        const R r = r2 * ir;
        R s, c;
        sin_cos(kappa * r, &s, &c);
        gr = c * ir;
        gi = CONJ ? -s * ir : s * ir;
    }
}

template <class P, bool CONJ, bool MASK>
__device__ __forceinline__ void green(double dx, double dy, double dz, typename P::Rt kappa,
                                      typename P::Rt& gr, typename P::Rt& gi) {
    double r2d = dx * dx;
    r2d = fma(dy, dy, r2d);
    if constexpr (P::dim == 3) r2d = fma(dz, dz, r2d);
    green_r2<P, CONJ, MASK>(r2d, kappa, gr, gi);
}

// Per-box record read with one scalar load.
struct alignas(32) BoxRec {
    int64_t voff;     // first entry
    int64_t hoff;     // first skeleton entry
    int32_t n;        // entries
    int32_t k;        // skeleton entries (0 at and above the top level)
    int64_t roff;     // first expanded source record of the pair kernel
};

// ---------------------------------------------------------------------------
// transfers with one right-hand side: batched GEMVs over the boxes of a level.
// A block owns one (box, group of RowMap<TT>::group rows); each lane holds the
// rows of one 8-byte load (one float64 or two float32 values; the columns are
// padded to 128-byte lines, so a load never straddles a column).  The columns
// are cut into at most chunks_max chunks whose length depends only on the box;
// the block's nw waves take chunks round-robin and the partials are added in
// chunk order, so the result does not depend on nw (a batch and a single apply
// agree bit for bit).  The vector entry of a column is wave-uniform (a scalar
// load).
// ---------------------------------------------------------------------------
template <int NV>
constexpr int chunks_max() { return 16 / NV; }

template <int NV>
__device__ __forceinline__ int chunk_len(int cols) {
    const int nch = min(chunks_max<NV>(), (cols + 31) / 32);
    return nch > 0 ? (cols + nch - 1) / nch : 0;
}

// leading dimension of a padded column of T or T^T (columns start on 128-byte lines)
__device__ __forceinline__ int64_t ld_pad(int x) { return (x + kTPad - 1) / kTPad * kTPad; }

template <typename TT>
struct Vec8;
template <>
struct Vec8<float> { using type = float2; };
template <>
struct Vec8<double> { using type = double; };

// Rows of a group: lane l holds rows vec l .. vec l + vec - 1.
template <typename TT>
struct RowMap {
    static constexpr int vec = 8 / static_cast<int>(sizeof(TT));
    static constexpr int group = 64 * vec;
};

// acc[e] += sum over columns c in [c0, c1) of A[lane row e, c] x[c], A column-major
// with leading dimension ld starting at the group's first row.
template <typename TT, int NV, typename XF>
__device__ __forceinline__ void gemv_chunk(const TT* __restrict__ A, int64_t ld, int rows, int lane, int c0,
                                           int c1, XF xf, double (&acc)[RowMap<TT>::vec][NV]) {
    using M = RowMap<TT>;
    using VT = typename Vec8<TT>::type;
    if (M::vec * lane >= rows) return;
#pragma unroll 4
    for (int c = c0; c < c1; ++c) {
        double x[NV];
        xf(c, x);
        const VT t = *reinterpret_cast<const VT*>(A + M::vec * lane + c * ld);
        const TT* te = reinterpret_cast<const TT*>(&t);
#pragma unroll
        for (int e = 0; e < M::vec; ++e)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[e][v] = fma(static_cast<double>(te[e]), x[v], acc[e][v]);
    }
}

// upward: qhat = q[0:k] + T q[k:n], written to Qh and to the parent's entries.
// Qin / Qout are the same workspace: reads touch this level's entries, writes
// the parent level's, so the two never overlap.
template <typename V, typename TT, int NV>
__global__ void __launch_bounds__(1024) k_up_gemv(const int2* __restrict__ work, const BoxRec* __restrict__ box,
                                                  const int64_t* __restrict__ toff,
                                                  const int32_t* __restrict__ pmap, const TT* __restrict__ T,
                                                  const V* __restrict__ Qin, V* __restrict__ Qout,
                                                  V* __restrict__ Qh, int nw) {
    using M = RowMap<TT>;
    constexpr int NC = chunks_max<NV>();
    __shared__ double part[NC][M::group * NV];
    const int2 wk = work[blockIdx.x];
    const BoxRec tb = box[wk.x];
    const int k = tb.k, m = tb.n - tb.k;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = wk.y * M::group;
    const TT* __restrict__ Tb = T + toff[wk.x] + r0;
    const int64_t ldk = ld_pad(k);
    const V* __restrict__ xr = Qin + (tb.voff + k) * NV;
    const int ch = chunk_len<NV>(m);
    const int nch = ch > 0 ? (m + ch - 1) / ch : 0;
    for (int c = wave; c < nch; c += nw) {
        double acc[M::vec][NV];
#pragma unroll
        for (int r = 0; r < M::vec; ++r)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[r][v] = 0.0;
        gemv_chunk<TT, NV>(Tb, ldk, k - r0, lane, c * ch, min(m, (c + 1) * ch),
                           [&](int j, double (&x)[NV]) {
#pragma unroll
                               for (int v = 0; v < NV; ++v) x[v] = static_cast<double>(xr[j * NV + v]);
                           },
                           acc);
#pragma unroll
        for (int e = 0; e < M::vec; ++e)
#pragma unroll
            for (int v = 0; v < NV; ++v) part[c][(M::vec * lane + e) * NV + v] = acc[e][v];
    }
    __syncthreads();
    const int rows = min(M::group, k - r0);
    for (int t = threadIdx.x; t < rows * NV; t += blockDim.x) {
        const int r = t / NV, v = t - r * NV;
        const int i = r0 + r;
        double sum = static_cast<double>(Qin[(tb.voff + i) * NV + v]);
        for (int c = 0; c < nch; ++c) sum += part[c][t];
        const V val = static_cast<V>(sum);
        Qh[(tb.hoff + i) * NV + v] = val;
        Qout[static_cast<int64_t>(pmap[tb.hoff + i]) * NV + v] = val;
    }
}

// The same two passes on a level of uncompressed boxes (k = n, no T), whose
// entries e0 + j and skeleton entries h0 + j correspond one to one: one
// thread per value instead of a block per box (the leaf level of a uniform
// cube holds 32,768 such boxes of ~32 points).  The arithmetic is that of
// k_up_gemv / k_down_gemv for such a box.
template <typename V, int NV>
__global__ void __launch_bounds__(256) k_up_flat(int64_t e0, int64_t h0, int64_t cnt,
                                                 const int32_t* __restrict__ pmap, const V* __restrict__ Qin,
                                                 V* __restrict__ Qout, V* __restrict__ Qh) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= cnt * NV) return;
    const int64_t j = t / NV, v = t - j * NV;
    const V val = Qin[(e0 + j) * NV + v];
    Qh[(h0 + j) * NV + v] = val;
    Qout[static_cast<int64_t>(pmap[h0 + j]) * NV + v] = val;
}

template <typename V, int NV>
__global__ void __launch_bounds__(256) k_down_flat(int64_t e0, int64_t h0, int64_t cnt,
                                                   const int32_t* __restrict__ pmap, const V* __restrict__ Uh,
                                                   const V* __restrict__ Upar, V* __restrict__ Uown) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= cnt * NV) return;
    const int64_t j = t / NV, v = t - j * NV;
    const double uh = static_cast<double>(Uh[(h0 + j) * NV + v]) +
                      static_cast<double>(Upar[static_cast<int64_t>(pmap[h0 + j]) * NV + v]);
    V* u = Uown + (e0 + j) * NV + v;
    *u = static_cast<V>(static_cast<double>(*u) + uh);
}

// downward: uhat = Uh + U_parent[pmap]; u[0:k] += uhat; u[k:n] += T^T uhat,
// with Tt = T^T stored column-major (m x k, columns padded) so rows of the
// result are contiguous; toff here holds the offsets of the transposes.
// Upar reads the parent level's entries, Uown updates this box's entries.
template <typename V, typename TT, int NV>
__global__ void __launch_bounds__(1024) k_down_gemv(const int2* __restrict__ work, const BoxRec* __restrict__ box,
                                                    const int64_t* __restrict__ toff,
                                                    const int32_t* __restrict__ pmap, const TT* __restrict__ Tt,
                                                    const V* __restrict__ Uh, const V* __restrict__ Upar,
                                                    V* __restrict__ Uown, int nw) {
    using M = RowMap<TT>;
    constexpr int NC = chunks_max<NV>();
    __shared__ double part[NC][M::group * NV];
    const int2 wk = work[blockIdx.x];
    const BoxRec tb = box[wk.x];
    const int k = tb.k, m = tb.n - tb.k;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = wk.y * M::group;
    const TT* __restrict__ Tb = Tt + toff[wk.x] + r0;
    const int64_t ldm = ld_pad(m);
    const V* __restrict__ uhb = Uh + tb.hoff * NV;
    const int32_t* __restrict__ pm = pmap + tb.hoff;
    const int ch = m > 0 ? chunk_len<NV>(k) : 0;   // an uncompressed box has no T
    const int nch = ch > 0 ? (k + ch - 1) / ch : 0;
    for (int c = wave; c < nch; c += nw) {
        double acc[M::vec][NV];
#pragma unroll
        for (int r = 0; r < M::vec; ++r)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[r][v] = 0.0;
        gemv_chunk<TT, NV>(Tb, ldm, m - r0, lane, c * ch, min(k, (c + 1) * ch),
                           [&](int i, double (&x)[NV]) {
                               const int64_t pe = static_cast<int64_t>(pm[i]) * NV;
#pragma unroll
                               for (int v = 0; v < NV; ++v)
                                   x[v] = static_cast<double>(uhb[i * NV + v]) + static_cast<double>(Upar[pe + v]);
                           },
                           acc);
#pragma unroll
        for (int e = 0; e < M::vec; ++e)
#pragma unroll
            for (int v = 0; v < NV; ++v) part[c][(M::vec * lane + e) * NV + v] = acc[e][v];
    }
    __syncthreads();
    const int rows = max(0, min(M::group, m - r0));
    for (int t = threadIdx.x; t < rows * NV; t += blockDim.x) {
        const int r = t / NV, v = t - r * NV;
        double sum = 0.0;
        for (int c = 0; c < nch; ++c) sum += part[c][t];
        V* u = Uown + (tb.voff + k + r0 + r) * NV + v;
        *u = static_cast<V>(static_cast<double>(*u) + sum);
    }
    // the first row group of a box also adds uhat to the skeleton entries
    if (r0 == 0) {
        for (int t = threadIdx.x; t < k * NV; t += blockDim.x) {
            const int ii = t / NV, v = t - ii * NV;
            V* u = Uown + (tb.voff + ii) * NV + v;
            const double uh = static_cast<double>(uhb[t]) + static_cast<double>(Upar[static_cast<int64_t>(pm[ii]) * NV + v]);
            *u = static_cast<V>(static_cast<double>(*u) + uh);
        }
    }
}

// ---------------------------------------------------------------------------
// near field: ifo, ifs, tfo and the top-level direct sum in one launch
// ---------------------------------------------------------------------------
// MODE 0: u += G w ;  1: u += G w, uh -= G wh ;  2: u += G w, uh -= G w ;  3: u += G (w - wh)
template <class P, int TPL, bool CONJ, int MODE, bool MASK>
__device__ __forceinline__ void near_loop(const Rec4<double>* __restrict__ X,
                                          const typename P::Vt* __restrict__ Q,
                                          const typename P::Vt* __restrict__ Qh, int s0, int s1,
                                          typename P::Rt kappa,
                                          const double (&xt)[TPL], const double (&yt)[TPL], const double (&zt)[TPL],
                                          typename P::At (&acc)[TPL][P::nv], typename P::At (&acch)[TPL][P::nv]) {
    using R = typename P::Rt;
    using A = typename P::At;
    constexpr int nv = P::nv;
#pragma unroll 2
    for (int s = s0; s < s1; ++s) {
        const Rec4<double> xs = X[s];
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
            green<P, CONJ, MASK>(xt[p] - xs.x, yt[p] - xs.y, zt[p] - xs.z, kappa, gr, gi);
            const A g = static_cast<A>(gr);
            if constexpr (P::kind == 0) {
                // a real kernel: each column on its own
#pragma unroll
                for (int v = 0; v < nv; ++v) {
                    acc[p][v] = fma(g, w[v], acc[p][v]);
                    if constexpr (MODE == 1) acch[p][v] = fma(-g, wh[v], acch[p][v]);
                    if constexpr (MODE == 2) acch[p][v] = fma(-g, w[v], acch[p][v]);
                }
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

// All translation types of one source box into the lane's targets.
template <class P, int TPL, bool CONJ, bool MASK>
__device__ __forceinline__ void near_segment(int mode, bool has_h, const Rec4<double>* __restrict__ Xs,
                                             const typename P::Vt* __restrict__ Qs,
                                             const typename P::Vt* __restrict__ Qhs, int sn, int sk,
                                             typename P::Rt kappa,
                                             const double (&xt)[TPL], const double (&yt)[TPL],
                                             const double (&zt)[TPL],
                                             typename P::At (&acc)[TPL][P::nv], typename P::At (&acch)[TPL][P::nv]) {
    if (mode == SEG_IFO) {
        if (has_h) {
            near_loop<P, TPL, CONJ, 1, MASK>(Xs, Qs, Qhs, 0, sk, kappa, xt, yt, zt, acc, acch);
            near_loop<P, TPL, CONJ, 0, MASK>(Xs, Qs, Qhs, sk, sn, kappa, xt, yt, zt, acc, acch);
        } else {
            near_loop<P, TPL, CONJ, 0, MASK>(Xs, Qs, Qhs, 0, sn, kappa, xt, yt, zt, acc, acch);
        }
    } else if (mode == SEG_IFS) {
        if (has_h) near_loop<P, TPL, CONJ, 2, MASK>(Xs, Qs, Qhs, 0, sn, kappa, xt, yt, zt, acc, acch);
        else near_loop<P, TPL, CONJ, 0, MASK>(Xs, Qs, Qhs, 0, sn, kappa, xt, yt, zt, acc, acch);
    } else if (mode == SEG_TFO) {
        near_loop<P, TPL, CONJ, 3, MASK>(Xs, Qs, Qhs, 0, sk, kappa, xt, yt, zt, acc, acch);
        near_loop<P, TPL, CONJ, 0, MASK>(Xs, Qs, Qhs, sk, sn, kappa, xt, yt, zt, acc, acch);
    } else {
        near_loop<P, TPL, CONJ, 0, MASK>(Xs, Qs, Qhs, 0, sn, kappa, xt, yt, zt, acc, acch);
    }
}

// One work item of the segment lists: TPL targets per lane of one target box
// against every source box on its list.  Segment modes carry SEG_SELF when the
// source box is the target box.
template <class P, int TPL, bool CONJ>
__device__ __forceinline__ void near_item(const Task tk, const int32_t* __restrict__ seg_ptr,
                                          const int2* __restrict__ segs, const BoxRec* __restrict__ box,
                                          const Rec4<double>* __restrict__ X, const typename P::Vt* __restrict__ Q,
                                          const typename P::Vt* __restrict__ Qh, typename P::Vt* __restrict__ U,
                                          typename P::Vt* __restrict__ Uh, typename P::Rt kappa, double scale,
                                          int lane) {
    using A = typename P::At;
    using V = typename P::Vt;
    constexpr int nv = P::nv;
    const BoxRec tb = box[tk.box];
    // boxes at or above the top level carry k = 0: no skeleton part
    const bool has_h = tk.t0 < tb.k;

    double xt[TPL], yt[TPL], zt[TPL];
    A acc[TPL][nv], acch[TPL][nv];
#pragma unroll
    for (int p = 0; p < TPL; ++p) {
        const int t = min(tk.t0 + lane + 64 * p, tb.n - 1);
        const Rec4<double> x = X[tb.voff + t];
        xt[p] = x.x; yt[p] = x.y; zt[p] = x.z;
#pragma unroll
        for (int v = 0; v < nv; ++v) { acc[p][v] = A(0); acch[p][v] = A(0); }
    }
    const int e1 = seg_ptr[tk.box + 1];
    for (int e = seg_ptr[tk.box]; e < e1; ++e) {
        const int2 sg = segs[e];
        const BoxRec sb = box[sg.x];
        const Rec4<double>* Xs = X + sb.voff;
        const V* Qs = Q + sb.voff * nv;
        const V* Qhs = Qh + sb.hoff * nv;
        const int mode = sg.y & SEG_MODE_MASK;
        if (sg.y & SEG_SELF)
            near_segment<P, TPL, CONJ, true>(mode, has_h, Xs, Qs, Qhs, sb.n, sb.k, kappa, xt, yt, zt, acc, acch);
        else
            near_segment<P, TPL, CONJ, false>(mode, has_h, Xs, Qs, Qhs, sb.n, sb.k, kappa, xt, yt, zt, acc, acch);
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

// One wavefront per work item; every pointer is a separate restrict argument so
// the compiler can prove the source data is never written by this kernel and
// read it with scalar loads.
template <class P, int TPL, bool CONJ>
__global__ void __launch_bounds__(256) k_near(const Task* __restrict__ tasks, int ntasks,
                                              const int32_t* __restrict__ seg_ptr, const int2* __restrict__ segs,
                                              const BoxRec* __restrict__ box,
                                              const Rec4<double>* __restrict__ X,
                                              const typename P::Vt* __restrict__ Q,
                                              const typename P::Vt* __restrict__ Qh,
                                              typename P::Vt* __restrict__ U, typename P::Vt* __restrict__ Uh,
                                              typename P::Rt kappa, double scale) {
    const int lane = threadIdx.x & 63;
    const int tid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tid >= ntasks) return;
    near_item<P, TPL, CONJ>(tasks[tid], seg_ptr, segs, box, X, Q, Qh, U, Uh, kappa, scale, lane);
}

// ---------------------------------------------------------------------------
// symmetric near field (real kernels, one right-hand side)
// ---------------------------------------------------------------------------
// For distinct colleagues i != j (and distinct boxes of the top level) the
// terms i <- j and j <- i use the same block G(B_i, B_j) of a symmetric kernel,
// the second as its transpose.  A work item holds up to 64 TPL targets of box i
// per pass in its lanes and walks the sources of box j in wave-uniform blocks of
// kSymBlock; each kernel value serves both directions:
//   forward  u_i[t]  += G(t, s) q_j[s]          uhat_i[t] -= G(t, s) qhat_j[s]
//   reverse  u_j[s]  += G(t, s) q_i[t]          uhat_j[s] -= G(t, s) qhat_i[t]
// (uhat parts for skeleton targets and sources only; top-level boxes have none).
// The forward sums stay in the lanes.  The reverse sums over the lanes are
// formed per block: each lane keeps its partial for every source of the block,
// the kSymBlock x 64 partials pass through the wave's own LDS tile, a group of
// lanes adds one source's column and cross-lane moves complete it.  All sums go to the item's
// private slots in a fixed order; k_sym_reduce adds them to u and uhat.

// s_waitcnt vmcnt(0) with the other counters left free (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVmcnt0 = 0x0F70;
constexpr int kSymBlock = 8;             // sources per block: their records fit the SGPRs
static_assert(kSymBlock - 1 <= kSymRecordPad, "a block may run past its box by kSymBlock - 1 records");
constexpr int kSymLanes = 64 / kSymBlock; // lanes that add one source's column
constexpr int kSymRow = 72;              // LDS row pitch: the column reads below hit distinct banks

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane moves within a row of 16 lanes (DPP): swap neighbours, swap
// pairs, mirror each half-row.  Together they add up groups of 2, 4 or 8
// consecutive lanes without leaving the vector ALU.
constexpr int kDppXor1 = 0xB1;           // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;           // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;    // row_half_mirror
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
struct IntPair {
    int lo, hi;
};
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const IntPair w = __builtin_bit_cast(IntPair, v);
    return __builtin_bit_cast(double, IntPair{__builtin_amdgcn_mov_dpp(w.lo, CTRL, 0xF, 0xF, false),
                                              __builtin_amdgcn_mov_dpp(w.hi, CTRL, 0xF, 0xF, false)});
}
// the sum over each aligned group of kSymLanes lanes, in all of them
template <typename B>
__device__ __forceinline__ B lane_group_sum(B v) {
    static_assert(kSymLanes == 8, "the DPP tree below adds groups of eight lanes");
    v += dpp_move<kDppXor1>(v);
    v += dpp_move<kDppXor2>(v);
    v += dpp_move<kDppHalfMirror>(v);
    return v;
}

// Column sums of the wave's kSymBlock x 64 partials r[c] (lane = column of the
// tile).  Returns, in every lane of group c (lanes kSymLanes c ..), the sum over
// the 64 lanes of r[c]: each lane of the group adds kSymBlock entries of the
// column, then the group's lanes are added.
template <typename B>
__device__ __forceinline__ B column_sum(const B (&r)[kSymBlock], B* tile, int lane) {
#pragma unroll
    for (int c = 0; c < kSymBlock; ++c) tile[c * kSymRow + lane] = r[c];
    wave_sync();
    const int c = lane / kSymLanes, q = lane % kSymLanes;
    B v = B(0);
#pragma unroll
    for (int i = 0; i < kSymBlock; ++i) v += tile[c * kSymRow + q + kSymLanes * i];
    wave_sync();
    return lane_group_sum(v);
}

// The same column sums formed in float64 (the compensated leaf sums).
template <typename B>
__device__ __forceinline__ double column_sum_f64(const B (&r)[kSymBlock], B* tile, int lane) {
#pragma unroll
    for (int c = 0; c < kSymBlock; ++c) tile[c * kSymRow + lane] = r[c];
    wave_sync();
    const int c = lane / kSymLanes, q = lane % kSymLanes;
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < kSymBlock; ++i) v += static_cast<double>(tile[c * kSymRow + q + kSymLanes * i]);
    wave_sync();
    return lane_group_sum(v);
}

// A block's sources are wave-uniform: each one is read with scalar loads into
// SGPRs (its position record and charges) and enters the lanes' arithmetic as
// an SGPR operand, so a pair costs no LDS traffic and no staging barrier.
// Exact form: the record is the source's coordinates.  Expanded form (see
// sym_pass): the record is (-2 (x_s - o), |x_s - o|^2) for the origin o of the
// source box, precomputed once per operator.  Float32 differences: the record
// is x_s - o in float32, and the targets hold t - o in float32.
// FM (form of |d|^2): 0 float64 differences, 1 expanded, 2 float32 differences.
template <int FM>
using SrcRec = typename std::conditional<FM == 2, Rec4<float>, Rec4<double>>::type;
template <int FM>
using CoordT = typename std::conditional<FM == 2, float, double>::type;

// One block of up to kSymBlock sources s0 .. s0 + cnt - 1 of box j (records
// Xs, charges Qs and Qhs, indexed from the box's first entry).  H: the pass
// holds skeleton targets and the block lies in j's skeleton, so the uhat terms
// run too.  MASK: zero the pairs at distance 0 (needed where a box meets
// itself).  Positions past cnt repeat the last source with zero charges (their
// reverse sums are not stored), so the block is branch-free.  Reverse sums go
// to rev_u[s] (and rev_h[s]), stored on the item's first pass and accumulated
// on later ones.
template <class P, int TPL, bool H, bool MASK, int FM>
__device__ __forceinline__ void sym_block(const SrcRec<FM>* __restrict__ Xs, const typename P::Vt* __restrict__ Qs,
                                          const typename P::Vt* __restrict__ Qhs, int s0, int cnt,
                                          const CoordT<FM> (&xt)[TPL], const CoordT<FM> (&yt)[TPL],
                                          const CoordT<FM> (&zt)[TPL], const double (&nt)[TPL],
                                          const typename P::Rt (&wi)[TPL][P::nv],
                                          const typename P::Rt (&whi)[TPL][P::nv],
                                          typename P::At (&acc)[TPL][P::nv], typename P::At (&acch)[TPL][P::nv],
                                          typename P::Rt* tile, int lane, double* __restrict__ rev_u,
                                          double* __restrict__ rev_h, bool first, double sc) {
    using R = typename P::Rt;
    using A = typename P::At;
    constexpr int NR = P::nv;   // interleaved columns (a real kernel)
    // The running reverse sums of earlier passes are fetched before the block's
    // arithmetic, so their latency overlaps it.  Every lane loads (its column's
    // slot, clamped into the block) and forms the new sum, and only the store
    // is masked: a load under a lane mask would leave the wait for it to a join
    // point, where it would also wait for the store just issued.
    const int last = s0 + cnt - 1;
    const int cs = lane / kSymLanes;
    const int cl = min(s0 + cs, last);
    const bool own = lane % kSymLanes == 0 && cs < cnt;
    double prev_u[NR], prev_h[NR];
#pragma unroll
    for (int v = 0; v < NR; ++v) { prev_u[v] = 0.0; prev_h[v] = 0.0; }
    if (!first) {
#pragma unroll
        for (int v = 0; v < NR; ++v) {
            prev_u[v] = rev_u[cl * NR + v];
            if constexpr (H) prev_h[v] = rev_h[cl * NR + v];
        }
    }
    R bacc[TPL][NR], bh[TPL][NR];
    R ru[NR][kSymBlock], rh[NR][kSymBlock];
#pragma unroll
    for (int p = 0; p < TPL; ++p)
#pragma unroll
        for (int v = 0; v < NR; ++v) { bacc[p][v] = R(0); bh[p][v] = R(0); }
    // the block's first source: constant offsets from here let the loads merge
    const SrcRec<FM>* __restrict__ Xb0 = Xs + s0;
    const typename P::Vt* __restrict__ Qb0 = Qs + static_cast<int64_t>(s0) * NR;
    const typename P::Vt* __restrict__ Qhb0 = Qhs + static_cast<int64_t>(s0) * NR;
#pragma unroll
    for (int c = 0; c < kSymBlock; ++c) {
        // Expanded and float32 records are padded per box (copies of its last
        // record), so the block reads them unclamped and the loads merge; the
        // charges past cnt are read within the arrays' spare tail and replaced
        // by zero.  Exact coordinates are read at the clamped index.
        const int ci = FM != 0 ? c : min(c, cnt - 1);
        const SrcRec<FM> sv = Xb0[ci];
        R svw[NR], svwh[NR];
#pragma unroll
        for (int v = 0; v < NR; ++v) {
            const R qs = static_cast<R>(Qb0[c * NR + v]);
            svw[v] = c < cnt ? qs : R(0);
            svwh[v] = R(0);
            if constexpr (H) {
                const R qh = static_cast<R>(Qhb0[c * NR + v]);
                svwh[v] = c < cnt ? qh : R(0);
            }
            ru[v][c] = R(0);
            rh[v][c] = R(0);
        }
#pragma unroll
        for (int p = 0; p < TPL; ++p) {
            R g, gi;
            if constexpr (FM == 1) {
                // |t - s|^2 = |t'|^2 + |s'|^2 - 2 t'.s' relative to the source box's origin
                const double r2 = fma(xt[p], sv.x, fma(yt[p], sv.y, fma(zt[p], sv.z, nt[p] + sv.w)));
                green_r2<P, false, MASK>(r2, R(0), g, gi);
            } else if constexpr (FM == 2) {
                // t' - s' in float32, both relative to the source box's origin
                const float dx = xt[p] - sv.x, dy = yt[p] - sv.y, dz = zt[p] - sv.z;
                green_r2<P, false, MASK>(fmaf(dx, dx, fmaf(dy, dy, dz * dz)), R(0), g, gi);
            } else {
                green<P, false, MASK>(xt[p] - sv.x, yt[p] - sv.y, zt[p] - sv.z, R(0), g, gi);
            }
#pragma unroll
            for (int v = 0; v < NR; ++v) {
                bacc[p][v] = fma(g, svw[v], bacc[p][v]);
                ru[v][c] = fma(g, wi[p][v], ru[v][c]);
                if constexpr (H) {
                    bh[p][v] = fma(g, svwh[v], bh[p][v]);
                    rh[v][c] = fma(g, whi[p][v], rh[v][c]);
                }
            }
        }
        // compensated leaf sums: the forward partials reach float64 every four sources
        if constexpr (P::comp && sizeof(R) == 4) {
            if (c % 4 == 3 && c != kSymBlock - 1) {
#pragma unroll
                for (int p = 0; p < TPL; ++p)
#pragma unroll
                    for (int v = 0; v < NR; ++v) {
                        acc[p][v] += static_cast<A>(bacc[p][v]);
                        bacc[p][v] = R(0);
                        if constexpr (H) {
                            acch[p][v] += static_cast<A>(bh[p][v]);
                            bh[p][v] = R(0);
                        }
                    }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < TPL; ++p)
#pragma unroll
        for (int v = 0; v < NR; ++v) {
            acc[p][v] += static_cast<A>(bacc[p][v]);
            if constexpr (H) acch[p][v] += static_cast<A>(bh[p][v]);
        }
    double nu[NR], nh[NR];
#pragma unroll
    for (int v = 0; v < NR; ++v) {
        if constexpr (P::comp && sizeof(R) == 4) nu[v] = prev_u[v] + sc * column_sum_f64<R>(ru[v], tile, lane);
        else nu[v] = prev_u[v] + sc * static_cast<double>(column_sum<R>(ru[v], tile, lane));
        nh[v] = 0.0;
        if constexpr (H) {
            if constexpr (P::comp && sizeof(R) == 4) nh[v] = prev_h[v] - sc * column_sum_f64<R>(rh[v], tile, lane);
            else nh[v] = prev_h[v] - sc * static_cast<double>(column_sum<R>(rh[v], tile, lane));
        }
    }
    // the reverse-sum loads have returned long ago; waiting for them here, in
    // every lane, keeps the wait out of the join after the masked store (where
    // it would also wait for that store)
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    if (own) {
#pragma unroll
        for (int v = 0; v < NR; ++v) {
            rev_u[cl * NR + v] = nu[v];
            if constexpr (H) rev_h[cl * NR + v] = nh[v];
        }
    }
}

// Sources [s_begin, n_j) of a pass in blocks: first the skeleton blocks
// [s_begin, kH) (kH = k_j when the uhat terms run, else s_begin), then the rest
// [kH, n_j), 16 at a time.
struct BlockPlan {
    int sb, kH, nbH, nb, n;
    __device__ void init(int s_begin, int k_h, int n_j) {
        sb = s_begin;
        kH = max(s_begin, k_h);
        n = n_j;
        nbH = (kH - sb + kSymBlock - 1) / kSymBlock;
        nb = nbH + (max(0, n - kH) + kSymBlock - 1) / kSymBlock;
    }
    __device__ void range(int b, int& s0, int& cnt) const {
        if (b < nbH) { s0 = sb + b * kSymBlock; cnt = min(kSymBlock, kH - s0); }
        else { s0 = kH + (b - nbH) * kSymBlock; cnt = min(kSymBlock, n - s0); }
    }
};

// Item context shared by its passes.
struct SymCtx {
    BoxRec bi, bj;
    int t0, t1;
    double* fwd_u;
    double* fwd_h;
    double* rev_u;
    double* rev_h;
    double sc;
};

// One pass: targets tp .. tp + 64 TPL - 1 of box i (those below t1) against all
// sources of box j.
template <class P, int TPL, bool SELF, int FM>
__device__ __forceinline__ void sym_pass(const SymCtx& cx, int tp, const Rec4<double>* __restrict__ X,
                                         const typename P::Vt* __restrict__ Q,
                                         const typename P::Vt* __restrict__ Qh,
                                         const Rec4<double>* __restrict__ Xs, const SrcRec<FM>* __restrict__ Xb,
                                         const typename P::Vt* __restrict__ Qs,
                                         const typename P::Vt* __restrict__ Qhs, typename P::Rt* tile, int lane) {
    using R = typename P::Rt;
    using A = typename P::At;
    const BoxRec& bi = cx.bi;
    const BoxRec& bj = cx.bj;
    const bool first = tp == cx.t0;
    // skeleton targets in this pass and a skeleton in box j: the uhat terms run
    const bool hp = tp < bi.k && bj.k > 0;
    // a box paired with itself: the diagonal tile (sources = this pass's
    // targets) is evaluated in the forward direction only, the sources after it
    // in both
    const int tile_end = SELF ? min(tp + 64 * TPL, cx.t1) : 0;
    BlockPlan bp;
    bp.init(tile_end, hp ? bj.k : 0, bj.n);
    constexpr int NR = P::nv;
    CoordT<FM> xt[TPL], yt[TPL], zt[TPL];
    double nt[TPL];
    R wi[TPL][NR], whi[TPL][NR];
    A acc[TPL][NR], acch[TPL][NR];
    // expanded form and float32 differences: target coordinates relative to
    // the origin of the source box (its first entry), the origin of the source
    // records Xb
    double o[3] = {0.0, 0.0, 0.0};
    if constexpr (FM != 0) {
        const Rec4<double> x0 = Xs[0];
        o[0] = x0.x; o[1] = x0.y; o[2] = x0.z;
    }
#pragma unroll
    for (int p = 0; p < TPL; ++p) {
        const int t = tp + lane + 64 * p;
        const bool ok = t < cx.t1;
        const int tc = ok ? t : cx.t1 - 1;
        const Rec4<double> x = X[bi.voff + tc];
        const double dx = x.x - o[0], dy = x.y - o[1], dz = x.z - o[2];
        xt[p] = static_cast<CoordT<FM>>(dx);
        yt[p] = static_cast<CoordT<FM>>(dy);
        zt[p] = static_cast<CoordT<FM>>(dz);
        nt[p] = FM == 1 ? fma(dx, dx, fma(dy, dy, dz * dz)) : 0.0;
#pragma unroll
        for (int v = 0; v < NR; ++v) {
            wi[p][v] = ok ? static_cast<R>(Q[(bi.voff + tc) * NR + v]) : R(0);
            whi[p][v] = (ok && t < bi.k) ? static_cast<R>(Qh[(bi.hoff + t) * NR + v]) : R(0);
            acc[p][v] = A(0);
            acch[p][v] = A(0);
        }
    }
    if constexpr (SELF) {
        A ad[TPL][NR], adh[TPL][NR];
#pragma unroll
        for (int p = 0; p < TPL; ++p)
#pragma unroll
            for (int v = 0; v < NR; ++v) { ad[p][v] = A(0); adh[p][v] = A(0); }
        if (hp) {
            near_loop<P, TPL, false, 1, true>(Xs, Qs, Qhs, tp, min(tile_end, bj.k), R(0), xt, yt, zt, ad, adh);
            near_loop<P, TPL, false, 0, true>(Xs, Qs, Qhs, max(tp, bj.k), tile_end, R(0), xt, yt, zt, ad, adh);
        } else {
            near_loop<P, TPL, false, 0, true>(Xs, Qs, Qhs, tp, tile_end, R(0), xt, yt, zt, ad, adh);
        }
        // near_loop accumulates the uhat part with its minus sign; the pair
        // blocks below accumulate it positive and the store negates
#pragma unroll
        for (int p = 0; p < TPL; ++p)
#pragma unroll
            for (int v = 0; v < NR; ++v) { acc[p][v] = ad[p][v]; acch[p][v] = -adh[p][v]; }
    }
    for (int b = 0; b < bp.nb; ++b) {
        int s0, cnt;
        bp.range(b, s0, cnt);
        if (b < bp.nbH)
            sym_block<P, TPL, true, SELF, FM>(Xb, Qs, Qhs, s0, cnt, xt, yt, zt, nt, wi, whi, acc, acch, tile, lane,
                                                cx.rev_u, cx.rev_h, first, cx.sc);
        else
            sym_block<P, TPL, false, SELF, FM>(Xb, Qs, Qhs, s0, cnt, xt, yt, zt, nt, wi, whi, acc, acch, tile, lane,
                                                 cx.rev_u, cx.rev_h, first, cx.sc);
    }
#pragma unroll
    for (int p = 0; p < TPL; ++p) {
        const int t = tp + lane + 64 * p;
        if (t < cx.t1) {
#pragma unroll
            for (int v = 0; v < NR; ++v) {
                cx.fwd_u[(t - cx.t0) * NR + v] = cx.sc * static_cast<double>(acc[p][v]);
                if (t < bi.k) cx.fwd_h[(t - cx.t0) * NR + v] = -cx.sc * static_cast<double>(acch[p][v]);
                // a self item's reverse row starts past the first diagonal tile; the
                // first pass writes zeros before it so the whole row is defined
                if (SELF && first) {
                    cx.rev_u[t * NR + v] = 0.0;
                    if (t < bi.k) cx.rev_h[t * NR + v] = 0.0;
                }
            }
        }
    }
}

// The last pass of an item when at most 64 TPL targets are left: it runs with
// the fewest targets per lane that hold them, so a ragged end wastes less than
// one wave's lanes.  The pass boundaries (and with them the diagonal tiles of a
// self item) are those of TPL-wide passes.  Every pass width is inlined at one
// call site (two copies of a wide pass cost the float32 variants spills).
template <class P, int TPL, bool SELF, int FM>
__device__ __forceinline__ void sym_tail(const SymCtx& cx, int tp, const Rec4<double>* __restrict__ X,
                                         const typename P::Vt* __restrict__ Q, const typename P::Vt* __restrict__ Qh,
                                         const Rec4<double>* __restrict__ Xs, const SrcRec<FM>* __restrict__ Xb,
                                         const typename P::Vt* __restrict__ Qs,
                                         const typename P::Vt* __restrict__ Qhs, typename P::Rt* tile, int lane) {
    if constexpr (TPL == 1) {
        sym_pass<P, 1, SELF, FM>(cx, tp, X, Q, Qh, Xs, Xb, Qs, Qhs, tile, lane);
    } else {
        if (cx.t1 - tp > 64 * (TPL - 1))
            sym_pass<P, TPL, SELF, FM>(cx, tp, X, Q, Qh, Xs, Xb, Qs, Qhs, tile, lane);
        else
            sym_tail<P, TPL - 1, SELF, FM>(cx, tp, X, Q, Qh, Xs, Xb, Qs, Qhs, tile, lane);
    }
}

// All passes of an item: TPL-wide while more than 64 (TPL - 1) targets are
// left (the last of them may be ragged), else the narrower tail.
template <class P, int TPL, bool SELF, int FM>
__device__ __forceinline__ void sym_passes(const SymCtx& cx, const Rec4<double>* __restrict__ X,
                                           const typename P::Vt* __restrict__ Q,
                                           const typename P::Vt* __restrict__ Qh,
                                           const Rec4<double>* __restrict__ Xs,
                                           const SrcRec<FM>* __restrict__ Xb,
                                           const typename P::Vt* __restrict__ Qs,
                                           const typename P::Vt* __restrict__ Qhs, typename P::Rt* tile, int lane) {
    for (int tp = cx.t0; tp < cx.t1;) {
        if (cx.t1 - tp > 64 * (TPL - 1)) {
            sym_pass<P, TPL, SELF, FM>(cx, tp, X, Q, Qh, Xs, Xb, Qs, Qhs, tile, lane);
            tp += 64 * TPL;
        } else {
            if constexpr (TPL > 1) sym_tail<P, TPL - 1, SELF, FM>(cx, tp, X, Q, Qh, Xs, Xb, Qs, Qhs, tile, lane);
            break;
        }
    }
}

// A pair item: its passes (sym_passes).
// A box paired with itself (bi == bj, one item over all its targets) evaluates
// each unordered pair of distinct entries once, except inside the diagonal
// tiles, which run in one direction with the zero distances masked.  F32D:
// the operator was built with f32_differences (a kernel of its own, so the
// default kernel carries no registers for the float32-difference form).
template <class P, int TPL, bool F32D>
__device__ __forceinline__ void sym_item(const SymTask it, const BoxRec* __restrict__ box,
                                         const Rec4<double>* __restrict__ X, const Rec4<double>* __restrict__ Xe,
                                         const Rec4<float>* __restrict__ Xf, const typename P::Vt* __restrict__ Q,
                                         const typename P::Vt* __restrict__ Qh, double* __restrict__ slots,
                                         double scale, typename P::Rt* tile, int lane) {
    using V = typename P::Vt;
    SymCtx cx;
    cx.bi = box[it.bi];
    cx.bj = box[it.bj];
    cx.t0 = it.t0;
    cx.t1 = it.t1;
    // uhat rows exist only where an item touches them (offsets < 0 are never
    // used); offsets count entries of P::nv values
    constexpr int NR = P::nv;
    cx.fwd_u = slots + NR * it.fwd_u;
    cx.fwd_h = slots + NR * (it.fwd_h >= 0 ? it.fwd_h : 0);
    cx.rev_u = slots + NR * it.rev_u;
    cx.rev_h = slots + NR * (it.rev_h >= 0 ? it.rev_h : 0);
    cx.sc = scale * P::gscale;
    const Rec4<double>* Xs = X + cx.bj.voff;
    const V* Qs = Q + cx.bj.voff * NR;
    const V* Qhs = Qh + cx.bj.hoff * NR;
    // float32 differences or the expanded |d|^2 serve the float32 evaluation of
    // items the build marked safe for them
    if constexpr (sizeof(typename P::Rt) == 4) {
        if (F32D && (it.flags & SYM_F32DIFF)) {
            sym_passes<P, TPL, false, 2>(cx, X, Q, Qh, Xs, Xf + cx.bj.roff, Qs, Qhs, tile, lane);
            return;
        }
        if (it.flags & SYM_EXPANDED) {
            sym_passes<P, TPL, false, 1>(cx, X, Q, Qh, Xs, Xe + cx.bj.roff, Qs, Qhs, tile, lane);
            return;
        }
    }
    if (it.bi != it.bj)
        sym_passes<P, TPL, false, 0>(cx, X, Q, Qh, Xs, Xs, Qs, Qhs, tile, lane);
    else
        sym_passes<P, TPL, true, 0>(cx, X, Q, Qh, Xs, Xs, Qs, Qhs, tile, lane);
}

// Waves per SIMD the pair kernel is compiled for: the float32 evaluation fits
// four waves' registers with up to two targets per lane, three with three.
template <class P, int TPL>
constexpr int sym_waves() {
    if (sizeof(typename P::Rt) != 4) return 1;
    if (P::rhs == 1) return TPL <= 2 ? 6 : (TPL == 3 ? 5 : 4);
    return TPL == 1 ? 6 : (TPL == 2 ? 5 : (TPL == 3 ? 4 : 1));
}

template <class P, int TPL, bool F32D = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sym_waves<P, TPL>(), 8))) k_near_sym(const SymTask* __restrict__ tasks, int ntasks,
                                                  const BoxRec* __restrict__ box,
                                                  const Rec4<double>* __restrict__ X,
                                                  const Rec4<double>* __restrict__ Xe,
                                                  const Rec4<float>* __restrict__ Xf,
                                                  const typename P::Vt* __restrict__ Q,
                                                  const typename P::Vt* __restrict__ Qh,
                                                  double* __restrict__ slots, double scale) {
    using R = typename P::Rt;
    __shared__ R tiles[4][kSymBlock * kSymRow];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tid = blockIdx.x * 4 + wv;
    if (tid >= ntasks) return;
    sym_item<P, TPL, F32D>(tasks[tid], box, X, Xe, Xf, Q, Qh, slots, scale, tiles[wv], lane);
}

// acc + p[0] + p[ld] + ... + p[(rows - 1) ld], added in row order; the loads of
// four rows are issued together.
__device__ __forceinline__ double add_rows(double acc, const double* __restrict__ p, int rows, int ld) {
    constexpr int kRows = 8;
    int i = 0;
    for (; i + kRows <= rows; i += kRows) {
        double a[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) a[u] = p[static_cast<int64_t>(i + u) * ld];
#pragma unroll
        for (int u = 0; u < kRows; ++u) acc += a[u];
    }
    for (; i < rows; ++i) acc += p[static_cast<int64_t>(i) * ld];
    return acc;
}

// u and uhat of one box += its slot rows, in row order (deterministic).  A
// block per receiving box; threads run over the box's entries (NV values
// each: a complex entry or interleaved columns), so every row is read with
// coalesced loads.
template <typename V, int NV>
__global__ void __launch_bounds__(256) k_sym_reduce(const SymRows* __restrict__ rows,
                                                    const BoxRec* __restrict__ box,
                                                    const double* __restrict__ slots, V* __restrict__ U,
                                                    V* __restrict__ Uh) {
    const SymRows r = rows[blockIdx.x];
    const BoxRec rec = box[r.box];
    for (int e = threadIdx.x; e < NV * rec.n; e += blockDim.x) {
        V* u = U + NV * rec.voff + e;
        *u = static_cast<V>(add_rows(static_cast<double>(*u), slots + NV * r.base_u + e, r.ru, NV * rec.n));
        if (e < NV * rec.k && r.rh > 0) {
            V* uh = Uh + NV * rec.hoff + e;
            *uh = static_cast<V>(add_rows(static_cast<double>(*uh), slots + NV * r.base_h + e, r.rh, NV * rec.k));
        }
    }
}

// ---------------------------------------------------------------------------
// many right-hand sides on the matrix cores (real kernels, float32 policy)
// ---------------------------------------------------------------------------
// With several right-hand sides the near field of a target tile is a product
// U[t, r] += sum_s G(t, s) Q[s, r] whose left factor is generated on the fly.
// A work item is one wavefront holding 32 targets x 32 RHS columns in a 32 x 32
// float32 accumulator tile of v_mfma_f32_32x32x2f32: each step takes two
// sources, every lane evaluates one kernel value G(target lane % 32, source
// lane / 32) -- exactly the A operand's layout (row lane % 32, k lane / 32) --
// and supplies Q[source lane / 32, column lane % 32] as the B operand.  The
// float32 tile of one source box is added to float64 totals (the accumulator
// layout: register v of lane l holds row 8 (v / 4) + 4 (l / 32) + v % 4,
// column l % 32), as the other float32 kernels do per source box.
typedef float floatx16 __attribute__((ext_vector_type(16)));
constexpr int kMfmaTile = 32;   // columns of one accumulator tile

// Sources [s0, s1) of one box, two per step, into NT column tiles.  MODE as in
// near_loop_mr: 0 u += G q; 1 u += G q, uh -= G qh; 2 u += G q, uh -= G q;
// 3 u += G (q - qh).  Steps run in groups of GS: the group's loads are issued
// together, then its kernel values and MFMAs, so one memory latency covers GS
// steps.  The last group's steps past s1 are skipped (a wave-uniform branch;
// their loads repeat the last source), and a step's second source past s1 gets
// a zero kernel value, which adds exact zeros.  With NT = 2, `two` is false
// when the second tile lies past the padded width (an odd tile count): its
// loads are skipped and its MFMAs accumulate zeros that are never stored.
template <class P, bool MASK, int MODE, int NT, int GS>
__device__ __forceinline__ void mfma_steps(const Rec4<double>* __restrict__ Xs, const float* __restrict__ Qs,
                                           const float* __restrict__ Qhs, int Wp, int s0, int s1, double xt,
                                           double yt, double zt, int row, int half, bool two, floatx16 (&cu)[NT],
                                           floatx16 (&ch)[NT]) {
    for (int sg = s0; sg < s1; sg += 2 * GS) {
        double sx[GS], sy[GS], sz[GS];
        float q[GS][NT], qh[GS][NT];
        bool ok[GS];
#pragma unroll
        for (int u = 0; u < GS; ++u) {
            const int s = sg + 2 * u + half;
            ok[u] = s < s1;
            const int sc = ok[u] ? s : s1 - 1;
            const Rec4<double> xs = Xs[sc];
            sx[u] = xs.x;
            sy[u] = xs.y;
            sz[u] = xs.z;
            const int64_t o = static_cast<int64_t>(sc) * Wp + row;
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                q[u][c] = 0.0f;
                qh[u][c] = 0.0f;
                if (c == 0 || two) {
                    q[u][c] = Qs[o + c * kMfmaTile];
                    if constexpr (MODE == 1 || MODE == 3) qh[u][c] = Qhs[o + c * kMfmaTile];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < GS; ++u) {
            if (u > 0 && sg + 2 * u >= s1) break;
            float g, gi;
            green<P, false, MASK>(xt - sx[u], yt - sy[u], zt - sz[u], 0.0f, g, gi);
            g = ok[u] ? g : 0.0f;
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const float bu = MODE == 3 ? q[u][c] - qh[u][c] : q[u][c];
                cu[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(g, bu, cu[c], 0, 0, 0);
                if constexpr (MODE == 1) ch[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(g, -qh[u][c], ch[c], 0, 0, 0);
                if constexpr (MODE == 2) ch[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(g, -q[u][c], ch[c], 0, 0, 0);
            }
        }
    }
}

// Steps per group of the one-tile kernel
constexpr int kMfmaGroup1 = 4;

template <class P, bool MASK, int MODE>
__device__ __forceinline__ void mfma_range(const Rec4<double>* __restrict__ Xs, const float* __restrict__ Qs,
                                           const float* __restrict__ Qhs, int Wp, int s0, int s1, double xt,
                                           double yt, double zt, int row, int half, floatx16& cu, floatx16& ch) {
    floatx16 u[1] = {cu}, h[1] = {ch};
    mfma_steps<P, MASK, MODE, 1, kMfmaGroup1>(Xs, Qs, Qhs, Wp, s0, s1, xt, yt, zt, row, half, false, u, h);
    cu = u[0];
    ch = h[0];
}

template <class P, bool MASK>
__device__ __forceinline__ void mfma_segment(int mode, bool has_h, const Rec4<double>* __restrict__ Xs,
                                             const float* __restrict__ Qs, const float* __restrict__ Qhs, int Wp,
                                             int sn, int sk, double xt, double yt, double zt, int row, int half,
                                             floatx16& cu, floatx16& ch) {
    if (mode == SEG_IFO) {
        if (has_h) {
            mfma_range<P, MASK, 1>(Xs, Qs, Qhs, Wp, 0, sk, xt, yt, zt, row, half, cu, ch);
            mfma_range<P, MASK, 0>(Xs, Qs, Qhs, Wp, sk, sn, xt, yt, zt, row, half, cu, ch);
        } else {
            mfma_range<P, MASK, 0>(Xs, Qs, Qhs, Wp, 0, sn, xt, yt, zt, row, half, cu, ch);
        }
    } else if (mode == SEG_IFS) {
        if (has_h) mfma_range<P, MASK, 2>(Xs, Qs, Qhs, Wp, 0, sn, xt, yt, zt, row, half, cu, ch);
        else mfma_range<P, MASK, 0>(Xs, Qs, Qhs, Wp, 0, sn, xt, yt, zt, row, half, cu, ch);
    } else if (mode == SEG_TFO) {
        mfma_range<P, MASK, 3>(Xs, Qs, Qhs, Wp, 0, sk, xt, yt, zt, row, half, cu, ch);
        mfma_range<P, MASK, 0>(Xs, Qs, Qhs, Wp, sk, sn, xt, yt, zt, row, half, cu, ch);
    } else {
        mfma_range<P, MASK, 0>(Xs, Qs, Qhs, Wp, 0, sn, xt, yt, zt, row, half, cu, ch);
    }
}

// Work item: (task of 32 targets, tile of 32 columns); Wp is a multiple of 32.
template <class P>
__global__ void __launch_bounds__(256) k_near_mfma(const Task* __restrict__ tasks, int ntasks, int ntiles, int Wp,
                                                   const int32_t* __restrict__ seg_ptr,
                                                   const int2* __restrict__ segs, const BoxRec* __restrict__ box,
                                                   const Rec4<double>* __restrict__ X, const float* __restrict__ Q,
                                                   const float* __restrict__ Qh, float* __restrict__ U,
                                                   float* __restrict__ Uh, double scale) {
    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wid >= ntasks * ntiles) return;
    const int c0 = 32 * (wid % ntiles);
    const Task tk = tasks[wid / ntiles];
    const BoxRec tb = box[tk.box];
    const bool has_h = tk.t0 < tb.k;
    const int row = lane & 31, half = lane >> 5;
    const Rec4<double> xr = X[tb.voff + min(tk.t0 + row, tb.n - 1)];
    double du[16], dh[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) { du[v] = 0.0; dh[v] = 0.0; }
    const int e1 = seg_ptr[tk.box + 1];
    for (int e = seg_ptr[tk.box]; e < e1; ++e) {
        const int2 sg = segs[e];
        const BoxRec sb = box[sg.x];
        const Rec4<double>* Xs = X + sb.voff;
        const float* Qs = Q + sb.voff * Wp + c0;
        const float* Qhs = Qh + sb.hoff * Wp + c0;
        floatx16 cu = {}, ch = {};
        if (sg.y & SEG_SELF)
            mfma_segment<P, true>(sg.y & SEG_MODE_MASK, has_h, Xs, Qs, Qhs, Wp, sb.n, sb.k, xr.x, xr.y, xr.z, row,
                                  half, cu, ch);
        else
            mfma_segment<P, false>(sg.y & SEG_MODE_MASK, has_h, Xs, Qs, Qhs, Wp, sb.n, sb.k, xr.x, xr.y, xr.z,
                                   row, half, cu, ch);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            du[v] += static_cast<double>(cu[v]);
            dh[v] += static_cast<double>(ch[v]);
        }
    }
    const double sc = scale * P::gscale;
    const int col = c0 + row;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int t = tk.t0 + 8 * (v / 4) + 4 * half + (v % 4);
        if (t < tb.n) {
            U[(tb.voff + t) * Wp + col] = static_cast<float>(du[v] * sc);
            if (has_h && t < tb.k) Uh[(tb.hoff + t) * Wp + col] = static_cast<float>(dh[v] * sc);
        }
    }
}

// Two column tiles per wave: each kernel value feeds the MFMAs of both tiles,
// halving the evaluations per column.  Per tile the MFMA sequence is that of
// the one-tile kernel, so the sums agree bit for bit.  Steps per group: the
// uhat modes hold four accumulator tiles and take smaller groups.
template <class P, bool MASK, int MODE>
__device__ __forceinline__ void mfma_range2(const Rec4<double>* __restrict__ Xs, const float* __restrict__ Qs,
                                            const float* __restrict__ Qhs, int Wp, int s0, int s1, double xt,
                                            double yt, double zt, int row, int half, bool two, floatx16 (&cu)[2],
                                            floatx16 (&ch)[2]) {
    mfma_steps<P, MASK, MODE, 2, (MODE == 1 || MODE == 2) ? 2 : 4>(Xs, Qs, Qhs, Wp, s0, s1, xt, yt, zt, row, half,
                                                                    two, cu, ch);
}

template <class P, bool MASK, bool H>
__device__ __forceinline__ void mfma_segment2(int mode, const Rec4<double>* __restrict__ Xs,
                                              const float* __restrict__ Qs, const float* __restrict__ Qhs, int Wp,
                                              int sn, int sk, double xt, double yt, double zt, int row, int half,
                                              bool two, floatx16 (&cu)[2], floatx16 (&ch)[2]) {
    if (mode == SEG_IFO && H) {
        mfma_range2<P, MASK, 1>(Xs, Qs, Qhs, Wp, 0, sk, xt, yt, zt, row, half, two, cu, ch);
        mfma_range2<P, MASK, 0>(Xs, Qs, Qhs, Wp, sk, sn, xt, yt, zt, row, half, two, cu, ch);
    } else if (mode == SEG_IFS && H) {
        mfma_range2<P, MASK, 2>(Xs, Qs, Qhs, Wp, 0, sn, xt, yt, zt, row, half, two, cu, ch);
    } else if (mode == SEG_TFO) {
        mfma_range2<P, MASK, 3>(Xs, Qs, Qhs, Wp, 0, sk, xt, yt, zt, row, half, two, cu, ch);
        mfma_range2<P, MASK, 0>(Xs, Qs, Qhs, Wp, sk, sn, xt, yt, zt, row, half, two, cu, ch);
    } else {
        mfma_range2<P, MASK, 0>(Xs, Qs, Qhs, Wp, 0, sn, xt, yt, zt, row, half, two, cu, ch);
    }
}

// Work item: (task of 32 targets, pair of 32-column tiles).  H: the task's
// targets lie in the box's skeleton (uhat rows); tasks are launched in two
// lists, with and without.
template <class P, bool H>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(H ? 2 : 3, 8))) k_near_mfma2(const Task* __restrict__ tasks, int ntasks, int npairs, int Wp,
                                                    const int32_t* __restrict__ seg_ptr,
                                                    const int2* __restrict__ segs, const BoxRec* __restrict__ box,
                                                    const Rec4<double>* __restrict__ X, const float* __restrict__ Q,
                                                    const float* __restrict__ Qh, float* __restrict__ U,
                                                    float* __restrict__ Uh, double scale) {
    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wid >= ntasks * npairs) return;
    const int c0 = 2 * kMfmaTile * (wid % npairs);
    const bool two = c0 + kMfmaTile < Wp;
    const Task tk = tasks[wid / npairs];
    const BoxRec tb = box[tk.box];
    const int row = lane & 31, half = lane >> 5;
    const Rec4<double> xr = X[tb.voff + min(tk.t0 + row, tb.n - 1)];
    double du[2][16], dh[2][16];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) { du[c][v] = 0.0; dh[c][v] = 0.0; }
    const int e1 = seg_ptr[tk.box + 1];
    for (int e = seg_ptr[tk.box]; e < e1; ++e) {
        const int2 sg = segs[e];
        const BoxRec sb = box[sg.x];
        const Rec4<double>* Xs = X + sb.voff;
        const float* Qs = Q + sb.voff * Wp + c0;
        const float* Qhs = Qh + sb.hoff * Wp + c0;
        floatx16 cu[2] = {{}, {}}, ch[2] = {{}, {}};
        if (sg.y & SEG_SELF)
            mfma_segment2<P, true, H>(sg.y & SEG_MODE_MASK, Xs, Qs, Qhs, Wp, sb.n, sb.k, xr.x, xr.y, xr.z, row, half,
                                      two, cu, ch);
        else
            mfma_segment2<P, false, H>(sg.y & SEG_MODE_MASK, Xs, Qs, Qhs, Wp, sb.n, sb.k, xr.x, xr.y, xr.z, row,
                                       half, two, cu, ch);
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                du[c][v] += static_cast<double>(cu[c][v]);
                if constexpr (H) dh[c][v] += static_cast<double>(ch[c][v]);
            }
    }
    const double sc = scale * P::gscale;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int t = tk.t0 + 8 * (v / 4) + 4 * half + (v % 4);
        if (t < tb.n) {
            float* u = U + (tb.voff + t) * Wp + c0 + row;
            u[0] = static_cast<float>(du[0][v] * sc);
            if (two) u[kMfmaTile] = static_cast<float>(du[1][v] * sc);
            if (H && t < tb.k) {
                float* uh = Uh + (tb.hoff + t) * Wp + c0 + row;
                uh[0] = static_cast<float>(dh[0][v] * sc);
                if (two) uh[kMfmaTile] = static_cast<float>(dh[1][v] * sc);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// many right-hand sides
// ---------------------------------------------------------------------------
// Gather / scatter between the caller's n x Win vectors and the leaf entries of
// the n_entries x Wp workspace (Wp = Win for one RHS; for several, Wp is a
// multiple of the RHS chunk, the gather zero-fills the padding and the scatter
// writes only the caller's columns).
// i = r w + c (0 <= c < w) for an index below total: 32-bit division (about a
// quarter of the instructions of a 64-bit one) whenever total fits it.
__device__ __forceinline__ void split_index(int64_t i, int64_t total, int w, int64_t& r, int64_t& c) {
    if (total <= 0xffffffffLL) {
        const uint32_t u = static_cast<uint32_t>(i), uw = static_cast<uint32_t>(w);
        const uint32_t q = u / uw;
        r = q;
        c = u - q * uw;
    } else {
        r = i / w;
        c = i - r * w;
    }
}

template <typename VI, typename VO>
__global__ void k_gather_pad(const int32_t* __restrict__ dst_e, const int32_t* __restrict__ src_p, int64_t cnt,
                             int Win, int Wp, const VI* __restrict__ in, VO* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cnt * Wp) return;
    int64_t r, c;
    split_index(i, cnt * Wp, Wp, r, c);
    out[static_cast<int64_t>(dst_e[r]) * Wp + c] =
        c < Win ? static_cast<VO>(in[static_cast<int64_t>(src_p[r]) * Win + c]) : VO(0);
}

// A forward and an adjoint column interleaved per entry (two real vectors
// through one sweep): in[0] and in[1] gathered to out[2 e], out[2 e + 1].
template <typename V>
__global__ void k_gather2(const int32_t* __restrict__ dst_e, const int32_t* __restrict__ src_p, int64_t cnt,
                          const V* __restrict__ a, const V* __restrict__ b, V* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const int64_t e = dst_e[i], p = src_p[i];
    out[2 * e] = a[p];
    out[2 * e + 1] = b[p];
}

template <typename V>
__global__ void k_scatter2(const int32_t* __restrict__ src_e, const int32_t* __restrict__ dst_p, int64_t cnt,
                           const V* __restrict__ in, V* __restrict__ a, V* __restrict__ b) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const int64_t e = src_e[i], p = dst_p[i];
    a[p] = in[2 * e];
    b[p] = in[2 * e + 1];
}

template <typename VI, typename VO>
__global__ void k_scatter_pad(const int32_t* __restrict__ src_e, const int32_t* __restrict__ dst_p, int64_t cnt,
                              int Win, int Wp, const VI* __restrict__ in, VO* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cnt * Win) return;
    int64_t r, c;
    split_index(i, cnt * Win, Win, r, c);
    out[static_cast<int64_t>(dst_p[r]) * Win + c] = static_cast<VO>(in[static_cast<int64_t>(src_e[r]) * Wp + c]);
}

// Transfer with lanes over right-hand-side columns:
//   acc[rr] = sum_j A[r0 + rr + j lda] x[j]   for the wave's RB rows
// A is column-major (contiguous along rows), so the RB coefficients of one
// column are one wave-uniform scalar load; x rows are coalesced vector loads.
constexpr int kRB = 16;

// upward: qhat = q[0:k] + T q[k:n]  (T column-major k x m, columns padded to ld_pad(k))
template <typename V, typename TT>
__global__ void __launch_bounds__(256) k_upward_mr(const BoxRec* __restrict__ box, const int64_t* __restrict__ toff,
                                                  const int32_t* __restrict__ pmap, int b0, int Wp,
                                                  const TT* __restrict__ T, V* __restrict__ Q,
                                                  V* __restrict__ Qh) {
    const int b = b0 + blockIdx.x;
    const BoxRec tb = box[b];
    const int k = tb.k, m = tb.n - tb.k;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TT* __restrict__ Tb = T + toff[b];
    for (int c0 = 0; c0 < Wp; c0 += 64) {
        const int c = c0 + lane;
        const bool act = c < Wp;
        for (int r0 = (blockIdx.y * 4 + wave) * kRB; r0 < k; r0 += gridDim.y * 4 * kRB) {
            double acc[kRB];
#pragma unroll
            for (int rr = 0; rr < kRB; ++rr) acc[rr] = 0.0;
            const int nr = min(kRB, k - r0);
            for (int j = 0; j < m; ++j) {
                const double x = act ? static_cast<double>(Q[(tb.voff + k + j) * Wp + c]) : 0.0;
                const TT* col = Tb + r0 + static_cast<int64_t>(j) * ld_pad(k);
                if (nr == kRB) {
#pragma unroll
                    for (int rr = 0; rr < kRB; ++rr) acc[rr] = fma(static_cast<double>(col[rr]), x, acc[rr]);
                } else {
#pragma unroll
                    for (int rr = 0; rr < kRB; ++rr)
                        if (rr < nr) acc[rr] = fma(static_cast<double>(col[rr]), x, acc[rr]);
                }
            }
            if (act) {
#pragma unroll
                for (int rr = 0; rr < kRB; ++rr) {
                    const int r = r0 + rr;
                    if (rr < nr) {
                        const V v = static_cast<V>(static_cast<double>(Q[(tb.voff + r) * Wp + c]) + acc[rr]);
                        Qh[(tb.hoff + r) * Wp + c] = v;
                        Q[static_cast<int64_t>(pmap[tb.hoff + r]) * Wp + c] = v;
                    }
                }
            }
        }
    }
}

// downward: uhat = Uh + U_parent[pmap]; u[0:k] += uhat; u[k:n] += T^T uhat.
// Tt holds T transposed (column-major m x k) so the second step has the same
// shape as the upward transfer.
template <typename V, typename TT>
__global__ void __launch_bounds__(256) k_downward_mr(const BoxRec* __restrict__ box, const int64_t* __restrict__ toff,
                                                    const int32_t* __restrict__ pmap, int b0, int Wp,
                                                    const TT* __restrict__ Tt, const V* __restrict__ Uh,
                                                    V* __restrict__ U) {
    const int b = b0 + blockIdx.x;
    const BoxRec tb = box[b];
    const int k = tb.k, m = tb.n - tb.k;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TT* __restrict__ Tb = Tt + toff[b];
    for (int c0 = 0; c0 < Wp; c0 += 64) {
        const int c = c0 + lane;
        const bool act = c < Wp;
        // redundant rows (reads uhat inputs: this box's Uh and the parent's U,
        // never this box's own skeleton entries, which the loop after updates)
        for (int r0 = (blockIdx.y * 4 + wave) * kRB; r0 < m; r0 += gridDim.y * 4 * kRB) {
            double acc[kRB];
#pragma unroll
            for (int rr = 0; rr < kRB; ++rr) acc[rr] = 0.0;
            const int nr = min(kRB, m - r0);
            for (int i = 0; i < k; ++i) {
                const double x = act ? static_cast<double>(Uh[(tb.hoff + i) * Wp + c]) +
                                           static_cast<double>(U[static_cast<int64_t>(pmap[tb.hoff + i]) * Wp + c])
                                     : 0.0;
                const TT* col = Tb + r0 + static_cast<int64_t>(i) * ld_pad(m);
                if (nr == kRB) {
#pragma unroll
                    for (int rr = 0; rr < kRB; ++rr) acc[rr] = fma(static_cast<double>(col[rr]), x, acc[rr]);
                } else {
#pragma unroll
                    for (int rr = 0; rr < kRB; ++rr)
                        if (rr < nr) acc[rr] = fma(static_cast<double>(col[rr]), x, acc[rr]);
                }
            }
            if (act) {
#pragma unroll
                for (int rr = 0; rr < kRB; ++rr) {
                    if (rr >= nr) continue;
                    const int64_t e = tb.voff + k + r0 + rr;
                    U[e * Wp + c] = static_cast<V>(static_cast<double>(U[e * Wp + c]) + acc[rr]);
                }
            }
        }
        // skeleton rows (once per box: the blocks of row 0 of the grid)
        for (int i = wave; i < k && act && blockIdx.y == 0; i += 4) {
            const double uh = static_cast<double>(Uh[(tb.hoff + i) * Wp + c]) +
                              static_cast<double>(U[static_cast<int64_t>(pmap[tb.hoff + i]) * Wp + c]);
            U[(tb.voff + i) * Wp + c] = static_cast<V>(static_cast<double>(U[(tb.voff + i) * Wp + c]) + uh);
        }
    }
}

// ---------------------------------------------------------------------------
// many right-hand sides, float32 policy: transfers on the matrix cores
// ---------------------------------------------------------------------------
// The upward transfer of a box is the product qhat = Q_S + T Q_R (T k x m,
// Q_R m x W); the downward one u_R += T^T X with X = uhat + the parent's u at
// the box's slots.  Both are GEMMs C += A B whose left factor A (T, or T^T) is
// read row by row: rows of T are the columns of the stored T^T copy and rows of
// T^T the columns of T, so each is contiguous and padded to a multiple of 32
// entries.  A work item is one block of WPB wavefronts over 32 WPB rows of C
// and one group of 32 NT columns; wave w owns the 32-row tile w and NT 32 x 32
// accumulator tiles of v_mfma_f32_32x32x2f32.  The inner dimension runs in
// chunks of kXK: the block stages the chunk's kXK rows of B in LDS (double
// buffered, one barrier per chunk, the next chunk's loads in flight during the
// current chunk's MFMAs), and each lane holds 16 consecutive entries of its A
// row, so MFMA step u of a chunk pairs column j0 + 16 h + u of A (lane half h)
// with row j0 + 16 h + u of B.  Every kXferFlush chunks the float32 tiles are
// added to float64 totals, so no float32 partial sum holds more than
// 32 kXferFlush products; the MFMA sequence of a tile is the same in every
// launch shape (WPB, NT), so all shapes give the same bits.
constexpr int kXK = 32;          // inner-dimension entries per LDS chunk (16 MFMA steps)
constexpr int kXPitch = 68;      // LDS row pitch in floats (16-byte aligned rows)
constexpr int kXferFlush = 2;    // chunks per float32 partial (64 products)
constexpr int kXferRowsPerWave = 32;

// Row of accumulator register v in a 32 x 32 tile (lane l: column l % 32).
__device__ __forceinline__ int mfma_row(int v, int half) { return 8 * (v / 4) + 4 * half + (v % 4); }

// The lane's 16 entries of its A row for chunk j0 (zeros for a row past the end).
__device__ __forceinline__ void xfer_load_a(const float* __restrict__ arow, int j0, int half, float4 (&a)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
        a[i] = arow ? *reinterpret_cast<const float4*>(arow + j0 + 16 * half + 4 * i) : make_float4(0.f, 0.f, 0.f, 0.f);
}

// 16 MFMA steps of one chunk: B rows from the staged LDS chunk.
template <int NT>
__device__ __forceinline__ void xfer_chunk(const float4 (&a)[4], const float* __restrict__ bs, int lane,
                                           floatx16 (&c)[NT]) {
    const int col = lane & 31, half = lane >> 5;
    const float* av = reinterpret_cast<const float*>(a);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const float* brow = bs + (16 * half + u) * kXPitch + col;
#pragma unroll
        for (int t = 0; t < NT; ++t) c[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], brow[32 * t], c[t], 0, 0, 0);
    }
}

// The GEMM of one work item.  arow: the lane's A row (null past the last row),
// K inner entries; brow(j, q) loads float4 q of B row j (j < K) of the column
// group; the result tiles land in acc (float64).
template <int WPB, int NT, typename BF>
__device__ __forceinline__ void xfer_gemm(const float* __restrict__ arow, bool wave_rows, int K, int ncol4,
                                          BF brow, float* __restrict__ smem, double (&acc)[NT][16]) {
    constexpr int NQ = 8 * NT;                        // float4 per staged row
    constexpr int PER = (kXK * NQ + 64 * WPB - 1) / (64 * WPB);
    const int tid = threadIdx.x, lane = tid & 63, half = lane >> 5;
    const int nch = (K + kXK - 1) / kXK;
    float4 breg[PER];
    auto fetch_b = [&](int j0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + i * 64 * WPB;
            const int r = idx / NQ, q = idx - r * NQ;
            breg[i] = (idx < kXK * NQ && j0 + r < K && q < ncol4) ? brow(j0 + r, q) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + i * 64 * WPB;
            const int r = idx / NQ, q = idx - r * NQ;
            if (idx < kXK * NQ) *reinterpret_cast<float4*>(smem + buf * kXK * kXPitch + r * kXPitch + 4 * q) = breg[i];
        }
    };
    floatx16 c[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) c[t] = floatx16{};
    float4 a[4], an[4];
    if (nch > 0) {
        fetch_b(0);
        if (wave_rows) xfer_load_a(arow, 0, half, a);
        store_b(0);
    }
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const bool more = ch + 1 < nch;
        if (more) {
            fetch_b((ch + 1) * kXK);
            if (wave_rows) xfer_load_a(arow, (ch + 1) * kXK, half, an);
        }
        if (wave_rows) xfer_chunk<NT>(a, smem + (ch & 1) * kXK * kXPitch, lane, c);
        if (wave_rows && (ch % kXferFlush == kXferFlush - 1 || !more)) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    acc[t][v] += static_cast<double>(c[t][v]);
                    c[t][v] = 0.0f;
                }
        }
        if (more) {
            store_b((ch + 1) & 1);
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = an[i];
        }
        __syncthreads();
    }
}

// upward: work item = (box, first row r0 of a block of 32 WPB of its k skeleton
// rows) x column group.  Writes qhat to Qh and to the parent's entries; reads
// this level's entries of Q and writes the parent level's: the two never overlap.
template <int WPB, int NT>
__global__ void __launch_bounds__(256) k_upward_mfma(const int2* __restrict__ work, int ngroups,
                                                    const BoxRec* __restrict__ box, const int64_t* __restrict__ ttoff,
                                                    const int32_t* __restrict__ pmap, int Wp,
                                                    const float* __restrict__ Tt, float* __restrict__ Q,
                                                    float* __restrict__ Qh) {
    __shared__ __align__(16) float smem[2 * kXK * kXPitch];
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int2 wk = work[blockIdx.x / ngroups];
    const int c0 = (blockIdx.x % ngroups) * kMfmaTile * NT;
    const int ncol4 = min(Wp - c0, kMfmaTile * NT) / 4;
    const BoxRec tb = box[wk.x];
    const int k = tb.k, m = tb.n - tb.k;
    const int r0w = wk.y + kXferRowsPerWave * wave;
    const bool wave_rows = r0w < k;
    const int r = r0w + col;
    // row r of T = column r of the stored T^T (m entries, padded)
    const float* arow = (wave_rows && r < k) ? Tt + ttoff[wk.x] + static_cast<int64_t>(r) * ld_pad(m) : nullptr;
    double acc[NT][16];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][v] = 0.0;
    const float* __restrict__ Qr = Q + (tb.voff + k) * Wp + c0;
    xfer_gemm<WPB, NT>(arow, wave_rows, m, ncol4,
                       [&](int j, int q) { return *reinterpret_cast<const float4*>(Qr + static_cast<int64_t>(j) * Wp + 4 * q); },
                       smem, acc);
    if (!wave_rows) return;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int rr = r0w + mfma_row(v, half);
        if (rr < k) {
            const int64_t pe = static_cast<int64_t>(pmap[tb.hoff + rr]) * Wp;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c = c0 + kMfmaTile * t + col;
                if (c >= Wp) continue;
                const float val = static_cast<float>(static_cast<double>(Q[(tb.voff + rr) * Wp + c]) + acc[t][v]);
                Qh[(tb.hoff + rr) * Wp + c] = val;
                Q[pe + c] = val;
            }
        }
    }
}

// downward, first step of a level: x = uhat + the parent's u at the box's slots,
// formed in place in uhat, so the level's GEMMs read contiguous rows.  uhat is
// not read again in the sweep.  Block (box, y) takes float4 elements
// [1024 y, 1024 (y + 1)) of the box's k x Wp values (Wp a multiple of 32), four
// per thread with all loads issued before the stores; gridDim.y covers the
// level's largest k, blocks past a smaller box's end return at once.
constexpr int kPrepUnroll = 4;
template <int UNROLL>
__global__ void __launch_bounds__(256) k_down_prep(const BoxRec* __restrict__ box, const int32_t* __restrict__ pmap,
                                                  int b0, int Wp, const float* __restrict__ U,
                                                  float* __restrict__ Uh) {
    const BoxRec tb = box[b0 + blockIdx.x];
    const int w4 = Wp >> 2;
    const int total = tb.k * w4;
    float4* __restrict__ x = reinterpret_cast<float4*>(Uh + tb.hoff * Wp);
    const int32_t* __restrict__ pm = pmap + tb.hoff;
    for (int e0 = blockIdx.y * (256 * UNROLL) + threadIdx.x; e0 < total; e0 += gridDim.y * (256 * UNROLL)) {
        float4 a[UNROLL], b[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int e = e0 + 256 * u;
            if (e < total) {
                const int i = e / w4;
                a[u] = x[e];
                b[u] = reinterpret_cast<const float4*>(U + static_cast<int64_t>(pm[i]) * Wp)[e - i * w4];
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int e = e0 + 256 * u;
            if (e < total) x[e] = make_float4(a[u].x + b[u].x, a[u].y + b[u].y, a[u].z + b[u].z, a[u].w + b[u].w);
        }
    }
}

// downward: work item = (box, first row r0 of a block of 32 WPB of its m
// redundant rows; a box without redundant rows has one item) x column group:
// u[k + r] += sum_i T^T[r, i] x_i with x (uhat + the parent's u at the slots)
// formed by k_down_prep; the items of row 0 also add x to the box's skeleton
// entries.  Reads x and writes this box's entries only.
template <int WPB, int NT>
__global__ void __launch_bounds__(256) k_downward_mfma(const int2* __restrict__ work, int ngroups,
                                                      const BoxRec* __restrict__ box, const int64_t* __restrict__ toff,
                                                      int Wp, const float* __restrict__ T, const float* __restrict__ X,
                                                      float* __restrict__ U) {
    __shared__ __align__(16) float smem[2 * kXK * kXPitch];
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int2 wk = work[blockIdx.x / ngroups];
    const int c0 = (blockIdx.x % ngroups) * kMfmaTile * NT;
    const int ncol4 = min(Wp - c0, kMfmaTile * NT) / 4;
    const BoxRec tb = box[wk.x];
    const int k = tb.k, m = tb.n - tb.k;
    const float* __restrict__ xb = X + tb.hoff * Wp + c0;
    if (m > 0) {
        const int r0w = wk.y + kXferRowsPerWave * wave;
        const bool wave_rows = r0w < m;
        const int r = r0w + col;
        // row r of T^T = column r of T (k entries, padded)
        const float* arow = (wave_rows && r < m) ? T + toff[wk.x] + static_cast<int64_t>(r) * ld_pad(k) : nullptr;
        double acc[NT][16];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[t][v] = 0.0;
        xfer_gemm<WPB, NT>(arow, wave_rows, k, ncol4,
                           [&](int i, int q) {
                               return *reinterpret_cast<const float4*>(xb + static_cast<int64_t>(i) * Wp + 4 * q);
                           },
                           smem, acc);
        if (wave_rows) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int rr = r0w + mfma_row(v, half);
                if (rr < m) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int c = c0 + kMfmaTile * t + col;
                        if (c >= Wp) continue;
                        float* u = U + (tb.voff + k + rr) * Wp + c;
                        *u = static_cast<float>(static_cast<double>(*u) + acc[t][v]);
                    }
                }
            }
        }
    }
    if (wk.y == 0) {
        const int w = 4 * ncol4;
        for (int e = threadIdx.x; e < k * w; e += blockDim.x) {
            const int i = e / w, c = c0 + e - i * w;
            float* u = U + (tb.voff + i) * Wp + c;
            *u = static_cast<float>(static_cast<double>(*u) + static_cast<double>(X[(tb.hoff + i) * Wp + c]));
        }
    }
}

// ---------------------------------------------------------------------------
// symmetric near field of the complex-symmetric Helmholtz kernels (one RHS)
// ---------------------------------------------------------------------------
// G(x, y) = G(y, x) holds for exp(i kappa r) / (4 pi r) and (i/4) H0^(1)(kappa r)
// as well (the kernel is complex symmetric, not Hermitian), so the terms
// i <- j and j <- i of two distinct colleagues (or distinct top-level boxes)
// share one evaluation of every kernel value, as in the real pair kernel:
//   forward  u_i[t]  += G(t, s) q_j[s]          uhat_i[t] -= G(t, s) qhat_j[s]
//   reverse  u_j[s]  += G(t, s) q_i[t]          uhat_j[s] -= G(t, s) qhat_i[t]
// with complex products (the adjoint conjugates G in both directions).  A box
// paired with itself is left to k_near.  A work item is one wavefront: passes
// of 64 TPL targets of box i in the lanes against the sources of box j in
// wave-uniform blocks of kSymBlockC, read with scalar loads.  Forward
// sums accumulate in float64 per product; reverse sums are formed per block in
// the lanes (TPL products), summed over the lanes in float64 through the
// wave's LDS tile (eight lanes per source and a shuffle tree), and added to
// the item's slot row.  Slot offsets count complex entries (two doubles).
constexpr int kSymBlockC = 8;
constexpr int kSymRowC = 72;     // LDS row pitch: the column reads of a half-wave hit distinct banks

// Column sums of kSymBlockC x 64 lane partials: every lane of source c's group
// of eight receives the float64 sum over the 64 lanes.
template <typename B>
__device__ __forceinline__ double column_sum_c(const B (&r)[kSymBlockC], B* tile, int lane) {
    constexpr int LPS = 64 / kSymBlockC;
#pragma unroll
    for (int c = 0; c < kSymBlockC; ++c) tile[c * kSymRowC + lane] = r[c];
    wave_sync();
    const int c = lane / LPS, q = lane % LPS;
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < kSymBlockC; ++i) v += static_cast<double>(tile[c * kSymRowC + q + LPS * i]);
    wave_sync();
    static_assert(LPS == kSymLanes, "one lane group per source");
    return lane_group_sum(v);
}

template <class P, int TPL, bool CONJ>
__device__ __forceinline__ void sym_pass_c(const SymTask& it, const BoxRec& bi, const BoxRec& bj, int tp,
                                           const Rec4<double>* __restrict__ X, const typename P::Vt* __restrict__ Q,
                                           const typename P::Vt* __restrict__ Qh, double* __restrict__ slots,
                                           typename P::Rt kappa, double sc, typename P::Rt* tile, int lane) {
    using R = typename P::Rt;
    using A = typename P::At;
    const bool first = tp == it.t0;
    const bool hp = tp < bi.k && bj.k > 0;
    double xt[TPL], yt[TPL], zt[TPL];
    R wi[TPL][2], whi[TPL][2];
    A acc[TPL][2], acch[TPL][2];
#pragma unroll
    for (int p = 0; p < TPL; ++p) {
        const int t = tp + lane + 64 * p;
        const bool ok = t < it.t1;
        const int tc = ok ? t : it.t1 - 1;
        const Rec4<double> x = X[bi.voff + tc];
        xt[p] = x.x; yt[p] = x.y; zt[p] = x.z;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            wi[p][v] = ok ? static_cast<R>(Q[(bi.voff + tc) * 2 + v]) : R(0);
            whi[p][v] = (ok && t < bi.k) ? static_cast<R>(Qh[(bi.hoff + t) * 2 + v]) : R(0);
            acc[p][v] = A(0);
            acch[p][v] = A(0);
        }
    }
    double* __restrict__ rev_u = slots + 2 * it.rev_u;
    double* __restrict__ rev_h = slots + 2 * (it.rev_h >= 0 ? it.rev_h : 0);
    // sources in blocks: the skeleton of j first (uhat terms when hp), then the rest
    const int kH = hp ? bj.k : 0;
    const int nbH = (kH + kSymBlockC - 1) / kSymBlockC;
    const int nb = nbH + (bj.n - kH + kSymBlockC - 1) / kSymBlockC;
    const Rec4<double>* __restrict__ Xs = X + bj.voff;
    const int cs = lane / (64 / kSymBlockC);
    for (int b = 0; b < nb; ++b) {
        const bool H = b < nbH;
        const int s0 = H ? b * kSymBlockC : kH + (b - nbH) * kSymBlockC;
        const int cnt = min(kSymBlockC, (H ? kH : bj.n) - s0);
        // the running reverse sums of earlier passes, fetched before the block's arithmetic
        const bool own = (lane % (64 / kSymBlockC)) == 0 && cs < cnt;
        double prev_u[2] = {0.0, 0.0}, prev_h[2] = {0.0, 0.0};
        if (own && !first) {
            prev_u[0] = rev_u[2 * (s0 + cs)];
            prev_u[1] = rev_u[2 * (s0 + cs) + 1];
            if (H) {
                prev_h[0] = rev_h[2 * (s0 + cs)];
                prev_h[1] = rev_h[2 * (s0 + cs) + 1];
            }
        }
        R ru[2][kSymBlockC], rh[2][kSymBlockC];
#pragma unroll
        for (int c = 0; c < kSymBlockC; ++c) {
            // the source's record and charges: wave-uniform scalar loads
            const int si = s0 + min(c, cnt - 1);
            const Rec4<double> sv = Xs[si];
            const bool live = c < cnt;
            const R w0 = live ? static_cast<R>(Q[(bj.voff + si) * 2]) : R(0);
            const R w1 = live ? static_cast<R>(Q[(bj.voff + si) * 2 + 1]) : R(0);
            const R h0 = (live && H) ? static_cast<R>(Qh[(bj.hoff + si) * 2]) : R(0);
            const R h1 = (live && H) ? static_cast<R>(Qh[(bj.hoff + si) * 2 + 1]) : R(0);
#pragma unroll
            for (int v = 0; v < 2; ++v) { ru[v][c] = R(0); rh[v][c] = R(0); }
#pragma unroll
            for (int p = 0; p < TPL; ++p) {
                R gr, gi;
                green<P, CONJ, false>(xt[p] - sv.x, yt[p] - sv.y, zt[p] - sv.z, kappa, gr, gi);
                const A g = static_cast<A>(gr), h = static_cast<A>(gi);
                // forward: acc += G w_j
                acc[p][0] = fma(g, static_cast<A>(w0), fma(-h, static_cast<A>(w1), acc[p][0]));
                acc[p][1] = fma(g, static_cast<A>(w1), fma(h, static_cast<A>(w0), acc[p][1]));
                // reverse partial: G w_i
                ru[0][c] = fma(gr, wi[p][0], fma(-gi, wi[p][1], ru[0][c]));
                ru[1][c] = fma(gr, wi[p][1], fma(gi, wi[p][0], ru[1][c]));
                if (H) {
                    acch[p][0] = fma(g, static_cast<A>(h0), fma(-h, static_cast<A>(h1), acch[p][0]));
                    acch[p][1] = fma(g, static_cast<A>(h1), fma(h, static_cast<A>(h0), acch[p][1]));
                    rh[0][c] = fma(gr, whi[p][0], fma(-gi, whi[p][1], rh[0][c]));
                    rh[1][c] = fma(gr, whi[p][1], fma(gi, whi[p][0], rh[1][c]));
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const double su = column_sum_c<R>(ru[v], tile, lane);
            if (own) rev_u[2 * (s0 + cs) + v] = prev_u[v] + sc * su;
        }
        if (H) {
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const double sh = column_sum_c<R>(rh[v], tile, lane);
                if (own) rev_h[2 * (s0 + cs) + v] = prev_h[v] - sc * sh;
            }
        }
    }
    double* __restrict__ fwd_u = slots + 2 * it.fwd_u;
    double* __restrict__ fwd_h = slots + 2 * (it.fwd_h >= 0 ? it.fwd_h : 0);
#pragma unroll
    for (int p = 0; p < TPL; ++p) {
        const int t = tp + lane + 64 * p;
        if (t < it.t1) {
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                fwd_u[2 * (t - it.t0) + v] = sc * static_cast<double>(acc[p][v]);
                if (t < bi.k) fwd_h[2 * (t - it.t0) + v] = -sc * static_cast<double>(acch[p][v]);
            }
        }
    }
}

template <class P, int TPL, bool CONJ>
__global__ void __launch_bounds__(256) k_near_sym_c(const SymTask* __restrict__ tasks, int ntasks,
                                                    const BoxRec* __restrict__ box,
                                                    const Rec4<double>* __restrict__ X,
                                                    const typename P::Vt* __restrict__ Q,
                                                    const typename P::Vt* __restrict__ Qh,
                                                    double* __restrict__ slots, typename P::Rt kappa, double scale) {
    using R = typename P::Rt;
    __shared__ R tiles[4][kSymBlockC * kSymRowC];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tid = blockIdx.x * 4 + wv;
    if (tid >= ntasks) return;
    const SymTask it = tasks[tid];
    const BoxRec bi = box[it.bi], bj = box[it.bj];
    const double sc = scale * P::gscale;
    for (int tp = it.t0; tp < it.t1; tp += 64 * TPL)
        sym_pass_c<P, TPL, CONJ>(it, bi, bj, tp, X, Q, Qh, slots, kappa, sc, tiles[wv], lane);
}

// Near field for NR right-hand sides per work item (one chunk of Wp): the
// kernel value of a pair is computed once and applied to NR columns.  Partial
// sums of one source box accumulate in Am (float32 for the single-precision
// policies) and are added to float64 totals at the end of the box.
template <class P, int NR, bool CONJ, int MODE, bool MASK, typename Am>
__device__ __forceinline__ void near_loop_mr(const Rec4<double>* __restrict__ X,
                                             const typename P::Vt* __restrict__ Q,
                                             const typename P::Vt* __restrict__ Qh, int Wp, int s0, int s1,
                                             typename P::Rt kappa, double xt, double yt, double zt,
                                             Am (&pu)[NR * P::nv], Am (&ph)[NR * P::nv]) {
    using R = typename P::Rt;
    constexpr int nv = P::nv;
    for (int s = s0; s < s1; ++s) {
        const Rec4<double> xs = X[s];
        R gr, gi;
        green<P, CONJ, MASK>(xt - xs.x, yt - xs.y, zt - xs.z, kappa, gr, gi);
        const Am g = static_cast<Am>(gr);
        const typename P::Vt* __restrict__ w = Q + static_cast<int64_t>(s) * Wp;
        const typename P::Vt* __restrict__ wh = Qh + static_cast<int64_t>(s) * Wp;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if constexpr (nv == 1) {
                Am a = static_cast<Am>(w[r]);
                if constexpr (MODE == 3) a -= static_cast<Am>(wh[r]);
                pu[r] = fma(g, a, pu[r]);
                if constexpr (MODE == 1) ph[r] = fma(-g, static_cast<Am>(wh[r]), ph[r]);
                if constexpr (MODE == 2) ph[r] = fma(-g, a, ph[r]);
            } else {
                const Am h = static_cast<Am>(gi);
                Am a0 = static_cast<Am>(w[2 * r]), a1 = static_cast<Am>(w[2 * r + 1]);
                if constexpr (MODE == 3) { a0 -= static_cast<Am>(wh[2 * r]); a1 -= static_cast<Am>(wh[2 * r + 1]); }
                pu[2 * r] = fma(g, a0, fma(-h, a1, pu[2 * r]));
                pu[2 * r + 1] = fma(g, a1, fma(h, a0, pu[2 * r + 1]));
                if constexpr (MODE == 1) {
                    const Am b0 = static_cast<Am>(wh[2 * r]), b1 = static_cast<Am>(wh[2 * r + 1]);
                    ph[2 * r] = fma(-g, b0, fma(h, b1, ph[2 * r]));
                    ph[2 * r + 1] = fma(-g, b1, fma(-h, b0, ph[2 * r + 1]));
                }
                if constexpr (MODE == 2) {
                    ph[2 * r] = fma(-g, a0, fma(h, a1, ph[2 * r]));
                    ph[2 * r + 1] = fma(-g, a1, fma(-h, a0, ph[2 * r + 1]));
                }
            }
        }
    }
}

template <class P, int NR, bool CONJ, typename Am>
__global__ void __launch_bounds__(256) k_near_mr(const Task* __restrict__ tasks, int ntasks, int nchunks,
                                                 int Wp, const int32_t* __restrict__ seg_ptr,
                                                 const int2* __restrict__ segs, const BoxRec* __restrict__ box,
                                                 const Rec4<double>* __restrict__ X,
                                                 const typename P::Vt* __restrict__ Q,
                                                 const typename P::Vt* __restrict__ Qh,
                                                 typename P::Vt* __restrict__ U, typename P::Vt* __restrict__ Uh,
                                                 typename P::Rt kappa, double scale) {
    using V = typename P::Vt;
    constexpr int nv = P::nv;
    constexpr int NW = NR * nv;
    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wid >= ntasks * nchunks) return;
    const int chunk = wid % nchunks;
    const Task tk = tasks[wid / nchunks];
    const BoxRec tb = box[tk.box];
    // boxes at or above the top level carry k = 0: no skeleton part
    const bool has_h = tk.t0 < tb.k;
    const int c0 = chunk * NW;
    const int t = min(tk.t0 + lane, tb.n - 1);
    const Rec4<double> xr = X[tb.voff + t];
    const double xt = xr.x, yt = xr.y, zt = xr.z;
    double au[NW], ah[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v) { au[v] = 0.0; ah[v] = 0.0; }
    const int e1 = seg_ptr[tk.box + 1];
    for (int e = seg_ptr[tk.box]; e < e1; ++e) {
        const int2 sg = segs[e];
        const BoxRec sb = box[sg.x];
        const Rec4<double>* Xs = X + sb.voff;
        const V* Qs = Q + sb.voff * Wp + c0;
        const V* Qhs = Qh + sb.hoff * Wp + c0;
        const int mode = sg.y & SEG_MODE_MASK;
        Am pu[NW], ph[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) { pu[v] = Am(0); ph[v] = Am(0); }
        const bool self = (sg.y & SEG_SELF) != 0;
#define SKF_MR(MD, A0, A1)                                                                                 \
        do {                                                                                               \
            if (self) near_loop_mr<P, NR, CONJ, MD, true, Am>(Xs, Qs, Qhs, Wp, A0, A1, kappa, xt, yt, zt, pu, ph); \
            else near_loop_mr<P, NR, CONJ, MD, false, Am>(Xs, Qs, Qhs, Wp, A0, A1, kappa, xt, yt, zt, pu, ph);    \
        } while (0)
        if (mode == SEG_IFO) {
            if (has_h) { SKF_MR(1, 0, sb.k); SKF_MR(0, sb.k, sb.n); }
            else SKF_MR(0, 0, sb.n);
        } else if (mode == SEG_IFS) {
            if (has_h) SKF_MR(2, 0, sb.n);
            else SKF_MR(0, 0, sb.n);
        } else if (mode == SEG_TFO) {
            SKF_MR(3, 0, sb.k); SKF_MR(0, sb.k, sb.n);
        } else {
            SKF_MR(0, 0, sb.n);
        }
#undef SKF_MR
#pragma unroll
        for (int v = 0; v < NW; ++v) { au[v] += static_cast<double>(pu[v]); ah[v] += static_cast<double>(ph[v]); }
    }
    const double sc = scale * P::gscale;
    const int tt = tk.t0 + lane;
    if (tt < tb.n) {
#pragma unroll
        for (int v = 0; v < NW; ++v) U[(tb.voff + tt) * Wp + c0 + v] = static_cast<V>(au[v] * sc);
        if (has_h && tt < tb.k) {
#pragma unroll
            for (int v = 0; v < NW; ++v) Uh[(tb.hoff + tt) * Wp + c0 + v] = static_cast<V>(ah[v] * sc);
        }
    }
}

}  // namespace kern
}  // namespace skelfmm
