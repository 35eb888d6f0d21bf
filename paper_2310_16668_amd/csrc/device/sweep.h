// Templates of the GPU sweep, shared by the translation units that
// instantiate it (one per kernel family, so they compile in parallel) and by
// the executor in exec.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "device.h"
#include "kernels.hip"

namespace skelfmm {

#define SKF_HIP(x)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) {                                                                    \
            if (e_ == hipErrorOutOfMemory) throw OutOfMemory(std::string(#x) + ": out of memory"); \
            throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_));                    \
        }                                                                                          \
    } while (0)

struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // 256 spare bytes keep merged wave-uniform loads at the end of an array in bounds
    void alloc(size_t b) {
        release();
        SKF_HIP(hipMalloc(&p, b + 256));
        bytes = b;
    }
    template <class T>
    void upload(const std::vector<T>& v) {
        alloc(v.size() * sizeof(T));
        if (!v.empty()) SKF_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

inline int dtype_is_complex(int dt) { return dt == SKELFMM_C128 || dt == SKELFMM_C64; }
inline int dtype_is_single(int dt) { return dt == SKELFMM_F32 || dt == SKELFMM_C64; }

inline constexpr int kDefaultTPL = 2;   // targets per lane in the single-RHS near-field kernels (1 .. 4)
inline constexpr int kChunkReals = 8;   // right-hand-side reals per multi-RHS near-field work item

inline int tpl_slot(int tpl) { return tpl - 1; }

// Several right-hand sides of a real kernel in the float32 policy run the near
// field on the matrix cores (k_near_mfma) from 8 columns on.
inline constexpr int kMfmaMinRhs = 8;
inline constexpr int kMfmaCols = 32;     // columns per accumulator tile

// Values per entry inside the workspace: nv for one RHS; several RHS are padded
// to a multiple of the near-field chunk (of the accumulator tile on the matrix
// core path).
inline int64_t padded_width(int64_t nrhs, int dtype, bool mfma) {
    const int64_t w = nrhs * (dtype_is_complex(dtype) ? 2 : 1);
    if (nrhs == 1) return w;
    const int64_t m = mfma ? kMfmaCols : kChunkReals;
    return (w + m - 1) / m * m;
}

inline unsigned blocks_for(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

// Launch shapes of the matrix-core transfers (wavefronts per block, 32-column
// tiles per wave).  None changes the arithmetic of an output tile, so they give
// identical results and only the fastest matters.
struct XferShape { int wpb, nt; };
inline constexpr XferShape kXferShapes[SKELFMM_NXFER] = {{4, 2}, {4, 1}, {2, 2}, {2, 1}};
inline constexpr int kDefaultXfer = 0;

// Workspace of one sweep: the entry vectors q, qhat, u, uhat (n_entries or
// n_hentries x padded width) and the pair kernel's float64 slots.
struct Work {
    void* Q;
    void* Qh;
    void* U;
    void* Uh;
    double* slots;
    bool marks;     // per-pass events when the operator's timing is on
};

// A level of uncompressed boxes whose entries [e0, e0 + cnt) and skeleton
// entries [h0, h0 + cnt) correspond one to one (cnt = 0: not such a level).
struct FlatLevel {
    int64_t e0 = 0, h0 = 0, cnt = 0;
};

struct DeviceOp {
    Layout L;
    bool f64_leaf = false;
    bool compensated = false;   // float32 pair kernel: compensated leaf sums
    int device = -1;
    bool uploaded = false;
    // static arrays
    DevMem voff, hoff, toff, ttoff, nb, kb, pmap, gather_e, gather_p;
    DevMem X64, T64, T32, Tt64, Tt32;             // T and its per-box transposes, columns padded
    DevMem XE64;                                  // expanded source records of the pair kernel
    DevMem XF32;                                  // float32 relative coordinates (f32_differences)
    DevMem seg_ptr, segs, boxrec;
    // one-RHS transfer work: (box, first row) items per level, and waves per item
    // [0]: float64 T row groups, [1]: float32, [2] / [3]: 64- / 128-row blocks of
    // the matrix-core transfers
    DevMem upwork[4], downwork[4];
    std::vector<int64_t> up_ptr[4], down_ptr[4];
    std::vector<int> up_nw, down_nw;
    std::vector<int> up_rows, down_rows;          // per level: most output rows of a box (k up, n - k down)
    std::vector<FlatLevel> flat;                  // per level: elementwise transfers (all boxes uncompressed)
    int tpl = kDefaultTPL;
    int tpl2 = kDefaultTPL;                       // the same for a forward + adjoint sweep (two columns)
    int xfer = kDefaultXfer;                      // launch shape of the matrix-core transfers
    DevMem tasks[SKELFMM_NTPL];                   // work lists for 1 .. 4 targets per lane
    int ntasks[SKELFMM_NTPL] = {};
    // symmetric near field (one RHS): segment lists without the paired ifo
    // terms, their work lists, the pair items, the slot reduction lists
    DevMem seg_ptr_ns, segs_ns, tasks_ns[SKELFMM_NTPL], symtasks, symrows, slots;
    int ntasks_ns[SKELFMM_NTPL] = {};
    DevMem tasks32;                               // 32-target work list of the matrix-core near field
    int ntasks32 = 0;
    int ntasks32h = 0;                            // its first ntasks32h items hold uhat rows
    int nsym = 0, nred = 0;
    // workspace
    DevMem Q, Qh, U, Uh;
    // per-pass timing
    bool timing = false;
    std::vector<std::array<hipEvent_t, SKELFMM_NPASS + 1>> pending;
    double pass_ms[SKELFMM_NPASS] = {};
    int64_t sweeps = 0;
    Work own_work() const { return Work{Q.p, Qh.p, U.p, Uh.p, slots.as<double>(), true}; }
    ~DeviceOp() {
        for (auto& ev : pending)
            for (auto e : ev) (void)hipEventDestroy(e);
    }
};

// The matrix-core near field serves several RHS of a real kernel in the
// float32 policy.
inline bool use_mfma(const DeviceOp* d, int64_t nrhs, int dtype) {
    return d->L.kind == 0 && dtype == SKELFMM_F32 && !d->f64_leaf && nrhs >= kMfmaMinRhs;
}

struct DeviceBatch {
    std::vector<DeviceOp*> ops;
    std::unique_ptr<DeviceOp> merged;
    std::vector<int64_t> gbase;                   // first gather-list index of each operator
};


// The caller's buffers of one operator and its range of leaf entries.
struct IO {
    const void* q;
    void* u;
    int64_t g0;     // first index into the gather lists
    int64_t cnt;    // number of points
    // a forward and an adjoint apply in one sweep (real kernels): the second
    // input and output, interleaved with q and u inside the sweep
    const void* q2 = nullptr;
    void* u2 = nullptr;
};

// Events bracketing the passes of one sweep (only when timing is on).
struct PassMarks {
    DeviceOp* d;
    hipStream_t s;
    bool on;
    std::array<hipEvent_t, SKELFMM_NPASS + 1> ev{};
    PassMarks(DeviceOp* d_, hipStream_t s_, bool allowed) : d(d_), s(s_), on(allowed && d_->timing) {
        if (!on) return;
        for (auto& e : ev) SKF_HIP(hipEventCreate(&e));
    }
    void mark(int i) {
        if (on) SKF_HIP(hipEventRecord(ev[i], s));
    }
    void done() {
        if (on) d->pending.push_back(ev);
    }
};

// The one-RHS near field: k_near over the segment lists; with symmetric pairing
// it covers what is left after pairing, then k_near_sym evaluates the pairs
// into slots and k_sym_reduce adds the slots to u and uhat.
template <class P, int TPL, bool CONJ>
void launch_near_t(const DeviceOp* d, hipStream_t s, void* Q, void* Qh, void* U, void* Uh, double* slots,
                   PassMarks* pm) {
    using R = typename P::Rt;
    using V = typename P::Vt;
    const int ts = tpl_slot(TPL);
    const bool sym = d->L.sym;
    const int ntasks = sym ? d->ntasks_ns[ts] : d->ntasks[ts];
    if (ntasks > 0) {
        hipLaunchKernelGGL((kern::k_near<P, TPL, CONJ>), dim3(blocks_for(ntasks, 4)), dim3(256), 0, s,
                           (sym ? d->tasks_ns[ts] : d->tasks[ts]).as<Task>(), ntasks,
                           (sym ? d->seg_ptr_ns : d->seg_ptr).as<int32_t>(), (sym ? d->segs_ns : d->segs).as<int2>(),
                           d->boxrec.as<kern::BoxRec>(), d->X64.as<kern::Rec4<double>>(), static_cast<const V*>(Q),
                           static_cast<const V*>(Qh), static_cast<V*>(U), static_cast<V*>(Uh),
                           static_cast<R>(d->L.kappa), kern::kscale<P>());
        SKF_HIP(hipGetLastError());
    }
    if (pm) pm->mark(3);
    if constexpr (P::kind == 0) {
        if (sym && d->nsym > 0) {
            const auto launch = [&](auto kern_fn) {
                hipLaunchKernelGGL(kern_fn, dim3(blocks_for(d->nsym, 4)), dim3(256), 0, s, d->symtasks.as<SymTask>(),
                                   d->nsym, d->boxrec.as<kern::BoxRec>(), d->X64.as<kern::Rec4<double>>(),
                                   d->XE64.as<kern::Rec4<double>>(), d->XF32.as<kern::Rec4<float>>(),
                                   static_cast<const V*>(Q), static_cast<const V*>(Qh), slots, kern::kscale<P>());
            };
            // the compensated leaf sums and the float32 differences only change the
            // float32 evaluation
            if constexpr (sizeof(R) == 4) {
                const bool f32d = d->L.allow_f32diff;
                if (d->compensated) {
                    if (f32d) launch(kern::k_near_sym<kern::WithComp<P>, TPL, true>);
                    else launch(kern::k_near_sym<kern::WithComp<P>, TPL, false>);
                } else {
                    if (f32d) launch(kern::k_near_sym<P, TPL, true>);
                    else launch(kern::k_near_sym<P, TPL, false>);
                }
            } else {
                launch(kern::k_near_sym<P, TPL, false>);
            }
            SKF_HIP(hipGetLastError());
        }
    }
    if constexpr (P::kind == 1) {
        if (sym && d->nsym > 0) {
            hipLaunchKernelGGL((kern::k_near_sym_c<P, TPL, CONJ>), dim3(blocks_for(d->nsym, 4)), dim3(256), 0, s,
                               d->symtasks.as<SymTask>(), d->nsym, d->boxrec.as<kern::BoxRec>(),
                               d->X64.as<kern::Rec4<double>>(), static_cast<const V*>(Q), static_cast<const V*>(Qh),
                               slots, static_cast<R>(d->L.kappa), kern::kscale<P>());
            SKF_HIP(hipGetLastError());
        }
    }
    if (pm) pm->mark(4);
    if constexpr (P::kind == 1) {
        if (sym && d->nred > 0) {
            hipLaunchKernelGGL((kern::k_sym_reduce<V, 2>), dim3(d->nred), dim3(256), 0, s, d->symrows.as<SymRows>(),
                               d->boxrec.as<kern::BoxRec>(), slots, static_cast<V*>(U), static_cast<V*>(Uh));
            SKF_HIP(hipGetLastError());
        }
    }
    if constexpr (P::kind == 0) {
        if (sym && d->nred > 0) {
            hipLaunchKernelGGL((kern::k_sym_reduce<V, P::nv>), dim3(d->nred), dim3(256), 0, s, d->symrows.as<SymRows>(),
                               d->boxrec.as<kern::BoxRec>(), slots, static_cast<V*>(U),
                               static_cast<V*>(Uh));
            SKF_HIP(hipGetLastError());
        }
    }
}

template <class P, bool CONJ>
void launch_near(const DeviceOp* d, hipStream_t s, const Work& w, PassMarks* pm = nullptr) {
    const int tpl = P::rhs == 2 ? d->tpl2 : d->tpl;
    if (tpl == 1) launch_near_t<P, 1, CONJ>(d, s, w.Q, w.Qh, w.U, w.Uh, w.slots, pm);
    else if (tpl == 3) launch_near_t<P, 3, CONJ>(d, s, w.Q, w.Qh, w.U, w.Uh, w.slots, pm);
    else if (tpl == 4) launch_near_t<P, 4, CONJ>(d, s, w.Q, w.Qh, w.U, w.Uh, w.slots, pm);
    else launch_near_t<P, 2, CONJ>(d, s, w.Q, w.Qh, w.U, w.Uh, w.slots, pm);
}

template <class P, bool CONJ, typename Am>
void launch_near_mr(const DeviceOp* d, hipStream_t s, int Wp, void* Q, void* Qh, void* U, void* Uh) {
    const int ntasks = d->ntasks[tpl_slot(1)];
    if (ntasks == 0) return;
    using R = typename P::Rt;
    using V = typename P::Vt;
    constexpr int NR = kChunkReals / P::nv;
    const int nchunks = Wp / kChunkReals;
    hipLaunchKernelGGL((kern::k_near_mr<P, NR, CONJ, Am>), dim3(blocks_for(int64_t(ntasks) * nchunks, 4)),
                       dim3(256), 0, s, d->tasks[tpl_slot(1)].as<Task>(), ntasks, nchunks, Wp,
                       d->seg_ptr.as<int32_t>(), d->segs.as<int2>(), d->boxrec.as<kern::BoxRec>(),
                       d->X64.as<kern::Rec4<double>>(), static_cast<const V*>(Q), static_cast<const V*>(Qh), static_cast<V*>(U), static_cast<V*>(Uh),
                       static_cast<R>(d->L.kappa), kern::kscale<P>());
    SKF_HIP(hipGetLastError());
}

// Tasks with uhat rows come first in the list (nh of them).  One column tile:
// k_near_mfma over every task; more: two tiles per wave, one launch per list.
template <class P>
void launch_near_mfma(const DeviceOp* d, hipStream_t s, int Wp, void* Q, void* Qh, void* U, void* Uh) {
    static_assert(kMfmaCols == kern::kMfmaTile, "one accumulator tile width");
    const int nt = d->ntasks32, nh = d->ntasks32h, nn = nt - nh;
    const int ntiles = Wp / kMfmaCols, npairs = (ntiles + 1) / 2;
    const Task* tl = d->tasks32.as<Task>();
    const auto* X = d->X64.as<kern::Rec4<double>>();
    const float* Qf = static_cast<const float*>(Q);
    const float* Qhf = static_cast<const float*>(Qh);
    float* Uf = static_cast<float*>(U);
    float* Uhf = static_cast<float*>(Uh);
    if (ntiles == 1) {
        if (nt > 0)
            hipLaunchKernelGGL((kern::k_near_mfma<P>), dim3(blocks_for(nt, 4)), dim3(256), 0, s, tl, nt, 1, Wp,
                               d->seg_ptr.as<int32_t>(), d->segs.as<int2>(), d->boxrec.as<kern::BoxRec>(), X, Qf,
                               Qhf, Uf, Uhf, kern::kscale<P>());
        SKF_HIP(hipGetLastError());
        return;
    }
    if (nh > 0)
        hipLaunchKernelGGL((kern::k_near_mfma2<P, true>), dim3(blocks_for(int64_t(nh) * npairs, 4)), dim3(256), 0,
                           s, tl, nh, npairs, Wp, d->seg_ptr.as<int32_t>(), d->segs.as<int2>(),
                           d->boxrec.as<kern::BoxRec>(), X, Qf, Qhf, Uf, Uhf, kern::kscale<P>());
    if (nn > 0)
        hipLaunchKernelGGL((kern::k_near_mfma2<P, false>), dim3(blocks_for(int64_t(nn) * npairs, 4)), dim3(256), 0,
                           s, tl + nh, nn, npairs, Wp, d->seg_ptr.as<int32_t>(), d->segs.as<int2>(),
                           d->boxrec.as<kern::BoxRec>(), X, Qf, Qhf, Uf, Uhf, kern::kscale<P>());
    SKF_HIP(hipGetLastError());
}

// Matrix-core transfers of one level (float32 policy, several RHS): one launch
// over the level's row blocks x column groups, in the operator's launch shape.
// The upward pass reads rows of T from the stored T^T, the downward pass rows of
// T^T from the stored T.
template <int WPB, int NT>
void xfer_level_t(const DeviceOp* d, hipStream_t s, bool up, int l, int Wp, const float* T, float* Q, float* Qh,
                  const float* Tt, float* Uh, float* U) {
    const int g = WPB == 2 ? 2 : 3;
    const auto& ptr = up ? d->up_ptr[g] : d->down_ptr[g];
    const int64_t w0 = ptr[l], nwk = ptr[l + 1] - w0;
    if (nwk <= 0) return;
    const int ng = (Wp + kMfmaCols * NT - 1) / (kMfmaCols * NT);
    const unsigned nb = static_cast<unsigned>(nwk * ng);
    if (up)
        hipLaunchKernelGGL((kern::k_upward_mfma<WPB, NT>), dim3(nb), dim3(64 * WPB), 0, s,
                           d->upwork[g].as<int2>() + w0, ng, d->boxrec.as<kern::BoxRec>(), d->ttoff.as<int64_t>(),
                           d->pmap.as<int32_t>(), Wp, Tt, Q, Qh);
    else {
        const int b0 = d->L.level_ptr[l], nbx = d->L.level_ptr[l + 1] - b0;
        const int64_t per_y = 256 * kern::kPrepUnroll, vals = int64_t(d->up_rows[l]) * (Wp / 4);
        const unsigned ny = static_cast<unsigned>(std::min<int64_t>(65535, std::max<int64_t>(1, (vals + per_y - 1) / per_y)));
        hipLaunchKernelGGL(kern::k_down_prep<kern::kPrepUnroll>, dim3(nbx, ny), dim3(256), 0, s, d->boxrec.as<kern::BoxRec>(),
                           d->pmap.as<int32_t>(), b0, Wp, U, Uh);
        SKF_HIP(hipGetLastError());
        hipLaunchKernelGGL((kern::k_downward_mfma<WPB, NT>), dim3(nb), dim3(64 * WPB), 0, s,
                           d->downwork[g].as<int2>() + w0, ng, d->boxrec.as<kern::BoxRec>(), d->toff.as<int64_t>(),
                           Wp, T, Uh, U);
    }
    SKF_HIP(hipGetLastError());
}

inline void xfer_level(const DeviceOp* d, hipStream_t s, bool up, int l, int Wp, const float* T, float* Q,
                       float* Qh, const float* Tt, float* Uh, float* U) {
    const XferShape sh = kXferShapes[d->xfer];
    if (sh.wpb == 4 && sh.nt == 2) xfer_level_t<4, 2>(d, s, up, l, Wp, T, Q, Qh, Tt, Uh, U);
    else if (sh.wpb == 4) xfer_level_t<4, 1>(d, s, up, l, Wp, T, Q, Qh, Tt, Uh, U);
    else if (sh.nt == 2) xfer_level_t<2, 2>(d, s, up, l, Wp, T, Q, Qh, Tt, Uh, U);
    else xfer_level_t<2, 1>(d, s, up, l, Wp, T, Q, Qh, Tt, Uh, U);
}

// One sweep.  V: stored values; TT: transfer matrices; P: near-field policy;
// Am: accumulator of one source box's partial sums in the multi-RHS near field.
template <typename V, typename TT, class P, typename Am>
void sweep(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
           const Work& w, const TT* T, const TT* Tt) {
    const Layout& L = d->L;
    const bool multi = nrhs > 1;
    const int Win = static_cast<int>(nrhs * P::nv);
    const bool mfma = use_mfma(d, nrhs, dtype);
    // one RHS: P::nv values per entry (a complex value, or a forward and an
    // adjoint column of a real kernel), unpadded
    const int Wp = multi ? static_cast<int>(padded_width(nrhs, dtype, mfma)) : P::nv;
    static_assert(P::rhs == 1 || P::kind == 0, "interleaved columns are for real kernels");
    V* Q = static_cast<V*>(w.Q);
    V* Qh = static_cast<V*>(w.Qh);
    V* U = static_cast<V*>(w.U);
    V* Uh = static_cast<V*>(w.Uh);
    const kern::BoxRec* br = d->boxrec.as<kern::BoxRec>();
    const int64_t* toff = d->toff.as<int64_t>();
    const int64_t* ttoff = d->ttoff.as<int64_t>();
    const int32_t* pmap = d->pmap.as<int32_t>();
    const int32_t* ge = d->gather_e.as<int32_t>();
    const int32_t* gp = d->gather_p.as<int32_t>();
    PassMarks pm(d, s, w.marks);
    pm.mark(0);
    for (const IO& x : io) {
        if (x.cnt <= 0) continue;
        if constexpr (P::rhs == 2)
            hipLaunchKernelGGL((kern::k_gather2<V>), dim3(blocks_for(x.cnt, 256)), dim3(256), 0, s, ge + x.g0,
                               gp + x.g0, x.cnt, static_cast<const V*>(x.q), static_cast<const V*>(x.q2), Q);
        else
            hipLaunchKernelGGL((kern::k_gather_pad<V, V>), dim3(blocks_for(x.cnt * Wp, 256)), dim3(256), 0, s,
                               ge + x.g0, gp + x.g0, x.cnt, Win, Wp, static_cast<const V*>(x.q), Q);
        SKF_HIP(hipGetLastError());
    }
    pm.mark(1);
    for (int l = L.max_level; l >= 2; --l) {
        const int b0 = L.level_ptr[l], nbx = L.level_ptr[l + 1] - b0;
        if (nbx <= 0) continue;
        if constexpr (std::is_same_v<V, float> && std::is_same_v<TT, float>) {
            if (mfma) {
                xfer_level(d, s, true, l, Wp, T, Q, Qh, Tt, Uh, U);
                continue;
            }
        }
        if (multi) {
            // row chunks of a box spread over the grid's second dimension (4 per block)
            const int gy = std::max(1, (d->up_rows[l] + 4 * kern::kRB - 1) / (4 * kern::kRB));
            hipLaunchKernelGGL((kern::k_upward_mr<V, TT>), dim3(nbx, gy), dim3(256), 0, s, br, toff, pmap, b0, Wp,
                               T, Q, Qh);
        } else if (const FlatLevel& fl = d->flat[l]; fl.cnt > 0) {
            hipLaunchKernelGGL((kern::k_up_flat<V, P::nv>), dim3(blocks_for(fl.cnt * P::nv, 256)), dim3(256), 0, s,
                               fl.e0, fl.h0, fl.cnt, pmap, Q, Q, Qh);
        } else {
            const int wg = sizeof(TT) == 4 ? 1 : 0;
            const int64_t w0 = d->up_ptr[wg][l], nwk = d->up_ptr[wg][l + 1] - w0;
            if (nwk <= 0) continue;
            const int nw = d->up_nw[l];
            const int2* wk = d->upwork[wg].as<int2>() + w0;
            if (P::nv == 1)
                hipLaunchKernelGGL((kern::k_up_gemv<V, TT, 1>), dim3(nwk), dim3(64 * nw), 0, s, wk, br, toff, pmap, T,
                                   Q, Q, Qh, nw);
            else
                hipLaunchKernelGGL((kern::k_up_gemv<V, TT, 2>), dim3(nwk), dim3(64 * nw), 0, s, wk, br, toff, pmap, T,
                                   Q, Q, Qh, nw);
        }
        SKF_HIP(hipGetLastError());
    }
    pm.mark(2);
    if (multi) {
        if constexpr (P::kind == 0 && sizeof(typename P::Rt) == 4) {
            if (mfma) launch_near_mfma<P>(d, s, Wp, Q, Qh, U, Uh);
            else launch_near_mr<P, false, Am>(d, s, Wp, Q, Qh, U, Uh);
        } else {
            if (adjoint && P::kind == 1) launch_near_mr<P, true, Am>(d, s, Wp, Q, Qh, U, Uh);
            else launch_near_mr<P, false, Am>(d, s, Wp, Q, Qh, U, Uh);
        }
        pm.mark(3);
        pm.mark(4);
    } else {
        if (adjoint && P::kind == 1) launch_near<P, true>(d, s, w, &pm);
        else launch_near<P, false>(d, s, w, &pm);
    }
    pm.mark(5);
    for (int l = 2; l <= L.max_level; ++l) {
        const int b0 = L.level_ptr[l], nbx = L.level_ptr[l + 1] - b0;
        if (nbx <= 0) continue;
        if constexpr (std::is_same_v<V, float> && std::is_same_v<TT, float>) {
            if (mfma) {
                xfer_level(d, s, false, l, Wp, T, Q, Qh, Tt, Uh, U);
                continue;
            }
        }
        if (multi) {
            const int gy = std::max(1, (d->down_rows[l] + 4 * kern::kRB - 1) / (4 * kern::kRB));
            hipLaunchKernelGGL((kern::k_downward_mr<V, TT>), dim3(nbx, gy), dim3(256), 0, s, br, ttoff, pmap, b0, Wp,
                               Tt, Uh, U);
        } else if (const FlatLevel& fl = d->flat[l]; fl.cnt > 0) {
            hipLaunchKernelGGL((kern::k_down_flat<V, P::nv>), dim3(blocks_for(fl.cnt * P::nv, 256)), dim3(256), 0,
                               s, fl.e0, fl.h0, fl.cnt, pmap, Uh, U, U);
        } else {
            const int wg = sizeof(TT) == 4 ? 1 : 0;
            const int64_t w0 = d->down_ptr[wg][l], nwk = d->down_ptr[wg][l + 1] - w0;
            if (nwk <= 0) continue;
            const int nw = d->down_nw[l];
            const int2* wk = d->downwork[wg].as<int2>() + w0;
            if (P::nv == 1)
                hipLaunchKernelGGL((kern::k_down_gemv<V, TT, 1>), dim3(nwk), dim3(64 * nw), 0, s, wk, br, ttoff, pmap,
                                   Tt, Uh, U, U, nw);
            else
                hipLaunchKernelGGL((kern::k_down_gemv<V, TT, 2>), dim3(nwk), dim3(64 * nw), 0, s, wk, br, ttoff, pmap,
                                   Tt, Uh, U, U, nw);
        }
        SKF_HIP(hipGetLastError());
    }
    pm.mark(6);
    for (const IO& x : io) {
        if (x.cnt <= 0) continue;
        if constexpr (P::rhs == 2)
            hipLaunchKernelGGL((kern::k_scatter2<V>), dim3(blocks_for(x.cnt, 256)), dim3(256), 0, s, ge + x.g0,
                               gp + x.g0, x.cnt, U, static_cast<V*>(x.u), static_cast<V*>(x.u2));
        else
            hipLaunchKernelGGL((kern::k_scatter_pad<V, V>), dim3(blocks_for(x.cnt * Win, 256)), dim3(256), 0, s,
                               ge + x.g0, gp + x.g0, x.cnt, Win, Wp, U, static_cast<V*>(x.u));
        SKF_HIP(hipGetLastError());
    }
    pm.mark(7);
    pm.done();
}

template <int DIM, int KIND>
void dispatch(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
              const Work& w) {
    if (dtype == SKELFMM_F64 || dtype == SKELFMM_C128) {
        using P = kern::Pol<double, double, double, DIM, KIND>;
        sweep<double, double, P, double>(d, io, nrhs, dtype, s, adjoint, w, d->T64.as<double>(), d->Tt64.as<double>());
    } else if (d->f64_leaf) {
        using P = kern::Pol<double, double, float, DIM, KIND>;
        sweep<float, float, P, double>(d, io, nrhs, dtype, s, adjoint, w, d->T32.as<float>(), d->Tt32.as<float>());
    } else {
        using P = kern::Pol<float, double, float, DIM, KIND>;
        sweep<float, float, P, float>(d, io, nrhs, dtype, s, adjoint, w, d->T32.as<float>(), d->Tt32.as<float>());
    }
}


// A forward apply (io's q -> u) and an adjoint apply (q2 -> u2) of a real
// kernel in one float32 sweep: the adjoint of a real symmetric kernel's
// operator is the operator itself (the skeletons and T serve rows and columns
// alike), so the two vectors go through the sweep as two interleaved columns
// and share every kernel value of the near field.
template <int DIM>
void dispatch_pair(DeviceOp* d, const std::vector<IO>& io, hipStream_t s, const Work& w) {
    using P = kern::Pol<float, double, float, DIM, 0, false, 2>;
    sweep<float, float, P, float>(d, io, 1, SKELFMM_F32, s, false, w, d->T32.as<float>(), d->Tt32.as<float>());
}

// Time the near-field launches for 1 .. 4 targets per lane on this operator
// (workspace contents are whatever the last apply left; timing does not depend
// on values) and keep the fastest.  pair: the two-column near field of the
// forward + adjoint sweep (its own setting, tpl2).
template <int DIM, int KIND>
void tune_near(DeviceOp* d, int dtype, hipStream_t s, float* ms_out, bool pair = false) {
    const bool single = dtype_is_single(dtype);
    int& tpl = pair ? d->tpl2 : d->tpl;
    for (int t : {1, 2, 3, 4}) {
        tpl = t;
        hipEvent_t a, b;
        SKF_HIP(hipEventCreate(&a));
        SKF_HIP(hipEventCreate(&b));
        for (int rep = 0; rep < 4; ++rep) {
            if (rep == 1) SKF_HIP(hipEventRecord(a, s));
            if constexpr (KIND == 0) {
                if (pair) {
                    using P = kern::Pol<float, double, float, DIM, 0, false, 2>;
                    launch_near<P, false>(d, s, d->own_work());
                    continue;
                }
            }
            if (!single) {
                using P = kern::Pol<double, double, double, DIM, KIND>;
                launch_near<P, false>(d, s, d->own_work());
            } else if (d->f64_leaf) {
                using P = kern::Pol<double, double, float, DIM, KIND>;
                launch_near<P, false>(d, s, d->own_work());
            } else {
                using P = kern::Pol<float, double, float, DIM, KIND>;
                launch_near<P, false>(d, s, d->own_work());
            }
        }
        SKF_HIP(hipEventRecord(b, s));
        SKF_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        SKF_HIP(hipEventElapsedTime(&ms, a, b));
        ms_out[tpl_slot(t)] = ms / 3.0f;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    int best = 1;
    for (int t : {1, 2, 3, 4})
        if (ms_out[tpl_slot(t)] < ms_out[tpl_slot(best)]) best = t;
    tpl = best;
}


// One sweep / near-field autotune per kernel family (sweep_*.hip).
void sweep_lap2(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
                 const Work& w);
void sweep_lap3(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
                 const Work& w);
void sweep_helm3(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
                 const Work& w);
void sweep_helm2(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
                 const Work& w);
void tune_lap2(DeviceOp* d, int dtype, hipStream_t s, float* ms_out, bool pair);
void tune_lap3(DeviceOp* d, int dtype, hipStream_t s, float* ms_out, bool pair);
void sweep_pair_lap2(DeviceOp* d, const std::vector<IO>& io, hipStream_t s, const Work& w);
void sweep_pair_lap3(DeviceOp* d, const std::vector<IO>& io, hipStream_t s, const Work& w);
void tune_helm3(DeviceOp* d, int dtype, hipStream_t s, float* ms_out);
void tune_helm2(DeviceOp* d, int dtype, hipStream_t s, float* ms_out);

}  // namespace skelfmm
