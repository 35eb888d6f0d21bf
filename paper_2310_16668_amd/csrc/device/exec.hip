// GPU executor: uploads a layout, owns the workspace, enqueues one sweep.
//
// The adjoint apply is the transposed sweep.  Transposing each forward step in
// reverse order gives: the output scatter becomes a gather of v into the leaf
// entries; the downward pass (uhat += u_parent[slot]; u += [I; T^*] uhat)
// becomes "uhat = [I T] u; parent's entries at the slots += uhat", which has
// exactly the form of the forward upward pass for a real T; every translation
// target <- source becomes source <- target with the conjugate kernel, and
// because colleagues are symmetric and fine neighbors are the inverse of
// coarse ones, the transposed ifs terms have the form of tfo terms and vice
// versa, so the segment lists are reused unchanged; the upward pass becomes a
// top-down pass of the downward form; the gather becomes the output scatter.
// The adjoint therefore runs the forward launches with the kernel conjugated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "device.h"
#include "kernels.hip"

namespace skelfmm {

#define SKF_HIP(x)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            if (e_ == hipErrorOutOfMemory) throw OutOfMemory(std::string(#x) + ": out of memory"); \
            throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_));             \
        }                                                                                   \
    } while (0)

namespace {

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
    void alloc(size_t b) {
        release();
        if (b == 0) b = 16;
        SKF_HIP(hipMalloc(&p, b));
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

int dtype_is_complex(int dt) { return dt == SKELFMM_C128 || dt == SKELFMM_C64; }
int dtype_is_single(int dt) { return dt == SKELFMM_F32 || dt == SKELFMM_C64; }

constexpr int kTPL = 2;              // targets per lane in the near-field kernel
constexpr int kTile = 64 * kTPL;     // targets per near-field work item

}  // namespace

struct DeviceOp {
    Layout L;
    bool f64_leaf = false;
    int device = -1;
    bool uploaded = false;
    // static arrays
    DevMem voff, hoff, toff, nb, kb, is_leaf, level, pmap, perm;
    DevMem gather_e, gather_p, topleaf_e, topleaf_p;
    DevMem X64, X32, T64, T32;
    DevMem seg_ptr, segs, tasks, boxrec;
    // workspace
    int64_t ws_nrhs = 0;
    int ws_dtype = -1;
    DevMem Q, Qh, U, Uh;
    // per-pass timing
    bool timing = false;
    std::vector<std::array<hipEvent_t, SKELFMM_NPASS + 1>> pending;
    double pass_ms[SKELFMM_NPASS] = {0, 0, 0, 0, 0};
    int64_t sweeps = 0;
    ~DeviceOp() {
        for (auto& ev : pending)
            for (auto e : ev) (void)hipEventDestroy(e);
    }
};

struct DeviceBatch {
    std::vector<DeviceOp*> ops;
};

DeviceOp* device_create(const Plan& p, bool keep_transparent, bool f64_leaf) {
    auto d = std::make_unique<DeviceOp>();
    d->L = make_layout(p, keep_transparent, kTile);
    d->f64_leaf = f64_leaf;
    int kmax = 0;
    for (int k : d->L.kb) kmax = std::max(kmax, k);
    if (kmax > 8192) throw NotSupported("skeleton rank above 8192 is not supported by the downward kernel");
    return d.release();
}

static void upload(DeviceOp* d, int dtype) {
    const Layout& L = d->L;
    if (!d->uploaded) {
        SKF_HIP(hipGetDevice(&d->device));
        d->voff.upload(L.voff);
        d->hoff.upload(L.hoff);
        d->toff.upload(L.toff);
        d->nb.upload(L.nb);
        d->kb.upload(L.kb);
        d->is_leaf.upload(L.is_leaf);
        d->level.upload(L.level);
        d->pmap.upload(L.pmap);
        d->perm.upload(L.perm);
        d->gather_e.upload(L.gather_e);
        d->gather_p.upload(L.gather_p);
        d->topleaf_e.upload(L.topleaf_e);
        d->topleaf_p.upload(L.topleaf_p);
        d->seg_ptr.upload(L.seg_ptr);
        std::vector<int2> sg(L.seg_src.size());
        for (size_t i = 0; i < sg.size(); ++i) sg[i] = make_int2(L.seg_src[i], L.seg_mode[i]);
        d->segs.upload(sg);
        d->tasks.upload(L.tasks);
        std::vector<kern::BoxRec> br(L.n_boxes);
        for (int b = 0; b < L.n_boxes; ++b)
            br[b] = kern::BoxRec{L.voff[b], L.hoff[b], L.nb[b], L.kb[b], L.level[b], L.is_leaf[b]};
        d->boxrec.upload(br);
        d->uploaded = true;
    }
    const bool single = dtype_is_single(dtype);
    const bool need64 = !single || d->f64_leaf;
    if (need64 && !d->X64.p) d->X64.upload(L.X);
    if (!need64 && !d->X32.p) {
        std::vector<float> x32(L.X.begin(), L.X.end());
        d->X32.upload(x32);
    }
    if (!single && !d->T64.p) d->T64.upload(L.T);
    if (single && !d->T32.p) {
        std::vector<float> t32(L.T.begin(), L.T.end());
        d->T32.upload(t32);
    }
}

void device_prepare(DeviceOp* d, int64_t nrhs, int dtype) {
    upload(d, dtype);
    const size_t vb = (dtype_is_single(dtype) ? 4 : 8) * (dtype_is_complex(dtype) ? 2 : 1);
    const size_t need_e = static_cast<size_t>(d->L.n_entries) * nrhs * vb;
    const size_t need_h = static_cast<size_t>(d->L.n_hentries) * nrhs * vb;
    if (d->Q.bytes < need_e) { d->Q.alloc(need_e); d->U.alloc(need_e); }
    if (d->Qh.bytes < need_h) { d->Qh.alloc(need_h); d->Uh.alloc(need_h); }
    d->ws_nrhs = std::max(d->ws_nrhs, nrhs);
}

namespace {

kern::BoxArgs box_args(const DeviceOp* d) {
    kern::BoxArgs a;
    a.voff = d->voff.as<int64_t>();
    a.hoff = d->hoff.as<int64_t>();
    a.toff = d->toff.as<int64_t>();
    a.nb = d->nb.as<int32_t>();
    a.kb = d->kb.as<int32_t>();
    a.is_leaf = d->is_leaf.as<int32_t>();
    a.level = d->level.as<int32_t>();
    a.pmap = d->pmap.as<int32_t>();
    a.perm = d->perm.as<int32_t>();
    return a;
}

inline unsigned blocks_for(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

template <class P, bool CONJ>
void launch_near(const DeviceOp* d, hipStream_t s, const void* X, void* Q, void* Qh, void* U, void* Uh) {
    const Layout& L = d->L;
    if (L.tasks.empty()) return;
    using R = typename P::Rt;
    using V = typename P::Vt;
    const int ntasks = static_cast<int>(L.tasks.size());
    hipLaunchKernelGGL((kern::k_near<P, kTPL, CONJ>), dim3(blocks_for(ntasks, 4)), dim3(256), 0, s,
                       d->tasks.as<Task>(), ntasks, L.top, d->seg_ptr.as<int32_t>(), d->segs.as<int2>(),
                       d->boxrec.as<kern::BoxRec>(), static_cast<const kern::Rec4<R>*>(X),
                       static_cast<const V*>(Q), static_cast<const V*>(Qh), static_cast<V*>(U),
                       static_cast<V*>(Uh), static_cast<R>(L.kappa), kern::kInv4Pi);
    SKF_HIP(hipGetLastError());
}

// Events bracketing the passes of one sweep (only when timing is on).
struct PassMarks {
    DeviceOp* d;
    hipStream_t s;
    std::array<hipEvent_t, SKELFMM_NPASS + 1> ev{};
    PassMarks(DeviceOp* d_, hipStream_t s_) : d(d_), s(s_) {
        if (!d->timing) return;
        for (auto& e : ev) SKF_HIP(hipEventCreate(&e));
    }
    void mark(int i) {
        if (d->timing) SKF_HIP(hipEventRecord(ev[i], s));
    }
    void done() {
        if (d->timing) d->pending.push_back(ev);
    }
};

// One sweep for nrhs == 1 with value type V (float or double), transfer-matrix
// type TT, near-field policy P.
template <typename V, typename TT, class P>
void sweep(DeviceOp* d, const V* q, V* u, hipStream_t s, bool adjoint, const TT* T, const void* X) {
    const Layout& L = d->L;
    constexpr int nv = P::nv;
    const int W = nv;
    V* Q = d->Q.as<V>();
    V* Qh = d->Qh.as<V>();
    V* U = d->U.as<V>();
    V* Uh = d->Uh.as<V>();
    const kern::BoxArgs ba = box_args(d);
    const int64_t N = L.n_points;
    PassMarks pm(d, s);
    pm.mark(0);
    hipLaunchKernelGGL((kern::k_gather<V, V>), dim3(blocks_for(N * W, 256)), dim3(256), 0, s,
                       d->gather_e.as<int32_t>(), d->gather_p.as<int32_t>(), N, W, q, Q);
    SKF_HIP(hipGetLastError());
    pm.mark(1);
    for (int l = L.max_level; l > L.top; --l) {
        const int b0 = L.level_ptr[l], nbx = L.level_ptr[l + 1] - b0;
        if (nbx <= 0) continue;
        hipLaunchKernelGGL((kern::k_upward<V, TT>), dim3(nbx), dim3(256), 0, s, ba, b0, W, T, Q, Qh);
        SKF_HIP(hipGetLastError());
    }
    pm.mark(2);
    if (adjoint && P::kind == 1) launch_near<P, true>(d, s, X, Q, Qh, U, Uh);
    else launch_near<P, false>(d, s, X, Q, Qh, U, Uh);
    pm.mark(3);
    int kmax = 0;
    for (int l = L.top + 1; l <= L.max_level; ++l) {
        const int b0 = L.level_ptr[l], nbx = L.level_ptr[l + 1] - b0;
        if (nbx <= 0) continue;
        kmax = 0;
        for (int b = b0; b < b0 + nbx; ++b) kmax = std::max(kmax, L.kb[b]);
        const size_t lds = std::max<size_t>(8, static_cast<size_t>(kmax) * sizeof(double));
        hipLaunchKernelGGL((kern::k_downward<V, TT, V>), dim3(nbx), dim3(256), lds, s, ba, b0, W, T, Uh, U, u);
        SKF_HIP(hipGetLastError());
    }
    pm.mark(4);
    const int64_t ntl = static_cast<int64_t>(L.topleaf_e.size());
    if (ntl > 0) {
        hipLaunchKernelGGL((kern::k_scatter<V, V>), dim3(blocks_for(ntl * W, 256)), dim3(256), 0, s,
                           d->topleaf_e.as<int32_t>(), d->topleaf_p.as<int32_t>(), ntl, W, U, u);
        SKF_HIP(hipGetLastError());
    }
    pm.mark(5);
    pm.done();
}

template <int DIM, int KIND>
void dispatch(DeviceOp* d, const void* q, void* u, int dtype, hipStream_t s, bool adjoint) {
    if (dtype == SKELFMM_F64 || dtype == SKELFMM_C128) {
        using P = kern::Pol<double, double, double, DIM, KIND>;
        sweep<double, double, P>(d, static_cast<const double*>(q), static_cast<double*>(u), s, adjoint,
                                 d->T64.as<double>(), d->X64.p);
    } else if (d->f64_leaf) {
        using P = kern::Pol<double, double, float, DIM, KIND>;
        sweep<float, float, P>(d, static_cast<const float*>(q), static_cast<float*>(u), s, adjoint,
                               d->T32.as<float>(), d->X64.p);
    } else {
        using P = kern::Pol<float, double, float, DIM, KIND>;
        sweep<float, float, P>(d, static_cast<const float*>(q), static_cast<float*>(u), s, adjoint,
                               d->T32.as<float>(), d->X32.p);
    }
}

}  // namespace

void device_apply(DeviceOp* d, const void* q, void* u, int64_t nrhs, int dtype, void* stream, bool adjoint) {
    if (nrhs != 1) throw NotSupported("this build applies one right-hand side per call");
    int dev = -1;
    SKF_HIP(hipGetDevice(&dev));
    if (d->uploaded && dev != d->device) throw std::invalid_argument("operator was prepared on another device");
    device_prepare(d, nrhs, dtype);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout& L = d->L;
    if (L.kind == 1) dispatch<3, 1>(d, q, u, dtype, s, adjoint);
    else if (L.dim == 3) dispatch<3, 0>(d, q, u, dtype, s, adjoint);
    else dispatch<2, 0>(d, q, u, dtype, s, adjoint);
}

void device_fill_stats(const DeviceOp* d, skelfmm_stats* out) {
    out->n_entries = d->L.n_entries;
    out->pairs_near = d->L.pairs_near;
    out->pairs_skel = d->L.pairs_skel;
    out->n_tasks = static_cast<int64_t>(d->L.tasks.size());
    out->tile_targets = d->L.tile;
}

void device_destroy(DeviceOp* d) { delete d; }

void device_timing(DeviceOp* d, bool enable) {
    for (auto& ev : d->pending)
        for (auto e : ev) (void)hipEventDestroy(e);
    d->pending.clear();
    std::fill(d->pass_ms, d->pass_ms + SKELFMM_NPASS, 0.0);
    d->sweeps = 0;
    d->timing = enable;
}

void device_timing_read(DeviceOp* d, double* ms, int64_t* sweeps) {
    for (auto& ev : d->pending) {
        SKF_HIP(hipEventSynchronize(ev[SKELFMM_NPASS]));
        for (int i = 0; i < SKELFMM_NPASS; ++i) {
            float t = 0.f;
            SKF_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
            d->pass_ms[i] += t;
        }
        for (auto e : ev) (void)hipEventDestroy(e);
        d->sweeps += 1;
    }
    d->pending.clear();
    std::copy(d->pass_ms, d->pass_ms + SKELFMM_NPASS, ms);
    *sweeps = d->sweeps;
}

DeviceBatch* batch_create(const std::vector<DeviceOp*>& ops) {
    auto* b = new DeviceBatch();
    b->ops = ops;
    return b;
}

void batch_apply(DeviceBatch* b, const void* const* q, void* const* u, int64_t nrhs, int dtype, void* stream,
                 bool adjoint) {
    for (size_t i = 0; i < b->ops.size(); ++i) device_apply(b->ops[i], q[i], u[i], nrhs, dtype, stream, adjoint);
}

void batch_destroy(DeviceBatch* b) { delete b; }

}  // namespace skelfmm
