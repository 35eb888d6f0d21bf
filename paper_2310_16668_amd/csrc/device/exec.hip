// GPU executor: uploads a layout, owns the workspace, enqueues one sweep.
//
// A sweep is: gather the caller's charges into the leaf entries; upward pass,
// one launch per level (deepest first); one near-field launch over every
// level; downward pass, one launch per level (coarsest first); scatter the
// leaf entries' potentials to the caller's output.  One right-hand side uses
// the single-RHS kernels; several use the kernels with lanes (transfers) or
// registers (near field) over right-hand-side columns.  A batch runs the same
// sweep over one merged layout of several operators, with one gather and one
// scatter per operator.
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

#define SKF_HIP(x)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) {                                                                    \
            if (e_ == hipErrorOutOfMemory) throw OutOfMemory(std::string(#x) + ": out of memory"); \
            throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_));                    \
        }                                                                                          \
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

int dtype_is_complex(int dt) { return dt == SKELFMM_C128 || dt == SKELFMM_C64; }
int dtype_is_single(int dt) { return dt == SKELFMM_F32 || dt == SKELFMM_C64; }

constexpr int kDefaultTPL = 2;   // targets per lane in the single-RHS near-field kernels (1 .. 4)
constexpr int kChunkReals = 8;   // right-hand-side reals per multi-RHS near-field work item

int tpl_slot(int tpl) { return tpl - 1; }

// Several right-hand sides of a real kernel in the float32 policy run the near
// field on the matrix cores (k_near_mfma) from 8 columns on.
constexpr int kMfmaMinRhs = 8;
constexpr int kMfmaCols = 32;     // columns per accumulator tile

// Values per entry inside the workspace: nv for one RHS; several RHS are padded
// to a multiple of the near-field chunk (of the accumulator tile on the matrix
// core path).
int64_t padded_width(int64_t nrhs, int dtype, bool mfma) {
    const int64_t w = nrhs * (dtype_is_complex(dtype) ? 2 : 1);
    if (nrhs == 1) return w;
    const int64_t m = mfma ? kMfmaCols : kChunkReals;
    return (w + m - 1) / m * m;
}

inline unsigned blocks_for(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

}  // namespace

struct DeviceOp {
    Layout L;
    bool f64_leaf = false;
    int device = -1;
    bool uploaded = false;
    // static arrays
    DevMem voff, hoff, toff, ttoff, nb, kb, pmap, gather_e, gather_p;
    DevMem X64, T64, T32, Tt64, Tt32;             // T and its per-box transposes, columns padded
    DevMem seg_ptr, segs, boxrec;
    // one-RHS transfer work: (box, first row) items per level, and waves per item
    DevMem upwork[2], downwork[2];                // [0]: float64 T row groups, [1]: float32
    std::vector<int64_t> up_ptr[2], down_ptr[2];
    std::vector<int> up_nw, down_nw;
    std::vector<int> up_rows, down_rows;          // per level: most output rows of a box (k up, n - k down)
    int tpl = kDefaultTPL;
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
    ~DeviceOp() {
        for (auto& ev : pending)
            for (auto e : ev) (void)hipEventDestroy(e);
    }
};

// The matrix-core near field serves several RHS of a real kernel in the
// float32 policy.
static bool use_mfma(const DeviceOp* d, int64_t nrhs, int dtype) {
    return d->L.kind == 0 && dtype == SKELFMM_F32 && !d->f64_leaf && nrhs >= kMfmaMinRhs;
}

struct DeviceBatch {
    std::vector<DeviceOp*> ops;
    std::unique_ptr<DeviceOp> merged;
    std::vector<int64_t> gbase;                   // first gather-list index of each operator
};

static void check_ranks(const Layout& L) {
    int kmax = 0;
    for (int k : L.kb) kmax = std::max(kmax, k);
    if (kmax > 8192) throw NotSupported("skeleton rank above 8192 is not supported by the downward kernel");
}

// Targets of the lane-side box per symmetric work item (a multiple of 64 x tpl
// for every tpl in 1 .. 4).
constexpr int kSymGroup = 768;

DeviceOp* device_create(const Plan& p, bool keep_transparent, bool f64_leaf, bool symmetric, bool expanded) {
    auto d = std::make_unique<DeviceOp>();
    d->L = make_layout(p, keep_transparent, 64 * kDefaultTPL);
    d->L.allow_expanded = expanded;
    // the pairing needs G(x, y) = G(y, x) with real values
    if (symmetric && p.kind == 0) make_symmetric(d->L, kSymGroup);
    d->f64_leaf = f64_leaf;
    check_ranks(d->L);
    return d.release();
}

// Work items of the one-RHS transfers: upward rows are a box's skeleton entries
// (k, with n - k columns), downward rows its redundant entries (n - k, with k
// columns; at least one item per box, which also updates the skeleton entries).
// Waves per item follow the level's mean column count.
static void build_transfer_work(DeviceOp* d) {
    const Layout& L = d->L;
    d->up_nw.assign(L.max_level + 1, 1);
    d->down_nw.assign(L.max_level + 1, 1);
    d->up_rows.assign(L.max_level + 1, 0);
    d->down_rows.assign(L.max_level + 1, 0);
    for (int l = 0; l <= L.max_level; ++l)
        for (int b = L.level_ptr[l]; b < L.level_ptr[l + 1]; ++b) {
            d->up_rows[l] = std::max(d->up_rows[l], L.kb[b]);
            d->down_rows[l] = std::max(d->down_rows[l], L.nb[b] - L.kb[b]);
        }
    for (int g = 0; g < 2; ++g) {
        // row groups: 64 rows of float64 T, 128 rows of float32 T (one 8-byte load per lane)
        const int G = g == 0 ? kern::RowMap<double>::group : kern::RowMap<float>::group;
        std::vector<int2> up, down;
        d->up_ptr[g].assign(L.max_level + 2, 0);
        d->down_ptr[g].assign(L.max_level + 2, 0);
        for (int l = 0; l <= L.max_level; ++l) {
            d->up_ptr[g][l] = static_cast<int64_t>(up.size());
            d->down_ptr[g][l] = static_cast<int64_t>(down.size());
            double cu = 0, cd = 0;
            int nbk = 0;
            for (int b = L.level_ptr[l]; b < L.level_ptr[l + 1]; ++b) {
                const int k = L.kb[b], m = L.nb[b] - L.kb[b];
                if (k <= 0) continue;
                ++nbk;
                cu += m;
                cd += k;
                for (int r = 0; r * G < k; ++r) up.push_back(make_int2(b, r));
                for (int r = 0; r * G < std::max(m, 1); ++r) down.push_back(make_int2(b, r));
            }
            if (g == 0 && nbk > 0) {
                d->up_nw[l] = std::min(16, std::max(1, static_cast<int>(cu / nbk / 32.0 + 0.5)));
                d->down_nw[l] = std::min(16, std::max(1, static_cast<int>(cd / nbk / 32.0 + 0.5)));
            }
        }
        d->up_ptr[g][L.max_level + 1] = static_cast<int64_t>(up.size());
        d->down_ptr[g][L.max_level + 1] = static_cast<int64_t>(down.size());
        d->upwork[g].upload(up);
        d->downwork[g].upload(down);
    }
}

// T (k x m per box) or its transpose (m x k) with columns padded to pad_ld rows,
// in the precision of the vectors; padding entries are zero.
template <typename TT>
static std::vector<TT> padded_t(const Layout& L, bool transpose) {
    std::vector<TT> out(static_cast<size_t>(transpose ? L.ttpad_size : L.tpad_size), TT(0));
    for (int b = 0; b < L.n_boxes; ++b) {
        const int64_t k = L.kb[b], m = L.nb[b] - L.kb[b];
        if (k <= 0 || m <= 0) continue;
        const double* src = L.T.data() + L.toff[b];
        if (!transpose) {
            const int64_t ld = pad_ld(k);
            TT* dst = out.data() + L.tpad[b];
            for (int64_t j = 0; j < m; ++j)
                for (int64_t i = 0; i < k; ++i) dst[i + j * ld] = static_cast<TT>(src[i + j * k]);
        } else {
            const int64_t ld = pad_ld(m);
            TT* dst = out.data() + L.ttpad[b];
            for (int64_t j = 0; j < m; ++j)
                for (int64_t i = 0; i < k; ++i) dst[j + i * ld] = static_cast<TT>(src[i + j * k]);
        }
    }
    return out;
}

static void upload(DeviceOp* d, int dtype) {
    const Layout& L = d->L;
    if (!d->uploaded) {
        SKF_HIP(hipGetDevice(&d->device));
        d->voff.upload(L.voff);
        d->hoff.upload(L.hoff);
        d->toff.upload(L.tpad);
        d->ttoff.upload(L.ttpad);
        d->nb.upload(L.nb);
        d->kb.upload(L.kb);
        d->pmap.upload(L.pmap);
        d->gather_e.upload(L.gather_e);
        d->gather_p.upload(L.gather_p);
        d->seg_ptr.upload(L.seg_ptr);
        std::vector<int2> sg(L.seg_src.size());
        for (size_t i = 0; i < sg.size(); ++i) sg[i] = make_int2(L.seg_src[i], L.seg_mode[i]);
        d->segs.upload(sg);
        for (int t : {1, 2, 3, 4}) {
            const std::vector<Task> tl = (64 * t == L.tile) ? L.tasks : make_tasks(L, 64 * t);
            d->tasks[tpl_slot(t)].upload(tl);
            d->ntasks[tpl_slot(t)] = static_cast<int>(tl.size());
        }
        {
            // items holding skeleton targets (uhat rows) first; the rest run two
            // column tiles per wave
            std::vector<Task> tl = make_tasks(L, 32);
            std::stable_partition(tl.begin(), tl.end(), [&](const Task& t) { return t.t0 < L.kb[t.box]; });
            d->ntasks32h = static_cast<int>(
                std::count_if(tl.begin(), tl.end(), [&](const Task& t) { return t.t0 < L.kb[t.box]; }));
            d->tasks32.upload(tl);
            d->ntasks32 = static_cast<int>(tl.size());
        }
        if (L.sym) {
            d->seg_ptr_ns.upload(L.seg_ptr_ns);
            std::vector<int2> sn(L.seg_src_ns.size());
            for (size_t i = 0; i < sn.size(); ++i) sn[i] = make_int2(L.seg_src_ns[i], L.seg_mode_ns[i]);
            d->segs_ns.upload(sn);
            d->symtasks.upload(L.sym_tasks);
            d->nsym = static_cast<int>(L.sym_tasks.size());
            for (int t : {1, 2, 3, 4}) {
                const std::vector<Task> tl = make_tasks(L, 64 * t, true);
                d->tasks_ns[tpl_slot(t)].upload(tl);
                d->ntasks_ns[tpl_slot(t)] = static_cast<int>(tl.size());
            }
            d->symrows.upload(L.sym_rows);
            d->nred = static_cast<int>(L.sym_rows.size());
            d->slots.alloc(static_cast<size_t>(L.slot_size) * sizeof(double));
        }
        std::vector<kern::BoxRec> br(L.n_boxes);
        for (int b = 0; b < L.n_boxes; ++b)
            br[b] = kern::BoxRec{L.voff[b], L.hoff[b], L.nb[b], L.kb[b], L.level[b], L.is_leaf[b]};
        d->boxrec.upload(br);
        d->X64.upload(L.X);   // coordinates are float64 in every precision policy
        build_transfer_work(d);
        d->uploaded = true;
    }
    const bool single = dtype_is_single(dtype);
    if (!single && !d->T64.p) d->T64.upload(padded_t<double>(L, false));
    if (single && !d->T32.p) d->T32.upload(padded_t<float>(L, false));
}

static void upload_transposes(DeviceOp* d, bool single) {
    if ((single && d->Tt32.p) || (!single && d->Tt64.p)) return;
    if (single) d->Tt32.upload(padded_t<float>(d->L, true));
    else d->Tt64.upload(padded_t<double>(d->L, true));
}

void device_prepare(DeviceOp* d, int64_t nrhs, int dtype) {
    upload(d, dtype);
    upload_transposes(d, dtype_is_single(dtype));
    const size_t vb = dtype_is_single(dtype) ? 4 : 8;
    const size_t wp = static_cast<size_t>(padded_width(nrhs, dtype, use_mfma(d, nrhs, dtype)));
    const size_t need_e = static_cast<size_t>(d->L.n_entries) * wp * vb;
    const size_t need_h = static_cast<size_t>(d->L.n_hentries) * wp * vb;
    if (d->Q.bytes < need_e) { d->Q.alloc(need_e); d->U.alloc(need_e); }
    if (d->Qh.bytes < need_h) { d->Qh.alloc(need_h); d->Uh.alloc(need_h); }
}

namespace {

// The caller's buffers of one operator and its range of leaf entries.
struct IO {
    const void* q;
    void* u;
    int64_t g0;     // first index into the gather lists
    int64_t cnt;    // number of points
};

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

// The one-RHS near field: k_near over the segment lists; with symmetric pairing
// it covers what is left after pairing, then k_near_sym evaluates the pairs
// into slots and k_sym_reduce adds the slots to u and uhat.
template <class P, int TPL, bool CONJ>
void launch_near_t(const DeviceOp* d, hipStream_t s, void* Q, void* Qh, void* U, void* Uh, PassMarks* pm) {
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
                           static_cast<R>(d->L.kappa), kern::kInv4Pi);
        SKF_HIP(hipGetLastError());
    }
    if (pm) pm->mark(3);
    if constexpr (P::kind == 0) {
        if (sym && d->nsym > 0) {
            hipLaunchKernelGGL((kern::k_near_sym<P, TPL>), dim3(blocks_for(d->nsym, 4)), dim3(256), 0, s,
                               d->symtasks.as<SymTask>(), d->nsym, d->boxrec.as<kern::BoxRec>(),
                               d->X64.as<kern::Rec4<double>>(), static_cast<const V*>(Q), static_cast<const V*>(Qh),
                               d->slots.as<double>(), kern::kInv4Pi);
            SKF_HIP(hipGetLastError());
        }
    }
    if (pm) pm->mark(4);
    if constexpr (P::kind == 0) {
        if (sym && d->nred > 0) {
            hipLaunchKernelGGL((kern::k_sym_reduce<V>), dim3(d->nred), dim3(256), 0, s, d->symrows.as<SymRows>(),
                               d->boxrec.as<kern::BoxRec>(), d->slots.as<double>(), static_cast<V*>(U),
                               static_cast<V*>(Uh));
            SKF_HIP(hipGetLastError());
        }
    }
}

template <class P, bool CONJ>
void launch_near(const DeviceOp* d, hipStream_t s, void* Q, void* Qh, void* U, void* Uh, PassMarks* pm = nullptr) {
    if (d->tpl == 1) launch_near_t<P, 1, CONJ>(d, s, Q, Qh, U, Uh, pm);
    else if (d->tpl == 3) launch_near_t<P, 3, CONJ>(d, s, Q, Qh, U, Uh, pm);
    else if (d->tpl == 4) launch_near_t<P, 4, CONJ>(d, s, Q, Qh, U, Uh, pm);
    else launch_near_t<P, 2, CONJ>(d, s, Q, Qh, U, Uh, pm);
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
                       static_cast<R>(d->L.kappa), kern::kInv4Pi);
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
                               Qhf, Uf, Uhf, kern::kInv4Pi);
        SKF_HIP(hipGetLastError());
        return;
    }
    if (nh > 0)
        hipLaunchKernelGGL((kern::k_near_mfma2<P, true>), dim3(blocks_for(int64_t(nh) * npairs, 4)), dim3(256), 0,
                           s, tl, nh, npairs, Wp, d->seg_ptr.as<int32_t>(), d->segs.as<int2>(),
                           d->boxrec.as<kern::BoxRec>(), X, Qf, Qhf, Uf, Uhf, kern::kInv4Pi);
    if (nn > 0)
        hipLaunchKernelGGL((kern::k_near_mfma2<P, false>), dim3(blocks_for(int64_t(nn) * npairs, 4)), dim3(256), 0,
                           s, tl + nh, nn, npairs, Wp, d->seg_ptr.as<int32_t>(), d->segs.as<int2>(),
                           d->boxrec.as<kern::BoxRec>(), X, Qf, Qhf, Uf, Uhf, kern::kInv4Pi);
    SKF_HIP(hipGetLastError());
}

// One sweep.  V: stored values; TT: transfer matrices; P: near-field policy;
// Am: accumulator of one source box's partial sums in the multi-RHS near field.
template <typename V, typename TT, class P, typename Am>
void sweep(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
           const TT* T, const TT* Tt) {
    const Layout& L = d->L;
    const bool multi = nrhs > 1;
    const int Win = static_cast<int>(nrhs * P::nv);
    const bool mfma = use_mfma(d, nrhs, dtype);
    const int Wp = static_cast<int>(padded_width(nrhs, dtype, mfma));
    V* Q = d->Q.as<V>();
    V* Qh = d->Qh.as<V>();
    V* U = d->U.as<V>();
    V* Uh = d->Uh.as<V>();
    const kern::BoxRec* br = d->boxrec.as<kern::BoxRec>();
    const int64_t* toff = d->toff.as<int64_t>();
    const int64_t* ttoff = d->ttoff.as<int64_t>();
    const int32_t* pmap = d->pmap.as<int32_t>();
    const int32_t* ge = d->gather_e.as<int32_t>();
    const int32_t* gp = d->gather_p.as<int32_t>();
    PassMarks pm(d, s);
    pm.mark(0);
    for (const IO& x : io) {
        if (x.cnt <= 0) continue;
        hipLaunchKernelGGL((kern::k_gather_pad<V, V>), dim3(blocks_for(x.cnt * Wp, 256)), dim3(256), 0, s,
                           ge + x.g0, gp + x.g0, x.cnt, Win, Wp, static_cast<const V*>(x.q), Q);
        SKF_HIP(hipGetLastError());
    }
    pm.mark(1);
    for (int l = L.max_level; l >= 2; --l) {
        const int b0 = L.level_ptr[l], nbx = L.level_ptr[l + 1] - b0;
        if (nbx <= 0) continue;
        if (multi) {
            // row chunks of a box spread over the grid's second dimension (4 per block)
            const int gy = std::max(1, (d->up_rows[l] + 4 * kern::kRB - 1) / (4 * kern::kRB));
            hipLaunchKernelGGL((kern::k_upward_mr<V, TT>), dim3(nbx, gy), dim3(256), 0, s, br, toff, pmap, b0, Wp,
                               T, Q, Qh);
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
        if (adjoint && P::kind == 1) launch_near<P, true>(d, s, Q, Qh, U, Uh, &pm);
        else launch_near<P, false>(d, s, Q, Qh, U, Uh, &pm);
    }
    pm.mark(5);
    for (int l = 2; l <= L.max_level; ++l) {
        const int b0 = L.level_ptr[l], nbx = L.level_ptr[l + 1] - b0;
        if (nbx <= 0) continue;
        if (multi) {
            const int gy = std::max(1, (d->down_rows[l] + 4 * kern::kRB - 1) / (4 * kern::kRB));
            hipLaunchKernelGGL((kern::k_downward_mr<V, TT>), dim3(nbx, gy), dim3(256), 0, s, br, ttoff, pmap, b0, Wp,
                               Tt, Uh, U);
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
        hipLaunchKernelGGL((kern::k_scatter_pad<V, V>), dim3(blocks_for(x.cnt * Win, 256)), dim3(256), 0, s,
                           ge + x.g0, gp + x.g0, x.cnt, Win, Wp, U, static_cast<V*>(x.u));
        SKF_HIP(hipGetLastError());
    }
    pm.mark(7);
    pm.done();
}

template <int DIM, int KIND>
void dispatch(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint) {
    if (dtype == SKELFMM_F64 || dtype == SKELFMM_C128) {
        using P = kern::Pol<double, double, double, DIM, KIND>;
        sweep<double, double, P, double>(d, io, nrhs, dtype, s, adjoint, d->T64.as<double>(), d->Tt64.as<double>());
    } else if (d->f64_leaf) {
        using P = kern::Pol<double, double, float, DIM, KIND>;
        sweep<float, float, P, double>(d, io, nrhs, dtype, s, adjoint, d->T32.as<float>(), d->Tt32.as<float>());
    } else {
        using P = kern::Pol<float, double, float, DIM, KIND>;
        sweep<float, float, P, float>(d, io, nrhs, dtype, s, adjoint, d->T32.as<float>(), d->Tt32.as<float>());
    }
}

void run(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, void* stream, bool adjoint) {
    if (nrhs > (int64_t(1) << 20)) throw std::invalid_argument("nrhs too large");
    int dev = -1;
    SKF_HIP(hipGetDevice(&dev));
    if (d->uploaded && dev != d->device) throw std::invalid_argument("operator was prepared on another device");
    device_prepare(d, nrhs, dtype);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout& L = d->L;
    if (L.kind == 1) dispatch<3, 1>(d, io, nrhs, dtype, s, adjoint);
    else if (L.dim == 3) dispatch<3, 0>(d, io, nrhs, dtype, s, adjoint);
    else dispatch<2, 0>(d, io, nrhs, dtype, s, adjoint);
}

}  // namespace

void device_apply(DeviceOp* d, const void* q, void* u, int64_t nrhs, int dtype, void* stream, bool adjoint) {
    run(d, {IO{q, u, 0, d->L.n_points}}, nrhs, dtype, stream, adjoint);
}

// Time the near-field launches for 1 .. 4 targets per lane on this operator
// (workspace contents are whatever the last apply left; timing does not depend
// on values) and keep the fastest.
template <int DIM, int KIND>
static void tune_near(DeviceOp* d, int dtype, hipStream_t s, float* ms_out) {
    const bool single = dtype_is_single(dtype);
    for (int t : {1, 2, 3, 4}) {
        d->tpl = t;
        hipEvent_t a, b;
        SKF_HIP(hipEventCreate(&a));
        SKF_HIP(hipEventCreate(&b));
        for (int rep = 0; rep < 4; ++rep) {
            if (rep == 1) SKF_HIP(hipEventRecord(a, s));
            if (!single) {
                using P = kern::Pol<double, double, double, DIM, KIND>;
                launch_near<P, false>(d, s, d->Q.p, d->Qh.p, d->U.p, d->Uh.p);
            } else if (d->f64_leaf) {
                using P = kern::Pol<double, double, float, DIM, KIND>;
                launch_near<P, false>(d, s, d->Q.p, d->Qh.p, d->U.p, d->Uh.p);
            } else {
                using P = kern::Pol<float, double, float, DIM, KIND>;
                launch_near<P, false>(d, s, d->Q.p, d->Qh.p, d->U.p, d->Uh.p);
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
    d->tpl = best;
}

int device_autotune(DeviceOp* d, int dtype, void* stream, float* ms_out) {
    device_prepare(d, 1, dtype);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout& L = d->L;
    if (L.kind == 1) tune_near<3, 1>(d, dtype, s, ms_out);
    else if (L.dim == 3) tune_near<3, 0>(d, dtype, s, ms_out);
    else tune_near<2, 0>(d, dtype, s, ms_out);
    return d->tpl;
}

void device_set_tpl(DeviceOp* d, int tpl) {
    if (tpl < 1 || tpl > SKELFMM_NTPL) throw std::invalid_argument("targets per lane must be 1 .. 4");
    d->tpl = tpl;
}

void device_fill_stats(const DeviceOp* d, skelfmm_stats* out) {
    out->n_entries = d->L.n_entries;
    out->pairs_near = d->L.pairs_near;
    out->pairs_skel = d->L.pairs_skel;
    out->n_tasks = d->uploaded ? (d->L.sym ? d->ntasks_ns : d->ntasks)[tpl_slot(d->tpl)]
                               : static_cast<int64_t>(d->L.tasks.size());
    out->tile_targets = 64 * d->tpl;
    out->n_sym_tasks = static_cast<int32_t>(d->L.sym_tasks.size());
    int64_t pc[4];
    sym_pair_counts(d->L, d->tpl, pc);
    out->pairs_sym = pc[0];
    out->pairs_sym_skel = pc[1];
    out->pairs_tile = pc[2];
    out->pairs_tile_skel = pc[3];
    out->n_sym_expanded = 0;
    for (const SymTask& st : d->L.sym_tasks) out->n_sym_expanded += (st.flags & SYM_EXPANDED) ? 1 : 0;
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
    auto b = std::make_unique<DeviceBatch>();
    b->ops = ops;
    std::vector<const Layout*> ls;
    for (auto* o : ops) {
        ls.push_back(&o->L);
        if (o->f64_leaf != ops[0]->f64_leaf) throw std::invalid_argument("batched operators must share f64_leaf");
    }
    std::vector<int64_t> ebase;
    b->merged = std::make_unique<DeviceOp>();
    b->merged->L = merge_layouts(ls, ebase);
    for (auto* o : ops)
        if (o->L.sym != ops[0]->L.sym || o->L.allow_expanded != ops[0]->L.allow_expanded)
            throw std::invalid_argument("batched operators must share the pairing options");
    b->merged->L.allow_expanded = ops[0]->L.allow_expanded;
    if (ops[0]->L.sym) make_symmetric(b->merged->L, kSymGroup);
    b->merged->f64_leaf = ops[0]->f64_leaf;
    check_ranks(b->merged->L);
    b->gbase.assign(ops.size() + 1, 0);
    for (size_t i = 0; i < ops.size(); ++i) b->gbase[i + 1] = b->gbase[i] + ops[i]->L.n_points;
    return b.release();
}

void batch_apply(DeviceBatch* b, const void* const* q, void* const* u, int64_t nrhs, int dtype, void* stream,
                 bool adjoint) {
    std::vector<IO> io;
    for (size_t i = 0; i < b->ops.size(); ++i) {
        if (!q[i] || !u[i]) throw std::invalid_argument("NULL vector in batch");
        if (q[i] == u[i]) throw std::invalid_argument("input and output must not alias");
        io.push_back(IO{q[i], u[i], b->gbase[i], b->gbase[i + 1] - b->gbase[i]});
    }
    run(b->merged.get(), io, nrhs, dtype, stream, adjoint);
}

void batch_destroy(DeviceBatch* b) { delete b; }

}  // namespace skelfmm
