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
#include <cmath>
#include <mutex>
#include <stdexcept>

#include "sweep.h"

// Workspace of skelfmm_apply_noalloc (see device_apply_noalloc): one copy per
// device, held until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace skelfmm {

static void check_ranks(const Layout& L) {
    int kmax = 0;
    for (int k : L.kb) kmax = std::max(kmax, k);
    if (kmax > 8192) throw NotSupported("skeleton rank above 8192 is not supported by the downward kernel");
}

// Targets of the lane-side box per symmetric work item (a multiple of 64 x tpl
// for every tpl in 1 .. 4).
constexpr int kSymGroup = 768;

DeviceOp* device_create(const Plan& p, bool keep_transparent, bool f64_leaf, bool symmetric, bool expanded, bool f32diff,
                        bool compensated) {
    auto d = std::make_unique<DeviceOp>();
    d->L = make_layout(p, keep_transparent, 64 * kDefaultTPL);
    d->L.allow_expanded = expanded;
    d->L.allow_f32diff = f32diff;
    // the pairing needs G(x, y) = G(y, x): the real Laplace kernels, and the
    // complex-symmetric Helmholtz kernels (distinct boxes only)
    if (symmetric) make_symmetric(d->L, kSymGroup, p.kind == 0);
    d->f64_leaf = f64_leaf;
    d->compensated = compensated;
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
    for (int g = 0; g < 4; ++g) {
        // row groups: 64 rows of float64 T, 128 rows of float32 T (one 8-byte load
        // per lane); blocks of 64 / 128 rows of the matrix-core transfers
        const int G = g == 0 ? kern::RowMap<double>::group
                             : (g == 1 ? kern::RowMap<float>::group : kern::kXferRowsPerWave * (g == 2 ? 2 : 4));
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
                for (int r = 0; r * G < k; ++r) up.push_back(make_int2(b, r * (g >= 2 ? G : 1)));
                for (int r = 0; r * G < std::max(m, 1); ++r) down.push_back(make_int2(b, r * (g >= 2 ? G : 1)));
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
    // levels whose boxes are all uncompressed (k = n, no T) with entries and
    // skeleton entries laid out alike: the transfers are elementwise there
    d->flat.assign(L.max_level + 1, FlatLevel{});
    for (int l = 2; l <= L.max_level; ++l) {
        const int b0 = L.level_ptr[l], b1 = L.level_ptr[l + 1];
        if (b1 <= b0) continue;
        bool ok = true;
        int64_t e = L.voff[b0], h = L.hoff[b0];
        for (int b = b0; b < b1 && ok; ++b) {
            ok = L.kb[b] == L.nb[b] && L.voff[b] == e && L.hoff[b] == h;
            e += L.nb[b];
            h += L.kb[b];
        }
        if (ok && e > L.voff[b0]) d->flat[l] = FlatLevel{L.voff[b0], L.hoff[b0], e - L.voff[b0]};
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
        const double* src = L.Tvec().data() + L.toff[b];
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

// Where the pair kernel's expanded source records of each box start: the
// boxes in entry order, each followed by kSymRecordPad extra records.
static std::vector<int64_t> record_offsets(const Layout& L) {
    std::vector<int> order(L.n_boxes);
    for (int b = 0; b < L.n_boxes; ++b) order[b] = b;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return L.voff[a] < L.voff[b]; });
    std::vector<int64_t> roff(L.n_boxes);
    for (int r = 0; r < L.n_boxes; ++r) roff[order[r]] = L.voff[order[r]] + static_cast<int64_t>(kSymRecordPad) * r;
    return roff;
}

// The pair kernel's expanded source records: for an entry x of box b with
// origin o = the first entry of b, (-2 (x - o), |x - o|^2), so that
// |t - x|^2 = |t - o|^2 + |x - o|^2 - 2 (t - o).(x - o) costs one add and three
// multiply-adds per pair.  Box b's records start at roff[b] and are followed by
// kSymRecordPad copies of its last record: a real source position, so every
// kernel value a block forms is finite, and the kernel gives these positions
// zero charges.
static std::vector<double> expanded_records(const Layout& L, const std::vector<int64_t>& roff) {
    const size_t total = static_cast<size_t>(L.n_entries) + static_cast<size_t>(kSymRecordPad) * L.n_boxes;
    std::vector<double> E(total * 4, 0.0);
    for (int b = 0; b < L.n_boxes; ++b) {
        if (L.nb[b] == 0) continue;
        const double* o = &L.X[static_cast<size_t>(L.voff[b]) * 4];
        for (int64_t e = 0; e < L.nb[b] + kSymRecordPad; ++e) {
            const int64_t src = std::min<int64_t>(e, L.nb[b] - 1);
            const double* x = &L.X[static_cast<size_t>(L.voff[b] + src) * 4];
            double* r = &E[static_cast<size_t>(roff[b] + e) * 4];
            const double dx = x[0] - o[0], dy = x[1] - o[1], dz = x[2] - o[2];
            r[0] = -2.0 * dx;
            r[1] = -2.0 * dy;
            r[2] = -2.0 * dz;
            r[3] = std::fma(dx, dx, std::fma(dy, dy, dz * dz));
        }
    }
    return E;
}

// The float32 coordinates of every entry relative to its box's first entry
// (laid out and padded like the expanded records).
static std::vector<float> relative_records(const Layout& L, const std::vector<int64_t>& roff) {
    const size_t total = static_cast<size_t>(L.n_entries) + static_cast<size_t>(kSymRecordPad) * L.n_boxes;
    std::vector<float> F(total * 4, 0.0f);
    for (int b = 0; b < L.n_boxes; ++b) {
        if (L.nb[b] == 0) continue;
        const double* o = &L.X[static_cast<size_t>(L.voff[b]) * 4];
        for (int64_t e = 0; e < L.nb[b] + kSymRecordPad; ++e) {
            const int64_t src = std::min<int64_t>(e, L.nb[b] - 1);
            const double* x = &L.X[static_cast<size_t>(L.voff[b] + src) * 4];
            float* r = &F[static_cast<size_t>(roff[b] + e) * 4];
            for (int c = 0; c < 3; ++c) r[c] = static_cast<float>(x[c] - o[c]);
        }
    }
    return F;
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
        }
        const std::vector<int64_t> roff = record_offsets(L);
        std::vector<kern::BoxRec> br(L.n_boxes);
        for (int b = 0; b < L.n_boxes; ++b) br[b] = kern::BoxRec{L.voff[b], L.hoff[b], L.nb[b], L.kb[b], roff[b]};
        d->boxrec.upload(br);
        d->X64.upload(L.X);   // coordinates are float64 in every precision policy
        d->XE64.upload(expanded_records(L, roff));
        if (L.allow_f32diff) d->XF32.upload(relative_records(L, roff));
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

// Bytes of the workspace one sweep of nrhs columns of dtype needs: entry
// vectors q and u, skeleton vectors qhat and uhat, the pair kernel's slots.
struct WorkBytes {
    size_t e, h, slots;
};
static WorkBytes work_bytes(const DeviceOp* d, int64_t nrhs, int dtype) {
    const size_t vb = dtype_is_single(dtype) ? 4 : 8;
    const size_t wp = static_cast<size_t>(padded_width(nrhs, dtype, use_mfma(d, nrhs, dtype)));
    return WorkBytes{static_cast<size_t>(d->L.n_entries) * wp * vb, static_cast<size_t>(d->L.n_hentries) * wp * vb,
                     d->L.sym ? static_cast<size_t>(d->L.slot_size) * sizeof(double) * (d->L.kind == 1 ? 2 : 1) : 0};
}

// Uploads the operator for dtype; nrhs >= 1 also sizes its own workspace.
void device_prepare(DeviceOp* d, int64_t nrhs, int dtype) {
    upload(d, dtype);
    upload_transposes(d, dtype_is_single(dtype));
    if (nrhs < 1) return;
    const WorkBytes wb = work_bytes(d, nrhs, dtype);
    if (d->Q.bytes < wb.e || !d->Q.p) { d->Q.alloc(wb.e); d->U.alloc(wb.e); }
    if (d->Qh.bytes < wb.h || !d->Qh.p) { d->Qh.alloc(wb.h); d->Uh.alloc(wb.h); }
    if (!d->slots.p) d->slots.alloc(wb.slots);
}

namespace {

void sweep_any(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
               const Work& w) {
    const Layout& L = d->L;
    if (L.kind == 1 && L.dim == 2) sweep_helm2(d, io, nrhs, dtype, s, adjoint, w);
    else if (L.kind == 1) sweep_helm3(d, io, nrhs, dtype, s, adjoint, w);
    else if (L.dim == 3) sweep_lap3(d, io, nrhs, dtype, s, adjoint, w);
    else sweep_lap2(d, io, nrhs, dtype, s, adjoint, w);
}

void run(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, void* stream, bool adjoint) {
    if (nrhs > (int64_t(1) << 20)) throw std::invalid_argument("nrhs too large");
    int dev = -1;
    SKF_HIP(hipGetDevice(&dev));
    if (d->uploaded && dev != d->device) throw std::invalid_argument("operator was prepared on another device");
    device_prepare(d, nrhs, dtype);
    hipStream_t s = static_cast<hipStream_t>(stream);
    sweep_any(d, io, nrhs, dtype, s, adjoint, d->own_work());
}

}  // namespace

void device_apply(DeviceOp* d, const void* q, void* u, int64_t nrhs, int dtype, void* stream, bool adjoint) {
    run(d, {IO{q, u, 0, d->L.n_points}}, nrhs, dtype, stream, adjoint);
}

// The forward + adjoint sweep of a real kernel in float32 (two interleaved
// columns): whether this operator and dtype take it.
static bool pair_sweep(const DeviceOp* d, int dtype) {
    return d->L.kind == 0 && dtype == SKELFMM_F32 && !d->f64_leaf;
}

// Its workspace: two values per entry and per skeleton entry, two per slot.
static void prepare_pair(DeviceOp* d) {
    device_prepare(d, 1, SKELFMM_F32);
    const size_t e = static_cast<size_t>(d->L.n_entries) * 2 * sizeof(float);
    const size_t h = static_cast<size_t>(d->L.n_hentries) * 2 * sizeof(float);
    const size_t sl = d->L.sym ? static_cast<size_t>(d->L.slot_size) * 2 * sizeof(double) : 0;
    if (d->Q.bytes < e) { d->Q.alloc(e); d->U.alloc(e); }
    if (d->Qh.bytes < h) { d->Qh.alloc(h); d->Uh.alloc(h); }
    if (d->slots.bytes < sl) d->slots.alloc(sl);
}

void device_apply_fwd_adj(DeviceOp* d, const void* q, const void* v, void* u, void* w, int dtype, void* stream) {
    if (!pair_sweep(d, dtype)) {
        // complex kernels, float64 and float64 leaf sums: the two sweeps in turn
        run(d, {IO{q, u, 0, d->L.n_points}}, 1, dtype, stream, false);
        run(d, {IO{v, w, 0, d->L.n_points}}, 1, dtype, stream, true);
        return;
    }
    int dev = -1;
    SKF_HIP(hipGetDevice(&dev));
    if (d->uploaded && dev != d->device) throw std::invalid_argument("operator was prepared on another device");
    prepare_pair(d);
    IO io{q, u, 0, d->L.n_points};
    io.q2 = v;
    io.u2 = w;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (d->L.dim == 3) sweep_pair_lap3(d, {io}, s, d->own_work());
    else sweep_pair_lap2(d, {io}, s, d->own_work());
}

int device_autotune_fwd_adj(DeviceOp* d, void* stream, float* ms_out) {
    if (!pair_sweep(d, SKELFMM_F32))
        throw NotSupported("the forward + adjoint sweep serves real kernels in float32");
    prepare_pair(d);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (d->L.dim == 3) tune_lap3(d, SKELFMM_F32, s, ms_out, true);
    else tune_lap2(d, SKELFMM_F32, s, ms_out, true);
    return d->tpl2;
}

// ---------------------------------------------------------------------------
// apply without allocation: the workspace lives in a static device array
// ---------------------------------------------------------------------------
// For callers that cannot allocate device memory while they apply (code under
// graph capture, serving loops).  Every sweep writes each workspace entry
// before it reads it, so the array needs no clearing between calls; it keeps
// the last call's contents, and calls that overlap on one device race on it.
namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // device address of `scratch`, per device

// The device address of the array on the current device, looked up once per
// device (the array's host-side name is not a device address).
void* scratch_on(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (static_cast<int>(g_scratch_ptr.size()) <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        SKF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

constexpr size_t kSpare = 256;   // as DevMem: merged wave-uniform loads at an array's end stay inside
size_t round_up(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

size_t device_scratch_bytes() { return kScratchBytes; }

void device_apply_noalloc(DeviceOp* d, const void* q, void* u, int64_t nrhs, int dtype, void* stream,
                          bool adjoint) {
    if (nrhs > (int64_t(1) << 20)) throw std::invalid_argument("nrhs too large");
    const bool single = dtype_is_single(dtype);
    if (!d->uploaded || (single ? !d->T32.p || !d->Tt32.p : !d->T64.p || !d->Tt64.p))
        throw std::invalid_argument("operator not uploaded for this dtype: call skelfmm_prepare (nrhs_max = 0 "
                                    "uploads it without a workspace) before skelfmm_apply_noalloc");
    int dev = -1;
    SKF_HIP(hipGetDevice(&dev));
    if (dev != d->device) throw std::invalid_argument("operator was prepared on another device");
    const WorkBytes wb = work_bytes(d, nrhs, dtype);
    const size_t oe = round_up(wb.e + kSpare), oh = round_up(wb.h + kSpare);
    const size_t need = 2 * oe + 2 * oh + round_up(wb.slots + kSpare);
    if (need > kScratchBytes)
        throw std::invalid_argument("this apply needs " + std::to_string(need) + " bytes of workspace; the static " +
                                    "scratch array holds " + std::to_string(kScratchBytes));
    unsigned char* base = static_cast<unsigned char*>(scratch_on(dev));
    // no per-pass events either: this path creates nothing
    const Work w{base, base + 2 * oe, base + oe, base + 2 * oe + oh,
                 reinterpret_cast<double*>(base + 2 * oe + 2 * oh), false};
    sweep_any(d, {IO{q, u, 0, d->L.n_points}}, nrhs, dtype, static_cast<hipStream_t>(stream), adjoint, w);
}

int device_autotune(DeviceOp* d, int dtype, void* stream, float* ms_out) {
    device_prepare(d, 1, dtype);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout& L = d->L;
    if (L.kind == 1 && L.dim == 2) tune_helm2(d, dtype, s, ms_out);
    else if (L.kind == 1) tune_helm3(d, dtype, s, ms_out);
    else if (L.dim == 3) tune_lap3(d, dtype, s, ms_out, false);
    else tune_lap2(d, dtype, s, ms_out, false);
    return d->tpl;
}

// Time the matrix-core transfers (every level, upward then downward) in each
// launch shape on this operator's workspace and keep the fastest.  Values do
// not matter for the timing, and no shape changes the results.
int device_autotune_xfer(DeviceOp* d, int64_t nrhs, void* stream, float* ms_out) {
    if (!use_mfma(d, nrhs, SKELFMM_F32))
        throw NotSupported("the matrix-core transfers serve float32 Laplace applies with at least 8 right-hand sides");
    device_prepare(d, nrhs, SKELFMM_F32);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout& L = d->L;
    const int Wp = static_cast<int>(padded_width(nrhs, SKELFMM_F32, true));
    const float* T = d->T32.as<float>();
    const float* Tt = d->Tt32.as<float>();
    float* Q = d->Q.as<float>();
    float* Qh = d->Qh.as<float>();
    float* U = d->U.as<float>();
    float* Uh = d->Uh.as<float>();
    hipEvent_t a, b;
    SKF_HIP(hipEventCreate(&a));
    SKF_HIP(hipEventCreate(&b));
    for (int c = 0; c < SKELFMM_NXFER; ++c) {
        d->xfer = c;
        for (int rep = 0; rep < 4; ++rep) {
            if (rep == 1) SKF_HIP(hipEventRecord(a, s));
            for (int l = L.max_level; l >= 2; --l) xfer_level(d, s, true, l, Wp, T, Q, Qh, Tt, Uh, U);
            for (int l = 2; l <= L.max_level; ++l) xfer_level(d, s, false, l, Wp, T, Q, Qh, Tt, Uh, U);
        }
        SKF_HIP(hipEventRecord(b, s));
        SKF_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        SKF_HIP(hipEventElapsedTime(&ms, a, b));
        ms_out[c] = ms / 3.0f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    int best = 0;
    for (int c = 1; c < SKELFMM_NXFER; ++c)
        if (ms_out[c] < ms_out[best]) best = c;
    d->xfer = best;
    return best;
}

void device_set_xfer(DeviceOp* d, int shape) {
    if (shape < 0 || shape >= SKELFMM_NXFER) throw std::invalid_argument("transfer launch shape out of range");
    d->xfer = shape;
}

DeviceOp* batch_merged(DeviceBatch* b) { return b->merged.get(); }

int batch_autotune_xfer(DeviceBatch* b, int64_t nrhs, void* stream, float* ms_out) {
    return device_autotune_xfer(b->merged.get(), nrhs, stream, ms_out);
}

void device_set_tpl(DeviceOp* d, int tpl) {
    if (tpl < 1 || tpl > SKELFMM_NTPL) throw std::invalid_argument("targets per lane must be 1 .. 4");
    d->tpl = tpl;
    d->tpl2 = tpl;
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
    out->n_sym_f32diff = 0;
    for (const SymTask& st : d->L.sym_tasks) {
        out->n_sym_expanded += (st.flags & SYM_EXPANDED) ? 1 : 0;
        out->n_sym_f32diff += (st.flags & SYM_F32DIFF) ? 1 : 0;
    }
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
        if (o->L.sym != ops[0]->L.sym || o->L.allow_expanded != ops[0]->L.allow_expanded ||
            o->L.allow_f32diff != ops[0]->L.allow_f32diff)
            throw std::invalid_argument("batched operators must share the pairing options");
    b->merged->L.allow_expanded = ops[0]->L.allow_expanded;
    b->merged->L.allow_f32diff = ops[0]->L.allow_f32diff;
    if (ops[0]->L.sym) make_symmetric(b->merged->L, kSymGroup, b->merged->L.kind == 0);
    b->merged->f64_leaf = ops[0]->f64_leaf;
    for (auto* o : ops)
        if (o->compensated != ops[0]->compensated)
            throw std::invalid_argument("batched operators must share compensated_leaf");
    b->merged->compensated = ops[0]->compensated;
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

