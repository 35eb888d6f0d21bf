// C ABI of the library: argument checks, error reporting, ownership.
// Every entry point catches all C++ exceptions and turns them into a status
// code plus a thread-local message.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>

#include "../../include/skelfmm.h"
#include "device/device.h"
#include "host/plan.h"

namespace {
thread_local std::string g_err;

skelfmm_status fail(skelfmm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

constexpr uint64_t kMagic = 0x736b656c666d6d31ULL;   // "skelfmm1"
constexpr uint64_t kDead = 0xdeaddeaddeaddeadULL;
}  // namespace

struct skelfmm_op {
    uint64_t magic = kMagic;
    skelfmm::Plan plan;
    skelfmm::DeviceOp* dev = nullptr;
    skelfmm_options opt{};
};

struct skelfmm_batch {
    uint64_t magic = kMagic;
    skelfmm::DeviceBatch* dev = nullptr;
    int kind = 0;
};

namespace {

bool alive(const skelfmm_op* op) { return op && op->magic == kMagic; }

template <class F>
skelfmm_status guarded(F&& f) {
    try {
        return f();
    } catch (const skelfmm::DeviceError& e) {
        return fail(SKELFMM_EDEVICE, e.what());
    } catch (const skelfmm::NotSupported& e) {
        return fail(SKELFMM_ENOTSUP, e.what());
    } catch (const std::invalid_argument& e) {
        return fail(SKELFMM_EINVAL, e.what());
    } catch (const std::bad_alloc&) {
        return fail(SKELFMM_ENOMEM, "allocation failed");
    } catch (const skelfmm::OutOfMemory& e) {
        return fail(SKELFMM_ENOMEM, e.what());
    } catch (const std::exception& e) {
        return fail(SKELFMM_EINTERNAL, e.what());
    } catch (...) {
        return fail(SKELFMM_EINTERNAL, "unknown error");
    }
}

skelfmm_status check_dtype(const skelfmm_op* op, skelfmm_dtype dtype) {
    const bool helm = op->plan.kind == SKELFMM_HELMHOLTZ;
    if (dtype != SKELFMM_F64 && dtype != SKELFMM_F32 && dtype != SKELFMM_C128 && dtype != SKELFMM_C64)
        return fail(SKELFMM_EINVAL, "unknown dtype");
    const bool cplx = dtype == SKELFMM_C128 || dtype == SKELFMM_C64;
    if (helm != cplx) return fail(SKELFMM_EINVAL, helm ? "Helmholtz needs a complex dtype" : "Laplace needs a real dtype");
    return SKELFMM_OK;
}

}  // namespace

extern "C" {

const char* skelfmm_last_error(void) { return g_err.c_str(); }

skelfmm_status skelfmm_build(const double* points, int64_t n, skelfmm_kernel kernel, double tol,
                             int32_t leaf_size, const skelfmm_options* opt, skelfmm_op** out) {
    if (!out) return fail(SKELFMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!points) return fail(SKELFMM_EINVAL, "points is NULL");
    if (n <= 0) return fail(SKELFMM_EINVAL, "n must be positive");
    if (n >= (int64_t(1) << 31)) return fail(SKELFMM_EINVAL, "n must be below 2^31");
    if (kernel.dim != 2 && kernel.dim != 3) return fail(SKELFMM_EINVAL, "dim must be 2 or 3");
    if (kernel.kind != SKELFMM_LAPLACE && kernel.kind != SKELFMM_HELMHOLTZ)
        return fail(SKELFMM_EINVAL, "unknown kernel kind");
    if (kernel.kind == SKELFMM_HELMHOLTZ && !(kernel.kappa >= 0.0 && std::isfinite(kernel.kappa)))
        return fail(SKELFMM_EINVAL, "kappa must be finite and >= 0");
    if (!(tol > 0.0 && tol < 1.0)) return fail(SKELFMM_EINVAL, "tol must be in (0, 1)");
    if (leaf_size < 1) return fail(SKELFMM_EINVAL, "leaf_size must be >= 1");
    for (int64_t i = 0; i < n * kernel.dim; ++i)
        if (!std::isfinite(points[i])) return fail(SKELFMM_EINVAL, "point coordinates must be finite");
    return guarded([&]() -> skelfmm_status {
        auto* op = new skelfmm_op();
        try {
            if (opt) op->opt = *opt;
            skelfmm::Plan& p = op->plan;
            p.dim = kernel.dim;
            p.kind = kernel.kind;
            p.kappa = kernel.kind == SKELFMM_HELMHOLTZ ? kernel.kappa : 0.0;
            p.n = n;
            p.pts.assign(points, points + n * kernel.dim);
            p.tol = tol;
            p.leaf_size = leaf_size;
            p.opt.proxy_shape = op->opt.proxy_shape;
            p.opt.proxy_points = op->opt.proxy_points;
            p.opt.proxy_scale = op->opt.proxy_scale;
            p.opt.no_compression = op->opt.no_compression;
            p.opt.num_threads = op->opt.num_threads;
            p.opt.gpu_build = op->opt.gpu_build;
            if (p.opt.proxy_shape < 0 || p.opt.proxy_shape > 2 || p.opt.proxy_points < 0 || p.opt.proxy_scale < 0)
                throw std::invalid_argument("invalid proxy options");
            if (p.opt.proxy_shape == 2 && p.dim == 3) throw std::invalid_argument("the proxy circle is 2D only");
            skelfmm::build_plan(p);
            const auto tl0 = std::chrono::steady_clock::now();
            op->dev = skelfmm::device_create(p, op->opt.keep_transparent != 0, op->opt.f64_leaf != 0,
                                             op->opt.nonsymmetric == 0, op->opt.no_expansion == 0,
                                             op->opt.f32_differences != 0, op->opt.compensated_leaf != 0);
            p.t_layout = std::chrono::duration<double>(std::chrono::steady_clock::now() - tl0).count();
        } catch (...) {
            delete op;
            throw;
        }
        *out = op;
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_prepare(skelfmm_op* op, int64_t nrhs_max, skelfmm_dtype dtype) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (nrhs_max < 0) return fail(SKELFMM_EINVAL, "nrhs_max must be >= 0");
    if (skelfmm_status s = check_dtype(op, dtype)) return s;
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_prepare(op->dev, nrhs_max, static_cast<int>(dtype));
        return SKELFMM_OK;
    });
}

static skelfmm_status apply_common(skelfmm_op* op, const void* q, void* u, int64_t nrhs,
                                   skelfmm_dtype dtype, void* stream, bool adjoint) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!q || !u) return fail(SKELFMM_EINVAL, "NULL vector");
    if (q == u) return fail(SKELFMM_EINVAL, "input and output must not alias");
    if (nrhs < 1) return fail(SKELFMM_EINVAL, "nrhs must be >= 1");
    if (skelfmm_status s = check_dtype(op, dtype)) return s;
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_apply(op->dev, q, u, nrhs, static_cast<int>(dtype), stream, adjoint);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_apply(skelfmm_op* op, const void* q, void* u, int64_t nrhs,
                             skelfmm_dtype dtype, void* hip_stream) {
    return apply_common(op, q, u, nrhs, dtype, hip_stream, false);
}

skelfmm_status skelfmm_apply_adjoint(skelfmm_op* op, const void* v, void* w, int64_t nrhs,
                                     skelfmm_dtype dtype, void* hip_stream) {
    return apply_common(op, v, w, nrhs, dtype, hip_stream, true);
}

skelfmm_status skelfmm_apply_fwd_adj(skelfmm_op* op, const void* q, const void* v, void* u, void* w,
                                     skelfmm_dtype dtype, void* hip_stream) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!q || !v || !u || !w) return fail(SKELFMM_EINVAL, "NULL vector");
    if (q == u || q == w || v == u || v == w || u == w)
        return fail(SKELFMM_EINVAL, "inputs and outputs must be distinct buffers");
    if (skelfmm_status s = check_dtype(op, dtype)) return s;
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_apply_fwd_adj(op->dev, q, v, u, w, static_cast<int>(dtype), hip_stream);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_autotune_fwd_adj(skelfmm_op* op, void* hip_stream, int32_t* chosen, float* ms) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!chosen) return fail(SKELFMM_EINVAL, "chosen is NULL");
    return guarded([&]() -> skelfmm_status {
        float t[SKELFMM_NTPL] = {};
        *chosen = skelfmm::device_autotune_fwd_adj(op->dev, hip_stream, t);
        if (ms) for (int i = 0; i < SKELFMM_NTPL; ++i) ms[i] = t[i];
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_apply_noalloc(skelfmm_op* op, const void* q, void* u, int64_t nrhs, skelfmm_dtype dtype,
                                    int32_t adjoint, void* hip_stream) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!q || !u) return fail(SKELFMM_EINVAL, "NULL vector");
    if (q == u) return fail(SKELFMM_EINVAL, "input and output must not alias");
    if (nrhs < 1) return fail(SKELFMM_EINVAL, "nrhs must be >= 1");
    if (skelfmm_status s = check_dtype(op, dtype)) return s;
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_apply_noalloc(op->dev, q, u, nrhs, static_cast<int>(dtype), hip_stream, adjoint != 0);
        return SKELFMM_OK;
    });
}

int64_t skelfmm_noalloc_scratch_bytes(void) { return static_cast<int64_t>(skelfmm::device_scratch_bytes()); }

skelfmm_status skelfmm_stats_get(const skelfmm_op* op, skelfmm_stats* out) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!out) return fail(SKELFMM_EINVAL, "out is NULL");
    return guarded([&]() -> skelfmm_status {
        std::memset(out, 0, sizeof(*out));
        const skelfmm::Plan& p = op->plan;
        out->n_points = p.n;
        out->n_boxes = p.n_boxes;
        int nl = 0;
        for (int b = 0; b < p.n_boxes; ++b) nl += p.is_leaf[b];
        out->n_leaves = nl;
        out->max_level = p.max_level;
        out->top_level = p.top_level;
        out->k_max = p.k_max;
        out->proxy_count = p.proxy_count;
        out->t_tree = p.t_tree;
        out->t_skel = p.t_skel;
        out->t_skel_qr = p.t_skel_qr;
        out->t_layout = p.t_layout;
        out->m_proj_elems = static_cast<int64_t>(p.T.size());
        skelfmm::device_fill_stats(op->dev, out);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_autotune(skelfmm_op* op, skelfmm_dtype dtype, void* hip_stream, int32_t* chosen, float* ms) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!chosen) return fail(SKELFMM_EINVAL, "chosen is NULL");
    if (skelfmm_status s = check_dtype(op, dtype)) return s;
    return guarded([&]() -> skelfmm_status {
        float t[SKELFMM_NTPL] = {};
        *chosen = skelfmm::device_autotune(op->dev, static_cast<int>(dtype), hip_stream, t);
        if (ms) for (int i = 0; i < SKELFMM_NTPL; ++i) ms[i] = t[i];
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_set_targets_per_lane(skelfmm_op* op, int32_t tpl) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (tpl < 1 || tpl > SKELFMM_NTPL) return fail(SKELFMM_EINVAL, "targets per lane must be 1 .. 4");
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_set_tpl(op->dev, tpl);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_autotune_transfers(skelfmm_op* op, int64_t nrhs, void* hip_stream, int32_t* chosen,
                                         float* ms) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!chosen) return fail(SKELFMM_EINVAL, "chosen is NULL");
    if (nrhs < 1) return fail(SKELFMM_EINVAL, "nrhs must be >= 1");
    if (skelfmm_status s = check_dtype(op, SKELFMM_F32)) return s;
    return guarded([&]() -> skelfmm_status {
        float t[SKELFMM_NXFER] = {};
        *chosen = skelfmm::device_autotune_xfer(op->dev, nrhs, hip_stream, t);
        if (ms) for (int i = 0; i < SKELFMM_NXFER; ++i) ms[i] = t[i];
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_set_transfer_shape(skelfmm_op* op, int32_t shape) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (shape < 0 || shape >= SKELFMM_NXFER) return fail(SKELFMM_EINVAL, "transfer launch shape out of range");
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_set_xfer(op->dev, shape);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_timing(skelfmm_op* op, int32_t enable) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_timing(op->dev, enable != 0);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_timing_read(skelfmm_op* op, double* ms, int64_t* sweeps) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!ms || !sweeps) return fail(SKELFMM_EINVAL, "NULL output");
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_timing_read(op->dev, ms, sweeps);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_export(const skelfmm_op* op, skelfmm_plan_view* out) {
    if (!alive(op)) return fail(SKELFMM_EINVAL, "invalid operator");
    if (!out) return fail(SKELFMM_EINVAL, "out is NULL");
    const skelfmm::Plan& p = op->plan;
    std::memset(out, 0, sizeof(*out));
    out->dim = p.dim;
    out->kind = p.kind;
    out->kappa = p.kappa;
    out->n_points = p.n;
    out->points = p.pts.data();
    out->n_boxes = p.n_boxes;
    out->max_level = p.max_level;
    out->top_level = p.top_level;
    out->level = p.level.data();
    out->parent = p.parent.data();
    out->is_leaf = p.is_leaf.data();
    out->child_ptr = p.child_ptr.data();
    out->child_idx = p.child_idx.data();
    out->coord = p.coord.data();
    out->idx_ptr = p.idx_ptr.data();
    out->idx = p.idx.data();
    out->pos = p.pos.data();
    out->rank = p.rank.data();
    out->T_ptr = p.T_ptr.data();
    out->T = p.T.data();
    out->coll_ptr = p.coll_ptr.data();
    out->coll_idx = p.coll_idx.data();
    out->coarse_ptr = p.coarse_ptr.data();
    out->coarse_idx = p.coarse_idx.data();
    out->fine_ptr = p.fine_ptr.data();
    out->fine_idx = p.fine_idx.data();
    for (int d = 0; d < 3; ++d) out->root_lo[d] = p.root_lo[d];
    out->root_side = p.root_side;
    return SKELFMM_OK;
}

skelfmm_status skelfmm_batch_create(skelfmm_op* const* ops, int32_t nops, skelfmm_batch** out) {
    if (!out) return fail(SKELFMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ops || nops < 1) return fail(SKELFMM_EINVAL, "need at least one operator");
    for (int i = 0; i < nops; ++i)
        if (!alive(ops[i])) return fail(SKELFMM_EINVAL, "invalid operator in batch");
    for (int i = 1; i < nops; ++i)
        if (ops[i]->plan.kind != ops[0]->plan.kind || ops[i]->plan.dim != ops[0]->plan.dim)
            return fail(SKELFMM_EINVAL, "batched operators must share kind and dim");
    return guarded([&]() -> skelfmm_status {
        std::vector<skelfmm::DeviceOp*> devs;
        for (int i = 0; i < nops; ++i) devs.push_back(ops[i]->dev);
        auto* b = new skelfmm_batch();
        b->kind = ops[0]->plan.kind;
        try {
            b->dev = skelfmm::batch_create(devs);
        } catch (...) {
            delete b;
            throw;
        }
        *out = b;
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_batch_apply(skelfmm_batch* b, const void* const* q, void* const* u,
                                   int64_t nrhs, skelfmm_dtype dtype, int32_t adjoint, void* hip_stream) {
    if (!b || b->magic != kMagic) return fail(SKELFMM_EINVAL, "invalid batch");
    if (!q || !u) return fail(SKELFMM_EINVAL, "NULL vector list");
    if (nrhs < 1) return fail(SKELFMM_EINVAL, "nrhs must be >= 1");
    {
        const bool cplx = dtype == SKELFMM_C128 || dtype == SKELFMM_C64;
        if (dtype != SKELFMM_F64 && dtype != SKELFMM_F32 && !cplx) return fail(SKELFMM_EINVAL, "unknown dtype");
        if ((b->kind == SKELFMM_HELMHOLTZ) != cplx)
            return fail(SKELFMM_EINVAL, cplx ? "Laplace needs a real dtype" : "Helmholtz needs a complex dtype");
    }
    return guarded([&]() -> skelfmm_status {
        skelfmm::batch_apply(b->dev, q, u, nrhs, static_cast<int>(dtype), hip_stream, adjoint != 0);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_batch_autotune_transfers(skelfmm_batch* b, int64_t nrhs, void* hip_stream, int32_t* chosen,
                                               float* ms) {
    if (!b || b->magic != kMagic) return fail(SKELFMM_EINVAL, "invalid batch");
    if (!chosen) return fail(SKELFMM_EINVAL, "chosen is NULL");
    if (nrhs < 1) return fail(SKELFMM_EINVAL, "nrhs must be >= 1");
    if (b->kind != SKELFMM_LAPLACE) return fail(SKELFMM_EINVAL, "the matrix-core transfers serve Laplace batches");
    return guarded([&]() -> skelfmm_status {
        float t[SKELFMM_NXFER] = {};
        *chosen = skelfmm::batch_autotune_xfer(b->dev, nrhs, hip_stream, t);
        if (ms) for (int i = 0; i < SKELFMM_NXFER; ++i) ms[i] = t[i];
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_batch_timing(skelfmm_batch* b, int32_t enable) {
    if (!b || b->magic != kMagic) return fail(SKELFMM_EINVAL, "invalid batch");
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_timing(skelfmm::batch_merged(b->dev), enable != 0);
        return SKELFMM_OK;
    });
}

skelfmm_status skelfmm_batch_timing_read(skelfmm_batch* b, double* ms, int64_t* sweeps) {
    if (!b || b->magic != kMagic) return fail(SKELFMM_EINVAL, "invalid batch");
    if (!ms || !sweeps) return fail(SKELFMM_EINVAL, "NULL output");
    return guarded([&]() -> skelfmm_status {
        skelfmm::device_timing_read(skelfmm::batch_merged(b->dev), ms, sweeps);
        return SKELFMM_OK;
    });
}

void skelfmm_batch_destroy(skelfmm_batch* b) {
    if (!b || b->magic != kMagic) return;
    try { skelfmm::batch_destroy(b->dev); } catch (...) {}
    b->magic = kDead;
    delete b;
}

void skelfmm_destroy(skelfmm_op* op) {
    if (!alive(op)) return;
    try { skelfmm::device_destroy(op->dev); } catch (...) {}
    op->magic = kDead;
    delete op;
}

}  // extern "C"
