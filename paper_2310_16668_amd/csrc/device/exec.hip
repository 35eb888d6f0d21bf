// GPU executor placeholder: the layout is packed on the host; the sweep
// itself is not built yet, so every GPU entry point reports ENOTSUP.
#include <hip/hip_runtime.h>

#include <memory>

#include "device.h"

namespace skelfmm {

struct DeviceOp {
    Layout L;
};
struct DeviceBatch {
    std::vector<DeviceOp*> ops;
};

DeviceOp* device_create(const Plan& p, bool keep_transparent, bool) {
    auto d = std::make_unique<DeviceOp>();
    d->L = make_layout(p, keep_transparent, 128);
    return d.release();
}
void device_prepare(DeviceOp*, int64_t, int) { throw NotSupported("GPU sweep not built"); }
void device_apply(DeviceOp*, const void*, void*, int64_t, int, void*, bool) { throw NotSupported("GPU sweep not built"); }
void device_fill_stats(const DeviceOp* d, skelfmm_stats* out) {
    out->n_entries = d->L.n_entries;
    out->pairs_near = d->L.pairs_near;
    out->pairs_skel = d->L.pairs_skel;
    out->n_tasks = static_cast<int64_t>(d->L.tasks.size());
    out->tile_targets = d->L.tile;
}
void device_destroy(DeviceOp* d) { delete d; }
DeviceBatch* batch_create(const std::vector<DeviceOp*>& ops) { return new DeviceBatch{ops}; }
void batch_apply(DeviceBatch*, const void* const*, void* const*, int64_t, int, void*, bool) {
    throw NotSupported("GPU sweep not built");
}
void batch_destroy(DeviceBatch* b) { delete b; }

}  // namespace skelfmm
