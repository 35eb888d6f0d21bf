// Sweep instantiation for one kernel family (3D Laplace).
#include "sweep.h"

namespace skelfmm {

void sweep_lap3(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
                 const Work& w) {
    dispatch<3, 0>(d, io, nrhs, dtype, s, adjoint, w);
}

void tune_lap3(DeviceOp* d, int dtype, hipStream_t s, float* ms_out, bool pair) {
    tune_near<3, 0>(d, dtype, s, ms_out, pair);
}

void sweep_pair_lap3(DeviceOp* d, const std::vector<IO>& io, hipStream_t s, const Work& w) {
    dispatch_pair<3>(d, io, s, w);
}

}  // namespace skelfmm
