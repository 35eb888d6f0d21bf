// Sweep instantiation for one kernel family (2D Laplace).
#include "sweep.h"

namespace skelfmm {

void sweep_lap2(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
                 const Work& w) {
    dispatch<2, 0>(d, io, nrhs, dtype, s, adjoint, w);
}

void tune_lap2(DeviceOp* d, int dtype, hipStream_t s, float* ms_out, bool pair) {
    tune_near<2, 0>(d, dtype, s, ms_out, pair);
}

void sweep_pair_lap2(DeviceOp* d, const std::vector<IO>& io, hipStream_t s, const Work& w) {
    dispatch_pair<2>(d, io, s, w);
}

}  // namespace skelfmm
