// Sweep instantiation for one kernel family (3D Laplace).
#include "sweep.h"

namespace skelfmm {

void sweep_lap3(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
                 const Work& w) {
    dispatch<3, 0>(d, io, nrhs, dtype, s, adjoint, w);
}

void tune_lap3(DeviceOp* d, int dtype, hipStream_t s, float* ms_out) { tune_near<3, 0>(d, dtype, s, ms_out); }

}  // namespace skelfmm
