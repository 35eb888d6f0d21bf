// Sweep instantiation for one kernel family (2D Helmholtz).
#include "sweep.h"

namespace skelfmm {

void sweep_helm2(DeviceOp* d, const std::vector<IO>& io, int64_t nrhs, int dtype, hipStream_t s, bool adjoint,
                 const Work& w) {
    dispatch<2, 1>(d, io, nrhs, dtype, s, adjoint, w);
}

void tune_helm2(DeviceOp* d, int dtype, hipStream_t s, float* ms_out) { tune_near<2, 1>(d, dtype, s, ms_out); }

}  // namespace skelfmm
