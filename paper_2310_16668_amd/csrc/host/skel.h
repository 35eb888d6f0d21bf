// Pieces of the skeletonization (section 3, "Build stage") shared by the host
// build and the device build of the interpolative decompositions.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "plan.h"

namespace skelfmm {

// One box's index set and skeleton.
struct BoxSkel {
    std::vector<int64_t> idx;     // natural order (original point indices)
    int k = 0;                    // skeleton size
    std::vector<int64_t> pos;     // [skeleton | redundant] positions within idx
    std::vector<double> T;        // k x (n - k), column-major
    // or, from the device build, the same k x (n - k) values held by the level
    // skeletonizer (valid while it lives): Tn entries at Tsrc
    const double* Tsrc = nullptr;
    int64_t Tn = 0;
    int64_t t_size() const { return Tsrc ? Tn : static_cast<int64_t>(T.size()); }
};

// The proxy surface of a box of side a centred at c is c + h U_r with
// h = (returned factor) * a and U the unit pattern (np x dim, row-major):
// 3D first-kind Chebyshev nodes on the faces of [-1, 1]^3, 2D the unit circle
// (or the square's edges).
double proxy_pattern(const Plan& p, std::vector<double>& U);

// Skeletonizes every box of a level at once (index sets given, k / pos / T
// filled); the device build implements it.
struct LevelSkeletonizer {
    virtual ~LevelSkeletonizer() = default;
    virtual void level(const Plan& p, int b0, int b1, std::vector<BoxSkel>& S) = 0;
};
std::unique_ptr<LevelSkeletonizer> make_device_skeletonizer(const Plan& p);

}  // namespace skelfmm
