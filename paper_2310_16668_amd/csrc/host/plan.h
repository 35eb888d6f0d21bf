// Host-side plan: the adaptive tree, its neighbor lists and the skeleton
// operators of every box (section 3, "Adaptive tree data structure" and
// "Build stage").  Built once in float64 on the host; the device layout is
// packed from it.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

namespace skelfmm {

// An allocator whose value-less construct leaves doubles uninitialised, so a
// large array that is written in full right after resize() is not zero-filled
// first.
template <class T>
struct DefaultInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = DefaultInitAlloc<U>;
    };
    DefaultInitAlloc() = default;
    template <class U>
    DefaultInitAlloc(const DefaultInitAlloc<U>&) noexcept {}
    template <class U>
    void construct(U* p) noexcept {
        ::new (static_cast<void*>(p)) U;
    }
    template <class U, class... Args>
    void construct(U* p, Args&&... args) {
        ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
    }
};
using DoubleArray = std::vector<double, DefaultInitAlloc<double>>;

struct BuildOptions {
    int proxy_shape = 0;       // 0 default (2D circle, 3D Chebyshev box), 1 box, 2 circle (2D)
    int proxy_points = 0;      // per side (box) or total (circle); 0 = default
    double proxy_scale = 0.0;  // box side / a (circle radius = scale/2 * a); 0 = default 2.95
    int no_compression = 0;    // force k = n everywhere (test mode)
    int max_depth = 20;
    int num_threads = 0;       // 0 = hardware concurrency
    int gpu_build = 0;         // 1: interpolative decompositions on the current HIP device
};

struct Plan {
    // problem
    int dim = 3;
    int kind = 0;              // 0 Laplace, 1 Helmholtz
    double kappa = 0.0;
    int64_t n = 0;
    std::vector<double> pts;   // n x dim, user order
    double tol = 1e-6;
    int leaf_size = 64;
    BuildOptions opt;

    // tree (boxes numbered level by level, Morton order within a level)
    double root_lo[3] = {0, 0, 0};
    double root_side = 1.0;
    int n_boxes = 0;
    int max_level = 0;         // L
    int top_level = 0;         // 1 if the root has children, else 0
    std::vector<int32_t> level_ptr;            // boxes of level l: [level_ptr[l], level_ptr[l+1])
    std::vector<int32_t> level, parent, is_leaf, child_ptr, child_idx;
    std::vector<int32_t> coord;                // n_boxes x 3 integer coords at own level
    std::vector<int32_t> coll_ptr, coll_idx;   // colleagues incl. self
    std::vector<int32_t> coarse_ptr, coarse_idx;
    std::vector<int32_t> fine_ptr, fine_idx;

    // per-box index sets and skeletons
    std::vector<int64_t> idx_ptr, idx;         // natural order: leaf points / children's skeletons
    std::vector<int32_t> rank;                 // k per box, -1 for boxes at or above the top level
    std::vector<int64_t> pos;                  // per box [sk positions | rd positions] in natural order
    std::vector<int64_t> T_ptr;                // offsets into T (n_boxes + 1)
    DoubleArray T;                             // column-major k x (n - k) per box

    // statistics
    double t_tree = 0.0, t_skel = 0.0;
    double t_skel_qr = 0.0;    // part of t_skel in the IDs themselves
    double t_layout = 0.0;     // packing the device layout
    int k_max = 0;
    int proxy_count = 0;
};

// Build the tree, neighbor lists and skeletons.  Throws std::runtime_error
// (std::invalid_argument for bad arguments) on failure.
void build_plan(Plan& p);

// Kernel value on the host (used only by the build's proxy matrices).
double host_kernel_real(const Plan& p, const double* x, const double* y);

}  // namespace skelfmm
