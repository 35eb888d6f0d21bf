// Interface between the C ABI and the GPU executor.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../../include/skelfmm.h"
#include "../host/plan.h"

namespace skelfmm {

struct DeviceError : std::runtime_error { using std::runtime_error::runtime_error; };
struct NotSupported : std::runtime_error { using std::runtime_error::runtime_error; };
struct OutOfMemory : std::runtime_error { using std::runtime_error::runtime_error; };

// Near-field segment modes (what a source box contributes to a target box).
enum SegMode : int32_t {
    SEG_DIRECT = 0,   // u += G q over all source entries (top level)
    SEG_IFO = 1,      // colleague: u += G q ; uhat -= G qhat over the source skeleton
    SEG_IFS = 2,      // coarse leaf: u += G q ; uhat -= G q
    SEG_TFO = 3,      // fine box of a leaf: u += G q - G qhat (skeleton part)
    SEG_MODE_MASK = 7,
    SEG_SELF = 8      // flag: the source box is the target box
};

struct Task {
    int32_t box;      // target box
    int32_t t0;       // first target entry (relative to the box)
};

// One symmetric colleague-pair work item: the kernel block G(B_i, B_j) is
// evaluated once and serves u_i (forward) and u_j (reverse).  Slot offsets:
// fwd_u / fwd_h are the slots of target t0 in box i's u / uhat row (target t at
// offset t - t0); rev_u / rev_h the first slot of box j's u / uhat row.
struct SymTask {
    int32_t bi, bj;   // target-side box (lanes) and source-side box (wave-uniform)
    int32_t t0, t1;   // target entries [t0, t1) of bi
    int32_t flags;    // SymFlags: how the float32 evaluation may form |d|^2
    int32_t pad;
    int64_t fwd_u, fwd_h, rev_u, rev_h;
};
// SYM_EXPANDED: |d|^2 may be expanded about the source box's origin (float64
// terms); SYM_F32DIFF: |d|^2 may come from float32 differences about it.
enum SymFlags : int32_t { SYM_EXPANDED = 1, SYM_F32DIFF = 2 };
// The pair kernel's expanded source records (and its float32 relative
// coordinates, laid out alike): box b's records start at
// voff[b] + kSymRecordPad * b and are followed by kSymRecordPad copies of its
// last record, so a block of up to kSymRecordPad + 1 sources is read without
// clamping its indices (the copies take zero charges).
constexpr int kSymRecordPad = 7;

// The slot rows of one box: ru rows of n entries from base_u (added to u) and
// rh rows of k entries from base_h (added to uhat).
struct SymRows {
    int32_t box, ru, rh, pad;
    int64_t base_u, base_h;
};

// Host copy of everything the GPU sweep reads.  Built without touching a GPU.
struct Layout {
    int dim = 3, kind = 0;
    double kappa = 0.0;
    int64_t n_points = 0;
    int n_boxes = 0, top = 0, max_level = 0;
    double center[3] = {0, 0, 0};
    std::vector<int32_t> level_ptr;
    // per box
    std::vector<int64_t> voff, hoff, toff;
    std::vector<int32_t> nb, kb, level, parent, is_leaf;
    // entries: index-set members of every box at or below the top level, per box
    // in [skeleton | redundant] order
    int64_t n_entries = 0, n_hentries = 0;
    std::vector<double> X;          // n_entries x 4 (x, y, z, 0), root-centred
    // per box: lower bound of the distance between its entries and any other point,
    // box centre (root-centred) and radius of its entries about it
    std::vector<double> dmin, bcenter, brad;
    std::vector<int32_t> perm;      // user index of leaf entries, -1 elsewhere
    std::vector<int32_t> pmap;      // skeleton entry -> entry in the parent's vector
    std::vector<int32_t> gather_e, gather_p;     // leaf entries and their user indices
    std::vector<int32_t> topleaf_e, topleaf_p;   // entries of top-level leaves
    // interpolation matrices, column-major per box (at toff): the plan's own
    // array (Tref, which outlives the layout) or, for a merged batch layout, T
    DoubleArray T;
    const DoubleArray* Tref = nullptr;
    const DoubleArray& Tvec() const { return Tref ? *Tref : T; }
    // device copies of T (k x m per box) and of its transpose (m x k) have their
    // columns padded to kTPad entries, so no 128-byte line is shared by two row
    // groups of a transfer; tpad / ttpad are the padded per-box offsets
    std::vector<int64_t> tpad, ttpad;
    int64_t tpad_size = 0, ttpad_size = 0;
    // near field
    std::vector<int32_t> seg_ptr;   // per target box
    std::vector<int32_t> seg_src, seg_mode;
    std::vector<Task> tasks;        // built for `tile` targets per work item
    int tile = 128;
    int64_t pairs_near = 0, pairs_skel = 0;
    // symmetric pairs (real kernels, one RHS): the colleague pairs they cover are
    // removed from the *_ns segment lists, which serve the one-RHS near field
    bool sym = false;
    bool allow_expanded = true;     // pair items may use the expanded |d|^2 where the bound allows
    bool allow_f32diff = false;     // pair items may use float32 differences where the bound allows
    std::vector<int32_t> seg_ptr_ns, seg_src_ns, seg_mode_ns;
    std::vector<SymTask> sym_tasks;
    std::vector<SymRows> sym_rows;               // boxes receiving slot rows
    int64_t slot_size = 0;
};

constexpr int kTPad = 32;
inline int64_t pad_ld(int64_t x) { return (x + kTPad - 1) / kTPad * kTPad; }
// Padded offsets of the device copies of T and T^T (tpad, ttpad).
void pad_transfer_offsets(Layout& L);

Layout make_layout(const Plan& p, bool keep_transparent, int tile);
// Work list for another tile size, largest estimated cost first, over the full
// segment lists (ns = false) or the lists left after symmetric pairing (ns = true).
std::vector<Task> make_tasks(const Layout& L, int tile, bool ns = false);
// Pair up colleague segments of compressed boxes for the symmetric near field;
// self_items: a box's segment with itself becomes one pair item too (else it
// stays on the segment lists).
void make_symmetric(Layout& L, int group, bool self_items);
// Kernel evaluations of the pair items with tpl targets per lane: out[0] pairs
// serving both directions, out[1] their skeleton pairs, out[2] one-direction
// evaluations in the diagonal tiles of self items, out[3] their skeleton pairs.
void sym_pair_counts(const Layout& L, int tpl, int64_t out[4]);
// One layout for several operators: boxes renumbered by (level, operator), entry,
// skeleton-entry and T offsets shifted, one cost-sorted work list over all of
// them.  entry_base / hentry_base receive each operator's first entry / skeleton entry.
Layout merge_layouts(const std::vector<const Layout*>& ls, std::vector<int64_t>& entry_base);

struct DeviceOp;
struct DeviceBatch;

DeviceOp* device_create(const Plan& p, bool keep_transparent, bool f64_leaf, bool symmetric, bool expanded, bool f32diff,
                        bool compensated);
void device_prepare(DeviceOp* d, int64_t nrhs_max, int dtype);
void device_apply(DeviceOp* d, const void* q, void* u, int64_t nrhs, int dtype, void* stream, bool adjoint);
// u = A q and w = A^H v; real kernels in float32 share one sweep
void device_apply_fwd_adj(DeviceOp* d, const void* q, const void* v, void* u, void* w, int dtype, void* stream);
int device_autotune_fwd_adj(DeviceOp* d, void* stream, float* ms_out);
void device_apply_noalloc(DeviceOp* d, const void* q, void* u, int64_t nrhs, int dtype, void* stream,
                          bool adjoint);
size_t device_scratch_bytes();
void device_fill_stats(const DeviceOp* d, skelfmm_stats* out);
void device_destroy(DeviceOp* d);
void device_timing(DeviceOp* d, bool enable);
int device_autotune(DeviceOp* d, int dtype, void* stream, float* ms_out);
void device_set_tpl(DeviceOp* d, int tpl);
int device_autotune_xfer(DeviceOp* d, int64_t nrhs, void* stream, float* ms_out);
void device_set_xfer(DeviceOp* d, int shape);
void device_timing_read(DeviceOp* d, double* ms, int64_t* sweeps);

DeviceBatch* batch_create(const std::vector<DeviceOp*>& ops);
void batch_apply(DeviceBatch* b, const void* const* q, void* const* u, int64_t nrhs, int dtype,
                 void* stream, bool adjoint);
void batch_destroy(DeviceBatch* b);
int batch_autotune_xfer(DeviceBatch* b, int64_t nrhs, void* stream, float* ms_out);
DeviceOp* batch_merged(DeviceBatch* b);   // the merged operator the batch's sweeps run on

}  // namespace skelfmm
