// Packs a built plan into the flat, level-sorted arrays the GPU sweep reads.
//
// Entries.  Every box at or below the top level owns a contiguous run of
// "entries", one per member of its index set, ordered [skeleton | redundant]
// (the skeleton positions first, as the build's pivot order gives them).  With
// that order the outgoing skeleton charges are qhat = q[0:k] + T q[k:n] and the
// downward pass adds uhat to u[0:k] and T^T uhat to u[k:n].  Boxes above the top
// level own no entries.  Boxes of one level are contiguous, so one launch per
// level covers its boxes.
//
// pmap sends skeleton entry i of a box to the entry of its parent that holds
// the same point, so the upward pass writes qhat straight into the parent's
// vector and the downward pass reads the parent's potential back from it.
//
// Near-field work.  For each target box, the list of source boxes ("segments")
// with their translation type; the work list splits every target box into
// tiles of `tile` entries, sorted by estimated cost (largest first) so one
// launch over all levels balances across compute units.
//
// A box that keeps all its points (k = n) is transparent: qhat = q and
// E = F = I.  An ifo pair of two transparent boxes adds A q to u and subtracts
// the same A q from uhat, which the downward pass then adds back to u, so the
// pair is skipped unless requested; likewise an ifs pair with a transparent
// target and a tfo pair with a transparent source.
#include <algorithm>
#include <cmath>
#include <limits>
#include <tuple>
#include <numeric>
#include <stdexcept>

#include "device.h"
#include "../host/parallel.h"

namespace skelfmm {

// Geometry for the float32 evaluation of the pair kernel (sym_flags below): a
// lower bound d of the distance between any two distinct entries of a box, and
// the box's centre and radius (the reach R of an item from its origin).
//
// Lower bound of the nearest-neighbor distance of every point: a leaf's points
// are compared with the points of the leaf itself, its colleague leaves, its
// coarse and its fine neighbor leaves; any other point lies at least half the
// leaf's side away (under strong balance every box touching a leaf is at most
// one level finer, and those are leaves on its fine list).
static void box_geometry(const Plan& p, Layout& L) {
    const int nb = p.n_boxes;
    const int dim = p.dim;
    std::vector<double> nn(static_cast<size_t>(p.n), std::numeric_limits<double>::infinity());
    std::vector<int32_t> leaves;
    for (int b = 0; b < nb; ++b)
        if (p.is_leaf[b] && p.idx_ptr[b + 1] > p.idx_ptr[b]) leaves.push_back(b);
    auto dist2 = [&](int64_t a, int64_t c) {
        double s2 = 0.0;
        for (int d = 0; d < dim; ++d) {
            const double t = p.pts[a * dim + d] - p.pts[c * dim + d];
            s2 += t * t;
        }
        return s2;
    };
    parallel_for(static_cast<int64_t>(leaves.size()), host_threads(p.opt.num_threads), [&](int64_t li) {
        const int b = leaves[li];
        const double half = 0.5 * std::ldexp(p.root_side, -p.level[b]);
        std::vector<int32_t> cand;
        for (int x = p.coll_ptr[b]; x < p.coll_ptr[b + 1]; ++x)
            if (p.is_leaf[p.coll_idx[x]]) cand.push_back(p.coll_idx[x]);
        for (int x = p.coarse_ptr[b]; x < p.coarse_ptr[b + 1]; ++x) cand.push_back(p.coarse_idx[x]);
        for (int x = p.fine_ptr[b]; x < p.fine_ptr[b + 1]; ++x) cand.push_back(p.fine_idx[x]);
        // the candidates' boxes: a box farther from the point than the best
        // distance so far cannot hold a nearer point
        std::vector<double> lo(cand.size() * 3), hi(cand.size() * 3);
        for (size_t q = 0; q < cand.size(); ++q) {
            const double side = std::ldexp(p.root_side, -p.level[cand[q]]);
            for (int d = 0; d < dim; ++d) {
                lo[3 * q + d] = p.root_lo[d] + p.coord[3 * cand[q] + d] * side;
                hi[3 * q + d] = lo[3 * q + d] + side;
            }
        }
        for (int64_t i = p.idx_ptr[b]; i < p.idx_ptr[b + 1]; ++i) {
            const int64_t a = p.idx[i];
            double m = half * half;
            for (size_t q = 0; q < cand.size(); ++q) {
                double g2 = 0.0;
                for (int d = 0; d < dim; ++d) {
                    const double x = p.pts[a * dim + d];
                    const double t = x < lo[3 * q + d] ? lo[3 * q + d] - x : (x > hi[3 * q + d] ? x - hi[3 * q + d] : 0.0);
                    g2 += t * t;
                }
                if (g2 >= m) continue;
                const int c = cand[q];
                for (int64_t j = p.idx_ptr[c]; j < p.idx_ptr[c + 1]; ++j)
                    if (p.idx[j] != a) m = std::min(m, dist2(a, p.idx[j]));
            }
            nn[a] = std::sqrt(m);
        }
    }, 16);
    L.dmin.assign(nb, 0.0);
    L.bcenter.assign(static_cast<size_t>(nb) * 3, 0.0);
    L.brad.assign(nb, 0.0);
    for (int b = 0; b < nb; ++b) {
        const double side = std::ldexp(p.root_side, -p.level[b]);
        double c[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) c[d] = p.root_lo[d] + (p.coord[3 * b + d] + 0.5) * side - L.center[d];
        double dm = std::numeric_limits<double>::infinity(), r2 = 0.0;
        for (int64_t i = p.idx_ptr[b]; i < p.idx_ptr[b + 1]; ++i) {
            const int64_t a = p.idx[i];
            dm = std::min(dm, nn[a]);
            double s2 = 0.0;
            for (int d = 0; d < dim; ++d) {
                const double t = (p.pts[a * dim + d] - L.center[d]) - c[d];
                s2 += t * t;
            }
            r2 = std::max(r2, s2);
        }
        L.dmin[b] = dm;
        for (int d = 0; d < 3; ++d) L.bcenter[3 * b + d] = c[d];
        L.brad[b] = std::sqrt(r2);
    }
}

// R / d for an item of boxes i != j: R the reach of the two boxes from the
// origin (the first entry of the source box j), d their smallest point spacing.
// The expanded |d|^2 = |t'|^2 + |s'|^2 - 2 t'.s' in float64 has terms of about
// R^2, so its absolute error is below 20 u R^2 (u = 2^-53) and its error
// relative to |d|^2 >= d^2 below 20 u (R/d)^2: with R <= 4096 d about 3.7e-8,
// 1.9e-8 on the kernel value, a third of the float32 rounding that follows.
static double reach_ratio(const Layout& L, int bi, int bj) {
    if (L.nb[bj] == 0 || L.dmin.empty()) return std::numeric_limits<double>::infinity();
    // the expanded records of box j are relative to its first entry
    const double* o = &L.X[static_cast<size_t>(L.voff[bj]) * 4];
    auto reach = [&](int b) {
        double s2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double t = L.bcenter[3 * b + d] - o[d];
            s2 += t * t;
        }
        return std::sqrt(s2) + L.brad[b];
    };
    const double R = std::max(reach(bi), reach(bj));
    const double d = std::min(L.dmin[bi], L.dmin[bj]);
    return d > 0.0 ? R / d : std::numeric_limits<double>::infinity();
}

// The float32 evaluation of an item of boxes i != j: float32 differences of
// coordinates relative to the source box's first entry where R <= 1024 d (each
// coordinate rounded once, so |d| is off by at most about R 2^-24 and a kernel
// value by (R / |d| + 1) 2^-24 relative), else the expanded form where
// R <= 4096 d, else float64 differences.
static int32_t sym_flags(const Layout& L, int bi, int bj) {
    if (!L.allow_expanded && !L.allow_f32diff) return 0;
    const double q = reach_ratio(L, bi, bj);
    if (L.allow_f32diff && q <= 1024.0) return SYM_F32DIFF;
    if (L.allow_expanded && q <= 4096.0) return SYM_EXPANDED;
    return 0;
}

Layout make_layout(const Plan& p, bool keep_transparent, int tile) {
    Layout L;
    L.dim = p.dim;
    L.kind = p.kind;
    L.kappa = p.kappa;
    L.n_points = p.n;
    L.n_boxes = p.n_boxes;
    L.top = p.top_level;
    L.max_level = p.max_level;
    L.level_ptr = p.level_ptr;
    L.tile = tile;
    const int nb = p.n_boxes;
    for (int d = 0; d < p.dim; ++d) L.center[d] = p.root_lo[d] + 0.5 * p.root_side;

    L.voff.assign(nb, 0);
    L.hoff.assign(nb, 0);
    L.toff.assign(nb, 0);
    L.nb.assign(nb, 0);
    L.kb.assign(nb, 0);
    L.level = p.level;
    L.parent = p.parent;
    L.is_leaf = p.is_leaf;
    int64_t e = 0, h = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t n = p.idx_ptr[b + 1] - p.idx_ptr[b];
        if (n >= (int64_t(1) << 31)) throw std::runtime_error("box too large");
        L.voff[b] = e;
        L.nb[b] = static_cast<int32_t>(n);
        L.kb[b] = p.level[b] > p.top_level ? p.rank[b] : 0;
        L.hoff[b] = h;
        L.toff[b] = p.T_ptr[b];
        e += n;
        h += L.kb[b];
    }
    L.n_entries = e;
    L.n_hentries = h;
    if (e >= (int64_t(1) << 31)) throw std::runtime_error("too many entries for 32-bit maps");

    // entry coordinates (root-centred) and leaf permutation
    L.X.assign(static_cast<size_t>(e) * 4, 0.0);
    L.perm.assign(e, -1);
    // leaf entries in box order: each box's first slot in the gather lists
    std::vector<int64_t> goff(nb + 1, 0), tgoff(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        goff[b + 1] = goff[b] + (p.is_leaf[b] ? L.nb[b] : 0);
        tgoff[b + 1] = tgoff[b] + (p.is_leaf[b] && p.level[b] == p.top_level ? L.nb[b] : 0);
    }
    L.gather_e.resize(goff[nb]);
    L.gather_p.resize(goff[nb]);
    L.topleaf_e.resize(tgoff[nb]);
    L.topleaf_p.resize(tgoff[nb]);
    parallel_for(nb, host_threads(p.opt.num_threads), [&](int64_t bb) {
        const int b = static_cast<int>(bb);
        const int64_t n = L.nb[b];
        const int64_t* ix = &p.idx[p.idx_ptr[b]];
        const int64_t* ps = &p.pos[p.idx_ptr[b]];
        for (int64_t i = 0; i < n; ++i) {
            const int64_t pt = ix[ps[i]];
            double* x = &L.X[static_cast<size_t>(L.voff[b] + i) * 4];
            for (int d = 0; d < p.dim; ++d) x[d] = p.pts[pt * p.dim + d] - L.center[d];
            if (p.is_leaf[b]) {
                L.perm[L.voff[b] + i] = static_cast<int32_t>(pt);
                L.gather_e[goff[b] + i] = static_cast<int32_t>(L.voff[b] + i);
                L.gather_p[goff[b] + i] = static_cast<int32_t>(pt);
                if (p.level[b] == p.top_level) {
                    L.topleaf_e[tgoff[b] + i] = static_cast<int32_t>(L.voff[b] + i);
                    L.topleaf_p[tgoff[b] + i] = static_cast<int32_t>(pt);
                }
            }
        }
    }, 64);
    if (static_cast<int64_t>(L.gather_e.size()) != p.n) throw std::runtime_error("leaves do not partition the points");

    // parent slots of skeleton entries
    L.pmap.assign(h, 0);
    for (int b = 0; b < nb; ++b) {
        if (p.level[b] <= p.top_level) continue;
        const int par = p.parent[b];
        // offset of b's block in the parent's natural order
        int64_t off = 0;
        for (int c = p.child_ptr[par]; c < p.child_ptr[par + 1]; ++c) {
            if (p.child_idx[c] == b) break;
            off += p.rank[p.child_idx[c]];
        }
        // inverse of the parent's [sk | rd] order
        const int64_t np = L.nb[par];
        const int64_t* pp = &p.pos[p.idx_ptr[par]];
        std::vector<int32_t> inv(np);
        for (int64_t i = 0; i < np; ++i) inv[pp[i]] = static_cast<int32_t>(i);
        for (int i = 0; i < L.kb[b]; ++i)
            L.pmap[L.hoff[b] + i] = static_cast<int32_t>(L.voff[par] + inv[off + i]);
    }
    L.Tref = &p.T;

    // near-field segments per target box
    auto transparent = [&](int b) { return L.kb[b] == L.nb[b]; };
    L.seg_ptr.assign(nb + 1, 0);
    std::vector<int32_t> top_boxes;
    for (int b = p.level_ptr[p.top_level]; b < p.level_ptr[p.top_level + 1]; ++b) top_boxes.push_back(b);
    for (int b = 0; b < nb; ++b) {
        const int lb = p.level[b];
        if (lb >= p.top_level) {
            if (lb == p.top_level) {
                for (int c : top_boxes) {
                    L.seg_src.push_back(c);
                    L.seg_mode.push_back(SEG_DIRECT | (c == b ? SEG_SELF : 0));
                }
            } else {
                for (int x = p.coll_ptr[b]; x < p.coll_ptr[b + 1]; ++x) {
                    const int c = p.coll_idx[x];
                    if (!keep_transparent && transparent(b) && transparent(c)) continue;
                    L.seg_src.push_back(c);
                    L.seg_mode.push_back(SEG_IFO | (c == b ? SEG_SELF : 0));
                }
                for (int x = p.coarse_ptr[b]; x < p.coarse_ptr[b + 1]; ++x) {
                    const int c = p.coarse_idx[x];
                    if (!keep_transparent && transparent(b)) continue;
                    L.seg_src.push_back(c); L.seg_mode.push_back(SEG_IFS);
                }
            }
            if (p.is_leaf[b])
                for (int x = p.fine_ptr[b]; x < p.fine_ptr[b + 1]; ++x) {
                    const int c = p.fine_idx[x];
                    if (!keep_transparent && transparent(c)) continue;
                    L.seg_src.push_back(c); L.seg_mode.push_back(SEG_TFO);
                }
        }
        L.seg_ptr[b + 1] = static_cast<int32_t>(L.seg_src.size());
    }

    pad_transfer_offsets(L);
    box_geometry(p, L);

    // work list and pair counts
    L.tasks = make_tasks(L, tile);
    for (int b = 0; b < nb; ++b) {
        if (L.level[b] < L.top || L.nb[b] == 0) continue;
        int64_t src = 0, skel_src = 0;
        for (int x = L.seg_ptr[b]; x < L.seg_ptr[b + 1]; ++x) {
            const int c = L.seg_src[x];
            const int mode = L.seg_mode[x] & SEG_MODE_MASK;
            src += L.nb[c];
            if (mode == SEG_IFO) skel_src += L.kb[c];
            if (mode == SEG_IFS) skel_src += L.nb[c];
        }
        L.pairs_near += int64_t(L.nb[b]) * src;
        L.pairs_skel += int64_t(std::min(L.kb[b], L.nb[b])) * skel_src;
    }
    return L;
}

// Symmetric near field.  An ifo segment (i <- j) and its mirror (j <- i) use the
// same kernel block, and so do two top-level boxes' direct segments, so every
// such unordered pair {i, j} (i != j; ifo pairs of two uncompressed boxes are
// already absent) becomes work items that evaluate G(B_i, B_j) once: lanes run
// over targets of box i, groups of at most `group` targets per item.  A box's
// segment with itself becomes one item over all its targets that evaluates each
// unordered pair of its entries once outside the diagonal tiles of its passes.
//
// Items write private slots laid out as dense rows per receiving box: for each
// pair, one u row (and one uhat row) of box i that its groups fill by target
// range, and per group one u row (and, when the group holds skeleton targets of
// i, one uhat row) of box j; a box paired with itself has a forward and a
// reverse row of each kind.  The reduction adds a box's rows to its u and uhat
// in row order, so results stay deterministic.
void make_symmetric(Layout& L, int group, bool self_items) {
    L.sym = true;
    const int nb = L.n_boxes;
    struct Pair { int32_t bi, bj; };
    std::vector<Pair> pairs_list;
    std::vector<std::vector<int32_t>> rem(nb), remm(nb);
    for (int b = 0; b < nb; ++b) {
        for (int x = L.seg_ptr[b]; x < L.seg_ptr[b + 1]; ++x) {
            const int c = L.seg_src[x];
            const int mode = L.seg_mode[x];
            const int mt = mode & SEG_MODE_MASK;
            if (mt != SEG_IFO && mt != SEG_DIRECT) {
                rem[b].push_back(c);
                remm[b].push_back(mode);
                continue;
            }
            if (c == b) {   // a box with itself: one item over all its targets
                if (!self_items) {
                    rem[b].push_back(c);
                    remm[b].push_back(mode);
                } else if (L.nb[b] > 0) {
                    pairs_list.push_back(Pair{b, b});
                }
                continue;
            }
            if (c < b) continue;   // the pair was handled from the smaller id
            // i = the box on the lanes: the side whose targets fill the passes
            // with fewer idle lane slots per source pair; on a tie the box with
            // more entries.  Full passes hold 64 TPL targets and the last pass
            // the fewest targets per lane that hold the rest, so m targets take
            // 64 ceil(m / 64) lane slots at any TPL.
            auto lanes = [](int64_t m) { return (m + 63) / 64 * 64; };
            const int64_t cost_b = lanes(L.nb[b]) * L.nb[c], cost_c = lanes(L.nb[c]) * L.nb[b];
            int bi = b, bj = c;
            if (cost_c < cost_b || (cost_c == cost_b && L.nb[c] > L.nb[b])) { bi = c; bj = b; }
            if (L.nb[bi] == 0 || L.nb[bj] == 0) continue;   // an empty box adds nothing either way
            pairs_list.push_back(Pair{bi, bj});
        }
    }
    // rows per receiving box
    std::vector<int32_t> ru(nb, 0), rh(nb, 0);
    for (const Pair& pr : pairs_list) {
        const int ni = L.nb[pr.bi], ki = L.kb[pr.bi], kj = L.kb[pr.bj];
        if (pr.bi == pr.bj) {   // forward row and reverse row
            ru[pr.bi] += 2;
            if (ki > 0) rh[pr.bi] += 2;
            continue;
        }
        ru[pr.bi] += 1;
        if (ki > 0) rh[pr.bi] += 1;
        for (int t0 = 0; t0 < ni; t0 += group) {
            ru[pr.bj] += 1;
            if (t0 < ki && kj > 0) rh[pr.bj] += 1;
        }
    }
    std::vector<int64_t> base_u(nb, 0), base_h(nb, 0);
    int64_t slot = 0;
    L.sym_rows.clear();
    for (int b = 0; b < nb; ++b) {
        base_u[b] = slot;
        slot += int64_t(ru[b]) * L.nb[b];
        base_h[b] = slot;
        slot += int64_t(rh[b]) * L.kb[b];
        if (ru[b] > 0 || rh[b] > 0) L.sym_rows.push_back(SymRows{b, ru[b], rh[b], 0, base_u[b], base_h[b]});
    }
    L.slot_size = slot;
    // items, rows assigned in pair order
    std::vector<int32_t> nu(nb, 0), nh(nb, 0);
    std::vector<std::pair<int64_t, SymTask>> items;
    for (const Pair& pr : pairs_list) {
        const int bi = pr.bi, bj = pr.bj;
        const int ni = L.nb[bi], nj = L.nb[bj], ki = L.kb[bi], kj = L.kb[bj];
        if (bi == bj) {
            SymTask st{bi, bi, 0, ni, 0, 0, base_u[bi] + int64_t(nu[bi]) * ni, -1,
                       base_u[bi] + int64_t(nu[bi] + 1) * ni, -1};
            nu[bi] += 2;
            if (ki > 0) {
                st.fwd_h = base_h[bi] + int64_t(nh[bi]) * ki;
                st.rev_h = base_h[bi] + int64_t(nh[bi] + 1) * ki;
                nh[bi] += 2;
            }
            // about half the block is evaluated; the reverse sums make it dearer per pair
            items.push_back({int64_t(ni) * ni * 5 / 8, st});
            continue;
        }
        const int64_t row_u = base_u[bi] + int64_t(nu[bi]++) * ni;
        const int64_t row_h = ki > 0 ? base_h[bi] + int64_t(nh[bi]++) * ki : -1;
        for (int t0 = 0; t0 < ni; t0 += group) {
            const int t1 = std::min(ni, t0 + group);
            SymTask st{bi, bj, t0, t1, sym_flags(L, bi, bj), 0, row_u + t0, -1,
                       base_u[bj] + int64_t(nu[bj]++) * nj, -1};
            if (t0 < ki) st.fwd_h = row_h + t0;
            if (t0 < ki && kj > 0) st.rev_h = base_h[bj] + int64_t(nh[bj]++) * kj;
            items.push_back({int64_t(t1 - t0) * nj, st});
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    L.sym_tasks.clear();
    for (auto& it : items) L.sym_tasks.push_back(it.second);
    // every slot a kernel or the reduction touches lies inside the slot array,
    // and every row is filled exactly once per sweep
    for (int b = 0; b < nb; ++b)
        if (nu[b] != ru[b] || nh[b] != rh[b]) throw std::logic_error("symmetric row count mismatch");
    for (const SymTask& st : L.sym_tasks) {
        const int ni = L.nb[st.bi], nj = L.nb[st.bj], ki = L.kb[st.bi], kj = L.kb[st.bj];
        const bool hrow = st.t0 < ki, hrev = st.t0 < ki && kj > 0;
        if ((st.bi == st.bj && (st.t0 != 0 || st.t1 != ni)) || st.t0 < 0 || st.t1 > ni || st.t0 >= st.t1 ||
            nj <= 0 ||
            st.fwd_u < base_u[st.bi] || st.fwd_u + (st.t1 - st.t0) > base_u[st.bi] + int64_t(ru[st.bi]) * ni ||
            (hrow && (st.fwd_h < base_h[st.bi] ||
                      st.fwd_h + (std::min(ki, st.t1) - st.t0) > base_h[st.bi] + int64_t(rh[st.bi]) * ki)) ||
            st.rev_u < base_u[st.bj] || st.rev_u + nj > base_u[st.bj] + int64_t(ru[st.bj]) * nj ||
            (hrev && (st.rev_h < base_h[st.bj] || st.rev_h + kj > base_h[st.bj] + int64_t(rh[st.bj]) * kj)) ||
            st.rev_u + nj > slot || (hrev && st.rev_h + kj > slot))
            throw std::logic_error("symmetric work item out of range");
    }
    L.seg_ptr_ns.assign(nb + 1, 0);
    L.seg_src_ns.clear();
    L.seg_mode_ns.clear();
    for (int b = 0; b < nb; ++b) {
        L.seg_src_ns.insert(L.seg_src_ns.end(), rem[b].begin(), rem[b].end());
        L.seg_mode_ns.insert(L.seg_mode_ns.end(), remm[b].begin(), remm[b].end());
        L.seg_ptr_ns[b + 1] = static_cast<int32_t>(L.seg_src_ns.size());
    }
}

void sym_pair_counts(const Layout& L, int tpl, int64_t out[4]) {
    out[0] = out[1] = out[2] = out[3] = 0;
    for (const SymTask& st : L.sym_tasks) {
        const int64_t ni = L.nb[st.bi], nj = L.nb[st.bj], ki = L.kb[st.bi], kj = L.kb[st.bj];
        if (st.bi != st.bj) {
            out[0] += int64_t(st.t1 - st.t0) * nj;
            out[1] += std::max<int64_t>(0, std::min<int64_t>(ki, st.t1) - st.t0) * kj;
            continue;
        }
        // passes of 64 tpl targets while more remain, then one pass over the
        // rest; the diagonal tiles run in one direction, the rest of the block
        // in both
        int64_t d = 0, dk = 0;
        for (int64_t tp = 0; tp < ni;) {
            const int64_t e = ni - tp > 64 * tpl ? tp + 64 * tpl : ni;
            d += (e - tp) * (e - tp);
            const int64_t ek = std::max<int64_t>(0, std::min(e, ki) - tp);
            dk += ek * ek;
            tp = e;
        }
        out[0] += (ni * ni - d) / 2;
        out[1] += (ki * ki - dk) / 2;
        out[2] += d;
        out[3] += dk;
    }
}

Layout merge_layouts(const std::vector<const Layout*>& ls, std::vector<int64_t>& entry_base) {
    Layout M;
    const Layout& L0 = *ls[0];
    M.dim = L0.dim;
    M.kind = L0.kind;
    M.kappa = L0.kappa;
    M.tile = L0.tile;
    M.top = L0.top;
    const int nops = static_cast<int>(ls.size());
    std::vector<int> box_base(nops + 1, 0);
    std::vector<int64_t> hbase(nops + 1, 0), tbase(nops + 1, 0);
    entry_base.assign(nops + 1, 0);
    for (int i = 0; i < nops; ++i) {
        const Layout& L = *ls[i];
        if (L.dim != M.dim || L.kind != M.kind || L.kappa != M.kappa)
            throw std::invalid_argument("batched operators must share kernel, dimension and wavenumber");
        box_base[i + 1] = box_base[i] + L.n_boxes;
        entry_base[i + 1] = entry_base[i] + L.n_entries;
        hbase[i + 1] = hbase[i] + L.n_hentries;
        tbase[i + 1] = tbase[i] + static_cast<int64_t>(L.Tvec().size());
        M.n_points += L.n_points;
        M.max_level = std::max(M.max_level, L.max_level);
        M.top = std::min(M.top, L.top);
        M.pairs_near += L.pairs_near;
        M.pairs_skel += L.pairs_skel;
    }
    M.n_boxes = box_base[nops];
    M.n_entries = entry_base[nops];
    M.n_hentries = hbase[nops];
    if (M.n_entries >= (int64_t(1) << 31)) throw std::runtime_error("too many entries for 32-bit maps");
    // merged numbering: by level, then operator, then the operator's own order
    std::vector<std::pair<int, int>> owner(M.n_boxes);   // merged id -> (op, local id)
    std::vector<std::vector<int>> newid(nops);
    {
        std::vector<std::tuple<int, int, int>> keys;
        keys.reserve(M.n_boxes);
        for (int i = 0; i < nops; ++i)
            for (int b = 0; b < ls[i]->n_boxes; ++b) keys.emplace_back(ls[i]->level[b], i, b);
        std::sort(keys.begin(), keys.end());
        for (int i = 0; i < nops; ++i) newid[i].assign(ls[i]->n_boxes, -1);
        M.level_ptr.assign(M.max_level + 2, 0);
        for (int g = 0; g < M.n_boxes; ++g) {
            const auto [lev, i, b] = keys[g];
            owner[g] = {i, b};
            newid[i][b] = g;
            M.level_ptr[lev + 1]++;
        }
        for (int l = 0; l <= M.max_level; ++l) M.level_ptr[l + 1] += M.level_ptr[l];
    }
    M.voff.resize(M.n_boxes); M.hoff.resize(M.n_boxes); M.toff.resize(M.n_boxes);
    M.dmin.resize(M.n_boxes); M.brad.resize(M.n_boxes); M.bcenter.resize(static_cast<size_t>(M.n_boxes) * 3);
    M.nb.resize(M.n_boxes); M.kb.resize(M.n_boxes); M.level.resize(M.n_boxes);
    M.parent.resize(M.n_boxes); M.is_leaf.resize(M.n_boxes);
    M.seg_ptr.assign(M.n_boxes + 1, 0);
    for (int g = 0; g < M.n_boxes; ++g) {
        const auto [i, b] = owner[g];
        const Layout& L = *ls[i];
        M.voff[g] = L.voff[b] + entry_base[i];
        M.hoff[g] = L.hoff[b] + hbase[i];
        M.toff[g] = L.toff[b] + tbase[i];
        M.nb[g] = L.nb[b];
        M.kb[g] = L.kb[b];
        M.dmin[g] = L.dmin.empty() ? 0.0 : L.dmin[b];
        M.brad[g] = L.brad.empty() ? 0.0 : L.brad[b];
        // centres stay in the operator's own frame, like its entry coordinates
        for (int d = 0; d < 3; ++d) M.bcenter[3 * g + d] = L.bcenter.empty() ? 0.0 : L.bcenter[3 * b + d];
        M.level[g] = L.level[b];
        M.parent[g] = L.parent[b] < 0 ? -1 : newid[i][L.parent[b]];
        M.is_leaf[g] = L.is_leaf[b];
        for (int x = L.seg_ptr[b]; x < L.seg_ptr[b + 1]; ++x) {
            M.seg_src.push_back(newid[i][L.seg_src[x]]);
            M.seg_mode.push_back(L.seg_mode[x]);
        }
        M.seg_ptr[g + 1] = static_cast<int32_t>(M.seg_src.size());
    }
    // per-entry and per-skeleton-entry arrays, concatenated in operator order
    M.X.reserve(static_cast<size_t>(M.n_entries) * 4);
    M.perm.reserve(M.n_entries);
    M.pmap.reserve(M.n_hentries);
    M.T.reserve(tbase[nops]);
    for (int i = 0; i < nops; ++i) {
        const Layout& L = *ls[i];
        M.X.insert(M.X.end(), L.X.begin(), L.X.end());
        M.perm.insert(M.perm.end(), L.perm.begin(), L.perm.end());
        for (int32_t v : L.pmap) M.pmap.push_back(static_cast<int32_t>(v + entry_base[i]));
        M.T.insert(M.T.end(), L.Tvec().begin(), L.Tvec().end());
        for (size_t j = 0; j < L.gather_e.size(); ++j) {
            M.gather_e.push_back(static_cast<int32_t>(L.gather_e[j] + entry_base[i]));
            M.gather_p.push_back(L.gather_p[j]);
        }
    }
    pad_transfer_offsets(M);
    M.tasks = make_tasks(M, M.tile);
    return M;
}

void pad_transfer_offsets(Layout& L) {
    L.tpad.assign(L.n_boxes, 0);
    L.ttpad.assign(L.n_boxes, 0);
    int64_t a = 0, b = 0;
    for (int i = 0; i < L.n_boxes; ++i) {
        const int64_t k = L.kb[i], m = L.nb[i] - L.kb[i];
        L.tpad[i] = a;
        L.ttpad[i] = b;
        if (k > 0 && m > 0) {
            a += pad_ld(k) * m;
            b += pad_ld(m) * k;
        }
    }
    L.tpad_size = a;
    L.ttpad_size = b;
}

std::vector<Task> make_tasks(const Layout& L, int tile, bool ns) {
    const std::vector<int32_t>& sp = ns ? L.seg_ptr_ns : L.seg_ptr;
    const std::vector<int32_t>& ss = ns ? L.seg_src_ns : L.seg_src;
    std::vector<std::pair<int64_t, Task>> work;
    for (int b = 0; b < L.n_boxes; ++b) {
        if (L.level[b] < L.top || L.nb[b] == 0) continue;
        int64_t src = 0;
        for (int x = sp[b]; x < sp[b + 1]; ++x) src += L.nb[ss[x]];
        for (int t0 = 0; t0 < L.nb[b]; t0 += tile) work.push_back({int64_t(tile) * src + 64, Task{b, t0}});
    }
    std::stable_sort(work.begin(), work.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    std::vector<Task> tasks;
    tasks.reserve(work.size());
    for (auto& w : work) tasks.push_back(w.second);
    return tasks;
}

}  // namespace skelfmm
