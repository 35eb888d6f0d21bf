// Adaptive 2^d-tree with strong 2:1 balance and the three neighbor relations
// the apply needs (section 3, "Adaptive tree data structure").
//
//  * root: a cube around the bounding box; a box with more than b points is
//    split into 2^d equal children, empty children are pruned;
//  * balance: a leaf adjacent to an existing box two or more levels finer is
//    split, repeated until stable (the paper balances adjacent leaves; the
//    stronger rule also keeps a leaf from touching a non-empty box far below);
//  * colleagues: boxes of the same level whose closed cubes touch, self included;
//  * coarse neighbors of B: leaves one level up that touch B itself;
//  * fine neighbors of a leaf: boxes one level down that touch it (inverse).
// Morton keys give the geometric lookups.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <unordered_map>

#include "parallel.h"
#include "plan.h"

namespace skelfmm {

namespace {

inline uint64_t spread3(uint64_t x) {   // 21 bits -> every third bit
    x &= 0x1fffffULL;
    x = (x | (x << 32)) & 0x1f00000000ffffULL;
    x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
    x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
    x = (x | (x << 2)) & 0x1249249249249249ULL;
    return x;
}
inline uint64_t spread2(uint64_t x) {   // 32 bits -> every second bit
    x &= 0xffffffffULL;
    x = (x | (x << 16)) & 0x0000ffff0000ffffULL;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffULL;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    x = (x | (x << 2)) & 0x3333333333333333ULL;
    x = (x | (x << 1)) & 0x5555555555555555ULL;
    return x;
}
inline uint64_t morton(int dim, const int32_t* c) {
    if (dim == 3) return spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
    return spread2(c[0]) | (spread2(c[1]) << 1);
}
// Unique key across levels: a leading 1 bit above the level's Morton code.
inline uint64_t box_key(int dim, int lev, const int32_t* c) {
    return (1ULL << (dim * lev)) | morton(dim, c);
}

struct TBox {
    int level;
    int32_t c[3];
    int64_t b, e;          // range in the Morton-sorted point order
    int leaf;
    int parent;
    int kids[8];
    int nkids;
};

struct Builder {
    Plan& p;
    int D;
    std::vector<uint64_t> pkey;        // Morton key of each sorted point at depth D
    std::vector<int64_t> order;        // sorted position -> user index
    std::vector<TBox> boxes;
    std::unordered_map<uint64_t, int> lookup;

    explicit Builder(Plan& plan) : p(plan), D(plan.opt.max_depth) {}

    int find(int lev, const int32_t* c) const {
        const int32_t lim = 1 << lev;
        for (int d = 0; d < p.dim; ++d)
            if (c[d] < 0 || c[d] >= lim) return -1;
        auto it = lookup.find(box_key(p.dim, lev, c));
        return it == lookup.end() ? -1 : it->second;
    }

    int add_box(int lev, const int32_t* c, int64_t b, int64_t e, int parent) {
        TBox t;
        t.level = lev;
        for (int d = 0; d < 3; ++d) t.c[d] = d < p.dim ? c[d] : 0;
        t.b = b; t.e = e; t.leaf = 1; t.parent = parent; t.nkids = 0;
        boxes.push_back(t);
        int id = static_cast<int>(boxes.size()) - 1;
        lookup[box_key(p.dim, lev, t.c)] = id;
        return id;
    }

    // Split box `id` into its non-empty children (Morton order).
    void split(int id) {
        const int lev = boxes[id].level;
        const int shift = p.dim * (D - lev - 1);
        const uint64_t mask = (1ULL << p.dim) - 1;
        int64_t s = boxes[id].b;
        const int64_t e = boxes[id].e;
        int32_t pc[3] = {boxes[id].c[0], boxes[id].c[1], boxes[id].c[2]};
        boxes[id].leaf = 0;
        while (s < e) {
            const uint64_t ch = (pkey[s] >> shift) & mask;
            int64_t t = s;
            while (t < e && ((pkey[t] >> shift) & mask) == ch) ++t;
            int32_t cc[3] = {0, 0, 0};
            for (int d = 0; d < p.dim; ++d) cc[d] = 2 * pc[d] + static_cast<int32_t>((ch >> d) & 1);
            int kid = add_box(lev + 1, cc, s, t, id);
            boxes[id].kids[boxes[id].nkids++] = kid;
            s = t;
        }
    }

    void build_unbalanced() {
        const int64_t n = p.n;
        const int dim = p.dim;
        double lo[3], hi[3];
        for (int d = 0; d < dim; ++d) { lo[d] = INFINITY; hi[d] = -INFINITY; }
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < dim; ++d) {
                const double x = p.pts[i * dim + d];
                if (!std::isfinite(x)) throw std::invalid_argument("point coordinates must be finite");
                lo[d] = std::min(lo[d], x);
                hi[d] = std::max(hi[d], x);
            }
        double ext = 0.0;
        for (int d = 0; d < dim; ++d) ext = std::max(ext, hi[d] - lo[d]);
        double side = ext > 0.0 ? ext * (1.0 + std::ldexp(1.0, -40)) : 1.0;
        for (int d = 0; d < 3; ++d) p.root_lo[d] = 0.0;
        for (int d = 0; d < dim; ++d) p.root_lo[d] = 0.5 * (lo[d] + hi[d]) - 0.5 * side;
        p.root_side = side;

        // quantize to the depth-D grid and sort by Morton key (ties by user index)
        const double scale = std::ldexp(1.0, D) / side;
        const int32_t cmax = (1 << D) - 1;
        std::vector<std::pair<uint64_t, int64_t>> kv(n);
        const int threads = host_threads(p.opt.num_threads);
        parallel_for(n, threads, [&](int64_t i) {
            int32_t c[3] = {0, 0, 0};
            for (int d = 0; d < dim; ++d) {
                double f = std::floor((p.pts[i * dim + d] - p.root_lo[d]) * scale);
                c[d] = static_cast<int32_t>(std::min<double>(std::max<double>(f, 0.0), cmax));
            }
            kv[i] = {morton(dim, c), i};
        }, 4096);
        // sorted runs in parallel, then merged pairwise (the order is total: the
        // user index breaks ties, so the result is that of one sort)
        const int64_t runs = std::max<int64_t>(1, std::min<int64_t>(threads, n / 65536));
        std::vector<int64_t> bnd(runs + 1);
        for (int64_t r = 0; r <= runs; ++r) bnd[r] = n * r / runs;
        parallel_for(runs, threads, [&](int64_t r) { std::sort(kv.begin() + bnd[r], kv.begin() + bnd[r + 1]); });
        for (int64_t width = 1; width < runs; width *= 2) {
            const int64_t pairs = (runs + 2 * width - 1) / (2 * width);
            parallel_for(pairs, threads, [&](int64_t q) {
                const int64_t a = 2 * width * q, m = std::min(a + width, runs), e = std::min(a + 2 * width, runs);
                if (m < e) std::inplace_merge(kv.begin() + bnd[a], kv.begin() + bnd[m], kv.begin() + bnd[e]);
            });
        }
        pkey.resize(n);
        order.resize(n);
        for (int64_t i = 0; i < n; ++i) { pkey[i] = kv[i].first; order[i] = kv[i].second; }

        int32_t zero[3] = {0, 0, 0};
        boxes.reserve(static_cast<size_t>(4 * (n / std::max(1, p.leaf_size) + 8)));
        add_box(0, zero, 0, n, -1);
        for (size_t i = 0; i < boxes.size(); ++i) {
            if (boxes[i].e - boxes[i].b > p.leaf_size && boxes[i].level < D) split(static_cast<int>(i));
        }
    }

    // Split every leaf that touches an existing box two or more levels finer.
    void balance() {
        const int dim = p.dim;
        const int noff = dim == 3 ? 27 : 9;
        for (;;) {
            std::vector<char> mark(boxes.size(), 0);
            bool any = false;
            const size_t nb = boxes.size();
            for (size_t i = 0; i < nb; ++i) {
                const TBox& B = boxes[i];
                if (B.level < 2) continue;
                for (int o = 0; o < noff; ++o) {
                    int32_t off[3] = {o % 3 - 1, (o / 3) % 3 - 1, (o / 9) % 3 - 1};
                    if (dim == 2) off[2] = 0;
                    if (off[0] == 0 && off[1] == 0 && off[2] == 0) continue;
                    int32_t c[3] = {0, 0, 0};
                    bool inside = true;
                    for (int d = 0; d < dim; ++d) {
                        c[d] = B.c[d] + off[d];
                        if (c[d] < 0 || c[d] >= (1 << B.level)) inside = false;
                    }
                    if (!inside) continue;
                    // deepest existing box containing that cell, at level <= B.level - 1
                    for (int lev = B.level - 1; lev >= 0; --lev) {
                        int32_t a[3] = {0, 0, 0};
                        for (int d = 0; d < dim; ++d) a[d] = c[d] >> (B.level - lev);
                        int id = find(lev, a);
                        if (id < 0) continue;
                        if (boxes[id].leaf && lev <= B.level - 2 && !mark[id]) { mark[id] = 1; any = true; }
                        break;
                    }
                }
            }
            if (!any) break;
            for (size_t i = 0; i < mark.size(); ++i)
                if (mark[i]) split(static_cast<int>(i));
        }
    }

    // Renumber level by level (Morton order inside a level) and fill the plan.
    void emit() {
        const int dim = p.dim;
        const int nb = static_cast<int>(boxes.size());
        int L = 0;
        for (auto& b : boxes) L = std::max(L, b.level);
        std::vector<int> ids(nb);
        for (int i = 0; i < nb; ++i) ids[i] = i;
        std::sort(ids.begin(), ids.end(), [&](int a, int b) {
            if (boxes[a].level != boxes[b].level) return boxes[a].level < boxes[b].level;
            return morton(dim, boxes[a].c) < morton(dim, boxes[b].c);
        });
        std::vector<int> newid(nb);
        for (int i = 0; i < nb; ++i) newid[ids[i]] = i;

        p.n_boxes = nb;
        p.max_level = L;
        p.level_ptr.assign(L + 2, 0);
        p.level.resize(nb); p.parent.resize(nb); p.is_leaf.resize(nb);
        p.coord.assign(static_cast<size_t>(nb) * 3, 0);
        p.child_ptr.assign(nb + 1, 0);
        p.child_idx.clear();
        for (int i = 0; i < nb; ++i) {
            const TBox& B = boxes[ids[i]];
            p.level[i] = B.level;
            p.parent[i] = B.parent < 0 ? -1 : newid[B.parent];
            p.is_leaf[i] = B.leaf;
            for (int d = 0; d < 3; ++d) p.coord[3 * i + d] = B.c[d];
            p.level_ptr[B.level + 1]++;
            std::vector<int> kids(B.kids, B.kids + B.nkids);
            for (auto& k : kids) k = newid[k];
            std::sort(kids.begin(), kids.end());
            for (int k : kids) p.child_idx.push_back(k);
            p.child_ptr[i + 1] = static_cast<int32_t>(p.child_idx.size());
        }
        for (int l = 0; l <= L; ++l) p.level_ptr[l + 1] += p.level_ptr[l];
        p.top_level = p.is_leaf[0] ? 0 : 1;

        // rebuild the lookup under the new numbering
        lookup.clear();
        for (int i = 0; i < nb; ++i) lookup[box_key(dim, p.level[i], &p.coord[3 * i])] = i;

        // leaf point lists (Morton-sorted order inside a leaf)
        leaf_range.assign(static_cast<size_t>(nb) * 2, 0);
        for (int i = 0; i < nb; ++i) {
            leaf_range[2 * i] = boxes[ids[i]].b;
            leaf_range[2 * i + 1] = boxes[ids[i]].e;
        }
    }

    std::vector<int64_t> leaf_range;

    void neighbors() {
        const int dim = p.dim;
        const int nb = p.n_boxes;
        const int noff = dim == 3 ? 27 : 9;
        std::vector<std::vector<int32_t>> coll(nb), coarse(nb), fine(nb);
        for (int i = 0; i < nb; ++i) {
            const int lev = p.level[i];
            const int32_t* c0 = &p.coord[3 * i];
            for (int o = 0; o < noff; ++o) {
                int32_t off[3] = {o % 3 - 1, (o / 3) % 3 - 1, (o / 9) % 3 - 1};
                if (dim == 2) off[2] = 0;
                int32_t c[3] = {0, 0, 0};
                for (int d = 0; d < dim; ++d) c[d] = c0[d] + off[d];
                int j = find(lev, c);
                if (j >= 0) coll[i].push_back(j);
                const bool self = off[0] == 0 && off[1] == 0 && off[2] == 0;
                if (self || lev == 0 || j >= 0) continue;
                // the cell holds no box of this level: a leaf one level up may cover it
                bool inside = true;
                for (int d = 0; d < dim; ++d) if (c[d] < 0 || c[d] >= (1 << lev)) inside = false;
                if (!inside) continue;
                int32_t a[3] = {0, 0, 0};
                for (int d = 0; d < dim; ++d) a[d] = c[d] >> 1;
                int L1 = find(lev - 1, a);
                if (L1 >= 0 && p.is_leaf[L1]) coarse[i].push_back(L1);
            }
            std::sort(coll[i].begin(), coll[i].end());
            std::sort(coarse[i].begin(), coarse[i].end());
            coarse[i].erase(std::unique(coarse[i].begin(), coarse[i].end()), coarse[i].end());
        }
        for (int i = 0; i < nb; ++i)
            for (int L1 : coarse[i]) fine[L1].push_back(i);
        auto to_csr = [&](std::vector<std::vector<int32_t>>& v, std::vector<int32_t>& ptr, std::vector<int32_t>& ix) {
            ptr.assign(nb + 1, 0);
            ix.clear();
            for (int i = 0; i < nb; ++i) {
                std::sort(v[i].begin(), v[i].end());
                ix.insert(ix.end(), v[i].begin(), v[i].end());
                ptr[i + 1] = static_cast<int32_t>(ix.size());
            }
        };
        to_csr(coll, p.coll_ptr, p.coll_idx);
        to_csr(coarse, p.coarse_ptr, p.coarse_idx);
        to_csr(fine, p.fine_ptr, p.fine_idx);
    }
};

}  // namespace

// Implemented in skel.cpp.
void skeletonize(Plan& p, const std::vector<int64_t>& order, const std::vector<int64_t>& leaf_range);

void build_plan(Plan& p) {
    if (p.dim != 2 && p.dim != 3) throw std::invalid_argument("dim must be 2 or 3");
    if (p.kind != 0 && p.kind != 1) throw std::invalid_argument("unknown kernel kind");
    if (p.kind == 1 && !(p.kappa >= 0.0 && std::isfinite(p.kappa))) throw std::invalid_argument("kappa must be >= 0");
    if (p.n <= 0) throw std::invalid_argument("n must be positive");
    if (!(p.tol > 0.0 && p.tol < 1.0)) throw std::invalid_argument("tol must be in (0, 1)");
    if (p.leaf_size < 1) throw std::invalid_argument("leaf_size must be >= 1");
    const int dmax = p.dim == 3 ? 20 : 30;
    if (p.opt.max_depth <= 0 || p.opt.max_depth > dmax) p.opt.max_depth = std::min(20, dmax);

    auto t0 = std::chrono::steady_clock::now();
    Builder B(p);
    B.build_unbalanced();
    B.balance();
    B.emit();
    B.neighbors();
    auto t1 = std::chrono::steady_clock::now();
    p.t_tree = std::chrono::duration<double>(t1 - t0).count();
    skeletonize(p, B.order, B.leaf_range);
    p.t_skel = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
}

}  // namespace skelfmm
