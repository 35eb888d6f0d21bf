/*
 * ORACLE -- test infrastructure only.  Nothing in the library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source with the library: it receives the
 * skeleton operators (tree, index sets, skeleton positions, interpolation
 * matrices, neighbor lists) as plain arrays and applies them its own way.
 *
 * O2: CPU float64 apply of given skeleton operators, following the FMM apply
 * of section 3 (Algorithm "FMM apply", equations (15)-(20) and the adaptive
 * terms after them) in the paper's order:
 *   leaves take their charges; upward pass l = L..1 (concatenate children's
 *   outgoing skeleton charges, then qhat = [I T] q); translations ifo, ifs,
 *   tfo; all pairs on the top level; downward pass l = 2..L
 *   (uhat += parent's potential at this box's slots, u += [I; T^*] uhat);
 *   leaves give the result.
 * Readings taken where the paper is loose:
 *   - the colleague list of a box contains the box itself;
 *   - ifo / ifs and uhat exist only below the top level (level >= 2 when the
 *     root has children); the top level is handled by the direct step alone;
 *   - the downward pass adds to a child's uhat the slice of the parent's u at
 *     the positions the child's skeleton occupies in the parent's index set;
 *   - a coarse neighbor of B is a leaf one level up adjacent to B itself;
 *     fine neighbors are the inverse relation.
 * A kernel entry is zero where the two original point indices coincide, or
 * where two distinct points sit at distance zero.
 *
 * O2T: the literal transpose of every step above in reverse order, giving
 * w = Atilde^H v for the same operators (each step's adjoint: gathers become
 * scatters, [I T] becomes [I; T^H], kernel blocks become conjugate
 * transposes).  Parity of the transpose is pinned by the dense matrix form.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define O_PI 3.14159265358979323846

void oracle_h0(double x, double* j0, double* y0);   /* hankel.c */

typedef struct {
    int32_t dim, kind;          /* kind 0 Laplace, 1 Helmholtz */
    double kappa;
    int64_t n_points;
    const double* pts;          /* n_points x dim */
    int32_t n_boxes, top_level, max_level;
    const int32_t *level, *parent, *is_leaf, *child_ptr, *child_idx;
    const int64_t *idx_ptr, *idx, *pos;   /* per box: natural-order point list; pos = [sk | rd] */
    const int32_t *rank;                  /* k per box (< 0 where not skeletonized) */
    const int64_t *T_ptr;
    const double  *T;                     /* column-major k x (n - k) per box */
    const int32_t *coll_ptr, *coll_idx, *coarse_ptr, *coarse_idx, *fine_ptr, *fine_idx;
} o2_plan;

typedef struct {
    int W;            /* doubles per point value: nrhs (real) or 2 nrhs (complex) */
    int nrhs, cplx;
    double **qb, **qh, **ub, **uh;
} o2_state;

static int64_t nb_of(const o2_plan* P, int b) { return P->idx_ptr[b + 1] - P->idx_ptr[b]; }
static int kb_of(const o2_plan* P, int b) { return P->rank[b]; }

/* Kernel value G(x_i, x_j) (section 2); returns 0 when excluded. */
static inline void kernel_value(const o2_plan* P, int64_t i, int64_t j, int conj,
                                double* gr, double* gi)
{
    *gr = 0.0; *gi = 0.0;
    if (i == j) return;
    const double* a = P->pts + i * P->dim;
    const double* b = P->pts + j * P->dim;
    double s = 0.0;
    for (int d = 0; d < P->dim; ++d) { double t = a[d] - b[d]; s += t * t; }
    const double r = sqrt(s);
    if (r == 0.0) return;
    if (P->kind == 0) {
        *gr = (P->dim == 2) ? -log(r) / (2.0 * O_PI) : 1.0 / (4.0 * O_PI * r);
    } else {
        if (P->dim == 3) {
            *gr = cos(P->kappa * r) / (4.0 * O_PI * r);
            *gi = sin(P->kappa * r) / (4.0 * O_PI * r);
        } else {
            /* (i/4) H0^(1)(kappa r) = (i/4)(J0 + i Y0) */
            double j0, y0;
            oracle_h0(P->kappa * r, &j0, &y0);
            *gr = -0.25 * y0;
            *gi = 0.25 * j0;
        }
        if (conj) *gi = -*gi;
    }
}

/* ut[a] += sign * sum_b G(x_ti[a], x_si[b]) ws[b]   (a kernel block times a vector) */
static void gblock(const o2_plan* P, const o2_state* S, int conj,
                   int64_t nt, const int64_t* ti, int64_t ns, const int64_t* si,
                   const double* ws, double sign, double* ut)
{
    const int W = S->W;
    for (int64_t a = 0; a < nt; ++a) {
        double* ua = ut + a * W;
        for (int64_t b = 0; b < ns; ++b) {
            double gr, gi;
            kernel_value(P, ti[a], si[b], conj, &gr, &gi);
            if (gr == 0.0 && gi == 0.0) continue;
            const double* wb = ws + b * W;
            if (!S->cplx) {
                for (int c = 0; c < W; ++c) ua[c] += sign * gr * wb[c];
            } else {
                for (int c = 0; c < S->nrhs; ++c) {
                    const double x = wb[2 * c], y = wb[2 * c + 1];
                    ua[2 * c]     += sign * (gr * x - gi * y);
                    ua[2 * c + 1] += sign * (gr * y + gi * x);
                }
            }
        }
    }
}

/* Original point indices of a box's natural order, and of its skeleton. */
static const int64_t* box_idx(const o2_plan* P, int b) { return P->idx + P->idx_ptr[b]; }
static int64_t* skel_idx(const o2_plan* P, int b)
{
    const int k = kb_of(P, b);
    int64_t* s = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
    const int64_t* pos = P->pos + P->idx_ptr[b];
    for (int i = 0; i < k; ++i) s[i] = box_idx(P, b)[pos[i]];
    return s;
}

/* Offset of child c's skeleton block inside its parent's concatenated index set. */
static int64_t child_slot(const o2_plan* P, int c)
{
    const int p = P->parent[c];
    int64_t off = 0;
    for (int32_t e = P->child_ptr[p]; e < P->child_ptr[p + 1]; ++e) {
        const int ch = P->child_idx[e];
        if (ch == c) return off;
        off += kb_of(P, ch);
    }
    return -1;
}

static int alloc_state(const o2_plan* P, o2_state* S)
{
    const int nb = P->n_boxes;
    S->qb = (double**)calloc((size_t)nb, sizeof(double*));
    S->qh = (double**)calloc((size_t)nb, sizeof(double*));
    S->ub = (double**)calloc((size_t)nb, sizeof(double*));
    S->uh = (double**)calloc((size_t)nb, sizeof(double*));
    if (!S->qb || !S->qh || !S->ub || !S->uh) return -1;
    for (int b = 0; b < nb; ++b) {
        const int64_t n = nb_of(P, b);
        const int k = kb_of(P, b) > 0 ? kb_of(P, b) : 0;
        S->qb[b] = (double*)calloc((size_t)(n * S->W + 1), sizeof(double));
        S->ub[b] = (double*)calloc((size_t)(n * S->W + 1), sizeof(double));
        S->qh[b] = (double*)calloc((size_t)(k * S->W + 1), sizeof(double));
        S->uh[b] = (double*)calloc((size_t)(k * S->W + 1), sizeof(double));
        if (!S->qb[b] || !S->ub[b] || !S->qh[b] || !S->uh[b]) return -1;
    }
    return 0;
}

static void free_state(const o2_plan* P, o2_state* S)
{
    for (int b = 0; b < P->n_boxes; ++b) {
        if (S->qb) free(S->qb[b]);
        if (S->qh) free(S->qh[b]);
        if (S->ub) free(S->ub[b]);
        if (S->uh) free(S->uh[b]);
    }
    free(S->qb); free(S->qh); free(S->ub); free(S->uh);
}

/* The index set of a tree box must be its children's skeletons, concatenated. */
static int check_concat(const o2_plan* P)
{
    for (int b = 0; b < P->n_boxes; ++b) {
        if (P->is_leaf[b] || P->level[b] < P->top_level) continue;
        int64_t off = 0;
        const int64_t* ib = box_idx(P, b);
        for (int32_t e = P->child_ptr[b]; e < P->child_ptr[b + 1]; ++e) {
            const int c = P->child_idx[e];
            const int k = kb_of(P, c);
            const int64_t* pc = P->pos + P->idx_ptr[c];
            for (int i = 0; i < k; ++i)
                if (ib[off + i] != box_idx(P, c)[pc[i]]) return -2;
            off += k;
        }
        if (off != nb_of(P, b)) return -2;
    }
    return 0;
}

/* y = [I T] x : yh[i] = x[sk_i] + sum_j T(i,j) x[rd_j]      (equation (15)/(17)) */
static void apply_F(const o2_plan* P, int b, int W, const double* x, double* yh)
{
    const int64_t n = nb_of(P, b);
    const int k = kb_of(P, b);
    const int64_t* pos = P->pos + P->idx_ptr[b];
    const double* T = P->T + P->T_ptr[b];
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < W; ++c) yh[i * W + c] = x[pos[i] * W + c];
    for (int64_t j = 0; j < n - k; ++j)
        for (int i = 0; i < k; ++i) {
            const double t = T[i + j * (int64_t)k];
            for (int c = 0; c < W; ++c) yh[i * W + c] += t * x[pos[k + j] * W + c];
        }
}

/* x += [I; T^*] yh : x[sk_i] += yh[i];  x[rd_j] += sum_i T(i,j) yh[i]  (equation (20)) */
static void apply_E(const o2_plan* P, int b, int W, const double* yh, double* x)
{
    const int64_t n = nb_of(P, b);
    const int k = kb_of(P, b);
    const int64_t* pos = P->pos + P->idx_ptr[b];
    const double* T = P->T + P->T_ptr[b];
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < W; ++c) x[pos[i] * W + c] += yh[i * W + c];
    for (int64_t j = 0; j < n - k; ++j)
        for (int i = 0; i < k; ++i) {
            const double t = T[i + j * (int64_t)k];   /* T is real: T^* = T^T */
            for (int c = 0; c < W; ++c) x[pos[k + j] * W + c] += t * yh[i * W + c];
        }
}

static void forward(const o2_plan* P, o2_state* S, const double* q, double* u, const uint8_t* mask)
{
    const int W = S->W, nb = P->n_boxes, L = P->max_level, top = P->top_level;
    /* leaves take the given charges */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int b = 0; b < nb; ++b)
        if (P->is_leaf[b]) {
            const int64_t* ib = box_idx(P, b);
            for (int64_t a = 0; a < nb_of(P, b); ++a)
                memcpy(S->qb[b] + a * W, q + ib[a] * W, sizeof(double) * (size_t)W);
        }
    /* upward pass l = L .. top: concatenate children's qhat, then qhat = [I T] q */
    for (int l = L; l >= top; --l) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int b = 0; b < nb; ++b) {
            if (P->level[b] != l) continue;
            if (!P->is_leaf[b]) {
                int64_t off = 0;
                for (int32_t e = P->child_ptr[b]; e < P->child_ptr[b + 1]; ++e) {
                    const int c = P->child_idx[e];
                    memcpy(S->qb[b] + off * W, S->qh[c], sizeof(double) * (size_t)(kb_of(P, c) * W));
                    off += kb_of(P, c);
                }
            }
            if (l > top) apply_F(P, b, W, S->qb[b], S->qh[b]);
        }
    }
    /* translations; each target box owns its u and uhat */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        const int l = P->level[b];
        if (l < top || (mask && !mask[b])) continue;
        const int64_t nbb = nb_of(P, b);
        const int64_t* ib = box_idx(P, b);
        if (l > top) {
            int64_t* sb = skel_idx(P, b);
            const int kb = kb_of(P, b);
            /* ifo: u_b += A(B_b, B_c) q_c ; uhat_b -= A(S_b, S_c) qhat_c */
            for (int32_t e = P->coll_ptr[b]; e < P->coll_ptr[b + 1]; ++e) {
                const int c = P->coll_idx[e];
                int64_t* sc = skel_idx(P, c);
                gblock(P, S, 0, nbb, ib, nb_of(P, c), box_idx(P, c), S->qb[c], 1.0, S->ub[b]);
                gblock(P, S, 0, kb, sb, kb_of(P, c), sc, S->qh[c], -1.0, S->uh[b]);
                free(sc);
            }
            /* ifs: u_b += A(B_b, L) q_L ; uhat_b -= A(S_b, L) q_L */
            for (int32_t e = P->coarse_ptr[b]; e < P->coarse_ptr[b + 1]; ++e) {
                const int c = P->coarse_idx[e];
                gblock(P, S, 0, nbb, ib, nb_of(P, c), box_idx(P, c), S->qb[c], 1.0, S->ub[b]);
                gblock(P, S, 0, kb, sb, nb_of(P, c), box_idx(P, c), S->qb[c], -1.0, S->uh[b]);
            }
            free(sb);
        }
        /* tfo (leaves): u_L += A(L, B_c) q_c - A(L, S_c) qhat_c */
        if (P->is_leaf[b])
            for (int32_t e = P->fine_ptr[b]; e < P->fine_ptr[b + 1]; ++e) {
                const int c = P->fine_idx[e];
                int64_t* sc = skel_idx(P, c);
                gblock(P, S, 0, nbb, ib, nb_of(P, c), box_idx(P, c), S->qb[c], 1.0, S->ub[b]);
                gblock(P, S, 0, nbb, ib, kb_of(P, c), sc, S->qh[c], -1.0, S->ub[b]);
                free(sc);
            }
        /* top level: all pairs directly */
        if (l == top)
            for (int c = 0; c < nb; ++c)
                if (P->level[c] == top)
                    gblock(P, S, 0, nbb, ib, nb_of(P, c), box_idx(P, c), S->qb[c], 1.0, S->ub[b]);
    }
    /* downward pass l = top+1 .. L */
    for (int l = top + 1; l <= L; ++l) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int b = 0; b < nb; ++b) {
            if (P->level[b] != l) continue;
            const int64_t o = child_slot(P, b);
            const double* up = S->ub[P->parent[b]] + o * W;
            for (int64_t x = 0; x < (int64_t)kb_of(P, b) * W; ++x) S->uh[b][x] += up[x];
            apply_E(P, b, W, S->uh[b], S->ub[b]);
        }
    }
    /* leaves give the result */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int b = 0; b < nb; ++b)
        if (P->is_leaf[b]) {
            const int64_t* ib = box_idx(P, b);
            for (int64_t a = 0; a < nb_of(P, b); ++a)
                memcpy(u + ib[a] * W, S->ub[b] + a * W, sizeof(double) * (size_t)W);
        }
}

/* inverse of a CSR relation over boxes (for the transposed translations) */
static void invert_rel(int nb, const int32_t* ptr, const int32_t* ix, int32_t** optr, int32_t** oix)
{
    int32_t* cnt = (int32_t*)calloc((size_t)nb + 1, sizeof(int32_t));
    for (int b = 0; b < nb; ++b)
        for (int32_t e = ptr[b]; e < ptr[b + 1]; ++e) cnt[ix[e] + 1]++;
    for (int b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
    int32_t* out = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt[nb] + 1));
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb + 1);
    memcpy(fill, cnt, sizeof(int32_t) * (size_t)nb);
    for (int b = 0; b < nb; ++b)
        for (int32_t e = ptr[b]; e < ptr[b + 1]; ++e) out[fill[ix[e]]++] = b;
    free(fill);
    *optr = cnt; *oix = out;
}

/* w = Atilde^H v: the forward steps transposed and taken in reverse order.
 * Adjoint state: ub/uh hold ubar/uhbar, qb/qh hold qbar/qhbar. */
static void adjoint(const o2_plan* P, o2_state* S, const double* v, double* w)
{
    const int W = S->W, nb = P->n_boxes, L = P->max_level, top = P->top_level;
    /* transpose of "leaves give the result": ubar_L = v[I_L] */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int b = 0; b < nb; ++b)
        if (P->is_leaf[b]) {
            const int64_t* ib = box_idx(P, b);
            for (int64_t a = 0; a < nb_of(P, b); ++a)
                memcpy(S->ub[b] + a * W, v + ib[a] * W, sizeof(double) * (size_t)W);
        }
    /* transpose of the downward pass, l = L .. top+1:
     *   uhbar_b += [I; T^*]^H ubar_b  (= [I T] ubar_b, T real) ; ubar_parent[slot_b] += uhbar_b */
    for (int l = L; l > top; --l) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int b = 0; b < nb; ++b) {
            if (P->level[b] != l) continue;
            const int k = kb_of(P, b);
            double* tmp = (double*)calloc((size_t)(k * W + 1), sizeof(double));
            apply_F(P, b, W, S->ub[b], tmp);
            for (int64_t x = 0; x < (int64_t)k * W; ++x) S->uh[b][x] += tmp[x];
            free(tmp);
        }
        /* parents at l-1 are distinct from boxes at l: a serial scatter keeps it plain */
        for (int b = 0; b < nb; ++b) {
            if (P->level[b] != l) continue;
            const int64_t o = child_slot(P, b);
            double* up = S->ub[P->parent[b]] + o * W;
            for (int64_t x = 0; x < (int64_t)kb_of(P, b) * W; ++x) up[x] += S->uh[b][x];
        }
    }
    /* transposed translations: every forward term target <- source becomes
     * source <- target with the conjugate kernel; accumulate per receiving box */
    int32_t *cop, *coi, *fip, *fii;
    invert_rel(nb, P->coarse_ptr, P->coarse_idx, &cop, &coi);   /* leaf L -> boxes having L as coarse nbr */
    invert_rel(nb, P->fine_ptr, P->fine_idx, &fip, &fii);       /* box c -> leaves having c as fine nbr */
    int32_t *clp, *cli;
    invert_rel(nb, P->coll_ptr, P->coll_idx, &clp, &cli);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nb; ++c) {
        const int l = P->level[c];
        if (l < top) continue;
        const int64_t nc = nb_of(P, c);
        const int64_t* ic = box_idx(P, c);
        int64_t* sc = (l > top) ? skel_idx(P, c) : NULL;
        const int kc = (l > top) ? kb_of(P, c) : 0;
        /* ifo^T: qbar_c += A(B_b,B_c)^H ubar_b ; qhbar_c -= A(S_b,S_c)^H uhbar_b, for b with c in coll(b) */
        if (l > top)
            for (int32_t e = clp[c]; e < clp[c + 1]; ++e) {
                const int b = cli[e];
                int64_t* sb = skel_idx(P, b);
                gblock(P, S, 1, nc, ic, nb_of(P, b), box_idx(P, b), S->ub[b], 1.0, S->qb[c]);
                gblock(P, S, 1, kc, sc, kb_of(P, b), sb, S->uh[b], -1.0, S->qh[c]);
                free(sb);
            }
        /* ifs^T (c is a coarse leaf of b): qbar_c += A(B_b,c)^H ubar_b - A(S_b,c)^H uhbar_b */
        for (int32_t e = cop[c]; e < cop[c + 1]; ++e) {
            const int b = coi[e];
            int64_t* sb = skel_idx(P, b);
            gblock(P, S, 1, nc, ic, nb_of(P, b), box_idx(P, b), S->ub[b], 1.0, S->qb[c]);
            gblock(P, S, 1, nc, ic, kb_of(P, b), sb, S->uh[b], -1.0, S->qb[c]);
            free(sb);
        }
        /* tfo^T (c is a fine neighbor of leaf b): qbar_c += A(b,B_c)^H ubar_b ; qhbar_c -= A(b,S_c)^H ubar_b */
        for (int32_t e = fip[c]; e < fip[c + 1]; ++e) {
            const int b = fii[e];
            gblock(P, S, 1, nc, ic, nb_of(P, b), box_idx(P, b), S->ub[b], 1.0, S->qb[c]);
            gblock(P, S, 1, kc, sc, nb_of(P, b), box_idx(P, b), S->ub[b], -1.0, S->qh[c]);
        }
        /* top level direct^T */
        if (l == top)
            for (int b = 0; b < nb; ++b)
                if (P->level[b] == top)
                    gblock(P, S, 1, nc, ic, nb_of(P, b), box_idx(P, b), S->ub[b], 1.0, S->qb[c]);
        free(sc);
    }
    free(cop); free(coi); free(fip); free(fii); free(clp); free(cli);
    /* transpose of the upward pass, l = top .. L:
     *   qbar_b += [I T]^H qhbar_b ; then children take qhbar_c += qbar_b[slot_c] */
    for (int l = top; l <= L; ++l) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int b = 0; b < nb; ++b) {
            if (P->level[b] != l) continue;
            if (l > top) apply_E(P, b, W, S->qh[b], S->qb[b]);
            if (!P->is_leaf[b]) {
                int64_t off = 0;
                for (int32_t e = P->child_ptr[b]; e < P->child_ptr[b + 1]; ++e) {
                    const int c = P->child_idx[e];
                    for (int64_t x = 0; x < (int64_t)kb_of(P, c) * W; ++x)
                        S->qh[c][x] += S->qb[b][off * W + x];
                    off += kb_of(P, c);
                }
            }
        }
    }
    /* transpose of "leaves take the given charges": w[I_L] = qbar_L */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int b = 0; b < nb; ++b)
        if (P->is_leaf[b]) {
            const int64_t* ib = box_idx(P, b);
            for (int64_t a = 0; a < nb_of(P, b); ++a)
                memcpy(w + ib[a] * W, S->qb[b] + a * W, sizeof(double) * (size_t)W);
        }
}

/*
 * oracle_apply: u = Atilde q (adjoint == 0) or u = Atilde^H q (adjoint == 1).
 *   q, u   n_points x nrhs (x2 interleaved for Helmholtz)
 *   mask   optional per-box flags (forward only): translations are evaluated
 *          only for flagged target boxes, so u is exact at leaves whose whole
 *          ancestor chain is flagged and meaningless elsewhere.
 * Returns 0; -1 on allocation failure; -2 if a tree box's index set is not the
 * concatenation of its children's skeletons.
 */
int oracle_apply(const o2_plan* P, int nrhs, const double* q, double* u, int adjoint_, const uint8_t* mask)
{
    if (check_concat(P)) return -2;
    o2_state S;
    memset(&S, 0, sizeof S);
    S.nrhs = nrhs;
    S.cplx = (P->kind == 1);
    S.W = S.cplx ? 2 * nrhs : nrhs;
    if (alloc_state(P, &S)) { free_state(P, &S); return -1; }
    memset(u, 0, sizeof(double) * (size_t)(P->n_points * S.W));
    if (adjoint_) adjoint(P, &S, q, u);
    else forward(P, &S, q, u, mask);
    free_state(P, &S);
    return 0;
}
