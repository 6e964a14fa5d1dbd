/*
 * Oracle: plain FP64 multigrid for Poisson's equation on an octree of 8^3-cell
 * boxes.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU solver.  It
 * is loaded only by the test-suite, by the smoke check and by the benchmark's
 * CPU-baseline leg.  It shares no code, header, table or helper with the GPU
 * library, and it never calls it.
 *
 * What it computes (paper section 2.1): the cell-centred potential phi with
 * lap(phi) = b on the leaf cells of a quadtree/octree mesh (section 2.1.1), by
 * a geometric multigrid solver (section 2.1.2) that uses an FMG cycle and
 * V-cycles in full-approximation-scheme form (the solution is kept on every
 * level) and red-black Gauss-Seidel smoothing.  Boxes carry a one-cell ghost
 * layer so they can be worked on independently (section 2.1.3).  The paper
 * leaves the details of the discretisation and of the cycle to its companion
 * paper; the readings used here are:
 *   - operator: 7-point (sum of 6 neighbours - 6 phi) / h^2 at every level;
 *   - physical ghosts: Dirichlet 2 g - phi_in (g the face value), Neumann
 *     phi_in, refreshed before each colour (so boundary cells are updated with
 *     the ghost of the previous iterate, "lagged");
 *   - refinement-boundary ghosts: quadratic interpolation in the normal
 *     direction through the two interior fine cells and a coarse value that is
 *     itself interpolated quadratically along the two tangential directions
 *     (weights 7/8, 5/32, -3/32; then 8/15, 2/3, -1/5);
 *   - restriction: mean of the 8 children; prolongation of the coarse
 *     correction: 1/4 of the parent cell plus 1/4 of each of its three face
 *     neighbours on the side of the fine cell;
 *   - coarsest level (the 8^3 root of each tree): exact dense Cholesky solve;
 *   - FMG: compute the FAS data top-down without smoothing, solve the
 *     coarsest level, then for every finer level prolong the correction and
 *     run one V-cycle with that level on top; then V-cycles until the
 *     volume-weighted L2 norm of the leaf residual, relative to that of the
 *     residual of phi = 0, is below the tolerance.
 *
 * Fields are stored per box as 10^3 arrays (8^3 interior plus ghosts).  Loops
 * run over the boxes of one level (optionally with OpenMP, the paper's
 * block-parallel scheme of section 2.1.3).  Nothing here is fused, blocked or
 * reordered beyond the definitions above.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENESTING (-2)
#define ORC_ENOMEM (-3)
#define ORC_ENOCONV (-5)
#define ORC_ESTATE (-6)
#define ORC_ETOPO (-7)

#define NG 10
#define BOX (NG * NG * NG)
#define AT(i, j, k) ((((k) + 1) * NG + ((j) + 1)) * NG + ((i) + 1))
#define MAXLEV 15

enum { F_PHI = 0, F_RHS = 1, F_OLD = 2, F_RES = 3, NFIELD = 4 };
enum { DIRICHLET = 0, NEUMANN = 1 };

typedef struct {
    int64_t n;
    int nlev, ntree;
    int32_t *lev, *bx, *by, *bz, *tid, *order;
    int32_t *parent, *child, *nbr, *cfq;
    int64_t lstart[MAXLEV + 2];
    double lo[3], len;
    int bct[6];
    double bcv[6];
    double *bcarr;           /* NULL or [n][6][64] per boundary face cell */
    double *f[NFIELD];       /* [n][1000] */
    uint64_t *hkey;
    int32_t *hval;
    int64_t hcap;
    double *chol;            /* lower Cholesky factor of the root operator */
    double *tree_beff;       /* [ntree] norm of the residual of phi = 0 */
    double *tree_rel;        /* [ntree] relative residual at the last check */
    double chol_h;
    int bad_lookup;          /* set when a required coarse cell is missing */
} otree;

static char g_err[256];
static void set_err(const char *s) { snprintf(g_err, sizeof g_err, "%s", s); }
const char *oracle_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ lookup */

static uint64_t okey(int tree, int l, int i, int j, int k) {
    return ((uint64_t)tree << 46) | ((uint64_t)l << 42) | ((uint64_t)i << 28) |
           ((uint64_t)j << 14) | (uint64_t)k;
}

static uint64_t hmix(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33;
    return x;
}

static void hput(otree *t, uint64_t key, int32_t v) {
    uint64_t h = hmix(key) & (uint64_t)(t->hcap - 1);
    while (t->hkey[h] != 0) h = (h + 1) & (uint64_t)(t->hcap - 1);
    t->hkey[h] = key + 1;
    t->hval[h] = v;
}

static int32_t hget(const otree *t, uint64_t key) {
    uint64_t h = hmix(key) & (uint64_t)(t->hcap - 1);
    while (t->hkey[h] != 0) {
        if (t->hkey[h] == key + 1) return t->hval[h];
        h = (h + 1) & (uint64_t)(t->hcap - 1);
    }
    return -1;
}

/* box at (tree, l, i, j, k) or -1; coordinates must be in range */
static int32_t find(const otree *t, int tree, int l, int i, int j, int k) {
    return hget(t, okey(tree, l, i, j, k));
}

static int in_range(int l, int i, int j, int k) {
    int n = 1 << (l - 1);
    return i >= 0 && j >= 0 && k >= 0 && i < n && j < n && k < n;
}

static double hlev(const otree *t, int l) { return t->len / (8.0 * (double)(1 << (l - 1))); }

/* ---------------------------------------------------------------- create */

typedef struct { uint64_t key; int32_t idx; } sortrec;

static uint64_t morton3(uint32_t i, uint32_t j, uint32_t k) {
    uint64_t m = 0;
    for (int b = 0; b < 14; b++) {
        m |= (uint64_t)((i >> b) & 1u) << (3 * b);
        m |= (uint64_t)((j >> b) & 1u) << (3 * b + 1);
        m |= (uint64_t)((k >> b) & 1u) << (3 * b + 2);
    }
    return m;
}

static int cmp_rec(const void *a, const void *b) {
    uint64_t x = ((const sortrec *)a)->key, y = ((const sortrec *)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

void oracle_destroy(otree *t) {
    if (!t) return;
    free(t->lev); free(t->bx); free(t->by); free(t->bz); free(t->tid); free(t->order);
    free(t->parent); free(t->child); free(t->nbr); free(t->cfq);
    free(t->bcarr);
    for (int q = 0; q < NFIELD; q++) free(t->f[q]);
    free(t->hkey); free(t->hval); free(t->chol);
    free(t->tree_beff); free(t->tree_rel);
    free(t);
}

static const int DIR[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

int oracle_create(otree **out, int64_t n, const int32_t *level, const int32_t *ijk,
                  const int32_t *tree, const double *lo, double len, const int32_t *bc_type,
                  const double *bc_val) {
    *out = NULL;
    if (n <= 0 || !level || !ijk || !lo || !bc_type || !bc_val || !(len > 0)) {
        set_err("invalid arguments");
        return ORC_EINVAL;
    }
    int nneu = 0;
    for (int d = 0; d < 6; d++) {
        if (bc_type[d] != DIRICHLET && bc_type[d] != NEUMANN) { set_err("bad bc type"); return ORC_EINVAL; }
        nneu += bc_type[d] == NEUMANN;
    }
    if (nneu == 6) { set_err("all-Neumann domain is singular"); return ORC_EINVAL; }
    int ntree = 0;
    for (int64_t b = 0; b < n; b++) {
        int l = level[b], tr = tree ? tree[b] : 0;
        if (l < 1 || l > MAXLEV || tr < 0 || tr >= 65536 ||
            !in_range(l, ijk[3 * b], ijk[3 * b + 1], ijk[3 * b + 2])) {
            snprintf(g_err, sizeof g_err, "box %lld: level or coordinates out of range", (long long)b);
            return ORC_EINVAL;
        }
        if (tr + 1 > ntree) ntree = tr + 1;
    }
    otree *t = (otree *)calloc(1, sizeof(otree));
    if (!t) return ORC_ENOMEM;
    t->n = n; t->ntree = ntree; t->len = len;
    for (int a = 0; a < 3; a++) t->lo[a] = lo[a];
    for (int d = 0; d < 6; d++) { t->bct[d] = bc_type[d]; t->bcv[d] = bc_val[d]; }
    t->hcap = 1;
    while (t->hcap < 2 * n + 16) t->hcap <<= 1;
    t->hkey = (uint64_t *)calloc((size_t)t->hcap, sizeof(uint64_t));
    t->hval = (int32_t *)calloc((size_t)t->hcap, sizeof(int32_t));
    sortrec *rec = (sortrec *)malloc((size_t)n * sizeof(sortrec));
    if (!t->hkey || !t->hval || !rec) { free(rec); oracle_destroy(t); return ORC_ENOMEM; }

    /* canonical order: level, then tree, then Morton index of (i, j, k) */
    for (int64_t b = 0; b < n; b++) {
        int tr = tree ? tree[b] : 0;
        rec[b].key = ((uint64_t)level[b] << 58) | ((uint64_t)tr << 42) |
                     morton3((uint32_t)ijk[3 * b], (uint32_t)ijk[3 * b + 1], (uint32_t)ijk[3 * b + 2]);
        rec[b].idx = (int32_t)b;
    }
    qsort(rec, (size_t)n, sizeof(sortrec), cmp_rec);
    for (int64_t b = 1; b < n; b++)
        if (rec[b].key == rec[b - 1].key) {
            snprintf(g_err, sizeof g_err, "duplicate box (input %d)", rec[b].idx);
            free(rec); oracle_destroy(t); return ORC_EINVAL;
        }
#define ALLOC32(p, m) do { (p) = (int32_t *)malloc((size_t)(m) * sizeof(int32_t)); if (!(p)) { free(rec); oracle_destroy(t); return ORC_ENOMEM; } } while (0)
    ALLOC32(t->lev, n); ALLOC32(t->bx, n); ALLOC32(t->by, n); ALLOC32(t->bz, n);
    ALLOC32(t->tid, n); ALLOC32(t->order, n); ALLOC32(t->parent, n);
    ALLOC32(t->child, 8 * n); ALLOC32(t->nbr, 6 * n); ALLOC32(t->cfq, 6 * n);
    int nlev = 0;
    for (int64_t b = 0; b < n; b++) {
        int32_t s = rec[b].idx;
        t->order[b] = s;
        t->lev[b] = level[s];
        t->bx[b] = ijk[3 * s]; t->by[b] = ijk[3 * s + 1]; t->bz[b] = ijk[3 * s + 2];
        t->tid[b] = tree ? tree[s] : 0;
        if (level[s] > nlev) nlev = level[s];
        hput(t, okey(t->tid[b], t->lev[b], t->bx[b], t->by[b], t->bz[b]), (int32_t)b);
    }
    free(rec);
    t->nlev = nlev;
    for (int l = 0; l <= MAXLEV + 1; l++) t->lstart[l] = n;
    for (int64_t b = n - 1; b >= 0; b--) t->lstart[t->lev[b]] = b;
    for (int l = MAXLEV; l >= 1; l--)
        if (t->lstart[l] > t->lstart[l + 1]) t->lstart[l] = t->lstart[l + 1];

    /* topology: every tree has its root, every box its parent, every
       refined box all eight children */
    for (int tr = 0; tr < ntree; tr++)
        if (find(t, tr, 1, 0, 0, 0) < 0) {
            snprintf(g_err, sizeof g_err, "tree %d has no root box", tr);
            oracle_destroy(t); return ORC_ETOPO;
        }
    for (int64_t b = 0; b < n; b++) {
        int l = t->lev[b];
        t->parent[b] = l > 1 ? find(t, t->tid[b], l - 1, t->bx[b] >> 1, t->by[b] >> 1, t->bz[b] >> 1) : -1;
        if (l > 1 && t->parent[b] < 0) {
            snprintf(g_err, sizeof g_err, "box %d has no parent", t->order[b]);
            oracle_destroy(t); return ORC_ETOPO;
        }
        int nch = 0;
        for (int c = 0; c < 8; c++) {
            int32_t ch = -1;
            if (l < MAXLEV)
                ch = find(t, t->tid[b], l + 1, 2 * t->bx[b] + (c & 1), 2 * t->by[b] + ((c >> 1) & 1),
                          2 * t->bz[b] + ((c >> 2) & 1));
            t->child[8 * b + c] = ch;
            nch += ch >= 0;
        }
        if (nch != 0 && nch != 8) {
            snprintf(g_err, sizeof g_err, "box %d has %d of 8 children", t->order[b], nch);
            oracle_destroy(t); return ORC_ETOPO;
        }
    }
    /* proper nesting over all 26 neighbours: the level-(l-1) box containing
       every neighbouring position of a level-l box must exist */
    for (int64_t b = 0; b < n; b++) {
        int l = t->lev[b];
        if (l < 2) continue;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int i = t->bx[b] + dx, j = t->by[b] + dy, k = t->bz[b] + dz;
                    if (!in_range(l, i, j, k)) continue;
                    if (find(t, t->tid[b], l - 1, i >> 1, j >> 1, k >> 1) < 0) {
                        snprintf(g_err, sizeof g_err, "box %d violates 2:1 nesting", t->order[b]);
                        oracle_destroy(t); return ORC_ENESTING;
                    }
                }
    }
    /* face neighbours: same-level box, -1 across a refinement boundary,
       -2 at the domain boundary; cfq = the coarser box across a -1 face */
    for (int64_t b = 0; b < n; b++) {
        int l = t->lev[b];
        for (int d = 0; d < 6; d++) {
            int i = t->bx[b] + DIR[d][0], j = t->by[b] + DIR[d][1], k = t->bz[b] + DIR[d][2];
            int32_t v = -2, q = -1;
            if (in_range(l, i, j, k)) {
                v = find(t, t->tid[b], l, i, j, k);
                if (v < 0) q = find(t, t->tid[b], l - 1, i >> 1, j >> 1, k >> 1);
            }
            t->nbr[6 * b + d] = v;
            t->cfq[6 * b + d] = q;
        }
    }
    for (int q = 0; q < NFIELD; q++) {
        t->f[q] = (double *)calloc((size_t)n * BOX, sizeof(double));
        if (!t->f[q]) { oracle_destroy(t); return ORC_ENOMEM; }
    }
    t->tree_beff = (double *)calloc((size_t)ntree, sizeof(double));
    t->tree_rel = (double *)calloc((size_t)ntree, sizeof(double));
    if (!t->tree_beff || !t->tree_rel) { oracle_destroy(t); return ORC_ENOMEM; }
    *out = t;
    return ORC_OK;
}

int oracle_info(const otree *t, int64_t *out) {
    int64_t leaf = 0;
    for (int64_t b = 0; b < t->n; b++) leaf += t->child[8 * b] < 0;
    out[0] = t->n; out[1] = t->nlev; out[2] = t->ntree; out[3] = leaf;
    for (int l = 1; l <= MAXLEV + 1; l++) out[3 + l] = t->lstart[l];
    return ORC_OK;
}

/* what: 0 order, 1 level, 2 ijk[3], 3 tree, 4 parent, 5 child[8], 6 nbr[6], 7 cfq[6] */
int oracle_index(const otree *t, int what, int32_t *out) {
    int64_t n = t->n;
    switch (what) {
    case 0: memcpy(out, t->order, (size_t)n * 4); break;
    case 1: memcpy(out, t->lev, (size_t)n * 4); break;
    case 2: for (int64_t b = 0; b < n; b++) { out[3 * b] = t->bx[b]; out[3 * b + 1] = t->by[b]; out[3 * b + 2] = t->bz[b]; } break;
    case 3: memcpy(out, t->tid, (size_t)n * 4); break;
    case 4: memcpy(out, t->parent, (size_t)n * 4); break;
    case 5: memcpy(out, t->child, (size_t)n * 32); break;
    case 6: memcpy(out, t->nbr, (size_t)n * 24); break;
    case 7: memcpy(out, t->cfq, (size_t)n * 24); break;
    default: set_err("bad index table id"); return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ fields */

int oracle_set_field(otree *t, int which, const double *nat) {
    if (which < 0 || which >= NFIELD) return ORC_EINVAL;
    double *f = t->f[which];
    for (int64_t b = 0; b < t->n; b++)
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) f[b * BOX + AT(i, j, k)] = nat[((b * 8 + k) * 8 + j) * 8 + i];
    return ORC_OK;
}

int oracle_get_field(const otree *t, int which, double *nat) {
    if (which < 0 || which >= NFIELD) return ORC_EINVAL;
    const double *f = t->f[which];
    for (int64_t b = 0; b < t->n; b++)
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) nat[((b * 8 + k) * 8 + j) * 8 + i] = f[b * BOX + AT(i, j, k)];
    return ORC_OK;
}

/* per boundary-face-cell Dirichlet values, [n][6][64] in canonical box order;
   the 64 values of a face are ordered (v, u) over its two tangential axes in
   increasing axis order, u fastest.  NULL restores the per-face constants. */
int oracle_set_bcval(otree *t, const double *vals) {
    free(t->bcarr);
    t->bcarr = NULL;
    if (!vals) return ORC_OK;
    t->bcarr = (double *)malloc((size_t)t->n * 6 * 64 * sizeof(double));
    if (!t->bcarr) return ORC_ENOMEM;
    memcpy(t->bcarr, vals, (size_t)t->n * 6 * 64 * sizeof(double));
    return ORC_OK;
}

/* ------------------------------------------------------------------ ghosts */

static void tang_axes(int a, int *t1, int *t2) {
    *t1 = a == 0 ? 1 : 0;
    *t2 = a == 2 ? 1 : 2;
}

/* Dirichlet value on face d of box b at the face cell with tangential
   coordinates (u, v); 0 in homogeneous mode */
static double face_value(const otree *t, int64_t b, int d, int u, int v, int homog) {
    if (homog) return 0.0;
    if (t->bcarr) return t->bcarr[(b * 6 + d) * 64 + v * 8 + u];
    return t->bcv[d];
}

/* value of field f at level-l global cell (I, J, K) of a tree; a position
   outside the domain (in one axis) gets the physical ghost value */
static double cell_value(otree *t, int tree, int l, int I, int J, int K, const double *f, int homog) {
    int n = 8 << (l - 1);
    int G[3] = {I, J, K};
    int out_axis = -1, side = 0;
    for (int a = 0; a < 3; a++) {
        if (G[a] < 0) { out_axis = a; side = 0; G[a] = 0; }
        else if (G[a] >= n) { out_axis = a; side = 1; G[a] = n - 1; }
    }
    int32_t b = find(t, tree, l, G[0] >> 3, G[1] >> 3, G[2] >> 3);
    if (b < 0) { t->bad_lookup = 1; return 0.0; }
    double v = f[(int64_t)b * BOX + AT(G[0] & 7, G[1] & 7, G[2] & 7)];
    if (out_axis < 0) return v;
    int d = 2 * out_axis + side;
    if (t->bct[d] == NEUMANN) return v;
    int t1, t2;
    tang_axes(out_axis, &t1, &t2);
    return 2.0 * face_value(t, b, d, G[t1] & 7, G[t2] & 7, homog) - v;
}

/* refresh the face ghosts of one box */
static void fill_box_ghosts(otree *t, int64_t b, double *f, int homog) {
    int l = t->lev[b];
    int B[3] = {t->bx[b], t->by[b], t->bz[b]};
    double *fb = f + b * BOX;
    for (int d = 0; d < 6; d++) {
        int a = d >> 1, s = d & 1, t1, t2;
        tang_axes(a, &t1, &t2);
        int32_t nb = t->nbr[6 * b + d];
        for (int v = 0; v < 8; v++)
            for (int u = 0; u < 8; u++) {
                int g[3], p1[3], p2[3], src[3];
                g[t1] = p1[t1] = p2[t1] = src[t1] = u;
                g[t2] = p1[t2] = p2[t2] = src[t2] = v;
                g[a] = s ? 8 : -1;
                p1[a] = s ? 7 : 0;
                p2[a] = s ? 6 : 1;
                src[a] = s ? 0 : 7;
                double f1 = fb[AT(p1[0], p1[1], p1[2])];
                double val;
                if (nb >= 0) {
                    val = f[(int64_t)nb * BOX + AT(src[0], src[1], src[2])];
                } else if (nb == -2) {
                    val = t->bct[d] == NEUMANN ? f1 : 2.0 * face_value(t, b, d, u, v, homog) - f1;
                } else {
                    /* refinement boundary: coarse cell containing the ghost,
                       interpolated along both tangential directions, then a
                       quadratic through it and the two interior fine cells */
                    int G[3], C[3];
                    for (int q = 0; q < 3; q++) { G[q] = 8 * B[q] + g[q]; C[q] = G[q] >> 1; }
                    double chat = 0.875 * cell_value(t, t->tid[b], l - 1, C[0], C[1], C[2], f, homog);
                    int ta[2] = {t1, t2};
                    for (int q = 0; q < 2; q++) {
                        int ax = ta[q];
                        double st = (G[ax] & 1) ? 1.0 : -1.0;
                        int Cp[3] = {C[0], C[1], C[2]}, Cm[3] = {C[0], C[1], C[2]};
                        Cp[ax] += 1; Cm[ax] -= 1;
                        double cp = cell_value(t, t->tid[b], l - 1, Cp[0], Cp[1], Cp[2], f, homog);
                        double cm = cell_value(t, t->tid[b], l - 1, Cm[0], Cm[1], Cm[2], f, homog);
                        chat += (1.0 / 32.0 + st / 8.0) * cp + (1.0 / 32.0 - st / 8.0) * cm;
                    }
                    double f2 = fb[AT(p2[0], p2[1], p2[2])];
                    val = (8.0 / 15.0) * chat + (2.0 / 3.0) * f1 - 0.2 * f2;
                }
                fb[AT(g[0], g[1], g[2])] = val;
            }
    }
}

static void fill_ghosts(otree *t, int l, double *f, int homog) {
    int64_t b0 = t->lstart[l], b1 = t->lstart[l + 1];
#pragma omp parallel for schedule(static)
    for (int64_t b = b0; b < b1; b++) fill_box_ghosts(t, b, f, homog);
}

/* ------------------------------------------------------------ operators */

static double lap_at(const double *fb, int i, int j, int k, double inv_h2) {
    double s = fb[AT(i - 1, j, k)] + fb[AT(i + 1, j, k)] + fb[AT(i, j - 1, k)] +
               fb[AT(i, j + 1, k)] + fb[AT(i, j, k - 1)] + fb[AT(i, j, k + 1)];
    return (s - 6.0 * fb[AT(i, j, k)]) * inv_h2;
}

/* n red-black Gauss-Seidel sweeps over all boxes of level l */
static void smooth(otree *t, int l, int nsweep) {
    double h = hlev(t, l), h2 = h * h;
    int64_t b0 = t->lstart[l], b1 = t->lstart[l + 1];
    double *phi = t->f[F_PHI], *rhs = t->f[F_RHS];
    for (int it = 0; it < nsweep; it++)
        for (int colour = 0; colour < 2; colour++) {
            fill_ghosts(t, l, phi, 0);
#pragma omp parallel for schedule(static)
            for (int64_t b = b0; b < b1; b++) {
                double *p = phi + b * BOX;
                const double *r = rhs + b * BOX;
                for (int k = 0; k < 8; k++)
                    for (int j = 0; j < 8; j++)
                        for (int i = 0; i < 8; i++) {
                            if (((i + j + k) & 1) != colour) continue;
                            double s = p[AT(i - 1, j, k)] + p[AT(i + 1, j, k)] + p[AT(i, j - 1, k)] +
                                       p[AT(i, j + 1, k)] + p[AT(i, j, k - 1)] + p[AT(i, j, k + 1)];
                            p[AT(i, j, k)] = (s - h2 * r[AT(i, j, k)]) / 6.0;
                        }
            }
        }
}

/* res = rhs - L phi on all boxes of level l (ghosts refreshed first) */
static void residual_level(otree *t, int l, int leaf_only) {
    double h = hlev(t, l), inv_h2 = 1.0 / (h * h);
    int64_t b0 = t->lstart[l], b1 = t->lstart[l + 1];
    double *phi = t->f[F_PHI], *rhs = t->f[F_RHS], *res = t->f[F_RES];
    fill_ghosts(t, l, phi, 0);
#pragma omp parallel for schedule(static)
    for (int64_t b = b0; b < b1; b++) {
        if (leaf_only && t->child[8 * b] >= 0) continue;
        const double *p = phi + b * BOX, *r = rhs + b * BOX;
        double *o = res + b * BOX;
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) o[AT(i, j, k)] = r[AT(i, j, k)] - lap_at(p, i, j, k, inv_h2);
    }
}

/* mean of the 8 children of every cell of the refined boxes of level l-1 */
static void restrict_field(otree *t, int l, double *f) {
    int64_t b0 = t->lstart[l - 1], b1 = t->lstart[l];
#pragma omp parallel for schedule(static)
    for (int64_t p = b0; p < b1; p++) {
        if (t->child[8 * p] < 0) continue;
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) {
                    int c = (i >> 2) + 2 * (j >> 2) + 4 * (k >> 2);
                    const double *fc = f + (int64_t)t->child[8 * p + c] * BOX;
                    int fi = 2 * (i & 3), fj = 2 * (j & 3), fk = 2 * (k & 3);
                    double s = 0.0;
                    for (int dk = 0; dk < 2; dk++)
                        for (int dj = 0; dj < 2; dj++)
                            for (int di = 0; di < 2; di++) s += fc[AT(fi + di, fj + dj, fk + dk)];
                    f[p * BOX + AT(i, j, k)] = 0.125 * s;
                }
    }
}

/* down-leg transfer from level l to level l-1 (full approximation scheme):
   residual on level l, restriction of phi and of the residual, old <- phi on
   the whole coarse level, and the coarse right-hand side L phi_c + r_c on the
   covered (refined) coarse boxes */
static void fas_down(otree *t, int l) {
    residual_level(t, l, 0);
    restrict_field(t, l, t->f[F_PHI]);
    restrict_field(t, l, t->f[F_RES]);
    int64_t b0 = t->lstart[l - 1], b1 = t->lstart[l];
    memcpy(t->f[F_OLD] + b0 * BOX, t->f[F_PHI] + b0 * BOX, (size_t)(b1 - b0) * BOX * sizeof(double));
    double h = hlev(t, l - 1), inv_h2 = 1.0 / (h * h);
    fill_ghosts(t, l - 1, t->f[F_PHI], 0);
#pragma omp parallel for schedule(static)
    for (int64_t p = b0; p < b1; p++) {
        if (t->child[8 * p] < 0) continue;
        const double *ph = t->f[F_PHI] + p * BOX, *rc = t->f[F_RES] + p * BOX;
        double *r = t->f[F_RHS] + p * BOX;
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) r[AT(i, j, k)] = lap_at(ph, i, j, k, inv_h2) + rc[AT(i, j, k)];
    }
}

/* up-leg: phi on level l += prolongation of (phi - old) on level l-1 */
static int prolong_up(otree *t, int l) {
    int64_t c0 = t->lstart[l - 1], c1 = t->lstart[l];
    double *del = t->f[F_RES];
    for (int64_t p = c0; p < c1; p++)
        for (int q = 0; q < BOX; q++) del[p * BOX + q] = t->f[F_PHI][p * BOX + q] - t->f[F_OLD][p * BOX + q];
    /* ghosts of the correction, homogeneous boundary conditions; a refined
       box never lies on a refinement boundary of its own level */
    for (int64_t p = c0; p < c1; p++) {
        if (t->child[8 * p] < 0) continue;
        for (int d = 0; d < 6; d++)
            if (t->nbr[6 * p + d] == -1) { set_err("refined box on a refinement boundary"); return ORC_ESTATE; }
        fill_box_ghosts(t, p, del, 1);
    }
    int64_t b0 = t->lstart[l], b1 = t->lstart[l + 1];
#pragma omp parallel for schedule(static)
    for (int64_t b = b0; b < b1; b++) {
        int32_t p = t->parent[b];
        const double *dp = del + (int64_t)p * BOX;
        int B[3] = {t->bx[b], t->by[b], t->bz[b]};
        int P[3] = {t->bx[p], t->by[p], t->bz[p]};
        double *ph = t->f[F_PHI] + b * BOX;
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) {
                    int loc[3] = {i, j, k}, C[3], s[3];
                    for (int a = 0; a < 3; a++) {
                        int G = 8 * B[a] + loc[a];
                        C[a] = (G >> 1) - 8 * P[a];
                        s[a] = (G & 1) ? 1 : -1;
                    }
                    double c0v = dp[AT(C[0], C[1], C[2])];
                    double cx = dp[AT(C[0] + s[0], C[1], C[2])];
                    double cy = dp[AT(C[0], C[1] + s[1], C[2])];
                    double cz = dp[AT(C[0], C[1], C[2] + s[2])];
                    ph[AT(i, j, k)] += 0.25 * c0v + 0.25 * (cx + cy + cz);
                }
    }
    return ORC_OK;
}

/* exact solve on the root box of every tree: dense Cholesky factorisation of
   M = -h^2 L (symmetric positive definite when a face is Dirichlet) */
static int coarse_solve(otree *t) {
    double h = hlev(t, 1);
    int N = 512;
    if (!t->chol) {
        double *M = (double *)calloc((size_t)N * N, sizeof(double));
        if (!M) return ORC_ENOMEM;
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) {
                    int p = (k * 8 + j) * 8 + i, c[3] = {i, j, k};
                    double diag = 6.0;
                    for (int d = 0; d < 6; d++) {
                        int a = d >> 1, s = d & 1, q[3] = {i, j, k};
                        q[a] += s ? 1 : -1;
                        if (q[a] < 0 || q[a] > 7) {
                            diag += t->bct[d] == DIRICHLET ? 1.0 : -1.0;
                        } else {
                            M[p * N + (q[2] * 8 + q[1]) * 8 + q[0]] = -1.0;
                        }
                        (void)c;
                    }
                    M[p * N + p] = diag;
                }
        for (int j = 0; j < N; j++) {
            double s = M[j * N + j];
            for (int q = 0; q < j; q++) s -= M[j * N + q] * M[j * N + q];
            if (!(s > 0)) { free(M); set_err("root operator not positive definite"); return ORC_ESTATE; }
            double d = sqrt(s);
            M[j * N + j] = d;
            for (int i = j + 1; i < N; i++) {
                double v = M[i * N + j];
                for (int q = 0; q < j; q++) v -= M[i * N + q] * M[j * N + q];
                M[i * N + j] = v / d;
            }
        }
        t->chol = M;
    }
    double *x = (double *)malloc(N * sizeof(double));
    for (int64_t b = t->lstart[1]; b < t->lstart[2]; b++) {
        double *ph = t->f[F_PHI] + b * BOX;
        const double *r = t->f[F_RHS] + b * BOX;
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) {
                    int p = (k * 8 + j) * 8 + i, c[3] = {i, j, k};
                    double rhs = r[AT(i, j, k)];
                    for (int d = 0; d < 6; d++) {
                        int a = d >> 1, s = d & 1;
                        int edge = s ? (c[a] == 7) : (c[a] == 0);
                        if (edge && t->bct[d] == DIRICHLET) {
                            int t1, t2;
                            tang_axes(a, &t1, &t2);
                            rhs -= 2.0 * face_value(t, b, d, c[t1], c[t2], 0) / (h * h);
                        }
                    }
                    x[p] = -h * h * rhs;
                }
        const double *L = t->chol;
        for (int i = 0; i < N; i++) {
            double v = x[i];
            for (int q = 0; q < i; q++) v -= L[i * N + q] * x[q];
            x[i] = v / L[i * N + i];
        }
        for (int i = N - 1; i >= 0; i--) {
            double v = x[i];
            for (int q = i + 1; q < N; q++) v -= L[q * N + i] * x[q];
            x[i] = v / L[i * N + i];
        }
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) ph[AT(i, j, k)] = x[(k * 8 + j) * 8 + i];
    }
    free(x);
    return ORC_OK;
}

/* ------------------------------------------------------------------ cycles */

typedef struct { int n_down, n_up; } cycopts;

static int vcycle(otree *t, int top, const cycopts *o) {
    for (int l = top; l >= 2; l--) {
        smooth(t, l, o->n_down);
        fas_down(t, l);
    }
    int rc = coarse_solve(t);
    if (rc) return rc;
    for (int l = 2; l <= top; l++) {
        if ((rc = prolong_up(t, l))) return rc;
        smooth(t, l, o->n_up);
    }
    return t->bad_lookup ? ORC_ESTATE : ORC_OK;
}

static void restrict_all(otree *t) {
    for (int l = t->nlev; l >= 2; l--) restrict_field(t, l, t->f[F_PHI]);
}

/* volume-weighted L2 norm (squared) and max norm of the residual over the
   leaf cells of each tree: sq[tree], mx[tree] */
static void leaf_norms(otree *t, double *sq, double *mx) {
    double *part = (double *)calloc((size_t)t->n, sizeof(double));
    double *pmax = (double *)calloc((size_t)t->n, sizeof(double));
    for (int l = 1; l <= t->nlev; l++) {
        residual_level(t, l, 1);
        double h = hlev(t, l), vol = h * h * h;
        int64_t b0 = t->lstart[l], b1 = t->lstart[l + 1];
#pragma omp parallel for schedule(static)
        for (int64_t b = b0; b < b1; b++) {
            if (t->child[8 * b] >= 0) continue;
            const double *r = t->f[F_RES] + b * BOX;
            double s = 0.0, m = 0.0;
            for (int k = 0; k < 8; k++)
                for (int j = 0; j < 8; j++)
                    for (int i = 0; i < 8; i++) {
                        double v = r[AT(i, j, k)];
                        s += v * v;
                        if (fabs(v) > m || v != v) m = v != v ? v : fabs(v);
                    }
            part[b] = s * vol;
            pmax[b] = m;
        }
    }
    for (int tr = 0; tr < t->ntree; tr++) sq[tr] = mx[tr] = 0.0;
    for (int64_t b = 0; b < t->n; b++) {
        int tr = t->tid[b];
        sq[tr] += part[b];
        if (pmax[b] > mx[tr] || pmax[b] != pmax[b]) mx[tr] = pmax[b];
    }
    free(part); free(pmax);
}

/* ---------------------------------------------------------- electric field */

/* Electric field of the current phi (paper section 2.3, E = -grad phi).  On
   the cell faces by central differences: the x-component at the face between
   cells i and i+1 is (phi_i - phi_{i+1}) / h, and likewise in y and z.  The
   field strength at a cell centre is sqrt(Ex^2 + Ey^2 + Ez^2), each component
   the mean of the cell's two face values.  Covered cells are first reset to
   the mean of their children and every box's ghosts are filled as for the
   residual, so a box-boundary face uses the box's own ghost.
   e_face (or NULL): [n][3][9][64], axis a, face f = 0..8 between cells f-1
   and f along a, tangential cell v*8 + u (u along the first other axis).
   e_norm (or NULL): [n][512], natural order (x fastest). */
int oracle_efield(otree *t, double *e_face, double *e_norm) {
    t->bad_lookup = 0;
    restrict_all(t);
    for (int l = 1; l <= t->nlev; l++) fill_ghosts(t, l, t->f[F_PHI], 0);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < t->n; b++) {
        const double *fb = t->f[F_PHI] + b * BOX;
        double h = hlev(t, t->lev[b]);
        double E[3][9][64];
        for (int a = 0; a < 3; a++) {
            int t1, t2;
            tang_axes(a, &t1, &t2);
            for (int f = 0; f <= 8; f++)
                for (int v = 0; v < 8; v++)
                    for (int u = 0; u < 8; u++) {
                        int lo[3], hi[3];
                        lo[t1] = hi[t1] = u;
                        lo[t2] = hi[t2] = v;
                        lo[a] = f - 1;
                        hi[a] = f;
                        E[a][f][v * 8 + u] =
                            (fb[AT(lo[0], lo[1], lo[2])] - fb[AT(hi[0], hi[1], hi[2])]) / h;
                    }
        }
        if (e_face) memcpy(e_face + b * 3 * 9 * 64, E, sizeof E);
        if (e_norm)
            for (int k = 0; k < 8; k++)
                for (int j = 0; j < 8; j++)
                    for (int i = 0; i < 8; i++) {
                        /* tangential index of the cell on each axis' faces */
                        double ex = (E[0][i][k * 8 + j] + E[0][i + 1][k * 8 + j]) / 2.0;
                        double ey = (E[1][j][k * 8 + i] + E[1][j + 1][k * 8 + i]) / 2.0;
                        double ez = (E[2][k][j * 8 + i] + E[2][k + 1][j * 8 + i]) / 2.0;
                        e_norm[b * 512 + (k * 8 + j) * 8 + i] = sqrt(ex * ex + ey * ey + ez * ez);
                    }
    }
    return t->bad_lookup ? ORC_ESTATE : ORC_OK;
}

/* ------------------------------------------------------- mesh adaptation */

/* Potential of tree `to` from tree `from` over the same domain (a regrid
   step, paper section 2.5).  Covered cells of `from` are first reset to the
   mean of their children.  A box of `to` that `from` also has (same tree,
   level and position) takes its values.  The others, from the coarsest level
   up, are interpolated from their parent in `to`, filled before them: a fine
   cell gets 1/4 of its parent cell plus 1/4 of each of the parent cell's three
   neighbours on the fine cell's side (the stencil of the correction
   prolongation, applied to phi; exact for linear functions), with the
   parent's ghost layer standing in for cells outside the parent. */
int oracle_transfer(otree *from, otree *to) {
    from->bad_lookup = to->bad_lookup = 0;
    restrict_all(from);
    char *have = (char *)calloc((size_t)to->n, 1);
    if (!have) return ORC_ENOMEM;
    for (int64_t b = 0; b < to->n; b++) {
        int32_t o = find(from, to->tid[b], to->lev[b], to->bx[b], to->by[b], to->bz[b]);
        if (o < 0) {
            if (to->lev[b] == 1) { free(have); set_err("transfer: a tree has no counterpart"); return ORC_EINVAL; }
            continue;
        }
        have[b] = 1;
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++)
                    to->f[F_PHI][b * BOX + AT(i, j, k)] = from->f[F_PHI][(int64_t)o * BOX + AT(i, j, k)];
    }
    for (int l = 2; l <= to->nlev; l++) {
        fill_ghosts(to, l - 1, to->f[F_PHI], 0);
        for (int64_t b = to->lstart[l]; b < to->lstart[l + 1]; b++) {
            if (have[b]) continue;
            const double *pb = to->f[F_PHI] + (int64_t)to->parent[b] * BOX;
            int ox = to->bx[b] & 1, oy = to->by[b] & 1, oz = to->bz[b] & 1;
            for (int k = 0; k < 8; k++)
                for (int j = 0; j < 8; j++)
                    for (int i = 0; i < 8; i++) {
                        int cx = 4 * ox + i / 2, cy = 4 * oy + j / 2, cz = 4 * oz + k / 2;
                        int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
                        double c = pb[AT(cx, cy, cz)];
                        double nx = pb[AT(cx + sx, cy, cz)], ny = pb[AT(cx, cy + sy, cz)],
                               nz = pb[AT(cx, cy, cz + sz)];
                        to->f[F_PHI][b * BOX + AT(i, j, k)] = 0.25 * c + 0.25 * (nx + ny + nz);
                    }
        }
    }
    free(have);
    return to->bad_lookup ? ORC_ESTATE : ORC_OK;
}

/* per-tree norm of the residual of phi = 0 (the right-hand side with the
   boundary data folded in) */
static void beff_norm(otree *t, double *beff) {
    size_t sz = (size_t)t->n * BOX * sizeof(double);
    double *save = (double *)malloc(sz);
    double *mx = (double *)malloc((size_t)t->ntree * sizeof(double));
    memcpy(save, t->f[F_PHI], sz);
    memset(t->f[F_PHI], 0, sz);
    leaf_norms(t, beff, mx);
    for (int tr = 0; tr < t->ntree; tr++) beff[tr] = sqrt(beff[tr]);
    memcpy(t->f[F_PHI], save, sz);
    free(save); free(mx);
}

/* stats layout (doubles): 0 rel, 1 l2, 2 linf, 3 beff_l2, 4 n_vcycles,
   5.. 5+64: relative residual after FMG (index 0) and after each V-cycle.
   A forest's trees are independent problems: rel is the largest relative
   residual over the trees (each relative to its own residual of phi = 0);
   l2, linf and beff_l2 are taken over all trees together. */
#define ST_HIST 5
#define ST_N (ST_HIST + 64)

static int check_and_record(otree *t, const double *beff, double *st, int k) {
    double *sq = (double *)malloc((size_t)t->ntree * sizeof(double));
    double *mx = (double *)malloc((size_t)t->ntree * sizeof(double));
    restrict_all(t);
    leaf_norms(t, sq, mx);
    double rel = 0.0, s = 0.0, m = 0.0, bsq = 0.0;
    for (int tr = 0; tr < t->ntree; tr++) {
        double l2 = sqrt(sq[tr]);
        double r = beff[tr] > 0 ? l2 / beff[tr] : l2;
        t->tree_rel[tr] = r;
        if (r > rel || r != r) rel = r;
        s += sq[tr];
        bsq += beff[tr] * beff[tr];
        if (mx[tr] > m || mx[tr] != mx[tr]) m = mx[tr];
    }
    free(sq); free(mx);
    st[0] = rel; st[1] = sqrt(s); st[2] = m; st[3] = sqrt(bsq);
    if (k < 64) st[ST_HIST + k] = rel;
    return isfinite(rel) ? ORC_OK : ORC_ENOCONV;
}

static int iterate(otree *t, const double *beff, double tol, int max_cycles, const cycopts *o, double *st) {
    int stall = 0;
    for (int k = 1; st[0] > tol; k++) {
        if (k > max_cycles) { set_err("no convergence within max_cycles"); return ORC_ENOCONV; }
        double prev = st[0];
        int rc = vcycle(t, t->nlev, o);
        if (rc) return rc;
        st[4] = k;
        if ((rc = check_and_record(t, beff, st, k))) { set_err("non-finite residual"); return rc; }
        stall = st[0] >= prev ? stall + 1 : 0;
        if (stall >= 3) { set_err("residual stagnates"); return ORC_ENOCONV; }
    }
    return ORC_OK;
}

int oracle_fmg_solve(otree *t, double tol, int max_cycles, int n_down, int n_up, double *st) {
    cycopts o = {n_down, n_up};
    for (int q = 0; q < ST_N; q++) st[q] = 0.0;
    t->bad_lookup = 0;
    memset(t->f[F_PHI], 0, (size_t)t->n * BOX * sizeof(double));
    beff_norm(t, t->tree_beff);
    const double *beff = t->tree_beff;
    for (int l = t->nlev; l >= 2; l--) fas_down(t, l);
    int rc = coarse_solve(t);
    if (rc) return rc;
    for (int l = 2; l <= t->nlev; l++) {
        if ((rc = prolong_up(t, l))) return rc;
        if ((rc = vcycle(t, l, &o))) return rc;
    }
    if ((rc = check_and_record(t, beff, st, 0))) { set_err("non-finite residual"); return rc; }
    return iterate(t, beff, tol, max_cycles, &o, st);
}

/* warm start: n V-cycles from the current phi (or until tol when n <= 0) */
int oracle_vcycles(otree *t, int ncyc, double tol, int n_down, int n_up, double *st) {
    cycopts o = {n_down, n_up};
    for (int q = 0; q < ST_N; q++) st[q] = 0.0;
    t->bad_lookup = 0;
    beff_norm(t, t->tree_beff);
    const double *beff = t->tree_beff;
    int rc = check_and_record(t, beff, st, 0);
    if (rc) return rc;
    if (ncyc <= 0) return iterate(t, beff, tol, 50, &o, st);
    for (int k = 1; k <= ncyc; k++) {
        if ((rc = vcycle(t, t->nlev, &o))) return rc;
        st[4] = k;
        if ((rc = check_and_record(t, beff, st, k))) return rc;
    }
    return ORC_OK;
}

int oracle_residual(otree *t, double *out) {
    double st[ST_N];
    beff_norm(t, t->tree_beff);
    check_and_record(t, t->tree_beff, st, 0);
    for (int q = 0; q < 4; q++) out[q] = st[q];
    return t->bad_lookup ? ORC_ESTATE : ORC_OK;
}

/* relative residual of every tree at the last residual check */
int oracle_tree_rel(const otree *t, double *out) {
    memcpy(out, t->tree_rel, (size_t)t->ntree * sizeof(double));
    return ORC_OK;
}

/* single steps of the cycle, for step-by-step comparisons:
   1 smooth(level, arg sweeps), 2 fas_down(level), 3 prolong_up(level),
   4 coarse solve, 5 restriction of phi over all levels, 6 V-cycle(top=level,
   arg = sweeps each way), 7 residual of level into the RES field */
int oracle_step(otree *t, int op, int level, int arg) {
    if (op != 4 && op != 5 && (level < 1 || level > t->nlev)) return ORC_EINVAL;
    t->bad_lookup = 0;
    cycopts o = {arg, arg};
    int rc = ORC_OK;
    switch (op) {
    case 1: smooth(t, level, arg); break;
    case 2: if (level < 2) return ORC_EINVAL; fas_down(t, level); break;
    case 3: if (level < 2) return ORC_EINVAL; rc = prolong_up(t, level); break;
    case 4: rc = coarse_solve(t); break;
    case 5: restrict_all(t); break;
    case 6: rc = vcycle(t, level, &o); break;
    case 7: residual_level(t, level, 0); break;
    default: return ORC_EINVAL;
    }
    if (!rc && t->bad_lookup) rc = ORC_ESTATE;
    return rc;
}

/* composite operator on the leaf cells: phi <- x on leaf boxes (canonical
   order, natural layout), covered cells <- mean of children, then
   y = L phi on every leaf cell; homog = 1 drops the boundary data */
int oracle_apply(otree *t, const double *x, double *y, int homog) {
    int64_t q = 0;
    for (int64_t b = 0; b < t->n; b++) {
        if (t->child[8 * b] >= 0) continue;
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) t->f[F_PHI][b * BOX + AT(i, j, k)] = x[q++];
    }
    restrict_all(t);
    t->bad_lookup = 0;
    q = 0;
    for (int l = 1; l <= t->nlev; l++) {
        fill_ghosts(t, l, t->f[F_PHI], homog);
        double h = hlev(t, l), inv_h2 = 1.0 / (h * h);
        for (int64_t b = t->lstart[l]; b < t->lstart[l + 1]; b++) {
            if (t->child[8 * b] >= 0) continue;
            const double *p = t->f[F_PHI] + b * BOX;
            for (int k = 0; k < 8; k++)
                for (int j = 0; j < 8; j++)
                    for (int i = 0; i < 8; i++) y[q++] = lap_at(p, i, j, k, inv_h2);
        }
    }
    return t->bad_lookup ? ORC_ESTATE : ORC_OK;
}

int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------ fluid model */
/* One explicit stage of the drift-diffusion-reaction model (paper section
   2.2 for the equations for n_e and n_i, section 2.3 for the spatial
   discretisation of the fluxes and the coefficient table, section 2.4 for
   the stages and the time-step limits), on the leaf cells of the tree:
     out_e = wa * n0_e + wb * (n_e + dt * R_e),  R_e = -div(flux) + S,
     out_i = wa * n0_i + wb * (n_i + dt * S),    S = alpha(E) mu(E) E n_e,
   with E = |E| at the cell centre.  The flux of electrons across a face in
   the +a direction is v n_face - D(E*) (n_R - n_L) / h, where v = -mu(E*) E_a
   (E_a the face component, E* the mean of the two cells' |E|), and n_face the
   Koren-limited upwind value of the paper (psi(x) = max(0, min(1, (2+x)/6,
   x)) applied to the ratio of consecutive differences; a zero denominator
   gives no correction).  Densities outside a box: the same-level box's cell
   (its mean over children if it is refined), the mirrored interior cell at
   the domain boundary (zero gradient), and across a refinement boundary a
   fine ghost = 1/4 of the coarse cell containing it plus 1/4 of the coarse
   cell's three neighbours on the ghost's side (linear interpolation), capped
   at twice the coarse value.  |E| outside a box: the same-level cell, the
   mirrored cell, or the containing coarse cell.  On a face with a refined
   neighbour the flux is the mean of the four fine fluxes on it (the coarse
   flux is their sum per area).  Coefficients: linear interpolation in a
   table of (mu, D, alpha) at E = k * emax / (ntab - 1), the last entry
   beyond emax.  dt limit: the minimum over leaf cells of 0.5 / V,
   1 / (V + 6 D / h^2) and eps0 / (e mu n_e), V = sum over axes of the larger
   |v| of the cell's two faces divided by h. */

#define Q_ELEM 1.602176634e-19   /* C (CODATA 2018, exact) */
#define EPS_VAC 8.8541878128e-12 /* F/m (CODATA 2018) */

double oracle_koren_psi(double x) {
    double m = 1.0;
    if ((2.0 + x) / 6.0 < m) m = (2.0 + x) / 6.0;
    if (x < m) m = x;
    return m > 0.0 ? m : 0.0;
}

void oracle_fluid_coeffs(const double *tab, int ntab, double emax, double E, double *out3) {
    double x = E / emax * (double)(ntab - 1);
    int k = (int)floor(x);
    if (k >= ntab - 1 || !(x >= 0.0)) {
        int q = k >= ntab - 1 ? ntab - 1 : 0;
        for (int c = 0; c < 3; c++) out3[c] = tab[3 * q + c];
        return;
    }
    double w = x - (double)k;
    for (int c = 0; c < 3; c++) out3[c] = (1.0 - w) * tab[3 * k + c] + w * tab[3 * (k + 1) + c];
}

typedef struct {
    otree *t;
    const double *n;      /* electron density, natural [n][512], covered boxes = mean of children */
    const double *ef, *en;
    const double *tab;
    int ntab;
    double emax;
} fctx;

static int mirror(int I, int N) { return I < 0 ? -1 - I : (I >= N ? 2 * N - 1 - I : I); }

/* field value (natural layout) at level-l global cell G of a tree, mirrored
   into the domain; -1 box if no level-l box holds it */
static double nat_at(const otree *t, const double *f, int tree, int l, const int G[3], int *found) {
    int N = 8 << (l - 1), M[3];
    for (int a = 0; a < 3; a++) M[a] = mirror(G[a], N);
    int32_t b = find(t, tree, l, M[0] >> 3, M[1] >> 3, M[2] >> 3);
    *found = b >= 0;
    if (b < 0) return 0.0;
    return f[(int64_t)b * 512 + ((M[2] & 7) * 8 + (M[1] & 7)) * 8 + (M[0] & 7)];
}

/* electron density at level-l global cell G of the tree of box b */
static double dens(fctx *c, int tree, int l, const int G[3]) {
    int found;
    double v = nat_at(c->t, c->n, tree, l, G, &found);
    if (found) return v;
    int C[3] = {G[0] >> 1, G[1] >> 1, G[2] >> 1};
    double cc = nat_at(c->t, c->n, tree, l - 1, C, &found);
    if (!found) { c->t->bad_lookup = 1; return 0.0; }
    double s = 0.0;
    for (int a = 0; a < 3; a++) {
        int D[3] = {C[0], C[1], C[2]};
        D[a] += (G[a] & 1) ? 1 : -1;
        s += nat_at(c->t, c->n, tree, l - 1, D, &found);
        if (!found) c->t->bad_lookup = 1;
    }
    double g = 0.25 * cc + 0.25 * s;
    return g < 2.0 * cc ? g : 2.0 * cc;
}

/* |E| at level-l global cell G: same level, mirrored, or the coarse cell */
static double enorm(fctx *c, int tree, int l, const int G[3]) {
    int found;
    double v = nat_at(c->t, c->en, tree, l, G, &found);
    if (found) return v;
    int C[3] = {G[0] >> 1, G[1] >> 1, G[2] >> 1};
    v = nat_at(c->t, c->en, tree, l - 1, C, &found);
    if (!found) c->t->bad_lookup = 1;
    return v;
}

/* flux in the +a direction across face f (between local cells f-1 and f)
   of box b at tangential cell (u, v); *vel receives the face velocity */
static double face_flux(fctx *c, int64_t b, int a, int f, int u, int v, double *vel) {
    otree *t = c->t;
    int l = t->lev[b], tree = t->tid[b];
    int B[3] = {t->bx[b], t->by[b], t->bz[b]}, t1, t2;
    tang_axes(a, &t1, &t2);
    double h = hlev(t, l);
    /* velocity from this box's face field */
    int G[3];
    G[t1] = 8 * B[t1] + u;
    G[t2] = 8 * B[t2] + v;
    G[a] = 8 * B[a] + f - 1;
    double eL = enorm(c, tree, l, G);
    G[a] = 8 * B[a] + f;
    double eR = enorm(c, tree, l, G);
    double co[3];
    oracle_fluid_coeffs(c->tab, c->ntab, c->emax, 0.5 * (eL + eR), co);
    double vx = -co[0] * c->ef[((b * 3 + a) * 9 + f) * 64 + v * 8 + u];
    *vel = vx;
    if (f == 0 || f == 8) {
        int32_t N = t->nbr[6 * b + 2 * a + (f == 8)];
        if (N >= 0 && t->child[8 * (int64_t)N] >= 0) {
            /* refined neighbour: mean of the four fine fluxes on this face */
            double s = 0.0, dummy;
            for (int dv = 0; dv < 2; dv++)
                for (int du = 0; du < 2; du++) {
                    int F[3];
                    F[t1] = 2 * G[t1] + du;
                    F[t2] = 2 * G[t2] + dv;
                    F[a] = f == 8 ? 16 * (B[a] + 1) : 16 * B[a] - 1;  /* fine cell beyond the face */
                    int32_t fb = find(t, tree, l + 1, F[0] >> 3, F[1] >> 3, F[2] >> 3);
                    if (fb < 0) { t->bad_lookup = 1; continue; }
                    s += face_flux(c, fb, a, f == 8 ? 0 : 8, F[t1] & 7, F[t2] & 7, &dummy);
                }
            return 0.25 * s;
        }
    }
    double n[4];
    for (int q = 0; q < 4; q++) {
        G[a] = 8 * B[a] + f - 2 + q;
        n[q] = dens(c, tree, l, G);
    }
    double nf;
    if (vx < 0.0) {
        double den = n[2] - n[1];
        nf = n[2] - (den == 0.0 ? 0.0 : oracle_koren_psi((n[3] - n[2]) / den) * den);
    } else {
        double den = n[2] - n[1];
        nf = n[1] + (den == 0.0 ? 0.0 : oracle_koren_psi((n[1] - n[0]) / den) * den);
    }
    return vx * nf - co[1] * (n[2] - n[1]) / h;
}

int oracle_fluid_stage(otree *t, const double *ne, const double *ni, const double *n0e,
                       const double *n0i, const double *e_face, const double *e_norm,
                       const double *tab, int ntab, double emax, double dt, double wa, double wb,
                       double *oute, double *outi, double *dtlim) {
    if (ntab < 2 || !(emax > 0.0)) return ORC_EINVAL;
    t->bad_lookup = 0;
    size_t sz = (size_t)t->n * 512;
    double *nr = (double *)malloc(sz * sizeof(double));
    if (!nr) return ORC_ENOMEM;
    memcpy(nr, ne, sz * sizeof(double));
    /* covered cells: mean of their children, finest levels first */
    for (int l = t->nlev; l >= 2; l--)
        for (int64_t p = t->lstart[l - 1]; p < t->lstart[l]; p++) {
            if (t->child[8 * p] < 0) continue;
            for (int k = 0; k < 8; k++)
                for (int j = 0; j < 8; j++)
                    for (int i = 0; i < 8; i++) {
                        const double *fc = nr + (int64_t)t->child[8 * p + (i >> 2) + 2 * (j >> 2) + 4 * (k >> 2)] * 512;
                        double s = 0.0;
                        for (int dk = 0; dk < 2; dk++)
                            for (int dj = 0; dj < 2; dj++)
                                for (int di = 0; di < 2; di++)
                                    s += fc[((2 * (k & 3) + dk) * 8 + 2 * (j & 3) + dj) * 8 + 2 * (i & 3) + di];
                        nr[p * 512 + (k * 8 + j) * 8 + i] = 0.125 * s;
                    }
        }
    fctx c = {t, nr, e_face, e_norm, tab, ntab, emax};
    double lim = INFINITY;
#pragma omp parallel for schedule(dynamic, 4) reduction(min : lim)
    for (int64_t b = 0; b < t->n; b++) {
        if (t->child[8 * b] >= 0) continue;
        double h = hlev(t, t->lev[b]);
        /* flux and velocity on every face of the box */
        double F[3][9][64], V[3][9][64];
        for (int a = 0; a < 3; a++)
            for (int f = 0; f <= 8; f++)
                for (int q = 0; q < 64; q++) F[a][f][q] = face_flux(&c, b, a, f, q & 7, q >> 3, &V[a][f][q]);
        for (int k = 0; k < 8; k++)
            for (int j = 0; j < 8; j++)
                for (int i = 0; i < 8; i++) {
                    int64_t x = b * 512 + (k * 8 + j) * 8 + i;
                    int idx[3] = {i, j, k};
                    double div = 0.0, vs = 0.0;
                    for (int a = 0; a < 3; a++) {
                        int t1, t2;
                        tang_axes(a, &t1, &t2);
                        int q = idx[t2] * 8 + idx[t1];
                        div += (F[a][idx[a] + 1][q] - F[a][idx[a]][q]) / h;
                        double v0 = fabs(V[a][idx[a]][q]), v1 = fabs(V[a][idx[a] + 1][q]);
                        vs += (v0 > v1 ? v0 : v1) / h;
                    }
                    double E = e_norm[x], co[3];
                    oracle_fluid_coeffs(tab, ntab, emax, E, co);
                    double S = co[2] * co[0] * E * ne[x];
                    oute[x] = wa * n0e[x] + wb * (ne[x] + dt * (S - div));
                    outi[x] = wa * n0i[x] + wb * (ni[x] + dt * S);
                    double cand = INFINITY;
                    if (vs > 0.0) cand = 0.5 / vs;
                    double ad = 1.0 / (vs + 6.0 * co[1] / (h * h));
                    if (ad < cand) cand = ad;
                    if (ne[x] > 0.0 && co[0] > 0.0) {
                        double dr = EPS_VAC / (Q_ELEM * co[0] * ne[x]);
                        if (dr < cand) cand = dr;
                    }
                    if (cand < lim) lim = cand;
                    /* Poisson right-hand side lap(phi) = -e (n_i - n_e) / eps0 */
                    t->f[F_RHS][b * BOX + AT(i, j, k)] = -Q_ELEM * (outi[x] - oute[x]) / EPS_VAC;
                }
    }
    free(nr);
    if (dtlim) *dtlim = lim;
    return t->bad_lookup ? ORC_ESTATE : ORC_OK;
}
