/*
 * mg.h - C ABI of the MI355X octree multigrid Poisson solver.
 *
 * The library solves lap(phi) = b on the leaf cells of a block-structured
 * octree of 8^3-cell boxes (paper section 2.1.1), with Dirichlet or Neumann
 * conditions on the six faces of a cubic domain.  b is the caller's
 * -rho/eps0 (the field equation of section 2.2); the library never applies
 * physical constants.  The solver is geometric multigrid in
 * full-approximation-scheme form with an FMG cycle, V-cycles and red-black
 * Gauss-Seidel smoothing (section 2.1.2).
 *
 * Conventions shared by every call:
 *   - A tree's root is one 8^3 box at level 1; a box at level l has integer
 *     coordinates 0 <= i, j, k < 2^(l-1) and cell spacing
 *     len / (8 * 2^(l-1)).  A refined box has all 8 children; neighbouring
 *     boxes (over all 26 neighbours) differ by at most one level (proper
 *     nesting, section 2.1.1).
 *   - Boxes are renumbered into a canonical order: by level, then tree id,
 *     then the Morton index of (i, j, k) (bit b of i, j, k goes to bit 3b,
 *     3b+1, 3b+2).  Every per-box array the library reads or writes is in
 *     canonical order; MG_IDX_ORDER maps canonical position -> caller index.
 *   - Cell data crossing the ABI ("natural layout") is [box][k][j][i],
 *     x fastest, 512 doubles per box.
 *   - All device memory is owned by the caller.  mg_tree_info() reports the
 *     workspace size; mg_tree_bind() attaches it.  The library does not
 *     allocate device memory; it owns only host-side tables.
 *   - Work is enqueued on the stream given to mg_tree_bind().  Calls that
 *     return scalars to the host (mg_fmg_solve, mg_vcycle, mg_residual)
 *     synchronise that stream before returning.
 *   - Calls on one tree are not re-entrant; different trees are independent.
 *   - Every call returns MG_OK (0) or a negative code; mg_last_error() gives
 *     a thread-local message naming the offending box, face or argument.
 */
#ifndef MG_H
#define MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MG_OK = 0,
    MG_EINVAL = -1,   /* bad argument, duplicate box, coordinate out of range */
    MG_ENESTING = -2, /* 2:1 proper nesting violated (26-neighbourhood)      */
    MG_ENOMEM = -3,   /* host allocation failed or workspace too small        */
    MG_EHIP = -4,     /* a HIP runtime call failed                            */
    MG_ENOCONV = -5,  /* no convergence: max_cycles, non-finite or stagnating */
    MG_ESTATE = -6,   /* call out of order (e.g. no workspace bound)          */
    MG_ETOPO = -7     /* missing root, missing parent or incomplete siblings  */
};

enum { MG_DIRICHLET = 0, MG_NEUMANN = 1 };

/* Domain [lo, lo+len]^3.  Faces are ordered -x, +x, -y, +y, -z, +z.
 * Dirichlet ghosts are 2 g - phi_in with g = bc_val[face] (or the per-cell
 * values of MG_FIELD_BCVAL when per_cell_bc is set); Neumann ghosts are
 * phi_in (zero normal derivative).  At least one face must be Dirichlet. */
typedef struct {
    double lo[3];
    double len;
    int32_t bc_type[6];
    double bc_val[6];
    int32_t per_cell_bc; /* 1: reserve [n][6][64] per-face-cell Dirichlet data */
} mg_domain;

typedef struct mg_tree mg_tree;

/* Sizes of a created tree. */
typedef struct {
    int64_t n_boxes;
    int32_t n_levels;
    int32_t n_trees;
    int64_t n_leaf_boxes;
    int64_t n_leaf_cells;        /* unknowns: 512 * n_leaf_boxes            */
    int64_t n_cf_faces;          /* box faces on a refinement boundary      */
    int64_t level_start[17];     /* boxes of level l: [level_start[l-1], level_start[l]) */
    int64_t workspace_bytes;     /* device bytes mg_tree_bind() needs       */
} mg_tree_info_t;

/*
 * mg_tree_create - validate a box list and build the tree's host tables.
 *   n       number of boxes (> 0)
 *   level   [n] host int32, 1 <= level <= 15
 *   ijk     [n*3] host int32, box coordinates (i, j, k) per box
 *   tree    [n] host int32 tree ids 0..T-1 (each tree needs a root), or NULL
 *   dom     domain and boundary conditions
 * Host-only: no device call is made.  Errors: MG_EINVAL (range, duplicates,
 * bad boundary types, all-Neumann domain), MG_ETOPO, MG_ENESTING.  The
 * arrays are copied; the caller keeps ownership.  *out is set on success.
 */
int mg_tree_create(mg_tree **out, const mg_domain *dom, int64_t n, const int32_t *level,
                   const int32_t *ijk, const int32_t *tree);
/* mg_tree_destroy synchronises the bound stream (work enqueued without a
 * host wait may still be running), then frees the host state. */
int mg_tree_destroy(mg_tree *t);
int mg_tree_info(const mg_tree *t, mg_tree_info_t *info);

/*
 * mg_tree_bind - attach a caller-owned device workspace and a stream.
 *   ws      device pointer, 256-byte aligned, >= info.workspace_bytes
 *   stream  hipStream_t (as void*), e.g. torch.cuda.current_stream()
 * Uploads the index tables into the workspace with one copy from a pinned
 * host staging buffer, zeroes the fields, and waits for both on the stream
 * before returning.  The staging buffer (the tables' size, a few hundred
 * bytes per box) is pooled: the library keeps the largest one it has used
 * until the process ends.  The workspace must stay valid until rebind or
 * destroy.  On an error the tree is left unbound (MG_ESTATE from the calls
 * that need a workspace until a bind succeeds).
 */
int mg_tree_bind(mg_tree *t, void *ws, int64_t ws_bytes, void *stream);

/* Index tables (host output, canonical order), for inspection and tests. */
enum {
    MG_IDX_ORDER = 0,  /* [n]    caller index of each canonical box            */
    MG_IDX_LEVEL = 1,  /* [n]                                                  */
    MG_IDX_IJK = 2,    /* [n*3]                                                */
    MG_IDX_TREE = 3,   /* [n]                                                  */
    MG_IDX_PARENT = 4, /* [n]    -1 for roots                                  */
    MG_IDX_CHILD = 5,  /* [n*8]  child (i&1)+2(j&1)+4(k&1), -1 for leaves      */
    MG_IDX_NBR = 6,    /* [n*6]  same-level face neighbour, -1 refinement
                                 boundary (coarser neighbour), -2 domain face  */
    MG_IDX_CFQ = 7     /* [n*6]  coarser box across a refinement boundary, -1  */
};
int mg_tree_index(const mg_tree *t, int what, int32_t *host_out);

/*
 * Field transfer between caller memory in natural layout and the library's
 * internal storage (colour-split: per box, the 256 cells with even i+j+k,
 * then the 256 with odd i+j+k).
 *   which   MG_FIELD_PHI (solution, all boxes), MG_FIELD_RHS (b; only leaf
 *           boxes matter, covered boxes are overwritten by the solver),
 *           MG_FIELD_OLD (the coarse values a down-leg keeps for the
 *           correction; scratch: a down-leg writes it only where a
 *           prolongation reads it, i.e. on boxes with children and on leaf
 *           boxes with a same-level face or edge neighbour that has children),
 *           MG_FIELD_E32 / _R32 / _OLD32 (FP32 fields, rounded on the way in),
 *           MG_FIELD_BCVAL ([n][6][64] Dirichlet values at the face-cell
 *           centres; per_cell_bc must be set; tangential axes in increasing
 *           order, first fastest)
 *   dev     device pointer to n*512 doubles (n*6*64 for BCVAL)
 * Asynchronous on the bound stream.
 */
enum { MG_FIELD_PHI = 0, MG_FIELD_RHS = 1, MG_FIELD_OLD = 2, MG_FIELD_BCVAL = 3,
       /* FP32 fields of the mixed-precision correction solve (converted to and
          from FP64 natural-layout arrays): correction, its right-hand side,
          and its old copy */
       MG_FIELD_E32 = 4, MG_FIELD_R32 = 5, MG_FIELD_OLD32 = 6 };
int mg_field_set(mg_tree *t, int which, const double *dev);
int mg_field_get(const mg_tree *t, int which, double *dev);

/*
 * mg_field - borrowed device pointer to a field's own storage in the bound
 * workspace (no copy), for callers that read or write the fields in place.
 *   which          MG_FIELD_PHI, _RHS, _OLD (dtype MG_DTYPE_F64), MG_FIELD_E32,
 *                  _R32, _OLD32 (MG_DTYPE_F32), MG_FIELD_BCVAL (F64, only with
 *                  per_cell_bc)
 *   dtype          must be the field's storage type (MG_EINVAL otherwise)
 *   dev_ptr        out: device pointer; valid until rebind or destroy
 *   n_elems        out (may be NULL): number of elements
 *   level_offsets  out (may be NULL): [n_levels + 1], first box of each level
 *                  in canonical order (level l: [lo[l-1], lo[l]))
 * Cell fields hold box b (canonical order) at elements [512 b, 512 b + 512),
 * and cell (i, j, k) of a box at ((i + j + k) & 1) * 256 + (k * 8 + j) * 4 +
 * (i >> 1): the colour-split order the red-black sweeps stream (the 256
 * cells with even i + j + k first), not the natural order of mg_field_set.
 * BCVAL is [n][6][64] as in mg_field_set.  The solver keeps values derived
 * from PHI (the refinement-boundary interpolation); a call to mg_field marks
 * them stale, so a caller that writes through the pointer calls mg_field
 * again after writing and before the next solve call.
 */
enum { MG_DTYPE_F64 = 0, MG_DTYPE_F32 = 1 };
int mg_field(mg_tree *t, int which, int dtype, void **dev_ptr, int64_t *n_elems, int64_t *level_offsets);

/* Solver options and statistics.
 * MG_FP64: the multigrid cycles run on the FP64 solution.
 * MG_MIXED: iterative refinement.  Each step computes the FP64 leaf residual
 *   r = b - L phi (after covered cells are reset to the mean of their
 *   children), stores it rounded to FP32 as the right-hand side of the
 *   correction problem L e = r with homogeneous boundary data, solves that
 *   in FP32 from e = 0 (an FMG pass in the first step, one V-cycle after),
 *   and updates phi += e in FP64.  The root solve stays FP64; the stopping
 *   test is the FP64 one, so the result meets the same tolerance.
 * MG_LEARNED: the FP64 solve with a learned correction step after every
 *   V-cycle that does not meet the tolerance (include/mg_nn.h: the network
 *   and its workspace are attached with mg_nn_bind; mg_fmg_solve only). */
enum { MG_FP64 = 0, MG_MIXED = 1, MG_LEARNED = 2 };
typedef struct {
    int32_t precision;   /* MG_FP64                                          */
    int32_t n_down;      /* Gauss-Seidel sweeps before restriction (2)       */
    int32_t n_up;        /* sweeps after prolongation (2)                    */
    int32_t max_cycles;  /* V-cycles after the FMG pass (50)                 */
    double rel_tol;      /* stop when |r|_2,V / |b_eff|_2,V <= rel_tol (1e-8)*/
    int32_t graphs;      /* 1: record the FMG pass and the V-cycle + residual
                            check once as HIP graphs and replay them on the
                            bound stream; 0: launch kernel by kernel.  Both
                            run the same kernels in the same order.  (1)     */
    int32_t final_check_only; /* mg_vcycle with n_cycles > 0 in MG_FP64: 1
                            runs the n cycles back to back and the residual
                            check only after the last (the time step of
                            section 2.1.2 needs no test in between); phi is
                            the same bits as with 0, rel_hist[0 .. n-1] are
                            NaN.  0 (default): a check before and after every
                            cycle.  Ignored elsewhere (mixed precision needs
                            each step's residual).                          */
    int32_t learned_placement; /* MG_LEARNED / mg_learned_solve: 0 (default) a
                            learned step after every V-cycle that does not
                            stop the solve; 1 a learned step on each level's
                            leaf boxes after that level's up-sweeps
                            (include/mg_nn.h)                               */
} mg_solve_opts;

typedef struct {
    int32_t n_vcycles;         /* V-cycles run after the FMG pass (MG_MIXED:
                                  refinement steps)                            */
    int32_t status;
    double rel_res;            /* final relative residual                      */
    double l2;                 /* volume-weighted L2 norm of the leaf residual */
    double linf;               /* max norm of the leaf residual                */
    double beff_l2;            /* norm of the residual of phi = 0              */
    double rel_hist[64];       /* after the FMG pass [0] and each V-cycle      */
    double t_ms;               /* host wall time of the call                   */
    int32_t nn_accepted;       /* MG_LEARNED: learned steps kept               */
    int32_t nn_fell_back;      /* MG_LEARNED: cycle at which the learned step
                                  was dropped for plain V-cycles, 0 if never   */
    int32_t launches_fmg;      /* mg_fmg_solve with graphs: kernel launches of
                                  the recorded FMG sequence (FP64: phi <- 0,
                                  FMG pass, stopping test; MG_MIXED: start and
                                  first correction step); 0 otherwise          */
    int32_t launches_cycle;    /* the same for one further cycle with its
                                  stopping test (FP64: V-cycle; MG_MIXED: FP32
                                  V-cycle and FP64 update); 0 if none ran      */
} mg_solve_stats;

void mg_default_opts(mg_solve_opts *o);

/*
 * mg_fmg_solve - solve from phi = 0: one FMG pass (section 2.1.2: the
 * initial potential), then V-cycles until the relative residual is below
 * rel_tol.  The residual is the leaf residual after covered cells are reset
 * to the mean of their children; its volume-weighted L2 norm is compared
 * with that of the residual of phi = 0.  Returns MG_ENOCONV after
 * max_cycles V-cycles, on a non-finite residual, or when it fails to
 * decrease for 3 cycles in a row.  stats may be NULL.
 */
int mg_fmg_solve(mg_tree *t, const mg_solve_opts *o, mg_solve_stats *s);

/*
 * mg_vcycle - n V-cycles warm-started from the current phi (section 2.1.2:
 * later updates of the potential reuse the previous one), then the residual
 * check.  n <= 0 iterates until rel_tol (at most max_cycles).  With stats
 * NULL, n > 0 and MG_FP64 no residual norm is computed and the host does not
 * wait for the GPU (the time step's field solves); phi is the same bits.
 */
int mg_vcycle(mg_tree *t, const mg_solve_opts *o, int n_cycles, mg_solve_stats *s);

/*
 * mg_efield - electric field of the current phi (section 2.3: E = -grad phi,
 * components on the cell faces, strength at the cell centres).  Covered
 * cells of phi are first reset to the mean of their children (as before a
 * residual check); each box then uses its own ghosts (same-level neighbour,
 * boundary condition, refinement-boundary interpolation), as the solver does.
 *   e_face  device, n*3*9*64 doubles, or NULL: for box b (canonical order),
 *           axis a (x, y, z) and face f = 0..8 across the box (face f lies
 *           between cells f-1 and f; faces 0 and 8 on the box boundary),
 *           E_a = (phi(f-1) - phi(f)) / h at index ((b*3 + a)*9 + f)*64 +
 *           v*8 + u, with u and v the cell indices along the other two axes
 *           in increasing order.
 *   e_norm  device, n*512 doubles, or NULL: sqrt(Ex^2 + Ey^2 + Ez^2) at each
 *           cell centre (natural order, x fastest), each component the mean
 *           of the cell's two face values.
 * Every box is written, covered ones included.  Asynchronous on the bound
 * stream; MG_EINVAL if both outputs are NULL.
 */
int mg_efield(mg_tree *t, double *e_face, double *e_norm);

/*
 * Mesh adaptation (section 2.5), one step at a time, as the charge moves:
 *   1. mg_refine_scores: per box, 27 refinement scores of the right-hand
 *      side on the GPU: scores[b*27 + r] = max |b| h^2 over the box's cells in
 *      region r = (sx+1) + 3(sy+1) + 9(sz+1), where along each axis s = -1
 *      takes cells 0..2, s = +1 cells 5..7 and s = 0 all cells (r = 13: the
 *      whole box; the others: the cells within 3 of a face, edge or corner).
 *      Only leaf boxes' scores are meaningful (the solver overwrites b on
 *      covered boxes).  scores: device, n*27 doubles.  Asynchronous.
 *   2. mg_regrid_plan (host): the new box list.  A leaf box below max_level
 *      is refined when |b| h^2 > c3 at one of its cells or at a cell of a
 *      same-level leaf neighbour within 3 cells (the paper's space-charge
 *      criterion h > sqrt(c3 eps0 / |rho|) with its 3-cell buffer).  The 8
 *      children of a box are removed when they are leaves, none is refined,
 *      no cell of theirs or of a same-level leaf neighbour within 3 cells
 *      exceeds deref*c3 (the paper: 1/8), their cell size is below h_deref
 *      (the paper's Delta x_deref; +inf: no floor), and no box two levels
 *      finer would touch the parent.
 *      Then 2:1 nesting over 26 neighbours is restored by refining coarse
 *      leaves.  scores: host copy of step 1.  Writes n_out boxes (level,
 *      ijk[3], tree; any order) if n_out <= cap, else MG_ENOMEM with n_out set.
 *   3. mg_tree_create + mg_tree_bind on the list, then mg_transfer.
 * mg_transfer: phi of `to` from `from` (same domain and trees): covered cells
 * of `from` are first reset to the mean of their children; boxes present in
 * both (same tree, level, position) are copied; the others, level by level,
 * are interpolated from their parent in `to` by the prolongation stencil
 * 1/4 p(C) + 1/4 (p(C+s_x) + p(C+s_y) + p(C+s_z)) on phi (exact for linear
 * potentials), with the parent's ghosts outside it.  Runs on to's stream and
 * synchronises it; `from` must not be in use meanwhile.  to's right-hand side
 * is the caller's (set it from the new boxes).  MG_EINVAL if a tree of `to`
 * has no root in `from` or the domains differ.
 */
int mg_refine_scores(mg_tree *t, double *scores);
int mg_regrid_plan(const mg_tree *t, const double *scores, double c3, double deref, double h_deref,
                   int max_level, int64_t cap, int32_t *level, int32_t *ijk, int32_t *tree, int64_t *n_out);
/*
 * The criterion of step 2 tests, per leaf box, one value: the largest score
 * over its cells and the cells of its same-level leaf neighbours within 3
 * cells (the 3-cell buffer of section 2.5).  mg_refine_near forms it on the
 * GPU from step 1's device scores:
 *   near[b] = max over o in the 27-neighbourhood of scores[N*27 + 26 - o]
 *   for the same-level leaf neighbour N = b + o (b's own scores[b*27 + 13]
 *   where there is none or it is refined), 0 for a refined box.
 *   scores, near: device, n*27 and n doubles.  Asynchronous, on the bound
 *   stream; the maximum is taken in the order of mg_regrid_plan's, so near
 *   is the same bits as the value the host plan forms.
 * mg_regrid_plan_near is mg_regrid_plan from a host copy of near (n doubles
 * instead of n*27): the same box list.  Errors as mg_regrid_plan.
 */
int mg_refine_near(mg_tree *t, const double *scores, double *near);
int mg_regrid_plan_near(const mg_tree *t, const double *near, double c3, double deref, double h_deref,
                        int max_level, int64_t cap, int32_t *level, int32_t *ijk, int32_t *tree,
                        int64_t *n_out);
int mg_transfer(mg_tree *from, mg_tree *to);

/*
 * Fluid model: the drift-diffusion-reaction equations (section 2.2) for the
 * electron and ion densities (SI units, m^-3), advanced with the explicit
 * trapezoidal rule and its time-step limits (section 2.4).  The fluxes, the
 * limiter, the refinement-boundary treatment and the coefficient table are
 * the spatial discretisation of section 2.3.  Densities are device arrays in natural layout
 * [box][k][j][i] over all boxes; only leaf boxes carry data (covered boxes
 * are overwritten with the mean of their children).  Per stage, on every
 * leaf cell:
 *   out_e = wa n0_e + wb (n_e + dt (S - div F)),  out_i = wa n0_i + wb (n_i + dt S),
 *   S = alpha(|E|) mu(|E|) |E| n_e,
 *   F (+a direction) = v n_face - D(E*) (n_R - n_L) / h,  v = -mu(E*) E_a,
 * E_a the face component of the field and E* the mean |E| of the two cells;
 * n_face is the upwind value corrected with the Koren limiter
 * psi(x) = max(0, min(1, (2 + x)/6, x)) of the ratio of consecutive
 * differences (a zero denominator gives no correction).  Ghosts: the
 * same-level cell, the mirrored cell at the domain boundary (zero
 * gradient), or across a refinement boundary 1/4 of the coarse cell holding
 * the ghost plus 1/4 of its three neighbours on the ghost's side, capped at
 * twice the coarse value.  The flux on the coarse side of a refinement
 * boundary is the mean of the four fine fluxes on it.  The stage also sets
 * the solver's right-hand side on leaf cells to -e (n_i - n_e) / eps0 of the
 * output, and gives the time-step bound min over leaf cells of 0.5 / V,
 * 1 / (V + 6 D / h^2) and eps0 / (e mu n_e), V = sum over axes of the larger
 * |v| of the cell's two faces, divided by h.  A stage with a non-finite
 * output density gives a NaN bound.
 *
 * mg_fluid_workspace_bytes: size of the fluid workspace for n_table table
 *   entries (-1 on bad arguments).
 * mg_fluid_bind: attaches it (device, 256-byte aligned, caller-owned) and
 *   uploads the transport table (host, [n_table][3] = (mu, D, alpha) at
 *   E = k e_max / (n_table - 1); linear interpolation, the last entry beyond
 *   e_max).  The tree must be bound.  Synchronises the tree's stream.
 * mg_fluid_stage: one stage; e_face [n][3][9][64] and e_norm [n][512] as
 *   mg_efield writes them; ne is read and its covered boxes are overwritten;
 *   out_e, out_i (leaf boxes written) must not alias the inputs.  dt_limit
 *   (host, may be NULL): the time-step bound, which synchronises the stream.
 * mg_fluid_step: one time step in place: keep (ne, ni), a stage with
 *   (wa, wb) = (0, 1) into the workspace, n_vcycles warm-started V-cycles and
 *   the field, a stage with (1/2, 1/2) from that result back into (ne, ni),
 *   n_vcycles V-cycles (no residual norms and no host round trip: phi is
 *   the same bits as after mg_vcycle).  phi must be the potential of
 *   (ne, ni) on entry.
 *   dt_next (host, may be NULL) = 0.9 x the bound of the second stage.
 *   MG_ENOCONV when a density of the step is not finite (a diverging step,
 *   e.g. dt far above the bound); the densities and phi are then not usable.
 * MG_ESTATE without a bound fluid workspace; MG_EINVAL on bad arguments.
 */
int64_t mg_fluid_workspace_bytes(const mg_tree *t, int32_t n_table);
int mg_fluid_bind(mg_tree *t, void *ws, int64_t bytes, const double *table, int32_t n_table, double e_max);
int mg_fluid_stage(mg_tree *t, const double *e_face, const double *e_norm, double *ne, const double *ni,
                   const double *n0e, const double *n0i, double dt, double wa, double wb, double *out_e,
                   double *out_i, double *dt_limit);
int mg_fluid_step(mg_tree *t, double *ne, double *ni, double dt, int32_t n_vcycles, double *dt_next);

/* Relative residual, L2 and max norms of the current phi on the leaf cells,
 * as the stopping test of mg_fmg_solve takes them (a reading of the
 * residual norm, which the paper does not give): covered cells first
 * reset to the mean of their children; r = b - L phi with the ghosts of the
 * solver; l2 = sqrt(sum r^2 h^3) over leaf cells (volume-weighted); linf =
 * max |r|; rel = l2 divided by the l2 of the residual of phi = 0 (boundary
 * data included), for a forest the largest over the trees.  Synchronises. */
int mg_residual(mg_tree *t, double *rel, double *l2, double *linf);

/*
 * Forests: the trees of one mg_tree are independent problems solved together
 * (every launch covers the boxes of one level of all trees).  The stopping
 * test applies to every tree: rel_res is the largest relative residual over
 * the trees, each relative to its own residual of phi = 0.
 * mg_tree_residuals writes each tree's relative residual at the last
 * residual check into rel[n_trees] (host memory).
 */
int mg_tree_residuals(const mg_tree *t, double *rel);

/*
 * mg_step - run one step of the cycle (diagnostics and step-by-step
 * comparisons).  op: MG_OP_SMOOTH (level, arg sweeps), MG_OP_FAS_DOWN
 * (residual, restriction, old copy and coarse right-hand side from level to
 * level-1), MG_OP_PROLONG (add the prolonged coarse correction to level),
 * MG_OP_COARSE (exact root solve), MG_OP_RESTRICT_ALL (covered cells <-
 * mean of children, all levels), MG_OP_VCYCLE (V-cycle with level on top,
 * arg sweeps each way).
 */
enum { MG_OP_SMOOTH = 1, MG_OP_FAS_DOWN = 2, MG_OP_PROLONG = 3, MG_OP_COARSE = 4,
       MG_OP_RESTRICT_ALL = 5, MG_OP_VCYCLE = 6,
       MG_OP_F32 = 0x100 /* or-ed in: apply the step to the FP32 correction
                            fields (homogeneous boundary data)            */ };
int mg_step(mg_tree *t, int op, int level, int arg);

/*
 * Kernel timing of the dominant kernel, the red-black Gauss-Seidel
 * half-sweep.  While enabled, the solver launches kernel by kernel (no graph
 * replay) and brackets the consecutive half-sweeps of every smoothing call
 * with a pair of HIP events on the bound stream.  mg_timing_read()
 * synchronises the stream and returns, summed over all pairs since the last
 * read, the half-sweep launch count, the event-pair time and the algorithmic
 * bytes (per box and half-sweep: this colour's right-hand side and the other
 * colour's solution read, this colour's solution written,
 * 3 x 256 x 8 = 6144 bytes in FP64, 3072 in FP32), in total and per level;
 * then it resets the sums.
 */
typedef struct {
    int64_t launches;
    double total_ms;
    double alg_bytes;
    int64_t level_launches[16]; /* the same sums per level (index level-1) */
    double level_ms[16];
    double level_bytes[16];
} mg_kernel_timing_t;
int mg_timing_enable(mg_tree *t, int enable);
int mg_timing_read(mg_tree *t, mg_kernel_timing_t *out);

/*
 * Autotuner of the Gauss-Seidel launch schedule.  Variant v = 2c + x:
 *   c = 0, 1, 2: half-sweeps (one colour per launch) with 1, 2 or 4 cells per
 *         thread;
 *   c = 3: fused sweeps (both colours in one launch: each box recomputes the
 *         red face layers of its same-level neighbours from the old field;
 *         sweeps ping-pong between the field and a buffer in the workspace,
 *         so a level is smoothed in pairs of sweeps and an odd last sweep
 *         runs as half-sweeps of variant 3);
 *   c = 4: half-sweeps over octets of sibling boxes (one workgroup per 16^3
 *         octet; faces between siblings come from LDS);
 *   c = 5, 6: half-sweeps by at most 2048 or 4096 persistent workgroups,
 *         each walking a run of boxes with the next box's data in flight;
 *   x = 1 selects the XCD-aware mapping of workgroups to boxes.
 * The entry of level 1 (never smoothed) selects how the two coarsest levels
 * run: 0 = step by step, any other value = one launch per V-cycle with one
 * workgroup per tree (the default); the tuner reports it as set.  For every
 * level >= 2 the tuner times reps half-sweeps of each variant (reps / 2
 * fused sweeps) with HIP events on the bound stream and keeps the fastest;
 * reps must be even, 2..1000.  precision selects the FP64 or the FP32
 * (MG_MIXED) kernels.  The field being swept is parked and restored, so the
 * solver state is unchanged.  schedule (host, [n_levels], may be NULL)
 * receives the chosen variant per level (index level-1); mg_set_schedule
 * applies a stored schedule (e.g. from a cache keyed by the tree's level
 * sizes) and rejects entries outside 0..MG_GSRB_VARIANTS-1.  All variants
 * compute the same values.
 */
#define MG_GSRB_VARIANTS 14
int mg_autotune(mg_tree *t, int precision, int reps, int32_t *schedule);
int mg_set_schedule(mg_tree *t, int precision, const int32_t *schedule);

/*
 * mg_set_fusion - which fused launch sequences the cycle uses (all by
 * default).  Every combination computes the same bits; the flags exist to
 * compare and time the sequences.
 *   MG_FUSE_PROLONG: on a level smoothed by half-sweeps, the prolongation of
 *     the coarse correction (section 2.1.2's interpolation between levels) is
 *     not a pass of its own: the first red and black half-sweeps after it form
 *     each prolonged value they read from the unprolonged field and the
 *     parent's correction, which saves reading and writing the level once.
 *   MG_FUSE_BEFF: the norm of the residual of phi = 0 (the divisor of the
 *     relative residual) comes from the FMG pass's top-down restriction,
 *     which starts from phi = 0: it reads no phi and also sums the norms of
 *     the leaf boxes, instead of a norm pass of its own.
 *   MG_FUSE_RESTRICT: before a stopping test, the restriction of the leaf
 *     boxes' values onto their parents' cells (the covered cells that the
 *     test's residual and c_hat read) is done by each level's last black
 *     half-sweep of the cycle, on the levels whose sweep variant is a
 *     one-box half-sweep, instead of by a pass of its own.
 *   MG_FUSE_IR: in the mixed-precision solve, the FP64 update phi += e and
 *     that restriction are done by the FP32 correction cycle's last black
 *     half-sweep of each level (from the lowest level of the run up to the
 *     finest whose sweep variant has it), instead of by passes of their own.
 * MG_EINVAL on unknown flags.  Changing the flags drops recorded graphs.
 */
enum { MG_FUSE_PROLONG = 1, MG_FUSE_BEFF = 2, MG_FUSE_RESTRICT = 4, MG_FUSE_IR = 8, MG_FUSE_ALL = 15 };
int mg_set_fusion(mg_tree *t, int flags);

/*
 * mg_stream_copy - copy `bytes` (a multiple of 16; both pointers device
 * memory, 16-byte aligned, not overlapping) from src to dst on `stream` with
 * 16-byte vector loads and stores in a grid-stride loop over `blocks`
 * workgroups of 256 threads (blocks <= 0: 4 per CU).  A measurement helper:
 * timing it gives the device's achievable streaming bandwidth, the second
 * reference (beside the specification peak) of the solver's roofline.
 * Asynchronous; MG_EINVAL on bad sizes or alignment.
 */
int mg_stream_copy(void *dst, const void *src, int64_t bytes, int blocks, void *stream);

const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
