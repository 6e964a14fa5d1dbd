// Kernel launchers for the octree multigrid (device code in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mg {

// Read-only geometry shared by the stencil kernels.
struct Geo {
    const int32_t *nbr;     // [n][6]
    const int32_t *cfslot;  // [n][6]
    const int32_t *cfq;     // [n][6]
    const int32_t *xt;      // [n][6][4][2] faces of the face neighbours
    const int32_t *n27;     // [n][27] same-level box at ijk + o, o in {-1,0,1}^3 (x fastest);
                            // -1 covered only by a coarser leaf, -2 outside the domain
    const int32_t *slotx;   // [nslot][8] Q, base t1, base t2, Q's neighbours -t1 +t1 -t2 +t2
    const int32_t *ijk;     // [n][4] (i, j, k, level)
    const int32_t *parent;  // [n]
    const double *bcval;    // [n][6][64] or null
    double bcv[6];
    int32_t bct[6];
    double len;
};

// Launchers are templates over the field type T (double, or float for the
// correction cycles of the mixed-precision solve); c_hat has the field's type.
template <typename T> void launch_fill(T *p, int64_t count, T v, hipStream_t s);
template <typename T> void launch_pack(const double *nat, T *cs, int64_t nbox, hipStream_t s);
template <typename T> void launch_unpack(const T *cs, double *nat, int64_t nbox, hipStream_t s);
// Gauss-Seidel launch variants: variant = 2 * c + x, with c = 0, 1, 2 for
// half-sweeps with 1, 2 or 4 cells per thread (256, 128 or 64 threads per
// box), c = 3 for fused sweeps (red and black in one launch, ping-ponging
// between the field and a second buffer), c = 4 for half-sweeps over octets
// of sibling boxes (one 512-thread workgroup per 16^3 octet; levels >= 2,
// whose boxes come in complete consecutive octets), c = 5, 6 for half-sweeps
// by at most 2048 or 4096 persistent workgroups that prefetch their next
// box, and x = 1 for the XCD-aware mapping.  All variants do the same
// arithmetic on every cell.
constexpr int kGsrbVariants = 14;
constexpr int kGsrbHalfVariants = 6;  // variants 0..5 are one-box half-sweeps
constexpr int kGsrbFusedVariant = 6;  // 6, 7: fused sweeps
constexpr int kGsrbOctVariant = 8;    // 8, 9: octet half-sweeps
constexpr int kGsrbPipeVariant = 10;  // 10..13: persistent prefetching half-sweeps
constexpr int kGsrbDefault = 3;       // 2 cells per thread, XCD mapping
// One colour in place; a fused variant, or an octet variant on a box count
// that is not a multiple of 8, falls back to kGsrbDefault.  Black colour
// only: with phi64 (FP32, variants with gsrb_updates) every box also adds its
// new correction to phi64 (phi64 += (double) e on all its cells) and the
// boxes with rmask[b] != 0 (rmask may be null) restrict the updated phi64
// onto their parents' cells; without phi64, rmask (variants with
// gsrb_restricts) makes those boxes restrict their swept values.
template <typename T>
void launch_gsrb(const Geo &g, T *phi, const T *rhs, const T *chat, int64_t b0, int64_t nb, T h2,
                 int colour, int variant, hipStream_t s, const int32_t *rmask = nullptr,
                 double *phi64 = nullptr);
constexpr bool gsrb_restricts(int variant) { return variant >= 0 && variant < kGsrbHalfVariants; }
constexpr bool gsrb_updates(int variant) {
    return gsrb_restricts(variant) || (variant >= kGsrbOctVariant && variant < kGsrbPipeVariant);
}
// One full sweep (red, then black) from src into dst (no aliasing).
template <typename T>
// fas = 1: also complete the FAS right-hand side L src + restricted
// residual on the boxes with children (isleaf == 0), smooth with it and
// store it in fasbuf; fas = 2: take those boxes' values from fasbuf and copy
// them into rhs (the sweep after a fas = 1 sweep).  inv_h2 = 1 / h^2.
void launch_gsrb_sweep(const Geo &g, const T *src, T *dst, T *rhs, const T *chat, int64_t b0,
                       int64_t nb, T h2, int xcd, hipStream_t s, int fas = 0,
                       const int32_t *isleaf = nullptr, T inv_h2 = (T)0, T *fasbuf = nullptr);
// The parent cells of every listed leaf box (level >= 2) <- mean of its
// cells under them, in one launch (the restriction a stopping test needs).
template <typename T>
void launch_restrict_leaves(const Geo &g, T *phi, const int32_t *leaf, int64_t nleaf, hipStream_t s);
template <typename T>
void launch_cf_coarse(const Geo &g, const T *phi, T *chat, const int32_t *slots, int64_t s0,
                      int64_t ns, hipStream_t s);
// partial != null: phi is zero everywhere (FMG start) and is not read; each
// leaf box also writes its norm partials (as k_leaf_norms) at leafpos[b].
template <typename T>
void launch_resid_restrict(const Geo &g, T *phi, T *rhs, T *old, const T *chat, int64_t b0,
                           int64_t nb, const int32_t *leaf_prev, int64_t nleaf_prev, T inv_h2,
                           hipStream_t s, const int32_t *leafpos = nullptr, double *partial = nullptr,
                           double vol = 0.0);
template <typename T>
void launch_fas_rhs(const Geo &g, const T *phi, T *rhs, const T *chat, const int32_t *list,
                    int64_t nlist, T inv_h2, hipStream_t s);
template <typename T>
void launch_prolong_cf(const Geo &g, T *phi, const T *old, int64_t b0, int64_t nb, T *chat,
                       const int32_t *slots, int64_t s0, int64_t ns, hipStream_t s);
// First red-black sweep after the prolongation into level l (l >= 2): the
// prolonged value of every cell a half-sweep reads is formed on the fly from
// the unprolonged field and the parent's correction phi - old, so the
// prolongation pass is not launched; colour 0 then colour 1.  The level
// ends with the values of prolongation + one sweep.  c_hat of the level
// must be current.
template <typename T>
void launch_gsrb_pro(const Geo &g, T *phi, const T *rhs, const T *pad, const T *chat, int64_t b0, int64_t nb,
                     T h2, int colour, hipStream_t s);
// The correction phi - old of the refined boxes refined[0..nref) of level l-1
// as padded 10^3 blocks (pad[k * 1000 ..]) for launch_gsrb_pro on level l,
// plus c_hat of the refinement-boundary slots [s0, s0+ns) of level l.
template <typename T>
void launch_delta_pad(const Geo &g, const T *phi, const T *old, const int32_t *refined, int64_t nref, T *pad,
                      T *chat, const int32_t *slots, int64_t s0, int64_t ns, hipStream_t s);
template <typename T>
void launch_coarse(const Geo &g, T *phi, const T *rhs, const double *eig, int64_t b0, int64_t nroot,
                   double h, hipStream_t s);
template <typename T>
void launch_restrict_phi(const Geo &g, T *phi, int64_t b0, int64_t nb, hipStream_t s);
// Bottom of the V-cycle (levels 1 and 2 of every tree) in one launch, one
// workgroup per tree: smooth(2, nd), residual + restriction + FAS rhs, root
// solve, prolongation, smooth(2, nu); fmg != 0 prepends the FMG pass's
// restriction, root solve and prolongation.  fas2 != 0 first completes the
// FAS right-hand side of the level-2 boxes with children (isleaf[b] == 0),
// rhs <- L phi + rhs, and stores it (the k_fas_rhs step after the
// restriction from level 3).  h2, h1: cell sizes of levels 2 and 1;
// root2[t]: first level-2 box of tree t, or -1.
template <typename T>
void launch_bottom(const Geo &g, T *phi, T *rhs, T *old, const double *eig, int64_t r0, int ntree,
                   const int32_t *root2, double h2, double h1, int nd, int nu, int fmg, int fas2,
                   const int32_t *isleaf, hipStream_t s);
void launch_leaf_norms(const Geo &g, const double *phi, const double *rhs, const double *chat,
                       const int32_t *leaf, int64_t nleaf, double *partial, float *r_out,
                       hipStream_t s);
// The same norms over the leaf boxes leaf[q0 .. q0+nq) of the level-grouped
// leaf list, into partial at their positions q (XCD shares of the list).
void launch_box_norms(const Geo &g, const double *phi, const double *rhs, const double *chat, const int32_t *leaf,
                      int64_t q0, int64_t nq, double *partial, float *r_out, hipStream_t s);
template <typename T>
void launch_leaf_apply(const Geo &g, const T *x, const T *chat, const int32_t *leaf, int64_t nleaf,
                       T *out, hipStream_t s);
void launch_ir_update(double *phi, const float *e, int64_t count, hipStream_t s);
// Mesh adaptation: per-box refinement scores (27 region maxima of |b| h^2),
// and the transfer of phi to a new tree (copy of boxes present in both, then
// level by level the interpolation of new boxes from their parents).
void launch_refine_scores(const Geo &g, const double *rhs, int64_t n, double *scores, hipStream_t s);
// xt[b][d][4][2] from the face tables nbr and cfslot ([n][6], on the device)
void launch_face_xt(const int32_t *nbr, const int32_t *cfslot, int64_t n, int32_t *xt, hipStream_t s);
// near[b] (leaf boxes): the largest score over b's cells and the cells of its
// same-level leaf neighbours within 3 cells; 0 for refined boxes
void launch_refine_near(const int32_t *n27, const int32_t *isleaf, const double *scores, int64_t n, double *near,
                        hipStream_t s);
void launch_transfer_copy(const double *from, double *to, const int32_t *src, int64_t n, hipStream_t s);
void launch_transfer_interp(const Geo &g, double *phi, const double *chat, const int32_t *list, int64_t nlist,
                            hipStream_t s);
// Electric field of phi on all n boxes (face components and cell strength).
void launch_efield(const Geo &g, const double *phi, const double *chat, int64_t n, double *e_face,
                   double *e_norm, hipStream_t s);
void launch_copy16(const void *src, void *dst, int64_t n16, int blocks, hipStream_t s);
constexpr int kReduceChunk = 2048;  // leaf positions per first-stage block of the norm reduction
void launch_reduce_trees(const double *partial, const int32_t *leaf_tree, const int32_t *chunk,
                         int64_t nchunk, const int32_t *choff, int ntree, double *part2,
                         double *result, hipStream_t s);

// Fluid model (fluid.hip).  Transport table of n entries (mu, D, alpha) at
// E = k emax / (n - 1), stored as interval rows of 6 doubles
// v[6 k ..] = (mu_k, mu_k+1, D_k, D_k+1, alpha_k, alpha_k+1), the last row
// repeating entry n-1; scale = (n - 1) / emax.
struct FluidTable {
    const double *v;
    int n;
    double scale;
};
struct FluidArgs {
    FluidTable tab;
    const int32_t *isleaf, *cfrev, *leaf, *slots;  // cfrev: [n][6][4] fine slots of a coarse face
    int64_t nleaf, nslot;
    double *ne;                                    // covered cells overwritten (mean of children)
    const double *ni, *n0e, *n0i, *ef, *en;
    double dt, wa, wb;
    double *oute, *outi, *rhs;                     // rhs: the solver's colour-split field
    double *cf;                                    // [nslot][4][64] scratch
    double *partial, *result;                      // [nleaf] scratch, [1] the time-step bound
};
// One stage: restriction of ne into covered cells, the refinement-boundary
// faces, the update of every leaf box and the minimum time-step bound.
void launch_fluid_stage(const Geo &g, const FluidArgs &a, hipStream_t s);

}  // namespace mg
