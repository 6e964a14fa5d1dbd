// C ABI and cycle driver of the octree multigrid solver.
//
// The driver enqueues the kernels of kernels.hip on the caller's stream in
// the order of the full-approximation-scheme FMG / V-cycle (paper section
// 2.1.2).  Fixed launch sequences (the FMG pass, one V-cycle plus residual
// check, and the steps of the mixed-precision refinement) are recorded once
// as HIP graphs and replayed; the only device-to-host transfer per cycle is
// the pair of reduced residual norms used by the stopping test.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <new>
#include <string>

#include "kernels.h"
#include "mg_internal.h"
#include "mg_nn.h"
#include "nn.h"

namespace mg {

thread_local std::string g_error;
void set_error(const std::string &msg) { g_error = msg; }

namespace {

hipStream_t stream_of(const mg_tree *t) { return (hipStream_t)t->cur_stream; }

double hlev(const mg_tree *t, int l) { return t->dom.len / (8.0 * (double)(1 << (l - 1))); }
int64_t lbeg(const mg_tree *t, int l) { return t->lstart[l - 1]; }
int64_t lcount(const mg_tree *t, int l) { return t->lstart[l] - t->lstart[l - 1]; }

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return MG_OK;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    set_error(buf);
    return MG_EHIP;
}

// Geometry and boundary data for the kernels.  The FP32 correction problem
// of the mixed-precision solve has homogeneous boundary data.
Geo geo(const mg_tree *t, bool homogeneous) {
    Geo g;
    g.nbr = t->d.nbr;
    g.cfslot = t->d.cfslot;
    g.cfq = t->d.cfq;
    g.xt = t->d.xt;
    g.n27 = t->d.n27;
    g.slotx = t->d.slotx;
    g.ijk = t->d.ijk;
    g.parent = t->d.parent;
    g.bcval = (!homogeneous && t->dom.per_cell_bc) ? t->d.bcval : nullptr;
    for (int d = 0; d < 6; d++) {
        g.bcv[d] = homogeneous ? 0.0 : t->dom.bc_val[d];
        g.bct[d] = t->dom.bc_type[d];
    }
    g.len = t->dom.len;
    return g;
}

// One set of multigrid fields: the FP64 solution or the FP32 correction.
template <typename T>
struct Fields {
    T *phi, *rhs, *old, *chat;
    bool *cf_valid;  // c_hat of level l is current (it depends on level l-1 only)
    Geo g;
};
Fields<double> f64(mg_tree *t) {
    return {t->d.phi, t->d.rhs, t->d.old, t->d.chat, t->cf_valid, geo(t, false)};
}
Fields<float> f32(mg_tree *t) {
    return {t->d.e32, t->d.r32, t->d.old32, t->d.chat32, t->cf_valid32, geo(t, true)};
}

template <typename T> void dirty(const Fields<T> &F, int l) {
    if (l + 1 <= kMaxLevel) F.cf_valid[l + 1] = false;
}
template <typename T> void dirty_all(const Fields<T> &F) {
    for (int l = 0; l <= kMaxLevel + 1; l++) F.cf_valid[l] = false;
}
template <typename T> void ensure_cf(mg_tree *t, const Fields<T> &F, int l) {
    if (l < 2 || l > t->nlev || F.cf_valid[l]) return;
    int64_t s0 = t->sstart[l], ns = t->sstart[l + 1] - t->sstart[l];
    launch_cf_coarse<T>(F.g, F.phi, F.chat, t->d.slots, s0, ns, stream_of(t));
    F.cf_valid[l] = true;
}
// c_hat of every level in one launch (slots are grouped by level, and each
// level's c_hat reads only the level below it).  Valid only where no level
// changes between this call and the use of a c_hat computed here: after the
// restriction pass, and at the start of an FMG pass from a zero field.
template <typename T> void ensure_cf_all(mg_tree *t, const Fields<T> &F) {
    bool any = false;
    for (int l = 2; l <= t->nlev; l++) any = any || !F.cf_valid[l];
    if (!any) return;
    int64_t s0 = t->sstart[2], ns = t->sstart[t->nlev + 1] - t->sstart[2];
    launch_cf_coarse<T>(F.g, F.phi, F.chat, t->d.slots, s0, ns, stream_of(t));
    for (int l = 2; l <= t->nlev; l++) F.cf_valid[l] = true;
}

// ---- optional event timing of the half-sweep launches
hipEvent_t take_event(mg_tree *t) {
    if (!t->ev_pool.empty()) {
        void *e = t->ev_pool.back();
        t->ev_pool.pop_back();
        return (hipEvent_t)e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
void give_event(mg_tree *t, hipEvent_t e) {
    if (e) t->ev_pool.push_back((void *)e);
}

// ---- steps of the cycle
// fas_first: the level's coarse FAS right-hand side is still to be formed
// (fas_down deferred it); the first pair of fused sweeps forms it.
template <typename T> bool smooth_fuses_fas(const mg_tree *t, int l, int nsweep) {
    int variant = t->sched[sizeof(T) == 4 ? 1 : 0][l];
    return nsweep >= 2 && l >= 2 && variant >= kGsrbFusedVariant && variant < kGsrbOctVariant;
}
// rmask / phi64: the last half-sweep (black) also restricts the boxes of the
// mask onto their parents (rst_fuses), or with phi64 (FP32) adds the
// correction to phi64 and restricts the updated values (ir_fuses).
template <typename T> void smooth(mg_tree *t, const Fields<T> &F, int l, int nsweep, bool fas_first = false,
                                  const int32_t *rmask = nullptr, double *phi64 = nullptr) {
    if (nsweep <= 0) return;
    ensure_cf(t, F, l);
    double h = hlev(t, l);
    T h2 = (T)(h * h);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (t->timing) {
        e0 = take_event(t);
        e1 = take_event(t);
        if (!e0 || !e1 || hipEventRecord(e0, stream_of(t)) != hipSuccess) {
            give_event(t, e0);
            give_event(t, e1);
            e0 = e1 = nullptr;
        }
    }
    int variant = t->sched[sizeof(T) == 4 ? 1 : 0][l];
    if (l < 2 && variant >= kGsrbOctVariant && variant < kGsrbPipeVariant)
        variant = kGsrbDefault;  // roots are not octets
    int64_t launches = 0;
    int it = 0;
    if (variant >= kGsrbFusedVariant && variant < kGsrbOctVariant) {
        // fused sweeps in pairs: field -> sweep buffer -> field
        T *swp = (T *)t->d.swp, *fbuf = (T *)t->d.fas;
        T inv_h2 = (T)(1.0 / (h * h));
        for (; it + 1 < nsweep; it += 2) {
            int f1 = fas_first && it == 0 ? 1 : 0, f2 = f1 ? 2 : 0;
            launch_gsrb_sweep<T>(F.g, F.phi, swp, F.rhs, F.chat, lbeg(t, l), lcount(t, l), h2,
                                 variant & 1, stream_of(t), f1, t->d.isleaf, inv_h2, fbuf);
            launch_gsrb_sweep<T>(F.g, swp, F.phi, F.rhs, F.chat, lbeg(t, l), lcount(t, l), h2,
                                 variant & 1, stream_of(t), f2, t->d.isleaf, inv_h2, fbuf);
            launches += 2;
        }
    }
    for (; it < nsweep; it++)  // half-sweeps (a fused schedule's odd last sweep: the default)
        for (int c = 0; c < 2; c++) {
            bool last = c == 1 && it == nsweep - 1;
            launch_gsrb<T>(F.g, F.phi, F.rhs, F.chat, lbeg(t, l), lcount(t, l), h2, c, variant,
                           stream_of(t), last ? rmask : nullptr, last ? phi64 : nullptr);
            launches++;
        }
    if (e0) {
        if (hipEventRecord(e1, stream_of(t)) == hipSuccess) {
            t->probes.push_back({(void *)e0, (void *)e1, l, launches,
                                 3.0 * 256 * sizeof(T) * (double)lcount(t, l) * 2 * nsweep});
        } else {
            give_event(t, e0);
            give_event(t, e1);
        }
    }
    dirty(F, l);
}

// defer_rhs: leave the coarse right-hand side L phi_c + r_c of the refined
// level-(l-1) boxes to the first fused sweep of level l-1 (smooth with
// fas_first), which forms it from the same values.
// zero_norms (FP64, phi = 0 everywhere): the residual kernel skips reading
// phi and leaves the norm partials of the residual of phi = 0 of the level's
// leaf boxes in the partial buffer (at their leaf positions).
template <typename T> void fas_down(mg_tree *t, const Fields<T> &F, int l, bool defer_rhs = false,
                                    bool zero_norms = false) {
    ensure_cf(t, F, l);
    double h = hlev(t, l);
    launch_resid_restrict<T>(F.g, F.phi, F.rhs, F.old, F.chat, lbeg(t, l), lcount(t, l),
                             t->d.oldcp + t->ostart[l - 1], t->ostart[l] - t->ostart[l - 1],
                             (T)(1.0 / (h * h)), stream_of(t), t->d.leafpos,
                             zero_norms ? t->d.partial : nullptr, h * h * h);
    dirty(F, l - 1);
    ensure_cf(t, F, l - 1);
    if (defer_rhs) return;
    double hc = hlev(t, l - 1);
    launch_fas_rhs<T>(F.g, F.phi, F.rhs, F.chat, t->d.refined + t->rstart[l - 1],
                      t->rstart[l] - t->rstart[l - 1], (T)(1.0 / (hc * hc)), stream_of(t));
}

// Prolongation into level l, fused with the c_hat pass of level l (both read
// only level l-1, which is final at this point of the up-leg).
template <typename T> void prolong(mg_tree *t, const Fields<T> &F, int l) {
    int64_t s0 = t->sstart[l], ns = t->sstart[l + 1] - t->sstart[l];
    launch_prolong_cf<T>(F.g, F.phi, F.old, lbeg(t, l), lcount(t, l), F.chat, t->d.slots, s0, ns,
                         stream_of(t));
    F.cf_valid[l] = true;
    dirty(F, l);
}

// Exact root solve (computed in FP64 for either field type).
template <typename T> void coarse(mg_tree *t, const Fields<T> &F) {
    launch_coarse<T>(F.g, F.phi, F.rhs, t->d.eig, lbeg(t, 1), lcount(t, 1), hlev(t, 1), stream_of(t));
    dirty(F, 1);
}

template <typename T> void restrict_all(mg_tree *t, const Fields<T> &F) {
    for (int l = t->nlev; l >= 2; l--) {
        launch_restrict_phi<T>(F.g, F.phi, lbeg(t, l), lcount(t, l), stream_of(t));
        dirty(F, l - 1);
    }
}

// With MG_FUSE_RESTRICT, does the last up-sweep of level l in a cycle of nu
// up-sweeps (FP64, the finest level on top) also do level l's part of the
// restriction before a stopping test?  Levels 1-2 of the one-launch bottom,
// sweep variants without the restricting kernel, cycles whose up-sweeps are
// all fused with the prolongation, and a per-level hook (it reads level l's
// residual after the sweeps) leave it to restrict_for_check.
bool rst_fuses(const mg_tree *t, int l, int nu) {
    if (!(t->fusion & MG_FUSE_RESTRICT) || t->level_hook || l < 2 || l > t->nlev) return false;
    if (t->bottom_ok && t->sched[0][1] != 0 && l < 3) return false;  // use_bottom<double>
    int variant = t->sched[0][l];
    if (!gsrb_restricts(variant)) return false;
    int plain = (t->fusion & MG_FUSE_PROLONG) && nu >= 1 ? nu - 1 : nu;
    return plain >= 1;
}

// With MG_FUSE_IR, does the last up-sweep of level l in an FP32 correction
// cycle of nu up-sweeps also add the level's correction to the FP64 field
// (and restrict it)?  Same exclusions as rst_fuses, with the FP32 schedule
// and the variants that have the update.
bool ir_fuses(const mg_tree *t, int l, int nu) {
    if (!(t->fusion & MG_FUSE_IR) || l < 2 || l > t->nlev) return false;
    if (t->bottom_ok && t->sched[1][1] != 0 && l < 3) return false;  // use_bottom<float>
    int variant = t->sched[1][l];
    if (!gsrb_updates(variant)) return false;
    int plain = (t->fusion & MG_FUSE_PROLONG) && nu >= 1 ? nu - 1 : nu;
    return plain >= 1;
}
// The lowest level of the run of levels up to the finest whose last up-sweep
// does the update (t->nlev + 1: none).  Level ir_low's own restriction stays
// after the cycle: its parents are updated only then.
int ir_low(const mg_tree *t, int nu) {
    int l = t->nlev;
    while (l >= 2 && ir_fuses(t, l, nu)) l--;
    return l + 1;
}

// Before a stopping test: parent cells <- the mean of their children, in one
// launch over the leaf boxes of the list cleaf.  A residual or c_hat reads a
// covered cell only next to a leaf cell of its own level, that is across the
// parent's outer face on the child's side where the parent's neighbour is a
// leaf box, and under 2:1 nesting such a cell has only leaf children; so the
// test sees exactly the values of restrict_all.  The next cycle's down-leg
// restricts every level before it reads it.
// nu >= 0 (FP64, after a cycle of nu up-sweeps that ran with rst): the levels
// whose last up-sweep restricted (rst_fuses) are skipped, the others go in
// one launch per run of consecutive levels.
template <typename T> void restrict_for_check(mg_tree *t, const Fields<T> &F, int nu = -1) {
    if (nu < 0 || sizeof(T) != 8) {
        launch_restrict_leaves<T>(F.g, F.phi, t->d.cleaf, (int64_t)t->cleaf.size(), stream_of(t));
    } else {
        for (int l = 2; l <= t->nlev;) {
            if (rst_fuses(t, l, nu)) {
                l++;
                continue;
            }
            int l1 = l;
            while (l1 + 1 <= t->nlev && !rst_fuses(t, l1 + 1, nu)) l1++;
            launch_restrict_leaves<T>(F.g, F.phi, t->d.cleaf + t->cstart[l], t->cstart[l1 + 1] - t->cstart[l],
                                      stream_of(t));
            l = l1 + 1;
        }
    }
    for (int l = t->nlev; l >= 2; l--) dirty(F, l - 1);
}

// Levels 1 and 2 as one launch (one workgroup per tree)?
template <typename T> bool use_bottom(const mg_tree *t) {
    return t->bottom_ok && t->sched[sizeof(T) == 4 ? 1 : 0][1] != 0;
}

// The bottom of the cycle in one launch: smooth(2, nd), fas_down(2),
// coarse, prolong(2), smooth(2, nu); with fmg, preceded by fas_down(2),
// coarse, prolong(2).  Leaves the c_hat state as that sequence does (level 2
// has no refinement-boundary faces, so it launches no c_hat pass).
// fas2: the restriction from level 3 deferred level 2's FAS right-hand side
// to this launch.
template <typename T> void bottom(mg_tree *t, const Fields<T> &F, int nd, int nu, bool fmg, bool fas2) {
    launch_bottom<T>(F.g, F.phi, F.rhs, F.old, t->d.eig, lbeg(t, 1), t->ntree, t->d.root2, hlev(t, 2),
                     hlev(t, 1), nd, nu, fmg ? 1 : 0, fas2 ? 1 : 0, t->d.isleaf, stream_of(t));
    F.cf_valid[2] = true;
    dirty(F, 2);
}

// Prolongation into level l followed by nsweep sweeps.  With the fusion on
// (and a half-sweep schedule on the level) the first sweep forms the
// prolonged values it reads on the fly and no prolongation pass runs; the
// result is the same bits.
template <typename T> void prolong_smooth(mg_tree *t, const Fields<T> &F, int l, int nsweep,
                                          const int32_t *rmask = nullptr, double *phi64 = nullptr) {
    int variant = t->sched[sizeof(T) == 4 ? 1 : 0][l];
    bool fused_sweeps = variant >= kGsrbFusedVariant && variant < kGsrbOctVariant;
    if (!(t->fusion & MG_FUSE_PROLONG) || nsweep < 1 || l < 2 || fused_sweeps) {
        prolong(t, F, l);
        smooth(t, F, l, nsweep, false, rmask, phi64);
        return;
    }
    // the parents' corrections as padded blocks, with c_hat of level l (both
    // read level l-1 only, final here)
    T *pad = (T *)t->d.dpad;
    int64_t s0 = t->sstart[l], ns = t->sstart[l + 1] - t->sstart[l];
    launch_delta_pad<T>(F.g, F.phi, F.old, t->d.refined + t->rstart[l - 1], t->rstart[l] - t->rstart[l - 1], pad,
                        F.chat, t->d.slots, s0, ns, stream_of(t));
    F.cf_valid[l] = true;
    double h = hlev(t, l);
    for (int c = 0; c < 2; c++)
        launch_gsrb_pro<T>(F.g, F.phi, F.rhs, pad, F.chat, lbeg(t, l), lcount(t, l), (T)(h * h), c,
                           stream_of(t));
    dirty(F, l);
    smooth(t, F, l, nsweep - 1, false, rmask, phi64);
}

// pro_top: the top level still needs the prolonged correction before its
// first smoothing (the FMG pass's interpolation to a new finest level).
// rst (FP64, top = finest level): the cycle ends in a stopping test, and the
// levels' last up-sweeps do their part of its restriction (rst_fuses); then
// call restrict_for_check(t, F, nu).  ir (FP32 correction cycle, top =
// finest level): the last up-sweeps of the levels from ir_low up also add
// the correction to the FP64 field and restrict it; then call ir_finish.
template <typename T> void vcycle(mg_tree *t, const Fields<T> &F, int top, int nd, int nu,
                                  bool pro_top = false, bool rst = false, bool ir = false) {
    bool one = use_bottom<T>(t) && top >= 2;
    int low = one ? 3 : 2;
    bool deferred = false;
    for (int l = top; l >= low; l--) {
        if (l == top && pro_top)
            prolong_smooth(t, F, l, nd);
        else
            smooth(t, F, l, nd, deferred);
        deferred = l - 1 >= low && smooth_fuses_fas<T>(t, l - 1, nd);
        fas_down(t, F, l, deferred || (one && l == low));
    }
    if (one) {
        bottom(t, F, nd, nu, false, top >= low);
    } else {
        coarse(t, F);
    }
    int lf = ir && sizeof(T) == 4 && top == t->nlev ? ir_low(t, nu) : t->nlev + 1;
    for (int l = low; l <= top; l++) {
        bool r = rst && sizeof(T) == 8 && top == t->nlev && rst_fuses(t, l, nu);
        if (l >= lf)
            prolong_smooth(t, F, l, nu, l > lf ? t->d.cmask : nullptr, t->d.phi);
        else
            prolong_smooth(t, F, l, nu, r ? t->d.cmask : nullptr);
        if (sizeof(T) == 8 && t->level_hook && !t->hook_rc) t->hook_rc = t->level_hook(t, l, t->hook_ctx);
    }
}

// FMG pass from the current (zero) field: FAS data top-down, root solve, then
// for each finer level the prolonged correction and one V-cycle on top.
// beff_slot >= 0 (FP64, from phi = 0): the top-down pass also gives the
// per-tree norms of the residual of phi = 0 (into result[beff_slot ..]), the
// norms the stopping test divides by, without a pass of their own.
template <typename T> void fmg_pass(mg_tree *t, const Fields<T> &F, int nd, int nu, int beff_slot = -1,
                                    bool rst = false, bool ir = false) {
    // the top-down FAS pass changes level l-1 only after the last use of
    // c_hat(l), and c_hat(l-1) reads level l-2, still untouched: every c_hat
    // it needs can be computed up front from the initial field
    ensure_cf_all(t, F);
    bool one = use_bottom<T>(t);
    int low = one ? 3 : 2;
    for (int l = t->nlev; l >= low; l--) fas_down(t, F, l, one && l == low, beff_slot >= 0);
    if (beff_slot >= 0) {
        // leaf boxes on levels below the top-down pass (those of a tree of one
        // or two levels): the norm kernel, on the still zero field
        int top = std::min(low - 1, t->nlev);
        launch_box_norms(f64(t).g, t->d.phi, t->d.rhs, t->d.chat, t->d.leaf, 0, t->fstart[top + 1],
                         t->d.partial, nullptr, stream_of(t));
        launch_reduce_trees(t->d.partial, t->d.leaf_tree, t->d.chunk, (int64_t)t->chunk.size() / 3, t->d.choff,
                            t->ntree, t->d.part2, t->d.result + beff_slot, stream_of(t));
    }
    if (one) {
        bottom(t, F, nd, nu, true, t->nlev >= low);  // fas_down(2), coarse, prolong(2), V-cycle(2)
    } else {
        coarse(t, F);
    }
    for (int l = low; l <= t->nlev; l++) vcycle(t, F, l, nd, nu, true, rst && l == t->nlev, ir && l == t->nlev);
}

// After an FP32 correction cycle run with ir: the update phi += e of the
// levels below ir_low (one launch over their boxes), then the restriction of
// the leaf boxes of levels 2 .. ir_low (their parents are updated now).
// Without ir: the update of every box, then restrict_for_check.
void ir_finish(mg_tree *t, int nu, bool ir) {
    Fields<double> F = f64(t);
    int lf = ir ? ir_low(t, nu) : t->nlev + 1;
    if (lf > t->nlev) {
        launch_ir_update(F.phi, f32(t).phi, 512 * t->n, stream_of(t));
        restrict_for_check(t, F);
        return;
    }
    launch_ir_update(F.phi, f32(t).phi, 512 * t->lstart[lf - 1], stream_of(t));
    launch_restrict_leaves<double>(F.g, F.phi, t->d.cleaf + t->cstart[2], t->cstart[lf + 1] - t->cstart[2],
                                   stream_of(t));
    for (int l = t->nlev; l >= 2; l--) dirty(F, l - 1);
}

// Per-tree leaf residual norms of the FP64 solution into result[slot + 2t],
// result[slot + 2t + 1] (sum of r^2 h^3, max |r|); r32 != null also stores
// the residual in FP32.
void norms_launch(mg_tree *t, int slot, float *r32) {
    Fields<double> F = f64(t);
    ensure_cf_all(t, F);
    launch_box_norms(F.g, F.phi, F.rhs, F.chat, t->d.leaf, 0, t->nleaf, t->d.partial, r32, stream_of(t));
    launch_reduce_trees(t->d.partial, t->d.leaf_tree, t->d.chunk, (int64_t)t->chunk.size() / 3, t->d.choff,
                        t->ntree, t->d.part2, t->d.result + slot, stream_of(t));
}

int read_results(mg_tree *t, int count) {
    int rc = hip_check(hipMemcpyAsync(t->host_result, t->d.result, count * sizeof(double),
                                      hipMemcpyDeviceToHost, (hipStream_t)t->stream), "norm readback");
    if (rc) return rc;
    return hip_check(hipStreamSynchronize((hipStream_t)t->stream), "stream synchronize");
}

int norms(mg_tree *t) {
    norms_launch(t, 0, nullptr);
    return read_results(t, 2 * t->ntree);
}

// Per-tree norm of the residual of phi = 0 (boundary data folded in), into
// t->beff_tree.  The current phi is parked in the old field, which holds no
// state between calls (every down-leg rewrites it before the up-leg reads it).
int beff_norm(mg_tree *t) {
    Fields<double> F = f64(t);
    size_t bytes = (size_t)t->n * 512 * sizeof(double);
    int rc = hip_check(hipMemcpyAsync(F.old, F.phi, bytes, hipMemcpyDeviceToDevice, stream_of(t)),
                       "park phi");
    if (rc) return rc;
    launch_fill<double>(F.phi, 512 * t->n, 0.0, stream_of(t));
    dirty_all(F);
    if ((rc = norms(t))) return rc;
    for (int tr = 0; tr < t->ntree; tr++) t->beff_tree[tr] = std::sqrt(t->host_result[2 * tr]);
    rc = hip_check(hipMemcpyAsync(F.phi, F.old, bytes, hipMemcpyDeviceToDevice, stream_of(t)),
                   "restore phi");
    dirty_all(F);
    return rc;
}

// ---- recorded launch sequences
//  SEQ_FMG:       phi <- 0, per-tree norms of the residual of phi = 0 into
//                 result[2T..4T), FMG pass, restriction pass, per-tree leaf
//                 norms into result[0..2T) (T trees).
//  SEQ_VCHECK:    V-cycle with the finest level on top, restriction pass, norms.
//  SEQ_MIX_START: phi <- 0, leaf residual (= residual of phi = 0) in FP64 with
//                 its FP32 copy as the correction's right-hand side, norms.
//  SEQ_MIX_FMG / SEQ_MIX_V: e <- 0, FP32 FMG pass (first refinement step) or
//                 one FP32 V-cycle on A e = r with homogeneous boundary data,
//                 phi += e in FP64, restriction pass, FP64 residual, norms.
void run_body(mg_tree *t, int seq, int nd, int nu) {
    Fields<double> F = f64(t);
    Fields<float> E = f32(t);
    switch (seq) {
    case mg_tree::SEQ_FMG:
        launch_fill<double>(F.phi, 512 * t->n, 0.0, stream_of(t));
        dirty_all(F);
        if (t->fusion & MG_FUSE_BEFF) {
            fmg_pass(t, F, nd, nu, 2 * t->ntree, true);
        } else {
            norms_launch(t, 2 * t->ntree, nullptr);
            fmg_pass(t, F, nd, nu, -1, true);
        }
        restrict_for_check(t, F, nu);
        norms_launch(t, 0, nullptr);
        break;
    case mg_tree::SEQ_VCHECK:
        vcycle(t, F, t->nlev, nd, nu, false, true);
        restrict_for_check(t, F, nu);
        norms_launch(t, 0, nullptr);
        break;
    case mg_tree::SEQ_V:
        // a check without its norms: the next cycle starts from the state a
        // check leaves (covered cells read by c_hat restricted, every
        // level's c_hat computed from them), so phi is the same bits
        vcycle(t, F, t->nlev, nd, nu, false, true);
        restrict_for_check(t, F, nu);
        ensure_cf_all(t, F);
        break;
    case mg_tree::SEQ_MIX_START:
        launch_fill<double>(F.phi, 512 * t->n, 0.0, stream_of(t));
        dirty_all(F);
        norms_launch(t, 0, E.rhs);
        break;
    case mg_tree::SEQ_MIX_FMG:
    case mg_tree::SEQ_MIX_V:
    {
        launch_fill<float>(E.phi, 512 * t->n, 0.0f, stream_of(t));
        dirty_all(E);
        bool ir = t->fusion & MG_FUSE_IR;
        if (seq == mg_tree::SEQ_MIX_FMG) fmg_pass(t, E, nd, nu, -1, false, ir);
        else vcycle(t, E, t->nlev, nd, nu, false, false, ir);
        dirty_all(F);
        ir_finish(t, nu, ir);
        norms_launch(t, 0, E.rhs);
        break;
    }
    }
}

void save_state(const mg_tree *t, bool s[2][kMaxLevel + 2]) {
    std::memcpy(s[0], t->cf_valid, sizeof t->cf_valid);
    std::memcpy(s[1], t->cf_valid32, sizeof t->cf_valid32);
}
void load_state(mg_tree *t, const bool s[2][kMaxLevel + 2]) {
    std::memcpy(t->cf_valid, s[0], sizeof t->cf_valid);
    std::memcpy(t->cf_valid32, s[1], sizeof t->cf_valid32);
}
bool same_state(const mg_tree *t, const bool s[2][kMaxLevel + 2]) {
    return !std::memcmp(s[0], t->cf_valid, sizeof t->cf_valid) &&
           !std::memcmp(s[1], t->cf_valid32, sizeof t->cf_valid32);
}

void drop_graph(mg_tree::Graph &g) {
    if (g.exec) (void)hipGraphExecDestroy((hipGraphExec_t)g.exec);
    g.exec = nullptr;
}

// Record a sequence into g on the private capture stream (nothing executes);
// the host-side state is left as it was on entry.
int record(mg_tree *t, mg_tree::Graph &g, int seq, int nd, int nu) {
    drop_graph(g);
    save_state(t, g.pre);
    hipStream_t cs = (hipStream_t)t->cap_stream;
    int rc = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "begin capture");
    if (rc) return rc;
    t->cur_stream = cs;
    run_body(t, seq, nd, nu);
    t->cur_stream = t->stream;
    save_state(t, g.post);
    load_state(t, g.pre);
    hipGraph_t graph = nullptr;
    if ((rc = hip_check(hipStreamEndCapture(cs, &graph), "end capture"))) return rc;
    size_t nodes = 0;
    (void)hipGraphGetNodes(graph, nullptr, &nodes);
    g.nodes = (int)nodes;
    hipGraphExec_t exec = nullptr;
    rc = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate graph");
    (void)hipGraphDestroy(graph);
    if (rc) return rc;
    g.exec = (void *)exec;
    g.nd = nd;
    g.nu = nu;
    return MG_OK;
}

// Run a sequence (replaying its graph when enabled and the host-side state
// matches the recorded one), then read back count result values.  Timing
// probes need events on the bound stream between launches, so the timing
// mode always launches kernel by kernel.
int run_seq(mg_tree *t, int seq, const mg_solve_opts *o, int count) {
    int nd = o->n_down, nu = o->n_up;
    mg_tree::Graph &g = t->graphs[seq];
    bool use = o->graphs && !t->timing;
    // Every sequence but the V-cycles starts by zeroing the fields it uses,
    // so c_hat validity on entry is irrelevant to it; reset it so that one
    // recorded graph serves every entry.  The V-cycles need the FP64 state
    // as it is and never touch the FP32 fields.
    dirty_all(f32(t));
    if (seq != mg_tree::SEQ_VCHECK && seq != mg_tree::SEQ_V) dirty_all(f64(t));
    if (use && !(g.exec && g.nd == nd && g.nu == nu && same_state(t, g.pre))) {
        int rc = record(t, g, seq, nd, nu);
        if (rc) return rc;
    }
    if (!use) {
        run_body(t, seq, nd, nu);
        return count ? read_results(t, count) : MG_OK;
    }
    int rc = hip_check(hipGraphLaunch((hipGraphExec_t)g.exec, (hipStream_t)t->stream), "graph launch");
    if (rc) return rc;
    load_state(t, g.post);
    return count ? read_results(t, count) : MG_OK;
}

// Turn the per-tree norms in host_result[0..2T) into statistics.  A forest's
// trees are independent problems: rel is the largest relative residual over
// the trees, each relative to its own residual of phi = 0; l2, linf and
// beff_l2 are taken over all trees together.
int record_check(mg_tree *t, mg_solve_stats *s, int k) {
    double rel = 0.0, sq = 0.0, mx = 0.0, bsq = 0.0;
    for (int tr = 0; tr < t->ntree; tr++) {
        double l2 = std::sqrt(t->host_result[2 * tr]), m = t->host_result[2 * tr + 1];
        double b = t->beff_tree[tr];
        double r = b > 0 ? l2 / b : l2;
        t->rel_tree[tr] = r;
        if (r > rel || r != r) rel = r;
        sq += t->host_result[2 * tr];
        bsq += b * b;
        if (m > mx || m != m) mx = m;
    }
    s->rel_res = rel;
    s->l2 = std::sqrt(sq);
    s->linf = mx;
    s->beff_l2 = std::sqrt(bsq);
    if (k < 64) s->rel_hist[k] = rel;
    if (!std::isfinite(rel)) {
        set_error("non-finite residual");
        return MG_ENOCONV;
    }
    return MG_OK;
}

int check_and_record(mg_tree *t, mg_solve_stats *s, int k) {
    restrict_for_check(t, f64(t));
    int rc = norms(t);
    if (rc) return rc;
    return record_check(t, s, k);
}

// Cycles until the stopping test holds: seq_of(k) names the sequence of step k.
template <typename SeqOf>
int iterate(mg_tree *t, const mg_solve_opts *o, mg_solve_stats *s, SeqOf seq_of) {
    int stall = 0;
    for (int k = 1; s->rel_res > o->rel_tol; k++) {
        if (k > o->max_cycles) {
            set_error("no convergence within max_cycles");
            return MG_ENOCONV;
        }
        double prev = s->rel_res;
        int rc = run_seq(t, seq_of(k), o, 2 * t->ntree);
        if (rc) return rc;
        s->n_vcycles = k;
        if ((rc = record_check(t, s, k))) return rc;
        stall = s->rel_res >= prev ? stall + 1 : 0;
        if (stall >= 3) {
            set_error("residual stagnates");
            return MG_ENOCONV;
        }
    }
    return MG_OK;
}

// n warm-started V-cycles for callers that need only the field: no residual
// norms and no host round trip.  The first cycle starts, and every cycle
// ends, in the state a stopping test leaves (covered cells that c_hat reads
// restricted, every level's c_hat computed from them), and the last is
// followed by the full restriction, so phi is the same bits as mg_vcycle's.
int vcycles_no_stats(mg_tree *t, const mg_solve_opts *o, int n) {
    restrict_for_check(t, f64(t));
    ensure_cf_all(t, f64(t));
    int rc = MG_OK;
    for (int k = 0; k < n && !rc; k++) rc = run_seq(t, mg_tree::SEQ_V, o, 0);
    if (!rc) restrict_all(t, f64(t));  // every covered cell: the mean of its children
    if (!rc) rc = hip_check(hipGetLastError(), "kernel launch");
    return rc;
}

int require_bound(const mg_tree *t) {
    if (!t) {
        set_error("null tree");
        return MG_EINVAL;
    }
    if (!t->ws) {
        set_error("no workspace bound (call mg_tree_bind first)");
        return MG_ESTATE;
    }
    return MG_OK;
}

int check_opts(const mg_solve_opts *o) {
    if (!o || (o->precision != MG_FP64 && o->precision != MG_MIXED && o->precision != MG_LEARNED) ||
        o->n_down < 0 ||
        o->n_up < 0 || o->max_cycles < 0 || o->max_cycles > 10000 || !(o->rel_tol >= 0) ||
        (o->final_check_only != 0 && o->final_check_only != 1) ||
        (o->learned_placement != 0 && o->learned_placement != 1)) {
        set_error("invalid solver options");
        return MG_EINVAL;
    }
    return MG_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ---- learned correction step
constexpr int kStepStride = kMaxLevel + 2;  // steps[tree][level], level 0 unused
constexpr double kLearnedKeep = 0.99;

struct LearnedWs {
    float *x, *y, *scale, *q;
    double *partial, *steps;
};

int64_t learned_layout(const mg_tree *t, char *base, LearnedWs *L) {
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        int64_t at = o;
        o += (bytes + 255) & ~(int64_t)255;
        return at;
    };
    int64_t nl = t->nleaf;
    int64_t ox = take(4 * 1000 * nl), oy = take(4 * 512 * nl), os = take(4 * nl);
    int64_t oq = take(4 * 3 * 512 * nl), op = take(8 * 9 * nl);
    int64_t ost = take(8 * (int64_t)t->ntree * kStepStride);
    if (base && L) {
        L->x = (float *)(base + ox);
        L->y = (float *)(base + oy);
        L->scale = (float *)(base + os);
        L->q = (float *)(base + oq);
        L->partial = (double *)(base + op);
        L->steps = (double *)(base + ost);
    }
    return o;
}

int check_learned_ws(const mg_tree *t, void *ws, int64_t bytes) {
    if (!ws || ((uintptr_t)ws & 255)) {
        set_error("learned workspace missing or not 256-byte aligned");
        return MG_EINVAL;
    }
    if (bytes < learned_layout(t, nullptr, nullptr)) {
        set_error("learned workspace too small");
        return MG_ENOMEM;
    }
    return MG_OK;
}

// Least squares per tree: minimise |r - sum_l s_l q_l| given the Gram matrix
// G (S x S, upper triangle filled) and g = (<r, q_l>).  Levels with a zero
// column get 0; a level whose pivot vanishes (a dependent column) is
// dropped and the factorisation restarted.
void solve_steps(const double *G, const double *g, double *s) {
    const int S = kStepStride;
    bool on[S];
    for (int l = 0; l < S; l++) {
        on[l] = G[l * S + l] > 0.0 && std::isfinite(G[l * S + l]);
        s[l] = 0.0;
    }
    for (int attempt = 0; attempt <= S; attempt++) {
        int idx[S], n = 0;
        for (int l = 0; l < S; l++)
            if (on[l]) idx[n++] = l;
        if (n == 0) return;
        double C[S][S] = {{0}};
        int bad = -1;
        for (int a = 0; a < n && bad < 0; a++) {
            for (int c = 0; c <= a; c++) {
                int la = idx[a], lc = idx[c];
                double v = la <= lc ? G[la * S + lc] : G[lc * S + la];
                for (int k = 0; k < c; k++) v -= C[a][k] * C[c][k];
                if (c == a) {
                    if (!(v > 1e-13 * G[la * S + la])) {
                        bad = la;
                        break;
                    }
                    C[a][a] = std::sqrt(v);
                } else {
                    C[a][c] = v / C[c][c];
                }
            }
        }
        if (bad >= 0) {
            on[bad] = false;
            continue;
        }
        double z[S];
        for (int a = 0; a < n; a++) {
            double v = g[idx[a]];
            for (int k = 0; k < a; k++) v -= C[a][k] * z[k];
            z[a] = v / C[a][a];
        }
        for (int a = n - 1; a >= 0; a--) {
            double v = z[a];
            for (int k = a + 1; k < n; k++) v -= C[k][a] * s[idx[k]];
            s[idx[a]] = v / C[a][a];
        }
        return;
    }
}

// One learned step on the current FP64 phi (see mg_nn.h).  The FP32
// correction fields serve as scratch: e32 holds the correction of one level
// class (levels = m mod 3, whose operator images do not overlap: a leaf cell
// of level j only sees corrections of levels j-1, j, j+1), r32 the residual.
int learned_step_impl(mg_tree *t, mg_nn *nn, const LearnedWs &L, double *steps_host) {
    Fields<double> F = f64(t);
    Fields<float> E = f32(t);
    hipStream_t s = stream_of(t);
    const int64_t nl = t->nleaf;
    restrict_all(t, F);
    norms_launch(t, 0, E.rhs);
    launch_nn_gather(E.rhs, t->d.leaf, nl, t->d.nbr, t->d.ijk, t->d.isleaf, t->dom.len, L.x, L.scale, s);
    launch_nn_forward(nn->prm, nn->pk, nl, nullptr, L.x, L.y, nullptr, nullptr, s);
    for (int m = 0; m < 3; m++) {
        launch_nn_scatter(L.y, L.scale, t->d.leaf, nl, t->d.ijk, m, E.phi, s);
        dirty_all(E);
        restrict_all(t, E);
        for (int l = 2; l <= t->nlev; l++) ensure_cf(t, E, l);
        launch_leaf_apply<float>(E.g, E.phi, E.chat, t->d.leaf, nl, L.q + (int64_t)m * nl * 512, s);
    }
    dirty_all(E);
    launch_nn_dots(E.rhs, L.q, t->d.leaf, nl, t->d.ijk, t->dom.len, L.partial, s);
    std::vector<double> part((size_t)9 * nl);
    int rc = hip_check(hipMemcpyAsync(part.data(), L.partial, part.size() * sizeof(double),
                                      hipMemcpyDeviceToHost, s), "step sums readback");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "stream synchronize");
    if (rc) return rc;
    const int S = kStepStride, T = t->ntree;
    std::vector<double> G((size_t)T * S * S, 0.0), g((size_t)T * S, 0.0), st((size_t)T * S, 0.0);
    for (int64_t q = 0; q < nl; q++) {
        int64_t b = t->leaf[q];
        int j = t->lev[b], tr = t->tid[b];
        const double *p = &part[9 * q];
        double *Gt = &G[(size_t)tr * S * S], *gt = &g[(size_t)tr * S];
        gt[j - 1] += p[0];
        gt[j] += p[1];
        gt[j + 1] += p[2];
        Gt[(j - 1) * S + j - 1] += p[3];
        Gt[(j - 1) * S + j] += p[4];
        Gt[(j - 1) * S + j + 1] += p[5];
        Gt[j * S + j] += p[6];
        Gt[j * S + j + 1] += p[7];
        Gt[(j + 1) * S + j + 1] += p[8];
    }
    for (int tr = 0; tr < T; tr++) {
        double *Gt = &G[(size_t)tr * S * S];
        for (int l = 0; l < S; l++) Gt[l] = Gt[l * S] = 0.0;  // no level 0
        solve_steps(Gt, &g[(size_t)tr * S], &st[(size_t)tr * S]);
    }
    rc = hip_check(hipMemcpyAsync(L.steps, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice, s),
                   "step upload");
    if (rc) return rc;
    launch_nn_update(F.phi, L.y, L.scale, t->d.leaf, nl, t->d.ijk, t->d.tid, L.steps, S, s);
    dirty_all(F);
    if (steps_host)
        for (int tr = 0; tr < T; tr++)
            for (int l = 0; l <= t->nlev; l++) steps_host[tr * (t->nlev + 1) + l] = st[(size_t)tr * S + l];
    rc = hip_check(hipGetLastError(), "learned step launch");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "stream synchronize");
    return rc;
}

// Per-level learned step on the leaf boxes of level l >= 3 (after the
// level's up-sweeps inside an FP64 V-cycle, or on the current state): the
// level's residual with the cycle's ghosts (covered cells as they are), the
// network's correction c on those boxes, q = A0 c with homogeneous boundary
// data (c is zero off the level's leaf boxes: refined same-level boxes hold
// 0, and the level's refinement-boundary values are set to 0), and per tree
// phi += s c with s = <r, q> / <q, q> (0 when not finite or not positive).
// steps_host (may be NULL): [ntree] the steps.  Synchronises.
int learned_level_step(mg_tree *t, mg_nn *nn, const LearnedWs &L, int l, double *steps_host) {
    if (l < 3 || l > t->nlev) return MG_OK;
    const int64_t q0 = t->fstart[l], nq = t->fstart[l + 1] - q0;
    if (nq <= 0) return MG_OK;
    Fields<double> F = f64(t);
    Fields<float> E = f32(t);
    hipStream_t s = stream_of(t);
    const int32_t *list = t->d.leaf + q0;
    ensure_cf(t, F, l);
    launch_leaf_norms(F.g, F.phi, F.rhs, F.chat, list, nq, L.partial, E.rhs, s);  // r in FP32
    launch_nn_gather(E.rhs, list, nq, t->d.nbr, t->d.ijk, t->d.isleaf, t->dom.len, L.x, L.scale, s);
    launch_nn_forward(nn->prm, nn->pk, nq, nullptr, L.x, L.y, nullptr, nullptr, s);
    launch_nn_scatter(L.y, L.scale, list, nq, t->d.ijk, -1, E.phi, s);
    int64_t c0 = t->sstart[l], nc = t->sstart[l + 1] - c0;
    launch_fill<float>(E.chat + c0 * 64, nc * 64, 0.0f, s);  // no correction on the coarse side
    launch_leaf_apply<float>(E.g, E.phi, E.chat, list, nq, L.q, s);
    dirty_all(E);
    launch_nn_dots1(E.rhs, L.q, list, nq, t->d.ijk, t->dom.len, L.partial, s);
    std::vector<double> part((size_t)2 * nq);
    int rc = hip_check(hipMemcpyAsync(part.data(), L.partial, part.size() * sizeof(double),
                                      hipMemcpyDeviceToHost, s), "level step sums readback");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "stream synchronize");
    if (rc) return rc;
    const int S = kStepStride, T = t->ntree;
    std::vector<double> rq(T, 0.0), qq(T, 0.0), st((size_t)T * S, 0.0);
    for (int64_t q = 0; q < nq; q++) {  // fixed order: leaf-list order
        int tr = t->tid[t->leaf[q0 + q]];
        rq[tr] += part[2 * q];
        qq[tr] += part[2 * q + 1];
    }
    for (int tr = 0; tr < T; tr++) {
        double v = qq[tr] > 0.0 ? rq[tr] / qq[tr] : 0.0;
        st[(size_t)tr * S + l] = std::isfinite(v) && v > 0.0 ? v : 0.0;
        if (steps_host) steps_host[tr] = st[(size_t)tr * S + l];
    }
    rc = hip_check(hipMemcpyAsync(L.steps, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice, s),
                   "step upload");
    if (rc) return rc;
    launch_nn_update(F.phi, L.y, L.scale, list, nq, t->d.ijk, t->d.tid, L.steps, S, s);
    dirty(F, l);
    return hip_check(hipGetLastError(), "level step launch");
}

struct LevelHookCtx {
    mg_nn *nn;
    const LearnedWs *L;
};
int level_hook_fn(mg_tree *t, int l, void *ctx) {
    auto *c = (LevelHookCtx *)ctx;
    return learned_level_step(t, c->nn, *c->L, l, nullptr);
}

// The per-level learned solve (opts learned_placement = 1): the FMG pass, one
// plain V-cycle (its residual factor is the plain factor), then V-cycles
// with the per-level step after every level's up-sweeps, launched kernel by
// kernel, while each such cycle's factor does not exceed the plain one; the
// first that does makes the remaining cycles plain (phi is kept).
int learned_solve_levels(mg_tree *t, mg_nn *nn, const LearnedWs &L, const mg_solve_opts *o, mg_solve_stats *s,
                         mg_learned_stats *lst) {
    const int T = t->ntree;
    double t0 = now_ms();
    int rc = run_seq(t, mg_tree::SEQ_FMG, o, 4 * T);
    if (rc) return s->status = rc;
    for (int tr = 0; tr < T; tr++) t->beff_tree[tr] = std::sqrt(t->host_result[2 * T + 2 * tr]);
    if ((rc = record_check(t, s, 0))) return s->status = rc;
    double plain = 0.0;
    bool use = true;
    int stall = 0;
    LevelHookCtx ctx{nn, &L};
    for (int k = 1; s->rel_res > o->rel_tol; k++) {
        if (k > o->max_cycles) {
            set_error("no convergence within max_cycles");
            return s->status = MG_ENOCONV;
        }
        double prev = s->rel_res;
        if (k == 1 || !use) {
            if ((rc = run_seq(t, mg_tree::SEQ_VCHECK, o, 2 * T))) return s->status = rc;
        } else {
            double tl = now_ms();
            dirty_all(f32(t));
            t->level_hook = level_hook_fn;
            t->hook_ctx = &ctx;
            t->hook_rc = MG_OK;
            run_body(t, mg_tree::SEQ_VCHECK, o->n_down, o->n_up);
            t->level_hook = nullptr;
            rc = t->hook_rc;
            if (!rc) rc = read_results(t, 2 * T);
            if (rc) return s->status = rc;
            lst->t_learned_ms += now_ms() - tl;
        }
        s->n_vcycles = k;
        if ((rc = record_check(t, s, k))) return s->status = rc;
        if (k == 1) {
            plain = prev > 0.0 ? s->rel_res / prev : 0.0;
        } else if (use) {
            if (s->rel_res / prev > plain) {
                use = false;
                lst->fallback_cycle = k;
            } else {
                lst->accepted++;
            }
        }
        stall = s->rel_res >= prev ? stall + 1 : 0;
        if (stall >= 3) {
            set_error("residual stagnates");
            return s->status = MG_ENOCONV;
        }
    }
    restrict_all(t, f64(t));
    rc = hip_check(hipGetLastError(), "kernel launch");
    s->t_ms = now_ms() - t0;
    s->nn_accepted = lst->accepted;
    s->nn_fell_back = lst->fallback_cycle;
    return s->status = rc;
}

// Network state in the caller's device memory.
int64_t nn_state_layout(char *base, mg_nn *nn) {
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        int64_t at = o;
        o += (bytes + 255) & ~(int64_t)255;
        return at;
    };
    int64_t op = take(4 * kNnParams), om = take(4 * kNnParams), ov = take(4 * kNnParams);
    int64_t og = take(4 * kNnParams), ok = take(2 * kNnPacked);
    if (base && nn) {
        nn->prm = (float *)(base + op);
        nn->m = (float *)(base + om);
        nn->v = (float *)(base + ov);
        nn->grad = (float *)(base + og);
        nn->pk = (uint16_t *)(base + ok);
    }
    return o;
}

hipStream_t nn_stream(const mg_nn *nn) { return (hipStream_t)nn->stream; }

// Forward with saved activations, backward and the fixed-order reduction of
// the gradient into nn->grad, with the training buffers at ws (laid out by
// nn_train_layout for nbox boxes); loss (host, may be NULL) synchronises.
int nn_gradient_run(mg_nn *nn, int64_t nbox, const int32_t *idx, const float *x, const float *target,
                    char *ws, double *loss) {
    NnTrainWs w;
    nn_train_layout(nbox, ws, &w);
    hipStream_t s = nn_stream(nn);
    launch_nn_forward(nn->prm, nn->pk, nbox, idx, x, w.y, w.a1, w.a2, s);
    launch_nn_backward(nn->prm, nbox, idx, x, target, w, nn->grad, s);
    int rc = hip_check(hipGetLastError(), "gradient launch");
    if (rc || !loss) return rc;
    rc = hip_check(hipMemcpyAsync(nn->host_loss, w.loss, sizeof(double), hipMemcpyDeviceToHost, s),
                   "loss readback");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "stream synchronize");
    if (!rc) *loss = *nn->host_loss;
    return rc;
}

int require_nn(const mg_nn *nn) {
    if (!nn) {
        set_error("null network");
        return MG_EINVAL;
    }
    return MG_OK;
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

const char *mg_last_error(void) { return g_error.c_str(); }

void mg_default_opts(mg_solve_opts *o) {
    o->precision = MG_FP64;
    o->n_down = 2;
    o->n_up = 2;
    o->max_cycles = 50;
    o->rel_tol = 1e-8;
    o->graphs = 1;
    o->final_check_only = 0;
    o->learned_placement = 0;
}

int mg_tree_create(mg_tree **out, const mg_domain *dom, int64_t n, const int32_t *level,
                   const int32_t *ijk, const int32_t *tree) {
    if (!out) {
        set_error("null output pointer");
        return MG_EINVAL;
    }
    *out = nullptr;
    mg_tree *t = new (std::nothrow) mg_tree();
    if (!t) return MG_ENOMEM;
    int rc;
    try {
        rc = build_tree(t, dom, n, level, ijk, tree);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        rc = MG_ENOMEM;
    }
    if (rc) {
        delete t;
        return rc;
    }
    *out = t;
    return MG_OK;
}

// Capture streams and pinned result buffers outlive the trees that used
// them: a mesh adaptation creates and destroys a tree per step, and creating
// a stream or a pinned buffer costs more than the new tree's table upload.
// A destroyed tree hands them back (its bound stream has been synchronised,
// and a capture stream never executes work); the next bind takes them.
std::mutex g_spare_mu;
std::vector<std::pair<int, void *>> g_spare_streams;    // (device, stream)
std::vector<std::pair<size_t, double *>> g_spare_pinned;  // (capacity, buffer)
// The pinned staging buffer of the table upload (the largest one used so
// far; a bind holds it until its upload has completed).
char *g_stage = nullptr;
size_t g_stage_cap = 0;

int take_capture_stream(int device, void **out) {
    {
        std::lock_guard<std::mutex> lk(g_spare_mu);
        for (size_t i = 0; i < g_spare_streams.size(); i++)
            if (g_spare_streams[i].first == device) {
                *out = g_spare_streams[i].second;
                g_spare_streams.erase(g_spare_streams.begin() + i);
                return MG_OK;
            }
    }
    hipStream_t cs = nullptr;
    int rc = hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
    *out = (void *)cs;
    return rc;
}
int take_pinned(size_t bytes, double **out, size_t *cap) {
    {
        std::lock_guard<std::mutex> lk(g_spare_mu);
        for (size_t i = 0; i < g_spare_pinned.size(); i++)
            if (g_spare_pinned[i].first >= bytes) {
                *cap = g_spare_pinned[i].first;
                *out = g_spare_pinned[i].second;
                g_spare_pinned.erase(g_spare_pinned.begin() + i);
                return MG_OK;
            }
    }
    *cap = std::max<size_t>(bytes, 4096);
    return hip_check(hipHostMalloc((void **)out, *cap), "pinned host buffer");
}

int take_stage(size_t bytes, char **out, size_t *cap) {
    {
        std::lock_guard<std::mutex> lk(g_spare_mu);
        if (g_stage && g_stage_cap >= bytes) {
            *out = g_stage;
            *cap = g_stage_cap;
            g_stage = nullptr;
            g_stage_cap = 0;
            return MG_OK;
        }
    }
    *cap = std::max<size_t>(bytes, 1 << 20);
    return hip_check(hipHostMalloc((void **)out, *cap), "pinned staging buffer");
}
// Keeps the larger of the returned buffer and the pooled one.
void give_stage(char *p, size_t cap) {
    char *drop = p;
    {
        std::lock_guard<std::mutex> lk(g_spare_mu);
        if (!g_stage || g_stage_cap < cap) {
            drop = g_stage;
            g_stage = p;
            g_stage_cap = cap;
        }
    }
    if (drop) (void)hipHostFree(drop);
}

int mg_tree_destroy(mg_tree *t) {
    if (!t) return MG_OK;
    // work enqueued without a host wait (mg_vcycle without statistics,
    // mg_fluid_step, mg_field_set) may still run on the bound stream and use
    // the graphs and the pinned buffer released below
    if (t->stream) (void)hipStreamSynchronize((hipStream_t)t->stream);
    for (auto &g : t->graphs) drop_graph(g);
    {
        std::lock_guard<std::mutex> lk(g_spare_mu);
        if (t->host_result) g_spare_pinned.push_back({t->host_result_bytes, t->host_result});
        if (t->cap_stream) g_spare_streams.push_back({t->cap_device, t->cap_stream});
    }
    for (auto &p : t->probes) {
        t->ev_pool.push_back(p.e0);
        t->ev_pool.push_back(p.e1);
    }
    for (void *e : t->ev_pool) (void)hipEventDestroy((hipEvent_t)e);
    delete t;
    return MG_OK;
}

int mg_tree_info(const mg_tree *t, mg_tree_info_t *info) {
    if (!t || !info) {
        set_error("null argument");
        return MG_EINVAL;
    }
    std::memset(info, 0, sizeof *info);
    info->n_boxes = t->n;
    info->n_levels = t->nlev;
    info->n_trees = t->ntree;
    info->n_leaf_boxes = t->nleaf;
    info->n_leaf_cells = 512 * t->nleaf;
    info->n_cf_faces = t->nslot;
    for (int l = 0; l <= 16; l++) info->level_start[l] = t->lstart[l];
    info->workspace_bytes = t->off.total;
    return MG_OK;
}

int mg_tree_index(const mg_tree *t, int what, int32_t *out) {
    if (!t || !out) {
        set_error("null argument");
        return MG_EINVAL;
    }
    const std::vector<int32_t> *v = nullptr;
    switch (what) {
    case MG_IDX_ORDER: v = &t->order; break;
    case MG_IDX_LEVEL: v = &t->lev; break;
    case MG_IDX_IJK: v = &t->ijk; break;
    case MG_IDX_TREE: v = &t->tid; break;
    case MG_IDX_PARENT: v = &t->parent; break;
    case MG_IDX_CHILD: v = &t->child; break;
    case MG_IDX_NBR: v = &t->nbr; break;
    case MG_IDX_CFQ: v = &t->cfq; break;
    default: set_error("unknown index table"); return MG_EINVAL;
    }
    std::memcpy(out, v->data(), v->size() * sizeof(int32_t));
    return MG_OK;
}

static int bind_tables(mg_tree *t, void *ws, void *stream);

int mg_tree_bind(mg_tree *t, void *ws, int64_t bytes, void *stream) {
    if (!t || !ws) {
        set_error("null argument");
        return MG_EINVAL;
    }
    if (bytes < t->off.total || ((uintptr_t)ws & 255)) {
        set_error("workspace too small or not 256-byte aligned");
        return MG_ENOMEM;
    }
    int rc = bind_tables(t, ws, stream);
    if (rc) t->ws = nullptr;  // a failed bind leaves the tree unbound, not half uploaded
    return rc;
}

static int bind_tables(mg_tree *t, void *ws, void *stream) {
    for (auto &g : t->graphs) drop_graph(g);
    t->ws = ws;
    t->stream = stream;
    t->cur_stream = stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (t->cap_stream && t->cap_device != dev) {  // rebound on another device
        std::lock_guard<std::mutex> lk(g_spare_mu);
        g_spare_streams.push_back({t->cap_device, t->cap_stream});
        t->cap_stream = nullptr;
    }
    if (!t->cap_stream) {
        int rc = take_capture_stream(dev, &t->cap_stream);
        if (rc) return rc;
        t->cap_device = dev;
    }
    char *base = (char *)ws;
    DevTables &d = t->d;
    d.nbr = (int32_t *)(base + t->off.nbr);
    d.cfslot = (int32_t *)(base + t->off.cfslot);
    d.cfq = (int32_t *)(base + t->off.cfq);
    d.xt = (int32_t *)(base + t->off.xt);
    d.n27 = (int32_t *)(base + t->off.n27);
    d.slotx = (int32_t *)(base + t->off.slotx);
    d.ijk = (int32_t *)(base + t->off.ijk);
    d.parent = (int32_t *)(base + t->off.parent);
    d.refined = (int32_t *)(base + t->off.refined);
    d.leaf = (int32_t *)(base + t->off.leaf);
    d.cleaf = (int32_t *)(base + t->off.cleaf);
    d.oldcp = (int32_t *)(base + t->off.oldcp);
    d.leafpos = (int32_t *)(base + t->off.leafpos);
    d.cmask = (int32_t *)(base + t->off.cmask);
    d.slots = (int32_t *)(base + t->off.slots);
    d.leaf_tree = (int32_t *)(base + t->off.leaf_tree);
    d.tree_off = (int32_t *)(base + t->off.tree_off);
    d.chunk = (int32_t *)(base + t->off.chunk);
    d.choff = (int32_t *)(base + t->off.choff);
    d.part2 = (double *)(base + t->off.part2);
    d.isleaf = (int32_t *)(base + t->off.isleaf);
    d.tid = (int32_t *)(base + t->off.tid);
    d.root2 = (int32_t *)(base + t->off.root2);
    d.eig = (double *)(base + t->off.eig);
    d.phi = (double *)(base + t->off.phi);
    d.rhs = (double *)(base + t->off.rhs);
    d.old = (double *)(base + t->off.old);
    d.chat = (double *)(base + t->off.chat);
    d.bcval = t->off.bcval >= 0 ? (double *)(base + t->off.bcval) : nullptr;
    d.partial = (double *)(base + t->off.partial);
    d.result = (double *)(base + t->off.result);
    d.e32 = (float *)(base + t->off.e32);
    d.r32 = (float *)(base + t->off.r32);
    d.old32 = (float *)(base + t->off.old32);
    d.chat32 = (float *)(base + t->off.chat32);
    d.swp = (void *)(base + t->off.swp);
    d.fas = (void *)(base + t->off.fas);
    d.dpad = (void *)(base + t->off.dpad);
    if (!t->host_result) {
        int rc = take_pinned(4 * t->ntree * sizeof(double), &t->host_result, &t->host_result_bytes);
        if (rc) return rc;
    }
    // The host-built tables fill [0, off.xt) of the workspace: staged at
    // their workspace offsets in one pinned buffer and uploaded by one copy
    // (the gaps and the device-only part2 carry whatever the buffer holds);
    // xt, the last table, is formed on the GPU right after.
    const size_t tab_bytes = (size_t)t->off.xt;
    char *stage = nullptr;
    size_t stage_cap = 0;
    int rc = take_stage(tab_bytes, &stage, &stage_cap);
    if (rc) return rc;
    auto put = [&](int64_t off, const void *src, size_t nbytes) {
        if (nbytes) std::memcpy(stage + off, src, nbytes);
    };
    put(t->off.nbr, t->nbr.data(), t->nbr.size() * 4);
    put(t->off.cfslot, t->cfslot.data(), t->cfslot.size() * 4);
    put(t->off.cfq, t->cfq.data(), t->cfq.size() * 4);
    put(t->off.n27, t->n27.data(), t->n27.size() * 4);
    put(t->off.slotx, t->slotx.data(), t->slotx.size() * 4);
    put(t->off.parent, t->parent.data(), t->parent.size() * 4);
    put(t->off.refined, t->refined.data(), t->refined.size() * 4);
    put(t->off.leaf, t->leaf.data(), t->leaf.size() * 4);
    put(t->off.cleaf, t->cleaf.data(), t->cleaf.size() * 4);
    put(t->off.oldcp, t->oldcp.data(), t->oldcp.size() * 4);
    put(t->off.leafpos, t->leafpos.data(), t->leafpos.size() * 4);
    put(t->off.cmask, t->cmask.data(), t->cmask.size() * 4);
    put(t->off.slots, t->slots.data(), t->slots.size() * 4);
    put(t->off.leaf_tree, t->leaf_tree.data(), t->leaf_tree.size() * 4);
    put(t->off.tree_off, t->tree_off.data(), t->tree_off.size() * 4);
    put(t->off.chunk, t->chunk.data(), t->chunk.size() * 4);
    put(t->off.choff, t->choff.data(), t->choff.size() * 4);
    put(t->off.tid, t->tid.data(), t->tid.size() * 4);
    put(t->off.root2, t->root2.data(), t->root2.size() * 4);
    put(t->off.eig, t->eig, sizeof t->eig);
    int32_t *ijk4 = (int32_t *)(stage + t->off.ijk), *isleaf = (int32_t *)(stage + t->off.isleaf);
    for (int64_t b = 0; b < t->n; b++) {
        for (int a = 0; a < 3; a++) ijk4[4 * b + a] = t->ijk[3 * b + a];
        ijk4[4 * b + 3] = t->lev[b];
        isleaf[b] = t->child[8 * b] < 0 ? 1 : 0;
    }
    hipStream_t s = stream_of(t);
    rc = hip_check(hipMemcpyAsync(ws, stage, tab_bytes, hipMemcpyHostToDevice, s), "table upload");
    if (rc) {
        (void)hipStreamSynchronize(s);
        give_stage(stage, stage_cap);
        return rc;
    }
    launch_face_xt(d.nbr, d.cfslot, t->n, d.xt, s);  // a gather of the uploaded face tables
    launch_fill<double>(d.phi, 512 * t->n, 0.0, s);
    launch_fill<double>(d.rhs, 512 * t->n, 0.0, s);
    launch_fill<double>(d.old, 512 * t->n, 0.0, s);
    launch_fill<float>(d.e32, 512 * t->n, 0.0f, s);
    launch_fill<float>(d.r32, 512 * t->n, 0.0f, s);
    launch_fill<float>(d.old32, 512 * t->n, 0.0f, s);
    if (d.bcval) launch_fill<double>(d.bcval, 6 * 64 * t->n, 0.0, s);
    dirty_all(f64(t));
    dirty_all(f32(t));
    // the staging buffer goes back to the pool once the upload has run
    rc = hip_check(hipStreamSynchronize(s), "bind");
    give_stage(stage, stage_cap);
    return rc;
}

int mg_field_set(mg_tree *t, int which, const double *dev) {
    int rc = require_bound(t);
    if (rc) return rc;
    hipStream_t s = stream_of(t);
    switch (which) {
    case MG_FIELD_PHI: launch_pack<double>(dev, t->d.phi, t->n, s); dirty_all(f64(t)); break;
    case MG_FIELD_RHS: launch_pack<double>(dev, t->d.rhs, t->n, s); break;
    case MG_FIELD_OLD: launch_pack<double>(dev, t->d.old, t->n, s); break;
    case MG_FIELD_E32: launch_pack<float>(dev, t->d.e32, t->n, s); dirty_all(f32(t)); break;
    case MG_FIELD_R32: launch_pack<float>(dev, t->d.r32, t->n, s); break;
    case MG_FIELD_OLD32: launch_pack<float>(dev, t->d.old32, t->n, s); break;
    case MG_FIELD_BCVAL:
        if (!t->d.bcval) {
            set_error("per-cell boundary data not enabled for this tree");
            return MG_ESTATE;
        }
        return hip_check(hipMemcpyAsync(t->d.bcval, dev, (size_t)t->n * 6 * 64 * sizeof(double),
                                        hipMemcpyDeviceToDevice, s), "bcval copy");
    default: set_error("unknown field"); return MG_EINVAL;
    }
    return hip_check(hipGetLastError(), "field set");
}

int mg_field_get(const mg_tree *t, int which, double *dev) {
    int rc = require_bound(t);
    if (rc) return rc;
    hipStream_t s = stream_of(t);
    switch (which) {
    case MG_FIELD_PHI: launch_unpack<double>(t->d.phi, dev, t->n, s); break;
    case MG_FIELD_RHS: launch_unpack<double>(t->d.rhs, dev, t->n, s); break;
    case MG_FIELD_OLD: launch_unpack<double>(t->d.old, dev, t->n, s); break;
    case MG_FIELD_E32: launch_unpack<float>(t->d.e32, dev, t->n, s); break;
    case MG_FIELD_R32: launch_unpack<float>(t->d.r32, dev, t->n, s); break;
    case MG_FIELD_OLD32: launch_unpack<float>(t->d.old32, dev, t->n, s); break;
    default: set_error("unknown field"); return MG_EINVAL;
    }
    return hip_check(hipGetLastError(), "field get");
}

int mg_field(mg_tree *t, int which, int dtype, void **dev_ptr, int64_t *n_elems, int64_t *level_offsets) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!dev_ptr) {
        set_error("mg_field: null dev_ptr");
        return MG_EINVAL;
    }
    void *p = nullptr;
    int want = MG_DTYPE_F64;
    int64_t n = (int64_t)512 * t->n;
    switch (which) {
    case MG_FIELD_PHI: p = t->d.phi; break;
    case MG_FIELD_RHS: p = t->d.rhs; break;
    case MG_FIELD_OLD: p = t->d.old; break;
    case MG_FIELD_E32: p = t->d.e32; want = MG_DTYPE_F32; break;
    case MG_FIELD_R32: p = t->d.r32; want = MG_DTYPE_F32; break;
    case MG_FIELD_OLD32: p = t->d.old32; want = MG_DTYPE_F32; break;
    case MG_FIELD_BCVAL:
        if (!t->d.bcval) {
            set_error("mg_field: no per-cell boundary data (per_cell_bc not set)");
            return MG_EINVAL;
        }
        p = t->d.bcval;
        n = (int64_t)6 * 64 * t->n;
        break;
    default: set_error("mg_field: unknown field"); return MG_EINVAL;
    }
    if (dtype != want) {
        set_error("mg_field: dtype does not match the field's storage type");
        return MG_EINVAL;
    }
    // the caller may write through the pointer: cached derived values are stale
    dirty_all(f64(t));
    dirty_all(f32(t));
    *dev_ptr = p;
    if (n_elems) *n_elems = n;
    if (level_offsets)
        for (int l = 0; l <= t->nlev; l++) level_offsets[l] = t->lstart[l];
    return MG_OK;
}

int mg_fmg_solve(mg_tree *t, const mg_solve_opts *o, mg_solve_stats *st) {
    int rc = require_bound(t);
    if (rc) return rc;
    if ((rc = check_opts(o))) return rc;
    if (o->precision == MG_LEARNED) {
        if (!t->nn) {
            set_error("MG_LEARNED: no network bound to the tree (mg_nn_bind)");
            return MG_ESTATE;
        }
        mg_solve_opts f = *o;
        f.precision = MG_FP64;
        return mg_learned_solve(t, t->nn, t->nn_ws, t->nn_ws_bytes, &f, st, nullptr);
    }
    mg_solve_stats local;
    mg_solve_stats *s = st ? st : &local;
    std::memset(s, 0, sizeof *s);
    double t0 = now_ms();
    int T = t->ntree;
    if (o->precision == MG_FP64) {
        if ((rc = run_seq(t, mg_tree::SEQ_FMG, o, 4 * T))) return s->status = rc;
        for (int tr = 0; tr < T; tr++) t->beff_tree[tr] = std::sqrt(t->host_result[2 * T + 2 * tr]);
        if ((rc = record_check(t, s, 0))) return s->status = rc;
        rc = iterate(t, o, s, [](int) { return (int)mg_tree::SEQ_VCHECK; });
    } else {
        // mixed precision: FP64 residual, FP32 correction cycles, FP64 update
        if ((rc = run_seq(t, mg_tree::SEQ_MIX_START, o, 2 * T))) return s->status = rc;
        for (int tr = 0; tr < T; tr++) t->beff_tree[tr] = std::sqrt(t->host_result[2 * tr]);
        if ((rc = record_check(t, s, 0))) return s->status = rc;
        rc = iterate(t, o, s, [](int k) {
            return (int)(k == 1 ? mg_tree::SEQ_MIX_FMG : mg_tree::SEQ_MIX_V);
        });
    }
    if (!rc) restrict_all(t, f64(t));  // every covered cell: the mean of its children
    if (!rc) rc = hip_check(hipGetLastError(), "kernel launch");
    if (o->graphs && !t->timing) {
        bool fp64 = o->precision == MG_FP64;
        s->launches_fmg = fp64 ? t->graphs[mg_tree::SEQ_FMG].nodes
                               : t->graphs[mg_tree::SEQ_MIX_START].nodes + t->graphs[mg_tree::SEQ_MIX_FMG].nodes;
        if (s->n_vcycles > 1 || (fp64 && s->n_vcycles > 0))
            s->launches_cycle = t->graphs[fp64 ? mg_tree::SEQ_VCHECK : mg_tree::SEQ_MIX_V].nodes;
    }
    s->t_ms = now_ms() - t0;
    return s->status = rc;
}

int mg_vcycle(mg_tree *t, const mg_solve_opts *o, int n_cycles, mg_solve_stats *st) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (o && o->precision == MG_LEARNED) {
        set_error("mg_vcycle: learned steps run inside mg_fmg_solve (MG_LEARNED)");
        return MG_EINVAL;
    }
    if ((rc = check_opts(o))) return rc;
    if (!st && o->precision == MG_FP64 && n_cycles > 0) return vcycles_no_stats(t, o, n_cycles);
    mg_solve_stats local;
    mg_solve_stats *s = st ? st : &local;
    std::memset(s, 0, sizeof *s);
    double t0 = now_ms();
    if ((rc = beff_norm(t))) return s->status = rc;
    if (o->precision == MG_FP64 && n_cycles > 0 && o->final_check_only) {
        // n - 1 cycles with no host round trip, then the last with its check.
        // Each cycle starts from the state the skipped check would leave
        // (restricted covered cells, c_hat of every level), so phi is the
        // same bits as with a check around every cycle.
        for (int k = 0; k < n_cycles && k < 64; k++) s->rel_hist[k] = std::nan("");
        restrict_for_check(t, f64(t));
        ensure_cf_all(t, f64(t));
        for (int k = 1; k < n_cycles && !rc; k++) rc = run_seq(t, mg_tree::SEQ_V, o, 0);
        if (!rc) rc = run_seq(t, mg_tree::SEQ_VCHECK, o, 2 * t->ntree);
        if (!rc) {
            s->n_vcycles = n_cycles;
            rc = record_check(t, s, n_cycles);
        }
        if (!rc) restrict_all(t, f64(t));  // every covered cell: the mean of its children
        if (!rc) rc = hip_check(hipGetLastError(), "kernel launch");
        s->t_ms = now_ms() - t0;
        return s->status = rc;
    }
    if ((rc = check_and_record(t, s, 0))) return s->status = rc;
    int seq = o->precision == MG_FP64 ? mg_tree::SEQ_VCHECK : mg_tree::SEQ_MIX_V;
    if (o->precision != MG_FP64) {
        // the FP32 correction's right-hand side is the FP64 leaf residual
        norms_launch(t, 0, t->d.r32);
        if ((rc = read_results(t, 2 * t->ntree))) return s->status = rc;
    }
    if (n_cycles <= 0) {
        rc = iterate(t, o, s, [seq](int) { return seq; });
    } else {
        for (int k = 1; k <= n_cycles && !rc; k++) {
            if ((rc = run_seq(t, seq, o, 2 * t->ntree))) break;
            s->n_vcycles = k;
            rc = record_check(t, s, k);
        }
    }
    if (!rc) restrict_all(t, f64(t));  // every covered cell: the mean of its children
    if (!rc) rc = hip_check(hipGetLastError(), "kernel launch");
    if (o->graphs && !t->timing) {
        bool fp64 = o->precision == MG_FP64;
        s->launches_fmg = fp64 ? t->graphs[mg_tree::SEQ_FMG].nodes
                               : t->graphs[mg_tree::SEQ_MIX_START].nodes + t->graphs[mg_tree::SEQ_MIX_FMG].nodes;
        if (s->n_vcycles > 1 || (fp64 && s->n_vcycles > 0))
            s->launches_cycle = t->graphs[fp64 ? mg_tree::SEQ_VCHECK : mg_tree::SEQ_MIX_V].nodes;
    }
    s->t_ms = now_ms() - t0;
    return s->status = rc;
}

int mg_efield(mg_tree *t, double *e_face, double *e_norm) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!e_face && !e_norm) {
        set_error("mg_efield: no output");
        return MG_EINVAL;
    }
    Fields<double> F = f64(t);
    restrict_all(t, F);
    ensure_cf_all(t, F);
    launch_efield(F.g, F.phi, F.chat, t->n, e_face, e_norm, stream_of(t));
    return hip_check(hipGetLastError(), "efield launch");
}

int mg_refine_scores(mg_tree *t, double *scores) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!scores) {
        set_error("mg_refine_scores: null output");
        return MG_EINVAL;
    }
    launch_refine_scores(geo(t, false), t->d.rhs, t->n, scores, stream_of(t));
    return hip_check(hipGetLastError(), "refine scores launch");
}

int mg_refine_near(mg_tree *t, const double *scores, double *near) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!scores || !near) {
        set_error("mg_refine_near: null argument");
        return MG_EINVAL;
    }
    launch_refine_near(t->d.n27, t->d.isleaf, scores, t->n, near, stream_of(t));
    return hip_check(hipGetLastError(), "refine near launch");
}

// mg_regrid_plan and mg_regrid_plan_near: the same plan, from the 27 region
// scores of every box or from their per-box reduction (near != 0).
static int plan_common(const mg_tree *t, const double *scores, const double *near, double c3, double deref,
                       double h_deref, int max_level, int64_t cap, int32_t *level, int32_t *ijk, int32_t *tree,
                       int64_t *n_out, const char *name) {
    if (!t || !(scores || near) || !n_out || !(c3 > 0) || !(deref >= 0) || !(h_deref > 0) || max_level < 1 ||
        max_level > kMaxLevel ||
        cap < 0 || (cap > 0 && (!level || !ijk || !tree))) {
        set_error(std::string(name) + ": invalid arguments");
        return MG_EINVAL;
    }
    std::vector<int32_t> lv, ij, tr;
    try {
        if (near)
            regrid_plan_near(t, near, c3, deref, h_deref, max_level, lv, ij, tr);
        else
            regrid_plan(t, scores, c3, deref, h_deref, max_level, lv, ij, tr);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return MG_ENOMEM;
    }
    *n_out = (int64_t)lv.size();
    if ((int64_t)lv.size() > cap) {
        set_error(std::string(name) + ": output capacity too small (n_out holds the size needed)");
        return MG_ENOMEM;
    }
    std::copy(lv.begin(), lv.end(), level);
    std::copy(ij.begin(), ij.end(), ijk);
    std::copy(tr.begin(), tr.end(), tree);
    return MG_OK;
}

int mg_regrid_plan(const mg_tree *t, const double *scores, double c3, double deref, double h_deref,
                   int max_level, int64_t cap, int32_t *level, int32_t *ijk, int32_t *tree, int64_t *n_out) {
    return plan_common(t, scores, nullptr, c3, deref, h_deref, max_level, cap, level, ijk, tree, n_out,
                       "mg_regrid_plan");
}

int mg_regrid_plan_near(const mg_tree *t, const double *near, double c3, double deref, double h_deref,
                        int max_level, int64_t cap, int32_t *level, int32_t *ijk, int32_t *tree,
                        int64_t *n_out) {
    if (!near) {
        set_error("mg_regrid_plan_near: null near");
        return MG_EINVAL;
    }
    return plan_common(t, nullptr, near, c3, deref, h_deref, max_level, cap, level, ijk, tree, n_out,
                       "mg_regrid_plan_near");
}

// ------------------------------------------------------------ fluid model

namespace {

void fluid_layout(const mg_tree *t, int32_t ntab, decltype(mg_tree::foff) &o) {
    int64_t at = 0;
    auto take = [&](int64_t bytes) {
        int64_t r = at;
        at += (bytes + 255) / 256 * 256;
        return r;
    };
    int64_t cells = t->n * 512 * (int64_t)sizeof(double);
    o.tab = take((int64_t)ntab * 6 * sizeof(double));
    o.cfrev = take(t->n * 24 * (int64_t)sizeof(int32_t));
    o.cf = take(t->nslot * 256 * (int64_t)sizeof(double));
    o.part = take(t->nleaf * (int64_t)sizeof(double));
    o.res = take(sizeof(double));
    o.n0e = take(cells);
    o.n0i = take(cells);
    o.n1e = take(cells);
    o.n1i = take(cells);
    o.ef = take(t->n * 1728 * (int64_t)sizeof(double));
    o.en = take(cells);
    o.total = at;
}

double *fdp(const mg_tree *t, int64_t off) { return (double *)((char *)t->fws + off); }
int32_t *fip(const mg_tree *t, int64_t off) { return (int32_t *)((char *)t->fws + off); }

int require_fluid(const mg_tree *t) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!t->fws) {
        set_error("no fluid workspace bound (call mg_fluid_bind first)");
        return MG_ESTATE;
    }
    return MG_OK;
}

int fluid_stage(mg_tree *t, const double *ef, const double *en, double *ne, const double *ni,
                const double *n0e, const double *n0i, double dt, double wa, double wb, double *oute,
                double *outi, double *lim) {
    hipStream_t s = stream_of(t);
    FluidArgs A;
    A.tab = {fdp(t, t->foff.tab), t->ntab, (double)(t->ntab - 1) / t->emax};
    A.isleaf = t->d.isleaf;
    A.cfrev = fip(t, t->foff.cfrev);
    A.leaf = t->d.leaf;
    A.slots = t->d.slots;
    A.nleaf = t->nleaf;
    A.nslot = t->nslot;
    A.ne = ne;
    A.ni = ni;
    A.n0e = n0e;
    A.n0i = n0i;
    A.ef = ef;
    A.en = en;
    A.dt = dt;
    A.wa = wa;
    A.wb = wb;
    A.oute = oute;
    A.outi = outi;
    A.rhs = t->d.rhs;
    A.cf = fdp(t, t->foff.cf);
    A.partial = fdp(t, t->foff.part);
    A.result = fdp(t, t->foff.res);
    launch_fluid_stage(geo(t, false), A, s);
    int rc = hip_check(hipGetLastError(), "fluid stage launch");
    if (rc || !lim) return rc;
    rc = hip_check(hipMemcpyAsync(t->host_result, A.result, sizeof(double), hipMemcpyDeviceToHost, s),
                   "fluid time-step bound copy");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "fluid stage");
    if (!rc) *lim = t->host_result[0];
    return rc;
}

}  // namespace

int64_t mg_fluid_workspace_bytes(const mg_tree *t, int32_t n_table) {
    if (!t || n_table < 2) {
        set_error("mg_fluid_workspace_bytes: null tree or fewer than 2 table entries");
        return -1;
    }
    decltype(mg_tree::foff) o;
    fluid_layout(t, n_table, o);
    return o.total;
}

int mg_fluid_bind(mg_tree *t, void *ws, int64_t bytes, const double *table, int32_t n_table, double e_max) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!ws || !table || n_table < 2 || !(e_max > 0.0) || !std::isfinite(e_max) || ((uintptr_t)ws & 255)) {
        set_error("mg_fluid_bind: null workspace or table, fewer than 2 entries, e_max <= 0, or a "
                  "workspace not aligned to 256 bytes");
        return MG_EINVAL;
    }
    for (int64_t q = 0; q < 3 * (int64_t)n_table; q++)
        if (!std::isfinite(table[q])) {
            set_error("mg_fluid_bind: non-finite table entry");
            return MG_EINVAL;
        }
    decltype(mg_tree::foff) o;
    fluid_layout(t, n_table, o);
    if (bytes < o.total) {
        set_error("mg_fluid_bind: workspace smaller than mg_fluid_workspace_bytes()");
        return MG_EINVAL;
    }
    // for a face of a leaf box whose same-level neighbour is refined: the
    // slots of the four children on it, ordered (t2 bit, t1 bit)
    std::vector<int32_t> rev((size_t)t->n * 24, -1);
    for (int64_t b = 0; b < t->n; b++)
        for (int d = 0; d < 6 && t->child[8 * b] < 0; d++) {
            int32_t N = t->nbr[6 * b + d];
            if (N < 0 || t->child[8 * (int64_t)N] < 0) continue;
            int a = d >> 1, t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            for (int tb2 = 0; tb2 < 2; tb2++)
                for (int tb1 = 0; tb1 < 2; tb1++) {
                    int bits[3];
                    bits[a] = (d & 1) ? 0 : 1;
                    bits[t1] = tb1;
                    bits[t2] = tb2;
                    int32_t c = t->child[8 * (int64_t)N + (bits[0] | (bits[1] << 1) | (bits[2] << 2))];
                    int32_t sl = c >= 0 ? t->cfslot[6 * (int64_t)c + (d ^ 1)] : -1;
                    if (sl < 0) {
                        set_error("mg_fluid_bind: a refined neighbour's child has no refinement-boundary slot");
                        return MG_ETOPO;
                    }
                    rev[(size_t)(b * 6 + d) * 4 + tb2 * 2 + tb1] = sl;
                }
        }
    // interval rows (entry k, entry k+1) per coefficient; the last row
    // repeats the last entry
    std::vector<double> rows((size_t)n_table * 6);
    for (int32_t k = 0; k < n_table; k++) {
        int32_t k1 = k + 1 < n_table ? k + 1 : k;
        for (int c = 0; c < 3; c++) {
            rows[6 * (size_t)k + 2 * c] = table[3 * (size_t)k + c];
            rows[6 * (size_t)k + 2 * c + 1] = table[3 * (size_t)k1 + c];
        }
    }
    hipStream_t s = stream_of(t);
    t->fws = ws;
    t->foff = o;
    t->ntab = n_table;
    t->emax = e_max;
    rc = hip_check(hipMemcpyAsync(fdp(t, o.tab), rows.data(), rows.size() * sizeof(double),
                                  hipMemcpyHostToDevice, s), "fluid table upload");
    if (!rc) rc = hip_check(hipMemcpyAsync(fip(t, o.cfrev), rev.data(), rev.size() * sizeof(int32_t),
                                           hipMemcpyHostToDevice, s), "fluid table upload");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "fluid bind");
    if (rc) t->fws = nullptr;
    return rc;
}

int mg_fluid_stage(mg_tree *t, const double *e_face, const double *e_norm, double *ne, const double *ni,
                   const double *n0e, const double *n0i, double dt, double wa, double wb, double *out_e,
                   double *out_i, double *dt_limit) {
    int rc = require_fluid(t);
    if (rc) return rc;
    if (!e_face || !e_norm || !ne || !ni || !n0e || !n0i || !out_e || !out_i || !std::isfinite(dt) ||
        dt < 0.0 || !std::isfinite(wa) || !std::isfinite(wb)) {
        set_error("mg_fluid_stage: null pointer or non-finite argument");
        return MG_EINVAL;
    }
    if (out_e == ne || out_e == ni || out_i == ne || out_i == ni || out_e == out_i) {
        set_error("mg_fluid_stage: outputs must not alias the inputs or each other");
        return MG_EINVAL;
    }
    return fluid_stage(t, e_face, e_norm, ne, ni, n0e, n0i, dt, wa, wb, out_e, out_i, dt_limit);
}

int mg_fluid_step(mg_tree *t, double *ne, double *ni, double dt, int32_t n_vcycles, double *dt_next) {
    int rc = require_fluid(t);
    if (rc) return rc;
    if (!ne || !ni || ne == ni || !std::isfinite(dt) || dt < 0.0 || n_vcycles < 1) {
        set_error("mg_fluid_step: null or aliased densities, bad dt, or n_vcycles < 1");
        return MG_EINVAL;
    }
    hipStream_t s = stream_of(t);
    size_t bytes = (size_t)t->n * 512 * sizeof(double);
    double *n0e = fdp(t, t->foff.n0e), *n0i = fdp(t, t->foff.n0i);
    double *n1e = fdp(t, t->foff.n1e), *n1i = fdp(t, t->foff.n1i);
    double *ef = fdp(t, t->foff.ef), *en = fdp(t, t->foff.en);
    rc = hip_check(hipMemcpyAsync(n0e, ne, bytes, hipMemcpyDeviceToDevice, s), "fluid step copy");
    if (!rc) rc = hip_check(hipMemcpyAsync(n0i, ni, bytes, hipMemcpyDeviceToDevice, s), "fluid step copy");
    mg_solve_opts o;
    mg_default_opts(&o);
    double lim = 0.0;
    // forward Euler stage, new field, second stage averaged with the kept
    // densities, new field (the explicit trapezoidal rule)
    if (!rc) rc = mg_efield(t, ef, en);
    if (!rc) rc = fluid_stage(t, ef, en, ne, ni, ne, ni, dt, 0.0, 1.0, n1e, n1i, nullptr);
    if (!rc) rc = vcycles_no_stats(t, &o, n_vcycles);
    if (!rc) rc = mg_efield(t, ef, en);
    if (!rc) rc = fluid_stage(t, ef, en, n1e, n1i, n0e, n0i, dt, 0.5, 0.5, ne, ni, &lim);
    if (!rc) rc = vcycles_no_stats(t, &o, n_vcycles);
    if (!rc && std::isnan(lim)) {
        set_error("mg_fluid_step: non-finite density after the step (time-step bound is NaN)");
        rc = MG_ENOCONV;
    }
    if (!rc && dt_next) *dt_next = 0.9 * lim;
    return rc;
}

int mg_transfer(mg_tree *from, mg_tree *to) {
    int rc = require_bound(from);
    if (!rc) rc = require_bound(to);
    if (rc) return rc;
    if (from == to) {
        set_error("mg_transfer: the two trees must differ");
        return MG_EINVAL;
    }
    for (int a = 0; a < 3; a++)
        if (from->dom.lo[a] != to->dom.lo[a]) rc = MG_EINVAL;
    if (rc || from->dom.len != to->dom.len) {
        set_error("mg_transfer: the trees cover different domains");
        return MG_EINVAL;
    }
    // the canonical order of both trees: (level, tree, Morton index), so one
    // merge pass over the two box arrays pairs the boxes
    auto key = [](const mg_tree *t, int64_t b) {
        return ((uint64_t)t->lev[b] << 58) | ((uint64_t)t->tid[b] << 42) |
               morton(t->ijk[3 * b], t->ijk[3 * b + 1], t->ijk[3 * b + 2]);
    };
    // new box -> old box with the same level and position (or -1); the boxes
    // without one, grouped by level, are interpolated from their parents
    std::vector<int32_t> src((size_t)to->n), list;
    std::vector<int64_t> lstart(to->nlev + 2, 0);
    try {
        int64_t a = 0;
        uint64_t ka = from->n ? key(from, 0) : ~0ull;
        for (int64_t b = 0; b < to->n; b++) {
            uint64_t kb = key(to, b);
            while (a < from->n && ka < kb) {
                a++;
                ka = a < from->n ? key(from, a) : ~0ull;
            }
            src[b] = a < from->n && ka == kb ? (int32_t)a : -1;
            if (src[b] < 0 && to->lev[b] == 1) {
                set_error("mg_transfer: a tree of the new forest has no counterpart in the old one");
                return MG_EINVAL;
            }
        }
        for (int l = 2; l <= to->nlev; l++) {
            lstart[l] = (int64_t)list.size();
            for (int64_t b = lbeg(to, l); b < lbeg(to, l) + lcount(to, l); b++)
                if (src[b] < 0) list.push_back((int32_t)b);
        }
        lstart[to->nlev + 1] = (int64_t)list.size();
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return MG_ENOMEM;
    }
    hipStream_t s = (hipStream_t)to->stream;
    // the maps go to the new tree's sweep buffer (scratch between calls)
    int32_t *d_src = (int32_t *)to->d.swp, *d_list = d_src + to->n;
    rc = hip_check(hipMemcpyAsync(d_src, src.data(), src.size() * 4, hipMemcpyHostToDevice, s), "map upload");
    if (!rc && !list.empty())
        rc = hip_check(hipMemcpyAsync(d_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, s),
                       "list upload");
    if (rc) return rc;
    // the old tree's covered cells <- mean of their children (on the new
    // tree's stream: the old tree must not be in use elsewhere)
    Fields<double> Fo = f64(from), Fn = f64(to);
    for (int l = from->nlev; l >= 2; l--) launch_restrict_phi<double>(Fo.g, Fo.phi, lbeg(from, l), lcount(from, l), s);
    dirty_all(Fo);
    launch_transfer_copy(Fo.phi, Fn.phi, d_src, to->n, s);
    for (int l = 2; l <= to->nlev; l++) {
        int64_t nl = lstart[l + 1] - lstart[l];
        if (nl <= 0) continue;
        // c_hat of the parents' level (reads level l-2, filled)
        launch_cf_coarse<double>(Fn.g, Fn.phi, Fn.chat, to->d.slots, to->sstart[l - 1],
                                 to->sstart[l] - to->sstart[l - 1], s);
        launch_transfer_interp(Fn.g, Fn.phi, Fn.chat, d_list + lstart[l], nl, s);
    }
    dirty_all(Fn);
    rc = hip_check(hipGetLastError(), "transfer launch");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "stream synchronize");  // host maps freed on return
    return rc;
}

int mg_residual(mg_tree *t, double *rel, double *l2, double *linf) {
    int rc = require_bound(t);
    if (rc) return rc;
    if ((rc = beff_norm(t))) return rc;
    mg_solve_stats s;
    std::memset(&s, 0, sizeof s);
    if ((rc = check_and_record(t, &s, 0))) return rc;
    if (rel) *rel = s.rel_res;
    if (l2) *l2 = s.l2;
    if (linf) *linf = s.linf;
    return MG_OK;
}

int mg_step(mg_tree *t, int op, int level, int arg) {
    int rc = require_bound(t);
    if (rc) return rc;
    bool fp32 = (op & MG_OP_F32) != 0;
    op &= ~MG_OP_F32;
    if (op != MG_OP_COARSE && op != MG_OP_RESTRICT_ALL && (level < 1 || level > t->nlev)) {
        set_error("level out of range");
        return MG_EINVAL;
    }
    if ((op == MG_OP_FAS_DOWN || op == MG_OP_PROLONG) && level < 2) {
        set_error("level out of range");
        return MG_EINVAL;
    }
    auto apply = [&](auto F) {
        switch (op) {
        case MG_OP_SMOOTH: smooth(t, F, level, arg); return (int)MG_OK;
        case MG_OP_FAS_DOWN: fas_down(t, F, level); return (int)MG_OK;
        case MG_OP_PROLONG: prolong(t, F, level); return (int)MG_OK;
        case MG_OP_COARSE: coarse(t, F); return (int)MG_OK;
        case MG_OP_RESTRICT_ALL: restrict_all(t, F); return (int)MG_OK;
        case MG_OP_VCYCLE: vcycle(t, F, level, arg, arg); return (int)MG_OK;
        default: set_error("unknown op"); return (int)MG_EINVAL;
        }
    };
    rc = fp32 ? apply(f32(t)) : apply(f64(t));
    if (rc) return rc;
    return hip_check(hipGetLastError(), "kernel launch");
}

int mg_tree_residuals(const mg_tree *t, double *rel) {
    if (!t || !rel) {
        set_error("null argument");
        return MG_EINVAL;
    }
    std::memcpy(rel, t->rel_tree.data(), t->rel_tree.size() * sizeof(double));
    return MG_OK;
}

int mg_autotune(mg_tree *t, int precision, int reps, int32_t *schedule) {
    // Near-ties go to the simpler launch: among the variants within kTuneTie
    // of the fastest, the lowest kernel family (v >> 1) wins, and within a
    // family the XCD-aware mapping (fewer HBM bytes).  Without it the choice
    // between variants a few tenths of a microsecond apart flips from run to
    // run on timing noise.
    constexpr double kTuneTie = 0.015;
    auto tune_rank = [](int v) { return 2 * (v >> 1) + ((v & 1) ? 0 : 1); };
    // warm-up, then the fastest of kTuneRuns timed runs of fn
    constexpr int kTuneRuns = 3;
    int rc = require_bound(t);
    if (rc) return rc;
    if ((precision != MG_FP64 && precision != MG_MIXED) || reps < 2 || reps > 1000 || (reps & 1)) {
        set_error("invalid autotune arguments (reps: even, 2..1000)");
        return MG_EINVAL;
    }
    bool fp32 = precision == MG_MIXED;
    hipStream_t s = (hipStream_t)t->stream;
    hipEvent_t e0 = take_event(t), e1 = take_event(t);
    if (!e0 || !e1) {
        set_error("event creation failed");
        return MG_EHIP;
    }
    // the sweeps change the field: park it in the old field (scratch between
    // calls) and restore it afterwards
    size_t bytes = (size_t)t->n * 512 * (fp32 ? sizeof(float) : sizeof(double));
    void *fld = fp32 ? (void *)t->d.e32 : (void *)t->d.phi;
    void *park = fp32 ? (void *)t->d.old32 : (void *)t->d.old;
    rc = hip_check(hipMemcpyAsync(park, fld, bytes, hipMemcpyDeviceToDevice, s), "park field");
    // level 1 is never smoothed: its entry (the bottom of the cycle as one
    // launch or step by step) is reported as set, not timed
    if (schedule) schedule[0] = t->sched[fp32 ? 1 : 0][1];
    auto time_ms = [&](auto &&fn) -> double {
        fn();
        double m = 1e30;
        for (int k = 0; k < kTuneRuns && !rc; k++) {
            rc = hip_check(hipEventRecord(e0, s), "event");
            fn();
            if (!rc) rc = hip_check(hipEventRecord(e1, s), "event");
            if (!rc) rc = hip_check(hipEventSynchronize(e1), "event sync");
            float ms = 0.0f;
            if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
            if (ms < m) m = ms;
        }
        return m;
    };
    for (int l = 2; l <= t->nlev && !rc; l++) {
        double h = hlev(t, l), best = 1e30;
        double tv[kGsrbVariants];
        // A level with refined boxes whose down-leg smoothing starts with a
        // fused pair gets its FAS right-hand side from that sweep, one
        // k_fas_rhs launch fewer per V-cycle: time the launches the timed
        // sweeps stand for (reps half-sweeps = reps / 8 V(2,2) cycles) on a
        // parked copy of the right-hand side and credit them to the fused
        // variants.
        double fas_ms = 0.0;
        const int64_t nref = t->rstart[l + 1] - t->rstart[l];
        if (l < t->nlev && nref > 0) {
            void *rh = fp32 ? (void *)t->d.r32 : (void *)t->d.rhs;
            auto fas_launches = [&](int k) {
                for (int q = 0; q < k; q++) {
                    if (fp32) {
                        Fields<float> F = f32(t);
                        launch_fas_rhs<float>(F.g, F.phi, F.rhs, F.chat, t->d.refined + t->rstart[l], nref,
                                              (float)(1.0 / (h * h)), s);
                    } else {
                        Fields<double> F = f64(t);
                        launch_fas_rhs<double>(F.g, F.phi, F.rhs, F.chat, t->d.refined + t->rstart[l], nref,
                                               1.0 / (h * h), s);
                    }
                }
            };
            rc = hip_check(hipMemcpyAsync(t->d.fas, rh, bytes, hipMemcpyDeviceToDevice, s), "park rhs");
            if (!rc) fas_ms = time_ms([&]() { fas_launches(reps / 8 > 0 ? reps / 8 : 1); });
            if (!rc) rc = hip_check(hipMemcpyAsync(rh, t->d.fas, bytes, hipMemcpyDeviceToDevice, s), "restore rhs");
        }
        for (int v = 0; v < kGsrbVariants && !rc; v++) {
            // reps half-sweeps, or reps/2 fused sweeps (the same work)
            auto sweeps = [&]() {
                bool fused = v >= kGsrbFusedVariant && v < kGsrbOctVariant;
                for (int q = 0; q < (fused ? reps / 2 : reps); q++) {
                    if (fp32) {
                        Fields<float> F = f32(t);
                        float *a = F.phi, *w = (float *)t->d.swp;
                        if (fused)
                            launch_gsrb_sweep<float>(F.g, q & 1 ? w : a, q & 1 ? a : w, F.rhs, F.chat,
                                                     lbeg(t, l), lcount(t, l), (float)(h * h), v & 1, s);
                        else
                            launch_gsrb<float>(F.g, F.phi, F.rhs, F.chat, lbeg(t, l), lcount(t, l),
                                               (float)(h * h), q & 1, v, s);
                    } else {
                        Fields<double> F = f64(t);
                        double *a = F.phi, *w = (double *)t->d.swp;
                        if (fused)
                            launch_gsrb_sweep<double>(F.g, q & 1 ? w : a, q & 1 ? a : w, F.rhs, F.chat,
                                                      lbeg(t, l), lcount(t, l), h * h, v & 1, s);
                        else
                            launch_gsrb<double>(F.g, F.phi, F.rhs, F.chat, lbeg(t, l), lcount(t, l),
                                                h * h, q & 1, v, s);
                    }
                }
            };
            tv[v] = time_ms(sweeps);
            if (v >= kGsrbFusedVariant && v < kGsrbOctVariant) tv[v] -= fas_ms;
            if (!rc && tv[v] < best) best = tv[v];
        }
        int pick = -1;
        for (int v = 0; v < kGsrbVariants && !rc; v++)
            if (tv[v] <= best * (1.0 + kTuneTie) && (pick < 0 || tune_rank(v) < tune_rank(pick))) pick = v;
        if (pick < 0) pick = kGsrbDefault;
        t->sched[fp32 ? 1 : 0][l] = pick;
        if (schedule) schedule[l - 1] = pick;
    }
    if (!rc) rc = hip_check(hipMemcpyAsync(fld, park, bytes, hipMemcpyDeviceToDevice, s), "restore field");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "stream synchronize");
    give_event(t, e0);
    give_event(t, e1);
    for (auto &g : t->graphs) drop_graph(g);  // re-record with the new schedule
    dirty_all(f64(t));
    dirty_all(f32(t));
    return rc;
}

int mg_set_fusion(mg_tree *t, int flags) {
    if (!t || (flags & ~MG_FUSE_ALL)) {
        set_error("mg_set_fusion: null tree or unknown flags");
        return MG_EINVAL;
    }
    if (flags != t->fusion) {
        for (auto &g : t->graphs) drop_graph(g);  // recorded sequences change
        t->fusion = flags;
    }
    return MG_OK;
}

int mg_set_schedule(mg_tree *t, int precision, const int32_t *schedule) {
    if (!t || !schedule || (precision != MG_FP64 && precision != MG_MIXED)) {
        set_error("invalid schedule arguments");
        return MG_EINVAL;
    }
    for (int l = 1; l <= t->nlev; l++) {
        if (schedule[l - 1] < 0 || schedule[l - 1] >= kGsrbVariants) {
            set_error("schedule entry out of range");
            return MG_EINVAL;
        }
    }
    for (int l = 1; l <= t->nlev; l++) t->sched[precision == MG_MIXED ? 1 : 0][l] = schedule[l - 1];
    for (auto &g : t->graphs) drop_graph(g);
    return MG_OK;
}

int mg_timing_enable(mg_tree *t, int enable) {
    if (!t) {
        set_error("null tree");
        return MG_EINVAL;
    }
    t->timing = enable != 0;
    return MG_OK;
}

int mg_timing_read(mg_tree *t, mg_kernel_timing_t *out) {
    int rc = require_bound(t);
    if (rc) return rc;
    if ((rc = hip_check(hipStreamSynchronize((hipStream_t)t->stream), "stream synchronize"))) return rc;
    mg_kernel_timing_t acc;
    std::memset(&acc, 0, sizeof acc);
    for (auto &p : t->probes) {
        float e = 0.0f;
        if ((rc = hip_check(hipEventElapsedTime(&e, (hipEvent_t)p.e0, (hipEvent_t)p.e1), "probe time")))
            return rc;
        acc.launches += p.launches;
        acc.total_ms += e;
        acc.alg_bytes += p.bytes;
        if (p.level >= 1 && p.level <= 16) {
            acc.level_launches[p.level - 1] += p.launches;
            acc.level_ms[p.level - 1] += e;
            acc.level_bytes[p.level - 1] += p.bytes;
        }
        give_event(t, (hipEvent_t)p.e0);
        give_event(t, (hipEvent_t)p.e1);
    }
    t->probes.clear();
    if (out) *out = acc;
    return MG_OK;
}

int mg_stream_copy(void *dst, const void *src, int64_t bytes, int blocks, void *stream) {
    if (!dst || !src || bytes < 0 || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) {
        set_error("stream copy: null pointer, or size or alignment not a multiple of 16");
        return MG_EINVAL;
    }
    if (blocks <= 0) {
        int dev = 0, cus = 0;
        int rc = hip_check(hipGetDevice(&dev), "current device");
        if (!rc) rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
                                "CU count");
        if (rc) return rc;
        blocks = 4 * cus;
    }
    launch_copy16(src, dst, bytes / 16, blocks, (hipStream_t)stream);
    return hip_check(hipGetLastError(), "stream copy launch");
}

// ---------------------------------------------------------- learned step

int64_t mg_nn_state_bytes(void) { return nn_state_layout(nullptr, nullptr); }

int mg_nn_create(mg_nn **out, void *state, int64_t state_bytes, void *stream) {
    if (!out || !state || ((uintptr_t)state & 255)) {
        set_error("null output, null state or state not 256-byte aligned");
        return MG_EINVAL;
    }
    *out = nullptr;
    if (state_bytes < mg_nn_state_bytes()) {
        set_error("network state too small");
        return MG_ENOMEM;
    }
    mg_nn *nn = new (std::nothrow) mg_nn();
    if (!nn) return MG_ENOMEM;
    nn_state_layout((char *)state, nn);
    nn->stream = stream;
    int rc = hip_check(hipGetDevice(&nn->device), "current device");
    if (!rc) rc = hip_check(hipHostMalloc((void **)&nn->host_loss, sizeof(double)), "pinned host buffer");
    if (!rc) {
        hipStream_t s = nn_stream(nn);
        for (float *p : {nn->prm, nn->m, nn->v, nn->grad}) launch_fill<float>(p, kNnParams, 0.0f, s);
        launch_nn_pack(nn->prm, nn->pk, s);
        rc = hip_check(hipGetLastError(), "network init");
        if (!rc) rc = hip_check(hipStreamSynchronize(s), "stream synchronize");
    }
    if (rc) {
        if (nn->host_loss) (void)hipHostFree(nn->host_loss);
        delete nn;
        return rc;
    }
    *out = nn;
    return MG_OK;
}

int mg_nn_destroy(mg_nn *nn) {
    if (!nn) return MG_OK;
    if (nn->host_loss) (void)hipHostFree(nn->host_loss);
    delete nn;
    return MG_OK;
}

int mg_nn_set_params(mg_nn *nn, const float *params) {
    int rc = require_nn(nn);
    if (rc) return rc;
    if (!params) {
        set_error("null parameters");
        return MG_EINVAL;
    }
    hipStream_t s = nn_stream(nn);
    rc = hip_check(hipMemcpyAsync(nn->prm, params, kNnParams * sizeof(float), hipMemcpyHostToDevice, s),
                   "parameter upload");
    if (rc) return rc;
    launch_fill<float>(nn->m, kNnParams, 0.0f, s);
    launch_fill<float>(nn->v, kNnParams, 0.0f, s);
    launch_nn_pack(nn->prm, nn->pk, s);
    nn->step = 0;
    rc = hip_check(hipGetLastError(), "parameter pack");
    return rc ? rc : hip_check(hipStreamSynchronize(s), "stream synchronize");
}

int mg_nn_get_params(mg_nn *nn, float *params) {
    int rc = require_nn(nn);
    if (rc) return rc;
    if (!params) {
        set_error("null parameters");
        return MG_EINVAL;
    }
    hipStream_t s = nn_stream(nn);
    rc = hip_check(hipMemcpyAsync(params, nn->prm, kNnParams * sizeof(float), hipMemcpyDeviceToHost, s),
                   "parameter readback");
    return rc ? rc : hip_check(hipStreamSynchronize(s), "stream synchronize");
}

int mg_nn_get_grad(mg_nn *nn, float *grad) {
    int rc = require_nn(nn);
    if (rc) return rc;
    if (!grad) {
        set_error("null gradient buffer");
        return MG_EINVAL;
    }
    hipStream_t s = nn_stream(nn);
    rc = hip_check(hipMemcpyAsync(grad, nn->grad, kNnParams * sizeof(float), hipMemcpyDeviceToHost, s),
                   "gradient readback");
    return rc ? rc : hip_check(hipStreamSynchronize(s), "stream synchronize");
}

int mg_nn_forward(mg_nn *nn, int64_t nbox, const float *x, float *y) {
    int rc = require_nn(nn);
    if (rc) return rc;
    if (nbox < 0 || nbox > INT32_MAX || (nbox > 0 && (!x || !y))) {
        set_error("invalid forward arguments");
        return MG_EINVAL;
    }
    launch_nn_forward(nn->prm, nn->pk, nbox, nullptr, x, y, nullptr, nullptr, nn_stream(nn));
    return hip_check(hipGetLastError(), "forward launch");
}

int64_t mg_nn_train_bytes(int64_t nbox) { return nn_train_layout(nbox < 0 ? 0 : nbox, nullptr, nullptr); }

int mg_nn_gradient(mg_nn *nn, int64_t nbox, const int32_t *idx, const float *x, const float *target,
                   void *ws, int64_t ws_bytes, double *loss) {
    int rc = require_nn(nn);
    if (rc) return rc;
    if (nbox <= 0 || nbox > INT32_MAX || !x || !target || !ws || ((uintptr_t)ws & 255)) {
        set_error("invalid gradient arguments");
        return MG_EINVAL;
    }
    if (ws_bytes < mg_nn_train_bytes(nbox)) {
        set_error("training workspace too small");
        return MG_ENOMEM;
    }
    return nn_gradient_run(nn, nbox, idx, x, target, (char *)ws, loss);
}

int mg_nn_gradient_static(mg_nn *nn, int64_t nbox, const int32_t *idx, const float *x,
                          const float *target, double *loss) {
    static_assert(MG_NN_STATIC_MAX_BOXES == kNnStaticBoxes && MG_NN_STATIC_BYTES == kNnStaticBytes,
                  "static training buffers: header and library disagree");
    int rc = require_nn(nn);
    if (rc) return rc;
    if (nbox <= 0 || !x || !target) {
        set_error("invalid gradient arguments");
        return MG_EINVAL;
    }
    if (nbox > MG_NN_STATIC_MAX_BOXES) {
        set_error("mg_nn_gradient_static: nbox " + std::to_string(nbox) + " exceeds " +
                  std::to_string(MG_NN_STATIC_MAX_BOXES) + " (use mg_nn_gradient with a workspace)");
        return MG_EINVAL;
    }
    void *ws = nullptr;
    if (nn_static_workspace(nn->device, &ws) != MG_OK) {
        set_error("mg_nn_gradient_static: no device address for the static training buffers");
        return MG_EHIP;
    }
    return nn_gradient_run(nn, nbox, idx, x, target, (char *)ws, loss);
}

int mg_nn_adam(mg_nn *nn, const mg_adam_opts *o) {
    int rc = require_nn(nn);
    if (rc) return rc;
    if (!o || !(o->lr >= 0) || !(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1) ||
        !(o->eps > 0)) {
        set_error("invalid Adam options");
        return MG_EINVAL;
    }
    nn->step++;
    double bc1 = 1.0 - std::pow(o->beta1, (double)nn->step), bc2 = 1.0 - std::pow(o->beta2, (double)nn->step);
    hipStream_t s = nn_stream(nn);
    launch_nn_adam(nn->prm, nn->m, nn->v, nn->grad, (float)o->lr, (float)o->beta1, (float)o->beta2,
                   (float)o->eps, (float)bc1, (float)bc2, s);
    launch_nn_pack(nn->prm, nn->pk, s);
    return hip_check(hipGetLastError(), "Adam launch");
}

int64_t mg_learned_bytes(const mg_tree *t) { return t ? learned_layout(t, nullptr, nullptr) : 0; }

int mg_nn_inputs(mg_tree *t, float *x, float *scale) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!x || !scale) {
        set_error("null output buffers");
        return MG_EINVAL;
    }
    Fields<float> E = f32(t);
    restrict_all(t, f64(t));
    norms_launch(t, 0, E.rhs);
    launch_nn_gather(E.rhs, t->d.leaf, t->nleaf, t->d.nbr, t->d.ijk, t->d.isleaf, t->dom.len, x, scale,
                     stream_of(t));
    return hip_check(hipGetLastError(), "input gather");
}

int mg_nn_targets(mg_tree *t, const double *ref, const float *scale, float *target) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!ref || !scale || !target) {
        set_error("null buffers");
        return MG_EINVAL;
    }
    launch_nn_targets(t->d.phi, ref, scale, t->d.leaf, t->nleaf, target, stream_of(t));
    return hip_check(hipGetLastError(), "targets");
}

int mg_learned_step(mg_tree *t, mg_nn *nn, void *ws, int64_t ws_bytes, double *steps) {
    int rc = require_bound(t);
    if (rc || (rc = require_nn(nn)) || (rc = check_learned_ws(t, ws, ws_bytes))) return rc;
    LearnedWs L;
    learned_layout(t, (char *)ws, &L);
    return learned_step_impl(t, nn, L, steps);
}

int mg_learned_level_step(mg_tree *t, mg_nn *nn, void *ws, int64_t ws_bytes, int level, double *steps) {
    int rc = require_bound(t);
    if (rc || (rc = require_nn(nn)) || (rc = check_learned_ws(t, ws, ws_bytes))) return rc;
    if (level < 3 || level > t->nlev) {
        set_error("mg_learned_level_step: level outside 3..n_levels");
        return MG_EINVAL;
    }
    LearnedWs L;
    learned_layout(t, (char *)ws, &L);
    if (steps)
        for (int tr = 0; tr < t->ntree; tr++) steps[tr] = 0.0;
    rc = learned_level_step(t, nn, L, level, steps);
    if (!rc) rc = hip_check(hipStreamSynchronize(stream_of(t)), "stream synchronize");
    return rc;
}

int mg_learned_solve(mg_tree *t, mg_nn *nn, void *ws, int64_t ws_bytes, const mg_solve_opts *o,
                     mg_solve_stats *st, mg_learned_stats *ls) {
    int rc = require_bound(t);
    if (rc || (rc = require_nn(nn)) || (rc = check_learned_ws(t, ws, ws_bytes)) || (rc = check_opts(o)))
        return rc;
    if (o->precision != MG_FP64) {
        set_error("the learned solve runs in FP64");
        return MG_EINVAL;
    }
    LearnedWs L;
    learned_layout(t, (char *)ws, &L);
    mg_solve_stats local;
    mg_solve_stats *s = st ? st : &local;
    std::memset(s, 0, sizeof *s);
    mg_learned_stats lloc;
    mg_learned_stats *lst = ls ? ls : &lloc;
    std::memset(lst, 0, sizeof *lst);
    if (o->learned_placement == 1) return learned_solve_levels(t, nn, L, o, s, lst);
    double t0 = now_ms();
    const int T = t->ntree;
    Fields<double> F = f64(t);
    const size_t bytes = (size_t)t->n * 512 * sizeof(double);
    if ((rc = run_seq(t, mg_tree::SEQ_FMG, o, 4 * T))) return s->status = rc;
    for (int tr = 0; tr < T; tr++) t->beff_tree[tr] = std::sqrt(t->host_result[2 * T + 2 * tr]);
    if ((rc = record_check(t, s, 0))) return s->status = rc;
    bool use = true;
    int stall = 0;
    for (int k = 1; s->rel_res > o->rel_tol; k++) {
        if (k > o->max_cycles) {
            set_error("no convergence within max_cycles");
            return s->status = MG_ENOCONV;
        }
        double prev = s->rel_res;
        if ((rc = run_seq(t, mg_tree::SEQ_VCHECK, o, 2 * T))) return s->status = rc;
        s->n_vcycles = k;
        if ((rc = record_check(t, s, k))) return s->status = rc;
        if (s->rel_res > o->rel_tol && use) {
            double tl = now_ms(), rel_v = s->rel_res;
            rc = hip_check(hipMemcpyAsync(F.old, F.phi, bytes, hipMemcpyDeviceToDevice, stream_of(t)),
                           "save phi");
            if (!rc) rc = learned_step_impl(t, nn, L, nullptr);
            if (rc) return s->status = rc;
            restrict_all(t, F);
            if ((rc = norms(t))) return s->status = rc;
            mg_solve_stats trial = *s;
            int rt = record_check(t, &trial, k);
            if (rt == MG_OK && trial.rel_res <= kLearnedKeep * rel_v) {
                *s = trial;
                lst->accepted++;
            } else {
                rc = hip_check(hipMemcpyAsync(F.phi, F.old, bytes, hipMemcpyDeviceToDevice, stream_of(t)),
                               "restore phi");
                if (rc) return s->status = rc;
                dirty_all(F);
                if ((rc = check_and_record(t, s, k))) return s->status = rc;
                use = false;
                lst->fallback_cycle = k;
            }
            lst->t_learned_ms += now_ms() - tl;
        }
        stall = s->rel_res >= prev ? stall + 1 : 0;
        if (stall >= 3) {
            set_error("residual stagnates");
            return s->status = MG_ENOCONV;
        }
    }
    restrict_all(t, F);  // every covered cell: the mean of its children
    rc = hip_check(hipGetLastError(), "kernel launch");
    s->t_ms = now_ms() - t0;
    s->nn_accepted = lst->accepted;
    s->nn_fell_back = lst->fallback_cycle;
    return s->status = rc;
}

int mg_nn_bind(mg_tree *t, mg_nn *nn, void *ws, int64_t ws_bytes) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!nn) {
        t->nn = nullptr;
        t->nn_ws = nullptr;
        t->nn_ws_bytes = 0;
        return MG_OK;
    }
    if ((rc = require_nn(nn)) || (rc = check_learned_ws(t, ws, ws_bytes))) return rc;
    t->nn = nn;
    t->nn_ws = ws;
    t->nn_ws_bytes = ws_bytes;
    return MG_OK;
}

}  // extern "C"
