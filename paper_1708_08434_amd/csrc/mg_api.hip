// C ABI and cycle driver of the octree multigrid solver.
//
// The driver enqueues the kernels of kernels.hip on the caller's stream in
// the order of the full-approximation-scheme FMG / V-cycle (paper section
// 2.1.2).  The only device-to-host transfer per cycle is the pair of
// reduced residual norms used by the stopping test.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "kernels.h"
#include "mg_internal.h"

namespace mg {

thread_local std::string g_error;
void set_error(const std::string &msg) { g_error = msg; }

namespace {

hipStream_t stream_of(const mg_tree *t) { return (hipStream_t)t->stream; }

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

Geo geo(const mg_tree *t) {
    Geo g;
    g.nbr = t->d.nbr;
    g.cfslot = t->d.cfslot;
    g.cfq = t->d.cfq;
    g.ijk = t->d.ijk;
    g.parent = t->d.parent;
    g.chat = t->d.chat;
    g.bcval = t->dom.per_cell_bc ? t->d.bcval : nullptr;
    for (int d = 0; d < 6; d++) {
        g.bcv[d] = t->dom.bc_val[d];
        g.bct[d] = t->dom.bc_type[d];
    }
    g.len = t->dom.len;
    return g;
}

// ---- refinement-boundary data: c_hat of level l depends on phi of level
// l-1 only; it is recomputed lazily after level l-1 changes.
void dirty(mg_tree *t, int l) {
    if (l + 1 <= kMaxLevel) t->cf_valid[l + 1] = false;
}
void dirty_all(mg_tree *t) {
    for (int l = 0; l <= kMaxLevel + 1; l++) t->cf_valid[l] = false;
}
void ensure_cf(mg_tree *t, int l) {
    if (l < 2 || l > t->nlev || t->cf_valid[l]) return;
    int64_t s0 = t->sstart[l], ns = t->sstart[l + 1] - t->sstart[l];
    launch_cf_coarse(geo(t), t->d.phi, t->d.chat, t->d.slots, s0, ns, stream_of(t));
    t->cf_valid[l] = true;
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

// ---- steps of the cycle
void smooth(mg_tree *t, int l, int nsweep) {
    if (nsweep <= 0) return;
    ensure_cf(t, l);
    double h = hlev(t, l), h2 = h * h;
    Geo g = geo(t);
    for (int it = 0; it < nsweep; it++)
        for (int c = 0; c < 2; c++) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (t->timing && (e0 = take_event(t)) && (e1 = take_event(t)))
                (void)hipEventRecord(e0, stream_of(t));
            launch_gsrb(g, t->d.phi, t->d.rhs, lbeg(t, l), lcount(t, l), h2, c, stream_of(t));
            if (e0 && e1) {
                (void)hipEventRecord(e1, stream_of(t));
                t->ev_pending.emplace_back((void *)e0, (void *)e1);
                t->ev_bytes += 6144.0 * (double)lcount(t, l);
            }
        }
    dirty(t, l);
}

void fas_down(mg_tree *t, int l) {
    ensure_cf(t, l);
    double h = hlev(t, l);
    launch_resid_restrict(geo(t), t->d.phi, t->d.rhs, t->d.old, lbeg(t, l), lcount(t, l),
                          t->d.leaf + t->fstart[l - 1], t->fstart[l] - t->fstart[l - 1],
                          1.0 / (h * h), stream_of(t));
    dirty(t, l - 1);
    ensure_cf(t, l - 1);
    double hc = hlev(t, l - 1);
    launch_fas_rhs(geo(t), t->d.phi, t->d.rhs, t->d.refined + t->rstart[l - 1],
                   t->rstart[l] - t->rstart[l - 1], 1.0 / (hc * hc), stream_of(t));
}

void prolong(mg_tree *t, int l) {
    launch_prolong(geo(t), t->d.phi, t->d.old, lbeg(t, l), lcount(t, l), stream_of(t));
    dirty(t, l);
}

void coarse(mg_tree *t) {
    launch_coarse(geo(t), t->d.phi, t->d.rhs, t->d.eig, lbeg(t, 1), lcount(t, 1), hlev(t, 1),
                  stream_of(t));
    dirty(t, 1);
}

void restrict_all(mg_tree *t) {
    for (int l = t->nlev; l >= 2; l--) {
        launch_restrict_phi(geo(t), t->d.phi, lbeg(t, l), lcount(t, l), stream_of(t));
        dirty(t, l - 1);
    }
}

void vcycle(mg_tree *t, int top, int nd, int nu) {
    for (int l = top; l >= 2; l--) {
        smooth(t, l, nd);
        fas_down(t, l);
    }
    coarse(t);
    for (int l = 2; l <= top; l++) {
        prolong(t, l);
        smooth(t, l, nu);
    }
}

int norms(mg_tree *t, double *l2, double *linf) {
    for (int l = 2; l <= t->nlev; l++) ensure_cf(t, l);
    launch_leaf_norms(geo(t), t->d.phi, t->d.rhs, t->d.leaf, t->nleaf, t->d.partial, stream_of(t));
    launch_reduce(t->d.partial, t->nleaf, t->d.result, stream_of(t));
    int rc = hip_check(hipMemcpyAsync(t->host_result, t->d.result, 2 * sizeof(double),
                                      hipMemcpyDeviceToHost, stream_of(t)), "norm readback");
    if (rc) return rc;
    if ((rc = hip_check(hipStreamSynchronize(stream_of(t)), "stream synchronize"))) return rc;
    *l2 = std::sqrt(t->host_result[0]);
    *linf = t->host_result[1];
    return MG_OK;
}

// Norm of the residual of phi = 0 (boundary data folded in).  The current
// phi is parked in the old field, which holds no state between calls (every
// down-leg rewrites it before the up-leg reads it).
int beff_norm(mg_tree *t, bool phi_is_zero, double *beff) {
    size_t bytes = (size_t)t->n * 512 * sizeof(double);
    int rc;
    double linf;
    if (!phi_is_zero) {
        if ((rc = hip_check(hipMemcpyAsync(t->d.old, t->d.phi, bytes, hipMemcpyDeviceToDevice,
                                           stream_of(t)), "park phi")))
            return rc;
        launch_fill(t->d.phi, 512 * t->n, 0.0, stream_of(t));
        dirty_all(t);
    }
    if ((rc = norms(t, beff, &linf))) return rc;
    if (!phi_is_zero) {
        if ((rc = hip_check(hipMemcpyAsync(t->d.phi, t->d.old, bytes, hipMemcpyDeviceToDevice,
                                           stream_of(t)), "restore phi")))
            return rc;
        dirty_all(t);
    }
    return MG_OK;
}

int check_and_record(mg_tree *t, double beff, mg_solve_stats *s, int k) {
    double l2, linf;
    restrict_all(t);
    int rc = norms(t, &l2, &linf);
    if (rc) return rc;
    double rel = beff > 0 ? l2 / beff : l2;
    s->rel_res = rel;
    s->l2 = l2;
    s->linf = linf;
    s->beff_l2 = beff;
    if (k < 64) s->rel_hist[k] = rel;
    if (!std::isfinite(rel)) {
        set_error("non-finite residual");
        return MG_ENOCONV;
    }
    return MG_OK;
}

int iterate(mg_tree *t, double beff, const mg_solve_opts *o, mg_solve_stats *s) {
    int stall = 0;
    for (int k = 1; s->rel_res > o->rel_tol; k++) {
        if (k > o->max_cycles) {
            set_error("no convergence within max_cycles");
            return MG_ENOCONV;
        }
        double prev = s->rel_res;
        vcycle(t, t->nlev, o->n_down, o->n_up);
        s->n_vcycles = k;
        int rc = check_and_record(t, beff, s, k);
        if (rc) return rc;
        stall = s->rel_res >= prev ? stall + 1 : 0;
        if (stall >= 3) {
            set_error("residual stagnates");
            return MG_ENOCONV;
        }
    }
    return MG_OK;
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
    if (!o || o->precision != MG_FP64 || o->n_down < 0 || o->n_up < 0 || o->max_cycles < 0 ||
        o->max_cycles > 10000 || !(o->rel_tol >= 0)) {
        set_error("invalid solver options");
        return MG_EINVAL;
    }
    return MG_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
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

int mg_tree_destroy(mg_tree *t) {
    if (!t) return MG_OK;
    if (t->host_result) (void)hipHostFree(t->host_result);
    for (auto &p : t->ev_pending) {
        t->ev_pool.push_back(p.first);
        t->ev_pool.push_back(p.second);
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

int mg_tree_bind(mg_tree *t, void *ws, int64_t bytes, void *stream) {
    if (!t || !ws) {
        set_error("null argument");
        return MG_EINVAL;
    }
    if (bytes < t->off.total || ((uintptr_t)ws & 255)) {
        set_error("workspace too small or not 256-byte aligned");
        return MG_ENOMEM;
    }
    t->ws = ws;
    t->stream = stream;
    char *base = (char *)ws;
    DevTables &d = t->d;
    d.nbr = (int32_t *)(base + t->off.nbr);
    d.cfslot = (int32_t *)(base + t->off.cfslot);
    d.cfq = (int32_t *)(base + t->off.cfq);
    d.ijk = (int32_t *)(base + t->off.ijk);
    d.parent = (int32_t *)(base + t->off.parent);
    d.refined = (int32_t *)(base + t->off.refined);
    d.leaf = (int32_t *)(base + t->off.leaf);
    d.slots = (int32_t *)(base + t->off.slots);
    d.eig = (double *)(base + t->off.eig);
    d.phi = (double *)(base + t->off.phi);
    d.rhs = (double *)(base + t->off.rhs);
    d.old = (double *)(base + t->off.old);
    d.chat = (double *)(base + t->off.chat);
    d.bcval = t->off.bcval >= 0 ? (double *)(base + t->off.bcval) : nullptr;
    d.partial = (double *)(base + t->off.partial);
    d.result = (double *)(base + t->off.result);
    if (!t->host_result) {
        int rc = hip_check(hipHostMalloc((void **)&t->host_result, 8 * sizeof(double)),
                           "pinned host buffer");
        if (rc) return rc;
    }
    std::vector<int32_t> ijk4((size_t)4 * t->n);
    for (int64_t b = 0; b < t->n; b++) {
        for (int a = 0; a < 3; a++) ijk4[4 * b + a] = t->ijk[3 * b + a];
        ijk4[4 * b + 3] = t->lev[b];
    }
    hipStream_t s = stream_of(t);
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "table upload")
                     : MG_OK;
    };
    int rc = MG_OK;
    rc = rc ? rc : up(d.nbr, t->nbr.data(), t->nbr.size() * 4);
    rc = rc ? rc : up(d.cfslot, t->cfslot.data(), t->cfslot.size() * 4);
    rc = rc ? rc : up(d.cfq, t->cfq.data(), t->cfq.size() * 4);
    rc = rc ? rc : up(d.ijk, ijk4.data(), ijk4.size() * 4);
    rc = rc ? rc : up(d.parent, t->parent.data(), t->parent.size() * 4);
    rc = rc ? rc : up(d.refined, t->refined.data(), t->refined.size() * 4);
    rc = rc ? rc : up(d.leaf, t->leaf.data(), t->leaf.size() * 4);
    rc = rc ? rc : up(d.slots, t->slots.data(), t->slots.size() * 4);
    rc = rc ? rc : up(d.eig, t->eig, sizeof t->eig);
    if (rc) return rc;
    launch_fill(d.phi, 512 * t->n, 0.0, s);
    launch_fill(d.rhs, 512 * t->n, 0.0, s);
    launch_fill(d.old, 512 * t->n, 0.0, s);
    if (d.bcval) launch_fill(d.bcval, 6 * 64 * t->n, 0.0, s);
    dirty_all(t);
    // the host vectors used as upload sources are freed on return
    return hip_check(hipStreamSynchronize(s), "bind");
}

int mg_field_set(mg_tree *t, int which, const double *dev) {
    int rc = require_bound(t);
    if (rc) return rc;
    hipStream_t s = stream_of(t);
    switch (which) {
    case MG_FIELD_PHI: launch_pack(dev, t->d.phi, t->n, s); dirty_all(t); break;
    case MG_FIELD_RHS: launch_pack(dev, t->d.rhs, t->n, s); break;
    case MG_FIELD_OLD: launch_pack(dev, t->d.old, t->n, s); break;
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
    case MG_FIELD_PHI: launch_unpack(t->d.phi, dev, t->n, s); break;
    case MG_FIELD_RHS: launch_unpack(t->d.rhs, dev, t->n, s); break;
    case MG_FIELD_OLD: launch_unpack(t->d.old, dev, t->n, s); break;
    default: set_error("unknown field"); return MG_EINVAL;
    }
    return hip_check(hipGetLastError(), "field get");
}

int mg_fmg_solve(mg_tree *t, const mg_solve_opts *o, mg_solve_stats *st) {
    int rc = require_bound(t);
    if (rc) return rc;
    if ((rc = check_opts(o))) return rc;
    mg_solve_stats local;
    mg_solve_stats *s = st ? st : &local;
    std::memset(s, 0, sizeof *s);
    double t0 = now_ms();
    launch_fill(t->d.phi, 512 * t->n, 0.0, stream_of(t));
    dirty_all(t);
    double beff;
    if ((rc = beff_norm(t, true, &beff))) return s->status = rc;
    for (int l = t->nlev; l >= 2; l--) fas_down(t, l);
    coarse(t);
    for (int l = 2; l <= t->nlev; l++) {
        prolong(t, l);
        vcycle(t, l, o->n_down, o->n_up);
    }
    if ((rc = check_and_record(t, beff, s, 0))) return s->status = rc;
    rc = iterate(t, beff, o, s);
    if (!rc) rc = hip_check(hipGetLastError(), "kernel launch");
    s->t_ms = now_ms() - t0;
    return s->status = rc;
}

int mg_vcycle(mg_tree *t, const mg_solve_opts *o, int n_cycles, mg_solve_stats *st) {
    int rc = require_bound(t);
    if (rc) return rc;
    if ((rc = check_opts(o))) return rc;
    mg_solve_stats local;
    mg_solve_stats *s = st ? st : &local;
    std::memset(s, 0, sizeof *s);
    double t0 = now_ms();
    double beff;
    if ((rc = beff_norm(t, false, &beff))) return s->status = rc;
    if ((rc = check_and_record(t, beff, s, 0))) return s->status = rc;
    if (n_cycles <= 0) {
        rc = iterate(t, beff, o, s);
    } else {
        for (int k = 1; k <= n_cycles && !rc; k++) {
            vcycle(t, t->nlev, o->n_down, o->n_up);
            s->n_vcycles = k;
            rc = check_and_record(t, beff, s, k);
        }
    }
    if (!rc) rc = hip_check(hipGetLastError(), "kernel launch");
    s->t_ms = now_ms() - t0;
    return s->status = rc;
}

int mg_residual(mg_tree *t, double *rel, double *l2, double *linf) {
    int rc = require_bound(t);
    if (rc) return rc;
    double beff, a, m;
    if ((rc = beff_norm(t, false, &beff))) return rc;
    restrict_all(t);
    if ((rc = norms(t, &a, &m))) return rc;
    if (rel) *rel = beff > 0 ? a / beff : a;
    if (l2) *l2 = a;
    if (linf) *linf = m;
    return MG_OK;
}

int mg_step(mg_tree *t, int op, int level, int arg) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (op != MG_OP_COARSE && op != MG_OP_RESTRICT_ALL && (level < 1 || level > t->nlev)) {
        set_error("level out of range");
        return MG_EINVAL;
    }
    switch (op) {
    case MG_OP_SMOOTH: smooth(t, level, arg); break;
    case MG_OP_FAS_DOWN:
        if (level < 2) { set_error("level out of range"); return MG_EINVAL; }
        fas_down(t, level);
        break;
    case MG_OP_PROLONG:
        if (level < 2) { set_error("level out of range"); return MG_EINVAL; }
        prolong(t, level);
        break;
    case MG_OP_COARSE: coarse(t); break;
    case MG_OP_RESTRICT_ALL: restrict_all(t); break;
    case MG_OP_VCYCLE: vcycle(t, level, arg, arg); break;
    default: set_error("unknown op"); return MG_EINVAL;
    }
    return hip_check(hipGetLastError(), "kernel launch");
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
    if ((rc = hip_check(hipStreamSynchronize(stream_of(t)), "stream synchronize"))) return rc;
    double ms = 0.0;
    for (auto &p : t->ev_pending) {
        float e = 0.0f;
        rc = hip_check(hipEventElapsedTime(&e, (hipEvent_t)p.first, (hipEvent_t)p.second), "event time");
        if (rc) return rc;
        ms += e;
        t->ev_pool.push_back(p.first);
        t->ev_pool.push_back(p.second);
    }
    if (out) {
        out->launches = (int64_t)t->ev_pending.size();
        out->total_ms = ms;
        out->alg_bytes = t->ev_bytes;
    }
    t->ev_pending.clear();
    t->ev_bytes = 0.0;
    return MG_OK;
}

}  // extern "C"
