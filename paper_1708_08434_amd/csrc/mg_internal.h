// Internal state of an mg_tree: host tables built by tree.cpp, device views
// carved out of the caller's workspace by mg_api.hip.
#pragma once
#include <algorithm>
#include <cstdint>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "mg.h"

namespace mg {

constexpr int kMaxLevel = 15;
constexpr int kCells = 512;      // cells per box
constexpr int kHalf = 256;       // cells of one colour per box

void set_error(const std::string &msg);

// f(lo, hi) over [0, n) in contiguous pieces on up to 16 host threads; one
// piece (the calling thread) below 16384 items per thread
template <typename F> void parallel_for(int64_t n, F f) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::min<int64_t>({(int64_t)(hw ? hw : 1), (int64_t)16, std::max<int64_t>(1, n / 16384)});
    if (nt <= 1) {
        f((int64_t)0, n);
        return;
    }
    int64_t per = (n + nt - 1) / nt;
    std::vector<std::thread> th;
    for (int64_t q = 1; q < nt; q++) {
        int64_t lo = q * per, hi = std::min(n, lo + per);
        if (lo < hi) th.emplace_back(f, lo, hi);
    }
    f((int64_t)0, std::min(n, per));
    for (auto &x : th) x.join();
}

// Host array of a trivially copyable type that is not value-initialised:
// the large index tables are filled by parallel loops that write every
// entry, so no serial prefill (and first touch) precedes them.
template <typename T> class RawArray {
  public:
    void reset(size_t n) {
        p_.reset(n ? new T[n] : nullptr);
        n_ = n;
    }
    T *data() { return p_.get(); }
    const T *data() const { return p_.get(); }
    size_t size() const { return n_; }
    T &operator[](size_t i) { return p_[i]; }
    const T &operator[](size_t i) const { return p_[i]; }

  private:
    std::unique_ptr<T[]> p_;
    size_t n_ = 0;
};

// Device-side views of the workspace; all pointers are into one allocation.
struct DevTables {
    int32_t *nbr = nullptr;      // [n][6]  face neighbour (-1 refinement boundary, -2 domain)
    int32_t *cfslot = nullptr;   // [n][6]  slot of a refinement-boundary face, or -1
    int32_t *cfq = nullptr;      // [n][6]  coarser box across a refinement-boundary face
    int32_t *xt = nullptr;       // [n][6][4][2] faces of the face neighbours (fused sweep)
    int32_t *n27 = nullptr;      // [n][27] same-level box at ijk + o (-1 coarser, -2 outside)
    int32_t *slotx = nullptr;    // [nslot][8] coarse-side indices of a slot's c_hat
    int32_t *ijk = nullptr;      // [n][4]  i, j, k, level
    int32_t *parent = nullptr;   // [n]
    int32_t *refined = nullptr;  // per-level lists of boxes with children
    int32_t *leaf = nullptr;     // per-level lists of boxes without children
    int32_t *cleaf = nullptr;    // leaf boxes whose parent cells a stopping test reads
    int32_t *oldcp = nullptr;    // per level: leaf boxes whose phi_old a prolongation reads
    int32_t *leafpos = nullptr;  // [n] position in the leaf list, -1 for boxes with children
    int32_t *cmask = nullptr;    // [n] 1 for the boxes of cleaf
    int32_t *slots = nullptr;    // [nslot][2] (box, face)
    int32_t *leaf_tree = nullptr;  // leaf-list positions grouped by tree (ascending within a tree)
    int32_t *tree_off = nullptr;   // [ntree+1] offsets into leaf_tree
    int32_t *chunk = nullptr;      // [nchunk][3] tree, begin, end of a norm-reduction chunk
    int32_t *choff = nullptr;      // [ntree+1] offsets into the chunks
    double *part2 = nullptr;       // [nchunk][2] first-stage sums
    int32_t *isleaf = nullptr;     // [n] 1 for a box without children
    int32_t *tid = nullptr;        // [n] tree of the box
    int32_t *root2 = nullptr;      // [ntree] first level-2 box of the tree, or -1
    double *eig = nullptr;       // root solve: Q_x, Q_y, Q_z (8x8, column = vector), then lambda_x,y,z
    double *phi = nullptr;       // [n][2][256] colour-split
    double *rhs = nullptr;
    double *old = nullptr;
    double *chat = nullptr;      // [nslot][64] tangentially interpolated coarse values
    double *bcval = nullptr;     // [n][6][64] or null
    double *partial = nullptr;   // [n_leaf][2] per-box residual sums
    double *result = nullptr;    // [4*ntree] per-tree (sum r^2 h^3, max |r|), then the same for phi = 0
    // FP32 correction fields of the mixed-precision solve (same layouts)
    float *e32 = nullptr;        // correction
    float *r32 = nullptr;        // its right-hand side (FP64 residual rounded, FAS data)
    float *old32 = nullptr;
    float *chat32 = nullptr;
    void *swp = nullptr;         // [n][512] FP64 (or FP32): target of the fused sweeps
    void *fas = nullptr;         // [n][512] FP64 (or FP32): FAS right-hand sides formed by a fused sweep
    void *dpad = nullptr;        // [refined boxes of a level][1000] FP64 (or FP32): padded corrections
};

}  // namespace mg

struct mg_nn;

struct mg_tree {
    // ---- host tables (canonical order) ----
    int64_t n = 0;
    int nlev = 0, ntree = 0;
    std::vector<int32_t> order, lev, ijk, tid, parent, child, nbr, cfq, cfslot, slotx;
    // (xt, the faces of the face neighbours, is formed on the GPU at bind)
    int64_t lstart[mg::kMaxLevel + 2] = {0};
    std::vector<int32_t> refined, leaf;                 // box ids grouped by level
    std::vector<int32_t> cleaf;                         // leaf boxes restricted before a stopping test
    std::vector<int32_t> oldcp;                         // per level: leaf boxes copied into phi_old
    std::vector<int32_t> leafpos;                       // [n] leaf-list position, -1 if refined
    std::vector<int32_t> cmask;                         // [n] 1 for the boxes of cleaf
    int64_t ostart[mg::kMaxLevel + 2] = {0};            // oldcp of level l: [ostart[l], ostart[l+1])
    int64_t rstart[mg::kMaxLevel + 2] = {0}, fstart[mg::kMaxLevel + 2] = {0};
    int64_t cstart[mg::kMaxLevel + 2] = {0};           // per-level offsets into cleaf
    std::vector<int32_t> slots;                         // (box, face) per slot
    mg::RawArray<int32_t> n27;                          // [n][27] same-level box at ijk + o, -1, -2
    std::vector<int32_t> root2;                         // first level-2 box per tree, or -1
    bool bottom_ok = false;                             // levels 1-2 can run as one launch
    std::vector<int32_t> leaf_tree, tree_off;           // leaf positions grouped by tree
    std::vector<int32_t> chunk, choff;                  // norm-reduction chunks (tree, begin, end)
    int64_t sstart[mg::kMaxLevel + 2] = {0};            // slots of level l: [sstart[l], sstart[l+1])
    int64_t nslot = 0, nleaf = 0;
    mg_domain dom{};
    double eig[3 * 64 + 3 * 8] = {0};
    // ---- workspace layout (byte offsets) ----
    struct { int64_t nbr, cfslot, cfq, xt, n27, slotx, ijk, parent, refined, leaf, cleaf, oldcp, leafpos, cmask, slots, leaf_tree, tree_off, chunk, choff, part2, isleaf, tid, root2, eig,
             phi, rhs, old, chat, bcval, partial, result, e32, r32, old32, chat32, swp, fas, dpad, total; } off{};
    // ---- fluid model (mg_fluid_bind): caller's second workspace ----
    void *fws = nullptr;
    int32_t ntab = 0;
    double emax = 0.0;
    struct { int64_t tab, cfrev, cf, part, res, n0e, n0i, n1e, n1i, ef, en, total; } foff{};
    // ---- bound device state ----
    void *ws = nullptr;
    void *stream = nullptr;      // caller's stream: every replay and direct launch goes here
    void *cur_stream = nullptr;  // stream the launchers use (the capture stream while capturing)
    void *cap_stream = nullptr;  // private stream used only to record graphs
    int cap_device = -1;         // device of cap_stream
    mg::DevTables d;
    bool cf_valid[mg::kMaxLevel + 2] = {false};    // c_hat of the FP64 field current per level
    bool cf_valid32[mg::kMaxLevel + 2] = {false};  // same for the FP32 correction field
    double *host_result = nullptr;  // pinned host buffer for norms, [4*ntree]
    size_t host_result_bytes = 0;    // its capacity
    std::vector<double> beff_tree, rel_tree;  // per tree: norm of the residual of phi = 0, last rel
    // ---- optional event timing of the half-sweep kernel ----
    // A probe is a pair of events around the consecutive half-sweeps of one
    // smoothing call, with its level, launch count and algorithmic bytes.
    struct Probe { void *e0, *e1; int level; int64_t launches; double bytes; };
    bool timing = false;
    std::vector<void *> ev_pool;       // hipEvent_t, reused
    std::vector<Probe> probes;         // probes since the last mg_timing_read
    // ---- recorded graphs (hipGraphExec_t), one per launch sequence ----
    struct Graph {
        void *exec = nullptr;
        int nd = -1, nu = -1;
        int nodes = 0;  // kernel launches recorded
        bool pre[2][mg::kMaxLevel + 2], post[2][mg::kMaxLevel + 2];  // c_hat validity
    };
    enum { SEQ_FMG = 0, SEQ_VCHECK, SEQ_MIX_START, SEQ_MIX_FMG, SEQ_MIX_V, SEQ_V, SEQ_COUNT };
    Graph graphs[SEQ_COUNT];
    // Gauss-Seidel launch variant per level, [0] FP64, [1] FP32 (autotuner);
    // the entry of level 1 (never smoothed) selects the bottom of the cycle:
    // 0 = levels 1 and 2 step by step, otherwise one launch (k_bottom)
    int32_t sched[2][mg::kMaxLevel + 2];
    int32_t fusion = MG_FUSE_ALL;  // mg_set_fusion flags
    // ---- hook after each level's up-sweeps in FP64 V-cycles (the per-level
    //      learned step; only set while V-cycles launch kernel by kernel) ----
    int (*level_hook)(mg_tree *, int level, void *ctx) = nullptr;
    void *hook_ctx = nullptr;
    int hook_rc = 0;
    // ---- network of MG_LEARNED solves (mg_nn_bind; caller-owned) ----
    mg_nn *nn = nullptr;
    void *nn_ws = nullptr;
    int64_t nn_ws_bytes = 0;
    mg_tree() {
        for (auto &row : sched)
            for (auto &v : row) v = 3;
    }
};

namespace mg {
int build_tree(mg_tree *t, const mg_domain *dom, int64_t n, const int32_t *level,
               const int32_t *ijk, const int32_t *tree);
// Morton code of a box position (bit b of i, j, k on bits 3b, 3b+1, 3b+2);
// within a level and tree, the canonical box order is increasing Morton code.
uint64_t morton(int32_t i, int32_t j, int32_t k);

// One regrid step (regrid.cpp): the new box list from per-box refinement
// scores; see mg_regrid_plan in mg.h.  regrid_near reduces the 27 scores of
// each leaf box and its neighbours to the one value the criterion tests
// (the host twin of k_refine_near), and regrid_plan_near plans from those.
int regrid_plan(const mg_tree *t, const double *scores, double c3, double deref, double h_deref,
                int max_level,
                std::vector<int32_t> &level, std::vector<int32_t> &ijk, std::vector<int32_t> &tree);
void regrid_near(const mg_tree *t, const double *scores, double *near);
int regrid_plan_near(const mg_tree *t, const double *near, double c3, double deref, double h_deref,
                     int max_level, std::vector<int32_t> &level, std::vector<int32_t> &ijk,
                     std::vector<int32_t> &tree);
void root_eigen(const int32_t bc_type[6], double *eig);
}
