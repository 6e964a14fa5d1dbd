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
    const int32_t *ijk;     // [n][4] (i, j, k, level)
    const int32_t *parent;  // [n]
    const double *chat;     // [nslot][64]
    const double *bcval;    // [n][6][64] or null
    double bcv[6];
    int32_t bct[6];
    double len;
};

void launch_fill(double *p, int64_t count, double v, hipStream_t s);
void launch_pack(const double *nat, double *cs, int64_t nbox, hipStream_t s);
void launch_unpack(const double *cs, double *nat, int64_t nbox, hipStream_t s);
void launch_gsrb(const Geo &g, double *phi, const double *rhs, int64_t b0, int64_t nb, double h2,
                 int colour, hipStream_t s);
void launch_cf_coarse(const Geo &g, const double *phi, double *chat, const int32_t *slots,
                      int64_t s0, int64_t ns, hipStream_t s);
void launch_resid_restrict(const Geo &g, double *phi, double *rhs, double *old, int64_t b0,
                           int64_t nb, const int32_t *leaf_prev, int64_t nleaf_prev,
                           double inv_h2, hipStream_t s);
void launch_fas_rhs(const Geo &g, const double *phi, double *rhs, const int32_t *list,
                    int64_t nlist, double inv_h2, hipStream_t s);
void launch_prolong(const Geo &g, double *phi, const double *old, int64_t b0, int64_t nb,
                    hipStream_t s);
void launch_coarse(const Geo &g, double *phi, const double *rhs, const double *eig, int64_t b0,
                   int64_t nroot, double h, hipStream_t s);
void launch_restrict_phi(const Geo &g, double *phi, int64_t b0, int64_t nb, hipStream_t s);
void launch_leaf_norms(const Geo &g, const double *phi, const double *rhs, const int32_t *leaf,
                       int64_t nleaf, double *partial, hipStream_t s);
void launch_reduce(const double *partial, int64_t n, double *result, hipStream_t s);

}  // namespace mg
