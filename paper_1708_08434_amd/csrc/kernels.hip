// HIP kernels (gfx950) for geometric multigrid on an octree of 8^3 boxes.
//
// Storage: every field is [box][colour][256] with colour = (i+j+k) & 1 and,
// inside a colour, index (k*8 + j)*4 + (i>>1).  A red (or black) half-sweep
// of red-black Gauss-Seidel (paper section 2.1.2) therefore streams this
// colour's right-hand side and the other colour's solution as contiguous
// 2 KB runs and writes one contiguous 2 KB run per box, which is the minimum
// traffic of a half-sweep.  Boxes of one level are consecutive (canonical
// order), so a launch over a level streams one contiguous range.
//
// Ghost values are never stored: each kernel evaluates the ghost of a face
// cell on the fly from (a) the same-level neighbour box, (b) the physical
// boundary condition, or (c) at a refinement boundary, the coarse value
// interpolated tangentially (precomputed per level visit by k_cf_coarse) and
// the two interior fine cells along the normal.
#include <cmath>

#include "kernels.h"

namespace mg {
namespace {

constexpr double kSixth = 1.0 / 6.0;
constexpr double kCfCoarse = 8.0 / 15.0;  // quadratic through the coarse value,
constexpr double kCfFine1 = 2.0 / 3.0;    // the first and the second interior
constexpr double kCfFine2 = 0.2;          // fine cell (ghost at the face + h/2)

__device__ __forceinline__ int cs_idx(int i, int j, int k) {
    return (((i + j + k) & 1) << 8) + ((k * 8 + j) << 2) + (i >> 1);
}

// Workgroups are handed to the 8 XCDs in turn; give each XCD a contiguous run
// of boxes so that face neighbours of a box usually sit in the same L2.
__device__ __forceinline__ int64_t xcd_map(int64_t blk, int64_t n) {
    int64_t per = (n + 7) >> 3;
    return (blk & 7) * per + (blk >> 3);
}
__host__ __device__ inline int64_t xcd_grid(int64_t n) { return 8 * ((n + 7) >> 3); }

// Ghost of the face cell (u, v) on face d of box b.  src = index of the
// mirrored cell in the neighbour box; own = this face cell; inward = the next
// cell inwards along the normal.
__device__ __forceinline__ double ghost(const Geo &g, const double *__restrict__ phi, int64_t b,
                                        int d, int nb, int u, int v, int src, double own,
                                        double inward) {
    if (nb >= 0) return phi[(int64_t)nb * 512 + src];
    if (nb == -2) {
        if (g.bct[d] == 1) return own;
        double gv = g.bcval ? g.bcval[(b * 6 + d) * 64 + v * 8 + u] : g.bcv[d];
        return 2.0 * gv - own;
    }
    int slot = g.cfslot[b * 6 + d];
    return kCfCoarse * g.chat[(int64_t)slot * 64 + v * 8 + u] + kCfFine1 * own - kCfFine2 * inward;
}

// Sum of the six neighbours of cell (i, j, k) of box b (ghosts included), in
// the order -x, +x, -y, +y, -z, +z.
__device__ __forceinline__ double nbr_sum(const Geo &g, const double *__restrict__ phi, int64_t b,
                                          const int nb[6], int i, int j, int k, double own) {
    const double *P = phi + b * 512;
    double xm, xp, ym, yp, zm, zp;
    if (i > 0) xm = P[cs_idx(i - 1, j, k)];
    else xm = ghost(g, phi, b, 0, nb[0], j, k, cs_idx(7, j, k), own, P[cs_idx(1, j, k)]);
    if (i < 7) xp = P[cs_idx(i + 1, j, k)];
    else xp = ghost(g, phi, b, 1, nb[1], j, k, cs_idx(0, j, k), own, P[cs_idx(6, j, k)]);
    if (j > 0) ym = P[cs_idx(i, j - 1, k)];
    else ym = ghost(g, phi, b, 2, nb[2], i, k, cs_idx(i, 7, k), own, P[cs_idx(i, 1, k)]);
    if (j < 7) yp = P[cs_idx(i, j + 1, k)];
    else yp = ghost(g, phi, b, 3, nb[3], i, k, cs_idx(i, 0, k), own, P[cs_idx(i, 6, k)]);
    if (k > 0) zm = P[cs_idx(i, j, k - 1)];
    else zm = ghost(g, phi, b, 4, nb[4], i, j, cs_idx(i, j, 7), own, P[cs_idx(i, j, 1)]);
    if (k < 7) zp = P[cs_idx(i, j, k + 1)];
    else zp = ghost(g, phi, b, 5, nb[5], i, j, cs_idx(i, j, 0), own, P[cs_idx(i, j, 6)]);
    return xm + xp + ym + yp + zm + zp;
}

__device__ __forceinline__ void load_nbr(const Geo &g, int64_t b, int nb[6]) {
#pragma unroll
    for (int d = 0; d < 6; d++) nb[d] = g.nbr[b * 6 + d];
}

// ------------------------------------------------------------------ kernels

__global__ void k_fill(double *p, int64_t count, double v) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) p[q] = v;
}

__global__ __launch_bounds__(256) void k_pack(const double *__restrict__ nat, double *__restrict__ cs,
                                              int64_t nbox) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nbox * 512) return;
    int64_t b = q >> 9;
    int c = (int)(q & 511), i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    cs[b * 512 + cs_idx(i, j, k)] = nat[q];
}

__global__ __launch_bounds__(256) void k_unpack(const double *__restrict__ cs, double *__restrict__ nat,
                                                int64_t nbox) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nbox * 512) return;
    int64_t b = q >> 9;
    int c = (int)(q & 511), i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    nat[q] = cs[b * 512 + cs_idx(i, j, k)];
}

// One colour of red-black Gauss-Seidel on boxes [b0, b0+nb): 256 threads per
// box, one cell of colour C each.
template <int C>
__global__ __launch_bounds__(256) void k_gsrb(Geo g, double *__restrict__ phi,
                                              const double *__restrict__ rhs, int64_t b0, int64_t nbx,
                                              double h2) {
    int64_t lb = xcd_map(blockIdx.x, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    int t = threadIdx.x;
    int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
    int i = 2 * m + ((j + k + C) & 1);
    int nb[6];
    load_nbr(g, b, nb);
    double *P = phi + b * 512 + C * 256;
    double own = P[t];
    double s = nbr_sum(g, phi, b, nb, i, j, k, own);
    P[t] = (s - h2 * rhs[b * 512 + C * 256 + t]) * kSixth;
}

// Coarse value of cell D = C + dir * e_ax (level l-1, relative to box Q),
// with the coarse physical ghost outside the domain.
__device__ __forceinline__ double coarse_at(const Geo &g, const double *__restrict__ phi, int64_t Q,
                                            const int C[3], int ax, int dir) {
    int D[3] = {C[0], C[1], C[2]};
    D[ax] += dir;
    if (D[ax] >= 0 && D[ax] < 8) return phi[Q * 512 + cs_idx(D[0], D[1], D[2])];
    int face = 2 * ax + (dir > 0 ? 1 : 0);
    int N = g.nbr[Q * 6 + face];
    if (N >= 0) {
        D[ax] = dir > 0 ? 0 : 7;
        return phi[(int64_t)N * 512 + cs_idx(D[0], D[1], D[2])];
    }
    double in = phi[Q * 512 + cs_idx(C[0], C[1], C[2])];
    if (N != -2 || g.bct[face] == 1) return in;  // -1 cannot occur under 26-neighbour nesting
    int f1 = ax == 0 ? 1 : 0, f2 = ax == 2 ? 1 : 2;
    double gv = g.bcval ? g.bcval[(Q * 6 + face) * 64 + C[f2] * 8 + C[f1]] : g.bcv[face];
    return 2.0 * gv - in;
}

// Tangential quadratic interpolation of the coarse level at the 64 ghosts of
// one refinement-boundary face: c_hat = 7/8 c + sum_t [(1/32 + s_t/8) c_{+t}
// + (1/32 - s_t/8) c_{-t}], s_t = +-1 the side of the ghost in the coarse
// cell.  One 64-lane wavefront per face.
__global__ __launch_bounds__(64) void k_cf_coarse(Geo g, const double *__restrict__ phi,
                                                  double *__restrict__ chat,
                                                  const int32_t *__restrict__ slots, int64_t s0) {
    int64_t s = s0 + blockIdx.x;
    int64_t b = slots[2 * s];
    int d = slots[2 * s + 1];
    int a = d >> 1, side = d & 1;
    int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    int lane = threadIdx.x, u = lane & 7, v = lane >> 3;
    int64_t Q = g.cfq[b * 6 + d];
    int C[3];
    C[a] = side ? 0 : 7;
    C[t1] = 4 * (g.ijk[b * 4 + t1] & 1) + (u >> 1);
    C[t2] = 4 * (g.ijk[b * 4 + t2] & 1) + (v >> 1);
    double acc = 0.875 * phi[Q * 512 + cs_idx(C[0], C[1], C[2])];
#pragma unroll
    for (int q = 0; q < 2; q++) {
        int ax = q ? t2 : t1;
        double st = (((q ? v : u) & 1) ? 1.0 : -1.0);
        double cp = coarse_at(g, phi, Q, C, ax, 1);
        double cm = coarse_at(g, phi, Q, C, ax, -1);
        acc += (1.0 / 32.0 + st / 8.0) * cp + (1.0 / 32.0 - st / 8.0) * cm;
    }
    chat[s * 64 + lane] = acc;
}

// Residual on level l and restriction to level l-1 (full approximation
// scheme): every thread owns one parent cell, computes the residual of its
// 2x2x2 children, and writes phi_c = mean(phi), old_c = phi_c and
// rhs_c = mean(residual) (the coarse right-hand side is completed by
// k_fas_rhs).  Extra blocks copy phi -> old on the leaf boxes of level l-1.
__global__ __launch_bounds__(64) void k_resid_restrict(Geo g, double *__restrict__ phi,
                                                       double *__restrict__ rhs, double *__restrict__ old,
                                                       int64_t b0, int64_t nbx,
                                                       const int32_t *__restrict__ leaf_prev,
                                                       int64_t nleaf_prev, double inv_h2) {
    int64_t blk = blockIdx.x;
    int t = threadIdx.x;
    int64_t nmain = xcd_grid(nbx);
    if (blk >= nmain) {
        int64_t q = blk - nmain;
        if (q >= nleaf_prev) return;
        int64_t p = leaf_prev[q];
        for (int c = t; c < 512; c += 64) old[p * 512 + c] = phi[p * 512 + c];
        return;
    }
    int64_t lb = xcd_map(blk, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    int nb[6];
    load_nbr(g, b, nb);
    int pi = t & 3, pj = (t >> 2) & 3, pk = t >> 4;
    double sphi = 0.0, sres = 0.0;
#pragma unroll
    for (int dk = 0; dk < 2; dk++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int di = 0; di < 2; di++) {
                int i = 2 * pi + di, j = 2 * pj + dj, k = 2 * pk + dk;
                int c = cs_idx(i, j, k);
                double own = phi[b * 512 + c];
                double s = nbr_sum(g, phi, b, nb, i, j, k, own);
                double r = rhs[b * 512 + c] - (s - 6.0 * own) * inv_h2;
                sphi += own;
                sres += r;
            }
    int64_t p = g.parent[b];
    int ci = 4 * (g.ijk[b * 4] & 1) + pi, cj = 4 * (g.ijk[b * 4 + 1] & 1) + pj,
        ck = 4 * (g.ijk[b * 4 + 2] & 1) + pk;
    int64_t pc = p * 512 + cs_idx(ci, cj, ck);
    double mphi = 0.125 * sphi;
    phi[pc] = mphi;
    old[pc] = mphi;
    rhs[pc] = 0.125 * sres;
}

// rhs <- L phi + rhs on the listed (refined) boxes: completes the coarse
// right-hand side L_c(R phi) + R r of the full approximation scheme.
__global__ __launch_bounds__(256) void k_fas_rhs(Geo g, const double *__restrict__ phi,
                                                 double *__restrict__ rhs,
                                                 const int32_t *__restrict__ list, int64_t nlist,
                                                 double inv_h2) {
    int64_t q = xcd_map(blockIdx.x, nlist);
    if (q >= nlist) return;
    int64_t b = list[q];
    int nb[6];
    load_nbr(g, b, nb);
    int t = threadIdx.x, m = t & 3, j = (t >> 2) & 7, k = t >> 5;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        int i = 2 * m + ((j + k + c) & 1);
        int64_t idx = b * 512 + c * 256 + t;
        double own = phi[idx];
        double s = nbr_sum(g, phi, b, nb, i, j, k, own);
        rhs[idx] = (s - 6.0 * own) * inv_h2 + rhs[idx];
    }
}

// Correction delta = phi - old of box p at cell C shifted by s along axis a;
// outside p: the same-level face neighbour or the homogeneous physical ghost.
__device__ __forceinline__ double delta_at(const Geo &g, const double *__restrict__ phi,
                                           const double *__restrict__ old, int64_t p, const int nbp[6],
                                           const int C[3], int a, int s) {
    int D[3] = {C[0], C[1], C[2]};
    D[a] += s;
    if (D[a] >= 0 && D[a] < 8) {
        int64_t q = p * 512 + cs_idx(D[0], D[1], D[2]);
        return phi[q] - old[q];
    }
    int face = 2 * a + (s > 0 ? 1 : 0);
    int N = nbp[face];
    if (N >= 0) {
        D[a] = s > 0 ? 0 : 7;
        int64_t q = (int64_t)N * 512 + cs_idx(D[0], D[1], D[2]);
        return phi[q] - old[q];
    }
    int64_t q = p * 512 + cs_idx(C[0], C[1], C[2]);
    double din = phi[q] - old[q];
    return g.bct[face] == 1 ? din : -din;
}

// phi_f += 1/4 delta(C) + 1/4 (delta(C + s_x) + delta(C + s_y) + delta(C + s_z))
// with C the parent cell and s the side of the fine cell inside it.
__global__ __launch_bounds__(256) void k_prolong(Geo g, double *__restrict__ phi,
                                                 const double *__restrict__ old, int64_t b0, int64_t nbx) {
    int64_t lb = xcd_map(blockIdx.x, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    int64_t p = g.parent[b];
    int nbp[6];
    load_nbr(g, p, nbp);
    int B[3] = {g.ijk[b * 4], g.ijk[b * 4 + 1], g.ijk[b * 4 + 2]};
    int t = threadIdx.x, m = t & 3, j = (t >> 2) & 7, k = t >> 5;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        int i = 2 * m + ((j + k + c) & 1);
        int loc[3] = {i, j, k}, C[3], s[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            C[a] = 4 * (B[a] & 1) + (loc[a] >> 1);
            s[a] = (loc[a] & 1) ? 1 : -1;
        }
        int64_t qc = p * 512 + cs_idx(C[0], C[1], C[2]);
        double d0 = phi[qc] - old[qc];
        double dx = delta_at(g, phi, old, p, nbp, C, 0, s[0]);
        double dy = delta_at(g, phi, old, p, nbp, C, 1, s[1]);
        double dz = delta_at(g, phi, old, p, nbp, C, 2, s[2]);
        int64_t idx = b * 512 + c * 256 + t;
        phi[idx] += 0.25 * d0 + 0.25 * (dx + dy + dz);
    }
}

// Exact solve on each root box by fast diagonalisation: with the 1-D
// eigenbases V_a, phi = (V_z x V_y x V_x) diag(h^2 / (l_x + l_y + l_z))
// (V_z x V_y x V_x)^T rhs, where rhs has the Dirichlet data folded in.
__global__ __launch_bounds__(512) void k_coarse(Geo g, double *__restrict__ phi,
                                                const double *__restrict__ rhs,
                                                const double *__restrict__ eig, int64_t b0, double h) {
    __shared__ double X[512], Y[512], V[192], L[24];
    int64_t b = b0 + blockIdx.x;
    int t = threadIdx.x, i = t & 7, j = (t >> 3) & 7, k = t >> 6;
    if (t < 192) V[t] = eig[t];
    if (t < 24) L[t] = eig[192 + t];
    int c[3] = {i, j, k};
    double r = rhs[b * 512 + cs_idx(i, j, k)];
#pragma unroll
    for (int d = 0; d < 6; d++) {
        int a = d >> 1, s = d & 1;
        bool edge = s ? (c[a] == 7) : (c[a] == 0);
        if (edge && g.bct[d] == 0) {
            int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            double gv = g.bcval ? g.bcval[(b * 6 + d) * 64 + c[t2] * 8 + c[t1]] : g.bcv[d];
            r -= 2.0 * gv / (h * h);
        }
    }
    X[t] = r;
    __syncthreads();
    // forward: contract each axis with V_a^T
    { double s = 0; for (int q = 0; q < 8; q++) s += V[0 * 64 + q * 8 + i] * X[(k * 8 + j) * 8 + q]; Y[t] = s; }
    __syncthreads();
    { double s = 0; for (int q = 0; q < 8; q++) s += V[1 * 64 + q * 8 + j] * Y[(k * 8 + q) * 8 + i]; X[t] = s; }
    __syncthreads();
    { double s = 0; for (int q = 0; q < 8; q++) s += V[2 * 64 + q * 8 + k] * X[(q * 8 + j) * 8 + i]; Y[t] = s; }
    __syncthreads();
    Y[t] = Y[t] * (h * h) / (L[i] + L[8 + j] + L[16 + k]);
    __syncthreads();
    // inverse: contract each axis with V_a
    { double s = 0; for (int q = 0; q < 8; q++) s += V[2 * 64 + k * 8 + q] * Y[(q * 8 + j) * 8 + i]; X[t] = s; }
    __syncthreads();
    { double s = 0; for (int q = 0; q < 8; q++) s += V[1 * 64 + j * 8 + q] * X[(k * 8 + q) * 8 + i]; Y[t] = s; }
    __syncthreads();
    { double s = 0; for (int q = 0; q < 8; q++) s += V[0 * 64 + i * 8 + q] * Y[(k * 8 + j) * 8 + q]; X[t] = s; }
    phi[b * 512 + cs_idx(i, j, k)] = X[t];
}

// Covered cells of level l-1 <- mean of their 8 children on level l.
__global__ __launch_bounds__(64) void k_restrict_phi(Geo g, double *__restrict__ phi, int64_t b0,
                                                     int64_t nbx) {
    int64_t lb = xcd_map(blockIdx.x, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    int t = threadIdx.x, pi = t & 3, pj = (t >> 2) & 3, pk = t >> 4;
    double s = 0.0;
#pragma unroll
    for (int dk = 0; dk < 2; dk++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int di = 0; di < 2; di++) s += phi[b * 512 + cs_idx(2 * pi + di, 2 * pj + dj, 2 * pk + dk)];
    int64_t p = g.parent[b];
    int ci = 4 * (g.ijk[b * 4] & 1) + pi, cj = 4 * (g.ijk[b * 4 + 1] & 1) + pj,
        ck = 4 * (g.ijk[b * 4 + 2] & 1) + pk;
    phi[p * 512 + cs_idx(ci, cj, ck)] = 0.125 * s;
}

__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// Leaf residual norms: per listed box, sum of r^2 h^3 and max |r|.
__global__ __launch_bounds__(256) void k_leaf_norms(Geo g, const double *__restrict__ phi,
                                                    const double *__restrict__ rhs,
                                                    const int32_t *__restrict__ leaf, int64_t nleaf,
                                                    double *__restrict__ partial) {
    __shared__ double S[4], M[4];
    int64_t q = xcd_map(blockIdx.x, nleaf);
    if (q >= nleaf) return;
    int64_t b = leaf[q];
    int l = g.ijk[b * 4 + 3];
    double h = g.len / (8.0 * (double)(1 << (l - 1)));
    double inv_h2 = 1.0 / (h * h), vol = h * h * h;
    int nb[6];
    load_nbr(g, b, nb);
    int t = threadIdx.x, m = t & 3, j = (t >> 2) & 7, k = t >> 5;
    double ss = 0.0, mx = 0.0;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        int i = 2 * m + ((j + k + c) & 1);
        int64_t idx = b * 512 + c * 256 + t;
        double own = phi[idx];
        double s = nbr_sum(g, phi, b, nb, i, j, k, own);
        double r = rhs[idx] - (s - 6.0 * own) * inv_h2;
        ss += r * r;
        mx = nanmax(fabs(r), mx);
    }
    for (int off = 32; off > 0; off >>= 1) {
        ss += __shfl_xor(ss, off);
        mx = nanmax(__shfl_xor(mx, off), mx);
    }
    if ((t & 63) == 0) { S[t >> 6] = ss; M[t >> 6] = mx; }
    __syncthreads();
    if (t == 0) {
        partial[2 * q] = ((S[0] + S[1]) + (S[2] + S[3])) * vol;
        partial[2 * q + 1] = nanmax(nanmax(M[0], M[1]), nanmax(M[2], M[3]));
    }
}

// Deterministic reduction of the per-box partials (fixed order, one block).
__global__ __launch_bounds__(1024) void k_reduce(const double *__restrict__ partial, int64_t n,
                                                 double *__restrict__ result) {
    __shared__ double S[1024], M[1024];
    int t = threadIdx.x;
    double s = 0.0, m = 0.0;
    for (int64_t q = t; q < n; q += 1024) {
        s += partial[2 * q];
        m = nanmax(partial[2 * q + 1], m);
    }
    S[t] = s;
    M[t] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) {
            S[t] += S[t + w];
            M[t] = nanmax(M[t + w], M[t]);
        }
        __syncthreads();
    }
    if (t == 0) {
        result[0] = S[0];
        result[1] = M[0];
    }
}

}  // namespace

// ------------------------------------------------------------- launchers

void launch_fill(double *p, int64_t count, double v, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
}
void launch_pack(const double *nat, double *cs, int64_t nbox, hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3((unsigned)(nbox * 2)), dim3(256), 0, s, nat, cs, nbox);
}
void launch_unpack(const double *cs, double *nat, int64_t nbox, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)(nbox * 2)), dim3(256), 0, s, cs, nat, nbox);
}
void launch_gsrb(const Geo &g, double *phi, const double *rhs, int64_t b0, int64_t nb, double h2,
                 int colour, hipStream_t s) {
    if (nb <= 0) return;
    dim3 grid((unsigned)xcd_grid(nb));
    if (colour == 0) hipLaunchKernelGGL(k_gsrb<0>, grid, dim3(256), 0, s, g, phi, rhs, b0, nb, h2);
    else hipLaunchKernelGGL(k_gsrb<1>, grid, dim3(256), 0, s, g, phi, rhs, b0, nb, h2);
}
void launch_cf_coarse(const Geo &g, const double *phi, double *chat, const int32_t *slots,
                      int64_t s0, int64_t ns, hipStream_t s) {
    if (ns <= 0) return;
    hipLaunchKernelGGL(k_cf_coarse, dim3((unsigned)ns), dim3(64), 0, s, g, phi, chat, slots, s0);
}
void launch_resid_restrict(const Geo &g, double *phi, double *rhs, double *old, int64_t b0,
                           int64_t nb, const int32_t *leaf_prev, int64_t nleaf_prev,
                           double inv_h2, hipStream_t s) {
    if (nb + nleaf_prev <= 0) return;
    dim3 grid((unsigned)(xcd_grid(nb) + nleaf_prev));
    hipLaunchKernelGGL(k_resid_restrict, grid, dim3(64), 0, s, g, phi, rhs, old, b0, nb, leaf_prev,
                       nleaf_prev, inv_h2);
}
void launch_fas_rhs(const Geo &g, const double *phi, double *rhs, const int32_t *list,
                    int64_t nlist, double inv_h2, hipStream_t s) {
    if (nlist <= 0) return;
    hipLaunchKernelGGL(k_fas_rhs, dim3((unsigned)xcd_grid(nlist)), dim3(256), 0, s, g, phi, rhs, list,
                       nlist, inv_h2);
}
void launch_prolong(const Geo &g, double *phi, const double *old, int64_t b0, int64_t nb,
                    hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_prolong, dim3((unsigned)xcd_grid(nb)), dim3(256), 0, s, g, phi, old, b0, nb);
}
void launch_coarse(const Geo &g, double *phi, const double *rhs, const double *eig, int64_t b0,
                   int64_t nroot, double h, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse, dim3((unsigned)nroot), dim3(512), 0, s, g, phi, rhs, eig, b0, h);
}
void launch_restrict_phi(const Geo &g, double *phi, int64_t b0, int64_t nb, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_restrict_phi, dim3((unsigned)xcd_grid(nb)), dim3(64), 0, s, g, phi, b0, nb);
}
void launch_leaf_norms(const Geo &g, const double *phi, const double *rhs, const int32_t *leaf,
                       int64_t nleaf, double *partial, hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_leaf_norms, dim3((unsigned)xcd_grid(nleaf)), dim3(256), 0, s, g, phi, rhs,
                       leaf, nleaf, partial);
}
void launch_reduce(const double *partial, int64_t n, double *result, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, partial, n, result);
}

}  // namespace mg
