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
// Each stencil kernel stages one box and its one-cell ghost layer in LDS
// (section 2.1.3: a ghost layer lets every box be worked on independently).
// Ghosts are never stored in HBM; dedicated threads evaluate them from
// (a) the same-level neighbour box, (b) the physical boundary condition, or
// (c) at a refinement boundary, the tangentially interpolated coarse value
// (precomputed per level visit by the coarse-face pass) and the two interior
// fine cells along the normal.  All global loads of a thread are independent
// of each other, so a kernel costs one memory round trip plus one barrier.
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
__device__ __forceinline__ int cs_idx3(const int c[3]) { return cs_idx(c[0], c[1], c[2]); }

// Workgroups are handed to the 8 XCDs in turn; give each XCD a contiguous run
// of boxes so that face neighbours of a box usually sit in the same L2.
__device__ __forceinline__ int64_t xcd_map(int64_t blk, int64_t n) {
    int64_t per = (n + 7) >> 3;
    return (blk & 7) * per + (blk >> 3);
}
__host__ __device__ inline int64_t xcd_grid(int64_t n) { return 8 * ((n + 7) >> 3); }

__device__ __forceinline__ void tangential(int a, int &t1, int &t2) {
    t1 = a == 0 ? 1 : 0;
    t2 = a == 2 ? 1 : 2;
}

// max that carries NaN through (a non-finite residual must reach the test)
// Loads of data that a launch reads exactly once (right-hand sides) carry
// the non-temporal hint, so that they do not displace from L2 the cells that
// neighbouring workgroups re-read as ghosts.
#ifndef MG_STREAM_RHS
#define MG_STREAM_RHS 1
#endif
template <typename T> struct StreamLd {
    static __device__ __forceinline__ T ld(const T *p) {
#if MG_STREAM_RHS
        return __builtin_nontemporal_load(p);
#else
        return *p;
#endif
    }
};
template <typename E, typename V, int N> struct StreamVec {
    typedef E native __attribute__((ext_vector_type(N)));
    static __device__ __forceinline__ V ld(const V *p) {
#if MG_STREAM_RHS
        native v = __builtin_nontemporal_load(reinterpret_cast<const native *>(p));
        V r;
#pragma unroll
        for (int i = 0; i < N; i++) reinterpret_cast<E *>(&r)[i] = v[i];
        return r;
#else
        return *p;
#endif
    }
};
template <> struct StreamLd<double2> : StreamVec<double, double2, 2> {};
template <> struct StreamLd<double4> : StreamVec<double, double4, 4> {};
template <> struct StreamLd<float2> : StreamVec<float, float2, 2> {};
template <> struct StreamLd<float4> : StreamVec<float, float4, 4> {};
template <typename T> __device__ __forceinline__ T ld_stream(const T *p) { return StreamLd<T>::ld(p); }

__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// Ghost values: Dirichlet face value gv reflected through the boundary cell,
// and the refinement-boundary quadratic through the coarse value ch and the
// first two interior fine cells.  Every kernel evaluates them through these
// two functions, so all paths round identically.
template <typename T> __device__ __forceinline__ T dirichlet_ghost(T gv, T own) {
    return (T)2 * gv - own;
}
// Fused multiply-adds written out, so that every kernel rounds the
// refinement-boundary ghost the same way whatever the compiler would contract.
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <typename T> __device__ __forceinline__ T cf_ghost(T ch, T own, T inward) {
    return fmadd((T)kCfCoarse, ch, fmadd((T)kCfFine1, own, -((T)kCfFine2 * inward)));
}
// Residual b - (s - 6 own) / h^2 of a cell with neighbour sum s, with the
// multiply-adds written out so that every kernel that forms a residual
// (restriction, stopping test, bottom of the cycle) rounds it alike.
template <typename T> __device__ __forceinline__ T resid_of(T b, T s, T own, T inv_h2) {
    return fmadd(-fmadd((T)-6, own, s), inv_h2, b);
}
template <typename T>
__device__ __forceinline__ T bc_value(const Geo &g, int64_t b, int d, int u, int v) {
    return (T)(g.bcval ? g.bcval[(b * 6 + d) * 64 + v * 8 + u] : g.bcv[d]);
}

// Ghost of face cell (u, v) on face d of box b, read straight from global
// memory.  nb = nbr[b][d]; slot = cfslot[b][d].  T is the field type (double,
// or float for the correction cycles of the mixed-precision solve).
template <typename T>
__device__ __forceinline__ T ghost_at(const Geo &g, const T *__restrict__ phi,
                                      const T *__restrict__ chat, int64_t b, int d, int nb, int slot,
                                      int u, int v) {
    int a = d >> 1, side = d & 1, t1, t2;
    tangential(a, t1, t2);
    int c[3];
    c[t1] = u;
    c[t2] = v;
    if (nb >= 0) {
        c[a] = side ? 0 : 7;  // mirrored cell in the neighbour
        return phi[(int64_t)nb * 512 + cs_idx3(c)];
    }
    c[a] = side ? 7 : 0;
    T own = phi[b * 512 + cs_idx3(c)];
    if (nb == -2) {
        if (g.bct[d] == 1) return own;
        return dirichlet_ghost<T>(bc_value<T>(g, b, d, u, v), own);
    }
    c[a] = side ? 6 : 1;
    T inward = phi[b * 512 + cs_idx3(c)];
    return cf_ghost<T>(chat[(int64_t)slot * 64 + v * 8 + u], own, inward);
}

// The face tables of box b, read with block-uniform addresses (scalar loads
// issued at kernel start), so that a ghost's value load waits on no vector
// load of an index.
struct FaceTab {
    int nb[6], slot[6];
};
__device__ __forceinline__ FaceTab face_tab(const Geo &g, int64_t b) {
    FaceTab f;
#pragma unroll
    for (int d = 0; d < 6; d++) {
        f.nb[d] = g.nbr[b * 6 + d];
        f.slot[d] = g.cfslot[b * 6 + d];
    }
    return f;
}
__device__ __forceinline__ int pick6(const int v[6], int d) {
    return d == 0 ? v[0] : d == 1 ? v[1] : d == 2 ? v[2] : d == 3 ? v[3] : d == 4 ? v[4] : v[5];
}

// Stage the whole box (both colours, colour-split order) into P[512] and all
// 6 x 64 face ghosts into H[d*64 + v*8 + u]; 256 threads.  Caller syncs.
template <typename T>
__device__ __forceinline__ void stage_full(const Geo &g, const T *__restrict__ phi,
                                           const T *__restrict__ chat, int64_t b, T *P, T *H) {
    int t = threadIdx.x;
    const FaceTab ft = face_tab(g, b);
    P[t] = phi[b * 512 + t];
    P[256 + t] = phi[b * 512 + 256 + t];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        int e = t + 256 * r;
        if (e < 384) {
            int d = e >> 6, w = e & 63;
            H[e] = ghost_at<T>(g, phi, chat, b, d, pick6(ft.nb, d), pick6(ft.slot, d), w & 7, w >> 3);
        }
    }
}

// Six-neighbour sum of cell (i, j, k) from a staged box, order -x, +x, -y,
// +y, -z, +z.
template <typename T>
__device__ __forceinline__ T sum_full(const T *P, const T *H, int i, int j, int k) {
    T xm = i > 0 ? P[cs_idx(i - 1, j, k)] : H[0 * 64 + k * 8 + j];
    T xp = i < 7 ? P[cs_idx(i + 1, j, k)] : H[1 * 64 + k * 8 + j];
    T ym = j > 0 ? P[cs_idx(i, j - 1, k)] : H[2 * 64 + k * 8 + i];
    T yp = j < 7 ? P[cs_idx(i, j + 1, k)] : H[3 * 64 + k * 8 + i];
    T zm = k > 0 ? P[cs_idx(i, j, k - 1)] : H[4 * 64 + j * 8 + i];
    T zp = k < 7 ? P[cs_idx(i, j, k + 1)] : H[5 * 64 + j * 8 + i];
    return xm + xp + ym + yp + zm + zp;
}

// ------------------------------------------------------------------ kernels

template <typename T>
__global__ void k_fill(T *p, int64_t count, T v) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) p[q] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pack(const double *__restrict__ nat, T *__restrict__ cs,
                                              int64_t nbox) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nbox * 512) return;
    int64_t b = q >> 9;
    int c = (int)(q & 511), i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    cs[b * 512 + cs_idx(i, j, k)] = (T)nat[q];
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(const T *__restrict__ cs, double *__restrict__ nat,
                                                int64_t nbox) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nbox * 512) return;
    int64_t b = q >> 9;
    int c = (int)(q & 511), i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    nat[q] = (double)cs[b * 512 + cs_idx(i, j, k)];
}

// One colour C of red-black Gauss-Seidel on boxes [b0, b0+nbx): 256/CPT
// threads per box, CPT neighbouring cells of colour C each (vector loads of
// CPT values, so a wave keeps CPT times the bytes in flight).  LDS holds the
// other colour S[256] and the 6 x 32 ghosts of this colour's face cells,
// H[d*32 + v*4 + (u>>1)].  XCD-aware box mapping when xcd != 0.  CPT and the
// mapping are the launch variants the autotuner chooses from; every variant
// performs the same arithmetic on every cell.
template <typename T>
__device__ __forceinline__ T gsrb_ghost_val(const Geo &g, const FaceTab &ft, const T *__restrict__ phi,
                                            const T *__restrict__ chat, int64_t b, int C, int e) {
    int d = e >> 5, q = e & 31, v = q >> 2;
    int layer = (d & 1) ? 7 : 0;
    int u = 2 * (q & 3) + ((layer + v + C) & 1);
    return ghost_at<T>(g, phi, chat, b, d, pick6(ft.nb, d), pick6(ft.slot, d), u, v);
}
template <typename T>
__device__ __forceinline__ void gsrb_ghost(const Geo &g, const FaceTab &ft, const T *__restrict__ phi,
                                           const T *__restrict__ chat, int64_t b, int C, int e, T *H) {
    H[e] = gsrb_ghost_val<T>(g, ft, phi, chat, b, C, e);
}

template <typename T, int N> struct VecN;
template <> struct VecN<double, 1> { using type = double; };
template <> struct VecN<double, 2> { using type = double2; };
template <> struct VecN<double, 4> { using type = double4; };
template <> struct VecN<float, 1> { using type = float; };
template <> struct VecN<float, 2> { using type = float2; };
template <> struct VecN<float, 4> { using type = float4; };

// Restriction of a box's 512 values (colour-split, in LDS) onto its parent's
// cells: the mean of the 8 children under each, k_restrict_leaves' order.
template <typename T>
__device__ __forceinline__ void restrict_box(const Geo &g, const T *U, int64_t b, T *__restrict__ dst, int e) {
    int pi = e & 3, pj = (e >> 2) & 3, pk = e >> 4;
    T sum = 0;
#pragma unroll
    for (int dk = 0; dk < 2; dk++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int di = 0; di < 2; di++) sum += U[cs_idx(2 * pi + di, 2 * pj + dj, 2 * pk + dk)];
    int64_t p = g.parent[b];
    int ci = 4 * (g.ijk[b * 4] & 1) + pi, cj = 4 * (g.ijk[b * 4 + 1] & 1) + pj, ck = 4 * (g.ijk[b * 4 + 2] & 1) + pk;
    dst[p * 512 + cs_idx(ci, cj, ck)] = (T)0.125 * sum;
}

// phi64 += (double) e on N cells of each colour at colour-half position q0
// (k_ir_update's arithmetic); the updated values are also left in U
// (colour-split) when U is set.
template <typename T, int N>
__device__ __forceinline__ void ir_add(double *__restrict__ phi64, int64_t b, int C, int q0, const T *eC,
                                       const T *eO, double *U) {
    using D = typename VecN<double, N>::type;
    D *pc = reinterpret_cast<D *>(phi64 + b * 512 + C * 256 + q0);
    D *po = reinterpret_cast<D *>(phi64 + b * 512 + (1 - C) * 256 + q0);
    D vc = *pc, vo = *po;
    double *xc = reinterpret_cast<double *>(&vc), *xo = reinterpret_cast<double *>(&vo);
#pragma unroll
    for (int w = 0; w < N; w++) {
        xc[w] += (double)eC[w];
        xo[w] += (double)eO[w];
    }
    *pc = vc;
    *po = vo;
    if (U) {
#pragma unroll
        for (int w = 0; w < N; w++) {
            U[C * 256 + q0 + w] = xc[w];
            U[(1 - C) * 256 + q0 + w] = xo[w];
        }
    }
}

// Modes of the black half-sweep when it is a box's last sweep of the cycle
// before a stopping test:
//  kSweepRestrict: boxes with rmask[b] != 0 also set their parent cells to
//    the mean of the 8 children under each, from the swept values.
//  kSweepIrUpdate (FP32 correction cycle): phi64 += e on all 512 cells of
//    the box (the refinement update), and boxes with rmask set restrict the
//    updated phi64 onto their parents (rmask may be null).
constexpr int kSweepPlain = 0, kSweepRestrict = 1, kSweepIrUpdate = 2;
template <int C, typename T, int CPT, int MODE = kSweepPlain>
__global__ __launch_bounds__(256 / CPT) void k_gsrb(Geo g, T *__restrict__ phi,
                                                    const T *__restrict__ rhs,
                                                    const T *__restrict__ chat, int64_t b0,
                                                    int64_t nbx, T h2, int xcd,
                                                    const int32_t *__restrict__ rmask = nullptr,
                                                    double *__restrict__ phi64 = nullptr) {
    using V = typename VecN<T, CPT>::type;
    constexpr int NT = 256 / CPT;
    __shared__ T SB[MODE == kSweepRestrict ? 512 : 256], H[192];
    __shared__ double U[MODE == kSweepIrUpdate ? 512 : 1];
    T *S = SB;
    int64_t lb = xcd ? xcd_map(blockIdx.x, nbx) : (int64_t)blockIdx.x;
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    int t = threadIdx.x;
    const FaceTab ft = face_tab(g, b);
    V o = reinterpret_cast<const V *>(phi + b * 512 + (1 - C) * 256)[t];
    V bv = ld_stream(reinterpret_cast<const V *>(rhs + b * 512 + C * 256) + t);
#pragma unroll
    for (int e = t; e < 192; e += NT) gsrb_ghost<T>(g, ft, phi, chat, b, C, e, H);
    reinterpret_cast<V *>(S)[t] = o;
    __syncthreads();
    const T *bb = reinterpret_cast<const T *>(&bv);
    V res;
    T *out = reinterpret_cast<T *>(&res);
#pragma unroll
    for (int w = 0; w < CPT; w++) {
        int cq = CPT * t + w;
        int m = cq & 3, j = (cq >> 2) & 7, k = cq >> 5;
        int i = 2 * m + ((j + k + C) & 1);
        int row = (k * 8 + j) * 4;
        T xm = i > 0 ? S[row + ((i - 1) >> 1)] : H[0 * 32 + k * 4 + (j >> 1)];
        T xp = i < 7 ? S[row + ((i + 1) >> 1)] : H[1 * 32 + k * 4 + (j >> 1)];
        T ym = j > 0 ? S[row - 4 + m] : H[2 * 32 + k * 4 + m];
        T yp = j < 7 ? S[row + 4 + m] : H[3 * 32 + k * 4 + m];
        T zm = k > 0 ? S[row - 32 + m] : H[4 * 32 + j * 4 + m];
        T zp = k < 7 ? S[row + 32 + m] : H[5 * 32 + j * 4 + m];
        T s = xm + xp + ym + yp + zm + zp;
        out[w] = (s - h2 * bb[w]) * (T)kSixth;
    }
    reinterpret_cast<V *>(phi + b * 512 + C * 256)[t] = res;
    if (MODE == kSweepRestrict && rmask[b]) {  // block-uniform
        // SB: colour 0 (the staged other colour) then colour 1 (this sweep's)
        reinterpret_cast<V *>(SB + 256)[t] = res;
        __syncthreads();
        for (int e = t; e < 64; e += NT) restrict_box<T>(g, SB, b, phi, e);
    }
    if (MODE == kSweepIrUpdate) {
        const bool r = rmask && rmask[b];  // block-uniform
        ir_add<T, CPT>(phi64, b, C, CPT * t, out, reinterpret_cast<const T *>(&o), r ? U : nullptr);
        if (r) {
            __syncthreads();
            for (int e = t; e < 64; e += NT) restrict_box<double>(g, U, b, phi64, e);
        }
    }
}

// Workgroup barrier that orders LDS only: global loads issued before it stay
// in flight (the prefetch of the next box), unlike __syncthreads().
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One colour C of red-black Gauss-Seidel with persistent workgroups of 128
// threads (2 cells each): workgroup w takes boxes base, base + step, ...
// (with the XCD mapping: the boxes of its XCD's contiguous range, in turn
// with the XCD's other workgroups), and while it updates one box it has the
// next box's cells, right-hand side and ghosts in flight and the face table
// of the one after.  The ghosts of a box read only the other colour and the
// box's own cells, which no workgroup writes during this half-sweep before
// the box itself is updated, so loading them early changes nothing.  Same
// arithmetic per cell as k_gsrb.
template <int C, typename T>
__global__ __launch_bounds__(128) void k_gsrb_pipe(Geo g, T *__restrict__ phi, const T *__restrict__ rhs,
                                                   const T *__restrict__ chat, int64_t b0, int64_t nbx,
                                                   T h2, int xcd) {
    using V = typename VecN<T, 2>::type;
    __shared__ T S[256], H[192];
    const int t = threadIdx.x;
    int64_t base, step, end;
    if (xcd) {
        int64_t per = (nbx + 7) >> 3, x = blockIdx.x & 7;
        base = x * per + (blockIdx.x >> 3);
        step = gridDim.x >> 3;
        end = min((x + 1) * per, nbx);
    } else {
        base = blockIdx.x;
        step = gridDim.x;
        end = nbx;
    }
    if (base >= end) return;
    int64_t b = b0 + base;
    FaceTab ft = face_tab(g, b);
    V o = reinterpret_cast<const V *>(phi + b * 512 + (1 - C) * 256)[t];
    V bv = ld_stream(reinterpret_cast<const V *>(rhs + b * 512 + C * 256) + t);
    T g0 = gsrb_ghost_val<T>(g, ft, phi, chat, b, C, t);
    T g1 = t < 64 ? gsrb_ghost_val<T>(g, ft, phi, chat, b, C, t + 128) : (T)0;
    int64_t nxt = base + step;
    FaceTab ftn = ft;
    if (nxt < end) ftn = face_tab(g, b0 + nxt);
    for (;;) {
        const bool more = nxt < end;
        const int64_t bn = b0 + nxt;
        V on = o, bvn = bv;
        T g0n = 0, g1n = 0;
        FaceTab ftnn = ftn;
        if (more) {
            on = reinterpret_cast<const V *>(phi + bn * 512 + (1 - C) * 256)[t];
            bvn = ld_stream(reinterpret_cast<const V *>(rhs + bn * 512 + C * 256) + t);
            g0n = gsrb_ghost_val<T>(g, ftn, phi, chat, bn, C, t);
            if (t < 64) g1n = gsrb_ghost_val<T>(g, ftn, phi, chat, bn, C, t + 128);
            if (nxt + step < end) ftnn = face_tab(g, bn + step);
        }
        reinterpret_cast<V *>(S)[t] = o;
        H[t] = g0;
        if (t < 64) H[t + 128] = g1;
        lds_sync();
        const T *bb = reinterpret_cast<const T *>(&bv);
        V res;
        T *out = reinterpret_cast<T *>(&res);
#pragma unroll
        for (int w = 0; w < 2; w++) {
            int cq = 2 * t + w;
            int m = cq & 3, j = (cq >> 2) & 7, k = cq >> 5;
            int i = 2 * m + ((j + k + C) & 1);
            int row = (k * 8 + j) * 4;
            T xm = i > 0 ? S[row + ((i - 1) >> 1)] : H[0 * 32 + k * 4 + (j >> 1)];
            T xp = i < 7 ? S[row + ((i + 1) >> 1)] : H[1 * 32 + k * 4 + (j >> 1)];
            T ym = j > 0 ? S[row - 4 + m] : H[2 * 32 + k * 4 + m];
            T yp = j < 7 ? S[row + 4 + m] : H[3 * 32 + k * 4 + m];
            T zm = k > 0 ? S[row - 32 + m] : H[4 * 32 + j * 4 + m];
            T zp = k < 7 ? S[row + 32 + m] : H[5 * 32 + j * 4 + m];
            T s = xm + xp + ym + yp + zm + zp;
            out[w] = (s - h2 * bb[w]) * (T)kSixth;
        }
        reinterpret_cast<V *>(phi + b * 512 + C * 256)[t] = res;
        lds_sync();
        if (!more) break;
        b = bn;
        o = on;
        bv = bvn;
        g0 = g0n;
        g1 = g1n;
        ftn = ftnn;
        nxt += step;
    }
}

// One colour C of red-black Gauss-Seidel on the octets (complete sets of 8
// sibling boxes, consecutive in canonical order) of boxes [b0, b0+8*noct):
// one 512-thread workgroup per octet, which is a 16^3 grid.  Faces between
// siblings are read from LDS, so only the octet's outer surface (6 x 128
// cells of this colour) needs ghosts: half the ghost traffic per cell of the
// one-box launches.  S holds the other colour of the 16^3 grid (colour-split
// rows: (K*16 + J)*8 + I/2); thread t owns one box row (4 cells) of colour C,
// read and written as one vector.  Same arithmetic per cell as k_gsrb.  IR:
// k_gsrb's kSweepIrUpdate mode (each box's 64 threads restrict it).
template <int C, typename T, bool IR = false>
__global__ __launch_bounds__(512) void k_gsrb_oct(Geo g, T *__restrict__ phi, const T *__restrict__ rhs,
                                                  const T *__restrict__ chat, int64_t b0, int64_t noct,
                                                  T h2, int xcd, const int32_t *__restrict__ rmask = nullptr,
                                                  double *__restrict__ phi64 = nullptr) {
    using V4 = typename VecN<T, 4>::type;
    __shared__ T S[2048], H[6 * 128];
    __shared__ double U[IR ? 8 * 512 : 1];
    int64_t lo = xcd ? xcd_map(blockIdx.x, noct) : (int64_t)blockIdx.x;
    if (lo >= noct) return;
    int64_t ob = b0 + 8 * lo;
    int t = threadIdx.x;
    int o = t >> 6, rw = t & 63, j = rw & 7, k = rw >> 3;  // box of the octet, row (j, k) in it
    int64_t bx = ob + o;
    int ox = 8 * (o & 1), oy = 8 * ((o >> 1) & 1), oz = 8 * (o >> 2);
    // other colour of row (j, k) of box o: 4 values, I/2 = ox/2 + m
    V4 so = reinterpret_cast<const V4 *>(phi + bx * 512 + (1 - C) * 256)[rw];
    V4 bv = ld_stream(reinterpret_cast<const V4 *>(rhs + bx * 512 + C * 256) + rw);
    // ghosts of the outer surface: entry e = d*128 + v*8 + u/2 over the
    // 16 x 16 face (u along t1, v along t2), cells of colour C
    for (int e = t; e < 768; e += 512) {
        int d = e >> 7, q = e & 127, v = q >> 3;
        int a = d >> 1, side = d & 1;
        int L = side ? 15 : 0;
        int u = 2 * (q & 7) + ((L + v + C) & 1);
        int c[3];  // octant of the box holding face cell (u, v)
        c[a] = side;
        c[a == 0 ? 1 : 0] = u >> 3;
        c[a == 2 ? 1 : 2] = v >> 3;
        int64_t gb = ob + (c[0] | (c[1] << 1) | (c[2] << 2));
        H[e] = ghost_at<T>(g, phi, chat, gb, d, g.nbr[gb * 6 + d], g.cfslot[gb * 6 + d], u & 7, v & 7);
    }
    {
        const T *sv = reinterpret_cast<const T *>(&so);
        int row = ((oz + k) * 16 + oy + j) * 8 + (ox >> 1);
#pragma unroll
        for (int m = 0; m < 4; m++) S[row + m] = sv[m];
    }
    __syncthreads();
    const T *bb = reinterpret_cast<const T *>(&bv);
    V4 res;
    T *out = reinterpret_cast<T *>(&res);
    int J = oy + j, K = oz + k, row = (K * 16 + J) * 8;
#pragma unroll
    for (int m = 0; m < 4; m++) {
        int I = ox + 2 * m + ((j + k + C) & 1);
        T xm = I > 0 ? S[row + ((I - 1) >> 1)] : H[0 * 128 + K * 8 + (J >> 1)];
        T xp = I < 15 ? S[row + ((I + 1) >> 1)] : H[1 * 128 + K * 8 + (J >> 1)];
        T ym = J > 0 ? S[row - 8 + (I >> 1)] : H[2 * 128 + K * 8 + (I >> 1)];
        T yp = J < 15 ? S[row + 8 + (I >> 1)] : H[3 * 128 + K * 8 + (I >> 1)];
        T zm = K > 0 ? S[row - 128 + (I >> 1)] : H[4 * 128 + J * 8 + (I >> 1)];
        T zp = K < 15 ? S[row + 128 + (I >> 1)] : H[5 * 128 + J * 8 + (I >> 1)];
        T s = xm + xp + ym + yp + zm + zp;
        out[m] = (s - h2 * bb[m]) * (T)kSixth;
    }
    reinterpret_cast<V4 *>(phi + bx * 512 + C * 256)[rw] = res;
    if (IR) {
        ir_add<T, 4>(phi64, bx, C, 4 * rw, out, reinterpret_cast<const T *>(&so), rmask ? U + o * 512 : nullptr);
        if (rmask) {
            __syncthreads();
            if (rmask[bx]) restrict_box<double>(g, U + o * 512, bx, phi64, rw);
        }
    }
}

// One full red-black sweep (red half, then black half) of boxes [b0, b0+nbx)
// of one level, reading src and writing both colours to dst (src is left
// unchanged, dst must not alias it).  The values are those of the two
// half-sweeps of k_gsrb: the black half needs the new red values of the
// neighbours' face layers, so each box recomputes the 6 x 32 red cells of its
// same-level face neighbours that touch its black face cells, with the red
// update's own arithmetic on the old field (a red cell reads only black cells
// and ghosts).  Their inputs are staged in LDS once: the neighbour's adjacent
// layer of black cells (which are also the ghosts of this box's red face
// cells), its second layer under the recomputed cells, their right-hand
// side, and the ghosts of the recomputed cells on the neighbour's edges.  One
// launch per sweep instead of two, with the same 24 B per cell plus the
// neighbours' face layers.  256 threads per box; thread t owns red cell t
// and black cell 256 + t (colour-split order), and for t < 192 face entry t:
// face d = t / 32, position q = t % 32 in the layer.
//
// The first sweep after a restriction can also complete the coarse
// right-hand side of the full approximation scheme (the values k_fas_rhs
// writes: L src + the restricted residual, on the boxes with children):
// fas = 1 computes it from src, which no workgroup writes, smooths with it
// and stores it in fasbuf; the right-hand side of a refined face neighbour
// under a recomputed red cell is formed the same way from the same inputs
// plus that cell's old value.  fas = 2 (the next sweep) reads those values
// from fasbuf and copies a box's own back into rhs; nothing reads rhs of a
// box with children meanwhile, so the copy races with no read.
template <typename T, bool FAS>
__global__ __launch_bounds__(256) void k_gsrb_sweep(Geo g, const T *__restrict__ src,
                                                    T *__restrict__ dst, T *__restrict__ rhs,
                                                    const T *__restrict__ chat, int64_t b0,
                                                    int64_t nbx, T h2, int xcd, int fas,
                                                    const int32_t *__restrict__ isleaf, T inv_h2,
                                                    T *__restrict__ fasbuf) {
    // P: red part = new red values (after the red half), black part = old
    // black values.  HR: ghosts of the red face cells (old field).  D2, BH:
    // second-layer black value and right-hand side of each recomputed red
    // cell.  EG: ghosts of the recomputed cells across the neighbour's
    // tangential faces (4 edges x 4 cells per face).  HB: per black face
    // cell, the recomputed red value across a same-level face, the Dirichlet
    // value at a domain face, or c_hat at a refinement boundary.  With
    // fas = 1 on a box with children: PR, the old red values, and GB, the
    // ghosts of the black face cells; NR, the old value of each recomputed
    // red cell of a neighbour with children.
    __shared__ T P[512], HR[192], D2[192], BH[192], EG[96], HB[192];
    __shared__ T PR[FAS ? 256 : 1], GB[FAS ? 192 : 1], NR[FAS ? 192 : 1];
    int64_t lb = xcd ? xcd_map(blockIdx.x, nbx) : (int64_t)blockIdx.x;
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    int t = threadIdx.x;
    const FaceTab ft = face_tab(g, b);
    if (!FAS) fas = 0;
    const bool own_fas = fas != 0 && isleaf[b] == 0;
    T ob = src[b * 512 + 256 + t];
    T br, bb;
    if (own_fas && fas == 2) {
        br = fasbuf[b * 512 + t];
        bb = fasbuf[b * 512 + 256 + t];
        rhs[b * 512 + t] = br;
        rhs[b * 512 + 256 + t] = bb;
    } else {
        br = rhs[b * 512 + t];
        bb = rhs[b * 512 + 256 + t];
    }
    T orr = (T)0;
    if (own_fas && fas == 1) orr = src[b * 512 + t];
    // face entry of this thread (t < 192): the black face cell (ub, v) of
    // face d, u along t1 and v along t2, at layer lx of this box
    int fd = t >> 5, fq = t & 31, fv = fq >> 2;
    int fa = fd >> 1, fside = fd & 1, ft1, ft2;
    tangential(fa, ft1, ft2);
    int flx = fside ? 7 : 0;
    int fub = 2 * (fq & 3) + ((flx + fv + 1) & 1);
    int fnb = t < 192 ? pick6(ft.nb, fd) : -3;
    bool nb_fas = fas != 0 && fnb >= 0 && isleaf[fnb] == 0;
    if (t < 192) {
        gsrb_ghost<T>(g, ft, src, chat, b, 0, t, HR);
        if (own_fas && fas == 1) gsrb_ghost<T>(g, ft, src, chat, b, 1, t, GB);
        if (fnb >= 0) {
            int c[3];
            c[ft1] = fub;
            c[ft2] = fv;
            c[fa] = fside ? 1 : 6;  // neighbour's second layer
            D2[t] = src[(int64_t)fnb * 512 + cs_idx3(c)];
            c[fa] = fside ? 0 : 7;  // neighbour's adjacent layer: the recomputed red cell
            if (nb_fas && fas == 2) {
                BH[t] = fasbuf[(int64_t)fnb * 512 + cs_idx3(c)];
            } else {
                BH[t] = rhs[(int64_t)fnb * 512 + cs_idx3(c)];
                if (nb_fas) NR[t] = src[(int64_t)fnb * 512 + cs_idx3(c)];
            }
            if (fq < 16) {
                // edge e4 of the neighbour's layer (-t1, +t1, -t2, +t2), cell idx
                int e4 = fq >> 2, idx = fq & 3;
                int cu = e4 == 0 ? 0 : e4 == 1 ? 7 : 2 * idx + ((flx + (e4 == 2 ? 1 : 0)) & 1);
                int cv = e4 == 2 ? 0 : e4 == 3 ? 7 : 2 * idx + ((flx + (e4 == 0 ? 1 : 0)) & 1);
                int ax = e4 < 2 ? ft1 : ft2, s1, s2;
                tangential(ax, s1, s2);
                c[ft1] = cu;
                c[ft2] = cv;
                const int32_t *xt = g.xt + (b * 6 + fd) * 8;
                EG[fd * 16 + fq] = ghost_at<T>(g, src, chat, fnb, 2 * ax + (e4 & 1), xt[2 * e4],
                                               xt[2 * e4 + 1], c[s1], c[s2]);
            }
        } else if (fnb == -2) {
            HB[t] = bc_value<T>(g, b, fd, fub, fv);
        } else {
            HB[t] = chat[(int64_t)pick6(ft.slot, fd) * 64 + fv * 8 + fub];
        }
    }
    P[256 + t] = ob;
    if (own_fas && fas == 1) PR[t] = orr;
    __syncthreads();
    int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
    int row = (k * 8 + j) * 4;
    if (own_fas && fas == 1) {  // black cell's right-hand side from the old field
        int i = 2 * m + ((j + k + 1) & 1);
        T xm = i > 0 ? PR[row + ((i - 1) >> 1)] : GB[0 * 32 + k * 4 + (j >> 1)];
        T xp = i < 7 ? PR[row + ((i + 1) >> 1)] : GB[1 * 32 + k * 4 + (j >> 1)];
        T ym = j > 0 ? PR[row - 4 + m] : GB[2 * 32 + k * 4 + m];
        T yp = j < 7 ? PR[row + 4 + m] : GB[3 * 32 + k * 4 + m];
        T zm = k > 0 ? PR[row - 32 + m] : GB[4 * 32 + j * 4 + m];
        T zp = k < 7 ? PR[row + 32 + m] : GB[5 * 32 + j * 4 + m];
        T s = xm + xp + ym + yp + zm + zp;
        bb = (s - (T)6 * ob) * inv_h2 + bb;
        fasbuf[b * 512 + 256 + t] = bb;
    }
    {  // red cell (i + j + k even)
        int i = 2 * m + ((j + k) & 1);
        const T *S = P + 256;
        T xm = i > 0 ? S[row + ((i - 1) >> 1)] : HR[0 * 32 + k * 4 + (j >> 1)];
        T xp = i < 7 ? S[row + ((i + 1) >> 1)] : HR[1 * 32 + k * 4 + (j >> 1)];
        T ym = j > 0 ? S[row - 4 + m] : HR[2 * 32 + k * 4 + m];
        T yp = j < 7 ? S[row + 4 + m] : HR[3 * 32 + k * 4 + m];
        T zm = k > 0 ? S[row - 32 + m] : HR[4 * 32 + j * 4 + m];
        T zp = k < 7 ? S[row + 32 + m] : HR[5 * 32 + j * 4 + m];
        T s = xm + xp + ym + yp + zm + zp;
        if (own_fas && fas == 1) {
            br = (s - (T)6 * orr) * inv_h2 + br;
            fasbuf[b * 512 + t] = br;
        }
        T nr = (s - h2 * br) * (T)kSixth;
        P[t] = nr;
        dst[b * 512 + t] = nr;
    }
    if (fnb >= 0) {  // recomputed red cell of the same-level neighbour
        const T *R = HR + fd * 32;
        const T *E = EG + fd * 16;
        int cx[3];
        cx[fa] = flx;
        cx[ft1] = fub;
        cx[ft2] = fv;
        T toward = P[cs_idx3(cx)];  // this box's black face cell (old)
        T away = D2[t];
        T nm = fside ? toward : away, np = fside ? away : toward;
        T um = fub == 0 ? E[0 + (fv >> 1)] : R[fv * 4 + ((fub - 1) >> 1)];
        T up = fub == 7 ? E[4 + (fv >> 1)] : R[fv * 4 + ((fub + 1) >> 1)];
        T vm = fv == 0 ? E[8 + (fub >> 1)] : R[(fv - 1) * 4 + (fub >> 1)];
        T vp = fv == 7 ? E[12 + (fub >> 1)] : R[(fv + 1) * 4 + (fub >> 1)];
        // axes: a = 0 -> (n, u, v); a = 1 -> (u, n, v); a = 2 -> (u, v, n)
        T xm = fa == 0 ? nm : um, xp = fa == 0 ? np : up;
        T ym = fa == 0 ? um : fa == 1 ? nm : vm, yp = fa == 0 ? up : fa == 1 ? np : vp;
        T zm = fa == 2 ? nm : vm, zp = fa == 2 ? np : vp;
        T s = xm + xp + ym + yp + zm + zp;
        T bh = BH[t];
        if (nb_fas && fas == 1) bh = (s - (T)6 * NR[t]) * inv_h2 + bh;
        HB[t] = (s - h2 * bh) * (T)kSixth;
    }
    __syncthreads();
    {  // black cell: neighbours are new red values; face ghosts as in the
       // black half-sweep (own = the old black value, inward = new red)
        int i = 2 * m + ((j + k + 1) & 1);
        auto face = [&](int d, T hv, T inward) -> T {
            int nb = pick6(ft.nb, d);
            if (nb >= 0) return hv;
            if (nb == -2) return g.bct[d] == 1 ? ob : dirichlet_ghost<T>(hv, ob);
            return cf_ghost<T>(hv, ob, inward);
        };
        T xm = i > 0 ? P[row + ((i - 1) >> 1)] : face(0, HB[0 * 32 + k * 4 + (j >> 1)], P[row]);
        T xp = i < 7 ? P[row + ((i + 1) >> 1)] : face(1, HB[1 * 32 + k * 4 + (j >> 1)], P[row + 3]);
        T ym = j > 0 ? P[row - 4 + m] : face(2, HB[2 * 32 + k * 4 + m], P[row + 4 + m]);
        T yp = j < 7 ? P[row + 4 + m] : face(3, HB[3 * 32 + k * 4 + m], P[row - 4 + m]);
        T zm = k > 0 ? P[row - 32 + m] : face(4, HB[4 * 32 + j * 4 + m], P[row + 32 + m]);
        T zp = k < 7 ? P[row + 32 + m] : face(5, HB[5 * 32 + j * 4 + m], P[row - 32 + m]);
        T s = xm + xp + ym + yp + zm + zp;
        dst[b * 512 + 256 + t] = (s - h2 * bb) * (T)kSixth;
    }
}

// Coarse value of cell D = C + dir * e_ax (level l-1, relative to box Q),
// with the coarse physical ghost outside the domain; N is Q's neighbour
// across the face D leaves Q through.
template <typename T>
__device__ __forceinline__ T coarse_at(const Geo &g, const T *__restrict__ phi, int64_t Q,
                                       const int C[3], int ax, int dir, int N) {
    int D[3] = {C[0], C[1], C[2]};
    D[ax] += dir;
    if (D[ax] >= 0 && D[ax] < 8) return phi[Q * 512 + cs_idx3(D)];
    int face = 2 * ax + (dir > 0 ? 1 : 0);
    if (N >= 0) {
        D[ax] = dir > 0 ? 0 : 7;
        return phi[(int64_t)N * 512 + cs_idx3(D)];
    }
    T in = phi[Q * 512 + cs_idx3(C)];
    if (N != -2 || g.bct[face] == 1) return in;  // -1 cannot occur under 26-neighbour nesting
    int f1, f2;
    tangential(ax, f1, f2);
    T gv = (T)(g.bcval ? g.bcval[(Q * 6 + face) * 64 + C[f2] * 8 + C[f1]] : g.bcv[face]);
    return (T)2 * gv - in;
}

// Tangential quadratic interpolation of the coarse level at the 64 ghosts of
// one refinement-boundary face: c_hat = 7/8 c + sum_t [(1/32 + s_t/8) c_{+t}
// + (1/32 - s_t/8) c_{-t}], s_t = +-1 the side of the ghost in the coarse
// cell.  One 64-lane wavefront per face (slot s).
template <typename T>
__device__ __forceinline__ void cf_face(const Geo &g, const T *__restrict__ phi, T *__restrict__ chat,
                                        const int32_t *__restrict__ slots, int64_t s, int lane) {
    int d = slots[2 * s + 1];
    const int32_t *x = g.slotx + 8 * s;  // Q, base t1, base t2, Q's neighbours
    int a = d >> 1, side = d & 1, t1, t2;
    tangential(a, t1, t2);
    int u = lane & 7, v = lane >> 3;
    int64_t Q = x[0];
    int C[3];
    C[a] = side ? 0 : 7;
    C[t1] = x[1] + (u >> 1);
    C[t2] = x[2] + (v >> 1);
    T acc = (T)0.875 * phi[Q * 512 + cs_idx3(C)];
#pragma unroll
    for (int q = 0; q < 2; q++) {
        int ax = q ? t2 : t1;
        T st = (((q ? v : u) & 1) ? (T)1 : (T)-1);
        T cp = coarse_at<T>(g, phi, Q, C, ax, 1, x[4 + 2 * q]);
        T cm = coarse_at<T>(g, phi, Q, C, ax, -1, x[3 + 2 * q]);
        acc += ((T)(1.0 / 32.0) + st / (T)8) * cp + ((T)(1.0 / 32.0) - st / (T)8) * cm;
    }
    chat[s * 64 + lane] = acc;
}

// Four refinement-boundary faces per 256-thread block: slots [s0, s0+ns).
template <typename T>
__global__ __launch_bounds__(256) void k_cf_coarse(Geo g, const T *__restrict__ phi,
                                                   T *__restrict__ chat,
                                                   const int32_t *__restrict__ slots, int64_t s0,
                                                   int64_t ns) {
    int64_t s = 4 * (int64_t)blockIdx.x + (threadIdx.x >> 6);
    if (s >= ns) return;
    cf_face<T>(g, phi, chat, slots, s0 + s, threadIdx.x & 63);
}

// Residual on level l and restriction to level l-1 (full approximation
// scheme): the residual of all 512 cells goes to LDS, then each of 64 threads
// owns one parent cell and writes phi_c = mean(phi), old_c = phi_c and
// rhs_c = mean(residual) (the coarse right-hand side is completed by
// k_fas_rhs).  Extra blocks copy phi -> old on the listed leaf boxes of level
// l-1 (those with a refined face or edge neighbour: the only leaf boxes whose
// old values a prolongation reads).
//
// ZERO: phi is zero on every level (the top-down pass of an FMG solve from
// phi = 0), so it is not read: the box is zero and its ghosts are those of
// the zero field (the boundary data and the refinement-boundary values
// c_hat of the zero field), which are the values the general path reads and
// forms.  The residual of a leaf box is then the residual of phi = 0, and
// the box also writes its volume-weighted sum of r^2 and max |r| at its leaf
// position leafpos[b] of `partial`, with the arithmetic and the summation
// order of k_leaf_norms (the norm the stopping test divides by).
template <typename T>
__device__ __forceinline__ T ghost_of_zero(const Geo &g, const T *__restrict__ chat, int64_t b, int d, int nb,
                                           int slot, int u, int v) {
    if (nb >= 0) return (T)0;
    if (nb == -2) return g.bct[d] == 1 ? (T)0 : dirichlet_ghost<T>(bc_value<T>(g, b, d, u, v), (T)0);
    return cf_ghost<T>(chat[(int64_t)slot * 64 + v * 8 + u], (T)0, (T)0);
}

template <typename T, bool ZERO>
__global__ __launch_bounds__(128) void k_resid_restrict(Geo g, T *__restrict__ phi, T *__restrict__ rhs,
                                                        T *__restrict__ old, const T *__restrict__ chat,
                                                        int64_t b0, int64_t nbx,
                                                        const int32_t *__restrict__ leaf_prev,
                                                        int64_t nleaf_prev, T inv_h2,
                                                        const int32_t *__restrict__ leafpos,
                                                        double *__restrict__ partial, double vol) {
    // 128 threads per box: thread u holds cell positions 2u and 2u+1 of both
    // colours (paired loads); the ZERO norm partials follow k_box_norms' tree
    using V = typename VecN<T, 2>::type;
    __shared__ T P[512], H[384], R[512];
    __shared__ double S[4], M[4];
    int64_t blk = blockIdx.x;
    const int u = threadIdx.x;
    int64_t nmain = xcd_grid(nbx);
    if (blk >= nmain) {
        int64_t q = blk - nmain;
        if (q >= nleaf_prev) return;
        int64_t p = leaf_prev[q];
        V *dst = reinterpret_cast<V *>(old + p * 512);
        const V *src = reinterpret_cast<const V *>(phi + p * 512);
        V z;
        z.x = (T)0;
        z.y = (T)0;
        dst[u] = ZERO ? z : src[u];
        dst[128 + u] = ZERO ? z : src[128 + u];
        return;
    }
    int64_t lb = xcd_map(blk, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    // indices of the parent cells, loaded with the data (not after the barriers)
    const int64_t p = g.parent[b];
    const int bi = g.ijk[b * 4] & 1, bj = g.ijk[b * 4 + 1] & 1, bk = g.ijk[b * 4 + 2] & 1;
    const V r0 = ld_stream(reinterpret_cast<const V *>(rhs + b * 512) + u);
    const V r1 = ld_stream(reinterpret_cast<const V *>(rhs + b * 512 + 256) + u);
    const FaceTab ft = face_tab(g, b);
    if (ZERO) {
        V z;
        z.x = (T)0;
        z.y = (T)0;
        reinterpret_cast<V *>(P)[u] = z;
        reinterpret_cast<V *>(P)[128 + u] = z;
#pragma unroll
        for (int r = 0; r < 3; r++) {
            int e = u + 128 * r, d = e >> 6, w = e & 63;
            H[e] = ghost_of_zero<T>(g, chat, b, d, pick6(ft.nb, d), pick6(ft.slot, d), w & 7, w >> 3);
        }
    } else {
        const V p0 = reinterpret_cast<const V *>(phi + b * 512)[u];
        const V p1 = reinterpret_cast<const V *>(phi + b * 512 + 256)[u];
#pragma unroll
        for (int r = 0; r < 3; r++) {
            int e = u + 128 * r, d = e >> 6, w = e & 63;
            H[e] = ghost_at<T>(g, phi, chat, b, d, pick6(ft.nb, d), pick6(ft.slot, d), w & 7, w >> 3);
        }
        reinterpret_cast<V *>(P)[u] = p0;
        reinterpret_cast<V *>(P)[128 + u] = p1;
    }
    __syncthreads();
    double ss[2] = {0.0, 0.0}, mx[2] = {0.0, 0.0};
#pragma unroll
    for (int sl = 0; sl < 2; sl++) {
        const int t = 2 * u + sl;
        const int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
#pragma unroll
        for (int c = 0; c < 2; c++) {
            int i = 2 * m + ((j + k + c) & 1);
            T rc = c ? (sl ? r1.y : r1.x) : (sl ? r0.y : r0.x);
            T r = resid_of<T>(rc, sum_full<T>(P, H, i, j, k), P[c * 256 + t], inv_h2);
            R[c * 256 + t] = r;
            if (ZERO) {
                ss[sl] = fmadd((double)r, (double)r, ss[sl]);
                mx[sl] = nanmax(fabs((double)r), mx[sl]);
            }
        }
    }
    if (ZERO && leafpos[b] >= 0) {  // block-uniform
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
#pragma unroll
            for (int sl = 0; sl < 2; sl++) {
                ss[sl] += __shfl_xor(ss[sl], off);
                mx[sl] = nanmax(__shfl_xor(mx[sl], off), mx[sl]);
            }
        }
        if ((u & 31) == 0) {
            S[u >> 5] = ss[0] + ss[1];
            M[u >> 5] = nanmax(mx[1], mx[0]);
        }
    }
    __syncthreads();
    if (ZERO && u == 0 && leafpos[b] >= 0) {
        int64_t q = leafpos[b];
        partial[2 * q] = ((S[0] + S[1]) + (S[2] + S[3])) * vol;
        partial[2 * q + 1] = nanmax(nanmax(M[0], M[1]), nanmax(M[2], M[3]));
    }
    if (u < 64) {
        int pi = u & 3, pj = (u >> 2) & 3, pk = u >> 4;
        T sphi = 0, sres = 0;
#pragma unroll
        for (int dk = 0; dk < 2; dk++)
#pragma unroll
            for (int dj = 0; dj < 2; dj++)
#pragma unroll
                for (int di = 0; di < 2; di++) {
                    int c = cs_idx(2 * pi + di, 2 * pj + dj, 2 * pk + dk);
                    sphi += P[c];
                    sres += R[c];
                }
        int ci = 4 * bi + pi, cj = 4 * bj + pj, ck = 4 * bk + pk;
        int64_t pc = p * 512 + cs_idx(ci, cj, ck);
        T mphi = (T)0.125 * sphi;
        phi[pc] = mphi;
        old[pc] = mphi;
        rhs[pc] = (T)0.125 * sres;
    }
}

// rhs <- L phi + rhs on the listed (refined) boxes: completes the coarse
// right-hand side L_c(R phi) + R r of the full approximation scheme.
template <typename T>
__global__ __launch_bounds__(128) void k_fas_rhs(Geo g, const T *__restrict__ phi, T *__restrict__ rhs,
                                                 const T *__restrict__ chat,
                                                 const int32_t *__restrict__ list, int64_t nlist,
                                                 T inv_h2) {
    // 128 threads per box: thread u holds cell positions 2u and 2u+1 of both
    // colours (paired loads and stores)
    using V = typename VecN<T, 2>::type;
    __shared__ T P[512], H[384];
    int64_t q = xcd_map(blockIdx.x, nlist);
    if (q >= nlist) return;
    int64_t b = list[q];
    const int u = threadIdx.x;
    const V r0 = ld_stream(reinterpret_cast<const V *>(rhs + b * 512) + u);
    const V r1 = ld_stream(reinterpret_cast<const V *>(rhs + b * 512 + 256) + u);
    const V p0 = reinterpret_cast<const V *>(phi + b * 512)[u];
    const V p1 = reinterpret_cast<const V *>(phi + b * 512 + 256)[u];
    const FaceTab ft = face_tab(g, b);
#pragma unroll
    for (int r = 0; r < 3; r++) {
        int e = u + 128 * r, d = e >> 6, w = e & 63;
        H[e] = ghost_at<T>(g, phi, chat, b, d, pick6(ft.nb, d), pick6(ft.slot, d), w & 7, w >> 3);
    }
    reinterpret_cast<V *>(P)[u] = p0;
    reinterpret_cast<V *>(P)[128 + u] = p1;
    __syncthreads();
    const T *rr0 = reinterpret_cast<const T *>(&r0), *rr1 = reinterpret_cast<const T *>(&r1);
#pragma unroll
    for (int c = 0; c < 2; c++) {
        V out;
        T *o = reinterpret_cast<T *>(&out);
#pragma unroll
        for (int sl = 0; sl < 2; sl++) {
            const int t = 2 * u + sl;
            const int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
            int i = 2 * m + ((j + k + c) & 1);
            T own = P[c * 256 + t];
            T s = sum_full<T>(P, H, i, j, k);
            o[sl] = (s - (T)6 * own) * inv_h2 + (c ? rr1[sl] : rr0[sl]);
        }
        reinterpret_cast<V *>(rhs + b * 512 + c * 256)[u] = out;
    }
}

// phi_f += 1/4 delta(C) + 1/4 (delta(C + s_x) + delta(C + s_y) + delta(C + s_z))
// with delta = phi - old on the parent level, C the parent cell and s the
// side of the fine cell inside it.  The parent's delta over the child's
// octant and its face-adjacent layer is staged in D[6][6][6] (outside the
// parent: the same-level neighbour or the homogeneous physical ghost).  Extra
// blocks compute c_hat for the refinement-boundary faces of level l (which
// read only level l-1, like the prolongation).
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_cf(Geo g, T *__restrict__ phi, const T *__restrict__ old,
                                                    int64_t b0, int64_t nbx, T *__restrict__ chat,
                                                    const int32_t *__restrict__ slots, int64_t s0,
                                                    int64_t ns) {
    __shared__ T D[216];
    int64_t blk = blockIdx.x;
    int t = threadIdx.x;
    int64_t nmain = xcd_grid(nbx);
    if (blk >= nmain) {
        int64_t s = 4 * (blk - nmain) + (t >> 6);
        if (s < ns) cf_face<T>(g, phi, chat, slots, s0 + s, t & 63);
        return;
    }
    int64_t lb = xcd_map(blk, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    int64_t p = g.parent[b];
    int o[3] = {g.ijk[b * 4] & 1, g.ijk[b * 4 + 1] & 1, g.ijk[b * 4 + 2] & 1};
    // this box's values, loaded with the correction (not after the barrier)
    T f0 = phi[b * 512 + t], f1 = phi[b * 512 + 256 + t];
    if (t < 216) {
        int c[3] = {t % 6 - 1, (t / 6) % 6 - 1, t / 36 - 1}, out = 0, oax = 0;
        for (int a = 0; a < 3; a++)
            if (c[a] < 0 || c[a] > 3) { out++; oax = a; }
        if (out <= 1) {
            int C[3] = {4 * o[0] + c[0], 4 * o[1] + c[1], 4 * o[2] + c[2]};
            T del;
            if (C[oax] >= 0 && C[oax] < 8) {
                int64_t q = p * 512 + cs_idx3(C);
                del = phi[q] - old[q];
            } else {
                int face = 2 * oax + (C[oax] > 7 ? 1 : 0);
                int N = g.nbr[p * 6 + face];  // the parent's face neighbour
                if (N >= 0) {
                    C[oax] = C[oax] > 7 ? 0 : 7;
                    int64_t q = (int64_t)N * 512 + cs_idx3(C);
                    del = phi[q] - old[q];
                } else {  // domain face (a refined box has no refinement-boundary face)
                    C[oax] = C[oax] > 7 ? 7 : 0;
                    int64_t q = p * 512 + cs_idx3(C);
                    T din = phi[q] - old[q];
                    del = g.bct[face] == 1 ? din : -din;
                }
            }
            D[t] = del;
        }
    }
    __syncthreads();
    int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        int i = 2 * m + ((j + k + c) & 1);
        int x = (i >> 1) + 1, y = (j >> 1) + 1, z = (k >> 1) + 1;
        int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
        int at = (z * 6 + y) * 6 + x;
        T d0 = D[at], dx = D[at + sx], dy = D[at + 6 * sy], dz = D[at + 36 * sz];
        int64_t idx = b * 512 + c * 256 + t;
        phi[idx] = (c ? f1 : f0) + ((T)0.25 * d0 + (T)0.25 * (dx + dy + dz));
    }
}

// ------------------------------------- prolongation fused into the up-sweep
// The first red-black sweep after the prolongation of a level reads the
// prolonged field only where the red and the black half-sweeps read it: the
// red half reads every black cell (its own, and the neighbours' face layers
// as ghosts) and, for the boundary ghosts of its face cells, the red face
// cells on domain and refinement-boundary faces; the black half reads the
// new red cells and, for the same boundary ghosts, its own black face cells
// on those faces.  Every other prolonged value is overwritten unread.  So the
// two half-sweeps below take the prolonged value f + p(delta) of each cell
// they read on the fly, from the unprolonged field and the parent's
// correction delta = phi - old, and nothing writes the prolongation itself:
// the level ends the sweep with the values of the prolongation followed by
// the two half-sweeps (same arithmetic in the same order, so the same bits).
//
// The correction is staged once per refined box P of level l-1 (k_delta_pad)
// as a padded block of 10^3 values, x fastest: delta over P's cells and one
// cell layer around them.  The layer comes from P's same-level face and edge
// neighbours (corners are never read: a fine cell's stencil steps at most
// one coarse cell along each of two axes from P's face layers), or outside
// the domain from P's own cell mirrored, with the sign of the homogeneous
// boundary condition (Dirichlet -, Neumann +), as k_prolong_cf takes it.  The
// children of the k-th refined box of level l-1 are the boxes 8k .. 8k+7 of
// level l (canonical order), octant = position & 7, and read the 6^3
// sub-block 4 o + 0..5 of block k.
template <typename T>
__global__ __launch_bounds__(256) void k_delta_pad(Geo g, const T *__restrict__ phi, const T *__restrict__ old,
                                                   const int32_t *__restrict__ refined, int64_t nref,
                                                   T *__restrict__ pad, T *__restrict__ chat,
                                                   const int32_t *__restrict__ slots, int64_t s0, int64_t ns) {
    __shared__ int32_t NP[27];
    int64_t blk = blockIdx.x;
    int t = threadIdx.x;
    int64_t nmain = xcd_grid(nref);
    if (blk >= nmain) {  // c_hat of the refinement-boundary faces of level l (reads level l-1 only)
        int64_t sl = 4 * (blk - nmain) + (t >> 6);
        if (sl < ns) cf_face<T>(g, phi, chat, slots, s0 + sl, t & 63);
        return;
    }
    int64_t k = xcd_map(blk, nref);
    if (k >= nref) return;
    int64_t P = refined[k];
    if (t < 27) NP[t] = g.n27[P * 27 + t];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; r++) {
        int e = t + 256 * r;
        if (e >= 1000) break;
        int c[3] = {e % 10 - 1, (e / 10) % 10 - 1, e / 100 - 1};
        int sd[3], nout = 0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            sd[a] = c[a] < 0 ? -1 : c[a] > 7 ? 1 : 0;
            nout += sd[a] != 0;
        }
        T v = (T)0;
        if (nout < 3) {
            bool neg = false;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                if (sd[a] == 0) continue;
                int fo = 13 + (a == 0 ? sd[a] : a == 1 ? 3 * sd[a] : 9 * sd[a]);
                if (NP[fo] == -2) {  // P's face on this side is a domain face: mirror
                    int face = 2 * a + (sd[a] > 0 ? 1 : 0);
                    c[a] = sd[a] < 0 ? 0 : 7;
                    sd[a] = 0;
                    if (g.bct[face] != 1) neg = !neg;
                }
            }
            int32_t q = NP[(sd[0] + 1) + 3 * (sd[1] + 1) + 9 * (sd[2] + 1)];
            if (q >= 0) {  // always, for every value a prolongation reads (proper nesting)
                int cc[3] = {c[0] & 7, c[1] & 7, c[2] & 7};
                int64_t at = (int64_t)q * 512 + cs_idx3(cc);
                T d = phi[at] - old[at];
                v = neg ? -d : d;
            }
        }
        pad[k * 1000 + e] = v;
    }
}
// Offset of the 6^3 correction region of the box at position lb of its level
// (octant lb & 7) in its parent's padded block, and of region cell e
// (x fastest) from there.
__device__ __forceinline__ int pad_corner(int64_t lb) {
    int o = (int)(lb & 7);
    return 4 * ((o & 1) + 10 * ((o >> 1) & 1) + 100 * (o >> 2));
}
__device__ __forceinline__ int pad_off(int e) { return e % 6 + 10 * ((e / 6) % 6) + 100 * (e / 36); }
// Prolonged correction at fine cell (i, j, k) of the box, i, j, k in -1..8
// (at most one outside 0..7: a face ghost), as k_prolong_cf adds it.
template <typename T>
__device__ __forceinline__ T prolonged(const T *D, int i, int j, int k) {
    int x = (i + 2) >> 1, y = (j + 2) >> 1, z = (k + 2) >> 1;
    int sx = ((i + 2) & 1) ? 1 : -1, sy = ((j + 2) & 1) ? 6 : -6, sz = ((k + 2) & 1) ? 36 : -36;
    int at = (z * 6 + y) * 6 + x;
    T d0 = D[at], dx = D[at + sx], dy = D[at + sy], dz = D[at + sz];
    return (T)0.25 * d0 + (T)0.25 * (dx + dy + dz);
}
// The face cell of face d at tangential (u, v) and layer `layer` (0..7, or
// -1 / 8 outside the box), as (i, j, k)
__device__ __forceinline__ void face_cell(int d, int layer, int u, int v, int &i, int &j, int &k) {
    int a = d >> 1, t1, t2;
    tangential(a, t1, t2);
    int c[3];
    c[a] = layer;
    c[t1] = u;
    c[t2] = v;
    i = c[0];
    j = c[1];
    k = c[2];
}

// Red half of the first sweep after the prolongation into boxes [b0,
// b0+nbx) of level l >= 2 (128 threads, 2 cells each, XCD-aware mapping).
// LDS: S the prolonged black cells, H the ghosts of the red face cells, D
// the correction region.  Same-level ghost: the neighbour's black cell +
// its prolonged correction; domain and refinement-boundary ghosts from the
// prolonged red face cell (and, at a refinement boundary, the prolonged
// black cell behind it).  Writes the red cells only.
template <typename T>
__global__ __launch_bounds__(128) void k_gsrb_pro_red(Geo g, T *__restrict__ phi, const T *__restrict__ rhs,
                                                      const T *__restrict__ pad, const T *__restrict__ chat,
                                                      int64_t b0, int64_t nbx, T h2) {
    using V = typename VecN<T, 2>::type;
    __shared__ T S[256], H[192], D[216];
    int64_t lb = xcd_map(blockIdx.x, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    const int t = threadIdx.x;
    const FaceTab ft = face_tab(g, b);
    V blk = reinterpret_cast<const V *>(phi + b * 512 + 256)[t];
    V bv = ld_stream(reinterpret_cast<const V *>(rhs + b * 512) + t);
    const T *pk = pad + (lb >> 3) * 1000 + pad_corner(lb);
    T dv0 = pk[pad_off(t)];
    T dv1 = t + 128 < 216 ? pk[pad_off(t + 128)] : (T)0;
    // ghost entries e = t, t + 128 (< 192): face d, red face cell (u, v) at layer L
    T raw[2], in_raw[2], ch[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        int e = t + 128 * r;
        raw[r] = in_raw[r] = ch[r] = (T)0;
        if (e >= 192) continue;
        int d = e >> 5, q = e & 31, v = q >> 2, L = (d & 1) ? 7 : 0;
        int u = 2 * (q & 3) + ((L + v) & 1);
        int nb = pick6(ft.nb, d), i, j, k;
        if (nb >= 0) {
            face_cell(d, (d & 1) ? 0 : 7, u, v, i, j, k);  // mirrored cell in the neighbour
            raw[r] = phi[(int64_t)nb * 512 + cs_idx(i, j, k)];
        } else {
            face_cell(d, L, u, v, i, j, k);
            raw[r] = phi[b * 512 + cs_idx(i, j, k)];
            if (nb == -1) {
                face_cell(d, (d & 1) ? 6 : 1, u, v, i, j, k);
                in_raw[r] = phi[b * 512 + cs_idx(i, j, k)];
                ch[r] = chat[(int64_t)pick6(ft.slot, d) * 64 + v * 8 + u];
            }
        }
    }
    D[t] = dv0;
    if (t + 128 < 216) D[t + 128] = dv1;
    __syncthreads();
    {
        const T *bl = reinterpret_cast<const T *>(&blk);
        V sv;
        T *so = reinterpret_cast<T *>(&sv);
#pragma unroll
        for (int w = 0; w < 2; w++) {
            int cq = 2 * t + w;
            int m = cq & 3, j = (cq >> 2) & 7, k = cq >> 5;
            int i = 2 * m + ((j + k + 1) & 1);
            so[w] = bl[w] + prolonged<T>(D, i, j, k);
        }
        reinterpret_cast<V *>(S)[t] = sv;
    }
#pragma unroll
    for (int r = 0; r < 2; r++) {
        int e = t + 128 * r;
        if (e >= 192) continue;
        int d = e >> 5, q = e & 31, v = q >> 2, L = (d & 1) ? 7 : 0;
        int u = 2 * (q & 3) + ((L + v) & 1);
        int nb = pick6(ft.nb, d), i, j, k;
        T gv;
        if (nb >= 0) {
            face_cell(d, (d & 1) ? 8 : -1, u, v, i, j, k);
            gv = raw[r] + prolonged<T>(D, i, j, k);
        } else {
            face_cell(d, L, u, v, i, j, k);
            T own = raw[r] + prolonged<T>(D, i, j, k);
            if (nb == -2) {
                gv = g.bct[d] == 1 ? own : dirichlet_ghost<T>(bc_value<T>(g, b, d, u, v), own);
            } else {
                face_cell(d, (d & 1) ? 6 : 1, u, v, i, j, k);
                gv = cf_ghost<T>(ch[r], own, in_raw[r] + prolonged<T>(D, i, j, k));
            }
        }
        H[e] = gv;
    }
    __syncthreads();
    const T *bb = reinterpret_cast<const T *>(&bv);
    V res;
    T *out = reinterpret_cast<T *>(&res);
#pragma unroll
    for (int w = 0; w < 2; w++) {
        int cq = 2 * t + w;
        int m = cq & 3, j = (cq >> 2) & 7, k = cq >> 5;
        int i = 2 * m + ((j + k) & 1);
        int row = (k * 8 + j) * 4;
        T xm = i > 0 ? S[row + ((i - 1) >> 1)] : H[0 * 32 + k * 4 + (j >> 1)];
        T xp = i < 7 ? S[row + ((i + 1) >> 1)] : H[1 * 32 + k * 4 + (j >> 1)];
        T ym = j > 0 ? S[row - 4 + m] : H[2 * 32 + k * 4 + m];
        T yp = j < 7 ? S[row + 4 + m] : H[3 * 32 + k * 4 + m];
        T zm = k > 0 ? S[row - 32 + m] : H[4 * 32 + j * 4 + m];
        T zp = k < 7 ? S[row + 32 + m] : H[5 * 32 + j * 4 + m];
        T sm = xm + xp + ym + yp + zm + zp;
        out[w] = (sm - h2 * bb[w]) * (T)kSixth;
    }
    reinterpret_cast<V *>(phi + b * 512)[t] = res;
}

// Black half of the first sweep after the prolongation: as k_gsrb<1, T, 2>,
// except that the ghosts of black face cells on domain and
// refinement-boundary faces take the prolonged black face cell (its
// unprolonged value + the correction, from the correction region, staged
// only by boxes with such faces).
template <typename T>
__global__ __launch_bounds__(128) void k_gsrb_pro_black(Geo g, T *__restrict__ phi, const T *__restrict__ rhs,
                                                        const T *__restrict__ pad, const T *__restrict__ chat,
                                                        int64_t b0, int64_t nbx, T h2) {
    using V = typename VecN<T, 2>::type;
    __shared__ T S[256], H[192], D[216];
    int64_t lb = xcd_map(blockIdx.x, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    const int t = threadIdx.x;
    const FaceTab ft = face_tab(g, b);
    bool bnd = false;
#pragma unroll
    for (int d = 0; d < 6; d++) bnd = bnd || ft.nb[d] < 0;
    V o = reinterpret_cast<const V *>(phi + b * 512)[t];
    V bv = ld_stream(reinterpret_cast<const V *>(rhs + b * 512 + 256) + t);
    T raw[2], in_new[2], ch[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        int e = t + 128 * r;
        raw[r] = in_new[r] = ch[r] = (T)0;
        if (e >= 192) continue;
        int d = e >> 5, q = e & 31, v = q >> 2, L = (d & 1) ? 7 : 0;
        int u = 2 * (q & 3) + ((L + v + 1) & 1);
        int nb = pick6(ft.nb, d), i, j, k;
        if (nb >= 0) {
            face_cell(d, (d & 1) ? 0 : 7, u, v, i, j, k);
            raw[r] = phi[(int64_t)nb * 512 + cs_idx(i, j, k)];  // the neighbour's new red cell
        } else {
            face_cell(d, L, u, v, i, j, k);
            raw[r] = phi[b * 512 + cs_idx(i, j, k)];  // own black face cell, unprolonged
            if (nb == -1) {
                face_cell(d, (d & 1) ? 6 : 1, u, v, i, j, k);
                in_new[r] = phi[b * 512 + cs_idx(i, j, k)];  // new red cell behind it
                ch[r] = chat[(int64_t)pick6(ft.slot, d) * 64 + v * 8 + u];
            }
        }
    }
    if (bnd) {
        const T *pk = pad + (lb >> 3) * 1000 + pad_corner(lb);
        T dv0 = pk[pad_off(t)];
        T dv1 = t + 128 < 216 ? pk[pad_off(t + 128)] : (T)0;
        D[t] = dv0;
        if (t + 128 < 216) D[t + 128] = dv1;
    }
    reinterpret_cast<V *>(S)[t] = o;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; r++) {
        int e = t + 128 * r;
        if (e >= 192) continue;
        int d = e >> 5, q = e & 31, v = q >> 2, L = (d & 1) ? 7 : 0;
        int u = 2 * (q & 3) + ((L + v + 1) & 1);
        int nb = pick6(ft.nb, d), i, j, k;
        T gv = raw[r];
        if (nb < 0) {
            face_cell(d, L, u, v, i, j, k);
            T own = raw[r] + prolonged<T>(D, i, j, k);
            if (nb == -2)
                gv = g.bct[d] == 1 ? own : dirichlet_ghost<T>(bc_value<T>(g, b, d, u, v), own);
            else
                gv = cf_ghost<T>(ch[r], own, in_new[r]);
        }
        H[e] = gv;
    }
    __syncthreads();
    const T *bb = reinterpret_cast<const T *>(&bv);
    V res;
    T *out = reinterpret_cast<T *>(&res);
#pragma unroll
    for (int w = 0; w < 2; w++) {
        int cq = 2 * t + w;
        int m = cq & 3, j = (cq >> 2) & 7, k = cq >> 5;
        int i = 2 * m + ((j + k + 1) & 1);
        int row = (k * 8 + j) * 4;
        T xm = i > 0 ? S[row + ((i - 1) >> 1)] : H[0 * 32 + k * 4 + (j >> 1)];
        T xp = i < 7 ? S[row + ((i + 1) >> 1)] : H[1 * 32 + k * 4 + (j >> 1)];
        T ym = j > 0 ? S[row - 4 + m] : H[2 * 32 + k * 4 + m];
        T yp = j < 7 ? S[row + 4 + m] : H[3 * 32 + k * 4 + m];
        T zm = k > 0 ? S[row - 32 + m] : H[4 * 32 + j * 4 + m];
        T zp = k < 7 ? S[row + 32 + m] : H[5 * 32 + j * 4 + m];
        T sm = xm + xp + ym + yp + zm + zp;
        out[w] = (sm - h2 * bb[w]) * (T)kSixth;
    }
    reinterpret_cast<V *>(phi + b * 512 + 256)[t] = res;
}

// Exact solve on each root box by fast diagonalisation: with the 1-D
// eigenbases V_a, phi = (V_z x V_y x V_x) diag(h^2 / (l_x + l_y + l_z))
// (V_z x V_y x V_x)^T rhs, where rhs has the Dirichlet data folded in.
template <typename T>
__global__ __launch_bounds__(512) void k_coarse(Geo g, T *__restrict__ phi, const T *__restrict__ rhs,
                                                const double *__restrict__ eig, int64_t b0, double h) {
    __shared__ double X[512], Y[512], V[192], L[24];
    int64_t b = b0 + blockIdx.x;
    int t = threadIdx.x, i = t & 7, j = (t >> 3) & 7, k = t >> 6;
    if (t < 192) V[t] = eig[t];
    if (t < 24) L[t] = eig[192 + t];
    int c[3] = {i, j, k};
    double r = (double)rhs[b * 512 + cs_idx(i, j, k)];
#pragma unroll
    for (int d = 0; d < 6; d++) {
        int a = d >> 1, s = d & 1;
        bool edge = s ? (c[a] == 7) : (c[a] == 0);
        if (edge && g.bct[d] == 0) {
            int t1, t2;
            tangential(a, t1, t2);
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
    phi[b * 512 + cs_idx(i, j, k)] = (T)X[t];
}

// ------------------------------------------------- bottom of the V-cycle
// The two coarsest levels of every tree in one launch, one workgroup of 1024
// threads per tree: Gauss-Seidel on the tree's eight level-2 boxes,
// residual and restriction to the root, the root's FAS right-hand side, its
// exact solve, prolongation of the correction and the up-sweeps.  Level 2 of
// a tree is empty or all 8 children of the root (Morton = octant order from
// root2[tree]), i.e. one uniform 16^3 grid whose only ghosts are domain
// ghosts; it is held in LDS (colour-split, rows x fastest) with its
// right-hand side, the doubled Dirichlet values of its six faces and the
// root's fields (natural order), so the ~20 dependent steps cost a
// workgroup barrier each instead of a launch each.  The arithmetic of every
// cell, and the order of every sum, are those of k_gsrb, k_resid_restrict,
// k_fas_rhs, k_coarse and k_prolong_cf.  fmg != 0 first runs the FMG pass's
// own bottom (restriction, root solve, prolongation, without smoothing).

template <typename T>
__device__ __forceinline__ T root_ghost(const Geo &g, int64_t r, int d, int u, int v, T own) {
    if (g.bct[d] == 1) return own;
    return dirichlet_ghost<T>(bc_value<T>(g, r, d, u, v), own);
}
// The 16^3 grid in LDS is colour-split like a box: colour (I+J+K)&1, then
// row K*16 + J, then I/2, so a wave of a half-sweep reads consecutive words.
__device__ __forceinline__ int cs16(int I, int J, int K) {
    return (((I + J + K) & 1) << 11) + ((K * 16 + J) << 3) + (I >> 1);
}
// (I, J, K) of colour-split index p of the 16^3 grid
__device__ __forceinline__ void cs16_cell(int p, int &I, int &J, int &K) {
    J = (p >> 3) & 15;
    K = (p >> 7) & 15;
    I = 2 * (p & 7) + ((J + K + (p >> 11)) & 1);
}
// six-neighbour sum of fine cell (I, J, K), order -x, +x, -y, +y, -z, +z.
// Domain ghosts: own (Neumann) or GB - own with GB = 2 g (Dirichlet), GB
// indexed by the face cell (v * 16 + u, u and v along the tangential axes in
// increasing order).
template <typename T>
__device__ __forceinline__ T bot_sum(const T *F2, const T *GB, const int nm[6], int I, int J, int K,
                                     T own) {
    const T *S = F2 + ((((I + J + K) & 1) ^ 1) << 11);  // the other colour
    int row = (K * 16 + J) << 3;
    T xm = I > 0 ? S[row + ((I - 1) >> 1)] : nm[0] ? own : GB[0 * 256 + K * 16 + J] - own;
    T xp = I < 15 ? S[row + ((I + 1) >> 1)] : nm[1] ? own : GB[1 * 256 + K * 16 + J] - own;
    T ym = J > 0 ? S[row - 8 + (I >> 1)] : nm[2] ? own : GB[2 * 256 + K * 16 + I] - own;
    T yp = J < 15 ? S[row + 8 + (I >> 1)] : nm[3] ? own : GB[3 * 256 + K * 16 + I] - own;
    T zm = K > 0 ? S[row - 128 + (I >> 1)] : nm[4] ? own : GB[4 * 256 + J * 16 + I] - own;
    T zp = K < 15 ? S[row + 128 + (I >> 1)] : nm[5] ? own : GB[5 * 256 + J * 16 + I] - own;
    return xm + xp + ym + yp + zm + zp;
}
// colour-split index c of a box -> (i, j, k)
__device__ __forceinline__ void cs_cell(int c, int &i, int &j, int &k) {
    int q = c & 255;
    j = (q >> 2) & 7;
    k = q >> 5;
    i = 2 * (q & 3) + ((j + k + (c >> 8)) & 1);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_bottom(Geo g, T *__restrict__ phi, T *__restrict__ rhs,
                                                 T *__restrict__ old, const double *__restrict__ eig,
                                                 int64_t r0, const int32_t *__restrict__ root2,
                                                 T h2_2, T inv_h2_2, T inv_h2_1, double h1, int nd,
                                                 int nu, int fmg, int fas2,
                                                 const int32_t *__restrict__ isleaf) {
    // F2, B2: level-2 field and right-hand side; GB: 2 g on the six faces of
    // the 16^3 grid; F1, B1, O1: the root's phi, rhs, old; W: the level-2
    // residual, then the root solve's X and Y, then the root correction
    // padded by its domain ghosts (10^3).
    __shared__ T F2[4096], B2[4096], GB[6 * 256], F1[512], B1[512], O1[512];
    __shared__ double W[4096], V[192], L[24];
    T *R2 = reinterpret_cast<T *>(W);
    double *X = W, *Y = W + 512;
    T *D1 = reinterpret_cast<T *>(W + 1024);
    const int tid = threadIdx.x;
    const int64_t r = r0 + blockIdx.x;
    const int64_t first2 = root2[blockIdx.x];
    const bool has2 = first2 >= 0;
    int nm[6];
#pragma unroll
    for (int d = 0; d < 6; d++) nm[d] = g.bct[d] == 1;
    // root cell of this thread (tid < 512), natural order
    const int ri = tid & 7, rj = (tid >> 3) & 7, rk = (tid >> 6) & 7;
    if (tid < 192) V[tid] = eig[tid];
    if (tid < 24) L[tid] = eig[192 + tid];
    if (tid < 512) {
        int i, j, k;
        cs_cell(tid, i, j, k);
        F1[i + 8 * j + 64 * k] = phi[r * 512 + tid];
        B1[i + 8 * j + 64 * k] = rhs[r * 512 + tid];
    }
    if (has2) {
#pragma unroll
        for (int w = 0; w < 4; w++) {
            int e = tid + 1024 * w, o = e >> 9, i, j, k;
            cs_cell(e & 511, i, j, k);
            int p = cs16(8 * (o & 1) + i, 8 * ((o >> 1) & 1) + j, 8 * (o >> 2) + k);
            F2[p] = phi[first2 * 512 + e];
            B2[p] = rhs[first2 * 512 + e];
        }
        for (int e = tid; e < 6 * 256; e += 1024) {
            int d = e >> 8, u = e & 15, v = (e >> 4) & 15, a = d >> 1, side = d & 1;
            int c[3];  // the face cell's box: octant side along a, u and v across it
            c[a] = side;
            c[a == 0 ? 1 : 0] = u >> 3;
            c[a == 2 ? 1 : 2] = v >> 3;
            int o = c[0] | (c[1] << 1) | (c[2] << 2);
            GB[e] = (T)2 * bc_value<T>(g, first2 + o, d, u & 7, v & 7);
        }
    }
    __syncthreads();
    // FAS right-hand side of the level-2 boxes with children, L phi + rhs
    // (the level-3 restriction has just written both), as k_fas_rhs forms
    // it: same neighbour order, same domain ghosts; stored for the rest of
    // the cycle
    if (fas2 && has2) {
#pragma unroll
        for (int w = 0; w < 4; w++) {
            int e = tid + 1024 * w, o = e >> 9, i, j, k;
            if (isleaf[first2 + o]) continue;
            cs_cell(e & 511, i, j, k);
            int I = 8 * (o & 1) + i, J = 8 * ((o >> 1) & 1) + j, K = 8 * (o >> 2) + k;
            int p = cs16(I, J, K);
            T own = F2[p];
            T s = bot_sum<T>(F2, GB, nm, I, J, K, own);
            T bn = (s - (T)6 * own) * inv_h2_2 + B2[p];
            B2[p] = bn;
            rhs[first2 * 512 + e] = bn;
        }
        __syncthreads();
    }

    auto half_sweep = [&](int C) __attribute__((always_inline)) {
#pragma unroll
        for (int w = 0; w < 2; w++) {
            int p = (C << 11) + tid + 1024 * w, I, J, K;
            cs16_cell(p, I, J, K);
            T s = bot_sum<T>(F2, GB, nm, I, J, K, F2[p]);
            F2[p] = (s - h2_2 * B2[p]) * (T)kSixth;
        }
        __syncthreads();
    };
    auto smooth = [&](int n) __attribute__((always_inline)) {
        for (int it = 0; it < n; it++) {
            half_sweep(0);
            half_sweep(1);
        }
    };
    // residual of level 2, restriction to the root, FAS right-hand side of
    // the root; a leaf root only copies phi -> old
    auto down = [&]() __attribute__((always_inline)) {
        if (!has2) {
            if (tid < 512) O1[tid] = F1[tid];
            __syncthreads();
            return;
        }
#pragma unroll
        for (int w = 0; w < 4; w++) {
            int p = tid + 1024 * w, I, J, K;
            cs16_cell(p, I, J, K);
            T own = F2[p];
            T sum = bot_sum<T>(F2, GB, nm, I, J, K, own);
            R2[p] = resid_of<T>(B2[p], sum, own, inv_h2_2);
        }
        __syncthreads();
        if (tid < 512) {
            T sphi = 0, sres = 0;
#pragma unroll
            for (int dk = 0; dk < 2; dk++)
#pragma unroll
                for (int dj = 0; dj < 2; dj++)
#pragma unroll
                    for (int di = 0; di < 2; di++) {
                        int p = cs16(2 * ri + di, 2 * rj + dj, 2 * rk + dk);
                        sphi += F2[p];
                        sres += R2[p];
                    }
            T mphi = (T)0.125 * sphi;
            F1[tid] = mphi;
            O1[tid] = mphi;
            B1[tid] = (T)0.125 * sres;
        }
        __syncthreads();
        if (tid < 512) {
            T own = F1[tid];
            T xm = ri > 0 ? F1[tid - 1] : root_ghost<T>(g, r, 0, rj, rk, own);
            T xp = ri < 7 ? F1[tid + 1] : root_ghost<T>(g, r, 1, rj, rk, own);
            T ym = rj > 0 ? F1[tid - 8] : root_ghost<T>(g, r, 2, ri, rk, own);
            T yp = rj < 7 ? F1[tid + 8] : root_ghost<T>(g, r, 3, ri, rk, own);
            T zm = rk > 0 ? F1[tid - 64] : root_ghost<T>(g, r, 4, ri, rj, own);
            T zp = rk < 7 ? F1[tid + 64] : root_ghost<T>(g, r, 5, ri, rj, own);
            T s = xm + xp + ym + yp + zm + zp;
            B1[tid] = (s - (T)6 * own) * inv_h2_1 + B1[tid];
        }
        __syncthreads();
    };
    // exact root solve, as k_coarse (threads < 512, root cell tid)
    auto coarse = [&]() __attribute__((always_inline)) {
        const int t = tid & 511, i = ri, j = rj, k = rk;
        if (tid < 512) {
            double rr = (double)B1[t];
#pragma unroll
            for (int d = 0; d < 6; d++) {
                int a = d >> 1, sd = d & 1;
                int ca = a == 0 ? i : a == 1 ? j : k;
                int u = a == 0 ? j : i, v = a == 2 ? j : k;  // coordinates along the tangential axes
                bool edge = sd ? (ca == 7) : (ca == 0);
                if (edge && g.bct[d] == 0) {
                    double gv = g.bcval ? g.bcval[(r * 6 + d) * 64 + v * 8 + u] : g.bcv[d];
                    rr -= 2.0 * gv / (h1 * h1);
                }
            }
            X[t] = rr;
        }
        __syncthreads();
        if (tid < 512) { double s = 0; for (int q = 0; q < 8; q++) s += V[0 * 64 + q * 8 + i] * X[(k * 8 + j) * 8 + q]; Y[t] = s; }
        __syncthreads();
        if (tid < 512) { double s = 0; for (int q = 0; q < 8; q++) s += V[1 * 64 + q * 8 + j] * Y[(k * 8 + q) * 8 + i]; X[t] = s; }
        __syncthreads();
        if (tid < 512) {
            double s = 0;
            for (int q = 0; q < 8; q++) s += V[2 * 64 + q * 8 + k] * X[(q * 8 + j) * 8 + i];
            Y[t] = s * (h1 * h1) / (L[i] + L[8 + j] + L[16 + k]);
        }
        __syncthreads();
        if (tid < 512) { double s = 0; for (int q = 0; q < 8; q++) s += V[2 * 64 + k * 8 + q] * Y[(q * 8 + j) * 8 + i]; X[t] = s; }
        __syncthreads();
        if (tid < 512) { double s = 0; for (int q = 0; q < 8; q++) s += V[1 * 64 + j * 8 + q] * X[(k * 8 + q) * 8 + i]; Y[t] = s; }
        __syncthreads();
        if (tid < 512) {
            double s = 0;
            for (int q = 0; q < 8; q++) s += V[0 * 64 + i * 8 + q] * Y[(k * 8 + j) * 8 + q];
            F1[t] = (T)s;
        }
        __syncthreads();
    };
    // prolongation: the root correction delta = phi - old padded by its
    // homogeneous domain ghosts (faces only) into D1[10^3], then
    // phi_f += 1/4 d0 + 1/4 (dx + dy + dz) on every level-2 cell
    auto prolong = [&]() __attribute__((always_inline)) {
        if (!has2) return;
        if (tid < 1000) {
            int x = tid % 10 - 1, y = (tid / 10) % 10 - 1, z = tid / 100 - 1;
            int face = x < 0 ? 0 : x > 7 ? 1 : y < 0 ? 2 : y > 7 ? 3 : z < 0 ? 4 : z > 7 ? 5 : -1;
            int out = (x < 0 || x > 7) + (y < 0 || y > 7) + (z < 0 || z > 7);
            int q = min(max(x, 0), 7) + 8 * min(max(y, 0), 7) + 64 * min(max(z, 0), 7);
            T din = F1[q] - O1[q];
            D1[tid] = out > 1 ? (T)0 : face < 0 ? din : nm[face] ? din : -din;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 4; w++) {
            int p = tid + 1024 * w, I, J, K;
            cs16_cell(p, I, J, K);
            int c = ((K >> 1) + 1) * 100 + ((J >> 1) + 1) * 10 + (I >> 1) + 1;
            int sx = (I & 1) ? 1 : -1, sy = (J & 1) ? 10 : -10, sz = (K & 1) ? 100 : -100;
            T d0 = D1[c], dx = D1[c + sx], dy = D1[c + sy], dz = D1[c + sz];
            F2[p] += (T)0.25 * d0 + (T)0.25 * (dx + dy + dz);
        }
        __syncthreads();
    };

    if (fmg) {
        down();
        coarse();
        prolong();
    }
    if (has2) smooth(nd);
    down();
    coarse();
    prolong();
    if (has2) smooth(nu);

    if (tid < 512) {
        int i, j, k;
        cs_cell(tid, i, j, k);
        int n = i + 8 * j + 64 * k;
        phi[r * 512 + tid] = F1[n];
        rhs[r * 512 + tid] = B1[n];
        old[r * 512 + tid] = O1[n];
    }
    if (has2) {
#pragma unroll
        for (int w = 0; w < 4; w++) {
            int e = tid + 1024 * w, o = e >> 9, i, j, k;
            cs_cell(e & 511, i, j, k);
            int p = cs16(8 * (o & 1) + i, 8 * ((o >> 1) & 1) + j, 8 * (o >> 2) + k);
            phi[first2 * 512 + e] = F2[p];
        }
    }
}

// Covered cells of level l-1 <- mean of their 8 children on level l.
template <typename T>
__global__ __launch_bounds__(64) void k_restrict_phi(Geo g, T *__restrict__ phi, int64_t b0,
                                                     int64_t nbx) {
    int64_t lb = xcd_map(blockIdx.x, nbx);
    if (lb >= nbx) return;
    int64_t b = b0 + lb;
    int t = threadIdx.x, pi = t & 3, pj = (t >> 2) & 3, pk = t >> 4;
    T s = 0;
#pragma unroll
    for (int dk = 0; dk < 2; dk++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int di = 0; di < 2; di++) s += phi[b * 512 + cs_idx(2 * pi + di, 2 * pj + dj, 2 * pk + dk)];
    int64_t p = g.parent[b];
    int ci = 4 * (g.ijk[b * 4] & 1) + pi, cj = 4 * (g.ijk[b * 4 + 1] & 1) + pj,
        ck = 4 * (g.ijk[b * 4 + 2] & 1) + pk;
    phi[p * 512 + cs_idx(ci, cj, ck)] = (T)0.125 * s;
}

// The parent cells of every leaf box of level >= 2 <- the mean of the box's
// 8 cells under each (the arithmetic of k_restrict_phi), all levels in one
// launch.  Under 2:1 nesting every covered cell that a residual or a c_hat
// reads has only leaf children, so this is the restriction a stopping test
// needs; covered cells whose children have children are left as they are.
template <typename T>
__global__ __launch_bounds__(64) void k_restrict_leaves(Geo g, T *__restrict__ phi,
                                                        const int32_t *__restrict__ leaf, int64_t nleaf) {
    int64_t q = xcd_map(blockIdx.x, nleaf);
    if (q >= nleaf) return;
    int64_t b = leaf[q];
    if (g.ijk[b * 4 + 3] < 2) return;
    int t = threadIdx.x, pi = t & 3, pj = (t >> 2) & 3, pk = t >> 4;
    T s = 0;
#pragma unroll
    for (int dk = 0; dk < 2; dk++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int di = 0; di < 2; di++) s += phi[b * 512 + cs_idx(2 * pi + di, 2 * pj + dj, 2 * pk + dk)];
    int64_t p = g.parent[b];
    int ci = 4 * (g.ijk[b * 4] & 1) + pi, cj = 4 * (g.ijk[b * 4 + 1] & 1) + pj,
        ck = 4 * (g.ijk[b * 4 + 2] & 1) + pk;
    phi[p * 512 + cs_idx(ci, cj, ck)] = (T)0.125 * s;
}


// Leaf residual norms: per listed box, sum of r^2 h^3 and max |r|.  When
// r_out is set the residual is also stored, rounded to FP32 (right-hand side
// of the mixed-precision correction solve).
__global__ __launch_bounds__(256) void k_leaf_norms(Geo g, const double *__restrict__ phi,
                                                    const double *__restrict__ rhs,
                                                    const double *__restrict__ chat,
                                                    const int32_t *__restrict__ leaf, int64_t nleaf,
                                                    double *__restrict__ partial,
                                                    float *__restrict__ r_out) {
    __shared__ double P[512], H[384], S[4], M[4];
    int64_t q = xcd_map(blockIdx.x, nleaf);
    if (q >= nleaf) return;
    int64_t b = leaf[q];
    int t = threadIdx.x;
    double r0 = rhs[b * 512 + t], r1 = rhs[b * 512 + 256 + t];
    int l = g.ijk[b * 4 + 3];
    stage_full<double>(g, phi, chat, b, P, H);
    __syncthreads();
    double h = g.len / (8.0 * (double)(1 << (l - 1)));
    double inv_h2 = 1.0 / (h * h), vol = h * h * h;
    int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
    double ss = 0.0, mx = 0.0;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        int i = 2 * m + ((j + k + c) & 1);
        double own = P[c * 256 + t];
        double s = sum_full<double>(P, H, i, j, k);
        double r = resid_of<double>(c ? r1 : r0, s, own, inv_h2);
        if (r_out) r_out[b * 512 + c * 256 + t] = (float)r;
        ss = fmadd(r, r, ss);
        mx = nanmax(fabs(r), mx);
    }
    for (int off = 32; off > 0; off >>= 1) {
        ss += __shfl_xor(ss, off);
        mx = nanmax(__shfl_xor(mx, off), mx);
    }
    if ((t & 63) == 0) {
        S[t >> 6] = ss;
        M[t >> 6] = mx;
    }
    __syncthreads();
    if (t == 0) {
        partial[2 * q] = ((S[0] + S[1]) + (S[2] + S[3])) * vol;
        partial[2 * q + 1] = nanmax(nanmax(M[0], M[1]), nanmax(M[2], M[3]));
    }
}

// The norms of k_leaf_norms on the leaf boxes leaf[q0 .. q0+nq), into
// partial at their leaf positions q.  Each XCD takes a contiguous share of
// the leaf list (XCD-aware mapping of q): over the box range instead, the
// refined boxes, which exit at once, crowd the first shares (on the
// two-streamer tree the busiest XCD had 14% more leaf boxes than the mean).
// 128 threads per box with paired loads keep twice the boxes in flight.
// Thread u holds cell positions 2u and 2u+1 of both colours; the per-box sum
// follows k_leaf_norms' tree over the 256 positions (the shuffles over u
// are its stages 32..2, the pair sum its stage 1), so the partials are the
// same bits.  With h = len 2^-(l+2), 1/h^2 and h^3 are the power-of-two
// scalings ilen2 2^(2(l+2)) and len3 2^(-3(l+2)) of ilen2 = 1/len^2 and
// len3 = len^3 (the same bits as dividing, in the normal range), so the
// kernel holds no divide.  OUT: the FP32 residual is also stored.
template <bool OUT>
__global__ __launch_bounds__(128) void k_box_norms(Geo g, const double *__restrict__ phi,
                                                   const double *__restrict__ rhs,
                                                   const double *__restrict__ chat,
                                                   const int32_t *__restrict__ leaf, int64_t q0, int64_t nq,
                                                   double *__restrict__ partial, float *__restrict__ r_out,
                                                   double ilen2, double len3) {
    __shared__ double P[512], H[384], S[4], M[4];
    int64_t lq = xcd_map(blockIdx.x, nq);
    if (lq >= nq) return;
    const int64_t q = q0 + lq;
    const int64_t b = leaf[q];
    const int u = threadIdx.x;
    const double2 p0 = reinterpret_cast<const double2 *>(phi + b * 512)[u];
    const double2 p1 = reinterpret_cast<const double2 *>(phi + b * 512 + 256)[u];
    const double2 r0 = ld_stream(reinterpret_cast<const double2 *>(rhs + b * 512) + u);
    const double2 r1 = ld_stream(reinterpret_cast<const double2 *>(rhs + b * 512 + 256) + u);
    const FaceTab ft = face_tab(g, b);
#pragma unroll
    for (int r = 0; r < 3; r++) {
        int e = u + 128 * r, d = e >> 6, w = e & 63;
        H[e] = ghost_at<double>(g, phi, chat, b, d, pick6(ft.nb, d), pick6(ft.slot, d), w & 7, w >> 3);
    }
    reinterpret_cast<double2 *>(P)[u] = p0;
    reinterpret_cast<double2 *>(P)[128 + u] = p1;
    __syncthreads();
    const int l = g.ijk[b * 4 + 3];
    const double inv_h2 = ldexp(ilen2, 2 * (l + 2)), vol = ldexp(len3, -3 * (l + 2));
    double ss[2], mx[2], rr[2][2];
#pragma unroll
    for (int sl = 0; sl < 2; sl++) {
        const int t = 2 * u + sl;
        const int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
        ss[sl] = 0.0;
        mx[sl] = 0.0;
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int i = 2 * m + ((j + k + c) & 1);
            const double rc = c ? (sl ? r1.y : r1.x) : (sl ? r0.y : r0.x);
            double r = resid_of<double>(rc, sum_full<double>(P, H, i, j, k), P[c * 256 + t], inv_h2);
            rr[c][sl] = r;
            ss[sl] = fmadd(r, r, ss[sl]);
            mx[sl] = nanmax(fabs(r), mx[sl]);
        }
    }
    if (OUT) {
        reinterpret_cast<float2 *>(r_out + b * 512)[u] = make_float2((float)rr[0][0], (float)rr[0][1]);
        reinterpret_cast<float2 *>(r_out + b * 512 + 256)[u] = make_float2((float)rr[1][0], (float)rr[1][1]);
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
#pragma unroll
        for (int sl = 0; sl < 2; sl++) {
            ss[sl] += __shfl_xor(ss[sl], off);
            mx[sl] = nanmax(__shfl_xor(mx[sl], off), mx[sl]);
        }
    }
    const double st = ss[0] + ss[1], mt = nanmax(mx[1], mx[0]);
    if ((u & 31) == 0) {
        S[u >> 5] = st;
        M[u >> 5] = mt;
    }
    __syncthreads();
    if (u == 0) {
        partial[2 * q] = ((S[0] + S[1]) + (S[2] + S[3])) * vol;
        partial[2 * q + 1] = nanmax(nanmax(M[0], M[1]), nanmax(M[2], M[3]));
    }
}

// out[q][e] = (L x)(cell e of leaf box leaf[q]) for the composite operator
// with the field's ghosts (same layout as the field, one 512-run per leaf
// position); the operator applications of the learned correction step.
template <typename T>
__global__ __launch_bounds__(256) void k_leaf_apply(Geo g, const T *__restrict__ x,
                                                    const T *__restrict__ chat,
                                                    const int32_t *__restrict__ leaf, int64_t nleaf,
                                                    T *__restrict__ out) {
    __shared__ T P[512], H[384];
    int64_t q = xcd_map(blockIdx.x, nleaf);
    if (q >= nleaf) return;
    int64_t b = leaf[q];
    int t = threadIdx.x;
    int l = g.ijk[b * 4 + 3];
    stage_full<T>(g, x, chat, b, P, H);
    __syncthreads();
    double h = g.len / (8.0 * (double)(1 << (l - 1)));
    T inv_h2 = (T)(1.0 / (h * h));
    int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        int i = 2 * m + ((j + k + c) & 1);
        T own = P[c * 256 + t];
        out[q * 512 + c * 256 + t] = (sum_full<T>(P, H, i, j, k) - (T)6 * own) * inv_h2;
    }
}

// Electric field of phi (section 2.3, E = -grad phi), one box per block:
// face components by central differences, (phi(f-1) - phi(f)) / h across face
// f = 0..8 of each axis (faces 0 and 8 with the box's ghosts), into
// e_face[((b*3 + a)*9 + f)*64 + v*8 + u]; and the strength at the cell
// centres, sqrt(Ex^2 + Ey^2 + Ez^2) with each component the mean of the
// cell's two faces, into e_norm[b*512 + natural index].  Either output may
// be null.  The 1728 face values are formed once (times 1/h) in LDS.
__global__ __launch_bounds__(256) void k_efield(Geo g, const double *__restrict__ phi,
                                                const double *__restrict__ chat, int64_t n,
                                                double *__restrict__ e_face, double *__restrict__ e_norm) {
    __shared__ double P[512], H[384], EF[1728];
    int64_t b = xcd_map(blockIdx.x, n);
    if (b >= n) return;
    int t = threadIdx.x;
    int l = g.ijk[b * 4 + 3];
    stage_full<double>(g, phi, chat, b, P, H);
    __syncthreads();
    const double inv_h = (8.0 * (double)(1 << (l - 1))) / g.len;
    // value of cell c along axis a (c = -1 or 8: the ghost on that face) at
    // tangential (u, v)
    auto val = [&](int a, int c, int u, int v) __attribute__((always_inline)) -> double {
        if (c < 0) return H[(2 * a) * 64 + v * 8 + u];
        if (c > 7) return H[(2 * a + 1) * 64 + v * 8 + u];
        int i = a == 0 ? c : u, j = a == 0 ? u : a == 1 ? c : v, k = a == 2 ? c : v;
        return P[cs_idx(i, j, k)];
    };
    for (int e = t; e < 3 * 9 * 64; e += 256) {
        int a = e / 576, r = e - 576 * a, f = r >> 6, v = (r >> 3) & 7, u = r & 7;
        double ef = (val(a, f - 1, u, v) - val(a, f, u, v)) * inv_h;
        EF[e] = ef;
        if (e_face) e_face[b * 1728 + e] = ef;
    }
    if (!e_norm) return;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 2; w++) {
        int c = t + 256 * w, i = c & 7, j = (c >> 3) & 7, k = c >> 6;
        double ex = (EF[0 * 576 + i * 64 + k * 8 + j] + EF[0 * 576 + (i + 1) * 64 + k * 8 + j]) / 2.0;
        double ey = (EF[1 * 576 + j * 64 + k * 8 + i] + EF[1 * 576 + (j + 1) * 64 + k * 8 + i]) / 2.0;
        double ez = (EF[2 * 576 + k * 64 + j * 8 + i] + EF[2 * 576 + (k + 1) * 64 + j * 8 + i]) / 2.0;
        e_norm[b * 512 + c] = sqrt(ex * ex + ey * ey + ez * ez);
    }
}

// Faces of the face neighbours, formed from the uploaded face tables: for
// box b, face d with a same-level neighbour N, and the 4 faces of N across
// the two axes tangential to d (-t1, +t1, -t2, +t2), the pair (nbr[N][d'],
// cfslot[N][d']) (the fused Gauss-Seidel sweep recomputes N's face layer
// and needs N's ghosts); all -2 where face d has no same-level neighbour.
// One thread per (box, face).
__global__ __launch_bounds__(256) void k_face_xt(const int32_t *__restrict__ nbr, const int32_t *__restrict__ cfslot,
                                                 int64_t n, int32_t *__restrict__ xt) {
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= 6 * n) return;
    const int d = (int)(e % 6);
    const int32_t N = nbr[e];
    int32_t *out = xt + e * 8;
    if (N < 0) {
#pragma unroll
        for (int q = 0; q < 8; q++) out[q] = -2;
        return;
    }
    const int a = d >> 1, t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    const int tf[4] = {2 * t1, 2 * t1 + 1, 2 * t2, 2 * t2 + 1};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        out[2 * q] = nbr[6 * (int64_t)N + tf[q]];
        out[2 * q + 1] = cfslot[6 * (int64_t)N + tf[q]];
    }
}

// Refinement scores (section 2.5, the space-charge criterion |b| h^2 > c3):
// for box b, scores[b*27 + r] = the largest |b| h^2 over its cells in region
// r = (sx+1) + 3 (sy+1) + 9 (sz+1), where along each axis s = -1 takes cells
// 0..2, s = +1 cells 5..7 and s = 0 all cells (so r = 13 is the whole box
// and the 26 others the cells within 3 of each face, edge and corner).
__global__ __launch_bounds__(256) void k_refine_scores(Geo g, const double *__restrict__ rhs, int64_t n,
                                                       double *__restrict__ scores) {
    __shared__ double W[4][27];
    int64_t b = xcd_map(blockIdx.x, n);
    if (b >= n) return;
    int t = threadIdx.x;
    int l = g.ijk[b * 4 + 3];
    double h = g.len / (8.0 * (double)(1 << (l - 1)));
    double m[27];
#pragma unroll
    for (int r = 0; r < 27; r++) m[r] = 0.0;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        int q = c * 256 + t, mm = q & 3, j = (q >> 2) & 7, k = (q >> 5) & 7;
        int i = 2 * mm + ((j + k + c) & 1);
        double v = fabs(rhs[b * 512 + q]) * (h * h);
        bool lo[3] = {i <= 2, j <= 2, k <= 2}, hi[3] = {i >= 5, j >= 5, k >= 5};
#pragma unroll
        for (int r = 0; r < 27; r++) {
            int sx = r % 3 - 1, sy = (r / 3) % 3 - 1, sz = r / 9 - 1;
            bool in = (sx == 0 || (sx < 0 ? lo[0] : hi[0])) && (sy == 0 || (sy < 0 ? lo[1] : hi[1])) &&
                      (sz == 0 || (sz < 0 ? lo[2] : hi[2]));
            if (in) m[r] = fmax(m[r], v);
        }
    }
#pragma unroll
    for (int r = 0; r < 27; r++) {
        double v = m[r];
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
        if ((t & 63) == 0) W[t >> 6][r] = v;
    }
    __syncthreads();
    if (t < 27) scores[b * 27 + t] = fmax(fmax(W[0][t], W[1][t]), fmax(W[2][t], W[3][t]));
}

// The refinement criterion with its 3-cell buffer (section 2.5) reduced to
// one value per box: for a leaf box b, near[b] = the largest score over b's
// cells and the cells of its same-level leaf neighbours within 3 cells of
// it (region 26 - o of neighbour b + o; a missing or refined neighbour
// contributes b's own whole-box score r = 13); 0 for a refined box.  The
// maximum is taken as (m < x) ? x : m in the order o = 0..26, the host
// planner's arithmetic, so the two give the same bits.
__global__ __launch_bounds__(256) void k_refine_near(const int32_t *__restrict__ n27,
                                                     const int32_t *__restrict__ isleaf,
                                                     const double *__restrict__ sc, int64_t n,
                                                     double *__restrict__ near) {
    int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= n) return;
    if (!isleaf[b]) {
        near[b] = 0.0;
        return;
    }
    const int32_t *nb = n27 + 27 * b;
    double m = sc[27 * b + 13];
    for (int o = 0; o < 27; o++) {
        int32_t N = nb[o];
        bool use = N >= 0 && isleaf[N];
        double x = sc[use ? 27 * (int64_t)N + (26 - o) : 27 * b + 13];
        m = (m < x) ? x : m;
    }
    near[b] = m;
}

// Transfer of phi to a new tree.  Copy: new box b takes the old box src[b]
// (same level and position) when src[b] >= 0.
__global__ __launch_bounds__(256) void k_transfer_copy(const double *__restrict__ from, double *__restrict__ to,
                                                       const int32_t *__restrict__ src, int64_t n) {
    int64_t b = xcd_map(blockIdx.x, n);
    if (b >= n) return;
    int64_t o = src[b];
    if (o < 0) return;
    int t = threadIdx.x;
    to[b * 512 + t] = from[o * 512 + t];
    to[b * 512 + 256 + t] = from[o * 512 + 256 + t];
}

// Interpolation: new box list[q] (level l, no counterpart in the old tree)
// from its parent in the new tree (already filled), with the stencil of the
// correction prolongation applied to phi itself, 1/4 p(C) + 1/4 (p(C + s_x) +
// p(C + s_y) + p(C + s_z)), C the parent cell and s the side of the fine cell
// in it; a neighbour outside the parent is the parent's ghost on that face
// (same-level neighbour, boundary condition or refinement-boundary value).
// Exact for linear functions.
__global__ __launch_bounds__(256) void k_transfer_interp(Geo g, double *__restrict__ phi,
                                                         const double *__restrict__ chat,
                                                         const int32_t *__restrict__ list, int64_t nlist) {
    __shared__ double P[512], H[384];
    int64_t q = xcd_map(blockIdx.x, nlist);
    if (q >= nlist) return;
    int64_t b = list[q];
    int64_t p = g.parent[b];
    int o[3] = {g.ijk[b * 4] & 1, g.ijk[b * 4 + 1] & 1, g.ijk[b * 4 + 2] & 1};
    int t = threadIdx.x;
    stage_full<double>(g, phi, chat, p, P, H);
    __syncthreads();
    // parent value at (x, y, z); at most one coordinate is -1 or 8 (a face ghost)
    auto pv = [&](int x, int y, int z) __attribute__((always_inline)) -> double {
        if (x < 0) return H[0 * 64 + z * 8 + y];
        if (x > 7) return H[1 * 64 + z * 8 + y];
        if (y < 0) return H[2 * 64 + z * 8 + x];
        if (y > 7) return H[3 * 64 + z * 8 + x];
        if (z < 0) return H[4 * 64 + y * 8 + x];
        if (z > 7) return H[5 * 64 + y * 8 + x];
        return P[cs_idx(x, y, z)];
    };
    int m = t & 3, j = (t >> 2) & 7, k = t >> 5;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        int i = 2 * m + ((j + k + c) & 1);
        int cx = 4 * o[0] + (i >> 1), cy = 4 * o[1] + (j >> 1), cz = 4 * o[2] + (k >> 1);
        int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
        double d0 = pv(cx, cy, cz), dx = pv(cx + sx, cy, cz), dy = pv(cx, cy + sy, cz),
               dz = pv(cx, cy, cz + sz);
        phi[b * 512 + c * 256 + t] = 0.25 * d0 + 0.25 * (dx + dy + dz);
    }
}

// phi (FP64) += e (FP32) on every cell: the update of the mixed-precision
// iterative refinement.
__global__ __launch_bounds__(256) void k_ir_update(double *__restrict__ phi, const float *__restrict__ e,
                                                   int64_t count) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < count) phi[q] += (double)e[q];
}

// Per-tree reduction of the per-box partials in a fixed order, in two
// stages.  Stage 1: block c sums the partials of the leaf boxes at positions
// leaf_tree[chunk[c].begin .. chunk[c].end) (a range of one tree, at most
// kReduceChunk long) into part2[c].  Stage 2: block t sums the chunks
// choff[t] .. choff[t+1] of tree t into result[2t] (sum) and result[2t+1]
// (max).
__device__ __forceinline__ void block_sum_max(double &s, double &m, double *S, double *M) {
    int t = threadIdx.x;
    S[t] = s;
    M[t] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            S[t] += S[t + w];
            M[t] = nanmax(M[t + w], M[t]);
        }
        __syncthreads();
    }
    s = S[0];
    m = M[0];
}

__global__ __launch_bounds__(256) void k_reduce_chunks(const double *__restrict__ partial,
                                                       const int32_t *__restrict__ leaf_tree,
                                                       const int32_t *__restrict__ chunk,
                                                       double *__restrict__ part2) {
    __shared__ double S[256], M[256];
    int c = blockIdx.x, t = threadIdx.x;
    int beg = chunk[3 * c + 1], end = chunk[3 * c + 2];
    double s = 0.0, m = 0.0;
    for (int q = beg + t; q < end; q += 256) {
        int64_t p = leaf_tree[q];
        s += partial[2 * p];
        m = nanmax(partial[2 * p + 1], m);
    }
    block_sum_max(s, m, S, M);
    if (t == 0) {
        part2[2 * c] = s;
        part2[2 * c + 1] = m;
    }
}

__global__ __launch_bounds__(256) void k_reduce_trees(const double *__restrict__ part2,
                                                      const int32_t *__restrict__ choff,
                                                      double *__restrict__ result) {
    __shared__ double S[256], M[256];
    int tr = blockIdx.x, t = threadIdx.x;
    double s = 0.0, m = 0.0;
    for (int c = choff[tr] + t; c < choff[tr + 1]; c += 256) {
        s += part2[2 * c];
        m = nanmax(part2[2 * c + 1], m);
    }
    block_sum_max(s, m, S, M);
    if (t == 0) {
        result[2 * tr] = s;
        result[2 * tr + 1] = m;
    }
}

// Streaming copy with 16-byte vector accesses, grid-stride: the achievable
// device bandwidth reference of the roofline.
__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                int64_t n16) {
    int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n16; q += stride) dst[q] = src[q];
}

}  // namespace

// ------------------------------------------------------------- launchers

template <typename T>
void launch_fill(T *p, int64_t count, T v, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
}
template <typename T>
void launch_pack(const double *nat, T *cs, int64_t nbox, hipStream_t s) {
    hipLaunchKernelGGL(k_pack<T>, dim3((unsigned)(nbox * 2)), dim3(256), 0, s, nat, cs, nbox);
}
template <typename T>
void launch_unpack(const T *cs, double *nat, int64_t nbox, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack<T>, dim3((unsigned)(nbox * 2)), dim3(256), 0, s, cs, nat, nbox);
}
template <typename T, int CPT>
void launch_gsrb_cpt(const Geo &g, T *phi, const T *rhs, const T *chat, int64_t b0, int64_t nb,
                     T h2, int colour, int xcd, hipStream_t s, const int32_t *rmask, double *phi64) {
    dim3 grid((unsigned)(xcd ? xcd_grid(nb) : nb)), block(256 / CPT);
    if (colour == 0)
        hipLaunchKernelGGL((k_gsrb<0, T, CPT>), grid, block, 0, s, g, phi, rhs, chat, b0, nb, h2, xcd,
                           nullptr, nullptr);
    else if (phi64)
        hipLaunchKernelGGL((k_gsrb<1, T, CPT, kSweepIrUpdate>), grid, block, 0, s, g, phi, rhs, chat, b0, nb,
                           h2, xcd, rmask, phi64);
    else if (rmask)
        hipLaunchKernelGGL((k_gsrb<1, T, CPT, kSweepRestrict>), grid, block, 0, s, g, phi, rhs, chat, b0, nb,
                           h2, xcd, rmask, nullptr);
    else
        hipLaunchKernelGGL((k_gsrb<1, T, CPT>), grid, block, 0, s, g, phi, rhs, chat, b0, nb, h2, xcd,
                           nullptr, nullptr);
}

template <typename T>
void launch_gsrb_sweep(const Geo &g, const T *src, T *dst, T *rhs, const T *chat, int64_t b0,
                       int64_t nb, T h2, int xcd, hipStream_t s, int fas, const int32_t *isleaf,
                       T inv_h2, T *fasbuf) {
    if (nb <= 0) return;
    dim3 grid((unsigned)(xcd ? xcd_grid(nb) : nb));
    if (fas)
        hipLaunchKernelGGL((k_gsrb_sweep<T, true>), grid, dim3(256), 0, s, g, src, dst, rhs, chat, b0, nb, h2,
                           xcd, fas, isleaf, inv_h2, fasbuf);
    else
        hipLaunchKernelGGL((k_gsrb_sweep<T, false>), grid, dim3(256), 0, s, g, src, dst, rhs, chat, b0, nb,
                           h2, xcd, 0, isleaf, inv_h2, fasbuf);
}

template <typename T>
void launch_gsrb(const Geo &g, T *phi, const T *rhs, const T *chat, int64_t b0, int64_t nb, T h2,
                 int colour, int variant, hipStream_t s, const int32_t *rmask, double *phi64) {
    if (nb <= 0) return;
    if (colour != 1 || (phi64 ? !gsrb_updates(variant) : !gsrb_restricts(variant))) {
        rmask = nullptr;  // callers check gsrb_restricts / gsrb_updates first
        phi64 = nullptr;
    }
    if (sizeof(T) != 4) phi64 = nullptr;
    if (variant >= kGsrbPipeVariant) {
        // persistent workgroups: at most 2048 (c = 5) or 4096 (c = 6)
        int64_t cap = variant >= kGsrbPipeVariant + 2 ? 4096 : 2048;
        int xcd = variant & 1;
        int64_t nw = nb < cap ? nb : cap;
        dim3 grid((unsigned)(xcd ? xcd_grid(nw) : nw));
        if (colour == 0)
            hipLaunchKernelGGL((k_gsrb_pipe<0, T>), grid, dim3(128), 0, s, g, phi, rhs, chat, b0, nb, h2, xcd);
        else
            hipLaunchKernelGGL((k_gsrb_pipe<1, T>), grid, dim3(128), 0, s, g, phi, rhs, chat, b0, nb, h2, xcd);
        return;
    }
    if (variant >= kGsrbOctVariant && (nb & 7) == 0) {
        int64_t noct = nb >> 3;
        int xcd = variant & 1;
        dim3 grid((unsigned)(xcd ? xcd_grid(noct) : noct));
        if (colour == 0)
            hipLaunchKernelGGL((k_gsrb_oct<0, T>), grid, dim3(512), 0, s, g, phi, rhs, chat, b0, noct, h2, xcd,
                               nullptr, nullptr);
        else if (phi64)
            hipLaunchKernelGGL((k_gsrb_oct<1, T, true>), grid, dim3(512), 0, s, g, phi, rhs, chat, b0, noct, h2,
                               xcd, rmask, phi64);
        else
            hipLaunchKernelGGL((k_gsrb_oct<1, T>), grid, dim3(512), 0, s, g, phi, rhs, chat, b0, noct, h2, xcd,
                               nullptr, nullptr);
        return;
    }
    if (variant >= kGsrbHalfVariants) variant = kGsrbDefault;
    int xcd = variant & 1;
    switch (variant >> 1) {
    case 0: launch_gsrb_cpt<T, 1>(g, phi, rhs, chat, b0, nb, h2, colour, xcd, s, rmask, phi64); break;
    case 2: launch_gsrb_cpt<T, 4>(g, phi, rhs, chat, b0, nb, h2, colour, xcd, s, rmask, phi64); break;
    default: launch_gsrb_cpt<T, 2>(g, phi, rhs, chat, b0, nb, h2, colour, xcd, s, rmask, phi64); break;
    }
}
template <typename T>
void launch_cf_coarse(const Geo &g, const T *phi, T *chat, const int32_t *slots, int64_t s0,
                      int64_t ns, hipStream_t s) {
    if (ns <= 0) return;
    hipLaunchKernelGGL(k_cf_coarse<T>, dim3((unsigned)((ns + 3) / 4)), dim3(256), 0, s, g, phi, chat,
                       slots, s0, ns);
}
template <typename T>
void launch_resid_restrict(const Geo &g, T *phi, T *rhs, T *old, const T *chat, int64_t b0,
                           int64_t nb, const int32_t *leaf_prev, int64_t nleaf_prev, T inv_h2,
                           hipStream_t s, const int32_t *leafpos, double *partial, double vol) {
    if (nb + nleaf_prev <= 0) return;
    dim3 grid((unsigned)(xcd_grid(nb) + nleaf_prev));
    if (partial)
        hipLaunchKernelGGL((k_resid_restrict<T, true>), grid, dim3(128), 0, s, g, phi, rhs, old, chat, b0, nb,
                           leaf_prev, nleaf_prev, inv_h2, leafpos, partial, vol);
    else
        hipLaunchKernelGGL((k_resid_restrict<T, false>), grid, dim3(128), 0, s, g, phi, rhs, old, chat, b0, nb,
                           leaf_prev, nleaf_prev, inv_h2, leafpos, partial, vol);
}
template <typename T>
void launch_fas_rhs(const Geo &g, const T *phi, T *rhs, const T *chat, const int32_t *list,
                    int64_t nlist, T inv_h2, hipStream_t s) {
    if (nlist <= 0) return;
    hipLaunchKernelGGL(k_fas_rhs<T>, dim3((unsigned)xcd_grid(nlist)), dim3(128), 0, s, g, phi, rhs,
                       chat, list, nlist, inv_h2);
}
template <typename T>
void launch_prolong_cf(const Geo &g, T *phi, const T *old, int64_t b0, int64_t nb, T *chat,
                       const int32_t *slots, int64_t s0, int64_t ns, hipStream_t s) {
    if (nb <= 0 && ns <= 0) return;
    dim3 grid((unsigned)(xcd_grid(nb) + (ns + 3) / 4));
    hipLaunchKernelGGL(k_prolong_cf<T>, grid, dim3(256), 0, s, g, phi, old, b0, nb, chat, slots, s0, ns);
}
template <typename T>
void launch_delta_pad(const Geo &g, const T *phi, const T *old, const int32_t *refined, int64_t nref, T *pad,
                      T *chat, const int32_t *slots, int64_t s0, int64_t ns, hipStream_t s) {
    if (nref <= 0 && ns <= 0) return;
    dim3 grid((unsigned)(xcd_grid(nref) + (ns + 3) / 4));
    hipLaunchKernelGGL(k_delta_pad<T>, grid, dim3(256), 0, s, g, phi, old, refined, nref, pad, chat, slots, s0, ns);
}
template <typename T>
void launch_gsrb_pro(const Geo &g, T *phi, const T *rhs, const T *pad, const T *chat, int64_t b0, int64_t nb,
                     T h2, int colour, hipStream_t s) {
    if (nb <= 0) return;
    dim3 grid((unsigned)xcd_grid(nb));
    if (colour == 0)
        hipLaunchKernelGGL(k_gsrb_pro_red<T>, grid, dim3(128), 0, s, g, phi, rhs, pad, chat, b0, nb, h2);
    else
        hipLaunchKernelGGL(k_gsrb_pro_black<T>, grid, dim3(128), 0, s, g, phi, rhs, pad, chat, b0, nb, h2);
}
template <typename T>
void launch_coarse(const Geo &g, T *phi, const T *rhs, const double *eig, int64_t b0, int64_t nroot,
                   double h, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse<T>, dim3((unsigned)nroot), dim3(512), 0, s, g, phi, rhs, eig, b0, h);
}
template <typename T>
void launch_bottom(const Geo &g, T *phi, T *rhs, T *old, const double *eig, int64_t r0, int ntree,
                   const int32_t *root2, double h2, double h1, int nd, int nu, int fmg, int fas2,
                   const int32_t *isleaf, hipStream_t s) {
    hipLaunchKernelGGL(k_bottom<T>, dim3((unsigned)ntree), dim3(1024), 0, s, g, phi, rhs, old, eig, r0, root2,
                       (T)(h2 * h2), (T)(1.0 / (h2 * h2)), (T)(1.0 / (h1 * h1)), h1, nd, nu, fmg, fas2,
                       isleaf);
}
template <typename T>
void launch_restrict_phi(const Geo &g, T *phi, int64_t b0, int64_t nb, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_restrict_phi<T>, dim3((unsigned)xcd_grid(nb)), dim3(64), 0, s, g, phi, b0, nb);
}
template <typename T>
void launch_restrict_leaves(const Geo &g, T *phi, const int32_t *leaf, int64_t nleaf, hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_restrict_leaves<T>, dim3((unsigned)xcd_grid(nleaf)), dim3(64), 0, s, g, phi, leaf,
                       nleaf);
}
void launch_leaf_norms(const Geo &g, const double *phi, const double *rhs, const double *chat,
                       const int32_t *leaf, int64_t nleaf, double *partial, float *r_out,
                       hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_leaf_norms, dim3((unsigned)xcd_grid(nleaf)), dim3(256), 0, s, g, phi, rhs,
                       chat, leaf, nleaf, partial, r_out);
}
void launch_box_norms(const Geo &g, const double *phi, const double *rhs, const double *chat, const int32_t *leaf,
                      int64_t q0, int64_t nq, double *partial, float *r_out, hipStream_t s) {
    if (nq <= 0) return;
    const double ilen2 = 1.0 / (g.len * g.len), len3 = g.len * g.len * g.len;
    if (r_out)
        hipLaunchKernelGGL(k_box_norms<true>, dim3((unsigned)xcd_grid(nq)), dim3(128), 0, s, g, phi, rhs, chat,
                           leaf, q0, nq, partial, r_out, ilen2, len3);
    else
        hipLaunchKernelGGL(k_box_norms<false>, dim3((unsigned)xcd_grid(nq)), dim3(128), 0, s, g, phi, rhs, chat,
                           leaf, q0, nq, partial, r_out, ilen2, len3);
}
template <typename T>
void launch_leaf_apply(const Geo &g, const T *x, const T *chat, const int32_t *leaf, int64_t nleaf,
                       T *out, hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_leaf_apply<T>, dim3((unsigned)xcd_grid(nleaf)), dim3(256), 0, s, g, x, chat, leaf,
                       nleaf, out);
}
template void launch_leaf_apply<float>(const Geo &, const float *, const float *, const int32_t *,
                                       int64_t, float *, hipStream_t);
void launch_efield(const Geo &g, const double *phi, const double *chat, int64_t n, double *e_face,
                   double *e_norm, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_efield, dim3((unsigned)xcd_grid(n)), dim3(256), 0, s, g, phi, chat, n, e_face, e_norm);
}
void launch_face_xt(const int32_t *nbr, const int32_t *cfslot, int64_t n, int32_t *xt, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_face_xt, dim3((unsigned)((6 * n + 255) / 256)), dim3(256), 0, s, nbr, cfslot, n, xt);
}
void launch_refine_near(const int32_t *n27, const int32_t *isleaf, const double *scores, int64_t n, double *near,
                        hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_refine_near, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n27, isleaf, scores, n,
                       near);
}
void launch_refine_scores(const Geo &g, const double *rhs, int64_t n, double *scores, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_refine_scores, dim3((unsigned)xcd_grid(n)), dim3(256), 0, s, g, rhs, n, scores);
}
void launch_transfer_copy(const double *from, double *to, const int32_t *src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_transfer_copy, dim3((unsigned)xcd_grid(n)), dim3(256), 0, s, from, to, src, n);
}
void launch_transfer_interp(const Geo &g, double *phi, const double *chat, const int32_t *list, int64_t nlist,
                            hipStream_t s) {
    if (nlist <= 0) return;
    hipLaunchKernelGGL(k_transfer_interp, dim3((unsigned)xcd_grid(nlist)), dim3(256), 0, s, g, phi, chat, list,
                       nlist);
}
void launch_ir_update(double *phi, const float *e, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_ir_update, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, phi, e, count);
}
void launch_copy16(const void *src, void *dst, int64_t n16, int blocks, hipStream_t s) {
    if (n16 <= 0) return;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst,
                       n16);
}
void launch_reduce_trees(const double *partial, const int32_t *leaf_tree, const int32_t *chunk,
                         int64_t nchunk, const int32_t *choff, int ntree, double *part2,
                         double *result, hipStream_t s) {
    if (nchunk > 0)
        hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)nchunk), dim3(256), 0, s, partial, leaf_tree,
                           chunk, part2);
    hipLaunchKernelGGL(k_reduce_trees, dim3((unsigned)ntree), dim3(256), 0, s, part2, choff, result);
}

#define MG_INSTANTIATE(T)                                                                        \
    template void launch_fill<T>(T *, int64_t, T, hipStream_t);                                  \
    template void launch_pack<T>(const double *, T *, int64_t, hipStream_t);                     \
    template void launch_unpack<T>(const T *, double *, int64_t, hipStream_t);                   \
    template void launch_gsrb<T>(const Geo &, T *, const T *, const T *, int64_t, int64_t, T, int, \
                                 int, hipStream_t, const int32_t *, double *);                   \
    template void launch_gsrb_sweep<T>(const Geo &, const T *, T *, T *, const T *, int64_t,       \
                                       int64_t, T, int, hipStream_t, int, const int32_t *, T, T *); \
    template void launch_restrict_leaves<T>(const Geo &, T *, const int32_t *, int64_t, hipStream_t); \
    template void launch_cf_coarse<T>(const Geo &, const T *, T *, const int32_t *, int64_t,     \
                                      int64_t, hipStream_t);                                     \
    template void launch_resid_restrict<T>(const Geo &, T *, T *, T *, const T *, int64_t,       \
                                           int64_t, const int32_t *, int64_t, T, hipStream_t,    \
                                           const int32_t *, double *, double);                   \
    template void launch_fas_rhs<T>(const Geo &, const T *, T *, const T *, const int32_t *,     \
                                    int64_t, T, hipStream_t);                                    \
    template void launch_prolong_cf<T>(const Geo &, T *, const T *, int64_t, int64_t, T *,       \
                                       const int32_t *, int64_t, int64_t, hipStream_t);          \
    template void launch_gsrb_pro<T>(const Geo &, T *, const T *, const T *, const T *, int64_t,   \
                                     int64_t, T, int, hipStream_t);                              \
    template void launch_delta_pad<T>(const Geo &, const T *, const T *, const int32_t *, int64_t, \
                                      T *, T *, const int32_t *, int64_t, int64_t, hipStream_t);   \
    template void launch_coarse<T>(const Geo &, T *, const T *, const double *, int64_t, int64_t, \
                                   double, hipStream_t);                                         \
    template void launch_restrict_phi<T>(const Geo &, T *, int64_t, int64_t, hipStream_t);        \
    template void launch_bottom<T>(const Geo &, T *, T *, T *, const double *, int64_t, int,     \
                                   const int32_t *, double, double, int, int, int, int,          \
                                   const int32_t *, hipStream_t);
MG_INSTANTIATE(double)
MG_INSTANTIATE(float)
#undef MG_INSTANTIATE

}  // namespace mg
