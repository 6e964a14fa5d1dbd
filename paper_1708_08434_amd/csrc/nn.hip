// Learned correction network for the octree multigrid (gfx950).
//
// The network maps a leaf box's scaled residual (8^3 plus its one-cell ghost
// layer, 10^3) to a correction on the box's 8^3 cells:
//   conv 3^3 valid 1->16, ReLU, conv 3^3 same 16->16, ReLU, conv 3^3 same 16->1.
// Weights, the input and both hidden activations are BF16 (round to nearest
// even), accumulation is FP32.  Parameters are kept as FP32 masters in the
// order W1[16][27], b1[16], W2[16 out][16 in][27], b2[16], W3[16][27], b3,
// with tap t = (dk*3 + dj)*3 + di.
//
// Forward: a box's activations stay in LDS (one box at a time per workgroup).
//  * layer 1 is an implicit GEMM [16 cells x 32 taps (27 used)] x [32 x 16
//    channels]: one 16x16x32 BF16 MFMA per 16-cell tile;
//  * layer 2 is an implicit GEMM with K = 27 taps x 16 channels, taken as 18
//    16x16x32 MFMAs per tile (the kernel rows of one z offset paired, 16
//    channels each, per instruction) and blocked along z, so that each
//    loaded input slice serves the three output slices it reaches;
//    activations are stored [padded cell][channel];
//  * layer 3 first forms Q[tap][cell] = sum_c W3[c][tap] a2[c][cell] with
//    16x16x16 MFMAs (N = taps), then y[cell] = b3 + sum_tap Q[tap][cell+tap-1],
//    which turns the 16->1 convolution into a dense GEMM plus a 27-term sum.
// The backward pass (training only) runs in FP32 on the vector units.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "mg.h"
#include "nn.h"

namespace mg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kW1 = 0, kB1 = 432, kW2 = 448, kB2 = 7360, kW3 = 7376, kB3 = 7808;
constexpr int kP1 = 0, kP2 = 512, kP3 = 512 + 18 * 512;  // offsets in the packed fragments

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
// The same rounding (nearest even) by the hardware conversion; a NaN stays a
// NaN (its payload may differ from f2bf's).  Two values per instruction.
__device__ __forceinline__ uint16_t f2bf_hw(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float round_bf(float f) { return bf2f(f2bf(f)); }
// max(z, 0) that propagates NaN (a non-finite weight must reach the output)
__device__ __forceinline__ float relu(float z) { return !(z <= 0.0f) ? z : 0.0f; }

// offset of tap t in a 10^3 block (x fastest)
__host__ __device__ constexpr int tap_off(int t) { return (t / 9) * 100 + ((t / 3) % 3) * 10 + t % 3; }

// colour-split index -> natural cell index (k*8 + j)*8 + i
__device__ __forceinline__ int cs_to_nat(int e) {
    int c = e >> 8, r = e & 255, m = r & 3, j = (r >> 2) & 7, k = r >> 5;
    int i = 2 * m + ((j + k + c) & 1);
    return (k * 8 + j) * 8 + i;
}
__device__ __forceinline__ int cs_idx(int i, int j, int k) {
    return (((i + j + k) & 1) << 8) + ((k * 8 + j) << 2) + (i >> 1);
}

template <typename T>
__device__ __forceinline__ T block_sum256(T v, T *S) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    int t = threadIdx.x;
    __syncthreads();
    if ((t & 63) == 0) S[t >> 6] = v;
    __syncthreads();
    return (S[0] + S[1]) + (S[2] + S[3]);
}

// ------------------------------------------------------------ weight packing
// Fragments in the lane order of the MFMA B operand (lane l holds column
// l % 16, K rows 8 (l / 16) .. +7 for 16x16x32, 4 (l / 16) .. +3 for 16x16x16).
__global__ __launch_bounds__(256) void k_nn_pack(const float *__restrict__ prm, uint16_t *__restrict__ pk) {
    for (int e = threadIdx.x; e < kNnPacked; e += 256) {
        float v = 0.0f;
        if (e < kP2) {
            int lane = e >> 3, q = e & 7, o = lane & 15, g = lane >> 4, t = 8 * g + q;
            if (t < 27) v = prm[kW1 + o * 27 + t];
        } else if (e < kP3) {
            // fragment f = (2 dk + type) 3 + di: type 0 has kernel rows dj = 0
            // in K groups 0-1 and dj = 1 in groups 2-3, type 1 dj = 2 in
            // groups 0-1 and zeros in 2-3
            int e2 = e - kP2, f = e2 >> 9, r = e2 & 511, lane = r >> 3, q = r & 7;
            int dk = f / 6, type = (f / 3) & 1, di = f % 3, o = lane & 15, g = lane >> 4, ch = 8 * (g & 1) + q;
            int dj = type == 0 ? (g < 2 ? 0 : 1) : (g < 2 ? 2 : -1);
            if (dj >= 0) v = prm[kW2 + (o * 16 + ch) * 27 + (dk * 3 + dj) * 3 + di];
        } else {
            int e3 = e - kP3, nt = e3 >> 8, r = e3 & 255, lane = r >> 2, q = r & 3;
            int n = lane & 15, g = lane >> 4, tap = 16 * nt + n, ch = 4 * g + q;
            if (tap < 27) v = prm[kW3 + ch * 27 + tap];
        }
        pk[e] = f2bf(v);
    }
}

// ------------------------------------------------------------------ forward
// x [nbox][1000] FP32 (10^3, x fastest), y [nbox][512] FP32 (natural order).
// idx (optional) maps output position q to input box idx[q].  SAVE stores a1
// and a2 (BF16, [nbox][16][512]) for training.
//
// Persistent workgroups of 4 waves: the weight fragments stay in registers
// while a workgroup walks over boxes q = blockIdx.x, + gridDim.x, ..., and
// each thread prefetches its part of the next box's input during the current
// box.  Tiles are 16 consecutive cells (two x-rows of 8), one MFMA row each.
//
// Layer 2 pairs the kernel rows within one z offset dk (dj = 0 with 1, and
// dj = 2 alone: 18 MFMAs per 16-cell tile, 27 taps in 32-wide K groups) so
// that a loaded input slice serves the three output slices it reaches: each
// wave walks the z-slices of its y-rows and loads every input fragment once
// (6 per slice), instead of once per output tile (15 per tile).  The
// x-shifted operands are loaded from A1 one cell to either side; its zero
// padding supplies the "same" convolution's zeros at the ends of the x-rows
// (moving one fragment across lanes with DPP row shifts instead costs 16
// vector instructions per pair for the shifts and row-end masks, which
// bounded an earlier version).  A1's rows and the layer-3 partial sums are
// padded so that the 16 lanes of an MFMA column group address different
// LDS banks.  Activations are rounded to BF16 (nearest even) by the
// hardware conversion.
constexpr int kFwdThreads = 256;  // 4 waves; 3 workgroups per CU

template <bool SAVE>
__global__ __launch_bounds__(kFwdThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_nn_fwd(const float *__restrict__ x, float *__restrict__ y,
                                                        const int32_t *__restrict__ idx, int64_t nbox,
                                                        const uint16_t *__restrict__ pk,
                                                        const float *__restrict__ prm,
                                                        uint16_t *__restrict__ a1o,
                                                        uint16_t *__restrict__ a2o) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[1008];
    // A1 [1000][16] BF16 (32000 bytes), later one half of Q, [16][kQs] FP32
    // (rows padded from 512 to kQs floats: the 16 lanes that store one MFMA
    // result column each write a different row, which then start in
    // different LDS banks)
    constexpr int kQs = 516;
    // A1 layout (u16 units): padded cell (x, y, z) at z*kA1z + y*kA1y + x*16,
    // each y-row 10 cells + 16 bytes, so that the two x-rows of a 16-cell
    // tile start in different LDS banks
    constexpr int kA1y = 168, kA1z = 10 * kA1y, kA1 = 10 * kA1z;
    constexpr int kR = (16 * kQs > kA1 / 2 ? 16 * kQs : kA1 / 2) / 4;
    __shared__ __attribute__((aligned(16))) uint4 R[kR];
    __shared__ __attribute__((aligned(16))) uint16_t A2[512 * 16];
    uint16_t *A1 = reinterpret_cast<uint16_t *>(R);
    float *Q = reinterpret_cast<float *>(R);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, row = lane & 15, g = lane >> 4;
    const int o = lane & 15;
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};

    // ---- weights, once per workgroup
    const bf16x8 B1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(pk + kP1 + lane * 8));
    bf16x8 B2[18];
#pragma unroll
    for (int f = 0; f < 18; f++)
        B2[f] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(pk + kP2 + (f * 64 + lane) * 8));
    s16x4 B3[2];
#pragma unroll
    for (int nt = 0; nt < 2; nt++) B3[nt] = *reinterpret_cast<const s16x4 *>(pk + kP3 + (nt * 64 + lane) * 4);
    const float bias1 = prm[kB1 + o], bias2 = prm[kB2 + o], b3 = prm[kB3];
    int off1[8];  // layer-1 taps of this lane's K group (-1: padding tap 27-31)
#pragma unroll
    for (int qq = 0; qq < 8; qq++) {
        int tp = 8 * g + qq;
        off1[qq] = tp < 27 ? tap_off(tp) : -1;
    }
    // layer 3: which of the 27 taps of this thread's two output cells lie
    // inside the box (the same for every box)
    uint32_t inside[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int c = t + 256 * h, ci = c & 7, cj = (c >> 3) & 7, ck = c >> 6;
        uint32_t msk = 0;
        for (int tp = 0; tp < 27; tp++) {
            int ii = ci + tp % 3 - 1, jj = cj + (tp / 3) % 3 - 1, kk = ck + tp / 9 - 1;
            if ((unsigned)ii < 8u && (unsigned)jj < 8u && (unsigned)kk < 8u) msk |= 1u << tp;
        }
        inside[h] = msk;
    }
    int64_t q = blockIdx.x;
    float xn[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (q < nbox) {
        const float *xb = x + (idx ? (int64_t)idx[q] : q) * 1000;
#pragma unroll
        for (int h = 0; h < 4; h++)
            if (t + 256 * h < 1000) xn[h] = xb[t + 256 * h];
    }
    for (; q < nbox; q += gridDim.x) {
        __syncthreads();  // the previous box is done with every LDS buffer
        // zero A1 (its padding must be 0; Q of the previous box overwrote it)
        for (int e = t; e < kA1 / 8; e += kFwdThreads) R[e] = make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int h = 0; h < 4; h++)
            if (t + 256 * h < 1000) xs[t + 256 * h] = f2bf_hw(xn[h]);
        const int64_t qn = q + gridDim.x;
        if (qn < nbox) {
            const float *xb = x + (idx ? (int64_t)idx[qn] : qn) * 1000;
#pragma unroll
            for (int h = 0; h < 4; h++)
                if (t + 256 * h < 1000) xn[h] = xb[t + 256 * h];
        }
        __syncthreads();
        // ---- layer 1: K = 27 taps (padded to 32) of the input
#pragma unroll 1
        for (int mm = 0; mm < 8; mm++) {
            const int m = w + 4 * mm;
            int cell = 16 * m + row, i = cell & 7, j = (cell >> 3) & 7, k = cell >> 6;
            int base = (k * 10 + j) * 10 + i;
            uint32_t wv[4];
#pragma unroll
            for (int h = 0; h < 4; h++) {
                uint32_t lo = off1[2 * h] >= 0 ? xs[base + off1[2 * h]] : 0u;
                uint32_t hi = off1[2 * h + 1] >= 0 ? xs[base + off1[2 * h + 1]] : 0u;
                wv[h] = lo | (hi << 16);
            }
            bf16x8 A = __builtin_bit_cast(bf16x8, make_uint4(wv[0], wv[1], wv[2], wv[3]));
            f32x4 D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B1, zero, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                int c = 16 * m + 4 * g + r, pi = c & 7, pj = (c >> 3) & 7, pk3 = c >> 6;
                A1[(pk3 + 1) * kA1z + (pj + 1) * kA1y + (pi + 1) * 16 + o] = f2bf_hw(relu(D[r] + bias1));
            }
        }
        __syncthreads();
        if (SAVE)  // a1 for training, [box][channel][cell]
            for (int e = t; e < 8192; e += kFwdThreads) {
                int ch = e >> 9, c = e & 511;
                a1o[(q * 16 + ch) * 512 + c] =
                    A1[((c >> 6) + 1) * kA1z + (((c >> 3) & 7) + 1) * kA1y + ((c & 7) + 1) * 16 + ch];
            }
        // ---- layer 2, blocked along z: wave w owns the output tiles of
        // y-rows (2w, 2w+1) at every z.  Each padded input slice zs is loaded
        // once (per x-shift di: the kernel rows dj = 0 | 1 in K groups 0-1 |
        // 2-3, and dj = 2 | nothing) and feeds the three output slices
        // k = zs - dk it reaches; an output slice is complete after its
        // input slice k + 2.  The x-shifted operands come from the
        // zero-padded A1 one cell to either side.
        {
            const int i = row & 7, jj = 2 * w + (row >> 3);
            const int colA = (g < 2 ? 0 : 1) * kA1y, colB = 2 * kA1y;  // kernel row dj of each K group
            f32x4 acc[3] = {zero, zero, zero};
#pragma unroll
            for (int zs = 0; zs < 10; zs++) {
                const uint16_t *src = A1 + zs * kA1z + jj * kA1y + i * 16 + 8 * (g & 1);
                uint4 FA[3], FB[3];
#pragma unroll
                for (int di = 0; di < 3; di++) {
                    FA[di] = *reinterpret_cast<const uint4 *>(src + colA + di * 16);
                    FB[di] = g < 2 ? *reinterpret_cast<const uint4 *>(src + colB + di * 16) : make_uint4(0, 0, 0, 0);
                }
#pragma unroll
                for (int dk = 0; dk < 3; dk++) {
                    const int k = zs - dk;
                    if (k < 0 || k > 7) continue;
#pragma unroll
                    for (int di = 0; di < 3; di++) {
                        acc[k % 3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, FA[di]), B2[(dk * 2 + 0) * 3 + di], acc[k % 3], 0, 0, 0);
                        acc[k % 3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, FB[di]), B2[(dk * 2 + 1) * 3 + di], acc[k % 3], 0, 0, 0);
                    }
                }
                const int kd = zs - 2;  // the output slice completed by this input slice
                if (kd >= 0) {
                    const int m = 4 * kd + w;
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        int c = 16 * m + 4 * g + r;
                        A2[c * 16 + o] = f2bf_hw(relu(acc[kd % 3][r] + bias2));
                    }
                    acc[kd % 3] = zero;
                }
            }
        }
        __syncthreads();  // A1 is dead; its space holds Q from here on
        if (SAVE)  // a2 for training, [box][channel][cell]
            for (int e = t; e < 8192; e += kFwdThreads) {
                int ch = e >> 9, c = e & 511;
                a2o[(q * 16 + ch) * 512 + c] = A2[c * 16 + ch];
            }
        // ---- layer 3: Q[tap][cell] = sum_c W3[c][tap] a2[c][cell], taps
        // 0-15 now and 16-26 after the first half of the sum
#pragma unroll 2
        for (int mm = 0; mm < 8; mm++) {
            const int m = w + 4 * mm;
            int cell = 16 * m + row;
            s16x4 A = *reinterpret_cast<const s16x4 *>(A2 + cell * 16 + 4 * g);
            f32x4 D = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B3[0], zero, 0, 0, 0);
            *reinterpret_cast<f32x4 *>(Q + o * kQs + 16 * m + 4 * g) = D;
        }
        __syncthreads();
        float s[2];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int c = t + 256 * h;
            s[h] = b3;
#pragma unroll
            for (int tp = 0; tp < 16; tp++)
                if ((inside[h] >> tp) & 1u) s[h] += Q[tp * kQs + c + (tp / 9 - 1) * 64 + ((tp / 3) % 3 - 1) * 8 + tp % 3 - 1];
        }
        __syncthreads();
#pragma unroll 2
        for (int mm = 0; mm < 8; mm++) {
            const int m = w + 4 * mm;
            int cell = 16 * m + row;
            s16x4 A = *reinterpret_cast<const s16x4 *>(A2 + cell * 16 + 4 * g);
            f32x4 D = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B3[1], zero, 0, 0, 0);
            if (o < 11) *reinterpret_cast<f32x4 *>(Q + o * kQs + 16 * m + 4 * g) = D;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int c = t + 256 * h;
#pragma unroll
            for (int tp = 16; tp < 27; tp++)
                if ((inside[h] >> tp) & 1u)
                    s[h] += Q[(tp - 16) * kQs + c + (tp / 9 - 1) * 64 + ((tp / 3) % 3 - 1) * 8 + tp % 3 - 1];
            y[q * 512 + c] = s[h];
        }
    }
}

// ----------------------------------------------------------------- backward
// Loss = mean over boxes and cells of (y - target)^2; gy = 2 (y - target) / N.
// Per box: gz2 = (transposed conv of gy with W3) * [a2 > 0] and
// gz1 = (transposed conv of gz2 with W2) * [a1 > 0], with the BF16-rounded
// weights the forward used.  Also the box's sum of squared errors.
__global__ __launch_bounds__(256) void k_nn_bwd_act(const float *__restrict__ y,
                                                    const float *__restrict__ tgt,
                                                    const int32_t *__restrict__ idx,
                                                    const uint16_t *__restrict__ a1o,
                                                    const uint16_t *__restrict__ a2o,
                                                    const float *__restrict__ prm, float scale2,
                                                    float *__restrict__ gz2o, float *__restrict__ gz1o,
                                                    double *__restrict__ lossp) {
    __shared__ float gyp[1000];
    __shared__ float W3s[432];
    __shared__ __attribute__((aligned(16))) float W2s[27 * 16 * 16];  // [tap][o][i]
    __shared__ float G2[16 * 1000];
    __shared__ double S[4];
    const int64_t q = blockIdx.x;
    const int64_t src = idx ? (int64_t)idx[q] : q;
    const int t = threadIdx.x;
    for (int e = t; e < 1000; e += 256) gyp[e] = 0.0f;
    for (int e = t; e < 16000; e += 256) G2[e] = 0.0f;
    for (int e = t; e < 432; e += 256) W3s[e] = round_bf(prm[kW3 + e]);
    for (int e = t; e < 6912; e += 256) {
        int tp = e % 27, oi = e / 27, o = oi >> 4, i = oi & 15;  // prm index (o*16 + i)*27 + tp
        W2s[(tp * 16 + o) * 16 + i] = round_bf(prm[kW2 + e]);
    }
    __syncthreads();
    double ls = 0.0;
    for (int c = t; c < 512; c += 256) {
        float d = y[q * 512 + c] - tgt[src * 512 + c];
        ls += (double)d * (double)d;
        int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
        gyp[((k + 1) * 10 + j + 1) * 10 + i + 1] = scale2 * d;
    }
    double tot = block_sum256(ls, S);
    if (t == 0) lossp[q] = tot;
    __syncthreads();
    for (int c = t; c < 512; c += 256) {
        int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
        float acc[16];
#pragma unroll
        for (int a = 0; a < 16; a++) acc[a] = 0.0f;
        for (int tp = 0; tp < 27; tp++) {
            int di = tp % 3, dj = (tp / 3) % 3, dk = tp / 9;
            float gv = gyp[((k - dk + 2) * 10 + j - dj + 2) * 10 + i - di + 2];
#pragma unroll
            for (int a = 0; a < 16; a++) acc[a] += W3s[a * 27 + tp] * gv;
        }
#pragma unroll
        for (int a = 0; a < 16; a++) {
            uint16_t bits = a2o[(q * 16 + a) * 512 + c];
            float g2 = (bits & 0x7fff) ? acc[a] : 0.0f;
            G2[a * 1000 + ((k + 1) * 10 + j + 1) * 10 + i + 1] = g2;
            gz2o[(q * 16 + a) * 512 + c] = g2;
        }
    }
    __syncthreads();
    for (int c = t; c < 512; c += 256) {
        int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
        float acc[16];
#pragma unroll
        for (int a = 0; a < 16; a++) acc[a] = 0.0f;
        for (int tp = 0; tp < 27; tp++) {
            int di = tp % 3, dj = (tp / 3) % 3, dk = tp / 9;
            int sidx = ((k - dk + 2) * 10 + j - dj + 2) * 10 + i - di + 2;
            for (int o = 0; o < 16; o++) {
                float gv = G2[o * 1000 + sidx];
                const float4 *wr = reinterpret_cast<const float4 *>(W2s + (tp * 16 + o) * 16);
#pragma unroll
                for (int v4 = 0; v4 < 4; v4++) {
                    float4 wv = wr[v4];
                    acc[4 * v4 + 0] += wv.x * gv;
                    acc[4 * v4 + 1] += wv.y * gv;
                    acc[4 * v4 + 2] += wv.z * gv;
                    acc[4 * v4 + 3] += wv.w * gv;
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 16; a++) {
            uint16_t bits = a1o[(q * 16 + a) * 512 + c];
            gz1o[(q * 16 + a) * 512 + c] = (bits & 0x7fff) ? acc[a] : 0.0f;
        }
    }
}

// Weight gradients: block r sums over boxes r, r + gridDim.x, ... and writes
// its partial gradient (parameter order) to part[r][kNnParams].
__global__ __launch_bounds__(256) void k_nn_wgrad(const float *__restrict__ x,
                                                  const float *__restrict__ y,
                                                  const float *__restrict__ tgt,
                                                  const int32_t *__restrict__ idx, int64_t nbox,
                                                  float scale2, const uint16_t *__restrict__ a1o,
                                                  const uint16_t *__restrict__ a2o,
                                                  const float *__restrict__ gz2o,
                                                  const float *__restrict__ gz1o,
                                                  float *__restrict__ part) {
    __shared__ uint16_t U[16 * 1000];  // a1 or a2, zero-padded 10^3 per channel
    __shared__ float V[16 * 512];      // gz2 or gz1
    __shared__ float X[1000];          // input (BF16-rounded) or gy
    const int t = threadIdx.x;
    const int o2 = t >> 4, c2 = t & 15;  // dW2 entry (o2, c2, all taps)
    float acc2[27];
#pragma unroll
    for (int tp = 0; tp < 27; tp++) acc2[tp] = 0.0f;
    float db2 = 0.0f, acc1[2] = {0.0f, 0.0f}, acc3[2] = {0.0f, 0.0f};
    for (int64_t q = blockIdx.x; q < nbox; q += gridDim.x) {
        const int64_t src = idx ? (int64_t)idx[q] : q;
        // ---- dW2, db2
        for (int e = t; e < 16000; e += 256) {
            int ch = e / 1000, p = e - ch * 1000, pi = p % 10, pj = (p / 10) % 10, pk = p / 100;
            uint16_t v = 0;
            if (pi >= 1 && pi <= 8 && pj >= 1 && pj <= 8 && pk >= 1 && pk <= 8)
                v = a1o[(q * 16 + ch) * 512 + ((pk - 1) * 8 + pj - 1) * 8 + pi - 1];
            U[e] = v;
        }
        for (int e = t; e < 8192; e += 256) V[e] = gz2o[q * 8192 + e];
        __syncthreads();
        for (int c = 0; c < 512; c++) {
            int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
            float gv = V[o2 * 512 + c];
            int base = c2 * 1000 + (k * 10 + j) * 10 + i;
#pragma unroll
            for (int tp = 0; tp < 27; tp++) acc2[tp] += gv * bf2f(U[base + tap_off(tp)]);
            db2 += gv;
        }
        __syncthreads();
        // ---- dW1, db1
        for (int e = t; e < 1000; e += 256) X[e] = round_bf(x[src * 1000 + e]);
        for (int e = t; e < 8192; e += 256) V[e] = gz1o[q * 8192 + e];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; s++) {
            int p = t + 256 * s;
            if (p < 432) {
                int o = p / 27, tp = p % 27, off = tap_off(tp);
                float a = 0.0f;
                for (int c = 0; c < 512; c++) {
                    int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
                    a += V[o * 512 + c] * X[(k * 10 + j) * 10 + i + off];
                }
                acc1[s] += a;
            } else if (p < 448) {
                float a = 0.0f;
                for (int c = 0; c < 512; c++) a += V[(p - 432) * 512 + c];
                acc1[s] += a;
            }
        }
        __syncthreads();
        // ---- dW3, db3
        for (int e = t; e < 16000; e += 256) {
            int ch = e / 1000, p = e - ch * 1000, pi = p % 10, pj = (p / 10) % 10, pk = p / 100;
            uint16_t v = 0;
            if (pi >= 1 && pi <= 8 && pj >= 1 && pj <= 8 && pk >= 1 && pk <= 8)
                v = a2o[(q * 16 + ch) * 512 + ((pk - 1) * 8 + pj - 1) * 8 + pi - 1];
            U[e] = v;
        }
        for (int c = t; c < 512; c += 256) X[c] = scale2 * (y[q * 512 + c] - tgt[src * 512 + c]);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; s++) {
            int p = t + 256 * s;
            if (p < 432) {
                int ch = p / 27, tp = p % 27, off = tap_off(tp);
                float a = 0.0f;
                for (int c = 0; c < 512; c++) {
                    int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
                    a += X[c] * bf2f(U[ch * 1000 + (k * 10 + j) * 10 + i + off]);
                }
                acc3[s] += a;
            } else if (p == 432) {
                float a = 0.0f;
                for (int c = 0; c < 512; c++) a += X[c];
                acc3[s] += a;
            }
        }
        __syncthreads();
    }
    float *pr = part + (int64_t)blockIdx.x * kNnParams;
#pragma unroll
    for (int tp = 0; tp < 27; tp++) pr[kW2 + (o2 * 16 + c2) * 27 + tp] = acc2[tp];
    if (c2 == 0) pr[kB2 + o2] = db2;
#pragma unroll
    for (int s = 0; s < 2; s++) {
        int p = t + 256 * s;
        if (p < 432) {
            pr[kW1 + p] = acc1[s];
            pr[kW3 + p] = acc3[s];
        } else if (p < 448) {
            pr[kB1 + p - 432] = acc1[s];
            if (p == 432) pr[kB3] = acc3[s];
        }
    }
}

// grad[p] = sum over blocks of part[block][p] (fixed order, FP64); block 0's
// thread 0 also writes the mean squared error.
__global__ __launch_bounds__(256) void k_nn_reduce(const float *__restrict__ part, int nblk,
                                                   const double *__restrict__ lossp, int64_t nbox,
                                                   float *__restrict__ grad, double *__restrict__ loss) {
    int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kNnParams) {
        double s = 0.0;
        for (int r = 0; r < nblk; r++) s += (double)part[(int64_t)r * kNnParams + p];
        grad[p] = (float)s;
    }
    if (blockIdx.x == 0) {
        __shared__ double S[4];
        double v = 0.0;
        for (int64_t b = threadIdx.x; b < nbox; b += 256) v += lossp[b];
        double tot = block_sum256(v, S);
        if (threadIdx.x == 0) *loss = tot / (512.0 * (double)nbox);
    }
}

__global__ __launch_bounds__(256) void k_nn_adam(float *__restrict__ p, float *__restrict__ m,
                                                 float *__restrict__ v, const float *__restrict__ g,
                                                 float lr, float b1, float b2, float eps, float bc1,
                                                 float bc2) {
    int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kNnParams) return;
    float gg = g[e];
    float mm = b1 * m[e] + (1.0f - b1) * gg;
    float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

// ------------------------------------------------------- learned tree step
// Network input of leaf position q: h^2 r on the box and on the face-ghost
// layers taken from same-level leaf neighbours (0 elsewhere), divided by the
// box's RMS of h^2 r (1 when that is 0).
__global__ __launch_bounds__(256) void k_nn_gather(const float *__restrict__ r32,
                                                   const int32_t *__restrict__ leaf,
                                                   const int32_t *__restrict__ nbr,
                                                   const int32_t *__restrict__ ijk4,
                                                   const int32_t *__restrict__ isleaf, double len,
                                                   float *__restrict__ x, float *__restrict__ scale) {
    __shared__ float X[1000];
    __shared__ double S[4];
    const int64_t q = blockIdx.x;
    const int64_t b = leaf[q];
    const int t = threadIdx.x;
    const int l = ijk4[b * 4 + 3];
    const double h = len / (8.0 * (double)(1 << (l - 1)));
    const float h2 = (float)(h * h);
    for (int e = t; e < 1000; e += 256) X[e] = 0.0f;
    __syncthreads();
    double ss = 0.0;
    for (int e = t; e < 512; e += 256) {
        int n = cs_to_nat(e), i = n & 7, j = (n >> 3) & 7, k = n >> 6;
        float v = h2 * r32[b * 512 + e];
        X[((k + 1) * 10 + j + 1) * 10 + i + 1] = v;
        ss += (double)v * (double)v;
    }
    for (int e = t; e < 384; e += 256) {
        int d = e >> 6, wv = e & 63, u = wv & 7, vv = wv >> 3;
        int nb = nbr[b * 6 + d];
        if (nb >= 0 && isleaf[nb]) {
            int a = d >> 1, side = d & 1, t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            int c[3], p[3];
            c[t1] = u;
            c[t2] = vv;
            c[a] = side ? 0 : 7;
            p[t1] = u + 1;
            p[t2] = vv + 1;
            p[a] = side ? 9 : 0;
            X[(p[2] * 10 + p[1]) * 10 + p[0]] = h2 * r32[(int64_t)nb * 512 + cs_idx(c[0], c[1], c[2])];
        }
    }
    double tot = block_sum256(ss, S);  // also orders the X writes before the reads below
    float rms = (float)sqrt(tot / 512.0);
    float sc = rms > 0.0f ? rms : 1.0f;
    for (int e = t; e < 1000; e += 256) x[q * 1000 + e] = X[e] / sc;
    if (t == 0) scale[q] = sc;
}

// e32 on leaf boxes <- scale * y (levels with level % 3 == mod3, or all when
// mod3 < 0; zero on the other leaf boxes).
__global__ __launch_bounds__(256) void k_nn_scatter(const float *__restrict__ y,
                                                    const float *__restrict__ scale,
                                                    const int32_t *__restrict__ leaf,
                                                    const int32_t *__restrict__ ijk4, int mod3,
                                                    float *__restrict__ e32) {
    const int64_t q = blockIdx.x;
    const int64_t b = leaf[q];
    const int l = ijk4[b * 4 + 3];
    const bool on = mod3 < 0 || l % 3 == mod3;
    const float sc = scale[q];
    for (int e = threadIdx.x; e < 512; e += 256)
        e32[b * 512 + e] = on ? sc * y[q * 512 + cs_to_nat(e)] : 0.0f;
}

// Per leaf position, with j its level and Q_m the operator applied to the
// correction of the levels = m (mod 3): the volume-weighted sums
// <r, q_{j-1}>, <r, q_j>, <r, q_{j+1}> and the six products of the q's.
__global__ __launch_bounds__(256) void k_nn_dots(const float *__restrict__ r32,
                                                 const float *__restrict__ q3,
                                                 const int32_t *__restrict__ leaf, int64_t nleaf,
                                                 const int32_t *__restrict__ ijk4, double len,
                                                 double *__restrict__ partial) {
    __shared__ double S[4];
    const int64_t q = blockIdx.x;
    const int64_t b = leaf[q];
    const int t = threadIdx.x;
    const int l = ijk4[b * 4 + 3];
    const double h = len / (8.0 * (double)(1 << (l - 1)));
    const float *qa = q3 + (int64_t)((l + 2) % 3) * nleaf * 512 + q * 512;
    const float *qc = q3 + (int64_t)(l % 3) * nleaf * 512 + q * 512;
    const float *qn = q3 + (int64_t)((l + 1) % 3) * nleaf * 512 + q * 512;
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = t; e < 512; e += 256) {
        double r = r32[b * 512 + e], a = qa[e], c = qc[e], n = qn[e];
        s[0] += r * a;
        s[1] += r * c;
        s[2] += r * n;
        s[3] += a * a;
        s[4] += a * c;
        s[5] += a * n;
        s[6] += c * c;
        s[7] += c * n;
        s[8] += n * n;
    }
    const double vol = h * h * h;
    for (int k = 0; k < 9; k++) {
        double v = block_sum256(s[k], S);
        if (t == 0) partial[q * 9 + k] = v * vol;
    }
}

// Per listed box: the volume-weighted sums <r, q> and <q, q> of one column
// (the per-level learned step).
__global__ __launch_bounds__(256) void k_nn_dots1(const float *__restrict__ r32, const float *__restrict__ q,
                                                  const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ ijk4, double len,
                                                  double *__restrict__ partial) {
    __shared__ double S[4];
    const int64_t p = blockIdx.x;
    const int64_t b = list[p];
    const int t = threadIdx.x;
    const int l = ijk4[b * 4 + 3];
    const double h = len / (8.0 * (double)(1 << (l - 1)));
    double rq = 0.0, qq = 0.0;
    for (int e = t; e < 512; e += 256) {
        double r = r32[b * 512 + e], c = q[p * 512 + e];
        rq += r * c;
        qq += c * c;
    }
    const double vol = h * h * h;
    double a = block_sum256(rq, S);
    double c = block_sum256(qq, S);
    if (t == 0) {
        partial[2 * p] = a * vol;
        partial[2 * p + 1] = c * vol;
    }
}

// phi += steps[tree][level] * (scale * y) on the leaf boxes (boxes whose
// step is 0 are left untouched, also where the correction is not finite).
__global__ __launch_bounds__(256) void k_nn_update(double *__restrict__ phi,
                                                   const float *__restrict__ y,
                                                   const float *__restrict__ scale,
                                                   const int32_t *__restrict__ leaf,
                                                   const int32_t *__restrict__ ijk4,
                                                   const int32_t *__restrict__ tid,
                                                   const double *__restrict__ steps, int stride) {
    const int64_t q = blockIdx.x;
    const int64_t b = leaf[q];
    const int l = ijk4[b * 4 + 3];
    const double st = steps[(int64_t)tid[b] * stride + l];
    const float sc = scale[q];
    if (st == 0.0) return;
    for (int e = threadIdx.x; e < 512; e += 256) {
        float c = sc * y[q * 512 + cs_to_nat(e)];
        phi[b * 512 + e] += st * (double)c;
    }
}

// Training target of leaf position q: (ref - phi) / scale in natural order,
// ref in natural order [n][512].
__global__ __launch_bounds__(256) void k_nn_targets(const double *__restrict__ phi,
                                                    const double *__restrict__ ref,
                                                    const float *__restrict__ scale,
                                                    const int32_t *__restrict__ leaf,
                                                    float *__restrict__ target) {
    const int64_t q = blockIdx.x;
    const int64_t b = leaf[q];
    const double sc = scale[q];
    for (int e = threadIdx.x; e < 512; e += 256) {
        int n = cs_to_nat(e);
        target[q * 512 + n] = (float)((ref[b * 512 + n] - phi[b * 512 + e]) / sc);
    }
}

}  // namespace

int64_t nn_train_layout(int64_t nbox, char *base, NnTrainWs *w) {
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        int64_t at = o;
        o += nn_align256(bytes);
        return at;
    };
    int64_t oy = take(4 * 512 * nbox), oa1 = take(2 * 8192 * nbox), oa2 = take(2 * 8192 * nbox);
    int64_t og2 = take(4 * 8192 * nbox), og1 = take(4 * 8192 * nbox), olp = take(8 * nbox);
    int64_t opart = take(4 * nn_wgrad_blocks(nbox) * kNnParams), oloss = take(8);
    if (base && w) {
        w->y = (float *)(base + oy);
        w->a1 = (uint16_t *)(base + oa1);
        w->a2 = (uint16_t *)(base + oa2);
        w->gz2 = (float *)(base + og2);
        w->gz1 = (float *)(base + og1);
        w->lossp = (double *)(base + olp);
        w->part = (float *)(base + opart);
        w->loss = (double *)(base + oloss);
    }
    return o;
}

void launch_nn_pack(const float *prm, uint16_t *pk, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_pack, dim3(1), dim3(256), 0, s, prm, pk);
}

void launch_nn_forward(const float *prm, const uint16_t *pk, int64_t nbox, const int32_t *idx,
                       const float *x, float *y, uint16_t *a1, uint16_t *a2, hipStream_t s) {
    if (nbox <= 0) return;
    unsigned grid = (unsigned)(nbox < kNnFwdBlocks ? nbox : kNnFwdBlocks);
    if (a1)
        hipLaunchKernelGGL(k_nn_fwd<true>, dim3(grid), dim3(kFwdThreads), 0, s, x, y, idx, nbox, pk, prm,
                           a1, a2);
    else
        hipLaunchKernelGGL(k_nn_fwd<false>, dim3(grid), dim3(kFwdThreads), 0, s, x, y, idx, nbox, pk, prm,
                           a1, a2);
}

void launch_nn_backward(const float *prm, int64_t nbox, const int32_t *idx, const float *x,
                        const float *target, const NnTrainWs &w, float *grad, hipStream_t s) {
    if (nbox <= 0) return;
    float scale2 = (float)(2.0 / (512.0 * (double)nbox));
    hipLaunchKernelGGL(k_nn_bwd_act, dim3((unsigned)nbox), dim3(256), 0, s, w.y, target, idx, w.a1,
                       w.a2, prm, scale2, w.gz2, w.gz1, w.lossp);
    int nblk = (int)nn_wgrad_blocks(nbox);
    hipLaunchKernelGGL(k_nn_wgrad, dim3((unsigned)nblk), dim3(256), 0, s, x, w.y, target, idx, nbox,
                       scale2, w.a1, w.a2, w.gz2, w.gz1, w.part);
    hipLaunchKernelGGL(k_nn_reduce, dim3((kNnParams + 255) / 256), dim3(256), 0, s, w.part, nblk,
                       w.lossp, nbox, grad, w.loss);
}

void launch_nn_adam(float *prm, float *m, float *v, const float *g, float lr, float b1, float b2,
                    float eps, float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_adam, dim3((kNnParams + 255) / 256), dim3(256), 0, s, prm, m, v, g, lr, b1,
                       b2, eps, bc1, bc2);
}

void launch_nn_gather(const float *r32, const int32_t *leaf, int64_t nleaf, const int32_t *nbr,
                      const int32_t *ijk4, const int32_t *isleaf, double len, float *x, float *scale,
                      hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_nn_gather, dim3((unsigned)nleaf), dim3(256), 0, s, r32, leaf, nbr, ijk4, isleaf,
                       len, x, scale);
}

void launch_nn_scatter(const float *y, const float *scale, const int32_t *leaf, int64_t nleaf,
                       const int32_t *ijk4, int mod3, float *e32, hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_nn_scatter, dim3((unsigned)nleaf), dim3(256), 0, s, y, scale, leaf, ijk4, mod3,
                       e32);
}

void launch_nn_dots(const float *r32, const float *q3, const int32_t *leaf, int64_t nleaf,
                    const int32_t *ijk4, double len, double *partial, hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_nn_dots, dim3((unsigned)nleaf), dim3(256), 0, s, r32, q3, leaf, nleaf, ijk4, len,
                       partial);
}

void launch_nn_dots1(const float *r32, const float *q, const int32_t *list, int64_t n, const int32_t *ijk4,
                     double len, double *partial, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_nn_dots1, dim3((unsigned)n), dim3(256), 0, s, r32, q, list, ijk4, len, partial);
}

void launch_nn_update(double *phi, const float *y, const float *scale, const int32_t *leaf,
                      int64_t nleaf, const int32_t *ijk4, const int32_t *tid, const double *steps,
                      int stride, hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_nn_update, dim3((unsigned)nleaf), dim3(256), 0, s, phi, y, scale, leaf, ijk4, tid,
                       steps, stride);
}

void launch_nn_targets(const double *phi, const double *ref, const float *scale,
                       const int32_t *leaf, int64_t nleaf, float *target, hipStream_t s) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_nn_targets, dim3((unsigned)nleaf), dim3(256), 0, s, phi, ref, scale, leaf,
                       target);
}

// ------------------------------------------------ allocation-free training
// The training buffers of mg_nn_gradient_static: one file-scope array, which
// every GPU the library runs on holds until the process ends.  In host code
// the name `scratch` is only a stand-in for the device address; the address
// on the current device comes from hipGetSymbolAddress, once per device.
__device__ __align__(256) char scratch[kNnStaticBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // device address of `scratch`, per device
}  // namespace

int nn_static_workspace(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return MG_EHIP;
        if (cur != device && hipSetDevice(device) != hipSuccess) return MG_EHIP;
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return MG_EHIP;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return MG_OK;
}

}  // namespace mg
