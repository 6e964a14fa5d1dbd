// Learned correction network: device state and launchers (kernels in nn.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace mg {

constexpr int kNnParams = 7809;   // 16*27 + 16 + 16*16*27 + 16 + 16*27 + 1
constexpr int kNnPacked = 10240;  // BF16 MFMA operand fragments of the weights
constexpr int kNnFwdBlocks = 768; // persistent forward workgroups (3 per CU)
constexpr int kNnWgradBlocks = 512;

constexpr int64_t nn_align256(int64_t bytes) { return (bytes + 255) & ~(int64_t)255; }
// Weight-gradient workgroups (one per box up to kNnWgradBlocks)
constexpr int64_t nn_wgrad_blocks(int64_t nbox) { return nbox < kNnWgradBlocks ? nbox : kNnWgradBlocks; }
// Bytes of the training buffers for nbox boxes (the layout of nn_train_layout)
constexpr int64_t nn_train_bytes_of(int64_t nbox) {
    return nn_align256(4 * 512 * nbox) + 2 * nn_align256(2 * 8192 * nbox) + 2 * nn_align256(4 * 8192 * nbox) +
           nn_align256(8 * nbox) + nn_align256(4 * nn_wgrad_blocks(nbox) * kNnParams) + nn_align256(8);
}
// Allocation-free training (mg_nn_gradient_static): the largest batch and the
// size of the file-scope device array that holds its buffers.
constexpr int64_t kNnStaticBoxes = 64;
constexpr int64_t kNnStaticBytes = nn_train_bytes_of(kNnStaticBoxes);
// Device address of that array on `device` (looked up once per device).
int nn_static_workspace(int device, void **out);

// Per-box training buffers (the caller's workspace), see nn_train_layout.
struct NnTrainWs {
    float *y, *gz1, *gz2, *part;
    uint16_t *a1, *a2;
    double *lossp, *loss;
};
int64_t nn_train_layout(int64_t nbox, char *base, NnTrainWs *w);

void launch_nn_pack(const float *prm, uint16_t *pk, hipStream_t s);
void launch_nn_forward(const float *prm, const uint16_t *pk, int64_t nbox, const int32_t *idx,
                       const float *x, float *y, uint16_t *a1, uint16_t *a2, hipStream_t s);
void launch_nn_backward(const float *prm, int64_t nbox, const int32_t *idx, const float *x,
                        const float *target, const NnTrainWs &w, float *grad, hipStream_t s);
void launch_nn_adam(float *prm, float *m, float *v, const float *g, float lr, float b1, float b2,
                    float eps, float bc1, float bc2, hipStream_t s);

// Learned step on a tree (leaf boxes in leaf-list order, fields colour-split).
void launch_nn_gather(const float *r32, const int32_t *leaf, int64_t nleaf, const int32_t *nbr,
                      const int32_t *ijk4, const int32_t *isleaf, double len, float *x, float *scale,
                      hipStream_t s);
void launch_nn_scatter(const float *y, const float *scale, const int32_t *leaf, int64_t nleaf,
                       const int32_t *ijk4, int mod3, float *e32, hipStream_t s);
void launch_nn_dots(const float *r32, const float *q3, const int32_t *leaf, int64_t nleaf,
                    const int32_t *ijk4, double len, double *partial, hipStream_t s);
void launch_nn_dots1(const float *r32, const float *q, const int32_t *list, int64_t n, const int32_t *ijk4,
                     double len, double *partial, hipStream_t s);
void launch_nn_update(double *phi, const float *y, const float *scale, const int32_t *leaf,
                      int64_t nleaf, const int32_t *ijk4, const int32_t *tid, const double *steps,
                      int stride, hipStream_t s);
void launch_nn_targets(const double *phi, const double *ref, const float *scale,
                       const int32_t *leaf, int64_t nleaf, float *target, hipStream_t s);

}  // namespace mg

// The network object behind the C ABI: FP32 master parameters, Adam moments,
// packed BF16 operand fragments and a gradient buffer, in the caller's
// device memory.
struct mg_nn {
    float *prm = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *pk = nullptr;
    void *stream = nullptr;       // stream of the standalone calls
    double *host_loss = nullptr;  // pinned
    int64_t step = 0;
    int device = 0;
};
