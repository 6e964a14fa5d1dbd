/*
 * mg_nn.h - C ABI of the learned correction step of the octree multigrid
 * solver (mg.h): a small 3-D convolutional network, trained on the device,
 * whose output on each leaf box is a correction applied between V-cycles
 * with least-squares step sizes.
 *
 * This extends the geometric multigrid of paper section 2.1.2 (red-black
 * Gauss-Seidel smoothing inside FMG / V-cycles) with a learned smoother in
 * the same place in the cycle: after the up-leg of a V-cycle.  The paper
 * does not define it; the definitions below are this library's.
 *
 * Network (one leaf box): input x[10][10][10] (k, j, i; x fastest), output
 * y[8][8][8] natural layout:
 *   a1 = relu(conv3x3x3_valid(x; W1, b1))           1 -> 16 channels
 *   a2 = relu(conv3x3x3_same(a1; W2, b2))          16 -> 16
 *   y  =      conv3x3x3_same(a2; W3, b3)           16 -> 1
 * where "same" pads with zeros.  x, the weights, a1 and a2 are rounded to
 * BF16 (round to nearest even); sums are accumulated in FP32.  Parameters
 * are FP32, MG_NN_PARAMS of them, in the order
 *   W1[16][27], b1[16], W2[16 out][16 in][27], b2[16], W3[16 in][27], b3[1]
 * with tap t = (dk*3 + dj)*3 + di for kernel offsets di, dj, dk in 0..2 and
 * conv(x)[cell] = sum_t W[t] x[cell + offset_t] (valid) or
 * x[cell + offset_t - 1] (same).
 *
 * Learned step on a tree, for the current phi:
 *   r    = b - L phi on the leaf cells (covered cells first reset to the
 *          mean of their children, as in the solver's stopping test);
 *   x    = network input of each leaf box: h^2 r on the box and, on each
 *          face-ghost layer, h^2 r of the adjacent same-level leaf box (0
 *          where the face neighbour is coarser, refined or outside the
 *          domain, and on the edges and corners of the 10^3 block), divided
 *          by the box's RMS of h^2 r (1 when that is 0);
 *   c    = scale * network(x) on each leaf box;
 *   q_l  = L0 c_l, the composite operator with homogeneous boundary data
 *          applied to c restricted to the leaf boxes of level l;
 *   s    = per tree, the step sizes s_l minimising the volume-weighted L2
 *          norm of r - sum_l s_l q_l over the tree's leaf cells (a level
 *          whose column vanishes gets 0);
 *   phi += sum_l s_l c_l.
 *
 * Conventions as in mg.h: device memory is the caller's; a tree's learned
 * calls run on the stream bound to the tree; leaf boxes are numbered in
 * canonical order restricted to leaves ("leaf position").  All functions
 * return MG_OK or a negative status code of mg.h and set mg_last_error().
 */
#ifndef MG_NN_H
#define MG_NN_H
#include <stdint.h>

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MG_NN_PARAMS 7809

typedef struct mg_nn mg_nn;

/* Bytes of device memory holding a network's state (parameters, Adam
 * moments, gradient, packed BF16 weights). */
int64_t mg_nn_state_bytes(void);

/*
 * mg_nn_create - a network on `state` (device, 256-byte aligned, at least
 * mg_nn_state_bytes(); owned by the caller and used until destroy), with
 * all parameters 0.  Standalone calls (set/get, forward, gradient, Adam)
 * run on `stream`.  MG_EINVAL on null or misaligned arguments, MG_ENOMEM
 * when state_bytes is too small, MG_EHIP on a HIP error.
 */
int mg_nn_create(mg_nn **out, void *state, int64_t state_bytes, void *stream);
int mg_nn_destroy(mg_nn *nn);

/* Host copies of the FP32 parameters ([MG_NN_PARAMS], order above).
 * Setting them resets the Adam moments and step count.  Both synchronise
 * the network's stream. */
int mg_nn_set_params(mg_nn *nn, const float *params);
int mg_nn_get_params(mg_nn *nn, float *params);

/* y[nbox][512] = network(x[nbox][1000]); device pointers, asynchronous. */
int mg_nn_forward(mg_nn *nn, int64_t nbox, const float *x, float *y);

/*
 * Training.  mg_nn_gradient computes the loss
 *   mean over boxes and cells of (network(x[idx[q]]) - target[idx[q]])^2
 * for q < nbox (idx: device int32, or NULL for the identity) and its
 * gradient with respect to the FP32 parameters (the BF16 rounding of the
 * weights taken as the identity; FP32 arithmetic on the vector units) into
 * the network's gradient buffer.  ws (device, 256-byte aligned) must hold
 * mg_nn_train_bytes(nbox) bytes.  loss (host) may be NULL; when given the
 * call synchronises the stream.  mg_nn_get_grad copies the gradient to the
 * host.  mg_nn_adam applies one Adam update (Kingma & Ba) to the
 * parameters from the gradient buffer (asynchronous).
 */
int64_t mg_nn_train_bytes(int64_t nbox);
int mg_nn_gradient(mg_nn *nn, int64_t nbox, const int32_t *idx, const float *x, const float *target,
                   void *ws, int64_t ws_bytes, double *loss);
int mg_nn_get_grad(mg_nn *nn, float *grad);

/*
 * mg_nn_gradient_static - mg_nn_gradient without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight training loops, harnesses that forbid hipMalloc).  It allocates
 * nothing: the training buffers are a file-scope device array of the library
 * (MG_NN_STATIC_BYTES bytes, held by every GPU the library runs on until the
 * process ends), whose address on the network's device is looked up on the
 * first call there.  nbox must be 1..MG_NN_STATIC_MAX_BOXES (MG_EINVAL
 * otherwise, with a message).  Every call on one GPU shares that GPU's array,
 * which keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other networks) race on it, so the caller serialises them.
 * Nothing in it needs to start at zero (every buffer is written before it is
 * read).  Results are those of mg_nn_gradient on the same arguments.
 */
#define MG_NN_STATIC_MAX_BOXES 64
#define MG_NN_STATIC_BYTES 8422400
int mg_nn_gradient_static(mg_nn *nn, int64_t nbox, const int32_t *idx, const float *x,
                          const float *target, double *loss);
typedef struct {
    double lr, beta1, beta2, eps;
} mg_adam_opts;
int mg_nn_adam(mg_nn *nn, const mg_adam_opts *o);

/*
 * Tree side.  mg_learned_bytes gives the workspace a learned call needs on
 * this tree (about 12.3 KB per leaf box).  mg_nn_inputs writes the network
 * inputs of every leaf box for the current phi (x: device float
 * [n_leaf_boxes][1000], scale: device float [n_leaf_boxes]); mg_nn_targets
 * writes (ref - phi) / scale per leaf box (ref: device double, natural
 * layout [n_boxes][512]; target: device float [n_leaf_boxes][512]).
 */
int64_t mg_learned_bytes(const mg_tree *t);
int mg_nn_inputs(mg_tree *t, float *x, float *scale);
int mg_nn_targets(mg_tree *t, const double *ref, const float *scale, float *target);

/*
 * mg_learned_step - one learned step on the current phi.  steps (host, may
 * be NULL) receives s as [n_trees][n_levels + 1] (index level; entry 0
 * unused).  Synchronises the tree's stream.
 */
int mg_learned_step(mg_tree *t, mg_nn *nn, void *ws, int64_t ws_bytes, double *steps);

/*
 * mg_learned_solve - as mg_fmg_solve (FP64 only; MG_EINVAL otherwise), but
 * every V-cycle whose residual check does not stop the solve is followed by
 * a learned step and a second check.  The step is kept while it lowers the
 * relative residual to at most 0.99 times its value after the V-cycle; the
 * first time it does not, phi is restored and the remaining cycles are
 * plain V-cycles (fallback).  n_vcycles counts V-cycles; rel_hist[k] is the
 * relative residual after cycle k including its learned step.
 */
/*
 * Per-level placement (mg_solve_opts.learned_placement = 1): inside every
 * V-cycle after the first, right after the up-sweeps of each level l >= 3
 * with leaf boxes, a learned step on that level alone:
 *   r    = b - L phi on the level's leaf boxes with the cycle's ghosts
 *          (covered cells as the cycle left them);
 *   x, c as above on those boxes (the same network);
 *   q    = L0 c with c zero off those boxes (homogeneous boundary data,
 *          zero coarse side at refinement boundaries);
 *   s    = per tree <r, q> / <q, q> over the level's leaf cells, 0 when not
 *          finite or not positive;  phi += s c.
 * The first V-cycle is plain and gives the plain residual factor; while a
 * cycle with the steps reduces the relative residual by at least that
 * factor it counts as accepted, and the first that does not makes the
 * remaining cycles plain (fallback; phi is kept).  These cycles launch
 * kernel by kernel (each step reads its sums back to the host).
 * mg_learned_level_step applies the step to one level of the current phi
 * (steps: host [n_trees], may be NULL); MG_EINVAL for a level outside
 * 3..n_levels.
 */
int mg_learned_level_step(mg_tree *t, mg_nn *nn, void *ws, int64_t ws_bytes, int level, double *steps);

typedef struct {
    int32_t accepted;       /* learned steps kept */
    int32_t fallback_cycle; /* cycle at which the step was dropped, 0 if never */
    double t_learned_ms;    /* host wall time spent in learned steps */
} mg_learned_stats;
int mg_learned_solve(mg_tree *t, mg_nn *nn, void *ws, int64_t ws_bytes, const mg_solve_opts *o,
                     mg_solve_stats *s, mg_learned_stats *ls);

/*
 * mg_nn_bind - attach a network and its learned-step workspace (as for
 * mg_learned_solve) to a tree, so that mg_fmg_solve with precision
 * MG_LEARNED runs that solve (its stats carry nn_accepted and nn_fell_back).
 * nn = NULL detaches.  Both stay owned by the caller and must outlive the
 * binding.  MG_EINVAL/MG_ENOMEM as mg_learned_solve checks them.
 */
int mg_nn_bind(mg_tree *t, mg_nn *nn, void *ws, int64_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif
