/*
 * lbm_cnn.h -- C ABI of the surrogate network and of the maps between
 * populations and coarse fields (same library as lbm.h).
 *
 * The surrogate advances the coarse density and momentum fields (rho, jx, jy)
 * of a lattice by a fixed number of lattice Boltzmann steps.  It is not part
 * of the paper's method; the lattice Boltzmann step (lbm.h) is its data
 * source and its judge.  Network: three 3x3 convolutions with circular
 * padding (periodic lattice), cin -> 32 -> 32 -> 3 channels, ReLU after the
 * first two, and a residual connection:
 *     y = x[:, 0:3] + conv3(relu(conv2(relu(conv1(x))))).
 * Tensors are NCHW float32 in device memory owned by the caller.  Weights
 * are stored as bfloat16 bits (uint16) [out][in][3][3]; products are taken
 * with the weights widened to float32 and summed in float32.  Biases are
 * float32.  Every call enqueues work on the caller's stream (hipStream_t
 * passed as void*) and never synchronises.  Errors as in lbm.h (LBM_EINVAL
 * for bad shapes or null pointers, LBM_EHIP for runtime errors; message in
 * lbm_last_error()).
 */
#ifndef LBM_CNN_H
#define LBM_CNN_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_cnn_shape {
    int32_t n;       /* samples (<= 65535) */
    int32_t cin;     /* input channels, 3..32 (the first three are the fields) */
    int32_t hidden;  /* hidden channels: must be 32 */
    int32_t cout;    /* output channels: must be 3 */
    int32_t h, w;    /* coarse field size (periodic) */
} lbm_cnn_shape;

typedef struct lbm_cnn_params {
    const uint16_t *w[3]; /* bf16 weights [hidden][cin][3][3], [hidden][hidden][3][3], [cout][hidden][3][3] */
    const float *b[3];    /* biases [hidden], [hidden], [cout] */
} lbm_cnn_params;

typedef struct lbm_cnn_grads {
    float *w[3]; /* float32, shapes of lbm_cnn_params.w */
    float *b[3];
} lbm_cnn_grads;

/* Device workspace bytes of lbm_cnn_forward / lbm_cnn_backward (0 if the shape
 * is invalid). */
size_t lbm_cnn_workspace_bytes(const lbm_cnn_shape *s);

/* Forward pass.  x [n][cin][h][w]; a1, a2 [n][32][h][w] receive the hidden
 * activations (after ReLU, kept for the backward pass); y [n][3][h][w]. */
int32_t lbm_cnn_forward(const lbm_cnn_shape *s, const lbm_cnn_params *p, const float *x, float *a1, float *a2,
                        float *y, void *ws, size_t ws_bytes, void *stream);

/* Loss and gradients of the mean squared error mean((y - target)^2) for the
 * forward pass that produced a1, a2, y from x.  g receives the gradients
 * (overwritten); loss is one device float. */
int32_t lbm_cnn_backward(const lbm_cnn_shape *s, const lbm_cnn_params *p, const float *x, const float *a1,
                         const float *a2, const float *y, const float *target, const lbm_cnn_grads *g,
                         float *loss, void *ws, size_t ws_bytes, void *stream);

/* One Adam step (Kingma & Ba, algorithm 1) at step t >= 1 on a float32 master
 * tensor theta[count] with moments m, v and gradient grad; with bf16_out the
 * updated theta is also written as bfloat16 (round to nearest even). */
int32_t lbm_cnn_adam(float *theta, float *m, float *v, const float *grad, int64_t count, float lr, float beta1,
                     float beta2, float eps, int64_t t, uint16_t *bf16_out, void *stream);

/* In place x[i][ch][..] = x[i][ch][..] * scale[ch] + shift[ch] for the first
 * nc of c channels of n samples of hw pixels (normalisation of the fields). */
int32_t lbm_channel_affine(float *x, int32_t n, int32_t c, int32_t nc, int64_t hw, const float *scale,
                           const float *shift, void *stream);

/* Per-sample relative L2 error of the first nc of c channels (n samples of
 * hw pixels): out[s] = |a_s - b_s| / |b_s| in float64 (device array of n). */
int32_t lbm_field_error(const float *a, const float *b, int32_t n, int32_t c, int32_t nc, int64_t hw, double *out,
                        void *stream);

/* Per-channel mean and standard deviation (population) of x [n][c][hw] in
 * float64 (device arrays of c), summed in a fixed order over many blocks per
 * channel.  ws: device workspace of lbm_channel_stats_workspace_bytes(c). */
size_t lbm_channel_stats_workspace_bytes(int32_t c);
int32_t lbm_channel_stats(const float *x, int32_t n, int32_t c, int64_t hw, double *mean, double *stdev, void *ws,
                          size_t ws_bytes, void *stream);

/* x[s][ch][:] = values[s] for s < n (device array of n floats). */
int32_t lbm_fill_channel(float *x, int32_t n, int32_t c, int32_t ch, int64_t hw, const float *values, void *stream);

/* Coarse fields of a stored F32 state f [7][ny][nx] (pitch nx): out
 * [3][ny/c][nx/c] = means over c x c blocks of sites of rho, jx, jy of the
 * streamed populations.  c divides nx and ny and is 1 or even. */
int32_t lbm_coarsen(const lbm_params *p, const float *f, int32_t c, float *out, void *stream);

/* Stored F32 state f [7][ny][nx] from coarse fields [3][ny/c][nx/c]: every
 * site of a block gets xi(rho, j/rho) of its block (steady state eq.
 * fssD2Q7 with u* = u; negative rho is treated as 0). */
int32_t lbm_lift(const lbm_params *p, const float *coarse, int32_t c, float *f, void *stream);

/* lbm_coarsen / lbm_lift for n lattices of the shape p in one launch.  bufs:
 * device array of n pointers to the lattices' stored F32 states; the coarse
 * fields of lattice l start at out + l * out_stride (resp. coarse + l *
 * in_stride), strides in floats, >= 3 (ny/c) (nx/c). */
int32_t lbm_coarsen_many(const lbm_params *p, int32_t n, const float *const *bufs, int32_t c, float *out,
                         int64_t out_stride, void *stream);
int32_t lbm_lift_many(const lbm_params *p, int32_t n, const float *coarse, int64_t in_stride, int32_t c,
                      float *const *bufs, void *stream);

/* ------------------------------------------------------------------------
 * The surrogate as one object: a host handle over a caller-owned parameter
 * block (float32 master weights and biases, Adam moments, bfloat16 weight
 * copies, the field normalisation) and a caller-owned workspace
 * (activations, gradients, a sweep's coarse fields).  Fields are
 * [n][cin][h][w] float32: rho, jx, jy, then (cin = 4) a constant channel
 * (the lattice's activity B in a sweep).  The network sees (x - mean) / std
 * per channel and its three outputs are mapped back by std and mean.  Work
 * is enqueued on the handle's stream; lbm_surrogate_create (with init) and
 * lbm_surrogate_destroy synchronise it.
 * ---------------------------------------------------------------------- */
typedef struct lbm_surrogate lbm_surrogate;

typedef struct lbm_surrogate_desc {
    int32_t cin;       /* input channels, 3 or 4 */
    int32_t h, w;      /* coarse grid (h * w <= 2^20) */
    int32_t coarse;    /* lattice sites per coarse cell side (1 or even) */
    int32_t k;         /* lattice Boltzmann steps one evaluation advances */
    int32_t max_batch; /* most samples per call (and lattices per sweep), <= 65535 */
} lbm_surrogate_desc;

/* Bytes of the parameter block / workspace (0 for an invalid description). */
size_t lbm_surrogate_param_bytes(const lbm_surrogate_desc *d);
size_t lbm_surrogate_workspace_bytes(const lbm_surrogate_desc *d);

/* A handle over params (256-byte aligned, lbm_surrogate_param_bytes) and ws
 * (256-byte aligned, ws_bytes >= lbm_surrogate_workspace_bytes), both
 * caller-owned and kept alive until lbm_surrogate_destroy.  init != 0 fills
 * params: He-uniform weights from seed (a tenth on the output layer), zero
 * biases and moments, identity normalisation; init == 0 takes params as they
 * are (e.g. a trained block).  The Adam step count starts at 0. */
int32_t lbm_surrogate_create(const lbm_surrogate_desc *d, void *params, int32_t init, uint64_t seed, void *ws,
                             size_t ws_bytes, void *stream, lbm_surrogate **out);

/* Normalisation from the per-channel mean and standard deviation of n
 * samples x (float64 statistics). */
int32_t lbm_surrogate_fit_normalisation(lbm_surrogate *s, const float *x, int32_t n);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) on the mean
 * squared error of the normalised output against the normalised target
 * fields, over the samples idx[0..n) of x and target (device int32 array;
 * NULL: the first n).  x and target are [N][cin][h][w] (only the first three
 * target channels are used), n <= max_batch.  loss: NULL or one device float
 * receiving this step's loss. */
int32_t lbm_surrogate_train_step(lbm_surrogate *s, const float *x, const float *target, const int32_t *idx,
                                 int32_t n, float lr, float *loss);

/* y [n][cin][h][w] = the network's fields k steps after x (channels 0..2)
 * and x's constant channels; n <= max_batch, y != x. */
int32_t lbm_surrogate_predict(lbm_surrogate *s, const float *x, int32_t n, float *y);

/* Where the tensors of a surrogate's parameter block are (device pointers
 * into it), for checkpoints and inspection: the float32 masters theta (w1,
 * b1, w2, b2, w3, b3, shapes as in lbm_cnn_params), their Adam moments, the
 * bfloat16 weight copies the network computes with (a caller that writes
 * theta must write these too), and norm = [4][cin]: input scale, input
 * shift, output scale, output shift. */
typedef struct lbm_surrogate_view {
    float *theta[6];
    float *m[6];
    float *v[6];
    int64_t count[6];
    uint16_t *w_bf16[3];
    float *norm;
    int64_t adam_steps; /* Adam steps taken by this handle */
} lbm_surrogate_view;

int32_t lbm_surrogate_view_of(const lbm_surrogate *s, lbm_surrogate_view *v);

/* Release the handle (after its stream's work). */
int32_t lbm_surrogate_destroy(lbm_surrogate *s);

#ifdef __cplusplus
}
#endif
#endif /* LBM_CNN_H */
