/*
 * Learned surrogate of an HDMR sparse-grid model: a 4-layer BF16 MLP trained
 * and served by hand-written gfx950 kernels, with the interpolant as its
 * fallback and the reference its error is measured against.  Not part of
 * the paper; the paper observes that order-2 terms of its models are far
 * smaller than order-1 terms (Sec. 5), which is what the network learns
 * here: the order-2 residual F - (c0 + sum_{|S|=1} u_S), with the order-1
 * part always evaluated exactly.
 *
 * Network: d -> w -> w -> w -> m linear layers, GELU after the first three
 * (erf to 1.5e-7 in the forward pass, exact in the backward).  Weights: FP32
 * masters, BF16 copies for the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
 * accumulation); activations and gradients
 * stored in BF16 between layers.  Targets are standardised per output;
 * loss = mean squared error over (batch, output); Adam (0.9, 0.999, 1e-8)
 * with a cosine learning-rate decay.
 *
 * Parameters are packed as [W0, b0, W1, b1, W2, b2, W3, b3] in FP32, W_l
 * row-major (out x in).  Points X are n x d FP64 row-major on the device;
 * targets and outputs n x m FP64 row-major on the device.
 *
 * Conventions as in hdmr.h: 0 or a negative HDMR_E* code; the message of the
 * last failure from hdmr_last_error(); calls are asynchronous on the given
 * stream unless stated; the caller owns its buffers, the library owns the
 * objects until the matching *_free.  A network holds one batch workspace:
 * calls on the same network (and on routes that borrow it) must not overlap.
 */
#ifndef HDMR_SURROGATE_H
#define HDMR_SURROGATE_H

#include "hdmr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlp_model mlp_model;
typedef struct mlp_route mlp_route;

/* Number of packed parameters of a (d, width, m) network. */
int mlp_param_count(int32_t d, int32_t width, int32_t m, int64_t *count);

/* A network with the given packed FP32 parameters (host).  d, m in [1, 4096],
 * width in [16, 4096]; every dimension is padded to a multiple of 8 inside. */
int mlp_create(int32_t d, int32_t width, int32_t m, const float *params, mlp_model **out);

/* Copy the FP32 master parameters back to the host (synchronous). */
int mlp_get_params(const mlp_model *net, float *params);

/* Per-output target standardisation y_std = (y - mean) / stdev (host arrays
 * of m values, stdev > 0), required before training.  mlp_fit_standardization
 * sets them to the mean and standard deviation (floored at 1e-12) of the
 * targets Y (dev, n x m FP64, n >= 2). */
int mlp_set_standardization(mlp_model *net, const float *mean, const float *stdev);
int mlp_fit_standardization(mlp_model *net, const double *Y, int64_t n, hdmr_stream_t stream);
int mlp_get_standardization(const mlp_model *net, float *mean, float *stdev);

/* Network prediction in target units (de-standardised) at n points:
 * Y (dev, n x m FP64). */
int mlp_forward(const mlp_model *net, const double *X, int64_t n, double *Y, hdmr_stream_t stream);

/* Loss and gradient of one batch (diagnostic; synchronous): the rows idx
 * (dev, batch int64) of X and Y (raw targets); grads (host, packed like the
 * parameters) and *loss (host) receive the results.  The parameters are not
 * changed. */
int mlp_loss_grads(mlp_model *net, const double *X, const double *Y, const int64_t *idx, int32_t batch,
                   float *grads, float *loss, hdmr_stream_t stream);

/* steps Adam steps on batches order[s*batch .. (s+1)*batch) (dev int64
 * row indices into X and Y, e.g. seeded permutations drawn by the caller),
 * learning rate lr0 (1 + cos(pi s / steps)) / 2 at step s.  losses (host,
 * steps floats) receives every step's batch loss when non-NULL (synchronous
 * then).  Adam's step counter continues across calls. */
int mlp_train(mlp_model *net, const double *X, const double *Y, const int64_t *order, int64_t steps,
              int32_t batch, float lr0, float *losses, hdmr_stream_t stream);

void mlp_free(mlp_model *net);

/* A model holding the chosen components (comps, n_comps ids; NULL = all) and
 * output columns (outs, n_outs ids; NULL = all) of src, with c0 restricted to
 * those outputs when with_c0 != 0 and zero otherwise.  Built on the current
 * device. */
int hdmr_model_select(const hdmr_model *src, int32_t n_comps, const int32_t *comps, int32_t n_outs,
                      const int32_t *outs, int32_t with_c0, hdmr_model **out);

/* Per-output routing (synchronous): on the validation points Xval (dev,
 * nval x d) the order-2 residual of the interpolant `full` is compared with
 * the network's prediction; output o is served by the network (plus the
 * exact order-1 part) iff its max-abs error is <= threshold, else by the
 * interpolant.  The route borrows `net` and copies what it needs of `full`. */
int mlp_route_create(mlp_model *net, const hdmr_model *full, const double *Xval, int64_t nval, double threshold,
                     mlp_route **out);
/* *n_mlp = outputs served by the network; err (host m) = validated max-abs
 * error per output; use_mlp (host m) = 1 where the network serves.  Any
 * output pointer may be NULL. */
int mlp_route_info(const mlp_route *route, int32_t *n_mlp, double *err, int32_t *use_mlp);
/* Y (dev, n x m FP64) at X (dev, n x d): network outputs = order-1 part +
 * network residual; the others from the interpolant (precision as in
 * hdmr_eval). */
int mlp_eval_routed(const mlp_route *route, const double *X, int64_t n, double *Y, int32_t precision,
                    hdmr_stream_t stream);
void mlp_route_free(mlp_route *route);

/* Per-point gate of a route (the ensemble-disagreement reading of the
 * surrogate's fallback): with a second network trained on the same data, a
 * point whose two predictions differ by more than tau in any output the
 * network serves takes those outputs from the interpolant `full` instead (the
 * other outputs are routed as before).  second = NULL switches the gate off.
 * The route borrows `second`; calls on the route must not overlap.  A gated
 * mlp_eval_routed synchronises its stream once (the number of gated points
 * sizes the fallback evaluation); mlp_route_gated returns that number for
 * the last call. */
int mlp_route_set_gate(mlp_route *route, mlp_model *second, const hdmr_model *full, double tau);
int mlp_route_gated(const mlp_route *route, int64_t *n_gated);

#ifdef __cplusplus
}
#endif

#endif /* HDMR_SURROGATE_H */
