/* Spectrum surrogate: a small multilayer perceptron that maps (log10 q, eta)
 * of the two-field preheating model to the binned field power spectrum the
 * lattice produces (Sec. 3.1 spectra of the preheating model of Sec. 8.1.1), trained on
 * the GPU on spectra the lattice itself generated.
 *
 * Network: 2 inputs -> 24 fixed features -> 256 -> 256 -> 256 -> 64, exact
 * (erf) GELU after each hidden layer, linear output, mean-squared-error loss,
 * Adam.  FP32 master weights; the matrix products run on the matrix cores
 * with BF16 operands and FP32 accumulation.  BF16 (round to nearest even) is
 * applied to: the weights fed to the products, the hidden activations
 * h1..h3, the output gradient and the hidden pre-activation gradients of
 * layers 3 and 2.  Biases, pre-activations, the features, the first layer
 * (K = 24, plain FMA) and all gradient sums stay FP32.
 *
 * Inputs and outputs are normalised inside the library:
 *   x_n = (x - in_shift) * in_scale,  y = y_n / out_scale + out_shift,
 *   target t_n = (t - out_shift) * out_scale.
 * The features of a row are the two normalised inputs followed by a Fourier
 * encoding of each: for input c and octave k = 0 .. SURR_N_FREQ_c - 1,
 *   sin(2^k enc_freq[c] x_n,c), cos(2^k enc_freq[c] x_n,c),
 * input 0's pairs first.  The encoding lets the first layer resolve the
 * resonance bands of the spectrum in q and its oscillation in eta, which a
 * plain MLP of this size smooths over.
 *
 * Conventions are those of cosmolat.h: 0 on success, negative LAT_* codes on
 * failure with the text in lattice_last_error(); the caller owns every
 * buffer (the device workspace is allocated by the caller, e.g. with torch);
 * all device work goes on the stream given at init; one handle per thread.
 */
#ifndef SURROGATE_H
#define SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "cosmolat.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SURR_N_IN 2
#define SURR_N_FREQ0 6      /* octaves of the encoding of input 0 (log10 q) */
#define SURR_N_FREQ1 5      /* octaves of the encoding of input 1 (eta) */
#define SURR_N_FEAT 24      /* SURR_N_IN + 2 (SURR_N_FREQ0 + SURR_N_FREQ1) */
#define SURR_WIDTH 256
#define SURR_N_OUT 64
#define SURR_NPARAMS 154432 /* 24*256+256 + 2*(256*256+256) + 256*64+64 */

typedef struct surrogate_t surrogate_t;

typedef struct surrogate_params {
  int32_t max_batch;        /* rows per training step: 64 .. 16384, multiple of 64 */
  int32_t reserved;         /* 0 */
  double beta1, beta2, eps; /* Adam moment decays and denominator offset */
  float in_shift[SURR_N_IN], in_scale[SURR_N_IN];
  float out_shift[SURR_N_OUT], out_scale[SURR_N_OUT];
  float enc_freq[SURR_N_IN]; /* base angular frequency of each input's encoding, finite */
} surrogate_params;

/* Device workspace bytes for p (weights, Adam moments, BF16 copies and the
 * activations of one training step).  Errors: LAT_EINVAL. */
int surrogate_workspace_size(const surrogate_params* p, size_t* bytes);

/* Validate p and bind the workspace and stream.  The weights are undefined
 * until surrogate_set_weights.  Errors: LAT_EINVAL, LAT_ENOMEM (ws_bytes too
 * small), LAT_EHIP. */
int surrogate_init(const surrogate_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
                   surrogate_t** out);

/* Load SURR_NPARAMS FP32 master weights from host memory, in this order:
 * W1[256][24], b1[256], W2[256][256], b2[256], W3[256][256], b3[256],
 * W4[64][256], b4[64] (W[out][in], a = W h + b).  Resets the Adam moments
 * and step count.  Synchronises the stream.  Errors: LAT_EINVAL, LAT_EHIP. */
int surrogate_set_weights(surrogate_t* h, const float* host_w);

/* Copy the FP32 master weights (same order) to host memory.  Synchronises. */
int surrogate_get_weights(surrogate_t* h, float* host_w);

/* Set the output normalisation from training targets: out_shift[c] = mean
 * of column c of dev_t (FP32 [n][64]), out_scale[c] = 1 / its standard
 * deviation (population, floored at 1e-6), both computed on the device in
 * FP64 (two passes).  host_shift, host_scale (64 doubles each, may be NULL)
 * receive the values.  Does not touch the weights.  Synchronises.
 * Errors: LAT_EINVAL (n < 2), LAT_ENONFINITE, LAT_EHIP. */
int surrogate_fit_output_scale(surrogate_t* h, const float* dev_t, int64_t n, double* host_shift,
                               double* host_scale);

/* Loss and gradient of one batch without an update.  Rows i = 0..n-1 of the
 * batch are rows rows[i] of dev_x (FP32 [*][2]) and dev_t (FP32 [*][64], raw
 * log10 spectra); rows == NULL means rows 0..n-1.  1 <= n <= max_batch.
 * dev_grad: device FP32 [SURR_NPARAMS], same order as the weights, of
 * L = mean over rows and outputs of (y_n - t_n)^2.  *loss receives L
 * (FP64).  Synchronises.  Errors: LAT_EINVAL, LAT_ENONFINITE, LAT_EHIP. */
int surrogate_loss_grad(surrogate_t* h, const float* dev_x, const float* dev_t, const int32_t* rows,
                        int32_t n, float* dev_grad, double* loss);

/* One pass over n samples in the order of dev_perm (device int32 [n]):
 * consecutive slices of max_batch rows (the last one may be shorter), each
 * followed by one Adam step with learning rate lr and the usual bias
 * correction.  At most 65536 steps per call.  *mean_loss receives the mean
 * of the per-step losses (before each update).  Synchronises.
 * Errors: LAT_EINVAL, LAT_ENONFINITE, LAT_EHIP. */
int surrogate_train_epoch(surrogate_t* h, const float* dev_x, const float* dev_t, const int32_t* dev_perm,
                          int64_t n, double lr, double* mean_loss);

/* Replay whole training epochs from a HIP graph (default on when the
 * handle's stream is a created stream, off on the null stream).  An epoch is
 * captured on the first call and replayed while dev_x, dev_t, dev_perm and n
 * are the same; refill the same perm buffer to reshuffle.  The learning rate
 * and the Adam step count live on the device, so a replay continues the run
 * exactly as eager launches would.  on = 0 launches every kernel directly.
 * Synchronises.  Errors: LAT_EINVAL (on with the null stream), LAT_EHIP. */
int surrogate_use_graph(surrogate_t* h, int on);

/* Forward pass for n query rows dev_x (FP32 [n][2], raw inputs) into dev_y (FP32
 * [n][64], denormalised log10 spectra), all layers fused in one kernel.
 * Asynchronous on the stream.  Errors: LAT_EINVAL, LAT_EHIP. */
int surrogate_predict(surrogate_t* h, const float* dev_x, int64_t n, float* dev_y);

/* Release the handle (not the workspace).  Synchronises the stream. */
int surrogate_destroy(surrogate_t* h);

#ifdef __cplusplus
}
#endif

#endif /* SURROGATE_H */
