/* rmhd_mlp.h -- learned starting guess for the two-fluid implicit stage (C ABI).
 *
 * The implicit stage of Sec. 2.2.1 (Eq. 10) is solved per cell by Newton iteration on the
 * seven source-carrying unknowns x = (Sbar/|mu1|, taubar/|mu1|, E) of the two-fluid model
 * (Sec. 3, Eqs. 27-30); the paper only says that a guess is made.  This library's plain
 * guess is x0 = R_x, the unknowns of the stage's right-hand side R.  The learned guess is
 *
 *     x0 = R_x + D * y,   y = tmean + tstd * net((f - fmean) / fstd),
 *
 * with 19 per-cell features f of R:
 *     f0 = log10(a mu1^2 D), a = gamma dt;   f_k = R_k / D, k = 1..17;   f18 = log10(a sigma)
 * (conserved order D, S(3), tau, Dbar, Sbar(3), taubar, B(3), E(3), psi, phi), and
 *     net(u) = W3 tanh(W2 tanh(W1 u + b1) + b2) + b3,   W1: 64x19, W2: 64x64, W3: 7x64.
 * Training targets are y* = (x* - R_x) / D with x* the converged stage solution.  The stage
 * always finishes with the FP64 Newton iteration and its tolerance, so the learned guess
 * changes the iteration count, never the accepted solution's tolerance; a cell whose Newton
 * fails from the learned guess is solved again from the plain guess.
 *
 * Arithmetic: FP32 master weights, used rounded to bfloat16 (nearest, ties to even).
 * Inference (the guess inside a step, and rmhd_mlp_forward with precision 1) multiplies
 * bfloat16 weights by bfloat16 activations on the matrix cores and accumulates in FP32.
 * Training (gradient, Adam) and rmhd_mlp_forward with precision 0 use FP32 activations.
 * The loss is the mean over samples of the squared error summed over the 7 standardised
 * outputs; Adam uses beta1 = 0.9, beta2 = 0.999, eps = 1e-8 with bias correction.
 *
 * Parameter vector (RMHD_MLP_NPARAMS floats): W1, b1, W2, b2, W3, b3, each row-major.
 * Normalisation vector (RMHD_MLP_NNORM floats): fmean[19], fstd[19], tmean[7], tstd[7].
 * Sample arrays: X[n][19] raw features, T[n][7] raw targets, Y[n][7] outputs in target
 * units, all float, row-major, in device memory.
 *
 * Return codes are those of rmhd.h (0 ok, -1 invalid argument, -2 HIP error, -3 out of
 * memory); rmhd_mlp_last_error() describes the last failure.  Work is enqueued on the stream
 * given at creation; functions that return values in host memory synchronise that stream.
 */
#ifndef RMHD_MLP_H
#define RMHD_MLP_H

#include "rmhd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RMHD_MLP_NIN 19
#define RMHD_MLP_NHID 64
#define RMHD_MLP_NOUT 7
#define RMHD_MLP_NPARAMS 5895
#define RMHD_MLP_NNORM 52
#define RMHD_MLP_MAX_BATCH 65536

typedef struct rmhd_mlp rmhd_mlp;

/* Create a network on the current device from host FP32 master weights params[NPARAMS]
 * (copied); normalisation starts at mean 0, std 1; Adam moments start at zero. */
int rmhd_mlp_create(const float *params, void *hip_stream, rmhd_mlp **out);
void rmhd_mlp_destroy(rmhd_mlp *m);

/* Host copies of the master weights / normalisation (synchronise the stream). */
int rmhd_mlp_get_params(rmhd_mlp *m, float *params);
int rmhd_mlp_get_norm(rmhd_mlp *m, float *norm);
/* Replace the normalisation from a host vector; every std must be > 0. */
int rmhd_mlp_set_norm(rmhd_mlp *m, const float *norm);

/* Normalisation from n >= 1 device samples (X[n][19], T[n][7]): column means and two-pass
 * population standard deviations in FP64, a std below 1e-12 (1 + |mean|) replaced by 1. */
int rmhd_mlp_fit_norm(rmhd_mlp *m, const float *X, const float *T, long n);

/* Outputs Y[n][7] (target units) for device features X[n][19]; precision 0: FP32
 * activations, 1: bfloat16 activations on the matrix cores (the inference arithmetic). */
int rmhd_mlp_forward(rmhd_mlp *m, const float *X, long n, float *Y, int precision);

/* Loss and its gradient with respect to the (bfloat16-rounded) weights over the
 * 1 <= n <= RMHD_MLP_MAX_BATCH device samples X, T; grad (device, NPARAMS floats) and loss
 * (device, one float) may each be NULL. */
int rmhd_mlp_loss_grad(rmhd_mlp *m, const float *X, const float *T, long n, float *grad, float *loss);

/* One Adam step on the minibatch of rows (first + r * stride) mod n, r = 0..batch-1
 * (1 <= batch <= RMHD_MLP_MAX_BATCH); loss: optional device float receiving the batch loss
 * before the update. */
int rmhd_mlp_train_step(rmhd_mlp *m, const float *X, const float *T, long n, long first, long stride, int batch,
                        float lr, float *loss);

/* epochs passes over the n device samples, each a fresh stride permutation drawn from seed,
 * in minibatches of batch rows, learning rate decaying linearly from lr0 to lr1 over all
 * steps.  loss_hist (host, may be NULL) receives the mean batch loss of each epoch. */
int rmhd_mlp_train(rmhd_mlp *m, const float *X, const float *T, long n, int batch, int epochs, float lr0,
                   float lr1, unsigned long long seed, float *loss_hist);

/* Number of Adam steps taken so far. */
long rmhd_mlp_steps(const rmhd_mlp *m);

const char *rmhd_mlp_last_error(const rmhd_mlp *m);

/* ---- use inside the two-fluid solver (rmhd.h) ------------------------------------------
 *
 * rmhd_set_harvest: while X (device [capacity][19]) and T (device [capacity][7]) are set,
 * every implicit stage of a two-fluid context, in rmhd_imex_step and rmhd_implicit_stage,
 * appends one (features, target) row per interior cell, in row-major cell order, as long as
 * the whole stage fits in the remaining capacity.  NULL arrays stop harvesting; the count
 * restarts at zero on every call.  Rows of cells whose Newton failed carry a zero target.
 *
 * rmhd_set_guess_model: while m is set, every implicit stage of the two-fluid context starts
 * Newton from the learned guess (one extra kernel per stage writes it to scratch), falling
 * back to the plain guess for a cell whose Newton fails.  NULL restores the plain guess.  The
 * network must outlive its use by the context.  Single-fluid contexts reject both. */
int rmhd_set_harvest(rmhd_ctx *ctx, float *X, float *T, long capacity);
long rmhd_harvest_count(const rmhd_ctx *ctx);
int rmhd_set_guess_model(rmhd_ctx *ctx, const rmhd_mlp *m);

/* The learned starting point that rmhd_set_guess_model feeds to an implicit stage (the same
 * kernel), written on its own: for every cell of the padded grid (ghosts included, row
 * padding excluded) the seven source-carrying planes of guess (Sbar, taubar, E; conserved
 * layout, ncons planes) receive x0 = R_x + D y, y the network's output on the cell's features
 * of R (f_0 = log10(a mu1^2 D), f_k = R_k / D, f_18 = log10(a sigma)), momentum and energy in
 * conserved units.  The other planes are not touched.  R and guess: device arrays of the
 * context's layout, not aliased.  Two-fluid contexts, a > 0. */
int rmhd_learned_guess(rmhd_ctx *ctx, const rmhd_mlp *m, double a, const double *R, double *guess);

#ifdef __cplusplus
}
#endif

#endif
