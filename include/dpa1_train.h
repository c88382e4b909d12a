/*
 * dpa1_train.h - C ABI of the student trainer of the MI355X DPA-1 library.
 *
 * Trains a small DP-SE-style student (Sec. II-B descriptor without the
 * attention refinement: embedding 16 -> 32 -> 64 with doubling residuals, any
 * axis <= 16, two tanh fitting layers of equal width H in {32, 64, 128, 256}
 * with an identity residual on the second) on energies and forces labelled by
 * a teacher.  Per batch of B frames of N atoms (same types and box for every
 * frame) the loss is
 *
 *   L = p_e / B * sum_f ((E_f - E^_f) / N)^2
 *     + p_f / (3 N B) * sum_f sum_k |F_fk - F^_fk|^2,
 *
 * with E = sum_i e_i (Eq. (5)) and F = -dE/dx (Eq. (2)), and its gradient is
 * exact: the force term is differentiated through the force computation
 * (second derivatives of the energy), not approximated.  Adam (Kingma and
 * Ba 2015) updates FP32 master weights; the forward, the force adjoint and
 * every matrix-core product run at the precision chosen in the options
 * (DP_PREC_BF16: BF16 operands, FP32 accumulation; per-pair embedding
 * arithmetic FP32, weight-gradient sums FP64).
 *
 * Arrays: frames [B][N][3] FP64 positions, types [N], e_label [B], f_label
 * [B][N][3] FP64 are device pointers; box is a host pointer as in dp_compute
 * (or NULL for open boundaries).  Every frame's atoms are all local (no ghost
 * atoms).  Parameters are exchanged in weights-file order (the tensors of the
 * weights file concatenated), FP64 on the host.
 *
 * Calls are synchronous: they enqueue on the given stream (NULL: default
 * stream) and return after the step's results are on the host.  A trainer is
 * not thread-safe.  Errors are reported as in dpa1.h (dp_last_error).
 */
#ifndef DPA1_TRAIN_H
#define DPA1_TRAIN_H

#include <stdint.h>

#include "dpa1.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dp_trainer dp_trainer;

typedef struct dp_train_options {
  double pref_e;  /* p_e, >= 0 */
  double pref_f;  /* p_f, >= 0 */
  double beta1;   /* Adam first-moment decay, in [0, 1) */
  double beta2;   /* Adam second-moment decay, in [0, 1) */
  double eps;     /* Adam denominator offset, > 0 */
  int precision;  /* DP_PREC_FP32 or DP_PREC_BF16 */
} dp_train_options;

/* Load the initial student weights and allocate the trainer on the current
 * device.  Returns DP_ERR_WEIGHTS when the model is not of the student family
 * described above, DP_ERR_ARG for bad options. */
int dp_train_create(const char *weights_path, double rcut, int sel, const dp_train_options *opt,
                    dp_trainer **out);

/* Loss of the batch at the current weights and, if grad is not NULL, its
 * gradient grad [nparams] (host, FP64, weights-file order).
 * loss [3] (host) receives L, its energy part and its force part. */
int dp_train_gradient(dp_trainer *t, const double *d_frames, const int32_t *d_types,
                      const double *box, int natoms, int nframes, const double *d_e_label,
                      const double *d_f_label, double *loss, double *grad, void *hip_stream);

/* One training step: the gradient of the batch at the current weights, then
 * one Adam update with step size lr.  loss [3] as above (before the update). */
int dp_train_step(dp_trainer *t, const double *d_frames, const int32_t *d_types,
                  const double *box, int natoms, int nframes, const double *d_e_label,
                  const double *d_f_label, double lr, double *loss, void *hip_stream);

/* Current master weights as FP64 (params may be NULL) and their count. */
int dp_train_params(const dp_trainer *t, double *params, int32_t *nparams);

/* Write the current weights as a weights file usable by dp_create. */
int dp_train_save(const dp_trainer *t, const char *path);

/* Checkpoint and resume: the FP32 master weights, the Adam moments m and v
 * and the step count, in a file of this library's own format (magic
 * "DPA1TRN", int32 count and step, then three FP32 arrays).  Resuming into a
 * trainer created from a model of the same shape continues the run exactly
 * (the same later steps give bit-identical weights); DP_ERR_WEIGHTS when the
 * file does not match the trainer. */
int dp_train_checkpoint(const dp_trainer *t, const char *path);
int dp_train_resume(dp_trainer *t, const char *path);

void dp_train_destroy(dp_trainer *t);

/* Largest n accepted by the force-error calls (3n + 2^16 fits an int). */
#define DP_FORCE_ERROR_MAX_ATOMS 700000000

/* Audit helper: over n atoms, rmse_max [2] (host) = (sqrt(sum |a - b|^2 / (3n)),
 * max_k,c |a_kc - b_kc|) of two device force arrays [n][3]; synchronous.
 * Allocates and frees a small device buffer for its partial sums per call.
 * DP_ERR_ARG for n < 0, n > DP_FORCE_ERROR_MAX_ATOMS or a NULL pointer. */
int dp_force_error(const double *d_a, const double *d_b, int n, double *rmse_max,
                   void *hip_stream);

/* The same audit reduction for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops): no hipMalloc, hipFree
 * or other allocation.  The per-block partial sums live in a fixed 4 KiB
 * device array inside the library (one copy per GPU, held until the process
 * ends); the 256-block cap of the reduction makes every accepted n fit.
 *   d_a, d_b     device force arrays [n][3] (FP64), caller-owned.
 *   d_rmse_max   device output [2]: (RMSE, max abs difference), the values
 *                dp_force_error returns (the partial sums are added in the
 *                same order); zeros for n = 0.
 *   hip_stream   stream to enqueue on (NULL: default stream); asynchronous.
 * DP_ERR_ARG for n < 0, n > DP_FORCE_ERROR_MAX_ATOMS or a NULL pointer,
 * before any device work.  Calls that overlap on one GPU share the array and
 * race: serialise them (one stream, or events). */
int dp_force_error_noalloc(const double *d_a, const double *d_b, int n, double *d_rmse_max,
                           void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* DPA1_TRAIN_H */
