/*
 * tdde_mlp.h -- learned initial guess for the BiCGSTAB solve of the Crank-Nicolson step.
 *
 * A pointwise network predicts psi_{n+1} for every state entry (instance, channel, component,
 * radial index) from the last four states and the field; BiCGSTAB to the same tolerance still
 * decides the result, so the guess changes iteration counts, never the solution.
 *
 *   rho   = sqrt(|psi_n|^2 + |psi_{n-1}|^2 + tau^2),   u_k = psi_{n-k} / rho   (k = 0..3)
 *   x     = [Re u_0, Im u_0, .., Re u_3, Im u_3, f(t_n + dt/2), f(t_n - dt/2), s, 0 x 21]  (32)
 *   h1    = silu(W1 x + b1), h2 = silu(W2 h1 + b2), y = W3 h2 + b3        (hidden width H = 256)
 *   out   = sum_k c[s][k] u_k + sigma (y_0 + i y_1),   guess = rho * out
 *
 * The linear skip c[s][k] (complex, FP64) is the least-squares four-step predictor of psi_{n+1}
 * per spinor component s, fitted on the training rows (tdde_mlp_fit_skip); its coefficients are
 * large and cancel, so it is kept and applied in FP64. sigma is the RMS residual of that fit, so
 * the network learns the remainder at unit scale. Weights are used in BF16 with FP32 accumulation
 * (gfx950 MFMA 16x16x32 bf16); FP32 master weights are updated by Adam. Flat FP32 parameter layout
 * (tdde_mlp_param_count() values): W1[256][32], b1[256], W2[256][256], b2[256], W3[2][256], b3[2].
 *
 * Training rows ("raw samples", device float64 [M][16]) hold, per row:
 *   [0..9]  Re/Im of psi_n, psi_{n-1}, psi_{n-2}, psi_{n-3}, psi_{n+1}
 *   [10] f(t_n + dt/2)  [11] f(t_n - dt/2)  [12] s  [13..15] unused
 * All device pointers are caller-owned; the context owns its parameters and training scratch.
 */
#ifndef TDDE_MLP_H
#define TDDE_MLP_H

#include <stdint.h>

#include "tdde.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdde_mlp tdde_mlp;

/* Create a network (hidden width 256) on hip_stream; train_rows is the largest training batch
 * (sizes the scratch buffers). Parameters start at zero: call tdde_mlp_set_params. */
tdde_status tdde_mlp_create(int32_t train_rows, double tau, void* hip_stream, tdde_mlp** out);
tdde_status tdde_mlp_destroy(tdde_mlp* m);
int64_t tdde_mlp_param_count(void);

/* Copy FP32 master parameters from / to the host (flat layout above). set_params also resets the
 * Adam moments and the step counter. */
tdde_status tdde_mlp_set_params(tdde_mlp* m, const float* host);
tdde_status tdde_mlp_get_params(tdde_mlp* m, float* host);
/* Last gradient (FP32, flat layout) to the host. */
tdde_status tdde_mlp_get_grads(tdde_mlp* m, float* host);

/* Least-squares fit of the skip coefficients on M raw samples (device float64 [M][16]): the Gram
 * matrices sum conj(u_k) u_l and right-hand sides sum conj(u_k) psi_{n+1}/rho per component are
 * reduced on the device in a fixed order, each 4x4 Hermitian system is solved on the device in
 * FP64 (Gaussian elimination, partial pivoting), and sigma is set to the RMS residual of the fit
 * (at least 1e-300). */
tdde_status tdde_mlp_fit_skip(tdde_mlp* m, const double* raw, int32_t M);
/* Set / read the skip coefficients c[2][4][2] (re, im) and sigma (host). */
tdde_status tdde_mlp_set_skip(tdde_mlp* m, const double* c, double sigma);
tdde_status tdde_mlp_get_skip(tdde_mlp* m, double* c, double* sigma);

/* Forward pass on M raw samples (device float64 [M][16]); writes out[M][2] (device float32): the
 * residual of the prediction in units of sigma, (out - psi_{n+1}/rho) / sigma, formed in FP64
 * (the residual is far below FP32 resolution of the prediction itself). M <= train_rows. */
tdde_status tdde_mlp_forward(tdde_mlp* m, const double* raw, int32_t M, float* out);

/* Forward + loss + backward on M raw samples: loss (host) = mean over rows of the squared residual
 * |out - psi_{n+1}/rho|^2 / sigma^2; gradients of the FP32 parameters stay on the device
 * (tdde_mlp_get_grads); the skip is not trained by gradients. */
tdde_status tdde_mlp_backward(tdde_mlp* m, const double* raw, int32_t M, double* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradients, then refresh the BF16
 * copies. */
tdde_status tdde_mlp_adam(tdde_mlp* m, float lr);

/* Pulses used by tdde_mlp_guess: host [batch][n_fields]; field index 0 of each instance enters the
 * features. Setup call (may allocate). */
tdde_status tdde_mlp_set_pulses(tdde_mlp* m, const tdde_pulse* pulses_host, int32_t batch, int32_t n_fields);

/* Guess for every entry of a batch of states: hist = device complex128 [batch][E] pointers of
 * psi_n, psi_{n-1}, psi_{n-2}, psi_{n-3}; nr = radial size (component of entry e is (e / nr) % 2).
 * Writes guess_out (device complex128 [batch][E], distinct from the history). batch must equal the
 * batch of tdde_mlp_set_pulses. Allocates nothing. */
tdde_status tdde_mlp_guess(tdde_mlp* m, const void* const hist[4], int32_t batch, int64_t E, int32_t nr,
                           double t_n, double dt, void* guess_out);

const char* tdde_mlp_last_error(const tdde_mlp* m);

#ifdef __cplusplus
}
#endif
#endif /* TDDE_MLP_H */
