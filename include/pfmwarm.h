/*
 * pfmwarm: learned warm start for the periodic FM-BEM solver (pfmbem.h).
 *
 * A multilayer perceptron maps the parameters of a solve, (ka, theta, r/a,
 * rho_fibre/rho_matrix, c_fibre/c_matrix), to the low Fourier modes of the
 * boundary densities of every fibre; the synthesised densities seed GMRES
 * (pfm_solve / pfm_solve_batch with use_x0 = 1), whose true residual decides
 * the result, so a poor prediction costs iterations, never accuracy.  The
 * network is this library's own addition to the method of the paper (which
 * starts GMRES from zero); its training runs on the GPU through the
 * forward, backward and Adam calls below.
 *
 * Network: sizes[0] inputs, hidden layers h_{l+1} = tanh(W_l h_l + b_l),
 * linear output layer.  Parameters are FP32, stored flat on the device,
 * layer by layer: W_l as [sizes[l+1]][sizes[l]] row-major, then b_l.
 * Loss: L = (1 / (B sizes[n])) sum (y - t)^2 over a batch of B rows.
 * Optimiser: Adam (Kingma & Ba 2015) with bias correction.
 * Inference in BF16: weights rounded to bfloat16 (round to nearest even),
 * activations rounded to bfloat16 at the matrix-core inputs, FP32
 * accumulation (MFMA 16x16x16), FP32 bias and tanh.
 *
 * Modal representation (per fibre f and density s = phi, varphi, with the
 * incident phase at the fibre centre c_f removed, d = (cos th, sin th)):
 *   c_{f,s,n} = (1/N) sum_e psi_{f,s}(e) e^{-2 pi i n e / N} e^{-i k c_f.d},
 *   n = -K/2 .. K/2-1, and psi_{f,s}(e) = e^{i k c_f.d} sum_n c_{f,s,n} e^{2 pi i n e / N};
 * vector layout [f][s][n][re, im] (FP32), 4 M K values per member.
 *
 * Conventions as in pfmbem.h: d_* are caller-owned device pointers; the
 * library allocates only in pfm_mlp_create and frees in pfm_mlp_destroy;
 * every call is queued on the handle's stream.  Errors: PFM_EINVAL for bad
 * sizes or null pointers, PFM_EDEVICE for HIP errors.
 */
#ifndef PFMWARM_H
#define PFMWARM_H

#include "pfmbem.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfm_mlp pfm_mlp;

#define PFM_MLP_MAX_LAYERS 8
#define PFM_MLP_MAX_WIDTH 4096

/* n_layers weight layers (1..8), widths sizes[0..n_layers] (1..4096);
 * max_batch rows per call.  Parameters drawn uniform in +-1/sqrt(fan_in)
 * from a counter-based generator (SplitMix64) seeded with `seed`. */
pfm_status pfm_mlp_create(const int* sizes, int n_layers, int max_batch, unsigned long long seed,
                          pfm_mlp** out);
void pfm_mlp_destroy(pfm_mlp* m);
pfm_status pfm_mlp_set_stream(pfm_mlp* m, void* hip_stream);

/* Number of parameters and the library-owned device arrays of parameters,
 * gradients (same layout) and Adam moments (valid until destroy). */
long long pfm_mlp_n_params(const pfm_mlp* m);
pfm_status pfm_mlp_buffers(pfm_mlp* m, float** d_params, float** d_grads);

/* Copy all parameters (FP32, flat layout above) to / from caller device memory. */
pfm_status pfm_mlp_get_params(pfm_mlp* m, float* d_dst);
pfm_status pfm_mlp_set_params(pfm_mlp* m, const float* d_src);
pfm_status pfm_mlp_get_grads(pfm_mlp* m, float* d_dst);

/* Fold an output affine map into the last layer: y_o -> scale[o] y_o + shift[o]
 * (d_scale, d_shift: sizes[n] FP32 each; used to undo target standardisation). */
pfm_status pfm_mlp_scale_output(pfm_mlp* m, const float* d_scale, const float* d_shift);

/* Statistics of training targets d_t [n][sizes[last]] (FP32, row-major):
 * per column the mean and the standard deviation (n - 1 in the denominator,
 * at least 1e-6), into d_mean and d_std (sizes[last] floats each). */
pfm_status pfm_mlp_target_stats(pfm_mlp* m, const float* d_t, int n, float* d_mean, float* d_std);
/* d_out = (d_t - mean) / std per column (d_out may be d_t). */
pfm_status pfm_mlp_standardise(pfm_mlp* m, const float* d_t, int n, const float* d_mean, const float* d_std,
                               float* d_out);
/* Shrink of the outputs towards zero from n <= max_batch held-back rows
 * (d_x inputs, d_t targets): per output o, s_o = clamp(1 - sum (y - t)^2 /
 * sum t^2, 0, 1) with y the FP32 forward, written to d_shrink and folded
 * into the last layer (outputs the network cannot predict are left out of a
 * start vector).  h_rel_err (optional, synchronises the stream): the
 * relative error sqrt(sum (s y - t)^2 / sum t^2) after the shrink.  Needs
 * max_batch >= 4. */
pfm_status pfm_mlp_validation_shrink(pfm_mlp* m, const float* d_x, const float* d_t, int n, float* d_shrink,
                                     float* h_rel_err);

/* FP32 forward of B <= max_batch rows: d_x [B][sizes[0]] -> d_y [B][sizes[n]].
 * Keeps the activations for pfm_mlp_backward_mse. */
pfm_status pfm_mlp_forward(pfm_mlp* m, const float* d_x, int B, float* d_y);

/* After pfm_mlp_forward on the same B rows: gradients of the MSE against
 * targets d_t [B][sizes[n]] into the gradient array (overwritten).  When
 * h_loss != NULL the loss is returned there (synchronises the stream). */
pfm_status pfm_mlp_backward_mse(pfm_mlp* m, const float* d_t, int B, float* h_loss);

/* One Adam step (t = 1, 2, ... counts the steps) on every parameter. */
pfm_status pfm_mlp_adam(pfm_mlp* m, float lr, float beta1, float beta2, float eps, int t);

/* Round the current weights to bfloat16 (kept until the next call). */
pfm_status pfm_mlp_to_bf16(pfm_mlp* m);
/* BF16 forward with the weights of the last pfm_mlp_to_bf16. */
pfm_status pfm_mlp_infer_bf16(pfm_mlp* m, const float* d_x, int B, float* d_y);

/* d_x [B][5] = 2 (d_draws - lo) / (hi - lo) - 1 with lo = (0.2, 0, 0.15, 0.5, 0.5),
 * hi = (8, pi/2, 0.4, 20, 2): draws (ka, theta, r/a, rho ratio, c ratio) in FP64. */
pfm_status pfm_warm_features(const double* d_draws, int B, float* d_x, void* hip_stream);

/* Modal analysis of B stacked densities [B][2MN] (complex128) of a handle at
 * its current frequency, member b at incidence angle thetas[b] (host array):
 * d_vec [B][4 M K] FP32.  K even, 2 <= K <= N. */
pfm_status pfm_modes_analyse(pfm_problem* pb, int K, int B, const double* thetas, const void* d_psi,
                             float* d_vec);
/* Synthesis: d_psi [B][2MN] complex128 from d_vec [B][4 M K]. */
pfm_status pfm_modes_synthesise(pfm_problem* pb, int K, int B, const double* thetas, const float* d_vec,
                                void* d_psi);

#ifdef __cplusplus
}
#endif

#endif
