/*
 * mclbm_nn.h -- C ABI of the learned surrogate of libmclbm: a 3-D convolutional
 * network that maps the macroscopic fields of the multicomponent model
 * (mole fractions X_a, temperature T, velocity u; the fields of Secs. 2.1 and
 * 3.2) at one time to the same fields K steps later, trained on the GPU by the
 * library's own BF16 matrix-core kernels on trajectories the lattice Boltzmann
 * step generates, with that step as fallback (mclbm_nn_advance below).
 *
 * Network: depth conv layers with 3x3x3 kernels, width 64, ReLU between layers,
 * BF16 weights and activations, FP32 accumulation. Layer 0 maps the C field
 * channels, P second terms and S conditioning channels to 64, the last layer 64
 * to the output channels. BF16 resolves a normalised input to about 3
 * significant digits; the first P field channels are therefore also given as a
 * second BF16 term, the rounding remainder of the first times 256, whose layer-0
 * weights are those of the field divided by 256 (tied, exact in BF16), so the
 * matrix cores see about 16 significant bits of these fields (hi + lo / 256)
 * with no extra parameters. The conditioning channels are constant per tube
 * (for instance the tube's molar masses and diffusivities, which the fields
 * alone do not reveal but which decide how they evolve). Padding: at the x ends
 * of a tube (its walls) every layer replicates the wall node, the mirror image a
 * wall without flux implies (the method of images); periodic in y and z, like the
 * lattice.
 *
 * Output, direct form (species = 0): the change of each of the C fields over
 * the K steps, y_c * out_scale[c]. Conservative form (species = M > 0, fields
 * laid out as mclbm_read_fields_f32: X_1..X_M, T, u, p): for each species s the
 * fluxes of its molar density n_s = p X_s / T (rho_s / m_s with R_U = 1)
 * through the faces between a node x and x + e_a, F_{s,a} = y_{3s+a} *
 * out_scale[3s+a], and the changes of T and u (channels 3M .. 3M+3). The new
 * densities are n_s(x) - sum_a [F_{s,a}(x) - F_{s,a}(x - e_a)], a discrete
 * divergence, so each tube keeps the moles of every species exactly (the mass
 * conservation of Sec. 2.2 item 1); faces at the walls carry no flux. Then
 * p = T sum_s n_s and X_s = n_s / sum n.
 *
 * Geometry: a network is created for a set of tubes (nx, ny, nz each), the same
 * concatenated node layout as a batched mclbm context (include/mclbm.h): a field
 * of C components holds, for tube t, C * n_t values at offset C * (n_0 + ... +
 * n_{t-1}), component-major inside the tube, x fastest.
 *
 * Parameters (host order for get/set): layer by layer, the weights
 * W[tap][out][in] with tap = 9 (dz+1) + 3 (dy+1) + (dx+1), followed by the bias
 * b[out]. Output channel o of a layer is b[o] + sum over taps and input
 * channels of W[tap][o][i] * in[i](x + dx, y + dy, z + dz).
 *
 * Conventions as in mclbm.h: 0 on success, negative MCLBM_E* codes on error,
 * calls ordered on the HIP stream given at creation, the caller owns the
 * workspace and every buffer it passes.
 */
#ifndef MCLBM_NN_H
#define MCLBM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "mclbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mclbm_nn mclbm_nn;

/* Workspace bytes of a network with `channels` field components C (<= 16),
 * `two_term` of them (the leading ones) also given as a second term P (<= C),
 * `conditioning` per-tube constants S (C + P + S <= 32), output form `species`
 * (0: direct; M > 0: conservative, needs C = M + 5 and 3 M + 4 <= 32), `depth`
 * conv layers (2..16) over ntubes tubes, dims = [ntubes][3] (nx, ny, nz). */
size_t mclbm_nn_workspace_bytes(int32_t channels, int32_t two_term, int32_t conditioning, int32_t species,
                                int32_t depth, const int32_t *dims, int32_t ntubes);

int mclbm_nn_create(int32_t channels, int32_t two_term, int32_t conditioning, int32_t species, int32_t depth,
                    const int32_t *dims, int32_t ntubes, void *dev_workspace, size_t bytes, void *hip_stream,
                    mclbm_nn **out);
void mclbm_nn_destroy(mclbm_nn *net);
const char *mclbm_nn_last_error(const mclbm_nn *net);

/* Number of parameters (host order above). */
int64_t mclbm_nn_param_count(const mclbm_nn *net);
/* Copy parameters or accumulated gradients (FP32, host order) to / from the host.
 * set_params also clears the optimiser state. */
int mclbm_nn_set_params(mclbm_nn *net, const float *host);
int mclbm_nn_get_params(mclbm_nn *net, float *host);
int mclbm_nn_get_grads(mclbm_nn *net, float *host);

/* Normalisation: network input channel c is (f_c - in_shift[c]) * in_scale[c]
 * (in_shift, in_scale: `channels` values); out_scale has one value per output
 * channel (C in the direct form, 3 M + 4 in the conservative form). */
int mclbm_nn_set_norm(mclbm_nn *net, const float *in_shift, const float *in_scale, const float *out_scale);

/* Conditioning values, host [ntubes][conditioning], used as given (already
 * normalised); all zero after creation. */
int mclbm_nn_set_conditioning(mclbm_nn *net, const float *host);

/* Device buffers of the network, each [channels][n] FP32 in the tube layout:
 * the input fields and the predicted fields. */
int mclbm_nn_io(mclbm_nn *net, float **fields_in, float **fields_out);

/* Forward pass: fields_in -> fields_out; keeps the activations for backward. */
int mclbm_nn_forward(mclbm_nn *net);

/* Mean squared error of the prediction against target (device, [channels][n]),
 * with per-channel weights w (host, `channels` values, may be NULL = 1).
 * Direct form: loss = (1/n) sum_nodes sum_c w_c ((pred_c - target_c) / out_scale[c])^2.
 * Conservative form, in physical units: loss = (1/n) sum_nodes [sum_s w_s (n_s -
 * n*_s)^2 + w_M (T - T*)^2 + sum_k w_{M+1+k} (u_k - u*_k)^2 + w_{M+4} sum_s
 * (F_{s,x} - F*_{s,x})^2], the last sum over the open x faces (the p slot of the
 * weights, which this form does not fit, weights the x fluxes). F*_{s,x}(x) =
 * -sum_{x' <= x} (n*_s - n_s)(x') along each x row: on a tube with walls and fields
 * uniform in y and z, the fluxes that produce the target change. The divergence
 * alone cannot see a uniform offset of the fluxes on every interior face, which
 * only the wall nodes then feel; this term fixes it.
 * Seeds the output gradient for backward. Synchronises the stream. */
int mclbm_nn_loss(mclbm_nn *net, const float *target, const float *channel_weight, double *loss);

/* Backward pass of the last forward and loss: adds the parameter gradients to
 * the accumulated ones. */
int mclbm_nn_backward(mclbm_nn *net);
int mclbm_nn_zero_grad(mclbm_nn *net);

/* Global 2-norm of the accumulated gradients (FP64 sum of squares over all
 * parameters), written to *norm (may be NULL). If max_norm > 0 and the norm exceeds
 * it, every gradient is scaled by max_norm / norm (clipping by global norm, before
 * the optimiser step); max_norm = 0 only measures. A non-finite norm is returned
 * and nothing is scaled. MCLBM_EARG for a negative or NaN max_norm. Synchronises
 * the stream. */
int mclbm_nn_clip_grad_norm(mclbm_nn *net, double max_norm, double *norm);

/* One Adam step (Kingma and Ba) on the accumulated gradients, then clears them. */
int mclbm_nn_adam_step(mclbm_nn *net, float lr, float beta1, float beta2, float eps);

/* Relative change of the moles of each species per tube between two field sets
 * a, b (device, [channels][n] in the layout of mclbm_read_fields_f32: X_1..X_M,
 * T at index M, p at index M + 4): with R_U = 1 the molar density of species s
 * is rho_s / m_s = p X_s / T, so the tube's moles are S_s = sum_x p X_s / T,
 * exactly what the lattice conserves; out[t] = max_s |S_s(b) - S_s(a)| / S_s(a).
 * out: host [ntubes]. Needs channels >= species + 5. */
int mclbm_nn_mole_residual(mclbm_nn *net, int32_t species, const float *a, const float *b, double *out);

/* Advance a lattice Boltzmann context by K steps with the network (trained for
 * K steps): read the fields, predict, and form the fields to install (mole
 * fractions clipped at 0 and renormalised). Two quantities decide whether the
 * prediction is used:
 *  - its residual, the largest relative change, over the tubes, of a species'
 *    mass or of the total energy of the local equilibrium those fields define,
 *    against the conserved sums of the current populations: the walled or
 *    periodic lattice keeps both (Sec. 2.2 item 1; the energy of eq
 *    g0momTotalEnergy), up to its rounding, and the network, which keeps the
 *    moles by construction but predicts T and u directly, does not;
 *  - its change, the largest |X_a(new) - X_a(now)| over the nodes and species:
 *    a trust region, since the network's error grows with the size of the hop
 *    it predicts (large where the mixture is far from equilibrium, as just
 *    after a sharp initial condition), which a conserved sum cannot detect.
 * If the fields are a feasible state, the residual is at most resid_tol and the
 * change at most change_tol (HUGE_VAL: no limit), the populations are
 * re-initialised at the local equilibrium of those fields; otherwise the K
 * lattice steps run instead (*used_fallback = 1). *max_residual and
 * *max_change (either may be NULL) receive the two (HUGE_VAL for an infeasible
 * prediction). The network's tubes must be the context's and its channels
 * M + 5 (X_1..X_M, T, u_x, u_y, u_z, p: the layout of mclbm_read_fields_f32).
 * The step count advances by K. MCLBM_EARG for a NaN tolerance; MCLBM_ENAN if
 * the current state is not finite; MCLBM_EUNSUPPORTED for a context whose
 * slaved species is not the last (mclbm_params.slaved other than 0 or M). */
int mclbm_nn_advance(mclbm_ctx *c, mclbm_nn *net, int32_t K, double resid_tol, double change_tol,
                     int32_t *used_fallback, double *max_residual, double *max_change);

#ifdef __cplusplus
}
#endif
#endif
