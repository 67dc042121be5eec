/*
 * pphd_mlp.h -- C ABI of the learned birth proposal of libpphd.
 *
 * Eq 6 of the paper draws the J_k birth particles from a proposal
 * p_k(. | Z_k) that may depend on the current measurements and weights them
 * by gamma_k(x) / (J_k p_k(x | Z_k)).  With birth_proposal 2 (pphd.h) the
 * filter takes as proposal the defensive mixture
 *   q(x | Z_k) = alpha gamma(x)/m_b + (1 - alpha) (1/M) sum_p q_phi(x | z_p),
 * where q_phi(. | z) is a 4-component Gaussian mixture with diagonal
 * covariance over the state [x, vx, y, vy] that a small network maps each
 * measurement to.  The weights stay those of Eq 6 for any network, so a poor
 * network costs accuracy, never correctness; alpha > 0 keeps the birth
 * density itself in the mixture.
 *
 * Network (all widths fixed):
 *   features  f(z) = ((s_x + r cos th - c_x)/h_x, (s_y + r sin th - c_y)/h_y),
 *             c the centre and h the half-widths of the surveillance region;
 *   layers    h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3),
 *             o = W4 h3 + b4, widths 2 -> 128 -> 128 -> 128 -> 36;
 *   mixture   component c reads o[9c .. 9c+8]: logit o[9c]; mean in the
 *             normalised state xi = ((x-c_x)/h_x, vx/sv, (y-c_y)/h_y, vy/sv)
 *             of (f_x + o[9c+1], o[9c+2], f_y + o[9c+3], o[9c+4]); log standard
 *             deviations clip(o[9c+5 .. 9c+8], -12, 6) in the same units;
 *             weights softmax of the logits.
 * Parameters: one float[PPHD_MLP_PARAMS] in the order W1 ([128][2], row =
 * output unit), b1[128], W2 ([128][128]), b2, W3, b3, W4 ([36][128]), b4[36].
 *
 * Training: minimise the mean negative log-likelihood of the normalised
 * state under the mixture, -log q~(xi | z), over pairs (z, x) with x drawn
 * from the birth density gamma/m_b and z from the sensor model given x (a
 * detection).  Layers 2-4 run on the matrix cores: BF16 operands (weights and
 * activations rounded to nearest even), FP32 accumulation; layer 1, the
 * mixture head and the loss run in FP32; master weights and Adam moments are
 * FP32.  The handle holds a dataset of simulated pairs in device memory and
 * takes Adam steps over it in order (minibatch t covers pairs
 * [t*batch mod dataset, +batch)).
 *
 * Conventions are those of pphd.h: pphd_status results, pphd_last_error(),
 * caller-owned device workspace, all device work on the handle's stream in
 * call order, calls that return host data synchronise that stream.  A
 * filter that uses the network (pphd_attach_mlp) reads its weights on the
 * filter's stream: the caller orders training before use when the two
 * streams differ.
 */
#ifndef PPHD_MLP_H
#define PPHD_MLP_H

#include "pphd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PPHD_MLP_HIDDEN 128
#define PPHD_MLP_OUTPUTS 36
#define PPHD_MLP_PARAMS 38052

typedef struct pphd_mlp pphd_mlp;

typedef struct {
    int32_t batch;     /* pairs per training step: a multiple of 64 in [64, 65536]    */
    int32_t dataset;   /* simulated pairs held in device memory: a multiple of batch */
    double lr;         /* Adam step size (pphd_mlp_train may override per call)       */
    double beta1, beta2, eps;  /* Adam moment decays and denominator floor            */
} pphd_mlp_config;

/* Bytes of device workspace for a network with this configuration. */
pphd_status pphd_mlp_workspace_size(const pphd_mlp_config* cfg, size_t* bytes);

/* Creates the network.  model: the filter model whose birth density, sensor
 * and region define the features, the normalised state and the simulated
 * pairs (only those fields are read).  workspace: caller-owned device memory
 * of pphd_mlp_workspace_size() bytes, 256-byte aligned, kept until destroy.
 * seed: Philox key of the simulated pairs and of pphd_mlp_init_params.
 * The parameters start at zero: call pphd_mlp_init_params or
 * pphd_mlp_set_params before use. */
pphd_status pphd_mlp_create(const pphd_model* model, const pphd_mlp_config* cfg, void* workspace,
                            size_t workspace_bytes, uint64_t seed, void* stream, pphd_mlp** out);

/* Uniform He initialisation from Philox (weights of layer l uniform in
 * +-sqrt(6/fan_in), the output layer scaled by 0.1; biases zero except the
 * log standard deviations of the output, log 0.05 for positions and 0 for
 * velocities).  Resets the Adam state. */
pphd_status pphd_mlp_init_params(pphd_mlp* h, uint32_t init_id);

/* Copies PPHD_MLP_PARAMS floats in (host or device pointer, on_device 0/1)
 * and resets the Adam state; or copies them out (synchronises). */
pphd_status pphd_mlp_set_params(pphd_mlp* h, const float* params, int32_t on_device);
pphd_status pphd_mlp_get_params(pphd_mlp* h, float* params, int32_t on_device);

/* Fills the dataset with simulated pairs: pair i uses the Philox blocks of
 * counter (i, 0, 6*16 + sub, run) for sub = 0 (position uniforms), 1
 * (velocity normals) and 2 (range and bearing noise); the bearing is wrapped
 * to [-pi, pi).  The pairs are kept in FP32. */
pphd_status pphd_mlp_simulate(pphd_mlp* h, uint32_t run);

/* Copies pairs [first, first+n) of the dataset out: z float[n][2]
 * (range, bearing), x float[n][4].  Synchronises. */
pphd_status pphd_mlp_read_dataset(pphd_mlp* h, int32_t first, int32_t n, float* z, float* x);

/* Mean loss and its gradient over n given pairs (1 <= n <= batch), without
 * changing the parameters.  z: float[n][2], x: float[n][4], on the host or
 * the device (on_device).  grad: host float[PPHD_MLP_PARAMS] (nullable);
 * loss: host double (nullable).  Synchronises. */
pphd_status pphd_mlp_loss_grad(pphd_mlp* h, const float* z, const float* x, int32_t n,
                               int32_t on_device, float* grad, double* loss);

/* steps Adam steps over the dataset with step size lr (lr <= 0: the
 * configuration's).  loss: nullable host float[steps], the mean loss of each
 * minibatch before its step.  Synchronises only when loss is given. */
pphd_status pphd_mlp_train(pphd_mlp* h, int32_t steps, double lr, float* loss);

/* Network outputs o (float[n][36]) for n measurements (double[n][2]; range,
 * bearing), n <= batch.  Pointers on the host or the device (on_device);
 * host results synchronise. */
pphd_status pphd_mlp_forward(pphd_mlp* h, const double* z, int32_t n, int32_t on_device, float* out);

/* Number of Adam steps taken since the last parameter reset. */
pphd_status pphd_mlp_steps(pphd_mlp* h, int64_t* steps);

pphd_status pphd_mlp_destroy(pphd_mlp* h);

/* ---- use by a filter (birth_proposal 2) --------------------------------- */

/* The network whose mixtures pphd_update draws the births from (NULL
 * detaches).  The network must outlive its use by the filter. */
pphd_status pphd_attach_mlp(pphd_filter* f, pphd_mlp* h);

/* Network outputs for the next pphd_update, in place of the attached
 * network's (stage tests): raw float[m][36] on the host or the device, m the
 * measurement count that update will pass.  Phase PREDICTED; used once. */
pphd_status pphd_set_birth_mixture(pphd_filter* f, const float* raw, int32_t m, int32_t on_device);

#ifdef __cplusplus
}
#endif
#endif /* PPHD_MLP_H */
