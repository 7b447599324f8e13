/*
 * fh_net.h -- C-ABI of the learned warm start for the FFT-preconditioned
 * finite-element homogenization solver (fh.h).
 *
 * The paper's solver starts every linear solve from the initial guess
 * u_(0) of the Newton scheme (Alg. 1), zero for a linear material.  The
 * warm start replaces that zero by the output of a small 3D convolutional
 * encoder-decoder evaluated on the phase field; PCG from zero stays the
 * fallback and the screen (fh_set_warm_start in fh.h).  Nothing of the
 * network is in the paper; its definition:
 *
 *   Input features per voxel: chi = [phase == 1], gamma chi, gamma, where
 *   gamma = log10(E_inclusion / E_matrix) / 3 is given per sample.
 *   Levels n, n/2, n/4, n/8 (n a multiple of 64) with 16/32/64/64 channels;
 *   per level two 3x3x3 convolutions with periodic wrap, bias and a leaky
 *   ReLU of slope 1/8; 2x2x2 average pooling down; nearest up-sampling
 *   concatenated with the skip of the same level ([up, skip]) up; a 1x1x1
 *   head with 18 outputs: the fluctuation fields of the 6 unit Mandel
 *   strains (load-major, 3 components each) in voxel units u n / l.
 *   Convolution: y[o][v] = b[o] + sum_t sum_c W[t][o][c] x[c][v + d_t],
 *   tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1), offset d_t = (dz, dy, dx).
 *   Loss: mean over samples, channels, voxels and the three directions of
 *   the squared periodic forward difference of (output - target).
 *   Optimiser: Adam with bias correction, optional global-norm clipping.
 *
 * Precision: weights, biases, activations and activation gradients are
 * stored in BF16 (round to nearest even); convolutions run on the matrix
 * cores with BF16 operands and FP32 accumulation; FP32 master weights,
 * weight gradients, Adam moments and the head output; FP64 loss sums.
 *
 * Flat parameter vector (FP32, fh_net_param_count() entries): for each of
 * the 14 convolutions in the order e0a (3->16), e0b (16->16), e1a (16->32),
 * e1b (32->32), e2a (32->64), e2b (64->64), b3a (64->64), b3b (64->64),
 * d2a (128->64), d2b (64->64), d1a (96->32), d1b (32->32), d0a (48->16),
 * d0b (16->16): W[27][cout][cin] then b[cout]; then the head Wh[18][16] and
 * bh[18].
 *
 * Layouts: phase fields uint8 [sample][z][y][x] (x fastest, n^3 each);
 * network output FP32 [sample][18][n^3]; training targets BF16 bit
 * patterns [sample][18][n^3].  Pointers ending in _dev are device pointers
 * on the device given to fh_net_create, others host pointers; the caller
 * owns every array.  Return codes are those of fh.h; fh_net_last_error()
 * describes the last failure.  A network object is not thread-safe.
 */
#ifndef FH_NET_H
#define FH_NET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef FH_NET_TYPEDEF
#define FH_NET_TYPEDEF
typedef struct fh_net fh_net;
#endif

/* Adam step: g <- g min(1, clip / |g|_2) if clip > 0 (global norm over all
 * parameters), then m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
typedef struct fh_adam {
  double lr, beta1, beta2, eps, clip;
} fh_adam;

/* kernel classes for fh_net_stats */
#define FH_NET_K_CONV 0   /* forward convolutions (MFMA)          */
#define FH_NET_K_DGRAD 1  /* input-gradient convolutions (MFMA)   */
#define FH_NET_K_WGRAD 2  /* weight gradients (MFMA) + reductions */
#define FH_NET_K_OTHER 3  /* pooling, concat, head, loss, Adam    */
#define FH_NET_K_NCLASS 4

typedef struct fh_net_stats {
  double kernel_ms[FH_NET_K_NCLASS];       /* summed HIP-event times     */
  long long kernel_launches[FH_NET_K_NCLASS];
  double flops[FH_NET_K_NCLASS];           /* algorithmic flops          */
  long long adam_steps;
} fh_net_stats;

/* Number of FP32 parameters of the network. */
long long fh_net_param_count(void);

/* Network for grids of n^3 voxels (n in {64, 128, 192, 256}) and batches of
 * up to max_batch samples (<= 64); allocates all device buffers once.
 * Parameters start at zero: set them with fh_net_set_params. */
int fh_net_create(fh_net **out, int device, int n, int max_batch);
void fh_net_destroy(fh_net *net);
const char *fh_net_last_error(const fh_net *net);
/* HIP stream for all later work (default: the null stream). */
int fh_net_set_stream(fh_net *net, void *hip_stream);

/* Copy the FP32 parameter vector in (resets the Adam moments and step) or
 * out. */
int fh_net_set_params(fh_net *net, const float *params);
int fh_net_get_params(fh_net *net, float *params);

/* Output for `batch` samples: phase_dev [batch][n^3], gamma [batch] (host),
 * out_dev [batch][18][n^3] FP32. */
int fh_net_forward(fh_net *net, int batch, const uint8_t *phase_dev, const float *gamma,
                   float *out_dev);

/* Loss and its gradient w.r.t. every parameter for one batch (no update):
 * target_dev [batch][18][n^3] BF16; *loss (host, may be NULL); grad
 * (host, fh_net_param_count() floats, may be NULL). */
int fh_net_gradient(fh_net *net, int batch, const uint8_t *phase_dev, const float *gamma,
                    const uint16_t *target_dev, double *loss, float *grad);

/* One Adam step with the given gradient (host) or, if grad is NULL, the
 * one of the last fh_net_gradient / training step. */
int fh_net_adam(fh_net *net, const float *grad, const fh_adam *opt);

/* `steps` Adam steps on minibatches of `batch` samples taken from a
 * training set of nsamples: phase_dev [nsamples][n^3], gamma [nsamples]
 * (host), target_dev [nsamples][18][n^3] BF16.  order (host, steps x
 * batch) lists the samples of each step (the caller draws it).  loss
 * (host, steps entries, may be NULL) receives the loss of each step before
 * its update. */
int fh_net_train(fh_net *net, int nsamples, const uint8_t *phase_dev, const float *gamma,
                 const uint16_t *target_dev, int batch, int steps, const int *order,
                 const fh_adam *opt, double *loss);

/* Warm start of one microstructure for nload macroscopic strains E (host,
 * nload x 6 Mandel): x_dev [nload][3][n^3] FP64 receives
 * u_(0) = (length / n) sum_j E_j O_j, each component shifted to zero mean,
 * with O the network output of phase_dev (n^3) and gamma; length = cell
 * edge. */
int fh_net_guess(fh_net *net, const uint8_t *phase_dev, float gamma, int nload, const double *E,
                 double length, double *x_dev);

/* Training target of one sample from solver fluctuations: u_dev
 * [6 loads][3][n^3] FP64 for the unit Mandel strains, scale = n / l;
 * target_dev [18][n^3] BF16. */
int fh_net_pack_target(fh_net *net, const double *u_dev, double scale, uint16_t *target_dev);

/* Kernel timing with HIP events on the network's stream (on != 0 resets
 * the counters), and the accumulated figures. */
/* One layer of the network on caller-given tensors: a test hook for the
 * MFMA kernels, with the network's current parameters (weights and biases
 * rounded to BF16 as in every forward pass).  layer 0..13 in the parameter
 * order; s = n >> level of the layer; cinp = cin rounded up to 16; tensors
 * are BF16 (uint16 bit patterns) channels last [batch][s^3][channels].
 *   FH_NET_OP_FORWARD: out = BF16(leaky(conv(x) + b)), x with cinp
 *     channels (padding channels zero), out with cout channels;
 *   FH_NET_OP_DGRAD: out = BF16(conv_input_grad(dz) (x leaky'(mask) when
 *     mask is not NULL)), dz with cout channels, out and mask with cinp
 *     channels; the first layer has none (FH_EINVAL);
 *   FH_NET_OP_WGRAD: out = float[27 cout cin + cout], the gradient of the
 *     layer's weights [tap][cout][cin] and bias from x and dz (it also
 *     overwrites that layer's slice of the gradient of the last
 *     fh_net_gradient call).
 * batch <= max_batch.  Synchronises the network's stream.                 */
#define FH_NET_OP_FORWARD 0
#define FH_NET_OP_DGRAD 1
#define FH_NET_OP_WGRAD 2
int fh_net_layer(fh_net *net, int layer, int op, int batch, const uint16_t *x_dev,
                 const uint16_t *dz_dev, const uint16_t *mask_dev, void *out_dev);

int fh_net_set_timing(fh_net *net, int on);
int fh_net_get_stats(fh_net *net, fh_net_stats *stats);

#ifdef __cplusplus
}
#endif

#endif
