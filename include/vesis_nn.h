/* vesis_nn.h - layers of the learned warm start (a 3-D U-Net on the cell
 * grid that predicts the equilibrium labels from the atoms), as stateless
 * HIP kernels for gfx950 behind a C ABI.
 *
 * The warm start is not part of the paper: the paper starts the level-set
 * relaxation from a loose or tight sphere (Sec. "Initial surfaces"); here
 * a network trained on labels the relaxation itself produced gives a start
 * closer to the equilibrium, and the relaxation (vesis_minimize_interface)
 * always finishes from it.
 *
 * Conventions.  Every pointer is device memory; `stream` is a hipStream_t
 * (NULL = the default stream); work is enqueued asynchronously on it and
 * nothing allocates.  Activations are BF16 (__bf16, 2 bytes) in channels-
 * last order: element (b, z, y, x, c) of an (n, d, h, w, C) tensor is at
 * (((b d + z) h + y) w + x) C + c.  Convolution weights are (27, Cout, Cin)
 * with tap = 9 (dz+1) + 3 (dy+1) + (dx+1); FP32 master weights, BF16 copies
 * for compute.  Calls return 0, VESIS_NN_E_ARG for a bad argument (nothing
 * launched) or VESIS_NN_E_DEVICE when a launch failed. */
#ifndef VESIS_NN_H
#define VESIS_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VESIS_NN_E_ARG (-1)
#define VESIS_NN_E_DEVICE (-6)
#define VESIS_NN_E_SCRATCH (-7)

/* y = [relu](conv3x3x3(x, w) + bias), zero padding, stride 1: an implicit
 * GEMM on the BF16 matrix cores with FP32 accumulation.  x: (n,d,h,w,cin)
 * BF16, w: (27,cout,cin) BF16, bias: cout FP32 or NULL, y: (n,d,h,w,cout)
 * BF16.  cin % 16 == 0, cout % 32 == 0.  With the flipped, transposed
 * weights of vesis_nn_prep_weights and no bias this is also the data
 * gradient of a convolution. */
int vesis_nn_conv3_fwd(void* stream, const void* x, const void* w, const float* bias, void* y,
                       int n, int d, int h, int wd, int cin, int cout, int relu);

/* y = [relu](conv3x3x3([up2(a) | b], w) + bias): the convolution of the
 * channel concatenation of a, upsampled 2x by nearest neighbour, and b,
 * read in place (no upsampled or concatenated tensor is formed; for
 * inference, where the decoder's inputs need not be kept).  a:
 * (n, d/2, h/2, w/2, ca), b: (n, d, h, w, cb), w: (27, cout, ca + cb),
 * y: (n, d, h, w, cout), all BF16.  ca % 16 == 0, cb % 16 == 0,
 * cout % 32 == 0, d, h, w even and w >= 16.  The result equals, bit for
 * bit, vesis_nn_conv3_fwd of vesis_nn_concat(vesis_nn_up2(a), b). */
int vesis_nn_conv3_fwd_upcat(void* stream, const void* a, int ca, const void* b, int cb,
                             const void* w, const float* bias, void* y, int n, int d, int h,
                             int wd, int cout, int relu);

/* Bytes of FP32 scratch vesis_nn_conv3_wgrad needs (one partial weight
 * gradient per chunk of 8192 positions, and per-channel partial sums for
 * the bias gradient). */
int vesis_nn_wgrad_workspace(int n, int d, int h, int wd, int cin, int cout, size_t* bytes);

/* Weight gradient dw (27,cout,cin FP32, overwritten) = sum over positions
 * of dy x shifted, on the matrix cores, chunk partials in ws summed in a
 * fixed order; db (cout FP32, overwritten; may be NULL) = sum of dy.
 * cin % 32 == 0, cout % 32 == 0.  dy is the gradient at the convolution's
 * output before any ReLU (see vesis_nn_relu_bwd). */
int vesis_nn_conv3_wgrad(void* stream, const void* x, const void* dy, float* dw, float* db,
                         float* ws, size_t ws_bytes, int n, int d, int h, int wd, int cin,
                         int cout);

/* From FP32 master weights w32 (27,cout,cin): wf = BF16 copy (same layout),
 * wb = BF16 (27,cin,cout) with wb[26-t][ci][co] = w32[t][co][ci], the
 * weights of the data gradient. */
int vesis_nn_prep_weights(void* stream, const float* w32, int cout, int cin, void* wf, void* wb);

/* dpre = dy where y > 0, else 0 (y = relu output); count elements. */
int vesis_nn_relu_bwd(void* stream, const void* y, const void* dy, void* dpre, int64_t count);

/* 2x2x2 average pooling of x (n,d,h,w,c) into y (n,d/2,h/2,w/2,c); with
 * backward != 0, x is the gradient at the pooled size and y receives the
 * gradient at the full size (d, h, w even). */
int vesis_nn_pool2(void* stream, const void* x, void* y, int n, int d, int h, int wd, int c,
                   int backward);

/* Nearest 2x upsampling to (n,d,h,w,c) from half size; with backward != 0,
 * x is the full-size gradient and y receives the half-size gradient. */
int vesis_nn_up2(void* stream, const void* x, void* y, int n, int d, int h, int wd, int c,
                 int backward);

/* y (p, ca+cb) = [a (p,ca) | b (p,cb)]; and the adjoint: da = dy[:, :ca],
 * db = dy[:, ca:] (added to db when accumulate_b != 0). */
int vesis_nn_concat(void* stream, const void* a, int ca, const void* b, int cb, void* y, int64_t p);
int vesis_nn_split(void* stream, const void* dy, int ca, int cb, void* da, void* db,
                   int accumulate_b, int64_t p);

/* y = a + b elementwise (BF16, summed in FP32); y may alias a or b. */
int vesis_nn_add(void* stream, const void* a, const void* b, void* y, int64_t count);

/* 1x1x1 head: logits (p FP32) = x (p,c) . w (c FP32) + b (1 FP32); and its
 * adjoint: dx (BF16) = dlogit w, dw = sum_p dlogit x, db = sum_p dlogit,
 * with FP32 scratch ws of at least 4 c ceil(p / 1024) bytes. */
int vesis_nn_head_fwd(void* stream, const void* x, const float* w, const float* b, float* logits,
                      int64_t p, int c);
int vesis_nn_head_bwd(void* stream, const float* dlogit, const void* x, const float* w, void* dx,
                      float* dw, float* db, float* ws, size_t ws_bytes, int64_t p, int c);

/* vesis_nn_head_bwd without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, serving loops,
 * harnesses that forbid hipMalloc): the channel partials go to a static
 * device array of the library (1 MiB per GPU, kept until the process ends),
 * so nothing is allocated.  Same kernels and summation order as
 * vesis_nn_head_bwd, hence the same results bit for bit.  Limit:
 * c * ceil(p / 1024) <= 262144 (e.g. c = 32 and p up to 8,388,608
 * positions), else VESIS_NN_E_SCRATCH and nothing is launched.  `stream`
 * must belong to the current device.  Calls that overlap on one GPU share
 * the array and race; every call overwrites the partials it reads, so no
 * state carries from one call to the next. */
int vesis_nn_head_bwd_noalloc(void* stream, const float* dlogit, const void* x, const float* w,
                              void* dx, float* dw, float* db, int64_t p, int c);

/* Mean binary cross-entropy of logits against labels (int8 per cell, -1 =
 * solute = target 1, +1 = solvent = target 0), solute cells weighted by
 * pos_weight: dlogit (p FP32) = its gradient, *loss (device FP64) = its
 * value (nblocks partial sums in `partial`, 1..4096). */
int vesis_nn_bce(void* stream, const float* logits, const int8_t* labels, int64_t p,
                 float pos_weight, float* dlogit, double* partial, int nblocks, double* loss);

/* Adam step on FP32 parameters (step counts from 1). */
int vesis_nn_adam(void* stream, float* w, const float* g, float* m, float* v, int64_t count,
                  float lr, float b1, float b2, float eps, int step);

/* Input features on a grid of n^3 cells of edge h centred at center[3]
 * (cell centres as in vesis_set_grid): x (n^3, c) BF16 with channel 0 =
 * sum_i exp(-|x - r_i|^2 / (2 s_i^2)), channel 1 = sum_i q_i exp(...),
 * s_i = sigma_i / 2 (cut at 4 s_i), other channels 0.  pos4: na x 4 FP64
 * (x, y, z, unused), sigma, q: na FP64.  c >= 2. */
int vesis_nn_featurize(void* stream, const double* pos4, const double* sigma, const double* q,
                       int64_t na, int n, double h, const double* center, int c, void* x);

#ifdef __cplusplus
}
#endif

#endif
