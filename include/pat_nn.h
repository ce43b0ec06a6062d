/*
 * pat_nn.h -- C ABI of the network layers of a learned update step.
 *
 * Not part of the paper's method: a small 3D convolutional network that maps
 * the current iterate p_k and the data-term gradient A^T C^T (C A p_k - f)
 * (eq. BP, computed by pat_adjoint) to the next iterate. These entry points
 * are its building blocks; the operator, the prox and the solver are in pat.h.
 *
 * Conventions (in addition to those of pat.h)
 *  - Activations are float32 [batch][channels][nz][ny][nx] (x fastest);
 *    convolution weights are float32 [c_out][c_in][3][3][3], biases [c_out].
 *    The convolution is a cross-correlation with one voxel of zero padding
 *    (output size = input size): y[co][z,y,x] = sum over ci and dz, dy, dx in
 *    {-1, 0, 1} of w[co][ci][dz+1][dy+1][dx+1] x[ci][z+dz, y+dy, x+dx].
 *  - Every operand of a product (activations, weights, gradients) is rounded
 *    to bfloat16 (nearest even) as it enters the matrix cores; products are
 *    summed in FP32 (weight gradients: FP32 per chunk of rows, chunks summed in
 *    FP64). Biases are added in FP32. Results are deterministic.
 *  - All pointers are device pointers unless stated otherwise, owned by the
 *    caller; `stream` is a hipStream_t (NULL: the default stream). Work is
 *    enqueued asynchronously; arguments are validated before anything is
 *    enqueued. Errors: PAT_ERR_INVALID (null pointer, non-positive size, too
 *    large), PAT_ERR_NOMEM (workspace too small), PAT_ERR_HIP (launch failed);
 *    pat_last_error() gives the message. batch = 0 enqueues nothing (the
 *    weight gradient then writes zeros).
 */
#ifndef PAT_NN_H
#define PAT_NN_H

#include <stddef.h>
#include <stdint.h>

#include "pat.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of device workspace pat_conv3d_forward and pat_conv3d_backward_input
 * need for a layer with these channel counts (0 for invalid counts): the
 * weights repacked as bfloat16 matrix-core operands. */
size_t pat_conv3d_workspace_bytes(int32_t c_in, int32_t c_out);

/* y = conv(x, w) + bias (bias may be NULL), then max(y, 0) if relu != 0.
 * x [batch][c_in][nz][ny][nx], y [batch][c_out][nz][ny][nx]; x and y must not
 * overlap. workspace: device scratch of at least pat_conv3d_workspace_bytes. */
pat_status pat_conv3d_forward(const float* x, const float* w, const float* bias, float* y, int32_t batch,
                              int32_t c_in, int32_t c_out, int32_t nz, int32_t ny, int32_t nx, int32_t relu,
                              void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): pat_conv3d_forward
 * with no workspace argument. The bfloat16-packed weights go to a device array
 * of PAT_CONV_STATIC_SCRATCH_BYTES inside the library, one per GPU, allocated
 * with the library's code and held until the process ends; nothing is
 * allocated by the call. Its device address is looked up once per GPU (first
 * call on that GPU, under a lock). Layers whose packed weights need more bytes
 * than the array holds (at most 64 (padded) input channels take the packed
 * path; e.g. 64 -> 256 channels needs 884 736 bytes) are rejected with
 * PAT_ERR_INVALID before anything is enqueued; wider inputs take the unpacked
 * path and use no scratch. Every call on one GPU shares the array and
 * overwrites it before use: calls that overlap in time on one GPU (different
 * streams or threads) race and may read each other's weights, so order them
 * (one stream, or events). Results equal pat_conv3d_forward's bit for bit. */
#define PAT_CONV_STATIC_SCRATCH_BYTES (1u << 20)
pat_status pat_conv3d_forward_static(const float* x, const float* w, const float* bias, float* y, int32_t batch,
                                     int32_t c_in, int32_t c_out, int32_t nz, int32_t ny, int32_t nx, int32_t relu,
                                     void* stream);

/* dx = gradient of sum(dy * conv(x, w)) with respect to x: the adjoint of the
 * convolution (weights transposed over channels, taps mirrored).
 * dy [batch][c_out][...], dx [batch][c_in][...] (overwritten); no overlap.
 * workspace as for pat_conv3d_forward. */
pat_status pat_conv3d_backward_input(const float* dy, const float* w, float* dx, int32_t batch, int32_t c_in,
                                     int32_t c_out, int32_t nz, int32_t ny, int32_t nx, void* workspace,
                                     size_t workspace_bytes, void* stream);

/* Bytes of device workspace pat_conv3d_backward_weight needs for these sizes
 * (0 for invalid sizes). */
size_t pat_conv3d_backward_weight_workspace_bytes(int32_t batch, int32_t c_in, int32_t c_out, int32_t nz, int32_t ny,
                                                  int32_t nx);

/* dw[co][ci][tap] = sum over batch and voxels of dy[co][v] x[ci][v + d(tap)]
 * and dbias[co] = sum of dy[co] (dbias may be NULL); both overwritten.
 * workspace: device buffer of at least the bytes above, used as scratch. */
pat_status pat_conv3d_backward_weight(const float* x, const float* dy, float* dw, float* dbias, int32_t batch,
                                      int32_t c_in, int32_t c_out, int32_t nz, int32_t ny, int32_t nx,
                                      void* workspace, size_t workspace_bytes, void* stream);

/* Resampling layers between the levels of the network. Tensors are float32
 * [channels][nz][ny][nx] with channels = batch * channels; the coarse voxel
 * (z, y, x) covers the fine voxels (2z + a, 2y + b, 2x + c), a, b, c in {0, 1}.
 * pat_pool2_*: (nz, ny, nx) is the fine grid (even sizes; the tensor read in
 * pairs, x of pool2_forward and dy of upsample2_backward, 8-byte
 * aligned); forward y = mean of the 8 children, backward dx = dy(parent) / 8.
 * pat_upsample2_*: (nz, ny, nx) is the coarse grid; forward y(child) = x,
 * backward dx = sum of dy over the 8 children. Errors: PAT_ERR_INVALID for
 * sizes, null pointers or alignment. */
pat_status pat_pool2_forward(const float* x, float* y, int64_t channels, int32_t nz, int32_t ny, int32_t nx,
                             void* stream);
pat_status pat_pool2_backward(const float* dy, float* dx, int64_t channels, int32_t nz, int32_t ny, int32_t nx,
                              void* stream);
pat_status pat_upsample2_forward(const float* x, float* y, int64_t channels, int32_t nz, int32_t ny, int32_t nx,
                                 void* stream);
pat_status pat_upsample2_backward(const float* dy, float* dx, int64_t channels, int32_t nz, int32_t ny, int32_t nx,
                                  void* stream);

/* y = a + b (b may be NULL: y = a), then max(y, 0) if relu != 0; n elements;
 * y may alias a or b. */
pat_status pat_add_act(const float* a, const float* b, float* y, int64_t n, int32_t relu, void* stream);

/* out = alpha x + beta y (y may be NULL: out = alpha x), then max(out, 0) if
 * clamp0 != 0; out may alias x or y. */
pat_status pat_axpby(const float* x, const float* y, float* out, int64_t n, float alpha, float beta, int32_t clamp0,
                     void* stream);

/* Squared-error loss of a against the target t over n elements:
 * *loss = mean((a - t)^2) as an FP64 device scalar (block partials summed in a
 * fixed order), and, if grad is not NULL, grad = 2 (a - t) / n, set to 0 where
 * a <= 0 when mask0 != 0 (the gradient through an output clamp max(0, .)).
 * workspace: device, >= pat_mse_workspace_bytes(), 8-byte aligned like loss;
 * n in [1, 2^40]. */
size_t pat_mse_workspace_bytes(void);
pat_status pat_mse(const float* a, const float* t, float* grad, int64_t n, int32_t mask0, double* loss,
                   void* workspace, size_t workspace_bytes, void* stream);

/* grad[i] = 0 where y[i] <= 0 (or NaN), in place: the ReLU's backward given its output y. */
pat_status pat_relu_backward(const float* y, float* grad, int64_t n, void* stream);

/* One Adam step on n parameters (step = 1, 2, ...): m and v are the moment
 * buffers (start at zero), updated in place with w. */
pat_status pat_adam_step(float* w, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                         float beta2, float eps, int32_t step, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PAT_NN_H */
