/*
 * hologen_nn.h -- C ABI of the learned initialisation for hologram
 * generation on MI355X (gfx950).
 *
 * The HoloGen paper (arXiv 2008.12214) starts its iterative algorithms from
 * a random phase ("Iterative Fourier Transform Algorithms" section).  This
 * library adds a learned start: a small convolutional network predicts the
 * replay-plane phase psi of a target amplitude T, the SLM start levels are
 * the projection of the inverse transform of T e^{i psi} (Background
 * section, Eqs. fouriertrans2d5c/d; projection as in the Example section,
 * Listing 1), and a few Gerchberg-Saxton iterations refine them.  The
 * network itself is not in the paper.
 *
 * Network (fixed): U-Net encoder-decoder on NHWC bfloat16 activations with
 * FP32 accumulation (MFMA).  Encoder levels 0..3 with 16, 32, 64, 128
 * channels: two 3x3 convolutions (zero padding 1, bias, ReLU) each, 2x2
 * average pooling between levels.  Decoder levels 2, 1, 0: nearest 2x
 * upsampling, concatenation with the encoder output of that level
 * (upsampled channels first), two 3x3 convolutions with ReLU.  Head: 1x1
 * convolution to two channels (a, b); the predicted phase is arg(a + i b).
 * The input is the target scaled to unit rms per image.
 *
 * Parameter vector (FP32, hg_nn_param_count() floats): layers in the order
 * e0a e0b e1a e1b e2a e2b e3a e3b d2a d2b d1a d1b d0a d0b head, each as its
 * weights (OHWI: [cout][3][3][cin], head [2][cin]) followed by its bias
 * [cout].  Gradients use the same layout.
 *
 * Loss (per image, global-phase invariant): l = 1 - |S| / W with
 * S = sum_p amp_p z_p conj(y_p), z = (a + ib)/|a + ib|, y = label/|label|,
 * W = sum_p amp_p; the batch loss is the mean of l over the images.
 *
 * Conventions are those of hologen.h: device pointers owned by the caller,
 * work enqueued on `stream` without synchronising, nothing allocated,
 * argument checks on the host before any launch (on error nothing is
 * enqueued and hg_last_error() holds the detail), 256-byte aligned
 * workspaces whose contents are clobbered.  bf16 buffers are passed as
 * void* and hold raw bfloat16 bit patterns (uint16).
 */
#ifndef HOLOGEN_NN_H
#define HOLOGEN_NN_H

#include "hologen.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- whole network ---------------------------------------------------- */

/* Number of FP32 parameters of the network. */
long hg_nn_param_count(void);

/* Workspace of hg_nn_forward / hg_nn_backward for `batch` images of h x w
 * (h and w multiples of 8); 0 if unsupported.  It holds the packed bf16
 * weights, every activation the backward pass needs and the gradient
 * buffers, about 770 bytes per pixel. */
size_t hg_nn_workspace_size(int batch, int h, int w);

/* Forward pass.
 *   params  FP32 parameter vector
 *   target  [batch][h][w] FP32 amplitudes (centred replay plane)
 *   out     [batch][h][w][2] FP32 head output (a, b); the layout of a
 *           complex64 array, so it can be passed as an hg_complex phasor
 * Keeps the activations in `workspace` for hg_nn_backward. */
hg_status hg_nn_forward(const float* params, const float* target, int batch, int h, int w, float* out,
                        void* workspace, size_t workspace_bytes, void* stream);

/* Backward pass of the loss above; must follow hg_nn_forward with the same
 * params, shape and workspace on the same stream.
 *   out      the forward's head output
 *   label    [batch][h][w] complex, only its phase is used (0 = phase 0)
 *   amp      [batch][h][w] FP32 loss weights (the target amplitude)
 *   grads    FP32 gradient of the batch loss, parameter layout (overwritten)
 *   loss_out nullable [batch] FP32 per-image loss */
hg_status hg_nn_backward(const float* params, const float* out, const hg_complex* label, const float* amp,
                         int batch, int h, int w, float* grads, float* loss_out, void* workspace,
                         size_t workspace_bytes, void* stream);

/* Adam (Kingma and Ba) on `count` FP32 values, step >= 1:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
hg_status hg_nn_adam(float* params, const float* grads, float* m, float* v, long count, float lr, float beta1,
                     float beta2, float eps, int step, void* stream);

/* SLM start levels from a replay-plane phase:
 * levels = P_L(IDFT(uncentre(T e^{i psi}))), per image, with
 * psi = arg(phasor) + (add_quadratic ? psi0 : 0) and the quadratic phase
 * psi0 = 2 pi ((u - nx/2)^2 / nx + (v - ny/2)^2 / ny) in centred indices.
 *   phasor        nullable [batch][ny][nx] complex, centred; only its phase
 *                 is used (NULL or 0 = phase 0); hg_nn_forward's `out`
 *                 qualifies
 *   target        [batch][ny][nx] FP32 amplitude (any positive scale)
 *   slm_levels    2..256; levels_out [batch][ny][nx] uint8
 * Grid sizes as in hologen.h (Fourier holograms).  The result is a valid
 * init_levels for hg_gs / hg_wgs / hg_problem. */
size_t hg_replay_phase_init_workspace_size(int batch, int ny, int nx);
hg_status hg_replay_phase_init(const hg_complex* phasor, const float* target, int batch, int ny, int nx,
                               int slm_levels, int add_quadratic, uint8_t* levels_out, void* workspace,
                               size_t workspace_bytes, void* stream);

/* field [batch][ny][nx] (centred) *= e^{sign i psi0}, sign = +1 or -1: moves a
 * replay-plane phase to or from its residual about the quadratic phase. */
hg_status hg_quadratic_phase_apply(hg_complex* field, int batch, int ny, int nx, int sign, void* stream);

/* ---- single layers (the steps of the two passes above) ---------------- */

/* Zero-padded weight row length of a 3x3 layer with k = 9 cin taps:
 * k rounded up to a multiple of 32. */
int hg_nn_kpad(int k);

/* Pack OHWI FP32 weights w [cout][3][3][cin] into bf16 GEMM operands.
 * flip = 0: wg [cout][kpad(9 cin)], wg[co][(ky 3 + kx) cin + ci] = w[co][ky][kx][ci]
 *           (forward);
 * flip = 1: wg [cin][kpad(9 cout)], wg[ci][(ky 3 + kx) cout + co] =
 *           w[co][2-ky][2-kx][ci] (the adjoint, for the data gradient). */
hg_status hg_nn_pack_weights(const float* w, void* wg, int cout, int cin, int flip, void* stream);

/* y = bf16(mask(relu(conv3x3(x, wg) + bias))): x [n][h][w][cin] bf16, wg
 * packed with flip = 0 (or flip = 1 for the data gradient, with cin and
 * cout exchanged), bias nullable FP32 [cout], relu 0/1, mask nullable bf16
 * with y's layout (y zeroed where mask <= 0), y [n][h][w][cout] bf16.
 * cout a multiple of 16. */
hg_status hg_nn_conv3x3(const void* x, const void* wg, const float* bias, const void* mask, void* y, int n, int h,
                        int w, int cin, int cout, int relu, void* stream);

/* Weight and bias gradients of a 3x3 layer: dw [cout][3][3][cin] FP32 =
 * sum over pixels of dy (x) im2col(x); db nullable [cout] = sum over pixels
 * of dy.  x [n][h][w][cin], dy [n][h][w][cout] bf16; cout a multiple of 16
 * up to 256.  Pixel blocks reduce in a fixed order: results are
 * deterministic. */
size_t hg_nn_wgrad_workspace_size(int n, int h, int w, int cin, int cout);
hg_status hg_nn_conv3x3_wgrad(const void* x, const void* dy, float* dw, float* db, int n, int h, int w, int cin,
                              int cout, void* workspace, size_t workspace_bytes, void* stream);

/* 2x2 average pooling, x [n][h][w][c] -> y [n][h/2][w/2][c] (h, w even). */
hg_status hg_nn_avgpool2(const void* x, void* y, int n, int h, int w, int c, void* stream);

/* Its backward: dx [n][h][w][c] = bf16(dy[pooled]/4 + dskip), zeroed where
 * mask <= 0; dskip and mask nullable, with dx's layout. */
hg_status hg_nn_avgpool2_backward(const void* dy, const void* dskip, const void* mask, void* dx, int n, int h, int w,
                                  int c, void* stream);

/* out [n][h][w][c1 + c2] = (nearest 2x upsampling of lo [n][h/2][w/2][c1],
 * skip [n][h][w][c2]). */
hg_status hg_nn_upsample_concat(const void* lo, const void* skip, void* out, int n, int h, int w, int c1, int c2,
                                void* stream);

/* Its backward: dlo = bf16(sum of the four upsampled copies), zeroed where
 * mask_lo <= 0 (nullable, dlo's layout); dskip = the last c2 channels. */
hg_status hg_nn_upsample_concat_backward(const void* dout, const void* mask_lo, void* dlo, void* dskip, int n, int h,
                                         int w, int c1, int c2, void* stream);

/* 1x1 head: out[p] = (x[p] . bf16(w[0]) + b[0], x[p] . bf16(w[1]) + b[1]),
 * x [pixels][c] bf16, w [2][c] FP32, b [2], out [pixels][2] FP32. */
hg_status hg_nn_head(const void* x, const float* w, const float* b, float* out, long pixels, int c, void* stream);

/* Head backward: dx = bf16(dout . bf16(w)) zeroed where x <= 0 (x is the
 * ReLU output feeding the head); dwb [2 c + 2] = weight gradient [2][c]
 * followed by the bias gradient [2].  c <= 127. */
size_t hg_nn_head_workspace_size(int c);
hg_status hg_nn_head_backward(const float* dout, const float* w, const void* x, void* dx, float* dwb, long pixels,
                              int c, void* workspace, size_t workspace_bytes, void* stream);

/* The loss above and its gradient dout [batch][hw][2] with respect to the
 * head output; loss nullable [batch]. */
size_t hg_nn_loss_workspace_size(int batch);
hg_status hg_nn_phase_loss(const float* out, const hg_complex* label, const float* amp, float* dout, float* loss,
                           int batch, long hw, void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HOLOGEN_NN_H */
