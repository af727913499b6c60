// nn.hpp -- launchers of the convolutional surrogate kernels (k_nn.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace pfk {

// FP32 master parameter layout (weights [tap][cin][cout], tap = 3 ky + kx):
//   W1 [9][3][32], b1 [32], W2 [9][32][32], b2 [32], W3 [9][32][32], b3 [32], W4 [9][32], b4
struct NNOffsets {
    int w1, b1, w2, b2, w3, b3, w4, b4, total;
};
// bf16 matrix-core B fragments: forward layers 1..3, input-gradient layers 2..3
struct NNFragOffsets {
    int f1, f2, f3, d2, d3, total;
};

NNOffsets nn_offsets();
NNFragOffsets nn_frag_offsets();
int nn_conv_blocks(int B, int H, int W);
int nn_wgrad_blocks(int B, int H, int W);
int nn_out_wgrad_blocks(int B, int H, int W);

void nn_prep_weights(const float* params, unsigned short* frag, unsigned short* w4, hipStream_t s);
void nn_pack_input(const float* c, const float* M, const float* kappa, unsigned short* a0, int B,
                   int HW, hipStream_t s);
// hidden layer `layer` (1..3): mode 0 forward (bias + relu), mode 1 input gradient (relu mask)
void nn_conv(int layer, int mode, const unsigned short* in, const unsigned short* frag,
             const float* bias, const unsigned short* mask, unsigned short* out, int B, int H, int W,
             hipStream_t s);
// the first two layers (forward) from the c, M, kappa planes, the first computed
// inside the second's tiles (a1 is not stored); w1, b1: the FP32 W1, b1
void nn_conv12_planes(const float* c, const float* M, const float* kappa, const float* w1, const float* b1,
                      const unsigned short* frag2, const float* bias2, unsigned short* out, int B, int H,
                      int W, hipStream_t s);
// the last hidden layer (forward) followed by the output layer's channel contraction:
// P[tap][p] = sum_ci W4[tap][ci] a3[p][ci] (FP32, 9 planes of B H W); a3 is not stored
void nn_conv3_taps(const unsigned short* in, const unsigned short* frag, const float* bias,
                   const unsigned short* w4, float* P, int B, int H, int W, hipStream_t s);
// d = b4 + sum_tap P[tap][p + tap], then c_hat = c + d - mean(d) per sample
// (part: B ceil(H W / 256) doubles; mean: B doubles, used where c, d, c_hat are not
// 16-byte aligned)
void nn_out_taps_project(const float* P, const float* params, const float* c, float* d, double* part,
                         double* mean, float* chat, int B, int H, int W, hipStream_t s);
// weight gradient partials of hidden layer `layer` (part: blocks x 9 x 32 x 32, partb: blocks x 32)
void nn_wgrad(int layer, const unsigned short* ain, const unsigned short* g, float* part, float* partb,
              int B, int H, int W, hipStream_t s);
// out[i] = sum over nb blocks of part[block][i]
void nn_sum_partials(const float* part, int nb, int n, float* out, hipStream_t s);
void nn_out_fwd(const unsigned short* a3, const unsigned short* w4, const float* params, float* d,
                int B, int H, int W, hipStream_t s);
void nn_sample_mean(const float* x, double* part, double* mean, int B, int HW, hipStream_t s);
void nn_project(const float* c, const float* d, const double* mean, const float* tgt, float* chat,
                float* g, float* r2, int B, int HW, hipStream_t s);
void nn_center(float* g, const double* mean, int B, int HW, hipStream_t s);
// output layer: input gradient (relu-masked, bf16) and weight-gradient partials (blocks x 289)
void nn_out_bwd(const unsigned short* a3, const unsigned short* w4, const float* g,
                unsigned short* ga3, float* part, int B, int H, int W, hipStream_t s);
void nn_adam(float* p, float* m, float* v, const float* g, int n, int t, double lr, double b1,
             double b2, double eps, hipStream_t s);
// residual check of a surrogate jump: out[3 b + 0..2] = (rho, sum(c_hat - c_prev),
// ||c_hat - c_prev|| / (K dt)); part: 3 B ceil(HW / 256) doubles
void nn_check(const float* chat, const float* cprev, const float* cstep, int B, int HW, double kdt,
              double dt, double* part, double* out, hipStream_t s);
// extract the first-layer gradient dW1[tap][ci < 3][co] from a [9][32][32] tile
void nn_extract_w1(const float* tile, float* dw1, hipStream_t s);

}  // namespace pfk
