// Internal interface of the warm-start network (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fse.h"

namespace fse {
namespace cnn {

// Architecture: 48x48x2 input, four 3x3 stride-2 convolutions with 32
// channels (48 -> 24 -> 12 -> 6 -> 3), ReLU, then a dense head from the
// 288 features to one logit per bin of the 64x64 transform.
constexpr int kCh = 32;
constexpr int kIn = 48;
constexpr int kFeat = 3 * 3 * kCh;  // 288
constexpr int kBins = 4096;
constexpr int kPatchElems = kIn * kIn * 2;
constexpr int kSteps = kFeat / 16;  // MFMA depth steps of the head product

// Offsets (elements) of the parameter tensors in the flat parameter vector:
// conv weights [32][3][3][Cin], biases [32], head weight [4096][288], bias.
constexpr int64_t kOffW[4] = {0, 608, 9856, 19104};
constexpr int64_t kOffB[4] = {576, 9824, 19072, 28320};
constexpr int64_t kOffHeadW = 28352;
constexpr int64_t kOffHeadB = kOffHeadW + (int64_t)kBins * kFeat;
constexpr int64_t kNumParams = kOffHeadB + kBins;
constexpr int kCin[4] = {2, kCh, kCh, kCh};
constexpr int kHin[4] = {48, 24, 12, 6};
constexpr int kKdim[4] = {18, 288, 288, 288};  // 9 * Cin
constexpr int kKpad[4] = {32, 288, 288, 288};  // padded to the MFMA depth
// Saved activations per sample (BF16, post-ReLU): a1 24x24x32, a2 12x12x32,
// a3 6x6x32, a4 3x3x32.
constexpr int kActOff[5] = {0, 18432, 23040, 24192, 24480};
constexpr int kActElems = 24480;

// Kernel launchers (stream-ordered, no allocation).
hipError_t patches(const uint8_t* img, const uint8_t* avail, int64_t pitch, int32_t H, int32_t W,
                   const void* blocks /* fse_block_t */, const int32_t* orig, int32_t n, uint16_t* x,
                   hipStream_t s);
hipError_t forward(const uint16_t* x, int32_t B, const uint16_t* prm, uint16_t* feats, uint16_t* acts,
                   hipStream_t s);
// Forward pass from the frames for the n blocks of a batch, FP32 logits to
// rows orig[b] (implemented with the network's state in cnn_api.cpp).
fse_status_t net_forward_blocks(fse_cnn_t net, const uint8_t* img, const uint8_t* avail, int64_t pitch, int32_t H,
                                int32_t W, const void* blocks, const int32_t* orig, int32_t n, float* d_logits,
                                hipStream_t s);
// Network inputs built from the frames for the n blocks of a batch (class
// order) and the convolution stack, no activations; the features go to row
// orig[b] of `feats` in fragment layout (rows in blocks of 32, see
// head_frag).
hipError_t forward_blocks(const uint8_t* img, const uint8_t* avail, int64_t pitch, int32_t H, int32_t W,
                          const void* blocks, const int32_t* orig, int32_t n, const uint16_t* prm, uint16_t* feats,
                          hipStream_t s);
// Head weights (row-major [4096][288] BF16) to fragment layout (same size).
hipError_t permute_head(const uint16_t* w, uint16_t* frag, hipStream_t s);
// logits[M x 4096] = features (fragment layout, ceil(M/32) row blocks) x
// head weights (fragment layout)^T + bias; bitwise equal to gemm_nt on the
// row-major operands.
hipError_t head_frag(const uint16_t* feats_frag, const uint16_t* w_frag, const uint16_t* bias, float* logits, int32_t M,
                     hipStream_t s);
// C[M x N] (FP32, ldc) = A[M x K] * B[N x K]^T (+ bias[N]), A and B BF16 with
// K contiguous; K % 16 == 0, lda and ldb multiples of 8.
hipError_t gemm_nt(const uint16_t* A, int lda, const uint16_t* B, int ldb, float* C, int ldc,
                   const uint16_t* bias_bf16, int M, int N, int K, hipStream_t s);
hipError_t transpose_u16(const uint16_t* in, int rows, int cols, int ld_in, uint16_t* out, int ld_out,
                         hipStream_t s);
hipError_t f32_to_bf16(const float* in, int64_t n, uint16_t* out, hipStream_t s);
hipError_t im2col(const uint16_t* act, int32_t B, int layer, uint16_t* col, hipStream_t s);
hipError_t col2im(const float* dcol, int32_t B, int layer, float* dact, hipStream_t s);
hipError_t relu_mask(const float* dact, const uint16_t* act, int per_sample, int64_t act_stride, int64_t n,
                     float* dz, uint16_t* dz_bf16, hipStream_t s);
hipError_t colsum_add(const float* in, int rows, int cols, float* out, hipStream_t s);
hipError_t bce(const float* logits, const uint32_t* target_bits, int32_t B, float pos_weight, float* dlogits,
               float* loss, hipStream_t s);
hipError_t adam(float* master, float* grad, float* m, float* v, uint16_t* work, int64_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t topk(const float* logits, int32_t B, int32_t K, int16_t* cand, int32_t* flags, hipStream_t s);

}  // namespace cnn
}  // namespace fse
