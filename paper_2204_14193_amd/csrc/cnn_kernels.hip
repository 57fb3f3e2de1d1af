// Warm-start network kernels for gfx950: BF16 storage, FP32 accumulation.
//
// Dense contractions (the four convolutions and the head, forward and
// backward) run on v_mfma_f32_32x32x16_bf16. Its operand layout: lane l
// supplies 8 consecutive K elements k = 8*(l/32)+i of row l%32 of A (M x K)
// and of column l%32 of B (K x N); accumulator i of lane l holds
// D[8*(i/4) + 4*(l/32) + i%4][l%32].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "cnn_internal.h"
#include "fse.h"

namespace fse {
namespace cnn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16, round to nearest even (NaN stays NaN): the hardware
// conversion of gfx950 (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

__device__ __forceinline__ int drow(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

// Sum over the 64 lanes of a wave, the same value in every lane.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xf, 0xf, false);  // row_half_mirror
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xf, 0xf, false);  // row_mirror
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// ------------------------------------------------------------------ patches
// Network input of block `b` (48x48 area) into `out` (one word per pixel:
// the two BF16 channels; rows of 48 words, or rows of `grid` words from
// (1, 1) on), by the 256 threads of a workgroup; `red` is 8 words of LDS.
// Channel 0 = (s - mean over A)/64 on A, channel 1 = 1 on A.
__device__ __forceinline__ void build_input(const uint8_t* img, const uint8_t* avail, int64_t pitch, int H, int W,
                                            const fse_block_t& bd, uint32_t* out, uint32_t (*red)[4], int t,
                                            int grid = 0) {
  const int bo = bd.border;
  const int ya = bd.y0 - bo, xa = bd.x0 - bo;
  const uint8_t* im = img + (int64_t)bd.frame * H * pitch;
  const uint8_t* av = avail + (int64_t)bd.frame * H * pitch;
  // pixel values and counts are integers, so their sums are exact in any order
  uint32_t sum = 0, cnt = 0;
  uint32_t sv[9];
  bool ia[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const int e = t + 256 * r;
    const int m = e / kIn, c = e % kIn;
    const int y = ya + m, xx = xa + c;
    const bool inB = m >= bo && m < bo + bd.bh && c >= bo && c < bo + bd.bw;
    const bool inside = !inB && y >= 0 && y < H && xx >= 0 && xx < W;
    const int64_t p = (int64_t)min(max(y, 0), H - 1) * pitch + min(max(xx, 0), W - 1);
    const uint32_t a = av[p], s = im[p];
    ia[r] = inside && a != 0;
    sv[r] = s;
    sum += ia[r] ? s : 0u;
    cnt += ia[r] ? 1u : 0u;
  }
  sum = wave_sum_u32(sum);
  cnt = wave_sum_u32(cnt);
  if ((t & 63) == 0) {
    red[0][t >> 6] = sum;
    red[1][t >> 6] = cnt;
  }
  __syncthreads();
  const uint32_t S = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  const uint32_t N = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  const float mu = N > 0 ? (float)S / (float)N : 0.f;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const int e = t + 256 * r;
    const int o = grid ? (e / kIn + 1) * grid + e % kIn + 1 : e;  // dense rows, or the guarded grid
    out[o] = ia[r] ? ((uint32_t)f2bf((sv[r] - mu) * (1.0f / 64.0f)) | (0x3f80u << 16)) : 0u;
  }
}

__global__ __launch_bounds__(256) void k_patches(const uint8_t* img, const uint8_t* avail, int64_t pitch, int H,
                                                 int W, const fse_block_t* blocks, const int32_t* orig, int n,
                                                 uint16_t* x) {
  __shared__ uint32_t red[2][4];
  const int b = blockIdx.x;
  if (b >= n) return;
  build_input(img, avail, pitch, H, W, blocks[b], reinterpret_cast<uint32_t*>(x + (int64_t)orig[b] * kPatchElems),
              red, threadIdx.x);
}

// ------------------------------------------------------------------ forward
// Layouts in LDS. A layer's input sits on a (H+1) x (H+1) grid whose row 0
// and column 0 are zero, the pixel (y, x) at (y+1, x+1): the taps of a 3x3
// stride-2 convolution with padding 1 then never leave the grid, and every
// A-operand read is a per-lane base plus a compile-time offset. The network
// input (2 channels) is one 32-bit word per grid point; 32-channel
// activations are four planes of 8 channels (16 bytes per grid point per
// plane), so that the stride-2 reads of consecutive lanes fall 32 bytes
// apart across the LDS banks.
template <int G>
__device__ __forceinline__ constexpr int plane_elems() { return G * G * 8; }

// Zero row 0 and column 0 of the four planes of a G x G grid.
template <int G>
__device__ __forceinline__ void zero_guard(uint16_t* buf, int t) {
  constexpr int PER = 2 * G - 1;
  for (int i = t; i < 4 * PER; i += 256) {
    const int g = i / PER, j = i % PER;
    const int px = j < G ? j : (j - G + 1) * G;
    reinterpret_cast<uint4*>(buf + g * plane_elems<G>())[px] = make_uint4(0u, 0u, 0u, 0u);
  }
}

// Weights of one layer as MFMA A fragments: lane l holds output channel
// l & 31 and depth values 16 ks + 8 (l >> 5) .. + 8 of step ks, and the
// biases of the output channels its accumulators hold (8 g + 4 (l >> 5) +
// 0..3 for g = 0..3), as BF16.
struct LayerW {
  uint4 w[18];
  uint2 b[4];
};

template <int CIN>
__device__ __forceinline__ void load_layer(const uint16_t* w, const uint16_t* bias, LayerW& L, int lane) {
  constexpr int K = 9 * CIN, KS = (K + 15) / 16;
  const int n = lane & 31, h = lane >> 5;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k0 = ks * 16 + 8 * h;
    if constexpr (CIN == kCh) {
      L.w[ks] = *reinterpret_cast<const uint4*>(w + n * K + k0);
    } else {
      uint32_t b4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 2 * q;
        const uint32_t lo = k < K ? w[n * K + k] : 0u;
        const uint32_t hi = k + 1 < K ? w[n * K + k + 1] : 0u;
        b4[q] = lo | (hi << 16);
      }
      L.w[ks] = make_uint4(b4[0], b4[1], b4[2], b4[3]);
    }
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) L.b[g] = *reinterpret_cast<const uint2*>(bias + 8 * g + 4 * h);
}

__device__ __forceinline__ uint32_t relu_pack(float a, float b) {
  return (uint32_t)f2bf(fmaxf(a, 0.f)) | ((uint32_t)f2bf(fmaxf(b, 0.f)) << 16);
}

// One 3x3 stride-2 convolution with bias and ReLU as an implicit GEMM:
// D[channel][pixel] = W[channel][depth] X[depth][pixel], depth = (tap,
// input channel), pixels in tiles of 32 (tile = wave, wave + 4, ... run two
// at a time). Each lane of the result holds one pixel and 16 output
// channels, 4 consecutive ones per 8-channel plane, stored as one 8-byte
// write per plane. The output goes to a guarded grid (PAD) or, for the last
// layer, to an unguarded 3x3 planar buffer.
template <int CIN, int HIN, bool PAD>
__device__ __forceinline__ void conv_layer(const uint16_t* in, uint16_t* out, const LayerW& L, int t) {
  constexpr int HO = HIN / 2, P = HO * HO, K = 9 * CIN, KS = (K + 15) / 16;
  constexpr int MT = (P + 31) / 32;
  constexpr int G = HIN + 1;            // input grid
  constexpr int GO = HO + 1;            // output grid (PAD)
  const int lane = t & 63, wave = t >> 6;
  const int h = lane >> 5;              // which 8 of the 16 depth values of a step
  // grid index of tap (0, 0) of the output pixel in column `lane & 31` of a
  // tile (columns past the end repeat the last pixel; they are not stored)
  auto base_of = [&](int tile) {
    const int m = min(tile * 32 + (lane & 31), P - 1);
    return 2 * (m / HO) * G + 2 * (m % HO);
  };
  auto gather = [&](int base, int ks) -> uint4 {
    if constexpr (CIN == kCh) {
      // step ks: tap ks/2, input channels (ks & 1)*16 + 8h .. +8, i.e. plane (ks & 1)*2 + h
      const int tap = ks >> 1;
      const uint16_t* p = in + ((ks & 1) * 2 + h) * plane_elems<G>() + (base + (tap / 3) * G + tap % 3) * 8;
      return *reinterpret_cast<const uint4*>(p);
    } else {
      // step ks, word q: tap 8*ks + 4h + q (both input channels), zero past tap 8
      const uint32_t* gw = reinterpret_cast<const uint32_t*>(in);
      uint32_t a4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t0 = 8 * ks + q, t1 = 8 * ks + 4 + q;  // the tap for h = 0 and h = 1
        const int o0 = t0 < 9 ? (t0 / 3) * G + t0 % 3 : 0;
        const int o1 = t1 < 9 ? (t1 / 3) * G + t1 % 3 : 0;
        const uint32_t v = gw[base + (h ? o1 : o0)];
        a4[q] = (h ? t1 < 9 : t0 < 9) ? v : 0u;
      }
      return make_uint4(a4[0], a4[1], a4[2], a4[3]);
    }
  };
  auto store = [&](int tile, const f32x16& acc) {
    const int p = tile * 32 + (lane & 31);
    if (p >= P) return;
    const int px = PAD ? (p / HO + 1) * GO + p % HO + 1 : p;
    constexpr int PE = PAD ? plane_elems<GO>() : P * 8;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const uint2 bb = L.b[g];
      const uint2 v = make_uint2(relu_pack(acc[4 * g] + bf2f(bb.x & 0xffff), acc[4 * g + 1] + bf2f(bb.x >> 16)),
                                 relu_pack(acc[4 * g + 2] + bf2f(bb.y & 0xffff), acc[4 * g + 3] + bf2f(bb.y >> 16)));
      *reinterpret_cast<uint2*>(out + g * PE + px * 8 + 4 * h) = v;
    }
  };
  for (int tile = wave; tile < MT; tile += 8) {
    const int tile2 = tile + 4;
    const int b1 = base_of(tile);
    f32x16 acc = {}, acc2 = {};
    if (tile2 < MT) {
      const int b2 = base_of(tile2);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const uint4 a1 = gather(b1, ks), a2 = gather(b2, ks);
        acc = mfma(L.w[ks], a1, acc);
        acc2 = mfma(L.w[ks], a2, acc2);
      }
      store(tile, acc);
      store(tile2, acc2);
    } else {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) acc = mfma(L.w[ks], gather(b1, ks), acc);
      store(tile, acc);
    }
  }
}

// A guarded planar 32-channel activation (H x H pixels) to NHWC in global
// memory.
template <int H>
__device__ __forceinline__ void copy_act_nhwc(const uint16_t* src, uint16_t* dst, int t) {
  constexpr int G = H + 1;
  for (int i = t; i < H * H * 4; i += 256) {
    const int px = i >> 2, g = i & 3;
    const int y = px / H, x = px % H;
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[g * G * G + (y + 1) * G + x + 1];
  }
}

// The whole convolution stack for one sample per workgroup, activations in
// LDS; writes the 288 features and, for training, every activation (NHWC).
// Two regions: X holds the input grid (49 x 49 words), then layer 2's
// output grid; Y holds layer 1's output grid, then layer 3's and layer 4's
// outputs. On entry the input grid (with its zero guard) is in X.
constexpr int kGridIn = kIn + 1;                                     // 49
constexpr int kXElems = 4 * 13 * 13 * 8;                             // layer-2 output grid, the larger user of X
constexpr int kYElems = 4 * 25 * 25 * 8;                             // layer-1 output grid
static_assert(kGridIn * kGridIn * 2 <= kXElems, "input grid fits region X");
constexpr int kA4Off = 4 * 7 * 7 * 8;                                // layer-4 output after layer 3's grid

// Number of 32-pixel tiles of the layer with input size HIN: the waves
// below it run the layer and load its weights.
constexpr int tiles_of(int hin) { return ((hin / 2) * (hin / 2) + 31) / 32; }

// Weights of layers 1 and 2, loaded before the input is built so that
// their latency overlaps it.
__device__ __forceinline__ void load_first_layers(const uint16_t* prm, LayerW& L1, LayerW& L2, int t) {
  const int lane = t & 63;
  load_layer<2>(prm + kOffW[0], prm + kOffB[0], L1, lane);
  load_layer<kCh>(prm + kOffW[1], prm + kOffB[1], L2, lane);
}

// Each later layer's weights are requested before the barrier that ends
// the previous layer. Returns the 3x3x32 features (planar: 8-channel plane
// g of pixel px at 72 g + 8 px), complete in LDS for every thread.
__device__ __forceinline__ const uint16_t* conv_stack(uint16_t* X, uint16_t* Y, const uint16_t* prm,
                                                      const LayerW& L1, const LayerW& L2, uint16_t* dst, int t) {
  const int lane = t & 63, wave = t >> 6;
  uint16_t* const a4 = Y + kA4Off;
  conv_layer<2, 48, true>(X, Y, L1, t);
  __syncthreads();
  if (dst) copy_act_nhwc<24>(Y, dst + kActOff[0], t);
  zero_guard<13>(X, t);  // the input grid is no longer read
  conv_layer<kCh, 24, true>(Y, X, L2, t);
  LayerW L3;
  if (wave < tiles_of(12)) load_layer<kCh>(prm + kOffW[2], prm + kOffB[2], L3, lane);
  __syncthreads();
  if (dst) copy_act_nhwc<12>(X, dst + kActOff[1], t);
  zero_guard<7>(Y, t);   // layer 1's grid is no longer read
  conv_layer<kCh, 12, true>(X, Y, L3, t);
  LayerW L4;
  if (wave < tiles_of(6)) load_layer<kCh>(prm + kOffW[3], prm + kOffB[3], L4, lane);
  __syncthreads();
  if (dst) copy_act_nhwc<6>(Y, dst + kActOff[2], t);
  conv_layer<kCh, 6, false>(Y, a4, L4, t);
  __syncthreads();
  return a4;
}

// Zero guard (row 0, column 0) of the 49 x 49 input grid of words.
__device__ __forceinline__ void zero_input_guard(uint32_t* grid, int t) {
  for (int i = t; i < 2 * kGridIn - 1; i += 256) grid[i < kGridIn ? i : (i - kGridIn + 1) * kGridIn] = 0u;
}

// Three workgroups per compute unit (the LDS allows three): at most 168
// registers per lane.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_forward(const uint16_t* x, int B, const uint16_t* prm, uint16_t* feats,
                                                 uint16_t* acts) {
  __shared__ __align__(16) uint16_t X[kXElems];
  __shared__ __align__(16) uint16_t Y[kYElems];
  const int b = blockIdx.x;
  if (b >= B) return;
  const int t = threadIdx.x;
  uint32_t* const grid = reinterpret_cast<uint32_t*>(X);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(x + (int64_t)b * kPatchElems);
  for (int e = t; e < kIn * kIn; e += 256) grid[(e / kIn + 1) * kGridIn + e % kIn + 1] = src[e];
  LayerW L1, L2;
  load_first_layers(prm, L1, L2, t);
  zero_input_guard(grid, t);
  zero_guard<25>(Y, t);
  __syncthreads();
  uint16_t* const dst = acts ? acts + (int64_t)b * kActElems : nullptr;
  const uint16_t* a4 = conv_stack(X, Y, prm, L1, L2, dst, t);
  for (int i = t; i < kFeat; i += 256) {
    const int px = i / kCh, c = i % kCh;
    const uint16_t v = a4[(c >> 3) * (9 * 8) + px * 8 + (c & 7)];
    feats[(int64_t)b * kFeat + i] = v;
    if (dst) dst[kActOff[3] + i] = v;
  }
}

// The same with the input of block b built in LDS straight from the frames;
// the features go to row orig[b] of a matrix in fragment layout (see
// k_head_frag).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_forward_blocks(const uint8_t* img, const uint8_t* avail, int64_t pitch,
                                                        int H, int W, const fse_block_t* blocks,
                                                        const int32_t* orig, int n, const uint16_t* prm,
                                                        uint16_t* feats) {
  __shared__ __align__(16) uint16_t X[kXElems];
  __shared__ __align__(16) uint16_t Y[kYElems];
  __shared__ uint32_t red[2][4];
  const int b = blockIdx.x;
  if (b >= n) return;
  const int t = threadIdx.x;
  uint32_t* const grid = reinterpret_cast<uint32_t*>(X);
  LayerW L1, L2;
  load_first_layers(prm, L1, L2, t);
  build_input(img, avail, pitch, H, W, blocks[b], grid, red, t, kGridIn);
  zero_input_guard(grid, t);
  zero_guard<25>(Y, t);
  __syncthreads();
  const uint16_t* a4 = conv_stack(X, Y, prm, L1, L2, nullptr, t);
  // features to row r = orig[b] of the fragment layout: 8 features (one
  // 8-channel plane of one pixel) per 16-byte piece
  if (t < kFeat / 8) {
    const int r = orig[b], s16 = t >> 1, h = t & 1;
    const uint4 v = *reinterpret_cast<const uint4*>(a4 + (t & 3) * 72 + (t >> 2) * 8);
    reinterpret_cast<uint4*>(feats)[((int64_t)(r >> 5) * kSteps + s16) * 64 + h * 32 + (r & 31)] = v;
  }
}

// ------------------------------------------------------------------ GEMM
// C = A * B^T: each wave computes one 32x32 tile, a workgroup 64x64.
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t* A, int lda, const uint16_t* Bm, int ldb, float* C,
                                                 int ldc, const uint16_t* bias, int M, int N, int K) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int tm = blockIdx.x * 64 + (wave & 1) * 32;
  const int tn = blockIdx.y * 64 + (wave >> 1) * 32;
  if (tm >= M || tn >= N) return;
  const int m = tm + (lane & 31), n = tn + (lane & 31);
  const int kh = 8 * (lane >> 5);
  const uint16_t* pa = A + (int64_t)m * lda + kh;
  const uint16_t* pb = Bm + (int64_t)n * ldb + kh;
  const bool ma = m < M, nb = n < N;
  f32x16 acc = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    const uint4 av = ma ? *reinterpret_cast<const uint4*>(pa + k0) : make_uint4(0u, 0u, 0u, 0u);
    const uint4 bv = nb ? *reinterpret_cast<const uint4*>(pb + k0) : make_uint4(0u, 0u, 0u, 0u);
    acc = mfma(av, bv, acc);
  }
  const int col = tn + (lane & 31);
  if (col >= N) return;
  const float bb = bias ? bf2f(bias[col]) : 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = tm + drow(i, lane);
    if (row < M) C[(int64_t)row * ldc + col] = acc[i] + bb;
  }
}

// C = A * B^T for large outputs: each wave computes WM x WN tiles of 32x32
// (A and B fragments reused across them), a workgroup 2x2 waves. Same
// arithmetic per element as k_gemm_nt (one MFMA chain over K in steps of 16).
template <int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm_nt_t(const uint16_t* A, int lda, const uint16_t* Bm, int ldb, float* C,
                                                   int ldc, const uint16_t* bias, int M, int N, int K) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int tm = blockIdx.x * (64 * WM) + (wave & 1) * (32 * WM);
  const int tn = blockIdx.y * (64 * WN) + (wave >> 1) * (32 * WN);
  if (tm >= M || tn >= N) return;
  const int kh = 8 * (lane >> 5);
  const uint16_t* pa[WM];
  const uint16_t* pb[WN];
  bool ma[WM], nb[WN];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    const int m = tm + 32 * i + (lane & 31);
    ma[i] = m < M;
    pa[i] = A + (int64_t)(ma[i] ? m : 0) * lda + kh;
  }
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int n = tn + 32 * j + (lane & 31);
    nb[j] = n < N;
    pb[j] = Bm + (int64_t)(nb[j] ? n : 0) * ldb + kh;
  }
  f32x16 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x16{};
  // Two register stages: the operands of the next depth step are loaded
  // before the current step multiplies (scheduling barriers keep that
  // order). The loads are unconditional (rows and columns past the edge
  // read row 0 and are never stored; a step past the end re-reads the last
  // one), so no branch forces a wait for all outstanding loads.
  uint4 a0[WM], b0[WN], a1[WM], b1[WN];
  auto load = [&](uint4 (&av)[WM], uint4 (&bv)[WN], int k0) {
    const int kk = min(k0, K - 16);
#pragma unroll
    for (int i = 0; i < WM; ++i) av[i] = *reinterpret_cast<const uint4*>(pa[i] + kk);
#pragma unroll
    for (int j = 0; j < WN; ++j) bv[j] = *reinterpret_cast<const uint4*>(pb[j] + kk);
  };
  auto mma = [&](const uint4 (&av)[WM], const uint4 (&bv)[WN]) {
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = mfma(av[i], bv[j], acc[i][j]);
  };
  load(a0, b0, 0);
  int k0 = 0;
  for (; k0 + 16 < K; k0 += 32) {
    load(a1, b1, k0 + 16);
    __builtin_amdgcn_sched_barrier(0);
    mma(a0, b0);
    load(a0, b0, k0 + 32);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, b1);
  }
  if (k0 < K) mma(a0, b0);  // an odd number of steps leaves the last in stage 0
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int col = tn + 32 * j + (lane & 31);
    if (col >= N) continue;
    const float bb = bias ? bf2f(bias[col]) : 0.f;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tm + 32 * i + drow(r, lane);
        if (row < M) C[(int64_t)row * ldc + col] = acc[i][j][r] + bb;
      }
  }
}

// ------------------------------------------------------------------ head
// Fragment layout of a matrix with 288 columns (the depth of the head
// product): rows in blocks of 32, and for block rb, depth step s (16
// columns) and lane l, the 16 bytes that lane l of an MFMA operand reads in
// step s: row 32 rb + (l & 31), columns 16 s + 8 (l >> 5) .. + 8, at uint4
// index (rb * 18 + s) * 64 + l. Each fragment read of a wave is then one
// contiguous 1 KiB.

// Head weights [4096][288] (row-major) to fragment layout.
__global__ __launch_bounds__(256) void k_permute_head(const uint16_t* w, uint4* frag) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kBins / 32 * kSteps * 64) return;
  const int l = i & 63, s16 = (i >> 6) % kSteps, cb = (i >> 6) / kSteps;
  frag[i] = *reinterpret_cast<const uint4*>(w + (int64_t)(cb * 32 + (l & 31)) * kFeat + 16 * s16 + 8 * (l >> 5));
}

// logits[M x 4096] (FP32, row-major) = F W^T + bias with F [M x 288] and the
// head weights W [4096 x 288] both in fragment layout (F with
// ceil(M / 32) row blocks). Workgroup tile 128 x 128, each wave 64 x 64
// (2 x 2 MFMA tiles of 32 x 32); the same arithmetic per element as
// k_gemm_nt (one MFMA chain over the depth in steps of 16, then the bias).
__global__ __launch_bounds__(256) void k_head_frag(const uint4* F, const uint4* Wf, const uint16_t* bias,
                                                   float* C, int M) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int rb0 = blockIdx.x * 4 + (wave & 1) * 2;   // row blocks rb0, rb0 + 1
  const int cb0 = blockIdx.y * 4 + (wave >> 1) * 2;  // column blocks
  const int nrb = (M + 31) >> 5;
  if (rb0 >= nrb) return;
  const int rb1 = min(rb0 + 1, nrb - 1);             // a block past the end repeats the last (never stored)
  const uint4* pa0 = F + (int64_t)rb0 * kSteps * 64 + lane;
  const uint4* pa1 = F + (int64_t)rb1 * kSteps * 64 + lane;
  const uint4* pb0 = Wf + (int64_t)cb0 * kSteps * 64 + lane;
  const uint4* pb1 = pb0 + kSteps * 64;
  f32x16 acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
  uint4 a0[2], b0[2], a1[2], b1[2];
  auto load = [&](uint4 (&av)[2], uint4 (&bv)[2], int st) {
    const int o = min(st, kSteps - 1) * 64;
    av[0] = pa0[o];
    av[1] = pa1[o];
    bv[0] = pb0[o];
    bv[1] = pb1[o];
  };
  auto mma = [&](const uint4 (&av)[2], const uint4 (&bv)[2]) {
    acc00 = mfma(av[0], bv[0], acc00);
    acc01 = mfma(av[0], bv[1], acc01);
    acc10 = mfma(av[1], bv[0], acc10);
    acc11 = mfma(av[1], bv[1], acc11);
  };
  load(a0, b0, 0);
#pragma unroll
  for (int st = 0; st < kSteps; st += 2) {
    load(a1, b1, st + 1);
    __builtin_amdgcn_sched_barrier(0);
    mma(a0, b0);
    load(a0, b0, st + 2);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, b1);
  }
  auto store = [&](const f32x16& acc, int rb, int cb) {
    const int col = cb * 32 + (lane & 31);
    const float bb = bf2f(bias[col]);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = rb * 32 + drow(r, lane);
      if (row < M) C[(int64_t)row * kBins + col] = acc[r] + bb;
    }
  };
  store(acc00, rb0, cb0);
  store(acc01, rb0, cb0 + 1);
  if (rb0 + 1 < nrb) {
    store(acc10, rb0 + 1, cb0);
    store(acc11, rb0 + 1, cb0 + 1);
  }
}

// ------------------------------------------------------------------ helpers
__global__ __launch_bounds__(256) void k_transpose_u16(const uint16_t* in, int rows, int cols, int ld_in,
                                                       uint16_t* out, int ld_out) {
  __shared__ uint16_t tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int y = by + r, x = bx + tx;
    if (y < rows && x < cols) tile[r][tx] = in[(int64_t)y * ld_in + x];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int y = bx + r, x = by + tx;  // out row = in column
    if (y < cols && x < rows) out[(int64_t)y * ld_out + x] = tile[tx][r];
  }
}

__global__ void k_f32_to_bf16(const float* in, int64_t n, uint16_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(in[i]);
}

// col[(b*P + p)][k] = input of layer `layer` under tap k of output pixel p.
template <int CIN, int HIN>
__global__ void k_im2col(const uint16_t* act, int B, int64_t act_stride, uint16_t* col) {
  constexpr int HO = HIN / 2, P = HO * HO, K = 9 * CIN, KP = (K + 15) / 16 * 16;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * P * KP) return;
  const int k = (int)(i % KP);
  const int64_t r = i / KP;
  const int p = (int)(r % P);
  const int b = (int)(r / P);
  uint16_t v = 0;
  if (k < K) {
    const int tap = k / CIN, c = k % CIN;
    const int iy = 2 * (p / HO) - 1 + tap / 3, ix = 2 * (p % HO) - 1 + tap % 3;
    if (iy >= 0 && iy < HIN && ix >= 0 && ix < HIN) v = act[b * act_stride + (iy * HIN + ix) * CIN + c];
  }
  col[i] = v;
}

// dact[b][q][c] = sum of dcol[b*P + p][tap*CIN + c] over the (p, tap) that
// read input pixel q (the adjoint of k_im2col, a gather, no atomics).
template <int CIN, int HIN>
__global__ void k_col2im(const float* dcol, int B, float* dact) {
  constexpr int HO = HIN / 2, P = HO * HO, K = 9 * CIN, KP = (K + 15) / 16 * 16;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * HIN * HIN * CIN) return;
  const int c = (int)(i % CIN);
  const int64_t r = i / CIN;
  const int q = (int)(r % (HIN * HIN));
  const int b = (int)(r / (HIN * HIN));
  const int iy = q / HIN, ix = q % HIN;
  float acc = 0.f;
#pragma unroll
  for (int ky = 0; ky < 3; ++ky) {
    const int ty = iy + 1 - ky;
    if (ty < 0 || (ty & 1) || (ty >> 1) >= HO) continue;
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
      const int tx = ix + 1 - kx;
      if (tx < 0 || (tx & 1) || (tx >> 1) >= HO) continue;
      const int p = (ty >> 1) * HO + (tx >> 1);
      acc += dcol[((int64_t)b * P + p) * KP + (ky * 3 + kx) * CIN + c];
    }
  }
  dact[i] = acc;
}

// dz = dact where the layer's (saved, per-sample strided) ReLU output is > 0.
__global__ void k_relu_mask(const float* dact, const uint16_t* act, int per_sample, int64_t act_stride, int64_t n,
                            float* dz, uint16_t* dzb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint16_t a = act[(i / per_sample) * act_stride + (i % per_sample)];
  const float v = (a != 0 && !(a & 0x8000)) ? dact[i] : 0.f;
  dz[i] = v;
  dzb[i] = f2bf(v);
}

// out[c] += sum over rows of in[row][c]; workgroups take row chunks.
__global__ __launch_bounds__(256) void k_colsum_add(const float* in, int rows, int cols, float* out) {
  __shared__ float part[256];
  const int t = threadIdx.x;
  const int groups = 256 / cols > 0 ? 256 / cols : 1;
  const int c = t % cols, g = t / cols;
  const int col_block = cols > 256 ? blockIdx.y * 256 : 0;
  float acc = 0.f;
  if (cols <= 256) {
    if (g < groups)
      for (int r = blockIdx.x * groups + g; r < rows; r += gridDim.x * groups) acc += in[(int64_t)r * cols + c];
    part[t] = acc;
    __syncthreads();
    if (g == 0) {
      for (int j = 1; j < groups; ++j) acc += part[t + j * cols];
      atomicAdd(&out[c], acc);
    }
  } else {
    const int cc = col_block + t;
    if (cc < cols) {
      for (int r = blockIdx.x; r < rows; r += gridDim.x) acc += in[(int64_t)r * cols + cc];
      atomicAdd(&out[cc], acc);
    }
  }
}

// Binary cross-entropy with logits, positives weighted, mean over B*4096:
// writes the gradient and adds the batch loss to *loss.
__global__ __launch_bounds__(256) void k_bce(const float* logits, const uint32_t* bits, int B, float pw,
                                             float* dlogits, float* loss) {
  __shared__ float red[256];
  const int b = blockIdx.x;
  if (b >= B) return;
  const int t = threadIdx.x;
  const float scale = 1.0f / ((float)B * (float)kBins);
  float acc = 0.f;
  for (int j = t; j < kBins; j += 256) {
    const float z = logits[(int64_t)b * kBins + j];
    const float y = (bits[(int64_t)b * (kBins / 32) + (j >> 5)] >> (j & 31)) & 1u ? 1.f : 0.f;
    const float sp_pos = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));   // softplus(z)  = -log(1 - s)
    const float sp_neg = sp_pos - z;                                 // softplus(-z) = -log s
    acc += pw * y * sp_neg + (1.f - y) * sp_pos;
    const float s = 1.f / (1.f + expf(-z));
    dlogits[(int64_t)b * kBins + j] = (pw * y * (s - 1.f) + (1.f - y) * s) * scale;
  }
  red[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) atomicAdd(loss, red[0] * scale);
}

// Adam on FP32 master weights; refreshes the BF16 working copy and clears
// the gradient for the next step.
__global__ void k_adam(float* master, float* grad, float* m, float* v, uint16_t* work, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float w = master[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  master[i] = w;
  work[i] = f2bf(w);
  grad[i] = 0.f;
}

// ------------------------------------------------------------------ top-K
// Per sample, the K bins with the largest logits (ties: lower bin first),
// written in ascending bin order; flags[b] = 1 if a logit is NaN.
__device__ __forceinline__ uint32_t order_key(float v) {
  uint32_t u = __float_as_uint(v);
  if (u == 0x80000000u) u = 0u;  // -0 ties with +0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}


// Sum over the 256-thread workgroup (four waves), same value in every lane.
// `slots` holds 2 x 4 words; `par` alternates so one barrier per call suffices.
__device__ __forceinline__ uint32_t block_sum(uint32_t x, uint32_t* slots, int& par) {
  const uint32_t w = wave_sum_u32(x);
  const int wave = threadIdx.x >> 6;
  slots[par * 4 + wave] = w;
  __syncthreads();
  const uint32_t r = slots[par * 4] + slots[par * 4 + 1] + slots[par * 4 + 2] + slots[par * 4 + 3];
  par ^= 1;
  return r;
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// Exclusive prefix sum over the 256 threads (four waves) and the total.
// `slots` holds 2 x 4 words used alternately (see block_sum).
__device__ __forceinline__ uint32_t block_exscan(uint32_t x, uint32_t* slots, int& par, uint32_t& total) {
  const uint32_t inc = wave_scan_u32(x);
  const int wave = threadIdx.x >> 6;
  slots[par * 4 + wave] = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
  __syncthreads();
  uint32_t before = 0;
  const uint32_t s0 = slots[par * 4], s1 = slots[par * 4 + 1], s2 = slots[par * 4 + 2], s3 = slots[par * 4 + 3];
  before = (wave > 0 ? s0 : 0u) + (wave > 1 ? s1 : 0u) + (wave > 2 ? s2 : 0u);
  total = s0 + s1 + s2 + s3;
  par ^= 1;
  return before + inc - x;
}

// Number of keys >= c among m keys in LDS, counted by one wave.
__device__ __forceinline__ uint32_t wave_count_ge(const uint32_t* v, uint32_t m, uint32_t c, int lane) {
  uint32_t n = 0;
  for (uint32_t i0 = 0; i0 < m; i0 += 64) {
    const uint32_t i = i0 + lane;
    n += (uint32_t)__builtin_popcountll(__ballot(i < m && v[i < m ? i : 0] >= c));
  }
  return n;
}

// Exact K-th largest order key T of the row, by bisection with block-wide
// counts: its top kPrefixBits bits over all keys, then the remaining bits
// over the keys sharing that prefix (compacted into bk). Every thread
// returns T.
constexpr int kPrefixBits = 14;

__device__ __forceinline__ uint32_t threshold_by_bisection(const uint32_t (&key)[16], uint32_t K, uint32_t* slots,
                                                           int& par, uint32_t* bk, int t) {
  auto count_ge = [&](uint32_t c) {
    uint32_t n = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) n += (uint32_t)__builtin_popcountll(__ballot(key[j] >= c));
    return n;
  };
  auto block_total = [&](uint32_t wave_n) {
    const int wave = threadIdx.x >> 6;
    slots[par * 4 + wave] = wave_n;  // uniform store
    __syncthreads();
    const uint32_t r = slots[par * 4] + slots[par * 4 + 1] + slots[par * 4 + 2] + slots[par * 4 + 3];
    par ^= 1;
    return r;
  };
  uint32_t T = 0;
  for (int bit = 31; bit >= 32 - kPrefixBits; --bit) {
    const uint32_t c = T | (1u << bit);
    if (block_total(count_ge(c)) >= K) T = c;
  }
  // keys with T's prefix; those above the prefix are all selected
  const uint32_t hi = T | ((1u << (32 - kPrefixBits)) - 1u);
  uint32_t above = 0, inb = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    above += key[j] > hi;
    inb += key[j] >= T && key[j] <= hi;
  }
  const uint32_t need = K - block_sum(above, slots, par);
  uint32_t m = 0;
  uint32_t pos = block_exscan(inb, slots, par, m);
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (key[j] >= T && key[j] <= hi) bk[pos++] = key[j];
  __syncthreads();
  for (int bit = 31 - kPrefixBits; bit >= 0; --bit) {
    const uint32_t c = T | (1u << bit);
    uint32_t n = 0;
    for (uint32_t i0 = 0; i0 < m; i0 += 256) {
      const uint32_t i = i0 + t;
      n += (uint32_t)__builtin_popcountll(__ballot(i < m && bk[i < m ? i : 0] >= c));
    }
    if (block_total(n) >= need) T = c;
  }
  return T;
}

// Sort the 256 values v[j] of lane l (element 4 l + j) of a wave into
// descending order (bitonic network; partners in other lanes via lane
// shuffles).
__device__ __forceinline__ void wave_sort256_desc(uint32_t (&v)[4], int lane) {
#pragma unroll
  for (int k = 2; k <= 256; k <<= 1) {
#pragma unroll
    for (int d = k >> 1; d > 0; d >>= 1) {
      if (d >= 4) {
        const int ld = d >> 2;
        const bool lower = (lane & ld) == 0;  // this lane holds the lower index of each pair
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int e = 4 * lane + j;
          const bool desc = (e & k) == 0;      // this block of the merge sorts descending
          const uint32_t o = (uint32_t)__shfl_xor((int)v[j], ld);
          // the lower index keeps the larger value in a descending block
          const bool keep_max = lower == desc;
          v[j] = keep_max ? max(v[j], o) : min(v[j], o);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if ((j & d) != 0) continue;
          const int e = 4 * lane + j;
          const bool desc = (e & k) == 0;
          const uint32_t a = v[j], b = v[j + d];
          v[j] = desc ? max(a, b) : min(a, b);
          v[j + d] = desc ? min(a, b) : max(a, b);
        }
      }
    }
  }
}

// Element i (0-based, uniform) of a wave's 256 values held as above.
__device__ __forceinline__ uint32_t wave_elem256(const uint32_t (&v)[4], int i) {
  const int j = i & 3;
  const uint32_t x = j == 0 ? v[0] : j == 1 ? v[1] : j == 2 ? v[2] : v[3];
  return (uint32_t)__builtin_amdgcn_readlane((int)x, i >> 2);
}

// Top K of each row of 4096 logits (ties to the lowest bin), as the bins in
// increasing order; flags[b] = 1 if the row holds a NaN. Exact selection of
// the K-th largest order key T in a few block-wide steps:
//  1. a sample of 256 keys (one per thread, spread over the columns of the
//     64 x 64 bin grid), sorted by one wave, brackets T between two sample
//     order statistics, K/16 -+ (3 standard deviations of a binomial count
//     + 2) in rank;
//  2. one pass counts the keys above the bracket and in it; if the bracket
//     holds the K-th key (it almost always does), the keys in it are
//     compacted and one wave finds T among them by bisection;
//  3. otherwise T comes from a bisection over all keys.
// The result depends only on the keys, never on the sample.
constexpr int kBracketRegs = 10;  // brackets of up to 640 keys are searched in registers

__global__ __launch_bounds__(256) void k_topk(const float* logits, int B, int K, int16_t* cand, int32_t* flags) {
  __shared__ uint32_t slots[8];
  __shared__ uint32_t red[3][4];
  __shared__ uint32_t bc[2];
  __shared__ uint32_t bk[kBins];
  const int b = blockIdx.x;
  if (b >= B) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint32_t key[16];
  uint32_t nan = 0;
  const float4* src = reinterpret_cast<const float4*>(logits + (int64_t)b * kBins + 16 * t);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = src[q];
    const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      nan |= (vv[r] != vv[r]) ? 1u : 0u;
      key[4 * q + r] = order_key(vv[r]);
    }
  }
  // 1. sample key: bin 16 t + ((t ^ (t >> 4)) & 15)
  {
    const int js = (t ^ (t >> 4)) & 15;
    uint32_t sv = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) sv = j == js ? key[j] : sv;
    bk[t] = sv;
  }
  __syncthreads();
  if (wave == 0) {
    const float p = (float)K * (1.0f / kBins);
    const int r = (K + 8) / 16;                                        // expected rank of T in the sample
    const int mg = (int)(3.0f * sqrtf(256.0f * p * (1.0f - p))) + 2;   // margin
    const int r_hi = r - mg, r_lo = r + mg;
    uint32_t sv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) sv[j] = bk[4 * lane + j];
    wave_sort256_desc(sv, lane);
    // the rank-r sample (1-based) is element r - 1 of the sorted sample
    const uint32_t qh = wave_elem256(sv, max(r_hi, 1) - 1), ql = wave_elem256(sv, min(r_lo, 256) - 1);
    if (lane == 0) {
      bc[0] = r_hi >= 1 ? qh : 0xffffffffu;  // no sample bound above: nothing is above the bracket
      bc[1] = r_lo <= 256 ? ql : 0u;         // none below: every key is at or above it
    }
  }
  __syncthreads();
  const uint32_t t_hi = bc[0], t_lo = bc[1];
  // 2. keys above the bracket, at or above its lower end, NaN flag
  uint32_t n_gt = 0, n_ge = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    n_gt += key[j] > t_hi;
    n_ge += key[j] >= t_lo;
  }
  n_gt = wave_sum_u32(n_gt);
  n_ge = wave_sum_u32(n_ge);
  nan = wave_sum_u32(nan);
  if (lane == 0) {
    red[0][wave] = n_gt;
    red[1][wave] = n_ge;
    red[2][wave] = nan;
  }
  __syncthreads();
  const uint32_t c_gt = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  const uint32_t c_ge = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  const bool any_nan = (red[2][0] | red[2][1] | red[2][2] | red[2][3]) != 0;
  int par = 0;
  uint32_t T;
  if (c_gt < (uint32_t)K && (uint32_t)K <= c_ge) {
    uint32_t inb = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) inb += key[j] >= t_lo && key[j] <= t_hi;
    uint32_t m = 0;
    uint32_t pos = block_exscan(inb, slots, par, m);  // m = c_ge - c_gt
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (key[j] >= t_lo && key[j] <= t_hi) bk[pos++] = key[j];
    __syncthreads();
    if (wave == 0) {
      // T in [t_lo, t_hi]: the bits above their highest differing bit are fixed
      const uint32_t need = (uint32_t)K - c_gt;
      const uint32_t d = t_lo ^ t_hi;
      const int top = d ? 31 - __builtin_clz(d) : -1;
      uint32_t v = top >= 31 ? 0u : (t_lo >> (top + 1)) << (top + 1);
      if (m <= 64 * kBracketRegs) {
        // the bracket in registers (0 pads: every tested value is >= 1)
        uint32_t r[kBracketRegs];
#pragma unroll
        for (int i = 0; i < kBracketRegs; ++i) r[i] = (uint32_t)(lane + 64 * i) < m ? bk[lane + 64 * i] : 0u;
        for (int bit = top; bit >= 0; --bit) {
          const uint32_t c = v | (1u << bit);
          uint32_t n = 0;
#pragma unroll
          for (int i = 0; i < kBracketRegs; ++i) n += r[i] >= c ? 1u : 0u;
          if (wave_sum_u32(n) >= need) v = c;
        }
      } else {
        for (int bit = top; bit >= 0; --bit) {
          const uint32_t c = v | (1u << bit);
          if (wave_count_ge(bk, m, c, lane) >= need) v = c;
        }
      }
      if (lane == 0) bc[0] = v;
    }
    __syncthreads();
    T = bc[0];
  } else {
    T = threshold_by_bisection(key, (uint32_t)K, slots, par, bk, t);
  }
  // output: greater keys, then ties at T from the lowest bins
  uint32_t gt = 0, eq = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    gt += key[j] > T;
    eq += key[j] == T;
  }
  uint32_t tot = 0;
  const uint32_t before = block_exscan((gt << 16) | eq, slots, par, tot);  // both counts < 2^16
  const uint32_t gt_before = before >> 16, eq_before = before & 0xffffu;
  const uint32_t remaining = (uint32_t)K - (tot >> 16);  // ties at T to take, lowest bins first
  // Ties taken before this thread and by it, written with min() only: a
  // subtraction guarded by a comparison was observed to be speculated with
  // a no-wrap flag that then let the optimiser drop the first min().
  const uint32_t taken_before = min(eq_before, remaining);
  const uint32_t eq_take = min(eq_before + eq, remaining) - taken_before;
  // selected before this thread: all greater keys, plus the ties taken
  uint32_t pos = gt_before + taken_before;
  uint32_t eq_seen = 0;
  int16_t* out = cand + (int64_t)b * K;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    bool take = key[j] > T;
    if (key[j] == T) {
      take = eq_seen < eq_take;
      ++eq_seen;
    }
    if (take && pos < (uint32_t)K) out[pos++] = (int16_t)(16 * t + j);
  }
  if (t == 0) flags[b] = any_nan ? 1 : 0;
}

}  // namespace

hipError_t patches(const uint8_t* img, const uint8_t* avail, int64_t pitch, int32_t H, int32_t W, const void* blocks,
                   const int32_t* orig, int32_t n, uint16_t* x, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_patches, dim3(n), dim3(256), 0, s, img, avail, pitch, H, W,
                     reinterpret_cast<const fse_block_t*>(blocks), orig, n, x);
  return hipGetLastError();
}

hipError_t forward(const uint16_t* x, int32_t B, const uint16_t* prm, uint16_t* feats, uint16_t* acts,
                   hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_forward, dim3(B), dim3(256), 0, s, x, B, prm, feats, acts);
  return hipGetLastError();
}

hipError_t forward_blocks(const uint8_t* img, const uint8_t* avail, int64_t pitch, int32_t H, int32_t W,
                          const void* blocks, const int32_t* orig, int32_t n, const uint16_t* prm, uint16_t* feats,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_forward_blocks, dim3(n), dim3(256), 0, s, img, avail, pitch, H, W,
                     reinterpret_cast<const fse_block_t*>(blocks), orig, n, prm, feats);
  return hipGetLastError();
}

hipError_t permute_head(const uint16_t* w, uint16_t* frag, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_head, dim3(kBins / 32 * kSteps * 64 / 256), dim3(256), 0, s, w,
                     reinterpret_cast<uint4*>(frag));
  return hipGetLastError();
}

hipError_t head_frag(const uint16_t* feats_frag, const uint16_t* w_frag, const uint16_t* bias, float* logits, int32_t M,
                     hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_head_frag, dim3((M + 127) / 128, kBins / 128), dim3(256), 0, s,
                     reinterpret_cast<const uint4*>(feats_frag), reinterpret_cast<const uint4*>(w_frag), bias, logits,
                     M);
  return hipGetLastError();
}

hipError_t gemm_nt(const uint16_t* A, int lda, const uint16_t* B, int ldb, float* C, int ldc,
                   const uint16_t* bias_bf16, int M, int N, int K, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if ((int64_t)M * N >= (int64_t)1 << 22) {
    hipLaunchKernelGGL((k_gemm_nt_t<2, 2>), dim3((M + 127) / 128, (N + 127) / 128), dim3(256), 0, s, A, lda, B, ldb,
                       C, ldc, bias_bf16, M, N, K);
  } else {
    hipLaunchKernelGGL(k_gemm_nt, dim3((M + 63) / 64, (N + 63) / 64), dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                       bias_bf16, M, N, K);
  }
  return hipGetLastError();
}

hipError_t transpose_u16(const uint16_t* in, int rows, int cols, int ld_in, uint16_t* out, int ld_out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_u16, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, s, in, rows, cols,
                     ld_in, out, ld_out);
  return hipGetLastError();
}

hipError_t f32_to_bf16(const float* in, int64_t n, uint16_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, n, out);
  return hipGetLastError();
}

hipError_t im2col(const uint16_t* act, int32_t B, int layer, uint16_t* col, hipStream_t s) {
  const int HO = kHin[layer] / 2;
  const int64_t n = (int64_t)B * HO * HO * kKpad[layer];
  const dim3 g((unsigned)((n + 255) / 256)), blk(256);
  // layer 0 reads the network input, the others the saved activations
  const int64_t st = layer == 0 ? kPatchElems : kActElems;
  switch (layer) {
    case 0: hipLaunchKernelGGL((k_im2col<2, 48>), g, blk, 0, s, act, B, st, col); break;
    case 1: hipLaunchKernelGGL((k_im2col<kCh, 24>), g, blk, 0, s, act, B, st, col); break;
    case 2: hipLaunchKernelGGL((k_im2col<kCh, 12>), g, blk, 0, s, act, B, st, col); break;
    default: hipLaunchKernelGGL((k_im2col<kCh, 6>), g, blk, 0, s, act, B, st, col); break;
  }
  return hipGetLastError();
}

hipError_t col2im(const float* dcol, int32_t B, int layer, float* dact, hipStream_t s) {
  const int64_t n = (int64_t)B * kHin[layer] * kHin[layer] * kCin[layer];
  const dim3 g((unsigned)((n + 255) / 256)), blk(256);
  switch (layer) {
    case 1: hipLaunchKernelGGL((k_col2im<kCh, 24>), g, blk, 0, s, dcol, B, dact); break;
    case 2: hipLaunchKernelGGL((k_col2im<kCh, 12>), g, blk, 0, s, dcol, B, dact); break;
    case 3: hipLaunchKernelGGL((k_col2im<kCh, 6>), g, blk, 0, s, dcol, B, dact); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t relu_mask(const float* dact, const uint16_t* act, int per_sample, int64_t act_stride, int64_t n,
                     float* dz, uint16_t* dz_bf16, hipStream_t s) {
  hipLaunchKernelGGL(k_relu_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dact, act, per_sample,
                     act_stride, n, dz, dz_bf16);
  return hipGetLastError();
}

hipError_t colsum_add(const float* in, int rows, int cols, float* out, hipStream_t s) {
  if (cols <= 256) {
    const int groups = 256 / cols;
    const int grid = std::min(1024, (rows + groups * 64 - 1) / (groups * 64) + 1);
    hipLaunchKernelGGL(k_colsum_add, dim3(grid), dim3(256), 0, s, in, rows, cols, out);
  } else {
    hipLaunchKernelGGL(k_colsum_add, dim3(std::min(rows, 64), (cols + 255) / 256), dim3(256), 0, s, in, rows, cols,
                       out);
  }
  return hipGetLastError();
}

hipError_t bce(const float* logits, const uint32_t* target_bits, int32_t B, float pos_weight, float* dlogits,
               float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_bce, dim3(B), dim3(256), 0, s, logits, target_bits, B, pos_weight, dlogits, loss);
  return hipGetLastError();
}

hipError_t adam(float* master, float* grad, float* m, float* v, uint16_t* work, int64_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, master, grad, m, v, work, n, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t topk(const float* logits, int32_t B, int32_t K, int16_t* cand, int32_t* flags, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_topk, dim3(B), dim3(256), 0, s, logits, B, K, cand, flags);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace fse
