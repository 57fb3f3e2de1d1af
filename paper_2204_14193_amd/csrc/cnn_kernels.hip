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
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16, round to nearest even (NaN stays NaN): the hardware
// conversion of gfx950 (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// 16 x 16 x 32 product: lane l supplies 8 K elements of row l%16 of A and
// of column l%16 of B (the same K elements in both, group l/16); accumulator
// i of lane l holds D[4*(l/16) + i][l%16].
__device__ __forceinline__ f32x4 mfma16(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

__device__ __forceinline__ int drow(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

// Workgroup barrier that orders LDS accesses only: global loads in flight
// (weights requested ahead of their layer) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

// Position of grid column gx within its row: a row holds its even columns
// first, then its odd ones, so that the stride-2 taps of consecutive output
// pixels are consecutive entries and a wave's tap reads are free of LDS
// bank conflicts. Tap dx = 0, 1, 2 of output column x lies at x, x + (G+1)/2
// and x + 1.
template <int G>
__device__ __forceinline__ constexpr int gpos(int gx) { return (gx & 1) ? (G + 1) / 2 + (gx >> 1) : gx >> 1; }
template <int G>
__device__ __forceinline__ constexpr int tap_col(int dx) { return dx == 0 ? 0 : dx == 1 ? (G + 1) / 2 : 1; }

// ------------------------------------------------------------------ patches
// Network input of a block (its 48x48 area): one word per pixel, the two
// BF16 channels, channel 0 = (s - mean over A)/64 on A, channel 1 = 1 on A
// (0 elsewhere). Built by four waves in two halves, so that a pipelined
// caller can put a barrier of its own between them: input_load (wave w of
// the four reads area rows w, w + 4, ..., lane l < 48 column l; a row's
// address is uniform, so a pixel costs its two byte loads) keeps the 12
// pixel values and the mask of those in A, and writes the wave's integer
// sums over A to red[.][w]; after a barrier, input_store forms the mean
// (integer sums: exact in any order) and writes the rows.
struct InputRows {
  uint32_t pv[3];  // 12 pixel values, four per word
  uint32_t in_a;   // bit r: row r's pixel lies in A
};

__device__ __forceinline__ InputRows input_load(const uint8_t* img, const uint8_t* avail, int64_t pitch, int H,
                                                int W, const fse_block_t& bd, uint32_t (*red)[4], int wave,
                                                int lane) {
  constexpr int R = kIn / 4;  // rows per wave
  const int bo = bd.border;
  const int ya = bd.y0 - bo, xa = bd.x0 - bo;
  const int c = min(lane, kIn - 1);
  const int x = xa + c;
  const bool col_in = lane < kIn && x >= 0 && x < W;
  const bool col_b = c >= bo && c < bo + bd.bw;
  const int xo = min(max(x, 0), W - 1);
  const uint8_t* const im = img + (int64_t)bd.frame * H * pitch;
  const uint8_t* const av = avail + (int64_t)bd.frame * H * pitch;
  InputRows out = {{0u, 0u, 0u}, 0u};
  uint32_t sum = 0, cnt = 0;
  // two passes of six rows, each with all of its loads first (row base
  // uniform, column offset per lane); a scheduling barrier keeps the second
  // pass's loads behind the first pass's use, which bounds the registers
#pragma unroll
  for (int r0 = 0; r0 < R; r0 += R / 2) {
    uint32_t sv[R / 2], ab[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      const int64_t ro = (int64_t)min(max(ya + wave + 4 * (r0 + i), 0), H - 1) * pitch;
      ab[i] = (av + ro)[(uint32_t)xo];
      sv[i] = (im + ro)[(uint32_t)xo];
    }
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      const int r = r0 + i;
      const int m = wave + 4 * r;
      const int y = ya + m;
      const bool row_in = y >= 0 && y < H;
      const bool row_b = m >= bo && m < bo + bd.bh;
      const bool ia = col_in && row_in && !(row_b && col_b) && ab[i] != 0;
      sum += ia ? sv[i] : 0u;
      cnt += ia ? 1u : 0u;
      out.in_a |= ia ? 1u << r : 0u;
      out.pv[r >> 2] |= sv[i] << (8 * (r & 3));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  sum = wave_sum_u32(sum);
  cnt = wave_sum_u32(cnt);
  if (lane == 0) {
    red[0][wave] = sum;
    red[1][wave] = cnt;
  }
  return out;
}

// Rows of 48 words, or (GRID) the guarded 49 x 49 grid from (1, 1) on.
template <bool GRID>
__device__ __forceinline__ void input_store(const InputRows& in, const uint32_t (*red)[4], uint32_t* out, int wave,
                                            int lane) {
  const uint32_t S = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  const uint32_t N = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  const float mu = N > 0 ? (float)S / (float)N : 0.f;
  if (lane < kIn) {
#pragma unroll
    for (int r = 0; r < kIn / 4; ++r) {
      const int m = wave + 4 * r;
      const uint32_t sv = (in.pv[r >> 2] >> (8 * (r & 3))) & 0xffu;
      const int o = GRID ? (m + 1) * (kIn + 1) + gpos<kIn + 1>(lane + 1) : m * kIn + lane;
      out[o] = ((in.in_a >> r) & 1u) ? ((uint32_t)f2bf((sv - mu) * (1.0f / 64.0f)) | (0x3f80u << 16)) : 0u;
    }
  }
}

__global__ __launch_bounds__(256) void k_patches(const uint8_t* img, const uint8_t* avail, int64_t pitch, int H,
                                                 int W, const fse_block_t* blocks, const int32_t* orig, int n,
                                                 uint16_t* x) {
  __shared__ uint32_t red[2][4];
  const int b = blockIdx.x;
  if (b >= n) return;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const InputRows in = input_load(img, avail, pitch, H, W, blocks[b], red, wave, lane);
  lds_barrier();
  input_store<false>(in, red, reinterpret_cast<uint32_t*>(x + (int64_t)orig[b] * kPatchElems), wave, lane);
}

// ------------------------------------------------------------------ forward
// Layouts in LDS. A layer's input sits on a (H+1) x (H+1) grid whose row 0
// and column 0 are zero, the pixel (y, x) at (y+1, x+1): the taps of a 3x3
// stride-2 convolution with padding 1 then never leave the grid, and every
// activation-operand read is a per-lane base plus a compile-time offset.
// Each grid row stores its even columns first, then its odd ones (gpos), so
// consecutive output pixels read consecutive entries. The network input (2
// channels) is one 32-bit word per grid point; 32-channel activations are
// four planes of 8 channels (16 bytes per grid point per plane).
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

// Weights of the first layer (2 input channels: depth 18, padded to 32) as
// fragments of the 32 x 32 x 16 product: lane l holds output channel l & 31
// and depth values 16 ks + 8 (l >> 5) .. + 8 of step ks. Depth 18, the first
// padding slot, holds the channel's bias and the input side supplies a 1
// there, so that the product adds the bias.
struct LayerW {
  uint4 w[2];
};

__device__ __forceinline__ void load_layer1(const uint16_t* w, const uint16_t* bias, LayerW& L, int lane) {
  constexpr int K = 9 * 2;
  const int n = lane & 31, h = lane >> 5;
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const int k0 = ks * 16 + 8 * h;
    uint32_t b4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 2 * q;  // even: depth K is a low half
      const uint32_t lo = k < K ? w[n * K + k] : k == K ? bias[n] : 0u;
      const uint32_t hi = k + 1 < K ? w[n * K + k + 1] : 0u;
      b4[q] = lo | (hi << 16);
    }
    L.w[ks] = make_uint4(b4[0], b4[1], b4[2], b4[3]);
  }
}

// ReLU of two values, rounded to BF16 and packed (a in the low half): one
// v_cvt_pk_bf16_f32, then a signed 16-bit maximum with 0 on both halves,
// which maps every negative BF16 value (-0 included) to +0 and keeps the
// others. Rounding and ReLU commute for ordered values; a NaN with the sign
// bit clear stays NaN.
__device__ __forceinline__ uint32_t relu_pack(float a, float b) {
  const f32x2 v = {a, b};
  const s16x2 h = __builtin_bit_cast(s16x2, __builtin_convertvector(v, bf16x2));
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(h, (s16x2){0, 0}));
}

// The first layer, a 3x3 stride-2 convolution of the 2-channel input with
// bias and ReLU as an implicit GEMM: D[channel][pixel] = W[channel][depth]
// X[depth][pixel], depth = (tap, input channel), pixels in tiles of 32 (tile
// = wave, wave + 4, ... run two at a time). Step 0 holds taps 0-3 (lanes
// l < 32) and 4-7 (l >= 32), step 1 tap 8 and the bias slot (l < 32) and
// zeros. Each lane of the result holds one pixel and 16 output channels, 4
// consecutive ones per 8-channel plane, stored as one 8-byte write per
// plane into the guarded 25 x 25 grid.
__device__ __forceinline__ void conv_layer1(const uint16_t* in, uint16_t* out, const LayerW& L, int t) {
  constexpr int HIN = kIn, HO = HIN / 2, P = HO * HO;
  constexpr int MT = (P + 31) / 32;
  constexpr int G = HIN + 1;            // input grid
  constexpr int GO = HO + 1;            // output grid
  const int lane = t & 63, wave = t >> 6;
  const int h = lane >> 5;              // which 8 of the 16 depth values of a step
  const uint32_t* gw = reinterpret_cast<const uint32_t*>(in);
  // word offsets of this lane's taps of step 0, relative to tap 0
  int off[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ta = q, tb = 4 + q;
    const int oa = (ta / 3) * G + tap_col<G>(ta % 3), ob = (tb / 3) * G + tap_col<G>(tb % 3);
    off[q] = h ? ob : oa;
  }
  constexpr int o8 = 2 * G + tap_col<G>(2);  // tap 8
  const uint32_t keep = h ? 0u : ~0u;        // lanes l >= 32 read the zero word 0 for step 1
  const uint32_t one = h ? 0u : 0x3f80u;     // BF16 1 against the bias slot
  // word of tap 0 of the output pixel in column `lane & 31` of a tile
  // (columns past the end repeat the last pixel; they are not stored)
  auto base_of = [&](int tile) {
    const int m = min(tile * 32 + (lane & 31), P - 1);
    return 2 * (m / HO) * G + m % HO;
  };
  auto gather0 = [&](int base) -> uint4 {
    return make_uint4(gw[base + off[0]], gw[base + off[1]], gw[base + off[2]], gw[base + off[3]]);
  };
  auto gather1 = [&](int base) -> uint4 { return make_uint4(gw[(base + o8) & keep], one, 0u, 0u); };
  auto store = [&](int tile, const f32x16& acc) {
    const int p = tile * 32 + (lane & 31);
    if (p >= P) return;
    const int px = (p / HO + 1) * GO + gpos<GO>(p % HO + 1);
    constexpr int PE = plane_elems<GO>();
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const uint2 v = make_uint2(relu_pack(acc[4 * g], acc[4 * g + 1]), relu_pack(acc[4 * g + 2], acc[4 * g + 3]));
      *reinterpret_cast<uint2*>(out + g * PE + px * 8 + 4 * h) = v;
    }
  };
  for (int tile = wave; tile < MT; tile += 8) {
    const int tile2 = tile + 4;
    const int b1 = base_of(tile);
    f32x16 acc = {}, acc2 = {};
    if (tile2 < MT) {
      const int b2 = base_of(tile2);
      const uint4 a1 = gather0(b1), a2 = gather0(b2);
      const uint4 c1 = gather1(b1), c2 = gather1(b2);
      acc = mfma(L.w[0], a1, acc);
      acc2 = mfma(L.w[0], a2, acc2);
      acc = mfma(L.w[1], c1, acc);
      acc2 = mfma(L.w[1], c2, acc2);
      store(tile, acc);
      store(tile2, acc2);
    } else {
      acc = mfma(L.w[0], gather0(b1), acc);
      acc = mfma(L.w[1], gather1(b1), acc);
      store(tile, acc);
    }
  }
}

// Weights of one 32-channel layer for the 16 x 16 x 32 product, half `hf`
// of its output channels: lane l holds output channel 16 hf + l%16 and the
// input channels 8 (l/16) .. + 8 of each of the 9 taps (one depth step per
// tap), and the biases of the 4 channels its accumulators hold (16 hf +
// 4 (l/16) + 0..3), widened to FP32 once.
struct HalfW {
  uint4 w[9];
  float4 b;
};

__device__ __forceinline__ void load_half(const uint16_t* w, const uint16_t* bias, HalfW& L, int hf, int lane) {
  const int n = 16 * hf + (lane & 15), g = lane >> 4;
#pragma unroll
  for (int s = 0; s < 9; ++s) L.w[s] = *reinterpret_cast<const uint4*>(w + n * (9 * kCh) + s * kCh + 8 * g);
  const uint2 bb = *reinterpret_cast<const uint2*>(bias + 16 * hf + 4 * g);
  L.b = make_float4(bf2f(bb.x & 0xffff), bf2f(bb.x >> 16), bf2f(bb.y & 0xffff), bf2f(bb.y >> 16));
}

// A 3x3 stride-2 convolution of 32 input channels with bias and ReLU on the
// 16 x 16 x 32 product: output tiles of 16 channels (half hf) x 16 pixels,
// depth step s = tap s over the 32 input channels, so that lane l reads the
// 16 bytes of plane l/16 at the tap's grid point of its pixel. The wave runs
// tiles first, first + 2, ... (two at a time); the other wave of its half
// takes the tiles in between. Output layout as conv_layer1, to a guarded
// grid (PAD) or, for the last layer, an unguarded 3x3 planar buffer.
template <int HIN, bool PAD>
__device__ __forceinline__ void conv32(const uint16_t* in, uint16_t* out, const HalfW& L, int hf, int first, int t) {
  constexpr int HO = HIN / 2, P = HO * HO, MT = (P + 15) / 16;
  constexpr int G = HIN + 1, GO = HO + 1;
  const int lane = t & 63, g = lane >> 4, col = lane & 15;
  const uint16_t* const inp = in + g * plane_elems<G>();
  // element offset of tap (0, 0) of the pixel in column `col` of a tile
  // (columns past the end repeat the last pixel; they are not stored)
  auto base_of = [&](int tile) {
    const int m = min(tile * 16 + col, P - 1);
    return (2 * (m / HO) * G + m % HO) * 8;
  };
  auto tap = [&](int base, int s) -> uint4 {
    return *reinterpret_cast<const uint4*>(inp + base + ((s / 3) * G + tap_col<G>(s % 3)) * 8);
  };
  auto store = [&](int tile, const f32x4& acc) {
    const int p = tile * 16 + col;
    if (p >= P) return;
    const int px = PAD ? (p / HO + 1) * GO + gpos<GO>(p % HO + 1) : p;
    constexpr int PE = PAD ? plane_elems<GO>() : P * 8;
    const int ch = 16 * hf + 4 * g;
    const uint2 v = make_uint2(relu_pack(acc[0] + L.b.x, acc[1] + L.b.y), relu_pack(acc[2] + L.b.z, acc[3] + L.b.w));
    *reinterpret_cast<uint2*>(out + (ch >> 3) * PE + px * 8 + (ch & 7)) = v;
  };
  for (int tile = first; tile < MT; tile += 4) {
    const int tile2 = tile + 2;
    const int b1 = base_of(tile);
    f32x4 acc = {}, acc2 = {};
    if (tile2 < MT) {
      const int b2 = base_of(tile2);
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        const uint4 a1 = tap(b1, s), a2 = tap(b2, s);
        acc = mfma16(L.w[s], a1, acc);
        acc2 = mfma16(L.w[s], a2, acc2);
      }
      store(tile, acc);
      store(tile2, acc2);
    } else {
#pragma unroll
      for (int s = 0; s < 9; ++s) acc = mfma16(L.w[s], tap(b1, s), acc);
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
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[g * G * G + (y + 1) * G + gpos<G>(x + 1)];
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

// Every layer's weights: layer 1 for the 32 x 32 x 16 product, layers 2-4
// for half (wave & 1) of their output channels. Layers 1 and 2 are loaded
// before the input is built, layers 3 and 4 once layer 1 is done, so that
// layer 2's products cover their latency.
struct NetW {
  LayerW L1;
  HalfW L2, L3, L4;
};

__device__ __forceinline__ void load_weights(const uint16_t* prm, NetW& N, int t) {
  const int lane = t & 63, hf = (t >> 6) & 1;
  load_layer1(prm + kOffW[0], prm + kOffB[0], N.L1, lane);
  load_half(prm + kOffW[1], prm + kOffB[1], N.L2, hf, lane);
}

__device__ __forceinline__ void load_late_weights(const uint16_t* prm, NetW& N, int t) {
  const int lane = t & 63, hf = (t >> 6) & 1;
  load_half(prm + kOffW[2], prm + kOffB[2], N.L3, hf, lane);
  load_half(prm + kOffW[3], prm + kOffB[3], N.L4, hf, lane);
}

// Returns the 3x3x32 features (planar: 8-channel plane g of pixel px at
// 72 g + 8 px), complete in LDS for every thread. Waves 0 and 1 (one per
// channel half) take the even pixel tiles of layers 2 and 4 and the odd
// ones of layer 3, waves 2 and 3 the others: 7 and 6 tiles of 9 products.
__device__ __forceinline__ const uint16_t* conv_stack(uint16_t* X, uint16_t* Y, const uint16_t* prm, NetW& N,
                                                      uint16_t* dst, int t) {
  const int wave = t >> 6, hf = wave & 1, q = wave >> 1;
  uint16_t* const a4 = Y + kA4Off;
  conv_layer1(X, Y, N.L1, t);
  load_late_weights(prm, N, t);
  lds_barrier();
  if (dst) copy_act_nhwc<24>(Y, dst + kActOff[0], t);
  zero_guard<13>(X, t);  // the input grid is no longer read
  conv32<24, true>(Y, X, N.L2, hf, q, t);
  lds_barrier();
  if (dst) copy_act_nhwc<12>(X, dst + kActOff[1], t);
  zero_guard<7>(Y, t);   // layer 1's grid is no longer read
  conv32<12, true>(X, Y, N.L3, hf, 1 - q, t);
  lds_barrier();
  if (dst) copy_act_nhwc<6>(Y, dst + kActOff[2], t);
  conv32<6, false>(Y, a4, N.L4, hf, q, t);
  lds_barrier();
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
  for (int e = t; e < kIn * kIn; e += 256) grid[(e / kIn + 1) * kGridIn + gpos<kGridIn>(e % kIn + 1)] = src[e];
  NetW N;
  load_weights(prm, N, t);
  zero_input_guard(grid, t);
  zero_guard<25>(Y, t);
  lds_barrier();
  uint16_t* const dst = acts ? acts + (int64_t)b * kActElems : nullptr;
  const uint16_t* a4 = conv_stack(X, Y, prm, N, dst, t);
  for (int i = t; i < kFeat; i += 256) {
    const int px = i / kCh, c = i % kCh;
    const uint16_t v = a4[(c >> 3) * (9 * 8) + px * 8 + (c & 7)];
    feats[(int64_t)b * kFeat + i] = v;
    if (dst) dst[kActOff[3] + i] = v;
  }
}

// The forward pass of the blocks of a batch, inputs built from the frames,
// as a pipeline over the blocks a workgroup takes (b = blockIdx.x + k *
// gridDim.x): waves 0-3 run layers 1 and 2 of block k while waves 4-7 run
// layers 3 and 4 of block k - 1 and build the input of block k + 1, so that
// the latency of the input loads and of the short chains of layers 3 and 4
// overlaps the heavy layers and the two halves carry similar work. Every
// stage has three workgroup barriers, executed by both halves: (A0) input
// of block k written to X and the features of block k - 2 stored from A4,
// (A) layer 1 of k (X -> Y) and layer 3 of k - 1 (Z -> V), (B) layer 2 of k
// (Y -> Z), layer 4 of k - 1 (V -> A4) and the loads for block k + 1. The
// features go to row orig[b] of a matrix in fragment layout (see
// k_head_frag). 63 KB of LDS: two workgroups per CU.
constexpr int kPipeY = 4 * 25 * 25 * 8;  // layer-1 output grid (BF16 elements)
constexpr int kPipeZ = 4 * 13 * 13 * 8;  // layer-2 output grid
constexpr int kPipeV = 4 * 7 * 7 * 8;    // layer-3 output grid
constexpr int kPipeA4 = 4 * 9 * 8;       // layer-4 output (planar, unguarded)

__device__ __forceinline__ void store_features(const uint16_t* a4, int r, uint16_t* feats, int t) {
  // 8 features (one 8-channel plane of one pixel) per 16-byte piece
  if (t < kFeat / 8) {
    const int s16 = t >> 1, h = t & 1;
    const uint4 v = *reinterpret_cast<const uint4*>(a4 + (t & 3) * 72 + (t >> 2) * 8);
    reinterpret_cast<uint4*>(feats)[((int64_t)(r >> 5) * kSteps + s16) * 64 + h * 32 + (r & 31)] = v;
  }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_forward_blocks(
    const uint8_t* img, const uint8_t* avail, int64_t pitch, int H, int W, const fse_block_t* blocks,
    const int32_t* orig, int n, const uint16_t* prm, uint16_t* feats) {
  __shared__ __align__(16) uint32_t X[kGridIn * kGridIn];
  __shared__ __align__(16) uint16_t Y[kPipeY];
  __shared__ __align__(16) uint16_t Z[kPipeZ];
  __shared__ __align__(16) uint16_t V[kPipeV];
  __shared__ __align__(16) uint16_t A4[kPipeA4];
  __shared__ uint32_t red[2][4];
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int g0 = blockIdx.x, gs = gridDim.x;
  const int nloc = (n - g0 + gs - 1) / gs;  // blocks of this workgroup (>= 1: the grid is at most n)
  zero_input_guard(X, t);
  zero_guard<25>(Y, t);
  zero_guard<13>(Z, t);
  zero_guard<7>(V, t);
  if (wave < 4) {
    const int hf = wave & 1, q = wave >> 1;
    LayerW L1;
    HalfW L2;
    load_layer1(prm + kOffW[0], prm + kOffB[0], L1, lane);
    load_half(prm + kOffW[1], prm + kOffB[1], L2, hf, lane);
    lds_barrier();
    for (int k = 0; k <= nloc; ++k) {
      const bool live = k < nloc;
      lds_barrier();  // A0
      if (live) conv_layer1(reinterpret_cast<const uint16_t*>(X), Y, L1, t);
      lds_barrier();  // A
      if (live) conv32<24, true>(Y, Z, L2, hf, q, t);
      lds_barrier();  // B
    }
  } else {
    const int w4 = wave - 4, hf = w4 & 1, q = w4 >> 1, t4 = t - 256;
    HalfW L3, L4;
    load_half(prm + kOffW[2], prm + kOffB[2], L3, hf, lane);
    load_half(prm + kOffW[3], prm + kOffB[3], L4, hf, lane);
    InputRows in = input_load(img, avail, pitch, H, W, blocks[g0], red, w4, lane);
    lds_barrier();
    for (int k = 0; k <= nloc; ++k) {
      if (k < nloc) input_store<true>(in, red, X, w4, lane);
      if (k >= 2) store_features(A4, orig[g0 + (k - 2) * gs], feats, t4);
      lds_barrier();  // A0
      if (k >= 1) conv32<12, true>(Z, V, L3, hf, 1 - q, t4);
      lds_barrier();  // A
      if (k >= 1) conv32<6, false>(V, A4, L4, hf, q, t4);
      if (k + 1 < nloc) in = input_load(img, avail, pitch, H, W, blocks[g0 + (k + 1) * gs], red, w4, lane);
      lds_barrier();  // B
    }
    store_features(A4, orig[g0 + (nloc - 1) * gs], feats, t4);
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
// Workgroups are handed to the eight XCDs in turn, so the tiles are ordered
// for that: XCD x takes the x-th contiguous eighth of the tiles (row tile
// major), and its L2 holds that slice of F and all of W (about 2.9 MB for
// 6432 rows) instead of all of both.
__global__ __launch_bounds__(256) void k_head_frag(const uint4* F, const uint4* Wf, const uint16_t* bias,
                                                   float* C, int M) {
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  constexpr int kColTiles = kBins / 128;
  const int tiles = ((M + 127) >> 7) * kColTiles;
  const int per_xcd = (tiles + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (tile >= tiles) return;
  const int rb0 = (tile / kColTiles) * 4 + (wave & 1) * 2;   // row blocks rb0, rb0 + 1
  const int cb0 = (tile % kColTiles) * 4 + (wave >> 1) * 2;  // column blocks
  const int nrb = (M + 31) >> 5;
  if (rb0 >= nrb) return;
  const int rb1 = min(rb0 + 1, nrb - 1);             // a block past the end repeats the last (never stored)
  // uniform fragment bases, one lane offset for all four operands
  const uint4* pa0 = F + (int64_t)rb0 * kSteps * 64;
  const uint4* pa1 = F + (int64_t)rb1 * kSteps * 64;
  const uint4* pb0 = Wf + (int64_t)cb0 * kSteps * 64;
  const uint4* pb1 = pb0 + kSteps * 64;
  f32x16 acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
  uint4 a0[2], b0[2], a1[2], b1[2];
  auto load = [&](uint4 (&av)[2], uint4 (&bv)[2], int st) {
    const int o = min(st, kSteps - 1) * 64 + lane;
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

// The value of lane (this lane xor ld): DPP moves for ld = 1, 2 (quad
// permutes) and 8 (row rotation), a swizzle for 4 and 16, a permute for 32.
__device__ __forceinline__ uint32_t xor_lanes(uint32_t x, int ld) {
  switch (ld) {
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
    case 8: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xf, 0xf, false);  // row_ror:8
    case 4: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x101f);               // xor 4 in 32 lanes
    case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401f);              // xor 16 in 32 lanes
    default: return (uint32_t)__shfl_xor((int)x, ld);
  }
}

// Sort the 256 values v[j] of lane l (element 4 l + j) of a wave into
// descending order (bitonic network; partners in other lanes by xor_lanes).
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
          const uint32_t o = xor_lanes(v[j], ld);
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
  uint64_t nan_lanes = 0;  // lanes holding a NaN (one unordered compare per pair of values)
  const float4* src = reinterpret_cast<const float4*>(logits + (int64_t)b * kBins + 16 * t);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = src[q];
    nan_lanes |= __ballot(__builtin_isunordered(v.x, v.y)) | __ballot(__builtin_isunordered(v.z, v.w));
    const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) key[4 * q + r] = order_key(vv[r]);
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
  const float p = (float)K * (1.0f / kBins);
  const int r = (K + 8) / 16;                                        // expected rank of T in the sample
  const int mg = (int)(3.0f * sqrtf(256.0f * p * (1.0f - p))) + 2;   // margin
  const int r_hi = r - mg, r_lo = r + mg;
  uint32_t sv[4];  // the sorted sample, kept by wave 0 for the bracket search
  if (wave == 0) {
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
  // this thread's keys in the bracket: keys at or above t_lo less those above
  // t_hi (t_lo <= t_hi; the clamp keeps it exact, 0, were they ever crossed)
  const uint32_t inb = n_ge > n_gt ? n_ge - n_gt : 0u;
  const uint32_t w_gt = wave_sum_u32(n_gt), w_ge = wave_sum_u32(n_ge);
  if (lane == 0) {
    red[0][wave] = w_gt;
    red[1][wave] = w_ge;
    red[2][wave] = nan_lanes != 0 ? 1u : 0u;
  }
  __syncthreads();
  const uint32_t c_gt = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  const uint32_t c_ge = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  const bool any_nan = (red[2][0] | red[2][1] | red[2][2] | red[2][3]) != 0;
  int par = 0;
  uint32_t T;
  if (c_gt < (uint32_t)K && (uint32_t)K <= c_ge) {
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
        auto count_ge = [&](uint32_t c) {
          uint32_t n = 0;
#pragma unroll
          for (int i = 0; i < kBracketRegs; ++i) n += r[i] >= c ? 1u : 0u;
          return wave_sum_u32(n);
        };
        // The sorted sample keys inside the bracket split it into pieces of
        // about 16 keys: a binary search over them (index e0 - 1 stands for
        // "above every key", e1 + 1 for t_lo) finds the piece [lo_k, hi_k]
        // that holds T, and how many bracket keys lie above it.
        const int e0 = max(r_hi, 1) - 1, e1 = min(r_lo, 256) - 1;
        int elo = e0 - 1, ehi = e1 + 1;  // count(elo) < need <= count(ehi)
        uint32_t above = 0;              // bracket keys at or above the key of elo
        while (ehi - elo > 1) {
          const int mid = (elo + ehi) >> 1;
          const uint32_t n = count_ge(wave_elem256(sv, mid));
          if (n >= need) {
            ehi = mid;
          } else {
            elo = mid;
            above = n;
          }
        }
        const uint32_t lo_k = ehi == e1 + 1 ? t_lo : wave_elem256(sv, ehi);
        const uint32_t hi_k = elo == e0 - 1 ? t_hi : wave_elem256(sv, elo) - 1u;
        uint64_t msk[kBracketRegs];
        uint32_t sub = 0;
#pragma unroll
        for (int i = 0; i < kBracketRegs; ++i) {
          msk[i] = __ballot((uint32_t)(lane + 64 * i) < m && r[i] >= lo_k && r[i] <= hi_k);
          sub += (uint32_t)__builtin_popcountll(msk[i]);
        }
        if (sub <= 128) {
          // the piece in two registers, then a bisection with two ballots per step
          uint32_t* const piece = bk + 64 * kBracketRegs;  // past the bracket keys
          uint32_t at = 0;
#pragma unroll
          for (int i = 0; i < kBracketRegs; ++i) {
            if ((msk[i] >> lane) & 1ull)
              piece[at + __builtin_amdgcn_mbcnt_hi((uint32_t)(msk[i] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)msk[i], 0u))] = r[i];
            at += (uint32_t)__builtin_popcountll(msk[i]);
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
          const uint32_t x0 = (uint32_t)lane < sub ? piece[lane] : 0u;  // 0 pads, as above
          const uint32_t x1 = (uint32_t)lane + 64u < sub ? piece[lane + 64] : 0u;
          const uint32_t need2 = need - above;
          const uint32_t d2 = lo_k ^ hi_k;
          const int top2 = d2 ? 31 - __builtin_clz(d2) : -1;
          v = top2 >= 31 ? 0u : (lo_k >> (top2 + 1)) << (top2 + 1);
          for (int bit = top2; bit >= 0; --bit) {
            const uint32_t c = v | (1u << bit);
            if ((uint32_t)(__builtin_popcountll(__ballot(x0 >= c)) + __builtin_popcountll(__ballot(x1 >= c))) >= need2)
              v = c;
          }
        } else {
          for (int bit = top; bit >= 0; --bit) {
            const uint32_t c = v | (1u << bit);
            if (count_ge(c) >= need) v = c;
          }
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
  char* const out = reinterpret_cast<char*>(cand + (int64_t)b * K);  // int16 entries at byte offsets 2 pos
  if ((tot & 0xffffu) == remaining) {
    // every tie at T is taken (the usual case): the keys at or above T
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (key[j] >= T && pos < (uint32_t)K) *reinterpret_cast<int16_t*>(out + 2 * pos) = (int16_t)(16 * t + j);
      pos += key[j] >= T ? 1u : 0u;
    }
  } else {
    uint32_t eq_seen = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      bool take = key[j] > T;
      if (key[j] == T) {
        take = eq_seen < eq_take;
        ++eq_seen;
      }
      if (take && pos < (uint32_t)K) *reinterpret_cast<int16_t*>(out + 2 * pos) = (int16_t)(16 * t + j);
      pos += take ? 1u : 0u;
    }
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
  // two workgroups per CU, each taking every grid-th block
  static int cus[64] = {0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (cus[dev] == 0) {
    int c = 0;
    if ((e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    cus[dev] = c > 0 ? c : 1;
  }
  const int grid = std::min(n, 2 * cus[dev]);
  hipLaunchKernelGGL(k_forward_blocks, dim3(grid), dim3(512), 0, s, img, avail, pitch, H, W,
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
  const int tiles = (M + 127) / 128 * (kBins / 128);
  hipLaunchKernelGGL(k_head_frag, dim3(8 * ((tiles + 7) / 8)), dim3(256), 0, s,
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
