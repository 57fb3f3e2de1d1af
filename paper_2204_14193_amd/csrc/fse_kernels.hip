// Persistent complex-valued FSE kernels for gfx950 (CDNA4, wave64).
//
// One workgroup conceals one lost block at a time and pulls the next block
// from a work queue until the class is exhausted. Per block:
//   1. gather the M x N area from HBM, weight it with the window of eq. (3)
//      on the support area A (zero on B, on lost pixels and off-frame);
//   2. one complex F x F FFT of z = s*w + j*alpha*w in LDS (eq. (11)), split
//      by conjugate symmetry into R_w = DFT(s*w) and W = DFT(w);
//   3. I iterations of Algorithm 1: argmax of |R_w|^2 (eq. (12), lowest
//      linear index k*F+l on ties), c = gamma*R_w[u,v]/W[0,0] (eq. (13)),
//      append (u,v,c) to the model (eq. (15)), R_w -= c*W shifted by (u,v)
//      over all bins (eq. (18)) fused with the next argmax;
//   4. the model is evaluated on B only, Re{sum c*phi_(u,v)} (the inverse
//      transform of G restricted to B), and written to HBM.
//
// Data placement: R_w lives in VGPRs. Wave w of the workgroup owns GR groups
// of RPG consecutive spectrum rows, group g being rows
// [g*F/GR + w*RPG, g*F/GR + (w+1)*RPG); its slots hold those rows' bins in
// ascending order, 64 consecutive bins per slot. W lives in LDS as its F
// rows plus copies of its first RPG-1 rows, so the rows a group reads for a
// shift (k-u) mod F are always consecutive and every load of the update
// uses a compile-time offset from one per-iteration base address per group.
// At F = 64 a group is 8 rows whatever the workgroup size, so W with its
// wrapped rows takes 71 rows (36 KB) and four workgroups fit a CU. The argmax is a
// DPP reduction inside the wave and one LDS exchange and barrier across
// waves.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "fse_internal.h"

namespace fse {
namespace {

// Scale of the window in the packed transform z = s*w + j*alpha*w: balances
// the two real signals (s in [0,255]) so the conjugate-symmetric split keeps
// W accurate; a power of two, so the scaling is exact.
constexpr float kAlpha = 128.0f;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

template <int N>
using fvec = float __attribute__((ext_vector_type(N)));

// DPP row operations of gfx9 used below.
constexpr int kQuadXor1 = 0xb1;      // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4e;      // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kRowBcast15 = 0x142;
constexpr int kRowBcast31 = 0x143;

// Lanes that receive no value keep the identity (0 for max, ~0 for min),
// so the move folds into the max/min instruction.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned dpp_umax(unsigned x) {
  return max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned dpp_umin(unsigned x) {
  return min(x, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)x, CTRL, ROW_MASK, 0xf, false));
}

// Maximum over the 64 lanes of a wave of non-negative floats given as bit
// patterns (which order like the values), returned wave-uniform.
__device__ __forceinline__ unsigned wave_max_bits(unsigned x) {
  x = dpp_umax<kQuadXor1, 0xf>(x);
  x = dpp_umax<kQuadXor2, 0xf>(x);
  x = dpp_umax<kRowHalfMirror, 0xf>(x);
  x = dpp_umax<kRowMirror, 0xf>(x);  // every lane holds its row maximum
  x = dpp_umax<kRowBcast15, 0xa>(x);  // into rows 1 and 3
  x = dpp_umax<kRowBcast31, 0xc>(x);  // into rows 2 and 3
  return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ unsigned wave_min_u32(unsigned x) {
  x = dpp_umin<kQuadXor1, 0xf>(x);
  x = dpp_umin<kQuadXor2, 0xf>(x);
  x = dpp_umin<kRowHalfMirror, 0xf>(x);
  x = dpp_umin<kRowMirror, 0xf>(x);
  x = dpp_umin<kRowBcast15, 0xa>(x);
  x = dpp_umin<kRowBcast31, 0xc>(x);
  return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

// One step of a 64-bit maximum across lanes (key = hi:lo), all rows active.
template <int CTRL>
__device__ __forceinline__ void dpp_max64(unsigned& hi, unsigned& lo) {
  const unsigned ohi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)hi, CTRL, 0xf, 0xf, false);
  const unsigned olo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)lo, CTRL, 0xf, 0xf, false);
  const unsigned long long a = ((unsigned long long)hi << 32) | lo;
  const unsigned long long b = ((unsigned long long)ohi << 32) | olo;
  const bool take = b > a;
  hi = take ? ohi : hi;
  lo = take ? olo : lo;
}

// Maximum (MAX) or minimum over each group of N consecutive lanes (N a power
// of two up to 16), left in every lane of the group.
template <int N, bool MAX>
__device__ __forceinline__ unsigned group_reduce(unsigned x) {
  auto step = [&](unsigned y) { return MAX ? max(x, y) : min(x, y); };
  if constexpr (N >= 2) x = step((unsigned)__builtin_amdgcn_update_dpp(0, (int)x, kQuadXor1, 0xf, 0xf, false));
  if constexpr (N >= 4) x = step((unsigned)__builtin_amdgcn_update_dpp(0, (int)x, kQuadXor2, 0xf, 0xf, false));
  if constexpr (N >= 8) x = step((unsigned)__builtin_amdgcn_update_dpp(0, (int)x, kRowHalfMirror, 0xf, 0xf, false));
  if constexpr (N >= 16) x = step((unsigned)__builtin_amdgcn_update_dpp(0, (int)x, kRowMirror, 0xf, 0xf, false));
  return x;
}

__device__ __forceinline__ float readlane_f(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// Byte offset 8 * ((u m + v n) mod F) of the phase factor of pixel (m, n)
// and a wave-uniform bin (u, v) in a table of F float2, from m8 = 8 m and
// n8 = 8 n: two full-rate 24-bit multiplies with u, v read from SGPRs (the
// compiler, seeing that only the low bits are kept, would otherwise pick
// the quarter-rate 32-bit multiply and a 64-bit multiply-add).
template <int F>
__device__ __forceinline__ uint32_t phase_byte(uint32_t u, uint32_t v, uint32_t m8, uint32_t n8) {
  uint32_t vn, r;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(vn) : "s"(v), "v"(n8));
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "s"(u), "v"(m8), "v"(vn));
  return r & (8 * F - 1);
}

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (a full __syncthreads waits for them too).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------------ FFT
// Forward DFT (exp(-j...)) of every row, then every column, of the F x F
// buffer Z, as Stockham passes of radix 8, 4 or 2. Each pass loads its
// butterflies into registers, waits, and writes the results back into the
// same buffer, so one F x F buffer suffices.

template <int R>
__device__ __forceinline__ void dft_small(float2 (&a)[R]) {
  if constexpr (R == 2) {
    const float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (R == 8) {
    // two 4-point DFTs of the even and odd samples, then
    // X[k] = E[k] + w^k O[k], X[k+4] = E[k] - w^k O[k], w = exp(-j 2 pi / 8)
    constexpr float h = 0.70710678118654752f;
    const float2 t0 = cadd(a[0], a[4]), t1 = csub(a[0], a[4]);
    const float2 t2 = cadd(a[2], a[6]), t3 = csub(a[2], a[6]);
    const float2 t4 = cadd(a[1], a[5]), t5 = csub(a[1], a[5]);
    const float2 t6 = cadd(a[3], a[7]), t7 = csub(a[3], a[7]);
    const float2 e0 = cadd(t0, t2), e2 = csub(t0, t2);
    const float2 e1 = make_float2(t1.x + t3.y, t1.y - t3.x);  // t1 - j*t3
    const float2 e3 = make_float2(t1.x - t3.y, t1.y + t3.x);  // t1 + j*t3
    const float2 o0 = cadd(t4, t6), o2 = csub(t4, t6);
    const float2 o1 = make_float2(t5.x + t7.y, t5.y - t7.x);
    const float2 o3 = make_float2(t5.x - t7.y, t5.y + t7.x);
    const float2 w1 = make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));    // (1 - j)/sqrt2 * o1
    const float2 w2 = make_float2(o2.y, -o2.x);                            // -j * o2
    const float2 w3 = make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));  // (-1 - j)/sqrt2 * o3
    a[0] = cadd(e0, o0);
    a[4] = csub(e0, o0);
    a[1] = cadd(e1, w1);
    a[5] = csub(e1, w1);
    a[2] = cadd(e2, w2);
    a[6] = csub(e2, w2);
    a[3] = cadd(e3, w3);
    a[7] = csub(e3, w3);
  } else {
    const float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const float2 t2 = cadd(a[1], a[3]), t3 = csub(a[1], a[3]);
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = make_float2(t1.x + t3.y, t1.y - t3.x);  // t1 - j*t3
    a[3] = make_float2(t1.x - t3.y, t1.y + t3.x);  // t1 + j*t3
  }
}

// TOUT writes the pass's output transposed (element (line, e) of a row pass
// to Z[e * F + line]); with more threads than butterflies the extra
// threads only take part in the barriers.
template <int F, int NT, int R, int NS, bool COLS, bool TOUT = false>
__device__ __forceinline__ void fft_pass(float2* Z, const float2* tw, int t) {
  constexpr int L = F / R;             // butterflies per line
  constexpr int NB = F * F / R;        // butterflies per pass
  constexpr int PER = NB >= NT ? NB / NT : 1;  // butterflies per thread
  static_assert(NB >= NT ? PER * NT == NB : NT % NB == 0, "pass does not tile the grid");
  static_assert(!TOUT || !COLS, "transposed output is for row passes");
  const bool active = NB >= NT || t < NB;
  float2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (!active) break;
    const int b = t + i * NT;
    const int line = COLS ? (b % F) : (b / L);
    const int j = COLS ? (b / F) : (b % L);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = j + r * L;
      v[i][r] = COLS ? Z[e * F + line] : Z[line * F + e];
    }
    if constexpr (NS > 1) {
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[(r * k * (F / (NS * R))) & (F - 1)]);
    }
    dft_small<R>(v[i]);
  }
  lds_barrier();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (!active) break;
    const int b = t + i * NT;
    const int line = COLS ? (b % F) : (b / L);
    const int j = COLS ? (b / F) : (b % L);
    const int o = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = o + r * NS;
      if (COLS || TOUT) Z[e * F + line] = v[i][r]; else Z[line * F + e] = v[i][r];
    }
  }
  lds_barrier();
}

// F = 64 and 128 use radix-8 passes (fewer LDS round trips and barriers);
// F = 32 keeps radix 4 so that every compiled workgroup size (down to one
// butterfly per thread) runs the same passes and gives the same bits.
template <int F, int NT, bool COLS>
__device__ __forceinline__ void fft_lines(float2* Z, const float2* tw, int t) {
  if constexpr (F == 32) {
    fft_pass<F, NT, 4, 1, COLS>(Z, tw, t);
    fft_pass<F, NT, 4, 4, COLS>(Z, tw, t);
    fft_pass<F, NT, 2, 16, COLS>(Z, tw, t);
  } else if constexpr (F == 64) {
    fft_pass<F, NT, 8, 1, COLS>(Z, tw, t);
    fft_pass<F, NT, 8, 8, COLS>(Z, tw, t);
  } else {
    static_assert(F == 128, "unsupported transform size");
    fft_pass<F, NT, 8, 1, COLS>(Z, tw, t);
    fft_pass<F, NT, 8, 8, COLS>(Z, tw, t);
    fft_pass<F, NT, 2, 64, COLS>(Z, tw, t);
  }
}

// ------------------------------------------------------------ synthesis
// The model on B: out(m, n) = Re{ sum_nu c_nu exp(j 2 pi (u m + v n) / F) }
// (the inverse transform of G restricted to B), for pixel p of the block at
// area position (bo + p / bw, bo + p % bw). Thread `t` of `NT` takes pixels
// t, t + NT, ... in passes of Q; each coefficient is read once per pass and
// its bin made wave-uniform. Per pixel the terms are added in list order.
template <int F, int NT, int Q>
__device__ __forceinline__ void synthesize(const int* cl_idx, const float2* cl_c, int n_coef, const float2* tw,
                                           int bh, int bw, int bo, float* out, int64_t out_pitch, int t,
                                           const uint8_t* lost_only = nullptr, int64_t av_pitch = 0) {
  const int np = bh * bw;
  for (int p0 = 0; p0 < np; p0 += NT * Q) {
    if (p0 + (t & ~63) >= np) break;  // wave-uniform: no pixel left for this wave
    int mq[Q], nq[Q];
    float acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int p = min(p0 + t + q * NT, np - 1);
      mq[q] = bo + p / bw;
      nq[q] = bo + p % bw;
      acc[q] = 0.f;
    }
    for (int it = 0; it < n_coef; ++it) {
      const int sidx = __builtin_amdgcn_readfirstlane(cl_idx[it]);
      const int u = sidx / F, v = sidx % F;
      const float2 c = cl_c[it];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const float2 e = tw[(u * mq[q] + v * nq[q]) & (F - 1)];  // exp(-j theta): Re{c e^{j theta}} = c.x e.x + c.y e.y
        acc[q] = fmaf(c.x, e.x, acc[q]);
        acc[q] = fmaf(c.y, e.y, acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int p = p0 + t + q * NT;
      // with a mask-driven loss area only the rectangle's lost pixels are written
      if (p < np && (!lost_only || lost_only[(int64_t)(mq[q] - bo) * av_pitch + (nq[q] - bo)] == 0))
        out[(int64_t)(mq[q] - bo) * out_pitch + (nq[q] - bo)] = acc[q];
    }
  }
}

// ------------------------------------------------------------------ kernel

template <int F, int NT>
struct Shape {
  static constexpr int NW = NT / 64;          // waves per workgroup
  static constexpr int BPL = F * F / NT;      // bins per lane
  static constexpr int RPW = F / NW;          // spectrum rows owned by one wave
  static constexpr int GR = (F == 64 && RPW > 8) ? RPW / 8 : 1;  // row groups of a wave
  static constexpr int RPG = RPW / GR;        // rows per group
  static constexpr int SPG = BPL / GR;        // slots per group
  static constexpr int WROWS = F + RPG - 1;   // W rows in LDS: F plus RPG-1 wrapped copies
  static constexpr int PH = F > 64 ? F / 64 : 1;  // column phases of a lane
  static_assert(NT % 64 == 0 && NW <= 16 && F % NW == 0 && BPL * NT == F * F && BPL * 64 == RPW * F,
                "bad tiling");
  static_assert(F <= 64 || (F % 64 == 0 && BPL % PH == 0), "bad tiling");
  static_assert(GR == 1 || (F == 64 && SPG * 64 == RPG * F), "bad row groups");
  // first row of group g of wave w, and the wave owning row k
  static __device__ __forceinline__ int group_row(int w, int g) { return g * (F / GR) + w * RPG; }
  static __device__ __forceinline__ int wave_of_row(int k) { return (int)(((unsigned)k % (F / GR)) / RPG); }
};

// LDS carve-up of one workgroup (dynamic shared memory).
struct Lds {
  float2* Wd;      // WROWS x F: FFT buffer, then the window spectrum W
  float2* tw;      // F twiddles exp(-j 2 pi q / F)
  int4* red;       // 2 x NW cross-wave argmax slots (|R|^2 bits, index, re, im)
  int* cl_idx;     // selections of the current block
  float2* cl_c;    // coefficients of the current block
  int* misc;       // [0]: block index popped from the queue, [1]: warm list length
  int* wl_idx;     // warm start: distinct bins chosen in the restricted phase
  float2* wl_c;    // warm start: their accumulated coefficients
};

// A block descriptor made wave-uniform (SGPRs), so that the geometry and
// the frame base addresses live on the scalar unit.
struct UBlock {
  int frame, y0, x0, bh, bw, border, iters;
};
__device__ __forceinline__ UBlock uniform_block(const fse_block_t* p) {
  const int* w = reinterpret_cast<const int*>(p);
  UBlock b;
  b.frame = __builtin_amdgcn_readfirstlane(w[0]);
  b.y0 = __builtin_amdgcn_readfirstlane(w[1]);
  b.x0 = __builtin_amdgcn_readfirstlane(w[2]);
  const int hw = __builtin_amdgcn_readfirstlane(w[3]);
  const int bf = __builtin_amdgcn_readfirstlane(w[4]);
  b.bh = (int)(int16_t)(hw & 0xffff);
  b.bw = hw >> 16;
  b.border = (int)(int16_t)(bf & 0xffff);
  b.iters = __builtin_amdgcn_readfirstlane(w[5]);
  return b;
}
static_assert(sizeof(fse_block_t) == 24, "block descriptor layout");

// Block status of the split warm start's transform kernel: the restricted
// kernel finishes the block and writes its status.
constexpr int kPending = 0x7fff;

// Conceal one block with every lane of the workgroup. All values that steer
// control flow (block geometry, W0, the selected bin) are wave-uniform, so
// every branch below is taken by all lanes together. Returns FSE_BLOCK_*.
// MODE kWarmFused compiles the warm-started form: KC candidate bins per
// block (from the network), KC/64 per lane of wave 0. MODE kWarmPrep stops
// a warm-started block after the transform and stages W (rows 0..F/2) and
// R_w at its KC candidates for the restricted kernel.
template <int F, int NT, int KC, int MODE>
__device__ __forceinline__ int conceal_block(const ClassArgs& a, const int bi, const Lds& s, const int t,
                                             int& parity) {
  using S = Shape<F, NT>;
  constexpr int BPL = S::BPL, NW = S::NW, RPG = S::RPG, SPG = S::SPG, GR = S::GR, PH = S::PH;
  constexpr int CPL = KC > 0 ? KC / 64 : 1;  // candidates per lane of wave 0
  constexpr bool FUSED = MODE == kWarmFused;
  static_assert(KC % 64 == 0 && KC <= 1024, "candidate count must be a multiple of 64");
  static_assert((MODE == kPlain || MODE == kPower) == (KC == 0), "warm modes need candidates");
  static_assert(MODE != kPower || F == 64, "the power spectrum is compiled for F = 64");
  static_assert(MODE != kWarmPrep || F == 64, "the split warm start is compiled for F = 64");
  const int lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  // linear index of the first bin of slot j is gbase[j / SPG] + (j % SPG) * 64
  int gbase[GR];
#pragma unroll
  for (int g = 0; g < GR; ++g) gbase[g] = S::group_row(wave, g) * F;
  // LDS element index of W[(k-u) mod F, (l-v) mod F] for the first bin of
  // each row group and column phase of this lane
  auto shifted_bases = [&](int u, int v, int (&wb)[GR][PH]) __attribute__((always_inline)) {
#pragma unroll
    for (int g = 0; g < GR; ++g) {
      const int r0 = (S::group_row(wave, g) - u) & (F - 1);
#pragma unroll
      for (int p = 0; p < PH; ++p) {
        const int lr = F <= 64 ? lane / F : 0;
        const int lc = F <= 64 ? lane % F : p * 64 + lane;
        wb[g][p] = (r0 + lr) * F + ((lc - v) & (F - 1));
      }
    }
  };
  float2* const Wd = s.Wd;

  const UBlock bd = uniform_block(a.blocks + bi);
  const int orig = __builtin_amdgcn_readfirstlane(a.orig[bi]);
  const int bh = bd.bh, bw = bd.bw, bo = bd.border;
  const int M = bh + 2 * bo, N = bw + 2 * bo;
  const int ya = bd.y0 - bo, xa = bd.x0 - bo;
  const int I = bd.iters;
  const int64_t fofs = (int64_t)bd.frame * a.H;
  const uint8_t* img = a.img + fofs * a.pitch;
  const uint8_t* av = a.avail + fofs * a.pitch;
  const int pitch = (int)a.pitch;  // a frame is below 2^31 bytes (checked by the host)

  // 1. gather and weight (eq. (3)); z = s*w + j*alpha*w on the F x F grid.
  // Loads go to clamped, always valid addresses and are issued in groups of
  // up to 8 elements per thread before any is used; the mask is applied
  // afterwards.
  {
    constexpr int EPT = F * F / NT;
    constexpr int G = EPT < 8 ? EPT : 8;
    static_assert(EPT % G == 0, "gather groups");
#pragma unroll
    for (int g0 = 0; g0 < EPT; g0 += G) {
      uint32_t pix[G], avb[G];
      float wv[G];
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int e = t + (g0 + r) * NT;
        const int m = e / F, n = e % F;
        const int y = min(max(ya + m, 0), a.H - 1), x = min(max(xa + n, 0), a.W - 1);
        const uint32_t p = (uint32_t)(y * pitch + x);
        pix[r] = img[p];
        avb[r] = av[p];
        const int da = min(abs(2 * m - (M - 1)), kWinStride - 1), db = min(abs(2 * n - (N - 1)), kWinStride - 1);
        wv[r] = a.wtab[da * kWinStride + db];
      }
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int e = t + (g0 + r) * NT;
        const int m = e / F, n = e % F;
        const int y = ya + m, x = xa + n;
        // B: the rectangle, or with a mask-driven loss area its lost pixels
        // (received pixels of the rectangle are then support)
        const bool inB = !a.masked_b && (m >= bo) && (m < bo + bh) && (n >= bo) && (n < bo + bw);
        const bool use = m < M && n < N && !inB && y >= 0 && y < a.H && x >= 0 && x < a.W && avb[r] != 0;
        const float w = wv[r];
        Wd[e] = use ? make_float2((float)pix[r] * w, kAlpha * w) : make_float2(0.f, 0.f);
      }
    }
  }
  lds_barrier();

  // 2. forward transform (eq. (7) on the F x F grid)
  fft_lines<F, NT, false>(Wd, s.tw, t);
  fft_lines<F, NT, true>(Wd, s.tw, t);

  if constexpr (MODE == kPower) {
    // |R_w|^2 of every bin, split and squared as the iterations below do
    float* pw = a.power + (int64_t)orig * (F * F);
    for (int e = t; e < F * F; e += NT) {
      const int k = e / F, l = e % F;
      const float2 zk = Wd[e];
      const float2 zn = Wd[((F - k) & (F - 1)) * F + ((F - l) & (F - 1))];
      const float rx = (zk.x + zn.x) * 0.5f, ry = (zk.y - zn.y) * 0.5f;
      pw[e] = fmaf(ry, ry, rx * rx);
    }
    lds_barrier();  // Wd is overwritten by the next block
    return kPending;
  }

  // Warm start: wave 0 takes R_w at its candidate bins straight from the
  // transform (same arithmetic as the split below, so the values are the
  // bits the split produces for those bins). A block whose network output
  // was unusable (flag set) runs plain FSE with the fallback count.
  const bool warm = KC > 0 && __builtin_amdgcn_readfirstlane(a.flags[orig]) == 0;
  const int I_full = KC > 0 && !warm ? a.fb_iters : I;
  if constexpr (MODE == kWarmPrep) {
    if (warm) {
      // stage W[k, l] for k <= F/2 (split as below) and R_w at the candidates
      float2* ws = a.stage_w + (int64_t)bi * (kHalfRows * F);
      for (int e = t; e < kHalfRows * F; e += NT) {
        const int k = e / F, l = e % F;
        const float2 zk = Wd[e];
        const float2 zn = Wd[((F - k) & (F - 1)) * F + ((F - l) & (F - 1))];
        ws[e] = make_float2((zk.y + zn.y) * (0.5f / kAlpha), (zn.x - zk.x) * (0.5f / kAlpha));
      }
      float2* rs = a.stage_r + (int64_t)bi * KC;
      for (int c = t; c < KC; c += NT) {
        const int ci = a.cand[(int64_t)orig * KC + c];
        const int k = ci / F, l = ci % F;
        const float2 zk = Wd[k * F + l];
        const float2 zn = Wd[((F - k) & (F - 1)) * F + ((F - l) & (F - 1))];
        rs[c] = make_float2((zk.x + zn.x) * 0.5f, (zk.y - zn.y) * 0.5f);
      }
      lds_barrier();  // Wd is overwritten by the next block
      return kPending;
    }
  }
  float cRx[CPL], cRy[CPL];
  int cIdx[CPL];
  if (FUSED && warm && wave == 0) {
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int ci = a.cand[(int64_t)orig * KC + j * 64 + lane];
      const int k = ci / F, l = ci % F;
      const float2 zk = Wd[k * F + l];
      const float2 zn = Wd[((F - k) & (F - 1)) * F + ((F - l) & (F - 1))];
      cIdx[j] = ci;
      cRx[j] = (zk.x + zn.x) * 0.5f;
      cRy[j] = (zk.y - zn.y) * 0.5f;
    }
  }

  // split Z = R_w + j*alpha*W by conjugate symmetry; R_w goes to VGPRs, W
  // is held until every thread has read Z, then written over it (rows
  // 0..RPG-2 also into their wrapped copies F..F+RPG-2).
  fvec<BPL> Rx, Ry;
  float2 Wv[BPL];
#pragma unroll
  for (int j = 0; j < BPL; ++j) {
    const int idx = gbase[j / SPG] + (j % SPG) * 64 + lane;
    const int k = idx / F, l = idx % F;
    const float2 zk = Wd[k * F + l];
    const float2 zn = Wd[((F - k) & (F - 1)) * F + ((F - l) & (F - 1))];
    Rx[j] = (zk.x + zn.x) * 0.5f;
    Ry[j] = (zk.y - zn.y) * 0.5f;
    Wv[j] = make_float2((zk.y + zn.y) * (0.5f / kAlpha), (zn.x - zk.x) * (0.5f / kAlpha));
  }
  const float W0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Wd[0].y))) * (1.0f / kAlpha);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < BPL; ++j) {
    const int idx = gbase[j / SPG] + (j % SPG) * 64 + lane;
    Wd[idx] = Wv[j];
    if (idx < (RPG - 1) * F) Wd[idx + F * F] = Wv[j];
  }
  __syncthreads();

  if (!(W0 > 0.f)) return FSE_BLOCK_EMPTY_SUPPORT;  // no received pixel in the area
  const float gW = a.gamma * (1.0f / W0);
  const float gWr = a.gamma_r * (1.0f / W0);

  // 3. iterations. |R_w|^2 is kept as its bit pattern: for values >= 0 the
  // unsigned order of the bits is the order of the values, so the argmax
  // runs on integer max/compare (a NaN sorts above every finite value and
  // is then reported as a non-finite coefficient).
  unsigned mb[BPL];
#pragma unroll
  for (int j = 0; j < BPL; ++j) mb[j] = __float_as_uint(fmaf(Ry[j], Ry[j], Rx[j] * Rx[j]));

  int tbase = 0;  // trace position of the first full iteration
  if constexpr (FUSED) {
    if (warm) {
      // Restricted phase (wave 0): FSE iterations whose argmax and update run
      // over the candidate bins only; the candidates are in ascending bin
      // order, so the lowest slot on ties is the lowest bin.
      if (wave == 0) {
        float cCx[CPL], cCy[CPL];
        unsigned cm[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          cCx[j] = 0.f;
          cCy[j] = 0.f;
          cm[j] = __float_as_uint(fmaf(cRy[j], cRy[j], cRx[j] * cRx[j]));
        }
        for (int it = 0; it < a.ir; ++it) {
          unsigned lm = cm[0];
#pragma unroll
          for (int j = 1; j < CPL; ++j) lm = max(lm, cm[j]);
          const unsigned wm = wave_max_bits(lm);
          int bj = CPL;
#pragma unroll
          for (int j = CPL - 1; j >= 0; --j) bj = (cm[j] == wm) ? j : bj;
          const unsigned key = wave_min_u32((unsigned)(bj * 64 + lane));
          const int wj = __builtin_amdgcn_readfirstlane((int)(key >> 6));
          const int wl = __builtin_amdgcn_readfirstlane((int)(key & 63));
          int bin = 0;
          float re = 0.f, im = 0.f;
#pragma unroll
          for (int j = 0; j < CPL; ++j) {
            if (j == wj) {
              bin = __builtin_amdgcn_readlane(cIdx[j], wl);
              re = readlane_f(cRx[j], wl);
              im = readlane_f(cRy[j], wl);
            }
          }
          const float cre = gWr * re, cim = gWr * im;    // eq. (13) with the restricted step
          s.cl_idx[it] = bin;                             // uniform stores
          s.cl_c[it] = make_float2(cre, cim);
          if (a.trace) {
            fse_trace_t rec;
            rec.u = (uint16_t)(bin / F);
            rec.v = (uint16_t)(bin % F);
            rec.c_re = cre;
            rec.c_im = cim;
            rec.r2 = __uint_as_float(wm);
            a.trace[(int64_t)orig * a.trace_stride + it] = rec;
          }
          const int u = bin / F, v = bin % F;
#pragma unroll
          for (int j = 0; j < CPL; ++j) {
            const bool hit = (j == wj) && (lane == wl);
            cCx[j] += hit ? cre : 0.f;
            cCy[j] += hit ? cim : 0.f;
            const int k = cIdx[j] / F, l = cIdx[j] % F;
            const float2 w = Wd[((k - u) & (F - 1)) * F + ((l - v) & (F - 1))];
            float rx = cRx[j], ry = cRy[j];
            rx = fmaf(-cre, w.x, rx);
            rx = fmaf(cim, w.y, rx);
            ry = fmaf(-cre, w.y, ry);
            ry = fmaf(-cim, w.x, ry);
            cRx[j] = rx;
            cRy[j] = ry;
            cm[j] = __float_as_uint(fmaf(ry, ry, rx * rx));
          }
        }
        // compact the candidates that received a coefficient
        int base = 0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const bool nz = cCx[j] != 0.f || cCy[j] != 0.f;
          const unsigned long long m = __ballot(nz);
          const int pos = base + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
          if (nz) {
            s.wl_idx[pos] = cIdx[j];
            s.wl_c[pos] = make_float2(cCx[j], cCy[j]);
          }
          base += __builtin_popcountll(m);
        }
        s.misc[1] = base;  // uniform store
      }
      __syncthreads();
      // Apply the restricted model to the whole spectrum (eq. (18) once per
      // distinct bin with its accumulated coefficient); not needed when no
      // full iteration follows.
      const int nw = I_full > 0 ? __builtin_amdgcn_readfirstlane(s.misc[1]) : 0;
      for (int q = 0; q < nw; ++q) {
        const int bin = __builtin_amdgcn_readfirstlane(s.wl_idx[q]);
        const float2 c = s.wl_c[q];
        const float cre = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c.x)));
        const float cim = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c.y)));
        const int u = bin / F, v = bin % F;
        int wb[GR][PH];
        shifted_bases(u, v, wb);
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
          const float2 w = Wd[wb[j / SPG][j % PH] + ((j % SPG) / PH) * 64 * PH];
          float rx = Rx[j], ry = Ry[j];
          rx = fmaf(-cre, w.x, rx);
          rx = fmaf(cim, w.y, rx);
          ry = fmaf(-cre, w.y, ry);
          ry = fmaf(-cim, w.x, ry);
          Rx[j] = rx;
          Ry[j] = ry;
        }
      }
#pragma unroll
      for (int j = 0; j < BPL; ++j) mb[j] = __float_as_uint(fmaf(Ry[j], Ry[j], Rx[j] * Rx[j]));
      tbase = a.ir;
    }
  }

  int sel = 0;
  float sre = 0.f, sim = 0.f, smag = 0.f;
  // Argmax over the workgroup, lowest linear index on ties. In a wave the
  // linear index grows with (slot j, lane), so the wave's winner is the
  // lowest slot, then the lowest lane, holding the wave maximum.
  auto select = [&]() {
    // The argmax is the serial part of an iteration, and the other waves of
    // the block wait for it at the barrier below: its instructions go ahead
    // of the update streams of the compute unit's other blocks.
    __builtin_amdgcn_s_setprio(3);
    // running maxima over slot pairs: pm[i] = max over slots 0 .. 2 i + 1
    constexpr int NP = (BPL + 1) / 2;
    unsigned pm[NP];
    pm[0] = BPL > 1 ? max(mb[0], mb[BPL > 1 ? 1 : 0]) : mb[0];
#pragma unroll
    for (int i = 1; i < NP; ++i) pm[i] = max(pm[i - 1], 2 * i + 1 < BPL ? max(mb[2 * i], mb[2 * i + 1]) : mb[2 * i]);
    const unsigned lm = pm[NP - 1];
    const unsigned wm = wave_max_bits(lm);
    const unsigned long long cand = __ballot(lm == wm);
    int wj = 0, wl;
    if (__builtin_popcountll(cand) == 1) {
      // usual case: one lane holds the maximum; on the scalar unit, the first
      // pair whose running maximum reaches it, then the slot within the pair
      wl = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(cand));
      int pi = NP - 1;
#pragma unroll
      for (int i = NP - 2; i >= 0; --i) pi = ((unsigned)__builtin_amdgcn_readlane((int)pm[i], wl) == wm) ? i : pi;
      const int j0 = __builtin_amdgcn_readfirstlane(2 * pi);
      wj = (j0 + 1 < BPL && (unsigned)__builtin_amdgcn_readlane((int)mb[j0], wl) != wm) ? j0 + 1 : j0;
    } else {
      // several lanes hold it (exact ties, e.g. conjugate bins): take the
      // lowest (slot, lane) key over the wave
      int bj = BPL;
#pragma unroll
      for (int j = BPL - 1; j >= 0; --j) bj = (mb[j] == wm) ? j : bj;
      const unsigned key = wave_min_u32((unsigned)(bj * 64 + lane));
      wj = (int)(key >> 6);
      wl = (int)(key & 63);
    }
    wj = __builtin_amdgcn_readfirstlane(wj);
    const float re = readlane_f(Rx[wj], wl);
    const float im = readlane_f(Ry[wj], wl);
    const int widx = __builtin_amdgcn_readfirstlane(gbase[wj / SPG]) + (wj % SPG) * 64 + wl;
    if constexpr (NW == 1) {
      sel = widx; sre = re; sim = im; smag = __uint_as_float(wm);
    } else {
      int4* slot = s.red + parity * NW;
      slot[wave] = make_int4((int)wm, widx, __float_as_int(re), __float_as_int(im));  // uniform
      __syncthreads();
      // lane i < NW holds wave i's candidate; key = (|R|^2 bits, ~index) so
      // the largest key is the largest value with the lowest index
      // Every group of NW lanes holds the NW entries: the largest value over
      // the group, then the lowest index among the entries holding it.
      const int4 o = slot[lane & (NW - 1)];
      const unsigned gm = group_reduce<NW, true>((unsigned)o.x);
      const unsigned key = group_reduce<NW, false>((unsigned)o.x == gm ? (unsigned)o.y : 0xffffffffu);
      sel = __builtin_amdgcn_readfirstlane((int)key);
      smag = __uint_as_float((unsigned)__builtin_amdgcn_readfirstlane((int)gm));
      // lane i holds wave i's entry: the winner's value without another LDS read
      const int ww = S::wave_of_row((int)((unsigned)sel / F));
      sre = __int_as_float(__builtin_amdgcn_readlane(o.z, ww));
      sim = __int_as_float(__builtin_amdgcn_readlane(o.w, ww));
      parity ^= 1;
    }
    __builtin_amdgcn_s_setprio(0);
  };
  if (I_full > 0) select();

  for (int it = 0; it < I_full; ++it) {
    const float cre = gW * sre, cim = gW * sim;          // eq. (13)
    // All lanes of wave 0 store the same uniform values: no lane-divergent
    // region inside the loops (see the persistent loop below).
    if (wave == 0) {
      s.cl_idx[tbase + it] = sel;                         // eq. (15): G[u,v] += F*F*c
      s.cl_c[tbase + it] = make_float2(cre, cim);
      if (a.trace) {
        fse_trace_t rec;
        rec.u = (uint16_t)(sel / F);
        rec.v = (uint16_t)(sel % F);
        rec.c_re = cre;
        rec.c_im = cim;
        rec.r2 = smag;
        a.trace[(int64_t)orig * a.trace_stride + tbase + it] = rec;
      }
    }
    if (it + 1 == I_full) break;
    const int u = sel / F, v = sel % F;
    // eq. (18): R_w[k,l] -= c * W[k-u, l-v] over the wave's bins, fused with
    // |R_w|^2. Within a row group the rows of later slots follow the first
    // one's row (k-u) mod F consecutively (wrapped copies cover the overflow).
    int wb[GR][PH];
    shifted_bases(u, v, wb);
#pragma unroll
    for (int j = 0; j < BPL; ++j) {
      const float2 w = Wd[wb[j / SPG][j % PH] + ((j % SPG) / PH) * 64 * PH];
      float rx = Rx[j], ry = Ry[j];
      rx = fmaf(-cre, w.x, rx);
      rx = fmaf(cim, w.y, rx);
      ry = fmaf(-cre, w.y, ry);
      ry = fmaf(-cim, w.x, ry);
      Rx[j] = rx;
      Ry[j] = ry;
      mb[j] = __float_as_uint(fmaf(ry, ry, rx * rx));
    }
    select();
  }
  // every coefficient (restricted phase included) must be finite; checked
  // once over the list instead of in every iteration (a NaN |R_w|^2 sorts
  // above every finite value, so it is selected and its coefficient listed)
  bool bad = false;
  for (int it = t; it < tbase + I_full; it += NT) {
    const float2 c = s.cl_c[it];
    bad = bad || !isfinite(c.x) || !isfinite(c.y);
  }
  if (__syncthreads_or(bad)) return FSE_BLOCK_NONFINITE;

  // 4. model on B
  synthesize<F, NT, 1>(s.cl_idx, s.cl_c, tbase + I_full, s.tw, bh, bw, bo,
                       a.out + (fofs + bd.y0) * a.out_pitch + bd.x0, a.out_pitch, t,
                       a.masked_b ? av + (int64_t)bd.y0 * pitch + bd.x0 : nullptr, pitch);
  return FSE_BLOCK_OK;
}

template <int F, int NT, int KC, int MODE>
// The transform kernel of the split warm start is held to 64 registers: with
// its LDS (38 KB without the fused form's lists) four 512-thread workgroups
// then share a compute unit.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MODE >= kWarmPrep ? 8 : 1))) void fse_persistent(
    ClassArgs a) {
  using S = Shape<F, NT>;
  extern __shared__ __align__(16) unsigned char smem[];
  Lds s;
  s.Wd = reinterpret_cast<float2*>(smem);
  s.tw = s.Wd + S::WROWS * F;
  s.red = reinterpret_cast<int4*>(s.tw + F);
  s.cl_c = reinterpret_cast<float2*>(s.red + 2 * S::NW);
  // the distinct-bin lists of the restricted phase exist in the fused form only
  constexpr int KCL = MODE == kWarmFused ? KC : 0;
  s.wl_c = s.cl_c + a.iters_cap;
  s.cl_idx = reinterpret_cast<int*>(s.wl_c + KCL);
  s.wl_idx = s.cl_idx + a.iters_cap;
  s.misc = s.wl_idx + KCL;

  const int t = threadIdx.x;
  for (int i = t; i < F; i += NT) s.tw[i] = a.twid[i];
  int parity = 0;

  // Persistent loop, one block per pass. The loop body contains no
  // lane-divergent region: the queue is popped by the whole first wave with
  // one lane adding 1 and the others 0, the result is made uniform with
  // readfirstlane, and bookkeeping stores are done by every lane of wave 0
  // with the same value. (A thread-0-only pop followed by a barrier is not
  // safe in a single-wave workgroup: without a real barrier the compiler may
  // let the other lanes run ahead into the next pass.)
  const int lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  if constexpr (MODE == kWarmPrep || MODE == kPower) {
    // The transform kernel of the split warm start costs the same for every
    // block: workgroup g takes blocks g, g + grid, ... without the queue,
    // whose single counter, contended by every workgroup, cost more per
    // block than the gather.
    for (int bi = blockIdx.x; bi < a.n; bi += gridDim.x) {
      int tb = t;
      asm volatile("" : "+v"(tb));
      const int code = conceal_block<F, NT, KC, MODE>(a, bi, s, tb, parity);
      if (wave == 0 && code != kPending) a.status[a.orig[bi]] = code;
    }
    return;
  }
  // The first block of a workgroup is its own index; each later one is
  // grid + (the queue's next value), popped as the previous block starts so
  // that the atomic's latency overlaps that block's work.
  int bi = blockIdx.x;  // the grid never exceeds the class's block count
  for (;;) {
    int nxv = 0;
    if (wave == 0) nxv = atomicAdd(&a.queue[0], lane == 0 ? 1 : 0);  // read after the block
    // An opaque copy of the thread index keeps the compiler from hoisting
    // every index-derived LDS address out of this loop, where they would
    // stay live in VGPRs for the whole kernel; recomputing them per block
    // costs a few instructions.
    int tb = t;
    asm volatile("" : "+v"(tb));
    const int code = conceal_block<F, NT, KC, MODE>(a, bi, s, tb, parity);
    if (wave == 0 && code != kPending) a.status[a.orig[bi]] = code;
    if constexpr (S::NW == 1) {
      bi = __builtin_amdgcn_readfirstlane(nxv) + (int)gridDim.x;
    } else {
      if (wave == 0) s.misc[0] = __builtin_amdgcn_readfirstlane(nxv) + (int)gridDim.x;
      __syncthreads();
      bi = __builtin_amdgcn_readfirstlane(s.misc[0]);
      __syncthreads();
    }
    if (bi >= a.n) break;
  }

  // the last workgroup to leave re-arms the queue for the next launch
  if (wave == 0) {
    __threadfence();
    const int done = __builtin_amdgcn_readfirstlane(atomicAdd(&a.queue[1], lane == 0 ? 1 : 0));
    if (done == (int)gridDim.x - 1 && lane == 0) {
      atomicExch(&a.queue[0], 0);
      atomicExch(&a.queue[1], 0);
    }
  }
}

// ------------------------------------------------------------ restricted
template <bool B>
struct BoolC {
  static constexpr bool value = B;
};

// Second kernel of the split warm start (F = 64): the restricted iterations
// of one block per workgroup of NWB waves, with W rows 0..32 in LDS (17 KB,
// so that many blocks share a compute unit and hide each other's latency)
// and the KC candidates in VGPRs: wave w holds candidates
// [w*KC/NWB, (w+1)*KC/NWB), KC/(64*NWB) consecutive ones per lane. Each
// iteration: argmax of |R_w|^2 over the candidates (eq. (12), lowest bin on
// ties), c = gamma*R_w[u,v]/W[0,0] (eq. (13)), R_w[k,l] -= c*W[k-u,l-v] at
// the candidates (eq. (18)); then the model is evaluated on B as in the
// persistent kernel. The arithmetic of every step is that of the fused
// warm-started form, so both give the same bits.
template <int KC, int NWB>
__global__ __launch_bounds__(64 * NWB) void fse_restricted(ClassArgs a) {
  constexpr int F = 64, NT = 64 * NWB, CPL = KC / NT;
  static_assert(NWB == 1 || NWB == 2, "one or two waves per block");
  static_assert(KC % NT == 0 && CPL >= 1 && CPL <= 16, "candidate count must be a multiple of the thread count");
  // W and the twiddles at fixed LDS addresses, so that every address into
  // them is an offset the compiler knows; the dynamic part holds the
  // cross-wave slots (two waves) and the coefficient list (large B only)
  __shared__ __align__(16) float2 Wh[kHalfRows * F];  // W rows 0..F/2
  __shared__ __align__(16) float2 tw[F];              // F twiddles
  extern __shared__ __align__(16) unsigned char smem[];
  int4* const xch = reinterpret_cast<int4*>(smem);    // 2 x NWB cross-wave argmax slots (two waves)
  float2* const cl_c = reinterpret_cast<float2*>(xch + (NWB == 2 ? 4 : 0));  // ir coefficients
  int* const cl_idx = reinterpret_cast<int*>(cl_c + a.ir);
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int bi = blockIdx.x;
  if (bi >= a.n) return;
  const int orig = __builtin_amdgcn_readfirstlane(a.orig[bi]);
  if (__builtin_amdgcn_readfirstlane(a.flags[orig]) != 0) return;  // concealed by the transform kernel

  {
    const float4* src = reinterpret_cast<const float4*>(a.stage_w + (int64_t)bi * (kHalfRows * F));
    float4* dst = reinterpret_cast<float4*>(Wh);
    for (int e = t; e < kHalfRows * F / 2; e += NT) dst[e] = src[e];
    if (t < F) tw[t] = a.twid[t];
  }
  // Candidate c = wave*KC/NWB + lane*CPL + j. Its bin (k, l) is kept as
  // xa = k*4096 + l*8: adding (64-u)*4096 + (64-v)*8 gives (k-u+64) above
  // bit 12 and (l-v+64)*8 in bits 3..9 (no borrow between the fields), so
  // the byte offset of W[(k-u) mod 64, (l-v) mod 64] (row pitch 512 B) is
  // ((y >> 3) & 0x7e00) | (y & 0x1f8); subtracting xa from
  // (64+u)*4096 + (64+v)*8 gives the mirrored bin the same way.
  fvec<CPL> Rx, Ry;
  int __attribute__((ext_vector_type(CPL))) xa;
  unsigned mb[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = wave * (KC / NWB) + lane * CPL + j;
    const int bin = a.cand[(int64_t)orig * KC + c];
    const int k = bin / F, l = bin % F;
    const float2 r = a.stage_r[(int64_t)bi * KC + c];
    Rx[j] = r.x;
    Ry[j] = r.y;
    xa[j] = k * 4096 + l * 8;
    mb[j] = __float_as_uint(fmaf(r.y, r.y, r.x * r.x));
  }
  const char* const Wb = reinterpret_cast<const char*>(Wh);
  __syncthreads();
  const float W0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Wh[0].x)));
  if (!(W0 > 0.f)) {
    if (wave == 0) a.status[orig] = FSE_BLOCK_EMPTY_SUPPORT;
    return;
  }
  const float gW = a.gamma_r * (1.0f / W0);  // the restricted step

  // The model on B (as in the persistent kernel) is accumulated inside the
  // loop when the block has at most NT*QI pixels (QI per thread), in the
  // same per-pixel order as the list-based synthesis after the loop, which
  // larger blocks use.
  constexpr int QI = 4 / NWB;
  static_assert(NT * QI == kRestrictedInloopPixels, "in-loop synthesis bound known to the host");
  const UBlock bd = uniform_block(a.blocks + bi);
  const int np = bd.bh * bd.bw;
  const bool inloop = np <= NT * QI;
  int mq[QI], nq[QI];  // area position of the thread's pixels, times 8 (byte scale of the twiddle table)
  float acc[QI];
#pragma unroll
  for (int q = 0; q < QI; ++q) {
    const int p = min(t + q * NT, np - 1);
    mq[q] = 8 * (bd.border + p / bd.bw);
    nq[q] = 8 * (bd.border + p % bd.bw);
    acc[q] = 0.f;
  }
  const char* const twb = reinterpret_cast<const char*>(tw);

  bool finite = true;
  int parity = 0;
  // The iteration loop, compiled once per combination of the two
  // block-uniform options (in-loop synthesis, trace), so that neither is
  // tested inside it.
  auto iterate = [&](auto inloop_c, auto trace_c) __attribute__((always_inline)) {
  constexpr bool kInloop = decltype(inloop_c)::value, kTrace = decltype(trace_c)::value;
  for (int it = 0; it < a.ir; ++it) {
    unsigned lm = mb[0];
#pragma unroll
    for (int j = 1; j < CPL; ++j) lm = max(lm, mb[j]);
    unsigned wm = wave_max_bits(lm);
    // the wave's lowest candidate holding its maximum: lowest lane, then j
    // (one lane mask per slot on the scalar unit)
    unsigned long long hm[CPL], hits = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      hm[j] = __ballot(mb[j] == wm);
      hits |= hm[j];
    }
    const int wl = (int)__builtin_ctzll(hits);
    int wj = CPL - 1;
#pragma unroll
    for (int j = CPL - 2; j >= 0; --j) wj = ((hm[j] >> wl) & 1) ? j : wj;
    // wj is uniform: the slot is picked by relative register addressing
    float re = readlane_f(Rx[wj], wl), im = readlane_f(Ry[wj], wl);
    int x = __builtin_amdgcn_readlane(xa[wj], wl);
    if constexpr (NWB == 2) {
      // across the two waves: the larger value, wave 0 (the lower
      // candidates) on a tie; every component made uniform before selecting
      xch[parity * 2 + wave] = make_int4((int)wm, x, __float_as_int(re), __float_as_int(im));  // uniform
      __syncthreads();
      const int4 s0 = xch[parity * 2], s1 = xch[parity * 2 + 1];
      const unsigned m0 = (unsigned)__builtin_amdgcn_readfirstlane(s0.x);
      const unsigned m1 = (unsigned)__builtin_amdgcn_readfirstlane(s1.x);
      const int x0 = __builtin_amdgcn_readfirstlane(s0.y), x1 = __builtin_amdgcn_readfirstlane(s1.y);
      const int r0 = __builtin_amdgcn_readfirstlane(s0.z), r1 = __builtin_amdgcn_readfirstlane(s1.z);
      const int i0 = __builtin_amdgcn_readfirstlane(s0.w), i1 = __builtin_amdgcn_readfirstlane(s1.w);
      const bool second = m1 > m0;
      wm = second ? m1 : m0;
      x = second ? x1 : x0;
      re = __int_as_float(second ? r1 : r0);
      im = __int_as_float(second ? i1 : i0);
      parity ^= 1;
    }
    const int u = x >> 12, v = (x >> 3) & 511;
    const float cre = gW * re, cim = gW * im;  // eq. (13)
    finite = finite & isfinite(cre) & isfinite(cim);  // no short circuit: no branch
    if constexpr (kInloop) {
#pragma unroll
      for (int q = 0; q < QI; ++q) {
        const float2 e = *reinterpret_cast<const float2*>(twb + phase_byte<F>(u, v, mq[q], nq[q]));  // as in synthesize: Re{c e^{j theta}} = c.x e.x + c.y e.y
        acc[q] = fmaf(cre, e.x, acc[q]);
        acc[q] = fmaf(cim, e.y, acc[q]);
      }
    }
    if (NWB == 1 || wave == 0) {
      if constexpr (!kInloop) {
        cl_idx[it] = u * F + v;  // uniform stores
        cl_c[it] = make_float2(cre, cim);
      }
      if constexpr (kTrace) {
        fse_trace_t rec;
        rec.u = (uint16_t)u;
        rec.v = (uint16_t)v;
        rec.c_re = cre;
        rec.c_im = cim;
        rec.r2 = __uint_as_float(wm);
        a.trace[(int64_t)orig * a.trace_stride + it] = rec;
      }
    }
    // eq. (18) at the candidates: W[k-u, l-v] from row (k-u) mod F when
    // that is <= F/2, else the conjugate of W[u-k, v-l]
    int ca = (F - u) * 4096 + (F - v) * 8;
    int cb = (F + u) * 4096 + (F + v) * 8;
    asm volatile("" : "+s"(ca), "+s"(cb));  // opaque: one add per candidate, not two
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int ya = xa[j] + ca, yb = cb - xa[j];
      const bool flip = (ya & 0x3f000) > (F / 2) * 4096;
      const int y = flip ? yb : ya;
      float2 w = *reinterpret_cast<const float2*>(Wb + (((y >> 3) & 0x7e00) | (y & 0x1f8)));
      w.y = flip ? -w.y : w.y;
      float rx = Rx[j], ry = Ry[j];
      rx = fmaf(-cre, w.x, rx);
      rx = fmaf(cim, w.y, rx);
      ry = fmaf(-cre, w.y, ry);
      ry = fmaf(-cim, w.x, ry);
      Rx[j] = rx;
      Ry[j] = ry;
      mb[j] = __float_as_uint(fmaf(ry, ry, rx * rx));
    }
  }
  };
  if (inloop) {
    if (a.trace) iterate(BoolC<true>{}, BoolC<true>{});
    else iterate(BoolC<true>{}, BoolC<false>{});
  } else {
    if (a.trace) iterate(BoolC<false>{}, BoolC<true>{});
    else iterate(BoolC<false>{}, BoolC<false>{});
  }
  // every coefficient must be finite (all waves computed the same ones)
  if (!finite) {
    if (wave == 0) a.status[orig] = FSE_BLOCK_NONFINITE;
    return;
  }
  const int64_t fofs = (int64_t)bd.frame * a.H;
  float* const ob = a.out + (fofs + bd.y0) * a.out_pitch + bd.x0;
  if (inloop) {
#pragma unroll
    for (int q = 0; q < QI; ++q)
      if (t + q * NT < np) ob[(int64_t)(mq[q] / 8 - bd.border) * a.out_pitch + (nq[q] / 8 - bd.border)] = acc[q];
  } else {
    __syncthreads();
    synthesize<F, NT, 4 / NWB>(cl_idx, cl_c, a.ir, tw, bd.bh, bd.bw, bd.border, ob, a.out_pitch, t);
  }
  if (wave == 0) a.status[orig] = FSE_BLOCK_OK;
}

template <int F, int NT, int KC = 0, int MODE = kPlain>
constexpr Variant make_variant() {
  return Variant{F, NT, KC, MODE, reinterpret_cast<const void*>(&fse_persistent<F, NT, KC, MODE>)};
}

// Workgroup shapes compiled for each transform size. The first entry of
// each size is the default; the autotuner may pick another per batch. The
// entries with KC > 0 are the warm-started forms.
const Variant kVariants[] = {
    make_variant<32, 64>(),  make_variant<32, 128>(), make_variant<32, 256>(),
    make_variant<64, 256>(), make_variant<64, 128>(), make_variant<64, 512>(),
    make_variant<128, 1024>(), make_variant<128, 512>(),
    make_variant<64, 256, 256, kWarmFused>(), make_variant<64, 256, 128, kWarmFused>(),
    make_variant<64, 256, 512, kWarmFused>(),
    make_variant<64, 512, 256, kWarmPrep>(), make_variant<64, 512, 128, kWarmPrep>(),
    make_variant<64, 512, 512, kWarmPrep>(), make_variant<64, 512, 384, kWarmPrep>(),
    make_variant<64, 512, 0, kPower>(),
};


// ------------------------------------------------------------ 3-D (video)
// cFSE of one lost volume per workgroup of kNT3 = 1024 threads, F = 64,
// Ft = 8 (the iteration of Section III on a 3-D grid). Bin (k, l, s) has
// the linear index (k F + l) Ft + s.
//
// Spectra without a round trip through memory: the temporal 8-point DFT of
// z = s w + j alpha w is taken first, per pixel, straight from the frames;
// the 64 x 64 spatial FFTs of its eight s-slices then run in LDS in four
// rounds of slices closed under s -> -s ({1, 7, 2, 6}, {3, 5}, {0}, {4}), so
// that the conjugate-symmetric split of a bin and of its mirror (-k, -l, -s)
// finds both slices in the same round. W is kept for l <= 32 (the rest is
// W[-k, -l, -s] conjugated) as eight s-slots of 33 x 64 values, [l][k]. The
// rounds fill the slots in the order they produce them, each round's FFT
// buffers lying over the slots not yet written (the values a round produces
// wait in registers until its buffers are dead); one permutation then puts
// slot s at W[., ., s].
constexpr int kSlot3 = kHalfCols3 * kF3;  // float2 entries per s-slot of W
// slot each s is produced into, 4 bits per s (the rounds write s = 1, 7, 2, 6, 3, 5, 0, 4)
constexpr uint32_t kSlotOf3 = 0x13574206u;
__host__ __device__ constexpr int slot_of3(int s) { return (int)((kSlotOf3 >> (4 * s)) & 7u); }
static_assert(slot_of3(1) == 0 && slot_of3(7) == 1 && slot_of3(2) == 2 && slot_of3(6) == 3 && slot_of3(3) == 4 &&
                  slot_of3(5) == 5 && slot_of3(0) == 6 && slot_of3(4) == 7,
              "slots in the order the rounds write them");
// LDS: twiddles [0, 512), argmax exchange [512, 1024), then W; the
// coefficient list follows W (over the last round's FFT buffer, dead by then)
constexpr int kW3Ofs = 1024;
constexpr int kW3Bytes = kFt3 * kSlot3 * 8;
constexpr int kFftBuf3 = kF3 * kF3;  // float2 entries of one FFT buffer
static_assert(4 * kFftBuf3 <= kFt3 * kSlot3 && 4 * kSlot3 + 2 * kFftBuf3 <= kFt3 * kSlot3 &&
                  6 * kSlot3 + kFftBuf3 <= kFt3 * kSlot3,
              "the buffers of rounds 1-3 lie inside W");

// 2-D FFT of a 64 x 64 buffer filled as [m][n]: columns first, then rows,
// the last pass written transposed, so that buf[l * 64 + k] holds Z(k, l)
// and a wave reading one l for 64 consecutive k reads consecutive entries.
template <int NT>
__device__ __forceinline__ void fft2_lk(float2* buf, const float2* tw, int t) {
  fft_pass<kF3, NT, 8, 1, true>(buf, tw, t);
  fft_pass<kF3, NT, 8, 8, true>(buf, tw, t);
  fft_pass<kF3, NT, 8, 1, false>(buf, tw, t);
  fft_pass<kF3, NT, 8, 8, false, true>(buf, tw, t);
}

// The split of slice S (buffer bs) against slice -S (buffer bm): with
// P = Z(k, l, S) and Q = Z(-k, -l, -S), R_w = (P + conj Q) / 2 and
// W = (P - conj Q) / (2 j alpha). The thread's columns are (k, l) =
// (lane, 4 wv + cc): R_w of the plain form goes to its registers, W for
// l <= 32 to wp. In the warm form waves 0-3 take R_w at their candidates
// (column (ck, cl), s = 4 h + j) instead.
template <bool WARM, int S, int NR>
__device__ __forceinline__ void split3(const float2* bs, const float2* bm, int wv, int kk, float (&Rx)[NR],
                                       float (&Ry)[NR], float2 (&wp)[4], int ck, int cl, int h) {
  constexpr int F = kF3;
  const int km = (F - kk) & (F - 1);
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    const int l = 4 * wv + cc;
    const bool needW = l <= F / 2;  // uniform
    wp[cc] = make_float2(0.f, 0.f);  // defined on every path (no value carried across volumes)
    if (WARM && !needW) continue;
    const float2 P = bs[l * F + kk], Q = bm[((F - l) & (F - 1)) * F + km];
    if constexpr (!WARM) {
      Rx[cc * kFt3 + S] = 0.5f * (P.x + Q.x);
      Ry[cc * kFt3 + S] = 0.5f * (P.y - Q.y);
      asm volatile("" : "+v"(Rx[cc * kFt3 + S]), "+v"(Ry[cc * kFt3 + S]));  // held as R_w, not as P and Q
    }
    if (needW) wp[cc] = make_float2((P.y + Q.y) * (0.5f / kAlpha), (Q.x - P.x) * (0.5f / kAlpha));
    asm volatile("" : "+v"(wp[cc].x), "+v"(wp[cc].y));  // held as W, not as P and Q
  }
  if constexpr (WARM) {
    if (wv < 4 && (S >> 2) == h) {
      const float2 P = bs[cl * F + ck], Q = bm[((F - cl) & (F - 1)) * F + ((F - ck) & (F - 1))];
      Rx[S & 3] = 0.5f * (P.x + Q.x);
      Ry[S & 3] = 0.5f * (P.y - Q.y);
      asm volatile("" : "+v"(Rx[S & 3]), "+v"(Ry[S & 3]));
    }
  }
  asm volatile("" ::: "memory");  // one slice's reads in flight at a time
}

template <int S>
__device__ __forceinline__ void store_w3(float2* Wl, const float2 (&wp)[4], int wv, int kk) {
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    const int l = 4 * wv + cc;
    if (l <= kF3 / 2) Wl[slot_of3(S) * kSlot3 + l * kF3 + kk] = wp[cc];
  }
}

__device__ __forceinline__ uint32_t bits_max_first(uint32_t bits, uint32_t& best) {
  return bits > best ? (best = bits, 1u) : 0u;
}

// WARM restricts the argmax to candidate bins: for each volume, kCand3
// columns (k, l) (a row of cand2, ascending) with all Ft values of s. Waves
// 0-3, one per SIMD, iterate: wave w holds the columns 64 (w & 1) + lane and
// s = 4 (w >> 1) + j, j < 4, so lane and j order is index order within a
// wave; the other waves only take part in the barrier of each iteration.
template <bool WARM>
__global__ __launch_bounds__(kNT3) void fse3d(Vol3Args a) {
  constexpr int F = kF3, FT = kFt3, NT = kNT3, BPT = F * F * FT / NT;  // 32 bins per thread
  extern __shared__ __align__(16) unsigned char smem[];
  float2* const tw = reinterpret_cast<float2*>(smem);
  int4* const xch = reinterpret_cast<int4*>(smem + 512);  // 2 x 16 argmax slots
  float2* const Wl = reinterpret_cast<float2*>(smem + kW3Ofs);
  float2* const cl_c = reinterpret_cast<float2*>(smem + kW3Ofs + kW3Bytes);
  int* const cl_idx = reinterpret_cast<int*>(cl_c + a.iters_cap);
  const int t0 = threadIdx.x;
  if (t0 < F) tw[t0] = a.twid[t0];
  int parity = 0;
  for (int vi = blockIdx.x; vi < a.n; vi += gridDim.x) {
    // opaque thread index: keeps index-derived addresses out of the volume loop
    int t = t0;
    asm volatile("" : "+v"(t));
    const fse_volume_t* vp = a.vols + vi;
    const int f0 = __builtin_amdgcn_readfirstlane(vp->frame);
    const int y0 = __builtin_amdgcn_readfirstlane(vp->y0), x0 = __builtin_amdgcn_readfirstlane(vp->x0);
    const int bt = __builtin_amdgcn_readfirstlane(vp->bt), bh = __builtin_amdgcn_readfirstlane(vp->bh);
    const int bw = __builtin_amdgcn_readfirstlane(vp->bw), bd = __builtin_amdgcn_readfirstlane(vp->border);
    const int td = __builtin_amdgcn_readfirstlane(vp->tborder), I = __builtin_amdgcn_readfirstlane(vp->iters);
    const int M = bh + 2 * bd, N = bw + 2 * bd, T = bt + 2 * td;
    const int ya = y0 - bd, xa = x0 - bd, ta = f0 - td;
    if constexpr (WARM) {
      // a candidate row the network could not provide: left to the caller
      if (__builtin_amdgcn_readfirstlane(a.flags[vi]) != 0) {
        if (t == 0) a.status[vi] = FSE_BLOCK_NONFINITE;
        continue;
      }
    }
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6), kk = t & (F - 1);

    // 1. gather, window (eq. (3)), z = s w + j alpha w, and the temporal DFT
    // of z per pixel; thread t takes the pixels (m, n) = (t / 64 + 16 q, t % 64).
    // The slices of the first round go to its four FFT buffers, the others
    // stay in registers for the later rounds.
    float2 keep[4][4];  // s = 3, 5, 0, 4
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = wv + 16 * q, n = kk;
      const int y = ya + m, x = xa + n;
      const bool inA = m < M && n < N && y >= 0 && y < a.H && x >= 0 && x < a.W;
      const bool inBmn = m >= bd && m < bd + bh && n >= bd && n < bd + bw;
      const int da = min(abs(2 * m - (M - 1)), kWinStride - 1), db = min(abs(2 * n - (N - 1)), kWinStride - 1);
      const uint32_t p = inA ? (uint32_t)(y * (int)a.pitch + x) : 0u;
      const int dab = da * kWinStride + db;
      // every load reads a valid address (a frame of the clip, pixel 0 when
      // unused), so that all of them issue before the first wait; the frame
      // offsets are uniform
      float2 z[FT];
#pragma unroll
      for (int sl = 0; sl < FT; ++sl) {
        const int f = ta + sl;
        const int64_t fo = (int64_t)min(max(f, 0), a.n_frames - 1) * a.H * a.pitch;
        const bool use = inA && sl < T && f >= 0 && f < a.n_frames && !(inBmn && sl >= td && sl < td + bt);
        const uint32_t o = use ? p : 0u;
        const uint8_t av = (a.avail + fo)[o], px = (a.img + fo)[o];
        const int dc = min(abs(2 * sl - (T - 1)), kWinStrideT - 1);
        const float w = (a.wtab3 + dc * kWinStride * kWinStride)[dab];
        // the window where the pixel counts, else +0 (a mask, not a branch)
        const float wu = __int_as_float(__float_as_int(w) & -(int)(use && av != 0));
        z[sl] = make_float2((float)px * wu, kAlpha * wu);
      }
      dft_small<FT>(z);  // z[s] = sum_t z_t exp(-j 2 pi s t / Ft)
      const int e = m * F + n;
      Wl[0 * kFftBuf3 + e] = z[1];
      Wl[1 * kFftBuf3 + e] = z[7];
      Wl[2 * kFftBuf3 + e] = z[2];
      Wl[3 * kFftBuf3 + e] = z[6];
      keep[q][0] = z[3];
      keep[q][1] = z[5];
      keep[q][2] = z[0];
      keep[q][3] = z[4];
      // the kept slices as values now (not their inputs), and one pixel's
      // loads in flight at a time
      asm volatile("" : "+v"(keep[q][0].x), "+v"(keep[q][0].y), "+v"(keep[q][1].x), "+v"(keep[q][1].y),
                   "+v"(keep[q][2].x), "+v"(keep[q][2].y), "+v"(keep[q][3].x), "+v"(keep[q][3].y)::"memory");
    }

    // 2. the spatial FFTs and the conjugate-symmetric split, round by round:
    // R_w into registers, W into its s-slots
    float Rx[WARM ? 4 : BPT], Ry[WARM ? 4 : BPT];
    if constexpr (WARM) {
#pragma unroll
      for (int j = 0; j < 4; ++j) Rx[j] = Ry[j] = 0.f;
    }
    int ck = 0, cl = 0, c2 = 0;
    const int h = wv >> 1;
    if constexpr (WARM) {
      if (wv < 4) {
        c2 = a.cand2[(int64_t)vi * kCand3 + (wv & 1) * 64 + kk];
        ck = c2 >> 6;
        cl = c2 & (F - 1);
      }
    }
    {  // round 1: s = 1, 7, 2, 6
      __syncthreads();
      fft2_lk<256>(Wl + (t >> 8) * kFftBuf3, tw, t & 255);
      float2 wp[4][4];
      split3<WARM, 1>(Wl + 0 * kFftBuf3, Wl + 1 * kFftBuf3, wv, kk, Rx, Ry, wp[0], ck, cl, h);
      split3<WARM, 7>(Wl + 1 * kFftBuf3, Wl + 0 * kFftBuf3, wv, kk, Rx, Ry, wp[1], ck, cl, h);
      split3<WARM, 2>(Wl + 2 * kFftBuf3, Wl + 3 * kFftBuf3, wv, kk, Rx, Ry, wp[2], ck, cl, h);
      split3<WARM, 6>(Wl + 3 * kFftBuf3, Wl + 2 * kFftBuf3, wv, kk, Rx, Ry, wp[3], ck, cl, h);
      lds_barrier();  // the buffers are dead
      store_w3<1>(Wl, wp[0], wv, kk);
      store_w3<7>(Wl, wp[1], wv, kk);
      store_w3<2>(Wl, wp[2], wv, kk);
      store_w3<6>(Wl, wp[3], wv, kk);
    }
    {  // round 2: s = 3, 5, over slots 4-7
      float2* const b3 = Wl + 4 * kSlot3;
      float2* const b5 = b3 + kFftBuf3;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        b3[(wv + 16 * q) * F + kk] = keep[q][0];
        b5[(wv + 16 * q) * F + kk] = keep[q][1];
      }
      lds_barrier();
      fft2_lk<512>(b3 + (t >> 9) * kFftBuf3, tw, t & 511);
      float2 wp[2][4];
      split3<WARM, 3>(b3, b5, wv, kk, Rx, Ry, wp[0], ck, cl, h);
      split3<WARM, 5>(b5, b3, wv, kk, Rx, Ry, wp[1], ck, cl, h);
      lds_barrier();
      store_w3<3>(Wl, wp[0], wv, kk);
      store_w3<5>(Wl, wp[1], wv, kk);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {  // rounds 3 and 4: s = 0 over slots 6-7, s = 4 over slot 7 and beyond
      float2* const b = Wl + (6 + r) * kSlot3;
#pragma unroll
      for (int q = 0; q < 4; ++q) b[(wv + 16 * q) * F + kk] = keep[q][2 + r];
      lds_barrier();
      fft2_lk<1024>(b, tw, t);
      float2 wp[4];
      if (r == 0) split3<WARM, 0>(b, b, wv, kk, Rx, Ry, wp, ck, cl, h);
      else split3<WARM, 4>(b, b, wv, kk, Rx, Ry, wp, ck, cl, h);
      lds_barrier();
      if (r == 0) store_w3<0>(Wl, wp, wv, kk);
      else store_w3<4>(Wl, wp, wv, kk);
    }
    // the slots into s order (slot s holds W[., ., s]): the six that move
    // form one cycle; each thread reads its entries of all six, then writes
    // them to their places
    {
      constexpr uint32_t kFrom = 0x764310u;   // the six moving slots, 4 bits each
      constexpr uint32_t kOrder = 0x40536271u;  // s held by each slot before the move, 4 bits per slot
      constexpr int kTail = kSlot3 - 2 * NT;    // 64 entries per slot past 2 NT
      static_assert(kTail > 0 && 6 * kTail <= NT, "slot tails fit one pass");
      float2 mv[6][2], mt = make_float2(0.f, 0.f);
      const int ti = (t / kTail) % 6;           // the slot whose tail entry t % kTail this thread moves
      const int tfrom = (int)((kFrom >> (4 * ti)) & 15u);
      lds_barrier();
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int r = 0; r < 2; ++r) mv[i][r] = Wl[(int)((kFrom >> (4 * i)) & 15u) * kSlot3 + t + r * NT];
      if (t < 6 * kTail) mt = Wl[tfrom * kSlot3 + 2 * NT + t % kTail];
      lds_barrier();
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const int to = (int)((kOrder >> (4 * ((kFrom >> (4 * i)) & 15u))) & 7u);
#pragma unroll
        for (int r = 0; r < 2; ++r) Wl[to * kSlot3 + t + r * NT] = mv[i][r];
      }
      if (t < 6 * kTail) Wl[(int)((kOrder >> (4 * tfrom)) & 7u) * kSlot3 + 2 * NT + t % kTail] = mt;
    }
    __syncthreads();
    const float W0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Wl[0].x)));
    if (!(W0 > 0.f)) {
      if (t == 0) a.status[vi] = FSE_BLOCK_EMPTY_SUPPORT;
      __syncthreads();  // LDS is overwritten by the next volume
      continue;
    }
    const float gW = a.gamma * (1.0f / W0);
    const unsigned char* const Wb = reinterpret_cast<const unsigned char*>(Wl);
    bool finite = true;
    if constexpr (!WARM) {
      // per-thread first maximum of |R_w|^2 (bits) and where it is
      uint32_t best = 0;
      int bj = 0;
#pragma unroll
      for (int j = 0; j < BPT; ++j) {
        const uint32_t b2 = __float_as_uint(fmaf(Ry[j], Ry[j], Rx[j] * Rx[j]));
        if (bits_max_first(b2, best)) bj = j;
      }
      // 3. iterations (eqs. (12), (13), (18))
      for (int it = 0; it < I; ++it) {
        // the thread's candidate, then the wave's (first lane: lowest k), then
        // the workgroup's (largest value, lowest bin index among equals)
        const uint32_t wm = wave_max_bits(best);
        const unsigned long long hits = __ballot(best == wm);
        const int wl = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(hits));
        const int jw = __builtin_amdgcn_readlane(bj, wl);  // uniform: one indexed register read
        const int widx = wl * (F * FT) + wv * BPT + jw;
        const float wre = readlane_f(Rx[jw], wl), wim = readlane_f(Ry[jw], wl);
        xch[parity * (NT / 64) + wv] = make_int4((int)wm, widx, __float_as_int(wre), __float_as_int(wim));  // uniform
        __syncthreads();
        int4 sv = make_int4(0, 0x7fffffff, 0, 0);
        if (kk < NT / 64) sv = xch[parity * (NT / 64) + kk];
        parity ^= 1;
        unsigned hi = (unsigned)sv.x, lo = ~(unsigned)sv.y;
        dpp_max64<kQuadXor1>(hi, lo);
        dpp_max64<kQuadXor2>(hi, lo);
        dpp_max64<kRowHalfMirror>(hi, lo);
        dpp_max64<kRowMirror>(hi, lo);  // lanes 0-15: the maximum over the 16 slots
        const uint32_t gm = (uint32_t)__builtin_amdgcn_readlane((int)hi, 0);
        const int gidx = (int)~(unsigned)__builtin_amdgcn_readlane((int)lo, 0);
        const int ws = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(__ballot(kk < NT / 64 && sv.y == gidx)));
        const float gre = __int_as_float(__builtin_amdgcn_readlane(sv.z, ws));
        const float gim = __int_as_float(__builtin_amdgcn_readlane(sv.w, ws));
        const int s0 = gidx & (FT - 1), v0 = (gidx >> 3) & (F - 1), u0 = gidx >> 9;
        const float cre = gW * gre, cim = gW * gim;  // eq. (13)
        finite = finite && isfinite(cre) && isfinite(cim);
        if (wv == 0) {
          cl_idx[it] = gidx;  // uniform stores
          cl_c[it] = make_float2(cre, cim);
          if (a.trace) {
            fse_trace_t rec;
            rec.u = (uint16_t)u0;
            rec.v = (uint16_t)(v0 * FT + s0);
            rec.c_re = cre;
            rec.c_im = cim;
            rec.r2 = __uint_as_float(gm);
            a.trace[(int64_t)vi * a.trace_stride + it] = rec;
          }
        }
        // eq. (18): R_w[k,l,s] -= c W[k-u, l-v, s-s0]. The row l' = (l - v)
        // mod 64 is uniform per column; for l' > 32 the stored value is
        // W[u-k, v-l, s0-s] and its conjugate is used, which swaps the sign of
        // two of the four products. The s-slot offsets are uniform.
        const int kq = ((kk - u0) & (F - 1)) * 8, kqf = ((u0 - kk) & (F - 1)) * 8;  // byte offsets
        const unsigned creb = __float_as_uint(cre), cimb = __float_as_uint(cim);
        best = 0;
        bj = 0;
#pragma unroll
        for (int cc = 0; cc < BPT / FT; ++cc) {
          const int lp = ((BPT / FT) * wv + cc - v0) & (F - 1);
          const bool flip = lp > F / 2;
          const int lrow = flip ? (F - lp) & (F - 1) : lp;
          const int base = (flip ? kqf : kq) + lrow * (F * 8);
          const float A = __uint_as_float(flip ? cimb ^ 0x80000000u : cimb);
          const float Bc = __uint_as_float(flip ? creb : creb ^ 0x80000000u);
          // the column's eight W values first, so that their loads overlap
          float2 wc[FT];
#pragma unroll
          for (int s3 = 0; s3 < FT; ++s3) {
            const int srot = (flip ? s0 - s3 : s3 - s0) & (FT - 1);
            wc[s3] = *reinterpret_cast<const float2*>(Wb + base + srot * (kSlot3 * 8));
          }
          // keeps the eight loads ahead of the arithmetic (the scheduler would
          // otherwise wait for each load before issuing the next)
          asm volatile("" : "+v"(wc[0].x), "+v"(wc[0].y), "+v"(wc[1].x), "+v"(wc[1].y), "+v"(wc[2].x), "+v"(wc[2].y),
                       "+v"(wc[3].x), "+v"(wc[3].y), "+v"(wc[4].x), "+v"(wc[4].y), "+v"(wc[5].x), "+v"(wc[5].y),
                       "+v"(wc[6].x), "+v"(wc[6].y), "+v"(wc[7].x), "+v"(wc[7].y));
#pragma unroll
          for (int s3 = 0; s3 < FT; ++s3) {
            const int j = cc * FT + s3;
            const float2 w = wc[s3];
            float rx = Rx[j], ry = Ry[j];
            rx = fmaf(-cre, w.x, rx);
            rx = fmaf(A, w.y, rx);
            ry = fmaf(Bc, w.y, ry);
            ry = fmaf(-cim, w.x, ry);
            Rx[j] = rx;
            Ry[j] = ry;
            if (bits_max_first(__float_as_uint(fmaf(ry, ry, rx * rx)), best)) bj = j;
          }
        }
      }
    } else if (wv < 4) {
      // warm start: four candidate bins per lane of waves 0-3
      uint32_t best = 0;
      int bj = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (bits_max_first(__float_as_uint(fmaf(Ry[j], Ry[j], Rx[j] * Rx[j])), best)) bj = j;
      for (int it = 0; it < I; ++it) {
        const uint32_t wm = wave_max_bits(best);
        const int wl = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(__ballot(best == wm)));
        const int jw = __builtin_amdgcn_readlane(bj, wl);
        const int widx = __builtin_amdgcn_readlane(c2, wl) * FT + 4 * h + jw;
        const float wre = readlane_f(Rx[jw], wl), wim = readlane_f(Ry[jw], wl);
        if (kk == 0) xch[parity * 4 + wv] = make_int4((int)wm, widx, __float_as_int(wre), __float_as_int(wim));
        __syncthreads();
        int4 sv = make_int4(0, 0x7fffffff, 0, 0);
        if (kk < 4) sv = xch[parity * 4 + kk];
        parity ^= 1;
        unsigned hi = (unsigned)sv.x, lo = ~(unsigned)sv.y;
        dpp_max64<kQuadXor1>(hi, lo);
        dpp_max64<kQuadXor2>(hi, lo);  // lanes 0-3: the maximum over the 4 slots
        const uint32_t gm = (uint32_t)__builtin_amdgcn_readlane((int)hi, 0);
        const int gidx = (int)~(unsigned)__builtin_amdgcn_readlane((int)lo, 0);
        const int ws = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(__ballot(kk < 4 && sv.y == gidx)));
        const float gre = __int_as_float(__builtin_amdgcn_readlane(sv.z, ws));
        const float gim = __int_as_float(__builtin_amdgcn_readlane(sv.w, ws));
        const int s0 = gidx & (FT - 1), v0 = (gidx >> 3) & (F - 1), u0 = gidx >> 9;
        const float cre = gW * gre, cim = gW * gim;  // eq. (13)
        finite = finite && isfinite(cre) && isfinite(cim);
        if (wv == 0 && kk == 0) {  // one lane
          cl_idx[it] = gidx;
          cl_c[it] = make_float2(cre, cim);
          if (a.trace) {
            fse_trace_t rec;
            rec.u = (uint16_t)u0;
            rec.v = (uint16_t)(v0 * FT + s0);
            rec.c_re = cre;
            rec.c_im = cim;
            rec.r2 = __uint_as_float(gm);
            a.trace[(int64_t)vi * a.trace_stride + it] = rec;
          }
        }
        // eq. (18) at the candidates: W[k-u, l-v, s-s0], from the mirrored
        // entry conjugated when (l - v) mod 64 > 32. The lane's column fixes
        // the row and k offset; the s-slot offsets of both cases are uniform
        // and the lane's case picks one with a mask.
        const int lp = (cl - v0) & (F - 1);
        const bool flip = lp > F / 2;
        const int row = flip ? (F - lp) & (F - 1) : lp;
        const int kx = (flip ? u0 - ck : ck - u0) & (F - 1);
        const int base = (row * F + kx) * 8;
        const int fm = flip ? -1 : 0;
        const float A = flip ? -cim : cim, Bc = flip ? cre : -cre;
        best = 0;
        bj = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int sj = 4 * h + j;
          const int on = ((sj - s0) & (FT - 1)) * (kSlot3 * 8);
          const int of = ((s0 - sj) & (FT - 1)) * (kSlot3 * 8);
          const float2 w = *reinterpret_cast<const float2*>(Wb + base + on + ((of - on) & fm));
          float rx = Rx[j], ry = Ry[j];
          rx = fmaf(-cre, w.x, rx);
          rx = fmaf(A, w.y, rx);
          ry = fmaf(Bc, w.y, ry);
          ry = fmaf(-cim, w.x, ry);
          Rx[j] = rx;
          Ry[j] = ry;
          if (bits_max_first(__float_as_uint(fmaf(ry, ry, rx * rx)), best)) bj = j;
        }
      }
    } else {
      for (int it = 0; it < I; ++it) __syncthreads();  // one barrier per iteration of waves 0-3
    }
    // the coefficient list is complete; every coefficient must be finite
    if (__syncthreads_or(!finite)) {
      if (t == 0) a.status[vi] = FSE_BLOCK_NONFINITE;
      __syncthreads();
      continue;
    }
    // 4. model on B (Algorithm 1, last loop, in 3-D): Re{sum c e^{j theta}}
    const int np = bh * bw * bt;
    for (int p = t; p < np; p += NT) {
      const int tt = p / (bh * bw), rem = p % (bh * bw), i = rem / bw, jj = rem % bw;
      const uint32_t m = (uint32_t)(bd + i), n = (uint32_t)(bd + jj), q = (uint32_t)(td + tt);
      float acc = 0.f;
      for (int it = 0; it < I; ++it) {
        const int gidx = __builtin_amdgcn_readfirstlane(cl_idx[it]);
        const uint32_t s3 = gidx & (FT - 1), v = (gidx >> 3) & (F - 1), u = gidx >> 9;
        const float2 c = cl_c[it];
        const float2 e = tw[(u * m + v * n + (F / FT) * s3 * q) & (F - 1)];  // exp(-j theta)
        acc = fmaf(c.x, e.x, acc);
        acc = fmaf(c.y, e.y, acc);
      }
      a.out[((int64_t)(f0 + tt) * a.H + y0 + i) * a.out_pitch + x0 + jj] = acc;
    }
    if (t == 0) a.status[vi] = FSE_BLOCK_OK;
    __syncthreads();  // LDS is overwritten by the next volume
  }
}

// ------------------------------------------------------------ rFSE
// Real-valued FSE (the model of eq. (2): a basis function and its conjugate
// per iteration) for F = 64, one block per 256-thread workgroup at a time.
// R_w of real data is Hermitian, so only the bins with l <= 32 are kept:
// thread (wave w, lane k) owns (k, l = w + 4 c), c < 9 (wave 0 holds the
// ninth column, l = 32). A pair is represented by its bin with l in 1..31,
// or with l in {0, 32} and k <= 32. The pair's weighted least-squares fit
// needs Q = W[2k, 2l]: with D = W0^2 - |Q|^2, A = 2 W0 / D and Bq = 2 Q / D
// (self-conjugate bins: A = 1 / W0, Bq = 0), the energy decrease is
// A |P|^2 - Re{Bq* P^2} and the coefficient A P* - Bq* P, held as
// a1 x^2 + a2 y^2 + a3 x y and (a1 x + a3 y / 2, -a2 y - a3 x / 2) for
// P = x + j y. SEL picks the form:
//   kRealDecrease  the pair of largest decrease; the constants depend on the
//                  window only, so the divisions are done once per block;
//   kRealInloop    the same selection with the constants, divisions
//                  included, recomputed for every bin in every iteration
//                  (the formulation whose cost the paper's runtime
//                  comparison describes);
//   kRealPower     the other reading of the selection: the pair holding the
//                  largest |P|^2 (the criterion of eq. (12)); the constants
//                  serve the winner's coefficient only.
constexpr int kRealNT = 256;

template <int SEL>
__global__ __launch_bounds__(kRealNT) void fse_real64(ClassArgs a) {
  constexpr bool INLOOP = SEL == kRealInloop;
  constexpr int F = 64, NT = kRealNT, NC = 9;
  extern __shared__ __align__(16) unsigned char smem[];
  float2* const Wd = reinterpret_cast<float2*>(smem);          // FFT buffer, then W[l][k] for l <= 32
  float2* const tw = Wd + F * F;
  int4* const red = reinterpret_cast<int4*>(tw + F);           // 2 parities x 4 waves x 2 slots
  float2* const cl_c = reinterpret_cast<float2*>(red + 16);
  int* const cl_idx = reinterpret_cast<int*>(cl_c + a.iters_cap);
  const int t0 = threadIdx.x;
  if (t0 < F) tw[t0] = a.twid[t0];
  int parity = 0;
  for (int bi = blockIdx.x; bi < a.n; bi += gridDim.x) {
    int t = t0;
    asm volatile("" : "+v"(t));
    const int kk = t & (F - 1), wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const UBlock bd = uniform_block(a.blocks + bi);
    const int orig = __builtin_amdgcn_readfirstlane(a.orig[bi]);
    const int bh = bd.bh, bw = bd.bw, bo = bd.border;
    const int M = bh + 2 * bo, N = bw + 2 * bo;
    const int ya = bd.y0 - bo, xa = bd.x0 - bo;
    const int I = bd.iters;
    const int64_t fofs = (int64_t)bd.frame * a.H;
    const uint8_t* img = a.img + fofs * a.pitch;
    const uint8_t* av = a.avail + fofs * a.pitch;
    const int pitch = (int)a.pitch;

    // 1. gather and weight (eq. (3)), z = s w + j alpha w, forward transform
    for (int r = 0; r < F * F / NT; ++r) {
      const int e = t + r * NT;
      const int m = e / F, n = e % F;
      const int y = ya + m, x = xa + n;
      const bool inB = m >= bo && m < bo + bh && n >= bo && n < bo + bw;
      float2 z = make_float2(0.f, 0.f);
      if (m < M && n < N && !inB && y >= 0 && y < a.H && x >= 0 && x < a.W) {
        const uint32_t p = (uint32_t)(y * pitch + x);
        if (av[p] != 0) {
          const int da = min(abs(2 * m - (M - 1)), kWinStride - 1), db = min(abs(2 * n - (N - 1)), kWinStride - 1);
          const float w = a.wtab[da * kWinStride + db];
          z = make_float2((float)img[p] * w, kAlpha * w);
        }
      }
      Wd[e] = z;
    }
    lds_barrier();
    fft_lines<F, NT, false>(Wd, tw, t);
    fft_lines<F, NT, true>(Wd, tw, t);

    // 2. split into R_w (registers) and W (LDS, [l][k] for l <= 32)
    float Rx[NC], Ry[NC];
    float2 Wv[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const int l = wv + 4 * cc;
      Rx[cc] = Ry[cc] = 0.f;
      Wv[cc] = make_float2(0.f, 0.f);
      if (l <= F / 2) {
        const float2 zk = Wd[kk * F + l];
        const float2 zn = Wd[((F - kk) & (F - 1)) * F + ((F - l) & (F - 1))];
        Rx[cc] = (zk.x + zn.x) * 0.5f;
        Ry[cc] = (zk.y - zn.y) * 0.5f;
        Wv[cc] = make_float2((zk.y + zn.y) * (0.5f / kAlpha), (zn.x - zk.x) * (0.5f / kAlpha));
      }
    }
    const float W0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Wd[0].y))) * (1.0f / kAlpha);
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const int l = wv + 4 * cc;
      if (l <= F / 2) Wd[l * F + kk] = Wv[cc];
    }
    __syncthreads();
    if (!(W0 > 0.f)) {
      if (t == 0) a.status[orig] = FSE_BLOCK_EMPTY_SUPPORT;
      continue;  // the next block's gather starts after the barrier above
    }

    // 3. per-bin constants of the pair fit
    float a1[NC], a2[NC], a3[NC];
    auto constants = [&](int cc) {
      const int l = wv + 4 * cc;
      a1[cc] = a2[cc] = a3[cc] = 0.f;
      if (l <= F / 2) {
        const int lq = (2 * l) & (F - 1);  // 0 or 2l <= 62: rows above 32 are read conjugated
        const bool fq = lq > F / 2;
        float2 q = Wd[(fq ? F - lq : lq) * F + ((fq ? -2 * kk : 2 * kk) & (F - 1))];
        q.y = fq ? -q.y : q.y;
        const bool sc = (kk == 0 || kk == F / 2) && (l == 0 || l == F / 2);
        const bool rep = (l != 0 && l != F / 2) || kk <= F / 2;
        const float D = fmaf(W0, W0, -fmaf(q.x, q.x, q.y * q.y));
        const float iD = 2.0f / D;
        const float A = sc ? 1.0f / W0 : W0 * iD;
        const float Br = sc ? 0.f : q.x * iD, Bi = sc ? 0.f : q.y * iD;
        a1[cc] = rep ? A - Br : 0.f;
        a2[cc] = rep ? A + Br : 0.f;
        a3[cc] = rep ? -2.0f * Bi : 0.f;
      }
    };
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) constants(cc);
    // 1 for the bins that represent a pair, 0 for the others
    float rp[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) rp[cc] = a1[cc] > 0.f ? 1.f : 0.f;
    auto decrease = [&](int cc) {
      const float x = Rx[cc], y = Ry[cc];
      if constexpr (SEL != kRealPower) {
        const float tq = fmaf(a3[cc], y, a1[cc] * x);
        const float d = fmaf(x, tq, (a2[cc] * y) * y);
        return __float_as_uint(fmaxf(d, 0.f));
      } else {
        return __float_as_uint(rp[cc] * fmaf(y, y, x * x));
      }
    };
    uint32_t best = 0;
    int bj = 0;
#pragma unroll
    for (int cc = 0; cc < NC; ++cc)
      if (bits_max_first(decrease(cc), best)) bj = cc;

    bool finite = true;
    const float hg = 0.5f * a.gamma;
    // 4. iterations
    for (int it = 0; it < I; ++it) {
      const uint32_t wm = wave_max_bits(best);
      const int wl = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(__ballot(best == wm)));
      const int jw = __builtin_amdgcn_readlane(bj, wl);
      const int bin = wl * F + wv + 4 * jw;
      red[(parity * 4 + wv) * 2] = make_int4((int)wm, bin, __float_as_int(readlane_f(Rx[jw], wl)),
                                             __float_as_int(readlane_f(Ry[jw], wl)));
      red[(parity * 4 + wv) * 2 + 1] = make_int4(__float_as_int(readlane_f(a1[jw], wl)),
                                                 __float_as_int(readlane_f(a2[jw], wl)),
                                                 __float_as_int(readlane_f(a3[jw], wl)), 0);
      __syncthreads();
      int4 s0 = make_int4(0, 0, 0, 0), s1 = make_int4(0, 0, 0, 0);
      if (kk < 4) {
        s0 = red[(parity * 4 + kk) * 2];
        s1 = red[(parity * 4 + kk) * 2 + 1];
      }
      parity ^= 1;
      uint32_t gm = __builtin_amdgcn_readlane(s0.x, 0);
      int ws = 0;
#pragma unroll
      for (int w2 = 1; w2 < 4; ++w2) {
        const uint32_t m2 = __builtin_amdgcn_readlane(s0.x, w2);
        ws = m2 > gm ? w2 : ws;  // the first wave wins ties
        gm = m2 > gm ? m2 : gm;
      }
      const int gbin = __builtin_amdgcn_readlane(s0.y, ws);
      const float x = __int_as_float(__builtin_amdgcn_readlane(s0.z, ws));
      const float y = __int_as_float(__builtin_amdgcn_readlane(s0.w, ws));
      const float g1 = __int_as_float(__builtin_amdgcn_readlane(s1.x, ws));
      const float g2 = __int_as_float(__builtin_amdgcn_readlane(s1.y, ws));
      const float h = 0.5f * __int_as_float(__builtin_amdgcn_readlane(s1.z, ws));
      // the pair's coefficient A P* - Bq* P, then the compensation gamma
      const float cre = fmaf(g1, x, h * y), cim = -fmaf(g2, y, h * x);
      const int u = gbin >> 6, v = gbin & (F - 1);
      finite = finite && isfinite(cre) && isfinite(cim);
      if (wv == 0) {
        cl_idx[it] = gbin;  // uniform stores; the model is Re{c phi*} = Re{conj(c) phi}
        cl_c[it] = make_float2(a.gamma * cre, -a.gamma * cim);
        if (a.trace) {
          // recorded for the pair's lower-index bin (the conjugate bin has the conjugate coefficient)
          const bool upper = u > F / 2;
          fse_trace_t rec;
          rec.u = (uint16_t)(upper ? F - u : u);
          rec.v = (uint16_t)(upper ? (F - v) & (F - 1) : v);
          rec.c_re = a.gamma * cre;
          rec.c_im = upper ? -a.gamma * cim : a.gamma * cim;
          rec.r2 = __uint_as_float(gm);
          a.trace[(int64_t)orig * a.trace_stride + it] = rec;
        }
      }
      // R_w[k,l] -= (gamma / 2) (c W[k+u, l+v] + c* W[k-u, l-v]); rows above
      // 32 are read as the conjugate of the mirrored entry
      // uniform factors on the scalar unit: sign flips are integer xors
      const uint32_t pb = __builtin_amdgcn_readfirstlane(__float_as_uint(hg * cre));
      const uint32_t qb = __builtin_amdgcn_readfirstlane(__float_as_uint(hg * cim));
      constexpr uint32_t kSign = 0x80000000u;
      int o1 = ((kk + u) & (F - 1)) * 8, o1f = ((-kk - u) & (F - 1)) * 8;
      int o2 = ((kk - u) & (F - 1)) * 8, o2f = ((u - kk) & (F - 1)) * 8;
      asm volatile("" : "+v"(o1), "+v"(o1f), "+v"(o2), "+v"(o2f));  // computed once, not per bin
      const unsigned char* Wb = reinterpret_cast<const unsigned char*>(Wd);
      best = 0;
      bj = 0;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const int l = wv + 4 * cc;
        if (cc == NC - 1 && wv != 0) continue;  // wave-uniform: only wave 0 holds l = 32
        const int l1 = (l + v) & (F - 1), l2 = (l - v) & (F - 1);
        const bool f1 = l1 > F / 2, f2 = l2 > F / 2;
        const float2 w1 = *reinterpret_cast<const float2*>(Wb + (f1 ? o1f : o1) + (f1 ? F - l1 : l1) * (F * 8));
        const float2 w2 = *reinterpret_cast<const float2*>(Wb + (f2 ? o2f : o2) + (f2 ? F - l2 : l2) * (F * 8));
        const uint32_t s1 = f1 ? kSign : 0u, s2 = f2 ? kSign : 0u;
        const float mp = __uint_as_float(pb ^ kSign), mq = __uint_as_float(qb ^ kSign), qq = __uint_as_float(qb);
        float rx = Rx[cc], ry = Ry[cc];
        rx = fmaf(mp, w1.x, rx);
        rx = fmaf(__uint_as_float(qb ^ s1), w1.y, rx);          // f1 ? -q : q
        ry = fmaf(__uint_as_float(pb ^ s1 ^ kSign), w1.y, ry);  // f1 ? p : -p
        ry = fmaf(mq, w1.x, ry);
        rx = fmaf(mp, w2.x, rx);
        rx = fmaf(__uint_as_float(qb ^ s2 ^ kSign), w2.y, rx);  // f2 ? q : -q
        ry = fmaf(__uint_as_float(pb ^ s2 ^ kSign), w2.y, ry);  // f2 ? p : -p
        ry = fmaf(qq, w2.x, ry);
        Rx[cc] = rx;
        Ry[cc] = ry;
        if constexpr (INLOOP) constants(cc);
        if (bits_max_first(decrease(cc), best)) bj = cc;
      }
    }
    __syncthreads();  // the coefficient list is complete
    if (!finite) {
      if (t == 0) a.status[orig] = FSE_BLOCK_NONFINITE;
      continue;
    }
    synthesize<F, NT, 1>(cl_idx, cl_c, I, tw, bh, bw, bo, a.out + (fofs + bd.y0) * a.out_pitch + bd.x0,
                         a.out_pitch, t);
    if (t == 0) a.status[orig] = FSE_BLOCK_OK;
    __syncthreads();  // Wd and the list are overwritten by the next block
  }
}

// ------------------------------------------------------------ fixed point
// cFSE in integer arithmetic (F = 64): every value is an integer with a
// fixed scale and every sum is exact in int64, so the result is one
// deterministic function of the input, reproducible bit for bit:
//   z = s wq + j 2^7 wq (wq = window, scale 2^15; twiddles T scale 2^14)
//   Y[m,l] = round(sum_n z[m,n] T[l n] / 2^14),  Z[k,l] = round(sum_m Y[m,l] T[k m] / 2^23)
//   R2 = Z + conj(Z[-k,-l]) (2^7 R_w),  W2 = -j (Z - conj(Z[-k,-l])) (2^14 W)
//   G = floor(gamma_q 2^33 / W2[0,0]): the only division, once per block
//   iterations: argmax R2x^2 + R2y^2 (exact, lowest index on ties),
//   c = round(R2[u,v] G / 2^26), R2 -= round(c W2[k-u, l-v] / 2^23)
//   model on B: round(sum Re{c conj(T[u m + v n])} / 2^22) / 2^8
// round(x / 2^s) is (x + 2^(s-1)) >> s. The transform is computed as two
// direct passes (an FFT would round between its stages).
constexpr int kFixedNT = 256;

__device__ __forceinline__ int32_t rshift_lo(int64_t x, int s) {
  // round(x / 2^s) when the result fits 32 bits
  return (int32_t)((x + ((int64_t)1 << (s - 1))) >> s);
}

__global__ __launch_bounds__(kFixedNT) void fse_fixed64(ClassArgs a) {
  constexpr int F = 64, NT = kFixedNT, NW = NT / 64, BPL = F * F / NT;  // 16 bins per lane
  extern __shared__ __align__(16) unsigned char smem[];
  int2* const zb = reinterpret_cast<int2*>(smem);    // z, then Z            [64][64]
  int2* const yb = zb + F * F;                        // Y [m][l], then W2    [64][64]
  int2* const tq = yb + F * F;                        // twiddles
  int4* const red = reinterpret_cast<int4*>(tq + F);  // 2 parities x NW x 2 slots
  int2* const cl_c = reinterpret_cast<int2*>(red + 4 * NW);
  int* const cl_idx = reinterpret_cast<int*>(cl_c + a.iters_cap);
  const int t0 = threadIdx.x;
  if (t0 < F) tq[t0] = a.twid_q[t0];
  int parity = 0;
  for (int bi = blockIdx.x; bi < a.n; bi += gridDim.x) {
    int t = t0;
    asm volatile("" : "+v"(t));
    const int lane = t & (F - 1), wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const UBlock bd = uniform_block(a.blocks + bi);
    const int orig = __builtin_amdgcn_readfirstlane(a.orig[bi]);
    const int bh = bd.bh, bw = bd.bw, bo = bd.border;
    const int M = bh + 2 * bo, N = bw + 2 * bo;
    const int ya = bd.y0 - bo, xa = bd.x0 - bo;
    const int I = bd.iters;
    const int64_t fofs = (int64_t)bd.frame * a.H;
    const uint8_t* img = a.img + fofs * a.pitch;
    const uint8_t* av = a.avail + fofs * a.pitch;
    const int pitch = (int)a.pitch;

    // 1. z on the area (rows and columns beyond M, N are never read)
    for (int e = t; e < F * F; e += NT) {
      const int m = e / F, n = e % F;
      const int y = ya + m, x = xa + n;
      const bool inB = m >= bo && m < bo + bh && n >= bo && n < bo + bw;
      int2 z = make_int2(0, 0);
      if (m < M && n < N && !inB && y >= 0 && y < a.H && x >= 0 && x < a.W) {
        const uint32_t p = (uint32_t)(y * pitch + x);
        if (av[p] != 0) {
          const int da = min(abs(2 * m - (M - 1)), kWinStride - 1), db = min(abs(2 * n - (N - 1)), kWinStride - 1);
          const int w = a.wtab_q[da * kWinStride + db];
          z = make_int2((int)img[p] * w, w << 7);
        }
      }
      zb[e] = z;
    }
    __syncthreads();
    // 2. row pass: lane l, rows m = wave, wave + NW, ...
    {
      const int l = lane;
      for (int m = wave; m < M; m += NW) {
        int64_t ar = 0, ai = 0;
        for (int n = 0; n < N; ++n) {
          const int2 z = zb[m * F + n];        // broadcast
          const int2 tw = tq[(l * n) & (F - 1)];
          ar += (int64_t)z.x * tw.x - (int64_t)z.y * tw.y;
          ai += (int64_t)z.x * tw.y + (int64_t)z.y * tw.x;
        }
        yb[m * F + l] = make_int2(rshift_lo(ar, 14), rshift_lo(ai, 14));
      }
    }
    __syncthreads();
    // 3. column pass: lane l, frequencies k = wave, wave + NW, ...; Z into zb
    {
      const int l = lane;
      for (int k = wave; k < F; k += NW) {
        int64_t ar = 0, ai = 0;
        for (int m = 0; m < M; ++m) {
          const int2 y = yb[m * F + l];
          const int2 tw = tq[(k * m) & (F - 1)];  // uniform
          ar += (int64_t)y.x * tw.x - (int64_t)y.y * tw.y;
          ai += (int64_t)y.x * tw.y + (int64_t)y.y * tw.x;
        }
        zb[k * F + l] = make_int2(rshift_lo(ar, 23), rshift_lo(ai, 23));
      }
    }
    __syncthreads();
    // 4. split: R2 into registers (bin wave*1024 + j*64 + lane), W2 into yb
    int Rx[BPL], Ry[BPL];
#pragma unroll
    for (int j = 0; j < BPL; ++j) {
      const int k = wave * BPL + j, l = lane;
      const int2 zk = zb[k * F + l];
      const int2 zn = zb[((F - k) & (F - 1)) * F + ((F - l) & (F - 1))];
      Rx[j] = zk.x + zn.x;
      Ry[j] = zk.y - zn.y;
      yb[k * F + l] = make_int2(zk.y + zn.y, zn.x - zk.x);
    }
    __syncthreads();
    const int W0 = __builtin_amdgcn_readfirstlane(yb[0].x);
    if (W0 <= 0) {
      if (t == 0) a.status[orig] = FSE_BLOCK_EMPTY_SUPPORT;
      __syncthreads();
      continue;
    }
    const int64_t G = ((int64_t)a.gamma_q << 33) / W0;
    // per-thread first maximum of the exact score
    uint64_t best = 0;
    int bj = 0;
#pragma unroll
    for (int j = 0; j < BPL; ++j) {
      const uint64_t sc = (uint64_t)((int64_t)Rx[j] * Rx[j] + (int64_t)Ry[j] * Ry[j]);
      bj = sc > best ? j : bj;
      best = sc > best ? sc : best;
    }
    for (int it = 0; it < I; ++it) {
      // wave: largest score (high word, then low word), then the lowest bin
      const uint32_t bh32 = (uint32_t)(best >> 32), bl32 = (uint32_t)best;
      const uint32_t mh = wave_max_bits(bh32);
      const uint32_t ml = wave_max_bits(bh32 == mh ? bl32 : 0u);
      const bool top = bh32 == mh && bl32 == ml;
      const uint32_t key = wave_min_u32(top ? (uint32_t)(bj * 64 + lane) : 0xffffffffu);
      const int wl = (int)(key & 63), jw = (int)(key >> 6);
      const int widx = wave * (BPL * 64) + (int)key;
      const int wrx = __builtin_amdgcn_readlane(Rx[jw], wl), wry = __builtin_amdgcn_readlane(Ry[jw], wl);
      red[(parity * NW + wave) * 2] = make_int4((int)mh, (int)ml, widx, 0);
      red[(parity * NW + wave) * 2 + 1] = make_int4(wrx, wry, 0, 0);
      __syncthreads();
      uint32_t gh = 0, gl = 0;
      int gidx = 0, gx = 0, gy = 0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) {
        const int4 v0 = red[(parity * NW + w2) * 2];
        const int4 v1 = red[(parity * NW + w2) * 2 + 1];
        const uint32_t h2 = (uint32_t)__builtin_amdgcn_readfirstlane(v0.x);
        const uint32_t l2 = (uint32_t)__builtin_amdgcn_readfirstlane(v0.y);
        const bool take = w2 == 0 || h2 > gh || (h2 == gh && l2 > gl);  // the first wave wins ties
        gh = take ? h2 : gh;
        gl = take ? l2 : gl;
        gidx = take ? __builtin_amdgcn_readfirstlane(v0.z) : gidx;
        gx = take ? __builtin_amdgcn_readfirstlane(v1.x) : gx;
        gy = take ? __builtin_amdgcn_readfirstlane(v1.y) : gy;
      }
      parity ^= 1;
      const int u = gidx >> 6, v = gidx & (F - 1);
      const int cr = (int)(((int64_t)gx * G + ((int64_t)1 << 25)) >> 26);  // eq. (13)
      const int ci = (int)(((int64_t)gy * G + ((int64_t)1 << 25)) >> 26);
      if (wave == 0) {
        cl_idx[it] = gidx;  // uniform stores
        cl_c[it] = make_int2(cr, ci);
        if (a.trace) {
          fse_trace_t rec;
          rec.u = (uint16_t)u;
          rec.v = (uint16_t)v;
          rec.c_re = (float)cr * (1.0f / 65536.0f);
          rec.c_im = (float)ci * (1.0f / 65536.0f);
          rec.r2 = (float)(((uint64_t)gh << 32) | gl);
          a.trace[(int64_t)orig * a.trace_stride + it] = rec;
        }
      }
      // eq. (18): R2[k,l] -= round(c W2[k-u, l-v] / 2^23); the row k - u is
      // uniform per register, the column per lane
      int col = ((lane - v) & (F - 1)) * 8;
      asm volatile("" : "+v"(col));
      const unsigned char* Wb = reinterpret_cast<const unsigned char*>(yb);
      constexpr int64_t kHalf = (int64_t)1 << 22;
      best = 0;
      bj = 0;
#pragma unroll
      for (int j = 0; j < BPL; ++j) {
        const int row = ((wave * BPL + j - u) & (F - 1)) * (F * 8);
        const int2 w = *reinterpret_cast<const int2*>(Wb + row + col);
        const int64_t dx = (int64_t)cr * w.x - (int64_t)ci * w.y + kHalf;
        const int64_t dy = (int64_t)cr * w.y + (int64_t)ci * w.x + kHalf;
        const int rx = Rx[j] - (int)(dx >> 23), ry = Ry[j] - (int)(dy >> 23);
        Rx[j] = rx;
        Ry[j] = ry;
        const uint64_t sc = (uint64_t)((int64_t)rx * rx + (int64_t)ry * ry);
        bj = sc > best ? j : bj;
        best = sc > best ? sc : best;
      }
    }
    __syncthreads();  // the coefficient list is complete
    // 5. model on B, exact int64 sums
    {
      const int np = bh * bw;
      float* ob = a.out + (fofs + bd.y0) * a.out_pitch + bd.x0;
      for (int p = t; p < np; p += NT) {
        const int m = bo + p / bw, n = bo + p % bw;
        int64_t acc = 0;
        for (int it = 0; it < I; ++it) {
          const int gidx = __builtin_amdgcn_readfirstlane(cl_idx[it]);
          const int2 c = cl_c[it];
          const int2 tw = tq[((gidx >> 6) * m + (gidx & (F - 1)) * n) & (F - 1)];
          acc += (int64_t)c.x * tw.x + (int64_t)c.y * tw.y;
        }
        ob[(int64_t)(p / bw) * a.out_pitch + p % bw] = (float)rshift_lo(acc, 22) * (1.0f / 256.0f);
      }
    }
    if (t == 0) a.status[orig] = FSE_BLOCK_OK;
    __syncthreads();  // the buffers and the list are overwritten by the next block
  }
}
}  // namespace

const Variant* variant_for(int F) {
  for (const Variant& v : kVariants)
    if (v.F == F && v.kc == 0 && v.mode == kPlain) return &v;
  return nullptr;
}

const Variant* power_variant_for(int F) {
  for (const Variant& v : kVariants)
    if (v.F == F && v.mode == kPower) return &v;
  return nullptr;
}

const Variant* warm_variant_for(int F, int kc, int mode) {
  for (const Variant& v : kVariants)
    if (v.F == F && v.kc == kc && kc > 0 && v.mode == mode) return &v;
  return nullptr;
}

int variants_for(int F, const Variant** out, int cap) {
  int n = 0;
  for (const Variant& v : kVariants)
    if (v.F == F && v.kc == 0 && v.mode == kPlain) {
      if (n < cap) out[n] = &v;
      ++n;
    }
  return n;
}

// Waves per block of the restricted kernel: one up to 256 candidates (the
// per-iteration reductions would dominate two waves of two candidates per
// lane), two above.
constexpr int restricted_waves(int kc) { return kc <= 256 ? 1 : 2; }

const void* restricted_kernel(int kc) {
  switch (kc) {
    case 128: return reinterpret_cast<const void*>(&fse_restricted<128, restricted_waves(128)>);
    case 256: return reinterpret_cast<const void*>(&fse_restricted<256, restricted_waves(256)>);
    case 384: return reinterpret_cast<const void*>(&fse_restricted<384, restricted_waves(384)>);
    case 512: return reinterpret_cast<const void*>(&fse_restricted<512, restricted_waves(512)>);
    default: return nullptr;
  }
}

int restricted_threads(int kc) { return 64 * restricted_waves(kc); }

size_t restricted_lds_bytes(int kc, int ir, bool lists) {
  return (restricted_waves(kc) == 2 ? 4 * 16 : 0) + (lists ? (size_t)ir * 12 : 0);
}

hipError_t launch_restricted(int kc, const ClassArgs& a, size_t lds, hipStream_t s) {
  const void* fn = restricted_kernel(kc);
  if (!fn || a.n <= 0) return hipErrorInvalidValue;
  void* args[] = {const_cast<ClassArgs*>(&a)};
  return hipLaunchKernel(fn, dim3(a.n), dim3(restricted_threads(kc)), args, lds, s);
}

// Staging of the allocation-free warm start (fse_warm_extrapolate_batch_noalloc).
// In host code `scratch` names a host-side stand-in: only the address from
// hipGetSymbolAddress may reach a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  addr.emplace(device, p);
  *out = p;
  return hipSuccess;
}

size_t lds_bytes(const Variant& v, int iters_cap) {
  const size_t F = (size_t)v.F;
  const size_t nw = (size_t)v.threads / 64;
  const size_t rpw = F / nw;
  const size_t rpg = (F == 64 && rpw > 8) ? 8 : rpw;  // rows per group, as Shape<F, NT>::RPG
  const size_t rows = F + rpg - 1;
  const size_t cap = (size_t)iters_cap;
  const size_t kc = v.mode == kWarmFused ? (size_t)v.kc : 0;  // as KCL in the kernel
  return rows * F * 8 + F * 8 + 2 * nw * 16 + (cap + kc) * 8 + (cap + kc) * 4 + 16;
}

hipError_t launch_class(const Variant& v, const ClassArgs& a, int grid, size_t lds, hipStream_t s) {
  void* args[] = {const_cast<ClassArgs*>(&a)};
  return hipLaunchKernel(v.fn, dim3(grid), dim3(v.threads), args, lds, s);
}

}  // namespace fse

namespace fse {
size_t lds_bytes3d(int iters_cap) {
  // the last round's FFT buffer (from slot 7 on) or W and the coefficient list
  return std::max((size_t)kW3Ofs + (size_t)(7 * kSlot3 + kFftBuf3) * 8,
                  (size_t)kW3Ofs + kW3Bytes + (size_t)iters_cap * 12);
}

const void* fse3d_kernel(bool warm) {
  return warm ? reinterpret_cast<const void*>(&fse3d<true>) : reinterpret_cast<const void*>(&fse3d<false>);
}

size_t real_lds_bytes(int iters_cap) { return (size_t)64 * 64 * 8 + 64 * 8 + 16 * 16 + (size_t)iters_cap * 12; }

const void* real_kernel(int sel) {
  switch (sel) {
    case kRealInloop: return reinterpret_cast<const void*>(&fse_real64<kRealInloop>);
    case kRealPower: return reinterpret_cast<const void*>(&fse_real64<kRealPower>);
    default: return reinterpret_cast<const void*>(&fse_real64<kRealDecrease>);
  }
}

int real_threads() { return kRealNT; }

size_t fixed_lds_bytes(int iters_cap) {
  return (size_t)2 * 64 * 64 * 8 + 64 * 8 + 4 * (kFixedNT / 64) * 16 + (size_t)iters_cap * 12;
}

const void* fixed_kernel() { return reinterpret_cast<const void*>(&fse_fixed64); }

int fixed_threads() { return kFixedNT; }

hipError_t launch_fixed(const ClassArgs& a, int grid, size_t lds, hipStream_t s) {
  void* args[] = {const_cast<ClassArgs*>(&a)};
  return hipLaunchKernel(reinterpret_cast<const void*>(&fse_fixed64), dim3(grid), dim3(kFixedNT), args, lds, s);
}

hipError_t launch_real(const ClassArgs& a, int sel, int grid, size_t lds, hipStream_t s) {
  void* args[] = {const_cast<ClassArgs*>(&a)};
  return hipLaunchKernel(real_kernel(sel), dim3(grid), dim3(kRealNT), args, lds, s);
}

hipError_t launch_fse3d(const Vol3Args& a, bool warm, int grid, size_t lds, hipStream_t s) {
  void* args[] = {const_cast<Vol3Args*>(&a)};
  return hipLaunchKernel(fse3d_kernel(warm), dim3(grid), dim3(kNT3), args, lds, s);
}
}  // namespace fse
