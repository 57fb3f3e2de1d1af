// Internal interface between the host API (fse_api.cpp) and the device code
// (fse_kernels.hip). Not installed; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fse.h"

namespace fse {

// Window table: wtab[a * kWinStride + b] = rho^(sqrt(a*a + b*b) / 2) for
// a = |2m - (M-1)|, b = |2n - (N-1)|, i.e. rho^distance-to-area-centre
// (eq. (3)) indexed by doubled integer offsets; a, b < kWinStride.
constexpr int kWinStride = 128;
constexpr int kMaxIters = 4096;

// Arguments of one launch over the blocks of a single transform size.
struct ClassArgs {
  const uint8_t* img;      // [n_frames][H][pitch]
  const uint8_t* avail;    // [n_frames][H][pitch]
  int64_t pitch;
  float* out;              // [n_frames][H][out_pitch]
  int64_t out_pitch;
  int32_t H, W;
  const fse_block_t* blocks;  // this class's blocks, longest first
  const int32_t* orig;        // index of each block in the caller's list
  int32_t n;                  // number of blocks in the class
  int32_t iters_cap;          // largest iteration count in the class
  int32_t* status;            // [caller's n_blocks]
  fse_trace_t* trace;         // null or [caller's n_blocks][trace_stride]
  int32_t trace_stride;
  const float* wtab;          // window table (see kWinStride)
  const float2* twid;         // F entries: exp(-j 2 pi q / F)
  float gamma;
  int32_t masked_b;           // nonzero: B = the lost pixels of each block's rectangle
  int32_t* queue;             // [2]: next block, finished workgroups
  // warm-started form only
  const int16_t* cand;        // [caller's n_blocks][kc] candidate bins, ascending
  const int32_t* flags;       // [caller's n_blocks]: nonzero = run plain FSE
  int32_t ir;                 // restricted iterations
  float gamma_r;              // step of the restricted iterations (gamma of eq. (13) there)
  int32_t fb_iters;           // full iterations of a block that falls back
  // split warm-started form: staging written by the transform kernel and
  // read by the restricted kernel, indexed by the block's position in this
  // launch's list (blocks[0 .. n))
  float2* stage_w;            // [n][kHalfRows * 64]: W rows 0..32
  float2* stage_r;            // [n][kc]: R_w at the candidates
  float* power;               // kPower mode: [caller's n_blocks][F * F] |R_w|^2 of the first transform
  // fixed-point form only (plan flag FSE_PLAN_FIXED)
  const int32_t* wtab_q;      // round(2^15 rho^(sqrt(a^2 + b^2) / 2)), [kWinStride][kWinStride]
  const int2* twid_q;         // round(2^14 exp(-j 2 pi q / 64)), 64 entries
  int32_t gamma_q;            // round(2^16 gamma)
};

// Rows of W kept by the split warm start for F = 64: W[k, l] for k <= 32;
// the others follow from W[-k, -l] = conj(W[k, l]) (w is real).
constexpr int kHalfRows = 33;

// Three dimensions: one workgroup of kNT3 threads per volume, F x F x Ft
// transform with F = 64, Ft = 8.
constexpr int kF3 = 64, kFt3 = 8, kNT3 = 1024;
constexpr int kHalfCols3 = kF3 / 2 + 1;  // W kept for l <= 32
// 3-D window table: wtab3[(c * kWinStride + a) * kWinStride + b] =
// rho^(sqrt(a*a + b*b + c*c) / 2) for doubled integer offsets a, b, c.
constexpr int kWinStrideT = 16;

struct Vol3Args {
  const uint8_t* img;    // [n_frames][H][pitch]
  const uint8_t* avail;  // [n_frames][H][pitch]
  int64_t pitch;
  float* out;            // [n_frames][H][out_pitch]
  int64_t out_pitch;
  int32_t n_frames, H, W;
  const fse_volume_t* vols;
  int32_t n;
  int32_t iters_cap;
  int32_t* status;
  fse_trace_t* trace;    // null or [n][trace_stride]
  int32_t trace_stride;
  const float* wtab3;
  const float2* twid;    // 64 entries exp(-j 2 pi q / 64)
  float gamma;
  // warm start only: candidate columns k * 64 + l per volume (ascending)
  // and the network's per-volume flags (nonzero: no usable candidates)
  const int16_t* cand2;  // [n][kCand3]
  const int32_t* flags;  // [n]
};

// Warm-started 3-D: candidate columns per volume; with all kFt3 values of s
// they give one candidate bin per thread.
constexpr int kCand3 = kNT3 / kFt3;

size_t lds_bytes3d(int iters_cap);
hipError_t launch_fse3d(const Vol3Args& a, bool warm, int grid, size_t lds, hipStream_t s);
const void* fse3d_kernel(bool warm);

// rFSE (real-valued model), F = 64: LDS bytes for a given iteration cap,
// the kernel (for the occupancy API), its workgroup size, and its launch;
// inloop selects the form that recomputes the pair constants in every
// iteration.
size_t real_lds_bytes(int iters_cap);
// rFSE forms: selection by the least-squares decrease (constants per block
// or per iteration) or by |R_w|^2.
enum RealSel : int { kRealDecrease = 0, kRealInloop = 1, kRealPower = 2 };
const void* real_kernel(int sel);
int real_threads();
hipError_t launch_real(const ClassArgs& a, int sel, int grid, size_t lds, hipStream_t s);

// Fixed-point cFSE, F = 64: the same four helpers.
size_t fixed_lds_bytes(int iters_cap);
const void* fixed_kernel();
int fixed_threads();
hipError_t launch_fixed(const ClassArgs& a, int grid, size_t lds, hipStream_t s);

// Kernel modes.
// kPower: transform only, |R_w|^2 of every bin written out (candidate sets
// taken from the initial spectrum).
enum Mode : int { kPlain = 0, kWarmFused = 1, kWarmPrep = 2, kPower = 3 };

// One compiled kernel variant for transform size F.
struct Variant {
  int F;
  int threads;         // workgroup size
  int kc;              // candidates per block (warm-started form), 0 = plain
  int mode;            // Mode
  const void* fn;      // kernel symbol
};

// Default kernel variant for transform size F (32, 64, 128), or null.
const Variant* variant_for(int F);

// Warm-started variant for F with kc candidates per block in the given mode
// (kWarmFused or kWarmPrep), or null.
const Variant* warm_variant_for(int F, int kc, int mode);

// Transform-only variant writing |R_w|^2 (mode kPower), or null.
const Variant* power_variant_for(int F);

// Restricted kernel of the split warm start (F = 64, one workgroup per
// block of the class, grid = class size): null if kc is not compiled.
const void* restricted_kernel(int kc);

// Dynamic LDS bytes of the restricted kernel for kc candidates and ir
// restricted iterations (W and the twiddles are static: 17 KB); `lists` =
// room for the per-block coefficient list, needed only by blocks with more
// than kRestrictedInloopPixels pixels in B. Then its threads per workgroup.
size_t restricted_lds_bytes(int kc, int ir, bool lists);
constexpr int kRestrictedInloopPixels = 256;
int restricted_threads(int kc);

// All compiled plain variants for F; returns their number, fills up to cap.
int variants_for(int F, const Variant** out, int cap);

// Dynamic LDS bytes a variant needs for a class whose largest iteration
// count is iters_cap.
size_t lds_bytes(const Variant& v, int iters_cap);

// Record the message returned by fse_last_error() on this thread.
void set_error(const char* msg);

// Launch one class; grid = number of persistent workgroups.
hipError_t launch_class(const Variant& v, const ClassArgs& a, int grid, size_t lds, hipStream_t s);

// Launch the restricted kernel over the n blocks of a class.
hipError_t launch_restricted(int kc, const ClassArgs& a, size_t lds, hipStream_t s);

// Device memory of the allocation-free warm start: a file-scope array of
// kScratchBytes on every device the library runs on, held until the
// process ends. scratch_address returns its address on `device` (which must
// be current), looked up on the first call per device and kept.
constexpr size_t kScratchBytes = (size_t)48 << 20;
hipError_t scratch_address(int device, void** out);

}  // namespace fse
