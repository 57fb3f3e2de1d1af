// Host side of the C ABI declared in include/fse.h: parameter checks, the
// FP64 window and twiddle tables, block validation and scheduling, device
// memory of a batch, and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "cnn_internal.h"
#include "fse.h"
#include "fse_internal.h"

namespace {

thread_local const char* g_error = "no error";

fse_status_t fail(fse_status_t code, const char* msg) {
  g_error = msg;
  return code;
}

}  // namespace

void fse::set_error(const char* msg) { g_error = msg; }

namespace {

constexpr int kSizes[3] = {128, 64, 32};  // class order: longest blocks first

int real_sel(uint32_t flags) {
  return (flags & FSE_PLAN_REAL_INLOOP) ? fse::kRealInloop : (flags & FSE_PLAN_REAL_POWER) ? fse::kRealPower
                                                                                        : fse::kRealDecrease;
}

int class_of(int F) {
  for (int c = 0; c < 3; ++c)
    if (kSizes[c] == F) return c;
  return -1;
}

struct DeviceTables {
  float* wtab = nullptr;          // kWinStride^2 floats
  float2* twid[3] = {nullptr, nullptr, nullptr};
};

// Candidate counts the warm start's staging is sized for: the largest
// compiled one, so that a later change of kc never reallocates it.
constexpr int kStageKcMax = 512;

// Byte offsets of a batch's device arrays inside one buffer (a caller's
// workspace), each 256-byte aligned.
struct WsLayout {
  size_t blocks = 0, orig = 0, queue = 0, wtab = 0, twid[3] = {0, 0, 0};
  size_t wtab_q = 0, twid_q = 0, stage_r = 0, stage_w = 0, total = 0;
};

}  // namespace

struct fse_plan_s {
  float rho = 0.f, gamma = 0.f;
  int32_t max_iters = 0;
  uint32_t flags = 0;
  std::vector<float> wtab;                 // host copy, FP64-computed
  std::vector<float2> twid[3];             // per class
  std::mutex mu;
  std::map<int, DeviceTables> dev;         // uploaded tables per device
};

struct fse_batch_s {
  fse_plan_t plan = nullptr;
  int device = 0, cus = 0;
  int32_t n = 0, n_frames = 0, H = 0, W = 0;
  int32_t max_iters = 0;
  fse_block_t* d_blocks = nullptr;
  int32_t* d_orig = nullptr;
  int32_t* d_queue = nullptr;              // 3 classes x 32 ints (own cache lines)
  const DeviceTables* tables = nullptr;
  struct Cls {
    const fse::Variant* v = nullptr;
    int32_t offset = 0, count = 0, iters_cap = 0;
    int32_t grid = 0, wg_per_cu = 0;
    size_t lds = 0;
  } cls[3];
  Cls warm;                                // warm-started launch of the F = 64 class
  int32_t warm_kc = 0, warm_ir = -1, warm_fb = -1;
  float warm_gamma = -1.f;                 // step of the restricted iterations; < 0: the plan's gamma
  bool warm_split = false;                 // transform kernel + restricted kernel
  size_t restricted_lds = 0;
  float2* d_stage_w = nullptr;             // split form's staging (caller's block order)
  float2* d_stage_r = nullptr;
  int32_t stage_kc = 0;
  // kernel timing hook: event pairs and what each recorded launch was
  std::vector<hipEvent_t> t_ev;
  std::vector<int32_t> t_kind, t_fft;
  int32_t t_count = 0;
  bool all_48 = false;                     // every area is 48 x 48 (network input size)
  bool all_small_b = false;                // every B has at most 256 pixels (restricted kernel
                                           // synthesises in its loop, no coefficient list)
  int32_t alt_grid = 0;                    // rFSE or fixed-point launch (FSE_PLAN_REAL, FSE_PLAN_FIXED)
  size_t alt_lds = 0;
  int32_t* d_wtab_q = nullptr;             // fixed point: integer window table
  int2* d_twid_q = nullptr;                // fixed point: integer twiddles
  bool in_workspace = false;               // device arrays lie in a caller's workspace (never freed here)
  DeviceTables ws_tables;                  // the plan tables' copy in that workspace
};

extern "C" const char* fse_last_error(void) { return g_error; }

extern "C" fse_status_t fse_plan_create(const fse_plan_desc_t* desc, fse_plan_t* out_plan) {
  if (!desc || !out_plan) return fail(FSE_ERR_INVALID_ARG, "null argument");
  *out_plan = nullptr;
  if (!(desc->rho > 0.f && desc->rho <= 1.f)) return fail(FSE_ERR_INVALID_ARG, "rho must lie in (0, 1]");
  if (!(desc->gamma >= 0.f && desc->gamma <= 1.f)) return fail(FSE_ERR_INVALID_ARG, "gamma must lie in [0, 1]");
  if (desc->max_iters < 0 || desc->max_iters > fse::kMaxIters)
    return fail(FSE_ERR_INVALID_ARG, "max_iters must lie in [0, 4096]");
  if ((desc->flags & ~(uint32_t)(FSE_PLAN_MASKED_B | FSE_PLAN_REAL | FSE_PLAN_FIXED | FSE_PLAN_REAL_INLOOP |
                                  FSE_PLAN_REAL_POWER)) != 0)
    return fail(FSE_ERR_INVALID_ARG, "unknown plan flag");
  if ((desc->flags & (FSE_PLAN_REAL_INLOOP | FSE_PLAN_REAL_POWER)) && !(desc->flags & FSE_PLAN_REAL))
    return fail(FSE_ERR_INVALID_ARG, "FSE_PLAN_REAL_INLOOP and FSE_PLAN_REAL_POWER modify FSE_PLAN_REAL");
  if ((desc->flags & FSE_PLAN_REAL_INLOOP) && (desc->flags & FSE_PLAN_REAL_POWER))
    return fail(FSE_ERR_INVALID_ARG, "FSE_PLAN_REAL_INLOOP and FSE_PLAN_REAL_POWER exclude each other");
  if (__builtin_popcount(desc->flags & ~(uint32_t)(FSE_PLAN_REAL_INLOOP | FSE_PLAN_REAL_POWER)) > 1)
    return fail(FSE_ERR_UNSUPPORTED, "FSE_PLAN_MASKED_B, FSE_PLAN_REAL and FSE_PLAN_FIXED exclude each other");
  fse_plan_s* p = new (std::nothrow) fse_plan_s;
  if (!p) return fail(FSE_ERR_OOM, "host allocation failed");
  p->rho = desc->rho;
  p->gamma = desc->gamma;
  p->max_iters = desc->max_iters;
  p->flags = desc->flags;
  // eq. (3): rho^distance, distance = sqrt(a^2 + b^2) / 2 for doubled offsets
  const int S = fse::kWinStride;
  p->wtab.resize((size_t)S * S);
  const double rho = (double)desc->rho;
  for (int a = 0; a < S; ++a)
    for (int b = 0; b < S; ++b)
      p->wtab[(size_t)a * S + b] = (float)std::pow(rho, 0.5 * std::sqrt((double)a * a + (double)b * b));
  for (int c = 0; c < 3; ++c) {
    const int F = kSizes[c];
    p->twid[c].resize(F);
    for (int q = 0; q < F; ++q) {
      const double ang = -2.0 * M_PI * (double)q / (double)F;
      p->twid[c][q] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    // exact values at the quarter points keep real-input symmetry exact
    p->twid[c][0] = make_float2(1.f, 0.f);
    p->twid[c][F / 4] = make_float2(0.f, -1.f);
    p->twid[c][F / 2] = make_float2(-1.f, 0.f);
    p->twid[c][3 * F / 4] = make_float2(0.f, 1.f);
  }
  *out_plan = p;
  return FSE_OK;
}

extern "C" void fse_plan_destroy(fse_plan_t plan) {
  if (!plan) return;
  if (!plan->dev.empty()) {  // a plan that never reached a GPU makes no HIP call
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    for (auto& kv : plan->dev) {
      if (hipSetDevice(kv.first) != hipSuccess) continue;
      (void)hipFree(kv.second.wtab);
      for (auto* t : kv.second.twid) (void)hipFree(t);
    }
    if (have) (void)hipSetDevice(cur);
  }
  delete plan;
}

extern "C" fse_status_t fse_validate_blocks(fse_plan_t plan, const fse_block_t* h_blocks, int32_t n_blocks,
                                            int32_t n_frames, int32_t H, int32_t W, int32_t* bad_index) {
  if (bad_index) *bad_index = -1;
  if (!plan) return fail(FSE_ERR_INVALID_ARG, "null plan");
  if (n_blocks < 0 || (n_blocks > 0 && !h_blocks)) return fail(FSE_ERR_INVALID_ARG, "bad block list");
  if (n_frames <= 0 || H <= 0 || W <= 0) return fail(FSE_ERR_INVALID_ARG, "frame dimensions must be positive");
  for (int32_t i = 0; i < n_blocks; ++i) {
    const fse_block_t& b = h_blocks[i];
    if (bad_index) *bad_index = i;
    if (class_of(b.fft) < 0) return fail(FSE_ERR_UNSUPPORTED, "fft must be 32, 64 or 128");
    if (b.bh < 1 || b.bw < 1 || b.border < 0) return fail(FSE_ERR_INVALID_ARG, "block size must be >= 1, border >= 0");
    if (b.bh + 2 * b.border > b.fft || b.bw + 2 * b.border > b.fft)
      return fail(FSE_ERR_UNSUPPORTED, "area larger than the transform");
    if (b.iters < 0 || b.iters > plan->max_iters) return fail(FSE_ERR_INVALID_ARG, "iters outside [0, max_iters]");
    if (b.frame < 0 || b.frame >= n_frames) return fail(FSE_ERR_INVALID_ARG, "frame index out of range");
    if (b.y0 < 0 || b.x0 < 0 || (int64_t)b.y0 + b.bh > H || (int64_t)b.x0 + b.bw > W)
      return fail(FSE_ERR_INVALID_ARG, "lost block outside the frame");
  }
  // overlap of loss areas: one bit per pixel
  const size_t npix = (size_t)n_frames * H * W;
  std::vector<uint64_t> bits((npix + 63) / 64, 0);
  for (int32_t i = 0; i < n_blocks; ++i) {
    const fse_block_t& b = h_blocks[i];
    for (int y = b.y0; y < b.y0 + b.bh; ++y) {
      for (int x = b.x0; x < b.x0 + b.bw; ++x) {
        const size_t p = ((size_t)b.frame * H + y) * W + x;
        const uint64_t m = 1ull << (p & 63);
        if (bits[p >> 6] & m) {
          if (bad_index) *bad_index = i;
          return fail(FSE_ERR_OVERLAP, "loss areas of two blocks overlap");
        }
        bits[p >> 6] |= m;
      }
    }
  }
  if (bad_index) *bad_index = -1;
  return FSE_OK;
}

extern "C" fse_status_t fse_blocks_from_mask(const uint8_t* h_avail, int32_t n_frames, int32_t H, int32_t W,
                                             int64_t pitch, int32_t cell, int32_t border, int32_t fft,
                                             int32_t iters, fse_block_t* h_out, int32_t cap, int32_t* n_out) {
  if (!h_avail || !n_out || (cap > 0 && !h_out)) return fail(FSE_ERR_INVALID_ARG, "null argument");
  *n_out = 0;
  if (n_frames <= 0 || H <= 0 || W <= 0 || pitch < W || cell < 1 || border < 0 || cap < 0 || iters < 0)
    return fail(FSE_ERR_INVALID_ARG, "bad mask or tile size");
  if (class_of(fft) < 0) return fail(FSE_ERR_UNSUPPORTED, "fft must be 32, 64 or 128");
  if (cell + 2 * border > fft) return fail(FSE_ERR_UNSUPPORTED, "area larger than the transform");
  int64_t count = 0;
  for (int32_t f = 0; f < n_frames; ++f)
    for (int32_t y0 = 0; y0 < H; y0 += cell)
      for (int32_t x0 = 0; x0 < W; x0 += cell) {
        const int32_t bh = std::min(cell, H - y0), bw = std::min(cell, W - x0);
        bool lost = false;
        for (int32_t y = y0; y < y0 + bh && !lost; ++y) {
          const uint8_t* row = h_avail + ((int64_t)f * H + y) * pitch + x0;
          for (int32_t x = 0; x < bw; ++x)
            if (row[x] == 0) {
              lost = true;
              break;
            }
        }
        if (!lost) continue;
        if (count < cap) {
          fse_block_t& b = h_out[count];
          b.frame = f;
          b.y0 = y0;
          b.x0 = x0;
          b.bh = (int16_t)bh;
          b.bw = (int16_t)bw;
          b.border = (int16_t)border;
          b.fft = (int16_t)fft;
          b.iters = iters;
        }
        if (++count > INT32_MAX) return fail(FSE_ERR_INVALID_ARG, "too many blocks");
      }
  *n_out = (int32_t)count;
  return FSE_OK;
}

namespace {

fse_status_t upload_tables(fse_plan_t plan, int device, const DeviceTables** out) {
  std::lock_guard<std::mutex> lock(plan->mu);
  auto it = plan->dev.find(device);
  if (it != plan->dev.end()) {
    *out = &it->second;
    return FSE_OK;
  }
  DeviceTables t;
  const size_t wbytes = plan->wtab.size() * sizeof(float);
  if (hipMalloc(&t.wtab, wbytes) != hipSuccess) return fail(FSE_ERR_OOM, "hipMalloc failed (window table)");
  if (hipMemcpy(t.wtab, plan->wtab.data(), wbytes, hipMemcpyHostToDevice) != hipSuccess)
    return fail(FSE_ERR_HIP, "hipMemcpy failed (window table)");
  for (int c = 0; c < 3; ++c) {
    const size_t b = plan->twid[c].size() * sizeof(float2);
    if (hipMalloc(&t.twid[c], b) != hipSuccess) return fail(FSE_ERR_OOM, "hipMalloc failed (twiddles)");
    if (hipMemcpy(t.twid[c], plan->twid[c].data(), b, hipMemcpyHostToDevice) != hipSuccess)
      return fail(FSE_ERR_HIP, "hipMemcpy failed (twiddles)");
  }
  auto res = plan->dev.emplace(device, t);
  *out = &res.first->second;
  return FSE_OK;
}

// Select variant v for class c: LDS size, resident workgroups per CU and
// the persistent grid (one wave of workgroups, never more than the blocks).
fse_status_t configure(fse_batch_s* b, fse_batch_s::Cls& c, const fse::Variant* v) {
  const size_t lds = fse::lds_bytes(*v, c.iters_cap);
  if (hipFuncSetAttribute(v->fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return fail(FSE_ERR_HIP, "hipFuncSetAttribute failed (LDS size)");
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, v->fn, v->threads, lds) != hipSuccess || per_cu < 1)
    return fail(FSE_ERR_UNSUPPORTED, "kernel does not fit on a compute unit (iteration count too large)");
  c.v = v;
  c.lds = lds;
  c.wg_per_cu = per_cu;
  c.grid = (int32_t)std::min<int64_t>(c.count, (int64_t)per_cu * b->cus);
  return FSE_OK;
}

void free_timing(fse_batch_s* b) {
  for (hipEvent_t e : b->t_ev) (void)hipEventDestroy(e);
  b->t_ev.clear();
  b->t_kind.clear();
  b->t_fft.clear();
  b->t_count = 0;
}

// Launch one kernel through `go`, bracketed by the timing events when the
// batch records timings and slots are left.
template <class Go>
hipError_t timed(fse_batch_s* b, int kind, int fft, hipStream_t s, Go go) {
  const int slot = b->t_count;
  const bool rec = slot < (int)b->t_kind.size();
  if (rec && hipEventRecord(b->t_ev[2 * slot], s) != hipSuccess) return hipErrorUnknown;
  const hipError_t e = go();
  if (rec && e == hipSuccess) {
    if (hipEventRecord(b->t_ev[2 * slot + 1], s) != hipSuccess) return hipErrorUnknown;
    b->t_kind[slot] = kind;
    b->t_fft[slot] = fft;
    b->t_count = slot + 1;
  }
  return e;
}

void free_batch(fse_batch_s* b) {
  free_timing(b);
  if (!b->in_workspace) {
    (void)hipFree(b->d_stage_w);
    (void)hipFree(b->d_stage_r);
    (void)hipFree(b->d_wtab_q);
    (void)hipFree(b->d_twid_q);
    (void)hipFree(b->d_blocks);
    (void)hipFree(b->d_orig);
    (void)hipFree(b->d_queue);
  }
  delete b;
}

bool valid_ws_flags(uint32_t ws_flags) { return (ws_flags & ~(uint32_t)FSE_WS_WARM) == 0; }

// A caller's workspace: non-null, 256-byte aligned, at least `need` bytes,
// and (checked last, the only device queries) device memory of the current
// device with the whole range inside one allocation.
fse_status_t check_workspace(void* d_workspace, size_t ws_bytes, size_t need) {
  if (!d_workspace) return fail(FSE_ERR_INVALID_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
    return fail(FSE_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < need) return fail(FSE_ERR_WORKSPACE, "workspace smaller than the size query's result");
  int dev = -1;
  hipPointerAttribute_t attr;
  hipDeviceptr_t base = nullptr;
  size_t extent = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FSE_ERR_HIP, "hipGetDevice failed");
  if (hipPointerGetAttributes(&attr, d_workspace) != hipSuccess || attr.type != hipMemoryTypeDevice ||
      attr.device != dev) {
    (void)hipGetLastError();
    return fail(FSE_ERR_INVALID_ARG, "workspace is not device memory of the current device");
  }
  if (hipMemGetAddressRange(&base, &extent, d_workspace) != hipSuccess ||
      static_cast<uint8_t*>(d_workspace) + need > static_cast<uint8_t*>(base) + extent) {
    (void)hipGetLastError();
    return fail(FSE_ERR_WORKSPACE, "workspace extends beyond its allocation");
  }
  return FSE_OK;
}

WsLayout ws_layout(fse_plan_t plan, int32_t n_blocks, uint32_t ws_flags) {
  WsLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const size_t n = (size_t)std::max(n_blocks, 0), nb = std::max<size_t>(n, 1);
  L.blocks = take(nb * sizeof(fse_block_t));
  L.orig = take(nb * sizeof(int32_t));
  L.queue = take(3 * 32 * sizeof(int32_t));
  L.wtab = take(plan->wtab.size() * sizeof(float));
  for (int c = 0; c < 3; ++c) L.twid[c] = take(plan->twid[c].size() * sizeof(float2));
  if (plan->flags & FSE_PLAN_FIXED) {
    L.wtab_q = take((size_t)fse::kWinStride * fse::kWinStride * sizeof(int32_t));
    L.twid_q = take(64 * sizeof(int2));
  }
  if (ws_flags & FSE_WS_WARM) {
    L.stage_r = take(n * kStageKcMax * sizeof(float2));
    L.stage_w = take(n * fse::kHalfRows * 64 * sizeof(float2));
  }
  L.total = off;
  return L;
}

// Batch creation; ws null: the library allocates the batch's device
// arrays, else they are carved from [ws, ws + ws_bytes) and the plan
// tables are copied there.
fse_status_t create_batch(fse_plan_t plan, const fse_block_t* h_blocks, int32_t n_blocks, int32_t n_frames,
                          int32_t H, int32_t W, uint8_t* ws, size_t ws_bytes, uint32_t ws_flags,
                          fse_batch_t* out_batch);

}  // namespace

extern "C" fse_status_t fse_batch_create(fse_plan_t plan, const fse_block_t* h_blocks, int32_t n_blocks,
                                         int32_t n_frames, int32_t H, int32_t W, fse_batch_t* out_batch) {
  return create_batch(plan, h_blocks, n_blocks, n_frames, H, W, nullptr, 0, 0, out_batch);
}

extern "C" fse_status_t fse_batch_workspace_size(fse_plan_t plan, int32_t n_blocks, uint32_t ws_flags,
                                                 size_t* bytes) {
  if (!plan || !bytes) return fail(FSE_ERR_INVALID_ARG, "null argument");
  *bytes = 0;
  if (n_blocks < 0) return fail(FSE_ERR_INVALID_ARG, "negative block count");
  if (!valid_ws_flags(ws_flags)) return fail(FSE_ERR_INVALID_ARG, "unknown workspace flag");
  if ((ws_flags & FSE_WS_WARM) && (plan->flags & (FSE_PLAN_MASKED_B | FSE_PLAN_REAL | FSE_PLAN_FIXED)))
    return fail(FSE_ERR_UNSUPPORTED, "the warm start needs a cFSE plan with rectangular loss areas");
  *bytes = ws_layout(plan, n_blocks, ws_flags).total;
  return FSE_OK;
}

extern "C" fse_status_t fse_batch_create_in(fse_plan_t plan, const fse_block_t* h_blocks, int32_t n_blocks,
                                            int32_t n_frames, int32_t H, int32_t W, void* d_workspace,
                                            size_t ws_bytes, uint32_t ws_flags, fse_batch_t* out_batch) {
  if (!out_batch) return fail(FSE_ERR_INVALID_ARG, "null argument");
  *out_batch = nullptr;
  size_t need = 0;
  fse_status_t st = fse_batch_workspace_size(plan, n_blocks, ws_flags, &need);
  if (st != FSE_OK) return st;
  st = check_workspace(d_workspace, ws_bytes, need);
  if (st != FSE_OK) return st;
  return create_batch(plan, h_blocks, n_blocks, n_frames, H, W, static_cast<uint8_t*>(d_workspace), ws_bytes,
                      ws_flags, out_batch);
}

namespace {
fse_status_t create_batch(fse_plan_t plan, const fse_block_t* h_blocks, int32_t n_blocks, int32_t n_frames,
                          int32_t H, int32_t W, uint8_t* ws, size_t ws_bytes, uint32_t ws_flags,
                          fse_batch_t* out_batch) {
  (void)ws_bytes;
  if (!out_batch) return fail(FSE_ERR_INVALID_ARG, "null argument");
  *out_batch = nullptr;
  fse_status_t st = fse_validate_blocks(plan, h_blocks, n_blocks, n_frames, H, W, nullptr);
  if (st != FSE_OK) return st;
  fse_batch_s* b = new (std::nothrow) fse_batch_s;
  if (!b) return fail(FSE_ERR_OOM, "host allocation failed");
  b->plan = plan;
  b->n = n_blocks;
  b->n_frames = n_frames;
  b->H = H;
  b->W = W;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return fail(FSE_ERR_HIP, "hipGetDevice failed");
  }
  // group by transform size (largest first), longest-running block first
  std::vector<int32_t> order(n_blocks);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const int cx = class_of(h_blocks[x].fft), cy = class_of(h_blocks[y].fft);
    if (cx != cy) return cx < cy;
    return h_blocks[x].iters > h_blocks[y].iters;
  });
  b->all_48 = true;
  b->all_small_b = true;
  for (int32_t i = 0; i < n_blocks; ++i) {
    const fse_block_t& hb = h_blocks[i];
    b->all_48 = b->all_48 && hb.bh + 2 * hb.border == 48 && hb.bw + 2 * hb.border == 48;
    b->all_small_b = b->all_small_b && (int)hb.bh * hb.bw <= fse::kRestrictedInloopPixels;
  }
  std::vector<fse_block_t> sorted(n_blocks);
  for (int32_t i = 0; i < n_blocks; ++i) {
    sorted[i] = h_blocks[order[i]];
    b->max_iters = std::max(b->max_iters, (int32_t)h_blocks[order[i]].iters);
    fse_batch_s::Cls& c = b->cls[class_of(sorted[i].fft)];
    if (c.count == 0) c.offset = i;
    c.count++;
    c.iters_cap = std::max(c.iters_cap, (int32_t)sorted[i].iters);
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
    delete b;
    return fail(FSE_ERR_HIP, "hipGetDeviceProperties failed");
  }
  b->cus = prop.multiProcessorCount;
  if (plan->flags & (FSE_PLAN_REAL | FSE_PLAN_FIXED)) {
    const bool real = plan->flags & FSE_PLAN_REAL;
    if (b->cls[class_of(64)].count != n_blocks) {
      delete b;
      return fail(FSE_ERR_UNSUPPORTED, real ? "rFSE is compiled for 64 x 64 transforms"
                                            : "fixed-point cFSE is compiled for 64 x 64 transforms");
    }
    const int cap = std::max(b->cls[class_of(64)].iters_cap, 1);
    const void* fn = real ? fse::real_kernel(real_sel(plan->flags)) : fse::fixed_kernel();
    b->alt_lds = real ? fse::real_lds_bytes(cap) : fse::fixed_lds_bytes(cap);
    int per_cu = 0;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->alt_lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, real ? fse::real_threads() : fse::fixed_threads(),
                                                     b->alt_lds) != hipSuccess ||
        per_cu < 1) {
      delete b;
      return fail(FSE_ERR_UNSUPPORTED, "kernel does not fit on a compute unit (iteration count too large)");
    }
    b->alt_grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(n_blocks, (int64_t)per_cu * b->cus));
  }
  for (int ci = 0; ci < 3; ++ci) {
    fse_batch_s::Cls& c = b->cls[ci];
    if (c.count == 0) continue;
    const fse::Variant* v = fse::variant_for(kSizes[ci]);
    st = v ? configure(b, c, v) : fail(FSE_ERR_UNSUPPORTED, "no kernel for this transform size");
    if (st != FSE_OK) {
      delete b;
      return st;
    }
  }
  const WsLayout L = ws_layout(plan, n_blocks, ws_flags);
  if (ws) {
    b->in_workspace = true;
    b->d_blocks = reinterpret_cast<fse_block_t*>(ws + L.blocks);
    b->d_orig = reinterpret_cast<int32_t*>(ws + L.orig);
    b->d_queue = reinterpret_cast<int32_t*>(ws + L.queue);
    b->ws_tables.wtab = reinterpret_cast<float*>(ws + L.wtab);
    for (int c = 0; c < 3; ++c) b->ws_tables.twid[c] = reinterpret_cast<float2*>(ws + L.twid[c]);
    b->tables = &b->ws_tables;
    if (plan->flags & FSE_PLAN_FIXED) {
      b->d_wtab_q = reinterpret_cast<int32_t*>(ws + L.wtab_q);
      b->d_twid_q = reinterpret_cast<int2*>(ws + L.twid_q);
    }
    if (ws_flags & FSE_WS_WARM) {
      b->d_stage_r = reinterpret_cast<float2*>(ws + L.stage_r);
      b->d_stage_w = reinterpret_cast<float2*>(ws + L.stage_w);
      b->stage_kc = kStageKcMax;
    }
    bool ok = hipMemcpy(b->ws_tables.wtab, plan->wtab.data(), plan->wtab.size() * sizeof(float),
                        hipMemcpyHostToDevice) == hipSuccess;
    for (int c = 0; c < 3 && ok; ++c)
      ok = hipMemcpy(b->ws_tables.twid[c], plan->twid[c].data(), plan->twid[c].size() * sizeof(float2),
                     hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
      free_batch(b);
      return fail(FSE_ERR_HIP, "upload of the plan tables failed");
    }
  } else {
    st = upload_tables(plan, b->device, &b->tables);
    if (st != FSE_OK) {
      delete b;
      return st;
    }
    const size_t nb = (size_t)std::max(n_blocks, 1);
    if (hipMalloc(&b->d_blocks, nb * sizeof(fse_block_t)) != hipSuccess ||
        hipMalloc(&b->d_orig, nb * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&b->d_queue, 3 * 32 * sizeof(int32_t)) != hipSuccess) {
      free_batch(b);
      return fail(FSE_ERR_OOM, "hipMalloc failed (batch)");
    }
  }
  if ((n_blocks > 0 &&
       (hipMemcpy(b->d_blocks, sorted.data(), n_blocks * sizeof(fse_block_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_orig, order.data(), n_blocks * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)) ||
      hipMemset(b->d_queue, 0, 3 * 32 * sizeof(int32_t)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    free_batch(b);
    return fail(FSE_ERR_HIP, "upload of the batch failed");
  }
  if (plan->flags & FSE_PLAN_FIXED) {
    // integer tables of the fixed-point encoding, FP64 on the host, rounded
    // once: window round(2^15 rho^(sqrt(a^2 + b^2) / 2)) for doubled
    // offsets, twiddles round(2^14 exp(-j 2 pi q / 64))
    const int S = fse::kWinStride;
    std::vector<int32_t> wq((size_t)S * S);
    for (int x = 0; x < S; ++x)
      for (int y = 0; y < S; ++y)
        wq[(size_t)x * S + y] = (int32_t)std::floor(
            std::pow((double)plan->rho, std::sqrt((double)x * x + (double)y * y) / 2.0) * 32768.0 + 0.5);
    std::vector<int2> tq(64);
    for (int q = 0; q < 64; ++q) {
      const double th = 2.0 * M_PI * q / 64.0;
      tq[q] = make_int2((int)std::floor(std::cos(th) * 16384.0 + 0.5), (int)std::floor(-std::sin(th) * 16384.0 + 0.5));
    }
    if (!ws && (hipMalloc(&b->d_wtab_q, wq.size() * sizeof(int32_t)) != hipSuccess ||
                hipMalloc(&b->d_twid_q, tq.size() * sizeof(int2)) != hipSuccess)) {
      free_batch(b);
      return fail(FSE_ERR_OOM, "hipMalloc failed (fixed-point tables)");
    }
    if (hipMemcpy(b->d_wtab_q, wq.data(), wq.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_twid_q, tq.data(), tq.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) {
      free_batch(b);
      return fail(FSE_ERR_HIP, "upload of the fixed-point tables failed");
    }
  }
  *out_batch = b;
  return FSE_OK;
}
}  // namespace

extern "C" void fse_batch_destroy(fse_batch_t batch) {
  if (!batch) return;
  (void)hipDeviceSynchronize();
  free_batch(batch);
}

extern "C" int32_t fse_batch_max_iters(fse_batch_t batch) { return batch ? batch->max_iters : 0; }

extern "C" fse_status_t fse_batch_launch_info(fse_batch_t batch, int32_t F, int32_t* threads, int32_t* wg_per_cu,
                                              int32_t* grid, int32_t* lds_bytes) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  const int ci = class_of(F);
  if (ci < 0 || batch->cls[ci].count == 0) return fail(FSE_ERR_INVALID_ARG, "no block of this transform size");
  if (batch->plan->flags & (FSE_PLAN_REAL | FSE_PLAN_FIXED)) {
    if (threads) *threads = (batch->plan->flags & FSE_PLAN_REAL) ? fse::real_threads() : fse::fixed_threads();
    if (wg_per_cu) *wg_per_cu = (batch->alt_grid + batch->cus - 1) / batch->cus;
    if (grid) *grid = batch->alt_grid;
    if (lds_bytes) *lds_bytes = (int32_t)batch->alt_lds;
    return FSE_OK;
  }
  const fse_batch_s::Cls& c = batch->cls[ci];
  if (threads) *threads = c.v->threads;
  if (wg_per_cu) *wg_per_cu = c.wg_per_cu;
  if (grid) *grid = c.grid;
  if (lds_bytes) *lds_bytes = (int32_t)c.lds;
  return FSE_OK;
}

// Warm-started launches run the blocks [start, start + count) of the warm
// class with the given staging (split form); count < 0 means all of them.
struct WarmRange {
  int32_t start = 0, count = -1;
  float2* stage_w = nullptr;
  float2* stage_r = nullptr;
};

static fse_status_t launch_one(fse_batch_t batch, int ci, const uint8_t* d_image, const uint8_t* d_avail,
                               int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                               fse_trace_t* d_trace, hipStream_t s, const int16_t* cand = nullptr,
                               const int32_t* flags = nullptr, const WarmRange& wr = WarmRange());

extern "C" fse_status_t fse_extrapolate_batch(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                              int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                              fse_trace_t* d_trace, void* stream) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  if (batch->n == 0) return FSE_OK;
  if (!d_image || !d_avail || !d_out || !d_status) return fail(FSE_ERR_INVALID_ARG, "null device pointer");
  if (pitch < batch->W || out_pitch < batch->W) return fail(FSE_ERR_INVALID_ARG, "pitch smaller than the width");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != batch->device)
    return fail(FSE_ERR_INVALID_ARG, "batch was created on another device");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int ci = 0; ci < 3; ++ci) {
    if (batch->cls[ci].count == 0) continue;
    fse_status_t st = launch_one(batch, ci, d_image, d_avail, pitch, d_out, out_pitch, d_status, d_trace, s);
    if (st != FSE_OK) return st;
  }
  return FSE_OK;
}

static fse_status_t launch_one(fse_batch_t batch, int ci, const uint8_t* d_image, const uint8_t* d_avail,
                               int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                               fse_trace_t* d_trace, hipStream_t s, const int16_t* cand, const int32_t* flags,
                               const WarmRange& wr) {
  // the kernels address a frame's pixels with 32-bit offsets
  if ((int64_t)batch->H * pitch >= ((int64_t)1 << 31))
    return fail(FSE_ERR_INVALID_ARG, "a frame (H x pitch bytes) must be smaller than 2 GiB");
  {
    const bool warm = cand != nullptr;
    const fse_batch_s::Cls& c = warm ? batch->warm : batch->cls[ci];
    fse::ClassArgs a;
    a.img = d_image;
    a.avail = d_avail;
    a.pitch = pitch;
    a.out = d_out;
    a.out_pitch = out_pitch;
    a.H = batch->H;
    a.W = batch->W;
    a.blocks = batch->d_blocks + c.offset;
    a.orig = batch->d_orig + c.offset;
    a.n = c.count;
    a.iters_cap = c.iters_cap;
    a.status = d_status;
    a.trace = d_trace;
    a.trace_stride = batch->max_iters;
    a.wtab = batch->tables->wtab;
    a.twid = batch->tables->twid[ci];
    a.gamma = batch->plan->gamma;
    a.masked_b = (batch->plan->flags & FSE_PLAN_MASKED_B) ? 1 : 0;
    a.queue = batch->d_queue + 32 * ci;
    a.cand = cand;
    a.flags = flags;
    a.ir = warm ? batch->warm_ir : 0;
    a.gamma_r = warm && batch->warm_gamma >= 0.f ? batch->warm_gamma : batch->plan->gamma;
    a.fb_iters = warm ? batch->warm_fb : 0;
    a.stage_w = nullptr;
    a.stage_r = nullptr;
    a.power = nullptr;
    a.wtab_q = nullptr;
    a.twid_q = nullptr;
    a.gamma_q = 0;
    int grid = c.grid;
    if (warm) {
      a.iters_cap = c.iters_cap;
      a.trace_stride = batch->warm_ir + std::max(batch->max_iters, batch->warm_fb);
      const int32_t count = wr.count < 0 ? c.count - wr.start : wr.count;
      if (wr.start < 0 || count < 0 || wr.start + count > c.count) return fail(FSE_ERR_INVALID_ARG, "bad block range");
      if (count == 0) return FSE_OK;
      a.blocks += wr.start;
      a.orig += wr.start;
      a.n = count;
      grid = (int32_t)std::min<int64_t>(count, (int64_t)c.wg_per_cu * batch->cus);
      if (batch->warm_split) {
        a.stage_w = wr.stage_w;
        a.stage_r = wr.stage_r;
        if (!a.stage_w || !a.stage_r) return fail(FSE_ERR_INVALID_ARG, "no staging for the split warm start");
      }
    }
    if (!warm && (batch->plan->flags & FSE_PLAN_REAL)) {
      if (timed(batch, FSE_KERNEL_REAL, 64, s, [&] {
            return fse::launch_real(a, real_sel(batch->plan->flags), batch->alt_grid, batch->alt_lds, s);
          }) !=
          hipSuccess)
        return fail(FSE_ERR_HIP, "kernel launch failed (rFSE)");
      return FSE_OK;
    }
    if (!warm && (batch->plan->flags & FSE_PLAN_FIXED)) {
      a.wtab_q = batch->d_wtab_q;
      a.twid_q = batch->d_twid_q;
      a.gamma_q = (int32_t)std::floor((double)batch->plan->gamma * 65536.0 + 0.5);
      if (timed(batch, FSE_KERNEL_FIXED, 64, s,
                [&] { return fse::launch_fixed(a, batch->alt_grid, batch->alt_lds, s); }) != hipSuccess)
        return fail(FSE_ERR_HIP, "kernel launch failed (fixed point)");
      return FSE_OK;
    }
    const int kind = !warm ? FSE_KERNEL_PLAIN : batch->warm_split ? FSE_KERNEL_WARM_PREP : FSE_KERNEL_WARM_FUSED;
    if (timed(batch, kind, c.v->F, s, [&] { return fse::launch_class(*c.v, a, grid, c.lds, s); }) != hipSuccess)
      return fail(FSE_ERR_HIP, "kernel launch failed");
    if (warm && batch->warm_split &&
        timed(batch, FSE_KERNEL_RESTRICTED, 64, s,
              [&] { return fse::launch_restricted(batch->warm_kc, a, batch->restricted_lds, s); }) != hipSuccess)
      return fail(FSE_ERR_HIP, "kernel launch failed (restricted iterations)");
  }
  return FSE_OK;
}

extern "C" fse_status_t fse_batch_set_timing(fse_batch_t batch, int32_t max_records) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  if (max_records < 0 || max_records > (1 << 20)) return fail(FSE_ERR_INVALID_ARG, "max_records must lie in [0, 2^20]");
  free_timing(batch);
  if (max_records == 0) return FSE_OK;
  batch->t_ev.assign(2 * (size_t)max_records, nullptr);
  for (hipEvent_t& e : batch->t_ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      free_timing(batch);
      return fail(FSE_ERR_HIP, "hipEventCreate failed");
    }
  batch->t_kind.assign(max_records, -1);
  batch->t_fft.assign(max_records, 0);
  return FSE_OK;
}

extern "C" int32_t fse_batch_kernel_times(fse_batch_t batch, float* ms, int32_t* kind, int32_t* fft, int32_t cap) {
  if (!batch || cap < 0) return fail(FSE_ERR_INVALID_ARG, "bad argument");
  const int32_t n = std::min(batch->t_count, cap);
  for (int32_t i = 0; i < n; ++i) {
    float t = 0.f;
    if (hipEventSynchronize(batch->t_ev[2 * i + 1]) != hipSuccess ||
        hipEventElapsedTime(&t, batch->t_ev[2 * i], batch->t_ev[2 * i + 1]) != hipSuccess)
      return fail(FSE_ERR_HIP, "hipEventElapsedTime failed");
    if (ms) ms[i] = t;
    if (kind) kind[i] = batch->t_kind[i];
    if (fft) fft[i] = batch->t_fft[i];
  }
  return batch->t_count;
}

extern "C" fse_status_t fse_batch_set_variant(fse_batch_t batch, int32_t F, int32_t threads) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  const int ci = class_of(F);
  if (ci < 0 || batch->cls[ci].count == 0) return fail(FSE_ERR_INVALID_ARG, "no block of this transform size");
  if (batch->plan->flags & (FSE_PLAN_REAL | FSE_PLAN_FIXED))
    return fail(FSE_ERR_UNSUPPORTED, "the rFSE and fixed-point kernels have one workgroup shape");
  const fse::Variant* vs[16];
  const int nv = std::min(fse::variants_for(F, vs, 16), 16);
  for (int i = 0; i < nv; ++i)
    if (vs[i]->threads == threads) return configure(batch, batch->cls[ci], vs[i]);
  return fail(FSE_ERR_UNSUPPORTED, "no compiled kernel with this workgroup shape");
}

namespace {

// Autotuner cache: one text line per decision, "key threads microseconds",
// the last line of a key winning. The key names the device (architecture
// and compute-unit count) and the class's shape: transform size, loss-area
// kind, and the block count and largest iteration count rounded up to
// powers of two.
int pow2_at_least(int64_t x) {
  int p = 0;
  while (p < 40 && ((int64_t)1 << p) < x) ++p;
  return p;
}

std::string tune_key(const hipDeviceProp_t& prop, const fse_batch_s* b, int ci) {
  std::string arch(prop.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  char buf[160];
  snprintf(buf, sizeof buf, "/%dcu/F%d/%s/n2^%d/i2^%d", prop.multiProcessorCount, kSizes[ci],
           (b->plan->flags & FSE_PLAN_MASKED_B) ? "masked" : "rect", pow2_at_least(b->cls[ci].count),
           pow2_at_least(b->cls[ci].iters_cap));
  return arch + buf;
}

int tune_lookup(const char* path, const std::string& key) {
  FILE* f = path ? std::fopen(path, "r") : nullptr;
  if (!f) return 0;
  int threads = 0;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char k[400];
    int t = 0;
    float us = 0.f;
    if (std::sscanf(line, "%399s %d %f", k, &t, &us) == 3 && key == k) threads = t;
  }
  std::fclose(f);
  return threads;
}

void tune_store(const char* path, const std::string& key, int threads, float us) {
  FILE* f = path ? std::fopen(path, "a") : nullptr;
  if (!f) return;
  std::fprintf(f, "%s %d %.3f\n", key.c_str(), threads, us);
  std::fclose(f);
}

}  // namespace

extern "C" fse_status_t fse_batch_autotune_cached(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                                  int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                                  int32_t reps, void* stream, char* report, size_t report_len,
                                                  const char* cache_path) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  if (reps < 1) return fail(FSE_ERR_INVALID_ARG, "reps must be >= 1");
  if (batch->plan->flags & (FSE_PLAN_REAL | FSE_PLAN_FIXED))
    return fail(FSE_ERR_UNSUPPORTED, "the rFSE and fixed-point kernels have one workgroup shape");
  if (report && report_len) report[0] = 0;
  size_t used = 0;
  hipDeviceProp_t prop;
  if (cache_path && hipGetDeviceProperties(&prop, batch->device) != hipSuccess)
    return fail(FSE_ERR_HIP, "hipGetDeviceProperties failed");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fse_status_t st = FSE_OK;
  for (int ci = 0; ci < 3 && st == FSE_OK; ++ci) {
    fse_batch_s::Cls& c = batch->cls[ci];
    if (c.count == 0) continue;
    const fse::Variant* vs[16];
    const int nv = std::min(fse::variants_for(kSizes[ci], vs, 16), 16);
    std::string key;
    if (cache_path) {
      // a cached decision for this device and class shape: no timing
      key = tune_key(prop, batch, ci);
      const int cached = tune_lookup(cache_path, key);
      bool hit = false;
      for (int i = 0; i < nv && cached > 0 && !hit; ++i)
        if (vs[i]->threads == cached && configure(batch, c, vs[i]) == FSE_OK) hit = true;
      if (hit) {
        if (report && used + 64 < report_len)
          used += (size_t)snprintf(report + used, report_len - used, "%d %d cached\n", kSizes[ci], cached);
        continue;
      }
    }
    if (!e0 && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
      st = fail(FSE_ERR_HIP, "hipEventCreate failed");
      break;
    }
    const fse::Variant* best = nullptr;
    float best_ms = 0.f;
    for (int i = 0; i < nv && st == FSE_OK; ++i) {
      if (configure(batch, c, vs[i]) != FSE_OK) continue;  // does not fit: skip
      st = launch_one(batch, ci, d_image, d_avail, pitch, d_out, out_pitch, d_status, nullptr, s);  // warm-up
      if (st != FSE_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) { st = fail(FSE_ERR_HIP, "hipEventRecord failed"); break; }
      for (int r = 0; r < reps && st == FSE_OK; ++r)
        st = launch_one(batch, ci, d_image, d_avail, pitch, d_out, out_pitch, d_status, nullptr, s);
      if (st != FSE_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(FSE_ERR_HIP, "event timing failed");
        break;
      }
      ms /= (float)reps;
      if (report && used + 64 < report_len)
        used += (size_t)snprintf(report + used, report_len - used, "%d %d %.3f\n", vs[i]->F, vs[i]->threads,
                                 1000.0 * ms);
      if (!best || ms < best_ms) {
        best = vs[i];
        best_ms = ms;
      }
    }
    if (st == FSE_OK) {
      if (!best) st = fail(FSE_ERR_UNSUPPORTED, "no variant fits");
      else st = configure(batch, c, best);
      if (st == FSE_OK && cache_path) tune_store(cache_path, key, best->threads, 1000.f * best_ms);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

extern "C" fse_status_t fse_batch_autotune(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                           int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                           int32_t reps, void* stream, char* report, size_t report_len) {
  return fse_batch_autotune_cached(batch, d_image, d_avail, pitch, d_out, out_pitch, d_status, reps, stream, report,
                                   report_len, nullptr);
}

extern "C" fse_status_t fse_cnn_patches(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                        int64_t pitch, uint16_t* d_x, void* stream) {
  if (!batch || !d_image || !d_avail || !d_x) return fail(FSE_ERR_INVALID_ARG, "null argument");
  if (!batch->all_48) return fail(FSE_ERR_UNSUPPORTED, "network inputs need 48x48 areas");
  if (batch->plan->flags & (FSE_PLAN_MASKED_B | FSE_PLAN_REAL | FSE_PLAN_FIXED))
    return fail(FSE_ERR_UNSUPPORTED, "the warm start needs a cFSE plan with rectangular loss areas");
  if (pitch < batch->W) return fail(FSE_ERR_INVALID_ARG, "pitch smaller than the width");
  if (fse::cnn::patches(d_image, d_avail, pitch, batch->H, batch->W, batch->d_blocks, batch->d_orig, batch->n, d_x,
                        reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(FSE_ERR_HIP, "kernel launch failed");
  return FSE_OK;
}

extern "C" fse_status_t fse_cnn_forward_blocks(fse_cnn_t net, fse_batch_t batch, const uint8_t* d_image,
                                               const uint8_t* d_avail, int64_t pitch, float* d_logits,
                                               void* stream) {
  if (!batch || !d_image || !d_avail) return fail(FSE_ERR_INVALID_ARG, "null argument");
  if (!batch->all_48) return fail(FSE_ERR_UNSUPPORTED, "network inputs need 48x48 areas");
  if (batch->plan->flags & (FSE_PLAN_MASKED_B | FSE_PLAN_REAL | FSE_PLAN_FIXED))
    return fail(FSE_ERR_UNSUPPORTED, "the warm start needs a cFSE plan with rectangular loss areas");
  if (pitch < batch->W) return fail(FSE_ERR_INVALID_ARG, "pitch smaller than the width");
  return fse::cnn::net_forward_blocks(net, d_image, d_avail, pitch, batch->H, batch->W, batch->d_blocks,
                                      batch->d_orig, batch->n, d_logits, reinterpret_cast<hipStream_t>(stream));
}

extern "C" int32_t fse_warm_trace_stride(fse_batch_t batch, int32_t restricted_iters, int32_t fallback_iters) {
  return batch ? restricted_iters + std::max(batch->max_iters, fallback_iters) : 0;
}

namespace {

fse_status_t warm_check(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail, int64_t pitch,
                        float* d_out, int64_t out_pitch, int32_t* d_status, const int16_t* d_cand,
                        const int32_t* d_flags, int32_t restricted_iters, int32_t fallback_iters) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  if (batch->plan->flags & (FSE_PLAN_MASKED_B | FSE_PLAN_REAL | FSE_PLAN_FIXED))
    return fail(FSE_ERR_UNSUPPORTED, "the warm start needs a cFSE plan with rectangular loss areas");
  if (batch->n == 0) return FSE_OK;
  if (!d_image || !d_avail || !d_out || !d_status || !d_cand || !d_flags)
    return fail(FSE_ERR_INVALID_ARG, "null device pointer");
  if (pitch < batch->W || out_pitch < batch->W) return fail(FSE_ERR_INVALID_ARG, "pitch smaller than the width");
  if (batch->cls[class_of(64)].count != batch->n) return fail(FSE_ERR_UNSUPPORTED, "the warm start needs F = 64 blocks only");
  if (restricted_iters < 0 || fallback_iters < 0 ||
      restricted_iters + std::max(batch->max_iters, fallback_iters) > batch->plan->max_iters)
    return fail(FSE_ERR_INVALID_ARG, "iteration counts outside the plan's limit");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != batch->device)
    return fail(FSE_ERR_INVALID_ARG, "batch was created on another device");
  return FSE_OK;
}

// Launch configuration of the warm-started form for (kc, ir, fb); host
// state and kernel attributes only, no device memory.
fse_status_t warm_configure(fse_batch_t batch, int32_t kc, int32_t restricted_iters, int32_t fallback_iters) {
  if (kc == batch->warm_kc && restricted_iters == batch->warm_ir && fallback_iters == batch->warm_fb)
    return FSE_OK;
  const int ci = class_of(64);
  // With no full iteration after the restricted ones, the transform and the
  // restricted iterations run as two kernels (split form); otherwise one
  // kernel does both phases.
  const bool split = batch->max_iters == 0;
  const fse::Variant* v = fse::warm_variant_for(64, kc, split ? fse::kWarmPrep : fse::kWarmFused);
  if (!v) return fail(FSE_ERR_UNSUPPORTED, "no warm-start kernel for this candidate count");
  fse_batch_s::Cls c = batch->cls[ci];
  c.iters_cap = split ? std::max(c.iters_cap, fallback_iters) : restricted_iters + std::max(c.iters_cap, fallback_iters);
  fse_status_t st = configure(batch, c, v);
  if (st != FSE_OK) return st;
  size_t lds = 0;
  if (split) {
    const void* rk = fse::restricted_kernel(kc);
    // without coefficient lists (and, with one wave, without the
    // cross-wave slots) a block needs 17 KB of LDS: nine per compute unit
    lds = fse::restricted_lds_bytes(kc, restricted_iters, !batch->all_small_b);
    if (!rk) return fail(FSE_ERR_UNSUPPORTED, "no restricted kernel for this candidate count");
    if (hipFuncSetAttribute(rk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return fail(FSE_ERR_HIP, "hipFuncSetAttribute failed (LDS size)");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rk, fse::restricted_threads(kc), lds) != hipSuccess ||
        per_cu < 1)
      return fail(FSE_ERR_UNSUPPORTED, "restricted kernel does not fit on a compute unit");
  }
  batch->restricted_lds = lds;
  batch->warm = c;
  batch->warm_split = split;
  batch->warm_kc = kc;
  batch->warm_ir = restricted_iters;
  batch->warm_fb = fallback_iters;
  return FSE_OK;
}

// Library-owned staging of the split form for every block of the batch,
// sized for kStageKcMax candidates; allocated once.
fse_status_t warm_staging(fse_batch_t batch) {
  if (!batch->warm_split || (batch->d_stage_w && batch->d_stage_r)) return FSE_OK;
  if (batch->in_workspace)
    return fail(FSE_ERR_WORKSPACE, "the batch's workspace holds no warm-start staging (FSE_WS_WARM)");
  if (hipMalloc(&batch->d_stage_r, (size_t)batch->n * kStageKcMax * sizeof(float2)) != hipSuccess) {
    batch->d_stage_r = nullptr;
    return fail(FSE_ERR_OOM, "hipMalloc failed (warm staging)");
  }
  if (hipMalloc(&batch->d_stage_w, (size_t)batch->n * fse::kHalfRows * 64 * sizeof(float2)) != hipSuccess) {
    batch->d_stage_w = nullptr;
    return fail(FSE_ERR_OOM, "hipMalloc failed (warm staging)");
  }
  batch->stage_kc = kStageKcMax;
  return FSE_OK;
}

}  // namespace

extern "C" fse_status_t fse_warm_prepare(fse_batch_t batch, int32_t kc, int32_t restricted_iters,
                                         int32_t fallback_iters) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  if (batch->plan->flags & (FSE_PLAN_MASKED_B | FSE_PLAN_REAL | FSE_PLAN_FIXED))
    return fail(FSE_ERR_UNSUPPORTED, "the warm start needs a cFSE plan with rectangular loss areas");
  if (batch->n == 0) return FSE_OK;
  if (batch->cls[class_of(64)].count != batch->n) return fail(FSE_ERR_UNSUPPORTED, "the warm start needs F = 64 blocks only");
  if (restricted_iters < 0 || fallback_iters < 0 ||
      restricted_iters + std::max(batch->max_iters, fallback_iters) > batch->plan->max_iters)
    return fail(FSE_ERR_INVALID_ARG, "iteration counts outside the plan's limit");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != batch->device)
    return fail(FSE_ERR_INVALID_ARG, "batch was created on another device");
  fse_status_t st = warm_configure(batch, kc, restricted_iters, fallback_iters);
  return st != FSE_OK ? st : warm_staging(batch);
}

extern "C" fse_status_t fse_warm_set_restricted_gamma(fse_batch_t batch, float gamma_r) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  if (!(gamma_r < 0.f || (gamma_r > 0.f && gamma_r <= 1.f)))
    return fail(FSE_ERR_INVALID_ARG, "the restricted step must lie in (0, 1], or be negative for the plan's gamma");
  batch->warm_gamma = gamma_r < 0.f ? -1.f : gamma_r;
  return FSE_OK;
}

extern "C" fse_status_t fse_warm_extrapolate_batch(fse_batch_t batch, const uint8_t* d_image,
                                                   const uint8_t* d_avail, int64_t pitch, float* d_out,
                                                   int64_t out_pitch, int32_t* d_status, fse_trace_t* d_trace,
                                                   const int16_t* d_cand, const int32_t* d_flags, int32_t kc,
                                                   int32_t restricted_iters, int32_t fallback_iters, void* stream) {
  fse_status_t st = warm_check(batch, d_image, d_avail, pitch, d_out, out_pitch, d_status, d_cand, d_flags,
                               restricted_iters, fallback_iters);
  if (st != FSE_OK || batch->n == 0) return st;
  if ((st = warm_configure(batch, kc, restricted_iters, fallback_iters)) != FSE_OK) return st;
  if ((st = warm_staging(batch)) != FSE_OK) return st;  // allocates only if fse_warm_prepare was not called
  WarmRange wr;
  wr.stage_w = batch->d_stage_w;
  wr.stage_r = batch->d_stage_r;
  return launch_one(batch, class_of(64), d_image, d_avail, pitch, d_out, out_pitch, d_status, d_trace,
                    reinterpret_cast<hipStream_t>(stream), d_cand, d_flags, wr);
}

extern "C" fse_status_t fse_initial_power(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                          int64_t pitch, float* d_power, void* stream) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  if (batch->plan->flags & (FSE_PLAN_MASKED_B | FSE_PLAN_REAL | FSE_PLAN_FIXED))
    return fail(FSE_ERR_UNSUPPORTED, "the initial spectrum needs a cFSE plan with rectangular loss areas");
  if (batch->n == 0) return FSE_OK;
  if (!d_image || !d_avail || !d_power) return fail(FSE_ERR_INVALID_ARG, "null device pointer");
  if (pitch < batch->W) return fail(FSE_ERR_INVALID_ARG, "pitch smaller than the width");
  const int ci = class_of(64);
  if (batch->cls[ci].count != batch->n) return fail(FSE_ERR_UNSUPPORTED, "the initial spectrum needs F = 64 blocks only");
  if ((int64_t)batch->H * pitch >= ((int64_t)1 << 31))
    return fail(FSE_ERR_INVALID_ARG, "a frame (H x pitch bytes) must be smaller than 2 GiB");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != batch->device)
    return fail(FSE_ERR_INVALID_ARG, "batch was created on another device");
  const fse::Variant* v = fse::power_variant_for(64);
  if (!v) return fail(FSE_ERR_UNSUPPORTED, "no power-spectrum kernel");
  fse_batch_s::Cls c = batch->cls[ci];
  c.iters_cap = 0;
  fse_status_t st = configure(batch, c, v);
  if (st != FSE_OK) return st;
  fse::ClassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.img = d_image;
  a.avail = d_avail;
  a.pitch = pitch;
  a.H = batch->H;
  a.W = batch->W;
  a.blocks = batch->d_blocks + c.offset;
  a.orig = batch->d_orig + c.offset;
  a.n = c.count;
  a.wtab = batch->tables->wtab;
  a.twid = batch->tables->twid[ci];
  a.gamma = batch->plan->gamma;
  a.power = d_power;
  if (fse::launch_class(*v, a, c.grid, c.lds, reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(FSE_ERR_HIP, "kernel launch failed (initial spectrum)");
  return FSE_OK;
}

extern "C" size_t fse_warm_noalloc_max_blocks(int32_t kc) {
  if (kc < 1 || kc > kStageKcMax) return 0;
  const size_t per_block = (size_t)fse::kHalfRows * 64 * sizeof(float2) + (size_t)kc * sizeof(float2);
  return (fse::kScratchBytes - 256) / per_block;
}

extern "C" fse_status_t fse_warm_extrapolate_batch_noalloc(fse_batch_t batch, const uint8_t* d_image,
                                                           const uint8_t* d_avail, int64_t pitch, float* d_out,
                                                           int64_t out_pitch, int32_t* d_status,
                                                           fse_trace_t* d_trace, const int16_t* d_cand,
                                                           const int32_t* d_flags, int32_t kc,
                                                           int32_t restricted_iters, int32_t fallback_iters,
                                                           void* stream) {
  fse_status_t st = warm_check(batch, d_image, d_avail, pitch, d_out, out_pitch, d_status, d_cand, d_flags,
                               restricted_iters, fallback_iters);
  if (st != FSE_OK || batch->n == 0) return st;
  if ((st = warm_configure(batch, kc, restricted_iters, fallback_iters)) != FSE_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int ci = class_of(64);
  if (!batch->warm_split)  // one kernel, no staging
    return launch_one(batch, ci, d_image, d_avail, pitch, d_out, out_pitch, d_status, d_trace, s, d_cand, d_flags);
  const size_t chunk = fse_warm_noalloc_max_blocks(kc);
  if (chunk == 0) return fail(FSE_ERR_UNSUPPORTED, "candidate count beyond the static staging");
  void* base = nullptr;
  if (fse::scratch_address(batch->device, &base) != hipSuccess)
    return fail(FSE_ERR_HIP, "hipGetSymbolAddress failed (static staging)");
  // W rows of each block first, then its candidates' R_w; 256-byte aligned
  WarmRange wr;
  wr.stage_w = reinterpret_cast<float2*>(base);
  const size_t wbytes = chunk * fse::kHalfRows * 64 * sizeof(float2);
  wr.stage_r = reinterpret_cast<float2*>(reinterpret_cast<char*>(base) + ((wbytes + 255) & ~(size_t)255));
  // consecutive ranges reuse the staging: each range's two kernels are
  // ordered on the stream before the next range's transform kernel
  for (int32_t start = 0; start < batch->n; start += (int32_t)chunk) {
    wr.start = start;
    wr.count = (int32_t)std::min<int64_t>((int64_t)chunk, batch->n - start);
    if ((st = launch_one(batch, ci, d_image, d_avail, pitch, d_out, out_pitch, d_status, d_trace, s, d_cand, d_flags,
                         wr)) != FSE_OK)
      return st;
  }
  return FSE_OK;
}

// ------------------------------------------------------------ 3-D (video)

struct fse_batch3d_s {
  fse_plan_t plan = nullptr;
  int device = 0;
  int32_t n = 0, n_frames = 0, H = 0, W = 0, max_iters = 0;
  int32_t grid = 0;
  size_t lds = 0;
  const DeviceTables* tables = nullptr;
  fse_volume_t* d_vols = nullptr;
  float* d_wtab3 = nullptr;
  bool in_workspace = false;               // device arrays lie in a caller's workspace (never freed here)
  DeviceTables ws_tables;                  // the F = 64 twiddles' copy in that workspace
};

namespace {
void free_batch3d(fse_batch3d_s* b) {
  if (!b->in_workspace) {
    (void)hipFree(b->d_vols);
    (void)hipFree(b->d_wtab3);
  }
  delete b;
}

// Byte offsets of a 3-D batch's arrays in a caller's workspace (256-byte
// aligned): volumes, the 3-D window table, the F = 64 twiddles.
struct Ws3Layout {
  size_t vols = 0, wtab3 = 0, twid = 0, total = 0;
};
Ws3Layout ws3_layout(fse_plan_t plan, int32_t n_volumes) {
  Ws3Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return at;
  };
  L.vols = take((size_t)std::max(n_volumes, 1) * sizeof(fse_volume_t));
  L.wtab3 = take((size_t)fse::kWinStrideT * fse::kWinStride * fse::kWinStride * sizeof(float));
  L.twid = take(plan->twid[class_of(fse::kF3)].size() * sizeof(float2));
  L.total = off;
  return L;
}

fse_status_t validate_volumes(fse_plan_t plan, const fse_volume_t* v, int32_t n, int32_t n_frames, int32_t H,
                              int32_t W, int32_t* bad) {
  if (bad) *bad = -1;
  if (!plan) return fail(FSE_ERR_INVALID_ARG, "null plan");
  if (plan->flags & (FSE_PLAN_MASKED_B | FSE_PLAN_REAL | FSE_PLAN_FIXED))
    return fail(FSE_ERR_UNSUPPORTED, "volumes need a cFSE plan with rectangular loss areas");
  if (n < 0 || (n > 0 && !v)) return fail(FSE_ERR_INVALID_ARG, "bad volume list");
  if (n_frames <= 0 || H <= 0 || W <= 0) return fail(FSE_ERR_INVALID_ARG, "clip dimensions must be positive");
  for (int32_t i = 0; i < n; ++i) {
    const fse_volume_t& b = v[i];
    if (bad) *bad = i;
    if (b.fft != fse::kF3 || b.fft_t != fse::kFt3) return fail(FSE_ERR_UNSUPPORTED, "volumes need a 64 x 64 x 8 transform");
    if (b.pad != 0) return fail(FSE_ERR_INVALID_ARG, "pad must be 0");
    if (b.bt < 1 || b.bh < 1 || b.bw < 1 || b.border < 0 || b.tborder < 0)
      return fail(FSE_ERR_INVALID_ARG, "volume size must be >= 1, borders >= 0");
    if (b.bh + 2 * b.border > b.fft || b.bw + 2 * b.border > b.fft || b.bt + 2 * b.tborder > b.fft_t)
      return fail(FSE_ERR_UNSUPPORTED, "area larger than the transform");
    if (b.iters < 0 || b.iters > plan->max_iters) return fail(FSE_ERR_INVALID_ARG, "iters outside [0, max_iters]");
    if (b.frame < 0 || (int64_t)b.frame + b.bt > n_frames || b.y0 < 0 || b.x0 < 0 || (int64_t)b.y0 + b.bh > H ||
        (int64_t)b.x0 + b.bw > W)
      return fail(FSE_ERR_INVALID_ARG, "lost volume outside the clip");
  }
  const size_t nvox = (size_t)n_frames * H * W;
  std::vector<uint64_t> bits((nvox + 63) / 64, 0);
  for (int32_t i = 0; i < n; ++i) {
    const fse_volume_t& b = v[i];
    for (int f = b.frame; f < b.frame + b.bt; ++f)
      for (int y = b.y0; y < b.y0 + b.bh; ++y)
        for (int x = b.x0; x < b.x0 + b.bw; ++x) {
          const size_t p = ((size_t)f * H + y) * W + x;
          const uint64_t m = 1ull << (p & 63);
          if (bits[p >> 6] & m) {
            if (bad) *bad = i;
            return fail(FSE_ERR_OVERLAP, "loss volumes of two entries overlap");
          }
          bits[p >> 6] |= m;
        }
  }
  if (bad) *bad = -1;
  return FSE_OK;
}
}  // namespace

namespace {
fse_status_t create_batch3d(fse_plan_t plan, const fse_volume_t* h_volumes, int32_t n_volumes, int32_t n_frames,
                            int32_t H, int32_t W, uint8_t* ws, fse_batch3d_t* out_batch, int32_t* bad_index);
}  // namespace

extern "C" fse_status_t fse_batch3d_create(fse_plan_t plan, const fse_volume_t* h_volumes, int32_t n_volumes,
                                           int32_t n_frames, int32_t H, int32_t W, fse_batch3d_t* out_batch,
                                           int32_t* bad_index) {
  return create_batch3d(plan, h_volumes, n_volumes, n_frames, H, W, nullptr, out_batch, bad_index);
}

extern "C" fse_status_t fse_batch3d_workspace_size(fse_plan_t plan, int32_t n_volumes, size_t* bytes) {
  if (!plan || !bytes) return fail(FSE_ERR_INVALID_ARG, "null argument");
  *bytes = 0;
  if (n_volumes < 0) return fail(FSE_ERR_INVALID_ARG, "negative volume count");
  *bytes = ws3_layout(plan, n_volumes).total;
  return FSE_OK;
}

extern "C" fse_status_t fse_batch3d_create_in(fse_plan_t plan, const fse_volume_t* h_volumes, int32_t n_volumes,
                                              int32_t n_frames, int32_t H, int32_t W, void* d_workspace,
                                              size_t ws_bytes, fse_batch3d_t* out_batch, int32_t* bad_index) {
  if (!out_batch) return fail(FSE_ERR_INVALID_ARG, "null argument");
  *out_batch = nullptr;
  if (bad_index) *bad_index = -1;
  size_t need = 0;
  fse_status_t st = fse_batch3d_workspace_size(plan, n_volumes, &need);
  if (st != FSE_OK) return st;
  st = check_workspace(d_workspace, ws_bytes, need);
  if (st != FSE_OK) return st;
  return create_batch3d(plan, h_volumes, n_volumes, n_frames, H, W, static_cast<uint8_t*>(d_workspace), out_batch,
                        bad_index);
}

namespace {
fse_status_t create_batch3d(fse_plan_t plan, const fse_volume_t* h_volumes, int32_t n_volumes, int32_t n_frames,
                            int32_t H, int32_t W, uint8_t* ws, fse_batch3d_t* out_batch, int32_t* bad_index) {
  if (!out_batch) return fail(FSE_ERR_INVALID_ARG, "null argument");
  *out_batch = nullptr;
  fse_status_t st = validate_volumes(plan, h_volumes, n_volumes, n_frames, H, W, bad_index);
  if (st != FSE_OK) return st;
  fse_batch3d_s* b = new (std::nothrow) fse_batch3d_s;
  if (!b) return fail(FSE_ERR_OOM, "host allocation failed");
  b->plan = plan;
  b->n = n_volumes;
  b->n_frames = n_frames;
  b->H = H;
  b->W = W;
  for (int32_t i = 0; i < n_volumes; ++i) b->max_iters = std::max(b->max_iters, h_volumes[i].iters);
  hipDeviceProp_t prop;
  if (hipGetDevice(&b->device) != hipSuccess || hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
    delete b;
    return fail(FSE_ERR_HIP, "hipGetDevice failed");
  }
  b->lds = fse::lds_bytes3d(std::max(b->max_iters, 1));
  const void* fn = fse::fse3d_kernel(false);
  int per_cu = 0;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds) != hipSuccess ||
      hipFuncSetAttribute(fse::fse3d_kernel(true), hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, fse::kNT3, b->lds) != hipSuccess || per_cu < 1) {
    delete b;
    return fail(FSE_ERR_UNSUPPORTED, "3-D kernel does not fit on a compute unit (iteration count too large)");
  }
  b->grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(n_volumes, (int64_t)per_cu * prop.multiProcessorCount));
  if (ws) {
    const Ws3Layout L = ws3_layout(plan, n_volumes);
    const std::vector<float2>& tw = plan->twid[class_of(fse::kF3)];
    b->in_workspace = true;
    b->d_vols = reinterpret_cast<fse_volume_t*>(ws + L.vols);
    b->d_wtab3 = reinterpret_cast<float*>(ws + L.wtab3);
    b->ws_tables.twid[class_of(fse::kF3)] = reinterpret_cast<float2*>(ws + L.twid);
    b->tables = &b->ws_tables;
    if (hipMemcpy(b->ws_tables.twid[class_of(fse::kF3)], tw.data(), tw.size() * sizeof(float2),
                  hipMemcpyHostToDevice) != hipSuccess) {
      free_batch3d(b);
      return fail(FSE_ERR_HIP, "upload of the twiddles failed");
    }
  } else {
    st = upload_tables(plan, b->device, &b->tables);
    if (st != FSE_OK) {
      delete b;
      return st;
    }
  }
  // eq. (3) in 3-D: rho^(sqrt(a^2 + b^2 + c^2) / 2) for doubled offsets, FP64, rounded once
  const int S = fse::kWinStride, ST = fse::kWinStrideT;
  std::vector<float> w3((size_t)ST * S * S);
  for (int c = 0; c < ST; ++c)
    for (int a = 0; a < S; ++a)
      for (int d = 0; d < S; ++d)
        w3[((size_t)c * S + a) * S + d] =
            (float)std::pow((double)plan->rho, 0.5 * std::sqrt((double)a * a + (double)d * d + (double)c * c));
  const size_t nv = (size_t)std::max(n_volumes, 1);
  if (!ws && (hipMalloc(&b->d_vols, nv * sizeof(fse_volume_t)) != hipSuccess ||
              hipMalloc(&b->d_wtab3, w3.size() * sizeof(float)) != hipSuccess)) {
    free_batch3d(b);
    return fail(FSE_ERR_OOM, "hipMalloc failed (3-D batch)");
  }
  if ((n_volumes > 0 && hipMemcpy(b->d_vols, h_volumes, (size_t)n_volumes * sizeof(fse_volume_t),
                                  hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(b->d_wtab3, w3.data(), w3.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    free_batch3d(b);
    return fail(FSE_ERR_HIP, "upload failed (3-D batch)");
  }
  *out_batch = b;
  return FSE_OK;
}
}  // namespace

extern "C" void fse_batch3d_destroy(fse_batch3d_t batch) {
  if (!batch) return;
  (void)hipDeviceSynchronize();
  free_batch3d(batch);
}

static fse_status_t launch3d(fse_batch3d_t batch, const uint8_t* d_frames, const uint8_t* d_avail, int64_t pitch,
                             float* d_out, int64_t out_pitch, int32_t* d_status, fse_trace_t* d_trace,
                             const int16_t* d_cand2, const int32_t* d_flags, void* stream) {
  if (!batch) return fail(FSE_ERR_INVALID_ARG, "null batch");
  if (batch->n == 0) return FSE_OK;
  if (!d_frames || !d_avail || !d_out || !d_status) return fail(FSE_ERR_INVALID_ARG, "null device pointer");
  if (pitch < batch->W || out_pitch < batch->W) return fail(FSE_ERR_INVALID_ARG, "pitch smaller than the width");
  if ((int64_t)batch->H * pitch >= ((int64_t)1 << 31))
    return fail(FSE_ERR_INVALID_ARG, "a frame (H x pitch bytes) must be smaller than 2 GiB");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != batch->device)
    return fail(FSE_ERR_INVALID_ARG, "batch was created on another device");
  fse::Vol3Args a;
  a.img = d_frames;
  a.avail = d_avail;
  a.pitch = pitch;
  a.out = d_out;
  a.out_pitch = out_pitch;
  a.n_frames = batch->n_frames;
  a.H = batch->H;
  a.W = batch->W;
  a.vols = batch->d_vols;
  a.n = batch->n;
  a.iters_cap = std::max(batch->max_iters, 1);
  a.status = d_status;
  a.trace = d_trace;
  a.trace_stride = batch->max_iters;
  a.wtab3 = batch->d_wtab3;
  a.twid = batch->tables->twid[class_of(fse::kF3)];
  a.gamma = batch->plan->gamma;
  a.cand2 = d_cand2;
  a.flags = d_flags;
  const bool warm = d_cand2 != nullptr;
  if (fse::launch_fse3d(a, warm, batch->grid, batch->lds, reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(FSE_ERR_HIP, "kernel launch failed (3-D)");
  return FSE_OK;
}

extern "C" fse_status_t fse_extrapolate3d_batch(fse_batch3d_t batch, const uint8_t* d_frames, const uint8_t* d_avail,
                                                int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                                fse_trace_t* d_trace, void* stream) {
  return launch3d(batch, d_frames, d_avail, pitch, d_out, out_pitch, d_status, d_trace, nullptr, nullptr, stream);
}

extern "C" fse_status_t fse_warm3d_extrapolate_batch(fse_batch3d_t batch, const uint8_t* d_frames,
                                                     const uint8_t* d_avail, int64_t pitch, float* d_out,
                                                     int64_t out_pitch, int32_t* d_status, fse_trace_t* d_trace,
                                                     const int16_t* d_cand2, const int32_t* d_flags, int32_t k2,
                                                     void* stream) {
  if (!d_cand2 || !d_flags) return fail(FSE_ERR_INVALID_ARG, "null candidate list");
  if (k2 != fse::kCand3) return fail(FSE_ERR_UNSUPPORTED, "the 3-D warm start takes 128 candidate columns per volume");
  return launch3d(batch, d_frames, d_avail, pitch, d_out, out_pitch, d_status, d_trace, d_cand2, d_flags, stream);
}
