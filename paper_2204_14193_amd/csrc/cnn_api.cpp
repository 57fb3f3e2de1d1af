// Host side of the warm-start network entry points of include/fse.h:
// parameter storage, forward, backward (gradients), Adam, top-K.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "cnn_internal.h"
#include "fse.h"
#include "fse_internal.h"

namespace {
fse_status_t cfail(fse_status_t code, const char* msg) {
  fse::set_error(msg);
  return code;
}
using namespace fse::cnn;

// Deterministic He-uniform initialisation from a 64-bit seed (splitmix64).
uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
}  // namespace

struct fse_cnn_s {
  int device = 0;
  int32_t max_batch = 0;
  int64_t step = 0;
  float* master = nullptr;   // FP32 master parameters
  float* grad = nullptr;     // FP32 gradient (cleared by every Adam step)
  float* m = nullptr;
  float* v = nullptr;
  uint16_t* work = nullptr;  // BF16 working copy used by every kernel
  uint16_t* feats = nullptr; // [max_batch][288]
  // inference head: features and head weights in fragment layout
  uint16_t* feats_frag = nullptr;  // [ceil(max_batch / 32) * 32][288]
  uint16_t* head_frag = nullptr;   // [4096][288]
  bool head_stale = false;         // `work` changed since head_frag was made (after Adam)
  // training scratch, allocated on the first backward call
  uint16_t* acts = nullptr;   // [max_batch][kActElems]
  float* dlog = nullptr;      // [B][4096]
  uint16_t* dlog_b = nullptr; // [B][4096]
  uint16_t* dlog_t = nullptr; // [4096][B]
  uint16_t* feat_t = nullptr; // [288][B]
  uint16_t* head_t = nullptr; // [288][4096]
  uint16_t* w_t = nullptr;    // [288][32]
  float* da = nullptr;        // [B * 576][32]
  float* dz = nullptr;
  uint16_t* dz_b = nullptr;
  uint16_t* dz_t = nullptr;
  uint16_t* col = nullptr;    // [B * 144][288] at most
  uint16_t* col_t = nullptr;
  float* dcol = nullptr;
  bool kept = false;          // activations of the last forward are stored
  int32_t kept_batch = 0;
};

namespace {
void free_net(fse_cnn_s* n) {
  void* ptrs[] = {n->master, n->grad, n->m, n->v, n->work, n->feats, n->feats_frag, n->head_frag, n->acts, n->dlog, n->dlog_b,
                  n->dlog_t, n->feat_t, n->head_t, n->w_t, n->da, n->dz, n->dz_b, n->dz_t, n->col,
                  n->col_t, n->dcol};
  for (void* p : ptrs) (void)hipFree(p);
  delete n;
}

template <class T>
bool dalloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) == hipSuccess;
}

fse_status_t ensure_training(fse_cnn_s* n) {
  if (n->acts) return FSE_OK;
  const size_t B = (size_t)n->max_batch;
  const bool ok = dalloc(&n->acts, B * kActElems) && dalloc(&n->dlog, B * kBins) && dalloc(&n->dlog_b, B * kBins) &&
                  dalloc(&n->dlog_t, B * kBins) && dalloc(&n->feat_t, B * kFeat) &&
                  dalloc(&n->head_t, (size_t)kBins * kFeat) && dalloc(&n->w_t, (size_t)288 * kCh) &&
                  dalloc(&n->da, B * 576 * kCh) && dalloc(&n->dz, B * 576 * kCh) &&
                  dalloc(&n->dz_b, B * 576 * kCh) && dalloc(&n->dz_t, B * 576 * kCh) &&
                  dalloc(&n->col, B * 144 * 288) && dalloc(&n->col_t, B * 144 * 288) &&
                  dalloc(&n->dcol, B * 144 * 288);
  return ok ? FSE_OK : cfail(FSE_ERR_OOM, "hipMalloc failed (training buffers)");
}

bool check_device(const fse_cnn_s* n) {
  int dev = -1;
  return hipGetDevice(&dev) == hipSuccess && dev == n->device;
}
}  // namespace

extern "C" int64_t fse_cnn_num_params(void) { return kNumParams; }

extern "C" fse_status_t fse_cnn_create(int32_t max_batch, uint64_t seed, fse_cnn_t* out) {
  if (!out) return cfail(FSE_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1 << 20)) return cfail(FSE_ERR_INVALID_ARG, "max_batch must lie in [1, 2^20]");
  fse_cnn_s* n = new (std::nothrow) fse_cnn_s;
  if (!n) return cfail(FSE_ERR_OOM, "host allocation failed");
  n->max_batch = max_batch;
  if (hipGetDevice(&n->device) != hipSuccess) {
    delete n;
    return cfail(FSE_ERR_HIP, "hipGetDevice failed");
  }
  const size_t P = (size_t)kNumParams;
  if (!dalloc(&n->master, P) || !dalloc(&n->grad, P) || !dalloc(&n->m, P) || !dalloc(&n->v, P) ||
      !dalloc(&n->work, P) || !dalloc(&n->feats, (size_t)max_batch * kFeat) ||
      !dalloc(&n->feats_frag, (size_t)(max_batch + 31) / 32 * 32 * kFeat) ||
      !dalloc(&n->head_frag, (size_t)kBins * kFeat)) {
    free_net(n);
    return cfail(FSE_ERR_OOM, "hipMalloc failed (parameters)");
  }
  // He-uniform weights (bound sqrt(6 / fan_in)), zero biases
  std::vector<float> h(P, 0.f);
  uint64_t st = seed;
  auto fill = [&](int64_t off, int64_t count, int fan_in) {
    const double lim = std::sqrt(6.0 / fan_in);
    for (int64_t i = 0; i < count; ++i) {
      const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
      h[off + i] = (float)((2.0 * u - 1.0) * lim);
    }
  };
  for (int l = 0; l < 4; ++l) fill(kOffW[l], (int64_t)kCh * kKdim[l], kKdim[l]);
  fill(kOffHeadW, (int64_t)kBins * kFeat, kFeat);
  if (hipMemcpy(n->master, h.data(), P * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n->grad, 0, P * 4) != hipSuccess || hipMemset(n->m, 0, P * 4) != hipSuccess ||
      hipMemset(n->v, 0, P * 4) != hipSuccess || f32_to_bf16(n->master, (int64_t)P, n->work, nullptr) != hipSuccess ||
      permute_head(n->work + kOffHeadW, n->head_frag, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    free_net(n);
    return cfail(FSE_ERR_HIP, "parameter upload failed");
  }
  *out = n;
  return FSE_OK;
}

extern "C" void fse_cnn_destroy(fse_cnn_t net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  free_net(net);
}

extern "C" fse_status_t fse_cnn_set_params(fse_cnn_t net, const float* h_params) {
  if (!net || !h_params) return cfail(FSE_ERR_INVALID_ARG, "null argument");
  if (!check_device(net)) return cfail(FSE_ERR_INVALID_ARG, "network was created on another device");
  const size_t P = (size_t)kNumParams;
  // the inference layout of the head is made here too, so that the first
  // forward pass after a parameter upload launches no set-up kernel
  if (hipMemcpy(net->master, h_params, P * 4, hipMemcpyHostToDevice) != hipSuccess ||
      f32_to_bf16(net->master, (int64_t)P, net->work, nullptr) != hipSuccess ||
      permute_head(net->work + kOffHeadW, net->head_frag, nullptr) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return cfail(FSE_ERR_HIP, "parameter upload failed");
  net->head_stale = false;
  return FSE_OK;
}

extern "C" fse_status_t fse_cnn_get_params(fse_cnn_t net, float* h_params, float* h_grads) {
  if (!net) return cfail(FSE_ERR_INVALID_ARG, "null argument");
  if (!check_device(net)) return cfail(FSE_ERR_INVALID_ARG, "network was created on another device");
  const size_t P = (size_t)kNumParams;
  if (hipDeviceSynchronize() != hipSuccess) return cfail(FSE_ERR_HIP, "hipDeviceSynchronize failed");
  if (h_params && hipMemcpy(h_params, net->master, P * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return cfail(FSE_ERR_HIP, "parameter download failed");
  if (h_grads && hipMemcpy(h_grads, net->grad, P * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return cfail(FSE_ERR_HIP, "gradient download failed");
  return FSE_OK;
}

extern "C" fse_status_t fse_cnn_forward(fse_cnn_t net, const uint16_t* d_x, int32_t B, float* d_logits,
                                        int32_t keep_activations, void* stream) {
  if (!net || !d_x || !d_logits) return cfail(FSE_ERR_INVALID_ARG, "null argument");
  if (B < 1 || B > net->max_batch) return cfail(FSE_ERR_INVALID_ARG, "batch size outside [1, max_batch]");
  if (!check_device(net)) return cfail(FSE_ERR_INVALID_ARG, "network was created on another device");
  if (keep_activations) {
    fse_status_t st = ensure_training(net);
    if (st != FSE_OK) return st;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (forward(d_x, B, net->work, net->feats, keep_activations ? net->acts : nullptr, s) != hipSuccess ||
      gemm_nt(net->feats, kFeat, net->work + kOffHeadW, kFeat, d_logits, kBins, net->work + kOffHeadB, B, kBins,
              kFeat, s) != hipSuccess)
    return cfail(FSE_ERR_HIP, "kernel launch failed");
  net->kept = keep_activations != 0;
  net->kept_batch = B;
  return FSE_OK;
}

namespace fse {
namespace cnn {
// Forward pass from the frames for the blocks of a batch (see
// fse_cnn_forward_blocks); argument checks on the batch are the caller's.
fse_status_t net_forward_blocks(fse_cnn_t net, const uint8_t* img, const uint8_t* avail, int64_t pitch, int32_t H,
                                int32_t W, const void* blocks, const int32_t* orig, int32_t n, float* d_logits,
                                hipStream_t s) {
  if (!net || !d_logits) return cfail(FSE_ERR_INVALID_ARG, "null argument");
  if (n > net->max_batch) return cfail(FSE_ERR_INVALID_ARG, "more blocks than the network's max_batch");
  if (!check_device(net)) return cfail(FSE_ERR_INVALID_ARG, "network was created on another device");
  if (n == 0) return FSE_OK;
  if (net->head_stale) {
    if (permute_head(net->work + kOffHeadW, net->head_frag, s) != hipSuccess)
      return cfail(FSE_ERR_HIP, "kernel launch failed");
    net->head_stale = false;
  }
  if (forward_blocks(img, avail, pitch, H, W, blocks, orig, n, net->work, net->feats_frag, s) != hipSuccess ||
      head_frag(net->feats_frag, net->head_frag, net->work + kOffHeadB, d_logits, n, s) != hipSuccess)
    return cfail(FSE_ERR_HIP, "kernel launch failed");
  net->kept = false;
  return FSE_OK;
}
}  // namespace cnn
}  // namespace fse

extern "C" fse_status_t fse_cnn_backward(fse_cnn_t net, const uint16_t* d_x, const float* d_logits,
                                         const uint32_t* d_target_bits, int32_t B, float pos_weight, float* d_loss,
                                         void* stream) {
  if (!net || !d_x || !d_logits || !d_target_bits || !d_loss) return cfail(FSE_ERR_INVALID_ARG, "null argument");
  if (!net->kept || net->kept_batch != B)
    return cfail(FSE_ERR_INVALID_ARG, "backward needs the activations of a forward over the same batch");
  if (B % 16 != 0) return cfail(FSE_ERR_INVALID_ARG, "training batch size must be a multiple of 16");
  if (!(pos_weight > 0.f)) return cfail(FSE_ERR_INVALID_ARG, "pos_weight must be positive");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bool ok = true;
  auto chk = [&](hipError_t e) { ok = ok && e == hipSuccess; };
  const int64_t Bl = B;
  // loss and dL/dlogits
  chk(bce(d_logits, d_target_bits, B, pos_weight, net->dlog, d_loss, s));
  // head: bias, weight, and gradient of the features
  chk(colsum_add(net->dlog, B, kBins, net->grad + kOffHeadB, s));
  chk(f32_to_bf16(net->dlog, Bl * kBins, net->dlog_b, s));
  chk(transpose_u16(net->dlog_b, B, kBins, kBins, net->dlog_t, B, s));
  chk(transpose_u16(net->feats, B, kFeat, kFeat, net->feat_t, B, s));
  chk(gemm_nt(net->dlog_t, B, net->feat_t, B, net->grad + kOffHeadW, kFeat, nullptr, kBins, kFeat, B, s));
  chk(transpose_u16(net->work + kOffHeadW, kBins, kFeat, kFeat, net->head_t, kBins, s));
  chk(gemm_nt(net->dlog_b, kBins, net->head_t, kBins, net->da, kFeat, nullptr, B, kFeat, kBins, s));
  // convolutions, last to first; da holds dL/d(output of layer l)
  for (int l = 3; l >= 0 && ok; --l) {
    const int HO = kHin[l] / 2;
    const int rows = B * HO * HO;
    const int K = kKdim[l], KP = kKpad[l];
    chk(relu_mask(net->da, net->acts + kActOff[l], HO * HO * kCh, kActElems, (int64_t)rows * kCh, net->dz,
                  net->dz_b, s));
    chk(colsum_add(net->dz, rows, kCh, net->grad + kOffB[l], s));
    chk(transpose_u16(net->dz_b, rows, kCh, kCh, net->dz_t, rows, s));
    const uint16_t* in = l == 0 ? d_x : net->acts + kActOff[l - 1];
    chk(im2col(in, B, l, net->col, s));
    chk(transpose_u16(net->col, rows, KP, KP, net->col_t, rows, s));
    chk(gemm_nt(net->dz_t, rows, net->col_t, rows, net->grad + kOffW[l], K, nullptr, kCh, K, rows, s));
    if (l > 0) {
      chk(transpose_u16(net->work + kOffW[l], kCh, K, K, net->w_t, kCh, s));
      chk(gemm_nt(net->dz_b, kCh, net->w_t, kCh, net->dcol, KP, nullptr, rows, KP, kCh, s));
      chk(col2im(net->dcol, B, l, net->da, s));
    }
  }
  return ok ? FSE_OK : cfail(FSE_ERR_HIP, "kernel launch failed");
}

extern "C" fse_status_t fse_cnn_adam(fse_cnn_t net, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!net) return cfail(FSE_ERR_INVALID_ARG, "null argument");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return cfail(FSE_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  net->step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)net->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)net->step)));
  if (adam(net->master, net->grad, net->m, net->v, net->work, kNumParams, lr, beta1, beta2, eps, c1, c2,
           reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return cfail(FSE_ERR_HIP, "kernel launch failed");
  net->head_stale = true;
  return FSE_OK;
}

extern "C" fse_status_t fse_cnn_topk(const float* d_logits, int32_t B, int32_t K, int16_t* d_cand, int32_t* d_flags,
                                     void* stream) {
  if (!d_logits || !d_cand || !d_flags) return cfail(FSE_ERR_INVALID_ARG, "null argument");
  if (B < 0 || K < 1 || K > kBins) return cfail(FSE_ERR_INVALID_ARG, "K must lie in [1, 4096]");
  if (topk(d_logits, B, K, d_cand, d_flags, reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return cfail(FSE_ERR_HIP, "kernel launch failed");
  return FSE_OK;
}
