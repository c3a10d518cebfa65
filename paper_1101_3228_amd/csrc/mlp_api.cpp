// C ABI of the pricing surrogate: workspace layout, validation and the
// launch sequences of inference and training.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "qtree_mlp.h"
#include "qtree_mlp_internal.hpp"
#include "qtree_plan.hpp"

using qtree::set_error;
namespace M = qtree::mlp;

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr int64_t kMaxBatch = int64_t(1) << 24;

// Byte offsets of every buffer in the workspace.
struct MlpLayout {
  size_t master, mom, vel, grad, w1, w4, w2f, w3f, w2t, w3t;
  size_t z1, z2, z3, h1, h2, dz1, dz2, dz3, u, dy, lossp, part;
  size_t total;
  int64_t bp;
};

MlpLayout mlp_layout(int64_t max_batch) {
  MlpLayout L{};
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  const size_t P = (size_t)M::kParams;
  L.master = take(4 * P);
  L.mom = take(4 * P);
  L.vel = take(4 * P);
  L.grad = take(4 * P);
  L.w1 = take(2 * M::kHid * 16);  // layer-1 fragments: 16 K-slots per row
  L.w4 = take(2 * M::kHid);
  L.w2f = take(2 * M::kHid * M::kHid);
  L.w3f = take(2 * M::kHid * M::kHid);
  L.w2t = take(2 * M::kHid * M::kHid);
  L.w3t = take(2 * M::kHid * M::kHid);
  const int64_t bp = (max_batch + M::kChunk - 1) / M::kChunk * M::kChunk;
  L.bp = bp;
  if (bp > 0) {
    const size_t per = (size_t)M::kHid * (size_t)bp;
    L.z1 = take(4 * per);
    L.z2 = take(4 * per);
    L.z3 = take(4 * per);
    L.h1 = take(2 * per);
    L.h2 = take(2 * per);
    L.dz1 = take(4 * per);
    L.dz2 = take(4 * per);
    L.dz3 = take(4 * per);
    L.u = take(4 * 8 * (size_t)bp);
    L.dy = take(4 * (size_t)bp);
    L.lossp = take(4 * (size_t)(bp / M::kWaveRows));
    L.part = take(4 * 2 * (size_t)(bp / M::kChunk) * M::kHid * M::kHid);
  }
  L.total = off;
  return L;
}

qtree_status hip_fail(hipError_t e, const char* what) {
  return set_error(QTREE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

struct qtree_mlp {
  char* ws = nullptr;
  MlpLayout lay{};
  int64_t max_batch = 0;
  int terms = 2;
  int64_t step = 0;
  M::Weights W{};

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

namespace {

M::AdamArgs adam_args(qtree_mlp* m) {
  M::AdamArgs a{};
  a.master = m->at<float>(m->lay.master);
  a.mom = m->at<float>(m->lay.mom);
  a.vel = m->at<float>(m->lay.vel);
  a.grad = m->at<float>(m->lay.grad);
  a.w1 = m->at<uint16_t>(m->lay.w1);
  a.w4 = m->at<uint16_t>(m->lay.w4);
  a.w2f = m->at<uint16_t>(m->lay.w2f);
  a.w3f = m->at<uint16_t>(m->lay.w3f);
  a.w2t = m->at<uint16_t>(m->lay.w2t);
  a.w3t = m->at<uint16_t>(m->lay.w3t);
  return a;
}

// Upload parameters, clear the Adam state and derive the BF16 copies.
qtree_status load_params(qtree_mlp* m, const float* params_host) {
  for (int i = 0; i < M::kParams; ++i)
    if (!std::isfinite(params_host[i])) return set_error(QTREE_EINVAL, "non-finite parameter");
  hipError_t e = hipMemcpy(m->ws + m->lay.master, params_host, sizeof(float) * M::kParams,
                           hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->ws + m->lay.mom, 0, sizeof(float) * M::kParams);
  if (e == hipSuccess) e = hipMemset(m->ws + m->lay.vel, 0, sizeof(float) * M::kParams);
  if (e != hipSuccess) return hip_fail(e, "parameter upload");
  M::AdamArgs a = adam_args(m);
  a.update = 0;
  e = M::launch_adam(a, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "weight copies");
  m->step = 0;
  return QTREE_OK;
}

qtree_status check_batch(const qtree_mlp* m, const float* x, const float* t, int64_t B) {
  if (!m) return set_error(QTREE_EINVAL, "mlp is NULL");
  if (m->max_batch == 0) return set_error(QTREE_EINVAL, "created for inference only");
  if (B < 1 || B > m->max_batch) return set_error(QTREE_EINVAL, "B must be in 1..max_batch");
  if (!x || !t) return set_error(QTREE_EINVAL, "x or t is NULL");
  return QTREE_OK;
}

M::Train train_args(const qtree_mlp* m, const float* x, const float* t, const float* w,
                    const int32_t* idx, int64_t B) {
  M::Train T{};
  T.x = x;
  T.t = t;
  T.w = w;
  T.idx = idx;
  T.B = B;
  T.Bp = (B + M::kChunk - 1) / M::kChunk * M::kChunk;
  T.inv_b = (float)(1.0 / (double)B);
  T.z1 = m->at<float>(m->lay.z1);
  T.z2 = m->at<float>(m->lay.z2);
  T.z3 = m->at<float>(m->lay.z3);
  T.h1 = m->at<uint16_t>(m->lay.h1);
  T.h2 = m->at<uint16_t>(m->lay.h2);
  T.dz1 = m->at<float>(m->lay.dz1);
  T.dz2 = m->at<float>(m->lay.dz2);
  T.dz3 = m->at<float>(m->lay.dz3);
  T.u = m->at<float>(m->lay.u);
  T.dy = m->at<float>(m->lay.dy);
  T.lossp = m->at<float>(m->lay.lossp);
  T.part = m->at<float>(m->lay.part);
  return T;
}

}  // namespace

extern "C" {

qtree_status qtree_mlp_workspace_size(int64_t max_batch, size_t* bytes) {
  if (!bytes) return set_error(QTREE_EINVAL, "bytes is NULL");
  if (max_batch < 0 || max_batch > kMaxBatch)
    return set_error(QTREE_EINVAL, "max_batch must be in 0..2^24");
  *bytes = mlp_layout(max_batch).total;
  return QTREE_OK;
}

qtree_status qtree_mlp_create(const float* params_host, const float* lo, const float* hi,
                              float out_scale, int32_t act_terms, int32_t baseline,
                              int64_t max_batch, void* workspace, size_t workspace_bytes,
                              qtree_mlp** out) {
  if (!out) return set_error(QTREE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params_host || !lo || !hi || !workspace)
    return set_error(QTREE_EINVAL, "NULL argument");
  if (act_terms != 1 && act_terms != 2) return set_error(QTREE_EINVAL, "act_terms must be 1 or 2");
  if (baseline != 0 && baseline != 1) return set_error(QTREE_EINVAL, "baseline must be 0 or 1");
  if (!std::isfinite(out_scale) || out_scale == 0.0f)
    return set_error(QTREE_EINVAL, "out_scale must be finite and nonzero");
  if (max_batch < 0 || max_batch > kMaxBatch)
    return set_error(QTREE_EINVAL, "max_batch must be in 0..2^24");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return set_error(QTREE_EINVAL, "workspace must be 256-byte aligned");
  for (int c = 0; c < M::kIn; ++c)
    if (!std::isfinite(lo[c]) || !std::isfinite(hi[c]) || !(lo[c] <= hi[c]))
      return set_error(QTREE_EINVAL, "box bounds must be finite with lo <= hi");
  if (baseline == 1 && !(lo[0] > 0.0f && lo[1] > 0.0f && lo[3] > 0.0f))
    return set_error(QTREE_EINVAL, "the Black-Scholes baseline needs S0/K, sigma, T > 0 in the box");
  const MlpLayout L = mlp_layout(max_batch);
  if (workspace_bytes < L.total) return set_error(QTREE_ENOMEM, "workspace too small");
  qtree_mlp* m = new qtree_mlp;
  m->ws = static_cast<char*>(workspace);
  m->lay = L;
  m->max_batch = max_batch;
  m->terms = act_terms;
  M::Weights& W = m->W;
  W.master = m->at<float>(L.master);
  W.w1 = m->at<uint16_t>(L.w1);
  W.w4 = m->at<uint16_t>(L.w4);
  W.w2f = m->at<uint16_t>(L.w2f);
  W.w3f = m->at<uint16_t>(L.w3f);
  W.w2t = m->at<uint16_t>(L.w2t);
  W.w3t = m->at<uint16_t>(L.w3t);
  for (int c = 0; c < M::kIn; ++c) {
    W.lo[c] = lo[c];
    W.hi[c] = hi[c];
    const bool fixed = hi[c] == lo[c];
    W.scale[c] = fixed ? 0.0f : (float)(2.0 / ((double)hi[c] - (double)lo[c]));
    W.shift[c] = fixed ? 0.0f : -1.0f;
  }
  W.out_scale = out_scale;
  W.baseline = baseline;
  const qtree_status st = load_params(m, params_host);
  if (st != QTREE_OK) {
    delete m;
    return st;
  }
  *out = m;
  return QTREE_OK;
}

void qtree_mlp_destroy(qtree_mlp* mlp) { delete mlp; }

qtree_status qtree_mlp_get_params(const qtree_mlp* mlp, float* params_host) {
  if (!mlp || !params_host) return set_error(QTREE_EINVAL, "NULL argument");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(params_host, mlp->ws + mlp->lay.master, sizeof(float) * M::kParams,
                  hipMemcpyDeviceToHost);
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "parameter download");
}

qtree_status qtree_mlp_set_params(qtree_mlp* mlp, const float* params_host) {
  if (!mlp || !params_host) return set_error(QTREE_EINVAL, "NULL argument");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  return load_params(mlp, params_host);
}

qtree_status qtree_mlp_forward(const qtree_mlp* mlp, const float* x, int64_t B, float* y,
                               uint8_t* in_range, void* stream) {
  if (!mlp) return set_error(QTREE_EINVAL, "mlp is NULL");
  if (B < 0 || B > (int64_t(1) << 40)) return set_error(QTREE_EINVAL, "B out of range");
  if (B == 0) return QTREE_OK;
  if (!x || !y) return set_error(QTREE_EINVAL, "x or y is NULL");
  const hipError_t e = M::launch_forward(mlp->W, mlp->terms, x, B, y, in_range,
                                         static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "forward launch");
}

qtree_status qtree_mlp_grad(qtree_mlp* mlp, const float* x, const float* t, const float* w,
                            const int32_t* idx, int64_t B, float* grad, float* loss,
                            void* stream) {
  qtree_status st = check_batch(mlp, x, t, B);
  if (st != QTREE_OK) return st;
  const M::Train T = train_args(mlp, x, t, w, idx, B);
  float* g = grad ? grad : mlp->at<float>(mlp->lay.grad);
  const hipError_t e = M::launch_train_grad(mlp->W, mlp->terms, T, g, loss,
                                            static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QTREE_OK : hip_fail(e, "gradient launch");
}

qtree_status qtree_mlp_train_step(qtree_mlp* mlp, const float* x, const float* t, const float* w,
                                  const int32_t* idx, int64_t B, const qtree_adam* opt,
                                  float* loss, void* stream) {
  qtree_status st = check_batch(mlp, x, t, B);
  if (st != QTREE_OK) return st;
  if (!opt) return set_error(QTREE_EINVAL, "opt is NULL");
  if (!(opt->lr >= 0.0f) || !(opt->beta1 >= 0.0f && opt->beta1 < 1.0f) ||
      !(opt->beta2 >= 0.0f && opt->beta2 < 1.0f) || !(opt->eps > 0.0f))
    return set_error(QTREE_EINVAL, "Adam parameters out of range");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const M::Train T = train_args(mlp, x, t, w, idx, B);
  hipError_t e = M::launch_train_grad(mlp->W, mlp->terms, T, mlp->at<float>(mlp->lay.grad),
                                      loss, s);
  if (e != hipSuccess) return hip_fail(e, "gradient launch");
  const int64_t step = mlp->step + 1;
  M::AdamArgs a = adam_args(mlp);
  a.lr = opt->lr;
  a.beta1 = opt->beta1;
  a.beta2 = opt->beta2;
  a.eps = opt->eps;
  a.c1 = (float)(1.0 / (1.0 - std::pow((double)opt->beta1, (double)step)));
  a.c2 = (float)(1.0 / (1.0 - std::pow((double)opt->beta2, (double)step)));
  a.update = 1;
  e = M::launch_adam(a, s);
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  mlp->step = step;
  return QTREE_OK;
}

}  // extern "C"
