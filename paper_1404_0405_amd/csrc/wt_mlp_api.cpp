// C ABI of the child-patch predictor network.
#include <hip/hip_runtime.h>

#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "wt.h"
#include "wt_mlp.hpp"

namespace wt {
int api_fail(int code, const std::string& msg);   // sets the thread-local message (wt_api.cpp)
}

struct wt_mlp {
  wt::MlpDev dev;
  hipStream_t own = nullptr, stream = nullptr;
};

namespace wt {
// Inference for the learned adjacent zone, on the grid's stream.
void mlp_predict(wt_mlp* m, const float* X, int64_t n, float* P, hipStream_t s) { m->dev.forward(X, n, P, s); }
}  // namespace wt

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

static_assert(wt::MLP_NP == WT_MLP_PARAMS && wt::MLP_NI == WT_MLP_INPUTS && wt::MLP_NO == WT_MLP_OUTPUTS,
              "network sizes");

extern "C" {

wt_mlp* wt_mlp_create(const float* params_host) {
  if (!params_host) {
    wt::api_fail(WT_EINVAL, "wt_mlp_create: null parameters");
    return nullptr;
  }
  wt_mlp* m = new wt_mlp;
  try {
    HIPCHK(hipStreamCreateWithFlags(&m->own, hipStreamNonBlocking));
    m->stream = m->own;
    m->dev.alloc();
    HIPCHK(hipMemcpy(m->dev.theta, params_host, wt::MLP_NP * sizeof(float), hipMemcpyHostToDevice));
    m->dev.pack(m->stream);
    HIPCHK(hipStreamSynchronize(m->stream));
    (void)wt::noalloc_scratch();   // set-up of the allocation-free gradient on this device
  } catch (const std::exception& e) {
    wt::api_fail(WT_EDEVICE, std::string("wt_mlp_create: ") + e.what());
    m->dev.release();
    if (m->own) (void)hipStreamDestroy(m->own);
    delete m;
    return nullptr;
  }
  return m;
}

void wt_mlp_destroy(wt_mlp* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  m->dev.release();
  if (m->own) (void)hipStreamDestroy(m->own);
  delete m;
}

int wt_mlp_set_stream(wt_mlp* m, void* s) {
  if (!m) return wt::api_fail(WT_EINVAL, "wt_mlp_set_stream: null network");
  m->stream = s ? static_cast<hipStream_t>(s) : m->own;
  return WT_OK;
}

int wt_mlp_get_params(wt_mlp* m, float* params_host) {
  if (!m || !params_host) return wt::api_fail(WT_EINVAL, "wt_mlp_get_params: null argument");
  try {
    HIPCHK(hipMemcpyAsync(params_host, m->dev.theta, wt::MLP_NP * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
  } catch (const std::exception& e) {
    return wt::api_fail(WT_EDEVICE, std::string("wt_mlp_get_params: ") + e.what());
  }
  return WT_OK;
}

int wt_mlp_forward(wt_mlp* m, const float* x, int64_t n, float* p) {
  if (!m || n < 0 || (n > 0 && (!x || !p))) return wt::api_fail(WT_EINVAL, "wt_mlp_forward: bad argument");
  try {
    m->dev.forward(x, n, p, m->stream);
  } catch (const std::exception& e) {
    return wt::api_fail(WT_EDEVICE, std::string("wt_mlp_forward: ") + e.what());
  }
  return WT_OK;
}

int wt_mlp_gradient(wt_mlp* m, const float* x, const float* y, int64_t n, float* grad_host, double* loss) {
  if (!m || n <= 0 || !x || !y) return wt::api_fail(WT_EINVAL, "wt_mlp_gradient: bad argument");
  try {
    m->dev.gradient(x, y, n, m->stream);
    std::vector<float> g(wt::MLP_NP + 1);
    HIPCHK(hipMemcpyAsync(g.data(), m->dev.grad, g.size() * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    if (grad_host) std::memcpy(grad_host, g.data(), wt::MLP_NP * sizeof(float));
    if (loss) *loss = double(g[wt::MLP_NP]) / (double(n) * wt::MLP_NO);
  } catch (const std::exception& e) {
    return wt::api_fail(WT_EDEVICE, std::string("wt_mlp_gradient: ") + e.what());
  }
  return WT_OK;
}

int wt_mlp_gradient_noalloc(wt_mlp* m, const float* x, const float* y, int64_t n, float* grad_device) {
  if (!m || n <= 0 || !x || !y || !grad_device) return wt::api_fail(WT_EINVAL, "wt_mlp_gradient_noalloc: bad argument");
  if (n > wt::MLP_NOALLOC_MAX)
    return wt::api_fail(WT_EINVAL, "wt_mlp_gradient_noalloc: at most " + std::to_string(wt::MLP_NOALLOC_MAX) +
                                       " samples per call");
  try {
    float* scr = wt::noalloc_scratch();
    if (wt::grad_scratch_floats(n) > wt::noalloc_scratch_floats())
      throw std::runtime_error("scratch array smaller than the sample bound");
    m->dev.gradient_into(x, y, n, scr, grad_device, m->stream);
  } catch (const std::exception& e) {
    return wt::api_fail(WT_EDEVICE, std::string("wt_mlp_gradient_noalloc: ") + e.what());
  }
  return WT_OK;
}

int wt_mlp_train_step(wt_mlp* m, const float* x, const float* y, int64_t n, double lr, double* loss) {
  if (!m || n <= 0 || !x || !y || !(lr > 0)) return wt::api_fail(WT_EINVAL, "wt_mlp_train_step: bad argument");
  try {
    m->dev.gradient(x, y, n, m->stream);
    if (loss) {
      float l = 0;
      HIPCHK(hipMemcpyAsync(&l, m->dev.grad + wt::MLP_NP, sizeof(float), hipMemcpyDeviceToHost, m->stream));
      HIPCHK(hipStreamSynchronize(m->stream));
      *loss = double(l) / (double(n) * wt::MLP_NO);
    }
    m->dev.adam(lr, m->stream);
  } catch (const std::exception& e) {
    return wt::api_fail(WT_EDEVICE, std::string("wt_mlp_train_step: ") + e.what());
  }
  return WT_OK;
}

}  // extern "C"
