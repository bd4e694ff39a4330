// Child-patch predictor network: parameter layout and device state.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace wt {

constexpr int MLP_NI = 64, MLP_NH = 128, MLP_NO = 4;
// flat parameter vector: W1 [64][128], b1 [128], W2 [128][128], b2 [128], W3 [128][4], b3 [4]
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_NI * MLP_NH;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_NH;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_NH * MLP_NH;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_NH;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_NH * MLP_NO;
constexpr int MLP_NP = MLP_OFF_B3 + MLP_NO;   // 25,348

// floats of scratch the gradient of n samples needs (per-tile contributions and group sums)
int64_t grad_scratch_floats(int64_t n);

// The allocation-free gradient: at most MLP_NOALLOC_MAX samples, scratch in a file-scope device
// array; noalloc_scratch() is its address on the current device (looked up once per device).
constexpr int64_t MLP_NOALLOC_MAX = 1024;
float* noalloc_scratch();
int64_t noalloc_scratch_floats();

struct MlpDev {
  float *theta = nullptr, *m = nullptr, *v = nullptr;   // FP32 master weights, Adam moments
  float* grad = nullptr;                                // last gradient (NP) and loss sum (entry NP)
  unsigned short* frag = nullptr;                       // bf16 operand fragments of the weights
  float* part = nullptr;                                // per-tile gradient contributions
  int64_t part_tiles = 0;
  int step = 0;                                         // Adam step count

  void alloc();
  void release();
  void pack(hipStream_t s);                             // fragments from theta
  // P[n][4] = sigmoid(network(X[n][64])), device arrays
  void forward(const float* X, int64_t n, float* P, hipStream_t s) const;
  // grad = d(mean BCE)/d theta on (X, Y), loss sum in grad[NP]
  void gradient(const float* X, const float* Y, int64_t n, hipStream_t s);
  // the same into out[NP + 1], with the caller's scratch of grad_scratch_floats(n) floats
  void gradient_into(const float* X, const float* Y, int64_t n, float* scratch, float* out, hipStream_t s) const;
  void adam(double lr, hipStream_t s);                  // one Adam step with grad, then pack
};

}  // namespace wt
