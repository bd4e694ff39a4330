// Child-patch predictor network of the learned adjacent zone: a 64-128-128-4 perceptron with
// ReLU hidden layers and sigmoid outputs, evaluated and trained on the matrix cores.
//
// Every matrix product runs on v_mfma_f32_16x16x16_bf16: bfloat16 operands (rounded to nearest
// even), FP32 accumulation.  One wavefront owns a tile of 16 samples and carries it through the
// whole network; hidden activations are re-laid out from the accumulator layout to the operand
// layout through LDS.  Weights are kept in FP32 (the master copy the optimiser updates) and
// re-packed after every update into bf16 operand fragments, so each lane fetches its 4 values of
// a B operand with one 8-byte load.  Training: the loss is the mean binary cross-entropy over
// samples and outputs; the per-tile gradients are written to scratch and summed in tile order
// (deterministic, no atomics), then one Adam step updates the master weights.
#include <hip/hip_runtime.h>

#include <mutex>

#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "wt_mlp.hpp"

namespace wt {

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int WAVES = 4;              // wavefronts (16-sample tiles) per workgroup
constexpr int TPB = 64 * WAVES;

// bf16 operand fragments: 64 lanes x 4 values per (tile, k-step); lane l supplies
// B[k = 16 s + 4 (l / 16) + v][j = 16 t + l % 16], v = 0..3.
constexpr int FRAG = 256;
constexpr int FR_W1 = 0;                       // W1 [64][128]:  8 column tiles x 4 k-steps
constexpr int FR_W2 = FR_W1 + 8 * 4 * FRAG;    // W2 [128][128]: 8 x 8
constexpr int FR_W3 = FR_W2 + 8 * 8 * FRAG;    // W3 [128][4]:   1 x 8 (columns 4..15 zero)
constexpr int FR_W2T = FR_W3 + 8 * FRAG;       // W2^T:          8 x 8
constexpr int FR_W3T = FR_W2T + 8 * 8 * FRAG;  // W3^T [4][128]: 8 x 1 (rows 4..15 zero)
constexpr int FR_TOTAL = FR_W3T + 8 * FRAG;

__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(unsigned(h) << 16); }

__device__ __forceinline__ v4s pack4(float a, float b, float c, float d) {
  v4s r;
  r[0] = (short)to_bf16(a);
  r[1] = (short)to_bf16(b);
  r[2] = (short)to_bf16(c);
  r[3] = (short)to_bf16(d);
  return r;
}

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ fragment packing
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ th, unsigned short* __restrict__ fr) {
  const int q = blockIdx.x * 256 + threadIdx.x;   // one (fragment, lane)
  if (q >= FR_TOTAL / 4) return;
  const int base = q * 4;
  const int lane = q % 64;
  const int kk = 4 * (lane / 16), jj = lane % 16;
  const float* W1 = th + MLP_OFF_W1;
  const float* W2 = th + MLP_OFF_W2;
  const float* W3 = th + MLP_OFF_W3;
  for (int v = 0; v < 4; ++v) {
    float x = 0.f;
    if (base < FR_W2) {
      const int f = (base - FR_W1) / FRAG, t = f / 4, s = f % 4;
      x = W1[(16 * s + kk + v) * MLP_NH + 16 * t + jj];
    } else if (base < FR_W3) {
      const int f = (base - FR_W2) / FRAG, t = f / 8, s = f % 8;
      x = W2[(16 * s + kk + v) * MLP_NH + 16 * t + jj];
    } else if (base < FR_W2T) {
      const int s = (base - FR_W3) / FRAG;
      x = jj < MLP_NO ? W3[(16 * s + kk + v) * MLP_NO + jj] : 0.f;
    } else if (base < FR_W3T) {
      const int f = (base - FR_W2T) / FRAG, t = f / 8, s = f % 8;
      x = W2[(16 * t + jj) * MLP_NH + 16 * s + kk + v];
    } else {
      const int t = (base - FR_W3T) / FRAG;
      x = (kk + v) < MLP_NO ? W3[(16 * t + jj) * MLP_NO + kk + v] : 0.f;
    }
    fr[base + v] = to_bf16(x);
  }
}

__device__ __forceinline__ v4s frag(const unsigned short* __restrict__ fr, int off, int lane) {
  const uint2 w = *reinterpret_cast<const uint2*>(fr + off + 4 * lane);
  v4s r;
  r[0] = (short)(w.x & 0xFFFFu);
  r[1] = (short)(w.x >> 16);
  r[2] = (short)(w.y & 0xFFFFu);
  r[3] = (short)(w.y >> 16);
  return r;
}

// ------------------------------------------------------------------ forward of one 16-sample tile
// Leaves relu(h1), relu(h2) (FP32) in the wave's LDS rows and returns the logits in accumulator
// layout: z[v] = logit of sample 4 (lane / 16) + v, output lane % 16 (valid for lane % 16 < 4).
__device__ __forceinline__ v4f tile_forward(const float* __restrict__ X, int64_t n, int64_t r0,
                                            const float* __restrict__ th, const unsigned short* __restrict__ fr,
                                            float (*h1)[MLP_NH], float (*h2)[MLP_NH], int lane) {
  const int lr = lane % 16, lq = lane / 16;
  // layer 1
  v4f acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  const int64_t row = r0 + lr;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f;
    if (row < n) {
      const float4 xv = *reinterpret_cast<const float4*>(X + row * MLP_NI + 16 * s + 4 * lq);
      x0 = xv.x; x1 = xv.y; x2 = xv.z; x3 = xv.w;
    }
    const v4s a = pack4(x0, x1, x2, x3);
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = mfma(a, frag(fr, FR_W1 + (t * 4 + s) * FRAG, 0), acc[t]);
  }
  const float* b1 = th + MLP_OFF_B1;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) h1[4 * lq + v][16 * t + lr] = fmaxf(acc[t][v] + b1[16 * t + lr], 0.f);
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS writes are visible to it
  __builtin_amdgcn_wave_barrier();
  // layer 2
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const float* hr = &h1[lr][16 * s + 4 * lq];
    const v4s a = pack4(hr[0], hr[1], hr[2], hr[3]);
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = mfma(a, frag(fr, FR_W2 + (t * 8 + s) * FRAG, 0), acc[t]);
  }
  const float* b2 = th + MLP_OFF_B2;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) h2[4 * lq + v][16 * t + lr] = fmaxf(acc[t][v] + b2[16 * t + lr], 0.f);
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  // layer 3
  v4f z = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const float* hr = &h2[lr][16 * s + 4 * lq];
    z = mfma(pack4(hr[0], hr[1], hr[2], hr[3]), frag(fr, FR_W3 + s * FRAG, 0), z);
  }
  const float b3 = lr < MLP_NO ? th[MLP_OFF_B3 + lr] : 0.f;
#pragma unroll
  for (int v = 0; v < 4; ++v) z[v] += b3;
  return z;
}

__device__ __forceinline__ float sigmoidf_(float z) { return 1.f / (1.f + expf(-z)); }

__global__ __launch_bounds__(TPB) void k_forward(const float* __restrict__ X, int64_t n,
                                                 const float* __restrict__ th,
                                                 const unsigned short* __restrict__ fr, float* __restrict__ P) {
  __shared__ float s_h1[WAVES][16][MLP_NH], s_h2[WAVES][16][MLP_NH];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t r0 = (int64_t(blockIdx.x) * WAVES + w) * 16;
  if (r0 >= n) return;   // uniform per wavefront; no workgroup barrier follows
  // operand fragments are read with the lane folded into the offset
  const unsigned short* frl = fr + 4 * lane;
  const v4f z = tile_forward(X, n, r0, th, frl, s_h1[w], s_h2[w], lane);
  const int lr = lane % 16, lq = lane / 16;
  if (lr < MLP_NO)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * lq + v;
      if (row < n) P[row * MLP_NO + lr] = sigmoidf_(z[v]);
    }
}

// ------------------------------------------------------------------ gradient of one tile
// Writes the tile's gradient contribution (NP values, the layout of the parameter vector) and
// its summed loss to part[tile * (NP + 1) ...].
__global__ __launch_bounds__(TPB) void k_grad_tiles(const float* __restrict__ X, const float* __restrict__ Y,
                                                    int64_t n, const float* __restrict__ th,
                                                    const unsigned short* __restrict__ fr,
                                                    float* __restrict__ part) {
  __shared__ float s_h1[WAVES][16][MLP_NH], s_h2[WAVES][16][MLP_NH], s_d[WAVES][16][MLP_NH];
  __shared__ float s_dz[WAVES][16][MLP_NO];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t tile = int64_t(blockIdx.x) * WAVES + w;
  const int64_t r0 = tile * 16;
  if (r0 >= n) return;
  const int lr = lane % 16, lq = lane / 16;
  const unsigned short* frl = fr + 4 * lane;
  float(*h1)[MLP_NH] = s_h1[w];
  float(*h2)[MLP_NH] = s_h2[w];
  float(*dd)[MLP_NH] = s_d[w];
  float(*dz)[MLP_NO] = s_dz[w];
  float* out = part + tile * (MLP_NP + 1);
  const v4f z = tile_forward(X, n, r0, th, frl, h1, h2, lane);

  // output error dz = (sigmoid(z) - y) / (4 n), loss terms softplus(z) - y z
  const float inv = 1.f / (float(n) * MLP_NO);
  float lsum = 0.f;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = r0 + 4 * lq + v;
    if (lr < MLP_NO) {
      float e = 0.f;
      if (row < n) {
        const float y = Y[row * MLP_NO + lr], zz = z[v];
        e = (sigmoidf_(zz) - y) * inv;
        lsum += fmaxf(zz, 0.f) + log1pf(expf(-fabsf(zz))) - y * zz;
      }
      dz[4 * lq + v][lr] = e;
    }
  }
  // rows of the tile beyond n carry zero error; their activations do not matter
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  // wave sum of the loss
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
  if (lane == 0) out[MLP_NP] = lsum;
  // b3 gradient: column sums of dz (FP32, not rounded)
  if (lane < MLP_NO) {
    float s = 0.f;
    for (int r = 0; r < 16; ++r) s += dz[r][lane];
    out[MLP_OFF_B3 + lane] = s;
  }
  // W3 gradient = h2^T dz : M = 128 (8 tiles), N = 16 (4 used), K = 16 samples
  {
    const v4s b = pack4(lr < MLP_NO ? dz[4 * lq + 0][lr] : 0.f, lr < MLP_NO ? dz[4 * lq + 1][lr] : 0.f,
                        lr < MLP_NO ? dz[4 * lq + 2][lr] : 0.f, lr < MLP_NO ? dz[4 * lq + 3][lr] : 0.f);
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
      const int i = 16 * mt + lr;
      const v4s a = pack4(h2[4 * lq + 0][i], h2[4 * lq + 1][i], h2[4 * lq + 2][i], h2[4 * lq + 3][i]);
      const v4f g = mfma(a, b, v4f{0.f, 0.f, 0.f, 0.f});
      if (lr < MLP_NO)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[MLP_OFF_W3 + (16 * mt + 4 * lq + v) * MLP_NO + lr] = g[v];
    }
  }
  // dh2 = (dz W3^T) * [h2 > 0] : M = 16 samples, N = 128 (8 tiles), K = 16 (4 outputs used)
  {
    const v4s a = pack4(lq == 0 ? dz[lr][0] : 0.f, lq == 0 ? dz[lr][1] : 0.f, lq == 0 ? dz[lr][2] : 0.f,
                        lq == 0 ? dz[lr][3] : 0.f);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const v4f g = mfma(a, frag(frl, FR_W3T + t * FRAG, 0), v4f{0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * lq + v, c = 16 * t + lr;
        dd[r][c] = h2[r][c] > 0.f ? g[v] : 0.f;
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  // b2 gradient: column sums of dh2; W2 gradient = h1^T dh2 (M = 128, N = 128, K = 16)
  for (int c = lane; c < MLP_NH; c += 64) {
    float s = 0.f;
    for (int r = 0; r < 16; ++r) s += dd[r][c];
    out[MLP_OFF_B2 + c] = s;
  }
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    const int j = 16 * nt + lr;
    const v4s b = pack4(dd[4 * lq + 0][j], dd[4 * lq + 1][j], dd[4 * lq + 2][j], dd[4 * lq + 3][j]);
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
      const int i = 16 * mt + lr;
      const v4s a = pack4(h1[4 * lq + 0][i], h1[4 * lq + 1][i], h1[4 * lq + 2][i], h1[4 * lq + 3][i]);
      const v4f g = mfma(a, b, v4f{0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int v = 0; v < 4; ++v) out[MLP_OFF_W2 + (16 * mt + 4 * lq + v) * MLP_NH + 16 * nt + lr] = g[v];
    }
  }
  // dh1 = (dh2 W2^T) * [h1 > 0] : M = 16, N = 128, K = 128; kept in registers, then LDS
  v4f acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const float* dr = &dd[lr][16 * s + 4 * lq];
    const v4s a = pack4(dr[0], dr[1], dr[2], dr[3]);
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = mfma(a, frag(frl, FR_W2T + (t * 8 + s) * FRAG, 0), acc[t]);
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();   // all reads of dh2 done before it is overwritten
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * lq + v, c = 16 * t + lr;
      dd[r][c] = h1[r][c] > 0.f ? acc[t][v] : 0.f;
    }
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  // b1 gradient; W1 gradient = x^T dh1 (M = 64, 4 tiles; N = 128; K = 16)
  for (int c = lane; c < MLP_NH; c += 64) {
    float s = 0.f;
    for (int r = 0; r < 16; ++r) s += dd[r][c];
    out[MLP_OFF_B1 + c] = s;
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int i = 16 * mt + lr;   // input feature
    float xa[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * lq + v;
      xa[v] = row < n ? X[row * MLP_NI + i] : 0.f;
    }
    const v4s a = pack4(xa[0], xa[1], xa[2], xa[3]);
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
      const int j = 16 * nt + lr;
      const v4s b = pack4(dd[4 * lq + 0][j], dd[4 * lq + 1][j], dd[4 * lq + 2][j], dd[4 * lq + 3][j]);
      const v4f g = mfma(a, b, v4f{0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int v = 0; v < 4; ++v) out[MLP_OFF_W1 + (16 * mt + 4 * lq + v) * MLP_NH + 16 * nt + lr] = g[v];
    }
  }
}

// Sum of the tile contributions in a fixed order (the loss sum is entry NP): groups of
// SUM_GROUP consecutive tiles first, then the groups.
constexpr int SUM_GROUP = 64;
__global__ __launch_bounds__(256) void k_sum_tiles(const float* __restrict__ part, int64_t ntile,
                                                   float* __restrict__ out) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q > MLP_NP) return;
  const int64_t t0 = int64_t(blockIdx.y) * SUM_GROUP, t1 = t0 + SUM_GROUP < ntile ? t0 + SUM_GROUP : ntile;
  float s = 0.f;
  for (int64_t t = t0; t < t1; ++t) s += part[t * (MLP_NP + 1) + q];
  out[int64_t(blockIdx.y) * (MLP_NP + 1) + q] = s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, float lr, float c1, float c2) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= MLP_NP) return;
  const float gq = g[q];
  const float mq = 0.9f * m[q] + 0.1f * gq;
  const float vq = 0.999f * v[q] + 0.001f * gq * gq;
  m[q] = mq;
  v[q] = vq;
  th[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + 1e-8f);
}

// ------------------------------------------------------------------ allocation-free gradient
// Scratch of wt_mlp_gradient_noalloc: the per-tile contributions and group sums of up to
// MLP_NOALLOC_MAX samples in a file-scope device array (6.6 MB per GPU, held until the process
// ends).  Host code never passes the array's name to a kernel (in host code it is only a stand-in
// for the symbol): its device address is looked up once per device with hipGetSymbolAddress and
// that address is used instead.
static __device__ __align__(256) float scratch[(MLP_NOALLOC_MAX / 16 + (MLP_NOALLOC_MAX / 16 + SUM_GROUP - 1) / SUM_GROUP) *
                                             (MLP_NP + 1)];
static_assert(MLP_NOALLOC_MAX % 16 == 0, "whole tiles");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

float* noalloc_scratch() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw std::runtime_error("noalloc scratch: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    float* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch)));
    if (!ptr) throw std::runtime_error("noalloc scratch: no device address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

int64_t noalloc_scratch_floats() { return int64_t(sizeof(scratch) / sizeof(float)); }

// ------------------------------------------------------------------ host side
void MlpDev::alloc() {
  HIPCHK(hipMalloc(&theta, MLP_NP * sizeof(float)));
  HIPCHK(hipMalloc(&m, MLP_NP * sizeof(float)));
  HIPCHK(hipMalloc(&v, MLP_NP * sizeof(float)));
  HIPCHK(hipMalloc(&grad, (MLP_NP + 1) * sizeof(float)));
  HIPCHK(hipMalloc(&frag, FR_TOTAL * sizeof(unsigned short)));
  HIPCHK(hipMemset(m, 0, MLP_NP * sizeof(float)));
  HIPCHK(hipMemset(v, 0, MLP_NP * sizeof(float)));
  step = 0;
}

void MlpDev::release() {
  void* ps[] = {theta, m, v, grad, frag, part};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  theta = m = v = grad = part = nullptr;
  frag = nullptr;
  part_tiles = 0;
}

void MlpDev::pack(hipStream_t s) {
  k_pack<<<(FR_TOTAL / 4 + 255) / 256, 256, 0, s>>>(theta, frag);
  HIPCHK(hipGetLastError());
}

void MlpDev::forward(const float* X, int64_t n, float* P, hipStream_t s) const {
  if (n <= 0) return;
  const int64_t tiles = (n + 15) / 16;
  k_forward<<<unsigned((tiles + WAVES - 1) / WAVES), TPB, 0, s>>>(X, n, theta, frag, P);
  HIPCHK(hipGetLastError());
}

int64_t grad_scratch_floats(int64_t n) {
  // tile contributions, then one row per group of tiles
  const int64_t tiles = (n + 15) / 16;
  return (tiles + (tiles + SUM_GROUP - 1) / SUM_GROUP) * (MLP_NP + 1);
}

void MlpDev::gradient_into(const float* X, const float* Y, int64_t n, float* scratch, float* out,
                           hipStream_t s) const {
  const int64_t tiles = (n + 15) / 16;
  // every entry of the scratch rows is written before it is read: no clearing
  k_grad_tiles<<<unsigned((tiles + WAVES - 1) / WAVES), TPB, 0, s>>>(X, Y, n, theta, frag, scratch);
  // group sums go to their own rows after the tile rows
  const int64_t groups = (tiles + SUM_GROUP - 1) / SUM_GROUP;
  float* gsum = scratch + tiles * (MLP_NP + 1);
  k_sum_tiles<<<dim3((MLP_NP + 1 + 255) / 256, unsigned(groups)), 256, 0, s>>>(scratch, tiles, gsum);
  k_sum_tiles<<<dim3((MLP_NP + 1 + 255) / 256, 1), 256, 0, s>>>(gsum, groups, out);
  HIPCHK(hipGetLastError());
}

void MlpDev::gradient(const float* X, const float* Y, int64_t n, hipStream_t s) {
  const int64_t tiles = (n + 15) / 16;
  if (tiles > part_tiles) {
    if (part) HIPCHK(hipFree(part));
    HIPCHK(hipMalloc(&part, grad_scratch_floats(n) * sizeof(float)));
    part_tiles = tiles;
  }
  gradient_into(X, Y, n, part, grad, s);
}

void MlpDev::adam(double lr, hipStream_t s) {
  ++step;
  const float c1 = float(1.0 - std::pow(0.9, step)), c2 = float(1.0 - std::pow(0.999, step));
  k_adam<<<(MLP_NP + 255) / 256, 256, 0, s>>>(theta, m, v, grad, float(lr), c1, c2);
  HIPCHK(hipGetLastError());
  pack(s);
}

}  // namespace wt
