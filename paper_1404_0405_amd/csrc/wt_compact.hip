// Work lists of the adaptive stage: stream compaction of byte predicates into index lists by
// wavefront ballot and prefix scan, and the predicates themselves (support rings of the active
// points, and the coarse entities of a level pair whose fine points lie in the support).
//
// Compaction is three launches: per-chunk counts (ballot + popcount), one workgroup scanning the
// chunk counts, and the scatter, where every lane finds its slot from the popcount of the ballot
// bits below it plus the chunk offset.  The output is in increasing index order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "wt_alloc.hpp"
#include "wt_compact.hpp"

namespace wt {

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(e_) + " at " #x); \
  } while (0)

constexpr int CB = 256;              // threads per workgroup
constexpr int CITEMS = 8;            // items per thread
constexpr int CHUNK = CB * CITEMS;   // indices per workgroup
constexpr int NWAVE = CB / 64;

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ unsigned long long lanes_below() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__global__ __launch_bounds__(CB) void k_count(const uint8_t* __restrict__ pred, int64_t n, int32_t* __restrict__ cnt) {
  __shared__ int s_w[NWAVE];
  const int64_t base = int64_t(blockIdx.x) * CHUNK;
  int c = 0;
#pragma unroll
  for (int it = 0; it < CITEMS; ++it) {
    const int64_t i = base + it * CB + threadIdx.x;
    const bool p = i < n && pred[i] != 0;
    c += __popcll(ballot(p));   // every lane holds the wave's count
  }
  if (lane_id() == 0) s_w[threadIdx.x / 64] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < NWAVE; ++w) t += s_w[w];
    cnt[blockIdx.x] = t;
  }
}

// Exclusive scan of the chunk counts by one workgroup; off[nchunk] = total.
__global__ __launch_bounds__(CB) void k_scan(const int32_t* __restrict__ cnt, int64_t nchunk, int64_t* __restrict__ off) {
  __shared__ int64_t s_sum[CB];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nchunk; b0 += CB) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t v = b < nchunk ? cnt[b] : 0;
    s_sum[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < CB; o <<= 1) {   // inclusive Hillis-Steele scan
      const int64_t a = threadIdx.x >= o ? s_sum[threadIdx.x - o] : 0;
      __syncthreads();
      s_sum[threadIdx.x] += a;
      __syncthreads();
    }
    if (b < nchunk) off[b] = carry + s_sum[threadIdx.x] - v;
    carry += s_sum[CB - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) off[nchunk] = carry;
}

__global__ __launch_bounds__(CB) void k_scatter(const uint8_t* __restrict__ pred, int64_t n,
                                                const int64_t* __restrict__ off, int32_t* __restrict__ out) {
  __shared__ int s_w[NWAVE];
  const int64_t base = int64_t(blockIdx.x) * CHUNK;
  int64_t slot = off[blockIdx.x];
  const int w = threadIdx.x / 64;
  for (int it = 0; it < CITEMS; ++it) {
    const int64_t i = base + it * CB + threadIdx.x;
    const bool p = i < n && pred[i] != 0;
    const unsigned long long m = ballot(p);
    if (lane_id() == 0) s_w[w] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
    for (int q = 0; q < NWAVE; ++q) {
      before += q < w ? s_w[q] : 0;
      total += s_w[q];
    }
    if (p) out[slot + before + __popcll(m & lanes_below())] = int32_t(i);
    slot += total;
    __syncthreads();
  }
}

__global__ void k_store_total(const int64_t* __restrict__ off, int64_t nchunk, int64_t* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = off[nchunk];
}

void compact(const uint8_t* pred, int64_t n, WorkList& L, CompactScratch& sc, hipStream_t s, int64_t* total_dev) {
  const int64_t nchunk = (n + CHUNK - 1) / CHUNK;
  if (nchunk + 1 > sc.cap) {
    // the previous scratch may still be read by queued work of this stream
    HIPCHK(hipStreamSynchronize(s));
    if (sc.cnt) HIPCHK(wt::dfree(sc.cnt));
    if (sc.off) HIPCHK(wt::dfree(sc.off));
    sc.cap = nchunk + 1;
    HIPCHK(wt::dmalloc(&sc.cnt, sc.cap * sizeof(int32_t)));
    HIPCHK(wt::dmalloc(&sc.off, sc.cap * sizeof(int64_t)));
  }
  if (!L.idx || L.cap < n) {
    if (L.idx) HIPCHK(wt::dfree(L.idx));
    L.cap = n > 0 ? n : 1;
    HIPCHK(wt::dmalloc(&L.idx, L.cap * sizeof(int32_t)));
  }
  if (n == 0) {
    L.n = 0;
    L.bound = 0;
    if (total_dev) HIPCHK(hipMemsetAsync(total_dev, 0, sizeof(int64_t), s));
    return;
  }
  k_count<<<unsigned(nchunk), CB, 0, s>>>(pred, n, sc.cnt);
  k_scan<<<1, CB, 0, s>>>(sc.cnt, nchunk, sc.off);
  k_scatter<<<unsigned(nchunk), CB, 0, s>>>(pred, n, sc.off, L.idx);
  HIPCHK(hipGetLastError());
  if (total_dev) {
    // the count stays on the device; the caller reads all counts of a batch at once
    k_store_total<<<1, 64, 0, s>>>(sc.off, nchunk, total_dev);
    HIPCHK(hipGetLastError());
    return;
  }
  int64_t total = 0;
  HIPCHK(hipMemcpyAsync(&total, sc.off + nchunk, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  L.n = total;
  L.bound = total;
}

// ------------------------------------------------------------------ batched compaction
// Several predicate arrays compacted by three launches: chunk counts of every job, one workgroup
// per job scanning its chunk counts, and the scatter.  A chunk finds its job by binary search
// over the jobs' first chunks.
struct CJob {
  const uint8_t* pred;
  int64_t n;
  int32_t* out;
  int64_t chunk0;
  int64_t* dn;   // the list's device count
};

__device__ __forceinline__ int job_of(const CJob* __restrict__ jobs, int njob, int64_t chunk) {
  int lo = 0, hi = njob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (jobs[mid].chunk0 <= chunk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(CB) void k_count_b(const CJob* __restrict__ jobs, int njob, int32_t* __restrict__ cnt) {
  __shared__ int s_w[NWAVE];
  const int64_t chunk = blockIdx.x;
  const CJob J = jobs[job_of(jobs, njob, chunk)];
  const int64_t base = (chunk - J.chunk0) * CHUNK;
  int c = 0;
#pragma unroll
  for (int it = 0; it < CITEMS; ++it) {
    const int64_t i = base + it * CB + threadIdx.x;
    c += __popcll(ballot(i < J.n && J.pred[i] != 0));
  }
  if (lane_id() == 0) s_w[threadIdx.x / 64] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < NWAVE; ++w) t += s_w[w];
    cnt[chunk] = t;
  }
}

__global__ __launch_bounds__(CB) void k_scan_b(const CJob* __restrict__ jobs, int njob, int64_t nchunk_total,
                                               const int32_t* __restrict__ cnt, int64_t* __restrict__ off,
                                               int64_t* __restrict__ totals) {
  __shared__ int64_t s_sum[CB];
  const int k = blockIdx.x;
  const int64_t c0 = jobs[k].chunk0, c1 = k + 1 < njob ? jobs[k + 1].chunk0 : nchunk_total;
  int64_t carry = 0;
  for (int64_t b0 = c0; b0 < c1; b0 += CB) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t v = b < c1 ? cnt[b] : 0;
    s_sum[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < CB; o <<= 1) {
      const int64_t a = threadIdx.x >= o ? s_sum[threadIdx.x - o] : 0;
      __syncthreads();
      s_sum[threadIdx.x] += a;
      __syncthreads();
    }
    if (b < c1) off[b] = carry + s_sum[threadIdx.x] - v;
    carry += s_sum[CB - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    totals[k] = carry;
    *jobs[k].dn = carry;
  }
}

__global__ __launch_bounds__(CB) void k_scatter_b(const CJob* __restrict__ jobs, int njob,
                                                  const int64_t* __restrict__ off) {
  __shared__ int s_w[NWAVE];
  const int64_t chunk = blockIdx.x;
  const CJob J = jobs[job_of(jobs, njob, chunk)];
  const int64_t base = (chunk - J.chunk0) * CHUNK;
  int64_t slot = off[chunk];
  const int w = threadIdx.x / 64;
  for (int it = 0; it < CITEMS; ++it) {
    const int64_t i = base + it * CB + threadIdx.x;
    const bool p = i < J.n && J.pred[i] != 0;
    const unsigned long long m = ballot(p);
    if (lane_id() == 0) s_w[w] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
    for (int q = 0; q < NWAVE; ++q) {
      before += q < w ? s_w[q] : 0;
      total += s_w[q];
    }
    if (p) J.out[slot + before + __popcll(m & lanes_below())] = int32_t(i);
    slot += total;
    __syncthreads();
  }
}

// -1 over idx[from, to) of up to PAD_JOBS lists (blockIdx.y = list)
constexpr int PAD_JOBS = 64;
struct PadJob {
  int32_t* idx;
  int64_t from, to;
};
struct PadJobs {
  PadJob j[PAD_JOBS];
};
__global__ __launch_bounds__(CB) void k_pad_b(PadJobs J) {
  const PadJob jb = J.j[blockIdx.y];
  for (int64_t i = jb.from + int64_t(blockIdx.x) * CB + threadIdx.x; i < jb.to; i += int64_t(gridDim.x) * CB)
    jb.idx[i] = -1;
}

// The padded bound of a list of n entries: 0 for an empty list (nothing is launched); kept while
// n <= bound <= 8 max(n, 256); otherwise the power of two at or above 2 max(n, 256) (capped by
// cap), so small drifts of n between adapts do not change the launches.
static int64_t list_bound(int64_t prev, int64_t n, int64_t cap) {
  if (n == 0) return 0;
  const int64_t m = n > 256 ? n : 256;
  if (prev >= n && prev <= cap && prev <= 8 * m) return prev;
  int64_t b = 256;
  while (b < 2 * m) b <<= 1;
  return b < cap ? b : cap;
}

void CompactBatch::add(const uint8_t* pred, int64_t n, WorkList& L) {
  if (!L.idx || L.cap < n) {
    // the list may still be read by queued work: let it drain before freeing
    if (L.idx) {
      HIPCHK(hipDeviceSynchronize());
      HIPCHK(wt::dfree(L.idx));
    }
    L.cap = n > 0 ? n : 1;
    HIPCHK(wt::dmalloc(&L.idx, L.cap * sizeof(int32_t)));
  }
  if (!L.dn) HIPCHK(wt::dmalloc(&L.dn, sizeof(int64_t)));
  jobs.push_back(Job{pred, n, &L});
}

void CompactBatch::run(hipStream_t s) {
  const int njob = int(jobs.size());
  if (njob == 0) return;
  std::vector<CJob> cj(njob);
  int64_t nchunk = 0;
  for (int k = 0; k < njob; ++k) {
    cj[k] = CJob{jobs[k].pred, jobs[k].n, jobs[k].list->idx, nchunk, jobs[k].list->dn};
    nchunk += std::max<int64_t>(1, (jobs[k].n + CHUNK - 1) / CHUNK);   // every job owns a chunk
  }
  if (njob > job_cap || nchunk > chunk_cap) {
    HIPCHK(hipStreamSynchronize(s));
    release();
    uploaded.clear();
    job_cap = std::max(njob, 64);
    chunk_cap = std::max<int64_t>(nchunk, 1024);
    HIPCHK(wt::dmalloc(&d_jobs, job_cap * sizeof(CJob)));
    HIPCHK(hipHostMalloc(&h_jobs, job_cap * sizeof(CJob), hipHostMallocDefault));
    HIPCHK(wt::dmalloc(&d_cnt, chunk_cap * sizeof(int32_t)));
    HIPCHK(wt::dmalloc(&d_off, chunk_cap * sizeof(int64_t)));
    HIPCHK(wt::dmalloc(&d_tot, job_cap * sizeof(int64_t)));
    HIPCHK(hipHostMalloc(&h_tot, job_cap * sizeof(int64_t), hipHostMallocDefault));
  }
  // the device keeps the job table of the last batch: an unchanged table (the usual case, the
  // same predicates into the same lists) is not uploaded again
  const unsigned char* cb = reinterpret_cast<const unsigned char*>(cj.data());
  const size_t nbytes = njob * sizeof(CJob);
  if (uploaded.size() != nbytes || std::memcmp(uploaded.data(), cb, nbytes) != 0) {
    // the pinned staging buffer may still feed a queued copy of the previous batch
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(h_jobs, cj.data(), nbytes);
    HIPCHK(hipMemcpyAsync(d_jobs, h_jobs, nbytes, hipMemcpyHostToDevice, s));
    uploaded.assign(cb, cb + nbytes);
  }
  const CJob* J = static_cast<const CJob*>(d_jobs);
  k_count_b<<<unsigned(nchunk), CB, 0, s>>>(J, njob, d_cnt);
  k_scan_b<<<unsigned(njob), CB, 0, s>>>(J, njob, nchunk, d_cnt, d_off, d_tot);
  k_scatter_b<<<unsigned(nchunk), CB, 0, s>>>(J, njob, d_off);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h_tot, d_tot, njob * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<PadJob> pads;
  for (int k = 0; k < njob; ++k) {
    WorkList& L = *jobs[k].list;
    L.n = h_tot[k];
    L.bound = list_bound(L.bound, L.n, L.cap);
    if (L.bound > L.n) pads.push_back(PadJob{L.idx, L.n, L.bound});
  }
  for (size_t k0 = 0; k0 < pads.size(); k0 += PAD_JOBS) {
    PadJobs J{};
    const size_t nk = std::min<size_t>(PAD_JOBS, pads.size() - k0);
    for (size_t k = 0; k < nk; ++k) J.j[k] = pads[k0 + k];
    k_pad_b<<<dim3(8, unsigned(nk)), CB, 0, s>>>(J);
    HIPCHK(hipGetLastError());
  }
  jobs.clear();
}

void CompactBatch::release() {
  void* dv[] = {d_jobs, d_cnt, d_off, d_tot};
  for (void* p : dv)
    if (p) (void)wt::dfree(p);
  if (h_jobs) (void)hipHostFree(h_jobs);
  if (h_tot) (void)hipHostFree(h_tot);
  d_jobs = nullptr;
  d_cnt = nullptr;
  d_off = nullptr;
  d_tot = nullptr;
  h_jobs = nullptr;
  h_tot = nullptr;
  job_cap = 0;
  chunk_cap = 0;
}

void free_list(WorkList& L) {
  if (L.idx) (void)wt::dfree(L.idx);
  if (L.dn) (void)wt::dfree(L.dn);
  L = WorkList{};
}

void free_scratch(CompactScratch& sc) {
  if (sc.cnt) (void)wt::dfree(sc.cnt);
  if (sc.off) (void)wt::dfree(sc.off);
  sc = CompactScratch{};
}

// ------------------------------------------------------------------ predicates
#define TIDX (int64_t(blockIdx.x) * CB + threadIdx.x)
static inline unsigned nbk(int64_t n) { return unsigned((n + CB - 1) / CB); }

// The predicates of several levels and pairs in one launch: blockIdx.y picks the job, whose
// entities the row's blocks cover with a grid-stride loop: triangles with an edge in the edge
// support; elements (node + the 3 edges it owns; poles own none) with a point in the support;
// coarse nodes, edges and triangles of a pair whose fine points lie in the fine support.  The lattice gives the edges of a
// triangle away from the lozenge's last row and column, and the fine copies, midpoints and
// half-edges of every coarse node and edge, by index arithmetic (canonical numbering: element
// (L,i,j) -> (L n + i) n + j, edges 3 id + d, triangles 2 id + t, poles last), so those tables are
// not read; the other triangles and the interior edges of coarse triangles use the tables.
__global__ __launch_bounds__(CB) void k_pred_b(PredJobs J) {
  const PredJob& jb = J.j[blockIdx.y];
  const int64_t stride = int64_t(gridDim.x) * CB;
  if (jb.kind == PRED_TRI) {
    const int sh = jb.sh;
    const int64_t n = int64_t(1) << sh, mk = n - 1;
    for (int64_t t = TIDX; t < jb.n; t += stride) {
      const int64_t id = t >> 1;
      const int64_t i = (id >> sh) & mk, j = id & mk;
      int64_t e0, e1, e2;
      if (i < n - 1 && j < n - 1) {
        if ((t & 1) == 0) {   // ((i,j), (i+1,j), (i+1,j+1))
          e0 = 3 * id; e1 = 3 * (id + n) + 2; e2 = 3 * id + 1;
        } else {              // ((i,j), (i+1,j+1), (i,j+1))
          e0 = 3 * id + 1; e1 = 3 * (id + 1); e2 = 3 * id + 2;
        }
      } else {
        e0 = jb.a[3 * t]; e1 = jb.a[3 * t + 1]; e2 = jb.a[3 * t + 2];
      }
      jb.o1[t] = (jb.se[e0] | jb.se[e1] | jb.se[e2]) ? 1 : 0;
    }
  } else if (jb.kind == PRED_ELEM) {
    for (int64_t i = TIDX; i < jb.n; i += stride) {
      bool p = jb.sn[i] != 0;
      if (i < jb.n_elem) p = p || jb.se[3 * i] || jb.se[3 * i + 1] || jb.se[3 * i + 2];
      jb.o1[i] = p ? 1 : 0;
    }
  } else {
    const int shc = jb.sh;
    const int64_t nc = int64_t(1) << shc, mk = nc - 1, nf = 2 * nc, lat = 10 * nc * nc;
    for (int64_t k = TIDX; k < jb.n; k += stride) {
      if (k < jb.Nc) {
        const int64_t f = k < lat ? (((k >> (2 * shc)) * nf + 2 * ((k >> shc) & mk)) * nf + 2 * (k & mk))
                                  : 10 * nf * nf + (k - lat);
        jb.o1[k] = jb.sn[f] ? 1 : 0;
      }
      if (k < jb.Ec) {
        const int64_t id = k / 3;
        const int d = int(k - 3 * id);
        const int64_t L = id >> (2 * shc), i = (id >> shc) & mk, j = id & mk;
        const int64_t f0 = (L * nf + 2 * i) * nf + 2 * j;
        const int64_t fm = (L * nf + 2 * i + (d < 2 ? 1 : 0)) * nf + 2 * j + (d > 0 ? 1 : 0);
        jb.o2[k] = (jb.sn[fm] | jb.se[3 * f0 + d] | jb.se[3 * fm + d]) ? 1 : 0;
      }
      if (k < jb.Tc) jb.o3[k] = (jb.se[jb.e[3 * k]] | jb.se[jb.e[3 * k + 1]] | jb.se[jb.e[3 * k + 2]]) ? 1 : 0;
    }
  }
}

PredJob pred_tri_job(int64_t T, int sh, const int32_t* t_e, const uint8_t* se, uint8_t* pt) {
  if (T != 20 * (int64_t(1) << (2 * sh))) throw std::runtime_error("pred_tri_job: triangle count does not match 2^sh");
  PredJob j{};
  j.kind = PRED_TRI; j.sh = sh; j.n = T; j.a = t_e; j.se = se; j.o1 = pt;
  return j;
}

PredJob pred_elem_job(int64_t N, int64_t n_elem, const uint8_t* sn, const uint8_t* se, uint8_t* pe) {
  PredJob j{};
  j.kind = PRED_ELEM; j.n = N; j.n_elem = n_elem; j.sn = sn; j.se = se; j.o1 = pe;
  return j;
}

PredJob pred_pair_job(const DevPair& P, int shc, const uint8_t* snf, const uint8_t* sef, uint8_t* pn,
                      uint8_t* pe, uint8_t* pt) {
  const int64_t nc = int64_t(1) << shc;
  if (P.Ec != 30 * nc * nc || P.Nc != 10 * nc * nc + 2 || P.Nf != 40 * nc * nc + 2)
    throw std::runtime_error("pred_pair_job: pair sizes do not match 2^shc");
  PredJob j{};
  j.kind = PRED_PAIR;
  j.sh = shc;
  j.Nc = P.Nc; j.Ec = P.Ec; j.Tc = P.Tc;
  j.n = P.Nc > P.Ec ? P.Nc : P.Ec;
  if (P.Tc > j.n) j.n = P.Tc;
  j.a = P.even; j.b = P.mid; j.c = P.h1; j.d = P.h2; j.e = P.int_e;
  j.sn = snf; j.se = sef; j.o1 = pn; j.o2 = pe; j.o3 = pt;
  return j;
}

void pred_batch(const PredJob* jobs, int njobs, hipStream_t s) {
  for (int k0 = 0; k0 < njobs; k0 += MAX_PRED_JOBS) {
    PredJobs J{};
    const int nk = njobs - k0 < MAX_PRED_JOBS ? njobs - k0 : MAX_PRED_JOBS;
    int64_t m = 1;
    for (int k = 0; k < nk; ++k) {
      J.j[k] = jobs[k0 + k];
      if (J.j[k].n > m) m = J.j[k].n;
    }
    const unsigned grid = nbk(m) < 4096u ? nbk(m) : 4096u;
    k_pred_b<<<dim3(grid, nk), CB, 0, s>>>(J);
    HIPCHK(hipGetLastError());
  }
}

}  // namespace wt
