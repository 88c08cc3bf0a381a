// Batched Arnoldi orthogonalisation for Krylov chains of matvecs (the
// iterative-solver setting that motivates fast block-Toeplitz products).
//
// One call advances any number of independent Arnoldi processes by one step:
// each job's new vector w = T v_j is orthogonalised against its basis
// v_0..v_{m-1} by classical Gram-Schmidt applied twice (CGS2), normalised,
// and written as v_m; the projections and the norm form column j of the
// Hessenberg matrix. All reductions accumulate in FP64 in a fixed order
// (per-block partial sums, then one ordered pass), so a job's results do not
// depend on which other jobs share the call.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "plan_internal.hpp"

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
// Work per thread (measured on one MI355X; one CGS2 step of a 3 x 128^3
// complex64 chain with 30 basis vectors): 4 entries and one basis vector per
// sweep keep the streaming kernels small (about 70 VGPRs) and took 1.44 ms,
// against 1.59 ms (2 vectors), 2.07 ms (4 vectors) and 3.31 ms (4 vectors of
// 8 entries)
constexpr int kPer = 4;                 // entries per thread of a chunk
constexpr int kChunk = kBlock * kPer;   // entries per partial-sum block
constexpr int kGroup = 1;               // basis vectors per sweep over a chunk
constexpr int kMaxM = 64;               // basis vectors per job
constexpr int kJobsPerLaunch = 24;

struct Job {
  const void* V;
  int64_t ldv;
  int64_t m;
  void* w;
  void* vout;
  int64_t n;
  double2* hcol;     // m+1 entries
  double2* part;     // partial sums: nchunk x (m or 1)
  double2* h;        // this pass's projections (m)
  int64_t chunk0;    // first block of this job in the launch
  int64_t nchunk;
};

struct JobTable {
  int njobs;
  Job j[kJobsPerLaunch];
};

__device__ __forceinline__ int find_job(const JobTable& t, int64_t blk) {
  int k = 0;
  while (k + 1 < t.njobs && blk >= t.j[k + 1].chunk0) ++k;
  return k;
}

template <typename C> __device__ __forceinline__ double2 to_d(C a) { return make_double2((double)a.x, (double)a.y); }

// Sum over the 64 lanes of a wavefront by a fixed butterfly of shuffles, so
// every lane gets the same, order-fixed result.
__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// Sum of one value per thread of the block in a fixed order: wavefront
// butterflies, then the kWaves wavefront sums in order (thread 0 returns it;
// red is kWaves entries of shared memory, one barrier inside).
__device__ __forceinline__ double2 block_sum(double2 v, double2* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int q = 0; q < kWaves; ++q) {
      s.x += red[q].x;
      s.y += red[q].y;
    }
  return s;
}

// partial[chunk][i] = sum_{k in chunk} conj(V_i[k]) w[k]. A sweep takes kGroup
// basis vectors at once (their loads in flight together); each thread's sums
// run over its entries in order, then wavefront butterflies and the wavefront
// sums in order, so a partial depends only on its job's data.
template <typename C>
__global__ void __launch_bounds__(kBlock) k_dots(JobTable t) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  const int64_t chunk = blockIdx.x - J.chunk0;
  const int64_t kb = chunk * kChunk + threadIdx.x;
  const C* V = (const C*)J.V;
  const C* w = (const C*)J.w;
  __shared__ double2 red[kWaves][kGroup];
  C wv[kPer];
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = kb + (int64_t)s * kBlock;
    wv[s] = k < J.n ? w[k] : C{0, 0};
  }
  const int wave = threadIdx.x >> 6;
  for (int64_t i0 = 0; i0 < J.m; i0 += kGroup) {
    C a[kGroup][kPer];
#pragma unroll
    for (int g = 0; g < kGroup; ++g)
#pragma unroll
      for (int s = 0; s < kPer; ++s) {
        const int64_t k = kb + (int64_t)s * kBlock;
        a[g][s] = (i0 + g < J.m && k < J.n) ? V[(i0 + g) * J.ldv + k] : C{0, 0};
      }
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int s = 0; s < kPer; ++s) {
        const double2 x = to_d(a[g][s]), y = to_d(wv[s]);
        sr += x.x * y.x + x.y * y.y;
        si += x.x * y.y - x.y * y.x;
      }
      const double2 v = wave_sum(make_double2(sr, si));
      if ((threadIdx.x & 63) == 0) red[wave][g] = v;
    }
    __syncthreads();
    if (threadIdx.x < kGroup && i0 + threadIdx.x < J.m) {
      double2 s = make_double2(0.0, 0.0);
      for (int q = 0; q < kWaves; ++q) {
        s.x += red[q][threadIdx.x].x;
        s.y += red[q][threadIdx.x].y;
      }
      J.part[chunk * J.m + i0 + threadIdx.x] = s;
    }
    __syncthreads();
  }
}

// One block per (job, i): h[i] = sum over the job's chunks (each thread sums
// the chunks c = tid, tid + kBlock, ... in order, then block_sum);
// hcol[i] = h[i] (first pass) or += h[i]
__global__ void __launch_bounds__(kBlock) k_dots_final(JobTable t, int accumulate) {
  const Job& J = t.j[blockIdx.x];
  const int64_t i = blockIdx.y;
  if (i >= J.m) return;  // whole block
  __shared__ double2 red[kWaves];
  double2 v = make_double2(0.0, 0.0);
  for (int64_t c = threadIdx.x; c < J.nchunk; c += kBlock) {
    v.x += J.part[c * J.m + i].x;
    v.y += J.part[c * J.m + i].y;
  }
  const double2 s = block_sum(v, red);
  if (threadIdx.x == 0) {
    J.h[i] = s;
    if (accumulate) {
      J.hcol[i].x += s.x;
      J.hcol[i].y += s.y;
    } else {
      J.hcol[i] = s;
    }
  }
}

// w[k] -= sum_i V_i[k] h[i]: a thread keeps its kPer entries in FP64 and
// takes the basis vectors kGroup at a time (their loads in flight together)
template <typename C>
__global__ void __launch_bounds__(kBlock) k_update(JobTable t) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  const int64_t kb = (blockIdx.x - J.chunk0) * kChunk + threadIdx.x;
  const C* V = (const C*)J.V;
  C* w = (C*)J.w;
  __shared__ double2 hs[kMaxM];
  for (int i = threadIdx.x; i < J.m; i += kBlock) hs[i] = J.h[i];
  __syncthreads();
  double2 acc[kPer];
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = kb + (int64_t)s * kBlock;
    acc[s] = k < J.n ? to_d(w[k]) : make_double2(0.0, 0.0);
  }
  for (int64_t i0 = 0; i0 < J.m; i0 += kGroup) {
    C a[kGroup][kPer];
#pragma unroll
    for (int g = 0; g < kGroup; ++g)
#pragma unroll
      for (int s = 0; s < kPer; ++s) {
        const int64_t k = kb + (int64_t)s * kBlock;
        a[g][s] = (i0 + g < J.m && k < J.n) ? V[(i0 + g) * J.ldv + k] : C{0, 0};
      }
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      if (i0 + g >= J.m) break;
      const double2 h = hs[i0 + g];
#pragma unroll
      for (int s = 0; s < kPer; ++s) {
        const double2 v = to_d(a[g][s]);
        acc[s].x -= v.x * h.x - v.y * h.y;
        acc[s].y -= v.x * h.y + v.y * h.x;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = kb + (int64_t)s * kBlock;
    if (k < J.n) {
      w[k].x = (decltype(C::x))acc[s].x;
      w[k].y = (decltype(C::x))acc[s].y;
    }
  }
}

// partial[chunk] = sum_{k in chunk} |w[k]|^2
template <typename C>
__global__ void __launch_bounds__(kBlock) k_norm(JobTable t) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  const int64_t chunk = blockIdx.x - J.chunk0;
  const int64_t kb = chunk * kChunk + threadIdx.x;
  const C* w = (const C*)J.w;
  __shared__ double2 red[kWaves];
  C a[kPer];
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = kb + (int64_t)s * kBlock;
    a[s] = k < J.n ? w[k] : C{0, 0};
  }
  double sq = 0.0;
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const double2 x = to_d(a[s]);
    sq += x.x * x.x + x.y * x.y;
  }
  const double2 tot = block_sum(make_double2(sq, 0.0), red);
  if (threadIdx.x == 0) J.part[chunk] = tot;
}

// One block per job: hcol[m] = sqrt(sum of partials in order); h[0] = 1/that
__global__ void __launch_bounds__(kBlock) k_norm_final(JobTable t) {
  const Job& J = t.j[blockIdx.x];
  __shared__ double2 red[kWaves];
  double2 v = make_double2(0.0, 0.0);
  for (int64_t c = threadIdx.x; c < J.nchunk; c += kBlock) v.x += J.part[c].x;
  const double2 s = block_sum(v, red);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(s.x);
    J.hcol[J.m] = make_double2(nrm, 0.0);
    J.h[0] = make_double2(nrm > 0.0 ? 1.0 / nrm : 0.0, 0.0);
  }
}

// vout[k] = w[k] / ||w||
template <typename C>
__global__ void __launch_bounds__(kBlock) k_scale(JobTable t) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  const int64_t kb = (blockIdx.x - J.chunk0) * kChunk + threadIdx.x;
  const C* w = (const C*)J.w;
  C* o = (C*)J.vout;
  const double inv = J.h[0].x;
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = kb + (int64_t)s * kBlock;
    if (k < J.n) {
      const double2 a = to_d(w[k]);
      o[k].x = (decltype(C::x))(a.x * inv);
      o[k].y = (decltype(C::x))(a.y * inv);
    }
  }
}

int64_t nchunks(int64_t n) { return (n + kChunk - 1) / kChunk; }

size_t job_scratch(const sfft_arnoldi_job& j) {
  // partial sums (nchunk x max(m, 1)) + projections (max(m, 1)), in double2
  const int64_t m = j.m > 0 ? j.m : 1;
  return sfft_rt_align256((size_t)(nchunks(j.n) * m + m) * sizeof(double2));
}

template <typename C> hipError_t run(std::vector<JobTable>& tabs, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int pass = 0; pass < 2; ++pass) {
    for (auto& t : tabs) {
      const int64_t blocks = t.j[t.njobs - 1].chunk0 + t.j[t.njobs - 1].nchunk;
      bool any = false;
      for (int k = 0; k < t.njobs; ++k) any |= t.j[k].m > 0;
      if (!any) continue;
      hipLaunchKernelGGL(k_dots<C>, dim3((unsigned)blocks), dim3(kBlock), 0, st, t);
      int64_t mmax = 1;
      for (int k = 0; k < t.njobs; ++k) mmax = t.j[k].m > mmax ? t.j[k].m : mmax;
      hipLaunchKernelGGL(k_dots_final, dim3(t.njobs, (unsigned)mmax), dim3(kBlock), 0, st, t, pass);
      hipLaunchKernelGGL(k_update<C>, dim3((unsigned)blocks), dim3(kBlock), 0, st, t);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  for (auto& t : tabs) {
    const int64_t blocks = t.j[t.njobs - 1].chunk0 + t.j[t.njobs - 1].nchunk;
    hipLaunchKernelGGL(k_norm<C>, dim3((unsigned)blocks), dim3(kBlock), 0, st, t);
    hipLaunchKernelGGL(k_norm_final, dim3(t.njobs), dim3(kBlock), 0, st, t);
    hipLaunchKernelGGL(k_scale<C>, dim3((unsigned)blocks), dim3(kBlock), 0, st, t);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return e;
}

}  // namespace

extern "C" {

sfft_status sfft_arnoldi_scratch_size(int njobs, const sfft_arnoldi_job* jobs, size_t* bytes) {
  if (njobs < 0 || (njobs > 0 && !jobs) || !bytes) return sfft_rt_fail(SFFT_INVALID_ARG, "null argument");
  size_t tot = 0;
  for (int i = 0; i < njobs; ++i) tot += job_scratch(jobs[i]);
  *bytes = tot;
  return SFFT_OK;
}

sfft_status sfft_arnoldi_step_multi(int njobs, const sfft_arnoldi_job* jobs, int dtype, void* scratch,
                                    size_t scratch_bytes, void* stream) {
  if (njobs < 0 || (njobs > 0 && !jobs)) return sfft_rt_fail(SFFT_INVALID_ARG, "null argument");
  if (dtype != SFFT_C64 && dtype != SFFT_C128) return sfft_rt_fail(SFFT_INVALID_ARG, "bad dtype");
  if (njobs == 0) return SFFT_OK;
  size_t need = 0;
  sfft_status s = sfft_arnoldi_scratch_size(njobs, jobs, &need);
  if (s != SFFT_OK) return s;
  if (!scratch || scratch_bytes < need) return sfft_rt_fail(SFFT_INVALID_ARG, "scratch too small");
  std::vector<JobTable> tabs;
  char* sp = (char*)scratch;
  for (int i = 0; i < njobs; ++i) {
    const sfft_arnoldi_job& q = jobs[i];
    if (!q.w || !q.vout || !q.hcol || q.n < 1 || q.m < 0 || q.m > kMaxM || (q.m > 0 && (!q.V || q.ldv < q.n)))
      return sfft_rt_fail(SFFT_INVALID_ARG, "bad Arnoldi job");
    if (tabs.empty() || tabs.back().njobs == kJobsPerLaunch) {
      JobTable t;
      std::memset(&t, 0, sizeof(t));
      tabs.push_back(t);
    }
    JobTable& t = tabs.back();
    Job& J = t.j[t.njobs];
    J.V = q.V;
    J.ldv = q.ldv;
    J.m = q.m;
    J.w = q.w;
    J.vout = q.vout;
    J.n = q.n;
    J.hcol = (double2*)q.hcol;
    J.nchunk = nchunks(q.n);
    J.chunk0 = t.njobs == 0 ? 0 : t.j[t.njobs - 1].chunk0 + t.j[t.njobs - 1].nchunk;
    const int64_t m = q.m > 0 ? q.m : 1;
    J.part = (double2*)sp;
    J.h = J.part + J.nchunk * m;
    sp += job_scratch(q);
    ++t.njobs;
  }
  hipError_t e = dtype == SFFT_C64 ? run<float2>(tabs, (hipStream_t)stream) : run<double2>(tabs, (hipStream_t)stream);
  if (e != hipSuccess) return sfft_rt_hip_fail(e, "Arnoldi step launch");
  return SFFT_OK;
}

}  // extern "C"
