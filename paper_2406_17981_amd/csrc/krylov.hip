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
constexpr int kChunk = kBlock * 16;  // entries per partial-sum block
constexpr int kMaxM = 64;            // basis vectors per job
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

// partial[chunk][i] = sum_{k in chunk} conj(V_i[k]) w[k]
template <typename C>
__global__ void __launch_bounds__(kBlock) k_dots(JobTable t) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  const int64_t chunk = blockIdx.x - J.chunk0;
  const int64_t k0 = chunk * kChunk;
  const C* V = (const C*)J.V;
  const C* w = (const C*)J.w;
  __shared__ double2 red[kBlock];
  constexpr int PER = kChunk / kBlock;
  double2 wv[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int64_t k = k0 + threadIdx.x + (int64_t)s * kBlock;
    wv[s] = k < J.n ? to_d(w[k]) : make_double2(0.0, 0.0);
  }
  for (int i = 0; i < J.m; ++i) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int64_t k = k0 + threadIdx.x + (int64_t)s * kBlock;
      if (k < J.n) {
        const double2 a = to_d(V[i * J.ldv + k]);
        sr += a.x * wv[s].x + a.y * wv[s].y;
        si += a.x * wv[s].y - a.y * wv[s].x;
      }
    }
    red[threadIdx.x] = make_double2(sr, si);
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        red[threadIdx.x].x += red[threadIdx.x + s].x;
        red[threadIdx.x].y += red[threadIdx.x + s].y;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) J.part[chunk * J.m + i] = red[0];
    __syncthreads();
  }
}

// h[i] = sum over chunks (in order); hcol[i] = h[i] (first pass) or += h[i]
__global__ void k_dots_final(JobTable t, int accumulate) {
  const Job& J = t.j[blockIdx.x];
  for (int i = threadIdx.x; i < J.m; i += blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int64_t c = 0; c < J.nchunk; ++c) {
      sr += J.part[c * J.m + i].x;
      si += J.part[c * J.m + i].y;
    }
    J.h[i] = make_double2(sr, si);
    if (accumulate) {
      J.hcol[i].x += sr;
      J.hcol[i].y += si;
    } else {
      J.hcol[i] = make_double2(sr, si);
    }
  }
}

// w[k] -= sum_i V_i[k] h[i]
template <typename C>
__global__ void __launch_bounds__(kBlock) k_update(JobTable t) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  const int64_t k0 = (blockIdx.x - J.chunk0) * kChunk;
  const C* V = (const C*)J.V;
  C* w = (C*)J.w;
  __shared__ double2 hs[kMaxM];
  for (int i = threadIdx.x; i < J.m; i += kBlock) hs[i] = J.h[i];
  __syncthreads();
  for (int64_t k = k0 + threadIdx.x; k < k0 + kChunk && k < J.n; k += kBlock) {
    double2 acc = to_d(w[k]);
    for (int i = 0; i < J.m; ++i) {
      const double2 v = to_d(V[i * J.ldv + k]);
      acc.x -= v.x * hs[i].x - v.y * hs[i].y;
      acc.y -= v.x * hs[i].y + v.y * hs[i].x;
    }
    w[k].x = (decltype(C::x))acc.x;
    w[k].y = (decltype(C::x))acc.y;
  }
}

// partial[chunk] = sum_{k in chunk} |w[k]|^2
template <typename C>
__global__ void __launch_bounds__(kBlock) k_norm(JobTable t) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  const int64_t chunk = blockIdx.x - J.chunk0;
  const int64_t k0 = chunk * kChunk;
  const C* w = (const C*)J.w;
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < k0 + kChunk && k < J.n; k += kBlock) {
    const double2 a = to_d(w[k]);
    s += a.x * a.x + a.y * a.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) J.part[chunk] = make_double2(red[0], 0.0);
}

// hcol[m] = sqrt(sum of partials); h[0] = 1/that
__global__ void k_norm_final(JobTable t) {
  const Job& J = t.j[blockIdx.x];
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int64_t c = 0; c < J.nchunk; ++c) s += J.part[c].x;
    const double nrm = sqrt(s);
    J.hcol[J.m] = make_double2(nrm, 0.0);
    J.h[0] = make_double2(nrm > 0.0 ? 1.0 / nrm : 0.0, 0.0);
  }
}

// vout[k] = w[k] / ||w||
template <typename C>
__global__ void __launch_bounds__(kBlock) k_scale(JobTable t) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  const int64_t k0 = (blockIdx.x - J.chunk0) * kChunk;
  const C* w = (const C*)J.w;
  C* o = (C*)J.vout;
  const double inv = J.h[0].x;
  for (int64_t k = k0 + threadIdx.x; k < k0 + kChunk && k < J.n; k += kBlock) {
    const double2 a = to_d(w[k]);
    o[k].x = (decltype(C::x))(a.x * inv);
    o[k].y = (decltype(C::x))(a.y * inv);
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
      hipLaunchKernelGGL(k_dots_final, dim3(t.njobs), dim3(64), 0, st, t, pass);
      hipLaunchKernelGGL(k_update<C>, dim3((unsigned)blocks), dim3(kBlock), 0, st, t);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  for (auto& t : tabs) {
    const int64_t blocks = t.j[t.njobs - 1].chunk0 + t.j[t.njobs - 1].nchunk;
    hipLaunchKernelGGL(k_norm<C>, dim3((unsigned)blocks), dim3(kBlock), 0, st, t);
    hipLaunchKernelGGL(k_norm_final, dim3(t.njobs), dim3(64), 0, st, t);
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
