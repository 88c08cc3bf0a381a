// Batched Arnoldi orthogonalisation for Krylov chains of matvecs (the
// iterative-solver setting that motivates fast block-Toeplitz products).
//
// One call advances any number of independent Arnoldi processes by one step:
// each job's new vector w = T v_j is orthogonalised against its basis
// v_0..v_{m-1} by classical Gram-Schmidt, normalised, and written as v_m; the
// projections and the norm form column j of the Hessenberg matrix. A second
// Gram-Schmidt pass runs only for a job whose first pass removed more than
// half of ||w||^2 (the Kahan-Parlett "twice is enough" test with
// alpha = 1/sqrt(2)): otherwise one projection against an orthonormal basis
// already leaves w orthogonal to working precision. All reductions
// accumulate in FP64 in a fixed order (per-block partial sums, then one
// ordered pass), and the test uses only the job's own sums, so a job's
// results do not depend on which other jobs share the call.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "plan_internal.hpp"

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
// Work per thread (measured on one MI355X; one two-pass step of a 3 x 128^3
// complex64 chain with 30 basis vectors): 4 entries and one basis vector per
// sweep keep the streaming kernels small and took 1.44 ms, against 1.59 ms
// (2 vectors), 2.07 ms (4 vectors) and 3.31 ms (4 vectors of 8 entries).
// Requesting the next vector's entries before the current one is reduced
// (k_dots: 70 VGPRs) or applied (k_update: 54) took a 96^3 GMRES(40) solve
// from 984 to 839 ms
constexpr int kPer = 4;                 // entries per thread of a chunk
constexpr int kChunk = kBlock * kPer;   // entries per partial-sum block
constexpr int kGroup = 1;               // basis vectors per sweep over a chunk
constexpr int kMaxM = 64;               // basis vectors per job
// second pass when ||w_1||^2 < kReorth2 ||w||^2 (w_1: w after one pass)
constexpr double kReorth2 = 0.5;
constexpr int kJobsPerLaunch = 24;

struct Job {
  const void* V;
  int64_t ldv;
  int64_t m;
  void* w;
  void* vout;
  int64_t n;
  double2* hcol;     // m+1 entries
  double2* part;     // partial sums: nchunk x (m + 1), column m for norms
  double2* h;        // m + 2: this pass's projections, ||w||^2, ||w_1||^2
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

// The job takes the second Gram-Schmidt pass (set once the first is done).
__device__ __forceinline__ bool reorth(const Job& J) { return J.h[J.m + 1].x < kReorth2 * J.h[J.m].x; }

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

// partial[chunk][i] = sum_{k in chunk} conj(V_i[k]) w[k], and on the first
// pass partial[chunk][m] = sum |w[k]|^2. A sweep takes kGroup basis vectors
// at once (their loads in flight together); each thread's sums run over its
// entries in order, then wavefront butterflies and the wavefront sums in
// order, so a partial depends only on its job's data. On the second pass a
// job that needs none exits (the whole block).
template <typename C>
__global__ void __launch_bounds__(kBlock) k_dots(JobTable t, int pass) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  if (pass == 1 && !reorth(J)) return;
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
  // the next sweep's basis entries are requested before this sweep's
  // reduction and barriers, so they arrive meanwhile
  C nx[kGroup][kPer];
#pragma unroll
  for (int g = 0; g < kGroup; ++g)
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      const int64_t k = kb + (int64_t)s * kBlock;
      nx[g][s] = (g < J.m && k < J.n) ? V[(int64_t)g * J.ldv + k] : C{0, 0};
    }
  for (int64_t i0 = 0; i0 < J.m; i0 += kGroup) {
    C a[kGroup][kPer];
#pragma unroll
    for (int g = 0; g < kGroup; ++g)
#pragma unroll
      for (int s = 0; s < kPer; ++s) {
        a[g][s] = nx[g][s];
        const int64_t k = kb + (int64_t)s * kBlock;
        const int64_t i1 = i0 + kGroup + g;
        nx[g][s] = (i1 < J.m && k < J.n) ? V[i1 * J.ldv + k] : C{0, 0};
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
      J.part[chunk * (J.m + 1) + i0 + threadIdx.x] = s;
    }
    __syncthreads();
  }
  if (pass == 0) {
    double sq = 0.0;
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      const double2 y = to_d(wv[s]);
      sq += y.x * y.x + y.y * y.y;
    }
    const double2 v = wave_sum(make_double2(sq, 0.0));
    if ((threadIdx.x & 63) == 0) red[wave][0] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double2 s = make_double2(0.0, 0.0);
      for (int q = 0; q < kWaves; ++q) s.x += red[q][0].x;
      J.part[chunk * (J.m + 1) + J.m] = s;
    }
  }
}

// One block per (job, i): h[i] = sum over the job's chunks (each thread sums
// the chunks c = tid, tid + kBlock, ... in order, then block_sum);
// hcol[i] = h[i] (first pass) or += h[i] (second); on the first pass block
// i = m sums the norm partials into h[m] = ||w||^2
__global__ void __launch_bounds__(kBlock) k_dots_final(JobTable t, int pass) {
  const Job& J = t.j[blockIdx.x];
  const int64_t i = blockIdx.y;
  if (i > J.m || (pass == 1 && (i == J.m || !reorth(J)))) return;  // whole block
  __shared__ double2 red[kWaves];
  double2 v = make_double2(0.0, 0.0);
  for (int64_t c = threadIdx.x; c < J.nchunk; c += kBlock) {
    v.x += J.part[c * (J.m + 1) + i].x;
    v.y += J.part[c * (J.m + 1) + i].y;
  }
  const double2 s = block_sum(v, red);
  if (threadIdx.x == 0) {
    J.h[i] = s;
    if (i < J.m) {
      if (pass == 1) {
        J.hcol[i].x += s.x;
        J.hcol[i].y += s.y;
      } else {
        J.hcol[i] = s;
      }
    }
  }
}

// w[k] -= sum_i V_i[k] h[i]: a thread keeps its kPer entries in FP64 and
// takes the basis vectors kGroup at a time (their loads in flight together);
// on the first pass partial[chunk][m] = sum |w_1[k]|^2 of the stored result
template <typename C>
__global__ void __launch_bounds__(kBlock) k_update(JobTable t, int pass) {
  const int jb = find_job(t, blockIdx.x);
  const Job& J = t.j[jb];
  if (pass == 1 && !reorth(J)) return;
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
  // the next sweep's basis entries are requested before this sweep's updates
  C nx[kGroup][kPer];
#pragma unroll
  for (int g = 0; g < kGroup; ++g)
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      const int64_t k = kb + (int64_t)s * kBlock;
      nx[g][s] = (g < J.m && k < J.n) ? V[(int64_t)g * J.ldv + k] : C{0, 0};
    }
  for (int64_t i0 = 0; i0 < J.m; i0 += kGroup) {
    C a[kGroup][kPer];
#pragma unroll
    for (int g = 0; g < kGroup; ++g)
#pragma unroll
      for (int s = 0; s < kPer; ++s) {
        a[g][s] = nx[g][s];
        const int64_t k = kb + (int64_t)s * kBlock;
        const int64_t i1 = i0 + kGroup + g;
        nx[g][s] = (i1 < J.m && k < J.n) ? V[i1 * J.ldv + k] : C{0, 0};
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
  double sq = 0.0;
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = kb + (int64_t)s * kBlock;
    C r;
    r.x = (decltype(C::x))acc[s].x;
    r.y = (decltype(C::x))acc[s].y;
    if (k < J.n) w[k] = r;
    const double2 y = to_d(r);  // 0 past the end
    sq += y.x * y.x + y.y * y.y;
  }
  if (pass == 0) {
    __shared__ double2 red[kWaves];
    const double2 tot = block_sum(make_double2(sq, 0.0), red);
    if (threadIdx.x == 0) J.part[(blockIdx.x - J.chunk0) * (J.m + 1) + J.m] = tot;
  }
}

// One block per job: h[m+1] = ||w_1||^2, the first pass's norm partials
// summed in order
__global__ void __launch_bounds__(kBlock) k_crit(JobTable t) {
  const Job& J = t.j[blockIdx.x];
  __shared__ double2 red[kWaves];
  double2 v = make_double2(0.0, 0.0);
  for (int64_t c = threadIdx.x; c < J.nchunk; c += kBlock) v.x += J.part[c * (J.m + 1) + J.m].x;
  const double2 s = block_sum(v, red);
  if (threadIdx.x == 0) J.h[J.m + 1] = s;
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
  // partial sums (nchunk x (m + 1)) + projections and the two squared norms
  // (m + 2), in double2
  return sfft_rt_align256((size_t)(nchunks(j.n) * (j.m + 1) + j.m + 2) * sizeof(double2));
}

template <typename C> hipError_t run(std::vector<JobTable>& tabs, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int pass = 0; pass < 2; ++pass) {
    for (auto& t : tabs) {
      const int64_t blocks = t.j[t.njobs - 1].chunk0 + t.j[t.njobs - 1].nchunk;
      bool any = false;
      for (int k = 0; k < t.njobs; ++k) any |= t.j[k].m > 0;
      if (!any) continue;
      hipLaunchKernelGGL(k_dots<C>, dim3((unsigned)blocks), dim3(kBlock), 0, st, t, pass);
      int64_t mmax = 1;
      for (int k = 0; k < t.njobs; ++k) mmax = t.j[k].m > mmax ? t.j[k].m : mmax;
      hipLaunchKernelGGL(k_dots_final, dim3(t.njobs, (unsigned)(mmax + 1)), dim3(kBlock), 0, st, t, pass);
      hipLaunchKernelGGL(k_update<C>, dim3((unsigned)blocks), dim3(kBlock), 0, st, t, pass);
      if (pass == 0) hipLaunchKernelGGL(k_crit, dim3(t.njobs), dim3(kBlock), 0, st, t);
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
    J.part = (double2*)sp;
    J.h = J.part + J.nchunk * (q.m + 1);
    sp += job_scratch(q);
    ++t.njobs;
  }
  hipError_t e = dtype == SFFT_C64 ? run<float2>(tabs, (hipStream_t)stream) : run<double2>(tabs, (hipStream_t)stream);
  if (e != hipSuccess) return sfft_rt_hip_fail(e, "Arnoldi step launch");
  return SFFT_OK;
}

}  // extern "C"
