// Restarted GMRES(m) with mixed-precision iterative refinement for the
// scattering operator A = I - diag(chi) T, T the block-Toeplitz matrix of a
// plan: the iterative-solver setting in which the paper's fast products are
// used (the matvec is the dominant cost of every Krylov step).
//
// Outer loop (FP64): r = b - A x with T applied by a complex128 plan,
// beta = ||r||; stop when beta <= tol ||b||.
// Inner cycle (the product dtype of the low plan, typically complex64):
// Arnoldi on v_0 = r / beta with w = A v_j = v_j - chi .* (T v_j), classical
// Gram-Schmidt with the on-demand second pass of sfft_arnoldi_step_multi;
// the Hessenberg columns come back to the host, where Givens rotations keep
// the least-squares residual estimate |g_{j+1}|; the cycle ends at m steps,
// at a breakdown or once the estimate meets the tolerance. The correction
// x += V_j y is accumulated in FP64 on the device. FP32 rounding in the inner
// cycle only limits how much one cycle reduces the FP64 residual, so the outer
// loop reaches tolerances far below FP32 precision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "plan_internal.hpp"

namespace {

using cd = std::complex<double>;

constexpr int kGmresMaxM = 64;

#define HIP_CHECK_RET(expr)                                  \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return sfft_rt_hip_fail(e_, #expr); \
  } while (0)

unsigned grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

// w <- v - chi .* w (compute dtype; chi given in complex128)
template <typename C>
__global__ void k_chi_apply(const C* __restrict__ v, C* __restrict__ w, const double2* __restrict__ chi, int64_t n) {
  using R = decltype(C::x);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 c = chi[i];
    const C t = w[i];
    const R cr = (R)c.x, ci = (R)c.y;
    w[i] = sfft::mk<C>(v[i].x - (cr * t.x - ci * t.y), v[i].y - (cr * t.y + ci * t.x));
  }
}

// r <- b - (x - chi .* tx), all complex128
__global__ void k_residual(const double2* __restrict__ b, const double2* __restrict__ x,
                           const double2* __restrict__ tx, const double2* __restrict__ chi, double2* __restrict__ r,
                           int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 c = chi[i], t = tx[i];
    r[i] = make_double2(b[i].x - x[i].x + (c.x * t.x - c.y * t.y), b[i].y - x[i].y + (c.x * t.y + c.y * t.x));
  }
}

// v (compute dtype) <- r (complex128), already scaled to unit norm
template <typename C>
__global__ void k_to_dtype(const double2* __restrict__ r, C* __restrict__ v, int64_t n) {
  using R = decltype(C::x);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = sfft::mk<C>((R)r[i].x, (R)r[i].y);
}

// x <- x + sum_k y_k V_k (x complex128, V the compute dtype, y complex128)
template <typename C>
__global__ void k_correct(double2* __restrict__ x, const C* __restrict__ V, int64_t ldv, const double2* __restrict__ y,
                          int k, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double re = x[i].x, im = x[i].y;
    for (int j = 0; j < k; ++j) {
      const C v = V[j * ldv + i];
      const double2 c = y[j];
      re += c.x * (double)v.x - c.y * (double)v.y;
      im += c.x * (double)v.y + c.y * (double)v.x;
    }
    x[i] = make_double2(re, im);
  }
}

size_t al(size_t x) { return sfft_rt_align256(x); }

struct Layout {
  size_t V, tx, r, hcol, ydev, arn, ws_lo, ws_hi, total;
};

// Workspace pieces (offsets in bytes): basis V (m+1 vectors of the low
// dtype), FP64 T x and r, the Hessenberg column and correction coefficients,
// Arnoldi scratch, and the two plans' apply workspaces.
sfft_status layout(const sfft_plan_s* lo, const sfft_plan_s* hi, int m, Layout* L) {
  const int64_t n = lo->b * lo->s;
  size_t off = 0;
  std::memset(L, 0, sizeof(*L));
  L->V = off;
  off += al((size_t)(m + 1) * n * lo->esz);
  L->tx = off;
  off += al((size_t)n * 16);
  L->r = off;
  off += al((size_t)n * 16);
  L->hcol = off;
  off += al((size_t)(m + 2) * 16);
  L->ydev = off;
  off += al((size_t)(m + 1) * 16);
  sfft_arnoldi_job job;
  std::memset(&job, 0, sizeof(job));
  job.n = n;
  job.ldv = n;
  job.m = m;
  size_t arn = 0;
  sfft_status s = sfft_arnoldi_scratch_size(1, &job, &arn);
  if (s != SFFT_OK) return s;
  L->arn = off;  // also serves the FP64 normalisations (m = 0 needs less)
  off += al(arn);
  L->ws_lo = off;
  off += al(sfft_rt_workspace_elems(lo, 1) * lo->esz);
  L->ws_hi = off;
  off += al(sfft_rt_workspace_elems(hi, 1) * hi->esz);
  L->total = off;
  return SFFT_OK;
}

sfft_status check_pair(const sfft_plan_s* lo, const sfft_plan_s* hi, int m) {
  if (!lo || !hi) return sfft_rt_fail(SFFT_INVALID_ARG, "plans must be non-null");
  if (hi->dtype != SFFT_C128) return sfft_rt_fail(SFFT_INVALID_ARG, "the residual plan must be complex128");
  if (lo->b != hi->b || lo->s != hi->s)
    return sfft_rt_fail(SFFT_INVALID_ARG, "the two plans must describe the same grid and block size");
  // the caller's levels of size > 1 (a plan may carry a long level as several)
  std::vector<int64_t> glo, ghi;
  for (int l = 0; l < lo->user_d; ++l)
    if (lo->user_n[l] > 1) glo.push_back(lo->user_n[l]);
  for (int l = 0; l < hi->user_d; ++l)
    if (hi->user_n[l] > 1) ghi.push_back(hi->user_n[l]);
  if (glo != ghi) return sfft_rt_fail(SFFT_INVALID_ARG, "the two plans must have the same grid");
  if (m < 1 || m > kGmresMaxM) return sfft_rt_fail(SFFT_INVALID_ARG, "m must be in 1..64");
  return SFFT_OK;
}

}  // namespace

extern "C" {

sfft_status sfft_gmres_workspace_size(sfft_plan lo, sfft_plan hi, int m, size_t* bytes) {
  if (!bytes) return sfft_rt_fail(SFFT_INVALID_ARG, "bytes is null");
  sfft_status s = check_pair(lo, hi, m);
  if (s != SFFT_OK) return s;
  Layout L;
  if ((s = layout(lo, hi, m, &L)) != SFFT_OK) return s;
  *bytes = L.total;
  return SFFT_OK;
}

sfft_status sfft_gmres_solve(sfft_plan lo, sfft_plan hi, const void* chi, const void* rhs, void* x, int m,
                             int max_cycles, double tol, void* workspace, size_t ws_bytes, void* stream,
                             sfft_gmres_info* info) {
  sfft_status s = check_pair(lo, hi, m);
  if (s != SFFT_OK) return s;
  if (!chi || !rhs || !x || !workspace) return sfft_rt_fail(SFFT_INVALID_ARG, "null device pointer");
  if (max_cycles < 1 || !(tol > 0.0)) return sfft_rt_fail(SFFT_INVALID_ARG, "max_cycles >= 1 and tol > 0 required");
  Layout L;
  if ((s = layout(lo, hi, m, &L)) != SFFT_OK) return s;
  if (ws_bytes < L.total) return sfft_rt_fail(SFFT_INVALID_ARG, "workspace too small: need " + std::to_string(L.total));
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = lo->b * lo->s;
  char* ws = (char*)workspace;
  char* V = ws + L.V;
  double2* tx = (double2*)(ws + L.tx);
  double2* r = (double2*)(ws + L.r);
  double2* hcol_d = (double2*)(ws + L.hcol);
  double2* y_d = (double2*)(ws + L.ydev);
  void* arn = ws + L.arn;
  const size_t arn_bytes = L.ws_lo - L.arn;
  void* ws_lo = ws + L.ws_lo;
  void* ws_hi = ws + L.ws_hi;
  const size_t ws_lo_bytes = L.ws_hi - L.ws_lo, ws_hi_bytes = L.total - L.ws_hi;
  const double2* b = (const double2*)rhs;
  double2* xd = (double2*)x;
  const double2* chid = (const double2*)chi;
  const bool c64 = lo->dtype == SFFT_C64;
  const size_t vb = (size_t)n * lo->esz;

  sfft_gmres_info out;
  std::memset(&out, 0, sizeof(out));
  std::vector<double2> hcol(m + 2);
  auto fetch = [&](double2* dst, const double2* src, int cnt) -> sfft_status {
    HIP_CHECK_RET(hipMemcpyAsync(dst, src, cnt * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIP_CHECK_RET(hipStreamSynchronize(st));
    return SFFT_OK;
  };
  // ||b|| through the FP64 Arnoldi normalisation of a copy of b
  auto fp64_norm_normalise = [&](double2* vec, double* nrm) -> sfft_status {
    sfft_arnoldi_job job;
    std::memset(&job, 0, sizeof(job));
    job.V = vec;
    job.ldv = n;
    job.m = 0;
    job.w = vec;
    job.vout = vec;
    job.n = n;
    job.hcol = hcol_d;
    sfft_status q = sfft_arnoldi_step_multi(1, &job, SFFT_C128, arn, arn_bytes, st);
    if (q != SFFT_OK) return q;
    double2 h;
    if ((q = fetch(&h, hcol_d, 1)) != SFFT_OK) return q;
    *nrm = h.x;
    return SFFT_OK;
  };
  // r = b - A x in FP64 (T x by the complex128 plan)
  auto true_residual = [&](double* beta) -> sfft_status {
    sfft_status q = sfft_rt_apply_one(hi, xd, tx, 1, ws_hi, ws_hi_bytes, st);
    if (q != SFFT_OK) return q;
    ++out.fp64_matvecs;
    hipLaunchKernelGGL(k_residual, dim3(grid_of(n)), dim3(256), 0, st, b, xd, tx, chid, r, n);
    HIP_CHECK_RET(hipGetLastError());
    return fp64_norm_normalise(r, beta);  // r <- r / ||r||
  };

  double bnorm = 0.0;
  HIP_CHECK_RET(hipMemcpyAsync(r, b, (size_t)n * 16, hipMemcpyDeviceToDevice, st));
  if ((s = fp64_norm_normalise(r, &bnorm)) != SFFT_OK) return s;
  if (bnorm == 0.0) {  // A x = 0: x = 0
    HIP_CHECK_RET(hipMemsetAsync(xd, 0, (size_t)n * 16, st));
    HIP_CHECK_RET(hipStreamSynchronize(st));
    out.converged = 1;
    if (info) *info = out;
    return SFFT_OK;
  }
  double beta = 0.0;
  if ((s = true_residual(&beta)) != SFFT_OK) return s;
  out.rel_residual = beta / bnorm;
  std::vector<cd> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  while (out.rel_residual > tol && out.cycles < max_cycles) {
    ++out.cycles;
    // v_0 = r / beta in the product dtype
    if (c64) hipLaunchKernelGGL(k_to_dtype<float2>, dim3(grid_of(n)), dim3(256), 0, st, r, (float2*)V, n);
    else HIP_CHECK_RET(hipMemcpyAsync(V, r, (size_t)n * 16, hipMemcpyDeviceToDevice, st));
    HIP_CHECK_RET(hipGetLastError());
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    int k = 0;  // basis vectors used by the correction
    for (int j = 0; j < m; ++j) {
      char* vj = V + (size_t)j * vb;
      char* w = V + (size_t)(j + 1) * vb;
      if ((s = sfft_rt_apply_one(lo, vj, w, 1, ws_lo, ws_lo_bytes, st)) != SFFT_OK) return s;
      ++out.matvecs;
      if (c64)
        hipLaunchKernelGGL(k_chi_apply<float2>, dim3(grid_of(n)), dim3(256), 0, st, (const float2*)vj, (float2*)w,
                           chid, n);
      else
        hipLaunchKernelGGL(k_chi_apply<double2>, dim3(grid_of(n)), dim3(256), 0, st, (const double2*)vj,
                           (double2*)w, chid, n);
      HIP_CHECK_RET(hipGetLastError());
      sfft_arnoldi_job job;
      std::memset(&job, 0, sizeof(job));
      job.V = V;
      job.ldv = n;
      job.m = j + 1;
      job.w = w;
      job.vout = w;
      job.n = n;
      job.hcol = hcol_d;
      if ((s = sfft_arnoldi_step_multi(1, &job, lo->dtype, arn, arn_bytes, st)) != SFFT_OK) return s;
      if ((s = fetch(hcol.data(), hcol_d, j + 2)) != SFFT_OK) return s;
      // column j of H, rotated by the previous Givens rotations
      for (int i = 0; i <= j + 1; ++i) H[(size_t)i * m + j] = cd(hcol[i].x, hcol[i].y);
      for (int i = 0; i < j; ++i) {
        const cd a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = std::conj(cs[i]) * a + std::conj(sn[i]) * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      // new rotation zeroing H[j+1][j]
      const cd a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
      const double den = std::sqrt(std::norm(a) + std::norm(c));
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / den;
        sn[j] = c / den;
      }
      H[(size_t)j * m + j] = std::conj(cs[j]) * a + std::conj(sn[j]) * c;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = std::conj(cs[j]) * g[j];
      k = j + 1;
      out.rel_residual_estimate = std::abs(g[j + 1]) / bnorm;
      // lucky breakdown (w in the span) or the estimate meets the target
      double colnorm = 0.0;
      for (int i = 0; i <= j + 1; ++i) colnorm += hcol[i].x * hcol[i].x + hcol[i].y * hcol[i].y;
      if (hcol[j + 1].x <= 1e-14 * std::sqrt(colnorm) || std::abs(g[j + 1]) <= 0.5 * tol * bnorm) break;
    }
    // y = H^-1 g (upper triangular, k x k), x += V y in FP64
    std::vector<cd> yv(k);
    for (int i = k - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= H[(size_t)i * m + l] * yv[l];
      yv[i] = acc / H[(size_t)i * m + i];
    }
    std::vector<double2> yh(k);
    for (int i = 0; i < k; ++i) yh[i] = make_double2(yv[i].real(), yv[i].imag());
    HIP_CHECK_RET(hipMemcpyAsync(y_d, yh.data(), k * sizeof(double2), hipMemcpyHostToDevice, st));
    if (c64)
      hipLaunchKernelGGL(k_correct<float2>, dim3(grid_of(n)), dim3(256), 0, st, xd, (const float2*)V, n, y_d, k, n);
    else
      hipLaunchKernelGGL(k_correct<double2>, dim3(grid_of(n)), dim3(256), 0, st, xd, (const double2*)V, n, y_d, k,
                         n);
    HIP_CHECK_RET(hipGetLastError());
    if ((s = true_residual(&beta)) != SFFT_OK) return s;
    out.rel_residual = beta / bnorm;
  }
  HIP_CHECK_RET(hipStreamSynchronize(st));
  out.converged = out.rel_residual <= tol;
  if (info) *info = out;
  return SFFT_OK;
}

}  // extern "C"
