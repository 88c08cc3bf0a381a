// Plan, schedule and C ABI of the split-FFT block-Toeplitz matvec.
//
// Plan creation builds the Fourier-space branch data T[bId] of Section II.C
// in FP64 on the GPU (embedded generator, 2n-point transforms along every
// level, parity de-interleave, 2^-d / prod(n) folded in) and stores it in the
// compute dtype in the order the leaf kernel's lanes consume it. Apply runs
// Algorithm 1 as a sequence of fused axis passes:
//
//   level l = 1 .. d-1 : FWD2  (FFT_l of the even child, phase + FFT_l of the odd child)
//   level d            : LEAF  (both children of the last level, mulBrn, iFFT_d, merge)
//   level l = d-1 .. 1 : INV2  (iFFT_l of both children, merge with conj phase)
//
// either breadth-first (all branches of a level in one launch) or in the
// lazy depth-first order of Algorithm 1 (one branch pair at a time, d-1
// workspace vectors).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "plan_internal.hpp"

using sfft::AxisOps;
using sfft::PassArgs;

#define SFFT_X(L) extern "C" const AxisOps* sfft_ops_##L(int);
#include "lengths.def"
#undef SFFT_X
extern "C" const AxisOps* sfft_ops_generic(int dtype, int64_t L);
#define SFFT_X(L) extern "C" int sfft_radix_##L(int, int, int*);
#include "lengths.def"
#undef SFFT_X
extern "C" int sfft_radix_generic(int64_t L, int* rads);

namespace {

const AxisOps* find_ops(int dtype, int64_t L) {
  switch (L) {
#define SFFT_X(LL) \
  case LL:         \
    return sfft_ops_##LL(dtype);
#include "lengths.def"
#undef SFFT_X
    default:
      return sfft_ops_generic(dtype, L);  // runtime-length kernels, or null
  }
}

// Radices of the kernels for pencil length L (passes, or the leaf), outermost
// stage first, into rads[0..7]; returns how many.
int find_radix(int dtype, int64_t L, bool leaf, int* rads) {
  switch (L) {
#define SFFT_X(LL) \
  case LL:         \
    return sfft_radix_##LL(dtype, leaf ? 1 : 0, rads);
#include "lengths.def"
#undef SFFT_X
    default:
      return sfft_radix_generic(L, rads);
  }
}

// LDS the runtime-length kernels of one level need: a pass stages up to three
// rows of the pencil length (two for a forward pass or a pass without a
// second child), a leaf 2b + 1 rows (split) or b + 1 (embedding).
bool generic_fits(const AxisOps* o, int dtype, int b, int npar, bool leaf, bool inv_two) {
  if (!o || !o->generic) return true;
  const size_t esz = dtype == SFFT_C64 ? 8 : 16;
  const size_t rows = leaf ? (size_t)(npar == 2 ? 2 * b : b) + 1 : (inv_two ? 3 : 2);
  return rows * (size_t)o->L * esz <= sfft::kMaxLds;
}

thread_local std::string g_err;

sfft_status fail(sfft_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

sfft_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? SFFT_OUT_OF_MEMORY : SFFT_HIP_ERROR;
}

#define HIP_TRY(expr, what)                   \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

struct Dims {
  int d;
  int64_t n[kMaxD];
};

// ---------------------------------------------------------------------------
// Auxiliary kernels
// ---------------------------------------------------------------------------

// tw[m] = exp(-i pi m / L), m < 2L, evaluated in FP64 with exact rational
// arguments and rounded once to the table type.
template <typename C>
__global__ void k_twiddle(C* tw, int L) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < 2 * L) {
    double s, c;
    sincospi((double)m / (double)L, &s, &c);
    tw[m] = sfft::mk<C>((decltype(C::x))c, (decltype(C::x))(-s));
  }
}

// Circulant embedding of one block component (introduction): along each
// level, offset r goes to position r mod 2n, position n holds 0.
__global__ void k_embed_generator(const double2* __restrict__ coeffs, double2* __restrict__ c, int comp,
                                  Dims dm, int64_t total) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = idx, src = 0, sstride = 1;
    bool pad = false;
    for (int l = dm.d - 1; l >= 0; --l) {
      const int64_t L2 = 2 * dm.n[l];
      const int64_t m = rem % L2;
      rem /= L2;
      if (m == dm.n[l]) pad = true;
      const int64_t r = m < dm.n[l] ? m : m - L2;
      src += (r + dm.n[l] - 1) * sstride;
      sstride *= 2 * dm.n[l] - 1;
    }
    c[idx] = pad ? sfft::mk<double2>(0.0, 0.0) : coeffs[(int64_t)comp * sstride + src];
  }
}

// Generator of a plan whose long levels are carried as several levels: plan
// entry (component ab, offset indices i_q) = caller entry
// ab * ncoef_in + cbase + sum_q i_q mult[q] (Regather).
__global__ void k_regather(const double2* __restrict__ src, double2* __restrict__ dst, Regather g,
                           int64_t total) {
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = o % g.ncoef_out;
    int64_t at = (o / g.ncoef_out) * g.ncoef_in + g.cbase;
    for (int q = g.dq - 1; q >= 0; --q) {
      const int64_t i = rem % g.ext[q];
      rem /= g.ext[q];
      at += i * g.mult[q];
    }
    dst[o] = src[at];
  }
}

// Parity de-interleave of one FP64 symbol component into the leaf layout of
// the split plan: [Q][p][tile][k][m][lane] with Q the branch prefix over
// levels 1..d-1 (level 1 most significant), p the last level's bit and k
// the stored component (NS per block).
template <typename C>
__global__ void k_scatter_split(const double2* __restrict__ full, C* __restrict__ sym, int ks, int NS, Dims dm,
                                int T, int E, int NT, int P, int64_t ntiles, int64_t npen, double scale,
                                int64_t total) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int tid = (int)(idx % NT);
    const int m = (int)((idx / NT) % E);
    const int64_t tile = (idx / ((int64_t)NT * E)) % ntiles;
    const int64_t pq = idx / ((int64_t)NT * E * ntiles);  // Q*2 + p
    const int p = (int)(pq & 1);
    const int64_t Q = pq >> 1;
    const int64_t pencil = tile * P + tid / T;
    const int64_t k = tid % T + (int64_t)T * m;
    const int64_t dst = (pq * ntiles + tile) * NS * E * NT + sfft::sym_offset(ks, m, tid, E, NT);
    if (pencil >= npen) {
      sym[dst] = sfft::mk<C>(0, 0);
      continue;
    }
    const int d = dm.d;
    int64_t fidx = 2 * k + p, fstride = 2 * dm.n[d - 1];
    int64_t rem = pencil;
    for (int l = d - 2; l >= 0; --l) {
      const int64_t j = rem % dm.n[l];
      rem /= dm.n[l];
      const int64_t bit = (Q >> (d - 2 - l)) & 1;
      fidx += (2 * j + bit) * fstride;
      fstride *= 2 * dm.n[l];
    }
    const double2 v = full[fidx];
    sym[dst] = sfft::mk<C>((decltype(C::x))(v.x * scale), (decltype(C::x))(v.y * scale));
  }
}

// Full symbol of the embedding baseline in the leaf layout: [tile][k][m][lane]
// over pencils of the 2n-grid.
template <typename C>
__global__ void k_scatter_embed(const double2* __restrict__ full, C* __restrict__ sym, int ks, int NS, int T,
                                int E, int NT, int P, int64_t ntiles, int64_t npen, int64_t L,
                                double scale, int64_t total) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int tid = (int)(idx % NT);
    const int m = (int)((idx / NT) % E);
    const int64_t tile = idx / ((int64_t)NT * E);
    const int64_t pencil = tile * P + tid / T;
    const int64_t k = tid % T + (int64_t)T * m;
    const int64_t dst = tile * NS * E * NT + sfft::sym_offset(ks, m, tid, E, NT);
    if (pencil >= npen) {
      sym[dst] = sfft::mk<C>(0, 0);
      continue;
    }
    const double2 v = full[pencil * L + k];
    sym[dst] = sfft::mk<C>((decltype(C::x))(v.x * scale), (decltype(C::x))(v.y * scale));
  }
}

// Mirrored storage of one FP64 symbol component (Section II.C): stored index
// s_l in [0, n_l] along every level, s_l < n_l/2+1 holding the even bin
// 2 s_l of the 2n_l lattice and the rest the odd bins 2 (s_l - n_l/2 - 1) + 1.
// With lane pairs (paired = 1; the leaf's T lanes hold E entries each, E a
// multiple of 4) the last level's row is the even part, (T + 1) lanes x E/2
// entries, then the odd part, T lanes x E/2 entries, each part ordered
// [e / 2][lane][e % 2]: lane u < T, entry e is index u + T e of that parity's
// half row, and the extra lane T of the even part repeats indexes T (e + 1).
// A leaf lane t then reads its entries m, m + 1 (m even) as one pair: its own
// below E/2, lane T - t (even) or T - 1 - t (odd), pair E - 2 - m, above.
template <typename C>
__global__ void k_scatter_mirror(const double2* __restrict__ full, C* __restrict__ sym, int ks, Dims dm,
                                 double scale, int64_t total, int paired, int T, int E, int64_t mrow) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = idx, fidx = 0, fstride = 1;
    for (int l = dm.d - 1; l >= 0; --l) {
      const int64_t n = dm.n[l];
      int64_t M;
      if (paired && l == dm.d - 1) {
        const int64_t pos = rem % mrow;
        rem /= mrow;
        const int64_t even_part = (int64_t)(T + 1) * (E / 2);
        const int par = pos < even_part ? 0 : 1;
        const int64_t q = par ? pos - even_part : pos;
        const int64_t W = par ? T : T + 1;
        const int64_t e = 2 * (q / (2 * W)) + (q % 2);
        const int64_t u = (q / 2) % W;
        const int64_t h = (par == 0 && u == T) ? T * (e + 1) : u + T * e;  // index in the half row
        M = 2 * h + par;
      } else {
        const int64_t sl = rem % (n + 1);
        rem /= n + 1;
        const int64_t m0 = n / 2 + 1;
        M = sl < m0 ? 2 * sl : 2 * (sl - m0) + 1;
      }
      fidx += M * fstride;
      fstride *= 2 * n;
    }
    const double2 v = full[fidx];
    sym[(int64_t)ks * total + idx] = sfft::mk<C>((decltype(C::x))(v.x * scale), (decltype(C::x))(v.y * scale));
  }
}

// x (nv, n...) -> zero-padded (nv, 2n...)
template <typename C>
__global__ void k_pad(const C* __restrict__ x, C* __restrict__ P, Dims dm, int64_t total) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = idx, src = 0, sstride = 1;
    bool inside = true;
    for (int l = dm.d - 1; l >= 0; --l) {
      const int64_t m = rem % (2 * dm.n[l]);
      rem /= 2 * dm.n[l];
      if (m >= dm.n[l]) inside = false;
      src += m * sstride;
      sstride *= dm.n[l];
    }
    P[idx] = inside ? x[rem * sstride + src] : sfft::mk<C>(0, 0);
  }
}

// One-shot pad and project of the embedding baseline (one or two entries per
// thread, indices decoded by multiply-high division), used while every index
// fits in 32 bits: per level the grid size and dividers by n and 2n.
struct PadGeo {
  int d;
  uint32_t n[kMaxD];
  sfft::FastDiv fn[kMaxD], f2n[kMaxD];
};

PadGeo pad_geo(const Dims& dm) {
  PadGeo g;
  std::memset(&g, 0, sizeof(g));
  g.d = dm.d;
  for (int l = 0; l < dm.d; ++l) {
    g.n[l] = (uint32_t)dm.n[l];
    g.fn[l] = sfft::FastDiv::make((uint32_t)dm.n[l]);
    g.f2n[l] = sfft::FastDiv::make((uint32_t)(2 * dm.n[l]));
  }
  return g;
}

// x (nv, n...) -> P (nv, 2n...): thread i writes padded entries 2i and 2i + 1,
// which share a row (the padded last length is even); the first n entries
// along every level come from x, the rest are zero
template <typename C>
__global__ void __launch_bounds__(256) k_pad2(const C* __restrict__ x, C* __restrict__ P, PadGeo g, uint32_t npairs) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= npairs) return;
  uint32_t rem = 2 * i, src = 0, sstride = 1, mlast = 0;
  bool inside = true;
  for (int l = g.d - 1; l >= 0; --l) {
    const uint32_t q = g.f2n[l].div(rem);
    const uint32_t m = rem - q * (2 * g.n[l]);
    if (l == g.d - 1) mlast = m;
    else inside = inside && m < g.n[l];
    src += m * sstride;
    sstride *= g.n[l];
    rem = q;
  }
  const uint32_t s0 = rem * sstride + src;  // rem is the vector index
  const uint32_t nl = g.n[g.d - 1];
  C a = sfft::mk<C>(0, 0), b = a;
  if (inside && mlast < nl) a = x[s0];
  if (inside && mlast + 1 < nl) b = x[s0 + 1];
  P[2 * (size_t)i] = a;
  P[2 * (size_t)i + 1] = b;
}

// y (nv, n...) <- the first n entries along every level of P (nv, 2n...)
template <typename C>
__global__ void __launch_bounds__(256) k_project2(const C* __restrict__ P, C* __restrict__ y, PadGeo g, uint32_t total) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= total) return;
  uint32_t rem = i, src = 0, sstride = 1;
  for (int l = g.d - 1; l >= 0; --l) {
    const uint32_t q = g.fn[l].div(rem);
    src += (rem - q * g.n[l]) * sstride;
    sstride *= 2 * g.n[l];
    rem = q;
  }
  y[i] = P[rem * sstride + src];
}

// zero-padded (nv, 2n...) -> y (nv, n...): keep the first n along every level
template <typename C>
__global__ void k_project(const C* __restrict__ P, C* __restrict__ y, Dims dm, int64_t total) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = idx, src = 0, sstride = 1;
    for (int l = dm.d - 1; l >= 0; --l) {
      const int64_t j = rem % dm.n[l];
      rem /= dm.n[l];
      src += j * sstride;
      sstride *= 2 * dm.n[l];
    }
    y[idx] = P[rem * sstride + src];
  }
}

// Block symmetry of the coefficients, exactly: for every pair a < c, bit 0 of
// flags[pair] is set if some offset has t[a,c] != t[c,a], bit 1 if some
// offset has t[a,c] != -t[c,a]. One atomic per wavefront that saw a mismatch.
// Every wavefront that finds a mismatch would otherwise hit the same few flag
// words (the symmetric Green blocks make every one of them "not
// antisymmetric"), so the workgroup first combines its bits in LDS and skips
// the atomic when the flag already holds them.
template <int B>
__global__ void __launch_bounds__(256) k_block_symmetry(const double2* __restrict__ coeffs, int64_t ncoef,
                                                        unsigned* flags) {
  constexpr int NPR = B * (B - 1) / 2;
  __shared__ unsigned wg_bits;
  if (threadIdx.x == 0) wg_bits = 0;
  __syncthreads();
  unsigned bits = 0;  // bit 2*pair + {0: not symmetric, 1: not antisymmetric}
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < ncoef;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double2 u[NPR], v[NPR];
    int pr = 0;
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int c = a + 1; c < B; ++c, ++pr) {
        u[pr] = coeffs[(int64_t)(a * B + c) * ncoef + idx];
        v[pr] = coeffs[(int64_t)(c * B + a) * ncoef + idx];
      }
#pragma unroll
    for (int q = 0; q < NPR; ++q) {
      if (!(u[q].x == v[q].x && u[q].y == v[q].y)) bits |= 1u << (2 * q);
      if (!(u[q].x == -v[q].x && u[q].y == -v[q].y)) bits |= 2u << (2 * q);
    }
  }
  for (int off = 32; off > 0; off >>= 1) bits |= __shfl_xor(bits, off, 64);
  if (bits && (threadIdx.x % 64) == 0) atomicOr(&wg_bits, bits);
  __syncthreads();
  if (threadIdx.x < NPR) {
    const unsigned f = (wg_bits >> (2 * threadIdx.x)) & 3u;
    if (f && (__atomic_load_n(&flags[threadIdx.x], __ATOMIC_RELAXED) & f) != f) atomicOr(&flags[threadIdx.x], f);
  }
}

// Declared per-(component, level) parity of the generator, checked exactly
// (Section II.C storage relies on it): for every block component ab with a
// declared parity and every level l, t(.., -r_l, ..)[ab] must equal
// t(.., r_l, ..)[ab] (EVEN) or its negation (ODD) at every offset; bit l of
// flags[ab] is set where it does not. The offset -r_l sits at index
// 2(n_l - 1) - i_l of the index i_l of r_l.
struct ParityCheck {
  int d;
  int nab;
  int64_t st[kMaxD];       // strides of the offset array per level
  int64_t ext[kMaxD];      // extents 2 n_l - 1
  int8_t par[16 * kMaxD];  // [(a*b + c)*d + l]
};

__global__ void __launch_bounds__(256) k_parity_check(const double2* __restrict__ coeffs, int64_t ncoef,
                                                      ParityCheck pc, unsigned* flags) {
  __shared__ unsigned wg[16];
  if (threadIdx.x < 16) wg[threadIdx.x] = 0;
  __syncthreads();
  const int64_t total = ncoef * pc.nab;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int ab = (int)(idx / ncoef);
    const int64_t e = idx - (int64_t)ab * ncoef;
    const double2 v = coeffs[idx];
    unsigned bits = 0;
    for (int l = 0; l < pc.d; ++l) {
      const int pr = pc.par[ab * pc.d + l];
      if (pr == SFFT_PARITY_NONE) continue;
      const int64_t il = (e / pc.st[l]) % pc.ext[l];
      const int64_t mirror = e + (pc.ext[l] - 1 - 2 * il) * pc.st[l];
      const double2 w = coeffs[(int64_t)ab * ncoef + mirror];
      const bool ok = pr == SFFT_PARITY_EVEN ? (w.x == v.x && w.y == v.y) : (w.x == -v.x && w.y == -v.y);
      if (!ok) bits |= 1u << l;
    }
    if (bits) atomicOr(&wg[ab], bits);
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)pc.nab && wg[threadIdx.x]) atomicOr(&flags[threadIdx.x], wg[threadIdx.x]);
}

unsigned grid_for(int64_t total, int block = 256) {
  int64_t g = (total + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace


// Scratch of sfft_apply_noalloc: a file-scope device array (each device holds
// its own copy, in the library's code object, for the life of the process).
// Host code never uses the array's name as an address: the device address
// comes from hipGetSymbolAddress, once per device with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of the current device's scratch array (looked up once per device).
sfft_status noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SFFT_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(SFFT_HIP_ERROR, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SFFT_OK;
}

}  // namespace

namespace {

int64_t vec_elems(const sfft_plan_s* p, int64_t nrhs) { return nrhs * p->b * p->s; }

// Slab schedule: level-1 indices per slab, so that one slab vector (all
// right-hand sides and components, those level-1 indices) is about the target
// size (SFFT_SLAB_MB, default 48 MB) and its leaf pencils start on tile
// boundaries.
int64_t slab_rows(const sfft_plan_s* p, int64_t nrhs) {
  double target = 48.0 * (1 << 20);
  const char* env = std::getenv("SFFT_SLAB_MB");
  if (env && std::atof(env) > 0) target = std::atof(env) * (1 << 20);
  const int64_t L0 = p->L[0];
  const int64_t row = p->s / L0;  // entries of one level-1 index of one vector
  int64_t cc = (int64_t)(target / ((double)nrhs * p->b * row * p->esz));
  const int64_t ppr = p->npen / L0, PL = p->ops[p->d - 1]->PL;
  int64_t gcd = PL, r = ppr;
  while (r) {
    const int64_t t = gcd % r;
    gcd = r;
    r = t;
  }
  const int64_t step = PL / gcd;  // cc * ppr must be a multiple of PL
  cc = cc < step ? step : cc / step * step;
  return cc > L0 ? L0 : cc;
}

size_t workspace_elems(const sfft_plan_s* p, int64_t nrhs) {
  const int64_t V = vec_elems(p, nrhs);
  if (p->method == SFFT_EMBED) return (size_t)((int64_t(1) << p->d) * V);
  if (p->d == 1) return 0;
  if (p->sched == SFFT_SCHED_SLAB && p->d >= 3) {
    const int64_t Vs = V / p->L[0] * slab_rows(p, nrhs);
    return (size_t)(V + (p->d - 1) * Vs);  // the odd child, then the slab's (d - 1) vectors
  }
  if (p->sched == SFFT_SCHED_DEPTH || p->sched == SFFT_SCHED_SLAB) return (size_t)((p->d - 1) * V);
  return (size_t)(((int64_t(1) << p->d) - 2) * V);
}

// The part of the vectors one product works on: all of them, or (out-of-core
// apply) a slab of len0 consecutive level-1 indices, whose leaf pencils are
// npen consecutive pencils from global pencil pen0 (a tile boundary).
struct Slab {
  int64_t len0;     // entries along level 1 (L_0 for whole vectors)
  int64_t pen0;     // global index of the slab's first leaf pencil
  int64_t npen;     // leaf pencils per component per right-hand side
  int first_level;  // level the depth-first walk starts at (0-based)
};

Slab whole(const sfft_plan_s* p) { return Slab{p->L[0], 0, p->npen, 0}; }

// Pass geometry of level l (0-based) for vectors (nv, len0, L_1, ..., L_{d-1}).
void level_geom(const sfft_plan_s* p, int l, int64_t nv, int64_t& outer, int64_t& inner, int64_t len0) {
  outer = nv;
  for (int m = 0; m < l; ++m) outer *= m == 0 ? len0 : p->L[m];
  inner = 1;
  for (int m = l + 1; m < p->d; ++m) inner *= p->L[m];
}

PassArgs base_args(const sfft_plan_s* p, int l, int64_t nv, int64_t len0) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  level_geom(p, l, nv, a.outer, a.inner, len0);
  a.tw = p->tw[l];
  a.len = p->L[l];
  a.nq = 1;
  a.tile_mode = p->tile_mode[l];
  return a;
}

hipEvent_t take_event(sfft_plan_s* p) {
  if (!p->prof_free.empty()) {
    hipEvent_t e = p->prof_free.back();
    p->prof_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// RAII bracket: records an event pair around one launch when its kind is profiled.
// Set while sfft_apply_noalloc runs on this thread: the profiling hooks then
// record nothing (taking an event may create one).
thread_local bool g_noalloc = false;

struct ProfScope {
  sfft_plan_s* p;
  hipStream_t st;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(const sfft_plan_s* pc, int k, hipStream_t s) : p(const_cast<sfft_plan_s*>(pc)), st(s), kind(k) {
    if (!g_noalloc && (p->prof_mask & (1u << k))) {
      {
        std::lock_guard<std::mutex> g(p->prof_mu);
        a = take_event(p);
        b = take_event(p);
      }
      if (a && b) (void)hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (!a && !b) return;
    if (a && b) (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> g(p->prof_mu);
    if (a && b) {
      p->prof_recs.push_back({kind, a, b});
    } else {
      if (a) p->prof_free.push_back(a);
      if (b) p->prof_free.push_back(b);
    }
  }
};

sfft_status run_pass(const sfft_plan_s* p, int l, int mode, const PassArgs& a, hipStream_t st) {
  const AxisOps* o = p->ops[l];
  ProfScope ps(p, mode == 0 ? SFFT_KIND_FORWARD : SFFT_KIND_INVERSE, st);
  hipError_t e = (l == p->d - 1) ? o->contig[mode](a, st) : o->strided[mode](a, st);
  if (e != hipSuccess) return hip_fail(e, "axis pass launch");
  return SFFT_OK;
}

// Leaf pass over branches q0 .. q0+nq-1 of levels 1..d-1 (q0 only matters
// for the symbols: its bits are the branch's parities).
// Leaf launch arguments over branches q0 .. q0+nq-1 of levels 1..d-1 (q0 only
// matters for the symbols: its bits are the branch's parities) and the
// kernels that take them (a single launch, and the grouped launch's prep and
// launch functions where the length has them).
sfft_status leaf_args(const sfft_plan_s* p, const void* in, void* out, int64_t in_bs, int64_t nq, int64_t q0,
                      int64_t nrhs, bool adj, const Slab& sl, PassArgs* ap, LeafSel* sel) {
  const int l = p->d - 1;
  const AxisOps* o = p->ops[l];
  PassArgs& a = *ap;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.in_bs = in_bs;
  a.out_bs = in_bs;
  a.nq = nq;
  a.tw = p->tw[l];
  a.len = p->L[l];
  a.npen = sl.npen;
  a.nrhs = nrhs;
  a.ntiles = (sl.npen + o->PL - 1) / o->PL;
  a.pen0 = sl.pen0;
  a.tile0 = sl.pen0 / o->PL;
  a.sym_ntiles = p->ntiles;
  // right-hand sides per workgroup: they share each symbol load
  int rb = 1;
  if (p->rb_pref > 0) {
    rb = p->rb_pref < o->RBMAX ? p->rb_pref : o->RBMAX;
  } else {
    while (rb < nrhs && rb < o->RBMAX) rb *= 2;
  }
  a.rb = rb;
  const void* sym = adj ? p->sym_adj : p->sym;
  *sel = LeafSel{};
  if (p->compressed) {
    a.sym = sym;
    a.sym_bs = 0;
    a.q0 = q0;
    a.d = p->d;
    for (int m = 0; m < p->d; ++m) {
      a.mn[m] = p->n[m];
      a.mst[m] = p->mst[m];
      if (m + 1 < p->d) a.mfd[m] = sfft::FastDiv::make((uint32_t)p->n[m]);
    }
    a.mcomp = p->mcomp;
    for (int k = 0; k < p->ns; ++k) a.odd[k] = adj ? p->odd_adj[k] : p->odd[k];
    sel->single = o->leaf_mirror[p->b].f[p->bsym];
    sel->prep = o->leaf_group_mirror[p->b].prep[p->bsym];
    sel->group = o->leaf_group_mirror[p->b].group[p->bsym];
  } else {
    a.sym = (const char*)sym + (size_t)(q0 * p->sym_bs) * p->esz;
    a.sym_bs = p->sym_bs;
    sel->single = o->leaf[p->b].f[p->method == SFFT_SPLIT ? 2 : 1][p->bsym];
    if (p->method == SFFT_SPLIT) {
      sel->prep = o->leaf_group[p->b].prep[p->bsym];
      sel->group = o->leaf_group[p->b].group[p->bsym];
    }
  }
  if (!sel->single) return fail(SFFT_UNSUPPORTED, "no leaf kernel for this block size");
  return SFFT_OK;
}

sfft_status run_leaf(const sfft_plan_s* p, const void* in, void* out, int64_t in_bs, int64_t nq, int64_t q0,
                     int64_t nrhs, hipStream_t st, bool adj, const Slab& sl) {
  PassArgs a;
  LeafSel sel;
  sfft_status s = leaf_args(p, in, out, in_bs, nq, q0, nrhs, adj, sl, &a, &sel);
  if (s != SFFT_OK) return s;
  ProfScope ps(p, SFFT_KIND_LEAF, st);
  hipError_t e = sel.single(a, st);
  if (e != hipSuccess) return hip_fail(e, "leaf launch");
  return SFFT_OK;
}

// Depth-first (Algorithm 1 order): src holds the branch after levels < l were
// transformed; dst receives that branch's merged result. Level l's odd child
// lives in workspace vector l - sl.first_level (levels 0-based).
sfft_status split_depth(const sfft_plan_s* p, int l, const void* src, void* dst, int64_t q, int64_t nrhs,
                        char* ws, hipStream_t st, bool adj, const Slab& sl) {
  const int64_t nv = nrhs * p->b;
  const int64_t V = nv * (p->s / p->L[0]) * sl.len0;
  if (l == p->d - 1) return run_leaf(p, src, dst, V, 1, q, nrhs, st, adj, sl);
  // the odd child of level l lives in workspace vector l - first_level
  void* odd = ws + (size_t)(l - sl.first_level) * V * p->esz;
  PassArgs a = base_args(p, l, nv, sl.len0);
  a.in = src;
  a.out = dst;
  a.out1 = odd;
  a.use_phase = 1;
  sfft_status s = run_pass(p, l, 0, a, st);
  if (s != SFFT_OK) return s;
  if ((s = split_depth(p, l + 1, dst, dst, 2 * q, nrhs, ws, st, adj, sl)) != SFFT_OK) return s;
  if ((s = split_depth(p, l + 1, odd, odd, 2 * q + 1, nrhs, ws, st, adj, sl)) != SFFT_OK) return s;
  PassArgs b = base_args(p, l, nv, sl.len0);
  b.in = dst;
  b.in1 = odd;
  b.out = dst;
  b.use_phase = 1;
  return run_pass(p, l, 1, b, st);
}

// One device's share when the product is split over 2^k devices by branch
// (after the splits of levels 1..k the branches are independent; Section II
// remarks that by linearity a branch may run on to a chosen termination
// point): along levels l < k only the child whose parity is bit l of prefix is
// formed and, on the way back, merged alone (the even child's inverse, or
// conj(Phi) times the odd child's); the subtree below level k runs
// depth-first with its odd children in workspace vectors 0 .. d-2-k. The
// 2^k shares sum to T x.
sfft_status split_prefix(const sfft_plan_s* p, int l, int k, uint32_t prefix, const void* src, void* dst,
                         int64_t q, int64_t nrhs, char* ws, hipStream_t st) {
  if (l == k) return split_depth(p, l, src, dst, q, nrhs, ws, st, false, Slab{p->L[0], 0, p->npen, k});
  const int par = (int)((prefix >> l) & 1u);
  const int64_t nv = nrhs * p->b;
  PassArgs a = base_args(p, l, nv, p->L[0]);
  a.in = src;
  a.out = par ? nullptr : dst;
  a.out1 = par ? dst : nullptr;
  a.use_phase = 1;
  sfft_status s = run_pass(p, l, 0, a, st);
  if (s != SFFT_OK) return s;
  if ((s = split_prefix(p, l + 1, k, prefix, dst, dst, 2 * q + par, nrhs, ws, st)) != SFFT_OK) return s;
  PassArgs b = base_args(p, l, nv, p->L[0]);
  b.in = dst;
  b.out = dst;
  b.use_phase = 1;
  b.in_odd = par;
  return run_pass(p, l, 1, b, st);
}

size_t subtree_workspace_elems(const sfft_plan_s* p, int k, int64_t nrhs) {
  return (size_t)((p->d - 1 - k) * vec_elems(p, nrhs));
}

// Slab schedule (d >= 3): level 1 over whole vectors; then, for each child
// and each slab of cc consecutive level-1 indices, the level-2 forward pass
// reads the slab straight from the child (one branch per vector, stride one
// vector) into two compact slab vectors, levels 3..d run depth-first on
// those (the out-of-core slab walk), and the level-2 inverse pass writes the
// merged slab back into the child. The slab vectors are small enough to stay
// in the memory-side cache between these launches, so only the child's read
// and write and the symbols cross HBM below level 1.
sfft_status split_slab(const sfft_plan_s* p, const void* x, void* y, int64_t nrhs, char* ws, hipStream_t st,
                       bool adj) {
  const int64_t nv = nrhs * p->b;
  const int64_t V = vec_elems(p, nrhs);
  const int64_t L0 = p->L[0];
  const int64_t row = p->s / L0;
  const int64_t cc = slab_rows(p, nrhs);
  const int64_t ppr = p->npen / L0;
  const size_t esz = p->esz;
  char* odd = ws;
  char* g0 = ws + (size_t)V * esz;
  char* g1 = g0 + (size_t)(nv * cc * row) * esz;
  char* deep = g1 + (size_t)(nv * cc * row) * esz;
  PassArgs a = base_args(p, 0, nv, L0);
  a.in = x;
  a.out = y;
  a.out1 = odd;
  a.use_phase = 1;
  sfft_status s = run_pass(p, 0, 0, a, st);
  if (s != SFFT_OK) return s;
  for (int c1 = 0; c1 < 2; ++c1) {
    char* child = c1 ? odd : (char*)y;
    for (int64_t j0 = 0; j0 < L0; j0 += cc) {
      const int64_t c = L0 - j0 < cc ? L0 - j0 : cc;
      const int64_t Vs = nv * c * row;  // entries of one compact slab vector
      PassArgs f = base_args(p, 1, 1, c);
      f.in = child + (size_t)(j0 * row) * esz;
      f.in_bs = p->s;  // branch q = vector q
      f.nq = nv;
      f.out = g0;
      f.out1 = g1;
      f.out_bs = c * row;
      f.use_phase = 1;
      if ((s = run_pass(p, 1, 0, f, st)) != SFFT_OK) return s;
      const Slab sl{c, j0 * ppr, c * ppr, 2};
      if ((s = split_depth(p, 2, g0, g0, 2 * c1, nrhs, deep, st, adj, sl)) != SFFT_OK) return s;
      if ((s = split_depth(p, 2, g1, g1, 2 * c1 + 1, nrhs, deep, st, adj, sl)) != SFFT_OK) return s;
      PassArgs v = base_args(p, 1, 1, c);
      v.in = g0;
      v.in1 = g1;
      v.in_bs = c * row;
      v.nq = nv;
      v.out = child + (size_t)(j0 * row) * esz;
      v.out_bs = p->s;
      v.use_phase = 1;
      if ((s = run_pass(p, 1, 1, v, st)) != SFFT_OK) return s;
      (void)Vs;
    }
  }
  PassArgs b = base_args(p, 0, nv, L0);
  b.in = y;
  b.in1 = odd;
  b.out = y;
  b.use_phase = 1;
  return run_pass(p, 0, 1, b, st);
}

// Breadth-first: level l's 2^(l+1) branch vectors live contiguously in
// workspace block l (branch index C-order over the parities of levels 0..l).
sfft_status split_breadth(const sfft_plan_s* p, const void* x, void* y, int64_t nrhs, char* ws,
                          hipStream_t st, bool adj) {
  const int d = p->d;
  const int64_t V = vec_elems(p, nrhs);
  const int64_t nv = nrhs * p->b;
  if (d == 1) return run_leaf(p, x, y, V, 1, 0, nrhs, st, adj, whole(p));
  char* blk[kMaxD];
  size_t off = 0;
  for (int l = 0; l < d - 1; ++l) {
    blk[l] = ws + off * p->esz;
    off += (size_t)(int64_t(2) << l) * V;
  }
  sfft_status s;
  for (int l = 0; l < d - 1; ++l) {
    PassArgs a = base_args(p, l, nv, p->L[0]);
    a.in = l == 0 ? x : (const void*)blk[l - 1];
    a.in_bs = V;
    a.nq = int64_t(1) << l;
    a.out = blk[l];
    a.out1 = blk[l] + V * p->esz;
    a.out_bs = 2 * V;
    a.use_phase = 1;
    if ((s = run_pass(p, l, 0, a, st)) != SFFT_OK) return s;
  }
  if ((s = run_leaf(p, blk[d - 2], blk[d - 2], V, int64_t(1) << (d - 1), 0, nrhs, st, adj, whole(p))) != SFFT_OK)
    return s;
  for (int l = d - 2; l >= 0; --l) {
    PassArgs a = base_args(p, l, nv, p->L[0]);
    a.in = blk[l];
    a.in1 = blk[l] + V * p->esz;
    a.in_bs = 2 * V;
    a.nq = int64_t(1) << l;
    a.out = l == 0 ? y : (void*)blk[l - 1];
    a.out_bs = V;
    a.use_phase = 1;
    if ((s = run_pass(p, l, 1, a, st)) != SFFT_OK) return s;
  }
  return SFFT_OK;
}

// Standard circulant embedding: pad, transform every level of the 2^d-times
// larger vector, block multiply, inverse transforms, project.
sfft_status embed_apply(const sfft_plan_s* p, const void* x, void* y, int64_t nrhs, char* ws, hipStream_t st,
                        bool adj) {
  const int d = p->d;
  const int64_t nv = nrhs * p->b;
  Dims dm;
  dm.d = d;
  for (int l = 0; l < d; ++l) dm.n[l] = p->n[l];
  const int64_t big = nv * p->s * (int64_t(1) << d);
  const bool idx32 = big < (int64_t(1) << 32);
  const PadGeo pg = pad_geo(dm);
  {
    ProfScope ps(p, SFFT_KIND_COPY, st);
    const uint32_t npairs = (uint32_t)(big / 2);
    const dim3 g2((npairs + 255) / 256);
    if (idx32 && p->dtype == SFFT_C64)
      hipLaunchKernelGGL(k_pad2<float2>, g2, dim3(256), 0, st, (const float2*)x, (float2*)ws, pg, npairs);
    else if (idx32)
      hipLaunchKernelGGL(k_pad2<double2>, g2, dim3(256), 0, st, (const double2*)x, (double2*)ws, pg, npairs);
    else if (p->dtype == SFFT_C64)
      hipLaunchKernelGGL(k_pad<float2>, dim3(grid_for(big)), dim3(256), 0, st, (const float2*)x, (float2*)ws, dm,
                         big);
    else
      hipLaunchKernelGGL(k_pad<double2>, dim3(grid_for(big)), dim3(256), 0, st, (const double2*)x, (double2*)ws,
                         dm, big);
  }
  HIP_TRY(hipGetLastError(), "pad launch");
  sfft_status s;
  for (int l = 0; l < d - 1; ++l) {
    PassArgs a = base_args(p, l, nv, p->L[0]);
    a.in = ws;
    a.out = ws;
    if ((s = run_pass(p, l, 0, a, st)) != SFFT_OK) return s;
  }
  const int64_t Vbig = big;
  if ((s = run_leaf(p, ws, ws, Vbig, 1, 0, nrhs, st, adj, whole(p))) != SFFT_OK) return s;
  for (int l = d - 2; l >= 0; --l) {
    PassArgs a = base_args(p, l, nv, p->L[0]);
    a.in = ws;
    a.out = ws;
    if ((s = run_pass(p, l, 1, a, st)) != SFFT_OK) return s;
  }
  const int64_t small = nv * p->s;
  {
    ProfScope ps(p, SFFT_KIND_COPY, st);
    const dim3 g1((unsigned)((small + 255) / 256));
    if (idx32 && p->dtype == SFFT_C64)
      hipLaunchKernelGGL(k_project2<float2>, g1, dim3(256), 0, st, (const float2*)ws, (float2*)y, pg,
                         (uint32_t)small);
    else if (idx32)
      hipLaunchKernelGGL(k_project2<double2>, g1, dim3(256), 0, st, (const double2*)ws, (double2*)y, pg,
                         (uint32_t)small);
    else if (p->dtype == SFFT_C64)
      hipLaunchKernelGGL(k_project<float2>, dim3(grid_for(small)), dim3(256), 0, st, (const float2*)ws, (float2*)y,
                         dm, small);
    else
      hipLaunchKernelGGL(k_project<double2>, dim3(grid_for(small)), dim3(256), 0, st, (const double2*)ws,
                         (double2*)y, dm, small);
  }
  HIP_TRY(hipGetLastError(), "project launch");
  return SFFT_OK;
}

// FP64 forward transform of a (2n_0, ..., 2n_{d-1}) array in place.
sfft_status fft64_inplace(const Dims& dm, double2* a, void* const* tw64, hipStream_t st) {
  for (int l = 0; l < dm.d; ++l) {
    const int64_t L = 2 * dm.n[l];
    const AxisOps* o = find_ops(SFFT_C128, L);
    if (!o) return fail(SFFT_UNSUPPORTED, "no FP64 kernels for length " + std::to_string(L));
    PassArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.outer = 1;
    for (int m = 0; m < l; ++m) pa.outer *= 2 * dm.n[m];
    pa.inner = 1;
    for (int m = l + 1; m < dm.d; ++m) pa.inner *= 2 * dm.n[m];
    pa.in = a;
    pa.out = a;
    pa.nq = 1;
    pa.tw = tw64[l];
    pa.len = L;
    hipError_t e = (l == dm.d - 1) ? o->contig[0](pa, st) : o->strided[0](pa, st);
    if (e != hipSuccess) return hip_fail(e, "FP64 symbol transform");
  }
  return SFFT_OK;
}

// Transient device buffers of plan creation, allocated and freed in order on
// its stream (hipFree would wait for all work on the device, including other
// streams' applies); plain hipMalloc / hipFree where the device has no
// stream-ordered pools.
bool pools_supported() {
  static const bool ok = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    return hipDeviceGetAttribute(&v, hipDeviceAttributeMemoryPoolsSupported, dev) == hipSuccess && v != 0;
  }();
  return ok;
}
hipError_t tmp_alloc(void** p, size_t n, hipStream_t st) {
  return pools_supported() ? hipMallocAsync(p, n, st) : hipMalloc(p, n);
}
void tmp_free(void* p, hipStream_t st) {
  if (!p) return;
  if (pools_supported()) (void)hipFreeAsync(p, st);
  else (void)hipFree(p);
}

// The caller's coefficients gathered into the generator of the plan's levels
// (Regather), in stream-ordered scratch the caller frees with tmp_free.
sfft_status regather_coeffs(const Regather& g, int b, const void* coeffs, hipStream_t st, double2** out) {
  *out = nullptr;
  const int64_t total = (int64_t)b * b * g.ncoef_out;
  void* dst = nullptr;
  HIP_TRY(tmp_alloc(&dst, (size_t)total * sizeof(double2), st), "coefficient gather scratch allocation");
  hipLaunchKernelGGL(k_regather, dim3(grid_for(total)), dim3(256), 0, st, (const double2*)coeffs, (double2*)dst,
                     g, total);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    tmp_free(dst, st);
    return hip_fail(e, "coefficient gather launch");
  }
  *out = (double2*)dst;
  return SFFT_OK;
}

// Plan levels (outer to inner) that carry one caller level of size n: n
// itself up to kMaxLevel; otherwise a factor pair, both at most kMaxLevel,
// preferring factors with length-specialised kernels (for the compute dtype
// and for the FP64 symbol generator's 2f points), then the most balanced
// pair; beyond kMaxLevel^2 the largest factor up to kMaxLevel comes off
// first. n has no prime factor above 7, so such factors exist.
std::vector<int64_t> level_factors(int64_t n, int dtype, int method) {
  auto special = [&](int64_t f) {
    const AxisOps* o = find_ops(dtype, method == SFFT_SPLIT ? f : 2 * f);
    const AxisOps* g = find_ops(SFFT_C128, 2 * f);
    return (o && !o->generic ? 1 : 0) + (g && !g->generic ? 1 : 0);
  };
  std::vector<int64_t> f;
  while (n > kMaxLevel) {
    int64_t best = 0, best_score = -1;
    for (int64_t a = 2; a <= kMaxLevel && a < n; ++a) {
      if (n % a) continue;
      const int64_t c = n / a;
      const int64_t score = c <= kMaxLevel ? ((int64_t)1 << 40) + (int64_t)(special(a) + special(c)) * ((int64_t)1 << 32) +
                                                 std::min(a, c)
                                           : a;
      if (score > best_score) {
        best_score = score;
        best = a;
      }
    }
    f.push_back(best);
    n /= best;
  }
  f.push_back(n);
  return f;
}
sfft_status make_table(int dtype, int64_t L, void** out, size_t* bytes, hipStream_t st, bool transient = false) {
  const size_t esz = dtype == SFFT_C64 ? 8 : 16;
  const size_t nb = (size_t)(2 * L) * esz;
  HIP_TRY(transient ? tmp_alloc(out, nb, st) : hipMalloc(out, nb), "twiddle table allocation");
  if (dtype == SFFT_C64)
    hipLaunchKernelGGL(k_twiddle<float2>, dim3(grid_for(2 * L)), dim3(256), 0, st, (float2*)*out, (int)L);
  else
    hipLaunchKernelGGL(k_twiddle<double2>, dim3(grid_for(2 * L)), dim3(256), 0, st, (double2*)*out, (int)L);
  HIP_TRY(hipGetLastError(), "twiddle launch");
  if (bytes) *bytes += nb;
  return SFFT_OK;
}

// Exact block (anti)symmetry of the coefficient array (b, b, 2n_1-1, ...):
// 1 if t[a,c] == t[c,a] at every offset for every pair, 2 if t[a,c] ==
// -t[c,a] everywhere, else 0. SFFT_NO_BLOCK_SYMMETRY=1 reports 0.
sfft_status detect_block_symmetry(const double2* coeffs, int b, int64_t ncoef, hipStream_t st, int* bsym) {
  *bsym = 0;
  const char* env = std::getenv("SFFT_NO_BLOCK_SYMMETRY");
  if (b < 2 || (env && env[0] && env[0] != '0')) return SFFT_OK;
  const int npair = b * (b - 1) / 2;
  unsigned* flags = nullptr;
  HIP_TRY(tmp_alloc((void**)&flags, npair * sizeof(unsigned), st), "symmetry flags allocation");
  std::vector<unsigned> h(npair, 0);
  hipError_t e = hipMemsetAsync(flags, 0, npair * sizeof(unsigned), st);
  if (e == hipSuccess) {
    const dim3 g(grid_for(ncoef));
    if (b == 2) hipLaunchKernelGGL(k_block_symmetry<2>, g, dim3(256), 0, st, coeffs, ncoef, flags);
    else if (b == 3) hipLaunchKernelGGL(k_block_symmetry<3>, g, dim3(256), 0, st, coeffs, ncoef, flags);
    else hipLaunchKernelGGL(k_block_symmetry<4>, g, dim3(256), 0, st, coeffs, ncoef, flags);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), flags, npair * sizeof(unsigned), hipMemcpyDeviceToHost, st);
  tmp_free(flags, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "block symmetry check");
  bool sym = true, anti = true;
  for (unsigned f : h) {
    sym = sym && !(f & 1u);
    anti = anti && !(f & 2u);
  }
  *bsym = sym ? 1 : (anti ? 2 : 0);
  return SFFT_OK;
}

// Checks a declared parity mask against the coefficients (k_parity_check);
// SFFT_INVALID_ARG naming the first (component, level) where it fails.
sfft_status check_parity(const double2* coeffs, int b, int d, const int64_t* n, const int32_t* parity,
                         hipStream_t st) {
  ParityCheck pc;
  std::memset(&pc, 0, sizeof(pc));
  pc.d = d;
  pc.nab = b * b;
  int64_t ncoef = 1;
  for (int l = d - 1; l >= 0; --l) {
    pc.st[l] = ncoef;
    pc.ext[l] = 2 * n[l] - 1;
    ncoef *= 2 * n[l] - 1;
  }
  for (int i = 0; i < b * b * d; ++i) pc.par[i] = (int8_t)parity[i];
  unsigned* flags = nullptr;
  HIP_TRY(tmp_alloc((void**)&flags, 16 * sizeof(unsigned), st), "parity flags allocation");
  unsigned h[16] = {0};
  hipError_t e = hipMemsetAsync(flags, 0, 16 * sizeof(unsigned), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_parity_check, dim3(grid_for(ncoef * b * b)), dim3(256), 0, st, coeffs, ncoef, pc, flags);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, flags, 16 * sizeof(unsigned), hipMemcpyDeviceToHost, st);
  tmp_free(flags, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "parity check");
  for (int ab = 0; ab < b * b; ++ab)
    for (int l = 0; l < d; ++l)
      if (h[ab] & (1u << l))
        return fail(SFFT_INVALID_ARG, "declared parity " +
                                          std::string(parity[ab * d + l] == SFFT_PARITY_EVEN ? "EVEN" : "ODD") +
                                          " of block component (" + std::to_string(ab / b) + ", " +
                                          std::to_string(ab % b) + ") along level " + std::to_string(l + 1) +
                                          " does not hold for the coefficients");
  return SFFT_OK;
}

sfft_status build_symbols(sfft_plan_s* p, const double2* coeffs, hipStream_t st) {
  const int d = p->d;
  Dims dm;
  dm.d = d;
  int64_t full = 1;
  for (int l = 0; l < d; ++l) {
    dm.n[l] = p->n[l];
    full *= 2 * p->n[l];
  }
  void* tw64[kMaxD] = {nullptr};
  double2* tmp = nullptr;
  sfft_status s = SFFT_OK;
  auto cleanup = [&]() {
    for (int l = 0; l < d; ++l) tmp_free(tw64[l], st);
    tmp_free(tmp, st);
    (void)hipStreamSynchronize(st);
  };
  for (int l = 0; l < d && s == SFFT_OK; ++l) s = make_table(SFFT_C128, 2 * p->n[l], &tw64[l], nullptr, st, true);
  if (s == SFFT_OK) {
    hipError_t e = tmp_alloc((void**)&tmp, (size_t)full * sizeof(double2), st);
    if (e != hipSuccess) s = hip_fail(e, "FP64 symbol scratch allocation");
  }
  const double scale = 1.0 / ((double)full);  // 2^-d / prod(n)
  const AxisOps* lo = p->ops[d - 1];
  for (int ks = 0; ks < p->ns && s == SFFT_OK; ++ks) {
    const int ab = p->comp_of[ks];
    hipLaunchKernelGGL(k_embed_generator, dim3(grid_for(full)), dim3(256), 0, st, coeffs, tmp, ab, dm, full);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      s = hip_fail(e, "embed generator launch");
      break;
    }
    if ((s = fft64_inplace(dm, tmp, tw64, st)) != SFFT_OK) break;
    if (p->compressed) {
      const int64_t total = p->mcomp;
      if (p->dtype == SFFT_C64)
        hipLaunchKernelGGL(k_scatter_mirror<float2>, dim3(grid_for(total)), dim3(256), 0, st, tmp, (float2*)p->sym,
                           ks, dm, scale, total, p->mpair, lo->LT, lo->LE, p->mrow);
      else
        hipLaunchKernelGGL(k_scatter_mirror<double2>, dim3(grid_for(total)), dim3(256), 0, st, tmp,
                           (double2*)p->sym, ks, dm, scale, total, p->mpair, lo->LT, lo->LE, p->mrow);
    } else if (p->method == SFFT_SPLIT) {
      const int64_t total = (int64_t(1) << d) * p->ntiles * lo->LE * lo->NTL;
      if (p->dtype == SFFT_C64)
        hipLaunchKernelGGL(k_scatter_split<float2>, dim3(grid_for(total)), dim3(256), 0, st, tmp, (float2*)p->sym,
                           ks, p->ns, dm, lo->LT, lo->LE, lo->NTL, lo->PL, p->ntiles, p->npen, scale, total);
      else
        hipLaunchKernelGGL(k_scatter_split<double2>, dim3(grid_for(total)), dim3(256), 0, st, tmp,
                           (double2*)p->sym, ks, p->ns, dm, lo->LT, lo->LE, lo->NTL, lo->PL, p->ntiles, p->npen,
                           scale, total);
    } else {
      const int64_t total = p->ntiles * lo->LE * lo->NTL;
      if (p->dtype == SFFT_C64)
        hipLaunchKernelGGL(k_scatter_embed<float2>, dim3(grid_for(total)), dim3(256), 0, st, tmp, (float2*)p->sym,
                           ks, p->ns, lo->LT, lo->LE, lo->NTL, lo->PL, p->ntiles, p->npen, p->L[d - 1], scale,
                           total);
      else
        hipLaunchKernelGGL(k_scatter_embed<double2>, dim3(grid_for(total)), dim3(256), 0, st, tmp,
                           (double2*)p->sym, ks, p->ns, lo->LT, lo->LE, lo->NTL, lo->PL, p->ntiles, p->npen,
                           p->L[d - 1], scale, total);
    }
    e = hipGetLastError();
    if (e != hipSuccess) s = hip_fail(e, "symbol scatter launch");
  }
  cleanup();
  if (s == SFFT_OK) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) s = hip_fail(e, "symbol generation");
  }
  return s;
}

// Symbols of T^H from those of T: the generator of T^H is t(-r)^H, whose
// embedded transform is the conjugate transpose of T's at every bin, so the
// parity parts T^H[bId] are conj(T[bId])^T. Stored component k of the adjoint
// is sign * conj(stored component src[k]) of the same (branch, parity, tile)
// block, per_comp entries per component.
struct AdjPerm {
  int src[16];
  int neg[16];
};

template <typename C>
__global__ void k_adjoint_symbols(const C* __restrict__ src, C* __restrict__ dst, int64_t per_comp, int NS,
                                  AdjPerm pm, int64_t total) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = idx / (NS * per_comp);
    const int64_t w = idx - blk * NS * per_comp;
    const int k = (int)(w / per_comp);
    const int64_t r = w - (int64_t)k * per_comp;
    const C v = src[(blk * NS + pm.src[k]) * per_comp + r];
    dst[idx] = pm.neg[k] ? sfft::mk<C>(-v.x, v.y) : sfft::mk<C>(v.x, -v.y);
  }
}

sfft_status build_adjoint(sfft_plan_s* p, hipStream_t st) {
  AdjPerm pm;
  std::memset(&pm, 0, sizeof(pm));
  for (int k = 0; k < p->ns; ++k) {
    const int a = p->comp_of[k] / p->b, c = p->comp_of[k] % p->b;
    pm.src[k] = k;
    if (p->bsym == 0) {  // all b^2 components stored: (a, c) of T^H comes from (c, a) of T
      for (int j = 0; j < p->ns; ++j)
        if (p->comp_of[j] == c * p->b + a) pm.src[k] = j;
    }
    pm.neg[k] = p->bsym == 2;  // t[c, a] = -t[a, c]
    p->odd_adj[k] = p->odd[pm.src[k]];
  }
  const int64_t total = (int64_t)(p->sym_bytes / p->esz);
  const AxisOps* lo = p->ops[p->d - 1];
  const int64_t per_comp = p->compressed ? p->mcomp : (int64_t)lo->LE * lo->NTL;
  if (p->dtype == SFFT_C64)
    hipLaunchKernelGGL(k_adjoint_symbols<float2>, dim3(grid_for(total)), dim3(256), 0, st, (const float2*)p->sym,
                       (float2*)p->sym_adj, per_comp, p->ns, pm, total);
  else
    hipLaunchKernelGGL(k_adjoint_symbols<double2>, dim3(grid_for(total)), dim3(256), 0, st, (const double2*)p->sym,
                       (double2*)p->sym_adj, per_comp, p->ns, pm, total);
  HIP_TRY(hipGetLastError(), "adjoint symbol launch");
  HIP_TRY(hipStreamSynchronize(st), "adjoint symbols");
  return SFFT_OK;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

sfft_status apply_one(sfft_plan_s* p, const void* x, void* y, int64_t nrhs, void* ws, size_t ws_bytes,
                      hipStream_t st, bool adj) {
  if (nrhs < 0) return fail(SFFT_INVALID_ARG, "nrhs must be >= 0");
  if (nrhs == 0) return SFFT_OK;  // empty batch: nothing is read or written
  if (!x || !y) return fail(SFFT_INVALID_ARG, "x and y must be non-null device pointers");
  const size_t vbytes = (size_t)vec_elems(p, nrhs) * p->esz;
  if (ranges_overlap(x, vbytes, y, vbytes)) return fail(SFFT_INVALID_ARG, "y must not overlap x");
  const size_t need = workspace_elems(p, nrhs) * p->esz;
  if (need > 0) {
    if (ws) {
      if (ws_bytes < need)
        return fail(SFFT_INVALID_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
      if (ranges_overlap(ws, need, x, vbytes) || ranges_overlap(ws, need, y, vbytes))
        return fail(SFFT_INVALID_ARG, "workspace overlaps x or y");
    } else {
      std::lock_guard<std::mutex> g(p->pool_mu);
      if (p->pool_bytes < need) {
        if (p->pool) {
          HIP_TRY(hipStreamSynchronize(st), "pool resize sync");
          HIP_TRY(hipFree(p->pool), "pool free");
          p->pool = nullptr;
          p->pool_bytes = 0;
        }
        HIP_TRY(hipMalloc(&p->pool, need), "workspace pool allocation");
        p->pool_bytes = need;
      }
      ws = p->pool;
    }
  }
  if (adj && !p->sym_adj) return fail(SFFT_INVALID_ARG, "adjoint symbols not built (sfft_plan_enable_adjoint)");
  if (p->method == SFFT_EMBED) return embed_apply(p, x, y, nrhs, (char*)ws, st, adj);
  if (p->sched == SFFT_SCHED_SLAB && p->d >= 3) return split_slab(p, x, y, nrhs, (char*)ws, st, adj);
  if ((p->sched == SFFT_SCHED_DEPTH || p->sched == SFFT_SCHED_SLAB) && p->d > 1)
    return split_depth(p, 0, x, y, 0, nrhs, (char*)ws, st, adj, whole(p));
  return split_breadth(p, x, y, nrhs, (char*)ws, st, adj);
}

// Out-of-core apply (the paper's remark on larger systems: the input
// pre-partitioned into even and odd parts that are processed independently).
// After the level-1 split the two children are independent products over
// levels 2..d, and along level 1 (now in the frequency domain) every index
// j_1 is independent too. So, with x, y and the two children in host memory:
//   1. column slabs (all of level 1, a range of the other indices) go to the
//      device, the level-1 forward pass splits them into both children, which
//      return to the host;
//   2. for each child, row slabs (a range of j_1, everything else) go to the
//      device and run levels 2..d depth-first there, results back in place;
//   3. column slabs of both children come back for the level-1 inverse pass
//      and merge, which writes y.
// Device memory holds only slabs (sized from the given budget) and the plan.
struct OocGeom {
  int64_t nv, inner, rowlen;  // vectors, columns per level-1 index, entries per (vector, j_1)
  int64_t w;                  // columns per slab of steps 1 and 3
  int64_t c;                  // level-1 indices per slab of step 2
  size_t dev_bytes;           // device workspace used (all buffers)
  int nbuf;                   // slab buffers: 2 when the budget holds two (copies overlap kernels)
  size_t buf_bytes;           // bytes of one buffer
};

sfft_status ooc_geometry_one(const sfft_plan_s* p, int64_t nrhs, size_t budget, OocGeom* g);

// Two slab buffers when they fit, so one slab's copies overlap the other's
// kernels; else one buffer. A buffer takes half the budget, at most an eighth
// of the vectors' bytes (but 64 MiB at least): with several slabs per step the
// copies and kernels keep overlapping (at 256x256x128 with 8 right-hand sides,
// 194 ms per product with 0.4 GB buffers, 242 ms with 3.2 GB ones).
sfft_status ooc_geometry(const sfft_plan_s* p, int64_t nrhs, size_t budget, OocGeom* g) {
  const size_t vbytes = (size_t)vec_elems(p, nrhs) * p->esz;
  const size_t cap = vbytes / 8 > ((size_t)64 << 20) ? vbytes / 8 : ((size_t)64 << 20);
  size_t half = budget / 2 < cap ? budget / 2 : cap;
  half = half / 256 * 256;  // each buffer 256-byte aligned inside the budget
  if (half > 0 && ooc_geometry_one(p, nrhs, half, g) == SFFT_OK) {
    g->nbuf = 2;
    g->buf_bytes = (g->dev_bytes + 255) / 256 * 256;
    g->dev_bytes = 2 * g->buf_bytes;
    return SFFT_OK;
  }
  sfft_status s = ooc_geometry_one(p, nrhs, budget, g);
  if (s != SFFT_OK) return s;
  g->nbuf = 1;
  g->buf_bytes = g->dev_bytes;
  return SFFT_OK;
}

sfft_status ooc_geometry_one(const sfft_plan_s* p, int64_t nrhs, size_t budget, OocGeom* g) {
  if (p->method != SFFT_SPLIT) return fail(SFFT_UNSUPPORTED, "out-of-core apply needs a split plan");
  if (p->d < 2) return fail(SFFT_UNSUPPORTED, "out-of-core apply needs at least two levels");
  const int64_t esz = (int64_t)p->esz;
  g->nv = nrhs * p->b;
  g->inner = p->s / p->L[0];
  g->rowlen = g->inner;
  // step 1 / 3: an input slab and two output slabs of nv x L_0 x w entries
  const int64_t per_col = 3 * g->nv * p->L[0] * esz;
  g->w = (int64_t)budget / per_col;
  if (g->w > g->inner) g->w = g->inner;
  // step 2: the slab in place plus d - 2 depth-first workspace slabs, each
  // nv x c x rowlen entries; c keeps the slab's first pencil on a tile boundary
  const int64_t per_row = (p->d - 1) * g->nv * g->rowlen * esz;
  const AxisOps* lo = p->ops[p->d - 1];
  const int64_t pen_per_row = p->npen / p->L[0];
  int64_t step = 1;
  while ((step * pen_per_row) % lo->PL) ++step;
  if (step > p->L[0]) step = p->L[0];  // then one slab holds every level-1 index
  g->c = (int64_t)budget / per_row;
  g->c = g->c >= p->L[0] ? p->L[0] : g->c / step * step;
  if (g->w < 1 || g->c < 1)
    return fail(SFFT_INVALID_ARG, "device budget too small for one out-of-core slab: need " +
                                      std::to_string(per_col > per_row * step ? per_col : per_row * step) + " bytes");
  const int64_t b1 = per_col * g->w, b2 = per_row * g->c;
  g->dev_bytes = (size_t)(b1 > b2 ? b1 : b2);
  return SFFT_OK;
}

// 2-D copy of `rows` runs of `width` bytes between pitched buffers
hipError_t copy2d(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t rows,
                  hipMemcpyKind kind, hipStream_t st) {
  if (rows == 0 || width == 0) return hipSuccess;
  return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, kind, st);
}

sfft_status apply_ooc(sfft_plan_s* p, const void* xh, void* yh, int64_t nrhs, void* host_ws, void* dev_ws,
                      const OocGeom& g, hipStream_t st) {
  const size_t esz = p->esz;
  const int64_t L0 = p->L[0];
  const size_t V = (size_t)g.nv * p->s;  // entries of all nrhs vectors
  char* child[2] = {(char*)host_ws, (char*)host_ws + V * esz};
  // slabs alternate between the buffers and streams: slab i uses buffer
  // i % nbuf on `st` (even i) or a second stream (odd i); a step's slabs are
  // independent, so the next slab's copies run beside this one's kernels, and
  // both streams join before the next step reads what this one wrote
  hipStream_t ss[2] = {st, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (g.nbuf == 2) {
    HIP_TRY(hipStreamCreateWithFlags(&ss[1], hipStreamNonBlocking), "out-of-core stream");
    hipError_t e = hipEventCreateWithFlags(&ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[1], hipEventDisableTiming);
    if (e != hipSuccess) {
      for (auto x : ev)
        if (x) (void)hipEventDestroy(x);
      (void)hipStreamDestroy(ss[1]);
      return hip_fail(e, "out-of-core events");
    }
  }
  auto fork = [&]() -> hipError_t {  // the second stream waits for st's work so far
    if (g.nbuf < 2) return hipSuccess;
    hipError_t e = hipEventRecord(ev[0], st);
    return e == hipSuccess ? hipStreamWaitEvent(ss[1], ev[0], 0) : e;
  };
  auto join = [&]() -> hipError_t {  // st waits for the second stream's slabs
    if (g.nbuf < 2) return hipSuccess;
    hipError_t e = hipEventRecord(ev[1], ss[1]);
    return e == hipSuccess ? hipStreamWaitEvent(st, ev[1], 0) : e;
  };
  sfft_status s = SFFT_OK;
  // steps 1 and 3: column slabs [i0, i0 + w) of every (vector, level-1 index) row
  auto column_pass = [&](int mode) -> sfft_status {
    const size_t slab = (size_t)g.nv * L0 * g.w;
    int64_t k = 0;
    for (int64_t i0 = 0; i0 < g.inner; i0 += g.w, ++k) {
      const int b = (int)(k % g.nbuf);
      hipStream_t sk = ss[b];
      char* dev = (char*)dev_ws + (size_t)b * g.buf_bytes;
      char* A = dev;
      char* B = dev + slab * esz;
      char* Cc = dev + 2 * slab * esz;
      const int64_t ww = g.inner - i0 < g.w ? g.inner - i0 : g.w;
      const size_t hp = (size_t)g.inner * esz, dp = (size_t)ww * esz, wid = (size_t)ww * esz;
      const size_t rows = (size_t)g.nv * L0;
      PassArgs a = base_args(p, 0, g.nv, L0);
      a.inner = ww;
      a.nq = 1;
      a.use_phase = 1;
      if (mode == 0) {
        HIP_TRY(copy2d(A, dp, (const char*)xh + i0 * esz, hp, wid, rows, hipMemcpyHostToDevice, sk), "x slab");
        a.in = A;
        a.out = B;
        a.out1 = Cc;
        if ((s = run_pass(p, 0, 0, a, sk)) != SFFT_OK) return s;
        HIP_TRY(copy2d(child[0] + i0 * esz, hp, B, dp, wid, rows, hipMemcpyDeviceToHost, sk), "even slab");
        HIP_TRY(copy2d(child[1] + i0 * esz, hp, Cc, dp, wid, rows, hipMemcpyDeviceToHost, sk), "odd slab");
      } else {
        HIP_TRY(copy2d(A, dp, child[0] + i0 * esz, hp, wid, rows, hipMemcpyHostToDevice, sk), "even slab");
        HIP_TRY(copy2d(B, dp, child[1] + i0 * esz, hp, wid, rows, hipMemcpyHostToDevice, sk), "odd slab");
        a.in = A;
        a.in1 = B;
        a.out = Cc;
        if ((s = run_pass(p, 0, 1, a, sk)) != SFFT_OK) return s;
        HIP_TRY(copy2d((char*)yh + i0 * esz, hp, Cc, dp, wid, rows, hipMemcpyDeviceToHost, sk), "y slab");
      }
    }
    return SFFT_OK;
  };
  // step 2: row slabs of each child through levels 2..d
  auto row_pass = [&]() -> sfft_status {
    const int64_t pen_per_row = p->npen / L0;
    int64_t k = 0;
    for (int c1 = 0; c1 < 2; ++c1) {
      for (int64_t j0 = 0; j0 < L0; j0 += g.c, ++k) {
        const int b = (int)(k % g.nbuf);
        hipStream_t sk = ss[b];
        char* dev = (char*)dev_ws + (size_t)b * g.buf_bytes;
        const int64_t cc = L0 - j0 < g.c ? L0 - j0 : g.c;
        const size_t hp = (size_t)p->s * esz, wid = (size_t)cc * g.rowlen * esz;
        char* S = dev;
        char* ws = dev + (size_t)g.nv * cc * g.rowlen * esz;
        HIP_TRY(copy2d(S, wid, child[c1] + (size_t)j0 * g.rowlen * esz, hp, wid, g.nv, hipMemcpyHostToDevice, sk),
                "child slab in");
        const Slab sl{cc, j0 * pen_per_row, cc * pen_per_row, 1};
        if ((s = split_depth(p, 1, S, S, c1, nrhs, ws, sk, false, sl)) != SFFT_OK) return s;
        HIP_TRY(copy2d(child[c1] + (size_t)j0 * g.rowlen * esz, hp, S, wid, wid, g.nv, hipMemcpyDeviceToHost, sk),
                "child slab out");
      }
    }
    return SFFT_OK;
  };
  auto run = [&]() -> sfft_status {
    HIP_TRY(fork(), "out-of-core fork");
    if ((s = column_pass(0)) != SFFT_OK) return s;
    HIP_TRY(join(), "out-of-core join");
    HIP_TRY(fork(), "out-of-core fork");
    if ((s = row_pass()) != SFFT_OK) return s;
    HIP_TRY(join(), "out-of-core join");
    HIP_TRY(fork(), "out-of-core fork");
    if ((s = column_pass(1)) != SFFT_OK) return s;
    HIP_TRY(join(), "out-of-core join");
    return SFFT_OK;
  };
  s = run();
  // both streams drain before the buffers, events and stream go away
  hipError_t e = hipStreamSynchronize(st);
  if (ss[1]) {
    const hipError_t e1 = hipStreamSynchronize(ss[1]);
    if (e == hipSuccess) e = e1;
    (void)hipStreamDestroy(ss[1]);
  }
  for (auto x : ev)
    if (x) (void)hipEventDestroy(x);
  if (s != SFFT_OK) return s;
  if (e != hipSuccess) return hip_fail(e, "out-of-core apply");
  return SFFT_OK;
}

}  // namespace

// Entry points shared with the batched / autotuning code (plan_internal.hpp).
sfft_status sfft_rt_fail(sfft_status s, const std::string& msg) { return fail(s, msg); }
sfft_status sfft_rt_hip_fail(hipError_t e, const char* what) { return hip_fail(e, what); }
size_t sfft_rt_workspace_elems(const sfft_plan_s* p, int64_t nrhs) { return workspace_elems(p, nrhs); }
sfft_status sfft_rt_apply_one(sfft_plan_s* p, const void* x, void* y, int64_t nrhs, void* ws, size_t ws_bytes,
                              hipStream_t st, bool adj) {
  return apply_one(p, x, y, nrhs, ws, ws_bytes, st, adj);
}
int sfft_rt_leaf_rbmax(const sfft_plan_s* p) { return p->ops[p->d - 1]->RBMAX; }
PassArgs sfft_rt_pass_args(const sfft_plan_s* p, int l, int64_t nv) { return base_args(p, l, nv, p->L[0]); }
sfft_status sfft_rt_leaf_args(const sfft_plan_s* p, const void* in, void* out, int64_t in_bs, int64_t nq,
                              int64_t nrhs, PassArgs* a, LeafSel* sel) {
  return leaf_args(p, in, out, in_bs, nq, 0, nrhs, false, whole(p), a, sel);
}
size_t sfft_rt_breadth_workspace_elems(const sfft_plan_s* p, int64_t nrhs) {
  const int64_t V = vec_elems(p, nrhs);
  if (p->method == SFFT_EMBED) return (size_t)((int64_t(1) << p->d) * V);
  if (p->d == 1) return 0;
  return (size_t)(((int64_t(1) << p->d) - 2) * V);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sfft_status_string(sfft_status s) {
  switch (s) {
    case SFFT_OK: return "SFFT_OK";
    case SFFT_INVALID_ARG: return "SFFT_INVALID_ARG";
    case SFFT_UNSUPPORTED: return "SFFT_UNSUPPORTED";
    case SFFT_OUT_OF_MEMORY: return "SFFT_OUT_OF_MEMORY";
    case SFFT_HIP_ERROR: return "SFFT_HIP_ERROR";
  }
  return "SFFT_UNKNOWN";
}

const char* sfft_last_error(void) { return g_err.c_str(); }

int sfft_length_supported(int64_t L) {
  const AxisOps* o = find_ops(SFFT_C64, L);
  return o == nullptr ? 0 : (o->generic ? 2 : 1);
}

sfft_status sfft_plan_create(sfft_plan* out, int d, const int64_t* n, int b, const void* coeffs, int dtype,
                             int method, const int32_t* parity, int64_t max_nrhs, int schedule, void* stream) {
  g_err.clear();
  if (!out) return fail(SFFT_INVALID_ARG, "out is null");
  *out = nullptr;
  if (!n || !coeffs) return fail(SFFT_INVALID_ARG, "n and coeffs must be non-null");
  if (d < 1) return fail(SFFT_INVALID_ARG, "d must be >= 1");
  if (d > kMaxD) return fail(SFFT_UNSUPPORTED, "d > 6");
  if (b < 1) return fail(SFFT_INVALID_ARG, "b must be >= 1");
  if (b > 4) return fail(SFFT_INVALID_ARG, "block size must be 1, 2, 3 or 4");
  if (dtype != SFFT_C64 && dtype != SFFT_C128) return fail(SFFT_INVALID_ARG, "bad dtype");
  if (method != SFFT_SPLIT && method != SFFT_EMBED) return fail(SFFT_INVALID_ARG, "bad method");
  if (schedule < SFFT_SCHED_AUTO || schedule > SFFT_SCHED_SLAB) return fail(SFFT_INVALID_ARG, "bad schedule");
  if (max_nrhs < 1) return fail(SFFT_INVALID_ARG, "max_nrhs must be >= 1");
  for (int l = 0; l < d; ++l)
    if (n[l] < 1) return fail(SFFT_INVALID_ARG, "level sizes must be >= 1");
  if (parity)
    for (int i = 0; i < b * b * d; ++i)
      if (parity[i] < SFFT_PARITY_NONE || parity[i] > SFFT_PARITY_ODD)
        return fail(SFFT_INVALID_ARG, "bad parity entry");
  // A level of size 1 has the single offset 0: the operator is block Toeplitz
  // over the other levels, with the same memory layout for coefficients and
  // vectors, so such levels are dropped (with their parity entries).
  const int user_d = d;
  const int64_t* user_n = n;
  int64_t n_eff[kMaxD];
  std::vector<int32_t> par_eff;
  {
    int k = 0;
    for (int l = 0; l < d; ++l)
      if (n[l] > 1) n_eff[k++] = n[l];
    if (k == 0) return fail(SFFT_UNSUPPORTED, "every level has size 1 (a single grid point)");
    if (parity) {
      for (int ab = 0; ab < b * b; ++ab)
        for (int l = 0; l < d; ++l)
          if (n[l] > 1) par_eff.push_back(parity[ab * d + l]);
      parity = par_eff.data();
    }
    d = k;
    n = n_eff;
  }
  for (int l = 0; l < d; ++l) {
    int64_t r = n[l];
    for (int f : {2, 3, 5, 7})
      while (r % f == 0) r /= f;
    if (r != 1)
      return fail(SFFT_UNSUPPORTED, "level size " + std::to_string(n[l]) + " has the prime factor " +
                                        std::to_string(r) + " (only 2, 3, 5 and 7 are supported)");
  }
  // levels longer than kMaxLevel: carried as several plan levels (Regather)
  int64_t n_plan[kMaxD];
  int eff_first[kMaxD] = {0};
  Regather rg;
  bool regather = false;
  {
    int dq = 0;
    int64_t wq[kMaxD], cstride[kMaxD];
    int grp[kMaxD];
    for (int e = 0; e < d; ++e) {
      const std::vector<int64_t> f = level_factors(n[e], dtype, method);
      if (f.size() > 1) regather = true;
      if (dq + (int)f.size() > kMaxD)
        return fail(SFFT_UNSUPPORTED, "levels above " + std::to_string(kMaxLevel) +
                                          " are carried as several levels; that makes more than 6");
      eff_first[e] = dq;
      int64_t w = 1;
      for (int k = (int)f.size() - 1; k >= 0; --k) {
        n_plan[dq + k] = f[k];
        wq[dq + k] = w;
        grp[dq + k] = e;
        w *= f[k];
      }
      dq += (int)f.size();
    }
    if (regather) {
      if (parity && method == SFFT_SPLIT)
        return fail(SFFT_UNSUPPORTED, "mirrored storage needs every level size <= " + std::to_string(kMaxLevel));
      int64_t st_in = 1;
      for (int e = d - 1; e >= 0; --e) {
        cstride[e] = st_in;
        st_in *= 2 * n[e] - 1;
      }
      rg.dq = dq;
      rg.ncoef_in = st_in;
      rg.ncoef_out = 1;
      rg.cbase = 0;
      for (int e = 0; e < d; ++e) rg.cbase += (n[e] - 1) * cstride[e];
      for (int q = 0; q < dq; ++q) {
        rg.ext[q] = 2 * n_plan[q] - 1;
        rg.mult[q] = wq[q] * cstride[grp[q]];
        rg.cbase -= (n_plan[q] - 1) * rg.mult[q];
        rg.ncoef_out *= rg.ext[q];
      }
      d = dq;
      n = n_plan;
    }
  }
  for (int l = 0; l < d; ++l) {
    if (n[l] > kMaxLevel)
      return fail(SFFT_UNSUPPORTED, "level size " + std::to_string(n[l]) + " above " + std::to_string(kMaxLevel));
    // the FP64 symbol generator transforms 2 n_l points along level l
    if (!find_ops(SFFT_C128, 2 * n[l]) || !generic_fits(find_ops(SFFT_C128, 2 * n[l]), SFFT_C128, b, 1, false, false))
      return fail(SFFT_UNSUPPORTED, "no kernels for length " + std::to_string(2 * n[l]));
    const int64_t L = method == SFFT_SPLIT ? n[l] : 2 * n[l];
    const AxisOps* o = find_ops(dtype, L);
    const bool leaf = l == d - 1;
    if (!o || !generic_fits(o, dtype, b, method == SFFT_SPLIT ? 2 : 1, leaf, method == SFFT_SPLIT))
      return fail(SFFT_UNSUPPORTED, "level of length " + std::to_string(L) + " needs more LDS than a workgroup has "
                                    "for b = " + std::to_string(b) + " in this dtype");
  }
  bool mirror = false;
  if (parity && method == SFFT_SPLIT) {
    for (int i = 0; i < b * b * d; ++i)
      if (parity[i] == SFFT_PARITY_NONE)
        return fail(SFFT_UNSUPPORTED, "mirrored storage needs every (component, level) even or odd");
    // the leaf addresses one component with 32-bit offsets (a bound: rows of
    // lane pairs hold up to n/2 - 1 more entries along the last level)
    double bytes = dtype == SFFT_C64 ? 8 : 16;
    for (int l = 0; l < d; ++l) bytes *= (double)(l == d - 1 ? n[l] + n[l] / 2 + 1 : n[l] + 1);
    if (bytes >= 4294967296.0)
      return fail(SFFT_UNSUPPORTED, "mirrored storage holds at most 4 GiB per block component");
    sfft_status sp = check_parity((const double2*)coeffs, b, d, n, parity, (hipStream_t)stream);
    if (sp != SFFT_OK) return sp;
    mirror = true;
  }

  sfft_plan_s* p = new sfft_plan_s();
  hipStream_t st = (hipStream_t)stream;
  p->d = d;
  p->user_d = user_d;
  for (int l = 0; l < user_d; ++l) p->user_n[l] = user_n[l];
  p->regather = regather;
  p->rg = rg;
  for (int e = 0; e < kMaxD; ++e) p->eff_first[e] = eff_first[e];
  p->b = b;
  p->dtype = dtype;
  p->method = method;
  p->max_nrhs = max_nrhs;
  p->esz = dtype == SFFT_C64 ? 8 : 16;
  p->s = 1;
  for (int l = 0; l < d; ++l) {
    p->n[l] = n[l];
    p->s *= n[l];
    p->L[l] = method == SFFT_SPLIT ? n[l] : 2 * n[l];
    p->ops[l] = find_ops(dtype, p->L[l]);
  }
  // schedule: Algorithm 1's lazy depth-first order (peak (d+1) vectors with x
  // and y) unless the caller asks otherwise; sfft_plan_autotune switches to
  // breadth-first where that is measurably faster
  p->sched = schedule == SFFT_SCHED_AUTO ? SFFT_SCHED_DEPTH : schedule;
  const AxisOps* lo = p->ops[d - 1];
  p->npen = 1;
  for (int l = 0; l < d - 1; ++l) p->npen *= p->L[l];
  p->ntiles = (p->npen + lo->PL - 1) / lo->PL;
  const int npar = method == SFFT_SPLIT ? 2 : 1;
  // the generator of the plan's levels (the caller's array unless a long
  // level is carried as several); the gathered copy is freed in stream order
  double2* gathered = nullptr;
  if (regather) {
    sfft_status sg = regather_coeffs(rg, b, coeffs, st, &gathered);
    if (sg != SFFT_OK) {
      delete p;
      return sg;
    }
    coeffs = gathered;
  }
  struct GatherFree {
    double2* g;
    hipStream_t st;
    ~GatherFree() { tmp_free(g, st); }
  } gather_free{gathered, st};
  {
    int64_t ncoef = 1;
    for (int l = 0; l < d; ++l) ncoef *= 2 * n[l] - 1;
    sfft_status sb = detect_block_symmetry((const double2*)coeffs, b, ncoef, st, &p->bsym);
    if (sb != SFFT_OK) {
      delete p;
      return sb;
    }
    p->ns = 0;
    for (int a = 0; a < b; ++a)
      for (int c = p->bsym ? a : 0; c < b; ++c) p->comp_of[p->ns++] = a * b + c;
  }
  if (mirror) {
    p->compressed = 1;
    // the length-specialised leaves read a lane's entries m and m + 1 as one
    // 16-byte pair (entries per lane a multiple of 4); the runtime-length
    // leaves keep the plain half rows
    p->mpair = (!lo->generic && lo->LE % 4 == 0) ? 1 : 0;
    p->mrow = p->mpair ? n[d - 1] + lo->LE / 2 : n[d - 1] + 1;
    p->mcomp = 1;
    for (int l = d - 1; l >= 0; --l) {
      p->mst[l] = p->mcomp;
      p->mcomp *= l == d - 1 ? p->mrow : n[l] + 1;
    }
    for (int i = 0; i < b * b * d; ++i) p->parity[i] = parity[i];
    for (int k = 0; k < p->ns; ++k)
      for (int l = 0; l < d; ++l)
        if (parity[p->comp_of[k] * d + l] == SFFT_PARITY_ODD) p->odd[k] |= (uint8_t)(1u << l);
    p->sym_bs = 0;
    p->sym_bytes = (size_t)(p->ns * p->mcomp) * p->esz;
  } else {
    p->sym_bs = (int64_t)npar * p->ntiles * p->ns * lo->LE * lo->NTL;
    const int64_t nbranch = method == SFFT_SPLIT ? (int64_t(1) << (d - 1)) : 1;
    p->sym_bytes = (size_t)(nbranch * p->sym_bs) * p->esz;
  }

  sfft_status s = SFFT_OK;
  for (int l = 0; l < d && s == SFFT_OK; ++l) s = make_table(dtype, p->L[l], &p->tw[l], &p->table_bytes, st);
  if (s == SFFT_OK) {
    hipError_t e = hipMalloc(&p->sym, p->sym_bytes);
    if (e != hipSuccess) s = hip_fail(e, "symbol allocation");
  }
  if (s == SFFT_OK) s = build_symbols(p, (const double2*)coeffs, st);
  if (s != SFFT_OK) {
    delete p;
    return s;
  }
  *out = p;
  return SFFT_OK;
}

sfft_status sfft_plan_update(sfft_plan plan, const void* coeffs, void* stream) {
  if (!plan || !coeffs) return fail(SFFT_INVALID_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  double2* gathered = nullptr;
  if (plan->regather) {
    sfft_status sg = regather_coeffs(plan->rg, plan->b, coeffs, st, &gathered);
    if (sg != SFFT_OK) return sg;
    coeffs = gathered;
  }
  struct GatherFree {
    double2* g;
    hipStream_t st;
    ~GatherFree() { tmp_free(g, st); }
  } gather_free{gathered, st};
  int64_t ncoef = 1;
  for (int l = 0; l < plan->d; ++l) ncoef *= 2 * plan->n[l] - 1;
  int bsym = 0;
  sfft_status s = detect_block_symmetry((const double2*)coeffs, plan->b, ncoef, st, &bsym);
  if (s != SFFT_OK) return s;
  if (bsym != plan->bsym)
    return fail(SFFT_INVALID_ARG, "block symmetry " + std::to_string(bsym) + " differs from the plan's " +
                                      std::to_string(plan->bsym));
  if (plan->compressed) {
    s = check_parity((const double2*)coeffs, plan->b, plan->d, plan->n, plan->parity, st);
    if (s != SFFT_OK) return s;
  }
  s = build_symbols(plan, (const double2*)coeffs, st);
  if (s == SFFT_OK && plan->sym_adj) s = build_adjoint(plan, st);
  return s;
}

sfft_status sfft_workspace_size(sfft_plan plan, int64_t nrhs, size_t* bytes) {
  if (!plan || !bytes) return fail(SFFT_INVALID_ARG, "null argument");
  if (nrhs < 0) return fail(SFFT_INVALID_ARG, "nrhs must be >= 0");
  *bytes = nrhs == 0 ? 0 : workspace_elems(plan, nrhs) * plan->esz;
  return SFFT_OK;
}

sfft_status sfft_apply(sfft_plan plan, const void* x, void* y, int64_t nrhs, void* workspace, size_t ws_bytes,
                       void* stream) {
  if (!plan) return fail(SFFT_INVALID_ARG, "plan is null");
  return apply_one(plan, x, y, nrhs, workspace, ws_bytes, (hipStream_t)stream, false);
}

sfft_status sfft_apply_noalloc(sfft_plan plan, const void* x, void* y, int64_t nrhs, void* stream) {
  if (!plan) return fail(SFFT_INVALID_ARG, "plan is null");
  if (nrhs < 0) return fail(SFFT_INVALID_ARG, "nrhs must be >= 0");
  const size_t need = nrhs == 0 ? 0 : workspace_elems(plan, nrhs) * plan->esz;
  if (need > kNoAllocScratchBytes)
    return fail(SFFT_INVALID_ARG, "sfft_apply_noalloc needs " + std::to_string(need) +
                                      " bytes of workspace; its static scratch holds " +
                                      std::to_string(kNoAllocScratchBytes));
  void* ws = nullptr;
  if (need > 0) {
    sfft_status s = noalloc_scratch(&ws);
    if (s != SFFT_OK) return s;
  }
  g_noalloc = true;
  sfft_status s = apply_one(plan, x, y, nrhs, ws, need, (hipStream_t)stream, false);
  g_noalloc = false;
  return s;
}

sfft_status sfft_ooc_sizes(sfft_plan plan, int64_t nrhs, size_t device_budget, size_t* host_ws_bytes,
                           size_t* device_ws_bytes) {
  if (!plan || !host_ws_bytes || !device_ws_bytes) return fail(SFFT_INVALID_ARG, "null argument");
  if (nrhs < 1) return fail(SFFT_INVALID_ARG, "nrhs must be >= 1");
  OocGeom g;
  sfft_status s = ooc_geometry(plan, nrhs, device_budget, &g);
  if (s != SFFT_OK) return s;
  *host_ws_bytes = 2 * (size_t)vec_elems(plan, nrhs) * plan->esz;
  *device_ws_bytes = g.dev_bytes;
  return SFFT_OK;
}

sfft_status sfft_apply_ooc(sfft_plan plan, const void* x_host, void* y_host, int64_t nrhs, void* host_ws,
                           size_t host_ws_bytes, void* device_ws, size_t device_ws_bytes, void* stream) {
  if (!plan) return fail(SFFT_INVALID_ARG, "plan is null");
  if (nrhs < 0) return fail(SFFT_INVALID_ARG, "nrhs must be >= 0");
  if (nrhs == 0) return SFFT_OK;
  if (!x_host || !y_host || !host_ws || !device_ws) return fail(SFFT_INVALID_ARG, "null pointer");
  OocGeom g;
  sfft_status s = ooc_geometry(plan, nrhs, device_ws_bytes, &g);
  if (s != SFFT_OK) return s;
  const size_t vb = (size_t)vec_elems(plan, nrhs) * plan->esz;
  if (host_ws_bytes < 2 * vb) return fail(SFFT_INVALID_ARG, "host workspace too small: need " + std::to_string(2 * vb));
  if (ranges_overlap(x_host, vb, y_host, vb) || ranges_overlap(host_ws, 2 * vb, x_host, vb) ||
      ranges_overlap(host_ws, 2 * vb, y_host, vb))
    return fail(SFFT_INVALID_ARG, "x, y and the host workspace must not overlap");
  return apply_ooc(plan, x_host, y_host, nrhs, host_ws, device_ws, g, (hipStream_t)stream);
}

sfft_status sfft_workspace_size_subtree(sfft_plan plan, int k, int64_t nrhs, size_t* bytes) {
  if (!plan || !bytes || nrhs < 0) return fail(SFFT_INVALID_ARG, "null plan/bytes or nrhs < 0");
  if (k < 0 || k > plan->d - 1) return fail(SFFT_INVALID_ARG, "k must lie in [0, d - 1]");
  *bytes = subtree_workspace_elems(plan, k, nrhs) * plan->esz;
  return SFFT_OK;
}

sfft_status sfft_apply_subtree(sfft_plan plan, int k, uint32_t prefix, const void* x, void* y, int64_t nrhs,
                               void* workspace, size_t ws_bytes, void* stream) {
  if (!plan) return fail(SFFT_INVALID_ARG, "null plan");
  if (plan->method != SFFT_SPLIT) return fail(SFFT_UNSUPPORTED, "subtree shares need a split plan");
  if (k < 0 || k > plan->d - 1) return fail(SFFT_INVALID_ARG, "k must lie in [0, d - 1]");
  if (k < 32 && (prefix >> k) != 0) return fail(SFFT_INVALID_ARG, "prefix must be below 2^k");
  if (nrhs < 0) return fail(SFFT_INVALID_ARG, "nrhs must be >= 0");
  if (nrhs == 0) return SFFT_OK;
  if (!x || !y) return fail(SFFT_INVALID_ARG, "x and y must be non-null device pointers");
  const size_t vbytes = (size_t)vec_elems(plan, nrhs) * plan->esz;
  if (ranges_overlap(x, vbytes, y, vbytes)) return fail(SFFT_INVALID_ARG, "y must not overlap x");
  const size_t need = subtree_workspace_elems(plan, k, nrhs) * plan->esz;
  if (need > 0) {
    if (!workspace || ws_bytes < need)
      return fail(SFFT_INVALID_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
    if (ranges_overlap(workspace, need, x, vbytes) || ranges_overlap(workspace, need, y, vbytes))
      return fail(SFFT_INVALID_ARG, "workspace overlaps x or y");
  }
  return split_prefix(plan, 0, k, prefix, x, y, 0, nrhs, (char*)workspace, (hipStream_t)stream);
}

sfft_status sfft_plan_enable_adjoint(sfft_plan plan, void* stream) {
  if (!plan) return fail(SFFT_INVALID_ARG, "plan is null");
  if (plan->sym_adj) return SFFT_OK;
  HIP_TRY(hipMalloc(&plan->sym_adj, plan->sym_bytes), "adjoint symbol allocation");
  sfft_status s = build_adjoint(plan, (hipStream_t)stream);
  if (s != SFFT_OK) {
    (void)hipFree(plan->sym_adj);
    plan->sym_adj = nullptr;
  }
  return s;
}

sfft_status sfft_apply_adjoint(sfft_plan plan, const void* x, void* y, int64_t nrhs, void* workspace,
                               size_t ws_bytes, void* stream) {
  if (!plan) return fail(SFFT_INVALID_ARG, "plan is null");
  return apply_one(plan, x, y, nrhs, workspace, ws_bytes, (hipStream_t)stream, true);
}

sfft_status sfft_workspace_size_multi(int nprob, const sfft_plan* plans, const int64_t* nrhs, size_t* bytes) {
  if (nprob < 0 || (nprob > 0 && (!plans || !nrhs)) || !bytes) return fail(SFFT_INVALID_ARG, "null argument");
  size_t total = 0;
  for (int i = 0; i < nprob; ++i) {
    if (!plans[i] || nrhs[i] < 0) return fail(SFFT_INVALID_ARG, "bad problem entry");
    if (nrhs[i] > 0) total += sfft_rt_align256(sfft_rt_breadth_workspace_elems(plans[i], nrhs[i]) * plans[i]->esz);
  }
  *bytes = total;
  return SFFT_OK;
}

sfft_status sfft_plan_info(sfft_plan plan, sfft_info* info) {
  if (!plan || !info) return fail(SFFT_INVALID_ARG, "null argument");
  std::memset(info, 0, sizeof(*info));
  info->d = plan->user_d;
  for (int l = 0; l < plan->user_d; ++l) info->n[l] = plan->user_n[l];
  info->b = plan->b;
  info->dtype = plan->dtype;
  info->method = plan->method;
  info->schedule = plan->sched;
  info->compressed = plan->compressed;
  info->block_symmetry = plan->bsym;
  info->max_nrhs = plan->max_nrhs;
  info->symbol_bytes = plan->sym_bytes;
  info->table_bytes = plan->table_bytes;
  info->workspace_bytes = workspace_elems(plan, plan->max_nrhs) * plan->esz;
  info->vector_elems = plan->b * plan->s;
  info->adjoint_symbol_bytes = plan->sym_adj ? plan->sym_bytes : 0;
  for (int l = 0, e = 0; l < plan->user_d; ++l)  // levels of size 1 have no pass
    if (plan->user_n[l] > 1) info->tile_mode[l] = plan->tile_mode[plan->eff_first[e++]];
  info->mirror_row = plan->compressed ? plan->mrow : 0;
  info->plan_d = plan->d;
  for (int l = 0; l < plan->d; ++l) {
    info->plan_n[l] = plan->n[l];
    info->pencil_len[l] = plan->L[l];
    find_radix(plan->dtype, plan->L[l], false, info->radix[l]);
  }
  find_radix(plan->dtype, plan->L[plan->d - 1], true, info->leaf_radix);
  info->peak_bytes = plan->sym_bytes + info->adjoint_symbol_bytes + plan->table_bytes + info->workspace_bytes +
                     2 * (size_t)(plan->max_nrhs * plan->b * plan->s) * plan->esz;
  return SFFT_OK;
}

sfft_status sfft_profile_enable(sfft_plan plan, unsigned mask) {
  if (!plan) return fail(SFFT_INVALID_ARG, "plan is null");
  plan->prof_mask = mask & 0xFu;
  return SFFT_OK;
}

sfft_status sfft_profile_read(sfft_plan plan, int kind, double* total_ms, int64_t* launches, int reset) {
  if (!plan || !total_ms || !launches) return fail(SFFT_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> g(plan->prof_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : plan->prof_recs) {
    if (r.kind != kind) continue;
    HIP_TRY(hipEventSynchronize(r.b), "profile event sync");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b), "profile elapsed time");
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  if (reset) {
    std::vector<sfft_plan_s::Rec> keep;
    for (auto& r : plan->prof_recs) {
      if (r.kind == kind) {
        plan->prof_free.push_back(r.a);
        plan->prof_free.push_back(r.b);
      } else {
        keep.push_back(r);
      }
    }
    plan->prof_recs.swap(keep);
  }
  return SFFT_OK;
}

sfft_status sfft_plan_destroy(sfft_plan plan) {
  if (!plan) return fail(SFFT_INVALID_ARG, "plan is null");
  sfft_rt_forget_plan(plan);
  delete plan;
  return SFFT_OK;
}

}  // extern "C"
