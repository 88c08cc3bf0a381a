// Runtime-length kernels: level sizes n_l (and embedding lengths 2 n_l) with
// prime factors in {2, 3, 5, 7} for which no length-specialised kernels are
// built. They compute exactly what the length-specialised passes and leaf
// compute (the Section II.A split on load, Algorithm 1's mulBrn, the merge on
// store), with the pencil length and its radix plan as launch arguments:
//
//   * a pencil tile is staged whole in LDS and transformed there by Stockham
//     autosort stages of radix 8, 4, 2, 3, 5 and 7 that ping-pong between two
//     LDS buffers, one butterfly per thread at a time;
//   * passes: W pencils per workgroup (W from the LDS budget), loads and
//     stores coalesced along the contiguous direction of the tile;
//   * leaf: one workgroup per (branch, pencil, right-hand side), the b input
//     rows kept in LDS while both children are transformed, multiplied by
//     their symbol blocks and transformed back; the odd child's merge adds
//     into the output the even child wrote.
//
// The symbol layout of the leaf is the general one of the length-specialised
// leaf with one lane per pencil: per (branch, parity, pencil) the stored
// components one after another, bins in natural order.
#include <map>
#include <memory>
#include <mutex>

#include "axis_kernels.hpp"

namespace sfft {
namespace {

constexpr int kGenMaxStages = 16;
constexpr int64_t kGenMaxLen = 4096;
constexpr size_t kGenLdsTarget = 48 * 1024;  // per pass workgroup: a few per CU

struct GenPlan {
  int nst;                  // stages
  int rad[kGenMaxStages];   // radix of each stage
  int W;                    // pencils per workgroup (passes)
  int64_t ntile;            // workgroups per branch (passes)
};

// Radices for L: 8 while possible, then 4 or 2, then 3, 5, 7; false when L
// has another prime factor.
bool factor(int64_t L, GenPlan* g) {
  if (L < 2 || L > kGenMaxLen) return false;
  int n = 0;
  int64_t r = L;
  while (r % 8 == 0) { g->rad[n++] = 8; r /= 8; }
  if (r % 4 == 0) { g->rad[n++] = 4; r /= 4; }
  if (r % 2 == 0) { g->rad[n++] = 2; r /= 2; }
  for (int p : {3, 5, 7})
    while (r % p == 0 && n < kGenMaxStages) { g->rad[n++] = p; r /= p; }
  g->nst = n;
  return r == 1;
}

// One Stockham stage of radix R over ncols pencils of length L: butterfly j
// of a pencil reads entries j + r L/R, scales entry r by W_{Ns R}^{r k}
// (k = j mod Ns, conjugated for the inverse) and writes its outputs to
// (j / Ns) Ns R + k + q Ns.
template <typename C, int R, int DIR>
__device__ __forceinline__ void gen_stage(const C* __restrict__ src, C* __restrict__ dst, int L, int Ns, int ncols,
                                          const C* __restrict__ tw) {
  const int NB = L / R;
  const int TWS = L / (Ns * R);
  for (int t = threadIdx.x; t < ncols * NB; t += blockDim.x) {
    const int c = t / NB, j = t - c * NB;
    const int k = j % Ns;
    const C* s = src + c * L;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * NB];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const C w = tw[2 * r * k * TWS];
        v[r] = DIR > 0 ? cmulc(v[r], w) : cmul(v[r], w);
      }
    }
    dft<R, DIR>(v);
    C* d = dst + c * L + (j / Ns) * Ns * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) d[q * Ns] = v[q];
  }
}

// Unnormalised DFT (DIR = -1 forward, +1 inverse) of ncols pencils stored
// one after another in a; b is scratch of the same size. Returns the buffer
// that holds the result (a or b). All threads of the workgroup call it.
template <typename C, int DIR>
__device__ C* gen_fft(C* a, C* b, const GenPlan& g, int L, int ncols, const C* tw) {
  int Ns = 1;
  for (int s = 0; s < g.nst; ++s) {
    switch (g.rad[s]) {
      case 2: gen_stage<C, 2, DIR>(a, b, L, Ns, ncols, tw); break;
      case 3: gen_stage<C, 3, DIR>(a, b, L, Ns, ncols, tw); break;
      case 4: gen_stage<C, 4, DIR>(a, b, L, Ns, ncols, tw); break;
      case 5: gen_stage<C, 5, DIR>(a, b, L, Ns, ncols, tw); break;
      case 7: gen_stage<C, 7, DIR>(a, b, L, Ns, ncols, tw); break;
      default: gen_stage<C, 8, DIR>(a, b, L, Ns, ncols, tw); break;
    }
    __syncthreads();
    C* t = a;
    a = b;
    b = t;
    Ns *= g.rad[s];
  }
  return a;
}

// Axis pass over a tile of W pencils (o, i) of one branch, pencils along the
// axis (outer, L, inner) as in the length-specialised passes.
//   MODE 0 (FWD2): out1 = FFT(Phi .* in) first (out1 must not alias in), then
//                  out = FFT(in) (out may alias in).
//   MODE 1 (INV2): out = iFFT(in) + conj(Phi) .* iFFT(in1)  (in1 may be absent;
//                  without it, in_odd makes out = conj(Phi) .* iFFT(in)).
template <typename Real, int MODE>
__global__ void __launch_bounds__(256) k_gen_pass(PassArgs a, GenPlan g) {
  using C = cx<Real>;
  extern __shared__ __align__(16) unsigned char gen_smem[];
  const int L = (int)a.len;
  const int W = g.W;
  C* A = reinterpret_cast<C*>(gen_smem);
  C* Bf = A + W * L;
  C* X = Bf + W * L;
  const int64_t cols = a.outer * a.inner;
  const int64_t q = blockIdx.x / g.ntile;
  const int64_t col0 = (blockIdx.x - q * g.ntile) * W;
  const int nc = (int)((cols - col0) < W ? (cols - col0) : W);
  const C* tw = (const C*)a.tw;
  // tile entry idx <-> (pencil c, element k): along k for a contiguous axis,
  // along c (neighbouring pencils) for a strided one, so that consecutive
  // threads touch consecutive addresses
  auto decode = [&](int idx, int& c, int& k) {
    if (a.inner == 1) {
      c = idx / L;
      k = idx - c * L;
    } else {
      k = idx / W;
      c = idx - k * W;
    }
  };
  auto goff = [&](int c, int k) -> int64_t {
    const int64_t col = col0 + c;
    const int64_t o = col / a.inner;
    const int64_t i = col - o * a.inner;
    return (o * L + k) * a.inner + i;
  };
  auto load = [&](C* dst, const C* src, bool ph) {
    for (int idx = threadIdx.x; idx < W * L; idx += blockDim.x) {
      int c, k;
      decode(idx, c, k);
      C v = czero<C>();
      if (c < nc) {
        v = src[goff(c, k)];
        if (ph) v = cmul(v, tw[k]);
      }
      dst[c * L + k] = v;
    }
    __syncthreads();
  };
  auto store = [&](C* dst, const C* src) {
    for (int idx = threadIdx.x; idx < W * L; idx += blockDim.x) {
      int c, k;
      decode(idx, c, k);
      if (c < nc) dst[goff(c, k)] = src[c * L + k];
    }
    __syncthreads();
  };
  const C* in = (const C*)a.in + q * a.in_bs;
  if constexpr (MODE == 0) {
    if (a.out1) {
      load(A, in, a.use_phase != 0);
      store((C*)a.out1 + q * a.out_bs, gen_fft<C, -1>(A, Bf, g, L, W, tw));
    }
    if (a.out) {
      load(A, in, false);
      store((C*)a.out + q * a.out_bs, gen_fft<C, -1>(A, Bf, g, L, W, tw));
    }
  } else {
    load(A, in, false);
    C* r1 = gen_fft<C, +1>(A, Bf, g, L, W, tw);
    if (a.in1) {
      load(X, (const C*)a.in1 + q * a.in_bs, false);
      const C* r2 = gen_fft<C, +1>(X, r1 == A ? Bf : A, g, L, W, tw);
      for (int idx = threadIdx.x; idx < W * L; idx += blockDim.x) {
        const int k = idx % L;
        r1[idx] = cadd(r1[idx], a.use_phase ? cmulc(r2[idx], tw[k]) : r2[idx]);
      }
      __syncthreads();
    } else if (a.in_odd) {
      for (int idx = threadIdx.x; idx < W * L; idx += blockDim.x) r1[idx] = cmulc(r1[idx], tw[idx % L]);
      __syncthreads();
    }
    store((C*)a.out + q * a.out_bs, r1);
  }
}

// Leaf of a runtime length: one workgroup per (branch q, pencil, right-hand
// side). Rows in LDS: the b input rows (split only), b working rows and one
// scratch row. Per child p: w[c] = Phi^p .* x[c], forward transforms,
// w[a] <- sum_c S_p[a, c] w[c] per bin, inverse transforms, then
// out[a] (+)= conj(Phi)^p .* w[a].
template <typename Real, int B, int NPAR, bool MIR, int BS>
__global__ void __launch_bounds__(256) k_gen_leaf(PassArgs a, GenPlan g) {
  using C = cx<Real>;
  using BSy = BlockSym<B, BS>;
  constexpr int NS = BSy::NS;
  extern __shared__ __align__(16) unsigned char gen_smem[];
  const int L = (int)a.len;
  C* xr = reinterpret_cast<C*>(gen_smem);
  C* wr = xr + (NPAR == 2 ? B * L : 0);
  C* sc = wr + B * L;
  const int64_t bx = blockIdx.x;
  const int64_t rhs = bx % a.nrhs;
  const int64_t t2 = bx / a.nrhs;
  const int64_t pen = t2 % a.npen;
  const int64_t q = t2 / a.npen;
  const C* tw = (const C*)a.tw;
  const C* in = (const C*)a.in + q * a.in_bs;
  C* out = (C*)a.out + q * a.out_bs;
  auto gpos = [&](int c) -> int64_t { return ((rhs * B + c) * a.npen + pen) * L; };

  // mirrored storage: this pencil fixes the outer levels' stored index and
  // which of them are read mirrored (as in the length-specialised leaf)
  int64_t mbase = 0;
  uint32_t osign = 0, lodd = 0;
  if constexpr (MIR) {
    const int64_t Q = a.q0 + q;
    int64_t rem = a.pen0 + pen;
    uint32_t mbits = 0;
    for (int l = a.d - 2; l >= 0; --l) {
      const int64_t n = a.mn[l];
      const int64_t j = rem % n;
      rem /= n;
      const int pl = (int)((Q >> (a.d - 2 - l)) & 1);
      int64_t jj = j;
      if (2 * j + pl > n) {
        jj = pl ? n - 1 - j : n - j;
        mbits |= 1u << l;
      }
      mbase += (pl * (n / 2 + 1) + jj) * a.mst[l];
    }
    for (int k = 0; k < NS; ++k) {
      const uint32_t odd = a.odd[k];
      osign |= (uint32_t)(__builtin_popcount(mbits & odd) & 1) << k;
      lodd |= ((odd >> (a.d - 1)) & 1u) << k;
    }
  }

  if constexpr (NPAR == 2) {
    for (int idx = threadIdx.x; idx < B * L; idx += blockDim.x) {
      const int c = idx / L, m = idx - c * L;
      xr[idx] = in[gpos(c) + m];
    }
    __syncthreads();
  }
  for (int p = 0; p < NPAR; ++p) {
    for (int idx = threadIdx.x; idx < B * L; idx += blockDim.x) {
      const int c = idx / L, m = idx - c * L;
      if constexpr (NPAR == 2) wr[idx] = p ? cmul(xr[idx], tw[m]) : xr[idx];
      else wr[idx] = in[gpos(c) + m];
    }
    __syncthreads();
    for (int c = 0; c < B; ++c) {
      C* r = gen_fft<C, -1>(wr + c * L, sc, g, L, 1, tw);
      if (r != wr + c * L) {
        for (int m = threadIdx.x; m < L; m += blockDim.x) wr[c * L + m] = sc[m];
        __syncthreads();
      }
    }
    // mulBrn: per bin, the b x b block of child p's symbol times the b spectra
    const C* sp = (const C*)a.sym + q * a.sym_bs + ((int64_t)p * a.sym_ntiles + a.tile0 + pen) * (int64_t)NS * L;
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
      C sv[NS];
      if constexpr (MIR) {
        const bool mir = 2 * m + p > L;
        const int64_t off = mbase + p * (L / 2 + 1) + (mir ? (p ? L - 1 - m : L - m) : m);
        const uint32_t flip = osign ^ (mir ? lodd : 0u);
#pragma unroll
        for (int k = 0; k < NS; ++k) sv[k] = cneg_if(((const C*)a.sym)[k * a.mcomp + off], (flip >> k) & 1u);
      } else {
#pragma unroll
        for (int k = 0; k < NS; ++k) sv[k] = sp[(int64_t)k * L + m];
      }
      C w[B], o[B];
#pragma unroll
      for (int c = 0; c < B; ++c) w[c] = wr[c * L + m];
#pragma unroll
      for (int ar = 0; ar < B; ++ar) {
        C u = czero<C>();
#pragma unroll
        for (int c = 0; c < B; ++c) {
          const C v = cmul(sv[BSy::idx(ar, c)], w[c]);
          u = BSy::neg(ar, c) ? csub(u, v) : cadd(u, v);
        }
        o[ar] = u;
      }
#pragma unroll
      for (int ar = 0; ar < B; ++ar) wr[ar * L + m] = o[ar];
    }
    __syncthreads();
    for (int c = 0; c < B; ++c) {
      C* r = gen_fft<C, +1>(wr + c * L, sc, g, L, 1, tw);
      if (r != wr + c * L) {
        for (int m = threadIdx.x; m < L; m += blockDim.x) wr[c * L + m] = sc[m];
        __syncthreads();
      }
    }
    // merge: out = iFFT(child 0) + conj(Phi) iFFT(child 1); the thread that
    // wrote an entry for child 0 adds child 1 to it
    for (int idx = threadIdx.x; idx < B * L; idx += blockDim.x) {
      const int c = idx / L, m = idx - c * L;
      const C v = wr[idx];
      C* dst = out + gpos(c) + m;
      if (p == 0) *dst = v;
      else *dst = cadd(*dst, cmulc(v, tw[m]));
    }
    __syncthreads();
  }
}

template <typename Real> constexpr size_t esz() { return sizeof(cx<Real>); }

template <typename Real, int MODE> hipError_t launch_gen_pass(const PassArgs& a, hipStream_t s) {
  GenPlan g;
  if (!factor(a.len, &g)) return hipErrorInvalidValue;
  const int nbuf = (MODE == 1 && a.in1) ? 3 : 2;
  const size_t row = (size_t)a.len * esz<Real>();
  int W = (int)(kGenLdsTarget / (nbuf * row));
  W = W < 1 ? 1 : (W > 64 ? 64 : W);
  if ((size_t)W * nbuf * row > kMaxLds) return hipErrorInvalidConfiguration;  // length beyond the LDS
  g.W = W;
  const int64_t cols = a.outer * a.inner;
  g.ntile = (cols + W - 1) / W;
  const int64_t blocks = a.nq * g.ntile;
  if (blocks <= 0) return hipSuccess;
  if (blocks >= kIdx32) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_gen_pass<Real, MODE>), dim3((unsigned)blocks), dim3(256), (size_t)W * nbuf * row, s, a, g);
  return hipGetLastError();
}

template <typename Real, int B, int NPAR, bool MIR = false, int BS = 0>
hipError_t launch_gen_leaf(const PassArgs& a, hipStream_t s) {
  GenPlan g;
  if (!factor(a.len, &g)) return hipErrorInvalidValue;
  g.W = 1;
  g.ntile = 0;
  const size_t smem = (size_t)((NPAR == 2 ? 2 * B : B) + 1) * a.len * esz<Real>();
  if (smem > kMaxLds) return hipErrorInvalidConfiguration;
  const int64_t blocks = a.nq * a.npen * a.nrhs;
  if (blocks <= 0) return hipSuccess;
  if (blocks >= kIdx32) return hipErrorInvalidConfiguration;
  const int nt = a.len >= 256 ? 256 : (a.len >= 128 ? 128 : 64);
  hipLaunchKernelGGL((k_gen_leaf<Real, B, NPAR, MIR, BS>), dim3((unsigned)blocks), dim3(nt), smem, s, a, g);
  return hipGetLastError();
}

template <typename Real, int B> AxisOps::LeafRow gen_leaf_row() {
  AxisOps::LeafRow r{};
  if constexpr (B == 1) {
    for (int bs = 0; bs < 3; ++bs) {
      r.f[1][bs] = launch_gen_leaf<Real, 1, 1>;
      r.f[2][bs] = launch_gen_leaf<Real, 1, 2>;
    }
  } else {
    r.f[1][0] = launch_gen_leaf<Real, B, 1, false, 0>;
    r.f[1][1] = launch_gen_leaf<Real, B, 1, false, 1>;
    r.f[1][2] = launch_gen_leaf<Real, B, 1, false, 2>;
    r.f[2][0] = launch_gen_leaf<Real, B, 2, false, 0>;
    r.f[2][1] = launch_gen_leaf<Real, B, 2, false, 1>;
    r.f[2][2] = launch_gen_leaf<Real, B, 2, false, 2>;
  }
  return r;
}

template <typename Real, int B> AxisOps::MirRow gen_mir_row() {
  AxisOps::MirRow r{};
  if constexpr (B == 1) {
    for (int bs = 0; bs < 3; ++bs) r.f[bs] = launch_gen_leaf<Real, 1, 2, true>;
  } else {
    r.f[0] = launch_gen_leaf<Real, B, 2, true, 0>;
    r.f[1] = launch_gen_leaf<Real, B, 2, true, 1>;
    r.f[2] = launch_gen_leaf<Real, B, 2, true, 2>;
  }
  return r;
}

template <typename Real> std::unique_ptr<AxisOps> make_gen_ops(int64_t L) {
  auto o = std::make_unique<AxisOps>();
  o->L = (int)L;
  o->T = 1;
  o->E = (int)L;
  o->W = 1;
  o->P = 1;
  o->LT = 1;
  o->LE = (int)L;
  o->PL = 1;
  o->NTL = 1;
  o->RBMAX = 1;
  o->strided[0] = o->contig[0] = launch_gen_pass<Real, 0>;
  o->strided[1] = o->contig[1] = launch_gen_pass<Real, 1>;
  o->leaf[1] = gen_leaf_row<Real, 1>();
  o->leaf[2] = gen_leaf_row<Real, 2>();
  o->leaf[3] = gen_leaf_row<Real, 3>();
  o->leaf[4] = gen_leaf_row<Real, 4>();
  o->leaf_mirror[1] = gen_mir_row<Real, 1>();
  o->leaf_mirror[2] = gen_mir_row<Real, 2>();
  o->leaf_mirror[3] = gen_mir_row<Real, 3>();
  o->leaf_mirror[4] = gen_mir_row<Real, 4>();
  o->generic = 1;
  return o;
}

}  // namespace
}  // namespace sfft

// Launch table of the runtime-length kernels for pencil length L (dtype 0:
// complex64, 1: complex128), or NULL when L is below 2, above 4096 or has a
// prime factor outside {2, 3, 5, 7}. Tables are built once and kept.
extern "C" const sfft::AxisOps* sfft_ops_generic(int dtype, int64_t L) {
  sfft::GenPlan g;
  if (!sfft::factor(L, &g)) return nullptr;
  static std::mutex mu;
  static std::map<std::pair<int, int64_t>, std::unique_ptr<sfft::AxisOps>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(dtype, L);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second.get();
  auto ops = dtype == 0 ? sfft::make_gen_ops<float>(L) : sfft::make_gen_ops<double>(L);
  const sfft::AxisOps* p = ops.get();
  cache.emplace(key, std::move(ops));
  return p;
}

// Radices of the runtime-length kernels for pencil length L (passes and leaf
// alike), outermost stage first; returns how many (at most 8), 0 when L has
// no such kernels.
extern "C" int sfft_radix_generic(int64_t L, int* rads) {
  sfft::GenPlan g;
  if (!sfft::factor(L, &g)) return 0;
  int n = 0;
  for (int i = 0; i < g.nst && n < 8; ++i) rads[n++] = g.rad[i];
  return n;
}
