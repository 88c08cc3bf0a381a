// Axis-pass kernels of the split-FFT block-Toeplitz matvec (and of the
// full-embedding baseline and the FP64 symbol generator, which reuse them).
//
// A pass works on a set of branch vectors; inside one branch the data is seen
// as (outer, L, inner): entry (o, k, i) at (o*L + k)*inner + i, and every
// (o, i) is a pencil of length L along the transformed axis.
//
//   FWD2  (Section II.A split, Algorithm 1 FFT_l + sptBrn fused):
//         out  = FFT_L(in)            (even child)
//         out1 = FFT_L(Phi .* in)     (odd child, Phi[k] = exp(-i pi k / L))
//         either output may be absent; in-place (out == in) is allowed.
//   INV2  (Algorithm 1 iFFT_l + mrgBrn fused, unnormalised, the 1/2 and 1/L
//         factors live in the symbols):
//         out = iFFT_L(in) + conj(Phi) .* iFFT_L(in1)      (in1 may be absent)
//         or, with in_odd set and no in1, out = conj(Phi) .* iFFT_L(in)
//         (one device's share of a product split over devices by branch)
//   LEAF  (innermost level: FFT, mulBrn, iFFT and the last merge fused):
//         out[a] = sum_p conj(Phi)^p .* iFFT_L( sum_c S_p[a, c] .* FFT_L(Phi^p .* in[c]) )
//         with p over {0, 1} (split) or {0} (embedding baseline).
//
// Strided passes (inner > 1) take a tile of W consecutive pencils, T lanes
// per pencil (W = 256 / T, or 128 / T for launches of few workgroups); the W
// lanes that hold row k of the tile read and write it as one contiguous run
// in HBM. Contiguous passes (inner = 1, the innermost
// level) stage a tile of whole pencils through LDS so that global loads and
// stores are linear. Launches of many workgroups run their tiles in an
// XCD-contiguous order (PassArgs::xm1, xm2).
#pragma once

#include <type_traits>

#include "fft_engine.hpp"

namespace sfft {

// Division of 32-bit numerators by a fixed divisor d >= 1 with a multiply-high
// and shifts (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
//   n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0),  t = mulhi(m, n).
struct FastDiv {
  uint32_t d, m, s1, s2;
  static FastDiv make(uint32_t d) {
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    FastDiv f;
    f.d = d;
    f.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    return f;
  }
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    const uint32_t t = __umulhi(m, n);
    return (t + ((n - t) >> s1)) >> s2;
  }
};

struct PassArgs {
  const void* in;    // branch q input at in + q*in_bs (elements)
  const void* in1;   // INV2: odd child, same branch stride as in
  void* out;         // branch q output at out + q*out_bs
  void* out1;        // FWD2: odd child, same branch stride as out
  int64_t in_bs;
  int64_t out_bs;
  int64_t nq;        // branches in this launch
  int64_t outer;     // per branch: pencils along the axis are (outer, inner)
  int64_t inner;
  const void* tw;    // 2L entries exp(-i pi m / L)
  int64_t len;       // pencil length L (read by the runtime-length kernels only)
  int use_phase;     // FWD2/INV2: multiply the odd child by Phi / conj(Phi)
  int in_odd;        // INV2 without in1: in is the odd child (out = conj(Phi) .* iFFT(in))
  int tile_mode;     // strided passes: 0 width by rule, 1 full-size, 2 half-size workgroups
  // LEAF only
  const void* sym;   // symbols for branch q at sym + q*sym_bs
  int64_t sym_bs;
  int64_t npen;      // pencils per component per right-hand side
  int64_t nrhs;
  int64_t ntiles;    // ceil(npen / P)
  // a slab of the pencils (out-of-core apply): the launch's pencil 0 is global
  // pencil pen0 = tile0 * P of a plan whose symbols hold sym_ntiles tiles per
  // parity (pen0 = tile0 = 0 and sym_ntiles = ntiles for a whole vector)
  int64_t pen0;
  int64_t tile0;
  int64_t sym_ntiles;
  int rb;            // right-hand sides per workgroup
  // LEAF with mirrored symbol storage (Section II.C): per component a
  // (n_1+1) x ... x (n_d+1) array; along level l the first n_l/2+1 entries
  // are the even bins 2j of the 2n_l lattice, the rest the odd bins 2j+1,
  // j <= n_l/2; a bin m > n_l is read as bin 2n_l - m, negated once per
  // level along which the component is odd.
  int64_t q0;        // branch index of job 0 (its bits are the parities of levels 1..d-1)
  int d;
  int64_t mn[6];     // level sizes
  int64_t mst[6];    // strides of the stored array
  int64_t mcomp;     // stored entries per component
  uint8_t odd[16];   // bit l of odd[k]: stored component k is odd along level l
  FastDiv mfd[6];    // divisions by the level sizes mn[l], l < d - 1
  // filled by the launchers: block and column decoding without 64-bit division
  FastDiv fd_a, fd_b;  // strided: tiles per branch, inner; leaf: rhs groups, tile groups of 8
  int idx32;           // every decoded index fits in 32 bits
  // block order of the strided and contiguous passes (set by their
  // launchers): workgroup b runs work item (b % 8) * xm1 + (b / 8) * xm2.
  // (1, 8) keeps the dispatch order; (grid / 8, 1) gives each XCD one
  // contiguous range of tiles, since workgroups are dispatched round-robin
  // over the 8 XCDs. Items >= nblk (the grid rounded up to a multiple of 8)
  // store nothing. Branch-free, so the work item needs no second round of
  // argument loads.
  uint32_t xm1, xm2, nblk;
  // grouped launches (one launch for the same pass of several problems):
  // this entry's workgroups start at blk_begin (a multiple of 8, so a
  // workgroup's XCD is the same as in a launch of its own)
  uint32_t blk_begin;
};

__device__ __forceinline__ uint32_t work_item(const PassArgs& a, uint32_t bid) {
  return (bid & 7u) * a.xm1 + (bid >> 3) * a.xm2;
}

// Entry of a grouped launch that holds workgroup bid (entries sorted by blk_begin).
__device__ __forceinline__ int find_entry(const PassArgs* __restrict__ tab, int nent, uint32_t bid) {
  int lo = 0, hi = nent - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].blk_begin <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Fills the block order fields for a pass of `blocks` workgroups; returns the grid.
inline int64_t set_block_order(PassArgs& b, int64_t blocks, bool xcd) {
  b.nblk = (uint32_t)blocks;
  if (xcd) {
    const int64_t grid = (blocks + 7) / 8 * 8;
    b.xm1 = (uint32_t)(grid / 8);
    b.xm2 = 1;
    return grid;
  }
  b.xm1 = 1;
  b.xm2 = 8;
  return blocks;
}

// Launch geometry per length.
template <typename Real, int L> struct Geo {
  using Sh = Shape<L>;
  static constexpr int T = Sh::T;
  static constexpr int E = Sh::E;
  static constexpr int NT = 256;                       // strided / contiguous passes
  static constexpr int W = NT / T;                     // strided tile width (pencils, full size)
  static constexpr int P = NT / T;                     // contiguous tile (pencils)
  static constexpr int LP = L + 1;                     // padded LDS row
  static constexpr bool WS = (64 % T) == 0;    // contiguous pass: pencil inside one wavefront
  // Passes of length 128 and more are bound by occupancy (about 170-200
  // VGPRs): they form the split phase Phi[t + T m] = Phi[t] Phi[T m] from one
  // per-lane value and lane-uniform table entries when needed. Shorter passes
  // are bound by latency: they load their E phases up front.
  static constexpr bool PH_ARRAY = L < 128;
  // Leaf kernel: its own radix plan (FP64 lanes hold fewer entries). A tile
  // is PL pencils (SL = PL * LT lanes, one symbol block); a workgroup takes
  // one tile for RB right-hand sides (RB chosen per launch, <= RBMAX).
  using LSh = typename std::conditional<sizeof(Real) == 4 && Shape<L>::E <= 8, Shape<L>, LeafShape<L>>::type;
  static constexpr int LT = LSh::T;
  static constexpr int LE = LSh::E;
  static constexpr int SL = LT >= 64 ? LT : 64;
  static constexpr int PL = SL / LT;
  static constexpr int NTL = SL;  // threads per right-hand side
  static constexpr bool LWS = (64 % LT) == 0;  // leaf: pencil inside one wavefront
  // LDS row of a (pencil, rhs) pair: LLP = LT (mod 32) complex entries, so
  // neighbouring rows start in different banks
  static constexpr int LLP = L + (((LT - L) % 32) + 32) % 32;
  static constexpr int RB_LDS = (int)((64 * 1024) / ((size_t)PL * LLP * sizeof(cx<Real>)));
  static constexpr int THR_CAP = (sizeof(Real) == 8 || L >= 256) ? 256 : 512;  // keeps the VGPR budget
  static constexpr int RB_THR = SL >= THR_CAP ? 1 : THR_CAP / SL;
  static constexpr int RBMAX_ = RB_LDS < RB_THR ? RB_LDS : RB_THR;
  static constexpr int RBMAX = RBMAX_ >= 8 ? 8 : (RBMAX_ >= 4 ? 4 : (RBMAX_ >= 2 ? 2 : 1));
  // LDS rows per (pencil, rhs) lane group: plans with two or more exchanges
  // transform all NPAR*B pencils of a lane in lockstep (one row each); with a
  // single exchange the pencils go one after another through one row, which
  // keeps LDS per workgroup (and so occupancy) low. So do leaves of length
  // 1024 and more, whose six lockstep rows (48 KB per two-wavefront pencil at
  // complex64) would leave about six wavefronts per CU (-11 to -13% on a
  // 1024^2 grid with one row)
  template <int B, int NPAR> static constexpr int leaf_rows() {
    return (LSh::S >= 3 && L < 1024) ? NPAR * B : 1;
  }
  // Leaves of length 128 and more run many wavefronts per SIMD and are bound
  // by instruction throughput: they use the multiply-add butterflies, block
  // product and merge (fewer VALU instructions, longer dependence chains);
  // shorter leaves, bound by latency, keep independent products and adds
  static constexpr bool LFMA = L >= 128;
  // LDS swizzle of the leaf's lockstep rows (fft_engine.hpp, lswz): the
  // complex64 length-128 leaf (32 lanes x 4 entries) had about 40% of its
  // LDS-active cycles in bank conflicts on the radix-4 exchanges; the
  // swizzle takes the leaf from about 1110 to 1010 us at 256x256x128
  // (general and mirrored symbols) without changing its occupancy. Other
  // lengths keep plain rows (no gain measured at length 64)
  static constexpr int LSWZ = (sizeof(Real) == 4 && L == 128 && LWS) ? 1 : 0;
  // mirrored 3x3 block-symmetric leaves of that length need 194 VGPRs with
  // the swizzle unless held to 3 wavefronts per SIMD (164, no spills)
  template <int B, bool MIR, int BS> static constexpr int leaf_waves() {
    return (MIR && B == 3 && BS != 0 && LSWZ) ? 3 : 1;
  }
};

// Stored block components. BS = 0: all B*B components, index a*B + c.
// BS = 1 (t(r)[a,c] = t(r)[c,a] at every offset) and BS = 2 (t(r)[a,c] =
// -t(r)[c,a]): the B(B+1)/2 components a <= c, the product reading (a, c)
// with a > c from (c, a), negated for BS = 2. The symbol inherits the
// relation component by component (the transforms are linear).
template <int B, int BS> struct BlockSym {
  static constexpr int NS = BS == 0 ? B * B : B * (B + 1) / 2;
  static constexpr int idx(int a, int c) {
    if (BS == 0) return a * B + c;
    const int i = a < c ? a : c, j = a < c ? c : a;
    return i * B - i * (i - 1) / 2 + (j - i);
  }
  static constexpr bool neg(int a, int c) { return BS == 2 && a > c; }
};

// Position of symbol entry (block component ab, home index m, lane) inside one
// (branch, parity, tile) block of B*B*E*NT entries. With E even, entries m and
// m+1 of a lane are adjacent so a lane reads them with one 16-byte (c64) or
// 32-byte (c128) load and a wavefront's load is one contiguous run.
__host__ __device__ inline int64_t sym_offset(int ab, int m, int lane, int E, int NT) {
  if (E % 2 == 0) return ((int64_t)(ab * (E / 2) + m / 2) * NT + lane) * 2 + (m & 1);
  return (int64_t)(ab * E + m) * NT + lane;
}

template <typename C> struct PairOf;
template <> struct PairOf<float2> { using type = float4; };
template <> struct PairOf<double2> { using type = double4; };

// ---------------------------------------------------------------------------
// Strided axis: tile of L rows x W = NT / T pencils, lane (c, t) = (tid % W, tid / W).
// ---------------------------------------------------------------------------
template <typename Real, int L, int MODE, int NT>
__device__ __forceinline__ void strided_body(const PassArgs& a, uint32_t bid) {
  using C = cx<Real>;
  using G = Geo<Real, L>;
  using Sh = typename G::Sh;
  constexpr int T = G::T, E = G::E, W = NT / T;
  __shared__ C lds[L * W];
  const int tid = threadIdx.x;
  const int c = tid % W, t = tid / W;
  const int64_t cols = a.outer * a.inner;
  // an item past the end (grid rounded up to 8) works on tile 0 and stores
  // nothing; no early exit, which would hold back the other argument loads
  const uint32_t wi = work_item(a, bid);
  const bool live = wi < a.nblk;
  const uint32_t bx = live ? wi : 0u;
  int64_t q, col, o, i;
  if (a.idx32) {
    const uint32_t bq = a.fd_a.div(bx);
    q = bq;
    col = (int64_t)(bx - bq * a.fd_a.d) * W + c;
    const uint32_t oc = a.fd_b.div((uint32_t)col);
    o = oc;
    i = (uint32_t)col - oc * a.fd_b.d;
  } else {
    const int64_t ntile = (cols + W - 1) / W;
    q = bx / ntile;
    col = (bx % ntile) * W + c;
    o = col / a.inner;
    i = col - o * a.inner;
  }
  const bool act = live && col < cols;
  if (!act) o = i = 0;
  const int64_t base = o * L * a.inner + i;
  const int64_t st = a.inner;
  const C* tw = (const C*)a.tw;
  C* lp = lds + c;
  LaneTw<C, Sh> lt;
  lt.load(t, tw);
  // split phases Phi[t + T m] of this lane's entries (Geo::PH_ARRAY)
  C ph[G::PH_ARRAY ? E : 1];
  if constexpr (G::PH_ARRAY) {
#pragma unroll
    for (int m = 0; m < E; ++m) ph[m] = tw[t + T * m];
  } else {
    ph[0] = tw[t];
  }
  auto phase = [&](int m) -> C {
    if constexpr (G::PH_ARRAY) return ph[m];
    else return m == 0 ? ph[0] : cmul(ph[0], tw[T * m]);
  };
  // loads are unconditional: an inactive column reads column 0 (base is 0
  // there), transforms it in its own LDS column and stores nothing, so no
  // load waits inside a branch
  C h[E];
  if constexpr (MODE == 0) {
    const C* in = (const C*)a.in + q * a.in_bs + base;
#pragma unroll
    for (int m = 0; m < E; ++m) h[m] = in[(t + T * m) * st];
    if (a.out) {
      C w[E];
#pragma unroll
      for (int m = 0; m < E; ++m) w[m] = h[m];
      fft_pencil<-1, Sh>(w, lp, W, t, lt);
      if (act) {
        C* out = (C*)a.out + q * a.out_bs + base;
#pragma unroll
        for (int m = 0; m < E; ++m) out[(t + T * m) * st] = w[m];
      }
    }
    if (a.out1) {
      C w[E];
#pragma unroll
      for (int m = 0; m < E; ++m) w[m] = a.use_phase ? cmul(h[m], phase(m)) : h[m];
      fft_pencil<-1, Sh>(w, lp, W, t, lt);
      if (act) {
        C* out = (C*)a.out1 + q * a.out_bs + base;
#pragma unroll
        for (int m = 0; m < E; ++m) out[(t + T * m) * st] = w[m];
      }
    }
  } else {
    const C* in = (const C*)a.in + q * a.in_bs + base;
#pragma unroll
    for (int m = 0; m < E; ++m) h[m] = in[(t + T * m) * st];
    C w[E];
    if (a.in1) {  // both children requested before either transform
      const C* in1 = (const C*)a.in1 + q * a.in_bs + base;
#pragma unroll
      for (int m = 0; m < E; ++m) w[m] = in1[(t + T * m) * st];
    }
    fft_pencil<+1, Sh>(h, lp, W, t, lt);
    if (a.in1) {
      fft_pencil<+1, Sh>(w, lp, W, t, lt);
#pragma unroll
      for (int m = 0; m < E; ++m) h[m] = cadd(h[m], a.use_phase ? cmulc(w[m], phase(m)) : w[m]);
    } else if (a.in_odd) {
#pragma unroll
      for (int m = 0; m < E; ++m) h[m] = cmulc(h[m], phase(m));
    }
    if (act) {
      C* out = (C*)a.out + q * a.out_bs + base;
#pragma unroll
      for (int m = 0; m < E; ++m) out[(t + T * m) * st] = h[m];
    }
  }
}

template <typename Real, int L, int MODE, int NT>
__global__ void __launch_bounds__(NT) k_strided(PassArgs a) {
  strided_body<Real, L, MODE, NT>(a, blockIdx.x);
}

// The same pass for several problems in one launch (entry table in device memory).
template <typename Real, int L, int MODE, int NT>
__global__ void __launch_bounds__(NT) k_strided_group(const PassArgs* __restrict__ tab, int nent) {
  const int e = find_entry(tab, nent, blockIdx.x);
  strided_body<Real, L, MODE, NT>(tab[e], blockIdx.x - tab[e].blk_begin);
}

// ---------------------------------------------------------------------------
// Contiguous axis helpers: a tile of P whole pencils staged through LDS.
// ---------------------------------------------------------------------------
template <typename C, int L, int P, int NT>
__device__ __forceinline__ void tile_load(C* lds, const C* src, int npen_here, int tid) {
  constexpr int LP = L + 1;
  for (int idx = tid; idx < P * L; idx += NT) {
    const int g = idx / L, k = idx - (idx / L) * L;
    lds[g * LP + k] = (g < npen_here) ? src[idx] : czero<C>();
  }
}

template <typename C, int L, int P, int NT>
__device__ __forceinline__ void tile_store(C* dst, const C* lds, int npen_here, int tid) {
  constexpr int LP = L + 1;
  for (int idx = tid; idx < P * L; idx += NT) {
    const int g = idx / L, k = idx - (idx / L) * L;
    if (g < npen_here) dst[idx] = lds[g * LP + k];
  }
}

// Writes home entries of lane (g, t) to LDS, then the whole tile to dst.
template <typename C, int L, int T, int E, int P, int NT>
__device__ __forceinline__ void store_home(C* dst, C* lds, const C (&h)[E], int g, int t, int npen_here,
                                           int tid) {
  constexpr int LP = L + 1;
#pragma unroll
  for (int m = 0; m < E; ++m) lds[g * LP + t + T * m] = h[m];
  __syncthreads();
  tile_store<C, L, P, NT>(dst, lds, npen_here, tid);
  __syncthreads();
}

template <typename Real, int L, int MODE>
__global__ void __launch_bounds__(256) k_contig(PassArgs a) {
  using C = cx<Real>;
  using G = Geo<Real, L>;
  using Sh = typename G::Sh;
  constexpr int T = G::T, E = G::E, P = G::P, LP = G::LP, NT = G::NT;
  __shared__ C lds[P * LP];
  const int tid = threadIdx.x;
  const int g = tid / T, t = tid % T;
  const uint32_t wi = work_item(a, blockIdx.x);
  const bool live = wi < a.nblk;  // past the end: tile 0, nothing loaded or stored
  const uint32_t bx = live ? wi : 0u;
  int64_t q, p0;
  if (a.idx32) {
    const uint32_t bq = a.fd_a.div(bx);
    q = bq;
    p0 = (int64_t)(bx - bq * a.fd_a.d) * P;
  } else {
    const int64_t ntile = (a.outer + P - 1) / P;
    q = bx / ntile;
    p0 = (bx % ntile) * P;
  }
  const int nh = live ? (int)((a.outer - p0) < P ? (a.outer - p0) : P) : 0;
  const C* tw = (const C*)a.tw;
  C* lp = lds + g * LP;
  LaneTw<C, Sh> lt;
  lt.load(t, tw);
  // split phases Phi[t + T m] of this lane's entries (Geo::PH_ARRAY)
  C ph[G::PH_ARRAY ? E : 1];
  if constexpr (G::PH_ARRAY) {
#pragma unroll
    for (int m = 0; m < E; ++m) ph[m] = tw[t + T * m];
  } else {
    ph[0] = tw[t];
  }
  auto phase = [&](int m) -> C {
    if constexpr (G::PH_ARRAY) return ph[m];
    else return m == 0 ? ph[0] : cmul(ph[0], tw[T * m]);
  };
  C h[E];
  tile_load<C, L, P, NT>(lds, (const C*)a.in + q * a.in_bs + p0 * L, nh, tid);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) h[m] = lp[t + T * m];
  __syncthreads();
  if constexpr (MODE == 0) {
    if (a.out) {
      C w[E];
#pragma unroll
      for (int m = 0; m < E; ++m) w[m] = h[m];
      fft_pencil<-1, Sh, G::WS>(w, lp, 1, t, lt);
      store_home<C, L, T, E, P, NT>((C*)a.out + q * a.out_bs + p0 * L, lds, w, g, t, nh, tid);
    }
    if (a.out1) {
      C w[E];
#pragma unroll
      for (int m = 0; m < E; ++m) w[m] = a.use_phase ? cmul(h[m], phase(m)) : h[m];
      fft_pencil<-1, Sh, G::WS>(w, lp, 1, t, lt);
      store_home<C, L, T, E, P, NT>((C*)a.out1 + q * a.out_bs + p0 * L, lds, w, g, t, nh, tid);
    }
  } else {
    fft_pencil<+1, Sh, G::WS>(h, lp, 1, t, lt);
    if (a.in1) {
      tile_load<C, L, P, NT>(lds, (const C*)a.in1 + q * a.in_bs + p0 * L, nh, tid);
      __syncthreads();
      C w[E];
#pragma unroll
      for (int m = 0; m < E; ++m) w[m] = lp[t + T * m];
      __syncthreads();
      fft_pencil<+1, Sh, G::WS>(w, lp, 1, t, lt);
#pragma unroll
      for (int m = 0; m < E; ++m) h[m] = cadd(h[m], a.use_phase ? cmulc(w[m], phase(m)) : w[m]);
    } else if (a.in_odd) {
#pragma unroll
      for (int m = 0; m < E; ++m) h[m] = cmulc(h[m], phase(m));
    }
    store_home<C, L, T, E, P, NT>((C*)a.out + q * a.out_bs + p0 * L, lds, h, g, t, nh, tid);
  }
}

// ---------------------------------------------------------------------------
// Leaf: innermost level with the b x b diagonal block product (mulBrn).
// Input / output per branch: (nrhs, B, npen, L). Both children of the last
// level are transformed from the same registers (even: x, odd: Phi x),
// multiplied by their symbol blocks, inverse transformed and merged:
//     out = iFFT(S_0 FFT(x)) + conj(Phi) iFFT(S_1 FFT(Phi x)).
// Lane (g, r, t) = tid: pencil g of the tile, right-hand side r of the
// workgroup's RB, lane t of the pencil; the RB lanes of one (g, t) read the
// same symbol addresses in one wavefront instruction, so a symbol block is
// fetched once for all RB right-hand sides. Symbols per (branch, parity,
// tile): [k][m/2][g*T + t][m%2] over the stored block components k
// (BlockSym, sym_offset), or mirrored storage.
// Workgroups of one tile are numbered 8 apart, so all of a tile's
// right-hand-side groups run on the same XCD and share its L2.
// ---------------------------------------------------------------------------
template <typename Real, int L, int B, int NPAR, bool MIR, int BS>
__device__ __forceinline__ void leaf_body(const PassArgs& a, uint32_t bid) {
  using C = cx<Real>;
  using G = Geo<Real, L>;
  using Sh = typename G::LSh;
  using C2 = typename PairOf<C>::type;
  constexpr int T = G::LT, E = G::LE, P = G::PL, LP = G::LLP, SL = G::SL;
  using BSy = BlockSym<B, BS>;
  constexpr int NS = BSy::NS;  // stored block components
  extern __shared__ __align__(16) unsigned char leaf_smem[];
  C* lds = reinterpret_cast<C*>(leaf_smem);
  const int RB = a.rb;
  const int tid = threadIdx.x;
  const int t = tid % T;
  const int gr = tid / T;
  const int rl = gr % RB;
  const int g = gr / RB;
  const int row = g * RB + rl;
  const int64_t lo = bid & 7;
  int64_t rg, tile, q;
  if (a.idx32) {
    const uint32_t t2 = bid >> 3;
    const uint32_t t3 = a.fd_a.div(t2);
    rg = t2 - t3 * a.fd_a.d;
    const uint32_t t4 = a.fd_b.div(t3);
    tile = (int64_t)(t3 - t4 * a.fd_b.d) * 8 + lo;
    q = t4;
  } else {
    const int64_t nrg = (a.nrhs + RB - 1) / RB;
    const int64_t ntiles8 = (a.ntiles + 7) / 8;
    const int64_t t2 = bid >> 3;
    rg = t2 % nrg;
    const int64_t t3 = t2 / nrg;
    tile = (t3 % ntiles8) * 8 + lo;
    q = t3 / ntiles8;
  }
  if (tile >= a.ntiles) return;  // whole workgroup exits together
  const int64_t p0 = tile * P;
  const int nh = (int)((a.npen - p0) < P ? (a.npen - p0) : P);
  const int64_t r0 = rg * RB;
  const int nr = (int)((a.nrhs - r0) < RB ? (a.nrhs - r0) : RB);
  const C* tw = (const C*)a.tw;
  const C* in = (const C*)a.in + q * a.in_bs;
  C* out = (C*)a.out + q * a.out_bs;
  constexpr int NROW = G::template leaf_rows<B, NPAR>();
  C* lp = lds + row * NROW * LP;
  LaneTw<C, Sh> lt;
  lt.load(t, tw);

  // load: every lane reads its own entries k = t + T*m of its pencil for all
  // components at once (runs of T consecutive entries per pencil)
  const bool act = (g < nh) && (rl < nr);
  const int64_t pbase = ((r0 + rl) * B * a.npen + p0 + g) * L + t;  // component 0
  // loads are unconditional: an inactive (pencil, rhs) row reads pencil 0 of
  // right-hand side 0, works on its own LDS row and stores nothing, so no load
  // waits inside a branch
  const int64_t lbase = act ? pbase : t;
  C x[B][E];
#pragma unroll
  for (int c = 0; c < B; ++c)
#pragma unroll
    for (int m = 0; m < E; ++m) x[c][m] = in[lbase + (int64_t)c * a.npen * L + T * m];

  // mirrored storage: this lane's pencil fixes the outer levels' stored index
  // and which of them are read mirrored
  int64_t mbase = 0;
  uint32_t mbits = 0;
  if constexpr (MIR) {
    const int64_t Q = a.q0 + q;
    // multiply-high divisions by the level sizes (mirrored plans keep every
    // component under 4 GiB, so pencil indexes fit in 32 bits)
    uint32_t rem = (uint32_t)(a.pen0 + p0 + (g < nh ? g : 0));
    uint32_t mb = 0;
    for (int l = a.d - 2; l >= 0; --l) {
      const uint32_t n = a.mfd[l].d;
      const uint32_t qt = a.mfd[l].div(rem);
      const uint32_t j = rem - qt * n;
      rem = qt;
      const uint32_t pl = (uint32_t)((Q >> (a.d - 2 - l)) & 1);
      uint32_t jj = j;
      if (2 * j + pl > n) {
        jj = pl ? n - 1 - j : n - j;
        mbits |= 1u << l;
      }
      mb += (pl * (n / 2 + 1) + jj) * (uint32_t)a.mst[l];
    }
    mbase = mb;
  }
  const int slane = g * T + t;  // lane inside the symbol block
  // mirrored storage: bit k of osign is set when stored component k enters
  // this lane's pencil negated through the outer levels' mirrors; bit k of
  // lodd when component k is odd along the last level (lane-uniform)
  uint32_t osign = 0, lodd = 0;
  if constexpr (MIR) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t odd = a.odd[k];
      osign |= (uint32_t)(__builtin_popcount(mbits & odd) & 1) << k;
      lodd |= ((odd >> (a.d - 1)) & 1u) << k;
    }
  }

  // symbols requested ahead: parity 0, entries 0..3, before the forward
  // transforms; parity 1, entries 0 and 1, before parity 0's product
  constexpr int MSP = (E % 2 == 0) ? 2 : 1;
  // groups requested ahead: two of parity 0 and one of parity 1 for up to 9
  // stored components; larger blocks (b = 4) keep one group, registers allow
  constexpr int NPF = (MSP == 2 && E >= 4 && NS <= 9) ? 2 : 1;
  constexpr bool PF1 = NS <= 9;
  C2 pf[NPF][NS];
  C2 pf1[PF1 ? NS : 1];
  auto sym_base = [&](int p) {
    return (const C*)a.sym + q * a.sym_bs + ((int64_t)p * a.sym_ntiles + a.tile0 + tile) * (NS * E * SL);
  };
  if constexpr (!MIR && MSP == 2) {
#pragma unroll
    for (int j = 0; j < NPF; ++j)
#pragma unroll
      for (int k = 0; k < NS; ++k) pf[j][k] = *(const C2*)(sym_base(0) + sym_offset(k, 2 * j, slane, E, SL));
  }
  // mirrored storage: the stored entries of group (p, m0) of every component,
  // with their sign flips (bit k of flip[j]). With E a multiple of 4 the
  // last level's rows are stored in lane pairs (the runtime's mirror
  // scatter): entries m0, m0 + 1 of a lane are one 16-byte load, from the
  // lane itself below E/2 and from its mirror lane (pair E - 2 - m0, halves
  // swapped) above; otherwise one 8-byte load per entry from the plain row.
  constexpr bool PAIRED = MIR && (E % 4 == 0);
  auto mir_group = [&](int p, int m0, C (&dst)[MSP][NS], uint32_t (&flip)[MSP]) {
#pragma unroll
    for (int j = 0; j < MSP; ++j) {
      const int k = t + T * (m0 + j);
      const bool mir = 2 * k + p > L;
      flip[j] = osign ^ (mir ? lodd : 0u);
    }
    if constexpr (PAIRED) {
      const bool upper = 2 * m0 >= E;  // compile-time once unrolled
      const int W = p ? T : T + 1;
      const int u = upper ? (p ? T - 1 - t : T - t) : t;
      const int P = upper ? (E - 2 - m0) / 2 : m0 / 2;
      const uint32_t off =
          ((uint32_t)mbase + (uint32_t)((p ? (T + 1) * (E / 2) : 0) + (P * W + u) * 2)) * (uint32_t)sizeof(C);
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const C2 v = *(const C2*)((const char*)a.sym + k * a.mcomp * (int64_t)sizeof(C) + off);
        dst[upper ? 1 : 0][k] = mk<C>(v.x, v.y);
        dst[upper ? 0 : 1][k] = mk<C>(v.z, v.w);
      }
    } else {
      uint32_t off[MSP];
#pragma unroll
      for (int j = 0; j < MSP; ++j) {
        const int k = t + T * (m0 + j);
        const bool mir = 2 * k + p > L;
        off[j] = ((uint32_t)mbase + (uint32_t)(p * (L / 2 + 1) + (mir ? (p ? L - 1 - k : L - k) : k))) *
                 (uint32_t)sizeof(C);
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const char* base = (const char*)a.sym + k * a.mcomp * (int64_t)sizeof(C);
#pragma unroll
        for (int j = 0; j < MSP; ++j) dst[j][k] = *(const C*)(base + off[j]);
      }
    }
  };
  // mirrored storage requests groups ahead as the general layout does: NPF
  // of parity 0 before the forward transforms, the first of parity 1 before
  // parity 0's product (-4% on the length-128 leaf: it then matches the
  // general one). Only complex64 leaves of length <= 128 with lane pairs
  // keep their occupancy with the extra registers (complex128, and lengths
  // 256 to 1024, drop a wavefront per SIMD); the others request one group.
  constexpr bool MPF = PAIRED && sizeof(Real) == 4 && L <= 128;
  constexpr int MNPF = MPF ? NPF : 1;
  constexpr bool MPF1 = MPF && PF1 && NPAR == 2;
  C mpf[MNPF][MSP][NS];
  uint32_t mpf_flip[MNPF][MSP];
  C mpf1[MPF1 ? MSP : 1][NS];
  uint32_t mpf1_flip[MSP];
  if constexpr (MIR) {
#pragma unroll
    for (int i = 0; i < MNPF; ++i) mir_group(0, i * MSP, mpf[i], mpf_flip[i]);
  }
  // mulBrn for one child p: w[.][m] <- S_p[., .](m) w[.][m]
  auto block_product = [&](C (&w)[B][E], int p) {
    if constexpr (!MIR && MSP == 2 && NPAR == 2 && PF1) {  // the embedding baseline has one child
      if (p == 0) {
#pragma unroll
        for (int k = 0; k < NS; ++k) pf1[k] = *(const C2*)(sym_base(1) + sym_offset(k, 0, slane, E, SL));
      }
    }
    if constexpr (MPF1) {
      if (p == 0) mir_group(1, 0, mpf1, mpf1_flip);
    }
    const C* sp = (const C*)a.sym + q * a.sym_bs + ((int64_t)p * a.sym_ntiles + a.tile0 + tile) * (NS * E * SL);
    constexpr int MS = (E % 2 == 0) ? 2 : 1;  // entries per symbol load
#pragma unroll
    for (int m0 = 0; m0 < E; m0 += MS) {
      C sm[MS][NS];
      if constexpr (MIR) {
        C raw[MSP][NS];
        uint32_t flip[MSP];
        if (p == 0 && m0 < MNPF * MSP) {
#pragma unroll
          for (int j = 0; j < MSP; ++j) {
            flip[j] = mpf_flip[m0 / MSP][j];
#pragma unroll
            for (int k = 0; k < NS; ++k) raw[j][k] = mpf[m0 / MSP][j][k];
          }
        } else if (MPF1 && p == 1 && m0 == 0) {
#pragma unroll
          for (int j = 0; j < MSP; ++j) {
            flip[j] = mpf1_flip[j];
#pragma unroll
            for (int k = 0; k < NS; ++k) raw[j][k] = mpf1[MPF1 ? j : 0][k];
          }
        } else {
          mir_group(p, m0, raw, flip);
        }
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
          for (int j = 0; j < MS; ++j) sm[j][k] = cneg_if(raw[j][k], (flip[j] >> k) & 1u);
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        if constexpr (MIR) {
        } else if constexpr (MS == 2) {
          const C2 v = (p == 0 && m0 < 2 * NPF) ? pf[m0 / 2][k]
                       : (PF1 && NPAR == 2 && p == 1 && m0 == 0) ? pf1[PF1 ? k : 0]
                                                                 : *(const C2*)(sp + sym_offset(k, m0, slane, E, SL));
          sm[0][k] = mk<C>(v.x, v.y);
          sm[1][k] = mk<C>(v.z, v.w);
        } else {
          sm[0][k] = sp[sym_offset(k, m0, slane, E, SL)];
        }
      }
#pragma unroll
      for (int j = 0; j < MS; ++j) {
        C o[B];
#pragma unroll
        for (int ar = 0; ar < B; ++ar) {
          C u;
          if constexpr (G::LFMA) {
            // first term a product, the others fused multiply-adds
            u = cmul(sm[j][BSy::idx(ar, 0)], w[0][m0 + j]);
            if (BSy::neg(ar, 0)) u = mk<C>(-u.x, -u.y);
#pragma unroll
            for (int c = 1; c < B; ++c) {
              const C sv = sm[j][BSy::idx(ar, c)];
              u = BSy::neg(ar, c) ? cfms(sv, w[c][m0 + j], u) : cfma(sv, w[c][m0 + j], u);
            }
          } else {
            u = czero<C>();
#pragma unroll
            for (int c = 0; c < B; ++c) {
              const C v = cmul(sm[j][BSy::idx(ar, c)], w[c][m0 + j]);
              u = BSy::neg(ar, c) ? csub(u, v) : cadd(u, v);
            }
          }
          o[ar] = u;
        }
#pragma unroll
        for (int ar = 0; ar < B; ++ar) w[ar][m0 + j] = o[ar];
      }
    }
  };

  // all children x components transformed together (one LDS row each);
  // the swizzled rows only up to 3x3 blocks (b = 4 mirrored leaves would spill)
  constexpr int NP = NPAR * B;
  constexpr int SWZ = (G::LSWZ && B <= 3) ? 1 : 0;
  C h[NP][E];
  // split phases Phi[t + T m] = Phi[t] Phi[T m]: one per-lane value and E
  // lane-uniform table entries, so the merge needs no second per-lane fetch
  const C ph0 = NPAR == 2 ? tw[t] : czero<C>();
  auto phase = [&](int m) -> C { return m == 0 ? ph0 : cmul(ph0, tw[T * m]); };
  if constexpr (NPAR == 2) {
    C ph[E];
#pragma unroll
    for (int m = 0; m < E; ++m) ph[m] = phase(m);
#pragma unroll
    for (int c = 0; c < B; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) {
        h[c][m] = x[c][m];
        h[B + c][m] = cmul(x[c][m], ph[m]);  // odd child: Phi x
      }
  } else {
#pragma unroll
    for (int c = 0; c < B; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) h[c][m] = x[c][m];
  }
  if constexpr (NROW == NP) {
    fft_pencils<-1, Sh, G::LWS, NP, G::LFMA, SWZ>(h, lp, LP, 1, t, lt);
  } else {
#pragma unroll
    for (int c = 0; c < NP; ++c) fft_pencil<-1, Sh, G::LWS, G::LFMA>(h[c], lp, 1, t, lt);
  }
  block_product(*reinterpret_cast<C(*)[B][E]>(&h[0]), 0);
  if constexpr (NPAR == 2) block_product(*reinterpret_cast<C(*)[B][E]>(&h[B]), 1);
  if constexpr (NROW == NP) {
    fft_pencils<+1, Sh, G::LWS, NP, G::LFMA, SWZ>(h, lp, LP, 1, t, lt);
  } else {
#pragma unroll
    for (int c = 0; c < NP; ++c) fft_pencil<+1, Sh, G::LWS, G::LFMA>(h[c], lp, 1, t, lt);
  }
  if constexpr (NPAR == 2) {
    // merge: even + conj(Phi) odd
#pragma unroll
    for (int c = 0; c < B; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m)
        x[c][m] = G::LFMA ? cfmac(h[B + c][m], phase(m), h[c][m]) : cadd(h[c][m], cmulc(h[B + c][m], phase(m)));
  } else {
#pragma unroll
    for (int c = 0; c < B; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) x[c][m] = h[c][m];
  }

  // store: every lane writes its own entries
  if (act) {
#pragma unroll
    for (int c = 0; c < B; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) out[pbase + (int64_t)c * a.npen * L + T * m] = x[c][m];
  }
}

template <typename Real, int L, int B, int NPAR, bool MIR, int BS>
__global__ void __launch_bounds__((Geo<Real, L>::RBMAX * Geo<Real, L>::SL))
    __attribute__((amdgpu_waves_per_eu(Geo<Real, L>::template leaf_waves<B, MIR, BS>()))) k_leaf(PassArgs a) {
  leaf_body<Real, L, B, NPAR, MIR, BS>(a, blockIdx.x);
}

template <typename Real, int L, int B, int NPAR, bool MIR, int BS>
__global__ void __launch_bounds__((Geo<Real, L>::RBMAX * Geo<Real, L>::SL))
    __attribute__((amdgpu_waves_per_eu(Geo<Real, L>::template leaf_waves<B, MIR, BS>() == 3 && BS == 1 ? 3 : 1)))
    k_leaf_group(const PassArgs* __restrict__ tab, int nent) {
  const int e = find_entry(tab, nent, blockIdx.x);
  leaf_body<Real, L, B, NPAR, MIR, BS>(tab[e], blockIdx.x - tab[e].blk_begin);
}

// ---------------------------------------------------------------------------
// Host-side launch table for one length.
// ---------------------------------------------------------------------------
typedef hipError_t (*pass_fn)(const PassArgs&, hipStream_t);
// Grouped launches: prep fills an entry's launch fields (index decoding,
// block order, leaf right-hand-side grouping) and returns its workgroups,
// rounded up to a multiple of 8 (or -1 beyond the 1-D grid); group launches
// the kernel over a table of prepared entries in device memory.
typedef int64_t (*prep_fn)(PassArgs&);
typedef hipError_t (*group_fn)(const PassArgs*, int nent, int64_t blocks, hipStream_t);
typedef int64_t (*leaf_prep_fn)(PassArgs&, size_t* smem);
typedef hipError_t (*leaf_group_fn)(const PassArgs*, int nent, int64_t blocks, int rb, size_t smem, hipStream_t);

struct AxisOps {
  int L, T, E, W, P;   // strided / contiguous passes
  int LT, LE, PL, NTL; // leaf: lanes per pencil, entries per lane, pencils per tile, lanes per tile
  int RBMAX;           // leaf: most right-hand sides per workgroup
  pass_fn strided[2];   // [0] FWD2, [1] INV2
  pass_fn contig[2];
  struct LeafRow {
    pass_fn f[3][3];  // [NPAR][block symmetry]
  };
  struct MirRow {
    pass_fn f[3];     // [block symmetry]
  };
  LeafRow leaf[5];    // [B]: general symbol storage, null where not built
  MirRow leaf_mirror[5];  // [B]: NPAR = 2, mirrored symbol storage
  int generic;        // 1: runtime-length kernels (pencil tiles staged whole in LDS)
  // grouped launches (null for the runtime-length kernels): strided passes
  // with full-size [0] or half-size [1] workgroups (half null where the tile
  // would be narrower than a 128-byte line), and the split leaf (NPAR = 2)
  prep_fn strided_prep[2];
  group_fn strided_group[2][2];  // [MODE][half]
  struct LeafGroupRow {
    leaf_prep_fn prep[3];  // [block symmetry]
    leaf_group_fn group[3];
  };
  LeafGroupRow leaf_group[5];         // [B], general symbols
  LeafGroupRow leaf_group_mirror[5];  // [B], mirrored symbols
};

constexpr int64_t kIdx32 = (int64_t)1 << 31;
constexpr size_t kMaxLds = 160 * 1024;  // LDS of one gfx950 workgroup
// passes of at least this many workgroups (many per CU) use the
// XCD-contiguous block order (1.4% on 256x256x128 passes); smaller launches
// keep dispatch order (their start latency counts), except narrow tiles
constexpr int64_t kXcdOrderFrom = 8192;

template <typename Real, int L, int NT> int64_t prep_strided_nt(PassArgs& b) {
  constexpr int W = NT / Geo<Real, L>::T;
  const int64_t cols = b.outer * b.inner;
  const int64_t ntile = (cols + W - 1) / W;
  const int64_t blocks = b.nq * ntile;
  if (blocks <= 0) return 0;
  if (blocks >= kIdx32) return -1;  // beyond the 1-D grid
  b.idx32 = blocks < kIdx32 && ntile * W < kIdx32;
  if (b.idx32) {
    b.fd_a = FastDiv::make((uint32_t)ntile);
    b.fd_b = FastDiv::make((uint32_t)b.inner);
  }
  // tiles narrower than a 128-byte line share lines with their neighbours:
  // in dispatch order those neighbours run on different XCDs and each XCD
  // fetches the line (a 1024-point pass moves 32-byte row segments); in
  // XCD-contiguous order they share one L2 (-20% on a 1024^2 grid)
  constexpr bool narrow = W * (int)sizeof(cx<Real>) < 128;
  const int64_t grid = set_block_order(b, blocks, blocks >= kXcdOrderFrom || (narrow && blocks >= 16));
  return (grid + 7) / 8 * 8;  // items past nblk store nothing
}

template <typename Real, int L, int MODE, int NT> hipError_t launch_strided_nt(const PassArgs& a, hipStream_t s) {
  PassArgs b = a;
  const int64_t grid = prep_strided_nt<Real, L, NT>(b);
  if (grid == 0) return hipSuccess;
  if (grid < 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_strided<Real, L, MODE, NT>), dim3((unsigned)grid), dim3(NT), 0, s, b);
  return hipGetLastError();
}

template <typename Real, int L, int MODE, int NT>
hipError_t group_strided_nt(const PassArgs* tab, int nent, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (blocks >= kIdx32) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_strided_group<Real, L, MODE, NT>), dim3((unsigned)blocks), dim3(NT), 0, s, tab, nent);
  return hipGetLastError();
}

// Launches of few workgroups use half-size ones (tiles still whole 128-byte
// lines) when the lengths allow: 384 workgroups of four wavefronts leave half
// of the CUs with twice the work of the others, 768 of two spread evenly.
constexpr int64_t kHalfTilesBelow = 2048;

template <typename Real, int L> constexpr bool half_tiles_ok() {
  using G = Geo<Real, L>;
  return (G::W / 2) * (int)sizeof(cx<Real>) >= 128;
}

template <typename Real, int L, int MODE> hipError_t launch_strided(const PassArgs& a, hipStream_t s) {
  using G = Geo<Real, L>;
  if constexpr (half_tiles_ok<Real, L>()) {
    const int64_t cols = a.outer * a.inner;
    const int64_t blocks = a.nq * ((cols + G::W - 1) / G::W);
    if (a.tile_mode == 2 || (a.tile_mode == 0 && blocks < kHalfTilesBelow))
      return launch_strided_nt<Real, L, MODE, G::NT / 2>(a, s);
  }
  return launch_strided_nt<Real, L, MODE, G::NT>(a, s);
}

template <typename Real, int L, int MODE> hipError_t launch_contig(const PassArgs& a, hipStream_t s) {
  using G = Geo<Real, L>;
  const int64_t ntile = (a.outer + G::P - 1) / G::P;
  const int64_t blocks = a.nq * ntile;
  if (blocks <= 0) return hipSuccess;
  if (blocks >= kIdx32) return hipErrorInvalidConfiguration;  // beyond the 1-D grid
  PassArgs b = a;
  b.idx32 = blocks < kIdx32;
  if (b.idx32) b.fd_a = FastDiv::make((uint32_t)ntile);
  const int64_t grid = set_block_order(b, blocks, blocks >= kXcdOrderFrom);
  hipLaunchKernelGGL((k_contig<Real, L, MODE>), dim3((unsigned)grid), dim3(G::NT), 0, s, b);
  return hipGetLastError();
}

// Right-hand sides per leaf workgroup (clamped to the kernel's limit and to
// 64 KB of LDS), decoding fields, workgroups and LDS bytes.
template <typename Real, int L, int B, int NPAR, bool MIR, int BS> int64_t prep_leaf(PassArgs& b, size_t* smem) {
  using G = Geo<Real, L>;
  constexpr size_t row_bytes = (size_t)G::PL * G::LLP * sizeof(cx<Real>) * G::template leaf_rows<B, NPAR>();
  constexpr int rb_lds = (int)((64 * 1024) / row_bytes) > 0 ? (int)((64 * 1024) / row_bytes) : 1;
  int rb = b.rb < 1 ? 1 : (b.rb > G::RBMAX ? G::RBMAX : b.rb);
  while (rb > rb_lds) rb /= 2;
  b.rb = rb;
  const int64_t nrg = (b.nrhs + rb - 1) / rb;
  const int64_t blocks = b.nq * ((b.ntiles + 7) / 8) * nrg * 8;
  if (blocks <= 0) return 0;
  b.idx32 = blocks < kIdx32;
  if (b.idx32) {
    b.fd_a = FastDiv::make((uint32_t)nrg);
    b.fd_b = FastDiv::make((uint32_t)((b.ntiles + 7) / 8));
  }
  *smem = (size_t)rb * row_bytes;
  if (*smem > kMaxLds || blocks >= kIdx32) return -1;  // beyond a workgroup's LDS or the grid
  return blocks;
}

template <typename Real, int L, int B, int NPAR, bool MIR = false, int BS = 0>
hipError_t launch_leaf(const PassArgs& a, hipStream_t s) {
  using G = Geo<Real, L>;
  PassArgs b = a;
  size_t smem = 0;
  const int64_t blocks = prep_leaf<Real, L, B, NPAR, MIR, BS>(b, &smem);
  if (blocks == 0) return hipSuccess;
  if (blocks < 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_leaf<Real, L, B, NPAR, MIR, BS>), dim3((unsigned)blocks), dim3(b.rb * G::SL), smem, s, b);
  return hipGetLastError();
}

template <typename Real, int L, int B, int NPAR, bool MIR, int BS>
hipError_t group_leaf(const PassArgs* tab, int nent, int64_t blocks, int rb, size_t smem, hipStream_t s) {
  using G = Geo<Real, L>;
  if (blocks <= 0) return hipSuccess;
  if (blocks >= kIdx32 || smem > kMaxLds) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_leaf_group<Real, L, B, NPAR, MIR, BS>), dim3((unsigned)blocks), dim3(rb * G::SL), smem, s,
                     tab, nent);
  return hipGetLastError();
}

template <typename Real, int L, int B, bool MIR> AxisOps::LeafGroupRow leaf_group_row() {
  AxisOps::LeafGroupRow r{};
  if constexpr (B == 1) {  // a scalar block has no block symmetry to exploit
    for (int bs = 0; bs < 3; ++bs) {
      r.prep[bs] = prep_leaf<Real, L, 1, 2, MIR, 0>;
      r.group[bs] = group_leaf<Real, L, 1, 2, MIR, 0>;
    }
  } else {
    r.prep[0] = prep_leaf<Real, L, B, 2, MIR, 0>;
    r.prep[1] = prep_leaf<Real, L, B, 2, MIR, 1>;
    r.prep[2] = prep_leaf<Real, L, B, 2, MIR, 2>;
    r.group[0] = group_leaf<Real, L, B, 2, MIR, 0>;
    r.group[1] = group_leaf<Real, L, B, 2, MIR, 1>;
    r.group[2] = group_leaf<Real, L, B, 2, MIR, 2>;
  }
  return r;
}

template <typename Real, int L, int B> constexpr AxisOps::LeafRow leaf_row_general() {
  AxisOps::LeafRow r{};
  if constexpr (B == 1) {  // a scalar block has no block symmetry to exploit
    for (int bs = 0; bs < 3; ++bs) {
      r.f[1][bs] = launch_leaf<Real, L, 1, 1>;
      r.f[2][bs] = launch_leaf<Real, L, 1, 2>;
    }
  } else {
    r.f[1][0] = launch_leaf<Real, L, B, 1, false, 0>;
    r.f[1][1] = launch_leaf<Real, L, B, 1, false, 1>;
    r.f[1][2] = launch_leaf<Real, L, B, 1, false, 2>;
    r.f[2][0] = launch_leaf<Real, L, B, 2, false, 0>;
    r.f[2][1] = launch_leaf<Real, L, B, 2, false, 1>;
    r.f[2][2] = launch_leaf<Real, L, B, 2, false, 2>;
  }
  return r;
}

template <typename Real, int L, int B> constexpr AxisOps::MirRow leaf_row_mirror() {
  AxisOps::MirRow r{};
  if constexpr (B == 1) {
    for (int bs = 0; bs < 3; ++bs) r.f[bs] = launch_leaf<Real, L, 1, 2, true>;
  } else {
    r.f[0] = launch_leaf<Real, L, B, 2, true, 0>;
    r.f[1] = launch_leaf<Real, L, B, 2, true, 1>;
    r.f[2] = launch_leaf<Real, L, B, 2, true, 2>;
  }
  return r;
}

template <typename Real, int L> const AxisOps* make_ops() {
  using G = Geo<Real, L>;
  static const AxisOps ops = {
      L, G::T, G::E, G::W, G::P, G::LT, G::LE, G::PL, G::NTL, G::RBMAX,
      {launch_strided<Real, L, 0>, launch_strided<Real, L, 1>},
      {launch_contig<Real, L, 0>, launch_contig<Real, L, 1>},
      {{}, leaf_row_general<Real, L, 1>(), leaf_row_general<Real, L, 2>(), leaf_row_general<Real, L, 3>(),
       leaf_row_general<Real, L, 4>()},
      {{}, leaf_row_mirror<Real, L, 1>(), leaf_row_mirror<Real, L, 2>(), leaf_row_mirror<Real, L, 3>(),
       leaf_row_mirror<Real, L, 4>()},
      0,
      {prep_strided_nt<Real, L, G::NT>, half_tiles_ok<Real, L>() ? prep_strided_nt<Real, L, G::NT / 2> : nullptr},
      {{group_strided_nt<Real, L, 0, G::NT>,
        half_tiles_ok<Real, L>() ? group_strided_nt<Real, L, 0, G::NT / 2> : nullptr},
       {group_strided_nt<Real, L, 1, G::NT>,
        half_tiles_ok<Real, L>() ? group_strided_nt<Real, L, 1, G::NT / 2> : nullptr}},
      {{}, leaf_group_row<Real, L, 1, false>(), leaf_group_row<Real, L, 2, false>(),
       leaf_group_row<Real, L, 3, false>(), leaf_group_row<Real, L, 4, false>()},
      {{}, leaf_group_row<Real, L, 1, true>(), leaf_group_row<Real, L, 2, true>(),
       leaf_group_row<Real, L, 3, true>(), leaf_group_row<Real, L, 4, true>()},
  };
  return &ops;
}

}  // namespace sfft
