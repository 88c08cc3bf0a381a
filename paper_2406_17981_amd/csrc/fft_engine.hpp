// Pencil FFT engine for gfx950: one length-L complex DFT spread over T lanes.
//
// Each lane owns E = L/T "home" entries of its pencil, the entries k = t + T*m
// (m = 0..E-1) for lane t. A transform is a chain of Stockham autosort radix
// stages (radices from Shape<L>); the first stage reads its butterfly inputs
// straight from the home registers and the last stage leaves its outputs in
// the home registers, so a two-stage transform crosses LDS exactly once. The
// output of a forward transform is in natural order, which is also the input
// order of an inverse transform, so a pointwise product between the two needs
// no data movement.
//
// Twiddles come from a per-length table tw[m] = exp(-2 pi i m / (2L)),
// m = 0..2L-1, generated once in FP64: W_L^m = tw[2m] and the split phase of
// the paper's Section II.A, exp(-i pi k / L), is tw[k].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfft {

template <typename R> struct CxOf;
template <> struct CxOf<float> { using type = float2; };
template <> struct CxOf<double> { using type = double2; };
template <typename R> using cx = typename CxOf<R>::type;

template <typename C> __device__ __forceinline__ C mk(decltype(C::x) a, decltype(C::x) b) {
  C c;
  c.x = a;
  c.y = b;
  return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
// The library is compiled without implicit contraction (-ffp-contract=off):
// every fused multiply-add is written out below, so a result's rounding is
// fixed by the source and never by how the compiler schedules one kernel
// instantiation against another (single and grouped launches, tile widths
// and schedules give bit-identical results).
// fused multiply-add, one rounding
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a * b: one product rounded, the other fused
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(fmar(a.x, b.x, -(a.y * b.y)), fmar(a.x, b.y, a.y * b.x));
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return mk<C>(fmar(a.x, b.x, a.y * b.y), fmar(a.y, b.x, -(a.x * b.y)));
}
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
// u + a * s for a real s
template <typename C> __device__ __forceinline__ C cfmas(C a, decltype(C::x) s, C u) {
  return mk<C>(fmar(a.x, s, u.x), fmar(a.y, s, u.y));
}
// u + a * b, u - a * b and u + a * conj(b) as four fused multiply-adds each
template <typename C> __device__ __forceinline__ C cfma(C a, C b, C u) {
  return mk<C>(fmar(-a.y, b.y, fmar(a.x, b.x, u.x)), fmar(a.y, b.x, fmar(a.x, b.y, u.y)));
}
template <typename C> __device__ __forceinline__ C cfms(C a, C b, C u) {
  return mk<C>(fmar(a.y, b.y, fmar(-a.x, b.x, u.x)), fmar(-a.y, b.x, fmar(-a.x, b.y, u.y)));
}
template <typename C> __device__ __forceinline__ C cfmac(C a, C b, C u) {
  return mk<C>(fmar(a.y, b.y, fmar(a.x, b.x, u.x)), fmar(-a.x, b.y, fmar(a.y, b.x, u.y)));
}
template <typename C> __device__ __forceinline__ C czero() { return mk<C>(0, 0); }
// -a when s is 1, a when s is 0 (sign bits flipped, no compare or select)
__device__ __forceinline__ float2 cneg_if(float2 a, uint32_t s) {
  const uint32_t m = s << 31;
  return make_float2(__uint_as_float(__float_as_uint(a.x) ^ m), __uint_as_float(__float_as_uint(a.y) ^ m));
}
__device__ __forceinline__ double2 cneg_if(double2 a, uint32_t s) {
  const unsigned long long m = (unsigned long long)s << 63;
  return make_double2(__longlong_as_double(__double_as_longlong(a.x) ^ (long long)m),
                      __longlong_as_double(__double_as_longlong(a.y) ^ (long long)m));
}
// (DIR * i) * a, DIR = -1 forward, +1 inverse
template <int DIR, typename C> __device__ __forceinline__ C mul_di(C a) {
  if constexpr (DIR > 0) return mk<C>(-a.y, a.x);
  else return mk<C>(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Small DFTs in registers, natural order in and out.
// ---------------------------------------------------------------------------
template <int DIR, typename C> __device__ __forceinline__ void dft2(C* v) {
  C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int DIR, typename C> __device__ __forceinline__ void dft3(C* v) {
  using R = decltype(C::x);
  const R c3 = (R)-0.5;
  const R s3 = (R)0.86602540378443864676372317075294;  // sin(2 pi / 3)
  C a = v[0];
  C sb = cadd(v[1], v[2]);
  C db = csub(v[1], v[2]);
  C m = cfmas(sb, c3, a);
  C r = mul_di<DIR>(db);
  v[0] = cadd(a, sb);
  v[1] = cfmas(r, s3, m);
  v[2] = cfmas(r, -s3, m);
}

template <int DIR, typename C> __device__ __forceinline__ void dft4(C* v) {
  C t0 = cadd(v[0], v[2]);
  C t1 = csub(v[0], v[2]);
  C t2 = cadd(v[1], v[3]);
  C t3 = mul_di<DIR>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <int DIR, typename C> __device__ __forceinline__ void dft5(C* v) {
  using R = decltype(C::x);
  const R c1 = (R)0.30901699437494742410229341718282;   // cos(2 pi / 5)
  const R c2 = (R)-0.80901699437494742410229341718282;  // cos(4 pi / 5)
  const R s1 = (R)0.95105651629515357211643933337938;   // sin(2 pi / 5)
  const R s2 = (R)0.58778525229247312916870595463907;   // sin(4 pi / 5)
  C a0 = v[0];
  C p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
  C p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
  C e1 = cfmas(p1, c1, cfmas(p2, c2, a0));
  C e2 = cfmas(p1, c2, cfmas(p2, c1, a0));
  C o1 = mul_di<DIR>(cfmas(m1, s1, cscale(m2, s2)));
  C o2 = mul_di<DIR>(cfmas(m1, s2, cscale(m2, -s1)));
  v[0] = cadd(a0, cadd(p1, p2));
  v[1] = cadd(e1, o1);
  v[4] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[3] = csub(e2, o2);
}

// Radix 7: with p_j = v_j + v_{7-j} and m_j = v_j - v_{7-j} (j = 1..3),
// X[k] = v_0 + sum_j p_j cos(2 pi jk/7) + DIR i sum_j m_j sin(2 pi jk/7) and
// X[7-k] the same with the sine sum negated (k = 1..3).
template <int DIR, typename C> __device__ __forceinline__ void dft7(C* v) {
  using R = decltype(C::x);
  const R c1 = (R)0.62348980185873353052500488400424;   // cos(2 pi / 7)
  const R c2 = (R)-0.22252093395631440428890256449680;  // cos(4 pi / 7)
  const R c3 = (R)-0.90096886790241912623610231950745;  // cos(6 pi / 7)
  const R s1 = (R)0.78183148246802980870844452667406;   // sin(2 pi / 7)
  const R s2 = (R)0.97492791218182360701813168299393;   // sin(4 pi / 7)
  const R s3 = (R)0.43388373911755812047576833284836;   // sin(6 pi / 7)
  const C a0 = v[0];
  const C p1 = cadd(v[1], v[6]), m1 = csub(v[1], v[6]);
  const C p2 = cadd(v[2], v[5]), m2 = csub(v[2], v[5]);
  const C p3 = cadd(v[3], v[4]), m3 = csub(v[3], v[4]);
  // cos(2 pi jk/7) and sin(2 pi jk/7) for jk mod 7 = 4, 5, 6 are c3, c2, c1 and -s3, -s2, -s1
  const C e1 = cfmas(p1, c1, cfmas(p2, c2, cfmas(p3, c3, a0)));
  const C e2 = cfmas(p1, c2, cfmas(p2, c3, cfmas(p3, c1, a0)));
  const C e3 = cfmas(p1, c3, cfmas(p2, c1, cfmas(p3, c2, a0)));
  const C o1 = mul_di<DIR>(cfmas(m1, s1, cfmas(m2, s2, cscale(m3, s3))));
  const C o2 = mul_di<DIR>(cfmas(m1, s2, cfmas(m2, -s3, cscale(m3, -s1))));
  const C o3 = mul_di<DIR>(cfmas(m1, s3, cfmas(m2, -s1, cscale(m3, s2))));
  v[0] = cadd(a0, cadd(p1, cadd(p2, p3)));
  v[1] = cadd(e1, o1);
  v[6] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[5] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[4] = csub(e3, o3);
}

// Second layer of a radix-8 DFT from the DFT4s e (even entries) and o (odd
// entries): o[k] *= W8^k with W8 = exp(DIR 2 pi i / 8); the sqrt(1/2) of
// k = 1, 3 is fused into the output butterflies.
template <int DIR, typename C> __device__ __forceinline__ void dft8_tail(C* v, const C* e, const C* o) {
  using R = decltype(C::x);
  const R h = (R)0.70710678118654752440084436210485;  // sqrt(1/2)
  const C t1 = cadd(o[1], mul_di<DIR>(o[1]));
  const C t2 = mul_di<DIR>(o[2]);
  const C t3 = csub(mul_di<DIR>(o[3]), o[3]);
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cfmas(t1, h, e[1]);
  v[5] = cfmas(t1, -h, e[1]);
  v[2] = cadd(e[2], t2);
  v[6] = csub(e[2], t2);
  v[3] = cfmas(t3, h, e[3]);
  v[7] = cfmas(t3, -h, e[3]);
}

template <int DIR, typename C> __device__ __forceinline__ void dft8(C* v) {
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  dft8_tail<DIR>(v, e, o);
}

template <int DIR, typename C> __device__ __forceinline__ void dft16(C* v) {
  using R = decltype(C::x);
  const R h = (R)0.70710678118654752440084436210485;   // cos(pi/4)
  const R c8 = (R)0.92387953251128675612818318939679;  // cos(pi/8)
  const R s8 = (R)0.38268343236508977172845998403040;  // sin(pi/8)
  // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
  C y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = v[4 * n1 + n2];
    dft4<DIR>(y[n2]);
  }
  // twiddle W16^(n2 k1), W16 = exp(DIR 2 pi i / 16) = c8 + DIR i s8
  const R D = (R)DIR;
  const C w1 = mk<C>(c8, D * s8);
  const C w2 = mk<C>(h, D * h);
  const C w3 = mk<C>(s8, D * c8);
  y[1][1] = cmul(y[1][1], w1);
  y[1][2] = cmul(y[1][2], w2);
  y[1][3] = cmul(y[1][3], w3);
  y[2][1] = cmul(y[2][1], w2);
  y[2][2] = mul_di<DIR>(y[2][2]);
  y[2][3] = cmul(y[2][3], mk<C>(-h, D * h));
  y[3][1] = cmul(y[3][1], w3);
  y[3][2] = cmul(y[3][2], mk<C>(-h, D * h));
  y[3][3] = cmul(y[3][3], mk<C>(-c8, -D * s8));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4<DIR>(z);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = z[k2];
  }
}

// Radix-4 DFT whose first layer is done: a0, a1 = e0 +- e2 and b0, b1 =
// e1 +- e3 of the inputs e0..e3.
template <int DIR, typename C> __device__ __forceinline__ void dft4_tail(C* v, C a0, C a1, C b0, C b1) {
  const C t3 = mul_di<DIR>(b1);
  v[0] = cadd(a0, b0);
  v[2] = csub(a0, b0);
  v[1] = cadd(a1, t3);
  v[3] = csub(a1, t3);
}

// Twiddled butterfly of a stage after the first: entries r >= 1 are scaled by
// w[r-1] (conjugated for the inverse) and the radix-R DFT follows. For R = 2,
// 4, 8, 16 the DFT's first layer pairs entries r and r + R/2; each pair is
// formed as y0 = a + w b with fused multiply-adds and y1 = 2a - y0, so the
// product w b of the pair's upper entry is never rounded on its own (the
// multiply-add butterfly of Linzer and Feig). It issues fewer instructions
// but chains more of them, so it pays in kernels with enough wavefronts to
// hide VALU latency and is selected per kernel (template flag FMA).
template <int R, int DIR, typename C> __device__ __forceinline__ void tw_dft(C* v, const C* w) {
  using Rl = decltype(C::x);
  constexpr int H = R / 2;
  C y0[H], y1[H];
#pragma unroll
  for (int r = 0; r < H; ++r) {
    C a = v[r];
    if (r > 0) a = (DIR > 0) ? cmulc(a, w[r - 1]) : cmul(a, w[r - 1]);
    const C b = v[r + H];
    const C s = (DIR > 0) ? cfmac(b, w[r + H - 1], a) : cfma(b, w[r + H - 1], a);
    y0[r] = s;
    y1[r] = mk<C>(fmar((Rl)2, a.x, -s.x), fmar((Rl)2, a.y, -s.y));
  }
  if constexpr (R == 2) {
    v[0] = y0[0];
    v[1] = y1[0];
  } else if constexpr (R == 4) {
    dft4_tail<DIR>(v, y0[0], y1[0], y0[1], y1[1]);
  } else if constexpr (R == 8) {
    // as dft8: e = DFT4 of the even entries, o = DFT4 of the odd ones
    C e[4], o[4];
    dft4_tail<DIR>(e, y0[0], y1[0], y0[2], y1[2]);
    dft4_tail<DIR>(o, y0[1], y1[1], y0[3], y1[3]);
    dft8_tail<DIR>(v, e, o);
  } else {
    static_assert(R == 16, "twiddled butterfly for radix 2, 4, 8, 16");
    // as dft16: n = 4 n1 + n2; the DFT4 over n1 of group n2 pairs entries
    // n2, n2 + 8 and n2 + 4, n2 + 12
    const Rl h = (Rl)0.70710678118654752440084436210485;
    const Rl c8 = (Rl)0.92387953251128675612818318939679;
    const Rl s8 = (Rl)0.38268343236508977172845998403040;
    C y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4_tail<DIR>(y[n2], y0[n2], y1[n2], y0[n2 + 4], y1[n2 + 4]);
    const Rl D = (Rl)DIR;
    const C w1 = mk<C>(c8, D * s8);
    const C w2 = mk<C>(h, D * h);
    const C w3 = mk<C>(s8, D * c8);
    y[1][1] = cmul(y[1][1], w1);
    y[1][2] = cmul(y[1][2], w2);
    y[1][3] = cmul(y[1][3], w3);
    y[2][1] = cmul(y[2][1], w2);
    y[2][2] = mul_di<DIR>(y[2][2]);
    y[2][3] = cmul(y[2][3], mk<C>(-h, D * h));
    y[3][1] = cmul(y[3][1], w3);
    y[3][2] = cmul(y[3][2], mk<C>(-h, D * h));
    y[3][3] = cmul(y[3][3], mk<C>(-c8, -D * s8));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      dft4<DIR>(z);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = z[k2];
    }
  }
}

template <int R, int DIR, typename C> __device__ __forceinline__ void dft(C* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 3) dft3<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 5) dft5<DIR>(v);
  else if constexpr (R == 7) dft7<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else if constexpr (R == 16) dft16<DIR>(v);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Radix plans. T lanes per pencil; the first and last radices are chosen so
// that T divides L/R_first and L/R_last (register-resident end stages).
// ---------------------------------------------------------------------------
template <int L> struct Shape;
#define SFFT_SHAPE(LEN, TT, ...)                                               \
  template <> struct Shape<LEN> {                                              \
    static constexpr int L = LEN;                                              \
    static constexpr int T = TT;                                               \
    static constexpr int E = LEN / TT;                                         \
    static constexpr int rads[] = {__VA_ARGS__};                               \
    static constexpr int S = sizeof(rads) / sizeof(int);                       \
    static constexpr int rad(int s) { return rads[s]; }                        \
    static constexpr int ns(int s) { return s == 0 ? 1 : ns(s - 1) * rads[s - 1]; } \
  };
SFFT_SHAPE(2, 1, 2)
SFFT_SHAPE(3, 1, 3)
SFFT_SHAPE(4, 1, 4)
SFFT_SHAPE(5, 1, 5)
SFFT_SHAPE(6, 1, 2, 3)
SFFT_SHAPE(8, 1, 8)
SFFT_SHAPE(10, 1, 2, 5)
SFFT_SHAPE(12, 1, 4, 3)
SFFT_SHAPE(16, 4, 4, 4)
SFFT_SHAPE(20, 4, 5, 4)
SFFT_SHAPE(24, 4, 2, 4, 3)
SFFT_SHAPE(32, 4, 8, 4)
SFFT_SHAPE(40, 4, 2, 4, 5)
SFFT_SHAPE(48, 4, 4, 4, 3)
SFFT_SHAPE(64, 8, 8, 8)
SFFT_SHAPE(80, 8, 2, 8, 5)
SFFT_SHAPE(96, 8, 4, 8, 3)
SFFT_SHAPE(128, 8, 8, 16)
SFFT_SHAPE(160, 16, 2, 4, 4, 5)
SFFT_SHAPE(192, 16, 4, 16, 3)
SFFT_SHAPE(256, 16, 16, 16)
SFFT_SHAPE(384, 32, 4, 8, 4, 3)
SFFT_SHAPE(512, 32, 16, 4, 8)
SFFT_SHAPE(768, 64, 4, 4, 16, 3)
SFFT_SHAPE(1024, 64, 16, 8, 8)
SFFT_SHAPE(2048, 128, 16, 8, 16)
#undef SFFT_SHAPE

// Radix plans of the leaf kernel, which holds b components and an accumulator
// per lane: fewer entries per lane (more lanes per pencil) where that keeps
// the first and last stages in registers.
template <int L> struct LeafShape : Shape<L> {};
#define SFFT_LEAF_SHAPE(LEN, TT, ...)                                          \
  template <> struct LeafShape<LEN> {                                          \
    static constexpr int L = LEN;                                              \
    static constexpr int T = TT;                                               \
    static constexpr int E = LEN / TT;                                         \
    static constexpr int rads[] = {__VA_ARGS__};                               \
    static constexpr int S = sizeof(rads) / sizeof(int);                       \
    static constexpr int rad(int s) { return rads[s]; }                        \
    static constexpr int ns(int s) { return s == 0 ? 1 : ns(s - 1) * rads[s - 1]; } \
  };
SFFT_LEAF_SHAPE(6, 2, 3, 2)
SFFT_LEAF_SHAPE(8, 2, 4, 2)
SFFT_LEAF_SHAPE(10, 2, 5, 2)
SFFT_LEAF_SHAPE(12, 4, 3, 4)
SFFT_LEAF_SHAPE(24, 8, 3, 2, 4)
SFFT_LEAF_SHAPE(32, 8, 4, 2, 4)
SFFT_LEAF_SHAPE(40, 8, 5, 8)
SFFT_LEAF_SHAPE(80, 16, 5, 4, 4)
SFFT_LEAF_SHAPE(160, 32, 5, 4, 8)
SFFT_LEAF_SHAPE(192, 32, 2, 4, 8, 3)
SFFT_LEAF_SHAPE(768, 128, 2, 4, 4, 8, 3)
SFFT_LEAF_SHAPE(48, 8, 2, 4, 2, 3)
SFFT_LEAF_SHAPE(64, 16, 4, 4, 4)
SFFT_LEAF_SHAPE(96, 16, 2, 4, 4, 3)
SFFT_LEAF_SHAPE(128, 32, 4, 4, 2, 4)
SFFT_LEAF_SHAPE(256, 64, 4, 4, 4, 4)
SFFT_LEAF_SHAPE(384, 64, 2, 4, 4, 4, 3)
SFFT_LEAF_SHAPE(512, 64, 8, 8, 8)
SFFT_LEAF_SHAPE(1024, 128, 8, 8, 4, 4)
SFFT_LEAF_SHAPE(2048, 256, 8, 8, 4, 8)
#undef SFFT_LEAF_SHAPE

template <typename Sh> constexpr bool shape_ok() {
  int p = 1;
  for (int s = 0; s < Sh::S; ++s) p *= Sh::rads[s];
  return p == Sh::L && Sh::L % Sh::T == 0;
}

// LDS exchange fence. WS (wave sync): every lane of a pencil sits in one
// wavefront and the pencil's LDS row is private to those lanes, so ordering
// the wavefront's own LDS traffic is enough; otherwise a workgroup barrier.
template <bool WS> __device__ __forceinline__ void xsync() {
  if constexpr (WS) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Twiddles of every stage s >= 1 that a lane's butterflies need. They depend
// only on the lane index t, so a kernel loads them once from the FP64-made
// table and reuses them for all its pencils, instead of fetching them from
// memory inside every stage.
template <typename C, typename Sh> struct LaneTw {
  static constexpr int per(int s) { return (Sh::L / Sh::rad(s) + Sh::T - 1) / Sh::T; }
  static constexpr int off(int s) { return s <= 1 ? 0 : off(s - 1) + per(s - 1) * (Sh::rad(s - 1) - 1); }
  static constexpr int N = Sh::S <= 1 ? 1 : off(Sh::S);
  C w[N];

  template <int s> __device__ __forceinline__ void load_stage(int t, const C* tw) {
    if constexpr (s < Sh::S) {
      constexpr int R = Sh::rad(s), Ns = Sh::ns(s), NB = Sh::L / R, TWS = Sh::L / (Ns * R);
#pragma unroll
      for (int u = 0; u < per(s); ++u) {
        const int j = t + Sh::T * u;
        const int k = (j < NB ? j : 0) % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) w[off(s) + u * (R - 1) + r - 1] = tw[2 * (r * k * TWS)];
      }
      load_stage<s + 1>(t, tw);
    }
  }
  __device__ __forceinline__ void load(int t, const C* tw) {
    if constexpr (Sh::S > 1) load_stage<1>(t, tw);
  }
};

// One stage (and, recursively, the following ones) of a pencil transform.
// lds: this pencil's LDS row, element k at lds[k * kst]. All lanes of the
// workgroup (WS = false) or of the wavefront (WS = true) call this together.
template <typename C, typename Sh, int DIR, int s, bool WS, bool FMA>
__device__ __forceinline__ void fft_stage(C (&home)[Sh::E], C* lds, int kst, int t, const LaneTw<C, Sh>& lt) {
  constexpr int L = Sh::L, T = Sh::T, S = Sh::S;
  constexpr int R = Sh::rad(s);
  constexpr int Ns = Sh::ns(s);
  constexpr int NB = L / R;
  constexpr int PER = (NB + T - 1) / T;
  constexpr bool EVEN = (NB % T) == 0;
  constexpr bool FIRST_REG = (s == 0) && EVEN;
  constexpr bool LAST_REG = (s == S - 1) && EVEN;

  if constexpr (s == 0 && !FIRST_REG) {
#pragma unroll
    for (int m = 0; m < Sh::E; ++m) lds[(t + T * m) * kst] = home[m];
    xsync<WS>();
  }

  C v[PER][R];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int j = t + T * u;
    if (EVEN || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (FIRST_REG) v[u][r] = home[u + r * (NB / T)];
        else v[u][r] = lds[(j + r * NB) * kst];
      }
      if constexpr (FMA && s > 0 && (R == 2 || R == 4 || R == 8 || R == 16)) {
        C w[R - 1];
#pragma unroll
        for (int r = 1; r < R; ++r) w[r - 1] = lt.w[LaneTw<C, Sh>::off(s) + u * (R - 1) + r - 1];
        tw_dft<R, DIR>(v[u], w);
      } else {
        if constexpr (s > 0) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const C w = lt.w[LaneTw<C, Sh>::off(s) + u * (R - 1) + r - 1];
            v[u][r] = (DIR > 0) ? cmulc(v[u][r], w) : cmul(v[u][r], w);
          }
        }
        dft<R, DIR>(v[u]);
      }
    }
  }

  if constexpr (LAST_REG) {
#pragma unroll
    for (int u = 0; u < PER; ++u)
#pragma unroll
      for (int q = 0; q < R; ++q) home[u + q * (NB / T)] = v[u][q];
    if constexpr (!FIRST_REG) xsync<WS>();  // LDS reads of this stage done before reuse
  } else {
    if constexpr (!FIRST_REG) xsync<WS>();  // every lane has read this stage's inputs
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int j = t + T * u;
      if (EVEN || j < NB) {
        const int k = j % Ns;
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) lds[(base + q * Ns) * kst] = v[u][q];
      }
    }
    xsync<WS>();
    if constexpr (s == S - 1) {
#pragma unroll
      for (int m = 0; m < Sh::E; ++m) home[m] = lds[(t + T * m) * kst];
      xsync<WS>();
    }
  }
  if constexpr (s + 1 < S) fft_stage<C, Sh, DIR, s + 1, WS, FMA>(home, lds, kst, t, lt);
}

// Unnormalised DFT of one pencil (DIR = -1 forward, +1 inverse).
template <int DIR, typename Sh, bool WS = false, bool FMA = false, typename C>
__device__ __forceinline__ void fft_pencil(C (&home)[Sh::E], C* lds, int kst, int t, const LaneTw<C, Sh>& lt) {
  static_assert(shape_ok<Sh>(), "bad radix plan");
  static_assert(!WS || (64 % Sh::T) == 0, "wave sync needs whole pencils per wavefront");
  fft_stage<C, Sh, DIR, 0, WS, FMA>(home, lds, kst, t, lt);
}

// LDS index of entry i of a pencil row under swizzle SWZ. 0: none. 1: bits
// 4-5 of i XOR-ed into bits 0-1 and 2-3 (a permutation inside every block of
// 16 entries, so rows of a multiple of 16 entries stay in place). For rows of
// 32-lane pencils with 4 entries per lane (length 128 with radices 4, 4, 2,
// 4) it moves the stride-4 writes of the first exchange (entries 4t + q) and
// the blocked writes of the second ((t / 4) 16 + t % 4 + 4q) onto distinct
// banks within each 16 lanes, while the unit-stride reads stay conflict free.
template <int SWZ> __device__ __forceinline__ int lswz(int i) {
  if constexpr (SWZ == 1) return i ^ (((i >> 4) & 3) * 5);
  else return i;
}

// NP pencils of one lane advanced stage by stage together: pencil p's LDS row
// is lds + p * pstride. Every exchange fences once for all NP pencils, and the
// NP independent butterfly chains give the scheduler work to overlap with
// LDS and memory latency.
template <typename C, typename Sh, int DIR, int s, bool WS, int NP, bool FMA, int SWZ>
__device__ __forceinline__ void fft_stage_multi(C (&home)[NP][Sh::E], C* lds, int pstride, int kst, int t,
                                                const LaneTw<C, Sh>& lt) {
  constexpr int L = Sh::L, T = Sh::T, S = Sh::S;
  constexpr int R = Sh::rad(s);
  constexpr int Ns = Sh::ns(s);
  constexpr int NB = L / R;
  constexpr int PER = (NB + T - 1) / T;
  constexpr bool EVEN = (NB % T) == 0;
  constexpr bool FIRST_REG = (s == 0) && EVEN;
  constexpr bool LAST_REG = (s == S - 1) && EVEN;

  if constexpr (s == 0 && !FIRST_REG) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int m = 0; m < Sh::E; ++m) lds[p * pstride + lswz<SWZ>(t + T * m) * kst] = home[p][m];
    xsync<WS>();
  }

  C v[NP][PER][R];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int j = t + T * u;
      if (EVEN || j < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if constexpr (FIRST_REG) v[p][u][r] = home[p][u + r * (NB / T)];
          else v[p][u][r] = lds[p * pstride + lswz<SWZ>(j + r * NB) * kst];
        }
        if constexpr (FMA && s > 0 && (R == 2 || R == 4 || R == 8 || R == 16)) {
          C w[R - 1];
#pragma unroll
          for (int r = 1; r < R; ++r) w[r - 1] = lt.w[LaneTw<C, Sh>::off(s) + u * (R - 1) + r - 1];
          tw_dft<R, DIR>(v[p][u], w);
        } else {
          if constexpr (s > 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
              const C w = lt.w[LaneTw<C, Sh>::off(s) + u * (R - 1) + r - 1];
              v[p][u][r] = (DIR > 0) ? cmulc(v[p][u][r], w) : cmul(v[p][u][r], w);
            }
          }
          dft<R, DIR>(v[p][u]);
        }
      }
    }

  if constexpr (LAST_REG) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int u = 0; u < PER; ++u)
#pragma unroll
        for (int q = 0; q < R; ++q) home[p][u + q * (NB / T)] = v[p][u][q];
    if constexpr (!FIRST_REG) xsync<WS>();
  } else {
    if constexpr (!FIRST_REG) xsync<WS>();
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int j = t + T * u;
        if (EVEN || j < NB) {
          const int k = j % Ns;
          const int base = (j / Ns) * Ns * R + k;
#pragma unroll
          for (int q = 0; q < R; ++q) lds[p * pstride + lswz<SWZ>(base + q * Ns) * kst] = v[p][u][q];
        }
      }
    xsync<WS>();
    if constexpr (s == S - 1) {
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int m = 0; m < Sh::E; ++m) home[p][m] = lds[p * pstride + lswz<SWZ>(t + T * m) * kst];
      xsync<WS>();
    }
  }
  if constexpr (s + 1 < S) fft_stage_multi<C, Sh, DIR, s + 1, WS, NP, FMA, SWZ>(home, lds, pstride, kst, t, lt);
}

// Unnormalised DFTs of NP pencils of the same lane (DIR = -1 forward, +1 inverse),
// their LDS rows indexed through lswz<SWZ>.
template <int DIR, typename Sh, bool WS, int NP, bool FMA = false, int SWZ = 0, typename C>
__device__ __forceinline__ void fft_pencils(C (&home)[NP][Sh::E], C* lds, int pstride, int kst, int t,
                                            const LaneTw<C, Sh>& lt) {
  static_assert(shape_ok<Sh>(), "bad radix plan");
  static_assert(!WS || (64 % Sh::T) == 0, "wave sync needs whole pencils per wavefront");
  static_assert(SWZ == 0 || Sh::L % 16 == 0, "the swizzle permutes blocks of 16 entries");
  fft_stage_multi<C, Sh, DIR, 0, WS, NP, FMA, SWZ>(home, lds, pstride, kst, t, lt);
}

}  // namespace sfft
