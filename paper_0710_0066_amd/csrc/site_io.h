// Per-site access to spinor fields of any storage type (double, float, h16). A reader
// yields the 12 components of one site at the arithmetic precision; a writer takes them
// one by one. For FP16 storage (h16) the components of a site are stored divided by the
// site norm (their largest magnitude, FP32): the reader scales by it, and the writer
// buffers the site and stores it, with its new norm, at close(); its components are stored
// in quads, one 16-byte word each (sidx). FP32 sites are stored as
// 6 pairs of components, one 16-byte word each (sidx): the reader loads a pair per two
// components (the compiler keeps one load for both), and the writer buffers the site and
// stores the 6 pairs at close(). For double a writer stores each component at once.
#pragma once
#include <type_traits>
#include "internal.h"

namespace sap {

template <class R> constexpr bool is_h16 = std::is_same<R, h16>::value;
template <class R> constexpr bool is_f32 = std::is_same<R, float>::value;
template <class R> using arith_t = typename arith<R>::type;

// norms of block (rhs, parity p) of an FP16 field
__device__ __forceinline__ float* norm_ptr16(const Field<h16>& f, int rhs, int p, long long Vhp) {
  return (float*)(f.ptr + rhs * f.rs + f.no) + (f.ps ? p : 0) * Vhp;
}

template <class R> struct SiteR {
  const typename vec2<R>::type* b;   // component 0 of the site; component c at b + c*TILE
                                     // (FP32: pair k = components 2k, 2k + 1 at b + 2k*TILE)
  float m;                           // h16: site norm
};

template <class R>
__device__ __forceinline__ SiteR<R> site_r(const Field<R>& f, int rhs, int p, long long j, long long Vhp) {
  SiteR<R> s;
  s.b = f.ptr + rhs * f.rs + p * f.ps + sidx<R>(j, 0);
  if constexpr (is_h16<R>) s.m = norm_ptr16(f, rhs, p, Vhp)[j];
  else s.m = 1.0f;
  return s;
}

typedef unsigned u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __half2 h2_of(unsigned u) { return __builtin_bit_cast(__half2, u); }
__device__ __forceinline__ unsigned u_of(__half2 h) { return __builtin_bit_cast(unsigned, h); }

// ---------------------------------------------------------------------------------
// Packed-FP16 form of one hop term (FP16 storage). A site's stored (norm-divided) half2
// components are projected with packed FP16 adds: each projected component is the sum of
// two halves rounded once, the value of an FP32 sum rounded to FP16. The SU(3) product
// runs on v_dot2_f32_f16: its two FP16 x FP16 products are exact in FP32 and added in
// FP32. Apart from the rounding of the projected half spinor (and of the rebuilt third
// link row) to FP16, the term is thus computed in FP32, without converting the stored
// components of the neighbour. The projection writes each colour component h of the
// half spinor as the two operands the complex products need:
//   w = u h:        re = dot2(u, (h.r, -h.i)),  im = dot2(u, (h.i,  h.r))
//   w = conj(u) h:  re = dot2(u, (h.r,  h.i)),  im = dot2(u, (h.i, -h.r))
// with u = (u.r, u.i) the stored link entry; the swaps and signs fold into the operand
// modifiers of the packed adds.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2v hv(unsigned u) { return __builtin_bit_cast(h2v, u); }

// the compiler's own dot2 (not inline asm: a DOT result read soon after by another DOT or
// VALU instruction needs wait states that only the compiler's hazard recognizer inserts)
__device__ __forceinline__ float dot2(unsigned a, h2v b, float c) { return __builtin_amdgcn_fdot2(hv(a), b, c, false); }

// the six stored entries (rows 0 and 1) of an FP16 link as half2 words: t points at the
// link's block of its tile row (p*24*Vhp + (j / 64)*24*64 + 6 mu*64), lane = j % 64 (a quad
// and a pair, see the layout of the reduced link copies)
__device__ __forceinline__ void load_link16_words(const __half2* t, int lane, unsigned e[6]) {
  const u4v q = *(const u4v*)(t + 4 * lane);
  typedef unsigned u2v __attribute__((ext_vector_type(2)));
  const u2v d = *(const u2v*)(t + 4 * TILE + 2 * lane);
  e[0] = q.x; e[1] = q.y; e[2] = q.z; e[3] = q.w; e[4] = d.x; e[5] = d.y;
}

// the nine entries of an FP16 link of the three-row copy as half2 words: t points at the
// link's block of its tile row (48*Vhp + p*36*Vhp + (j / 64)*36*64 + 9 mu*64), lane =
// j % 64 (two quads and a single entry; three loads)
__device__ __forceinline__ void load_link16x3_words(const __half2* t, int lane, unsigned e[9]) {
  const u4v q0 = *(const u4v*)(t + 4 * lane);
  const u4v q1 = *(const u4v*)(t + 4 * TILE + 4 * lane);
  e[0] = q0.x; e[1] = q0.y; e[2] = q0.z; e[3] = q0.w;
  e[4] = q1.x; e[5] = q1.y; e[6] = q1.z; e[7] = q1.w;
  e[8] = *(const unsigned*)(t + 8 * TILE + lane);
}

// e[6..8] = third row of the link from its stored rows e[0..5], rebuilt in FP32 (unitarity
// and unit determinant) and rounded to FP16
__device__ __forceinline__ void third_row16(unsigned e[9]) {
  cx<float> m[9];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float2 f = __half22float2(h2_of(e[i]));
    m[i] = {f.x, f.y};
  }
  third_row<float>(m);
#pragma unroll
  for (int i = 6; i < 9; ++i) e[i] = u_of(__floats2half2_rn(m[i].r, m[i].i));
}

// the (1 -/+ gamma_mu) projection of the chiral basis (device_common.h, project) of
// packed components s[3*spin + colour], as the operand pairs (x, y) of the products with
// U (plus false) or U^dagger (plus true); G5I: gamma_5 is applied to s first
template <bool G5I>
__device__ __forceinline__ void project16(int mu, bool plus, const unsigned s[12], h2v x[2][3], h2v y[2][3]) {
  auto ti = [](h2v v) { return h2v{-v.y, v.x}; };   // i v
  // h = u + dp
  auto put2 = [&](h2v u, h2v dp, h2v& hx, h2v& hy) {
    if (!plus) {
      hx = h2v{u.x, -u.y} + h2v{dp.x, -dp.y};
      hy = h2v{u.y, u.x} + h2v{dp.y, dp.x};
    } else {
      hx = u + dp;
      hy = h2v{u.y, -u.x} + h2v{dp.y, -dp.x};
    }
  };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const h2v u0 = hv(s[c]), u1 = hv(s[3 + c]);
    h2v d0 = hv(s[6 + c]), d1 = hv(s[9 + c]);
    if (G5I) { d0 = -d0; d1 = -d1; }
    switch (mu) {
      case 0:
        put2(u0, plus ? -d0 : d0, x[0][c], y[0][c]);
        put2(u1, plus ? -d1 : d1, x[1][c], y[1][c]);
        break;
      case 1:
        put2(u0, plus ? -ti(d1) : ti(d1), x[0][c], y[0][c]);
        put2(u1, plus ? -ti(d0) : ti(d0), x[1][c], y[1][c]);
        break;
      case 2:
        put2(u0, plus ? -d1 : d1, x[0][c], y[0][c]);
        put2(u1, plus ? d0 : -d0, x[1][c], y[1][c]);
        break;
      default:
        put2(u0, plus ? -ti(d0) : ti(d0), x[0][c], y[0][c]);
        put2(u1, plus ? ti(d1) : -ti(d1), x[1][c], y[1][c]);
        break;
    }
  }
}

// w = U h (dag false) or U^dagger h (dag true) for the link entries e[9] (row-major half2
// words) and the operand pairs of one projected colour vector h
__device__ __forceinline__ void su3_dot2(bool dag, const unsigned e[9], const h2v x[3], const h2v y[3],
                                         cx<float> w[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    auto U = [&](int b) { return dag ? e[3 * b + a] : e[3 * a + b]; };
    float re = dot2(U(0), x[0], 0.0f);
    float im = dot2(U(0), y[0], 0.0f);
    re = dot2(U(1), x[1], re);
    im = dot2(U(1), y[1], im);
    re = dot2(U(2), x[2], re);
    im = dot2(U(2), y[2], im);
    w[a] = {re, im};
  }
}

// w = U h or U^dagger h (plus) of the projection of the packed spinor s
template <bool G5I>
__device__ __forceinline__ void hop16_term(int mu, bool plus, const unsigned e[9], const unsigned s[12],
                                           cx<float> w[2][3]) {
  h2v x[2][3], y[2][3];
  project16<G5I>(mu, plus, s, x, y);
  su3_dot2(plus, e, x[0], y[0], w[0]);
  su3_dot2(plus, e, x[1], y[1], w[1]);
}

template <class R> __device__ __forceinline__ cx<arith_t<R>> get(const SiteR<R>& s, int c) {
  if constexpr (is_h16<R>) {
    const u4v w = *(const u4v*)(s.b + (c & ~3) * TILE);
    const unsigned u = (c & 3) == 0 ? w.x : (c & 3) == 1 ? w.y : (c & 3) == 2 ? w.z : w.w;
    const float2 v = __half22float2(h2_of(u));
    return {v.x * s.m, v.y * s.m};
  } else if constexpr (is_f32<R>) {
    const f4v w = *(const f4v*)(s.b + (c & ~1) * TILE);
    return (c & 1) ? cx<float>{w.z, w.w} : cx<float>{w.x, w.y};
  } else {
    return ld<R>(s.b + c * TILE);
  }
}

template <class R> struct SiteW {
  typename vec2<R>::type* b;
  float* n;                              // h16: where the site norm goes
  cx<float> v[(is_h16<R> || is_f32<R>) ? 12 : 1];   // h16, FP32: the buffered site
};

template <class R>
__device__ __forceinline__ SiteW<R> site_w(const Field<R>& f, int rhs, int p, long long j, long long Vhp) {
  SiteW<R> w;
  w.b = f.ptr + rhs * f.rs + p * f.ps + sidx<R>(j, 0);
  if constexpr (is_h16<R>) w.n = norm_ptr16(f, rhs, p, Vhp) + j;
  else w.n = nullptr;
  return w;
}

template <class R> __device__ __forceinline__ void put(SiteW<R>& w, int c, cx<arith_t<R>> a) {
  if constexpr (is_h16<R> || is_f32<R>) w.v[c] = a;
  else st<R>(w.b + c * TILE, a);
}

template <class R> __device__ __forceinline__ void close(SiteW<R>& w) {
  if constexpr (is_h16<R>) {
    float m = 0.0f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(w.v[c].r), fabsf(w.v[c].i)));
    const float inv = m > 0.0f ? 1.0f / m : 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      u4v q;
      q.x = u_of(__floats2half2_rn(w.v[4 * k].r * inv, w.v[4 * k].i * inv));
      q.y = u_of(__floats2half2_rn(w.v[4 * k + 1].r * inv, w.v[4 * k + 1].i * inv));
      q.z = u_of(__floats2half2_rn(w.v[4 * k + 2].r * inv, w.v[4 * k + 2].i * inv));
      q.w = u_of(__floats2half2_rn(w.v[4 * k + 3].r * inv, w.v[4 * k + 3].i * inv));
      *(u4v*)(w.b + 4 * k * TILE) = q;
    }
    *w.n = m;
  } else if constexpr (is_f32<R>) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
      *(f4v*)(w.b + 2 * k * TILE) = f4v{w.v[2 * k].r, w.v[2 * k].i, w.v[2 * k + 1].r, w.v[2 * k + 1].i};
  }
}

}  // namespace sap
