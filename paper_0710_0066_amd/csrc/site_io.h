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

// the six stored entries of an FP16 link: t points at the link's block of its tile row
// (p*24*Vhp + (j / 64)*24*64 + 6 mu*64), lane = j % 64 (a quad and a pair, see the layout)
__device__ __forceinline__ void load_link16_raw(const __half2* t, int lane, cx<float> raw[6]) {
  const u4v q = *(const u4v*)(t + 4 * lane);
  typedef unsigned u2v __attribute__((ext_vector_type(2)));
  const u2v d = *(const u2v*)(t + 4 * TILE + 2 * lane);
  const unsigned e[6] = {q.x, q.y, q.z, q.w, d.x, d.y};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float2 h = __half22float2(h2_of(e[i]));
    raw[i] = {h.x, h.y};
  }
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
