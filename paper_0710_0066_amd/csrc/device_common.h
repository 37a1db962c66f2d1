// Device-side helpers shared by the gfx950 kernels: complex arithmetic, the even-odd
// site indexing of the library layout, SU(3) x colour-vector products and the
// (1 -/+ gamma_mu) half-spinor projections of the chiral basis.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace sap {

// ---------------------------------------------------------------------------------
// complex numbers
template <class R> struct cx { R r, i; };

template <class R> __device__ __forceinline__ cx<R> cmk(R r, R i) { return {r, i}; }
template <class R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.r + b.r, a.i + b.i}; }
template <class R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.r - b.r, a.i - b.i}; }
template <class R> __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.r, -a.i}; }
template <class R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.r, s * a.i}; }
template <class R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
// conj(a) * b
template <class R> __device__ __forceinline__ cx<R> cjmul(cx<R> a, cx<R> b) {
  return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
// a * conj(b)
template <class R> __device__ __forceinline__ cx<R> cmulj(cx<R> a, cx<R> b) {
  return {a.r * b.r + a.i * b.i, a.i * b.r - a.r * b.i};
}
template <class R> __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.i, a.r}; }
template <class R> __device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.i, -a.r}; }
template <class R> __device__ __forceinline__ cx<R> cfma(cx<R> acc, cx<R> a, cx<R> b) {
  acc.r = fma(a.r, b.r, acc.r); acc.r = fma(-a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i); acc.i = fma(a.i, b.r, acc.i);
  return acc;
}
// acc + conj(a) * b
template <class R> __device__ __forceinline__ cx<R> cjfma(cx<R> acc, cx<R> a, cx<R> b) {
  acc.r = fma(a.r, b.r, acc.r); acc.r = fma(a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i); acc.i = fma(-a.i, b.r, acc.i);
  return acc;
}

// third row of an SU(3) matrix from its first two (m[0..5], row-major): the rows are
// orthonormal with unit determinant, so row 3 = conj(row 1 x row 2)
template <class R> __device__ __forceinline__ void third_row(cx<R> m[9]) {
  const cx<R> a0 = m[0], a1 = m[1], a2 = m[2], b0 = m[3], b1 = m[4], b2 = m[5];
  const cx<R> c0 = cmul(a1, b2) - cmul(a2, b1);
  const cx<R> c1 = cmul(a2, b0) - cmul(a0, b2);
  const cx<R> c2 = cmul(a0, b1) - cmul(a1, b0);
  m[6] = {c0.r, -c0.i};
  m[7] = {c1.r, -c1.i};
  m[8] = {c2.r, -c2.i};
}

// FP16 storage tag: spinor components as half2 with one FP32 norm per site (the largest
// component magnitude of the site), links as plain half2; arithmetic in FP32
struct h16 {};

// storage vector type of one complex number
template <class R> struct vec2;
template <> struct vec2<double> { typedef double2 type; };
template <> struct vec2<float> { typedef float2 type; };
template <> struct vec2<h16> { typedef __half2 type; };

// arithmetic type of a storage type
template <class S> struct arith { typedef S type; };
template <> struct arith<h16> { typedef float type; };

template <class R> __device__ __forceinline__ cx<R> ld(const typename vec2<R>::type* p) {
  typename vec2<R>::type v = *p;
  return {v.x, v.y};
}
template <class R> __device__ __forceinline__ void st(typename vec2<R>::type* p, cx<R> a) {
  typename vec2<R>::type v;
  v.x = a.r; v.y = a.i;
  *p = v;
}

// ---------------------------------------------------------------------------------
// Tiled structure-of-arrays ("AoSoA") addressing of the library layout: sites of one
// parity are grouped in tiles of TILE = 64 (one wavefront); inside a tile block all
// NC components are stored one after the other, each as TILE consecutive complex
// numbers. A wavefront load of one component of 64 consecutive sites is one contiguous
// run, and the whole footprint of a tile is a few KB instead of NC far-apart streams.
constexpr int TILE = 64;
__device__ __host__ __forceinline__ long long tiled(long long j, int c, int NC) {
  return ((j >> 6) * NC + c) * TILE + (j & (TILE - 1));
}

// Spinor sites in storage R. FP64 fields keep the tiled layout above (12 components of 16
// bytes). FP32 fields store the 12 complex components of a site in 6 pairs (2k, 2k + 1),
// each pair one 16-byte word, in the same tiled scheme with 6 components: pair k of site j
// is float4 number tiled(j, k, 6) of the (rhs, parity) block, i.e. complex number
// ((j / 64) * 12 + 2k) * 64 + 2 (j % 64) + (c % 2) for component c = 2k + c % 2. A work-item
// then moves a site with 6 loads or stores instead of 12. FP16 fields (two-half complex,
// 4 bytes) store the components in quads (4k .. 4k + 3), one 16-byte word each: entry
// ((j / 64) * 12 + 4k) * 64 + 4 (j % 64) + (c % 4) for component c = 4k + c % 4, so a site
// is 3 loads.
template <class R> __device__ __host__ __forceinline__ long long sidx(long long j, int c) {
  if constexpr (std::is_same<R, float>::value) return ((j >> 6) * 12 + (c & ~1)) * TILE + 2 * (j & (TILE - 1)) + (c & 1);
  else if constexpr (std::is_same<R, h16>::value)
    return ((j >> 6) * 12 + (c & ~3)) * TILE + 4 * (j & (TILE - 1)) + (c & 3);
  else return tiled(j, c, 12);
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

// the 12 components of site j of one (rhs, parity) block of a spinor field
template <class R>
__device__ __forceinline__ void ld_site(const typename vec2<R>::type* blk, long long j, cx<R> v[12]) {
  if constexpr (std::is_same<R, float>::value) {
    const f4v* q = (const f4v*)blk + tiled(j, 0, 6);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const f4v w = q[k * TILE];
      v[2 * k] = {w.x, w.y};
      v[2 * k + 1] = {w.z, w.w};
    }
  } else {
    const typename vec2<R>::type* q = blk + tiled(j, 0, 12);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const typename vec2<R>::type w = q[c * TILE];
      v[c] = {w.x, w.y};
    }
  }
}

// store the 12 components of site j (NT: non-temporal stores)
template <class R, bool NT = false>
__device__ __forceinline__ void st_site(typename vec2<R>::type* blk, long long j, const cx<R> v[12]) {
  if constexpr (std::is_same<R, float>::value) {
    f4v* q = (f4v*)blk + tiled(j, 0, 6);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const f4v w = {v[2 * k].r, v[2 * k].i, v[2 * k + 1].r, v[2 * k + 1].i};
      if (NT) __builtin_nontemporal_store(w, q + k * TILE);
      else q[k * TILE] = w;
    }
  } else {
    typename vec2<R>::type* q = blk + tiled(j, 0, 12);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      if (NT) {
        __builtin_nontemporal_store(v[c].r, &q[c * TILE].x);
        __builtin_nontemporal_store(v[c].i, &q[c * TILE].y);
      } else {
        typename vec2<R>::type w;
        w.x = v[c].r;
        w.y = v[c].i;
        q[c * TILE] = w;
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// geometry of the even-odd layout: site j of a parity is the lexicographic index / 2,
// j = ((x0*L1 + x1)*L2 + x2)*L3h + x3h with L3h = L3/2 and x3 = 2*x3h + b,
// b = (p + x0 + x1 + x2) & 1.
struct Geo {
  int L0, L1, L2, L3;
  int L3h;        // L3 / 2
  int V3h;        // L1*L2*L3/2: sites of one parity in one x0 slice
  long long Vh;   // V / 2
  long long Vhp;  // Vh rounded up to a multiple of TILE (storage sites per parity)
};

struct Site {
  int x0, x1, x2, x3h, b;   // b: low bit of x3
};

__device__ __forceinline__ Site decode(const Geo& g, long long j, int p) {
  Site s;
  long long r = j / g.L3h;
  s.x3h = (int)(j - r * g.L3h);
  long long r2 = r / g.L2;
  s.x2 = (int)(r - r2 * g.L2);
  long long r3 = r2 / g.L1;
  s.x1 = (int)(r2 - r3 * g.L1);
  s.x0 = (int)r3;
  s.b = (p + s.x0 + s.x1 + s.x2) & 1;
  return s;
}

// eo index of the neighbour x +/- mu (opposite parity). dir = +1 forward, -1 backward.
__device__ __forceinline__ long long nbr(const Geo& g, const Site& s, long long j, int mu, int dir) {
  switch (mu) {
    case 0: {
      int y = s.x0 + dir;
      if (y == g.L0) return j - (long long)(g.L0 - 1) * g.V3h;
      if (y < 0) return j + (long long)(g.L0 - 1) * g.V3h;
      return j + (long long)dir * g.V3h;
    }
    case 1: {
      long long st = (long long)g.L2 * g.L3h;
      int y = s.x1 + dir;
      if (y == g.L1) return j - (long long)(g.L1 - 1) * st;
      if (y < 0) return j + (long long)(g.L1 - 1) * st;
      return j + dir * st;
    }
    case 2: {
      int y = s.x2 + dir;
      if (y == g.L2) return j - (long long)(g.L2 - 1) * g.L3h;
      if (y < 0) return j + (long long)(g.L2 - 1) * g.L3h;
      return j + (long long)dir * g.L3h;
    }
    default: {
      long long row = j - s.x3h;
      int h;
      if (dir > 0) {
        h = s.b ? s.x3h + 1 : s.x3h;
        if (h == g.L3h) h = 0;
      } else {
        h = s.b ? s.x3h : s.x3h - 1;
        if (h < 0) h = g.L3h - 1;
      }
      return row + h;
    }
  }
}

// ---------------------------------------------------------------------------------
// SU(3) (3x3 complex, row-major m[3*row+col]) times colour vectors
template <class R>
__device__ __forceinline__ void su3_mul(const cx<R> m[9], const cx<R> v[3], cx<R> w[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> t = cmul(m[3 * a], v[0]);
    t = cfma(t, m[3 * a + 1], v[1]);
    t = cfma(t, m[3 * a + 2], v[2]);
    w[a] = t;
  }
}
// m^dagger v
template <class R>
__device__ __forceinline__ void su3_dag_mul(const cx<R> m[9], const cx<R> v[3], cx<R> w[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> t = cjmul(m[a], v[0]);
    t = cjfma(t, m[3 + a], v[1]);
    t = cjfma(t, m[6 + a], v[2]);
    w[a] = t;
  }
}

// ---------------------------------------------------------------------------------
// Half-spinor projection of the chiral basis. Spinor s[spin][colour], upper spins u =
// (s0, s1), lower d = (s2, s3). MINUS = (1 - gamma_mu), PLUS = (1 + gamma_mu).
//   mu=0: (1-g0): h = u + d,            lower = h
//         (1+g0): h = u - d,            lower = -h
//   mu=1: (1-g1): h = (u0 + i d1, u1 + i d0),  lower = (-i h1, -i h0)
//         (1+g1): h = (u0 - i d1, u1 - i d0),  lower = ( i h1,  i h0)
//   mu=2: (1-g2): h = (u0 + d1, u1 - d0),      lower = (-h1,  h0)
//         (1+g2): h = (u0 - d1, u1 + d0),      lower = ( h1, -h0)
//   mu=3: (1-g3): h = (u0 + i d0, u1 - i d1),  lower = (-i h0,  i h1)
//         (1+g3): h = (u0 - i d0, u1 + i d1),  lower = ( i h0, -i h1)
template <class R>
__device__ __forceinline__ void project(int mu, bool plus, const cx<R> s[4][3], cx<R> h[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> u0 = s[0][c], u1 = s[1][c], d0 = s[2][c], d1 = s[3][c];
    switch (mu) {
      case 0:
        h[0][c] = plus ? u0 - d0 : u0 + d0;
        h[1][c] = plus ? u1 - d1 : u1 + d1;
        break;
      case 1:
        h[0][c] = plus ? u0 - times_i(d1) : u0 + times_i(d1);
        h[1][c] = plus ? u1 - times_i(d0) : u1 + times_i(d0);
        break;
      case 2:
        h[0][c] = plus ? u0 - d1 : u0 + d1;
        h[1][c] = plus ? u1 + d0 : u1 - d0;
        break;
      default:
        h[0][c] = plus ? u0 - times_i(d0) : u0 + times_i(d0);
        h[1][c] = plus ? u1 + times_i(d1) : u1 - times_i(d1);
        break;
    }
  }
}

// acc += reconstruct(g)
template <class R>
__device__ __forceinline__ void accum_recon(int mu, bool plus, const cx<R> g[2][3], cx<R> acc[4][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[0][c] = acc[0][c] + g[0][c];
    acc[1][c] = acc[1][c] + g[1][c];
    switch (mu) {
      case 0:
        if (plus) { acc[2][c] = acc[2][c] - g[0][c]; acc[3][c] = acc[3][c] - g[1][c]; }
        else      { acc[2][c] = acc[2][c] + g[0][c]; acc[3][c] = acc[3][c] + g[1][c]; }
        break;
      case 1:
        if (plus) { acc[2][c] = acc[2][c] + times_i(g[1][c]); acc[3][c] = acc[3][c] + times_i(g[0][c]); }
        else      { acc[2][c] = acc[2][c] - times_i(g[1][c]); acc[3][c] = acc[3][c] - times_i(g[0][c]); }
        break;
      case 2:
        if (plus) { acc[2][c] = acc[2][c] + g[1][c]; acc[3][c] = acc[3][c] - g[0][c]; }
        else      { acc[2][c] = acc[2][c] - g[1][c]; acc[3][c] = acc[3][c] + g[0][c]; }
        break;
      default:
        if (plus) { acc[2][c] = acc[2][c] + times_i(g[0][c]); acc[3][c] = acc[3][c] - times_i(g[1][c]); }
        else      { acc[2][c] = acc[2][c] - times_i(g[0][c]); acc[3][c] = acc[3][c] + times_i(g[1][c]); }
        break;
    }
  }
}

// acc += w * reconstruct(g) (w real), with one fused multiply-add per real component
template <class R>
__device__ __forceinline__ void accum_recon_scaled(int mu, bool plus, const cx<R> g[2][3], R w, cx<R> acc[4][3]) {
  auto fma_c = [&](cx<R>& a, const cx<R>& v, R s) {   // a += s * v (contracted to FMA)
    a.r = s * v.r + a.r;
    a.i = s * v.i + a.i;
  };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    fma_c(acc[0][c], g[0][c], w);
    fma_c(acc[1][c], g[1][c], w);
    switch (mu) {
      case 0:
        fma_c(acc[2][c], g[0][c], plus ? -w : w);
        fma_c(acc[3][c], g[1][c], plus ? -w : w);
        break;
      case 1:
        fma_c(acc[2][c], times_i(g[1][c]), plus ? w : -w);
        fma_c(acc[3][c], times_i(g[0][c]), plus ? w : -w);
        break;
      case 2:
        fma_c(acc[2][c], g[1][c], plus ? w : -w);
        fma_c(acc[3][c], g[0][c], plus ? -w : w);
        break;
      default:
        fma_c(acc[2][c], times_i(g[0][c]), plus ? w : -w);
        fma_c(acc[3][c], times_i(g[1][c]), plus ? -w : w);
        break;
    }
  }
}

// Is a site on slice x0 in a selected x0 block of length slb (slb = 0: no restriction)?
// block >= 0: only that block; else colour 0 all, 1 black (odd index), 2 white (even).
__device__ __forceinline__ bool block_sel(int x0, int slb, int block, int colour) {
  if (!slb) return true;
  const int blk = x0 / slb;
  if (block >= 0) return blk == block;
  return colour == 0 || ((colour == 1) == ((blk & 1) == 1));
}

// Block selection code used by the block-restricted kernels: 0 all blocks, 1 black (odd
// block index), 2 white (even), 3 + b the single block b.
__device__ __host__ __forceinline__ bool block_selected(int sel, int blk) {
  if (sel >= 3) return blk == sel - 3;
  return sel == 0 || ((sel == 1) == ((blk & 1) == 1));
}

// XCD-aware workgroup order: the hardware deals consecutive workgroup ids round-robin
// to the 8 XCDs; when the grid is a multiple of 8, renumber so that each XCD walks a
// contiguous range of logical workgroups (neighbouring tiles share that XCD's L2).
__device__ __forceinline__ long long xcd_logical_block(long long w, long long nwg) {
  if ((nwg & 7) != 0) return w;
  return (w & 7) * (nwg >> 3) + (w >> 3);
}

}  // namespace sap
