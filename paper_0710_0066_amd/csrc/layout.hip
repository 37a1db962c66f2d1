// Conversions between the canonical interchange layout (lexicographic sites,
// array-of-structures complex128) and the library's even-odd structure-of-arrays
// layout. One work-item per site (and rhs); not on the hot path.
#include "internal.h"
#include "link_copies.h"

namespace sap {

struct Lex {
  int x0, x1, x2, x3;
};

__device__ __forceinline__ Lex lex_coords(const Geo& g, long long i) {
  Lex c;
  c.x3 = (int)(i % g.L3); i /= g.L3;
  c.x2 = (int)(i % g.L2); i /= g.L2;
  c.x1 = (int)(i % g.L1);
  c.x0 = (int)(i / g.L1);
  return c;
}

template <class R>
__global__ void pack_spinor_kernel(Geo g, typename vec2<R>::type* out, const double2* in, int nrhs) {
  const long long V = 2 * g.Vh;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V * nrhs) return;
  const long long rhs = t / V, i = t - rhs * V;
  const Lex c = lex_coords(g, i);
  const int p = (c.x0 + c.x1 + c.x2 + c.x3) & 1;
  const long long j = i >> 1;
  typename vec2<R>::type* o = out + (rhs * 2 + p) * 12 * g.Vhp;
  const double2* src = in + (rhs * V + i) * 12;
  for (int k = 0; k < 12; ++k) {
    double2 v = src[k];
    typename vec2<R>::type w;
    w.x = (R)v.x; w.y = (R)v.y;
    o[sidx<R>(j, k)] = w;
  }
}

template <class R>
__global__ void unpack_spinor_kernel(Geo g, double2* out, const typename vec2<R>::type* in, int nrhs) {
  const long long V = 2 * g.Vh;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V * nrhs) return;
  const long long rhs = t / V, i = t - rhs * V;
  const Lex c = lex_coords(g, i);
  const int p = (c.x0 + c.x1 + c.x2 + c.x3) & 1;
  const long long j = i >> 1;
  const typename vec2<R>::type* src = in + (rhs * 2 + p) * 12 * g.Vhp;
  double2* o = out + (rhs * V + i) * 12;
  for (int k = 0; k < 12; ++k) {
    typename vec2<R>::type v = src[sidx<R>(j, k)];
    o[k] = make_double2((double)v.x, (double)v.y);
  }
}

__global__ void pack_gauge_kernel(Geo g, double2* U64, float2* U32, const double2* in) {
  const long long V = 2 * g.Vh;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const Lex c = lex_coords(g, i);
  const int p = (c.x0 + c.x1 + c.x2 + c.x3) & 1;
  const long long j = i >> 1;
  for (int mu = 0; mu < 4; ++mu)
    for (int e = 0; e < 9; ++e) {
      double2 v = in[(i * 4 + mu) * 9 + e];
      long long k = p * 36 * g.Vhp + tiled(j, 9 * mu + e, 36);
      U64[k] = v;
      if (U32) U32[k] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void unpack_gauge_kernel(Geo g, double2* out, const double2* U64) {
  const long long V = 2 * g.Vh;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const Lex c = lex_coords(g, i);
  const int p = (c.x0 + c.x1 + c.x2 + c.x3) & 1;
  const long long j = i >> 1;
  for (int mu = 0; mu < 4; ++mu)
    for (int e = 0; e < 9; ++e)
      out[(i * 4 + mu) * 9 + e] = U64[p * 36 * g.Vhp + tiled(j, 9 * mu + e, 36)];
}

// FP64 / FP32 / FP16 link copies keep the first two rows of each link (6 of 9 entries):
// entry (parity p, site j, component c = 6 mu + e) of the FP64 and FP16 copies is at
// p*24*Vhp + tiled(j, c, 24). The FP32 copy stores the entries of a tile row in pairs
// (2k, 2k + 1) of one link, one 16-byte word per lane:
//   p*24*Vhp + (j / 64)*24*64 + (c - c % 2)*64 + 2*(j % 64) + c % 2,
// so that a link is three 16-byte loads per work-item. The FP16 copy stores the six
// entries of a link of a tile row as a quad (e = 0..3, one 16-byte word per lane) and a
// pair (e = 4, 5, 8 bytes per lane):
//   p*24*Vhp + (j / 64)*24*64 + 6 mu*64 + (e < 4 ? 4*(j % 64) + e : 256 + 2*(j % 64) + e - 4),
// two loads per link. The LDS-staged FP16 hop, with one rhs per work-item, reads a
// three-row copy instead, so that it does not rebuild the third row for every term: after
// the two-row copy (at U16 + 48*Vhp) it holds all nine entries of a link of a tile row as
// two quads (e = 0..3, 4..7) and a single entry,
//   p*36*Vhp + (j / 64)*36*64 + 9 mu*64 + (e < 4 ? 4*(j % 64) + e : e < 8 ? 256 + 4*(j % 64) + e - 4 : 512 + j % 64),
// each entry rounded from the FP64 link (the third row is not rebuilt from rounded rows).
// internal.h (write_link_copies) writes all copies of one link; this kernel runs it with
// one work-item per link (site j fastest).
__global__ void gauge_to_f32_kernel(long long Vhp, LinkCopies lc, const double2* U64) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 8 * Vhp) return;
  const long long j = k % Vhp, r = k / Vhp;
  const int mu = (int)(r % 4), p = (int)(r / 4);
  double2 e[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) e[c] = U64[p * 36 * Vhp + tiled(j, 9 * mu + c, 36)];
  write_link_copies(lc, Vhp, p, j, mu, e);
}

// FP16 spinor fields: components divided by the site norm (the largest component
// magnitude), in quads of components (sidx), norm in FP32 (rhs blocks of 26*Vhp
// four-byte entries)
__global__ void pack_spinor16_kernel(Geo g, __half2* out, const double2* in, int nrhs) {
  const long long V = 2 * g.Vh;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V * nrhs) return;
  const long long rhs = t / V, i = t - rhs * V;
  const Lex c = lex_coords(g, i);
  const int p = (c.x0 + c.x1 + c.x2 + c.x3) & 1;
  const long long j = i >> 1;
  __half2* blk = out + rhs * 26 * g.Vhp;
  const double2* src = in + (rhs * V + i) * 12;
  float m = 0.0f;
  for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf((float)src[k].x), fabsf((float)src[k].y)));
  const float inv = m > 0.0f ? 1.0f / m : 0.0f;
  for (int k = 0; k < 12; ++k)
    blk[p * 12 * g.Vhp + sidx<h16>(j, k)] = __floats2half2_rn((float)src[k].x * inv, (float)src[k].y * inv);
  ((float*)(blk + 24 * g.Vhp))[p * g.Vhp + j] = m;
}

__global__ void unpack_spinor16_kernel(Geo g, double2* out, const __half2* in, int nrhs) {
  const long long V = 2 * g.Vh;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V * nrhs) return;
  const long long rhs = t / V, i = t - rhs * V;
  const Lex c = lex_coords(g, i);
  const int p = (c.x0 + c.x1 + c.x2 + c.x3) & 1;
  const long long j = i >> 1;
  const __half2* blk = in + rhs * 26 * g.Vhp;
  const float m = ((const float*)(blk + 24 * g.Vhp))[p * g.Vhp + j];
  double2* o = out + (rhs * V + i) * 12;
  for (int k = 0; k < 12; ++k) {
    const float2 v = __half22float2(blk[p * 12 * g.Vhp + sidx<h16>(j, k)]);
    o[k] = make_double2((double)(v.x * m), (double)(v.y * m));
  }
}

__global__ void pack_momenta_kernel(Geo g, double* out, const double* in, int to_sap) {
  const long long V = 2 * g.Vh;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const Lex c = lex_coords(g, i);
  const int p = (c.x0 + c.x1 + c.x2 + c.x3) & 1;
  const long long j = i >> 1;
  for (int mu = 0; mu < 4; ++mu)
    for (int a = 0; a < 8; ++a) {
      long long ks = p * 32 * g.Vhp + tiled(j, 8 * mu + a, 32);
      long long kc = (i * 4 + mu) * 8 + a;
      if (to_sap) out[ks] = in[kc];
      else out[kc] = in[ks];
    }
}

static inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

template <class R>
void launch_pack_spinor(const Geo& g, typename vec2<R>::type* out, const double2* in, int nrhs,
                        hipStream_t s) {
  long long n = 2 * g.Vh * nrhs;
  hipLaunchKernelGGL(pack_spinor_kernel<R>, dim3(nblk(n, 256)), dim3(256), 0, s, g, out, in, nrhs);
}
template <class R>
void launch_unpack_spinor(const Geo& g, double2* out, const typename vec2<R>::type* in, int nrhs,
                          hipStream_t s) {
  long long n = 2 * g.Vh * nrhs;
  hipLaunchKernelGGL(unpack_spinor_kernel<R>, dim3(nblk(n, 256)), dim3(256), 0, s, g, out, in, nrhs);
}
template void launch_pack_spinor<double>(const Geo&, double2*, const double2*, int, hipStream_t);
template void launch_pack_spinor<float>(const Geo&, float2*, const double2*, int, hipStream_t);
template void launch_unpack_spinor<double>(const Geo&, double2*, const double2*, int, hipStream_t);
template void launch_unpack_spinor<float>(const Geo&, double2*, const float2*, int, hipStream_t);

void launch_pack_gauge(const Geo& g, double2* U64, float2* U32, const double2* in, hipStream_t s) {
  hipLaunchKernelGGL(pack_gauge_kernel, dim3(nblk(2 * g.Vh, 128)), dim3(128), 0, s, g, U64, U32, in);
}
void launch_unpack_gauge(const Geo& g, double2* out, const double2* U64, hipStream_t s) {
  hipLaunchKernelGGL(unpack_gauge_kernel, dim3(nblk(2 * g.Vh, 128)), dim3(128), 0, s, g, out, U64);
}
void launch_gauge_to_f32(const Geo& g, double2* U64c, float2* U32, __half2* U16, const double2* U64, hipStream_t s) {
  const long long n = 8LL * g.Vhp;   // links: 2 parities x Vhp sites x 4 directions
  hipLaunchKernelGGL(gauge_to_f32_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, g.Vhp, LinkCopies{U64c, U32, U16}, U64);
}
void launch_pack_spinor16(const Geo& g, __half2* out, const double2* in, int nrhs, hipStream_t s) {
  long long n = 2 * g.Vh * nrhs;
  hipLaunchKernelGGL(pack_spinor16_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, g, out, in, nrhs);
}
void launch_unpack_spinor16(const Geo& g, double2* out, const __half2* in, int nrhs, hipStream_t s) {
  long long n = 2 * g.Vh * nrhs;
  hipLaunchKernelGGL(unpack_spinor16_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, g, out, in, nrhs);
}
void launch_pack_momenta(const Geo& g, double* out, const double* in, hipStream_t s) {
  hipLaunchKernelGGL(pack_momenta_kernel, dim3(nblk(2 * g.Vh, 128)), dim3(128), 0, s, g, out, in, 1);
}
void launch_unpack_momenta(const Geo& g, double* out, const double* in, hipStream_t s) {
  hipLaunchKernelGGL(pack_momenta_kernel, dim3(nblk(2 * g.Vh, 128)), dim3(128), 0, s, g, out, in, 0);
}

}  // namespace sap
