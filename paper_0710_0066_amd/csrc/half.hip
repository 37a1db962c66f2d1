// FP16 storage: the Wilson hop on FP16 spinors (per-site FP32 norm) and FP16 links (Sec. 1,
// eq. 2; the same operator as dslash.hip). Each hop term runs on the stored halves
// (site_io.h, hop16_term: packed FP16 projection, v_dot2_f32_f16 products summed in FP32);
// the neighbour's norm scales the term in the FP32 reconstruction, and on store the
// output site's norm is recomputed as its largest component magnitude.
//
// Two work-item mappings: one (output site, rhs) per work-item with workgroups
// rhs-fastest and renumbered per XCD (SITE), and the x0-marching order of dslash.hip with
// NR = 1, 2 or 4 rhs per work-item sharing every link load (MARCH1/2/4; the walking and
// band maps, which exist for FP32/FP64 only, fall back to the marching order).
#include "internal.h"
#include "site_io.h"

namespace sap {

// all eight hops of output site j of parity p for the rhs r0 .. r0 + nr - 1 (nr <= NR):
// out = a x + b (g5_out) D (g5_in in), zero on unselected sites; each link is loaded once.
// G5I / G5O: A.g5_in / A.g5_out, as template arguments so that the signs are not selected
// per component at run time.
template <int NR, bool G5I, bool G5O>
__device__ __forceinline__ void hop16_site(const HopArgs<h16>& A, int p, long long j, int r0, int nr) {
  const Geo& g = A.g;
  const long long Vhp = g.Vhp;
  const Site s = decode(g, j, p);
  const bool sel = block_sel(s.x0, A.slb, A.block, A.colour);
  cx<float> acc[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[r][a][c] = {0.0f, 0.0f};
  if (sel) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
      for (int dir = 0; dir < 2; ++dir) {
        const bool on = dir == 0 ? !(A.lb && mu == 0 && (s.x0 % A.lb) == A.lb - 1)
                                 : !(A.lb && mu == 0 && (s.x0 % A.lb) == 0);
        if (!on) continue;
        const long long jn = nbr(g, s, j, mu, dir == 0 ? +1 : -1);
        unsigned e[9];
        if (dir == 0)
          load_link16_words(A.U + p * 24 * Vhp + (j >> 6) * (24 * TILE) + 6 * mu * TILE, (int)(j & (TILE - 1)), e);
        else
          load_link16_words(A.U + (1 - p) * 24 * Vhp + (jn >> 6) * (24 * TILE) + 6 * mu * TILE,
                            (int)(jn & (TILE - 1)), e);
        third_row16(e);
        const bool flip = mu == 0 && (dir == 0 ? s.x0 == g.L0 - 1 : s.x0 == 0);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r >= nr) continue;
          // the stored (norm-divided) components; the site norm goes into the
          // multiply-adds of the reconstruction
          const SiteR<h16> in = site_r(A.in, r0 + r, 1 - p, jn, Vhp);
          unsigned sw[12];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const u4v q = *(const u4v*)(in.b + 4 * k * TILE);
            sw[4 * k] = q.x; sw[4 * k + 1] = q.y; sw[4 * k + 2] = q.z; sw[4 * k + 3] = q.w;
          }
          const float w = flip ? -in.m : in.m;
          cx<float> uh[2][3];
          hop16_term<G5I>(mu, dir == 1, e, sw, uh);
          accum_recon_scaled<float>(mu, dir == 1, uh, w, acc[r]);
        }
      }
    }
  }
  const bool with_x = sel && A.x.ptr;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) continue;
    SiteR<h16> xr;
    if (with_x) xr = site_r(A.x, r0 + r, p, j, Vhp);
    SiteW<h16> ow = site_w(A.out, r0 + r, p, j, Vhp);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cx<float> hv = acc[r][a][c];
        if (G5O && a >= 2) hv = -hv;
        cx<float> v = A.b * hv;
        if (with_x) v = v + A.a * get(xr, 3 * a + c);
        put(ow, 3 * a + c, sel ? v : cx<float>{0.0f, 0.0f});
      }
    close(ow);
  }
}

template <bool FULL, bool G5I, bool G5O>
__global__ __launch_bounds__(256) void hop16_kernel(HopArgs<h16> A) {
  const long long nwg = gridDim.x;
  const long long w = xcd_logical_block(blockIdx.x, nwg);
  const int rhs = (int)(w % A.nrhs);
  const long long chunk = w / A.nrhs;
  int p;
  long long j;
  if (FULL) {
    p = threadIdx.x >> 7;
    j = chunk * 128 + (threadIdx.x & 127);
  } else {
    p = A.parity_out;
    j = chunk * 256 + threadIdx.x;
  }
  if (j >= A.g.Vh) return;
  hop16_site<1, G5I, G5O>(A, p, j, rhs, 1);
}

// x0-marching order (as hop_march_kernel in dslash.hip): the slice-local sites of each
// parity are cut into 8 contiguous pieces, one per XCD (workgroup id % 8), and each XCD
// walks its piece slice by slice in increasing x0 with the rhs groups of a chunk back to
// back. A workgroup is 128 sites of one parity, or 64 sites of each parity (full operator).
template <bool FULL, int NR, bool G5I, bool G5O>
__global__ __launch_bounds__(128) void hop16_march_kernel(HopArgs<h16> A, int nck) {
  const int xcd = blockIdx.x & 7;
  const long long l = blockIdx.x >> 3;
  const int ngroups = (A.nrhs + NR - 1) / NR;
  const long long per_slice = (long long)nck * ngroups;
  const int x0 = (int)(l / per_slice);
  const long long rem = l - x0 * per_slice;
  const int chunk = (int)(rem / ngroups);
  const int r0 = (int)(rem - (long long)chunk * ngroups) * NR;
  if (x0 >= A.g.L0) return;
  const int lo = (int)((long long)A.g.V3h * xcd / 8);
  const int hi = (int)((long long)A.g.V3h * (xcd + 1) / 8);
  int p, s;
  if (FULL) {
    p = threadIdx.x >> 6;
    s = lo + chunk * 64 + (threadIdx.x & 63);
  } else {
    p = A.parity_out;
    s = lo + chunk * 128 + threadIdx.x;
  }
  if (s >= hi) return;
  hop16_site<NR, G5I, G5O>(A, p, (long long)x0 * A.g.V3h + s, r0, min(NR, A.nrhs - r0));
}

template <int NR> static void launch_march16(const HopArgs<h16>& A, hipStream_t st) {
  const bool full = A.parity_out < 0;
  const int piece = (A.g.V3h + 7) / 8;
  const int per = full ? 64 : 128;
  const int nck = (piece + per - 1) / per;
  const long long groups = (A.nrhs + NR - 1) / NR;
  const dim3 grid((unsigned)(8LL * A.g.L0 * nck * groups)), blk(128);
#define SAP_M16(FULL, G5I, G5O) hipLaunchKernelGGL((hop16_march_kernel<FULL, NR, G5I, G5O>), grid, blk, 0, st, A, nck)
#define SAP_M16_G5(FULL)                                   \
  do {                                                     \
    if (A.g5_in && A.g5_out) SAP_M16(FULL, true, true);    \
    else if (A.g5_in) SAP_M16(FULL, true, false);          \
    else if (A.g5_out) SAP_M16(FULL, false, true);         \
    else SAP_M16(FULL, false, false);                      \
  } while (0)
  if (full) SAP_M16_G5(true);
  else SAP_M16_G5(false);
#undef SAP_M16_G5
#undef SAP_M16
}

template <> void launch_hop<h16>(const HopArgs<h16>& A, hipStream_t st) {
  switch (A.map) {
    case HOP_MAP_MARCH1:
    case HOP_MAP_WALK1:
    case HOP_MAP_BAND1:
    case HOP_MAP_SLAB1:
    case HOP_MAP_SLAB1W: launch_march16<1>(A, st); return;
    case HOP_MAP_SLABD:
      if (A.parity_out < 0) launch_march16<1>(A, st);
      else launch_slabd16(A, st);
      return;
    case HOP_MAP_MARCH2:
    case HOP_MAP_WALK2:
    case HOP_MAP_SLAB2: launch_march16<2>(A, st); return;
    case HOP_MAP_MARCH4: launch_march16<4>(A, st); return;
    default: break;
  }
  const bool full = A.parity_out < 0;
  const long long per = full ? 128 : 256;
  const long long chunks = (A.g.Vh + per - 1) / per;
  const long long n = chunks * A.nrhs;
  const dim3 grid((unsigned)((n + 7) / 8 * 8)), blk(256);
#define SAP_S16(FULL, G5I, G5O) hipLaunchKernelGGL((hop16_kernel<FULL, G5I, G5O>), grid, blk, 0, st, A)
#define SAP_S16_G5(FULL)                                   \
  do {                                                     \
    if (A.g5_in && A.g5_out) SAP_S16(FULL, true, true);    \
    else if (A.g5_in) SAP_S16(FULL, true, false);          \
    else if (A.g5_out) SAP_S16(FULL, false, true);         \
    else SAP_S16(FULL, false, false);                      \
  } while (0)
  if (full) SAP_S16_G5(true);
  else SAP_S16_G5(false);
#undef SAP_S16_G5
#undef SAP_S16
}

}  // namespace sap
