// FP16 storage: the Wilson hop on FP16 spinors (per-site FP32 norm) and FP16 links with
// FP32 arithmetic (Sec. 1, eq. 2; the same operator as dslash.hip), one work-item per
// (output site, rhs) with workgroups rhs-fastest and renumbered per XCD. Loads and stores
// are per site: a site's 12 components are scaled by its norm on load, and on store the
// norm is recomputed as the largest component magnitude.
#include "internal.h"
#include "site_io.h"

namespace sap {

__device__ __forceinline__ void load_link16(const __half2* U, long long Vhp, int mu, int par, long long j,
                                            cx<float> m[9]) {
  const __half2* p = U + par * 36 * Vhp + tiled(j, 9 * mu, 36);
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const float2 v = __half22float2(p[e * TILE]);
    m[e] = {v.x, v.y};
  }
}

template <bool FULL>
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
  const Geo& g = A.g;
  if (j >= g.Vh) return;
  const long long Vhp = g.Vhp;
  const Site s = decode(g, j, p);
  const bool sel = block_sel(s.x0, A.slb, A.block, A.colour);
  cx<float> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[a][c] = {0.0f, 0.0f};
  if (sel) {
    const bool g5i = A.g5_in != 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
      for (int dir = 0; dir < 2; ++dir) {
        const bool on = dir == 0 ? !(A.lb && mu == 0 && (s.x0 % A.lb) == A.lb - 1)
                                 : !(A.lb && mu == 0 && (s.x0 % A.lb) == 0);
        if (!on) continue;
        const long long jn = nbr(g, s, j, mu, dir == 0 ? +1 : -1);
        cx<float> sp[4][3], h[2][3], uh[2][3], m[9];
        {
          const SiteR<h16> r = site_r(A.in, rhs, 1 - p, jn, Vhp);
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const cx<float> v = get(r, 3 * a + c);
              sp[a][c] = (g5i && a >= 2) ? -v : v;
            }
        }
        project<float>(mu, dir == 1, sp, h);
        if (dir == 0) {
          load_link16(A.U, Vhp, mu, p, j, m);
          su3_mul<float>(m, h[0], uh[0]);
          su3_mul<float>(m, h[1], uh[1]);
        } else {
          load_link16(A.U, Vhp, mu, 1 - p, jn, m);
          su3_dag_mul<float>(m, h[0], uh[0]);
          su3_dag_mul<float>(m, h[1], uh[1]);
        }
        if (mu == 0 && (dir == 0 ? s.x0 == g.L0 - 1 : s.x0 == 0))
#pragma unroll
          for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
        accum_recon<float>(mu, dir == 1, uh, acc);
      }
    }
  }
  const bool with_x = sel && A.x.ptr;
  SiteR<h16> xr;
  if (with_x) xr = site_r(A.x, rhs, p, j, Vhp);
  SiteW<h16> ow = site_w(A.out, rhs, p, j, Vhp);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<float> hv = acc[a][c];
      if (A.g5_out && a >= 2) hv = -hv;
      cx<float> r = A.b * hv;
      if (with_x) r = r + A.a * get(xr, 3 * a + c);
      put(ow, 3 * a + c, sel ? r : cx<float>{0.0f, 0.0f});
    }
  close(ow);
}

template <> void launch_hop<h16>(const HopArgs<h16>& A, hipStream_t st) {
  const bool full = A.parity_out < 0;
  const long long per = full ? 128 : 256;
  const long long chunks = (A.g.Vh + per - 1) / per;
  const long long n = chunks * A.nrhs;
  const dim3 grid((unsigned)((n + 7) / 8 * 8)), blk(256);
  if (full) hipLaunchKernelGGL(hop16_kernel<true>, grid, blk, 0, st, A);
  else hipLaunchKernelGGL(hop16_kernel<false>, grid, blk, 0, st, A);
}

}  // namespace sap
