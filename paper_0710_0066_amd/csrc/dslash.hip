// Wilson hop stencil for gfx950 (Sec. 1, eq. 2):
//   (D psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
// with the antiperiodic x0 wrap, optional removal of the hops between x0 blocks of
// length lb (the block operator W of the one-dimensional Schwarz decomposition), and
//   out = a * x + b * D(in)
// on both parities (M = 1 - kappa D) or on one parity (the even-odd half hops).
//
// Bandwidth-bound 8-point gather: one work-item per (output site, rhs), tiled
// structure-of-arrays complex loads that coalesce across the 64-lane wavefront,
// half-spinor projection before the SU(3) product (2 colour vectors per link instead of
// 4), FP64 or FP32 arithmetic matching the storage. Workgroups are numbered rhs-fastest
// and renumbered per XCD; with several rhs four of them share each link load.
#include "internal.h"

namespace sap {

template <class R>
__device__ __forceinline__ void load_spinor(const typename vec2<R>::type* p, long long j, bool g5,
                                            cx<R> s[4][3]) {
  const typename vec2<R>::type* q = p + tiled(j, 0, 12);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<R> v = ld<R>(q + (sp * 3 + c) * TILE);
      s[sp][c] = (g5 && sp >= 2) ? -v : v;
    }
}

template <class R>
__device__ __forceinline__ void load_link(const typename vec2<R>::type* U, long long Vhp, int mu,
                                          int par, long long j, cx<R> m[9]) {
  const typename vec2<R>::type* p = U + par * 36 * Vhp + tiled(j, 9 * mu, 36);
#pragma unroll
  for (int e = 0; e < 9; ++e) m[e] = ld<R>(p + e * TILE);
}

// Work-item mappings (MAP):
//  SITE  one work-item per (site, rhs); a workgroup holds 256 sites of one parity (half
//        hop) or 128 sites of each parity (full operator), workgroups rhs-fastest.
//  LANE4 a wavefront holds 16 sites x 4 rhs: the four lanes of a site read the same link
//        address in the same load instruction, so the link is fetched once for 4 rhs; a
//        workgroup holds 64 sites (half hop) or 32 sites of each parity (full).
//  WAVE4 a workgroup holds 64 sites (half hop; full: 32 sites of each parity) x 4 rhs with
//        one rhs per wavefront: the wavefronts of a workgroup load the same links back to
//        back through the CU's L1, and each keeps 64 consecutive sites for neighbour reuse.
template <class R, bool FULL, int MAP>
__global__ __launch_bounds__(256) void hop_kernel(HopArgs<R> A) {
  typedef typename vec2<R>::type V2;
  const long long nwg = gridDim.x;
  const long long w = xcd_logical_block(blockIdx.x, nwg);
  int p, rhs;
  long long j;
  if (MAP == HOP_MAP_SITE) {
    rhs = (int)(w % A.nrhs);
    const long long chunk = w / A.nrhs;
    if (FULL) {
      p = threadIdx.x >> 7;
      j = chunk * 128 + (threadIdx.x & 127);
    } else {
      p = A.parity_out;
      j = chunk * 256 + threadIdx.x;
    }
  } else if (MAP == HOP_MAP_LANE4) {
    const int ngroups = (A.nrhs + 3) >> 2;
    const long long chunk = w / ngroups;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    rhs = (int)(w % ngroups) * 4 + (lane >> 4);
    if (rhs >= A.nrhs) return;
    if (FULL) {
      p = wave >> 1;
      j = chunk * 32 + (wave & 1) * 16 + (lane & 15);
    } else {
      p = A.parity_out;
      j = chunk * 64 + wave * 16 + (lane & 15);
    }
  } else {
    const int ngroups = (A.nrhs + 3) >> 2;
    const long long chunk = w / ngroups;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    rhs = (int)(w % ngroups) * 4 + wave;
    if (rhs >= A.nrhs) return;
    if (FULL) {
      p = lane >> 5;
      j = chunk * 32 + (lane & 31);
    } else {
      p = A.parity_out;
      j = chunk * 64 + lane;
    }
  }
  const Geo& g = A.g;
  if (j >= g.Vh) return;
  const long long Vhp = g.Vhp;
  const Site s = decode(g, j, p);

  V2* o = A.out.ptr + rhs * A.out.rs + p * A.out.ps + tiled(j, 0, 12);
  if (A.slb) {
    const int blk = s.x0 / A.slb;
    bool sel;
    if (A.block >= 0) sel = (blk == A.block);
    else sel = (A.colour == 0) || ((A.colour == 1) == ((blk & 1) == 1));
    if (!sel) {
      cx<R> z = {R(0), R(0)};
#pragma unroll
      for (int c = 0; c < 12; ++c) st<R>(o + c * TILE, z);
      return;
    }
  }

  cx<R> acc[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[sp][c] = {R(0), R(0)};

  const V2* inb = A.in.ptr + rhs * A.in.rs + (1 - p) * A.in.ps;
  const bool g5i = A.g5_in != 0;

#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    // forward hop: (1 - gamma_mu) U_mu(x) psi(x + mu)
    const bool fwd_on = !(A.lb && mu == 0 && (s.x0 % A.lb) == A.lb - 1);
    if (fwd_on) {
      const long long jn = nbr(g, s, j, mu, +1);
      cx<R> sp[4][3], h[2][3], uh[2][3], m[9];
      load_spinor<R>(inb, jn, g5i, sp);
      project<R>(mu, false, sp, h);
      load_link<R>(A.U, Vhp, mu, p, j, m);
      su3_mul<R>(m, h[0], uh[0]);
      su3_mul<R>(m, h[1], uh[1]);
      if (mu == 0 && s.x0 == g.L0 - 1) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
      }
      accum_recon<R>(mu, false, uh, acc);
    }
    // backward hop: (1 + gamma_mu) U_mu(x - mu)^+ psi(x - mu)
    const bool bwd_on = !(A.lb && mu == 0 && (s.x0 % A.lb) == 0);
    if (bwd_on) {
      const long long jn = nbr(g, s, j, mu, -1);
      cx<R> sp[4][3], h[2][3], uh[2][3], m[9];
      load_spinor<R>(inb, jn, g5i, sp);
      project<R>(mu, true, sp, h);
      load_link<R>(A.U, Vhp, mu, 1 - p, jn, m);
      su3_dag_mul<R>(m, h[0], uh[0]);
      su3_dag_mul<R>(m, h[1], uh[1]);
      if (mu == 0 && s.x0 == 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
      }
      accum_recon<R>(mu, true, uh, acc);
    }
  }

  if (A.g5_out) {
#pragma unroll
    for (int sp = 2; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[sp][c] = -acc[sp][c];
  }
  if (A.x.ptr) {
    const V2* xp = A.x.ptr + rhs * A.x.rs + p * A.x.ps + tiled(j, 0, 12);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cx<R> xv = ld<R>(xp + (sp * 3 + c) * TILE);
        cx<R> r = {A.a * xv.r + A.b * acc[sp][c].r, A.a * xv.i + A.b * acc[sp][c].i};
        st<R>(o + (sp * 3 + c) * TILE, r);
      }
  } else {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) st<R>(o + (sp * 3 + c) * TILE, A.b * acc[sp][c]);
  }
}

static inline long long round8(long long n) { return (n + 7) / 8 * 8; }

template <class R> void launch_hop(const HopArgs<R>& A, hipStream_t st) {
  const bool full = A.parity_out < 0;
  const int map = A.nrhs > 1 ? A.map : HOP_MAP_SITE;
  const bool grouped = map != HOP_MAP_SITE;
  const long long per = grouped ? (full ? 32 : 64) : (full ? 128 : 256);
  const long long groups = grouped ? (A.nrhs + 3) / 4 : A.nrhs;
  const long long chunks = (A.g.Vh + per - 1) / per;
  const dim3 grid((unsigned)round8(chunks * groups)), blk(256);
  if (full) {
    if (map == HOP_MAP_LANE4) hipLaunchKernelGGL((hop_kernel<R, true, HOP_MAP_LANE4>), grid, blk, 0, st, A);
    else if (map == HOP_MAP_WAVE4) hipLaunchKernelGGL((hop_kernel<R, true, HOP_MAP_WAVE4>), grid, blk, 0, st, A);
    else hipLaunchKernelGGL((hop_kernel<R, true, HOP_MAP_SITE>), grid, blk, 0, st, A);
  } else {
    if (map == HOP_MAP_LANE4) hipLaunchKernelGGL((hop_kernel<R, false, HOP_MAP_LANE4>), grid, blk, 0, st, A);
    else if (map == HOP_MAP_WAVE4) hipLaunchKernelGGL((hop_kernel<R, false, HOP_MAP_WAVE4>), grid, blk, 0, st, A);
    else hipLaunchKernelGGL((hop_kernel<R, false, HOP_MAP_SITE>), grid, blk, 0, st, A);
  }
}

template void launch_hop<double>(const HopArgs<double>&, hipStream_t);
template void launch_hop<float>(const HopArgs<float>&, hipStream_t);

}  // namespace sap
