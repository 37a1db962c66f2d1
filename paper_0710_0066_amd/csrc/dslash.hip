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
#include "site_io.h"

namespace sap {

template <class R>
__device__ __forceinline__ void load_spinor(const typename vec2<R>::type* p, long long j, bool g5,
                                            cx<R> s[4][3]) {
  cx<R> v[12];
  ld_site<R>(p, j, v);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[sp][c] = (g5 && sp >= 2) ? -v[sp * 3 + c] : v[sp * 3 + c];
}

// out site j of the (rhs, parity) block ob: a x + b (gamma_5 if g5o) acc, or zero when the
// site is not selected; xb: the same block of x, or null (NT: non-temporal stores)
template <class R, bool NT>
__device__ __forceinline__ void store_out(typename vec2<R>::type* ob, const typename vec2<R>::type* xb, long long j,
                                          bool sel, bool g5o, R a, R b, const cx<R> acc[4][3],
                                          double* n2 = nullptr) {
  cx<R> v[12], xv[12];
  if (sel && xb) ld_site<R>(xb, j, xv);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = sp * 3 + c;
      cx<R> h = acc[sp][c];
      if (g5o && sp >= 2) h = -h;
      cx<R> r = {b * h.r, b * h.i};
      if (xb) {
        r.r += a * xv[k].r;
        r.i += a * xv[k].i;
      }
      v[k] = sel ? r : cx<R>{R(0), R(0)};
      if (n2) *n2 += (double)v[k].r * v[k].r + (double)v[k].i * v[k].i;
    }
  st_site<R, NT>(ob, j, v);
}

// store_out with reductions of the stored values v (red[0..2], see HopArgs::red): RED 1
// ||v||^2; RED 3 <v, x> and ||v||^2. The 12 components of the site are summed at the
// arithmetic precision and the site sums added in FP64.
template <class R, bool NT, int RED>
__device__ __forceinline__ void store_out_red(typename vec2<R>::type* ob, const typename vec2<R>::type* xb,
                                              long long j, bool sel, bool g5o, R a, R b, const cx<R> acc[4][3],
                                              double red[3]) {
  cx<R> v[12], xv[12];
  R s0 = R(0), s1 = R(0), s2 = R(0);
  if (sel && xb) ld_site<R>(xb, j, xv);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = sp * 3 + c;
      cx<R> h = acc[sp][c];
      if (g5o && sp >= 2) h = -h;
      cx<R> r = {b * h.r, b * h.i};
      if (xb) {
        r.r += a * xv[k].r;
        r.i += a * xv[k].i;
      }
      v[k] = sel ? r : cx<R>{R(0), R(0)};
      if (RED == 1 || RED == 3) s2 += v[k].r * v[k].r + v[k].i * v[k].i;
      if (RED == 3 && sel && xb) {
        s0 += v[k].r * xv[k].r + v[k].i * xv[k].i;
        s1 += v[k].r * xv[k].i - v[k].i * xv[k].r;
      }
    }
  if (RED == 1) red[0] += (double)s2;
  if (RED == 3) {
    red[0] += (double)s0;
    red[1] += (double)s1;
    red[2] += (double)s2;
  }
  st_site<R, NT>(ob, j, v);
}

// The hop kernels read two-row link copies (FP64 or FP32) and rebuild the third row from
// unitarity and unit determinant: row 3 = conj(row 1 x row 2). o24 is the offset of the
// site's tile row, tiled(j, 0, 24) with the lane j % 64. FP64 entries are 16 bytes each
// (entry e of link mu at o24 + (6 mu + e) * 64). The FP32 copy holds the six entries of a
// link as three pairs, each pair one 16-byte word per lane: pair k = (2k, 2k + 1) of link mu
// at float2 offset  tile * 24 * 64 + (6 mu + 2k) * 64 + 2 lane  (+1 for the odd entry),
// so that a link takes three 16-byte loads.
template <class R>
__device__ __forceinline__ void load_link_at(const typename vec2<R>::type* U, long long Vhp, int mu, int par,
                                             long long o24, cx<R> m[9]) {
  if constexpr (std::is_same<R, float>::value) {
    const long long lane = o24 & (TILE - 1);
    const float4* p = (const float4*)(U + par * 24 * Vhp + (o24 - lane) + 6 * mu * TILE) + lane;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 v = p[k * TILE];
      m[2 * k] = {v.x, v.y};
      m[2 * k + 1] = {v.z, v.w};
    }
  } else {
    const typename vec2<R>::type* p = U + par * 24 * Vhp + o24 + 6 * mu * TILE;
#pragma unroll
    for (int e = 0; e < 6; ++e) m[e] = ld<R>(p + e * TILE);
  }
  third_row<R>(m);
}
template <class R>
__device__ __forceinline__ void load_link(const typename vec2<R>::type* U, long long Vhp, int mu,
                                          int par, long long j, cx<R> m[9]) {
  load_link_at<R>(U, Vhp, mu, par, tiled(j, 0, 24), m);
}
// the two stored rows only (entries 0..5), for kernels that load a link ahead of its use
template <class R>
__device__ __forceinline__ void load_link_raw(const typename vec2<R>::type* U, long long Vhp, int mu, int par,
                                              long long o24, cx<R> m[6]) {
  if constexpr (std::is_same<R, float>::value) {
    const long long lane = o24 & (TILE - 1);
    const float4* p = (const float4*)(U + par * 24 * Vhp + (o24 - lane) + 6 * mu * TILE) + lane;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 v = p[k * TILE];
      m[2 * k] = {v.x, v.y};
      m[2 * k + 1] = {v.z, v.w};
    }
  } else {
    const typename vec2<R>::type* p = U + par * 24 * Vhp + o24 + 6 * mu * TILE;
#pragma unroll
    for (int e = 0; e < 6; ++e) m[e] = ld<R>(p + e * TILE);
  }
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
template <class R, bool FULL, int MAP, bool SWEEP>
__global__ __launch_bounds__(256) void hop_kernel(HopArgs<R> A, long long nchunk) {
  typedef typename vec2<R>::type V2;
  const long long nwg = gridDim.x;
  const long long w = xcd_logical_block(blockIdx.x, nwg);
  int p, rhs;
  long long j;
  if (MAP == HOP_MAP_SITE) {
    rhs = SWEEP ? (int)(w / nchunk) : (int)(w % A.nrhs);
    const long long chunk = SWEEP ? w % nchunk : w / A.nrhs;
    if (rhs >= A.nrhs) return;
    if (FULL) {
      p = threadIdx.x >> 7;
      j = chunk * 128 + (threadIdx.x & 127);
    } else {
      p = A.parity_out;
      j = chunk * 256 + threadIdx.x;
    }
  } else if (MAP == HOP_MAP_LANE4) {
    const int ngroups = (A.nrhs + 3) >> 2;
    const long long chunk = SWEEP ? w % nchunk : w / ngroups;
    const int group = SWEEP ? (int)(w / nchunk) : (int)(w % ngroups);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    rhs = group * 4 + (lane >> 4);
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
    const long long chunk = SWEEP ? w % nchunk : w / ngroups;
    const int group = SWEEP ? (int)(w / nchunk) : (int)(w % ngroups);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    rhs = group * 4 + wave;
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

  V2* o = A.out.ptr + rhs * A.out.rs + p * A.out.ps;
  const V2* xo = A.x.ptr ? A.x.ptr + rhs * A.x.rs + p * A.x.ps : nullptr;
  if (A.slb) {
    const int blk = s.x0 / A.slb;
    bool sel;
    if (A.block >= 0) sel = (blk == A.block);
    else sel = (A.colour == 0) || ((A.colour == 1) == ((blk & 1) == 1));
    if (!sel) {
      const cx<R> z[4][3] = {};
      store_out<R, false>(o, nullptr, j, false, false, R(0), R(0), z);
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

  store_out<R, false>(o, xo, j, true, A.g5_out != 0, A.a, A.b, acc);
}

// x0-streaming even-odd hop (output parity p, input parity q = 1 - p). A workgroup owns
// S consecutive slice-local sites s (site j = x0*V3h + s of its parity) for one rhs and
// walks a chunk of x0 slices. The time neighbours of output (x0, s) are the inputs
// (x0 +/- 1, s) with the same s, so each input is loaded once per chunk: its (1 + g0)
// projection is carried in registers for the backward hop two slices later, and the
// whole input slice is staged in LDS (double buffered), from where the spatial
// neighbours inside [s0, s0 + S) are read; only neighbours outside the range are loaded
// from memory. Links are used once per half hop and are read directly.
template <class R, int S>
__global__ __launch_bounds__(S) void hop_stream_kernel(HopArgs<R> A, int T, int nrange, int nchunk) {
  typedef typename vec2<R>::type V2;
  extern __shared__ char smem_raw[];
  V2* plane = (V2*)smem_raw;                       // [2 buffers][12 components][S]
  const Geo& g = A.g;
  const long long nwg = gridDim.x;
  const long long w = xcd_logical_block(blockIdx.x, nwg);
  const int rhs = (int)(w % A.nrhs);
  const long long rest = w / A.nrhs;
  const int range = (int)(rest % nrange);
  const int chunk = (int)(rest / nrange);
  if (chunk >= nchunk) return;                     // whole workgroup: padding of the grid
  const int p = A.parity_out, q = 1 - p;
  const int t = threadIdx.x;
  const int s0 = range * S;
  const int s = s0 + t;
  const bool active = s < g.V3h;
  const int x0a = chunk * T;
  const int x0b = min(x0a + T, g.L0);
  const long long Vhp = g.Vhp;
  const V2* inb = A.in.ptr + rhs * A.in.rs + q * A.in.ps;
  const bool g5i = A.g5_in != 0;
  const int lb = A.lb;

  auto ldsp = [&](int buf, int tt, cx<R> sp[4][3]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cx<R> v = ld<R>(plane + ((buf * 12) + a * 3 + c) * S + tt);
        sp[a][c] = (g5i && a >= 2) ? -v : v;
      }
  };
  auto put = [&](int buf, const cx<R> sp[4][3]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) st<R>(plane + ((buf * 12) + a * 3 + c) * S + t, sp[a][c]);
  };
  auto slice_j = [&](int x0) { return (long long)x0 * g.V3h + s; };
  auto wrap = [&](int x0) { return x0 < 0 ? x0 + g.L0 : (x0 >= g.L0 ? x0 - g.L0 : x0); };

  // carried (1 + g0) projections of the inputs on the two previous slices
  cx<R> carry[2][2][3];
  cx<R> sp[4][3];
  if (active) {
    const bool need_prev = !(lb && (x0a % lb) == 0);
    if (need_prev) {
      load_spinor<R>(inb, slice_j(wrap(x0a - 1)), g5i, sp);
      project<R>(0, true, sp, carry[(x0a - 1) & 1]);
    }
    load_spinor<R>(inb, slice_j(x0a), false, sp);      // raw copy to LDS, g5 applied on read
    put(x0a & 1, sp);
    if (g5i)
#pragma unroll
      for (int c = 0; c < 3; ++c) { sp[2][c] = -sp[2][c]; sp[3][c] = -sp[3][c]; }
    project<R>(0, true, sp, carry[x0a & 1]);
  }
  __syncthreads();

  for (int x0 = x0a; x0 < x0b; ++x0) {
    const int buf = x0 & 1;
    if (active) {
      const long long j = slice_j(x0);
      const Site st_ = decode(g, j, p);
      V2* o = A.out.ptr + rhs * A.out.rs + p * A.out.ps;
      bool sel = true;
      if (A.slb) {
        const int blk = x0 / A.slb;
        sel = A.block >= 0 ? (blk == A.block) : ((A.colour == 0) || ((A.colour == 1) == ((blk & 1) == 1)));
      }
      // next input slice: time-forward neighbour, staged for the next step
      cx<R> nx[4][3];
      const bool fwd_on = !(lb && (x0 % lb) == lb - 1);
      if (fwd_on || x0 + 1 < x0b) {
        load_spinor<R>(inb, slice_j(wrap(x0 + 1)), false, nx);
      } else {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) nx[a][c] = {R(0), R(0)};
      }
      if (x0 + 1 < x0b) put(buf ^ 1, nx);
      if (g5i)
#pragma unroll
        for (int c = 0; c < 3; ++c) { nx[2][c] = -nx[2][c]; nx[3][c] = -nx[3][c]; }
      if (!sel) {
        const cx<R> z[4][3] = {};
        store_out<R, false>(o, nullptr, j, false, false, R(0), R(0), z);
      } else {
        cx<R> acc[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[a][c] = {R(0), R(0)};
        // spatial directions: neighbours from LDS when inside this workgroup's range
#pragma unroll
        for (int mu = 1; mu < 4; ++mu) {
#pragma unroll
          for (int dir = 0; dir < 2; ++dir) {
            const long long jn = nbr(g, st_, j, mu, dir == 0 ? +1 : -1);
            const int sn = (int)(jn - (long long)x0 * g.V3h);
            cx<R> nb[4][3], h[2][3], uh[2][3], m[9];
            if (sn >= s0 && sn < s0 + S) ldsp(buf, sn - s0, nb);
            else load_spinor<R>(inb, jn, g5i, nb);
            project<R>(mu, dir == 1, nb, h);
            if (dir == 0) {
              load_link<R>(A.U, Vhp, mu, p, j, m);
              su3_mul<R>(m, h[0], uh[0]);
              su3_mul<R>(m, h[1], uh[1]);
            } else {
              load_link<R>(A.U, Vhp, mu, q, jn, m);
              su3_dag_mul<R>(m, h[0], uh[0]);
              su3_dag_mul<R>(m, h[1], uh[1]);
            }
            accum_recon<R>(mu, dir == 1, uh, acc);
          }
        }
        // time forward: (1 - g0) U_0(x) in(x + 0)
        if (fwd_on) {
          cx<R> h[2][3], uh[2][3], m[9];
          project<R>(0, false, nx, h);
          load_link<R>(A.U, Vhp, 0, p, j, m);
          su3_mul<R>(m, h[0], uh[0]);
          su3_mul<R>(m, h[1], uh[1]);
          if (x0 == g.L0 - 1)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
              for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
          accum_recon<R>(0, false, uh, acc);
        }
        // time backward: (1 + g0) U_0(x - 0)^+ in(x - 0), projection carried
        if (!(lb && (x0 % lb) == 0)) {
          cx<R> uh[2][3], m[9];
          load_link<R>(A.U, Vhp, 0, q, slice_j(wrap(x0 - 1)), m);
          su3_dag_mul<R>(m, carry[(x0 - 1) & 1][0], uh[0]);
          su3_dag_mul<R>(m, carry[(x0 - 1) & 1][1], uh[1]);
          if (x0 == 0)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
              for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
          accum_recon<R>(0, true, uh, acc);
        }
        const V2* xo = A.x.ptr ? A.x.ptr + rhs * A.x.rs + p * A.x.ps : nullptr;
        store_out<R, false>(o, xo, j, true, A.g5_out != 0, A.a, A.b, acc);
      }
      // the input of this step's forward hop is the backward input two steps later
      project<R>(0, true, nx, carry[(x0 + 1) & 1]);
    }
    __syncthreads();
  }
}

// Pieces of the register-blocked hop on one output site j of parity p for the right-hand
// sides r0 .. r0 + nr - 1 (nr <= NR): each loaded link is applied to the nr input spinors.

// is the output site in a selected x0 block (always true without a block restriction)?
template <class R>
__device__ __forceinline__ bool hop_selected(const HopArgs<R>& A, int x0) {
  if (!A.slb) return true;
  const int blk = x0 / A.slb;
  if (A.block >= 0) return blk == A.block;
  return (A.colour == 0) || ((A.colour == 1) == ((blk & 1) == 1));
}

// acc[r] += the hops of direction mu (dir 0 forward, 1 backward), if present
template <class R, int NR>
__device__ __forceinline__ void hop_dir(const HopArgs<R>& A, int p, long long j, const Site& s, int mu, int dir,
                                        int r0, int nr, cx<R> acc[NR][4][3]) {
  typedef typename vec2<R>::type V2;
  const Geo& g = A.g;
  const bool on = dir == 0 ? !(A.lb && mu == 0 && (s.x0 % A.lb) == A.lb - 1)
                           : !(A.lb && mu == 0 && (s.x0 % A.lb) == 0);
  if (!on) return;
  const V2* inb = A.in.ptr + (1 - p) * A.in.ps;
  const bool g5i = A.g5_in != 0;
  const long long jn = nbr(g, s, j, mu, dir == 0 ? +1 : -1);
  cx<R> m[9];
  if (dir == 0) load_link<R>(A.U, g.Vhp, mu, p, j, m);
  else load_link<R>(A.U, g.Vhp, mu, 1 - p, jn, m);
  const bool flip = mu == 0 && (dir == 0 ? s.x0 == g.L0 - 1 : s.x0 == 0);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nr) {
      cx<R> sp[4][3], h[2][3], uh[2][3];
      load_spinor<R>(inb + (r0 + r) * A.in.rs, jn, g5i, sp);
      project<R>(mu, dir == 1, sp, h);
      if (dir == 0) {
        su3_mul<R>(m, h[0], uh[0]);
        su3_mul<R>(m, h[1], uh[1]);
      } else {
        su3_dag_mul<R>(m, h[0], uh[0]);
        su3_dag_mul<R>(m, h[1], uh[1]);
      }
      if (flip)
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
      accum_recon<R>(mu, dir == 1, uh, acc[r]);
    }
  }
}

template <class R> __device__ __forceinline__ void st_nt(typename vec2<R>::type* p, cx<R> a) {
  __builtin_nontemporal_store(a.r, &p->x);
  __builtin_nontemporal_store(a.i, &p->y);
}

// out = a x + b (g5_out) acc, or zero for an unselected site; NT: non-temporal stores
// (the result is not read again by this launch)
template <class R, int NR, bool NT>
__device__ __forceinline__ void hop_store(const HopArgs<R>& A, int p, long long j, int r0, int nr, bool sel,
                                          cx<R> acc[NR][4][3]) {
  typedef typename vec2<R>::type V2;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) continue;
    V2* o = A.out.ptr + (r0 + r) * A.out.rs + p * A.out.ps;
    const V2* xo = A.x.ptr ? A.x.ptr + (r0 + r) * A.x.rs + p * A.x.ps : nullptr;
    store_out<R, NT>(o, xo, j, sel, A.g5_out != 0, A.a, A.b, acc[r]);
  }
}

// all eight hops of output site j (NT: non-temporal output stores)
template <class R, int NR, bool NT = false>
__device__ __forceinline__ void hop_site_rhs(const HopArgs<R>& A, int p, long long j, int r0, int nr) {
  const Site s = decode(A.g, j, p);
  const bool sel = hop_selected(A, s.x0);
  cx<R> acc[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[r][a][c] = {R(0), R(0)};
  if (sel) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      hop_dir<R, NR>(A, p, j, s, mu, 0, r0, nr, acc);
      hop_dir<R, NR>(A, p, j, s, mu, 1, r0, nr, acc);
    }
  }
  hop_store<R, NR, NT>(A, p, j, r0, nr, sel, acc);
}

// Register-blocked kernel, chunk order: a workgroup holds 256 consecutive sites of one
// parity (128 of each for the full operator) for one group of NR rhs; workgroups are
// ordered group-fastest (SWEEP: group-slowest, each group sweeps the lattice like a
// small-rhs launch) and renumbered per XCD.
template <class R, bool FULL, int NR, bool SWEEP>
__global__ __launch_bounds__(256) void hop_reg_kernel(HopArgs<R> A, long long nchunk) {
  const long long nwg = gridDim.x;
  const long long w = xcd_logical_block(blockIdx.x, nwg);
  const int ngroups = (A.nrhs + NR - 1) / NR;
  const int r0 = (SWEEP ? (int)(w / nchunk) : (int)(w % ngroups)) * NR;
  const long long chunk = SWEEP ? w % nchunk : w / ngroups;
  if (r0 >= A.nrhs) return;
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
  hop_site_rhs<R, NR>(A, p, j, r0, min(NR, A.nrhs - r0));
}

// x0-marching order. The slice-local sites s in [0, V3h) of each parity (site j =
// x0*V3h + s) are cut into 8 contiguous pieces, one per XCD (the hardware deals
// workgroup ids round-robin to the 8 XCDs, so id % 8 names the XCD); each XCD walks its
// piece slice by slice in increasing x0, with all rhs groups of a chunk back to back.
// The time neighbours of a slice then lie 1/8 of a slice of every rhs behind or ahead in
// that XCD's stream and are still in its L2, links are shared by the rhs groups through
// L2, and only spatial neighbours across piece boundaries are fetched by two XCDs. A
// workgroup is 128 sites of one parity, or 64 sites of each parity for the full operator.
template <class R, bool FULL, int NR>
__global__ __launch_bounds__(128) void hop_march_kernel(HopArgs<R> A, int nck) {
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
  hop_site_rhs<R, NR, true>(A, p, (long long)x0 * A.g.V3h + s, r0, min(NR, A.nrhs - r0));
}

// x0-walking even-odd hop. A work-item owns the slice-local site s (j = x0*V3h + s) of the
// output parity for a group of NR rhs and walks the T slices x0a .. x0b - 1. The time
// neighbours of output (x0, s) are the inputs (x0 +/- 1, s) with the same s (a step in x0
// flips the parity and keeps the x3 bit), so each input is loaded once per walk for the
// time hops: its (1 - g0) projection serves the forward hop of output x0 - 1 at once, and
// its (1 + g0) projection is carried in registers to the backward hop of output x0 + 1
// two steps later. Spatial hops read memory. The slice-local range is cut into 8 pieces,
// one per XCD (workgroup id % 8), and the walks of an XCD run side by side, so spatial
// neighbours are read by concurrently running workgroups of the same XCD; the result is
// stored non-temporally. A workgroup is 128 consecutive slice-local sites.
template <class R, int NR>
__global__ __launch_bounds__(128) void hop_walk_kernel(HopArgs<R> A, int nck, int T) {
  typedef typename vec2<R>::type V2;
  const int xcd = blockIdx.x & 7;
  const long long l = blockIdx.x >> 3;
  const int ngroups = (A.nrhs + NR - 1) / NR;
  const long long per_walk = (long long)nck * ngroups;
  const int walk = (int)(l / per_walk);
  const long long rem = l - walk * per_walk;
  const int chunk = (int)(rem / ngroups);
  const int r0 = (int)(rem - (long long)chunk * ngroups) * NR;
  const Geo& g = A.g;
  const int x0a = walk * T;
  if (x0a >= g.L0) return;
  const int x0b = min(x0a + T, g.L0);
  const int lo = (int)((long long)g.V3h * xcd / 8);
  const int hi = (int)((long long)g.V3h * (xcd + 1) / 8);
  const int s = lo + chunk * 128 + threadIdx.x;
  if (s >= hi) return;
  const int nr = min(NR, A.nrhs - r0);
  const int p = A.parity_out, q = 1 - p;
  const V2* inb = A.in.ptr + q * A.in.ps;
  const bool g5i = A.g5_in != 0;
  const int lb = A.lb;
  const long long V3h = g.V3h;
  auto fwd_on = [&](int x) { return !(lb && (x % lb) == lb - 1); };
  auto bwd_on = [&](int x) { return !(lb && (x % lb) == 0); };
  auto wrap = [&](int x) { return x < 0 ? x + g.L0 : (x >= g.L0 ? x - g.L0 : x); };

  // (1 + g0) projections of the inputs on slices x0 - 1 (cp) and x0 (cc) at step x0;
  // rotated by register moves (a runtime slot index would put the arrays in scratch)
  cx<R> cp[NR][2][3], cc[NR][2][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 3; ++c) cp[r][h][c] = cc[r][h][c] = {R(0), R(0)};
  const bool need_p = bwd_on(x0a), need_c = x0a + 1 < x0b && bwd_on(x0a + 1);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nr) {
      cx<R> sp[4][3];
      if (need_p) {
        load_spinor<R>(inb + (r0 + r) * A.in.rs, (long long)wrap(x0a - 1) * V3h + s, g5i, sp);
        project<R>(0, true, sp, cp[r]);
      }
      if (need_c) {
        load_spinor<R>(inb + (r0 + r) * A.in.rs, (long long)x0a * V3h + s, g5i, sp);
        project<R>(0, true, sp, cc[r]);
      }
    }
  }

  for (int x0 = x0a; x0 < x0b; ++x0) {
    const long long j = (long long)x0 * V3h + s;
    const Site st_ = decode(g, j, p);
    const bool sel = hop_selected(A, x0);
    cx<R> acc[NR][4][3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r][a][c] = {R(0), R(0)};
    // backward time hop from the carried projection of input x0 - 1
    if (sel && bwd_on(x0)) {
      cx<R> m[9];
      load_link<R>(A.U, g.Vhp, 0, q, (long long)wrap(x0 - 1) * V3h + s, m);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nr) {
          cx<R> uh[2][3];
          su3_dag_mul<R>(m, cp[r][0], uh[0]);
          su3_dag_mul<R>(m, cp[r][1], uh[1]);
          if (x0 == 0)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
              for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
          accum_recon<R>(0, true, uh, acc[r]);
        }
      }
    }
    // input x0 + 1: forward time hop of output x0 now, carried for output x0 + 2
    const bool use_f = sel && fwd_on(x0);
    const bool keep = x0 + 2 < x0b && bwd_on(x0 + 2);
    if (use_f || keep) {
      const long long jn = (long long)wrap(x0 + 1) * V3h + s;
      cx<R> m[9];
      if (use_f) load_link<R>(A.U, g.Vhp, 0, p, j, m);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nr) {
          cx<R> sp[4][3];
          load_spinor<R>(inb + (r0 + r) * A.in.rs, jn, g5i, sp);
          if (use_f) {
            cx<R> h[2][3], uh[2][3];
            project<R>(0, false, sp, h);
            su3_mul<R>(m, h[0], uh[0]);
            su3_mul<R>(m, h[1], uh[1]);
            if (x0 == g.L0 - 1)
#pragma unroll
              for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
            accum_recon<R>(0, false, uh, acc[r]);
          }
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < 3; ++c) cp[r][h][c] = cc[r][h][c];
          if (keep) project<R>(0, true, sp, cc[r]);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int c = 0; c < 3; ++c) cp[r][h][c] = cc[r][h][c];
    }
    if (sel) {
#pragma unroll
      for (int mu = 1; mu < 4; ++mu) {
        hop_dir<R, NR>(A, p, j, st_, mu, 0, r0, nr, acc);
        hop_dir<R, NR>(A, p, j, st_, mu, 1, r0, nr, acc);
      }
    }
    hop_store<R, NR, true>(A, p, j, r0, nr, sel, acc);
  }
}

// x0-band even-odd hop. XCD k (workgroup id % 8) owns the output slices
// [L0 k / 8, L0 (k + 1) / 8) and every slice-local site of them; a work-item owns the site
// s (j = x0*V3h + s) for a group of NR rhs and steps through the input slices x = x0a - 1
// .. x0b. At step x it loads the input (x, s) once: its (1 - g0) projection completes
// output (x - 1, s) with the forward time hop, and its (1 + g0) projection times
// U_0(x, s)^+ is carried in registers to output (x + 1, s) (a step in x0 keeps s and flips
// the parity). The spatial hops of output (x, s) read the inputs (x, s +/- mu), which the
// neighbouring work-items load in the same step, so an input site is fetched once per
// band and reused through L2 while it is in flight, not across steps. The band edges add
// two input slices per XCD. A workgroup is 128 consecutive slice-local sites; the result
// is stored non-temporally.
template <class R, int NR>
__global__ __launch_bounds__(128) void hop_band_kernel(HopArgs<R> A, int nck) {
  typedef typename vec2<R>::type V2;
  const int xcd = blockIdx.x & 7;
  const long long l = blockIdx.x >> 3;
  const int ngroups = (A.nrhs + NR - 1) / NR;
  const int chunk = (int)(l / ngroups);
  const int r0 = (int)(l - (long long)chunk * ngroups) * NR;
  const Geo& g = A.g;
  const int x0a = (int)((long long)g.L0 * xcd / 8), x0b = (int)((long long)g.L0 * (xcd + 1) / 8);
  const int s = chunk * 128 + threadIdx.x;
  if (chunk >= nck || x0a >= x0b || s >= g.V3h || r0 >= A.nrhs) return;
  const int nr = min(NR, A.nrhs - r0);
  const int p = A.parity_out, q = 1 - p;
  const V2* inb = A.in.ptr + q * A.in.ps;
  const bool g5i = A.g5_in != 0;
  const int lb = A.lb;
  const long long V3h = g.V3h;
  auto fwd_on = [&](int x) { return !(lb && (x % lb) == lb - 1); };
  auto bwd_on = [&](int x) { return !(lb && (x % lb) == 0); };

  cx<R> accp[NR][4][3];   // output x - 1: spatial and backward time hops done
  cx<R> carry[NR][2][3];  // U_0^+ (1 + g0) input (x - 1), for the backward time hop of output x
  bool have_carry = false;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) accp[r][a][c] = {R(0), R(0)};
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 3; ++c) carry[r][h][c] = {R(0), R(0)};
  }

  for (int x = x0a - 1; x <= x0b; ++x) {
    const bool out_prev = x - 1 >= x0a;
    const bool out_cur = x >= x0a && x < x0b;
    const bool sel_prev = out_prev && hop_selected(A, x - 1);
    const bool sel_cur = out_cur && hop_selected(A, x);
    const bool need_f = sel_prev && fwd_on(x - 1);
    const bool need_b = x + 1 < x0b && hop_selected(A, x + 1) && bwd_on(x + 1);
    const int xw = x < 0 ? x + g.L0 : (x >= g.L0 ? x - g.L0 : x);
    const long long jin = (long long)xw * V3h + s;
    // input (x, s): both time projections; the forward one completes output x - 1
    cx<R> hb[NR][2][3];
    if (need_f || need_b) {
      cx<R> hf[NR][2][3];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nr) {
          cx<R> sp[4][3];
          load_spinor<R>(inb + (r0 + r) * A.in.rs, jin, g5i, sp);
          project<R>(0, false, sp, hf[r]);
          project<R>(0, true, sp, hb[r]);
        }
      }
      if (need_f) {
        cx<R> m[9];
        load_link<R>(A.U, g.Vhp, 0, p, (long long)(x - 1) * V3h + s, m);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r < nr) {
            cx<R> uh[2][3];
            su3_mul<R>(m, hf[r][0], uh[0]);
            su3_mul<R>(m, hf[r][1], uh[1]);
            if (x - 1 == g.L0 - 1)
#pragma unroll
              for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
            accum_recon<R>(0, false, uh, accp[r]);
          }
        }
      }
    }
    if (out_prev) hop_store<R, NR, true>(A, p, (long long)(x - 1) * V3h + s, r0, nr, sel_prev, accp);
    // output x starts from the backward time hop carried from input x - 1
    cx<R> acc[NR][4][3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r][a][c] = {R(0), R(0)};
    if (sel_cur && have_carry)
#pragma unroll
      for (int r = 0; r < NR; ++r) accum_recon<R>(0, true, carry[r], acc[r]);
    // the backward time hop of output x + 1 from input x
    if (need_b) {
      cx<R> m[9];
      load_link<R>(A.U, g.Vhp, 0, q, jin, m);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nr) {
          su3_dag_mul<R>(m, hb[r][0], carry[r][0]);
          su3_dag_mul<R>(m, hb[r][1], carry[r][1]);
          if (x + 1 == 0)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
              for (int c = 0; c < 3; ++c) carry[r][k][c] = -carry[r][k][c];
        }
      }
    }
    have_carry = need_b;
    if (out_cur) {
      const long long j = (long long)x * V3h + s;
      if (sel_cur) {
        const Site st_ = decode(g, j, p);
#pragma unroll
        for (int mu = 1; mu < 4; ++mu) {
          hop_dir<R, NR>(A, p, j, st_, mu, 0, r0, nr, acc);
          hop_dir<R, NR>(A, p, j, st_, mu, 1, r0, nr, acc);
        }
      }
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) accp[r][a][c] = acc[r][a][c];
    }
  }
}

// x0-band even-odd hop with the slice tile staged in LDS ("slab"). XCD k (workgroup id % 8)
// owns the output slices [L0 k / 8, L0 (k + 1) / 8), as in the band order. A workgroup owns
// a spatial tile of the slice, TA x1 values x TB x2 values x every x3 (S = TA TB L3h sites of
// one parity), for one group of NR rhs, and walks the band: work-item t owns slice-local
// site s(t) of the output parity and of the input parity alike (a step in x0 keeps s). At
// step x0 it loads its input (x0 + 1, s) once: that input gives the forward time hop of
// output (x0, s) and is written to the LDS copy of slice x0 + 1; the six spatial hops of
// output (x0, s) read the slice-x0 copy for neighbours inside the tile (each input site of
// the tile serves up to six outputs there) and memory only for the halo, which belongs to
// the neighbouring tiles of the same band step; the backward time hop
// U_0(x0 - 1, s)^+ (1 + g0) in(x0 - 1, s) is formed one step earlier from the LDS copy and
// carried in registers. The LDS holds two slice copies (one barrier per step). Workgroups of
// one XCD are ordered tile-major with the rhs groups of a tile adjacent, so the groups of a
// tile read each link at about the same time (L2 hits after the first). Tiles tile the
// slice exactly (TA | L1, TB | L2); work-items t >= S only join the barriers.
//
// The walk keeps the work-item's geometry fixed: the x1 / x2 neighbours and their LDS slots
// are worked out once, the x3 neighbour follows from the x3 bit, which flips with x0, and
// with V3h a multiple of 64 (LIN) every address advances by a constant per slice. Time
// flips, block drops and selections depend on x0 only (uniform over the workgroup). The
// LDS is read through volatile address-space-3 pointers, so that the compiler cannot merge
// the LDS read of a tile neighbour with the memory load of a halo neighbour into one load
// through a generic (flat) address. The link of the next spatial hop is loaded while the
// current one is computed (after the current hop's halo spinor, since loads complete in
// issue order). The FP32 one-rhs kernel is held to three waves per SIMD (at most 168
// registers), the occupancy the pipelined loop is measured fastest at.
template <class T> using lds_ptr = __attribute__((address_space(3))) T*;

template <class R, int NR, bool LIN, bool G5I, bool G5O>
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu((std::is_same<R, float>::value && NR == 1) ? 3 : 2)))
void hop_slab_kernel(HopArgs<R> A, int TA, int TB) {
  typedef typename vec2<R>::type V2;
  extern __shared__ char smem_raw[];
  // LDS: [2 copies][NR][NU 16-byte units][S]; a unit is a pair of FP32 components or one
  // FP64 component
  typedef typename std::conditional<std::is_same<R, float>::value, f4v, d2v>::type UNIT;
  constexpr int NU = std::is_same<R, float>::value ? 6 : 12;
  const lds_ptr<UNIT> lds = (lds_ptr<UNIT>)smem_raw;
  const Geo& g = A.g;
  const int L3h = g.L3h;
  const int S = TA * TB * L3h;
  const int nt2 = g.L2 / TB, ntile = (g.L1 / TA) * nt2;
  const int ngroups = (A.nrhs + NR - 1) / NR;
  const int xcd = blockIdx.x & 7;
  const int l = blockIdx.x >> 3;
  const int tile = l / ngroups;
  const int r0 = (l - tile * ngroups) * NR;
  const int x0a = (int)((long long)g.L0 * xcd / 8), x0b = (int)((long long)g.L0 * (xcd + 1) / 8);
  if (tile >= ntile || x0a >= x0b) return;      // whole workgroup, before any barrier
  const int nr = min(NR, A.nrhs - r0);
  const int x1a = (tile / nt2) * TA, x2a = (tile % nt2) * TB;
  const int t = threadIdx.x;
  const bool act = t < S;
  const int lx3 = act ? t % L3h : 0;
  const int lx2 = act ? (t / L3h) % TB : 0;
  const int lx1 = act ? t / (L3h * TB) : 0;
  const int x1 = x1a + lx1, x2 = x2a + lx2;
  const int s = (x1 * g.L2 + x2) * L3h + lx3;
  const int p = A.parity_out, q = 1 - p;
  const long long V3h = g.V3h, Vhp = g.Vhp;
  const int lb = A.lb;
  const int b_even = (p + x1 + x2) & 1;           // x3 bit of the site at even x0

  // x1 / x2 neighbours (index d: 0 x1+, 1 x1-, 2 x2+, 3 x2-): slice-local index offset and
  // LDS slot (-1: in a neighbouring tile)
  int dsn[4], kn[4];
  {
    const int y1f = x1 + 1 == g.L1 ? 0 : x1 + 1, y1b = x1 == 0 ? g.L1 - 1 : x1 - 1;
    const int y2f = x2 + 1 == g.L2 ? 0 : x2 + 1, y2b = x2 == 0 ? g.L2 - 1 : x2 - 1;
    const int st1 = g.L2 * L3h;
    dsn[0] = (y1f - x1) * st1;
    dsn[1] = (y1b - x1) * st1;
    dsn[2] = (y2f - x2) * L3h;
    dsn[3] = (y2b - x2) * L3h;
    kn[0] = (y1f - x1a >= 0 && y1f - x1a < TA) ? t + (y1f - x1) * L3h * TB : -1;
    kn[1] = (y1b - x1a >= 0 && y1b - x1a < TA) ? t + (y1b - x1) * L3h * TB : -1;
    kn[2] = (y2f - x2a >= 0 && y2f - x2a < TB) ? t + (y2f - x2) * L3h : -1;
    kn[3] = (y2b - x2a >= 0 && y2b - x2a < TB) ? t + (y2b - x2) * L3h : -1;
  }
  // offset (complex numbers) of component 0 of slice-local site sl in slice x0 of a field
  // with NC components per site
  auto off = [&](int x0, int sl, int NC) -> long long {
    if constexpr (LIN) return (long long)x0 * V3h * NC + tiled(sl, 0, NC);
    else return tiled((long long)x0 * V3h + sl, 0, NC);
  };
  // site (x0, sl) in the FP32 pair layout or the FP64 tiled layout (sidx)
  auto soff = [&](int x0, int sl) -> long long {
    if constexpr (LIN) return (long long)x0 * V3h * 12 + sidx<R>(sl, 0);
    else return sidx<R>((long long)x0 * V3h + sl, 0);
  };
  const V2* inb = A.in.ptr + q * A.in.ps;
  auto load_sp = [&](int r, long long o, cx<R> sp[4][3]) {
    const V2* b = inb + (r0 + r) * A.in.rs + o;
    cx<R> v[12];
    if constexpr (std::is_same<R, float>::value) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const f4v w = *(const f4v*)(b + 2 * k * TILE);
        v[2 * k] = {w.x, w.y};
        v[2 * k + 1] = {w.z, w.w};
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = ld<R>(b + c * TILE);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) sp[a][c] = (G5I && a >= 2) ? -v[a * 3 + c] : v[a * 3 + c];
  };
  auto link = [&](int mu, int par, long long o24, cx<R> m[9]) { load_link_at<R>(A.U, Vhp, mu, par, o24, m); };
  auto slot = [&](int cp, int r, int u, int k) { return lds + ((cp * NR + r) * NU + u) * S + k; };
  auto put = [&](int cp, int r, const cx<R> sp[4][3]) {
    const cx<R>* v = &sp[0][0];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if constexpr (std::is_same<R, float>::value)
        *slot(cp, r, u, t) = f4v{v[2 * u].r, v[2 * u].i, v[2 * u + 1].r, v[2 * u + 1].i};
      else
        *slot(cp, r, u, t) = d2v{v[u].r, v[u].i};
    }
  };
  // volatile: the LDS reads stay LDS reads (ds_read), never merged with the memory load
  // that may overwrite them into one load through a generic address
  auto get = [&](int cp, int r, int k, cx<R> sp[4][3]) {
    cx<R>* v = &sp[0][0];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const volatile __attribute__((address_space(3))) UNIT* q = slot(cp, r, u, k);
      const UNIT w = *q;
      if constexpr (std::is_same<R, float>::value) {
        v[2 * u] = {w.x, w.y};
        v[2 * u + 1] = {w.z, w.w};
      } else {
        v[u] = {w.x, w.y};
      }
    }
  };
  auto fwd_on = [&](int x) { return !(lb && (x % lb) == lb - 1); };
  auto bwd_on = [&](int x) { return !(lb && (x % lb) == 0); };

  // U_0(x0 - 1, s)^+ (1 + g0) in(x0 - 1, s) for the backward time hop of the current output
  cx<R> carry[NR][2][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 3; ++c) carry[r][h][c] = {R(0), R(0)};
  if (act) {
    const bool need_c = hop_selected(A, x0a) && bwd_on(x0a);
    const int xp = x0a == 0 ? g.L0 - 1 : x0a - 1;
    cx<R> m[9];
    if (need_c) link(0, q, off(xp, s, 24), m);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r < nr) {
        cx<R> sp[4][3];
        load_sp(r, soff(x0a, s), sp);
        put(0, r, sp);
        if (need_c) {
          cx<R> h[2][3];
          load_sp(r, soff(xp, s), sp);
          project<R>(0, true, sp, h);
          su3_dag_mul<R>(m, h[0], carry[r][0]);
          su3_dag_mul<R>(m, h[1], carry[r][1]);
          if (x0a == 0)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
              for (int c = 0; c < 3; ++c) carry[r][k][c] = -carry[r][k][c];
        }
      }
    }
  }
  __syncthreads();

  for (int x0 = x0a; x0 < x0b; ++x0) {
    const int cp = (x0 - x0a) & 1;
    const bool sel = hop_selected(A, x0);
    const bool use_f = sel && fwd_on(x0), use_b = sel && bwd_on(x0);
    const bool stage = x0 + 1 < x0b;
    const bool carry_next = stage && hop_selected(A, x0 + 1) && bwd_on(x0 + 1);
    if (act) {
      const long long o24 = off(x0, s, 24);
      cx<R> acc[NR][4][3];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[r][a][c] = {R(0), R(0)};
      // input (x0 + 1, s): forward time hop now, LDS copy for the next step
      if (use_f || stage) {
        const int xn = x0 + 1 == g.L0 ? 0 : x0 + 1;
        cx<R> m[9];
        if (use_f) link(0, p, o24, m);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r < nr) {
            cx<R> sp[4][3];
            load_sp(r, soff(xn, s), sp);
            if (stage) put(cp ^ 1, r, sp);
            if (use_f) {
              cx<R> h[2][3], uh[2][3];
              project<R>(0, false, sp, h);
              su3_mul<R>(m, h[0], uh[0]);
              su3_mul<R>(m, h[1], uh[1]);
              if (x0 == g.L0 - 1)
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                  for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
              accum_recon<R>(0, false, uh, acc[r]);
            }
          }
        }
      }
      if (use_b)
#pragma unroll
        for (int r = 0; r < NR; ++r) accum_recon<R>(0, true, carry[r], acc[r]);
      // spatial hop i = 2 (mu - 1) + dir: neighbour site sn and its LDS slot k (-1: halo);
      // x3 neighbours follow from the x3 bit of this slice and are always in the tile
      const int b = b_even ^ (x0 & 1);
      const int h3f = b ? (lx3 + 1 == L3h ? 0 : lx3 + 1) : lx3;
      const int h3b = b ? lx3 : (lx3 == 0 ? L3h - 1 : lx3 - 1);
      auto nbr_of = [&](int i, int& sn, int& k) {
        if (i >= 4) {
          const int h = i == 4 ? h3f : h3b;
          sn = s - lx3 + h;
          k = t - lx3 + h;
        } else {
          sn = s + dsn[i];
          k = kn[i];
        }
      };
      // one spatial hop: spinors sp (one per rhs) through link m (all three rows)
      auto hop_acc = [&](int i, const cx<R> m[9], cx<R> sp[NR][4][3]) {
        const int mu = 1 + i / 2, dir = i & 1;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r < nr) {
            cx<R> h[2][3], uh[2][3];
            project<R>(mu, dir == 1, sp[r], h);
            if (dir == 0) {
              su3_mul<R>(m, h[0], uh[0]);
              su3_mul<R>(m, h[1], uh[1]);
            } else {
              su3_dag_mul<R>(m, h[0], uh[0]);
              su3_dag_mul<R>(m, h[1], uh[1]);
            }
            accum_recon<R>(mu, dir == 1, uh, acc[r]);
          }
        }
      };
      // FP32: the link of the next hop is loaded before the current hop's arithmetic, so
      // that its latency overlaps with it; its two stored rows wait in nxt (FP64 has no
      // registers to spare for that and loads each link just before its hop)
      constexpr bool PIPE = std::is_same<R, float>::value;
      // raw two-row link of hop i (i = 6: U_0(x0, s) of the input parity for the carry)
      auto link_raw = [&](int i, cx<R> raw[6]) {
        int sn, k;
        nbr_of(i, sn, k);
        const int mu = i < 6 ? 1 + i / 2 : 0;
        const int par = i == 6 || (i & 1) ? q : p;
        load_link_raw<R>(A.U, Vhp, mu, par, i < 6 && (i & 1) ? off(x0, sn, 24) : o24, raw);
      };
      cx<R> nxt[PIPE ? 6 : 1];
      if constexpr (PIPE) {
        if (sel) link_raw(0, nxt);
        else if (carry_next) link_raw(6, nxt);
        if (sel) {
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            int sn, k;
            nbr_of(i, sn, k);
            cx<R> m[9], sp[NR][4][3];
#pragma unroll
            for (int e = 0; e < 6; ++e) m[e] = nxt[e];
            // the halo spinor is requested before the next link, so that waiting for it
            // leaves the link's loads in flight (loads complete in issue order)
#pragma unroll
            for (int r = 0; r < NR; ++r) {
              if (r < nr) {
                get(cp, r, k >= 0 ? k : t, sp[r]);
                if (k < 0) load_sp(r, soff(x0, sn), sp[r]);
              }
            }
            if (i < 5) link_raw(i + 1, nxt);
            else if (carry_next) link_raw(6, nxt);
            third_row<R>(m);
            hop_acc(i, m, sp);
          }
        }
      } else if (sel) {
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          const int mu = 1 + i / 2, dir = i & 1;
          int sn, k;
          nbr_of(i, sn, k);
          cx<R> m[9];
          if (dir == 0) link(mu, p, o24, m);
          else link(mu, q, off(x0, sn, 24), m);
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            if (r < nr) {
              cx<R> sp[4][3], h[2][3], uh[2][3];
              get(cp, r, k >= 0 ? k : t, sp);
              if (k < 0) load_sp(r, soff(x0, sn), sp);
              project<R>(mu, dir == 1, sp, h);
              if (dir == 0) {
                su3_mul<R>(m, h[0], uh[0]);
                su3_mul<R>(m, h[1], uh[1]);
              } else {
                su3_dag_mul<R>(m, h[0], uh[0]);
                su3_dag_mul<R>(m, h[1], uh[1]);
              }
              accum_recon<R>(mu, dir == 1, uh, acc[r]);
            }
          }
        }
      }
      // out = a x + b (g5) acc, zero on unselected slices, non-temporal
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r >= nr) continue;
        V2* o = A.out.ptr + (r0 + r) * A.out.rs + p * A.out.ps;
        const V2* xo = A.x.ptr ? A.x.ptr + (r0 + r) * A.x.rs + p * A.x.ps : nullptr;
        store_out<R, true>(o, xo, (long long)x0 * V3h + s, sel, G5O, A.a, A.b, acc[r]);
      }
      // the backward time hop of output (x0 + 1, s) from input (x0, s) (LDS copy); its link
      // is already in nxt
      if (carry_next) {
        cx<R> m[9];
        if constexpr (PIPE) {
#pragma unroll
          for (int e = 0; e < 6; ++e) m[e] = nxt[e];
          third_row<R>(m);
        } else {
          link(0, q, o24, m);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r < nr) {
            cx<R> sp[4][3], h[2][3];
            get(cp, r, t, sp);
            project<R>(0, true, sp, h);
            su3_dag_mul<R>(m, h[0], carry[r][0]);
            su3_dag_mul<R>(m, h[1], carry[r][1]);
          }
        }
      }
    }
    __syncthreads();
  }
}

// FP16 output site j of parity p and rhs r: out = a x + b (g5) acc, zero on unselected
// sites, stored as three quad words (non-temporal) divided by the site norm (the largest
// component magnitude), and the norm. Fused reductions of the values before their
// rounding to FP16 (summed over the site in FP32, added in FP64): RED 1: red[0] +=
// ||out||^2; RED 3: red[0..2] += Re <out, x>, Im <out, x> (out conjugated), ||out||^2.
template <int RED>
__device__ __forceinline__ void store_out16(const Field<h16>& out, const Field<h16>& x, int r, int p, long long j,
                                            long long Vhp, bool sel, bool g5o, float a, float b,
                                            const cx<float> acc[4][3], double red[3]) {
  cx<float> v[12];
  const bool wx = sel && x.ptr;
  float xq[24];
  if (wx) {
    const __half2* xb = x.ptr + r * x.rs + p * x.ps + sidx<h16>(j, 0);
    const float xm = ((const float*)(x.ptr + r * x.rs + x.no))[(x.ps ? p : 0) * Vhp + j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const u4v w = *(const u4v*)(xb + 4 * k * TILE);
      const unsigned e[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 h = __half22float2(h2_of(e[i]));
        xq[8 * k + 2 * i] = h.x * xm;
        xq[8 * k + 2 * i + 1] = h.y * xm;
      }
    }
  }
  float m = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = sp * 3 + c;
      cx<float> h = acc[sp][c];
      if (g5o && sp >= 2) h = -h;
      cx<float> val = {b * h.r, b * h.i};
      if (wx) {
        val.r += a * xq[2 * k];
        val.i += a * xq[2 * k + 1];
      }
      v[k] = sel ? val : cx<float>{0.0f, 0.0f};
      m = fmaxf(m, fmaxf(fabsf(v[k].r), fabsf(v[k].i)));
      if (RED == 1 || RED == 3) s2 = fmaf(v[k].r, v[k].r, fmaf(v[k].i, v[k].i, s2));
      if (RED == 3 && wx) {
        s0 = fmaf(v[k].r, xq[2 * k], fmaf(v[k].i, xq[2 * k + 1], s0));
        s1 = fmaf(v[k].r, xq[2 * k + 1], fmaf(-v[k].i, xq[2 * k], s1));
      }
    }
  if (RED == 1) red[0] += (double)s2;
  if (RED == 3) {
    red[0] += (double)s0;
    red[1] += (double)s1;
    red[2] += (double)s2;
  }
  const float inv = m > 0.0f ? 1.0f / m : 0.0f;
  __half2* ob = out.ptr + r * out.rs + p * out.ps + sidx<h16>(j, 0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    u4v w;
    w.x = u_of(__floats2half2_rn(v[4 * k].r * inv, v[4 * k].i * inv));
    w.y = u_of(__floats2half2_rn(v[4 * k + 1].r * inv, v[4 * k + 1].i * inv));
    w.z = u_of(__floats2half2_rn(v[4 * k + 2].r * inv, v[4 * k + 2].i * inv));
    w.w = u_of(__floats2half2_rn(v[4 * k + 3].r * inv, v[4 * k + 3].i * inv));
    __builtin_nontemporal_store(w, (u4v*)(ob + 4 * k * TILE));
  }
  __builtin_nontemporal_store(m, (float*)(out.ptr + r * out.rs + out.no) + (out.ps ? p : 0) * Vhp + j);
}

// x0 band (XCD share, bands [L0 k / 8, L0 (k + 1) / 8)) holding slice x
__device__ __host__ __forceinline__ int slice_band(int L0, int x) {
  int k = 0;
  while (k < 7 && L0 * (k + 1) / 8 <= x) ++k;
  return k;
}

// Slab hop with direct memory-to-LDS staging (FP32 storage and arithmetic, or FP16 storage
// with the packed FP16 hop terms of site_io.h; one rhs per workgroup). The band and
// tile are those of the slab kernel, but the LDS holds one input slice of the tile together
// with its x1 / x2 halo, written by global_load_lds (16 bytes per lane, no registers) after
// a barrier, so that every spatial neighbour of a step is read from LDS and the memory
// latency of a step is paid once, in the load of the next slice. The forward time hop of
// output x0 - 1 uses the same LDS copy of slice x0 at the start of the step, so the partial
// output x0 - 1 (spatial hops and backward hop) is held in registers across the load; the
// backward half-spinor of output x0 + 1 is computed from slice x0 before it is replaced.
// A halo site is also the input of a neighbouring tile's workgroup in the same step; it is
// read from L2 only while the two workgroups stay within a fraction of a step of each
// other. LDS: [NW 16-byte words][kSlabdUnit] holding S tile sites, then H halo sites
// (2 TB L3h in x1, 2 TA L3h in x2; none where the tile spans the direction), S + H <=
// kSlabdUnit; the fixed stride keeps the word offsets immediate. A site is 6 pair words in
// FP32 and 3 quad words, plus an FP32 norm in a [kSlabdUnit] array after the words, in
// FP16 (larger FP16 tiles, 4 x 8 x 12 on 24^3 in 35 KB, ran slower: two 6-wave
// workgroups per CU hide the loads of a step less well than four 3-wave ones).
constexpr int kSlabdUnit = 416;
template <class SR> constexpr size_t slabd_lds() {
  return std::is_same<SR, h16>::value ? (size_t)kSlabdUnit * (3 * 16 + 4) : (size_t)kSlabdUnit * 96;
}

template <class SR, bool LIN, bool G5I, bool G5O, int RED>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3)))
void hop_slabd_kernel(HopArgs<SR> A, int TA, int TB) {
  typedef float R;
  typedef typename vec2<SR>::type V2;
  constexpr bool F16 = std::is_same<SR, h16>::value;
  constexpr int NW = F16 ? 3 : 6;               // 16-byte words per site
  using LW = std::conditional_t<F16, unsigned, cx<float>>;   // a stored link entry
  constexpr int NL = F16 ? 9 : 6;               // entries per link (FP16: the three-row copy)
  extern __shared__ char smem_raw[];
  const lds_ptr<f4v> lds = (lds_ptr<f4v>)smem_raw;   // FP16: the words' bits
  const lds_ptr<float> ldn = (lds_ptr<float>)(smem_raw + NW * kSlabdUnit * 16);   // FP16 norms
  const Geo& g = A.g;
  const int L3h = g.L3h;
  const int S = TA * TB * L3h;
  const int F1 = TA < g.L1 ? TB * L3h : 0, F2 = TB < g.L2 ? TA * L3h : 0;   // halo face sizes
  const int H = 2 * (F1 + F2);
  constexpr int SH = kSlabdUnit;
  const int nt2 = g.L2 / TB, ntile = (g.L1 / TA) * nt2;
  // XCD k walks x0 band k of 8 over all tiles, the rhs of a tile next to each other (they
  // share its links)
  const int xcd = blockIdx.x & 7;
  const int l = blockIdx.x >> 3;
  const int tile = l / A.nrhs;
  const int r0 = l - tile * A.nrhs;
  const int x0a = g.L0 * xcd / 8, x0b = g.L0 * (xcd + 1) / 8;
  if (tile >= ntile || x0a >= x0b) return;      // whole workgroup, before any barrier
  const int x1a = (tile / nt2) * TA, x2a = (tile % nt2) * TB;
  const int t = threadIdx.x;
  const bool act = t < S, hact = t < H;
  const int lx3 = act ? t % L3h : 0;
  const int lx2 = act ? (t / L3h) % TB : 0;
  const int lx1 = act ? t / (L3h * TB) : 0;
  const int x1 = x1a + lx1, x2 = x2a + lx2;
  const int s = (x1 * g.L2 + x2) * L3h + lx3;
  const int p = A.parity_out, q = 1 - p;
  const long long V3h = g.V3h, Vhp = g.Vhp;
  const int lb = A.lb;
  const int b_even = (p + x1 + x2) & 1;           // x3 bit of the site at even x0

  // halo site loaded by this thread (t < H), faces in the order x1+, x1-, x2+, x2-
  int hs = 0;
  if (hact) {
    int y1, y2, idx;
    if (t < 2 * F1) {
      idx = t < F1 ? t : t - F1;
      y1 = t < F1 ? (x1a + TA == g.L1 ? 0 : x1a + TA) : (x1a == 0 ? g.L1 - 1 : x1a - 1);
      y2 = x2a + idx / L3h;
    } else {
      const int u = t - 2 * F1;
      idx = u < F2 ? u : u - F2;
      y2 = u < F2 ? (x2a + TB == g.L2 ? 0 : x2a + TB) : (x2a == 0 ? g.L2 - 1 : x2a - 1);
      y1 = x1a + idx / L3h;
    }
    hs = (y1 * g.L2 + y2) * L3h + idx % L3h;
  }
  // x1 / x2 neighbours (d: 0 x1+, 1 x1-, 2 x2+, 3 x2-): slice-local index offset (for the
  // backward links) and LDS slot (tile or halo)
  int dsn[4], kn[4];
  {
    const int y1f = x1 + 1 == g.L1 ? 0 : x1 + 1, y1b = x1 == 0 ? g.L1 - 1 : x1 - 1;
    const int y2f = x2 + 1 == g.L2 ? 0 : x2 + 1, y2b = x2 == 0 ? g.L2 - 1 : x2 - 1;
    const int st1 = g.L2 * L3h;
    dsn[0] = (y1f - x1) * st1;
    dsn[1] = (y1b - x1) * st1;
    dsn[2] = (y2f - x2) * L3h;
    dsn[3] = (y2b - x2) * L3h;
    const int f1 = lx2 * L3h + lx3, f2 = lx1 * L3h + lx3;
    kn[0] = (y1f - x1a >= 0 && y1f - x1a < TA) ? t + (y1f - x1) * L3h * TB : S + f1;
    kn[1] = (y1b - x1a >= 0 && y1b - x1a < TA) ? t + (y1b - x1) * L3h * TB : S + F1 + f1;
    kn[2] = (y2f - x2a >= 0 && y2f - x2a < TB) ? t + (y2f - x2) * L3h : S + 2 * F1 + f2;
    kn[3] = (y2b - x2a >= 0 && y2b - x2a < TB) ? t + (y2b - x2) * L3h : S + 2 * F1 + F2 + f2;
  }
  // 16-byte word of site (x0, sl) in a 64-site tile row of W words per site: a slice base
  // (uniform) plus a 32-bit site offset when the slices are whole tile rows (LIN)
  auto word = [&](const f4v* base, int x0, int sl, int W) -> const f4v* {
    if constexpr (LIN) return base + (long long)x0 * V3h * W + ((sl >> 6) * (64 * W) + (sl & 63));
    else {
      const long long j = (long long)x0 * V3h + sl;
      return base + (j >> 6) * (64 * W) + (j & 63);
    }
  };
  const f4v* inb = (const f4v*)(A.in.ptr + r0 * A.in.rs + q * A.in.ps);
  const float* inn = F16 ? (const float*)(A.in.ptr + r0 * A.in.rs + A.in.no) + (A.in.ps ? q : 0) * Vhp : nullptr;
  // words (and FP16 norm) of slice-local site sl of slice x to LDS slot base + lane
  auto dma = [&](int x, int sl, int base) {
    const f4v* src = word(inb, x, sl, NW);
#pragma unroll
    for (int u = 0; u < NW; ++u)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + u * TILE),
                                       (__attribute__((address_space(3))) void*)(lds + u * SH + base), 16, 0, 0);
    if constexpr (F16)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(inn + (long long)x * V3h + sl),
                                       (__attribute__((address_space(3))) void*)(ldn + base), 4, 0, 0);
  };
  // slice x (tile, and halo if asked) into LDS; lane i of a wave writes slot base + i
  auto stage = [&](int x, bool halo) {
    const int w64 = t & ~63;
    if (act) dma(x, s, w64);
    if (halo && hact) dma(x, hs, S + w64);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's loads have landed
    __syncthreads();
  };
  cx<R> acc[4][3], carry[2][3];
  // FP32: spinor of LDS slot k (volatile: stays a ds_read); gamma5 on input applied here.
  // Returns 1, the factor the reconstruction multiplies by (FP16 uses term16 below).
  auto get = [&](int k, cx<R> sp[4][3]) -> R {
    cx<R> v[12];
    const R m = R(1);
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const volatile __attribute__((address_space(3))) f4v* a = lds + u * SH + k;
      const f4v w = *a;
      v[2 * u] = {w.x, w.y};
      v[2 * u + 1] = {w.z, w.w};
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) sp[a][c] = (G5I && a >= 2) ? -v[a * 3 + c] : v[a * 3 + c];
    return m;
  };
  // acc += w * reconstruct(g)
  auto recon = [&](int mu, bool plus, const cx<R> g[2][3], R w) {
    if constexpr (F16) accum_recon_scaled<R>(mu, plus, g, w, acc);
    else accum_recon<R>(mu, plus, g, acc);
  };
  // FP32: carry = U^+ h (w = 1)
  auto carry_of = [&](const cx<R> m[9], const cx<R> h[2][3], R) {
    su3_dag_mul<R>(m, h[0], carry[0]);
    su3_dag_mul<R>(m, h[1], carry[1]);
  };
  auto fwd_on = [&](int x) { return !(lb && (x % lb) == lb - 1); };
  auto bwd_on = [&](int x) { return !(lb && (x % lb) == 0); };
  // stored entries of a link: U_mu at slice-local site sl of slice x, parity par (FP32: the
  // two rows of the FP32 copy, three pair words per link; FP16: the nine entries of the
  // three-row FP16 copy, two quads and a single entry)
  auto link_raw = [&](int mu, int par, int x, int sl, LW raw[NL]) {
    if constexpr (F16) {
      const __half2* ub = A.U + 48 * Vhp + par * 36 * Vhp + 9 * mu * TILE;
      if constexpr (LIN) load_link16x3_words(ub + (long long)x * V3h * 36 + (sl >> 6) * (64 * 36), sl & 63, raw);
      else {
        const long long j = (long long)x * V3h + sl;
        load_link16x3_words(ub + (j >> 6) * (64 * 36), (int)(j & 63), raw);
      }
    } else {
      const f4v* u = word((const f4v*)A.U + par * 12 * Vhp, x, sl, 12) + 192 * mu;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const f4v v = u[64 * k];
        raw[2 * k] = {v.x, v.y};
        raw[2 * k + 1] = {v.z, v.w};
      }
    }
  };

  // FP16: w = U h (plus false) or U^dagger h (plus true) of the projection of LDS slot k,
  // in packed FP16 (hop16_term) with the nine link entries lw of the three-row copy;
  // returns the site norm of slot k (the factor the callers fold into the reconstruction)
  auto term16 = [&](int mu, bool plus, int k, const LW lw[NL], cx<R> w[2][3]) -> R {
    if constexpr (F16) {
      unsigned e[9], sw[12];
#pragma unroll
      for (int i = 0; i < 9; ++i) e[i] = lw[i];
      const R m = *(const volatile __attribute__((address_space(3))) float*)(ldn + k);
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const volatile __attribute__((address_space(3))) f4v* a = lds + u * SH + k;
        // the whole word is reinterpreted (a bit cast of one vector element reads the
        // vector's first element with this compiler)
        const u4v v = __builtin_bit_cast(u4v, (f4v)*a);
        sw[4 * u] = v.x;
        sw[4 * u + 1] = v.y;
        sw[4 * u + 2] = v.z;
        sw[4 * u + 3] = v.w;
      }
      hop16_term<G5I>(mu, plus, e, sw, w);
      return m;
    } else {
      return R(0);
    }
  };
  // FP16: carry = w * uh
  auto carry16 = [&](const cx<R> uh[2][3], R w) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int c = 0; c < 3; ++c) carry[kk][c] = {w * uh[kk][c].r, w * uh[kk][c].i};
  };

  // fused reductions (A.npart, RED = A.red): per-thread sums over the outputs of the
  // current block of A.nlb slices, reduced over the workgroup when the block ends; the
  // partials of (system, tile, band) go to slot tile + ntile * (band - first band of the
  // block), and the workgroup of the first band zeroes the slots no band fills
  constexpr bool nrm = RED > 0;
  constexpr int NV = RED == 1 ? 1 : 3;          // values per slot
  double nacc[3] = {0.0, 0.0, 0.0};
  __shared__ double nsh[3][8];
  auto flush = [&](int blk) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double v = nacc[i];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if ((t & 63) == 0) nsh[i][t >> 6] = v;
    }
    __syncthreads();
    if (t == 0) {
      const int xa = blk * A.nlb, xb = min(xa + A.nlb, g.L0) - 1;
      const int first = slice_band(g.L0, xa), last = slice_band(g.L0, xb);
      double* dst = A.npart + ((long long)r0 * (g.L0 / A.nlb) + blk) * A.nslot * NV;
      for (int i = 0; i < NV; ++i) {
        double sum = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += nsh[i][w];
        dst[(tile + ntile * (xcd - first)) * NV + i] = sum;
      }
      if (xcd == first)
        for (int pc = 1; pc < A.nslot / ntile; ++pc) {
          const int k = first + pc;
          if (k > last || g.L0 * k / 8 == g.L0 * (k + 1) / 8)
            for (int i = 0; i < NV; ++i) dst[(tile + ntile * pc) * NV + i] = 0.0;
        }
    }
    __syncthreads();
    nacc[0] = nacc[1] = nacc[2] = 0.0;
  };

  LW nxt[NL], alt[NL];   // alt: FP16 only (odd spatial hops)
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[a][c] = {R(0), R(0)};
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < 3; ++c) carry[h][c] = {R(0), R(0)};

  // prologue: the backward half-spinor of output x0a from slice x0a - 1, then slice x0a
  if (hop_selected(A, x0a) && bwd_on(x0a)) {
    const int xp = x0a == 0 ? g.L0 - 1 : x0a - 1;
    if (act) link_raw(0, q, xp, s, nxt);
    stage(xp, false);
    if (act) {
      if constexpr (F16) {
        cx<R> uh[2][3];
        const R w = term16(0, true, t, nxt, uh);
        carry16(uh, w);
      } else {
        cx<R> m[9], sp[4][3], h[2][3];
#pragma unroll
        for (int e = 0; e < 6; ++e) m[e] = nxt[e];
        third_row<R>(m);
        const R w = get(t, sp);
        project<R>(0, true, sp, h);
        carry_of(m, h, w);
      }
      if (x0a == 0)
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) carry[k][c] = -carry[k][c];
    }
    __syncthreads();
  }
  stage(x0a, hop_selected(A, x0a));

  for (int x0 = x0a; x0 <= x0b; ++x0) {
    // LDS: slice x0 (x0 == x0b: tile only, wrapped); acc: output x0 - 1 without its forward
    // time hop; carry: backward half-spinor of output x0
    const int xo = x0 - 1;                        // output finished in this step
    const bool last = x0 == x0b;
    const bool sel = !last && hop_selected(A, x0);
    const bool fin = x0 > x0a;
    const bool use_f = fin && hop_selected(A, xo) && fwd_on(xo);
    const bool carry_next = !last && x0 + 1 < x0b && hop_selected(A, x0 + 1) && bwd_on(x0 + 1);
    if (nrm && fin && xo > x0a && xo / A.nlb != (xo - 1) / A.nlb) flush((xo - 1) / A.nlb);
    if (act) {
      if (fin) {
        if (use_f) {
          if constexpr (F16) {
            cx<R> uh[2][3];
            const R w = term16(0, false, t, nxt, uh);    // link loaded with this slice
            recon(0, false, uh, xo == g.L0 - 1 ? -w : w);
          } else {
            cx<R> m[9], sp[4][3], h[2][3], uh[2][3];
#pragma unroll
            for (int e = 0; e < 6; ++e) m[e] = nxt[e];   // loaded with this slice
            third_row<R>(m);
            const R w = get(t, sp);
            project<R>(0, false, sp, h);
            su3_mul<R>(m, h[0], uh[0]);
            su3_mul<R>(m, h[1], uh[1]);
            if (xo == g.L0 - 1)
#pragma unroll
              for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) uh[k][c] = -uh[k][c];
            recon(0, false, uh, w);
          }
        }
        if constexpr (F16) {
          store_out16<RED>(A.out, A.x, r0, p, (long long)xo * V3h + s, Vhp, hop_selected(A, xo), G5O, A.a, A.b,
                           acc, nacc);
        } else {
          V2* o = A.out.ptr + r0 * A.out.rs + p * A.out.ps;
          const V2* xv = A.x.ptr ? A.x.ptr + r0 * A.x.rs + p * A.x.ps : nullptr;
          store_out_red<R, true, RED>(o, xv, (long long)xo * V3h + s, hop_selected(A, xo), G5O, A.a, A.b, acc,
                                      nacc);
        }
      }
      if (!last) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[a][c] = {R(0), R(0)};
        if (sel && bwd_on(x0)) accum_recon<R>(0, true, carry, acc);
        if (sel) {
          const int b = b_even ^ (x0 & 1);
          const int h3f = b ? (lx3 + 1 == L3h ? 0 : lx3 + 1) : lx3;
          const int h3b = b ? lx3 : (lx3 == 0 ? L3h - 1 : lx3 - 1);
          // spatial hop i = 2 (mu - 1) + dir; the link of hop i + 1 is loaded before the
          // arithmetic of hop i
          auto hop_link = [&](int i, LW raw[NL]) {
            const int mu = 1 + i / 2;
            if (i & 1) link_raw(mu, q, x0, i >= 4 ? s - lx3 + h3b : s + dsn[i], raw);
            else link_raw(mu, p, x0, s, raw);
          };
          hop_link(0, nxt);
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            const int mu = 1 + i / 2, dir = i & 1;
            const int k = i >= 4 ? t - lx3 + (i == 4 ? h3f : h3b) : kn[i];
            if constexpr (F16) {
              // the links of hops 0, 2, 4 in nxt and of 1, 3, 5 in alt, so that the next
              // link is loaded into the other buffer without copying the current one
              cx<R> uh[2][3];
              R w;
              if (i & 1) {
                if (i < 5) hop_link(i + 1, nxt);
                else if (carry_next) link_raw(0, q, x0, s, nxt);
                w = term16(mu, dir == 1, k, alt, uh);
              } else {
                hop_link(i + 1, alt);
                w = term16(mu, dir == 1, k, nxt, uh);
              }
              recon(mu, dir == 1, uh, w);
            } else {
              cx<R> m[9], sp[4][3], h[2][3], uh[2][3];
#pragma unroll
              for (int e = 0; e < 6; ++e) m[e] = nxt[e];
              if (i < 5) hop_link(i + 1, nxt);
              else if (carry_next) link_raw(0, q, x0, s, nxt);
              const R w = get(k, sp);
              third_row<R>(m);
              project<R>(mu, dir == 1, sp, h);
              if (dir == 0) {
                su3_mul<R>(m, h[0], uh[0]);
                su3_mul<R>(m, h[1], uh[1]);
              } else {
                su3_dag_mul<R>(m, h[0], uh[0]);
                su3_dag_mul<R>(m, h[1], uh[1]);
              }
              recon(mu, dir == 1, uh, w);
            }
            // the accumulator is next read in the following step: without this pin the
            // compiler sinks the arithmetic of all six hops below their loads and spills
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int c = 0; c < 3; ++c) asm volatile("" : "+v"(acc[a][c].r), "+v"(acc[a][c].i));
          }
        }
        // backward half-spinor of output x0 + 1 from slice x0
        if (carry_next) {
          if constexpr (F16) {
            LW cur[NL];
            if (sel) {
#pragma unroll
              for (int e = 0; e < NL; ++e) cur[e] = nxt[e];
            } else {
              link_raw(0, q, x0, s, cur);
            }
            cx<R> uh[2][3];
            const R w = term16(0, true, t, cur, uh);
            carry16(uh, w);
          } else {
            cx<R> m[9], sp[4][3], h[2][3];
            if (sel) {
#pragma unroll
              for (int e = 0; e < 6; ++e) m[e] = nxt[e];
            } else {
              link_raw(0, q, x0, s, m);
            }
            third_row<R>(m);
            const R w = get(t, sp);
            project<R>(0, true, sp, h);
            carry_of(m, h, w);
          }
        }
      }
    }
    if (!last) {
      // replace slice x0 by slice x0 + 1 (tile only for the last one, which serves the
      // forward hop of output x0b - 1)
      const int xn = x0 + 1 == g.L0 ? 0 : x0 + 1;
      const bool f_next = hop_selected(A, x0) && fwd_on(x0);   // forward hop of output x0
      __syncthreads();
      if (x0 + 1 < x0b || f_next) {
        if (act && f_next) link_raw(0, p, x0, s, nxt);
        stage(xn, x0 + 1 < x0b && hop_selected(A, x0 + 1));
      }
    }
  }
  if (nrm) flush((x0b - 1) / A.nlb);
}

static inline long long round8(long long n) { return (n + 7) / 8 * 8; }

template <class R, int NR, bool SWEEP> static void launch_reg(const HopArgs<R>& A, hipStream_t st) {
  const bool full = A.parity_out < 0;
  const long long per = full ? 128 : 256;
  const long long chunks = (A.g.Vh + per - 1) / per;
  const long long groups = (A.nrhs + NR - 1) / NR;
  const dim3 grid((unsigned)round8(chunks * groups)), blk(256);
  if (full) hipLaunchKernelGGL((hop_reg_kernel<R, true, NR, SWEEP>), grid, blk, 0, st, A, chunks);
  else hipLaunchKernelGGL((hop_reg_kernel<R, false, NR, SWEEP>), grid, blk, 0, st, A, chunks);
}

template <class R, int NR> static void launch_march(const HopArgs<R>& A, hipStream_t st) {
  const bool full = A.parity_out < 0;
  const int piece = (A.g.V3h + 7) / 8;                 // largest of the 8 pieces
  const int per = full ? 64 : 128;
  const int nck = (piece + per - 1) / per;
  const long long groups = (A.nrhs + NR - 1) / NR;
  const dim3 grid((unsigned)(8LL * A.g.L0 * nck * groups)), blk(128);
  if (full) hipLaunchKernelGGL((hop_march_kernel<R, true, NR>), grid, blk, 0, st, A, nck);
  else hipLaunchKernelGGL((hop_march_kernel<R, false, NR>), grid, blk, 0, st, A, nck);
}

template <class R, int NR> static void launch_walk(const HopArgs<R>& A, hipStream_t st) {
  const int piece = (A.g.V3h + 7) / 8;
  const int nck = (piece + 127) / 128;
  const int T = A.g.L0 < HOP_WALK_T ? A.g.L0 : HOP_WALK_T;
  const int nwalk = (A.g.L0 + T - 1) / T;
  const long long groups = (A.nrhs + NR - 1) / NR;
  const dim3 grid((unsigned)(8LL * nwalk * nck * groups)), blk(128);
  hipLaunchKernelGGL((hop_walk_kernel<R, NR>), grid, blk, 0, st, A, nck, T);
}

template <class R, int NR> static void launch_band(const HopArgs<R>& A, hipStream_t st) {
  const int nck = (A.g.V3h + 127) / 128;
  const long long groups = (A.nrhs + NR - 1) / NR;
  const dim3 grid((unsigned)(8LL * nck * groups)), blk(128);
  hipLaunchKernelGGL((hop_band_kernel<R, NR>), grid, blk, 0, st, A, nck);
}

// Tile of the slab kernel: TA | L1 x1 values by TB | L2 x2 values (every x3), with at most
// smax sites (TA TB L3h), chosen to minimise the halo per tile site 2 (1/TA + 1/TB), then to
// maximise the tile.
static void slab_tile(const Geo& g, int smax, int& TA, int& TB) {
  TA = TB = 1;
  double best = 1e30;
  for (int a = 1; a <= g.L1; ++a) {
    if (g.L1 % a) continue;
    for (int b = 1; b <= g.L2; ++b) {
      if (g.L2 % b || a * b * g.L3h > smax) continue;
      const double halo = 2.0 / a + 2.0 / b;
      if (halo < best - 1e-12 || (halo < best + 1e-12 && a * b > TA * TB)) {
        best = halo;
        TA = a;
        TB = b;
      }
    }
  }
}

// LDS budget per workgroup of the slab kernel (two slice copies of the tile for NR rhs)
template <class R, int NR> static void launch_slab(const HopArgs<R>& A, hipStream_t st, int lds_budget) {
  typedef typename vec2<R>::type V2;
  const int per_site = 2 * NR * 12 * (int)sizeof(V2);
  const int smax = min(512, max(A.g.L3h, lds_budget / per_site));
  int TA, TB;
  slab_tile(A.g, smax, TA, TB);
  const int S = TA * TB * A.g.L3h;
  const int ntile = (A.g.L1 / TA) * (A.g.L2 / TB);
  const long long groups = (A.nrhs + NR - 1) / NR;
  const dim3 grid((unsigned)(8LL * ntile * groups)), blk((S + 63) / 64 * 64);
  const size_t lds = (size_t)S * per_site;
  const bool lin = A.g.V3h % TILE == 0;
#define SAP_SLAB(LIN, G5I, G5O) hipLaunchKernelGGL((hop_slab_kernel<R, NR, LIN, G5I, G5O>), grid, blk, lds, st, A, TA, TB)
#define SAP_SLAB_G5(LIN)                                      \
  do {                                                        \
    if (A.g5_in && A.g5_out) SAP_SLAB(LIN, true, true);       \
    else if (A.g5_in) SAP_SLAB(LIN, true, false);             \
    else if (A.g5_out) SAP_SLAB(LIN, false, true);            \
    else SAP_SLAB(LIN, false, false);                         \
  } while (0)
  if (lin) SAP_SLAB_G5(true);
  else SAP_SLAB_G5(false);
#undef SAP_SLAB_G5
#undef SAP_SLAB
}

// Tile of the LDS-staged slab kernel: TA x TB x L3h sites whose slice and x1 / x2 halo fit
// the unit LDS slots, with the fewest halo sites per tile site, then the largest tile.
static void slabd_tile(const Geo& g, int unit, int& TA, int& TB, int& S, int& H) {
  TA = TB = 1;
  double best = 1e30;
  for (int a = 1; a <= g.L1; ++a) {
    if (g.L1 % a) continue;
    for (int b = 1; b <= g.L2; ++b) {
      if (g.L2 % b) continue;
      const int s = a * b * g.L3h;
      const int h = 2 * ((a < g.L1 ? b * g.L3h : 0) + (b < g.L2 ? a * g.L3h : 0));
      if (s + h > unit || s > 512 || h > 512) continue;
      const double ratio = (double)h / s;
      if (ratio < best - 1e-12 || (ratio < best + 1e-12 && a * b > TA * TB)) {
        best = ratio;
        TA = a;
        TB = b;
      }
    }
  }
  S = TA * TB * g.L3h;
  H = 2 * ((TA < g.L1 ? TB * g.L3h : 0) + (TB < g.L2 ? TA * g.L3h : 0));
}

// FP32 and FP16 storage; FP64 runs the slab kernel of the same tile budget
template <class R> static void launch_slabd(const HopArgs<R>& A, hipStream_t st) {
  if constexpr (std::is_same<R, double>::value) {
    launch_slab<R, 1>(A, st, 40 * 1024);
  } else {
    int TA, TB, S, H;
    slabd_tile(A.g, kSlabdUnit, TA, TB, S, H);
    const int ntile = (A.g.L1 / TA) * (A.g.L2 / TB);
    const dim3 grid((unsigned)(8LL * ntile * A.nrhs)), blk((std::max(S, H) + 63) / 64 * 64);
    const size_t lds = slabd_lds<R>();
    const bool lin = A.g.V3h % TILE == 0;
#define SAP_SLABD(LIN, G5I, G5O, RED) \
  hipLaunchKernelGGL((hop_slabd_kernel<R, LIN, G5I, G5O, RED>), grid, blk, lds, st, A, TA, TB)
    // the fused reductions exist without gamma_5 on the input (the solvers' second half
    // hops; they set npart only there): the norm with and without gamma_5 on the output
    // (CG), the dot product and norm without (BiCGstab)
#define SAP_SLABD_G5(LIN)                                                                  \
  do {                                                                                     \
    if (A.npart && A.red == 1 && !A.g5_in && A.g5_out) SAP_SLABD(LIN, false, true, 1);     \
    else if (A.npart && A.red == 1 && !A.g5_in) SAP_SLABD(LIN, false, false, 1);           \
    else if (A.npart && A.red == 3 && !A.g5_in && !A.g5_out) SAP_SLABD(LIN, false, false, 3); \
    else if (A.g5_in && A.g5_out) SAP_SLABD(LIN, true, true, 0);                           \
    else if (A.g5_in) SAP_SLABD(LIN, true, false, 0);                                      \
    else if (A.g5_out) SAP_SLABD(LIN, false, true, 0);                                     \
    else SAP_SLABD(LIN, false, false, 0);                                                  \
  } while (0)
    if (lin) SAP_SLABD_G5(true);
    else SAP_SLABD_G5(false);
#undef SAP_SLABD_G5
#undef SAP_SLABD
  }
}

void launch_slabd16(const HopArgs<h16>& A, hipStream_t st) { launch_slabd<h16>(A, st); }

int slabd_norm_slots(const Geo& g, int nlb) {
  if (nlb <= 0 || g.L0 % nlb) return 0;
  int TA, TB, S, H;
  slabd_tile(g, kSlabdUnit, TA, TB, S, H);
  const int ntile = (g.L1 / TA) * (g.L2 / TB);
  int maxp = 0;
  for (int xa = 0; xa < g.L0; xa += nlb) maxp = std::max(maxp, slice_band(g.L0, xa + nlb - 1) - slice_band(g.L0, xa) + 1);
  return ntile * maxp;
}

template <class R> static void launch_stream(const HopArgs<R>& A, hipStream_t st) {
  typedef typename vec2<R>::type V2;
  constexpr int S = sizeof(R) == 8 ? 128 : 256;     // 48 KB of LDS either way
  const int T = A.lb ? A.lb : (A.g.L0 >= 8 ? 8 : A.g.L0);
  const int nrange = (A.g.V3h + S - 1) / S;
  const int nchunk = (A.g.L0 + T - 1) / T;
  const long long nwg = round8((long long)nrange * nchunk * A.nrhs);
  const size_t lds = 2 * 12 * S * sizeof(V2);
  hipLaunchKernelGGL((hop_stream_kernel<R, S>), dim3((unsigned)nwg), dim3(S), lds, st, A, T, nrange, nchunk);
}

template <class R> void launch_hop(const HopArgs<R>& A, hipStream_t st) {
  const bool full = A.parity_out < 0;
  if (A.map == HOP_MAP_STREAM && !full) {
    launch_stream<R>(A, st);
    return;
  }
  switch (A.map) {
    case HOP_MAP_MARCH1: launch_march<R, 1>(A, st); return;
    case HOP_MAP_MARCH2: launch_march<R, 2>(A, st); return;
    case HOP_MAP_MARCH4: launch_march<R, 4>(A, st); return;
    case HOP_MAP_WALK1:
      if (full) launch_march<R, 1>(A, st);
      else launch_walk<R, 1>(A, st);
      return;
    case HOP_MAP_WALK2:
      if (full) launch_march<R, 2>(A, st);
      else launch_walk<R, 2>(A, st);
      return;
    case HOP_MAP_BAND1:
      if (full) launch_march<R, 1>(A, st);
      else launch_band<R, 1>(A, st);
      return;
    case HOP_MAP_SLAB1:
      if (full) launch_march<R, 1>(A, st);
      else launch_slab<R, 1>(A, st, 40 * 1024);
      return;
    case HOP_MAP_SLAB1W:
      if (full) launch_march<R, 1>(A, st);
      else launch_slab<R, 1>(A, st, 80 * 1024);
      return;
    case HOP_MAP_SLAB2:
      if (full) launch_march<R, 2>(A, st);
      else launch_slab<R, 2>(A, st, 80 * 1024);
      return;
    case HOP_MAP_SLABD:
      if (full) launch_march<R, 1>(A, st);
      else launch_slabd<R>(A, st);
      return;
    default: break;
  }
  if (A.nrhs > 1) {
    switch (A.map) {
      case HOP_MAP_REG2: launch_reg<R, 2, false>(A, st); return;
      case HOP_MAP_REG4: launch_reg<R, 4, false>(A, st); return;
      case HOP_MAP_REG2_SWEEP: launch_reg<R, 2, true>(A, st); return;
      case HOP_MAP_REG4_SWEEP: launch_reg<R, 4, true>(A, st); return;
      default: break;
    }
  }
  int map = (A.map == HOP_MAP_STREAM || A.map >= HOP_MAP_REG2) ? HOP_MAP_SITE : A.map;
  const bool sweep = map >= HOP_SWEEP;
  if (sweep) map -= HOP_SWEEP;
  if (A.nrhs == 1) map = HOP_MAP_SITE;                       // LANE4 / WAVE4 need several rhs
  const bool grouped = map != HOP_MAP_SITE;
  const long long per = grouped ? (full ? 32 : 64) : (full ? 128 : 256);
  const long long groups = grouped ? (A.nrhs + 3) / 4 : A.nrhs;
  const long long chunks = (A.g.Vh + per - 1) / per;
  const dim3 grid((unsigned)round8(chunks * groups)), blk(256);
#define SAP_HOP(F, M, SW) hipLaunchKernelGGL((hop_kernel<R, F, M, SW>), grid, blk, 0, st, A, chunks)
#define SAP_HOP_MAPS(F, SW)                                                              \
  do {                                                                                   \
    if (map == HOP_MAP_LANE4) SAP_HOP(F, HOP_MAP_LANE4, SW);                             \
    else if (map == HOP_MAP_WAVE4) SAP_HOP(F, HOP_MAP_WAVE4, SW);                        \
    else SAP_HOP(F, HOP_MAP_SITE, SW);                                                   \
  } while (0)
  if (full) {
    if (sweep) SAP_HOP_MAPS(true, true);
    else SAP_HOP_MAPS(true, false);
  } else {
    if (sweep) SAP_HOP_MAPS(false, true);
    else SAP_HOP_MAPS(false, false);
  }
#undef SAP_HOP_MAPS
#undef SAP_HOP
}

template void launch_hop<double>(const HopArgs<double>&, hipStream_t);
template void launch_hop<float>(const HopArgs<float>&, hipStream_t);

}  // namespace sap
