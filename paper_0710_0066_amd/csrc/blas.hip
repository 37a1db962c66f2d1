// BLAS-1 kernels and per-system reductions for the batched Krylov solvers.
//
// A "system" is one (rhs, x0-block) pair: block b of length lb holds the sites
// j in [b*Vb, (b+1)*Vb) of each parity, Vb = lb * V3h (lb = L0 for the full lattice).
// Every kernel here runs on the grid (chunk, block, rhs) with CHUNK sites per workgroup,
// so a workgroup never straddles two systems. Sums accumulate in FP64: per-thread
// partials -> wavefront shuffle tree -> LDS across the 4 wavefronts -> one partial per
// workgroup; the finalize kernels add the partials of a system in index order. The
// result is bitwise reproducible run to run.
#include "blas.h"
#include "site_io.h"

namespace sap {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over the 256 threads of a workgroup; valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[4];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;
}

struct Tile {
  bool selected;
  int rhs, blk;
  long long j0, j1;   // site range of this workgroup within its parity
  long long sys;
};

__device__ __forceinline__ Tile tile_of(const SysGrid& G) {
  Tile t;
  t.rhs = blockIdx.z;
  t.blk = blockIdx.y;
  t.sys = (long long)t.rhs * G.nblk + t.blk;
  t.selected = block_selected(G.colour, t.blk);
  t.j0 = (long long)t.blk * G.Vb + (long long)blockIdx.x * CHUNK;
  t.j1 = (long long)t.blk * G.Vb + G.Vb;
  if (t.j0 + CHUNK < t.j1) t.j1 = t.j0 + CHUNK;
  return t;
}

template <class R>
__global__ __launch_bounds__(256) void k_norm2(SysGrid G, Field<R> a, int npar, double* part) {
  const Tile t = tile_of(G);
  double acc = 0.0;
  if (t.selected) {
    for (int p = 0; p < npar; ++p)
      for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
        const SiteR<R> av = site_r(a, t.rhs, p, j, G.Vhp);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const cx<arith_t<R>> v = get(av, c);
          acc += (double)v.r * v.r + (double)v.i * v.i;
        }
      }
  }
  double s = block_sum(acc);
  if (threadIdx.x == 0) part[t.sys * G.nchunk + blockIdx.x] = s;
}

// s -= alpha q ; partial ||s||^2
template <class R>
__global__ __launch_bounds__(256) void k_cg_s(SysGrid G, Field<R> s, Field<R> q, const double* alpha,
                                              double* part) {
  typedef arith_t<R> A;
  const Tile t = tile_of(G);
  double acc = 0.0;
  if (t.selected) {
    const A al = (A)alpha[t.sys];
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
      const SiteR<R> sr = site_r(s, t.rhs, 0, j, G.Vhp), qr = site_r(q, t.rhs, 0, j, G.Vhp);
      SiteW<R> sw = site_w(s, t.rhs, 0, j, G.Vhp);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        cx<A> sv = get(sr, c);
        const cx<A> qv = get(qr, c);
        sv.r -= al * qv.r; sv.i -= al * qv.i;
        put(sw, c, sv);
        acc += (double)sv.r * sv.r + (double)sv.i * sv.i;
      }
      close(sw);
    }
  }
  double sm = block_sum(acc);
  if (threadIdx.x == 0) part[t.sys * G.nchunk + blockIdx.x] = sm;
}

// x += alpha p ; p = r + beta p  (the solution update of an iteration, deferred to the
// direction update so that p is read once)
template <class R>
__global__ __launch_bounds__(256) void k_cg_xp(SysGrid G, Field<R> x, Field<R> p, Field<R> r, const double* alpha,
                                               const double* beta) {
  typedef arith_t<R> A;
  const Tile t = tile_of(G);
  if (!t.selected) return;
  const A al = (A)alpha[t.sys], be = (A)beta[t.sys];
  for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
    const SiteR<R> xr = site_r(x, t.rhs, 0, j, G.Vhp), pr = site_r(p, t.rhs, 0, j, G.Vhp);
    const SiteR<R> rr = site_r(r, t.rhs, 0, j, G.Vhp);
    SiteW<R> xw = site_w(x, t.rhs, 0, j, G.Vhp), pw = site_w(p, t.rhs, 0, j, G.Vhp);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      cx<A> xv = get(xr, c), pv = get(pr, c);
      const cx<A> rv = get(rr, c);
      xv.r += al * pv.r; xv.i += al * pv.i;
      pv.r = rv.r + be * pv.r;
      pv.i = rv.i + be * pv.i;
      put(xw, c, xv);
      put(pw, c, pv);
    }
    close(xw);
    close(pw);
  }
}

// out = src (both parities if npar == 2), converting precision
template <class Ro, class Ri>
__global__ __launch_bounds__(256) void k_convert(SysGrid G, Field<Ro> out, Field<Ri> in, int npar) {
  typedef arith_t<Ro> Ao;
  const Tile t = tile_of(G);
  for (int p = 0; p < npar; ++p)
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
      const SiteR<Ri> ir = site_r(in, t.rhs, p, j, G.Vhp);
      SiteW<Ro> ow = site_w(out, t.rhs, p, j, G.Vhp);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const cx<arith_t<Ri>> v = get(ir, c);
        cx<Ao> w = {(Ao)v.r, (Ao)v.i};
        if (!t.selected) w = {Ao(0), Ao(0)};
        put(ow, c, w);
      }
      close(ow);
    }
}

// x64 += e (both parities), e at the inner precision
template <class R>
__global__ __launch_bounds__(256) void k_add_mixed(SysGrid G, Field<double> x, Field<R> e) {
  const Tile t = tile_of(G);
  if (!t.selected) return;
  for (int p = 0; p < 2; ++p) {
    double2* xb = x.ptr + t.rhs * x.rs + p * x.ps;
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
      const SiteR<R> er = site_r(e, t.rhs, p, j, G.Vhp);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const long long o = tiled(j, c, 12);
        cx<double> xv = ld<double>(xb + o);
        const cx<arith_t<R>> ev = get(er, c);
        xv.r += (double)ev.r;
        xv.i += (double)ev.i;
        st<double>(xb + o, xv);
      }
    }
  }
}

// r = b - Ax (FP64, the first npar parities: 2 both, 1 even only), partial ||r||^2
__global__ __launch_bounds__(256) void k_resid(SysGrid G, Field<double> r, Field<double> b,
                                               Field<double> Ax, double* part, int npar) {
  const Tile t = tile_of(G);
  double acc = 0.0;
  for (int p = 0; p < npar; ++p) {
    double2* rb = r.ptr + t.rhs * r.rs + p * r.ps;
    const double2* bb = b.ptr + t.rhs * b.rs + p * b.ps;
    const double2* ab = Ax.ptr + t.rhs * Ax.rs + p * Ax.ps;
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256)
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const long long o = tiled(j, c, 12);
        cx<double> bv = ld<double>(bb + o), av = ld<double>(ab + o);
        cx<double> rv = t.selected ? bv - av : cx<double>{0.0, 0.0};
        st<double>(rb + o, rv);
        acc += rv.r * rv.r + rv.i * rv.i;
      }
  }
  double sm = block_sum(acc);
  if (threadIdx.x == 0) part[t.sys * G.nchunk + blockIdx.x] = sm;
}

// out[sys] = sum of the partials of sys, in chunk order
__device__ __forceinline__ double sys_total(const double* part, long long sys, int nchunk) {
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[sys * nchunk + c];
  return s;
}

__global__ void k_fin_sum(int nsys, int nchunk, const double* part, double* out) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) out[s] = sys_total(part, s, nchunk);
}

// Start of an inner CG: bb = ||b_hat||^2 (part_b), gam = ||r||^2 (part_r);
// the system is active unless unselected or already below its target.
__global__ void k_fin_init(SysScal S, int nsys, int nchunk, const double* part_b, const double* part_r,
                           const int* selected, const double* target2) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    const double bb = sys_total(part_b, s, nchunk);
    const double gm = sys_total(part_r, s, nchunk);
    S.ss[s] = bb;
    S.gam[s] = gm;
    S.alpha[s] = 0.0;
    S.beta[s] = 0.0;
    const int act = selected[s] && bb > target2[s] && gm > 0.0;
    S.active[s] = act;
    if (!(isfinite(bb) && isfinite(gm))) S.flags[0] = 1;
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) S.flags[1] = cnt;
}

__global__ void k_fin_alpha(SysScal S, int nsys, int nchunk, const double* part_q) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    const double qq = sys_total(part_q, s, nchunk);
    if (!isfinite(qq)) S.flags[0] = 2;
    S.alpha[s] = (S.active[s] && qq > 0.0) ? S.gam[s] / qq : 0.0;
  }
}

__global__ void k_fin_beta(SysScal S, int nsys, int nchunk, const double* part_s, int nchunk_r,
                           const double* part_r, const double* target2) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    const double ss = sys_total(part_s, s, nchunk);
    const double gm = sys_total(part_r, s, nchunk_r);
    if (!(isfinite(ss) && isfinite(gm))) S.flags[0] = 3;
    int act = S.active[s];
    if (act) {
      S.iters[s] += 1;
      S.ss[s] = ss;
      S.beta[s] = S.gam[s] > 0.0 ? gm / S.gam[s] : 0.0;
      S.gam[s] = gm;
      if (ss <= target2[s] || gm == 0.0) act = 0;
    } else {
      S.beta[s] = 0.0;
    }
    S.active[s] = act;
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) S.flags[1] = cnt;
}

// ---- BiCGstab and geometric series ---------------------------------------------------

// three sums over the 256 threads of a workgroup, written by thread 0 to out[0..2]
__device__ __forceinline__ void block_sum3(double a, double b, double c, double* out) {
  __shared__ double sh[3][4];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wid] = a;
    sh[1][wid] = b;
    sh[2][wid] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) out[k] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
}

__device__ __forceinline__ cx<double> cs_get(const double* cs, long long sys, int k) {
  return {cs[8 * sys + 2 * k], cs[8 * sys + 2 * k + 1]};
}
__device__ __forceinline__ void cs_set(double* cs, long long sys, int k, cx<double> v) {
  cs[8 * sys + 2 * k] = v.r;
  cs[8 * sys + 2 * k + 1] = v.i;
}
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.r * b.r + b.i * b.i;
  return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
enum { CS_RHO = 0, CS_ALPHA = 1, CS_OMEGA = 2, CS_BETA = 3 };

template <class R>
__global__ __launch_bounds__(256) void k_cdot3(SysGrid G, Field<R> a, Field<R> b, Field<R> c, double* part) {
  typedef arith_t<R> A;
  const Tile t = tile_of(G);
  double sr = 0.0, si = 0.0, sc = 0.0;
  if (t.selected) {
    const bool with_c = c.ptr != nullptr;
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
      const SiteR<R> ar = site_r(a, t.rhs, 0, j, G.Vhp), br = site_r(b, t.rhs, 0, j, G.Vhp);
      SiteR<R> cr;
      if (with_c) cr = site_r(c, t.rhs, 0, j, G.Vhp);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cx<A> av = get(ar, k), bv = get(br, k);
        sr += (double)av.r * bv.r + (double)av.i * bv.i;
        si += (double)av.r * bv.i - (double)av.i * bv.r;
        if (with_c) {
          const cx<A> cv = get(cr, k);
          sc += (double)cv.r * cv.r + (double)cv.i * cv.i;
        }
      }
    }
  }
  block_sum3(sr, si, sc, part + 3 * (t.sys * G.nchunk + blockIdx.x));
}

template <class R>
__global__ __launch_bounds__(256) void k_bicg_p(SysGrid G, Field<R> p, Field<R> r, Field<R> v, const double* cs) {
  typedef arith_t<R> A;
  const Tile t = tile_of(G);
  if (!t.selected) return;
  const cx<double> be = cs_get(cs, t.sys, CS_BETA), om = cs_get(cs, t.sys, CS_OMEGA);
  const cx<A> b = {(A)be.r, (A)be.i}, w = {(A)om.r, (A)om.i};
  for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
    const SiteR<R> pr = site_r(p, t.rhs, 0, j, G.Vhp), rr = site_r(r, t.rhs, 0, j, G.Vhp);
    const SiteR<R> vr = site_r(v, t.rhs, 0, j, G.Vhp);
    SiteW<R> pw = site_w(p, t.rhs, 0, j, G.Vhp);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cx<A> d = get(pr, k) - cmul(w, get(vr, k));
      put(pw, k, get(rr, k) + cmul(b, d));
    }
    close(pw);
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_bicg_s(SysGrid G, Field<R> r, Field<R> v, const double* cs, double* part) {
  typedef arith_t<R> A;
  const Tile t = tile_of(G);
  double acc = 0.0;
  if (t.selected) {
    const cx<double> al = cs_get(cs, t.sys, CS_ALPHA);
    const cx<A> a = {(A)al.r, (A)al.i};
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
      const SiteR<R> rr = site_r(r, t.rhs, 0, j, G.Vhp), vr = site_r(v, t.rhs, 0, j, G.Vhp);
      SiteW<R> rw = site_w(r, t.rhs, 0, j, G.Vhp);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cx<A> sv = get(rr, k) - cmul(a, get(vr, k));
        put(rw, k, sv);
        acc += (double)sv.r * sv.r + (double)sv.i * sv.i;
      }
      close(rw);
    }
  }
  const double sm = block_sum(acc);
  if (threadIdx.x == 0) part[t.sys * G.nchunk + blockIdx.x] = sm;
}

template <class R>
__global__ __launch_bounds__(256) void k_bicg_xr(SysGrid G, Field<R> x, Field<R> p, Field<R> r, Field<R> tt,
                                                 Field<R> r0, const double* cs, double* part) {
  typedef arith_t<R> A;
  const Tile t = tile_of(G);
  double sr = 0.0, si = 0.0, sc = 0.0;
  if (t.selected) {
    const cx<double> al = cs_get(cs, t.sys, CS_ALPHA), om = cs_get(cs, t.sys, CS_OMEGA);
    const cx<A> a = {(A)al.r, (A)al.i}, w = {(A)om.r, (A)om.i};
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
      const SiteR<R> xr = site_r(x, t.rhs, 0, j, G.Vhp), pr = site_r(p, t.rhs, 0, j, G.Vhp);
      const SiteR<R> rr = site_r(r, t.rhs, 0, j, G.Vhp), tr = site_r(tt, t.rhs, 0, j, G.Vhp);
      const SiteR<R> qr = site_r(r0, t.rhs, 0, j, G.Vhp);
      SiteW<R> xw = site_w(x, t.rhs, 0, j, G.Vhp), rw = site_w(r, t.rhs, 0, j, G.Vhp);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cx<A> sv = get(rr, k), tv = get(tr, k);
        put(xw, k, get(xr, k) + cmul(a, get(pr, k)) + cmul(w, sv));
        const cx<A> rn = sv - cmul(w, tv);
        put(rw, k, rn);
        const cx<A> q = get(qr, k);
        sr += (double)q.r * rn.r + (double)q.i * rn.i;
        si += (double)q.r * rn.i - (double)q.i * rn.r;
        sc += (double)rn.r * rn.r + (double)rn.i * rn.i;
      }
      close(xw);
      close(rw);
    }
  }
  block_sum3(sr, si, sc, part + 3 * (t.sys * G.nchunk + blockIdx.x));
}

__device__ __forceinline__ void sys_total3(const double* part, long long sys, int nchunk, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  for (int c = 0; c < nchunk; ++c)
    for (int k = 0; k < 3; ++k) out[k] += part[3 * (sys * nchunk + c) + k];
}

// Close an iteration (init: start the solve): rho_new = <r0, r>, stop on ||r||^2 <= target2,
// beta = (rho_new / rho) (alpha / omega). A breakdown (|<r0, r>|^2 <= 1e-24 ||r0||^2 ||r||^2,
// a zero rho or omega, or ||r|| > 1e6 ||r0||) stops the system, which the defect-correction
// loop then restarts from its current solution.
__global__ void k_fin_bicg_rho(SysScal S, double* cs, int nsys, int nchunk, const double* part, const int* sel,
                               const double* target2, int init) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    double v[3];
    sys_total3(part, s, nchunk, v);
    const cx<double> rn = {v[0], v[1]};
    const double rr = v[2];
    if (!(isfinite(v[0]) && isfinite(v[1]) && isfinite(rr))) S.flags[0] = 4;
    int act;
    cx<double> rho, al, om;
    if (init) {
      act = sel[s] && rr > target2[s];
      rho = {1.0, 0.0};
      al = {1.0, 0.0};
      om = {1.0, 0.0};
    } else {
      act = S.active[s] && rr > target2[s];
      rho = cs_get(cs, s, CS_RHO);
      al = cs_get(cs, s, CS_ALPHA);
      om = cs_get(cs, s, CS_OMEGA);
    }
    S.ss[s] = rr;
    if (init) S.gam[s] = rr;   // ||r0||^2 (r0 = r at the start)
    const double rho2 = rho.r * rho.r + rho.i * rho.i, om2 = om.r * om.r + om.i * om.i;
    const double rn2 = rn.r * rn.r + rn.i * rn.i;
    // breakdown: <r0, r> (nearly) orthogonal, or a vanishing rho or omega; growth of the
    // residual beyond 1e6 ||r0|| (which would overflow FP32 iterates) stops the system too
    if (act && (rho2 == 0.0 || om2 == 0.0 || !(rn2 > 1e-24 * S.gam[s] * rr) || rr > 1e12 * S.gam[s])) act = 0;
    if (act) {
      cs_set(cs, s, CS_BETA, cmul(cdiv(rn, rho), cdiv(al, om)));
      cs_set(cs, s, CS_RHO, rn);
      cs_set(cs, s, CS_ALPHA, al);        // (1, 0) at the start, else unchanged
      cs_set(cs, s, CS_OMEGA, om);
    } else {
      const cx<double> z = {0.0, 0.0};
      cs_set(cs, s, CS_BETA, z);
      cs_set(cs, s, CS_ALPHA, z);
      cs_set(cs, s, CS_OMEGA, z);
    }
    S.active[s] = act;
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) S.flags[1] = cnt;
}

__global__ void k_fin_bicg_alpha(SysScal S, double* cs, int nsys, int nchunk, const double* part) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    double v[3];
    sys_total3(part, s, nchunk, v);
    if (!(isfinite(v[0]) && isfinite(v[1]))) S.flags[0] = 5;
    const cx<double> den = {v[0], v[1]};
    if (S.active[s] && (den.r != 0.0 || den.i != 0.0)) {
      cs_set(cs, s, CS_ALPHA, cdiv(cs_get(cs, s, CS_RHO), den));
    } else {
      cs_set(cs, s, CS_ALPHA, {0.0, 0.0});
      S.active[s] = 0;
    }
  }
}

// omega = <t, s> / ||t||^2. When ||s||^2 already meets the target the step ends with
// x += alpha p (omega = 0, r = s); when <t, s> (nearly) vanishes the system stops after
// that same update (breakdown, restarted by the defect-correction loop).
__global__ void k_fin_bicg_omega(SysScal S, double* cs, int nsys, int nchunk, const double* part, int nchunk_s,
                                 const double* part_s, const double* target2) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    double v[3];
    sys_total3(part, s, nchunk, v);
    const double ss = sys_total(part_s, s, nchunk_s);
    if (!(isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) && isfinite(ss))) S.flags[0] = 6;
    cx<double> om = {0.0, 0.0};
    if (S.active[s]) {
      S.iters[s] += 1;
      const double ts2 = v[0] * v[0] + v[1] * v[1];
      if (ss <= target2[s]) {
        // converged on s: omega stays 0
      } else if (v[2] > 0.0 && ts2 > 1e-24 * v[2] * ss) {
        om = {v[0] / v[2], v[1] / v[2]};
      } else {
        S.active[s] = 0;
      }
    }
    cs_set(cs, s, CS_OMEGA, om);
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_lin3(SysGrid G, Field<R> y, Field<R> u, Field<R> w, Field<R> q,
                                              const double* coef, double* part) {
  typedef arith_t<R> A;
  const Tile t = tile_of(G);
  double sr = 0.0, si = 0.0, sc = 0.0;
  if (t.selected) {
    const double* cf = coef + 6 * t.sys;
    const cx<A> c0 = {(A)cf[0], (A)cf[1]}, c1 = {(A)cf[2], (A)cf[3]}, c2 = {(A)cf[4], (A)cf[5]};
    const bool keep_y = cf[0] != 0.0 || cf[1] != 0.0;   // c0 = 0: y is not read (may be unset)
    const bool with_w = w.ptr != nullptr, with_q = q.ptr != nullptr;
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
      const SiteR<R> ur = site_r(u, t.rhs, 0, j, G.Vhp);
      SiteR<R> yr, wr, qr;
      if (keep_y) yr = site_r(y, t.rhs, 0, j, G.Vhp);
      if (with_w) wr = site_r(w, t.rhs, 0, j, G.Vhp);
      if (with_q) qr = site_r(q, t.rhs, 0, j, G.Vhp);
      SiteW<R> yw = site_w(y, t.rhs, 0, j, G.Vhp);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        cx<A> v = cmul(c1, get(ur, k));
        if (keep_y) v = v + cmul(c0, get(yr, k));
        if (with_w) v = v + cmul(c2, get(wr, k));
        put(yw, k, v);
        if (with_q) {
          const cx<A> qv = get(qr, k);
          sr += (double)qv.r * v.r + (double)qv.i * v.i;
          si += (double)qv.r * v.i - (double)qv.i * v.r;
        }
        sc += (double)v.r * v.r + (double)v.i * v.i;
      }
      close(yw);
    }
  }
  if (part) block_sum3(sr, si, sc, part + 3 * (t.sys * G.nchunk + blockIdx.x));
}

__global__ void k_fin_sum3(int nsys, int nchunk, const double* part, double* out) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    double v[3];
    sys_total3(part, s, nchunk, v);
    for (int k = 0; k < 3; ++k) out[3 * s + k] = v[k];
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_geom_add(SysGrid G, Field<R> x, Field<R> tf, const int* active) {
  const Tile t = tile_of(G);
  if (!t.selected || !active[t.sys]) return;
  for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256) {
    const SiteR<R> xr = site_r(x, t.rhs, 0, j, G.Vhp), tr = site_r(tf, t.rhs, 0, j, G.Vhp);
    SiteW<R> xw = site_w(x, t.rhs, 0, j, G.Vhp);
#pragma unroll
    for (int k = 0; k < 12; ++k) put(xw, k, get(xr, k) + get(tr, k));
    close(xw);
  }
}

// Geometric series: init marks the systems with ||t_0||^2 = ||b_hat||^2 above target
// (ss keeps it as the divergence reference); a later call stops a system once the new
// term satisfies ||t||^2 <= target2, and flags a divergence once ||t||^2 > 1e30 ||b_hat||^2.
__global__ void k_fin_geom(SysScal S, int nsys, int nchunk, const double* part, const int* sel,
                           const double* target2, int init) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    const double tt = sys_total(part, s, nchunk);
    if (!isfinite(tt)) S.flags[0] = 7;
    int act;
    if (init) {
      act = sel[s] && tt > target2[s];
      S.ss[s] = tt;
    } else {
      act = S.active[s];
      if (act) {
        S.iters[s] += 1;
        if (tt <= target2[s]) act = 0;
        else if (!(tt <= 1e30 * S.ss[s])) {
          S.flags[2] = 1;
          act = 0;
        }
      }
    }
    S.active[s] = act;
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) S.flags[1] = cnt;
}

// ---------------------------------------------------------------------------------
static inline dim3 grid_of(const SysGrid& G, int nrhs) { return dim3(G.nchunk, G.nblk, nrhs); }

template <class R> void blas_norm2(const SysGrid& G, int nrhs, Field<R> a, int npar, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2<R>, grid_of(G, nrhs), dim3(256), 0, s, G, a, npar, part);
}
template <class R> void blas_cg_s(const SysGrid& G, int nrhs, Field<R> sf, Field<R> q, const double* alpha,
                                  double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_s<R>, grid_of(G, nrhs), dim3(256), 0, s, G, sf, q, alpha, part);
}
template <class R> void blas_cg_xp(const SysGrid& G, int nrhs, Field<R> x, Field<R> p, Field<R> r,
                                   const double* alpha, const double* beta, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_xp<R>, grid_of(G, nrhs), dim3(256), 0, s, G, x, p, r, alpha, beta);
}
template <class Ro, class Ri> void blas_convert(const SysGrid& G, int nrhs, Field<Ro> out, Field<Ri> in,
                                                int npar, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<Ro, Ri>), grid_of(G, nrhs), dim3(256), 0, s, G, out, in, npar);
}
template <class R> void blas_add_mixed(const SysGrid& G, int nrhs, Field<double> x, Field<R> e, hipStream_t s) {
  hipLaunchKernelGGL(k_add_mixed<R>, grid_of(G, nrhs), dim3(256), 0, s, G, x, e);
}
void blas_resid(const SysGrid& G, int nrhs, Field<double> r, Field<double> b, Field<double> Ax, double* part,
                hipStream_t s, int npar) {
  hipLaunchKernelGGL(k_resid, grid_of(G, nrhs), dim3(256), 0, s, G, r, b, Ax, part, npar);
}
void fin_sum(int nsys, int nchunk, const double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_sum, dim3(1), dim3(256), 0, s, nsys, nchunk, part, out);
}
void fin_init(const SysScal& S, int nsys, int nchunk, const double* pb, const double* pr, const int* sel,
              const double* target2, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(256), 0, s, S, nsys, nchunk, pb, pr, sel, target2);
}
void fin_alpha(const SysScal& S, int nsys, int nchunk, const double* pq, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(256), 0, s, S, nsys, nchunk, pq);
}
void fin_beta(const SysScal& S, int nsys, int nchunk, const double* ps_, int nchunk_r, const double* pr,
              const double* target2, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(256), 0, s, S, nsys, nchunk, ps_, nchunk_r, pr, target2);
}

template <class R> void blas_cdot3(const SysGrid& G, int nrhs, Field<R> a, Field<R> b, Field<R> c, double* part,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_cdot3<R>, grid_of(G, nrhs), dim3(256), 0, s, G, a, b, c, part);
}
template <class R> void blas_bicg_p(const SysGrid& G, int nrhs, Field<R> p, Field<R> r, Field<R> v,
                                    const double* cs, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_p<R>, grid_of(G, nrhs), dim3(256), 0, s, G, p, r, v, cs);
}
template <class R> void blas_bicg_s(const SysGrid& G, int nrhs, Field<R> r, Field<R> v, const double* cs,
                                    double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_s<R>, grid_of(G, nrhs), dim3(256), 0, s, G, r, v, cs, part);
}
template <class R> void blas_bicg_xr(const SysGrid& G, int nrhs, Field<R> x, Field<R> p, Field<R> r,
                                     Field<R> t, Field<R> r0, const double* cs, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_xr<R>, grid_of(G, nrhs), dim3(256), 0, s, G, x, p, r, t, r0, cs, part);
}
void fin_bicg_rho(const SysScal& S, double* cs, int nsys, int nchunk, const double* part, const int* sel,
                  const double* target2, int init, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_bicg_rho, dim3(1), dim3(256), 0, s, S, cs, nsys, nchunk, part, sel, target2, init);
}
void fin_bicg_alpha(const SysScal& S, double* cs, int nsys, int nchunk, const double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_bicg_alpha, dim3(1), dim3(256), 0, s, S, cs, nsys, nchunk, part);
}
void fin_bicg_omega(const SysScal& S, double* cs, int nsys, int nchunk, const double* part, int nchunk_s,
                    const double* part_s, const double* target2, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_bicg_omega, dim3(1), dim3(256), 0, s, S, cs, nsys, nchunk, part, nchunk_s, part_s,
                     target2);
}
template <class R> void blas_geom_add(const SysGrid& G, int nrhs, Field<R> x, Field<R> t, const int* active,
                                      hipStream_t s) {
  hipLaunchKernelGGL(k_geom_add<R>, grid_of(G, nrhs), dim3(256), 0, s, G, x, t, active);
}
template <class R> void blas_lin3(const SysGrid& G, int nrhs, Field<R> y, Field<R> u, Field<R> w, Field<R> q,
                                  const double* coef, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_lin3<R>, grid_of(G, nrhs), dim3(256), 0, s, G, y, u, w, q, coef, part);
}
void fin_sum3(int nsys, int nchunk, const double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_sum3, dim3(1), dim3(256), 0, s, nsys, nchunk, part, out);
}
void fin_geom(const SysScal& S, int nsys, int nchunk, const double* part, const int* sel, const double* target2,
              int init, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_geom, dim3(1), dim3(256), 0, s, S, nsys, nchunk, part, sel, target2, init);
}

#define INST(R)                                                                                         \
  template void blas_norm2<R>(const SysGrid&, int, Field<R>, int, double*, hipStream_t);                 \
  template void blas_cg_s<R>(const SysGrid&, int, Field<R>, Field<R>, const double*, double*, hipStream_t); \
  template void blas_cg_xp<R>(const SysGrid&, int, Field<R>, Field<R>, Field<R>, const double*,           \
                              const double*, hipStream_t);                                               \
  template void blas_add_mixed<R>(const SysGrid&, int, Field<double>, Field<R>, hipStream_t);           \
  template void blas_cdot3<R>(const SysGrid&, int, Field<R>, Field<R>, Field<R>, double*, hipStream_t);  \
  template void blas_bicg_p<R>(const SysGrid&, int, Field<R>, Field<R>, Field<R>, const double*, hipStream_t); \
  template void blas_bicg_s<R>(const SysGrid&, int, Field<R>, Field<R>, const double*, double*, hipStream_t); \
  template void blas_bicg_xr<R>(const SysGrid&, int, Field<R>, Field<R>, Field<R>, Field<R>, Field<R>,   \
                                const double*, double*, hipStream_t);                                    \
  template void blas_geom_add<R>(const SysGrid&, int, Field<R>, Field<R>, const int*, hipStream_t);      \
  template void blas_lin3<R>(const SysGrid&, int, Field<R>, Field<R>, Field<R>, Field<R>, const double*,  \
                             double*, hipStream_t);
INST(double)
INST(float)
INST(h16)
template void blas_convert<double, double>(const SysGrid&, int, Field<double>, Field<double>, int, hipStream_t);
template void blas_convert<float, double>(const SysGrid&, int, Field<float>, Field<double>, int, hipStream_t);
template void blas_convert<h16, double>(const SysGrid&, int, Field<h16>, Field<double>, int, hipStream_t);

}  // namespace sap
