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
    for (int p = 0; p < npar; ++p) {
      const typename vec2<R>::type* base = a.ptr + t.rhs * a.rs + p * a.ps;
      for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256)
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          cx<R> v = ld<R>(base + tiled(j, c, 12));
          acc += (double)v.r * v.r + (double)v.i * v.i;
        }
    }
  }
  double s = block_sum(acc);
  if (threadIdx.x == 0) part[t.sys * G.nchunk + blockIdx.x] = s;
}

// x += alpha p ; s -= alpha q ; partial ||s||^2
template <class R>
__global__ __launch_bounds__(256) void k_cg_xs(SysGrid G, Field<R> x, Field<R> p, Field<R> s,
                                               Field<R> q, const double* alpha, double* part) {
  const Tile t = tile_of(G);
  double acc = 0.0;
  if (t.selected) {
    const R al = (R)alpha[t.sys];
    typename vec2<R>::type* xb = x.ptr + t.rhs * x.rs;
    const typename vec2<R>::type* pb = p.ptr + t.rhs * p.rs;
    typename vec2<R>::type* sb = s.ptr + t.rhs * s.rs;
    const typename vec2<R>::type* qb = q.ptr + t.rhs * q.rs;
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256)
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const long long o = tiled(j, c, 12);
        cx<R> xv = ld<R>(xb + o), pv = ld<R>(pb + o), sv = ld<R>(sb + o), qv = ld<R>(qb + o);
        xv.r += al * pv.r; xv.i += al * pv.i;
        sv.r -= al * qv.r; sv.i -= al * qv.i;
        st<R>(xb + o, xv);
        st<R>(sb + o, sv);
        acc += (double)sv.r * sv.r + (double)sv.i * sv.i;
      }
  }
  double sm = block_sum(acc);
  if (threadIdx.x == 0) part[t.sys * G.nchunk + blockIdx.x] = sm;
}

// p = r + beta p
template <class R>
__global__ __launch_bounds__(256) void k_xpay(SysGrid G, Field<R> p, Field<R> r, const double* beta) {
  const Tile t = tile_of(G);
  if (!t.selected) return;
  const R be = (R)beta[t.sys];
  typename vec2<R>::type* pb = p.ptr + t.rhs * p.rs;
  const typename vec2<R>::type* rb = r.ptr + t.rhs * r.rs;
  for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256)
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const long long o = tiled(j, c, 12);
      cx<R> pv = ld<R>(pb + o), rv = ld<R>(rb + o);
      pv.r = rv.r + be * pv.r;
      pv.i = rv.i + be * pv.i;
      st<R>(pb + o, pv);
    }
}

// out = src (both parities if npar == 2), converting precision
template <class Ro, class Ri>
__global__ __launch_bounds__(256) void k_convert(SysGrid G, Field<Ro> out, Field<Ri> in, int npar) {
  const Tile t = tile_of(G);
  for (int p = 0; p < npar; ++p) {
    typename vec2<Ro>::type* ob = out.ptr + t.rhs * out.rs + p * out.ps;
    const typename vec2<Ri>::type* ib = in.ptr + t.rhs * in.rs + p * in.ps;
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256)
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const long long o = tiled(j, c, 12);
        cx<Ri> v = ld<Ri>(ib + o);
        cx<Ro> w = {(Ro)v.r, (Ro)v.i};
        if (!t.selected) w = {Ro(0), Ro(0)};
        st<Ro>(ob + o, w);
      }
  }
}

// x64 += e (both parities), e at the inner precision
template <class R>
__global__ __launch_bounds__(256) void k_add_mixed(SysGrid G, Field<double> x, Field<R> e) {
  const Tile t = tile_of(G);
  if (!t.selected) return;
  for (int p = 0; p < 2; ++p) {
    double2* xb = x.ptr + t.rhs * x.rs + p * x.ps;
    const typename vec2<R>::type* eb = e.ptr + t.rhs * e.rs + p * e.ps;
    for (long long j = t.j0 + threadIdx.x; j < t.j1; j += 256)
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const long long o = tiled(j, c, 12);
        cx<double> xv = ld<double>(xb + o);
        cx<R> ev = ld<R>(eb + o);
        xv.r += (double)ev.r;
        xv.i += (double)ev.i;
        st<double>(xb + o, xv);
      }
  }
}

// r = b - Ax (FP64, both parities), partial ||r||^2
__global__ __launch_bounds__(256) void k_resid(SysGrid G, Field<double> r, Field<double> b,
                                               Field<double> Ax, double* part) {
  const Tile t = tile_of(G);
  double acc = 0.0;
  for (int p = 0; p < 2; ++p) {
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
    if (!isfinite(qq)) S.flags[0] = 1;
    S.alpha[s] = (S.active[s] && qq > 0.0) ? S.gam[s] / qq : 0.0;
  }
}

__global__ void k_fin_beta(SysScal S, int nsys, int nchunk, const double* part_s, const double* part_r,
                           const double* target2) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    const double ss = sys_total(part_s, s, nchunk);
    const double gm = sys_total(part_r, s, nchunk);
    if (!(isfinite(ss) && isfinite(gm))) S.flags[0] = 1;
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

// ---------------------------------------------------------------------------------
static inline dim3 grid_of(const SysGrid& G, int nrhs) { return dim3(G.nchunk, G.nblk, nrhs); }

template <class R> void blas_norm2(const SysGrid& G, int nrhs, Field<R> a, int npar, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2<R>, grid_of(G, nrhs), dim3(256), 0, s, G, a, npar, part);
}
template <class R> void blas_cg_xs(const SysGrid& G, int nrhs, Field<R> x, Field<R> p, Field<R> sf,
                                   Field<R> q, const double* alpha, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_xs<R>, grid_of(G, nrhs), dim3(256), 0, s, G, x, p, sf, q, alpha, part);
}
template <class R> void blas_xpay(const SysGrid& G, int nrhs, Field<R> p, Field<R> r, const double* beta,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_xpay<R>, grid_of(G, nrhs), dim3(256), 0, s, G, p, r, beta);
}
template <class Ro, class Ri> void blas_convert(const SysGrid& G, int nrhs, Field<Ro> out, Field<Ri> in,
                                                int npar, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<Ro, Ri>), grid_of(G, nrhs), dim3(256), 0, s, G, out, in, npar);
}
template <class R> void blas_add_mixed(const SysGrid& G, int nrhs, Field<double> x, Field<R> e, hipStream_t s) {
  hipLaunchKernelGGL(k_add_mixed<R>, grid_of(G, nrhs), dim3(256), 0, s, G, x, e);
}
void blas_resid(const SysGrid& G, int nrhs, Field<double> r, Field<double> b, Field<double> Ax, double* part,
                hipStream_t s) {
  hipLaunchKernelGGL(k_resid, grid_of(G, nrhs), dim3(256), 0, s, G, r, b, Ax, part);
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
void fin_beta(const SysScal& S, int nsys, int nchunk, const double* ps_, const double* pr,
              const double* target2, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(256), 0, s, S, nsys, nchunk, ps_, pr, target2);
}

#define INST(R)                                                                                         \
  template void blas_norm2<R>(const SysGrid&, int, Field<R>, int, double*, hipStream_t);                 \
  template void blas_cg_xs<R>(const SysGrid&, int, Field<R>, Field<R>, Field<R>, Field<R>, const double*, \
                              double*, hipStream_t);                                                     \
  template void blas_xpay<R>(const SysGrid&, int, Field<R>, Field<R>, const double*, hipStream_t);       \
  template void blas_add_mixed<R>(const SysGrid&, int, Field<double>, Field<R>, hipStream_t);
INST(double)
INST(float)
template void blas_convert<double, double>(const SysGrid&, int, Field<double>, Field<double>, int, hipStream_t);
template void blas_convert<float, double>(const SysGrid&, int, Field<float>, Field<double>, int, hipStream_t);

}  // namespace sap
