// Declarations of the BLAS-1 / reduction launchers (blas.hip) used by the solvers.
#pragma once
#include "internal.h"

namespace sap {

constexpr int CHUNK = 1024;   // sites of one parity per workgroup in the BLAS kernels

// Systems of a batched solve: nblk x0 blocks of Vb sites per parity (nblk = 1, Vb = Vh
// for the full lattice), selection of the blocks (block_selected code: 0 all, 1 black,
// 2 white, 3 + b block b).
struct SysGrid {
  int nblk;
  long long Vb;
  int nchunk;       // ceil(Vb / CHUNK)
  int colour;
  long long Vh;
};

// Per-system scalars of the CG iteration (device arrays of nsys entries) and flags:
// flags[0] = non-finite value seen, flags[1] = number of active systems.
struct SysScal {
  double *gam, *ss, *alpha, *beta;
  int *active, *iters, *flags;
};

inline SysGrid make_sysgrid(long long Vh, int V3h, int lb, int L0, int colour) {
  SysGrid G;
  G.nblk = lb ? L0 / lb : 1;
  G.Vb = lb ? (long long)lb * V3h : Vh;
  G.nchunk = (int)((G.Vb + CHUNK - 1) / CHUNK);
  G.colour = lb ? colour : 0;
  G.Vh = Vh;
  return G;
}

template <class R> void blas_norm2(const SysGrid& G, int nrhs, Field<R> a, int npar, double* part, hipStream_t s);
template <class R> void blas_cg_xs(const SysGrid& G, int nrhs, Field<R> x, Field<R> p, Field<R> sf, Field<R> q,
                                   const double* alpha, double* part, hipStream_t s);
template <class R> void blas_xpay(const SysGrid& G, int nrhs, Field<R> p, Field<R> r, const double* beta,
                                  hipStream_t s);
template <class Ro, class Ri> void blas_convert(const SysGrid& G, int nrhs, Field<Ro> out, Field<Ri> in,
                                                int npar, hipStream_t s);
template <class R> void blas_add_mixed(const SysGrid& G, int nrhs, Field<double> x, Field<R> e, hipStream_t s);
void blas_resid(const SysGrid& G, int nrhs, Field<double> r, Field<double> b, Field<double> Ax, double* part,
                hipStream_t s);
void fin_sum(int nsys, int nchunk, const double* part, double* out, hipStream_t s);
void fin_init(const SysScal& S, int nsys, int nchunk, const double* pb, const double* pr, const int* sel,
              const double* target2, hipStream_t s);
void fin_alpha(const SysScal& S, int nsys, int nchunk, const double* pq, hipStream_t s);
void fin_beta(const SysScal& S, int nsys, int nchunk, const double* ps_, const double* pr,
              const double* target2, hipStream_t s);

}  // namespace sap
