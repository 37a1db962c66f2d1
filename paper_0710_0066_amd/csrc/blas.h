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
  long long Vhp;     // storage sites per parity (locates the site norms of FP16 fields)
};

// Per-system scalars of the CG iteration (device arrays of nsys entries) and flags:
// flags[0] = non-finite value seen (the code of the finalize kernel that saw it: 1 CG init,
// 2 CG alpha, 3 CG beta, 4 BiCGstab rho, 5 BiCGstab alpha, 6 BiCGstab omega, 7 series),
// flags[1] = number of active systems, flags[2] = a geometric series diverged.
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
  G.Vhp = (Vh + TILE - 1) / TILE * TILE;
  return G;
}

template <class R> void blas_norm2(const SysGrid& G, int nrhs, Field<R> a, int npar, double* part, hipStream_t s);
// s -= alpha q with partial ||s||^2 per system
template <class R> void blas_cg_s(const SysGrid& G, int nrhs, Field<R> sf, Field<R> q, const double* alpha,
                                  double* part, hipStream_t s);
// x += alpha p, then p = r + beta p
template <class R> void blas_cg_xp(const SysGrid& G, int nrhs, Field<R> x, Field<R> p, Field<R> r,
                                   const double* alpha, const double* beta, hipStream_t s);
template <class Ro, class Ri> void blas_convert(const SysGrid& G, int nrhs, Field<Ro> out, Field<Ri> in,
                                                int npar, hipStream_t s);
template <class R> void blas_add_mixed(const SysGrid& G, int nrhs, Field<double> x, Field<R> e, hipStream_t s);
// r = b - Ax over the first npar parities (2: both; 1: the even sites), partial ||r||^2
void blas_resid(const SysGrid& G, int nrhs, Field<double> r, Field<double> b, Field<double> Ax, double* part,
                hipStream_t s, int npar = 2);
void fin_sum(int nsys, int nchunk, const double* part, double* out, hipStream_t s);
void fin_init(const SysScal& S, int nsys, int nchunk, const double* pb, const double* pr, const int* sel,
              const double* target2, hipStream_t s);
void fin_alpha(const SysScal& S, int nsys, int nchunk, const double* pq, hipStream_t s);
// ps_ holds nchunk partials per system, pr nchunk_r
void fin_beta(const SysScal& S, int nsys, int nchunk, const double* ps_, int nchunk_r, const double* pr,
              const double* target2, hipStream_t s);

// ---- BiCGstab on the even-odd system: complex per-system scalars in cs[8 * sys] =
// (rho, alpha, omega, beta) as (re, im) pairs; partials hold three values per
// (system, chunk): re <a, b>, im <a, b>, ||c||^2.
template <class R> void blas_cdot3(const SysGrid& G, int nrhs, Field<R> a, Field<R> b, Field<R> c, double* part,
                                   hipStream_t s);
// p = r + beta (p - omega v)
template <class R> void blas_bicg_p(const SysGrid& G, int nrhs, Field<R> p, Field<R> r, Field<R> v,
                                    const double* cs, hipStream_t s);
// s = r - alpha v (into r), partial ||s||^2 (one per chunk)
template <class R> void blas_bicg_s(const SysGrid& G, int nrhs, Field<R> r, Field<R> v, const double* cs,
                                    double* part, hipStream_t s);
// x += alpha p + omega s ; r = s - omega t (s is held in r) ; partials <r0, r>, ||r||^2
template <class R> void blas_bicg_xr(const SysGrid& G, int nrhs, Field<R> x, Field<R> p, Field<R> r,
                                     Field<R> t, Field<R> r0, const double* cs, double* part, hipStream_t s);
// start (init) or close an iteration: rho_new = <r0, r>, convergence on ||r||^2, beta
void fin_bicg_rho(const SysScal& S, double* cs, int nsys, int nchunk, const double* part, const int* sel,
                  const double* target2, int init, hipStream_t s);
void fin_bicg_alpha(const SysScal& S, double* cs, int nsys, int nchunk, const double* part, hipStream_t s);
// part: nchunk triples per system (<t, s>, ||t||^2), part_s: nchunk_s partials of ||s||^2
void fin_bicg_omega(const SysScal& S, double* cs, int nsys, int nchunk, const double* part, int nchunk_s,
                    const double* part_s, const double* target2, hipStream_t s);

// y = c0 y + c1 u + c2 w (w.ptr may be null; y is not read when c0 = 0) with complex
// per-system coefficients
// coef[6 * sys] = (c0, c1, c2); if part: partials <q, y>, ||y||^2 (three per chunk)
template <class R> void blas_lin3(const SysGrid& G, int nrhs, Field<R> y, Field<R> u, Field<R> w, Field<R> q,
                                  const double* coef, double* part, hipStream_t s);
// out[3 * sys + k] = sum over the chunks of the three partials
void fin_sum3(int nsys, int nchunk, const double* part, double* out, hipStream_t s);

// ---- geometric series: x += t on active systems; start / close an iteration on ||t||^2
// (flags[2] = 1 when a series diverges)
template <class R> void blas_geom_add(const SysGrid& G, int nrhs, Field<R> x, Field<R> t, const int* active,
                                      hipStream_t s);
void fin_geom(const SysScal& S, int nsys, int nchunk, const double* part, const int* sel, const double* target2,
              int init, hipStream_t s);

}  // namespace sap
