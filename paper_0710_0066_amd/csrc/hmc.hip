// Host drivers of the pseudo-fermion forces, the Schwarz boundary term and the HMC
// trajectory (Sec. 1: factorised pseudo-fermion action with W1 and the black-block
// boundary operator; Sec. 2: T_U / T_P steps, leap-frog and Sexton-Weingarten levels
// nested on two time scales; Metropolis).
//
// Schwarz term (Omega = black x0 blocks, Omega* = white; Pi = (1 - g0)/2 on the first and
// (1 + g0)/2 on the last slice of every black block):
//   D_dOm* = P_Om* M P_Om,  D_dOm = P_Om M P_Om*,
//   heat bath   chi = R_hat Pi g = Pi g - Pi W1^{-1}|_Om D_dOm W1^{-1}|_Om* D_dOm* Pi g,
//   action      S_R = ||eta||^2,  eta = chi - Pi psi,  psi = M^{-1} D_dOm* chi,
//   force       F = 2 Re <xi, dM psi> - 2 Re <P_Om* xi, dM chi>,  xi = M^{-dagger} Pi eta,
// with M^{-dagger} = g5 M^{-1} g5 and W1^{-dagger} = g5 W1^{-1} g5.
#include <cmath>
#include <cstring>
#include "force.h"

using namespace sap;

int sap_solve_any(sap_ctx* c, double* x, const double* b, int nrhs, int lb, int colour,
                  const sap_solve_opts* o, sap_solve_info* info, hipStream_t st);
int sap_solve_eo_shift(sap_ctx* c, double* x, const double* b, int nrhs, int lb, double rho,
                       const sap_solve_opts* o, sap_solve_info* info, hipStream_t st);

// Scratch fields: pf_force f[0..2]; schwarz_terms, heat_bath and check_chi f[3..6]; the
// even-odd terms f[0..4], their heat baths f[4..6]. The trajectories keep phi1 in f[7] and
// chi (the level-1 Schwarz field) in f[8]; the four-part trajectory also phi2 in f[9] and
// chi3 in f[10]; f[11] stages the heat-bath noise.
struct ForceWS {
  double2* f[12];      // full FP64 spinor fields of one rhs
  double* mom;         // momenta (sap layout)
  double* part;        // reduction partials (one per 128-site tile pair)
  double* scal;        // device scalars
  double* h_scal;      // pinned host mirror
  double* sx;          // per-link step scale s_mu(x0), [L0][4]
  double2* Utmp;       // gauge field scratch (translations)
  double* prof;        // force profile: partials (2 * L0 * nck) then the result (2 * L0)
  long long iters;     // inner iterations accumulated by the drivers below
};

static ForceWS* fws(sap_ctx* c) { return (ForceWS*)c->forces; }

int sap_force_create(sap_ctx* c) {
  ForceWS* w = new ForceWS();
  std::memset(w, 0, sizeof(*w));
  c->forces = w;
  const size_t fb = (size_t)24 * c->Vhp * sizeof(double2);
  bool ok = true;
  for (int i = 0; i < 12; ++i) ok = ok && hipMalloc((void**)&w->f[i], fb) == hipSuccess;
  ok = ok && hipMalloc((void**)&w->mom, (size_t)64 * c->Vhp * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&w->part, (size_t)((c->Vh + 127) / 128 + 8) * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&w->scal, 64 * 8) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&w->h_scal, 64 * 8, 0) == hipSuccess;
  ok = ok && hipMalloc((void**)&w->sx, (size_t)c->geom.L[0] * 4 * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&w->Utmp, (size_t)72 * c->Vhp * sizeof(double2)) == hipSuccess;
  ok = ok && hipMalloc((void**)&w->prof, (size_t)2 * c->geom.L[0] * (force_profile_nck(c->g) + 1) * 8) ==
                 hipSuccess;
  if (!ok) return sap_fail(c, SAP_E_NOMEM, "cannot allocate the force workspace");
  for (int i = 0; i < 12; ++i) (void)hipMemset(w->f[i], 0, fb);
  return SAP_OK;
}

void sap_force_destroy(sap_ctx* c) {
  ForceWS* w = fws(c);
  if (!w) return;
  for (int i = 0; i < 12; ++i)
    if (w->f[i]) (void)hipFree(w->f[i]);
  if (w->mom) (void)hipFree(w->mom);
  if (w->part) (void)hipFree(w->part);
  if (w->scal) (void)hipFree(w->scal);
  if (w->h_scal) (void)hipHostFree(w->h_scal);
  if (w->sx) (void)hipFree(w->sx);
  if (w->Utmp) (void)hipFree(w->Utmp);
  if (w->prof) (void)hipFree(w->prof);
  delete w;
  c->forces = nullptr;
}

namespace {

// |f|^2 of one full FP64 field, read back to the host (synchronises)
int norm2_host(sap_ctx* c, const double2* f, double* out, hipStream_t s) {
  ForceWS* w = fws(c);
  launch_norm2_full(c->g, f, w->part, w->scal, s);
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_scal, w->scal, 8, hipMemcpyDeviceToHost, s));
  SAP_HIP_CHECK(c, hipStreamSynchronize(s));
  *out = w->h_scal[0];
  return SAP_OK;
}

// out = A in on the sites of the selected colour of the inner blocks, 0 elsewhere, with
// A = M (outer = 0) or W_outer
void hop_sel(sap_ctx* c, double2* out, const double2* in, int colour, int outer, int inner, hipStream_t s) {
  HopArgs<double> A;
  const long long Vhp = c->Vhp;
  A.out = {out, 24 * Vhp, 12 * Vhp};
  A.in = {(double2*)in, 24 * Vhp, 12 * Vhp};
  A.x = A.in;
  A.U = gauge_of<double>(c);
  A.g = c->g;
  A.nrhs = 1;
  A.parity_out = -1;
  A.lb = outer;
  A.slb = inner;
  A.colour = colour;
  A.block = -1;
  A.a = 1.0;
  A.b = -c->geom.kappa;
  A.g5_in = A.g5_out = 0;
  A.map = HOP_MAP_SITE;
  launch_hop<double>(A, s);
}

// options for a solve of a block (lb > 0) or even-site system: SAP_SAP_BICGSTAB, which
// solves M x = b only, becomes even-odd BiCGstab with the same tolerances
const sap_solve_opts* sub_opts(const sap_solve_opts* o, sap_solve_opts* tmp) {
  if (o->method != SAP_SAP_BICGSTAB) return o;
  *tmp = *o;
  tmp->method = SAP_BICGSTAB;
  return tmp;
}

int solve1(sap_ctx* c, double2* x, const double2* b, int lb, int colour, const sap_solve_opts* o,
           hipStream_t s) {
  sap_solve_opts tmp;
  if (lb) o = sub_opts(o, &tmp);
  sap_solve_info inf[64];
  const int nsys = lb ? c->geom.L[0] / lb : 1;
  sap_solve_info* ip = nsys <= 64 ? inf : nullptr;
  int rc = sap_solve_any(c, (double*)x, (const double*)b, 1, lb, colour, o, ip, s);
  if (ip)
    for (int i = 0; i < nsys; ++i) fws(c)->iters += inf[i].iters;
  return rc;
}

int check_opts(sap_ctx* c, const sap_solve_opts* o) { return check_solve_opts(c, o); }

int pf_force(sap_ctx* c, double* F, double coef, const double2* phi, const sap_solve_opts* o, double* S,
             hipStream_t s, const double* sx = nullptr) {
  ForceWS* w = fws(c);
  const int l0 = c->geom.l0;
  double2 *X = w->f[0], *T = w->f[1], *Y = w->f[2];
  int rc = solve1(c, X, phi, l0, SAP_ALL, o, s);                 // X = W1^{-1} phi
  if (rc) return rc;
  if (S && (rc = norm2_host(c, X, S, s))) return rc;
  launch_spin_op(c->g, 0, l0, T, X, nullptr, s);                 // Y = g5 W1^{-1} g5 X
  if ((rc = solve1(c, Y, T, l0, SAP_ALL, o, s))) return rc;
  launch_spin_op(c->g, 0, l0, Y, Y, nullptr, s);
  // F += coef * (-2 Re <Y, dW1 X>)
  launch_pair_force(c->g, F, c->geom.kappa * coef, Y, X, c->U64, l0, s, sx);
  SAP_HIP_CHECK(c, hipGetLastError());
  return SAP_OK;
}

// Schwarz term of the outer operator A over its inner blocks: A = M with the level-1
// blocks (outer = 0, the factor det^2(M W1^-1)), or A = W1 with the level-2 blocks
// (outer = l0, the factor det^2(W1 W2^-1) of the four-part action).
int inner_of(sap_ctx* c, int outer) { return outer ? c->geom.l0_sub : c->geom.l0; }

int schwarz_terms(sap_ctx* c, double* F, double coef, const double2* chi, const sap_solve_opts* o,
                  double* S_R, hipStream_t s, const double* sx = nullptr, int outer = 0) {
  ForceWS* w = fws(c);
  const int l0 = inner_of(c, outer);
  double2 *v = w->f[3], *psi = w->f[4], *eta = w->f[5], *t = w->f[6];
  hop_sel(c, v, chi, SAP_WHITE, outer, l0, s);                   // v = D_dOm* chi
  int rc = solve1(c, psi, v, outer, SAP_ALL, o, s);              // psi = A^{-1} v
  if (rc) return rc;
  launch_spin_op(c->g, 3, l0, eta, chi, psi, s, outer);          // eta = chi - Pi psi
  if (S_R && (rc = norm2_host(c, eta, S_R, s))) return rc;
  if (!F) return SAP_OK;
  launch_spin_op(c->g, 1, l0, t, eta, nullptr, s, outer);        // t = g5 Pi eta
  launch_spin_op(c->g, 0, l0, t, t, nullptr, s);
  if ((rc = solve1(c, v, t, outer, SAP_ALL, o, s))) return rc;   // xi = g5 A^{-1} g5 Pi eta
  launch_spin_op(c->g, 0, l0, v, v, nullptr, s);
  launch_pair_force(c->g, F, -c->geom.kappa * coef, v, psi, c->U64, outer, s, sx);
  launch_spin_op(c->g, 2, l0, t, v, nullptr, s);                 // P_Om* xi
  launch_pair_force(c->g, F, c->geom.kappa * coef, t, chi, c->U64, outer, s, sx);
  SAP_HIP_CHECK(c, hipGetLastError());
  return SAP_OK;
}

int heat_bath(sap_ctx* c, double2* chi, const double2* g, const sap_solve_opts* o, hipStream_t s, int outer = 0) {
  ForceWS* w = fws(c);
  const int l0 = inner_of(c, outer);
  double2 *pg = w->f[3], *v = w->f[4], *x = w->f[5], *u = w->f[6];
  launch_spin_op(c->g, 1, l0, pg, g, nullptr, s, outer);         // Pi g
  hop_sel(c, v, pg, SAP_WHITE, outer, l0, s);                    // D_dOm* Pi g
  int rc = solve1(c, x, v, l0, SAP_WHITE, o, s);                 // white-block solves
  if (rc) return rc;
  hop_sel(c, u, x, SAP_BLACK, outer, l0, s);                     // D_dOm (x vanishes on black)
  if ((rc = solve1(c, v, u, l0, SAP_BLACK, o, s))) return rc;    // black-block solves
  launch_spin_op(c->g, 3, l0, chi, pg, v, s, outer);             // chi = Pi g - Pi z
  SAP_HIP_CHECK(c, hipGetLastError());
  return SAP_OK;
}

int check_chi(sap_ctx* c, const double2* chi, hipStream_t s, int outer = 0) {
  ForceWS* w = fws(c);
  double n_chi = 0, n_off = 0;
  int rc = norm2_host(c, chi, &n_chi, s);
  if (rc) return rc;
  launch_spin_op(c->g, 3, inner_of(c, outer), w->f[6], chi, chi, s, outer);   // chi - Pi chi
  if ((rc = norm2_host(c, w->f[6], &n_off, s))) return rc;
  if (!(n_off <= 1e-24 * n_chi))
    return sap_fail(c, SAP_E_ARG, "chi is not supported on the black-block boundaries in the range of Pi");
  return SAP_OK;
}

// ---- even-odd pseudo-fermion terms of the four-part action (level-2 blocks) ----------
// W2eo = 1 - k^2 D_eo D_oe on the even sites with the hops of the level-2 blocks, W3eo =
// W2eo + rho. kind 1: S1 = ||W3eo^-1 phi||^2; kind 2: S2 = ||phi + rho W2eo^-1 phi||^2.
// The force uses dW_eo = -k^2 P_e (dD P_o D + D P_o dD) P_e:
//   S1: X = W3eo^-1 phi, Z = W3eo^-dag X, F = -k [pf(Z, P_o D X) + pf(P_o D^dag Z, X)]
//   S2: Y = W2eo^-1 phi, X = phi + rho Y, Z = W2eo^-dag X, F = -rho k [pf(Z, P_o D Y) + pf(P_o D^dag Z, Y)]
// where pf(a, b) = 2 Re <a, dW b> is what launch_pair_force adds with the factor -c / k.

// out = P_o D in (g5: P_o D^dag in = P_o g5 D g5 in); the even half of out is zeroed
int hop_odd(sap_ctx* c, double2* out, const double2* in, bool dag, hipStream_t s) {
  const long long Vhp = c->Vhp;
  SAP_HIP_CHECK(c, hipMemsetAsync(out, 0, (size_t)12 * Vhp * sizeof(double2), s));
  HopArgs<double> A;
  A.out = {out, 24 * Vhp, 12 * Vhp};
  A.in = {(double2*)in, 24 * Vhp, 12 * Vhp};
  A.x = {nullptr, 0, 0};
  A.U = gauge_of<double>(c); A.g = c->g; A.nrhs = 1; A.parity_out = 1;
  A.lb = c->geom.l0_sub; A.slb = 0; A.colour = 0; A.block = -1;
  A.a = 0.0; A.b = 1.0; A.g5_in = A.g5_out = dag ? 1 : 0; A.map = HOP_MAP_SITE;
  launch_hop<double>(A, s);
  return SAP_OK;
}

// out = (W2eo + rho) in for an even-site field; the odd half of out is zeroed (tmp: scratch)
int apply_weo(sap_ctx* c, double2* out, const double2* in, double rho, double2* tmp, hipStream_t s) {
  int rc = hop_odd(c, tmp, in, false, s);
  if (rc) return rc;
  const long long Vhp = c->Vhp;
  SAP_HIP_CHECK(c, hipMemsetAsync(out + 12 * Vhp, 0, (size_t)12 * Vhp * sizeof(double2), s));
  HopArgs<double> A;
  A.out = {out, 24 * Vhp, 12 * Vhp};
  A.in = {tmp, 24 * Vhp, 12 * Vhp};
  A.x = {(double2*)in, 24 * Vhp, 12 * Vhp};
  A.U = gauge_of<double>(c); A.g = c->g; A.nrhs = 1; A.parity_out = 0;
  A.lb = c->geom.l0_sub; A.slb = 0; A.colour = 0; A.block = -1;
  const double k = c->geom.kappa;
  A.a = 1.0 + rho; A.b = -k * k; A.g5_in = A.g5_out = 0; A.map = HOP_MAP_SITE;
  launch_hop<double>(A, s);
  SAP_HIP_CHECK(c, hipGetLastError());
  return SAP_OK;
}

int solve_eo1(sap_ctx* c, double2* x, const double2* b, double rho, const sap_solve_opts* o, hipStream_t s) {
  sap_solve_opts tmp;
  o = sub_opts(o, &tmp);
  sap_solve_info inf[64];
  const int nsys = c->geom.L[0] / c->geom.l0_sub;
  sap_solve_info* ip = nsys <= 64 ? inf : nullptr;
  int rc = sap_solve_eo_shift(c, (double*)x, (const double*)b, 1, c->geom.l0_sub, rho, o, ip, s);
  if (ip)
    for (int i = 0; i < nsys; ++i) fws(c)->iters += inf[i].iters;
  return rc;
}

int eo_pf_terms(sap_ctx* c, double* F, double coef, const double2* phi, int kind, double rho,
                const sap_solve_opts* o, double* S, hipStream_t s, const double* sx = nullptr) {
  ForceWS* w = fws(c);
  double2 *X = w->f[0], *Y = w->f[1], *Z = w->f[2], *T = w->f[3], *T2 = w->f[4];
  int rc;
  const double2* B;          // the field the second factor of dW acts on (X for S1, Y for S2)
  if (kind == 1) {
    if ((rc = solve_eo1(c, X, phi, rho, o, s))) return rc;                  // X = W3eo^-1 phi
    B = X;
  } else {
    if ((rc = solve_eo1(c, Y, phi, 0.0, o, s))) return rc;                  // Y = W2eo^-1 phi
    launch_lincomb(c->g, X, 1.0, phi, rho, Y, s);                          // X = phi + rho Y
    B = Y;
  }
  if (S && (rc = norm2_host(c, X, S, s))) return rc;
  if (!F) return SAP_OK;
  const double rz = kind == 1 ? rho : 0.0;
  launch_spin_op(c->g, 0, c->geom.l0, T, X, nullptr, s);                   // Z = g5 W^-1 g5 X
  if ((rc = solve_eo1(c, Z, T, rz, o, s))) return rc;
  launch_spin_op(c->g, 0, c->geom.l0, Z, Z, nullptr, s);
  if ((rc = hop_odd(c, T, B, false, s)) || (rc = hop_odd(c, T2, Z, true, s))) return rc;
  const double k = c->geom.kappa;
  const double cf = coef * k * k * (kind == 1 ? 1.0 : rho);
  launch_pair_force(c->g, F, cf, Z, T, c->U64, c->geom.l0_sub, s, sx);
  launch_pair_force(c->g, F, cf, T2, B, c->U64, c->geom.l0_sub, s, sx);
  SAP_HIP_CHECK(c, hipGetLastError());
  return SAP_OK;
}

// heat baths: kind 1 phi = W3eo P_e xi; kind 2 phi = W3eo^-1 W2eo P_e xi
int eo_heat_bath(sap_ctx* c, double2* phi, const double2* xi, int kind, double rho, const sap_solve_opts* o,
                 hipStream_t s) {
  ForceWS* w = fws(c);
  double2 *E = w->f[5], *T = w->f[6];
  const long long Vhp = c->Vhp;
  SAP_HIP_CHECK(c, hipMemcpyAsync(E, xi, (size_t)12 * Vhp * sizeof(double2), hipMemcpyDeviceToDevice, s));
  SAP_HIP_CHECK(c, hipMemsetAsync(E + 12 * Vhp, 0, (size_t)12 * Vhp * sizeof(double2), s));   // P_e xi
  if (kind == 1) return apply_weo(c, phi, E, rho, T, s);
  int rc = apply_weo(c, w->f[4], E, 0.0, T, s);
  if (rc) return rc;
  return solve_eo1(c, phi, w->f[4], rho, o, s);
}

int gauge_action_host(sap_ctx* c, double beta, double* S, hipStream_t s) {
  ForceWS* w = fws(c);
  launch_plaq_sum(c->g, c->U64, w->part, w->scal, s);
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_scal, w->scal, 8, hipMemcpyDeviceToHost, s));
  SAP_HIP_CHECK(c, hipStreamSynchronize(s));
  *S = -beta / 3.0 * w->h_scal[0];
  return SAP_OK;
}

int kinetic_host(sap_ctx* c, const double* P, double* K, hipStream_t s) {
  ForceWS* w = fws(c);
  launch_kinetic(c->g, P, w->part, w->scal, s);
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_scal, w->scal, 8, hipMemcpyDeviceToHost, s));
  SAP_HIP_CHECK(c, hipStreamSynchronize(s));
  *K = w->h_scal[0];
  return SAP_OK;
}

void links_changed(sap_ctx* c, hipStream_t s) { launch_gauge_to_f32(c->g, c->U64c, c->U32, c->U16, c->U64, s); }
LinkCopies copies_of(sap_ctx* c) { return LinkCopies{c->U64c, c->U32, c->U16}; }

// ---- the two-level integrator --------------------------------------------------------
struct Traj {
  sap_ctx* c;
  const sap_hmc_params* P;
  const double2 *phi1, *chi;
  hipStream_t s;
  const double* sx;    // per-link step scale (device) or null
};

int kick_pf(Traj& T, double dt) {
  int rc = pf_force(T.c, fws(T.c)->mom, -dt, T.phi1, &T.P->force_solve, nullptr, T.s, T.sx);
  if (rc) return rc;
  return schwarz_terms(T.c, fws(T.c)->mom, -dt, T.chi, &T.P->force_solve, nullptr, T.s, T.sx);
}
int kick_g(Traj& T, double dt) {
  launch_gauge_force(T.c->g, fws(T.c)->mom, -dt * T.P->beta / 6.0, T.c->U64, T.s, T.sx);
  SAP_HIP_CHECK(T.c, hipGetLastError());
  return SAP_OK;
}
int move_links(Traj& T, double dt) {
  launch_update_links(T.c->g, T.c->U64, copies_of(T.c), fws(T.c)->mom, dt, T.s, T.sx);   // copies too
  SAP_HIP_CHECK(T.c, hipGetLastError());
  return SAP_OK;
}
// level 0: gauge action
int step0(Traj& T, double dt) {
  int rc;
  const double l = T.P->lambda;
  if (T.P->scheme_inner == 0) {
    if ((rc = kick_g(T, 0.5 * dt)) || (rc = move_links(T, dt)) || (rc = kick_g(T, 0.5 * dt))) return rc;
  } else {
    if ((rc = kick_g(T, l * dt)) || (rc = move_links(T, 0.5 * dt)) || (rc = kick_g(T, (1 - 2 * l) * dt)) ||
        (rc = move_links(T, 0.5 * dt)) || (rc = kick_g(T, l * dt)))
      return rc;
  }
  return SAP_OK;
}
// level 1: pseudo-fermion action, n_inner steps of level 0 per step
int step1(Traj& T, double dt) {
  int rc;
  const int n = T.P->n_inner;
  const double d0 = dt / n, l = T.P->lambda;
  if (T.P->scheme_outer == 0) {
    if ((rc = kick_pf(T, 0.5 * dt))) return rc;
    for (int i = 0; i < n; ++i)
      if ((rc = step0(T, d0))) return rc;
    return kick_pf(T, 0.5 * dt);
  }
  if ((rc = kick_pf(T, l * dt))) return rc;
  for (int i = 0; i < n / 2; ++i)
    if ((rc = step0(T, d0))) return rc;
  if ((rc = kick_pf(T, (1 - 2 * l) * dt))) return rc;
  for (int i = 0; i < n / 2; ++i)
    if ((rc = step0(T, d0))) return rc;
  return kick_pf(T, l * dt);
}

int hamiltonian(Traj& T, double* K, double* SG, double* SW, double* SR) {
  int rc;
  if ((rc = kinetic_host(T.c, fws(T.c)->mom, K, T.s))) return rc;
  if ((rc = gauge_action_host(T.c, T.P->beta, SG, T.s))) return rc;
  ForceWS* w = fws(T.c);
  if ((rc = solve1(T.c, w->f[0], T.phi1, T.c->geom.l0, SAP_ALL, &T.P->action_solve, T.s))) return rc;
  if ((rc = norm2_host(T.c, w->f[0], SW, T.s))) return rc;
  return schwarz_terms(T.c, nullptr, 0.0, T.chi, &T.P->action_solve, SR, T.s);
}

// ---- the five-level integrator of the four-part action (Sec. 2) ---------------------
// solver options of part j = 1..4 inside the molecular dynamics and for its heat bath and
// action (part_solve, else the common force_solve / action_solve)
const sap_solve_opts* force_opts4(const sap_hmc4_params* P, int j) {
  return P->part_solve ? &P->part_solve[j - 1] : &P->force_solve;
}
const sap_solve_opts* action_opts4(const sap_hmc4_params* P, int j) {
  return P->part_solve ? &P->part_solve[3 + j] : &P->action_solve;
}

struct Traj4 {
  sap_ctx* c;
  const sap_hmc4_params* P;
  const double2 *phi1, *phi2, *chi3, *chi4;
  hipStream_t s;
  const double* sx;
};

// T_P of level j: p -= dt F_j (0 gauge, 1 S1, 2 S2, 3 S3, 4 S4)
int kick4(Traj4& T, int j, double dt) {
  sap_ctx* c = T.c;
  double* mom = fws(c)->mom;
  const sap_solve_opts* o = j ? force_opts4(T.P, j) : nullptr;
  switch (j) {
    case 0:
      launch_gauge_force(c->g, mom, -dt * T.P->beta / 6.0, c->U64, T.s, T.sx);
      SAP_HIP_CHECK(c, hipGetLastError());
      return SAP_OK;
    case 1: return eo_pf_terms(c, mom, -dt, T.phi1, 1, T.P->rho, o, nullptr, T.s, T.sx);
    case 2: return eo_pf_terms(c, mom, -dt, T.phi2, 2, T.P->rho, o, nullptr, T.s, T.sx);
    case 3: return schwarz_terms(c, mom, -dt, T.chi3, o, nullptr, T.s, T.sx, c->geom.l0);
    default: return schwarz_terms(c, mom, -dt, T.chi4, o, nullptr, T.s, T.sx, 0);
  }
}

int move4(Traj4& T, double dt) {
  launch_update_links(T.c->g, T.c->U64, copies_of(T.c), fws(T.c)->mom, dt, T.s, T.sx);   // copies too
  SAP_HIP_CHECK(T.c, hipGetLastError());
  return SAP_OK;
}

// one step of level j of length dt: leap-frog (kick dt/2, inner, kick dt/2) or
// Sexton-Weingarten (kick l dt, inner/2, kick (1-2l) dt, inner/2, kick l dt); the inner
// part is T_U for level 0, else n_{j-1} steps of level j-1 of length dt / n_{j-1}
int step4(Traj4& T, int j, double dt) {
  int rc;
  const double l = T.P->lambda;
  const int n = j ? T.P->n[j - 1] : 1;
  auto inner = [&](int count, double len) -> int {
    if (j == 0) return move4(T, len);
    for (int i = 0; i < count; ++i)
      if (int r = step4(T, j - 1, dt / n)) return r;
    return SAP_OK;
  };
  if (T.P->scheme[j] == 0) {
    if ((rc = kick4(T, j, 0.5 * dt)) || (rc = inner(n, dt))) return rc;
    return kick4(T, j, 0.5 * dt);
  }
  if ((rc = kick4(T, j, l * dt)) || (rc = inner(n / 2, 0.5 * dt))) return rc;
  if ((rc = kick4(T, j, (1 - 2 * l) * dt)) || (rc = inner(n / 2, 0.5 * dt))) return rc;
  return kick4(T, j, l * dt);
}

int hamiltonian4(Traj4& T, double* K, double S[5]) {
  int rc;
  sap_ctx* c = T.c;
  const sap_hmc4_params* P = T.P;
  if ((rc = kinetic_host(c, fws(c)->mom, K, T.s))) return rc;
  if ((rc = gauge_action_host(c, P->beta, &S[0], T.s))) return rc;
  if ((rc = eo_pf_terms(c, nullptr, 0.0, T.phi1, 1, P->rho, action_opts4(P, 1), &S[1], T.s))) return rc;
  if ((rc = eo_pf_terms(c, nullptr, 0.0, T.phi2, 2, P->rho, action_opts4(P, 2), &S[2], T.s))) return rc;
  if ((rc = schwarz_terms(c, nullptr, 0.0, T.chi3, action_opts4(P, 3), &S[3], T.s, nullptr, c->geom.l0)))
    return rc;
  return schwarz_terms(c, nullptr, 0.0, T.chi4, action_opts4(P, 4), &S[4], T.s, nullptr, 0);
}

}  // namespace

// Largest deviation of the context's FP64 links from SU(3) (host output; synchronises).
int su3_deviation_host(sap_ctx* c, double* dev, hipStream_t s) {
  ForceWS* w = fws(c);
  launch_su3_dev(c->g, c->U64, w->part, w->scal, s);
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_scal, w->scal, 8, hipMemcpyDeviceToHost, s));
  SAP_HIP_CHECK(c, hipStreamSynchronize(s));
  *dev = w->h_scal[0];
  return SAP_OK;
}


extern "C" {

int eo_pf_heat_bath(sap_ctx* c, double* phi, const double* xi, int kind, double rho, const sap_solve_opts* o,
                    void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!phi || !xi || phi == xi) return sap_fail(c, SAP_E_ARG, "phi and xi must be distinct non-NULL fields");
  if (kind != 1 && kind != 2) return sap_fail(c, SAP_E_ARG, "kind must be 1 (S1) or 2 (S2)");
  if (!(rho >= 0.0 && std::isfinite(rho))) return sap_fail(c, SAP_E_ARG, "rho must be finite and >= 0");
  if (c->geom.l0_sub <= 0) return sap_fail(c, SAP_E_ARG, "the even-odd terms need level-2 blocks (l0_sub > 0)");
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  return eo_heat_bath(c, (double2*)phi, (const double2*)xi, kind, rho, o, (hipStream_t)stream);
}

int eo_pf_force(sap_ctx* c, double* F, double coef, const double* phi, int kind, double rho,
                const sap_solve_opts* o, double* S_out, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!phi || (!F && !S_out)) return sap_fail(c, SAP_E_ARG, "phi is NULL, or neither F nor S_out given");
  if (kind != 1 && kind != 2) return sap_fail(c, SAP_E_ARG, "kind must be 1 (S1) or 2 (S2)");
  if (!(rho >= 0.0 && std::isfinite(rho))) return sap_fail(c, SAP_E_ARG, "rho must be finite and >= 0");
  if (c->geom.l0_sub <= 0) return sap_fail(c, SAP_E_ARG, "the even-odd terms need level-2 blocks (l0_sub > 0)");
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  return eo_pf_terms(c, F, coef, (const double2*)phi, kind, rho, o, S_out, (hipStream_t)stream);
}

int schwarz2_heat_bath(sap_ctx* c, double* chi, const double* g, const sap_solve_opts* o, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!chi || !g || chi == g) return sap_fail(c, SAP_E_ARG, "chi and g must be distinct non-NULL fields");
  if (c->geom.l0_sub <= 0) return sap_fail(c, SAP_E_ARG, "the level-2 Schwarz term needs l0_sub > 0");
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  return heat_bath(c, (double2*)chi, (const double2*)g, o, (hipStream_t)stream, c->geom.l0);
}

int schwarz2_force(sap_ctx* c, double* F, double coef, const double* chi, const sap_solve_opts* o,
                   double* S_out, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!chi || (!F && !S_out)) return sap_fail(c, SAP_E_ARG, "chi is NULL, or neither F nor S_out given");
  if (c->geom.l0_sub <= 0) return sap_fail(c, SAP_E_ARG, "the level-2 Schwarz term needs l0_sub > 0");
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_chi(c, (const double2*)chi, s, c->geom.l0))) return rc;
  return schwarz_terms(c, F, coef, (const double2*)chi, o, S_out, s, nullptr, c->geom.l0);
}

int block_pf_force(sap_ctx* c, double* F, double coef, const double* phi, const sap_solve_opts* o,
                   double* S_out, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!F || !phi) return sap_fail(c, SAP_E_ARG, "F or phi is NULL");
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  return pf_force(c, F, coef, (const double2*)phi, o, S_out, (hipStream_t)stream);
}

int schwarz_boundary_force(sap_ctx* c, double* F, double coef, const double* chi, const sap_solve_opts* o,
                           double* S_R_out, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!F || !chi) return sap_fail(c, SAP_E_ARG, "F or chi is NULL");
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_chi(c, (const double2*)chi, s))) return rc;
  return schwarz_terms(c, F, coef, (const double2*)chi, o, S_R_out, s);
}

int schwarz_heat_bath(sap_ctx* c, double* chi, const double* g, const sap_solve_opts* o, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!chi || !g || chi == g) return sap_fail(c, SAP_E_ARG, "chi and g must be distinct non-NULL fields");
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  return heat_bath(c, (double2*)chi, (const double2*)g, o, (hipStream_t)stream);
}

int schwarz_action(sap_ctx* c, const double* chi, const sap_solve_opts* o, double* S_R_out, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!chi || !S_R_out) return sap_fail(c, SAP_E_ARG, "chi or S_R_out is NULL");
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_chi(c, (const double2*)chi, s))) return rc;
  return schwarz_terms(c, nullptr, 0.0, (const double2*)chi, o, S_R_out, s);
}

int gauge_force(sap_ctx* c, double* F, double coef, double beta, double* S_G_out, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!F) return sap_fail(c, SAP_E_ARG, "F is NULL");
  if (!std::isfinite(beta)) return sap_fail(c, SAP_E_ARG, "beta must be finite");
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  hipStream_t s = (hipStream_t)stream;
  launch_gauge_force(c->g, F, coef * beta / 6.0, c->U64, s);
  SAP_HIP_CHECK(c, hipGetLastError());
  if (S_G_out) return gauge_action_host(c, beta, S_G_out, s);
  return SAP_OK;
}

int sap_update_links(sap_ctx* c, const double* p, double dt, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!p) return sap_fail(c, SAP_E_ARG, "p is NULL");
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  hipStream_t s = (hipStream_t)stream;
  launch_update_links(c->g, c->U64, copies_of(c), p, dt, s);   // writes the reduced copies too
  SAP_HIP_CHECK(c, hipGetLastError());
  return SAP_OK;
}

int sap_plaquette(sap_ctx* c, double* plaq_out, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!plaq_out) return sap_fail(c, SAP_E_ARG, "plaq_out is NULL");
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  double S;
  int rc = gauge_action_host(c, -3.0, &S, (hipStream_t)stream);    // S = sum Re tr U_P
  if (rc) return rc;
  *plaq_out = S / (18.0 * (double)c->V);
  return SAP_OK;
}

int sap_force_profile(sap_ctx* c, const double* F, double* prof, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!F || !prof) return sap_fail(c, SAP_E_ARG, "F or prof is NULL");
  ForceWS* w = fws(c);
  hipStream_t s = (hipStream_t)stream;
  const int L0 = c->geom.L[0];
  double* out = w->prof + (size_t)2 * L0 * force_profile_nck(c->g);
  launch_force_profile(c->g, F, w->prof, out, s);
  SAP_HIP_CHECK(c, hipGetLastError());
  SAP_HIP_CHECK(c, hipMemcpyAsync(prof, out, (size_t)2 * L0 * 8, hipMemcpyDeviceToHost, s));
  SAP_HIP_CHECK(c, hipStreamSynchronize(s));
  return SAP_OK;
}

int sap_shift_gauge(sap_ctx* c, int n, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  hipStream_t s = (hipStream_t)stream;
  ForceWS* w = fws(c);
  launch_shift_links(c->g, w->Utmp, c->U64, n, s);
  SAP_HIP_CHECK(c, hipMemcpyAsync(c->U64, w->Utmp, (size_t)72 * c->Vhp * sizeof(double2),
                                  hipMemcpyDeviceToDevice, s));
  links_changed(c, s);
  SAP_HIP_CHECK(c, hipGetLastError());
  return SAP_OK;
}

int sap_set_gauge(sap_ctx* ctx, const double* U, void* stream);
int sap_get_gauge(sap_ctx* ctx, double* U, void* stream);
int sap_pack_spinor(sap_ctx* ctx, void* out, const double* in, int nrhs, sap_prec prec, void* stream);

int hmc_trajectory(sap_ctx* c, double* U, const sap_hmc_params* P, sap_hmc_info* info, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!U || !P || !info) return sap_fail(c, SAP_E_ARG, "U, params and info must be non-NULL");
  if (!P->p0 || !P->xi1 || !P->xi2) return sap_fail(c, SAP_E_ARG, "p0, xi1 and xi2 must be given");
  if (P->n_outer < 1 || P->n_inner < 1) return sap_fail(c, SAP_E_ARG, "n_outer and n_inner must be >= 1");
  if ((P->scheme_outer != 0 && P->scheme_outer != 1) || (P->scheme_inner != 0 && P->scheme_inner != 1))
    return sap_fail(c, SAP_E_ARG, "scheme must be 0 (leap-frog) or 1 (Sexton-Weingarten)");
  if (P->scheme_outer == 1 && (P->n_inner % 2))
    return sap_fail(c, SAP_E_ARG, "a Sexton-Weingarten outer level needs an even n_inner");
  if (!(P->tau > 0) || !std::isfinite(P->beta) || !std::isfinite(P->lambda))
    return sap_fail(c, SAP_E_ARG, "tau must be > 0, beta and lambda finite");
  int rc;
  if ((rc = check_opts(c, &P->force_solve)) || (rc = check_opts(c, &P->action_solve))) return rc;
  if (P->step_scale)
    for (int i = 0; i < 4 * c->geom.L[0]; ++i)
      if (!(P->step_scale[i] >= 0.0 && std::isfinite(P->step_scale[i])))
        return sap_fail(c, SAP_E_ARG, "step_scale entries must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  ForceWS* w = fws(c);
  if (P->step_scale)
    SAP_HIP_CHECK(c, hipMemcpyAsync(w->sx, P->step_scale, (size_t)4 * c->geom.L[0] * 8, hipMemcpyHostToDevice, s));
  w->iters = 0;
  std::memset(info, 0, sizeof(*info));
  if ((rc = sap_set_gauge(c, U, stream))) return rc;
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->mom, P->p0, (size_t)64 * c->Vhp * 8, hipMemcpyDeviceToDevice, s));
  // heat bath: phi1 = W1 xi1, chi = R_hat Pi xi2 (xi staged in f[0])
  double2 *phi1 = w->f[7], *chi = w->f[8];
  if ((rc = sap_pack_spinor(c, w->f[0], P->xi1, 1, SAP_F64, stream))) return rc;
  HopArgs<double> A;
  const long long Vhp = c->Vhp;
  A.out = {phi1, 24 * Vhp, 12 * Vhp};
  A.in = {w->f[0], 24 * Vhp, 12 * Vhp};
  A.x = A.in;
  A.U = gauge_of<double>(c); A.g = c->g; A.nrhs = 1; A.parity_out = -1;
  A.lb = c->geom.l0; A.slb = c->geom.l0; A.colour = 0; A.block = -1;
  A.a = 1.0; A.b = -c->geom.kappa; A.g5_in = A.g5_out = 0; A.map = HOP_MAP_SITE;
  launch_hop<double>(A, s);
  if ((rc = sap_pack_spinor(c, w->f[0], P->xi2, 1, SAP_F64, stream))) return rc;
  if ((rc = heat_bath(c, chi, w->f[0], &P->action_solve, s))) goto fail;
  {
    Traj T = {c, P, phi1, chi, s, P->step_scale ? w->sx : nullptr};
    double K0, K1;
    if ((rc = hamiltonian(T, &K0, &info->S_G0, &info->S_W0, &info->S_R0))) goto fail;
    info->H0 = K0 + info->S_G0 + info->S_W0 + info->S_R0;
    const double dt = P->tau / P->n_outer;
    for (int k = 0; k < P->n_outer; ++k)
      if ((rc = step1(T, dt))) goto fail;
    if ((rc = hamiltonian(T, &K1, &info->S_G1, &info->S_W1, &info->S_R1))) goto fail;
    info->H1 = K1 + info->S_G1 + info->S_W1 + info->S_R1;
    info->dH = info->H1 - info->H0;
    info->accepted = P->u_metropolis < std::exp(-info->dH);
    if (!info->accepted && (rc = sap_set_gauge(c, U, stream))) goto fail;
    if (P->time_shift && (rc = sap_shift_gauge(c, P->time_shift, stream))) goto fail;
    if ((info->accepted || P->time_shift) && (rc = sap_get_gauge(c, U, stream))) goto fail;
    info->solver_iters = w->iters;
    if ((rc = sap_plaquette(c, &info->plaq, stream))) return rc;
    return SAP_OK;
  }
fail : {
  const std::string m = c->err;
  (void)sap_set_gauge(c, U, stream);     // leave the context on the caller's field
  c->err = m;
  return rc;
}
}

int hmc_trajectory_4pf(sap_ctx* c, double* U, const sap_hmc4_params* P, sap_hmc4_info* info, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!U || !P || !info) return sap_fail(c, SAP_E_ARG, "U, params and info must be non-NULL");
  if (!P->p0 || !P->xi1 || !P->xi2 || !P->g3 || !P->g4)
    return sap_fail(c, SAP_E_ARG, "p0, xi1, xi2, g3 and g4 must be given");
  if (c->geom.l0_sub <= 0) return sap_fail(c, SAP_E_ARG, "the four-part action needs level-2 blocks (l0_sub > 0)");
  for (int j = 0; j < 5; ++j) {
    if (P->n[j] < 1) return sap_fail(c, SAP_E_ARG, "every n_j must be >= 1");
    if (P->scheme[j] != 0 && P->scheme[j] != 1)
      return sap_fail(c, SAP_E_ARG, "scheme must be 0 (leap-frog) or 1 (Sexton-Weingarten)");
    if (j > 0 && P->scheme[j] == 1 && (P->n[j - 1] % 2))
      return sap_fail(c, SAP_E_ARG, "a Sexton-Weingarten level j > 0 needs an even n_{j-1}");
  }
  if (!(P->tau > 0) || !std::isfinite(P->beta) || !std::isfinite(P->lambda) || !(P->rho >= 0 && std::isfinite(P->rho)))
    return sap_fail(c, SAP_E_ARG, "tau must be > 0, beta and lambda finite, rho finite and >= 0");
  int rc;
  if ((rc = check_opts(c, &P->force_solve)) || (rc = check_opts(c, &P->action_solve))) return rc;
  if (P->part_solve)
    for (int k = 0; k < 8; ++k)
      if ((rc = check_opts(c, &P->part_solve[k]))) return rc;
  if (P->step_scale)
    for (int i = 0; i < 4 * c->geom.L[0]; ++i)
      if (!(P->step_scale[i] >= 0.0 && std::isfinite(P->step_scale[i])))
        return sap_fail(c, SAP_E_ARG, "step_scale entries must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  ForceWS* w = fws(c);
  if (P->step_scale)
    SAP_HIP_CHECK(c, hipMemcpyAsync(w->sx, P->step_scale, (size_t)4 * c->geom.L[0] * 8, hipMemcpyHostToDevice, s));
  w->iters = 0;
  std::memset(info, 0, sizeof(*info));
  if ((rc = sap_set_gauge(c, U, stream))) return rc;
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->mom, P->p0, (size_t)64 * c->Vhp * 8, hipMemcpyDeviceToDevice, s));
  // heat baths (noise staged in f[11]): phi1 = W3eo P_e xi1, phi2 = W3eo^-1 W2eo P_e xi2,
  // chi3 = R_hat_2 Pi_2 g3, chi4 = R_hat Pi g4
  double2 *phi1 = w->f[7], *chi4 = w->f[8], *phi2 = w->f[9], *chi3 = w->f[10], *stage = w->f[11];
  if ((rc = sap_pack_spinor(c, stage, P->xi1, 1, SAP_F64, stream)) ||
      (rc = eo_heat_bath(c, phi1, stage, 1, P->rho, action_opts4(P, 1), s)))
    goto fail;
  if ((rc = sap_pack_spinor(c, stage, P->xi2, 1, SAP_F64, stream)) ||
      (rc = eo_heat_bath(c, phi2, stage, 2, P->rho, action_opts4(P, 2), s)))
    goto fail;
  if ((rc = sap_pack_spinor(c, stage, P->g3, 1, SAP_F64, stream)) ||
      (rc = heat_bath(c, chi3, stage, action_opts4(P, 3), s, c->geom.l0)))
    goto fail;
  if ((rc = sap_pack_spinor(c, stage, P->g4, 1, SAP_F64, stream)) ||
      (rc = heat_bath(c, chi4, stage, action_opts4(P, 4), s, 0)))
    goto fail;
  {
    Traj4 T = {c, P, phi1, phi2, chi3, chi4, s, P->step_scale ? w->sx : nullptr};
    double K0, K1;
    if ((rc = hamiltonian4(T, &K0, info->S0))) goto fail;
    info->H0 = K0;
    for (int j = 0; j < 5; ++j) info->H0 += info->S0[j];
    const double dt = P->tau / P->n[4];
    for (int k = 0; k < P->n[4]; ++k)
      if ((rc = step4(T, 4, dt))) goto fail;
    if ((rc = hamiltonian4(T, &K1, info->S1))) goto fail;
    info->H1 = K1;
    for (int j = 0; j < 5; ++j) info->H1 += info->S1[j];
    info->dH = info->H1 - info->H0;
    info->accepted = P->u_metropolis < std::exp(-info->dH);
    if (!info->accepted && (rc = sap_set_gauge(c, U, stream))) goto fail;
    if (P->time_shift && (rc = sap_shift_gauge(c, P->time_shift, stream))) goto fail;
    if ((info->accepted || P->time_shift) && (rc = sap_get_gauge(c, U, stream))) goto fail;
    info->solver_iters = w->iters;
    if ((rc = sap_plaquette(c, &info->plaq, stream))) return rc;
    return SAP_OK;
  }
fail : {
  const std::string m = c->err;
  (void)sap_set_gauge(c, U, stream);
  c->err = m;
  return rc;
}
}

}  // extern "C"
