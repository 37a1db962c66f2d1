// Batched Krylov solves of M x = b (full lattice) and W x = b (every selected x0 block
// an independent system), all systems and right-hand sides advanced together in each
// kernel launch.
//
// Inner solve: even-odd reduced system (Sec. 1, W_eo: M = [[1, -k D_eo], [-k D_oe, 1]],
// M_hat = 1 - k^2 D_eo D_oe), by one of
//  * CG on the normal equations in the CGLS form, which carries s = b_hat - M_hat x;
//    M_hat^dagger = g5 M_hat g5 is applied by the same hop kernel with gamma_5 folded
//    into its input and output;
//  * BiCGstab (van der Vorst) on M_hat directly, with complex per-system scalars;
//  * the geometric series x_e = sum_n (k^2 D_eo D_oe)^n b_hat (Sec. 3 uses it for the block
//    terms), whose residual after n terms is the next term; for the shifted even-site
//    system (M_hat + rho) x_e = b_e of the mass-preconditioned parts every term carries a
//    factor 1 / (1 + rho) and the residual after n terms is (1 + rho) times the next term.
// Per-system scalars stay on the device; converged systems are frozen while the others
// continue; the host reads one counter every few iterations.
// Outer loop: FP64 defect correction r = b - A x (A applied in FP64), inner solve in
// FP32 or FP64, x += e, until ||b - A x|| / ||b|| <= tol recomputed in FP64.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>
#include "blas.h"

using namespace sap;

namespace sap {
int apply_op_any(sap_ctx* ctx, void* out, const void* in, int nrhs, int lb, int colour, int block,
                 sap_prec prec, hipStream_t s);
}

struct SolverWS {
  int max_rhs, max_sys, max_chunk;
  size_t part_cap;                       // doubles in each of partA / partB / partC
  double2 *hx, *s, *r, *p, *q, *t;       // half fields (sized for FP64, max_rhs)
  double2 *x64, *r64, *ax, *rin, *e;     // full fields
  double *partA, *partB, *partC;
  double *gam, *ss, *alpha, *beta, *target2, *bnorm2, *rnorm2;
  double* cs;                            // BiCGstab: complex (rho, alpha, omega, beta) per system
  int *active, *iters, *flags, *selected;
  // pinned host mirrors
  double *h_rnorm2, *h_bnorm2;
  int *h_flags, *h_iters, *h_selected;
  // captured inner-loop graphs (ITERS_PER_GRAPH CG iterations each), replayed on the
  // caller's stream; captured on a private non-blocking stream of default priority
  hipStream_t cap;
  struct G { int nrhs, lb, sel, prec, method; double rho; hipGraphExec_t exec; };
  std::vector<G> graphs;
};

constexpr int ITERS_PER_GRAPH = 8;

static SolverWS* ws_of(sap_ctx* c) { return (SolverWS*)c->solver; }
struct SapWS;
static SapWS* sap_ws(sap_ctx* c);   // Schwarz-preconditioned BiCGstab workspace (below)

extern "C" int sap_solver_create(sap_ctx* c) {
  SolverWS* w = new SolverWS();   // value-initialised: every pointer starts null
  c->solver = w;
  const int minlb = c->geom.l0_sub > 0 ? c->geom.l0_sub : c->geom.l0;
  w->max_rhs = c->geom.max_rhs;
  w->max_sys = (c->geom.L[0] / minlb) * w->max_rhs;
  if (w->max_sys < w->max_rhs) w->max_sys = w->max_rhs;
  w->max_chunk = (int)((c->Vh + CHUNK - 1) / CHUNK);
  const size_t half = (size_t)12 * c->Vhp * w->max_rhs * sizeof(double2);
  const size_t full = 2 * half;
  // three partials per (system, chunk); a level of nblk blocks has at most max_chunk + nblk
  // chunks per rhs
  size_t npart = (size_t)3 * w->max_rhs * (w->max_chunk + c->geom.L[0] / minlb + 1);
  // room for the hop-fused reductions too (three values per slot; systems of l0, l0_sub
  // or all L0 slices)
  for (int nlb : {c->geom.l0, c->geom.l0_sub, c->geom.L[0]})
    if (nlb > 0)
      npart = std::max(npart, (size_t)3 * w->max_rhs * (c->geom.L[0] / nlb) * slabd_norm_slots(c->g, nlb));
  w->part_cap = npart;
  auto A = [&](void** p, size_t n) { return hipMalloc(p, n) == hipSuccess; };
  bool ok = A((void**)&w->hx, half) && A((void**)&w->s, half) && A((void**)&w->r, half) &&
            A((void**)&w->p, half) && A((void**)&w->q, half) && A((void**)&w->t, half) &&
            A((void**)&w->x64, full) && A((void**)&w->r64, full) && A((void**)&w->ax, full) &&
            A((void**)&w->rin, full) && A((void**)&w->e, full) &&
            A((void**)&w->partA, npart * 8) && A((void**)&w->partB, npart * 8) &&
            A((void**)&w->partC, npart * 8);
  const size_t ns = (size_t)w->max_sys;
  ok = ok && A((void**)&w->gam, ns * 8) && A((void**)&w->ss, ns * 8) && A((void**)&w->alpha, ns * 8) &&
       A((void**)&w->beta, ns * 8) && A((void**)&w->target2, ns * 8) && A((void**)&w->bnorm2, ns * 8) &&
       A((void**)&w->rnorm2, ns * 8) && A((void**)&w->cs, ns * 64) && A((void**)&w->active, ns * 4) &&
       A((void**)&w->iters, ns * 4) &&
       A((void**)&w->flags, 16) && A((void**)&w->selected, ns * 4);
  ok = ok && hipHostMalloc((void**)&w->h_rnorm2, ns * 8, 0) == hipSuccess &&
       hipHostMalloc((void**)&w->h_bnorm2, ns * 8, 0) == hipSuccess &&
       hipHostMalloc((void**)&w->h_flags, 16, 0) == hipSuccess &&
       hipHostMalloc((void**)&w->h_iters, ns * 4, 0) == hipSuccess &&
       hipHostMalloc((void**)&w->h_selected, ns * 4, 0) == hipSuccess;
  if (!ok) return sap_fail(c, SAP_E_NOMEM, "cannot allocate the solver workspace");
  if (hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking) != hipSuccess)
    return sap_fail(c, SAP_E_HIP, "cannot create the capture stream");
  // the Schwarz-preconditioned BiCGstab workspace too, so that no solve allocates fields
  if (!sap_ws(c)) return sap_fail(c, SAP_E_NOMEM, "cannot allocate the Schwarz-preconditioned BiCGstab workspace");
  return SAP_OK;
}

static void drop_graphs(SolverWS* w) {
  for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.exec);
  w->graphs.clear();
}

extern "C" void sap_solver_destroy(sap_ctx* c) {
  SolverWS* w = ws_of(c);
  if (!w) return;
  void* dev[] = {w->hx, w->s, w->r, w->p, w->q, w->t, w->x64, w->r64, w->ax, w->rin, w->e,
                 w->partA, w->partB, w->partC, w->gam, w->ss, w->alpha, w->beta, w->target2,
                 w->bnorm2, w->rnorm2, w->cs, w->active, w->iters, w->flags, w->selected};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  void* host[] = {w->h_rnorm2, w->h_bnorm2, w->h_flags, w->h_iters, w->h_selected};
  for (void* p : host)
    if (p) (void)hipHostFree(p);
  drop_graphs(w);
  if (w->cap) (void)hipStreamDestroy(w->cap);
  delete w;
  c->solver = nullptr;
}

__global__ void k_targets(int nsys, const double* partb, int nchunk, const double* bnorm2, double inner2,
                          double abs2, double* target2) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    double bb = 0.0;
    for (int c = 0; c < nchunk; ++c) bb += partb[(long long)s * nchunk + c];
    target2[s] = fmax(inner2 * bb, abs2 * bnorm2[s]);
  }
}

namespace {

// out = a*x + b*D(in) on one parity or both, block-restricted
// npart (even-odd FP32 hop with the LDS-staged slab mapping only, g5i = 0): also write the
// partial reductions red of each system of nlb slices, nslot per system (slabd_norm_slots):
// 1 ||out||^2, 3 <out, x> and ||out||^2 (HopArgs::red)
template <class R>
void hop(sap_ctx* c, const void* U, Field<R> out, Field<R> in, Field<R> x, int parity_out, int nrhs, int lb,
         int colour, typename arith<R>::type a, typename arith<R>::type b, int g5i, int g5o, hipStream_t st,
         double* npart = nullptr, int nlb = 0, int nslot = 0, int red = 1) {
  HopArgs<R> A;
  A.out = out;
  A.in = in;
  A.x = x;
  A.U = (const typename vec2<R>::type*)U;
  A.g = c->g;
  A.nrhs = nrhs;
  A.parity_out = parity_out;
  A.lb = lb;
  A.slb = lb;
  A.colour = colour < 3 ? colour : 0;
  A.block = colour < 3 ? -1 : colour - 3;
  A.a = a;
  A.b = b;
  A.g5_in = g5i;
  A.g5_out = g5o;
  A.map = hop_map_for(c, parity_out < 0, prec_of<R>(), nrhs);
  A.npart = npart;
  A.nlb = nlb;
  A.nslot = nslot;
  A.red = red;
  launch_hop<R>(A, st);
}

}  // namespace

template <class R>
// eo_only: solve (M_hat + rho) x_e = b_e on the even sites (x and b vanish on the odd
// sites; no reconstruction; residual on the even sites), the form the mass-preconditioned
// action parts need. Otherwise rho must be 0.
static int solve_impl(sap_ctx* c, double* x, const double* b, int nrhs, int lb, int colour,
                      const sap_solve_opts* o, sap_solve_info* info, hipStream_t st, double rho = 0.0,
                      bool eo_only = false) {
  typedef typename arith<R>::type Ar;
  SolverWS* w = ws_of(c);
  const long long Vh = c->Vh, Vhp = c->Vhp;
  const SysGrid G = make_sysgrid(Vh, c->g.V3h, lb, c->geom.L[0], colour);
  const int nsys = G.nblk * nrhs;
  const double kap = c->geom.kappa;
  const void* U = gauge_of<R>(c);
  const Ar kR = (Ar)kap, k2R = (Ar)(-kap * kap);
  const Ar aI = (Ar)(1.0 + rho);               // unit term of M_hat + rho
  const size_t fullb = (size_t)24 * Vhp * nrhs * sizeof(double2);
  const size_t fullR = full_bytes<R>(Vhp, nrhs), halfR = half_bytes<R>(Vhp, nrhs);
  if (rho != 0.0 && !eo_only) return sap_fail(c, SAP_E_ARG, "a shift needs the even-site system");
  // geometric series: terms t_0 = b_hat / (1 + rho), t_{n+1} = k^2 / (1 + rho) D_eo D_oe t_n,
  // residual (1 + rho) t_{n+1}: the series works on t, so b_hat and the target are scaled
  const bool geom = o->method == SAP_GEOM;
  const double shift_inv = 1.0 / (1.0 + rho);

  Field<double> X = {(double2*)x, 24 * Vhp, 12 * Vhp}, B = {(double2*)b, 24 * Vhp, 12 * Vhp};
  Field<double> R64 = {w->r64, 24 * Vhp, 12 * Vhp}, AX = {w->ax, 24 * Vhp, 12 * Vhp};
  Field<R> RIN = full_field<R>(w->rin, Vhp), E = full_field<R>(w->e, Vhp);
  Field<R> Ee = E;                             // the even half of E
  Ee.ps = 0;
  Field<R> S = half_field<R>(w->s, Vhp), Rr = half_field<R>(w->r, Vhp), P = half_field<R>(w->p, Vhp);
  Field<R> Q = half_field<R>(w->q, Vhp), T = half_field<R>(w->t, Vhp);
  Field<R> HX = half_field<R>(w->hx, Vhp);
  const int method = (int)o->method;
  Field<R> NONE = {nullptr, 0, 0, 0};
  SysScal SC = {w->gam, w->ss, w->alpha, w->beta, w->active, w->iters, w->flags};

  // selection of systems
  for (int r = 0; r < nrhs; ++r)
    for (int k = 0; k < G.nblk; ++k)
      w->h_selected[r * G.nblk + k] = block_selected(G.colour, k);
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->selected, w->h_selected, nsys * 4, hipMemcpyHostToDevice, st));
  SAP_HIP_CHECK(c, hipMemsetAsync(w->iters, 0, nsys * 4, st));
  SAP_HIP_CHECK(c, hipMemsetAsync(x, 0, fullb, st));

  // ||b||^2 per system; first residual r = b
  blas_norm2<double>(G, nrhs, B, 2, w->partA, st);
  fin_sum(nsys, G.nchunk, w->partA, w->bnorm2, st);
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->r64, b, fullb, hipMemcpyDeviceToDevice, st));
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->rnorm2, w->bnorm2, nsys * 8, hipMemcpyDeviceToDevice, st));
  SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_bnorm2, w->bnorm2, nsys * 8, hipMemcpyDeviceToHost, st));

  const double tol = o->tol;
  const double inner_tol = (std::is_same<R, double>::value && o->inner_tol <= 0) ? tol : o->inner_tol;
  long long total_iters = 0;
  int outer = 0;
  int status = SAP_OK;
  for (;;) {
    SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_rnorm2, w->rnorm2, nsys * 8, hipMemcpyDeviceToHost, st));
    SAP_HIP_CHECK(c, hipStreamSynchronize(st));
    bool all = true, finite = true;
    for (int s = 0; s < nsys; ++s) {
      if (!w->h_selected[s]) continue;
      const double bb = w->h_bnorm2[s], rr = w->h_rnorm2[s];
      if (!std::isfinite(rr) || !std::isfinite(bb)) finite = false;
      if (bb > 0 && rr > tol * tol * bb) all = false;
    }
    if (!finite) { status = sap_fail(c, SAP_E_NONFINITE, "non-finite residual"); break; }
    if (all) break;
    if (outer >= o->max_outer || total_iters >= o->max_iter) {
      status = sap_fail(c, SAP_E_NOCONV, "solver did not reach tol within max_outer / max_iter");
      break;
    }
    ++outer;
    // inner right-hand side at the inner precision
    blas_convert<R, double>(G, nrhs, RIN, R64, 2, st);
    // b_hat_e = r_e + k D_eo r_o  (into S; times 1 / (1 + rho) for the series)
    hop<R>(c, U, S, RIN, RIN, 0, nrhs, lb, colour, geom ? (Ar)shift_inv : Ar(1),
           geom ? (Ar)(kap * shift_inv) : kR, 0, 0, st);
    SAP_HIP_CHECK(c, hipMemsetAsync(w->e, 0, fullR, st));
    blas_norm2<R>(G, nrhs, S, 1, w->partB, st);
    // stop the inner solve at ||s|| <= max(inner_tol ||b_hat||, 0.3 tol ||b||): the outer
    // residual after x += e equals the inner one up to rounding
    hipLaunchKernelGGL(k_targets, dim3(1), dim3(256), 0, st, nsys, w->partB, G.nchunk, w->bnorm2,
                       inner_tol * inner_tol, 0.09 * tol * tol * (geom ? shift_inv * shift_inv : 1.0),
                       w->target2);
    SAP_HIP_CHECK(c, hipMemsetAsync(w->flags, 0, 16, st));
    const size_t halfb = halfR;
    if (method == SAP_CG) {
      // r = M_hat^dagger s = s - k^2 g5 D_eo D_oe g5 s
      hop<R>(c, U, T, S, NONE, 1, nrhs, lb, colour, Ar(0), Ar(1), 1, 0, st);
      hop<R>(c, U, Rr, T, S, 0, nrhs, lb, colour, aI, k2R, 0, 1, st);
      blas_norm2<R>(G, nrhs, Rr, 1, w->partC, st);
      fin_init(SC, nsys, G.nchunk, w->partB, w->partC, w->selected, w->target2, st);
      SAP_HIP_CHECK(c, hipMemcpyAsync(w->p, w->r, halfb, hipMemcpyDeviceToDevice, st));
    } else if (method == SAP_BICGSTAB) {
      // r = s = b_hat (x_e = 0), shadow residual r0 = r, p = v = 0
      SAP_HIP_CHECK(c, hipMemcpyAsync(w->r, w->s, halfb, hipMemcpyDeviceToDevice, st));
      SAP_HIP_CHECK(c, hipMemsetAsync(w->p, 0, halfb, st));
      SAP_HIP_CHECK(c, hipMemsetAsync(w->q, 0, halfb, st));
      blas_cdot3<R>(G, nrhs, Rr, S, S, w->partA, st);
      fin_bicg_rho(SC, w->cs, nsys, G.nchunk, w->partA, w->selected, w->target2, 1, st);
    } else {
      // first term t_0 = b_hat in S
      fin_geom(SC, nsys, G.nchunk, w->partB, w->selected, w->target2, 1, st);
    }
    SAP_HIP_CHECK(c, hipGetLastError());
    // the LDS-staged hop (FP32 and FP16 storage) writes the reductions of its output
    // itself: ||M_hat p||^2 and ||M_hat^dagger s||^2 (CG), <t, s> and ||t||^2 (BiCGstab,
    // three values per slot); FP16 sums the values before their rounding to FP16
    int nslot = 0;
    if ((std::is_same<R, float>::value || std::is_same<R, h16>::value) && method != SAP_GEOM &&
        hop_map_for(c, false, prec_of<R>(), nrhs) == HOP_MAP_SLABD) {
      nslot = slabd_norm_slots(c->g, lb ? lb : c->geom.L[0]);
      const size_t per = method == SAP_CG ? 1 : 3;
      if (per * nslot * nsys > w->part_cap) nslot = 0;   // no room in the partial buffers
    }
    const int nlb = lb ? lb : c->geom.L[0];
    const int nq = nslot ? nslot : G.nchunk;
    // iterations on all systems (no host interaction; scalars stay on the device)
    auto iterate = [&](hipStream_t q) {
      if (method == SAP_CG) {
        // q = M_hat p
        hop<R>(c, U, T, P, NONE, 1, nrhs, lb, colour, Ar(0), Ar(1), 0, 0, q);
        hop<R>(c, U, Q, T, P, 0, nrhs, lb, colour, aI, k2R, 0, 0, q, nslot ? w->partA : nullptr, nlb, nslot);
        if (!nslot) blas_norm2<R>(G, nrhs, Q, 1, w->partA, q);
        fin_alpha(SC, nsys, nq, w->partA, q);
        // s -= alpha q (x += alpha p waits for the direction update)
        blas_cg_s<R>(G, nrhs, S, Q, w->alpha, w->partB, q);
        // r = M_hat^dagger s
        hop<R>(c, U, T, S, NONE, 1, nrhs, lb, colour, Ar(0), Ar(1), 1, 0, q);
        hop<R>(c, U, Rr, T, S, 0, nrhs, lb, colour, aI, k2R, 0, 1, q, nslot ? w->partC : nullptr, nlb, nslot);
        if (!nslot) blas_norm2<R>(G, nrhs, Rr, 1, w->partC, q);
        fin_beta(SC, nsys, G.nchunk, w->partB, nq, w->partC, w->target2, q);
        // x += alpha p, p = r + beta p
        blas_cg_xp<R>(G, nrhs, Ee, P, Rr, w->alpha, w->beta, q);
      } else if (method == SAP_BICGSTAB) {
        // residual r in S, shadow r0 in Rr, v in Q, t in HX
        blas_bicg_p<R>(G, nrhs, P, S, Q, w->cs, q);
        hop<R>(c, U, T, P, NONE, 1, nrhs, lb, colour, Ar(0), Ar(1), 0, 0, q);
        hop<R>(c, U, Q, T, P, 0, nrhs, lb, colour, aI, k2R, 0, 0, q);
        blas_cdot3<R>(G, nrhs, Rr, Q, NONE, w->partB, q);
        fin_bicg_alpha(SC, w->cs, nsys, G.nchunk, w->partB, q);
        blas_bicg_s<R>(G, nrhs, S, Q, w->cs, w->partB, q);
        hop<R>(c, U, T, S, NONE, 1, nrhs, lb, colour, Ar(0), Ar(1), 0, 0, q);
        hop<R>(c, U, HX, T, S, 0, nrhs, lb, colour, aI, k2R, 0, 0, q, nslot ? w->partC : nullptr, nlb, nslot, 3);
        if (!nslot) blas_cdot3<R>(G, nrhs, HX, S, HX, w->partC, q);
        fin_bicg_omega(SC, w->cs, nsys, nq, w->partC, G.nchunk, w->partB, w->target2, q);
        blas_bicg_xr<R>(G, nrhs, Ee, P, S, HX, Rr, w->cs, w->partA, q);
        fin_bicg_rho(SC, w->cs, nsys, G.nchunk, w->partA, w->selected, w->target2, 0, q);
      } else {
        // two terms: S -> HX -> S (x_e += t on active systems; t <- k^2 D_eo D_oe t)
        for (int h = 0; h < 2; ++h) {
          Field<R> from = h == 0 ? S : HX, to = h == 0 ? HX : S;
          blas_geom_add<R>(G, nrhs, Ee, from, w->active, q);
          hop<R>(c, U, T, from, NONE, 1, nrhs, lb, colour, Ar(0), Ar(1), 0, 0, q);
          hop<R>(c, U, to, T, NONE, 0, nrhs, lb, colour, Ar(0), (Ar)(kap * kap * shift_inv), 0, 0, q);
          blas_norm2<R>(G, nrhs, to, 1, w->partA, q);
          fin_geom(SC, nsys, G.nchunk, w->partA, w->selected, w->target2, 0, q);
        }
      }
    };
    // iterations per graph (a geometric-series call of iterate adds two terms)
    const int per_call = method == SAP_GEOM ? 2 : 1;
    const int calls = ITERS_PER_GRAPH / per_call;
    hipGraphExec_t exec = nullptr;
    for (auto& g : w->graphs)
      if (g.nrhs == nrhs && g.lb == lb && g.sel == colour && g.prec == prec_of<R>() && g.method == method &&
          g.rho == rho)
        exec = g.exec;
    if (!exec) {
      hipGraph_t graph;
      if (hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        for (int k = 0; k < calls; ++k) iterate(w->cap);
        if (hipStreamEndCapture(w->cap, &graph) == hipSuccess) {
          if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
          (void)hipGraphDestroy(graph);
        }
      }
      (void)hipGetLastError();
      if (exec) w->graphs.push_back({nrhs, lb, colour, prec_of<R>(), method, rho, exec});
    }
    for (;;) {
      SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_flags, w->flags, 12, hipMemcpyDeviceToHost, st));
      SAP_HIP_CHECK(c, hipStreamSynchronize(st));
      if (w->h_flags[0])
        return sap_fail(c, SAP_E_NONFINITE,
                        "non-finite value in the inner solve (stage " + std::to_string(w->h_flags[0]) + ")");
      if (w->h_flags[2]) return sap_fail(c, SAP_E_NOCONV, "the geometric series diverges (spectral radius >= 1)");
      if (w->h_flags[1] == 0) break;
      if (total_iters >= o->max_iter) break;
      if (exec) {
        SAP_HIP_CHECK(c, hipGraphLaunch(exec, st));
      } else {
        for (int k = 0; k < calls; ++k) iterate(st);
      }
      total_iters += ITERS_PER_GRAPH;
    }
    // e_o = r_o + k D_oe e_e ; x += e ; r = b - A x (FP64)
    if (!eo_only) hop<R>(c, U, E, Ee, RIN, 1, nrhs, lb, colour, Ar(1), kR, 0, 0, st);
    blas_add_mixed<R>(G, nrhs, X, E, st);
    if (eo_only) {
      // A x = (M_hat + rho) x_e on the even sites, via the odd half of AX
      const Field<double> NONE64 = {nullptr, 0, 0};
      hop<double>(c, gauge_of<double>(c), AX, X, NONE64, 1, nrhs, lb, colour, 0.0, 1.0, 0, 0, st);
      hop<double>(c, gauge_of<double>(c), AX, AX, X, 0, nrhs, lb, colour, 1.0 + rho, -kap * kap, 0, 0, st);
      blas_resid(G, nrhs, R64, B, AX, w->partA, st, 1);
    } else {
      int rc = apply_op_any(c, w->ax, x, nrhs, lb, colour < 3 ? colour : 0, colour < 3 ? -1 : colour - 3,
                            SAP_F64, st);
      if (rc) return rc;
      blas_resid(G, nrhs, R64, B, AX, w->partA, st);
    }
    fin_sum(nsys, G.nchunk, w->partA, w->rnorm2, st);
    SAP_HIP_CHECK(c, hipGetLastError());
  }
  if (info) {
    SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_iters, w->iters, nsys * 4, hipMemcpyDeviceToHost, st));
    SAP_HIP_CHECK(c, hipMemcpyAsync(w->h_rnorm2, w->rnorm2, nsys * 8, hipMemcpyDeviceToHost, st));
    SAP_HIP_CHECK(c, hipStreamSynchronize(st));
    for (int s = 0; s < nsys; ++s) {
      const double bb = w->h_bnorm2[s];
      info[s].iters = w->h_selected[s] ? w->h_iters[s] : 0;
      info[s].outer = w->h_selected[s] ? outer : 0;
      info[s].true_rel_res = (w->h_selected[s] && bb > 0) ? std::sqrt(w->h_rnorm2[s] / bb) : 0.0;
    }
  }
  return status;
}

// ---- hop-mapping autotuner -------------------------------------------------------------
template <class R>
static int tune_one(sap_ctx* c, bool full, int nrhs, hipStream_t st, float* us_out) {
  SolverWS* w = ws_of(c);
  typedef typename arith<R>::type Ar;
  const long long Vhp = c->Vhp;
  const bool f16 = std::is_same<R, h16>::value;
  HopArgs<R> A;
  A.out = full_field<R>(w->ax, Vhp);
  A.in = full_field<R>(w->r64, Vhp);
  A.x = full ? A.in : Field<R>{nullptr, 0, 0, 0};
  A.U = gauge_of<R>(c);
  A.g = c->g;
  A.nrhs = nrhs;
  A.parity_out = full ? -1 : 0;
  A.lb = A.slb = 0;
  A.colour = 0;
  A.block = -1;
  A.a = Ar(1);
  A.b = Ar(-c->geom.kappa);
  A.g5_in = A.g5_out = 0;
  hipEvent_t e0, e1;
  SAP_HIP_CHECK(c, hipEventCreate(&e0));
  SAP_HIP_CHECK(c, hipEventCreate(&e1));
  int best = HOP_MAP_SITE;
  float best_ms = 1e30f;
  for (int m = 0; m < HOP_NMAP; ++m) {
    const bool one_rhs_alias = m == HOP_MAP_LANE4 || m == HOP_MAP_WAVE4 ||
                               (m >= HOP_SWEEP && m != HOP_MAP_MARCH1 && m != HOP_MAP_WALK1 &&
                                m != HOP_MAP_BAND1 && m != HOP_MAP_SLAB1 && m != HOP_MAP_SLAB1W &&
                                m != HOP_MAP_SLABD);
    // the LDS-staged slab kernel exists for FP32 and FP16 storage (FP64 runs SLAB1)
    const bool f64_alias = m == HOP_MAP_SLABD && std::is_same<R, double>::value;
    const bool half_only = m == HOP_MAP_STREAM || m >= HOP_MAP_WALK1;
    // FP16 storage has the site and marching kernels only
    const bool f16_alias = f16 && m != HOP_MAP_SITE && m != HOP_MAP_MARCH1 && m != HOP_MAP_MARCH2 && m != HOP_MAP_SLABD &&
                           m != HOP_MAP_MARCH4;
    if ((full && half_only) || (nrhs == 1 && one_rhs_alias) || f16_alias || f64_alias) {
      // the streaming, walking and band kernels exist for half hops only (the full
      // operator runs the walking and band maps as MARCH1 / MARCH2); with one rhs the
      // grouped and sweep orders coincide with SITE, MARCH2 / MARCH4 with MARCH1 and
      // WALK2 with WALK1
      if (us_out) us_out[m] = -1.0f;
      continue;
    }
    A.map = m;
    for (int k = 0; k < 2; ++k) launch_hop<R>(A, st);
    SAP_HIP_CHECK(c, hipEventRecord(e0, st));
    const int reps = 6;
    for (int k = 0; k < reps; ++k) launch_hop<R>(A, st);
    SAP_HIP_CHECK(c, hipEventRecord(e1, st));
    SAP_HIP_CHECK(c, hipEventSynchronize(e1));
    float ms = 0;
    SAP_HIP_CHECK(c, hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    if (hipGetLastError() != hipSuccess) ms = 1e30f;   // variant not launchable here
    if (us_out) us_out[m] = ms * 1e3f;
    if (ms < best_ms) { best_ms = ms; best = m; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->hop_map[full ? 1 : 0][prec_of<R>()][nrhs] = (signed char)best;
  return SAP_OK;
}

extern "C" int sap_tune(sap_ctx* c, int nrhs, float* us_out, void* stream) {
  if (c && c->solver) drop_graphs(ws_of(c));   // captured graphs hold the old mappings
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (nrhs < 1 || nrhs > c->geom.max_rhs) return sap_fail(c, SAP_E_ARG, "nrhs must be in [1, max_rhs]");
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  hipStream_t st = (hipStream_t)stream;
  SolverWS* w = ws_of(c);
  const size_t fb = (size_t)24 * c->Vhp * nrhs * sizeof(double2);
  SAP_HIP_CHECK(c, hipMemsetAsync(w->r64, 0, fb, st));
  SAP_HIP_CHECK(c, hipMemsetAsync(w->ax, 0, fb, st));
  int rc;
  if ((rc = tune_one<double>(c, true, nrhs, st, us_out ? us_out + 0 * HOP_NMAP : nullptr))) return rc;
  if ((rc = tune_one<float>(c, true, nrhs, st, us_out ? us_out + 1 * HOP_NMAP : nullptr))) return rc;
  if ((rc = tune_one<double>(c, false, nrhs, st, us_out ? us_out + 2 * HOP_NMAP : nullptr))) return rc;
  if ((rc = tune_one<float>(c, false, nrhs, st, us_out ? us_out + 3 * HOP_NMAP : nullptr))) return rc;
  if ((rc = tune_one<h16>(c, true, nrhs, st, us_out ? us_out + 4 * HOP_NMAP : nullptr))) return rc;
  if ((rc = tune_one<h16>(c, false, nrhs, st, us_out ? us_out + 5 * HOP_NMAP : nullptr))) return rc;
  return SAP_OK;
}

extern "C" int sap_set_hop_map(sap_ctx* c, int full, sap_prec prec, int nrhs, int map) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (nrhs < 1 || nrhs > 64) return sap_fail(c, SAP_E_ARG, "nrhs must be in [1, 64]");
  if (map < -1 || map >= HOP_NMAP) return sap_fail(c, SAP_E_ARG, "unknown mapping");
  if (full && map == HOP_MAP_STREAM) return sap_fail(c, SAP_E_ARG, "the streaming mapping is for the even-odd hop only");
  if (prec != SAP_F64 && prec != SAP_F32 && prec != SAP_F16) return sap_fail(c, SAP_E_ARG, "unknown precision");
  if (c->solver) drop_graphs(ws_of(c));
  c->hop_map[full ? 1 : 0][prec][nrhs] = (signed char)map;
  return SAP_OK;
}

int sap::check_solve_opts(sap_ctx* c, const sap_solve_opts* o) {
  if (!o) return sap_fail(c, SAP_E_ARG, "opts is NULL");
  if (!(o->tol > 0 && o->tol < 1)) return sap_fail(c, SAP_E_ARG, "tol must be in (0, 1)");
  if (o->max_iter < 1 || o->max_outer < 1) return sap_fail(c, SAP_E_ARG, "max_iter and max_outer must be >= 1");
  if (o->inner_prec != SAP_F64 && o->inner_prec != SAP_F32 && o->inner_prec != SAP_F16)
    return sap_fail(c, SAP_E_ARG, "unknown inner precision");
  if (o->inner_prec != SAP_F64 && !(o->inner_tol > 0 && o->inner_tol < 1))
    return sap_fail(c, SAP_E_ARG, "inner_tol must be in (0, 1) for an FP32 or FP16 inner solve");
  if (o->method != SAP_CG && o->method != SAP_BICGSTAB && o->method != SAP_GEOM && o->method != SAP_SAP_BICGSTAB)
    return sap_fail(c, SAP_E_ARG, "unknown method");
  if (o->sap_block_terms < 0 || o->sap_block_terms > 100000)
    return sap_fail(c, SAP_E_ARG, "sap_block_terms must be in [0, 100000]");
  if (o->method == SAP_SAP_BICGSTAB &&
      (o->sap_ncy < 1 || !(o->sap_block_terms > 0 || (o->inner_tol > 0 && o->inner_tol < 1))))
    return sap_fail(c, SAP_E_ARG,
                    "SAP_SAP_BICGSTAB needs sap_ncy >= 1 and inner_tol in (0, 1) or sap_block_terms > 0");
  return SAP_OK;
}

// ---- Schwarz-preconditioned BiCGstab for M x = b ----------------------------------------
// FP64 BiCGstab on the full lattice, right-preconditioned (M K y = b, x = K y) by K = ncy
// cycles of the multiplicative Schwarz alternating procedure on the level-1 x0 blocks: for
// the black blocks, then the white blocks, y = W1^{-1} (v - M x_K) restricted to that
// colour's blocks (W1 is block diagonal) and x_K += y. The block systems of a colour are one
// batched solve_impl call (CG at inner_prec to the relative residual inner_tol). The few
// outer iterations are driven from the host, which holds the complex scalars.
//
// A full FP64 field [rhs][parity][tiles] is read as 2 * nrhs half fields of stride 12 Vhp,
// so the per-system BLAS kernels apply; the host adds the two parities of every sum.
struct SapWS {
  int nrhs_cap;
  double2 *r, *r0, *p, *v, *t, *ph, *sh, *kx, *kr, *ky, *mt;
  double2 *g1, *g2;     // series block solves: b_hat (even half), D_oe y (odd half)
  double *part, *dev3, *coef;
  double *ck_res, *ck_add;   // device coefficients of the preconditioner's two fixed updates
  double *h3, *hcoef;
};

static void sap_ws_free(SapWS* a) {
  void* dev[] = {a->r, a->r0, a->p, a->v, a->t, a->ph, a->sh, a->kx, a->kr, a->ky, a->mt, a->g1, a->g2, a->part, a->dev3,
                 a->coef, a->ck_res, a->ck_add};
  for (void* q : dev)
    if (q) (void)hipFree(q);
  if (a->h3) (void)hipHostFree(a->h3);
  if (a->hcoef) (void)hipHostFree(a->hcoef);
  delete a;
}

extern "C" void sap_sapws_destroy(sap_ctx* c) {
  if (c->sapws) sap_ws_free((SapWS*)c->sapws);
  c->sapws = nullptr;
}

// allocated by sap_create (sap_solver_create); later calls return it
static SapWS* sap_ws(sap_ctx* c) {
  if (c->sapws) return (SapWS*)c->sapws;
  SapWS* a = new SapWS();
  const int n = c->geom.max_rhs;
  a->nrhs_cap = n;
  const size_t fb = (size_t)24 * c->Vhp * n * sizeof(double2);
  const size_t nsys = 2 * (size_t)n;
  const size_t nchunk = (size_t)((c->Vh + CHUNK - 1) / CHUNK);
  bool ok = true;
  double2** fields[] = {&a->r, &a->r0, &a->p, &a->v, &a->t, &a->ph, &a->sh, &a->kx, &a->kr, &a->ky, &a->mt,
                        &a->g1, &a->g2};
  for (double2** f : fields) ok = ok && hipMalloc((void**)f, fb) == hipSuccess;
  ok = ok && hipMalloc((void**)&a->part, 3 * nsys * nchunk * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&a->dev3, 3 * nsys * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&a->coef, 6 * nsys * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&a->ck_res, 6 * nsys * 8) == hipSuccess;
  ok = ok && hipMalloc((void**)&a->ck_add, 6 * nsys * 8) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&a->h3, 3 * nsys * 8, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&a->hcoef, 12 * nsys * 8, 0) == hipSuccess;   // two coefficient sets
  if (!ok) {
    sap_ws_free(a);
    return nullptr;
  }
  c->sapws = a;
  return a;
}

typedef std::complex<double> zd;

static int sap_bicgstab(sap_ctx* c, double* x, const double* b, int nrhs, const sap_solve_opts* o,
                        sap_solve_info* info, hipStream_t st) {
  SapWS* a = sap_ws(c);
  if (!a) return sap_fail(c, SAP_E_NOMEM, "cannot allocate the Schwarz-preconditioned BiCGstab workspace");
  const long long Vhp = c->Vhp;
  const SysGrid G = make_sysgrid(c->Vh, c->g.V3h, 0, c->geom.L[0], 0);   // full lattice, one block
  const int nh = 2 * nrhs;                                                 // half-field systems
  auto H = [&](double2* f) { return Field<double>{f, 12 * Vhp, 0}; };
  const Field<double> NONE = {nullptr, 0, 0};
  const size_t fullb = (size_t)24 * Vhp * nrhs * sizeof(double2);
  std::vector<zd> rho(nrhs), alpha(nrhs), omega(nrhs);
  std::vector<double> bb(nrhs), rr(nrhs);
  std::vector<int> act(nrhs), its(nrhs, 0);

  // per-rhs sums of the three partials (parities added): s3[r] = (<q, y>, ||y||^2)
  auto sums = [&](std::vector<zd>& dot, std::vector<double>& nrm) -> int {
    fin_sum3(nh, G.nchunk, a->part, a->dev3, st);
    SAP_HIP_CHECK(c, hipMemcpyAsync(a->h3, a->dev3, 3 * nh * 8, hipMemcpyDeviceToHost, st));
    SAP_HIP_CHECK(c, hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) {
      const double* u = a->h3 + 6 * r;
      dot[r] = zd(u[0] + u[3], u[1] + u[4]);
      nrm[r] = u[2] + u[5];
    }
    return SAP_OK;
  };
  // y = c0 y + c1 u + c2 w on every rhs (coefficients per rhs, copied to both parities)
  auto lin3 = [&](double2* y, const double2* u, const double2* w, const double2* q, const std::vector<zd>& c0,
                  const std::vector<zd>& c1, const std::vector<zd>& c2, bool want) -> int {
    for (int r = 0; r < nrhs; ++r)
      for (int par = 0; par < 2; ++par) {
        double* cf = a->hcoef + 6 * (2 * r + par);
        cf[0] = c0[r].real(); cf[1] = c0[r].imag();
        cf[2] = c1[r].real(); cf[3] = c1[r].imag();
        cf[4] = c2[r].real(); cf[5] = c2[r].imag();
      }
    SAP_HIP_CHECK(c, hipMemcpyAsync(a->coef, a->hcoef, 6 * nh * 8, hipMemcpyHostToDevice, st));
    blas_lin3<double>(G, nh, H(y), H((double2*)u), w ? H((double2*)w) : NONE, q ? H((double2*)q) : NONE, a->coef,
                      want ? a->part : nullptr, st);
    // the host buffer is rewritten by the next call: wait until the copy has been consumed
    SAP_HIP_CHECK(c, hipStreamSynchronize(st));
    return SAP_OK;
  };
  auto cdot = [&](const double2* q, const double2* y, const double2* z, std::vector<zd>& dot,
                  std::vector<double>& nrm) -> int {
    blas_cdot3<double>(G, nh, H((double2*)q), H((double2*)y), z ? H((double2*)z) : NONE, a->part, st);
    return sums(dot, nrm);
  };
  const std::vector<zd> one(nrhs, zd(1, 0)), zero(nrhs, zd(0, 0)), mone(nrhs, zd(-1, 0));
  // block solves of the preconditioner
  sap_solve_opts bo = *o;
  bo.tol = o->inner_tol;
  bo.inner_tol = o->inner_prec == SAP_F32   ? std::max(o->inner_tol, 1e-5)
                 : o->inner_prec == SAP_F16 ? std::max(o->inner_tol, 2e-3)
                                            : o->inner_tol;
  bo.max_outer = 40;
  bo.max_iter = 1 << 30;
  bo.method = SAP_CG;
  long long block_iters = 0;
  std::vector<sap_solve_info> binfo((size_t)nrhs * (c->geom.L[0] / c->geom.l0));
  // the preconditioner's fixed updates kr = in - M kx (0, 1, -1) and kx += ky (1, 1, 0),
  // uploaded once so that applying K needs no host synchronisation
  for (int sys = 0; sys < nh; ++sys) {
    const double res_c[6] = {0, 0, 1, 0, -1, 0}, add_c[6] = {1, 0, 1, 0, 0, 0};
    for (int e = 0; e < 6; ++e) {
      a->hcoef[6 * sys + e] = res_c[e];
      a->hcoef[6 * nh + 6 * sys + e] = add_c[e];
    }
  }
  SAP_HIP_CHECK(c, hipMemcpyAsync(a->ck_res, a->hcoef, 6 * nh * 8, hipMemcpyHostToDevice, st));
  SAP_HIP_CHECK(c, hipMemcpyAsync(a->ck_add, a->hcoef + 6 * nh, 6 * nh * 8, hipMemcpyHostToDevice, st));
  SAP_HIP_CHECK(c, hipStreamSynchronize(st));
  // out = K in
  auto K = [&](double2* out, const double2* in) -> int {
    SAP_HIP_CHECK(c, hipMemsetAsync(a->kx, 0, fullb, st));
    for (int cyc = 0; cyc < o->sap_ncy; ++cyc)
      for (int col = 0; col < 2; ++col) {
        const int colour = col == 0 ? SAP_BLACK : SAP_WHITE;
        const double* rhs = (const double*)in;
        if (cyc > 0 || col > 0) {
          int rc = apply_op_any(c, a->mt, a->kx, nrhs, 0, 0, -1, SAP_F64, st);
          if (rc) return rc;
          blas_lin3<double>(G, nh, H(a->kr), H((double2*)in), H(a->mt), NONE, a->ck_res, nullptr, st);
          rhs = (const double*)a->kr;
        }
        if (o->sap_block_terms > 0) {
          // y = the first N terms of the even-odd geometric series of W1 y = rhs on the blocks
          // of this colour (Horner form y_e <- b_hat_e + k^2 D_eo D_oe y_e), then
          // y_o = rhs_o + k D_oe y_e; every other block of y is set to zero
          const Field<double> RHS = full_field<double>((void*)rhs, Vhp), Y = full_field<double>(a->ky, Vhp);
          const Field<double> BH = full_field<double>(a->g1, Vhp), Z = full_field<double>(a->g2, Vhp);
          const Field<double> NONE64 = {nullptr, 0, 0, 0};
          const double kap = c->geom.kappa;
          const int lb = c->geom.l0;
          hop<double>(c, gauge_of<double>(c), BH, RHS, RHS, 0, nrhs, lb, colour, 1.0, kap, 0, 0, st);
          hop<double>(c, gauge_of<double>(c), Y, RHS, RHS, 0, nrhs, lb, colour, 1.0, kap, 0, 0, st);
          for (int n = 1; n < o->sap_block_terms; ++n) {
            hop<double>(c, gauge_of<double>(c), Z, Y, NONE64, 1, nrhs, lb, colour, 0.0, 1.0, 0, 0, st);
            hop<double>(c, gauge_of<double>(c), Y, Z, BH, 0, nrhs, lb, colour, 1.0, kap * kap, 0, 0, st);
          }
          hop<double>(c, gauge_of<double>(c), Y, Y, RHS, 1, nrhs, lb, colour, 1.0, kap, 0, 0, st);
          SAP_HIP_CHECK(c, hipGetLastError());
        } else {
          int rc = o->inner_prec == SAP_F64
                       ? solve_impl<double>(c, (double*)a->ky, rhs, nrhs, c->geom.l0, colour, &bo, binfo.data(), st)
                   : o->inner_prec == SAP_F32
                       ? solve_impl<float>(c, (double*)a->ky, rhs, nrhs, c->geom.l0, colour, &bo, binfo.data(), st)
                       : solve_impl<h16>(c, (double*)a->ky, rhs, nrhs, c->geom.l0, colour, &bo, binfo.data(), st);
          if (rc) return rc;
          for (auto& e : binfo) block_iters += e.iters;
        }
        blas_lin3<double>(G, nh, H(a->kx), H(a->ky), NONE, NONE, a->ck_add, nullptr, st);
        SAP_HIP_CHECK(c, hipGetLastError());
      }
    SAP_HIP_CHECK(c, hipMemcpyAsync(out, a->kx, fullb, hipMemcpyDeviceToDevice, st));
    return SAP_OK;
  };

  SAP_HIP_CHECK(c, hipMemsetAsync(x, 0, fullb, st));
  {
    std::vector<zd> d(nrhs);
    int rc = cdot((const double2*)b, (const double2*)b, nullptr, d, bb);
    if (rc) return rc;
    for (int r = 0; r < nrhs; ++r) bb[r] = d[r].real();
  }
  const double tol2 = o->tol * o->tol;
  int status = SAP_OK, restarts = 0;
  long long total = 0;
  for (;;) {
    // r = b - M x ; r0 = r
    int rc = apply_op_any(c, a->mt, x, nrhs, 0, 0, -1, SAP_F64, st);
    if (rc) return rc;
    SAP_HIP_CHECK(c, hipMemcpyAsync(a->r, b, fullb, hipMemcpyDeviceToDevice, st));
    std::vector<zd> rn(nrhs);
    if ((rc = lin3(a->r, a->mt, nullptr, a->r, one, mone, zero, true))) return rc;
    if ((rc = sums(rn, rr))) return rc;
    bool done = true, finite = true;
    for (int r = 0; r < nrhs; ++r) {
      if (!std::isfinite(rr[r])) finite = false;
      act[r] = bb[r] > 0 && rr[r] > tol2 * bb[r];
      if (act[r]) done = false;
    }
    if (!finite) { status = sap_fail(c, SAP_E_NONFINITE, "non-finite residual"); break; }
    if (done) break;
    if (restarts >= o->max_outer || total >= o->max_iter) {
      status = sap_fail(c, SAP_E_NOCONV, "solver did not reach tol within max_outer / max_iter");
      break;
    }
    ++restarts;
    SAP_HIP_CHECK(c, hipMemcpyAsync(a->r0, a->r, fullb, hipMemcpyDeviceToDevice, st));
    SAP_HIP_CHECK(c, hipMemsetAsync(a->p, 0, fullb, st));
    SAP_HIP_CHECK(c, hipMemsetAsync(a->v, 0, fullb, st));
    for (int r = 0; r < nrhs; ++r) rho[r] = alpha[r] = omega[r] = zd(1, 0);
    // rn holds <r0, r> = ||r||^2 at the start
    for (int r = 0; r < nrhs; ++r) rn[r] = zd(rr[r], 0);
    while (total < o->max_iter) {
      bool any = false;
      std::vector<zd> beta(nrhs), mbo(nrhs);
      for (int r = 0; r < nrhs; ++r) {
        if (act[r] && (rr[r] <= tol2 * bb[r] || std::abs(rho[r]) == 0 || std::abs(omega[r]) == 0 ||
                       std::abs(rn[r]) == 0))
          act[r] = 0;
        beta[r] = act[r] ? (rn[r] / rho[r]) * (alpha[r] / omega[r]) : zd(0, 0);
        mbo[r] = -beta[r] * omega[r];
        if (act[r]) rho[r] = rn[r];
        any = any || act[r];
      }
      if (!any) break;
      // p = r + beta (p - omega v) ; ph = K p ; v = M ph
      if ((rc = lin3(a->p, a->r, a->v, nullptr, beta, one, mbo, false))) return rc;
      if ((rc = K(a->ph, a->p))) return rc;
      if ((rc = apply_op_any(c, a->v, a->ph, nrhs, 0, 0, -1, SAP_F64, st))) return rc;
      std::vector<zd> den(nrhs), ma(nrhs), dts(nrhs), mo(nrhs), al_c(nrhs), om_c(nrhs);
      std::vector<double> dummy(nrhs), tt(nrhs);
      if ((rc = cdot(a->r0, a->v, nullptr, den, dummy))) return rc;
      for (int r = 0; r < nrhs; ++r) {
        if (act[r] && std::abs(den[r]) == 0) act[r] = 0;
        alpha[r] = act[r] ? rho[r] / den[r] : zd(0, 0);
        ma[r] = -alpha[r];
      }
      // s = r - alpha v (in r) ; sh = K s ; t = M sh ; omega = <t, s> / <t, t>
      if ((rc = lin3(a->r, a->v, nullptr, nullptr, one, ma, zero, false))) return rc;
      if ((rc = K(a->sh, a->r))) return rc;
      if ((rc = apply_op_any(c, a->t, a->sh, nrhs, 0, 0, -1, SAP_F64, st))) return rc;
      if ((rc = cdot(a->t, a->r, a->t, dts, tt))) return rc;
      for (int r = 0; r < nrhs; ++r) {
        omega[r] = (act[r] && tt[r] > 0) ? dts[r] / tt[r] : zd(0, 0);
        mo[r] = -omega[r];
        al_c[r] = alpha[r];
        om_c[r] = omega[r];
        if (act[r]) its[r] += 1;
      }
      // x += alpha ph + omega sh ; r = s - omega t, with <r0, r> and ||r||^2
      if ((rc = lin3((double2*)x, a->ph, a->sh, nullptr, one, al_c, om_c, false))) return rc;
      if ((rc = lin3(a->r, a->t, nullptr, a->r0, one, mo, zero, true))) return rc;
      if ((rc = sums(rn, rr))) return rc;
      for (int r = 0; r < nrhs; ++r)
        if (!std::isfinite(rr[r])) return sap_fail(c, SAP_E_NONFINITE, "non-finite value in BiCGstab");
      ++total;
    }
  }
  if (info) {
    // true residuals (the loop above ends with them in rr)
    for (int r = 0; r < nrhs; ++r) {
      info[r].iters = its[r];
      info[r].outer = restarts;
      info[r].true_rel_res = bb[r] > 0 ? std::sqrt(rr[r] / bb[r]) : 0.0;
    }
  }
  (void)block_iters;
  return status;
}

// (M_hat + rho) x_e = b_e on the blocks of length lb (0: full lattice), even sites only
int sap_solve_eo_shift(sap_ctx* c, double* x, const double* b, int nrhs, int lb, double rho,
                       const sap_solve_opts* o, sap_solve_info* info, hipStream_t st) {
  if (o->method == SAP_SAP_BICGSTAB) return sap_fail(c, SAP_E_ARG, "SAP_SAP_BICGSTAB solves M x = b only");
  if (o->inner_prec == SAP_F64) return solve_impl<double>(c, x, b, nrhs, lb, 0, o, info, st, rho, true);
  if (o->inner_prec == SAP_F32) return solve_impl<float>(c, x, b, nrhs, lb, 0, o, info, st, rho, true);
  return solve_impl<h16>(c, x, b, nrhs, lb, 0, o, info, st, rho, true);
}

int sap_solve_any(sap_ctx* c, double* x, const double* b, int nrhs, int lb, int colour,
                  const sap_solve_opts* o, sap_solve_info* info, hipStream_t st) {
  if (o->method == SAP_SAP_BICGSTAB) {
    if (lb != 0) return sap_fail(c, SAP_E_ARG, "SAP_SAP_BICGSTAB solves the full lattice only");
    return sap_bicgstab(c, x, b, nrhs, o, info, st);
  }
  if (o->inner_prec == SAP_F64) return solve_impl<double>(c, x, b, nrhs, lb, colour, o, info, st);
  if (o->inner_prec == SAP_F32) return solve_impl<float>(c, x, b, nrhs, lb, colour, o, info, st);
  return solve_impl<h16>(c, x, b, nrhs, lb, colour, o, info, st);
}

extern "C" {

int solve_full(sap_ctx* c, double* x, const double* b, int nrhs, const sap_solve_opts* o,
               sap_solve_info* info, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!x || !b) return sap_fail(c, SAP_E_ARG, "x or b is NULL");
  if (x == b) return sap_fail(c, SAP_E_ARG, "x and b must not alias");
  if (nrhs < 1 || nrhs > c->geom.max_rhs) return sap_fail(c, SAP_E_ARG, "nrhs must be in [1, max_rhs]");
  int rc = check_solve_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  return sap_solve_any(c, x, b, nrhs, 0, 0, o, info, (hipStream_t)stream);
}

int solve_blocks(sap_ctx* c, double* x, const double* b, int nrhs, int level, sap_color color, int block,
                 const sap_solve_opts* o, sap_solve_info* info, void* stream) {
  if (!c) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!x || !b) return sap_fail(c, SAP_E_ARG, "x or b is NULL");
  if (x == b) return sap_fail(c, SAP_E_ARG, "x and b must not alias");
  if (nrhs < 1 || nrhs > c->geom.max_rhs) return sap_fail(c, SAP_E_ARG, "nrhs must be in [1, max_rhs]");
  int lb;
  if (level == 1) lb = c->geom.l0;
  else if (level == 2 && c->geom.l0_sub > 0) lb = c->geom.l0_sub;
  else return sap_fail(c, SAP_E_ARG, "level must be 1, or 2 with l0_sub set");
  if (color != SAP_ALL && color != SAP_BLACK && color != SAP_WHITE)
    return sap_fail(c, SAP_E_ARG, "unknown colour");
  if (block < -1 || block >= c->geom.L[0] / lb) return sap_fail(c, SAP_E_ARG, "block out of range");
  int rc = check_solve_opts(c, o);
  if (rc) return rc;
  if (!c->have_gauge) return sap_fail(c, SAP_E_STATE, "no gauge field set");
  const int sel = block >= 0 ? 3 + block : (int)color;
  return sap_solve_any(c, x, b, nrhs, lb, sel, o, info, (hipStream_t)stream);
}

}  // extern "C"
