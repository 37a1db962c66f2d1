// extern "C" entry points of libsapmi: argument checks (host only, before any HIP
// call), context lifetime, layout conversions and the operator calls. Solver, force
// and HMC entry points live in solver.hip, force.hip and hmc.hip.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include "internal.h"

using namespace sap;

static thread_local std::string g_noctx_err;

int sap_fail(sap_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_noctx_err = msg;
  return code;
}

static std::string geom_problem(const sap_geom* g) {
  if (!g) return "geometry pointer is NULL";
  for (int mu = 0; mu < 4; ++mu) {
    if (g->L[mu] < 2 || (g->L[mu] & 1))
      return "L[" + std::to_string(mu) + "] = " + std::to_string(g->L[mu]) + " must be even and >= 2";
    if (g->L[mu] > (1 << 16)) return "L[" + std::to_string(mu) + "] too large";
  }
  if (g->l0 < 2) return "l0 must be >= 2 (a black block needs distinct first and last slices)";
  if (g->L[0] % (2 * g->l0) != 0) return "L0 must be a multiple of 2*l0 (red/black blocks)";
  if (g->l0_sub != 0) {
    if (g->l0_sub < 2) return "l0_sub must be 0 (unused) or >= 2";
    if (g->l0 % (2 * g->l0_sub) != 0) return "l0 must be a multiple of 2*l0_sub";
  }
  if (!std::isfinite(g->kappa)) return "kappa must be finite";
  if (g->max_rhs < 1 || g->max_rhs > 64) return "max_rhs must be in [1, 64]";
  const long long V = (long long)g->L[0] * g->L[1] * g->L[2] * g->L[3];
  if (V / 2 / 128 * g->max_rhs > (1LL << 30)) return "lattice too large for one launch";
  return "";
}

extern "C" {

int sap_version(void) { return 102; }

int sap_check_geom(const sap_geom* g) {
  std::string p = geom_problem(g);
  if (!p.empty()) return sap_fail(nullptr, SAP_E_ARG, p);
  return SAP_OK;
}

const char* sap_last_error(const sap_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_noctx_err.c_str();
}

size_t sap_field_bytes(const sap_ctx* ctx, sap_prec prec, int nrhs) {
  if (!ctx || nrhs < 1) return 0;
  if (prec == SAP_F16) return full_bytes<h16>(ctx->Vhp, nrhs);
  const size_t per = prec == SAP_F64 ? sizeof(double2) : sizeof(float2);
  return (size_t)ctx->Vhp * 24 * per * (size_t)nrhs;
}

size_t sap_momenta_bytes(const sap_ctx* ctx) {
  if (!ctx) return 0;
  return (size_t)ctx->Vhp * 64 * sizeof(double);
}

void sap_solver_destroy(sap_ctx* ctx);   // solver.hip
void sap_sapws_destroy(sap_ctx* ctx);    // solver.hip
int sap_solver_create(sap_ctx* ctx);     // solver.hip
}  // extern "C"
int sap_force_create(sap_ctx* ctx);      // hmc.hip
void sap_force_destroy(sap_ctx* ctx);    // hmc.hip
int sap_noalloc_setup(sap_ctx* ctx);     // noalloc.hip
int su3_deviation_host(sap_ctx* c, double* dev, hipStream_t s);   // hmc.hip
extern "C" {

int sap_create(const sap_geom* g, sap_ctx** out) {
  if (!out) return sap_fail(nullptr, SAP_E_ARG, "out pointer is NULL");
  *out = nullptr;
  std::string p = geom_problem(g);
  if (!p.empty()) return sap_fail(nullptr, SAP_E_ARG, p);
  sap_ctx* c = new sap_ctx();
  c->geom = *g;
  c->g = make_geo(g->L);
  c->V = 2 * c->g.Vh;
  c->Vh = c->g.Vh;
  c->Vhp = c->g.Vhp;
  c->have_gauge = false;
  c->U64 = nullptr;
  c->U64c = nullptr;
  c->U32 = nullptr;
  c->U16 = nullptr;
  c->solver = nullptr;
  c->forces = nullptr;
  c->sapws = nullptr;
  std::memset(c->hop_map, -1, sizeof(c->hop_map));
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return sap_fail(nullptr, SAP_E_HIP, "hipGetDevice failed (no HIP device?)");
  }
  const size_t nlink = (size_t)72 * c->Vhp, nlink2 = (size_t)48 * c->Vhp;   // 2-row copies: 6 of 9
  if (hipMalloc((void**)&c->U64, nlink * sizeof(double2)) != hipSuccess ||
      hipMalloc((void**)&c->U64c, nlink2 * sizeof(double2)) != hipSuccess ||
      hipMalloc((void**)&c->U32, nlink2 * sizeof(float2)) != hipSuccess ||
      hipMalloc((void**)&c->U16, (nlink2 + nlink) * sizeof(__half2)) != hipSuccess) {   // 2-row + 3-row
    sap_destroy(c);
    return sap_fail(nullptr, SAP_E_NOMEM, "cannot allocate the gauge copies");
  }
  int rc = sap_solver_create(c);
  if (rc == SAP_OK) rc = sap_force_create(c);
  if (rc == SAP_OK) rc = sap_noalloc_setup(c);
  if (rc != SAP_OK) {
    std::string m = c->err;
    sap_destroy(c);
    return sap_fail(nullptr, rc, m);
  }
  *out = c;
  return SAP_OK;
}

void sap_destroy(sap_ctx* ctx) {
  if (!ctx) return;
  sap_sapws_destroy(ctx);
  sap_solver_destroy(ctx);
  sap_force_destroy(ctx);
  if (ctx->U64) (void)hipFree(ctx->U64);
  if (ctx->U64c) (void)hipFree(ctx->U64c);
  if (ctx->U32) (void)hipFree(ctx->U32);
  if (ctx->U16) (void)hipFree(ctx->U16);
  delete ctx;
}

int sap_set_gauge(sap_ctx* ctx, const double* U, void* stream) {
  if (!ctx) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!U) return sap_fail(ctx, SAP_E_ARG, "U is NULL");
  hipStream_t s = (hipStream_t)stream;
  ctx->have_gauge = false;
  launch_pack_gauge(ctx->g, ctx->U64, nullptr, (const double2*)U, s);
  launch_gauge_to_f32(ctx->g, ctx->U64c, ctx->U32, ctx->U16, ctx->U64, s);
  SAP_HIP_CHECK(ctx, hipGetLastError());
  // the hop kernels rebuild the third row of every link from the first two, which holds
  // for SU(3) only: refuse anything else
  double dev = 0.0;
  int rc = su3_deviation_host(ctx, &dev, s);
  if (rc) return rc;
  if (!(dev <= SAP_SU3_TOL)) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "links are not SU(3): max |U U^+ - 1|, |det U - 1| = %.3e > %.0e", dev,
                  SAP_SU3_TOL);
    return sap_fail(ctx, SAP_E_ARG, msg);
  }
  ctx->have_gauge = true;
  return SAP_OK;
}

int sap_get_gauge(sap_ctx* ctx, double* U, void* stream) {
  if (!ctx) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!U) return sap_fail(ctx, SAP_E_ARG, "U is NULL");
  if (!ctx->have_gauge) return sap_fail(ctx, SAP_E_STATE, "no gauge field set");
  launch_unpack_gauge(ctx->g, (double2*)U, ctx->U64, (hipStream_t)stream);
  SAP_HIP_CHECK(ctx, hipGetLastError());
  return SAP_OK;
}

static int check_fields(sap_ctx* ctx, const void* a, const void* b, int nrhs, int prec) {
  if (!ctx) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!a || !b) return sap_fail(ctx, SAP_E_ARG, "field pointer is NULL");
  if (nrhs < 1 || nrhs > ctx->geom.max_rhs)
    return sap_fail(ctx, SAP_E_ARG, "nrhs must be in [1, max_rhs]");
  if (prec != SAP_F64 && prec != SAP_F32 && prec != SAP_F16) return sap_fail(ctx, SAP_E_ARG, "unknown precision");
  return SAP_OK;
}

int sap_pack_spinor(sap_ctx* ctx, void* out, const double* in, int nrhs, sap_prec prec, void* stream) {
  int rc = check_fields(ctx, out, in, nrhs, prec);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (prec == SAP_F64) launch_pack_spinor<double>(ctx->g, (double2*)out, (const double2*)in, nrhs, s);
  else if (prec == SAP_F32) launch_pack_spinor<float>(ctx->g, (float2*)out, (const double2*)in, nrhs, s);
  else launch_pack_spinor16(ctx->g, (__half2*)out, (const double2*)in, nrhs, s);
  SAP_HIP_CHECK(ctx, hipGetLastError());
  return SAP_OK;
}

int sap_unpack_spinor(sap_ctx* ctx, double* out, const void* in, int nrhs, sap_prec prec, void* stream) {
  int rc = check_fields(ctx, out, in, nrhs, prec);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (prec == SAP_F64) launch_unpack_spinor<double>(ctx->g, (double2*)out, (const double2*)in, nrhs, s);
  else if (prec == SAP_F32) launch_unpack_spinor<float>(ctx->g, (double2*)out, (const float2*)in, nrhs, s);
  else launch_unpack_spinor16(ctx->g, (double2*)out, (const __half2*)in, nrhs, s);
  SAP_HIP_CHECK(ctx, hipGetLastError());
  return SAP_OK;
}

int sap_pack_momenta(sap_ctx* ctx, double* out, const double* in, void* stream) {
  if (!ctx) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!out || !in) return sap_fail(ctx, SAP_E_ARG, "pointer is NULL");
  launch_pack_momenta(ctx->g, out, in, (hipStream_t)stream);
  SAP_HIP_CHECK(ctx, hipGetLastError());
  return SAP_OK;
}

int sap_unpack_momenta(sap_ctx* ctx, double* out, const double* in, void* stream) {
  if (!ctx) return sap_fail(nullptr, SAP_E_ARG, "ctx is NULL");
  if (!out || !in) return sap_fail(ctx, SAP_E_ARG, "pointer is NULL");
  launch_unpack_momenta(ctx->g, out, in, (hipStream_t)stream);
  SAP_HIP_CHECK(ctx, hipGetLastError());
  return SAP_OK;
}

}  // extern "C"

namespace sap {

template <class R>
static void full_op(sap_ctx* ctx, void* out, const void* in, int nrhs, int lb, int colour,
                    int block, hipStream_t s) {
  HopArgs<R> A;
  typedef typename arith<R>::type Ar;
  const long long Vhp = ctx->Vhp;
  A.out = full_field<R>(out, Vhp);
  A.in = full_field<R>((void*)in, Vhp);
  A.x = A.in;
  A.U = gauge_of<R>(ctx);
  A.g = ctx->g;
  A.nrhs = nrhs;
  A.parity_out = -1;
  A.lb = lb;
  A.slb = lb;
  A.colour = colour;
  A.block = block;
  A.a = Ar(1);
  A.b = Ar(-ctx->geom.kappa);
  A.g5_in = 0;
  A.g5_out = 0;
  A.map = hop_map_for(ctx, true, prec_of<R>(), nrhs);
  launch_hop<R>(A, s);
}

template <class R>
static void eo_hop(sap_ctx* ctx, void* out, const void* in, int nrhs, int parity, hipStream_t s) {
  HopArgs<R> A;
  typedef typename arith<R>::type Ar;
  const long long Vhp = ctx->Vhp;
  A.out = full_field<R>(out, Vhp);
  A.in = full_field<R>((void*)in, Vhp);
  A.x = {nullptr, 0, 0, 0};
  A.U = gauge_of<R>(ctx);
  A.g = ctx->g;
  A.nrhs = nrhs;
  A.parity_out = parity;
  A.lb = 0;
  A.slb = 0;
  A.colour = 0;
  A.block = -1;
  A.a = Ar(0);
  A.b = Ar(1);
  A.g5_in = 0;
  A.g5_out = 0;
  A.map = hop_map_for(ctx, false, prec_of<R>(), nrhs);
  launch_hop<R>(A, s);
}

int eo_hop_any(sap_ctx* ctx, void* out, const void* in, int nrhs, int parity, sap_prec prec, hipStream_t s) {
  if (prec == SAP_F64) eo_hop<double>(ctx, out, in, nrhs, parity, s);
  else if (prec == SAP_F32) eo_hop<float>(ctx, out, in, nrhs, parity, s);
  else eo_hop<h16>(ctx, out, in, nrhs, parity, s);
  SAP_HIP_CHECK(ctx, hipGetLastError());
  return SAP_OK;
}

int apply_op_any(sap_ctx* ctx, void* out, const void* in, int nrhs, int lb, int colour, int block,
                 sap_prec prec, hipStream_t s) {
  if (prec == SAP_F64) full_op<double>(ctx, out, in, nrhs, lb, colour, block, s);
  else if (prec == SAP_F32) full_op<float>(ctx, out, in, nrhs, lb, colour, block, s);
  else full_op<h16>(ctx, out, in, nrhs, lb, colour, block, s);
  SAP_HIP_CHECK(ctx, hipGetLastError());
  return SAP_OK;
}

}  // namespace sap

extern "C" {

int apply_M(sap_ctx* ctx, void* out, const void* in, int nrhs, sap_prec prec, void* stream) {
  int rc = check_fields(ctx, out, in, nrhs, prec);
  if (rc) return rc;
  if (out == in) return sap_fail(ctx, SAP_E_ARG, "out and in must not alias");
  if (!ctx->have_gauge) return sap_fail(ctx, SAP_E_STATE, "no gauge field set");
  return apply_op_any(ctx, out, in, nrhs, 0, 0, -1, prec, (hipStream_t)stream);
}

int apply_Dslash_eo(sap_ctx* ctx, void* out, const void* in, int nrhs, int parity, sap_prec prec,
                    void* stream) {
  int rc = check_fields(ctx, out, in, nrhs, prec);
  if (rc) return rc;
  if (out == in) return sap_fail(ctx, SAP_E_ARG, "out and in must not alias");
  if (parity != 0 && parity != 1) return sap_fail(ctx, SAP_E_ARG, "parity must be 0 or 1");
  if (!ctx->have_gauge) return sap_fail(ctx, SAP_E_STATE, "no gauge field set");
  return eo_hop_any(ctx, out, in, nrhs, parity, prec, (hipStream_t)stream);
}

int apply_W1_block(sap_ctx* ctx, void* out, const void* in, int nrhs, int level, int block,
                   sap_color color, sap_prec prec, void* stream) {
  int rc = check_fields(ctx, out, in, nrhs, prec);
  if (rc) return rc;
  if (out == in) return sap_fail(ctx, SAP_E_ARG, "out and in must not alias");
  if (!ctx->have_gauge) return sap_fail(ctx, SAP_E_STATE, "no gauge field set");
  int lb;
  if (level == 1) lb = ctx->geom.l0;
  else if (level == 2 && ctx->geom.l0_sub > 0) lb = ctx->geom.l0_sub;
  else return sap_fail(ctx, SAP_E_ARG, "level must be 1, or 2 with l0_sub set");
  const int nb = ctx->geom.L[0] / lb;
  if (block < -1 || block >= nb) return sap_fail(ctx, SAP_E_ARG, "block out of range");
  if (color != SAP_ALL && color != SAP_BLACK && color != SAP_WHITE)
    return sap_fail(ctx, SAP_E_ARG, "unknown colour");
  return apply_op_any(ctx, out, in, nrhs, lb, (int)color, block, prec, (hipStream_t)stream);
}

}  // extern "C"
