// Host-side internals of libsapmi: the context, field descriptors and the launchers
// each translation unit provides.
#pragma once
#include <hip/hip_runtime.h>
#include <string>
#include <type_traits>
#include <vector>
#include "../../include/sapmi.h"
#include "device_common.h"

namespace sap {

// A spinor field in the library layout: element (rhs, parity, component c, site j) of
// complex type at  ptr + rhs*rs + parity*ps + sidx<R>(j, c)  (in complex numbers;
// tiled(j, c, 12) for FP64 and FP16, pairs of components per 16-byte word for FP32).
// Full fields: rs = 24*Vhp, ps = 12*Vhp. Single-parity fields: rs = 12*Vhp, ps = 0.
// FP16 (h16) fields also hold one FP32 norm per site: the components are stored divided
// by it, and the norms of (rhs, parity) start at  (float*)(ptr + rhs*rs + no) + parity*Vhp.
// Full FP16 fields: rs = 26*Vhp, ps = 12*Vhp, no = 24*Vhp; single-parity: rs = 13*Vhp,
// ps = 0, no = 12*Vhp (a half2 and a float are both 4 bytes).
// Gauge field: link (parity p, site j, mu, entry e = 3*row + col) at
//   p*36*Vhp + tiled(j, 9*mu + e, 36)   (FP64);
// the copies the hop kernels read (FP64, FP32, FP16) hold rows 0 and 1 only (e < 6), at
// p*24*Vhp + tiled(j, 6*mu + e, 24) (FP32: the entries of a tile row stored in pairs, one
// 16-byte word per lane; FP16: a quad and a pair of entries per link, see
// gauge_to_f32_kernel), and the kernels rebuild row 2 from
// unitarity and unit determinant.
// Momenta / forces (float64): (p, j, mu, a) at  p*32*Vhp + tiled(j, 8*mu + a, 32).
template <class R> struct Field {
  typename vec2<R>::type* ptr;
  long long rs;
  long long ps;
  long long no;            // FP16 only: offset of the norms in an rhs block (complex units)
};

// field descriptors of the library's full and single-parity fields for storage type S
template <class S> inline Field<S> full_field(void* p, long long Vhp) {
  if constexpr (std::is_same<S, h16>::value) return {(typename vec2<S>::type*)p, 26 * Vhp, 12 * Vhp, 24 * Vhp};
  else return {(typename vec2<S>::type*)p, 24 * Vhp, 12 * Vhp, 0};
}
template <class S> inline Field<S> half_field(void* p, long long Vhp) {
  if constexpr (std::is_same<S, h16>::value) return {(typename vec2<S>::type*)p, 13 * Vhp, 0, 12 * Vhp};
  else return {(typename vec2<S>::type*)p, 12 * Vhp, 0, 0};
}
// bytes of nrhs full / single-parity fields
template <class S> inline size_t full_bytes(long long Vhp, int nrhs) {
  if constexpr (std::is_same<S, h16>::value) return (size_t)26 * Vhp * nrhs * 4;
  else return (size_t)24 * Vhp * nrhs * sizeof(typename vec2<S>::type);
}
template <class S> inline size_t half_bytes(long long Vhp, int nrhs) {
  if constexpr (std::is_same<S, h16>::value) return (size_t)13 * Vhp * nrhs * 4;
  else return (size_t)12 * Vhp * nrhs * sizeof(typename vec2<S>::type);
}

template <class R> struct HopArgs {
  Field<R> out, in, x;     // out = a*x + b*D(in); x.ptr may be null
  const typename vec2<R>::type* U;   // gauge field in the tiled layout
  Geo g;
  int nrhs;
  int parity_out;          // -1: both parities (full operator); 0/1: that parity only
  int lb;                  // hops between x0 blocks of this length are dropped (0: none)
  int slb;                 // output restricted to x0 blocks of this length (0: all sites)
  int colour;              // selection for slb: 0 all, 1 black (odd b), 2 white (even b)
  int block;               // >= 0: only this block (colour ignored)
  typename arith<R>::type a, b;
  int g5_in, g5_out;       // multiply the hop input / the hop result by gamma_5
  int map;                 // work-item mapping (HOP_MAP_*), nrhs > 1 only
  // optional (HOP_MAP_SLABD only): per-system partial reductions of the output over
  // systems (rhs, block of nlb slices), nslot partials per system (see slabd_norm_slots):
  //   red = 1: ||out||^2 at npart[sys * nslot + k];
  //   red = 3: (Re, Im <out, x>, ||out||^2) with out conjugated, at
  //   npart[3 (sys * nslot + k) + i].
  double* npart = nullptr;
  int nlb = 0, nslot = 0, red = 0;
};

// Work-item mappings of the hop kernel for several right-hand sides.
enum { HOP_MAP_SITE = 0,    // one (site, rhs) per work-item, workgroups rhs-fastest
       HOP_MAP_LANE4 = 1,   // wavefront = 16 sites x 4 rhs: four lanes share each link load
       HOP_MAP_WAVE4 = 2,   // workgroup = 64 sites x 4 rhs, one rhs per wavefront
       HOP_MAP_STREAM = 3,  // half hop only: x0-streaming, input slice staged in LDS
       HOP_SWEEP = 4,       // added to SITE/LANE4/WAVE4: workgroups rhs(-group)-slowest, so
                            // each rhs sweeps the lattice like a single-rhs launch
       HOP_MAP_REG2 = 7,    // one work-item per site for 2 rhs held in registers: each
       HOP_MAP_REG4 = 8,    //   link is loaded once and applied to 2 (4) rhs
       HOP_MAP_REG2_SWEEP = 9,   // REG2 / REG4 with workgroups group-slowest: each group
       HOP_MAP_REG4_SWEEP = 10,  //   of rhs sweeps the lattice like a small-rhs launch
       HOP_MAP_MARCH1 = 11, // x0-marching: each XCD owns 1/8 of every x0 slice and walks the
       HOP_MAP_MARCH2 = 12, //   slices in order, 1 / 2 / 4 rhs per work-item (any nrhs for
       HOP_MAP_MARCH4 = 13, //   MARCH1)
       HOP_MAP_WALK1 = 14,  // even-odd hop only: x0-walking, time neighbours carried in
       HOP_MAP_WALK2 = 15,  //   registers, 1 / 2 rhs per work-item
       HOP_MAP_BAND1 = 16,  // even-odd hop only: each XCD owns a band of x0 slices, time
                            //   hops carried in registers, 1 rhs per work-item
       HOP_MAP_SLAB1 = 17,  // even-odd hop only: band order, a workgroup owns a spatial tile
       HOP_MAP_SLAB1W = 18, //   of the slice staged in LDS and walks the band; 1 rhs per
       HOP_MAP_SLAB2 = 19,  //   work-item (SLAB1W: tiles up to twice as large), or 2 (SLAB2)
       HOP_MAP_SLABD = 20,  // even-odd FP32 / FP16 hop only: the slab order with the slice
                            //   and its x1 / x2 halo staged in LDS by direct memory-to-LDS
                            //   loads, 1 rhs per work-item (FP64: as SLAB1)
       HOP_NMAP = 21 };
constexpr int HOP_WALK_T = 8;   // slices per walk

template <class R> void launch_hop(const HopArgs<R>& A, hipStream_t s);
// partials per system of the norm the LDS-staged slab kernel (HOP_MAP_SLABD, FP32 even-odd
// hop) can add to its output for systems of nlb slices
int slabd_norm_slots(const Geo& g, int nlb);
// the LDS-staged slab kernel on FP16 storage (even-odd hop; dslash.hip)
void launch_slabd16(const HopArgs<h16>& A, hipStream_t s);
template <> void launch_hop<h16>(const HopArgs<h16>& A, hipStream_t s);   // half.hip

// layout conversions
template <class R>
void launch_pack_spinor(const Geo& g, typename vec2<R>::type* out, const double2* in, int nrhs,
                        hipStream_t s);
template <class R>
void launch_unpack_spinor(const Geo& g, double2* out, const typename vec2<R>::type* in,
                          int nrhs, hipStream_t s);
void launch_pack_gauge(const Geo& g, double2* U64, float2* U32, const double2* in, hipStream_t s);
void launch_unpack_gauge(const Geo& g, double2* out, const double2* U64, hipStream_t s);
// the reduced link copies of the hop kernels from the FP64 links: two-row FP64, FP32 and
// FP16 copies, then the three-row FP16 copy of the LDS-staged FP16 hop (layouts in
// layout.hip)
void launch_gauge_to_f32(const Geo& g, double2* U64c, float2* U32, __half2* U16, const double2* U64, hipStream_t s);
void launch_pack_spinor16(const Geo& g, __half2* out, const double2* in, int nrhs, hipStream_t s);
void launch_unpack_spinor16(const Geo& g, double2* out, const __half2* in, int nrhs, hipStream_t s);
void launch_pack_momenta(const Geo& g, double* out, const double* in, hipStream_t s);
void launch_unpack_momenta(const Geo& g, double* out, const double* in, hipStream_t s);

inline Geo make_geo(const int L[4]) {
  Geo g;
  g.L0 = L[0]; g.L1 = L[1]; g.L2 = L[2]; g.L3 = L[3];
  g.L3h = L[3] / 2;
  g.V3h = L[1] * L[2] * L[3] / 2;
  g.Vh = (long long)L[0] * L[1] * L[2] * L[3] / 2;
  g.Vhp = (g.Vh + TILE - 1) / TILE * TILE;
  return g;
}

}  // namespace sap

struct sap_ctx {
  sap_geom geom;
  sap::Geo g;
  long long V, Vh, Vhp;
  int device;
  bool have_gauge;
  double2* U64;   // tiled gauge layout, 72*Vhp complex (whole links: forces, link updates)
  double2* U64c;  // two-row FP64 copy read by the hop kernels (48*Vhp complex)
  float2* U32;    // two-row FP32 copy
  __half2* U16;   // two-row FP16 copy (48*Vhp), then the three-row FP16 copy (72*Vhp) the
                  // LDS-staged FP16 hop reads (all copies kept in step with U64)
  std::string err;
  void* solver;   // solver workspace (solver.hip)
  void* forces;   // force / trajectory workspace (hmc.hip)
  void* sapws;    // Schwarz-preconditioned BiCGstab workspace (solver.hip), allocated by sap_create
  // tuned hop mapping per [full operator?][precision (sap_prec)][nrhs] (-1: not tuned)
  signed char hop_map[2][3][65];
};

// largest deviation from SU(3) (|U U^+ - 1| entries, |det U - 1|) sap_set_gauge accepts
constexpr double SAP_SU3_TOL = 1e-10;

// precision code (sap_prec) of a storage type
template <class S> constexpr int prec_of() {
  return std::is_same<S, double>::value ? SAP_F64 : std::is_same<S, float>::value ? SAP_F32 : SAP_F16;
}

// mapping used for a hop launch: the tuned (or set) one, else SITE for one rhs and LANE4
// for several (LANE4 is SITE for FP16 storage)
inline int hop_map_for(const sap_ctx* c, bool full, int prec, int nrhs) {
  const int m = c->hop_map[full ? 1 : 0][prec][nrhs > 64 ? 64 : nrhs];
  if (m >= 0) return m;
  return nrhs <= 1 ? sap::HOP_MAP_SITE : sap::HOP_MAP_LANE4;
}

// error helpers (api.hip)
int sap_fail(sap_ctx* ctx, int code, const std::string& msg);
#define SAP_HIP_CHECK(ctx, call)                                                     \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return sap_fail((ctx), SAP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace sap {
// validation of solve options shared by every entry point that solves (solver.hip)
int check_solve_opts(sap_ctx* c, const sap_solve_opts* o);
}

// the context's link copy for storage type S
template <class S> inline const typename sap::vec2<S>::type* gauge_of(const sap_ctx* c) {
  if constexpr (std::is_same<S, double>::value) return c->U64c;
  else if constexpr (std::is_same<S, float>::value) return c->U32;
  else return c->U16;
}
