/*
 * sapmi.h - C ABI of the MI355X (gfx950) library for the hot path of the
 * Schwarz-preconditioned two-flavour HMC with a one-dimensional (x0-only) domain
 * decomposition (M. Hasenbusch, Lattice 2007, arXiv:0710.0066).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice (Sec. 1): sites x = (x0, x1, x2, x3), 0 <= x_mu < L_mu, lexicographic index
 *   i = ((x0*L1 + x1)*L2 + x2)*L3 + x3 (x0 slowest), parity p(x) = (x0+x1+x2+x3) mod 2.
 *   Gauge links periodic; fermion hops periodic in space and antiperiodic in x0.
 *   All L_mu must be even.
 * Gamma matrices (Sec. 1, eq. 2 leaves the representation open): chiral basis,
 *   gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i sigma_k],[i sigma_k,0]] (2x2 blocks),
 *   gamma_5 = diag(1,1,-1,-1).
 * x0 blocks (Sec. 1, one-dimensional decomposition): level 1 has blocks of l0 slices,
 *   level 2 of l0_sub slices; block b = floor(x0 / l). Colours: black = odd b.
 *   Requires L0 % (2*l0) == 0 and l0 >= 2; level 2 requires l0 % (2*l0_sub) == 0 and
 *   l0_sub >= 2.
 *
 * Canonical interchange layout (device memory, complex128 = two float64):
 *   gauge   U[i][mu][row][col]                 9 complex per link
 *   spinor  psi[rhs][i][spin][colour]          12 complex per site and rhs
 *   force   F[i][mu][a] (float64, a = 0..7)    coefficients on T^a = lambda^a / 2
 * Library field layout ("sap layout"), used by every hot entry point: even-odd,
 *   tiled structure of arrays. Within a parity, site j = i / 2; sites are grouped in
 *   tiles of 64 (j / 64), Vhp = V/2 rounded up to a multiple of 64.
 *   spinor  complex number (rhs, parity, c = 3*spin + colour, j) at index
 *           ((rhs*2 + parity)*12*Vhp) + ((j/64)*12 + c)*64 + j%64   (SAP_F64, complex128)
 *           ((rhs*2 + parity)*12*Vhp) + ((j/64)*12 + c - c%2)*64 + 2*(j%64) + c%2
 *                                                                   (SAP_F32, complex64:
 *           the components 2k and 2k + 1 of a site are adjacent, one 16-byte word).
 *           SAP_F16: a half-precision complex (two FP16, 4 bytes) per entry at
 *           ((rhs*26 + parity*12)*Vhp) + ((j/64)*12 + c - c%4)*64 + 4*(j%64) + c%4
 *           (the components 4k .. 4k + 3 of a site are adjacent, one 16-byte word),
 *           rhs blocks of 26*Vhp entries: parity 0 and 1 components
 *           (24*Vhp), then one FP32 norm per (parity, j) at float index
 *           rhs*26*Vhp + 24*Vhp + parity*Vhp + j; a component's value is the stored one
 *           times the norm of its site (the largest component magnitude of the site).
 *   momentum / force (float64, a = 0..7) (parity, j, mu, a) at
 *           parity*32*Vhp + ((j/64)*32 + 8*mu + a)*64 + j%64.
 *   sap_field_bytes() / sap_momenta_bytes() give the sizes; sap_pack_* / sap_unpack_*
 *   convert from / to the canonical layout.
 *
 * Ownership and streams: every array argument is a DEVICE pointer allocated and freed
 * by the caller unless its comment says "host". The library never keeps a caller
 * pointer past the call. A context owns its gauge copies and workspace (allocated by
 * sap_create / sap_set_gauge; hot calls do not allocate). All work is queued on the
 * caller's HIP stream (passed as void*, NULL = default stream); calls that return
 * host scalars synchronise that stream before returning. A context is not
 * thread-safe; use one per stream.
 *
 * Errors: every call returns a sap_status; nothing aborts or throws across the ABI.
 * Argument checks run on the host before any HIP call. sap_last_error() describes
 * the last failure of a context.
 */
#ifndef SAPMI_H
#define SAPMI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sap_ctx sap_ctx;

typedef enum {
  SAP_OK = 0,
  SAP_E_ARG = -1,        /* invalid argument or geometry */
  SAP_E_NOMEM = -2,      /* device allocation failed */
  SAP_E_HIP = -3,        /* a HIP runtime call failed */
  SAP_E_NOCONV = -4,     /* solver stopped at max_iter / max_outer; info is filled */
  SAP_E_NONFINITE = -5,  /* NaN or Inf met in a residual */
  SAP_E_STATE = -6       /* call out of order (e.g. no gauge field set) */
} sap_status;

/* storage precision; arithmetic is FP64 for SAP_F64 and FP32 for SAP_F32. SAP_F16: FP16
 * spinors with a per-site FP32 norm and FP16 links; each hop term projects the stored
 * halves with one FP16 rounding and multiplies them by the link in FP16 x FP16 products
 * (exact in FP32) summed in FP32; accumulation, norms and BLAS work are FP32 */
typedef enum { SAP_F64 = 0, SAP_F32 = 1, SAP_F16 = 2 } sap_prec;
typedef enum { SAP_ALL = 0, SAP_BLACK = 1, SAP_WHITE = 2 } sap_color;

typedef struct {
  int L[4];          /* L0 (x0 extent) .. L3 */
  int l0;            /* level-1 block length along x0 */
  int l0_sub;        /* level-2 block length (0: level 2 unused) */
  double kappa;      /* hopping parameter of eq. 2 */
  int max_rhs;       /* largest nrhs any call will pass (sizes the workspace) */
} sap_geom;

/* Method of the inner solve (Sec. 3 names the geometric series for the block terms and
 * BiCGstab with even-odd and Schwarz preconditioning for the full-lattice term). */
typedef enum {
  SAP_CG = 0,           /* CG on the normal equations of the even-odd system (CGLS form) */
  SAP_BICGSTAB = 1,     /* BiCGstab on the even-odd system */
  SAP_GEOM = 2,         /* geometric series of the even-odd system: x_e = sum_n (k^2 D_eo D_oe)^n
                         * b_hat; SAP_E_NOCONV when it diverges (spectral radius >= 1) */
  SAP_SAP_BICGSTAB = 3  /* solve_full only: FP64 BiCGstab on M, right-preconditioned by
                         * sap_ncy cycles of the Schwarz alternating procedure on the
                         * level-1 blocks (black, then white); the block systems are solved
                         * with CG at inner_prec to the relative residual inner_tol
                         * (raised to 1e-5 for SAP_F32 and 2e-3 for SAP_F16), or by
                         * sap_block_terms terms of their geometric series */
} sap_method;

typedef struct {
  double tol;        /* stop when ||b - A x|| / ||b|| <= tol, recomputed in FP64 */
  int max_iter;      /* cap on inner iterations summed over outer cycles (SAP_SAP_BICGSTAB:
                      * on BiCGstab iterations) */
  sap_prec inner_prec; /* storage precision of the inner Krylov solve (FP32 arithmetic for
                        * SAP_F32; for SAP_F16 see sap_prec) */
  double inner_tol;  /* relative reduction asked of each inner solve (defect correction);
                      * must lie in (0, 1) for SAP_F32 and SAP_F16 (about 1e-5 and 2e-3
                      * suit their rounding); <= 0 with SAP_F64 means tol */
  int max_outer;     /* cap on FP64 defect-correction cycles (SAP_SAP_BICGSTAB: restarts) */
  sap_method method; /* inner method; 0 (SAP_CG) is the default */
  int sap_ncy;       /* SAP_SAP_BICGSTAB: Schwarz cycles per preconditioner application */
  int sap_block_terms; /* SAP_SAP_BICGSTAB: 0 solves every block system to inner_tol; N > 0
                        * applies the first N terms of the block systems' even-odd
                        * geometric series in FP64 instead (a fixed linear approximation
                        * of the block inverse; inner_prec and inner_tol are then unused) */
} sap_solve_opts;

typedef struct {
  int iters;            /* inner iterations in which this system was still active */
  int outer;            /* defect-correction cycles */
  double true_rel_res;  /* ||b - A x|| / ||b|| recomputed in FP64 at the end */
} sap_solve_info;

typedef struct {
  double beta;          /* gauge coupling of the Wilson plaquette action */
  double tau;           /* trajectory length */
  double lambda;        /* Sexton-Weingarten parameter (1/6 in the paper) */
  int n_outer;          /* steps of the pseudo-fermion level per trajectory */
  int n_inner;          /* gauge steps per pseudo-fermion step (even for SW) */
  int scheme_outer;     /* 0 leap-frog, 1 Sexton-Weingarten */
  int scheme_inner;
  sap_solve_opts force_solve;   /* solves inside the molecular dynamics */
  sap_solve_opts action_solve;  /* solves for the actions entering dH */
  const double* p0;     /* momenta, sap layout */
  const double* xi1;    /* heat-bath noise for phi1 = W1 xi1, canonical spinor */
  const double* xi2;    /* heat-bath noise for chi = R_hat Pi xi2, canonical spinor */
  double u_metropolis;  /* uniform number in [0,1) for the accept step */
  const double* step_scale; /* host [L0][4]: step of link (x0, mu) = dt * s (Sec. 2, x0-dependent
                            * step size; s = 0 freezes the link); NULL: s = 1 */
  int time_shift;       /* translate the resulting field by this many slices in x0
                         * (U'(x0) = U(x0 + n)) after the accept step (Sec. 2); 0: none */
} sap_hmc_params;

typedef struct {
  double dH, H0, H1;
  double S_G0, S_G1, S_W0, S_W1, S_R0, S_R1;
  double plaq;          /* mean plaquette of the returned field */
  int accepted;
  long long solver_iters; /* inner iterations of every solve in the trajectory */
} sap_hmc_info;

/* Trajectory with the paper's four-part pseudo-fermion action (Sec. 1, end; Sec. 2):
 * det^2 M = det^2(M W1^-1) det^2(W1 W2^-1) det^2(W2eo W3eo^-1) det^2(W3eo), W3eo = W2eo + rho,
 * integrated on five levels: 0 gauge action, 1 S1 = ||W3eo^-1 phi1||^2,
 * 2 S2 = ||phi2 + rho W2eo^-1 phi2||^2, 3 S3 (Schwarz term of W1 over the level-2
 * blocks), 4 S4 (Schwarz term of M over the level-1 blocks). */
typedef struct {
  double beta, tau, lambda;
  double rho;             /* mass-preconditioning shift of W3eo */
  int n[5];               /* n_j: steps of level j inside one step of level j + 1
                           * (n_4: steps per trajectory), Table 1 */
  int scheme[5];          /* per level: 0 leap-frog, 1 Sexton-Weingarten (the paper: 1, 1,
                           * 0, 0, 0); a Sexton-Weingarten level j > 0 needs an even n_{j-1} */
  sap_solve_opts force_solve, action_solve;
  const double* p0;       /* momenta, sap layout (device) */
  const double* xi1;      /* heat-bath noise, canonical spinors (device): phi1 = W3eo P_e xi1, */
  const double* xi2;      /*   phi2 = W3eo^-1 W2eo P_e xi2, */
  const double* g3;       /*   chi3 = R_hat_2 Pi_2 g3, */
  const double* g4;       /*   chi4 = R_hat Pi g4 */
  double u_metropolis;
  const double* step_scale; /* host [L0][4] or NULL, as in sap_hmc_params */
  int time_shift;
  const sap_solve_opts* part_solve; /* host array of 8 entries, or NULL: the solves of S1..S4
                          * inside the molecular dynamics (entries 0..3) and for their heat
                          * baths and the actions in dH (entries 4..7); NULL gives force_solve /
                          * action_solve to every part. Sec. 3's assignment is SAP_GEOM for S1,
                          * S2 and S3 and SAP_SAP_BICGSTAB for S4. A part whose options name
                          * SAP_SAP_BICGSTAB solves its full-lattice systems (M x = b) with it
                          * and its block systems (the heat bath of S4) or even-site systems
                          * with even-odd BiCGstab under the same tolerances. */
} sap_hmc4_params;

typedef struct {
  double dH, H0, H1;
  double S0[5], S1[5];    /* (S_G, S1, S2, S3, S4) at the start and at the end */
  double plaq;
  int accepted;
  long long solver_iters;
} sap_hmc4_info;

/* ---- context ---------------------------------------------------------------- */

/* Version of this ABI (major*100 + minor): 102 (hop mapping 20 added; sap_tune writes 126
 * floats). */
int sap_version(void);

/* Host-only geometry check (no HIP call): SAP_OK or SAP_E_ARG. */
int sap_check_geom(const sap_geom* g);

/* Create a context on the current HIP device; allocates its gauge copies and the
 * solver workspace for g->max_rhs right-hand sides. *out = NULL on failure. */
int sap_create(const sap_geom* g, sap_ctx** out);
void sap_destroy(sap_ctx* ctx);
const char* sap_last_error(const sap_ctx* ctx);

/* Bytes of one spinor field of nrhs right-hand sides in the sap layout. */
size_t sap_field_bytes(const sap_ctx* ctx, sap_prec prec, int nrhs);
/* Bytes of one momentum / force field in the sap layout. */
size_t sap_momenta_bytes(const sap_ctx* ctx);

/* Load the gauge field from the canonical layout (device, complex128) into the
 * context's FP64 links and the FP64, FP32 and FP16 copies the hop kernels read. The links
 * must be SU(3): the hop copies keep the first two rows of each link and the hop kernels
 * of every precision rebuild the third from unitarity and unit determinant (the force,
 * gauge-force and link-update kernels read the whole FP64 links). Checked on the device:
 * if the largest entry modulus of U U^+ - 1 or |det U - 1| over all links exceeds 1e-10
 * (or is not finite) the call returns SAP_E_ARG and the context holds no gauge field
 * (later calls that need one return SAP_E_STATE) until a valid field is set.
 * Synchronises. */
int sap_set_gauge(sap_ctx* ctx, const double* U, void* stream);
/* Copy the context's FP64 gauge field back to the canonical layout. */
int sap_get_gauge(sap_ctx* ctx, double* U, void* stream);

/* Canonical complex128 spinor(s) -> sap layout at precision prec, and back. */
int sap_pack_spinor(sap_ctx* ctx, void* out, const double* in, int nrhs, sap_prec prec,
                    void* stream);
int sap_unpack_spinor(sap_ctx* ctx, double* out, const void* in, int nrhs, sap_prec prec,
                      void* stream);
/* Canonical float64 [i][mu][8] <-> sap-layout momentum / force field. */
int sap_pack_momenta(sap_ctx* ctx, double* out, const double* in, void* stream);
int sap_unpack_momenta(sap_ctx* ctx, double* out, const double* in, void* stream);

/* ---- operators ---------------------------------------------------------------- */

/* out = M in (Sec. 1, eq. 2) for nrhs fields in the sap layout at precision prec
 * (FP64: float64 arithmetic; FP32: float32 storage and arithmetic; FP16: FP16 storage
 * with per-site norms and FP16 links, FP16 products summed in float32 (see sap_prec), each
 * output site rounded once).
 * out and in must not overlap. */
int apply_M(sap_ctx* ctx, void* out, const void* in, int nrhs, sap_prec prec, void* stream);

/* out = W_level in: M with every hop between different x0 blocks of the given level
 * removed (Sec. 1, block decomposition; level 1: l0, level 2: l0_sub). Only sites of
 * the selected blocks are written with W in; every other site of out is set to zero.
 * block >= 0 selects that single block (color is then ignored), block = -1 selects
 * all blocks of the given colour. */
int apply_W1_block(sap_ctx* ctx, void* out, const void* in, int nrhs, int level, int block,
                   sap_color color, sap_prec prec, void* stream);

/* Even-odd hop (Sec. 1, W_eo: M = [[1, -kappa D_eo], [-kappa D_oe, 1]] in the (even, odd)
 * partition): on the sites of parity `parity` (0 even, 1 odd), out = D in, where D is
 * the hop sum of eq. 2 without the factor -kappa and without the unit term, reading `in`
 * on the other parity only. Sites of the other parity of out are not written. Fields:
 * nrhs fields in the sap layout at precision prec; out and in must not overlap. This is
 * the operator that the even-odd solvers apply four times per iteration. */
int apply_Dslash_eo(sap_ctx* ctx, void* out, const void* in, int nrhs, int parity, sap_prec prec,
                    void* stream);

/* Autotuner of the hop kernel for nrhs right-hand sides (1 <= nrhs <= max_rhs): times each
 * work-item mapping on this context's lattice for the full operator and the even-odd hop
 * in FP64 and FP32, and keeps the fastest for every later call with that nrhs (apply_M,
 * apply_W1_block, apply_Dslash_eo and the solvers). The mappings: 0 site (one rhs per
 * work-item), 1 lane4 (4 rhs sharing link loads within a wavefront), 2 wave4 (4 rhs on
 * the 4 wavefronts of a workgroup), 3 stream (even-odd hop only: x0-streaming, time
 * neighbours kept in registers, each input slice staged in LDS), 4..6 = 0..2 with the
 * workgroups rhs-slowest, 7 / 8 reg2 / reg4 (each loaded link applied to 2 / 4 rhs held in
 * registers), 9 / 10 reg2 / reg4 group-slowest, 11 / 12 / 13 march1 / 2 / 4 (regN with
 * each of the 8 XCDs owning 1/8 of every x0 slice and walking the slices in increasing
 * x0), 14 / 15 walk1 / walk2 (even-odd hop: each work-item walks 8 slices at a fixed
 * spatial site with 1 / 2 rhs, loads every time neighbour once and carries its
 * projection in registers; the full operator runs them as march1 / march2), 16 band1
 * (even-odd hop: each XCD owns a band of x0 slices and each work-item steps through it at
 * a fixed spatial site, loading every input once and carrying the time hops in registers;
 * the full operator runs it as march1), 17 / 18 / 19 slab1 / slab1w / slab2 (even-odd hop:
 * band order with a workgroup owning a spatial tile of every slice of the band, TA x1
 * values by TB x2 values by all of x3, staged in LDS so that the spatial hops inside the
 * tile read the LDS copy; 1 rhs per work-item with tiles of up to 40 KB / 80 KB of LDS
 * (slab1 / slab1w) or 2 rhs per work-item (slab2); the full operator runs them as march1 /
 * march1 / march2), 20 slabd (even-odd FP32 / FP16 hop: the slab order with each slice of the
 * tile and its x1 / x2 halo staged in LDS by direct memory-to-LDS loads, so that every
 * spatial neighbour is read from LDS; FP64 runs it as slab1, the full operator as march1).
 * FP16 storage has site, march1 / 2 / 4 and slabd (even-odd hop only) (the other maps run
 * as march1 or march2).
 * us_out (host, may be NULL): 126 floats, microseconds per launch (-1: not applicable),
 * ordered [full f64, full f32, even-odd f64, even-odd f32, full f16, even-odd f16] x the
 * 21 mappings. Uses the solver
 * workspace; synchronises. Untuned calls use site for one rhs and lane4 (FP16: site) for
 * several. */
int sap_tune(sap_ctx* ctx, int nrhs, float* us_out, void* stream);

/* Set the hop mapping used for nrhs right-hand sides by hand (map: 0 site, 1 lane4,
 * 2 wave4, 3 stream (even-odd hop only, full = 0), 4..6 = 0..2 with rhs-slowest workgroup
 * order, 7 reg2, 8 reg4, 9 / 10 reg2 / reg4 group-slowest, 11 / 12 / 13 x0-marching with
 * 1 / 2 / 4 rhs per work-item, 14 / 15 x0-walking with 1 / 2 rhs (march1 / march2 for
 * the full operator), 16 x0-band (march1 for the full operator), 17 / 18 / 19 slab1 /
 * slab1w / slab2 (march1 / march1 / march2 for the full operator), 20 slabd (FP32 and FP16;
 * slab1 for FP64, march1 for the full operator); -1 restores the
 * default), for the full operator (full = 1) or the even-odd hop (full = 0) at precision
 * prec. */
int sap_set_hop_map(sap_ctx* ctx, int full, sap_prec prec, int nrhs, int map);

/* ---- solvers ------------------------------------------------------------------ */

/* Solve M x = b for nrhs FP64 fields (sap layout): the even-odd reduced system (the Schur
 * complement of Sec. 1's W_eo construction applied to M) solved by opts->method (CG on
 * the normal equations, BiCGstab or the geometric series) in opts->inner_prec inside an
 * FP64 defect-correction loop, or (SAP_SAP_BICGSTAB) Schwarz-preconditioned BiCGstab on
 * M, until ||b - M x|| / ||b|| <= opts->tol with M applied in FP64. x is overwritten (the
 * initial content is ignored). info: host array of nrhs entries (may be NULL).
 * Returns SAP_E_NOCONV if a system misses tol within the caps. Synchronises. */
int solve_full(sap_ctx* ctx, double* x, const double* b, int nrhs, const sap_solve_opts* opts,
               sap_solve_info* info, void* stream);

/* Solve W_level x = b on every selected block as an independent system (all selected
 * blocks and all nrhs fields batched in each kernel launch), by opts->method (SAP_CG,
 * SAP_BICGSTAB or SAP_GEOM; SAP_SAP_BICGSTAB is rejected). block >= 0 selects that
 * single block (color is then ignored), block = -1 all blocks of the colour. Sites
 * outside the selection are set to zero in x. info: host array of nblocks(level)*nrhs
 * entries ordered [rhs][block] (entries of unselected blocks are zeroed). Synchronises. */
int solve_blocks(sap_ctx* ctx, double* x, const double* b, int nrhs, int level,
                 sap_color color, int block, const sap_solve_opts* opts, sap_solve_info* info,
                 void* stream);

/* ---- forces -------------------------------------------------------------------- */

/* F += coef * dS/dw for S = ||W1^{-1} phi||^2 (Sec. 1, eq. factorpf with W = W1) along
 * U_mu(x) -> exp(i w T^a) U_mu(x); phi is one FP64 field (sap layout), F is a sap-layout
 * momentum field. *S_out (host, may be NULL) receives S. Synchronises. */
int block_pf_force(sap_ctx* ctx, double* F, double coef, const double* phi,
                   const sap_solve_opts* opts, double* S_out, void* stream);

/* F += coef * dS_R/dw for the Schwarz boundary action S_R = ||R_hat^{-1} chi||^2 of
 * det^2(W1^{-1} M) on the black-block boundaries (Sec. 1). chi: one FP64 field (sap
 * layout) that vanishes off the first/last slices of black level-1 blocks and lies in
 * the range of the spin projector (1 -/+ gamma_0)/2 there (checked: SAP_E_ARG).
 * *S_R_out (host, may be NULL) receives S_R. Needs two full solves. Synchronises. */
int schwarz_boundary_force(sap_ctx* ctx, double* F, double coef, const double* chi,
                           const sap_solve_opts* opts, double* S_R_out, void* stream);

/* Heat bath of the Schwarz boundary field (Sec. 1): chi = R_hat Pi g with
 *   R_hat = Pi - Pi D_Om^{-1} D_dOm D_Om*^{-1} D_dOm* Pi   (block solves only),
 * Omega = black level-1 blocks, D_Om / D_Om* = W1 on Omega / Omega*,
 * D_dOm* = P_Om* M P_Om, D_dOm = P_Om M P_Om*, Pi = (1 - gamma_0)/2 on the first and
 * (1 + gamma_0)/2 on the last slice of each black block. g: one FP64 field (sap layout),
 * normally Gaussian noise with density exp(-|g|^2); chi: output field (sap layout). */
int schwarz_heat_bath(sap_ctx* ctx, double* chi, const double* g, const sap_solve_opts* opts,
                      void* stream);

/* S_R = ||R_hat^{-1} chi||^2 with R_hat^{-1} chi = chi - Pi M^{-1} D_dOm* chi (one full
 * solve). chi as for schwarz_boundary_force. *S_R_out (host) receives S_R. */
int schwarz_action(sap_ctx* ctx, const double* chi, const sap_solve_opts* opts, double* S_R_out,
                   void* stream);

/* Gauge force of the Wilson plaquette action S_G (Sec. 1): F += coef * dS_G/dw.
 * *S_G_out (host, may be NULL) receives S_G. */
int gauge_force(sap_ctx* ctx, double* F, double coef, double beta, double* S_G_out,
                void* stream);

/* The link step T_U(dt) of Sec. 2, eq. 3 on the context's gauge field:
 * U_mu(x) <- exp(i dt P_mu(x)) U_mu(x), P = sum_a p^a T^a from the sap-layout momenta p
 * (FP64 exponential, reunitarised). */
int sap_update_links(sap_ctx* ctx, const double* p, double dt, void* stream);

/* x0 profile of a force (the analogue of Fig. 1 of Sec. 3, the average force on the spatial
 * links against x0). F (device): a force / momentum field in the sap momenta layout
 * (sap_momenta_bytes), e.g. the output of gauge_force, block_pf_force or
 * schwarz_boundary_force. prof (host, 2*L0 doubles) receives
 *   prof[x0]      = mean over the sites x of slice x0 and mu = 1, 2, 3 of |F(x, mu)|,
 *   prof[L0 + x0] = mean over the sites x of slice x0 of |F(x, 0)|,
 * |F| = (sum_a F^a F^a)^(1/2), the norm of the su(3) element in the T^a = lambda^a/2
 * basis. Fixed-order sums (deterministic); needs no gauge field; synchronises. */
int sap_force_profile(sap_ctx* ctx, const double* F, double* prof, void* stream);

/* Allocation-free variant of sap_force_profile, for callers that cannot allocate device
 * memory (code under HIP graph capture, loops that must not allocate). The same profile
 * as sap_force_profile, computed by the same kernels, but prof is a DEVICE array of 2*L0
 * doubles (same order) written on the stream, and the call does not synchronise. The
 * call allocates nothing: its partial sums live in one fixed array of
 * sap_force_profile_noalloc_max() doubles (2 MiB) per GPU, which the GPU holds until the
 * process ends. The lattice must need at most that many, 2*L0*ceil(L1*L2*L3/256)
 * (SAP_E_ARG otherwise). Every call on a GPU uses that GPU's array: calls that overlap
 * in time on one GPU (several streams, threads or contexts) race and give wrong profiles.
 * Errors: SAP_E_ARG (NULL pointer, lattice too large), SAP_E_STATE (array address not
 * resolved by sap_create on this device), SAP_E_HIP (launch failed). */
int sap_force_profile_noalloc(sap_ctx* ctx, const double* F, double* prof, void* stream);
/* Capacity, in doubles, of the fixed array of sap_force_profile_noalloc. */
size_t sap_force_profile_noalloc_max(void);

/* Translate the context's gauge field by n slices in x0: U'(x0, ...) = U(x0 + n, ...)
 * (Sec. 2: shift after each trajectory for ergodicity of the inactive links). */
int sap_shift_gauge(sap_ctx* ctx, int n, void* stream);

/* Mean plaquette (1/6V) sum_{x, mu>nu} (1/3) Re Tr U_P of the context's gauge field (host
 * output). Synchronises. */
int sap_plaquette(sap_ctx* ctx, double* plaq_out, void* stream);

/* ---- the four-part action (Sec. 1, end) ------------------------------------------ */

/* Even-odd pseudo-fermion parts on the level-2 blocks (needs l0_sub > 0): W2eo =
 * 1 - k^2 D_eo D_oe with the hops of the level-2 blocks, on the even sites; W3eo = W2eo +
 * rho (rho >= 0). kind 1: S1 = ||W3eo^-1 phi||^2; kind 2: S2 = ||phi + rho W2eo^-1 phi||^2
 * (= ||W2eo^-1 W3eo phi||^2). Fields are FP64 sap-layout spinors whose odd half is zero.
 * Heat bath: phi = W3eo P_e xi (kind 1) or W3eo^-1 W2eo P_e xi (kind 2), so that S equals
 * ||P_e xi||^2. Force: F += coef * dS/dw (F NULL: action only); *S_out (host, may be
 * NULL) receives S. Solves by opts on the even-site systems: CG, BiCGstab, or (SAP_GEOM, the
 * solver Sec. 3 uses for these parts) the geometric series
 * x = sum_n (k^2 D_eo D_oe / (1 + rho))^n b / (1 + rho), which converges where the spectral
 * radius of k^2 D_eo D_oe is below 1 + rho; SAP_SAP_BICGSTAB runs as BiCGstab. Synchronise. */
int eo_pf_heat_bath(sap_ctx* ctx, double* phi, const double* xi, int kind, double rho,
                    const sap_solve_opts* opts, void* stream);
int eo_pf_force(sap_ctx* ctx, double* F, double coef, const double* phi, int kind, double rho,
                const sap_solve_opts* opts, double* S_out, void* stream);

/* The factor det^2(W1 W2^-1): the Schwarz term of W1 over the level-2 blocks (needs
 * l0_sub > 0). Black level-2 blocks have odd index; Pi_2 is (1 - g0)/2 on the first and
 * (1 + g0)/2 on the last slice of each black level-2 block where W1 has the crossing hop
 * (a slice next to a level-1 block boundary has none and is left out).
 * Heat bath: chi = R_hat_2 Pi_2 g. Force: F += coef * dS/dw of S = ||R_hat_2^-1 chi||^2
 * (F NULL: action only; chi must lie in the range of Pi_2, else SAP_E_ARG). Synchronise. */
int schwarz2_heat_bath(sap_ctx* ctx, double* chi, const double* g, const sap_solve_opts* opts,
                       void* stream);
int schwarz2_force(sap_ctx* ctx, double* F, double coef, const double* chi, const sap_solve_opts* opts,
                   double* S_out, void* stream);

/* ---- HMC ------------------------------------------------------------------------ */

/* One HMC trajectory (Sec. 2) with two time scales: the outer level integrates
 * S_pf = ||W1^{-1} phi1||^2 + ||R_hat^{-1} chi||^2, the inner level the gauge action;
 * steps T_U: U -> exp(i dt P) U (FP64 exponential + reunitarisation) and
 * T_P: p -> p - dt F; leap-frog or Sexton-Weingarten per level; Metropolis with
 * p->u_metropolis, then the optional x0 translation. U: canonical gauge field, replaced
 * by the resulting field (the new one if accepted, else the old one, translated when
 * time_shift != 0); the context's gauge copies end equal to U. info: host. */
int hmc_trajectory(sap_ctx* ctx, double* U, const sap_hmc_params* p, sap_hmc_info* info,
                   void* stream);

/* One HMC trajectory with the four-part action on five time scales (Sec. 2: level j
 * integrates S_j, n_j steps of level j in one step of level j + 1, a trajectory is n_4
 * steps of level 4; Table 1 uses Sexton-Weingarten for levels 0, 1 and leap-frog for 2..4),
 * heat baths from the given noise, Metropolis with u_metropolis, optional x0-dependent
 * step sizes and translation as in hmc_trajectory. U: canonical gauge field, replaced by
 * the resulting one. Needs l0_sub > 0. info: host. */
int hmc_trajectory_4pf(sap_ctx* ctx, double* U, const sap_hmc4_params* p, sap_hmc4_info* info,
                       void* stream);

/* ---- benchmark aid ---------------------------------------------------------------- */

/* Streaming probe of the bandwidth a plain kernel reaches on this GPU, to set the hop
 * kernels against: mode 0 copies bytes from src to dst, mode 1 does the same with
 * non-temporal stores, mode 2 reads src and writes one float partial sum per workgroup to
 * dst (sap_stream_probe_blocks() floats). 16-byte accesses in a grid-stride loop of
 * sap_stream_probe_blocks() workgroups. bytes must be a positive multiple of 16 and both
 * pointers 16-byte aligned device pointers (SAP_E_ARG otherwise); queued on the stream,
 * no synchronisation. Needs no context. */
int sap_stream_probe(void* dst, const void* src, size_t bytes, int mode, void* stream);
int sap_stream_probe_blocks(void);

#ifdef __cplusplus
}
#endif
#endif /* SAPMI_H */
