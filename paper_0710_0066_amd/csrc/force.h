// Launchers of the force / molecular-dynamics kernels (force.hip).
#pragma once
#include "internal.h"
#include "link_copies.h"

namespace sap {
// F += c * Im tr(lambda^a Q) per link (c = -kappa * coef), W = M (lb = 0) or x0 blocks of lb
// sx (device, [L0][4], or null): per-link step scale s_mu(x0) multiplying c
void launch_pair_force(const Geo& g, double* F, double c, const double2* a, const double2* b,
                       const double2* U, int lb, hipStream_t s, const double* sx = nullptr);
// F += c * Im tr(lambda^a U A) (c = coef * beta / 6)
void launch_gauge_force(const Geo& g, double* F, double c, const double2* U, hipStream_t s,
                        const double* sx = nullptr);
// out = in translated by n slices in x0 (out(x0) = in(x0 + n)); out != in
void launch_shift_links(const Geo& g, double2* out, const double2* in, int n, hipStream_t s);
// out[0] = sum_x sum_{mu>nu} Re tr U_P (part: ceil(Vh/128) doubles of scratch)
void launch_plaq_sum(const Geo& g, const double2* U, double* part, double* out, hipStream_t s);
// out[0] = max over the links of max(max_e |(U U^+ - 1)_e|, |det U - 1|) (NaN if any is NaN)
void launch_su3_dev(const Geo& g, const double2* U, double* part, double* out, hipStream_t s);
void launch_kinetic(const Geo& g, const double* P, double* part, double* out, hipStream_t s);
void launch_norm2_full(const Geo& g, const double2* f, double* part, double* out, hipStream_t s);
// U <- exp(dt P) U on every link (scaled per link by sx when given), also writing the
// reduced copies lc of the updated links (write_link_copies)
void launch_update_links(const Geo& g, double2* U, const LinkCopies& lc, const double* P, double dt, hipStream_t s,
                         const double* sx = nullptr);
// mode 0: gamma5; 1: Pi (black-boundary projector, blocks of l0); 2: keep white blocks; 3: in - Pi in2.
// outer > 0: Pi keeps only the boundary slices whose crossing hop exists in W_outer.
void launch_spin_op(const Geo& g, int mode, int l0, double2* out, const double2* in, const double2* in2,
                    hipStream_t s, int outer = 0);
// out = a x + b y (FP64 spinor fields, both parities)
void launch_lincomb(const Geo& g, double2* out, double a, const double2* x, double b, const double2* y,
                    hipStream_t s);
// x0 profile of |F| (out: [2][L0], spatial then time means; part: 2 * L0 * nck doubles
// with nck = force_profile_nck(g))
int force_profile_nck(const Geo& g);
void launch_force_profile(const Geo& g, const double* F, double* part, double* out, hipStream_t s);
void launch_axpy_mom(const Geo& g, double* p, double c, const double* F, hipStream_t s);
}  // namespace sap
