// Entry points whose implementation has not landed yet: they fail with SAP_E_STATE.
#include "internal.h"

extern "C" {
int block_pf_force(sap_ctx* c, double*, double, const double*, const sap_solve_opts*, double*, void*) {
  return sap_fail(c, SAP_E_STATE, "block_pf_force not available in this build");
}
int schwarz_boundary_force(sap_ctx* c, double*, double, const double*, const sap_solve_opts*, double*, void*) {
  return sap_fail(c, SAP_E_STATE, "schwarz_boundary_force not available in this build");
}
int gauge_force(sap_ctx* c, double*, double, double, double*, void*) {
  return sap_fail(c, SAP_E_STATE, "gauge_force not available in this build");
}
int hmc_trajectory(sap_ctx* c, double*, const sap_hmc_params*, sap_hmc_info*, void*) {
  return sap_fail(c, SAP_E_STATE, "hmc_trajectory not available in this build");
}
}
