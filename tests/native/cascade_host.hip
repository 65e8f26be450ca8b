// cascade_host.hip -- host build of the GPU path's per-node arithmetic
// (paper_1202_6351_amd/csrc/cascade.h, FP64 instantiation) for CPU tests
// against the oracle.  No kernels; exported as plain C for ctypes.
#include "cascade.h"

namespace {
lbm::Rates<double> rates_of(const double* w, double rho0) {
  return lbm::make_rates<double>(w, rho0);
}
}  // namespace

extern "C" {

// The step kernels' collision (force = 0: no body force).
void host_collide_step(const double* d, double Fx, double Fy, const double* w, double rho0, int force,
                       double* out) {
  if (force) lbm::collide_step<double, true>(rates_of(w, rho0), Fx, Fy, d, out);
  else lbm::collide_step<double, false>(rates_of(w, rho0), 0.0, 0.0, d, out);
}

// Transposed Jacobian of the collision at d (the adjoint kernels' collide_adj):
// ad = J_d^T aout, aF = J_F^T aout.
void host_collide_adj(const double* d, double Fx, double Fy, const double* w, double rho0, const double* aout,
                      double* ad, double* aF) {
  double ax = 0.0, ay = 0.0;
  lbm::collide_adj(rates_of(w, rho0), Fx, Fy, d, aout, ad, ax, ay);
  aF[0] = ax;
  aF[1] = ay;
}

// Initial-state deviations f^eq - S/2 - w rho0 of one node.
void host_init(double rho, double ux, double uy, double Fx, double Fy, double rho0, double* out) {
  double Cs[3][3], Y[3][3];
  lbm::equilibrium_cm(rho0, rho - rho0, ux, uy, -0.5 * Fx, -0.5 * Fy, Cs);
  lbm::populations(ux, uy, Cs, Y, out);
}

// Reverse of host_init: cotangent aout -> (a_rho, a_ux, a_uy, a_Fx, a_Fy).
void host_init_T(double rho, double ux, double uy, double Fx, double Fy, double rho0, const double* aout,
                 double* g) {
  double Cs[3][3], Y[3][3], v[9], aCs[3][3];
  lbm::equilibrium_cm(rho0, rho - rho0, ux, uy, -0.5 * Fx, -0.5 * Fy, Cs);
  lbm::populations(ux, uy, Cs, Y, v);
  double aux = 0, auy = 0, adrho = 0, ahx = 0, ahy = 0;
  lbm::populations_T(ux, uy, Cs, Y, aout, aCs, aux, auy);
  lbm::equilibrium_cm_T(rho0, ux, uy, aCs, adrho, aux, auy, ahx, ahy);
  g[0] = adrho;
  g[1] = aux;
  g[2] = auy;
  g[3] = -0.5 * ahx;
  g[4] = -0.5 * ahy;
}

}  // extern "C"
