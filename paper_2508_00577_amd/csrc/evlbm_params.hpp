// Model parameters as the kernels take them (shared by the lattice and batch
// sources).
#pragma once

#include "lbm_device.hpp"

namespace evlbm {

template <typename R>
inline StepParams<R> model_params(int eos, double Rg, double a, double b, double kappa, double tau, double lambda,
                                  double sphi, double prandtl = 1.0)
{
    StepParams<R> p;
    p.nx = p.ny = p.nz = 1;
    p.N = 1;
    p.ds = 1;
    p.eos = eos;
    p.a = (R)a;
    p.b = (R)b;
    p.kappa = (R)kappa;
    const double beta = 1.0 / (2.0 * tau + 1.0);  // eq. beta with dt = 1
    p.two_beta = (R)(2.0 * beta);
    p.wstar = (R)((1.0 / lambda) * (1.0 - beta));
    // energy populations relax with tau_g = tau/Pr (Pr = 1: the same beta)
    const double beta_g = prandtl == 1.0 ? beta : 1.0 / (2.0 * tau / prandtl + 1.0);
    p.two_beta_g = (R)(2.0 * beta_g);
    p.wstar_g = (R)((1.0 / lambda) * (1.0 - beta_g));
    p.qe = (R)(2.0 * (beta_g - beta));
    p.vpr = prandtl != 1.0 ? 1 : 0;
    p.lambda = (R)lambda;
    p.sphi = (R)sphi;
    p.Rgas = (R)Rg;
    p.refst = nullptr;
    return p;
}

}  // namespace evlbm
