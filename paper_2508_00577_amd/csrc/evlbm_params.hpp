// Model parameters as the kernels take them (shared by the lattice and batch
// sources).
#pragma once

#include "lbm_device.hpp"

namespace evlbm {

void reference_populations(int D, double R, double b, double rho, double T, double out[54]);

template <typename R>
inline StepParams<R> model_params(int D, int storage, double Rg, double a, double b, double kappa, double tau,
                                  double lambda, double sphi, double ref_rho, double ref_T)
{
    StepParams<R> p;
    p.nx = p.ny = p.nz = 1;
    p.N = 1;
    p.ds = 1;
    p.a = (R)a;
    p.b = (R)b;
    p.kappa = (R)kappa;
    const double beta = 1.0 / (2.0 * tau + 1.0);  // eq. beta with dt = 1
    p.two_beta = (R)(2.0 * beta);
    p.wstar = (R)((1.0 / lambda) * (1.0 - beta));
    p.lambda = (R)lambda;
    p.sphi = (R)sphi;
    p.Rgas = (R)Rg;
    double ref[54];
    if (storage == EVLBM_F16DEV || storage == EVLBM_BF16DEV) {
        // per unit density: the equilibrium at rest is proportional to rho at
        // fixed theta and RT
        reference_populations(D, Rg, b, ref_rho, ref_T, ref);
        for (int i = 0; i < 54; ++i) ref[i] /= ref_rho;
    } else {
        for (int i = 0; i < 54; ++i) ref[i] = 0.0;
    }
    for (int i = 0; i < 54; ++i) p.ref[i] = (R)ref[i];
    p.refrho = nullptr;
    return p;
}

}  // namespace evlbm
