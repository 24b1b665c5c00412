#pragma once

namespace lbt {

// Maxwell coexistence of p0 = rho T/(1 - b rho) - a rho^2 (equal p0 and mu).
bool vdw_coexistence(double a, double b, double T, double* rho_l, double* rho_g);

// Wall gradient (normal into the fluid) for an equilibrium contact angle.
bool binary_wall_gradient(double kappa, double A, double B, double theta_deg, double* G);
bool vdw_wall_gradient(double kappa, double a, double b, double T, double theta_deg, double* G);

}  // namespace lbt
