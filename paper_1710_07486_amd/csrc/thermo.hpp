// thermo.hpp -- host thermodynamics of the Carnahan-Starling EOS (Eq. 4).
#pragma once

namespace telbm {

double cs_pressure(double a, double b, double R, double T, double rho);
double cs_mu(double a, double b, double R, double T, double rho);
bool critical_point(double a, double b, double R, double* Tc, double* rho_c);
bool maxwell(double a, double b, double R, double T, double* rho_g, double* rho_l, double* C, double* Psi0);
bool temperature_for_ratio(double a, double b, double R, double ratio, double* T);

}  // namespace telbm
