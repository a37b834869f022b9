// thermo.hpp -- host thermodynamics of the liquid-gas equation of state of the
// bulk free energy: Carnahan-Starling (Eq. 4) and the van der Waals and
// Peng-Robinson alternatives the paper names beside it.
#pragma once

namespace telbm {

double cs_pressure(double a, double b, double R, double T, double rho);
double cs_mu(double a, double b, double R, double T, double rho);
bool critical_point(double a, double b, double R, double* Tc, double* rho_c);
bool maxwell(double a, double b, double R, double T, double* rho_g, double* rho_l, double* C, double* Psi0);
bool temperature_for_ratio(double a, double b, double R, double ratio, double* T);

// kind: 0 Carnahan-Starling, 1 van der Waals, 2 Peng-Robinson (acentric
// factor omega).  Kind 0 forwards to the functions above.
struct EosSpec {
    int kind;
    double a, b, R, omega;
};
// Attraction coefficient at T: a, or a alpha(T) for Peng-Robinson.
double eos_attraction(const EosSpec& e, double T);
bool eos_critical_point(const EosSpec& e, double* Tc, double* rho_c);
bool eos_maxwell(const EosSpec& e, double T, double* rho_g, double* rho_l, double* C, double* Psi0);
bool eos_temperature_for_ratio(const EosSpec& e, double ratio, double* T);

// The equation of state a parameter set names.
template <class P>
inline EosSpec eos_of(const P& p) {
    return EosSpec{p.eos, p.a, p.b, p.R, p.omega};
}

}  // namespace telbm
