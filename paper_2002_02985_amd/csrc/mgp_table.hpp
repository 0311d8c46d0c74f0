// Host-side construction of the MGP-family kernel table (Section
// "New-generation nonlocal KEDFs", eq. "MGP").
//
// omega_{x,y}(q) = omega_WT(q) - x C_WT int_0^1 t^y d/dt G_NL(eta(q,t)) dt with
// eta(q, t) = eta t^(-1/3), eta = q / (2 k_F) (the kernel is the functional
// integral along the uniformly scaled density t rho, whose Fermi wavevector
// is t^(1/3) k_F).  Integrating by parts ([t^y G] vanishes at t = 0, G stays
// bounded) and substituting u = t^y,
//   omega_{x,y} = C_WT [(1 - x) G_NL(eta) + x J(eta)],
//   J(eta) = int_0^1 G_NL(eta u^(-1/(3y))) du,
// so the kernel depends on eta and y only through J, which is smooth at
// eta = 1 where G_NL has its logarithmic kink.  As in step s2 (the kernel
// evaluated once at discrete eta and interpolated), J is tabulated once and
// interpolated linearly by the kernels:
//   nodes eta_j = j / 2048, j = 0 .. 8192 (eta <= 4), then w = 1/eta^2 on
//   w_k = k / 16384, k = 0 .. 1024 (w = 0 at eta = infinity, J = -8/5).
// Each node is integrated with the tanh-sinh (double-exponential) rule,
// split where the argument passes 1 (u = eta^(3y)), which converges to FP64
// precision despite the kinks at the ends of the pieces.
#pragma once
#include <cmath>
#include <vector>

namespace ofdft {

constexpr int MGP_NA = 8192;           // intervals in eta, spacing 1/2048, eta <= 4
constexpr int MGP_NB = 1024;           // intervals in w = 1/eta^2, spacing 1/16384
constexpr int MGP_TAB = MGP_NA + 1 + MGP_NB + 1;
constexpr double MGP_SA = 2048.0;      // 1 / eta spacing
constexpr double MGP_SB = 16384.0;     // 1 / w spacing

// G_NL(e) on the host in FP64: the log1p form below 1.6, the series
// -1 - S/P in u = 1/e^2 above (no cancellation between 1/F and 3 e^2)
inline double mgp_gnl_host(double e)
{
    if (!(e > 0.0)) return 0.0;
    if (e == 1.0) return -2.0;
    if (e < 1.6) {
        const bool lo = e < 1.0;
        const double d = lo ? 1.0 - e : e - 1.0;
        const double num = lo ? 2.0 * e : 2.0;
        const double m = lo ? (1.0 - e) * (1.0 + e) : -((e - 1.0) * (e + 1.0));
        const double F = 0.5 + m / (4.0 * e) * std::log1p(num / d);
        return 1.0 / F - 3.0 * e * e - 1.0;
    }
    const double u = 1.0 / (e * e);
    double P = 0.0, S = 0.0;
    for (int n = 48; n >= 1; --n) P = P * u + 1.0 / ((2.0 * n - 1.0) * (2.0 * n + 1.0));
    for (int n = 48; n >= 2; --n) S = S * u + 3.0 / ((2.0 * n - 1.0) * (2.0 * n + 1.0));
    return -1.0 - S / P;
}

// int_a^b f(u) du by the tanh-sinh rule with step 1/64; abscissae are placed
// from the nearer endpoint (a + half d, b - half d with d = 1 - tanh z) so
// that points close to an end are resolved
template <class Fn>
inline double mgp_tanh_sinh(Fn f, double a, double b)
{
    const double half = 0.5 * (b - a), mid = 0.5 * (a + b);
    const double h = 1.0 / 64.0, hp = 1.5707963267948966;
    double sum = hp * f(mid);
    for (int k = 1; k < 1024; ++k) {
        const double tau = k * h;
        const double z = hp * std::sinh(tau);
        const double ch = std::cosh(z);
        const double w = hp * std::cosh(tau) / (ch * ch);
        const double d = 2.0 / (1.0 + std::exp(2.0 * z));
        if (w * half < 1e-20 || half * d == 0.0) break;
        sum += w * (f(a + half * d) + f(b - half * d));
    }
    return h * half * sum;
}

// J(eta) = int_0^1 G_NL(eta u^(-1/(3y))) du
inline double mgp_J(double eta, double y)
{
    if (eta == 0.0) return 0.0;
    const double a = 1.0 / (3.0 * y);
    auto f = [&](double u) { return u > 0.0 ? mgp_gnl_host(eta * std::pow(u, -a)) : -1.6; };
    if (eta < 1.0) {
        const double us = std::pow(eta, 3.0 * y);
        return mgp_tanh_sinh(f, 0.0, us) + mgp_tanh_sinh(f, us, 1.0);
    }
    return mgp_tanh_sinh(f, 0.0, 1.0);
}

// the table: MGP_NA + 1 values on eta_j, then MGP_NB + 1 values on w_k
inline std::vector<double> mgp_build_table(double y)
{
    std::vector<double> t(MGP_TAB);
    for (int j = 0; j <= MGP_NA; ++j) t[j] = mgp_J(j / MGP_SA, y);
    t[MGP_NA + 1] = -1.6;
    for (int k = 1; k <= MGP_NB; ++k) t[MGP_NA + 1 + k] = mgp_J(1.0 / std::sqrt(k / MGP_SB), y);
    return t;
}

}  // namespace ofdft
