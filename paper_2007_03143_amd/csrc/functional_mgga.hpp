// TPSS meta-GGA (Tao, Perdew, Staroverov, Scuseria, Phys. Rev. Lett. 91,
// 146401 (2003)), spin-unpolarised, per grid point: e(rho, sigma, tau) and
// its three partial derivatives. tau is the kinetic energy density
// 1/2 sum_mn P_mn grad phi_m . grad phi_n (the extra intermediate a
// meta-GGA needs, Sec. 2.1).
//
// The energy is written once, over a forward-mode dual number carrying the
// three partial derivatives with respect to (rho, sigma, tau), so the
// potentials are exact derivatives of the coded energy (rounding aside)
// without a hand-derived expression.
//
//   exchange: e_x = e_x^LDA F_x, F_x = 1 + kappa - kappa/(1 + x/kappa),
//     p = sigma/(4 k_F^2 rho^(8/3)), tau_W = sigma/(8 rho), z = tau_W/tau,
//     alpha = (tau - tau_W)/tau_unif, tau_unif = (3/10) k_F^2 rho^(5/3),
//     q_b = (9/20)(alpha - 1)/sqrt(1 + b alpha (alpha - 1)) + 2p/3,
//     x = {[10/81 + c z^2/(1+z^2)^2] p + 146/2025 q_b^2
//          - 73/405 q_b sqrt((3z/5)^2/2 + p^2/2) + (10/81)^2 p^2/kappa
//          + 2 sqrt(e) 10/81 (3z/5)^2 + e mu p^3} / (1 + sqrt(e) p)^2;
//   correlation: e_c = rho eps_rev (1 + d eps_rev z^3),
//     eps_rev = eps_PBE(1 + C z^2) - (1 + C) z^2 max(eps_PBE^pol, eps_PBE),
//     C = 0.53 (zeta = 0, grad zeta = 0), d = 2.8, eps_PBE^pol the PBE
//     correlation of the fully polarised density rho/2 with |grad|^2 =
//     sigma/4 (ferromagnetic PW92 fit, phi = 2^(-1/3)).
// Where tau < tau_W (only rounding or an indefinite P get there) z is held
// at 1 and tau taken as tau_W. The square root of the x term is formed,
// for z < 1, as sigma sqrt(((3/5)/(8 rho tau))^2/2 + (p/sigma)^2/2), equal for
// sigma >= 0 and free of 0/0 in its sigma derivative at sigma = 0.
#pragma once

#include <hip/hip_runtime.h>

namespace xc {
namespace mgga {

// value and partial derivatives with respect to (rho, sigma, tau)
struct D3 {
    double v, g0, g1, g2;
};

__device__ inline D3 dc(double v) { return {v, 0.0, 0.0, 0.0}; }
__device__ inline D3 chain(const D3& a, double f, double df) {
    return {f, df * a.g0, df * a.g1, df * a.g2};
}
__device__ inline D3 operator+(const D3& a, const D3& b) {
    return {a.v + b.v, a.g0 + b.g0, a.g1 + b.g1, a.g2 + b.g2};
}
__device__ inline D3 operator-(const D3& a, const D3& b) {
    return {a.v - b.v, a.g0 - b.g0, a.g1 - b.g1, a.g2 - b.g2};
}
__device__ inline D3 operator-(const D3& a) { return {-a.v, -a.g0, -a.g1, -a.g2}; }
__device__ inline D3 operator+(const D3& a, double b) { return {a.v + b, a.g0, a.g1, a.g2}; }
__device__ inline D3 operator+(double b, const D3& a) { return a + b; }
__device__ inline D3 operator-(const D3& a, double b) { return {a.v - b, a.g0, a.g1, a.g2}; }
__device__ inline D3 operator-(double b, const D3& a) { return {b - a.v, -a.g0, -a.g1, -a.g2}; }
__device__ inline D3 operator*(const D3& a, const D3& b) {
    return {a.v * b.v, a.g0 * b.v + a.v * b.g0, a.g1 * b.v + a.v * b.g1,
            a.g2 * b.v + a.v * b.g2};
}
__device__ inline D3 operator*(const D3& a, double b) {
    return {a.v * b, a.g0 * b, a.g1 * b, a.g2 * b};
}
__device__ inline D3 operator*(double b, const D3& a) { return a * b; }
__device__ inline D3 operator/(const D3& a, const D3& b) {
    const double q = a.v / b.v, ib = 1.0 / b.v;
    return {q, (a.g0 - q * b.g0) * ib, (a.g1 - q * b.g1) * ib, (a.g2 - q * b.g2) * ib};
}
__device__ inline D3 operator/(const D3& a, double b) {
    return {a.v / b, a.g0 / b, a.g1 / b, a.g2 / b};
}
__device__ inline D3 operator/(double a, const D3& b) {
    const double q = a / b.v;
    return chain(b, q, -q / b.v);
}
__device__ inline D3 dsqrt(const D3& a) {
    const double f = sqrt(a.v);
    return chain(a, f, 0.5 / f);
}
__device__ inline D3 dlog1p(const D3& a) { return chain(a, log1p(a.v), 1.0 / (1.0 + a.v)); }
__device__ inline D3 dexpm1(const D3& a) {
    const double f = expm1(a.v);
    return chain(a, f, f + 1.0);
}
__device__ inline D3 dpow(const D3& a, double k) {
    const double f = pow(a.v, k);
    return chain(a, f, k * f / a.v);
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kKF = 3.09366772628013593097;    // (3 pi^2)^(1/3): k_F = kKF rho^(1/3)
constexpr double kKF2 = 9.57078000062730605314;   // (3 pi^2)^(2/3)
constexpr double kCx = 0.738558766382022405884;   // (3/4)(3/pi)^(1/3)
constexpr double kRs = 0.620350490899400016668;   // (3/(4 pi))^(1/3): r_s = kRs rho^(-1/3)
constexpr double kGamma = 0.0310906908696548950349;  // (1 - ln 2)/pi^2
constexpr double kBeta = 0.06672455060314922;
constexpr double kPhiPol = 0.793700525984099737376;  // 2^(-1/3)
constexpr double kKappa = 0.804, kB = 0.40, kC = 1.59096, kE = 1.537, kMu = 0.21951;
constexpr double kSqrtE = 1.23975804090959619797;    // sqrt(1.537)
constexpr double kC00 = 0.53, kD = 2.8;

// PW92 fit -2A(1 + a1 rs) ln(1 + 1/(2A(b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2)))
__device__ inline D3 pw_fit_d(const D3& rs, double A, double a1, double b1, double b2, double b3,
                              double b4) {
    const D3 sr = dsqrt(rs);
    const D3 den = 2.0 * A * (b1 * sr + b2 * rs + b3 * rs * sr + b4 * rs * rs);
    return -2.0 * A * (1.0 + a1 * rs) * dlog1p(1.0 / den);
}

// PBE correlation energy per particle of density n with |grad n|^2 = sig;
// pol: fully polarised (ferromagnetic fit, phi = 2^(-1/3)), else unpolarised.
__device__ inline D3 pbe_eps_c(const D3& n, const D3& sig, bool pol) {
    const D3 rs = kRs * dpow(n, -1.0 / 3.0);
    const D3 eps = pol ? pw_fit_d(rs, 0.01554535, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517)
                       : pw_fit_d(rs, 0.0310907, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294);
    const double phi = pol ? kPhiPol : 1.0;
    const D3 ks2 = (4.0 * kKF / kPi) * dpow(n, 1.0 / 3.0);
    const D3 t2 = sig / (4.0 * phi * phi * ks2 * n * n);
    const double g3 = kGamma * phi * phi * phi;
    const double bg = kBeta / kGamma;
    const D3 A = bg / dexpm1(-eps / g3);
    const D3 At2 = A * t2;
    const D3 H = g3 * dlog1p(bg * t2 * (1.0 + At2) / (1.0 + At2 + At2 * At2));
    return eps + H;
}

// e = e_x + e_c of TPSS and (v_rho, v_sigma, v_tau); rho above the point
// threshold, sigma >= 0.
__device__ inline void tpss(double rho_, double sigma_, double tau_, double& e, double& vr,
                            double& vs, double& vt) {
    const D3 rho = {rho_, 1.0, 0.0, 0.0};
    const D3 sigma = {sigma_, 0.0, 1.0, 0.0};
    const D3 tau = {tau_, 0.0, 0.0, 1.0};
    const D3 tau_w = sigma / (8.0 * rho);
    const bool clamp = tau.v <= tau_w.v;
    const D3 z = clamp ? dc(1.0) : tau_w / tau;
    const D3 r83 = dpow(rho, 8.0 / 3.0);
    const D3 p = sigma / (4.0 * kKF2 * r83);
    const D3 tau_unif = 0.3 * kKF2 * dpow(rho, 5.0 / 3.0);
    const D3 alpha = clamp ? dc(0.0) : (tau - tau_w) / tau_unif;
    const D3 qb = 0.45 * (alpha - 1.0) / dsqrt(1.0 + kB * alpha * (alpha - 1.0)) + (2.0 / 3.0) * p;
    D3 root;
    if (clamp) {
        root = dsqrt(0.18 + 0.5 * p * p);
    } else {
        const D3 a = 0.6 / (8.0 * rho * tau);
        const D3 b = 1.0 / (4.0 * kKF2 * r83);
        root = sigma * dsqrt(0.5 * a * a + 0.5 * b * b);
    }
    const D3 z2 = z * z;
    const D3 opz2 = 1.0 + z2;
    const D3 num = (10.0 / 81.0 + kC * z2 / (opz2 * opz2)) * p + (146.0 / 2025.0) * qb * qb -
                   (73.0 / 405.0) * qb * root + ((10.0 / 81.0) * (10.0 / 81.0) / kKappa) * p * p +
                   (2.0 * kSqrtE * (10.0 / 81.0) * 0.36) * z2 + (kE * kMu) * p * p * p;
    const D3 den = 1.0 + kSqrtE * p;
    const D3 x = num / (den * den);
    const D3 fx = 1.0 + kKappa - kKappa / (1.0 + x / kKappa);
    const D3 ex = -kCx * dpow(rho, 4.0 / 3.0) * fx;
    const D3 eps_pbe = pbe_eps_c(rho, sigma, false);
    const D3 eps_pol = pbe_eps_c(0.5 * rho, 0.25 * sigma, true);
    const D3 eps_t = eps_pol.v >= eps_pbe.v ? eps_pol : eps_pbe;
    const D3 eps_rev = eps_pbe * (1.0 + kC00 * z2) - (1.0 + kC00) * z2 * eps_t;
    const D3 ec = rho * eps_rev * (1.0 + kD * eps_rev * z2 * z);
    const D3 tot = ex + ec;
    e = tot.v;
    vr = tot.g0;
    vs = tot.g1;
    vt = tot.g2;
}

}  // namespace mgga
}  // namespace xc
