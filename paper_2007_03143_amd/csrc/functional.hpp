// Spin-unpolarised exchange-correlation functionals evaluated per grid point
// on the device (the per-point step of Sec. 2.2 eq. eval_xc_batch).
//
// Each routine returns e = rho * eps (energy per unit volume), v_rho = de/drho
// and, for the GGA, v_sigma = de/dsigma with sigma = |grad rho|^2.
//   LDA: Slater exchange + VWN5 correlation (paramagnetic fit).
//   GGA: PBE exchange (kappa = 0.804, mu = 0.2195149727645171) + PBE
//        correlation on the PW92 uniform-gas correlation.
// Derivatives are analytic. Constants derived from pi are written to 20
// significant digits with the expression they come from.
#pragma once

#include <hip/hip_runtime.h>

namespace xc {
namespace fn {

constexpr double kCx = 0.73855876638202240588;   // (3/4) (3/pi)^(1/3)
constexpr double kRs = 0.62035049089940001667;   // (3/(4 pi))^(1/3): r_s = kRs rho^(-1/3)
constexpr double kS2 = 0.026121172985233599568;  // 1/(4 (3 pi^2)^(2/3)): s^2 = kS2 sigma rho^(-8/3)
constexpr double kT2 = 0.063468206097703704202;  // pi/(16 (3 pi^2)^(1/3)): t^2 = kT2 sigma rho^(-7/3)
constexpr double kGamma = 0.031090690869654895035;  // (1 - ln 2)/pi^2

// VWN5 correlation per particle eps(x) and d eps/dx, x = sqrt(r_s).
__device__ inline void vwn5_eps(double x, double& eps, double& deps_dx) {
    constexpr double A = 0.0310907, b = 3.72744, c = 12.9352, x0 = -0.10498;
    constexpr double X0 = x0 * x0 + b * x0 + c;
    constexpr double bx0 = b * x0 / X0;
    const double Q = sqrt(4.0 * c - b * b);
    const double X = x * (x + b) + c;
    const double t = 2.0 * x + b;
    const double at = atan(Q / t);
    const double xm = x - x0;
    eps = A * (log(x * x / X) + (2.0 * b / Q) * at -
               bx0 * (log(xm * xm / X) + (2.0 * (b + 2.0 * x0) / Q) * at));
    // the arctangent terms differentiate to -b/X and -(b + 2 x0)/X since t^2 + Q^2 = 4X
    const double iX = 1.0 / X;
    deps_dx = A * (2.0 / x - (t + b) * iX - bx0 * (2.0 / xm - (t + b + 2.0 * x0) * iX));
}

__device__ inline void lda_svwn5(double rho, double& e, double& vrho) {
    const double r13 = cbrt(rho);
    const double ex = -kCx * rho * r13;
    const double vx = (-4.0 / 3.0) * kCx * r13;
    const double x = sqrt(kRs / r13);
    double ec, dec;
    vwn5_eps(x, ec, dec);
    e = ex + rho * ec;
    vrho = vx + ec - x * dec * (1.0 / 6.0);
}

// PW92 unpolarised correlation per particle and its r_s derivative.
__device__ inline void pw92(double rs, double& eps, double& deps) {
    constexpr double A = 0.0310907, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876,
                     b3 = 1.6382, b4 = 0.49294;
    const double sr = sqrt(rs);
    const double Q0 = -2.0 * A * (1.0 + a1 * rs);
    const double Q1 = 2.0 * A * sr * (b1 + sr * (b2 + sr * (b3 + b4 * sr)));
    const double Q1p = A * (b1 / sr + 2.0 * b2 + sr * (3.0 * b3 + 4.0 * b4 * sr));
    const double L = log1p(1.0 / Q1);
    eps = Q0 * L;
    deps = -2.0 * A * a1 * L - Q0 * Q1p / (Q1 * (Q1 + 1.0));
}

__device__ inline void gga_pbe(double rho, double sigma, double& e, double& vrho,
                               double& vsigma) {
    constexpr double kappa = 0.804, mu = 0.2195149727645171;
    constexpr double beta = 0.06672455060314922;
    constexpr double bg = beta / kGamma;
    const double r13 = cbrt(rho);
    const double ir = 1.0 / rho;
    // exchange: e_x = e_x^LDA F_x(s^2)
    const double exl = -kCx * rho * r13;
    const double r83 = rho * rho * r13 * r13;
    const double s2 = kS2 * sigma / r83;
    const double den = 1.0 + (mu / kappa) * s2;
    const double Fx = 1.0 + kappa - kappa / den;
    const double dF = mu / (den * den);
    const double ex = exl * Fx;
    const double vxr = (-4.0 / 3.0) * kCx * r13 * Fx - (8.0 / 3.0) * exl * dF * s2 * ir;
    const double vxs = exl * dF * kS2 / r83;
    // correlation: rho (eps_PW92 + H(t^2, A))
    const double rs = kRs / r13;
    double ec, decdrs;
    pw92(rs, ec, decdrs);
    const double decdr = -decdrs * rs * (1.0 / 3.0) * ir;
    const double r73 = rho * rho * r13;
    const double t2 = kT2 * sigma / r73;
    const double em1 = expm1(-ec / kGamma);
    const double Ac = bg / em1;
    const double At2 = Ac * t2;
    const double N = 1.0 + At2;
    const double D = N + At2 * At2;
    const double iD2 = 1.0 / (D * D);
    const double F = bg * t2 * N / D;
    const double H = kGamma * log1p(F);
    const double Fy = bg * (N * D + t2 * (Ac * D - N * (Ac + 2.0 * Ac * At2))) * iD2;
    const double FA = bg * t2 * t2 * (D - N * (1.0 + 2.0 * At2)) * iD2;
    const double i1F = kGamma / (1.0 + F);
    const double Hy = Fy * i1F, HA = FA * i1F;
    const double dAde = bg * (em1 + 1.0) / (kGamma * em1 * em1);
    const double dt2dr = (-7.0 / 3.0) * t2 * ir;
    e = ex + rho * (ec + H);
    vrho = vxr + ec + H + rho * (decdr + Hy * dt2dr + HA * dAde * decdr);
    vsigma = vxs + rho * Hy * kT2 / r73;
}

}  // namespace fn
}  // namespace xc
