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

// ----------------------------------------------------- spin-polarised ----
// Unrestricted (two spin densities) versions. Exchange by spin scaling,
// e_x = (e_x[2 rho_a] + e_x[2 rho_b])/2, a spin's term only where
// rho_s >= thr. Correlation on rho = rho_a + rho_b and
// zeta = (rho_a - rho_b)/rho held within [-1 + 1e-10, 1 - 1e-10] (where it
// is held, e does not depend on zeta). The spin interpolation of both
// correlation forms is eps = e0 + ac f(zeta)/f''(0) (1 - zeta^4)
// + (e1 - e0) f(zeta) zeta^4, f(zeta) = ((1+zeta)^(4/3) + (1-zeta)^(4/3) - 2)
// /(2^(4/3) - 2). Callers skip points with rho < thr.
constexpr double kZetaMax = 1.0 - 1e-10;
constexpr double kFz = 1.9236610509315362;     // 1/(2^(4/3) - 2)
constexpr double kFpp0 = 1.7099209341613653;   // f''(0) = 4/(9 (2^(1/3) - 1))

// Generic VWN fit G(x; A, b, c, x0) and dG/dx, x = sqrt(r_s).
__device__ inline void vwn_fit(double x, double A, double b, double c, double x0, double& G,
                               double& dG) {
    const double X0 = x0 * x0 + b * x0 + c;
    const double bx0 = b * x0 / X0;
    const double Q = sqrt(4.0 * c - b * b);
    const double X = x * (x + b) + c;
    const double t = 2.0 * x + b;
    const double at = atan(Q / t);
    const double xm = x - x0;
    const double iX = 1.0 / X;
    G = A * (log(x * x * iX) + (2.0 * b / Q) * at -
             bx0 * (log(xm * xm * iX) + (2.0 * (b + 2.0 * x0) / Q) * at));
    dG = A * (2.0 / x - (t + b) * iX - bx0 * (2.0 / xm - (t + b + 2.0 * x0) * iX));
}

// Generic PW92 fit G(rs; A, a1, b1..b4) and dG/drs.
__device__ inline void pw_fit(double rs, double A, double a1, double b1, double b2, double b3,
                              double b4, double& G, double& dG) {
    const double sr = sqrt(rs);
    const double Q0 = -2.0 * A * (1.0 + a1 * rs);
    const double Q1 = 2.0 * A * sr * (b1 + sr * (b2 + sr * (b3 + b4 * sr)));
    const double Q1p = A * (b1 / sr + 2.0 * b2 + sr * (3.0 * b3 + 4.0 * b4 * sr));
    const double L = log1p(1.0 / Q1);
    G = Q0 * L;
    dG = -2.0 * A * a1 * L - Q0 * Q1p / (Q1 * (Q1 + 1.0));
}

// zeta (held), f, f' and the interpolation weights g = f/f''(0) (1 - z^4),
// h = f z^4 with their zeta derivatives; free = false where zeta is held.
struct ZetaParts {
    double z, g, gz, h, hz;
    bool free;
};
__device__ inline ZetaParts zeta_parts(double ra, double rb, double rho) {
    ZetaParts p;
    double z = (ra - rb) / rho;
    p.free = z > -kZetaMax && z < kZetaMax;
    z = fmin(fmax(z, -kZetaMax), kZetaMax);
    p.z = z;
    const double opz = 1.0 + z, omz = 1.0 - z;
    const double c1 = cbrt(opz), c2 = cbrt(omz);
    const double f = (opz * c1 + omz * c2 - 2.0) * kFz;
    const double fz = (4.0 / 3.0) * (c1 - c2) * kFz;
    const double z3 = z * z * z, z4 = z3 * z;
    p.g = f / kFpp0 * (1.0 - z4);
    p.gz = (fz * (1.0 - z4) - 4.0 * z3 * f) / kFpp0;
    p.h = f * z4;
    p.hz = fz * z4 + 4.0 * z3 * f;
    return p;
}

// Slater exchange of one spin density rho_s: e = (e_x[2 rho_s])/2, v = de/drho_s.
__device__ inline void slater_spin(double rs_, double& e, double& v) {
    const double r2 = 2.0 * rs_;
    const double r13 = cbrt(r2);
    e = -0.5 * kCx * r2 * r13;
    v = (-4.0 / 3.0) * kCx * r13;
}

__device__ inline void lda_svwn5_spin(double ra, double rb, double thr, double& e, double& va,
                                      double& vb) {
    e = va = vb = 0.0;
    double ex, vx;
    if (ra >= thr) {
        slater_spin(ra, ex, vx);
        e += ex;
        va += vx;
    }
    if (rb >= thr) {
        slater_spin(rb, ex, vx);
        e += ex;
        vb += vx;
    }
    const double rho = ra + rb;
    const ZetaParts zp = zeta_parts(ra, rb, rho);
    const double x = sqrt(kRs / cbrt(rho));
    double P, dP, F, dF, Ac, dAc;
    vwn_fit(x, 0.0310907, 3.72744, 12.9352, -0.10498, P, dP);
    vwn_fit(x, 0.01554535, 7.06042, 18.0578, -0.32500, F, dF);
    vwn_fit(x, -0.01688686394038963, 1.13107, 13.0045, -0.0047584, Ac, dAc);  // A = -1/(6 pi^2)
    const double eps = P + Ac * zp.g + (F - P) * zp.h;
    const double deps_dx = dP + dAc * zp.g + (dF - dP) * zp.h;
    const double deps_dz = zp.free ? Ac * zp.gz + (F - P) * zp.hz : 0.0;
    const double vr = eps - x * deps_dx * (1.0 / 6.0);   // d(rho eps)/d rho at fixed zeta
    e += rho * eps;
    va += vr + deps_dz * (1.0 - zp.z);
    vb += vr - deps_dz * (1.0 + zp.z);
}

// Unpolarised PBE exchange: e, de/drho, de/dsigma.
__device__ inline void pbe_x_u(double rho, double sigma, double& e, double& vr, double& vs) {
    constexpr double kappa = 0.804, mu = 0.2195149727645171;
    const double r13 = cbrt(rho);
    const double exl = -kCx * rho * r13;
    const double r83 = rho * rho * r13 * r13;
    const double s2 = kS2 * sigma / r83;
    const double den = 1.0 + (mu / kappa) * s2;
    const double Fx = 1.0 + kappa - kappa / den;
    const double dF = mu / (den * den);
    e = exl * Fx;
    vr = (-4.0 / 3.0) * kCx * r13 * Fx - (8.0 / 3.0) * exl * dF * s2 / rho;
    vs = exl * dF * kS2 / r83;
}

__device__ inline void gga_pbe_spin(double ra, double rb, double saa, double sab, double sbb,
                                    double thr, double& e, double& va, double& vb,
                                    double& vsaa, double& vsab, double& vsbb) {
    e = va = vb = vsaa = vsab = vsbb = 0.0;
    double ex, vxr, vxs;
    if (ra >= thr) {
        pbe_x_u(2.0 * ra, 4.0 * saa, ex, vxr, vxs);
        e += 0.5 * ex;
        va += vxr;
        vsaa += 2.0 * vxs;
    }
    if (rb >= thr) {
        pbe_x_u(2.0 * rb, 4.0 * sbb, ex, vxr, vxs);
        e += 0.5 * ex;
        vb += vxr;
        vsbb += 2.0 * vxs;
    }
    constexpr double beta = 0.06672455060314922;
    constexpr double bg = beta / kGamma;
    const double rho = ra + rb;
    const double ir = 1.0 / rho;
    const ZetaParts zp = zeta_parts(ra, rb, rho);
    const double r13 = cbrt(rho);
    const double rs = kRs / r13;
    double e0, d0, e1, d1, ma, dma;
    pw_fit(rs, 0.0310907, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294, e0, d0);
    pw_fit(rs, 0.01554535, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517, e1, d1);
    pw_fit(rs, 0.0168869, 0.11125, 10.357, 3.6231, 0.88026, 0.49671, ma, dma);  // -alpha_c
    const double eps = e0 - ma * zp.g + (e1 - e0) * zp.h;
    const double deps_drs = d0 - dma * zp.g + (d1 - d0) * zp.h;
    const double deps_dz = -ma * zp.gz + (e1 - e0) * zp.hz;
    const double deps_dr = -deps_drs * rs * (1.0 / 3.0) * ir;
    // phi(zeta) and its derivative
    const double c1 = cbrt(1.0 + zp.z), c2 = cbrt(1.0 - zp.z);
    const double phi = 0.5 * (c1 * c1 + c2 * c2);
    const double dphi = (1.0 / 3.0) * (1.0 / c1 - 1.0 / c2);
    const double g3 = kGamma * phi * phi * phi;
    const double sigma = saa + 2.0 * sab + sbb;
    const double r73 = rho * rho * r13;
    const double y = kT2 * sigma / (phi * phi * r73);   // t^2
    const double em1 = expm1(-eps / g3);
    const double Ac = bg / em1;
    const double Ay = Ac * y;
    const double N = 1.0 + Ay;
    const double D = N + Ay * Ay;
    const double iD2 = 1.0 / (D * D);
    const double F = bg * y * N / D;
    const double L = log1p(F);
    const double H = g3 * L;
    const double Fy = bg * (N * D + y * (Ac * D - N * (Ac + 2.0 * Ac * Ay))) * iD2;
    const double FA = bg * y * y * (D - N * (1.0 + 2.0 * Ay)) * iD2;
    const double Hy = g3 * Fy / (1.0 + F), HA = g3 * FA / (1.0 + F);
    const double A_e = bg * (em1 + 1.0) / (g3 * em1 * em1);   // dA/deps at fixed phi
    const double A_p = -A_e * 3.0 * eps / phi;                // dA/dphi at fixed eps
    const double dedr = eps + H + rho * (deps_dr + Hy * (-7.0 / 3.0) * y * ir + HA * A_e * deps_dr);
    double dedz = 0.0;
    if (zp.free)
        dedz = rho * (deps_dz + 3.0 * kGamma * phi * phi * L * dphi + Hy * (-2.0 * y * dphi / phi) +
                      HA * (A_e * deps_dz + A_p * dphi));
    const double deds = rho * Hy * kT2 / (phi * phi * r73);
    e += rho * (eps + H);
    va += dedr + (1.0 - zp.z) * ir * dedz;
    vb += dedr - (1.0 + zp.z) * ir * dedz;
    vsaa += deds;
    vsab += 2.0 * deds;
    vsbb += deds;
}

}  // namespace fn
}  // namespace xc
