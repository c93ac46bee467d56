// ndgp_screening.hip -- host functions: Vainshtein screening of the fifth
// force in NFW haloes and the refinement level from which the scalar-field
// iterations may be truncated (arXiv:1511.08200, Sec. II.B and Sec. V).
//
// In a spherically symmetric halo the field equation integrates to a quadratic
// in phi_,r / r (Eq. eomvarphi_sph) whose positive root is Eq. (eomvarphi_sph2)
// with the Vainshtein radius of Eq. (rv).  Dividing F_5th = phi_,r / 2 by
// F_GR = G M(<r) / r^2 leaves
//
//     G_eff - 1 = F_5th / F_GR = 2 / (3 beta (1 + sqrt(1 + x))),
//     x = (r_V / r)^3 = (16/9) (r_c H0)^2 (G M(<r) / r^3) / (H0^2 beta^2),
//
// written in this form so that nothing cancels as x -> 0.  For an NFW profile
// (Eqs. nfw, nfwparams) with M_200 inside R_200 at 200 times the critical
// density (Eq. r200, exponent 1/3), G M(<r) / r^3 = 100 H(z)^2 mu(c s) / (mu(c) s^3)
// with s = r / R_200 and mu(y) = ln(1 + y) - y / (1 + y): the ratio depends on
// r / R_200 and c_200 only, not on M_200 (Sec. II.B).

#include "ndgp.h"
#include "ndgp_internal.h"

#include <cmath>
#include <string>

namespace {

constexpr double kG = 4.30091727e-9;   // Newton's constant, Mpc (km/s)^2 / M_sun
constexpr double kH0 = 100.0;          // H0 in h km/s/Mpc
constexpr double kPi = 3.14159265358979323846;

// mu(y) = ln(1 + y) - y / (1 + y); its power series below y = 1/64, where the
// two terms cancel to y^2 / 2
double nfw_mu(double y) {
    if (y < 1.0 / 64.0) {
        double term = y * y, sum = 0.0;
        for (int k = 2; k <= 12; ++k) {
            sum += (k & 1 ? -1.0 : 1.0) * (double)(k - 1) / (double)k * term;
            term *= y;
        }
        return sum;
    }
    return std::log1p(y) - y / (1.0 + y);
}

// (r_V / r)^3 at s = r / R_200
double vainshtein_x(double s, double c200, double rc, double beta, double e_z) {
    const double mean_density = 100.0 * e_z * e_z * nfw_mu(c200 * s) / (nfw_mu(c200) * s * s * s);
    return 16.0 / 9.0 * rc * rc * mean_density / (beta * beta);
}

double ratio_at(double s, double c200, double rc, double beta, double e_z) {
    const double x = vainshtein_x(s, c200, rc, beta, e_z);
    return 2.0 / (3.0 * beta * (1.0 + std::sqrt(1.0 + x)));
}

bool halo_ok(double m200, double c200, double rc, double beta, double e_z) {
    if (!(std::isfinite(m200) && m200 > 0.0) || !(std::isfinite(c200) && c200 > 0.0) ||
        !(std::isfinite(rc) && rc >= 0.0) || !(std::isfinite(beta) && beta > 0.0) ||
        !(std::isfinite(e_z) && e_z > 0.0)) {
        ndgp::set_last_error("need m200, c200, beta, e_z > 0 and rc >= 0, all finite");
        return false;
    }
    return true;
}

} // namespace

extern "C" {

double ndgp_nfw_r200(double m200, double e_z) {
    if (!(std::isfinite(m200) && m200 > 0.0) || !(std::isfinite(e_z) && e_z > 0.0)) {
        ndgp::set_last_error("need m200 > 0 and e_z > 0, finite");
        return NAN;
    }
    const double H = kH0 * e_z;
    const double rho_c = 3.0 * H * H / (8.0 * kPi * kG);
    return std::cbrt(3.0 * m200 / (4.0 * kPi * 200.0 * rho_c));
}

double ndgp_nfw_force_ratio(double r, double m200, double c200, double rc, double beta,
                            double e_z) {
    if (!halo_ok(m200, c200, rc, beta, e_z)) return NAN;
    if (!(std::isfinite(r) && r > 0.0)) {
        ndgp::set_last_error("need r > 0, finite");
        return NAN;
    }
    return ratio_at(r / ndgp_nfw_r200(m200, e_z), c200, rc, beta, e_z);
}

double ndgp_nfw_screening_radius(double fraction, double m200, double c200, double rc,
                                 double beta, double e_z) {
    if (!halo_ok(m200, c200, rc, beta, e_z)) return NAN;
    if (!std::isfinite(fraction)) {
        ndgp::set_last_error("fraction must be finite");
        return NAN;
    }
    if (fraction <= 0.0) return 0.0;
    if (rc == 0.0 || 3.0 * beta * fraction >= 1.0) return INFINITY; // never screened that far
    // ratio = fraction  <=>  x = (2 / (3 beta fraction) - 1)^2 - 1; x(s) falls
    // monotonically with s (the mean density inside r falls), so bisect on log s
    const double q = 2.0 / (3.0 * beta * fraction) - 1.0;
    const double xt = q * q - 1.0;
    double lo = -40.0, hi = 40.0; // natural log of s
    for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (vainshtein_x(std::exp(mid), c200, rc, beta, e_z) > xt)
            lo = mid;
        else
            hi = mid;
    }
    return std::exp(0.5 * (lo + hi)) * ndgp_nfw_r200(m200, e_z);
}

int32_t ndgp_nfw_trunc_level(double h_domain, double fraction, double m200, double c200,
                             double rc, double beta, double e_z) {
    if (!(std::isfinite(h_domain) && h_domain > 0.0)) {
        ndgp::set_last_error("need h_domain > 0, finite");
        return -1;
    }
    if (!(std::isfinite(fraction) && fraction > 0.0)) {
        ndgp::set_last_error("need fraction > 0, finite");
        return -1;
    }
    const double rt = ndgp_nfw_screening_radius(fraction, m200, c200, rc, beta, e_z);
    if (std::isnan(rt)) return -1;
    int32_t k = 1;
    while (k < 60 && std::ldexp(h_domain, -k) > rt) ++k;
    return k;
}

} // extern "C"
