// axpic_tables.cpp -- host construction of the energy quantile tables.
//
// The thermal channels draw x = E/T by inverting a cumulative distribution:
//   Compton-like : number density x^4/(e^x - 1)/(24 zeta5)  (the number form of the
//                  power kernel E^5/(e^{E/T}-1), Sec. II.G)
//   brems        : Gamma(k, 1) density x^{k-1} e^{-x}/Gamma(k) (Sec. II.H)
// The quantile x(u) is tabulated against z = ln(u/(1-u)).  It obeys the ODE
//   dy/dz = u(1-u) / (x f(x)),  y = ln x,  u(1-u) = 1/(2 + 2 cosh z),
// which is integrated with classical RK4 from a starting point obtained by
// Newton iteration on the small-x expansion of the CDF.
#include <cmath>
#include <vector>

#include "axpic_tables.h"

namespace axpic_host {

static const double kZeta5 = 1.0369277551433699263;

// Bernoulli numbers B_0..B_20 (B_1 = -1/2): t/(e^t - 1) = sum B_n t^n / n!.
static const double kB[21] = {1.0, -0.5, 1.0 / 6, 0.0, -1.0 / 30, 0.0, 1.0 / 42, 0.0, -1.0 / 30,
                              0.0, 5.0 / 66, 0.0, -691.0 / 2730, 0.0, 7.0 / 6, 0.0,
                              -3617.0 / 510, 0.0, 43867.0 / 798, 0.0, -174611.0 / 330};

// x f(x) for the two distributions.
static double xf_compton(double x) { return std::pow(x, 5) / std::expm1(x) / (24.0 * kZeta5); }
static double xf_gamma(double x, double k) {
    return std::exp(k * std::log(x) - x - std::lgamma(k));
}

// Small-x CDFs: Compton: (1/(24 zeta5)) sum_n B_n x^{n+4} / (n! (n+4));
// Gamma: x^k e^{-x} sum_n x^n / Gamma(k+n+1).
static double cdf_small_compton(double x) {
    double s = 0.0, fact = 1.0, xp = std::pow(x, 4);
    for (int n = 0; n <= 20; ++n) {
        if (n > 0) fact *= n;
        s += kB[n] * xp / (fact * (n + 4));
        xp *= x;
    }
    return s / (24.0 * kZeta5);
}
static double cdf_small_gamma(double x, double k) {
    double s = 0.0, term = std::exp(-std::lgamma(k + 1.0));
    for (int n = 0; n < 60; ++n) {
        s += term;
        term *= x / (k + n + 1.0);
    }
    return std::exp(k * std::log(x) - x) * s;
}

// Upper tails: Compton: (1/(24 zeta5)) sum_j e^{-jx} (x^4/j + 4x^3/j^2 + 12x^2/j^3
// + 24x/j^4 + 24/j^5); Gamma: the Legendre continued fraction of Q(k, x).
static double tail_compton(double x) {
    double s = 0.0;
    for (int j = 1; j < 400; ++j) {
        const double dj = j, e = std::exp(-dj * x);
        const double t = e * ((((x / dj + 4.0 / (dj * dj)) * x + 12.0 / (dj * dj * dj)) * x +
                               24.0 / (dj * dj * dj * dj)) * x + 24.0 / std::pow(dj, 5));
        s += t;
        if (t < 1e-18 * s) break;
    }
    return s / (24.0 * kZeta5);
}
static double tail_gamma(double x, double k) {
    const double tiny = 1e-300;
    double b = x + 1.0 - k, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 10000; ++i) {
        const double an = -(double)i * ((double)i - k);
        b += 2.0;
        d = an * d + b; if (std::fabs(d) < tiny) d = tiny;
        c = b + an / c; if (std::fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        const double del = d * c;
        h *= del;
        if (std::fabs(del - 1.0) < 1e-17) break;
    }
    return std::exp(-x + k * std::log(x) - std::lgamma(k)) * h;
}

// The quantile ODE is integrated upwards from z0 up to z = 18, where it is stable
// (a too large x makes the slope smaller), and downwards from z1 to z = 18 from a
// Newton solution of the tail, the stable direction there; the lower part is the
// table of the plain (uncut) samplers, the upper part serves the cut spectra.
constexpr double kTabZMid = 18.0;

template <class CDF, class XF, class TAIL>
static void build(double* tab, CDF cdf_small, XF xf, TAIL tail) {
    const int N = kTabN;
    const double h = (kTabZ1 - kTabZ0) / N;
    const double u0 = 1.0 / (1.0 + std::exp(-kTabZ0));
    // starting point: Newton on the small-x CDF, dC/dx = f(x)
    double x = 0.05;
    for (int it = 0; it < 200; ++it) {
        double f = xf(x) / x;
        double dx = (cdf_small(x) - u0) / f;
        double xn = x - dx;
        if (!(xn > 0.0)) xn = 0.5 * x;
        if (std::fabs(xn - x) < 1e-16 * x) { x = xn; break; }
        x = xn;
    }
    auto rhs = [&](double z, double y) {
        double uu = 1.0 / (2.0 + 2.0 * std::cosh(z));
        return uu / xf(std::exp(y));
    };
    double y = std::log(x);
    const int sub = 32;
    const double hs = h / sub;
    const int jmid = (int)std::lround((kTabZMid - kTabZ0) / h);
    for (int j = 0; j <= jmid; ++j) {
        double z = kTabZ0 + j * h;
        tab[j] = y;
        tab[N + 1 + j] = rhs(z, y);
        if (j == jmid) break;
        for (int s = 0; s < sub; ++s) {
            double zz = z + s * hs;
            double k1 = rhs(zz, y);
            double k2 = rhs(zz + 0.5 * hs, y + 0.5 * hs * k1);
            double k3 = rhs(zz + 0.5 * hs, y + 0.5 * hs * k2);
            double k4 = rhs(zz + hs, y + hs * k3);
            y += hs / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4);
        }
    }
    if (jmid >= N) return;
    // tail start: ln Q(x) = ln q1, q1 = 1/(1 + e^{z1}), by Newton (d ln Q/dx = -f/Q)
    const double lq = -kTabZ1 - std::log1p(std::exp(-kTabZ1));
    x = 40.0;
    for (int it = 0; it < 200; ++it) {
        const double Q = tail(x);
        const double g = std::log(Q) - lq;
        const double dg = -(xf(x) / x) / Q;
        double xn = x - g / dg;
        if (!(xn > 0.5 * x)) xn = 0.5 * x;
        if (std::fabs(xn - x) < 1e-15 * x) { x = xn; break; }
        x = xn;
    }
    y = std::log(x);
    for (int j = N; j > jmid; --j) {
        double z = kTabZ0 + j * h;
        tab[j] = y;
        tab[N + 1 + j] = rhs(z, y);
        for (int s = 0; s < sub; ++s) {
            double zz = z - s * hs;
            double k1 = rhs(zz, y);
            double k2 = rhs(zz - 0.5 * hs, y - 0.5 * hs * k1);
            double k3 = rhs(zz - 0.5 * hs, y - 0.5 * hs * k2);
            double k4 = rhs(zz - hs, y - hs * k3);
            y -= hs / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4);
        }
    }
}

void build_compton_table(double* tab) {
    build(tab, [](double x) { return cdf_small_compton(x); },
          [](double x) { return xf_compton(x); }, [](double x) { return tail_compton(x); });
}

void build_gamma_table(double* tab, double k) {
    build(tab, [k](double x) { return cdf_small_gamma(x, k); },
          [k](double x) { return xf_gamma(x, k); }, [k](double x) { return tail_gamma(x, k); });
}

}  // namespace axpic_host
