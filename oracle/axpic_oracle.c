/* axpic_oracle.c -- FP64 CPU oracle of the axion Monte-Carlo operators.
 *
 * TEST INFRASTRUCTURE ONLY (see axpic_oracle.h).  Every function is the plain
 * definition of what the method computes, written from the paper:
 *   "An axion framework for Particle-in-Cell codes with Monte-Carlo sampling"
 *   (Radford et al., arXiv:2604.24627).
 * Section / equation labels below refer to that paper.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC.
 * Contraction is off so that the Poisson inversion and the FP32 push follow
 * exactly the operation order written here.
 */
#include "axpic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Constants (CODATA 2018).  The paper rounds m_e c^2 to 511 keV and 1 keV to
 * 1.602e-9 erg; the exact values are used here.                             */
/* ------------------------------------------------------------------------ */
#define OR_PI 3.14159265358979323846
#define OR_ALPHA (1.0 / 137.035999084)
#define OR_HBARC_GEVCM 1.973269804e-14
#define OR_HBARC_KEVCM 1.973269804e-8
#define OR_C_CMS 2.99792458e10
#define OR_ME_KEV 510.99895000
#define OR_KEV_ERG 1.602176634e-9
#define OR_KEV_T7 1.160451812 /* T_7 = T / 10^7 K per keV */
#define OR_MU_G 1.66053906660e-24
#define OR_ZETA3 1.2020569031595942854
#define OR_ZETA5 1.0369277551433699263
#define OR_ZETA6 1.0173430619844491397
#define OR_LAMBDA_HARD_CAP 64.0
#define OR_KMAX 255

int32_t or_num_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops that follow (the CPU-baseline timing runs the oracle on
 * all host cores and on one). */
void or_set_num_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

double or_const(int which) {
    switch (which) {
    case 0: return OR_ALPHA;
    case 1: return OR_HBARC_GEVCM;
    case 2: return OR_HBARC_KEVCM;
    case 3: return OR_C_CMS;
    case 4: return OR_ME_KEV;
    case 5: return OR_KEV_ERG;
    case 6: return OR_KEV_T7;
    case 7: return OR_MU_G;
    case 8: return OR_ZETA3;
    case 9: return OR_ZETA5;
    case 10: return OR_ZETA6;
    case 11: return OR_LAMBDA_HARD_CAP;
    case 12: return (double)OR_KMAX;
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Counter-based RNG: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).     */
/* ------------------------------------------------------------------------ */
static void or_mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t prod = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(prod >> 32);
    *lo = (uint32_t)prod;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { /* key schedule: Weyl sequence bump between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        or_mulhilo(0xD2511F53u, c0, &hi0, &lo0);
        or_mulhilo(0xCD9E8D57u, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw contract: key = (seed lo, seed hi); counter = (id lo, id hi, step,
 * stream << 24 | block).  Streams: 0 Primakoff count, 1 thermal counts
 * (words 0-1 Compton, 2-3 brems), 2 Compton event k, 3 brems event k,
 * 4 absorption (words 0-1 thermal absorption, 2-3 a->gamma count).        */
void or_draw(uint64_t seed, uint64_t id, uint32_t step, uint32_t stream, uint32_t block,
             uint32_t out[4]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, (stream << 24) | (block & 0xFFFFFFu)};
    or_philox4x32_10(ctr, key, out);
}

/* Uniform in [0,1) with 53 random bits: (a>>5)*2^26 + (b>>6), times 2^-53. */
double or_u53(uint32_t a, uint32_t b) {
    double hi = (double)(a >> 5);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo) * (1.0 / 9007199254740992.0);
}

/* Uniform in (0,1) on the odd multiples of 2^-24 (exact in FP32). */
double or_u24(uint32_t a) {
    return (double)(2u * (a >> 9) + 1u) * (1.0 / 16777216.0);
}

/* Poisson(lam) by sequential inversion of the CDF (eq. poisson_macro): the
 * smallest k with u < sum_{j<=k} lam^j e^-lam / j!.  Fixed operation order. */
static int32_t or_poisson_kmax(double lam, double u, int32_t kmax) {
    if (!(lam > 0.0)) return 0;
    int32_t k = 0;
    double p = exp(-lam);
    double F = p;
    while (u >= F && k < kmax) {
        k += 1;
        p = p * lam;
        p = p / (double)k;
        F = F + p;
    }
    return k;
}

int32_t or_poisson(double lam, double u) {
    if (!(lam > 0.0)) return 0;
    int32_t k = 0;
    double p = exp(-lam);
    double F = p;
    while (u >= F && k < OR_KMAX) {
        k += 1;
        p = p * lam;
        p = p / (double)k;
        F = F + p;
    }
    return k;
}

void or_poisson_batch(const double* lam, const double* u, int32_t* k, int64_t n) {
    for (int64_t i = 0; i < n; ++i) k[i] = or_poisson(lam[i], u[i]);
}

/* Poisson-mean capping with weight rescale (eq. lambda_eff, eq. wa_rescaled).
 * The user cap is bounded by the sampler's own limit; the rescale keeps the
 * expected physical yield unchanged either way.                             */
static double or_cap(double lam_macro, const or_params* prm, double* wscale, int* capped) {
    double cap = prm->lambda_cap;
    if (!(cap <= OR_LAMBDA_HARD_CAP)) cap = OR_LAMBDA_HARD_CAP;
    double le = lam_macro < cap ? lam_macro : cap;
    *capped = lam_macro > cap;
    *wscale = (lam_macro > cap) ? lam_macro / le : 1.0;
    return le;
}

/* ------------------------------------------------------------------------ */
/* Screened Primakoff kernel (eq. prim_F).                                    */
/* ------------------------------------------------------------------------ */
/* Evaluated in extended precision; below s = 1e-4, where the closed form
 * cancels even there, by its Taylor series sum_n (-1)^{n+1} s^n/(n(n+1)). */
double or_F(double s) {
    if (!(s > 0.0)) return 0.0;
    if (s < 1e-4) return s / 2.0 - s * s / 6.0 + s * s * s / 12.0 - s * s * s * s / 20.0;
    long double S = (long double)s;
    return (double)((1.0L + 1.0L / S) * log1pl(S) - 1.0L);
}

double or_dt_phys(const or_grid* g) { return g->dt / g->omega0; }   /* eq. dt_phys */

double or_V_cell(const or_grid* g) {
    double L = g->dx * OR_C_CMS / g->omega0;
    return L * L * L;
}

/* ------------------------------------------------------------------------ */
/* Local plasma state (Sec. II.E) and channel rates (Secs. II.F-II.H).       */
/* ------------------------------------------------------------------------ */
void or_cell_state(const or_grid* g, const or_params* prm, int64_t ncell, const double* T,
                   const double* dens_e, int32_t nion, const double* dens_ion,
                   const double* Zion, const double* Aion, or_cell* out) {
    (void)g;
    const double alpha_ae = prm->g_ae * prm->g_ae / (4.0 * OR_PI);
    const double aratio = alpha_ae / 1.60e-23;
    const double meanC_over_T = 5.0 * OR_ZETA6 / OR_ZETA5;
    const double meanB_over_T = prm->brems_k * prm->brems_theta;
    for (int64_t c = 0; c < ncell; ++c) {
        or_cell* o = &out[c];
        memset(o, 0, sizeof(*o));
        double nZ = 0.0, nZ2 = 0.0, rho = 0.0, rhoH = 0.0;
        for (int32_t s = 0; s < nion; ++s) {
            double ni = dens_ion[(int64_t)s * ncell + c];
            nZ += Zion[s] * ni;
            nZ2 += Zion[s] * Zion[s] * ni;                 /* effective charge-weighted targets */
            rho += ni * Aion[s] * OR_MU_G;                 /* eq. rho_def */
            if (Zion[s] == 1.0 && Aion[s] < 1.5) rhoH += ni * Aion[s] * OR_MU_G;
        }
        double ne_dep = dens_e ? dens_e[c] : 0.0;
        double ne = prm->quasi_neutral ? nZ : ne_dep;      /* eq. qn_def */
        double Tk = T[c];
        o->T = Tk; o->n_e = ne; o->n_e_dep = ne_dep; o->nZ = nZ; o->nZ2 = nZ2; o->rho = rho;
        o->XH = rho > 0.0 ? rhoH / rho : 0.0;
        /* Debye screening, eq. kappa_debye, in keV^2: 4 pi alpha n_eff (hbar c)^3 / T */
        if (prm->kappa_mode == 1) {
            o->kappa2 = prm->kappa_fixed_keV * prm->kappa_fixed_keV;
        } else {
            double neff = ne + nZ2;
            double hc3 = OR_HBARC_KEVCM * OR_HBARC_KEVCM * OR_HBARC_KEVCM;
            o->kappa2 = 4.0 * OR_PI * OR_ALPHA * neff * hc3 / Tk;
        }
        /* Primakoff: Gamma = n_t sigma c with sigma = alpha g^2 Z^2 F(s) (hbar c)^2 / 8
         * and n_t Z^2 -> sum_i Z_i^2 n_i (eqs. prim_xs, prim_rate).               */
        double targets = prm->prim_targets ? (ne + nZ2) : nZ2;
        double hc2 = OR_HBARC_GEVCM * OR_HBARC_GEVCM;
        o->G_P0 = prm->boost * (OR_ALPHA * prm->g_agg_GeV * prm->g_agg_GeV / 8.0) * hc2 *
                  OR_C_CMS * targets;
        /* Compton-like: eqs. epsC, QC, GammaC */
        double T7 = Tk * OR_KEV_T7;
        double XH = o->XH;
        double epsC = 2.67e-2 * (1.0 + XH) * pow(T7, 6.0) * aratio;
        o->Q_C = rho * epsC;
        o->meanE_C = meanC_over_T * Tk;
        /* Bremsstrahlung: eqs. eps_eZ, eps_ee; screening fit factors kept >= 0 */
        double rho2 = rho / 100.0;
        double eta = (3.0 + XH) * rho2 / (T7 * T7);
        double base = 0.150 * pow(T7, 2.5) * rho2 * (1.0 + XH) * aratio;
        double sZ = 1.0 - 6.98e-2 * eta; if (sZ < 0.0) sZ = 0.0;
        double se = 1.0 - 0.140 * eta; if (se < 0.0) se = 0.0;
        double epsZ = base * sZ;
        double epsE = base * (1.0 + XH) / (2.0 * sqrt(2.0)) * se;
        double epsB = epsZ + (prm->brems_ee ? epsE : 0.0);
        o->Q_B = rho * epsB;
        o->meanE_B = meanB_over_T * Tk;
        if (ne > 0.0) {
            o->G_C = prm->boost * o->Q_C / (ne * o->meanE_C * OR_KEV_ERG);
            o->G_B = prm->boost * o->Q_B / (ne * o->meanE_B * OR_KEV_ERG);
        }
    }
}

double or_gamma_prim(const or_cell* c, const or_params* prm, double omega_keV) {
    (void)prm;
    double s = 4.0 * omega_keV * omega_keV / c->kappa2;   /* eq. prim_xs */
    return c->G_P0 * or_F(s);
}

/* ------------------------------------------------------------------------ */
/* Finite-mass axions.  The paper gives the kinematics E = sqrt(p^2 + m^2)   */
/* and the sub-luminal velocity (Sec. II.B) and says that thresholds and     */
/* absorption coefficients change with the mass, without printing them.     */
/* Readings (c = 1, energies and momenta in keV):                           */
/*  M1 E = sqrt(m_e^2 |p|^2 + m^2), push velocity p / sqrt(|p|^2 + (m/m_e)^2).*/
/*  M2 photon (momentum k = omega) -> axion (momentum p = sqrt(k^2 - m^2))  */
/*     on a screened static charge: the massless amplitude |k x p|^2 over   */
/*     q^2 (q^2 + kappa^2), q = k - p, with the final-state factor p/k, so   */
/*     Gamma = G_P0 (p/k) F_mass(k, p); zero for omega <= m.  F_mass is 2x  */
/*     the angular integral int_{-1}^{1} dc k^2 p^2 (1-c^2)/(q^2(q^2+kappa^2))*/
/*     in closed form; F_mass(k, k) = F(4 k^2/kappa^2).                     */
/*  M3 the axion keeps the photon's direction with |p|; a->gamma turns an   */
/*     axion of energy E into a photon of energy E along it, at the rate    */
/*     prim_inv_ratio (k/p) Gamma_{gamma->a}(E) (the massive phase space in */
/*     detailed balance) = prim_inv_ratio G_P0 F_mass(E, p).                 */
/*  M4 thermal emission: the sampled number spectrum is cut at E = m; the   */
/*     rate is the massless one times the spectrum's fraction above m and   */
/*     energies are drawn by inversion at F(m/T) + u (1 - F(m/T)).          */
/*  M5 absorption: the massive equilibrium density dn_eq/dE = E p f(E/T) /  */
/*     (2 pi^2 (hbar c)^3) gives Gamma_abs the factor E/p (zero below m).   */
/* Energy exchanged with the plasma is the total energy E.                  */
/* ------------------------------------------------------------------------ */
double or_axion_energy(const or_params* prm, double p2) {
    double mu = prm->m_a_keV / OR_ME_KEV;
    return OR_ME_KEV * sqrt(p2 + mu * mu);
}

double or_F_mass(double k, double p, double kappa2) {
    if (!(k > 0.0) || !(p > 0.0)) return 0.0;
    if (p >= k) return or_F(4.0 * k * k / kappa2);
    /* with a = 4kp, A = (k-p)^2 + kappa^2: the logarithms are log1p(a/A) and
     * log1p(a/(k-p)^2), which keeps them accurate when p << k */
    long double K = k, P = p, k2 = kappa2;
    long double a = 4.0L * K * P, am = (K - P) * (K - P), A = am + k2;
    long double t1 = (A + a) * A / (a * k2) * log1pl(a / A);
    long double t2 = am * (am + a) / (a * k2) * log1pl(a / am);
    return (double)(t1 - t2 - 1.0L);
}

static void or_gl_init(void);
static double or_gl_x[10], or_gl_w[10];

/* The same angular integral by quadrature: with t = 1 - cos(theta) it is
 * (1/2) int_0^2 t (2 - t) / ((t + b1)(t + b2)) dt, b1 = (k-p)^2/(2kp),
 * b2 = ((k-p)^2 + kappa^2)/(2kp); 10-point Gauss-Legendre panels halving
 * towards t = 0 down to well below the smaller nonzero of b1, b2.          */
double or_F_mass_quad(double k, double p, double kappa2) {
    if (!(k > 0.0) || !(p > 0.0)) return 0.0;
    or_gl_init();
    const double b1 = (k - p) * (k - p) / (2.0 * k * p);
    const double b2 = ((k - p) * (k - p) + kappa2) / (2.0 * k * p);
    const double bmin = (b1 > 0.0 && b1 < b2) ? b1 : b2;   /* finest feature of the integrand */
    int J = 12;
    while (2.0 * pow(0.5, J) > 1e-3 * bmin && J < 200) ++J;
    double sum = 0.0, hi = 2.0;
    for (int j = 1; j <= J + 1; ++j) {
        double lo = (j <= J) ? 2.0 * pow(0.5, j) : 0.0;
        double h = 0.5 * (hi - lo), m = 0.5 * (hi + lo), acc = 0.0;
        for (int i = 0; i < 10; ++i) {
            double t = m + h * or_gl_x[i];
            acc += or_gl_w[i] * t * (2.0 - t) / ((t + b1) * (t + b2));
        }
        sum += acc * h;
        hi = lo;
    }
    return 0.5 * sum;
}

/* Gamma_{gamma->a} of a photon of energy omega (M2; the massless eq. prim_rate
 * when m = 0). */
double or_gamma_conv(const or_cell* c, const or_params* prm, double omega_keV) {
    const double m = prm->m_a_keV;
    if (!(m > 0.0)) return or_gamma_prim(c, prm, omega_keV);
    if (!(omega_keV > m)) return 0.0;
    const double k = omega_keV, p = sqrt((k - m) * (k + m));
    return c->G_P0 * (p / k) * or_F_mass(k, p, c->kappa2);
}

/* Normalised number spectra that the thermal samplers draw from.           */
static double or_pdf_compton(double E, double T) {          /* x^4/(e^x-1)/(24 zeta5) / T */
    double x = E / T;
    return x * x * x * x / expm1(x) / (24.0 * OR_ZETA5 * T);
}
static double or_pdf_brems(double E, double T, double k, double th) {
    double y = E / (th * T);
    return exp((k - 1.0) * log(y) - y - lgamma(k)) / (th * T);
}
/* Equilibrium spectra dn_eq/dE (BE or MB), Sec. II.I. */
static double or_dneq(double E, double T, int mb) {
    double hc3 = OR_HBARC_KEVCM * OR_HBARC_KEVCM * OR_HBARC_KEVCM;
    double occ = mb ? exp(-E / T) : 1.0 / expm1(E / T);
    return E * E / (2.0 * OR_PI * OR_PI * hc3) * occ;
}

/* Detailed-balance absorption rate, eq. gamma_abs: (dn_dot/dE)/(dn_eq/dE),
 * with dn_dot/dE = n_e Gamma_c p_c(E) for each active thermal channel.     */
double or_gamma_abs(const or_cell* c, const or_params* prm, double E_keV, double* parts) {
    double gC = 0.0, gB = 0.0;
    double neq = or_dneq(E_keV, c->T, prm->eq_stats);
    const double m = prm->m_a_keV;
    if (m > 0.0)   /* M5: E p instead of E^2 in dn_eq/dE */
        neq = E_keV > m ? neq * sqrt((E_keV - m) * (E_keV + m)) / E_keV : 0.0;
    if (neq > 0.0) {
        if (prm->channels & OR_CH_C)
            gC = c->n_e_dep * c->G_C * or_pdf_compton(E_keV, c->T) / neq;
        if (prm->channels & OR_CH_B)
            gB = c->n_e_dep * c->G_B * or_pdf_brems(E_keV, c->T, prm->brems_k, prm->brems_theta) / neq;
    }
    if (parts) { parts[0] = gC; parts[1] = gB; }
    return gC + gB;
}

/* ------------------------------------------------------------------------ */
/* Exact inverse-CDF samplers.                                               */
/* ------------------------------------------------------------------------ */
static double or_gl_x[10], or_gl_w[10];
static int or_gl_ready = 0;

static void or_gl_init(void) {       /* 10-point Gauss-Legendre on [-1,1] */
    if (or_gl_ready) return;
    const int n = 10;
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2; p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        or_gl_x[i] = z;
        or_gl_w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
    or_gl_ready = 1;
}

static double or_compton_integrand(double x) {
    if (x <= 0.0) return 0.0;
    return x * x * x * x / expm1(x);
}

static double or_gl_panel(double a, double b) {
    double h = 0.5 * (b - a), m = 0.5 * (b + a), s = 0.0;
    for (int i = 0; i < 10; ++i) s += or_gl_w[i] * or_compton_integrand(m + h * or_gl_x[i]);
    return s * h;
}

/* Integral of x^4/(e^x-1) over [a,b] by composite Gauss-Legendre, unit panels. */
static double or_compton_integral(double a, double b) {
    or_gl_init();
    double s = 0.0;
    double lo = a;
    while (lo < b) {
        double hi = floor(lo) + 1.0;
        if (hi > b) hi = b;
        s += or_gl_panel(lo, hi);
        lo = hi;
    }
    return s;
}

double or_compton_cdf(double X) {
    if (!(X > 0.0)) return 0.0;
    return or_compton_integral(0.0, X) / (24.0 * OR_ZETA5);
}

/* Upper tail.  For X >= 2 by the mixture identity 1/(e^x-1) = sum_j e^{-jx}:
 * Q(X) = sum_j j^-5 Gamma(5, jX)/(24 zeta5), Gamma(5,y) = 24 e^-y sum_{m<5} y^m/m!
 * (positive terms, e^{-jX} convergence); below, by quadrature.            */
double or_compton_ccdf(double X) {
    if (!(X > 0.0)) return 1.0;
    if (X < 2.0) return or_compton_integral(X, X + 60.0) / (24.0 * OR_ZETA5);
    double s = 0.0;
    for (int j = 1; j < 200; ++j) {
        double y = (double)j * X;
        double poly = 1.0 + y + y * y / 2.0 + y * y * y / 6.0 + y * y * y * y / 24.0;
        double t = exp(-y) * poly / pow((double)j, 5.0);
        s += t;
        if (t < 1e-18 * s) break;
    }
    return s / OR_ZETA5;
}

/* Safeguarded Newton on a monotone CDF: f(x) = F(x) - target, f' = pdf. */
static double or_invert(double (*cdf)(double, const double*), double (*pdf)(double, const double*),
                        const double* par, double target, int upper, double lo, double hi) {
    double x = (5.0 > lo && 5.0 < hi) ? 5.0 : 0.5 * (lo + hi);
    for (int it = 0; it < 400; ++it) {
        double F = cdf(x, par);
        double f = upper ? (target - F) : (F - target);   /* increasing in x */
        if (f > 0.0) hi = x; else lo = x;
        double d = pdf(x, par);
        double xn = (d > 0.0) ? x - f / d : 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-14 * fabs(x) || hi - lo <= 1e-14 * fabs(x)) { x = xn; break; }
        x = xn;
    }
    return x;
}

static double cdf_c(double x, const double* par) { (void)par; return or_compton_cdf(x); }
static double ccdf_c(double x, const double* par) { (void)par; return or_compton_ccdf(x); }
static double pdf_c(double x, const double* par) {
    (void)par;
    return or_compton_integrand(x) / (24.0 * OR_ZETA5);
}

/* x = E/T of a Compton-like event: number density x^4/(e^x-1)/(24 zeta(5)).
 * (The power spectrum of eq. compton_kernel is x times this density.)       */
double or_compton_x(double u) {
    if (u <= 0.5) return or_invert(cdf_c, pdf_c, NULL, u, 0, 0.0, 200.0);
    return or_invert(ccdf_c, pdf_c, NULL, 1.0 - u, 1, 0.0, 200.0);
}

/* Regularised lower incomplete gamma P(a, y) by its power series. */
double or_gammainc_P(double a, double y) {
    if (!(y > 0.0)) return 0.0;
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 100000; ++n) {
        term *= y / (a + n);
        sum += term;
        if (term < sum * 1e-18) break;
    }
    return sum * exp(-y + a * log(y) - lgamma(a));
}

/* Regularised upper incomplete gamma Q(a, y): Legendre's continued fraction
 * for y >= a + 1, evaluated by the modified Lentz algorithm (Lentz, Appl.
 * Opt. 15 (1976) 668; Thompson and Barnett, J. Comput. Phys. 64 (1986) 490;
 * as presented in Press et al., Numerical Recipes, Sec. 6.2), otherwise
 * 1 - P.                                                                   */
double or_gammainc_Q(double a, double y) {
    if (!(y > 0.0)) return 1.0;
    if (y < a + 1.0) return 1.0 - or_gammainc_P(a, y);
    const double tiny = 1e-300;
    double b = y + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 100000; ++i) {
        double an = -(double)i * ((double)i - a);
        b += 2.0;
        d = an * d + b; if (fabs(d) < tiny) d = tiny;
        c = b + an / c; if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double del = d * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-17) break;
    }
    return exp(-y + a * log(y) - lgamma(a)) * h;
}

static double cdf_g(double y, const double* par) { return or_gammainc_P(par[0], y); }
static double ccdf_g(double y, const double* par) { return or_gammainc_Q(par[0], y); }
static double pdf_g(double y, const double* par) {
    if (!(y > 0.0)) return 0.0;
    return exp((par[0] - 1.0) * log(y) - y - lgamma(par[0]));
}

/* y such that P(k, y) = u (the Gamma(k,1) quantile). */
double or_gamma_x(double k, double u) {
    double par[1] = {k};
    if (u <= 0.5) return or_invert(cdf_g, pdf_g, par, u, 0, 0.0, 200.0);
    return or_invert(ccdf_g, pdf_g, par, 1.0 - u, 1, 0.0, 200.0);
}

/* Quantiles by upper-tail probability q (the x with P(X > x) = q), for
 * checking tables far into the tail where 1 - u is not representable.    */
double or_compton_x_tail(double q) {
    return or_invert(ccdf_c, pdf_c, NULL, q, 1, 0.0, 400.0);
}

double or_gamma_x_tail(double k, double q) {
    double par[1] = {k};
    return or_invert(ccdf_g, pdf_g, par, q, 1, 0.0, 400.0);
}

/* Draws from the spectra cut below a threshold (M4): the quantile at
 * F(xm) + u (1 - F(xm)), the upper tail (1 - u)(1 - F(xm)) inverted directly
 * where it is the smaller side.  xm = 0 reproduces the uncut draws.         */
double or_compton_x_above(double xm, double u) {
    const double F = or_compton_cdf(xm), Q = or_compton_ccdf(xm);
    const double lo = F + u * Q, up = (1.0 - u) * Q;
    if (lo <= 0.5) return or_invert(cdf_c, pdf_c, NULL, lo, 0, 0.0, 200.0);
    return or_invert(ccdf_c, pdf_c, NULL, up, 1, 0.0, 200.0);
}

double or_gamma_x_above(double k, double ym, double u) {
    double par[1] = {k};
    const double F = or_gammainc_P(k, ym), Q = or_gammainc_Q(k, ym);
    const double lo = F + u * Q, up = (1.0 - u) * Q;
    if (lo <= 0.5) return or_invert(cdf_g, pdf_g, par, lo, 0, 0.0, 200.0);
    return or_invert(ccdf_g, pdf_g, par, up, 1, 0.0, 200.0);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics: energy histogram bin (App. B).                              */
/* ------------------------------------------------------------------------ */
int32_t or_hist_bin(const or_params* prm, double E) {
    int32_t nb = prm->hist_nbins;
    double t;
    if (prm->hist_log) t = log(E / prm->hist_lo_keV) / log(prm->hist_hi_keV / prm->hist_lo_keV);
    else t = (E - prm->hist_lo_keV) / (prm->hist_hi_keV - prm->hist_lo_keV);
    double b = floor(t * (double)nb);
    if (!(b >= 0.0)) return nb;          /* underflow (and NaN) */
    if (b >= (double)nb) return nb + 1;  /* overflow */
    return (int32_t)b;
}

static void or_hist_add(double* hist, const or_params* prm, int ch, double E_keV, double wphys) {
    if (!hist) return;
    int32_t b = or_hist_bin(prm, E_keV);
    hist[(int64_t)ch * (prm->hist_nbins + 2) + b] += wphys * E_keV;
}

/* ------------------------------------------------------------------------ */
/* Deposit (NGP): density = sum of physical weights in the cell / volume.    */
/* ------------------------------------------------------------------------ */
void or_deposit(const or_species* s, int64_t ncell, double V, double* dens) {
    double* acc = (double*)calloc((size_t)ncell, sizeof(double));
    for (int64_t i = 0; i < s->n; ++i) acc[s->cell[i]] += s->w[i];
    for (int64_t c = 0; c < ncell; ++c) dens[c] = acc[c] / V;
    free(acc);
}

static uint64_t or_product_id(uint64_t next_id, int64_t rank) {
    return (next_id + (uint64_t)rank) | (1ull << 63);
}

static void or_put(or_products* out, int64_t slot, const or_species* par, int64_t i,
                   const double p[3], double w, uint64_t id, int ch) {
    for (int d = 0; d < 3; ++d) {
        out->x[d][slot] = par->x[d] ? par->x[d][i] : 0.0;
        out->p[d][slot] = p[d];
    }
    out->w[slot] = w;
    out->id[slot] = id;
    out->cell[slot] = par->cell[i];
    if (out->parent) out->parent[slot] = i;
    if (out->chan) out->chan[slot] = ch;
}

/* ------------------------------------------------------------------------ */
/* Macro-event count of a conversion operator (Sec. II.F.1, eq. poisson_macro) */
/* for a parent of physical weight w whose products weigh wprod.  The paper   */
/* depletes the parent by the converted weight and says nothing of a parent   */
/* lighter than one product.  Reading: such a parent converts whole, with     */
/* probability lambda wprod / w (the conversion probability P of the plain    */
/* rate), so the mean converted weight stays w P; light_mode = 1 keeps the    */
/* Poisson count for it, which converts it whole whenever K >= 1 and moves on */
/* average only w P (w / wprod).                                              */
/* ------------------------------------------------------------------------ */
static int32_t or_conversion_count(const or_params* prm, double lam, double lam_eff, double w,
                                   double wprod, double u) {
    if (prm->light_mode == 0 && w < wprod)
        return (lam > 0.0 && u < lam / (w / wprod)) ? 1 : 0;
    return or_poisson(lam_eff, u);
}

/* ------------------------------------------------------------------------ */
/* Forward Primakoff conversion on photon macroparticles (Sec. II.F.1).      */
/* Returns the number of products, or -(required) when out->cap is too small
 * (then nothing is modified).                                              */
/* ------------------------------------------------------------------------ */
int64_t or_emit_primakoff(const or_grid* g, const or_params* prm, const or_cell* cells,
                          or_species* ph, const double* lam_in, int64_t step,
                          uint64_t next_id, or_products* out, double* hist, double* stats,
                          double* lam_out, int32_t* K_out) {
    const int64_t n = ph->n;
    const double dtp = or_dt_phys(g);
    const double wprod = prm->w_a * prm->wa_mul[0];
    double* lam = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t* K = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t total = 0;
#pragma omp parallel for reduction(+ : total) if (n > 8192)
    for (int64_t i = 0; i < n; ++i) {
        double l;
        if (lam_in) {
            l = lam_in[i];
        } else {
            double px = ph->p[0][i], py = ph->p[1][i], pz = ph->p[2][i];
            double om = OR_ME_KEV * sqrt(px * px + py * py + pz * pz);
            double G = or_gamma_conv(&cells[ph->cell[i]], prm, om);    /* eq. prim_rate, M2 */
            double P = -expm1(-G * dtp);                                /* eq. prim_prob */
            l = ph->w[i] * P / wprod;                                   /* lambda_P */
        }
        if (!(ph->w[i] > 0.0)) l = 0.0;
        lam[i] = l;
        double ws; int capped;
        double le = or_cap(l, prm, &ws, &capped);
        uint32_t r[4];
        or_draw(prm->seed, ph->id[i], (uint32_t)step, 0, 0, r);
        K[i] = or_conversion_count(prm, l, le, ph->w[i], wprod, or_u53(r[0], r[1]));
        total += K[i];
    }
    if (lam_out) memcpy(lam_out, lam, sizeof(double) * (size_t)n);
    if (K_out) memcpy(K_out, K, sizeof(int32_t) * (size_t)n);
    if (!out || total > out->cap) { free(lam); free(K); return -total; }
    int64_t rank = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (K[i] == 0) continue;
        double ws; int capped;
        (void)or_cap(lam[i], prm, &ws, &capped);
        double wp = wprod * ws;                        /* eq. wa_rescaled */
        double dep = (double)K[i] * wp;
        if (dep > ph->w[i]) {                          /* convert the whole parent */
            wp = ph->w[i] / (double)K[i];
            dep = ph->w[i];
            if (stats) stats[OR_ST_OVERDEPLETED] += 1.0;
        }
        if (stats && capped) stats[OR_ST_CAPPED] += 1.0;
        double p[3] = {ph->p[0][i], ph->p[1][i], ph->p[2][i]};     /* product inherits p */
        double E = OR_ME_KEV * sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        if (prm->m_a_keV > 0.0) {                      /* M3: energy kept, |p| reduced */
            const double sc = E > prm->m_a_keV ? sqrt((E - prm->m_a_keV) * (E + prm->m_a_keV)) / E
                                               : 0.0;     /* (a mean handed in below threshold) */
            p[0] *= sc; p[1] *= sc; p[2] *= sc;
        }
        for (int32_t k = 0; k < K[i]; ++k) {
            or_put(out, rank, ph, i, p, wp, or_product_id(next_id, rank), 0);
            ++rank;
            or_hist_add(hist, prm, 0, E, wp);
            if (stats) {
                stats[OR_ST_EVENTS_P] += 1.0;
                stats[OR_ST_NUM_P] += wp;
                stats[OR_ST_EN_P] += wp * E;
            }
        }
        ph->w[i] = (dep >= ph->w[i]) ? 0.0 : ph->w[i] - dep;   /* number-conserving depletion */
    }
    free(lam); free(K);
    return total;
}

/* Isotropic unit vector from two uniforms (cos theta = 2u-1, phi = 2 pi u). */
static void or_isotropic(double u1, double u2, double n[3]) {
    double mu = 2.0 * u1 - 1.0;
    double phi = 2.0 * OR_PI * u2;
    double s = sqrt(fmax(0.0, 1.0 - mu * mu));
    n[0] = s * cos(phi); n[1] = s * sin(phi); n[2] = mu;
}

/* ------------------------------------------------------------------------ */
/* Thermal-bath emission on electrons: Compton-like (Sec. II.G) and          */
/* bremsstrahlung (Sec. II.H).  lam_in (optional) is [2][n]: Compton, brems. */
/* fb is [ncell][4]: dE (m_e c^2 * count), dPx, dPy, dPz (m_e c * count).    */
/* ------------------------------------------------------------------------ */
/* Fraction of channel ch's sampled number spectrum above the axion mass (M4);
 * 1 for massless axions. */
static double or_thermal_fraction(const or_params* prm, int ch, double T) {
    const double m = prm->m_a_keV;
    if (!(m > 0.0)) return 1.0;
    return ch == 1 ? or_compton_ccdf(m / T)
                   : or_gammainc_Q(prm->brems_k, m / (prm->brems_theta * T));
}

/* Energy E [keV] and momentum magnitude pm [m_e c] of a thermal product of
 * channel ch (1 Compton-like, 2 brems) drawn at uniform u (Secs. II.G-H; M4). */
static void or_thermal_energy(const or_params* prm, int ch, double T, double u, double* E,
                              double* pm) {
    const double m = prm->m_a_keV;
    double x;
    if (!(m > 0.0)) {
        x = (ch == 1) ? or_compton_x(u) : prm->brems_theta * or_gamma_x(prm->brems_k, u);
        *E = T * x;
        *pm = *E / OR_ME_KEV;
        return;
    }
    x = (ch == 1) ? or_compton_x_above(m / T, u)
                  : prm->brems_theta * or_gamma_x_above(prm->brems_k, m / (prm->brems_theta * T), u);
    *E = T * x;
    *pm = (*E > m) ? sqrt((*E - m) * (*E + m)) / OR_ME_KEV : 0.0;
}

int64_t or_emit_thermal(const or_grid* g, const or_params* prm, const or_cell* cells,
                        const or_species* el, const double* lam_in, int64_t step,
                        uint64_t next_id, or_products* out, double* fb, double* hist,
                        double* stats, double* lam_out, int32_t* K_out) {
    const int64_t n = el->n;
    const double dtp = or_dt_phys(g);
    const double wC = prm->w_a * prm->wa_mul[1], wB = prm->w_a * prm->wa_mul[2];
    const int onC = (prm->channels & OR_CH_C) != 0, onB = (prm->channels & OR_CH_B) != 0;
    double* lam = (double*)malloc(sizeof(double) * (size_t)(2 * n + 1));
    int32_t* K = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * n + 1));
    int64_t total = 0;
#pragma omp parallel for reduction(+ : total) if (n > 8192)
    for (int64_t i = 0; i < n; ++i) {
        const or_cell* c = &cells[el->cell[i]];
        double lC, lB;
        if (lam_in) { lC = lam_in[i]; lB = lam_in[n + i]; }
        else {
            lC = el->w[i] * c->G_C * dtp / wC;      /* eq. lambda_macro */
            lB = el->w[i] * c->G_B * dtp / wB;
            lC *= or_thermal_fraction(prm, 1, c->T);   /* M4: the part above m */
            lB *= or_thermal_fraction(prm, 2, c->T);
        }
        if (!onC) lC = 0.0;
        if (!onB) lB = 0.0;
        lam[i] = lC; lam[n + i] = lB;
        uint32_t r[4];
        or_draw(prm->seed, el->id[i], (uint32_t)step, 1, 0, r);
        double ws; int capped;
        K[i] = or_poisson(or_cap(lC, prm, &ws, &capped), or_u53(r[0], r[1]));
        K[n + i] = or_poisson(or_cap(lB, prm, &ws, &capped), or_u53(r[2], r[3]));
        total += K[i] + K[n + i];
    }
    if (lam_out) memcpy(lam_out, lam, sizeof(double) * (size_t)(2 * n));
    if (K_out) memcpy(K_out, K, sizeof(int32_t) * (size_t)(2 * n));
    if (!out || total > out->cap) { free(lam); free(K); return -total; }
    int64_t rank = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int ch = 1; ch <= 2; ++ch) {
            int32_t Kc = K[(ch - 1) * n + i];
            if (Kc == 0) continue;
            const or_cell* c = &cells[el->cell[i]];
            double ws; int capped;
            (void)or_cap(lam[(ch - 1) * n + i], prm, &ws, &capped);
            if (stats && capped) stats[OR_ST_CAPPED] += 1.0;
            double wp = (ch == 1 ? wC : wB) * ws;
            for (int32_t k = 0; k < Kc; ++k) {
                uint32_t r[4];
                or_draw(prm->seed, el->id[i], (uint32_t)step, (uint32_t)(ch + 1), (uint32_t)k, r);
                double u = or_u24(r[0]);
                double E, pm;
                or_thermal_energy(prm, ch, c->T, u, &E, &pm);
                double nh[3];
                or_isotropic(or_u24(r[1]), or_u24(r[2]), nh);
                double p[3] = {pm * nh[0], pm * nh[1], pm * nh[2]};
                or_put(out, rank, el, i, p, wp, or_product_id(next_id, rank), ch);
                ++rank;
                or_hist_add(hist, prm, ch, E, wp);
                if (fb) {                               /* energy/momentum leave the plasma */
                    double* f = &fb[(int64_t)el->cell[i] * 4];
                    f[0] -= wp * E / OR_ME_KEV;
                    f[1] -= wp * p[0]; f[2] -= wp * p[1]; f[3] -= wp * p[2];
                }
                if (stats) {
                    stats[OR_ST_EVENTS_P + ch] += 1.0;
                    stats[OR_ST_NUM_P + ch] += wp;
                    stats[OR_ST_EN_P + ch] += wp * E;
                }
            }
        }
    }
    free(lam); free(K);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Thermal emission by per-cell superposition.                               */
/* In a cell the electrons' macro-event counts are independent,              */
/* K_e ~ Poisson(lambda_e) with lambda_e = w_e coef (eq. lambda_macro), coef  */
/* = Gamma dt_phys / w_prod per channel.  The same joint law is obtained by  */
/* drawing the cell's total N ~ Poisson(Lambda), Lambda = sum_e lambda_e (a   */
/* sum of independent Poisson variables is Poisson) and assigning each of    */
/* the N events to electron e with probability lambda_e / Lambda (given the  */
/* sum, the counts are multinomial).  Capped electrons (eqs. lambda_eff,     */
/* wa_rescaled) enter with min(lambda_e, cap) and their products carry the   */
/* weight factor lambda_e / cap.  Work is per cell and per event instead of  */
/* per electron.                                                             */
/* Electrons are grouped by cell: off[c] .. off[c+1]-1.  coef_in[2 ncell]    */
/* (Compton, brems) and W_in[ncell] (sum of the cell's weights) replace the  */
/* computed values when given.  Lambda in a cell is coef W when no electron  */
/* of the cell reaches the cap, else the sum of min(w_e coef, cap) in index  */
/* order.  A mean above 500 is split into m = ceil(Lambda/500) equal parts, */
/* each drawn by inversion (a sum of independent Poisson variables).         */
/* Random numbers: the cell's counts from stream 5 keyed by the cell index,  */
/* block = part (words 0-1 Compton, 2-3 brems); event j of channel ch: the   */
/* electron from stream 6, block (ch-1) 2^23 + j (words 0-1, u53, inverse    */
/* CDF over the cell's electrons in index order), energy and direction from  */
/* stream 6 + ch, block j, as the per-electron operator draws them.  Product */
/* order: cell, then channel, then j.                                        */
/* ------------------------------------------------------------------------ */
int64_t or_emit_thermal_cells(const or_grid* g, const or_params* prm, const or_cell* cells,
                              const or_species* el, const int64_t* off, int64_t ncell,
                              const double* coef_in, const double* W_in, int64_t step,
                              uint64_t next_id, or_products* out, double* fb, double* hist,
                              double* stats, double* Lambda_out, int32_t* N_out) {
    const double dtp = or_dt_phys(g);
    const double wprod[3] = {0.0, prm->w_a * prm->wa_mul[1], prm->w_a * prm->wa_mul[2]};
    const int on[3] = {0, (prm->channels & OR_CH_C) != 0, (prm->channels & OR_CH_B) != 0};
    double cap = prm->lambda_cap;
    if (!(cap <= OR_LAMBDA_HARD_CAP)) cap = OR_LAMBDA_HARD_CAP;
    double* coef = (double*)malloc(sizeof(double) * (size_t)(2 * ncell + 1));
    double* Lam = (double*)malloc(sizeof(double) * (size_t)(2 * ncell + 1));
    int32_t* N = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * ncell + 1));
    int64_t total = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        double W = 0.0, wmax = 0.0;
        for (int64_t e = off[c]; e < off[c + 1]; ++e) {
            W += el->w[e];
            if (el->w[e] > wmax) wmax = el->w[e];
        }
        if (W_in) W = W_in[c];
        for (int ch = 1; ch <= 2; ++ch) {
            double k = coef_in ? coef_in[(ch - 1) * ncell + c]
                               : (ch == 1 ? cells[c].G_C : cells[c].G_B) * dtp / wprod[ch] *
                                     or_thermal_fraction(prm, ch, cells[c].T);
            if (!on[ch]) k = 0.0;
            coef[(ch - 1) * ncell + c] = k;
            double L;
            if (!(wmax * k > cap)) L = k * W;
            else {
                L = 0.0;
                for (int64_t e = off[c]; e < off[c + 1]; ++e) {
                    double le = el->w[e] * k;
                    L += le < cap ? le : cap;
                }
            }
            Lam[(ch - 1) * ncell + c] = L;
            const int32_t parts = L > 500.0 ? (int32_t)ceil(L / 500.0) : 1;
            const double Lp = L / (double)parts;
            int32_t Nc = 0;
            for (int32_t q = 0; q < parts; ++q) {
                uint32_t r[4];
                or_draw(prm->seed, (uint64_t)c, (uint32_t)step, 5, (uint32_t)q, r);
                Nc += or_poisson_kmax(Lp, ch == 1 ? or_u53(r[0], r[1]) : or_u53(r[2], r[3]),
                                      1 << 30);
            }
            N[(ch - 1) * ncell + c] = Nc;
            total += Nc;
        }
    }
    if (Lambda_out) memcpy(Lambda_out, Lam, sizeof(double) * (size_t)(2 * ncell));
    if (N_out) memcpy(N_out, N, sizeof(int32_t) * (size_t)(2 * ncell));
    if (!out || total > out->cap) { free(coef); free(Lam); free(N); return -total; }
    int64_t rank = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        double W = 0.0, wmax = 0.0;
        for (int64_t e = off[c]; e < off[c + 1]; ++e) {
            W += el->w[e];
            if (el->w[e] > wmax) wmax = el->w[e];
        }
        if (W_in) W = W_in[c];
        for (int ch = 1; ch <= 2; ++ch) {
            const double k = coef[(ch - 1) * ncell + c];
            const double L = Lam[(ch - 1) * ncell + c];
            const int capped_cell = wmax * k > cap;
            for (int32_t j = 0; j < N[(ch - 1) * ncell + c]; ++j) {
                uint32_t r[4];
                or_draw(prm->seed, (uint64_t)c, (uint32_t)step, 6,
                        (uint32_t)((ch - 1) * (1 << 23) + j), r);
                /* the electron: inverse CDF of lambda_e / Lambda in index order */
                const double target = or_u53(r[0], r[1]) * (capped_cell ? L : W);
                int64_t pick = -1, last = -1;
                double acc = 0.0;
                for (int64_t e = off[c]; e < off[c + 1]; ++e) {
                    if (!(el->w[e] > 0.0)) continue;
                    double le = el->w[e] * k;
                    acc += capped_cell ? (le < cap ? le : cap) : el->w[e];
                    last = e;
                    if (acc > target) { pick = e; break; }
                }
                if (pick < 0) pick = last;
                const double le = el->w[pick] * k;
                const int capped = le > cap;
                const double wp = wprod[ch] * (capped ? le / cap : 1.0);
                if (stats && capped) stats[OR_ST_CAPPED] += 1.0;
                or_draw(prm->seed, (uint64_t)c, (uint32_t)step, (uint32_t)(6 + ch), (uint32_t)j, r);
                double u = or_u24(r[0]);
                double E, pm;
                or_thermal_energy(prm, ch, cells[c].T, u, &E, &pm);
                double nh[3];
                or_isotropic(or_u24(r[1]), or_u24(r[2]), nh);
                double p[3] = {pm * nh[0], pm * nh[1], pm * nh[2]};
                or_put(out, rank, el, pick, p, wp, or_product_id(next_id, rank), ch);
                ++rank;
                or_hist_add(hist, prm, ch, E, wp);
                if (fb) {
                    double* f = &fb[c * 4];
                    f[0] -= wp * E / OR_ME_KEV;
                    f[1] -= wp * p[0]; f[2] -= wp * p[1]; f[3] -= wp * p[2];
                }
                if (stats) {
                    stats[OR_ST_EVENTS_P + ch] += 1.0;
                    stats[OR_ST_NUM_P + ch] += wp;
                    stats[OR_ST_EN_P + ch] += wp * E;
                }
            }
        }
    }
    free(coef); free(Lam); free(N);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Inverse operators on axions (Sec. II.I and Sec. II.F.1): detailed-balance */
/* absorption for the thermal channels, then a->gamma conversion of what     */
/* survives.  pabs_in / lam_in optionally replace the computed probability / */
/* mean of the start-of-step axion.  Products (photons) are written to out.   */
/* ------------------------------------------------------------------------ */
int64_t or_absorb(const or_grid* g, const or_params* prm, const or_cell* cells,
                  or_species* ax, const double* pabs_in, const double* lam_in, int64_t step,
                  uint64_t next_id, or_products* out, double* fb, double* stats,
                  double* pabs_out, double* lam_out, int32_t* K_out, int32_t* absorbed_out) {
    const int64_t n = ax->n;
    const double dtp = or_dt_phys(g);
    const int thermal = prm->inverse && (prm->channels & (OR_CH_C | OR_CH_B));
    const int a2g = prm->inverse && (prm->channels & OR_CH_P);
    const double wg = prm->w_gamma_prod;
    double* pab = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* lam = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    int32_t* K = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* dead = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t total = 0;
#pragma omp parallel for reduction(+ : total) if (n > 8192)
    for (int64_t i = 0; i < n; ++i) {
        pab[i] = 0.0; lam[i] = 0.0; K[i] = 0; dead[i] = 0;
        double w = ax->w[i];
        if (!(w > 0.0)) continue;
        const or_cell* c = &cells[ax->cell[i]];
        double px = ax->p[0][i], py = ax->p[1][i], pz = ax->p[2][i];
        double p2 = px * px + py * py + pz * pz;
        double E = prm->m_a_keV > 0.0 ? or_axion_energy(prm, p2) : OR_ME_KEV * sqrt(p2);
        uint32_t r[4];
        or_draw(prm->seed, ax->id[i], (uint32_t)step, 4, 0, r);
        double P = 0.0;
        if (thermal) {
            P = pabs_in ? pabs_in[i] : -expm1(-or_gamma_abs(c, prm, E, NULL) * dtp);
            pab[i] = P;
            if (prm->absorb_mode == 0) {
                if (or_u53(r[0], r[1]) < P) { dead[i] = 1; w = 0.0; }
            } else {
                w = w - w * P;
            }
        }
        if (a2g && w > 0.0) {
            /* the mean of the start-of-step weight (eq. prim_prob: lambda is
             * proportional to the parent's weight); after a weight reduction
             * (reading O8) the survivor converts with the mean of its reduced
             * weight, i.e. that mean times (1 - P_abs) */
            double l;
            if (lam_in) l = lam_in[i];
            else {
                double G = prm->m_a_keV > 0.0
                               ? prm->prim_inv_ratio * c->G_P0 *
                                     or_F_mass(E, OR_ME_KEV * sqrt(p2), c->kappa2)   /* M3 */
                               : prm->prim_inv_ratio * or_gamma_prim(c, prm, E);
                l = ax->w[i] * (-expm1(-G * dtp)) / wg;
            }
            if (thermal && prm->absorb_mode == 1) l = l * (1.0 - P);
            lam[i] = l;
            double ws; int capped;
            K[i] = or_conversion_count(prm, l, or_cap(l, prm, &ws, &capped), w, wg,
                                       or_u53(r[2], r[3]));
        }
        total += K[i];
    }
    if (pabs_out) memcpy(pabs_out, pab, sizeof(double) * (size_t)n);
    if (lam_out) memcpy(lam_out, lam, sizeof(double) * (size_t)n);
    if (K_out) memcpy(K_out, K, sizeof(int32_t) * (size_t)n);
    if (absorbed_out) memcpy(absorbed_out, dead, sizeof(int32_t) * (size_t)n);
    if (!out || total > out->cap) { free(pab); free(lam); free(K); free(dead); return -total; }
    int64_t rank = 0;
    for (int64_t i = 0; i < n; ++i) {
        double w = ax->w[i];
        if (!(w > 0.0)) continue;
        double p[3] = {ax->p[0][i], ax->p[1][i], ax->p[2][i]};
        double pm = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        double E = prm->m_a_keV > 0.0 ? or_axion_energy(prm, pm * pm) : OR_ME_KEV * pm;
        double* f = fb ? &fb[(int64_t)ax->cell[i] * 4] : NULL;
        if (thermal) {
            double dw = dead[i] ? w : (prm->absorb_mode == 1 ? w * pab[i] : 0.0);
            if (dw > 0.0) {
                if (f) {
                    f[0] += dw * E / OR_ME_KEV;
                    f[1] += dw * p[0]; f[2] += dw * p[1]; f[3] += dw * p[2];
                }
                if (stats) {
                    stats[OR_ST_ABS_NUM] += dw; stats[OR_ST_ABS_EN] += dw * E;
                    if (dead[i]) stats[OR_ST_ABS_EVENTS] += 1.0;
                }
            }
            w = dead[i] ? 0.0 : w - dw;
            ax->w[i] = w;
        }
        if (K[i] > 0) {
            double ws; int capped;
            (void)or_cap(lam[i], prm, &ws, &capped);
            if (stats && capped) stats[OR_ST_CAPPED] += 1.0;
            double wp = wg * ws;
            double dep = (double)K[i] * wp;
            if (dep > w) { wp = w / (double)K[i]; dep = w; if (stats) stats[OR_ST_OVERDEPLETED] += 1.0; }
            double pg[3] = {p[0], p[1], p[2]};            /* M3: the photon carries E */
            if (prm->m_a_keV > 0.0) {
                const double sc = E / (OR_ME_KEV * pm);
                pg[0] *= sc; pg[1] *= sc; pg[2] *= sc;
            }
            for (int32_t k = 0; k < K[i]; ++k) {
                or_put(out, rank, ax, i, pg, wp, or_product_id(next_id, rank), 3);
                ++rank;
                if (stats) { stats[OR_ST_AG_EVENTS] += 1.0; stats[OR_ST_AG_NUM] += wp; stats[OR_ST_AG_EN] += wp * E; }
            }
            ax->w[i] = (dep >= w) ? 0.0 : w - dep;
        }
    }
    free(pab); free(lam); free(K); free(dead);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium check of the thermal inverse operators (Sec. II.I, eq.        */
/* gamma_abs: the net source vanishes bin by bin at n_eq; the relaxation     */
/* plateau of Sec. III.E).  For a population s (physical weights) and the    */
/* histogram grid of prm, per bin k (the nbins bins, then [0, lo) and        */
/* [hi, inf) as or_hist_bin numbers them):                                   */
/*   NUM   sum of w over the particles of the bin (w > 0)                     */
/*   EN    sum of w E [keV]                                                   */
/*   W2    sum of w^2                                                         */
/*   NEQ   sum over cells of V int_bin dn_eq/dE dE at the cell's T            */
/*   UEQ   the same with E dn_eq/dE                                           */
/*   NFIX  sum over cells of V int_bin dn_eq/dE q(g) (1 - e^{-t g}) dE with   */
/*         g(E) = Gamma_abs(E) dt_phys over the enabled thermal channels and  */
/*         q(g) = g / (1 - e^{-g}): the content after t steps of the Jacobi   */
/*         recursion n_{t+1} = n_t e^{-g} + n_eq g started empty (reading O6; */
/*         emission per step V n_eq g by construction of Gamma_abs); t <= 0   */
/*         gives its fixed point n_eq q(g), which tends to n_eq as g -> 0     */
/*   Z     (NUM - NFIX) / sqrt(W2), 0 where W2 = 0                            */
/* out is [7][nbins + 2].  dn_eq/dE is that of one axion state, BE or MB     */
/* (eq_stats); with mass m, E p f(E/T) / (2 pi^2 (hbar c)^3), zero below m.  */
/* Integrals: composite 10-point Gauss-Legendre on panels no wider than     */
/* T/16 inside a bin, [0, lo) on the geometric panels [lo 2^-(j+1), lo 2^-j], */
/* [hi, inf) cut at hi + 64 T; with mass, the panel starting at m is taken   */
/* in s = sqrt(E - m) (the square-root edge of p) on geometric panels.       */
/* ------------------------------------------------------------------------ */
typedef struct { const or_cell* c; const or_params* prm; double dt, t, V; } or_eq_ctx;

static void or_eq_point(const or_eq_ctx* q, double E, double out[3]) {
    out[0] = out[1] = out[2] = 0.0;
    const double m = q->prm->m_a_keV, T = q->c->T;
    if (!(E > 0.0) || !(T > 0.0) || (m > 0.0 && !(E > m))) return;
    double neq = or_dneq(E, T, q->prm->eq_stats);
    if (m > 0.0) neq *= sqrt((E - m) * (E + m)) / E;
    const double g = or_gamma_abs(q->c, q->prm, E, NULL) * q->dt;
    const double qg = g > 0.0 ? g / -expm1(-g) : 1.0;
    const double grow = q->t > 0.0 ? -expm1(-q->t * g) : 1.0;
    out[0] = q->V * neq;
    out[1] = q->V * neq * E;
    out[2] = q->V * neq * qg * grow;
}

/* 10-point Gauss-Legendre over [a, b]. */
static void or_eq_panel(const or_eq_ctx* q, double a, double b, double acc[3]) {
    double v[3];
    const double h = 0.5 * (b - a), mid = 0.5 * (b + a);
    for (int i = 0; i < 10; ++i) {
        or_eq_point(q, mid + h * or_gl_x[i], v);
        for (int k = 0; k < 3; ++k) acc[k] += h * or_gl_w[i] * v[k];
    }
}

/* The same over E = m + s^2, s in [s0, s1]. */
static void or_eq_panel_s(const or_eq_ctx* q, double m, double s0, double s1, double acc[3]) {
    double v[3];
    const double h = 0.5 * (s1 - s0), mid = 0.5 * (s1 + s0);
    for (int i = 0; i < 10; ++i) {
        const double sx = mid + h * or_gl_x[i];
        or_eq_point(q, m + sx * sx, v);
        for (int k = 0; k < 3; ++k) acc[k] += h * or_gl_w[i] * v[k] * 2.0 * sx;
    }
}

/* [a, b] in panels no wider than hmax, split at the mass m; the panel starting at m
 * is taken in s = sqrt(E - m) on the geometric panels [S 2^-(j+1), S 2^-j], which
 * resolve the growth of Gamma_abs ~ E/p towards the threshold. */
static void or_eq_range(const or_eq_ctx* q, double a, double b, double hmax, double acc[3]) {
    const double m = q->prm->m_a_keV;
    if (m > 0.0) {
        if (b <= m) return;
        if (a < m) {
            const double e = fmin(b, m + hmax), S = sqrt(e - m);
            for (int j = 0; j < 48; ++j) or_eq_panel_s(q, m, ldexp(S, -(j + 1)), ldexp(S, -j), acc);
            a = e;
        }
    }
    if (!(b > a)) return;
    const int np = (int)ceil((b - a) / hmax);
    const int n = np < 1 ? 1 : np;
    for (int j = 0; j < n; ++j)
        or_eq_panel(q, a + (b - a) * j / n, j + 1 == n ? b : a + (b - a) * (j + 1) / n, acc);
}

void or_equilibrium(const or_grid* g, const or_params* prm, const or_cell* cells, int64_t ncell,
                    const or_species* s, double t_steps, double* out) {
    or_gl_init();
    const int32_t nb = prm->hist_nbins, nbh = nb + 2;
    for (int64_t k = 0; k < 7 * (int64_t)nbh; ++k) out[k] = 0.0;
    double* NUM = out; double* EN = out + nbh; double* W2 = out + 2 * nbh;
    double* NEQ = out + 3 * nbh; double* UEQ = out + 4 * nbh; double* NFIX = out + 5 * nbh;
    double* Z = out + 6 * nbh;
    for (int64_t i = 0; i < s->n; ++i) {
        const double w = s->w[i];
        if (!(w > 0.0)) continue;
        const double p2 = s->p[0][i] * s->p[0][i] + s->p[1][i] * s->p[1][i] + s->p[2][i] * s->p[2][i];
        const double E = prm->m_a_keV > 0.0 ? or_axion_energy(prm, p2) : OR_ME_KEV * sqrt(p2);
        const int32_t b = or_hist_bin(prm, E);
        NUM[b] += w; EN[b] += w * E; W2[b] += w * w;
    }
    double* per = (double*)malloc(sizeof(double) * 3 * (size_t)nbh * (size_t)(ncell > 0 ? ncell : 1));
    const double lo = prm->hist_lo_keV, hi = prm->hist_hi_keV;
#pragma omp parallel for schedule(dynamic, 4) if (ncell > 16)
    for (int64_t c = 0; c < ncell; ++c) {
        or_eq_ctx q = {&cells[c], prm, or_dt_phys(g), t_steps, or_V_cell(g)};
        const double T = cells[c].T, hmax = T / 16.0;
        double* r = per + 3 * (size_t)nbh * (size_t)c;
        for (int32_t k = 0; k < nbh; ++k) {
            double acc[3] = {0.0, 0.0, 0.0};
            if (T > 0.0) {
                if (k < nb) {
                    double a, b;
                    if (prm->hist_log) { a = lo * pow(hi / lo, (double)k / nb); b = lo * pow(hi / lo, (double)(k + 1) / nb); }
                    else { a = lo + (hi - lo) * k / nb; b = lo + (hi - lo) * (k + 1) / nb; }
                    or_eq_range(&q, a, b, hmax, acc);
                } else if (k == nb) {
                    for (int j = 0; j < 60 && lo > 0.0; ++j)
                        or_eq_range(&q, ldexp(lo, -(j + 1)), ldexp(lo, -j), hmax, acc);
                } else {
                    or_eq_range(&q, hi, hi + 64.0 * T, hmax, acc);
                }
            }
            r[3 * k] = acc[0]; r[3 * k + 1] = acc[1]; r[3 * k + 2] = acc[2];
        }
    }
    for (int64_t c = 0; c < ncell; ++c) {
        const double* r = per + 3 * (size_t)nbh * (size_t)c;
        for (int32_t k = 0; k < nbh; ++k) { NEQ[k] += r[3 * k]; UEQ[k] += r[3 * k + 1]; NFIX[k] += r[3 * k + 2]; }
    }
    free(per);
    for (int32_t k = 0; k < nbh; ++k) Z[k] = W2[k] > 0.0 ? (NUM[k] - NFIX[k]) / sqrt(W2[k]) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Canonical buffer order: a stable counting sort by cell -- the particles of */
/* each cell in their previous order -- dropping the particles of zero weight */
/* (and any whose cell is off the grid).  In place; returns the new length.  */
/* off[ncell+1] (optional) receives the cell offsets.                        */
/* ------------------------------------------------------------------------ */
int64_t or_sort_cells(or_species* s, int64_t ncell, int64_t* off) {
    const int64_t n = s->n;
    int64_t* start = (int64_t*)calloc((size_t)(ncell + 1), sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        if (s->w[i] > 0.0 && s->cell[i] >= 0 && s->cell[i] < ncell) start[s->cell[i] + 1] += 1;
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    const int64_t m = start[ncell];
    if (off) memcpy(off, start, sizeof(int64_t) * (size_t)(ncell + 1));
    double* tmp = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * 8);
    uint64_t* tid = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
    int32_t* tcell = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int64_t* next = start;              /* next free slot of each cell */
    for (int64_t i = 0; i < n; ++i) {
        if (!(s->w[i] > 0.0) || s->cell[i] < 0 || s->cell[i] >= ncell) continue;
        const int64_t d = next[s->cell[i]]++;
        for (int k = 0; k < 3; ++k) { tmp[8 * d + k] = s->x[k][i]; tmp[8 * d + 3 + k] = s->p[k][i]; }
        tmp[8 * d + 6] = s->w[i];
        tid[d] = s->id[i];
        tcell[d] = s->cell[i];
    }
    for (int64_t d = 0; d < m; ++d) {
        for (int k = 0; k < 3; ++k) { s->x[k][d] = tmp[8 * d + k]; s->p[k][d] = tmp[8 * d + 3 + k]; }
        s->w[d] = tmp[8 * d + 6];
        s->id[d] = tid[d];
        s->cell[d] = tcell[d];
    }
    free(tmp); free(tid); free(tcell); free(start);
    s->n = m;
    return m;
}

/* ------------------------------------------------------------------------ */
/* Conservative feedback: affine momentum remap (Sec. II.J.1, eqs.           */
/* cell_moments to b_def) and temperature estimate/relaxation (Sec. II.J.2,  */
/* eqs. Te_est, Te_relax).  Electrons are grouped by cell (off[ncell+1]).    */
/* moments_out (optional) is [ncell][5]: W, Px, Py, Pz, U2 before the remap. */
/* ------------------------------------------------------------------------ */
void or_feedback(const or_grid* g, const or_params* prm, int64_t ncell, const int64_t* off,
                 or_species* el, const double* fb, double* T, double* stats,
                 double* moments_out) {
    (void)g;
    const double mu = 1.0;   /* electrons: mass in units of m_e */
    for (int64_t c = 0; c < ncell; ++c) {
        double W = 0.0, P[3] = {0.0, 0.0, 0.0}, U2 = 0.0;
        for (int64_t i = off[c]; i < off[c + 1]; ++i) {
            double w = el->w[i];
            double px = el->p[0][i], py = el->p[1][i], pz = el->p[2][i];
            W += w;
            P[0] += w * px; P[1] += w * py; P[2] += w * pz;
            U2 += w * (px * px + py * py + pz * pz);
        }
        if (moments_out) {
            double* m = &moments_out[c * 5];
            m[0] = W; m[1] = P[0]; m[2] = P[1]; m[3] = P[2]; m[4] = U2;
        }
        if (!(W > 0.0)) continue;
        const double* f = fb ? &fb[c * 4] : NULL;
        double dE = f ? f[0] : 0.0;
        double dP[3] = {f ? f[1] : 0.0, f ? f[2] : 0.0, f ? f[3] : 0.0};
        double P2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
        double var = U2 - P2 / W;                                       /* eq. var_unnormalized */
        double pbar[3] = {P[0] / W, P[1] / W, P[2] / W};
        double delta[3] = {dP[0] / W, dP[1] / W, dP[2] / W};            /* eq. delta_def */
        double dP2 = delta[0] * delta[0] + delta[1] * delta[1] + delta[2] * delta[2];
        double dotdP = delta[0] * P[0] + delta[1] * P[1] + delta[2] * P[2];
        double dEbulk = (2.0 * dotdP + W * dP2) / (2.0 * mu);          /* eq. dE_bulk */
        double dEth = dE - dEbulk;                                      /* eq. dE_th */
        double var_new = var + 2.0 * mu * dEth;                         /* eq. var_new */
        int cold = !(var > 1e-14 * (U2 + 1e-300));
        double S = 1.0;
        if (cold) {
            var_new = var;
            if (stats) { stats[OR_ST_COLD_CELLS] += 1.0; stats[OR_ST_UNAPPLIED_E] += dEth; }
        } else {
            if (var_new < 0.0) {
                if (stats) { stats[OR_ST_CLAMPED_CELLS] += 1.0; stats[OR_ST_UNAPPLIED_E] += -var_new / (2.0 * mu); }
                var_new = 0.0;
            }
            S = sqrt(var_new / var);                                    /* eq. s_def */
        }
        if (prm->feedback) {
            double b[3];
            for (int d = 0; d < 3; ++d) b[d] = (1.0 - S) * pbar[d] + delta[d];   /* eq. b_def */
            for (int64_t i = off[c]; i < off[c + 1]; ++i)
                for (int d = 0; d < 3; ++d) el->p[d][i] = S * el->p[d][i] + b[d];  /* eq. affine_map */
        }
        if (prm->T_mode == 2) {
            double Test = OR_ME_KEV / 3.0 * var_new / W;                /* eq. Te_est */
            double Tn = (1.0 - prm->r_relax) * T[c] + prm->r_relax * Test;   /* eq. Te_relax */
            if (Tn < prm->T_floor_keV) Tn = prm->T_floor_keV;
            if (Tn > prm->T_ceil_keV) Tn = prm->T_ceil_keV;
            T[c] = Tn;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Ballistic push of massless particles, v = p/|p| (Sec. II.B), periodic,    */
/* then the NGP cell index.  The positions are advanced in the precision of  */
/* the particle storage (prec32 = 1: binary32) with correctly rounded       */
/* operations only, so that the cell index is decided identically by any    */
/* IEEE implementation of the same steps.                                    */
/* ------------------------------------------------------------------------ */
void or_push(const or_grid* g, or_species* ax, int32_t prec32, double m_a_keV) {
    const double dtdx64 = g->dt / g->dx;
    const float dtdx32 = (float)dtdx64;
    const double mu = m_a_keV / OR_ME_KEV, mu2 = mu * mu;   /* v = p / sqrt(p^2 + mu^2) */
    const float mu2f = (float)mu2;
    for (int64_t i = 0; i < ax->n; ++i) {
        int64_t cell = 0, stride = 1;
        if (prec32) {
            float px = (float)ax->p[0][i], py = (float)ax->p[1][i], pz = (float)ax->p[2][i];
            float s = fmaf(pz, pz, fmaf(py, py, fmaf(px, px, mu2f)));   /* M1 */
            float inv = s > 0.0f ? 1.0f / sqrtf(s) : 0.0f;
            float pv[3] = {px, py, pz};
            for (int d = 0; d < 3; ++d) {
                int32_t nd = g->n[d];
                float x = (float)ax->x[d][i];
                if (d < g->ndim) {
                    float v = pv[d] * inv;
                    x = fmaf(v, dtdx32, x);
                    if (x < 0.0f) x = x + (float)nd;
                    if (x >= (float)nd) x = x - (float)nd;
                    ax->x[d][i] = (double)x;
                }
                int64_t ix = (int64_t)floorf(x);
                if (ix < 0) ix = 0;
                if (ix > nd - 1) ix = nd - 1;
                cell += ix * stride;
                stride *= nd;
            }
        } else {
            double px = ax->p[0][i], py = ax->p[1][i], pz = ax->p[2][i];
            double s = fma(pz, pz, fma(py, py, fma(px, px, mu2)));
            double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
            double pv[3] = {px, py, pz};
            for (int d = 0; d < 3; ++d) {
                int32_t nd = g->n[d];
                double x = ax->x[d][i];
                if (d < g->ndim) {
                    double v = pv[d] * inv;
                    x = fma(v, dtdx64, x);
                    if (x < 0.0) x = x + (double)nd;
                    if (x >= (double)nd) x = x - (double)nd;
                    ax->x[d][i] = x;
                }
                int64_t ix = (int64_t)floor(x);
                if (ix < 0) ix = 0;
                if (ix > nd - 1) ix = nd - 1;
                cell += ix * stride;
                stride *= nd;
            }
        }
        ax->cell[i] = (int32_t)cell;
    }
}

/* ------------------------------------------------------------------------ */
/* Rate-surrogate training data.                                            */
/* ------------------------------------------------------------------------ */

/* F(s) by quadrature of the angular integral behind the screened cross
 * section: with t = 1 - cos(theta) it reads (1/2) int_0^2 (2 - t)/(t + b) dt,
 * b = 2/s; composite 10-point Gauss-Legendre on panels that halve towards
 * t = 0, down to well below the screening width b.                         */
double or_F_quad(double s) {
    if (!(s > 0.0)) return 0.0;
    or_gl_init();
    const double b = 2.0 / s;
    int J = 12;
    while (2.0 * pow(0.5, J) > 1e-3 * b && J < 200) ++J;
    double sum = 0.0, hi = 2.0;
    for (int j = 1; j <= J + 1; ++j) {
        double lo = (j <= J) ? 2.0 * pow(0.5, j) : 0.0;
        double h = 0.5 * (hi - lo), m = 0.5 * (hi + lo), acc = 0.0;
        for (int i = 0; i < 10; ++i) {
            double t = m + h * or_gl_x[i];
            acc += or_gl_w[i] * (2.0 - t) / (t + b);
        }
        sum += acc * h;
        hi = lo;
    }
    return 0.5 * sum;
}

/* log R for surrogate training samples: one uniform cell per sample with
 * electron density ne, ions of charge Z (A = 1 for Z = 1, 4 for Z = 2) at
 * density ne/Z, temperature T; omega = x T.  Channels: 0 Primakoff
 * (R = Gamma_{gamma->a}/g_agg^2, F by quadrature), 1 Compton-like, 2 e-Z
 * brems, 3 e-e brems (R = Gamma_abs/g_ae^2, eq. gamma_abs, params' eq_stats).
 * The brems targets exclude the cell's screening-fit factor 1 - a eta of
 * eqs. eps_eZ / eps_ee (a = 6.98e-2 e-Z, 0.140 e-e), a per-cell constant
 * that the inference multiplies back: R_c / (1 - a eta).  Where that factor
 * is <= 0 the channel's rate is zero and the sample has no target (NaN).
 * Also returns log(kappa/T).                                               */
void or_surrogate_labels(const or_params* prm, int64_t n, const double* T, const double* ne,
                         const double* Z, const double* x, const int32_t* ch, double* out,
                         double* logkT) {
    or_grid g = {1, {1, 1, 1}, 0.2, 0.1, 1e17};
#pragma omp parallel for if (n > 4096)
    for (int64_t i = 0; i < n; ++i) {
        or_params p = *prm;
        p.g_agg_GeV = 1.0; p.g_ae = 1.0; p.boost = 1.0; p.inverse = 1; p.m_a_keV = 0.0;
        double Zi = Z[i], Ai = (Zi == 1.0) ? 1.0 : 4.0;
        double di = ne[i] / Zi;
        or_cell c;
        double E = x[i] * T[i];
        double R = 0.0;
        if (ch[i] == 0) {
            p.channels = OR_CH_P;
            or_cell_state(&g, &p, 1, &T[i], &ne[i], 1, &di, &Zi, &Ai, &c);
            R = c.G_P0 * or_F_quad(4.0 * E * E / c.kappa2);
        } else if (ch[i] == 1) {
            p.channels = OR_CH_C;
            or_cell_state(&g, &p, 1, &T[i], &ne[i], 1, &di, &Zi, &Ai, &c);
            R = or_gamma_abs(&c, &p, E, NULL);
        } else {
            p.channels = OR_CH_B;
            p.brems_ee = 0;
            or_cell_state(&g, &p, 1, &T[i], &ne[i], 1, &di, &Zi, &Ai, &c);
            double RZ = or_gamma_abs(&c, &p, E, NULL);
            if (ch[i] == 2) R = RZ;
            else {
                or_cell c2;
                p.brems_ee = 1;
                or_cell_state(&g, &p, 1, &T[i], &ne[i], 1, &di, &Zi, &Ai, &c2);
                R = or_gamma_abs(&c2, &p, E, NULL) - RZ;
            }
            double T7 = T[i] * OR_KEV_T7;
            double eta = (3.0 + c.XH) * (c.rho / 100.0) / (T7 * T7);
            double supp = 1.0 - (ch[i] == 2 ? 6.98e-2 : 0.140) * eta;
            R = supp > 0.0 ? R / supp : NAN;
        }
        out[i] = log(R);
        logkT[i] = 0.5 * log(c.kappa2) - log(T[i]);
    }
}
