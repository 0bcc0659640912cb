/* axpic_oracle.h -- FP64 CPU oracle of the axion Monte-Carlo operators.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the HIP
 * path is checked against.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or constant generator with the HIP path.
 *
 * Units: momenta in m_e c, energies of massless particles E = m_e c^2 |p|
 * (axions of mass m: E = sqrt(m_e^2 c^4 |p|^2 + m^2 c^4)),
 * positions in cell units, weights are PHYSICAL particle counts, temperatures
 * in keV, densities in cm^-3, rates in s^-1.
 */
#ifndef AXPIC_ORACLE_H
#define AXPIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_CH_P = 1, OR_CH_C = 2, OR_CH_B = 4 };

typedef struct {
    int32_t ndim;
    int32_t n[3];
    double dx;       /* cell size, c/omega0 */
    double dt;       /* step, 1/omega0 */
    double omega0;   /* s^-1 */
} or_grid;

typedef struct {
    double g_agg_GeV, g_ae;
    int32_t channels, inverse;
    double w_a;
    double wa_mul[3];
    double w_gamma_prod;      /* physical weight of a photon made by a->gamma */
    double lambda_cap, boost;
    int32_t eq_stats, kappa_mode;
    double kappa_fixed_keV;
    int32_t prim_targets;
    double prim_inv_ratio;
    int32_t brems_ee;
    double brems_k, brems_theta;
    int32_t absorb_mode, quasi_neutral, T_mode, feedback;
    double r_relax, T_floor_keV, T_ceil_keV;
    uint64_t seed;
    double hist_lo_keV, hist_hi_keV;
    int32_t hist_nbins, hist_log;
    double m_a_keV;           /* axion mass; 0: massless */
    int32_t light_mode;       /* 0: light parents convert whole with probability P; 1: Poisson */
} or_params;

typedef struct {
    double *x[3], *p[3], *w;
    uint64_t *id;
    int32_t *cell;
    int64_t n;
} or_species;

/* Output buffer for products (appended at 0..cap-1). */
typedef struct {
    double *x[3], *p[3], *w;
    uint64_t *id;
    int32_t *cell;
    int64_t *parent;   /* index of the parent in its buffer */
    int32_t *chan;     /* 0 Primakoff, 1 Compton, 2 brems, 3 a->gamma */
    int64_t cap;
} or_products;

typedef struct {
    double T, n_e, n_e_dep, nZ, nZ2, rho, XH, kappa2;
    double G_P0;             /* Gamma_{gamma->a}(omega) = G_P0 * F(4 omega^2/kappa^2) [s^-1] */
    double G_C, G_B;         /* per-electron production rates [s^-1] */
    double Q_C, Q_B;         /* emissivities [erg cm^-3 s^-1] */
    double meanE_C, meanE_B; /* keV */
} or_cell;

/* statistics slots (FP64, accumulated) */
enum {
    OR_ST_EVENTS_P = 0, OR_ST_EVENTS_C, OR_ST_EVENTS_B,
    OR_ST_NUM_P, OR_ST_NUM_C, OR_ST_NUM_B,
    OR_ST_EN_P, OR_ST_EN_C, OR_ST_EN_B,
    OR_ST_ABS_NUM, OR_ST_ABS_EN, OR_ST_AG_EVENTS, OR_ST_AG_NUM, OR_ST_AG_EN,
    OR_ST_CAPPED, OR_ST_OVERDEPLETED, OR_ST_COLD_CELLS, OR_ST_CLAMPED_CELLS,
    OR_ST_UNAPPLIED_E, OR_ST_ABS_EVENTS,
    OR_ST_COUNT
};

/* ---- constants ---- */
double or_const(int which);
int32_t or_num_threads(void);
void or_set_num_threads(int32_t n);

/* ---- RNG ---- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_draw(uint64_t seed, uint64_t id, uint32_t step, uint32_t stream, uint32_t block,
             uint32_t out[4]);
double or_u53(uint32_t a, uint32_t b);
double or_u24(uint32_t a);
int32_t or_poisson(double lam, double u);
void or_poisson_batch(const double* lam, const double* u, int32_t* k, int64_t n);

/* ---- rate building blocks ---- */
double or_F(double s);
void or_cell_state(const or_grid* g, const or_params* prm, int64_t ncell, const double* T,
                   const double* dens_e, int32_t nion, const double* dens_ion /* [nion][ncell] */,
                   const double* Zion, const double* Aion, or_cell* out);
double or_gamma_prim(const or_cell* c, const or_params* prm, double omega_keV);
/* Finite-mass axions (prm->m_a_keV > 0). */
double or_F_mass(double k, double p, double kappa2);
double or_F_mass_quad(double k, double p, double kappa2);
double or_gamma_conv(const or_cell* c, const or_params* prm, double omega_keV);
double or_axion_energy(const or_params* prm, double p2);
double or_compton_x_above(double xm, double u);
double or_compton_x_tail(double q);
double or_gamma_x_tail(double k, double q);
double or_gamma_x_above(double k, double ym, double u);
double or_gamma_abs(const or_cell* c, const or_params* prm, double E_keV, double* parts);
double or_dt_phys(const or_grid* g);
double or_V_cell(const or_grid* g);

/* ---- samplers (exact inverse CDFs) ---- */
double or_compton_cdf(double X);
double or_compton_ccdf(double X);
double or_compton_x(double u);
double or_gammainc_P(double a, double y);
double or_gammainc_Q(double a, double y);
double or_gamma_x(double k, double u);

/* ---- diagnostics ---- */
int32_t or_hist_bin(const or_params* prm, double E_keV);
void or_equilibrium(const or_grid* g, const or_params* prm, const or_cell* cells, int64_t ncell,
                    const or_species* s, double t_steps, double* out /* [7][nbins+2] */);

/* ---- operators ---- */
void or_deposit(const or_species* s, int64_t ncell, double V, double* dens);
int64_t or_emit_primakoff(const or_grid* g, const or_params* prm, const or_cell* cells,
                          or_species* ph, const double* lam_in, int64_t step,
                          uint64_t next_id, or_products* out, double* hist, double* stats,
                          double* lam_out, int32_t* K_out);
int64_t or_emit_thermal_cells(const or_grid* g, const or_params* prm, const or_cell* cells,
                              const or_species* el, const int64_t* off, int64_t ncell,
                              const double* coef_in, const double* W_in, int64_t step,
                              uint64_t next_id, or_products* out, double* fb, double* hist,
                              double* stats, double* Lambda_out, int32_t* N_out);
int64_t or_emit_thermal(const or_grid* g, const or_params* prm, const or_cell* cells,
                        const or_species* el, const double* lam_in, int64_t step,
                        uint64_t next_id, or_products* out, double* fb, double* hist,
                        double* stats, double* lam_out, int32_t* K_out);
int64_t or_absorb(const or_grid* g, const or_params* prm, const or_cell* cells,
                  or_species* ax, const double* pabs_in, const double* lam_in, int64_t step,
                  uint64_t next_id, or_products* out, double* fb, double* stats,
                  double* pabs_out, double* lam_out, int32_t* K_out, int32_t* absorbed_out);
void or_feedback(const or_grid* g, const or_params* prm, int64_t ncell, const int64_t* off,
                 or_species* el, const double* fb, double* T, double* stats,
                 double* moments_out);
void or_push(const or_grid* g, or_species* ax, int32_t prec32, double m_a_keV);
int64_t or_sort_cells(or_species* s, int64_t ncell, int64_t* off);

/* ---- surrogate training data ---- */
double or_F_quad(double s);
void or_surrogate_labels(const or_params* prm, int64_t n, const double* T, const double* ne,
                         const double* Z, const double* x, const int32_t* ch, double* out,
                         double* logkT);

#ifdef __cplusplus
}
#endif
#endif
