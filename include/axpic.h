/* axpic.h -- C ABI of the MI355X (gfx950) axion Monte-Carlo operators.
 *
 * Implements the per-macroparticle Monte-Carlo operators of
 *   Radford et al., "An axion framework for Particle-in-Cell codes with
 *   Monte-Carlo sampling: emission, absorption, and detailed balance in
 *   plasmas", arXiv:2604.24627,
 * for one GPU's share of a uniform Cartesian grid.  Section and equation
 * labels in the comments refer to that paper.
 *
 * Conventions
 *  - Every pointer inside the structs and every array argument is a DEVICE
 *    pointer unless marked [host].  The structs themselves live in host memory.
 *  - All calls are asynchronous on `stream` (a hipStream_t passed as void*).
 *    No call allocates or frees memory or synchronises the device; all
 *    scratch space is the caller's `ws` workspace.
 *  - The caller owns every buffer.  Appending calls never write at or beyond
 *    `capacity`: when the products do not fit they write the required length
 *    to status[0], set AXPIC_FLAG_CAPACITY in status[1], modify nothing else,
 *    and the caller may grow the buffer and repeat the call with the same
 *    arguments, which gives bit-identical results (the random numbers are
 *    keyed by (seed, particle id, step), see below).
 *  - Chained calls.  The appending calls, axpic_sort_cells and axpic_feedback
 *    take an optional `chain`, a device int64[AXPIC_CHAIN_N] = {axion count,
 *    photon count, next id, skip flag, axions at the start of the step}.  With
 *    a chain, a call takes its output offset and its first product id from
 *    the chain instead of the species' n and the next_id argument, advances
 *    both on the device, and does nothing (but report AXPIC_FLAG_SKIPPED) once
 *    the skip flag is set; a call that runs out of capacity sets the flag.
 *    axpic_sort_cells writes the number it keeps to the axion count and the
 *    start-of-step word; axpic_absorb acts on the first min(n, start-of-step
 *    word) axions.  A time step can then be issued without reading any count
 *    back: the caller reads the chain once at the end, and after an overflow
 *    grows the buffer named by that call's status and repeats the calls from
 *    it on (the skipped ones modified nothing).
 *  - Particle ids key the random numbers.  A buffer may declare its first
 *    n_implicit ids as id0 + i (plasma in creation order) so that the hot
 *    kernels need not read them; appended products always store theirs.
 *  - Host-side argument errors return AXPIC_E_INVAL before any launch; a
 *    failed launch returns AXPIC_E_DEVICE.  No C++ exception crosses the ABI.
 *
 * Units: positions in cell units (x/dx); momenta in m_e c; the energy of a
 * massless particle is m_e c^2 |p| (Sec. II.B); time step and cell size in
 * the PIC normalisation (1/omega0, c/omega0); weights are RELATIVE: the
 * physical weight is w_ref * w.  Temperatures in keV, densities in cm^-3.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 * (seed lo, seed hi) and counter (id lo, id hi, step, stream<<24 | block).
 * Streams: 0 Primakoff count; 1 thermal counts (words 0-1 Compton, 2-3
 * brems); 2 Compton event k (block k); 3 brems event k; 4 absorption
 * (words 0-1 thermal absorption, 2-3 a->gamma count).  u53 = ((a>>5)*2^26 +
 * (b>>6)) 2^-53; u24 = (2(a>>9)+1) 2^-24.  Counts are drawn by FP64 inversion
 * of the Poisson CDF (eq. poisson_macro); absorption is u53 < P_abs.
 */
#ifndef AXPIC_H
#define AXPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AXPIC_MAX_IONS 4
#define AXPIC_PREF_N 8      /* per-cell prefactors (see axpic_cell_state) */
#define AXPIC_STATE_N 16    /* per-cell FP64 local state */
#define AXPIC_STATUS_N 4    /* int64 status words */

typedef enum {
    AXPIC_OK = 0,
    AXPIC_E_INVAL = -1,
    AXPIC_E_CAPACITY = -2,
    AXPIC_E_DOMAIN = -3,
    AXPIC_E_DEVICE = -4,
    AXPIC_E_UNSUPPORTED = -5,
    AXPIC_E_SCRATCH = -6       /* input larger than an allocation-free call's static scratch */
} axpic_status;

/* status[1] flag bits */
#define AXPIC_FLAG_CAPACITY 1
#define AXPIC_FLAG_SKIPPED 4      /* a chained call after an overflow: nothing done */

/* chain words (see Conventions) */
#define AXPIC_CHAIN_AXIONS 0
#define AXPIC_CHAIN_PHOTONS 1
#define AXPIC_CHAIN_NEXT_ID 2
#define AXPIC_CHAIN_SKIP 3
#define AXPIC_CHAIN_AX_START 4    /* axions present when the step's operators begin */
#define AXPIC_CHAIN_N 5

typedef enum { AXPIC_PRIMAKOFF = 1, AXPIC_COMPTON = 2, AXPIC_BREMS = 4 } axpic_channel;
typedef enum { AXPIC_F32 = 0, AXPIC_F64 = 1 } axpic_dtype;
typedef enum { AXPIC_ELECTRON = 0, AXPIC_ION = 1, AXPIC_PHOTON = 2, AXPIC_AXION = 3 } axpic_kind;

/* Periodic grid of n[0] x n[1] x n[2] cells (unused dimensions have n = 1);
 * cell index = ix + n0 (iy + n1 iz).  Every cell has volume (dx c/omega0)^3. */
typedef struct {
    int32_t ndim;
    int32_t n[3];
    double dx;       /* cell size [c/omega0] */
    double dt;       /* time step [1/omega0]; dt_phys = dt/omega0 (eq. dt_phys) */
    double omega0;   /* normalising frequency [s^-1] */
} axpic_grid;

/* Structure-of-arrays macroparticle buffer.  x[d], p[d], w are `dtype`
 * arrays of length >= capacity; id is uint64, cell int32.  Photon and
 * electron buffers of the plasma are grouped by cell in cell order. */
typedef struct {
    void* x[3];
    void* p[3];
    void* w;
    uint64_t* id;
    int32_t* cell;
    int64_t n;          /* [host] live length */
    int64_t capacity;   /* [host] allocated length */
    int32_t dtype;      /* axpic_dtype */
    int32_t kind;       /* axpic_kind */
    double w_ref;       /* [host] physical weight of w = 1 */
    double Z, A;        /* [host] ion charge state and mass number */
    uint64_t id0;       /* [host] particles i < n_implicit have id id0 + i and their */
    int64_t n_implicit; /*        id[] entries are not read (0: every id is stored) */
    const int64_t* off; /* device, [ncell+1] or NULL: particles i < n_sorted lie in cell */
    int64_t n_sorted;   /* [host] order, cell c holding off[c] <= i < off[c+1] (cell[] stays
                           valid; the Primakoff count reads it only where off is NULL or the
                           cells of a 1024-particle tile are more than 256) */
    void* p2;           /* device, `dtype` [capacity] or NULL: |p|^2 of each particle as
                           axpic_fill_p2 evaluates it from p (a cache for buffers whose
                           momenta do not change).  Given for photons, the massless
                           conversion count reads it instead of p; axpic_absorb writes it
                           for the photons it appends and axpic_compact carries it, when
                           their output has one.  Keeping it equal to p is the caller's. */
} axpic_species;

/* Per-cell tables.  dens: [1+AXPIC_MAX_IONS][ncell] FP64 deposited physical
 * densities (slot 0 electrons, slot 1+s ion species s).  state: [ncell]
 * records of AXPIC_STATE_N doubles: T, n_e, n_e_dep, nZ, nZ2, rho, X_H,
 * kappa^2 [keV^2], G_P0, G_C, G_B [s^-1], Q_C, Q_B [erg cm^-3 s^-1],
 * <E>_C, <E>_B [keV], domain flag (1 when the cell's temperature or a density
 * is negative or not finite: its prefactors are then all 0, so that no event
 * happens there; else 0).  pref32 / pref64: [ncell] records of AXPIC_PREF_N
 * prefactors in FP32 / FP64 (filled by axpic_cell_state). */
typedef struct {
    int64_t ncell;
    double* T_keV;
    double* dens;
    double* state;
    float* pref32;
    double* pref64;
    int32_t nion;                 /* [host] */
    double Zion[AXPIC_MAX_IONS];  /* [host] */
    double Aion[AXPIC_MAX_IONS];  /* [host] */
    double w_ref_e, w_ref_g;      /* [host] reference weights baked into the prefactors;
                                     written by axpic_cell_state */
} axpic_cells;

/* Method parameters [host]; the fields mirror the options the paper names. */
typedef struct {
    double g_agg_GeV;       /* axion-photon coupling [GeV^-1] (Sec. II.C) */
    double g_ae;            /* axion-electron coupling */
    int32_t channels;       /* axpic_channel mask */
    int32_t inverse;        /* 1: inverse operators active (Sec. II.I) */
    double w_a;             /* axion macro-weight (Sec. II.D.1) */
    double wa_mul[3];       /* product base weights / w_a for Primakoff, Compton, brems */
    double w_gamma_prod;    /* physical weight of an a->gamma photon (0: photon w_ref) */
    double lambda_cap;      /* Poisson-mean cap (eq. lambda_eff); bounded by 64 */
    double boost;           /* common multiplier of every rate */
    int32_t eq_stats;       /* 0 Bose-Einstein, 1 Maxwell-Boltzmann equilibrium */
    int32_t kappa_mode;     /* 0 Debye (eq. kappa_debye), 1 fixed */
    double kappa_fixed_keV;
    int32_t prim_targets;   /* 0: sum_i Z_i^2 n_i (ions); 1: plus electrons */
    double prim_inv_ratio;  /* Gamma(a->gamma)/Gamma(gamma->a) */
    int32_t brems_ee;       /* include the e-e term (eq. eps_ee) */
    double brems_k;         /* brems energy sampler: x = E/T ~ Gamma(k, theta) */
    double brems_theta;
    int32_t absorb_mode;    /* 0 Bernoulli deletion, 1 weight reduction */
    int32_t quasi_neutral;  /* n_e from sum Z_i n_i (eq. qn_def) */
    int32_t T_mode;         /* 0 fixed, 1 prescribed field, 2 evolved (Sec. II.J.2) */
    int32_t feedback;       /* apply the affine remap (Sec. II.J.1) */
    double r_relax;         /* eq. Te_relax */
    double T_floor_keV, T_ceil_keV;
    uint64_t seed;
    double hist_lo_keV, hist_hi_keV;
    int32_t hist_nbins;     /* histogram bins (+2 under/overflow slots) per channel, <= 1000 */
    int32_t hist_log;       /* 1: logarithmic bins */
    double m_a_keV;         /* axion mass [keV]; 0: massless.  Sec. II.B gives only the
                               kinematics E = sqrt(p^2 + m^2); with m > 0 the push moves at
                               p/E, photons convert above omega = m with the massive screened
                               kernel and keep their energy, thermal spectra are cut at m and
                               absorption uses the massive equilibrium density (E p instead
                               of E^2).  The rate surrogate is massless only. */
    int32_t light_mode;     /* parents lighter than the product weight w' of their operator
                               (photon->axion: w_a wa_mul[0]; a->gamma: w_gamma_prod).
                               0: such a parent converts whole with probability lambda w'/w
                               (the conversion probability P of Sec. II.F.1), one draw
                               u < lambda w'/w in place of the Poisson count, which keeps the
                               mean converted weight w P; 1: the Poisson count of
                               eq. poisson_macro for them too, the parent converted whole
                               when K w' exceeds its weight (mean transfer w P w/w'). */
} axpic_params;

/* Statistics slots (FP64, accumulated by the calls that own them). */
enum {
    AXPIC_ST_EVENTS_P = 0, AXPIC_ST_EVENTS_C, AXPIC_ST_EVENTS_B,
    AXPIC_ST_NUM_P, AXPIC_ST_NUM_C, AXPIC_ST_NUM_B,
    AXPIC_ST_EN_P, AXPIC_ST_EN_C, AXPIC_ST_EN_B,
    AXPIC_ST_ABS_NUM, AXPIC_ST_ABS_EN, AXPIC_ST_AG_EVENTS, AXPIC_ST_AG_NUM, AXPIC_ST_AG_EN,
    AXPIC_ST_CAPPED, AXPIC_ST_OVERDEPLETED, AXPIC_ST_COLD_CELLS, AXPIC_ST_CLAMPED_CELLS,
    AXPIC_ST_UNAPPLIED_E, AXPIC_ST_ABS_EVENTS,
    AXPIC_ST_COUNT
};

const char* axpic_status_string(int32_t status);
int32_t axpic_version(void);

/* Bytes of workspace the calls below need for parents / axions of up to
 * n_max particles. */
size_t axpic_workspace_bytes(int64_t n_max);

/* axpic_fill_p2 -- sp->p2[i] = |p_i|^2 for from <= i < sp->n, in `dtype`, in the fixed
 * multiply-add order every kernel uses for |p|^2 (so that a rate from the cache equals
 * one from p bit for bit).  AXPIC_E_INVAL without p2 or p, or for from outside [0, n]. */
axpic_status axpic_fill_p2(axpic_species* sp, int64_t from, void* stream);

/* axpic_bin_cells -- Sec. II.B, II.E.  For a species of rest mass m_keV
 * (axions; 0 massless): if `push` != 0 advance x by v dt/dx with
 * v = p / sqrt(|p|^2 + (m/m_e c^2)^2) (= p/|p| when massless; periodic), then
 * recompute `cell` by nearest-grid-point binning of x (always).  Position
 * arithmetic uses only correctly rounded IEEE operations (fma, sqrt, div) in
 * the storage precision.  Returns AXPIC_E_INVAL for a NULL array, a negative
 * mass or a species whose dims exceed the grid. */
axpic_status axpic_bin_cells(const axpic_grid* g, axpic_species* sp, int32_t push, double m_keV,
                             void* stream);

/* axpic_deposit -- Sec. II.E (NGP deposit).  dens[slot][c] = w_ref * sum of
 * w over the particles of cell c / V_cell, for a species grouped by cell
 * with offsets off[ncell+1] (int64).  Deterministic (sequential per cell). */
axpic_status axpic_deposit(const axpic_grid* g, const axpic_species* sp, const int64_t* off,
                           axpic_cells* cells, int32_t slot, void* stream);

/* axpic_cell_state -- Sec. II.E-II.I.  From dens and T_keV computes the FP64
 * local state (eqs. rho_def, qn_def, kappa_debye, prim_xs, prim_rate, epsC,
 * QC, GammaC, eps_eZ, eps_ee) and the per-cell prefactors, in pref32 and
 * pref64: [0] T, [1] 4 (m_e c^2)^2/kappa^2, [2] G_P0 dt_phys,
 * [3] G_P0 dt_phys w_ref_g/(w_a wa_mul[0]), [4] w_ref_e G_C dt_phys/(w_a wa_mul[1]),
 * [5] w_ref_e G_B dt_phys/(w_a wa_mul[2]), [6] Compton absorption coefficient,
 * [7] brems absorption coefficient (eq. gamma_abs times dt_phys).
 * w_ref_e / w_ref_g: reference weights of the emitting electrons / photons. */
axpic_status axpic_cell_state(const axpic_grid* g, axpic_cells* cells, const axpic_params* prm,
                              double w_ref_e, double w_ref_g, void* stream);

/* axpic_rates -- per-particle rate materialisation (FP32 for f32 species,
 * FP64 for f64), written to out[n] of the species' dtype:
 *   photons,   AXPIC_PRIMAKOFF: lambda_P = w P_{gamma->a}/w_a (Sec. II.F.1, eq. prim_prob)
 *   electrons, AXPIC_COMPTON / AXPIC_BREMS: lambda_macro (eq. lambda_macro)
 *   axions,    AXPIC_COMPTON|AXPIC_BREMS: P_abs = 1 - exp(-Gamma_abs dt_phys) (eq. gamma_abs)
 *   axions,    AXPIC_PRIMAKOFF: a->gamma mean lambda (before the thermal absorption)
 * These are exactly the values the fused sampling calls compute internally. */
axpic_status axpic_rates(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                         const axpic_species* sp, int32_t channel, void* out, void* stream);

/* axpic_sample_emit -- Secs. II.D, II.F.1, II.G, II.H.  Forward operators on
 * the first parent->n particles of `parent`:
 *   photons (AXPIC_PRIMAKOFF): K ~ Poisson(min(lambda_P, cap)) conversions,
 *     each product inherits x and p, parent weight depleted by K w_a';
 *   electrons (AXPIC_COMPTON and/or AXPIC_BREMS): K per channel, each event
 *     an axion at the emitter's position with E = T x, x from the channel's
 *     number spectrum (Compton x^4/(e^x-1); brems Gamma(k, theta)) and an
 *     isotropic direction; fb[cell] -= (w E, w p).
 * Products are appended to `axions` at axions->n .. in the canonical order
 * (parent index, channel, event k) with ids (next_id + rank) | 2^63.
 * lam_in: NULL (fused rates) or the per-parent means (photons: [n];
 * electrons: [2][n] Compton then brems) in the parent's dtype.
 * hist: [3][nbins+2] FP64 power histogram (w_phys E [keV]) or NULL;
 * fb: [ncell][4] FP64 (dE [m_e c^2], dP [m_e c]) or NULL; stats:
 * [AXPIC_ST_COUNT] or NULL; status: int64[AXPIC_STATUS_N] (status[2] =
 * products written).  On return axions->n is NOT updated (the count is on
 * the device); the caller reads status[2]. */
axpic_status axpic_sample_emit(const axpic_grid* g, const axpic_cells* cells,
                               const axpic_params* prm, axpic_species* parent, int32_t channels,
                               const void* lam_in, int64_t step, uint64_t next_id,
                               axpic_species* axions, double* fb, double* hist, double* stats,
                               int64_t* status, void* ws, size_t ws_bytes, int64_t* chain, void* stream);

/* axpic_cell_weights -- for the superposed emission below: out[c] = sum of
 * the relative weights of electrons off[c] .. off[c+1]-1 (FP64, a fixed
 * reduction order), out[ncell + c] = the largest of them.  The electrons must
 * be grouped by cell; electron weights do not change during a run (the
 * feedback remaps momenta), so the result can be kept. */
axpic_status axpic_cell_weights(const axpic_species* electrons, const int64_t* off, int64_t ncell,
                                double* out, void* stream);

/* axpic_sample_emit_cells -- thermal emission (Secs. II.D, II.G, II.H) by
 * per-cell superposition: in cell c the electrons' independent counts
 * K_e ~ Poisson(lambda_e), lambda_e = w_e coef_ch (eq. lambda_macro), are
 * drawn as the cell total N ~ Poisson(Lambda), Lambda = sum_e lambda_e,
 * each event assigned to electron e with probability lambda_e / Lambda (the
 * same joint law: a sum of independent Poisson counts is Poisson and its
 * split is multinomial).  Electrons at the cap enter with min(lambda_e, cap)
 * and carry lambda_e / cap in the product weight (eqs. lambda_eff,
 * wa_rescaled).  The work is per cell and per event, not per electron.
 * Electrons are grouped by cell (off[ncell+1], int64, device); cellw from
 * axpic_cell_weights.  Lambda = coef W when no electron of the cell reaches
 * the cap, else the sum of min(w_e coef, cap) in index order; a mean above
 * 500 is drawn as ceil(Lambda/500) equal parts.  Random numbers: the cell
 * totals from stream 5 keyed by the cell index (block = part); event j of
 * channel ch: the electron from stream 6 (block (ch-1) 2^23 + j, inverse CDF
 * over the cell in index order), energy and direction from stream 6 + ch
 * (block j).  Products are appended in the order (cell, channel, j) with
 * ids (next_id + rank) | 2^63; everything else as axpic_sample_emit.  The
 * workspace must hold axpic_workspace_bytes(4 ncell). */
axpic_status axpic_sample_emit_cells(const axpic_grid* g, const axpic_cells* cells,
                                     const axpic_params* prm, axpic_species* electrons,
                                     const int64_t* off, const double* cellw, int32_t channels,
                                     int64_t step, uint64_t next_id, axpic_species* axions,
                                     double* fb, double* hist, double* stats, int64_t* status,
                                     void* ws, size_t ws_bytes, int64_t* chain, void* stream);

/* axpic_absorb -- Sec. II.I and the inverse of Sec. II.F.1.  On the first
 * axions->n axions (with a chain: the first min(axions->n,
 * chain[AXPIC_CHAIN_AX_START])): thermal absorption (delete with probability P_abs or
 * reduce the weight by it; fb[cell] += (w E, w p)), then a->gamma conversion
 * of what survives (products appended to `photons` with ids as above).
 * pabs_in / lam_in optionally replace the computed P_abs / a->gamma means, both
 * of the axions as they are at the start of the step (what axpic_rates writes).
 * With weight reduction (absorb_mode 1) an axion converts with the mean of its
 * reduced weight, i.e. the start-of-step mean times (1 - P_abs) (eq. prim_prob:
 * the mean is proportional to the parent's weight), taken in FP64 whether the
 * mean is computed or handed in.  The exchange is summed without atomics, in a fixed
 * order, when the axions are in cell order (off set, n_sorted >= n). */
axpic_status axpic_absorb(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                          axpic_species* axions, const void* pabs_in, const void* lam_in,
                          int64_t step, uint64_t next_id, axpic_species* photons, double* fb,
                          double* stats, int64_t* status, void* ws, size_t ws_bytes,
                          int64_t* chain, void* stream);

/* axpic_feedback -- Sec. II.J.  Per cell over the electrons (grouped by cell,
 * offsets off[ncell+1]): FP64 moments W, P, U2 (eq. cell_moments), the
 * affine remap p' = S p + b (eqs. delta_def .. b_def, applied when
 * prm->feedback) and the temperature update (eqs. Te_est, Te_relax, clamp)
 * when prm->T_mode == 2.  moments: [ncell][5] FP64 output (before the remap)
 * or NULL.  stats (or NULL): the cold cells, the clamped cells and the energy
 * they could not take (O10) are added in a fixed order through `ws`, which must
 * then hold axpic_workspace_bytes(2 ncell) bytes (else NULL). */
axpic_status axpic_feedback(const axpic_grid* g, axpic_cells* cells, const axpic_params* prm,
                            axpic_species* electrons, const int64_t* off, const double* fb,
                            double* moments, double* stats, void* ws, size_t ws_bytes,
                            int64_t* chain, void* stream);

/* axpic_sort_cells -- the canonical buffer order (Sec. II.E: the operators are local to
 * a cell; the order within a buffer is this library's convention): a stable counting
 * sort of `in` by cell -- the particles of each cell in their order in `in` -- with the
 * particles of zero weight dropped (and any whose cell is not on the grid), written to
 * `out` (distinct arrays, same dtype, out->capacity >= the number kept; ids written
 * explicitly).  off (device int64[ncell + 1], may be NULL) receives the cell offsets of
 * `out`; status[2] the number kept.  When it does not fit, status[0] holds the length
 * needed, status[1] AXPIC_FLAG_CAPACITY, and nothing else is written.
 *
 * path selects how the per-cell counts and places are taken (the result is the same):
 * AXPIC_SORT_SPARSE one atomic per run of equal cells in a wavefront, AXPIC_SORT_DENSE
 * one per cell and block of 1024 particles, AXPIC_SORT_AUTO the second from 32
 * particles per cell on.  AXPIC_E_INVAL for another value.
 *
 * With chain (may be NULL), the number kept also goes to chain[AXPIC_CHAIN_AXIONS] and
 * chain[AXPIC_CHAIN_AX_START], and a set skip flag makes the call do nothing.
 *
 * Deterministic: the placement does not depend on the order of the device's atomics.
 * ws: at least axpic_sort_ws_bytes(g, in->n) bytes; in->n < 2^32. */
#define AXPIC_SORT_AUTO 0
#define AXPIC_SORT_SPARSE 1
#define AXPIC_SORT_DENSE 2
size_t axpic_sort_ws_bytes(const axpic_grid* g, int64_t n);
axpic_status axpic_sort_cells(const axpic_grid* g, const axpic_species* in, int32_t path,
                              axpic_species* out, int64_t* off, int64_t* status, void* ws,
                              size_t ws_bytes, int64_t* chain, void* stream);

/* axpic_compact -- stable removal of particles with w <= 0 from `in` into
 * `out` (distinct buffers, same dtype, out->capacity >= in->n).  status[2]
 * receives the surviving count. */
axpic_status axpic_compact(const axpic_species* in, axpic_species* out, int64_t* status,
                           void* ws, size_t ws_bytes, void* stream);

/* axpic_diag -- Sec. III.E: out[0] = N_a = sum w_ref w, out[1] = U_a =
 * sum w_ref w E [keV] over the species (FP64, deterministic order), with
 * E = sqrt(m_e^2 |p|^2 + m^2) for particles of rest mass m_keV (0: massless). */
axpic_status axpic_diag(const axpic_species* sp, double m_keV, double* out, void* ws,
                        size_t ws_bytes, void* stream);

/* axpic_diag_noalloc -- axpic_diag without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and the same result, bit for bit, with the
 * per-block partial sums in a static device array of the library (4 MiB per GPU, held
 * until the process ends).  It allocates and frees nothing.  Limit: at most 2^28
 * particles (262144 blocks of 1024); a larger species returns AXPIC_E_SCRATCH before
 * any launch.  The array is shared by every call on that GPU and keeps the last call's
 * partials: calls that overlap on one GPU (on different streams) race and must be
 * ordered by the caller.  The first call on a device looks up the array's address on
 * that device. */
axpic_status axpic_diag_noalloc(const axpic_species* sp, double m_keV, double* out, void* stream);

/* axpic_equilibrium -- the FP64 equilibrium check of the thermal inverse operators
 * (Sec. II.I, eq. gamma_abs: the net source vanishes energy bin by energy bin at
 * n_eq; the relaxation plateau of Sec. III.E).  On the histogram grid of prm (nbins
 * bins, then [0, lo) and [hi, inf) as the power histograms number them) writes
 * out[AXPIC_EQ_FIELDS][nbins + 2] (device, FP64):
 *   NUM   sum of w_ref w over the particles of sp in the bin (w > 0)
 *   EN    sum of w_ref w E [keV]  (E = sqrt(m_e^2 |p|^2 + m^2), m = prm->m_a_keV)
 *   W2    sum of (w_ref w)^2
 *   NEQ   sum over cells of V_cell int_bin dn_eq/dE dE: the equilibrium number of one
 *         axion state at the cell's temperature, BE or MB (prm->eq_stats); with mass,
 *         dn_eq/dE = E p f(E/T) / (2 pi^2 (hbar c)^3), zero below m
 *   UEQ   the same with E dn_eq/dE
 *   NFIX  sum over cells of V_cell int_bin dn_eq/dE q(g) (1 - e^{-t g}) dE, with
 *         g(E) = Gamma_abs(E) dt_phys of the thermal channels whose absorption
 *         coefficients axpic_cell_state wrote into cells->pref64 and
 *         q(g) = g / (1 - e^{-g}): the expected content after t = t_steps steps of
 *         the recursion n_{t+1} = n_t e^{-g} + n_eq g of operators that each act on
 *         the start-of-step population, started empty; t_steps <= 0 gives its fixed
 *         point n_eq q(g), which tends to n_eq as g -> 0
 *   Z     (NUM - NFIX) / sqrt(W2), 0 where W2 = 0.
 * Every sum is taken in an order fixed by the data (segments of 4096 particles, chunks
 * of 256 cells, then the partials in order), so the result does not depend on launch
 * geometry or scheduling.  Bin integrals: 8-point Gauss-Legendre on panels no wider
 * than T/16 (the overflow bin cut at hi + 64 T, the underflow bin on geometric panels;
 * with mass, the part just above m in sqrt(E - m) on geometric panels).
 * ws: at least axpic_equilibrium_ws_bytes(sp->n, ncell, nbins) bytes of device memory.
 * AXPIC_E_INVAL for missing arrays, a grid/cell mismatch or a short workspace. */
#define AXPIC_EQ_FIELDS 7
enum { AXPIC_EQ_NUM = 0, AXPIC_EQ_EN, AXPIC_EQ_W2, AXPIC_EQ_NEQ, AXPIC_EQ_UEQ, AXPIC_EQ_NFIX,
       AXPIC_EQ_Z };
size_t axpic_equilibrium_ws_bytes(int64_t n, int64_t ncell, int32_t nbins);
axpic_status axpic_equilibrium(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                               const axpic_species* sp, double t_steps, double* out, void* ws,
                               size_t ws_bytes, void* stream);

/* axpic_sampler_table -- host-only access to the thermal energy samplers'
 * quantile tables (no device work).  which = 0: Compton-like number spectrum
 * x^4/(e^x-1) (Sec. II.G); which = 1: Gamma(k, 1) (Sec. II.H).  out receives
 * 2*(2048+1) doubles: y = ln x at z_j = -18 + 36 j/2048 (z = ln(u/(1-u))),
 * then dy/dz at the same nodes. */
axpic_status axpic_sampler_table(int32_t which, double k, double* out);

/* axpic_stream_copy -- plain device copy of `bytes` (a multiple of 16, both
 * pointers 16-byte aligned): the calibration kernel for achievable HBM
 * bandwidth and for scaling the profiler's byte counters. */
axpic_status axpic_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Rate surrogate (learned rate backend).  A perceptron 8 -> 128 x4 -> 1 with
 * hard-swish activations h(z) = z clamp(z/6 + 1/2, 0, 1), bfloat16 weights
 * and FP32 accumulation on the matrix cores predicts the residual y of
 *   log R = mu_ch + sum_i lin_ch[i] f_i + sigma_ch y
 * from the features x = (log(omega/T), log(kappa/T), log n_e, Z), normalised
 * as f_i = (x_i - feat_lo_i) feat_sc_i - 1, plus a one-hot channel (Primakoff,
 * Compton-like, e-Z brems, e-e brems); R = Gamma/g^2 of the Primakoff
 * conversion (Sec. II.F) or of the detailed-balance absorption (eq.
 * gamma_abs) of the channel, the brems channels without the cell's
 * screening-fit factor of eqs. eps_eZ / eps_ee, which the rate kernel applies.
 * Outside the training box the plain rate is used for that particle.
 * FP32 master parameters (padded training layout, AXPIC_MLP_PARAMS floats):
 * W1 [32][128], b1 [128], W2, b2, W3, b3, W4, b4 ([128][128], [128]),
 * W5 [128][32], b5 [32]; only inputs 0..7 and output 0 are live.
 */
#define AXPIC_MLP_PARAMS 57888
#define AXPIC_MLP_BLOB_BYTES 112704

typedef struct {
    const void* blob;                 /* device: axpic_mlp_pack output */
    float feat_lo[4], feat_sc[4];     /* [host] feature normalisation */
    float out_mu[4], out_sigma[4];    /* [host] per-channel log-rate de-normalisation */
    float out_lin[4][4];              /* [host] per-channel linear term in the normalised features */
    double T_lo, T_hi, ne_lo, ne_hi, x_lo, x_hi;   /* [host] training box (keV, cm^-3, omega/T) */
} axpic_mlp;

/* Normalisation of a training set: f_i = (x_i - lo_i) sc_i - 1 maps the valid
 * rows' range of feature i onto [-1, 1] (Z: [1, 2]); per channel c the
 * least-squares affine fit log R ~ mu_c + lin_c . f over the valid rows of c and
 * the standard deviation sigma_c of its residual (at least 1e-3).  A row is
 * valid when its log R is finite. */
typedef struct {
    double lo[4], sc[4];
    double mu[4], lin[4][4], sigma[4];
    int64_t count[4];              /* valid rows per channel */
} axpic_mlp_norm;

/* Device workspace of axpic_mlp_prepare. */
size_t axpic_mlp_prepare_ws_bytes(void);
/* axpic_mlp_prepare -- fills *norm [host] from feat [n][4], logR [n] and ch [n]
 * (device; the output of axpic_surrogate_samples): FP64 reductions on the GPU in a
 * fixed order, the 5 x 5 normal equations solved on the host.  Synchronises
 * `stream`.  AXPIC_E_DOMAIN if a feature range is empty or a channel has too few
 * valid rows for the fit. */
axpic_status axpic_mlp_prepare(const double* feat, const double* logR, const int32_t* ch, int64_t n,
                               void* ws, size_t ws_bytes, axpic_mlp_norm* norm, void* stream);
/* axpic_mlp_design -- training rows X [n][32] (16-byte aligned) = normalised
 * features, channel one-hot, zeros; Y [n] = (log R - mu_c - lin_c . f) / sigma_c,
 * NaN for an invalid row (the loss skips it). */
axpic_status axpic_mlp_design(const double* feat, const double* logR, const int32_t* ch, int64_t n,
                              const axpic_mlp_norm* norm, float* X, float* Y, void* stream);
/* axpic_mlp_batch -- minibatch Xb [batch][32], Yb [batch] of rows drawn with
 * replacement from X [n][32] (n < 2^32): row floor(u n / 2^32), u the first word
 * of Philox4x32-10 at counter (b, step, 0x4D4C5042, 0) under key seed. */
axpic_status axpic_mlp_batch(const float* X, const float* Y, int64_t n, int64_t batch, uint64_t seed,
                             int64_t step, float* Xb, float* Yb, void* stream);

/* Training samples generated by the plain rates (FP64, device arrays of n):
 * for each (T [keV], n_e [cm^-3], Z, x = omega/T, channel) writes the raw
 * features feat[4i..4i+3] = (log x, log(kappa/T), log n_e, Z) and log R. */
axpic_status axpic_surrogate_samples(const axpic_params* prm, int64_t n, const double* T,
                                     const double* ne, const double* Z, const double* x,
                                     const int32_t* ch, double* feat, double* logR, void* stream);
/* Bytes of the packed inference blob (bf16 MFMA fragments + FP32 biases). */
size_t axpic_mlp_blob_bytes(void);
/* Workspace of the training calls for a batch (a multiple of 32). */
size_t axpic_mlp_train_ws_bytes(int64_t batch);
/* Pack FP32 master parameters into the inference blob (rounding to bf16). */
axpic_status axpic_mlp_pack(const float* master, void* blob, void* stream);
/* Arithmetic of the training calls: AXPIC_MLP_BF16 rounds every matrix-product operand
 * (weights, layer inputs, back-propagated gradients) to bfloat16 and accumulates in FP32
 * on the matrix cores (the training mode); AXPIC_MLP_F32 keeps FP32 throughout (the
 * mode in which gradients are checked at FP32 accuracy). */
#define AXPIC_MLP_BF16 0
#define AXPIC_MLP_F32 1
/* Training forward pass: X [batch][32] (features in columns 0..7, zeros after),
 * y [batch] (may be NULL); activations are kept in ws for axpic_mlp_loss_grad. */
axpic_status axpic_mlp_forward(const float* master, const float* X, int64_t batch, int32_t precision,
                               void* ws, size_t ws_bytes, float* y, void* stream);
/* Mean squared error of y against Y and its gradient (AXPIC_MLP_PARAMS floats);
 * rows whose target is NaN contribute neither (the mean still divides by batch). */
axpic_status axpic_mlp_loss_grad(const float* master, const float* X, const float* Y, int64_t batch,
                                 int32_t precision, void* ws, size_t ws_bytes, float* grad,
                                 double* loss, void* stream);
/* Adam step on the FP32 master parameters (step counts from 1). */
axpic_status axpic_mlp_adam(float* master, const float* grad, float* m, float* v, int64_t step,
                            float lr, float beta1, float beta2, float eps, void* stream);
/* Surrogate rates, written like axpic_rates: photons + AXPIC_PRIMAKOFF ->
 * lambda_P; axions + (AXPIC_COMPTON|AXPIC_BREMS) -> thermal P_abs; axions +
 * AXPIC_PRIMAKOFF -> a->gamma mean.  n_fallback (device, may be NULL) counts
 * the particles evaluated by the plain rate because they lie outside the box. */
axpic_status axpic_rates_mlp(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                             const axpic_species* sp, int32_t channel, const axpic_mlp* net,
                             void* out, unsigned long long* n_fallback, void* stream);

/* ---------------------------------------------------------------------------
 * Per-cell surrogate tables.  Of the surrogate's inputs only omega varies
 * inside a cell (T, kappa, n_e and Z are the cell's, Sec. II.E), so the
 * network can be evaluated once per cell on a grid of u = ln(omega/T) and the
 * per-particle rate interpolated: the matrix-core work then scales with
 * cells x nodes instead of particles.
 * Grid: u_j = ln x_lo + j h, h = (ln x_hi - ln x_lo)/(nodes - 1), j = 0 .. nodes-1,
 * 4 <= nodes <= AXPIC_TAB_MAX_NODES.  Table (device, FP32, caller-owned):
 * table[(2 c + s) nodes + j] for cell c, slot s:
 *   s = 0  log R of the Primakoff conversion (R = Gamma_{gamma->a}/g_agg^2);
 *   s = 1  log of the sum over the thermal channels enabled in prm (Compton-like,
 *          e-Z brems, e-e brems if brems_ee) of the absorption rate per g_ae^2
 *          (eq. gamma_abs), brems times the cell's screening-fit factor
 *          max(0, 1 - a eta) of eqs. eps_eZ / eps_ee; -inf when that sum is 0.
 * A cell outside the training box (T, n_e, or not one ion species of Z 1 or 2)
 * gets NaN in every entry of the slots written.
 */
#define AXPIC_TAB_MAX_NODES 64

/* axpic_mlp_table -- fill slot 0 if channel has AXPIC_PRIMAKOFF, slot 1 if it
 * has AXPIC_COMPTON or AXPIC_BREMS, for every cell, from the network `net` on
 * the grid over [x_lo, x_hi], which must lie inside the training range
 * [net->x_lo, net->x_hi] (particles outside it take the plain rate).
 * AXPIC_E_INVAL for a missing pointer, nodes or range out of bounds, or no slot
 * requested. */
axpic_status axpic_mlp_table(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                             int32_t channel, const axpic_mlp* net, int32_t nodes, double x_lo,
                             double x_hi, float* table, void* stream);

/* axpic_rates_table -- per-particle rates from a table (any source, laid out as
 * above on the grid of nodes over [x_lo, x_hi]); outputs and (species, channel)
 * pairs as axpic_rates_mlp.  With t = (ln(omega/T) - ln x_lo)/h and
 * k = clamp(floor(t) - 1, 0, nodes - 4), log R is the cubic through nodes
 * k .. k+3 (Lagrange form, FP64) at t; then Gamma = g^2 boost R and the rate
 * follows as in axpic_rates (eq. lambda_macro for lambda, 1 - exp(-Gamma dt)).
 * Particles with omega/T outside [x_lo, x_hi] or in a NaN cell take the plain
 * rate and are counted in n_fallback (device, may be NULL).  The slot read
 * (0 for AXPIC_PRIMAKOFF, 1 for thermal absorption) must have been filled. */
axpic_status axpic_rates_table(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                               const axpic_species* sp, int32_t channel, int32_t nodes, double x_lo,
                               double x_hi, const float* table, void* out,
                               unsigned long long* n_fallback, void* stream);

/* axpic_timing_enable / axpic_timing_read -- instrumentation.  While enabled,
 * every kernel the library launches is bracketed by HIP events recorded on
 * its own stream.  axpic_timing_read waits for those events and writes one
 * line "kernel_name launches total_ms" per kernel into buf (NUL-terminated),
 * then resets the counters; AXPIC_E_CAPACITY if buf was too short.
 * axpic_timing_only: time only the launches of the kernel so named (NULL: all),
 * so that the others run without events between them. */
void axpic_timing_enable(int32_t on);
void axpic_timing_only(const char* name);
axpic_status axpic_timing_read(char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif
