// axpic_device.hpp -- device building blocks of the axion Monte-Carlo operators
// (gfx950).  Counter-based random numbers, Poisson inversion, the screened
// Primakoff kernel, quantile-table energy samplers and small reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/axpic.h"

namespace axpic {

// Physical constants (CODATA 2018; cgs / keV).
constexpr double kPi = 3.14159265358979323846;
constexpr double kAlpha = 1.0 / 137.035999084;
constexpr double kHbarcGeVcm = 1.973269804e-14;
constexpr double kHbarcKeVcm = 1.973269804e-8;
constexpr double kC = 2.99792458e10;
constexpr double kMe = 510.99895000;          // m_e c^2 [keV]
constexpr double kKeVerg = 1.602176634e-9;
constexpr double kKeVT7 = 1.160451812;        // T_7 per keV
constexpr double kMu = 1.66053906660e-24;     // atomic mass unit [g]
constexpr double kZeta5 = 1.0369277551433699263;
constexpr double kZeta6 = 1.0173430619844491397;
constexpr double kLambdaHardCap = 64.0;       // bound of the inversion sampler
constexpr int kKmax = 255;

constexpr int kTabN = 3072;                   // quantile-table intervals (h = 9/512)
constexpr double kTabZ0 = -18.0, kTabZ1 = 36.0;   // z = ln(u/(1-u)); the upper half serves cut spectra

// Kernel-side parameter block (derived on the host from axpic_params).
struct KParams {
    double dt_phys;
    double w_a;
    double wa_mul[3];
    double w_gamma_prod;        // physical
    double cap;                 // min(lambda_cap, 64)
    double ag_unit;             // inv_ratio * w_a^2 * wa_mul0 / (w_ref_g * w_gamma_prod)
    double inv_ratio;
    double brems_k, brems_theta;
    double brems_km3, brems_c1;  // k - 3 and 1 - 1/theta of the brems absorption shape
    double hist_lo, hist_scale; // bin = floor(scale * log(E/lo)) or floor(scale * (E - lo))
    double r_relax, T_floor, T_ceil;
    double dtdx;
    uint32_t seed_lo, seed_hi;
    int32_t channels, inverse, absorb_mode, eq_stats, T_mode, feedback;
    int32_t nbins, hist_log;
    int32_t ndim;
    int32_t n[3];
    double m_a;                 // axion mass [keV] (0: massless)
    double mu2;                 // (m_a / m_e c^2)^2
    int32_t massive;
    int32_t light_mode;         // 0: a parent lighter than one product converts whole w.p. P
};

// ---------------------------------------------------------------- Philox4x32-10
// a ^ b ^ c in one instruction (gfx950 v_bitop3_b32; 0x96 is the truth table of XOR3)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        // full 64-bit products: one v_mad_u64_u32 each instead of a mul_lo/mul_hi pair
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                       xor3((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
    }
    return c;
}

__device__ __forceinline__ uint4 draw(const KParams& kp, uint64_t id, int64_t step,
                                      uint32_t stream, uint32_t block) {
    uint4 c = make_uint4((uint32_t)id, (uint32_t)(id >> 32), (uint32_t)step,
                         (stream << 24) | (block & 0xFFFFFFu));
    return philox4x32_10(c, kp.seed_lo, kp.seed_hi);
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}
__device__ __forceinline__ double u24(uint32_t a) {
    return (double)(2u * (a >> 9) + 1u) * (1.0 / 16777216.0);
}

// Poisson(lam) by sequential CDF inversion in FP64 (fixed operation order).
// The leading test is an exact shortcut: exp(-lam) >= 1 - lam, and the FP64
// exponential is within one ulp, so u < fl(1 - lam) - 2^-50 implies K = 0.
__device__ __forceinline__ int poisson_inv_k(double lam, double u, int kmax) {
#pragma clang fp contract(off)
    if (!(lam > 0.0)) return 0;
    if (u < (1.0 - lam) - 8.881784197001252e-16) return 0;
    int k = 0;
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
__device__ __forceinline__ int poisson_inv(double lam, double u) { return poisson_inv_k(lam, u, kKmax); }

// FP32 pre-tests that only ever decide what the FP64 draw decides.  The leading 24 bits
// of u53(a, b) bound it: (a >> 8) 2^-24 <= u53 < ((a >> 8) + 1) 2^-24, both exact in FP32.
__device__ __forceinline__ float u_lo24(uint32_t a) { return (float)(a >> 8) * 5.9604644775390625e-08f; }
__device__ __forceinline__ float u_hi24(uint32_t a) { return (float)((a >> 8) + 1u) * 5.9604644775390625e-08f; }

// True only if poisson_inv(min(lam, cap), u53(a, .)) is 0 for the FP32 rate lam: each of
// the two FP32 roundings moves 1 - lam - 2^-22 by at most 2^-25, so u stays below
// 1 - lam - 2^-23 and hence below the FP64 shortcut's bound (1 - min(lam, cap)) - 2^-50.
// False for NaN or infinite rates, which then take the FP64 path.
__device__ __forceinline__ bool poisson_surely_zero(float lam, uint32_t a) {
    return u_hi24(a) < (1.0f - lam) - 2.384185791015625e-07f;
}

// True only if a light parent (weight below one product) surely does not convert: the
// FP64 test is u53 < P with P = lam wprod / w; here pf = lam (wprod / w_ref) / wt with
// the reciprocal and three roundings (relative error below 2^-21.6), raised by 2^-20,
// is compared with the lower bound of u.  u_lo24 > 0 also covers a P that underflows.
__device__ __forceinline__ bool light_surely_zero(float lam, float ratio, float wt, uint32_t a) {
    const float pf = lam * ratio * __builtin_amdgcn_rcpf(wt);
    const float lo = u_lo24(a);
    return lo > 0.0f && lo >= pf * 1.00000095367431640625f;
}

// Macro-event count of a conversion operator (Sec. II.F.1) for a parent of physical
// weight w whose products weigh wprod.  A parent lighter than one product converts whole,
// with probability lam wprod / w (the plain rate's conversion probability P), so its mean
// converted weight is w P; light_mode 1 keeps the Poisson count for it.
__device__ __forceinline__ int conversion_count(const KParams& kp, double lam, double lam_eff,
                                                double w, double wprod, double u) {
    if (kp.light_mode == 0 && w < wprod) return (lam > 0.0 && u < lam / (w / wprod)) ? 1 : 0;
    return poisson_inv(lam_eff, u);
}

// Cap and rescale (eqs. lambda_eff, wa_rescaled): returns lambda_eff, *ws = w'/w.
__device__ __forceinline__ double cap_lambda(double lam, double cap, double* ws, int* capped) {
    const bool c = lam > cap;
    *capped = c;
    const double le = c ? cap : lam;
    *ws = c ? lam / le : 1.0;
    return le;
}

// ---------------------------------------------------------------- fast FP32 functions
// The per-particle FP32 rates are bound by vector instructions; they use the
// hardware log2, exp2, reciprocal and square root (v_log_f32, v_exp_f32,
// v_rcp_f32, v_sqrt_f32, about one ulp) and short Taylor series where a closed
// form would cancel.  Relative error of each rate below 5e-6 (the FP64 paths
// keep the correctly rounded library functions).
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945f; }
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896f); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// 1 - e^{-y} for y >= 0: Taylor series below 1/4, else through exp2
__device__ __forceinline__ float f_1mexp(float y) {
    if (y < 0.25f) {
        float a = 0.0f;
#pragma unroll
        for (int k = 8; k >= 1; --k) {
            float f = 1.0f;
            for (int q = 2; q <= k; ++q) f *= (float)q;
            a = a * y + ((k & 1) ? 1.0f : -1.0f) / f;
        }
        return a * y;
    }
    return 1.0f - fexp(-y);
}

// ---------------------------------------------------------------- screening F(s)
// F(s) = (1 + 1/s) ln(1 + s) - 1 (eq. prim_F).  Below s = 0.35 (single) or
// 1/100 (double) the closed form cancels; its series
// sum_{n>=1} (-1)^{n+1} s^n / (n (n+1)) is used instead.
__device__ __forceinline__ float screenF(float s) {
    if (!(s > 0.0f)) return 0.0f;
    if (s < 0.35f) {
        // F(s)/s = sum_n (-1)^(n+1) s^(n-1) / (n (n+1)) on [0, 0.35] by a degree-6
        // Chebyshev fit (relative error 9e-10; with FP32 Horner 5e-8, as the 16-term
        // series it replaces)
        float acc = 7.609401364e-03f;
        acc = fmaf(acc, s, -1.974492148e-02f);
        acc = fmaf(acc, s, 3.245352209e-02f);
        acc = fmaf(acc, s, -4.989826679e-02f);
        acc = fmaf(acc, s, 8.332762122e-02f);
        acc = fmaf(acc, s, -1.666665375e-01f);
        acc = fmaf(acc, s, 0.5f);
        return acc * s;
    }
    return (1.0f + frcp(s)) * flog(1.0f + s) - 1.0f;
}
__device__ __forceinline__ double screenF(double s) {
    if (!(s > 0.0)) return 0.0;
    if (s < 0.01) {
        double acc = 0.0;
#pragma unroll
        for (int n = 12; n >= 1; --n) {
            const double c = ((n & 1) ? 1.0 : -1.0) / (double)(n * (n + 1));
            acc = acc * s + c;
        }
        return acc * s;
    }
    return (1.0 + 1.0 / s) * log1p(s) - 1.0;
}

// (1 - e^-x)/x, accurate for tiny (or underflowed) x.
__device__ __forceinline__ float one_minus_exp_over(float x) {
    if (x < 0.25f) {
        // sum_k (-x)^k / (k+1)!, k <= 6: truncation below 2e-9 relative at x = 0.25
        float a = 0.0f;
#pragma unroll
        for (int k = 6; k >= 0; --k) {
            float f = 1.0f;
            for (int q = 2; q <= k + 1; ++q) f *= (float)q;
            a = a * x + ((k & 1) ? -1.0f : 1.0f) / f;
        }
        return a;
    }
    return f_1mexp(x) * frcp(x);
}
__device__ __forceinline__ double one_minus_exp_over(double x) {
    if (x < 1e-5) return 1.0 - 0.5 * x + x * x * (1.0 / 6.0);
    return -expm1(-x) / x;
}

template <typename T> __device__ __forceinline__ T dev_expm1(T x);
template <> __device__ __forceinline__ float dev_expm1(float x) { return expm1f(x); }
template <> __device__ __forceinline__ double dev_expm1(double x) { return expm1(x); }
template <typename T> __device__ __forceinline__ T dev_exp(T x);
template <> __device__ __forceinline__ float dev_exp(float x) { return expf(x); }
template <> __device__ __forceinline__ double dev_exp(double x) { return exp(x); }
template <typename T> __device__ __forceinline__ T dev_log(T x);
template <> __device__ __forceinline__ float dev_log(float x) { return logf(x); }
template <> __device__ __forceinline__ double dev_log(double x) { return log(x); }
template <typename T> __device__ __forceinline__ T dev_sqrt(T x);
template <> __device__ __forceinline__ float dev_sqrt(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double dev_sqrt(double x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T dev_fma(T a, T b, T c);
template <> __device__ __forceinline__ float dev_fma(float a, float b, float c) { return fmaf(a, b, c); }
template <> __device__ __forceinline__ double dev_fma(double a, double b, double c) { return fma(a, b, c); }
template <typename T> __device__ __forceinline__ T dev_floor(T x);
template <> __device__ __forceinline__ float dev_floor(float x) { return floorf(x); }
template <> __device__ __forceinline__ double dev_floor(double x) { return floor(x); }

// ---------------------------------------------------------------- samplers
// Quantile tables: y = ln x on a uniform grid of z = ln(u/(1-u)) with slopes
// dy/dz, evaluated by cubic Hermite interpolation (FP64).  tab[0..N] = y,
// tab[N+1..2N+1] = dy/dz.
__device__ __forceinline__ double quantile_z(const double* __restrict__ tab, double z) {
    const double h = (kTabZ1 - kTabZ0) / kTabN;
    double t = (z - kTabZ0) / h;
    int j = (int)floor(t);
    j = j < 0 ? 0 : (j > kTabN - 1 ? kTabN - 1 : j);
    const double f = t - (double)j;
    const double y0 = tab[j], y1 = tab[j + 1];
    const double m0 = tab[kTabN + 1 + j] * h, m1 = tab[kTabN + 2 + j] * h;
    const double f2 = f * f, f3 = f2 * f;
    const double y = (2 * f3 - 3 * f2 + 1) * y0 + (f3 - 2 * f2 + f) * m0 +
                     (-2 * f3 + 3 * f2) * y1 + (f3 - f2) * m1;
    return exp(y);
}
__device__ __forceinline__ double quantile(const double* __restrict__ tab, double u) {
    return quantile_z(tab, log(u) - log1p(-u));
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Inclusive scan over the 64 lanes of a wavefront (every lane active): within each row
// of 16 lanes by DPP row shifts of 1, 2, 4 and 8, then the last lane of row 0 and 2 into
// rows 1 and 3 (row_bcast:15) and that of row 1 into rows 2 and 3 (row_bcast:31); six
// DPP adds, no LDS traffic.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
    (void)lane;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// ---------------------------------------------------------------- local state
// Sec. II.E-II.H for one cell from its deposits: composition (eqs. rho_def,
// qn_def), Debye screening (eq. kappa_debye), the Primakoff rate prefactor
// (eqs. prim_xs, prim_rate: Gamma = G_P0 F(s)) and the per-electron
// Compton-like and bremsstrahlung production rates (eqs. epsC, QC, GammaC,
// eps_eZ, eps_ee).  The boost multiplies every rate.
// Screening-fit factor 1 - a eta of the brems emissivities (eqs. eps_eZ, eps_ee;
// a = 6.98e-2 for e-Z, 0.140 for e-e), eta = (3 + X_H) rho_2 / T_7^2, unclipped.
__device__ __forceinline__ double brems_suppression(double T_keV, double rho, double XH, bool ee) {
    const double T7 = T_keV * kKeVT7;
    const double eta = (3.0 + XH) * (rho * 0.01) / (T7 * T7);
    return 1.0 - (ee ? 0.140 : 6.98e-2) * eta;
}

struct LocalState {
    double T, ne, ne_dep, nZ, nZ2, rho, XH, kappa2;
    double G_P0, G_C, G_B, Q_C, Q_B, meanC, meanB;
    double G_BeZ, G_Bee;    // e-Z and e-e parts of G_B (the e-e part is zero when switched off)
};

__device__ __forceinline__ LocalState local_state(double T, double ne_dep, double nZ, double nZ2,
                                                  double rho, double rhoH, const axpic_params& prm) {
    LocalState L;
    L.T = T; L.ne_dep = ne_dep; L.nZ = nZ; L.nZ2 = nZ2; L.rho = rho;
    L.ne = prm.quasi_neutral ? nZ : ne_dep;
    L.XH = rho > 0.0 ? rhoH / rho : 0.0;
    const double hc3 = kHbarcKeVcm * kHbarcKeVcm * kHbarcKeVcm;
    L.kappa2 = prm.kappa_mode == 1 ? prm.kappa_fixed_keV * prm.kappa_fixed_keV
                                   : 4.0 * kPi * kAlpha * (L.ne + nZ2) * hc3 / T;
    const double targets = prm.prim_targets ? (L.ne + nZ2) : nZ2;
    L.G_P0 = prm.boost * kAlpha * prm.g_agg_GeV * prm.g_agg_GeV * 0.125 *
             (kHbarcGeVcm * kHbarcGeVcm) * kC * targets;
    const double a_ae = prm.g_ae * prm.g_ae / (4.0 * kPi) / 1.60e-23;
    const double T7 = T * kKeVT7;
    const double T7sq = T7 * T7;
    const double XH = L.XH;
    L.Q_C = rho * 2.67e-2 * (1.0 + XH) * (T7sq * T7sq * T7sq) * a_ae;
    const double rho2 = rho * 0.01;
    const double base = 0.150 * T7sq * sqrt(T7) * rho2 * (1.0 + XH) * a_ae;
    const double fZ = fmax(0.0, brems_suppression(T, rho, XH, false));
    const double fE = fmax(0.0, brems_suppression(T, rho, XH, true));
    const double epsZ = base * fZ;
    const double epsE = prm.brems_ee ? base * (1.0 + XH) * (0.25 * sqrt(2.0)) * fE : 0.0;
    L.Q_B = rho * (epsZ + epsE);
    L.meanC = 5.0 * kZeta6 / kZeta5 * T;
    L.meanB = prm.brems_k * prm.brems_theta * T;
    const double ne = L.ne;
    L.G_C = ne > 0.0 ? prm.boost * L.Q_C / (ne * L.meanC * kKeVerg) : 0.0;
    L.G_BeZ = ne > 0.0 ? prm.boost * rho * epsZ / (ne * L.meanB * kKeVerg) : 0.0;
    L.G_Bee = ne > 0.0 ? prm.boost * rho * epsE / (ne * L.meanB * kKeVerg) : 0.0;
    L.G_B = ne > 0.0 ? prm.boost * L.Q_B / (ne * L.meanB * kKeVerg) : 0.0;
    return L;
}

// ---------------------------------------------------------------- per-particle rates
// |p|^2 in one fixed order of fused multiply-adds, so that every kernel evaluating a
// rate from the same momentum gets the same bits (no choice left to contraction)
template <typename T>
__device__ __forceinline__ T p2_of(T a, T b, T c) { return dev_fma<T>(c, c, dev_fma<T>(b, b, a * a)); }

template <typename T>
__device__ __forceinline__ T psq(const T* __restrict__ px, const T* __restrict__ py,
                                 const T* __restrict__ pz, int64_t i) {
    return p2_of<T>(px[i], py[i], pz[i]);
}

template <typename T> struct PrefOf;
template <> struct PrefOf<float> { static __device__ const float* get(const float* p32, const double*) { return p32; } };
template <> struct PrefOf<double> { static __device__ const double* get(const float*, const double* p64) { return p64; } };

// A cell's prefactor record (AXPIC_PREF_N = 8 entries, 32-byte aligned in FP32,
// 64-byte in FP64) into registers with 16-byte loads: the count kernels load
// all their parents' records before the arithmetic instead of one dependent
// load chain per parent.
__device__ __forceinline__ void load_pref(const float* __restrict__ rec, float* out, int nq) {
    for (int q = 0; q < nq; ++q) {
        const float4 v = ((const float4*)rec)[q];
        out[4 * q] = v.x; out[4 * q + 1] = v.y; out[4 * q + 2] = v.z; out[4 * q + 3] = v.w;
    }
}
__device__ __forceinline__ void load_pref(const double* __restrict__ rec, double* out, int nq) {
    for (int q = 0; q < 2 * nq; ++q) {
        const double2 v = ((const double2*)rec)[q];
        out[2 * q] = v.x; out[2 * q + 1] = v.y;
    }
}

// lambda_P = w P_{gamma->a} / w_prod with P = 1 - exp(-c_P F(s)) (eqs. prim_xs, prim_prob)
template <typename T>
__device__ __forceinline__ T lambda_primakoff(const T* __restrict__ pc, T w, T p2) {
    const T s = pc[1] * p2;
    const T F = screenF(s);
    const T x = pc[2] * F;
    return w * pc[3] * F * one_minus_exp_over(x);
}

// Particle energy in keV from |p|^2 (units of m_e c) for the rate functions
__device__ __forceinline__ float energy_keV(float p2) { return (float)kMe * fsqrt(p2); }
__device__ __forceinline__ double energy_keV(double p2) { return kMe * sqrt(p2); }

// Thermal absorption probability, eq. gamma_abs: Gamma_abs dt = aC E^2 g_C + aB g_B
template <typename T>
__device__ __forceinline__ T pabs_thermal(const KParams& kp, const T* __restrict__ pc, T E);

template <>
__device__ __forceinline__ float pabs_thermal<float>(const KParams& kp, const float* __restrict__ pc,
                                                     float E) {
    const float x = E * frcp(pc[0]);
    float g = 0.0f;
    if (pc[6] != 0.0f) {
        // BE equilibrium: occupation factor 1; MB: 1/(1 - e^{-x})
        const float e2 = pc[6] * E * E;
        g += kp.eq_stats ? e2 * frcp(f_1mexp(x)) : e2;
    }
    if (pc[7] != 0.0f) {
        // x^{k-3} e^{x (1 - 1/theta)}, times (1 - e^{-x}) for BE
        const float l2 = __builtin_amdgcn_logf(x);
        const float e = __builtin_amdgcn_exp2f((float)kp.brems_km3 * l2 +
                                               (float)kp.brems_c1 * x * 1.44269504088896f);
        g += pc[7] * e * (kp.eq_stats ? 1.0f : f_1mexp(x));
    }
    return f_1mexp(g);
}

// Gamma_abs dt of the thermal channels at energy E from the cell's temperature Tk
// and absorption coefficients c6 (Compton-like) and c7 (brems), FP64.
__device__ __forceinline__ double gabs_dt(const KParams& kp, double Tk, double c6, double c7,
                                          double E) {
    const double x = E / Tk;
    double g = 0.0;
    if (c6 != 0.0) {
        double occ = kp.eq_stats ? -expm1(-x) : 1.0;
        g += c6 * E * E / occ;
    }
    if (c7 != 0.0) {
        const double th = kp.brems_theta, k = kp.brems_k;
        const double pw = exp((k - 3.0) * log(x));
        // MB: e^{x(1-1/theta)}; BE: e^{-x/theta} (e^x - 1), with expm1 for small x
        double shape;
        if (kp.eq_stats || x > 60.0) shape = exp(x * (1.0 - 1.0 / th));
        else shape = exp(-x / th) * expm1(x);
        g += c7 * pw * shape;
    }
    return g;
}

template <>
__device__ __forceinline__ double pabs_thermal<double>(const KParams& kp, const double* __restrict__ pc,
                                                       double E) {
    return -expm1(-gabs_dt(kp, pc[0], pc[6], pc[7], E));
}

// a->gamma mean: w_a-weight * (w_a/w_gamma_prod) * (1 - exp(-ratio c_P F))
template <typename T>
__device__ __forceinline__ T lambda_ag(const KParams& kp, const T* __restrict__ pc, T w, T p2) {
    const T s = pc[1] * p2;
    const T F = screenF(s);
    const T x = (T)kp.inv_ratio * pc[2] * F;
    const T unit = (T)((double)pc[3] * kp.ag_unit);
    return w * unit * F * one_minus_exp_over(x);
}

// ---------------------------------------------------------------- finite mass
// Axions of mass m = kp.m_a [keV] (kp.mu2 = (m / m_e c^2)^2): energy
// E = m_e c^2 sqrt(p^2 + mu^2), push velocity p / sqrt(p^2 + mu^2) (Sec. II.B).
// A photon of momentum k > m converts to an axion of momentum p = sqrt(k^2 - m^2)
// at Gamma = G_P0 (p/k) F_m(k, p), F_m being twice the angular integral of the
// screened amplitude |k x p|^2 / (q^2 (q^2 + kappa^2)), q = k - p.  In closed form,
// with a = 4kp and A = (k-p)^2 + kappa^2,
//   F_m = (A + a) A ln(1 + a/A) / (a kappa^2)
//         - (k-p)^2 ((k-p)^2 + a) ln(1 + a/(k-p)^2) / (a kappa^2) - 1,
// which is F(4k^2/kappa^2) at p = k.
__device__ __forceinline__ double F_mass(double k, double p, double kappa2) {
    if (!(k > 0.0) || !(p > 0.0)) return 0.0;
    if (p >= k) return screenF(4.0 * k * k / kappa2);
    const double a = 4.0 * k * p, am = (k - p) * (k - p), A = am + kappa2;
    const double t1 = (A + a) * A / (a * kappa2) * log1p(a / A);
    const double t2 = am * (am + a) / (a * kappa2) * log1p(a / am);
    return t1 - t2 - 1.0;
}

// |p|^2 in FP64 from the stored components (the massive rates resolve the
// threshold region, where binary32 |p|^2 would not do)
template <typename T>
__device__ __forceinline__ double psq_d(const T* __restrict__ px, const T* __restrict__ py,
                                        const T* __restrict__ pz, int64_t i) {
    return p2_of<double>((double)px[i], (double)py[i], (double)pz[i]);
}

__device__ __forceinline__ double axion_energy(const KParams& kp, double p2) {
    return kMe * sqrt(p2 + kp.mu2);
}

// lambda_P of a photon whose products have mass m (FP64 from the cell's prefactors:
// kappa^2 = 4 m_e^2 / pc[1], c_P = pc[2] = Gamma_P0 dt, pc[3] the lambda unit); zero
// at or below the threshold omega = m.
template <typename T>
__device__ __forceinline__ T lambda_primakoff_m(const KParams& kp, const T* __restrict__ pc, T w,
                                                double p2) {
    const double k = kMe * sqrt(p2);
    if (!(k > kp.m_a)) return (T)0;
    const double p = sqrt((k - kp.m_a) * (k + kp.m_a));
    const double F = p / k * F_mass(k, p, 4.0 * kMe * kMe / (double)pc[1]);
    const double x = (double)pc[2] * F;
    const double om = x > 1e-12 ? -expm1(-x) / x : 1.0 - 0.5 * x;
    return (T)((double)w * (double)pc[3] * F * om);
}

// a->gamma mean of an axion of mass m: the photon takes its energy E; Gamma_{a->gamma}
// = ratio (k/p) Gamma_{gamma->a}(E) = ratio Gamma_P0 F_m(E, p).
template <typename T>
__device__ __forceinline__ T lambda_ag_m(const KParams& kp, const T* __restrict__ pc, T w, double p2) {
    const double p = kMe * sqrt(p2);
    if (!(p > 0.0)) return (T)0;
    const double E = axion_energy(kp, p2);
    const double F = F_mass(E, p, 4.0 * kMe * kMe / (double)pc[1]);
    const double x = kp.inv_ratio * (double)pc[2] * F;
    const double om = x > 1e-12 ? -expm1(-x) / x : 1.0 - 0.5 * x;
    return (T)((double)w * (double)pc[3] * kp.ag_unit * F * om);
}

// Thermal absorption probability of an axion of mass m: the massive equilibrium
// density (E p instead of E^2) multiplies Gamma_abs by E/p.
template <typename T>
__device__ __forceinline__ T pabs_thermal_m(const KParams& kp, const T* __restrict__ pc, double p2) {
    const double p = kMe * sqrt(p2);
    if (!(p > 0.0)) return (T)0;
    const double E = axion_energy(kp, p2);
    const double g = gabs_dt(kp, (double)pc[0], (double)pc[6], (double)pc[7], E) * (E / p);
    return (T)(-expm1(-g));
}

// Fractions of the thermal samplers' number spectra above x (FP64).
// Compton-like x^4/(e^x - 1)/(24 zeta5): below x = 1/4 one minus the series
// sum_n B_n x^{n+4}/(n! (n+4)) (B_n the Bernoulli numbers), above it the sum
// over j of e^{-jx} (x^4/j + 4x^3/j^2 + 12x^2/j^3 + 24x/j^4 + 24/j^5), both
// divided by 24 zeta(5).
__device__ __forceinline__ double compton_tail(double x) {
    constexpr double kNorm = 24.0 * 1.0369277551433699263;
    if (!(x > 0.0)) return 1.0;
    if (x < 0.25) {
        const double B[11] = {1.0, -0.5, 1.0 / 6.0, 0.0, -1.0 / 30.0, 0.0, 1.0 / 42.0, 0.0,
                              -1.0 / 30.0, 0.0, 5.0 / 66.0};
        double s = 0.0, xp = x * x * x * x, fact = 1.0;
        for (int n = 0; n <= 10; ++n) {
            if (n > 0) fact *= n;
            s += B[n] * xp / (fact * (n + 4));
            xp *= x;
        }
        return 1.0 - s / kNorm;
    }
    double s = 0.0;
    for (int j = 1; j < 4000; ++j) {
        const double dj = (double)j, e = exp(-dj * x);
        const double t = e * ((((x / dj + 4.0 / (dj * dj)) * x + 12.0 / (dj * dj * dj)) * x +
                               24.0 / (dj * dj * dj * dj)) * x + 24.0 / (dj * dj * dj * dj * dj));
        s += t;
        if (t < 1e-17 * s) break;
    }
    return s / kNorm;
}

// Upper regularised incomplete gamma Q(k, y) of the Gamma(k, 1) sampler: one minus
// the power series of P below y = k + 1, above it Legendre's continued fraction by
// the modified Lentz algorithm (Lentz 1976; Thompson and Barnett 1986; Press et al.,
// Numerical Recipes, Sec. 6.2).
__device__ __forceinline__ double gamma_tail(double k, double y) {
    if (!(y > 0.0)) return 1.0;
    const double pre = exp(-y + k * log(y) - lgamma(k));
    if (y < k + 1.0) {
        double term = 1.0 / k, sum = term;
        for (int n = 1; n < 2000; ++n) {
            term *= y / (k + n);
            sum += term;
            if (term < sum * 1e-17) break;
        }
        return 1.0 - sum * pre;
    }
    const double tiny = 1e-300;
    double b = y + 1.0 - k, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 2000; ++i) {
        const double an = -(double)i * ((double)i - k);
        b += 2.0;
        d = an * d + b; if (fabs(d) < tiny) d = tiny;
        c = b + an / c; if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        const double del = d * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return pre * h;
}

// Energy E [keV] and momentum magnitude pm [m_e c] of a thermal product of channel
// ch (1 Compton-like, 2 brems) in a cell at temperature Tc, drawn at uniform u by
// the quantile table; with mass m the spectrum is cut at E = m: the quantile is
// taken at F + u Q, Q = 1 - F the fraction above m, in z = ln(F + u Q) - ln((1 - u) Q).
template <bool M>
__device__ __forceinline__ void thermal_energy(const KParams& kp, int ch, double Tc, double u,
                                               const double* __restrict__ tab, double* E,
                                               double* pm) {
    const double xs = ch == 1 ? 1.0 : kp.brems_theta;
    if (!M) {
        *E = Tc * xs * quantile(tab, u);
        *pm = *E / kMe;
        return;
    }
    const double xm = kp.m_a / (xs * Tc);
    const double Q = ch == 1 ? compton_tail(xm) : gamma_tail(kp.brems_k, xm);
    const double z = log((1.0 - Q) + u * Q) - log((1.0 - u) * Q);
    *E = Tc * xs * quantile_z(tab, z);
    *pm = *E > kp.m_a ? sqrt((*E - kp.m_a) * (*E + kp.m_a)) / kMe : 0.0;
}

}  // namespace axpic
