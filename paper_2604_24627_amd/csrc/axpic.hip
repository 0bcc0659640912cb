// axpic.hip -- HIP (gfx950) implementation of the axion Monte-Carlo operators
// behind the C ABI in include/axpic.h.
//
// Layout of the work: every per-particle operator that creates products runs
// over the parent stream as
//   count : rates + Philox + Poisson per parent and per-block totals; the
//           emission counts compact each tile's converting parents into a list,
//           the absorption count keeps a 16-bit decision code per axion;
//   scan  : one workgroup turns the block totals into exclusive offsets and
//           checks the capacity;
//   expand + events (emission): one record per product from the lists, then one
//           product per lane (recomputing its parent's rate bitwise the same);
//   apply (absorption): blocks with activity recompute their axions' rates, scan
//           the codes in axion order and write products;
//   finish: the per-block histogram and statistics records and the boundary
//           sums of the exchange, in block order.
// Products therefore land in the canonical order (parent, channel, event) and
// their ids come from the offset, never from an atomic slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/axpic.h"
#include "axpic_device.hpp"
#include "axpic_timing.hpp"
#include "axpic_tables.h"

using namespace axpic;

namespace {

constexpr int kThreads = 256;          // threads per workgroup
constexpr int kPer = 4;                // parents per thread in the count/apply kernels
constexpr int kBlockParents = kThreads * kPer;
static_assert(kPer == 4, "st_codes packs four 16-bit codes per thread");
constexpr int kStatSlots = 12;         // per-thread statistics registers
// histogram bins per channel (+2 under/overflow); the events kernels hold a private copy
// of two channels per wavefront in LDS: 4 x 2 x 1002 doubles stay within 64 KiB
constexpr int kMaxBins = 1000;
constexpr int kRecMax = 2 * (kMaxBins + 2) + AXPIC_ST_COUNT;   // doubles of a block's record
constexpr int kScanThreads = 1024;
constexpr int kEventBlocks = 1024;     // grid of the event kernels (grid-stride over events)

__device__ double g_tab_compton[2 * (kTabN + 1)];
__device__ double g_tab_gamma[2 * (kTabN + 1)];

// Static device scratch of the allocation-free entry point axpic_diag_noalloc: the
// per-block partial sums (N, U) of the population, kDiagScratchPairs blocks of
// kBlockParents particles at most.  Each GPU holds its own copy until the process ends;
// host code uses only the address that hipGetSymbolAddress returns for the current
// device, never this name.
constexpr int64_t kDiagScratchPairs = 262144;                  // 4 MiB, 2^28 particles
static __device__ __align__(256) double scratch[2 * kDiagScratchPairs];

// ------------------------------------------------------------------ workspace
struct Workspace {
    uint16_t* code;      // [n_max] 16-bit codes, or (as list) 32-bit entries
    uint32_t* bsum;      // [nb] products per block
    uint32_t* bact;      // [nb] active parents per block
    uint64_t* boff;      // [nb] exclusive product offsets
    double* rec;         // per-block records: histogram bins, then statistics
    int32_t* bkey;       // [2 nbmax] boundary cells of the blocks (fixed-order fb sums)
    double* bval;        // [2 nbmax][4] their sums
    int64_t* ctrl;       // [8]: 0 skip flag, 1 total
    uint32_t* list() const { return (uint32_t*)code; }   // [n_max] active-parent entries
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
inline int64_t nblocks_for(int64_t n) { return (n + kBlockParents - 1) / kBlockParents; }

// records: an events kernel's grid of histogram + statistics records, or one statistics
// record per block of parents; boundary records: two per block of either
size_t rec_doubles(int64_t nb) {
    return std::max<size_t>((size_t)kEventBlocks * kRecMax, (size_t)nb * AXPIC_ST_COUNT);
}
size_t bnd_count(int64_t nb) { return 2 * (size_t)std::max<int64_t>(kEventBlocks, nb); }

size_t ws_bytes_for(int64_t n) {
    int64_t nb = nblocks_for(std::max<int64_t>(n, 1));
    return align256(sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1)) + align256(4 * (size_t)nb) +
           align256(4 * (size_t)nb) + align256(8 * (size_t)nb) +
           align256(sizeof(double) * rec_doubles(nb)) + align256(4 * bnd_count(nb)) +
           align256(sizeof(double) * 4 * bnd_count(nb)) + 256;
}

bool carve(void* ws, size_t bytes, int64_t n, Workspace* w) {
    if (!ws || bytes < ws_bytes_for(n)) return false;
    int64_t nb = nblocks_for(std::max<int64_t>(n, 1));
    char* p = (char*)ws;
    w->code = (uint16_t*)p; p += align256(sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1));
    w->bsum = (uint32_t*)p; p += align256(4 * (size_t)nb);
    w->bact = (uint32_t*)p; p += align256(4 * (size_t)nb);
    w->boff = (uint64_t*)p; p += align256(8 * (size_t)nb);
    w->rec = (double*)p; p += align256(sizeof(double) * rec_doubles(nb));
    w->bkey = (int32_t*)p; p += align256(4 * bnd_count(nb));
    w->bval = (double*)p; p += align256(sizeof(double) * 4 * bnd_count(nb));
    w->ctrl = (int64_t*)p;
    return true;
}

// ------------------------------------------------------------------ host params
KParams make_kparams(const axpic_grid* g, const axpic_params* prm, double w_ref_g) {
    KParams k;
    std::memset(&k, 0, sizeof(k));
    k.dt_phys = g->dt / g->omega0;
    k.w_a = prm->w_a;
    for (int i = 0; i < 3; ++i) k.wa_mul[i] = prm->wa_mul[i];
    k.w_gamma_prod = prm->w_gamma_prod > 0.0 ? prm->w_gamma_prod : w_ref_g;
    k.cap = (prm->lambda_cap <= kLambdaHardCap) ? prm->lambda_cap : kLambdaHardCap;
    k.inv_ratio = prm->prim_inv_ratio;
    k.ag_unit = (w_ref_g > 0.0 && k.w_gamma_prod > 0.0)
                    ? prm->prim_inv_ratio * prm->w_a * prm->w_a * prm->wa_mul[0] /
                          (w_ref_g * k.w_gamma_prod)
                    : 0.0;
    k.brems_k = prm->brems_k;
    k.brems_theta = prm->brems_theta;
    k.brems_km3 = prm->brems_k - 3.0;
    k.brems_c1 = 1.0 - 1.0 / prm->brems_theta;
    k.nbins = prm->hist_nbins;
    k.hist_log = prm->hist_log;
    k.hist_lo = prm->hist_lo_keV;
    k.hist_scale = prm->hist_log ? prm->hist_nbins / std::log(prm->hist_hi_keV / prm->hist_lo_keV)
                                 : prm->hist_nbins / (prm->hist_hi_keV - prm->hist_lo_keV);
    k.r_relax = prm->r_relax;
    k.T_floor = prm->T_floor_keV;
    k.T_ceil = prm->T_ceil_keV;
    k.dtdx = g->dt / g->dx;
    k.seed_lo = (uint32_t)prm->seed;
    k.seed_hi = (uint32_t)(prm->seed >> 32);
    k.channels = prm->channels;
    k.inverse = prm->inverse;
    k.absorb_mode = prm->absorb_mode;
    k.eq_stats = prm->eq_stats;
    k.T_mode = prm->T_mode;
    k.feedback = prm->feedback;
    k.ndim = g->ndim;
    for (int d = 0; d < 3; ++d) k.n[d] = g->n[d];
    k.m_a = prm->m_a_keV;
    k.mu2 = (prm->m_a_keV / kMe) * (prm->m_a_keV / kMe);
    k.massive = prm->m_a_keV > 0.0;
    k.light_mode = prm->light_mode;
    return k;
}

bool grid_ok(const axpic_grid* g) {
    if (!g || g->ndim < 1 || g->ndim > 3) return false;
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 1) return false;
        if (d >= g->ndim && g->n[d] != 1) return false;
    }
    if (!(g->dx > 0.0) || !(g->dt > 0.0) || !(g->omega0 > 0.0)) return false;
    if ((int64_t)g->n[0] * g->n[1] * g->n[2] > INT32_MAX) return false;
    return true;
}

bool params_ok(const axpic_params* p) {
    if (!p) return false;
    if (!(p->lambda_cap > 0.0) || !(p->w_a > 0.0)) return false;
    if (!(p->r_relax >= 0.0 && p->r_relax <= 1.0)) return false;
    if (!(p->m_a_keV >= 0.0 && p->m_a_keV < 1e6)) return false;
    if (p->light_mode != 0 && p->light_mode != 1) return false;
    if (p->hist_nbins < 1 || p->hist_nbins > kMaxBins || !(p->hist_hi_keV > p->hist_lo_keV))
        return false;
    if (p->hist_log && !(p->hist_lo_keV > 0.0)) return false;
    if (!(p->brems_k > 0.0) || !(p->brems_theta >= 1.0)) return false;
    for (int i = 0; i < 3; ++i)
        if (!(p->wa_mul[i] > 0.0)) return false;
    return true;
}

int64_t ncell_of(const axpic_grid* g) { return (int64_t)g->n[0] * g->n[1] * g->n[2]; }

bool species_ok(const axpic_species* s, bool need_p) {
    if (!s || s->n < 0 || s->capacity < s->n) return false;
    if (s->dtype != AXPIC_F32 && s->dtype != AXPIC_F64) return false;
    if (s->n == 0) return true;
    if (s->n_implicit < 0 || s->n_implicit > s->n) return false;
    if (!s->w || !s->cell || (!s->id && s->n_implicit < s->n)) return false;
    if (s->off && (s->n_sorted < 0 || s->n_sorted > s->n)) return false;
    if (need_p && (!s->p[0] || !s->p[1] || !s->p[2])) return false;
    return true;
}

// Sampler tables: per device, uploaded on first use and when brems_k changes.
std::mutex g_tab_mutex;
struct TabState { bool compton = false; double k = -1.0; };
std::vector<TabState> g_tab_state;

axpic_status ensure_tables(double k) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return AXPIC_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_tab_mutex);
    if ((int)g_tab_state.size() <= dev) g_tab_state.resize(dev + 1);
    TabState& st = g_tab_state[dev];
    static std::vector<double> buf(2 * (kTabN + 1));
    if (!st.compton) {
        axpic_host::build_compton_table(buf.data());
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_tab_compton), buf.data(), sizeof(double) * buf.size()) !=
            hipSuccess)
            return AXPIC_E_DEVICE;
        st.compton = true;
    }
    if (st.k != k) {
        axpic_host::build_gamma_table(buf.data(), k);
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_tab_gamma), buf.data(), sizeof(double) * buf.size()) !=
            hipSuccess)
            return AXPIC_E_DEVICE;
        st.k = k;
    }
    return AXPIC_OK;
}

inline axpic_status launched() {
    return hipGetLastError() == hipSuccess ? AXPIC_OK : AXPIC_E_DEVICE;
}


// ------------------------------------------------------------------ kernel timing
struct PendingTime { const char* name; hipEvent_t a, b, ma, mb; };
struct TimingState {
    std::mutex mu;
    bool on = false;
    std::string only;                     // time only the launches of this kernel (if set)
    std::vector<hipEvent_t> pool;
    std::vector<PendingTime> pending;
    std::vector<std::pair<std::string, std::pair<long long, double>>> acc;
};
TimingState& timing() { static TimingState t; return t; }

hipEvent_t pool_get(TimingState& t) {
    if (!t.pool.empty()) { hipEvent_t e = t.pool.back(); t.pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// ------------------------------------------------------------------ device helpers
__device__ __forceinline__ int hist_bin(const KParams& kp, double E) {
    double t = kp.hist_log ? log(E / kp.hist_lo) * kp.hist_scale : (E - kp.hist_lo) * kp.hist_scale;
    double b = floor(t);
    if (!(b >= 0.0)) return kp.nbins;
    if (b >= (double)kp.nbins) return kp.nbins + 1;
    return (int)b;
}

// Particle ids: the first n_implicit particles of a buffer have id id0 + i
// (plasma species keep their creation order), the rest are stored.
struct IdView {
    const uint64_t* id;
    uint64_t id0;
    int64_t nimp;
    __device__ __forceinline__ uint64_t operator()(int64_t i) const {
        return i < nimp ? id0 + (uint64_t)i : id[i];
    }
    // ids of the run i0 .. i0 + kPer - 1 (VEC: the run lies in the buffer, 16-byte loads)
    template <bool VEC> __device__ __forceinline__ void run(int64_t i0, int64_t n, uint64_t* v) const;
};

// A thread's run of kPer consecutive parents i0 .. i0 + kPer - 1.  With VEC (the whole
// workgroup's parents lie in the buffer and the base pointers are 16-byte aligned; i0 is
// a multiple of kPer) each array is read with 16-byte loads, else with one clamped
// scalar load per parent.  The kernels instantiate both and branch once per workgroup.
template <bool VEC>
__device__ __forceinline__ void ld_run(const float* __restrict__ p, int64_t i0, int64_t n, float* v) {
    if (VEC) {
        const float4 q = *(const float4*)(p + i0);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int q = 0; q < kPer; ++q) v[q] = p[i0 + q < n ? i0 + q : n - 1];
    }
}
template <bool VEC>
__device__ __forceinline__ void ld_run(const double* __restrict__ p, int64_t i0, int64_t n, double* v) {
    if (VEC) {
        const double2 a = *(const double2*)(p + i0), b = *(const double2*)(p + i0 + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
#pragma unroll
        for (int q = 0; q < kPer; ++q) v[q] = p[i0 + q < n ? i0 + q : n - 1];
    }
}
template <bool VEC>
__device__ __forceinline__ void ld_run(const int32_t* __restrict__ p, int64_t i0, int64_t n, int32_t* v) {
    if (VEC) {
        const int4 q = *(const int4*)(p + i0);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int q = 0; q < kPer; ++q) v[q] = p[i0 + q < n ? i0 + q : n - 1];
    }
}
template <bool VEC>
__device__ __forceinline__ void IdView::run(int64_t i0, int64_t n, uint64_t* v) const {
    if (i0 + kPer <= nimp) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) v[q] = id0 + (uint64_t)(i0 + q);
    } else if (VEC && i0 >= nimp) {
        const ulonglong2 a = *(const ulonglong2*)(id + i0), b = *(const ulonglong2*)(id + i0 + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
#pragma unroll
        for (int q = 0; q < kPer; ++q) v[q] = (*this)(i0 + q < n ? i0 + q : n - 1);
    }
}
// The kPer 16-bit codes of a run (vec: one 8-byte store).
template <bool VEC>
__device__ __forceinline__ void st_codes(uint16_t* __restrict__ code, int64_t i0, int64_t n,
                                         const uint32_t* cd) {
    if (VEC) {
        *(uint2*)(code + i0) = make_uint2(cd[0] | (cd[1] << 16), cd[2] | (cd[3] << 16));
    } else {
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (i0 + q < n) code[i0 + q] = (uint16_t)cd[q];
    }
}


// ------------------------------------------------------------------ block scan
// Exclusive scan of one value per thread across the workgroup (kThreads).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds_w, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) lds_w[wave] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        uint32_t s = lds_w[w];
        if (w < wave) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* lds_w) {
    uint32_t tot;
    (void)block_excl_scan(v, lds_w, &tot);
    return tot;
}

struct StatMap { int m[kStatSlots]; };

// ------------------------------------------------------------------ fixed-order sums
// The FP64 sums of the operators -- histograms, statistics, the per-cell exchange fb --
// take no floating-point atomics: within a wavefront they run through fixed shuffle
// trees, across the wavefronts and tiles of a block in a fixed sequence, and across
// blocks through per-block records summed in block order (k_acc_reduce) and the cells
// a block shares with its neighbours (k_fb_bounds).  Repeated runs give the same bits.

// Adds v at bin (bin < 0: nothing) to this wavefront's private histogram h: the 64
// (bin, lane) pairs sorted by a bitonic network, equal bins summed by a segmented
// scan, one add per distinct bin.  Every lane of the wavefront must call it.
__device__ __forceinline__ void wave_hist_add(double* __restrict__ h, int bin, double v) {
    const int lane = threadIdx.x & 63;
    if (!__any(bin >= 0)) return;
    uint32_t key = bin >= 0 ? ((uint32_t)bin << 6) | (uint32_t)lane : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t ok = __shfl_xor(key, j, 64);
            const bool up = (lane & k) == 0, lower = (lane & j) == 0;
            if (lower == up ? ok < key : ok > key) key = ok;
        }
    }
    // the keys carry their lane: the values follow in one gather
    double val = __shfl(bin >= 0 ? v : 0.0, (int)(key & 63u), 64);
    const uint32_t b = key >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double pv = __shfl_up(val, o, 64);
        const uint32_t pb = __shfl_up(b, o, 64);
        if (lane >= o && pb == b) val += pv;
    }
    const uint32_t nb = __shfl_down(b, 1, 64);
    if (key != 0xFFFFFFFFu && (lane == 63 || nb != b)) h[b] += val;
}

// The block's record: histogram column k = the wavefronts' private copies (wh, h columns
// each) summed in order; then the statistics, st of each thread through the wavefront
// butterfly and the wavefronts in order into the slots map names (every other statistics
// column 0).  Column k at rec[k * cstride].  lds: kThreads/64 * kStatSlots doubles.
__device__ __forceinline__ void rec_write(const double* wh, int h, const double* st,
                                          const StatMap& map, double* lds,
                                          double* __restrict__ rec, int64_t cstride = 1) {
    constexpr int kWaves = kThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kStatSlots; ++k) {
        const double v = wave_sum(st[k]);
        if (lane == 0) lds[wave * kStatSlots + k] = v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < h; k += kThreads) {
        double s = 0.0;
        for (int w2 = 0; w2 < kWaves; ++w2) s += wh[w2 * h + k];
        rec[k * cstride] = s;
    }
    for (int k = threadIdx.x; k < AXPIC_ST_COUNT; k += kThreads) {
        double s = 0.0;
        for (int q = 0; q < kStatSlots; ++q)
            if (map.m[q] == k)
                for (int w2 = 0; w2 < kWaves; ++w2) s += lds[w2 * kStatSlots + q];
        rec[(h + k) * cstride] = s;
    }
}

// Per-cell exchange sums over a block's events in their (cell-ordered) sequence.  Each
// tile of kThreads events: a segmented scan per wavefront; the runs inside a wavefront
// are whole cells of this block and are added to fb at once; the first and last run of
// each wavefront are stitched by thread 0 in sequence.  The block's first and last cell
// may continue in the neighbouring blocks: they go to its two boundary records (key,
// four sums), which k_fb_bounds adds up.  Events past the block's range carry key -1
// and come last.
struct FbStitch {
    int32_t fkey[kThreads / 64], lkey[kThreads / 64];     // lkey -2: one run only
    double fs[kThreads / 64][4], ls[kThreads / 64][4];
    int32_t dkey[2 * (kThreads / 64)];                    // runs completed by the stitching,
    double ds[2 * (kThreads / 64)][4];                    // added to fb by as many threads
    int32_t nd;
};
struct FbOpen {                 // thread 0's state across the tiles of a block
    int32_t key = -1;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    bool first_done = false;
};

// A completed run: the block's first to its first boundary record, any later one to the
// list S (added to fb after the tile's barrier; runs summing to zero are skipped, S NULL:
// added here).
__device__ __forceinline__ void fb_close(FbOpen& o, FbStitch* S, double* __restrict__ fb,
                                         int32_t* __restrict__ bkey, double* __restrict__ bval,
                                         int64_t b) {
    if (o.key < 0) return;
    if (!o.first_done) {
        bkey[2 * b] = o.key;
        for (int q = 0; q < 4; ++q) bval[8 * b + q] = o.s[q];
        o.first_done = true;
    } else if (o.s[0] != 0.0 || o.s[1] != 0.0 || o.s[2] != 0.0 || o.s[3] != 0.0) {
        if (S) {
            S->dkey[S->nd] = o.key;
            for (int q = 0; q < 4; ++q) S->ds[S->nd][q] = o.s[q];
            ++S->nd;
        } else {
            double* f = fb + (int64_t)o.key * 4;
            for (int q = 0; q < 4; ++q) f[q] += o.s[q];
        }
    }
}

__device__ __forceinline__ void fb_tile(FbStitch& S, FbOpen& o, int32_t key, const double* v,
                                        double* __restrict__ fb, int32_t* __restrict__ bkey,
                                        double* __restrict__ bval, int64_t b) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double s[4] = {v[0], v[1], v[2], v[3]};
    // a wavefront without exchange has every run sum zero: no scan, no interior add
    const bool some = __any(v[0] != 0.0 || v[1] != 0.0 || v[2] != 0.0 || v[3] != 0.0);
    if (some) {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t pk = __shfl_up(key, off, 64);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double pv = __shfl_up(s[q], off, 64);
                if (lane >= off && pk == key) s[q] += pv;
            }
        }
    }
    const int32_t nk = __shfl_down(key, 1, 64);
    const int32_t k0 = __shfl(key, 0, 64);
    const bool tail = key >= 0 && (lane == 63 || nk != key);
    const bool first = key == k0;                        // the run holding lane 0
    const bool last = lane == 63 || nk < 0;              // the wavefront's last event run
    if (some && tail && !first && !last) {
        double* f = fb + (int64_t)key * 4;
        for (int q = 0; q < 4; ++q) f[q] += s[q];
    }
    // lane 0's words first, then the tail lanes' (one wavefront: program order)
    if (lane == 0) { S.fkey[wave] = k0; S.lkey[wave] = -2; }
    if (tail && first) for (int q = 0; q < 4; ++q) S.fs[wave][q] = s[q];
    if (tail && last && !first) {
        S.lkey[wave] = key;
        for (int q = 0; q < 4; ++q) S.ls[wave][q] = s[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        S.nd = 0;
        for (int w2 = 0; w2 < kThreads / 64; ++w2) {
            if (S.fkey[w2] < 0) break;                   // no event here nor after
            if (S.fkey[w2] == o.key) {
                for (int q = 0; q < 4; ++q) o.s[q] += S.fs[w2][q];
            } else {
                fb_close(o, &S, fb, bkey, bval, b);
                o.key = S.fkey[w2];
                for (int q = 0; q < 4; ++q) o.s[q] = S.fs[w2][q];
            }
            if (S.lkey[w2] != -2) {
                fb_close(o, &S, fb, bkey, bval, b);
                o.key = S.lkey[w2];
                for (int q = 0; q < 4; ++q) o.s[q] = S.ls[w2][q];
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < S.nd) {                       // distinct cells, one thread each
        double* f = fb + (int64_t)S.dkey[threadIdx.x] * 4;
        for (int q = 0; q < 4; ++q) f[q] += S.ds[threadIdx.x][q];
    }
}

// Thread 0 at the end of a block: the last run to the second boundary record (a block of
// one run has it in the first, and the second holds the same key and zeros).
__device__ __forceinline__ void fb_finish(FbOpen& o, double* __restrict__ fb,
                                          int32_t* __restrict__ bkey, double* __restrict__ bval,
                                          int64_t b) {
    if (threadIdx.x != 0) return;
    if (!o.first_done) {
        fb_close(o, nullptr, fb, bkey, bval, b);
        bkey[2 * b + 1] = o.key;
        for (int q = 0; q < 4; ++q) bval[8 * b + 4 + q] = 0.0;
        if (o.key < 0) bkey[2 * b] = -1;
    } else {
        bkey[2 * b + 1] = o.key;
        for (int q = 0; q < 4; ++q) bval[8 * b + 4 + q] = o.s[q];
    }
}

// Blocks of an events grid of nb blocks that get events when `total` events are split
// over it: as many as there are tiles of kThreads events, at most the grid.
__device__ __forceinline__ int64_t ev_blocks(int64_t total, int64_t nb) {
    const int64_t tiles = (total + kThreads - 1) / kThreads;
    return tiles < nb ? tiles : nb;
}

// The boundary records of nb blocks in block order: each first record of a run of equal
// keys sums the run in order and adds it to fb (key -1: none); block b of this part takes
// records b kThreads ...  Nothing after an overflow.  ev: the blocks of an events grid, of
// which only the first ev_blocks(ctrl[1]) wrote.
__device__ __forceinline__ void fb_bounds_part(int64_t b, int64_t nb,
                                               const int32_t* __restrict__ bkey,
                                               const double* __restrict__ bval,
                                               const int64_t* __restrict__ ctrl,
                                               double* __restrict__ fb, int ev) {
    if (ctrl[0]) return;
    if (ev) nb = ev_blocks(ctrl[1], nb);
    const int64_t i = b * kThreads + threadIdx.x;
    if (i >= 2 * nb) return;
    const int32_t k = bkey[i];
    if (k < 0 || (i > 0 && bkey[i - 1] == k)) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t j = i; j < 2 * nb && bkey[j] == k; ++j)
        for (int q = 0; q < 4; ++q) s[q] += bval[4 * j + q];
    double* f = fb + (int64_t)k * 4;
    for (int q = 0; q < 4; ++q) f[q] += s[q];
}

// The contiguous range of events of block b (empty for the blocks beyond ev_blocks).
__device__ __forceinline__ void ev_range(int64_t total, int64_t* lo, int64_t* hi) {
    const int64_t ga = ev_blocks(total, (int64_t)gridDim.x);
    const int64_t b = blockIdx.x;
    if (b >= ga) { *lo = *hi = 0; return; }
    *lo = total * b / ga;
    *hi = total * (b + 1) / ga;
}

// ------------------------------------------------------------------ scan kernel
// One workgroup: exclusive offsets of the block product counts, capacity check.
// Each thread scans 16 consecutive block totals held in registers (four
// 16-byte loads, eight 16-byte stores); a tile covers 16384 blocks.
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

__global__ void __launch_bounds__(kScanThreads)
k_scan(const uint32_t* __restrict__ bsum, uint64_t* __restrict__ boff, int64_t nb,
       int64_t n_out, int64_t capacity, int64_t* __restrict__ ctrl, int64_t* __restrict__ status,
       uint64_t next_id, int64_t* __restrict__ chain, int chain_slot) {
    __shared__ uint64_t wsum[kScanThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // the chain's words, read before the scan so that their latency overlaps it: output
    // offset and first id (the chain's when chained, else the host's; a call without an
    // output species, chain_slot < 0, only honours the skip word)
    int64_t base = n_out, id0 = (int64_t)next_id;
    bool skip = false;
    if (t == 0 && chain) {
        if (chain_slot >= 0) base = chain[chain_slot];
        id0 = chain[AXPIC_CHAIN_NEXT_ID];
        skip = chain[AXPIC_CHAIN_SKIP] != 0;
    }
    uint64_t carry = 0;
    for (int64_t t0 = 0; t0 < nb; t0 += kScanTile) {
        const int64_t b0 = t0 + (int64_t)t * kScanPer;
        uint32_t v[kScanPer];
        if (b0 + kScanPer <= nb) {
            const uint4* src = (const uint4*)(bsum + b0);
#pragma unroll
            for (int q = 0; q < kScanPer / 4; ++q) {
                const uint4 u = src[q];
                v[4 * q] = u.x; v[4 * q + 1] = u.y; v[4 * q + 2] = u.z; v[4 * q + 3] = u.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < kScanPer; ++q) v[q] = b0 + q < nb ? bsum[b0 + q] : 0u;
        }
        uint64_t sum = 0;
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) sum += v[q];
        uint64_t inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint64_t base = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kScanThreads / 64; ++w) {
            const uint64_t ws = wsum[w];
            if (w < wave) base += ws;
            tot += ws;
        }
        uint64_t run = carry + base + inc - sum;
        uint64_t o[kScanPer];
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) { o[q] = run; run += v[q]; }
        if (b0 + kScanPer <= nb) {
            ulonglong2* dst = (ulonglong2*)(boff + b0);
#pragma unroll
            for (int q = 0; q < kScanPer / 2; ++q) dst[q] = make_ulonglong2(o[2 * q], o[2 * q + 1]);
        } else {
#pragma unroll
            for (int q = 0; q < kScanPer; ++q)
                if (b0 + q < nb) boff[b0 + q] = o[q];
        }
        carry += tot;
        __syncthreads();
    }
    if (t == 0) {
        const bool full = base + (int64_t)carry > capacity;
        const bool over = skip || full;
        ctrl[0] = over ? 1 : 0;
        ctrl[1] = (int64_t)carry;
        ctrl[2] = base;
        ctrl[3] = id0;
        if (status) {
            status[0] = base + (int64_t)carry;
            status[1] = (skip ? AXPIC_FLAG_SKIPPED : 0) | (full ? AXPIC_FLAG_CAPACITY : 0);
            status[2] = over ? 0 : (int64_t)carry;
            status[3] = 0;
        }
        if (chain) {
            if (over) chain[AXPIC_CHAIN_SKIP] = 1;
            else if (chain_slot >= 0) {
                chain[chain_slot] = base + (int64_t)carry;
                chain[AXPIC_CHAIN_NEXT_ID] = id0 + (int64_t)carry;
            }
        }
    }
}

// Column j of the nrec records (record r's column j at rec[r * rstride + j * cstride], in
// block order): histogram column j < nh into hist[j], the others into stats[j - nh].  One
// block per column: each thread sums its records in order, then the wavefront butterfly
// and the wavefronts in order.
__device__ __forceinline__ void acc_column(int j, const double* __restrict__ rec, int64_t nrec,
                                           int64_t rstride, int64_t cstride, int nh,
                                           const int64_t* __restrict__ ctrl,
                                           double* __restrict__ hist, double* __restrict__ stats,
                                           int ev) {
    __shared__ double lds[kThreads / 64];
    if (ctrl && ctrl[0]) return;
    if (ev) nrec = ev_blocks(ctrl[1], nrec);      // an events grid: its writing blocks
    double s = 0.0;
    // eight loads in flight, added in the same order as one at a time
    int64_t r = threadIdx.x;
    for (; r + 7 * kThreads < nrec; r += 8 * kThreads) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = rec[(r + u * kThreads) * rstride + j * cstride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; r < nrec; r += kThreads) s += rec[r * rstride + j * cstride];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    s = 0.0;
    for (int w2 = 0; w2 < kThreads / 64; ++w2) s += lds[w2];
    if (s == 0.0) return;
    if (j < nh) { if (hist) hist[j] += s; }
    else if (stats) stats[j - nh] += s;
}

// The end of an accumulating call in one launch: blocks 0 .. ncol-1 sum the record
// columns (acc_column), the blocks after add the boundary records of nbb blocks to fb
// (fb_bounds_part); either part may be empty.
__global__ void __launch_bounds__(kThreads)
k_finish(const double* __restrict__ rec, int64_t nrec, int64_t rstride, int64_t cstride, int nh,
         int ncol, double* __restrict__ hist, double* __restrict__ stats, int64_t nbb,
         const int32_t* __restrict__ bkey, const double* __restrict__ bval,
         double* __restrict__ fb, const int64_t* __restrict__ ctrl, int ev) {
    if ((int)blockIdx.x < ncol)
        acc_column((int)blockIdx.x, rec, nrec, rstride, cstride, nh, ctrl, hist, stats, ev);
    else
        fb_bounds_part((int64_t)blockIdx.x - ncol, nbb, bkey, bval, ctrl, fb, ev);
}

// ------------------------------------------------------------------ cell state
__global__ void __launch_bounds__(kThreads)
k_cell_state(int64_t ncell, const double* __restrict__ Tk, const double* __restrict__ dens,
             int32_t nion, double Z0, double Z1, double Z2, double Z3, double A0, double A1,
             double A2, double A3, axpic_params prm, double dt_phys, double w_ref_e,
             double w_ref_g, double* __restrict__ state, float* __restrict__ p32,
             double* __restrict__ p64) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const double Zs[4] = {Z0, Z1, Z2, Z3}, As[4] = {A0, A1, A2, A3};
    // the model's domain: a finite, non-negative temperature and densities
    bool dom = isfinite(Tk[c]) && Tk[c] >= 0.0 && isfinite(dens[c]) && dens[c] >= 0.0;
    double nZ = 0.0, nZ2 = 0.0, rho = 0.0, rhoH = 0.0;
    for (int s = 0; s < nion; ++s) {
        const double ni = dens[(int64_t)(1 + s) * ncell + c];
        dom = dom && isfinite(ni) && ni >= 0.0;
        nZ += Zs[s] * ni;
        nZ2 += Zs[s] * Zs[s] * ni;
        const double m = ni * As[s] * kMu;
        rho += m;
        if (Zs[s] == 1.0 && As[s] < 1.5) rhoH += m;
    }
    const LocalState L = local_state(Tk[c], dens[c], nZ, nZ2, rho, rhoH, prm);
    const double T = L.T, ne = L.ne, ne_dep = L.ne_dep, XH = L.XH, kappa2 = L.kappa2;
    const double G_P0 = L.G_P0, G_C = L.G_C, G_B = L.G_B, Q_C = L.Q_C, Q_B = L.Q_B;
    const double meanC = L.meanC, meanB = L.meanB;
    const double hc3 = kHbarcKeVcm * kHbarcKeVcm * kHbarcKeVcm;
    double* st = state + c * AXPIC_STATE_N;
    st[0] = T; st[1] = ne; st[2] = ne_dep; st[3] = nZ; st[4] = nZ2; st[5] = rho; st[6] = XH;
    st[7] = kappa2; st[8] = G_P0; st[9] = G_C; st[10] = G_B; st[11] = Q_C; st[12] = Q_B;
    st[13] = meanC; st[14] = meanB; st[15] = dom ? 0.0 : 1.0;
    const bool onP = prm.channels & AXPIC_PRIMAKOFF, onC = prm.channels & AXPIC_COMPTON,
               onB = prm.channels & AXPIC_BREMS;
    double pr[AXPIC_PREF_N];
    pr[0] = T;
    pr[1] = 4.0 * kMe * kMe / kappa2;
    pr[2] = G_P0 * dt_phys;
    pr[3] = onP ? G_P0 * dt_phys * w_ref_g / (prm.w_a * prm.wa_mul[0]) : 0.0;
    pr[4] = onC ? w_ref_e * G_C * dt_phys / (prm.w_a * prm.wa_mul[1]) : 0.0;
    pr[5] = onB ? w_ref_e * G_B * dt_phys / (prm.w_a * prm.wa_mul[2]) : 0.0;
    if (prm.m_a_keV > 0.0) {     // massive axions: only the spectrum above the mass is emitted
        if (T > 0.0) {
            pr[4] *= compton_tail(prm.m_a_keV / T);
            pr[5] *= gamma_tail(prm.brems_k, prm.m_a_keV / (prm.brems_theta * T));
        } else {
            pr[4] = pr[5] = 0.0;
        }
    }
    // detailed-balance absorption coefficients (eq. gamma_abs) times dt_phys
    const double twopi2hc3 = 2.0 * kPi * kPi * hc3;
    pr[6] = (prm.inverse && onC && T > 0.0)
                ? ne_dep * G_C * twopi2hc3 * dt_phys / (24.0 * kZeta5 * T * T * T * T * T) : 0.0;
    const double k = prm.brems_k, th = prm.brems_theta;
    pr[7] = (prm.inverse && onB && T > 0.0)
                ? ne_dep * G_B * twopi2hc3 * dt_phys / (exp(lgamma(k)) * pow(th, k) * T * T * T) : 0.0;
    if (!dom)                                   // outside the domain: nothing happens there
        for (int i = 0; i < AXPIC_PREF_N; ++i) pr[i] = 0.0;
    for (int i = 0; i < AXPIC_PREF_N; ++i) {
        p64[c * AXPIC_PREF_N + i] = pr[i];
        p32[c * AXPIC_PREF_N + i] = (float)pr[i];
    }
}

// ------------------------------------------------------------------ deposit
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_deposit(int64_t ncell, const T* __restrict__ w, const int64_t* __restrict__ off, double scale,
          double* __restrict__ dens_slot) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    double s = 0.0;
    for (int64_t i = off[c]; i < off[c + 1]; ++i) s += (double)w[i];
    dens_slot[c] = s * scale;
}

// |p|^2 of particles from .. n-1 (the cache axpic_species.p2).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fill_p2(int64_t from, int64_t n, const T* __restrict__ px, const T* __restrict__ py,
          const T* __restrict__ pz, T* __restrict__ p2) {
    const int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p2[i] = p2_of<T>(px[i], py[i], pz[i]);
}

// ------------------------------------------------------------------ bin_cells
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_bin(int64_t n, KParams kp, int push, T* __restrict__ x0, T* __restrict__ x1, T* __restrict__ x2,
      const T* __restrict__ px, const T* __restrict__ py, const T* __restrict__ pz,
      int32_t* __restrict__ cell) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T* xs[3] = {x0, x1, x2};
    T pv[3] = {px[i], py[i], pz[i]};
    T inv = (T)0;
    if (push) {
        // |p|^2 + (m/m_e)^2: the mass term makes a massive axion sub-luminal (Sec. II.B)
        const T s = dev_fma<T>(pv[2], pv[2], dev_fma<T>(pv[1], pv[1], dev_fma<T>(pv[0], pv[0], (T)kp.mu2)));
        inv = s > (T)0 ? (T)1 / dev_sqrt<T>(s) : (T)0;
    }
    const T dtdx = (T)kp.dtdx;
    int64_t c = 0, stride = 1;
    for (int d = 0; d < 3; ++d) {
        const int nd = kp.n[d];
        T x = (d < kp.ndim) ? xs[d][i] : (T)0;
        if (d < kp.ndim && push) {
            const T v = pv[d] * inv;
            x = dev_fma<T>(v, dtdx, x);
            if (x < (T)0) x = x + (T)nd;
            if (x >= (T)nd) x = x - (T)nd;
            xs[d][i] = x;
        }
        int64_t ix = (int64_t)dev_floor<T>(x);
        ix = ix < 0 ? 0 : (ix > nd - 1 ? nd - 1 : ix);
        c += ix * stride;
        stride *= nd;
    }
    cell[i] = (int32_t)c;
}

// ------------------------------------------------------------------ rates
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_rates(int64_t n, KParams kp, int mode, const float* __restrict__ p32, const double* __restrict__ p64,
        const T* __restrict__ w, const T* __restrict__ px, const T* __restrict__ py,
        const T* __restrict__ pz, const int32_t* __restrict__ cell, T* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T* pc = PrefOf<T>::get(p32, p64) + (int64_t)cell[i] * AXPIC_PREF_N;
    const T wt = w[i];
    T r = (T)0;
    if (mode == 0) {                       // photons, Primakoff
        r = wt > (T)0 ? (kp.massive ? lambda_primakoff_m<T>(kp, pc, wt, psq_d<T>(px, py, pz, i))
                                    : lambda_primakoff<T>(pc, wt, psq<T>(px, py, pz, i)))
                      : (T)0;
    } else if (mode == 1) {                // electrons, Compton
        r = wt * pc[4];
    } else if (mode == 2) {                // electrons, brems
        r = wt * pc[5];
    } else if (mode == 3) {                // axions, thermal absorption probability
        r = wt > (T)0 ? (kp.massive ? pabs_thermal_m<T>(kp, pc, psq_d<T>(px, py, pz, i))
                                    : pabs_thermal<T>(kp, pc, energy_keV(psq<T>(px, py, pz, i))))
                      : (T)0;
    } else {                               // axions, a->gamma mean
        r = wt > (T)0 ? (kp.massive ? lambda_ag_m<T>(kp, pc, wt, psq_d<T>(px, py, pz, i))
                                    : lambda_ag<T>(kp, pc, wt, psq<T>(px, py, pz, i)))
                      : (T)0;
    }
    out[i] = r;
}

// ------------------------------------------------------------------ Primakoff emission
constexpr int kStageCells = 256;   // cells a workgroup of the cell-ordered prefix stages in LDS

// What the conversion count reads besides w and id: p, the photons' |p|^2 cache
// (massless only), or given means.
enum PrimSrc { kSrcP = 0, kSrcP2 = 1, kSrcLam = 2 };

// The photon data of a thread's run (x holds |p|^2 or the means when that is the source;
// the cells only where the rate is computed).
template <typename T, int SRC>
struct PrimRun {
    T w[kPer], x[kPer], y[kPer], z[kPer];
    uint64_t id[kPer];
    int32_t c[kPer];
    template <bool VEC>
    __device__ __forceinline__ void load(int64_t i0, int64_t n, const T* __restrict__ wp,
                                         const T* __restrict__ px, const T* __restrict__ py,
                                         const T* __restrict__ pz, const T* __restrict__ p2in,
                                         const IdView& idv, const int32_t* __restrict__ cell,
                                         const T* __restrict__ lam_in) {
        ld_run<VEC>(wp, i0, n, w);
        idv.template run<VEC>(i0, n, id);
        if constexpr (SRC == kSrcLam) ld_run<VEC>(lam_in, i0, n, x);
        else if constexpr (SRC == kSrcP2) ld_run<VEC>(p2in, i0, n, x);
        else { ld_run<VEC>(px, i0, n, x); ld_run<VEC>(py, i0, n, y); ld_run<VEC>(pz, i0, n, z); }
        if constexpr (SRC != kSrcLam) ld_run<VEC>(cell, i0, n, c);
    }
};

// Counts of the thread's run of photons into cd from its data and its cells' prefactor
// records pcv; returns the run's product total.
template <typename T, bool M, int SRC, bool VEC>
__device__ __forceinline__ uint32_t prim_count_run(
    int64_t i0, int64_t n, int64_t step, const KParams& kp, double w_ref,
    const PrimRun<T, SRC>& d, const T (*pcv)[4], float wt_heavy, uint32_t* cd) {
    const T* wv = d.w; const T* xv = d.x; const T* yv = d.y; const T* zv = d.z;
    const uint64_t* idv = d.id;
    const double wprod = kp.w_a * kp.wa_mul[0];
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        cd[j] = 0;
        if (!VEC && i0 + j >= n) continue;
        const T wt = wv[j];
        T l = (T)0;
        if (wt > (T)0) {
            if constexpr (SRC == kSrcLam) l = xv[j];
            else if constexpr (M)
                l = lambda_primakoff_m<T>(kp, pcv[j], wt, p2_of<double>(xv[j], yv[j], zv[j]));
            else
                l = lambda_primakoff<T>(pcv[j], wt,
                                        SRC == kSrcP2 ? xv[j] : p2_of<T>(xv[j], yv[j], zv[j]));
        }
        int K = 0;
        if (l > (T)0) {
            const uint4 r = draw(kp, idv[j], step, 0, 0);
            // a parent surely heavier than one product with a surely-zero count skips FP64
            const bool zero = sizeof(T) == 4 && (float)wt >= wt_heavy &&
                              poisson_surely_zero((float)l, r.x);
            if (!zero) {
                double ws; int cp;
                const double le = cap_lambda((double)l, kp.cap, &ws, &cp);
                K = conversion_count(kp, (double)l, le, (double)wt * w_ref, wprod, u53(r.x, r.y));
            }
        }
        cd[j] = (uint32_t)K;
        tot += K;
    }
    return tot;
}

// The tile's totals and its list of active parents: entry = index in the tile (bits
// 0-9) | counts << 10 (channel 0 or 1 in bits 10-17, brems in 18-25), in parent order at
// list[tile start ..]; bsum / bact the tile's products and active parents.
__device__ __forceinline__ void tile_list(int64_t b, int32_t t0, uint32_t tot, const uint32_t* cd,
                                          uint32_t* __restrict__ list, uint32_t* __restrict__ bsum,
                                          uint32_t* __restrict__ bact, uint32_t* lds) {
    uint32_t na = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) na += cd[q] != 0u;
    // one scan of both: active parents in bits 0-10 (at most 1024 a tile), products
    // above (at most 2 x 255 per parent, 522240 < 2^21 a tile)
    static_assert(kBlockParents <= 1024, "tile_list packs the active count in 11 bits");
    uint32_t bp;
    const uint32_t ex = block_excl_scan(na | (tot << 11), lds, &bp);
    uint32_t slot = ex & 0x7FFu;
    const uint32_t ba = bp & 0x7FFu, bt = bp >> 11;
    if (na) {
        uint32_t* L = list + b * kBlockParents;
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (cd[q]) L[slot++] = (uint32_t)(t0 + q) | (cd[q] << 10);
    }
    if (threadIdx.x == 0) { bsum[b] = bt; bact[b] = ba; }
}

template <typename T, bool M, int SRC>
__global__ void __launch_bounds__(kThreads)
k_prim_count(int64_t n, int64_t step, KParams kp, double w_ref, const float* __restrict__ p32,
             const double* __restrict__ p64, const T* __restrict__ w, const T* __restrict__ px,
             const T* __restrict__ py, const T* __restrict__ pz, const T* __restrict__ p2in,
             IdView id, const int32_t* __restrict__ cell, const T* __restrict__ lam_in,
             uint32_t* __restrict__ list, uint32_t* __restrict__ bsum, uint32_t* __restrict__ bact,
             int aligned, float wt_heavy,
             const int64_t* __restrict__ off, int64_t n_sorted) {
    __shared__ uint32_t lds[kThreads / 64];
    __shared__ float4 s_pref[kStageCells];
    const T* pref = PrefOf<T>::get(p32, p64);
    const int64_t base = (int64_t)blockIdx.x * kBlockParents;
    // each thread takes kPer consecutive parents (the workgroup covers the same
    // kBlockParents as the expand pass); all loads first, then the arithmetic
    const int64_t i0 = base + (int64_t)kPer * threadIdx.x;
    const int32_t t0 = kPer * (int32_t)threadIdx.x;
    const bool vec = aligned && base + kBlockParents <= n;
    // the run's own loads first: they are in flight while the cells are staged
    PrimRun<T, SRC> d;
    if (vec) d.template load<true>(i0, n, w, px, py, pz, p2in, id, cell, lam_in);
    else d.template load<false>(i0, n, w, px, py, pz, p2in, id, cell, lam_in);
    // A workgroup inside the cell-ordered prefix spans the cells of its first and last
    // photon; when they are few, their first prefactor records go to LDS, indexed by the
    // photon's cell relative to the first (the kernel is bound by instruction issue, so
    // the 4-byte cell read is cheaper than finding the cells from the offsets)
    int32_t c_first = 0, m = 0;
    if (sizeof(T) == 4 && SRC != kSrcLam && off && vec && base + kBlockParents <= n_sorted) {
        c_first = cell[base];
        const int32_t mm = cell[base + kBlockParents - 1] - c_first + 1;
        if (mm >= 1 && mm <= kStageCells) {
            for (int t = threadIdx.x; t < mm; t += kThreads)
                s_pref[t] = *(const float4*)(p32 + (int64_t)(c_first + t) * AXPIC_PREF_N);
            __syncthreads();
            m = mm;
        }
    }
    T pcv[kPer][4];
    if (m > 0) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const float4 v = s_pref[d.c[j] - c_first];
            pcv[j][0] = v.x; pcv[j][1] = v.y; pcv[j][2] = v.z; pcv[j][3] = v.w;
        }
    } else if (SRC != kSrcLam) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) load_pref(pref + (int64_t)d.c[j] * AXPIC_PREF_N, pcv[j], 1);
    }
    uint32_t cd[kPer], tot;
    if (vec) tot = prim_count_run<T, M, SRC, true>(i0, n, step, kp, w_ref, d, pcv, wt_heavy, cd);
    else tot = prim_count_run<T, M, SRC, false>(i0, n, step, kp, w_ref, d, pcv, wt_heavy, cd);
    tile_list(blockIdx.x, t0, tot, cd, list, bsum, bact, lds);
}

// Event records: the expand pass writes one record per product into the product's id
// slot -- parent index (bits 0-39), event k (40-47), channel (48-55: 0 Primakoff, 1
// Compton, 2 brems), the parent's count in that channel (56-63) -- and the event kernels,
// one product per lane, replace it with the final id after filling the product.
constexpr uint64_t kRecParentMask = (1ull << 40) - 1;

// One wavefront per tile (grid-stride over the tiles): the tile's active-parent entries,
// 64 at a time, a wavefront scan of their event counts, the records from the tile's
// product offset on.
__global__ void __launch_bounds__(kThreads)
k_expand(int64_t nb, int thermal, const uint32_t* __restrict__ list,
         const uint32_t* __restrict__ bact, const uint64_t* __restrict__ boff,
         const int64_t* __restrict__ ctrl, int64_t out_cap, uint64_t* __restrict__ rec) {
    if (ctrl[0]) return;
    const int64_t out_n = ctrl[2];
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); t < nb; t += nw) {
        const uint32_t na = bact[t];                       // wave-uniform
        int64_t slot0 = out_n + (int64_t)boff[t];
        const uint32_t* L = list + t * kBlockParents;
        for (uint32_t c = 0; c < na; c += 64) {
            const uint32_t e = c + lane < na ? L[c + lane] : 0u;
            const uint32_t K0 = (e >> 10) & 0xFFu, K1 = thermal ? (e >> 18) & 0xFFu : 0u;
            const uint32_t inc = wave_incl_scan(K0 + K1, lane);
            int64_t slot = slot0 + (int64_t)(inc - K0 - K1);
            const uint64_t i = (uint64_t)(t * kBlockParents + (int64_t)(e & 0x3FFu));
            const uint64_t h0 = i | ((uint64_t)(thermal ? 1 : 0) << 48) | ((uint64_t)K0 << 56);
            for (uint32_t k = 0; k < K0; ++k, ++slot)
                if (slot < out_cap) rec[slot] = h0 | ((uint64_t)k << 40);
            const uint64_t h1 = i | (2ull << 48) | ((uint64_t)K1 << 56);
            for (uint32_t k = 0; k < K1; ++k, ++slot)
                if (slot < out_cap) rec[slot] = h1 | ((uint64_t)k << 40);
            slot0 += (int64_t)__shfl(inc, 63, 64);
        }
    }
}

// One thread per converting photon: the thread that meets the parent's first
// event record writes the positions, momenta, weights and cells of all K
// products (contiguous slots) and depletes the parent, so no other thread
// reads a weight while it changes.  Every thread replaces only its own
// slot's record by the final id: a record is never overwritten before the
// thread that owns it has read it.
template <typename T, bool M>
__global__ void __launch_bounds__(kThreads)
k_prim_events(int64_t n, int64_t step, uint64_t next_id, KParams kp, double w_ref_g,
              const float* __restrict__ p32, const double* __restrict__ p64, T* __restrict__ w,
              const T* __restrict__ x0, const T* __restrict__ x1, const T* __restrict__ x2,
              const T* __restrict__ px, const T* __restrict__ py, const T* __restrict__ pz,
              const int32_t* __restrict__ cell, const T* __restrict__ lam_in,
              const int64_t* __restrict__ ctrl, int64_t out_n,
              T* __restrict__ ax0, T* __restrict__ ax1, T* __restrict__ ax2, T* __restrict__ apx,
              T* __restrict__ apy, T* __restrict__ apz, T* __restrict__ aw,
              uint64_t* __restrict__ aid, int32_t* __restrict__ acell, double* __restrict__ rec,
              StatMap smap) {
    extern __shared__ double wh[];                          // per wavefront: channel 0's bins
    __shared__ double lst[(kThreads / 64) * kStatSlots];
    if (ctrl[0]) return;
    out_n = ctrl[2];
    next_id = (uint64_t)ctrl[3];
    const int64_t total = ctrl[1];
    int64_t lo, hi;
    ev_range(total, &lo, &hi);
    if (lo >= hi) return;                 // no events: no record (the reduction skips it)
    const T* pref = PrefOf<T>::get(p32, p64);
    const int nbh = kp.nbins + 2;
    for (int k = threadIdx.x; k < (kThreads / 64) * nbh; k += kThreads) wh[k] = 0.0;
    __syncthreads();
    double* myh = wh + (threadIdx.x >> 6) * nbh;
    double st[kStatSlots];
    for (int s = 0; s < kStatSlots; ++s) st[s] = 0.0;
    for (int64_t t0 = lo; t0 < hi; t0 += kThreads) {
        const int64_t e = t0 + threadIdx.x;
        int bin = -1;
        double hv = 0.0;
        // the parent's first event writes its K products
        const uint64_t rc = e < hi ? aid[out_n + e] : 0ull;
        if (e < hi) aid[out_n + e] = (next_id + (uint64_t)e) | (1ull << 63);
        const int64_t i = (int64_t)(rc & kRecParentMask);
        const uint32_t K = (uint32_t)(rc >> 56);
        if (e < hi && ((rc >> 40) & 0xFFu) == 0 && i < n && (int64_t)K <= total - e) {
            const T wt = w[i];
            const T* pci = pref + (int64_t)cell[i] * AXPIC_PREF_N;
            const T l = lam_in ? lam_in[i]
                               : (M ? lambda_primakoff_m<T>(kp, pci, wt, psq_d<T>(px, py, pz, i))
                                    : lambda_primakoff<T>(pci, wt, psq<T>(px, py, pz, i)));
            double ws; int cp;
            (void)cap_lambda((double)l, kp.cap, &ws, &cp);
            double wp = kp.w_a * kp.wa_mul[0] * ws;            // physical product weight
            const double wpar = w_ref_g * (double)wt;
            double dep = (double)K * wp;
            const bool over = dep > wpar;
            if (over) { wp = wpar / (double)K; dep = wpar; }
            T pxv = px[i], pyv = py[i], pzv = pz[i];
            const double E = kMe * sqrt((double)pxv * pxv + (double)pyv * pyv + (double)pzv * pzv);
            if (M) {              // the axion keeps the photon's energy: |p| = sqrt(E^2 - m^2)
                const double sc = E > kp.m_a ? sqrt((E - kp.m_a) * (E + kp.m_a)) / E : 0.0;
                pxv = (T)((double)pxv * sc); pyv = (T)((double)pyv * sc); pzv = (T)((double)pzv * sc);
            }
            const T xv0 = x0[i], xv1 = x1 ? x1[i] : (T)0, xv2 = x2 ? x2[i] : (T)0;
            const T wrel = (T)(wp / kp.w_a);
            const int32_t c = cell[i];
            for (uint32_t k = 0; k < K; ++k) {
                const int64_t slot = out_n + e + k;
                ax0[slot] = xv0;
                if (ax1) ax1[slot] = xv1;
                if (ax2) ax2[slot] = xv2;
                apx[slot] = pxv; apy[slot] = pyv; apz[slot] = pzv;
                aw[slot] = wrel;
                acell[slot] = c;
            }
            bin = hist_bin(kp, E);
            hv = (double)K * wp * E;
            st[0] += (double)K; st[3] += (double)K * wp; st[6] += (double)K * wp * E;
            st[9] += cp ? 1.0 : 0.0;
            st[10] += over ? 1.0 : 0.0;
            w[i] = (dep >= wpar) ? (T)0 : (T)((wpar - dep) / w_ref_g);
        }
        wave_hist_add(myh, bin, hv);
    }
    __syncthreads();
    rec_write(wh, nbh, st, smap, lst, rec + blockIdx.x, kEventBlocks);
}

// ------------------------------------------------------------------ thermal emission
// Compton-like and brems counts of the thread's run of electrons into cd (Compton in
// bits 0-7, brems in 8-15); returns the run's product total.
template <typename T, bool VEC>
__device__ __forceinline__ uint32_t therm_count_run(
    int64_t i0, int64_t n, int64_t step, const KParams& kp, const T* __restrict__ pref,
    const T* __restrict__ w, const IdView& id, const int32_t* __restrict__ cell,
    const T* __restrict__ lam_in, bool lam_b_vec, uint32_t* cd) {
    const bool onC = kp.channels & AXPIC_COMPTON, onB = kp.channels & AXPIC_BREMS;
    T lCv[kPer], lBv[kPer];
    uint64_t idv[kPer];
    id.template run<VEC>(i0, n, idv);
    if (lam_in) {
        ld_run<VEC>(lam_in, i0, n, lCv);
        if (VEC && lam_b_vec) ld_run<true>(lam_in + n, i0, n, lBv);
        else ld_run<false>(lam_in + n, i0, n, lBv);
    } else {
        T wv[kPer];
        int32_t cv[kPer];
        ld_run<VEC>(w, i0, n, wv);
        ld_run<VEC>(cell, i0, n, cv);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const T* pc = pref + (int64_t)cv[j] * AXPIC_PREF_N;
            lCv[j] = wv[j] * pc[4];
            lBv[j] = wv[j] * pc[5];
        }
    }
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        cd[j] = 0;
        if (!VEC && i0 + j >= n) continue;
        T lC = lCv[j], lB = lBv[j];
        if (!onC) lC = (T)0;
        if (!onB) lB = (T)0;
        int KC = 0, KB = 0;
        if (lC > (T)0 || lB > (T)0) {
            const uint4 r = draw(kp, idv[j], step, 1, 0);
            // both counts surely zero: no FP64 inversion
            const bool zero = sizeof(T) == 4 && (poisson_surely_zero((float)lC, r.x) &
                                                 poisson_surely_zero((float)lB, r.z));
            if (!zero) {
                double ws; int cp;
                KC = poisson_inv(cap_lambda((double)lC, kp.cap, &ws, &cp), u53(r.x, r.y));
                KB = poisson_inv(cap_lambda((double)lB, kp.cap, &ws, &cp), u53(r.z, r.w));
            }
        }
        cd[j] = (uint32_t)(KC | (KB << 8));
        tot += KC + KB;
    }
    return tot;
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_therm_count(int64_t n, int64_t step, KParams kp, const float* __restrict__ p32,
              const double* __restrict__ p64, const T* __restrict__ w,
              IdView id, const int32_t* __restrict__ cell,
              const T* __restrict__ lam_in, uint32_t* __restrict__ list,
              uint32_t* __restrict__ bsum, uint32_t* __restrict__ bact,
              int aligned) {
    __shared__ uint32_t lds[kThreads / 64];
    const T* pref = PrefOf<T>::get(p32, p64);
    const int64_t base = (int64_t)blockIdx.x * kBlockParents;
    const int64_t i0 = base + (int64_t)kPer * threadIdx.x;
    // the brems half of lam_in starts at n: 16-byte aligned runs only if n % kPer == 0
    const bool lam_b_vec = (n % kPer) == 0;
    uint32_t cd[kPer], tot;
    if (aligned && base + kBlockParents <= n)
        tot = therm_count_run<T, true>(i0, n, step, kp, pref, w, id, cell, lam_in, lam_b_vec, cd);
    else
        tot = therm_count_run<T, false>(i0, n, step, kp, pref, w, id, cell, lam_in, lam_b_vec, cd);
    tile_list(blockIdx.x, kPer * (int32_t)threadIdx.x, tot, cd, list, bsum, bact, lds);
}

template <typename T, bool M>
__global__ void __launch_bounds__(kThreads)
k_therm_events(int64_t n, int64_t step, uint64_t next_id, KParams kp,
               const float* __restrict__ p32, const double* __restrict__ p64,
               const double* __restrict__ state, const T* __restrict__ w, const T* __restrict__ x0,
               const T* __restrict__ x1, const T* __restrict__ x2, IdView id,
               const int32_t* __restrict__ cell, const T* __restrict__ lam_in,
               const int64_t* __restrict__ ctrl, int64_t out_n, T* __restrict__ ax0,
               T* __restrict__ ax1, T* __restrict__ ax2, T* __restrict__ apx, T* __restrict__ apy,
               T* __restrict__ apz, T* __restrict__ aw, uint64_t* __restrict__ aid,
               int32_t* __restrict__ acell, double* __restrict__ fb, double* __restrict__ rec,
               int32_t* __restrict__ bkey, double* __restrict__ bval, StatMap smap) {
    extern __shared__ double wh[];                          // per wavefront: channels 1, 2
    __shared__ double lst[(kThreads / 64) * kStatSlots];
    __shared__ FbStitch fbs;
    if (ctrl[0]) return;
    out_n = ctrl[2];
    next_id = (uint64_t)ctrl[3];
    const int64_t total = ctrl[1];
    int64_t lo, hi;
    ev_range(total, &lo, &hi);
    if (lo >= hi) return;                 // no events: no records (the reductions skip them)
    const T* pref = PrefOf<T>::get(p32, p64);
    const int nbh = kp.nbins + 2;
    const int H = 2 * nbh;
    for (int k = threadIdx.x; k < (kThreads / 64) * H; k += kThreads) wh[k] = 0.0;
    __syncthreads();
    double* myh = wh + (threadIdx.x >> 6) * H;
    double st[kStatSlots];
    for (int s = 0; s < kStatSlots; ++s) st[s] = 0.0;
    FbOpen open;
    for (int64_t t0 = lo; t0 < hi; t0 += kThreads) {
        const int64_t e = t0 + threadIdx.x;
        const int64_t slot = out_n + e;
        const uint64_t rc = e < hi ? aid[slot] : 0ull;
        const int64_t i = (int64_t)(rc & kRecParentMask);
        const uint32_t k = (uint32_t)((rc >> 40) & 0xFFu);
        const int ch = (int)((rc >> 48) & 0xFFu);          // 1 Compton, 2 brems
        int bin = -1;
        double hv = 0.0;
        int32_t key = -1;                                   // the product's cell
        double fv[4] = {0.0, 0.0, 0.0, 0.0};
        if (e < hi && i < n && (ch == 1 || ch == 2)) {      // always, for a well-formed record
            const int32_t c = cell[i];
            const T* pc = pref + (int64_t)c * AXPIC_PREF_N;
            const double Tc = state[(int64_t)c * AXPIC_STATE_N + 0];
            const T l = lam_in ? lam_in[(int64_t)(ch - 1) * n + i] : w[i] * pc[3 + ch];
            double ws; int cp;
            (void)cap_lambda((double)l, kp.cap, &ws, &cp);
            const double wp = kp.w_a * kp.wa_mul[ch] * ws;
            const double* tab = ch == 1 ? g_tab_compton : g_tab_gamma;
            const uint4 r = draw(kp, id(i), step, 1 + ch, k);
            double E, pm;
            thermal_energy<M>(kp, ch, Tc, u24(r.x), tab, &E, &pm);
            const double eu = M ? E / kMe : pm;            // energy in m_e c^2
            const double mu = 2.0 * u24(r.y) - 1.0;
            const double phi = 2.0 * kPi * u24(r.z);
            const double sn = sqrt(fmax(0.0, 1.0 - mu * mu));
            double sphi, cphi;
            sincos(phi, &sphi, &cphi);
            const double pa[3] = {pm * sn * cphi, pm * sn * sphi, pm * mu};
            ax0[slot] = x0[i];
            if (ax1) ax1[slot] = x1 ? x1[i] : (T)0;
            if (ax2) ax2[slot] = x2 ? x2[i] : (T)0;
            apx[slot] = (T)pa[0]; apy[slot] = (T)pa[1]; apz[slot] = (T)pa[2];
            aw[slot] = (T)(kp.wa_mul[ch] * ws);
            aid[slot] = (next_id + (uint64_t)e) | (1ull << 63);
            acell[slot] = c;
            bin = (ch - 1) * nbh + hist_bin(kp, E);
            hv = wp * E;
            key = c;
            fv[0] = -wp * eu; fv[1] = -wp * pa[0]; fv[2] = -wp * pa[1]; fv[3] = -wp * pa[2];
            st[ch] += 1.0; st[3 + ch] += wp; st[6 + ch] += wp * E;
            if (k == 0) st[9] += cp ? 1.0 : 0.0;
        }
        wave_hist_add(myh, bin, hv);
        if (fb) fb_tile(fbs, open, key, fv, fb, bkey, bval, blockIdx.x);
    }
    if (fb) fb_finish(open, fb, bkey, bval, blockIdx.x);
    __syncthreads();
    rec_write(wh, H, st, smap, lst, rec + blockIdx.x, kEventBlocks);
}

// ------------------------------------------------------------------ absorption
// The a->gamma mean of an axion (Sec. II.F.1, eq. prim_prob): that of its start-of-step
// weight wt0 (computed, or handed in as lam), times (1 - P_abs) after a weight reduction
// (reading O8), which is the mean of the reduced weight; FP64 so that the handed-in and
// the computed forms give the same value.
template <typename T, bool M>
__device__ __forceinline__ double ag_mean(const KParams& kp, const T* __restrict__ pc, T lam,
                                          bool given, T wt0, T p2, double p2d, T P) {
    double l = given ? (double)lam
                     : (double)(M ? lambda_ag_m<T>(kp, pc, wt0, p2d) : lambda_ag<T>(kp, pc, wt0, p2));
    if (kp.absorb_mode == 1) l = l * (1.0 - (double)P);
    return l;
}

// Decisions for the thread's run of axions; returns the run's photon total, *act the
// axions with a nonzero code.
template <typename T, bool M, bool VEC>
__device__ __forceinline__ uint32_t abs_count_run(
    int64_t i0, int64_t n, int64_t step, const KParams& kp, double w_ref_a, const T* __restrict__ pref,
    const T* __restrict__ w, const T* __restrict__ px, const T* __restrict__ py,
    const T* __restrict__ pz, const IdView& id, const int32_t* __restrict__ cell,
    const T* __restrict__ pabs_in, const T* __restrict__ lam_in, uint16_t* __restrict__ code,
    float wt_heavy, float wt_light, float prod_ratio, const float4* __restrict__ stage,
    int32_t c_first, int32_t m_stage, uint32_t* act) {
    const bool thermal = kp.inverse && (kp.channels & (AXPIC_COMPTON | AXPIC_BREMS));
    const bool a2g = kp.inverse && (kp.channels & AXPIC_PRIMAKOFF);
    T wv[kPer], xv[kPer], yv[kPer], zv[kPer], Pv[kPer], lv[kPer];
    int32_t cv[kPer];
    uint64_t idv[kPer];
    ld_run<VEC>(w, i0, n, wv);
    ld_run<VEC>(px, i0, n, xv);
    ld_run<VEC>(py, i0, n, yv);
    ld_run<VEC>(pz, i0, n, zv);
    ld_run<VEC>(cell, i0, n, cv);
    id.template run<VEC>(i0, n, idv);
    if (pabs_in) ld_run<VEC>(pabs_in, i0, n, Pv);
    if (lam_in) ld_run<VEC>(lam_in, i0, n, lv);
    T pcv[kPer][AXPIC_PREF_N];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int32_t r = cv[j] - c_first;
        if (sizeof(T) == 4 && stage && r >= 0 && r < m_stage) {   // the tile's records, in LDS
            const float4 a = stage[2 * r], b = stage[2 * r + 1];
            pcv[j][0] = a.x; pcv[j][1] = a.y; pcv[j][2] = a.z; pcv[j][3] = a.w;
            pcv[j][4] = b.x; pcv[j][5] = b.y; pcv[j][6] = b.z; pcv[j][7] = b.w;
        } else {
            load_pref(pref + (int64_t)cv[j] * AXPIC_PREF_N, pcv[j], 2);
        }
    }
    uint32_t cdv[kPer], tot = 0, nact = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        cdv[j] = 0;
        if (!VEC && i0 + j >= n) continue;
        const T wt0 = wv[j];
        T wt = wt0;
        uint32_t cd = 0;
        if (wt > (T)0) {
            const T* pc = pcv[j];
            const T p2 = p2_of<T>(xv[j], yv[j], zv[j]);
            const double p2d = p2_of<double>(xv[j], yv[j], zv[j]);
            const uint4 r = draw(kp, idv[j], step, 4, 0);
            T P = (T)0;
            if (thermal) {
                P = pabs_in ? Pv[j]
                            : (M ? pabs_thermal_m<T>(kp, pc, p2d)
                                 : pabs_thermal<T>(kp, pc, energy_keV(p2)));
                if (kp.absorb_mode == 0) {
                    // u53 < P is decided by the leading 24 bits of u unless P falls
                    // between their bounds
                    bool absorbed;
                    if (sizeof(T) == 4 && u_lo24(r.x) >= (float)P) absorbed = false;
                    else if (sizeof(T) == 4 && u_hi24(r.x) <= (float)P) absorbed = true;
                    else absorbed = u53(r.x, r.y) < (double)P;
                    if (absorbed) { cd |= 256u; wt = (T)0; }
                } else {
                    wt = (T)((double)wt - (double)wt * (double)P);
                }
            }
            if (a2g && wt > (T)0) {
                const double l = ag_mean<T, M>(kp, pc, lam_in ? lv[j] : (T)0, lam_in != nullptr,
                                               wt0, p2, p2d, thermal ? P : (T)0);
                // surely heavy with a surely-zero count, or surely light and surely not
                // converting: no FP64
                const bool zero =
                    sizeof(T) == 4 && l > 0.0 &&
                    (((float)wt >= wt_heavy && poisson_surely_zero((float)l, r.z)) ||
                     ((float)wt < wt_light && light_surely_zero((float)l, prod_ratio, (float)wt, r.z)));
                if (!zero) {
                    double ws; int cp;
                    cd |= (uint32_t)conversion_count(kp, l, cap_lambda(l, kp.cap, &ws, &cp),
                                                     (double)wt * w_ref_a, kp.w_gamma_prod,
                                                     u53(r.z, r.w));
                }
            }
        }
        cdv[j] = cd;
        tot += cd & 0xFFu;
        nact += cd != 0;
    }
    st_codes<VEC>(code, i0, n, cdv);
    *act = nact;
    return tot;
}

// code: bits 0-7 a->gamma count, bit 8 absorbed (deletion mode)
template <typename T, bool M>
__global__ void __launch_bounds__(kThreads)
k_abs_count(int64_t n, int64_t step, KParams kp, double w_ref_a, const float* __restrict__ p32,
            const double* __restrict__ p64, const T* __restrict__ w, const T* __restrict__ px,
            const T* __restrict__ py, const T* __restrict__ pz, IdView id,
            const int32_t* __restrict__ cell, const T* __restrict__ pabs_in,
            const T* __restrict__ lam_in, uint16_t* __restrict__ code, uint32_t* __restrict__ bsum,
            uint32_t* __restrict__ bact, int aligned,
            float wt_heavy, float wt_light, float prod_ratio, int64_t n_sorted,
            const int64_t* __restrict__ chain) {
    __shared__ uint32_t lds[kThreads / 64];
    __shared__ float4 s_pref[2 * kStageCells];
    if (chain) n = min(n, chain[AXPIC_CHAIN_AX_START]);   // the axions of the step's start
    const T* pref = PrefOf<T>::get(p32, p64);
    const bool thermal = kp.inverse && (kp.channels & (AXPIC_COMPTON | AXPIC_BREMS));
    const int64_t base = (int64_t)blockIdx.x * kBlockParents;
    const int64_t i0 = base + (int64_t)kPer * threadIdx.x;
    const bool vec = aligned && base + kBlockParents <= n;
    // a tile inside the cell-ordered prefix spans the cells of its first and last axion:
    // when they are few, their prefactor records go to LDS (one read per cell)
    const float4* stage = nullptr;
    int32_t c_first = 0, m_stage = 0;
    if (sizeof(T) == 4 && vec && base + kBlockParents <= n_sorted) {
        c_first = cell[base];
        const int32_t m = cell[base + kBlockParents - 1] - c_first + 1;
        if (m >= 1 && m <= kStageCells) {
            for (int t = threadIdx.x; t < 2 * m; t += kThreads)
                s_pref[t] = ((const float4*)(p32 + (int64_t)c_first * AXPIC_PREF_N))[t];
            __syncthreads();
            stage = s_pref;
            m_stage = m;
        }
    }
    uint32_t tot, act;
    if (vec)
        tot = abs_count_run<T, M, true>(i0, n, step, kp, w_ref_a, pref, w, px, py, pz, id, cell,
                                        pabs_in, lam_in, code, wt_heavy, wt_light, prod_ratio,
                                        stage, c_first, m_stage, &act);
    else
        tot = abs_count_run<T, M, false>(i0, n, step, kp, w_ref_a, pref, w, px, py, pz, id, cell,
                                         pabs_in, lam_in, code, wt_heavy, wt_light, prod_ratio,
                                         nullptr, 0, 0, &act);
    const uint32_t bt = block_sum_u32(tot, lds);
    const uint32_t ba = block_sum_u32(act, lds);
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = bt;
        // in weight-reduction mode every block with live axions must be applied
        bact[blockIdx.x] = (kp.absorb_mode == 1 && thermal) ? 1u + ba : ba;
    }
}

template <typename T, bool M>
__global__ void __launch_bounds__(kThreads)
k_abs_apply(int64_t n, int64_t step, uint64_t next_id, KParams kp, double w_ref_a,
            const float* __restrict__ p32, const double* __restrict__ p64, T* __restrict__ w,
            const T* __restrict__ x0, const T* __restrict__ x1, const T* __restrict__ x2,
            const T* __restrict__ px, const T* __restrict__ py, const T* __restrict__ pz,
            const int32_t* __restrict__ cell, const T* __restrict__ pabs_in,
            const T* __restrict__ lam_in, const uint16_t* __restrict__ code,
            const uint32_t* __restrict__ bact, const uint64_t* __restrict__ boff,
            const int64_t* __restrict__ ctrl, int64_t out_n, int64_t out_cap, T* __restrict__ gx0,
            T* __restrict__ gx1, T* __restrict__ gx2, T* __restrict__ gpx, T* __restrict__ gpy,
            T* __restrict__ gpz, T* __restrict__ gp2, T* __restrict__ gw, uint64_t* __restrict__ gid,
            int32_t* __restrict__ gcell, double w_ref_g, double* __restrict__ fb,
            double* __restrict__ rec, int32_t* __restrict__ bkey, double* __restrict__ bval,
            int det, const int64_t* __restrict__ chain, StatMap smap) {
    __shared__ uint32_t lds[kThreads / 64];
    __shared__ double lst[(kThreads / 64) * kStatSlots];
    __shared__ FbStitch fbs;
    if (ctrl[0]) return;
    if (chain) n = min(n, chain[AXPIC_CHAIN_AX_START]);
    const int64_t base = (int64_t)blockIdx.x * kBlockParents;
    double* myrec = rec + blockIdx.x;                  // column-major: nb records
    const bool fixed = det && fb;       // fb in fixed order: the axions are in cell order
    if (bact[blockIdx.x] == 0) {        // nothing to apply: a zero record and boundary cells
        for (int k = threadIdx.x; k < AXPIC_ST_COUNT; k += kThreads) myrec[k * gridDim.x] = 0.0;
        if (fixed && threadIdx.x == 0) {
            const int64_t last = (base + kBlockParents < n ? base + kBlockParents : n) - 1;
            bkey[2 * blockIdx.x] = base < n ? cell[base] : -1;
            bkey[2 * blockIdx.x + 1] = base < n ? cell[last] : -1;
            for (int q = 0; q < 8; ++q) bval[8 * blockIdx.x + q] = 0.0;
        }
        return;
    }
    out_n = ctrl[2];
    next_id = (uint64_t)ctrl[3];
    const T* pref = PrefOf<T>::get(p32, p64);
    const bool thermal = kp.inverse && (kp.channels & (AXPIC_COMPTON | AXPIC_BREMS));
    double st[kStatSlots];
    for (int s = 0; s < kStatSlots; ++s) st[s] = 0.0;
    FbOpen open;
    uint64_t run = boff[blockIdx.x];
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = base + j * kThreads + threadIdx.x;
        const uint32_t cd = (i < n) ? code[i] : 0u;
        const uint32_t K = cd & 0xFFu;
        uint32_t segtot;
        const uint32_t pre = block_excl_scan(K, lds, &segtot);
        const bool live = i < n && w[i] > (T)0;
        double fv[4] = {0.0, 0.0, 0.0, 0.0};
        if (live && (cd != 0 || (thermal && kp.absorb_mode == 1))) {
            const T wt0 = w[i];
            T wt = wt0;
            const int32_t c = cell[i];
            const T* pc = pref + (int64_t)c * AXPIC_PREF_N;
            const T pxv = px[i], pyv = py[i], pzv = pz[i];
            const T p2 = p2_of<T>(pxv, pyv, pzv);
            const double pp = psq_d<T>(px, py, pz, i);
            const double pm = sqrt(pp);
            const double E = M ? axion_energy(kp, pp) : kMe * pm;
            const double eu = M ? E / kMe : pm;                // energy in m_e c^2
            double wphys = w_ref_a * (double)wt;
            T P = (T)0;
            if (thermal) {
                double dw = 0.0;
                if (kp.absorb_mode == 1)
                    P = pabs_in ? pabs_in[i]
                                : (M ? pabs_thermal_m<T>(kp, pc, pp)
                                     : pabs_thermal<T>(kp, pc, energy_keV(p2)));
                if (cd & 256u) dw = wphys;
                else if (kp.absorb_mode == 1) {
                    dw = wphys * (double)P;
                    wt = (T)((wphys - dw) / w_ref_a);
                }
                if (dw > 0.0) {
                    fv[0] = dw * eu; fv[1] = dw * (double)pxv;
                    fv[2] = dw * (double)pyv; fv[3] = dw * (double)pzv;
                    if (fb && !fixed) {
                        double* f = fb + (int64_t)c * 4;
                        for (int q = 0; q < 4; ++q) atomicAdd(&f[q], fv[q]);
                    }
                    st[0] += dw; st[1] += dw * E;
                    if (cd & 256u) st[7] += 1.0;
                }
                if (cd & 256u) wt = (T)0;
                wphys = w_ref_a * (double)wt;
            }
            if (K > 0) {
                const double l = ag_mean<T, M>(kp, pc, lam_in ? lam_in[i] : (T)0,
                                               lam_in != nullptr, wt0, p2, pp, P);
                double ws; int cp;
                (void)cap_lambda(l, kp.cap, &ws, &cp);
                st[5] += cp ? 1.0 : 0.0;
                double wp = kp.w_gamma_prod * ws;
                double dep = (double)K * wp;
                if (dep > wphys) { wp = wphys / (double)K; dep = wphys; st[6] += 1.0; }
                const T wrel = (T)(wp / w_ref_g);
                T gxv = pxv, gyv = pyv, gzv = pzv;
                if (M) {          // the photon takes the axion's energy: |p_gamma| = E / m_e
                    const double sc = pm > 0.0 ? E / (kMe * pm) : 0.0;
                    gxv = (T)((double)pxv * sc); gyv = (T)((double)pyv * sc); gzv = (T)((double)pzv * sc);
                }
                for (uint32_t k = 0; k < K; ++k) {
                    const uint64_t rank = run + pre + k;
                    const int64_t slot = out_n + (int64_t)rank;
                    if (slot < out_cap) {
                        gx0[slot] = x0 ? x0[i] : (T)0;
                        if (gx1) gx1[slot] = x1 ? x1[i] : (T)0;
                        if (gx2) gx2[slot] = x2 ? x2[i] : (T)0;
                        gpx[slot] = gxv; gpy[slot] = gyv; gpz[slot] = gzv;
                        if (gp2) gp2[slot] = p2_of<T>(gxv, gyv, gzv);
                        gw[slot] = wrel;
                        gid[slot] = (next_id + rank) | (1ull << 63);
                        gcell[slot] = c;
                    }
                }
                st[2] += (double)K; st[3] += (double)K * wp; st[4] += (double)K * wp * E;
                wt = (dep >= wphys) ? (T)0 : (T)((wphys - dep) / w_ref_a);
            }
            w[i] = wt;
        }
        if (fixed) fb_tile(fbs, open, i < n ? cell[i] : -1, fv, fb, bkey, bval, blockIdx.x);
        run += segtot;
    }
    if (fixed) fb_finish(open, fb, bkey, bval, blockIdx.x);
    rec_write(nullptr, 0, st, smap, lst, myrec, gridDim.x);
}

// ------------------------------------------------------------------ feedback
// A wavefront takes 64 consecutive cells, finds those with work (an exchange, or every
// cell when T evolves or the moments are requested) and works on them 64 / L at a time,
// L lanes per cell (16, or 8 where the cells hold fewer electrons): FP64 moments by
// strided loads and an L-lane shuffle reduction, then the affine remap and the
// temperature update of each cell.  Cells without work cost one record read.
constexpr int kCellLanes = 16;
constexpr int kFbCache = 4;            // electrons per lane kept in registers

template <int L>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double group_sum16(double v) { return group_sum<16>(v); }

template <typename T, int L>
__global__ void __launch_bounds__(kThreads)
k_feedback(int64_t ncell, KParams kp, double w_ref, const int64_t* __restrict__ off,
           const T* __restrict__ w, T* __restrict__ px, T* __restrict__ py, T* __restrict__ pz,
           const double* __restrict__ fb, double* __restrict__ Tk, double* __restrict__ moments,
           double* __restrict__ stats, double* __restrict__ ecell, int64_t* __restrict__ flag,
           int64_t token, unsigned int* __restrict__ done, const int64_t* __restrict__ chain) {
    __shared__ uint8_t s_act[kThreads];            // per wavefront: its cells with work, in order
    // a chained step whose appending calls were skipped after an overflow is repeated
    // whole: the feedback of its partial exchange must not be applied
    if (chain && chain[AXPIC_CHAIN_SKIP]) return;
    constexpr int G = 64 / L;                      // cells worked on at once
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, sub = lane & (L - 1);
    const int64_t cw = ((int64_t)blockIdx.x * (kThreads / 64) + wave) * 64;
    // the energy a cold or clamped cell leaves unapplied goes to its own slot (0 for every
    // other cell) and the call's token to *flag; k_fb_unapplied then sums the slots in
    // cell order.  The cell counts are exact in any order.
    if (ecell && blockIdx.x == 0 && threadIdx.x == 0) *done = 0u;   // for k_fb_unapplied
    int nact;
    {
        const int64_t c = cw + lane;
        bool work = false;
        if (c < ncell) {
            if (moments || kp.T_mode == 2) work = true;
            else if (fb) {
                const double* f = fb + c * 4;
                work = f[0] != 0.0 || f[1] != 0.0 || f[2] != 0.0 || f[3] != 0.0;
            }
            if (ecell && !work) ecell[c] = 0.0;
        }
        const uint64_t m = __ballot(work);
        nact = __popcll(m);
        if (work) s_act[wave * 64 + __popcll(m & ((1ull << lane) - 1ull))] = (uint8_t)lane;
    }
    __syncthreads();
    for (int k0 = 0; k0 < nact; k0 += G) {
        const int k = k0 + lane / L;
        const bool work = k < nact;
        const int64_t c = work ? cw + s_act[wave * 64 + k] : 0;
        const double* f = (fb && work) ? fb + c * 4 : nullptr;
        const double dE = f ? f[0] : 0.0;
        const double f1 = f ? f[1] : 0.0, f2 = f ? f[2] : 0.0, f3 = f ? f[3] : 0.0;
        const bool has_fb = dE != 0.0 || f1 != 0.0 || f2 != 0.0 || f3 != 0.0;
        const int64_t lo = work ? off[c] : 0, hi = work ? off[c + 1] : 0;
        double W = 0.0, P0 = 0.0, P1 = 0.0, P2 = 0.0, U2 = 0.0;
        // the first kFbCache electrons of each lane stay in registers for the remap
        T cx[kFbCache], cy[kFbCache], cz[kFbCache];
#pragma unroll
        for (int q = 0; q < kFbCache; ++q) {
            const int64_t i = lo + sub + (int64_t)q * L;
            cx[q] = cy[q] = cz[q] = (T)0;
            if (i < hi) {
                const double wi = w_ref * (double)w[i];
                cx[q] = px[i]; cy[q] = py[i]; cz[q] = pz[i];
                const double a = cx[q], b = cy[q], d = cz[q];
                W += wi; P0 += wi * a; P1 += wi * b; P2 += wi * d;
                U2 += wi * (a * a + b * b + d * d);
            }
        }
        for (int64_t i = lo + sub + (int64_t)kFbCache * L; i < hi; i += L) {
            const double wi = w_ref * (double)w[i];
            const double a = px[i], b = py[i], d = pz[i];
            W += wi; P0 += wi * a; P1 += wi * b; P2 += wi * d;
            U2 += wi * (a * a + b * b + d * d);
        }
        W = group_sum<L>(W); P0 = group_sum<L>(P0); P1 = group_sum<L>(P1);
        P2 = group_sum<L>(P2); U2 = group_sum<L>(U2);
        if (!work) continue;
        if (moments && sub == 0) {
            double* mo = moments + c * 5;
            mo[0] = W; mo[1] = P0; mo[2] = P1; mo[3] = P2; mo[4] = U2;
        }
        double unapplied = 0.0;
        if (W > 0.0) {
            const double d0 = f1 / W, d1 = f2 / W, d2 = f3 / W;
            const double var = U2 - (P0 * P0 + P1 * P1 + P2 * P2) / W;
            const double dEbulk =
                (2.0 * (d0 * P0 + d1 * P1 + d2 * P2) + W * (d0 * d0 + d1 * d1 + d2 * d2)) * 0.5;
            const double dEth = dE - dEbulk;
            double var_new = var + 2.0 * dEth;
            const bool cold = !(var > 1e-14 * (U2 + 1e-300));
            double S = 1.0;
            if (cold) {
                var_new = var;
                if (sub == 0 && stats) {
                    atomicAdd(&stats[AXPIC_ST_COLD_CELLS], 1.0);
                    unapplied = dEth;
                    *flag = token;
                }
            } else {
                if (var_new < 0.0) {
                    if (sub == 0 && stats) {
                        atomicAdd(&stats[AXPIC_ST_CLAMPED_CELLS], 1.0);
                        unapplied = -var_new * 0.5;
                        *flag = token;
                    }
                    var_new = 0.0;
                }
                S = sqrt(var_new / var);
            }
            if (kp.feedback && has_fb) {
                const double b0 = (1.0 - S) * (P0 / W) + d0, b1 = (1.0 - S) * (P1 / W) + d1,
                             b2 = (1.0 - S) * (P2 / W) + d2;
#pragma unroll
                for (int q = 0; q < kFbCache; ++q) {
                    const int64_t i = lo + sub + (int64_t)q * L;
                    if (i < hi) {
                        px[i] = (T)(S * (double)cx[q] + b0);
                        py[i] = (T)(S * (double)cy[q] + b1);
                        pz[i] = (T)(S * (double)cz[q] + b2);
                    }
                }
                for (int64_t i = lo + sub + (int64_t)kFbCache * L; i < hi; i += L) {
                    px[i] = (T)(S * (double)px[i] + b0);
                    py[i] = (T)(S * (double)py[i] + b1);
                    pz[i] = (T)(S * (double)pz[i] + b2);
                }
            }
            if (kp.T_mode == 2 && sub == 0) {
                const double Test = kMe / 3.0 * var_new / W;
                double Tn = (1.0 - kp.r_relax) * Tk[c] + kp.r_relax * Test;
                Tn = Tn < kp.T_floor ? kp.T_floor : (Tn > kp.T_ceil ? kp.T_ceil : Tn);
                Tk[c] = Tn;
            }
        }
        if (ecell && sub == 0) ecell[c] = unapplied;
    }
}

constexpr int kFbParts = 256;          // blocks of k_fb_unapplied (parts in the workspace records)

// After k_feedback: when a cell of this call (token) left energy unapplied, the slots of
// all cells summed in cell order into stats[AXPIC_ST_UNAPPLIED_E]: block b sums the b-th
// of gridDim.x equal runs of cells (each thread a strided part, then the butterfly and
// the wavefronts in order) into part[b], and the block that finishes last adds the
// parts in block order.  Nothing at all when no cell of the call was flagged.
__global__ void __launch_bounds__(kThreads)
k_fb_unapplied(int64_t ncell, const double* __restrict__ ecell, const int64_t* __restrict__ flag,
               int64_t token, const int64_t* __restrict__ chain, double* __restrict__ part,
               unsigned int* __restrict__ done, double* __restrict__ stats) {
    __shared__ double lds[kThreads / 64];
    __shared__ bool last;
    if ((chain && chain[AXPIC_CHAIN_SKIP]) || *flag != token) return;
    const int64_t per = (ncell + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = (int64_t)blockIdx.x * per, c1 = c0 + per < ncell ? c0 + per : ncell;
    double s = 0.0;
    int64_t c = c0 + threadIdx.x;
    for (; c + 7 * kThreads < c1; c += 8 * kThreads) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ecell[c + u * kThreads];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < c1; c += kThreads) s += ecell[c];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int w2 = 0; w2 < kThreads / 64; ++w2) b += lds[w2];
        part[blockIdx.x] = b;
        __threadfence();                                  // the part before the count
        last = atomicAdd(done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    __threadfence();                                      // every part after the count
    double t = 0.0;
    for (unsigned int b = 0; b < gridDim.x; ++b) t += part[b];
    stats[AXPIC_ST_UNAPPLIED_E] += t;
}

// ------------------------------------------------------------------ superposed thermal emission
// In a cell the electrons' Poisson counts K_e ~ Poisson(lambda_e), lambda_e =
// w_e coef (eq. lambda_macro), have the joint law of a cell total
// N ~ Poisson(sum_e lambda_e) split multinomially with probabilities
// lambda_e / Lambda; electrons at the cap (eqs. lambda_eff, wa_rescaled) enter
// with min(lambda_e, cap) and carry lambda_e / cap in their product weight.
// The work is per cell and per event instead of per electron.  The electrons
// of cell c are off[c] .. off[c+1]-1; cellw[c] = sum of their relative
// weights, cellw[ncell + c] = the largest.

// Cell weight sums: 16 lanes per cell, fixed reduction order.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cell_weights(int64_t ncell, const int64_t* __restrict__ off, const T* __restrict__ w,
               double* __restrict__ out) {
    const int sub = threadIdx.x & (kCellLanes - 1);
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kCellLanes;
    const bool valid = c < ncell;
    const int64_t lo = valid ? off[c] : 0, hi = valid ? off[c + 1] : 0;
    double s = 0.0, m = 0.0;
    for (int64_t i = lo + sub; i < hi; i += kCellLanes) {
        const double v = (double)w[i];
        s += v;
        m = fmax(m, v);
    }
    s = group_sum16(s);
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (valid && sub == 0) { out[c] = s; out[ncell + c] = m; }
}

// Lambda of a cell and channel: coef W when no electron reaches the cap, else
// the sum of min(w_e coef, cap) in index order.
template <typename T>
__device__ __forceinline__ double sup_lambda(double k, double W, double wmax, double cap,
                                             int64_t lo, int64_t hi, const T* __restrict__ w) {
#pragma clang fp contract(off)
    if (!(wmax * k > cap)) return k * W;
    double L = 0.0;
    for (int64_t e = lo; e < hi; ++e) {
        const double le = (double)w[e] * k;
        L += le < cap ? le : cap;
    }
    return L;
}

// N ~ Poisson(L) by inversion; a mean above 500 as ceil(L/500) equal parts
// (stream 5, block = part, words 0-1 Compton, 2-3 brems).
__device__ __forceinline__ uint32_t sup_poisson(const KParams& kp, int64_t c, int64_t step, int ch,
                                                double L) {
    if (!(L > 0.0)) return 0u;
    const int parts = L > 500.0 ? (int)ceil(L / 500.0) : 1;
    const double Lp = L / (double)parts;
    uint32_t N = 0;
    for (int q = 0; q < parts; ++q) {
        const uint4 r = draw(kp, (uint64_t)c, step, 5, (uint32_t)q);
        N += (uint32_t)poisson_inv_k(Lp, ch == 1 ? u53(r.x, r.y) : u53(r.z, r.w), 1 << 30);
    }
    return N;
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_sup_count(int64_t ncell, int64_t step, KParams kp, const float* __restrict__ p32,
            const double* __restrict__ p64, const int64_t* __restrict__ off,
            const T* __restrict__ w, const double* __restrict__ cellw,
            uint32_t* __restrict__ counts, uint32_t* __restrict__ bsum,
            uint32_t* __restrict__ bact) {
    __shared__ uint32_t lds[kThreads / 64];
    const T* pref = PrefOf<T>::get(p32, p64);
    const bool onC = kp.channels & AXPIC_COMPTON, onB = kp.channels & AXPIC_BREMS;
    const int64_t base = (int64_t)blockIdx.x * kBlockParents;
    uint32_t tot = 0, act = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t c = base + j * kThreads + threadIdx.x;
        if (c >= ncell) break;
        const T* pc = pref + c * AXPIC_PREF_N;
        const double W = cellw[c], wmax = cellw[ncell + c];
        const int64_t lo = off[c], hi = off[c + 1];
        const double kC = onC ? (double)pc[4] : 0.0, kB = onB ? (double)pc[5] : 0.0;
        const uint32_t NC = sup_poisson(kp, c, step, 1, sup_lambda<T>(kC, W, wmax, kp.cap, lo, hi, w));
        const uint32_t NB = sup_poisson(kp, c, step, 2, sup_lambda<T>(kB, W, wmax, kp.cap, lo, hi, w));
        counts[2 * c] = NC;
        counts[2 * c + 1] = NB;
        tot += NC + NB;
        act += (NC + NB) > 0;
    }
    const uint32_t bt = block_sum_u32(tot, lds);
    const uint32_t ba = block_sum_u32(act, lds);
    if (threadIdx.x == 0) { bsum[blockIdx.x] = bt; bact[blockIdx.x] = ba; }
}

// Records of the superposed events in canonical order (cell, channel, j):
// cell (bits 0-31), j (32-61), channel (62-63).
__global__ void __launch_bounds__(kThreads)
k_sup_expand(int64_t ncell, const uint32_t* __restrict__ counts, const uint32_t* __restrict__ bact,
             const uint64_t* __restrict__ boff, const int64_t* __restrict__ ctrl, int64_t out_n,
             int64_t out_cap, uint64_t* __restrict__ rec) {
    __shared__ uint32_t lds[kThreads / 64];
    if (ctrl[0] || bact[blockIdx.x] == 0) return;
    out_n = ctrl[2];
    const int64_t c0 = (int64_t)blockIdx.x * kBlockParents + (int64_t)kPer * threadIdx.x;
    uint32_t n[2 * kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const bool ok = c0 + q < ncell;
        n[2 * q] = ok ? counts[2 * (c0 + q)] : 0u;
        n[2 * q + 1] = ok ? counts[2 * (c0 + q) + 1] : 0u;
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < 2 * kPer; ++q) cnt += n[q];
    uint32_t segtot;
    const uint32_t pre = block_excl_scan(cnt, lds, &segtot);
    if (cnt == 0) return;
    int64_t slot = out_n + (int64_t)(boff[blockIdx.x] + pre);
    for (int q = 0; q < kPer; ++q)
        for (int ch = 1; ch <= 2; ++ch)
            for (uint32_t j = 0; j < n[2 * q + ch - 1]; ++j, ++slot)
                if (slot < out_cap)
                    rec[slot] = (uint64_t)(c0 + q) | ((uint64_t)j << 32) | ((uint64_t)ch << 62);
}

template <typename T, bool M>
__global__ void __launch_bounds__(kThreads)
k_sup_events(int64_t ncell, int64_t step, uint64_t next_id, KParams kp,
             const float* __restrict__ p32, const double* __restrict__ p64,
             const double* __restrict__ state, const int64_t* __restrict__ off,
             const T* __restrict__ w, const T* __restrict__ x0, const T* __restrict__ x1,
             const T* __restrict__ x2, const double* __restrict__ cellw,
             const int64_t* __restrict__ ctrl, int64_t out_n, T* __restrict__ ax0,
             T* __restrict__ ax1, T* __restrict__ ax2, T* __restrict__ apx, T* __restrict__ apy,
             T* __restrict__ apz, T* __restrict__ aw, uint64_t* __restrict__ aid,
             int32_t* __restrict__ acell, double* __restrict__ fb, double* __restrict__ rec,
             int32_t* __restrict__ bkey, double* __restrict__ bval, StatMap smap) {
#pragma clang fp contract(off)
    extern __shared__ double wh[];                          // per wavefront: channels 1, 2
    __shared__ double lst[(kThreads / 64) * kStatSlots];
    __shared__ FbStitch fbs;
    if (ctrl[0]) return;
    out_n = ctrl[2];
    next_id = (uint64_t)ctrl[3];
    const int64_t total = ctrl[1];
    int64_t elo, ehi;
    ev_range(total, &elo, &ehi);
    if (elo >= ehi) return;               // no events: no records (the reductions skip them)
    const T* pref = PrefOf<T>::get(p32, p64);
    const int nbh = kp.nbins + 2;
    const int H = 2 * nbh;
    for (int k = threadIdx.x; k < (kThreads / 64) * H; k += kThreads) wh[k] = 0.0;
    __syncthreads();
    double* myh = wh + (threadIdx.x >> 6) * H;
    double st[kStatSlots];
    for (int s = 0; s < kStatSlots; ++s) st[s] = 0.0;
    FbOpen open;
    for (int64_t t0 = elo; t0 < ehi; t0 += kThreads) {
        const int64_t e = t0 + threadIdx.x;
        const int64_t slot = out_n + e;
        const uint64_t rc = e < ehi ? aid[slot] : 0ull;
        const int64_t c = (int64_t)(rc & 0xFFFFFFFFull);
        const uint32_t j = (uint32_t)((rc >> 32) & 0x3FFFFFFFull);
        const int ch = (int)(rc >> 62);                     // 1 Compton, 2 brems
        int bin = -1;
        double hv = 0.0;
        int32_t key = -1;
        double fv[4] = {0.0, 0.0, 0.0, 0.0};
        if (e < ehi && c < ncell && (ch == 1 || ch == 2)) { // always, for a well-formed record
            key = (int32_t)c;
            const T* pc = pref + c * AXPIC_PREF_N;
            const double k = (double)pc[3 + ch];
            const double W = cellw[c], wmax = cellw[ncell + c];
            const int64_t lo = off[c], hi = off[c + 1];
            const bool capped_cell = wmax * k > kp.cap;
            const double L = sup_lambda<T>(k, W, wmax, kp.cap, lo, hi, w);
            // the electron: inverse CDF of lambda_e / Lambda over the cell in index order,
            // eight weights loaded at a time
            uint4 r = draw(kp, (uint64_t)c, step, 6, (uint32_t)(ch - 1) * (1u << 23) + j);
            const double target = u53(r.x, r.y) * (capped_cell ? L : W);
            int64_t pick = -1, last = -1;
            double a = 0.0;
            for (int64_t e0 = lo; e0 < hi && pick < 0; e0 += 8) {
                T v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = e0 + q < hi ? w[e0 + q] : (T)0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (pick >= 0 || !(v[q] > (T)0)) continue;
                    const double wv = (double)v[q];
                    const double le = wv * k;
                    a += capped_cell ? (le < kp.cap ? le : kp.cap) : wv;
                    last = e0 + q;
                    if (a > target) pick = e0 + q;
                }
            }
            if (pick < 0) pick = last;
            if (pick >= 0) {                                // none: no electron with weight (N is 0)
                const double le = (double)w[pick] * k;
                const double ws = le > kp.cap ? le / kp.cap : 1.0;
                const double wp = kp.w_a * kp.wa_mul[ch] * ws;
                const double Tc = state[c * AXPIC_STATE_N + 0];
                const double* tab = ch == 1 ? g_tab_compton : g_tab_gamma;
                r = draw(kp, (uint64_t)c, step, 6 + ch, j);
                double E, pm;
                thermal_energy<M>(kp, ch, Tc, u24(r.x), tab, &E, &pm);
                const double eu = M ? E / kMe : pm;        // energy in m_e c^2
                const double mu = 2.0 * u24(r.y) - 1.0;
                const double phi = 2.0 * kPi * u24(r.z);
                const double sn = sqrt(fmax(0.0, 1.0 - mu * mu));
                double sphi, cphi;
                sincos(phi, &sphi, &cphi);
                const double pa[3] = {pm * sn * cphi, pm * sn * sphi, pm * mu};
                ax0[slot] = x0[pick];
                if (ax1) ax1[slot] = x1 ? x1[pick] : (T)0;
                if (ax2) ax2[slot] = x2 ? x2[pick] : (T)0;
                apx[slot] = (T)pa[0]; apy[slot] = (T)pa[1]; apz[slot] = (T)pa[2];
                aw[slot] = (T)(kp.wa_mul[ch] * ws);
                aid[slot] = (next_id + (uint64_t)e) | (1ull << 63);
                acell[slot] = (int32_t)c;
                bin = (ch - 1) * nbh + hist_bin(kp, E);
                hv = wp * E;
                fv[0] = -wp * eu; fv[1] = -wp * pa[0]; fv[2] = -wp * pa[1]; fv[3] = -wp * pa[2];
                st[ch] += 1.0; st[3 + ch] += wp; st[6 + ch] += wp * E;
                if (le > kp.cap) st[9] += 1.0;
            }
        }
        wave_hist_add(myh, bin, hv);
        if (fb) fb_tile(fbs, open, key, fv, fb, bkey, bval, blockIdx.x);
    }
    if (fb) fb_finish(open, fb, bkey, bval, blockIdx.x);
    __syncthreads();
    rec_write(wh, H, st, smap, lst, rec + blockIdx.x, kEventBlocks);
}

// ------------------------------------------------------------------ compaction
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_live_count(int64_t n, const T* __restrict__ w, uint16_t* __restrict__ code,
             uint32_t* __restrict__ bsum, uint32_t* __restrict__ bact) {
    __shared__ uint32_t lds[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kBlockParents;
    uint32_t tot = 0;
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = base + j * kThreads + threadIdx.x;
        if (i >= n) break;
        const uint32_t a = w[i] > (T)0 ? 1u : 0u;
        code[i] = (uint16_t)a;
        tot += a;
    }
    const uint32_t bt = block_sum_u32(tot, lds);
    if (threadIdx.x == 0) { bsum[blockIdx.x] = bt; bact[blockIdx.x] = bt; }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_compact_apply(int64_t n, const uint16_t* __restrict__ code, const uint64_t* __restrict__ boff,
                const int64_t* __restrict__ ctrl, int64_t out_cap, int ndim,
                const T* __restrict__ x0, const T* __restrict__ x1, const T* __restrict__ x2,
                const T* __restrict__ px, const T* __restrict__ py, const T* __restrict__ pz,
                const T* __restrict__ w, IdView id,
                const int32_t* __restrict__ cell, const T* __restrict__ p2, T* __restrict__ ox0,
                T* __restrict__ ox1, T* __restrict__ ox2, T* __restrict__ opx, T* __restrict__ opy,
                T* __restrict__ opz, T* __restrict__ ow, uint64_t* __restrict__ oid,
                int32_t* __restrict__ ocell, T* __restrict__ op2) {
    __shared__ uint32_t lds[kThreads / 64];
    if (ctrl[0]) return;
    const int64_t base = (int64_t)blockIdx.x * kBlockParents;
    uint64_t run = boff[blockIdx.x];
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = base + j * kThreads + threadIdx.x;
        const uint32_t a = (i < n) ? code[i] : 0u;
        uint32_t segtot;
        const uint32_t pre = block_excl_scan(a, lds, &segtot);
        if (a) {
            const int64_t s = (int64_t)(run + pre);
            if (s < out_cap) {
                ox0[s] = x0[i];
                if (ndim > 1) ox1[s] = x1[i];
                if (ndim > 2) ox2[s] = x2[i];
                opx[s] = px[i]; opy[s] = py[i]; opz[s] = pz[i];
                ow[s] = w[i]; oid[s] = id(i); ocell[s] = cell[i];
                if (op2) op2[s] = p2 ? p2[i] : p2_of<T>(px[i], py[i], pz[i]);
            }
        }
        run += segtot;
    }
}

// ------------------------------------------------------------------ canonical order
// Stable counting sort by cell with the particles of zero weight dropped: counts per
// cell, offsets by a scan over the cells, source indices scattered into their cell's
// range in any order, then each index ranked among its cell's indices -- ascending
// index is the stable order -- and the particle moved to its slot.  The result does not
// depend on the scatter's order.  Consecutive particles of one cell in a wavefront (the
// usual case: the input is the previous step's order) share one atomic.
constexpr int kSortCellsPerBlock = kThreads * kPer;     // cells per block of the offset scan
constexpr int kSortSlots = kThreads * kPer;             // sorted slots per block of the gather
constexpr int kSortWindow = 4 * kSortSlots;             // source indices staged in LDS

__global__ void __launch_bounds__(kThreads)
k_fill_u32(int64_t n, uint32_t* __restrict__ a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0u;
}

// The cell of particle i when it takes part (positive weight, cell on the grid), else -1;
// the same test in the count and the scatter.
template <typename T>
__device__ __forceinline__ int32_t sort_key(int64_t i, int64_t n, const T* __restrict__ w,
                                            const int32_t* __restrict__ cell, int64_t ncell) {
    if (i >= n) return -1;
    const int32_t c = cell[i];
    return (w[i] > (T)0 && c >= 0 && (int64_t)c < ncell) ? c : -1;
}

// Runs of equal keys in adjacent lanes of a wavefront: the first lane of this lane's run
// and the run's length.  Every lane of the wavefront must call it.
struct WaveRun { int head; uint32_t len; };
__device__ __forceinline__ WaveRun wave_run(int32_t key) {
    const int lane = threadIdx.x & 63;
    const int32_t prev = __shfl_up(key, 1, 64);
    const uint64_t heads = __ballot(lane == 0 || prev != key);
    const uint64_t upto = heads & ((2ull << lane) - 1ull);          // heads at or below lane
    const uint64_t above = heads & ~((2ull << lane) - 1ull);
    WaveRun r;
    r.head = 63 - __clzll((long long)upto);
    const int next = above ? __ffsll((unsigned long long)above) - 1 : 64;
    r.len = (uint32_t)(next - r.head);
    return r;
}

// The wavefront's keys sorted ascending, each tagged with its lane: (key << 6) | lane,
// the lanes without a key (k < 0) last.  A bitonic network over the 64 lanes; runs of a
// cell are then as long as the cell's particles in the wavefront, not only its adjacent
// ones (the particles that moved to a neighbouring cell break no run).
__device__ __forceinline__ uint64_t wave_sort_keys(int32_t k) {
    const int lane = threadIdx.x & 63;
    uint64_t key = k >= 0 ? ((uint64_t)(uint32_t)k << 6) | (uint64_t)lane : ~0ull;
#pragma unroll
    for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            const uint64_t ok = __shfl_xor(key, j, 64);
            const bool up = (lane & kk) == 0, lower = (lane & j) == 0;
            if (lower == up ? ok < key : ok > key) key = ok;
        }
    }
    return key;
}

// Blocks go round robin over the eight XCDs; this gives each XCD a contiguous range of
// block indices, so that neighbouring ranges of particles share that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblk) {
    const int64_t q = nblk / 8, r = nblk % 8, x = b % 8, k = b / 8;
    return x * q + (x < r ? x : r) + k;
}

// A block's open-addressed LDS table of the cells its particles fall in (more slots
// than particles, so an insertion always ends).  Returns the slot of cell c.
constexpr int kSortHashBits = 11;
constexpr int kSortHash = 1 << kSortHashBits;
static_assert(kSortHash >= 2 * kSortSlots, "the cell table must outnumber the particles");
__device__ __forceinline__ int sort_hash_slot(int32_t c, int32_t* hkey) {
    uint32_t h = ((uint32_t)c * 2654435761u) >> (32 - kSortHashBits);
    for (;;) {
        const int32_t old = atomicCAS(&hkey[h], -1, c);
        if (old == -1 || old == c) return (int)h;
        h = (h + 1) & (kSortHash - 1);
    }
}

__device__ __forceinline__ void sort_hash_clear(int32_t* hkey, uint32_t* hval) {
    for (int h = threadIdx.x; h < kSortHash; h += kThreads) { hkey[h] = -1; hval[h] = 0u; }
}

// The smallest and largest of the block's keys (*hi < *lo: none), in every thread.
constexpr int kSortWin = 4096;          // cells of a block's direct-mapped LDS window
__device__ __forceinline__ void block_key_range(const int32_t* c, int32_t* lds, int32_t* lo,
                                                int32_t* hi) {
    int32_t mn = INT32_MAX, mx = -1;
#pragma unroll
    for (int q = 0; q < kPer; ++q)
        if (c[q] >= 0) { mn = min(mn, c[q]); mx = max(mx, c[q]); }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o, 64));
        mx = max(mx, __shfl_xor(mx, o, 64));
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { lds[2 * wave] = mn; lds[2 * wave + 1] = mx; }
    __syncthreads();
    mn = INT32_MAX; mx = -1;
#pragma unroll
    for (int v = 0; v < kThreads / 64; ++v) { mn = min(mn, lds[2 * v]); mx = max(mx, lds[2 * v + 1]); }
    *lo = mn; *hi = mx;
}

// kSortSlots particles per block: counts per cell.  With TABLE, gathered by runs of a
// wavefront into the block's cell table (one atomic per cell and block: it pays where
// the cells are dense); else, when the block's cells span fewer than kSortWin indices
// (a cell-ordered input moved by a step: a block's cells and their neighbours), counted
// in a direct-mapped LDS window and added once per cell and block, otherwise one atomic
// per run of a wavefront's sorted cells.
template <typename T, bool TABLE>
__global__ void __launch_bounds__(kThreads)
k_sort_count(int64_t n, int64_t ncell, const T* __restrict__ w,
             const int32_t* __restrict__ cell, uint32_t* __restrict__ cnt) {
    __shared__ int32_t hkey[TABLE ? kSortHash : 1];
    __shared__ uint32_t hval[TABLE ? kSortHash : kSortWin];
    __shared__ int32_t rng[2 * (kThreads / 64)];
    const int lane = threadIdx.x & 63;
    const int64_t base = (int64_t)blockIdx.x * kSortSlots;
    if (!TABLE) {
        int32_t c[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            c[q] = sort_key<T>(base + q * kThreads + threadIdx.x, n, w, cell, ncell);
        int32_t lo, hi;
        block_key_range(c, rng, &lo, &hi);
        if (hi < lo) return;                                    // uniform: no live particle
        if (hi - lo < kSortWin) {
            for (int e = threadIdx.x; e <= hi - lo; e += kThreads) hval[e] = 0u;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kPer; ++q)
                if (c[q] >= 0) atomicAdd(&hval[c[q] - lo], 1u);
            __syncthreads();
            for (int e = threadIdx.x; e <= hi - lo; e += kThreads)
                if (hval[e]) atomicAdd(&cnt[lo + e], hval[e]);
            return;
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            if (!__any(c[q] >= 0)) continue;                    // wave-uniform
            const uint64_t key = wave_sort_keys(c[q]);
            const int32_t cs = key == ~0ull ? -1 : (int32_t)(key >> 6);
            const WaveRun r = wave_run(cs);
            if (cs >= 0 && r.head == lane) atomicAdd(&cnt[cs], r.len);
        }
        return;
    }
    sort_hash_clear(hkey, hval);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int32_t c = sort_key<T>(base + q * kThreads + threadIdx.x, n, w, cell, ncell);
        const WaveRun r = wave_run(c);
        if (c >= 0 && r.head == lane) atomicAdd(&hval[sort_hash_slot(c, hkey)], r.len);
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kSortHash; h += kThreads)
        if (hkey[h] >= 0) atomicAdd(&cnt[hkey[h]], hval[h]);
}

// Per block of kSortCellsPerBlock cells: the sum of their counts.
__global__ void __launch_bounds__(kThreads)
k_sort_blocksum(int64_t ncell, const uint32_t* __restrict__ cnt, uint32_t* __restrict__ bsum) {
    __shared__ uint32_t lds[kThreads / 64];
    const int64_t c0 = (int64_t)blockIdx.x * kSortCellsPerBlock + (int64_t)kPer * threadIdx.x;
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) v += c0 + q < ncell ? cnt[c0 + q] : 0u;
    const uint32_t t = block_sum_u32(v, lds);
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// Cell offsets off[c] = block offset + exclusive scan of the block's counts; off[ncell] =
// the total (also to the chain's axion and start-of-step words).  Nothing when the output
// does not fit or the chain says skip (ctrl[0]).
__global__ void __launch_bounds__(kThreads)
k_sort_offsets(int64_t ncell, const uint32_t* __restrict__ cnt, const uint64_t* __restrict__ boff,
               const int64_t* __restrict__ ctrl, int64_t* __restrict__ off,
               int64_t* __restrict__ chain) {
    __shared__ uint32_t lds[kThreads / 64];
    if (ctrl[0]) return;
    const int64_t c0 = (int64_t)blockIdx.x * kSortCellsPerBlock + (int64_t)kPer * threadIdx.x;
    uint32_t v[kPer], tot = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) { v[q] = c0 + q < ncell ? cnt[c0 + q] : 0u; tot += v[q]; }
    uint32_t segtot;
    uint64_t run = boff[blockIdx.x] + block_excl_scan(tot, lds, &segtot);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (c0 + q < ncell) off[c0 + q] = (int64_t)run;
        run += v[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        off[ncell] = ctrl[1];
        if (chain) chain[AXPIC_CHAIN_AXIONS] = chain[AXPIC_CHAIN_AX_START] = ctrl[1];
    }
}

// Source index of every live particle into its cell's range.  The per-cell count is
// consumed as a countdown: one atomic per cell and block reserving the block's share
// (with TABLE through the block's cell table, else through the direct-mapped window when
// the block's cells fit), within which each particle takes the place its run and the
// table, or an LDS countdown, give; else one atomic per run of a wavefront's sorted
// cells.  The order within a cell is whatever the atomics give.  Nothing when the
// output does not fit (ctrl[0]).
template <typename T, bool TABLE>
__global__ void __launch_bounds__(kThreads)
k_sort_scatter(int64_t n, int64_t ncell, const T* __restrict__ w, const int32_t* __restrict__ cell,
               const int64_t* __restrict__ off, const int64_t* __restrict__ ctrl,
               uint32_t* __restrict__ cnt, uint32_t* __restrict__ idx) {
    __shared__ int32_t hkey[TABLE ? kSortHash : 1];
    __shared__ uint32_t hval[TABLE ? kSortHash : kSortWin];   // a cell's count in the block
    __shared__ uint32_t hbase[TABLE ? 1 : kSortWin];          // the block's base in the cell
    __shared__ int32_t rng[2 * (kThreads / 64)];
    if (ctrl[0]) return;                     // uniform over the grid
    const int lane = threadIdx.x & 63;
    const int64_t base = (int64_t)blockIdx.x * kSortSlots;
    if (!TABLE) {
        int32_t cc[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            cc[q] = sort_key<T>(base + q * kThreads + threadIdx.x, n, w, cell, ncell);
        int32_t lo, hi;
        block_key_range(cc, rng, &lo, &hi);
        if (hi < lo) return;                                // uniform: no live particle
        if (hi - lo < kSortWin) {
            for (int e = threadIdx.x; e <= hi - lo; e += kThreads) hval[e] = 0u;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kPer; ++q)
                if (cc[q] >= 0) atomicAdd(&hval[cc[q] - lo], 1u);
            __syncthreads();
            for (int e = threadIdx.x; e <= hi - lo; e += kThreads) {
                const uint32_t t = hval[e];
                if (t) hbase[e] = atomicSub(&cnt[lo + e], t) - t;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kPer; ++q)
                if (cc[q] >= 0) {
                    const int e = cc[q] - lo;
                    const uint32_t pos = atomicSub(&hval[e], 1u) - 1u;
                    idx[off[cc[q]] + hbase[e] + pos] = (uint32_t)(base + q * kThreads + threadIdx.x);
                }
            return;
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int64_t i0 = base + q * kThreads + (threadIdx.x & ~63);   // the wave's first
            const int32_t c0 = cc[q];
            if (!__any(c0 >= 0)) continue;                  // wave-uniform
            const uint64_t key = wave_sort_keys(c0);
            const int32_t c = key == ~0ull ? -1 : (int32_t)(key >> 6);
            const WaveRun r = wave_run(c);
            uint32_t l = 0;
            if (c >= 0 && r.head == lane) l = atomicSub(&cnt[c], r.len) - r.len;
            l = __shfl(l, r.head, 64) + (uint32_t)(lane - r.head);
            if (c >= 0) idx[off[c] + l] = (uint32_t)(i0 + (int64_t)(key & 63u));
        }
        return;
    }
    sort_hash_clear(hkey, hval);
    __syncthreads();
    int32_t cq[kPer];
    int slot[kPer];
    uint32_t loc[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int32_t c = sort_key<T>(base + q * kThreads + threadIdx.x, n, w, cell, ncell);
        const WaveRun r = wave_run(c);
        int h = 0;
        uint32_t l = 0;
        if (c >= 0 && r.head == lane) {
            h = sort_hash_slot(c, hkey);
            l = atomicAdd(&hval[h], r.len);
        }
        slot[q] = __shfl(h, r.head, 64);
        loc[q] = __shfl(l, r.head, 64) + (uint32_t)(lane - r.head);
        cq[q] = c;
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kSortHash; h += kThreads)
        if (hkey[h] >= 0) {
            const uint32_t t = hval[h];
            hval[h] = atomicSub(&cnt[hkey[h]], t) - t;
        }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q)
        if (cq[q] >= 0)
            idx[off[cq[q]] + hval[slot[q]] + loc[q]] = (uint32_t)(base + q * kThreads + threadIdx.x);
}

// The arrays a sort moves: particle i of `in` to slot d of `out` (SortVal).
template <typename T>
struct SortIO {
    int ndim;
    const T* x[3];
    const T* p[3];
    const T* w;
    IdView id;
    T* ox[3];
    T* op[3];
    T* ow;
    uint64_t* oid;
    int32_t* ocell;
};

// One particle's arrays in registers (the gather loads a thread's particles first and
// then stores them, so that their loads are in flight together).
template <typename T>
struct SortVal {
    T x[3], p[3], w;
    uint64_t id;
    __device__ __forceinline__ void load(const SortIO<T>& io, int64_t i) {
        x[0] = io.x[0][i];
        x[1] = io.ndim > 1 ? io.x[1][i] : (T)0;
        x[2] = io.ndim > 2 ? io.x[2][i] : (T)0;
        p[0] = io.p[0][i]; p[1] = io.p[1][i]; p[2] = io.p[2][i];
        w = io.w[i];
        id = io.id(i);
    }
    __device__ __forceinline__ void store(const SortIO<T>& io, int64_t d, int32_t c) const {
        io.ox[0][d] = x[0];
        if (io.ndim > 1) io.ox[1][d] = x[1];
        if (io.ndim > 2) io.ox[2][d] = x[2];
        io.op[0][d] = p[0]; io.op[1][d] = p[1]; io.op[2][d] = p[2];
        io.ow[d] = w;
        io.oid[d] = id;
        io.ocell[d] = c;
    }
};

// Number of entries below s in src[a, b).
__device__ __forceinline__ uint32_t count_below(const uint32_t* __restrict__ src, int64_t a,
                                                int64_t b, uint32_t s) {
    uint32_t r = 0;
    for (int64_t m = a; m < b; ++m) r += src[m] < s ? 1u : 0u;
    return r;
}

// kSortSlots consecutive sorted slots per block.  The source indices of the cells these
// slots belong to are staged in LDS (at most kSortWindow of them, the rest read from
// global memory); the slot of each particle is its cell's offset plus the number of the
// cell's source indices below its own, and the particle is copied there.
// With XCD, neighbouring blocks of slots run on one XCD (pays where the cells are sparse
// and a block's sources spread over many lines).
template <typename T, bool XCD>
__global__ void __launch_bounds__(kThreads)
k_sort_gather(int64_t ncell, const int64_t* __restrict__ off, const uint32_t* __restrict__ idx,
              const int64_t* __restrict__ ctrl, const int32_t* __restrict__ cell, SortIO<T> io) {
    __shared__ uint32_t win[kSortWindow];
    if (ctrl[0]) return;                                 // uniform over the grid
    const int64_t total = off[ncell];
    const int64_t j0 = (XCD ? xcd_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x) * kSortSlots;
    if (j0 >= total) return;                             // uniform over the block
    const int64_t j1 = j0 + kSortSlots < total ? j0 + kSortSlots : total;
    // the window: every cell the block's slots belong to, clipped to kSortWindow entries
    // around them (kSortWindow >= kSortSlots, so the slots themselves always fit)
    int64_t wlo = off[cell[idx[j0]]], whi = off[cell[idx[j1 - 1]] + 1];
    if (whi - wlo > kSortWindow) {
        const int64_t lo2 = j0 - (kSortWindow - kSortSlots) / 2;
        wlo = wlo > lo2 ? wlo : lo2;
        whi = whi < wlo + kSortWindow ? whi : wlo + kSortWindow;
    }
    for (int64_t m = wlo + threadIdx.x; m < whi; m += kThreads) win[m - wlo] = idx[m];
    __syncthreads();
    // the thread's kPer slots stage by stage (source, its cell, the cell's range, the
    // particle), so each stage's loads are in flight together
    const int64_t jt = j0 + threadIdx.x;
    uint32_t sv[kPer];
    int32_t cv[kPer];
    int64_t lov[kPer], hiv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) sv[q] = jt + q * kThreads < j1 ? win[jt + q * kThreads - wlo] : 0u;
#pragma unroll
    for (int q = 0; q < kPer; ++q) cv[q] = jt + q * kThreads < j1 ? cell[sv[q]] : 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q)
        if (jt + q * kThreads < j1) { lov[q] = off[cv[q]]; hiv[q] = off[cv[q] + 1]; }
    SortVal<T> v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q)
        if (jt + q * kThreads < j1) v[q].load(io, (int64_t)sv[q]);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (jt + q * kThreads >= j1) break;
        const uint32_t s = sv[q];
        const int64_t lo = lov[q], hi = hiv[q];
        const int a = (int)((lo > wlo ? lo : wlo) - wlo), b = (int)((hi < whi ? hi : whi) - wlo);
        uint32_t rank = 0;
        for (int m = a; m < b; ++m) rank += win[m] < s ? 1u : 0u;
        if (lo < wlo) rank += count_below(idx, lo, wlo, s);
        if (hi > whi) rank += count_below(idx, whi, hi, s);
        v[q].store(io, lo + rank, cv[q]);
    }
}

// ------------------------------------------------------------------ diagnostics
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_diag_partial(int64_t n, double w_ref, double mu2, const T* __restrict__ w, const T* __restrict__ px,
               const T* __restrict__ py, const T* __restrict__ pz, double* __restrict__ part) {
    __shared__ double lds[2 * (kThreads / 64)];
    const int64_t base = (int64_t)blockIdx.x * kBlockParents;
    double N = 0.0, U = 0.0;
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = base + j * kThreads + threadIdx.x;
        if (i >= n) break;
        const double wi = w_ref * (double)w[i];
        if (wi > 0.0) {
            const double a = px[i], b = py[i], c = pz[i];
            N += wi;
            U += wi * kMe * sqrt(a * a + b * b + c * c + mu2);
        }
    }
    N = wave_sum(N); U = wave_sum(U);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { lds[2 * wave] = N; lds[2 * wave + 1] = U; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < kThreads / 64; ++k) { a += lds[2 * k]; b += lds[2 * k + 1]; }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ void __launch_bounds__(64)
k_diag_final(int64_t nb, const double* __restrict__ part, double* __restrict__ out) {
    const int lane = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t k = lane; k < nb; k += 64) { a += part[2 * k]; b += part[2 * k + 1]; }
    a = wave_sum(a); b = wave_sum(b);
    if (lane == 0) { out[0] = a; out[1] = b; }
}


// ------------------------------------------------------------------ equilibrium check
// The FP64 equilibrium check of the thermal inverse operators (Sec. II.I, eq.
// gamma_abs; the relaxation plateau of Sec. III.E), in an order fixed by the data:
// the population columns are summed per segment of kEqSeg particles by one wavefront
// (64 particles at a time; equal bins grouped by ballot and summed by one butterfly,
// added into the segment's LDS histogram in particle order), the reference columns per
// chunk of kEqCells cells (one thread per cell and bin, a fixed tree over the chunk),
// and the partials of the segments and chunks in their order.
constexpr int kEqSeg = 4096;
constexpr int kEqCells = 256;

template <typename T>
__global__ void __launch_bounds__(64)
k_eq_pop(int64_t n, KParams kp, double w_ref, const T* __restrict__ w, const T* __restrict__ px,
         const T* __restrict__ py, const T* __restrict__ pz, double* __restrict__ part) {
    extern __shared__ double h[];                       // [3][nbh]
    const int lane = threadIdx.x, nbh = kp.nbins + 2;
    for (int k = lane; k < 3 * nbh; k += 64) h[k] = 0.0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kEqSeg;
    for (int it = 0; it < kEqSeg / 64; ++it) {
        const int64_t i = base + (int64_t)it * 64 + lane;
        if (!__any(i < n)) break;
        double wp = 0.0, E = 0.0;
        int bin = -1;
        if (i < n) {
            wp = w_ref * (double)w[i];
            if (wp > 0.0) {
                const double pp = psq_d<T>(px, py, pz, i);
                E = kp.massive ? axion_energy(kp, pp) : kMe * sqrt(pp);
                bin = hist_bin(kp, E);
            }
        }
        uint64_t todo = __ballot(bin >= 0);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int b = __shfl(bin, leader, 64);
            const bool mine = bin == b;
            const uint64_t mask = __ballot(mine);
            const double s0 = wave_sum(mine ? wp : 0.0);
            const double s1 = wave_sum(mine ? wp * E : 0.0);
            const double s2 = wave_sum(mine ? wp * wp : 0.0);
            if (lane == 0) { h[b] += s0; h[nbh + b] += s1; h[2 * nbh + b] += s2; }
            todo &= ~mask;
        }
    }
    __syncthreads();
    double* out = part + (int64_t)blockIdx.x * 3 * nbh;
    for (int k = lane; k < 3 * nbh; k += 64) out[k] = h[k];
}

// 8-point Gauss-Legendre nodes and weights on [-1, 1] (Abramowitz and Stegun, Table 25.4)
__constant__ double kGL8x[4] = {0.1834346424956498049, 0.5255324099163289858,
                                0.7966664774136267396, 0.9602898564975362317};
__constant__ double kGL8w[4] = {0.3626837833783619830, 0.3137066458778872873,
                                0.2223810344533744706, 0.1012285362903762591};

struct EqCell {
    double T, c6, c7, V, t;
    // (V dn_eq/dE, V E dn_eq/dE, V dn_eq/dE q(g) (1 - e^{-t g})) at energy E
    __device__ void point(const KParams& kp, double E, double* v) const {
        v[0] = v[1] = v[2] = 0.0;
        if (!(E > 0.0) || (kp.massive && !(E > kp.m_a))) return;
        const double x = E / T;
        const double hc3 = kHbarcKeVcm * kHbarcKeVcm * kHbarcKeVcm;
        double dn = E * E / (2.0 * kPi * kPi * hc3) * (kp.eq_stats ? exp(-x) : 1.0 / expm1(x));
        double g = gabs_dt(kp, T, c6, c7, E);
        if (kp.massive) {              // E p instead of E^2; Gamma_abs gains E/p
            const double pr = sqrt((E - kp.m_a) * (E + kp.m_a));
            dn *= pr / E;
            g *= E / pr;
        }
        const double q = g > 0.0 ? g / -expm1(-g) : 1.0;
        const double grow = t > 0.0 ? -expm1(-t * g) : 1.0;
        v[0] = V * dn; v[1] = V * dn * E; v[2] = V * dn * q * grow;
    }
    // Gauss-Legendre over u in [a, b]; sub: the energy is m + u^2 (the square-root edge
    // of p at the mass), with the Jacobian 2u
    __device__ void panel(const KParams& kp, double a, double b, bool sub, double* acc) const {
        double v[3];
        const double h = 0.5 * (b - a), mid = 0.5 * (a + b);
        for (int q = 0; q < 8; ++q) {
            const double xi = (q & 1) ? kGL8x[q >> 1] : -kGL8x[q >> 1];
            const double u = mid + h * xi;
            const double wq = h * kGL8w[q >> 1];
            if (sub) {
                point(kp, kp.m_a + u * u, v);
                for (int k = 0; k < 3; ++k) acc[k] += wq * v[k] * 2.0 * u;
            } else {
                point(kp, u, v);
                for (int k = 0; k < 3; ++k) acc[k] += wq * v[k];
            }
        }
    }
    // [a, b] in panels no wider than hmax, split at the mass; the panel from the mass
    // in u = sqrt(E - m) on geometric panels [S 2^-(j+1), S 2^-j] (Gamma_abs grows like
    // E/p towards the threshold)
    __device__ void range(const KParams& kp, double a, double b, double hmax, double* acc) const {
        if (kp.massive) {
            if (!(b > kp.m_a)) return;
            if (a < kp.m_a) {
                const double e = fmin(b, kp.m_a + hmax), S = sqrt(e - kp.m_a);
                for (int j = 0; j < 48; ++j) panel(kp, ldexp(S, -(j + 1)), ldexp(S, -j), true, acc);
                a = e;
            }
        }
        if (!(b > a)) return;
        const int np = (int)ceil((b - a) / hmax);
        const int nn = np < 1 ? 1 : np;
        for (int j = 0; j < nn; ++j)
            panel(kp, a + (b - a) * j / nn, j + 1 == nn ? b : a + (b - a) * (j + 1) / nn, false, acc);
    }
};

__global__ void __launch_bounds__(kEqCells)
k_eq_ref(int64_t ncell, KParams kp, const double* __restrict__ p64, double V, double t_steps,
         double lo, double hi, double* __restrict__ part) {
    __shared__ double red[3][kEqCells / 64];
    const int k = blockIdx.y, nb = kp.nbins;
    const int64_t c = (int64_t)blockIdx.x * kEqCells + threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    if (c < ncell) {
        const double* pc = p64 + c * AXPIC_PREF_N;
        const EqCell q{pc[0], pc[6], pc[7], V, t_steps};
        if (q.T > 0.0) {
            const double hmax = q.T / 16.0;
            if (k < nb) {
                double a, b;
                if (kp.hist_log) {
                    a = lo * pow(hi / lo, (double)k / nb);
                    b = lo * pow(hi / lo, (double)(k + 1) / nb);
                } else {
                    a = lo + (hi - lo) * k / nb;
                    b = lo + (hi - lo) * (k + 1) / nb;
                }
                q.range(kp, a, b, hmax, acc);
            } else if (k == nb) {
                for (int j = 0; j < 60 && lo > 0.0; ++j)
                    q.range(kp, ldexp(lo, -(j + 1)), ldexp(lo, -j), hmax, acc);
            } else {
                q.range(kp, hi, hi + 64.0 * q.T, hmax, acc);
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < 3; ++j) {
        const double s = wave_sum(acc[j]);
        if (lane == 0) red[j][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* out = part + ((int64_t)k * gridDim.x + blockIdx.x) * 3;
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int v = 0; v < kEqCells / 64; ++v) s += red[j][v];
            out[j] = s;
        }
    }
}

__global__ void __launch_bounds__(kThreads)
k_eq_final(int nbh, int64_t nseg, int64_t nchunk, const double* __restrict__ pop,
           const double* __restrict__ ref, double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nbh) return;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t sg = 0; sg < nseg; ++sg)
        for (int j = 0; j < 3; ++j) v[j] += pop[(sg * 3 + j) * nbh + k];
    for (int64_t ch = 0; ch < nchunk; ++ch)
        for (int j = 0; j < 3; ++j) v[3 + j] += ref[((int64_t)k * nchunk + ch) * 3 + j];
    for (int j = 0; j < 6; ++j) out[(int64_t)j * nbh + k] = v[j];
    out[(int64_t)6 * nbh + k] = v[2] > 0.0 ? (v[0] - v[5]) / sqrt(v[2]) : 0.0;
}

// ------------------------------------------------------------------ copy calibration
__global__ void __launch_bounds__(kThreads)
k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n4) {
    // four independent 16-byte loads in flight per thread, then the stores
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a; dst[i + stride] = b; dst[i + 2 * stride] = c; dst[i + 3 * stride] = d;
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

// Status of a call whose input buffer is empty: nothing is appended.
__global__ void k_status_empty(int64_t* __restrict__ status, int64_t out_n,
                               const int64_t* __restrict__ chain, int chain_slot) {
    if (threadIdx.x == 0) {
        const bool skip = chain && chain[AXPIC_CHAIN_SKIP] != 0;
        status[0] = (chain && chain_slot >= 0) ? chain[chain_slot] : out_n;
        status[1] = skip ? AXPIC_FLAG_SKIPPED : 0;
        status[2] = 0; status[3] = 0;
    }
}

// ------------------------------------------------------------------ host launch helpers
inline dim3 grid1(int64_t n, int t = kThreads) { return dim3((unsigned)((n + t - 1) / t)); }

const StatMap kEmitMap = {{AXPIC_ST_EVENTS_P, AXPIC_ST_EVENTS_C, AXPIC_ST_EVENTS_B, AXPIC_ST_NUM_P,
                           AXPIC_ST_NUM_C, AXPIC_ST_NUM_B, AXPIC_ST_EN_P, AXPIC_ST_EN_C,
                           AXPIC_ST_EN_B, AXPIC_ST_CAPPED, AXPIC_ST_OVERDEPLETED, -1}};
const StatMap kAbsMap = {{AXPIC_ST_ABS_NUM, AXPIC_ST_ABS_EN, AXPIC_ST_AG_EVENTS, AXPIC_ST_AG_NUM,
                          AXPIC_ST_AG_EN, AXPIC_ST_CAPPED, AXPIC_ST_OVERDEPLETED,
                          AXPIC_ST_ABS_EVENTS, -1, -1, -1, -1}};

template <typename T> inline T* TP(void* p) { return (T*)p; }
template <typename T> inline const T* TCP(const void* p) { return (const T*)p; }

inline IdView idv(const axpic_species* sp) { return IdView{sp->id, sp->id0, sp->n_implicit}; }

// 16-byte alignment of every pointer a count kernel reads with run loads (null counts
// as aligned: it is not read)
inline bool al16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
inline int runs_aligned(std::initializer_list<const void*> ps) {
    for (const void* p : ps)
        if (!al16(p)) return 0;
    return 1;
}

// Smallest FP32 parent weight (in units of w_ref) that is surely not lighter than one
// product of weight wprod, i.e. fl64(wt w_ref) >= wprod for every FP32 wt at or above it;
// 0 when no parent converts as a light one, +inf when none is surely heavy.
inline float heavy_threshold(double wprod, double w_ref, int light_mode) {
    if (light_mode != 0 || !(wprod > 0.0)) return 0.0f;
    if (!(w_ref > 0.0)) return INFINITY;
    const double th = wprod / w_ref * (1.0 + 1e-9);
    if (!(th < 3.0e38)) return INFINITY;
    float f = (float)th;
    if ((double)f < th) f = std::nextafter(f, INFINITY);
    return f;
}

// Largest FP32 parent weight below which a parent is surely lighter than one product:
// fl64(wt w_ref) < wprod for every FP32 wt under it (0: no light parents).
inline float light_threshold(double wprod, double w_ref, int light_mode) {
    if (light_mode != 0 || !(wprod > 0.0)) return 0.0f;
    if (!(w_ref > 0.0)) return INFINITY;
    const double th = wprod / w_ref * (1.0 - 1e-9);
    if (!(th < 3.0e38)) return 3.0e38f;
    float f = (float)th;
    if ((double)f > th) f = std::nextafter(f, 0.0f);
    return f;
}

// wprod / w_ref in FP32 for the light-parent pre-test (+inf when undefined)
inline float product_ratio(double wprod, double w_ref) {
    if (!(w_ref > 0.0) || !(wprod >= 0.0)) return INFINITY;
    const double r = wprod / w_ref;
    return r < 3.0e38 ? (float)r : INFINITY;
}

// The end of the last accumulating kernel: its per-block records (nrec records of ncol
// columns, the first nh of them histogram bins for hist; column-major, column j at
// j nrec) summed into hist and stats, and, with fb, the boundary records of its nb
// blocks added to fb.  ev: an events grid of nrec (= nb) blocks, of which only those
// that got events wrote.
void finish(const Workspace& W, int64_t nrec, int ncol, int nh, double* hist, double* stats,
            int64_t nb, double* fb, hipStream_t s, bool ev) {
    const int cols = (hist || stats) ? ncol : 0;
    const int64_t fbb = fb ? (2 * nb + kThreads - 1) / kThreads : 0;
    if (cols + fbb == 0) return;
    LAUNCH("k_finish", k_finish, dim3((unsigned)(cols + fbb)), dim3(kThreads), 0, s, W.rec, nrec,
           (int64_t)1, nrec, nh, cols, hist, stats, nb, W.bkey, W.bval, fb, W.ctrl, ev ? 1 : 0);
}

struct SpT {   // typed view of a species
    void* x[3]; void* p[3]; void* w; uint64_t* id; int32_t* cell;
};

// Event records of the active-parent lists of nb tiles (after k_scan).
void expand(const Workspace& W, int64_t nb, bool thermal, axpic_species* ax, hipStream_t s) {
    const int64_t g = std::min<int64_t>((nb + kThreads / 64 - 1) / (kThreads / 64), 2048);
    LAUNCH("k_expand", k_expand, dim3((unsigned)g), dim3(kThreads), 0, s, nb, thermal ? 1 : 0,
           W.list(), W.bact, W.boff, W.ctrl, ax->capacity, ax->id);
}

template <typename T>
axpic_status emit_primakoff(const KParams& kp, const axpic_cells* cells, axpic_species* ph,
                            const void* lam_in, int64_t step, uint64_t next_id,
                            axpic_species* ax, double* hist, double* stats, int64_t* status,
                            const Workspace& W, int64_t* chain, hipStream_t s) {
    const int64_t n = ph->n, nb = nblocks_for(std::max<int64_t>(n, 1));
    // massive axions take their own instantiations, so the massless kernels are unchanged
    const auto k_count =
        lam_in ? (kp.massive ? k_prim_count<T, true, kSrcLam> : k_prim_count<T, false, kSrcLam>)
        : kp.massive ? k_prim_count<T, true, kSrcP>
        : ph->p2 ? k_prim_count<T, false, kSrcP2> : k_prim_count<T, false, kSrcP>;
    const auto k_events = kp.massive ? k_prim_events<T, true> : k_prim_events<T, false>;
    LAUNCH("k_prim_count", k_count, dim3((unsigned)nb), dim3(kThreads), 0, s, n, step, kp,
                       ph->w_ref, cells->pref32, cells->pref64, TCP<T>(ph->w), TCP<T>(ph->p[0]),
                       TCP<T>(ph->p[1]), TCP<T>(ph->p[2]), TCP<T>(ph->p2), idv(ph), ph->cell,
                       TCP<T>(lam_in), W.list(), W.bsum, W.bact,
                       runs_aligned({ph->w, ph->p[0], ph->p[1], ph->p[2], ph->p2, ph->cell, ph->id,
                                     lam_in}),
                       heavy_threshold(kp.w_a * kp.wa_mul[0], ph->w_ref, kp.light_mode),
                       ph->off, ph->off ? ph->n_sorted : (int64_t)0);
    LAUNCH("k_scan", k_scan, dim3(1), dim3(kScanThreads), 0, s, W.bsum, W.boff, nb, ax->n,
           ax->capacity, W.ctrl, status, next_id, chain, (int)AXPIC_CHAIN_AXIONS);
    expand(W, nb, false, ax, s);
    const int nbh = kp.nbins + 2;
    LAUNCH("k_prim_events", k_events, dim3(kEventBlocks), dim3(kThreads),
           sizeof(double) * (kThreads / 64) * (size_t)nbh, s, n, step,
           next_id, kp, ph->w_ref, cells->pref32, cells->pref64, TP<T>(ph->w), TCP<T>(ph->x[0]),
           TCP<T>(ph->x[1]), TCP<T>(ph->x[2]), TCP<T>(ph->p[0]), TCP<T>(ph->p[1]),
           TCP<T>(ph->p[2]), ph->cell, TCP<T>(lam_in), W.ctrl, ax->n, TP<T>(ax->x[0]),
           TP<T>(ax->x[1]), TP<T>(ax->x[2]), TP<T>(ax->p[0]), TP<T>(ax->p[1]), TP<T>(ax->p[2]),
           TP<T>(ax->w), ax->id, ax->cell, W.rec, kEmitMap);
    finish(W, kEventBlocks, nbh + AXPIC_ST_COUNT, nbh, hist, stats, kEventBlocks, nullptr, s,
           true);
    return launched();
}

template <typename T>
axpic_status emit_thermal(const KParams& kp, const axpic_cells* cells, axpic_species* el,
                          const void* lam_in, int64_t step, uint64_t next_id, axpic_species* ax,
                          double* fb, double* hist, double* stats, int64_t* status,
                          const Workspace& W, int64_t* chain, hipStream_t s) {
    const int64_t n = el->n, nb = nblocks_for(std::max<int64_t>(n, 1));
    LAUNCH("k_therm_count", k_therm_count<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, n, step, kp,
                       cells->pref32, cells->pref64, TCP<T>(el->w), idv(el), el->cell,
                       TCP<T>(lam_in), W.list(), W.bsum, W.bact,
                       runs_aligned({el->w, el->cell, el->id, lam_in}));
    LAUNCH("k_scan", k_scan, dim3(1), dim3(kScanThreads), 0, s, W.bsum, W.boff, nb, ax->n,
           ax->capacity, W.ctrl, status, next_id, chain, (int)AXPIC_CHAIN_AXIONS);
    expand(W, nb, true, ax, s);
    const auto k_events = kp.massive ? k_therm_events<T, true> : k_therm_events<T, false>;
    const int nbh = kp.nbins + 2;
    LAUNCH("k_therm_events", k_events, dim3(kEventBlocks), dim3(kThreads),
           sizeof(double) * (kThreads / 64) * 2 * (size_t)nbh, s, n, step,
           next_id, kp, cells->pref32, cells->pref64, cells->state, TCP<T>(el->w),
           TCP<T>(el->x[0]), TCP<T>(el->x[1]), TCP<T>(el->x[2]), idv(el), el->cell, TCP<T>(lam_in),
           W.ctrl, ax->n, TP<T>(ax->x[0]), TP<T>(ax->x[1]), TP<T>(ax->x[2]), TP<T>(ax->p[0]),
           TP<T>(ax->p[1]), TP<T>(ax->p[2]), TP<T>(ax->w), ax->id,
                       ax->cell, fb, W.rec, W.bkey, W.bval, kEmitMap);
    finish(W, kEventBlocks, 2 * nbh + AXPIC_ST_COUNT, 2 * nbh, hist ? hist + nbh : nullptr, stats,
           kEventBlocks, fb, s, true);
    return launched();
}

template <typename T>
axpic_status emit_thermal_cells(const KParams& kp, const axpic_cells* cells, axpic_species* el,
                                const int64_t* off, const double* cellw, int64_t step,
                                uint64_t next_id, axpic_species* ax, double* fb, double* hist,
                                double* stats, int64_t* status, const Workspace& W, int64_t* chain, hipStream_t s) {
    const int64_t ncell = cells->ncell, nb = nblocks_for(std::max<int64_t>(ncell, 1));
    uint32_t* counts = (uint32_t*)W.code;
    LAUNCH("k_sup_count", k_sup_count<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, ncell, step, kp,
           cells->pref32, cells->pref64, off, TCP<T>(el->w), cellw, counts, W.bsum, W.bact);
    LAUNCH("k_scan", k_scan, dim3(1), dim3(kScanThreads), 0, s, W.bsum, W.boff, nb, ax->n,
           ax->capacity, W.ctrl, status, next_id, chain, (int)AXPIC_CHAIN_AXIONS);
    LAUNCH("k_sup_expand", k_sup_expand, dim3((unsigned)nb), dim3(kThreads), 0, s, ncell, counts,
           W.bact, W.boff, W.ctrl, ax->n, ax->capacity, ax->id);
    const auto k_events = kp.massive ? k_sup_events<T, true> : k_sup_events<T, false>;
    const int nbh = kp.nbins + 2;
    LAUNCH("k_sup_events", k_events, dim3(kEventBlocks), dim3(kThreads),
           sizeof(double) * (kThreads / 64) * 2 * (size_t)nbh, s, ncell, step,
           next_id, kp, cells->pref32, cells->pref64, cells->state, off, TCP<T>(el->w),
           TCP<T>(el->x[0]), TCP<T>(el->x[1]), TCP<T>(el->x[2]), cellw, W.ctrl, ax->n,
           TP<T>(ax->x[0]), TP<T>(ax->x[1]), TP<T>(ax->x[2]), TP<T>(ax->p[0]), TP<T>(ax->p[1]),
           TP<T>(ax->p[2]), TP<T>(ax->w), ax->id, ax->cell, fb, W.rec, W.bkey, W.bval, kEmitMap);
    finish(W, kEventBlocks, 2 * nbh + AXPIC_ST_COUNT, 2 * nbh, hist ? hist + nbh : nullptr, stats,
           kEventBlocks, fb, s, true);
    return launched();
}

template <typename T>
axpic_status absorb_impl(const KParams& kp, const axpic_cells* cells, axpic_species* ax,
                         const void* pabs_in, const void* lam_in, int64_t step, uint64_t next_id,
                         axpic_species* ph, double* fb, double* stats, int64_t* status,
                         const Workspace& W, int64_t* chain, hipStream_t s) {
    const int64_t n = ax->n, nb = nblocks_for(std::max<int64_t>(n, 1));
    const auto k_count = kp.massive ? k_abs_count<T, true> : k_abs_count<T, false>;
    const auto k_apply = kp.massive ? k_abs_apply<T, true> : k_abs_apply<T, false>;
    LAUNCH("k_abs_count", k_count, dim3((unsigned)nb), dim3(kThreads), 0, s, n, step, kp,
                       ax->w_ref, cells->pref32, cells->pref64, TCP<T>(ax->w), TCP<T>(ax->p[0]),
                       TCP<T>(ax->p[1]), TCP<T>(ax->p[2]), idv(ax), ax->cell, TCP<T>(pabs_in),
                       TCP<T>(lam_in), W.code, W.bsum, W.bact,
                       runs_aligned({ax->w, ax->p[0], ax->p[1], ax->p[2], ax->cell, ax->id, pabs_in,
                                     lam_in, W.code}),
                       heavy_threshold(kp.w_gamma_prod, ax->w_ref, kp.light_mode),
                       light_threshold(kp.w_gamma_prod, ax->w_ref, kp.light_mode),
                       product_ratio(kp.w_gamma_prod, ax->w_ref),
                       ax->off ? std::min<int64_t>(ax->n_sorted, n) : (int64_t)0,
                       (const int64_t*)chain);
    const int64_t out_n = ph ? ph->n : 0, out_cap = ph ? ph->capacity : 0;
    // the exchange in fixed order needs the axions in cell order (as the sort leaves them)
    const bool det = ax->off && ax->n_sorted >= n;
    LAUNCH("k_scan", k_scan, dim3(1), dim3(kScanThreads), 0, s, W.bsum, W.boff, nb, out_n,
           out_cap, W.ctrl, status, next_id, chain, ph ? (int)AXPIC_CHAIN_PHOTONS : -1);
    LAUNCH("k_abs_apply", k_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, n, step, next_id,
                       kp, ax->w_ref, cells->pref32, cells->pref64, TP<T>(ax->w), TCP<T>(ax->x[0]),
                       TCP<T>(ax->x[1]), TCP<T>(ax->x[2]), TCP<T>(ax->p[0]), TCP<T>(ax->p[1]),
                       TCP<T>(ax->p[2]), ax->cell, TCP<T>(pabs_in), TCP<T>(lam_in), W.code, W.bact,
                       W.boff, W.ctrl, out_n, out_cap, ph ? TP<T>(ph->x[0]) : nullptr,
                       ph ? TP<T>(ph->x[1]) : nullptr, ph ? TP<T>(ph->x[2]) : nullptr,
                       ph ? TP<T>(ph->p[0]) : nullptr, ph ? TP<T>(ph->p[1]) : nullptr,
                       ph ? TP<T>(ph->p[2]) : nullptr, ph ? TP<T>(ph->p2) : nullptr,
                       ph ? TP<T>(ph->w) : nullptr,
                       ph ? ph->id : nullptr, ph ? ph->cell : nullptr, ph ? ph->w_ref : 1.0, fb,
                       W.rec, W.bkey, W.bval, det ? 1 : 0, (const int64_t*)chain, kAbsMap);
    finish(W, nb, AXPIC_ST_COUNT, 0, nullptr, stats, nb, det ? fb : nullptr, s, false);
    return launched();
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

const char* axpic_status_string(int32_t s) {
    switch (s) {
    case AXPIC_OK: return "ok";
    case AXPIC_E_INVAL: return "invalid argument";
    case AXPIC_E_CAPACITY: return "output capacity exceeded";
    case AXPIC_E_DOMAIN: return "value outside the model's domain";
    case AXPIC_E_DEVICE: return "HIP launch or runtime failure";
    case AXPIC_E_UNSUPPORTED: return "unsupported configuration";
    case AXPIC_E_SCRATCH: return "input exceeds the static scratch of an allocation-free call";
    default: return "unknown status";
    }
}

int32_t axpic_version(void) { return 1; }

size_t axpic_workspace_bytes(int64_t n_max) { return ws_bytes_for(n_max) + 64 * sizeof(int); }

}  // extern "C"

// ------------------------------------------------------------------ ABI entry points
namespace {
inline hipStream_t S(void* s) { return (hipStream_t)s; }
}

namespace {

struct SortWs {
    uint32_t *cnt, *bsum, *idx;
    uint64_t* boff;
    int64_t *offw, *ctrl;
};

// Workspace layout; returns its size (ws may be NULL to only size it).
size_t sort_ws_layout(int64_t n, int64_t ncell, void* ws, SortWs* W) {
    const int64_t nblk = (ncell + kSortCellsPerBlock - 1) / kSortCellsPerBlock;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += align256(bytes); return at; };
    const size_t o_cnt = take(4 * (size_t)ncell), o_bsum = take(4 * (size_t)nblk),
                 o_boff = take(8 * (size_t)nblk),
                 o_idx = take(4 * (size_t)std::max<int64_t>(n, 1)),
                 o_offw = take(8 * (size_t)(ncell + 1)), o_ctrl = take(256);
    if (ws && W) {
        char* p = (char*)ws;
        W->cnt = (uint32_t*)(p + o_cnt); W->bsum = (uint32_t*)(p + o_bsum);
        W->boff = (uint64_t*)(p + o_boff); W->idx = (uint32_t*)(p + o_idx);
        W->offw = (int64_t*)(p + o_offw); W->ctrl = (int64_t*)(p + o_ctrl);
    }
    return o;
}

template <typename T>
SortIO<T> sort_io(const axpic_grid* g, const axpic_species* in, axpic_species* out) {
    SortIO<T> io;
    io.ndim = 1;
    if (in->x[1] && g->ndim > 1) io.ndim = 2;
    if (in->x[2] && g->ndim > 2) io.ndim = 3;
    for (int d = 0; d < 3; ++d) {
        io.x[d] = (const T*)in->x[d]; io.p[d] = (const T*)in->p[d];
        io.ox[d] = (T*)out->x[d]; io.op[d] = (T*)out->p[d];
    }
    io.w = (const T*)in->w; io.id = idv(in);
    io.ow = (T*)out->w; io.oid = out->id; io.ocell = out->cell;
    return io;
}

// The general sort: counts, offsets, scatter of source indices, gather with ranks.  DENSE
// (many particles per cell) aggregates the atomics per block and walks the slots in
// order; otherwise one atomic per run and the gather's blocks grouped by XCD.
template <typename T, bool DENSE>
void sort_general(const axpic_grid* g, const axpic_species* in, axpic_species* out, int64_t* off,
                  int64_t* status, SortWs& W, int64_t* chain, hipStream_t s) {
    const int64_t ncell = ncell_of(g), n = in->n;
    const int64_t nblk = (ncell + kSortCellsPerBlock - 1) / kSortCellsPerBlock;
    const dim3 nb((unsigned)((n + kSortSlots - 1) / kSortSlots));
    const T* w = (const T*)in->w;
    LAUNCH("k_fill_u32", k_fill_u32, dim3((unsigned)std::min<int64_t>((ncell + kThreads - 1) /
                                                                      kThreads, 8192)),
           dim3(kThreads), 0, s, ncell, W.cnt);
    if (n > 0)
        LAUNCH("k_sort_count", (k_sort_count<T, DENSE>), nb, dim3(kThreads), 0, s, n, ncell, w,
               in->cell, W.cnt);
    LAUNCH("k_sort_blocksum", k_sort_blocksum, dim3((unsigned)nblk), dim3(kThreads), 0, s, ncell,
           W.cnt, W.bsum);
    LAUNCH("k_scan", k_scan, dim3(1), dim3(kScanThreads), 0, s, W.bsum, W.boff, nblk, (int64_t)0,
           out->capacity, W.ctrl, status, (uint64_t)0, chain, -1);
    LAUNCH("k_sort_offsets", k_sort_offsets, dim3((unsigned)nblk), dim3(kThreads), 0, s, ncell,
           W.cnt, W.boff, W.ctrl, off, chain);
    if (n == 0) return;
    LAUNCH("k_sort_scatter", (k_sort_scatter<T, DENSE>), nb, dim3(kThreads), 0, s, n, ncell, w,
           in->cell, (const int64_t*)off, (const int64_t*)W.ctrl, W.cnt, W.idx);
    LAUNCH("k_sort_gather", (k_sort_gather<T, !DENSE>), nb, dim3(kThreads), 0, s, ncell,
           (const int64_t*)off, (const uint32_t*)W.idx, (const int64_t*)W.ctrl, in->cell,
           sort_io<T>(g, in, out));
}

// The general sort's per-block aggregation of its atomics pays from kSortDense particles
// per cell on.
constexpr int64_t kSortDense = 32;

template <typename T>
void sort_launch(const axpic_grid* g, const axpic_species* in, int32_t path, axpic_species* out,
                 int64_t* off, int64_t* status, SortWs& W, int64_t* chain, hipStream_t s) {
    if (path == AXPIC_SORT_AUTO)
        path = in->n >= kSortDense * ncell_of(g) ? AXPIC_SORT_DENSE : AXPIC_SORT_SPARSE;
    if (path == AXPIC_SORT_DENSE)
        sort_general<T, true>(g, in, out, off, status, W, chain, s);
    else
        sort_general<T, false>(g, in, out, off, status, W, chain, s);
}

}  // namespace

extern "C" {

axpic_status axpic_bin_cells(const axpic_grid* g, axpic_species* sp, int32_t push, double m_keV,
                             void* stream) {
    if (!grid_ok(g) || !species_ok(sp, push != 0) || !(m_keV >= 0.0 && m_keV < 1e6))
        return AXPIC_E_INVAL;
    if (sp->n == 0) return AXPIC_OK;
    for (int d = 0; d < g->ndim; ++d)
        if (!sp->x[d]) return AXPIC_E_INVAL;
    if (push && (!sp->p[0] || !sp->p[1] || !sp->p[2])) return AXPIC_E_INVAL;
    axpic_params dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    dummy.m_a_keV = m_keV;
    KParams kp = make_kparams(g, &dummy, 1.0);
    if (sp->dtype == AXPIC_F32)
        LAUNCH("k_bin", k_bin<float>, grid1(sp->n), dim3(kThreads), 0, S(stream), sp->n, kp,
                           push, (float*)sp->x[0], (float*)sp->x[1], (float*)sp->x[2],
                           (const float*)sp->p[0], (const float*)sp->p[1], (const float*)sp->p[2],
                           sp->cell);
    else
        LAUNCH("k_bin", k_bin<double>, grid1(sp->n), dim3(kThreads), 0, S(stream), sp->n, kp,
                           push, (double*)sp->x[0], (double*)sp->x[1], (double*)sp->x[2],
                           (const double*)sp->p[0], (const double*)sp->p[1],
                           (const double*)sp->p[2], sp->cell);
    return launched();
}

axpic_status axpic_deposit(const axpic_grid* g, const axpic_species* sp, const int64_t* off,
                           axpic_cells* cells, int32_t slot, void* stream) {
    if (!grid_ok(g) || !sp || !off || !cells || !cells->dens) return AXPIC_E_INVAL;
    if (slot < 0 || slot > AXPIC_MAX_IONS || cells->ncell != ncell_of(g)) return AXPIC_E_INVAL;
    if (sp->n > 0 && !sp->w) return AXPIC_E_INVAL;
    const double L = g->dx * kC / g->omega0;
    const double scale = sp->w_ref / (L * L * L);
    double* dst = cells->dens + (int64_t)slot * cells->ncell;
    if (sp->dtype == AXPIC_F32)
        LAUNCH("k_deposit", k_deposit<float>, grid1(cells->ncell), dim3(kThreads), 0, S(stream),
                           cells->ncell, (const float*)sp->w, off, scale, dst);
    else
        LAUNCH("k_deposit", k_deposit<double>, grid1(cells->ncell), dim3(kThreads), 0, S(stream),
                           cells->ncell, (const double*)sp->w, off, scale, dst);
    return launched();
}

axpic_status axpic_fill_p2(axpic_species* sp, int64_t from, void* stream) {
    if (!species_ok(sp, true) || !sp->p2 || from < 0 || from > sp->n) return AXPIC_E_INVAL;
    if (from == sp->n) return AXPIC_OK;
    const int64_t m = sp->n - from;
    if (sp->dtype == AXPIC_F32)
        LAUNCH("k_fill_p2", k_fill_p2<float>, grid1(m), dim3(kThreads), 0, S(stream), from, sp->n,
               (const float*)sp->p[0], (const float*)sp->p[1], (const float*)sp->p[2],
               (float*)sp->p2);
    else
        LAUNCH("k_fill_p2", k_fill_p2<double>, grid1(m), dim3(kThreads), 0, S(stream), from,
               sp->n, (const double*)sp->p[0], (const double*)sp->p[1], (const double*)sp->p[2],
               (double*)sp->p2);
    return launched();
}

axpic_status axpic_cell_state(const axpic_grid* g, axpic_cells* cells, const axpic_params* prm,
                              double w_ref_e, double w_ref_g, void* stream) {
    if (!grid_ok(g) || !params_ok(prm) || !cells || cells->ncell != ncell_of(g)) return AXPIC_E_INVAL;
    if (!cells->T_keV || !cells->dens || !cells->state || !cells->pref32 || !cells->pref64)
        return AXPIC_E_INVAL;
    if (cells->nion < 0 || cells->nion > AXPIC_MAX_IONS) return AXPIC_E_INVAL;
    axpic_status st = ensure_tables(prm->brems_k);
    if (st != AXPIC_OK) return st;
    const double dtp = g->dt / g->omega0;
    cells->w_ref_e = w_ref_e;
    cells->w_ref_g = w_ref_g;
    const double* Z = cells->Zion; const double* A = cells->Aion;
    LAUNCH("k_cell_state", k_cell_state, grid1(cells->ncell), dim3(kThreads), 0, S(stream),
                       cells->ncell, cells->T_keV, cells->dens, cells->nion, Z[0], Z[1], Z[2], Z[3],
                       A[0], A[1], A[2], A[3], *prm, dtp, w_ref_e, w_ref_g, cells->state,
                       cells->pref32, cells->pref64);
    return launched();
}

axpic_status axpic_rates(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                         const axpic_species* sp, int32_t channel, void* out, void* stream) {
    if (!grid_ok(g) || !params_ok(prm) || !cells || !species_ok(sp, true) || (!out && sp->n))
        return AXPIC_E_INVAL;
    int mode;
    if (sp->kind == AXPIC_PHOTON && channel == AXPIC_PRIMAKOFF) mode = 0;
    else if (sp->kind == AXPIC_ELECTRON && channel == AXPIC_COMPTON) mode = 1;
    else if (sp->kind == AXPIC_ELECTRON && channel == AXPIC_BREMS) mode = 2;
    else if (sp->kind == AXPIC_AXION && channel != 0 && (channel & ~(AXPIC_COMPTON | AXPIC_BREMS)) == 0) mode = 3;
    else if (sp->kind == AXPIC_AXION && channel == AXPIC_PRIMAKOFF) mode = 4;
    else return AXPIC_E_INVAL;
    if (sp->n == 0) return AXPIC_OK;
    axpic_params p2 = *prm;
    if (mode == 3) p2.channels = prm->channels & channel;
    KParams kp = make_kparams(g, &p2, cells->w_ref_g);
    if (sp->dtype == AXPIC_F32)
        LAUNCH("k_rates", k_rates<float>, grid1(sp->n), dim3(kThreads), 0, S(stream), sp->n, kp,
                           mode, cells->pref32, cells->pref64, (const float*)sp->w,
                           (const float*)sp->p[0], (const float*)sp->p[1], (const float*)sp->p[2],
                           sp->cell, (float*)out);
    else
        LAUNCH("k_rates", k_rates<double>, grid1(sp->n), dim3(kThreads), 0, S(stream), sp->n, kp,
                           mode, cells->pref32, cells->pref64, (const double*)sp->w,
                           (const double*)sp->p[0], (const double*)sp->p[1],
                           (const double*)sp->p[2], sp->cell, (double*)out);
    return launched();
}

axpic_status axpic_sample_emit(const axpic_grid* g, const axpic_cells* cells,
                               const axpic_params* prm, axpic_species* parent, int32_t channels,
                               const void* lam_in, int64_t step, uint64_t next_id,
                               axpic_species* axions, double* fb, double* hist, double* stats,
                               int64_t* status, void* ws, size_t ws_bytes, int64_t* chain,
                               void* stream) {
    if (!grid_ok(g) || !params_ok(prm) || !cells || !status) return AXPIC_E_INVAL;
    if (!species_ok(parent, parent && parent->kind == AXPIC_PHOTON) || !species_ok(axions, false))
        return AXPIC_E_INVAL;
    if (axions->dtype != parent->dtype || axions->kind != AXPIC_AXION) return AXPIC_E_INVAL;
    if (!axions->x[0] || !axions->p[0] || !axions->p[1] || !axions->p[2] || !axions->w ||
        !axions->id || !axions->cell || axions->n_implicit != 0 || !parent->x[0])
        return AXPIC_E_INVAL;
    for (int d = 1; d < g->ndim; ++d)
        if (!axions->x[d] || !parent->x[d]) return AXPIC_E_INVAL;
    Workspace W;
    if (!carve(ws, ws_bytes, parent->n, &W)) return AXPIC_E_INVAL;
    if (std::fabs(axions->w_ref - prm->w_a) > 1e-12 * prm->w_a) return AXPIC_E_INVAL;
    if (parent->n == 0) {
        LAUNCH("k_status_empty", k_status_empty, dim3(1), dim3(64), 0, S(stream), status, axions->n,
               (const int64_t*)chain, (int)AXPIC_CHAIN_AXIONS);
        return launched();
    }
    axpic_status st = ensure_tables(prm->brems_k);
    if (st != AXPIC_OK) return st;
    axpic_params p2 = *prm;
    p2.channels = prm->channels & channels;
    if (parent->kind == AXPIC_PHOTON && std::fabs(parent->w_ref - cells->w_ref_g) > 1e-12 * parent->w_ref)
        return AXPIC_E_INVAL;
    if (parent->kind == AXPIC_ELECTRON && std::fabs(parent->w_ref - cells->w_ref_e) > 1e-12 * parent->w_ref)
        return AXPIC_E_INVAL;
    KParams kp = make_kparams(g, &p2, cells->w_ref_g);
    const bool f64 = parent->dtype == AXPIC_F64;
    if (parent->kind == AXPIC_PHOTON) {
        if (!(p2.channels & AXPIC_PRIMAKOFF)) return AXPIC_E_INVAL;
        return f64 ? emit_primakoff<double>(kp, cells, parent, lam_in, step, next_id, axions, hist,
                                            stats, status, W, chain, S(stream))
                   : emit_primakoff<float>(kp, cells, parent, lam_in, step, next_id, axions, hist,
                                           stats, status, W, chain, S(stream));
    }
    if (parent->kind == AXPIC_ELECTRON) {
        if (!(p2.channels & (AXPIC_COMPTON | AXPIC_BREMS))) return AXPIC_E_INVAL;
        return f64 ? emit_thermal<double>(kp, cells, parent, lam_in, step, next_id, axions, fb,
                                          hist, stats, status, W, chain, S(stream))
                   : emit_thermal<float>(kp, cells, parent, lam_in, step, next_id, axions, fb, hist,
                                         stats, status, W, chain, S(stream));
    }
    return AXPIC_E_INVAL;
}

axpic_status axpic_cell_weights(const axpic_species* el, const int64_t* off, int64_t ncell,
                                double* out, void* stream) {
    if (!el || !off || !out || ncell <= 0 || !el->w || el->n < 0) return AXPIC_E_INVAL;
    if (el->dtype != AXPIC_F32 && el->dtype != AXPIC_F64) return AXPIC_E_INVAL;
    const int64_t threads = ncell * kCellLanes;
    if (el->dtype == AXPIC_F32)
        LAUNCH("k_cell_weights", k_cell_weights<float>, grid1(threads), dim3(kThreads), 0, S(stream),
               ncell, off, (const float*)el->w, out);
    else
        LAUNCH("k_cell_weights", k_cell_weights<double>, grid1(threads), dim3(kThreads), 0, S(stream),
               ncell, off, (const double*)el->w, out);
    return launched();
}

axpic_status axpic_sample_emit_cells(const axpic_grid* g, const axpic_cells* cells,
                                     const axpic_params* prm, axpic_species* electrons,
                                     const int64_t* off, const double* cellw, int32_t channels,
                                     int64_t step, uint64_t next_id, axpic_species* axions,
                                     double* fb, double* hist, double* stats, int64_t* status,
                                     void* ws, size_t ws_bytes, int64_t* chain, void* stream) {
    if (!grid_ok(g) || !params_ok(prm) || !cells || !status || !off || !cellw) return AXPIC_E_INVAL;
    if (!species_ok(electrons, false) || electrons->kind != AXPIC_ELECTRON || !electrons->x[0])
        return AXPIC_E_INVAL;
    if (!species_ok(axions, false) || axions->kind != AXPIC_AXION ||
        axions->dtype != electrons->dtype)
        return AXPIC_E_INVAL;
    if (!axions->x[0] || !axions->p[0] || !axions->p[1] || !axions->p[2] || !axions->w ||
        !axions->id || !axions->cell || axions->n_implicit != 0)
        return AXPIC_E_INVAL;
    for (int d = 1; d < g->ndim; ++d)
        if (!axions->x[d] || !electrons->x[d]) return AXPIC_E_INVAL;
    if (!cells->state || !cells->pref32 || !cells->pref64 || cells->ncell <= 0) return AXPIC_E_INVAL;
    if (cells->ncell >= ((int64_t)1 << 32)) return AXPIC_E_INVAL;
    if (std::fabs(axions->w_ref - prm->w_a) > 1e-12 * prm->w_a) return AXPIC_E_INVAL;
    if (std::fabs(electrons->w_ref - cells->w_ref_e) > 1e-12 * electrons->w_ref) return AXPIC_E_INVAL;
    Workspace W;
    if (!carve(ws, ws_bytes, 4 * cells->ncell, &W)) return AXPIC_E_INVAL;
    axpic_params p2 = *prm;
    p2.channels = prm->channels & channels & (AXPIC_COMPTON | AXPIC_BREMS);
    if (!p2.channels) return AXPIC_E_INVAL;
    axpic_status st = ensure_tables(prm->brems_k);
    if (st != AXPIC_OK) return st;
    KParams kp = make_kparams(g, &p2, cells->w_ref_g);
    return electrons->dtype == AXPIC_F64
               ? emit_thermal_cells<double>(kp, cells, electrons, off, cellw, step, next_id, axions,
                                            fb, hist, stats, status, W, chain, S(stream))
               : emit_thermal_cells<float>(kp, cells, electrons, off, cellw, step, next_id, axions,
                                           fb, hist, stats, status, W, chain, S(stream));
}

axpic_status axpic_absorb(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                          axpic_species* axions, const void* pabs_in, const void* lam_in,
                          int64_t step, uint64_t next_id, axpic_species* photons, double* fb,
                          double* stats, int64_t* status, void* ws, size_t ws_bytes,
                          int64_t* chain, void* stream) {
    if (!grid_ok(g) || !params_ok(prm) || !cells || !status) return AXPIC_E_INVAL;
    if (!species_ok(axions, true) || axions->kind != AXPIC_AXION) return AXPIC_E_INVAL;
    const bool a2g = prm->inverse && (prm->channels & AXPIC_PRIMAKOFF);
    if (a2g) {
        if (!species_ok(photons, true) || photons->kind != AXPIC_PHOTON ||
            photons->dtype != axions->dtype || !photons->x[0] || !photons->w || !photons->id ||
            !photons->cell || !photons->p[0] || !photons->p[1] || !photons->p[2])
            return AXPIC_E_INVAL;
        for (int d = 1; d < g->ndim; ++d)
            if (!photons->x[d]) return AXPIC_E_INVAL;
    }
    for (int d = 0; d < g->ndim; ++d)
        if (axions->n && !axions->x[d]) return AXPIC_E_INVAL;
    Workspace W;
    if (!carve(ws, ws_bytes, axions->n, &W)) return AXPIC_E_INVAL;
    if (axions->n == 0) {
        LAUNCH("k_status_empty", k_status_empty, dim3(1), dim3(64), 0, S(stream), status,
               a2g ? photons->n : 0, (const int64_t*)chain, a2g ? (int)AXPIC_CHAIN_PHOTONS : -1);
        return launched();
    }
    if (a2g && std::fabs(photons->w_ref - cells->w_ref_g) > 1e-12 * photons->w_ref)
        return AXPIC_E_INVAL;
    if (std::fabs(axions->w_ref - prm->w_a) > 1e-12 * prm->w_a) return AXPIC_E_INVAL;
    KParams kp = make_kparams(g, prm, cells->w_ref_g);
    axpic_species* ph = a2g ? photons : nullptr;
    if (axions->dtype == AXPIC_F64)
        return absorb_impl<double>(kp, cells, axions, pabs_in, lam_in, step, next_id, ph, fb, stats,
                                   status, W, chain, S(stream));
    return absorb_impl<float>(kp, cells, axions, pabs_in, lam_in, step, next_id, ph, fb, stats,
                              status, W, chain, S(stream));
}

axpic_status axpic_feedback(const axpic_grid* g, axpic_cells* cells, const axpic_params* prm,
                            axpic_species* el, const int64_t* off, const double* fb,
                            double* moments, double* stats, void* ws, size_t ws_bytes,
                            int64_t* chain, void* stream) {
    if (!grid_ok(g) || !params_ok(prm) || !cells || !off || !cells->T_keV) return AXPIC_E_INVAL;
    if (!species_ok(el, true) || el->kind != AXPIC_ELECTRON) return AXPIC_E_INVAL;
    if (cells->ncell != ncell_of(g)) return AXPIC_E_INVAL;
    KParams kp = make_kparams(g, prm, 0.0);
    // eight lanes per cell where the cells hold fewer than 48 electrons on average
    const bool narrow = el->n < 48 * cells->ncell;
    const int64_t ncell = cells->ncell, threads = ncell;   // one lane per cell to find the work
    // with statistics: one FP64 slot per cell (the per-parent region of a workspace for 2
    // ncell parents) and a flag word stamped with a token of this call
    double* ecell = nullptr;
    double* part = nullptr;
    int64_t* flag = nullptr;
    unsigned int* done = nullptr;
    static std::atomic<int64_t> next_token{1};
    const int64_t token = next_token.fetch_add(1) | (int64_t)1 << 62;
    if (stats) {
        Workspace W;
        if (!carve(ws, ws_bytes, 2 * ncell, &W)) return AXPIC_E_INVAL;
        ecell = (double*)W.code;
        part = W.rec;
        flag = W.ctrl + 7;
        done = (unsigned int*)(W.ctrl + 6);
    }
    hipStream_t s = S(stream);
    if (el->dtype == AXPIC_F32)
        LAUNCH("k_feedback", (narrow ? k_feedback<float, 8> : k_feedback<float, 16>),
               grid1(threads), dim3(kThreads), 0, s, ncell, kp,
               el->w_ref, off, (const float*)el->w, (float*)el->p[0], (float*)el->p[1],
               (float*)el->p[2], fb, cells->T_keV, moments, stats, ecell, flag, token, done,
               (const int64_t*)chain);
    else
        LAUNCH("k_feedback", (narrow ? k_feedback<double, 8> : k_feedback<double, 16>),
               grid1(threads), dim3(kThreads), 0, s, ncell, kp,
               el->w_ref, off, (const double*)el->w, (double*)el->p[0], (double*)el->p[1],
               (double*)el->p[2], fb, cells->T_keV, moments, stats, ecell, flag, token, done,
               (const int64_t*)chain);
    if (stats)
        LAUNCH("k_fb_unapplied", k_fb_unapplied, dim3(kFbParts), dim3(kThreads), 0, s, ncell,
               ecell, (const int64_t*)flag, token, (const int64_t*)chain, part, done, stats);
    return launched();
}

axpic_status axpic_compact(const axpic_species* in, axpic_species* out, int64_t* status, void* ws,
                           size_t ws_bytes, void* stream) {
    if (!species_ok(in, true) || !out || !status || out->dtype != in->dtype) return AXPIC_E_INVAL;
    if (out->capacity < in->n || !out->x[0] || !out->w || !out->id || !out->cell || !out->p[0] ||
        !out->p[1] || !out->p[2] || !in->x[0])
        return AXPIC_E_INVAL;
    int ndim = 1;
    if (in->x[1]) { ndim = 2; if (!out->x[1]) return AXPIC_E_INVAL; }
    if (in->x[2]) { ndim = 3; if (!in->x[1] || !out->x[2]) return AXPIC_E_INVAL; }
    Workspace W;
    if (!carve(ws, ws_bytes, in->n, &W)) return AXPIC_E_INVAL;
    if (in->n == 0) {
        LAUNCH("k_status_empty", k_status_empty, dim3(1), dim3(64), 0, S(stream), status, (int64_t)0,
               (const int64_t*)nullptr, 0);
        return launched();
    }
    const int64_t n = in->n, nb = nblocks_for(std::max<int64_t>(n, 1));
    hipStream_t s = S(stream);
#define AXPIC_COMPACT(T)                                                                           \
    LAUNCH("k_live_count", k_live_count<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, n,              \
                       (const T*)in->w, W.code, W.bsum, W.bact);                                   \
    LAUNCH("k_scan", k_scan, dim3(1), dim3(kScanThreads), 0, s, W.bsum, W.boff, nb, (int64_t)0, \
           out->capacity, W.ctrl, status, (uint64_t)0, (int64_t*)nullptr, 0);                       \
    LAUNCH("k_compact_apply", k_compact_apply<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, n, W.code,   \
                       W.boff, W.ctrl, out->capacity, ndim, (const T*)in->x[0],                   \
                       (const T*)in->x[1], (const T*)in->x[2], (const T*)in->p[0],                \
                       (const T*)in->p[1], (const T*)in->p[2], (const T*)in->w, idv(in), in->cell, \
                       (const T*)in->p2, (T*)out->x[0], (T*)out->x[1], (T*)out->x[2],             \
                       (T*)out->p[0], (T*)out->p[1], (T*)out->p[2], (T*)out->w, out->id, out->cell, \
                       (T*)out->p2)
    if (in->dtype == AXPIC_F32) { AXPIC_COMPACT(float); }
    else { AXPIC_COMPACT(double); }
#undef AXPIC_COMPACT
    return launched();
}


size_t axpic_sort_ws_bytes(const axpic_grid* g, int64_t n) {
    if (!grid_ok(g) || n < 0) return 0;
    return sort_ws_layout(n, ncell_of(g), nullptr, nullptr);
}

axpic_status axpic_sort_cells(const axpic_grid* g, const axpic_species* in, int32_t path,
                              axpic_species* out, int64_t* off, int64_t* status, void* ws,
                              size_t ws_bytes, int64_t* chain, void* stream) {
    if (!grid_ok(g) || !species_ok(in, true) || !out || !status) return AXPIC_E_INVAL;
    if (out->dtype != in->dtype || out == in || !out->x[0] || !out->w || !out->id || !out->cell ||
        !out->p[0] || !out->p[1] || !out->p[2])
        return AXPIC_E_INVAL;
    // the gather reads `in` while it writes `out`: no array may be shared
    if (out->w == in->w || out->x[0] == in->x[0] || out->p[0] == in->p[0] ||
        out->cell == in->cell || (in->id && out->id == in->id))
        return AXPIC_E_INVAL;
    for (int d = 0; d < g->ndim; ++d)
        if ((in->n && !in->x[d]) || !out->x[d]) return AXPIC_E_INVAL;
    if (in->n >= ((int64_t)1 << 32)) return AXPIC_E_INVAL;
    if (path < AXPIC_SORT_AUTO || path > AXPIC_SORT_DENSE) return AXPIC_E_INVAL;
    if (!ws || ws_bytes < axpic_sort_ws_bytes(g, in->n)) return AXPIC_E_INVAL;
    SortWs W;
    sort_ws_layout(in->n, ncell_of(g), ws, &W);
    if (!off) off = W.offw;
    hipStream_t s = S(stream);
    if (in->dtype == AXPIC_F32)
        sort_launch<float>(g, in, path, out, off, status, W, chain, s);
    else
        sort_launch<double>(g, in, path, out, off, status, W, chain, s);
    return launched();
}

axpic_status axpic_diag(const axpic_species* sp, double m_keV, double* out, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!species_ok(sp, true) || !out || !(m_keV >= 0.0)) return AXPIC_E_INVAL;
    const double mu2 = (m_keV / kMe) * (m_keV / kMe);
    const int64_t nb = nblocks_for(std::max<int64_t>(sp->n, 1));
    if (!ws || ws_bytes < sizeof(double) * 2 * (size_t)nb) return AXPIC_E_INVAL;
    double* part = (double*)ws;
    hipStream_t s = S(stream);
    if (sp->dtype == AXPIC_F32)
        LAUNCH("k_diag_partial", k_diag_partial<float>, dim3((unsigned)nb), dim3(kThreads), 0, s, sp->n,
                           sp->w_ref, mu2, (const float*)sp->w, (const float*)sp->p[0],
                           (const float*)sp->p[1], (const float*)sp->p[2], part);
    else
        LAUNCH("k_diag_partial", k_diag_partial<double>, dim3((unsigned)nb), dim3(kThreads), 0, s, sp->n,
                           sp->w_ref, mu2, (const double*)sp->w, (const double*)sp->p[0],
                           (const double*)sp->p[1], (const double*)sp->p[2], part);
    LAUNCH("k_diag_final", k_diag_final, dim3(1), dim3(64), 0, s, nb, part, out);
    return launched();
}

size_t axpic_equilibrium_ws_bytes(int64_t n, int64_t ncell, int32_t nbins) {
    if (n < 0 || ncell < 0 || nbins < 1) return 0;
    const int64_t nbh = nbins + 2;
    const int64_t nseg = std::max<int64_t>((n + kEqSeg - 1) / kEqSeg, 1);
    const int64_t nchunk = std::max<int64_t>((ncell + kEqCells - 1) / kEqCells, 1);
    return align256(sizeof(double) * (size_t)(nseg * 3 * nbh)) +
           align256(sizeof(double) * (size_t)(nchunk * 3 * nbh));
}

axpic_status axpic_equilibrium(const axpic_grid* g, const axpic_cells* cells, const axpic_params* prm,
                               const axpic_species* sp, double t_steps, double* out, void* ws,
                               size_t ws_bytes, void* stream) {
    if (!grid_ok(g) || !params_ok(prm) || !cells || !out || !species_ok(sp, true))
        return AXPIC_E_INVAL;
    if (cells->ncell != ncell_of(g) || !cells->pref64) return AXPIC_E_INVAL;
    if (!(t_steps == t_steps)) return AXPIC_E_INVAL;
    const int64_t n = sp->n, ncell = cells->ncell;
    const int nbh = prm->hist_nbins + 2;
    if (!ws || ws_bytes < axpic_equilibrium_ws_bytes(n, ncell, prm->hist_nbins)) return AXPIC_E_INVAL;
    const int64_t nseg = std::max<int64_t>((n + kEqSeg - 1) / kEqSeg, 1);
    const int64_t nchunk = std::max<int64_t>((ncell + kEqCells - 1) / kEqCells, 1);
    if (nchunk > 2147483647 || nseg > 2147483647) return AXPIC_E_INVAL;
    double* pop = (double*)ws;
    double* ref = (double*)((char*)ws + align256(sizeof(double) * (size_t)(nseg * 3 * nbh)));
    KParams kp = make_kparams(g, prm, cells->w_ref_g);
    const double L = g->dx * kC / g->omega0;
    hipStream_t s = S(stream);
    const size_t shm = sizeof(double) * 3 * (size_t)nbh;
    if (sp->dtype == AXPIC_F32)
        LAUNCH("k_eq_pop", k_eq_pop<float>, dim3((unsigned)nseg), dim3(64), shm, s, n, kp, sp->w_ref,
               (const float*)sp->w, (const float*)sp->p[0], (const float*)sp->p[1],
               (const float*)sp->p[2], pop);
    else
        LAUNCH("k_eq_pop", k_eq_pop<double>, dim3((unsigned)nseg), dim3(64), shm, s, n, kp, sp->w_ref,
               (const double*)sp->w, (const double*)sp->p[0], (const double*)sp->p[1],
               (const double*)sp->p[2], pop);
    LAUNCH("k_eq_ref", k_eq_ref, dim3((unsigned)nchunk, (unsigned)nbh), dim3(kEqCells), 0, s, ncell,
           kp, cells->pref64, L * L * L, t_steps, prm->hist_lo_keV, prm->hist_hi_keV, ref);
    LAUNCH("k_eq_final", k_eq_final, grid1(nbh), dim3(kThreads), 0, s, nbh, nseg, nchunk, pop, ref,
           out);
    return launched();
}

axpic_status axpic_diag_noalloc(const axpic_species* sp, double m_keV, double* out, void* stream) {
    if (!species_ok(sp, true) || !out || !(m_keV >= 0.0)) return AXPIC_E_INVAL;
    const int64_t nb = nblocks_for(std::max<int64_t>(sp->n, 1));
    if (nb > kDiagScratchPairs) return AXPIC_E_SCRATCH;
    double* part = nullptr;
    {
        // the scratch array's device address on the current device, looked up once
        static std::mutex mu;
        static std::vector<double*> addr;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return AXPIC_E_DEVICE;
        std::lock_guard<std::mutex> lock(mu);
        if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
        if (!addr[dev]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
                return AXPIC_E_DEVICE;
            addr[dev] = (double*)ptr;
        }
        part = addr[dev];
    }
    const double mu2 = (m_keV / kMe) * (m_keV / kMe);
    hipStream_t s = S(stream);
    // every partial the final sum reads is written first by its block: nothing to clear
    if (sp->dtype == AXPIC_F32)
        LAUNCH("k_diag_partial", k_diag_partial<float>, dim3((unsigned)nb), dim3(kThreads), 0, s, sp->n,
               sp->w_ref, mu2, (const float*)sp->w, (const float*)sp->p[0], (const float*)sp->p[1],
               (const float*)sp->p[2], part);
    else
        LAUNCH("k_diag_partial", k_diag_partial<double>, dim3((unsigned)nb), dim3(kThreads), 0, s, sp->n,
               sp->w_ref, mu2, (const double*)sp->w, (const double*)sp->p[0], (const double*)sp->p[1],
               (const double*)sp->p[2], part);
    LAUNCH("k_diag_final", k_diag_final, dim3(1), dim3(64), 0, s, nb, part, out);
    return launched();
}

axpic_status axpic_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
        return AXPIC_E_INVAL;
    const int64_t n4 = (int64_t)(bytes / 16);
    if (n4 == 0) return AXPIC_OK;
    const int64_t blocks = std::min<int64_t>((n4 + kThreads - 1) / kThreads, 256 * 64);
    LAUNCH("k_stream_copy", k_stream_copy, dim3((unsigned)blocks), dim3(kThreads), 0, S(stream),
           (const float4*)src, (float4*)dst, n4);
    return launched();
}

/* Host-side access to the sampler tables (no device work): which = 0 Compton,
 * 1 Gamma(k).  out has 2 (2048 + 1) doubles: y = ln x on the z grid, then dy/dz. */
axpic_status axpic_sampler_table(int32_t which, double k, double* out) {
    if (!out || (which != 0 && which != 1) || (which == 1 && !(k > 0.0))) return AXPIC_E_INVAL;
    if (which == 0) axpic_host::build_compton_table(out);
    else axpic_host::build_gamma_table(out, k);
    return AXPIC_OK;
}

}  // extern "C"

namespace axpic_timing {
bool begin(const char* name, hipEvent_t ev[4]) {
    TimingState& t = timing();
    std::lock_guard<std::mutex> lock(t.mu);
    if (!t.on || (!t.only.empty() && t.only != name)) return false;
    for (int k = 0; k < 4; ++k) {
        ev[k] = pool_get(t);
        if (!ev[k]) {
            for (int j = 0; j < k; ++j) t.pool.push_back(ev[j]);
            return false;
        }
    }
    t.pending.push_back({name, ev[0], ev[1], ev[2], ev[3]});
    return true;
}
}  // namespace axpic_timing

extern "C" {

void axpic_timing_enable(int32_t on) {
    TimingState& t = timing();
    std::lock_guard<std::mutex> lock(t.mu);
    t.on = on != 0;
}

void axpic_timing_only(const char* name) {
    TimingState& t = timing();
    std::lock_guard<std::mutex> lock(t.mu);
    t.only = name ? name : "";
}

axpic_status axpic_timing_read(char* buf, size_t len) {
    TimingState& t = timing();
    std::lock_guard<std::mutex> lock(t.mu);
    hipEvent_t prev_stop = nullptr;
    for (auto& p : t.pending) {
        // the dispatch's own events give the kernel's duration, but their start has been
        // seen to lie far too early on a queue shared with other work; the stream markers
        // around the launch bound the duration from above, and so does the time from the
        // previous launch's end to this one's (launches in order on one stream): the
        // smallest is kept (the last bound fails only across an idle gap, where the
        // dispatch's own start is right)
        float ms = 0.0f, mm = 0.0f;
        if (hipEventSynchronize(p.mb) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess ||
            hipEventElapsedTime(&mm, p.ma, p.mb) != hipSuccess)
            return AXPIC_E_DEVICE;
        ms = std::min(ms, mm);
        float mc = 0.0f;
        if (prev_stop && hipEventElapsedTime(&mc, prev_stop, p.b) == hipSuccess && mc > 0.0f)
            ms = std::min(ms, mc);
        prev_stop = p.b;
        bool found = false;
        for (auto& e : t.acc)
            if (e.first == p.name) { e.second.first += 1; e.second.second += ms; found = true; break; }
        if (!found) t.acc.push_back({p.name, {1, (double)ms}});
        t.pool.push_back(p.a); t.pool.push_back(p.b); t.pool.push_back(p.ma); t.pool.push_back(p.mb);
    }
    t.pending.clear();
    if (!buf || len == 0) return AXPIC_E_INVAL;
    std::string out;
    char line[256];
    for (auto& e : t.acc) {
        std::snprintf(line, sizeof(line), "%s %lld %.6f\n", e.first.c_str(), e.second.first, e.second.second);
        out += line;
    }
    t.acc.clear();
    std::snprintf(buf, len, "%s", out.c_str());
    return out.size() < len ? AXPIC_OK : AXPIC_E_CAPACITY;
}

}  // extern "C"
