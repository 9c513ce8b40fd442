// Exact SURE threshold by histogram refinement.
//
// For coefficients b_1..b_N of one component the risk estimate of soft
// thresholding at unit noise is SURE(t) = N - 2 #{|b| <= t} + sum min(b^2, t^2).
// Between consecutive candidates t in {0} U {|b_k|} it increases with t, so the
// minimum is attained on the candidate set.
//
// The magnitude |b| is keyed by its IEEE bit pattern (monotone for
// non-negative numbers).  Each pass histograms the keys inside the current
// range [klo, khi) into 4096 bins of width 2^shift, recording per bin the
// count, the sum of squares and the smallest and largest key.  The select
// step then knows exactly, for every bin:
//   C = #values below the bin, S = their sum of squares;
//   SURE at the largest value of the bin, t_max (an exact candidate):
//     N - 2(C + c) + S + s + (N - C - c) t_max^2;
//   a lower bound over every candidate t in the bin:
//     N - 2(C + c) + S + (N - C) t_min^2.
// Bins whose lower bound exceeds the best exact value seen are discarded.
// When the surviving bins hold at most kSureCap values, the next pass
// collects exactly those values and the finish sorts them and evaluates SURE
// at every one of them: the count and sum of squares of the values not above
// it are the totals below its bin plus those of its own bin up to it.
// Otherwise the next pass refines the key range spanned by the surviving bins
// (bins of width 1 are exact too).  The smallest minimising candidate is
// returned.
//
// One kernel per pass: blocks of 1024 threads take 16384 coefficients of one
// component each and merge their histogram into the component's bins; the
// last block of the component to finish (a counter, with device-scope fences
// around it) then runs the select, or the finish after a gather pass.
#include "hyres_internal.hpp"

namespace hyres {

template <typename T> struct KeyTraits;
template <> struct KeyTraits<float> {
    typedef uint32_t K;
    static constexpr uint64_t kEnd = 0x80000000ull;
    static constexpr int kRounds = kSureRoundsF32;
    __device__ static K key(float v) { return __float_as_uint(v) & 0x7fffffffu; }
    __device__ static double val(uint64_t k) { return (double)__uint_as_float((uint32_t)k); }
};
template <> struct KeyTraits<double> {
    typedef unsigned long long K;
    static constexpr uint64_t kEnd = 0x8000000000000000ull;
    static constexpr int kRounds = kSureRoundsF64;
    __device__ static K key(double v) {
        return (unsigned long long)__double_as_longlong(v) & 0x7fffffffffffffffull;
    }
    __device__ static double val(uint64_t k) { return __longlong_as_double((long long)k); }
};

constexpr int kSureThreads = 1024;                    // threads of a pass block
constexpr int kSureWaves = kSureThreads / 64;
constexpr int kSureChunk = 16 * kSureThreads;         // smallest work item (coefficients)
constexpr int kGatherPer = 16;                        // gathered coefficients per thread and step
constexpr int kBinsPer = kSureBins / kSureThreads;    // bins per thread in the select
constexpr int kSureGroup = 4;   // chunks per block after the first pass (fewer partial merges)
constexpr int64_t kSureGroupSpan = 65536;   // ... while a block's range stays within this many values

__host__ __device__ inline int sure_shift_for(uint64_t span) {
    int s = 0;
    while (((span + ((1ull << s) - 1)) >> s) > (uint64_t)kSureBins) ++s;
    return s;
}

__device__ __forceinline__ int64_t sure_count(const CubeDesc& d) {
    return d.scope == HYRES_SCOPE_DETAIL ? d.ll_off : d.nc;
}

// counters of component comp: [0] blocks done in this pass, [1] values gathered, [2..3] exact zeros
__device__ __forceinline__ unsigned long long* sure_zeros(const CubeDesc& d, int comp) {
    return reinterpret_cast<unsigned long long*>(d.sctr + 4 * comp + 2);
}

// Field-by-field store of a search state (a struct copy from LDS to global
// memory would go through a private temporary, which the compiler places in
// LDS indexed by the flat thread id, read from the dispatch packet).
__device__ __forceinline__ void put_state(SureState* dst, const SureState& s) {
    dst->klo = s.klo;
    dst->khi = s.khi;
    dst->width = s.width;
    dst->below_cnt = s.below_cnt;
    dst->below_sum = s.below_sum;
    dst->best_s = s.best_s;
    dst->best_t = s.best_t;
    dst->pad0 = s.pad0;
    dst->round = s.round;
    dst->done = s.done;
    dst->inexact = s.inexact;
    dst->gather = s.gather;
    dst->nsurv = s.nsurv;
    dst->pad = s.pad;
}

// Reset the search state, the counters and the global bins of every component.
template <typename T>
__global__ void k_sure_init(const CubeDesc* __restrict__ descs, const int* __restrict__ items, int ncubes) {
    typedef KeyTraits<T> KT;
    const int total = items[ncubes];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int comp = item - items[c];
        const int64_t base = (int64_t)comp * kSureBins;
        for (int b = threadIdx.x; b < kSureBins; b += blockDim.x) {
            gmem(d.hcnt)[base + b] = 0;
            gmem(d.hsum)[base + b] = 0.0;
            gmem(d.hmin)[base + b] = ~0ull;
            gmem(d.hmax)[base + b] = 0;
        }
        if (threadIdx.x < 4) gmem(d.sctr)[4 * comp + threadIdx.x] = 0u;
        if (threadIdx.x == 0) {
            SureState st;
            st.klo = 0;
            st.khi = KT::kEnd;
            st.width = sure_shift_for(KT::kEnd);
            st.below_cnt = 0;
            st.below_sum = 0.0;
            st.best_s = __builtin_inf();
            st.best_t = 0.0;
            st.pad0 = 0;
            st.round = 0;
            st.done = 0;
            st.inexact = 0;
            st.gather = 0;
            st.nsurv = 0;
            st.pad = 0;
            d.sst[comp] = st;
        }
    }
}

// ---- wave primitives (whole wave active) ----
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
// Inclusive prefix sums over the 64 lanes: rows by DPP row shifts, then the
// totals of the rows before (fixed order).
__device__ __forceinline__ uint32_t wave_incl_u32(uint32_t v) {
    v += dpp_u32<0x111>(v);
    v += dpp_u32<0x112>(v);
    v += dpp_u32<0x114>(v);
    v += dpp_u32<0x118>(v);
    const uint32_t t0 = readlane_u32(v, 15), t1 = readlane_u32(v, 31), t2 = readlane_u32(v, 47);
    const int row = (threadIdx.x & 63) >> 4;
    uint32_t off = row >= 1 ? t0 : 0u;
    off += row >= 2 ? t1 : 0u;
    off += row >= 3 ? t2 : 0u;
    return v + off;
}
__device__ __forceinline__ double wave_incl_f64(double v) {
    v += dpp_shift_f64<0x111>(v);
    v += dpp_shift_f64<0x112>(v);
    v += dpp_shift_f64<0x114>(v);
    v += dpp_shift_f64<0x118>(v);
    const double t0 = readlane_f64(v, 15), t1 = readlane_f64(v, 31), t2 = readlane_f64(v, 47);
    const int row = (threadIdx.x & 63) >> 4;
    double off = row >= 1 ? t0 : 0.0;
    off = row >= 2 ? off + t1 : off;
    off = row >= 3 ? off + t2 : off;
    return v + off;
}
// (value, t) pairs: smaller value, then smaller t, over the wave (every lane gets it)
__device__ __forceinline__ void wave_argmin(double& b, double& t) {
#define HYRES_AM(CTRL)                                                 \
    {                                                                  \
        const double ob = dpp_f64<CTRL>(b), ot = dpp_f64<CTRL>(t);    \
        if (ob < b || (ob == b && ot < t)) { b = ob; t = ot; }         \
    }
    HYRES_AM(0xB1) HYRES_AM(0x4E) HYRES_AM(0x141) HYRES_AM(0x140)
#undef HYRES_AM
    double bb = readlane_f64(b, 0), tt = readlane_f64(t, 0);
    for (int r = 16; r < 64; r += 16) {
        const double ob = readlane_f64(b, r), ot = readlane_f64(t, r);
        if (ob < bb || (ob == bb && ot < tt)) { bb = ob; tt = ot; }
    }
    b = bb;
    t = tt;
}
template <bool MAX>
__device__ __forceinline__ int wave_minmax_i32(int v) {
#define HYRES_MM(CTRL)                                                         \
    {                                                                          \
        const int o = (int)dpp_u32<CTRL>((uint32_t)v);                          \
        v = MAX ? (o > v ? o : v) : (o < v ? o : v);                           \
    }
    HYRES_MM(0xB1) HYRES_MM(0x4E) HYRES_MM(0x141) HYRES_MM(0x140)
#undef HYRES_MM
    int r = __builtin_amdgcn_readlane(v, 0);
    for (int l = 16; l < 64; l += 16) {
        const int o = __builtin_amdgcn_readlane(v, l);
        r = MAX ? (o > r ? o : r) : (o < r ? o : r);
    }
    return r;
}

// LDS of a pass block: the histogram of its chunk, or the keys of the finish.
template <typename T> struct SureLds {
    typedef typename KeyTraits<T>::K K;
    static constexpr size_t kHist = (size_t)kSureBins * (4 + 8 + 2 * sizeof(K));
    static constexpr size_t kFinish = (size_t)kSureBins * 8 + 16 + (size_t)kSureCap * 8;
    static constexpr size_t kBytes = kHist > kFinish ? kHist : kFinish;
};

// Small per-block state.
struct SureShared {
    SureState st;
    uint32_t wc[kSureWaves], wm[kSureWaves];
    double ws[kSureWaves], bs[kSureWaves], bt[kSureWaves];
    int wf[kSureWaves], wl[kSureWaves], wx[kSureWaves];
    uint32_t bits[kSureBins / 32];
    unsigned long long zeros;
    uint32_t base;
    int last;
};

// Histogram of the coefficients e0..e1-1 inside [klo, khi), merged into the
// component's bins.
template <typename T>
__device__ void sure_hist_range(const CubeDesc& d, int comp, int64_t e0, int64_t e1, const SureState& st,
                                unsigned char* lds, SureShared& sh) {
    typedef KeyTraits<T> KT;
    typedef typename KT::K K;
    uint32_t* lc = reinterpret_cast<uint32_t*>(lds);
    double* ls = reinterpret_cast<double*>(lds + kSureBins * 4);
    K* lmin = reinterpret_cast<K*>(lds + kSureBins * 12);
    K* lmax = lmin + kSureBins;
    const int tid = threadIdx.x;
    for (int b = tid; b < kSureBins; b += kSureThreads) {
        lc[b] = 0;
        ls[b] = 0.0;
        lmin[b] = (K)~0ull;
        lmax[b] = 0;
    }
    if (tid == 0) sh.zeros = 0;
    __syncthreads();
    const T* cf = gmem(static_cast<const T*>(d.coef)) + (int64_t)comp * d.ncs;
    const uint64_t klo = st.klo, khi = st.khi;
    const int shf = (int)st.width;
    unsigned long long nz = 0;
    constexpr int U = 8;
    for (int64_t e = e0 + tid; e < e1; e += U * kSureThreads) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = e + (int64_t)u * kSureThreads;
            v[u] = idx < e1 ? cf[idx] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (e + (int64_t)u * kSureThreads < e1) {
                const K k = KT::key(v[u]);
                if (st.round == 0 && k == 0) ++nz;
                if ((uint64_t)k >= klo && (uint64_t)k < khi) {
                    const int b = (int)(((uint64_t)k - klo) >> shf);
                    atomicAdd(&lc[b], 1u);
                    atomicAdd(&ls[b], (double)v[u] * (double)v[u]);
                    atomicMin(&lmin[b], k);
                    atomicMax(&lmax[b], k);
                }
            }
        }
    }
    if (nz) atomicAdd(&sh.zeros, nz);
    __syncthreads();
    const int64_t base = (int64_t)comp * kSureBins;
    for (int b = tid; b < kSureBins; b += kSureThreads) {
        if (lc[b]) {
            atomicAdd(&gmem(d.hcnt)[base + b], lc[b]);
            atomicAdd(&gmem(d.hsum)[base + b], ls[b]);
            atomicMin(&gmem(d.hmin)[base + b], (unsigned long long)lmin[b]);
            atomicMax(&gmem(d.hmax)[base + b], (unsigned long long)lmax[b]);
        }
    }
    if (tid == 0 && sh.zeros) atomicAdd(sure_zeros(d, comp), sh.zeros);
}

// The magnitudes among e0..e1-1 (at most kGatherPer per thread) that fall in surviving
// bins (bitmap in sh.bits), appended to the component's list: one reservation
// per block, then plain stores.
template <typename T>
__device__ void sure_gather_chunk(const CubeDesc& d, int comp, int64_t e0, int64_t e1, const SureState& st,
                                  SureShared& sh) {
    typedef KeyTraits<T> KT;
    typedef typename KT::K K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const T* cf = gmem(static_cast<const T*>(d.coef)) + (int64_t)comp * d.ncs;
    const uint64_t klo = st.klo, khi = st.khi;
    const int shf = (int)st.width;
    K kv[kGatherPer];
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < kGatherPer; ++j) {
        const int64_t e = e0 + tid + (int64_t)j * kSureThreads;
        kv[j] = 0;
        if (e < e1) {
            const K k = KT::key(cf[e]);
            if ((uint64_t)k >= klo && (uint64_t)k < khi) {
                const int b = (int)(((uint64_t)k - klo) >> shf);
                if ((sh.bits[b >> 5] >> (b & 31)) & 1u) {
                    kv[j] = k;
                    m |= 1u << j;
                }
            }
        }
    }
    const uint32_t cnt = (uint32_t)__builtin_popcount(m);
    const uint32_t inc = wave_incl_u32(cnt);
    if (lane == 63) sh.wc[wave] = inc;
    __syncthreads();
    uint32_t off = inc - cnt, tot = 0;
    for (int w = 0; w < kSureWaves; ++w) {
        if (w < wave) off += sh.wc[w];
        tot += sh.wc[w];
    }
    if (tid == 0) sh.base = tot ? atomicAdd(&gmem(d.sctr)[4 * comp + 1], tot) : 0u;
    __syncthreads();
    uint64_t* out = gmem(d.cand) + (int64_t)comp * kSureCap;
    uint32_t pos = sh.base + off;
#pragma unroll
    for (int j = 0; j < kGatherPer; ++j) {
        if ((m >> j) & 1u) {
            if (pos < (uint32_t)kSureCap) out[pos] = (uint64_t)kv[j];
            ++pos;
        }
    }
}

// Exact finish from the gathered values: grouped by bin (counting sort in
// LDS), then SURE at each value: the count and sum of squares of its bin's
// values not above it, added to the totals below the bin.
template <typename T>
__device__ void sure_finish(const CubeDesc& d, int comp, double N, unsigned char* lds, SureShared& sh) {
    typedef KeyTraits<T> KT;
    uint32_t* bcnt = reinterpret_cast<uint32_t*>(lds);              // kSureBins
    uint32_t* boff = bcnt + kSureBins;                               // kSureBins + 1
    uint64_t* keys = reinterpret_cast<uint64_t*>(lds + (size_t)kSureBins * 8 + 16);   // kSureCap
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const SureState st = sh.st;
    // the gather re-reads the values the last histogram counted, so the
    // surviving bins hold exactly nsurv (<= kSureCap) values
    const uint32_t got = gmem(d.sctr)[4 * comp + 1];
    const int nc = (int)(got < (uint32_t)kSureCap ? got : (uint32_t)kSureCap);
    const uint64_t klo = st.klo;
    const int shf = (int)st.width;
    const uint64_t* src = gmem(d.cand) + (int64_t)comp * kSureCap;
    for (int b = tid; b < kSureBins; b += kSureThreads) bcnt[b] = 0u;
    __syncthreads();
    for (int i = tid; i < nc; i += kSureThreads) atomicAdd(&bcnt[(int)((src[i] - klo) >> shf)], 1u);
    __syncthreads();
    // segment offsets: exclusive prefix of the bin counts
    {
        uint32_t c[kBinsPer], tc = 0;
#pragma unroll
        for (int j = 0; j < kBinsPer; ++j) {
            c[j] = bcnt[tid * kBinsPer + j];
            tc += c[j];
        }
        const uint32_t inc = wave_incl_u32(tc);
        if (lane == 63) sh.wc[wave] = inc;
        __syncthreads();
        uint32_t o = inc - tc;
        for (int w = 0; w < wave; ++w) o += sh.wc[w];
#pragma unroll
        for (int j = 0; j < kBinsPer; ++j) {
            boff[tid * kBinsPer + j] = o;
            bcnt[tid * kBinsPer + j] = 0u;
            o += c[j];
        }
        if (tid == kSureThreads - 1) boff[kSureBins] = o;
    }
    __syncthreads();
    for (int i = tid; i < nc; i += kSureThreads) {
        const uint64_t key = src[i];
        const int b = (int)((key - klo) >> shf);
        keys[boff[b] + atomicAdd(&bcnt[b], 1u)] = key;
    }
    __syncthreads();
    double bs = __builtin_inf(), bt = 0.0;
    for (int i = tid; i < nc; i += kSureThreads) {
        const uint64_t key = keys[i];
        const int b = (int)((key - klo) >> shf);
        const int s0 = (int)boff[b], s1 = (int)boff[b + 1];
        double cw = 0.0, sw = 0.0;
        int j = s0;
        for (; j + 4 <= s1; j += 4) {             // four reads in flight, added in order
            uint64_t kq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) kq[u] = keys[j + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (kq[u] <= key) {
                    const double vj = KT::val(kq[u]);
                    cw += 1.0;
                    sw = fma(vj, vj, sw);
                }
            }
        }
        for (; j < s1; ++j) {
            const uint64_t kj = keys[j];
            if (kj <= key) {
                const double vj = KT::val(kj);
                cw += 1.0;
                sw = fma(vj, vj, sw);
            }
        }
        const int64_t bi = (int64_t)comp * kSureBins + b;
        const double c = (double)d.spre[bi] + cw;
        const double S = d.sspre[bi] + sw;
        const double v = KT::val(key);
        const double sv = N - 2.0 * c + S + (N - c) * v * v;
        if (sv < bs || (sv == bs && v < bt)) {
            bs = sv;
            bt = v;
        }
    }
    wave_argmin(bs, bt);
    if (lane == 0) {
        sh.bs[wave] = bs;
        sh.bt[wave] = bt;
    }
    __syncthreads();
    if (tid == 0) {
        SureState ns = st;
        double b_s = st.best_s, b_t = st.best_t;
        for (int w = 0; w < kSureWaves; ++w) {
            if (sh.bs[w] < b_s || (sh.bs[w] == b_s && sh.bt[w] < b_t)) {
                b_s = sh.bs[w];
                b_t = sh.bt[w];
            }
        }
        ns.best_s = b_s;
        ns.best_t = b_t;
        ns.done = 1;
        ns.round = st.round + 1;
        if (got != st.nsurv) ns.inexact = 1;
        d.lambda[comp] = b_t;
        if (d.sure) d.sure[comp] = b_s;
        if (ns.inexact) set_status(d.status, HYRES_DEV_SURE_INEXACT);
        put_state(&d.sst[comp], ns);
    }
}

// Select step of a component after its histogram pass: exact prefix sums,
// bounds, survivors, then either the next range or a gather of the surviving
// values.
template <typename T>
__device__ void sure_select(const CubeDesc& d, int comp, double N, SureShared& sh) {
    typedef KeyTraits<T> KT;
    constexpr int PER = kBinsPer;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)comp * kSureBins;
    const SureState st = sh.st;
    uint32_t cnt[PER];
    double sum[PER];
    uint64_t kmin[PER], kmax[PER];
    uint32_t tc = 0;                  // counts stay below 2^32 (at most 2^31 pixels)
    double ts = 0.0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int b = tid * PER + j;
        cnt[j] = gmem(d.hcnt)[base + b];
        sum[j] = gmem(d.hsum)[base + b];
        kmin[j] = gmem(d.hmin)[base + b];
        kmax[j] = gmem(d.hmax)[base + b];
        tc += cnt[j];
        ts += sum[j];
    }
    // exclusive prefix over threads of the counts and sums: waves by DPP and
    // readlane, then the totals of the waves before (fixed order)
    const uint32_t ic = wave_incl_u32(tc);
    const double is = wave_incl_f64(ts);
    const double is_prev = __shfl_up(is, 1, 64);
    if (lane == 63) {
        sh.wc[wave] = ic;
        sh.ws[wave] = is;
    }
    for (int w = tid; w < kSureBins / 32; w += kSureThreads) sh.bits[w] = 0u;
    __syncthreads();
    uint32_t oc = 0;
    double os = 0.0;
    for (int w = 0; w < wave; ++w) {
        oc += sh.wc[w];
        os += sh.ws[w];
    }
    unsigned long long pc = (unsigned long long)(oc + ic - tc);
    double ps = lane == 0 ? os : os + is_prev;
    double bs = __builtin_inf(), bt = 0.0;
    if (st.round == 0 && tid == 0) {
        bs = N - 2.0 * (double)*sure_zeros(d, comp);   // candidate t = 0
        bt = 0.0;
    }
    double lbv[PER];
    unsigned long long pcs[PER];
    double pss[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        pcs[j] = pc;
        pss[j] = ps;
        lbv[j] = __builtin_inf();
        if (cnt[j]) {
            const double C = (double)(st.below_cnt + pc);
            const double S = st.below_sum + ps;
            const double cc = (double)cnt[j];
            const double tmax = KT::val(kmax[j]), tmin = KT::val(kmin[j]);
            const double smax = N - 2.0 * (C + cc) + (S + sum[j]) + (N - C - cc) * tmax * tmax;
            lbv[j] = N - 2.0 * (C + cc) + S + (N - C) * tmin * tmin;
            if (smax < bs || (smax == bs && tmax < bt)) {
                bs = smax;
                bt = tmax;
            }
        }
        pc += cnt[j];
        ps += sum[j];
    }
    wave_argmin(bs, bt);
    if (lane == 0) {
        sh.bs[wave] = bs;
        sh.bt[wave] = bt;
    }
    __syncthreads();
    double best_s = sh.bs[0], best_t = sh.bt[0];
    for (int w = 1; w < kSureWaves; ++w) {
        if (sh.bs[w] < best_s || (sh.bs[w] == best_s && sh.bt[w] < best_t)) {
            best_s = sh.bs[w];
            best_t = sh.bt[w];
        }
    }
    if (st.best_s < best_s || (st.best_s == best_s && st.best_t < best_t)) {
        best_s = st.best_s;
        best_t = st.best_t;
    }
    const double U = best_s + 1e-12 * (fabs(best_s) + N);
    int f = 0x7fffffff, l = -1;
    uint32_t m = 0, mx = 0;
    bool surv[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        surv[j] = cnt[j] && lbv[j] <= U;
        if (surv[j]) {
            const int b = tid * PER + j;
            f = b < f ? b : f;
            l = b > l ? b : l;
            m += cnt[j];
            mx = cnt[j] > mx ? cnt[j] : mx;
        }
    }
    // first and last surviving bin, largest surviving bin, surviving values
    const int wf = wave_minmax_i32<false>(f), wl = wave_minmax_i32<true>(l);
    const int wmx = wave_minmax_i32<true>((int)mx);
    const uint32_t im = wave_incl_u32(m);
    if (lane == 63) sh.wm[wave] = im;
    if (lane == 0) {
        sh.wf[wave] = wf;
        sh.wl[wave] = wl;
        sh.wx[wave] = wmx;
    }
    __syncthreads();
    int fb = sh.wf[0], lb = sh.wl[0];
    unsigned int mxv = (unsigned int)sh.wx[0];
    uint32_t msum = 0;
    for (int w = 0; w < kSureWaves; ++w) {
        msum += sh.wm[w];
        if (w > 0) {
            fb = sh.wf[w] < fb ? sh.wf[w] : fb;
            lb = sh.wl[w] > lb ? sh.wl[w] : lb;
            mxv = (unsigned int)sh.wx[w] > mxv ? (unsigned int)sh.wx[w] : mxv;
        }
    }
    const unsigned long long msurv = msum;
    const bool gather = lb >= 0 && st.width > 0 && msurv <= (unsigned long long)kSureCap &&
                        mxv <= (unsigned)kSureBinCap;
    if (gather) {
        // bitmap of the surviving bins and the counts and sums below each
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (surv[j]) {
                const int b = tid * PER + j;
                atomicOr(&sh.bits[b >> 5], 1u << (b & 31));
                d.spre[base + b] = st.below_cnt + pcs[j];
                d.sspre[base + b] = st.below_sum + pss[j];
            }
        }
        __syncthreads();
        for (int w = tid; w < kSureBins / 32; w += kSureThreads)
            d.sbits[(int64_t)comp * (kSureBins / 32) + w] = sh.bits[w];
    }
    // the prefix before the first surviving bin
    if (!gather && tid == fb / PER && fb != 0x7fffffff) {
        const int j = fb - tid * PER;
        unsigned long long c0 = 0;
        double s0 = 0.0;
#pragma unroll
        for (int jj = 0; jj < PER; ++jj)
            if (jj == j) {
                c0 = pcs[jj];
                s0 = pss[jj];
            }
        sh.st.below_cnt = st.below_cnt + c0;
        sh.st.below_sum = st.below_sum + s0;
    }
    __syncthreads();
    if (tid == 0) {
        SureState ns = sh.st;
        ns.best_s = best_s;
        ns.best_t = best_t;
        ns.round = st.round + 1;
        if (st.width == 0 || lb < 0) {
            ns.done = 1;
        } else if (gather) {
            ns.gather = 1;
            ns.nsurv = (unsigned int)msurv;
        } else {
            ns.klo = st.klo + ((uint64_t)fb << st.width);
            const uint64_t hi = st.klo + ((uint64_t)(lb + 1) << st.width);
            ns.khi = hi < st.khi ? hi : st.khi;
            ns.width = sure_shift_for(ns.khi - ns.klo);
            if (ns.round >= KT::kRounds) {
                ns.done = 1;
                ns.inexact = 1;
            }
        }
        if (ns.done) {
            d.lambda[comp] = ns.best_t;
            if (d.sure) d.sure[comp] = ns.best_s;
            if (ns.inexact) set_status(d.status, HYRES_DEV_SURE_INEXACT);
        }
        put_state(&d.sst[comp], ns);
        gmem(d.sctr)[4 * comp] = 0u;        // block counter of the next pass
        gmem(d.sctr)[4 * comp + 1] = 0u;    // gathered values
    }
    // clear the bins for the next pass
    for (int b = tid; b < kSureBins; b += kSureThreads) {
        gmem(d.hcnt)[base + b] = 0;
        gmem(d.hsum)[base + b] = 0.0;
        gmem(d.hmin)[base + b] = ~0ull;
        gmem(d.hmax)[base + b] = 0;
    }
}

// One pass over every component still searching: histogram or gather of each
// chunk; the last block of a component runs its select or finish.
template <typename T>
__global__ __launch_bounds__(kSureThreads) void k_sure_round(const CubeDesc* __restrict__ descs,
                                                             const int* __restrict__ items, int ncubes) {
    __shared__ __align__(16) unsigned char lds[SureLds<T>::kBytes];
    __shared__ SureShared sh;
    const int total = items[ncubes];
    const int tid = threadIdx.x;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int64_t N = sure_count(d);
        const int64_t ch = d.schunk;
        const int nch = (int)((N + ch - 1) / ch);
        const int local = item - items[c];
        const int comp = local / nch;
        const int chunk = local - comp * nch;
        __syncthreads();
        if (tid == 0) sh.st = d.sst[comp];
        __syncthreads();
        if (sh.st.done) continue;   // uniform across the block
        const SureState st = sh.st;
        // in refinement passes few values are in range: a block takes up to
        // kSureGroup small chunks (the others of the group only count themselves)
        const int64_t gmax = kSureGroupSpan / ch;
        const int grp = st.round == 0 || st.gather ? 1 : (int)(gmax < 1 ? 1 : (gmax > kSureGroup ? kSureGroup : gmax));
        if (chunk % grp == 0) {
            const int64_t e0 = (int64_t)chunk * ch;
            const int64_t eg = e0 + (int64_t)grp * ch;
            const int64_t e1 = eg < N ? eg : N;
            if (st.gather) {
                for (int w = tid; w < kSureBins / 32; w += kSureThreads)
                    sh.bits[w] = d.sbits[(int64_t)comp * (kSureBins / 32) + w];
                constexpr int64_t span = (int64_t)kGatherPer * kSureThreads;
                for (int64_t a = e0; a < e1; a += span) {
                    __syncthreads();
                    sure_gather_chunk<T>(d, comp, a, a + span < e1 ? a + span : e1, st, sh);
                }
            } else {
                sure_hist_range<T>(d, comp, e0, e1, st, lds, sh);
            }
        }
        // Every wave waits for its global atomics and stores to be acknowledged;
        // then one release fence (device scope) for the block before it is
        // counted, and one acquire fence in the last block before its reads.
        // The L1 and L2 the fences act on are shared by the waves of the block.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            const bool last = atomicAdd(&gmem(d.sctr)[4 * comp], 1u) == (unsigned)(nch - 1);
            if (last) __threadfence();
            sh.last = last;
        }
        __syncthreads();
        if (!sh.last) continue;
        if (st.gather) sure_finish<T>(d, comp, (double)N, lds, sh);
        else sure_select<T>(d, comp, (double)N, sh);
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_sure_init(int dtype, const CubeDesc* descs, const int* items, int ncubes, int grid,
                            hipStream_t s) {
    if (dtype == HYRES_F64)
        hipLaunchKernelGGL(k_sure_init<double>, dim3(grid), dim3(256), 0, s, descs, items, ncubes);
    else
        hipLaunchKernelGGL(k_sure_init<float>, dim3(grid), dim3(256), 0, s, descs, items, ncubes);
    return hipGetLastError();
}

hipError_t launch_sure_round(int dtype, const CubeDesc* descs, const int* items, int ncubes, int grid,
                             hipStream_t s) {
    if (dtype == HYRES_F64)
        hipLaunchKernelGGL(k_sure_round<double>, dim3(grid), dim3(kSureThreads), 0, s, descs, items, ncubes);
    else
        hipLaunchKernelGGL(k_sure_round<float>, dim3(grid), dim3(kSureThreads), 0, s, descs, items, ncubes);
    return hipGetLastError();
}

// One more pass than refinement rounds, so a gather decided in the last
// refinement round is still finished.
int sure_rounds(int dtype) { return (dtype == HYRES_F64 ? kSureRoundsF64 : kSureRoundsF32) + 1; }
// Coefficients per work item: about one item per compute unit over all the
// components of a program (each block then streams its item once per pass),
// at least kSureChunk, a multiple of the block size.
int64_t sure_chunk_for(int64_t total_coef, int num_cu) {
    int64_t ch = (total_coef + num_cu - 1) / (num_cu > 0 ? num_cu : 1);
    ch = (ch + kSureThreads - 1) / kSureThreads * kSureThreads;
    return ch > kSureChunk ? ch : kSureChunk;
}

}  // namespace hyres
