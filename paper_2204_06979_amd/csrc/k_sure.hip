// Exact SURE threshold by histogram refinement.
//
// For coefficients b_1..b_N of one component the risk estimate of soft
// thresholding at unit noise is SURE(t) = N - 2 #{|b| <= t} + sum min(b^2, t^2).
// Between consecutive candidates t in {0} U {|b_k|} it increases with t, so the
// minimum is attained on the candidate set.
//
// The magnitude |b| is keyed by its IEEE bit pattern (monotone for
// non-negative numbers).  Each round histograms the keys inside the current
// range [klo, khi) into 4096 bins of width 2^shift, recording per bin the
// count, the sum of squares and the smallest and largest key.  The select
// kernel then knows exactly, for every bin:
//   C = #values below the bin, S = their sum of squares;
//   SURE at the largest value of the bin, t_max (an exact candidate):
//     N - 2(C + c) + S + s + (N - C - c) t_max^2;
//   a lower bound over every candidate t in the bin:
//     N - 2(C + c) + S + (N - C) t_min^2.
// Bins whose lower bound exceeds the best exact value seen are discarded.
// When the surviving bins hold at most kSureCap values, the next pass
// collects exactly those values, grouped by bin, and the select kernel
// finishes exactly: for every collected value it adds the count and sum of
// squares of the values of its own bin that do not exceed it to the totals
// below the bin, and evaluates SURE there.  Otherwise the next round refines the
// key range spanned by the surviving bins (bins of width 1 are exact too).
// The smallest minimising candidate is returned.
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

constexpr int kSureChunk = 16384;   // coefficients per histogram work item
constexpr int kSureThreads = 256;

__host__ __device__ inline int sure_shift_for(uint64_t span) {
    int s = 0;
    while (((span + ((1ull << s) - 1)) >> s) > (uint64_t)kSureBins) ++s;
    return s;
}

__device__ __forceinline__ int64_t sure_count(const CubeDesc& d) {
    return d.scope == HYRES_SCOPE_DETAIL ? d.ll_off : d.nc;
}

// Reset the search state and the global bins of every component.
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
            d.hcnt[base + b] = 0;
            d.hsum[base + b] = 0.0;
            d.hmin[base + b] = ~0ull;
            d.hmax[base + b] = 0;
        }
        if (threadIdx.x == 0) {
            SureState st;
            st.klo = 0;
            st.khi = KT::kEnd;
            st.width = sure_shift_for(KT::kEnd);
            st.below_cnt = 0;
            st.below_sum = 0.0;
            st.best_s = __builtin_inf();
            st.best_t = 0.0;
            st.zeros = 0;
            st.round = 0;
            st.done = 0;
            st.inexact = 0;
            st.gather = 0;
            st.nsurv = 0;
            d.sst[comp] = st;
        }
    }
}

// Collect the magnitudes that fall in surviving bins (bitmap) into the
// candidate list of the component, grouped by bin: bin b owns the segment
// starting at scb[b] (order inside a segment is irrelevant).
template <typename T>
__device__ void sure_gather(const CubeDesc& d, int comp, int chunk, int64_t N, const SureState& st,
                            uint32_t* lds_bits) {
    typedef KeyTraits<T> KT;
    typedef typename KT::K K;
    __syncthreads();
    for (int w = threadIdx.x; w < kSureBins / 32; w += kSureThreads)
        lds_bits[w] = d.sbits[(int64_t)comp * (kSureBins / 32) + w];
    __syncthreads();
    const T* cf = static_cast<const T*>(d.coef) + (int64_t)comp * d.ncs;
    const int64_t e0 = (int64_t)chunk * kSureChunk;
    const int64_t e1 = e0 + kSureChunk < N ? e0 + kSureChunk : N;
    const uint64_t klo = st.klo, khi = st.khi;
    const int sh = (int)st.width;
    const int64_t base = (int64_t)comp * kSureBins;
    uint64_t* out = d.cand + (int64_t)comp * kSureCap;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kSureThreads) {
        const K k = KT::key(cf[e]);
        if ((uint64_t)k >= klo && (uint64_t)k < khi) {
            const int b = (int)(((uint64_t)k - klo) >> sh);
            if ((lds_bits[b >> 5] >> (b & 31)) & 1u) {
                const unsigned int pos = d.scb[base + b] + atomicAdd(&d.sfill[base + b], 1u);
                if (pos < (unsigned)kSureCap) out[pos] = (uint64_t)k;
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kSureThreads) void k_sure_hist(const CubeDesc* __restrict__ descs,
                                                            const int* __restrict__ items, int ncubes) {
    typedef KeyTraits<T> KT;
    typedef typename KT::K K;
    __shared__ uint32_t lc[kSureBins];
    __shared__ double ls[kSureBins];
    __shared__ K lmin[kSureBins], lmax[kSureBins];
    __shared__ unsigned long long lz;
    const int total = items[ncubes];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int64_t N = sure_count(d);
        const int nch = (int)((N + kSureChunk - 1) / kSureChunk);
        const int local = item - items[c];
        const int comp = local / nch;
        const int chunk = local - comp * nch;
        const SureState st = d.sst[comp];
        if (st.done) continue;   // uniform across the block
        if (st.gather) {
            sure_gather<T>(d, comp, chunk, N, st, reinterpret_cast<uint32_t*>(lc));
            continue;
        }
        __syncthreads();
        for (int b = threadIdx.x; b < kSureBins; b += kSureThreads) {
            lc[b] = 0;
            ls[b] = 0.0;
            lmin[b] = (K)~0ull;
            lmax[b] = 0;
        }
        if (threadIdx.x == 0) lz = 0;
        __syncthreads();
        const T* cf = static_cast<const T*>(d.coef) + (int64_t)comp * d.ncs;
        const int64_t e0 = (int64_t)chunk * kSureChunk;
        const int64_t e1 = e0 + kSureChunk < N ? e0 + kSureChunk : N;
        const uint64_t klo = st.klo, khi = st.khi;
        const int sh = (int)st.width;
        unsigned long long nz = 0;
        constexpr int U = 8;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += U * kSureThreads) {
            T v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t idx = e + (int64_t)u * kSureThreads;
                v[u] = idx < e1 ? cf[idx] : (T)-1;       // -1 marks "no element" (its key is out of range)
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!(v[u] == (T)-1 && e + (int64_t)u * kSureThreads >= e1)) {
                    const K k = KT::key(v[u]);
                    if (st.round == 0 && k == 0) ++nz;
                    if ((uint64_t)k >= klo && (uint64_t)k < khi) {
                        const int b = (int)(((uint64_t)k - klo) >> sh);
                        atomicAdd(&lc[b], 1u);
                        atomicAdd(&ls[b], (double)v[u] * (double)v[u]);
                        atomicMin(&lmin[b], k);
                        atomicMax(&lmax[b], k);
                    }
                }
            }
        }
        if (nz) atomicAdd(&lz, nz);
        __syncthreads();
        const int64_t base = (int64_t)comp * kSureBins;
        for (int b = threadIdx.x; b < kSureBins; b += kSureThreads) {
            if (lc[b]) {
                atomicAdd(&d.hcnt[base + b], lc[b]);
                atomicAdd(&d.hsum[base + b], ls[b]);
                atomicMin(&d.hmin[base + b], (unsigned long long)lmin[b]);
                atomicMax(&d.hmax[base + b], (unsigned long long)lmax[b]);
            }
        }
        if (threadIdx.x == 0 && lz) atomicAdd((unsigned long long*)&d.sst[comp].zeros, lz);
    }
}

constexpr int kSelThreads = 1024;
constexpr int kSelWaves = kSelThreads / 64;

// ---- wave and block primitives of the select kernel (whole block active) ----
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

// Exact finish of a component from its collected candidates: for every
// candidate v in bin b, the count and sum of squares of the values <= v are
// the totals below the bin plus those of the bin's own values <= v (a scan of
// the bin's segment, at most kSureBinCap values).
template <typename T>
__device__ void sure_finish(const CubeDesc& d, int comp, SureState& st, double N, double* raw) {
    typedef KeyTraits<T> KT;
    uint64_t* keys = reinterpret_cast<uint64_t*>(raw);     // kSureCap
    __shared__ double s_bs2[kSelThreads], s_bt2[kSelThreads];
    const int tid = threadIdx.x;
    // the gather pass re-reads the values the last histogram counted, so the
    // surviving bins hold exactly nsurv (<= kSureCap) values
    const unsigned int nc = st.nsurv < (unsigned)kSureCap ? st.nsurv : (unsigned)kSureCap;
    const uint64_t* src = d.cand + (int64_t)comp * kSureCap;
    for (int i = tid; i < (int)nc; i += kSelThreads) keys[i] = src[i];
    __syncthreads();
    const uint64_t klo = st.klo;
    const int sh = (int)st.width;
    double bs = __builtin_inf(), bt = 0.0;
    for (int j = tid; j < (int)nc; j += kSelThreads) {
        const uint64_t key = keys[j];
        const double v = KT::val(key);
        const int b = (int)((key - klo) >> sh);
        const int64_t bi = (int64_t)comp * kSureBins + b;
        const unsigned int s0 = d.scb[bi], s1 = s0 + d.sfill[bi];
        double cw = 0.0, sw = 0.0;
        for (unsigned int i = s0; i < s1 && i < nc; ++i) {
            const uint64_t ki = keys[i];
            if (ki <= key) {
                const double vi = KT::val(ki);
                cw += 1.0;
                sw = fma(vi, vi, sw);
            }
        }
        const double c = (double)d.spre[bi] + cw;
        const double S = d.sspre[bi] + sw;
        const double sv = N - 2.0 * c + S + (N - c) * v * v;
        if (sv < bs || (sv == bs && v < bt)) {
            bs = sv;
            bt = v;
        }
    }
    s_bs2[tid] = bs;
    s_bt2[tid] = bt;
    __syncthreads();
    for (int o = kSelThreads / 2; o >= 1; o >>= 1) {
        if (tid < o) {
            const double ob = s_bs2[tid + o], ot = s_bt2[tid + o];
            if (ob < s_bs2[tid] || (ob == s_bs2[tid] && ot < s_bt2[tid])) {
                s_bs2[tid] = ob;
                s_bt2[tid] = ot;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        double b_s = s_bs2[0], b_t = s_bt2[0];
        if (st.best_s < b_s || (st.best_s == b_s && st.best_t < b_t)) {
            b_s = st.best_s;
            b_t = st.best_t;
        }
        st.best_s = b_s;
        st.best_t = b_t;
        st.done = 1;
    }
}

// One block per component: exact prefix sums, bounds, survivors, then either
// the next range, a gather of the surviving values, or (after a gather) the
// exact finish.
template <typename T>
__global__ __launch_bounds__(kSelThreads) void k_sure_select(const CubeDesc* __restrict__ descs,
                                                             const int* __restrict__ items, int ncubes) {
    typedef KeyTraits<T> KT;
    constexpr int PER = kSureBins / kSelThreads;   // bins per thread
    __shared__ double raw[kSureCap];               // keys of the exact finish
    __shared__ SureState s_st;
    // per-wave totals of the select round
    __shared__ uint32_t s_wc[kSelWaves], s_wm[kSelWaves];
    __shared__ double s_ws[kSelWaves], s_bs[kSelWaves], s_bt[kSelWaves];
    __shared__ int s_wf[kSelWaves], s_wl[kSelWaves], s_wx[kSelWaves];
    const int total = items[ncubes];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int comp = item - items[c];
        __syncthreads();
        if (tid == 0) s_st = d.sst[comp];
        __syncthreads();
        if (s_st.done) continue;
        const double N = (double)sure_count(d);
        const int64_t base = (int64_t)comp * kSureBins;
        if (s_st.gather) {
            sure_finish<T>(d, comp, s_st, N, raw);
            __syncthreads();
            if (tid == 0) {
                s_st.round += 1;
                d.lambda[comp] = s_st.best_t;
                if (d.sure) d.sure[comp] = s_st.best_s;
                if (s_st.inexact) set_status(d.status, HYRES_DEV_SURE_INEXACT);
                d.sst[comp] = s_st;
            }
            continue;
        }
        const SureState st = s_st;
        uint32_t cnt[PER];
        double sum[PER];
        uint64_t kmin[PER], kmax[PER];
        uint32_t tc = 0;                  // counts stay below 2^32 (at most 2^31 pixels)
        double ts = 0.0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int b = tid * PER + j;
            cnt[j] = d.hcnt[base + b];
            sum[j] = d.hsum[base + b];
            kmin[j] = d.hmin[base + b];
            kmax[j] = d.hmax[base + b];
            tc += cnt[j];
            ts += sum[j];
        }
        // exclusive prefix over threads of the counts and sums: waves by DPP and
        // readlane, then the totals of the waves before (fixed order)
        const uint32_t ic = wave_incl_u32(tc);
        const double is = wave_incl_f64(ts);
        const double is_prev = __shfl_up(is, 1, 64);
        if (lane == 63) {
            s_wc[wave] = ic;
            s_ws[wave] = is;
        }
        __syncthreads();
        uint32_t oc = 0;
        double os = 0.0;
        for (int w = 0; w < wave; ++w) {
            oc += s_wc[w];
            os += s_ws[w];
        }
        unsigned long long pc = (unsigned long long)(oc + ic - tc);
        double ps = lane == 0 ? os : os + is_prev;
        double bs = __builtin_inf(), bt = 0.0;
        if (st.round == 0 && tid == 0) {
            bs = N - 2.0 * (double)st.zeros;   // candidate t = 0
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
            s_bs[wave] = bs;
            s_bt[wave] = bt;
        }
        __syncthreads();
        double best_s = s_bs[0], best_t = s_bt[0];
        for (int w = 1; w < kSelWaves; ++w) {
            if (s_bs[w] < best_s || (s_bs[w] == best_s && s_bt[w] < best_t)) {
                best_s = s_bs[w];
                best_t = s_bt[w];
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
        // first and last surviving bin, largest surviving bin, and the prefix of
        // surviving counts (the offsets of the gathered values)
        const int wf = wave_minmax_i32<false>(f), wl = wave_minmax_i32<true>(l);
        const int wmx = wave_minmax_i32<true>((int)mx);
        const uint32_t im = wave_incl_u32(m);
        if (lane == 63) s_wm[wave] = im;
        if (lane == 0) {
            s_wf[wave] = wf;
            s_wl[wave] = wl;
            s_wx[wave] = wmx;
        }
        __syncthreads();
        int fb = s_wf[0], lb = s_wl[0];
        unsigned int s_mxv = (unsigned int)s_wx[0];
        uint32_t om = 0, msum = 0;
        for (int w = 0; w < kSelWaves; ++w) {
            if (w < wave) om += s_wm[w];
            msum += s_wm[w];
            if (w > 0) {
                fb = s_wf[w] < fb ? s_wf[w] : fb;
                lb = s_wl[w] > lb ? s_wl[w] : lb;
                s_mxv = (unsigned int)s_wx[w] > s_mxv ? (unsigned int)s_wx[w] : s_mxv;
            }
        }
        const unsigned long long msurv = msum;
        const bool gather = lb >= 0 && st.width > 0 && msurv <= (unsigned long long)kSureCap &&
                            s_mxv <= (unsigned)kSureBinCap;
        if (gather) {
            // bitmap, counts below each surviving bin, and collected-value offsets
            uint32_t mo = om + im - m;
            for (int w = tid; w < kSureBins / 32; w += kSelThreads) d.sbits[(int64_t)comp * (kSureBins / 32) + w] = 0u;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < PER; ++j) d.sfill[base + tid * PER + j] = 0u;
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                if (surv[j]) {
                    const int b = tid * PER + j;
                    atomicOr(&d.sbits[(int64_t)comp * (kSureBins / 32) + (b >> 5)], 1u << (b & 31));
                    d.spre[base + b] = st.below_cnt + pcs[j];
                    d.sspre[base + b] = st.below_sum + pss[j];
                    d.scb[base + b] = (uint32_t)mo;
                    mo += cnt[j];
                }
            }
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
            s_st.below_cnt = st.below_cnt + c0;
            s_st.below_sum = st.below_sum + s0;
        }
        __syncthreads();
        if (tid == 0) {
            SureState ns = s_st;
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
            d.sst[comp] = ns;
        }
        // clear the bins for the next round
        for (int b = tid; b < kSureBins; b += kSelThreads) {
            d.hcnt[base + b] = 0;
            d.hsum[base + b] = 0.0;
            d.hmin[base + b] = ~0ull;
            d.hmax[base + b] = 0;
        }
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

hipError_t launch_sure_round(int dtype, const CubeDesc* descs, const int* hist_items, const int* sel_items,
                             int ncubes, int hist_grid, int sel_grid, hipStream_t s) {
    if (dtype == HYRES_F64) {
        hipLaunchKernelGGL(k_sure_hist<double>, dim3(hist_grid), dim3(kSureThreads), 0, s, descs, hist_items, ncubes);
        hipLaunchKernelGGL(k_sure_select<double>, dim3(sel_grid), dim3(kSelThreads), 0, s, descs, sel_items, ncubes);
    } else {
        hipLaunchKernelGGL(k_sure_hist<float>, dim3(hist_grid), dim3(kSureThreads), 0, s, descs, hist_items, ncubes);
        hipLaunchKernelGGL(k_sure_select<float>, dim3(sel_grid), dim3(kSelThreads), 0, s, descs, sel_items, ncubes);
    }
    return hipGetLastError();
}

// One more pass than refinement rounds, so a gather decided in the last
// refinement round is still finished.
int sure_rounds(int dtype) { return (dtype == HYRES_F64 ? kSureRoundsF64 : kSureRoundsF32) + 1; }
int sure_chunk() { return kSureChunk; }

}  // namespace hyres
