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
    __shared__ double raw[kSureCap];               // finish: keys; select: scratch below
    __shared__ SureState s_st;
    __shared__ unsigned int s_mx;
    unsigned long long* s_cnt = reinterpret_cast<unsigned long long*>(raw);
    double* s_sum = raw + kSelThreads;
    double* s_bs = raw + 2 * kSelThreads;
    double* s_bt = raw + 3 * kSelThreads;
    int* s_f = reinterpret_cast<int*>(raw + 4 * kSelThreads);
    int* s_l = s_f + kSelThreads;
    unsigned long long* s_m = reinterpret_cast<unsigned long long*>(raw + 5 * kSelThreads);
    const int total = items[ncubes];
    const int tid = threadIdx.x;
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
        unsigned long long tc = 0;
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
        // exclusive scan over threads (Hillis-Steele in LDS; fixed order of additions)
        s_cnt[tid] = tc;
        s_sum[tid] = ts;
        __syncthreads();
        for (int o = 1; o < kSelThreads; o <<= 1) {
            const unsigned long long ac = tid >= o ? s_cnt[tid - o] : 0ull;
            const double as = tid >= o ? s_sum[tid - o] : 0.0;
            __syncthreads();
            s_cnt[tid] += ac;
            s_sum[tid] += as;
            __syncthreads();
        }
        unsigned long long pc = s_cnt[tid] - tc;
        double ps = tid > 0 ? s_sum[tid - 1] : 0.0;
        __syncthreads();
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
        s_bs[tid] = bs;
        s_bt[tid] = bt;
        __syncthreads();
        for (int o = kSelThreads / 2; o >= 1; o >>= 1) {
            if (tid < o) {
                const double ob = s_bs[tid + o], ot = s_bt[tid + o];
                if (ob < s_bs[tid] || (ob == s_bs[tid] && ot < s_bt[tid])) {
                    s_bs[tid] = ob;
                    s_bt[tid] = ot;
                }
            }
            __syncthreads();
        }
        double best_s = s_bs[0], best_t = s_bt[0];
        if (st.best_s < best_s || (st.best_s == best_s && st.best_t < best_t)) {
            best_s = st.best_s;
            best_t = st.best_t;
        }
        const double U = best_s + 1e-12 * (fabs(best_s) + N);
        int f = 0x7fffffff, l = -1;
        unsigned long long m = 0;
        unsigned int mx = 0;
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
        s_f[tid] = f;
        s_l[tid] = l;
        s_m[tid] = m;
        if (tid == 0) s_mx = 0;
        __syncthreads();
        if (mx) atomicMax(&s_mx, mx);
        // inclusive scan of surviving counts (for the candidate offsets) and min/max of f, l
        for (int o = 1; o < kSelThreads; o <<= 1) {
            const unsigned long long am = tid >= o ? s_m[tid - o] : 0ull;
            __syncthreads();
            s_m[tid] += am;
            __syncthreads();
        }
        for (int o = kSelThreads / 2; o >= 1; o >>= 1) {
            if (tid < o) {
                s_f[tid] = s_f[tid + o] < s_f[tid] ? s_f[tid + o] : s_f[tid];
                s_l[tid] = s_l[tid + o] > s_l[tid] ? s_l[tid + o] : s_l[tid];
            }
            __syncthreads();
        }
        const int fb = s_f[0], lb = s_l[0];
        const unsigned long long msurv = s_m[kSelThreads - 1];
        const bool gather = lb >= 0 && st.width > 0 && msurv <= (unsigned long long)kSureCap &&
                            s_mx <= (unsigned)kSureBinCap;
        if (gather) {
            // bitmap, counts below each surviving bin, and collected-value offsets
            unsigned long long mo = s_m[tid] - m;
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
