// Band Gram G = Y^T Y of a hyperspectral cube (the first pass over Y).
//
// FP32 cubes: a symmetric rank-k update on the matrix cores.  Each work item
// ("slot") is a contiguous pixel range of one cube.  A block of 8 waves stages
// 32 pixels x p bands in LDS, every wave loads the 16-band fragments of the 4
// pixel rows of one k-step and issues v_mfma_f32_16x16x4f32 for its share of
// the T(T+1)/2 upper 16x16 tiles of G (T = ceil(p/16)).  Each slot writes one
// FP32 partial Gram; k_gram_reduce sums the slots of a cube in FP64 in a fixed
// order, so the result is bitwise reproducible.  Inside a slot the MFMA
// accumulates one 64-pixel chunk in FP32 and chunks are summed in FP64, so the
// rounding error of G stays near one FP32 rounding of each partial.  A NaN or
// Inf in band a makes G_aa non-finite: the reduce flags it (no per-value test).
//
// FP64 cubes: one thread per upper-triangle entry and slot, plain FP64 FMAs.
#include "hyres_internal.hpp"

namespace hyres {

// Upper 16x16 tiles of G in row-major order.  P = 0: all of them; P = 1..NP:
// one of NP consecutive parts (for large T one launch per part keeps the
// per-wave accumulators in registers, at the price of rereading Y; a program
// of few slots splits every slot's tiles over NPX blocks of one launch).
template <int T, int P = 0, int NPX = 0>
struct TileMap {
    static constexpr int NT = T * (T + 1) / 2;    // all tiles (partial layout)
    static constexpr int NP = NPX ? NPX : (T >= 13 ? 3 : 2);   // parts when split
    static constexpr int T0 = P == 0 ? 0 : (P - 1) * NT / NP;
    static constexpr int T1 = P == 0 ? NT : P * NT / NP;
    static constexpr int S = (T1 - T0 + 7) / 8 > 0 ? (T1 - T0 + 7) / 8 : 1;   // tiles per wave
    __host__ __device__ static constexpr int ti(int t) {
        int i = 0, rem = t;
        while (rem >= T - i) { rem -= T - i; ++i; }
        return i;
    }
    __host__ __device__ static constexpr int tj(int t) {
        int i = 0, rem = t;
        while (rem >= T - i) { rem -= T - i; ++i; }
        return i + rem;
    }
};

constexpr int kGramKB = 64;                        // pixels per LDS stage

template <int T>
__host__ __device__ constexpr int gram_ldw() { return (T & 1) ? 16 * T : 16 * T + 16; }

// Values each thread stages per chunk: float4 path (contiguous, 16-byte aligned
// rows) and scalar path.
template <int T> __host__ __device__ constexpr int gram_nv4() { return (kGramKB * 4 * T + kGramThreads - 1) / kGramThreads; }
template <int T> __host__ __device__ constexpr int gram_nv1() { return (kGramKB * 16 * T + kGramThreads - 1) / kGramThreads; }
// one register array serves both paths (float4 groups or single floats)
template <int T> __host__ __device__ constexpr int gram_nr() {
    return 4 * gram_nv4<T>() > gram_nv1<T>() ? 4 * gram_nv4<T>() : gram_nv1<T>();
}

// Wave WV owns the contiguous run of upper tiles [WV*S, WV*S + S) in row-major
// order: the fragment of the tile row stays in registers while the column
// fragment is loaded per tile.
template <int T, int P, int WV, int NPX = 0>
__device__ __forceinline__ void gram_wave(const float* __restrict__ tile, int lane,
                                          v4f (&acc)[TileMap<T, P, NPX>::S]) {
    using TM = TileMap<T, P, NPX>;
    constexpr int LDW = gram_ldw<T>();
    constexpr int S = TM::S;
    const int col = lane & 15, row = lane >> 4;
#pragma unroll 2
    for (int s = 0; s < kGramKB / 4; ++s) {
        const float* rowp = tile + (4 * s + row) * LDW + col;
        float fi = 0.f;
        static_for<S>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int t = TM::T0 + WV * S + q;
            if constexpr (t < TM::T1) {
                constexpr int i = TM::ti(t), j = TM::tj(t);
                if constexpr (q == 0 || TM::ti(t - 1) != i) fi = rowp[16 * i];
                if constexpr (i == j) {
                    acc[q] = mfma4(fi, fi, acc[q]);
                } else {
                    acc[q] = mfma4(fi, rowp[16 * j], acc[q]);
                }
            }
        });
    }
}

// Load one chunk of kGramKB pixels (all 16T band slots) into registers.
// kVec: 16-byte aligned pixel vectors, p % 4 == 0, and the 64 pixels of a chunk
// consecutive in memory (a contiguous cube, or whole chunks per image row).
// kDense: the chunk is 64 p consecutive floats (float i of the thread is float
// tid + 512 i of it).  kScalar: one float per band slot.
template <int T, int M>
__device__ __forceinline__ void gram_fetch(const CubeDesc& d, int64_t q, int64_t q1, float (&r)[gram_nr<T>()]) {
    const int tid = threadIdx.x;
    if constexpr (M == kVec) {
        const float* base = pixel_ptr<float>(d, q);   // a chunk never crosses an image row
        const int g4 = d.p >> 2;                     // float4 groups per pixel
#pragma unroll
        for (int i = 0; i < gram_nv4<T>(); ++i) {
            const int e = tid + kGramThreads * i;    // over kGramKB x 4T
            const int k = e / (4 * T), g = e - k * (4 * T);
            v4f v = {0.f, 0.f, 0.f, 0.f};
            if (k < kGramKB && g < g4 && q + k < q1)
                v = *reinterpret_cast<const v4f*>(base + (int64_t)k * d.pitch + 4 * g);
#pragma unroll
            for (int c = 0; c < 4; ++c) r[4 * i + c] = v[c];
        }
    } else if constexpr (M == kDense) {
        const float* base = pixel_ptr<float>(d, q);
        const int64_t m = q1 - q;
        const int lim = (int)(m < kGramKB ? m : kGramKB) * d.p;
#pragma unroll
        for (int i = 0; i < gram_nv1<T>(); ++i) {
            const int e = tid + kGramThreads * i;
            r[i] = e < lim ? base[e] : 0.f;
        }
    } else {
#pragma unroll
        for (int i = 0; i < gram_nv1<T>(); ++i) {
            const int e = tid + kGramThreads * i;    // over kGramKB x 16T
            const int k = e / (16 * T), b = e - k * (16 * T);
            float v = 0.f;
            if (k < kGramKB && b < d.p && q + k < q1) v = pixel_ptr<float>(d, q + k)[b];
            r[i] = v;
        }
    }
}

// kDense leaves the band slots from p on as they were: an entry of G reads only
// its own two bands, and those of bands >= p are never stored.
template <int T, int M>
__device__ __forceinline__ void gram_stage(float* __restrict__ tile, const CubeDesc& d, const float (&r)[gram_nr<T>()]) {
    constexpr int LDW = gram_ldw<T>();
    const int tid = threadIdx.x;
    if constexpr (M == kVec) {
#pragma unroll
        for (int i = 0; i < gram_nv4<T>(); ++i) {
            const int e = tid + kGramThreads * i;
            const int k = e / (4 * T), g = e - k * (4 * T);
            if (k < kGramKB) {
                const v4f v = {r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3]};
                *reinterpret_cast<v4f*>(tile + k * LDW + 4 * g) = v;
            }
        }
    } else if constexpr (M == kDense) {
        const int p = d.p;
#pragma unroll
        for (int i = 0; i < gram_nv1<T>(); ++i) {
            const int e = tid + kGramThreads * i;
            if (e < kGramKB * p) {
                const int k = div_p(e, d.pmag);
                tile[k * LDW + (e - k * p)] = r[i];
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < gram_nv1<T>(); ++i) {
            const int e = tid + kGramThreads * i;
            const int k = e / (16 * T), b = e - k * (16 * T);
            if (k < kGramKB) tile[k * LDW + b] = r[i];
        }
    }
}

// The FP32 partial Gram of pixels [q0, q1) of one slot (load path M).  The
// chunk tile is double-buffered (`tile` holds two of kGramKB x LDW floats):
// the next chunk is staged while the matrix cores read the current one, one
// barrier per chunk.
template <int T, int P, int M, int NPX = 0>
__device__ __forceinline__ void gram_slot(const CubeDesc& d, int64_t q0, int64_t q1, float* tile, int lane,
                                          int wave, v4f (&acc)[TileMap<T, P, NPX>::S],
                                          double (&accd)[TileMap<T, P, NPX>::S][4]) {
    constexpr int S = TileMap<T, P, NPX>::S;
    constexpr int TS = kGramKB * gram_ldw<T>();
    float rg[gram_nr<T>()];
    if (q0 >= q1) return;
    gram_fetch<T, M>(d, q0, q1, rg);
    gram_stage<T, M>(tile, d, rg);
    __syncthreads();
    int cur = 0;
    for (int64_t q = q0; q < q1; q += kGramKB) {
        const bool more = q + kGramKB < q1;
        if (more) gram_fetch<T, M>(d, q + kGramKB, q1, rg);   // overlaps the MFMAs
        const float* tb = tile + cur * TS;
        switch (wave) {
            case 0: gram_wave<T, P, 0, NPX>(tb, lane, acc); break;
            case 1: gram_wave<T, P, 1, NPX>(tb, lane, acc); break;
            case 2: gram_wave<T, P, 2, NPX>(tb, lane, acc); break;
            case 3: gram_wave<T, P, 3, NPX>(tb, lane, acc); break;
            case 4: gram_wave<T, P, 4, NPX>(tb, lane, acc); break;
            case 5: gram_wave<T, P, 5, NPX>(tb, lane, acc); break;
            case 6: gram_wave<T, P, 6, NPX>(tb, lane, acc); break;
            default: gram_wave<T, P, 7, NPX>(tb, lane, acc); break;
        }
        // the other buffer was last read before the previous barrier
        if (more) gram_stage<T, M>(tile + (cur ^ 1) * TS, d, rg);
        // FP32 sums over one chunk only; chunks accumulate in FP64
#pragma unroll
        for (int q2 = 0; q2 < S; ++q2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) accd[q2][i] += (double)acc[q2][i];
            acc[q2] = v4f{0.f, 0.f, 0.f, 0.f};
        }
        __syncthreads();
        cur ^= 1;
    }
}

// The slots of the launch (part P of NPX, or all tiles), the chunk tile in
// `tile`.  LM: the load path of every cube of the launch (the others are
// compiled out), or kAnyLayout (chosen per cube).
template <int T, int P, int LM, int NPX>
__device__ __forceinline__ void gram_f32_items(const CubeDesc* __restrict__ descs, const int* __restrict__ items,
                                               int ncubes, float* tile) {
    using TM = TileMap<T, P, NPX>;
    constexpr int NT = TM::NT;
    constexpr int S = TM::S;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int total = items[ncubes];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int slot = item - items[c];
        const int64_t n = d.n;
        int64_t per = (n + d.gslots - 1) / d.gslots;
        per = (per + kGramKB - 1) / kGramKB * kGramKB;
        const int64_t q0 = (int64_t)slot * per;
        const int64_t q1 = q0 + per < n ? q0 + per : n;
        v4f acc[S];
        double accd[S][4];
#pragma unroll
        for (int q = 0; q < S; ++q) {
            acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; ++i) accd[q][i] = 0.0;
        }
        if constexpr (LM != kAnyLayout) {
            gram_slot<T, P, LM, NPX>(d, q0, q1, tile, lane, wave, acc, accd);
        } else {
            const int m = load_mode(d);
            if (m == kVec) gram_slot<T, P, kVec, NPX>(d, q0, q1, tile, lane, wave, acc, accd);
            else if (m == kDense) gram_slot<T, P, kDense, NPX>(d, q0, q1, tile, lane, wave, acc, accd);
            else gram_slot<T, P, kScalar, NPX>(d, q0, q1, tile, lane, wave, acc, accd);
        }
        float* out = gmem(static_cast<float*>(d.gpart)) + (int64_t)(d.gslot0 + slot) * NT * 256;
        const int col = lane & 15, row = lane >> 4;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int t = TM::T0 + wave * S + q;
            if (t < TM::T1) {
#pragma unroll
                for (int i = 0; i < 4; ++i) out[t * 256 + (4 * row + i) * 16 + col] = (float)accd[q][i];
            }
        }
    }
}

template <int T, int P, int LM>
__global__ __launch_bounds__(kGramThreads) void k_gram_f32(const CubeDesc* __restrict__ descs,
                                                          const int* __restrict__ items, int ncubes) {
    __shared__ __attribute__((aligned(16))) float tile[2 * kGramKB * gram_ldw<T>()];
    gram_f32_items<T, P, LM, 0>(descs, items, ncubes, tile);
}

// A program of few slots (a small cube alone): the tiles of every slot are
// split over gram_wide_parts<T>() blocks (blockIdx.y), each staging the whole
// chunk and computing its part.  Every tile of a slot is summed exactly as in
// the one-block kernel, so G is the same to the bit.
template <int T> __host__ __device__ constexpr int gram_wide_parts() {
    return T * (T + 1) / 2 >= 64 ? 8 : T * (T + 1) / 2 >= 32 ? 4 : T * (T + 1) / 2 >= 16 ? 2 : 1;
}

template <int T, int LM>
__global__ __launch_bounds__(kGramThreads) void k_gram_f32_wide(const CubeDesc* __restrict__ descs,
                                                               const int* __restrict__ items, int ncubes) {
    constexpr int NPX = gram_wide_parts<T>();
    __shared__ __attribute__((aligned(16))) float tile[2 * kGramKB * gram_ldw<T>()];
    const int part = blockIdx.y;
    static_for<NPX>([&](auto pc) {
        constexpr int pp = decltype(pc)::value;
        if (part == pp) gram_f32_items<T, pp + 1, LM, NPX>(descs, items, ncubes, tile);
    });
}

// ------------------------------------------------------------------------
// Mixed precision: each value is split y = hi + lo with hi = bf16(y) and
// lo = bf16(y - hi); G is accumulated on v_mfma_f32_16x16x32_bf16 as
// hi.hi + hi.lo + lo.hi (FP32 accumulation).  The missing lo.lo term has a
// random sign off the diagonal, but on the diagonal it is a positive bias of
// about 2^-16 y^2 that the noise regression would amplify, so diagonal tiles
// also add lo.lo.  The tile in LDS is band-major so that one 16-byte read
// gives a lane its 8 consecutive pixels of one band.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v4f mfma_bf16(bf16x8 a, bf16x8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int kGramLDP = kGramKB + 8;   // bf16 elements per band row (16-byte aligned rows)

template <int T, int P, int WV>
__device__ __forceinline__ void gramb_wave(const __bf16* __restrict__ th, const __bf16* __restrict__ tl,
                                           int lane, v4f (&acc)[TileMap<T, P>::S]) {
    using TM = TileMap<T, P>;
    constexpr int S = TM::S;
    const int col = lane & 15, row = lane >> 4;
#pragma unroll 1
    for (int s = 0; s < kGramKB / 32; ++s) {
        const int base = col * kGramLDP + 32 * s + 8 * row;
        bf16x8 hi_i = {}, lo_i = {};
        static_for<S>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int t = TM::T0 + WV * S + q;
            if constexpr (t < TM::T1) {
                constexpr int i = TM::ti(t), j = TM::tj(t);
                if constexpr (q == 0 || TM::ti(t - 1) != i) {
                    hi_i = *reinterpret_cast<const bf16x8*>(th + base + 16 * i * kGramLDP);
                    lo_i = *reinterpret_cast<const bf16x8*>(tl + base + 16 * i * kGramLDP);
                }
                if constexpr (i == j) {
                    acc[q] = mfma_bf16(hi_i, hi_i, acc[q]);
                    acc[q] = mfma_bf16(hi_i, lo_i, acc[q]);
                    acc[q] = mfma_bf16(lo_i, hi_i, acc[q]);
                    acc[q] = mfma_bf16(lo_i, lo_i, acc[q]);
                } else {
                    const bf16x8 hi_j = *reinterpret_cast<const bf16x8*>(th + base + 16 * j * kGramLDP);
                    const bf16x8 lo_j = *reinterpret_cast<const bf16x8*>(tl + base + 16 * j * kGramLDP);
                    acc[q] = mfma_bf16(hi_i, hi_j, acc[q]);
                    acc[q] = mfma_bf16(hi_i, lo_j, acc[q]);
                    acc[q] = mfma_bf16(lo_i, hi_j, acc[q]);
                }
                // many tiles per wave: keep the scheduler from reading every
                // tile's fragments ahead (registers), two tiles at a time
                if constexpr (S > 8 && (q & 1)) __builtin_amdgcn_sched_barrier(0);
            }
        });
    }
}

// BF16 staging: a task is 8 consecutive pixels x 4 bands; its values are
// split and written as 16-byte rows of the band-major hi and lo tiles.  Task
// pairs differ in the pixel block, so that the 16-byte writes of 8 adjacent
// lanes (4 band groups x 2 pixel blocks) fall in distinct banks; a wave's
// loads are two runs of consecutive band groups.
__device__ __forceinline__ void gramb_task(int task, int T, int& blk, int& g) {
    const int half = task >> 1;
    g = half % (4 * T);
    blk = 2 * (half / (4 * T)) + (task & 1);
}
template <int T> __host__ __device__ constexpr int gramb_ntask() { return (kGramKB / 8) * 4 * T; }
template <int T> __host__ __device__ constexpr int gramb_nt() {
    return (gramb_ntask<T>() + kGramThreads - 1) / kGramThreads;
}

template <int T>
__device__ __forceinline__ void gramb_fetch(const CubeDesc& d, int64_t q, int64_t q1, v4f (&r)[gramb_nt<T>()][8]) {
    const int tid = threadIdx.x;
    const float* base = pixel_ptr<float>(d, q);   // a chunk never crosses an image row
    const int g4 = d.p >> 2;
#pragma unroll
    for (int i = 0; i < gramb_nt<T>(); ++i) {
        const int task = tid + kGramThreads * i;
        int blk, g;
        gramb_task(task, T, blk, g);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = 8 * blk + u;
            v4f v = {0.f, 0.f, 0.f, 0.f};
            if (task < gramb_ntask<T>() && g < g4 && q + k < q1)
                v = *reinterpret_cast<const v4f*>(base + (int64_t)k * d.pitch + 4 * g);
            r[i][u] = v;
        }
    }
}

template <int T>
__device__ __forceinline__ void gramb_stage(__bf16* __restrict__ th, __bf16* __restrict__ tl,
                                           const v4f (&r)[gramb_nt<T>()][8]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < gramb_nt<T>(); ++i) {
        const int task = tid + kGramThreads * i;
        int blk, g;
        gramb_task(task, T, blk, g);
        if (task < gramb_ntask<T>()) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                bf16x8 h8, l8;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float v = r[i][u][c];
                    const __bf16 h = (__bf16)v;
                    h8[u] = h;
                    l8[u] = (__bf16)(v - (float)h);
                }
                *reinterpret_cast<bf16x8*>(th + (4 * g + c) * kGramLDP + 8 * blk) = h8;
                *reinterpret_cast<bf16x8*>(tl + (4 * g + c) * kGramLDP + 8 * blk) = l8;
            }
        }
    }
}

// Scalar staging (strided or unaligned cubes).
template <int T>
__device__ __forceinline__ void gramb_stage_scalar(__bf16* __restrict__ th, __bf16* __restrict__ tl,
                                                  const float (&r)[gram_nr<T>()]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < gram_nv1<T>(); ++i) {
        const int e = tid + kGramThreads * i;
        const int k = e / (16 * T), b = e - k * (16 * T);
        if (k < kGramKB) {
            const float v = r[i];
            const __bf16 h = (__bf16)v;
            th[b * kGramLDP + k] = h;
            tl[b * kGramLDP + k] = (__bf16)(v - (float)h);
        }
    }
}

// Dense BF16 path: a task is 8 consecutive pixels of one band.  Consecutive
// lanes take consecutive bands, so each of the 8 loads of a wave reads one
// run of the chunk and each 16-byte row written to the band-major tiles lands
// in its own banks.  Band slots from p on are left as they were (an entry of G
// reads only its own two bands, and those of bands >= p are never stored).
template <int T> __host__ __device__ constexpr int gramd_nt() { return (kGramKB / 8 * 16 * T + kGramThreads - 1) / kGramThreads; }

template <int T>
__device__ __forceinline__ void gramd_fetch(const CubeDesc& d, int64_t q, int64_t q1, float (&r)[8 * gramd_nt<T>()]) {
    const int tid = threadIdx.x;
    const int p = d.p;
    const float* base = pixel_ptr<float>(d, q);
    const int64_t m64 = q1 - q;
    const int m = (int)(m64 < kGramKB ? m64 : kGramKB);
#pragma unroll
    for (int i = 0; i < gramd_nt<T>(); ++i) {
        const int t = tid + kGramThreads * i;      // over (kGramKB / 8) x p
        const int blk = div_p(t, d.pmag), b = t - blk * p;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = 8 * blk + u;
            r[8 * i + u] = (t < (kGramKB / 8) * p && k < m) ? base[k * p + b] : 0.f;
        }
    }
}

template <int T>
__device__ __forceinline__ void gramd_stage(__bf16* __restrict__ th, __bf16* __restrict__ tl, int p, uint32_t pmag,
                                           const float (&r)[8 * gramd_nt<T>()]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < gramd_nt<T>(); ++i) {
        const int t = tid + kGramThreads * i;
        if (t < (kGramKB / 8) * p) {
            const int blk = div_p(t, pmag), b = t - blk * p;
            bf16x8 h8, l8;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float v = r[8 * i + u];
                const __bf16 h = (__bf16)v;
                h8[u] = h;
                l8[u] = (__bf16)(v - (float)h);
            }
            *reinterpret_cast<bf16x8*>(th + b * kGramLDP + 8 * blk) = h8;
            *reinterpret_cast<bf16x8*>(tl + b * kGramLDP + 8 * blk) = l8;
        }
    }
}

// FP64: chunk sums flushed into FP64 accumulators (else acc keeps summing the
// whole slot in FP32).  M: load path.  The hi/lo tiles are double-buffered
// (th, tl hold two tiles of 16T x kGramLDP each): while the matrix cores read
// one chunk, the next is split and staged into the other buffer, one barrier
// per chunk.
template <int T, int P, int M, bool FP64>
__device__ __forceinline__ void gramb_slot(const CubeDesc& d, int64_t q0, int64_t q1, __bf16* th, __bf16* tl,
                                           int lane, int wave, v4f (&acc)[TileMap<T, P>::S],
                                           double (&accd)[FP64 ? TileMap<T, P>::S : 1][4]) {
    constexpr int S = TileMap<T, P>::S;
    constexpr int TS = 16 * T * kGramLDP;     // elements per buffer
    v4f rv[M == kVec ? gramb_nt<T>() : 1][8];
    float rd[M == kDense ? 8 * gramd_nt<T>() : 1];
    float rs[M == kScalar ? gram_nr<T>() : 1];
    auto fetch = [&](int64_t q) {
        if constexpr (M == kVec) gramb_fetch<T>(d, q, q1, rv);
        else if constexpr (M == kDense) gramd_fetch<T>(d, q, q1, rd);
        else gram_fetch<T, kScalar>(d, q, q1, rs);
    };
    auto stage = [&](int b) {
        if constexpr (M == kVec) gramb_stage<T>(th + b * TS, tl + b * TS, rv);
        else if constexpr (M == kDense) gramd_stage<T>(th + b * TS, tl + b * TS, d.p, d.pmag, rd);
        else gramb_stage_scalar<T>(th + b * TS, tl + b * TS, rs);
    };
    if (q0 >= q1) return;
    fetch(q0);
    stage(0);
    __syncthreads();
    int cur = 0;
    for (int64_t q = q0; q < q1; q += kGramKB) {
        const bool more = q + kGramKB < q1;
        if (more) fetch(q + kGramKB);
        const __bf16* h = th + cur * TS;
        const __bf16* l = tl + cur * TS;
        switch (wave) {
            case 0: gramb_wave<T, P, 0>(h, l, lane, acc); break;
            case 1: gramb_wave<T, P, 1>(h, l, lane, acc); break;
            case 2: gramb_wave<T, P, 2>(h, l, lane, acc); break;
            case 3: gramb_wave<T, P, 3>(h, l, lane, acc); break;
            case 4: gramb_wave<T, P, 4>(h, l, lane, acc); break;
            case 5: gramb_wave<T, P, 5>(h, l, lane, acc); break;
            case 6: gramb_wave<T, P, 6>(h, l, lane, acc); break;
            default: gramb_wave<T, P, 7>(h, l, lane, acc); break;
        }
        // the other buffer was last read before the previous barrier
        if (more) stage(cur ^ 1);
        if constexpr (FP64) {
#pragma unroll
            for (int q2 = 0; q2 < S; ++q2) {
#pragma unroll
                for (int i = 0; i < 4; ++i) accd[q2][i] += (double)acc[q2][i];
                acc[q2] = v4f{0.f, 0.f, 0.f, 0.f};
            }
        }
        __syncthreads();
        cur ^= 1;
    }
}

// From T = kGramSplitT on, the FP64 accumulators of all upper tiles would not
// fit in registers: the tiles of a slot then accumulate in FP32 across the
// whole slot (a few thousand pixels; the FP64 reduce over slots follows), one
// launch reads Y once.  The split-BF16 products themselves carry a relative
// error near 2^-16, above what the FP32 sums add.
constexpr int kGramSplitT = 11;

template <int T, int P, int LM>
__global__ __launch_bounds__(kGramThreads) void k_gram_bf16(const CubeDesc* __restrict__ descs,
                                                           const int* __restrict__ items, int ncubes) {
    using TM = TileMap<T, P>;
    constexpr int NT = TM::NT;
    constexpr int S = TM::S;
    constexpr bool FP64 = T < kGramSplitT;
    __shared__ __attribute__((aligned(16))) __bf16 th[2 * 16 * T * kGramLDP];
    __shared__ __attribute__((aligned(16))) __bf16 tl[2 * 16 * T * kGramLDP];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int total = items[ncubes];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int slot = item - items[c];
        const int64_t n = d.n;
        int64_t per = (n + d.gslots - 1) / d.gslots;
        per = (per + kGramKB - 1) / kGramKB * kGramKB;
        const int64_t q0 = (int64_t)slot * per;
        const int64_t q1 = q0 + per < n ? q0 + per : n;
        v4f acc[S];
        double accd[FP64 ? S : 1][4];
#pragma unroll
        for (int q = 0; q < S; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < (FP64 ? S : 1); ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) accd[q][i] = 0.0;
        if constexpr (LM != kAnyLayout) {
            gramb_slot<T, P, LM, FP64>(d, q0, q1, th, tl, lane, wave, acc, accd);
        } else {
            const int m = load_mode(d);
            if (m == kVec) gramb_slot<T, P, kVec, FP64>(d, q0, q1, th, tl, lane, wave, acc, accd);
            else if (m == kDense) gramb_slot<T, P, kDense, FP64>(d, q0, q1, th, tl, lane, wave, acc, accd);
            else gramb_slot<T, P, kScalar, FP64>(d, q0, q1, th, tl, lane, wave, acc, accd);
        }
        float* out = gmem(static_cast<float*>(d.gpart)) + (int64_t)(d.gslot0 + slot) * NT * 256;
        const int col = lane & 15, row = lane >> 4;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int t = TM::T0 + wave * S + q;
            if (t < TM::T1) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v;
                    if constexpr (FP64) v = (float)accd[q][i];
                    else v = acc[q][i];
                    out[t * 256 + (4 * row + i) * 16 + col] = v;
                }
            }
        }
    }
}

// Sum the FP32 partials of every slot of a cube in FP64 (fixed order) into G.
// A block reduces 32 entries; its 8 thread groups each sum every 8th slot
// (eight loads in flight per thread), then the 8 group sums are added in order.
constexpr int kRedGroups = 8;

__global__ __launch_bounds__(256) void k_gram_reduce_f32(const CubeDesc* __restrict__ descs,
                                                        const int* __restrict__ cubes, int ncubes_in_class) {
    __shared__ double part[kRedGroups][32];
    const int k = blockIdx.y;
    if (k >= ncubes_in_class) return;
    const CubeDesc& d = descs[cubes[k]];
    const int T = d.T, NT = T * (T + 1) / 2;
    const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int e = blockIdx.x * 32 + lane;
    const bool live = e < NT * 256;
    const int64_t stride = (int64_t)NT * 256;
    const float* pbase = gmem(static_cast<const float*>(d.gpart)) + (int64_t)d.gslot0 * stride + (live ? e : 0);
    double s = 0.0;
    int sl = grp;
    for (; sl + 7 * kRedGroups < d.gslots; sl += 8 * kRedGroups) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pbase[(int64_t)(sl + u * kRedGroups) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; sl < d.gslots; sl += kRedGroups) s += (double)pbase[(int64_t)sl * stride];
    part[grp][lane] = s;
    __syncthreads();
    if (grp == 0 && live) {
        double tot = 0.0;
#pragma unroll
        for (int g = 0; g < kRedGroups; ++g) tot += part[g][lane];
        const int t = e >> 8, m = (e >> 4) & 15, nn = e & 15;
        int i = 0, rem = t;
        while (rem >= T - i) { rem -= T - i; ++i; }
        const int j = i + rem;
        const int a = 16 * i + m, b = 16 * j + nn;
        // a diagonal tile holds both (a, b) and (b, a); the products of the split
        // BF16 path reach them in different orders, so only the upper entry is
        // written, to both places (one writer per address)
        if (a < d.p && b < d.p && a <= b) {
            d.G[(int64_t)a * d.p + b] = tot;
            d.G[(int64_t)b * d.p + a] = tot;
            // a NaN or Inf anywhere in band a makes G_aa non-finite
            if (a == b && !__builtin_isfinite(tot)) set_status(d.status, HYRES_DEV_NONFINITE);
        }
    }
}

// FP64 Gram: grid.x covers upper-triangle entries, grid.y the slots of one cube.
__global__ void k_gram_f64(const CubeDesc* __restrict__ descs, int cube) {
    const CubeDesc& d = descs[cube];
    const int p = d.p;
    const int ntri = p * (p + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int slot = blockIdx.y;
    if (e >= ntri || slot >= d.gslots) return;
    int a = 0, rem = e;
    while (rem >= p - a) { rem -= p - a; ++a; }
    const int b = a + rem;
    const int64_t per = (d.n + d.gslots - 1) / d.gslots;
    const int64_t q0 = (int64_t)slot * per;
    const int64_t q1 = q0 + per < d.n ? q0 + per : d.n;
    double s = 0.0;
    int bad = 0;
    for (int64_t q = q0; q < q1; ++q) {
        const double* y = pixel_ptr<double>(d, q);
        const double ya = y[a], yb = y[b];
        if (a == b) bad |= !__builtin_isfinite(ya);
        s = fma(ya, yb, s);
    }
    if (bad) set_status(d.status, HYRES_DEV_NONFINITE);
    gmem(static_cast<double*>(d.gpart))[(int64_t)(d.gslot0 + slot) * ntri + e] = s;
}

__global__ void k_gram_reduce_f64(const CubeDesc* __restrict__ descs, int cube) {
    const CubeDesc& d = descs[cube];
    const int p = d.p;
    const int ntri = p * (p + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntri) return;
    int a = 0, rem = e;
    while (rem >= p - a) { rem -= p - a; ++a; }
    const int b = a + rem;
    const double* part = gmem(static_cast<const double*>(d.gpart)) + (int64_t)d.gslot0 * ntri + e;
    double s = 0.0;
    for (int sl = 0; sl < d.gslots; ++sl) s += part[(int64_t)sl * ntri];
    d.G[(int64_t)a * p + b] = s;
    d.G[(int64_t)b * p + a] = s;
}

// ---------------------------------------------------------------- launchers
typedef void (*GramF32Kernel)(const CubeDesc*, const int*, int);

// FP32 cubes in native precision: from T = kGramSplitT up, with the scalar
// load path compiled in, the FP64 accumulators of all tiles no longer fit in
// the registers of 8 waves; the tiles are then split over two launches (three
// from T = 13).

template <int T, int P, int LM>
static void launch_gram_k(const CubeDesc* descs, const int* items, int ncubes, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_gram_f32<T, P, LM>), dim3(grid), dim3(kGramThreads), 0, s, descs, items, ncubes);
}

// the scalar load path needs more registers: from T = kGramSplitT on the tiles
// are split over launches
template <int T, int LM>
static void launch_gram_parts(const CubeDesc* descs, const int* items, int ncubes, int grid, hipStream_t s) {
    if constexpr (T < kGramSplitT) {
        launch_gram_k<T, 0, LM>(descs, items, ncubes, grid, s);
    } else {
        launch_gram_k<T, 1, LM>(descs, items, ncubes, grid, s);
        launch_gram_k<T, 2, LM>(descs, items, ncubes, grid, s);
        if constexpr (TileMap<T, 1>::NP == 3) launch_gram_k<T, 3, LM>(descs, items, ncubes, grid, s);
    }
}

template <int T>
static hipError_t launch_gram_t(int lm, const CubeDesc* descs, const int* items, int ncubes, int grid,
                                hipStream_t s, bool wide) {
    // the split launch for the vector and dense load paths (strided cubes keep
    // the one-block kernel)
    if (wide && gram_wide_parts<T>() > 1 && (lm == kVec || lm == kDense)) {
        const dim3 g((unsigned)grid, (unsigned)gram_wide_parts<T>());
        if (lm == kVec) hipLaunchKernelGGL((k_gram_f32_wide<T, kVec>), g, dim3(kGramThreads), 0, s, descs, items, ncubes);
        else hipLaunchKernelGGL((k_gram_f32_wide<T, kDense>), g, dim3(kGramThreads), 0, s, descs, items, ncubes);
        return hipGetLastError();
    }
    // with one load path compiled in, every tile's FP64 accumulators stay in
    // registers up to T = 14: one pass over Y
    if (lm == kVec) {
        launch_gram_k<T, 0, kVec>(descs, items, ncubes, grid, s);
    } else if (lm == kDense) {
        // from T = 13 the dense staging's registers push the accumulators out
        if constexpr (T >= 13) launch_gram_parts<T, kDense>(descs, items, ncubes, grid, s);
        else launch_gram_k<T, 0, kDense>(descs, items, ncubes, grid, s);
    } else if (lm == kScalar) {
        launch_gram_parts<T, kScalar>(descs, items, ncubes, grid, s);
    } else {
        launch_gram_parts<T, kAnyLayout>(descs, items, ncubes, grid, s);
    }
    return hipGetLastError();
}

template <int T>
static hipError_t launch_gramb_t(int lm, const CubeDesc* descs, const int* items, int ncubes, int grid,
                                 hipStream_t s) {
    if (lm == kVec) hipLaunchKernelGGL((k_gram_bf16<T, 0, kVec>), dim3(grid), dim3(kGramThreads), 0, s, descs, items, ncubes);
    else if (lm == kDense) hipLaunchKernelGGL((k_gram_bf16<T, 0, kDense>), dim3(grid), dim3(kGramThreads), 0, s, descs, items, ncubes);
    else if (lm == kScalar) hipLaunchKernelGGL((k_gram_bf16<T, 0, kScalar>), dim3(grid), dim3(kGramThreads), 0, s, descs, items, ncubes);
    else hipLaunchKernelGGL((k_gram_bf16<T, 0, kAnyLayout>), dim3(grid), dim3(kGramThreads), 0, s, descs, items, ncubes);
    return hipGetLastError();
}

hipError_t launch_gram_bf16(int T, int lm, const CubeDesc* descs, const int* items, int ncubes, int grid,
                            hipStream_t s) {
    switch (T) {
#define HYRES_G(TT) case TT: return launch_gramb_t<TT>(lm, descs, items, ncubes, grid, s);
        HYRES_G(1) HYRES_G(2) HYRES_G(3) HYRES_G(4) HYRES_G(5) HYRES_G(6) HYRES_G(7)
        HYRES_G(8) HYRES_G(9) HYRES_G(10) HYRES_G(11) HYRES_G(12) HYRES_G(13) HYRES_G(14)
#undef HYRES_G
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gram_f32(int T, int lm, const CubeDesc* descs, const int* items, int ncubes, int grid,
                           hipStream_t s, bool wide) {
    switch (T) {
#define HYRES_G(TT) case TT: return launch_gram_t<TT>(lm, descs, items, ncubes, grid, s, wide);
        HYRES_G(1) HYRES_G(2) HYRES_G(3) HYRES_G(4) HYRES_G(5) HYRES_G(6) HYRES_G(7)
        HYRES_G(8) HYRES_G(9) HYRES_G(10) HYRES_G(11) HYRES_G(12) HYRES_G(13) HYRES_G(14)
#undef HYRES_G
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gram_reduce_f32(int T, const CubeDesc* descs, const int* cubes, int ncls,
                                  hipStream_t s) {
    const int NT = T * (T + 1) / 2;
    dim3 grid((NT * 256 + 31) / 32, ncls);
    hipLaunchKernelGGL(k_gram_reduce_f32, grid, dim3(256), 0, s, descs, cubes, ncls);
    return hipGetLastError();
}

hipError_t launch_gram_f64(const CubeDesc* descs, int cube, int p, int gslots, hipStream_t s) {
    const int ntri = p * (p + 1) / 2;
    hipLaunchKernelGGL(k_gram_f64, dim3((ntri + 255) / 256, gslots), dim3(256), 0, s, descs, cube);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_reduce_f64, dim3((ntri + 255) / 256), dim3(256), 0, s, descs, cube);
    return hipGetLastError();
}

}  // namespace hyres
