// Loaders of one 64-pixel tile of an FP32 cube (all 16T band slots) into
// registers and from there into an LDS tile of stride proj_ldw<T>() floats per
// pixel, shared by the projection and the adjoint's pixel products.  D is a
// CubeDesc or a CubeView.
#pragma once
#include "hyres_internal.hpp"

namespace hyres {

// LDS row stride (floats) of a 64-pixel x 16T-band tile; the MFMA A fragment
// reads 16 rows x 4 columns, so rows are offset by 4 banks.
template <int T>
__host__ __device__ constexpr int proj_ldw() { return 16 * T + 4; }
template <int T> __host__ __device__ constexpr int proj_nv4() { return (kPixTile * 4 * T + 255) / 256; }
template <int T> __host__ __device__ constexpr int proj_nv1() { return (kPixTile * 16 * T + 255) / 256; }

// Registers holding one 64-pixel tile of the cube (all 16T band slots).
// One register array serves both load paths: T float4 groups or 4T floats.
static_assert(proj_nv1<1>() == 4 * proj_nv4<1>(), "projection staging sizes");

template <int T, int M, typename D>
__device__ __forceinline__ void proj_fetch(const D& d, int64_t q0, v4f (&r4)[proj_nv4<T>()]) {
    const int tid = threadIdx.x;
    const int64_t nleft = d.n - q0;
    if constexpr (M == kVec) {
        const float* base = pixel_ptr<float>(d, q0);   // a tile never crosses an image row
        const int g4 = d.p >> 2;
#pragma unroll
        for (int i = 0; i < proj_nv4<T>(); ++i) {
            const int e = tid + 256 * i;
            const int k = e / (4 * T), g = e - k * (4 * T);
            v4f v = {0.f, 0.f, 0.f, 0.f};
            if (k < kPixTile && g < g4 && k < nleft)
                v = *reinterpret_cast<const v4f*>(base + (int64_t)k * d.pitch + 4 * g);
            r4[i] = v;
        }
    } else if constexpr (M == kDense) {
        // consecutive lanes read consecutive floats of the tile (float i of the
        // thread is float tid + 256 i)
        const float* base = pixel_ptr<float>(d, q0);
        const int lim = (int)(nleft < kPixTile ? nleft : kPixTile) * d.p;   // floats of the tile
#pragma unroll
        for (int i = 0; i < proj_nv1<T>(); ++i) {
            const int e = tid + 256 * i;
            r4[i >> 2][i & 3] = e < lim ? base[e] : 0.f;
        }
    } else {
#pragma unroll
        for (int i = 0; i < proj_nv1<T>(); ++i) {
            const int e = tid + 256 * i;
            const int k = e / (16 * T), b = e - k * (16 * T);
            float v = 0.f;
            if (k < kPixTile && b < d.p && k < nleft) v = pixel_ptr<float>(d, q0 + k)[b];
            r4[i >> 2][i & 3] = v;
        }
    }
}

// kVec and kScalar write every band slot of the tile (zeros from band p on);
// kDense writes bands [0, p) only and clears the slots [p, zlo) that an earlier
// tile of more bands left behind (slots from zlo on are known to be zero).
template <int T, int M, typename D>
__device__ __forceinline__ void proj_stage(float* __restrict__ tile, const D& d, int& zlo,
                                           const v4f (&r4)[proj_nv4<T>()]) {
    constexpr int LDW = proj_ldw<T>();
    const int tid = threadIdx.x;
    if constexpr (M == kVec) {
#pragma unroll
        for (int i = 0; i < proj_nv4<T>(); ++i) {
            const int e = tid + 256 * i;
            const int k = e / (4 * T), g = e - k * (4 * T);
            if (k < kPixTile) *reinterpret_cast<v4f*>(tile + k * LDW + 4 * g) = r4[i];
        }
    } else if constexpr (M == kDense) {
        const int p = d.p;
        if (p < zlo) {
            const int w = zlo - p;
            for (int e = tid; e < kPixTile * w; e += 256) {
                const int k = e / w;
                tile[k * LDW + p + (e - k * w)] = 0.f;
            }
        }
#pragma unroll
        for (int i = 0; i < proj_nv1<T>(); ++i) {
            const int e = tid + 256 * i;
            if (e < kPixTile * p) {
                const int k = div_p(e, d.pmag);
                tile[k * LDW + (e - k * p)] = r4[i >> 2][i & 3];
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < proj_nv1<T>(); ++i) {
            const int e = tid + 256 * i;
            const int k = e / (16 * T), b = e - k * (16 * T);
            if (k < kPixTile) tile[k * LDW + b] = r4[i >> 2][i & 3];
        }
    }
    zlo = d.p;
}

template <int T, typename D>
__device__ __forceinline__ void proj_fetch_any(const D& d, int64_t q0, v4f (&r4)[proj_nv4<T>()]) {
    const int m = load_mode(d);
    if (m == kVec) proj_fetch<T, kVec>(d, q0, r4);
    else if (m == kDense) proj_fetch<T, kDense>(d, q0, r4);
    else proj_fetch<T, kScalar>(d, q0, r4);
}

// Stage with the load path chosen per cube.
template <int T, typename D>
__device__ __forceinline__ void proj_stage_any(float* __restrict__ tile, const D& d, int& zlo,
                                               const v4f (&r4)[proj_nv4<T>()]) {
    const int m = load_mode(d);
    if (m == kVec) proj_stage<T, kVec>(tile, d, zlo, r4);
    else if (m == kDense) proj_stage<T, kDense>(tile, d, zlo, r4);
    else proj_stage<T, kScalar>(tile, d, zlo, r4);
}

}  // namespace hyres
