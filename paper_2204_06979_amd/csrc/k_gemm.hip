// Projection Z = Y (D^-1 V) and back-projection Xhat = Zhat (V^T D).
//
// Both are skinny products (r <= 16 columns) that stream the cube once; they
// are HBM-bound.  FP32 cubes run them on the matrix cores
// (v_mfma_f32_16x16x4f32): a 16 x 16 output tile per wave, 16 pixels by 16
// components (projection) or 16 pixels by 16 bands (back-projection).  The
// cube tile of the projection is staged through LDS with coalesced loads; the
// small matrices stay in registers as MFMA fragments.  FP64 cubes use plain
// FP64 FMAs, one pixel per thread.
#include "tile_stage.hpp"

namespace hyres {

// LM: the load path of every cube of the launch, or kAnyLayout (chosen per
// cube).  With the vector or dense path alone the registers stay within two
// waves per SIMD.
template <int T, int LM>
__global__ __launch_bounds__(256, LM == kVec || LM == kDense ? 2 : 1) void k_project_f32(const CubeDesc* __restrict__ descs,
                                                    const int* __restrict__ items, int ncubes) {
    constexpr int LDW = proj_ldw<T>();
    __shared__ __attribute__((aligned(16))) float tile[kPixTile * LDW];
    __shared__ float s_m[4][256];            // per-wave Z^T Z of a tile (mixed solves)
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, row = lane >> 4;
    const int total = items[ncubes];
    int cur = -1;
    float bf[4 * T];
    v4f r4[proj_nv4<T>()];
    int zlo = 16 * T;                        // band slots from zlo on are zero in the tile
    int item = blockIdx.x;
    if (item < total) {
        const int c = find_cube(items, ncubes, item);
        if constexpr (LM != kAnyLayout) proj_fetch<T, LM>(descs[c], (int64_t)(item - items[c]) * kPixTile, r4);
        else proj_fetch_any<T>(descs[c], (int64_t)(item - items[c]) * kPixTile, r4);
    }
    for (; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        if (c != cur) {
            cur = c;
#pragma unroll
            for (int s = 0; s < 4 * T; ++s) bf[s] = gmem(d.P32)[(4 * s + row) * 16 + col];
        }
        const int64_t q0 = (int64_t)(item - items[c]) * kPixTile;
        __syncthreads();
        if constexpr (LM != kAnyLayout) {
            proj_stage<T, LM>(tile, d, zlo, r4);
        } else {
            proj_stage_any<T>(tile, d, zlo, r4);
        }
        __syncthreads();
        const int nxt = item + gridDim.x;
        if (nxt < total) {
            const int c2 = find_cube(items, ncubes, nxt);
            if constexpr (LM != kAnyLayout) proj_fetch<T, LM>(descs[c2], (int64_t)(nxt - items[c2]) * kPixTile, r4);
            else proj_fetch_any<T>(descs[c2], (int64_t)(nxt - items[c2]) * kPixTile, r4);
        }
        // four independent accumulator chains (consecutive MFMAs do not wait
        // on each other's results), added in a fixed order
        v4f ac[4] = {};
        const float* arow = tile + (16 * wave + col) * LDW + row;
#pragma unroll
        for (int s = 0; s < 4 * T; ++s) {
            ac[s & 3] = mfma4(arow[4 * s], bf[s], ac[s & 3]);
            // bounded look-ahead of the LDS reads: the registers stay low
            // enough for two waves per SIMD
            if ((s & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        const v4f acc = (ac[0] + ac[1]) + (ac[2] + ac[3]);
        // lane holds component col of pixels q0 + 16 wave + 4 row + i
        if (col < d.r) {
            float* z = gmem(static_cast<float*>(d.Z)) + (int64_t)col * d.nz + q0 + 16 * wave + 4 * row;
            *reinterpret_cast<v4f*>(z) = acc;
        }
        if (d.rpart) {
            // Z^T Z over the tile for the Rayleigh-Ritz refinement: register i of
            // acc holds pixels {4g + i} of the wave's 16 in exactly the operand
            // layout of a 4-deep MFMA step, so four steps cover the 16 pixels
            v4f m = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; ++i) m = mfma4(acc[i], acc[i], m);
#pragma unroll
            for (int i = 0; i < 4; ++i) s_m[wave][(4 * row + i) * 16 + col] = m[i];
            __syncthreads();
            const int e = threadIdx.x;
            gmem(d.rpart)[(q0 / kPixTile) * 256 + e] = ((s_m[0][e] + s_m[1][e]) + s_m[2][e]) + s_m[3][e];
        }
    }
}

// X is written once and not read again here: non-temporal stores.
template <int T>
__global__ __launch_bounds__(256) void k_backproject_f32(const CubeDesc* __restrict__ descs,
                                                        const int* __restrict__ items, int ncubes) {
    constexpr int P16 = 16 * T;
    constexpr int LDO = P16 + 4;
    __shared__ __attribute__((aligned(16))) float ot[kPixTile * LDO];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, row = lane >> 4;
    const int total = items[ncubes];
    int cur = -1;
    float bq[4][T];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int r = d.r, p = d.p;
        const int R4 = (r + 3) >> 2;
        if (c != cur) {
            cur = c;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < T; ++j) bq[q][j] = gmem(d.Q32)[(4 * q + row) * P16 + 16 * j + col];
        }
        const int64_t q0 = (int64_t)(item - items[c]) * kPixTile;
        // A fragments: Zhat[comp 4q + row][pixel q0 + 16 wave + col]
        float a[4];
        const float* zh = gmem(static_cast<const float*>(d.Z));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int comp = 4 * q + row;
            a[q] = (q < R4 && comp < r) ? zh[(int64_t)comp * d.nz + q0 + 16 * wave + col] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < T; ++j) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < R4) acc = mfma4(a[q], bq[q][j], acc);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) ot[(16 * wave + 4 * row + i) * LDO + 16 * j + col] = acc[i];
        }
        const int64_t nleft = d.n - q0;
        __syncthreads();
        if (d.xvec4) {
            // whole 64-pixel tiles per image row: the pixels are consecutive in memory
            const int g4 = p >> 2;
            const int64_t y0 = q0 / d.W, x0 = q0 - y0 * d.W;
            float* base = gmem(static_cast<float*>(d.X)) + y0 * d.xrow_pitch + x0 * d.xpitch;
            for (int e = threadIdx.x; e < kPixTile * g4; e += 256) {
                const int k = e / g4, g = e - k * g4;
                if (k < nleft)
                    __builtin_nontemporal_store(*reinterpret_cast<const v4f*>(ot + k * LDO + 4 * g),
                                                reinterpret_cast<v4f*>(base + (int64_t)k * d.xpitch + 4 * g));
            }
        } else if (d.xdense) {
            // unpadded pixels: the tile is 64 p consecutive floats, written as float4s
            float* base = gmem(static_cast<float*>(d.X)) + (q0 / d.W) * d.xrow_pitch + (q0 % d.W) * p;
            const int lim = (int)(nleft < kPixTile ? nleft : kPixTile) * p;
            for (int e = 4 * threadIdx.x; e < lim; e += 4 * 256) {
                v4f v;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int k = div_p(e + c, d.pmag);   // k < 64: e + 3 < 64 p
                    v[c] = ot[k * LDO + (e + c - k * p)];
                }
                if (e + 3 < lim) {
                    __builtin_nontemporal_store(v, reinterpret_cast<v4f*>(base + e));
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (e + c < lim) __builtin_nontemporal_store(v[c], base + e + c);
                }
            }
        } else {
            for (int e = threadIdx.x; e < kPixTile * p; e += 256) {
                const int k = div_p(e, d.pmag), b = e - k * p;
                if (k < nleft) {
                    const int64_t q = q0 + k;
                    const int64_t y = q / d.W, x = q - y * d.W;
                    __builtin_nontemporal_store(ot[k * LDO + b],
                                                gmem(static_cast<float*>(d.X)) + y * d.xrow_pitch + x * d.xpitch + b);
                }
            }
        }
    }
}

// Sliding-window back-projection in one pass over the output image.  An item
// is a run of 64 pixels of one image row; for every tile covering part of the
// run, the matrix cores form that tile's Zhat Q (16 pixels by 16 bands per
// wave and MFMA block), and each pixel adds its blend weight (the two 1-D
// weights of the tile) times the product, tiles in raster order.  X is written
// once, without reading it (non-temporal stores).  Blocks take contiguous runs
// of items, so the Q fragments stay in registers across the runs inside one
// tile.
template <int T>
__global__ __launch_bounds__(256) void k_blend_f32(const CubeDesc* __restrict__ descs, const BlendGrid g) {
    constexpr int P16 = 16 * T;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, row = lane >> 4;
    const int p = g.p;
    const int nseg = (g.W + kPixTile - 1) / kPixTile;
    const int64_t total = (int64_t)g.H * nseg;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per;
    const int64_t i1 = i0 + per < total ? i0 + per : total;
    int cur = -1;
    float bq[4][T];
    for (int64_t item = i0; item < i1; ++item) {
        const int y = (int)(item / nseg);
        const int x0 = (int)(item - (int64_t)y * nseg) * kPixTile;
        v4f acc[T];
#pragma unroll
        for (int j = 0; j < T; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int iy = 0; iy < g.ny; ++iy) {
            const int ly = y - g.sy[iy];
            if (ly < 0 || ly >= g.th) continue;
            for (int ix = 0; ix < g.nx; ++ix) {
                const int sx = g.sx[ix];
                if (sx >= x0 + kPixTile || sx + g.tw <= x0) continue;
                const int t = iy * g.nx + ix;
                const CubeDesc& d = descs[t];
                if (t != cur) {
                    cur = t;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int j = 0; j < T; ++j) bq[q][j] = gmem(d.Q32)[(4 * q + row) * P16 + 16 * j + col];
                }
                const int r = d.r, R4 = (r + 3) >> 2;
                // A fragments: Zhat[comp 4q + row] at the tile pixel of image column x0 + 16 wave + col
                const int lxa = x0 + 16 * wave + col - sx;
                const bool va = lxa >= 0 && lxa < g.tw;
                const int64_t qa = (int64_t)ly * g.tw + (va ? lxa : 0);
                const float* zh = gmem(static_cast<const float*>(d.Z));
                float a[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int comp = 4 * q + row;
                    a[q] = (va && q < R4 && comp < r) ? zh[(int64_t)comp * d.nz + qa] : 0.f;
                }
                // blend weights of this lane's output pixels x0 + 16 wave + 4 row + i
                const double wy = d.bwy[ly];
                float w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int lx = x0 + 16 * wave + 4 * row + i - sx;
                    w[i] = (lx >= 0 && lx < g.tw) ? (float)(wy * d.bwx[lx]) : 0.f;
                }
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    v4f pr = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (q < R4) pr = mfma4(a[q], bq[q][j], pr);
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[j][i] = fmaf(w[i], pr[i], acc[j][i]);
                }
            }
        }
        // straight from the accumulators: 16 lanes store 16 consecutive bands
        // of one pixel (64 bytes), no staging through LDS
        const int m = g.W - x0 < kPixTile ? g.W - x0 : kPixTile;   // pixels of the run
        float* base = static_cast<float*>(g.X) + (int64_t)y * g.xrow_pitch + (int64_t)x0 * g.xpitch;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int px = 16 * wave + 4 * row + i;
            if (px < m) {
                float* dst = base + (int64_t)px * g.xpitch + col;
#pragma unroll
                for (int j = 0; j < T; ++j)
                    if (16 * j + col < p) __builtin_nontemporal_store(acc[j][i], dst + 16 * j);
            }
        }
    }
}

// FP64: one pixel per thread.
__global__ void k_project_f64(const CubeDesc* __restrict__ descs, int cube) {
    const CubeDesc& d = descs[cube];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    const double* y = pixel_ptr<double>(d, q);
    double acc[kMaxRank];
    for (int g = 0; g < kMaxRank; ++g) acc[g] = 0.0;
    for (int b = 0; b < d.p; ++b) {
        const double v = y[b];
        for (int g = 0; g < d.r; ++g) acc[g] = fma(v, d.P64[(int64_t)b * d.r + g], acc[g]);
    }
    double* z = gmem(static_cast<double*>(d.Z));
    for (int g = 0; g < d.r; ++g) z[(int64_t)g * d.nz + q] = acc[g];
}

__global__ void k_backproject_f64(const CubeDesc* __restrict__ descs, int cube) {
    const CubeDesc& d = descs[cube];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    const double* zh = gmem(static_cast<const double*>(d.Z));
    double a[kMaxRank];
    for (int g = 0; g < d.r; ++g) a[g] = zh[(int64_t)g * d.nz + q];
    const int64_t y = q / d.W, x = q - y * d.W;
    double* xo = gmem(static_cast<double*>(d.X)) + y * d.xrow_pitch + x * d.xpitch;
    bool first = true;
    const double w = d.bwy ? blend_weight(d, y, x, &first) : 1.0;
    for (int b = 0; b < d.p; ++b) {
        double s = 0.0;
        for (int g = 0; g < d.r; ++g) s = fma(a[g], d.Q64[(int64_t)g * d.p + b], s);
        if (d.bwy) s = first ? s * w : fma(s, w, xo[b]);
        xo[b] = s;
    }
}

// ---------------------------------------------------------------- launchers
template <int T>
static void launch_proj_t(int lm, const CubeDesc* descs, const int* items, int ncubes, int grid, hipStream_t s) {
    if (lm == kVec) hipLaunchKernelGGL((k_project_f32<T, kVec>), dim3(grid), dim3(256), 0, s, descs, items, ncubes);
    else if (lm == kDense) hipLaunchKernelGGL((k_project_f32<T, kDense>), dim3(grid), dim3(256), 0, s, descs, items, ncubes);
    else if (lm == kScalar) hipLaunchKernelGGL((k_project_f32<T, kScalar>), dim3(grid), dim3(256), 0, s, descs, items, ncubes);
    else hipLaunchKernelGGL((k_project_f32<T, kAnyLayout>), dim3(grid), dim3(256), 0, s, descs, items, ncubes);
}
template <int T>
static void launch_bp_t(const CubeDesc* descs, const int* items, int ncubes, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_backproject_f32<T>, dim3(grid), dim3(256), 0, s, descs, items, ncubes);
}

hipError_t launch_project_f32(int T, int lm, const CubeDesc* descs, const int* items, int ncubes, int grid,
                              hipStream_t s) {
    switch (T) {
#define HYRES_P(TT) case TT: launch_proj_t<TT>(lm, descs, items, ncubes, grid, s); break;
        HYRES_P(1) HYRES_P(2) HYRES_P(3) HYRES_P(4) HYRES_P(5) HYRES_P(6) HYRES_P(7)
        HYRES_P(8) HYRES_P(9) HYRES_P(10) HYRES_P(11) HYRES_P(12) HYRES_P(13) HYRES_P(14)
#undef HYRES_P
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_backproject_f32(int T, const CubeDesc* descs, const int* items, int ncubes, int grid,
                                  hipStream_t s) {
    switch (T) {
#define HYRES_B(TT) case TT: launch_bp_t<TT>(descs, items, ncubes, grid, s); break;
        HYRES_B(1) HYRES_B(2) HYRES_B(3) HYRES_B(4) HYRES_B(5) HYRES_B(6) HYRES_B(7)
        HYRES_B(8) HYRES_B(9) HYRES_B(10) HYRES_B(11) HYRES_B(12) HYRES_B(13) HYRES_B(14)
#undef HYRES_B
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_blend_f32(int T, const CubeDesc* descs, const BlendGrid& g, int grid, hipStream_t s) {
    switch (T) {
#define HYRES_B(TT) \
    case TT: hipLaunchKernelGGL(k_blend_f32<TT>, dim3(grid), dim3(256), 0, s, descs, g); break;
        HYRES_B(1) HYRES_B(2) HYRES_B(3) HYRES_B(4) HYRES_B(5) HYRES_B(6) HYRES_B(7)
        HYRES_B(8) HYRES_B(9) HYRES_B(10) HYRES_B(11) HYRES_B(12) HYRES_B(13) HYRES_B(14)
#undef HYRES_B
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_project_f64(const CubeDesc* descs, int cube, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_project_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, descs, cube);
    return hipGetLastError();
}

hipError_t launch_backproject_f64(const CubeDesc* descs, int cube, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_backproject_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, descs, cube);
    return hipGetLastError();
}

}  // namespace hyres
