// One level of the periodised 2-D Daubechies-4 transform and its inverse.
//
// Analysis along one axis of length N: if N is odd the axis is first extended
// by repeating its last sample (N' = N + 1); then
//   a[k] = sum_m h[m] x[(2k+m) mod N'],  d[k] = sum_m g[m] x[(2k+m) mod N'].
// Synthesis is the transpose: x[2t]   = h0 a[t] + h2 a[t-1] + g0 d[t] + g2 d[t-1],
//                             x[2t+1] = h1 a[t] + h3 a[t-1] + g1 d[t] + g3 d[t-1],
// indices of a, d taken mod N'/2, and the repeated sample is dropped.
//
// A block computes a TY x TX tile of outputs.  The input window it needs
// (with the periodic / odd-length index map applied) is staged in LDS with
// coalesced loads, so every input element is read from HBM about once.  The
// inverse applies the soft threshold sign(b) max(|b| - lambda, 0) as the
// coefficients are loaded, so thresholded coefficients are never stored.
//
// The adjoint of the solve needs the transposes of both maps.  At an odd
// length they differ from the other direction only at the extra sample: the
// transpose of the inverse is the analysis with a zero extra sample
// (kModeZeroPad), and the transpose of the analysis is the synthesis with the
// extra output sample added to the last one (kModeFold).
#include "hyres_internal.hpp"

namespace hyres {

template <typename T>
struct Filt {
    static constexpr T h0 = (T)kH0, h1 = (T)kH1, h2 = (T)kH2, h3 = (T)kH3;
    // g[m] = (-1)^m h[3-m]
    static constexpr T g0 = (T)kH3, g1 = (T)(-kH2), g2 = (T)kH1, g3 = (T)(-kH0);
};

template <typename T>
__device__ __forceinline__ T soft(T v, T lam) {
    const T a = (v < (T)0 ? -v : v) - lam;
    return a > (T)0 ? (v < (T)0 ? -a : a) : (T)0;
}

// Approximation buffer of level l (l >= 1) inside the temp area of a component.
template <typename T>
__device__ __forceinline__ T* ll_buf(const CubeDesc& d, int comp, int l) {
    return gmem(static_cast<T*>(d.tmp)) + (int64_t)comp * d.tps + ((l & 1) ? 0 : d.tmp_off2);
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_dwt_level(const CubeDesc* __restrict__ descs,
                                                     const int* __restrict__ items, int ncubes, int level) {
    constexpr int WW = 2 * TX + 2, WH = 2 * TY + 2;
    __shared__ T win[WH][WW + 1];
    using F = Filt<T>;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int total = items[ncubes];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int h = d.lh[level - 1], w = d.lw[level - 1];
        const int h2 = d.lh[level], w2 = d.lw[level];
        const int ntx = (w2 + TX - 1) / TX, nty = (h2 + TY - 1) / TY;
        const int local = item - items[c];
        const int comp = local / (ntx * nty);
        const int rem = local - comp * ntx * nty;
        const int oy0 = (rem / ntx) * TY, ox0 = (rem % ntx) * TX;
        const T* src = level == 1 ? gmem(static_cast<const T*>(d.Z)) + (int64_t)comp * d.nz
                                  : ll_buf<T>(d, comp, level - 1);
        const int he = h + (h & 1), we = w + (w & 1);
        // the extra sample of an odd length repeats the last one, or is zero
        // for the transpose of the inverse transform
        const bool zpad = (d.mode & kModeZeroPad) != 0;
        constexpr int NV = (WH * WW + TX * TY - 1) / (TX * TY);
        T vals[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int e = threadIdx.x + TX * TY * i;
            if (e < WH * WW) {
                const int wy = e / WW, wx = e - wy * WW;
                int ey = 2 * oy0 + wy;
                ey = ey >= he ? ey - he : ey;
                ey = ey >= he ? ey % he : ey;
                const bool xy = ey == h;
                ey = xy ? h - 1 : ey;
                int ex = 2 * ox0 + wx;
                ex = ex >= we ? ex - we : ex;
                ex = ex >= we ? ex % we : ex;
                const bool xx = ex == w;
                ex = xx ? w - 1 : ex;
                const T v = src[(int64_t)ey * w + ex];
                vals[i] = zpad && (xy || xx) ? (T)0 : v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int e = threadIdx.x + TX * TY * i;
            if (e < WH * WW) {
                const int wy = e / WW, wx = e - wy * WW;
                win[wy][wx] = vals[i];
            }
        }
        __syncthreads();
        const int oy = oy0 + ty, ox = ox0 + tx;
        if (oy < h2 && ox < w2) {
            T lo[4], hi[4];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const T* x = &win[2 * ty + rr][2 * tx];
                lo[rr] = F::h0 * x[0] + F::h1 * x[1] + F::h2 * x[2] + F::h3 * x[3];
                hi[rr] = F::g0 * x[0] + F::g1 * x[1] + F::g2 * x[2] + F::g3 * x[3];
            }
            const T ll = F::h0 * lo[0] + F::h1 * lo[1] + F::h2 * lo[2] + F::h3 * lo[3];
            const T hl = F::g0 * lo[0] + F::g1 * lo[1] + F::g2 * lo[2] + F::g3 * lo[3];
            const T lh = F::h0 * hi[0] + F::h1 * hi[1] + F::h2 * hi[2] + F::h3 * hi[3];
            const T hh = F::g0 * hi[0] + F::g1 * hi[1] + F::g2 * hi[2] + F::g3 * hi[3];
            const int64_t blk = (int64_t)h2 * w2;
            const int64_t o = (int64_t)oy * w2 + ox;
            T* cf = gmem(static_cast<T*>(d.coef)) + (int64_t)comp * d.ncs + d.loff[level];
            cf[o] = lh;
            cf[blk + o] = hl;
            cf[2 * blk + o] = hh;
            T* llo = level == d.L ? gmem(static_cast<T*>(d.coef)) + (int64_t)comp * d.ncs + d.ll_off
                                  : ll_buf<T>(d, comp, level);
            llo[o] = ll;
        }
    }
}

// Level 1 of a mixed-precision solve with the Rayleigh-Ritz rotation applied
// as Z is loaded: a block takes one TY x TX output tile of every component of
// a cube.  Each window pixel's r component values are read once, rotated in
// registers (the pixel's row of Z R, summed in the order of the component
// index) and staged in LDS, one window per component; then every component's
// four subbands come from its rotated window.  Z itself stays unrotated (the
// inverse transform overwrites it), so the rotation costs no pass of its own.
template <int TX, int TY, int RM>
__global__ __launch_bounds__(TX* TY) void k_dwt_level1_rot(const CubeDesc* __restrict__ descs,
                                                          const int* __restrict__ items, int ncubes) {
    // RM: largest rank of the launch's cubes, 8 or kMaxRank.  At 8 the
    // rotation stays in registers; at 16 it is read from LDS per use.
    constexpr int WW = 2 * TX + 2, WH = 2 * TY + 2, WS = WH * (WW + 1);
    extern __shared__ float dwin[];                 // one WH x (WW + 1) window per component
    __shared__ __attribute__((aligned(16))) float R[kMaxRank][kMaxRank];   // rows 16-byte aligned
    using F = Filt<float>;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int total = items[ncubes];
    int cur = -1;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int h = d.lh[0], w = d.lw[0];
        const int h2 = d.lh[1], w2 = d.lw[1];
        const int ntx = (w2 + TX - 1) / TX;
        const int local = item - items[c];
        const int oy0 = (local / ntx) * TY, ox0 = (local % ntx) * TX;
        const int r = d.r;
        __syncthreads();                            // the previous item's windows and R are read
        if (c != cur) {
            for (int e = threadIdx.x; e < 256; e += TX * TY) R[e >> 4][e & 15] = (float)d.rrot[e];
            __syncthreads();
            cur = c;
        }
        const float* z = gmem(static_cast<const float*>(d.Z));
        const int he = h + (h & 1), we = w + (w & 1);
        for (int e = threadIdx.x; e < WH * WW; e += TX * TY) {
            const int wy = e / WW, wx = e - wy * WW;
            int ey = 2 * oy0 + wy;
            ey = ey >= he ? ey - he : ey;
            ey = ey >= he ? ey % he : ey;
            ey = ey == h ? h - 1 : ey;
            int ex = 2 * ox0 + wx;
            ex = ex >= we ? ex - we : ex;
            ex = ex >= we ? ex % we : ex;
            ex = ex == w ? w - 1 : ex;
            const int64_t off = (int64_t)ey * w + ex;
            float in[RM];
#pragma unroll
            for (int j = 0; j < RM; ++j) in[j] = j < r ? z[(int64_t)j * d.nz + off] : 0.f;
            if constexpr (RM <= 8) {
#pragma unroll
                for (int k = 0; k < RM; ++k) {
                    if (k < r) {
                        float v = 0.f;
#pragma unroll
                        for (int j = 0; j < RM; ++j)
                            if (j < r) v = fmaf(in[j], R[j][k], v);
                        dwin[k * WS + wy * (WW + 1) + wx] = v;
                    }
                }
            } else {
                // four output components at a time: one 16-byte read of R per input
#pragma unroll 1
                for (int k0 = 0; k0 < r; k0 += 4) {
                    v4f v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int j = 0; j < RM; ++j)
                        if (j < r) {
                            const v4f rk = *reinterpret_cast<const v4f*>(&R[j][k0]);
#pragma unroll
                            for (int c4 = 0; c4 < 4; ++c4) v[c4] = fmaf(in[j], rk[c4], v[c4]);
                        }
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4)
                        if (k0 + c4 < r) dwin[(k0 + c4) * WS + wy * (WW + 1) + wx] = v[c4];
                }
            }
        }
        __syncthreads();
        const int oy = oy0 + ty, ox = ox0 + tx;
        if (oy < h2 && ox < w2) {
            const int64_t blk = (int64_t)h2 * w2;
            const int64_t o = (int64_t)oy * w2 + ox;
            for (int k = 0; k < r; ++k) {
                const float* wk = dwin + k * WS;
                float lo[4], hi[4];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const float* x = wk + (2 * ty + rr) * (WW + 1) + 2 * tx;
                    lo[rr] = F::h0 * x[0] + F::h1 * x[1] + F::h2 * x[2] + F::h3 * x[3];
                    hi[rr] = F::g0 * x[0] + F::g1 * x[1] + F::g2 * x[2] + F::g3 * x[3];
                }
                const float ll = F::h0 * lo[0] + F::h1 * lo[1] + F::h2 * lo[2] + F::h3 * lo[3];
                const float hl = F::g0 * lo[0] + F::g1 * lo[1] + F::g2 * lo[2] + F::g3 * lo[3];
                const float lh = F::h0 * hi[0] + F::h1 * hi[1] + F::h2 * hi[2] + F::h3 * hi[3];
                const float hh = F::g0 * hi[0] + F::g1 * hi[1] + F::g2 * hi[2] + F::g3 * hi[3];
                float* cf = gmem(static_cast<float*>(d.coef)) + (int64_t)k * d.ncs + d.loff[1];
                cf[o] = lh;
                cf[blk + o] = hl;
                cf[2 * blk + o] = hh;
                float* llo = d.L == 1 ? gmem(static_cast<float*>(d.coef)) + (int64_t)k * d.ncs + d.ll_off
                                      : ll_buf<float>(d, k, 1);
                llo[o] = ll;
            }
        }
    }
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_idwt_level(const CubeDesc* __restrict__ descs,
                                                      const int* __restrict__ items, int ncubes, int level) {
    // window of coefficient rows s0-1 .. s0+TY-1 and columns u0-1 .. u0+TX-1, 4 subbands
    __shared__ T cw[4][TY + 1][TX + 2];
    using F = Filt<T>;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int total = items[ncubes];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int h = d.lh[level - 1], w = d.lw[level - 1];
        const int h2 = d.lh[level], w2 = d.lw[level];
        const int ntx = (w2 + TX - 1) / TX, nty = (h2 + TY - 1) / TY;
        const int local = item - items[c];
        const int comp = local / (ntx * nty);
        const int rem = local - comp * ntx * nty;
        const int s0 = (rem / ntx) * TY, u0 = (rem % ntx) * TX;
        const bool thr = (d.mode & 8) != 0;
        const T lam = thr ? (T)d.lambda[comp] : (T)0;
        const bool thr_ll = thr && level == d.L && d.scope == HYRES_SCOPE_ALL;
        const T* cf = gmem(static_cast<const T*>(d.coef)) + (int64_t)comp * d.ncs;
        const T* det = cf + d.loff[level];
        const T* llsrc = level == d.L ? cf + d.ll_off : ll_buf<T>(d, comp, level);
        const int64_t blk = (int64_t)h2 * w2;
        constexpr int NE = 4 * (TY + 1) * (TX + 1);
        constexpr int NV = (NE + TX * TY - 1) / (TX * TY);
        T vals[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int e = threadIdx.x + TX * TY * i;
            if (e < NE) {
                const int sb = e / ((TY + 1) * (TX + 1));
                const int r2 = e - sb * (TY + 1) * (TX + 1);
                const int wy = r2 / (TX + 1), wx = r2 - wy * (TX + 1);
                int cy = s0 - 1 + wy;
                cy = cy < 0 ? cy + h2 : (cy >= h2 ? cy % h2 : cy);
                int cx = u0 - 1 + wx;
                cx = cx < 0 ? cx + w2 : (cx >= w2 ? cx % w2 : cx);
                const int64_t o = (int64_t)cy * w2 + cx;
                vals[i] = sb == 0 ? llsrc[o] : det[(sb - 1) * blk + o];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int e = threadIdx.x + TX * TY * i;
            if (e < NE) {
                const int sb = e / ((TY + 1) * (TX + 1));
                const int r2 = e - sb * (TY + 1) * (TX + 1);
                const int wy = r2 / (TX + 1), wx = r2 - wy * (TX + 1);
                T v = vals[i];
                if (sb == 0 ? thr_ll : thr) v = soft(v, lam);
                cw[sb][wy][wx] = v;
            }
        }
        __syncthreads();
        const int s = s0 + ty, u = u0 + tx;
        if (s < h2 && u < w2) {
            // c[sb][dy][dx] = coefficient at (s - dy, u - dx)
            T o00 = 0, o01 = 0, o10 = 0, o11 = 0;
#pragma unroll
            for (int sb = 0; sb < 4; ++sb) {
                const T c00 = cw[sb][ty + 1][tx + 1], c01 = cw[sb][ty + 1][tx];
                const T c10 = cw[sb][ty][tx + 1], c11 = cw[sb][ty][tx];
                // sb: 0 LL (h,h), 1 LH (h along y, g along x), 2 HL (g, h), 3 HH (g, g)
                const bool gy = sb >= 2, gx = (sb & 1) != 0;
                const T fy0 = gy ? F::g0 : F::h0, fy1 = gy ? F::g1 : F::h1;
                const T fy2 = gy ? F::g2 : F::h2, fy3 = gy ? F::g3 : F::h3;
                const T fx0 = gx ? F::g0 : F::h0, fx1 = gx ? F::g1 : F::h1;
                const T fx2 = gx ? F::g2 : F::h2, fx3 = gx ? F::g3 : F::h3;
                // along x first: row dy, output column parity b
                const T r0b0 = fx0 * c00 + fx2 * c01, r0b1 = fx1 * c00 + fx3 * c01;   // dy = 0
                const T r1b0 = fx0 * c10 + fx2 * c11, r1b1 = fx1 * c10 + fx3 * c11;   // dy = 1
                o00 += fy0 * r0b0 + fy2 * r1b0;
                o01 += fy0 * r0b1 + fy2 * r1b1;
                o10 += fy1 * r0b0 + fy3 * r1b0;
                o11 += fy1 * r0b1 + fy3 * r1b1;
            }
            T* dst = level == 1 ? gmem(static_cast<T*>(d.Z)) + (int64_t)comp * d.nz
                                : ll_buf<T>(d, comp, level - 1);
            const int y0 = 2 * s, x0 = 2 * u;
            if (d.mode & kModeFold) {
                // transpose of the analysis: the extra sample of an odd length
                // is added to the last one instead of being dropped
                if (y0 + 1 == h) {
                    o00 += o10;
                    o01 += o11;
                }
                if (x0 + 1 == w) {
                    o00 += o01;
                    o10 += o11;
                }
            }
            dst[(int64_t)y0 * w + x0] = o00;
            if (x0 + 1 < w) dst[(int64_t)y0 * w + x0 + 1] = o01;
            if (y0 + 1 < h) {
                dst[(int64_t)(y0 + 1) * w + x0] = o10;
                if (x0 + 1 < w) dst[(int64_t)(y0 + 1) * w + x0 + 1] = o11;
            }
        }
    }
}

// ---------------------------------------------------------------- launchers
// Tile shapes selectable at run time (the autotuner picks among these).
#define HYRES_DWT_SHAPES(X) X(64, 4) X(32, 8) X(16, 16) X(128, 2)

template <typename T>
static hipError_t dwt_dispatch(int tx, int ty, bool inverse, const CubeDesc* descs, const int* items,
                               int ncubes, int level, int grid, hipStream_t s) {
#define HYRES_D(TX, TY)                                                                              \
    if (tx == TX && ty == TY) {                                                                      \
        if (inverse)                                                                                 \
            hipLaunchKernelGGL((k_idwt_level<T, TX, TY>), dim3(grid), dim3(TX * TY), 0, s, descs,  \
                               items, ncubes, level);                                                \
        else                                                                                         \
            hipLaunchKernelGGL((k_dwt_level<T, TX, TY>), dim3(grid), dim3(TX * TY), 0, s, descs,   \
                               items, ncubes, level);                                                \
        return hipGetLastError();                                                                    \
    }
    HYRES_DWT_SHAPES(HYRES_D)
#undef HYRES_D
    return hipErrorInvalidValue;
}

// Level 1 with the rotation (FP32): rmax is the largest rank of the launch's
// cubes (one LDS window per component).
template <int TX, int TY, int RM>
static hipError_t launch_rot_k(const CubeDesc* descs, const int* items, int ncubes, int grid, size_t bytes,
                               hipStream_t s) {
    if (bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dwt_level1_rot<TX, TY, RM>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_dwt_level1_rot<TX, TY, RM>), dim3(grid), dim3(TX * TY), bytes, s, descs, items, ncubes);
    return hipGetLastError();
}

template <int TX, int TY>
static hipError_t launch_rot_t(const CubeDesc* descs, const int* items, int ncubes, int grid, int rmax,
                               hipStream_t s) {
    const size_t bytes = (size_t)rmax * (2 * TY + 2) * (2 * TX + 3) * sizeof(float);
    if (rmax <= 8) return launch_rot_k<TX, TY, 8>(descs, items, ncubes, grid, bytes, s);
    return launch_rot_k<TX, TY, kMaxRank>(descs, items, ncubes, grid, bytes, s);
}

hipError_t launch_dwt_level1_rot(int tx, int ty, const CubeDesc* descs, const int* items, int ncubes, int grid,
                                 int rmax, hipStream_t s) {
#define HYRES_R(TX, TY) \
    if (tx == TX && ty == TY) return launch_rot_t<TX, TY>(descs, items, ncubes, grid, rmax, s);
    HYRES_DWT_SHAPES(HYRES_R)
#undef HYRES_R
    return hipErrorInvalidValue;
}

hipError_t launch_dwt_level(int dtype, int tx, int ty, bool inverse, const CubeDesc* descs, const int* items,
                            int ncubes, int level, int grid, hipStream_t s) {
    if (dtype == HYRES_F64) return dwt_dispatch<double>(tx, ty, inverse, descs, items, ncubes, level, grid, s);
    return dwt_dispatch<float>(tx, ty, inverse, descs, items, ncubes, level, grid, s);
}

}  // namespace hyres
