// Adjoint of the HyRes solve with the thresholds held as inputs, and the
// derivative of the SURE risk with respect to a threshold.
//
// Forward (per cube, n pixels, p bands, rank r):
//   G = Y^T Y,  sigma_j = (n [G^-1]_jj)^(-1/2),  C = D^-1 G D^-1  (D = diag sigma),
//   C u_k = lambda_k u_k (top r),  P = D^-1 V,  Z = Y P,  B = W Z (transform per component),
//   Bh = soft(B, lambda),  Zh = W^+ Bh (inverse transform),  Q = V^T D,  X = Zh Q.
// Reverse, given dX:
//   dZh = dX Q^T,  dQ = Zh^T dX                              (k_adj_apply, k_adj_xprod)
//   dBh = (W^+)^T dZh        (analysis with zero extension)  (transform kernels)
//   dB = dBh 1[|B| > lambda],  dlambda_k = -sum dBh sign(B) 1[|B| > lambda]  (k_adj_thresh)
//   dZ = W^T dB              (synthesis, extra sample folded back)  (transform kernels)
//   dP = Y^T dZ,  dY  = dZ P^T + 2 Y dG                        (k_adj_xprod, k_adj_dy)
//   dV = D^-1 dP + D dQ^T,  dsigma from P, Q and C
//   eigenvectors: dC = sum_k sym(w_k u_k^T), w_k = sum_{i != k} u_i u_i^T dV_k / (lambda_k - lambda_i):
//     explicit inside the top-r subspace, outside it from the positive definite
//     (lambda_k I - C + U Lambda U^T) y = (I - U U^T) dV_k   (k_adj_sweep, with G^-1)
//   dG = D^-1 dC D^-1 + G^-1 diag(n sigma_j^3 dsigma_j / 2) G^-1      (k_adj_dc, k_adj_dg)
// Small dense algebra runs in FP64 in one workgroup per system; the pixel
// loops run in the element type of the cube with FP64 accumulation where
// they reduce over pixels.
#include "tile_stage.hpp"

namespace hyres {



constexpr int kAdjChunk = 16384;   // coefficients per threshold-adjoint block
typedef double v4d __attribute__((ext_vector_type(4)));

int adj_chunk() { return kAdjChunk; }

template <typename T>
__device__ __forceinline__ const T* adj_pix(const void* base, int64_t q, int W, int64_t pitch, int64_t rpitch) {
    const int64_t y = q / W, x = q - y * W;
    return static_cast<const T*>(base) + y * rpitch + x * pitch;
}

// FP64 cubes: dZh[k][q] = sum_b dX[q][b] Q[k][b], one pixel per thread, Q staged in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_apply(AdjDesc a) {
    __shared__ double sq[kMaxRank * kMaxBands];
    const int p = a.p, r = a.r;
    for (int i = threadIdx.x; i < r * p; i += blockDim.x) sq[i] = a.Q64[i];
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n) return;
    const T* x = adj_pix<T>(a.dX, q, a.W, a.dxp, a.dxrp);
    double acc[kMaxRank];
#pragma unroll
    for (int k = 0; k < kMaxRank; ++k) acc[k] = 0.0;
    for (int b = 0; b < p; ++b) {
        const double v = (double)x[b];
#pragma unroll
        for (int k = 0; k < kMaxRank; ++k)
            if (k < r) acc[k] = fma(v, sq[k * p + b], acc[k]);
    }
    T* out = static_cast<T*>(a.A);
#pragma unroll
    for (int k = 0; k < kMaxRank; ++k)
        if (k < r) out[(int64_t)k * a.nz + q] = (T)acc[k];
}

// FP32 cubes: dZh = dX Q^T on the matrix cores, as the projection computes
// Z = Y P: a 64-pixel tile of dX per block staged through LDS, a 16-pixel x
// 16-component output tile per wave, Q^T as FP32 B fragments in registers
// (v_mfma_f32_16x16x4f32, four accumulator chains).  One tile per block, so
// that few registers stay live and several blocks share a compute unit.
template <int NT, int LM>
__global__ __launch_bounds__(256, 2) void k_adj_apply_f32(AdjDesc a, CubeView dx) {
    constexpr int LDW = proj_ldw<NT>();
    __shared__ __attribute__((aligned(16))) float tile[kPixTile * LDW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, row = lane >> 4;
    const int p = a.p, r = a.r;
    const int64_t q0 = (int64_t)blockIdx.x * kPixTile;
    {
        v4f r4[proj_nv4<NT>()];
        int zlo = 16 * NT;
        proj_fetch<NT, LM>(dx, q0, r4);
        proj_stage<NT, LM>(tile, dx, zlo, r4);
    }
    float bf[4 * NT];
#pragma unroll
    for (int s = 0; s < 4 * NT; ++s) {
        const int b = 4 * s + row;
        bf[s] = (b < p && col < r) ? (float)a.Q64[(int64_t)col * p + b] : 0.f;
    }
    __syncthreads();
    v4f ac[4] = {};
    const float* arow = tile + (16 * wave + col) * LDW + row;
#pragma unroll
    for (int s = 0; s < 4 * NT; ++s) {
        ac[s & 3] = mfma4(arow[4 * s], bf[s], ac[s & 3]);
        if ((s & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    const v4f acc = (ac[0] + ac[1]) + (ac[2] + ac[3]);
    // lane holds component col of pixels q0 + 16 wave + 4 row + i (the planes
    // are padded to whole tiles; the tile rows past the cube are zero)
    if (col < r)
        *reinterpret_cast<v4f*>(static_cast<float*>(a.A) + (int64_t)col * a.nz + q0 + 16 * wave + 4 * row) = acc;
}

// FP32 cubes: part[slot][k][b] = sum over the slot's pixels of
// planes[k][q] * cube[q][b] with the cube staged through LDS as 64-pixel tiles
// (coalesced loads, the next tile prefetched into registers) on the matrix
// cores (v_mfma_f32_16x16x4f32: FP32 products summed in FP32 over one tile,
// then added in FP64).  A wave owns every fourth 16-band tile of the result
// (rotated with the block, so that the waves with one tile more fall on
// different SIMDs) over all 64 pixels of a tile: step (m, s) takes pixel
// 16 m + 4 (lane / 16) + s, so a lane's plane values of one m are one 16-byte
// load and the cube values one LDS read per band tile.  A block runs the
// tiles slot, slot + slots, ...; no sum across waves is needed.
template <int NT, int LM>
__global__ __launch_bounds__(256, LM == kScalar ? 1 : 2) void k_adj_xprod_f32(AdjDesc a, const float* __restrict__ planes,
                                                                           CubeView cv) {
    constexpr int LDW = proj_ldw<NT>();
    constexpr int NW = (NT + 3) / 4;               // band tiles per wave, at most
    __shared__ __attribute__((aligned(16))) float tile[kPixTile * LDW];
    const int p = a.p, r = a.r, E = r * p;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kk = lane >> 4, jj = lane & 15;
    const int rot = (wave + blockIdx.x) & 3;       // this wave's band tiles: rot, rot + 4, ...
    const int64_t ntiles = (a.n + kPixTile - 1) / kPixTile;
    double accd[NW][4];
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int v = 0; v < 4; ++v) accd[w][v] = 0.0;
    v4f r4[proj_nv4<NT>()];
    int zlo = 16 * NT;
    int64_t t = blockIdx.x;
    if (t < ntiles) proj_fetch<NT, LM>(cv, t * kPixTile, r4);
    for (; t < ntiles; t += gridDim.x) {
        const int64_t q0 = t * kPixTile;
        v4f bv[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            bv[m] = v4f{0.f, 0.f, 0.f, 0.f};
            if (jj < r) bv[m] = *reinterpret_cast<const v4f*>(planes + (int64_t)jj * a.nz + q0 + 16 * m + 4 * kk);
        }
        __syncthreads();
        proj_stage<NT, LM>(tile, cv, zlo, r4);
        __syncthreads();
        if (t + gridDim.x < ntiles) proj_fetch<NT, LM>(cv, (t + gridDim.x) * kPixTile, r4);
        v4f acc[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) acc[w] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int64_t qb = q0 + 16 * m + 4 * kk;
            const float* arow = tile + (16 * m + 4 * kk) * LDW + 16 * rot + jj;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                // pixels past the cube: their tile rows are zero, their plane values unknown
                const float b = qb + s < a.n ? bv[m][s] : 0.f;
#pragma unroll
                for (int w = 0; w < NW; ++w)
                    if (rot + 4 * w < NT) acc[w] = mfma4(arow[s * LDW + 64 * w], b, acc[w]);
            }
        }
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int v = 0; v < 4; ++v) accd[w][v] += (double)acc[w][v];
    }
    // lane holds band 16 u + 4 kk + v and component jj of band tile u = rot + 4 w
    if (jj < r) {
        double* out = a.part + (int64_t)blockIdx.x * E + (int64_t)jj * p;
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int band = 16 * (rot + 4 * w) + 4 * kk + v;
                if (rot + 4 * w < NT && band < p) out[band] = accd[w][v];
            }
    }
}

// FP64 cubes: part[slot][k][b] = sum over the slot's pixels of planes[k][q] *
// cube[q][b], on the FP64 matrix cores (v_mfma_f64_16x16x4f64): D (16 bands x 16
// components) += A (16 bands x 4 pixels) B (4 pixels x 16 components), one
// accumulator per 16-band tile.  A lane takes pixel lane / 16 of the step and
// band / component lane % 16 of the tile; D holds band lane / 16 + 4 v and
// component lane % 16 in its element v (the FP64 layout, unlike the FP32
// one's 4 (lane / 16) + v).  Each wave runs a quarter of the
// slot's pixels; the waves' sums are added in wave order through LDS.
template <typename T, int NT>
__global__ __launch_bounds__(256) void k_adj_xprod(AdjDesc a, const void* planes, const void* cube, int64_t cp,
                                                   int64_t crp) {
    __shared__ double red[kMaxRank][NT * 16];
    const int p = a.p, r = a.r, E = r * p;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kk = lane >> 4, jj = lane & 15;
    const int slot = blockIdx.x;
    int64_t per = (a.n + a.slots - 1) / a.slots;
    per = (per + 15) / 16 * 16;
    const int64_t q0 = (int64_t)slot * per;
    const int64_t q1 = q0 + per < a.n ? q0 + per : a.n;
    const int64_t quarter = per / 4;
    const int64_t w0 = q0 + wave * quarter;
    const int64_t w1 = w0 + quarter < q1 ? w0 + quarter : q1;
    const T* pl = static_cast<const T*>(planes) + (int64_t)jj * a.nz;
    v4d acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    // the lane's pixel, tracked as (y, x) while it advances by 4
    int64_t q = w0 + kk;
    int64_t y = q / a.W, x = q - y * a.W;
    for (int64_t qs = w0; qs < w1; qs += 4) {
        const bool in = q < w1;
        const double bv = (in && jj < r) ? (double)pl[q] : 0.0;
        const T* row = static_cast<const T*>(cube) + y * crp + x * cp;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int band = 16 * t + jj;
            const double av = (in && band < p) ? (double)row[band] : 0.0;
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
        q += 4;
        x += 4;
        while (x >= a.W) {
            x -= a.W;
            ++y;
        }
    }
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int band = 16 * t + kk + 4 * v;
                    if (jj < r) red[jj][band] = w == 0 ? acc[t][v] : red[jj][band] + acc[t][v];
                }
        }
        __syncthreads();
    }
    for (int e = tid; e < E; e += 256) {
        const int k = e / p, b = e - k * p;
        a.part[(int64_t)slot * E + e] = red[k][b];
    }
}

// out[e] = sum over slots of part[slot][e]: one wave per entry, each lane
// summing the slots congruent to it in slot order, then the wave's fixed tree.
__global__ __launch_bounds__(64) void k_adj_reduce(const double* __restrict__ part, int slots, int E,
                                                   double* __restrict__ out) {
    const int e = blockIdx.x, lane = threadIdx.x;
    double s = 0.0;
#pragma unroll 4
    for (int i = lane; i < slots; i += 64) s += part[(int64_t)i * E + e];
    s = wave_sum(s);
    if (lane == 0) out[e] = s;
}

template <typename T>
__device__ __forceinline__ double block_sum256(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// Threshold adjoint in place on dB; per-block partial of dlambda.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_thresh(AdjDesc a) {
    __shared__ double red[4];
    const int comp = blockIdx.y, chunk = blockIdx.x;
    const T* bf = static_cast<const T*>(a.B) + (int64_t)comp * a.ncs;
    T* g = static_cast<T*>(a.dB) + (int64_t)comp * a.ncs;
    const T lam = (T)a.lambda[comp];
    const int64_t lim = a.scope == HYRES_SCOPE_DETAIL ? a.ll_off : a.nc;
    const int64_t e0 = (int64_t)chunk * kAdjChunk;
    const int64_t e1 = e0 + kAdjChunk < lim ? e0 + kAdjChunk : lim;
    double s = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const T b = bf[e];
        const T v = g[e];
        const bool m = (b < (T)0 ? -b : b) > lam;
        if (m) s -= (double)(b < (T)0 ? -v : v);
        g[e] = m ? v : (T)0;
    }
    s = block_sum256<T>(s, red);
    if (threadIdx.x == 0) a.lpart[(int64_t)comp * a.nchunk + chunk] = s;
}

// #{|b| > lambda} per block (the SURE derivative is 2 lambda times the count).
template <typename T>
__global__ __launch_bounds__(256) void k_sure_count(const T* __restrict__ coef, int64_t stride, int64_t N,
                                                    const double* __restrict__ lambda, int nchunk,
                                                    double* __restrict__ part) {
    __shared__ double red[4];
    const int comp = blockIdx.y, chunk = blockIdx.x;
    const T* bf = coef + (int64_t)comp * stride;
    const T lam = (T)lambda[comp];
    const int64_t e0 = (int64_t)chunk * kAdjChunk;
    const int64_t e1 = e0 + kAdjChunk < N ? e0 + kAdjChunk : N;
    double s = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const T b = bf[e];
        s += (b < (T)0 ? -b : b) > lam ? 1.0 : 0.0;
    }
    s = block_sum256<T>(s, red);
    if (threadIdx.x == 0) part[(int64_t)comp * nchunk + chunk] = s;
}

// out[k] = scale_k * sum over chunks of part[k][chunk] (scale_k = 2 lambda_k or 1).
__global__ void k_chunk_reduce(const double* __restrict__ part, int nchunk, int r, const double* __restrict__ lambda,
                               int twice_lambda, double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r) return;
    double s = 0.0;
    for (int i = 0; i < nchunk; ++i) s += part[(int64_t)k * nchunk + i];
    out[k] = twice_lambda ? 2.0 * lambda[k] * s : s;
}

// dC = sum_k sym(w_k v_k^T) and the noise term gsc_j = n sigma_j^3 dsigma_j / 2
// (one workgroup; w_k from the eigen-adjoint sweeps).
__global__ __launch_bounds__(1024) void k_adj_dc(AdjDesc a) {
    __shared__ double sw[kMaxRank][kMaxBands], sv[kMaxRank][kMaxBands], ssig[kMaxBands];
    const int p = a.p, r = a.r, tid = threadIdx.x;
    const double n = (double)a.n;
    for (int e = tid; e < r * p; e += blockDim.x) {
        sw[e / p][e % p] = a.Wsol[e];
        sv[e / p][e % p] = a.V[e];
    }
    for (int j = tid; j < p; j += blockDim.x) ssig[j] = a.sigma[j];
    __syncthreads();
    for (int e = tid; e < p * p; e += blockDim.x) {
        const int i = e / p, j = e - i * p;
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += sw[k][i] * sv[k][j] + sw[k][j] * sv[k][i];
        a.dC[e] = 0.5 * s;
    }
    __syncthreads();
    for (int j = tid; j < p; j += blockDim.x) {
        const double sj = ssig[j];
        double ds = 0.0;
        for (int k = 0; k < r; ++k) {
            const double v = sv[k][j];
            ds += -a.dPt[(int64_t)k * p + j] * v / (sj * sj) + a.dQ[(int64_t)k * p + j] * v;
        }
        double t = 0.0;
#pragma unroll 8
        for (int i = 0; i < p; ++i) t = fma(a.dC[(int64_t)i * p + j], a.G[(int64_t)i * p + j] / (ssig[i] * sj), t);
        ds -= 2.0 * t / sj;
        a.gsc[j] = 0.5 * n * sj * sj * sj * ds;
    }
}

// dG2 = 2 (D^-1 dC D^-1 + G^-1 diag(gsc) G^-1), one row per workgroup.
__global__ __launch_bounds__(256) void k_adj_dg(AdjDesc a) {
    __shared__ double srow[kMaxBands];
    const int p = a.p, i = blockIdx.x, tid = threadIdx.x;
    for (int l = tid; l < p; l += blockDim.x) srow[l] = a.Ginv[(int64_t)i * p + l] * a.gsc[l];
    __syncthreads();
    const double si = a.sigma[i];
    for (int j = tid; j < p; j += blockDim.x) {
        double s = a.dC[(int64_t)i * p + j] / (si * a.sigma[j]);
#pragma unroll 8
        for (int l = 0; l < p; ++l) s = fma(srow[l], a.Ginv[(int64_t)l * p + j], s);
        a.dG2[(int64_t)i * p + j] = 2.0 * s;
    }
}

// FP64 cubes: dY[q][b] = sum_k dZ[k][q] P[b][k] + sum_j Y[q][j] dG2[j][b]; a
// block owns 32 pixels x 32 bands.
constexpr int kDyPix = 32, kDyCol = 32;
template <typename T>
__global__ __launch_bounds__(256) void k_adj_dy(AdjDesc a) {
    __shared__ T yt[kDyPix][kMaxBands + 1];
    __shared__ T gt[kMaxBands][kDyCol + 1];
    __shared__ T zt[kMaxRank][kDyPix];
    __shared__ T pt[kDyCol][kMaxRank + 1];
    const int p = a.p, r = a.r;
    const int64_t q0 = (int64_t)blockIdx.x * kDyPix;
    const int b0 = blockIdx.y * kDyCol;
    for (int e = threadIdx.x; e < kDyPix * p; e += 256) {
        const int k = e / p, j = e - k * p;
        const int64_t q = q0 + k;
        yt[k][j] = q < a.n ? adj_pix<T>(a.Y, q, a.W, a.pitch, a.row_pitch)[j] : (T)0;
    }
    for (int e = threadIdx.x; e < p * kDyCol; e += 256) {
        const int j = e / kDyCol, c = e - j * kDyCol;
        gt[j][c] = b0 + c < p ? (T)a.dG2[(int64_t)j * p + b0 + c] : (T)0;
    }
    const T* zp = static_cast<const T*>(a.A);
    for (int e = threadIdx.x; e < r * kDyPix; e += 256) {
        const int k = e / kDyPix, i = e - k * kDyPix;
        const int64_t q = q0 + i;
        zt[k][i] = q < a.n ? zp[(int64_t)k * a.nz + q] : (T)0;
    }
    for (int e = threadIdx.x; e < kDyCol * r; e += 256) {
        const int c = e / r, k = e - c * r;
        pt[c][k] = b0 + c < p ? (T)a.P64[(int64_t)(b0 + c) * r + k] : (T)0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kDyPix * kDyCol; e += 256) {
        const int i = e / kDyCol, c = e - i * kDyCol;
        const int64_t q = q0 + i;
        if (q >= a.n || b0 + c >= p) continue;
        T s = (T)0;
        for (int k = 0; k < r; ++k) s = fma(zt[k][i], pt[c][k], s);
        for (int j = 0; j < p; ++j) s = fma(yt[i][j], gt[j][c], s);
        const int64_t y = q / a.W, x = q - y * a.W;
        static_cast<T*>(a.dY)[y * a.dyrp + x * a.dyp + b0 + c] = s;
    }
}

// FP32 cubes: dY = Y dG2 + dZ P^T on the matrix cores.  A block owns one
// 64-pixel tile of Y, staged through LDS, and four 16-band column tiles of dY
// (one per wave; blockIdx.y picks the group).  Each wave keeps its column of
// dG2 and of P^T as FP32 B fragments in registers and computes 16 pixels x
// 16 bands per accumulator, four pixel groups (v_mfma_f32_16x16x4f32, four
// accumulator chains).  One tile per block: the loads of the tile, the
// fragments and dZ are all in flight at once, and other blocks of the compute
// unit cover their latency.
template <int NT, int LM>
__global__ __launch_bounds__(256, 2) void k_adj_dy_f32(AdjDesc a, CubeView yv) {
    constexpr int LDW = proj_ldw<NT>();
    __shared__ __attribute__((aligned(16))) float tile[kPixTile * LDW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, row = lane >> 4;
    const int p = a.p, r = a.r;
    const int ct = 4 * blockIdx.y + wave;          // column tile of this wave
    const int b = 16 * ct + col;                   // its output band
    const int64_t q0 = (int64_t)blockIdx.x * kPixTile;
    {
        v4f r4[proj_nv4<NT>()];
        int zlo = 16 * NT;
        proj_fetch<NT, LM>(yv, q0, r4);
        proj_stage<NT, LM>(tile, yv, zlo, r4);
    }
    float bg[4 * NT], bp[4];
#pragma unroll
    for (int s = 0; s < 4 * NT; ++s) {
        const int j = 4 * s + row;
        bg[s] = (j < p && b < p) ? (float)a.dG2[(int64_t)j * p + b] : 0.f;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + row;
        bp[s] = (k < r && b < p) ? (float)a.P64[(int64_t)b * r + k] : 0.f;
    }
    // A fragments of dZ P^T: dZ[comp 4 s + row][pixel q0 + 16 g + col] (the
    // planes are padded to whole tiles)
    const int R4 = (r + 3) >> 2;
    const float* zp = static_cast<const float*>(a.A) + q0 + col;
    float az[4][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = 4 * s + row;
            az[g][s] = (s < R4 && k < r) ? zp[(int64_t)k * a.nz + 16 * g] : 0.f;
        }
    __syncthreads();
    if (16 * ct >= p) return;                      // a wave past the last band tile
    // pixel indices in 32 bits (n <= 2^31, so q + 63 < 2^32)
    const unsigned n = (unsigned)a.n, Wd = (unsigned)a.W;
    float* dy = static_cast<float*>(a.dY);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        v4f ac[4] = {};
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (s < R4) ac[s] = mfma4(az[g][s], bp[s], ac[s]);
        const float* arow = tile + (16 * g + col) * LDW + row;
#pragma unroll
        for (int s = 0; s < 4 * NT; ++s) {
            ac[s & 3] = mfma4(arow[4 * s], bg[s], ac[s & 3]);
            if ((s & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        const v4f acc = (ac[0] + ac[1]) + (ac[2] + ac[3]);
        // lane holds band b of pixels q0 + 16 g + 4 row + i
        if (b < p) {
            const unsigned qa = (unsigned)q0 + 16 * g + 4 * row;
            unsigned y = qa / Wd, x = qa - y * Wd;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (qa + i < n) dy[(int64_t)y * a.dyrp + (int64_t)x * a.dyp + b] = acc[i];
                if (++x == Wd) {
                    x = 0;
                    ++y;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_xprod_t(const AdjDesc& a, const void* planes, const void* cube, int64_t cp, int64_t crp,
                          hipStream_t s) {
    const int nt = (a.p + 15) / 16;
#define HYRES_X(N) \
    case N: hipLaunchKernelGGL((k_adj_xprod<T, N>), dim3(a.slots), dim3(256), 0, s, a, planes, cube, cp, crp); break;
    switch (nt) {
        HYRES_X(1) HYRES_X(2) HYRES_X(3) HYRES_X(4) HYRES_X(5) HYRES_X(6) HYRES_X(7)
        HYRES_X(8) HYRES_X(9) HYRES_X(10) HYRES_X(11) HYRES_X(12) HYRES_X(13) HYRES_X(14)
        default: return hipErrorInvalidValue;
    }
#undef HYRES_X
    return hipGetLastError();
}

// FP32 tile kernels specialised on the cube's load path (one path per kernel
// keeps the staging registers low).
#define LAUNCH_LM(K, N, view, grid, ...)                                                   \
    do {                                                                                   \
        if ((view).vec4) hipLaunchKernelGGL((K<N, kVec>), grid, dim3(256), 0, s, __VA_ARGS__); \
        else if ((view).dense) hipLaunchKernelGGL((K<N, kDense>), grid, dim3(256), 0, s, __VA_ARGS__); \
        else hipLaunchKernelGGL((K<N, kScalar>), grid, dim3(256), 0, s, __VA_ARGS__);   \
    } while (0)
#define HYRES_NT_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

hipError_t launch_xprod(int dtype, const AdjDesc& a, const void* planes, const void* cube, int64_t cp, int64_t crp,
                        hipStream_t s) {
    if (dtype == HYRES_F64) return launch_xprod_t<double>(a, planes, cube, cp, crp, s);
    const CubeView cv = cube_view(cube, a.W, a.p, a.n, cp, crp, HYRES_F32);
    const float* pl = static_cast<const float*>(planes);
    switch ((a.p + 15) / 16) {
#define HYRES_X(N) \
    case N: LAUNCH_LM(k_adj_xprod_f32, N, cv, dim3(a.slots), a, pl, cv); break;
        HYRES_NT_CASES(HYRES_X)
#undef HYRES_X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


hipError_t launch_adjoint_pre(const AdjDesc& a, int dtype, hipStream_t s) {
    // dZh and dQ
    if (dtype == HYRES_F64) {
        const unsigned gb = (unsigned)((a.n + 255) / 256);
        hipLaunchKernelGGL(k_adj_apply<double>, dim3(gb), dim3(256), 0, s, a);
    } else {
        const CubeView dx = cube_view(a.dX, a.W, a.p, a.n, a.dxp, a.dxrp, HYRES_F32);
        const unsigned g = (unsigned)((a.n + kPixTile - 1) / kPixTile);
        switch ((a.p + 15) / 16) {
#define HYRES_X(N) \
    case N: LAUNCH_LM(k_adj_apply_f32, N, dx, dim3(g), a, dx); break;
            HYRES_NT_CASES(HYRES_X)
#undef HYRES_X
            default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = launch_xprod(dtype, a, a.Zh, a.dX, a.dxp, a.dxrp, s);
    if (e != hipSuccess) return e;
    const int E = a.r * a.p;
    hipLaunchKernelGGL(k_adj_reduce, dim3(E), dim3(64), 0, s, a.part, a.slots, E, a.dQ);
    return hipGetLastError();
}

hipError_t launch_adjoint_thresh(const AdjDesc& a, int dtype, hipStream_t s) {
    const dim3 grid(a.nchunk, a.r);
    if (dtype == HYRES_F64) hipLaunchKernelGGL(k_adj_thresh<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_adj_thresh<float>, grid, dim3(256), 0, s, a);
    if (a.dlambda)
        hipLaunchKernelGGL(k_chunk_reduce, dim3(1), dim3(64), 0, s, a.lpart, a.nchunk, a.r, a.lambda, 0, a.dlambda);
    return hipGetLastError();
}

hipError_t launch_adjoint_post(const AdjDesc& a, int dtype, hipStream_t s) {
    // dP^T, the small FP64 algebra, then dY
    hipError_t e = launch_xprod(dtype, a, a.A, a.Y, a.pitch, a.row_pitch, s);
    if (e != hipSuccess) return e;
    const int E = a.r * a.p;
    hipLaunchKernelGGL(k_adj_reduce, dim3(E), dim3(64), 0, s, a.part, a.slots, E, a.dPt);
    e = launch_adj_sweep(a, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_dc, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_adj_dg, dim3(a.p), dim3(256), 0, s, a);
    if (dtype == HYRES_F64) {
        const dim3 grid((unsigned)((a.n + kDyPix - 1) / kDyPix), (unsigned)((a.p + kDyCol - 1) / kDyCol));
        hipLaunchKernelGGL(k_adj_dy<double>, grid, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const CubeView yv = cube_view(a.Y, a.W, a.p, a.n, a.pitch, a.row_pitch, HYRES_F32);
    const int nt = (a.p + 15) / 16, groups = (nt + 3) / 4;
    const dim3 grid((unsigned)((a.n + kPixTile - 1) / kPixTile), (unsigned)groups);
    switch (nt) {
#define HYRES_X(N) \
    case N: LAUNCH_LM(k_adj_dy_f32, N, yv, grid, a, yv); break;
        HYRES_NT_CASES(HYRES_X)
#undef HYRES_X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// out[k][b] = sum over the pixels of planes[k][q] cube[q][b] (r x p, FP64 sums).
hipError_t launch_planes_cube(int dtype, const AdjDesc& a, const void* planes, const void* cube, int64_t cp,
                              int64_t crp, double* out, hipStream_t s) {
    hipError_t e = launch_xprod(dtype, a, planes, cube, cp, crp, s);
    if (e != hipSuccess) return e;
    const int E = a.r * a.p;
    hipLaunchKernelGGL(k_adj_reduce, dim3(E), dim3(64), 0, s, a.part, a.slots, E, out);
    return hipGetLastError();
}

hipError_t launch_sure_grad(int dtype, const void* coef, int64_t stride, int64_t N, int batch, const double* lambda,
                            double* part, int nchunk, double* out, hipStream_t s) {
    const dim3 grid(nchunk, batch);
    if (dtype == HYRES_F64)
        hipLaunchKernelGGL(k_sure_count<double>, grid, dim3(256), 0, s, static_cast<const double*>(coef), stride, N,
                           lambda, nchunk, part);
    else
        hipLaunchKernelGGL(k_sure_count<float>, grid, dim3(256), 0, s, static_cast<const float*>(coef), stride, N,
                           lambda, nchunk, part);
    hipLaunchKernelGGL(k_chunk_reduce, dim3((batch + 63) / 64), dim3(64), 0, s, part, nchunk, batch, lambda, 1, out);
    return hipGetLastError();
}

}  // namespace hyres
