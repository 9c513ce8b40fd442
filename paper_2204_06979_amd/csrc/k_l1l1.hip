// HyMiNoR's sparse-noise stage (Section 2.1: HyRes first, then an l1-l1
// problem solved by split Bregman): per pixel spectrum h (p bands),
//     x = argmin ||h - x||_1 + lam ||D x||_1,   (D x)_i = x_{i+1} - x_i,
// by split Bregman with s = h - x, u = D x, penalties mu1, mu2, everything
// starting at zero, K sweeps; the x step solves (mu1 I + mu2 D^T D) x = rhs
// exactly.
//
// One pixel is owned by S = 1, 2 or 4 consecutive lanes, each holding a
// segment of M bands of x, b1 and b2 in registers (indices resolved at compile
// time) and its part of h in LDS.  The shrinkage and Bregman updates of sweep
// k are fused into the forward elimination of sweep k+1 (they only need x of
// sweep k), with the clipped Bregman variables as the state:
//   t = h - x + b1,  b1' = clip(t, 1/mu1),  h - s + b1' = h - t + 2 b1'
//   v = x_{i+1} - x_i + b2_i,  b2_i' = clip(v, lam/mu2),  u_i - b2_i' = v - 2 b2_i'
// The tridiagonal solve of a pixel runs as S local Thomas solves of the
// diagonal blocks of M, after which the S - 1 couplings are restored exactly:
// the block solution y_s is corrected by the spikes of its block (the block's
// solution for the coupling entry -mu2 at its last or first row) times the
// interface values, which come from the 2(S-1) x 2(S-1) interface system (its
// inverse is formed once per block).  Segments at the boundaries exchange the
// x of the band across the boundary before each sweep; the lane after a
// boundary recomputes the boundary's Bregman update from the same operands as
// the lane before it, so both hold the same value.
#include <type_traits>

#include "hyres_internal.hpp"

namespace hyres {

namespace {

template <typename T>
__device__ __forceinline__ T clip(T v, T t);
template <>
__device__ __forceinline__ float clip<float>(float v, float t) {
    return __builtin_amdgcn_fmed3f(v, -t, t);
}
template <>
__device__ __forceinline__ double clip<double>(double v, double t) {
    return fmin(fmax(v, -t), t);
}

// Zero that the compiler cannot see through: table and h reads indexed with it
// stay inside the sweep loop instead of being hoisted into registers (which
// would double the registers a lane needs).
__device__ __forceinline__ int opaque_zero() {
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

}  // namespace

template <typename T, int M, int S>
__global__ __launch_bounds__(64) void k_l1l1(L1Args a, int64_t groups) {
    constexpr int PPB = 64 / S;                 // pixels per block
    constexpr int NI = 2 * (S - 1);             // interface unknowns
    __shared__ T s_h[M][64];                    // h, band-major (lane-private columns)
    __shared__ T s_inv[S][M], s_f[S][M];        // block Thomas: 1 / beta_i and -e / beta_i = mu2 / beta_i
    __shared__ T s_wr[S][M], s_wl[S][M];        // spikes of the last / first row coupling
    __shared__ T s_r[NI > 0 ? NI : 1][NI > 0 ? NI : 1];   // inverse of the interface system
    __shared__ double s_tip[S][2][2];           // spike values at the ends of each block [s][wr/wl][first/last]
    __shared__ double s_beta[S][M], s_w[S][M];  // FP64 pivots and a spike being formed

    const int lane = threadIdx.x;
    const int seg = lane % S;
    const int p = a.p;
    const int lenS = [&] {
        const int l = p - seg * M;
        return l < 0 ? 0 : (l > M ? M : l);
    }();
    const double mu1 = a.mu1, mu2 = a.mu2;

    // ---------------------------------------------------------- block tables
    // Factors of each diagonal block of M = mu1 I + mu2 D^T D and its spikes
    // (the block's solution for -mu2 at its last / first row), in FP64, one
    // lane per block.
    if (lane < S) {
        const int s = lane;
        const int g0 = s * M;
        const int L = p - g0 < M ? p - g0 : M;
        const double e = -mu2;
        for (int i = 0; i < L; ++i) {
            const int g = g0 + i;
            const double dg = p == 1 ? mu1 : (g == 0 || g == p - 1) ? mu1 + mu2 : mu1 + 2.0 * mu2;
            s_beta[s][i] = i == 0 ? dg : dg - e * e / s_beta[s][i - 1];
        }
        for (int i = 0; i < M; ++i) {
            s_inv[s][i] = i < L ? (T)(1.0 / s_beta[s][i]) : (T)0;
            // the last row of a block does not couple forward inside the block
            s_f[s][i] = i < L - 1 ? (T)(mu2 / s_beta[s][i]) : (T)0;
            s_wr[s][i] = (T)0;
            s_wl[s][i] = (T)0;
        }
        auto unit = [&](int row) {
            double z = 0.0;
            for (int i = 0; i < L; ++i) {
                z = ((i == row ? e : 0.0) - (i > 0 ? e * z : 0.0)) / s_beta[s][i];
                s_w[s][i] = z;
            }
            for (int i = L - 2; i >= 0; --i) s_w[s][i] -= e / s_beta[s][i] * s_w[s][i + 1];
        };
        for (int k = 0; k < 4; ++k) s_tip[s][k >> 1][k & 1] = 0.0;
        if (s < S - 1) {
            unit(L - 1);
            for (int i = 0; i < L; ++i) s_wr[s][i] = (T)s_w[s][i];
            s_tip[s][0][0] = s_w[s][0];
            s_tip[s][0][1] = s_w[s][L - 1];
        }
        if (s > 0) {
            unit(0);
            for (int i = 0; i < L; ++i) s_wl[s][i] = (T)s_w[s][i];
            s_tip[s][1][0] = s_w[s][0];
            s_tip[s][1][1] = s_w[s][L - 1];
        }
    }
    __syncthreads();
    if constexpr (NI > 0) {
        if (lane == 0) {
            // unknowns u[2j] = x at the last band of block j, u[2j+1] = x at the
            // first band of block j+1; K u = tips of the block solutions
            double K[NI][2 * NI];
            for (int i = 0; i < NI; ++i)
                for (int j = 0; j < 2 * NI; ++j) K[i][j] = (j == i || j == NI + i) ? 1.0 : 0.0;
            for (int j = 0; j < S - 1; ++j) {
                K[2 * j][2 * j + 1] += s_tip[j][0][1];
                if (j > 0) K[2 * j][2 * (j - 1)] += s_tip[j][1][1];
                if (j + 1 < S - 1) K[2 * j + 1][2 * (j + 1) + 1] += s_tip[j + 1][0][0];
                K[2 * j + 1][2 * j] += s_tip[j + 1][1][0];
            }
            // Gauss-Jordan on [K | I]; K is diagonally dominant for mu1 > 0
            for (int c = 0; c < NI; ++c) {
                const double inv = 1.0 / K[c][c];
                for (int j = 0; j < 2 * NI; ++j) K[c][j] *= inv;
                for (int i = 0; i < NI; ++i) {
                    if (i == c) continue;
                    const double f = K[i][c];
                    for (int j = 0; j < 2 * NI; ++j) K[i][j] -= f * K[c][j];
                }
            }
            for (int i = 0; i < NI; ++i)
                for (int j = 0; j < NI; ++j) s_r[i][j] = (T)K[i][NI + j];
        }
        __syncthreads();
    }

    const T t1 = (T)(1.0 / mu1), t2 = (T)(a.lam / mu2);
    const T m1 = (T)mu1, m2 = (T)mu2;
    // rows of D this lane owns: every band but the cube's last; the last band
    // of a block before a boundary uses the next block's first x
    const int vlen = seg < S - 1 ? M : lenS - 1;
    const int64_t n = (int64_t)a.H * a.W;
    const int base = lane - seg;                // first lane of this pixel

    for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        const int64_t pix = grp * PPB + lane / S;
        const bool live = pix < n;
        int64_t yy = 0, xx = 0;
        if (live) {
            yy = pix / a.W;
            xx = pix - yy * a.W;
        }
        {
            const T* src = static_cast<const T*>(a.Hc) + yy * a.row_pitch + xx * a.pitch + seg * M;
#pragma unroll
            for (int i = 0; i < M; ++i) s_h[i][lane] = (live && i < lenS) ? src[i] : (T)0;
        }
        T x[M], b1[M], b2[M];
        T b2x = (T)0;                            // copy of the boundary Bregman variable before this block
#pragma unroll
        for (int i = 0; i < M; ++i) {
            x[i] = (T)0;
            b1[i] = (T)0;
            b2[i] = (T)0;
        }

        auto sweep = [&](auto first_c) {
            constexpr bool FIRST = decltype(first_c)::value;
            const int z0 = opaque_zero();
            const T* hcol = &s_h[0][lane + z0];
            const T* tinv = &s_inv[seg][z0];
            const T* tf = &s_f[seg][z0];
            const T* twr = &s_wr[seg][z0];
            const T* twl = &s_wl[seg][z0];
            T xn = (T)0, cprev = (T)0;
            if constexpr (S > 1 && !FIRST) {
                // x across the boundaries: the next block's first, the previous block's last
                const T nxt = __shfl(x[0], base + (seg + 1 < S ? seg + 1 : seg), 64);
                const T prv = __shfl(x[M - 1], base + (seg > 0 ? seg - 1 : seg), 64);
                xn = seg + 1 < S ? nxt : (T)0;
                if (seg > 0) {
                    const T v = (x[0] - prv) + b2x;
                    const T nb = clip(v, t2);
                    b2x = nb;
                    cprev = fma((T)-2, nb, v);
                }
            }
            T zprev = (T)0;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const T hi = hcol[i * 64];
                T a1, c;
                if constexpr (FIRST) {
                    a1 = hi;
                    c = (T)0;
                } else {
                    const T t = (hi - x[i]) + b1[i];
                    const T nb1 = clip(t, t1);
                    a1 = fma((T)2, nb1, hi - t);
                    b1[i] = nb1;
                    const T xnext = i + 1 < M ? x[i + 1] : xn;
                    const T v = (xnext - x[i]) + b2[i];
                    const T nb2 = clip(v, t2);
                    const bool has = i < vlen;
                    c = has ? fma((T)-2, nb2, v) : (T)0;
                    b2[i] = has ? nb2 : (T)0;
                }
                const T rhs = fma(m1, a1, m2 * (cprev - c));
                const T z = fma(m2, zprev, rhs) * tinv[i];
                x[i] = z;
                zprev = z;
                cprev = c;
            }
#pragma unroll
            for (int i = M - 2; i >= 0; --i) x[i] = fma(tf[i], x[i + 1], x[i]);
            if constexpr (S > 1) {
                // tips of the block solutions, then the interface values this block needs
                // (every block but the last is full: (S - 1) M < p)
                T tip[NI];
#pragma unroll
                for (int j = 0; j < S - 1; ++j) {
                    tip[2 * j] = __shfl(x[M - 1], base + j, 64);
                    tip[2 * j + 1] = __shfl(x[0], base + j + 1, 64);
                }
                T xr = (T)0, xl = (T)0;
                const int rr = seg < S - 1 ? 2 * seg + 1 : 0;
                const int rl = seg > 0 ? 2 * (seg - 1) : 0;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    xr = fma(s_r[rr][j], tip[j], xr);
                    xl = fma(s_r[rl][j], tip[j], xl);
                }
                xr = seg < S - 1 ? xr : (T)0;
                xl = seg > 0 ? xl : (T)0;
#pragma unroll
                for (int i = 0; i < M; ++i) x[i] = fma(-xr, twr[i], fma(-xl, twl[i], x[i]));
            }
        };
        sweep(std::integral_constant<bool, true>{});
        for (int k = 1; k < a.iters; ++k) sweep(std::integral_constant<bool, false>{});

        if (live) {
            T* dst = static_cast<T*>(a.X) + yy * a.xrow_pitch + xx * a.xpitch + seg * M;
#pragma unroll
            for (int i = 0; i < M; ++i)
                if (i < lenS) dst[i] = x[i];
        }
    }
}

// Lanes per pixel and segment length for p bands: segments of at most 64
// (FP32) or 32/48/56 (FP64) bands in registers, every segment non-empty.
bool l1l1_shape(int p, int dtype, int* S, int* M) {
    auto up8 = [](int v) { return (v + 7) / 8 * 8; };
    int s, m;
    if (dtype == HYRES_F32) {
        if (p <= 64) s = 1;
        else if (p <= 128) s = 2;
        else s = 4;
    } else {
        if (p <= 32) s = 1;
        else if (p <= 96) s = 2;
        else s = 4;
    }
    m = up8((p + s - 1) / s);
    if (p < 1 || p > kMaxBands || m > kL1MaxSeg || (s - 1) * m >= p) return false;
    *S = s;
    *M = m;
    return true;
}

hipError_t launch_l1l1(const L1Args& a, int num_cu, hipStream_t st) {
    int S = 0, M = 0;
    if (!l1l1_shape(a.p, a.dtype, &S, &M)) return hipErrorInvalidValue;
    const int64_t n = (int64_t)a.H * a.W;
    const int64_t groups = (n * S + 63) / 64;
    const int64_t cap = (int64_t)num_cu * 16;
    const int grid = (int)(groups < cap ? groups : cap);
    if (grid < 1) return hipSuccess;
#define HYRES_L1(T, MM, SS) \
    if (M == MM && S == SS) { \
        hipLaunchKernelGGL((k_l1l1<T, MM, SS>), dim3(grid), dim3(64), 0, st, a, groups); \
        return hipGetLastError(); \
    }
    if (a.dtype == HYRES_F32) {
        HYRES_L1(float, 8, 1) HYRES_L1(float, 16, 1) HYRES_L1(float, 24, 1) HYRES_L1(float, 32, 1)
        HYRES_L1(float, 40, 1) HYRES_L1(float, 48, 1) HYRES_L1(float, 56, 1) HYRES_L1(float, 64, 1)
        HYRES_L1(float, 40, 2) HYRES_L1(float, 48, 2) HYRES_L1(float, 56, 2) HYRES_L1(float, 64, 2)
        HYRES_L1(float, 40, 4) HYRES_L1(float, 48, 4) HYRES_L1(float, 56, 4)
    } else {
        HYRES_L1(double, 8, 1) HYRES_L1(double, 16, 1) HYRES_L1(double, 24, 1) HYRES_L1(double, 32, 1)
        HYRES_L1(double, 24, 2) HYRES_L1(double, 32, 2) HYRES_L1(double, 40, 2) HYRES_L1(double, 48, 2)
        HYRES_L1(double, 32, 4) HYRES_L1(double, 40, 4) HYRES_L1(double, 48, 4) HYRES_L1(double, 56, 4)
    }
#undef HYRES_L1
    return hipErrorInvalidValue;
}

}  // namespace hyres
