// FORPDN (Section 2.1: full-rank, wavelet-based, first-order spectral
// roughness penalty, for Gaussian noise).  The cube is whitened by the
// per-band noise, transformed band by band with the periodised 2-D db2
// wavelet, and every coefficient vector (one position, all p bands) of a
// wavelet group (the details of one level, or the coarsest approximation) is
// replaced by (I + lam D^T D)^-1 c with the group's lam chosen by SURE.
//
// The bands of one position stay together from start to end (the cube is
// pixel-major; the coefficients are stored position-major, p contiguous
// values per position), so
//   k_vdwt_level   one analysis level: each thread computes the four subband
//                  values of one (position, band) from a 4 x 4 window read
//                  across the bands of neighbouring positions (coalesced over
//                  the bands); the first level scales by 1/sigma on load;
//   (the band Gram of each group is the pixel-major Gram kernel of HyRes run
//    on the group's positions as a "cube")
//   k_forpdn_lambda one block per group: the energies of the coefficient
//                  matrix in the DCT-II eigenbasis of D^T D from the group's
//                  Gram, then SURE of the smoother on the lam grid in closed
//                  form and its argmin;
//   k_forpdn_filter the tridiagonal solve of every coefficient vector (rows
//                  staged through LDS with coalesced loads and stores);
//   k_vidwt_level  one synthesis level; the last scales by sigma on store.
#include <algorithm>

#include "hyres_internal.hpp"

namespace hyres {

namespace {
constexpr double kG0 = kH3, kG1 = -kH2, kG2 = kH1, kG3 = -kH0;   // g[m] = (-1)^m h[3 - m]

__device__ __forceinline__ int ext_index(int i, int N, int Ne) {
    i %= Ne;
    return i == N ? N - 1 : i;      // an odd length repeats its last sample
}
}  // namespace

// A thread computes a 2 x 2 block of output positions of one band: the 6 x 6
// input window is read once (9 loads per position instead of 16).
template <typename T>
__global__ __launch_bounds__(256) void k_vdwt_level(VLevel a) {
    const T hf[4] = {(T)kH0, (T)kH1, (T)kH2, (T)kH3};
    const T gf[4] = {(T)kG0, (T)kG1, (T)kG2, (T)kG3};
    const int p = a.p;
    const int Hext = a.Hin + (a.Hin & 1), Wext = a.Win + (a.Win & 1);
    const int bh = (a.h + 1) / 2, bw = (a.w + 1) / 2;         // 2 x 2 blocks of outputs
    const int64_t nq = (int64_t)bh * bw;
    constexpr int QB = 64;                                   // blocks per work item
    const int64_t nitem = (nq + QB - 1) / QB;
    const int span = QB * p;
    const int64_t sub = (int64_t)a.h * a.w * p;              // one detail block
    for (int64_t it = blockIdx.x; it < nitem; it += gridDim.x) {
        for (int e = threadIdx.x; e < span; e += blockDim.x) {
            const int ql = (int)__umulhi((uint32_t)e, a.pmag);   // e / p
            const int b = e - ql * p;
            const int64_t q = it * QB + ql;
            if (q >= nq) break;
            const int by = (int)(q / bw), bx = (int)(q - (int64_t)by * bw);
            const int y0 = 2 * by, x0 = 2 * bx;
            const T sc = a.scale ? (T)(1.0 / a.scale[b]) : (T)1;
            const T* in = static_cast<const T*>(a.in) + b;
            int64_t cx[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) cx[c] = (int64_t)ext_index(2 * x0 + c, a.Win, Wext) * a.ip;
            // along x first (two output columns), in tap order
            T rl[6][2], rh[6][2];
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const T* row = in + (int64_t)ext_index(2 * y0 + r, a.Hin, Hext) * a.irow;
                T v[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) v[c] = row[cx[c]] * sc;
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    rl[r][o] = hf[0] * v[2 * o] + hf[1] * v[2 * o + 1] + hf[2] * v[2 * o + 2] + hf[3] * v[2 * o + 3];
                    rh[r][o] = gf[0] * v[2 * o] + gf[1] * v[2 * o + 1] + gf[2] * v[2 * o + 2] + gf[3] * v[2 * o + 3];
                }
            }
#pragma unroll
            for (int oy = 0; oy < 2; ++oy) {
                const int y = y0 + oy;
#pragma unroll
                for (int ox = 0; ox < 2; ++ox) {
                    const int x = x0 + ox;
                    if (y < a.h && x < a.w) {
                        // rows 2 oy .. 2 oy + 3 of the window
                        const T l0 = rl[2 * oy][ox], l1 = rl[2 * oy + 1][ox], l2 = rl[2 * oy + 2][ox], l3 = rl[2 * oy + 3][ox];
                        const T h0 = rh[2 * oy][ox], h1 = rh[2 * oy + 1][ox], h2 = rh[2 * oy + 2][ox], h3 = rh[2 * oy + 3][ox];
                        const T ll = hf[0] * l0 + hf[1] * l1 + hf[2] * l2 + hf[3] * l3;
                        const T hl = gf[0] * l0 + gf[1] * l1 + gf[2] * l2 + gf[3] * l3;
                        const T lh = hf[0] * h0 + hf[1] * h1 + hf[2] * h2 + hf[3] * h3;
                        const T hh = gf[0] * h0 + gf[1] * h1 + gf[2] * h2 + gf[3] * h3;
                        const int64_t o = ((int64_t)y * a.w + x) * p + b;
                        T* det = static_cast<T*>(a.det) + o;
                        det[0] = lh;
                        det[sub] = hl;
                        det[2 * sub] = hh;
                        static_cast<T*>(a.ll)[o] = ll;
                    }
                }
            }
        }
    }
}

// A thread computes a 2 x 2 block of output pixels of one band: pixels
// (2Y + py, 2X + px) all take the coefficients at rows Y and Y - 1 and columns
// X and X - 1 (mod the subband size), taps py, py + 2 and px, px + 2.
template <typename T>
__global__ __launch_bounds__(256) void k_vidwt_level(VSyn a) {
    const T hf[4] = {(T)kH0, (T)kH1, (T)kH2, (T)kH3};
    const T gf[4] = {(T)kG0, (T)kG1, (T)kG2, (T)kG3};
    const int p = a.p;
    const int64_t nq = (int64_t)a.h * a.w;                   // one block per subband position
    constexpr int QB = 64;
    const int64_t nitem = (nq + QB - 1) / QB;
    const int span = QB * p;
    const T* LL = static_cast<const T*>(a.ll);
    const T* LH = static_cast<const T*>(a.det);
    const T* HL = LH + nq * p;
    const T* HH = HL + nq * p;
    for (int64_t it = blockIdx.x; it < nitem; it += gridDim.x) {
        for (int e = threadIdx.x; e < span; e += blockDim.x) {
            const int ql = (int)__umulhi((uint32_t)e, a.pmag);
            const int b = e - ql * p;
            const int64_t q = it * QB + ql;
            if (q >= nq) break;
            const int Y = (int)(q / a.w), X = (int)(q - (int64_t)Y * a.w);
            const int Ym = Y == 0 ? a.h - 1 : Y - 1, Xm = X == 0 ? a.w - 1 : X - 1;
            const int64_t i00 = ((int64_t)Y * a.w + X) * p + b, i01 = ((int64_t)Y * a.w + Xm) * p + b;
            const int64_t i10 = ((int64_t)Ym * a.w + X) * p + b, i11 = ((int64_t)Ym * a.w + Xm) * p + b;
            // [row Y or Y - 1][column X or X - 1]
            const T ll[2][2] = {{LL[i00], LL[i01]}, {LL[i10], LL[i11]}};
            const T hl[2][2] = {{HL[i00], HL[i01]}, {HL[i10], HL[i11]}};
            const T lh[2][2] = {{LH[i00], LH[i01]}, {LH[i10], LH[i11]}};
            const T hh[2][2] = {{HH[i00], HH[i01]}, {HH[i10], HH[i11]}};
            const T sc = a.scale ? (T)a.scale[b] : (T)1;
#pragma unroll
            for (int py = 0; py < 2; ++py) {
                const int iy = 2 * Y + py;
                if (iy >= a.Hin) continue;
                // along y first: lo_x from LL and HL, hi_x from LH and HH (taps py then py + 2)
                T lo[2], hi[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    lo[c] = (hf[py] * ll[0][c] + gf[py] * hl[0][c]) + (hf[py + 2] * ll[1][c] + gf[py + 2] * hl[1][c]);
                    hi[c] = (hf[py] * lh[0][c] + gf[py] * hh[0][c]) + (hf[py + 2] * lh[1][c] + gf[py + 2] * hh[1][c]);
                }
#pragma unroll
                for (int px = 0; px < 2; ++px) {
                    const int ix = 2 * X + px;
                    if (ix >= a.Win) continue;
                    T v = (hf[px] * lo[0] + gf[px] * hi[0]) + (hf[px + 2] * lo[1] + gf[px + 2] * hi[1]);
                    if (a.scale) v *= sc;
                    static_cast<T*>(a.out)[(int64_t)iy * a.orow + (int64_t)ix * a.op + b] = v;
                }
            }
        }
    }
}

// One block per group: e_k = q_k^T G q_k in the DCT-II basis q_k(i) =
// n_k cos(pi k (2i + 1) / (2p)), formed from the sums of G along its
// anti-diagonals (A_s = sum_{r+c=s} G_rc) and diagonals (B_t = sum_{r-c=t} G_rc)
// by the product-to-sum identity, O(p^2) per group; then SURE of the smoother
// (I + lam D^T D)^-1 at unit noise on the grid lam = 10^(t/10), t = -40..40, in
// closed form, SURE(lam) = sum_k e_k (lam d_k / (1 + lam d_k))^2 - N p
// + 2 N sum_k 1 / (1 + lam d_k), d_k = 2 - 2 cos(pi k / p), and its argmin
// (the smallest lam among equal minima).  With given thresholds only SURE at them.
__global__ __launch_bounds__(256) void k_forpdn_lambda(FLambda a) {
    constexpr int NT = 256;
    __shared__ double s_cos[4 * kMaxBands];       // cos(pi m / (2p)), m < 4p
    __shared__ double s_A[2 * kMaxBands], s_B[kMaxBands];   // anti-diagonal sums; diagonal sums for |t| (both signs)
    __shared__ double s_e[kMaxBands], s_d[kMaxBands];
    __shared__ double s_sure[kForpdnGrid];
    const int j = blockIdx.x, t = threadIdx.x, p = a.p, P4 = 4 * p;
    const double* G = a.G[j];
    const double N = (double)a.count[j];
    for (int m = t; m < P4; m += NT) s_cos[m] = cos(M_PI * (double)m / (2.0 * p));
    for (int sidx = t; sidx < 2 * p - 1; sidx += NT) {
        double acc = 0.0;
        const int r0 = sidx < p ? 0 : sidx - p + 1, r1 = sidx < p ? sidx : p - 1;
#pragma unroll 8
        for (int r = r0; r <= r1; ++r) acc += G[(int64_t)r * p + (sidx - r)];
        s_A[sidx] = acc;
    }
    for (int d = t; d < p; d += NT) {
        double acc = 0.0;
#pragma unroll 8
        for (int c = 0; c + d < p; ++c) acc += G[(int64_t)(c + d) * p + c];
        if (d > 0) {
#pragma unroll 8
            for (int c = 0; c + d < p; ++c) acc += G[(int64_t)c * p + (c + d)];
        }
        s_B[d] = acc;
    }
    __syncthreads();
    // q_k^T G q_k = n_k^2 / 2 (sum_s A_s cos(pi k (s + 1) / p) + sum_t B_t cos(pi k t / p))
    const double c0 = 1.0 / p, ck = 2.0 / p;
    for (int k = t; k < p; k += NT) {
        double sa = 0.0, sb = 0.0;
        for (int sidx = 0; sidx < 2 * p - 1; ++sidx) sa = fma(s_A[sidx], s_cos[(2 * k * (sidx + 1)) % P4], sa);
        for (int d = 0; d < p; ++d) sb = fma(s_B[d], s_cos[(2 * k * d) % P4], sb);
        s_e[k] = 0.5 * (k == 0 ? c0 : ck) * (sa + sb);
        s_d[k] = 2.0 - 2.0 * s_cos[(2 * k) % P4];
    }
    __syncthreads();
    auto sure_at = [&](double lam) {
        double res = 0.0, tr = 0.0;
        for (int k = 0; k < p; ++k) {
            const double f = 1.0 / (1.0 + lam * s_d[k]);
            const double o = 1.0 - f;
            res = fma(s_e[k] * o, o, res);
            tr += f;
        }
        return res - N * p + 2.0 * N * tr;
    };
    if (a.lambda_in) {
        if (t == 0) {
            const double lam = a.lambda_in[j];
            a.lambda[j] = lam;
            a.sure[j] = sure_at(lam);
        }
        return;
    }
    for (int g = t; g < kForpdnGrid; g += NT) s_sure[g] = sure_at(pow(10.0, (double)(g - kForpdnGrid / 2) / 10.0));
    __syncthreads();
    if (t == 0) {
        int best = 0;
        for (int g = 1; g < kForpdnGrid; ++g)
            if (s_sure[g] < s_sure[best]) best = g;
        a.lambda[j] = pow(10.0, (double)(best - kForpdnGrid / 2) / 10.0);
        a.sure[j] = s_sure[best];
    }
}

// Each lane owns one coefficient vector (a position): a wave stages its 64
// positions (64 p consecutive values) through LDS with coalesced loads, solves
// (I + lam_j D^T D) x = c in its row (Thomas; factors per group formed in
// FP64 once per block), and writes the rows back the same way.
template <typename T>
__global__ __launch_bounds__(64) void k_forpdn_filter(FFilter a) {
    extern __shared__ unsigned char s_raw[];
    const int p = a.p, G = a.groups, SP = p | 1;
    T* s_inv = reinterpret_cast<T*>(s_raw);                 // [G][p]
    T* s_f = s_inv + (size_t)G * p;                         // [G][p]
    T* s_row = s_f + (size_t)G * p;                         // [64][SP]
    const int lane = threadIdx.x;
    for (int j = lane; j < G; j += 64) {
        const double lam = a.lambda[j];
        double beta = 0.0;
        for (int i = 0; i < p; ++i) {
            const double d = p == 1 ? 1.0 : (i == 0 || i == p - 1) ? 1.0 + lam : 1.0 + 2.0 * lam;
            beta = i == 0 ? d : d - lam * lam / beta;
            s_inv[j * p + i] = (T)(1.0 / beta);
            s_f[j * p + i] = (T)(lam / beta);
        }
    }
    __syncthreads();
    const int64_t npos = a.npos;
    const int64_t nblk = (npos + 63) / 64;
    T* coef = static_cast<T*>(a.coef);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t pos0 = blk * 64;
        const int cnt = npos - pos0 < 64 ? (int)(npos - pos0) : 64;
        const int span = cnt * p;
        T* src = coef + pos0 * p;
        // eight loads in flight per lane before their LDS stores
#pragma unroll 8
        for (int e = lane; e < span; e += 64) {
            const int r = (int)__umulhi((uint32_t)e, a.pmag);
            s_row[r * SP + (e - r * p)] = src[e];
        }
        __syncthreads();
        if (lane < cnt) {
            const int64_t pos = pos0 + lane;
            int j = 0;
            while (j + 1 < G && pos >= a.goff[j + 1]) ++j;
            const double lamd = a.lambda[j];
            const T lam = (T)lamd;
            const T* inv = s_inv + j * p;
            const T* f = s_f + j * p;
            T* row = s_row + lane * SP;
            T z = row[0] * inv[0];
            row[0] = z;
#pragma unroll 8
            for (int i = 1; i < p; ++i) {
                z = fma(lam, z, row[i]) * inv[i];
                row[i] = z;
            }
            T x = z;
#pragma unroll 8
            for (int i = p - 2; i >= 0; --i) {
                x = fma(f[i], x, row[i]);
                row[i] = x;
            }
        }
        __syncthreads();
#pragma unroll 8
        for (int e = lane; e < span; e += 64) {
            const int r = (int)__umulhi((uint32_t)e, a.pmag);
            src[e] = s_row[r * SP + (e - r * p)];
        }
        __syncthreads();
    }
}

hipError_t launch_vdwt_level(int dtype, const VLevel& a, int num_cu, hipStream_t s) {
    const int64_t nblk = ((int64_t)((a.h + 1) / 2) * ((a.w + 1) / 2) + 63) / 64;
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(nblk, 1), (int64_t)num_cu * 8);
    if (dtype == HYRES_F32) hipLaunchKernelGGL(k_vdwt_level<float>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_vdwt_level<double>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vidwt_level(int dtype, const VSyn& a, int num_cu, hipStream_t s) {
    const int64_t nblk = ((int64_t)a.h * a.w + 63) / 64;
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(nblk, 1), (int64_t)num_cu * 8);
    if (dtype == HYRES_F32) hipLaunchKernelGGL(k_vidwt_level<float>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_vidwt_level<double>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_forpdn_lambda(const FLambda& a, int groups, hipStream_t s) {
    hipLaunchKernelGGL(k_forpdn_lambda, dim3(groups), dim3(256), 0, s, a);
    return hipGetLastError();
}

size_t forpdn_filter_lds(int dtype, int p, int groups) {
    const size_t es = dtype == HYRES_F64 ? 8 : 4;
    return es * ((size_t)2 * groups * p + (size_t)64 * (p | 1));
}

hipError_t launch_forpdn_filter(int dtype, const FFilter& a, int num_cu, hipStream_t s) {
    const int64_t nblk = (a.npos + 63) / 64;
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(nblk, 1), (int64_t)num_cu * 8);
    const size_t lds = forpdn_filter_lds(dtype, a.p, a.groups);
    if (dtype == HYRES_F32) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_forpdn_filter<float>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_forpdn_filter<float>, dim3(grid), dim3(64), lds, s, a);
    } else {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_forpdn_filter<double>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_forpdn_filter<double>, dim3(grid), dim3(64), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace hyres
