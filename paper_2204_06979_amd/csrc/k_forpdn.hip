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

template <typename T>
__global__ __launch_bounds__(256) void k_vdwt_level(VLevel a) {
    const T h0 = (T)kH0, h1 = (T)kH1, h2 = (T)kH2, h3 = (T)kH3;
    const T g0 = (T)kG0, g1 = (T)kG1, g2 = (T)kG2, g3 = (T)kG3;
    const int p = a.p;
    const int Hext = a.Hin + (a.Hin & 1), Wext = a.Win + (a.Win & 1);
    const int64_t npos = (int64_t)a.h * a.w;
    constexpr int PB = 64;                                  // positions per block
    const int64_t nblk = (npos + PB - 1) / PB;
    const int span = PB * p;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        for (int e = threadIdx.x; e < span; e += blockDim.x) {
            const int pl = (int)__umulhi((uint32_t)e, a.pmag);   // e / p
            const int b = e - pl * p;
            const int64_t pos = blk * PB + pl;
            if (pos >= npos) break;
            const int y = (int)(pos / a.w), x = (int)(pos - (int64_t)y * a.w);
            const T sc = a.scale ? (T)(1.0 / a.scale[b]) : (T)1;
            const T* in = static_cast<const T*>(a.in) + b;
            int cx[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) cx[c] = ext_index(2 * x + c, a.Win, Wext);
            T rl[4], rh[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int iy = ext_index(2 * y + r, a.Hin, Hext);
                const T* row = in + (int64_t)iy * a.irow;
                const T v0 = row[(int64_t)cx[0] * a.ip] * sc, v1 = row[(int64_t)cx[1] * a.ip] * sc;
                const T v2 = row[(int64_t)cx[2] * a.ip] * sc, v3 = row[(int64_t)cx[3] * a.ip] * sc;
                // along x first, in tap order
                rl[r] = h0 * v0 + h1 * v1 + h2 * v2 + h3 * v3;
                rh[r] = g0 * v0 + g1 * v1 + g2 * v2 + g3 * v3;
            }
            const T ll = h0 * rl[0] + h1 * rl[1] + h2 * rl[2] + h3 * rl[3];
            const T hl = g0 * rl[0] + g1 * rl[1] + g2 * rl[2] + g3 * rl[3];
            const T lh = h0 * rh[0] + h1 * rh[1] + h2 * rh[2] + h3 * rh[3];
            const T hh = g0 * rh[0] + g1 * rh[1] + g2 * rh[2] + g3 * rh[3];
            T* det = static_cast<T*>(a.det) + pos * p + b;
            det[0] = lh;
            det[npos * p] = hl;
            det[2 * npos * p] = hh;
            static_cast<T*>(a.ll)[pos * p + b] = ll;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_vidwt_level(VSyn a) {
    const T hf[4] = {(T)kH0, (T)kH1, (T)kH2, (T)kH3};
    const T gf[4] = {(T)kG0, (T)kG1, (T)kG2, (T)kG3};
    const int p = a.p;
    const int Hext = a.Hin + (a.Hin & 1), Wext = a.Win + (a.Win & 1);
    const int64_t npos = (int64_t)a.Hin * a.Win;
    const int64_t nsub = (int64_t)a.h * a.w;
    constexpr int PB = 64;
    const int64_t nblk = (npos + PB - 1) / PB;
    const int span = PB * p;
    const T* LL = static_cast<const T*>(a.ll);
    const T* LH = static_cast<const T*>(a.det);
    const T* HL = LH + nsub * p;
    const T* HH = HL + nsub * p;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        for (int e = threadIdx.x; e < span; e += blockDim.x) {
            const int pl = (int)__umulhi((uint32_t)e, a.pmag);
            const int b = e - pl * p;
            const int64_t pos = blk * PB + pl;
            if (pos >= npos) break;
            const int iy = (int)(pos / a.Win), ix = (int)(pos - (int64_t)iy * a.Win);
            // taps m of parity i, and the coefficient k with (2k + m) mod Next == i
            const int my0 = iy & 1, my1 = my0 + 2;
            const int ky0 = (iy - my0) >> 1, ky1 = ((iy - my1 + Hext) % Hext) >> 1;
            const int mx0 = ix & 1, mx1 = mx0 + 2;
            const int kx0 = (ix - mx0) >> 1, kx1 = ((ix - mx1 + Wext) % Wext) >> 1;
            auto at = [&](const T* s, int ky, int kx) { return s[((int64_t)ky * a.w + kx) * p + b]; };
            // along y first (lo_x from LL and HL, hi_x from LH and HH), then along x
            T lo[2], hi[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int kx = c ? kx1 : kx0;
                lo[c] = (hf[my0] * at(LL, ky0, kx) + gf[my0] * at(HL, ky0, kx)) +
                        (hf[my1] * at(LL, ky1, kx) + gf[my1] * at(HL, ky1, kx));
                hi[c] = (hf[my0] * at(LH, ky0, kx) + gf[my0] * at(HH, ky0, kx)) +
                        (hf[my1] * at(LH, ky1, kx) + gf[my1] * at(HH, ky1, kx));
            }
            T v = (hf[mx0] * lo[0] + gf[mx0] * hi[0]) + (hf[mx1] * lo[1] + gf[mx1] * hi[1]);
            if (a.scale) v *= (T)a.scale[b];
            static_cast<T*>(a.out)[(int64_t)iy * a.orow + (int64_t)ix * a.op + b] = v;
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
        for (int r = r0; r <= r1; ++r) acc += G[(int64_t)r * p + (sidx - r)];
        s_A[sidx] = acc;
    }
    for (int d = t; d < p; d += NT) {
        double acc = 0.0;
        for (int c = 0; c + d < p; ++c) acc += G[(int64_t)(c + d) * p + c];
        if (d > 0)
            for (int c = 0; c + d < p; ++c) acc += G[(int64_t)c * p + (c + d)];
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
            for (int i = 1; i < p; ++i) {
                z = fma(lam, z, row[i]) * inv[i];
                row[i] = z;
            }
            T x = z;
            for (int i = p - 2; i >= 0; --i) {
                x = fma(f[i], x, row[i]);
                row[i] = x;
            }
        }
        __syncthreads();
        for (int e = lane; e < span; e += 64) {
            const int r = (int)__umulhi((uint32_t)e, a.pmag);
            src[e] = s_row[r * SP + (e - r * p)];
        }
        __syncthreads();
    }
}

hipError_t launch_vdwt_level(int dtype, const VLevel& a, int num_cu, hipStream_t s) {
    const int64_t nblk = ((int64_t)a.h * a.w + 63) / 64;
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(nblk, 1), (int64_t)num_cu * 8);
    if (dtype == HYRES_F32) hipLaunchKernelGGL(k_vdwt_level<float>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_vdwt_level<double>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vidwt_level(int dtype, const VSyn& a, int num_cu, hipStream_t s) {
    const int64_t nblk = ((int64_t)a.Hin * a.Win + 63) / 64;
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
