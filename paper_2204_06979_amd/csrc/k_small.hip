// FP64 small solves of one cube in one 1024-thread workgroup:
//   noise   sigma_i^2 = 1 / (n [G^-1]_ii)           (Gauss-Jordan sweep of the band Gram)
//   whiten  C = D^-1 G D^-1,  D = diag(sigma)
//   eigen   Householder tridiagonalisation of C, every eigenvalue by Sturm-count
//           multisection, the top-r eigenvectors of the tridiagonal matrix from a
//           twisted factorisation, modified Gram-Schmidt, back-transformation.
//
// The regression of band i on the other bands leaves the residual sum of
// squares 1/[G^-1]_ii (Schur complement), which is why the noise estimate only
// needs the diagonal of the inverse Gram.
//
// The p x p matrix lives in registers: thread (tr, tc) of a ROWS x COLS grid
// holds the entries (tr + ROWS a, tc + COLS b), a < BR, b < BC.  Up to
// p = 128 the grid is 16 x 16 (256 threads, one wave per SIMD), up to 176 it is
// 32 x 16 (512 threads): few waves keep the two barriers of every elimination
// step cheap, and a row sum is a 16-lane DPP reduction.  Beyond, 24 x 32
// (768 threads).  A column is broadcast through LDS.
#include "hyres_internal.hpp"

namespace hyres {

constexpr int kSmallP = 256;   // LDS vector length (p <= 224)

// Sturm count: number of eigenvalues of the symmetric tridiagonal (ds, e2s)
// smaller than x, from the sign changes of the leading principal minors
// p_i(x) = (d_i - x) p_{i-1}(x) - e_{i-1}^2 p_{i-2}(x) (a minor that is
// exactly zero counts as positive); both minors are rescaled by a power of two
// every 8 steps so the recursion stays in range.
__device__ __forceinline__ int sgnbit(double v) { return (int)((unsigned)__double2hiint(v) >> 31); }

template <bool PRE>
__device__ __forceinline__ int sturm_count(const double* __restrict__ ds, const double* __restrict__ e2s,
                                           int p, double x) {
    double pm2 = 1.0, pm1 = ds[0] - x;
    int neg = sgnbit(pm1);
    int cnt = neg;
    int i = 1;
    // blocks of 8 steps; with PRE the next block's entries are read while this
    // one runs (16 more registers)
    double dd[8], ee[8];
    if (PRE && i + 8 <= p) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dd[u] = ds[i + u];
            ee[u] = e2s[i + u - 1];
        }
    }
    for (; i + 8 <= p; i += 8) {
        double dn[8], en[8];
        const bool more = PRE && i + 16 <= p;
        if (!PRE) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                dd[u] = ds[i + u];
                ee[u] = e2s[i + u - 1];
            }
        }
        if (more) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                dn[u] = ds[i + 8 + u];
                en[u] = e2s[i + 7 + u];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double pi = fma(dd[u] - x, pm1, -ee[u] * pm2);
            const int sg = sgnbit(pi);
            cnt += sg ^ neg;
            neg = sg;
            pm2 = pm1;
            pm1 = pi;
        }
        int e1, e2;
        frexp(pm1, &e1);
        frexp(pm2, &e2);
        const int e = e1 > e2 ? e1 : e2;
        pm1 = ldexp(pm1, -e);
        pm2 = ldexp(pm2, -e);
        if (more) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                dd[u] = dn[u];
                ee[u] = en[u];
            }
        }
    }
    for (; i < p; ++i) {
        const double pi = fma(ds[i] - x, pm1, -e2s[i - 1] * pm2);
        const int sg = sgnbit(pi);
        cnt += sg ^ neg;
        neg = sg;
        pm2 = pm1;
        pm1 = pi;
    }
    return cnt;
}

// In place: lo = max and hi = min over each aligned group of M lanes (M = 4, 16, 32 or 64).
__device__ __forceinline__ void group_maxmin(double& lo, double& hi, int M) {
    double a;
    a = dpp_f64<0xB1>(lo); lo = a > lo ? a : lo;      // quad_perm [1,0,3,2]
    a = dpp_f64<0xB1>(hi); hi = a < hi ? a : hi;
    a = dpp_f64<0x4E>(lo); lo = a > lo ? a : lo;      // quad_perm [2,3,0,1]
    a = dpp_f64<0x4E>(hi); hi = a < hi ? a : hi;
    if (M == 4) return;
    a = dpp_f64<0x141>(lo); lo = a > lo ? a : lo;     // row_half_mirror
    a = dpp_f64<0x141>(hi); hi = a < hi ? a : hi;
    a = dpp_f64<0x140>(lo); lo = a > lo ? a : lo;     // row_mirror
    a = dpp_f64<0x140>(hi); hi = a < hi ? a : hi;
    if (M == 16) return;
    const double l0 = readlane_f64(lo, 0), l1 = readlane_f64(lo, 16), l2 = readlane_f64(lo, 32),
                 l3 = readlane_f64(lo, 48);
    const double h0 = readlane_f64(hi, 0), h1 = readlane_f64(hi, 16), h2 = readlane_f64(hi, 32),
                 h3 = readlane_f64(hi, 48);
    const double la = l0 > l1 ? l0 : l1, lb = l2 > l3 ? l2 : l3;
    const double ha = h0 < h1 ? h0 : h1, hb = h2 < h3 ? h2 : h3;
    if (M == 32) {
        const bool upper = (threadIdx.x & 32) != 0;
        lo = upper ? lb : la;
        hi = upper ? hb : ha;
        return;
    }
    lo = la > lb ? la : lb;
    hi = ha < hb ? ha : hb;
}

// Gauss-Jordan sweep of the symmetric positive definite p x p matrix M held
// in the register tile A (thread (tr, tc) of the ROWS x COLS grid holds the
// entries (tr + ROWS a, tc + COLS b); entries beyond p hold the identity).
// Afterwards A = -M^-1.  diag: the diagonal of M in LDS, for the pivot test (a
// pivot below 1e-12 of its diagonal entry is replaced by 1 and reported as
// HYRES_DEV_NOT_PD).  Every thread of the block takes part (barriers).
template <int BR, int BC, int ROWS, int COLS>
__device__ __forceinline__ int gj_sweep(double (&A)[BR][BC], int p, int tr, int tc, const double* diag,
                                        double (*s_col)[kSmallP], double (*s_col2)[kSmallP]) {
    constexpr int NTH = ROWS * COLS;
    int flags = 0;
    // pivots in pairs (k0, k1): one barrier per pair.  The column k1 after
    // the k0 step is formed from the two broadcast columns exactly as the
    // k0 step forms it in the registers of its owners, so the result is
    // that of sweeping the pivots one at a time.  Grids of more than 512
    // threads (a tighter register budget) sweep one pivot per barrier.
    constexpr bool kPairs = NTH <= 512;
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
        for (int kk = 0; kk < COLS; kk += kPairs ? 2 : 1) {
            const int k0 = COLS * bb + kk, k1 = k0 + 1;
            if (k0 >= p) break;
            const bool two = kPairs && k1 < p;
            const int buf = (kPairs ? k0 >> 1 : k0) & 1;
            if (tc == kk) {
#pragma unroll
                for (int a = 0; a < BR; ++a) s_col[buf][tr + ROWS * a] = A[a][bb];
            }
            if (two && tc == kk + 1) {
#pragma unroll
                for (int a = 0; a < BR; ++a) s_col2[buf][tr + ROWS * a] = A[a][bb];
            }
            __syncthreads();
            // the pivot is the regression residual of band k on the bands swept so far
            double d0 = s_col[buf][k0];
            if (!(d0 > 1e-12 * diag[k0])) {
                flags |= HYRES_DEV_NOT_PD;
                d0 = 1.0;
            }
            const double inv0 = 1.0 / d0;
            double cj[BC];
#pragma unroll
            for (int b = 0; b < BC; ++b) cj[b] = s_col[buf][tc + COLS * b];
#pragma unroll
            for (int a = 0; a < BR; ++a) {
                const int i = tr + ROWS * a;
                const double ci = s_col[buf][i] * inv0;
                if (i == k0) {
#pragma unroll
                    for (int b = 0; b < BC; ++b) A[a][b] = cj[b] * inv0;
                    if (tc == kk) A[a][bb] = -inv0;
                } else {
#pragma unroll
                    for (int b = 0; b < BC; ++b) A[a][b] = fma(-ci, cj[b], A[a][b]);
                    if (tc == kk) A[a][bb] = ci;
                }
            }
            if (two) {
                const double ck1 = s_col[buf][k1];
                // column k1 after the k0 step
                auto ep = [&](int i) {
                    return i == k0 ? ck1 * inv0 : fma(-(s_col[buf][i] * inv0), ck1, s_col2[buf][i]);
                };
                double d1 = ep(k1);
                if (!(d1 > 1e-12 * diag[k1])) {
                    flags |= HYRES_DEV_NOT_PD;
                    d1 = 1.0;
                }
                const double inv1 = 1.0 / d1;
#pragma unroll
                for (int b = 0; b < BC; ++b) cj[b] = ep(tc + COLS * b);
#pragma unroll
                for (int a = 0; a < BR; ++a) {
                    const int i = tr + ROWS * a;
                    const double ci = ep(i) * inv1;
                    if (i == k1) {
#pragma unroll
                        for (int b = 0; b < BC; ++b) A[a][b] = cj[b] * inv1;
                        if (tc == kk + 1) A[a][bb] = -inv1;
                    } else {
#pragma unroll
                        for (int b = 0; b < BC; ++b) A[a][b] = fma(-ci, cj[b], A[a][b]);
                        if (tc == kk + 1) A[a][bb] = ci;
                    }
                }
            }
        }
    }
    return flags;
}

template <int BR, int BC, int ROWS, int COLS>
__global__ __launch_bounds__(ROWS * COLS) void k_small(const CubeDesc* __restrict__ descs,
                                                       const int* __restrict__ cubes, int ncls) {
    constexpr int NTH = ROWS * COLS;
    constexpr int NW = NTH / 64;           // waves
    constexpr int VPW = (kMaxRank + NW - 1) / NW;   // eigenvectors per wave
    if ((int)blockIdx.x >= ncls) return;
    const CubeDesc& d = descs[cubes[blockIdx.x]];
    const int p = d.p, r = d.r;
    const double nn = (double)d.n;
    const int t = threadIdx.x, tc = t % COLS, tr = t / COLS, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);

    __shared__ double s_col[2][kSmallP];
    __shared__ double s_col2[2][kSmallP];
    __shared__ double s_ub[kSmallP];
    __shared__ double s_sig[kSmallP];
    __shared__ double s_dd[kSmallP], s_ee[kSmallP], s_e2[kSmallP], s_hb[kSmallP], s_ev[kSmallP];
    __shared__ double s_zD[kSmallP * kMaxRank];      // pivots of the top-down factorisation [i][g]
    __shared__ double s_zU[kSmallP * kMaxRank];      // multipliers of the bottom-up one    [i][g]
    __shared__ double s_z[kMaxRank][kSmallP];        // eigenvectors of the tridiagonal / of C
    __shared__ double s_red[4];
    __shared__ double s_vav[NW];                     // per-wave shares of v^T A v
    __shared__ int s_kb[kMaxRank];                   // twist indices
    __shared__ double s_cross[kMaxRank][kMaxRank + 1];   // rank by SURE: sum_{j>=k} l_i / (l_i - l_j), [i][k]
    __shared__ int s_rank;                           // rank used
    __shared__ double s_chk[3][NW];                  // eigenpair check: residual, norm of C, orthonormality
    __shared__ int s_flags;

    if (t == 0) s_flags = 0;
    // the Householder step reads the broadcast column and u over the whole column
    // range of the thread grid, which can reach past its row range: zero first
    for (int i = t; i < kSmallP; i += NTH) {
        s_col[0][i] = s_col[1][i] = 0.0;
        s_ub[i] = 0.0;
    }
    __syncthreads();
    int flags = 0;
    HYRES_STAMP(d, 0);
    double A[BR][BC];

#pragma unroll
    for (int a = 0; a < BR; ++a)
#pragma unroll
        for (int b = 0; b < BC; ++b) {
            const int i = tr + ROWS * a, j = tc + COLS * b;
            A[a][b] = (i < p && j < p) ? d.G[(int64_t)i * p + j] : (i == j ? 1.0 : 0.0);
        }

    // ---------------------------------------------------------------- noise
    if (d.mode & 1) {
        // diagonal of G for the pivot test (s_ev is free until the eigenvalues)
        for (int i = t; i < p; i += NTH) s_ev[i] = d.G[(int64_t)i * p + i];
        flags |= gj_sweep<BR, BC, ROWS, COLS>(A, p, tr, tc, s_ev, s_col, s_col2);
        // after sweeping every index, A = -G^-1
#pragma unroll
        for (int a = 0; a < BR; ++a)
#pragma unroll
            for (int b = 0; b < BC; ++b) {
                const int i = tr + ROWS * a, j = tc + COLS * b;
                if (i == j && i < p) {
                    const double gii = -A[a][b];
                    double s = 1.0;
                    if (gii > 0.0 && !(flags & HYRES_DEV_NOT_PD)) s = sqrt(1.0 / (nn * gii));
                    else flags |= HYRES_DEV_NOT_PD;
                    s_sig[i] = s;
                    d.sigma[i] = s;
                }
            }
    } else if (t < p) {
        const double s = d.sigma_in ? d.sigma_in[t] : 1.0;
        s_sig[t] = s;
        d.sigma[t] = s;
    }
    __syncthreads();

    HYRES_STAMP(d, 1);
    if (d.mode & 2) {
        // ------------------------------------------------------- whitened Gram
#pragma unroll
        for (int a = 0; a < BR; ++a)
#pragma unroll
            for (int b = 0; b < BC; ++b) {
                const int i = tr + ROWS * a, j = tc + COLS * b;
                A[a][b] = (i < p && j < p) ? d.G[(int64_t)i * p + j] / (s_sig[i] * s_sig[j]) : 0.0;
            }

        // ------------------------------------------------ tridiagonalisation
        // (register column bb a compile-time index: the tile stays in registers)
        static_for<BC>([&](auto bbc) {
            constexpr int bb = decltype(bbc)::value;
            for (int kk = 0; kk < COLS; ++kk) {
                const int k = COLS * bb + kk;
                if (k >= p - 2) break;
                const int buf = k & 1;
                if (tc == kk) {
                    // column k below the diagonal; the entries at and above it go out as
                    // zeros (rows beyond p are zero already), so readers need no masks
#pragma unroll
                    for (int a = 0; a < BR; ++a) {
                        const int i = tr + ROWS * a;
                        s_col[buf][i] = i > k ? A[a][bb] : 0.0;
                        if (i == k) s_dd[k] = A[a][bb];
                    }
                }
                __syncthreads();
                // A v with v = x - alpha e_{k+1} (x: column k below the diagonal)
                // is A x - alpha A e_{k+1}: the products with x start before the
                // norm that gives alpha is known
                // LDS reads are unconditional (every index of the thread grid is
                // inside the vectors) and masked by selects: no divergent branches
                double xc[BC];
#pragma unroll
                for (int b = 0; b < BC; ++b) xc[b] = s_col[buf][tc + COLS * b];
                double ps[BR];
#pragma unroll
                for (int a = 0; a < BR; ++a) {
                    double sa = 0.0;
                    if (ROWS * a + ROWS - 1 > k) {
#pragma unroll
                        for (int b = 0; b < BC; ++b)
                            if (COLS * b + COLS - 1 > k) sa = fma(A[a][b], xc[b], sa);
                    }
                    ps[a] = sa;
                }
                double ss = 0.0;
                for (int i = k + 1 + lane; i < p; i += 64) {
                    const double v = s_col[buf][i];
                    ss = fma(v, v, ss);
                }
                ss = wave_sum(ss);
                const double x1 = s_col[buf][k + 1];
                const double nrm = sqrt(ss);
                const double alpha = x1 >= 0.0 ? -nrm : nrm;
                const double vtv = 2.0 * alpha * (alpha - x1);
                const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
                const double v1 = x1 - alpha;
                // column k + 1 sits in register column bb (next thread column) or bb + 1 (thread column 0)
                const bool own1 = kk + 1 < COLS ? tc == kk + 1 : tc == 0;
                double q = 0.0;
#pragma unroll
                for (int a = 0; a < BR; ++a) {
                    const int i = tr + ROWS * a;
                    if (ROWS * a + ROWS - 1 > k) {
                        const double ci = s_col[buf][i];
                        const double vi = i == k + 1 ? v1 : ci;
                        const double a1 = kk + 1 < COLS ? A[a][bb] : A[a][bb + 1 < BC ? bb + 1 : bb];
                        if (own1) ps[a] = fma(-alpha, a1, ps[a]);
                        q = fma(vi, ps[a], q);    // this thread's share of v^T A v
                    }
                }
                q = wave_sum(q);
                // v = x with v1 at k + 1: column k + 1 is register column bb of thread
                // column kk + 1, or register column bb + 1 of thread column 0
                double vc[BC];
#pragma unroll
                for (int b = 0; b < BC; ++b) vc[b] = xc[b];
                if (kk + 1 < COLS) {
                    if (tc == kk + 1) vc[bb] = v1;
                } else if constexpr (bb + 1 < BC) {
                    if (tc == 0) vc[bb + 1] = v1;
                }
#pragma unroll
                for (int a = 0; a < BR; ++a) {
                    double sa = 0.0;
                    if (ROWS * a + ROWS - 1 > k) sa = COLS == 32 ? half_sum(ps[a]) : row16_sum(ps[a]);
                    if (tc == 0) s_ub[tr + ROWS * a] = beta * sa;
                }
                if (lane == 0) s_vav[wave] = q;
                if (t == 0) {
                    s_ee[k] = alpha;
                    s_hb[k] = beta;
                }
                if (t > k && t < p) d.hv[(int64_t)k * p + t] = (t == k + 1) ? v1 : s_col[buf][t];
                __syncthreads();
                // u = beta A v, w = u - (beta/2)(u^T v) v, A <- A - v w^T - w v^T
                double vav = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) vav += s_vav[w];
                const double K = 0.5 * beta * (beta * vav);
                double wc[BC];
#pragma unroll
                for (int b = 0; b < BC; ++b) {
                    const int j = tc + COLS * b;
                    const double uj = s_ub[j];
                    wc[b] = j > k ? uj - K * vc[b] : 0.0;      // u and v vanish beyond p
                }
#pragma unroll
                for (int a = 0; a < BR; ++a) {
                    if (ROWS * a + ROWS - 1 > k) {
                        const int i = tr + ROWS * a;
                        const double ci = s_col[buf][i], ui = s_ub[i];
                        const double vi = i == k + 1 ? v1 : ci;
                        const double wi = i > k ? ui - K * vi : 0.0;
#pragma unroll
                        for (int b = 0; b < BC; ++b) {
                            if (COLS * b + COLS - 1 > k) A[a][b] = fma(-wi, vc[b], fma(-vi, wc[b], A[a][b]));
                        }
                    }
                }
            }
        });
        __syncthreads();
#pragma unroll
        for (int a = 0; a < BR; ++a)
#pragma unroll
            for (int b = 0; b < BC; ++b) {
                const int i = tr + ROWS * a, j = tc + COLS * b;
                if (i == j && i >= p - 2 && i < p) s_dd[i] = A[a][b];
                if (i == p - 1 && j == p - 2) s_ee[p - 2] = A[a][b];
            }
        __syncthreads();

        HYRES_STAMP(d, 2);
        // ------------------------------------------------ eigenvalues (all)
        if (wave == 0) {
            double m = 0.0;
            for (int i = lane; i < p; i += 64) {
                double rr = fabs(s_dd[i]);
                if (i > 0) rr += fabs(s_ee[i - 1]);
                if (i < p - 1) rr += fabs(s_ee[i]);
                m = rr > m ? rr : m;
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double q = __shfl_xor(m, o, 64);
                m = q > m ? q : m;
            }
            if (lane == 0) s_red[0] = m > 0.0 ? m : 1.0;
        }
        __syncthreads();
        const double gmax = s_red[0];
        const double sc = 1.0 / gmax;
        for (int i = t; i < p; i += NTH) {
            s_ub[i] = s_dd[i] * sc;
            if (i < p - 1) {
                const double es = s_ee[i] * sc;
                s_e2[i] = es * es;
            }
        }
        __syncthreads();
        // Multisection: M lanes per eigenvalue evaluate the Sturm count at M
        // interior points, shrinking the bracket M+1 times per iteration.
        // Only the top r+1 eigenvalues are needed by the solve; all p are
        // computed when requested.
        {
            const int nev = (d.mode & 16) ? p : (r + 1 < p ? r + 1 : p);
            const int M = nev * 64 <= NTH ? 64 : (nev * 16 <= 2 * NTH ? 16 : 4);
            const int iters = M == 64 ? 9 : (M == 16 ? 14 : 24);
            const double inv_m1 = 1.0 / (double)(M + 1);
            const int m = t % M;
            const int nslot = NTH / M;
            for (int g0 = 0; g0 < nev; g0 += nslot) {
                const int g = g0 + t / M;
                if (g < nev) {
                    const int midx = p - 1 - g;        // ascending index of the g-th largest
                    double lo = -1.0 - 1e-12, hi = 1.0 + 1e-12;
                    for (int it = 0; it < iters; ++it) {
                        const double x = lo + (hi - lo) * ((double)(m + 1) * inv_m1);
                        const int cnt = sturm_count<false>(s_ub, s_e2, p, x);
                        const bool below = cnt <= midx;   // x <= lambda
                        double lo_c = below ? x : lo;
                        double hi_c = below ? hi : x;
                        // largest lower and smallest upper end over the M lanes of
                        // the group: quads and rows by DPP, whole waves by readlane
                        group_maxmin(lo_c, hi_c, M);
                        lo = lo_c;
                        hi = hi_c;
                    }
                    if (m == 0) {
                        const double ev = 0.5 * (lo + hi) * gmax;
                        s_ev[g] = ev;
                        if (d.evals) d.evals[g] = ev;
                    }
                }
            }
        }
        __syncthreads();

        // ----------------------------------------------- data-chosen rank
        // (eigenvalues in s_ev, descending).  HySime on the whitened cube:
        // every eigenvalue above twice the noise power n.  SURE: the rank k
        // minimising sum_{j>=k} lambda_j - n p + 2 df(k) (0-based j), df(k) =
        // k (n - p + 1) + k (k - 1) + 2 sum_{i<k<=j} lambda_i / (lambda_i -
        // lambda_j), every eigenvalue known; the cross sums are spread over
        // the threads, one (i, k) pair each.
        if (t == 0) s_rank = r;
        if (d.mode & kModeRankSure) {
            for (int e = t; e < r * r; e += NTH) {
                const int i = e / r, k = e % r + 1;
                double acc = 0.0;
                if (i < k) {
                    const double li = s_ev[i];
                    for (int j = k; j < p; ++j) acc += li / (li - s_ev[j]);
                }
                s_cross[i][k] = acc;
            }
            __syncthreads();
            if (t == 0) {
                const double n = (double)d.n, pp = (double)p;
                double tail = 0.0;                       // sum_{j >= k} lambda_j
                for (int j = r; j < p; ++j) tail += s_ev[j];
                double best = __builtin_inf();
                int bk = 1;
                for (int k = r; k >= 1; --k) {
                    double cr = 0.0;
                    for (int i = 0; i < k; ++i) cr += s_cross[i][k];
                    const double df = k * (n - pp + 1.0) + k * (k - 1.0) + 2.0 * cr;
                    const double sv = tail - n * pp + 2.0 * df;
                    if (sv <= best) {     // descending k: the last minimum is the smallest rank
                        best = sv;
                        bk = k;
                    }
                    tail += s_ev[k - 1];
                }
                s_rank = bk;
            }
        } else if ((d.mode & kModeRankHySime) && t == 0) {
            const double thr = 2.0 * (double)d.n;
            int k = 0;
            while (k < r && s_ev[k] > thr) ++k;
            s_rank = k < 1 ? 1 : k;
        }
        __syncthreads();
        const int kr = s_rank;

        HYRES_STAMP(d, 3);
        // ---------------------------- eigenvectors of the tridiagonal matrix
        // Twisted factorisation at each eigenvalue mu: the top-down pivots D_i
        // (wave 0) and the bottom-up pivots R_i with multipliers U_i (wave 1)
        // run at the same time; the twist index minimises |D_i + R_i - (d_i - mu)|
        // (largest index on ties); then the two halves of the vector are
        // solved from the twist outwards, again on two waves.
        const double pivmin = gmax * 1e-290;
        if (wave == 0 && lane < r) {
            const int g = lane;
            const double mu = s_ev[g];
            double D = s_dd[0] - mu;
#pragma unroll 4
            for (int i = 0; i < p - 1; ++i) {
                if (fabs(D) < pivmin) D = D < 0.0 ? -pivmin : pivmin;
                s_zD[i * kMaxRank + g] = D;
                const double e = s_ee[i];
                D = (s_dd[i + 1] - mu) - e * (e / D);
            }
            if (fabs(D) < pivmin) D = D < 0.0 ? -pivmin : pivmin;
            s_zD[(p - 1) * kMaxRank + g] = D;
        } else if (wave == 1 && lane < r) {
            const int g = lane;
            const double mu = s_ev[g];
            double R = s_dd[p - 1] - mu;
            if (fabs(R) < pivmin) R = R < 0.0 ? -pivmin : pivmin;
            s_z[g][p - 1] = R;
#pragma unroll 4
            for (int i = p - 2; i >= 0; --i) {
                const double e = s_ee[i];
                const double U = e / R;
                s_zU[i * kMaxRank + g] = U;
                R = (s_dd[i] - mu) - U * e;
                if (fabs(R) < pivmin) R = R < 0.0 ? -pivmin : pivmin;
                s_z[g][i] = R;
            }
        }
        __syncthreads();
        // twist index of vector g = wave + NW v: argmin over the lanes of the wave
        int kb_w[VPW];
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            const int g = wave + NW * v;
            kb_w[v] = 0;
            if (g < r) {
                const double mu = s_ev[g];
                double best = __builtin_inf();
                int bi = -1;
                for (int i = lane; i < p; i += 64) {
                    const double gam = fabs(s_zD[i * kMaxRank + g] + s_z[g][i] - (s_dd[i] - mu));
                    if (gam <= best) {           // ascending i: the last minimum is the largest index
                        best = gam;
                        bi = i;
                    }
                }
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    const double ob = __shfl_xor(best, o, 64);
                    const int oi = __shfl_xor(bi, o, 64);
                    if (ob < best || (ob == best && oi > bi)) {
                        best = ob;
                        bi = oi;
                    }
                }
                kb_w[v] = bi;
            }
        }
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                const int g = wave + NW * v;
                if (g < r) s_kb[g] = kb_w[v];
            }
        }
        __syncthreads();
        if (wave == 0 && lane < r) {
            const int g = lane, kb = s_kb[g];
            double z = 1.0;
            s_z[g][kb] = 1.0;
#pragma unroll 4
            for (int i = kb - 1; i >= 0; --i) {
                z = -(s_ee[i] / s_zD[i * kMaxRank + g]) * z;
                s_z[g][i] = z;
            }
        } else if (wave == 1 && lane < r) {
            const int g = lane, kb = s_kb[g];
            double z = 1.0;
#pragma unroll 4
            for (int i = kb; i < p - 1; ++i) {
                z = -s_zU[i * kMaxRank + g] * z;
                s_z[g][i + 1] = z;
            }
        }
        __syncthreads();

        HYRES_STAMP(d, 4);
        // ---- modified Gram-Schmidt; vector g = wave + NW*v stays in registers of its wave
        double zr[VPW][4];
#pragma unroll
        for (int v = 0; v < VPW; ++v) {
            const int g = wave + NW * v;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = lane + 64 * q;
                zr[v][q] = (g < r && i < p) ? s_z[g][i] : 0.0;
            }
        }
        __syncthreads();
        for (int i = 0; i < r; ++i) {
            double* shared_zi = s_col[i & 1];
            if (wave == i % NW) {
#pragma unroll
                for (int v = 0; v < VPW; ++v) {
                    if (v == i / NW) {
                        double s = 0.0;
#pragma unroll
                        for (int q = 0; q < 4; ++q) s = fma(zr[v][q], zr[v][q], s);
                        s = wave_sum(s);
                        const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            zr[v][q] *= inv;
                            shared_zi[lane + 64 * q] = zr[v][q];
                        }
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                const int g = wave + NW * v;
                if (g > i && g < r) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) s = fma(shared_zi[lane + 64 * q], zr[v][q], s);
                    s = wave_sum(s);
#pragma unroll
                    for (int q = 0; q < 4; ++q) zr[v][q] = fma(-s, shared_zi[lane + 64 * q], zr[v][q]);
                }
            }
        }

        HYRES_STAMP(d, 5);
        // -------------------------- back-transformation v = H_0 ... H_{p-3} z
        // Reflectors are staged from global memory into LDS eight at a time by
        // the whole block (coalesced), then applied by the waves owning vectors.
        {
            constexpr int RB = 8;
            constexpr int SPT = (RB * kSmallP + NTH - 1) / NTH;   // staged entries per thread
            double* stage = s_zD;                       // free now: RB x kSmallP doubles
            // the next group's reflectors are read into registers while the
            // current group is applied
            double nxt[SPT];
            auto fetch = [&](int k1) {
                const int k0 = k1 - RB + 1 < 0 ? 0 : k1 - RB + 1;
#pragma unroll
                for (int j = 0; j < SPT; ++j) {
                    const int e = t + j * NTH;
                    const int kk = k1 - e / kSmallP, i = e % kSmallP;
                    nxt[j] = (e < RB * kSmallP && kk >= k0 && i > kk && i < p) ? d.hv[(int64_t)kk * p + i] : 0.0;
                }
            };
            if (p - 3 >= 0) fetch(p - 3);
            for (int k1 = p - 3; k1 >= 0; k1 -= RB) {
                const int k0 = k1 - RB + 1 < 0 ? 0 : k1 - RB + 1;
                __syncthreads();
#pragma unroll
                for (int j = 0; j < SPT; ++j) {
                    const int e = t + j * NTH;
                    if (e < RB * kSmallP) stage[e] = nxt[j];
                }
                __syncthreads();
                if (k1 - RB >= 0) fetch(k1 - RB);
                if (wave < r) {
                    for (int k = k1; k >= k0; --k) {
                        const double* hk = stage + (k1 - k) * kSmallP;
                        double h[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) h[q] = hk[lane + 64 * q];
                        const double hb = s_hb[k];
#pragma unroll
                        for (int v = 0; v < VPW; ++v) {
                            if (wave + NW * v < r) {
                                double sdot = 0.0;
#pragma unroll
                                for (int q = 0; q < 4; ++q) sdot = fma(h[q], zr[v][q], sdot);
                                sdot = wave_sum(sdot) * hb;
#pragma unroll
                                for (int q = 0; q < 4; ++q) zr[v][q] = fma(-sdot, h[q], zr[v][q]);
                            }
                        }
                    }
                }
            }
        }
        HYRES_STAMP(d, 6);
        if (wave < r) {
            // sign rule: the entry of largest magnitude is positive (lowest index on ties)
#pragma unroll
            for (int v = 0; v < VPW; ++v) {
                const int g = wave + NW * v;
                if (g < r) {
                    double bv = -1.0, bs = 1.0;
                    int bi = 0x7fffffff;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int i = lane + 64 * q;
                        if (i < p && fabs(zr[v][q]) > bv) {
                            bv = fabs(zr[v][q]);
                            bi = i;
                            bs = zr[v][q];
                        }
                    }
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) {
                        const double ov = __shfl_xor(bv, o, 64);
                        const int oi = __shfl_xor(bi, o, 64);
                        const double os = __shfl_xor(bs, o, 64);
                        if (ov > bv || (ov == bv && oi < bi)) {
                            bv = ov;
                            bi = oi;
                            bs = os;
                        }
                    }
                    const double sgn = bs < 0.0 ? -1.0 : 1.0;
                    int bad = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int i = lane + 64 * q;
                        if (i < p) {
                            // components beyond the chosen rank are zero
                            const double val = g < kr ? zr[v][q] * sgn : 0.0;
                            bad |= !__builtin_isfinite(val);
                            s_z[g][i] = val;
                            d.V[(int64_t)g * p + i] = val;
                        }
                    }
                    if (__any(bad)) flags |= HYRES_DEV_EIGH_NOCONV;
                }
            }
        }
        __syncthreads();

        // ------------------------------- projection / back-projection matrices
        const int P16 = 16 * d.T;
        for (int e = t; e < P16 * 16; e += NTH) {
            const int i = e >> 4, g = e & 15;
            const bool ok = i < p && g < r;
            const double v = ok ? s_z[g][i] : 0.0;
            const double s = i < p ? s_sig[i] : 1.0;
            d.P32[e] = (float)(v / s);
            d.Q32[(int64_t)g * P16 + i] = (float)(v * s);
            if (ok) {
                d.P64[(int64_t)i * r + g] = v / s;
                d.Q64[(int64_t)g * p + i] = v * s;
            }
        }
        if (d.eig_check) {
            // accuracy of the computed eigenpairs of C = D^-1 G D^-1 (G is intact):
            // ||C V - V Lambda||_F / ||C||_F and max |V^T V - I| over the kr used
            double rs = 0.0, cs = 0.0, os = 0.0;
            for (int e = t; e < p * kr; e += NTH) {
                const int g = e / p, i = e - g * p;
                const double* gi = d.G + (int64_t)i * p;
                const double si = s_sig[i];
                double acc = 0.0;
                for (int j = 0; j < p; ++j) acc = fma(gi[j] / (si * s_sig[j]), s_z[g][j], acc);
                const double res = fma(-s_ev[g], s_z[g][i], acc);
                rs = fma(res, res, rs);
            }
            for (int e = t; e < p * p; e += NTH) {
                const int i = e / p, j = e - i * p;
                const double c = d.G[e] / (s_sig[i] * s_sig[j]);
                cs = fma(c, c, cs);
            }
            for (int e = t; e < kr * kr; e += NTH) {
                const int g = e / kr, k = e - g * kr;
                double dot = 0.0;
                for (int i = 0; i < p; ++i) dot = fma(s_z[g][i], s_z[k][i], dot);
                os = fmax(os, fabs(dot - (g == k ? 1.0 : 0.0)));
            }
            rs = wave_sum(rs);
            cs = wave_sum(cs);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) os = fmax(os, __shfl_xor(os, o, 64));
            if (lane == 0) {
                s_chk[0][wave] = rs;
                s_chk[1][wave] = cs;
                s_chk[2][wave] = os;
            }
            __syncthreads();
            if (t == 0) {
                double a = 0.0, b = 0.0, m = 0.0;
                for (int w = 0; w < NW; ++w) {
                    a += s_chk[0][w];
                    b += s_chk[1][w];
                    m = fmax(m, s_chk[2][w]);
                }
                d.eig_check[0] = b > 0.0 ? sqrt(a / b) : 0.0;
                d.eig_check[1] = m;
            }
        }
        if (t == 0) {
            double gp = __builtin_inf();
            if (kr < p) {
                gp = s_ev[kr - 1] / s_ev[kr];
                if (!(gp >= 1.0 + 1e-6)) flags |= HYRES_DEV_DEGENERATE;
            }
            d.gap[0] = gp;
            if (d.rank_out) *d.rank_out = kr;
        }
    }
    if (flags) atomicOr(&s_flags, flags);
    __syncthreads();
    if (t == 0 && s_flags) set_status(d.status, s_flags);
    HYRES_STAMP(d, 7);
}

// Eigen-adjoint systems (block k < r) and the inverse Gram (block r), one
// workgroup each, by the register sweep above.  For component k the system is
// (lambda_k I - C_perp) y = (I - U U^T) dV_k, C_perp = C - U Lambda U^T with the
// top r eigenpairs (U, Lambda) of C removed: it is symmetric positive
// definite (eigenvalue lambda_k on the top-r directions, lambda_k - lambda_i > 0
// on the others), so the sweep needs no pivoting.  y is the part of the
// eigenvector derivative outside the top-r subspace; inside it the derivative
// is explicit:  w_k = y + sum_{i<r, i!=k} u_i (u_i^T dV_k) / (lambda_k - lambda_i),
// the same w_k as the solution of (lambda_k I - C + lambda_k u_k u_k^T) w =
// (I - u_k u_k^T) dV_k.  dV_k = D^-1 dP_k + D dQ_k.
template <int BR, int BC, int ROWS, int COLS>
__global__ __launch_bounds__(ROWS * COLS) void k_adj_sweep(AdjDesc a) {
    constexpr int NTH = ROWS * COLS;
    constexpr int NW = NTH / 64;
    __shared__ double s_col[2][kSmallP];
    __shared__ double s_col2[2][kSmallP];
    __shared__ double s_diag[kSmallP], s_sig[kSmallP], s_rhs[kSmallP];
    __shared__ double s_u[kMaxRank][kSmallP];
    __shared__ double s_ev[kMaxRank], s_dot[kMaxRank];
    __shared__ double s_part[kSmallP][COLS];          // row partial sums of M^-1 rhs
    const int p = a.p, r = a.r, k = blockIdx.x;
    const int t = threadIdx.x, tc = t % COLS, tr = t / COLS, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    for (int i = t; i < p; i += NTH) s_sig[i] = a.sigma[i];
    for (int e = t; e < r * p; e += NTH) s_u[e / p][e % p] = a.V[e];
    if (t < r) s_ev[t] = a.evals[t];
    __syncthreads();
    const bool eig = k < r;
    const double lk = eig ? s_ev[k] : 0.0;
    if (eig) {
        for (int i = t; i < p; i += NTH) s_rhs[i] = a.dPt[(int64_t)k * p + i] / s_sig[i] + s_sig[i] * a.dQ[(int64_t)k * p + i];
        __syncthreads();
        for (int m = wave; m < r; m += NW) {
            double d = 0.0;
            for (int i = lane; i < p; i += 64) d = fma(s_u[m][i], s_rhs[i], d);
            d = wave_sum(d);
            if (lane == 0) s_dot[m] = d;
        }
        __syncthreads();
        for (int i = t; i < p; i += NTH) {
            double v = s_rhs[i];
            for (int m = 0; m < r; ++m) v = fma(-s_u[m][i], s_dot[m], v);
            s_rhs[i] = v;
            double dg = lk - a.G[(int64_t)i * p + i] / (s_sig[i] * s_sig[i]);
            for (int m = 0; m < r; ++m) dg = fma(s_ev[m] * s_u[m][i], s_u[m][i], dg);
            s_diag[i] = dg;
        }
    } else {
        for (int i = t; i < p; i += NTH) s_diag[i] = a.G[(int64_t)i * p + i];
    }
    double A[BR][BC];
#pragma unroll
    for (int aa = 0; aa < BR; ++aa)
#pragma unroll
        for (int b = 0; b < BC; ++b) {
            const int i = tr + ROWS * aa, j = tc + COLS * b;
            double v = i == j ? 1.0 : 0.0;
            if (i < p && j < p) {
                const double g = a.G[(int64_t)i * p + j];
                if (eig) {
                    v = (i == j ? lk : 0.0) - g / (s_sig[i] * s_sig[j]);
                    for (int m = 0; m < r; ++m) v = fma(s_ev[m] * s_u[m][i], s_u[m][j], v);
                } else {
                    v = g;
                }
            }
            A[aa][b] = v;
        }
    __syncthreads();
    const int flags = gj_sweep<BR, BC, ROWS, COLS>(A, p, tr, tc, s_diag, s_col, s_col2);
    if (flags && t == 0) set_status(a.status, flags);
    if (eig) {
        // y = M^-1 rhs = -A rhs: partial sums over this thread's columns, then rows in column order
#pragma unroll
        for (int aa = 0; aa < BR; ++aa) {
            double part = 0.0;
#pragma unroll
            for (int b = 0; b < BC; ++b) {
                const int j = tc + COLS * b;
                part = fma(A[aa][b], j < p ? s_rhs[j] : 0.0, part);
            }
            s_part[tr + ROWS * aa][tc] = part;
        }
        __syncthreads();
        for (int i = t; i < p; i += NTH) {
            double y = 0.0;
            for (int c = 0; c < COLS; ++c) y -= s_part[i][c];
            for (int m = 0; m < r; ++m)
                if (m != k) y = fma(s_u[m][i], s_dot[m] / (lk - s_ev[m]), y);
            a.Wsol[(int64_t)k * p + i] = y;
        }
    } else {
#pragma unroll
        for (int aa = 0; aa < BR; ++aa)
#pragma unroll
            for (int b = 0; b < BC; ++b) {
                const int i = tr + ROWS * aa, j = tc + COLS * b;
                if (i < p && j < p) a.Ginv[(int64_t)i * p + j] = -A[aa][b];
            }
    }
}

hipError_t launch_adj_sweep(const AdjDesc& a, hipStream_t s) {
    const int p = a.p;
    const dim3 grid(a.r + 1);
#define HYRES_A(BR, BC, RW, CL) hipLaunchKernelGGL((k_adj_sweep<BR, BC, RW, CL>), grid, dim3(RW * CL), 0, s, a)
    if (p <= 32) HYRES_A(2, 2, 16, 16);
    else if (p <= 64) HYRES_A(4, 4, 16, 16);
    else if (p <= 96) HYRES_A(6, 6, 16, 16);
    else if (p <= 128) HYRES_A(8, 8, 16, 16);
    else if (p <= 144) HYRES_A(5, 9, 32, 16);
    else if (p <= 160) HYRES_A(5, 10, 32, 16);
    else if (p <= 176) HYRES_A(11, 6, 16, 32);
    else if (p <= 192) HYRES_A(8, 6, 24, 32);
    else if (p <= 224) HYRES_A(7, 7, 32, 32);
    else return hipErrorInvalidValue;
#undef HYRES_A
    return hipGetLastError();
}

// Kernel variant for p bands: (BR, BC, ROWS).
hipError_t launch_small(int p, const CubeDesc* descs, const int* cubes, int ncls, hipStream_t s) {
#define HYRES_S(BR, BC, RW, CL) \
    hipLaunchKernelGGL((k_small<BR, BC, RW, CL>), dim3(ncls), dim3(RW * CL), 0, s, descs, cubes, ncls)
    if (p <= 32) HYRES_S(2, 2, 16, 16);
    else if (p <= 64) HYRES_S(4, 4, 16, 16);
    else if (p <= 96) HYRES_S(6, 6, 16, 16);
    else if (p <= 128) HYRES_S(8, 8, 16, 16);
    else if (p <= 144) HYRES_S(5, 9, 32, 16);
    else if (p <= 160) HYRES_S(5, 10, 32, 16);
    else if (p <= 176) HYRES_S(11, 6, 16, 32);
    else if (p <= 192) HYRES_S(8, 6, 24, 32);
    else if (p <= 224) HYRES_S(7, 7, 32, 32);
    else return hipErrorInvalidValue;
#undef HYRES_S
    return hipGetLastError();
}

}  // namespace hyres
