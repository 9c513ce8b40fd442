// Rayleigh-Ritz refinement of the subspace (mixed-precision solves).
//
// In the mixed solve the eigenvectors V0 come from a band Gram built from
// split-BF16 products.  The projection then computes T = Y D^-1 V0 from the
// FP32 cube, so M = T^T T = V0^T C V0 holds C to FP32-product accuracy.  Its
// FP64 eigendecomposition M = U Lambda U^T gives the Ritz pairs inside
// span(V0): V = V0 U (sign rule re-applied), Z = T U, and Lambda, the top
// eigenvalues at FP32 accuracy.  This is the one FP32 pass that recovers what
// the BF16 products lose in the orientation of the basis and the eigenvalues.
//
//   (k_project_f32 writes T^T T of every 64-pixel tile, FP32, from its MFMA
//    accumulators)
//   k_ritz_reduce  FP64 sums over groups of tiles (tile order, no atomics)
//   k_ritz         one workgroup per cube: group sums in FP64, cyclic Jacobi
//                  (parallel pair ordering), sort, sign rule, new V, evals,
//                  projection matrices and the r x r rotation
//   (the first analysis level applies Z <- Z R as it loads Z)
#include "hyres_internal.hpp"

namespace hyres {

// The r x r entries (a, b) of the tile products that the refinement reads,
// spread over the 256 threads of a block: thread t takes entry t % E of part
// t / E (E = r r, P = 256 / E parts).  Part k sums the items k, k + P, ... of
// a range in order; the parts are then added in order (a fixed order for a
// given rank, whatever the grid).
__device__ __forceinline__ double ritz_part_sum(const float* __restrict__ src, int64_t i0, int64_t i1, int P,
                                                int part) {
    double s = 0.0;
    int64_t i = i0 + part;
    for (; i + 31 * (int64_t)P < i1; i += 32 * (int64_t)P) {
        float v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = src[(i + u * (int64_t)P) * 256];
#pragma unroll
        for (int u = 0; u < 32; ++u) s += (double)v[u];
    }
    for (; i < i1; i += P) s += (double)src[i * 256];
    return s;
}

// rsum[g][a * 16 + b] = sum over the tiles of group g of the FP32 tile
// products (FP64; the parts of the block in order).
__global__ __launch_bounds__(256) void k_ritz_reduce(const CubeDesc* __restrict__ descs,
                                                     const int* __restrict__ items, int ncubes) {
    __shared__ double part_s[256];
    const int total = items[ncubes];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int c = find_cube(items, ncubes, item);
        const CubeDesc& d = descs[c];
        const int g = item - items[c];
        const int r = d.r, E = r * r, P = 256 / E;
        const int64_t ntiles = (d.n + kPixTile - 1) / kPixTile;
        const int64_t t0 = (int64_t)g * kRitzGroup;
        const int64_t t1 = t0 + kRitzGroup < ntiles ? t0 + kRitzGroup : ntiles;
        const int t = threadIdx.x, e = t % E, pt = t / E;
        const int a = e / r, b = e - a * r;
        __syncthreads();
        part_s[t] = pt < P ? ritz_part_sum(gmem(d.rpart) + a * 16 + b, t0, t1, P, pt) : 0.0;
        __syncthreads();
        if (t < E) {
            double s = part_s[t];
            for (int k = 1; k < P; ++k) s += part_s[t + k * E];
            gmem(d.rsum)[(int64_t)g * 256 + a * 16 + b] = s;
        }
    }
}

// Partner of index x (0..m-1, m even) in round t of the circle schedule: every
// pair meets once in m - 1 rounds.
__device__ __forceinline__ int ritz_partner(int x, int t, int m) {
    const int n = m - 1;
    if (x == 0) return t + 1;
    int y = (2 * (t + 1) - x) % n;
    y = y < 0 ? y + n : y;
    y = y == 0 ? n : y;
    return y == x ? 0 : y;
}

// The rotation of pair (x, y) that zeroes M[x][y]: c, and s signed as
// J[y][x], stored by index x.  t = sgn(tau) / (|tau| + sqrt(1 + tau^2)),
// tau = dd / hh, is written without the quotient tau: one square root, one
// division and one reciprocal square root on the chain instead of two square
// roots and three divisions.
__device__ __forceinline__ void jacobi_params(const double (*M)[17], int x, int y, double* cs, double* sn) {
    const int lo = x < y ? x : y, hi = x < y ? y : x;
    double c = 1.0, s = 0.0;
    const double apq = M[lo][hi];
    if (apq != 0.0) {
        const double dd = M[hi][hi] - M[lo][lo], hh = 2.0 * apq;
        const double sg = (dd == 0.0 || (dd > 0.0) == (hh > 0.0)) ? 1.0 : -1.0;
        const double tt = sg * fabs(hh) / (fabs(dd) + sqrt(fma(dd, dd, hh * hh)));
        c = rsqrt(fma(tt, tt, 1.0));
        s = tt * c;
    }
    cs[x] = c;
    sn[x] = x == lo ? -s : s;
}

// Cyclic Jacobi on the symmetric m x m matrix Mb[0] (m even, at most 16;
// Ub[0] the identity): the pairs of each round come from the circle schedule,
// every rotation of a round is applied at once, and the two buffers
// alternate.  Returns the buffer holding the diagonalised matrix and the
// accumulated rotations.  Called by all 256 threads of the block
// (thread (i, j) = (tid / 16, tid % 16)).
__device__ __forceinline__ int jacobi16(double (*Mb)[16][17], double (*Ub)[16][17], double* cs, double* sn, int m, double* s_off,
                        double* s_diag) {
    const int tid = threadIdx.x, i = tid >> 4, j = tid & 15;
    int cb = 0;
    for (int sweep = 0; sweep < 12 && m > 1; ++sweep) {
        const double (*M)[17] = Mb[cb];
        if (tid < 64) {
            double off = 0.0, dg = 0.0;
            for (int e = tid; e < 256; e += 64) {
                const int a = e >> 4, b = e & 15;
                if (a < m && b < m) {
                    if (a == b) dg += M[a][a] * M[a][a];
                    else off += M[a][b] * M[a][b];
                }
            }
            off = wave_sum(off);
            dg = wave_sum(dg);
            if (tid == 0) {
                *s_off = off;
                *s_diag = dg;
            }
        }
        __syncthreads();
        if (!(*s_off > 1e-26 * *s_diag)) break;     // off-diagonal below 1e-13 of the diagonal
        for (int t = 0; t < m - 1; ++t) {
            const double (*M)[17] = Mb[cb];
            const double (*U)[17] = Ub[cb];
            // rotation of every pair (x, y), x < y: [c s; -s c] diagonalises the 2 x 2 block
            if (tid < m) {
                const int x = tid, y = ritz_partner(x, t, m);
                jacobi_params(M, x, y, cs, sn);
            }
            __syncthreads();
            // the rotated matrices go to the other buffer: no barrier between reads and writes
            if (i < m && j < m) {
                const int pi = ritz_partner(i, t, m), pj = ritz_partner(j, t, m);
                const double ci = cs[i], si = sn[i], cj = cs[j], sj = sn[j];
                Mb[cb ^ 1][i][j] = ci * (M[i][j] * cj + M[i][pj] * sj) + si * (M[pi][j] * cj + M[pi][pj] * sj);
                Ub[cb ^ 1][i][j] = U[i][j] * cj + U[i][pj] * sj;
            } else {
                Mb[cb ^ 1][i][j] = M[i][j];
                Ub[cb ^ 1][i][j] = U[i][j];
            }
            cb ^= 1;
            __syncthreads();
        }
    }
    return cb;
}

// LDS written by some lanes of a wave, then read by others of the same wave:
// the wave's LDS operations are done in order; this keeps the compiler from
// moving them across (no barrier of the block).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// jacobi16 for m <= 8, run by the first wave alone (lane (i, j) = (lane / 8,
// lane % 8) owns entry (i, j) of the m x m block, the only part read
// afterwards): the same rounds and arithmetic, its steps passed through LDS
// within the wave instead of through block barriers.
__device__ int jacobi8_wave(double (*Mb)[16][17], double (*Ub)[16][17], double* cs, double* sn, int m) {
    const int lane = threadIdx.x & 63, i = lane >> 3, j = lane & 7;
    const bool in = i < m && j < m;
    int cb = 0;
    for (int sweep = 0; sweep < 12 && m > 1; ++sweep) {
        const double v = Mb[cb][i][j];
        const double off = wave_sum(in && i != j ? v * v : 0.0);
        const double dg = wave_sum(in && i == j ? v * v : 0.0);
        if (!(off > 1e-26 * dg)) break;
        for (int t = 0; t < m - 1; ++t) {
            const double (*M)[17] = Mb[cb];
            const double (*U)[17] = Ub[cb];
            if (lane < m) jacobi_params(M, lane, ritz_partner(lane, t, m), cs, sn);
            wave_lds_sync();
            if (in) {
                const int pi = ritz_partner(i, t, m), pj = ritz_partner(j, t, m);
                const double ci = cs[i], si = sn[i], cj = cs[j], sj = sn[j];
                Mb[cb ^ 1][i][j] = ci * (M[i][j] * cj + M[i][pj] * sj) + si * (M[pi][j] * cj + M[pi][pj] * sj);
                Ub[cb ^ 1][i][j] = U[i][j] * cj + U[i][pj] * sj;
            }
            cb ^= 1;
            wave_lds_sync();
        }
    }
    return cb;
}

// jacobi16 or, for m <= 8, jacobi8_wave in the first wave; called by every
// thread of the block, returns the buffer index to all.
__device__ __forceinline__ int jacobi_any(double (*Mb)[16][17], double (*Ub)[16][17], double* cs, double* sn, int m,
                                          double* s_off, double* s_diag, int* s_cb) {
    if (m > 8) return jacobi16(Mb, Ub, cs, sn, m, s_off, s_diag);
    if (threadIdx.x < 64) {
        const int cb = jacobi8_wave(Mb, Ub, cs, sn, m);
        if (threadIdx.x == 0) *s_cb = cb;
    }
    __syncthreads();
    return *s_cb;
}

__global__ __launch_bounds__(256) void k_ritz(const CubeDesc* __restrict__ descs, const int* __restrict__ cubes,
                                              int ncls) {
    __shared__ double Mb[2][16][17], Ub[2][16][17];   // Jacobi rounds alternate between the two
    __shared__ double cs[16], sn[16];
    __shared__ double v0[kMaxBands][kMaxRank];
    __shared__ int perm[16];
    __shared__ double sgn[16];
    __shared__ double s_off, s_diag;
    __shared__ int s_cb;
    __shared__ double s_part[256];
    __shared__ double s_sig[kMaxBands];           // the noise, read once (the output loop stores to global memory)
    const int cube = cubes[blockIdx.x];
    const CubeDesc& d = descs[cube];
    const int r = d.r, p = d.p, tid = threadIdx.x;
    const int i = tid >> 4, j = tid & 15;
    const int m = (r + 1) & ~1;                   // even size; a padding index stays decoupled
    // M from the group sums: thread (entry tid % E, part tid / E) sums the
    // groups part, part + P, ... in order, the parts are added in order, and
    // the upper entry is mirrored (M exactly symmetric)
    {
        const int E = r * r, P = 256 / E;
        const int e = tid % E, pt = tid / E;
        const int a = e / r, b = e - a * r;
        double s = 0.0;
        if (pt < P) {
            const double* src = gmem(d.rsum) + a * 16 + b;
            int k = pt;
            for (; k + 15 * P < d.rgroups; k += 16 * P) {
                double v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = src[(int64_t)(k + u * P) * 256];
#pragma unroll
                for (int u = 0; u < 16; ++u) s += v[u];
            }
            for (; k < d.rgroups; k += P) s += src[(int64_t)k * 256];
        }
        s_part[tid] = s;
        __syncthreads();
        const int ai = i <= j ? i : j, bj = i <= j ? j : i;
        double m = 0.0;
        if (ai < r && bj < r) {
            const int eu = ai * r + bj;
            m = s_part[eu];
            for (int k = 1; k < P; ++k) m += s_part[eu + k * E];
        }
        Mb[0][i][j] = m;
        Ub[0][i][j] = i == j ? 1.0 : 0.0;
    }
    for (int e = tid; e < p * r; e += 256) {
        const int row = e / r, k = e - row * r;
        v0[row][k] = d.V[(int64_t)k * p + row];
    }
    for (int b = tid; b < p; b += 256) s_sig[b] = d.sigma[b];
    __syncthreads();
    const int cb = jacobi_any(Mb, Ub, cs, sn, m, &s_off, &s_diag, &s_cb);
    const double (*M)[17] = Mb[cb];
    const double (*U)[17] = Ub[cb];
    // descending order of the Ritz values (ties: lower index first)
    if (tid < r) {
        int rank = 0;
        for (int k = 0; k < r; ++k)
            if (M[k][k] > M[tid][tid] || (M[k][k] == M[tid][tid] && k < tid)) ++rank;
        perm[rank] = tid;
    }
    __syncthreads();
    // sign rule on V = V0 U: the largest-magnitude entry positive (lowest index on ties)
    for (int k = tid >> 6; k < r; k += 4) {
        const int lane = tid & 63, col = perm[k];
        double best = -1.0, bv = 0.0;
        int bi = p;
        for (int row = lane; row < p; row += 64) {
            double v = 0.0;
            for (int jj = 0; jj < r; ++jj) v = fma(v0[row][jj], U[jj][col], v);
            if (fabs(v) > best) {
                best = fabs(v);
                bi = row;
                bv = v;
            }
        }
        for (int o = 32; o >= 1; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64), ov = __shfl_xor(bv, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
                bv = ov;
            }
        }
        if (lane == 0) sgn[k] = bv < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    // outputs: rotation, V, projection matrices, Ritz values
    if (i < 16 && j < 16) d.rrot[i * 16 + j] = (i < r && j < r) ? U[i][perm[j]] * sgn[j] : 0.0;
    const int P16 = 16 * d.T;
    for (int e = tid; e < p * r; e += 256) {
        const int row = e / r, k = e - row * r;
        const int col = perm[k];
        double v = 0.0;
        for (int jj = 0; jj < r; ++jj) v = fma(v0[row][jj], U[jj][col], v);
        v *= sgn[k];
        const double s = s_sig[row];
        d.V[(int64_t)k * p + row] = v;
        d.P64[(int64_t)row * r + k] = v / s;
        d.Q64[(int64_t)k * p + row] = v * s;
        d.Q32[(int64_t)k * P16 + row] = (float)(v * s);
    }
    if (tid < r && d.evals) d.evals[tid] = M[perm[tid]][perm[tid]];
    __syncthreads();
    if (tid == 0 && d.evals && r < p) {
        const double gp = d.evals[r - 1] / d.evals[r];
        d.gap[0] = gp;
        if (!(gp >= 1.0 + 1e-6)) set_status(d.status, HYRES_DEV_DEGENERATE);
    }
}

// WSRRR's Procrustes step: the orthonormal factor of the polar decomposition
// of Mw = D^-1 (Y^T Zh) (p x r; M holds Y^T Zh transposed, r x p), V = Mw
// (Mw^T Mw)^-1/2 from the Jacobi eigendecomposition of the r x r matrix
// Mw^T Mw, over the components whose column of Mw is not zero (squared norm
// above 1e-24 of the largest).  A zero column (a component thresholded to
// zero) leaves its direction free: it keeps the previous one, orthonormalised
// against the other columns in index order.  Written as the cube's subspace
// with its projection and back-projection matrices.
__global__ __launch_bounds__(256) void k_polar(const CubeDesc* __restrict__ descs, const double* __restrict__ M) {
    __shared__ double Mb[2][16][17], Ub[2][16][17];
    __shared__ double cs[16], sn[16];
    __shared__ double mw[kMaxBands][kMaxRank], vold[kMaxBands][kMaxRank], vnew[kMaxBands][kMaxRank];
    __shared__ double S[16][17];
    __shared__ double s_sig[kMaxBands];           // the noise, read once (the output loop stores to global memory)
    __shared__ double s_off, s_diag, s_nmax;
    __shared__ int s_cb;
    __shared__ int live[16];
    const CubeDesc& d = descs[0];
    const int r = d.r, p = d.p, tid = threadIdx.x, i = tid >> 4, j = tid & 15, lane = tid & 63;
    const int m = (r + 1) & ~1;
    for (int b = tid; b < p; b += 256) s_sig[b] = d.sigma[b];
    __syncthreads();
    for (int e = tid; e < r * p; e += 256) {
        const int k = e / p, b = e - k * p;
        mw[b][k] = M[e] / s_sig[b];
        vold[b][k] = d.V[e];
    }
    __syncthreads();
    double g = 0.0;
    if (i < r && j < r)
        for (int b = 0; b < p; ++b) g = fma(mw[b][i], mw[b][j], g);
    Mb[0][i][j] = g;
    Ub[0][i][j] = i == j ? 1.0 : 0.0;
    __syncthreads();
    if (tid == 0) {
        double mx = 0.0;
        for (int k = 0; k < r; ++k) mx = fmax(mx, Mb[0][k][k]);
        s_nmax = mx;
    }
    __syncthreads();
    if (tid < 16) live[tid] = tid < r && Mb[0][tid][tid] > 1e-24 * s_nmax;
    __syncthreads();
    if (!(live[i] && live[j])) Mb[0][i][j] = 0.0;      // the zero components stay decoupled
    __syncthreads();
    const int cb = jacobi_any(Mb, Ub, cs, sn, m, &s_off, &s_diag, &s_cb);
    double sv = 0.0;
    if (i < r && j < r)
        for (int k = 0; k < r; ++k)
            if (live[k]) sv += Ub[cb][i][k] * Ub[cb][j][k] / sqrt(Mb[cb][k][k]);
    S[i][j] = sv;
    __syncthreads();
    for (int e = tid; e < p * r; e += 256) {
        const int row = e / r, k = e - row * r;
        double v = 0.0;
        if (live[k])
            for (int jj = 0; jj < r; ++jj) v = fma(mw[row][jj], S[jj][k], v);
        vnew[row][k] = v;
    }
    __syncthreads();
    // free columns, in index order, by one wave
    if (tid < 64) {
        for (int k = 0; k < r; ++k) {
            if (live[k]) continue;
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = lane + 64 * q < p ? vold[lane + 64 * q][k] : 0.0;
            for (int jj = 0; jj < r; ++jj) {
                if (!(live[jj] || jj < k)) continue;
                double dt = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (lane + 64 * q < p) dt = fma(vnew[lane + 64 * q][jj], v[q], dt);
                dt = wave_sum(dt);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (lane + 64 * q < p) v[q] = fma(-dt, vnew[lane + 64 * q][jj], v[q]);
            }
            double nn = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) nn = fma(v[q], v[q], nn);
            nn = wave_sum(nn);
            const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (lane + 64 * q < p) vnew[lane + 64 * q][k] = v[q] * inv;
        }
    }
    __syncthreads();
    const int P16 = 16 * d.T;
    for (int e = tid; e < P16 * 16; e += 256) {
        const int row = e >> 4, k = e & 15;
        const bool ok = row < p && k < r;
        const double v = ok ? vnew[row][k] : 0.0;
        const double sg = row < p ? s_sig[row] : 1.0;
        d.P32[e] = (float)(v / sg);
        d.Q32[(int64_t)k * P16 + row] = (float)(v * sg);
        if (ok) {
            d.V[(int64_t)k * p + row] = v;
            d.P64[(int64_t)row * r + k] = v / sg;
            d.Q64[(int64_t)k * p + row] = v * sg;
        }
    }
}

hipError_t launch_polar(const CubeDesc* descs, const double* M, hipStream_t s) {
    hipLaunchKernelGGL(k_polar, dim3(1), dim3(256), 0, s, descs, M);
    return hipGetLastError();
}

hipError_t launch_ritz(const CubeDesc* descs, const int* group_items, const int* cube_list, int ncls, int ncubes,
                       int grid_sum, hipStream_t s) {
    hipLaunchKernelGGL(k_ritz_reduce, dim3(grid_sum), dim3(256), 0, s, descs, group_items, ncubes);
    hipLaunchKernelGGL(k_ritz, dim3(ncls), dim3(256), 0, s, descs, cube_list, ncls);
    return hipGetLastError();
}

}  // namespace hyres
