// Internal types and device helpers of the HyRes library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "../../include/hyres.h"

namespace hyres {

constexpr int kMaxLevels = 8;
constexpr int kMaxRank = 16;
constexpr int kMaxBands = 224;        // FP64 small solver keeps a 224 x 224 matrix in registers
constexpr int kSureBins = 4096;       // histogram bins per refinement round
constexpr int kSureRoundsF32 = 5;     // 31-bit keys, >= 12 bits resolved per round when narrow
constexpr int kSureRoundsF64 = 10;    // 63-bit keys
constexpr int kGramThreads = 512;
constexpr int kSmallThreads = 1024;
constexpr int kPixTile = 64;          // pixels per projection / back-projection block
constexpr int kRitzGroup = 128;       // projection tiles per first-level Rayleigh-Ritz sum

// Daubechies 4-tap orthonormal scaling filter h = ((1+s3),(3+s3),(3-s3),(1-s3)) / (4 sqrt 2),
// s3 = sqrt 3, and its quadrature mirror g[m] = (-1)^m h[3-m].
constexpr double kH0 = 0.48296291314453416;
constexpr double kH1 = 0.83651630373780794;
constexpr double kH2 = 0.22414386804201339;
constexpr double kH3 = -0.12940952255126037;

// Per-component state of the SURE refinement search.
struct SureState {
    uint64_t klo, khi, width;   // current key range [klo, khi) and bin width
    uint64_t below_cnt;         // number of magnitudes with key < klo
    double below_sum;           // sum of their squares
    double best_s;              // smallest SURE value seen at an exact candidate
    double best_t;              // the candidate attaining it
    uint64_t pad0;
    int round;
    int done;
    int inexact;
    int gather;                 // 1: the next pass collects the values of the surviving bins
    unsigned int nsurv;         // number of values in the surviving bins
    unsigned int pad;
};

constexpr int kSureCap = 8192;        // values finished exactly in one block
constexpr int kSureBinCap = 1024;     // largest surviving bin the exact finish accepts

// CubeDesc::mode bits
constexpr int kModeSigma = 1;      // estimate the noise
constexpr int kModeEigen = 2;      // eigensolve
constexpr int kModeThreshold = 8;  // the inverse transform soft-thresholds its input
constexpr int kModeAllEvals = 16;  // every eigenvalue
constexpr int kModeZeroPad = 32;   // analysis with a zero extra sample (transpose of the inverse)
constexpr int kModeFold = 64;      // synthesis folding the extra sample (transpose of the analysis)
constexpr int kModeRankHySime = 128;   // rank chosen by HySime on the whitened cube
constexpr int kModeRankSure = 256;     // rank chosen by SURE of the truncated whitened cube

// Everything a kernel needs to know about one cube.  Pointers are device pointers.
struct CubeDesc {
    const void* Y;  int64_t pitch, row_pitch;
    void* X;        int64_t xpitch, xrow_pitch;
    int H, W, p, r, L, scope, T, dtype;     // T = ceil(p / 16)
    int64_t n;                              // H * W
    int lh[kMaxLevels + 1], lw[kMaxLevels + 1];  // approximation sizes after l levels (l=0: H, W)
    int64_t loff[kMaxLevels + 1];           // offset of the detail blocks of level l in a coefficient vector
    int64_t ll_off;                         // offset of LL_L
    int64_t nc, ncs;                        // coefficients per component, component stride
    int64_t nz;                             // plane stride of the component images
    int64_t tps, tmp_off2;                  // temp plane stride, offset of the second LL buffer
    // workspace arrays
    void* gpart; int gslot0, gslots;        // Gram partial sums (slots of this cube)
    double* G;                              // p x p band Gram
    double* sigma;                          // p
    const double* sigma_in;                 // optional caller sigma
    double* hv;                             // Householder vectors, p x p
    double* V;                              // p x r column-major
    double* evals;                          // p, descending
    double* gap;                            // 1
    int* rank_out;                          // 1: the rank used (may be null)
    double* eig_check;                      // 2: eigenpair residual and orthonormality (may be null)
    float* P32; float* Q32;                 // (16T x 16) projection and (16 x 16T) back-projection
    double* P64; double* Q64;               // (p x r) and (r x p)
    float* rpart;                           // Rayleigh-Ritz: T^T T per 64-pixel tile, 16 x 16 (mixed solves)
    double* rsum;                           // the tile sums per group of kRitzGroup tiles, FP64
    double* rrot;                           // Rayleigh-Ritz rotation, 16 x 16
    int rgroups;                            // number of tile groups
    void* Z;                                // r x nz component images (also the denoised ones)
    void* coef;                             // r x ncs coefficients
    void* tmp;                              // r x tps approximation buffers
    uint32_t* hcnt; double* hsum; uint64_t* hmin; uint64_t* hmax;  // r x kSureBins
    SureState* sst;                         // r
    uint32_t* sbits;                        // r x kSureBins/32 surviving-bin bitmap
    uint64_t* spre;                         // r x kSureBins: values below each bin (gather round)
    double* sspre;                          // r x kSureBins: their sum of squares
    uint32_t* sctr;                         // r x 4: blocks done in the pass, values gathered, zeros (u64)
    int64_t schunk;                         // coefficients per SURE work item (a multiple of 1024)
    uint64_t* cand;                         // r x kSureCap collected magnitudes (keys)
    double* lambda; double* sure;           // r
    const double* lambda_in;                // optional caller thresholds
    // sliding-window blend in the back-projection (bwy null: plain write).  A
    // tile adds w_y[y] w_x[x] Xhat to X, where w are its 1-D weights divided by
    // the sum over all tiles; the first tile to reach a pixel writes instead.
    // Tiles are applied in passes of non-overlapping tiles; bcy/bcx hold, per
    // row/column of this tile, the bit mask of the pass colours covering it.
    const double* bwy; const double* bwx;
    const unsigned char* bcy; const unsigned char* bcx;
    int bpass, bncx;                        // this tile's pass = colour_y * bncx + colour_x
    int* status;                            // device status word (may be null)
    int mode;                               // kMode* bits
    int vec4;                               // Y is contiguous with 16-byte aligned pixel rows, p % 4 == 0
    int xvec4;                              // the same for X
    int dense;                              // F32 Y, pitch == p, 16-byte aligned: a 64-pixel tile is 64 p consecutive floats
    int xdense;                             // the same for X
    uint32_t pmag;                          // floor(2^32 / p) + 1: e / p == umulhi(e, pmag) for 0 <= e < 64 p
    unsigned long long* dbg;                // phase time stamps (timing builds only; null otherwise)
};

// Per-pixel spectral l1-l1 problem by split Bregman (HyMiNoR's sparse stage).
constexpr int kL1MaxSeg = 64;      // bands of one pixel held by one lane
struct L1Args {
    const void* Hc; int64_t pitch, row_pitch;
    void* X;        int64_t xpitch, xrow_pitch;
    int H, W, p, iters, dtype;
    double lam, mu1, mu2;
};
bool l1l1_shape(int p, int dtype, int* S, int* M);
hipError_t launch_l1l1(const L1Args& a, int num_cu, hipStream_t st);

// FORPDN: one analysis / synthesis level of the wavelet on position-major
// vectors (p bands per position), the per-group threshold choice and the
// spectral smoother.
constexpr int kForpdnMaxGroups = kMaxLevels + 1;
constexpr int kForpdnGrid = 81;    // lam = 10^(t/10), t = -40..40
struct VLevel {
    const void* in; int64_t ip, irow;       // input level (element strides of a position and a row)
    const double* scale;                    // per-band divisor on load (sigma at the first level) or null
    void* ll;                               // LL output, h x w positions, dense
    void* det;                              // LH, HL, HH blocks of h x w positions each
    int Hin, Win, h, w, p;
    uint32_t pmag;                          // floor(2^32 / p) + 1
};
struct VSyn {
    const void* ll; const void* det;        // this level's LL and detail blocks (dense)
    void* out; int64_t op, orow;            // the level below (element strides)
    const double* scale;                    // per-band factor on store (sigma at the last level) or null
    int Hin, Win, h, w, p;
    uint32_t pmag;
};
struct FLambda {
    const double* G[kForpdnMaxGroups];      // p x p band Gram of each group's coefficient vectors
    int64_t count[kForpdnMaxGroups];        // vectors per group
    const double* lambda_in;                // given thresholds or null
    double* lambda; double* sure;           // per group
    int p;
};
struct FFilter {
    void* coef; int64_t npos;               // position-major coefficients (p per position)
    int64_t goff[kForpdnMaxGroups + 1];     // first position of each group
    const double* lambda;
    int p, groups;
    uint32_t pmag;
};
hipError_t launch_vdwt_level(int dtype, const VLevel& a, int num_cu, hipStream_t s);
hipError_t launch_vidwt_level(int dtype, const VSyn& a, int num_cu, hipStream_t s);
hipError_t launch_forpdn_lambda(const FLambda& a, int groups, hipStream_t s);
size_t forpdn_filter_lds(int dtype, int p, int groups);
hipError_t launch_forpdn_filter(int dtype, const FFilter& a, int num_cu, hipStream_t s);

// Tile grid of a sliding-window solve (FP32), for the back-projection that
// blends the tiles in one pass over the output image.
constexpr int kMaxTilesAxis = 64;
struct BlendGrid {
    int ny, nx, th, tw, H, W, p;
    int sy[kMaxTilesAxis], sx[kMaxTilesAxis];   // tile starts along y and x
    void* X; int64_t xpitch, xrow_pitch;        // the output image
};

// Everything the adjoint kernels need (one cube; passed by value).
struct AdjDesc {
    int H, W, p, r, L, scope;
    int64_t n, nz, ncs, nc, ll_off;
    const void* Y; int64_t pitch, row_pitch;
    const void* Zh;          // forward reconstructed component images (r x nz)
    const void* B;           // forward coefficients (r x ncs)
    const double* G;         // p x p
    const double* sigma;     // p
    const double* V;         // p x r, column-major
    const double* evals;     // top r eigenvalues of C
    const double* lambda;    // r thresholds
    const double* P64;       // p x r, [b * r + k]
    const double* Q64;       // r x p, [k * p + b]
    const void* dX; int64_t dxp, dxrp;
    void* dY; int64_t dyp, dyrp;
    double* dlambda;         // r (may be null)
    void* A;                 // r x nz: dZh, later dZ
    void* dB;                // r x ncs
    double* part;            // slots x r x p
    double* dQ;              // r x p
    double* dPt;             // r x p (dP transposed)
    double* lpart;           // r x nchunk
    double* Wsol;            // p x r, column-major
    double* Ginv;            // p x p
    double* dC;              // p x p
    double* dG2;             // p x p: 2 dG
    double* gsc;             // p: n sigma_j^3 dsigma_j / 2
    int slots, nchunk;
    int* status;
};
hipError_t launch_adj_sweep(const AdjDesc& a, hipStream_t s);
hipError_t launch_planes_cube(int dtype, const AdjDesc& a, const void* planes, const void* cube, int64_t cp,
                              int64_t crp, double* out, hipStream_t s);
hipError_t launch_polar(const CubeDesc* descs, const double* M, hipStream_t s);

#ifdef HYRES_PHASE_TIMING
#define HYRES_STAMP(d, i) \
    do { if (threadIdx.x == 0 && (d).dbg) (d).dbg[i] = __builtin_amdgcn_s_memrealtime(); } while (0)
#else
#define HYRES_STAMP(d, i) do { } while (0)
#endif

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// index of the cube owning flattened work item `item` (offsets[0..ncubes])
__device__ __forceinline__ int find_cube(const int* __restrict__ off, int ncubes, int item) {
    int lo = 0, hi = ncubes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1.
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// DPP move of a double (both halves) with a row-level permutation (quad_perm,
// row_half_mirror, row_mirror): every lane has a source, so no old value is
// needed (no zero-initialised destination).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    static_assert(CTRL <= 0xFF || CTRL == 0x140 || CTRL == 0x141, "permutation controls only");
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
// DPP row shift of a double: lanes without a source read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_shift_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
// Sum over the 16 lanes of each DPP row, returned to every lane of the row:
// quad_perm xor 1, quad_perm xor 2, row_half_mirror, row_mirror.
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return v;
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
// Sum over each half-wave (32 lanes), returned to every lane of the half: the
// four row sums are read into scalar registers (no LDS round trip).  Call with
// the whole wave active.
__device__ __forceinline__ double half_sum(double v) {
    v = row16_sum(v);
    const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
    const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
    return (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
}
// Sum over the wave, returned to every lane ((r0 + r1) + (r2 + r3) of the row sums).
__device__ __forceinline__ double wave_sum(double v) {
    v = row16_sum(v);
    const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
    const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
    return (r0 + r1) + (r2 + r3);
}

// Blend weight of tile pixel (y, x) and whether an earlier pass already wrote it.
__device__ __forceinline__ double blend_weight(const CubeDesc& d, int64_t y, int64_t x, bool* first) {
    const unsigned my = d.bcy[y], mx = d.bcx[x];
    bool before = false;
    for (int k = 0; k < d.bpass; ++k) {
        const int cy = k / d.bncx, cx = k - cy * d.bncx;
        before |= ((my >> cy) & (mx >> cx) & 1u) != 0;
    }
    *first = !before;
    return d.bwy[y] * d.bwx[x];
}

__device__ __forceinline__ void set_status(int* st, int bits) {
    if (st && bits) atomicOr(st, bits);
}

// Load paths of the kernels that stream Y in 64-pixel tiles: 16-byte pixel
// vectors (kVec), unpadded pixels whose tile is 64 p consecutive floats
// (kDense: loads across pixel boundaries), any other layout (kScalar).
constexpr int kVec = 0, kDense = 1, kScalar = 2;
constexpr int kAnyLayout = 3;      // a launch whose cubes take different paths (chosen per cube)

// Global-memory views of device pointers.  A pointer read from a descriptor in
// memory is generic to the compiler, and generic accesses compile to FLAT
// instructions, which count against the LDS wait counter as well: every wait
// for an LDS read then also waits for the global loads in flight (a tile
// prefetched during the matrix work stalls it).  Accesses through a pointer
// derived from gmem() (with arithmetic on it, or kept in its own type) are
// global_* instructions.  The address-space qualifier exists in the device
// pass only; the host pass sees plain pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define HYRES_GLOBAL __attribute__((address_space(1)))
#else
#define HYRES_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ HYRES_GLOBAL T* gmem(T* p) { return (HYRES_GLOBAL T*)p; }

// An FP32 cube as the 64-pixel tile loaders see it (a CubeDesc carries the
// same fields under the same names): pixel q = y W + x at Y + y row_pitch +
// x pitch, flags as in CubeDesc.
struct CubeView {
    const void* Y; int64_t pitch, row_pitch;
    int64_t n; int W, p;
    int vec4, dense;
    uint32_t pmag;
};
// The view of an FP32 cube with its load-path flags (host).
CubeView cube_view(const void* Y, int W, int p, int64_t n, int64_t pitch, int64_t row_pitch, int dtype);
template <typename D>
__device__ __forceinline__ int load_mode(const D& d) { return d.vec4 ? kVec : d.dense ? kDense : kScalar; }

// e / p for 0 <= e < 64 p (exact while e p < 2^32) with the per-cube multiplier
__device__ __forceinline__ int div_p(int e, uint32_t pmag) { return (int)__umulhi((uint32_t)e, pmag); }

template <typename T, typename D>
__device__ __forceinline__ const T* pixel_ptr(const D& d, int64_t q) {
    int64_t y = q / d.W, x = q - y * d.W;
    return gmem(static_cast<const T*>(d.Y)) + y * d.row_pitch + x * d.pitch;
}

}  // namespace hyres
