// Host side of the C ABI: validation, workspace planning and the launch
// sequence of each entry point.  No call allocates device memory or waits on
// the host (hyres_autotune aside); cube descriptors and work-item tables are
// written into the caller's workspace by a small kernel that receives them by
// value, so every sequence can be captured in a HIP graph.
//
// Every entry point goes through one executor: a list of cubes (one for the
// single-cube calls, many for a batch), their workspace plans and descriptors,
// and a launch program.  Each launch of the program covers every cube of one
// kernel class (the kernels that are specialised on the band count) with a
// prefix-summed work-item table over the whole cube list, in which cubes
// outside the class own no items; the kernels are persistent over that table.
#include <algorithm>
#include <cmath>
#include <functional>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hyres_internal.hpp"

#define HYRES_API extern "C" __attribute__((visibility("default")))

namespace hyres {
hipError_t launch_gram_f32(int T, int lm, const CubeDesc*, const int*, int, int, hipStream_t, bool wide);
hipError_t launch_gram_bf16(int T, int lm, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_gram_reduce_f32(int T, const CubeDesc*, const int*, int, hipStream_t);
hipError_t launch_gram_f64(const CubeDesc*, int, int, int, hipStream_t);
hipError_t launch_small(int p, const CubeDesc*, const int*, int, hipStream_t);
hipError_t launch_project_f32(int T, int lm, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_backproject_f32(int T, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_blend_f32(int T, const CubeDesc*, const BlendGrid&, int, hipStream_t);
hipError_t launch_project_f64(const CubeDesc*, int, int64_t, hipStream_t);
hipError_t launch_backproject_f64(const CubeDesc*, int, int64_t, hipStream_t);
hipError_t launch_dwt_level1_rot(int tx, int ty, const CubeDesc*, const int*, int, int, int, hipStream_t);
hipError_t launch_dwt_level(int dtype, int tx, int ty, bool inverse, const CubeDesc*, const int*, int, int,
                            int, hipStream_t);
hipError_t launch_sure_init(int dtype, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_sure_round(int dtype, const CubeDesc*, const int*, int, int, hipStream_t);
int sure_rounds(int dtype);
int64_t sure_chunk_for(int64_t total_coef, int num_cu);
hipError_t launch_ritz(const CubeDesc*, const int*, const int*, int, int, int, hipStream_t);
hipError_t launch_adjoint_pre(const AdjDesc&, int dtype, hipStream_t);
hipError_t launch_adjoint_thresh(const AdjDesc&, int dtype, hipStream_t);
hipError_t launch_adjoint_post(const AdjDesc&, int dtype, hipStream_t);
hipError_t launch_sure_grad(int dtype, const void* coef, int64_t stride, int64_t N, int batch, const double* lambda,
                            double* part, int nchunk, double* out, hipStream_t);
int adj_chunk();
}  // namespace hyres

using namespace hyres;

namespace {
// DWT tile shapes (threads along x, along y) the autotuner chooses among; the
// kernels are instantiated for exactly these.
constexpr int kTileCands = 4;
constexpr int kTileTX[kTileCands] = {64, 32, 16, 128};
constexpr int kTileTY[kTileCands] = {4, 8, 16, 2};
constexpr int kWidthClasses = 16;   // class of a level width w: ceil(log2 w), capped

int width_class(int w) {
    int b = 0;
    while ((1 << b) < w && b < kWidthClasses - 1) ++b;
    return b;
}

// Untuned choice: the widest tile that a level of this width fills.
int default_tile(int wclass) { return wclass <= 4 ? 2 : (wclass == 5 ? 1 : 0); }
}  // namespace

struct hyres_handle {
    int device;
    int num_cu;
    std::string arch;              // device key of the tuning cache
    unsigned prof_mask;
    struct Rec { int stage; hipEvent_t a, b; unsigned run; };
    unsigned runs = 0;             // programs run so far (a stage's records of one run count once)
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    // DWT tile choice per [dtype][inverse][width class], and whether it was tuned
    unsigned char tile[2][2][kWidthClasses];
    unsigned char tuned[2][2][kWidthClasses];
    float tile_us[2][2][kWidthClasses];
    // side streams (default priority) on which the small solves of different
    // band-count classes run beside each other, with their fork/join events
    static constexpr int kSide = 8;
    hipStream_t side[kSide];
    hipEvent_t fork, join[kSide];
    hipEvent_t chain[kSide];       // end of a cube group's Gram stage (groups of a batch or tile grid)
    void* scratch = nullptr;       // device address of this device's no-allocation scratch array
};

// Scratch of hyres_denoise_noalloc: a file-scope array that every device
// holds its own copy of from code-object load to process end.  In host code the
// name `scratch` is only a host-side stand-in; kernels get the device address
// that hipGetSymbolAddress gives with the device current (scratch_address).
static __device__ __align__(256) unsigned char scratch[HYRES_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];      // resolved device address per device (null: not yet)

// The device address of `scratch` on `device`, which must be current.
// Resolved once per device and kept.
hipError_t scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

hipEvent_t prof_event(hyres_handle* h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around one stage when that stage is profiled.
struct StageTimer {
    hyres_handle* h;
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(hyres_handle* h_, hipStream_t s_, int st) : h(h_), s(s_), stage(st) {
        if (h->prof_mask & (1u << stage)) {
            a = prof_event(h);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~StageTimer() {
        if (a) {
            hipEvent_t b = prof_event(h);
            if (b) {
                (void)hipEventRecord(b, s);
                h->pending.push_back({stage, a, b, h->runs});
            } else {
                h->pool.push_back(a);
            }
        }
    }
};

constexpr size_t kAlign = 256;
constexpr int kUploadBytes = 3072;

struct UploadChunk {
    int nbytes;
    int pad;
    int64_t offset;
    unsigned char data[kUploadBytes];
};

__global__ void k_upload(UploadChunk c, unsigned char* base) {
    for (int i = threadIdx.x; i < c.nbytes; i += blockDim.x) base[c.offset + i] = c.data[i];
}

__global__ void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t upload(void* ws, size_t offset, const void* src, size_t bytes, hipStream_t s) {
    const unsigned char* p = static_cast<const unsigned char*>(src);
    for (size_t done = 0; done < bytes; done += kUploadBytes) {
        UploadChunk c;
        c.nbytes = (int)std::min<size_t>(kUploadBytes, bytes - done);
        c.pad = 0;
        c.offset = (int64_t)(offset + done);
        std::memcpy(c.data, p + done, c.nbytes);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, c, static_cast<unsigned char*>(ws));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

struct Layout {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t o = (total + kAlign - 1) / kAlign * kAlign;
        total = o + bytes;
        return o;
    }
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Geometry and workspace layout of one cube.
struct CubePlan {
    int H = 0, W = 0, p = 0, r = 0, L = 0, dtype = 0, scope = 0, T = 0, gslots = 1, precision = 0;
    int64_t n = 0, nz = 0, nc = 0, ncs = 0, tps = 0, tmp_off2 = 0, ll_off = 0;
    int lh[kMaxLevels + 1] = {0}, lw[kMaxLevels + 1] = {0};
    int64_t loff[kMaxLevels + 1] = {0};
    size_t o_gpart = 0, o_G = 0, o_sigma = 0, o_hv = 0, o_V = 0, o_evals = 0, o_gap = 0, o_P32 = 0, o_Q32 = 0,
           o_P64 = 0, o_Q64 = 0, o_Z = 0, o_coef = 0, o_tmp = 0, o_hcnt = 0, o_hsum = 0, o_hmin = 0,
           o_hmax = 0, o_sst = 0, o_lambda = 0, o_sure = 0, o_sbits = 0, o_spre = 0, o_sspre = 0, o_sctr = 0,
           o_cand = 0, o_rpart = 0, o_rsum = 0, o_rrot = 0;
    int rgroups = 0;
    bool has_lambda = false;   // thresholds given by the caller: no SURE search
};

int esize(int dtype) { return dtype == HYRES_F64 ? 8 : 4; }

bool level_geometry(int H, int W, int L, int* lh, int* lw, int64_t* loff, int64_t* ll_off, int64_t* nc) {
    if (H < 1 || W < 1 || L < 1 || L > kMaxLevels) return false;
    lh[0] = H;
    lw[0] = W;
    int64_t o = 0;
    for (int l = 1; l <= L; ++l) {
        if (lh[l - 1] < 4 || lw[l - 1] < 4) return false;
        lh[l] = (lh[l - 1] + 1) / 2;
        lw[l] = (lw[l - 1] + 1) / 2;
        loff[l] = o;
        o += 3 * (int64_t)lh[l] * lw[l];
    }
    *ll_off = o;
    *nc = o + (int64_t)lh[L] * lw[L];
    return true;
}

// Which per-cube arrays a call needs.
enum Parts { P_GRAM = 1, P_SMALL = 2, P_IMG = 4, P_SURE = 8 };

void plan_cube(CubePlan& c, Layout& lay, int parts) {
    c.T = (c.p + 15) / 16;
    c.n = (int64_t)c.H * c.W;
    if (parts & P_GRAM) {
        c.gslots = (int)std::max<int64_t>(1, std::min<int64_t>(256, cdiv(c.n, 2048)));
        const size_t per = c.dtype == HYRES_F64 ? (size_t)c.p * (c.p + 1) / 2 * 8
                                                : (size_t)c.T * (c.T + 1) / 2 * 256 * 4;
        c.o_gpart = lay.add(per * c.gslots);
        c.o_G = lay.add((size_t)c.p * c.p * 8);
    }
    if (parts & P_SMALL) {
        c.o_sigma = lay.add((size_t)c.p * 8);
        c.o_hv = lay.add((size_t)c.p * c.p * 8);
        c.o_V = lay.add((size_t)c.p * std::max(c.r, 1) * 8);
        c.o_evals = lay.add((size_t)c.p * 8);
        c.o_gap = lay.add(8);
        c.o_P32 = lay.add((size_t)16 * c.T * 16 * 4);
        c.o_Q32 = lay.add((size_t)16 * c.T * 16 * 4);
        c.o_P64 = lay.add((size_t)c.p * std::max(c.r, 1) * 8);
        c.o_Q64 = lay.add((size_t)c.p * std::max(c.r, 1) * 8);
        if ((parts & P_GRAM) && c.precision == HYRES_PREC_MIXED) {
            const int64_t ntiles = cdiv(c.n, kPixTile);
            c.rgroups = (int)cdiv(ntiles, kRitzGroup);
            c.o_rpart = lay.add((size_t)ntiles * 256 * 4);
            c.o_rsum = lay.add((size_t)c.rgroups * 256 * 8);
            c.o_rrot = lay.add(256 * 8);
        }
    }
    const int es = esize(c.dtype);
    if (parts & P_IMG) {
        c.nz = rup(c.n, kPixTile);
        c.o_Z = lay.add((size_t)c.r * c.nz * es);
        c.ncs = rup(c.nc, 64);
        c.o_coef = lay.add((size_t)c.r * c.ncs * es);
        const int64_t a1 = c.L >= 1 ? rup((int64_t)c.lh[1] * c.lw[1], 64) : 0;
        const int64_t a2 = c.L >= 2 ? rup((int64_t)c.lh[2] * c.lw[2], 64) : 0;
        c.tmp_off2 = a1;
        c.tps = a1 + a2;
        c.o_tmp = lay.add((size_t)std::max<int64_t>(1, c.r * c.tps) * es);
    }
    if (parts & P_SURE) {
        const size_t nb = (size_t)c.r * kSureBins;
        c.o_hcnt = lay.add(nb * 4);
        c.o_hsum = lay.add(nb * 8);
        c.o_hmin = lay.add(nb * 8);
        c.o_hmax = lay.add(nb * 8);
        c.o_sst = lay.add((size_t)c.r * sizeof(SureState));
        c.o_sbits = lay.add((size_t)c.r * (kSureBins / 32) * 4);
        c.o_spre = lay.add(nb * 8);
        c.o_sspre = lay.add(nb * 8);
        c.o_sctr = lay.add((size_t)c.r * 16);
        c.o_cand = lay.add((size_t)c.r * kSureCap * 8);
        c.o_lambda = lay.add((size_t)c.r * 8);
        c.o_sure = lay.add((size_t)c.r * 8);
    }
}

template <typename P>
P* at(void* ws, size_t off) {
    return reinterpret_cast<P*>(static_cast<unsigned char*>(ws) + off);
}

#ifdef HYRES_PHASE_TIMING
void* g_phase_buf = nullptr;
#endif

CubeDesc make_desc(const CubePlan& c, void* ws) {
    CubeDesc d;
    std::memset(&d, 0, sizeof(d));
#ifdef HYRES_PHASE_TIMING
    d.dbg = static_cast<unsigned long long*>(g_phase_buf);
#endif
    d.H = c.H; d.W = c.W; d.p = c.p; d.r = c.r; d.L = c.L; d.scope = c.scope; d.T = c.T; d.dtype = c.dtype;
    d.n = c.n;
    d.pmag = c.p > 0 ? (uint32_t)((((uint64_t)1) << 32) / (uint64_t)c.p + 1) : 0;
    for (int l = 0; l <= kMaxLevels; ++l) {
        d.lh[l] = c.lh[l];
        d.lw[l] = c.lw[l];
        d.loff[l] = c.loff[l];
    }
    d.ll_off = c.ll_off; d.nc = c.nc; d.ncs = c.ncs; d.nz = c.nz; d.tps = c.tps; d.tmp_off2 = c.tmp_off2;
    d.gslot0 = 0; d.gslots = c.gslots;
    if (c.o_G) {
        d.gpart = at<void>(ws, c.o_gpart);
        d.G = at<double>(ws, c.o_G);
    }
    if (c.o_sigma) {
        d.sigma = at<double>(ws, c.o_sigma);
        d.hv = at<double>(ws, c.o_hv);
        d.V = at<double>(ws, c.o_V);
        d.evals = at<double>(ws, c.o_evals);
        d.gap = at<double>(ws, c.o_gap);
        d.P32 = at<float>(ws, c.o_P32);
        d.Q32 = at<float>(ws, c.o_Q32);
        d.P64 = at<double>(ws, c.o_P64);
        d.Q64 = at<double>(ws, c.o_Q64);
        if (c.o_rpart) {
            d.rpart = at<float>(ws, c.o_rpart);
            d.rsum = at<double>(ws, c.o_rsum);
            d.rrot = at<double>(ws, c.o_rrot);
            d.rgroups = c.rgroups;
        }
    }
    if (c.o_Z || c.o_coef) {
        d.Z = at<void>(ws, c.o_Z);
        d.coef = at<void>(ws, c.o_coef);
        d.tmp = at<void>(ws, c.o_tmp);
    }
    if (c.o_hcnt) {
        d.hcnt = at<uint32_t>(ws, c.o_hcnt);
        d.hsum = at<double>(ws, c.o_hsum);
        d.hmin = at<uint64_t>(ws, c.o_hmin);
        d.hmax = at<uint64_t>(ws, c.o_hmax);
        d.sst = at<SureState>(ws, c.o_sst);
        d.sbits = at<uint32_t>(ws, c.o_sbits);
        d.spre = at<uint64_t>(ws, c.o_spre);
        d.sspre = at<double>(ws, c.o_sspre);
        d.sctr = at<uint32_t>(ws, c.o_sctr);
        d.cand = at<uint64_t>(ws, c.o_cand);
        d.lambda = at<double>(ws, c.o_lambda);
        d.sure = at<double>(ws, c.o_sure);
    }
    return d;
}

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t _e = (x);                        \
        if (_e != hipSuccess) return HYRES_E_HIP;   \
    } while (0)

hyres_status set_device(hyres_handle* h) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return HYRES_E_HIP;
    if (cur != h->device && hipSetDevice(h->device) != hipSuccess) return HYRES_E_HIP;
    return HYRES_OK;
}

// ------------------------------------------------------------------ program
// Stages of a call, in execution order (bits of Program::stages).
enum { S_GRAM = 1, S_SMALL = 2, S_PROJ = 4, S_DWT = 8, S_SURE = 16, S_IDWT = 32, S_BP = 64 };

enum Kind {
    K_GRAM_F32, K_GRAM_BF16, K_GRAM_RED, K_GRAM_F64, K_SMALL, K_PROJ_F32, K_PROJ_F64, K_DWT, K_IDWT,
    K_SURE_INIT, K_SURE_ROUND, K_COPY, K_BP_F32, K_BP_F64, K_RITZ, K_BLEND_F32
};

struct Launch {
    int kind;
    int stage;          // HYRES_STAGE_* for the stage timers
    int key;            // T, band count, or tile candidate
    int a, b;           // table offsets (ints) or a cube index
    int n;              // cubes covered by the table, or length of a cube list
    int nlist;          // Rayleigh-Ritz: length of the cube list
    int grid, grid2;
    int level;
    int64_t n64;
    const double* src;
    double* dst;
    int grp;            // cube group whose stream runs it (-1: after every group, on the caller's stream)
    bool chain;         // last launch of its group's Gram stage
};

// Small-solve kernel classes by band count (the kernel is specialised on the
// register tiling of the p x p matrix).
constexpr int kSmallClassMax[] = {32, 64, 96, 128, 144, 160, 176, 192, 224};
constexpr int kSmallClasses = (int)(sizeof(kSmallClassMax) / sizeof(int));
int small_class(int p) {
    for (int i = 0; i < kSmallClasses; ++i)
        if (p <= kSmallClassMax[i]) return i;
    return kSmallClasses - 1;
}

// Upper bound on the tables of one program: per band-tile class (14) Gram,
// projection items and the reduce list; back-projection items per class, or
// per blend pass of a tile grid (whose tiles share one class); per small-solve
// class a list; SURE component and histogram items; per level, direction and
// tile candidate the DWT items; the Rayleigh-Ritz slot and pixel items and
// cube list; plus one scratch table for the tuner.
// Cube groups (see Exec::group_of) repeat the SURE, transform and
// Rayleigh-Ritz tables once per group.
constexpr int kMaxColours = 8;    // blend colours per axis of a tile grid
constexpr int kMaxGroups = 4;
constexpr int kMaxTables = 3 * 14 + std::max(14, kMaxColours * kMaxColours) + kSmallClasses +
                           kMaxGroups * (2 + 2 * kMaxLevels * kTileCands + 3) + 1;
size_t table_ints(int count) { return (size_t)kMaxTables * (count + 1); }

struct Exec {
    hyres_handle* h = nullptr;
    void* ws = nullptr;
    int count = 0, dtype = 0, precision = 0;
    std::vector<CubePlan> plan;
    std::vector<CubeDesc> desc;
    Layout lay;
    size_t o_desc = 0, o_tab = 0;
    std::vector<int> tab;
    std::vector<Launch> prog;
    std::vector<int> pass_of;   // blend pass of each tile (empty: no blending)
    // Cube groups: each group runs its stages on a stream of its own, and a
    // group's Gram stage starts when the previous group's has ended, so that
    // one group's small solves (a few workgroups) overlap the next group's
    // bandwidth-bound stages.  A blended back-projection runs after every group.
    std::vector<int> group_of;
    int ngroups = 1;
    // FP32 tile grids: the back-projection blends the tiles in one pass over X
    bool blend1 = false;
    BlendGrid bg{};

    const CubeDesc* descs() const { return at<const CubeDesc>(ws, o_desc); }
    const int* table(int off) const { return at<const int>(ws, o_tab) + off; }
    int grid(int64_t nitems, int per_cu) const {
        return (int)std::max<int64_t>(1, std::min<int64_t>(nitems, (int64_t)h->num_cu * per_cu));
    }
    // Appends a prefix table of per-cube item counts; returns its offset.
    int counts(const std::vector<int64_t>& cnt, int64_t* total) {
        const int off = (int)tab.size();
        int64_t acc = 0;
        tab.push_back(0);
        for (int64_t v : cnt) {
            acc += v;
            tab.push_back((int)acc);
        }
        *total = acc;
        return off;
    }
    int list(const std::vector<int>& ids) {
        const int off = (int)tab.size();
        tab.insert(tab.end(), ids.begin(), ids.end());
        return off;
    }
};

// Lays out the descriptor table, the work tables and every cube's arrays.
void plan_exec(Exec& x, int parts) {
    x.o_desc = x.lay.add(sizeof(CubeDesc) * x.count);
    x.o_tab = x.lay.add(sizeof(int) * table_ints(x.count));
    for (auto& c : x.plan) plan_cube(c, x.lay, parts);
}

int tile_of(const hyres_handle* h, int dtype, bool inverse, int w) {
    return h->tile[dtype == HYRES_F64][inverse][width_class(w)];
}

bool in_group(const Exec& x, int i, int grp) { return grp < 0 || x.ngroups <= 1 || x.group_of[i] == grp; }

void add_dwt(Exec& x, bool inverse, int grp, bool rotate_l1 = false) {
    int Lmax = 0;
    for (int i = 0; i < x.count; ++i)
        if (in_group(x, i, grp)) Lmax = std::max(Lmax, x.plan[i].L);
    for (int k = 0; k < Lmax; ++k) {
        const int l = inverse ? Lmax - k : k + 1;
        // the first analysis level of a mixed FP32 solve applies the
        // Rayleigh-Ritz rotation as it loads Z: one item per tile of all components
        // (one launch per rank class, at most 8 or more: the kernel keeps the
        // rotation of the lower class in registers)
        const bool rot = rotate_l1 && !inverse && l == 1;
        for (int cls = 0; cls < (rot ? 2 : 1); ++cls)
        for (int cand = 0; cand < kTileCands; ++cand) {
            std::vector<int64_t> cnt(x.count, 0);
            bool any = false;
            int rmax = 0;
            for (int i = 0; i < x.count; ++i) {
                const CubePlan& c = x.plan[i];
                if (!in_group(x, i, grp) || c.L < l || tile_of(x.h, x.dtype, inverse, c.lw[l]) != cand) continue;
                if (rot && (c.r > 8) != (cls == 1)) continue;
                cnt[i] = (rot ? 1 : c.r) * cdiv(c.lw[l], kTileTX[cand]) * cdiv(c.lh[l], kTileTY[cand]);
                rmax = std::max(rmax, c.r);
                any = true;
            }
            if (!any) continue;
            int64_t tot;
            Launch L{};
            L.kind = inverse ? K_IDWT : K_DWT;
            L.stage = inverse ? HYRES_STAGE_IDWT : HYRES_STAGE_DWT;
            L.key = cand;
            L.a = x.counts(cnt, &tot);
            L.n = x.count;
            L.level = l;
            L.grid = x.grid(tot, 8);
            L.grid2 = rot ? rmax : 0;
            L.grp = grp;
            x.prog.push_back(L);
        }
    }
}

// Appends the launches of the stages in `stages` for the cubes of group `grp`
// (every cube when grp < 0 or the executor has one group).
void build_group(Exec& x, int stages, int grp) {
    const int N = x.count;
    const bool f64 = x.dtype == HYRES_F64;
    std::vector<int> Ts;
    for (int i = 0; i < N; ++i)
        if (in_group(x, i, grp)) Ts.push_back(x.plan[i].T);
    std::sort(Ts.begin(), Ts.end());
    Ts.erase(std::unique(Ts.begin(), Ts.end()), Ts.end());
    const size_t first = x.prog.size();

    // cubes of band-tile class T (and of blend pass `pass` when pass >= 0) in the group
    auto member = [&](int i, int T, int pass) {
        return in_group(x, i, grp) && (T < 0 || x.plan[i].T == T) && (pass < 0 || x.pass_of[i] == pass);
    };
    auto per_T = [&](int kind, int stage, int per_cu, auto items_of, int pass = -1) {
        for (int T : Ts) {
            std::vector<int64_t> cnt(N, 0);
            bool any = false;
            for (int i = 0; i < N; ++i)
                if (member(i, T, pass)) {
                    cnt[i] = items_of(x.plan[i]);
                    any = true;
                }
            if (!any) continue;
            int64_t tot;
            Launch L{};
            L.kind = kind;
            L.stage = stage;
            L.key = T;
            L.a = x.counts(cnt, &tot);
            L.n = N;
            L.grid = x.grid(tot, per_cu);
            if (kind == K_PROJ_F32 || kind == K_GRAM_F32 || kind == K_GRAM_BF16) {
                // one load path for every cube of the class: the kernel without the others
                bool vec = true, dense = true, scalar = true;
                for (int i = 0; i < N; ++i) {
                    if (!cnt[i]) continue;
                    if (!x.desc[i].vec4) vec = false;
                    if (!x.desc[i].dense) dense = false;
                    if (x.desc[i].vec4 || x.desc[i].dense) scalar = false;
                }
                L.b = vec ? kVec : dense ? kDense : scalar ? kScalar : kAnyLayout;
            }
            // native FP32 Gram of fewer slots than half the compute units (a
            // small cube alone): each slot's tiles split over several blocks
            if (kind == K_GRAM_F32 && x.h && tot * 2 < x.h->num_cu) L.grid2 = 1;
            x.prog.push_back(L);
            if (kind == K_GRAM_F32 || kind == K_GRAM_BF16) {
                std::vector<int> ids;
                for (int i = 0; i < N; ++i)
                    if (member(i, T, -1)) ids.push_back(i);
                Launch R{};
                R.kind = K_GRAM_RED;
                R.stage = stage;
                R.key = T;
                R.a = x.list(ids);
                R.n = (int)ids.size();
                x.prog.push_back(R);
            }
        }
    };
    auto per_cube = [&](int kind, int stage, int pass = -1) {
        for (int i = 0; i < N; ++i) {
            if (!member(i, -1, pass)) continue;
            Launch L{};
            L.kind = kind;
            L.stage = stage;
            L.key = x.plan[i].p;
            L.a = i;
            L.grid = x.plan[i].gslots;
            L.n64 = x.plan[i].n;
            x.prog.push_back(L);
        }
    };

    if (stages & S_GRAM) {
        if (f64) per_cube(K_GRAM_F64, HYRES_STAGE_GRAM);
        else per_T(x.precision == HYRES_PREC_MIXED ? K_GRAM_BF16 : K_GRAM_F32, HYRES_STAGE_GRAM, 2,
                   [](const CubePlan& c) { return (int64_t)c.gslots; });
    }
    if (stages & S_SMALL) {
        for (int k = 0; k < kSmallClasses; ++k) {
            std::vector<int> ids;
            for (int i = 0; i < N; ++i)
                if (in_group(x, i, grp) && small_class(x.plan[i].p) == k) ids.push_back(i);
            if (ids.empty()) continue;
            Launch L{};
            L.kind = K_SMALL;
            L.stage = HYRES_STAGE_SMALL;
            L.key = kSmallClassMax[k];
            L.a = x.list(ids);
            L.n = (int)ids.size();
            x.prog.push_back(L);
        }
    }
    if (stages & S_PROJ) {
        if (f64) per_cube(K_PROJ_F64, HYRES_STAGE_PROJECT);
        else per_T(K_PROJ_F32, HYRES_STAGE_PROJECT, 8, [](const CubePlan& c) { return cdiv(c.n, kPixTile); });
        if (x.precision == HYRES_PREC_MIXED && !f64) {
            // the FP32 refinement of the subspace (Rayleigh-Ritz on T^T T)
            // (the rotation of Z by the Ritz vectors is applied by the first
            // analysis level as it loads Z)
            std::vector<int64_t> slots(N, 0);
            std::vector<int> ids;
            for (int i = 0; i < N; ++i) {
                if (!in_group(x, i, grp)) continue;
                slots[i] = x.plan[i].rgroups;
                ids.push_back(i);
            }
            int64_t ns;
            Launch R{};
            R.kind = K_RITZ;
            R.stage = HYRES_STAGE_PROJECT;
            R.a = x.counts(slots, &ns);
            R.key = x.list(ids);
            R.n = N;
            R.nlist = (int)ids.size();
            R.grid = x.grid(ns, 4);
            x.prog.push_back(R);
        }
    }
    if (stages & S_DWT) add_dwt(x, false, grp, x.precision == HYRES_PREC_MIXED && !f64 && (stages & S_PROJ));
    if (stages & S_SURE) {
        std::vector<int64_t> comp(N, 0), hist(N, 0);
        // one work-item size for the whole program: about one item per compute unit
        int64_t total_coef = 0;
        for (int i = 0; i < N; ++i) {
            const CubePlan& c = x.plan[i];
            if (in_group(x, i, grp) && !c.has_lambda) total_coef += (int64_t)c.r * (c.scope == HYRES_SCOPE_DETAIL ? c.ll_off : c.nc);
        }
        const int64_t ch = sure_chunk_for(total_coef, x.h ? x.h->num_cu : 256);
        for (int i = 0; i < N; ++i) {
            const CubePlan& c = x.plan[i];
            if (!in_group(x, i, grp) || c.has_lambda) continue;
            const int64_t ns = c.scope == HYRES_SCOPE_DETAIL ? c.ll_off : c.nc;
            comp[i] = c.r;
            x.desc[i].schunk = ch;
            hist[i] = c.r * cdiv(ns, ch);
        }
        int64_t ncomp, nh;
        const int tc = x.counts(comp, &ncomp);
        const int th = x.counts(hist, &nh);
        if (ncomp > 0) {
            Launch I{};
            I.kind = K_SURE_INIT;
            I.stage = HYRES_STAGE_SURE;
            I.a = tc;
            I.n = N;
            I.grid = (int)ncomp;
            x.prog.push_back(I);
            for (int k = 0; k < sure_rounds(x.dtype); ++k) {
                Launch R{};
                R.kind = K_SURE_ROUND;
                R.stage = HYRES_STAGE_SURE;
                R.a = th;
                R.n = N;
                R.grid = x.grid(nh, 1);
                x.prog.push_back(R);
            }
        }
        for (int i = 0; i < N; ++i) {
            if (!in_group(x, i, grp) || !x.plan[i].has_lambda) continue;
            Launch C{};
            C.kind = K_COPY;
            C.stage = HYRES_STAGE_SURE;
            C.src = x.desc[i].lambda_in;
            C.dst = x.desc[i].lambda;
            C.n = x.plan[i].r;
            x.prog.push_back(C);
        }
    }
    if (stages & S_IDWT) add_dwt(x, true, grp);
    if ((stages & S_BP) && x.blend1 && !f64) {
        Launch L{};
        L.kind = K_BLEND_F32;
        L.stage = HYRES_STAGE_BACKPROJECT;
        L.key = x.plan[0].T;
        L.grid = x.grid((int64_t)x.bg.H * cdiv(x.bg.W, kPixTile), 4);
        x.prog.push_back(L);
    } else if (stages & S_BP) {
        // blended tiles: one launch per pass of non-overlapping tiles, in pass order
        int npass = 1;
        for (int v : x.pass_of) npass = std::max(npass, v + 1);
        for (int k = 0; k < npass; ++k) {
            const int pass = x.pass_of.empty() ? -1 : k;
            if (f64) per_cube(K_BP_F64, HYRES_STAGE_BACKPROJECT, pass);
            else per_T(K_BP_F32, HYRES_STAGE_BACKPROJECT, 8, [](const CubePlan& c) { return cdiv(c.n, kPixTile); },
                       pass);
        }
    }
    for (size_t k = first; k < x.prog.size(); ++k) x.prog[k].grp = grp < 0 ? -1 : grp;
}

// Builds the launch program of the stages in `stages` over every cube: one
// run of stages per cube group, then (tile grids) the blended back-projection.
void build_program(Exec& x, int stages) {
    x.tab.clear();
    x.prog.clear();
    if (x.ngroups <= 1) {
        build_group(x, stages, 0);
        return;
    }
    const int joint = x.pass_of.empty() ? 0 : (stages & S_BP);
    for (int g = 0; g < x.ngroups; ++g) {
        const size_t first = x.prog.size();
        build_group(x, stages & ~joint, g);
        for (size_t k = x.prog.size(); k > first; --k)
            if (x.prog[k - 1].stage == HYRES_STAGE_GRAM) {
                x.prog[k - 1].chain = true;
                break;
            }
    }
    if (joint) build_group(x, joint, -1);
}

hipError_t launch_one(const Exec& x, const Launch& L, hipStream_t s) {
    const CubeDesc* D = x.descs();
    switch (L.kind) {
        case K_GRAM_F32: return launch_gram_f32(L.key, L.b, D, x.table(L.a), L.n, L.grid, s, L.grid2 != 0);
        case K_GRAM_BF16: return launch_gram_bf16(L.key, L.b, D, x.table(L.a), L.n, L.grid, s);
        case K_GRAM_RED: return launch_gram_reduce_f32(L.key, D, x.table(L.a), L.n, s);
        case K_GRAM_F64: return launch_gram_f64(D, L.a, L.key, L.grid, s);
        case K_SMALL: return launch_small(L.key, D, x.table(L.a), L.n, s);
        case K_PROJ_F32: return launch_project_f32(L.key, L.b, D, x.table(L.a), L.n, L.grid, s);
        case K_PROJ_F64: return launch_project_f64(D, L.a, L.n64, s);
        case K_DWT:
            if (L.grid2)
                return launch_dwt_level1_rot(kTileTX[L.key], kTileTY[L.key], D, x.table(L.a), L.n, L.grid, L.grid2, s);
            return launch_dwt_level(x.dtype, kTileTX[L.key], kTileTY[L.key], false, D, x.table(L.a), L.n, L.level,
                                    L.grid, s);
        case K_IDWT:
            return launch_dwt_level(x.dtype, kTileTX[L.key], kTileTY[L.key], L.kind == K_IDWT, D, x.table(L.a),
                                    L.n, L.level, L.grid, s);
        case K_SURE_INIT: return launch_sure_init(x.dtype, D, x.table(L.a), L.n, L.grid, s);
        case K_SURE_ROUND:
            return launch_sure_round(x.dtype, D, x.table(L.a), L.n, L.grid, s);
        case K_COPY:
            hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(64), 0, s, L.src, L.dst, L.n);
            return hipGetLastError();
        case K_BP_F32: return launch_backproject_f32(L.key, D, x.table(L.a), L.n, L.grid, s);
        case K_BP_F64: return launch_backproject_f64(D, L.a, L.n64, s);
        case K_BLEND_F32: return launch_blend_f32(L.key, D, x.bg, L.grid, s);
        case K_RITZ:
            return launch_ritz(D, x.table(L.a), x.table(L.key), L.nlist, L.n, L.grid, s);
    }
    return hipErrorInvalidValue;
}

// Batch groups: the cubes of one small-solve class, largest band counts (the
// longest small solves) first; classes beyond kMaxGroups share the last group.
void group_by_small_class(Exec& x) {
    std::vector<int> cls;
    for (auto& c : x.plan) cls.push_back(small_class(c.p));
    std::vector<int> order(cls);
    std::sort(order.begin(), order.end(), std::greater<int>());
    order.erase(std::unique(order.begin(), order.end()), order.end());
    x.ngroups = std::min<int>((int)order.size(), kMaxGroups);
    x.group_of.assign(x.count, 0);
    for (int i = 0; i < x.count; ++i) {
        const int rank = (int)(std::find(order.begin(), order.end(), cls[i]) - order.begin());
        x.group_of[i] = std::min(rank, x.ngroups - 1);
    }
}

// Tile-grid groups: consecutive tiles in raster order, kMaxGroups of them, of
// decreasing size (shares 8 : 7 : 6 : 4 of the tiles): the last group's small
// solves end last, and the fewer tiles it holds, the sooner its remaining
// stages (and then the blend) are done.
void group_tiles(Exec& x) {
    x.ngroups = std::min(kMaxGroups, x.count);
    x.group_of.assign(x.count, 0);
    if (x.ngroups < kMaxGroups) {
        for (int t = 0; t < x.count; ++t) x.group_of[t] = t;
        return;
    }
    static constexpr int kShare[kMaxGroups] = {8, 7, 6, 4};
    int tot = 0;
    for (int g = 0; g < kMaxGroups; ++g) tot += kShare[g];
    int acc = 0, t = 0;
    for (int g = 0; g < kMaxGroups; ++g) {
        acc += kShare[g];
        // tiles [t, end) form group g; every group keeps at least one tile
        int end = (int)((int64_t)x.count * acc / tot);
        end = std::max(end, t + 1);
        end = std::min(end, x.count - (kMaxGroups - 1 - g));
        if (g == kMaxGroups - 1) end = x.count;
        for (; t < end; ++t) x.group_of[t] = g;
    }
}

// Writes the descriptors and work tables into the workspace (stream-ordered).
hyres_status upload_exec(const Exec& x, hipStream_t s) {
    // the last table of the region is the tuner's
    if (x.tab.size() > table_ints(x.count) - (size_t)(x.count + 1)) return HYRES_E_UNSUPPORTED;
    const size_t db = sizeof(CubeDesc) * x.count, tb = sizeof(int) * x.tab.size();
    if (!x.tab.empty() && x.o_tab >= x.o_desc + db && x.o_tab - (x.o_desc + db) < kAlign) {
        // descriptors and tables adjacent (up to the alignment gap): one
        // upload covers both (a single launch for one cube)
        std::vector<unsigned char> buf(x.o_tab - x.o_desc + tb, 0);
        std::memcpy(buf.data(), x.desc.data(), db);
        std::memcpy(buf.data() + (x.o_tab - x.o_desc), x.tab.data(), tb);
        HIPCHK(upload(x.ws, x.o_desc, buf.data(), buf.size(), s));
        return HYRES_OK;
    }
    HIPCHK(upload(x.ws, x.o_desc, x.desc.data(), db, s));
    if (!x.tab.empty()) HIPCHK(upload(x.ws, x.o_tab, x.tab.data(), tb, s));
    return HYRES_OK;
}

// Stream and event operations of a launch program.  A program names streams
// by slot (0: the caller's stream, k >= 1: the handle's side stream k - 1) and
// events by id (kEvFork, kEvJoin + k, kEvChain + k).  HipOps issues them;
// DryOps only records them, for the host-side check of a program.
constexpr int kEvFork = 0;
constexpr int kEvJoin = 1;
constexpr int kEvChain = 1 + hyres_handle::kSide;
constexpr int kNumEv = 1 + 2 * hyres_handle::kSide;

struct StreamOps {
    virtual ~StreamOps() {}
    virtual hipError_t record(int ev, int slot) = 0;
    virtual hipError_t wait(int slot, int ev) = 0;
    virtual hipError_t launch(const Launch& L, int slot) = 0;
    virtual hipStream_t stream(int slot) = 0;   // the stream of a slot (slot 0 may be the null stream)
    virtual bool live() const = 0;              // enqueues on a device (false: a host-only dry run)
};

struct HipOps : StreamOps {
    const Exec& x;
    hipStream_t s;
    bool capturing;   // the caller's stream is being captured into a graph
    HipOps(const Exec& x_, hipStream_t s_, bool cap) : x(x_), s(s_), capturing(cap) {}
    hipEvent_t event(int ev) const {
        hyres_handle* h = x.h;
        return ev == kEvFork ? h->fork : ev < kEvChain ? h->join[ev - kEvJoin] : h->chain[ev - kEvChain];
    }
    hipStream_t stream(int slot) override { return slot == 0 ? s : x.h->side[slot - 1]; }
    bool live() const override { return true; }
    // Under capture every enqueue must leave the stream in an active capture
    // (a dependency the capture cannot represent invalidates it).
    hipError_t captured(int slot) {
        if (!capturing) return hipSuccess;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(stream(slot), &cs);
        if (e != hipSuccess) return e;
        return cs == hipStreamCaptureStatusActive ? hipSuccess : hipErrorStreamCaptureInvalidated;
    }
    hipError_t record(int ev, int slot) override {
        hipError_t e = hipEventRecord(event(ev), stream(slot));
        return e != hipSuccess ? e : captured(slot);
    }
    hipError_t wait(int slot, int ev) override {
        hipError_t e = hipStreamWaitEvent(stream(slot), event(ev), 0);
        return e != hipSuccess ? e : captured(slot);
    }
    hipError_t launch(const Launch& L, int slot) override {
        hipError_t e = launch_one(x, L, stream(slot));
        return e != hipSuccess ? e : captured(slot);
    }
};

struct DryOps : StreamOps {
    struct Op { char kind; int a, b; };   // 'r' (event a on slot b), 'w' (slot a waits on event b), 'l' (slot a)
    std::vector<Op> ops;
    hipError_t record(int ev, int slot) override { ops.push_back({'r', ev, slot}); return hipSuccess; }
    hipError_t wait(int slot, int ev) override { ops.push_back({'w', slot, ev}); return hipSuccess; }
    hipError_t launch(const Launch&, int slot) override { ops.push_back({'l', slot, 0}); return hipSuccess; }
    hipStream_t stream(int) override { return nullptr; }
    bool live() const override { return false; }
};

// Enqueues a program through `ops`, refusing any wait on an event that the
// program has not recorded before it (such a wait would depend on whatever an
// earlier call left in the event, and inside a graph capture on work outside
// the capture).  Side streams that were forked are joined back into the
// caller's stream on every return, errors included, so that a capture can
// always be ended.
struct ProgramRun {
    const Exec& x;
    StreamOps& ops;
    bool rec[kNumEv] = {};
    bool forked[hyres_handle::kSide + 1] = {};
    ProgramRun(const Exec& x_, StreamOps& o) : x(x_), ops(o) {}
    hyres_status record(int ev, int slot) {
        if (ops.record(ev, slot) != hipSuccess) return HYRES_E_HIP;
        rec[ev] = true;
        return HYRES_OK;
    }
    hyres_status wait(int slot, int ev) {
        if (!rec[ev]) return HYRES_E_HIP;
        return ops.wait(slot, ev) != hipSuccess ? HYRES_E_HIP : HYRES_OK;
    }
    hyres_status fork(int slot) {
        hyres_status st = wait(slot, kEvFork);
        if (!st) forked[slot] = true;
        return st;
    }
    // joins every forked side stream that is still apart into slot 0
    hyres_status join_all() {
        hyres_status first = HYRES_OK;
        for (int k = 1; k <= hyres_handle::kSide; ++k) {
            if (!forked[k]) continue;
            hyres_status st = record(kEvJoin + k - 1, k);
            if (!st) st = wait(0, kEvJoin + k - 1);
            if (st && !first) first = st;
            forked[k] = false;
        }
        return first;
    }
    hyres_status finish(hyres_status st) {
        hyres_status j = join_all();
        return st ? st : j;
    }
    hyres_status launch(const Launch& L, int slot) {
        return ops.launch(L, slot) != hipSuccess ? HYRES_E_HIP : HYRES_OK;
    }
};

// Cube groups: each group runs on its own stream (group 0 on the caller's),
// forked from the caller's stream; group g's first launch waits for the end
// of group g - 1's Gram stage; the joint launches (grp < 0) run on the
// caller's stream after every group has been joined back.
hyres_status run_grouped(const Exec& x, StreamOps& ops, bool timed) {
    hyres_handle* h = x.h;
    const int G = x.ngroups;
    ProgramRun pr(x, ops);
    // stage timers per group, on the group's stream (slot G: the joint launches)
    std::unique_ptr<StageTimer> tm[kMaxGroups + 1];
    int cur[kMaxGroups + 1];
    for (int g = 0; g <= G; ++g) cur[g] = -1;
    hyres_status st = pr.record(kEvFork, 0);
    for (int g = 1; g < G && !st; ++g) st = pr.fork(g);
    int prev = 0;
    bool joined = false;
    for (size_t k = 0; k < x.prog.size() && !st; ++k) {
        const Launch& L = x.prog[k];
        if (L.grp < 0 && !joined) {
            for (int g = 0; g < G; ++g) tm[g].reset();
            if ((st = pr.join_all())) break;
            joined = true;
        }
        if (L.grp > prev) {
            // this group's Gram stage follows the previous group's
            if ((st = pr.wait(L.grp, kEvChain + L.grp - 1))) break;
            prev = L.grp;
        }
        const int slot = L.grp < 0 ? 0 : L.grp;
        const int tslot = L.grp < 0 ? G : L.grp;
        if (timed && ops.live() && L.stage != cur[tslot]) {
            tm[tslot].reset();
            tm[tslot].reset(new StageTimer(h, ops.stream(slot), L.stage));
            cur[tslot] = L.stage;
        }
        if ((st = pr.launch(L, slot))) break;
        if (L.chain && L.grp >= 0 && L.grp + 1 < G) st = pr.record(kEvChain + L.grp, slot);
    }
    for (int g = 0; g <= G; ++g) tm[g].reset();
    return pr.finish(st);
}

// Enqueues the program; `timed` wraps each stage in the handle's stage timers.
// Consecutive small-solve launches (one per band-count class, each a handful of
// workgroups) run beside each other: the first on the caller's stream, the
// others on the handle's side streams, forked from and joined back into it by
// events (a capture of the caller's stream records them as parallel branches).
hyres_status run_program(const Exec& x, StreamOps& ops, bool timed) {
    if (x.h) ++x.h->runs;
    if (x.ngroups > 1 && x.h) return run_grouped(x, ops, timed);
    ProgramRun pr(x, ops);
    std::unique_ptr<StageTimer> tm;
    int cur = -1;
    const size_t np = x.prog.size();
    hyres_status st = HYRES_OK;
    for (size_t k = 0; k < np && !st; ++k) {
        const Launch& L = x.prog[k];
        if (timed && ops.live() && L.stage != cur) {
            tm.reset();
            tm.reset(new StageTimer(x.h, ops.stream(0), L.stage));
            cur = L.stage;
        }
        size_t m = 1;
        if (L.kind == K_SMALL && x.h && x.ngroups <= 1)
            while (k + m < np && m <= (size_t)hyres_handle::kSide && x.prog[k + m].kind == K_SMALL) ++m;
        if (m == 1) {
            st = pr.launch(L, 0);
            continue;
        }
        if ((st = pr.record(kEvFork, 0))) break;
        for (size_t i = 1; i < m && !st; ++i) {
            if ((st = pr.fork((int)i))) break;
            st = pr.launch(x.prog[k + i], (int)i);
        }
        if (!st) st = pr.launch(L, 0);
        if (!st) st = pr.join_all();
        k += m - 1;
    }
    tm.reset();
    return pr.finish(st);
}

hyres_status run_program(const Exec& x, hipStream_t s, bool timed, bool capturing = false) {
    HipOps ops(x, s, capturing);
    return run_program(x, ops, timed);
}

// Host-side check of a program's stream order (no device is touched): the
// program is run through DryOps, which refuses a wait on an event not yet
// recorded; then every side stream must start with a wait (it joins the
// caller's dependency chain) and end with a join record that the caller's
// stream waits on, with nothing enqueued on the side stream after it.
hyres_status dry_check(const Exec& x, hyres_program_stats* stats) {
    DryOps ops;
    hyres_status st = run_program(x, ops, false);
    if (st) return st;
    const auto& v = ops.ops;
    int n_l = 0, n_r = 0, n_w = 0, used = 1;
    for (int k = 1; k <= hyres_handle::kSide; ++k) {
        int first = -1, last = -1;
        for (int i = 0; i < (int)v.size(); ++i) {
            const int slot = v[i].kind == 'r' ? v[i].b : v[i].a;
            if (slot != k) continue;
            if (first < 0) first = i;
            last = i;
        }
        if (first < 0) continue;
        ++used;
        if (v[first].kind != 'w') return HYRES_E_HIP;
        if (v[last].kind != 'r') return HYRES_E_HIP;
        const int ev = v[last].a;
        bool waited = false;
        for (int i = last + 1; i < (int)v.size(); ++i) {
            if (v[i].kind == 'r' && v[i].a == ev) break;          // re-recorded before any wait
            if (v[i].kind == 'w' && v[i].a == 0 && v[i].b == ev) {
                waited = true;
                break;
            }
        }
        if (!waited) return HYRES_E_HIP;
    }
    for (const auto& o : v) {
        n_l += o.kind == 'l';
        n_r += o.kind == 'r';
        n_w += o.kind == 'w';
    }
    if (stats) {
        stats->launches = n_l;
        stats->records = n_r;
        stats->waits = n_w;
        stats->streams = used;
        stats->groups = x.ngroups;
    }
    return HYRES_OK;
}

// A handle with no device behind it, for host-only planning.
void init_host_handle(hyres_handle& h) {
    h.device = -1;
    h.num_cu = 256;
    h.prof_mask = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int w = 0; w < kWidthClasses; ++w) {
                h.tile[a][b][w] = (unsigned char)default_tile(w);
                h.tuned[a][b][w] = 0;
                h.tile_us[a][b][w] = 0.f;
            }
}

bool valid_dtype(int dt) { return dt == HYRES_F32 || dt == HYRES_F64; }

// FP32 cube with 16-byte aligned pixel vectors whose 64-pixel chunks are
// consecutive in memory (contiguous cube, or image rows of whole chunks, as in
// a tile of a larger cube): the kernels use float4 accesses.
int vec4_ok(const void* ptr, int W, int p, int64_t pitch, int64_t row_pitch, int dtype) {
    return dtype == HYRES_F32 && p % 4 == 0 && pitch % 4 == 0 && row_pitch % 4 == 0 &&
           (row_pitch == (int64_t)W * pitch || W % kPixTile == 0) && (reinterpret_cast<uintptr_t>(ptr) % 16) == 0;
}

// Unpadded FP32 pixels (pitch == p) whose 64-pixel tiles are each 64 p consecutive,
// 16-byte aligned floats: a contiguous cube, or whole tiles per image row.
int dense_ok(const void* ptr, int W, int p, int64_t pitch, int64_t row_pitch, int dtype) {
    return dtype == HYRES_F32 && pitch == p && (reinterpret_cast<uintptr_t>(ptr) % 16) == 0 &&
           (row_pitch == (int64_t)W * p || (W % kPixTile == 0 && row_pitch % 4 == 0));
}

hyres_status check_shape(int H, int W, int p, int64_t pitch, int64_t row_pitch) {
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    if (pitch < p || row_pitch < (int64_t)(W - 1) * pitch + p) return HYRES_E_SHAPE;
    if ((int64_t)H * W > (int64_t)1 << 31) return HYRES_E_UNSUPPORTED;
    return HYRES_OK;
}

hyres_status check_cube(const void* Y, int H, int W, int p, int64_t pitch, int64_t row_pitch, int dtype) {
    if (!Y) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    return check_shape(H, W, p, pitch, row_pitch);
}

hyres_status check_ws(const void* ws, size_t have, size_t need) {
    if (need == 0) return HYRES_OK;
    if (!ws) return HYRES_E_WORKSPACE;
    if (have < need) return HYRES_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HYRES_E_WORKSPACE;
    return HYRES_OK;
}

// Plan of a cube-taking call: geometry, then workspace layout.
hyres_status plan_cubes(Exec& x, int parts) {
    for (auto& c : x.plan) {
        if (parts & (P_IMG | P_SURE)) {
            if (!level_geometry(c.H, c.W, c.L, c.lh, c.lw, c.loff, &c.ll_off, &c.nc)) return HYRES_E_SHAPE;
        }
    }
    plan_exec(x, parts);
    return HYRES_OK;
}

hyres_status check_prec_scope(int precision, int scope, int dtype) {
    if (scope != HYRES_SCOPE_ALL && scope != HYRES_SCOPE_DETAIL) return HYRES_E_SHAPE;
    if (precision != HYRES_PREC_NATIVE && precision != HYRES_PREC_MIXED) return HYRES_E_DTYPE;
    if (precision == HYRES_PREC_MIXED && dtype != HYRES_F32) return HYRES_E_DTYPE;
    return HYRES_OK;
}

hyres_status check_rank_levels(int r, int L, int p) {
    if (r < 1 || r > kMaxRank || r > p) return HYRES_E_SHAPE;
    if (L < 1 || L > kMaxLevels) return HYRES_E_SHAPE;
    return HYRES_OK;
}

hyres_status check_opts(const hyres_options* opt, int p, int dtype) {
    if (!opt) return HYRES_E_NULL;
    hyres_status st = check_rank_levels(opt->rank, opt->levels, p);
    if (st) return st;
    constexpr int kRankFlags = HYRES_FLAG_RANK_HYSIME | HYRES_FLAG_RANK_SURE;
    if ((opt->flags & kRankFlags) == kRankFlags) return HYRES_E_UNSUPPORTED;
    return check_prec_scope(opt->precision, opt->scope, dtype);
}

constexpr int kAllParts = P_GRAM | P_SMALL | P_IMG | P_SURE;
constexpr int kAllStages = S_GRAM | S_SMALL | S_PROJ | S_DWT | S_SURE | S_IDWT | S_BP;

// Descriptor of one cube of a full solve: workspace arrays, then the caller's pointers.
CubeDesc solve_desc(const CubePlan& c, void* ws, const void* Y, int64_t pitch, int64_t row_pitch, void* X,
                    int64_t x_pitch, int64_t x_row_pitch, const double* sigma_in, const double* lambda_in,
                    int flags, const hyres_outputs* out) {
    CubeDesc d = make_desc(c, ws);
    d.Y = Y; d.pitch = pitch; d.row_pitch = row_pitch;
    d.X = X; d.xpitch = x_pitch; d.xrow_pitch = x_row_pitch;
    d.vec4 = vec4_ok(Y, c.W, c.p, pitch, row_pitch, c.dtype);
    d.xvec4 = vec4_ok(X, c.W, c.p, x_pitch, x_row_pitch, c.dtype);
    d.dense = dense_ok(Y, c.W, c.p, pitch, row_pitch, c.dtype);
    d.xdense = dense_ok(X, c.W, c.p, x_pitch, x_row_pitch, c.dtype);
    d.sigma_in = sigma_in;
    d.lambda_in = lambda_in;
    d.mode = (sigma_in ? 0 : 1) | 2 | 8 | ((flags & (HYRES_FLAG_ALL_EVALS | HYRES_FLAG_RANK_SURE)) ? 16 : 0) |
             ((flags & HYRES_FLAG_RANK_HYSIME) ? kModeRankHySime : 0) |
             ((flags & HYRES_FLAG_RANK_SURE) ? kModeRankSure : 0);
    if (out) {
        if (out->sigma) d.sigma = out->sigma;
        if (out->V) d.V = out->V;
        if (out->evals) d.evals = out->evals;
        if (out->gap) d.gap = out->gap;
        if (out->lambda) d.lambda = out->lambda;
        if (out->sure) d.sure = out->sure;
        d.status = out->status;
        d.rank_out = out->rank;
        d.eig_check = out->eig_check;
    }
    return d;
}

}  // namespace

namespace hyres {
CubeView cube_view(const void* Y, int W, int p, int64_t n, int64_t pitch, int64_t row_pitch, int dtype) {
    CubeView v;
    v.Y = Y; v.pitch = pitch; v.row_pitch = row_pitch;
    v.n = n; v.W = W; v.p = p;
    v.vec4 = vec4_ok(Y, W, p, pitch, row_pitch, dtype);
    v.dense = dense_ok(Y, W, p, pitch, row_pitch, dtype);
    v.pmag = (uint32_t)((((uint64_t)1) << 32) / (uint64_t)p + 1);
    return v;
}
}  // namespace hyres

// =========================================================================
HYRES_API hyres_status hyres_create(hyres_handle** handle, int device) {
    if (!handle) return HYRES_E_NULL;
    *handle = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HYRES_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HYRES_E_HIP;
    hyres_handle* h = new (std::nothrow) hyres_handle();
    if (!h) return HYRES_E_HIP;
    h->device = device;
    h->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    char key[320];
    std::snprintf(key, sizeof(key), "%s/%dcu", prop.gcnArchName, h->num_cu);
    for (char* q = key; *q; ++q)
        if (*q == '"' || *q == '\\') *q = '_';
    h->arch = key;
    h->prof_mask = 0;
    {
        int prev = 0;
        bool ok = hipGetDevice(&prev) == hipSuccess && hipSetDevice(device) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; i < hyres_handle::kSide && ok; ++i) {
            ok = hipStreamCreateWithFlags(&h->side[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&h->join[i], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&h->chain[i], hipEventDisableTiming) == hipSuccess;
        }
        // the device address of this device's no-allocation scratch, with the device current
        ok = ok && scratch_address(device, &h->scratch) == hipSuccess;
        (void)hipSetDevice(prev);
        if (!ok) {
            hyres_destroy(h);
            return HYRES_E_HIP;
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int w = 0; w < kWidthClasses; ++w) {
                h->tile[a][b][w] = (unsigned char)default_tile(w);
                h->tuned[a][b][w] = 0;
                h->tile_us[a][b][w] = 0.f;
            }
    *handle = h;
    return HYRES_OK;
}

HYRES_API void hyres_destroy(hyres_handle* handle) {
    if (!handle) return;
    for (auto& r : handle->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : handle->pool) (void)hipEventDestroy(e);
    for (int i = 0; i < hyres_handle::kSide; ++i) {
        if (handle->side[i]) (void)hipStreamDestroy(handle->side[i]);
        if (handle->join[i]) (void)hipEventDestroy(handle->join[i]);
        if (handle->chain[i]) (void)hipEventDestroy(handle->chain[i]);
    }
    if (handle->fork) (void)hipEventDestroy(handle->fork);
    delete handle;
}

#ifdef HYRES_PHASE_TIMING
// Timing builds only: device buffer receiving phase time stamps of the small solve.
HYRES_API void hyres_debug_set_phase_buffer(void* dev_ptr) { g_phase_buf = dev_ptr; }
#endif

HYRES_API hyres_status hyres_profile_enable(hyres_handle* h, unsigned mask) {
    if (!h) return HYRES_E_NULL;
    h->prof_mask = mask & ((1u << HYRES_NUM_STAGES) - 1);
    return HYRES_OK;
}

HYRES_API hyres_status hyres_profile_read(hyres_handle* h, double* ms_out, int* count_out) {
    if (!h || !ms_out || !count_out) return HYRES_E_NULL;
    hyres_status st = set_device(h);
    if (st) return st;
    // records of one program run (one per cube group) add up to one timed stage
    std::vector<std::pair<int, unsigned>> seen;
    for (auto& r : h->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess) return HYRES_E_HIP;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return HYRES_E_HIP;
        ms_out[r.stage] += ms;
        const std::pair<int, unsigned> key(r.stage, r.run);
        if (std::find(seen.begin(), seen.end(), key) == seen.end()) {
            seen.push_back(key);
            count_out[r.stage] += 1;
        }
        h->pool.push_back(r.a);
        h->pool.push_back(r.b);
    }
    h->pending.clear();
    return HYRES_OK;
}

HYRES_API const char* hyres_status_string(int status) {
    switch (status) {
        case HYRES_OK: return "ok";
        case HYRES_E_NULL: return "a required pointer is NULL";
        case HYRES_E_SHAPE: return "invalid shape, rank, level count or pitch";
        case HYRES_E_DTYPE: return "invalid element type or precision";
        case HYRES_E_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
        case HYRES_E_HIP: return "HIP runtime error";
        case HYRES_E_UNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

HYRES_API int64_t hyres_coeff_count(int H, int W, int L) {
    int lh[kMaxLevels + 1], lw[kMaxLevels + 1];
    int64_t loff[kMaxLevels + 1], ll, nc;
    if (!level_geometry(H, W, L, lh, lw, loff, &ll, &nc)) return 0;
    return nc;
}

// Single-cube executor of the given geometry.
static void one_cube(Exec& x, hyres_handle* h, int H, int W, int p, int r, int L, int dtype, int scope,
                     int precision = HYRES_PREC_NATIVE) {
    x.h = h;
    x.count = 1;
    x.dtype = dtype;
    x.precision = precision;
    x.plan.resize(1);
    CubePlan& c = x.plan[0];
    c.H = H; c.W = W; c.p = p; c.r = r; c.L = L; c.dtype = dtype; c.scope = scope; c.precision = precision;
}

// ------------------------------------------------------------- noise
HYRES_API hyres_status hyres_estimate_noise_workspace_size(int H, int W, int p, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    Exec x;
    one_cube(x, nullptr, H, W, p, 1, 1, dtype, 0);
    hyres_status st = plan_cubes(x, P_GRAM | P_SMALL);
    if (st) return st;
    *bytes = x.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_estimate_noise(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                            int64_t row_pitch, int dtype, double* sigma_out, double* gram_out,
                                            int* status, void* workspace, size_t workspace_bytes,
                                            hyres_stream_t stream) {
    if (!h || !sigma_out) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    Exec x;
    one_cube(x, h, H, W, p, 1, 1, dtype, 0);
    if ((st = plan_cubes(x, P_GRAM | P_SMALL))) return st;
    if ((st = check_ws(workspace, workspace_bytes, x.lay.total))) return st;
    if ((st = set_device(h))) return st;
    x.ws = workspace;
    CubeDesc d = make_desc(x.plan[0], workspace);
    d.Y = Y; d.pitch = pitch; d.row_pitch = row_pitch;
    d.vec4 = vec4_ok(Y, W, p, pitch, row_pitch, dtype);
    d.dense = dense_ok(Y, W, p, pitch, row_pitch, dtype);
    d.sigma = sigma_out;
    if (gram_out) d.G = gram_out;
    d.status = status;
    d.mode = 1;
    x.desc.assign(1, d);
    build_program(x, S_GRAM | S_SMALL);
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_exec(x, s))) return st;
    return run_program(x, s, false);
}

// ------------------------------------------------------------- subspace
HYRES_API hyres_status hyres_subspace_workspace_size(int H, int W, int p, int r, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands || r < 1 || r > kMaxRank || r > p) return HYRES_E_SHAPE;
    Exec x;
    one_cube(x, nullptr, H, W, p, r, 1, dtype, 0);
    hyres_status st = plan_cubes(x, P_GRAM | P_SMALL);
    if (st) return st;
    *bytes = x.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_subspace(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                      int64_t row_pitch, int dtype, const double* sigma, int r, double* V_out,
                                      double* evals_out, int* status, void* workspace, size_t workspace_bytes,
                                      hyres_stream_t stream) {
    if (!h || !V_out) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    if (r < 1 || r > kMaxRank || r > p) return HYRES_E_SHAPE;
    Exec x;
    one_cube(x, h, H, W, p, r, 1, dtype, 0);
    if ((st = plan_cubes(x, P_GRAM | P_SMALL))) return st;
    if ((st = check_ws(workspace, workspace_bytes, x.lay.total))) return st;
    if ((st = set_device(h))) return st;
    x.ws = workspace;
    CubeDesc d = make_desc(x.plan[0], workspace);
    d.Y = Y; d.pitch = pitch; d.row_pitch = row_pitch;
    d.vec4 = vec4_ok(Y, W, p, pitch, row_pitch, dtype);
    d.dense = dense_ok(Y, W, p, pitch, row_pitch, dtype);
    d.sigma_in = sigma;
    d.V = V_out;
    if (evals_out) d.evals = evals_out;
    d.status = status;
    d.mode = 2 | 16;
    x.desc.assign(1, d);
    build_program(x, S_GRAM | S_SMALL);
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_exec(x, s))) return st;
    return run_program(x, s, false);
}

// ------------------------------------------------------------- wavelets
// A batch of images is planned as one "cube" whose components are the images.
static hyres_status plan_images(Exec& x, hyres_handle* h, int batch, int H, int W, int L, int dtype) {
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (batch < 1) return HYRES_E_SHAPE;
    one_cube(x, h, H, W, 2, batch, L, dtype, 0);
    CubePlan& c = x.plan[0];
    if (!level_geometry(H, W, L, c.lh, c.lw, c.loff, &c.ll_off, &c.nc)) return HYRES_E_SHAPE;
    c.n = (int64_t)H * W;
    c.T = 1;
    plan_exec(x, 0);
    const int es = esize(dtype);
    const int64_t a1 = rup((int64_t)c.lh[1] * c.lw[1], 64);
    const int64_t a2 = L >= 2 ? rup((int64_t)c.lh[2] * c.lw[2], 64) : 0;
    c.tmp_off2 = a1;
    c.tps = a1 + a2;
    c.o_tmp = x.lay.add((size_t)batch * c.tps * es);
    c.nz = c.n;
    c.ncs = c.nc;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_dwt2_workspace_size(int batch, int H, int W, int L, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    Exec x;
    hyres_status st = plan_images(x, nullptr, batch, H, W, L, dtype);
    if (st) return st;
    *bytes = x.lay.total;
    return HYRES_OK;
}

static hyres_status dwt_common(hyres_handle* h, const void* in, int batch, int H, int W, int L, int dtype,
                               void* out, const double* lambda, int scope, bool inverse, void* ws, size_t wsb,
                               hyres_stream_t stream) {
    if (!h || !in || !out) return HYRES_E_NULL;
    Exec x;
    hyres_status st = plan_images(x, h, batch, H, W, L, dtype);
    if (st) return st;
    if (scope != HYRES_SCOPE_ALL && scope != HYRES_SCOPE_DETAIL) return HYRES_E_SHAPE;
    if ((st = check_ws(ws, wsb, x.lay.total))) return st;
    if ((st = set_device(h))) return st;
    x.ws = ws;
    x.plan[0].scope = scope;
    CubeDesc d = make_desc(x.plan[0], ws);
    d.tmp = at<void>(ws, x.plan[0].o_tmp);
    if (inverse) {
        d.coef = const_cast<void*>(in);
        d.Z = out;
        if (lambda) {
            d.lambda = const_cast<double*>(lambda);
            d.mode = 8;
        }
    } else {
        d.Z = const_cast<void*>(in);
        d.coef = out;
    }
    x.desc.assign(1, d);
    build_program(x, inverse ? S_IDWT : S_DWT);
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_exec(x, s))) return st;
    return run_program(x, s, false);
}

HYRES_API hyres_status hyres_dwt2(hyres_handle* h, const void* x, int batch, int H, int W, int L, int dtype,
                                  void* coeffs, void* workspace, size_t workspace_bytes, hyres_stream_t stream) {
    return dwt_common(h, x, batch, H, W, L, dtype, coeffs, nullptr, 0, false, workspace, workspace_bytes, stream);
}

HYRES_API hyres_status hyres_idwt2(hyres_handle* h, const void* coeffs, int batch, int H, int W, int L, int dtype,
                                   const double* lambda, int scope, void* x_out, void* workspace,
                                   size_t workspace_bytes, hyres_stream_t stream) {
    return dwt_common(h, coeffs, batch, H, W, L, dtype, x_out, lambda, scope, true, workspace, workspace_bytes,
                      stream);
}

// ------------------------------------------------------------- SURE
static hyres_status plan_sure(Exec& x, hyres_handle* h, int batch, int64_t Nc, int dtype) {
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (batch < 1 || Nc < 1 || Nc > ((int64_t)1 << 31)) return HYRES_E_SHAPE;
    one_cube(x, h, 1, 1, 2, batch, 0, dtype, 0);
    CubePlan& c = x.plan[0];
    c.nc = Nc;
    c.ll_off = Nc;
    plan_exec(x, P_SURE);
    return HYRES_OK;
}

HYRES_API hyres_status hyres_sure_workspace_size(int batch, int64_t Nc, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    Exec x;
    hyres_status st = plan_sure(x, nullptr, batch, Nc, dtype);
    if (st) return st;
    *bytes = x.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_sure_threshold(hyres_handle* h, const void* coeffs, int batch, int64_t Nc,
                                            int64_t stride, int dtype, double* lambda_out, double* sure_min_out,
                                            int* status, void* workspace, size_t workspace_bytes,
                                            hyres_stream_t stream) {
    if (!h || !coeffs || !lambda_out) return HYRES_E_NULL;
    Exec x;
    hyres_status st = plan_sure(x, h, batch, Nc, dtype);
    if (st) return st;
    if (stride < Nc) return HYRES_E_SHAPE;
    if ((st = check_ws(workspace, workspace_bytes, x.lay.total))) return st;
    if ((st = set_device(h))) return st;
    x.ws = workspace;
    x.plan[0].ncs = stride;
    CubeDesc d = make_desc(x.plan[0], workspace);
    d.coef = const_cast<void*>(coeffs);
    d.lambda = lambda_out;
    d.sure = sure_min_out ? sure_min_out : d.sure;
    d.status = status;
    x.desc.assign(1, d);
    build_program(x, S_SURE);
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_exec(x, s))) return st;
    return run_program(x, s, false);
}

// ------------------------------------------------------------- denoise
HYRES_API hyres_status hyres_denoise_workspace_size(int H, int W, int p, const hyres_options* opt, int dtype,
                                                    size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    hyres_status st = check_opts(opt, p, dtype);
    if (st) return st;
    Exec x;
    one_cube(x, nullptr, H, W, p, opt->rank, opt->levels, dtype, opt->scope, opt->precision);
    if ((st = plan_cubes(x, kAllParts))) return st;
    *bytes = x.lay.total;
    return HYRES_OK;
}

// One solve of one cube.  noalloc: the workspace is the device's no-allocation
// scratch (the plan must fit it; the stage timers stay off, they create events).
static hyres_status denoise_one(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                int64_t row_pitch, int dtype, const hyres_options* opt, const double* sigma_in,
                                const double* lambda_in, void* X, int64_t x_pitch, int64_t x_row_pitch,
                                const hyres_outputs* out, bool noalloc, void* workspace, size_t workspace_bytes,
                                hyres_stream_t stream) {
    if (!h || !X) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    if ((st = check_opts(opt, p, dtype))) return st;
    if (x_pitch < p || x_row_pitch < (int64_t)(W - 1) * x_pitch + p) return HYRES_E_SHAPE;
    Exec x;
    one_cube(x, h, H, W, p, opt->rank, opt->levels, dtype, opt->scope, opt->precision);
    x.plan[0].has_lambda = lambda_in != nullptr;
    if ((st = plan_cubes(x, kAllParts))) return st;
    if (noalloc) {
        if (!h->scratch) return HYRES_E_HIP;
        if (x.lay.total > HYRES_NOALLOC_SCRATCH_BYTES) return HYRES_E_WORKSPACE;
        workspace = h->scratch;
    } else if ((st = check_ws(workspace, workspace_bytes, x.lay.total))) {
        return st;
    }
    if ((st = set_device(h))) return st;
    x.ws = workspace;
    x.desc.assign(1, solve_desc(x.plan[0], workspace, Y, pitch, row_pitch, X, x_pitch, x_row_pitch, sigma_in,
                                lambda_in, opt->flags, out));
    build_program(x, kAllStages);
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_exec(x, s))) return st;
    return run_program(x, s, !noalloc);
}

HYRES_API hyres_status hyres_denoise(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                     int64_t row_pitch, int dtype, const hyres_options* opt,
                                     const double* sigma_in, const double* lambda_in, void* X, int64_t x_pitch,
                                     int64_t x_row_pitch, const hyres_outputs* out, void* workspace,
                                     size_t workspace_bytes, hyres_stream_t stream) {
    return denoise_one(h, Y, H, W, p, pitch, row_pitch, dtype, opt, sigma_in, lambda_in, X, x_pitch, x_row_pitch,
                       out, false, workspace, workspace_bytes, stream);
}

HYRES_API hyres_status hyres_denoise_noalloc(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                             int64_t row_pitch, int dtype, const hyres_options* opt,
                                             const double* sigma_in, const double* lambda_in, void* X,
                                             int64_t x_pitch, int64_t x_row_pitch, const hyres_outputs* out,
                                             hyres_stream_t stream) {
    return denoise_one(h, Y, H, W, p, pitch, row_pitch, dtype, opt, sigma_in, lambda_in, X, x_pitch, x_row_pitch,
                       out, true, nullptr, 0, stream);
}

// ------------------------------------------------------------- HyMiNoR
static hyres_status check_l1l1(int H, int W, int p, int64_t pitch, int64_t row_pitch, int dtype,
                               const hyres_l1l1_options* o, int64_t x_pitch, int64_t x_row_pitch) {
    if (!o) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 1 || p > kMaxBands) return HYRES_E_SHAPE;
    if (pitch < p || row_pitch < (int64_t)(W - 1) * pitch + p) return HYRES_E_SHAPE;
    if (x_pitch < p || x_row_pitch < (int64_t)(W - 1) * x_pitch + p) return HYRES_E_SHAPE;
    if ((int64_t)H * W > (int64_t)1 << 31) return HYRES_E_UNSUPPORTED;
    if (!(o->mu1 > 0.0) || !(o->mu2 > 0.0) || !(o->lam >= 0.0) || o->iters < 1 ||
        !std::isfinite(o->mu1) || !std::isfinite(o->mu2) || !std::isfinite(o->lam))
        return HYRES_E_SHAPE;
    int S = 0, M = 0;
    if (!l1l1_shape(p, dtype, &S, &M)) return HYRES_E_UNSUPPORTED;
    return HYRES_OK;
}

static hyres_status enqueue_l1l1(hyres_handle* h, const void* Hc, int H, int W, int p, int64_t pitch,
                                 int64_t row_pitch, int dtype, const hyres_l1l1_options* o, void* X, int64_t x_pitch,
                                 int64_t x_row_pitch, hipStream_t s) {
    L1Args a{};
    a.Hc = Hc; a.pitch = pitch; a.row_pitch = row_pitch;
    a.X = X; a.xpitch = x_pitch; a.xrow_pitch = x_row_pitch;
    a.H = H; a.W = W; a.p = p; a.iters = o->iters; a.dtype = dtype;
    a.lam = o->lam; a.mu1 = o->mu1; a.mu2 = o->mu2;
    return launch_l1l1(a, h->num_cu, s) == hipSuccess ? HYRES_OK : HYRES_E_HIP;
}

HYRES_API hyres_status hyres_l1l1_spectral(hyres_handle* h, const void* Hc, int H, int W, int p, int64_t pitch,
                                           int64_t row_pitch, int dtype, const hyres_l1l1_options* opt, void* X,
                                           int64_t x_pitch, int64_t x_row_pitch, hyres_stream_t stream) {
    if (!h || !Hc || !X) return HYRES_E_NULL;
    hyres_status st = check_l1l1(H, W, p, pitch, row_pitch, dtype, opt, x_pitch, x_row_pitch);
    if (st) return st;
    // in place only with the same layout (each pixel is read whole before it is written)
    if (X == Hc && (pitch != x_pitch || row_pitch != x_row_pitch)) return HYRES_E_SHAPE;
    if ((st = set_device(h))) return st;
    return enqueue_l1l1(h, Hc, H, W, p, pitch, row_pitch, dtype, opt, X, x_pitch, x_row_pitch,
                        (hipStream_t)stream);
}

HYRES_API hyres_status hyres_hyminor(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                     int64_t row_pitch, int dtype, const hyres_options* opt,
                                     const double* sigma_in, const double* lambda_in, const hyres_l1l1_options* l1,
                                     void* X, int64_t x_pitch, int64_t x_row_pitch, const hyres_outputs* out,
                                     void* workspace, size_t workspace_bytes, hyres_stream_t stream) {
    if (!h || !Y || !X) return HYRES_E_NULL;
    hyres_status st = check_l1l1(H, W, p, pitch, row_pitch, dtype, l1, x_pitch, x_row_pitch);
    if (st) return st;
    st = denoise_one(h, Y, H, W, p, pitch, row_pitch, dtype, opt, sigma_in, lambda_in, X, x_pitch, x_row_pitch,
                     out, false, workspace, workspace_bytes, stream);
    if (st) return st;
    return enqueue_l1l1(h, X, H, W, p, x_pitch, x_row_pitch, dtype, l1, X, x_pitch, x_row_pitch,
                        (hipStream_t)stream);
}

// ------------------------------------------------------------- WSRRR
namespace {
// The HyRes workspace of the cube, then Y^T Zh (r x p) and its per-slot partial sums.
// Slots (blocks, partial sums) of the pixel cross products Y^T Zh and the
// adjoint's: about 256 pixels each, at most two blocks per compute unit of a
// 256-unit device (each block runs its tiles in turn; fewer partials make the
// sum over slots cheaper).
int cross_slots(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(512, cdiv(n, 256))); }

struct WsrrrPlan {
    Exec x;
    int slots = 1;
    size_t o_M = 0, o_part = 0;
};

hyres_status plan_wsrrr(WsrrrPlan& w, hyres_handle* h, int H, int W, int p, const hyres_options* opt, int dtype,
                        int iters) {
    if (!opt) return HYRES_E_NULL;
    hyres_status st = check_opts(opt, p, dtype);
    if (st) return st;
    if (opt->precision != HYRES_PREC_NATIVE || (opt->flags & (HYRES_FLAG_RANK_HYSIME | HYRES_FLAG_RANK_SURE)))
        return HYRES_E_UNSUPPORTED;
    if (iters < 0) return HYRES_E_SHAPE;
    one_cube(w.x, h, H, W, p, opt->rank, opt->levels, dtype, opt->scope, opt->precision);
    if ((st = plan_cubes(w.x, kAllParts))) return st;
    const CubePlan& c = w.x.plan[0];
    w.slots = cross_slots(c.n);
    w.o_M = w.x.lay.add((size_t)c.r * p * 8);
    w.o_part = w.x.lay.add((size_t)w.slots * c.r * p * 8);
    return HYRES_OK;
}
}  // namespace

HYRES_API hyres_status hyres_wsrrr_workspace_size(int H, int W, int p, const hyres_options* opt, int dtype,
                                                  size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    WsrrrPlan w;
    hyres_status st = plan_wsrrr(w, nullptr, H, W, p, opt, dtype, 0);
    if (st) return st;
    *bytes = w.x.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_wsrrr(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                   int64_t row_pitch, int dtype, const hyres_options* opt, int iters,
                                   const double* sigma_in, const double* lambda_in, void* X, int64_t x_pitch,
                                   int64_t x_row_pitch, const hyres_outputs* out, void* workspace,
                                   size_t workspace_bytes, hyres_stream_t stream) {
    if (!h || !X) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    if (x_pitch < p || x_row_pitch < (int64_t)(W - 1) * x_pitch + p) return HYRES_E_SHAPE;
    WsrrrPlan w;
    if ((st = plan_wsrrr(w, h, H, W, p, opt, dtype, iters))) return st;
    Exec& x = w.x;
    x.plan[0].has_lambda = lambda_in != nullptr;
    if ((st = check_ws(workspace, workspace_bytes, x.lay.total))) return st;
    if ((st = set_device(h))) return st;
    x.ws = workspace;
    x.desc.assign(1, solve_desc(x.plan[0], workspace, Y, pitch, row_pitch, X, x_pitch, x_row_pitch, sigma_in,
                                lambda_in, opt->flags, out));
    const CubeDesc& d = x.desc[0];
    hipStream_t s = (hipStream_t)stream;
    // HyRes up to the denoised component images (noise, subspace, thresholds)
    build_program(x, kAllStages & ~S_BP);
    if ((st = upload_exec(x, s)) || (st = run_program(x, s, false))) return st;
    AdjDesc a;
    std::memset(&a, 0, sizeof(a));
    a.W = W; a.p = p; a.r = d.r; a.n = d.n; a.nz = d.nz;
    a.slots = w.slots;
    a.part = at<double>(workspace, w.o_part);
    double* M = at<double>(workspace, w.o_M);
    if (iters > 0) {
        // every alternation runs the same program: its tables go up once
        // (stream-ordered after the program above, which has read its own)
        build_program(x, S_PROJ | S_DWT | S_IDWT);
        if ((st = upload_exec(x, s))) return st;
    }
    for (int it = 0; it < iters; ++it) {
        // V <- polar factor of Yw^T Zh, then F <- soft(W^T Yw V, lambda) with the thresholds held
        HIPCHK(launch_planes_cube(dtype, a, d.Z, Y, pitch, row_pitch, M, s));
        HIPCHK(launch_polar(x.descs(), M, s));
        if ((st = run_program(x, s, false))) return st;
    }
    build_program(x, S_BP);
    if ((st = upload_exec(x, s))) return st;
    return run_program(x, s, false);
}

// ------------------------------------------------------------- FORPDN
namespace {
// Workspace of one FORPDN solve: the noise program (unless sigma is given),
// the position-major coefficients, two approximation buffers, the Gram
// program over the L + 1 coefficient groups, and the small outputs.
struct ForpdnPlan {
    Exec noise, grams;
    bool need_noise = true;
    int H = 0, W = 0, p = 0, L = 0, dtype = 0, G = 0;
    int lh[kMaxLevels + 1] = {0}, lw[kMaxLevels + 1] = {0};
    int64_t loff[kMaxLevels + 1] = {0}, ll_off = 0, nc = 0;
    int64_t goff[kForpdnMaxGroups + 1] = {0};
    size_t o_noise = 0, o_grams = 0, o_coef = 0, o_tmp[2] = {0, 0}, o_sigma = 0, o_lambda = 0, o_sure = 0;
    size_t total = 0;
};

uint32_t pmag_of(int p) { return (uint32_t)(0xffffffffu / (uint32_t)p) + 1u; }

hyres_status plan_forpdn(ForpdnPlan& f, hyres_handle* h, int H, int W, int p, int L, int dtype, bool need_noise) {
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    if (!level_geometry(H, W, L, f.lh, f.lw, f.loff, &f.ll_off, &f.nc)) return HYRES_E_SHAPE;
    if ((int64_t)H * W > (int64_t)1 << 31 || f.nc * p > ((int64_t)1 << 40)) return HYRES_E_UNSUPPORTED;
    f.H = H; f.W = W; f.p = p; f.L = L; f.dtype = dtype; f.G = L + 1;
    f.need_noise = need_noise;
    for (int l = 1; l <= L; ++l) f.goff[l - 1] = f.loff[l];
    f.goff[L] = f.ll_off;
    f.goff[L + 1] = f.nc;
    Layout lay;
    const int es = esize(dtype);
    if (need_noise) {
        one_cube(f.noise, h, H, W, p, 1, 1, dtype, 0);
        hyres_status st = plan_cubes(f.noise, P_GRAM | P_SMALL);
        if (st) return st;
        f.o_noise = lay.add(f.noise.lay.total);
    }
    f.o_coef = lay.add((size_t)f.nc * p * es);
    f.o_tmp[0] = lay.add((size_t)f.lh[1] * f.lw[1] * p * es);
    f.o_tmp[1] = lay.add(L >= 2 ? (size_t)f.lh[2] * f.lw[2] * p * es : 0);
    // the coefficient groups as "cubes" of positions for the Gram kernels:
    // the three detail blocks of level l (3 h_l rows of w_l), then LL_L
    Exec& g = f.grams;
    g.h = h;
    g.count = f.G;
    g.dtype = dtype;
    g.precision = HYRES_PREC_NATIVE;
    g.plan.resize(f.G);
    for (int j = 0; j < f.G; ++j) {
        CubePlan& c = g.plan[j];
        c.H = j < L ? 3 * f.lh[j + 1] : f.lh[L];
        c.W = j < L ? f.lw[j + 1] : f.lw[L];
        c.p = p; c.r = 1; c.L = 0; c.dtype = dtype; c.scope = 0; c.precision = HYRES_PREC_NATIVE;
    }
    plan_exec(g, P_GRAM);
    f.o_grams = lay.add(g.lay.total);
    f.o_sigma = lay.add((size_t)p * 8);
    f.o_lambda = lay.add((size_t)f.G * 8);
    f.o_sure = lay.add((size_t)f.G * 8);
    f.total = lay.total;
    return HYRES_OK;
}
}  // namespace

HYRES_API hyres_status hyres_forpdn_workspace_size(int H, int W, int p, int levels, int dtype, int sigma_given,
                                                   size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    ForpdnPlan f;
    hyres_status st = plan_forpdn(f, nullptr, H, W, p, levels, dtype, !sigma_given);
    if (st) return st;
    *bytes = f.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_forpdn(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                    int64_t row_pitch, int dtype, int levels, const double* sigma_in,
                                    const double* lambda_in, void* X, int64_t x_pitch, int64_t x_row_pitch,
                                    double* sigma_out, double* lambda_out, double* sure_out, int* status,
                                    void* workspace, size_t workspace_bytes, hyres_stream_t stream) {
    if (!h || !X) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    if (x_pitch < p || x_row_pitch < (int64_t)(W - 1) * x_pitch + p) return HYRES_E_SHAPE;
    ForpdnPlan f;
    if ((st = plan_forpdn(f, h, H, W, p, levels, dtype, sigma_in == nullptr))) return st;
    if ((st = check_ws(workspace, workspace_bytes, f.total))) return st;
    if ((st = set_device(h))) return st;
    hipStream_t s = (hipStream_t)stream;
    const int es = esize(dtype);
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    double* sigma = sigma_out ? sigma_out : reinterpret_cast<double*>(ws + f.o_sigma);
    double* lambda = lambda_out ? lambda_out : reinterpret_cast<double*>(ws + f.o_lambda);
    double* sure = sure_out ? sure_out : reinterpret_cast<double*>(ws + f.o_sure);
    unsigned char* coef = ws + f.o_coef;
    unsigned char* tmp[2] = {ws + f.o_tmp[0], ws + f.o_tmp[1]};
    const double* sg = sigma_in;
    // F1: noise (the regression estimator of HyRes)
    if (f.need_noise) {
        Exec& x = f.noise;
        x.ws = ws + f.o_noise;
        CubeDesc d = make_desc(x.plan[0], x.ws);
        d.Y = Y; d.pitch = pitch; d.row_pitch = row_pitch;
        d.vec4 = vec4_ok(Y, W, p, pitch, row_pitch, dtype);
        d.dense = dense_ok(Y, W, p, pitch, row_pitch, dtype);
        d.sigma = sigma;
        d.status = status;
        d.mode = kModeSigma;
        x.desc.assign(1, d);
        build_program(x, S_GRAM | S_SMALL);
        if ((st = upload_exec(x, s))) return st;
        if ((st = run_program(x, s, false))) return st;
        sg = sigma;
    } else if (sigma_out) {
        if (hipMemcpyAsync(sigma_out, sigma_in, (size_t)p * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return HYRES_E_HIP;
    }
    // F2: analysis, level by level (the first divides by sigma on load);
    // LL_l (l < L) in tmp[(l - 1) & 1], LL_L in the coefficients
    const uint32_t pm = pmag_of(p);
    for (int l = 1; l <= levels; ++l) {
        VLevel a{};
        if (l == 1) {
            a.in = Y; a.ip = pitch; a.irow = row_pitch;
        } else {
            a.in = tmp[(l - 2) & 1]; a.ip = p; a.irow = (int64_t)f.lw[l - 1] * p;
        }
        a.scale = l == 1 ? sg : nullptr;
        a.ll = l == levels ? coef + (size_t)f.ll_off * p * es : tmp[(l - 1) & 1];
        a.det = coef + (size_t)f.loff[l] * p * es;
        a.Hin = f.lh[l - 1]; a.Win = f.lw[l - 1]; a.h = f.lh[l]; a.w = f.lw[l]; a.p = p; a.pmag = pm;
        if (launch_vdwt_level(dtype, a, h->num_cu, s) != hipSuccess) return HYRES_E_HIP;
    }
    // F5: band Gram of every group, then the thresholds
    {
        Exec& x = f.grams;
        x.ws = ws + f.o_grams;
        x.desc.resize(f.G);
        for (int j = 0; j < f.G; ++j) {
            CubeDesc d = make_desc(x.plan[j], x.ws);
            const void* gy = coef + (size_t)f.goff[j] * p * es;
            const int64_t rp = (int64_t)x.plan[j].W * p;
            d.Y = gy; d.pitch = p; d.row_pitch = rp;
            d.vec4 = vec4_ok(gy, x.plan[j].W, p, p, rp, dtype);
            d.dense = dense_ok(gy, x.plan[j].W, p, p, rp, dtype);
            x.desc[j] = d;
        }
        build_program(x, S_GRAM);
        if ((st = upload_exec(x, s))) return st;
        if ((st = run_program(x, s, false))) return st;
        FLambda la{};
        for (int j = 0; j < f.G; ++j) {
            la.G[j] = x.desc[j].G;
            la.count[j] = f.goff[j + 1] - f.goff[j];
        }
        la.lambda_in = lambda_in;
        la.lambda = lambda;
        la.sure = sure;
        la.p = p;
        if (launch_forpdn_lambda(la, f.G, s) != hipSuccess) return HYRES_E_HIP;
    }
    // F4: the smoother on every coefficient vector
    {
        FFilter ff{};
        ff.coef = coef;
        ff.npos = f.nc;
        for (int j = 0; j <= f.G; ++j) ff.goff[j] = f.goff[j];
        ff.lambda = lambda;
        ff.p = p;
        ff.groups = f.G;
        ff.pmag = pm;
        if (launch_forpdn_filter(dtype, ff, h->num_cu, s) != hipSuccess) return HYRES_E_HIP;
    }
    // F6: synthesis, coarsest level first; the last level writes X times sigma
    for (int l = levels; l >= 1; --l) {
        VSyn a{};
        a.ll = l == levels ? coef + (size_t)f.ll_off * p * es : tmp[(l - 1) & 1];
        a.det = coef + (size_t)f.loff[l] * p * es;
        if (l == 1) {
            a.out = X; a.op = x_pitch; a.orow = x_row_pitch;
        } else {
            a.out = tmp[(l - 2) & 1]; a.op = p; a.orow = (int64_t)f.lw[l - 1] * p;
        }
        a.scale = l == 1 ? sg : nullptr;
        a.Hin = f.lh[l - 1]; a.Win = f.lw[l - 1]; a.h = f.lh[l]; a.w = f.lw[l]; a.p = p; a.pmag = pm;
        if (launch_vidwt_level(dtype, a, h->num_cu, s) != hipSuccess) return HYRES_E_HIP;
    }
    return HYRES_OK;
}

// ------------------------------------------------------------- batches
struct hyres_batch {
    hyres_handle* h = nullptr;
    Exec x;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~hyres_batch() {
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

static hyres_status plan_batch(Exec& x, hyres_handle* h, const hyres_cube* cubes, int count, int dtype,
                               const hyres_options* opt, bool need_ptrs) {
    if (!cubes || !opt) return HYRES_E_NULL;
    if (count < 1 || count > (1 << 16)) return HYRES_E_SHAPE;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    hyres_status st = check_prec_scope(opt->precision, opt->scope, dtype);
    if (st) return st;
    x.h = h;
    x.count = count;
    x.dtype = dtype;
    x.precision = opt->precision;
    x.plan.resize(count);
    for (int i = 0; i < count; ++i) {
        const hyres_cube& k = cubes[i];
        if (need_ptrs) {
            if (!k.Y || !k.X) return HYRES_E_NULL;
            if (k.x_pitch < k.p || k.x_row_pitch < (int64_t)(k.W - 1) * k.x_pitch + k.p) return HYRES_E_SHAPE;
        }
        const int64_t pitch = need_ptrs ? k.pitch : k.p;
        const int64_t rp = need_ptrs ? k.row_pitch : (int64_t)k.W * k.p;
        if ((st = check_shape(k.H, k.W, k.p, pitch, rp))) return st;
        if ((st = check_rank_levels(k.rank, k.levels, k.p))) return st;
        CubePlan& c = x.plan[i];
        c.H = k.H; c.W = k.W; c.p = k.p; c.r = k.rank; c.L = k.levels; c.dtype = dtype; c.scope = opt->scope;
        c.precision = opt->precision;
        c.has_lambda = k.lambda_in != nullptr;
    }
    return plan_cubes(x, kAllParts);
}

HYRES_API hyres_status hyres_batch_workspace_size(const hyres_cube* cubes, int count, int dtype,
                                                  const hyres_options* opt, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    Exec x;
    hyres_status st = plan_batch(x, nullptr, cubes, count, dtype, opt, false);
    if (st) return st;
    *bytes = x.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_batch_create(hyres_handle* h, const hyres_cube* cubes, int count, int dtype,
                                          const hyres_options* opt, void* workspace, size_t workspace_bytes,
                                          hyres_stream_t stream, hyres_batch** batch) {
    if (!h || !batch) return HYRES_E_NULL;
    *batch = nullptr;
    std::unique_ptr<hyres_batch> b(new (std::nothrow) hyres_batch);
    if (!b) return HYRES_E_UNSUPPORTED;
    b->h = h;
    Exec& x = b->x;
    hyres_status st = plan_batch(x, h, cubes, count, dtype, opt, true);
    if (st) return st;
    if ((st = check_ws(workspace, workspace_bytes, x.lay.total))) return st;
    if ((st = set_device(h))) return st;
    x.ws = workspace;
    x.desc.resize(count);
    for (int i = 0; i < count; ++i) {
        const hyres_cube& k = cubes[i];
        x.desc[i] = solve_desc(x.plan[i], workspace, k.Y, k.pitch, k.row_pitch, k.X, k.x_pitch, k.x_row_pitch,
                               k.sigma_in, k.lambda_in, opt->flags, &k.out);
    }
    group_by_small_class(x);
    build_program(x, kAllStages);
    if ((st = upload_exec(x, (hipStream_t)stream))) return st;
    *batch = b.release();
    return HYRES_OK;
}

HYRES_API hyres_status hyres_batch_run(hyres_batch* b, hyres_stream_t stream) {
    if (!b) return HYRES_E_NULL;
    hyres_status st = set_device(b->h);
    if (st) return st;
    return run_program(b->x, (hipStream_t)stream, true);
}

HYRES_API hyres_status hyres_batch_launch_graph(hyres_batch* b, hyres_stream_t stream) {
    if (!b) return HYRES_E_NULL;
    hyres_status st = set_device(b->h);
    if (st) return st;
    if (!b->exec) {
        if (!b->cap) HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        st = run_program(b->x, b->cap, false, true);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (st || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st ? st : HYRES_E_HIP;
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            b->drop_graph();
            return HYRES_E_HIP;
        }
    }
    HIPCHK(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return HYRES_OK;
}

HYRES_API void hyres_batch_destroy(hyres_batch* b) { delete b; }

HYRES_API hyres_status hyres_denoise_batched(hyres_handle* h, const hyres_cube* cubes, int count, int dtype,
                                             const hyres_options* opt, void* workspace, size_t workspace_bytes,
                                             hyres_stream_t stream) {
    hyres_batch* b = nullptr;
    hyres_status st = hyres_batch_create(h, cubes, count, dtype, opt, workspace, workspace_bytes, stream, &b);
    if (st) return st;
    st = run_program(b->x, (hipStream_t)stream, true);
    delete b;
    return st;
}

HYRES_API hyres_status hyres_batch_check_program(const hyres_cube* cubes, int count, int dtype,
                                                 const hyres_options* opt, hyres_program_stats* stats) {
    hyres_handle h;
    init_host_handle(h);
    Exec x;
    hyres_status st = plan_batch(x, &h, cubes, count, dtype, opt, false);
    if (st) return st;
    x.desc.resize(count);
    for (int i = 0; i < count; ++i) {
        const hyres_cube& k = cubes[i];
        hyres_outputs o{};
        x.desc[i] = solve_desc(x.plan[i], nullptr, nullptr, k.p, (int64_t)k.W * k.p, nullptr, k.p,
                               (int64_t)k.W * k.p, nullptr, k.lambda_in, opt->flags, &o);
    }
    group_by_small_class(x);
    build_program(x, kAllStages);
    return dry_check(x, stats);
}

// ------------------------------------------------------------- adjoint
namespace {

// Backward workspace: two transform descriptors (analysis with zero extra
// sample, synthesis with folding), their tables, and the adjoint buffers.
struct BwdPlan {
    Exec fwd;                 // layout of the forward workspace
    Exec xa, xs;              // transform executors over the backward buffers
    Layout lay;
    int slots = 1, nchunk = 1;
    size_t o_desc = 0, o_tab = 0, o_A = 0, o_dB = 0, o_tmp = 0, o_part = 0, o_dQ = 0, o_dPt = 0, o_lpart = 0,
           o_gsc = 0, o_W = 0, o_Ginv = 0, o_dC = 0, o_dG2 = 0;
};

hyres_status plan_backward(BwdPlan& b, hyres_handle* h, int H, int W, int p, const hyres_options* opt, int dtype) {
    if (!opt) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    hyres_status st = check_opts(opt, p, dtype);
    if (st) return st;
    // a mixed-precision forward keeps a Rayleigh-Ritz basis that is not an
    // eigenbasis of the Gram the eigen-adjoint differentiates
    if (opt->precision == HYRES_PREC_MIXED) return HYRES_E_UNSUPPORTED;
    // a data-chosen rank is piecewise constant; the adjoint takes the rank as given
    if (opt->flags & (HYRES_FLAG_RANK_HYSIME | HYRES_FLAG_RANK_SURE)) return HYRES_E_UNSUPPORTED;
    one_cube(b.fwd, h, H, W, p, opt->rank, opt->levels, dtype, opt->scope, opt->precision);
    if ((st = plan_cubes(b.fwd, kAllParts))) return st;
    const CubePlan& c = b.fwd.plan[0];
    const int r = c.r, es = esize(dtype);
    Layout& L = b.lay;
    b.o_desc = L.add(2 * sizeof(CubeDesc));
    b.o_tab = L.add(2 * sizeof(int) * table_ints(1));
    b.o_A = L.add((size_t)r * c.nz * es);
    b.o_dB = L.add((size_t)r * c.ncs * es);
    b.o_tmp = L.add((size_t)std::max<int64_t>(1, r * c.tps) * es);
    b.slots = cross_slots(c.n);
    b.o_part = L.add((size_t)b.slots * r * p * 8);
    b.o_dQ = L.add((size_t)r * p * 8);
    b.o_dPt = L.add((size_t)r * p * 8);
    const int64_t lim = c.scope == HYRES_SCOPE_DETAIL ? c.ll_off : c.nc;
    b.nchunk = (int)std::max<int64_t>(1, cdiv(lim, adj_chunk()));
    b.o_lpart = L.add((size_t)r * b.nchunk * 8);
    b.o_gsc = L.add((size_t)p * 8);
    b.o_W = L.add((size_t)p * r * 8);
    b.o_Ginv = L.add((size_t)p * p * 8);
    b.o_dC = L.add((size_t)p * p * 8);
    b.o_dG2 = L.add((size_t)p * p * 8);
    return HYRES_OK;
}

}  // namespace

HYRES_API hyres_status hyres_denoise_backward_workspace_size(int H, int W, int p, const hyres_options* opt, int dtype,
                                                             size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    BwdPlan b;
    hyres_status st = plan_backward(b, nullptr, H, W, p, opt, dtype);
    if (st) return st;
    *bytes = b.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_denoise_backward(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                              int64_t row_pitch, int dtype, const hyres_options* opt,
                                              const void* fwd_workspace, size_t fwd_workspace_bytes,
                                              const hyres_outputs* fwd_out, const void* dX, int64_t dx_pitch,
                                              int64_t dx_row_pitch, void* dY, int64_t dy_pitch,
                                              int64_t dy_row_pitch, double* dlambda, int* status, void* workspace,
                                              size_t workspace_bytes, hyres_stream_t stream) {
    if (!h || !dX || !dY || !fwd_out || !fwd_workspace) return HYRES_E_NULL;
    if (!fwd_out->sigma || !fwd_out->V || !fwd_out->evals || !fwd_out->lambda) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    if (dx_pitch < p || dx_row_pitch < (int64_t)(W - 1) * dx_pitch + p) return HYRES_E_SHAPE;
    if (dy_pitch < p || dy_row_pitch < (int64_t)(W - 1) * dy_pitch + p) return HYRES_E_SHAPE;
    BwdPlan b;
    if ((st = plan_backward(b, h, H, W, p, opt, dtype))) return st;
    if ((st = check_ws(workspace, workspace_bytes, b.lay.total))) return st;
    if (fwd_workspace_bytes < b.fwd.lay.total || reinterpret_cast<uintptr_t>(fwd_workspace) % kAlign)
        return HYRES_E_WORKSPACE;
    if ((st = set_device(h))) return st;
    void* fws = const_cast<void*>(fwd_workspace);
    const CubePlan& c = b.fwd.plan[0];
    // transform executors: analysis of dZh with a zero extra sample, synthesis with folding
    CubeDesc d = make_desc(c, workspace);
    d.Z = at<void>(workspace, b.o_A);
    d.coef = at<void>(workspace, b.o_dB);
    d.tmp = at<void>(workspace, b.o_tmp);
    d.lambda = nullptr;
    d.status = status;
    for (int k = 0; k < 2; ++k) {
        Exec& x = k == 0 ? b.xa : b.xs;
        x.h = h;
        x.count = 1;
        x.dtype = dtype;
        x.ws = workspace;
        x.plan.assign(1, c);
        x.o_desc = b.o_desc + k * sizeof(CubeDesc);
        x.o_tab = b.o_tab + k * sizeof(int) * table_ints(1);
        CubeDesc dk = d;
        dk.mode = k == 0 ? kModeZeroPad : kModeFold;
        x.desc.assign(1, dk);
        build_program(x, k == 0 ? S_DWT : S_IDWT);
    }
    AdjDesc a;
    std::memset(&a, 0, sizeof(a));
    a.H = H; a.W = W; a.p = p; a.r = c.r; a.L = c.L; a.scope = c.scope;
    a.n = c.n; a.nz = c.nz; a.ncs = c.ncs; a.nc = c.nc; a.ll_off = c.ll_off;
    a.Y = Y; a.pitch = pitch; a.row_pitch = row_pitch;
    a.Zh = at<void>(fws, c.o_Z);
    a.B = at<void>(fws, c.o_coef);
    a.G = at<double>(fws, c.o_G);
    a.sigma = fwd_out->sigma;
    a.V = fwd_out->V;
    a.evals = fwd_out->evals;
    a.lambda = fwd_out->lambda;
    a.P64 = at<double>(fws, c.o_P64);
    a.Q64 = at<double>(fws, c.o_Q64);
    a.dX = dX; a.dxp = dx_pitch; a.dxrp = dx_row_pitch;
    a.dY = dY; a.dyp = dy_pitch; a.dyrp = dy_row_pitch;
    a.dlambda = dlambda;
    a.A = at<void>(workspace, b.o_A);
    a.dB = at<void>(workspace, b.o_dB);
    a.part = at<double>(workspace, b.o_part);
    a.dQ = at<double>(workspace, b.o_dQ);
    a.dPt = at<double>(workspace, b.o_dPt);
    a.lpart = at<double>(workspace, b.o_lpart);
    a.gsc = at<double>(workspace, b.o_gsc);
    a.Wsol = at<double>(workspace, b.o_W);
    a.Ginv = at<double>(workspace, b.o_Ginv);
    a.dC = at<double>(workspace, b.o_dC);
    a.dG2 = at<double>(workspace, b.o_dG2);
    a.slots = b.slots;
    a.nchunk = b.nchunk;
    a.status = status;
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_exec(b.xa, s)) || (st = upload_exec(b.xs, s))) return st;
    HIPCHK(launch_adjoint_pre(a, dtype, s));
    if ((st = run_program(b.xa, s, false))) return st;
    HIPCHK(launch_adjoint_thresh(a, dtype, s));
    if ((st = run_program(b.xs, s, false))) return st;
    HIPCHK(launch_adjoint_post(a, dtype, s));
    return HYRES_OK;
}

HYRES_API hyres_status hyres_sure_grad_workspace_size(int batch, int64_t Nc, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    if (batch < 1 || Nc < 1 || Nc > ((int64_t)1 << 31)) return HYRES_E_SHAPE;
    *bytes = (size_t)batch * cdiv(Nc, adj_chunk()) * 8;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_sure_grad(hyres_handle* h, const void* coeffs, int batch, int64_t Nc, int64_t stride,
                                       int dtype, const double* lambda, double* dsure_out, void* workspace,
                                       size_t workspace_bytes, hyres_stream_t stream) {
    if (!h || !coeffs || !lambda || !dsure_out) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (batch < 1 || Nc < 1 || Nc > ((int64_t)1 << 31) || stride < Nc) return HYRES_E_SHAPE;
    const int nchunk = (int)cdiv(Nc, adj_chunk());
    hyres_status st = check_ws(workspace, workspace_bytes, (size_t)batch * nchunk * 8);
    if (st) return st;
    if ((st = set_device(h))) return st;
    HIPCHK(launch_sure_grad(dtype, coeffs, stride, Nc, batch, lambda, static_cast<double*>(workspace), nchunk,
                            dsure_out, (hipStream_t)stream));
    return HYRES_OK;
}

// ------------------------------------------------------------- sliding window
namespace {


// Tile starts along one axis: steps of tile - overlap, the last start clamped
// so that the tile ends at the border; one tile when it covers the axis.
int tile_starts(int size, int tile, int overlap, int* starts) {
    if (tile >= size) {
        starts[0] = 0;
        return 1;
    }
    const int step = tile - overlap;
    int n = 0;
    for (int k = 0;; ++k) {
        const int s = std::min(k * step, size - tile);
        if (n >= kMaxTilesAxis) return n + 1;
        starts[n++] = s;
        if (s + tile >= size) break;
    }
    return n;
}

// Greedy colouring: each tile takes the smallest colour that no earlier tile
// overlapping it has, so tiles of one colour never overlap.
int tile_colours(const int* starts, int n, int tile, unsigned char* colour) {
    int nc = 0;
    for (int i = 0; i < n; ++i) {
        unsigned used = 0;
        for (int j = 0; j < i; ++j)
            if (starts[i] < starts[j] + tile) used |= 1u << colour[j];
        int c = 0;
        while ((used >> c) & 1u) ++c;
        colour[i] = (unsigned char)c;
        nc = std::max(nc, c + 1);
    }
    return nc;
}

struct BlendAxis {
    int n, tile, size, overlap;
    int start[kMaxTilesAxis];
    unsigned char colour[kMaxTilesAxis];
};

// Weight of sample k of a tile: sin^2 ramps over the first and the last
// `overlap` samples, except on a side touching the image border.
__device__ double ramp_weight(int start, int k, int tile, int size, int overlap) {
    double w = 1.0;
    if (start > 0 && k < overlap) {
        const double t = sin(0.5 * M_PI * (k + 0.5) / overlap);
        w = t * t;
    }
    if (start + tile < size && k >= tile - overlap) {
        const double t = sin(0.5 * M_PI * (tile - 1 - k + 0.5) / overlap);
        w = t * t;
    }
    return w;
}

// Per tile and sample: weight divided by the sum over all tiles covering the
// sample, and the mask of the colours of those tiles.
__global__ void k_blend_axis(BlendAxis a, double* __restrict__ w, unsigned char* __restrict__ cov) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n * a.tile) return;
    const int t = idx / a.tile, k = idx - t * a.tile;
    const int g = a.start[t] + k;
    double sum = 0.0;
    unsigned mask = 0;
    for (int u = 0; u < a.n; ++u) {
        const int ku = g - a.start[u];
        if (ku < 0 || ku >= a.tile) continue;
        sum += ramp_weight(a.start[u], ku, a.tile, a.size, a.overlap);
        mask |= 1u << a.colour[u];
    }
    w[idx] = ramp_weight(a.start[t], k, a.tile, a.size, a.overlap) / sum;
    cov[idx] = (unsigned char)mask;
}

struct TileGrid {
    int ny = 0, nx = 0, th = 0, tw = 0, ncy = 0, ncx = 0;
    BlendAxis ay{}, ax{};
    size_t o_bwy = 0, o_bwx = 0, o_bcy = 0, o_bcx = 0;
};

hyres_status plan_tiled(Exec& x, TileGrid& g, hyres_handle* h, int H, int W, int p, int tile, int overlap,
                        const hyres_options* opt, int dtype) {
    if (!opt) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    if (tile < 4 || overlap < 0 || 2 * overlap > tile) return HYRES_E_SHAPE;
    hyres_status st = check_opts(opt, p, dtype);
    if (st) return st;
    g.th = std::min(tile, H);
    g.tw = std::min(tile, W);
    g.ny = tile_starts(H, tile, overlap, g.ay.start);
    g.nx = tile_starts(W, tile, overlap, g.ax.start);
    if (g.ny > kMaxTilesAxis || g.nx > kMaxTilesAxis) return HYRES_E_UNSUPPORTED;
    g.ncy = tile_colours(g.ay.start, g.ny, g.th, g.ay.colour);
    g.ncx = tile_colours(g.ax.start, g.nx, g.tw, g.ax.colour);
    if (g.ncy > kMaxColours || g.ncx > kMaxColours) return HYRES_E_UNSUPPORTED;
    g.ay.n = g.ny; g.ay.tile = g.th; g.ay.size = H; g.ay.overlap = overlap;
    g.ax.n = g.nx; g.ax.tile = g.tw; g.ax.size = W; g.ax.overlap = overlap;
    x.h = h;
    x.count = g.ny * g.nx;
    x.dtype = dtype;
    x.precision = opt->precision;
    x.plan.resize(x.count);
    x.pass_of.resize(x.count);
    for (int iy = 0; iy < g.ny; ++iy)
        for (int ix = 0; ix < g.nx; ++ix) {
            const int t = iy * g.nx + ix;
            CubePlan& c = x.plan[t];
            c.H = g.th; c.W = g.tw; c.p = p; c.r = opt->rank; c.L = opt->levels; c.dtype = dtype;
            c.scope = opt->scope; c.precision = opt->precision;
            x.pass_of[t] = g.ay.colour[iy] * g.ncx + g.ax.colour[ix];
        }
    if ((st = plan_cubes(x, kAllParts))) return st;
    g.o_bwy = x.lay.add((size_t)g.ny * g.th * 8);
    g.o_bwx = x.lay.add((size_t)g.nx * g.tw * 8);
    g.o_bcy = x.lay.add((size_t)g.ny * g.th);
    g.o_bcx = x.lay.add((size_t)g.nx * g.tw);
    return HYRES_OK;
}

}  // namespace

HYRES_API hyres_status hyres_tile_grid(int size, int tile, int overlap, int* starts, int* count) {
    if (!count) return HYRES_E_NULL;
    if (size < 1 || tile < 4 || overlap < 0 || 2 * overlap > tile) return HYRES_E_SHAPE;
    int buf[kMaxTilesAxis];
    const int n = tile_starts(size, tile, overlap, buf);
    if (n > kMaxTilesAxis) return HYRES_E_UNSUPPORTED;
    *count = n;
    if (starts)
        for (int i = 0; i < n; ++i) starts[i] = buf[i];
    return HYRES_OK;
}

HYRES_API hyres_status hyres_tiled_workspace_size(int H, int W, int p, int tile, int overlap,
                                                  const hyres_options* opt, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    Exec x;
    TileGrid g;
    hyres_status st = plan_tiled(x, g, nullptr, H, W, p, tile, overlap, opt, dtype);
    if (st) return st;
    *bytes = x.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_denoise_tiled(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                           int64_t row_pitch, int dtype, int tile, int overlap,
                                           const hyres_options* opt, void* X, int64_t x_pitch, int64_t x_row_pitch,
                                           double* lambda_out, double* sigma_out, int* status, void* workspace,
                                           size_t workspace_bytes, hyres_stream_t stream) {
    if (!h || !X) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    if (x_pitch < p || x_row_pitch < (int64_t)(W - 1) * x_pitch + p) return HYRES_E_SHAPE;
    Exec x;
    TileGrid g;
    if ((st = plan_tiled(x, g, h, H, W, p, tile, overlap, opt, dtype))) return st;
    if ((st = check_ws(workspace, workspace_bytes, x.lay.total))) return st;
    if ((st = set_device(h))) return st;
    x.ws = workspace;
    const int es = esize(dtype);
    x.desc.resize(x.count);
    for (int iy = 0; iy < g.ny; ++iy)
        for (int ix = 0; ix < g.nx; ++ix) {
            const int t = iy * g.nx + ix;
            const int64_t sy = g.ay.start[iy], sx = g.ax.start[ix];
            const void* Yt = static_cast<const unsigned char*>(Y) + (sy * row_pitch + sx * pitch) * es;
            void* Xt = static_cast<unsigned char*>(X) + (sy * x_row_pitch + sx * x_pitch) * es;
            hyres_outputs o{};
            if (sigma_out) o.sigma = sigma_out + (int64_t)t * p;
            if (lambda_out) o.lambda = lambda_out + (int64_t)t * opt->rank;
            o.status = status;
            CubeDesc d = solve_desc(x.plan[t], workspace, Yt, pitch, row_pitch, Xt, x_pitch, x_row_pitch, nullptr,
                                    nullptr, opt->flags, &o);
            d.bwy = at<double>(workspace, g.o_bwy) + (int64_t)iy * g.th;
            d.bwx = at<double>(workspace, g.o_bwx) + (int64_t)ix * g.tw;
            d.bcy = at<unsigned char>(workspace, g.o_bcy) + (int64_t)iy * g.th;
            d.bcx = at<unsigned char>(workspace, g.o_bcx) + (int64_t)ix * g.tw;
            d.bpass = x.pass_of[t];
            d.bncx = g.ncx;
            x.desc[t] = d;
        }
    if (dtype == HYRES_F32) {
        BlendGrid& b = x.bg;
        b.ny = g.ny; b.nx = g.nx; b.th = g.th; b.tw = g.tw; b.H = H; b.W = W; b.p = p;
        for (int i = 0; i < g.ny; ++i) b.sy[i] = g.ay.start[i];
        for (int i = 0; i < g.nx; ++i) b.sx[i] = g.ax.start[i];
        b.X = X; b.xpitch = x_pitch; b.xrow_pitch = x_row_pitch;
        x.blend1 = true;
    }
    group_tiles(x);
    build_program(x, kAllStages);
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_exec(x, s))) return st;
    hipLaunchKernelGGL(k_blend_axis, dim3((g.ny * g.th + 255) / 256), dim3(256), 0, s, g.ay,
                       at<double>(workspace, g.o_bwy), at<unsigned char>(workspace, g.o_bcy));
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_blend_axis, dim3((g.nx * g.tw + 255) / 256), dim3(256), 0, s, g.ax,
                       at<double>(workspace, g.o_bwx), at<unsigned char>(workspace, g.o_bcx));
    HIPCHK(hipGetLastError());
    return run_program(x, s, true);
}

HYRES_API hyres_status hyres_tiled_check_program(int H, int W, int p, int tile, int overlap,
                                                 const hyres_options* opt, int dtype, hyres_program_stats* stats) {
    hyres_handle h;
    init_host_handle(h);
    Exec x;
    TileGrid g;
    hyres_status st = plan_tiled(x, g, &h, H, W, p, tile, overlap, opt, dtype);
    if (st) return st;
    x.desc.resize(x.count);
    for (int t = 0; t < x.count; ++t) {
        hyres_outputs o{};
        x.desc[t] = solve_desc(x.plan[t], nullptr, nullptr, p, (int64_t)W * p, nullptr, p, (int64_t)W * p,
                               nullptr, nullptr, opt->flags, &o);
        x.desc[t].bpass = x.pass_of[t];
    }
    if (dtype == HYRES_F32) {
        x.bg.ny = g.ny; x.bg.nx = g.nx; x.bg.th = g.th; x.bg.tw = g.tw; x.bg.H = H; x.bg.W = W; x.bg.p = p;
        x.blend1 = true;
    }
    group_tiles(x);
    build_program(x, kAllStages);
    return dry_check(x, stats);
}

// ------------------------------------------------------------- autotuner
namespace {

// Tuning cache: a JSON object whose "entries" array holds one object per
// (device, dtype, direction, width class) with the chosen tile and its time.
const char* kCacheFormat = "hyres-dwt-tiles-1";
constexpr int kTuneLaunches = 5;

void load_cache(hyres_handle* h, const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
    std::fclose(f);
    if (text.find(kCacheFormat) == std::string::npos) return;
    size_t pos = 0;
    while ((pos = text.find("{\"device\": \"", pos)) != std::string::npos) {
        char dev[320] = {0};
        int dt = -1, inv = -1, wc = -1, tx = 0, ty = 0;
        float us = 0.f;
        const int got = std::sscanf(text.c_str() + pos,
                                    "{\"device\": \"%319[^\"]\", \"dtype\": %d, \"inverse\": %d, \"wclass\": %d, "
                                    "\"tx\": %d, \"ty\": %d, \"us\": %f}",
                                    dev, &dt, &inv, &wc, &tx, &ty, &us);
        pos += 1;
        if (got != 7 || h->arch != dev || dt < 0 || dt > 1 || inv < 0 || inv > 1 || wc < 0 ||
            wc >= kWidthClasses)
            continue;
        for (int c = 0; c < kTileCands; ++c) {
            if (kTileTX[c] == tx && kTileTY[c] == ty) {
                h->tile[dt][inv][wc] = (unsigned char)c;
                h->tuned[dt][inv][wc] = 1;
                h->tile_us[dt][inv][wc] = us;
            }
        }
    }
}

// Writes this handle's tuned entries and keeps other devices' entries.
bool save_cache(const hyres_handle* h, const char* path) {
    std::vector<std::string> keep;
    FILE* f = std::fopen(path, "rb");
    if (f) {
        std::string text;
        char buf[4096];
        size_t k;
        while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
        std::fclose(f);
        size_t pos = 0;
        while ((pos = text.find("{\"device\": \"", pos)) != std::string::npos) {
            const size_t end = text.find('}', pos);
            if (end == std::string::npos) break;
            std::string e = text.substr(pos, end - pos + 1);
            const std::string mine = "{\"device\": \"" + h->arch + "\"";
            if (e.compare(0, mine.size(), mine) != 0) keep.push_back(e);
            pos = end;
        }
    }
    const std::string tmp = std::string(path) + ".tmp";
    f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\"format\": \"%s\", \"entries\": [", kCacheFormat);
    bool first = true;
    for (auto& e : keep) {
        std::fprintf(f, "%s\n  %s", first ? "" : ",", e.c_str());
        first = false;
    }
    for (int dt = 0; dt < 2; ++dt)
        for (int inv = 0; inv < 2; ++inv)
            for (int wc = 0; wc < kWidthClasses; ++wc) {
                if (!h->tuned[dt][inv][wc]) continue;
                const int c = h->tile[dt][inv][wc];
                std::fprintf(f,
                             "%s\n  {\"device\": \"%s\", \"dtype\": %d, \"inverse\": %d, \"wclass\": %d, "
                             "\"tx\": %d, \"ty\": %d, \"us\": %.3f}",
                             first ? "" : ",", h->arch.c_str(), dt, inv, wc, kTileTX[c], kTileTY[c],
                             h->tile_us[dt][inv][wc]);
                first = false;
            }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

HYRES_API hyres_status hyres_autotune(hyres_handle* h, hyres_batch* b, const char* cache_path,
                                      hyres_stream_t stream) {
    if (!h || !b) return HYRES_E_NULL;
    if (b->h != h) return HYRES_E_UNSUPPORTED;
    hyres_status st = set_device(h);
    if (st) return st;
    if (cache_path) load_cache(h, cache_path);
    Exec& x = b->x;
    const int dt = x.dtype == HYRES_F64;
    hipStream_t s = (hipStream_t)stream;
    // width classes of this batch still untuned, per direction
    bool need[2][kWidthClasses] = {};
    bool any = false;
    for (auto& c : x.plan)
        for (int l = 1; l <= c.L; ++l)
            for (int inv = 0; inv < 2; ++inv) {
                const int wc = width_class(c.lw[l]);
                if (!h->tuned[dt][inv][wc]) {
                    need[inv][wc] = true;
                    any = true;
                }
            }
    if (any) {
        // one solve leaves realistic values in every buffer the transforms read
        build_program(x, kAllStages);
        if ((st = upload_exec(x, s))) return st;
        if ((st = run_program(x, s, false))) return st;
        const int scratch = (int)(table_ints(x.count) - (x.count + 1));   // the tuner's table
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHK(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return HYRES_E_HIP;
        }
        int Lmax = 0;
        for (auto& c : x.plan) Lmax = std::max(Lmax, c.L);
        hyres_status res = HYRES_OK;
        for (int inv = 0; inv < 2 && !res; ++inv)
            for (int wc = 0; wc < kWidthClasses && !res; ++wc) {
                if (!need[inv][wc]) continue;
                float best = 0.f;
                int best_c = default_tile(wc);
                for (int cand = 0; cand < kTileCands && !res; ++cand) {
                    float total = 0.f;
                    for (int l = 1; l <= Lmax && !res; ++l) {
                        std::vector<int> tabv(x.count + 1, 0);
                        int64_t tot = 0;
                        for (int i = 0; i < x.count; ++i) {
                            const CubePlan& c = x.plan[i];
                            if (c.L >= l && width_class(c.lw[l]) == wc)
                                tot += c.r * cdiv(c.lw[l], kTileTX[cand]) * cdiv(c.lh[l], kTileTY[cand]);
                            tabv[i + 1] = (int)tot;
                        }
                        if (tot == 0) continue;
                        if (upload(x.ws, x.o_tab + sizeof(int) * scratch, tabv.data(), sizeof(int) * tabv.size(),
                                   s) != hipSuccess) {
                            res = HYRES_E_HIP;
                            break;
                        }
                        const int grid = x.grid(tot, 8);
                        const int* t = x.table(scratch);
                        // best of three timings of kTuneLaunches launches, after one warm-up timing
                        float rep_best = 0.f;
                        for (int rep = 0; rep < 4 && !res; ++rep) {
                            if (hipEventRecord(e0, s) != hipSuccess) res = HYRES_E_HIP;
                            for (int k = 0; k < kTuneLaunches && !res; ++k)
                                if (launch_dwt_level(x.dtype, kTileTX[cand], kTileTY[cand], inv != 0, x.descs(), t,
                                                     x.count, l, grid, s) != hipSuccess)
                                    res = HYRES_E_HIP;
                            if (res || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                                res = HYRES_E_HIP;
                                break;
                            }
                            float ms = 0.f;
                            (void)hipEventElapsedTime(&ms, e0, e1);
                            if (rep == 1 || (rep > 1 && ms < rep_best)) rep_best = ms;
                        }
                        total += rep_best / kTuneLaunches;
                    }
                    if (!res && (cand == 0 || total < best)) {
                        best = total;
                        best_c = cand;
                    }
                }
                if (!res) {
                    h->tile[dt][inv][wc] = (unsigned char)best_c;
                    h->tuned[dt][inv][wc] = 1;
                    h->tile_us[dt][inv][wc] = best * 1000.f;
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (res) return res;
    }
    // rebuild the batch's program with the chosen tiles
    b->drop_graph();
    build_program(x, kAllStages);
    if ((st = upload_exec(x, s))) return st;
    if (cache_path && any && !save_cache(h, cache_path)) return HYRES_E_UNSUPPORTED;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_tile_choice(hyres_handle* h, int dtype, int inverse, int width, int* tx, int* ty,
                                         int* tuned) {
    if (!h || !tx || !ty) return HYRES_E_NULL;
    if (!valid_dtype(dtype) || width < 1) return HYRES_E_SHAPE;
    const int wc = width_class(width);
    const int c = h->tile[dtype == HYRES_F64][inverse != 0][wc];
    *tx = kTileTX[c];
    *ty = kTileTY[c];
    if (tuned) *tuned = h->tuned[dtype == HYRES_F64][inverse != 0][wc];
    return HYRES_OK;
}
