// Host side of the C ABI: validation, workspace planning and the launch
// sequence of each entry point.  No call allocates device memory or waits on
// the host; cube descriptors and work-item tables are written into the
// caller's workspace by a small kernel that receives them by value, so every
// sequence can be captured in a HIP graph.
#include <algorithm>
#include <cstring>
#include <vector>

#include "hyres_internal.hpp"

#define HYRES_API extern "C" __attribute__((visibility("default")))

namespace hyres {
hipError_t launch_gram_f32(int T, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_gram_bf16(int T, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_gram_reduce_f32(int T, const CubeDesc*, const int*, int, hipStream_t);
hipError_t launch_gram_f64(const CubeDesc*, int, int, int, hipStream_t);
hipError_t launch_small(int p, const CubeDesc*, const int*, int, hipStream_t);
hipError_t launch_project_f32(int T, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_backproject_f32(int T, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_project_f64(const CubeDesc*, int, int64_t, hipStream_t);
hipError_t launch_backproject_f64(const CubeDesc*, int, int64_t, hipStream_t);
hipError_t launch_dwt_level(int dtype, int tx, int ty, bool inverse, const CubeDesc*, const int*, int, int,
                            int, hipStream_t);
hipError_t launch_sure_init(int dtype, const CubeDesc*, const int*, int, int, hipStream_t);
hipError_t launch_sure_round(int dtype, const CubeDesc*, const int*, const int*, int, int, int, hipStream_t);
int sure_rounds(int dtype);
int sure_chunk();
}  // namespace hyres

using namespace hyres;

struct hyres_handle {
    int device;
    int num_cu;
    int dwt_tx, dwt_ty;
    unsigned prof_mask;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
};

namespace {
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

// Scope object: records an event pair around one stage when it is profiled.
struct StageTimer {
    hyres_handle* h;
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(hyres_handle* h_, hipStream_t s_, int st) : h(h_), s(s_), stage(st) {
        if (h->prof_mask & (1u << stage)) {
            a = prof_event(h);
            if (a) hipEventRecord(a, s);
        }
    }
    ~StageTimer() {
        if (a) {
            hipEvent_t b = prof_event(h);
            if (b) {
                hipEventRecord(b, s);
                h->pending.push_back({stage, a, b});
            } else {
                h->pool.push_back(a);
            }
        }
    }
};
}  // namespace

namespace {

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

// Work-item stages (one table of ncubes+1 prefix offsets each).
enum Stage {
    ST_GRAM = 0, ST_PROJ, ST_BP, ST_COMP, ST_HIST, ST_CLASS,
    ST_DWT0,                          // + (level-1)
    ST_IDWT0 = ST_DWT0 + kMaxLevels,  // + (level-1)
    ST_COUNT = ST_IDWT0 + kMaxLevels
};

// Geometry and workspace layout of one cube.
struct CubePlan {
    int H = 0, W = 0, p = 0, r = 0, L = 0, dtype = 0, scope = 0, T = 0, gslots = 1, precision = 0;
    int64_t n = 0, nz = 0, nc = 0, ncs = 0, tps = 0, tmp_off2 = 0, ll_off = 0;
    int lh[kMaxLevels + 1] = {0}, lw[kMaxLevels + 1] = {0};
    int64_t loff[kMaxLevels + 1] = {0};
    size_t o_gpart = 0, o_G = 0, o_sigma = 0, o_hv = 0, o_V = 0, o_evals = 0, o_gap = 0, o_P32 = 0, o_Q32 = 0,
           o_P64 = 0, o_Q64 = 0, o_Z = 0, o_coef = 0, o_tmp = 0, o_hcnt = 0, o_hsum = 0, o_hmin = 0,
           o_hmax = 0, o_sst = 0, o_lambda = 0, o_sure = 0, o_sbits = 0, o_spre = 0, o_sspre = 0, o_scb = 0,
           o_cand = 0, o_sfill = 0;
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

// Plan the per-cube workspace.  `parts` selects which arrays are needed.
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
        c.o_scb = lay.add(nb * 4);
        c.o_sfill = lay.add(nb * 4);
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
        d.scb = at<uint32_t>(ws, c.o_scb);
        d.sfill = at<uint32_t>(ws, c.o_sfill);
        d.cand = at<uint64_t>(ws, c.o_cand);
        d.lambda = at<double>(ws, c.o_lambda);
        d.sure = at<double>(ws, c.o_sure);
    }
    return d;
}

// Item counts of a single cube for every stage.
void single_items(const CubePlan& c, int tx, int ty, int items[ST_COUNT][2]) {
    for (int s = 0; s < ST_COUNT; ++s) items[s][0] = items[s][1] = 0;
    items[ST_GRAM][1] = c.gslots;
    items[ST_PROJ][1] = (int)cdiv(c.n, kPixTile);
    items[ST_BP][1] = (int)cdiv(c.n, kPixTile);
    items[ST_COMP][1] = c.r;
    const int64_t ns = c.scope == HYRES_SCOPE_DETAIL ? c.ll_off : c.nc;
    items[ST_HIST][1] = (int)(c.r * cdiv(ns, sure_chunk()));
    items[ST_CLASS][1] = 0;   // the class list itself: cube index 0 (stored as {0, 0})
    for (int l = 1; l <= c.L; ++l) {
        const int t = (int)(c.r * cdiv(c.lw[l], tx) * cdiv(c.lh[l], ty));
        items[ST_DWT0 + l - 1][1] = t;
        items[ST_IDWT0 + l - 1][1] = t;
    }
}

struct Ctx {
    hyres_handle* h;
    hipStream_t s;
    void* ws;
    size_t o_desc, o_items;
    const CubeDesc* descs() const { return at<const CubeDesc>(ws, o_desc); }
    const int* items(int stage) const { return at<const int>(ws, o_items) + stage * 2; }
    int grid(int nitems, int per_cu) const {
        return std::max(1, std::min(nitems, h->num_cu * per_cu));
    }
};

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

hyres_status begin(Ctx& x, const CubePlan& c, const CubeDesc& d, Layout& lay_unused) {
    (void)lay_unused;
    int items[ST_COUNT][2];
    single_items(c, x.h->dwt_tx, x.h->dwt_ty, items);
    HIPCHK(upload(x.ws, x.o_desc, &d, sizeof(CubeDesc), x.s));
    HIPCHK(upload(x.ws, x.o_items, items, sizeof(items), x.s));
    return HYRES_OK;
}

hyres_status run_gram(Ctx& x, const CubePlan& c) {
    if (c.dtype == HYRES_F64) {
        HIPCHK(launch_gram_f64(x.descs(), 0, c.p, c.gslots, x.s));
    } else {
        if (c.precision == HYRES_PREC_MIXED)
            HIPCHK(launch_gram_bf16(c.T, x.descs(), x.items(ST_GRAM), 1, c.gslots, x.s));
        else
            HIPCHK(launch_gram_f32(c.T, x.descs(), x.items(ST_GRAM), 1, c.gslots, x.s));
        HIPCHK(launch_gram_reduce_f32(c.T, x.descs(), x.items(ST_CLASS), 1, x.s));
    }
    return HYRES_OK;
}

hyres_status run_dwt(Ctx& x, const CubePlan& c, bool inverse) {
    for (int k = 0; k < c.L; ++k) {
        const int l = inverse ? c.L - k : k + 1;
        const int st = (inverse ? ST_IDWT0 : ST_DWT0) + l - 1;
        const int nit = (int)(c.r * cdiv(c.lw[l], x.h->dwt_tx) * cdiv(c.lh[l], x.h->dwt_ty));
        HIPCHK(launch_dwt_level(c.dtype, x.h->dwt_tx, x.h->dwt_ty, inverse, x.descs(), x.items(st), 1, l,
                                x.grid(nit, 8), x.s));
    }
    return HYRES_OK;
}

hyres_status run_sure(Ctx& x, const CubePlan& c) {
    HIPCHK(launch_sure_init(c.dtype, x.descs(), x.items(ST_COMP), 1, c.r, x.s));
    const int64_t ns = c.scope == HYRES_SCOPE_DETAIL ? c.ll_off : c.nc;
    const int nh = (int)(c.r * cdiv(ns, sure_chunk()));
    for (int k = 0; k < sure_rounds(c.dtype); ++k)
        HIPCHK(launch_sure_round(c.dtype, x.descs(), x.items(ST_HIST), x.items(ST_COMP), 1, x.grid(nh, 2), c.r,
                                 x.s));
    return HYRES_OK;
}

bool valid_dtype(int dt) { return dt == HYRES_F32 || dt == HYRES_F64; }

// Contiguous FP32 cube with 16-byte aligned pixel rows: the kernels use float4 accesses.
int vec4_ok(const void* ptr, int W, int p, int64_t pitch, int64_t row_pitch, int dtype) {
    return dtype == HYRES_F32 && p % 4 == 0 && pitch % 4 == 0 && row_pitch == (int64_t)W * pitch &&
           (reinterpret_cast<uintptr_t>(ptr) % 16) == 0;
}

hyres_status check_cube(const void* Y, int H, int W, int p, int64_t pitch, int64_t row_pitch, int dtype) {
    if (!Y) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    if (pitch < p || row_pitch < (int64_t)(W - 1) * pitch + p) return HYRES_E_SHAPE;
    if ((int64_t)H * W > (int64_t)1 << 31) return HYRES_E_UNSUPPORTED;
    return HYRES_OK;
}

hyres_status check_ws(const void* ws, size_t have, size_t need) {
    if (need == 0) return HYRES_OK;
    if (!ws) return HYRES_E_WORKSPACE;
    if (have < need) return HYRES_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HYRES_E_WORKSPACE;
    return HYRES_OK;
}

// Common front end of the entry points that take a cube.
struct CubeCall {
    CubePlan c;
    Layout lay;
    size_t o_desc = 0, o_items = 0;
};

hyres_status plan_cube_call(CubeCall& k, int H, int W, int p, int r, int L, int dtype, int scope, int parts) {
    CubePlan& c = k.c;
    c.H = H; c.W = W; c.p = p; c.r = r; c.L = L; c.dtype = dtype; c.scope = scope;
    if (parts & (P_IMG | P_SURE)) {
        if (!level_geometry(H, W, L, c.lh, c.lw, c.loff, &c.ll_off, &c.nc)) return HYRES_E_SHAPE;
    }
    k.o_desc = k.lay.add(sizeof(CubeDesc));
    k.o_items = k.lay.add(sizeof(int) * ST_COUNT * 2);
    plan_cube(c, k.lay, parts);
    return HYRES_OK;
}

}  // namespace

// =========================================================================
HYRES_API hyres_status hyres_create(hyres_handle** handle, int device) {
    if (!handle) return HYRES_E_NULL;
    *handle = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HYRES_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HYRES_E_HIP;
    hyres_handle* h = new (std::nothrow) hyres_handle;
    if (!h) return HYRES_E_HIP;
    h->device = device;
    h->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    h->dwt_tx = 64;
    h->dwt_ty = 4;
    h->prof_mask = 0;
    *handle = h;
    return HYRES_OK;
}

HYRES_API void hyres_destroy(hyres_handle* handle) {
    if (!handle) return;
    for (auto& r : handle->pending) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : handle->pool) hipEventDestroy(e);
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
    for (auto& r : h->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess) return HYRES_E_HIP;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return HYRES_E_HIP;
        ms_out[r.stage] += ms;
        count_out[r.stage] += 1;
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

// ------------------------------------------------------------- noise
HYRES_API hyres_status hyres_estimate_noise_workspace_size(int H, int W, int p, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    CubeCall k;
    hyres_status st = plan_cube_call(k, H, W, p, 1, 1, dtype, 0, P_GRAM | P_SMALL);
    if (st) return st;
    *bytes = k.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_estimate_noise(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                            int64_t row_pitch, int dtype, double* sigma_out, double* gram_out,
                                            int* status, void* workspace, size_t workspace_bytes,
                                            hyres_stream_t stream) {
    if (!h || !sigma_out) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    CubeCall k;
    if ((st = plan_cube_call(k, H, W, p, 1, 1, dtype, 0, P_GRAM | P_SMALL))) return st;
    if ((st = check_ws(workspace, workspace_bytes, k.lay.total))) return st;
    if ((st = set_device(h))) return st;
    CubeDesc d = make_desc(k.c, workspace);
    d.Y = Y; d.pitch = pitch; d.row_pitch = row_pitch;
    d.vec4 = vec4_ok(Y, W, p, pitch, row_pitch, dtype);
    d.sigma = sigma_out;
    if (gram_out) d.G = gram_out;
    d.status = status;
    d.mode = 1;
    Ctx x{h, (hipStream_t)stream, workspace, k.o_desc, k.o_items};
    if ((st = begin(x, k.c, d, k.lay))) return st;
    if ((st = run_gram(x, k.c))) return st;
    HIPCHK(launch_small(p, x.descs(), x.items(ST_CLASS), 1, x.s));
    return HYRES_OK;
}

// ------------------------------------------------------------- subspace
HYRES_API hyres_status hyres_subspace_workspace_size(int H, int W, int p, int r, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands || r < 1 || r > kMaxRank || r > p) return HYRES_E_SHAPE;
    CubeCall k;
    hyres_status st = plan_cube_call(k, H, W, p, r, 1, dtype, 0, P_GRAM | P_SMALL);
    if (st) return st;
    *bytes = k.lay.total;
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
    CubeCall k;
    if ((st = plan_cube_call(k, H, W, p, r, 1, dtype, 0, P_GRAM | P_SMALL))) return st;
    if ((st = check_ws(workspace, workspace_bytes, k.lay.total))) return st;
    if ((st = set_device(h))) return st;
    CubeDesc d = make_desc(k.c, workspace);
    d.Y = Y; d.pitch = pitch; d.row_pitch = row_pitch;
    d.vec4 = vec4_ok(Y, W, p, pitch, row_pitch, dtype);
    d.sigma_in = sigma;
    d.V = V_out;
    if (evals_out) d.evals = evals_out;
    d.status = status;
    d.mode = 2 | 16;
    Ctx x{h, (hipStream_t)stream, workspace, k.o_desc, k.o_items};
    if ((st = begin(x, k.c, d, k.lay))) return st;
    if ((st = run_gram(x, k.c))) return st;
    HIPCHK(launch_small(p, x.descs(), x.items(ST_CLASS), 1, x.s));
    return HYRES_OK;
}

// ------------------------------------------------------------- wavelets
static hyres_status plan_images(CubeCall& k, int batch, int H, int W, int L, int dtype, int parts) {
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (batch < 1) return HYRES_E_SHAPE;
    CubePlan& c = k.c;
    c.H = H; c.W = W; c.p = 2; c.r = batch; c.L = L; c.dtype = dtype; c.scope = 0;
    if (!level_geometry(H, W, L, c.lh, c.lw, c.loff, &c.ll_off, &c.nc)) return HYRES_E_SHAPE;
    c.n = (int64_t)H * W;
    c.T = 1;
    k.o_desc = k.lay.add(sizeof(CubeDesc));
    k.o_items = k.lay.add(sizeof(int) * ST_COUNT * 2);
    const int es = esize(dtype);
    const int64_t a1 = rup((int64_t)c.lh[1] * c.lw[1], 64);
    const int64_t a2 = L >= 2 ? rup((int64_t)c.lh[2] * c.lw[2], 64) : 0;
    c.tmp_off2 = a1;
    c.tps = a1 + a2;
    c.o_tmp = k.lay.add((size_t)batch * c.tps * es);
    c.nz = c.n;
    c.ncs = c.nc;
    (void)parts;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_dwt2_workspace_size(int batch, int H, int W, int L, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    CubeCall k;
    hyres_status st = plan_images(k, batch, H, W, L, dtype, 0);
    if (st) return st;
    *bytes = k.lay.total;
    return HYRES_OK;
}

static hyres_status dwt_common(hyres_handle* h, const void* in, int batch, int H, int W, int L, int dtype,
                               void* out, const double* lambda, int scope, bool inverse, void* ws, size_t wsb,
                               hyres_stream_t stream) {
    if (!h || !in || !out) return HYRES_E_NULL;
    CubeCall k;
    hyres_status st = plan_images(k, batch, H, W, L, dtype, 0);
    if (st) return st;
    if (scope != HYRES_SCOPE_ALL && scope != HYRES_SCOPE_DETAIL) return HYRES_E_SHAPE;
    if ((st = check_ws(ws, wsb, k.lay.total))) return st;
    if ((st = set_device(h))) return st;
    k.c.scope = scope;
    CubeDesc d = make_desc(k.c, ws);
    d.tmp = at<void>(ws, k.c.o_tmp);
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
    Ctx x{h, (hipStream_t)stream, ws, k.o_desc, k.o_items};
    if ((st = begin(x, k.c, d, k.lay))) return st;
    return run_dwt(x, k.c, inverse);
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
static hyres_status plan_sure(CubeCall& k, int batch, int64_t Nc, int dtype) {
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (batch < 1 || Nc < 1 || Nc > ((int64_t)1 << 31)) return HYRES_E_SHAPE;
    CubePlan& c = k.c;
    c.r = batch; c.dtype = dtype; c.nc = Nc; c.ll_off = Nc; c.L = 0; c.scope = 0;
    k.o_desc = k.lay.add(sizeof(CubeDesc));
    k.o_items = k.lay.add(sizeof(int) * ST_COUNT * 2);
    plan_cube(c, k.lay, P_SURE);
    return HYRES_OK;
}

HYRES_API hyres_status hyres_sure_workspace_size(int batch, int64_t Nc, int dtype, size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    CubeCall k;
    hyres_status st = plan_sure(k, batch, Nc, dtype);
    if (st) return st;
    *bytes = k.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_sure_threshold(hyres_handle* h, const void* coeffs, int batch, int64_t Nc,
                                            int64_t stride, int dtype, double* lambda_out, double* sure_min_out,
                                            int* status, void* workspace, size_t workspace_bytes,
                                            hyres_stream_t stream) {
    if (!h || !coeffs || !lambda_out) return HYRES_E_NULL;
    CubeCall k;
    hyres_status st = plan_sure(k, batch, Nc, dtype);
    if (st) return st;
    if (stride < Nc) return HYRES_E_SHAPE;
    if ((st = check_ws(workspace, workspace_bytes, k.lay.total))) return st;
    if ((st = set_device(h))) return st;
    k.c.ncs = stride;
    CubeDesc d = make_desc(k.c, workspace);
    d.coef = const_cast<void*>(coeffs);
    d.lambda = lambda_out;
    d.sure = sure_min_out ? sure_min_out : d.sure;
    d.status = status;
    Ctx x{h, (hipStream_t)stream, workspace, k.o_desc, k.o_items};
    if ((st = begin(x, k.c, d, k.lay))) return st;
    return run_sure(x, k.c);
}

// ------------------------------------------------------------- denoise
static hyres_status check_opts(const hyres_options* opt, int p, int dtype) {
    if (!opt) return HYRES_E_NULL;
    if (opt->rank < 1 || opt->rank > kMaxRank || opt->rank > p) return HYRES_E_SHAPE;
    if (opt->levels < 1 || opt->levels > kMaxLevels) return HYRES_E_SHAPE;
    if (opt->scope != HYRES_SCOPE_ALL && opt->scope != HYRES_SCOPE_DETAIL) return HYRES_E_SHAPE;
    if (opt->precision != HYRES_PREC_NATIVE && opt->precision != HYRES_PREC_MIXED) return HYRES_E_DTYPE;
    if (opt->precision == HYRES_PREC_MIXED && dtype != HYRES_F32) return HYRES_E_DTYPE;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_denoise_workspace_size(int H, int W, int p, const hyres_options* opt, int dtype,
                                                    size_t* bytes) {
    if (!bytes) return HYRES_E_NULL;
    if (!valid_dtype(dtype)) return HYRES_E_DTYPE;
    if (H < 1 || W < 1 || p < 2 || p > kMaxBands) return HYRES_E_SHAPE;
    hyres_status st = check_opts(opt, p, dtype);
    if (st) return st;
    CubeCall k;
    if ((st = plan_cube_call(k, H, W, p, opt->rank, opt->levels, dtype, opt->scope,
                             P_GRAM | P_SMALL | P_IMG | P_SURE)))
        return st;
    *bytes = k.lay.total;
    return HYRES_OK;
}

HYRES_API hyres_status hyres_denoise(hyres_handle* h, const void* Y, int H, int W, int p, int64_t pitch,
                                     int64_t row_pitch, int dtype, const hyres_options* opt,
                                     const double* sigma_in, const double* lambda_in, void* X, int64_t x_pitch,
                                     int64_t x_row_pitch, const hyres_outputs* out, void* workspace,
                                     size_t workspace_bytes, hyres_stream_t stream) {
    if (!h || !X) return HYRES_E_NULL;
    hyres_status st = check_cube(Y, H, W, p, pitch, row_pitch, dtype);
    if (st) return st;
    if ((st = check_opts(opt, p, dtype))) return st;
    if (x_pitch < p || x_row_pitch < (int64_t)(W - 1) * x_pitch + p) return HYRES_E_SHAPE;
    CubeCall k;
    if ((st = plan_cube_call(k, H, W, p, opt->rank, opt->levels, dtype, opt->scope,
                             P_GRAM | P_SMALL | P_IMG | P_SURE)))
        return st;
    k.c.precision = opt->precision;
    if ((st = check_ws(workspace, workspace_bytes, k.lay.total))) return st;
    if ((st = set_device(h))) return st;
    CubeDesc d = make_desc(k.c, workspace);
    d.Y = Y; d.pitch = pitch; d.row_pitch = row_pitch;
    d.X = X; d.xpitch = x_pitch; d.xrow_pitch = x_row_pitch;
    d.vec4 = vec4_ok(Y, W, p, pitch, row_pitch, dtype);
    d.xvec4 = vec4_ok(X, W, p, x_pitch, x_row_pitch, dtype);
    d.sigma_in = sigma_in;
    d.lambda_in = lambda_in;
    d.mode = (sigma_in ? 0 : 1) | 2 | 8 | ((opt->flags & HYRES_FLAG_ALL_EVALS) ? 16 : 0);
    if (out) {
        if (out->sigma) d.sigma = out->sigma;
        if (out->V) d.V = out->V;
        if (out->evals) d.evals = out->evals;
        if (out->gap) d.gap = out->gap;
        if (out->lambda) d.lambda = out->lambda;
        if (out->sure) d.sure = out->sure;
        d.status = out->status;
    }
    hipStream_t s = (hipStream_t)stream;
    Ctx x{h, s, workspace, k.o_desc, k.o_items};
    const CubePlan& c = k.c;
    if ((st = begin(x, c, d, k.lay))) return st;
    {
        StageTimer tm(h, s, HYRES_STAGE_GRAM);
        if ((st = run_gram(x, c))) return st;
    }
    {
        StageTimer tm(h, s, HYRES_STAGE_SMALL);
        HIPCHK(launch_small(p, x.descs(), x.items(ST_CLASS), 1, s));
    }
    const int nt = (int)cdiv(c.n, kPixTile);
    {
        StageTimer tm(h, s, HYRES_STAGE_PROJECT);
        if (dtype == HYRES_F64) HIPCHK(launch_project_f64(x.descs(), 0, c.n, s));
        else HIPCHK(launch_project_f32(c.T, x.descs(), x.items(ST_PROJ), 1, x.grid(nt, 8), s));
    }
    {
        StageTimer tm(h, s, HYRES_STAGE_DWT);
        if ((st = run_dwt(x, c, false))) return st;
    }
    {
        StageTimer tm(h, s, HYRES_STAGE_SURE);
        if (lambda_in) {
            hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(64), 0, s, lambda_in, d.lambda, c.r);
            HIPCHK(hipGetLastError());
        } else if ((st = run_sure(x, c))) {
            return st;
        }
    }
    {
        StageTimer tm(h, s, HYRES_STAGE_IDWT);
        if ((st = run_dwt(x, c, true))) return st;
    }
    {
        StageTimer tm(h, s, HYRES_STAGE_BACKPROJECT);
        if (dtype == HYRES_F64) HIPCHK(launch_backproject_f64(x.descs(), 0, c.n, s));
        else HIPCHK(launch_backproject_f32(c.T, x.descs(), x.items(ST_BP), 1, x.grid(nt, 8), s));
    }
    return HYRES_OK;
}
