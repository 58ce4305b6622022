// Host side of libfastcod.so: argument checks, workspaces, launch sequence, error model.
// The C-ABI is declared in include/fastcod.h.
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "fastcod.h"
#include "internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(FASTCOD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define FC_HIP(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)

// smallest float >= n
float float_bound(int32_t n) {
    float f = (float)n;
    if ((double)f < (double)n) f = nextafterf(f, INFINITY);
    return f;
}

int bit_width(uint32_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// Device buffer that only grows.  Growth frees the old buffer (hipFree waits for the device).
struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t bytes, bool zero) {
        if (bytes <= n && p) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            n = 0;
            if (e != hipSuccess) return e;
        }
        size_t want = bytes < 256 ? 256 : bytes;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        n = want;
        if (zero) {
            e = hipMemset(p, 0, want);
            if (e == hipSuccess) e = hipDeviceSynchronize();
        }
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

struct Workspace {
    std::mutex mu;      // held for the whole enqueue of one call
    DevBuf compact;     // fastcod_count's per-call compact volume
    DevBuf first;       // chunk -> first streamline
    DevBuf ovf;         // overflow counter + queue
    DevBuf fallback;    // fallback scratch (all-zero between launches)
    DevBuf flags;       // validation flags
    DevBuf ct;          // transposed accumulation copy of C
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

int current_device(int *dev) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return FASTCOD_OK;
}

Workspace *workspace_for(int dev, hipStream_t st) {
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto &w = g_ws[{dev, st}];
    if (!w) w = new Workspace();
    return w;
}

int cu_count(int dev) {
    static std::mutex mu;
    static std::map<int, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev] = n;
    return n;
}

// ---- compact volume layout ----
constexpr int32_t kMaxCoarseWords = 8192;   // 32 KB of LDS per counting workgroup
struct CompactLayout {
    int32_t SBX, SBY, SBZ;
    int64_t W;        // words
    int64_t ntiles;
    int64_t nvox;
    bool packed;
    int32_t rbits;
    int32_t cs, CBX, CBY, CBZ, ncoarse_words;
    size_t off_mb, off_tiles, off_coarse, off_codes, bytes;
};

bool compact_layout(const int32_t dims[3], int32_t N, int32_t M, CompactLayout &L) {
    L.SBX = (dims[0] + 15) / 16;
    L.SBY = (dims[1] + 7) / 8;
    L.SBZ = (dims[2] + 7) / 8;
    L.W = (int64_t)L.SBX * L.SBY * L.SBZ * 32;
    L.nvox = (int64_t)dims[0] * dims[1] * dims[2];
    // word indices are uint32 and padding must stay modest (thin grids use raster lookups)
    if (L.W >= (int64_t(1) << 31) || L.W * 32 > 8 * L.nvox + (int64_t(1) << 22)) return false;
    if ((int64_t)L.SBX * L.SBY >= (int64_t(1) << 31)) return false;
    L.ntiles = (L.W + fc::kScanTile - 1) / fc::kScanTile;
    const int rb = bit_width((uint32_t)N), lb = bit_width((uint32_t)M);
    L.packed = rb + lb <= 32;
    L.rbits = rb;
    // buffer-resource offsets are 32-bit: occupancy pairs and codes must stay below 4 GB
    if (8 * L.W >= (int64_t(1) << 32) || (L.packed ? 4 : 8) * L.nvox >= (int64_t(1) << 32)) return false;
    // coarse occupancy (kept in LDS by the counting kernel): smallest block side 8, 16 or 32 whose
    // bit map fits kMaxCoarseWords
    for (L.cs = 3; L.cs <= 5; ++L.cs) {
        const int32_t c = 1 << L.cs;
        L.CBX = (dims[0] + c - 1) / c;
        L.CBY = (dims[1] + c - 1) / c;
        L.CBZ = (dims[2] + c - 1) / c;
        const int64_t ncb = (int64_t)L.CBX * L.CBY * L.CBZ;
        L.ncoarse_words = (int32_t)(2 * ((ncb + 63) / 64));
        if (L.ncoarse_words <= kMaxCoarseWords) break;
    }
    if (L.cs > 5) return false;
    auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
    L.off_mb = 0;
    L.off_tiles = align(L.off_mb + 8 * (size_t)L.W);
    L.off_coarse = align(L.off_tiles + 4 * (size_t)L.ntiles);
    L.off_codes = align(L.off_coarse + 4 * (size_t)L.ncoarse_words);
    L.bytes = L.off_codes + (L.packed ? 4 : 8) * (size_t)L.nvox;   // at most every voxel occupied
    return true;
}

fc::CompactVol compact_view(void *buf, const CompactLayout &L, int32_t N, int32_t M) {
    char *b = static_cast<char *>(buf);
    fc::CompactVol cv;
    cv.mb = reinterpret_cast<const uint2 *>(b + L.off_mb);
    cv.coarse = reinterpret_cast<const uint32_t *>(b + L.off_coarse);
    cv.cs = L.cs;
    cv.CBX = L.CBX;
    cv.CBXY = L.CBX * L.CBY;
    cv.ncoarse_words = L.ncoarse_words;
    cv.codes32 = reinterpret_cast<const uint32_t *>(b + L.off_codes);
    cv.codes64 = reinterpret_cast<const int2 *>(b + L.off_codes);
    cv.SBX = L.SBX;
    cv.SBXY = L.SBX * L.SBY;
    cv.rbits = L.rbits;
    cv.rmask = L.rbits >= 32 ? 0xFFFFFFFFu : ((1u << L.rbits) - 1u);
    cv.N = N;
    cv.M = M;
    cv.packed = L.packed ? 1 : 0;
    cv.W = L.W;
    cv.ncodes = L.nvox;
    return cv;
}

fc::Grid make_grid(const int32_t dims[3]) {
    fc::Grid g;
    g.X = dims[0];
    g.Y = dims[1];
    g.Z = dims[2];
    g.Xf = float_bound(dims[0]);
    g.Yf = float_bound(dims[1]);
    g.Zf = float_bound(dims[2]);
    return g;
}

int check_volume_args(const int32_t *roi, const int32_t *lab, const int32_t dims[3], int32_t N, int32_t M) {
    if (!dims) return fail(FASTCOD_EINVAL, "dims is NULL");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return fail(FASTCOD_EINVAL, "dims must be >= 1");
    if ((int64_t)dims[0] * dims[1] * dims[2] >= (int64_t(1) << 31)) return fail(FASTCOD_EINVAL, "X*Y*Z must be < 2^31");
    if (N < 1 || M < 1) return fail(FASTCOD_EINVAL, "N and M must be >= 1");
    if ((int64_t)N * M >= (int64_t(1) << 31)) return fail(FASTCOD_EINVAL, "N*M must be < 2^31");
    if (!roi || !lab) return fail(FASTCOD_EINVAL, "volume pointer is NULL");
    return FASTCOD_OK;
}

int check_stream_args(const float *points, const int64_t *offsets, int64_t S, int32_t *C, const fastcod_opts &o) {
    if (S < 0 || S > INT32_MAX) return fail(FASTCOD_EINVAL, "n_streamlines must be in [0, INT32_MAX]");
    if (!offsets) return fail(FASTCOD_EINVAL, "offsets is NULL");
    if (S > 0 && !points) return fail(FASTCOD_EINVAL, "points is NULL");
    if (!C) return fail(FASTCOD_EINVAL, "C_out is NULL");
    if (o.upsample != 1) return fail(FASTCOD_EINVAL, "upsample must be 1");
    if (!(o.scale == o.scale) || o.scale <= 0.0f || isinf(o.scale)) return fail(FASTCOD_EINVAL, "scale must be finite and > 0");
    if (o.variant < FASTCOD_VARIANT_AUTO || o.variant > FASTCOD_VARIANT_STREAM) return fail(FASTCOD_EINVAL, "unknown variant");
    if (o.batch != 0 && o.batch != 2 && o.batch != 4 && o.batch != 8) return fail(FASTCOD_EINVAL, "batch must be 0, 2, 4 or 8");
    if (o.blocks_per_cu < 0) return fail(FASTCOD_EINVAL, "blocks_per_cu must be >= 0");
    if (o.depth != 0 && o.depth != 1 && o.depth != 2) return fail(FASTCOD_EINVAL, "depth must be 0, 1 or 2");
    return FASTCOD_OK;
}

constexpr int kBlocksPerCU = 8;            // resident 256-thread workgroups per CU (count kernels)
constexpr int kRangesPerWave = 4;          // flat-stream point ranges per wavefront, handed out dynamically

int fallback_scratch(Workspace &ws, int32_t N, int32_t M, fc::FallbackScratch &fs) {
    fs.nwordsN = (N + 31) / 32;
    fs.nwordsM = (M + 31) / 32;
    fs.stride = ((int64_t)fs.nwordsN + fs.nwordsM + M + 63) & ~int64_t(63);
    int64_t blocks = (int64_t(256) << 20) / (4 * fs.stride);   // <= 256 MiB of scratch
    if (blocks > 64) blocks = 64;
    if (blocks < 1) blocks = 1;
    fs.blocks = (int32_t)blocks;
    FC_HIP(ws.fallback.ensure((size_t)(4 * fs.stride * blocks), true));
    fs.words = static_cast<uint32_t *>(ws.fallback.p);
    return FASTCOD_OK;
}

int run_validate(Workspace &ws, const int64_t *offsets, int64_t S, const int32_t *roi, const int32_t *lab,
                 const int32_t dims[3], int32_t N, int32_t M, hipStream_t st, int dev) {
    FC_HIP(ws.flags.ensure(256, false));
    int32_t *d = static_cast<int32_t *>(ws.flags.p);
    const int64_t nvox = (int64_t)dims[0] * dims[1] * dims[2];
    FC_HIP(fc::launch_validate(offsets, S, roi, lab, nvox, N, M, d, cu_count(dev), st));
    int32_t h = 0;
    FC_HIP(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st));
    FC_HIP(hipStreamSynchronize(st));
    if (h) {
        std::string m = "validation failed:";
        if (h & 1) m += " offsets not starting at 0 / decreasing;";
        if (h & 2) m += " ROI value >= N;";
        if (h & 4) m += " label value >= M;";
        return fail(FASTCOD_ERANGE, m);
    }
    return FASTCOD_OK;
}

// The counting sequence on one stream, against a raster or a compact volume.
int enqueue_count(Workspace &ws, int dev, const float *points, const int64_t *offsets, int64_t S,
                  const fc::Grid &g, int32_t N, int32_t M, const fc::RasterVol *rv, const fc::CompactVol *cv,
                  int32_t *C, const fastcod_opts &o, hipStream_t st) {
    const int cus = cu_count(dev);
    // The flat-stream path accumulates into a transposed workspace copy CT[M][N]: the rows of one
    // streamline are neighbouring ROI indices, so its pair updates share memory lines there.
    const bool transposed = cv != nullptr && S > 0 && M > 1 && N >= 64;
    if (!(o.flags & FASTCOD_ACCUMULATE) && !transposed) FC_HIP(fc::launch_fill_i32(C, (int64_t)N * M, 0, cus, st));
    if (S == 0) {
        if (o.event_begin) FC_HIP(hipEventRecord((hipEvent_t)o.event_begin, st));
        if (o.event_end) FC_HIP(hipEventRecord((hipEvent_t)o.event_end, st));
        return FASTCOD_OK;
    }
    FC_HIP(ws.ovf.ensure(256 + 8 * (size_t)S, false));
    fc::CountArgs a;
    a.pts = points;
    a.offsets = offsets;
    a.S = S;
    a.g = g;
    a.scale = o.scale;
    a.C = C;
    a.si = (uint32_t)M;
    a.sm = 1u;
    if (transposed) {
        FC_HIP(ws.ct.ensure(4 * (size_t)N * (size_t)M, false));
        a.C = static_cast<int32_t *>(ws.ct.p);
        a.si = 1u;
        a.sm = (uint32_t)N;
        FC_HIP(fc::launch_fill_i32(a.C, (int64_t)N * M, 0, cus, st));
    }
    a.ovf.count = static_cast<unsigned long long *>(ws.ovf.p);
    a.ovf.list = reinterpret_cast<int64_t *>(static_cast<char *>(ws.ovf.p) + 256);
    a.ovf.cap = S;
    a.ovf.work = static_cast<unsigned long long *>(ws.ovf.p) + 1;
    fc::FallbackScratch fs;
    int rc = fallback_scratch(ws, N, M, fs);
    if (rc) return rc;
    FC_HIP(fc::launch_fill_u64(a.ovf.count, 2, cus, st));   // overflow count and range counter
    const int64_t resident = (int64_t)cus * kBlocksPerCU;
    if (cv) {
        const int batch = o.batch == 2 || o.batch == 8 ? o.batch : 4;
        const int depth = o.depth == 2 ? 2 : 1;
        int per_cu = fc::count_stream_blocks_per_cu(o.scale != 1.0f, cv->packed != 0, batch, depth,
                                                    4 * (size_t)cv->ncoarse_words);
        if (o.blocks_per_cu > 0 && o.blocks_per_cu < per_cu) per_cu = o.blocks_per_cu;
        const int64_t blocks = (int64_t)cus * per_cu;
        const int64_t nparts = blocks * fc::kWavesPerBlock * kRangesPerWave;
        FC_HIP(ws.first.ensure(4 * (size_t)(nparts + 1), false));
        int32_t *first = static_cast<int32_t *>(ws.first.p);
        FC_HIP(fc::launch_partition(offsets, S, nparts, first, cus, st));
        if (o.event_begin) FC_HIP(hipEventRecord((hipEvent_t)o.event_begin, st));
        FC_HIP(fc::launch_count_stream(a, *cv, first, nparts, (int)blocks, batch, depth, st));
        if (o.event_end) FC_HIP(hipEventRecord((hipEvent_t)o.event_end, st));
        FC_HIP(fc::launch_fallback_compact(a, *cv, fs, st));
        if (transposed) FC_HIP(fc::launch_transpose(a.C, C, N, M, (o.flags & FASTCOD_ACCUMULATE) != 0, st));
    } else {
        int64_t blocks = (S + fc::kWavesPerBlock - 1) / fc::kWavesPerBlock;
        if (blocks > resident) blocks = resident;
        if (o.event_begin) FC_HIP(hipEventRecord((hipEvent_t)o.event_begin, st));
        FC_HIP(fc::launch_count_wave(a, *rv, (int)blocks, st));
        if (o.event_end) FC_HIP(hipEventRecord((hipEvent_t)o.event_end, st));
        FC_HIP(fc::launch_fallback_raster(a, *rv, fs, st));
    }
    (void)N;
    return FASTCOD_OK;
}

}  // namespace

struct fastcod_volume {
    int device;
    int32_t dims[3];
    int32_t N, M;
    CompactLayout L;
    void *buf;
    hipEvent_t ready;
};

extern "C" {

fastcod_opts fastcod_default_opts(void) {
    fastcod_opts o;
    o.scale = 1.0f;
    o.upsample = 1;
    o.flags = 0;
    o.variant = FASTCOD_VARIANT_AUTO;
    o.event_begin = nullptr;
    o.event_end = nullptr;
    o.batch = 0;
    o.blocks_per_cu = 0;
    o.depth = 0;
    return o;
}

const char *fastcod_strerror(int status) {
    switch (status) {
        case FASTCOD_OK: return "ok";
        case FASTCOD_EINVAL: return "invalid argument";
        case FASTCOD_ERANGE: return "input data out of range";
        case FASTCOD_ENOMEM: return "out of device memory or over budget";
        case FASTCOD_EHIP: return "HIP runtime error";
        case FASTCOD_EBUSY: return "busy";
        case FASTCOD_ECANCELED: return "cancelled";
        case FASTCOD_ETIMEDOUT: return "timed out";
        default: return "unknown status";
    }
}

const char *fastcod_last_error(void) { return g_last_error.c_str(); }

int fastcod_count_ex(const float *points, const int64_t *offsets, int64_t S, const int32_t *roi, const int32_t *lab,
                     const int32_t dims[3], int32_t N, int32_t M, int32_t *C, const fastcod_opts *opts, void *stream) {
    g_last_error.clear();
    const fastcod_opts o = opts ? *opts : fastcod_default_opts();
    int rc = check_volume_args(roi, lab, dims, N, M);
    if (rc) return rc;
    rc = check_stream_args(points, offsets, S, C, o);
    if (rc) return rc;
    int dev;
    rc = current_device(&dev);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace &ws = *workspace_for(dev, st);
    std::lock_guard<std::mutex> lock(ws.mu);
    if (o.flags & FASTCOD_VALIDATE) {
        rc = run_validate(ws, offsets, S, roi, lab, dims, N, M, st, dev);
        if (rc) return rc;
    }
    const fc::Grid g = make_grid(dims);
    CompactLayout L;
    const bool compact_ok = compact_layout(dims, N, M, L);
    if (o.variant == FASTCOD_VARIANT_STREAM && !compact_ok)
        return fail(FASTCOD_EINVAL, "grid too thin for the compact volume; use FASTCOD_VARIANT_WAVE");
    if (o.variant == FASTCOD_VARIANT_WAVE || !compact_ok) {
        fc::RasterVol rv{roi, lab, dims[0], dims[0] * dims[1], N, M};
        return enqueue_count(ws, dev, points, offsets, S, g, N, M, &rv, nullptr, C, o, st);
    }
    FC_HIP(ws.compact.ensure(L.bytes, false));
    fc::CompactVol cv = compact_view(ws.compact.p, L, N, M);
    char *b = static_cast<char *>(ws.compact.p);
    FC_HIP(fc::launch_compact_build(roi, lab, g, N, M, cv, reinterpret_cast<uint32_t *>(b + L.off_mb), b + L.off_codes,
                                    reinterpret_cast<uint32_t *>(b + L.off_tiles),
                                    reinterpret_cast<uint32_t *>(b + L.off_coarse), L.W, cu_count(dev), st));
    return enqueue_count(ws, dev, points, offsets, S, g, N, M, nullptr, &cv, C, o, st);
}

int fastcod_count(const float *points, const int64_t *offsets, int64_t S, const int32_t *roi, const int32_t *lab,
                  const int32_t dims[3], int32_t N, int32_t M, int32_t *C, void *stream) {
    return fastcod_count_ex(points, offsets, S, roi, lab, dims, N, M, C, nullptr, stream);
}

int fastcod_volume_create(const int32_t *roi, const int32_t *lab, const int32_t dims[3], int32_t N, int32_t M,
                          void *stream, fastcod_volume **out) {
    g_last_error.clear();
    if (!out) return fail(FASTCOD_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_volume_args(roi, lab, dims, N, M);
    if (rc) return rc;
    CompactLayout L;
    if (!compact_layout(dims, N, M, L)) return fail(FASTCOD_EINVAL, "grid too thin for a compact volume");
    int dev;
    rc = current_device(&dev);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *buf = nullptr;
    hipError_t e = hipMalloc(&buf, L.bytes);
    if (e != hipSuccess) return fail(FASTCOD_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    fastcod_volume *v = new fastcod_volume();
    v->device = dev;
    memcpy(v->dims, dims, sizeof(v->dims));
    v->N = N;
    v->M = M;
    v->L = L;
    v->buf = buf;
    v->ready = nullptr;
    const fc::Grid g = make_grid(dims);
    fc::CompactVol cv = compact_view(buf, L, N, M);
    char *b = static_cast<char *>(buf);
    {
        Workspace &ws = *workspace_for(dev, st);
        std::lock_guard<std::mutex> lock(ws.mu);
        e = fc::launch_compact_build(roi, lab, g, N, M, cv, reinterpret_cast<uint32_t *>(b + L.off_mb), b + L.off_codes,
                                     reinterpret_cast<uint32_t *>(b + L.off_tiles),
                                     reinterpret_cast<uint32_t *>(b + L.off_coarse), L.W, cu_count(dev), st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&v->ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(v->ready, st);
    }
    if (e != hipSuccess) {
        if (v->ready) (void)hipEventDestroy(v->ready);
        (void)hipFree(buf);
        delete v;
        return hip_fail(e, "volume build");
    }
    *out = v;
    return FASTCOD_OK;
}

size_t fastcod_volume_bytes(const fastcod_volume *vol) { return vol ? vol->L.bytes : 0; }

int fastcod_volume_count(const fastcod_volume *vol, const float *points, const int64_t *offsets, int64_t S,
                         int32_t *C, const fastcod_opts *opts, void *stream) {
    g_last_error.clear();
    if (!vol) return fail(FASTCOD_EINVAL, "vol is NULL");
    const fastcod_opts o = opts ? *opts : fastcod_default_opts();
    int rc = check_stream_args(points, offsets, S, C, o);
    if (rc) return rc;
    if (o.variant == FASTCOD_VARIANT_WAVE) return fail(FASTCOD_EINVAL, "a resident volume has no raster form");
    if (o.flags & FASTCOD_VALIDATE) return fail(FASTCOD_EINVAL, "validate the source volumes before creating the handle");
    int dev;
    rc = current_device(&dev);
    if (rc) return rc;
    if (dev != vol->device) return fail(FASTCOD_EINVAL, "volume lives on another device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace &ws = *workspace_for(dev, st);
    std::lock_guard<std::mutex> lock(ws.mu);
    FC_HIP(hipStreamWaitEvent(st, vol->ready, 0));
    const fc::Grid g = make_grid(vol->dims);
    fc::CompactVol cv = compact_view(vol->buf, vol->L, vol->N, vol->M);
    return enqueue_count(ws, dev, points, offsets, S, g, vol->N, vol->M, nullptr, &cv, C, o, st);
}

int fastcod_volume_destroy(fastcod_volume *vol) {
    g_last_error.clear();
    if (!vol) return FASTCOD_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(vol->device);
    hipError_t e = hipDeviceSynchronize();
    if (vol->ready) (void)hipEventDestroy(vol->ready);
    (void)hipFree(vol->buf);
    (void)hipSetDevice(prev);
    delete vol;
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    return FASTCOD_OK;
}

int fastcod_validate(const int64_t *offsets, int64_t S, const int32_t *roi, const int32_t *lab, const int32_t dims[3],
                     int32_t N, int32_t M, void *stream) {
    g_last_error.clear();
    int rc = check_volume_args(roi, lab, dims, N, M);
    if (rc) return rc;
    if (S < 0 || S > INT32_MAX || !offsets) return fail(FASTCOD_EINVAL, "bad offsets / n_streamlines");
    int dev;
    rc = current_device(&dev);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace &ws = *workspace_for(dev, st);
    std::lock_guard<std::mutex> lock(ws.mu);
    return run_validate(ws, offsets, S, roi, lab, dims, N, M, st, dev);
}

int fastcod_release(void) {
    g_last_error.clear();
    std::lock_guard<std::mutex> g(g_ws_mu);
    int prev = 0;
    (void)hipGetDevice(&prev);
    for (auto &kv : g_ws) {
        (void)hipSetDevice(kv.first.first);
        (void)hipDeviceSynchronize();
        Workspace *w = kv.second;
        w->compact.release();
        w->first.release();
        w->ovf.release();
        w->fallback.release();
        w->flags.release();
        w->ct.release();
        delete w;
    }
    g_ws.clear();
    (void)hipSetDevice(prev);
    return FASTCOD_OK;
}

}  // extern "C"
