// Host-side helpers shared by the library's translation units: error slot, device buffers,
// compact-volume layout, grid bounds, argument checks.
#pragma once

#include <math.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>

#include "fastcod.h"
#include "internal.h"

namespace fch {

// detail of the last failing call on this thread
inline std::string &last_error() {
    thread_local std::string s;
    return s;
}

inline int fail(int status, const std::string &msg) {
    last_error() = msg;
    return status;
}

inline int hip_fail(hipError_t e, const char *what) {
    return fail(FASTCOD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define FC_HIP(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)

// smallest float >= n
inline float float_bound(int32_t n) {
    float f = (float)n;
    if ((double)f < (double)n) f = nextafterf(f, INFINITY);
    return f;
}

inline int bit_width(uint32_t v) {
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

inline int current_device(int *dev) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return FASTCOD_OK;
}

inline int cu_count(int dev) {
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
constexpr int32_t kMaxCoarseWords = 8192;      // 32 KB of LDS per counting workgroup
constexpr int32_t kBatchedCoarseWords = 512;   // per-wavefront LDS coarse map of the batched kernel (2 KB)
struct CompactLayout {
    int32_t SBX, SBY, SBZ;
    int64_t W;        // words
    int64_t ntiles;
    int64_t nvox;
    bool packed;
    int32_t rbits;
    int32_t csx, csyz, CBX, CBY, CBZ, ncoarse_words;
    int64_t ncodes;   // capacity of the code array (every voxel unless sized by compact_layout_fit)
    size_t off_mb, off_tiles, off_coarse, off_codes, bytes;
};

inline bool compact_layout(const int32_t dims[3], int32_t N, int32_t M, CompactLayout &L,
                           int32_t max_coarse_words = kMaxCoarseWords, bool brick_coarse = false) {
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
    // coarse occupancy (kept in LDS by the counting kernel): one bit per 16x8x8 super-brick when
    // brick_coarse is asked for and the map fits max_coarse_words (the kernel then reuses the
    // super-brick index), else the smallest cube side 8, 16 or 32 whose map fits
    auto coarse_words = [&](int32_t csx, int32_t csyz) {
        L.csx = csx;
        L.csyz = csyz;
        L.CBX = (dims[0] + (1 << csx) - 1) >> csx;
        L.CBY = (dims[1] + (1 << csyz) - 1) >> csyz;
        L.CBZ = (dims[2] + (1 << csyz) - 1) >> csyz;
        const int64_t ncb = (int64_t)L.CBX * L.CBY * L.CBZ;
        L.ncoarse_words = (int32_t)(2 * ((ncb + 63) / 64));
        return L.ncoarse_words;
    };
    bool fits = brick_coarse && coarse_words(4, 3) <= max_coarse_words;
    for (int32_t c = 3; !fits && c <= 5; ++c) fits = coarse_words(c, c) <= max_coarse_words;
    if (!fits) return false;
    auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
    L.off_mb = 0;
    L.off_tiles = align(L.off_mb + 8 * (size_t)L.W);
    L.off_coarse = align(L.off_tiles + 4 * (size_t)L.ntiles);
    L.off_codes = align(L.off_coarse + 4 * (size_t)L.ncoarse_words);
    L.ncodes = L.nvox;
    L.bytes = L.off_codes + (L.packed ? 4 : 8) * (size_t)L.nvox;   // at most every voxel occupied
    // the counting kernel reads pairs and codes through one buffer resource with 32-bit offsets
    if (L.bytes >= (size_t(1) << 32) - 16) return false;
    return true;
}

// Shrinks the code array to `occupied` entries: the number of voxels with 0 <= roi < N or
// 0 <= lab < M, the test the build uses to set occupancy bits (counted by the caller).
inline void compact_layout_fit(CompactLayout &L, int64_t occupied) {
    L.ncodes = occupied;
    L.bytes = L.off_codes + (L.packed ? 4 : 8) * (size_t)(occupied > 0 ? occupied : 1);
}

inline fc::CompactVol compact_view(void *buf, const CompactLayout &L, int32_t N, int32_t M) {
    char *b = static_cast<char *>(buf);
    fc::CompactVol cv;
    cv.mb = reinterpret_cast<const uint2 *>(b + L.off_mb);
    cv.coarse = reinterpret_cast<const uint32_t *>(b + L.off_coarse);
    cv.csx = L.csx;
    cv.csyz = L.csyz;
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
    cv.ncodes = L.ncodes;
    cv.codes_off = (uint32_t)L.off_codes;
    cv.span = (uint32_t)(L.off_codes + (L.packed ? 4 : 8) * (size_t)L.ncodes);
    return cv;
}

inline fc::Grid make_grid(const int32_t dims[3]) {
    fc::Grid g;
    g.X = dims[0];
    g.Y = dims[1];
    g.Z = dims[2];
    g.Xf = float_bound(dims[0]);
    g.Yf = float_bound(dims[1]);
    g.Zf = float_bound(dims[2]);
    return g;
}

// Builds the compact volume of (roi, lab) into `buf` (L.bytes, laid out by compact_layout) on `st`.
inline hipError_t enqueue_compact_build(const int32_t *roi, const int32_t *lab, const int32_t dims[3], int32_t N,
                                        int32_t M, const CompactLayout &L, void *buf, int cus, hipStream_t st) {
    const fc::CompactVol cv = compact_view(buf, L, N, M);
    char *b = static_cast<char *>(buf);
    return fc::launch_compact_build(roi, lab, make_grid(dims), N, M, cv, reinterpret_cast<uint32_t *>(b + L.off_mb),
                                    b + L.off_codes, reinterpret_cast<uint32_t *>(b + L.off_tiles),
                                    reinterpret_cast<uint32_t *>(b + L.off_coarse), L.W, cus, st);
}

inline int check_volume_args(const int32_t *roi, const int32_t *lab, const int32_t dims[3], int32_t N, int32_t M) {
    if (!dims) return fail(FASTCOD_EINVAL, "dims is NULL");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return fail(FASTCOD_EINVAL, "dims must be >= 1");
    if ((int64_t)dims[0] * dims[1] * dims[2] >= (int64_t(1) << 31)) return fail(FASTCOD_EINVAL, "X*Y*Z must be < 2^31");
    if (N < 1 || M < 1) return fail(FASTCOD_EINVAL, "N and M must be >= 1");
    if ((int64_t)N * M >= (int64_t(1) << 31)) return fail(FASTCOD_EINVAL, "N*M must be < 2^31");
    if (!roi || !lab) return fail(FASTCOD_EINVAL, "volume pointer is NULL");
    return FASTCOD_OK;
}

}  // namespace fch
