// Host side of libfastcod.so: argument checks, workspaces, launch sequence, error model.
// The C-ABI is declared in include/fastcod.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <tuple>
#include <cstdio>
#include <map>
#include <vector>
#include <mutex>
#include <string>
#include <utility>

#include "fastcod.h"
#include "host.h"
#include "internal.h"

using namespace fch;

namespace {

struct Workspace {
    std::mutex mu;      // held for the whole enqueue of one call
    DevBuf compact;     // fastcod_count's per-call compact volume
    DevBuf first;       // chunk -> first streamline
    DevBuf ovf;         // overflow counter + queue
    DevBuf fallback;    // fallback scratch (all-zero between launches)
    DevBuf flags;       // validation flags
    DevBuf ct;          // transposed accumulation copy of C (C beyond the histogram's tiles)
    DevBuf ends;        // per-streamline end labels of the endpoint modes
    DevBuf pairs;       // appended C updates: slice lengths, tile histogram, slices, sorted copy
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;


Workspace *workspace_for(int dev, hipStream_t st) {
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto &w = g_ws[{dev, st}];
    if (!w) w = new Workspace();
    return w;
}

int check_stream_args(const float *points, const int64_t *offsets, int64_t S, int32_t *C, const fastcod_opts &o) {
    if (S < 0 || S > INT32_MAX) return fail(FASTCOD_EINVAL, "n_streamlines must be in [0, INT32_MAX]");
    if (!offsets) return fail(FASTCOD_EINVAL, "offsets is NULL");
    if (S > 0 && !points) return fail(FASTCOD_EINVAL, "points is NULL");
    if (!C) return fail(FASTCOD_EINVAL, "C_out is NULL");
    if (o.upsample < 1 || o.upsample > 4) return fail(FASTCOD_EINVAL, "upsample must be 1, 2, 3 or 4");
    if (o.upsample > 1 && o.mode != FASTCOD_MODE_PASSTHROUGH)
        return fail(FASTCOD_EINVAL, "upsampling is available for the pass-through mode only");
    if (!(o.scale == o.scale) || o.scale <= 0.0f || isinf(o.scale)) return fail(FASTCOD_EINVAL, "scale must be finite and > 0");
    if (o.variant < FASTCOD_VARIANT_AUTO || o.variant > FASTCOD_VARIANT_STREAM) return fail(FASTCOD_EINVAL, "unknown variant");
    if (o.batch != 0 && o.batch != 2 && o.batch != 4) return fail(FASTCOD_EINVAL, "batch must be 0, 2 or 4");
    if (o.blocks_per_cu < 0) return fail(FASTCOD_EINVAL, "blocks_per_cu must be >= 0");
    if (o.mode < FASTCOD_MODE_PASSTHROUGH || o.mode > FASTCOD_MODE_SEED_END) return fail(FASTCOD_EINVAL, "unknown mode");
    if (o.pair_capacity < 0) return fail(FASTCOD_EINVAL, "pair_capacity must be >= 0");
    return FASTCOD_OK;
}

constexpr int kBlocksPerCU = 8;            // resident 256-thread workgroups per CU (count kernels)
// Flat-stream point ranges per wavefront (on average), handed out dynamically.  Each range start
// costs a few dependent loads and a pipeline fill, so smaller calls take fewer, longer ranges; from
// kLongRangesFrom streamlines the ranges are long anyway, and more of them (tapering, largest
// first) let the wavefronts finish together.
constexpr int kRangesPerWave = 4;
constexpr int kRangesPerWaveShort = 2;
constexpr int64_t kLongRangesFrom = int64_t(1) << 21;   // also the threshold for 4-window batches

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
    if (o.mode == FASTCOD_MODE_SEED_END) {
        // Alg. 1's count: one update per streamline, straight into C
        if (!(o.flags & FASTCOD_ACCUMULATE)) FC_HIP(fc::launch_fill_i32(C, (int64_t)N * M, 0, cus, st));
        fc::CountArgs a{};
        a.pts = points;
        a.offsets = offsets;
        a.S = S;
        a.g = g;
        a.scale = o.scale;
        a.C = C;
        a.si = (uint32_t)M;
        a.sm = 1u;
        if (o.event_begin) FC_HIP(hipEventRecord((hipEvent_t)o.event_begin, st));
        FC_HIP(fc::launch_count_seed_end(a, rv, cv, cus, st));
        if (o.event_end) FC_HIP(hipEventRecord((hipEvent_t)o.event_end, st));
        return FASTCOD_OK;
    }
    // The flat-stream path appends its pair updates to per-wavefront slices and adds their
    // histogram into C tile by tile.  Past kMaxPairTiles tiles it accumulates atomically into a
    // transposed workspace copy CT[M][N] instead: the rows of one streamline are neighbouring ROI
    // indices, so its pair updates share memory lines there.
    const int64_t NM = (int64_t)N * M;
    const int64_t ntiles = (NM + (1 << fc::kPairTileLog2) - 1) >> fc::kPairTileLog2;
    const bool append = cv != nullptr && S > 0 && ntiles <= fc::kMaxPairTiles;
    const bool transposed = !append && cv != nullptr && S > 0 && M > 1 && N >= 64;
    const bool zero_c = !(o.flags & FASTCOD_ACCUMULATE) && !transposed;
    // the compact path's partition launch zeroes C and the per-call counters itself
    const bool fused_zero = cv != nullptr && S > 0;
    if (zero_c && !fused_zero) FC_HIP(fc::launch_fill_i32(C, (int64_t)N * M, 0, cus, st));
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
    a.up = o.upsample;
    a.ends = fc::EndLabels{0, nullptr, nullptr};
    if (o.mode == FASTCOD_MODE_END || o.mode == FASTCOD_MODE_BOTH_ENDS) {
        const int nl = o.mode == FASTCOD_MODE_BOTH_ENDS ? 2 : 1;
        FC_HIP(ws.ends.ensure(4 * (size_t)S * nl, false));
        int32_t *last = static_cast<int32_t *>(ws.ends.p);
        int32_t *first = nl == 2 ? last + S : nullptr;
        a.ends = fc::EndLabels{o.mode, last, first};
        FC_HIP(fc::launch_end_labels(a, rv, cv, o.mode, last, first, cus, st));
    }
    a.ovf.count = static_cast<unsigned long long *>(ws.ovf.p);
    a.ovf.list = reinterpret_cast<int64_t *>(static_cast<char *>(ws.ovf.p) + 256);
    a.ovf.cap = S;
    a.ovf.work = static_cast<unsigned long long *>(ws.ovf.p) + 1;
    fc::FallbackScratch fs;
    int rc = fallback_scratch(ws, N, M, fs);
    if (rc) return rc;
    if (!fused_zero) FC_HIP(fc::launch_fill_u64(a.ovf.count, 2, cus, st));   // overflow count and range counter
    const int64_t resident = (int64_t)cus * kBlocksPerCU;
    if (cv) {
        // 4-window batches keep more loads in flight per wavefront; they pay off once each
        // wavefront's point ranges are long enough to amortise their deeper pipeline start
        const bool long_ranges = S >= kLongRangesFrom;
        const int batch = o.batch != 0 ? o.batch : (long_ranges ? 4 : 2);
        int per_cu = fc::count_stream_blocks_per_cu(o.scale != 1.0f, cv->packed != 0, batch, a.ends.mode != 0,
                                                    a.up, 4 * (size_t)cv->ncoarse_words);
        if (o.blocks_per_cu > 0 && o.blocks_per_cu < per_cu) per_cu = o.blocks_per_cu;
        const int64_t blocks = (int64_t)cus * per_cu;
        const int64_t nparts = blocks * fc::kWavesPerBlock * (long_ranges ? kRangesPerWave : kRangesPerWaveShort);
        FC_HIP(ws.first.ensure(4 * (size_t)(nparts + 1), false));
        int32_t *first = static_cast<int32_t *>(ws.first.p);
        // pair slices: pair_capacity entries in all (default 8 per streamline, between 2^20 and
        // 2^28), split evenly between the wavefronts; a full slice sends the rest of its
        // wavefront's updates to C as atomics
        const int64_t nwaves = blocks * fc::kWavesPerBlock;
        int64_t total = o.pair_capacity > 0 ? o.pair_capacity : std::min<int64_t>(std::max<int64_t>(8 * S, 1 << 20), 1 << 28);
        total = std::min<int64_t>(total, INT32_MAX);
        const int64_t cap = append ? total / nwaves : 0;
        auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
        const size_t off_hist = align(4 * (size_t)nwaves);
        const size_t off_pairs = align(off_hist + 4 * (size_t)fc::pair_hist_words(ntiles));
        const size_t off_sorted = align(off_pairs + 4 * (size_t)(nwaves * cap));
        FC_HIP(ws.pairs.ensure(off_sorted + 4 * (size_t)(nwaves * cap), false));
        char *pb = static_cast<char *>(ws.pairs.p);
        fc::PairOut po;
        po.counts = reinterpret_cast<uint32_t *>(pb);
        po.pairs = reinterpret_cast<uint32_t *>(pb + off_pairs);
        po.cap = (uint32_t)cap;
        fc::ZeroRanges z;
        if (zero_c) {
            z.w32[0] = C;
            z.n32[0] = NM;
        }
        if (append) {
            z.w32[1] = reinterpret_cast<int32_t *>(pb + off_hist);
            z.n32[1] = fc::pair_hist_cursor_words(ntiles);
        }
        z.w64 = a.ovf.count;   // overflow count and range counter
        z.n64 = 2;
        // tapering ranges (largest first) end the launch evenly when ranges are long; short ones
        // would only add per-range work
        FC_HIP(fc::launch_partition(offsets, S, nparts, first, z, long_ranges, cus, st));
        if (o.event_begin) FC_HIP(hipEventRecord((hipEvent_t)o.event_begin, st));
        FC_HIP(fc::launch_count_stream(a, *cv, first, nparts, (int)blocks, batch, po, st));
        if (o.event_end) FC_HIP(hipEventRecord((hipEvent_t)o.event_end, st));
        FC_HIP(fc::launch_fallback_compact(a, *cv, fs, st));
        if (append)
            FC_HIP(fc::launch_pair_histogram(po, (int32_t)nwaves, (int32_t)ntiles, C, NM,
                                             reinterpret_cast<uint32_t *>(pb + off_hist),
                                             reinterpret_cast<uint32_t *>(pb + off_sorted), cus, st));
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

// ---- batched plans ----

struct PlanSched {
    int batch = 4, blocks_per_cu = 0, items_per_wave = 4;
    float ms = 0.f;
};

std::string arch_name(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

int log2_bucket(double v) {
    int b = 0;
    while (v >= 2.0) {
        v /= 2.0;
        ++b;
    }
    return b;
}

bool read_tune_cache(const char *path, const std::string &key, PlanSched &out) {
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char k[512];
    PlanSched ps;
    bool found = false;
    while (fscanf(f, "%511s %d %d %d %f", k, &ps.batch, &ps.blocks_per_cu, &ps.items_per_wave, &ps.ms) == 5)
        if (key == k) {
            out = ps;
            found = true;
        }
    fclose(f);
    return found;
}

void append_tune_cache(const char *path, const std::string &key, const PlanSched &ps) {
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %.4f\n", key.c_str(), ps.batch, ps.blocks_per_cu, ps.items_per_wave, ps.ms);
    fclose(f);
}

}  // namespace


struct fastcod_plan {
    int device = 0;
    int32_t n = 0;
    std::vector<fc::StreamSubject> subs;   // host copy of the descriptor table
    std::vector<int64_t> points;           // P of every subject (read at creation)
    std::vector<int64_t> sizes;            // N*M of every subject
    std::vector<void *> volumes;           // owned compact volumes and the transposed copies of C
    std::vector<fc::TransposeJob> transposed;   // subjects counted into CT[M][N], transposed into C_out
    int64_t transpose_tiles = 0;
    DevBuf d_transposed;                        // device copy of `transposed`
    DevBuf d_subs, d_sizes, d_item_base, d_items, d_ovf, d_fallback;
    fc::FallbackScratch fs{};
    fc::Overflow ovf{};
    PlanSched sched;
    int64_t nitems = 0;
    int blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Work-item split for a schedule: items in proportion to every subject's points.
int plan_items(fastcod_plan &pl, const PlanSched &ps, int cus, hipStream_t st) {
    int per_cu = fc::count_batched_blocks_per_cu(ps.batch, kBatchedCoarseWords);
    if (ps.blocks_per_cu > 0 && ps.blocks_per_cu < per_cu) per_cu = ps.blocks_per_cu;
    pl.blocks = cus * per_cu;
    const int64_t total = (int64_t)pl.blocks * fc::kWavesPerBlock * ps.items_per_wave;
    double ptot = 0;
    for (int64_t p : pl.points) ptot += (double)p;
    std::vector<int64_t> base(pl.n + 1, 0);
    for (int32_t k = 0; k < pl.n; ++k) {
        int64_t ni = 0;
        if (pl.subs[k].S > 0) {
            ni = ptot > 0 ? (int64_t)((double)total * (double)pl.points[k] / ptot + 0.5) : 1;
            if (ni < 1) ni = 1;
            if (ni > pl.subs[k].S) ni = pl.subs[k].S;
        }
        base[k + 1] = base[k] + ni;
    }
    pl.nitems = base[pl.n];
    FC_HIP(pl.d_item_base.ensure(8 * (size_t)(pl.n + 1), false));
    FC_HIP(pl.d_items.ensure(8 * (size_t)(pl.nitems + 1), false));
    FC_HIP(hipMemcpyAsync(pl.d_item_base.p, base.data(), 8 * (size_t)(pl.n + 1), hipMemcpyHostToDevice, st));
    FC_HIP(hipStreamSynchronize(st));
    return FASTCOD_OK;
}

// The launch sequence (eager or under capture).
int plan_enqueue(fastcod_plan &pl, int cus, hipStream_t st) {
    const auto *subs = static_cast<const fc::StreamSubject *>(pl.d_subs.p);
    FC_HIP(fc::launch_zero_subjects(subs, static_cast<const int64_t *>(pl.d_sizes.p), pl.n, cus, st));
    FC_HIP(fc::launch_fill_u64(pl.ovf.count, 2, cus, st));
    if (pl.nitems > 0) {
        FC_HIP(fc::launch_partition_batched(subs, static_cast<const int64_t *>(pl.d_item_base.p), pl.n, pl.nitems,
                                            static_cast<int2 *>(pl.d_items.p), cus, st));
        FC_HIP(fc::launch_count_batched(subs, static_cast<const int2 *>(pl.d_items.p), pl.nitems, pl.ovf,
                                        kBatchedCoarseWords, pl.blocks, pl.sched.batch, st));
        FC_HIP(fc::launch_fallback_batched(subs, pl.n, pl.ovf, pl.fs, st));
    }
    FC_HIP(fc::launch_transpose_many(static_cast<const fc::TransposeJob *>(pl.d_transposed.p),
                                     (int32_t)pl.transposed.size(), pl.transpose_tiles, cus, st));
    return FASTCOD_OK;
}

int plan_capture(fastcod_plan &pl, int cus) {
    hipStream_t cs = nullptr;
    FC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = FASTCOD_OK;
    if (e == hipSuccess) rc = plan_enqueue(pl, cus, cs);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    pl.graph = g;
    FC_HIP(hipGraphInstantiate(&pl.exec, g, nullptr, nullptr, 0));
    return FASTCOD_OK;
}

void plan_free(fastcod_plan *pl) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    for (void *v : pl->volumes) (void)hipFree(v);
    pl->d_subs.release();
    pl->d_sizes.release();
    pl->d_item_base.release();
    pl->d_items.release();
    pl->d_ovf.release();
    pl->d_fallback.release();
    pl->d_transposed.release();
    delete pl;
}

int plan_check(const fastcod_subject *subjects, int32_t n) {
    for (int32_t k = 0; k < n; ++k) {
        const fastcod_subject &u = subjects[k];
        int rc = check_volume_args(u.roi_index_vol, u.target_label_vol, u.dims, u.N, u.M);
        if (rc) return fail(rc, "subject " + std::to_string(k) + ": " + last_error());
        fastcod_opts o = fastcod_default_opts();
        o.scale = u.scale;
        rc = check_stream_args(u.points, u.offsets, u.n_streamlines, u.C_out, o);
        if (rc) return fail(rc, "subject " + std::to_string(k) + ": " + last_error());
        CompactLayout L;
        if (!compact_layout(u.dims, u.N, u.M, L, kBatchedCoarseWords))
            return fail(FASTCOD_EINVAL, "subject " + std::to_string(k) + ": grid too thin for the compact volume");
    }
    return FASTCOD_OK;
}

int plan_build(const fastcod_subject *subjects, int32_t n, uint32_t flags, const char *tune_cache, hipStream_t st,
               fastcod_plan *pl) {
    int dev;
    int rc = current_device(&dev);
    if (rc) return rc;
    pl->device = dev;
    pl->n = n;
    const int cus = cu_count(dev);
    // validate, and build one compact volume per distinct volume pair
    struct Key {
        const int32_t *roi, *lab;
        int32_t X, Y, Z, N, M;
        bool operator<(const Key &o) const {
            return std::tie(roi, lab, X, Y, Z, N, M) < std::tie(o.roi, o.lab, o.X, o.Y, o.Z, o.N, o.M);
        }
    };
    std::map<Key, fc::CompactVol> built;
    int64_t total_s = 0, max_nw_n = 1, max_nw_m = 1, max_m = 1;
    for (int32_t k = 0; k < n; ++k) {
        const fastcod_subject &u = subjects[k];
        rc = check_volume_args(u.roi_index_vol, u.target_label_vol, u.dims, u.N, u.M);
        if (rc) return fail(rc, "subject " + std::to_string(k) + ": " + last_error());
        fastcod_opts o = fastcod_default_opts();
        o.scale = u.scale;
        rc = check_stream_args(u.points, u.offsets, u.n_streamlines, u.C_out, o);
        if (rc) return fail(rc, "subject " + std::to_string(k) + ": " + last_error());
        CompactLayout L;
        if (!compact_layout(u.dims, u.N, u.M, L, kBatchedCoarseWords))
            return fail(FASTCOD_EINVAL, "subject " + std::to_string(k) + ": grid too thin for the compact volume");
        const Key key{u.roi_index_vol, u.target_label_vol, u.dims[0], u.dims[1], u.dims[2], u.N, u.M};
        fc::CompactVol cv;
        auto it = built.find(key);
        if (it == built.end()) {
            void *buf = nullptr;
            hipError_t e = hipMalloc(&buf, L.bytes);
            if (e != hipSuccess) return fail(FASTCOD_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
            pl->volumes.push_back(buf);
            cv = compact_view(buf, L, u.N, u.M);
            FC_HIP(enqueue_compact_build(u.roi_index_vol, u.target_label_vol, u.dims, u.N, u.M, L, buf, cus, st));
            built[key] = cv;
        } else {
            cv = it->second;
        }
        fc::StreamSubject ss;
        ss.pts = u.points;
        ss.offsets = u.offsets;
        ss.S = u.n_streamlines;
        ss.s_begin = 0;
        ss.g = make_grid(u.dims);
        ss.scale = u.scale;
        ss.cv = cv;
        ss.C = u.C_out;
        ss.si = (uint32_t)u.M;
        ss.sm = 1u;
        ss.ends = fc::EndLabels{0, nullptr, nullptr};
        ss.up = 1;
        pl->subs.push_back(ss);
        pl->sizes.push_back((int64_t)u.N * u.M);
        total_s += u.n_streamlines;
        max_nw_n = std::max<int64_t>(max_nw_n, (u.N + 31) / 32);
        max_nw_m = std::max<int64_t>(max_nw_m, (u.M + 31) / 32);
        max_m = std::max<int64_t>(max_m, u.M);
    }
    // point counts (the item split follows them)
    pl->points.assign(n, 0);
    for (int32_t k = 0; k < n; ++k)
        if (pl->subs[k].S > 0)
            FC_HIP(hipMemcpyAsync(&pl->points[k], pl->subs[k].offsets + pl->subs[k].S, 8, hipMemcpyDeviceToHost, st));
    FC_HIP(hipStreamSynchronize(st));
    // Subjects with a C of their own (no other subject writes its C_out) count into a transposed
    // copy CT[M][N] in one plan-owned allocation, transposed into C_out at the end of each launch:
    // a streamline's rows are neighbouring ROI indices, so its updates under one label share memory
    // lines there, where C[N][M] spreads them one row apart.
    {
        std::map<const int32_t *, int> writers;
        for (const auto &ss : pl->subs) writers[ss.C]++;
        std::vector<int32_t> pick;
        size_t words = 0;
        for (int32_t k = 0; k < n; ++k) {
            const fastcod_subject &u = subjects[k];
            if (pl->subs[k].S > 0 && u.M > 1 && u.N >= 64 && writers[u.C_out] == 1) {
                pick.push_back(k);
                words += (size_t)u.N * (size_t)u.M;
            }
        }
        if (words > 0) {
            void *buf = nullptr;
            hipError_t e = hipMalloc(&buf, 4 * words);
            if (e != hipSuccess) return fail(FASTCOD_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
            pl->volumes.push_back(buf);
            int32_t *ct = static_cast<int32_t *>(buf);
            for (int32_t k : pick) {
                const fastcod_subject &u = subjects[k];
                pl->transposed.push_back({ct, u.C_out, u.N, u.M, pl->transpose_tiles});
                pl->transpose_tiles += (int64_t)((u.N + fc::kTransposeTile - 1) / fc::kTransposeTile) *
                                       (int64_t)((u.M + fc::kTransposeTile - 1) / fc::kTransposeTile);
                pl->subs[k].C = ct;
                pl->subs[k].si = 1u;
                pl->subs[k].sm = (uint32_t)u.N;
                ct += (size_t)u.N * (size_t)u.M;
            }
        }
    }
    // device tables
    if (!pl->transposed.empty()) {
        const size_t tb = sizeof(fc::TransposeJob) * pl->transposed.size();
        FC_HIP(pl->d_transposed.ensure(tb, false));
        FC_HIP(hipMemcpyAsync(pl->d_transposed.p, pl->transposed.data(), tb, hipMemcpyHostToDevice, st));
    }
    FC_HIP(pl->d_subs.ensure(sizeof(fc::StreamSubject) * (size_t)n, false));
    FC_HIP(pl->d_sizes.ensure(8 * (size_t)n, false));
    FC_HIP(hipMemcpyAsync(pl->d_subs.p, pl->subs.data(), sizeof(fc::StreamSubject) * (size_t)n, hipMemcpyHostToDevice, st));
    FC_HIP(hipMemcpyAsync(pl->d_sizes.p, pl->sizes.data(), 8 * (size_t)n, hipMemcpyHostToDevice, st));
    FC_HIP(pl->d_ovf.ensure(256 + 8 * (size_t)std::max<int64_t>(total_s, 1), false));
    pl->ovf.count = static_cast<unsigned long long *>(pl->d_ovf.p);
    pl->ovf.work = pl->ovf.count + 1;
    pl->ovf.list = reinterpret_cast<int64_t *>(static_cast<char *>(pl->d_ovf.p) + 256);
    pl->ovf.cap = std::max<int64_t>(total_s, 1);
    pl->fs.nwordsN = (int32_t)max_nw_n;
    pl->fs.nwordsM = (int32_t)max_nw_m;
    pl->fs.stride = (max_nw_n + max_nw_m + max_m + 63) & ~int64_t(63);
    int64_t fb = (int64_t(256) << 20) / (4 * pl->fs.stride);
    fb = std::min<int64_t>(std::max<int64_t>(fb, 1), 64);
    pl->fs.blocks = (int32_t)fb;
    FC_HIP(pl->d_fallback.ensure((size_t)(4 * pl->fs.stride * fb), true));
    pl->fs.words = static_cast<uint32_t *>(pl->d_fallback.p);
    // schedule: cache, tuner, or defaults
    double ptot = 0, nm = 0, spts = 0;
    for (int32_t k = 0; k < n; ++k) {
        ptot += (double)pl->points[k];
        nm += (double)pl->sizes[k];
        spts += (double)pl->subs[k].S;
    }
    const std::string key = arch_name(dev) + ":cu" + std::to_string(cus) + ":n" + std::to_string(log2_bucket(n)) +
                            ":P" + std::to_string(log2_bucket(ptot)) + ":NM" + std::to_string(log2_bucket(nm / n)) +
                            ":T" + std::to_string(log2_bucket(spts > 0 ? ptot / spts : 0));
    PlanSched ps;
    if (read_tune_cache(tune_cache, key, ps)) {
        pl->sched = ps;
    } else if (flags & FASTCOD_PLAN_TUNE) {
        hipEvent_t e0, e1;
        FC_HIP(hipEventCreate(&e0));
        FC_HIP(hipEventCreate(&e1));
        PlanSched best;
        best.ms = -1.f;
        for (int batch : {2, 4}) {
            const int occ = fc::count_batched_blocks_per_cu(batch, kBatchedCoarseWords);
            for (int bpc : {occ, occ - 1, occ - 2}) {
                if (bpc < 1) continue;
                for (int ipw : {2, 4, 8, 16}) {
                    PlanSched c;
                    c.batch = batch;
                    c.blocks_per_cu = bpc;
                    c.items_per_wave = ipw;
                    rc = plan_items(*pl, c, cus, st);
                    if (rc) return rc;
                    pl->sched = c;
                    float ms = 0.f;
                    for (int rep = 0; rep < 2; ++rep) {
                        FC_HIP(hipEventRecord(e0, st));
                        rc = plan_enqueue(*pl, cus, st);
                        if (rc) return rc;
                        FC_HIP(hipEventRecord(e1, st));
                        FC_HIP(hipEventSynchronize(e1));
                        FC_HIP(hipEventElapsedTime(&ms, e0, e1));
                    }
                    c.ms = ms;
                    if (best.ms < 0.f || ms < best.ms) best = c;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        pl->sched = best;
        append_tune_cache(tune_cache, key, best);
    } else {
        pl->sched = PlanSched{};
    }
    rc = plan_items(*pl, pl->sched, cus, st);
    if (rc) return rc;
    return plan_capture(*pl, cus);
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
    o.mode = FASTCOD_MODE_PASSTHROUGH;
    o.pair_capacity = 0;
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

const char *fastcod_last_error(void) { return last_error().c_str(); }

int fastcod_count_ex(const float *points, const int64_t *offsets, int64_t S, const int32_t *roi, const int32_t *lab,
                     const int32_t dims[3], int32_t N, int32_t M, int32_t *C, const fastcod_opts *opts, void *stream) {
    last_error().clear();
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
    const bool compact_ok = compact_layout(dims, N, M, L, kMaxCoarseWords, true);
    if (o.variant == FASTCOD_VARIANT_STREAM && !compact_ok)
        return fail(FASTCOD_EINVAL, "grid too thin for the compact volume; use FASTCOD_VARIANT_WAVE");
    if (o.variant == FASTCOD_VARIANT_WAVE || !compact_ok) {
        fc::RasterVol rv{roi, lab, dims[0], dims[0] * dims[1], N, M};
        return enqueue_count(ws, dev, points, offsets, S, g, N, M, &rv, nullptr, C, o, st);
    }
    FC_HIP(ws.compact.ensure(L.bytes, false));
    fc::CompactVol cv = compact_view(ws.compact.p, L, N, M);
    FC_HIP(enqueue_compact_build(roi, lab, dims, N, M, L, ws.compact.p, cu_count(dev), st));
    return enqueue_count(ws, dev, points, offsets, S, g, N, M, nullptr, &cv, C, o, st);
}

int fastcod_count(const float *points, const int64_t *offsets, int64_t S, const int32_t *roi, const int32_t *lab,
                  const int32_t dims[3], int32_t N, int32_t M, int32_t *C, void *stream) {
    return fastcod_count_ex(points, offsets, S, roi, lab, dims, N, M, C, nullptr, stream);
}

int fastcod_volume_create(const int32_t *roi, const int32_t *lab, const int32_t dims[3], int32_t N, int32_t M,
                          void *stream, fastcod_volume **out) {
    last_error().clear();
    if (!out) return fail(FASTCOD_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_volume_args(roi, lab, dims, N, M);
    if (rc) return rc;
    CompactLayout L;
    if (!compact_layout(dims, N, M, L, kMaxCoarseWords, true)) return fail(FASTCOD_EINVAL, "grid too thin for a compact volume");
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
    {
        Workspace &ws = *workspace_for(dev, st);
        std::lock_guard<std::mutex> lock(ws.mu);
        e = enqueue_compact_build(roi, lab, dims, N, M, L, buf, cu_count(dev), st);
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
    last_error().clear();
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
    last_error().clear();
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
    last_error().clear();
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

int fastcod_parcellate(const int32_t *C, int32_t N, int32_t M, int32_t *label_out, float *frac_out,
                       int64_t *sums_out, void *stream) {
    last_error().clear();
    if (N < 0 || M < 1) return fail(FASTCOD_EINVAL, "need N >= 0 and M >= 1");
    if ((int64_t)N * M >= (int64_t(1) << 31)) return fail(FASTCOD_EINVAL, "N*M must be < 2^31");
    if (N > 0 && !C) return fail(FASTCOD_EINVAL, "C is NULL");
    int dev;
    const int rc = current_device(&dev);
    if (rc) return rc;
    FC_HIP(fc::launch_parcellate(C, N, M, label_out, frac_out, sums_out, cu_count(dev),
                                 static_cast<hipStream_t>(stream)));
    return FASTCOD_OK;
}

int fastcod_release(void) {
    last_error().clear();
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
        w->ends.release();
        delete w;
    }
    g_ws.clear();
    (void)hipSetDevice(prev);
    return FASTCOD_OK;
}

int fastcod_plan_create(const fastcod_subject *subjects, int32_t n, uint32_t flags, const char *tune_cache,
                        void *stream, fastcod_plan **out) {
    last_error().clear();
    if (!out) return fail(FASTCOD_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !subjects) return fail(FASTCOD_EINVAL, "need at least one subject");
    const int rc0 = plan_check(subjects, n);   // argument errors before any HIP call
    if (rc0) return rc0;
    fastcod_plan *pl = new fastcod_plan();
    const int rc = plan_build(subjects, n, flags, tune_cache, static_cast<hipStream_t>(stream), pl);
    if (rc) {
        const std::string msg = last_error();
        (void)hipDeviceSynchronize();
        plan_free(pl);
        return fail(rc, msg);
    }
    *out = pl;
    return FASTCOD_OK;
}

int fastcod_plan_launch(fastcod_plan *plan, void *stream) {
    last_error().clear();
    if (!plan || !plan->exec) return fail(FASTCOD_EINVAL, "plan is NULL");
    int dev;
    const int rc = current_device(&dev);
    if (rc) return rc;
    if (dev != plan->device) return fail(FASTCOD_EINVAL, "plan lives on another device");
    FC_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    return FASTCOD_OK;
}

int fastcod_plan_get_schedule(const fastcod_plan *plan, fastcod_schedule *out) {
    last_error().clear();
    if (!plan || !out) return fail(FASTCOD_EINVAL, "NULL argument");
    out->batch = plan->sched.batch;
    out->blocks_per_cu = plan->blocks / std::max(1, cu_count(plan->device));
    out->items_per_wave = plan->sched.items_per_wave;
    out->tuned_ms = plan->sched.ms;
    return FASTCOD_OK;
}

int fastcod_plan_destroy(fastcod_plan *plan) {
    last_error().clear();
    if (!plan) return FASTCOD_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(plan->device);
    const hipError_t e = hipDeviceSynchronize();
    plan_free(plan);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    return FASTCOD_OK;
}

int fastcod_count_batched(const fastcod_subject *subjects, int32_t n, void *stream) {
    fastcod_plan *pl = nullptr;
    int rc = fastcod_plan_create(subjects, n, 0, nullptr, stream, &pl);
    if (rc) return rc;
    rc = fastcod_plan_launch(pl, stream);
    if (rc == FASTCOD_OK) {
        const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    }
    const std::string msg = last_error();
    fastcod_plan_destroy(pl);
    if (rc) return fail(rc, msg);
    return FASTCOD_OK;
}

}  // extern "C"
