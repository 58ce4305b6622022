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
#include <thread>
#include <utility>

#include "fastcod.h"
#include "fastcod_probe.h"
#include "host.h"
#include "internal.h"

using namespace fch;

namespace {

struct Workspace {
    std::mutex mu;      // held for the whole enqueue of one call
    int refs = 0;       // calls holding the workspace (guarded by g_ws_mu)
    uint64_t last_use = 0;   // (guarded by g_ws_mu)
    DevBuf compact;     // fastcod_count's per-call compact volume
    DevBuf first;       // chunk -> first streamline
    DevBuf ovf;         // overflow counter + queue
    DevBuf fallback;    // fallback scratch (all-zero between launches)
    DevBuf flags;       // validation flags
    DevBuf ct;          // transposed accumulation copy of C (C beyond the histogram's tiles)
    DevBuf ends;        // per-streamline end labels of the endpoint modes
    DevBuf pairs;       // appended C updates: slice lengths, tile histogram, slices, sorted copy
    void free_buffers() {
        for (DevBuf *b : {&compact, &first, &ovf, &fallback, &flags, &ct, &ends, &pairs}) b->release();
    }
};

// Workspaces are kept per (device, stream): calls on one stream are serialised by that stream, so
// they can reuse one set of buffers.  hipStreamPerThread names a different stream in every thread,
// so for that handle the calling thread is part of the key.  At most kMaxWorkspacesPerDevice are
// kept per device; a new one then replaces the least recently used idle one, after a device
// synchronisation (its stream may still be using it).
struct WsKey {
    int dev;
    hipStream_t st;
    std::thread::id tid;
    bool operator<(const WsKey &o) const { return std::tie(dev, st, tid) < std::tie(o.dev, o.st, o.tid); }
};
constexpr int kMaxWorkspacesPerDevice = 8;
std::mutex g_ws_mu;
std::map<WsKey, Workspace *> g_ws;
uint64_t g_ws_clock = 0;

// with g_ws_mu held and `dev` current: frees idle workspaces of dev until fewer than the limit remain
void evict_workspaces(int dev) {
    for (;;) {
        int n = 0;
        auto lru = g_ws.end();
        for (auto it = g_ws.begin(); it != g_ws.end(); ++it) {
            if (it->first.dev != dev) continue;
            ++n;
            if (it->second->refs == 0 && (lru == g_ws.end() || it->second->last_use < lru->second->last_use)) lru = it;
        }
        if (n < kMaxWorkspacesPerDevice || lru == g_ws.end()) return;
        (void)hipDeviceSynchronize();
        lru->second->free_buffers();
        delete lru->second;
        g_ws.erase(lru);
    }
}

// A workspace held for the duration of one call (dev must be the current device).
class WsRef {
  public:
    WsRef(int dev, hipStream_t st) {
        std::lock_guard<std::mutex> g(g_ws_mu);
        const WsKey k{dev, st, st == hipStreamPerThread ? std::this_thread::get_id() : std::thread::id()};
        auto it = g_ws.find(k);
        if (it != g_ws.end()) {
            w_ = it->second;
        } else {
            evict_workspaces(dev);
            w_ = new Workspace();
            g_ws[k] = w_;
        }
        ++w_->refs;
        w_->last_use = ++g_ws_clock;
    }
    ~WsRef() {
        std::lock_guard<std::mutex> g(g_ws_mu);
        --w_->refs;
    }
    WsRef(const WsRef &) = delete;
    WsRef &operator=(const WsRef &) = delete;
    Workspace &operator*() const { return *w_; }
    Workspace *operator->() const { return w_; }

  private:
    Workspace *w_;
};

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
// Flat-stream point ranges per wavefront (on average), handed out largest first by the range
// queues, their sizes falling linearly from 1.5x to 0.5x the mean, so that the wavefronts finish
// together.  Each range start costs a few dependent loads and a pipeline fill.
constexpr int kRangesPerWave = 6;
constexpr int64_t kLongRangesFrom = int64_t(1) << 21;   // 4-window batches from this many streamlines
constexpr int64_t kDirectMaxStreamlines = int64_t(1) << 17;   // calls below this many streamlines ...
constexpr int64_t kDirectMaxEntries = int64_t(1) << 20;       // ... on a C of at most this many entries
                                                              // add their updates to C as atomics

// Fallback scratch layout for a C of N rows and M labels: per workgroup an N-bit map, an M-bit map
// and an M-entry label list, as many workgroups (<= 64) as fit `max_bytes`; false if not even one.
bool fallback_layout(int32_t N, int32_t M, int64_t max_bytes, fc::FallbackScratch &fs) {
    fs.nwordsN = (N + 31) / 32;
    fs.nwordsM = (M + 31) / 32;
    fs.stride = ((int64_t)fs.nwordsN + fs.nwordsM + M + 63) & ~int64_t(63);
    int64_t blocks = max_bytes / (4 * fs.stride);
    if (blocks > 64) blocks = 64;
    fs.blocks = (int32_t)(blocks < 1 ? 1 : blocks);
    fs.words = nullptr;
    return blocks >= 1;
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

// Decisions and scratch sizes of one counting call, fixed before anything is enqueued.
struct CountPlan {
    bool seed_end = false;     // Alg. 1's count: one update per streamline straight into C
    bool append = false;       // pair updates appended to slices, added into C by the tile histogram
    bool transposed = false;   // counted atomically into a transposed copy CT[M][N], then transposed
    bool zero_c = false;       // C overwritten (zeroed first)
    bool fused_zero = false;   // the partition launch does the zeroing
    int nl = 0;                // end labels per streamline (endpoint modes)
    int64_t NM = 0, ntiles = 0;
    int batch = 2;
    int64_t blocks = 0, nparts = 0, nwaves = 0, cap = 0;
    fc::FallbackScratch fs{};
    size_t off_hist = 0, off_pairs = 0, off_sorted = 0;
    // bytes of each scratch region (0 = not needed)
    size_t ovf_bytes = 0, ct_bytes = 0, ends_bytes = 0, fb_bytes = 0, first_bytes = 0, pairs_bytes = 0;
};

// Scratch regions of one call (device pointers, sized by CountPlan).  `fallback` must be all-zero.
struct CountScratch {
    void *ovf = nullptr;        // overflow count, range counter (256 B), then the overflow queue
    int32_t *ct = nullptr;      // transposed copy of C
    int32_t *ends = nullptr;    // end labels: last[S] (and first[S])
    uint32_t *fallback = nullptr;
    int32_t *first = nullptr;   // nparts + 1 range starts
    char *pairs = nullptr;      // slice lengths | tile histogram | slices | sorted copy
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// noalloc: a variant for a fixed scratch area -- no transposed copy of C (updates beyond the tile
// histogram go to C as atomics) and at most max_pairs appended updates.
int make_count_plan(int64_t S, int32_t N, int32_t M, const fc::CompactVol *cv, const fastcod_opts &o, int cus,
                    bool noalloc, int64_t max_pairs, int64_t max_fallback_bytes, CountPlan &cp) {
    cp = CountPlan{};
    if (o.mode == FASTCOD_MODE_SEED_END) {
        cp.seed_end = true;
        return FASTCOD_OK;
    }
    // The flat-stream path appends its pair updates to per-wavefront slices and adds their
    // histogram into C tile by tile.  Past kMaxPairTiles tiles it accumulates atomically into a
    // transposed workspace copy CT[M][N] instead: the rows of one streamline are neighbouring ROI
    // indices, so its pair updates share memory lines there.
    // Small calls (fewer than 2^17 streamlines) on a small C add their updates to C as atomics
    // instead: there the histogram's three launches cost more than the atomics they replace (10k
    // streamlines on a 64^3 grid: 41 against 62 us a call).  At 1M streamlines the pair buffer still
    // keeps the counting kernel 5-8% shorter; the whole call is then within a few percent either way.
    // An explicit pair_capacity keeps the pair buffer.
    cp.NM = (int64_t)N * M;
    cp.ntiles = (cp.NM + (1 << fc::kPairTileLog2) - 1) >> fc::kPairTileLog2;
    const bool direct = o.pair_capacity == 0 && S < kDirectMaxStreamlines && cp.NM <= kDirectMaxEntries;
    cp.append = cv != nullptr && S > 0 && cp.ntiles <= fc::kMaxPairTiles && !direct;
    cp.transposed = !noalloc && !cp.append && !direct && cv != nullptr && S > 0 && M > 1 && N >= 64;
    cp.zero_c = !(o.flags & FASTCOD_ACCUMULATE) && !cp.transposed;
    cp.fused_zero = cv != nullptr && S > 0;
    if (S == 0) return FASTCOD_OK;
    cp.ovf_bytes = fc::overflow_header_bytes(1) + 8 * (size_t)S;
    if (cp.transposed) cp.ct_bytes = 4 * (size_t)N * (size_t)M;
    if (o.mode == FASTCOD_MODE_END || o.mode == FASTCOD_MODE_BOTH_ENDS) {
        cp.nl = o.mode == FASTCOD_MODE_BOTH_ENDS ? 2 : 1;
        cp.ends_bytes = 4 * (size_t)S * cp.nl;
    }
    if (!fallback_layout(N, M, max_fallback_bytes, cp.fs))
        return fail(FASTCOD_ENOMEM, "the overflow fallback's bit maps for this N and M exceed the scratch area");
    cp.fb_bytes = 4 * (size_t)cp.fs.stride * (size_t)cp.fs.blocks;
    if (!cv) {
        int64_t blocks = (S + fc::kWavesPerBlock - 1) / fc::kWavesPerBlock;
        cp.blocks = std::min<int64_t>(blocks, (int64_t)cus * kBlocksPerCU);
        return FASTCOD_OK;
    }
    // 4-window batches keep more loads in flight per wavefront; they pay off once each
    // wavefront's point ranges are long enough to amortise their deeper pipeline start
    const bool long_ranges = S >= kLongRangesFrom;
    cp.batch = o.batch != 0 ? o.batch : (long_ranges ? 4 : 2);
    int per_cu = fc::count_stream_blocks_per_cu(o.scale != 1.0f, cv->packed != 0, cp.batch, cp.nl != 0, o.upsample,
                                                4 * (size_t)cv->ncoarse_words);
    if (o.blocks_per_cu > 0 && o.blocks_per_cu < per_cu) per_cu = o.blocks_per_cu;
    cp.blocks = (int64_t)cus * per_cu;
    cp.nparts = cp.blocks * fc::kWavesPerBlock * kRangesPerWave;
    cp.first_bytes = 4 * (size_t)(cp.nparts + 1);
    // pair slices: pair_capacity entries in all (default 8 per streamline, between 2^20 and
    // 2^28), split evenly between the wavefronts; a full slice sends the rest of its
    // wavefront's updates to C as atomics
    cp.nwaves = cp.blocks * fc::kWavesPerBlock;
    int64_t total = o.pair_capacity > 0 ? o.pair_capacity : std::min<int64_t>(std::max<int64_t>(8 * S, 1 << 20), 1 << 28);
    total = std::min<int64_t>(std::min<int64_t>(total, INT32_MAX), max_pairs);
    cp.cap = cp.append ? (total / cp.nwaves) & ~int64_t(3) : 0;   // 16-byte aligned slices
    if (cp.append) {
        cp.off_hist = align256(4 * (size_t)cp.nwaves);
        cp.off_pairs = align256(cp.off_hist + 4 * (size_t)fc::pair_hist_words(cp.ntiles));
        cp.off_sorted = align256(cp.off_pairs + 4 * (size_t)(cp.nwaves * cp.cap));
        cp.pairs_bytes = cp.off_sorted + 4 * (size_t)(cp.nwaves * cp.cap);
    } else {
        cp.pairs_bytes = 4 * (size_t)cp.nwaves;   // slice lengths only (every update is an atomic)
    }
    return FASTCOD_OK;
}

// The counting sequence on one stream, against a raster or a compact volume, with the scratch
// regions of `sc` (sized by `cp`).
int enqueue_count(const CountPlan &cp, const CountScratch &sc, int dev, const float *points, const int64_t *offsets,
                  int64_t S, const fc::Grid &g, int32_t N, int32_t M, const fc::RasterVol *rv,
                  const fc::CompactVol *cv, int32_t *C, const fastcod_opts &o, hipStream_t st) {
    const int cus = cu_count(dev);
    if (cp.seed_end) {
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
    if (cp.zero_c && !cp.fused_zero) FC_HIP(fc::launch_fill_i32(C, cp.NM, 0, cus, st));
    if (S == 0) {
        if (o.event_begin) FC_HIP(hipEventRecord((hipEvent_t)o.event_begin, st));
        if (o.event_end) FC_HIP(hipEventRecord((hipEvent_t)o.event_end, st));
        return FASTCOD_OK;
    }
    fc::CountArgs a;
    a.pts = points;
    a.offsets = offsets;
    a.S = S;
    a.g = g;
    a.scale = o.scale;
    a.C = C;
    a.si = (uint32_t)M;
    a.sm = 1u;
    if (cp.transposed) {
        a.C = sc.ct;
        a.si = 1u;
        a.sm = (uint32_t)N;
        FC_HIP(fc::launch_fill_i32(a.C, cp.NM, 0, cus, st));
    }
    a.up = o.upsample;
    a.ends = fc::EndLabels{0, nullptr, nullptr};
    if (cp.nl > 0) {
        int32_t *last = sc.ends;
        int32_t *first = cp.nl == 2 ? last + S : nullptr;
        a.ends = fc::EndLabels{o.mode, last, first};
        FC_HIP(fc::launch_end_labels(a, rv, cv, o.mode, last, first, cus, st));
    }
    a.ovf.count = static_cast<unsigned long long *>(sc.ovf);
    a.ovf.list = reinterpret_cast<int64_t *>(static_cast<char *>(sc.ovf) + fc::overflow_header_bytes(1));
    a.ovf.cap = S;
    a.ovf.work = a.ovf.count + fc::kQueueWords;
    fc::FallbackScratch fs = cp.fs;
    fs.words = sc.fallback;
    // overflow count and range queues
    const int64_t header_words = (int64_t)(fc::overflow_header_bytes(1) / 8);
    if (!cp.fused_zero) FC_HIP(fc::launch_fill_u64(a.ovf.count, header_words, cus, st));
    if (cv) {
        char *pb = sc.pairs;
        fc::PairOut po;
        po.counts = reinterpret_cast<uint32_t *>(pb);
        po.pairs = cp.append ? reinterpret_cast<uint32_t *>(pb + cp.off_pairs) : nullptr;
        po.cap = (uint32_t)cp.cap;
        fc::ZeroRanges z;
        if (cp.zero_c) {
            z.w32[0] = C;
            z.n32[0] = cp.NM;
        }
        if (cp.append) {
            z.w32[1] = reinterpret_cast<int32_t *>(pb + cp.off_hist);
            z.n32[1] = fc::pair_hist_cursor_words(cp.ntiles);
        }
        z.w64 = a.ovf.count;   // overflow count and range queues
        z.n64 = header_words;
        // tapering ranges (largest first) end the launch evenly
        FC_HIP(fc::launch_partition(offsets, S, cp.nparts, sc.first, z, true, cus, st));
        if (o.event_begin) FC_HIP(hipEventRecord((hipEvent_t)o.event_begin, st));
        FC_HIP(fc::launch_count_stream(a, *cv, sc.first, cp.nparts, (int)cp.blocks, cp.batch, po, st));
        if (o.event_end) FC_HIP(hipEventRecord((hipEvent_t)o.event_end, st));
        FC_HIP(fc::launch_fallback_compact(a, *cv, fs, st));
        if (cp.append)
            FC_HIP(fc::launch_pair_histogram(po, (int32_t)cp.nwaves, (int32_t)cp.ntiles, C, cp.NM,
                                             reinterpret_cast<uint32_t *>(pb + cp.off_hist),
                                             reinterpret_cast<uint32_t *>(pb + cp.off_sorted), cus, st));
        if (cp.transposed) FC_HIP(fc::launch_transpose(a.C, C, N, M, (o.flags & FASTCOD_ACCUMULATE) != 0, st));
    } else {
        if (o.event_begin) FC_HIP(hipEventRecord((hipEvent_t)o.event_begin, st));
        FC_HIP(fc::launch_count_wave(a, *rv, (int)cp.blocks, st));
        if (o.event_end) FC_HIP(hipEventRecord((hipEvent_t)o.event_end, st));
        FC_HIP(fc::launch_fallback_raster(a, *rv, fs, st));
    }
    return FASTCOD_OK;
}

// The counting sequence with the scratch regions taken from (and grown in) the stream's workspace.
int enqueue_count_ws(Workspace &ws, int dev, const float *points, const int64_t *offsets, int64_t S,
                     const fc::Grid &g, int32_t N, int32_t M, const fc::RasterVol *rv, const fc::CompactVol *cv,
                     int32_t *C, const fastcod_opts &o, hipStream_t st) {
    CountPlan cp;
    int rc = make_count_plan(S, N, M, cv, o, cu_count(dev), false, INT32_MAX, int64_t(256) << 20, cp);
    if (rc) return rc;
    CountScratch sc;
    if (cp.ovf_bytes) {
        FC_HIP(ws.ovf.ensure(cp.ovf_bytes, false));
        sc.ovf = ws.ovf.p;
    }
    if (cp.ct_bytes) {
        FC_HIP(ws.ct.ensure(cp.ct_bytes, false));
        sc.ct = static_cast<int32_t *>(ws.ct.p);
    }
    if (cp.ends_bytes) {
        FC_HIP(ws.ends.ensure(cp.ends_bytes, false));
        sc.ends = static_cast<int32_t *>(ws.ends.p);
    }
    if (cp.fb_bytes) {
        FC_HIP(ws.fallback.ensure(cp.fb_bytes, true));   // zeroed once; the fallback keeps it zero
        sc.fallback = static_cast<uint32_t *>(ws.fallback.p);
    }
    if (cp.first_bytes) {
        FC_HIP(ws.first.ensure(cp.first_bytes, false));
        sc.first = static_cast<int32_t *>(ws.first.p);
    }
    if (cp.pairs_bytes) {
        FC_HIP(ws.pairs.ensure(cp.pairs_bytes, false));
        sc.pairs = static_cast<char *>(ws.pairs.p);
    }
    return enqueue_count(cp, sc, dev, points, offsets, S, g, N, M, rv, cv, C, o, st);
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
    int blocks = 0;                             // workgroups of the pass-through launch (the schedule's)
    // Table entries are grouped by kind of subject (fc::BatchedKind): entries [kind_lo[k], kind_lo[k+1])
    // and their work items [item_lo[k], item_lo[k+1]) are counted by launch k
    int32_t kind_lo[fc::kBatchedKinds + 1] = {};
    int64_t item_lo[fc::kBatchedKinds + 1] = {};
    int kind_blocks[fc::kBatchedKinds] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Work-item split for a schedule: items in proportion to every subject's points (subjects of the
// seed-to-end kind take none: their kernel walks their streamlines directly).
int plan_items(fastcod_plan &pl, const PlanSched &ps, int cus, hipStream_t st) {
    int per_cu = fc::count_batched_blocks_per_cu(ps.batch, kBatchedCoarseWords);
    if (ps.blocks_per_cu > 0 && ps.blocks_per_cu < per_cu) per_cu = ps.blocks_per_cu;
    pl.blocks = cus * per_cu;
    for (int k = 0; k < fc::kBatchedKinds; ++k) {
        const int occ = fc::count_batched_blocks_per_cu(ps.batch, kBatchedCoarseWords, (fc::BatchedKind)k);
        pl.kind_blocks[k] = cus * std::max(1, std::min(per_cu, occ));
    }
    pl.kind_blocks[0] = pl.blocks;
    const int64_t total = (int64_t)pl.blocks * fc::kWavesPerBlock * ps.items_per_wave;
    double ptot = 0;
    for (int32_t k = 0; k < pl.n; ++k)
        if (k < pl.kind_lo[(int)fc::BatchedKind::kSeedEnd]) ptot += (double)pl.points[k];
    std::vector<int64_t> base(pl.n + 1, 0);
    for (int32_t k = 0; k < pl.n; ++k) {
        int64_t ni = 0;
        if (pl.subs[k].S > 0 && k < pl.kind_lo[(int)fc::BatchedKind::kSeedEnd]) {
            ni = ptot > 0 ? (int64_t)((double)total * (double)pl.points[k] / ptot + 0.5) : 1;
            if (ni < 1) ni = 1;
            if (ni > pl.subs[k].S) ni = pl.subs[k].S;
        }
        base[k + 1] = base[k] + ni;
    }
    pl.nitems = base[pl.n];
    for (int k = 0; k <= fc::kBatchedKinds; ++k) pl.item_lo[k] = base[pl.kind_lo[k]];
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
    // overflow count and every kind's work-item queues: zeroed by the partition launch (by a fill
    // when no subject has work items)
    const int64_t header_words = (int64_t)(fc::overflow_header_bytes(fc::kBatchedKinds) / 8);
    if (pl.nitems == 0) FC_HIP(fc::launch_fill_u64(pl.ovf.count, header_words, cus, st));
    const int32_t *kl = pl.kind_lo;
    const int ends = (int)fc::BatchedKind::kEnds, seed = (int)fc::BatchedKind::kSeedEnd;
    FC_HIP(fc::launch_end_labels_batched(subs, kl[ends], kl[ends + 1] - kl[ends], cus, st));
    if (pl.nitems > 0) {
        FC_HIP(fc::launch_partition_batched(subs, static_cast<const int64_t *>(pl.d_item_base.p), pl.n, pl.nitems,
                                            static_cast<int2 *>(pl.d_items.p), pl.ovf.count, header_words, cus, st));
        const int2 *items = static_cast<const int2 *>(pl.d_items.p);
        for (int k = 0; k < seed; ++k) {
            fc::Overflow o = pl.ovf;
            o.work = pl.ovf.count + fc::kQueueWords * (1 + (size_t)k * fc::kRangeQueues);
            FC_HIP(fc::launch_count_batched(subs, items + pl.item_lo[k], pl.item_lo[k + 1] - pl.item_lo[k], o,
                                            kBatchedCoarseWords, pl.kind_blocks[k], pl.sched.batch,
                                            (fc::BatchedKind)k, st));
        }
        FC_HIP(fc::launch_fallback_batched(subs, pl.n, pl.ovf, pl.fs, st));
    }
    FC_HIP(fc::launch_count_seed_end_batched(subs, kl[seed], kl[seed + 1] - kl[seed], cus, st));
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

// Options of subject u as counting options (upsample 0 means 1).
fastcod_opts subject_opts(const fastcod_subject &u) {
    fastcod_opts o = fastcod_default_opts();
    o.scale = u.scale;
    o.mode = u.mode;
    o.upsample = u.upsample == 0 ? 1 : u.upsample;
    return o;
}

int plan_check(const fastcod_subject *subjects, int32_t n) {
    for (int32_t k = 0; k < n; ++k) {
        const fastcod_subject &u = subjects[k];
        int rc = check_volume_args(u.roi_index_vol, u.target_label_vol, u.dims, u.N, u.M);
        if (rc) return fail(rc, "subject " + std::to_string(k) + ": " + last_error());
        rc = check_stream_args(u.points, u.offsets, u.n_streamlines, u.C_out, subject_opts(u));
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
    // table order: subjects grouped by kind (stable), so that each kind's launch takes a contiguous
    // range of entries and work items
    std::vector<int32_t> order(n);
    for (int32_t k = 0; k < n; ++k) order[k] = k;
    auto kind_of = [&](int32_t k) {
        const fastcod_opts o = subject_opts(subjects[k]);
        return (int)fc::batched_kind(o.mode, o.upsample);
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return kind_of(a) < kind_of(b); });
    for (int k = 0; k <= fc::kBatchedKinds; ++k) {
        int32_t c = 0;
        for (int32_t t = 0; t < n; ++t) c += kind_of(order[t]) < k ? 1 : 0;
        pl->kind_lo[k] = c;
    }
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
    size_t ends_words = 0;
    for (int32_t t = 0; t < n; ++t) {
        const int32_t k = order[t];
        const fastcod_subject &u = subjects[k];
        rc = check_volume_args(u.roi_index_vol, u.target_label_vol, u.dims, u.N, u.M);
        if (rc) return fail(rc, "subject " + std::to_string(k) + ": " + last_error());
        const fastcod_opts o = subject_opts(u);
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
        if (o.mode == FASTCOD_MODE_END || o.mode == FASTCOD_MODE_BOTH_ENDS) {
            ss.ends.mode = o.mode;   // label arrays placed below
            ends_words += (size_t)u.n_streamlines * (o.mode == FASTCOD_MODE_BOTH_ENDS ? 2 : 1);
        }
        ss.up = o.upsample;
        pl->subs.push_back(ss);
        pl->sizes.push_back((int64_t)u.N * u.M);
        total_s += u.n_streamlines;
        max_nw_n = std::max<int64_t>(max_nw_n, (u.N + 31) / 32);
        max_nw_m = std::max<int64_t>(max_nw_m, (u.M + 31) / 32);
        max_m = std::max<int64_t>(max_m, u.M);
    }
    // end labels of the endpoint-mode subjects: one plan-owned allocation, last[S] (and first[S]) each
    if (ends_words > 0) {
        void *buf = nullptr;
        hipError_t e = hipMalloc(&buf, 4 * ends_words);
        if (e != hipSuccess) return fail(FASTCOD_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        pl->volumes.push_back(buf);
        int32_t *p = static_cast<int32_t *>(buf);
        for (auto &ss : pl->subs) {
            if (ss.ends.mode == 0) continue;
            ss.ends.last = p;
            p += ss.S;
            if (ss.ends.mode == FASTCOD_MODE_BOTH_ENDS) {
                ss.ends.first = p;
                p += ss.S;
            }
        }
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
        for (int32_t t = 0; t < n; ++t) {
            const fastcod_subject &u = subjects[order[t]];
            if (pl->subs[t].S > 0 && u.M > 1 && u.N >= 64 && writers[u.C_out] == 1) {
                pick.push_back(t);
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
                const fastcod_subject &u = subjects[order[k]];
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
    const size_t header = fc::overflow_header_bytes(fc::kBatchedKinds);
    FC_HIP(pl->d_ovf.ensure(header + 8 * (size_t)std::max<int64_t>(total_s, 1), false));
    pl->ovf.count = static_cast<unsigned long long *>(pl->d_ovf.p);
    pl->ovf.work = pl->ovf.count + fc::kQueueWords;
    pl->ovf.list = reinterpret_cast<int64_t *>(static_cast<char *>(pl->d_ovf.p) + header);
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
    int kinds = 0;
    for (int k = 0; k < fc::kBatchedKinds; ++k) kinds |= (pl->kind_lo[k + 1] > pl->kind_lo[k] ? 1 : 0) << k;
    const std::string key = arch_name(dev) + ":cu" + std::to_string(cus) + ":n" + std::to_string(log2_bucket(n)) +
                            ":P" + std::to_string(log2_bucket(ptot)) + ":NM" + std::to_string(log2_bucket(nm / n)) +
                            ":T" + std::to_string(log2_bucket(spts > 0 ? ptot / spts : 0)) + ":K" + std::to_string(kinds);
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

// ---- fixed scratch area of fastcod_volume_count_noalloc ----
// One static device array (each device that loads the library holds its own copy until the process
// ends).  In host code `scratch` is only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is ever handed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(72) << 20;
constexpr int64_t kNoAllocMaxStreamlines = int64_t(1) << 21;
constexpr int64_t kNoAllocMaxPairs = int64_t(1) << 21;          // appended updates (the rest go to C as atomics)
constexpr int64_t kNoAllocFallbackBytes = int64_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;

// device address of `scratch` on dev (the current device)
int noalloc_scratch(int dev, char **out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return FASTCOD_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<char *>(p);
    *out = static_cast<char *>(p);
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
    WsRef ref(dev, st);
    Workspace &ws = *ref;
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
        return enqueue_count_ws(ws, dev, points, offsets, S, g, N, M, &rv, nullptr, C, o, st);
    }
    FC_HIP(ws.compact.ensure(L.bytes, false));
    fc::CompactVol cv = compact_view(ws.compact.p, L, N, M);
    FC_HIP(enqueue_compact_build(roi, lab, dims, N, M, L, ws.compact.p, cu_count(dev), st));
    return enqueue_count_ws(ws, dev, points, offsets, S, g, N, M, nullptr, &cv, C, o, st);
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
        WsRef ref(dev, st);
        std::lock_guard<std::mutex> lock(ref->mu);
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
    WsRef ref(dev, st);
    Workspace &ws = *ref;
    std::lock_guard<std::mutex> lock(ws.mu);
    FC_HIP(hipStreamWaitEvent(st, vol->ready, 0));
    const fc::Grid g = make_grid(vol->dims);
    fc::CompactVol cv = compact_view(vol->buf, vol->L, vol->N, vol->M);
    return enqueue_count_ws(ws, dev, points, offsets, S, g, vol->N, vol->M, nullptr, &cv, C, o, st);
}

int fastcod_volume_count_noalloc(const fastcod_volume *vol, const float *points, const int64_t *offsets, int64_t S,
                                 int32_t *C, const fastcod_opts *opts, void *stream) {
    last_error().clear();
    if (!vol) return fail(FASTCOD_EINVAL, "vol is NULL");
    const fastcod_opts o = opts ? *opts : fastcod_default_opts();
    int rc = check_stream_args(points, offsets, S, C, o);
    if (rc) return rc;
    if (o.variant == FASTCOD_VARIANT_WAVE) return fail(FASTCOD_EINVAL, "a resident volume has no raster form");
    if (o.flags & FASTCOD_VALIDATE) return fail(FASTCOD_EINVAL, "validate the source volumes before creating the handle");
    if (S > kNoAllocMaxStreamlines)
        return fail(FASTCOD_EINVAL, "fastcod_volume_count_noalloc counts at most 2^21 streamlines per call");
    int dev;
    rc = current_device(&dev);
    if (rc) return rc;
    if (dev != vol->device) return fail(FASTCOD_EINVAL, "volume lives on another device");
    char *base = nullptr;
    rc = noalloc_scratch(dev, &base);
    if (rc) return rc;
    const fc::CompactVol cv = compact_view(vol->buf, vol->L, vol->N, vol->M);
    CountPlan cp;
    rc = make_count_plan(S, vol->N, vol->M, &cv, o, cu_count(dev), true, kNoAllocMaxPairs, kNoAllocFallbackBytes, cp);
    if (rc) return rc;
    // carve the regions out of the fixed area; reject before anything is enqueued if they do not fit
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        if (!bytes) return nullptr;
        char *p = base + off;
        off = align256(off + bytes);
        return p;
    };
    CountScratch sc;
    sc.ovf = take(cp.ovf_bytes);
    sc.ct = reinterpret_cast<int32_t *>(take(cp.ct_bytes));
    sc.ends = reinterpret_cast<int32_t *>(take(cp.ends_bytes));
    sc.fallback = reinterpret_cast<uint32_t *>(take(cp.fb_bytes));
    sc.first = reinterpret_cast<int32_t *>(take(cp.first_bytes));
    sc.pairs = take(cp.pairs_bytes);
    if (off > kNoAllocScratchBytes)
        return fail(FASTCOD_ENOMEM, "this call needs " + std::to_string(off) + " bytes of scratch; the fixed area holds " +
                                        std::to_string(kNoAllocScratchBytes));
    hipStream_t st = static_cast<hipStream_t>(stream);
    FC_HIP(hipStreamWaitEvent(st, vol->ready, 0));
    // the fallback's bit maps must start all-zero; an earlier call may have left other contents there
    if (cp.fb_bytes) FC_HIP(fc::launch_fill_i32(reinterpret_cast<int32_t *>(sc.fallback), (int64_t)(cp.fb_bytes / 4), 0,
                                                cu_count(dev), st));
    const fc::Grid g = make_grid(vol->dims);
    return enqueue_count(cp, sc, dev, points, offsets, S, g, vol->N, vol->M, nullptr, &cv, C, o, st);
}

int fastcod_probe_stream(const float *points, int64_t P, uint32_t *sink, void *stream) {
    last_error().clear();
    if (P < 0 || P >= (int64_t(1) << 37)) return fail(FASTCOD_EINVAL, "n_points must be in [0, 2^37)");
    if ((P > 0 && !points) || !sink) return fail(FASTCOD_EINVAL, "NULL pointer");
    int dev;
    const int rc = current_device(&dev);
    if (rc) return rc;
    FC_HIP(fc::launch_probe_stream(points, P, cu_count(dev), sink, static_cast<hipStream_t>(stream)));
    return FASTCOD_OK;
}

int fastcod_probe_atomics(int32_t *target, int64_t n_words, const uint32_t *idx, int64_t n_idx, void *stream) {
    last_error().clear();
    if (n_words < 0 || n_idx < 0) return fail(FASTCOD_EINVAL, "sizes must be >= 0");
    if ((n_idx > 0 && !idx) || (n_words > 0 && !target)) return fail(FASTCOD_EINVAL, "NULL pointer");
    int dev;
    const int rc = current_device(&dev);
    if (rc) return rc;
    FC_HIP(fc::launch_probe_atomics(target, n_words, idx, n_idx, cu_count(dev), static_cast<hipStream_t>(stream)));
    return FASTCOD_OK;
}

int fastcod_probe_lookup(const fastcod_volume *vol, const float *points, int64_t P, float scale, uint32_t *sink,
                         void *stream) {
    last_error().clear();
    if (!vol || !sink || (P > 0 && !points)) return fail(FASTCOD_EINVAL, "NULL pointer");
    if (P < 0 || P >= (int64_t(1) << 37)) return fail(FASTCOD_EINVAL, "n_points must be in [0, 2^37)");
    if (!(scale == scale) || scale <= 0.0f || isinf(scale)) return fail(FASTCOD_EINVAL, "scale must be finite and > 0");
    int dev;
    const int rc = current_device(&dev);
    if (rc) return rc;
    if (dev != vol->device) return fail(FASTCOD_EINVAL, "volume lives on another device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    FC_HIP(hipStreamWaitEvent(st, vol->ready, 0));
    fc::StreamSubject sub{};
    sub.pts = points;
    sub.g = make_grid(vol->dims);
    sub.scale = scale;
    sub.cv = compact_view(vol->buf, vol->L, vol->N, vol->M);
    sub.up = 1;
    FC_HIP(fc::launch_probe_lookup(sub, P, cu_count(dev), sink, st));
    return FASTCOD_OK;
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
    WsRef ref(dev, st);
    Workspace &ws = *ref;
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
    bool busy = false;
    hipError_t err = hipSuccess;
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        Workspace *w = it->second;
        if (w->refs > 0) {   // a call is enqueueing with it right now
            busy = true;
            ++it;
            continue;
        }
        (void)hipSetDevice(it->first.dev);
        const hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess && err == hipSuccess) err = e;
        w->free_buffers();
        delete w;
        it = g_ws.erase(it);
    }
    (void)hipSetDevice(prev);
    if (busy) return fail(FASTCOD_EBUSY, "a workspace was in use by a call in progress; it was kept");
    if (err != hipSuccess) return hip_fail(err, "hipDeviceSynchronize");
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
