// Request server: the HIP executor of the scheduling core (server_core.h) and the
// fastcod_server_* entry points declared in include/fastcod.h.
//
// Device work runs on three streams owned by the server, all at the default priority:
//   compute  volume builds, request set-up (zero C, offsets upload), counting launches;
//   copy     uploads of host points (pieces of about chunk_points points);
//   out      result copies of C to host memory, each after an event of the compute stream.
// A counting launch ("tick") is the batched kernel over a descriptor table with one entry per
// active request: streamlines [s0, s1) of that request, its device arrays, volume, scale and C.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "fastcod.h"
#include "host.h"
#include "internal.h"
#include "server_core.h"

using namespace fch;

namespace {

constexpr int kTickSlots = 4;            // descriptor tables in rotation (> ticks in flight)
constexpr int kItemsPerWave = 4;         // work items per wavefront of a full launch
constexpr int64_t kMinItemPoints = 256;  // smaller launches get fewer, larger items

class HipExecutor final : public fcs::Executor {
  public:
    ~HipExecutor() override { teardown(); }

    int init(int dev, const fcs::Config &cfg) {
        dev_ = dev;
        cfg_ = cfg;
        cus_ = cu_count(dev);
        blocks_ = cus_ * fc::count_batched_blocks_per_cu(4, kBatchedCoarseWords);
        for (int k = 0; k < fc::kBatchedKinds; ++k)
            kind_blocks_[k] = cus_ * fc::count_batched_blocks_per_cu(4, kBatchedCoarseWords, (fc::BatchedKind)k);
        items_full_ = (int64_t)blocks_ * fc::kWavesPerBlock * kItemsPerWave;
        hipError_t e = hipMalloc(&base_, cfg.budget);
        if (e != hipSuccess) {
            base_ = nullptr;
            return fail(FASTCOD_ENOMEM, std::string("server budget allocation: ") + hipGetErrorString(e));
        }
        FC_HIP(hipStreamCreateWithFlags(&comp_, hipStreamNonBlocking));
        FC_HIP(hipStreamCreateWithFlags(&copy_, hipStreamNonBlocking));
        FC_HIP(hipStreamCreateWithFlags(&out_, hipStreamNonBlocking));
        const int64_t nsub = cfg.max_active;
        // the subject table and the item bases in one block (host and device alike): one upload a launch
        desc_base_off_ = (sizeof(fc::StreamSubject) * (size_t)nsub + 255) & ~size_t(255);
        const size_t desc_bytes = desc_base_off_ + 8 * (size_t)(nsub + 1);
        for (Slot &s : slots_) {
            FC_HIP(hipHostMalloc(reinterpret_cast<void **>(&s.h_desc), desc_bytes, hipHostMallocDefault));
            s.h_subs = reinterpret_cast<fc::StreamSubject *>(s.h_desc);
            s.h_base = reinterpret_cast<int64_t *>(s.h_desc + desc_base_off_);
            FC_HIP(s.d_desc.ensure(desc_bytes, false));
            FC_HIP(s.d_items.ensure(8 * (size_t)(items_full_ + nsub + 1), false));
            FC_HIP(hipEventCreateWithFlags(&s.last, hipEventDisableTiming));
            FC_HIP(hipEventRecord(s.last, comp_));
        }
        // offsets-check flags: one per request being set up, and at most max_active are
        const int nflags = 2 * cfg.max_active;
        FC_HIP(d_flags_.ensure(4 * (size_t)nflags, false));
        FC_HIP(hipHostMalloc(reinterpret_cast<void **>(&h_flags_), 4 * (size_t)nflags, hipHostMallocDefault));
        for (int k = nflags - 1; k >= 0; --k) free_flags_.push_back(k);
        const size_t header = fc::overflow_header_bytes(fc::kBatchedKinds);
        FC_HIP(d_ovf_.ensure(header + 8 * (size_t)cfg.tick_streamlines, false));
        ovf_.count = static_cast<unsigned long long *>(d_ovf_.p);
        ovf_.work = ovf_.count + fc::kQueueWords;
        ovf_.list = reinterpret_cast<int64_t *>(static_cast<char *>(d_ovf_.p) + header);
        ovf_.cap = cfg.tick_streamlines;
        return FASTCOD_OK;
    }

    std::string detail() const override { return err_; }

    int volume_bytes(const fcs::Volume &v, uint64_t *bytes, uint64_t *tmp_bytes) override {
        CompactLayout L;
        if (!compact_layout(v.dims, v.N, v.M, L, kBatchedCoarseWords))
            return err(FASTCOD_EINVAL, "grid too thin for the compact volume");
        // codes only for the occupied voxels, counted on the host copy with the build's own test
        int64_t occ = 0;
        for (int64_t i = 0; i < L.nvox; ++i)
            occ += (int)((uint32_t)v.roi[i] < (uint32_t)v.N) | (int)((uint32_t)v.lab[i] < (uint32_t)v.M);
        compact_layout_fit(L, occ);
        layouts_[v.id] = L;
        *bytes = L.bytes;
        *tmp_bytes = 2 * fcs::Arena::round(4 * (uint64_t)L.nvox);
        return FASTCOD_OK;
    }

    int build_volume(const fcs::Volume &v, fcs::Token *t) override {
        const CompactLayout &L = layouts_.at(v.id);
        char *roi = base_ + v.tmp_off;
        char *lab = roi + fcs::Arena::round(4 * (uint64_t)L.nvox);
        if (hip(hipMemcpyAsync(roi, v.roi.data(), 4 * (size_t)L.nvox, hipMemcpyHostToDevice, comp_), "volume upload") ||
            hip(hipMemcpyAsync(lab, v.lab.data(), 4 * (size_t)L.nvox, hipMemcpyHostToDevice, comp_), "volume upload") ||
            hip(enqueue_compact_build(reinterpret_cast<const int32_t *>(roi), reinterpret_cast<const int32_t *>(lab),
                                      v.dims, v.N, v.M, L, base_ + v.off, cus_, comp_),
                "compact build"))
            return FASTCOD_EHIP;
        return record(comp_, t);
    }

    int after_stream(void *stream, fcs::Token *t) override {
        TokenRec *rec = nullptr;
        if (int rc = take(&rec, t)) return rc;
        if (hip(hipEventRecord(rec->ev, static_cast<hipStream_t>(stream)), "hipEventRecord on the request's stream")) {
            release(*t);
            *t = 0;
            return FASTCOD_EHIP;
        }
        return FASTCOD_OK;
    }

    // On the copy stream: the offsets (8 MB for a million streamlines) cross PCIe while the compute
    // stream keeps counting the requests before this one; the core counts this request only once
    // the token has completed.
    // The offsets are checked on the device copy (nondecreasing); the flag comes back to a pinned
    // slot that setup_status reads once the token has completed.
    int begin_request(const fcs::Request &r, fcs::Token *t) override {
        if (r.ready && (r.ready > toks_.size() ||
                        hip(hipStreamWaitEvent(copy_, toks_[r.ready - 1].ev, 0), "hipStreamWaitEvent")))
            return r.ready > toks_.size() ? err(FASTCOD_EINVAL, "unknown token") : FASTCOD_EHIP;
        if (free_flags_.empty()) return err(FASTCOD_EBUSY, "no free set-up flag");
        const int slot = free_flags_.back();
        const auto *d_off = reinterpret_cast<const int64_t *>(base_ + r.off_offsets);
        int32_t *d_flag = static_cast<int32_t *>(d_flags_.p) + slot;
        if (hip(fc::launch_fill_i32(device_C(r), (int64_t)r.N * r.M, 0, cus_, copy_), "zero fill") ||
            hip(hipMemcpyAsync(base_ + r.off_offsets, r.offsets, 8 * (size_t)(r.S + 1), hipMemcpyHostToDevice, copy_),
                "offsets upload") ||
            hip(fc::launch_validate(d_off, r.S, nullptr, nullptr, 0, 1, 1, d_flag, cus_, copy_), "offsets check") ||
            hip(hipMemcpyAsync(h_flags_ + slot, d_flag, 4, hipMemcpyDeviceToHost, copy_), "offsets check"))
            return FASTCOD_EHIP;
        free_flags_.pop_back();
        flag_of_[r.id] = slot;
        return record(copy_, t);
    }
    int setup_status(const fcs::Request &r) override {
        auto it = flag_of_.find(r.id);
        if (it == flag_of_.end()) return FASTCOD_OK;
        const int32_t f = h_flags_[it->second];
        free_flags_.push_back(it->second);
        flag_of_.erase(it);
        return f ? FASTCOD_ERANGE : FASTCOD_OK;
    }

    int upload(const fcs::Request &r, int64_t s0, int64_t s1, fcs::Token *t) override {
        // (clamped to [0, P]: the offsets may not have been checked yet)
        const int64_t p0 = std::min<int64_t>(std::max<int64_t>(r.offsets[s0], 0), r.P);
        const int64_t p1 = std::min<int64_t>(std::max<int64_t>(r.offsets[s1], p0), r.P);
        if (p1 > p0 && hip(hipMemcpyAsync(base_ + r.off_points + 12 * p0, r.points + 3 * p0, 12 * (size_t)(p1 - p0),
                                          hipMemcpyHostToDevice, copy_),
                           "points upload"))
            return FASTCOD_EHIP;
        return record(copy_, t);
    }

    int launch_tick(const std::vector<fcs::Chunk> &chunks_in, fcs::Token *t) override {
        const int32_t n = (int32_t)chunks_in.size();
        if (n < 1 || n > cfg_.max_active) return err(FASTCOD_EINVAL, "launch of an unexpected size");
        Slot &s = slots_[next_slot_++ % kTickSlots];
        if (hip(hipEventSynchronize(s.last), "descriptor slot")) return FASTCOD_EHIP;
        // table entries grouped by kind of request (each kind has a launch of its own)
        auto kind_of = [](const fcs::Chunk &c) { return (int)fc::batched_kind(c.req->mode, c.req->up); };
        std::vector<fcs::Chunk> chunks(chunks_in);
        std::stable_sort(chunks.begin(), chunks.end(),
                         [&](const fcs::Chunk &a, const fcs::Chunk &b) { return kind_of(a) < kind_of(b); });
        int32_t kind_lo[fc::kBatchedKinds + 1];
        for (int k = 0; k <= fc::kBatchedKinds; ++k) {
            kind_lo[k] = 0;
            for (const fcs::Chunk &c : chunks) kind_lo[k] += kind_of(c) < k ? 1 : 0;
        }
        const int seed = (int)fc::BatchedKind::kSeedEnd, ends = (int)fc::BatchedKind::kEnds;
        // fallback scratch for the largest volume of this launch
        int32_t maxN = 1, maxM = 1;
        for (const fcs::Chunk &c : chunks) {
            maxN = std::max(maxN, c.vol->N);
            maxM = std::max(maxM, c.vol->M);
        }
        if (int rc = ensure_fallback(maxN, maxM)) return rc;
        int64_t total = 0;
        for (int32_t k = 0; k < kind_lo[seed]; ++k) total += chunks[k].req->offsets[chunks[k].s1] - chunks[k].req->offsets[chunks[k].s0];
        const int64_t want = std::max<int64_t>(1, std::min<int64_t>(items_full_, total / kMinItemPoints));
        s.h_base[0] = 0;
        for (int32_t k = 0; k < n; ++k) {
            const fcs::Chunk &c = chunks[k];
            const fcs::Request &r = *c.req;
            const fcs::Volume &v = *c.vol;
            fc::StreamSubject &ss = s.h_subs[k];
            ss.pts = (r.flags & FASTCOD_REQ_DEVICE_POINTS) ? r.points
                                                           : reinterpret_cast<const float *>(base_ + r.off_points);
            ss.offsets = reinterpret_cast<const int64_t *>(base_ + r.off_offsets);
            ss.S = c.s1;
            ss.s_begin = c.s0;
            ss.g = make_grid(v.dims);
            ss.scale = r.scale;
            ss.cv = compact_view(base_ + v.off, layouts_.at(v.id), v.N, v.M);
            ss.C = device_C(r);
            ss.si = (uint32_t)v.M;
            ss.sm = 1u;
            ss.ends = fc::EndLabels{0, nullptr, nullptr};
            if (r.mode == FASTCOD_MODE_END || r.mode == FASTCOD_MODE_BOTH_ENDS) {
                int32_t *last = reinterpret_cast<int32_t *>(base_ + r.off_ends);
                ss.ends = fc::EndLabels{r.mode, last, r.mode == FASTCOD_MODE_BOTH_ENDS ? last + r.S : nullptr};
            }
            ss.up = r.up;
            int64_t ni = 0;
            if (k < kind_lo[seed]) {   // the seed-to-end kind takes no work items
                const int64_t pts = r.offsets[c.s1] - r.offsets[c.s0];
                ni = total > 0 ? (int64_t)((double)want * (double)pts / (double)total + 0.5) : 1;
                ni = std::max<int64_t>(1, std::min<int64_t>(ni, c.s1 - c.s0));
            }
            s.h_base[k + 1] = s.h_base[k] + ni;
        }
        const int64_t nitems = s.h_base[n];
        if (nitems + 1 > (int64_t)(s.d_items.n / 8)) return err(FASTCOD_EINVAL, "work item table overflow");
        const auto *subs = static_cast<const fc::StreamSubject *>(s.d_desc.p);
        const auto *d_base = reinterpret_cast<const int64_t *>(static_cast<const char *>(s.d_desc.p) + desc_base_off_);
        const int2 *items = static_cast<const int2 *>(s.d_items.p);
        // the counters and range queues are reset by the partition launch (by a fill without items)
        const int64_t header_words = (int64_t)(fc::overflow_header_bytes(fc::kBatchedKinds) / 8);
        if (hip(hipMemcpyAsync(s.d_desc.p, s.h_desc, desc_base_off_ + 8 * (size_t)(n + 1), hipMemcpyHostToDevice, comp_),
                "descriptor upload") ||
            (nitems == 0 && hip(fc::launch_fill_u64(ovf_.count, header_words, cus_, comp_), "counter reset")) ||
            hip(fc::launch_end_labels_batched(subs, kind_lo[ends], kind_lo[ends + 1] - kind_lo[ends], cus_, comp_),
                "end labels"))
            return FASTCOD_EHIP;
        if (nitems > 0) {
            if (hip(fc::launch_partition_batched(subs, d_base, n, nitems, static_cast<int2 *>(s.d_items.p), ovf_.count,
                                                 header_words, cus_, comp_),
                    "partition"))
                return FASTCOD_EHIP;
            for (int k = 0; k < seed; ++k) {
                const int64_t lo = s.h_base[kind_lo[k]], hi = s.h_base[kind_lo[k + 1]];
                fc::Overflow o = ovf_;
                o.work = ovf_.count + fc::kQueueWords * (1 + (size_t)k * fc::kRangeQueues);
                if (hip(fc::launch_count_batched(subs, items + lo, hi - lo, o, kBatchedCoarseWords, kind_blocks_[k], 4,
                                                 (fc::BatchedKind)k, comp_),
                        "count"))
                    return FASTCOD_EHIP;
            }
            if (hip(fc::launch_fallback_batched(subs, n, ovf_, fs_, comp_), "fallback")) return FASTCOD_EHIP;
        }
        if (hip(fc::launch_count_seed_end_batched(subs, kind_lo[seed], kind_lo[seed + 1] - kind_lo[seed], cus_, comp_),
                "seed-to-end count") ||
            hip(hipEventRecord(s.last, comp_), "hipEventRecord"))
            return FASTCOD_EHIP;
        return record(comp_, t);
    }

    int finalize(const fcs::Request &r, fcs::Token *t) override {
        if (r.flags & FASTCOD_REQ_DEVICE_C) return record(comp_, t);
        TokenRec *rec = nullptr;
        if (int rc = take(&rec, t)) return rc;
        if (hip(hipEventRecord(rec->link, comp_), "hipEventRecord") ||
            hip(hipStreamWaitEvent(out_, rec->link, 0), "hipStreamWaitEvent") ||
            hip(hipMemcpyAsync(r.C_out, base_ + r.off_C, 4 * (size_t)r.N * r.M, hipMemcpyDeviceToHost, out_),
                "result copy") ||
            hip(hipEventRecord(rec->ev, out_), "hipEventRecord"))
            return FASTCOD_EHIP;
        return FASTCOD_OK;
    }

    int query(fcs::Token t) override {
        if (t == 0 || t > toks_.size()) return err(FASTCOD_EINVAL, "unknown token");
        const hipError_t e = hipEventQuery(toks_[t - 1].ev);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        return err(FASTCOD_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
    }

    void release(fcs::Token t) override {
        if (t >= 1 && t <= toks_.size()) free_toks_.push_back(t);
    }

    void pause() override { std::this_thread::sleep_for(std::chrono::microseconds(10)); }

  private:
    struct TokenRec {
        hipEvent_t ev = nullptr, link = nullptr;
    };
    struct Slot {
        char *h_desc = nullptr;                 // pinned: subject table, then (at desc_base_off_) item bases
        fc::StreamSubject *h_subs = nullptr;
        int64_t *h_base = nullptr;
        DevBuf d_desc, d_items;                 // d_desc: the same layout as h_desc
        hipEvent_t last = nullptr;
    };

    int err(int rc, const std::string &m) {
        err_ = m;
        return rc;
    }
    // true on failure
    bool hip(hipError_t e, const char *what) {
        if (e == hipSuccess) return false;
        err_ = std::string(what) + ": " + hipGetErrorString(e);
        return true;
    }

    int32_t *device_C(const fcs::Request &r) const {
        return (r.flags & FASTCOD_REQ_DEVICE_C) ? r.C_out : reinterpret_cast<int32_t *>(base_ + r.off_C);
    }

    int take(TokenRec **rec, fcs::Token *t) {
        if (free_toks_.empty()) {
            TokenRec tr;
            if (hip(hipEventCreateWithFlags(&tr.ev, hipEventDisableTiming), "hipEventCreate") ||
                hip(hipEventCreateWithFlags(&tr.link, hipEventDisableTiming), "hipEventCreate"))
                return FASTCOD_EHIP;
            toks_.push_back(tr);
            free_toks_.push_back(toks_.size());
        }
        *t = free_toks_.back();
        free_toks_.pop_back();
        *rec = &toks_[*t - 1];
        return FASTCOD_OK;
    }

    int record(hipStream_t st, fcs::Token *t) {
        TokenRec *rec = nullptr;
        if (int rc = take(&rec, t)) return rc;
        if (hip(hipEventRecord(rec->ev, st), "hipEventRecord")) return FASTCOD_EHIP;
        return FASTCOD_OK;
    }

    int ensure_fallback(int32_t N, int32_t M) {
        if (N <= fbN_ && M <= fbM_) return FASTCOD_OK;
        fbN_ = std::max(fbN_, N);
        fbM_ = std::max(fbM_, M);
        fs_.nwordsN = (fbN_ + 31) / 32;
        fs_.nwordsM = (fbM_ + 31) / 32;
        fs_.stride = ((int64_t)fs_.nwordsN + fs_.nwordsM + fbM_ + 63) & ~int64_t(63);
        int64_t blocks = (int64_t(64) << 20) / (4 * fs_.stride);   // <= 64 MiB of scratch
        fs_.blocks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, blocks));
        // earlier launches may still read the old scratch: the growth waits for the device
        if (hip(hipDeviceSynchronize(), "hipDeviceSynchronize") ||
            hip(d_fb_.ensure((size_t)(4 * fs_.stride * fs_.blocks), true), "fallback scratch"))
            return FASTCOD_EHIP;
        fs_.words = static_cast<uint32_t *>(d_fb_.p);
        return FASTCOD_OK;
    }

    void teardown() {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(dev_);
        for (hipStream_t st : {comp_, copy_, out_})
            if (st) (void)hipStreamSynchronize(st);
        for (TokenRec &tr : toks_) {
            if (tr.ev) (void)hipEventDestroy(tr.ev);
            if (tr.link) (void)hipEventDestroy(tr.link);
        }
        toks_.clear();
        for (Slot &s : slots_) {
            if (s.h_desc) (void)hipHostFree(s.h_desc);
            if (s.last) (void)hipEventDestroy(s.last);
            s.h_desc = nullptr;
            s.h_subs = nullptr;
            s.h_base = nullptr;
            s.last = nullptr;
            s.d_desc.release();
            s.d_items.release();
        }
        d_ovf_.release();
        d_fb_.release();
        d_flags_.release();
        if (h_flags_) (void)hipHostFree(h_flags_);
        h_flags_ = nullptr;
        free_flags_.clear();
        flag_of_.clear();
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
        for (hipStream_t *st : {&comp_, &copy_, &out_})
            if (*st) {
                (void)hipStreamDestroy(*st);
                *st = nullptr;
            }
        (void)hipSetDevice(prev);
    }

    int dev_ = 0, cus_ = 256, blocks_ = 256;
    int kind_blocks_[fc::kBatchedKinds] = {};
    int64_t items_full_ = 0;
    fcs::Config cfg_;
    char *base_ = nullptr;
    hipStream_t comp_ = nullptr, copy_ = nullptr, out_ = nullptr;
    Slot slots_[kTickSlots];
    DevBuf d_flags_;                      // offsets-check flags of requests being set up
    int32_t *h_flags_ = nullptr;          // (pinned mirror)
    std::vector<int> free_flags_;
    std::map<uint64_t, int> flag_of_;     // request id -> flag slot
    size_t desc_base_off_ = 0;   // offset of the item bases in a slot's descriptor block
    uint64_t next_slot_ = 0;
    std::vector<TokenRec> toks_;
    std::vector<fcs::Token> free_toks_;
    std::map<int32_t, CompactLayout> layouts_;
    DevBuf d_ovf_, d_fb_;
    fc::Overflow ovf_{};
    fc::FallbackScratch fs_{};
    int32_t fbN_ = 0, fbM_ = 0;
    std::string err_;
};

}  // namespace

struct fastcod_server {
    int device = 0;
    std::unique_ptr<fcs::Service> svc;
};

extern "C" {

int fastcod_server_create(const fastcod_server_config *cfg_in, fastcod_server **out) {
    last_error().clear();
    if (!out) return fail(FASTCOD_EINVAL, "out is NULL");
    *out = nullptr;
    fastcod_server_config c{};
    if (cfg_in) c = *cfg_in;
    if (c.tick_points < 0 || c.chunk_points < 0 || c.max_active < 0 || c.max_active > 1024 || c.reserved != 0)
        return fail(FASTCOD_EINVAL, "bad server configuration");
    int dev;
    int rc = current_device(&dev);
    if (rc) return rc;
    fcs::Config cfg;
    cfg.budget = c.memory_budget;
    if (cfg.budget == 0) {
        size_t fr = 0, tot = 0;
        FC_HIP(hipMemGetInfo(&fr, &tot));
        cfg.budget = (uint64_t)((double)fr * 0.8);
    }
    cfg.budget &= ~uint64_t(255);
    if (cfg.budget < (1u << 20)) return fail(FASTCOD_EINVAL, "memory_budget must be at least 1 MiB");
    if (c.tick_points) cfg.tick_points = c.tick_points;
    if (c.chunk_points) cfg.chunk_points = c.chunk_points;
    if (c.max_active) cfg.max_active = c.max_active;
    auto ex = std::make_unique<HipExecutor>();
    rc = ex->init(dev, cfg);
    if (rc) return rc;   // ex's destructor frees what init took
    fastcod_server *s = new fastcod_server();
    s->device = dev;
    s->svc = std::make_unique<fcs::Service>(cfg, std::move(ex), [dev]() { (void)hipSetDevice(dev); });
    *out = s;
    return FASTCOD_OK;
}

int fastcod_server_add_volume(fastcod_server *srv, const int32_t *roi, const int32_t *lab, const int32_t dims[3],
                              int32_t N, int32_t M, int32_t *volume_id) {
    last_error().clear();
    if (!srv || !volume_id) return fail(FASTCOD_EINVAL, "NULL argument");
    int rc = check_volume_args(roi, lab, dims, N, M);
    if (rc) return rc;
    std::string msg;
    rc = srv->svc->add_volume(roi, lab, dims, N, M, volume_id, &msg);
    return rc ? fail(rc, msg) : FASTCOD_OK;
}

int fastcod_server_submit(fastcod_server *srv, const fastcod_request *req, uint64_t *request_id) {
    last_error().clear();
    if (!srv || !req || !request_id) return fail(FASTCOD_EINVAL, "NULL argument");
    std::string msg;
    const int rc = srv->svc->submit(*req, request_id, &msg);
    return rc ? fail(rc, msg) : FASTCOD_OK;
}

int fastcod_server_wait(fastcod_server *srv, uint64_t request_id, int64_t timeout_us, fastcod_request_info *info) {
    last_error().clear();
    if (!srv) return fail(FASTCOD_EINVAL, "srv is NULL");
    const int rc = srv->svc->wait(request_id, timeout_us, info);
    if (rc == FASTCOD_EINVAL) return fail(rc, "unknown request id");
    if (rc != FASTCOD_OK && rc != FASTCOD_ETIMEDOUT && rc != FASTCOD_ECANCELED)
        return fail(rc, srv->svc->locked([](fcs::Core &c) { return c.fail_message(); }));
    return rc;
}

int fastcod_server_cancel(fastcod_server *srv, uint64_t request_id) {
    last_error().clear();
    if (!srv) return fail(FASTCOD_EINVAL, "srv is NULL");
    const int rc = srv->svc->cancel(request_id);
    return rc ? fail(rc, "unknown or finished request id") : FASTCOD_OK;
}

int fastcod_server_get_stats(fastcod_server *srv, fastcod_server_stats *out) {
    last_error().clear();
    if (!srv || !out) return fail(FASTCOD_EINVAL, "NULL argument");
    srv->svc->locked([out](fcs::Core &c) {
        memset(out, 0, sizeof(*out));
        out->budget_bytes = c.arena().size();
        out->used_bytes = c.arena().used();
        out->pending = (int64_t)c.pending_count();
        out->active = (int64_t)c.active_count();
        out->completed = (int64_t)c.completed();
        out->launches = (int64_t)c.ticks_launched();
        out->volume_builds = (int64_t)c.volume_builds();
        out->evictions = (int64_t)c.evictions();
        out->failed = c.failed();
        return 0;
    });
    return FASTCOD_OK;
}

int fastcod_server_destroy(fastcod_server *srv) {
    last_error().clear();
    if (!srv) return FASTCOD_OK;
    srv->svc->shutdown();
    srv->svc.reset();   // frees the executor's device memory, streams and events
    delete srv;
    return FASTCOD_OK;
}

}  // extern "C"
