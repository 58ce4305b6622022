// Scheduling core of the request server (host-only C++; no HIP types).
//
// Requests name a resident volume pair and bring streamlines (points on the host or the device,
// offsets on the host) and a C destination.  The core decides, step by step:
//   - admission: strictly first come, first served, when the request's device bytes (offsets,
//     host points, the device copy of C) plus its volume's compact form and build scratch, if that
//     volume is not resident, fit into an arena of fixed size; idle volumes are evicted least
//     recently used first to make room;
//   - uploads of host points in pieces of about chunk_points points, a bounded number in flight;
//   - continuous batching: every counting launch ("tick") takes the next ready streamline range of
//     every active request, so a new request joins the very next launch instead of waiting for the
//     ones before it.  Each request gets at least chunk_points points of a tick (an equal part of it
//     when that is less); the rest of tick_points goes to the oldest requests first, so that they
//     finish, and their results leave over PCIe, while the others are still counting;
//   - finalisation (C to its destination) once every streamline of a request has been counted,
//     completion, cancellation and failure.
// Each count of a streamline range adds exact integers into the request's C, so C does not
// depend on how the request was cut or interleaved (Section 2: C is a sum over streamlines).
//
// Every device operation is asynchronous and goes through Executor, which hands back a token
// that the core polls; the library implements Executor with HIP streams and events, host tests
// with a simulated executor.  The core is not thread-safe: Service wraps it with a mutex and a
// scheduler thread.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fastcod.h"

namespace fcs {

inline int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ---------------------------------------------------------------------------------------------
// Arena: offsets into one device allocation of fixed size, best fit, neighbours coalesced.
// ---------------------------------------------------------------------------------------------
class Arena {
  public:
    static constexpr uint64_t kAlign = 256;
    static uint64_t round(uint64_t b) { return ((b ? b : 1) + kAlign - 1) & ~(kAlign - 1); }

    void reset(uint64_t size) {
        free_.clear();
        live_.clear();
        size_ = size & ~(kAlign - 1);
        used_ = 0;
        if (size_) free_[0] = size_;
    }
    // offset of `bytes` (rounded up to 256) or -1
    int64_t alloc(uint64_t bytes) {
        bytes = round(bytes);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return -1;
        const uint64_t off = best->first, sz = best->second;
        free_.erase(best);
        if (sz > bytes) free_[off + bytes] = sz - bytes;
        live_[off] = bytes;
        used_ += bytes;
        return (int64_t)off;
    }
    void release(int64_t off) {
        if (off < 0) return;
        auto it = live_.find((uint64_t)off);
        if (it == live_.end()) return;
        uint64_t o = it->first, sz = it->second;
        live_.erase(it);
        used_ -= sz;
        auto nx = free_.lower_bound(o);
        if (nx != free_.end() && o + sz == nx->first) {
            sz += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == o) {
                pv->second += sz;
                return;
            }
        }
        free_[o] = sz;
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t largest_free() const {
        uint64_t m = 0;
        for (const auto &f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t live_blocks() const { return live_.size(); }
    size_t free_blocks() const { return free_.size(); }

  private:
    std::map<uint64_t, uint64_t> free_, live_;   // offset -> size
    uint64_t size_ = 0, used_ = 0;
};

// ---------------------------------------------------------------------------------------------
// records
// ---------------------------------------------------------------------------------------------
using Token = uint64_t;   // 0 = none

struct Config {
    uint64_t budget = 0;              // arena bytes
    // points per counting launch, over all requests: each launch has a fixed cost (partition,
    // fallback, histogram and completion work), so a busy server gains from long ones (2^27: about
    // twice the requests per second of 2^25 on a mixed stream); a lone request's launch holds only
    // its own points either way
    int64_t tick_points = int64_t(1) << 27;
    int64_t tick_streamlines = 1 << 20;
    int64_t chunk_points = 1 << 20;   // points per host upload piece, and the smallest share of a tick
    int32_t max_active = 64;          // admitted requests still counting, at most
    int32_t upload_window = 8;        // upload pieces in flight
    int32_t ticks_in_flight = 2;      // counting launches queued on the device at once
};

struct Volume {
    int32_t id = -1;
    int32_t dims[3] = {0, 0, 0};
    int32_t N = 0, M = 0;
    std::vector<int32_t> roi, lab;    // host copies, [Z][Y][X]
    uint64_t bytes = 0, tmp_bytes = 0;
    int64_t off = -1, tmp_off = -1;   // arena offsets (resident / build scratch)
    Token build = 0;
    int users = 0;                    // admitted requests using it
    uint64_t last_use = 0;
    uint64_t builds = 0;              // times it was built (evictions show as rebuilds)
};

enum class State { Pending, Active, Finalizing, Done };

struct Request {
    uint64_t id = 0;
    int32_t vol = -1;
    uint32_t flags = 0;
    const float *points = nullptr;
    const int64_t *offsets = nullptr;   // host
    int64_t S = 0, P = 0;
    float scale = 1.0f;
    int32_t mode = FASTCOD_MODE_PASSTHROUGH;
    int32_t up = 1;                     // upsampling factor
    int32_t *C_out = nullptr;
    int32_t N = 0, M = 0;
    State state = State::Pending;
    int status = FASTCOD_OK;
    bool cancel = false;
    int cancel_status = FASTCOD_ECANCELED;          // FASTCOD_ERANGE: offsets found decreasing at set-up
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    int64_t off_C = -1, off_offsets = -1, off_points = -1;
    int64_t off_ends = -1;                           // end labels (endpoint modes): last[S] (and first[S])
    int64_t issued_s = 0, ready_s = 0, next_s = 0;
    std::deque<std::pair<Token, int64_t>> uploads;   // (token, streamline end) in issue order
    Token ready = 0;                                 // FASTCOD_REQ_AFTER_STREAM: the caller's stream at submission
    Token begin = 0, final = 0;
    uint64_t last_tick = 0;                          // sequence number of the latest tick using it
    int64_t chunks = 0, ticks = 0;
};

struct Chunk {
    const Request *req;
    const Volume *vol;
    int64_t s0, s1;
};

// Device side of the core.  Every call is asynchronous; a nonzero return is a FASTCOD_* error
// and fails the server.
class Executor {
  public:
    virtual ~Executor() {}
    // device bytes of a volume's compact form and of the scratch its build needs (the host copies
    // of the volume are already in v)
    virtual int volume_bytes(const Volume &v, uint64_t *bytes, uint64_t *tmp_bytes) = 0;
    virtual int build_volume(const Volume &v, Token *t) = 0;
    // a marker of the work enqueued so far on a caller's stream (submission time); begin_request
    // orders the request's device work after r.ready
    virtual int after_stream(void *stream, Token *t) {
        (void)stream;
        *t = 0;
        return FASTCOD_OK;
    }
    // zero the request's C, upload its offsets and check them (after r.ready); the request joins
    // ticks only once the token has completed and setup_status has accepted it
    virtual int begin_request(const Request &r, Token *t) = 0;
    // once the set-up token has completed: FASTCOD_OK, or FASTCOD_ERANGE if the offsets decrease
    virtual int setup_status(const Request &r) {
        (void)r;
        return FASTCOD_OK;
    }
    // host points of streamlines [s0, s1) to the request's device copy
    virtual int upload(const Request &r, int64_t s0, int64_t s1, Token *t) = 0;
    // count every chunk (ordered after begin_request and the volume build)
    virtual int launch_tick(const std::vector<Chunk> &chunks, Token *t) = 0;
    // C to its destination, after every tick that used the request
    virtual int finalize(const Request &r, Token *t) = 0;
    // 1 done, 0 not yet, < 0 error
    virtual int query(Token t) = 0;
    virtual void release(Token t) = 0;
    // a short pause while device work is in flight
    virtual void pause() = 0;
    // detail of the last failed operation
    virtual std::string detail() const { return std::string(); }
};

// ---------------------------------------------------------------------------------------------
// Core
// ---------------------------------------------------------------------------------------------
class Core {
  public:
    Core(const Config &cfg, Executor *ex) : cfg_(cfg), ex_(ex) {
        if (cfg_.tick_points < 1) cfg_.tick_points = 1;
        if (cfg_.tick_streamlines < 1) cfg_.tick_streamlines = 1;
        if (cfg_.chunk_points < 1) cfg_.chunk_points = 1;
        if (cfg_.max_active < 1) cfg_.max_active = 1;
        if (cfg_.upload_window < 1) cfg_.upload_window = 1;
        if (cfg_.ticks_in_flight < 1) cfg_.ticks_in_flight = 1;
        arena_.reset(cfg_.budget);
    }

    const Config &config() const { return cfg_; }
    const Arena &arena() const { return arena_; }
    int failed() const { return failed_; }
    const std::string &fail_message() const { return fail_msg_; }

    // Registers a volume pair (host copies taken); it becomes resident when a request needs it.
    int add_volume(const int32_t *roi, const int32_t *lab, const int32_t dims[3], int32_t N, int32_t M,
                   int32_t *id, std::string *err) {
        if (failed_) return set_err(err, failed_, fail_msg_);
        auto v = std::make_unique<Volume>();
        v->id = (int32_t)vols_.size();
        for (int k = 0; k < 3; ++k) v->dims[k] = dims[k];
        v->N = N;
        v->M = M;
        const size_t n = (size_t)dims[0] * dims[1] * dims[2];
        if (roi) v->roi.assign(roi, roi + n);
        if (lab) v->lab.assign(lab, lab + n);
        int rc = ex_->volume_bytes(*v, &v->bytes, &v->tmp_bytes);
        if (rc) return set_err(err, rc, "volume rejected by the executor");
        if (Arena::round(v->bytes) + Arena::round(v->tmp_bytes) > arena_.size())
            return set_err(err, FASTCOD_ENOMEM, "volume does not fit the server's memory budget");
        *id = v->id;
        vols_.push_back(std::move(v));
        return FASTCOD_OK;
    }
    const Volume *volume(int32_t id) const {
        return (id >= 0 && id < (int32_t)vols_.size()) ? vols_[id].get() : nullptr;
    }
    int32_t volume_count() const { return (int32_t)vols_.size(); }

    // end labels a request keeps on the device (endpoint modes)
    static uint64_t ends_bytes(int64_t S, int32_t mode) {
        if (mode == FASTCOD_MODE_END) return 4 * (uint64_t)S;
        if (mode == FASTCOD_MODE_BOTH_ENDS) return 8 * (uint64_t)S;
        return 0;
    }
    // Device bytes a request holds while admitted (volume excluded).
    static uint64_t request_bytes(int64_t S, int64_t P, int32_t N, int32_t M, uint32_t flags, int32_t mode = 0) {
        uint64_t b = Arena::round(8 * (uint64_t)(S + 1));
        if (!(flags & FASTCOD_REQ_DEVICE_POINTS)) b += Arena::round(12 * (uint64_t)P);
        if (!(flags & FASTCOD_REQ_DEVICE_C)) b += Arena::round(4 * (uint64_t)N * (uint64_t)M);
        if (ends_bytes(S, mode)) b += Arena::round(ends_bytes(S, mode));
        return b;
    }

    int submit(const fastcod_request &q, uint64_t *id, std::string *err) {
        if (failed_) return set_err(err, failed_, fail_msg_);
        if (stopping_) return set_err(err, FASTCOD_EBUSY, "server is shutting down");
        const Volume *v = volume(q.volume_id);
        if (!v) return set_err(err, FASTCOD_EINVAL, "unknown volume id");
        if (q.n_streamlines < 0 || q.n_streamlines > INT32_MAX)
            return set_err(err, FASTCOD_EINVAL, "n_streamlines must be in [0, INT32_MAX]");
        if (!q.offsets) return set_err(err, FASTCOD_EINVAL, "offsets is NULL");
        if (!q.C_out) return set_err(err, FASTCOD_EINVAL, "C_out is NULL");
        if (q.flags & ~(uint32_t)(FASTCOD_REQ_DEVICE_POINTS | FASTCOD_REQ_DEVICE_C | FASTCOD_REQ_AFTER_STREAM))
            return set_err(err, FASTCOD_EINVAL, "unknown request flag");
        if (!(q.scale == q.scale) || q.scale <= 0.0f || q.scale > 3.4e38f)
            return set_err(err, FASTCOD_EINVAL, "scale must be finite and > 0");
        if (q.mode < FASTCOD_MODE_PASSTHROUGH || q.mode > FASTCOD_MODE_SEED_END)
            return set_err(err, FASTCOD_EINVAL, "unknown mode");
        const int32_t up = q.upsample == 0 ? 1 : q.upsample;
        if (up < 1 || up > 4) return set_err(err, FASTCOD_EINVAL, "upsample must be 0..4");
        if (up > 1 && q.mode != FASTCOD_MODE_PASSTHROUGH)
            return set_err(err, FASTCOD_EINVAL, "upsampling is available for the pass-through mode only");
        // offsets (host): the first and the last are checked here; that none decreases is checked on
        // the device during the set-up (reading a million of them here would take the submitting
        // thread about a millisecond)
        const int64_t S = q.n_streamlines;
        if (q.offsets[0] != 0) return set_err(err, FASTCOD_ERANGE, "offsets[0] must be 0");
        const int64_t P = q.offsets[S];
        if (P < 0) return set_err(err, FASTCOD_ERANGE, "offsets decrease");
        if (P > 0 && !q.points) return set_err(err, FASTCOD_EINVAL, "points is NULL");
        if (P >= (int64_t(1) << 47)) return set_err(err, FASTCOD_EINVAL, "too many points");
        const uint64_t need = request_bytes(S, P, v->N, v->M, q.flags, q.mode) + Arena::round(v->bytes) +
                              Arena::round(v->tmp_bytes);
        if (need > arena_.size())
            return set_err(err, FASTCOD_ENOMEM, "request needs " + std::to_string(need) +
                                                    " device bytes, more than the server's budget of " +
                                                    std::to_string(arena_.size()));
        auto r = std::make_unique<Request>();
        r->id = ++next_id_;
        r->vol = q.volume_id;
        r->flags = q.flags;
        r->points = q.points;
        r->offsets = q.offsets;
        r->S = S;
        r->P = P;
        r->scale = q.scale;
        r->mode = q.mode;
        r->up = up;
        r->C_out = q.C_out;
        r->N = v->N;
        r->M = v->M;
        if (q.flags & FASTCOD_REQ_AFTER_STREAM) {
            const int rc = ex_->after_stream(q.stream, &r->ready);
            if (rc) return set_err(err, rc, "could not record the request's stream: " + ex_->detail());
        }
        r->t_submit = now_ns();
        pending_.push_back(r.get());
        *id = r->id;
        reqs_[r->id] = std::move(r);
        return FASTCOD_OK;
    }

    // Pending: finished at once.  Admitted: no further uploads or ticks; finished once the device
    // work already issued for it has drained.  Finished or unknown ids: EINVAL.
    int cancel(uint64_t id) {
        auto it = reqs_.find(id);
        if (it == reqs_.end() || it->second->state == State::Done) return FASTCOD_EINVAL;
        Request &r = *it->second;
        r.cancel = true;
        if (r.state == State::Pending) {
            pending_.erase(std::remove(pending_.begin(), pending_.end(), &r), pending_.end());
            finish(r, FASTCOD_ECANCELED);
        }
        return FASTCOD_OK;
    }

    const Request *request(uint64_t id) const {
        auto it = reqs_.find(id);
        return it == reqs_.end() ? nullptr : it->second.get();
    }
    // drops a finished request's record
    void forget(uint64_t id) {
        auto it = reqs_.find(id);
        if (it != reqs_.end() && it->second->state == State::Done) reqs_.erase(it);
    }

    // Cancels everything; the owner keeps calling step() until idle().
    void stop() {
        stopping_ = true;
        std::vector<uint64_t> ids;
        for (auto &kv : reqs_)
            if (kv.second->state != State::Done) ids.push_back(kv.first);
        for (uint64_t id : ids) cancel(id);
    }

    // True while device work is in flight or admitted work remains.
    bool busy() const {
        if (!ticks_.empty()) return true;
        for (const auto &v : vols_)
            if (v->build) return true;
        return !active_.empty();
    }
    bool idle() const { return !busy() && pending_.empty(); }

    // One scheduling pass.  Returns true if it issued or retired anything.
    bool step() {
        if (failed_) return false;
        bool progress = poll();
        if (failed_) return true;
        progress |= admit();
        if (failed_) return true;
        progress |= issue_uploads();
        if (failed_) return true;
        progress |= issue_tick();
        if (failed_) return true;
        progress |= issue_finals();
        return progress;
    }

    // statistics
    uint64_t ticks_launched() const { return tick_seq_; }
    uint64_t volume_builds() const { return builds_; }
    uint64_t evictions() const { return evictions_; }
    size_t pending_count() const { return pending_.size(); }
    size_t active_count() const { return active_.size(); }
    uint64_t completed() const { return completed_; }

  private:
    static int set_err(std::string *err, int rc, const std::string &m) {
        if (err) *err = m;
        return rc;
    }

    void fail(int rc, const std::string &msg) {
        failed_ = rc;
        const std::string d = ex_->detail();
        fail_msg_ = d.empty() ? msg : msg + " (" + d + ")";
        // every unfinished request ends with the error; device memory is left as it is
        for (auto &kv : reqs_) {
            Request &r = *kv.second;
            if (r.state == State::Done) continue;
            r.state = State::Done;
            r.status = rc;
            r.t_done = now_ns();
            ++completed_;
        }
        pending_.clear();
        active_.clear();
    }

    void finish(Request &r, int status) {
        arena_.release(r.off_C);
        arena_.release(r.off_offsets);
        arena_.release(r.off_points);
        arena_.release(r.off_ends);
        r.off_C = r.off_offsets = r.off_points = r.off_ends = -1;
        if (r.ready) {
            ex_->release(r.ready);
            r.ready = 0;
        }
        if (r.state == State::Active || r.state == State::Finalizing) {
            Volume &v = *vols_[r.vol];
            --v.users;
            v.last_use = ++use_clock_;
            active_.erase(std::remove(active_.begin(), active_.end(), &r), active_.end());
        }
        r.state = State::Done;
        r.status = status;
        r.t_done = now_ns();
        ++completed_;
    }

    // 1 done, 0 not yet; errors fail the server
    int check(Token &t, const char *what) {
        if (!t) return 1;
        const int q = ex_->query(t);
        if (q < 0) {
            fail(q, std::string("device operation failed: ") + what);
            return 0;
        }
        if (q == 1) {
            ex_->release(t);
            t = 0;
        }
        return q;
    }

    bool poll() {
        bool progress = false;
        while (!ticks_.empty()) {
            Token t = ticks_.front().second;
            const int q = check(t, "counting launch");
            if (failed_) return true;
            if (!q) break;
            done_tick_ = ticks_.front().first;
            ticks_.pop_front();
            progress = true;
        }
        for (auto &vp : vols_) {
            Volume &v = *vp;
            if (!v.build) continue;
            if (!check(v.build, "volume build")) {
                if (failed_) return true;
                continue;
            }
            arena_.release(v.tmp_off);
            v.tmp_off = -1;
            progress = true;
        }
        std::vector<Request *> act = active_;
        for (Request *rp : act) {
            Request &r = *rp;
            if (r.begin) {
                const int q = check(r.begin, "request set-up");
                if (failed_) return true;
                if (q) {   // set up: its offsets checked on the device
                    const int st = ex_->setup_status(r);
                    if (st != FASTCOD_OK && !r.cancel) {
                        r.cancel = true;   // ends like a cancelled request, once its uploads are done
                        r.cancel_status = st;
                    }
                    progress = true;
                }
            }
            while (!r.uploads.empty()) {
                Token t = r.uploads.front().first;
                const int q = check(t, "point upload");
                if (failed_) return true;
                if (!q) break;
                r.ready_s = r.uploads.front().second;
                r.uploads.pop_front();
                --uploads_in_flight_;
                progress = true;
            }
            if (r.state == State::Finalizing) {
                const int q = check(r.final, "result copy");
                if (failed_) return true;
                if (q) {
                    finish(r, FASTCOD_OK);
                    progress = true;
                }
            } else if (r.cancel && !r.begin && r.uploads.empty() && r.last_tick <= done_tick_) {
                finish(r, r.cancel_status);
                progress = true;
            }
        }
        return progress;
    }

    bool evict_one(const Volume *keep) {
        Volume *victim = nullptr;
        for (auto &vp : vols_) {
            Volume &v = *vp;
            if (&v == keep || v.off < 0 || v.users > 0 || v.build) continue;
            if (!victim || v.last_use < victim->last_use) victim = &v;
        }
        if (!victim) return false;
        arena_.release(victim->off);
        victim->off = -1;
        ++evictions_;
        return true;
    }

    // Bytes that evicting every idle resident volume other than `keep` would free.
    uint64_t evictable_bytes(const Volume *keep) const {
        uint64_t b = 0;
        for (const auto &vp : vols_)
            if (vp.get() != keep && vp->off >= 0 && vp->users == 0 && !vp->build) b += Arena::round(vp->bytes);
        return b;
    }

    bool try_admit(Request &r) {
        Volume &v = *vols_[r.vol];
        uint64_t need = Arena::round(8 * (uint64_t)(r.S + 1));
        if (v.off < 0) need += Arena::round(v.bytes) + Arena::round(v.tmp_bytes);
        if (!(r.flags & FASTCOD_REQ_DEVICE_POINTS)) need += Arena::round(12 * (uint64_t)r.P);
        if (!(r.flags & FASTCOD_REQ_DEVICE_C)) need += Arena::round(4 * (uint64_t)r.N * (uint64_t)r.M);
        const uint64_t eb = ends_bytes(r.S, r.mode);
        if (eb) need += Arena::round(eb);
        for (;;) {
            int64_t offs[6] = {-1, -1, -1, -1, -1, -1};
            bool ok = true;
            auto take = [&](int k, uint64_t bytes) {
                if (!ok) return;
                offs[k] = arena_.alloc(bytes);
                ok = offs[k] >= 0;
            };
            if (v.off < 0) {
                take(0, v.bytes);
                take(1, v.tmp_bytes);
            }
            take(2, 8 * (uint64_t)(r.S + 1));
            if (!(r.flags & FASTCOD_REQ_DEVICE_POINTS)) take(3, 12 * (uint64_t)r.P);
            if (!(r.flags & FASTCOD_REQ_DEVICE_C)) take(4, 4 * (uint64_t)r.N * (uint64_t)r.M);
            if (eb) take(5, eb);
            if (ok) {
                if (v.off < 0) {
                    v.off = offs[0];
                    v.tmp_off = offs[1];
                    const int rc = ex_->build_volume(v, &v.build);
                    if (rc) {
                        fail(rc, "volume build could not be issued");
                        return false;
                    }
                    ++v.builds;
                    ++builds_;
                }
                r.off_offsets = offs[2];
                r.off_points = offs[3];
                r.off_C = offs[4];
                r.off_ends = offs[5];
                return true;
            }
            for (int64_t o : offs) arena_.release(o);
            // evict only when that can make room; otherwise wait for admitted requests to finish
            if (arena_.size() - arena_.used() + evictable_bytes(&v) < need) return false;
            if (!evict_one(&v)) return false;
        }
    }

    // admitted requests still counting: those whose result is on its way out make room for the next
    int32_t counting() const {
        int32_t n = 0;
        for (const Request *r : active_) n += r->state == State::Active ? 1 : 0;
        return n;
    }

    bool admit() {
        bool progress = false;
        while (!pending_.empty() && counting() < cfg_.max_active) {
            Request &r = *pending_.front();
            if (!try_admit(r)) break;
            if (failed_) return true;
            pending_.pop_front();
            Volume &v = *vols_[r.vol];
            ++v.users;
            v.last_use = ++use_clock_;
            r.state = State::Active;
            r.t_admit = now_ns();
            active_.push_back(&r);
            const int rc = ex_->begin_request(r, &r.begin);
            if (rc) {
                fail(rc, "request set-up could not be issued");
                return true;
            }
            if (r.ready) {   // begin_request has ordered the request's device work after it
                ex_->release(r.ready);
                r.ready = 0;
            }
            if (r.flags & FASTCOD_REQ_DEVICE_POINTS) r.issued_s = r.ready_s = r.S;
            progress = true;
        }
        return progress;
    }

    // end of the range that starts at s0 and holds at least `pts` points (one streamline at least)
    static int64_t range_end(const Request &r, int64_t s0, int64_t pts, int64_t limit) {
        if (s0 >= limit) return limit;
        const int64_t target = r.offsets[s0] + pts;
        const int64_t *b = r.offsets + s0 + 1, *e = r.offsets + limit + 1;
        const int64_t *it = std::lower_bound(b, e, target);   // first s1 with offsets[s1] >= target
        const int64_t s1 = it == e ? limit : (int64_t)(it - r.offsets);
        return std::max<int64_t>(std::min<int64_t>(s1, limit), s0 + 1);
    }

    bool issue_uploads() {
        bool progress = false;
        if (active_.empty()) return false;
        // round robin over active requests with host points left to send
        for (bool any = true; any && uploads_in_flight_ < cfg_.upload_window;) {
            any = false;
            for (size_t k = 0; k < active_.size() && uploads_in_flight_ < cfg_.upload_window; ++k) {
                Request &r = *active_[(upload_rr_ + k) % active_.size()];
                if (r.cancel || r.state != State::Active || r.issued_s >= r.S) continue;
                const int64_t s1 = range_end(r, r.issued_s, cfg_.chunk_points, r.S);
                Token t = 0;
                const int rc = ex_->upload(r, r.issued_s, s1, &t);
                if (rc) {
                    fail(rc, "point upload could not be issued");
                    return true;
                }
                r.uploads.emplace_back(t, s1);
                r.issued_s = s1;
                ++uploads_in_flight_;
                any = progress = true;
            }
            ++upload_rr_;
        }
        return progress;
    }

    bool issue_tick() {
        if ((int32_t)ticks_.size() >= cfg_.ticks_in_flight) return false;
        std::vector<Request *> ready;   // in admission order: oldest first
        for (Request *r : active_)   // (set-up done: C zeroed, offsets on the device)
            if (!r->cancel && r->state == State::Active && !r->begin && r->next_s < r->ready_s) ready.push_back(r);
        if (ready.empty()) return false;
        // a floor share for every ready request; the spare points of the tick to the oldest first
        const int64_t n = (int64_t)ready.size();
        const int64_t floor_pts = std::min<int64_t>(cfg_.chunk_points, std::max<int64_t>(1, cfg_.tick_points / n));
        int64_t spare = cfg_.tick_points;
        for (Request *r : ready) spare -= std::min<int64_t>(floor_pts, r->offsets[r->ready_s] - r->offsets[r->next_s]);
        int64_t pts = 0, sl = 0;
        std::vector<Chunk> chunks;
        for (Request *r : ready) {
            if (pts >= cfg_.tick_points || sl >= cfg_.tick_streamlines) break;
            const int64_t left = r->offsets[r->ready_s] - r->offsets[r->next_s];
            const int64_t base = std::min<int64_t>(floor_pts, left);
            const int64_t extra = std::min<int64_t>(std::max<int64_t>(spare, 0), left - base);
            spare -= extra;
            const int64_t want = std::min<int64_t>(base + extra, cfg_.tick_points - pts);
            const int64_t lim = std::min<int64_t>(r->ready_s, r->next_s + (cfg_.tick_streamlines - sl));
            const int64_t s1 = range_end(*r, r->next_s, want, lim);
            chunks.push_back(Chunk{r, vols_[r->vol].get(), r->next_s, s1});
            pts += r->offsets[s1] - r->offsets[r->next_s];
            sl += s1 - r->next_s;
        }
        Token t = 0;
        const int rc = ex_->launch_tick(chunks, &t);
        if (rc) {
            fail(rc, "counting launch could not be issued");
            return true;
        }
        const uint64_t seq = ++tick_seq_;
        ticks_.emplace_back(seq, t);
        for (const Chunk &c : chunks) {
            Request *r = const_cast<Request *>(c.req);
            r->next_s = c.s1;
            r->last_tick = seq;
            ++r->chunks;
            ++r->ticks;
        }
        return true;
    }

    bool issue_finals() {
        bool progress = false;
        for (Request *r : active_) {   // (after the set-up: a request without streamlines has no tick)
            if (r->cancel || r->state != State::Active || r->begin || r->next_s < r->S) continue;
            const int rc = ex_->finalize(*r, &r->final);
            if (rc) {
                fail(rc, "result copy could not be issued");
                return true;
            }
            r->state = State::Finalizing;
            progress = true;
        }
        return progress;
    }

    Config cfg_;
    Executor *ex_;
    Arena arena_;
    std::vector<std::unique_ptr<Volume>> vols_;
    std::map<uint64_t, std::unique_ptr<Request>> reqs_;
    std::deque<Request *> pending_;
    std::vector<Request *> active_;
    std::deque<std::pair<uint64_t, Token>> ticks_;   // (sequence, token) in issue order
    uint64_t tick_seq_ = 0, done_tick_ = 0, next_id_ = 0, use_clock_ = 0;
    uint64_t builds_ = 0, evictions_ = 0, completed_ = 0;
    int32_t uploads_in_flight_ = 0;
    size_t upload_rr_ = 0;
    int failed_ = 0;
    bool stopping_ = false;
    std::string fail_msg_;
};

// ---------------------------------------------------------------------------------------------
// Service: the core behind a mutex, driven by one scheduler thread.
// ---------------------------------------------------------------------------------------------
class Service {
  public:
    // `thread_init` runs first on the scheduler thread (e.g. to make the device current).
    Service(const Config &cfg, std::unique_ptr<Executor> ex, std::function<void()> thread_init = nullptr)
        : ex_(std::move(ex)), core_(cfg, ex_.get()) {
        th_ = std::thread([this, thread_init]() {
            if (thread_init) thread_init();
            loop();
        });
    }
    ~Service() { shutdown(); }

    void shutdown() {
        {
            std::lock_guard<std::mutex> g(mu_);
            if (quit_) return;
            core_.stop();
            quit_ = true;
        }
        work_.notify_all();
        if (th_.joinable()) th_.join();
    }

    template <typename F>
    auto locked(F &&f) -> decltype(f(std::declval<Core &>())) {
        std::lock_guard<std::mutex> g(mu_);
        return f(core_);
    }

    int add_volume(const int32_t *roi, const int32_t *lab, const int32_t dims[3], int32_t N, int32_t M, int32_t *id,
                   std::string *err) {
        std::lock_guard<std::mutex> g(mu_);
        return core_.add_volume(roi, lab, dims, N, M, id, err);
    }
    int submit(const fastcod_request &q, uint64_t *id, std::string *err) {
        int rc;
        {
            std::lock_guard<std::mutex> g(mu_);
            rc = core_.submit(q, id, err);
        }
        if (!rc) work_.notify_all();
        return rc;
    }
    int cancel(uint64_t id) {
        int rc;
        {
            std::lock_guard<std::mutex> g(mu_);
            rc = core_.cancel(id);
        }
        work_.notify_all();
        return rc;
    }
    // Request status once finished (its record is then dropped), FASTCOD_ETIMEDOUT if it is still
    // running after timeout_us (< 0: no limit), FASTCOD_EINVAL for an unknown id.
    int wait(uint64_t id, int64_t timeout_us, fastcod_request_info *info) {
        std::unique_lock<std::mutex> lk(mu_);
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::microseconds(timeout_us);
        for (;;) {
            const Request *r = core_.request(id);
            if (!r) return FASTCOD_EINVAL;
            if (r->state == State::Done) {
                if (info) {
                    info->status = r->status;
                    info->t_submit_ns = r->t_submit;
                    info->t_admit_ns = r->t_admit;
                    info->t_done_ns = r->t_done;
                    info->chunks = r->chunks;
                    info->device_bytes = (int64_t)Core::request_bytes(r->S, r->P, r->N, r->M, r->flags, r->mode);
                }
                const int st = r->status;
                core_.forget(id);
                return st;
            }
            if (timeout_us < 0) {
                done_.wait(lk);
            } else if (done_.wait_until(lk, deadline) == std::cv_status::timeout) {
                const Request *r2 = core_.request(id);
                if (r2 && r2->state == State::Done) continue;
                return FASTCOD_ETIMEDOUT;
            }
        }
    }

  private:
    void loop() {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            const uint64_t before = core_.completed();
            core_.step();
            if (core_.completed() != before) done_.notify_all();
            if (core_.failed()) {
                done_.notify_all();
                if (quit_) break;
                work_.wait(lk);
                continue;
            }
            if (quit_ && core_.idle()) break;
            if (core_.busy()) {
                lk.unlock();
                ex_->pause();
                lk.lock();
            } else if (!quit_) {
                work_.wait(lk);   // nothing in flight: until a submit, cancel or shutdown
            }
        }
        done_.notify_all();
    }

    std::unique_ptr<Executor> ex_;
    Core core_;
    std::mutex mu_;
    std::condition_variable work_, done_;
    bool quit_ = false;
    std::thread th_;
};

}  // namespace fcs
