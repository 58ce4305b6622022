// Host test harness of the request server's scheduling core (paper_2302_09247_amd/csrc/server_core.h):
// a simulated executor whose device operations only record what was asked and complete when the
// test says so, plus a C API for ctypes.  Built with g++ by the tests; no HIP, no counting.
#include <stdint.h>
#include <string.h>

#include <map>
#include <memory>
#include <vector>

#include "server_core.h"

namespace {

enum Kind { kBuild = 0, kBegin = 1, kUpload = 2, kTick = 3, kFinal = 4, kKinds = 5 };

struct Op {
    int64_t kind, a, b, c, d;   // build: vol; begin/final: req; upload: req, s0, s1; tick: seq, req, s0, s1
};

class SimExecutor final : public fcs::Executor {
  public:
    uint64_t next_bytes = 1 << 20, next_tmp = 1 << 20;
    int auto_polls = -1;                 // >= 0: a token completes after this many queries
    int fail_issue[kKinds] = {0, 0, 0, 0, 0};   // next issue of that kind returns this status
    bool fail_done[kKinds] = {false, false, false, false, false};   // queries of that kind report an error
    std::vector<Op> ops;
    std::vector<int64_t> chunk_log;      // (tick, req, s0, s1)
    int64_t ticks = 0;
    struct Tok {
        int kind;
        bool done;
        int polls;
    };
    std::map<fcs::Token, Tok> toks;
    fcs::Token next_tok = 0;
    int64_t live_tokens = 0;

    int volume_bytes(const fcs::Volume &, uint64_t *bytes, uint64_t *tmp) override {
        *bytes = next_bytes;
        *tmp = next_tmp;
        return FASTCOD_OK;
    }
    int build_volume(const fcs::Volume &v, fcs::Token *t) override {
        if (int rc = issue(kBuild, t)) return rc;
        ops.push_back({kBuild, v.id, v.off, v.tmp_off, 0});
        return FASTCOD_OK;
    }
    int begin_request(const fcs::Request &r, fcs::Token *t) override {
        if (int rc = issue(kBegin, t)) return rc;
        ops.push_back({kBegin, (int64_t)r.id, r.off_C, r.off_offsets, r.off_points});
        return FASTCOD_OK;
    }
    // the device check of the set-up, done on the host copy: no offset may decrease
    int setup_status(const fcs::Request &r) override {
        for (int64_t s = 0; s < r.S; ++s)
            if (r.offsets[s + 1] < r.offsets[s]) return FASTCOD_ERANGE;
        return FASTCOD_OK;
    }
    int upload(const fcs::Request &r, int64_t s0, int64_t s1, fcs::Token *t) override {
        if (int rc = issue(kUpload, t)) return rc;
        ops.push_back({kUpload, (int64_t)r.id, s0, s1, 0});
        return FASTCOD_OK;
    }
    int launch_tick(const std::vector<fcs::Chunk> &chunks, fcs::Token *t) override {
        if (int rc = issue(kTick, t)) return rc;
        ++ticks;
        for (const fcs::Chunk &c : chunks) {
            chunk_log.push_back(ticks);
            chunk_log.push_back((int64_t)c.req->id);
            chunk_log.push_back(c.s0);
            chunk_log.push_back(c.s1);
            // a chunk never reaches past the streamlines whose uploads have completed
            if (c.s1 > c.req->ready_s || c.s0 != c.req->next_s) chunk_log.push_back(-999);
        }
        ops.push_back({kTick, ticks, (int64_t)chunks.size(), 0, 0});
        return FASTCOD_OK;
    }
    int finalize(const fcs::Request &r, fcs::Token *t) override {
        if (int rc = issue(kFinal, t)) return rc;
        ops.push_back({kFinal, (int64_t)r.id, 0, 0, 0});
        return FASTCOD_OK;
    }
    int query(fcs::Token t) override {
        auto it = toks.find(t);
        if (it == toks.end()) return FASTCOD_EINVAL;
        Tok &k = it->second;
        if (fail_done[k.kind]) return FASTCOD_EHIP;
        if (auto_polls >= 0 && ++k.polls > auto_polls) k.done = true;
        return k.done ? 1 : 0;
    }
    void release(fcs::Token t) override {
        if (toks.erase(t)) --live_tokens;
    }
    void pause() override {}
    std::string detail() const override { return "simulated"; }

    void complete(int kind) {
        for (auto &kv : toks)
            if (kind < 0 || kv.second.kind == kind) kv.second.done = true;
    }

  private:
    int issue(int kind, fcs::Token *t) {
        if (fail_issue[kind]) {
            const int rc = fail_issue[kind];
            fail_issue[kind] = 0;
            return rc;
        }
        *t = ++next_tok;
        toks[*t] = Tok{kind, false, 0};
        ++live_tokens;
        return FASTCOD_OK;
    }
};

struct Sim {
    SimExecutor *ex;   // owned by core's owner below
    std::unique_ptr<SimExecutor> own;
    std::unique_ptr<fcs::Core> core;
};

struct Svc {
    SimExecutor *ex;
    std::unique_ptr<fcs::Service> svc;
};

const float kDummyPoint[3] = {0.f, 0.f, 0.f};
int32_t g_dummy_c[1];

fcs::Config make_cfg(uint64_t budget, int64_t tick_points, int64_t tick_streamlines, int64_t chunk_points,
                     int32_t max_active, int32_t upload_window, int32_t ticks_in_flight) {
    fcs::Config c;
    c.budget = budget;
    c.tick_points = tick_points;
    c.tick_streamlines = tick_streamlines;
    c.chunk_points = chunk_points;
    c.max_active = max_active;
    c.upload_window = upload_window;
    c.ticks_in_flight = ticks_in_flight;
    return c;
}

fastcod_request make_req(int32_t vol, uint32_t flags, const int64_t *offsets, int64_t S) {
    fastcod_request q;
    memset(&q, 0, sizeof(q));
    q.volume_id = vol;
    q.flags = flags;
    q.points = kDummyPoint;
    q.offsets = offsets;
    q.n_streamlines = S;
    q.scale = 1.0f;
    q.C_out = g_dummy_c;
    return q;
}

}  // namespace

extern "C" {

// ---- arena ----
void *arena_new(uint64_t size) {
    auto *a = new fcs::Arena();
    a->reset(size);
    return a;
}
int64_t arena_alloc(void *a, uint64_t bytes) { return static_cast<fcs::Arena *>(a)->alloc(bytes); }
void arena_free(void *a, int64_t off) { static_cast<fcs::Arena *>(a)->release(off); }
uint64_t arena_used(void *a) { return static_cast<fcs::Arena *>(a)->used(); }
uint64_t arena_largest(void *a) { return static_cast<fcs::Arena *>(a)->largest_free(); }
int64_t arena_free_blocks(void *a) { return (int64_t)static_cast<fcs::Arena *>(a)->free_blocks(); }
void arena_delete(void *a) { delete static_cast<fcs::Arena *>(a); }

// ---- core, stepped by the test ----
void *sim_create(uint64_t budget, int64_t tick_points, int64_t tick_streamlines, int64_t chunk_points,
                 int32_t max_active, int32_t upload_window, int32_t ticks_in_flight) {
    auto *s = new Sim();
    s->own = std::make_unique<SimExecutor>();
    s->ex = s->own.get();
    s->core = std::make_unique<fcs::Core>(
        make_cfg(budget, tick_points, tick_streamlines, chunk_points, max_active, upload_window, ticks_in_flight),
        s->ex);
    return s;
}
void sim_destroy(void *p) { delete static_cast<Sim *>(p); }

int sim_add_volume(void *p, int32_t N, int32_t M, uint64_t bytes, uint64_t tmp_bytes, int32_t *id) {
    Sim *s = static_cast<Sim *>(p);
    s->ex->next_bytes = bytes;
    s->ex->next_tmp = tmp_bytes;
    const int32_t dims[3] = {4, 4, 4};
    std::string err;
    return s->core->add_volume(nullptr, nullptr, dims, N, M, id, &err);
}

int sim_submit(void *p, int32_t vol, uint32_t flags, const int64_t *offsets, int64_t S, uint64_t *id) {
    Sim *s = static_cast<Sim *>(p);
    std::string err;
    return s->core->submit(make_req(vol, flags, offsets, S), id, &err);
}

int sim_step(void *p) { return static_cast<Sim *>(p)->core->step() ? 1 : 0; }
void sim_complete(void *p, int kind) { static_cast<Sim *>(p)->ex->complete(kind); }
void sim_auto(void *p, int polls) { static_cast<Sim *>(p)->ex->auto_polls = polls; }
void sim_fail_issue(void *p, int kind, int status) { static_cast<Sim *>(p)->ex->fail_issue[kind] = status; }
void sim_fail_done(void *p, int kind) { static_cast<Sim *>(p)->ex->fail_done[kind] = true; }
int sim_cancel(void *p, uint64_t id) { return static_cast<Sim *>(p)->core->cancel(id); }
void sim_stop(void *p) { static_cast<Sim *>(p)->core->stop(); }
int sim_idle(void *p) { return static_cast<Sim *>(p)->core->idle() ? 1 : 0; }

// state: 0 pending, 1 active, 2 finalizing, 3 done; returns -1 for an unknown id
int sim_state(void *p, uint64_t id, int32_t *state, int32_t *status, int64_t *chunks) {
    const fcs::Request *r = static_cast<Sim *>(p)->core->request(id);
    if (!r) return -1;
    *state = (int32_t)r->state;
    *status = r->status;
    *chunks = r->chunks;
    return 0;
}

int64_t sim_chunks(void *p, int64_t *out, int64_t cap) {
    const auto &v = static_cast<Sim *>(p)->ex->chunk_log;
    const int64_t n = std::min<int64_t>(cap, (int64_t)v.size());
    if (out) memcpy(out, v.data(), 8 * n);
    return (int64_t)v.size();
}

int64_t sim_ops(void *p, int64_t *out, int64_t cap) {
    const auto &v = static_cast<Sim *>(p)->ex->ops;
    const int64_t n = std::min<int64_t>(cap, (int64_t)v.size());
    for (int64_t i = 0; i < n; ++i) {
        out[5 * i] = v[i].kind;
        out[5 * i + 1] = v[i].a;
        out[5 * i + 2] = v[i].b;
        out[5 * i + 3] = v[i].c;
        out[5 * i + 4] = v[i].d;
    }
    return (int64_t)v.size();
}

// [used, size, pending, active, completed, ticks, builds, evictions, failed, largest_free, live_tokens]
void sim_stats(void *p, int64_t *out) {
    Sim *s = static_cast<Sim *>(p);
    const fcs::Core &c = *s->core;
    out[0] = (int64_t)c.arena().used();
    out[1] = (int64_t)c.arena().size();
    out[2] = (int64_t)c.pending_count();
    out[3] = (int64_t)c.active_count();
    out[4] = (int64_t)c.completed();
    out[5] = (int64_t)c.ticks_launched();
    out[6] = (int64_t)c.volume_builds();
    out[7] = (int64_t)c.evictions();
    out[8] = c.failed();
    out[9] = (int64_t)c.arena().largest_free();
    out[10] = s->ex->live_tokens;
}

// ---- threaded service with a self-completing executor ----
void *svc_create(uint64_t budget, int64_t tick_points, int64_t chunk_points, int32_t max_active, int32_t polls) {
    auto ex = std::make_unique<SimExecutor>();
    ex->auto_polls = polls;
    auto *v = new Svc();
    v->ex = ex.get();
    v->svc = std::make_unique<fcs::Service>(make_cfg(budget, tick_points, 1 << 20, chunk_points, max_active, 8, 2),
                                            std::move(ex));
    return v;
}
int svc_add_volume(void *p, int32_t N, int32_t M, uint64_t bytes, int32_t *id) {
    Svc *v = static_cast<Svc *>(p);
    return v->svc->locked([&](fcs::Core &c) {
        v->ex->next_bytes = bytes;
        v->ex->next_tmp = 256;
        const int32_t dims[3] = {4, 4, 4};
        std::string err;
        return c.add_volume(nullptr, nullptr, dims, N, M, id, &err);
    });
}
int svc_submit(void *p, int32_t vol, const int64_t *offsets, int64_t S, uint64_t *id) {
    std::string err;
    return static_cast<Svc *>(p)->svc->submit(make_req(vol, 0, offsets, S), id, &err);
}
int svc_wait(void *p, uint64_t id, int64_t timeout_us, int64_t *t_submit, int64_t *t_done) {
    fastcod_request_info info;
    memset(&info, 0, sizeof(info));
    const int rc = static_cast<Svc *>(p)->svc->wait(id, timeout_us, &info);
    *t_submit = info.t_submit_ns;
    *t_done = info.t_done_ns;
    return rc;
}
int svc_cancel(void *p, uint64_t id) { return static_cast<Svc *>(p)->svc->cancel(id); }
void svc_destroy(void *p) { delete static_cast<Svc *>(p); }

}  // extern "C"
