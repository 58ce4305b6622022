// Device code of libfastcod.so (gfx950, wave64): pass-through connectivity counting.
//
// The operation is FastCod's Alg. 2 (Section 2, "Method"): for every streamline, the set of ROI
// rows it passes through (passthrough) and the set of target labels it passes through
// (loc2region applied to its points) are formed, and every (row, label) pair of the two sets adds
// one to C.  The stages here:
//   * compact volume build: one read of both volumes -> occupancy bits + packed codes;
//   * partition: chunks of whole streamlines, equal or tapering (a binary search per chunk); the same
//     launch zeroes the call's per-call state;
//   * count kernels (wave-per-streamline over raster volumes, or flat point stream over the
//     compact volume): voxelise each point, look it up, de-duplicate the hits of each streamline
//     in a per-wavefront LDS hash set, and emit its |I| x |M| pair updates: the flat-stream
//     kernel appends them to per-wavefront slices of a pair buffer, the others (and a full slice)
//     add them into C with global atomics;
//   * pair histogram: a counting sort of the appended updates by tile of C, then one LDS
//     histogram per tile added into C;
//   * fallback: streamlines with more distinct keys than the LDS set holds, one workgroup each,
//     with global bit maps.
// Integer counting is exact and additions commute, so every variant gives the same C.
#include "internal.h"

#include <algorithm>

namespace fc {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kLabelTag = 0x80000000u;

__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// number of set bits of m below this lane
__device__ __forceinline__ int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// this lane's bit of a wave-uniform mask, which the hardware takes directly as a lane predicate
__device__ __forceinline__ bool in_mask(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Global-memory views of pointers the compiler cannot place by itself (pointers read from a table
// in memory rather than passed as kernel arguments).  It would access them with flat instructions,
// which also count against the LDS wait counter: every LDS wait after one would wait for it too.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gview(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
// C[k] += 1 as a device-scope atomic without return, in global memory
__device__ __forceinline__ void add_one(int32_t *p) {
    __hip_atomic_fetch_add((__attribute__((address_space(1))) int32_t *)p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lanes_between(int lo, int hi) {  // bits [lo, hi)
    const uint64_t below_hi = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    return below_hi & ~((1ull << lo) - 1ull);
}

__device__ __forceinline__ float load_stream(const float *p) { return __builtin_nontemporal_load(p); }

// Voxel of one point: per axis t = fl32(fl32(p*s) + 0.5) and floor(t), inside iff 0 <= t < size.
// (floor(t) >= 0 iff t >= 0, and floor(t) < size iff t < size; NaN fails both.)  __fmul_rn /
// __fadd_rn are never contracted into an FMA.
template <bool SCALED>
__device__ __forceinline__ bool voxelise(float x, float y, float z, float s, const Grid &g, int &ix,
                                         int &iy, int &iz) {
    if (SCALED) {
        x = __fmul_rn(x, s);
        y = __fmul_rn(y, s);
        z = __fmul_rn(z, s);
    }
    const float tx = __fadd_rn(x, 0.5f), ty = __fadd_rn(y, 0.5f), tz = __fadd_rn(z, 0.5f);
    const bool in = (tx >= 0.0f) & (tx < g.Xf) & (ty >= 0.0f) & (ty < g.Yf) & (tz >= 0.0f) & (tz < g.Zf);
    ix = in ? (int)tx : 0;  // truncation == floor for t >= 0
    iy = in ? (int)ty : 0;
    iz = in ? (int)tz : 0;
    return in;
}

// ---------------------------------------------------------------------------------------------
// volume lookups
// ---------------------------------------------------------------------------------------------

__device__ __forceinline__ void raster_get(const RasterVol &v, int ix, int iy, int iz, int &r, int &m) {
    const int lin = ix + v.X * iy + v.XY * iz;
    const int rv = v.roi[lin], mv = v.lab[lin];
    r = (unsigned)rv < (unsigned)v.N ? rv : -1;
    m = (unsigned)mv < (unsigned)v.M ? mv : -1;
}

__device__ __forceinline__ uint32_t compact_word(const CompactVol &c, int ix, int iy, int iz, uint32_t &bit) {
    const uint32_t sb = (uint32_t)(ix >> 4) + (uint32_t)c.SBX * (uint32_t)(iy >> 3) +
                        (uint32_t)c.SBXY * (uint32_t)(iz >> 3);
    const uint32_t b = (uint32_t)(ix & 15) | ((uint32_t)(iy & 7) << 4) | ((uint32_t)(iz & 7) << 7);
    bit = b & 31u;
    return (sb << 5) | (b >> 5);
}

__device__ __forceinline__ void compact_get(const CompactVol &c, int ix, int iy, int iz, int &r, int &m) {
    uint32_t bit;
    const uint32_t w = compact_word(c, ix, iy, iz, bit);
    const uint2 e = c.mb[w];
    r = -1;
    m = -1;
    if (!((e.x >> bit) & 1u)) return;
    const uint32_t rank = e.y + __popc(e.x & ((1u << bit) - 1u));
    if (c.packed) {
        const uint32_t code = c.codes32[rank];
        const uint32_t rv = code & c.rmask, mv = code >> c.rbits;
        r = rv < (uint32_t)c.N ? (int)rv : -1;
        m = mv < (uint32_t)c.M ? (int)mv : -1;
    } else {
        const int2 code = c.codes64[rank];
        r = code.x;
        m = code.y;
    }
}

struct RasterLookup {
    RasterVol v;
    __device__ void get(int ix, int iy, int iz, int &r, int &m) const { raster_get(v, ix, iy, iz, r, m); }
};
struct CompactLookup {
    CompactVol v;
    __device__ void get(int ix, int iy, int iz, int &r, int &m) const { compact_get(v, ix, iy, iz, r, m); }
};

// ---------------------------------------------------------------------------------------------
// per-wavefront set of the open streamline's distinct keys (LDS, open addressing)
//   key = row for ROI hits, label | kLabelTag for target hits (rows and labels are < 2^31 - 1)
//   slots[0 .. nI) hold the table slots of rows, slots[CAP/2 - nM .. CAP/2) those of labels;
//   nI + nM <= CAP/2 keeps the table at most half full, so probing always ends.
// ---------------------------------------------------------------------------------------------

template <int CAP>
struct WaveSet {
    static constexpr int kLog2 = __builtin_ctz(CAP);
    static constexpr int kHalf = CAP / 2;
    uint32_t *tab;
    uint32_t *slots;
    int nI, nM;
    bool skip;  // the open streamline overflowed: its hits are ignored until it closes

    __device__ void init(uint32_t *t, uint32_t *s) {
        tab = t;
        slots = s;
        nI = nM = 0;
        skip = false;
        for (int k = lane_id(); k < CAP; k += kWave) tab[k] = kEmpty;
    }

    // Insert the keys of the lanes in `cand`; returns the lanes whose key was not yet present.
    // The lanes still probing are a wave-uniform mask; the outcome ballots count those lanes only
    // (a lane outside `cand` may hold any value, kEmpty included, as its key).
    __device__ uint64_t insert(uint64_t cand, uint32_t key, uint32_t &slot) {
        uint64_t act = cand, fresh = 0ull;
        uint32_t h = (__umul24(key ^ (key >> 20), 0x9E3779u) >> 12) & (CAP - 1);
        while (act) {
            uint32_t old = 0u;
            if (in_mask(act)) old = atomicCAS(&tab[h], kEmpty, key);
            const uint64_t got = __ballot(old == kEmpty) & act, dup = __ballot(old == key) & act;
            if (in_mask(got)) slot = h;
            fresh |= got;
            act &= ~(got | dup);
            h = (h + 1u) & (CAP - 1);
        }
        return fresh;
    }

    // Adds the candidate rows / labels; false when the set could outgrow its capacity.
    __device__ bool add(uint64_t candR, int r, uint64_t candM, int m) {
        if (nI + nM + __popcll(candR) + __popcll(candM) > kHalf) return false;
        uint32_t slotR = 0, slotM = 0;
        const uint64_t newR = candR ? insert(candR, (uint32_t)r, slotR) : 0ull;
        const uint64_t newM = candM ? insert(candM, (uint32_t)m | kLabelTag, slotM) : 0ull;
        if (in_mask(newR)) slots[nI + mbcnt(newR)] = slotR;
        if (in_mask(newM)) slots[kHalf - 1 - (nM + mbcnt(newM))] = slotM;
        nI += __popcll(newR);
        nM += __popcll(newM);
        return true;
    }

    __device__ void clear_entries() {
        for (int k = lane_id(); k < nI; k += kWave) tab[slots[k]] = kEmpty;
        for (int k = lane_id(); k < nM; k += kWave) tab[slots[kHalf - 1 - k]] = kEmpty;
        nI = nM = 0;
    }

    // The streamline ends: C(i, m) += 1 for all its rows i and labels m (through `sink`), then reset.
    template <typename Sink>
    __device__ void close(Sink &sink, uint32_t si, uint32_t sm) {
        if (!skip && nI > 0 && nM > 0) {
            for (int b = 0; b < nI; b += kWave) {
                const int k = b + lane_id();
                const uint64_t ok = __ballot(k < nI);
                const uint32_t i = in_mask(ok) ? tab[slots[k]] : 0u;
                const uint32_t row = i * si;   // N*M < 2^31
                for (int j = 0; j < nM; ++j) {
                    const uint32_t mk = __builtin_amdgcn_readfirstlane(tab[slots[kHalf - 1 - j]]) & ~kLabelTag;
                    sink.push_lanes(ok, row + mk * sm);
                }
            }
        }
        clear_entries();
        skip = false;
    }
};

// C updates straight to global memory (one atomic per pair).
struct DirectSink {
    int32_t *C;
    __device__ void push_lanes(uint64_t vm, uint32_t idx) {   // the lanes in vm (wave-uniform)
        if (in_mask(vm)) add_one(C + idx);
    }
    __device__ void push(bool valid, uint32_t idx) { push_lanes(__ballot(valid), idx); }
};

// C updates buffered per wavefront in LDS and issued 64 at a time: a wave-wide atomic
// instruction instead of one per closing streamline.  On this architecture every vector memory
// wait also waits for older atomics, so fewer, fuller atomic instructions stall the stream less.
struct BufferedSink {
    uint32_t *buf;  // [kWave] LDS
    int n;          // pending entries (wave-uniform)
    int32_t *C;
    __device__ void init(uint32_t *b, int32_t *c) {
        buf = b;
        n = 0;
        C = c;
    }
    __device__ void push(bool valid, uint32_t idx) { push_lanes(__ballot(valid), idx); }
    __device__ void push_lanes(uint64_t vm, uint32_t idx) {   // the lanes in vm (wave-uniform)
        if (!vm) return;
        const bool valid = in_mask(vm);
        const int pos = n + mbcnt(vm);
        if (valid && pos < kWave) buf[pos] = idx;
        const int cnt = __popcll(vm);
        if (n + cnt >= kWave) {
            add_one(C + buf[lane_id()]);
            if (valid && pos >= kWave) buf[pos - kWave] = idx;
            n = n + cnt - kWave;
        } else {
            n += cnt;
        }
    }
    __device__ void drain() {
        if (lane_id() < n) add_one(C + buf[lane_id()]);
        n = 0;
    }
};

// C updates appended to this wavefront's slice of a pair buffer for a later histogram pass,
// kSinkCap at a time: 16 bytes per lane per store instruction, one store per 256 updates.  On this
// architecture every later vector-memory wait also waits for older stores, so fewer, fuller
// stores stall the stream less (a cached store is acknowledged once the cache takes it; an atomic
// must first fetch its line of C).  Once the slice is full, updates go to C as atomics.
// (kSinkCap: 256 or 512, a multiple of 256; the LDS it takes limits the workgroups per CU.)
template <int kSinkCap>
struct AppendSink {
    static_assert(kSinkCap == 4 * kWave || kSinkCap == 8 * kWave, "one or two 16-byte stores per lane");
    uint32_t *buf;   // [kSinkCap] LDS, 16-byte aligned
    int n;           // pending entries (wave-uniform)
    uint32_t *out;   // next free entry of this wavefront's slice (16-byte aligned)
    uint32_t room;   // free entries left in the slice
    int32_t *C;
    __device__ void init(uint32_t *b, int32_t *c, const PairOut &po, uint32_t wave) {
        buf = b;
        n = 0;
        C = c;
        out = po.pairs + (size_t)wave * po.cap;   // (po.cap is a multiple of 4)
        room = po.cap;
    }
    __device__ void emit(int cnt) {   // the first cnt (<= kSinkCap) entries of buf
        const int lane = lane_id();
        if (cnt == kSinkCap && (uint32_t)cnt <= room) {
            const uint4 v = reinterpret_cast<const uint4 *>(buf)[lane];
            if constexpr (kSinkCap == 8 * kWave) {
                const uint4 v2 = reinterpret_cast<const uint4 *>(buf)[lane + kWave];
                reinterpret_cast<uint4 *>(out)[lane] = v;
                reinterpret_cast<uint4 *>(out)[lane + kWave] = v2;
            } else {
                reinterpret_cast<uint4 *>(out)[lane] = v;
            }
            out += kSinkCap;
            room -= (uint32_t)kSinkCap;
        } else if ((uint32_t)cnt <= room) {
            for (int k = lane; k < cnt; k += kWave) out[k] = buf[k];
            out += cnt;
            room -= (uint32_t)cnt;
        } else {
            for (int k = lane; k < cnt; k += kWave) add_one(C + buf[k]);
        }
    }
    __device__ void push(bool valid, uint32_t idx) { push_lanes(__ballot(valid), idx); }
    __device__ void push_lanes(uint64_t vm, uint32_t idx) {   // the lanes in vm (wave-uniform)
        if (!vm) return;
        const bool valid = in_mask(vm);
        const int pos = n + mbcnt(vm);
        if (valid && pos < kSinkCap) buf[pos] = idx;
        const int cnt = __popcll(vm);
        if (n + cnt >= kSinkCap) {
            emit(kSinkCap);
            if (valid && pos >= kSinkCap) buf[pos - kSinkCap] = idx;
            n = n + cnt - kSinkCap;
        } else {
            n += cnt;
        }
    }
    // flushes the pending entries and records the slice's length
    __device__ void drain(const PairOut &po, uint32_t wave) {
        if (n) emit(n);
        n = 0;
        if (lane_id() == 0) po.counts[wave] = po.cap - room;
    }
};

// Per-wavefront state of the flat-stream kernel's open streamline: raw candidate lists (hits
// that differ from the previous point's), de-duplicated only when the streamline closes and only
// if it has both rows and labels.  tab is an open-addressing set, empty between closes; it holds
// at most RCAP + LCAP <= TCAP/2 keys, so probing always ends.
template <int RCAP, int LCAP, int TCAP>
struct DeferredSet {
    static_assert(RCAP + LCAP <= TCAP / 2, "set must stay at most half full");
    uint32_t *rows;   // [RCAP] raw row candidates; at close: table slot of each new row, or kEmpty
    uint32_t *labs;   // [LCAP] raw label candidates; at close: table slot of each new label, or kEmpty
    uint32_t *ulab;   // [LCAP] distinct labels (at close)
    uint32_t *tab;    // [TCAP]
    int nR, nL;
    bool skip;        // the open streamline overflowed: its hits go to the fallback kernel

    __device__ void init(uint32_t *base) {
        rows = base;
        labs = rows + RCAP;
        ulab = labs + LCAP;
        tab = ulab + LCAP;
        nR = nL = 0;
        skip = false;
        for (int k = lane_id(); k < TCAP; k += kWave) tab[k] = kEmpty;
    }
    __device__ bool has_state() const { return (nR | nL) != 0 || skip; }

    // Endpoint modes: the open streamline's labels are its end labels (ml, mf; -1 = none) instead of
    // its points' labels (none were appended).  Nothing to do without rows.
    __device__ void add_end_labels(int ml, int mf) {
        if (skip || nR == 0) return;
        const int addl = ml >= 0 ? 1 : 0, addf = (mf >= 0 && mf != ml) ? 1 : 0;
        if (lane_id() == 0) {
            if (addl) labs[nL] = (uint32_t)ml;
            if (addf) labs[nL + addl] = (uint32_t)mf;
        }
        nL += addl + addf;
    }

    // Appends the candidates of the lanes in cR (rows) and cM (labels); false when a list is full.
    __device__ bool append(uint64_t cR, int r, uint64_t cM, int m) {
        const int addR = __popcll(cR), addM = __popcll(cM);
        if (nR + addR > RCAP || nL + addM > LCAP) return false;
        if (in_mask(cR)) rows[nR + mbcnt(cR)] = (uint32_t)r;
        if (in_mask(cM)) labs[nL + mbcnt(cM)] = (uint32_t)m;
        nR += addR;
        nL += addM;
        return true;
    }

    __device__ static uint32_t slot_of(uint32_t key) {
        return (key ^ (key >> 9) ^ (key >> 18) ^ (key >> 27)) & (TCAP - 1);
    }
    // Inserts the key of every lane in `cand`; returns the lanes whose key was new (slot set).
    // The lanes still probing are a wave-uniform mask; the outcome ballots count those lanes only
    // (a lane outside `cand` may hold any value as its key).  Each lane's slot ends where its key
    // was found or put.
    __device__ uint64_t insert(uint64_t cand, uint32_t key, uint32_t &slot) const {
        uint64_t act = cand, fresh = 0ull;
        uint32_t h = slot_of(key);
        while (act) {
            uint32_t old = 0u;
            if (in_mask(act)) {
                old = atomicCAS(&tab[h], kEmpty, key);
                slot = h;
            }
            const uint64_t got = __ballot(old == kEmpty) & act, dup = __ballot(old == key) & act;
            fresh |= got;
            act &= ~(got | dup);
            h = (h + 1u) & (TCAP - 1);
        }
        return fresh;
    }

    // The streamline ends: C(i, m) += 1 for each distinct row i and distinct label m, then reset.
    template <typename Sink>
    __device__ void close(Sink &sink, uint32_t si, uint32_t sm) {
        if (!skip && nR > 0 && nL > 0) {
            const int lane = lane_id();
            int nU = 0;
            // (lane conditions as wave-uniform masks throughout: no per-lane booleans carried
            // across loads and loops)
            for (int b = 0; b < nL; b += kWave) {
                const int k = b + lane;
                const uint64_t ok = __ballot(k < nL);
                const uint32_t m = in_mask(ok) ? labs[k] : 0u;
                uint32_t slot = 0;
                const uint64_t fresh = insert(ok, m | kLabelTag, slot);
                if (in_mask(fresh)) ulab[nU + mbcnt(fresh)] = m;
                if (in_mask(ok)) labs[k] = in_mask(fresh) ? slot : kEmpty;
                nU += __popcll(fresh);
            }
            const float rcp = 1.0f / (float)nU;
            for (int b = 0; b < nR; b += kWave) {
                const int k = b + lane;
                const uint64_t ok = __ballot(k < nR);
                const uint32_t i = in_mask(ok) ? rows[k] : 0u;
                uint32_t slot = 0;
                const uint64_t fresh = insert(ok, i, slot);
                if (in_mask(ok)) rows[k] = in_mask(fresh) ? slot : kEmpty;
                // the nF new rows x the nU distinct labels, 64 pairs per push.  The new rows move to
                // lanes 0 .. nF-1 (a permutation of all 64 lanes: the others fill nF .. 63); pair q is
                // row q / nU and label q % nU.  q < 4096, so the float quotient is at most one low,
                // and only at exact multiples of nU.
                const int nF = __popcll(fresh);
                if (nF == 0) continue;
                const int to = in_mask(fresh) ? mbcnt(fresh) : nF + mbcnt(~fresh);
                const int frow = __builtin_amdgcn_ds_permute(to << 2, (int)(i * si));   // N*M < 2^31
                const int tot = nF * nU;
                for (int q0 = 0; q0 < tot; q0 += kWave) {
                    const int q = q0 + lane;
                    const uint64_t live = __ballot(q < tot);
                    int rq = (int)((float)q * rcp);
                    rq += (rq + 1) * nU <= q ? 1 : 0;
                    const int uq = q - rq * nU;
                    const uint32_t row = (uint32_t)__builtin_amdgcn_ds_bpermute((in_mask(live) ? rq : 0) << 2, frow);
                    const uint32_t lab = ulab[in_mask(live) ? uq : 0];
                    sink.push_lanes(live, row + lab * sm);
                }
            }
            for (int k = lane; k < nL; k += kWave)
                if (labs[k] != kEmpty) tab[labs[k]] = kEmpty;
            for (int k = lane; k < nR; k += kWave)
                if (rows[k] != kEmpty) tab[rows[k]] = kEmpty;
        }
        nR = nL = 0;
        skip = false;
    }
};

// Queue entries: point index in bits 0..47, subject in bits 48..62.
constexpr int kSubjectShift = 48;
__device__ __forceinline__ void push_overflow(const Overflow &o, int64_t point_index, int32_t subject = 0) {
    if (lane_id() == 0) {
        const unsigned long long k = atomicAdd(o.count, 1ull);
        if ((int64_t)k < o.cap) o.list[k] = point_index | ((int64_t)subject << kSubjectShift);
    }
}

// ---------------------------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------------------------

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *__restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

static int fill_blocks(int64_t n, int cus) {
    int64_t b = (n + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cus * 16;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, int cus, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<fill_blocks(n, cus), kBlock, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, int cus, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<fill_blocks(n, cus), kBlock, 0, st>>>(p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// compact volume build
// ---------------------------------------------------------------------------------------------

// Occupancy word (index into the {word, base} pairs) and bit of voxel lin; false when the voxel
// is not occupied (0 <= roi < N or 0 <= lab < M).
__device__ __forceinline__ bool occupancy_bit(int32_t lin, int32_t r, int32_t m, const Grid &g, int32_t N, int32_t M,
                                              int32_t SBX, int32_t SBXY, uint32_t &word, uint32_t &bit) {
    if (!((unsigned)r < (unsigned)N || (unsigned)m < (unsigned)M)) return false;
    const int32_t t = lin / g.X;
    const int x = lin - t * g.X;
    const int y = t % g.Y;
    const int z = t / g.Y;
    const uint32_t sb = (uint32_t)(x >> 4) + (uint32_t)SBX * (uint32_t)(y >> 3) + (uint32_t)SBXY * (uint32_t)(z >> 3);
    const uint32_t b = (uint32_t)(x & 15) | ((uint32_t)(y & 7) << 4) | ((uint32_t)(z & 7) << 7);
    word = (sb << 5) | (b >> 5);
    bit = 1u << (b & 31u);
    return true;
}

// Sets the occupancy bit of voxel lin.
__device__ __forceinline__ void mark_voxel(int32_t lin, int32_t r, int32_t m, const Grid &g, int32_t N, int32_t M,
                                           int32_t SBX, int32_t SBXY, uint32_t *mb) {
    uint32_t w, bit;
    if (occupancy_bit(lin, r, m, g, N, M, SBX, SBXY, w, bit)) atomicOr(&mb[2 * w], bit);
}

// Sets the occupancy bits of voxels lin0 .. lin0+3 with one atomic per run of them in one word
// (four neighbours along x share a word unless a row or a 16-voxel run ends among them).
__device__ __forceinline__ void mark_voxels4(int32_t lin0, const int32_t (&r)[4], const int32_t (&m)[4], const Grid &g,
                                             int32_t N, int32_t M, int32_t SBX, int32_t SBXY, uint32_t *mb) {
    uint32_t word = 0u, bits = 0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t w, bit;
        if (occupancy_bit(lin0 + q, r[q], m[q], g, N, M, SBX, SBXY, w, bit)) {
            if (bits && w != word) {
                atomicOr(&mb[2 * word], bits);
                bits = 0u;
            }
            word = w;
            bits |= bit;
        }
    }
    if (bits) atomicOr(&mb[2 * word], bits);
}

// One pass over both volumes (X*Y*Z < 2^31): four voxels per thread and step with 16-byte loads
// when both volumes are 16-byte aligned (VEC), else one.
template <bool VEC>
__global__ void k_compact_mark(const int32_t *__restrict__ roi, const int32_t *__restrict__ lab, Grid g,
                               int32_t N, int32_t M, int32_t SBX, int32_t SBXY, uint32_t *__restrict__ mb) {
    const int32_t nvox = g.X * g.Y * g.Z;
    const int32_t stride = gridDim.x * blockDim.x;
    if (VEC) {
        const int32_t n4 = nvox >> 2;
        typedef int32_t v4i __attribute__((ext_vector_type(4)));
        const v4i *r4 = reinterpret_cast<const v4i *>(roi);
        const v4i *m4 = reinterpret_cast<const v4i *>(lab);
        // two groups of loads in flight before any mark: the marks are atomics, and on this
        // architecture a wait for a later load also waits for every earlier atomic
        for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += 2 * stride) {
            const int32_t i2 = i + stride;
            const v4i r = __builtin_nontemporal_load(r4 + i), m = __builtin_nontemporal_load(m4 + i);
            v4i r2 = {-1, -1, -1, -1}, m2 = {-1, -1, -1, -1};
            if (i2 < n4) {
                r2 = __builtin_nontemporal_load(r4 + i2);
                m2 = __builtin_nontemporal_load(m4 + i2);
            }
            {
                const int32_t ra[4] = {r.x, r.y, r.z, r.w}, ma[4] = {m.x, m.y, m.z, m.w};
                mark_voxels4(4 * i, ra, ma, g, N, M, SBX, SBXY, mb);
            }
            {
                const int32_t ra[4] = {r2.x, r2.y, r2.z, r2.w}, ma[4] = {m2.x, m2.y, m2.z, m2.w};
                mark_voxels4(4 * i2, ra, ma, g, N, M, SBX, SBXY, mb);
            }
        }
        for (int32_t lin = 4 * n4 + blockIdx.x * blockDim.x + threadIdx.x; lin < nvox; lin += stride)
            mark_voxel(lin, roi[lin], lab[lin], g, N, M, SBX, SBXY, mb);
    } else {
        for (int32_t lin = blockIdx.x * blockDim.x + threadIdx.x; lin < nvox; lin += stride)
            mark_voxel(lin, roi[lin], lab[lin], g, N, M, SBX, SBXY, mb);
    }
}

// inclusive scan of one value per thread over a 256-thread block; returns the block total in `total`
__device__ uint32_t block_scan_incl(uint32_t v, uint32_t *lds4, uint32_t &total) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    if (lane == kWave - 1) lds4[w] = v;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += lds4[k];
    total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
    __syncthreads();
    return v + before;
}

constexpr int kWordsPerThread = kScanTile / kBlock;  // 8

// Popcount of each kScanTile-word tile.  With `brick_coarse` (a coarse map of one bit per 16x8x8
// super-brick, 32 words each) it also writes the map: tile b is super-bricks 64b .. 64b+63, words
// 2b and 2b+1 of the map, four threads per super-brick.
__global__ void k_compact_tile_sums(const uint32_t *__restrict__ mb, int64_t W, uint32_t *__restrict__ tile_sums,
                                    uint32_t *__restrict__ brick_coarse) {
    static_assert(kScanTile == 64 * 32 && kWordsPerThread * 4 == 32, "a tile is 64 super-bricks, 4 threads each");
    __shared__ uint32_t lds4[4];
    __shared__ uint32_t bits16[4];
    const int64_t w0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kWordsPerThread;
    uint32_t s = 0, any = 0;
    for (int k = 0; k < kWordsPerThread; ++k)
        if (w0 + k < W) {
            const uint32_t wd = mb[2 * (w0 + k)];
            s += __popc(wd);
            any |= wd;
        }
    if (brick_coarse) {
        // lanes 4q .. 4q+3 of a wavefront cover super-brick q of its 16
        uint64_t occ = __ballot(any != 0u);
        occ |= occ >> 1;
        occ |= occ >> 2;
        uint32_t b16 = 0u;
        for (int q = 0; q < 16; ++q) b16 |= (uint32_t)((occ >> (4 * q)) & 1ull) << q;
        if ((threadIdx.x & 63) == 0) bits16[threadIdx.x >> 6] = b16;
    }
    uint32_t total;
    block_scan_incl(s, lds4, total);   // (its barriers also publish bits16)
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
    if (brick_coarse && threadIdx.x < 2)
        brick_coarse[2 * blockIdx.x + threadIdx.x] = bits16[2 * threadIdx.x] | (bits16[2 * threadIdx.x + 1] << 16);
}

// one block: exclusive scan of the tile sums in place
__global__ void k_compact_scan_tiles(uint32_t *__restrict__ tile_sums, int64_t ntiles) {
    __shared__ uint32_t lds4[4];
    uint32_t carry = 0;
    for (int64_t a = 0; a < ntiles; a += kBlock) {
        const int64_t i = a + threadIdx.x;
        const uint32_t v = i < ntiles ? tile_sums[i] : 0u;
        uint32_t total;
        const uint32_t incl = block_scan_incl(v, lds4, total);
        if (i < ntiles) tile_sums[i] = carry + incl - v;
        carry += total;
    }
}

// Rank base of every occupancy word: the number of occupied voxels in the words before it.
// Rank bases of tile b's words.  kSumTiles: tile_base holds the tiles' popcounts, and the workgroup
// sums those before b itself (for up to kBasesSumTiles tiles); else tile_base holds their scan.
constexpr int64_t kBasesSumTiles = 1024;
template <bool kSumTiles>
__global__ void k_compact_bases(uint32_t *__restrict__ mb, const uint32_t *__restrict__ tile_base, int64_t W) {
    __shared__ uint32_t lds4[4];
    uint32_t tbase;
    if (kSumTiles) {
        uint32_t part = 0u;
        for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += blockDim.x) part += tile_base[t];
        block_scan_incl(part, lds4, tbase);   // tbase = the sum over the workgroup
    } else {
        tbase = tile_base[blockIdx.x];
    }
    const int64_t w0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kWordsPerThread;
    uint32_t words[kWordsPerThread];
    uint32_t s = 0;
    for (int k = 0; k < kWordsPerThread; ++k) {
        words[k] = (w0 + k < W) ? mb[2 * (w0 + k)] : 0u;
        s += __popc(words[k]);
    }
    uint32_t total;
    uint32_t run = tbase + block_scan_incl(s, lds4, total) - s;
    for (int k = 0; k < kWordsPerThread; ++k) {
        if (w0 + k >= W) break;
        mb[2 * (w0 + k) + 1] = run;
        run += __popc(words[k]);
    }
}

// Codes of the occupied voxels, in rank order.  A wavefront takes 64 words at a time and fills the
// occupied ones two by two: word w covers x in [16 sbx, 16 sbx + 16) of rows y and y + 1 (y even) of
// one z, so its 32 lanes read two runs of 16 consecutive voxels.
// Occupancy words per wavefront group of the code fill: small, so that a solidly occupied region
// (an ROI, a whole group of occupied words) is spread over many wavefronts.
constexpr int kFillGroup = 16;

template <bool PACKED>
__global__ void k_compact_fill_codes(const uint32_t *__restrict__ mb, int64_t W, const int32_t *__restrict__ roi,
                                     const int32_t *__restrict__ lab, Grid g, CompactVol cv, int32_t SBY,
                                     void *__restrict__ codes) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t grp = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6); grp * kFillGroup < W;
         grp += nwaves) {
        // lanes 0 .. kFillGroup-1 read the group's words; lane k then names word k in the loop below
        const int64_t w = grp * kFillGroup + lane;
        uint32_t word = 0u, base = 0u;
        if (lane < kFillGroup && w < W) {
            word = mb[2 * w];
            base = mb[2 * w + 1];
        }
        uint64_t todo = __ballot(word != 0u);
        while (todo) {
            const int ka = __builtin_ctzll(todo);
            todo &= todo - 1ull;
            const int kb = todo ? __builtin_ctzll(todo) : ka;   // second word of the pair (or the first again)
            if (todo) todo &= todo - 1ull;
            const bool upper = lane >= 32;
            const int k = upper ? kb : ka;
            const uint32_t wda = (uint32_t)__builtin_amdgcn_readlane((int)word, ka);
            const uint32_t wdb = (uint32_t)__builtin_amdgcn_readlane((int)word, kb);
            const uint32_t bsa = (uint32_t)__builtin_amdgcn_readlane((int)base, ka);
            const uint32_t bsb = (uint32_t)__builtin_amdgcn_readlane((int)base, kb);
            const uint32_t wd = upper ? wdb : wda, bs = upper ? bsb : bsa;
            const uint32_t j = (uint32_t)lane & 31u;
            if (((wd >> j) & 1u) && !(upper && kb == ka)) {
                const uint32_t ww = (uint32_t)(grp * kFillGroup + k);
                const uint32_t sb = ww >> 5, wl = ww & 31u;
                const uint32_t b = (wl << 5) | j;
                const int x = (int)(sb % (uint32_t)cv.SBX) * 16 + (int)(b & 15u);
                const int y = (int)((sb / (uint32_t)cv.SBX) % (uint32_t)SBY) * 8 + (int)((b >> 4) & 7u);
                const int z = (int)(sb / (uint32_t)cv.SBXY) * 8 + (int)(b >> 7);
                const int64_t lin = (int64_t)x + (int64_t)g.X * ((int64_t)y + (int64_t)g.Y * z);
                const int32_t r = roi[lin], m = lab[lin];
                const bool rv = (unsigned)r < (unsigned)cv.N, mv = (unsigned)m < (unsigned)cv.M;
                const uint32_t at = bs + __popc(wd & ((1u << j) - 1u));
                if (PACKED) {
                    const uint32_t rf = rv ? (uint32_t)r : cv.rmask;
                    const uint32_t mf = mv ? (uint32_t)m : (0xFFFFFFFFu >> cv.rbits);
                    static_cast<uint32_t *>(codes)[at] = rf | (mf << cv.rbits);
                } else {
                    static_cast<int2 *>(codes)[at] = make_int2(rv ? r : -1, mv ? m : -1);
                }
            }
        }
    }
}

// Coarse occupancy: bit of block (cx, cy, cz) of side 2^cs is set iff an occupancy word covering
// it has a bit inside it.  One thread per block, 64 blocks per wavefront packed with a ballot.
__global__ void k_compact_coarse(const uint32_t *__restrict__ mb, int32_t SBX, int32_t SBY, int32_t SBZ, int32_t csx,
                                 int32_t csyz, int32_t CBX, int32_t CBY, int32_t CBZ, uint32_t *__restrict__ coarse) {
    const int64_t ncb = (int64_t)CBX * CBY * CBZ;
    const int64_t cb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool occ = false;
    if (cb < ncb) {
        const int cx = (int)(cb % CBX);
        const int64_t t = cb / CBX;
        const int cy = (int)(t % CBY), cz = (int)(t / CBY);
        if (csx == 3) {
            // half of one 16x8x8 super-brick: x in [0,8) are bits 0-7 and 16-23 of each word
            const uint32_t half = (cx & 1) ? 0xFF00FF00u : 0x00FF00FFu;
            const int64_t sb = (cx >> 1) + (int64_t)SBX * (cy + (int64_t)SBY * cz);
            for (int wl = 0; wl < 32; ++wl) occ |= (mb[2 * (sb * 32 + wl)] & half) != 0u;
        } else {
            // whole super-bricks: 1 << (csx - 4) in x, 1 << (csyz - 3) in y and z
            const int fx = 1 << (csx - 4), fyz = 1 << (csyz - 3);
            for (int sz = cz * fyz; sz < (cz + 1) * fyz && sz < SBZ; ++sz)
                for (int sy = cy * fyz; sy < (cy + 1) * fyz && sy < SBY; ++sy)
                    for (int sx = cx * fx; sx < (cx + 1) * fx && sx < SBX; ++sx) {
                        const int64_t sb = sx + (int64_t)SBX * (sy + (int64_t)SBY * sz);
                        for (int wl = 0; wl < 32; ++wl) occ |= mb[2 * (sb * 32 + wl)] != 0u;
                    }
        }
    }
    const uint64_t bits = __ballot(occ);
    const int64_t w = cb >> 6;   // this wavefront's 64 blocks
    if ((threadIdx.x & 63) == 0) {
        coarse[2 * w] = (uint32_t)bits;
        coarse[2 * w + 1] = (uint32_t)(bits >> 32);
    }
}

hipError_t launch_compact_build(const int32_t *roi, const int32_t *lab, Grid g, int32_t N, int32_t M, CompactVol cv,
                                uint32_t *mb, void *codes, uint32_t *tile_sums, uint32_t *coarse, int64_t W, int cus,
                                hipStream_t st) {
    const int64_t ntiles = (W + kScanTile - 1) / kScanTile;
    const int32_t SBY = cv.SBXY / cv.SBX;
    k_fill_i32<<<fill_blocks(2 * W, cus), kBlock, 0, st>>>(reinterpret_cast<int32_t *>(mb), 2 * W, 0);
    const int64_t nvox = (int64_t)g.X * g.Y * g.Z;
    const bool vec = ((reinterpret_cast<uintptr_t>(roi) | reinterpret_cast<uintptr_t>(lab)) & 15u) == 0;
    if (vec) k_compact_mark<true><<<fill_blocks(nvox / 4, cus * 2), kBlock, 0, st>>>(roi, lab, g, N, M, cv.SBX, cv.SBXY, mb);
    else k_compact_mark<false><<<fill_blocks(nvox, cus * 2), kBlock, 0, st>>>(roi, lab, g, N, M, cv.SBX, cv.SBXY, mb);
    // the brick layout's coarse map (one bit per super-brick) comes from the tile sums pass
    const bool brick = cv.csx == 4 && cv.csyz == 3;
    k_compact_tile_sums<<<(unsigned)ntiles, kBlock, 0, st>>>(mb, W, tile_sums, brick ? coarse : nullptr);
    if (ntiles <= kBasesSumTiles) {
        k_compact_bases<true><<<(unsigned)ntiles, kBlock, 0, st>>>(mb, tile_sums, W);
    } else {
        k_compact_scan_tiles<<<1, kBlock, 0, st>>>(tile_sums, ntiles);
        k_compact_bases<false><<<(unsigned)ntiles, kBlock, 0, st>>>(mb, tile_sums, W);
    }
    const int64_t groups = (W + kFillGroup - 1) / kFillGroup;
    const unsigned fblocks = (unsigned)std::min<int64_t>((groups + kWavesPerBlock - 1) / kWavesPerBlock, (int64_t)cus * 8);
    if (cv.packed) k_compact_fill_codes<true><<<fblocks, kBlock, 0, st>>>(mb, W, roi, lab, g, cv, SBY, codes);
    else k_compact_fill_codes<false><<<fblocks, kBlock, 0, st>>>(mb, W, roi, lab, g, cv, SBY, codes);
    const int32_t SBZ = (int32_t)(W / 32 / cv.SBXY);
    const int32_t CBY = (g.Y + (1 << cv.csyz) - 1) >> cv.csyz, CBZ = (g.Z + (1 << cv.csyz) - 1) >> cv.csyz;
    const int64_t nthreads = (int64_t)cv.ncoarse_words * 32;
    if (!brick)
        k_compact_coarse<<<(unsigned)((nthreads + kBlock - 1) / kBlock), kBlock, 0, st>>>(
            mb, cv.SBX, SBY, SBZ, cv.csx, cv.csyz, cv.CBX, CBY, CBZ, coarse);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// partition: first[i] = first streamline starting at or after point floor(i * P / nparts),
// first[nparts] = S, with P = offsets[S] read on the device (launches stay asynchronous)
// ---------------------------------------------------------------------------------------------

__global__ void k_partition(const int64_t *__restrict__ offsets, int64_t S, int64_t nparts, int32_t *__restrict__ first,
                            ZeroRanges z, int taper) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int r = 0; r < 2; ++r)
        for (int64_t i = t0; i < z.n32[r]; i += stride) z.w32[r][i] = 0;
    for (int64_t i = t0; i < z.n64; i += stride) z.w64[i] = 0ull;
    int64_t P = offsets[S];
    if (P < 0) P = 0;
    for (int64_t i = t0; i <= nparts; i += stride) {
        if (i == nparts) {
            first[i] = (int32_t)S;
            continue;
        }
        // range i starts at the streamline holding point P * g(i / nparts).  Equal ranges: g(x) = x.
        // Tapered: g(x) = 1.5 x - 0.5 x^2, the ranges shrinking linearly from 1.5x to 0.5x the mean
        // in the order they are handed out, so that the last ones to start end close together.
        const int64_t target =
            taper ? (int64_t)(((__int128)P * i * (3 * nparts - i)) / ((__int128)2 * nparts * nparts))
                  : (int64_t)(((__int128)i * P) / nparts);
        int64_t lo = 0, hi = S;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (offsets[mid] < target) lo = mid + 1;
            else hi = mid;
        }
        first[i] = (int32_t)lo;
    }
}

hipError_t launch_partition(const int64_t *offsets, int64_t S, int64_t nparts, int32_t *first, const ZeroRanges &z,
                            bool taper, int cus, hipStream_t st) {
    const int64_t n = std::max<int64_t>(std::max<int64_t>(nparts + 1, z.n64), std::max(z.n32[0], z.n32[1]));
    k_partition<<<fill_blocks(n, cus), kBlock, 0, st>>>(offsets, S, nparts, first, z, taper ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// count, variant 1: one wavefront per streamline, raster lookups
// ---------------------------------------------------------------------------------------------

constexpr int kMaxUp = 4;   // largest upsampling factor

template <bool SCALED>
__global__ void __launch_bounds__(kBlock) k_count_wave(CountArgs a, RasterVol rv) {
    __shared__ uint32_t s_tab[kWavesPerBlock * kSetCap];
    __shared__ uint32_t s_slots[kWavesPerBlock * (kSetCap / 2)];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    WaveSet<kSetCap> set;
    set.init(s_tab + wv * kSetCap, s_slots + wv * (kSetCap / 2));
    DirectSink sink{a.C};
    const int64_t Ptot = a.offsets[a.S] > 0 ? a.offsets[a.S] : 0;
    const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
    const bool endmode = a.ends.mode != 0;   // endpoint modes: labels come from a.ends at the close
    const int up = a.up < 1 ? 1 : (a.up > kMaxUp ? kMaxUp : a.up);   // upsampling factor
    for (int64_t s = (int64_t)blockIdx.x * kWavesPerBlock + wv; s < a.S; s += nw) {
        const int64_t b0 = clamp64(a.offsets[s], 0, Ptot);
        const int64_t b1 = clamp64(a.offsets[s + 1], b0, Ptot);
        int last_r = -1, last_m = -1;
        for (int64_t w0 = b0; w0 < b1; w0 += kWave) {
            const int64_t p = w0 + lane;
            const bool here = p < b1, next = p + 1 < b1;
            // the lane's scaled point and (upsampling) the step to the next one
            float qx = 0.f, qy = 0.f, qz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f;
            if (here) {
                qx = load_stream(a.pts + 3 * p);
                qy = load_stream(a.pts + 3 * p + 1);
                qz = load_stream(a.pts + 3 * p + 2);
                if (SCALED) {
                    qx = __fmul_rn(qx, a.scale);
                    qy = __fmul_rn(qy, a.scale);
                    qz = __fmul_rn(qz, a.scale);
                }
                if (up > 1 && next) {
                    float ux = a.pts[3 * p + 3], uy = a.pts[3 * p + 4], uz = a.pts[3 * p + 5];
                    if (SCALED) {
                        ux = __fmul_rn(ux, a.scale);
                        uy = __fmul_rn(uy, a.scale);
                        uz = __fmul_rn(uz, a.scale);
                    }
                    dx = __fsub_rn(ux, qx);
                    dy = __fsub_rn(uy, qy);
                    dz = __fsub_rn(uz, qz);
                }
            }
            // sub-point t: the point itself (t = 0) or a_t of the way to the next one
            int rr[kMaxUp], mm[kMaxUp];
#pragma unroll
            for (int t = 0; t < kMaxUp; ++t) {
                rr[t] = mm[t] = -1;
                if (t < up && here && (t == 0 || next)) {
                    float x = qx, y = qy, z = qz;
                    if (t > 0) {
                        const float at = (float)((double)t / (double)up);
                        x = __fadd_rn(qx, __fmul_rn(at, dx));
                        y = __fadd_rn(qy, __fmul_rn(at, dy));
                        z = __fadd_rn(qz, __fmul_rn(at, dz));
                    }
                    int ix, iy, iz, r, m;
                    if (voxelise<false>(x, y, z, 1.0f, a.g, ix, iy, iz)) {
                        raster_get(rv, ix, iy, iz, r, m);
                        rr[t] = r;
                        mm[t] = endmode ? -1 : m;
                    }
                }
            }
            int rl = rr[0], ml = mm[0];   // the lane's last sub-point
#pragma unroll
            for (int t = 1; t < kMaxUp; ++t)
                if (t == up - 1) {
                    rl = rr[t];
                    ml = mm[t];
                }
            // drop a hit equal to the hit before it in streamline order, then the LDS set
            int rp = __shfl_up(rl, 1), mp = __shfl_up(ml, 1);
            if (lane == 0) {
                rp = last_r;
                mp = last_m;
            }
            last_r = __shfl(rl, kWave - 1);
            last_m = __shfl(ml, kWave - 1);
#pragma unroll
            for (int t = 0; t < kMaxUp; ++t) {
                if (t >= up) break;
                const int pr = t == 0 ? rp : rr[t > 0 ? t - 1 : 0], pm = t == 0 ? mp : mm[t > 0 ? t - 1 : 0];
                const uint64_t candR = __ballot(rr[t] >= 0 && rr[t] != pr);
                const uint64_t candM = __ballot(mm[t] >= 0 && mm[t] != pm);
                if ((candR | candM) == 0ull || set.skip) continue;
                if (!set.add(candR, rr[t], candM, mm[t])) {
                    push_overflow(a.ovf, b0);
                    set.clear_entries();
                    set.skip = true;
                }
            }
        }
        if (endmode && !set.skip && set.nI > 0) {
            const int ml = a.ends.last[s], mf = a.ends.mode == 2 ? a.ends.first[s] : -1;
            const uint64_t cand = __ballot((lane == 0 && ml >= 0) || (lane == 1 && mf >= 0 && mf != ml));
            if (cand && !set.add(0ull, 0, cand, lane == 0 ? ml : mf)) {
                push_overflow(a.ovf, b0);
                set.clear_entries();
                set.skip = true;
            }
        }
        set.close(sink, a.si, a.sm);
    }
}

hipError_t launch_count_wave(const CountArgs &a, const RasterVol &rv, int blocks, hipStream_t st) {
    if (a.scale != 1.0f) k_count_wave<true><<<blocks, kBlock, 0, st>>>(a, rv);
    else k_count_wave<false><<<blocks, kBlock, 0, st>>>(a, rv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// count, variant 2: flat point stream over ranges of whole streamlines
// ---------------------------------------------------------------------------------------------
//
// Wavefront w owns the streamlines [first[w], first[w+1]): one contiguous range of about P/W
// points.  It walks the range in batches of kBatch 64-point windows regardless of streamline
// boundaries.  Per batch: voxelise, occupancy-bit gathers (a 2-3 MB structure that stays in L2),
// and for the few flagged lanes the rank and code gathers; only then are the next batch's
// streaming loads issued (vector loads return in issue order, so no gather wait of this batch
// covers them), and the windows are folded into the open streamline's LDS set while they are in
// flight.  The streamline starts inside a window come from a block of 64 offsets held one per
// lane; each start closes the open streamline.
//
// All global reads go through buffer resources: out-of-range offsets read zero instead of
// faulting, so the point stream needs no per-lane clamping (lanes past the range are masked by
// their index) and a lane's load offset is one constant register plus a scalar batch offset.

constexpr uint32_t kRsrcWord3 = 0x00020000u;   // raw 32-bit buffer, gfx9-family descriptor
constexpr int kAuxStream = 2;                  // non-temporal: points are read once
constexpr int kAuxCached = 0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint64_t bytes) {
    const uint32_t n = bytes > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, (int)kRsrcWord3);
}

__device__ __forceinline__ uint32_t fbits(float f) { return __float_as_uint(f); }

// wave-uniform copies (the values are uniform already; this tells the compiler)
__device__ __forceinline__ int uniform32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t readlane64(int64_t v, int k) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), k);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A wave-uniform read of memory that no launch in flight writes (the end labels, filled by an
// earlier launch), through the scalar data cache: a vector load would make the wavefront wait for
// every gather and point load it has in flight, as vector-memory loads complete in issue order.
__device__ __forceinline__ int32_t uniform_const_load(const int32_t *p, int64_t i) {
    return ((const __attribute__((address_space(4))) int32_t *)p)[i];
}

// Next point range (work item) of wavefront `wave`: queue c = wave mod Q holds ranges c, c + Q,
// c + 2Q, ..., handed out in that order by its own counter (Q: kRangeQueues, or the largest power of
// two not above the grid's wavefronts, so that every queue has wavefronts).
__device__ __forceinline__ int64_t next_range(const Overflow &ovf, uint32_t wave) {
    const uint32_t nw = gridDim.x * (uint32_t)kWavesPerBlock;
    const uint32_t q = nw >= (uint32_t)kRangeQueues ? (uint32_t)kRangeQueues : (1u << (31 - __builtin_clz(nw)));
    const uint32_t c = wave & (q - 1u);
    // (the range index is formed in lane 0 and broadcast: forming it from the broadcast count
    // costs the surrounding loop about 20 vector registers)
    unsigned long long t = 0;
    if (lane_id() == 0) t = (unsigned long long)c + (unsigned long long)q * atomicAdd(ovf.work + (size_t)c * kQueueWords, 1ull);
    return uniform64((int64_t)t);
}

constexpr int kRCap = 192, kLCap = 64, kTCap = 512;   // per-wave candidate lists and set
constexpr int64_t kMaxRangePoints = int64_t(1) << 28;  // longest point range the flat-stream loop takes
constexpr int kSetWords = kRCap + 2 * kLCap + kTCap;
using StreamSet = DeferredSet<kRCap, kLCap, kTCap>;

// Counts streamlines [s0, s1) of one subject (whole streamlines only) into sub.C through `sink`.
// `coarse` is the subject's coarse occupancy map in LDS.  PACKED: 0/1 = code width known at compile
// time, 2 = read from cv.packed.
template <bool SCALED, int PACKED, int kBatch, bool kEnds, int kUp, bool kBrick, typename Sink>
__device__ void stream_range(const StreamSubject &sub, const uint32_t *coarse, int64_t s0, int64_t s1, int32_t subject,
                             const Overflow &ovf, StreamSet &set, Sink &sink) {
    constexpr int kV = kBatch * kUp;   // lookups per batch: kUp sub-points of each of kBatch windows
    const int lane = lane_id();
    const CompactVol &cv = sub.cv;
    const int64_t S = sub.S;
    const auto offs = gview(sub.offsets);
    const int64_t Ptot = uniform64(offs[S] > 0 ? offs[S] : 0);
    // occupancy pairs and codes share one allocation and one resource (codes at cv.codes_off)
    const __amdgpu_buffer_rsrc_t rvol = make_rsrc(cv.mb, cv.span);
    const int codes_off = uniform32((int)cv.codes_off);
    const uint32_t lane12 = 12u * (uint32_t)lane;
    // the grid bounds live in VGPRs: as scalars they crowd out the loop's lane masks
    uint32_t bX = fbits(sub.g.Xf), bY = fbits(sub.g.Yf), bZ = fbits(sub.g.Zf);
    asm volatile("" : "+v"(bX), "+v"(bY), "+v"(bZ));
    const uint32_t SBX = (uint32_t)cv.SBX, SBXY = (uint32_t)cv.SBXY;
    const uint32_t csx = (uint32_t)cv.csx, csyz = (uint32_t)cv.csyz, CBX = (uint32_t)cv.CBX, CBXY = (uint32_t)cv.CBXY;
    constexpr uint32_t kOutOfRange = 0xFFFFFFF8u;   // buffer offset past every resource: reads 0, no traffic
    const int64_t P0 = uniform64(clamp64(offs[s0], 0, Ptot));
    const int64_t P1 = uniform64(clamp64(offs[s1], P0, Ptot));
    if (P0 >= P1) return;
    if (P1 - P0 > kMaxRangePoints) {
        // positions below are 32-bit offsets from P0: a range this long (a few giant streamlines
        // make one) goes to the fallback kernel, one entry per non-empty streamline
        for (int64_t s = s0; s < s1; ++s) {
            const int64_t b = uniform64(clamp64(offs[s], P0, P1));
            const int64_t e = uniform64(clamp64(offs[s + 1], b, P1));
            if (e > b) push_overflow(ovf, b, subject);
        }
        return;
    }
    const uint32_t L = (uint32_t)(P1 - P0);   // points of the range; positions are relative to P0
    // endpoint modes (kEnds instantiations only): no point contributes its label; each closing
    // streamline gets its end labels
    const bool endmode = kEnds && uniform32(sub.ends.mode) != 0;
    // upsampling (kUp > 1 instantiations): sub-point t = 1 .. up-1 of a point lies a_t = fl32(t/up)
    // of the way to the next point of its streamline, in scaled coordinates
    const int up = kUp > 1 ? uniform32(sub.up) : 1;
    float at[kUp];
#pragma unroll
    for (int t = 0; t < kUp; ++t) at[t] = (float)((double)t / (double)up);
    // Starts of streamlines s0+1 .. s1-1 (relative to P0), 64 at a time, one per lane (L = "no
    // more starts"); k0 of them are consumed and `nxt` (uniform) is the next unconsumed start.
    int64_t vb = s0 + 1;
    uint32_t voff = 0, nxt = L;
    int k0 = 0;
    auto load_starts = [&]() {
        voff = (vb + lane < s1) ? (uint32_t)(clamp64(offs[vb + lane], P0, P1) - P0) : L;
        k0 = 0;
        nxt = (uint32_t)__builtin_amdgcn_readlane((int)voff, 0);
    };
    auto consumed = [&](uint64_t taken) {
        k0 += __popcll(taken);
        if (k0 >= kWave) {
            vb += kWave;
            load_starts();
        } else {
            nxt = (uint32_t)__builtin_amdgcn_readlane((int)voff, k0);
        }
    };
    // starts in [wb, wend) (wend <= wb + 64) as lane bits relative to wb; consumes them.  `mult`
    // (endpoint modes) counts the streamlines starting at each lane: empty streamlines share a start.
    auto take_starts = [&](uint32_t wb, uint32_t wend, int &mult) -> uint64_t {
        uint64_t starts = 0;
        while (nxt < wend) {
            const uint64_t inwin = __ballot(lane >= k0) & __ballot(voff < wend);
            const uint32_t qv = min(voff - wb, (uint32_t)(kWave - 1));   // lane of the start (in-window lanes)
            uint64_t it = inwin;
            while (it) {
                const int k = __builtin_ctzll(it);
                it &= it - 1ull;
                const int q = __builtin_amdgcn_readlane((int)qv, k);
                starts |= 1ull << q;
                if (endmode) mult += lane == q ? 1 : 0;
            }
            consumed(inwin);
        }
        return starts;
    };
    auto skip_starts = [&](uint32_t limit) {
        while (nxt < limit) consumed(__ballot(lane >= k0) & __ballot(voff < limit));
    };
    load_starts();
    // the open streamline is vb - 1 + k0: the last one whose start has been consumed
    auto close_open = [&](int64_t id) {
        if (endmode) {
            id = id < s0 ? s0 : (id >= s1 ? s1 - 1 : id);
            set.add_end_labels(uniform_const_load(sub.ends.last, id), sub.ends.mode == 2 ? uniform_const_load(sub.ends.first, id) : -1);
        }
        set.close(sink, sub.si, sub.sm);
    };
    int last_r = -1, last_m = -1;
    // points [P0, P1): loads at or past the range's end read zero without memory traffic, so the
    // next batch can always be issued
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(sub.pts + 3 * P0, 12ull * L);
    constexpr uint32_t BW = kWave * kBatch;   // points per batch

    // one register set of points: the lookup stage of a batch consumes it, and the points of the
    // batch after next are then loaded into it (see the pipeline below)
    // kUp > 1: each lane also holds the next point (the same load one point further on: it hits
    // the lines the window itself brings in)
    constexpr int kNext = kUp > 1 ? kBatch : 1;
    float ax[kBatch], ay[kBatch], az[kBatch], nx[kNext], ny[kNext], nz[kNext];
    auto load_batch = [&](uint32_t w) {
        const uint32_t so = 12u * w;
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b96(rp, lane12, so + 768u * b, kAuxStream);
            ax[b] = __uint_as_float(v[0]);
            ay[b] = __uint_as_float(v[1]);
            az[b] = __uint_as_float(v[2]);
        }
        if (kUp > 1) {
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b96(rp, lane12 + 12u, so + 768u * b, kAuxCached);
                nx[b] = __uint_as_float(v[0]);
                ny[b] = __uint_as_float(v[1]);
                nz[b] = __uint_as_float(v[2]);
            }
        }
    };
    // Lookup stage of the batch at w0 (its points are in ax.. / nx..): gather offsets and bit
    // indices.
    auto lookup = [&](uint32_t w0, uint32_t (&addr)[kV], uint32_t (&bix)[kV]) {
        const uint32_t left = w0 < L ? L - w0 : 0u;
        const int rem = left > BW ? (int)BW : (int)left;          // valid points in this batch
        const int remn = left > BW ? (int)BW + 1 : (int)left;     // lane + 1 < remn: a next point exists
        // voxelise and test the coarse occupancy bit in LDS; only lookups in occupied coarse
        // blocks gather their occupancy word and rank base (8 bytes): the others read past the
        // resource (zero, no traffic), so the gathered word alone decides the hit.  Lookup
        // v = b*kUp + t is sub-point t of window b.
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            float qx = ax[b], qy = ay[b], qz = az[b];
            if (SCALED) {
                qx = __fmul_rn(qx, sub.scale);
                qy = __fmul_rn(qy, sub.scale);
                qz = __fmul_rn(qz, sub.scale);
            }
            float dx = 0.f, dy = 0.f, dz = 0.f;
            if (kUp > 1) {
                float mx = nx[b], my = ny[b], mz = nz[b];
                if (SCALED) {
                    mx = __fmul_rn(mx, sub.scale);
                    my = __fmul_rn(my, sub.scale);
                    mz = __fmul_rn(mz, sub.scale);
                }
                dx = __fsub_rn(mx, qx);
                dy = __fsub_rn(my, qy);
                dz = __fsub_rn(mz, qz);
            }
#pragma unroll
            for (int t = 0; t < kUp; ++t) {
                const int v = b * kUp + t;
                float x = qx, y = qy, z = qz;
                if (t > 0) {
                    x = __fadd_rn(qx, __fmul_rn(at[t], dx));
                    y = __fadd_rn(qy, __fmul_rn(at[t], dy));
                    z = __fadd_rn(qz, __fmul_rn(at[t], dz));
                }
                const float tx = __fadd_rn(x, 0.5f), ty = __fadd_rn(y, 0.5f), tz = __fadd_rn(z, 0.5f);
                // 0 <= t < bound  <=>  bits(t) < bits(bound) as unsigned (t is never -0; NaN and
                // negative values compare above every finite positive bound)
                // (bitwise & throughout: no short-circuit branches)
                const int valid = t == 0 ? (int)(lane + b * kWave < rem) : (int)(t < up) & (int)(lane + b * kWave + 1 < remn);
                const bool ok = valid & (int)(fbits(tx) < bX) & (int)(fbits(ty) < bY) & (int)(fbits(tz) < bZ);
                const uint32_t ix = (uint32_t)(int)tx, iy = (uint32_t)(int)ty, iz = (uint32_t)(int)tz;
                uint32_t sb = __umul24(iz >> 3, SBXY) + __umul24(iy >> 3, SBX) + (ix >> 4);
                asm("" : "+v"(sb));   // keeps the 24-bit multiplies: (sb << 8) must not fold into them
                // coarse block: the super-brick itself (kBrick: the volume's map is per super-brick)
                // or a cube of 8, 16 or 32
                const uint32_t cb = kBrick ? sb : __umul24(iz >> csyz, CBXY) + __umul24(iy >> csyz, CBX) + (ix >> csx);
                const uint32_t cw = coarse[ok ? (cb >> 5) : 0u];
                const bool hit = (int)ok & (int)(__builtin_amdgcn_ubfe(cw, cb, 1) != 0u);   // bfe: offset mod 32
                // byte offset of the (word, base) pair: 32 words of 16x2x1 voxels per super-brick,
                // word (y/2 mod 4) + 4 (z mod 8), bit (x mod 16) + 16 (y mod 2)
                addr[v] = hit ? (sb << 8) | ((iy << 2) & 0x18u) | ((iz << 5) & 0xE0u) : kOutOfRange;
                bix[v] = (ix & 15u) | ((iy & 1u) << 4);
            }
        }
    };
    // (word, base) pairs of a batch's lookups.  Always issued: lanes that failed the coarse test
    // read past the resource (zero, no traffic), so every path through the loop issues the same
    // vector-memory sequence and each wait covers exactly what it needs.
    auto gather_pairs = [&](const uint32_t (&addr)[kV], uint32_t (&mw)[kV], uint32_t (&base)[kV]) {
#pragma unroll
        for (int v = 0; v < kV; ++v) {
            const auto e = __builtin_amdgcn_raw_buffer_load_b64(rvol, addr[v], 0, kAuxCached);
            mw[v] = e[0];
            base[v] = e[1];
        }
    };
    // The rest of a batch once its codes are in: candidates, streamline starts and closes.
    auto tail = [&](uint32_t w0, const int (&r)[kV], const int (&m)[kV], const bool (&flag)[kV]) {
        uint64_t fl[kBatch];
        uint64_t fall = 0;
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            fl[b] = 0ull;
#pragma unroll
            for (int t = 0; t < kUp; ++t) fl[b] |= __ballot(flag[b * kUp + t]);
            fall |= fl[b];
        }
        if (fall == 0ull) {
            // nothing looked up: only a streamline start inside the batch matters (it closes the
            // open streamline, whose hits all came earlier)
            const uint32_t bend = (w0 + BW < L) ? w0 + BW : L;
            if (nxt < bend) {
                if (set.has_state()) close_open(vb - 1 + k0);
                skip_starts(bend);
            }
            last_r = last_m = -1;
            return;
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const uint32_t wb = w0 + (uint32_t)b * kWave;
            if (wb >= L) break;
            const uint32_t wend = (wb + kWave < L) ? wb + kWave : L;
            // streamline starts inside this window -> bit q of `starts` for lane q
            const int64_t id0 = vb - 1 + k0;   // the streamline open at the window's first point
            int mult = 0;
            const uint64_t starts = (nxt < wend) ? take_starts(wb, wend, mult) : 0ull;
            if (fl[b] == 0ull) {
                if (starts && set.has_state()) close_open(id0);
                last_r = last_m = -1;
                continue;
            }
            // sub-points t >= 1 exist only where the next point continues the lane's streamline:
            // not before a start, not at the range's end
            uint64_t nextok = ~0ull;
            if (kUp > 1) {
                uint64_t brk = starts >> 1;
                if (wb + kWave >= L || nxt == wb + kWave) brk |= 1ull << (kWave - 1);
                const uint32_t lastp = L - 1 - wb;   // lane of the range's last point
                if (lastp < (uint32_t)kWave) brk |= ~0ull << lastp;
                nextok = ~brk;
            }
            int rr[kUp], mm[kUp];
#pragma unroll
            for (int t = 0; t < kUp; ++t) {
                const bool ok = t == 0 || in_mask(nextok);
                rr[t] = ok ? r[b * kUp + t] : -1;
                mm[t] = (ok && !endmode) ? m[b * kUp + t] : -1;
            }
            // each lane's last counted sub-point (t = up - 1) precedes the next lane's point
            int rl = rr[0], ml = mm[0];
#pragma unroll
            for (int t = 1; t < kUp; ++t)
                if (t == up - 1) {
                    rl = rr[t];
                    ml = mm[t];
                }
            // drop a hit equal to the hit just before it in streamline order: sub-point 0 against
            // the previous lane's last sub-point (lane 0: the previous window's), t >= 1 against t - 1
            int rp_ = __builtin_amdgcn_update_dpp(last_r, rl, 0x138, 0xF, 0xF, false);   // wave_shr:1
            int mp_ = __builtin_amdgcn_update_dpp(last_m, ml, 0x138, 0xF, 0xF, false);
            if (in_mask(starts)) rp_ = mp_ = -1;  // first point of a streamline
            uint64_t candR[kUp], candM[kUp];
            // (one ballot per comparison: each compare writes its lane mask directly)
            candR[0] = __ballot(rr[0] >= 0) & __ballot(rr[0] != rp_);
            candM[0] = __ballot(mm[0] >= 0) & __ballot(mm[0] != mp_);
#pragma unroll
            for (int t = 1; t < kUp; ++t) {
                candR[t] = __ballot(rr[t] >= 0) & __ballot(rr[t] != rr[t - 1]);
                candM[t] = __ballot(mm[t] >= 0) & __ballot(mm[t] != mm[t - 1]);
            }
            last_r = __builtin_amdgcn_readlane(rl, kWave - 1);
            last_m = __builtin_amdgcn_readlane(ml, kWave - 1);
            // the candidates of the lanes in `seg` into the open streamline's set
            auto add = [&](uint64_t seg, uint32_t at) {
#pragma unroll
                for (int t = 0; t < kUp; ++t) {
                    const uint64_t cR = candR[t] & seg, cM = candM[t] & seg;
                    if ((cR | cM) && !set.skip && !set.append(cR, rr[t], cM, mm[t])) {
                        push_overflow(ovf, P0 + (int64_t)at, subject);
                        set.nR = set.nL = 0;
                        set.skip = true;
                    }
                }
            };
            if (!starts) {   // the whole window belongs to the open streamline
                add(~0ull, wb);
                continue;
            }
            int pos = 0;
            int64_t id = id0;
            uint64_t st = starts;
            for (;;) {
                const int end = st ? __builtin_ctzll(st) : kWave;
                add(lanes_between(pos, end), wb + pos);
                if (!st) break;
                close_open(id);
                if (endmode) id += __builtin_amdgcn_readlane(mult, end);
                pos = end;
                st &= st - 1ull;
            }
        }
    };
    // Software pipeline over batches k: the pair gathers of batch k + 1 are in flight while batch k's
    // codes return and its tail runs.  Vector-memory loads complete in issue order, so each
    // iteration issues: the codes of k, the pairs of k + 1, the points of k + 2; batch k's decode
    // then waits for its codes only, and the next iteration's flags for the pairs of k + 1 only.
    const bool packed = PACKED == 1 || (PACKED == 2 && cv.packed);
    const uint32_t code_oob = kOutOfRange - (uint32_t)codes_off;   // with the code offset: past the resource
    uint32_t bix[kV], mw[kV], rank[kV];
    {
        uint32_t addr[kV];
        load_batch(0u);
        lookup(0u, addr, bix);
        __builtin_amdgcn_sched_barrier(0);
        gather_pairs(addr, mw, rank);
        __builtin_amdgcn_sched_barrier(0);
        load_batch(BW);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (uint32_t w0 = 0; w0 < L; w0 += BW) {
        // flags of batch k and its code gathers (unflagged lanes read past the resource)
        bool flag[kV];
#pragma unroll
        for (int v = 0; v < kV; ++v) flag[v] = __builtin_amdgcn_ubfe(mw[v], bix[v], 1) != 0u;
        uint32_t c0[kV], c1[kV];
#pragma unroll
        for (int v = 0; v < kV; ++v) {
            const uint32_t at = rank[v] + __popc(__builtin_amdgcn_ubfe(mw[v], 0, bix[v]));
            if (packed) {
                c0[v] = __builtin_amdgcn_raw_buffer_load_b32(rvol, flag[v] ? at << 2 : code_oob, codes_off, kAuxCached);
                c1[v] = 0u;
            } else {
                const auto c2 = __builtin_amdgcn_raw_buffer_load_b64(rvol, flag[v] ? at << 3 : code_oob, codes_off,
                                                                     kAuxCached);
                c0[v] = c2[0];
                c1[v] = c2[1];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // lookups and pair gathers of batch k + 1 (its points arrived during the last iteration),
        // then the points of batch k + 2 into the registers the lookups just freed
        uint32_t bix2[kV], mw2[kV], rank2[kV];
        {
            uint32_t addr[kV];
            lookup(w0 + BW, addr, bix2);
            __builtin_amdgcn_sched_barrier(0);
            gather_pairs(addr, mw2, rank2);
        }
        __builtin_amdgcn_sched_barrier(0);
        load_batch(w0 + 2 * BW);
        __builtin_amdgcn_sched_barrier(0);
        // codes of batch k
        int r[kV], m[kV];
#pragma unroll
        for (int v = 0; v < kV; ++v) {
            if (packed) {
                const uint32_t rv = c0[v] & cv.rmask, mv = c0[v] >> cv.rbits;
                r[v] = (flag[v] && rv < (uint32_t)cv.N) ? (int)rv : -1;
                m[v] = (flag[v] && mv < (uint32_t)cv.M) ? (int)mv : -1;
            } else {
                r[v] = flag[v] ? (int)c0[v] : -1;
                m[v] = flag[v] ? (int)c1[v] : -1;
            }
        }
        tail(w0, r, m, flag);
#pragma unroll
        for (int v = 0; v < kV; ++v) {
            bix[v] = bix2[v];
            mw[v] = mw2[v];
            rank[v] = rank2[v];
        }
    }
    close_open(vb - 1 + k0);
}

// The flat-stream kernel's body: ranges from this wavefront's queue, pair updates through its
// append sink.
template <bool SCALED, bool PACKED, int kBatch, bool kEnds, bool kBrick>
__device__ __forceinline__ void count_stream_body(const StreamSubject &sub, const Overflow &ovf,
                                                  const int32_t *__restrict__ first, int64_t nparts, const PairOut &po) {
    // 4-window batches run 6 wavefronts per SIMD (their scalar registers), so they can afford the
    // LDS of 512 buffered updates; 2-window batches keep 8 per SIMD with 256
    constexpr int kSinkCap = kBatch == 4 ? 8 * kWave : 4 * kWave;
    __shared__ uint32_t s_set[kWavesPerBlock * kSetWords];
    __shared__ __align__(16) uint32_t s_pend[kWavesPerBlock * kSinkCap];
    extern __shared__ uint32_t s_coarse[];   // coarse occupancy bit map, cv.ncoarse_words words
    const int wv = uniform32(threadIdx.x >> 6);
    for (int k = threadIdx.x; k < sub.cv.ncoarse_words; k += blockDim.x) s_coarse[k] = sub.cv.coarse[k];
    __syncthreads();
    StreamSet set;
    set.init(s_set + wv * kSetWords);
    const uint32_t wave = blockIdx.x * kWavesPerBlock + wv;
    AppendSink<kSinkCap> sink;
    sink.init(s_pend + wv * kSinkCap, sub.C, po, wave);
    for (;;) {
        // next point range: streamlines [first[part], first[part+1])
        const int64_t part = next_range(ovf, wave);
        if (part >= nparts) break;
        const int64_t s0 = uniform64(clamp64(first[part], 0, sub.S));
        const int64_t s1 = uniform64(clamp64(first[part + 1], s0, sub.S));
        if (s0 >= s1) continue;
        stream_range<SCALED, PACKED ? 1 : 0, kBatch, kEnds, 1, kBrick>(sub, s_coarse, s0, s1, 0, ovf, set, sink);
    }
    sink.drain(po, wave);
}

// Two-window batches (the short-call schedule) need few vector registers; with at most 80 scalar
// registers a SIMD holds 8 of these wavefronts.  (Each wavefront's scalar allocation is its count
// rounded up to 16, plus 16 more: 800 / (96 + 16) = 7 wavefronts at 81..96 registers, 6 above that.)
template <bool SCALED, bool PACKED, bool kEnds, bool kBrick>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_num_sgpr(80)))
k_count_stream2(StreamSubject sub, Overflow ovf, const int32_t *__restrict__ first, int64_t nparts, PairOut po) {
    count_stream_body<SCALED, PACKED, 2, kEnds, kBrick>(sub, ovf, first, nparts, po);
}

template <bool SCALED, bool PACKED, bool kEnds, bool kBrick>
__global__ void __launch_bounds__(kBlock)
k_count_stream4(StreamSubject sub, Overflow ovf, const int32_t *__restrict__ first, int64_t nparts, PairOut po) {
    count_stream_body<SCALED, PACKED, 4, kEnds, kBrick>(sub, ovf, first, nparts, po);
}

// Upsampled pass-through (up = 2 .. kUp): the scale is always applied (multiplying by 1.0f is
// exact) and the code width is read from the volume, so two instantiations cover every case.
template <int kUp>
__global__ void __launch_bounds__(kBlock) k_count_stream_up(StreamSubject sub, Overflow ovf,
                                                            const int32_t *__restrict__ first, int64_t nparts, PairOut po) {
    constexpr int kB = kUp == 2 ? 2 : 1;   // kB * kUp lookups per batch, as the plain kernel's 4
    constexpr int kSinkCap = 4 * kWave;
    __shared__ uint32_t s_set[kWavesPerBlock * kSetWords];
    __shared__ __align__(16) uint32_t s_pend[kWavesPerBlock * kSinkCap];
    extern __shared__ uint32_t s_coarse[];
    const int wv = uniform32(threadIdx.x >> 6);
    for (int k = threadIdx.x; k < sub.cv.ncoarse_words; k += blockDim.x) s_coarse[k] = sub.cv.coarse[k];
    __syncthreads();
    StreamSet set;
    set.init(s_set + wv * kSetWords);
    const uint32_t wave = blockIdx.x * kWavesPerBlock + wv;
    AppendSink<kSinkCap> sink;
    sink.init(s_pend + wv * kSinkCap, sub.C, po, wave);
    for (;;) {
        const int64_t part = next_range(ovf, wave);
        if (part >= nparts) break;
        const int64_t s0 = uniform64(clamp64(first[part], 0, sub.S));
        const int64_t s1 = uniform64(clamp64(first[part + 1], s0, sub.S));
        if (s0 >= s1) continue;
        stream_range<true, 2, kB, false, kUp, false>(sub, s_coarse, s0, s1, 0, ovf, set, sink);
    }
    sink.drain(po, wave);
}

// Batched form: work items (subject, first streamline) from every subject, handed out by one
// counter; each wavefront keeps the coarse map of the subject it last worked on in its own LDS.
// The scale is always applied (multiplying by 1.0f is exact), the code width is read per subject.
// One instantiation per kind of subject: pass-through (kEnds false, kUp 1), the endpoint modes
// (kEnds: labels from sub.ends at each close), and upsampled pass-through (kUp 2 or 4, with
// sub.up <= kUp); a launch takes the items of subjects of one kind only.
template <int kBatch, bool kEnds, int kUp>
__global__ void __launch_bounds__(kBlock) k_count_batched(const StreamSubject *__restrict__ subs,
                                                          const int2 *__restrict__ items, int64_t nitems,
                                                          Overflow ovf, int32_t coarse_words) {
    __shared__ uint32_t s_set[kWavesPerBlock * kSetWords];
    __shared__ uint32_t s_pend[kWavesPerBlock * kWave];
    extern __shared__ uint32_t s_coarse[];   // kWavesPerBlock * coarse_words
    const int lane = lane_id(), wv = uniform32(threadIdx.x >> 6);
    uint32_t *coarse = s_coarse + wv * coarse_words;
    StreamSet set;
    set.init(s_set + wv * kSetWords);
    // updates go to C as atomics: with many hits per point, this form's cost is the hit processing
    BufferedSink sink;
    sink.init(s_pend + wv * kWave, nullptr);
    int loaded = -1;
    const uint32_t wave = blockIdx.x * kWavesPerBlock + wv;
    for (;;) {
        const int64_t item = next_range(ovf, wave);
        if (item >= nitems) break;
        const int2 it = items[item];
        const int subject = uniform32(it.x);
        const StreamSubject &sub = subs[subject];
        const int64_t s0 = uniform64(clamp64(it.y, 0, sub.S));
        int64_t s1 = sub.S;
        if (item + 1 < nitems) {
            const int2 nx = items[item + 1];
            if (nx.x == subject) s1 = nx.y;
        }
        s1 = uniform64(clamp64(s1, s0, sub.S));
        if (s0 >= s1) continue;
        if (subject != loaded) {
            for (int k = lane; k < sub.cv.ncoarse_words; k += kWave) coarse[k] = gview(sub.cv.coarse)[k];
            loaded = subject;
        }
        sink.C = sub.C;
        stream_range<true, 2, kBatch, kEnds, kUp, false>(sub, coarse, s0, s1, subject, ovf, set, sink);
        sink.drain();   // the next item may belong to another subject's C
    }
}

template <bool SCALED, bool PACKED, int B, bool E>
static int blocks_per_cu_of(size_t dyn) {
    const void *fn = B == 2 ? reinterpret_cast<const void *>(&k_count_stream2<SCALED, PACKED, E, true>)
                            : reinterpret_cast<const void *>(&k_count_stream4<SCALED, PACKED, E, true>);
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kBlock, dyn);
    return (e == hipSuccess && n > 0) ? n : 4;
}

template <int B, bool E>
static int blocks_per_cu_b(bool scaled, bool packed, size_t dyn) {
    if (scaled) return packed ? blocks_per_cu_of<true, true, B, E>(dyn) : blocks_per_cu_of<true, false, B, E>(dyn);
    return packed ? blocks_per_cu_of<false, true, B, E>(dyn) : blocks_per_cu_of<false, false, B, E>(dyn);
}

template <int U>
static int blocks_per_cu_up(size_t dyn) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, reinterpret_cast<const void *>(&k_count_stream_up<U>), kBlock, dyn);
    return (e == hipSuccess && n > 0) ? n : 4;
}

int count_stream_blocks_per_cu(bool scaled, bool packed, int batch, bool ends, int up, size_t dyn) {
    if (up > 1) return up == 2 ? blocks_per_cu_up<2>(dyn) : blocks_per_cu_up<4>(dyn);
    if (ends) return batch == 2 ? blocks_per_cu_b<2, true>(scaled, packed, dyn) : blocks_per_cu_b<4, true>(scaled, packed, dyn);
    return batch == 2 ? blocks_per_cu_b<2, false>(scaled, packed, dyn) : blocks_per_cu_b<4, false>(scaled, packed, dyn);
}

static StreamSubject stream_subject(const CountArgs &a, const CompactVol &cv) {
    StreamSubject s;
    s.pts = a.pts;
    s.offsets = a.offsets;
    s.S = a.S;
    s.s_begin = 0;
    s.g = a.g;
    s.scale = a.scale;
    s.cv = cv;
    s.C = a.C;
    s.si = a.si;
    s.sm = a.sm;
    s.ends = a.ends;
    s.up = a.up;
    return s;
}

template <int B, bool E, bool K>
static void launch_stream_bk(const CountArgs &a, const CompactVol &cv, const int32_t *first, int64_t nparts, int blocks,
                             const PairOut &po, hipStream_t st) {
    const bool scaled = a.scale != 1.0f;
    const size_t dyn = 4 * (size_t)cv.ncoarse_words;
    const StreamSubject sub = stream_subject(a, cv);
#define FC_LAUNCH_STREAM(S_, P_)                                                                               \
    do {                                                                                                       \
        if (B == 2) k_count_stream2<S_, P_, E, K><<<blocks, kBlock, dyn, st>>>(sub, a.ovf, first, nparts, po); \
        else k_count_stream4<S_, P_, E, K><<<blocks, kBlock, dyn, st>>>(sub, a.ovf, first, nparts, po);       \
    } while (0)
    if (scaled && cv.packed) FC_LAUNCH_STREAM(true, true);
    else if (scaled) FC_LAUNCH_STREAM(true, false);
    else if (cv.packed) FC_LAUNCH_STREAM(false, true);
    else FC_LAUNCH_STREAM(false, false);
#undef FC_LAUNCH_STREAM
}

// the super-brick coarse map (csx 4, csyz 3) has its own instantiations
template <int B, bool E>
static void launch_stream_b(const CountArgs &a, const CompactVol &cv, const int32_t *first, int64_t nparts, int blocks,
                            const PairOut &po, hipStream_t st) {
    if (cv.csx == 4 && cv.csyz == 3) launch_stream_bk<B, E, true>(a, cv, first, nparts, blocks, po, st);
    else launch_stream_bk<B, E, false>(a, cv, first, nparts, blocks, po, st);
}

hipError_t launch_count_stream(const CountArgs &a, const CompactVol &cv, const int32_t *first, int64_t nparts,
                               int blocks, int batch, const PairOut &po, hipStream_t st) {
    if (a.up > 1) {
        const size_t dyn = 4 * (size_t)cv.ncoarse_words;
        const StreamSubject sub = stream_subject(a, cv);
        if (a.up == 2) k_count_stream_up<2><<<blocks, kBlock, dyn, st>>>(sub, a.ovf, first, nparts, po);
        else k_count_stream_up<4><<<blocks, kBlock, dyn, st>>>(sub, a.ovf, first, nparts, po);
        return hipGetLastError();
    }
    const bool ends = a.ends.mode != 0;
    if (batch == 2) {
        if (ends) launch_stream_b<2, true>(a, cv, first, nparts, blocks, po, st);
        else launch_stream_b<2, false>(a, cv, first, nparts, blocks, po, st);
    } else {
        if (ends) launch_stream_b<4, true>(a, cv, first, nparts, blocks, po, st);
        else launch_stream_b<4, false>(a, cv, first, nparts, blocks, po, st);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// fallback for overflowed streamlines: one workgroup per queued streamline, global bit maps
// ---------------------------------------------------------------------------------------------

// One overflowed streamline (the one containing point p), counted by a whole workgroup with the
// workgroup's all-zero scratch: a bit map over rows, one over labels and a list of the labels.
// Sub-point k of the streamline [b0, b1) upsampled by `up` (0 <= k < (b1 - b0 - 1) * up + 1):
// point j = b0 + k / up itself when t = k % up is 0, else the point a_t = fl32(t / up) of the way to
// point j + 1, in scaled coordinates.  False when it has no voxel.
template <typename Lookup, bool SCALED>
__device__ bool sub_lookup(const float *__restrict__ pts, int64_t b0, int64_t k, int up, float scale, const Grid &g,
                           const Lookup &lk, int &r, int &m) {
    const int64_t j = b0 + k / up;
    const int t = (int)(k % up);
    float x = pts[3 * j], y = pts[3 * j + 1], z = pts[3 * j + 2];
    if (SCALED) {
        x = __fmul_rn(x, scale);
        y = __fmul_rn(y, scale);
        z = __fmul_rn(z, scale);
    }
    if (t > 0) {
        float ux = pts[3 * j + 3], uy = pts[3 * j + 4], uz = pts[3 * j + 5];
        if (SCALED) {
            ux = __fmul_rn(ux, scale);
            uy = __fmul_rn(uy, scale);
            uz = __fmul_rn(uz, scale);
        }
        const float a = (float)((double)t / (double)up);
        x = __fadd_rn(x, __fmul_rn(a, __fsub_rn(ux, x)));
        y = __fadd_rn(y, __fmul_rn(a, __fsub_rn(uy, y)));
        z = __fadd_rn(z, __fmul_rn(a, __fsub_rn(uz, z)));
    }
    int ix, iy, iz;
    if (!voxelise<false>(x, y, z, 1.0f, g, ix, iy, iz)) return false;
    lk.get(ix, iy, iz, r, m);
    return true;
}

constexpr int kFallbackCached = 4;   // sub-points per thread whose lookup is kept for the later passes

template <typename Lookup, bool SCALED>
__device__ void fallback_streamline(const float *__restrict__ pts, const int64_t *__restrict__ offsets, int64_t S,
                                    const Grid &g, float scale, const Lookup &lk, int32_t *__restrict__ C, uint32_t si,
                                    uint32_t sm, int64_t p, uint32_t *bmN, uint32_t *bmM, uint32_t *labels,
                                    int *s_nlab, const EndLabels &ends, int up) {
    const int64_t Ptot = offsets[S] > 0 ? offsets[S] : 0;
    // streamline containing point p: the last s with offsets[s] <= p.  The offsets never decrease,
    // so of blockDim.x evenly spaced candidates the ones at or below p are a prefix of the threads,
    // and their count narrows [lo, hi) blockDim.x-fold per round (3 rounds for 5M streamlines).
    int64_t lo = 0, hi = S;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + blockDim.x - 1) / blockDim.x;
        const int64_t idx = lo + (int64_t)threadIdx.x * step;
        const int at_or_below = (threadIdx.x > 0 && idx < hi && offsets[idx] <= p) ? 1 : 0;
        lo += (int64_t)__syncthreads_count(at_or_below) * step;
        hi = min(hi, lo + step);
    }
    const int64_t b0 = clamp64(offsets[lo], 0, Ptot);
    const int64_t b1 = clamp64(offsets[lo + 1], b0, Ptot);
    const int64_t nsub = b1 > b0 ? (b1 - b0 - 1) * up + 1 : 0;   // points after upsampling
    if (threadIdx.x == 0) *s_nlab = 0;
    // each sub-point is looked up once: thread t's sub-points t + j * blockDim.x, j < kFallbackCached,
    // keep (r, m) in registers for the three passes; the rest (streamlines of more than
    // kFallbackCached * blockDim.x sub-points) are looked up again in each pass.  -1: none.
    int cr[kFallbackCached], cm[kFallbackCached];
#pragma unroll
    for (int j = 0; j < kFallbackCached; ++j) {
        const int64_t k = threadIdx.x + (int64_t)j * blockDim.x;
        int r = -1, m = -1;
        if (k >= nsub || !sub_lookup<Lookup, SCALED>(pts, b0, k, up, scale, g, lk, r, m)) r = m = -1;
        cr[j] = r;
        cm[j] = m;
    }
    const int64_t k_rest = threadIdx.x + (int64_t)kFallbackCached * blockDim.x;
    auto lookup_rest = [&](int64_t k, int &r, int &m) {
        if (!sub_lookup<Lookup, SCALED>(pts, b0, k, up, scale, g, lk, r, m)) r = m = -1;
    };
    __syncthreads();
    // endpoint modes: the labels are the streamline's end labels
    if (ends.mode != 0 && threadIdx.x == 0) {
        const int ml = ends.last[lo], mf = ends.mode == 2 ? ends.first[lo] : -1;
        int n = 0;
        if (ml >= 0) atomicExch(&labels[n++], (uint32_t)ml);
        if (mf >= 0 && mf != ml) atomicExch(&labels[n++], (uint32_t)mf);
        *s_nlab = n;
    }
    // distinct labels
    auto add_label = [&](int m) {
        if (m >= 0) {
            const uint32_t bitm = 1u << (m & 31);
            if (!(atomicOr(&bmM[m >> 5], bitm) & bitm)) {
                const int k = atomicAdd(s_nlab, 1);
                atomicExch(&labels[k], (uint32_t)m);
            }
        }
    };
    if (ends.mode == 0) {
#pragma unroll
        for (int j = 0; j < kFallbackCached; ++j) add_label(cm[j]);
        for (int64_t k = k_rest; k < nsub; k += blockDim.x) {
            int r, m;
            lookup_rest(k, r, m);
            add_label(m);
        }
    }
    __syncthreads();
    const int nlab = *s_nlab;
    // distinct rows: the first claimant of each row adds its pairs
    auto add_row = [&](int r) {
        if (r >= 0) {
            const uint32_t bitr = 1u << (r & 31);
            if (!(atomicOr(&bmN[r >> 5], bitr) & bitr)) {
                int32_t *row = C + (uint32_t)r * si;
                for (int k = 0; k < nlab; ++k)
                    atomicAdd(row + __hip_atomic_load(&labels[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) * sm, 1);
            }
        }
    };
    if (nlab > 0) {
#pragma unroll
        for (int j = 0; j < kFallbackCached; ++j) add_row(cr[j]);
        for (int64_t k = k_rest; k < nsub; k += blockDim.x) {
            int r, m;
            lookup_rest(k, r, m);
            add_row(r);
        }
    }
    __syncthreads();
    // restore the all-zero scratch (bit maps and label list)
    auto clear = [&](int r, int m) {
        if (r >= 0) atomicExch(&bmN[r >> 5], 0u);
        if (m >= 0) atomicExch(&bmM[m >> 5], 0u);
    };
#pragma unroll
    for (int j = 0; j < kFallbackCached; ++j) clear(cr[j], cm[j]);
    for (int64_t k = k_rest; k < nsub; k += blockDim.x) {
        int r, m;
        lookup_rest(k, r, m);
        clear(r, m);
    }
    for (int k = threadIdx.x; k < nlab; k += blockDim.x) atomicExch(&labels[k], 0u);
    __syncthreads();
}

constexpr int64_t kPointMask = (int64_t(1) << kSubjectShift) - 1;

template <typename Lookup, bool SCALED>
__global__ void __launch_bounds__(kBlock) k_fallback(CountArgs a, Lookup lk, FallbackScratch fs) {
    __shared__ int s_nlab;
    uint32_t *bmN = fs.words + (int64_t)blockIdx.x * fs.stride;
    uint32_t *bmM = bmN + fs.nwordsN;
    uint32_t *labels = bmM + fs.nwordsM;
    const int64_t nq = (int64_t)*a.ovf.count;
    const int64_t nq_c = nq < a.ovf.cap ? nq : a.ovf.cap;
    for (int64_t q = blockIdx.x; q < nq_c; q += gridDim.x)
        fallback_streamline<Lookup, SCALED>(a.pts, a.offsets, a.S, a.g, a.scale, lk, a.C, a.si, a.sm,
                                            a.ovf.list[q] & kPointMask, bmN, bmM, labels, &s_nlab, a.ends, a.up);
}

// Batched fallback: the queue entry names its subject.
__global__ void __launch_bounds__(kBlock) k_fallback_batched(const StreamSubject *__restrict__ subs, int32_t nsub,
                                                             Overflow ovf, FallbackScratch fs) {
    __shared__ int s_nlab;
    uint32_t *bmN = fs.words + (int64_t)blockIdx.x * fs.stride;
    uint32_t *bmM = bmN + fs.nwordsN;
    uint32_t *labels = bmM + fs.nwordsM;
    const int64_t nq = (int64_t)*ovf.count;
    const int64_t nq_c = nq < ovf.cap ? nq : ovf.cap;
    for (int64_t q = blockIdx.x; q < nq_c; q += gridDim.x) {
        const int64_t e = ovf.list[q];
        int32_t subject = (int32_t)(e >> kSubjectShift);
        subject = subject < 0 ? 0 : (subject >= nsub ? nsub - 1 : subject);
        const StreamSubject &sub = subs[subject];
        fallback_streamline<CompactLookup, true>(sub.pts, sub.offsets, sub.S, sub.g, sub.scale, CompactLookup{sub.cv},
                                                 sub.C, sub.si, sub.sm, e & kPointMask, bmN, bmM, labels, &s_nlab,
                                                 sub.ends, sub.up);
    }
}

// ---------------------------------------------------------------------------------------------
// endpoint modes: per-streamline end labels; Alg. 1's seed-to-endpoint count
// ---------------------------------------------------------------------------------------------

template <typename Lookup, bool SCALED>
__device__ __forceinline__ void lookup_point(const float *p, float scale, const Grid &g, const Lookup &lk, int &r,
                                             int &m) {
    int ix, iy, iz;
    r = m = -1;
    if (voxelise<SCALED>(p[0], p[1], p[2], scale, g, ix, iy, iz)) lk.get(ix, iy, iz, r, m);
}

// last[s] = label of streamline s's last point, first[s] (mode 2) = label of its first point; -1
// for an empty streamline or a point without a label.  One thread per streamline.
template <typename Lookup, bool SCALED>
__global__ void k_end_labels(CountArgs a, Lookup lk, int32_t mode, int32_t *__restrict__ last,
                             int32_t *__restrict__ first) {
    const int64_t Ptot = a.offsets[a.S] > 0 ? a.offsets[a.S] : 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.S; s += stride) {
        const int64_t b0 = clamp64(a.offsets[s], 0, Ptot);
        const int64_t b1 = clamp64(a.offsets[s + 1], b0, Ptot);
        int r, ml = -1, mf = -1;
        if (b1 > b0) {
            lookup_point<Lookup, SCALED>(a.pts + 3 * (b1 - 1), a.scale, a.g, lk, r, ml);
            if (mode == 2) lookup_point<Lookup, SCALED>(a.pts + 3 * b0, a.scale, a.g, lk, r, mf);
        }
        last[s] = ml;
        if (mode == 2) first[s] = mf;
    }
}

// C(row of the first point, label of the last point) += 1 per streamline (the seed is the first
// point).  One thread per streamline.
template <typename Lookup, bool SCALED>
__global__ void k_count_seed_end(CountArgs a, Lookup lk) {
    const int64_t Ptot = a.offsets[a.S] > 0 ? a.offsets[a.S] : 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.S; s += stride) {
        const int64_t b0 = clamp64(a.offsets[s], 0, Ptot);
        const int64_t b1 = clamp64(a.offsets[s + 1], b0, Ptot);
        if (b1 <= b0) continue;
        int r, m, r2, m2;
        lookup_point<Lookup, SCALED>(a.pts + 3 * b0, a.scale, a.g, lk, r, m);
        lookup_point<Lookup, SCALED>(a.pts + 3 * (b1 - 1), a.scale, a.g, lk, r2, m2);
        if (r >= 0 && m2 >= 0) atomicAdd(a.C + (uint32_t)r * a.si + (uint32_t)m2 * a.sm, 1);
    }
}

template <typename Lookup>
static void launch_end_labels_l(const CountArgs &a, const Lookup &lk, int mode, int32_t *last, int32_t *first,
                                int cus, hipStream_t st) {
    const unsigned blocks = fill_blocks(a.S, cus);
    if (a.scale != 1.0f) k_end_labels<Lookup, true><<<blocks, kBlock, 0, st>>>(a, lk, mode, last, first);
    else k_end_labels<Lookup, false><<<blocks, kBlock, 0, st>>>(a, lk, mode, last, first);
}

hipError_t launch_end_labels(const CountArgs &a, const RasterVol *rv, const CompactVol *cv, int mode, int32_t *last,
                             int32_t *first, int cus, hipStream_t st) {
    if (a.S <= 0) return hipSuccess;
    if (rv) launch_end_labels_l(a, RasterLookup{*rv}, mode, last, first, cus, st);
    else launch_end_labels_l(a, CompactLookup{*cv}, mode, last, first, cus, st);
    return hipGetLastError();
}

template <typename Lookup>
static void launch_seed_end_l(const CountArgs &a, const Lookup &lk, int cus, hipStream_t st) {
    const unsigned blocks = fill_blocks(a.S, cus);
    if (a.scale != 1.0f) k_count_seed_end<Lookup, true><<<blocks, kBlock, 0, st>>>(a, lk);
    else k_count_seed_end<Lookup, false><<<blocks, kBlock, 0, st>>>(a, lk);
}

hipError_t launch_count_seed_end(const CountArgs &a, const RasterVol *rv, const CompactVol *cv, int cus,
                                 hipStream_t st) {
    if (a.S <= 0) return hipSuccess;
    if (rv) launch_seed_end_l(a, RasterLookup{*rv}, cus, st);
    else launch_seed_end_l(a, CompactLookup{*cv}, cus, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// parcellation outputs of C: one wavefront per row
// ---------------------------------------------------------------------------------------------

// label[i] = lowest m holding the row's maximum (-1 when no entry is positive), sums[i] = row sum,
// frac[i][m] = C[i][m] / sums[i] taken in double and rounded to float (0 when the sum is not
// positive).  Any output may be null.
constexpr int kParcVals = 6;   // row entries per lane kept in registers (rows of up to 384 labels)

__global__ void __launch_bounds__(kBlock) k_parcellate(const int32_t *__restrict__ C, int32_t N, int32_t M,
                                                       int32_t *__restrict__ label, float *__restrict__ frac,
                                                       int64_t *__restrict__ sums) {
    const int lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
    // each lane keeps entries lane + 64 q (q < kParcVals) of its wavefront's row in registers, and
    // the next row's are loaded while this one is reduced; entries past kParcVals * 64 are read
    // from memory
    int v[kParcVals], vn[kParcVals];
    auto load_row = [&](int64_t i, int (&dst)[kParcVals]) {
#pragma unroll
        for (int q = 0; q < kParcVals; ++q) {
            const int m = lane + q * kWave;
            dst[q] = (i < N && m < M) ? C[i * (int64_t)M + m] : 0;
        }
    };
    int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    load_row(i, v);
    for (; i < N; i += nw) {
        load_row(i + nw, vn);
        const int32_t *row = C + i * (int64_t)M;
        long long total = 0;
        int best = 0, bidx = -1;   // largest positive value seen and its lowest column
#pragma unroll
        for (int q = 0; q < kParcVals; ++q) {
            const int m = lane + q * kWave;
            total += v[q];
            if (m < M && v[q] > best) {
                best = v[q];
                bidx = m;
            }
        }
        for (int m = lane + kParcVals * kWave; m < M; m += kWave) {
            const int x = row[m];
            total += x;
            if (x > best) {
                best = x;
                bidx = m;
            }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            total += __shfl_xor(total, off);
            const int ob = __shfl_xor(best, off), oi = __shfl_xor(bidx, off);
            if (ob > best || (ob == best && ob > 0 && oi < bidx)) {
                best = ob;
                bidx = oi;
            }
        }
        if (lane == 0) {
            if (label) label[i] = bidx;
            if (sums) sums[i] = total;
        }
        if (frac) {
            const double d = (double)total;
            float *out = frac + i * (int64_t)M;
#pragma unroll
            for (int q = 0; q < kParcVals; ++q) {
                const int m = lane + q * kWave;
                if (m < M) out[m] = total > 0 ? (float)((double)v[q] / d) : 0.0f;
            }
            for (int m = lane + kParcVals * kWave; m < M; m += kWave)
                out[m] = total > 0 ? (float)((double)row[m] / d) : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < kParcVals; ++q) v[q] = vn[q];
    }
}

hipError_t launch_parcellate(const int32_t *C, int32_t N, int32_t M, int32_t *label, float *frac, int64_t *sums,
                             int cus, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    int64_t blocks = ((int64_t)N + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > (int64_t)cus * 8) blocks = (int64_t)cus * 8;
    k_parcellate<<<(unsigned)blocks, kBlock, 0, st>>>(C, N, M, label, frac, sums);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// batched form: work items, zero fill of every C, launchers
// ---------------------------------------------------------------------------------------------

// items[i] = (subject, first streamline of [s_begin, S) at or after point P0 + floor(j * (P - P0) / n_s))
// for the j-th of the subject's n_s items (P0 = offsets[s_begin], P = offsets[S]); item_base[s] ..
// item_base[s+1] are subject s's items.  The same launch zeroes zero[0 .. nzero) (the counting
// launches' overflow count and range queues), which saves a launch of its own.
__global__ void k_partition_batched(const StreamSubject *__restrict__ subs, const int64_t *__restrict__ item_base,
                                    int32_t nsub, int2 *__restrict__ items, unsigned long long *__restrict__ zero,
                                    int64_t nzero) {
    const int64_t n = item_base[nsub];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nzero; i += stride) zero[i] = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int lo = 0, hi = nsub;   // subject: last s with item_base[s] <= i
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (item_base[mid] <= i) lo = mid;
            else hi = mid;
        }
        const StreamSubject &sub = subs[lo];
        const int64_t j = i - item_base[lo], ns = item_base[lo + 1] - item_base[lo];
        const int64_t sb = clamp64(sub.s_begin, 0, sub.S);
        const int64_t P0 = sub.offsets[sb];
        int64_t P = sub.offsets[sub.S];
        if (P < P0) P = P0;
        const int64_t target = P0 + (int64_t)(((__int128)j * (P - P0)) / ns);
        int64_t a = sb, b = sub.S;
        while (a < b) {
            const int64_t mid = (a + b) >> 1;
            if (sub.offsets[mid] < target) a = mid + 1;
            else b = mid;
        }
        items[i] = make_int2(lo, (int)a);
    }
}

// C of every subject set to zero (blockIdx.y = subject)
__global__ void k_zero_subjects(const StreamSubject *__restrict__ subs, const int64_t *__restrict__ sizes) {
    const StreamSubject &sub = subs[blockIdx.y];
    const int64_t n = sizes[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) sub.C[i] = 0;
}

hipError_t launch_zero_subjects(const StreamSubject *subs, const int64_t *sizes, int32_t nsub, int cus, hipStream_t st) {
    k_zero_subjects<<<dim3((unsigned)(cus > 0 ? cus : 64), (unsigned)nsub), kBlock, 0, st>>>(subs, sizes);
    return hipGetLastError();
}

hipError_t launch_partition_batched(const StreamSubject *subs, const int64_t *item_base, int32_t nsub, int64_t nitems,
                                    int2 *items, unsigned long long *zero, int64_t nzero, int cus, hipStream_t st) {
    k_partition_batched<<<fill_blocks(std::max<int64_t>(nitems, nzero), cus), kBlock, 0, st>>>(subs, item_base, nsub,
                                                                                             items, zero, nzero);
    return hipGetLastError();
}

template <int B, bool E, int U>
static int batched_blocks_per_cu_of(size_t dyn) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, reinterpret_cast<const void *>(&k_count_batched<B, E, U>), kBlock, dyn);
    return (e == hipSuccess && n > 0) ? n : 4;
}

int count_batched_blocks_per_cu(int batch, int coarse_words, BatchedKind kind) {
    const size_t dyn = 4 * (size_t)kWavesPerBlock * (size_t)coarse_words;
    switch (kind) {
        case BatchedKind::kEnds:
            return batch == 2 ? batched_blocks_per_cu_of<2, true, 1>(dyn) : batched_blocks_per_cu_of<4, true, 1>(dyn);
        case BatchedKind::kUp2: return batched_blocks_per_cu_of<2, false, 2>(dyn);
        case BatchedKind::kUp4: return batched_blocks_per_cu_of<1, false, 4>(dyn);
        default:
            return batch == 2 ? batched_blocks_per_cu_of<2, false, 1>(dyn) : batched_blocks_per_cu_of<4, false, 1>(dyn);
    }
}

hipError_t launch_count_batched(const StreamSubject *subs, const int2 *items, int64_t nitems, const Overflow &ovf,
                                int32_t coarse_words, int blocks, int batch, BatchedKind kind, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const size_t dyn = 4 * (size_t)kWavesPerBlock * (size_t)coarse_words;
    switch (kind) {
        case BatchedKind::kEnds:
            if (batch == 2) k_count_batched<2, true, 1><<<blocks, kBlock, dyn, st>>>(subs, items, nitems, ovf, coarse_words);
            else k_count_batched<4, true, 1><<<blocks, kBlock, dyn, st>>>(subs, items, nitems, ovf, coarse_words);
            break;
        case BatchedKind::kUp2:   // two windows of two lookups each per batch, as k_count_stream_up<2>
            k_count_batched<2, false, 2><<<blocks, kBlock, dyn, st>>>(subs, items, nitems, ovf, coarse_words);
            break;
        case BatchedKind::kUp4:
            k_count_batched<1, false, 4><<<blocks, kBlock, dyn, st>>>(subs, items, nitems, ovf, coarse_words);
            break;
        default:
            if (batch == 2) k_count_batched<2, false, 1><<<blocks, kBlock, dyn, st>>>(subs, items, nitems, ovf, coarse_words);
            else k_count_batched<4, false, 1><<<blocks, kBlock, dyn, st>>>(subs, items, nitems, ovf, coarse_words);
            break;
    }
    return hipGetLastError();
}

// End labels of table entries [lo, lo + gridDim.y) in an endpoint mode: sub.ends.last[s] (and, mode 2,
// sub.ends.first[s]) for streamlines [s_begin, S) of each, as k_end_labels for one subject.
__global__ void k_end_labels_batched(const StreamSubject *__restrict__ subs, int32_t lo) {
    const StreamSubject &sub = subs[lo + blockIdx.y];
    const int mode = sub.ends.mode;
    if (mode != 1 && mode != 2) return;
    const int64_t Ptot = sub.offsets[sub.S] > 0 ? sub.offsets[sub.S] : 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const CompactLookup lk{sub.cv};
    for (int64_t s = clamp64(sub.s_begin, 0, sub.S) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < sub.S;
         s += stride) {
        const int64_t b0 = clamp64(sub.offsets[s], 0, Ptot);
        const int64_t b1 = clamp64(sub.offsets[s + 1], b0, Ptot);
        int r, ml = -1, mf = -1;
        if (b1 > b0) {
            lookup_point<CompactLookup, true>(sub.pts + 3 * (b1 - 1), sub.scale, sub.g, lk, r, ml);
            if (mode == 2) lookup_point<CompactLookup, true>(sub.pts + 3 * b0, sub.scale, sub.g, lk, r, mf);
        }
        const_cast<int32_t *>(sub.ends.last)[s] = ml;   // the plan's or request's own label arrays
        if (mode == 2) const_cast<int32_t *>(sub.ends.first)[s] = mf;
    }
}

// Alg. 1's count for table entries [lo, lo + gridDim.y): C(row of the first point, label of the last
// point) += 1 for streamlines [s_begin, S) of each, as k_count_seed_end for one subject.
__global__ void k_count_seed_end_batched(const StreamSubject *__restrict__ subs, int32_t lo) {
    const StreamSubject &sub = subs[lo + blockIdx.y];
    const int64_t Ptot = sub.offsets[sub.S] > 0 ? sub.offsets[sub.S] : 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const CompactLookup lk{sub.cv};
    for (int64_t s = clamp64(sub.s_begin, 0, sub.S) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < sub.S;
         s += stride) {
        const int64_t b0 = clamp64(sub.offsets[s], 0, Ptot);
        const int64_t b1 = clamp64(sub.offsets[s + 1], b0, Ptot);
        if (b1 <= b0) continue;
        int r, m, r2, m2;
        lookup_point<CompactLookup, true>(sub.pts + 3 * b0, sub.scale, sub.g, lk, r, m);
        lookup_point<CompactLookup, true>(sub.pts + 3 * (b1 - 1), sub.scale, sub.g, lk, r2, m2);
        if (r >= 0 && m2 >= 0) atomicAdd(sub.C + (uint32_t)r * sub.si + (uint32_t)m2 * sub.sm, 1);
    }
}

hipError_t launch_end_labels_batched(const StreamSubject *subs, int32_t lo, int32_t n, int cus, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_end_labels_batched<<<dim3((unsigned)(cus > 0 ? cus : 64) * 2, (unsigned)n), kBlock, 0, st>>>(subs, lo);
    return hipGetLastError();
}

hipError_t launch_count_seed_end_batched(const StreamSubject *subs, int32_t lo, int32_t n, int cus, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_count_seed_end_batched<<<dim3((unsigned)(cus > 0 ? cus : 64) * 2, (unsigned)n), kBlock, 0, st>>>(subs, lo);
    return hipGetLastError();
}

hipError_t launch_fallback_batched(const StreamSubject *subs, int32_t nsub, const Overflow &ovf, FallbackScratch fs,
                                   hipStream_t st) {
    k_fallback_batched<<<fs.blocks, kBlock, 0, st>>>(subs, nsub, ovf, fs);
    return hipGetLastError();
}

template <typename Lookup>
static hipError_t launch_fallback(const CountArgs &a, const Lookup &lk, FallbackScratch fs, hipStream_t st) {
    if (a.scale != 1.0f) k_fallback<Lookup, true><<<fs.blocks, kBlock, 0, st>>>(a, lk, fs);
    else k_fallback<Lookup, false><<<fs.blocks, kBlock, 0, st>>>(a, lk, fs);
    return hipGetLastError();
}

hipError_t launch_fallback_raster(const CountArgs &a, const RasterVol &rv, FallbackScratch fs, hipStream_t st) {
    return launch_fallback(a, RasterLookup{rv}, fs, st);
}

hipError_t launch_fallback_compact(const CountArgs &a, const CompactVol &cv, FallbackScratch fs, hipStream_t st) {
    return launch_fallback(a, CompactLookup{cv}, fs, st);
}

// ---------------------------------------------------------------------------------------------
// transpose of the accumulation layout: C[i][m] (+)= CT[m][i], 32x32 tiles through LDS
// ---------------------------------------------------------------------------------------------

template <bool ACC>
__global__ void __launch_bounds__(256) k_transpose(const int32_t *__restrict__ CT, int32_t *__restrict__ C, int32_t N,
                                                   int32_t M) {
    __shared__ int32_t tile[32][33];
    const int i0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    int32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = m0 + ty + 8 * q, i = i0 + tx;
        v[q] = (m < M && i < N) ? CT[(int64_t)m * N + i] : 0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) tile[ty + 8 * q][tx] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = ty + 8 * q, i = i0 + k, m = m0 + tx;
        if (i < N && m < M) {
            int32_t *dst = C + (int64_t)i * M + m;
            *dst = ACC ? *dst + tile[tx][k] : tile[tx][k];
        }
    }
}

hipError_t launch_transpose(const int32_t *CT, int32_t *C, int32_t N, int32_t M, bool accumulate, hipStream_t st) {
    const dim3 grid((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32));
    if (accumulate) k_transpose<true><<<grid, 256, 0, st>>>(CT, C, N, M);
    else k_transpose<false><<<grid, 256, 0, st>>>(CT, C, N, M);
    return hipGetLastError();
}

// Grid-stride over the tiles of all jobs; each tile finds its job by a binary search over
// first_tile (block-uniform, so the barriers stay uniform).  A 64x64 tile gives every thread 16
// loads in flight before its stores.
__global__ void __launch_bounds__(256) k_transpose_many(const TransposeJob *__restrict__ jobs, int32_t njobs,
                                                        int64_t ntiles) {
    constexpr int T = kTransposeTile;
    __shared__ int32_t tile[T][T + 1];
    const int tx = threadIdx.x & (T - 1), ty = threadIdx.x / T;   // T x (256 / T)
    constexpr int R = 256 / T;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int lo = 0, hi = njobs;   // jobs[lo].first_tile <= t, and t < jobs[hi].first_tile (or ntiles)
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (jobs[mid].first_tile <= t) lo = mid;
            else hi = mid;
        }
        const TransposeJob j = jobs[lo];
        const int64_t local = t - j.first_tile;
        const int64_t tn = (j.N + T - 1) / T;
        const int i0 = (int)(local % tn) * T, m0 = (int)(local / tn) * T;
        int32_t v[T / R];   // (a fixed trip count, so that all the loads issue before the LDS stores)
#pragma unroll
        for (int q = 0; q < T / R; ++q) {
            const int m = m0 + ty + q * R, i = i0 + tx;
            v[q] = (m < j.M && i < j.N) ? j.CT[(int64_t)m * j.N + i] : 0;
        }
#pragma unroll
        for (int q = 0; q < T / R; ++q) tile[ty + q * R][tx] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < T / R; ++q) {
            const int i = i0 + ty + q * R, m = m0 + tx;
            if (i < j.N && m < j.M) j.C[(int64_t)i * j.M + m] = tile[tx][ty + q * R];
        }
        __syncthreads();   // the tile is rewritten by the next iteration
    }
}

hipError_t launch_transpose_many(const TransposeJob *jobs, int32_t njobs, int64_t ntiles, int cus, hipStream_t st) {
    if (njobs <= 0 || ntiles <= 0) return hipSuccess;
    const int64_t cap = (int64_t)(cus > 0 ? cus : 64) * 16;
    const unsigned blocks = (unsigned)std::min<int64_t>(ntiles, cap);
    k_transpose_many<<<blocks, 256, 0, st>>>(jobs, njobs, ntiles);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// histogram of appended C updates: a counting sort by tile of C, then one LDS histogram per tile
// ---------------------------------------------------------------------------------------------

constexpr uint32_t kNoEntry = 0xFFFFFFFFu;   // never an update (updates index C: < 2^31)
constexpr int kPairUnroll = 8;               // independent loads in flight per thread

// Slices [w0, w1) of workgroup b out of nblk.
__device__ __forceinline__ void slice_range(int32_t nwaves, int b, int nblk, int32_t &w0, int32_t &w1) {
    w0 = (int32_t)((int64_t)nwaves * b / nblk);
    w1 = (int32_t)((int64_t)nwaves * (b + 1) / nblk);
}

constexpr int kMaxSlicesPerBlock = 64;   // nblk >= nwaves / 64 (checked by the launcher)

// Calls f(entry) for every update in this workgroup's slices, taken as one flat index range (pre:
// LDS prefix of the slice lengths) so that every thread keeps kPairUnroll loads in flight.
template <typename F>
__device__ __forceinline__ void for_each_update(const PairOut &po, int32_t nwaves, uint32_t *pre, F &&f) {
    int32_t w0, w1;
    slice_range(nwaves, blockIdx.x, gridDim.x, w0, w1);
    const int ns = w1 - w0;
    if (threadIdx.x < (unsigned)ns) pre[threadIdx.x + 1] = min(po.counts[w0 + threadIdx.x], po.cap);
    if (threadIdx.x == 0) pre[0] = 0u;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k <= ns; ++k) pre[k] += pre[k - 1];
    __syncthreads();
    const uint32_t total = pre[ns];
    for (uint32_t k0 = threadIdx.x; k0 < total; k0 += kPairUnroll * blockDim.x) {
        uint32_t v[kPairUnroll];
#pragma unroll
        for (int j = 0; j < kPairUnroll; ++j) {
            const uint32_t k = k0 + j * blockDim.x;
            v[j] = kNoEntry;
            if (k < total) {
                int lo = 0, hi = ns - 1;   // the slice holding flat index k: pre[lo] <= k < pre[lo + 1]
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                v[j] = __builtin_nontemporal_load(po.pairs + (size_t)(w0 + lo) * po.cap + (k - pre[lo]));
            }
        }
#pragma unroll
        for (int j = 0; j < kPairUnroll; ++j)
            if (v[j] != kNoEntry) f(v[j]);
    }
}

// Tile histogram of workgroup b's updates; reserves b's run inside each tile with one atomic on
// the tile's cursor (cursors one 128-byte line apart): boff[b * ntiles + t] = offset of the run.
__global__ void __launch_bounds__(1024) k_pair_tile_counts(PairOut po, int32_t nwaves, int32_t ntiles,
                                                           uint32_t *__restrict__ cursor, uint32_t *__restrict__ boff) {
    __shared__ uint32_t h[kMaxPairTiles];
    __shared__ uint32_t pre[kMaxSlicesPerBlock + 1];
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) h[t] = 0u;
    __syncthreads();
    for_each_update(po, nwaves, pre, [&](uint32_t e) {
        const uint32_t t = e >> kPairTileLog2;
        if (t < (uint32_t)ntiles) atomicAdd(&h[t], 1u);
    });
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
        boff[(size_t)blockIdx.x * ntiles + t] = h[t] ? atomicAdd(&cursor[32 * t], h[t]) : 0u;
}

// Exclusive scan of c[0 .. n) in LDS (n <= kMaxPairTiles) by a 1024-thread workgroup; thread i
// owns entries 4i .. 4i+3 and gets their counts back in own[].  wsum: 16 words of LDS.
__device__ __forceinline__ uint32_t block_scan_tiles(uint32_t *c, int32_t n, uint32_t (&own)[4], uint32_t *wsum) {
    static_assert(kMaxPairTiles == 4 * 1024, "four tiles per thread");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t s = 0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = 4 * tid + q;
        own[q] = t < n ? c[t] : 0u;
        s += own[q];
    }
    uint32_t x = s;   // inclusive scan over the wavefront
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    uint32_t before = 0u, total = 0u;
    for (int k = 0; k < 16; ++k) {
        const uint32_t w = wsum[k];
        before += k < wv ? w : 0u;
        total += w;
    }
    uint32_t run = before + x - s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = 4 * tid + q;
        if (t < n) c[t] = run;
        run += own[q];
    }
    return total;
}

constexpr int kScatterUnroll = 6;                      // loads in flight per thread (64 VGPRs in all)
constexpr int kScatterRound = kScatterUnroll * 1024;   // updates staged in LDS per round

// Each update into its tile's run of `sorted`, at workgroup b's reserved offset.  Every workgroup
// first scans the tile totals (cursor[32 t]) into the tiles' bases; workgroup 0 also stores them in
// base[0 .. ntiles] for the tile pass.  A round of up to kScatterRound updates is then grouped by
// tile in LDS and the stores go out in that order, so neighbouring lanes write neighbouring entries
// of a run instead of one entry per run each.  Two workgroups per CU: 64 VGPRs and 57.9 KB of LDS
// each.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_pair_scatter(PairOut po, int32_t nwaves, int32_t ntiles, const uint32_t *__restrict__ cursor,
               uint32_t *__restrict__ base, const uint32_t *__restrict__ boff, uint32_t *__restrict__ sorted) {
    __shared__ uint32_t cur[kMaxPairTiles];     // next entry of this workgroup's run in each tile
    __shared__ uint32_t cnt[kMaxPairTiles];     // the round's count per tile, then its offset in stage
    __shared__ uint32_t stage[kScatterRound];   // the round's updates, grouped by tile
    __shared__ uint32_t pre[kMaxSlicesPerBlock + 1];
    __shared__ uint32_t wsum[16];
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) cnt[t] = cursor[32 * t];   // tile totals
    __syncthreads();
    {
        uint32_t own[4];
        const uint32_t all = block_scan_tiles(cnt, ntiles, own, wsum);   // cnt: the tiles' bases
        __syncthreads();
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
            cur[t] = cnt[t] + boff[(size_t)blockIdx.x * ntiles + t];
            if (blockIdx.x == 0) base[t] = cnt[t];
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) base[ntiles] = all;
        __syncthreads();
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) cnt[t] = 0u;
    }
    int32_t w0, w1;
    slice_range(nwaves, blockIdx.x, gridDim.x, w0, w1);
    const int ns = w1 - w0;
    if (threadIdx.x < (unsigned)ns) pre[threadIdx.x + 1] = min(po.counts[w0 + threadIdx.x], po.cap);
    if (threadIdx.x == 0) pre[0] = 0u;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k <= ns; ++k) pre[k] += pre[k - 1];
    __syncthreads();
    const uint32_t total = pre[ns];
    for (uint32_t r0 = 0; r0 < total; r0 += kScatterRound) {   // uniform over the workgroup
        uint32_t v[kScatterUnroll], rank[kScatterUnroll];
#pragma unroll
        for (int j = 0; j < kScatterUnroll; ++j) {
            const uint32_t k = r0 + threadIdx.x + j * 1024u;
            v[j] = kNoEntry;
            if (k < total) {
                int lo = 0, hi = ns - 1;   // the slice holding flat index k: pre[lo] <= k < pre[lo + 1]
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                v[j] = __builtin_nontemporal_load(po.pairs + (size_t)(w0 + lo) * po.cap + (k - pre[lo]));
            }
        }
#pragma unroll
        for (int j = 0; j < kScatterUnroll; ++j) {
            const uint32_t t = v[j] >> kPairTileLog2;   // kNoEntry: t >= ntiles
            if (t < (uint32_t)ntiles) rank[j] = atomicAdd(&cnt[t], 1u);
            else v[j] = kNoEntry;
        }
        __syncthreads();
        uint32_t own[4];
        const uint32_t n = block_scan_tiles(cnt, ntiles, own, wsum);   // cnt: offsets in stage
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kScatterUnroll; ++j)
            if (v[j] != kNoEntry) stage[cnt[v[j] >> kPairTileLog2] + rank[j]] = v[j];
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += 1024u) {
            const uint32_t e = stage[i], t = e >> kPairTileLog2;
            sorted[cur[t] + (i - cnt[t])] = e;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = 4 * (int)threadIdx.x + q;
            if (t < ntiles) {
                cur[t] += own[q];
                cnt[t] = 0u;
            }
        }
        __syncthreads();
    }
}

// One workgroup per tile: C[tile] += the histogram of the tile's updates.
__global__ void __launch_bounds__(512) k_pair_tile_add(const uint32_t *__restrict__ sorted,
                                                       const uint32_t *__restrict__ base, int32_t *__restrict__ Cm,
                                                       int64_t NM) {
    constexpr uint32_t kTile = 1u << kPairTileLog2;
    __shared__ uint32_t h[kTile];
    for (uint32_t k = threadIdx.x; k < kTile; k += blockDim.x) h[k] = 0u;
    __syncthreads();
    const uint32_t b = base[blockIdx.x], e = base[blockIdx.x + 1];
    for (uint32_t k0 = b + threadIdx.x; k0 < e; k0 += kPairUnroll * blockDim.x) {
        uint32_t v[kPairUnroll];
#pragma unroll
        for (int j = 0; j < kPairUnroll; ++j) {
            const uint32_t k = k0 + j * blockDim.x;
            v[j] = k < e ? __builtin_nontemporal_load(sorted + k) : kNoEntry;
        }
#pragma unroll
        for (int j = 0; j < kPairUnroll; ++j)
            if (v[j] != kNoEntry) atomicAdd(&h[v[j] & (kTile - 1u)], 1u);
    }
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x << kPairTileLog2;
    int32_t *C = Cm + t0;   // the tile's entries of C
    const uint32_t len = (uint32_t)min((int64_t)kTile, NM - t0);
    if (len == kTile && (reinterpret_cast<uintptr_t>(C) & 15u) == 0) {
        // whole tile: four entries per thread and step, all loads of C first
        constexpr int kSteps = kTile / (4 * 512);
        int4 c[kSteps];
        int4 *C4 = reinterpret_cast<int4 *>(C);
        const uint4 *h4 = reinterpret_cast<const uint4 *>(h);
#pragma unroll
        for (int j = 0; j < kSteps; ++j) c[j] = C4[threadIdx.x + j * 512];
#pragma unroll
        for (int j = 0; j < kSteps; ++j) {
            const uint4 a = h4[threadIdx.x + j * 512];
            c[j].x += (int)a.x;
            c[j].y += (int)a.y;
            c[j].z += (int)a.z;
            c[j].w += (int)a.w;
            C4[threadIdx.x + j * 512] = c[j];
        }
    } else {
        for (uint32_t k = threadIdx.x; k < len; k += blockDim.x) C[k] += (int32_t)h[k];
    }
}

hipError_t launch_pair_histogram(const PairOut &po, int32_t nwaves, int32_t ntiles, int32_t *C, int64_t NM,
                                 uint32_t *hist, uint32_t *sorted, int cus, hipStream_t st) {
    if (ntiles < 1 || ntiles > kMaxPairTiles || nwaves < 1) return hipErrorInvalidValue;
    const int nblk = pair_hist_blocks(ntiles);
    if ((int64_t)nblk * kMaxSlicesPerBlock < nwaves) return hipErrorInvalidValue;
    // hist: cursors (32 words per tile, zero on entry) | tile bases (ntiles + 1) | per-workgroup offsets
    uint32_t *cursor = hist;
    uint32_t *base = cursor + 32 * (size_t)kMaxPairTiles;
    uint32_t *boff = base + kMaxPairTiles + 64;
    (void)cus;
    k_pair_tile_counts<<<nblk, 1024, 0, st>>>(po, nwaves, ntiles, cursor, boff);
    k_pair_scatter<<<nblk, 1024, 0, st>>>(po, nwaves, ntiles, cursor, base, boff, sorted);
    k_pair_tile_add<<<ntiles, 512, 0, st>>>(sorted, base, C, NM);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// ceiling probes: what the counting path can reach on this device at best
// ---------------------------------------------------------------------------------------------

constexpr uint32_t kProbeMagic = 0x9E3779B9u;   // a folded value that (practically) never occurs

// Points [P][3] streamed read-only with the counting kernel's access pattern: one contiguous range
// per wavefront, 64 x 12-byte non-temporal buffer loads, kBatch windows per step.  The loaded bits
// are folded into one word per lane, stored only if it equals kProbeMagic, so the loads stay.
template <int kBatch>
__global__ void __launch_bounds__(kBlock) k_probe_stream(const float *__restrict__ pts, int64_t P, int64_t nwaves,
                                                         uint32_t *__restrict__ sink) {
    const int lane = lane_id();
    // (the wave index through readfirstlane: a range derived from threadIdx would make the buffer
    // resource divergent and put every load in a loop over lanes)
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + uniform32((int)(threadIdx.x >> 6));
    const int64_t per = (P + nwaves - 1) / nwaves;
    const int64_t p0 = min(P, wave * per), p1 = min(P, p0 + per);
    const uint32_t L = (uint32_t)(p1 - p0);
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(pts + 3 * p0, 12ull * L);
    const uint32_t lane12 = 12u * (uint32_t)lane;
    uint32_t acc = 0u;
    for (uint32_t w0 = 0; w0 < L; w0 += kBatch * kWave) {
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b96(rp, lane12, 12u * w0 + 768u * b, kAuxStream);
            acc ^= v[0] ^ (v[1] << 1) ^ (v[2] << 2);
        }
    }
    if (acc == kProbeMagic) sink[0] = acc;
}

// No-return int32 atomic adds C[idx[k]] += 1, k < n (indices >= n_words are skipped), four index
// loads in flight per thread before their atomics.
__global__ void __launch_bounds__(kBlock) k_probe_atomics(int32_t *__restrict__ C, int64_t n_words,
                                                          const uint32_t *__restrict__ idx, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k0 < n; k0 += 4 * stride) {
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t k = k0 + j * stride;
            v[j] = k < n ? idx[k] : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((int64_t)v[j] < n_words) atomicAdd(C + v[j], 1);
    }
}

// The counting kernel's per-point lookups without its per-streamline work: the point stream of
// k_probe_stream, voxelisation, the coarse test in LDS, the (word, rank base) gather and, for
// occupied voxels, the code gather, in the counting kernel's software pipeline (each iteration
// issues batch k's code gathers, batch k+1's pair gathers and batch k+2's points, then decodes
// batch k).  The decoded rows and labels are folded like the stream probe.  No de-duplication,
// no pair updates: the stream-plus-lookup ceiling of the flat-stream kernel.
template <int kBatch, bool kBrick>
__global__ void __launch_bounds__(kBlock) k_probe_lookup(StreamSubject sub, int64_t P, int64_t nwaves,
                                                         uint32_t *__restrict__ sink) {
    extern __shared__ uint32_t s_coarse[];
    const CompactVol &cv = sub.cv;
    for (int k = threadIdx.x; k < cv.ncoarse_words; k += blockDim.x) s_coarse[k] = cv.coarse[k];
    __syncthreads();
    const int lane = lane_id();
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + uniform32((int)(threadIdx.x >> 6));
    const int64_t per = (P + nwaves - 1) / nwaves;
    const int64_t p0 = min(P, wave * per), p1 = min(P, p0 + per);
    const uint32_t L = (uint32_t)(p1 - p0);
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(sub.pts + 3 * p0, 12ull * L);
    const __amdgpu_buffer_rsrc_t rvol = make_rsrc(cv.mb, cv.span);
    const uint32_t lane12 = 12u * (uint32_t)lane;
    uint32_t bX = fbits(sub.g.Xf), bY = fbits(sub.g.Yf), bZ = fbits(sub.g.Zf);
    asm volatile("" : "+v"(bX), "+v"(bY), "+v"(bZ));
    const uint32_t SBX = (uint32_t)cv.SBX, SBXY = (uint32_t)cv.SBXY;
    const uint32_t csx = (uint32_t)cv.csx, csyz = (uint32_t)cv.csyz, CBX = (uint32_t)cv.CBX, CBXY = (uint32_t)cv.CBXY;
    const int codes_off = uniform32((int)cv.codes_off);
    constexpr uint32_t kOutOfRange = 0xFFFFFFF8u;
    const uint32_t code_oob = kOutOfRange - (uint32_t)codes_off;
    constexpr uint32_t BW = kWave * kBatch;
    float ax[kBatch], ay[kBatch], az[kBatch];
    auto load_batch = [&](uint32_t w) {
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b96(rp, lane12, 12u * w + 768u * b, kAuxStream);
            ax[b] = __uint_as_float(v[0]);
            ay[b] = __uint_as_float(v[1]);
            az[b] = __uint_as_float(v[2]);
        }
    };
    auto lookup = [&](uint32_t w0, uint32_t (&addr)[kBatch], uint32_t (&bix)[kBatch]) {
        const uint32_t left = w0 < L ? L - w0 : 0u;
        const int rem = left > BW ? (int)BW : (int)left;
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const float tx = __fadd_rn(__fmul_rn(ax[b], sub.scale), 0.5f);
            const float ty = __fadd_rn(__fmul_rn(ay[b], sub.scale), 0.5f);
            const float tz = __fadd_rn(__fmul_rn(az[b], sub.scale), 0.5f);
            const bool ok = (int)(lane + b * kWave < rem) & (int)(fbits(tx) < bX) & (int)(fbits(ty) < bY) &
                            (int)(fbits(tz) < bZ);
            const uint32_t ix = (uint32_t)(int)tx, iy = (uint32_t)(int)ty, iz = (uint32_t)(int)tz;
            uint32_t sb = __umul24(iz >> 3, SBXY) + __umul24(iy >> 3, SBX) + (ix >> 4);
            asm("" : "+v"(sb));
            const uint32_t cb = kBrick ? sb : __umul24(iz >> csyz, CBXY) + __umul24(iy >> csyz, CBX) + (ix >> csx);
            const uint32_t cw = s_coarse[ok ? (cb >> 5) : 0u];
            const bool hit = (int)ok & (int)(__builtin_amdgcn_ubfe(cw, cb, 1) != 0u);
            addr[b] = hit ? (sb << 8) | ((iy << 2) & 0x18u) | ((iz << 5) & 0xE0u) : kOutOfRange;
            bix[b] = (ix & 15u) | ((iy & 1u) << 4);
        }
    };
    auto gather_pairs = [&](const uint32_t (&addr)[kBatch], uint32_t (&mw)[kBatch], uint32_t (&base)[kBatch]) {
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const auto e = __builtin_amdgcn_raw_buffer_load_b64(rvol, addr[b], 0, kAuxCached);
            mw[b] = e[0];
            base[b] = e[1];
        }
    };
    uint32_t acc = 0u;
    uint32_t bix[kBatch], mw[kBatch], base[kBatch];
    {
        uint32_t addr[kBatch];
        load_batch(0u);
        lookup(0u, addr, bix);
        __builtin_amdgcn_sched_barrier(0);
        gather_pairs(addr, mw, base);
        __builtin_amdgcn_sched_barrier(0);
        load_batch(BW);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (uint32_t w0 = 0; w0 < L; w0 += BW) {
        bool flag[kBatch];
        uint32_t c[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            flag[b] = __builtin_amdgcn_ubfe(mw[b], bix[b], 1) != 0u;
            const uint32_t at = base[b] + __popc(__builtin_amdgcn_ubfe(mw[b], 0, bix[b]));
            const uint32_t off = flag[b] ? (cv.packed ? at << 2 : at << 3) : code_oob;
            c[b] = __builtin_amdgcn_raw_buffer_load_b32(rvol, off, codes_off, kAuxCached);
        }
        __builtin_amdgcn_sched_barrier(0);
        uint32_t bix2[kBatch], mw2[kBatch], base2[kBatch];
        {
            uint32_t addr[kBatch];
            lookup(w0 + BW, addr, bix2);
            __builtin_amdgcn_sched_barrier(0);
            gather_pairs(addr, mw2, base2);
        }
        __builtin_amdgcn_sched_barrier(0);
        load_batch(w0 + 2 * BW);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const uint32_t rv = c[b] & cv.rmask, mv = c[b] >> cv.rbits;
            acc += flag[b] ? (rv ^ (mv << 3)) : 0u;
            bix[b] = bix2[b];
            mw[b] = mw2[b];
            base[b] = base2[b];
        }
    }
    if (acc == kProbeMagic) sink[0] = acc;
}

hipError_t launch_probe_stream(const float *pts, int64_t P, int cus, uint32_t *sink, hipStream_t st) {
    if (P <= 0) return hipSuccess;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_probe_stream<4>),
                                                     kBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 4;
    const int64_t blocks = (int64_t)cus * per_cu;
    k_probe_stream<4><<<(unsigned)blocks, kBlock, 0, st>>>(pts, P, blocks * kWavesPerBlock, sink);
    return hipGetLastError();
}

hipError_t launch_probe_atomics(int32_t *C, int64_t n_words, const uint32_t *idx, int64_t n, int cus, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)cus * 8);
    k_probe_atomics<<<(unsigned)blocks, kBlock, 0, st>>>(C, n_words, idx, n);
    return hipGetLastError();
}

hipError_t launch_probe_lookup(const StreamSubject &sub, int64_t P, int cus, uint32_t *sink, hipStream_t st) {
    if (P <= 0) return hipSuccess;
    const size_t dyn = 4 * (size_t)sub.cv.ncoarse_words;
    const bool brick = sub.cv.csx == 4 && sub.cv.csyz == 3;
    const void *fn = brick ? reinterpret_cast<const void *>(&k_probe_lookup<4, true>)
                           : reinterpret_cast<const void *>(&k_probe_lookup<4, false>);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, dyn) != hipSuccess || per_cu < 1) per_cu = 4;
    const int64_t blocks = (int64_t)cus * per_cu;
    if (brick) k_probe_lookup<4, true><<<(unsigned)blocks, kBlock, dyn, st>>>(sub, P, blocks * kWavesPerBlock, sink);
    else k_probe_lookup<4, false><<<(unsigned)blocks, kBlock, dyn, st>>>(sub, P, blocks * kWavesPerBlock, sink);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------------------------

__global__ void k_validate(const int64_t *__restrict__ offsets, int64_t S, const int32_t *__restrict__ roi,
                           const int32_t *__restrict__ lab, int64_t nvox, int32_t N, int32_t M, int32_t *flags) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int f = 0;
    if (t0 == 0 && offsets[0] != 0) f |= 1;
    for (int64_t s = t0; s < S; s += stride)
        if (offsets[s + 1] < offsets[s]) f |= 1;
    for (int64_t v = t0; v < nvox; v += stride) {
        if (roi[v] >= N) f |= 2;
        if (lab[v] >= M) f |= 4;
    }
    if (f) atomicOr(flags, f);
}

hipError_t launch_validate(const int64_t *offsets, int64_t S, const int32_t *roi, const int32_t *lab, int64_t nvox,
                           int32_t N, int32_t M, int32_t *flags, int cus, hipStream_t st) {
    k_fill_i32<<<1, kWave, 0, st>>>(flags, 1, 0);
    const int64_t n = S > nvox ? S : nvox;
    k_validate<<<fill_blocks(n, cus), kBlock, 0, st>>>(offsets, S, roi, lab, nvox, N, M, flags);
    return hipGetLastError();
}

}  // namespace fc
