// Internal declarations shared by the kernels and the host side of libfastcod.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fc {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;               // 256-thread workgroups
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kSetCap = 512;                    // LDS hash slots per wavefront (load <= 1/2)

// Exclusive upper bounds of t = fl32(q + 0.5) per axis: the smallest float >= the grid size,
// so that `t < bound` holds exactly when floor(t) < size, also for sizes above 2^24.
struct Grid {
    int32_t X, Y, Z;
    float Xf, Yf, Zf;
};

// Raster lookup straight from the caller's volumes.
struct RasterVol {
    const int32_t *roi;
    const int32_t *lab;
    int32_t X, XY;
    int32_t N, M;
};

// Compact lookup: occupancy bits in 16x8x8 super-bricks (32 words of 32 voxels each), every
// occupancy word paired with the number of occupied voxels before it (its rank base), and one
// code per occupied voxel in that order.
struct CompactVol {
    const uint2 *mb;          // [W] {occupancy word, rank base}
    const uint32_t *coarse;   // one bit per (2^cs)^3 block: any occupied voxel inside
    int32_t csx, csyz;        // log2 of the coarse block's x and y/z sides: 3,3 / 4,4 / 5,5 (cubes) or
                              // 4,3 (one 16x8x8 super-brick per block, coarse index = super-brick index)
    int32_t CBX, CBXY;        // coarse blocks along x, and per z-slab
    int32_t ncoarse_words;    // words of `coarse` (a multiple of 2)
    const uint32_t *codes32;  // packed (row | label << rbits), if packed
    const int2 *codes64;      // (row, label) pairs, if not packed
    int32_t SBX, SBXY;        // super-bricks along x, and per z-slab
    int32_t rbits;            // bits of the row field in a packed code
    uint32_t rmask;           // (1 << rbits) - 1
    int32_t N, M;
    int32_t packed;
    int64_t W;                // occupancy words
    int64_t ncodes;           // capacity of the code array (bounds of every code read)
    uint32_t codes_off;       // byte offset of the code array from mb (one allocation)
    uint32_t span;            // bytes from mb to the end of the code array (< 2^32 - 16)
};

// Streamlines whose distinct (row, label) keys outgrow the per-wave LDS set are handed to a
// fallback kernel through this queue of point indices (one point inside each such streamline).
// Per-wavefront slices of appended C updates (flat-stream kernel, plain path): wavefront w writes
// its entries to pairs[w * cap ...] and their number to counts[w]; cap 0 = every update is an atomic.
struct PairOut {
    uint32_t *pairs;
    uint32_t *counts;
    uint32_t cap;
};

// Histogram of the appended updates into C, tile by tile in LDS.
constexpr int kPairTileLog2 = 14;                   // 16K counters (64 KB of LDS) per tile of C
constexpr int kMaxPairTiles = 4096;                 // up to 2^26 entries of C take this path
// Workgroups (1024 threads) of the tile-count and scatter passes: 512, two per CU of a 256-CU
// device, all resident at once.  Each keeps ntiles offsets; every tile cursor takes one atomic
// per workgroup, so more workgroups mean a longer queue of atomics on each cursor (1024 measured
// slower, 256 leave too few loads in flight).
inline int pair_hist_blocks(int64_t ntiles) {
    (void)ntiles;
    return 512;
}

struct Overflow {
    unsigned long long *count;
    int64_t *list;
    int64_t cap;
    unsigned long long *work;   // the range (work item) queues' counters (flat-stream and batched
                                // kernels), kQueueWords apart; zeroed per launch
};

// Point ranges (work items) are handed out by kRangeQueues counters, each in a 128-byte line of its
// own: wavefront w takes the ranges c, c + Q, c + 2Q, ... of queue c = w mod Q (Q = kRangeQueues, or
// fewer for a small grid), so that no counter is contended by more than a few dozen wavefronts
// (a single counter serialises every wavefront's fetch).  Counter block: one 128-byte line for the
// overflow count, then the queues.
constexpr int kRangeQueues = 64;
constexpr int kQueueWords = 16;                                   // 64-bit words per counter line
constexpr size_t kQueueBlockBytes = 128 * (size_t)kRangeQueues;  // one launch's queues
// bytes before the overflow list: count line + `launches` blocks of queues (256-aligned)
inline size_t overflow_header_bytes(int launches) {
    return (128 + kQueueBlockBytes * (size_t)launches + 255) & ~size_t(255);
}

// Per-workgroup scratch of the fallback kernel; bit maps are all-zero between launches.
struct FallbackScratch {
    uint32_t *words;      // [blocks][stride]: N-bit map, M-bit map, M-entry label list
    int64_t stride;
    int32_t blocks;
    int32_t nwordsN, nwordsM;
};

// C is addressed as C[i * si + m * sm]: row-major [N][M] (si = M, sm = 1) or the transposed
// accumulation layout [M][N] (si = 1, sm = N); N * M < 2^31.
// Target labels of the endpoint modes.  mode 0: every point's label (pass-through); mode 1: the
// label of each streamline's last point only; mode 2: the labels of its first and last points.
// last[s] / first[s]: those labels per streamline (-1 = none), computed before the count.
struct EndLabels {
    int32_t mode;
    const int32_t *last;
    const int32_t *first;
};

struct CountArgs {
    const float *pts;
    const int64_t *offsets;
    int64_t S;
    Grid g;
    float scale;
    int32_t *C;
    uint32_t si, sm;
    Overflow ovf;
    EndLabels ends;
    int32_t up;   // upsampling factor: up - 1 points inserted between neighbouring points (1 = none)
};

// Everything the flat-stream kernels need about one subject (also the device-side descriptor of
// the batched form): streamlines [s_begin, S) of (pts, offsets) are counted into C.  s_begin > 0
// lets a caller count one streamline range of a larger set (offsets stay absolute).
struct StreamSubject {
    const float *pts;
    const int64_t *offsets;
    int64_t S;
    int64_t s_begin;
    Grid g;
    float scale;
    CompactVol cv;
    int32_t *C;
    uint32_t si, sm;
    EndLabels ends;
    int32_t up;   // upsampling factor (1 = none)
};

// ---- launchers (kernels.hip); every launcher returns the hipError_t of its launch ----
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, int cus, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, int cus, hipStream_t st);

// compact volume build: mb holds W {word, base} pairs, tile_sums ceil(W / kScanTile) words
constexpr int kScanTile = 2048;
hipError_t launch_compact_build(const int32_t *roi, const int32_t *lab, Grid g, int32_t N, int32_t M,
                                CompactVol cv, uint32_t *mb, void *codes, uint32_t *tile_sums, uint32_t *coarse,
                                int64_t W, int cus, hipStream_t st);

// Per-call state zeroed by the partition launch, so that it needs no launches of its own: C when
// it is not accumulated into, the pair histogram's tile cursors, the overflow and range counters.
// Each range may be empty.
struct ZeroRanges {
    int32_t *w32[2] = {nullptr, nullptr};
    int64_t n32[2] = {0, 0};
    unsigned long long *w64 = nullptr;
    int64_t n64 = 0;
};
// nparts ranges of whole streamlines, of equal point counts or (taper) of point counts falling
// linearly from 1.5x to 0.5x the mean in range order: first[nparts + 1]; also zeroes `z`
hipError_t launch_partition(const int64_t *offsets, int64_t S, int64_t nparts, int32_t *first, const ZeroRanges &z,
                            bool taper, int cus, hipStream_t st);
// resident 256-thread workgroups per CU of the flat-stream kernel
int count_stream_blocks_per_cu(bool scaled, bool packed, int batch, bool ends, int up, size_t dyn_lds);

hipError_t launch_count_wave(const CountArgs &a, const RasterVol &rv, int blocks, hipStream_t st);
// endpoint modes: last[s] (and, mode 2, first[s]) = label of streamline s's last (first) point,
// looked up in the raster volume when rv is given, else in the compact volume cv
hipError_t launch_end_labels(const CountArgs &a, const RasterVol *rv, const CompactVol *cv, int mode, int32_t *last,
                             int32_t *first, int cus, hipStream_t st);
// parcellation outputs of C [N][M]: label [N], frac [N][M], sums [N] (each may be null)
hipError_t launch_parcellate(const int32_t *C, int32_t N, int32_t M, int32_t *label, float *frac, int64_t *sums,
                             int cus, hipStream_t st);
// Alg. 1's count: C(row of the first point, label of the last point) += 1 for every streamline
hipError_t launch_count_seed_end(const CountArgs &a, const RasterVol *rv, const CompactVol *cv, int cus,
                                 hipStream_t st);
// wavefronts take the nparts ranges of `first` from ovf.work; batch: 64-point windows per
// pipelined batch (2 or 4)
hipError_t launch_count_stream(const CountArgs &a, const CompactVol &cv, const int32_t *first, int64_t nparts,
                               int blocks, int batch, const PairOut &po, hipStream_t st);
// C[NM] += histogram of the updates in the slices (nwaves slices of po.cap entries, lengths in
// po.counts), ntiles = ceil(NM / 16K).  hist: pair_hist_words(ntiles) words, of which the first
// pair_hist_cursor_words(ntiles) (the tile cursors) must be zero on entry; sorted: nwaves * po.cap
// words.
hipError_t launch_pair_histogram(const PairOut &po, int32_t nwaves, int32_t ntiles, int32_t *C, int64_t NM,
                                 uint32_t *hist, uint32_t *sorted, int cus, hipStream_t st);
inline int64_t pair_hist_cursor_words(int64_t ntiles) { return 32 * ntiles; }   // one 128-byte line per tile
inline int64_t pair_hist_words(int64_t ntiles) {
    return 32 * (int64_t)kMaxPairTiles + kMaxPairTiles + 64 + pair_hist_blocks(ntiles) * ntiles;
}
hipError_t launch_fallback_raster(const CountArgs &a, const RasterVol &rv, FallbackScratch fs,
                                  hipStream_t st);
hipError_t launch_fallback_compact(const CountArgs &a, const CompactVol &cv, FallbackScratch fs,
                                   hipStream_t st);

// C[i][m] = CT[m][i] (or += with accumulate), C [N][M], CT [M][N]
hipError_t launch_transpose(const int32_t *CT, int32_t *C, int32_t N, int32_t M, bool accumulate, hipStream_t st);

// One transpose of a batch: C[i][m] = CT[m][i] over kTransposeTile^2 tiles, tiles numbered from
// first_tile (the running sum of ceil(N/kTransposeTile) * ceil(M/kTransposeTile) over the jobs before it)
constexpr int kTransposeTile = 64;
struct TransposeJob {
    const int32_t *CT;
    int32_t *C;
    int32_t N, M;
    int64_t first_tile;
};
// every job of `jobs` (device array of njobs, first_tile increasing from 0; ntiles tiles in all)
hipError_t launch_transpose_many(const TransposeJob *jobs, int32_t njobs, int64_t ntiles, int cus, hipStream_t st);

// batched form
hipError_t launch_zero_subjects(const StreamSubject *subs, const int64_t *sizes, int32_t nsub, int cus, hipStream_t st);
// (also zeroes zero[0 .. nzero): the counting launches' overflow count and range queues)
hipError_t launch_partition_batched(const StreamSubject *subs, const int64_t *item_base, int32_t nsub, int64_t nitems,
                                    int2 *items, unsigned long long *zero, int64_t nzero, int cus, hipStream_t st);
// Kinds of subject of the batched form, each counted by its own launch (subjects of one kind are
// neighbours in the descriptor table): pass-through, endpoint modes 1/2 (end labels first),
// upsampled pass-through (u = 2, or u = 3..4), Alg. 1's seed-to-end count (no work items).
enum class BatchedKind : int { kPass = 0, kEnds = 1, kUp2 = 2, kUp4 = 3, kSeedEnd = 4 };
constexpr int kBatchedKinds = 5;
inline BatchedKind batched_kind(int mode, int up) {
    if (mode == 3) return BatchedKind::kSeedEnd;
    if (up > 2) return BatchedKind::kUp4;
    if (up == 2) return BatchedKind::kUp2;
    return mode == 1 || mode == 2 ? BatchedKind::kEnds : BatchedKind::kPass;
}
int count_batched_blocks_per_cu(int batch, int coarse_words, BatchedKind kind = BatchedKind::kPass);
// items[0, nitems) of subjects of one kind (kPass, kEnds, kUp2, kUp4)
hipError_t launch_count_batched(const StreamSubject *subs, const int2 *items, int64_t nitems, const Overflow &ovf,
                                int32_t coarse_words, int blocks, int batch, BatchedKind kind, hipStream_t st);
// table entries [lo, lo + n): end labels of their streamlines [s_begin, S) (entries in an endpoint mode)
hipError_t launch_end_labels_batched(const StreamSubject *subs, int32_t lo, int32_t n, int cus, hipStream_t st);
// table entries [lo, lo + n): Alg. 1's count of their streamlines [s_begin, S)
hipError_t launch_count_seed_end_batched(const StreamSubject *subs, int32_t lo, int32_t n, int cus, hipStream_t st);
hipError_t launch_fallback_batched(const StreamSubject *subs, int32_t nsub, const Overflow &ovf, FallbackScratch fs,
                                   hipStream_t st);

// ceiling probes (measurement only): the read-only point stream, no-return atomics C[idx[k]] += 1,
// and the stream with the compact-volume lookups of every point; sink: one device word
hipError_t launch_probe_stream(const float *pts, int64_t P, int cus, uint32_t *sink, hipStream_t st);
hipError_t launch_probe_atomics(int32_t *C, int64_t n_words, const uint32_t *idx, int64_t n, int cus, hipStream_t st);
hipError_t launch_probe_lookup(const StreamSubject &sub, int64_t P, int cus, uint32_t *sink, hipStream_t st);

hipError_t launch_validate(const int64_t *offsets, int64_t S, const int32_t *roi, const int32_t *lab,
                           int64_t nvox, int32_t N, int32_t M, int32_t *flags, int cus, hipStream_t st);

}  // namespace fc
