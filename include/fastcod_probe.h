/*
 * fastcod_probe.h -- ceiling probes of libfastcod.so (measurement only, not part of the counting path).
 *
 * Three microbenchmarks bound what the pass-through count (Section 2, Alg. 2) can reach on the
 * device it runs on, each isolating one of its costs:
 *   - the point stream: every point read once, 12 bytes, by the counting kernel's access pattern;
 *   - the C update of Alg. 2 (one increment per (row, label) pair): no-return int32 atomic adds at
 *     caller-chosen indices;
 *   - the stream plus the per-point voxel lookups in a resident compact volume (the loc2region /
 *     passthrough lookups), without the per-streamline de-duplication or any update of C.
 * Each call only enqueues its kernel on `stream` (a hipStream_t, NULL = the null stream); time it
 * with events around the call.  Conventions (pointers, errors, no allocation by the caller's
 * arrays) are those of fastcod.h.
 */
#ifndef FASTCOD_PROBE_H
#define FASTCOD_PROBE_H

#include <stddef.h>
#include <stdint.h>

#include "fastcod.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Reads points [n_points][3] float32 (device) once.  sink: one device uint32 word that the kernel
 * writes only with a value that practically never occurs (it keeps the loads from being removed).
 * Bytes moved: 12 * n_points.  Errors: EINVAL (n_points < 0 or >= 2^37, NULL pointers), EHIP. */
int fastcod_probe_stream(const float *points, int64_t n_points, uint32_t *sink, void *stream);

/* target[idx[k]] += 1 for k < n_idx with no-return device atomics (indices >= n_words are skipped).
 * target [n_words] int32 and idx [n_idx] uint32 are device arrays.  Atomics issued: the in-range
 * indices.  Errors: EINVAL (negative sizes, NULL pointers), EHIP. */
int fastcod_probe_atomics(int32_t *target, int64_t n_words, const uint32_t *idx, int64_t n_idx, void *stream);

/* Streams points [n_points][3] float32 (device), scales each coordinate by `scale` (fl32(p*s), as
 * fastcod_opts.scale), voxelises it and looks it up in the resident volume `vol` as the counting
 * kernel does.  sink as fastcod_probe_stream.  Errors: EINVAL (bad sizes, scale, NULL pointers,
 * another device), EHIP. */
int fastcod_probe_lookup(const fastcod_volume *vol, const float *points, int64_t n_points, float scale,
                         uint32_t *sink, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FASTCOD_PROBE_H */
