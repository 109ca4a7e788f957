/*
 * vate_batch.h - batched VATE (part of libvate.so).
 *
 * Not part of the paper: several independent sketches (each created with
 * vate_create, with its own pool size, AT width, window k and g) are advanced
 * through a time slice together - Alg. 4's advance/preserve, scan, census and
 * estimation - by one persistent launch per phase whose workgroups claim
 * tiles over all sketches, so uneven packet counts share the chip.  The slice
 * can be captured once as a hipGraph and replayed; launch shapes are chosen
 * by a built-in autotuner.  Results per sketch are identical to running the
 * sketch alone with vate_ingest / vate_close_slice / vate_estimate.
 *
 * Conventions as in vate.h.  Member sketches must not be driven through the
 * single-sketch calls while the batch is in use, and must stay alive until
 * vate_batch_destroy.
 */
#ifndef VATE_BATCH_H
#define VATE_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "vate.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vate_batch vate_batch;

/* Launch shape of each batched phase. */
typedef struct vate_batch_tune {
    uint32_t ingest_tile;     /* packets per claimed tile, multiple of 512 */
    uint32_t census_tile;     /* 16-byte pool chunks per tile (exact widths: groups
                                 of 32 counters), multiple of 256 */
    uint32_t estimate_block;  /* threads per estimate workgroup (64, 128 or 256) */
    uint32_t grid_preserve, grid_ingest, grid_census, grid_estimate;  /* workgroups */
    uint32_t estimate_lanes;  /* lanes sharing one host's g gathers (1, 4 or 16);
                                 hosts per estimate tile = estimate_block / estimate_lanes */
    uint32_t census_unroll;   /* pool chunks in flight per census thread (1, 2 or 4) */
} vate_batch_tune;

/* Device bytes (256-byte aligned block) for a batch of n sketches, n <= 64. */
int vate_batch_bytes(uint32_t n, size_t *bytes);

/* Build a batch over n distinct sketches.  batch_dev: caller-owned device
 * block of vate_batch_bytes(n); n_pairs_dev: caller-owned device array of n
 * uint64 packet counts that each slice reads (sketch i ingests
 * n_pairs_dev[i] packets from its pair buffer).  Synchronous.
 * Errors: VATE_E_INVAL, VATE_E_NOMEM, VATE_E_DEVICE. */
int vate_batch_create(vate_sketch *const *sketches, uint32_t n, void *batch_dev,
                      const uint64_t *n_pairs_dev, vate_batch **out);

/* Set sketch i's per-slice buffers (fixed addresses; contents may change
 * between slices): pairs_dev (16-byte aligned, room for pairs_capacity
 * packets; a slice ingests min(n_pairs_dev[i], pairs_capacity) of them),
 * hosts to estimate with window kprime, est_dev (n_hosts floats) and
 * live_dev (nullable).  Synchronous. */
int vate_batch_set_io(vate_batch *b, uint32_t i, const uint32_t *pairs_dev, uint64_t pairs_capacity,
                      const uint32_t *hosts_dev, uint32_t n_hosts, uint32_t kprime, float *est_dev,
                      uint32_t *live_dev);

/* Enqueue one slice for every sketch: advance + preserve (sketches whose
 * previous slice is closed), ingest, census, estimate.  Afterwards every
 * member sketch is closed (vate_read_state / vate_read_census work on it). */
int vate_batch_slice(vate_batch *b, void *stream);

/* Capture one steady-state slice (every sketch advances) as a hipGraph on a
 * non-default stream; vate_batch_replay then launches it.  Replay requires
 * every sketch closed (e.g. after one vate_batch_slice). */
int vate_batch_capture(vate_batch *b, void *stream);
int vate_batch_replay(vate_batch *b, void *stream);

/* Read / set the launch shapes (setting drops a captured graph's validity:
 * capture again). */
int vate_batch_get_tune(const vate_batch *b, vate_batch_tune *t);
int vate_batch_set_tune(vate_batch *b, const vate_batch_tune *t);

/* Time candidate launch shapes of the ingest (tile x grid), census (tile x
 * chunks in flight per thread x grid) and estimate (workgroup size x lanes
 * per host x grid) phases on the current slice (every sketch closed) and
 * keep the fastest per phase; outputs stay those of the slice.  report
 * (nullable) receives a JSON text of the candidates and the choice (cut at
 * report_len).  Synchronises `stream` and drops any captured graph.
 * Errors: VATE_E_INVAL, VATE_E_STATE (a sketch not closed), VATE_E_DEVICE. */
int vate_batch_autotune(vate_batch *b, void *stream, char *report, size_t report_len);

const char *vate_batch_last_error(const vate_batch *b);
void vate_batch_destroy(vate_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* VATE_BATCH_H */
