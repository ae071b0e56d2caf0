/*
 * xrt_batch.h -- many x-ray transform problems of uneven size in
 * persistent launches (one for the forward, two for the adjoint), optionally
 * replayed as a HIP graph, with a run-time autotuner.  C ABI of libxrt.so.
 *
 * Each problem is what xrt_plan_create takes (a grid, a degree 0..3 or
 * XRT_BOX3, a line list, eq. (4) and its adjoint as in xrt.h); problems of
 * different bases mix in one batch.  The batch builds one plan per
 * problem and owns, per problem, three device buffers: the coefficient image
 * (input of the forward), the sinogram (output of the forward, input of the
 * adjoint) and the back-projected image (output of the adjoint).  Their
 * addresses are fixed for the life of the batch, which is what lets a
 * captured graph be replayed.
 *
 * Work is split into items: (problem, strip of 128 grid rows, block of lines)
 * for the forward -- a problem's items strip by strip, so the workgroups in
 * flight share one strip of its coefficient layouts -- and (problem, pixel
 * tile) for the adjoint, listed largest problem first.  The adjoint takes
 * two persistent launches: the lines closer to vertical on 64 x 32 tiles,
 * which write the images, then the lines closer to horizontal on 32 x 64
 * tiles, which add into them (a tile is 64 pixels across the lines it
 * takes).  A fixed grid of workgroups (blocks_per_cu per compute unit) takes
 * items from one atomic counter per launch until the list is exhausted; each
 * item is computed by one workgroup, which alone writes its pixels in that
 * launch (the adjoint stays a gather, with no atomics on the images).
 * Results are identical for every configuration: a line's per-strip sum
 * (summed over strips in a fixed order) or a tile's gather never depends on
 * which workgroup runs it.
 *
 * Conventions are those of xrt.h (status codes, streams, xrt_last_error).
 */
#ifndef XRT_BATCH_H
#define XRT_BATCH_H

#include <stdint.h>

#include "xrt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xrt_batch xrt_batch;

typedef struct {
    xrt_grid grid;
    int32_t degree;
    xrt_lines lines;   /* device pointers, read during xrt_batch_create only */
} xrt_problem;

typedef struct {
    int32_t fwd_blocks_per_cu;   /* persistent forward grid: 1..32 workgroups per CU */
    int32_t lines_per_item;      /* lines per forward work item: 256, 512, 1024 or 2048 */
    int32_t adj_blocks_per_cu;   /* persistent adjoint grid: 1..32 workgroups per CU */
    int32_t pad;
} xrt_batch_config;

/* Plans for `count` >= 1 problems (as xrt_plan_create: synchronises with
 * `stream`), the per-problem buffers (zeroed) and the work lists.  Errors:
 * those of xrt_plan_create, EINVAL (null, count < 1), ENOMEM. */
xrt_status xrt_batch_create(const xrt_problem* problems, int32_t count, void* stream, xrt_batch** out);
void xrt_batch_destroy(xrt_batch* b);

/* Device addresses of problem p's buffers (coefficients [ny][nx], sinogram
 * [n lines], back-projection [ny][nx]); any output pointer may be NULL.
 * Errors: EINVAL. */
xrt_status xrt_batch_buffers(const xrt_batch* b, int32_t p, float** coeffs, float** sino, float** back);

/* Totals: lines over all problems, forward and adjoint work items. */
xrt_status xrt_batch_info(const xrt_batch* b, int64_t* total_lines, int32_t* fwd_items, int32_t* adj_items);

/* sino_p = H_p coeffs_p for every p (one persistent launch after the
 * per-problem layout passes); back_p = H_p^T sino_p (two persistent launches
 * after the per-problem sinogram reordering).  No synchronisation, no
 * allocation.  Errors: EINVAL, EHIP. */
xrt_status xrt_batch_forward(xrt_batch* b, void* stream);
xrt_status xrt_batch_adjoint(xrt_batch* b, void* stream);

/* Forward then adjoint.  use_graph != 0: the sequence is captured into a
 * HIP graph on the first call (and again after a configuration change) and
 * replayed; the graph contains kernel launches only (the work counters are
 * reset by a kernel).  Errors: EINVAL, EHIP. */
xrt_status xrt_batch_run(xrt_batch* b, int32_t use_graph, void* stream);

xrt_status xrt_batch_get_config(const xrt_batch* b, xrt_batch_config* cfg);
/* Rebuilds the forward work list if lines_per_item changes.  Errors: EINVAL
 * (a field out of range). */
xrt_status xrt_batch_set_config(xrt_batch* b, const xrt_batch_config* cfg);

/* Times every forward configuration (blocks per CU x lines per item) and
 * every adjoint configuration (blocks per CU) on the batch's current
 * buffers, `reps` >= 1 timed runs each after one warm-up (HIP events on
 * `stream`), keeps the fastest and returns it in *best (may be NULL).
 * Synchronises with `stream`.  Errors: EINVAL, EHIP. */
xrt_status xrt_batch_autotune(xrt_batch* b, int32_t reps, xrt_batch_config* best, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* XRT_BATCH_H */
