/*
 * fbnn — exact brute-force nearest-neighbour search over 8-bit patches on
 * AMD MI355X (gfx950), the second data-parallel workload of the library.
 *
 * The operation is the bottleneck of the natural-image entropy estimate of
 * Sec. 6.4 ("Estimating the Entropy of Natural Scenes"): for every target
 * patch find, by comparing it with every patch of a neighbour set, the
 * neighbour at the smallest Euclidean distance, exactly.  The paper's table
 * for this application times 4096 targets of 8 x 8 pixels against 4096 to
 * 1,048,576 neighbours.
 *
 *   dist[t] = min_m  sum_{d<D} (targets[t][d] - neighbors[m][d])^2
 *   idx[t]  = the lowest m attaining dist[t]
 *
 * Conventions (shared with fbcorr.h: status codes, error messages, tuning
 * report, thread rules):
 *  - Patches are rows of D unsigned 8-bit pixels, C order: targets[T][D],
 *    neighbors[M][D].  D is a multiple of 16 in [16, 512] (64 for 8 x 8
 *    patches).  Outputs idx[T] and dist[T] are int32: dist is the squared
 *    distance (at most 65025 * D, exact), idx the neighbour row.
 *  - The result is exact and deterministic: all arithmetic is integer, and
 *    ties go to the lowest index, as in a sequential scan.
 *  - Kernels are generated and compiled at plan time with hiprtc from the
 *    problem (T, M, D) and a configuration, cached like the correlation
 *    kernels, and tuned by fbnn_tune; the tuning database keys them as
 *    "<arch> nearest u8 <T> <M> <D>".
 *  - All pointers passed to fbnn_search are device pointers, 16-byte
 *    aligned; the caller owns them.  The library allocates no device memory
 *    during a search: the caller passes a workspace of at least
 *    fbnn_workspace_size() bytes.  Work is enqueued on the caller's stream
 *    (a hipStream_t passed as void*; NULL = the default stream); nothing is
 *    synchronised.
 */
#ifndef FBNN_H
#define FBNN_H

#include "fbcorr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fbnn_desc {
    int64_t n_targets;     /* T >= 0 (T = 0: a search does nothing) */
    int64_t n_neighbors;   /* M >= 1, M + 16 < 2^31 */
    int32_t dim;           /* D: bytes per patch, multiple of 16, 16..512 */
    int32_t flags;         /* must be 0 */
} fbnn_desc;

typedef struct fbnn_plan_s* fbnn_plan_t;

/* Create a plan on HIP device `device`: validates the descriptor, picks the
 * configuration (tuning database, else a heuristic) and compiles the five
 * kernels (neighbour norms, prefix sums, parity partition, scan, final
 * selection).  FBCORR_ERR_INVALID_ARGUMENT for a bad descriptor,
 * FBCORR_ERR_NO_DEVICE, FBCORR_ERR_UNSUPPORTED for a device that is not
 * gfx950 or more rows than the index type holds, FBCORR_ERR_COMPILE with the
 * hiprtc log. */
FBCORR_API fbcorr_status fbnn_plan(const fbnn_desc* desc, int device, fbnn_plan_t* out);
FBCORR_API fbcorr_status fbnn_plan_destroy(fbnn_plan_t plan);

/* Workspace bytes for pass 0 = fbnn_search, 1 = fbnn_tune.  Depends on the
 * configuration (the number of neighbour chunks). */
FBCORR_API fbcorr_status fbnn_workspace_size(fbnn_plan_t plan, int pass, size_t* bytes);

/* Nearest neighbour of every target.  targets [T][D] and neighbors [M][D]
 * (uint8), idx [T] and dist [T] (int32), workspace of fbnn_workspace_size(0)
 * bytes; all device pointers, 16-byte aligned.  Enqueues five kernels on
 * `stream`.  FBCORR_ERR_INVALID_ARGUMENT for NULL or misaligned pointers,
 * FBCORR_ERR_WORKSPACE for a short workspace, FBCORR_ERR_LAUNCH if HIP
 * refuses a launch (the plan is then not guaranteed usable). */
FBCORR_API fbcorr_status fbnn_search(fbnn_plan_t plan, const uint8_t* targets, const uint8_t* neighbors,
                                     int32_t* idx, int32_t* dist, void* workspace, size_t workspace_bytes,
                                     void* stream);

/* Auto-tuning (Sec. 4.1 and 6.2 applied to this search): enumerates
 * configurations (targets per wave, waves per workgroup, neighbour chunk
 * length, tiles per tracking group, load-ahead), compiles them in
 * parallel, requires each to return the default's idx and dist bit for bit
 * on the caller's data, times the survivors with HIP events (median of
 * opts->reps) and installs the fastest.
 * opts->role is ignored; opts->flags bit 1 records the winner in the tuning
 * database.  Synchronises `stream`. */
FBCORR_API fbcorr_status fbnn_tune(fbnn_plan_t plan, const uint8_t* targets, const uint8_t* neighbors,
                                   void* workspace, size_t workspace_bytes, void* stream,
                                   const fbcorr_tune_opts* opts, fbcorr_tune_report* report);

/* Configuration text ("algo=nn ch=512 nt=4 ..."); set_config compiles the
 * given keys over the current configuration, keeping it on any error. */
FBCORR_API fbcorr_status fbnn_plan_get_config(fbnn_plan_t plan, char* buf, size_t len);
FBCORR_API fbcorr_status fbnn_plan_set_config(fbnn_plan_t plan, const char* cfg);

/* Kernel timing with HIP events on the caller's stream: ms[0..2] = total
 * milliseconds of the neighbour preparation (norms, prefix sums, parity
 * partition: three kernels), the scan kernel and the final selection;
 * calls[0..2] = searches timed.  read_timing synchronises the events. */
FBCORR_API fbcorr_status fbnn_plan_enable_timing(fbnn_plan_t plan, int enable);
FBCORR_API fbcorr_status fbnn_plan_read_timing(fbnn_plan_t plan, double* ms, int64_t* calls, int reset);

/* Generate and compile (hiprtc, no device needed) the five kernels of a
 * descriptor and configuration for `arch` (NULL = "gfx950"); reports the
 * total code-object size.  Host-only. */
FBCORR_API fbcorr_status fbnn_compile_check(const fbnn_desc* desc, const char* cfg, const char* arch,
                                            size_t* code_bytes);

#ifdef __cplusplus
}
#endif

#endif /* FBNN_H */
