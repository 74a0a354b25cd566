/*
 * fbcorr — run-time-specialised multi-channel 2-D filter-bank correlation
 * for AMD Instinct MI355X (gfx950).
 *
 * The operation is the "3D filter-bank convolution" that the Computational
 * Visual Neuroscience application (Sec. 6.2) generates and auto-tunes at run
 * time, with the shapes of the table "Performance of RTCG auto-tuning on 3D
 * filter-bank convolutions": a bank of N filters, each fh x fw x D and
 * spanning the full input depth, slid over an H x W x D input:
 *
 *   y[b,i,j,n] = sum_{u<fh} sum_{v<fw} sum_{d<D} x[b,i+u,j+v,d] * w[n,u,v,d]
 *
 * for 0 <= i < Ho = H-fh+1, 0 <= j < Wo = W-fw+1 (valid extent, stride one,
 * no flip).  The paper states the operation only in words and by shape;
 * these readings are the library's contract.
 *
 * Following the paper's method (Sec. 4.1 automated tuning, Sec. 4.2 the cost
 * of flexibility, Sec. 5 and Fig. 2 the compile cache, Sec. 5.3 keyword
 * substitution), every kernel is HIP source compiled at plan time by hiprtc
 * for the device's architecture with the filter size, depth, bank size,
 * tile shape and unroll factors substituted as compile-time constants; code
 * objects are cached in-process by (source, options, architecture, compiler
 * version).  fbcorr_tune times retained variants and keeps the fastest.
 *
 * Conventions for every entry point below:
 *  - Layouts are C-contiguous float32: x[batch][H][W][D], w[N][fh][fw][D],
 *    y and dy[batch][Ho][Wo][N], dx like x, dw like w.
 *  - Tensor pointers are DEVICE pointers, 16-byte aligned, owned by the
 *    caller, and must stay valid until the work queued on `stream` is done.
 *    The library never allocates device memory for them; scratch space is
 *    the caller's workspace of at least fbcorr_workspace_size() bytes
 *    (16-byte aligned; NULL is allowed when that size is 0).
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Kernels are queued on it asynchronously.
 *  - Accumulation is always float32.  Results never depend on timing: there
 *    are no floating-point atomics, and every reduction has a fixed order.
 *  - Errors are reported, never fatal (Sec. 5: errors are detected and
 *    turned into recoverable conditions).  A call returns a status; the
 *    calling thread's fbcorr_last_error() then holds a message.  After any
 *    status other than FBCORR_ERR_LAUNCH the plan stays usable.
 *  - A plan may be used from several threads at once on different streams
 *    with separate workspaces, except during fbcorr_tune,
 *    fbcorr_plan_set_config and fbcorr_plan_set_epilogue.
 */
#ifndef FBCORR_H
#define FBCORR_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define FBCORR_API __attribute__((visibility("default")))
#else
#define FBCORR_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fbcorr_status {
    FBCORR_OK = 0,
    FBCORR_ERR_INVALID_ARGUMENT = 1, /* null handle/pointer, size <= 0, misaligned pointer */
    FBCORR_ERR_SHAPE = 2,            /* filter larger than the input, batch/depth mismatch */
    FBCORR_ERR_UNSUPPORTED = 3,      /* combination not provided (e.g. a configuration that does not fit) */
    FBCORR_ERR_COMPILE = 4,          /* hiprtc failed; the log is in fbcorr_last_error() */
    FBCORR_ERR_LAUNCH = 5,           /* a HIP call failed (launch, event, graph, module load) */
    FBCORR_ERR_WORKSPACE = 6,        /* workspace smaller than fbcorr_workspace_size() */
    FBCORR_ERR_NO_DEVICE = 7,        /* no usable HIP device / device index out of range */
    FBCORR_ERR_INTERNAL = 8
} fbcorr_status;

/* Operand precision.  Accumulation and outputs are float32 in every mode.
 * BF16 and FP16 round x and w to nearest-even after scaling each filter by a
 * power of two, s_n = 2^-floor(log2 max|w[n]|), and divide the accumulated
 * result by s_n again (exact).  FP16 inputs keep their full float32 range:
 * every FP16 forward first takes max|x| over the whole input (an extra read
 * of x), and when it reaches 2^15 the input is scaled by 2^-k while staged
 * (max|x| * 2^-k < 2^15) and the outputs by 2^k, both exact; below 2^15
 * (k = 0) nothing changes.  Values that the scale pushes below fp16's
 * subnormal range round to zero, as any fp16 rounding would at that
 * magnitude relative to the tensor's maximum.  Inputs must be finite. */
typedef enum fbcorr_precision {
    FBCORR_FP32 = 0,
    FBCORR_BF16 = 1,
    FBCORR_FP16 = 2
} fbcorr_precision;

/* Forward algorithm.  DIRECT: vector-ALU kernel, each thread accumulating a
 * block of outputs from LDS-staged input tiles and filter slices.  IGEMM:
 * implicit GEMM on the matrix cores, C[pixel, filter] = A[pixel, (u,v,d)] *
 * B[(u,v,d), filter], with A gathered from LDS-staged input tiles and never
 * materialised; two kernels implement it (configuration algo=igemm: filter
 * slices staged through LDS; algo=rgemm: filters repacked in matrix-core
 * fragment order and streamed from L2 into registers), the tuning database
 * or fbcorr_plan_set_config picks one.  AUTO: the tuned choice, else IGEMM. */
typedef enum fbcorr_algo {
    FBCORR_ALGO_AUTO = 0,
    FBCORR_ALGO_DIRECT = 1,
    FBCORR_ALGO_IGEMM = 2
} fbcorr_algo;

/* Problem descriptor.  batch >= 1 images share one filter bank. */
typedef struct fbcorr_desc {
    int32_t batch, H, W, D, N, fh, fw;
    int32_t precision; /* fbcorr_precision */
    int32_t algo;      /* fbcorr_algo */
    uint32_t flags;    /* FBCORR_FLAG_* bits; others must be 0 */
} fbcorr_desc;

/* fbcorr_backward with both gradients runs dW on a plan-owned side stream
 * (default priority), forked from and joined back into the caller's stream,
 * concurrently with dX.  Off by default: the kernels then run one after the
 * other on the caller's stream, so each one's time is its own. */
#define FBCORR_FLAG_OVERLAP_BACKWARD 1u

typedef struct fbcorr_plan_s* fbcorr_plan_t;

/* Kernel roles inside a plan (for configuration strings and timing). */
typedef enum fbcorr_role {
    FBCORR_ROLE_FORWARD = 0,   /* the forward correlation kernel */
    FBCORR_ROLE_BACKWARD_X = 1,/* the input-gradient kernel */
    FBCORR_ROLE_BACKWARD_W = 2,/* the filter-gradient split-K kernel */
    FBCORR_ROLE_COUNT = 3
} fbcorr_role;

/* Options and report of fbcorr_tune.  Zero fields take the defaults
 * (warmup 2, reps 10, no candidate limit). */
typedef struct fbcorr_tune_opts {
    int32_t warmup, reps;
    int32_t max_candidates;
    int32_t role;      /* fbcorr_role to tune */
    uint32_t flags;    /* bit 0: also try the DIRECT algorithm for the forward role;
                          bit 1: record the winner in the tuning database;
                          bit 2: tune the DIRECT algorithm only (fp32 forward) */
} fbcorr_tune_opts;

typedef struct fbcorr_tune_report {
    int32_t n_tried, n_compiled, n_rejected_resources, n_rejected_parity, n_failed;
    double best_ms, default_ms;
    char best_cfg[256];
    char default_cfg[256];
} fbcorr_tune_report;

/* ---- plans --------------------------------------------------------------
 * fbcorr_plan: validates the descriptor (Sec. 6.2's operation; any dim <= 0
 * -> INVALID_ARGUMENT, fh > H or fw > W -> SHAPE), selects default kernel
 * configurations, generates their source and compiles them with hiprtc for
 * `device` (cached), and loads them.  Default configurations come from the
 * tuning database (Sec. 6.2: ship a database of configurations per
 * platform; file tuning_db.txt beside the library or $FBCORR_TUNING_DB,
 * lines "<arch> <role> <precision> <batch> <H> <W> <D> <N> <fh> <fw> :
 * <config>"), else from built-in heuristics.  The plan owns host state; the
 * compiled modules belong to the process-wide cache.  *out is written only
 * on success. */
FBCORR_API fbcorr_status fbcorr_plan(const fbcorr_desc* desc, int device, fbcorr_plan_t* out);

/* Releases a plan (Sec. 5: resources can be released explicitly).  All work
 * queued with the plan must have completed.  NULL is accepted. */
FBCORR_API fbcorr_status fbcorr_plan_destroy(fbcorr_plan_t plan);

/* Bytes of workspace needed by a pass: pass 0 = forward, pass 1 = backward
 * (both gradients), pass 2 = fbcorr_tune (any role).  The value depends on the plan's current configuration
 * and may change after fbcorr_tune or fbcorr_plan_set_config. */
FBCORR_API fbcorr_status fbcorr_workspace_size(fbcorr_plan_t plan, int pass, size_t* bytes);

/* ---- compute ------------------------------------------------------------
 * fbcorr_forward: y = correlation(x, w) as defined at the top of this file.
 * x, w, y: device pointers in the layouts above. */
FBCORR_API fbcorr_status fbcorr_forward(fbcorr_plan_t plan, const float* x, const float* w, float* y,
                             void* workspace, size_t workspace_bytes, void* stream);

/* fbcorr_forward_noalloc: fbcorr_forward for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Runs the same kernels with the
 * forward role's scratch -- the packed filter bank of the 16-bit and
 * register-streamed matrix-core kernels, or the tap-major filter copy of the
 * direct kernel's scalar-weight variant -- taken from a static device array
 * of 16 MiB instead of a caller workspace; it calls no allocator.  Each GPU
 * the library runs on holds its own array until the process ends (its
 * address is looked up once per device, on the first call there).  Every
 * call on one GPU shares that GPU's array: calls whose work overlaps on one
 * GPU (other streams, other threads, other plans) race and must be
 * serialised by the caller.  The kernels write every scratch byte they
 * read, so nothing needs clearing between calls.  A plan whose forward role
 * needs more than 16 MiB of scratch (fbcorr_workspace_size pass 0) gets
 * FBCORR_ERR_WORKSPACE and nothing is launched.  x, w, y as for
 * fbcorr_forward. */
FBCORR_API fbcorr_status fbcorr_forward_noalloc(fbcorr_plan_t plan, const float* x, const float* w, float* y,
                                                void* stream);

/* fbcorr_backward: gradients of L = sum(dy * y) (the adjoint of the forward
 * map; the paper has no backward pass):
 *   dx[b,p,q,d] = sum_n sum_{u,v: 0<=p-u<Ho, 0<=q-v<Wo} dy[b,p-u,q-v,n] * w[n,u,v,d]
 *   dw[n,u,v,d] = sum_b sum_{i<Ho,j<Wo} dy[b,i,j,n] * x[b,i+u,j+v,d]
 * dx or dw may be NULL to skip that gradient (x may then be NULL when dw is
 * NULL).  Always float32 operands. */
FBCORR_API fbcorr_status fbcorr_backward(fbcorr_plan_t plan, const float* x, const float* w, const float* dy,
                              float* dx, float* dw, void* workspace, size_t workspace_bytes,
                              void* stream);

/* fbcorr_tune: automated tuning (Sec. 4.1; Sec. 6.2's coarse grid search
 * over unroll depth, block dimensions, thread work size and shared-memory
 * padding).  For the role in opts (forward if opts is NULL) it enumerates a
 * grid of configurations, drops those that do not fit the device (LDS,
 * registers), compiles the rest, checks each candidate's output bit for bit
 * against the plan's default configuration on integer-valued data it
 * generates itself, times the survivors with HIP events on `stream`
 * (synchronising it), and installs the fastest.  Uses the caller's buffers:
 * for the forward role x, w, y (y is overwritten); for the backward roles
 * x, w, y (as dy) and ws.  Their contents are preserved except y.  With the
 * environment variable FBCORR_TUNE_PROGRESS=1 the tuner prints a progress
 * line to stderr every 25 candidates compiled and timed. */
FBCORR_API fbcorr_status fbcorr_tune(fbcorr_plan_t plan, const float* x, const float* w, float* y,
                          void* workspace, size_t workspace_bytes, void* stream,
                          const fbcorr_tune_opts* opts, fbcorr_tune_report* report);

/* ---- many uneven images in one launch ----------------------------------
 * fbcorr_plan_batched: `count` independent problems (each desc has batch 1,
 * its own H, W, D, N, fh, fw and its own filter bank; FP32 only).  One
 * persistent kernel is generated holding exactly the variants the distinct
 * (fh, fw, D, N) keys need (Sec. 4.2: code for exactly one purpose); a work
 * table of tiles sorted by cost is built at plan time. */
FBCORR_API fbcorr_status fbcorr_plan_batched(int32_t count, const fbcorr_desc* descs, int device,
                                  fbcorr_plan_t* out);

/* fbcorr_forward_batched: xs, ws_, ys are DEVICE arrays of `count` device
 * pointers (the i-th problem's x, w, y).  use_graph != 0 captures the launch
 * into a HIP graph on the first call per stream (which must be a created
 * stream, not the null stream) and replays it afterwards;
 * the pointer arrays are then read at replay time, so their contents may
 * change between calls but their addresses and the workspace must not.
 * The plan's work table lives in the workspace: it is written on the first
 * call with a given workspace address (synchronously), so that memory must
 * not be reused for anything else while the plan uses it.  Calls from
 * several threads are serialised inside the plan. */
FBCORR_API fbcorr_status fbcorr_forward_batched(fbcorr_plan_t plan, const float* const* xs,
                                     const float* const* ws_, float* const* ys,
                                     void* workspace, size_t workspace_bytes, void* stream,
                                     int use_graph);

/* ---- introspection, configuration, timing ------------------------------ */

/* Text form of the configuration of `role` ("algo=igemm th=4 nt=2 ..."). */
FBCORR_API fbcorr_status fbcorr_plan_get_config(fbcorr_plan_t plan, int role, char* buf, size_t len);

/* Replace the configuration of `role` by one given in the same text form
 * (keys not given keep their defaults).  Compiles it; on any error the
 * previous configuration stays in place. */
FBCORR_API fbcorr_status fbcorr_plan_set_config(fbcorr_plan_t plan, int role, const char* cfg);

/* Fused elementwise epilogue for the forward pass (the static nonlinearity
 * that follows each filtering layer in the vision model family of Sec. 6.2,
 * Fig. 5b), generated into the forward kernel's store like the paper's
 * elementwise kernels (Sec. 5.2, Fig. 4): `expr` is a single-line C
 * expression of `v` (the float output value) and `c` (its filter index),
 * e.g. "fminf(fmaxf(v, 0.f), 1.f)".  NULL or "" removes it.  The forward
 * kernel is recompiled; a compile error leaves the previous kernel in place
 * (FBCORR_ERR_COMPILE with the log).  Plans with an epilogue have no
 * backward pass (FBCORR_ERR_UNSUPPORTED). */
FBCORR_API fbcorr_status fbcorr_plan_set_epilogue(fbcorr_plan_t plan, const char* expr);

/* Kernel timing: when enabled, the library records HIP events around all
 * the kernels of each role (filter preparation, the main kernel, and for
 * the filter gradient the fixed-order sum of the partials) on the stream
 * they are launched on, and accumulates the elapsed time when
 * fbcorr_plan_read_timing is called (which synchronises the events).
 * ms[role] = total milliseconds, calls[role] = role executions.  A batched
 * plan records role 0 around its persistent kernel (eager launches) or its
 * graph launch. */
FBCORR_API fbcorr_status fbcorr_plan_enable_timing(fbcorr_plan_t plan, int enable);
FBCORR_API fbcorr_status fbcorr_plan_read_timing(fbcorr_plan_t plan, double* ms, int64_t* calls, int reset);

/* Generate (without compiling) the HIP source and compile options of a role
 * for a descriptor and configuration; writes NUL-terminated text.  Host-only;
 * needs no device.  *len is set to the bytes required. */
FBCORR_API fbcorr_status fbcorr_codegen(const fbcorr_desc* desc, int role, const char* cfg,
                             char* source, size_t* source_len, char* options, size_t* options_len);

/* Compile a role's kernel for an architecture name (e.g. "gfx950") with
 * hiprtc, without a device, and report the code-object size.  Host-only. */
FBCORR_API fbcorr_status fbcorr_compile_check(const fbcorr_desc* desc, int role, const char* cfg,
                                   const char* arch, size_t* code_bytes);

/* Generate and compile the persistent batched kernel for `count`
 * descriptors (as fbcorr_plan_batched would) for an architecture name,
 * without a device.  Host-only. */
FBCORR_API fbcorr_status fbcorr_compile_check_batched(int32_t count, const fbcorr_desc* descs, const char* arch,
                                                      size_t* code_bytes);

/* Code-object cache statistics: in-memory hits, compilations (misses),
 * in-memory entries, and entries read from the on-disk cache.  The on-disk
 * cache (Fig. 2: compiled code is kept across runs and reused while source
 * and environment are unchanged) lives in $FBCORR_CACHE_DIR, else in
 * _rtc_cache/ beside the library; FBCORR_CACHE=0 disables it.  Entries are
 * checksummed; a damaged entry is recompiled and rewritten. */
FBCORR_API fbcorr_status fbcorr_cache_stats(int64_t* hits, int64_t* misses, int64_t* entries, int64_t* disk_hits);

/* Drop the in-memory code-object cache (loaded modules stay valid) and
 * re-read the tuning database on next use. */
FBCORR_API fbcorr_status fbcorr_cache_clear(void);

FBCORR_API const char* fbcorr_last_error(void);              /* thread-local; valid until the next call */
FBCORR_API const char* fbcorr_status_string(fbcorr_status s);
FBCORR_API int fbcorr_version(void);                          /* major*10000 + minor*100 + patch */

#ifdef __cplusplus
}
#endif

#endif /* FBCORR_H */
