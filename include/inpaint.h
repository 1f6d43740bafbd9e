/*
 * inpaint.h -- C ABI of libinpaint.so: exemplar-based object removal
 * (Criminisi-style best-first patch filling) on AMD Instinct MI355X (gfx950).
 *
 * The method (paper, Section 3): a source image S has a target region (hole)
 * Omega to fill; Phi = S - Omega is the known region.  Each iteration
 *   1. finds the fill front dOmega (hole pixels next to known pixels),
 *   2. scores each front pixel p with the priority P(p) = C(p) * D(p)
 *      (confidence term times data term, Eq. 1 and Eq. 2) and takes the
 *      maximum,
 *   3. searches the source region for the patch that minimises the sum of
 *      squared RGB differences to the known pixels of the patch around p
 *      (findBestPatch, Eq. 3 and Eq. 4),
 *   4. copies that patch's pixels into the hole pixels of p's patch, which
 *      take p's confidence,
 * until the hole is empty.  The search may be restricted to a window around
 * the hole (search factor alpha, Section 5.3, Eq. 6).
 *
 * Conventions for every call:
 *   - Every function returns an int32_t status (INPAINT_OK, INPAINT_DONE or a
 *     negative error).  Outputs are written only on success.  No C++
 *     exception crosses the ABI.
 *   - Pixel (x, y) has raster index y * width + x.  Rectangles are half-open
 *     [x0, x1) x [y0, y1).
 *   - A patch has radius r (1 <= r <= 8) and side P = 2r + 1.
 *   - Device memory passed in (workspaces) is owned by the caller and must
 *     outlive the object using it; host buffers are only read or written
 *     during the call.
 *   - All device work of a context is enqueued on the hipStream_t given at
 *     creation.  Calls documented as synchronising wait for that stream.
 *   - A context or batch must not be used by two threads at once; distinct
 *     contexts may be used concurrently from different threads.
 *   - INPAINT_DEVICE is sticky: after a device error the context only
 *     accepts inpaint_destroy and inpaint_last_error.
 *
 * Exact-arithmetic contract: exemplar indices, SSDs and output images are
 * bit-exact integers; priorities are IEEE binary64 computed in one fixed
 * operation order with no fused multiply-add, so the fill order is
 * reproducible on any IEEE machine that follows the same order.
 */
#ifndef INPAINT_H
#define INPAINT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define INPAINT_OK                0
#define INPAINT_DONE              1   /* not an error: the hole is empty      */
#define INPAINT_INVALID_ARGUMENT (-1)
#define INPAINT_NO_CANDIDATE     (-2) /* no valid source centre in the rect   */
#define INPAINT_OUT_OF_MEMORY    (-3) /* workspace too small / host alloc     */
#define INPAINT_DEVICE           (-4) /* HIP error; the context is unusable   */

/* ------------------------------------------------------------- parameters */
#define INPAINT_SEARCH_FULL  0   /* every valid centre of the image          */
#define INPAINT_SEARCH_ALPHA 1   /* window around the hole, Eq. 6            */
#define INPAINT_SEARCH_RECT  2   /* caller-given rectangle of centres        */

/* Execution forms of inpaint_run.  PLAIN, STREAM and GRAPH run the same two
 * kernels per iteration (exemplar search, then commit) and differ in how the
 * host drives them; kernels skip their work once the hole is empty or the
 * iteration limit is reached, so overshooting a batch of iterations is
 * harmless.  PERSISTENT runs up to iters_per_check whole iterations inside
 * one dispatch whose work-groups are all resident at once: one work-group
 * commits while the others keep their search tiles resident in LDS and
 * score every target in turn, with no kernel boundary between search and
 * commit.  When the tiles outnumber the work-groups that fit on the device,
 * each search work-group takes several tiles (up to 64).  It needs the
 * default candidate domain (and the SIMT path with tile_rows 8); otherwise
 * inpaint_run uses STREAM instead -- inpaint_run_form tells which.
 * Persistent dispatches of one process never overlap (the library
 * serialises them; each call waits for its dispatch's end). */
#define INPAINT_FORM_PLAIN  0    /* launch one iteration, host check, repeat  */
#define INPAINT_FORM_STREAM 1    /* enqueue iters_per_check iterations, check */
#define INPAINT_FORM_GRAPH  2    /* replay a hipGraph of iters_per_check      */
#define INPAINT_FORM_PERSISTENT 3 /* one dispatch of iters_per_check, check  */

#define INPAINT_PATH_AUTO 0
#define INPAINT_PATH_SIMT 1      /* integer dot-product SSD on the VALU      */
#define INPAINT_PATH_MFMA 2      /* int8 matrix-core cross term (exact)      */
/* The SIMT search with no LDS staging: each lane reads its source words from
 * device memory through the vector caches, as the paper's kernel without
 * local memory does (Alg. 1, against the local-memory kernel of Alg. 2).
 * Same results; slower.  It exists for that comparison: PLAIN, STREAM and
 * GRAPH forms only (PERSISTENT runs as STREAM), and inpaint_batch_step
 * searches every attached job with the staged kernel. */
#define INPAINT_PATH_SIMT_DIRECT 3

/* Candidate domain of the exemplar search.  The default reads Eq. 4 as
 * Criminisi does: a candidate's whole window lies in the image and in the
 * ORIGINAL known region Phi_0, so filled pixels never become sources.  The
 * paper's own wording allows two other readings, which these fields select.
 *
 * source_policy CURRENT: the source region is the current known region
 *   (Section 3 defines Phi = S - Omega, and Omega shrinks as the fill
 *   proceeds), so filled pixels become sources.  It is evaluated on the
 *   state at the start of each iteration.
 * scoring INTERSECT: Eq. 4 read literally, as Section 5.4 describes for
 *   candidates that overlap the object.
 *   - A candidate is any centre of the search rect that is itself a source
 *     pixel; its window may overlap the hole or leave the image.
 *   - Its SSD runs over the offsets where the target pixel is known and the
 *     candidate pixel is in the image and in the source region.
 *   - The copy fills only the target's hole pixels whose source pixel
 *     qualifies; the others stay in the hole for a later iteration.
 *
 * The two fields combine freely.  Any non-default value needs the SIMT
 * search (path SIMT, SIMT_DIRECT or AUTO; MFMA gives INVALID_ARGUMENT) and
 * runs in the PLAIN, STREAM or GRAPH form (PERSISTENT runs as STREAM).
 * Such a context cannot be attached to a batch. */
#define INPAINT_SOURCE_ORIGINAL 0
#define INPAINT_SOURCE_CURRENT  1
#define INPAINT_SCORE_WHOLE     0
#define INPAINT_SCORE_INTERSECT 1

typedef struct {
    const uint8_t *data;   /* host pixels, row-major, 8 bits per channel     */
    int32_t width;
    int32_t height;
    int32_t stride_bytes;  /* bytes between rows (>= width * channels)       */
    int32_t channels;      /* 3 (RGB) or 4 (RGBA/RGBX; the 4th is ignored)  */
} inpaint_image;

typedef struct {
    int32_t x0, y0, x1, y1;   /* half-open, in candidate-centre coordinates */
} inpaint_rect;

typedef struct {
    int32_t patch_radius;  /* r, 1..8; the paper's patch size P = 2r + 1     */
    int32_t search_mode;   /* INPAINT_SEARCH_*                               */
    int32_t alpha_num;     /* search factor alpha = alpha_num / alpha_den,  */
    int32_t alpha_den;     /*   used by INPAINT_SEARCH_ALPHA (alpha >= 0)   */
    inpaint_rect rect;     /* used by INPAINT_SEARCH_RECT; clipped to image */
    int32_t path;          /* INPAINT_PATH_*                                 */
    int32_t form;          /* inpaint_run execution form, INPAINT_FORM_*     */
    int32_t iters_per_check; /* STREAM / GRAPH forms: iterations enqueued   */
                           /*   (or replayed as one hipGraph) between two   */
                           /*   host checks of termination; PERSISTENT:     */
                           /*   iterations per dispatch (1 .. 33554430)     */
    int32_t log_capacity;  /* device log records kept (>= 0), one per fill   */
                           /*   iteration; -1 = width*height, enough for    */
                           /*   any mask (a removal never needs more than   */
                           /*   its hole-pixel count)                       */
    int32_t tile_rows;     /* search tile: candidate rows per thread (0 =   */
                           /*   default; 4, 8 or 16)                        */
    int32_t source_policy; /* INPAINT_SOURCE_* (0 = ORIGINAL, the default)  */
    int32_t scoring;       /* INPAINT_SCORE_* (0 = WHOLE, the default)      */
    int32_t reserved[1];   /* must be zero                                   */
} inpaint_params;

/* One fill iteration (64 bytes). */
typedef struct {
    int64_t target_index;  /* front pixel p^ that was filled                 */
    int64_t source_index;  /* centre q^ of the copied source patch           */
    uint32_t ssd;          /* d(Psi_p^, Psi_q^), Eq. 4                        */
    int32_t known_k;       /* known pixels in the target patch               */
    int32_t n_filled;      /* hole pixels filled                             */
    int32_t reserved;
    double priority;       /* P(p^) = C(p^) D(p^)                             */
    double confidence;     /* C(p^)                                          */
    double data_term;      /* D(p^)                                          */
    int64_t remaining;     /* hole pixels left after this iteration          */
} inpaint_step_info;

typedef struct inpaint_ctx inpaint_ctx;
typedef struct inpaint_batch inpaint_batch;

/* ----------------------------------------------------------- single image */

/* Device bytes one job of width x height with params *p needs; this is also
 * its footprint for admission in a serving loop.  INVALID_ARGUMENT for sizes
 * below the patch or a bad radius. */
int32_t inpaint_workspace_bytes(int32_t width, int32_t height, const inpaint_params *p,
                                uint64_t *bytes);

/* Initialisation stage (Section 4.2): uploads the image and the mask
 * (nonzero = pixel of the object to remove, i.e. the hole Omega_0) into the
 * caller's device workspace, zeroes the hole pixels, builds the gray image,
 * the confidence map (1 on the known region, 0 in the hole), the validity map
 * of source centres (whole patch inside the image and inside the ORIGINAL
 * known region) and the initial priorities, and selects the first target.
 * The host buffers may be freed on return.  d_workspace must be 256-byte
 * aligned, at least inpaint_workspace_bytes large, and stay allocated until
 * inpaint_destroy.  hip_stream is a hipStream_t (NULL = default stream).
 * Synchronises.  Errors: INVALID_ARGUMENT (bad sizes or params, empty hole,
 * no known pixel, no valid source centre in the search rectangle),
 * OUT_OF_MEMORY (workspace too small), DEVICE (also when the hole the
 * device counted in the uploaded mask, or its bounding box, differs from
 * the caller's mask: the initialisation did not read the caller's bytes). */
int32_t inpaint_create(const inpaint_image *img, const uint8_t *mask, int32_t mask_stride,
                       const inpaint_params *p, void *d_workspace, uint64_t ws_bytes,
                       void *hip_stream, inpaint_ctx **out);

/* findBestPatch (Alg. 1, Eq. 3-4) as a pure query on the current state: the
 * centre q in search_rect (clipped to the image) whose whole patch of radius
 * patch_radius lies in the image and the original known region, minimising
 * the SSD over R, G, B of the target patch's known pixels; ties go to the
 * lowest raster index.  Does not change the state.  Synchronises.
 * Errors: INVALID_ARGUMENT (target outside the image, radius out of 1..8,
 * x0 > x1 or y0 > y1), NO_CANDIDATE (no valid centre in the rect). */
int32_t inpaint_find_exemplar(inpaint_ctx *ctx, int32_t target_x, int32_t target_y,
                              int32_t patch_radius, inpaint_rect search_rect,
                              int64_t *source_index, uint32_t *ssd);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * query as inpaint_find_exemplar, same arguments, results and errors, but
 * its scratch (target stage, one partial minimum per search tile, result
 * key) lives in a static device array of the library (258 KiB, one per GPU,
 * held until the process ends) instead of the context's workspace.  The
 * call allocates nothing.  A search rect that needs more
 * than 32768 search tiles (about 67 M candidate centres with the default
 * SIMT tile, 134 M with the MFMA tile) is rejected with INVALID_ARGUMENT.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two threads, or two streams) race and must not be issued; it keeps
 * only the last call's contents, none of which a call reads before writing.
 * Synchronises. */
int32_t inpaint_find_exemplar_static(inpaint_ctx *ctx, int32_t target_x, int32_t target_y,
                                     int32_t patch_radius, inpaint_rect search_rect,
                                     int64_t *source_index, uint32_t *ssd);

/* One iteration of the fill loop of Section 3: compute the fill front, take
 * the front pixel of maximum priority P = C D (Eq. 1-2; ties to the lowest
 * raster index), find its best exemplar (Eq. 3-4) in the context's search
 * rectangle, copy the exemplar into the target's hole pixels and give them
 * the target's confidence.  Fills *info (may be NULL).  Returns INPAINT_DONE
 * without work if the hole is already empty.  Synchronises. */
int32_t inpaint_step(inpaint_ctx *ctx, inpaint_step_info *info);

/* The fill loop of Section 3 (repeat the iteration of inpaint_step until the
 * target region is empty; at most |Omega_0| iterations, Section 5.4 gives
 * their rough count).  Iterates until the hole is empty or max_iters
 * iterations (max_iters < 0:
 * no limit) have run, in the form chosen by params.form.  Writes the
 * number of iterations run to *iters_done and, when log is not NULL, the
 * first min(log_cap, iterations, log capacity) records of this call.  Returns
 * INPAINT_DONE when the hole is empty, INPAINT_OK when stopped by max_iters.
 * Synchronises. */
int32_t inpaint_run(inpaint_ctx *ctx, int64_t max_iters, int64_t *iters_done,
                    inpaint_step_info *log, int64_t log_cap);

/* Records [first, first + count) of the device log (records are numbered from
 * the context's first iteration).  INVALID_ARGUMENT if outside what the log
 * holds.  Synchronises. */
int32_t inpaint_read_log(inpaint_ctx *ctx, int64_t first, int64_t count, inpaint_step_info *out);

/* Copies the current RGB image to host rows of `stride` bytes (3 bytes per
 * pixel).  Synchronises. */
int32_t inpaint_read_image(inpaint_ctx *ctx, uint8_t *rgb, int32_t stride);

/* Copies the current hole (1 = still to fill) and confidence maps, each
 * width*height row-major; either pointer may be NULL.  Synchronises. */
int32_t inpaint_read_state(inpaint_ctx *ctx, uint8_t *mask, double *conf);

/* Hole pixels still to fill.  Synchronises. */
int32_t inpaint_remaining(inpaint_ctx *ctx, int64_t *remaining);

/* Iterations committed so far and hole pixels left (either may be NULL).
 * Synchronises. */
int32_t inpaint_progress(inpaint_ctx *ctx, int64_t *iterations, int64_t *remaining);

/* Resume / iterative editing (the interactive workflow of Section 6).
 * Replaces the fill state of `ctx` by a checkpoint of the same removal, as
 * inpaint_read_image, inpaint_read_state and inpaint_progress return it:
 *   - the image: `rgb`, rows of `rgb_stride` bytes, `channels` 3 or 4;
 *   - the hole still to fill: `hole`, nonzero = to fill, rows of
 *     `hole_stride` bytes;
 *   - the confidence map: `conf`, width*height doubles, row-major;
 *   - `iterations` already done.
 * Continuing from it gives exactly what the uninterrupted run gives: the
 * same fill order, with log records numbered from `iterations` on (size
 * log_capacity for the whole removal).
 *
 * Only pixels of the context's original hole change: those still in the
 * checkpoint's hole become hole again, and the others take the checkpoint's
 * colour and confidence.  Pixels outside the original hole keep the values
 * given at create, so a context created from the checkpoint image and the
 * original mask can resume.  Host inputs are copied.  Legal between runs on
 * a context not attached to a batch.
 *
 * Errors: INVALID_ARGUMENT, with the state unchanged, if
 *   - the hole leaves the original hole;
 *   - a filled pixel's confidence is not in [0, 1];
 *   - iterations < 0;
 *   - a pointer is NULL, channels is wrong or a stride is too small.
 * DEVICE (sticky) if a kernel did not run to completion, or if the hole the
 * device counted after the overlay differs from the caller's hole map (the
 * import did not read the caller's bytes).
 * Synchronises. */
int32_t inpaint_import_state(inpaint_ctx *ctx, const uint8_t *rgb, int32_t rgb_stride, int32_t channels,
                             const uint8_t *hole, int32_t hole_stride, const double *conf, int64_t iterations);

/* The context's search rectangle after clipping (alpha windows resolved) and
 * the number of valid source centres in it, i.e. patch evaluations per
 * search.  No device work. */
int32_t inpaint_search_info(const inpaint_ctx *ctx, inpaint_rect *rect, int64_t *candidates);

/* Measurement: with enable != 0, every exemplar-search launch of the fill
 * loop is bracketed by HIP events on the context's stream, and
 * inpaint_search_time reports the summed kernel time and the number of
 * searches timed since the last enable.  Off by default.  Supported in the
 * PLAIN and STREAM forms; inpaint_run in the GRAPH form returns
 * INVALID_ARGUMENT while timing is on. */
int32_t inpaint_profile_search(inpaint_ctx *ctx, int32_t enable);
int32_t inpaint_search_time(inpaint_ctx *ctx, double *total_ms, int64_t *searches);

/* The execution form inpaint_run uses for this context: params.form, except
 * that PERSISTENT becomes STREAM when its work-groups cannot all be
 * co-resident.  In the PERSISTENT form the timing above brackets each whole
 * dispatch (search and commit of up to iters_per_check iterations) and
 * `searches` counts dispatches. */
int32_t inpaint_run_form(const inpaint_ctx *ctx, int32_t *form);

/* Releases the context (not the caller's workspace).  Waits for its work. */
int32_t inpaint_destroy(inpaint_ctx *ctx);

const char *inpaint_status_string(int32_t status);
/* Last error message of ctx ("" if none); valid until the next call on ctx.
 * With ctx == NULL, the last error of a failed inpaint_create on this
 * thread. */
const char *inpaint_last_error(const inpaint_ctx *ctx);

/* ------------------------------------------------------------------ batch */

/* Many images advanced together: each batch step runs, for every attached
 * unfinished image, G fill iterations (the fill loop of Section 3 per image).
 * Two forms:
 *  - PERSISTENT: one persistent dispatch per step (the int8-MFMA images of
 *    radius 1..5 share one dispatch; the others one per search form and
 *    radius) runs all G iterations of every image; one work-group per image
 *    commits (front, priority, copy), every other co-resident work-group
 *    searches (image, tile) items of whichever image has a staged target.
 *    Images of up to 64 tiles per search work-group.
 *  - GRAPH: per iteration, a persistent search kernel over a static (image,
 *    tile) work list, then one commit work-group per image; G iterations are
 *    captured once into a hipGraph and replayed.  Tile shape and grid may be
 *    autotuned. */
typedef struct {
    int32_t capacity;        /* maximum attached contexts (slots), >= 1     */
    int32_t graph_iters;     /* G: iterations per step, 1 .. 33554430       */
    int32_t autotune;        /* 1 = time tile shapes and the persistent grid */
                             /*   of the graph form on first use, 0 = defaults */
    int32_t form;            /* 0 = PERSISTENT once the running images fit  */
                             /*   a few tiles per search work-group (4),    */
                             /*   else GRAPH; or                            */
                             /*   INPAINT_FORM_GRAPH / INPAINT_FORM_PERSISTENT */
                             /*   (a step that does not fit then fails with  */
                             /*   INVALID_ARGUMENT)                          */
    const char *tune_cache;  /* JSON file caching autotuned choices, or NULL */
} inpaint_batch_params;

/* Allocates the batch's small device tables (slot table, work list) with
 * hipMalloc.  hip_stream as for inpaint_create. */
int32_t inpaint_batch_create(const inpaint_batch_params *bp, void *hip_stream,
                             inpaint_batch **out);

/* Attaches a created context to a free slot (returned in *slot, may be
 * NULL).  Legal only between inpaint_batch_step calls.  The context must use
 * the batch's stream or a stream the caller orders with it.
 * INVALID_ARGUMENT when full or already attached. */
int32_t inpaint_batch_attach(inpaint_batch *b, inpaint_ctx *ctx, int32_t *slot);

/* Detaches a context (finished or not); its state stays readable. */
int32_t inpaint_batch_detach(inpaint_batch *b, inpaint_ctx *ctx);

/* Runs G iterations for every attached image and writes the number of
 * attached images still unfinished to *active.  Synchronises once. */
int32_t inpaint_batch_step(inpaint_batch *b, int32_t G, int64_t *active);

/* The form (INPAINT_FORM_PERSISTENT or INPAINT_FORM_GRAPH) the last step
 * ran in. */
int32_t inpaint_batch_form(const inpaint_batch *b, int32_t *form);

/* *room = 1 when the batch's running images together with ctx (not yet
 * attached) fit the persistent form with at most tiles_per_group search
 * tiles per search work-group of each batched dispatch (1: every tile stays
 * resident in LDS), else 0.  A scheduler that attaches only while this holds
 * bounds how far sharing slows each image below its solo iteration time.
 * No device work.  INVALID_ARGUMENT for NULL arguments, an attached ctx or
 * tiles_per_group outside 1 .. 64. */
int32_t inpaint_batch_room(inpaint_batch *b, const inpaint_ctx *ctx, int32_t tiles_per_group, int32_t *room);

/* State of a slot as of the end of the last inpaint_batch_step:
 * 0 empty, 1 running, 2 finished (hole empty), 3 device error.  No device
 * work. */
#define INPAINT_SLOT_EMPTY    0
#define INPAINT_SLOT_RUNNING  1
#define INPAINT_SLOT_FINISHED 2
#define INPAINT_SLOT_ERROR    3
int32_t inpaint_batch_status(const inpaint_batch *b, int32_t slot, int32_t *status);

int32_t inpaint_batch_destroy(inpaint_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* INPAINT_H */
