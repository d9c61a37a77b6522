/*
 * pocketgs.h - C ABI of the gfx950 differentiable Gaussian-splatting library.
 *
 * Implements the hot path of the training operator T of PocketGS (arXiv
 * 2601.17354, Sec. "Hardware-Aligned Differentiable Splatting Optimization"):
 * projection of 3D Gaussians to 2D conics, tile binning with a (tile, depth)
 * key sort, front-to-back compositing that records the forward replay trace
 * S = {id, C_in, alpha} with per-pixel counters, the backward of the
 * compositing recursion that replays S, and the index-mapped scatter of
 * gradients to the canonical parameter buffer.  Support calls (losses, Adam,
 * KNN/PCA seeding of Sec. "Prior-Conditioned Gaussian Parameterization") use
 * the same conventions.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every pointer argument named *_dev is DEVICE memory (hipMalloc or any
 *    allocator returning device pointers, e.g. PyTorch's caching allocator).
 *    Pointers named *_host are host memory read during the call.  The caller
 *    owns all memory; the library never allocates, frees or synchronises
 *    inside these calls, so they are safe to enqueue under stream capture.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Calls only enqueue work and return; results are ready when the stream is.
 *  - Return value: PGS_OK, or PGS_ERR_INVALID_ARG (bad size, unsupported
 *    option or null pointer; nothing was enqueued) or PGS_ERR_HIP (a launch
 *    failed; pgs_last_error() describes it).  Capacity overflow is detected on
 *    the device and reported through a flags word (PGS_FLAG_*): outputs are
 *    then incomplete and the caller must grow the buffer and run again.
 *  - Canonical parameter buffer (float32, row-major [F][n], one row per
 *    scalar field, F = 11 + 3 (D+1)^2 for SH degree D <= 3):
 *      rows 0..2 mean, 3..5 log-scale, 6..9 quaternion (w, x, y, z, need not
 *      be unit), 10 opacity logit, 11 + 3k + ch SH coefficient k of channel ch
 *      (k = l*l + l + m, real orthonormal basis with the Condon-Shortley
 *      phase).  Gradients and Adam moments use the same layout.  The
 *      canonical order is never permuted (index-mapping subsection).
 *  - Images are float32 planar [3][H][W]; pixel (x, y) has centre
 *    (x + 1/2, y + 1/2).  Tiles are TW x TH pixels, TX = ceil(W/TW),
 *    TY = ceil(H/TH), tile index ty*TX + tx.
 */
#ifndef POCKETGS_H
#define POCKETGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pgs_status {
    PGS_OK = 0,
    PGS_ERR_INVALID_ARG = 1,
    PGS_ERR_HIP = 2,
    PGS_ERR_CAPACITY = 3, /* pgs_check_flags: a pair or trace buffer overflowed */
} pgs_status;

/* Bits of the device flags word. */
#define PGS_FLAG_PAIR_OVERFLOW 1u  /* more (tile, Gaussian) pairs than capacity */
#define PGS_FLAG_CACHE_OVERFLOW 2u /* a tile's pairs exceed the trace's pair capacity */

/* Projected Gaussians: one 64-byte record per Gaussian, float32
 * [n][PGS_PROJ_STRIDE] with the fields below at these slots (slots 12..15
 * are written as zero), so that staging one splat reads one cache line. */
#define PGS_PROJ_U 0       /* pixel-space mean x */
#define PGS_PROJ_V 1       /* pixel-space mean y */
#define PGS_PROJ_DEPTH 2   /* camera-space z, the depth of the sort key */
#define PGS_PROJ_A 3       /* conic [[A, B], [B, C]] = inverse 2D covariance */
#define PGS_PROJ_B 4
#define PGS_PROJ_C 5
#define PGS_PROJ_OPACITY 6 /* sigmoid(logit) */
#define PGS_PROJ_R 7       /* view-dependent colour */
#define PGS_PROJ_G 8
#define PGS_PROJ_BLUE 9
#define PGS_PROJ_EXTENT_X 10 /* half-extents of the pixels where alpha can reach */
#define PGS_PROJ_EXTENT_Y 11 /* 1/255 (conservative; -1 = nowhere, inf = unknown) */
#define PGS_PROJ_FIELDS 12
#define PGS_PROJ_STRIDE 16

/* 2D gradients: one 64-byte record per Gaussian, float32
 * [n][PGS_GRAD2D_STRIDE] with dL/d(u, v, A, B, C, opacity, r, g, b) at
 * slots 0..8 (slots 9..15 are never written), so that the nine atomic adds
 * of one splat meet one cache line. */
#define PGS_GRAD2D_FIELDS 9
#define PGS_GRAD2D_STRIDE 16

typedef struct pgs_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float viewmat[12]; /* world -> camera, row-major 3x4 [R | t], OpenCV axes */
} pgs_camera;

/* Forward replay trace S = {id, C_in, alpha} (replay-cache subsection),
 * stored per wave of 64 pixels (lanes = row-major pixels of the tile, wave w
 * holds pixels 64w .. 64w+63) as groups, one group per sorted splat id:
 *   mask_dev   [TW*TH/64][pair_capacity] uint64 (wave-major, so that a wave
 *              writes and reads 64 consecutive masks as one run): bit l of
 *              mask[w][id] is set when pixel (lane l of wave w) recorded an
 *              entry for splat id
 *              (id = index in the sorted pair list; values[id] is the
 *              canonical index, the permutation pi of the index map)
 *   steps_dev  [n_tiles][TW*TH/64] uint32: per wave, the number of list
 *              positions (from the tile's start) whose masks are valid; the
 *              per-iteration counter that replaces a cache clear
 *   base_dev   [n_tiles][TW*TH/64] uint32: first entry of the wave's region
 *   used_dev   [1] uint64 device counter of entries handed out; reset by the
 *              forward, which leaves the total demand of the pass in it
 *   entry_dev  [entry_capacity][entry_words] float32, 16-byte aligned: per
 *              entry (C_in r, g, b, alpha) with entry_words = 4, the cache of
 *              the replay-cache subsection - C_in the colour of everything
 *              behind the splat at that pixel, alpha the clamped alpha it had
 *              there - or (C_in r, g, b) with entry_words = 3, the backward
 *              then recomputing alpha from the splat it stages anyway with the
 *              forward's arithmetic (the same bits; 12 instead of 16 bytes an
 *              entry, written once and read once)
 *   count_dev  [H*W] uint32 entries per pixel, count(u)
 * A wave's entries are base + cursor, where cursor counts the wave's entries
 * of earlier groups and a group's entries follow in lane order; each wave
 * takes a region of exactly its entry count.  entry_capacity <= 2^32 - 1.
 * A wave whose region does not fit, and every tile whose pairs exceed
 * pair_capacity, goes unrecorded (steps 0, count 0) and the forward raises
 * PGS_FLAG_CACHE_OVERFLOW; used_dev then tells how many entries the pass
 * needed.  pgs_trace_entries gives a capacity that can never overflow. */
typedef struct pgs_replay {
    uint64_t* mask_dev;
    uint32_t* steps_dev;
    uint32_t* base_dev;
    uint64_t* used_dev;
    float* entry_dev;
    uint32_t* count_dev;
    uint64_t entry_capacity;
    uint32_t pair_capacity;
    uint32_t entry_words; /* 3 or 4, see entry_dev */
} pgs_replay;

/* Entry capacity that no pass with at most `pair_capacity` pairs can exceed
 * (64 entries per wave and listed splat: TW*TH*pair_capacity). */
size_t pgs_trace_entries(uint32_t pair_capacity, int32_t tile_w, int32_t tile_h);

/* A batch of views rendered by one launch (not in PocketGS, which renders one
 * view at a time).  Tiles of all views share one numbering: view v's tiles
 * are tile_offset[v] + row-major local index, with tile_offset[0] = 0 and
 * tile_offset[v+1] = tile_offset[v] + ceil(W_v/tile_w) * ceil(H_v/tile_h).
 * Per-pixel arrays (image planes, t_final, n_contrib, count, dL/dimage) are
 * the views' own arrays concatenated: view v starts at pixel_offset[v] =
 * sum of W_u H_u over u < v, and a 3-channel array holds view v's planar
 * [3][H_v][W_v] block at 3 * pixel_offset[v].  Per-Gaussian arrays are
 * stacked per view: proj [n_views][n][PGS_PROJ_STRIDE], rect
 * [n_views][2][n], touched [n_views][n], 2D gradients
 * [n_views][n][PGS_GRAD2D_STRIDE].
 *   cams     host array [n_views]
 *   tile_w/h one of 16x16, 8x8, 16x8, 32x8, 8x32 (compositing kernels)
 *   batch    splats staged per LDS batch: 32, 64, 128 or 256
 *   blocks   workgroups of the persistent compositing launches; 0 = as many
 *            as the device keeps resident */
#define PGS_MAX_VIEWS 16
typedef struct pgs_view_batch {
    int32_t n_views;
    const pgs_camera* cams;
    int32_t tile_w, tile_h;
    int32_t batch;
    int32_t blocks;
} pgs_view_batch;

/* Tile offsets [n_views+1] and pixel offsets [n_views+1] (host arrays, may
 * be NULL) of a batch; returns the total tile count, or -1 on a bad batch. */
int32_t pgs_views_layout(const pgs_view_batch* views, int32_t* tile_offsets, int64_t* pixel_offsets);

/* Library version string (static storage). */
const char* pgs_version(void);

/* Description of the last PGS_ERR_* returned on the calling thread
 * (thread-local static storage, valid until the next failing call). */
const char* pgs_last_error(void);

/*
 * pgs_check_flags - the overflow protocol's host side: waits for `stream`,
 * copies the device flags word flags_dev (as given to pgs_bin_sort /
 * pgs_render_fwd) into *flags_host and returns PGS_ERR_CAPACITY when
 * PGS_FLAG_PAIR_OVERFLOW or PGS_FLAG_CACHE_OVERFLOW is set (the outputs of
 * the calls since the flags were cleared are then incomplete: grow the pair
 * capacity to *num_pairs_dev or the trace entries to *used_dev and run
 * again), PGS_OK otherwise.  Unlike every other call it synchronises, so it
 * must not be recorded in a graph.  The caller clears the word (a fill
 * kernel, e.g. a tensor's zero_()) before the next pass.
 */
pgs_status pgs_check_flags(const uint32_t* flags_dev, uint32_t* flags_host, void* stream);

/*
 * Graphs of library calls (not part of PocketGS: the batched training step
 * replays a whole step without host work).  pgs_graph_begin starts stream
 * capture on `stream` (not the null stream; thread-local capture mode);
 * every call enqueued on it until pgs_graph_end is recorded instead of run
 * (library calls allocate and synchronise nothing, and clear their counters
 * with kernels, so they record as kernel nodes only).  pgs_graph_end ends the
 * capture and instantiates the graph into *graph_out (owned by the caller,
 * freed by pgs_graph_destroy).  pgs_graph_launch replays it on a stream:
 * the recorded calls run again on the same device pointers and with the
 * same host arguments they were recorded with.  Errors: PGS_ERR_INVALID_ARG
 * for null arguments, PGS_ERR_HIP when HIP refuses (e.g. a synchronising
 * call was enqueued during capture).
 */
typedef struct pgs_graph pgs_graph;
pgs_status pgs_graph_begin(void* stream);
pgs_status pgs_graph_end(void* stream, pgs_graph** graph_out);
pgs_status pgs_graph_launch(const pgs_graph* graph, void* stream);
void pgs_graph_destroy(pgs_graph* graph);

/*
 * pgs_project - EWA projection of one view (inherited by PocketGS from 3D
 * Gaussian Splatting; the compositing subsection consumes its "depth-sorted
 * visible Gaussians").
 *   params_dev   [F][n] canonical parameters, F = 11 + 3 (sh_degree+1)^2
 *   cam_host     camera; near plane 0.2, dilation 0.3, J clamp 1.3 x half-FOV
 *   tile_w/h     tile shape used for the rectangle
 *   proj_dev     out [n][PGS_PROJ_STRIDE]
 *   radius_dev   out [n] int32 ceil(3 sqrt(lambda_max)), 0 if culled
 *   rect_dev     out [2][n] uint32 inclusive tile rectangle, packed
 *                (x0 | y0 << 16) then (x1 | y1 << 16); 0 if culled
 *   touched_dev  out [n] uint32 number of tiles in the rectangle, 0 if culled
 * Every per-Gaussian quantity is computed in float64 and rounded once to
 * float32.  n may be 0.  Errors: n < 0, sh_degree outside 0..3, non-positive
 * image or tile size, more than 65535 tiles along an axis.
 */
pgs_status pgs_project(const float* params_dev, int32_t n, int32_t sh_degree,
                       const pgs_camera* cam_host, int32_t tile_w, int32_t tile_h,
                       float* proj_dev, int32_t* radius_dev, uint32_t* rect_dev,
                       uint32_t* touched_dev, void* stream);

/* Workspace bytes pgs_bin_sort needs for n Gaussians and `capacity` pairs. */
size_t pgs_bin_sort_workspace(int32_t n, uint32_t capacity);

/*
 * pgs_bin_sort - tile binning and the sort that yields the permutation pi of
 * the index-mapping subsection.  Emits one pair per (Gaussian, tile of its
 * rectangle), key = (view_tile_offset + tile) << 32 | bits(float32 depth),
 * value = canonical index, in canonical order with each rectangle row-major;
 * stable-sorts them by key with a device LSD radix sort over the significant
 * key bits only; writes per-tile [start, end) ranges ([0, 0) when empty).
 *   touched_dev, rect_dev, proj_dev   outputs of pgs_project
 *   tiles_x                           TX of the view
 *   n_tiles                           number of tiles to range (>= offset + TX*TY)
 *   view_tile_offset                  first global tile index of this view
 *   keys_dev/values_dev   out [capacity] sorted pairs
 *   ranges_dev            out [2][n_tiles]: start row then end row
 *   num_pairs_dev         out, one uint32: total pairs (may exceed capacity)
 *   flags_dev             in/out uint32 flags word; PGS_FLAG_PAIR_OVERFLOW is
 *                         OR-ed in when pairs > capacity (then only the first
 *                         `capacity` pairs are emitted and sorted)
 *   workspace_dev         >= pgs_bin_sort_workspace(n, capacity) bytes
 * The pair count never travels to the host.
 */
pgs_status pgs_bin_sort(int32_t n, const float* proj_dev, const uint32_t* rect_dev,
                        const uint32_t* touched_dev, int32_t tiles_x, int32_t n_tiles,
                        int32_t view_tile_offset, uint32_t capacity,
                        uint64_t* keys_dev, uint32_t* values_dev, uint32_t* ranges_dev,
                        uint32_t* num_pairs_dev, uint32_t* flags_dev,
                        void* workspace_dev, size_t workspace_bytes, void* stream);

/* Workspace bytes pgs_sort_pairs needs for `capacity` pairs. */
size_t pgs_sort_workspace(uint32_t capacity);

/*
 * pgs_sort_pairs - the stable LSD radix sort used by pgs_bin_sort, exposed on
 * its own: sorts keys_dev[0..count) (count read from count_dev, clamped to
 * capacity) ascending by their low `key_bits` bits (1..64; higher bits must
 * be zero), carrying values_dev along; equal keys keep their input order.
 * Sorted in place (the workspace holds the ping-pong copy).
 */
pgs_status pgs_sort_pairs(uint64_t* keys_dev, uint32_t* values_dev, const uint32_t* count_dev,
                          uint32_t capacity, int32_t key_bits, void* workspace_dev,
                          size_t workspace_bytes, void* stream);

/*
 * pgs_sort_pairs_noalloc - pgs_sort_pairs for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and result, with the
 * workspace taken from a fixed array of PGS_SORT_NOALLOC_SCRATCH_BYTES that
 * the library holds in device memory on every GPU it runs on until the
 * process ends.  The call allocates and frees nothing.
 *   capacity  at most PGS_SORT_NOALLOC_MAX_PAIRS; larger capacities are
 *             rejected with PGS_ERR_INVALID_ARG (use pgs_sort_pairs)
 * Other arguments as pgs_sort_pairs.  The array is looked up on a device's
 * first call (with that device current; PGS_ERR_HIP if the lookup fails).
 * Every call on one GPU uses the same array, which keeps the last call's
 * contents: calls that overlap on one GPU (several streams, several host
 * threads) race and must be serialised by the caller.
 */
#define PGS_SORT_NOALLOC_MAX_PAIRS (1u << 20)
#define PGS_SORT_NOALLOC_SCRATCH_BYTES (16u << 20)
pgs_status pgs_sort_pairs_noalloc(uint64_t* keys_dev, uint32_t* values_dev, const uint32_t* count_dev,
                                  uint32_t capacity, int32_t key_bits, void* stream);

/*
 * pgs_render_fwd - per-tile front-to-back compositing (compositing subsection,
 * equation C_out = C_in (1 - alpha) + alpha c, unrolled front to back):
 * per pixel and splat of its tile's sorted list, alpha = min(0.99, o e^power),
 * power = -1/2 d^T Q d; splats with power > 0 or alpha < 1/255 are skipped;
 * the pixel stops before a splat that would take T below 1e-4.
 *   width/height, tile_w/tile_h       image and tile shape: 16x16, 8x8, 16x8,
 *                                     32x8 or 8x32 tiles
 *   proj_dev, values_dev, ranges_dev  from pgs_project / pgs_bin_sort
 *   bg_host                           3 floats, background colour
 *   image_dev    out [3][H][W]
 *   t_final_dev  out [H][W] transmittance after the last contributor
 *   n_contrib_dev out [H][W] one plus the list position (within the tile's
 *                range) of the last contributor, 0 if none
 *   cache        NULL: no trace (recompute-T backward).  Otherwise the trace
 *                S = {id, C_in, alpha}, the per-wave step counters and
 *                count(u) are written (replay-cache subsection; layout at
 *                pgs_replay); flags_dev must then be given.
 */
pgs_status pgs_render_fwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                          const float* proj_dev, int32_t n, const uint32_t* values_dev,
                          const uint32_t* ranges_dev, int32_t view_tile_offset,
                          const float* bg_host, float* image_dev, float* t_final_dev,
                          uint32_t* n_contrib_dev, const pgs_replay* cache,
                          uint32_t* flags_dev, const uint32_t* tile_order_dev, void* stream);

/*
 * pgs_tile_order - a launch order for the render kernels (scheduling only,
 * results do not depend on it): the view's tiles sorted by list length,
 * longest first, in 8-pair buckets, so long tiles do not form a tail.
 *   ranges_dev      from pgs_bin_sort ([2][n_tiles])
 *   order_dev       out [tiles_in_view] local tile indices; pass it as
 *                   tile_order_dev to pgs_render_fwd / pgs_render_bwd
 *                   (NULL there means natural order)
 */
pgs_status pgs_tile_order(const uint32_t* ranges_dev, int32_t tiles_in_view, int32_t view_tile_offset,
                          int32_t n_tiles, uint32_t* order_dev, void* stream);

/*
 * pgs_render_bwd - backward of the compositing recursion (equation
 * "backward_chain": dL/dC_in = dL/dC_out (1 - alpha), dL/dc = alpha dL/dC_out,
 * dL/dalpha = <dL/dC_out, c - C_in>), chained through alpha to the 2D
 * parameters and scattered to canonical index values[id] (index-mapping
 * equation).
 *   cache != NULL  replays the trace front to back over each pixel's entries
 *                  (the paper's backward), visiting only recorded groups;
 *   cache == NULL  recomputes alpha and T back to front from t_final and
 *                  n_contrib (the recompute-based backward of 3DGS).
 *   dl_dimage_dev  [3][H][W]
 *   grad2d_dev     [n][PGS_GRAD2D_STRIDE], ACCUMULATED (+=) with float atomics;
 *                  the caller zeroes it.
 */
pgs_status pgs_render_bwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                          const float* proj_dev, int32_t n, const uint32_t* values_dev,
                          const uint32_t* ranges_dev, int32_t view_tile_offset,
                          const float* bg_host, const float* t_final_dev,
                          const uint32_t* n_contrib_dev, const pgs_replay* cache,
                          const float* dl_dimage_dev, float* grad2d_dev,
                          const uint32_t* tile_order_dev, void* stream);

/*
 * pgs_project_bwd - chain the 2D gradients of one view back to the canonical
 * parameters (exact derivative of pgs_project with culling and clamps frozen:
 * no gradient through a clamped colour channel or a clamped J entry).
 *   grad2d_dev  [n][PGS_GRAD2D_STRIDE] from pgs_render_bwd
 *   radius_dev  from pgs_project (culled Gaussians get no gradient)
 *   grads_dev   [F][n] ACCUMULATED (+=); one thread per Gaussian, no atomics,
 *               so views must be enqueued one after another on one stream.
 */
pgs_status pgs_project_bwd(const float* params_dev, int32_t n, int32_t sh_degree,
                           const pgs_camera* cam_host, const int32_t* radius_dev,
                           const float* grad2d_dev, float* grads_dev, void* stream);

/*
 * pgs_loss_l1_dssim - photometric loss (the paper does not state it; the 3D
 * Gaussian Splatting form): L = (1 - lambda) mean|x - y| + lambda (1 - SSIM),
 * SSIM with an 11x11 Gaussian window (sigma 1.5), C1 = 1e-4, C2 = 9e-4, zero
 * padding, mean over pixels and channels.  lambda = 0 gives plain L1 and
 * skips the SSIM kernels.
 *   x_dev, y_dev   [3][H][W] rendered and target images
 *   loss_dev       out, one float (overwritten)
 *   dl_dx_dev      out [3][H][W] (overwritten)
 *   workspace_dev  >= pgs_loss_workspace(width, height) bytes
 */
size_t pgs_loss_workspace(int32_t width, int32_t height);
pgs_status pgs_loss_l1_dssim(const float* x_dev, const float* y_dev, int32_t width,
                             int32_t height, float lambda, float* loss_dev,
                             float* dl_dx_dev, void* workspace_dev, size_t workspace_bytes,
                             void* stream);

/*
 * pgs_psnr - evaluation metric (Sec. Experiments, "Datasets and metrics"):
 * both images clamped to [0, 1], MSE over 3HW, PSNR = 10 log10(1 / MSE).
 *   out_dev        out, two floats: MSE, PSNR (+inf when MSE = 0)
 *   workspace_dev  >= 4096 bytes (pgs_loss_workspace also suffices)
 */
pgs_status pgs_psnr(const float* x_dev, const float* y_dev, int32_t width, int32_t height,
                    float* out_dev, void* workspace_dev, size_t workspace_bytes, void* stream);

/*
 * pgs_adam_step - Adam (Kingma & Ba) on the canonical layout, moments aligned
 * with their parameters (index-mapping subsection):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr_row * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 *   params/grads/m/v  [rows][n] device; lr_host [rows] host; rows <= 64;
 *   step >= 1.
 */
pgs_status pgs_adam_step(float* params_dev, const float* grads_dev, float* m_dev,
                         float* v_dev, int32_t rows, int32_t n, const float* lr_host,
                         int32_t step, float beta1, float beta2, float eps, void* stream);

/*
 * pgs_project_views - pgs_project of every view of a batch in one pass over
 * the Gaussians (the projection inherited from 3D Gaussian Splatting; the
 * view-independent part, rotation, scales and 3D covariance, is computed
 * once per Gaussian and the parameters are read once).  Outputs per view,
 * identical in layout to pgs_project's with the batch's tile shape:
 *   proj_all_dev [n_views][n][PGS_PROJ_STRIDE]; radius_all_dev [n_views][n];
 *   rect_all_dev [n_views][2][n]; touched_all_dev [n_views][n].
 * Views are taken eight per launch.  Errors: PGS_ERR_INVALID_ARG for a bad batch,
 * degree or null pointer (nothing is enqueued).
 */
pgs_status pgs_project_views(const pgs_view_batch* views, const float* params_dev, int32_t n,
                             int32_t sh_degree, float* proj_all_dev, int32_t* radius_all_dev,
                             uint32_t* rect_all_dev, uint32_t* touched_all_dev, void* stream);

/*
 * pgs_project_bwd_views - pgs_project_bwd of every view of a batch in one
 * pass: each Gaussian's canonical rows are read once, every view's
 * contribution is added in float64 and rounded to float32 in view order
 * (as enqueuing pgs_project_bwd view by view does), and the rows are written
 * once; views in which the Gaussian was culled add nothing.
 *   radius_all_dev [n_views][n] and grad2d_all_dev [n_views][n][PGS_GRAD2D_STRIDE]
 *   (per view, from pgs_project_views and pgs_render_bwd_views);
 *   grads_dev [F][n] ACCUMULATED (+=).
 * Views are taken eight per launch.  Errors as pgs_project_views.
 */
pgs_status pgs_project_bwd_views(const pgs_view_batch* views, const float* params_dev, int32_t n,
                                 int32_t sh_degree, const int32_t* radius_all_dev,
                                 const float* grad2d_all_dev, float* grads_dev, void* stream);

/*
 * pgs_bin_sort_views - pgs_bin_sort over every view of a batch with one key
 * sort: the pairs of view v carry key (tile_offset[v] + local tile) * 2^32 +
 * bits(float32 depth_v) and value = canonical id, emitted view by view in
 * canonical order, so the sorted list is the per-view lists one after the
 * other and ranges index the global tiles.
 *   proj_all_dev [n_views][n][PGS_PROJ_STRIDE]; rect_all_dev [n_views][2][n];
 *   touched_all_dev [n_views][n] (pgs_project of each view with the batch's
 *   tile shape); ranges_dev out [2][total tiles];
 *   workspace >= pgs_bin_sort_workspace(n_views * n, capacity).
 * Other arguments and the overflow protocol as pgs_bin_sort.
 */
pgs_status pgs_bin_sort_views(const pgs_view_batch* views, int32_t n, const float* proj_all_dev,
                              const uint32_t* rect_all_dev, const uint32_t* touched_all_dev,
                              uint32_t capacity, uint64_t* keys_dev, uint32_t* values_dev,
                              uint32_t* ranges_dev, uint32_t* num_pairs_dev, uint32_t* flags_dev,
                              void* workspace_dev, size_t workspace_bytes, void* stream);

/*
 * pgs_render_fwd_views - pgs_render_fwd of every view of a batch as one
 * persistent launch: workgroups take global tiles from queue_dev (a device
 * uint32 the call resets) in the order tile_order_dev gives (NULL = tile
 * index order; pgs_tile_order over all tiles gives heavy-first order) until
 * all are done.  Outputs as pgs_render_fwd, concatenated per the batch
 * layout; the trace (optional) is shared by all views: its steps_dev is
 * [total tiles][TW*TH/64] and count_dev [total pixels].
 */
pgs_status pgs_render_fwd_views(const pgs_view_batch* views, const float* proj_all_dev, int32_t n,
                                const uint32_t* values_dev, const uint32_t* ranges_dev,
                                const float* bg_host, float* image_all_dev, float* t_final_all_dev,
                                uint32_t* n_contrib_all_dev, const pgs_replay* cache, uint32_t* flags_dev,
                                const uint32_t* tile_order_dev, uint32_t* queue_dev, void* stream);

/*
 * pgs_render_bwd_views - pgs_render_bwd of every view of a batch as one
 * persistent launch (same queue protocol as pgs_render_fwd_views).  View v's
 * 2D gradients are accumulated (+=) into grad2d_all_dev[v].
 *   dl_all_dev  [3 * total pixels] dL/dimage, concatenated per the layout
 */
pgs_status pgs_render_bwd_views(const pgs_view_batch* views, const float* proj_all_dev, int32_t n,
                                const uint32_t* values_dev, const uint32_t* ranges_dev,
                                const float* bg_host, const float* t_final_all_dev,
                                const uint32_t* n_contrib_all_dev, const pgs_replay* cache,
                                const float* dl_all_dev, float* grad2d_all_dev,
                                const uint32_t* tile_order_dev, uint32_t* queue_dev, void* stream);

/*
 * pgs_adam_step_dev - pgs_adam_step with the step counter on the device, for
 * callers that capture the step in a graph and replay it: the call first
 * advances state_dev[0] (uint32 step count, 0 before the first step) and
 * stores 1 - beta1^step, 1 - beta2^step as float32 bits in state_dev[1..2],
 * then updates every element with them.
 *   state_dev  [4] uint32 device words, owned by the caller
 */
pgs_status pgs_adam_step_dev(float* params_dev, const float* grads_dev, float* m_dev, float* v_dev,
                             int32_t rows, int32_t n, const float* lr_host, uint32_t* state_dev,
                             float beta1, float beta2, float eps, void* stream);

/*
 * pgs_knn - exact k nearest neighbours (Sec. "Local Surface Statistics
 * Estimation", K_n = 16): for every point i of points_dev [3][m] (float32),
 * the k other points with the smallest squared distance
 * ((dx*dx) + (dy*dy)) + (dz*dz) formed in float64, ties broken by the
 * smaller index.  k in {4, 8, 16, 32}, m > k.  Searched through a uniform
 * grid of at most 128^3 cells over the points' bounding box; the result
 * equals a brute-force search bit for bit.
 *   nbr_dev    out [k][m] int32 neighbour indices, nearest first
 *   d2_dev     out [k][m] float64 squared distances
 *   workspace  >= pgs_knn_workspace(m) bytes (grid cells, points in cell order)
 */
size_t pgs_knn_workspace(int32_t m);
pgs_status pgs_knn(const float* points_dev, int32_t m, int32_t k, int32_t* nbr_dev,
                   double* d2_dev, void* workspace_dev, size_t workspace_bytes, void* stream);

/*
 * pgs_pca_seed - disc-like covariance seeding (Sec. "Disc-Like Covariance
 * Seeding"): from the 16 neighbours, C_i = (1/16) sum (p - pbar)(p - pbar)^T,
 * normal = eigenvector of its smallest eigenvalue, s_t = mean distance to the
 * first 3 neighbours, s_n = r_normal s_t; writes canonical SH-degree-0
 * parameters: mean = the point, log-scales (log s_t, log s_t, log s_n),
 * quaternion whose local z is the normal, opacity logit(0.1), DC colour from
 * colours_dev.
 *   points_dev   [3][m] float32;  colours_dev [3][m] float32 in [0, 1]
 *   nbr_dev/d2_dev  pgs_knn output with k >= 16
 *   params_dev   out [14][m]
 */
pgs_status pgs_pca_seed(const float* points_dev, const float* colours_dev, int32_t m,
                        const int32_t* nbr_dev, const double* d2_dev, int32_t k,
                        float r_normal, float* params_dev, void* stream);

/*
 * Learned seeding network.  Not part of PocketGS: a network that corrects
 * the disc-like seed of pgs_pca_seed (Sec. "Disc-Like Covariance Seeding")
 * from the point's neighbourhood.  Layers 64 -> 64 -> 64 -> 64 -> 8 with
 * exact-erf GELU after each hidden layer; every product multiplies bfloat16
 * operands (float32 values rounded to nearest, ties to even) and
 * accumulates in float32.  Weights: one float32 vector of
 * pgs_mlp_weight_count() = 13000 values, [W1 (64 x 64, row = output), b1,
 * W2, b2, W3, b3, W4 (8 x 64), b4].  Outputs per row: (d log-scale x3,
 * q_out (w, x, y, z), d logit).
 */
int32_t pgs_mlp_weight_count(void);

/*
 * pgs_mlp_features - network inputs and base seed of every point.  Frame
 * R = [e1 e2 e3] (columns): eigenvectors of C_i for its largest and middle
 * eigenvalue, each signed so that sum_k ((p_k - p_i) . e)^3 >= 0 over the
 * 16 neighbours, e3 = e1 x e2.
 *   points_dev  [3][m] float32; nbr_dev/d2_dev pgs_knn output with k >= 16
 *   x_dev       out [m][64] float32: (p_k - p_i) in the frame / s_t for the
 *               16 neighbours (neighbour-major), R^T C_i R / s_t^2
 *               (row-major), 7 zeros
 *   base_dev    out [m][16] float32: R row-major (9), log-scales
 *               (log s_t, log s_t, log(r_normal s_t)) (3), quaternion of R
 *               (w, x, y, z) (4)
 */
pgs_status pgs_mlp_features(const float* points_dev, int32_t m, const int32_t* nbr_dev,
                            const double* d2_dev, int32_t k, float r_normal, float* x_dev,
                            float* base_dev, void* stream);

/*
 * pgs_mlp_forward - y = network(x) for m >= 0 rows.
 *   weights_dev  [13000] float32
 *   x_dev        [m][64] float32, 16-byte aligned
 *   y_dev        out [m][8] float32, 16-byte aligned
 */
pgs_status pgs_mlp_forward(const float* weights_dev, const float* x_dev, int32_t m, float* y_dev,
                           void* stream);

/*
 * pgs_mlp_backward - dweights = d(sum(dy * network(x)))/dweights, the
 * forward recomputed inside.  Weight gradients multiply the bfloat16-rounded
 * output gradient and activation; bias gradients sum the float32 output
 * gradient.  Deterministic for a given m.  dweights_dev is overwritten
 * (zeros for m = 0).
 *   dy_dev        [m][8] float32
 *   workspace     >= pgs_mlp_backward_workspace(m) bytes (per-block partial
 *                 gradients, at most 256 x 13000 floats)
 */
size_t pgs_mlp_backward_workspace(int32_t m);
pgs_status pgs_mlp_backward(const float* weights_dev, const float* x_dev, int32_t m,
                            const float* dy_dev, float* dweights_dev, void* workspace_dev,
                            size_t workspace_bytes, void* stream);

/*
 * pgs_seed_targets - training targets from trained canonical parameters
 * [F][n] (rows 3..5 log-scales, 6..9 quaternion, 10 opacity logit):
 * log S = R diag(2 s) R^T, the matrix logarithm of the covariance.
 *   targets_dev  out [n][8]: logS00, logS11, logS22, logS01, logS02, logS12,
 *                logit, 0
 */
pgs_status pgs_seed_targets(const float* params_dev, int32_t n, float* targets_dev, void* stream);

/*
 * pgs_seed_loss - scale * sum over rows of ||log S_hat - log S*||_F^2 +
 * (logit(0.1) + y[7] - logit*)^2 with q = y[3:7]/|y[3:7]|,
 * R_hat = R_base R(q), log S_hat = R_hat diag(2 (base log-scales + y[0:3]))
 * R_hat^T; float64 inside.  scale = 1/m gives the mean.
 *   y_dev [m][8], base_dev [m][16] (pgs_mlp_features), target_dev [m][8]
 *   loss_dev   out [1] float32
 *   dy_dev     out [m][8] float32 gradient of the scaled loss, or NULL
 *   workspace  >= pgs_seed_loss_workspace(m) bytes
 */
size_t pgs_seed_loss_workspace(int32_t m);
pgs_status pgs_seed_loss(const float* y_dev, const float* base_dev, const float* target_dev,
                         int32_t m, float scale, float* loss_dev, float* dy_dev, void* workspace_dev,
                         size_t workspace_bytes, void* stream);

/*
 * pgs_seed_apply - canonical SH-degree-0 parameters from network outputs:
 * log-scales = base + y[0:3], quaternion = q_base (x) y[3:7]/|y[3:7]|
 * (Hamilton product), logit = logit(0.1) + y[7]; means and colours from
 * pca_params_dev.  A row falls back to its pca_params_dev column when y is
 * not finite, |y[3:7]| < 1e-6, some |y[k]| > 2 (k < 3), or the axis of the
 * smallest predicted scale is more than 60 degrees from e3.
 *   pca_params_dev  [14][m] (pgs_pca_seed output); params_dev out [14][m],
 *                   may equal pca_params_dev
 *   fallback_dev    out [m] uint8 (1 = fell back), or NULL
 *   fallback_count_dev  device counter incremented by the number of
 *                   fallbacks (the caller clears it), or NULL
 */
pgs_status pgs_seed_apply(const float* y_dev, const float* base_dev, const float* pca_params_dev,
                          int32_t m, float* params_dev, uint8_t* fallback_dev,
                          uint32_t* fallback_count_dev, void* stream);

/*
 * Bundle adjustment (subsection "GPU-Native Global BA as Mobile MAP
 * Refinement"): the robustified reprojection objective of equation ba_obj,
 * sum over observations (i, j) of rho(|pi(T_i, P_j) - p_ij|^2) with the Huber
 * loss rho (unit information W_ij), scale-aware gauge fixing and the normal
 * equation solved through the reduced camera system (Schur complement over
 * the block-diagonal 3x3 point blocks).  Everything is float64.
 *
 * Camera i: rotation R_i (world to camera, 3x3 row-major) and centre c_i,
 * x = R_i (P - c_i), pixel (fx x0/x2 + cx, fy x1/x2 + cy).  A step is
 * dpose_i = (dphi, dc) and dP_j: R_i <- R_i exp([dphi]x), c_i <- c_i + dc,
 * P_j <- P_j + dP.  Gauge: camera 0's six parameters and camera 1's centre
 * coordinate gauge_axis are fixed (their step entries are 0).
 *
 * Observations are ordered by point: point j's are [point_start[j],
 * point_start[j+1]); obs_cam / obs_pt give each one's camera and point;
 * cam_obs lists the observation ids of each camera,
 * [cam_start[i], cam_start[i+1]).  All arrays are device memory owned by
 * the caller.  At most PGS_BA_MAX_CAMS cameras (keyframes): the reduced
 * camera system is factored by one workgroup with its panels in LDS.
 */
#define PGS_BA_MAX_CAMS 128

typedef struct pgs_ba_problem {
    int32_t n_cams, n_points, n_obs;
    int32_t gauge_axis;             /* 0..2 */
    double fx, fy, cx, cy;
    double huber_delta;             /* pixels, > 0 */
    const uint32_t* obs_cam_dev;    /* [n_obs] */
    const uint32_t* obs_pt_dev;     /* [n_obs] */
    const double* obs_uv_dev;       /* [n_obs][2] measured pixels */
    const uint32_t* point_start_dev;/* [n_points + 1] */
    const uint32_t* cam_obs_dev;    /* [n_obs] */
    const uint32_t* cam_start_dev;  /* [n_cams + 1] */
} pgs_ba_problem;

/* Workspace bytes of pgs_ba_cost / pgs_ba_step for a problem of this size. */
size_t pgs_ba_workspace(int32_t n_cams, int32_t n_points, int32_t n_obs);

/*
 * pgs_ba_cost - robust cost sum rho(|r|^2) of the state (rot_dev [n_cams][9],
 * centre_dev [n_cams][3], points_dev [n_points][3]) into *cost_dev (one
 * double), summed in a fixed order.  Errors: PGS_ERR_INVALID_ARG for a bad
 * problem (2 <= n_cams <= PGS_BA_MAX_CAMS, non-empty, gauge_axis 0..2,
 * huber_delta > 0, no null pointer) or a small workspace.
 */
pgs_status pgs_ba_cost(const pgs_ba_problem* problem, const double* rot_dev, const double* centre_dev,
                       const double* points_dev, double* cost_dev, void* workspace_dev,
                       size_t workspace_bytes, void* stream);

/*
 * pgs_ba_step - one Levenberg-Marquardt step of the iteratively reweighted
 * Gauss-Newton normal equations, (H + lambda diag(H)) Delta = b over the
 * free parameters (H = sum w J^T J, b = -sum w J^T r, w the Huber weight
 * min(1, delta/|r|)), through the reduced camera system: dpose_dev
 * [n_cams][6] (fixed entries 0) and dpoint_dev [n_points][3], overwritten.
 * Errors as pgs_ba_cost, and lambda < 0.
 */
pgs_status pgs_ba_step(const pgs_ba_problem* problem, const double* rot_dev, const double* centre_dev,
                       const double* points_dev, double lambda, double* dpose_dev, double* dpoint_dev,
                       void* workspace_dev, size_t workspace_bytes, void* stream);

/*
 * pgs_ba_apply - the state after a step: rot_out = R exp([dphi]x),
 * centre_out = c + dc, points_out = P + dP (outputs may not alias inputs).
 */
pgs_status pgs_ba_apply(int32_t n_cams, int32_t n_points, const double* rot_dev, const double* centre_dev,
                        const double* points_dev, const double* dpose_dev, const double* dpoint_dev,
                        double* rot_out_dev, double* centre_out_dev, double* points_out_dev, void* stream);

/*
 * pgs_ba_refine - one pass of the iterative geometric refinement around the
 * bundle adjustment (refinement paragraph of the BA subsection): every point
 * re-triangulated as the least-squares intersection of its observation rays
 * (sum (I - d d^T) P = sum (I - d d^T) c_i, d the unit world ray of the
 * measured pixel) with the poses rot_dev / centre_dev, into points_out_dev
 * [n_points][3]; keep_point_dev [n_points] = 1 when the system is solvable
 * (det > 1e-12 trace^3), at least two observations lie in front of their
 * cameras, their mean reprojection error is <= max_err pixels and the
 * largest angle between two of their camera-to-point rays is >= min_angle
 * (radians); keep_obs_dev [n_obs] = 1 for the observations of kept points
 * that lie in front of their camera.  Errors as pgs_ba_cost.
 */
pgs_status pgs_ba_refine(const pgs_ba_problem* problem, const double* rot_dev, const double* centre_dev,
                         double max_err, double min_angle, double* points_out_dev, uint8_t* keep_point_dev,
                         uint8_t* keep_obs_dev, void* stream);

/* Workspace bytes of pgs_ba_compact. */
size_t pgs_ba_compact_workspace(int32_t n_points, int32_t n_obs);

/*
 * pgs_ba_compact - the problem restricted to the kept points and
 * observations (order preserved, points renumbered in order): the new
 * observation arrays (obs_cam, obs_pt, obs_uv, by point), point_start
 * [kept points + 1], cam_obs (the kept observations by camera, stable),
 * cam_start [n_cams + 1] and the kept points' coordinates, written to
 * caller-owned device arrays sized like the input problem's, and
 * counts_out_dev [2] = (kept points, kept observations).  A camera may be
 * left without observations.
 */
pgs_status pgs_ba_compact(const pgs_ba_problem* problem, const uint8_t* keep_point_dev,
                          const uint8_t* keep_obs_dev, const double* points_dev, uint32_t* obs_cam_out_dev,
                          uint32_t* obs_pt_out_dev, double* obs_uv_out_dev, uint32_t* point_start_out_dev,
                          uint32_t* cam_obs_out_dev, uint32_t* cam_start_out_dev, double* points_out_dev,
                          uint32_t* counts_out_dev, void* workspace_dev, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Single-reference cost-volume multi-view stereo (subsection
 * "Single-Reference Cost-Volume MVS").  All views share one image size
 * width x height (the cameras' own width/height fields are not read); the
 * cameras are a device array cams_dev[n_views] of pgs_camera, read as
 * float64.  Images are 8-bit greyscale [n_views][height][width].
 * ------------------------------------------------------------------------ */
typedef struct pgs_mvs_params {
    int32_t n_planes;   /* depth hypotheses: 64, 128, 192 or 256 */
    int32_t p1, p2;     /* SGM penalties for a one-plane / a larger jump, 0..1000
                           (pgs_mvs_sgm: p2 <= 207, path costs kept in bytes) */
    double conf_min;    /* confidence filter, 0.4 in the paper */
    double b_target;    /* preferred baseline (scene units), reference score */
    double sigma_b;     /* > 0, width of the baseline term */
    double alpha_min;   /* > 0 radians, angle scale of the reference score */
} pgs_mvs_params;

/*
 * pgs_mvs_census - 7 x 7 Census transform (matching-cost paragraph): 48
 * bits per pixel, bit b (row-major over the window, centre skipped) set when
 * the neighbour is darker than the centre; neighbours outside the image take
 * the nearest border pixel.  grey_dev [n_views][height][width] uint8 ->
 * census_dev [n_views][height][width] uint64.
 */
pgs_status pgs_mvs_census(const uint8_t* grey_dev, int32_t n_views, int32_t width, int32_t height,
                          uint64_t* census_dev, void* stream);

/* Workspace bytes of pgs_mvs_depth_range. */
size_t pgs_mvs_range_workspace(int32_t n_views, int32_t n_points);

/*
 * pgs_mvs_depth_range - probabilistic depth range (paragraph "Probabilistic
 * Depth Range Estimation"): per view, the camera depths z > 0 of the sparse
 * points points_dev [n_points][3] (float64, world) whose pixel lies in
 * [-0.5, width - 0.5) x [-0.5, height - 0.5); with their sorted depths z_i
 * and q(p) = z_i + (z_{i+1} - z_i)(h - i), h = (n - 1) p, i = floor(h):
 * range_dev [n_views][2] = (0.5 q(0.05), 1.5 q(0.95)), (0, 0) when no point
 * projects into the view.  Every product and sum is an unfused float64
 * operation in a fixed order, so the result is reproducible bit for bit.
 */
pgs_status pgs_mvs_depth_range(const pgs_camera* cams_dev, int32_t n_views, int32_t width, int32_t height,
                               const double* points_dev, int32_t n_points, double* range_dev,
                               void* workspace_dev, size_t workspace_bytes, void* stream);

/*
 * pgs_mvs_select_ref - single-reference selection (equation S_ref): for
 * each view, among all other views the one maximising
 * exp(-(b - b_target)^2 / (2 sigma_b^2)) * max(alpha / alpha_min, 1), b the
 * distance between the camera centres, alpha the angle between the optical
 * axes; ref_dev [n_views] int32 (smallest index on ties; -1 with one view).
 */
pgs_status pgs_mvs_select_ref(const pgs_camera* cams_dev, int32_t n_views, const pgs_mvs_params* params,
                              int32_t* ref_dev, void* stream);

/*
 * pgs_mvs_cost - plane-sweep Census cost volume (matching-cost paragraph)
 * for the target views targets_dev [n_targets] against their references
 * ref_dev[view]: n_planes fronto-parallel planes uniform in inverse depth
 * over range_dev[view] (plane 0 the farthest,
 * 1/d_k = 1/d_max + k (1/d_min - 1/d_max)/(n_planes - 1)); target pixel
 * (x, y) at d_k maps to X = d_k ((x - cx)/fx, (y - cy)/fy, 1), to the
 * reference as M X + m (M = R_r R_t^T, m = t_r - M t_t) and to its nearest
 * pixel floor(fx x/z + cx + 0.5), likewise y (M, m, d_k and the rays are
 * float64 rounded to float32; the per pixel-plane arithmetic is unfused
 * float32 in a fixed order); cost = Hamming distance of the Census strings, 48 where z <= 0,
 * the pixel is outside the image, the range is empty or the view has no
 * reference (ref_dev[view] < 0, as pgs_mvs_select_ref gives a lone view).
 * cost_dev [n_targets][height][width][n_planes] uint8.
 */
pgs_status pgs_mvs_cost(const pgs_camera* cams_dev, int32_t width, int32_t height, const uint64_t* census_dev,
                        const int32_t* targets_dev, int32_t n_targets, const int32_t* ref_dev,
                        const double* range_dev, const pgs_mvs_params* params, uint8_t* cost_dev, void* stream);

/* Workspace bytes of pgs_mvs_sgm (one direction's path costs as bytes,
 * then the path-cost sum as uint16). */
size_t pgs_mvs_sgm_workspace(int32_t n_targets, int32_t width, int32_t height, int32_t n_planes);

/*
 * pgs_mvs_sgm - SGM aggregation over 4 paths (left-right, right-left,
 * top-bottom, bottom-top), L_r(p,k) = C(p,k) + min(L_r(p-r,k),
 * L_r(p-r,k+-1) + p1, min_i L_r(p-r,i) + p2) - min_i L_r(p-r,i), then per
 * pixel the winner k* (smallest sum S, smallest plane on ties), S2 = min S
 * over |k - k*| >= 2 and the confidence filter: kept when 0 < k* < n_planes-1,
 * S2 > 0 and S(k*) <= (1 - conf_min) S2, with the parabola-refined depth
 * 1/d = 1/d_max + (k* + delta) h.  depth_dev [n_targets][height][width]
 * float32 (0 where rejected), conf_dev the same shape (1 - S(k*)/S2).
 * agg_out_dev (optional, [n_targets][height][width][n_planes] uint16)
 * receives S; without it the partial sums live in the workspace, which is
 * required either way.  p2 <= 207 (each path cost, <= 48 + p2, is stored in
 * a byte between the two sweeps of a line).
 */
pgs_status pgs_mvs_sgm(const uint8_t* cost_dev, int32_t width, int32_t height, const int32_t* targets_dev,
                       int32_t n_targets, const double* range_dev, const pgs_mvs_params* params, float* depth_dev,
                       float* conf_dev, uint16_t* agg_out_dev, void* workspace_dev, size_t workspace_bytes,
                       void* stream);

/* Workspace bytes of pgs_mvs_fuse. */
size_t pgs_mvs_fuse_workspace(int32_t n_targets, int32_t height);

/*
 * pgs_mvs_fuse - fusion into the dense cloud P: the kept pixels (depth > 0)
 * of each target view, numbered in target order and row-major pixel order,
 * back-projected to the world, R^T (z ((x - cx)/fx, (y - cy)/fy, 1) - t);
 * kept pixel i becomes point i / stride when stride divides i, written to
 * points_dev [3][capacity] float32 (the point-cloud layout of pgs_knn and
 * pgs_pca_seed) and, when colour_dev is given, its intensity
 * grey_dev[view][y][x] / 255 to all three rows of colour_dev [3][capacity].
 * *count_dev = the number of kept pixels (points beyond capacity are not
 * written).
 */
pgs_status pgs_mvs_fuse(const pgs_camera* cams_dev, const int32_t* targets_dev, int32_t n_targets, int32_t width,
                        int32_t height, const float* depth_dev, const uint8_t* grey_dev, uint32_t stride,
                        float* points_dev, float* colour_dev, uint32_t capacity, uint32_t* count_dev,
                        void* workspace_dev, size_t workspace_bytes, void* stream);

/*
 * pgs_stream_copy - plain streaming copy of `bytes` (a multiple of 16, both
 * pointers 16-byte aligned) from src_dev to dst_dev.  A measurement aid, not
 * part of the method: it defines the achievable HBM bandwidth the kernels are
 * compared with and calibrates hardware traffic counters (it reads and
 * writes exactly `bytes`).
 */
pgs_status pgs_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream);

/*
 * pgs_atomic_scatter - float-atomic throughput reference for the gradient
 * scatter of pgs_render_bwd (index-mapping equation, the "+=" into the 2D
 * gradient records): for every i < n_targets adds 1.0f to fields 0..8 of
 * record targets_dev[i] of records_dev [n_records][PGS_GRAD2D_STRIDE]
 * (targets >= n_records are skipped), 256 targets per workgroup in the
 * order the render backward flushes a batch of splats.  Given the sorted
 * pair values of a view as targets, it issues the backward's atomics at the
 * backward's contention.  A measurement aid, not part of the method.
 */
pgs_status pgs_atomic_scatter(float* records_dev, uint32_t n_records, const uint32_t* targets_dev,
                              uint32_t n_targets, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* POCKETGS_H */
