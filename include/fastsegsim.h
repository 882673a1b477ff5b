/*
 * fastsegsim.h -- C ABI of the MI355X (gfx950) surfel feature rasterizer.
 *
 * The library renders C-channel feature images from 2D Gaussian surfels, the
 * rendering path of Fast-SegSim (arXiv 2604.10951):
 *
 *   fs_preprocess       per (view, surfel): tangent frame, the homogeneous
 *                       tangent->screen matrix T, depth key, culling, the
 *                       screen conic and the count of tiles it touches
 *                       (Sec. 3.1 Eq. 1; Sec. 3.2 "Perspective-Corrected
 *                       Conic Matrix Derivation", "Snugbox and AccuTile")
 *   fs_bin              exclusive scan of the tile counts and emission of one
 *                       (tile, depth) key per touched tile (Sec. 3.2)
 *   fs_sort             stable radix sort of the keys and per-tile ranges
 *                       (surfels are blended depth-sorted, Sec. 3.1)
 *   fs_render_forward   per-pixel front-to-back blending of C-channel features,
 *                       full (Sec. 3.1 Eq. 2) or Top-K hard selection
 *                       (Sec. 3.4, F_TopK)
 *   fs_render_labels    the same render reduced per pixel to the argmax channel
 *                       and its value (segmentation masks, Sec. 3.3, 3.5)
 *   fs_instance_labels  per-Gaussian instance labels from instance queries
 *                       (feature similarity x spatial proximity, softmax;
 *                       Sec. 3.3): the channels the label render blends
 *   fs_render_backward  gradients of a loss on the rendered features w.r.t.
 *                       surfel centres, scales, rotations, opacities and
 *                       features (the renderer is trained end to end, Sec. 3.5)
 *
 * Conventions shared by every entry point
 *   - Pointers named *_dev, and every array argument unless stated otherwise,
 *     are DEVICE memory owned by the caller.  The library never allocates,
 *     frees or keeps pointers beyond a call; scratch memory comes from the
 *     caller's `workspace` (size from fs_workspace_bytes), except for
 *     fs_bin_noalloc, whose scratch is a static device buffer of the library.
 *   - Work is enqueued on `stream` in call order.  Calls return after
 *     enqueueing; the only host synchronisation is fs_bin's optional readback
 *     of the pair count (num_pairs_host != NULL).
 *   - Arguments are validated before anything is enqueued: FS_ERR_ARG means
 *     nothing ran.  A failed launch returns FS_ERR_HIP (the HIP error is
 *     available through fs_last_hip_error).  No entry point aborts or throws.
 *   - Calls that share a workspace must not overlap; distinct workspaces may
 *     run concurrently on different streams.
 *
 * Scene arrays (float32, row-major, N surfels):
 *   means   N x 3   world-space centre p (Sec. 3.1 Eq. 1)
 *   scales  N x 2   tangent scales (r_u, r_v), linear, > 0
 *   quats   N x 4   rotation (w, x, y, z), need not be unit length; columns 0
 *                   and 1 of its rotation matrix are t_u and t_v
 *   opacity N       o in (0, 1)
 *   feats   N x C   per-surfel feature vector c (float32 or bfloat16)
 *
 * Per-view outputs are packed view after view; view v starts at pixel
 * cams[v].pixel_offset (set by fs_layout_views).  Pixel (px, py) of view v is
 * element pixel_offset + py * width + px, and its sample point is the pixel
 * centre (px + 0.5, py + 0.5).
 */
#ifndef FASTSEGSIM_H
#define FASTSEGSIM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fs_status {
    FS_OK = 0,
    FS_ERR_ARG = 1,         /* invalid argument; nothing was enqueued */
    FS_ERR_CAPACITY = 2,    /* the key/value buffers are too small for the pair count */
    FS_ERR_HIP = 3,         /* a HIP launch or runtime call failed */
    FS_ERR_UNSUPPORTED = 4, /* a valid but unimplemented option combination */
    FS_ERR_SCRATCH = 5      /* the input needs more scratch than the library's static
                               buffer holds (fs_bin_noalloc); nothing was enqueued */
} fs_status;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  A world point p
 * maps to camera space as p_c = R p + t; intrinsics K = [[fx,0,cx],[0,fy,cy],
 * [0,0,1]] (the camera part of T in Sec. 3.2).  88 bytes. */
typedef struct fs_camera {
    int32_t width, height;  /* pixels */
    float fx, fy, cx, cy;
    float R[9];             /* world -> camera rotation, row-major */
    float t[3];             /* world -> camera translation */
    float z_near;           /* surfels whose cutoff disk reaches depth <= z_near are culled */
    int32_t tile_offset;    /* first global tile id of this view (fs_layout_views) */
    int64_t pixel_offset;   /* first packed pixel of this view (fs_layout_views) */
} fs_camera;

enum { FS_TILES_PRECISE = 0, FS_TILES_BBOX = 1, FS_TILES_LINEARISED = 2 };
enum { FS_FEAT_F32 = 0, FS_FEAT_BF16 = 1 };

typedef struct fs_opts {
    int32_t tile;        /* binning tile side in pixels: 8, 16 or 32 */
    int32_t topk;        /* 0: full blend (Eq. 2); K in [1, 64]: Top-K hard selection (Sec. 3.4) */
    int32_t tile_mode;   /* FS_TILES_PRECISE: exact footprint tiles (SnugBox + AccuTile);
                            FS_TILES_BBOX: every tile of the ellipse's circumscribed square;
                            FS_TILES_LINEARISED: the paper-literal assignment of Sec. 3.2 --
                            tiles holding a pixel centre inside the ellipse of the linearised
                            projected covariance Sigma' = J J^T, J the Jacobian of the
                            perspective map at the tangent origin.  Pixels of the exact
                            footprint outside those tiles are not blended (the renderers
                            still test the exact footprint), so images can differ from
                            PRECISE; the other two modes give identical images */
    int32_t feat_dtype;  /* FS_FEAT_F32 or FS_FEAT_BF16 storage of feats (math is float32) */
    float alpha_min;     /* a surfel contributes to a pixel iff o f(u) >= alpha_min (1/255) */
    float alpha_max;     /* alpha = min(alpha_max, o f(u)) (0.99) */
    float t_stop;        /* a pixel stops before the surfel that would take its
                            transmittance below t_stop (1e-4) */
    int32_t batch;       /* list entries staged in LDS per step: 16 or 32 (0 = 32) */
    int32_t schedule;    /* FS_SCHED_GRID: one workgroup per render block;
                            FS_SCHED_PERSISTENT: a grid sized to the device pulls render
                            blocks, longest tile list first, from a work queue;
                            FS_SCHED_SPLIT (topk > 0 only): a selection pass writes every
                            pixel's Top-K (surfel, weight) list to the workspace, then a
                            gather pass blends the feature rows; same results as the
                            other two, bit for bit */
    int32_t topk_mode;   /* which K surfels a Top-K pixel blends (Sec. 3.4):
                            FS_TOPK_FIRST: the first K it accepts, front to back;
                            FS_TOPK_WEIGHT: the K of largest weight alpha T over its
                            whole front-to-back walk (equal weights: the front one),
                            blended front to back with those weights; T_final is the
                            walk's.  FS_TOPK_WEIGHT needs FS_SCHED_SPLIT and topk <= 16
                            (else FS_ERR_UNSUPPORTED) and has no backward. */
    int32_t lowpass;     /* 1: the screen-space low-pass filter of 2D Gaussian splatting
                            (not in the paper): the response is exp(-d2 / 2) with
                            d2 = min(u^2 + v^2, 2 |x - mu|^2), mu the projected centre, so
                            a surfel also covers the pixel centres within sqrt(k^2 / 2)
                            px of mu (tiles included).  No backward (FS_ERR_UNSUPPORTED).
                            0: the pure ray-splat response */
} fs_opts;

enum { FS_SCHED_GRID = 0, FS_SCHED_PERSISTENT = 1, FS_SCHED_SPLIT = 2 };
enum { FS_TOPK_FIRST = 0, FS_TOPK_WEIGHT = 1 };

/* Per (view, surfel), fs_preprocess leaves FS_TILE_CACHE_WORDS uint32 for
   fs_bin: the depth key and, for footprints of at most FS_INLINE_TILES tiles,
   the tiles themselves (layout under fs_preprocess). */
#define FS_INLINE_TILES 8
#define FS_TILE_CACHE_WORDS 4
#define FS_TILE_CACHE_NONE 0xffffffffu

/* Size of the record fs_preprocess writes per (view, surfel). */
#define FS_RECORD_BYTES 96
/* Floats of per-record geometry gradient fs_render_backward accumulates. */
#define FS_GRAD_RECORD_FLOATS 12

/*
 * fs_layout_views (host only): fill cams_host[v].tile_offset and
 * .pixel_offset for views packed in order, for the given tile size, and
 * return the totals.  cams_host is HOST memory.  FS_ERR_ARG on a bad tile
 * size, a non-positive image size or an image wider than 32767 pixels.
 */
fs_status fs_layout_views(fs_camera* cams_host, int32_t num_views, int32_t tile, int64_t* total_tiles,
                          int64_t* total_pixels);

/*
 * fs_workspace_bytes (host only): scratch bytes every stage needs for n
 * surfels, num_views views, total_tiles tiles and pair_capacity key/value
 * slots.  One workspace serves all stages of a frame.
 */
size_t fs_workspace_bytes(int64_t n, int32_t num_views, int64_t total_tiles, int64_t pair_capacity,
                          const fs_opts* opts);

/*
 * fs_preprocess (Sec. 3.1 Eq. 1; Sec. 3.2).  For every view v and surfel i:
 * tangent frame from the quaternion, camera-space frame, T = K [U | V | p_c],
 * the depth key (float32 bits of the centre's camera depth), culling, the
 * cutoff k^2 = 2 ln(o / alpha_min), the screen conic of u^2+v^2 = k^2 and its
 * tile count (exact per-pixel footprint for FS_TILES_PRECISE).
 *   records        out, num_views * n * FS_RECORD_BYTES, record v*n+i; written
 *                  only for surfels with a nonzero tile count (the only ones a
 *                  key list refers to), others left untouched
 *   tiles_touched  out, num_views * n uint32 (0 for culled surfels)
 *   tile_cache     out, num_views * n * FS_TILE_CACHE_WORDS uint32 (16-byte
 *                  aligned); words w[0..3] of record r at
 *                  [r * FS_TILE_CACHE_WORDS]: w[0] the depth key; for a tile
 *                  count c <= 3, w[1..c] the tiles as view-local tx | ty << 16;
 *                  for 4 <= c <= FS_INLINE_TILES, w[1] = bx | by << 16 and byte
 *                  k < c of w[2], w[3] (w[2] holds bytes 0-3, low byte first)
 *                  = dx | dy << 4 for tile (bx + dx, by + dy), or w[1] =
 *                  FS_TILE_CACHE_NONE when some tile lies more than 15 tiles
 *                  from the base; for larger c, w[1] = FS_TILE_CACHE_NONE.
 *                  Words not named are unspecified; nothing is written for
 *                  c = 0.
 * cams_dev is a device array of num_views cameras laid out by fs_layout_views.
 */
fs_status fs_preprocess(const float* means, const float* scales, const float* quats, const float* opacity, int64_t n,
                        const fs_camera* cams_dev, int32_t num_views, const fs_opts* opts, void* records,
                        uint32_t* tiles_touched, uint32_t* tile_cache, hipStream_t stream);

/*
 * fs_bin (Sec. 3.2).  Exclusive scan of tiles_touched over (view, surfel) in
 * record order, then every record writes, for each touched tile, key =
 * (global tile id << 32) | depth key and value = record index v*n+i at its
 * scanned offset.  Depth keys and tiles come from tile_cache (fs_preprocess's
 * output) when it holds the footprint's tiles; other footprints are
 * re-derived from the parameters (bit-identical to fs_preprocess).
 *   keys, vals       out, pair_capacity slots each
 *   num_pairs_dev    out, device int64: the pair count P (written even if it
 *                    exceeds pair_capacity; then keys beyond capacity are dropped)
 *   num_pairs_host   optional HOST int64: if non-NULL the call waits for P,
 *                    stores it and returns FS_ERR_CAPACITY when P > pair_capacity.
 */
fs_status fs_bin(const float* means, const float* scales, const float* quats, const float* opacity, int64_t n,
                 const fs_camera* cams_dev, int32_t num_views, const fs_opts* opts, const uint32_t* tiles_touched,
                 const uint32_t* tile_cache, uint64_t* keys, uint32_t* vals, int64_t pair_capacity, int64_t* num_pairs_dev,
                 int64_t* num_pairs_host, void* workspace, hipStream_t stream);

/*
 * fs_bin_noalloc: fs_bin for callers that cannot allocate device memory or
 * pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * fs_bin, without `workspace`: the bin stage's scratch (partition totals,
 * overflow counter and overflow queue) lives in a static device buffer of
 * FS_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends.  Nothing in it has to start at zero.
 *   - n * num_views must not exceed FS_NOALLOC_MAX_RECORDS; a larger input
 *     returns FS_ERR_SCRATCH before anything is enqueued.
 *   - The call allocates nothing; its first call on a device looks up that
 *     device's buffer (the current device must be the stream's device).
 *   - Every call on one device shares that device's buffer: calls that
 *     overlap in time on one device (other streams, other threads) race and
 *     must be ordered by the caller.
 */
#define FS_NOALLOC_MAX_RECORDS 4194304
#define FS_NOALLOC_SCRATCH_BYTES (FS_NOALLOC_MAX_RECORDS * 8 + 131072)
fs_status fs_bin_noalloc(const float* means, const float* scales, const float* quats, const float* opacity, int64_t n,
                         const fs_camera* cams_dev, int32_t num_views, const fs_opts* opts,
                         const uint32_t* tiles_touched, const uint32_t* tile_cache, uint64_t* keys, uint32_t* vals,
                         int64_t pair_capacity, int64_t* num_pairs_dev, int64_t* num_pairs_host, hipStream_t stream);

/*
 * fs_sort (Sec. 3.1: blending runs over depth-sorted surfels).  Orders the
 * first P = min(*num_pairs_dev, pair_capacity) pairs by (key, value): by tile,
 * then depth key, then record index -- the order a stable sort by key gives
 * to fs_bin's emission order.  Result in place in keys/vals (counting sort by
 * tile, then a sort of every tile's run).  tile_ranges (out, 2 * total_tiles
 * uint32) receives [start, end) of every tile's run (start == end if empty).
 * num_pairs_hint >= 0 is the host's copy of P, used only to size launches;
 * pass -1 to size by capacity.  Keys whose tile is >= total_tiles are
 * dropped (fs_bin never emits them).
 */
fs_status fs_sort(uint64_t* keys, uint32_t* vals, int64_t pair_capacity, const int64_t* num_pairs_dev,
                  int64_t num_pairs_hint, int64_t total_tiles, uint32_t* tile_ranges, void* workspace,
                  hipStream_t stream);

/*
 * fs_render_forward (Sec. 3.1 Eq. 2; Sec. 3.4).  Per pixel, walks its tile's
 * sorted list (keys and vals from fs_sort) front to back:
 *   (u, v) = ray-splat intersection; alpha = min(alpha_max, o exp(-(u^2+v^2)/2));
 *   skip if alpha < alpha_min; stop before a surfel with T (1 - alpha) < t_stop;
 *   w = alpha T; F += w c; T *= 1 - alpha; with topk = K > 0 stop after the
 *   K-th blended surfel (Top-K hard selection, selected set = first K
 *   contributors in depth order, weights = transmittance).
 * Math in float32 (features read as float32 or bfloat16).
 *   out_feat   out, total_pixels x C float32 (pixel-major, channels contiguous)
 *   out_T      out, total_pixels float32 final transmittance
 *   out_n      out, total_pixels int32 number of blended surfels
 *   out_last   optional out, total_pixels int32: list position of the last
 *              blended surfel, -1 if none (needed by fs_render_backward)
 *   out_idx    optional out, total_pixels x topk int32 record indices of the
 *              blended surfels front to back, -1 padded (topk > 0 only)
 *   out_depth  optional out, total_pixels float32: sum of w z over the
 *              blended surfels, z the camera depth of the ray-splat
 *              intersection point (divide by 1 - T for the mean depth);
 *              needs keys (the depth of the centre is read from the key's
 *              low 32 bits)
 *   out_normal optional out, total_pixels x 3 float32: sum of w n, n the
 *              surfel's camera-space unit normal t_u x t_v (Sec. 3.1) turned
 *              to face the camera
 *              Depth and normal follow the same blend (and Top-K selection)
 *              as the features; FS_ERR_UNSUPPORTED with FS_TOPK_WEIGHT.
 *   counters   optional in/out, 4 uint64 added to: [0] list entries walked
 *              (over all 8x8 or 16x16 render blocks), [1] feature rows the
 *              blocks need (one per block and entry blended by any of its
 *              pixels), [2] blended (pixel, surfel) pairs, [3] blocks run
 *   keys       the sorted keys of fs_sort, read only for out_depth (else NULL)
 */
fs_status fs_render_forward(const void* records, const uint64_t* keys, const uint32_t* vals,
                            const uint32_t* tile_ranges, const void* feats, int32_t C, int64_t n,
                            const fs_camera* cams_dev, int32_t num_views, int64_t total_tiles, const fs_opts* opts,
                            float* out_feat, float* out_T, int32_t* out_n, int32_t* out_last, int32_t* out_idx,
                            float* out_depth, float* out_normal, uint64_t* counters, void* workspace,
                            hipStream_t stream);

/*
 * fs_render_labels (Sec. 3.3, Sec. 3.5: segmentation masks come from
 * blending per-Gaussian class or instance scores as channels; a pixel's label
 * is read here as its best-scoring channel).  The
 * Top-K render of fs_render_forward with the split schedule (opts->schedule
 * = FS_SCHED_SPLIT, topk >= 1, either topk_mode), where each pixel's
 * blended vector F (the same float32 values fs_render_forward writes) is
 * reduced to
 *   out_label  out, total_pixels int32: argmax_c F[c], the lowest c among
 *              equal maxima (0 for a pixel that blends nothing)
 *   out_score  optional out, total_pixels float32: F[out_label]
 * instead of being stored; the C floats per pixel never reach memory.
 * out_T, out_n, counters, workspace and the other arguments as in
 * fs_render_forward.  FS_ERR_UNSUPPORTED for another schedule or C > 1024.
 */
fs_status fs_render_labels(const void* records, const uint32_t* vals, const uint32_t* tile_ranges, const void* feats,
                           int32_t C, int64_t n, const fs_camera* cams_dev, int32_t num_views, int64_t total_tiles,
                           const fs_opts* opts, int32_t* out_label, float* out_score, float* out_T, int32_t* out_n,
                           uint64_t* counters, void* workspace, hipStream_t stream);

/*
 * fs_instance_labels (Sec. 3.3, query-guided instance segmentation).  Per
 * scene Gaussian g (centre p_g, instance feature f_g) and query q (feature
 * f_q, 3D Gaussian with centre p_q and covariance Sigma_q):
 *   S(q, g) = sigmoid(f_q . f_g)
 *   D(q, g) = phi_q(p_g) / phi_q(p_q) = exp(-(p_g - p_q)^T Sigma_q^-1 (p_g - p_q) / 2)
 *   out[g, :] = softmax over q of A(q, g) = S D
 * The Q outputs per Gaussian are the instance-label channels the renderers
 * blend (fs_render_forward / fs_render_labels with C = Q).  Float32 math
 * (the Cholesky factor of each Sigma_q in double).
 *   ins_feats     n x dim float32, rows 16-byte aligned (dim % 4 == 0)
 *   means         n x 3 float32 Gaussian centres (the scene's means)
 *   query_feats   num_queries x dim float32, 16-byte aligned
 *   query_means   num_queries x 3 float32
 *   query_covs    num_queries x 6 float32 symmetric covariances (xx, xy, xz,
 *                 yy, yz, zz), positive definite (otherwise the outputs of
 *                 every Gaussian are NaN)
 *   out_labels    out, n x num_queries float32 (16-byte aligned when
 *                 num_queries % 4 == 0); each row sums to 1
 * n == 0 enqueues nothing.  FS_ERR_ARG for null pointers, misalignment or
 * dim / num_queries < 1; FS_ERR_UNSUPPORTED for dim % 4 != 0 or num_queries
 * > FS_MAX_QUERIES.
 */
#define FS_MAX_QUERIES 64
fs_status fs_instance_labels(const float* ins_feats, int32_t dim, const float* means, int64_t n,
                             const float* query_feats, const float* query_means, const float* query_covs,
                             int32_t num_queries, float* out_labels, hipStream_t stream);

/*
 * fs_render_backward.  Given dL/dF (grad_feat, total_pixels x C float32) for
 * the image fs_render_forward produced with the same inputs, accumulates
 * (adds to) the gradients of L w.r.t. means (N x 3), scales (N x 2), quats
 * (N x 4, w.r.t. the raw quaternion), opacity (N) and feats (N x C, float32
 * even for bfloat16 storage).  Gradient buffers must be zeroed by the caller.
 * The blend's discrete choices (accepted surfels, stopping points, the Top-K
 * set, the alpha clamp) are held fixed, so only the selected surfels receive
 * gradient.  grad_records is caller scratch of num_views * n *
 * FS_GRAD_RECORD_FLOATS floats (zeroed by this call).  Gradients are summed
 * with float atomics, so their last bits depend on scheduling.  C <= 128,
 * or with 1 <= topk <= 16 and C a multiple of 4 (8 for
 * bfloat16 storage) up to 256 (512) channels (FS_ERR_UNSUPPORTED otherwise,
 * and for the low-pass option).  Only the feature
 * image is differentiated (depth and normal outputs carry no gradient).  Any
 * tile mode works: the backward walks the same lists.  The forward outputs out_T / out_last must come
 * from fs_render_forward on the same records, vals and tile_ranges.  With
 * topk > 0 the selection is recomputed exactly as the forward made it (the
 * transmittance chain in the forward's double-precision order), in
 * `workspace` (fs_workspace_bytes with the same opts), and out_T / out_n /
 * out_last are not read.
 */
fs_status fs_render_backward(const float* means, const float* scales, const float* quats, const float* opacity,
                             const void* records, const uint32_t* vals, const uint32_t* tile_ranges,
                             const void* feats, int32_t C, int64_t n, const fs_camera* cams_dev, int32_t num_views,
                             int64_t total_tiles, const fs_opts* opts, const float* out_T, const int32_t* out_n,
                             const int32_t* out_last, const float* grad_feat, float* grad_records, float* grad_means,
                             float* grad_scales, float* grad_quats, float* grad_opacity, float* grad_feats,
                             void* workspace, hipStream_t stream);

/* Human-readable name of a status code (static storage). */
const char* fs_status_string(fs_status status);

/* The last HIP error code a call of this thread turned into FS_ERR_HIP. */
int32_t fs_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTSEGSIM_H */
