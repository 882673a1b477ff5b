// api.hip -- extern "C" entry points of libfastsegsim: argument validation,
// workspace layout and dispatch to the kernels.  See include/fastsegsim.h.
#include <string.h>

#include "fs_internal.h"

int64_t fs_sort_scan_parts(int64_t total_tiles);
int64_t fs_bin_scan_parts(int64_t items);

namespace {

thread_local int32_t g_last_hip_error = 0;

fs_status hip_status(hipError_t e) {
    if (e == hipSuccess) return FS_OK;
    g_last_hip_error = (int32_t)e;
    return FS_ERR_HIP;
}

bool valid_opts(const fs_opts* o) {
    if (!o) return false;
    if (o->tile != 8 && o->tile != 16 && o->tile != 32) return false;
    if (o->topk < 0 || o->topk > 64) return false;
    if (o->tile_mode != FS_TILES_PRECISE && o->tile_mode != FS_TILES_BBOX && o->tile_mode != FS_TILES_LINEARISED)
        return false;
    if (o->lowpass != 0 && o->lowpass != 1) return false;
    if (o->feat_dtype != FS_FEAT_F32 && o->feat_dtype != FS_FEAT_BF16) return false;
    if (!(o->alpha_min > 0.f) || !(o->alpha_max <= 1.f) || !(o->alpha_min < o->alpha_max)) return false;
    if (!(o->t_stop >= 0.f) || !(o->t_stop < 1.f)) return false;
    if (o->batch != 0 && o->batch != 16 && o->batch != 32) return false;
    if (o->schedule != FS_SCHED_GRID && o->schedule != FS_SCHED_PERSISTENT && o->schedule != FS_SCHED_SPLIT)
        return false;
    if (o->schedule == FS_SCHED_SPLIT && o->topk < 1) return false;
    if (o->topk_mode != FS_TOPK_FIRST && o->topk_mode != FS_TOPK_WEIGHT) return false;
    if (o->topk_mode == FS_TOPK_WEIGHT && o->topk < 1) return false;
    return true;
}

// Valid options this build cannot run: Top-K by weight outside the split
// schedule or beyond the compact lists.
bool unsupported_opts(const fs_opts* o) {
    return o->topk_mode == FS_TOPK_WEIGHT && (o->schedule != FS_SCHED_SPLIT || o->topk > FS_TOPK_COMPACT_K);
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// Every stage lays its scratch out from the start of the caller's workspace:
// no scratch state outlives the stage that wrote it, and stages sharing a
// workspace are ordered on one stream, so the regions may overlap.
bool fs_workspace_layout(void* base, int64_t n, int32_t num_views, int64_t total_tiles, int64_t pair_capacity,
                         const fs_opts* opts, FsWorkspace* ws, size_t* bytes) {
    if (n < 0 || num_views < 1 || total_tiles < 0 || pair_capacity < 0) return false;
    FsWorkspace w;
    memset(&w, 0, sizeof(w));
    char* b = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t sz) -> void* {
        off = align_up(off, 256);
        void* p = b ? b + off : nullptr;
        off += sz;
        return p;
    };
    // bin stage
    const int64_t items = n * (int64_t)num_views;
    w.scan_parts = fs_bin_scan_parts(items);
    w.scan_status = static_cast<uint64_t*>(take(sizeof(uint64_t) * (size_t)(w.scan_parts > 0 ? w.scan_parts : 1)));
    w.scan_ticket = static_cast<uint32_t*>(take(sizeof(uint32_t) * 16));
    w.bin_over_sums = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)(w.scan_parts > 0 ? w.scan_parts : 1)));
    w.bin_overflow = static_cast<uint2*>(take(sizeof(uint2) * (size_t)(items > 0 ? items : 1)));
    const size_t bin_bytes = align_up(off, 256);
    // sort stage
    off = 0;
    const int64_t tiles = total_tiles > 0 ? total_tiles : 1;
    w.tile_cnt = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)tiles));
    w.tile_fill = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)tiles));
    w.sort_status = static_cast<uint64_t*>(take(sizeof(uint64_t) * (size_t)fs_sort_scan_parts(tiles)));
    w.sort_ticket = static_cast<uint32_t*>(take(sizeof(uint32_t) * 16));
    w.runs = static_cast<uint2*>(take(sizeof(uint2) * (size_t)(pair_capacity > 0 ? pair_capacity : 1)));
    w.long_list = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)tiles));
    const size_t sort_bytes = align_up(off, 256);
    // render stage: work queue of render blocks (at most 16 per tile: 8x8 blocks of a 32x32 tile)
    off = 0;
    w.render_ticket = static_cast<uint32_t*>(take(sizeof(uint32_t) * kRenderQueues * kTicketStride));
    w.render_max_blocks = (total_tiles > 0 ? total_tiles : 1) * 16;
    w.render_gcnt_words = (w.render_max_blocks + 255) / 256 * 64;
    w.render_gcnt = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)w.render_gcnt_words));
    w.render_order = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)w.render_max_blocks));
    w.sel_long = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)w.render_max_blocks));
    w.sel_counts = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)((w.render_max_blocks + 255) / 256)));
    if (opts && opts->topk > 0) {
        // Top-K lists: the split forward and the Top-K backward
        const int64_t sb = opts->tile / 8;
        const int64_t nblocks = (total_tiles > 0 ? total_tiles : 1) * sb * sb;
        w.topk_pair_slots = nblocks * 64 * (int64_t)opts->topk;
        w.topk_pairs = static_cast<uint2*>(take(sizeof(uint2) * (size_t)w.topk_pair_slots));
        w.topk_rows = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)w.topk_pair_slots));
        w.topk_nrows = static_cast<uint32_t*>(take(sizeof(uint32_t) * (size_t)nblocks));
        w.topk_counts = static_cast<int32_t*>(take(sizeof(int32_t) * (size_t)(nblocks * 64)));
    }
    const size_t render_bytes = align_up(off, 256);
    size_t total = bin_bytes > sort_bytes ? bin_bytes : sort_bytes;
    total = total > render_bytes ? total : render_bytes;
    if (ws) *ws = w;
    if (bytes) *bytes = total;
    return true;
}

extern "C" {

fs_status fs_layout_views(fs_camera* cams_host, int32_t num_views, int32_t tile, int64_t* total_tiles,
                          int64_t* total_pixels) {
    if (!cams_host || num_views < 1 || (tile != 8 && tile != 16 && tile != 32)) return FS_ERR_ARG;
    int64_t toff = 0, poff = 0;
    for (int v = 0; v < num_views; ++v) {
        fs_camera& c = cams_host[v];
        if (c.width < 1 || c.height < 1 || c.width > 32767 || c.height > 32767) return FS_ERR_ARG;
        if (toff > INT32_MAX) return FS_ERR_ARG;
        c.tile_offset = (int32_t)toff;
        c.pixel_offset = poff;
        toff += (int64_t)((c.width + tile - 1) / tile) * ((c.height + tile - 1) / tile);
        poff += (int64_t)c.width * c.height;
    }
    if (toff >= (int64_t(1) << 31)) return FS_ERR_ARG;
    if (total_tiles) *total_tiles = toff;
    if (total_pixels) *total_pixels = poff;
    return FS_OK;
}

size_t fs_workspace_bytes(int64_t n, int32_t num_views, int64_t total_tiles, int64_t pair_capacity,
                          const fs_opts* opts) {
    size_t bytes = 0;
    if (!fs_workspace_layout(nullptr, n, num_views, total_tiles, pair_capacity, opts, nullptr, &bytes)) return 0;
    return bytes;
}

fs_status fs_preprocess(const float* means, const float* scales, const float* quats, const float* opacity, int64_t n,
                        const fs_camera* cams_dev, int32_t num_views, const fs_opts* opts, void* records,
                        uint32_t* tiles_touched, uint32_t* tile_cache, hipStream_t stream) {
    if (!valid_opts(opts) || n < 0 || num_views < 1 || !cams_dev) return FS_ERR_ARG;
    if (n > 0 && (!means || !scales || !quats || !opacity || !records || !tiles_touched || !tile_cache))
        return FS_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(tile_cache) % 16 != 0) return FS_ERR_ARG;
    if (n * (int64_t)num_views >= (int64_t(1) << 32)) return FS_ERR_ARG;
    return hip_status(fs_launch_preprocess(means, scales, quats, opacity, n, cams_dev, num_views, *opts,
                                           static_cast<FsRecord*>(records), tiles_touched, tile_cache, stream));
}

fs_status fs_bin(const float* means, const float* scales, const float* quats, const float* opacity, int64_t n,
                 const fs_camera* cams_dev, int32_t num_views, const fs_opts* opts, const uint32_t* tiles_touched,
                 const uint32_t* tile_cache, uint64_t* keys, uint32_t* vals, int64_t pair_capacity, int64_t* num_pairs_dev,
                 int64_t* num_pairs_host, void* workspace, hipStream_t stream) {
    if (!valid_opts(opts) || n < 0 || num_views < 1 || !cams_dev || !num_pairs_dev || pair_capacity < 0)
        return FS_ERR_ARG;
    if (n > 0 && (!means || !scales || !quats || !opacity || !tiles_touched || !tile_cache || !workspace))
        return FS_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(tile_cache) % 16 != 0) return FS_ERR_ARG;
    if (pair_capacity > 0 && (!keys || !vals)) return FS_ERR_ARG;
    if (pair_capacity >= (int64_t(1) << 30)) return FS_ERR_ARG;
    FsWorkspace ws;
    if (!fs_workspace_layout(workspace, n, num_views, 1, pair_capacity, opts, &ws, nullptr)) return FS_ERR_ARG;
    fs_status st = hip_status(fs_launch_bin(means, scales, quats, opacity, n, cams_dev, num_views, *opts,
                                            tiles_touched, tile_cache, keys, vals, pair_capacity, num_pairs_dev, ws, stream));
    if (st != FS_OK || !num_pairs_host) return st;
    int64_t p = 0;
    st = hip_status(hipMemcpyAsync(&p, num_pairs_dev, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    if (st != FS_OK) return st;
    st = hip_status(hipStreamSynchronize(stream));
    if (st != FS_OK) return st;
    *num_pairs_host = p;
    return p > pair_capacity ? FS_ERR_CAPACITY : FS_OK;
}

fs_status fs_bin_noalloc(const float* means, const float* scales, const float* quats, const float* opacity,
                         int64_t n, const fs_camera* cams_dev, int32_t num_views, const fs_opts* opts,
                         const uint32_t* tiles_touched, const uint32_t* tile_cache, uint64_t* keys, uint32_t* vals,
                         int64_t pair_capacity, int64_t* num_pairs_dev, int64_t* num_pairs_host, hipStream_t stream) {
    if (!valid_opts(opts) || n < 0 || num_views < 1 || !cams_dev || !num_pairs_dev || pair_capacity < 0)
        return FS_ERR_ARG;
    if (n > 0 && (!means || !scales || !quats || !opacity || !tiles_touched || !tile_cache)) return FS_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(tile_cache) % 16 != 0) return FS_ERR_ARG;
    if (pair_capacity > 0 && (!keys || !vals)) return FS_ERR_ARG;
    if (pair_capacity >= (int64_t(1) << 30)) return FS_ERR_ARG;
    if (n * (int64_t)num_views > (int64_t)FS_NOALLOC_MAX_RECORDS) return FS_ERR_SCRATCH;
    // the bin stage's part of the workspace layout (no sort or render regions)
    fs_opts bin_opts = *opts;
    bin_opts.topk = 0;
    size_t need = 0;
    if (!fs_workspace_layout(nullptr, n, num_views, 1, 0, &bin_opts, nullptr, &need)) return FS_ERR_ARG;
    void* base = nullptr;
    size_t have = 0;
    fs_status st = hip_status(fs_noalloc_scratch(&base, &have));
    if (st != FS_OK) return st;
    if (need > have) return FS_ERR_SCRATCH;
    FsWorkspace ws;
    if (!fs_workspace_layout(base, n, num_views, 1, 0, &bin_opts, &ws, nullptr)) return FS_ERR_ARG;
    st = hip_status(fs_launch_bin(means, scales, quats, opacity, n, cams_dev, num_views, *opts, tiles_touched,
                                  tile_cache, keys, vals, pair_capacity, num_pairs_dev, ws, stream));
    if (st != FS_OK || !num_pairs_host) return st;
    int64_t p = 0;
    st = hip_status(hipMemcpyAsync(&p, num_pairs_dev, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    if (st != FS_OK) return st;
    st = hip_status(hipStreamSynchronize(stream));
    if (st != FS_OK) return st;
    *num_pairs_host = p;
    return p > pair_capacity ? FS_ERR_CAPACITY : FS_OK;
}

fs_status fs_sort(uint64_t* keys, uint32_t* vals, int64_t pair_capacity, const int64_t* num_pairs_dev,
                  int64_t num_pairs_hint, int64_t total_tiles, uint32_t* tile_ranges, void* workspace,
                  hipStream_t stream) {
    if (!num_pairs_dev || !workspace || !tile_ranges || total_tiles < 1 || pair_capacity < 0) return FS_ERR_ARG;
    if (pair_capacity > 0 && (!keys || !vals)) return FS_ERR_ARG;
    if (pair_capacity >= (int64_t(1) << 30) || total_tiles >= (int64_t(1) << 31)) return FS_ERR_ARG;
    fs_opts dummy{16, 0, 0, 0, 1.f / 255.f, 0.99f, 1e-4f, 0, 0};
    FsWorkspace ws;
    // the sort part of the layout only depends on capacity and tile count
    if (!fs_workspace_layout(workspace, 0, 1, total_tiles, pair_capacity, &dummy, &ws, nullptr)) return FS_ERR_ARG;
    return hip_status(
        fs_launch_sort(keys, vals, pair_capacity, num_pairs_dev, num_pairs_hint, total_tiles, tile_ranges, ws, stream));
}

fs_status fs_render_forward(const void* records, const uint64_t* keys, const uint32_t* vals,
                            const uint32_t* tile_ranges, const void* feats, int32_t C, int64_t n,
                            const fs_camera* cams_dev, int32_t num_views, int64_t total_tiles, const fs_opts* opts,
                            float* out_feat, float* out_T, int32_t* out_n, int32_t* out_last, int32_t* out_idx,
                            float* out_depth, float* out_normal, uint64_t* counters, void* workspace,
                            hipStream_t stream) {
    if (!valid_opts(opts) || C < 1 || n < 1 || num_views < 1 || total_tiles < 1 || !cams_dev) return FS_ERR_ARG;
    if (!records || !tile_ranges || !feats || !out_feat || !out_T || !out_n) return FS_ERR_ARG;
    if (out_idx && opts->topk < 1) return FS_ERR_ARG;
    if (out_depth && !keys) return FS_ERR_ARG;
    if (C > 1024 || unsupported_opts(opts)) return FS_ERR_UNSUPPORTED;
    const bool ext = opts->lowpass != 0 || out_depth || out_normal;
    if (ext && opts->topk_mode == FS_TOPK_WEIGHT) return FS_ERR_UNSUPPORTED;
    FsWorkspace ws;
    memset(&ws, 0, sizeof(ws));
    if (opts->schedule != FS_SCHED_GRID) {
        if (!workspace) return FS_ERR_ARG;
        if (!fs_workspace_layout(workspace, 0, 1, total_tiles, 0, opts, &ws, nullptr)) return FS_ERR_ARG;
    }
    if (opts->schedule == FS_SCHED_SPLIT)
        return hip_status(fs_launch_render_topk_split(static_cast<const FsRecord*>(records), keys, vals, tile_ranges,
                                                      feats, C, n, cams_dev, num_views, total_tiles, *opts, out_feat,
                                                      nullptr, nullptr, out_T, out_n, out_last, out_idx, out_depth,
                                                      out_normal, counters, ws, stream));
    return hip_status(fs_launch_render_forward(static_cast<const FsRecord*>(records), keys, vals, tile_ranges, feats,
                                               C, n, cams_dev, num_views, total_tiles, *opts, out_feat, out_T, out_n,
                                               out_last, out_idx, out_depth, out_normal, counters, ws, stream));
}

fs_status fs_render_labels(const void* records, const uint32_t* vals, const uint32_t* tile_ranges, const void* feats,
                           int32_t C, int64_t n, const fs_camera* cams_dev, int32_t num_views, int64_t total_tiles,
                           const fs_opts* opts, int32_t* out_label, float* out_score, float* out_T, int32_t* out_n,
                           uint64_t* counters, void* workspace, hipStream_t stream) {
    if (!valid_opts(opts) || C < 1 || n < 1 || num_views < 1 || total_tiles < 1 || !cams_dev) return FS_ERR_ARG;
    if (!records || !tile_ranges || !feats || !out_label || !out_T || !out_n || !workspace) return FS_ERR_ARG;
    if (C > 1024 || unsupported_opts(opts) || opts->schedule != FS_SCHED_SPLIT) return FS_ERR_UNSUPPORTED;
    if (opts->lowpass != 0 && opts->topk_mode == FS_TOPK_WEIGHT) return FS_ERR_UNSUPPORTED;
    FsWorkspace ws;
    memset(&ws, 0, sizeof(ws));
    if (!fs_workspace_layout(workspace, 0, 1, total_tiles, 0, opts, &ws, nullptr)) return FS_ERR_ARG;
    return hip_status(fs_launch_render_topk_split(static_cast<const FsRecord*>(records), nullptr, vals, tile_ranges,
                                                  feats, C, n, cams_dev, num_views, total_tiles, *opts, nullptr,
                                                  out_label, out_score, out_T, out_n, nullptr, nullptr, nullptr,
                                                  nullptr, counters, ws, stream));
}

fs_status fs_instance_labels(const float* ins_feats, int32_t dim, const float* means, int64_t n,
                             const float* query_feats, const float* query_means, const float* query_covs,
                             int32_t num_queries, float* out_labels, hipStream_t stream) {
    if (n < 0 || dim < 1 || num_queries < 1) return FS_ERR_ARG;
    if (!ins_feats || !means || !query_feats || !query_means || !query_covs || !out_labels) return FS_ERR_ARG;
    if (dim % 4 != 0 || num_queries > FS_MAX_QUERIES) return FS_ERR_UNSUPPORTED;
    const uintptr_t out_align = num_queries % 4 == 0 ? 16 : 4;
    if ((uintptr_t)ins_feats % 16 || (uintptr_t)query_feats % 16 || (uintptr_t)out_labels % out_align ||
        (uintptr_t)means % 4 || (uintptr_t)query_means % 4 || (uintptr_t)query_covs % 4)
        return FS_ERR_ARG;
    return hip_status(fs_launch_instance_labels(ins_feats, dim, means, n, query_feats, query_means, query_covs,
                                                num_queries, out_labels, stream));
}

fs_status fs_render_backward(const float* means, const float* scales, const float* quats, const float* opacity,
                             const void* records, const uint32_t* vals, const uint32_t* tile_ranges,
                             const void* feats, int32_t C, int64_t n, const fs_camera* cams_dev, int32_t num_views,
                             int64_t total_tiles, const fs_opts* opts, const float* out_T, const int32_t* out_n,
                             const int32_t* out_last, const float* grad_feat, float* grad_records, float* grad_means,
                             float* grad_scales, float* grad_quats, float* grad_opacity, float* grad_feats,
                             void* workspace, hipStream_t stream) {
    if (!valid_opts(opts) || C < 1 || n < 1 || num_views < 1 || total_tiles < 1 || !cams_dev) return FS_ERR_ARG;
    if (!means || !scales || !quats || !opacity || !records || !tile_ranges || !feats || !out_T || !out_n ||
        !out_last || !grad_feat || !grad_records || !grad_means || !grad_scales || !grad_quats || !grad_opacity ||
        !grad_feats)
        return FS_ERR_ARG;
    // the Top-K gradient pass takes rows of up to 64 16-byte vectors (C <= 256
    // float32, 512 bfloat16); the full-blend backward one 128-channel chunk
    const int ve = opts->feat_dtype == FS_FEAT_BF16 ? 8 : 4;
    const bool topk_rows = opts->topk > 0 && opts->topk <= FS_TOPK_COMPACT_K && C % ve == 0 && C / ve <= 64;
    if (C > 128 && !topk_rows) return FS_ERR_UNSUPPORTED;
    if (opts->topk_mode == FS_TOPK_WEIGHT) return FS_ERR_UNSUPPORTED;   // no backward of the by-weight selection
    if (opts->lowpass != 0) return FS_ERR_UNSUPPORTED;                 // no backward of the low-pass response
    FsWorkspace ws;
    memset(&ws, 0, sizeof(ws));
    if (opts->topk > 0) {
        if (!workspace) return FS_ERR_ARG;
        if (!fs_workspace_layout(workspace, 0, 1, total_tiles, 0, opts, &ws, nullptr)) return FS_ERR_ARG;
    }
    return hip_status(fs_launch_render_backward(means, scales, quats, opacity, static_cast<const FsRecord*>(records),
                                                vals, tile_ranges, feats, C, n, cams_dev, num_views, total_tiles,
                                                *opts, out_T, out_n, out_last, grad_feat, grad_records, grad_means,
                                                grad_scales, grad_quats, grad_opacity, grad_feats, ws, stream));
}

const char* fs_status_string(fs_status status) {
    switch (status) {
        case FS_OK: return "ok";
        case FS_ERR_ARG: return "invalid argument";
        case FS_ERR_CAPACITY: return "pair capacity exceeded";
        case FS_ERR_HIP: return "HIP error";
        case FS_ERR_UNSUPPORTED: return "unsupported option combination";
        case FS_ERR_SCRATCH: return "input exceeds the static scratch buffer";
    }
    return "unknown status";
}

int32_t fs_last_hip_error(void) { return g_last_hip_error; }

}  // extern "C"
