// preprocess.hip -- per (view, surfel) projection, culling, record and tile
// count (Sec. 3.1 Eq. 1; Sec. 3.2 conic, SnugBox and AccuTile).
//
// One lane per (view, surfel); 256-lane workgroups, grid.y = view.  Geometry
// runs in double precision (gfx950 runs fp64 at the fp32 vector rate), so the
// tile count is the exact per-pixel footprint count.
#include <cmath>

#include "fs_internal.h"

static_assert(FS_INLINE_TILES == 8 && FS_TILE_CACHE_WORDS == 4, "the cache is one uint4 per record");

namespace {

constexpr int kThreads = 256;

// Conservative view test before the double-precision projection.  The cutoff
// disk (semi-axes k r_u, k r_v in the tangent plane, k^2 = 2 ln(o / alpha_min))
// lies inside the ball of radius rho = kmax max(r_u, r_v) around the centre,
// kmax = sqrt(2 ln(1 / alpha_min)) >= k for o <= 1.  If that ball is in front
// of the near plane and beyond one side plane of the image's frustum (x < 0,
// x > W, y < 0 or y > H for every point), no pixel centre can be in the
// footprint: the surfel has no tiles, whatever the full path would compute
// near the threshold (the centres are at least half a pixel inside).  Planes
// through the camera centre, e.g. fx X + cx Z < 0 for x < 0; |n| is bounded
// by the sum of the absolute components.  Anything the test cannot decide
// (o > 1, non-finite input, a ball reaching the near plane) takes the full path.
FS_DEV bool fs_outside_view(const float* pm, const float* ps, float op, const fs_camera& cam, double kmax) {
    if (!(op <= 1.f)) return false;
    const double p0 = pm[0], p1 = pm[1], p2 = pm[2];
    const double s0 = ps[0], s1 = ps[1];
    double pc[3];
    for (int r = 0; r < 3; ++r)
        pc[r] = (((double)cam.R[3 * r] * p0 + (double)cam.R[3 * r + 1] * p1) + (double)cam.R[3 * r + 2] * p2) +
                (double)cam.t[r];
    const double rho = kmax * (s0 > s1 ? s0 : s1) * (1.0 + 1e-6) + 1e-9 * (fabs(pc[0]) + fabs(pc[1]) + fabs(pc[2]));
    if (!(rho >= 0.0) || !(pc[2] - rho > (double)cam.z_near)) return false;
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy, W = cam.width, H = cam.height;
    const double xl = fx * pc[0] + cx * pc[2], xr = fx * pc[0] + (cx - W) * pc[2];
    const double yt = fy * pc[1] + cy * pc[2], yb = fy * pc[1] + (cy - H) * pc[2];
    return xl + rho * (fabs(fx) + fabs(cx)) < 0.0 || xr - rho * (fabs(fx) + fabs(cx - W)) > 0.0 ||
           yt + rho * (fabs(fy) + fabs(cy)) < 0.0 || yb - rho * (fabs(fy) + fabs(cy - H)) > 0.0;
}

// Render coefficients of a projected surfel, anchored at fp's anchor pixel
// and normalised (h2 = 1 at the projected centre); the pixel box is left to
// the caller.
FS_DEV void fs_fill_record(const FsGeo& g, const FsFootprint& fp, float op, FsRecord& rec) {
    const double mx = g.T[2] / g.T[8], my = g.T[5] / g.T[8];
    const double s = (g.H[6] * mx + g.H[7] * my) + g.H[8];
    const double is = 1.0 / s;
    const double xa = fp.q.ax + 0.5, ya = fp.q.ay + 0.5;
    rec.h0 = ((g.H[0] * xa + g.H[1] * ya) + g.H[2]) * is;
    rec.h1 = ((g.H[3] * xa + g.H[4] * ya) + g.H[5]) * is;
    rec.h2 = ((g.H[6] * xa + g.H[7] * ya) + g.H[8]) * is;
    rec.gx0 = g.H[0] * is;
    rec.gx1 = g.H[3] * is;
    rec.gx2 = g.H[6] * is;
    rec.gy0 = g.H[1] * is;
    rec.gy1 = g.H[4] * is;
    rec.gy2 = g.H[7] * is;
    rec.o = op;
    rec.k2 = g.k2;
    rec.ax = (int16_t)fp.q.ax;
    rec.ay = (int16_t)fp.q.ay;
}

// Each workgroup first runs the view test on its kThreads surfels, then
// packs the undecided ones into its first waves (in surfel order) so that
// the double-precision path runs on full waves and the waves left without
// a surfel end at once; every surfel still writes only its own outputs.
// At least four waves per SIMD (128 VGPRs): the double-precision work is
// latency-bound and needs the occupancy.  EXT: the tile mode is LINEARISED
// or the low-pass option is on (tiles from fs_sweep_tiles_ext / the widened
// bounding box; the record's box covers the low-pass disc too).
template <bool EXT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
preprocess_kernel(const float* __restrict__ means, const float* __restrict__ scales, const float* __restrict__ quats,
                  const float* __restrict__ opacity, int64_t n, const fs_camera* __restrict__ cams, fs_opts o,
                  FsRecord* __restrict__ records, uint32_t* __restrict__ tiles_touched, uint4* __restrict__ tile_cache,
                  double kmax) {
    __shared__ uint32_t s_cand[kThreads];
    __shared__ int s_count[kThreads / 64];
    const int v = blockIdx.y;
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kThreads;
    const fs_camera cam = cams[v];
    bool cand = false;
    if (i0 + tid < n) {
        const int64_t k = i0 + tid;
        // (the test bounds the exact footprint only: the linearised ellipse and
        // the low-pass disc may reach further, so EXT runs every surfel)
        if (!EXT && fs_outside_view(means + 3 * k, scales + 2 * k, opacity[k], cam, kmax))
            tiles_touched[(int64_t)v * n + k] = 0u;   // nothing else is written for a surfel without tiles
        else
            cand = true;
    }
    const uint64_t m = __ballot(cand);
    if (lane == 0) s_count[wave] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        before += w < wave ? s_count[w] : 0;
        total += s_count[w];
    }
    if (cand) s_cand[before + __popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)tid;
    __syncthreads();
    if (tid >= total) return;
    const int64_t i = i0 + s_cand[tid];
    const int64_t r = (int64_t)v * n + i;
    FsRecord rec;
    rec.h0 = rec.h1 = rec.h2 = 0.0;
    rec.gx0 = rec.gx1 = rec.gx2 = 0.0;
    rec.gy0 = rec.gy1 = rec.gy2 = 0.0;
    rec.k2 = -1.0;
    rec.o = 0.f;
    rec.ax = rec.ay = 0;
    rec.x0 = 1;
    rec.x1 = 0;
    rec.y0 = 1;
    rec.y1 = 0;
    uint32_t count = 0;
    // the footprint's tiles for fs_bin: the first three as tx | ty << 16, and
    // the first eight as 4-bit offsets from the base tile (bx, by) of its
    // candidate range, while every offset fits
    uint32_t ids[3] = {0u, 0u, 0u};
    uint32_t off[2] = {0u, 0u};
    bool fits = true;
    int bx = 0, by = 0;
    auto note = [&](int tx, int ty) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (count == (uint32_t)k) ids[k] = (uint32_t)tx | ((uint32_t)ty << 16);
        const int dx = tx - bx, dy = ty - by;
        fits = fits && dx >= 0 && dx <= 15 && dy >= 0 && dy <= 15;
        const uint32_t byte = (uint32_t)(dx & 15) | ((uint32_t)(dy & 15) << 4);
        if (count < 4u)
            off[0] |= byte << (8u * count);
        else if (count < 8u)
            off[1] |= byte << (8u * (count - 4u));
        ++count;
    };
    FsGeo g;
    const float op = opacity[i];
    if (EXT && fs_project(means + 3 * i, scales + 2 * i, quats + 4 * i, op, cam, (double)o.alpha_min, g)) {
        FsFootprint fp;
        const bool exact_ok = fs_footprint(g, cam.width, cam.height, fp);
        FsAssign a;
        fs_assign_setup(g, fp, exact_ok, cam.width, cam.height, o.tile_mode == FS_TILES_LINEARISED, o.lowpass != 0, a);
        const int S = o.tile;
        if (o.tile_mode == FS_TILES_BBOX) {
            int tx0, tx1, ty0, ty1;
            if (fs_bbox_tiles_ext(fp, exact_ok, a, cam.width, cam.height, S, tx0, tx1, ty0, ty1)) {
                const uint32_t nt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                bx = tx0;
                by = ty0;
                if (nt <= FS_INLINE_TILES) {
                    for (int ty = ty0; ty <= ty1; ++ty)
                        for (int tx = tx0; tx <= tx1; ++tx) note(tx, ty);
                } else {
                    count = nt;
                }
            }
        } else if (a.have_ar) {
            bx = a.ar[0] / S;
            by = a.ar[2] / S;
            fs_sweep_tiles_ext(fp, a, S, note);
        }
        if (count > 0) {
            fs_fill_record(g, fp, op, rec);
            if (a.have_box) {
                rec.x0 = (int16_t)a.box[0];
                rec.x1 = (int16_t)a.box[1];
                rec.y0 = (int16_t)a.box[2];
                rec.y1 = (int16_t)a.box[3];
            }
        }
    } else if (!EXT && fs_project(means + 3 * i, scales + 2 * i, quats + 4 * i, op, cam, (double)o.alpha_min, g)) {
        FsFootprint fp;
        if (fs_footprint(g, cam.width, cam.height, fp)) {
            const int S = o.tile;
            if (o.tile_mode == FS_TILES_BBOX) {
                int tx0, tx1, ty0, ty1;
                if (fs_bbox_tiles(fp, cam.width, cam.height, S, tx0, tx1, ty0, ty1)) {
                    const uint32_t nt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                    bx = tx0;
                    by = ty0;
                    if (nt <= FS_INLINE_TILES) {
                        for (int ty = ty0; ty <= ty1; ++ty)
                            for (int tx = tx0; tx <= tx1; ++tx) note(tx, ty);
                    } else {
                        count = nt;
                    }
                }
            } else {
                bx = fp.px0 / S;
                by = fp.py0 / S;
                fs_sweep_tiles(fp, S, note);
            }
        }
        if (count > 0) {
            fs_fill_record(g, fp, op, rec);
            rec.x0 = (int16_t)fp.px0;
            rec.x1 = (int16_t)fp.px1;
            rec.y0 = (int16_t)fp.py0;
            rec.y1 = (int16_t)fp.py1;
        }
    }
    tiles_touched[r] = count;
    if (count == 0u) return;   // no list refers to this record: neither it nor its cache is read
    records[r] = rec;
    if (count <= 3u)
        tile_cache[r] = make_uint4(g.zkey, ids[0], ids[1], ids[2]);
    else if (count <= (uint32_t)FS_INLINE_TILES && fits)
        tile_cache[r] = make_uint4(g.zkey, (uint32_t)bx | ((uint32_t)by << 16), off[0], off[1]);
    else
        tile_cache[r] = make_uint4(g.zkey, FS_TILE_CACHE_NONE, 0u, 0u);
}

}  // namespace

hipError_t fs_launch_preprocess(const float* means, const float* scales, const float* quats, const float* opacity,
                                int64_t n, const fs_camera* cams, int32_t num_views, const fs_opts& o,
                                FsRecord* records, uint32_t* tiles_touched, uint32_t* tile_cache, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)num_views);
    // bound on the cutoff radius k for opacities <= 1, widened against rounding
    const double kmax = std::sqrt(2.0 * std::log(1.0 / (double)o.alpha_min)) * (1.0 + 1e-9);
    const bool ext = o.tile_mode == FS_TILES_LINEARISED || o.lowpass != 0;
    hipLaunchKernelGGL(ext ? preprocess_kernel<true> : preprocess_kernel<false>, grid, dim3(kThreads), 0, s, means,
                       scales, quats, opacity, n, cams, o, records, tiles_touched,
                       reinterpret_cast<uint4*>(tile_cache), kmax);
    return hipGetLastError();
}
