// bin.hip -- exclusive scan of per-(view, surfel) tile counts and emission of
// one (tile, depth) key per touched tile (Sec. 3.2: every tile the precise
// intersection assigns a surfel to gets one list entry).
//
// Two passes over the counts: the first writes the total of every partition
// of 512 counts; the second has every partition add up the totals before it
// (no workgroup ever waits on another; with many partitions one workgroup
// scans the totals in between instead), scan its own counts with wave-level
// prefix sums and emit its keys.  Emission takes the depth key and the tiles
// fs_preprocess kept (up to FS_INLINE_TILES of them, as ids or as offsets
// from a base tile); the other footprints are queued and re-derived by a
// second kernel with the same double-precision code preprocess counted them
// with, so the emitted tiles are exactly the counted ones.
#include <mutex>

#include "fs_internal.h"

// Scratch of fs_bin_noalloc: the bin stage's workspace region (partition
// totals, overflow counter and overflow queue) for up to
// FS_NOALLOC_MAX_RECORDS (view, surfel) records, resident on every device
// the library runs on until the process ends.  Host code never passes this
// name to a kernel: fs_noalloc_scratch looks up its device address.
static __device__ __align__(256) unsigned char scratch[FS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
hipError_t fs_noalloc_scratch(void** ptr, size_t* bytes) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

namespace {

// A footprint whose tiles the cache does not hold: re-derived by the
// overflow pass.  Reads the cache only for counts it may hold in offset form.
FS_DEV bool bin_overflows(uint32_t c, const uint4* __restrict__ tile_cache, int64_t r) {
    return c > 3u && (c > (uint32_t)FS_INLINE_TILES || tile_cache[r].y == FS_TILE_CACHE_NONE);
}

constexpr int kThreads = 256;
constexpr int kItems = 2;                       // counts per lane (4: bin 21.6 us, 2: 19.5 us on the
                                                // 1M-surfel 1280x720 frame; 8: 27.5 us)
constexpr int kPart = kThreads * kItems;        // counts per partition
constexpr int64_t kSumParts = 4096;             // partitions up to which each sums those before it

__global__ void zero_count_kernel(int64_t* p) { *p = 0; }

FS_DEV uint32_t wave_inclusive_scan(uint32_t x) { return __ockl_wfscan_add_u32(x, true); }

// Pass 1 of the scan: the total count of every partition of kPart counts and
// its number of footprints whose tiles the cache does not hold.
__global__ void __launch_bounds__(kThreads)
bin_sums_kernel(const uint32_t* __restrict__ counts, const uint4* __restrict__ tile_cache, int64_t items,
                uint64_t* __restrict__ sums, uint32_t* __restrict__ over_sums) {
    __shared__ uint64_t s_wave[kThreads / 64];
    __shared__ uint32_t s_over[kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kPart + (int64_t)tid * kItems;
    uint64_t sum = 0;
    uint32_t over = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t c = (base + j < items) ? counts[base + j] : 0u;
        sum += c;
        over += bin_overflows(c, tile_cache, base + j) ? 1u : 0u;
    }
    sum = __ockl_wfred_add_u64(sum);
    over = __ockl_wfred_add_u32(over);
    if (lane == 0) {
        s_wave[wave] = sum;
        s_over[wave] = over;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t t = 0;
        uint32_t v = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
            t += s_wave[w];
            v += s_over[w];
        }
        sums[blockIdx.x] = t;
        over_sums[blockIdx.x] = v;
    }
}

// Pass 1b: the partitions' exclusive prefixes of the totals and overflow
// counts, in place, by one workgroup walking them in tiles of 8192: each
// tile is loaded coalesced into LDS, every thread scans eight consecutive
// entries there, one workgroup scan places the threads, and the tile is
// written back coalesced.
__global__ void __launch_bounds__(1024)
bin_prefix_kernel(uint64_t* __restrict__ sums, uint32_t* __restrict__ over_sums, int64_t parts) {
    constexpr int kTile = 8192, kPer = kTile / 1024;
    __shared__ uint64_t s_v[kTile];
    __shared__ uint32_t s_ov[kTile];
    __shared__ uint64_t s_w[16];
    __shared__ uint32_t s_o[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t carry = 0;
    uint32_t ocarry = 0;
    for (int64_t b0 = 0; b0 < parts; b0 += kTile) {
        const int n = parts - b0 < kTile ? (int)(parts - b0) : kTile;
        for (int i = tid; i < kTile; i += 1024) {
            s_v[i] = i < n ? sums[b0 + i] : 0ull;
            s_ov[i] = i < n ? over_sums[b0 + i] : 0u;
        }
        __syncthreads();
        uint64_t t = 0;
        uint32_t ot = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            t += s_v[tid * kPer + j];
            ot += s_ov[tid * kPer + j];
        }
        uint64_t ti = t;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = __shfl_up(ti, d, 64);
            if (lane >= d) ti += y;
        }
        const uint32_t oti = __ockl_wfscan_add_u32(ot, true);
        if (lane == 63) {
            s_w[wave] = ti;
            s_o[wave] = oti;
        }
        __syncthreads();
        uint64_t run = carry + (ti - t), tot = 0;
        uint32_t orun = ocarry + (oti - ot), otot = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) {
                run += s_w[w];
                orun += s_o[w];
            }
            tot += s_w[w];
            otot += s_o[w];
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint64_t v = s_v[tid * kPer + j];
            const uint32_t ov = s_ov[tid * kPer + j];
            s_v[tid * kPer + j] = run;
            s_ov[tid * kPer + j] = orun;
            run += v;
            orun += ov;
        }
        carry += tot;
        ocarry += otot;
        __syncthreads();
        for (int i = tid; i < n; i += 1024) {
            sums[b0 + i] = s_v[i];
            over_sums[b0 + i] = s_ov[i];
        }
        __syncthreads();   // the tile buffers and s_w, s_o are rewritten in the next round
    }
}

// Pass 2: every partition takes the total of the partitions before it
// (summed here when they are few, read from the prefix pass otherwise), scans
// its counts and emits its pairs.
__global__ void __launch_bounds__(kThreads)
bin_kernel(const float* __restrict__ means, const float* __restrict__ scales, const float* __restrict__ quats,
           const float* __restrict__ opacity, int64_t n, const fs_camera* __restrict__ cams, fs_opts o,
           const uint32_t* __restrict__ counts, const uint4* __restrict__ tile_cache, int64_t items,
           uint2* __restrict__ overflow, uint64_t* __restrict__ keys,
           uint32_t* __restrict__ vals, int64_t capacity, int64_t* __restrict__ num_pairs,
           const uint64_t* __restrict__ sums, const uint32_t* __restrict__ over_sums,
           uint32_t* __restrict__ over_total, int64_t parts, int prefixed) {
    __shared__ uint64_t s_wave[kThreads / 64];
    __shared__ uint64_t s_pre[kThreads / 64];
    __shared__ uint32_t s_over[kThreads / 64];
    __shared__ uint32_t s_over_pre[kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t part = blockIdx.x;
    // totals of partitions [0, part)
    uint64_t pre = 0;
    uint32_t opre = 0;
    if (!prefixed) {
        for (int64_t k = tid; k < part; k += kThreads) {
            pre += sums[k];
            opre += over_sums[k];
        }
    }
    pre = __ockl_wfred_add_u64(pre);
    opre = __ockl_wfred_add_u32(opre);
    if (lane == 0) {
        s_pre[wave] = pre;
        s_over_pre[wave] = opre;
    }
    const int64_t base = part * kPart + (int64_t)tid * kItems;
    uint32_t c[kItems];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        c[j] = (base + j < items) ? counts[base + j] : 0u;
        sum += c[j];
    }
    // partition-local exclusive prefix of this lane's items (64-bit totals)
    const uint32_t incl = wave_inclusive_scan(sum);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint64_t wave_excl = 0, total = 0, prefix = 0;
    uint32_t over_prefix = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) wave_excl += s_wave[w];
        total += s_wave[w];
        prefix += s_pre[w];
        over_prefix += s_over_pre[w];
    }
    if (prefixed) {
        prefix = sums[part];
        over_prefix = over_sums[part];
    }
    uint64_t off = prefix + wave_excl + (incl - sum);
    // emission: footprints whose tiles fs_preprocess kept are emitted from
    // the cache; the others go to the overflow list
    const int S = o.tile;
    // overflow slots in record order: partition prefix, then wave and lane
    // the lane's tile caches, all loads in flight together (the cache of a
    // record without tiles is never written, so it is not read)
    uint4 cch[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) cch[j] = c[j] > 0u ? tile_cache[base + j] : make_uint4(0u, 0u, 0u, 0u);
    uint32_t nover = 0;
    bool ov[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        // as bin_overflows, on the loaded cache
        ov[j] = c[j] > 3u && (c[j] > (uint32_t)FS_INLINE_TILES || cch[j].y == FS_TILE_CACHE_NONE);
        nover += ov[j] ? 1u : 0u;
    }
    const uint32_t over_incl = wave_inclusive_scan(nover);
    if (lane == 63) s_over[wave] = over_incl;
    __syncthreads();
    uint32_t over_slot = over_prefix + over_incl - nover;
    for (int w = 0; w < wave; ++w) over_slot += s_over[w];
    if (tid == 0 && part == parts - 1) {
        uint32_t own = 0;
        for (int w = 0; w < kThreads / 64; ++w) own += s_over[w];
        *num_pairs = (int64_t)(prefix + total);
        *over_total = over_prefix + own;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t r = base + j;
        const uint64_t o0 = off;
        off += c[j];
        if (ov[j]) {
            overflow[over_slot++] = make_uint2((uint32_t)r, (uint32_t)(o0 < (uint64_t)capacity ? o0 : capacity));
            continue;
        }
        if (c[j] == 0 || o0 >= (uint64_t)capacity) continue;
        const int v = (int)(r / n);
        const fs_camera& cam = cams[v];
        const uint32_t tiles_x = ((uint32_t)cam.width + (uint32_t)S - 1u) / (uint32_t)S;
        const uint4 cache = cch[j];
        const uint64_t zk = cache.x;
        auto emit = [&](int k, uint32_t tx, uint32_t ty) {
            if ((uint32_t)k < c[j] && o0 + k < (uint64_t)capacity) {
                const uint64_t t = (uint64_t)cam.tile_offset + (uint64_t)ty * tiles_x + tx;
                keys[o0 + k] = (t << 32) | zk;
                vals[o0 + k] = (uint32_t)r;
            }
        };
        if (c[j] <= 3u) {
            // the tiles themselves
            const uint32_t id[3] = {cache.y, cache.z, cache.w};
#pragma unroll
            for (int k = 0; k < 3; ++k) emit(k, id[k] & 0xffffu, id[k] >> 16);
        } else {
            // base tile and one byte of (dx, dy) per tile
            const uint32_t bx = cache.y & 0xffffu, by = cache.y >> 16;
#pragma unroll
            for (int k = 0; k < FS_INLINE_TILES; ++k) {
                const uint32_t b = ((k < 4 ? cache.z : cache.w) >> (8 * (k & 3))) & 0xffu;
                emit(k, bx + (b & 15u), by + (b >> 4));
            }
        }
    }
}

// Footprints whose tiles the cache does not hold: one lane per record,
// re-derived from the parameters with the code fs_preprocess counted them with
// (EXT: the linearised tile mode or the low-pass option).
template <bool EXT>
__global__ void __launch_bounds__(kThreads)
bin_overflow_kernel(const float* __restrict__ means, const float* __restrict__ scales,
                    const float* __restrict__ quats, const float* __restrict__ opacity, int64_t n,
                    const fs_camera* __restrict__ cams, fs_opts o, const uint32_t* __restrict__ counts,
                    const uint2* __restrict__ overflow, const uint32_t* __restrict__ ticket,
                    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, int64_t capacity) {
    const uint32_t total = ticket[1];
    const int S = o.tile;
    for (uint32_t k = blockIdx.x * kThreads + threadIdx.x; k < total; k += gridDim.x * kThreads) {
        const uint2 e = overflow[k];
        const int64_t r = e.x;
        const int v = (int)(r / n);
        const int64_t i = r - (int64_t)v * n;
        const fs_camera& cam = cams[v];
        const int tiles_x = (cam.width + S - 1) / S;
        FsGeo g;
        FsFootprint fp;
        if (!fs_project(means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i], cam, (double)o.alpha_min, g))
            continue;
        const bool exact_ok = fs_footprint(g, cam.width, cam.height, fp);
        if (!EXT && !exact_ok) continue;
        const uint64_t zk = g.zkey;
        const int64_t toff = cam.tile_offset;
        uint64_t o0 = e.y;
        const uint64_t end = o0 + counts[r];
        auto emit = [&](int tx, int ty) {
            if (o0 < end && o0 < (uint64_t)capacity) {
                keys[o0] = ((uint64_t)(toff + (int64_t)ty * tiles_x + tx) << 32) | zk;
                vals[o0] = (uint32_t)r;
            }
            ++o0;
        };
        if constexpr (EXT) {
            FsAssign a;
            fs_assign_setup(g, fp, exact_ok, cam.width, cam.height, o.tile_mode == FS_TILES_LINEARISED,
                            o.lowpass != 0, a);
            if (o.tile_mode == FS_TILES_BBOX) {
                int tx0, tx1, ty0, ty1;
                if (fs_bbox_tiles_ext(fp, exact_ok, a, cam.width, cam.height, S, tx0, tx1, ty0, ty1))
                    for (int ty = ty0; ty <= ty1; ++ty)
                        for (int tx = tx0; tx <= tx1; ++tx) emit(tx, ty);
            } else {
                fs_sweep_tiles_ext(fp, a, S, emit);
            }
        } else if (o.tile_mode == FS_TILES_BBOX) {
            int tx0, tx1, ty0, ty1;
            if (fs_bbox_tiles(fp, cam.width, cam.height, S, tx0, tx1, ty0, ty1))
                for (int ty = ty0; ty <= ty1; ++ty)
                    for (int tx = tx0; tx <= tx1; ++tx) emit(tx, ty);
        } else {
            fs_sweep_tiles(fp, S, emit);
        }
    }
}

}  // namespace

// Partitions of the bin stage's scan over `items` tile counts (its
// workspace holds one 64-bit total and one overflow count per partition).
int64_t fs_bin_scan_parts(int64_t items) { return (items + kPart - 1) / kPart; }

hipError_t fs_launch_bin(const float* means, const float* scales, const float* quats, const float* opacity, int64_t n,
                         const fs_camera* cams, int32_t num_views, const fs_opts& o, const uint32_t* tiles_touched,
                         const uint32_t* tile_cache, uint64_t* keys, uint32_t* vals, int64_t capacity,
                         int64_t* num_pairs, const FsWorkspace& ws, hipStream_t s) {
    const int64_t items = n * (int64_t)num_views;
    const int64_t parts = fs_bin_scan_parts(items);
    if (parts == 0) {
        hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(1), 0, s, num_pairs);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(bin_sums_kernel, dim3((unsigned)parts), dim3(kThreads), 0, s, tiles_touched,
                       reinterpret_cast<const uint4*>(tile_cache), items, ws.scan_status, ws.bin_over_sums);
    // each partition sums the totals before it while they are few (no extra
    // launch); beyond that, one workgroup scans them first (the summing is
    // quadratic in the partition count: the 1M-surfel frame's 1,954
    // partitions bin in 19.5 us summing and 24.2 us with the scan, the
    // 16-view frame's 31,250 take 0.24 ms summing)
    const int prefixed = parts > kSumParts ? 1 : 0;
    if (prefixed)
        hipLaunchKernelGGL(bin_prefix_kernel, dim3(1), dim3(1024), 0, s, ws.scan_status, ws.bin_over_sums, parts);
    hipLaunchKernelGGL(bin_kernel, dim3((unsigned)parts), dim3(kThreads), 0, s, means, scales, quats, opacity, n, cams, o,
                       tiles_touched, reinterpret_cast<const uint4*>(tile_cache), items, ws.bin_overflow, keys, vals,
                       capacity, num_pairs, ws.scan_status, ws.bin_over_sums, ws.scan_ticket + 1, parts, prefixed);
    // overflow records: a grid of about one lane per 16 records, each lane striding
    const int64_t ob = (items / 16 + kThreads - 1) / kThreads;
    const unsigned oblocks = (unsigned)(ob < 1 ? 1 : (ob > 4096 ? 4096 : ob));
    const bool ext = o.tile_mode == FS_TILES_LINEARISED || o.lowpass != 0;
    hipLaunchKernelGGL(ext ? bin_overflow_kernel<true> : bin_overflow_kernel<false>, dim3(oblocks), dim3(kThreads), 0,
                       s, means, scales, quats, opacity, n, cams, o, tiles_touched, ws.bin_overflow, ws.scan_ticket,
                       keys, vals, capacity);
    return hipGetLastError();
}
