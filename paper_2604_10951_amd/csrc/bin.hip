// bin.hip -- exclusive scan of per-(view, surfel) tile counts and emission of
// one (tile, depth) key per touched tile (Sec. 3.2: every tile the precise
// intersection assigns a surfel to gets one list entry).
//
// Single pass: each workgroup takes a partition of 1024 counts by atomic
// ticket (so partitions are claimed in order and a workgroup only ever waits
// on partitions that are already running), scans it with wave-level prefix
// sums, resolves its global offset by decoupled look-back over the partition
// status words, and then emits the keys of its surfels.  Emission re-derives
// each footprint with the same double-precision code as preprocess, so the
// emitted tiles are exactly the counted ones.
#include "fs_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;                       // counts per lane
constexpr int kPart = kThreads * kItems;        // counts per partition
constexpr uint64_t kFlagAgg = 1ull << 62;       // partition aggregate available
constexpr uint64_t kFlagPre = 2ull << 62;       // inclusive prefix available
constexpr uint64_t kValMask = (1ull << 62) - 1;

__global__ void zero_count_kernel(int64_t* p) { *p = 0; }

__global__ void clear_u64_kernel(uint64_t* p, int64_t count, uint32_t* ticket) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
    if (i == 0) *ticket = 0;
}

FS_DEV uint32_t wave_inclusive_scan(uint32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__global__ void __launch_bounds__(kThreads)
bin_kernel(const float* __restrict__ means, const float* __restrict__ scales, const float* __restrict__ quats,
           const float* __restrict__ opacity, int64_t n, const fs_camera* __restrict__ cams, fs_opts o,
           const uint32_t* __restrict__ counts, int64_t items, uint64_t* __restrict__ keys,
           uint32_t* __restrict__ vals, int64_t capacity, int64_t* __restrict__ num_pairs,
           uint64_t* __restrict__ status, uint32_t* __restrict__ ticket, int64_t parts) {
    __shared__ uint32_t s_part;
    __shared__ uint64_t s_wave[kThreads / 64];
    __shared__ uint64_t s_prefix;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_part = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t part = s_part;
    if (part >= parts) return;
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
    uint64_t wave_excl = 0, total = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) wave_excl += s_wave[w];
        total += s_wave[w];
    }
    if (wave == 0) {
        // decoupled look-back, one wave: lane l reads the status of partition
        // j - l, so each round trip covers 64 predecessors
        uint64_t prefix = 0;
        if (part == 0) {
            if (lane == 0)
                __hip_atomic_store(status + part, kFlagPre | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(status + part, kFlagAgg | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t j = part - 1;
            while (true) {
                const int64_t idx = j - lane;
                const uint64_t st = idx >= 0 ? __hip_atomic_load(status + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                             : kFlagPre;   // before partition 0: an empty inclusive prefix
                const uint64_t flag = st & ~kValMask;
                const uint64_t notready = __ballot(flag == 0);
                const uint64_t pre = __ballot(flag == kFlagPre);
                const int limit = notready ? __builtin_ctzll(notready) : 64;
                const int first_pre = pre ? __builtin_ctzll(pre) : 64;
                const bool found = first_pre < limit;
                const int take = found ? first_pre + 1 : limit;     // lanes [0, take) are summed
                uint64_t v = lane < take ? (st & kValMask) : 0ull;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) v += __shfl_xor(v, d, 64);
                prefix += v;
                if (found) break;
                j -= take;
                if (take == 0) __builtin_amdgcn_s_sleep(1);
            }
            if (lane == 0)
                __hip_atomic_store(status + part, kFlagPre | (prefix + total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            s_prefix = prefix;
            if (part == parts - 1) *num_pairs = (int64_t)(prefix + total);
        }
    }
    __syncthreads();
    uint64_t off = s_prefix + wave_excl + (incl - sum);
    // emission
    const int S = o.tile;
#pragma unroll 1
    for (int j = 0; j < kItems; ++j) {
        const int64_t r = base + j;
        if (c[j] == 0) continue;
        const int v = (int)(r / n);
        const int64_t i = r - (int64_t)v * n;
        const fs_camera& cam = cams[v];
        const int tiles_x = (cam.width + S - 1) / S;
        FsGeo g;
        FsFootprint fp;
        uint64_t o0 = off;
        off += c[j];
        if (!fs_project(means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i], cam, (double)o.alpha_min, g))
            continue;
        if (!fs_footprint(g, cam.width, cam.height, fp)) continue;
        const uint64_t zk = g.zkey;
        const int64_t toff = cam.tile_offset;
        uint64_t end = o0 + c[j];
        auto emit = [&](int tx, int ty) {
            if (o0 < end && o0 < (uint64_t)capacity) {
                keys[o0] = ((uint64_t)(toff + (int64_t)ty * tiles_x + tx) << 32) | zk;
                vals[o0] = (uint32_t)r;
            }
            ++o0;
        };
        if (o.tile_mode == FS_TILES_BBOX) {
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

hipError_t fs_launch_bin(const float* means, const float* scales, const float* quats, const float* opacity, int64_t n,
                         const fs_camera* cams, int32_t num_views, const fs_opts& o, const uint32_t* tiles_touched,
                         uint64_t* keys, uint32_t* vals, int64_t capacity, int64_t* num_pairs, const FsWorkspace& ws,
                         hipStream_t s) {
    const int64_t items = n * (int64_t)num_views;
    const int64_t parts = (items + kPart - 1) / kPart;
    if (parts == 0) {
        hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(1), 0, s, num_pairs);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(clear_u64_kernel, dim3((unsigned)((parts + 255) / 256)), dim3(256), 0, s, ws.scan_status, parts,
                       ws.scan_ticket);
    hipLaunchKernelGGL(bin_kernel, dim3((unsigned)parts), dim3(kThreads), 0, s, means, scales, quats, opacity, n, cams, o,
                       tiles_touched, items, keys, vals, capacity, num_pairs, ws.scan_status, ws.scan_ticket, parts);
    return hipGetLastError();
}
