// sort.hip -- stable LSD radix sort of (tile << 32 | depth-key, record) pairs
// and per-tile ranges (surfels are blended depth-sorted, Sec. 3.1; the
// pipeline is tile based, Sec. 3.2).
//
// Structure ("onesweep"): one kernel builds the 256-bucket histograms of every
// 8-bit digit in a single read of the keys; a one-workgroup kernel scans them
// into per-pass digit offsets and marks passes whose digit is the same for
// every key (those are identity permutations and are skipped on the device,
// which keeps graph capture free of host decisions); then one kernel per pass
// ranks and scatters.  A pass kernel takes 4096-key partitions by atomic
// ticket, ranks keys inside each wave64 with ballot-based digit matching
// (stable: keys are visited in index order), combines the four waves in LDS,
// and resolves the partition's global position per digit by decoupled
// look-back over 32-bit status words (2 flag bits + 30-bit count).
#include "fs_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kPart = kThreads * kItems;   // 4096 keys per partition
constexpr int kRadix = 256;
constexpr uint32_t kAgg = 1u << 30;
constexpr uint32_t kPre = 2u << 30;
constexpr uint32_t kCnt = (1u << 30) - 1u;
constexpr int kMaxPass = 8;

__global__ void sort_clear_kernel(uint32_t* hist, int64_t nhist, uint32_t* status, int64_t nstatus, uint32_t* tickets,
                                  int npass, uint32_t* ranges, int64_t nranges) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nstatus; i += stride) status[i] = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nranges; i += stride) ranges[i] = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nhist; i += stride) hist[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < npass) tickets[threadIdx.x] = 0;
}

FS_DEV int64_t load_count(const int64_t* num_pairs, int64_t capacity) {
    int64_t p = *num_pairs;
    return p < capacity ? p : capacity;
}

__global__ void __launch_bounds__(kThreads)
sort_hist_kernel(const uint64_t* __restrict__ keys, const int64_t* __restrict__ num_pairs, int64_t capacity,
                 int npass, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kMaxPass * kRadix];
    for (int i = threadIdx.x; i < npass * kRadix; i += kThreads) h[i] = 0;
    __syncthreads();
    const int64_t P = load_count(num_pairs, capacity);
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < P; i += stride) {
        const uint64_t k = keys[i];
        for (int p = 0; p < npass; ++p) atomicAdd(&h[p * kRadix + ((k >> (8 * p)) & 0xff)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * kRadix; i += kThreads)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void __launch_bounds__(kThreads)
sort_scan_kernel(const uint32_t* __restrict__ hist, const int64_t* __restrict__ num_pairs, int64_t capacity,
                 int npass, uint32_t* __restrict__ digit_off, int32_t* __restrict__ ctrl) {
    __shared__ uint32_t s[kRadix];
    __shared__ int trivial[kMaxPass];
    const int d = threadIdx.x;
    const int64_t P = load_count(num_pairs, capacity);
    if (d < kMaxPass) trivial[d] = 0;
    __syncthreads();
    for (int p = 0; p < npass; ++p) {
        const uint32_t c = hist[p * kRadix + d];
        if ((int64_t)c == P) trivial[p] = 1;
        s[d] = c;
        __syncthreads();
        // exclusive scan over 256 buckets (Hillis-Steele in LDS)
        uint32_t x = c;
        for (int off = 1; off < kRadix; off <<= 1) {
            const uint32_t y = d >= off ? s[d - off] : 0u;
            __syncthreads();
            x += y;
            s[d] = x;
            __syncthreads();
        }
        digit_off[p * kRadix + d] = x - c;
        __syncthreads();
    }
    if (d == 0) {
        int cur = 0;
        for (int p = 0; p < npass; ++p) {
            if (trivial[p]) {
                ctrl[p] = -1;
            } else {
                ctrl[p] = cur;
                cur ^= 1;
            }
        }
        ctrl[npass] = cur;
    }
}

__global__ void __launch_bounds__(kThreads)
sort_pass_kernel(uint64_t* __restrict__ keys0, uint32_t* __restrict__ vals0, uint64_t* __restrict__ keys1,
                 uint32_t* __restrict__ vals1, const int64_t* __restrict__ num_pairs, int64_t capacity, int pass,
                 const uint32_t* __restrict__ digit_off, const int32_t* __restrict__ ctrl,
                 uint32_t* __restrict__ status, uint32_t* __restrict__ ticket, int64_t parts_cap) {
    __shared__ uint32_t wh[kThreads / 64][kRadix];
    __shared__ uint32_t s_part;
    const int src = ctrl[pass];
    if (src < 0) return;
    const int64_t P = load_count(num_pairs, capacity);
    const int64_t parts = (P + kPart - 1) / kPart;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_part = atomicAdd(ticket + pass, 1u);
    for (int w = 0; w < kThreads / 64; ++w) wh[w][tid] = 0;
    __syncthreads();
    const int64_t part = s_part;
    if (part >= parts || part >= parts_cap) return;
    const uint64_t* sk = src ? keys1 : keys0;
    const uint32_t* sv = src ? vals1 : vals0;
    uint64_t* dk = src ? keys0 : keys1;
    uint32_t* dv = src ? vals0 : vals1;
    const int shift = 8 * pass;
    const int64_t base = part * kPart + (int64_t)wave * (kPart / 4);
    uint64_t k[kItems];
    uint32_t val[kItems];
    uint32_t rank[kItems];
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < P;
        k[r] = valid ? sk[idx] : 0ull;
        val[r] = valid ? sv[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < P;
        const uint32_t d = (uint32_t)(k[r] >> shift) & 0xffu;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t prev = wh[wave][d];
        rank[r] = prev + (uint32_t)__popcll(peers & lt);
        if (valid && ((peers >> lane) >> 1) == 0ull) wh[wave][d] = prev + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per-digit partition totals and per-wave offsets (thread = digit)
    {
        const int d = tid;
        uint32_t cw[kThreads / 64];
        uint32_t total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            cw[w] = total;
            total += wh[w][d];
        }
        uint32_t* st = status + ((int64_t)pass * parts_cap) * kRadix;
        uint32_t excl = 0;
        if (part == 0) {
            __hip_atomic_store(st + d, kPre | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(st + part * kRadix + d, kAgg | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // look-back 8 predecessors per round trip (independent loads in flight)
            int64_t j = part - 1;
            while (true) {
                uint32_t sv[8];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    sv[k] = j - k >= 0 ? __hip_atomic_load(st + (j - k) * kRadix + d, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT)
                                       : kPre;   // before partition 0: an empty inclusive prefix
                int k = 0;
                bool found = false;
                for (; k < 8; ++k) {
                    const uint32_t flag = sv[k] & ~kCnt;
                    if (flag == 0u) break;
                    excl += sv[k] & kCnt;
                    if (flag == kPre) {
                        found = true;
                        break;
                    }
                }
                if (found) break;
                j -= k;
                if (k == 0) __builtin_amdgcn_s_sleep(1);
            }
            __hip_atomic_store(st + part * kRadix + d, kPre | (excl + total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint32_t gbase = digit_off[pass * kRadix + d] + excl;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) wh[w][d] = gbase + cw[w];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        if (idx < P) {
            const uint32_t d = (uint32_t)(k[r] >> shift) & 0xffu;
            const uint32_t pos = wh[wave][d] + rank[r];
            if ((int64_t)pos < P) {
                dk[pos] = k[r];
                dv[pos] = val[r];
            }
        }
    }
}

__global__ void __launch_bounds__(kThreads)
sort_ranges_kernel(uint64_t* __restrict__ keys0, uint32_t* __restrict__ vals0, const uint64_t* __restrict__ keys1,
                   const uint32_t* __restrict__ vals1, const int64_t* __restrict__ num_pairs, int64_t capacity,
                   const int32_t* __restrict__ ctrl, int npass, int64_t total_tiles, uint32_t* __restrict__ ranges) {
    const int64_t P = load_count(num_pairs, capacity);
    const bool alt = ctrl[npass] != 0;
    const uint64_t* k = alt ? keys1 : keys0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < P; i += stride) {
        const uint64_t key = k[i];
        const int64_t t = (int64_t)(key >> 32);
        if (t < total_tiles) {
            if (i == 0 || (k[i - 1] >> 32) != (uint64_t)t) ranges[2 * t] = (uint32_t)i;
            if (i == P - 1 || (k[i + 1] >> 32) != (uint64_t)t) ranges[2 * t + 1] = (uint32_t)(i + 1);
        }
        if (alt) {
            keys0[i] = key;
            vals0[i] = vals1[i];
        }
    }
}

}  // namespace

int fs_sort_passes(int64_t total_tiles) {
    int tile_bits = 1;
    while (tile_bits < 32 && (int64_t(1) << tile_bits) < total_tiles) ++tile_bits;
    return (32 + tile_bits + 7) / 8;
}

int64_t fs_sort_parts(int64_t capacity) { return (capacity + kPart - 1) / kPart; }

hipError_t fs_launch_sort(uint64_t* keys, uint32_t* vals, int64_t capacity, const int64_t* num_pairs, int64_t hint,
                          int64_t total_tiles, uint32_t* ranges, const FsWorkspace& ws, hipStream_t s) {
    const int npass = ws.npass;
    const int64_t parts_cap = ws.sort_parts;
    const int64_t pmax = hint >= 0 ? (hint < capacity ? hint : capacity) : capacity;
    const int64_t parts = (pmax + kPart - 1) / kPart;
    const int64_t nstatus = (int64_t)npass * parts_cap * kRadix;
    {
        int64_t work = nstatus > 2 * total_tiles ? nstatus : 2 * total_tiles;
        unsigned blocks = (unsigned)((work + 255) / 256);
        blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
        hipLaunchKernelGGL(sort_clear_kernel, dim3(blocks), dim3(256), 0, s, ws.hist, (int64_t)npass * kRadix,
                           ws.sort_status, nstatus, ws.sort_ticket, npass, ranges, 2 * total_tiles);
    }
    {
        unsigned blocks = (unsigned)((pmax + kThreads * 8 - 1) / (kThreads * 8));
        blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
        hipLaunchKernelGGL(sort_hist_kernel, dim3(blocks), dim3(kThreads), 0, s, keys, num_pairs, capacity, npass,
                           ws.hist);
    }
    hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(kThreads), 0, s, ws.hist, num_pairs, capacity, npass,
                       ws.digit_off, ws.sort_ctrl);
    if (parts > 0) {
        for (int p = 0; p < npass; ++p)
            hipLaunchKernelGGL(sort_pass_kernel, dim3((unsigned)parts), dim3(kThreads), 0, s, keys, vals, ws.keys_alt,
                               ws.vals_alt, num_pairs, capacity, p, ws.digit_off, ws.sort_ctrl, ws.sort_status,
                               ws.sort_ticket, parts_cap);
    }
    {
        unsigned blocks = (unsigned)((pmax + kThreads * 4 - 1) / (kThreads * 4));
        blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
        hipLaunchKernelGGL(sort_ranges_kernel, dim3(blocks), dim3(kThreads), 0, s, keys, vals, ws.keys_alt,
                           ws.vals_alt, num_pairs, capacity, ws.sort_ctrl, npass, total_tiles, ranges);
    }
    return hipGetLastError();
}
