// sort.hip -- per-tile depth ordering of the (tile << 32 | depth-key, record)
// pairs and per-tile ranges (surfels are blended depth-sorted, Sec. 3.1; the
// pipeline is tile based, Sec. 3.2).
//
// The required order is (tile, depth key, record): the order a stable sort on
// the 64-bit key gives, since a record is emitted at most once per tile and
// records are emitted in increasing order.  It is produced in two steps that
// suit a list split into many short per-tile runs:
//   1. a counting sort by tile: per-tile counts (LDS histograms over the tile
//      window of each 8192-pair chunk), one exclusive scan that also yields
//      every tile's [start, end)
//      range, and a scatter that places each pair at its tile's start plus a
//      cursor (any order inside the tile);
//   2. a sort of every tile's run by (depth key, record), as 64-bit composite
//      keys: runs of up to kWaveCap entries by one wave each (bitonic network
//      in the wave's registers), up to kMergeCap by a workgroup (waves sort
//      512-entry chunks in registers, then pairwise merges in LDS), up to
//      kLargeCap by a workgroup bitonic network in 64 KB of LDS, longer runs
//      by a stable one-workgroup LSD radix sort
//      through global memory.
// Every launch is sized from the capacity, not from the device-side pair
// count, so the sequence can be captured in a graph.
#include "fs_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaveCap = 512;     // entries per run sorted by one wave (8 per lane, in registers)
constexpr int kLargeCap = 8192;   // entries per run sorted in LDS by a workgroup (64 KB)
constexpr int kMergeCap = 4096;   // entries per run sorted by chunk sorts and merges (two 32 KB buffers)
constexpr int kLdsTiles = 16384;  // tile counts kept in LDS by the count and scatter kernels
constexpr int kChunk = 8192;      // pairs per workgroup in the count and scatter kernels
constexpr int kChunkThreads = 1024;
constexpr int kPerThread = kChunk / kChunkThreads;   // pairs per thread and chunk
constexpr int kLongGrid = 512;    // workgroups working through the long-run list
constexpr int kLongThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanPart = kThreads * kScanItems;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPre = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

FS_DEV int64_t load_count(const int64_t* num_pairs, int64_t capacity) {
    const int64_t p = *num_pairs;
    return p < capacity ? p : capacity;
}

__global__ void sort_clear_kernel(uint32_t* __restrict__ cnt, uint32_t* __restrict__ fill, int64_t tiles,
                                  uint64_t* __restrict__ status, int64_t parts, uint32_t* __restrict__ ticket) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tiles; i += stride) {
        cnt[i] = 0;
        fill[i] = 0;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < parts; i += stride) status[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 2) ticket[threadIdx.x] = 0;   // scan ticket, long-run count
}

// Tile window of a chunk of pairs: [lo, hi] over its valid tile ids (lo >
// hi when it has none), reduced over the workgroup.  Pairs are emitted
// record by record and records view by view, so a chunk's tiles lie within
// one view (two where it straddles a boundary): the window of a view with at
// most kLdsTiles tiles fits the LDS histograms below whatever the total.
FS_DEV void chunk_window(const uint64_t* __restrict__ keys, int64_t c0, int64_t c1, int64_t tiles, uint32_t& lo,
                         uint32_t& hi, uint32_t* s_red) {
    uint32_t a = 0xffffffffu, b = 0u;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kChunkThreads) {
        const uint64_t t = keys[i] >> 32;
        if (t < (uint64_t)tiles) {
            a = (uint32_t)t < a ? (uint32_t)t : a;
            b = (uint32_t)t > b ? (uint32_t)t : b;
        }
    }
    a = __ockl_wfred_min_u32(a);
    b = __ockl_wfred_max_u32(b);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_red[2 * wave] = a;
        s_red[2 * wave + 1] = b;
    }
    __syncthreads();
    lo = 0xffffffffu;
    hi = 0u;
    for (int w = 0; w < kChunkThreads / 64; ++w) {
        lo = s_red[2 * w] < lo ? s_red[2 * w] : lo;
        hi = s_red[2 * w + 1] > hi ? s_red[2 * w + 1] : hi;
    }
}

// Per-tile counts.  Every workgroup counts a chunk of kChunk pairs: in an LDS
// histogram over the chunk's tile window when it spans at most kLdsTiles
// tiles, adding its non-zero bins to the global counts (a tile with many
// pairs costs one global atomic per workgroup, not one per pair); with global
// atomics per pair otherwise.
__global__ void __launch_bounds__(kChunkThreads)
sort_count_kernel(const uint64_t* __restrict__ keys, const int64_t* __restrict__ num_pairs, int64_t capacity,
                  int64_t tiles, uint32_t* __restrict__ cnt) {
    __shared__ uint32_t h[kLdsTiles];
    __shared__ uint32_t s_red[2 * (kChunkThreads / 64)];
    const int64_t P = load_count(num_pairs, capacity);
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    if (c0 >= P) return;   // uniform across the workgroup
    const int64_t c1 = c0 + kChunk < P ? c0 + kChunk : P;
    uint32_t lo = 0u, hi = (uint32_t)(tiles - 1);   // all tiles fit: no window needed
    if (tiles > kLdsTiles) {
        chunk_window(keys, c0, c1, tiles, lo, hi, s_red);
        if (hi < lo) return;
    }
    const uint32_t W = hi - lo + 1u;
    if (W > (uint32_t)kLdsTiles) {
        for (int64_t i = c0 + threadIdx.x; i < c1; i += kChunkThreads) {
            const uint64_t t = keys[i] >> 32;
            if (t < (uint64_t)tiles) atomicAdd(&cnt[t], 1u);
        }
        return;
    }
    // the thread's keys of the chunk, all loads in flight together
    uint64_t kk[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const int64_t i = c0 + threadIdx.x + (int64_t)u * kChunkThreads;
        kk[u] = i < c1 ? keys[i] : ~0ull;
    }
    for (uint32_t i = threadIdx.x; i < W; i += kChunkThreads) h[i] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const uint64_t t = kk[u] >> 32;
        if (t < (uint64_t)tiles) atomicAdd(&h[(uint32_t)t - lo], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < W; i += kChunkThreads)
        if (h[i]) atomicAdd(&cnt[lo + i], h[i]);
}

FS_DEV uint32_t wave_inclusive_scan(uint32_t x) { return __ockl_wfscan_add_u32(x, true); }

// Exclusive scan of the tile counts into ranges (single pass: partitions by
// atomic ticket, decoupled look-back with one wave reading 64 predecessors
// per round trip).
__global__ void __launch_bounds__(kThreads)
sort_scan_kernel(const uint32_t* __restrict__ cnt, int64_t tiles, uint32_t* __restrict__ ranges,
                 uint64_t* __restrict__ status, uint32_t* __restrict__ ticket, int64_t parts) {
    __shared__ uint32_t s_part;
    __shared__ uint64_t s_wave[kThreads / 64];
    __shared__ uint64_t s_prefix;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_part = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t part = s_part;
    if (part >= parts) return;
    const int64_t base = part * kScanPart + (int64_t)tid * kScanItems;
    uint32_t c[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        c[j] = base + j < tiles ? cnt[base + j] : 0u;
        sum += c[j];
    }
    const uint32_t incl = wave_inclusive_scan(sum);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint64_t wave_excl = 0, total = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) wave_excl += s_wave[w];
        total += s_wave[w];
    }
    if (wave == 0) {
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
                const uint64_t st = idx >= 0 ? __hip_atomic_load(status + idx, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT)
                                             : kFlagPre;   // before partition 0: an empty inclusive prefix
                const uint64_t flag = st & ~kValMask;
                const uint64_t notready = __ballot(flag == 0);
                const uint64_t pre = __ballot(flag == kFlagPre);
                const int limit = notready ? __builtin_ctzll(notready) : 64;
                const int first_pre = pre ? __builtin_ctzll(pre) : 64;
                const bool found = first_pre < limit;
                const int take = found ? first_pre + 1 : limit;
                uint64_t v = lane < take ? (st & kValMask) : 0ull;
                prefix += __ockl_wfred_add_u64(v);
                if (found) break;
                j -= take;
                if (take == 0) __builtin_amdgcn_s_sleep(1);
            }
            if (lane == 0)
                __hip_atomic_store(status + part, kFlagPre | (prefix + total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) s_prefix = prefix;
    }
    __syncthreads();
    uint64_t off = s_prefix + wave_excl + (incl - sum);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < tiles) {
            ranges[2 * (base + j)] = (uint32_t)off;
            ranges[2 * (base + j) + 1] = (uint32_t)(off + c[j]);
        }
        off += c[j];
    }
}

// Pair i goes to its tile's start plus a cursor, as (depth key, record).
// Per chunk, as in the count: over an LDS window of at most kLdsTiles tiles
// the workgroup reserves, per tile, one run of positions for its whole chunk
// (one global atomic per tile it touches) and hands them out with LDS
// cursors; otherwise every pair takes a global atomic.
__global__ void __launch_bounds__(kChunkThreads)
sort_scatter_kernel(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                    const int64_t* __restrict__ num_pairs, int64_t capacity, int64_t tiles,
                    const uint32_t* __restrict__ ranges, uint32_t* __restrict__ fill, uint2* __restrict__ out) {
    __shared__ uint32_t h[kLdsTiles];
    __shared__ uint32_t s_red[2 * (kChunkThreads / 64)];
    const int64_t P = load_count(num_pairs, capacity);
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    if (c0 >= P) return;   // uniform across the workgroup
    const int64_t c1 = c0 + kChunk < P ? c0 + kChunk : P;
    uint32_t lo = 0u, hi = (uint32_t)(tiles - 1);   // all tiles fit: no window needed
    if (tiles > kLdsTiles) {
        chunk_window(keys, c0, c1, tiles, lo, hi, s_red);
        if (hi < lo) return;
    }
    const uint32_t W = hi - lo + 1u;
    if (W > (uint32_t)kLdsTiles) {
        for (int64_t i = c0 + threadIdx.x; i < c1; i += kChunkThreads) {
            const uint64_t k = keys[i];
            const uint64_t t = k >> 32;
            if (t < (uint64_t)tiles) {
                const uint32_t pos = ranges[2 * t] + atomicAdd(&fill[t], 1u);
                if ((int64_t)pos < P) out[pos] = make_uint2((uint32_t)k, vals[i]);
            }
        }
        return;
    }
    // the thread's pairs of the chunk, all loads in flight together; kept in
    // registers for the scatter below
    uint64_t kk[kPerThread];
    uint32_t vv[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const int64_t i = c0 + threadIdx.x + (int64_t)u * kChunkThreads;
        kk[u] = i < c1 ? keys[i] : ~0ull;
        vv[u] = i < c1 ? vals[i] : 0u;
    }
    for (uint32_t i = threadIdx.x; i < W; i += kChunkThreads) h[i] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const uint64_t t = kk[u] >> 32;
        if (t < (uint64_t)tiles) atomicAdd(&h[(uint32_t)t - lo], 1u);
    }
    __syncthreads();
    // first position of this chunk's run in every tile it touches: the
    // (memory-side) reservations of a thread are independent, so all are
    // issued before the first result is waited for
    static_assert(kLdsTiles % kChunkThreads == 0, "whole rounds of bins");
    constexpr int kRounds = kLdsTiles / kChunkThreads;
    uint32_t cnt[kRounds], got[kRounds], first[kRounds];
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        const uint32_t i = threadIdx.x + (uint32_t)k * kChunkThreads;
        cnt[k] = i < W ? h[i] : 0u;
        got[k] = 0u;
        first[k] = 0u;
        if (cnt[k] != 0u) {
            got[k] = atomicAdd(&fill[lo + i], cnt[k]);
            first[k] = ranges[2 * (lo + i)];
        }
    }
#pragma unroll
    for (int k = 0; k < kRounds; ++k)
        if (cnt[k] != 0u) h[threadIdx.x + k * kChunkThreads] = first[k] + got[k];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const uint64_t t = kk[u] >> 32;
        if (t < (uint64_t)tiles) {
            const uint32_t pos = atomicAdd(&h[(uint32_t)t - lo], 1u);
            if ((int64_t)pos < P) out[pos] = make_uint2((uint32_t)kk[u], vv[u]);
        }
    }
}

FS_DEV uint64_t composite(uint2 e) { return ((uint64_t)e.x << 32) | e.y; }

// Bitonic sort of s[0, n2) (n2 a power of two, padding = ~0) by the workgroup.
template <int NT>
FS_DEV void bitonic_lds(uint64_t* s, int n2) {
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < (n2 >> 1); i += NT) {
                const int a = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const int b = a + j;
                const bool up = (a & k) == 0;
                const uint64_t x = s[a], y = s[b];
                if ((x > y) == up) {
                    s[a] = y;
                    s[b] = x;
                }
            }
            __syncthreads();
        }
    }
}

FS_DEV int next_pow2(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Sort one run of 2 <= n <= capacity of s entries in LDS and write the final
// keys and values.
template <int NT>
FS_DEV void sort_run_lds(uint64_t* s, const uint2* __restrict__ in, uint64_t tile, uint32_t start, int n,
                         uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int n2 = next_pow2(n);
    for (int i = threadIdx.x; i < n2; i += NT) s[i] = i < n ? composite(in[start + i]) : ~0ull;
    __syncthreads();
    bitonic_lds<NT>(s, n2);
    for (int i = threadIdx.x; i < n; i += NT) {
        const uint64_t c = s[i];
        keys[start + i] = (tile << 32) | (c >> 32);
        vals[start + i] = (uint32_t)c;
    }
}

// Bitonic sort of one run of 1 <= n <= 64 E entries by one wave, in
// registers: element i = lane * E + e of the padded run (padding = ~0) is
// x[e] of its lane.  Compare-exchange partners i ^ j with j < E sit in the
// same lane; with j >= E they are the same register of lane ^ (j / E),
// fetched by a shuffle.  The network is the textbook one (stage k, distance
// j, ascending where i & k == 0), so the result is the sorted run.
template <int LOGE>
FS_DEV void sort_run_wave(const uint2* __restrict__ in, uint64_t tile, uint32_t start, int n,
                          uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    constexpr int E = 1 << LOGE;
    const int lane = (int)threadIdx.x & 63;
    uint64_t x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        x[e] = i < n ? composite(in[start + i]) : ~0ull;
    }
    wave_network<LOGE>(x);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        if (i < n) {
            keys[start + i] = (tile << 32) | (x[e] >> 32);
            vals[start + i] = (uint32_t)x[e];
        }
    }
}

// Sort of one run of kWaveCap < n <= kMergeCap entries by the workgroup:
// wave w sorts entries [512 w, 512 w + 512) of the run in registers (padding
// = ~0, which sorts last), then runs of 512, 1024, ... are merged pairwise
// through LDS, ping-ponging between the two halves of s.  Every thread
// makes 8 outputs per round: it finds, by binary search along the merge
// path, how many of its first output's predecessors come from the left run
// (keys are distinct), then merges 8 entries.  At most three rounds.
FS_DEV void sort_run_merge(uint64_t* s, const uint2* __restrict__ in, uint64_t tile, uint32_t start, int n,
                           uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    static_assert(kLongThreads * 8 >= kMergeCap && 2 * kMergeCap <= kLargeCap, "buffers of the merge rounds");
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = (n + kWaveCap - 1) / kWaveCap;   // sorted chunks, 2 .. kMergeCap / kWaveCap
    const int N = m * kWaveCap;
    uint64_t* a = s;
    uint64_t* b = s + kMergeCap;
    if (wave < m) {
        uint64_t x[8];
        const int base = wave * kWaveCap + lane * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = base + e < n ? composite(in[start + base + e]) : ~0ull;
        wave_network<3>(x);
#pragma unroll
        for (int e = 0; e < 8; ++e) a[base + e] = x[e];
    }
    __syncthreads();
    for (int width = kWaveCap; width < N; width *= 2) {
        const int o = tid * 8;   // first output of this thread
        if (o < N) {
            const int ps = (o / (2 * width)) * (2 * width);
            const int na = N - ps < width ? N - ps : width;
            const int nb = N - ps - na < width ? N - ps - na : width;
            const uint64_t* A = a + ps;
            const uint64_t* B = A + na;
            const int d = o - ps;
            int lo = d - nb > 0 ? d - nb : 0, hi = d < na ? d : na;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (A[mid] < B[d - 1 - mid])
                    lo = mid + 1;
                else
                    hi = mid;
            }
            int i = lo, j = d - lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool take_a = j >= nb || (i < na && A[i] < B[j]);
                b[o + e] = take_a ? A[i] : B[j];
                i += take_a ? 1 : 0;
                j += take_a ? 0 : 1;
            }
        }
        __syncthreads();
        uint64_t* t = a;
        a = b;
        b = t;
    }
    for (int i = tid; i < n; i += kLongThreads) {
        const uint64_t c = a[i];
        keys[start + i] = (tile << 32) | (c >> 32);
        vals[start + i] = (uint32_t)c;
    }
}

// One wave per tile: runs of up to kWaveCap entries are sorted in the wave's
// registers (1, 2, 4 or 8 entries per lane by run length); longer runs are
// appended to the list the long-run kernel works through.
__global__ void __launch_bounds__(kThreads)
sort_short_runs_kernel(const uint2* __restrict__ in, const uint32_t* __restrict__ ranges, int64_t tiles,
                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* __restrict__ long_list,
                       uint32_t* __restrict__ long_count) {
    static_assert(kWaveCap == 512, "runs up to 8 entries per lane");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + wave;
    if (t >= tiles) return;   // uniform per wave
    const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
    const int n = (int)(end - start);
    if (n == 0) return;
    if (n > kWaveCap) {
        if (lane == 0) long_list[atomicAdd(long_count, 1u)] = (uint32_t)t;
        return;
    }
    if (n <= 64)
        sort_run_wave<0>(in, (uint64_t)t, start, n, keys, vals);
    else if (n <= 128)
        sort_run_wave<1>(in, (uint64_t)t, start, n, keys, vals);
    else if (n <= 256)
        sort_run_wave<2>(in, (uint64_t)t, start, n, keys, vals);
    else
        sort_run_wave<3>(in, (uint64_t)t, start, n, keys, vals);
}

// Stable LSD radix sort of one run through global memory, 8-bit digits of the
// 64-bit composite key, ping-ponging between a[start, start + n) (input) and
// b[start, start + n); passes whose digit is the same for the whole run are
// skipped.  Ends with the sorted run written as final keys and values (b may
// alias the keys: each thread reads its element before writing it).
template <int NT>
FS_DEV void sort_run_global(uint2* a, uint2* b, uint64_t tile, uint32_t start, uint32_t n,
                            uint64_t* keys, uint32_t* __restrict__ vals, uint32_t* hist, uint32_t* wcnt,
                            uint32_t* flag) {
    constexpr int kWaves = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    uint2* src = a + start;
    uint2* dst = b + start;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        if (tid < 256) hist[tid] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < n; i += NT) atomicAdd(&hist[(composite(src[i]) >> shift) & 0xff], 1u);
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            uint32_t single = 0;
            for (int d = 0; d < 256; ++d) {
                const uint32_t c = hist[d];
                if (c == n) single = 1;   // one digit value: identity permutation
                hist[d] = acc;
                acc += c;
            }
            *flag = single;
        }
        __syncthreads();
        if (*flag) continue;   // uniform
        for (uint32_t c0 = 0; c0 < n; c0 += NT) {
            const uint32_t i = c0 + tid;
            const bool valid = i < n;
            const uint2 e = valid ? src[i] : make_uint2(0u, 0u);
            const uint32_t d = (uint32_t)(composite(e) >> shift) & 0xffu;
            // rank among equal digits of this chunk: inside the wave by ballot
            // matching, across waves from per-wave digit counts
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const bool x = (d >> bit) & 1u;
                const uint64_t bb = __ballot(x);
                peers &= x ? bb : ~bb;
            }
            for (int i = tid; i < kWaves * 256; i += NT) wcnt[i] = 0;
            __syncthreads();
            if (valid && ((peers >> lane) >> 1) == 0ull) wcnt[wave * 256 + d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t before = 0;
                for (int w = 0; w < wave; ++w) before += wcnt[w * 256 + d];
                dst[hist[d] + before + (uint32_t)__popcll(peers & lt)] = e;
            }
            __syncthreads();
            if (tid < 256) {
                uint32_t tot = 0;
                for (int w = 0; w < kWaves; ++w) tot += wcnt[w * 256 + tid];
                hist[tid] += tot;
            }
            __syncthreads();
        }
        uint2* tmp = src;
        src = dst;
        dst = tmp;
    }
    for (uint32_t i = tid; i < n; i += NT) {
        const uint2 e = src[i];
        keys[start + i] = (tile << 32) | e.x;
        vals[start + i] = e.y;
    }
}

// Runs longer than kWaveCap, from the list: up to kLargeCap entries by a
// workgroup bitonic network in LDS, longer ones by the global radix sort.
// Two workgroups per CU (64 VGPRs at most) keep every long run of a frame
// in flight at once.
__global__ void __launch_bounds__(kLongThreads) __attribute__((amdgpu_waves_per_eu(8)))
sort_long_runs_kernel(uint2* __restrict__ in, const uint32_t* __restrict__ ranges,
                      const uint32_t* __restrict__ long_list, const uint32_t* __restrict__ long_count,
                      uint64_t* keys, uint32_t* __restrict__ vals) {
    __shared__ uint64_t s[kLargeCap];
    const uint32_t count = *long_count;
    for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
        const uint64_t t = long_list[it];
        const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
        const uint32_t n = end - start;
        if (n <= (uint32_t)kMergeCap) {
            sort_run_merge(s, in, t, start, (int)n, keys, vals);
        } else if (n <= (uint32_t)kLargeCap) {
            sort_run_lds<kLongThreads>(s, in, t, start, (int)n, keys, vals);
        } else {
            // the run's own slice of the key array is the radix passes' second
            // buffer; LDS holds their counters
            uint32_t* hist = reinterpret_cast<uint32_t*>(s);
            uint32_t* wcnt = hist + 256;
            uint32_t* flag = wcnt + (kLongThreads / 64) * 256;
            sort_run_global<kLongThreads>(in, reinterpret_cast<uint2*>(keys), t, start, n, keys, vals, hist, wcnt, flag);
        }
        __syncthreads();   // LDS is reused by the next run
    }
}

}  // namespace

int64_t fs_sort_scan_parts(int64_t total_tiles) { return (total_tiles + kScanPart - 1) / kScanPart; }

hipError_t fs_launch_sort(uint64_t* keys, uint32_t* vals, int64_t capacity, const int64_t* num_pairs, int64_t hint,
                          int64_t total_tiles, uint32_t* ranges, const FsWorkspace& ws, hipStream_t s) {
    if (total_tiles >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    const int64_t pmax = hint >= 0 ? (hint < capacity ? hint : capacity) : capacity;
    const int64_t parts = fs_sort_scan_parts(total_tiles);
    {
        const int64_t work = total_tiles > parts ? total_tiles : parts;
        unsigned blocks = (unsigned)((work + 255) / 256);
        blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
        hipLaunchKernelGGL(sort_clear_kernel, dim3(blocks), dim3(256), 0, s, ws.tile_cnt, ws.tile_fill, total_tiles,
                           ws.sort_status, parts, ws.sort_ticket);
    }
    const int64_t chunks = (pmax + kChunk - 1) / kChunk;
    if (chunks >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    const unsigned pblocks = (unsigned)(chunks < 1 ? 1 : chunks);
    hipLaunchKernelGGL(sort_count_kernel, dim3(pblocks), dim3(kChunkThreads), 0, s, keys, num_pairs, capacity,
                       total_tiles, ws.tile_cnt);
    hipLaunchKernelGGL(sort_scan_kernel, dim3((unsigned)parts), dim3(kThreads), 0, s, ws.tile_cnt, total_tiles, ranges,
                       ws.sort_status, ws.sort_ticket, parts);
    hipLaunchKernelGGL(sort_scatter_kernel, dim3(pblocks), dim3(kChunkThreads), 0, s, keys, vals, num_pairs, capacity,
                       total_tiles, ranges, ws.tile_fill, ws.runs);
    const unsigned sblocks = (unsigned)((total_tiles + kThreads / 64 - 1) / (kThreads / 64));
    hipLaunchKernelGGL(sort_short_runs_kernel, dim3(sblocks), dim3(kThreads), 0, s, ws.runs, ranges, total_tiles, keys,
                       vals, ws.long_list, ws.sort_ticket + 1);
    hipLaunchKernelGGL(sort_long_runs_kernel, dim3(kLongGrid), dim3(kLongThreads), 0, s, ws.runs, ranges, ws.long_list,
                       ws.sort_ticket + 1, keys, vals);
    return hipGetLastError();
}
