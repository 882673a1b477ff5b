// render_topk.hip -- Top-K hard selection (Sec. 3.4) as two passes.
//
// Selection (lanes = pixels, one wave per 8x8 block): walks the block's
// depth-sorted tile list front to back with exactly the per-pixel arithmetic
// of the fused renderer (ray-splat response, alpha, transmittance, the T_stop
// and K tests) and writes, for every pixel, the row slot and blend weight
// w = alpha T of each of its first K blended surfels (or, by weight, of the K
// heaviest of its walk) to the workspace, the block's row list (slot ->
// surfel), plus the final transmittance, blend count and optional index
// outputs.  It holds no feature data, so it runs at high occupancy and hides
// the latency of its dependent list -> record loads behind other waves.
//
// Gather (one workgroup per block, a few lanes per pixel, each owning some
// 16-byte channel vectors of it): stages the block's lists and its rows in
// LDS, then every thread accumulates w * c over its pixels' lists in list
// order with the same fused multiply-adds as the fused renderer, so both
// schedules give the same bits.  A thread walks its pixels' lists one after
// the other (LDS pair read, then row read), so few pixels per thread and
// several vectors each keep those chains short.
// This pass is a stream: the feature image written (pixel-major, C floats per
// pixel) dominates its traffic, and the rows it reads are shared by
// neighbouring blocks and served mostly by L2.
//
// Both launches hand the XCDs one tile row of blocks each in turn
// (neighbouring tiles share surfels, so their records and rows stay in that
// XCD's L2, while every XCD gets its share of the dense regions; one
// contiguous eighth of the image per XCD left the XCDs holding the dense
// bands last: render 216 vs 209 us on the 1280x720 frame).
#include "fs_internal.h"

namespace {

constexpr int kSelBatch = 32;   // list entries staged per step in the selection pass
constexpr int kEvalPairs = 2;   // (entry, pixel) pairs a selection lane evaluates per round
constexpr uint32_t kSelLong = 48;   // blocks with longer tile lists are selected first
constexpr int kSelGroup = 256;       // blocks per group of the long-block list
constexpr int kGatherThreads = 256;
constexpr int kGatherUnroll = 8;  // (surfel, weight) pairs whose row loads are in flight together
constexpr int kStagedK = 16;      // largest K of the staged gather (its lists live in LDS)
constexpr int kCompactK = FS_TOPK_COMPACT_K;   // K up to which the selection writes compact lists
static_assert(kStagedK <= kCompactK, "the staged gather reads compact lists");

// KC > 0: every pixel's list (at most KC pairs) is kept in LDS during the
// walk and written compactly at the end; KC = 0: lists written in place.
template <int KC, bool BYW, bool EXT>
struct SelShared {
    FsRecord rec[kSelBatch];
    uint32_t recid[kSelBatch];
    uint32_t sidx[kSelBatch];
    int pre[kSelBatch];            // exclusive prefix of the entries' pair counts
    uint64_t pixels[kSelBatch];    // per entry: pixels of the block inside its box that are still walking
    uint32_t mask[64];             // per pixel: entries of the batch it accepts
    uint2 list[64 * (KC > 0 ? KC : 1)];   // per pixel: (batch entry, then row slot; weight)
    uint32_t uniq[BYW ? 64 * KC : 1];     // by weight: the block's distinct selected records
    double2 mu[EXT ? kSelBatch : 1];      // low-pass: projected centre relative to the anchor
    float4 geo[EXT ? kSelBatch : 1];      // depth and normal outputs: camera-facing normal, centre depth
};

// The blocks whose tile list holds more than kSelLong entries, per group of
// kSelGroup consecutive blocks: their indices at long[g * kSelGroup ..] and
// their number at counts[g].  No atomics and nothing to clear beforehand.
__global__ void __launch_bounds__(kSelGroup)
select_long_kernel(const uint32_t* __restrict__ ranges, int sb2, int64_t nblocks, uint32_t* __restrict__ lng,
                   uint32_t* __restrict__ counts) {
    __shared__ uint32_t s_wave[kSelGroup / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b = (int64_t)blockIdx.x * kSelGroup + tid;
    bool is_long = false;
    if (b < nblocks) {
        const int64_t t = b / sb2;
        is_long = ranges[2 * t + 1] - ranges[2 * t] > kSelLong;
    }
    const uint64_t m = __ballot(is_long);
    if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kSelGroup / 64; ++w) {
        before += w < wave ? s_wave[w] : 0u;
        total += s_wave[w];
    }
    if (is_long) lng[(int64_t)blockIdx.x * kSelGroup + before + __popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)b;
    if (tid == 0) counts[blockIdx.x] = total;
}

// Synchronisation of one selection wave with itself.  A workgroup holds
// WPG independent selection waves (one 8x8 block each); a wave's LDS
// operations complete in issue order, so the waves need no workgroup barrier,
// only a fence that keeps the compiler from moving LDS accesses across it.
template <int WPG>
FS_DEV void sel_sync() {
    if constexpr (WPG == 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Block of a selection wave.  The first ceil(nblocks / WPG) workgroups
// (dispatched first) take the long-list blocks, the i-th wave of them the
// i-th long block; the others take every block in grid order, WPG
// consecutive blocks per workgroup, and skip the long ones.  Returns -1 for
// a wave without a block.
template <int WPG>
FS_DEV int64_t select_block_of(int64_t nblocks, const fs_camera* cams, int S, int sb2, const uint32_t* ranges,
                               const uint32_t* lng, const uint32_t* counts) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nwg = (nblocks + WPG - 1) / WPG;   // workgroups of each part
    const int64_t wg = blockIdx.x;
    if (wg >= nwg) {
        const int64_t chunk = block_row_chunk(cams, S) / WPG;
        const int64_t b = xcd_remap_chunked(wg - nwg, nwg, chunk > 0 ? chunk : 1) * WPG + wave;
        if (b >= nblocks) return -1;
        const int64_t t = b / sb2;
        return ranges[2 * t + 1] - ranges[2 * t] > kSelLong ? -1 : b;
    }
    const int64_t g = wg * WPG + wave;   // the long block of this wave
    // the group holding long block g: running sum of the groups' counts
    const int64_t ngroups = (nblocks + kSelGroup - 1) / kSelGroup;
    uint32_t run = 0;
    for (int64_t c0 = 0; c0 < ngroups; c0 += 64) {
        const uint32_t c = c0 + lane < ngroups ? counts[c0 + lane] : 0u;
        const uint32_t incl = __ockl_wfscan_add_u32(c, true);
        const uint64_t past = __ballot((int64_t)(run + incl) > g);
        if (past) {
            const int l = __builtin_ctzll(past);
            const uint32_t excl = run + __builtin_amdgcn_readlane(incl, l) - __builtin_amdgcn_readlane(c, l);
            return lng[(c0 + l) * kSelGroup + (g - excl)];
        }
        run += __builtin_amdgcn_readlane(incl, 63);
    }
    return -1;   // fewer long blocks than g + 1
}

// List layout in the workspace, per 8x8 block b (region b * 64 * K of the
// pair array): with KC > 0 the pairs of pixel p start at the sum of the
// counts of pixels 0 .. p - 1 (compact), and nrows[b] = rows | pairs << 16;
// with KC = 0 they start at p * K and nrows[b] = rows.
// BYW (Top-K by weight, KC > 0): no pixel stops at K; each keeps, in its LDS
// list and in depth order, the K blended entries of largest weight seen so
// far (list position, weight).  After the walk the block's distinct selected
// list positions are sorted and numbered: they are its row list, in list
// order as in the first-K mode, and every pair's position becomes its slot.
// EXT (first K only): the low-pass response (o.lowpass) and the depth and
// normal outputs, summed with the weights the lists hold.
template <int KC, bool BYW, bool EXT, int WPG>
__global__ void __launch_bounds__(64 * WPG)
topk_select_kernel(const FsRecord* __restrict__ records, const uint64_t* __restrict__ keys,
                   const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges, uint32_t n,
                   int64_t num_records, const fs_camera* __restrict__ cams, int num_views, int S, fs_opts o,
                   int64_t nblocks, uint2* __restrict__ pairs, uint32_t* __restrict__ rows,
                   uint32_t* __restrict__ nrows, float* __restrict__ out_T, int32_t* __restrict__ out_n,
                   int32_t* __restrict__ out_last, int32_t* __restrict__ out_idx, float* __restrict__ out_depth,
                   float* __restrict__ out_normal, uint64_t* __restrict__ counters,
                   const uint32_t* __restrict__ lng, const uint32_t* __restrict__ lcounts) {
    constexpr int BG = kSelBatch;
    constexpr int kQ = FS_RECORD_BYTES / 16;          // float4 per record
    constexpr int kRecSlots = (BG * kQ + 63) / 64;    // record float4 per lane
    static_assert(!BYW || KC > 0, "the by-weight lists live in LDS");
    static_assert(!(BYW && EXT), "no extended outputs for the by-weight selection");
    __shared__ SelShared<KC, BYW, EXT> sm_waves[WPG];
    SelShared<KC, BYW, EXT>& sm = sm_waves[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int sb2 = (S / 8) * (S / 8);
    const int64_t block = select_block_of<WPG>(nblocks, cams, S, sb2, ranges, lng, lcounts);
    if (block < 0) return;   // uniform across the wave
    const BlockPos bp = locate_block(block, S, 8, cams, num_views);
    if (!bp.valid) return;
    const fs_camera& cam = cams[bp.view];
    const int px = bp.x0 + (lane & 7), py = bp.y0 + (lane >> 3);
    const bool inside = px < cam.width && py < cam.height;
    const int64_t pix = cam.pixel_offset + (int64_t)py * cam.width + px;
    const uint32_t start = ranges[2 * bp.tile], end = ranges[2 * bp.tile + 1];
    const int K = o.topk;
    uint2* __restrict__ mine = pairs + (block * 64 + lane) * (int64_t)K;
    uint32_t* __restrict__ rowlist = rows + block * 64 * (int64_t)K;

    double T = 1.0;
    int cnt = 0;
    int last = -1;
    bool done = !inside;
    const double t_stop = o.t_stop;
    const float neg_half_log2e = -0.72134752044448170f;   // -log2(e) / 2
    uint32_t walked = 0;
    uint32_t nslots = 0;   // rows of the block's row list so far
    const bool lowpass = EXT && o.lowpass != 0;
    const bool geo = EXT && (out_depth != nullptr || out_normal != nullptr);
    float gD = 0.f, gN0 = 0.f, gN1 = 0.f, gN2 = 0.f;   // depth and normal sums

    // list values of batch b + 2 and records of batch b + 1 are in flight
    // while batch b is walked
    float4 pre[kRecSlots];
    uint32_t pre_rid[kRecSlots];
    uint32_t nxt_rid[kRecSlots];
    auto fetch_vals = [&](uint32_t b0, uint32_t* rid) {
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int e = (lane + j * 64) / kQ;
            rid[j] = (e < BG && b0 + (uint32_t)e < end) ? vals[b0 + e] : 0xffffffffu;
        }
    };
    auto fetch_records = [&](const uint32_t* rid) {
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int q = (lane + j * 64) % kQ;
            pre_rid[j] = rid[j];
            pre[j] = make_float4(0.f, 0.f, 0.f, 0.f);
            if ((int64_t)rid[j] < num_records) pre[j] = reinterpret_cast<const float4*>(records + rid[j])[q];
        }
    };
    if (start < end) {
        uint32_t r0[kRecSlots];
        fetch_vals(start, r0);
        fetch_records(r0);
        fetch_vals(start + BG, nxt_rid);
    }

    for (uint32_t b0 = start; b0 < end; b0 += BG) {
        const int nb = (int)(end - b0 < (uint32_t)BG ? end - b0 : (uint32_t)BG);
        sel_sync<WPG>();   // the previous batch's records are no longer read
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int t = lane + j * 64;
            const int e = t / kQ, q = t - e * kQ;
            if (e < nb) {
                float4 v4 = pre[j];
                uint32_t rid = pre_rid[j];
                if ((int64_t)rid >= num_records) {   // never happens for a well-formed list
                    rid = 0u;
                    v4 = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (q == 4) v4.w = __int_as_float((int)0xbff00000);   // k2 = -1: never accepted
                    if (q == 5) v4.z = __int_as_float(1);                 // empty box
                }
                reinterpret_cast<float4*>(&sm.rec[e])[q] = v4;
                if (q == 0) {
                    sm.recid[e] = rid;
                    sm.sidx[e] = rid % n;
                }
            }
        }
        sel_sync<WPG>();
        if (b0 + BG < end) {
            fetch_records(nxt_rid);
            fetch_vals(b0 + 2 * BG, nxt_rid);
        }
        walked += (uint32_t)nb;
        // (a) responses, compacted to the footprints: every entry's pixel box
        //     is clipped to the block and to the pixels still walking, the
        //     (entry, pixel) pairs of the batch are numbered consecutively and
        //     one lane evaluates one pair, so the FP64 work follows the
        //     footprints' area over the active pixels, not 64 pixels per
        //     entry.  Accepted pairs leave a mask bit in LDS.
        const uint64_t walking = __ballot(!done);
        int ecount = 0;
        uint64_t epix = 0ull;
        if (lane < nb) {
            const FsRecord& r = sm.rec[lane];
            if constexpr (EXT) {
                if (lowpass) {
                    double mx, my;
                    fs_record_centre(r, mx, my);
                    sm.mu[lane] = make_double2(mx, my);
                }
                if (geo) {
                    const float3 nrm = fs_record_normal(r, cam);
                    // the centre depth is needed (and keys given) only for the depth output
                    sm.geo[lane] = make_float4(nrm.x, nrm.y, nrm.z,
                                               keys ? __uint_as_float((uint32_t)keys[b0 + lane]) : 0.f);
                }
            }
            const int x0 = max((int)r.x0, bp.x0), x1 = min((int)r.x1, bp.x0 + 7);
            const int y0 = max((int)r.y0, bp.y0), y1 = min((int)r.y1, bp.y0 + 7);
            if (x0 <= x1 && y0 <= y1) {
                const uint64_t row = ((1ull << (x1 - x0 + 1)) - 1ull) << (x0 - bp.x0);   // bits of one pixel row
                const int ny = y1 - y0 + 1;
                const uint64_t rows = (ny == 8 ? ~0ull : ((1ull << (8 * ny)) - 1ull)) << (8 * (y0 - bp.y0));
                epix = (row * 0x0101010101010101ull) & rows & walking;
                ecount = __popcll(epix);
            }
        }
        const int incl = __ockl_wfscan_add_i32(ecount, true);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        if (lane < BG) {
            sm.pre[lane] = lane < nb ? incl - ecount : total;
            sm.pixels[lane] = epix;
        }
        sm.mask[lane] = 0u;
        sel_sync<WPG>();
        // kEvalPairs pairs per lane and round, as straight-line code (pairs
        // past the end evaluate the last pair again and set no bit), so the
        // dependent LDS reads and FP64 chains of the pairs overlap
        for (int k0 = 0; k0 < total; k0 += 64 * kEvalPairs) {
            int pe[kEvalPairs], pp[kEvalPairs];
            bool hitp[kEvalPairs];
#pragma unroll
            for (int u = 0; u < kEvalPairs; ++u) {
                const int k0u = k0 + u * 64 + lane;
                const int k = k0u < total ? k0u : total - 1;
                int e = 0;   // the entry owning pair k: last e with pre[e] <= k
#pragma unroll
                for (int step = BG / 2; step > 0; step >>= 1)
                    if (sm.pre[e + step] <= k) e += step;
                // the m-th set bit of the entry's pixel mask
                int m = k - sm.pre[e];
                uint64_t x = sm.pixels[e];
                int p = 0;
#pragma unroll
                for (int sh = 32; sh >= 1; sh >>= 1) {
                    const int c = __popcll(x & ((1ull << sh) - 1ull));
                    if (m >= c) {
                        m -= c;
                        x >>= sh;
                        p += sh;
                    }
                }
                pe[u] = e;
                pp[u] = p;
            }
#pragma unroll
            for (int u = 0; u < kEvalPairs; ++u) {
                const int e = pe[u], p = pp[u];
                const int lx = p & 7, ly = p >> 3;
                const FsRecord& r = sm.rec[e];
                const double ddx = (double)(bp.x0 + lx - r.ax), ddy = (double)(bp.y0 + ly - r.ay);
                FsResp rs = fs_response(r, ddx, ddy);
                if constexpr (EXT)
                    if (lowpass) fs_lowpass_d2(rs, ddx, ddy, sm.mu[e].x, sm.mu[e].y);
                hitp[u] = k0 + u * 64 + lane < total && rs.d2 <= r.k2;
            }
#pragma unroll
            for (int u = 0; u < kEvalPairs; ++u)
                if (hitp[u]) atomicOr(&sm.mask[pp[u]], 1u << pe[u]);
        }
        sel_sync<WPG>();
        // (b) lane = pixel: front-to-back transmittance over its accepted
        //     entries (alpha recomputed from the same response: the accepted
        //     pairs are few, and keeping alpha for every pair would cost LDS,
        //     hence occupancy); with KC > 0 every blended entry's weight
        //     w = alpha T goes to the pixel's LDS list here
        uint32_t hit = done ? 0u : sm.mask[lane];
        uint32_t bm = 0u;
        const int c_start = cnt;
        const double T_start = T;
        auto resp_of = [&](int e) {
            const FsRecord& r = sm.rec[e];
            const double ddx = (double)(px - r.ax), ddy = (double)(py - r.ay);
            FsResp rs = fs_response(r, ddx, ddy);
            if constexpr (EXT)
                if (lowpass) fs_lowpass_d2(rs, ddx, ddy, sm.mu[e].x, sm.mu[e].y);
            return rs;
        };
        auto alpha_from = [&](int e, const FsResp& rs) {
            const float G = __builtin_amdgcn_exp2f(neg_half_log2e * (float)rs.d2);
            return fminf(o.alpha_max, sm.rec[e].o * G);
        };
        auto alpha_of = [&](int e) { return alpha_from(e, resp_of(e)); };
        while (hit != 0u && !done) {
            const int e = __builtin_ctz(hit);
            hit &= hit - 1u;
            const FsResp rs = resp_of(e);
            const float al = alpha_from(e, rs);
            const double Tn = T * (1.0 - (double)al);
            if (Tn < t_stop) {
                done = true;
            } else if constexpr (BYW) {
                // the entry a full list drops: the lightest, the back one on
                // ties; a new entry enters only if strictly heavier
                const float w = (float)((double)al * T);
                uint2* __restrict__ lst = &sm.list[lane * KC];
                if (cnt < K) {
                    lst[cnt] = make_uint2(b0 + (uint32_t)e, __float_as_uint(w));
                    ++cnt;
                } else {
                    int m = 0;
                    float wm = __uint_as_float(lst[0].y);
                    for (int j = 1; j < K; ++j) {
                        const float wj = __uint_as_float(lst[j].y);
                        if (wj <= wm) {
                            wm = wj;
                            m = j;
                        }
                    }
                    if (w > wm) {
                        for (int j = m; j < K - 1; ++j) lst[j] = lst[j + 1];
                        lst[K - 1] = make_uint2(b0 + (uint32_t)e, __float_as_uint(w));
                    }
                }
                T = Tn;
                last = (int)(b0 + e);
            } else {
                bm |= 1u << e;
                if constexpr (KC > 0) {
                    sm.list[lane * KC + cnt] = make_uint2((uint32_t)e, __float_as_uint((float)((double)al * T)));
                    if (out_idx) out_idx[pix * K + cnt] = (int32_t)sm.recid[e];
                }
                if constexpr (EXT) {
                    if (geo) {
                        const float w = (float)((double)al * T);
                        const float4 gg = sm.geo[e];
                        gD = fmaf(w, (float)((double)gg.w * rs.rh), gD);
                        gN0 = fmaf(w, gg.x, gN0);
                        gN1 = fmaf(w, gg.y, gN1);
                        gN2 = fmaf(w, gg.z, gN2);
                    }
                }
                T = Tn;
                ++cnt;
                last = (int)(b0 + e);
                if (cnt == K) done = true;
            }
        }
        if constexpr (BYW) {
            if (__all(done)) break;
            continue;   // rows are numbered after the walk
        }
        // (c) row slots: the entries any pixel of the block blends get
        //     consecutive slots of the block's row list, in list order
        const uint32_t used = __ockl_wfred_or_u32(bm);
        if constexpr (KC > 0) {
            for (int j = c_start; j < cnt; ++j) {
                const uint32_t e = sm.list[lane * KC + j].x;
                sm.list[lane * KC + j].x = nslots + (uint32_t)__popc(used & ((1u << e) - 1u));
            }
        } else {
            // the blended entries again, in order, with the same arithmetic:
            // w = alpha T and T *= 1 - alpha from the batch's starting T
            uint32_t mm = bm;
            int j = c_start;
            double Tr = T_start;
            while (mm != 0u) {
                const int e = __builtin_ctz(mm);
                mm &= mm - 1u;
                const float al = alpha_of(e);
                const float w = (float)((double)al * Tr);
                Tr = Tr * (1.0 - (double)al);
                const uint32_t slot = nslots + (uint32_t)__popc(used & ((1u << e) - 1u));
                mine[j] = make_uint2(slot, __float_as_uint(w));
                if (out_idx) out_idx[pix * K + j] = (int32_t)sm.recid[e];
                ++j;
            }
        }
        if (lane < BG && ((used >> lane) & 1u))
            rowlist[nslots + (uint32_t)__popc(used & ((1u << lane) - 1u))] = sm.sidx[lane];
        nslots += (uint32_t)__popc(used);
        if (__all(done)) break;
    }

    if constexpr (BYW) {
        constexpr int LOGE = KC == 8 ? 3 : 4;
        static_assert(KC == (1 << LOGE), "one register per list slot");
        uint2* __restrict__ lst = &sm.list[lane * KC];
        // the block's distinct selected list positions, sorted (a record
        // holds one position of the tile's list, and numbering rows by
        // position keeps every pixel's slots increasing, as the gather's
        // row windows need): element lane * KC + j is x[j]
        uint64_t x[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            x[j] = ~0ull;
            if (j < cnt) {
                x[j] = lst[j].x;
                if (out_idx) out_idx[pix * K + j] = (int32_t)vals[lst[j].x];
            }
        }
        wave_network<LOGE>(x);
        const uint64_t before = __shfl_up(x[KC - 1], 1, 64);
        uint32_t heads = 0u;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const uint64_t prev = j > 0 ? x[j - 1] : (lane > 0 ? before : ~0ull);
            if (x[j] != ~0ull && x[j] != prev) heads |= 1u << j;
        }
        const int nh = __popc(heads);
        int incl = nh;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        const uint32_t R = (uint32_t)__shfl(incl, 63, 64);
        int rank = incl - nh;
#pragma unroll
        for (int j = 0; j < KC; ++j)
            if ((heads >> j) & 1u) sm.uniq[rank++] = (uint32_t)x[j];
        sel_sync<WPG>();
        // every pair's row slot: the rank of its position
        for (int j = 0; j < cnt; ++j) {
            const uint32_t pos = lst[j].x;
            uint32_t lo = 0u, hi = R;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (sm.uniq[mid] < pos)
                    lo = mid + 1u;
                else
                    hi = mid;
            }
            lst[j].x = lo;
        }
        for (uint32_t t = (uint32_t)lane; t < R; t += 64u) rowlist[t] = vals[sm.uniq[t]] % n;
        nslots = R;
    }
    if (counters != nullptr) {
        int c = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) c += __shfl_xor(c, d, 64);
        if (lane == 0) {
            atomicAdd((unsigned long long*)&counters[0], (unsigned long long)walked);
            atomicAdd((unsigned long long*)&counters[1], (unsigned long long)nslots);
            atomicAdd((unsigned long long*)&counters[2], (unsigned long long)c);
            atomicAdd((unsigned long long*)&counters[3], 1ull);
        }
    }
    if constexpr (KC > 0) {
        // compact lists: pixel p's pairs after those of pixels 0 .. p - 1
        const int incl = __ockl_wfscan_add_i32(cnt, true);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        uint2* __restrict__ dst = pairs + block * 64 * (int64_t)K + (incl - cnt);
        for (int j = 0; j < cnt; ++j) dst[j] = sm.list[lane * KC + j];
        if (lane == 0) nrows[block] = nslots | ((uint32_t)total << 16);
    } else {
        if (lane == 0) nrows[block] = nslots;
    }
    if (inside) {
        if (out_T) out_T[pix] = (float)T;
        out_n[pix] = cnt;
        if (out_last) out_last[pix] = last;
        if (out_idx)
            for (int j = cnt; j < K; ++j) out_idx[pix * K + j] = -1;
        if constexpr (EXT) {
            if (out_depth) out_depth[pix] = gD;
            if (out_normal) {
                out_normal[3 * pix] = gN0;
                out_normal[3 * pix + 1] = gN1;
                out_normal[3 * pix + 2] = gN2;
            }
        }
    }
}

// Feature vector of VE elements (16 bytes, or one element when C does not
// allow aligned vectors) widened to float32.
template <typename FT, int VE>
struct Vec;
template <>
struct Vec<float, 4> {
    using raw = float4;
    FS_DEV static raw load(const float* p) { return *reinterpret_cast<const float4*>(p); }
    FS_DEV static float at(const raw& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
};
template <>
struct Vec<float, 1> {
    using raw = float;
    FS_DEV static raw load(const float* p) { return *p; }
    FS_DEV static float at(const raw& v, int) { return v; }
};
template <>
struct Vec<uint16_t, 8> {
    using raw = uint4;
    FS_DEV static raw load(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
    FS_DEV static float at(const raw& v, int i) {
        const uint32_t w = i < 2 ? v.x : i < 4 ? v.y : i < 6 ? v.z : v.w;
        return __uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
    }
};
template <>
struct Vec<uint16_t, 1> {
    using raw = uint16_t;
    FS_DEV static raw load(const uint16_t* p) { return *p; }
    FS_DEV static float at(const raw& v, int) { return __uint_as_float((uint32_t)v << 16); }
};

// Store VE accumulated channels at dst[c0 ...] (c0 + VE <= C for vectors).
// The feature image is written once and not read back by this pass:
// non-temporal stores stream it out without evicting the feature rows that
// neighbouring blocks still read from L2, where one store instruction fills
// whole lines (VE = 4: a wave writes 1 KB contiguously).  With VE = 8 each
// instruction covers only every other 16 bytes of its lines; streamed that
// way the lines go out half-written, so those use ordinary stores, which
// L2 merges (measured: 0.77 -> 0.67 ms for the C = 256 bfloat16 frame).
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int VE>
FS_DEV void store_vec(float* __restrict__ dst, int c0, const float* acc) {
    if constexpr (VE == 4) {
        __builtin_nontemporal_store(f32x4{acc[0], acc[1], acc[2], acc[3]}, reinterpret_cast<f32x4*>(dst + c0));
    } else if constexpr (VE == 8) {
        *reinterpret_cast<f32x4*>(dst + c0) = f32x4{acc[0], acc[1], acc[2], acc[3]};
        *reinterpret_cast<f32x4*>(dst + c0 + 4) = f32x4{acc[4], acc[5], acc[6], acc[7]};
    } else {
        __builtin_nontemporal_store(acc[0], dst + c0);
    }
}

// Label epilogue: in place of its feature vector a pixel gets the channel
// holding its largest blended value (equal values go to the lower channel)
// and that value.  Each thread reduces its own channels, then the TPP lanes
// of the pixel (consecutive lanes of one wave) exchange their candidates.
FS_DEV void argmax_take(float x, int c, float& v, int& cv) {
    if (x > v || (x == v && c < cv)) {
        v = x;
        cv = c;
    }
}
template <int TPP>
FS_DEV void argmax_lanes(float& v, int& c) {
#pragma unroll
    for (int d = 1; d < TPP; d <<= 1)
        argmax_take(__uint_as_float(lane_xor32(__float_as_uint(v), d)), (int)lane_xor32((uint32_t)c, d), v, c);
}

// Value of lane l (0 <= l < TPP) of the caller's group of TPP consecutive
// lanes; l may differ between groups.  For groups of four, the four quad
// broadcasts and a selection, in the vector pipeline.
template <int TPP>
FS_DEV int group_lane(int v, int l) {
    if constexpr (TPP == 4) {
        const int b0 = __builtin_amdgcn_mov_dpp(v, 0x00, 0xF, 0xF, false);   // quad_perm [0, 0, 0, 0]
        const int b1 = __builtin_amdgcn_mov_dpp(v, 0x55, 0xF, 0xF, false);   // quad_perm [1, 1, 1, 1]
        const int b2 = __builtin_amdgcn_mov_dpp(v, 0xAA, 0xF, 0xF, false);   // quad_perm [2, 2, 2, 2]
        const int b3 = __builtin_amdgcn_mov_dpp(v, 0xFF, 0xF, 0xF, false);   // quad_perm [3, 3, 3, 3]
        return l == 0 ? b0 : l == 1 ? b1 : l == 2 ? b2 : b3;
    } else {
        return __shfl(v, ((int)threadIdx.x & 63 & ~(TPP - 1)) + l, 64);
    }
}
// Largest v over aligned groups of TPP lanes, every lane of the group
// getting it: in-row DPP moves (quad swaps, then the mirrors within 8 and 16
// lanes, each combining two halves already reduced) and one cross-row
// exchange per further doubling.  Every lane of the wave must be active.
template <int CTRL>
FS_DEV float max_dpp(float v) {
    return fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false)));
}
template <int TPP>
FS_DEV float lanes_max(float v) {
    v = max_dpp<0xb1>(v);                                  // quad_perm [1, 0, 3, 2]
    v = max_dpp<0x4e>(v);                                  // quad_perm [2, 3, 0, 1]
    if constexpr (TPP >= 8) v = max_dpp<0x141>(v);         // row_half_mirror
    if constexpr (TPP >= 16) v = max_dpp<0x140>(v);        // row_mirror
    if constexpr (TPP >= 32) v = fmaxf(v, __shfl_xor(v, 16, 64));
    if constexpr (TPP >= 64) v = fmaxf(v, __shfl_xor(v, 32, 64));
    return v;
}
constexpr float kNoValue = -__builtin_huge_valf();
constexpr int kNoChannel = 0x7fffffff;

// Gather, general form: TPP threads per pixel (a power of two, 4..64), each
// taking channel vectors q, q + TPP, ... of its pixel and reading the pixel's
// (slot, weight) list and the block's row list from memory.  A workgroup
// covers 256 / TPP pixels of one 8x8 block.  Used when a pixel has more
// channels or list slots than the staged form holds.
template <typename FT, int VE, int TPP, bool LABEL>
__global__ void __launch_bounds__(kGatherThreads)
topk_gather_general_kernel(const uint2* __restrict__ pairs, const int32_t* __restrict__ counts,
                           const uint32_t* __restrict__ rows, const FT* __restrict__ feats, int C, int K,
                           const fs_camera* __restrict__ cams, int num_views, int S, int64_t ngroups,
                           float* __restrict__ out_feat, int32_t* __restrict__ out_label,
                           float* __restrict__ out_score) {
    using V = Vec<FT, VE>;
    constexpr int kPix = kGatherThreads / TPP;   // pixels per workgroup
    constexpr int kGroups = 64 / kPix;           // workgroups per block
    __shared__ int s_off[64];
    const int64_t g = xcd_remap(blockIdx.x, ngroups);
    const int64_t block = g / kGroups;
    const BlockPos bp = locate_block(block, S, 8, cams, num_views);
    if (!bp.valid) return;   // uniform over the workgroup
    const fs_camera& cam = cams[bp.view];
    const bool compact = K <= kCompactK;   // the selection's list layout
    if (compact) {
        // offsets of the pixels' lists: prefix of the block's counts
        const int t = (int)threadIdx.x;
        if (t < 64) {
            const int qx = bp.x0 + (t & 7), qy = bp.y0 + (t >> 3);
            const int c = (qx < cam.width && qy < cam.height) ? counts[cam.pixel_offset + (int64_t)qy * cam.width + qx]
                                                              : 0;
            const int incl = __ockl_wfscan_add_i32(c, true);
            s_off[t] = incl - c;
        }
        __syncthreads();
    }
    const int p = (int)(g % kGroups) * kPix + (int)threadIdx.x / TPP;   // pixel of the block
    const int q0 = (int)threadIdx.x % TPP;
    const int px = bp.x0 + (p & 7), py = bp.y0 + (p >> 3);
    if (px >= cam.width || py >= cam.height) return;
    const int64_t pix = cam.pixel_offset + (int64_t)py * cam.width + px;
    const int cnt = counts[pix];
    const uint2* __restrict__ mine = pairs + block * 64 * (int64_t)K + (compact ? s_off[p] : p * K);
    const uint32_t* __restrict__ rowlist = rows + block * 64 * (int64_t)K;
    const int nv = (C + VE - 1) / VE;
    float* __restrict__ dst = LABEL ? nullptr : out_feat + pix * C;
    float best = kNoValue;
    int best_c = kNoChannel;
    for (int q = q0; q < nv; q += TPP) {
        const int c0 = q * VE;
        float acc[VE];
#pragma unroll
        for (int i = 0; i < VE; ++i) acc[i] = 0.f;
        for (int j0 = 0; j0 < cnt; j0 += kGatherUnroll) {
            uint2 pr[kGatherUnroll];
#pragma unroll
            for (int u = 0; u < kGatherUnroll; ++u)
                if (j0 + u < cnt) pr[u] = mine[j0 + u];
            uint32_t sidx[kGatherUnroll];
#pragma unroll
            for (int u = 0; u < kGatherUnroll; ++u)
                if (j0 + u < cnt) sidx[u] = rowlist[pr[u].x];
            typename V::raw row[kGatherUnroll];
#pragma unroll
            for (int u = 0; u < kGatherUnroll; ++u)
                if (j0 + u < cnt) row[u] = V::load(feats + (int64_t)sidx[u] * C + c0);
#pragma unroll
            for (int u = 0; u < kGatherUnroll; ++u) {
                if (j0 + u < cnt) {
                    const float w = __uint_as_float(pr[u].y);
#pragma unroll
                    for (int i = 0; i < VE; ++i) acc[i] = fmaf(w, V::at(row[u], i), acc[i]);
                }
            }
        }
        if constexpr (LABEL) {
#pragma unroll
            for (int i = 0; i < VE; ++i) argmax_take(acc[i], c0 + i, best, best_c);
        } else {
            store_vec<VE>(dst, c0, acc);
        }
    }
    if constexpr (LABEL) {
        argmax_lanes<TPP>(best, best_c);
        if (q0 == 0) {
            out_label[pix] = best_c;
            if (out_score) out_score[pix] = best;
        }
    }
}

// Gather, staged form: one workgroup per 8x8 block.  The block's (slot,
// weight) lists and counts go to LDS, then its feature rows are staged in
// windows of W rows with direct global -> LDS loads (all of a window's loads
// in flight together), and every pixel adds the rows of its list that fall
// in the window, front to back.  TPP threads per pixel, each owning NVT
// 16-byte channel vectors (q, q + TPP, ...) of kPasses pixels of the block.
template <typename FT, int TPP, int W, int KC, bool LABEL, int NVT>
__global__ void __launch_bounds__(kGatherThreads)
topk_gather_lds_kernel(const uint2* __restrict__ pairs, const int32_t* __restrict__ counts,
                       const uint32_t* __restrict__ rows, const uint32_t* __restrict__ nrows,
                       const FT* __restrict__ feats, int C, int K, const fs_camera* __restrict__ cams, int num_views,
                       int S, int64_t nblocks, float* __restrict__ out_feat, int32_t* __restrict__ out_label,
                       float* __restrict__ out_score) {
    constexpr int VE = 16 / (int)sizeof(FT);
    using V = Vec<FT, VE>;
    constexpr int kPix = kGatherThreads / TPP;   // pixels per pass
    constexpr int kPasses = 64 / kPix;           // pixels per thread
    __shared__ __align__(16) uint4 s_rows[W * TPP * NVT];   // W rows of at most TPP NVT vectors
    __shared__ uint2 s_pairs[64 * KC];   // the block's compact lists (K <= KC)
    __shared__ int s_cnt[64];
    __shared__ int s_off[64];                  // first pair of each pixel's list
    __shared__ uint32_t s_rowid[64 * KC];         // the block's row list (R <= 64 K)
    const int tid = (int)threadIdx.x;
    const int64_t block = xcd_remap_chunked(blockIdx.x, nblocks, block_row_chunk(cams, S));
    const BlockPos bp = locate_block(block, S, 8, cams, num_views);
    if (!bp.valid) return;   // uniform over the workgroup
    const fs_camera& cam = cams[bp.view];
    const int nv = C / VE;                       // vectors per row (C % VE == 0)
    const int q = tid % TPP, sub = tid / TPP;
    bool has_vec[NVT];
#pragma unroll
    for (int v = 0; v < NVT; ++v) has_vec[v] = q + v * TPP < nv;
    const uint32_t nr = nrows[block];
    const uint32_t R = nr & 0xffffu, NP = nr >> 16;   // rows and listed pairs of the block
    const uint32_t* __restrict__ rowlist = rows + block * 64 * (int64_t)K;
    // lists, counts and the row list: one round trip (a block
    // no pixel of which blends anything has R = 0 and only writes zeros)
    if (R > 0)
        for (int t = tid; t < (int)NP; t += kGatherThreads) s_pairs[t] = pairs[block * 64 * (int64_t)K + t];
    if (tid < 64 && R > 0) {
        const int px = bp.x0 + (tid & 7), py = bp.y0 + (tid >> 3);
        s_cnt[tid] = (px < cam.width && py < cam.height) ? counts[cam.pixel_offset + (int64_t)py * cam.width + px] : 0;
    }
    for (int t = tid; t < (int)R; t += kGatherThreads) s_rowid[t] = rowlist[t];
    float acc[kPasses][NVT * VE];
    int cur[kPasses];
#pragma unroll
    for (int k = 0; k < kPasses; ++k) {
        cur[k] = 0;
#pragma unroll
        for (int i = 0; i < NVT * VE; ++i) acc[k][i] = 0.f;
    }
    __syncthreads();
    if (tid < 64) {
        const int c = s_cnt[tid];
        const int incl = __ockl_wfscan_add_i32(c, true);
        s_off[tid] = incl - c;   // visible after the staging barrier below
    }
    for (uint32_t s0 = 0; s0 < R; s0 += W) {
        const int nw = (int)(R - s0 < (uint32_t)W ? R - s0 : (uint32_t)W);
        // stage rows [s0, s0 + nw): vector v of the window is row v / nv,
        // column v % nv; lane l of an instruction lands at base + 16 l
        const int nvec = nw * nv;
        for (int i0 = (tid >> 6) * 64; i0 < nvec; i0 += kGatherThreads) {
            const int v = i0 + (tid & 63);
            if (v < nvec) {
                const int r = v / nv, c = v - r * nv;
                const FT* src = feats + (int64_t)s_rowid[s0 + r] * C + c * VE;
                __builtin_amdgcn_global_load_lds((const void*)src,
                                                 (__attribute__((address_space(3))) void*)&s_rows[i0], 16, 0, 0);
            }
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        // accumulate: pairs of each pixel are in slot order
#pragma unroll
        for (int k = 0; k < kPasses; ++k) {
            const int p = k * kPix + sub;
            const int c = s_cnt[p];
            int j = cur[k];
            while (j < c) {
                const uint2 pr = s_pairs[s_off[p] + j];
                if (pr.x >= s0 + (uint32_t)nw) break;
                const float w = __uint_as_float(pr.y);
#pragma unroll
                for (int v = 0; v < NVT; ++v) {
                    if (has_vec[v]) {
                        const typename V::raw f = *reinterpret_cast<const typename V::raw*>(
                            reinterpret_cast<const unsigned char*>(s_rows) + ((pr.x - s0) * nv + q + v * TPP) * 16);
#pragma unroll
                        for (int i = 0; i < VE; ++i) acc[k][v * VE + i] = fmaf(w, V::at(f, i), acc[k][v * VE + i]);
                    }
                }
                ++j;
            }
            cur[k] = j;
        }
        if (s0 + W < R) __syncthreads();   // the window is consumed
    }
#pragma unroll
    for (int k = 0; k < kPasses; ++k) {
        const int p = k * kPix + sub;
        const int px = bp.x0 + (p & 7), py = bp.y0 + (p >> 3);
        const bool on = px < cam.width && py < cam.height;
        if constexpr (LABEL) {
            // within vector v, lane q holds channels (q + v TPP) VE .. + VE - 1,
            // so lane order is channel order: the best of vector v is the own
            // best of the lowest lane whose best equals the maximum; the
            // vectors then combine in channel order
            float m = kNoValue;
            int label = kNoChannel;
#pragma unroll
            for (int v = 0; v < NVT; ++v) {
                float best = kNoValue;
                int best_c = kNoChannel;
                if (has_vec[v])
#pragma unroll
                    for (int i = 0; i < VE; ++i) argmax_take(acc[k][v * VE + i], (q + v * TPP) * VE + i, best, best_c);
                const float mv = lanes_max<TPP>(best);   // every lane of the workgroup is here
                const int base = (tid & 63) & ~(TPP - 1);
                const uint64_t seg = TPP == 64 ? ~0ull : ((1ull << TPP) - 1);
                const uint64_t hit = (__ballot(best == mv) >> base) & seg;   // mv is some lane's best (finite sums)
                const int lv = group_lane<TPP>(best_c, hit ? __builtin_ctzll(hit) : 0);
                argmax_take(mv, lv, m, label);
            }
            if (on && q == 0) {
                const int64_t pix = cam.pixel_offset + (int64_t)py * cam.width + px;
                out_label[pix] = label;
                if (out_score) out_score[pix] = m;
            }
        } else {
            float* dst = out_feat + (cam.pixel_offset + (int64_t)py * cam.width + px) * C;
#pragma unroll
            for (int v = 0; v < NVT; ++v)
                if (on && has_vec[v]) store_vec<VE>(dst, (q + v * TPP) * VE, &acc[k][v * VE]);
        }
    }
}

template <typename FT, int VE, bool LABEL>
hipError_t launch_gather(const uint2* pairs, const int32_t* counts, const uint32_t* rows, const uint32_t* nrows,
                         const void* feats, int C, int K, const fs_camera* cams, int num_views, int S,
                         int64_t nblocks, float* out_feat, int32_t* out_label, float* out_score, hipStream_t s) {
    const int nv = (C + VE - 1) / VE;
    const FT* f = static_cast<const FT*>(feats);
    int tpp = 4;
    while (tpp < nv && tpp < 64) tpp <<= 1;
    if (VE > 1 && nv <= 64 && K <= kStagedK) {
        if (nblocks >= (int64_t(1) << 32)) return hipErrorInvalidValue;
        // Threads per pixel: 8 when the feature image is written (one store
        // instruction then fills whole 128-B lines), 4 for labels; each
        // thread owns NVT vectors, q, q + TPP, ..., and 64 TPP / 256 pixels,
        // whose list walks it runs one after the other.  Measured on the
        // 1280x720 C = 128 float32 frame (render, features / labels): 32
        // threads x 1 vector 0.204 / 0.186 ms, 16 x 2 0.192 / 0.171, 8 x 4
        // 0.188 / 0.162, 4 x 8 0.225 / 0.157.  Row windows of about 16 KB
        // (32 rows of 512 B measured best for C = 128 float32 against 16,
        // 24 and 40).
#define FS_GATHER_LDS(TPP, W, NVT)                                                                                \
    if (K <= 8)                                                                                                    \
        hipLaunchKernelGGL((topk_gather_lds_kernel<FT, TPP, W, 8, LABEL, NVT>), dim3((unsigned)nblocks),          \
                           dim3(kGatherThreads), 0, s, pairs, counts, rows, nrows, f, C, K, cams, num_views, S,   \
                           nblocks, out_feat, out_label, out_score);                                               \
    else                                                                                                           \
        hipLaunchKernelGGL((topk_gather_lds_kernel<FT, TPP, W, kStagedK, LABEL, NVT>), dim3((unsigned)nblocks),    \
                           dim3(kGatherThreads), 0, s, pairs, counts, rows, nrows, f, C, K, cams, num_views, S,   \
                           nblocks, out_feat, out_label, out_score)
        constexpr int T = LABEL ? 4 : 8;
        if (nv <= 4) {
            FS_GATHER_LDS(4, 64, 1);
        } else if (nv <= T) {
            FS_GATHER_LDS(T, 64, 8 / T);
        } else if (nv <= 16) {
            FS_GATHER_LDS(T, 64, 16 / T);
        } else if (nv <= 32) {
            FS_GATHER_LDS(T, 32, 32 / T);
        } else {
            FS_GATHER_LDS(T, 24, 64 / T);
        }
#undef FS_GATHER_LDS
        return hipGetLastError();
    }
    const int64_t groups = nblocks * 64 * tpp / kGatherThreads;
    if (groups >= (int64_t(1) << 32)) return hipErrorInvalidValue;
#define FS_GATHER(TPP)                                                                                            \
    hipLaunchKernelGGL((topk_gather_general_kernel<FT, VE, TPP, LABEL>), dim3((unsigned)groups),                   \
                       dim3(kGatherThreads), 0, s, pairs, counts, rows, f, C, K, cams, num_views, S, groups, out_feat, \
                       out_label, out_score)
    switch (tpp) {
        case 4: FS_GATHER(4); break;
        case 8: FS_GATHER(8); break;
        case 16: FS_GATHER(16); break;
        case 32: FS_GATHER(32); break;
        default: FS_GATHER(64); break;
    }
#undef FS_GATHER
    return hipGetLastError();
}

}  // namespace

hipError_t fs_launch_topk_select(const FsRecord* records, const uint64_t* keys, const uint32_t* vals,
                                 const uint32_t* ranges, int64_t n, const fs_camera* cams, int num_views,
                                 int64_t total_tiles, const fs_opts& o, float* out_T, int32_t* out_n,
                                 int32_t* out_last, int32_t* out_idx, float* out_depth, float* out_normal,
                                 uint64_t* counters, const FsWorkspace& ws, hipStream_t s) {
    const int sb = o.tile / 8;
    const int64_t nblocks = total_tiles * sb * sb;
    if (ws.topk_pairs == nullptr || ws.topk_rows == nullptr || ws.topk_nrows == nullptr ||
        ws.topk_pair_slots < nblocks * 64 * (int64_t)o.topk || nblocks >= (int64_t(1) << 31))
        return hipErrorInvalidValue;
    const bool ext = o.lowpass != 0 || out_depth != nullptr || out_normal != nullptr;
    if (ext && o.topk_mode == FS_TOPK_WEIGHT) return hipErrorInvalidValue;
#define FS_SEL_KERN(WPG)                                                                                       \
    (o.topk_mode == FS_TOPK_WEIGHT                                                                              \
         ? (o.topk <= 8 ? topk_select_kernel<8, true, false, WPG> : topk_select_kernel<kCompactK, true, false, WPG>) \
     : ext ? (o.topk <= 8 ? topk_select_kernel<8, false, true, WPG>                                             \
                          : (o.topk <= kCompactK ? topk_select_kernel<kCompactK, false, true, WPG>               \
                                                 : topk_select_kernel<0, false, true, WPG>))                    \
           : (o.topk <= 8 ? topk_select_kernel<8, false, false, WPG>                                            \
                          : (o.topk <= kCompactK ? topk_select_kernel<kCompactK, false, false, WPG>              \
                                                 : topk_select_kernel<0, false, false, WPG>)))
    // long-list blocks first: their list, then nblocks waves for them and
    // nblocks for the grid order
    if (ws.sel_long == nullptr || ws.sel_counts == nullptr || nblocks > ws.render_max_blocks ||
        2 * nblocks >= (int64_t(1) << 31))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(select_long_kernel, dim3((unsigned)((nblocks + kSelGroup - 1) / kSelGroup)), dim3(kSelGroup), 0,
                       s, ranges, sb * sb, nblocks, ws.sel_long, ws.sel_counts);
#define FS_SEL_LAUNCH(WPG)                                                                                      \
    hipLaunchKernelGGL(FS_SEL_KERN(WPG), dim3((unsigned)(2 * ((nblocks + WPG - 1) / WPG))), dim3(64 * WPG), 0, s,  \
                       records, keys, vals, ranges, (uint32_t)n, n * num_views, cams, num_views, o.tile, o, nblocks,  \
                       ws.topk_pairs, ws.topk_rows, ws.topk_nrows, out_T, out_n, out_last, out_idx, out_depth,        \
                       out_normal, counters, ws.sel_long, ws.sel_counts)
    // two selection waves per workgroup (one block each): measured on the
    // 1280x720 C = 128 frame, Top-K render 0.1887 / 0.1862 / 0.1951 ms for
    // one, two and four waves per workgroup
    FS_SEL_LAUNCH(2);
#undef FS_SEL_LAUNCH
#undef FS_SEL_KERN
    return hipGetLastError();
}

hipError_t fs_launch_render_topk_split(const FsRecord* records, const uint64_t* keys, const uint32_t* vals,
                                       const uint32_t* ranges, const void* feats, int C, int64_t n,
                                       const fs_camera* cams, int num_views, int64_t total_tiles, const fs_opts& o,
                                       float* out_feat, int32_t* out_label, float* out_score, float* out_T,
                                       int32_t* out_n, int32_t* out_last, int32_t* out_idx, float* out_depth,
                                       float* out_normal, uint64_t* counters, const FsWorkspace& ws,
                                       hipStream_t s) {
    if (total_tiles == 0) return hipSuccess;
    const int sb = o.tile / 8;
    const int64_t nblocks = total_tiles * sb * sb;
    if (ws.topk_pairs == nullptr || ws.topk_rows == nullptr || ws.topk_nrows == nullptr ||
        ws.topk_pair_slots < nblocks * 64 * (int64_t)o.topk || nblocks >= (int64_t(1) << 31) ||
        (out_feat == nullptr) == (out_label == nullptr))
        return hipErrorInvalidValue;
    hipError_t e = fs_launch_topk_select(records, keys, vals, ranges, n, cams, num_views, total_tiles, o, out_T,
                                         out_n, out_last, out_idx, out_depth, out_normal, counters, ws, s);
    if (e != hipSuccess) return e;
    const bool bf16 = o.feat_dtype == FS_FEAT_BF16;
    const bool vec = C % (bf16 ? 8 : 4) == 0;
#define FS_GATHER_FORM(FT, VE, LABEL)                                                                             \
    launch_gather<FT, VE, LABEL>(ws.topk_pairs, out_n, ws.topk_rows, ws.topk_nrows, feats, C, o.topk, cams,      \
                                 num_views, o.tile, nblocks, out_feat, out_label, out_score, s)
    if (out_label) {
        if (bf16) return vec ? FS_GATHER_FORM(uint16_t, 8, true) : FS_GATHER_FORM(uint16_t, 1, true);
        return vec ? FS_GATHER_FORM(float, 4, true) : FS_GATHER_FORM(float, 1, true);
    }
    if (bf16) return vec ? FS_GATHER_FORM(uint16_t, 8, false) : FS_GATHER_FORM(uint16_t, 1, false);
    return vec ? FS_GATHER_FORM(float, 4, false) : FS_GATHER_FORM(float, 1, false);
#undef FS_GATHER_FORM
}
