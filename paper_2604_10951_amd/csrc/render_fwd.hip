// render_fwd.hip -- per-pixel front-to-back blending of C-channel features,
// full (Sec. 3.1 Eq. 2) or with Top-K hard selection (Sec. 3.4).
//
// Work decomposition.  A workgroup renders one render block (8x8 pixels per
// wave; 1 wave = 8x8 block, 4 waves = 16x16 block) of a binning tile and one
// chunk of at most 64*CPL channels.  The tile's depth-sorted list is walked in
// batches of BG entries:
//   1. stage: the BG records (FS_RECORD_BYTES = 96 B each) are copied to LDS;
//   2. weights (lanes = pixels): every lane walks the batch in depth order for
//      its pixel -- ray-splat (u, v), alpha, transmittance, the stop and Top-K
//      tests -- and writes its blend weight w = alpha T per accepted entry to
//      LDS plus a bit mask of accepted entries.  A wave skips entries whose
//      footprint box misses its 8x8 pixels;
//   3. fetch: the feature rows of entries accepted by any pixel of the block
//      are loaded once, coalesced, into LDS (float32 or bfloat16 storage);
//   4. accumulate (lanes = channels): for each of its 64 pixels (a static,
//      unrolled loop, so the accumulators stay in VGPRs) a wave walks the
//      accepted entries and adds w * c to CPL channels per lane: one FMA per
//      channel per (pixel, contributor) with no idle lanes, and every LDS read
//      is either a broadcast (w) or conflict-free (the row).
// The block exits as soon as every pixel has stopped (T_stop, or K blended
// surfels), which is where Top-K saves work.  Feature images are written
// pixel-major (channels contiguous), 64*CPL*4 bytes per pixel per chunk.
#include <type_traits>

#include "fs_internal.h"

namespace {

FS_DEV float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <typename FT>
FS_DEV float feat_to_f32(FT x);
template <>
FS_DEV float feat_to_f32<float>(float x) { return x; }
template <>
FS_DEV float feat_to_f32<uint16_t>(uint16_t x) { return bf16_to_f32(x); }

FS_DEV uint32_t wave_or(uint32_t x) { return __ockl_wfred_or_u32(x); }

// Bytes of a vector load of feature elements (16 B when C allows it).
template <typename FT, bool VEC>
struct RowVec {
    static constexpr int kElems = VEC ? 16 / (int)sizeof(FT) : 1;
};

template <int CPL, typename FT, int WAVES, int BG, bool EXT>
struct FwdShared {
    FsRecord rec[BG];
    uint32_t recid[BG];
    __align__(16) FT feat[BG][64 * CPL];
    float w[WAVES][BG][64];
    uint32_t used;
    int active;
    int list[BG];
    uint32_t item;
    double2 mu[EXT ? BG : 1];    // low-pass: projected centre relative to the anchor
    float4 geo[EXT ? BG : 1];    // depth and normal outputs: camera-facing normal, centre depth
};

// Per-entry data of the extended render (low-pass option, depth and normal
// outputs), staged once per batch by the entry's own thread.
FS_DEV void stage_ext(const FsRecord& r, const fs_camera& cam, const uint64_t* __restrict__ keys, uint32_t pos,
                      bool lowpass, bool geo, double2& mu, float4& g) {
    if (lowpass) {
        double mx, my;
        fs_record_centre(r, mx, my);
        mu = make_double2(mx, my);
    }
    if (geo) {
        const float3 nrm = fs_record_normal(r, cam);
        // the centre depth is needed (and keys given) only for the depth output
        g = make_float4(nrm.x, nrm.y, nrm.z, keys ? __uint_as_float((uint32_t)keys[pos]) : 0.f);
    }
}

// One render block: the walk over its tile's list (see the file comment).
// EXT: the low-pass response (o.lowpass) and the depth and normal outputs
// (out_depth / out_normal, chunk 0 only) are available.
template <int CPL, typename FT, int WAVES, int BG, bool VEC, bool EXT>
FS_DEV void render_block(int64_t block, FwdShared<CPL, FT, WAVES, BG, EXT>& sm, const FsRecord* __restrict__ records,
                         const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                         const uint32_t* __restrict__ ranges, const FT* __restrict__ feats, int C, int64_t n,
                         int64_t num_records, const fs_camera* __restrict__ cams, int num_views, int S,
                         const fs_opts& o, float* __restrict__ out_feat, float* __restrict__ out_T,
                         int32_t* __restrict__ out_n, int32_t* __restrict__ out_last, int32_t* __restrict__ out_idx,
                         float* __restrict__ out_depth, float* __restrict__ out_normal,
                         uint64_t* __restrict__ counters) {
    constexpr int NT = WAVES * 64;
    constexpr int kChunk = 64 * CPL;
    constexpr int RB = WAVES == 1 ? 8 : 16;
    constexpr int kQ = FS_RECORD_BYTES / 16;                 // float4 per record
    constexpr int kRecSlots = (BG * kQ + NT - 1) / NT;       // record float4 per thread
    constexpr int kVE = RowVec<FT, VEC>::kElems;             // feature elements per vector load
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const BlockPos bp = locate_block(block, S, RB, cams, num_views);
    if (!bp.valid) return;   // uniform across the workgroup
    const fs_camera& cam = cams[bp.view];
    const int chunk = blockIdx.y;
    const int c0 = chunk * kChunk;
    const int clen = C - c0 < kChunk ? C - c0 : kChunk;
    const int wx0 = bp.x0 + (WAVES == 1 ? 0 : (wave & 1) * 8);
    const int wy0 = bp.y0 + (WAVES == 1 ? 0 : (wave >> 1) * 8);
    const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
    const bool inside = px < cam.width && py < cam.height;
    const int64_t pix = cam.pixel_offset + (int64_t)py * cam.width + px;
    const uint32_t start = ranges[2 * bp.tile], end = ranges[2 * bp.tile + 1];
    const int K = o.topk;
    const bool write_idx = out_idx != nullptr && chunk == 0 && K > 0;
    const bool lowpass = EXT && o.lowpass != 0;
    const bool geo = EXT && chunk == 0 && (out_depth != nullptr || out_normal != nullptr);
    float gD = 0.f, gN0 = 0.f, gN1 = 0.f, gN2 = 0.f;   // depth and normal sums

    double T = 1.0;
    int cnt = 0;
    int last = -1;
    bool done = !inside;
    float acc[64][CPL];
#pragma unroll
    for (int p = 0; p < 64; ++p)
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[p][c] = 0.f;

    const double t_stop = o.t_stop;
    const float neg_half_log2e = -0.72134752044448170f;   // -log2(e) / 2
    uint32_t walked = 0, fetched = 0;

    // Prefetch pipeline: the list values of batch b + 2 and the records of
    // batch b + 1 are in flight while batch b is processed, so the dependent
    // load (record address from list value) never stalls the walk.
    float4 pre[kRecSlots];
    uint32_t pre_rid[kRecSlots];
    uint32_t nxt_rid[kRecSlots];
    auto fetch_vals = [&](uint32_t b0, uint32_t* rid) {
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int e = (tid + j * NT) / kQ;
            rid[j] = (e < BG && b0 + (uint32_t)e < end) ? vals[b0 + e] : 0xffffffffu;
        }
    };
    auto fetch_records = [&](const uint32_t* rid) {
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int q = (tid + j * NT) % kQ;
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
        // 1. stage the prefetched records
        if (tid == 0) {
            sm.used = 0u;
            sm.active = 0;
        }
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int t = tid + j * NT;
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
                if (q == 0) sm.recid[e] = rid;
            }
        }
        __syncthreads();
        if (b0 + BG < end) {
            fetch_records(nxt_rid);
            fetch_vals(b0 + 2 * BG, nxt_rid);
        }
        if constexpr (EXT) {
            if ((lowpass || geo) && tid < nb)
                stage_ext(sm.rec[tid], cam, keys, b0 + (uint32_t)tid, lowpass, geo, sm.mu[tid], sm.geo[tid]);
            __syncthreads();
        }
        // 2. weights, lanes = pixels
        uint32_t mask = 0u;
        if (!__all(done)) {
            for (int e = 0; e < nb; ++e) {
                const FsRecord& r = sm.rec[e];
                if (r.x1 < wx0 || r.x0 > wx0 + 7 || r.y1 < wy0 || r.y0 > wy0 + 7) continue;
                if (!done) {
                    FsResp rs = fs_response(r, (double)(px - r.ax), (double)(py - r.ay));
                    if constexpr (EXT)
                        if (lowpass) fs_lowpass_d2(rs, (double)(px - r.ax), (double)(py - r.ay), sm.mu[e].x, sm.mu[e].y);
                    if (rs.d2 <= r.k2 && fs_in_box(r, px, py)) {
                        const float G = __builtin_amdgcn_exp2f(neg_half_log2e * (float)rs.d2);
                        const float alpha = fminf(o.alpha_max, r.o * G);
                        const double Tn = T * (1.0 - (double)alpha);
                        if (Tn < t_stop) {
                            done = true;
                        } else {
                            const float w = (float)((double)alpha * T);
                            sm.w[wave][e][lane] = w;
                            if constexpr (EXT) {
                                if (geo) {
                                    const float4 gg = sm.geo[e];
                                    gD = fmaf(w, (float)((double)gg.w * rs.rh), gD);
                                    gN0 = fmaf(w, gg.x, gN0);
                                    gN1 = fmaf(w, gg.y, gN1);
                                    gN2 = fmaf(w, gg.z, gN2);
                                }
                            }
                            mask |= 1u << e;
                            T = Tn;
                            if (write_idx) out_idx[pix * K + cnt] = (int32_t)sm.recid[e];
                            ++cnt;
                            last = (int)(b0 + e);
                            if (K > 0 && cnt == K) done = true;
                        }
                    }
                }
                if ((e & 7) == 7 && __all(done)) break;
            }
        }
        const uint32_t wused = wave_or(mask);
        const uint64_t active_px = __ballot(mask != 0u);
        const bool wactive = !__all(done);
        if (lane == 0) {
            if (wused) atomicOr(&sm.used, wused);
            if (wactive) atomicAdd(&sm.active, 1);
        }
        __syncthreads();
        const uint32_t used = sm.used;
        const int active = sm.active;   // latched: wave 0 re-zeroes both at the next batch
        const int nu = __popc(used);
        if (tid < BG && ((used >> tid) & 1u)) sm.list[__popc(used & ((1u << tid) - 1u))] = tid;
        walked += (uint32_t)nb;
        fetched += (uint32_t)nu;
        __syncthreads();
        // 3. fetch the feature rows of accepted entries: every load is issued
        //    before the first LDS store
        if (VEC) {
            // direct global -> LDS loads, 16 B per lane, rows packed in the
            // order of the compacted list (row j of the batch at sm.feat[j])
            constexpr int kRowBytes = kChunk * (int)sizeof(FT);
            constexpr int kLanesPerRow = kRowBytes / 16;
            constexpr int kRowsPerInst = 64 / kLanesPerRow;
            const int ninst = (nu + kRowsPerInst - 1) / kRowsPerInst;
            const int lrow = lane / kLanesPerRow, lcol = lane - lrow * kLanesPerRow;
            for (int i = wave; i < ninst; i += WAVES) {
                const int row = i * kRowsPerInst + lrow;
                if (row < nu && lcol * kVE < clen) {
                    const int64_t sidx = fs_surfel_of(sm.recid[sm.list[row]], n);
                    const FT* src = feats + sidx * C + c0 + lcol * kVE;
                    __builtin_amdgcn_global_load_lds(
                        (const void*)src, (__attribute__((address_space(3))) void*)&sm.feat[i * kRowsPerInst][0], 16,
                        0, 0);
                }
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        } else {
            for (int t = tid; t < nu * kChunk; t += NT) {
                const int j = t / kChunk, c = t - j * kChunk;
                if (c < clen) {
                    const int e = sm.list[j];
                    const int64_t sidx = fs_surfel_of(sm.recid[e], n);
                    sm.feat[j][c] = feats[sidx * C + c0 + c];
                }
            }
        }
        __syncthreads();
        // 4. accumulate, lanes = channels
#pragma unroll
        for (int p = 0; p < 64; ++p) {
            if ((active_px >> p) & 1ull) {
                uint32_t m = __builtin_amdgcn_readlane(mask, p);
                while (m) {
                    const int e = __builtin_ctz(m);
                    m &= m - 1u;
                    const int j = __popc(used & ((1u << e) - 1u));   // row slot of entry e
                    const float w = sm.w[wave][e][p];
                    if (CPL == 2 && sizeof(FT) == 4) {
                        const float2 f = *reinterpret_cast<const float2*>(&sm.feat[j][lane * 2]);
                        acc[p][0] = fmaf(w, f.x, acc[p][0]);
                        acc[p][CPL - 1] = fmaf(w, f.y, acc[p][CPL - 1]);
                    } else {
#pragma unroll
                        for (int c = 0; c < CPL; ++c)
                            acc[p][c] = fmaf(w, feat_to_f32(sm.feat[j][lane * CPL + c]), acc[p][c]);
                    }
                }
            }
        }
        if (active == 0) break;
    }

    if (counters != nullptr && chunk == 0) {
        int c = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) c += __shfl_xor(c, d, 64);
        if (lane == 0) atomicAdd((unsigned long long*)&counters[2], (unsigned long long)c);
        if (tid == 0) {
            atomicAdd((unsigned long long*)&counters[0], (unsigned long long)walked);
            atomicAdd((unsigned long long*)&counters[1], (unsigned long long)fetched);
            atomicAdd((unsigned long long*)&counters[3], 1ull);
        }
    }
    if (chunk == 0 && inside) {
        out_T[pix] = (float)T;
        out_n[pix] = cnt;
        if (out_last) out_last[pix] = last;
        if (write_idx)
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
    const int cl = lane * CPL;
#pragma unroll
    for (int p = 0; p < 64; ++p) {
        const int qx = wx0 + (p & 7), qy = wy0 + (p >> 3);
        if (qx < cam.width && qy < cam.height) {
            float* dst = out_feat + (cam.pixel_offset + (int64_t)qy * cam.width + qx) * C + c0 + cl;
            if (CPL == 2 && cl + 1 < clen && ((C & 1) == 0)) {
                *reinterpret_cast<float2*>(dst) = make_float2(acc[p][0], acc[p][CPL - 1]);
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (cl + c < clen) dst[c] = acc[p][c];
            }
        }
    }
}

// Grid launch (order == nullptr): workgroup b renders block b.  Persistent
// launch: workgroups take positions of `order` (blocks sorted by list
// length, longest first) from atomic tickets until the queues are empty.
template <int CPL, typename FT, int WAVES, int BG, bool VEC, bool EXT>
__global__ void __launch_bounds__(WAVES * 64)
render_fwd_kernel(const FsRecord* __restrict__ records, const uint64_t* __restrict__ keys,
                  const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges, const FT* __restrict__ feats,
                  int C, int64_t n, int64_t num_records, const fs_camera* __restrict__ cams, int num_views, int S,
                  fs_opts o, float* __restrict__ out_feat, float* __restrict__ out_T, int32_t* __restrict__ out_n,
                  int32_t* __restrict__ out_last, int32_t* __restrict__ out_idx, float* __restrict__ out_depth,
                  float* __restrict__ out_normal, uint64_t* __restrict__ counters,
                  const uint32_t* __restrict__ order, uint32_t* __restrict__ ticket, uint32_t nblocks) {
    __shared__ FwdShared<CPL, FT, WAVES, BG, EXT> sm;
    if (order == nullptr) {
        // the XCDs take one tile row of blocks each in turn: neighbouring
        // blocks share an L2 and dense regions are spread over all XCDs
        // (full blend of the 1280x720 frame: 1.77 -> 1.41 ms)
        constexpr int RBv = WAVES == 1 ? 8 : 16;
        const int64_t tiles_x = ((int64_t)cams[0].width + S - 1) / S, sb = S / RBv;
        const int64_t blk = xcd_remap_chunked(blockIdx.x, gridDim.x, tiles_x * sb * sb);
        render_block<CPL, FT, WAVES, BG, VEC, EXT>(blk, sm, records, keys, vals, ranges, feats, C, n, num_records,
                                                   cams, num_views, S, o, out_feat, out_T, out_n, out_last, out_idx,
                                                   out_depth, out_normal, counters);
        return;
    }
    const uint32_t nq = gridDim.x < kRenderQueues ? gridDim.x : kRenderQueues;   // as in render_wide_kernel
    const uint32_t q = blockIdx.x % nq;
    for (;;) {
        __syncthreads();   // every wave is done with the previous item (and sm.item)
        if (threadIdx.x == 0) sm.item = atomicAdd(ticket + q * kTicketStride, 1u);
        __syncthreads();
        const uint32_t it = sm.item * nq + q;
        if (it >= nblocks) break;
        render_block<CPL, FT, WAVES, BG, VEC, EXT>(order[it], sm, records, keys, vals, ranges, feats, C, n,
                                                   num_records, cams, num_views, S, o, out_feat, out_T, out_n,
                                                   out_last, out_idx, out_depth, out_normal, counters);
    }
}

// ---------------------------------------------------------------------------
// Wide render block (8x8 binning tiles): one 8x8 pixel block per workgroup of
// NW waves, so a long list is walked NW times faster than by one wave.  Per
// batch of BG entries:
//   a. alpha: the (entry, pixel) pairs inside each entry's pixel box (on
//      average an eighth of the block) are packed over all threads of the
//      workgroup -- a prefix count of the boxes' pixels, then a bisection
//      per thread for its pair -- and each pair's alpha (or -1: not
//      accepted) goes to LDS; pixels outside an entry's box keep -1;
//   b. walk (lanes = pixels): every wave loads the batch's alphas of its
//      lane's pixel into registers and runs the same front-to-back
//      transmittance walk in depth order (stop and Top-K tests, FP64 T), so
//      each knows the accepted entries of every pixel without an exchange,
//      and stores the weights w = alpha T of its own 64 / NW pixels;
//   c. rows: the feature rows of entries accepted anywhere in the block go
//      to LDS by direct global -> LDS loads, issued right after the walk and
//      consumed one batch later (double buffer), so the load latency is
//      hidden behind the next batch's alpha pass;
//   d. accumulate (lanes = channels): each wave adds w * c for its own
//      pixels, one FMA per channel per (pixel, contributor).
// Every pixel sees the same sequence of FP64 transmittance updates and FP32
// FMAs as in render_block, so the two give identical results.
template <int CPL, typename FT, int NW, int BG, bool EXT>
struct WideShared {
    FsRecord rec[BG];
    uint32_t recid[2][BG];
    __align__(16) FT feat[2][BG][64 * CPL];
    float a[BG][64];              // alpha per accepted (entry, pixel)
    uint32_t amask[2][64];        // per pixel: the batch's accepted entries (double buffer)
    uint8_t rowlist[NW][32];      // per wave: entry of each compacted feature row
    float w[BG][64];              // weights; column p is written and read by pixel p's wave only
    float z[EXT ? BG : 1][64];    // depth output: camera depth of the ray-plane point
    double2 mu[EXT ? BG : 1];
    float4 geo[EXT ? BG : 1];
    uint32_t item;
};

template <int CPL, typename FT, int NW, int BG, bool VEC, bool EXT>
FS_DEV void render_block_wide(int64_t block, WideShared<CPL, FT, NW, BG, EXT>& sm,
                              const FsRecord* __restrict__ records, const uint64_t* __restrict__ keys,
                              const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges,
                              const FT* __restrict__ feats, int C, int64_t n, int64_t num_records,
                              const fs_camera* __restrict__ cams, int num_views, int S, const fs_opts& o,
                              float* __restrict__ out_feat, float* __restrict__ out_T, int32_t* __restrict__ out_n,
                              int32_t* __restrict__ out_last, int32_t* __restrict__ out_idx,
                              float* __restrict__ out_depth, float* __restrict__ out_normal,
                              uint64_t* __restrict__ counters) {
    static_assert(BG <= 32 && 64 % NW == 0, "batch masks are 32-bit; pixel groups split the 64 pixels evenly");
    constexpr int NT = NW * 64;
    constexpr int PPW = 64 / NW;                             // pixels accumulated per wave
    constexpr int kChunk = 64 * CPL;
    constexpr int kQ = FS_RECORD_BYTES / 16;
    constexpr int kRecSlots = (BG * kQ + NT - 1) / NT;
    constexpr int kVE = RowVec<FT, VEC>::kElems;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const BlockPos bp = locate_block(block, S, 8, cams, num_views);
    if (!bp.valid) return;   // uniform across the workgroup
    const fs_camera& cam = cams[bp.view];
    const int chunk = blockIdx.y;
    const int c0 = chunk * kChunk;
    const int clen = C - c0 < kChunk ? C - c0 : kChunk;
    const int px = bp.x0 + (lane & 7), py = bp.y0 + (lane >> 3);
    const bool inside = px < cam.width && py < cam.height;
    const int64_t pix = cam.pixel_offset + (int64_t)py * cam.width + px;
    const bool mine = lane / PPW == wave;                    // lane's pixel is accumulated by this wave
    const uint32_t start = ranges[2 * bp.tile], end = ranges[2 * bp.tile + 1];
    const int K = o.topk;
    const bool write_idx = out_idx != nullptr && chunk == 0 && K > 0 && wave == 0;
    const bool lowpass = EXT && o.lowpass != 0;
    const bool geo = EXT && chunk == 0 && (out_depth != nullptr || out_normal != nullptr);
    float gD = 0.f, gN0 = 0.f, gN1 = 0.f, gN2 = 0.f;

    double T = 1.0;
    int cnt = 0;
    int last = -1;
    bool done = !inside;
    float acc[PPW][CPL];
#pragma unroll
    for (int p = 0; p < PPW; ++p)
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[p][c] = 0.f;
    const double t_stop = o.t_stop;
    const float neg_half_log2e = -0.72134752044448170f;   // -log2(e) / 2
    uint32_t walked = 0, fetched = 0;

    // records of batch i + 1 and list values of batch i + 2 are in flight
    // while batch i is processed
    float4 pre[kRecSlots];
    uint32_t pre_rid[kRecSlots];
    uint32_t nxt_rid[kRecSlots];
    auto fetch_vals = [&](uint32_t b0, uint32_t* rid) {
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int e = (tid + j * NT) / kQ;
            rid[j] = (e < BG && b0 + (uint32_t)e < end) ? vals[b0 + e] : 0xffffffffu;
        }
    };
    auto fetch_records = [&](const uint32_t* rid) {
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int q = (tid + j * NT) % kQ;
            pre_rid[j] = rid[j];
            pre[j] = make_float4(0.f, 0.f, 0.f, 0.f);
            if ((int64_t)rid[j] < num_records) pre[j] = reinterpret_cast<const float4*>(records + rid[j])[q];
        }
    };

    // accumulate batch rows already in feat[buf] into the wave's own pixels,
    // two contributors of a pixel per step (both LDS reads in flight before
    // the FMAs), in entry order
    auto accumulate = [&](int buf, uint32_t used, uint32_t mask, uint64_t active_px) {
#pragma unroll
        for (int q = 0; q < PPW; ++q) {
            const int p = wave * PPW + q;
            if ((active_px >> p) & 1ull) {
                uint32_t m = __builtin_amdgcn_readlane(mask, p);
                while (m) {
                    const int e0 = __builtin_ctz(m);
                    m &= m - 1u;
                    const bool two = m != 0u;
                    const int e1 = two ? __builtin_ctz(m) : e0;
                    if (two) m &= m - 1u;
                    const int j0 = __popc(used & ((1u << e0) - 1u));   // row slots
                    const int j1 = __popc(used & ((1u << e1) - 1u));
                    const float w0 = sm.w[e0][p];
                    const float w1 = sm.w[e1][p];
                    if (CPL == 2 && sizeof(FT) == 4) {
                        const float2 f0 = *reinterpret_cast<const float2*>(&sm.feat[buf][j0][lane * 2]);
                        const float2 f1 = *reinterpret_cast<const float2*>(&sm.feat[buf][j1][lane * 2]);
                        acc[q][0] = fmaf(w0, f0.x, acc[q][0]);
                        acc[q][CPL - 1] = fmaf(w0, f0.y, acc[q][CPL - 1]);
                        if (two) {
                            acc[q][0] = fmaf(w1, f1.x, acc[q][0]);
                            acc[q][CPL - 1] = fmaf(w1, f1.y, acc[q][CPL - 1]);
                        }
                    } else {
                        float f0[CPL], f1[CPL];
#pragma unroll
                        for (int c = 0; c < CPL; ++c) {
                            f0[c] = feat_to_f32(sm.feat[buf][j0][lane * CPL + c]);
                            f1[c] = feat_to_f32(sm.feat[buf][j1][lane * CPL + c]);
                        }
#pragma unroll
                        for (int c = 0; c < CPL; ++c) acc[q][c] = fmaf(w0, f0[c], acc[q][c]);
                        if (two)
#pragma unroll
                            for (int c = 0; c < CPL; ++c) acc[q][c] = fmaf(w1, f1[c], acc[q][c]);
                    }
                }
            }
        }
    };

    uint32_t p_used = 0u, p_mask = 0u;   // previous batch: entries with rows in flight, lane's accepted entries
    uint64_t p_active = 0ull;
    int pbuf = -1;                       // feat buffer of the previous batch (-1: none)
    if (start < end) {
        uint32_t r0[kRecSlots];
        fetch_vals(start, r0);
        fetch_records(r0);
        fetch_vals(start + BG, nxt_rid);
    }
    int it = 0;
    for (uint32_t b0 = start; b0 < end; b0 += BG, ++it) {
        const int nb = (int)(end - b0 < (uint32_t)BG ? end - b0 : (uint32_t)BG);
        const int cur = it & 1;
        // stage the prefetched records (the previous batch's alpha pass, the
        // last reader of sm.rec, ended before the previous barrier B)
#pragma unroll
        for (int j = 0; j < kRecSlots; ++j) {
            const int t = tid + j * NT;
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
                if (q == 0) sm.recid[cur][e] = rid;
            }
        }
        // accepted-entry masks of this batch (their last reader, the walk two
        // batches back, ended before the previous barrier A)
        if (tid < 64) sm.amask[cur][tid] = 0u;
        __syncthreads();   // A: records staged; every wave has finished the previous walk
        if (b0 + BG < end) {
            fetch_records(nxt_rid);
            fetch_vals(b0 + 2 * BG, nxt_rid);
        }
        if constexpr (EXT) {
            if ((lowpass || geo) && tid < nb)
                stage_ext(sm.rec[tid], cam, keys, b0 + (uint32_t)tid, lowpass, geo, sm.mu[tid], sm.geo[tid]);
            __syncthreads();
        }
        // a. alpha over the pairs inside the entries' pixel boxes.  Lane e
        //    (< nb) of every wave takes entry e's box clipped to the block:
        //    origin, width, a reciprocal for the division by the width, and
        //    its pixel count; an inclusive scan of the counts numbers the
        //    pairs, and pair m belongs to the entry whose scan first exceeds m.
        {
            int cnt_e = 0, packed = 0;
            if (lane < nb) {
                const FsRecord& r = sm.rec[lane];
                const int xa = r.x0 > bp.x0 ? r.x0 : bp.x0;
                const int ya = r.y0 > bp.y0 ? r.y0 : bp.y0;
                int xb = r.x1 < bp.x0 + 7 ? r.x1 : bp.x0 + 7;
                int yb = r.y1 < bp.y0 + 7 ? r.y1 : bp.y0 + 7;
                xb = xb < cam.width - 1 ? xb : cam.width - 1;
                yb = yb < cam.height - 1 ? yb : cam.height - 1;
                if (xb >= xa && yb >= ya) {
                    const int rw = xb - xa + 1, rh = yb - ya + 1;
                    cnt_e = rw * rh;
                    const int inv = (65536 + rw - 1) / rw;   // exact division of counts < 64 by rw <= 8
                    packed = (xa - bp.x0) | ((ya - bp.y0) << 3) | (rw << 6) | (inv << 10);
                }
            }
            // inclusive prefix of the entries' pair counts (lanes 0-31 hold the
            // batch's entries; the bisection below reads only those)
            const int S = __ockl_wfscan_add_i32(cnt_e, true);
            const int M = __builtin_amdgcn_readlane(S, 31);
            for (int base = wave * 64; base < M; base += NT) {   // uniform per wave: every lane shuffles
                const int m = base + lane;
                int e = 0;
#pragma unroll
                for (int step = BG / 2; step >= 1; step >>= 1)
                    if (__shfl(S, e + step - 1, 64) <= m) e += step;
                const int prev = __shfl(S, e > 0 ? e - 1 : 0, 64);
                const int pk = __shfl(packed, e, 64);
                if (m < M) {
                    const int local = m - (e > 0 ? prev : 0);
                    const int rw = (pk >> 6) & 15, inv = pk >> 10;
                    const int dy = (local * inv) >> 16, dx = local - dy * rw;
                    const int lx = (pk & 7) + dx, ly = ((pk >> 3) & 7) + dy;
                    const int qx = bp.x0 + lx, qy = bp.y0 + ly;
                    const FsRecord& r = sm.rec[e];
                    FsResp rs = fs_response(r, (double)(qx - r.ax), (double)(qy - r.ay));
                    if constexpr (EXT)
                        if (lowpass) fs_lowpass_d2(rs, (double)(qx - r.ax), (double)(qy - r.ay), sm.mu[e].x, sm.mu[e].y);
                    if (rs.d2 <= r.k2) {
                        const float G = __builtin_amdgcn_exp2f(neg_half_log2e * (float)rs.d2);
                        sm.a[e][ly * 8 + lx] = fminf(o.alpha_max, r.o * G);
                        atomicOr(&sm.amask[cur][ly * 8 + lx], 1u << e);
                        if constexpr (EXT)
                            if (geo) sm.z[e][ly * 8 + lx] = (float)((double)sm.geo[e].w * rs.rh);
                    }
                }
            }
        }
        // the previous batch's rows (issued before this batch's alpha pass)
        if (VEC) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();   // B: alpha of this batch and rows of the previous batch are in LDS
        if (pbuf >= 0) accumulate(pbuf, p_used, p_mask, p_active);
        // b. the transmittance walk, identical in every wave: each lane
        //    visits only its pixel's accepted entries, in depth order, with
        //    the next entry's alpha read ahead
        uint32_t mask = 0u;
        {
            uint32_t macc = done ? 0u : sm.amask[cur][lane];
            int e = macc ? __builtin_ctz(macc) : 0;
            float al = sm.a[e][lane];
            while (macc != 0u && !done) {
                macc &= macc - 1u;
                const int en = macc ? __builtin_ctz(macc) : 0;
                const float aln = sm.a[en][lane];
                const double Tn = T * (1.0 - (double)al);
                if (Tn < t_stop) {
                    done = true;
                } else {
                    const float w = (float)((double)al * T);
                    if (mine) sm.w[e][lane] = w;
                    if constexpr (EXT) {
                        if (geo) {
                            const float4 gg = sm.geo[e];
                            gD = fmaf(w, sm.z[e][lane], gD);
                            gN0 = fmaf(w, gg.x, gN0);
                            gN1 = fmaf(w, gg.y, gN1);
                            gN2 = fmaf(w, gg.z, gN2);
                        }
                    }
                    mask |= 1u << e;
                    T = Tn;
                    if (write_idx) out_idx[pix * K + cnt] = (int32_t)sm.recid[cur][e];
                    ++cnt;
                    last = (int)(b0 + e);
                    if (K > 0 && cnt == K) done = true;
                }
                e = en;
                al = aln;
            }
        }
        const uint32_t used = wave_or(mask);
        const uint64_t active_px = __ballot(mask != 0u);
        const bool wactive = !__all(done);
        const int nu = __popc(used);
        walked += (uint32_t)nb;
        fetched += (uint32_t)nu;
        // c. issue this batch's rows into feat[cur] (last read by the
        //    accumulation two batches back, before barrier B)
        if (VEC) {
            constexpr int kRowBytes = kChunk * (int)sizeof(FT);
            constexpr int kLanesPerRow = kRowBytes / 16;
            constexpr int kRowsPerInst = 64 / kLanesPerRow;
            const int ninst = (nu + kRowsPerInst - 1) / kRowsPerInst;
            const int lrow = lane / kLanesPerRow, lcol = lane - lrow * kLanesPerRow;
            // the wave's own list of the compacted rows' entries (written and
            // read by this wave only; LDS operations of a wave are in order)
            if (lane < 32 && ((used >> lane) & 1u)) sm.rowlist[wave][__popc(used & ((1u << lane) - 1u))] = (uint8_t)lane;
            // the wave's instructions take rows i * kRowsPerInst + lrow
            for (int i = wave; i < ninst; i += NW) {
                const int row = i * kRowsPerInst + lrow;
                if (row < nu && lcol * kVE < clen) {
                    const int e = sm.rowlist[wave][row];
                    const int64_t sidx = fs_surfel_of(sm.recid[cur][e], n);
                    const FT* src = feats + sidx * C + c0 + lcol * kVE;
                    __builtin_amdgcn_global_load_lds(
                        (const void*)src,
                        (__attribute__((address_space(3))) void*)&sm.feat[cur][i * kRowsPerInst][0], 16, 0, 0);
                }
            }
        } else {
            for (int t = tid; t < nu * kChunk; t += NT) {
                const int j = t / kChunk, c = t - j * kChunk;
                if (c < clen) {
                    uint32_t mm = used;
                    for (int k = 0; k < j; ++k) mm &= mm - 1u;
                    const int e = __builtin_ctz(mm);
                    const int64_t sidx = fs_surfel_of(sm.recid[cur][e], n);
                    sm.feat[cur][j][c] = feats[sidx * C + c0 + c];
                }
            }
        }
        p_used = used;
        p_mask = mask;
        p_active = active_px;
        pbuf = cur;
        if (!wactive) break;   // identical in every wave
    }
    if (pbuf >= 0) {
        if (VEC) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        accumulate(pbuf, p_used, p_mask, p_active);
    }

    if (counters != nullptr && chunk == 0 && wave == 0) {
        int c = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) c += __shfl_xor(c, d, 64);
        if (lane == 0) {
            atomicAdd((unsigned long long*)&counters[2], (unsigned long long)c);
            atomicAdd((unsigned long long*)&counters[0], (unsigned long long)walked);
            atomicAdd((unsigned long long*)&counters[1], (unsigned long long)fetched);
            atomicAdd((unsigned long long*)&counters[3], 1ull);
        }
    }
    if (chunk == 0 && inside && wave == 0) {
        out_T[pix] = (float)T;
        out_n[pix] = cnt;
        if (out_last) out_last[pix] = last;
        if (write_idx)
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
    const int cl = lane * CPL;
#pragma unroll
    for (int q = 0; q < PPW; ++q) {
        const int p = wave * PPW + q;
        const int qx = bp.x0 + (p & 7), qy = bp.y0 + (p >> 3);
        if (qx < cam.width && qy < cam.height) {
            float* dst = out_feat + (cam.pixel_offset + (int64_t)qy * cam.width + qx) * C + c0 + cl;
            if (CPL == 2 && cl + 1 < clen && ((C & 1) == 0)) {
                // non-temporal: the image is not read back by this kernel
                typedef float f32x2 __attribute__((ext_vector_type(2)));
                __builtin_nontemporal_store(f32x2{acc[q][0], acc[q][CPL - 1]}, reinterpret_cast<f32x2*>(dst));
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (cl + c < clen) dst[c] = acc[q][c];
            }
        }
    }
}

template <int CPL, typename FT, int NW, int BG, bool VEC, bool EXT>
__global__ void __launch_bounds__(NW * 64)
render_wide_kernel(const FsRecord* __restrict__ records, const uint64_t* __restrict__ keys,
                   const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges, const FT* __restrict__ feats,
                   int C, int64_t n, int64_t num_records, const fs_camera* __restrict__ cams, int num_views, int S,
                   fs_opts o, float* __restrict__ out_feat, float* __restrict__ out_T, int32_t* __restrict__ out_n,
                   int32_t* __restrict__ out_last, int32_t* __restrict__ out_idx, float* __restrict__ out_depth,
                   float* __restrict__ out_normal, uint64_t* __restrict__ counters,
                   const uint32_t* __restrict__ order, uint32_t* __restrict__ ticket, uint32_t nblocks) {
    __shared__ WideShared<CPL, FT, NW, BG, EXT> sm;
    if (order == nullptr) {
        const int64_t tiles_x = ((int64_t)cams[0].width + S - 1) / S;
        const int64_t blk = xcd_remap_chunked(blockIdx.x, gridDim.x, tiles_x);
        render_block_wide<CPL, FT, NW, BG, VEC, EXT>(blk, sm, records, keys, vals, ranges, feats, C, n, num_records,
                                                     cams, num_views, S, o, out_feat, out_T, out_n, out_last,
                                                     out_idx, out_depth, out_normal, counters);
        return;
    }
    // nq queues: workgroup g takes items q, q + nq, q + 2 nq, .. (q = g mod
    // nq) from a ticket of its own, so the tickets (memory-side atomics,
    // each serialised per address) are shared by a grid's nq-th part only
    const uint32_t nq = gridDim.x < kRenderQueues ? gridDim.x : kRenderQueues;
    const uint32_t q = blockIdx.x % nq;
    for (;;) {
        __syncthreads();   // every wave is done with the previous item (and sm.item)
        if (threadIdx.x == 0) sm.item = atomicAdd(ticket + q * kTicketStride, 1u);
        __syncthreads();
        const uint32_t it = sm.item * nq + q;
        if (it >= nblocks) break;
        render_block_wide<CPL, FT, NW, BG, VEC, EXT>(order[it], sm, records, keys, vals, ranges, feats, C, n,
                                                     num_records, cams, num_views, S, o, out_feat, out_T, out_n,
                                                     out_last, out_idx, out_depth, out_normal, counters);
    }
}

// Work order for the persistent launch: blocks bucketed by 4 log2(1 + list
// length) (64 buckets), longest bucket first.
FS_DEV int cost_bucket(uint32_t len) {
    const float b = 4.f * __log2f(1.f + (float)len);
    const int k = (int)b;
    return 63 - (k > 63 ? 63 : k);
}

// Pass 1: per group of 256 blocks, its blocks per cost bucket (no atomics
// outside LDS, nothing to clear beforehand); group 0 also zeroes the work
// queues' tickets.
__global__ void __launch_bounds__(256)
order_count_kernel(const uint32_t* __restrict__ ranges, int sb2, uint32_t nblocks, uint32_t* __restrict__ gcnt,
                   uint32_t* __restrict__ ticket) {
    __shared__ uint32_t h[64];
    const uint32_t tid = threadIdx.x;
    if (tid < 64) h[tid] = 0u;
    __syncthreads();
    const uint32_t b = blockIdx.x * 256u + tid;
    if (b < nblocks) {
        const uint32_t t = b / sb2;
        atomicAdd(&h[cost_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u);
    }
    __syncthreads();
    if (tid < 64) gcnt[blockIdx.x * 64u + tid] = h[tid];
    if (blockIdx.x == 0 && tid < kRenderQueues) ticket[tid * kTicketStride] = 0u;
}

// Pass 2: every group finds where its blocks of each bucket start -- the
// blocks of all groups in earlier buckets, then those of earlier groups in
// the same bucket -- and places them (ranks within the group by LDS
// cursors, so the order inside a bucket is not fixed).
__global__ void __launch_bounds__(256)
order_place_kernel(const uint32_t* __restrict__ ranges, int sb2, uint32_t nblocks, const uint32_t* __restrict__ gcnt,
                   uint32_t ngroups, uint32_t* __restrict__ order) {
    __shared__ uint32_t s_tot[4][64], s_bef[4][64], base[64];
    const uint32_t tid = threadIdx.x, k = tid & 63u, qtr = tid >> 6;
    uint32_t tot = 0u, bef = 0u;
    for (uint32_t w = qtr; w < ngroups; w += 4u) {
        const uint32_t c = gcnt[w * 64u + k];
        tot += c;
        bef += w < blockIdx.x ? c : 0u;
    }
    s_tot[qtr][k] = tot;
    s_bef[qtr][k] = bef;
    __syncthreads();
    if (tid < 64) {
        const uint32_t T = s_tot[0][k] + s_tot[1][k] + s_tot[2][k] + s_tot[3][k];
        const uint32_t B = s_bef[0][k] + s_bef[1][k] + s_bef[2][k] + s_bef[3][k];
        uint32_t incl = T;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, 64);
            if ((int)tid >= d) incl += y;
        }
        base[k] = incl - T + B;
    }
    __syncthreads();
    const uint32_t b = blockIdx.x * 256u + tid;
    if (b < nblocks) {
        const uint32_t t = b / sb2;
        const uint32_t pos = atomicAdd(&base[cost_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u);
        if (pos < nblocks) order[pos] = b;
    }
}

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    }
    return cus;
}

template <int CPL, typename FT, int WAVES, int BG, bool EXT>
hipError_t launch(const FsRecord* records, const uint64_t* keys, const uint32_t* vals, const uint32_t* ranges,
                  const void* feats, int C, int64_t n, const fs_camera* cams, int num_views, int64_t total_tiles,
                  const fs_opts& o, float* out_feat, float* out_T, int32_t* out_n, int32_t* out_last,
                  int32_t* out_idx, float* out_depth, float* out_normal, uint64_t* counters, const FsWorkspace& ws,
                  hipStream_t s) {
    constexpr int RB = WAVES == 1 ? 8 : 16;
    const int sb = o.tile / RB;
    const int64_t blocks = total_tiles * sb * sb;
    if (blocks >= (int64_t(1) << 32)) return hipErrorInvalidValue;
    const int chunks = (C + 64 * CPL - 1) / (64 * CPL);
    const bool vec = (C % (16 / (int)sizeof(FT))) == 0;
    auto kern = vec ? render_fwd_kernel<CPL, FT, WAVES, BG, true, EXT> : render_fwd_kernel<CPL, FT, WAVES, BG, false, EXT>;
    if (o.schedule == FS_SCHED_PERSISTENT && chunks == 1 && blocks <= ws.render_max_blocks) {
        const uint32_t nb = (uint32_t)blocks;
        const hipError_t e = fs_launch_block_order(ranges, sb * sb, nb, ws, s);
        if (e != hipSuccess) return e;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), WAVES * 64, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        int64_t grid = (int64_t)device_cus() * per_cu;
        if (grid > blocks) grid = blocks;
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(WAVES * 64), 0, s, records, keys, vals, ranges,
                           static_cast<const FT*>(feats), C, n, n * num_views, cams, num_views, o.tile, o, out_feat,
                           out_T, out_n, out_last, out_idx, out_depth, out_normal, counters, ws.render_order,
                           ws.render_ticket, nb);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks, (unsigned)chunks), dim3(WAVES * 64), 0, s, records, keys, vals,
                       ranges, static_cast<const FT*>(feats), C, n, n * num_views, cams, num_views, o.tile, o,
                       out_feat, out_T, out_n, out_last, out_idx, out_depth, out_normal, counters,
                       (const uint32_t*)nullptr, (uint32_t*)nullptr, 0u);
    return hipGetLastError();
}

template <int CPL, typename FT, int NW, int BG, bool EXT>
hipError_t launch_wide(const FsRecord* records, const uint64_t* keys, const uint32_t* vals, const uint32_t* ranges,
                       const void* feats, int C, int64_t n, const fs_camera* cams, int num_views, int64_t total_tiles,
                       const fs_opts& o, float* out_feat, float* out_T, int32_t* out_n, int32_t* out_last,
                       int32_t* out_idx, float* out_depth, float* out_normal, uint64_t* counters,
                       const FsWorkspace& ws, hipStream_t s) {
    const int64_t blocks = total_tiles;   // one 8x8 block per tile
    if (blocks >= (int64_t(1) << 32)) return hipErrorInvalidValue;
    const int chunks = (C + 64 * CPL - 1) / (64 * CPL);
    const bool vec = (C % (16 / (int)sizeof(FT))) == 0;
    auto kern = vec ? render_wide_kernel<CPL, FT, NW, BG, true, EXT> : render_wide_kernel<CPL, FT, NW, BG, false, EXT>;
    if (o.schedule == FS_SCHED_PERSISTENT && chunks == 1 && blocks <= ws.render_max_blocks) {
        const uint32_t nb = (uint32_t)blocks;
        const hipError_t e = fs_launch_block_order(ranges, 1, nb, ws, s);
        if (e != hipSuccess) return e;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), NW * 64, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        int64_t grid = (int64_t)device_cus() * per_cu;
        if (grid > blocks) grid = blocks;
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NW * 64), 0, s, records, keys, vals, ranges,
                           static_cast<const FT*>(feats), C, n, n * num_views, cams, num_views, o.tile, o, out_feat,
                           out_T, out_n, out_last, out_idx, out_depth, out_normal, counters, ws.render_order,
                           ws.render_ticket, nb);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks, (unsigned)chunks), dim3(NW * 64), 0, s, records, keys, vals,
                       ranges, static_cast<const FT*>(feats), C, n, n * num_views, cams, num_views, o.tile, o,
                       out_feat, out_T, out_n, out_last, out_idx, out_depth, out_normal, counters,
                       (const uint32_t*)nullptr, (uint32_t*)nullptr, 0u);
    return hipGetLastError();
}

template <int CPL, typename FT>
hipError_t launch_waves(const FsRecord* records, const uint64_t* keys, const uint32_t* vals, const uint32_t* ranges,
                        const void* feats, int C, int64_t n, const fs_camera* cams, int num_views,
                        int64_t total_tiles, const fs_opts& o, float* out_feat, float* out_T, int32_t* out_n,
                        int32_t* out_last, int32_t* out_idx, float* out_depth, float* out_normal,
                        uint64_t* counters, const FsWorkspace& ws, hipStream_t s) {
    // 8x8 tiles: one-wave blocks; larger tiles: 16x16 blocks of four waves sharing the list staging
    const bool small = o.tile == 8;
    const bool bg16 = o.batch == 16;
    // the low-pass response and the depth / normal outputs run in their own
    // instantiations (32-entry batches), so the plain render carries none of
    // their registers
    const bool ext = o.lowpass != 0 || out_depth != nullptr || out_normal != nullptr;
#define FS_LAUNCH(W, B, X)                                                                                         \
    return launch<CPL, FT, W, B, X>(records, keys, vals, ranges, feats, C, n, cams, num_views, total_tiles, o,     \
                                    out_feat, out_T, out_n, out_last, out_idx, out_depth, out_normal, counters, ws, \
                                    s)
#define FS_WIDE(B, X)                                                                                           \
    return launch_wide<CPL, FT, 4, B, X>(records, keys, vals, ranges, feats, C, n, cams, num_views, total_tiles, o, \
                                         out_feat, out_T, out_n, out_last, out_idx, out_depth, out_normal, counters, \
                                         ws, s)
    if (ext) {
        if (small) FS_WIDE(32, true);
        FS_LAUNCH(4, 32, true);
    }
    if (small) {
        if (bg16) FS_WIDE(16, false);
        FS_WIDE(32, false);
    }
    if (bg16) FS_LAUNCH(4, 16, false);
    FS_LAUNCH(4, 32, false);
#undef FS_WIDE
#undef FS_LAUNCH
}

}  // namespace

hipError_t fs_launch_block_order(const uint32_t* ranges, int sb2, uint32_t nblocks, const FsWorkspace& ws,
                                 hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    if ((int64_t)nblocks > ws.render_max_blocks || ws.render_order == nullptr) return hipErrorInvalidValue;
    const unsigned g = (nblocks + 255) / 256;
    if (ws.render_gcnt == nullptr || (int64_t)g * 64 > ws.render_gcnt_words) return hipErrorInvalidValue;
    hipLaunchKernelGGL(order_count_kernel, dim3(g), dim3(256), 0, s, ranges, sb2, nblocks, ws.render_gcnt,
                       ws.render_ticket);
    hipLaunchKernelGGL(order_place_kernel, dim3(g), dim3(256), 0, s, ranges, sb2, nblocks, ws.render_gcnt, g,
                       ws.render_order);
    return hipGetLastError();
}

hipError_t fs_launch_render_forward(const FsRecord* records, const uint64_t* keys, const uint32_t* vals,
                                    const uint32_t* ranges, const void* feats, int C, int64_t n,
                                    const fs_camera* cams, int num_views, int64_t total_tiles, const fs_opts& o,
                                    float* out_feat, float* out_T, int32_t* out_n, int32_t* out_last,
                                    int32_t* out_idx, float* out_depth, float* out_normal, uint64_t* counters,
                                    const FsWorkspace& ws, hipStream_t s) {
    if (total_tiles == 0) return hipSuccess;
    const bool bf16 = o.feat_dtype == FS_FEAT_BF16;
#define FS_WAVES(CPLv, FTv)                                                                                          \
    return launch_waves<CPLv, FTv>(records, keys, vals, ranges, feats, C, n, cams, num_views, total_tiles, o,      \
                                   out_feat, out_T, out_n, out_last, out_idx, out_depth, out_normal, counters, ws, s)
    if (C <= 64) {
        if (bf16) FS_WAVES(1, uint16_t);
        FS_WAVES(1, float);
    }
    if (bf16) FS_WAVES(2, uint16_t);
    FS_WAVES(2, float);
#undef FS_WAVES
}
