// render_bwd.hip -- gradients of L = sum_p g_p . F_p through the blend
// (Sec. 3.1 Eq. 2, Top-K of Sec. 3.4), the ray-splat intersection and the
// projection (Sec. 3.1 Eq. 1, Sec. 3.2 T) back to the surfel parameters.
//
// With contributors m of a pixel in depth order, w_m = alpha_m T_m:
//   dL/dc_m     = w_m g
//   dL/dalpha_m = T_m (g . c_m) - S_m / (1 - alpha_m),  S_m = sum_{l > m} w_l (g . c_l)
//   alpha = o exp(-d2 / 2) unless clamped at alpha_max (then no gradient)
//   d2 = u^2 + v^2, (u, v) = (h0 / h2, h1 / h2), h = L (1, dx, dy)
// where L is the anchored, normalised 3x3 coefficient matrix of the record.
// The blend's discrete choices are those of the forward pass: the same
// double-precision response decides acceptance, and entries after the
// pixel's last blended position are skipped.
//
// Kernel 1 (per 8x8 block, one wave): the tile list is walked back to front
// in batches.  Lanes = pixels recover T by division from the forward's final
// transmittance and form the weights; lanes = channels form g . c_m (a wave
// reduction per contribution) and accumulate w g into per-entry LDS rows;
// lanes = pixels then run the scalar chain to dL/dL (9) and dL/do, reduced
// over the wave per entry.  Per-entry results go to global memory with
// atomics (float, so the sum order, hence the last bits, can vary).
// Kernel 2 (per surfel): dL/dL -> dL/dadj(T) -> dL/dT -> centre, scales,
// quaternion, summed over views, in double precision.
#include "fs_internal.h"

namespace {

constexpr int BG = 32;
constexpr int kGradFloats = FS_GRAD_RECORD_FLOATS;   // 9 (dL/dL) + 1 (dL/do) + 2 pad

FS_DEV float bf16_to_f32b(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
template <typename FT>
FS_DEV float to_f32(FT x);
template <>
FS_DEV float to_f32<float>(float x) { return x; }
template <>
FS_DEV float to_f32<uint16_t>(uint16_t x) { return bf16_to_f32b(x); }

// Butterfly sum over the wave (every lane gets the same bits).
FS_DEV float wave_sum(float x) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) x += __uint_as_float(lane_xor32(__float_as_uint(x), d));
    return x;
}

// dL/dalpha of one (pixel, record) contribution -> dL/dL (9, rows of the
// record's coefficient matrix times (1, dx, dy)) and dL/do, through alpha = o
// exp(-d2 / 2) (no gradient when clamped at alpha_max), d2 = u^2 + v^2 and
// (u, v) = (h0, h1) / h2.
FS_DEV void blend_chain(const FsRecord& r, const FsResp& rs, double ddx, double ddy, float Gs, float dalpha,
                        float* g) {
    g[9] = Gs * dalpha;   // dL/do
    const float dG = r.o * dalpha;
    const float dd2 = -0.5f * Gs * dG;
    const float u = (float)rs.u, vv = (float)rs.v, rh = (float)rs.rh;
    const float du = 2.f * u * dd2, dv = 2.f * vv * dd2;
    const float dh0 = du * rh, dh1 = dv * rh, dh2 = -(u * du + vv * dv) * rh;
    const float fx = (float)ddx, fy = (float)ddy;
    g[0] = dh0;
    g[1] = dh0 * fx;
    g[2] = dh0 * fy;
    g[3] = dh1;
    g[4] = dh1 * fx;
    g[5] = dh1 * fy;
    g[6] = dh2;
    g[7] = dh2 * fx;
    g[8] = dh2 * fy;
}

__global__ void zero_f32_kernel(float* p, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0.f;
}

template <int CPL, typename FT>
__global__ void __launch_bounds__(64)
render_bwd_kernel(const FsRecord* __restrict__ records, const uint32_t* __restrict__ vals,
                  const uint32_t* __restrict__ ranges, const FT* __restrict__ feats, int C, int64_t n,
                  int64_t num_records, const fs_camera* __restrict__ cams, int num_views, int S, fs_opts o,
                  const float* __restrict__ out_T, const int32_t* __restrict__ out_last,
                  const float* __restrict__ grad_feat, float* __restrict__ grad_records,
                  float* __restrict__ grad_feats) {
    constexpr int kChunk = 64 * CPL;
    __shared__ FsRecord s_rec[BG];
    __shared__ uint32_t s_recid[BG];
    __shared__ float s_feat[BG][kChunk];
    __shared__ float s_dfeat[BG][kChunk];
    __shared__ float s_w[BG][64];
    __shared__ float s_D[BG][64];
    __shared__ float s_grec[BG][kGradFloats];

    const int lane = threadIdx.x;
    // block position (8x8 pixels inside a binning tile); the XCDs take one
    // tile row of blocks each in turn (4.38 -> 3.99 ms on the 640x480
    // full-blend backward)
    const int sb = S / 8;
    const int64_t b = xcd_remap_chunked(blockIdx.x, gridDim.x, block_row_chunk(cams, S));
    const int64_t tile = b / (sb * sb);
    const int sub = (int)(b % (sb * sb));
    const int v = fs_view_of_tile(cams, num_views, tile);
    const fs_camera& cam = cams[v];
    const int tiles_x = (cam.width + S - 1) / S;
    const int64_t local = tile - cam.tile_offset;
    const int wx0 = (int)(local % tiles_x) * S + (sub % sb) * 8;
    const int wy0 = (int)(local / tiles_x) * S + (sub / sb) * 8;
    if (wx0 >= cam.width || wy0 >= cam.height) return;
    const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
    const bool inside = px < cam.width && py < cam.height;
    const int64_t pix = cam.pixel_offset + (int64_t)py * cam.width + px;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    const int last = inside ? out_last[pix] : -1;
    // walk back from the block's last blended entry
    int maxlast = last;
    maxlast = __ockl_wfred_max_i32(maxlast);
    if (maxlast < (int)start) return;   // nothing was blended in this block
    // a last position from another frame's lists must not walk past this
    // tile's run into the next tile's entries
    const uint32_t top = min((uint32_t)maxlast + 1u, end);
    if (top <= start) return;
    double T = inside ? (double)out_T[pix] : 1.0;
    float suffix = 0.f;                 // S: sum over later contributors of w (g . c)

    // upstream gradient of the block's pixels, lanes = channels
    float G[64][CPL];
#pragma unroll
    for (int p = 0; p < 64; ++p) {
        const int qx = wx0 + (p & 7), qy = wy0 + (p >> 3);
        const bool in = qx < cam.width && qy < cam.height;
        const int64_t q = cam.pixel_offset + (int64_t)qy * cam.width + qx;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int ch = lane * CPL + c;
            G[p][c] = (in && ch < C) ? grad_feat[q * C + ch] : 0.f;
        }
    }

    const uint32_t nbatch = (top - start + BG - 1) / BG;
    for (uint32_t bi = nbatch; bi-- > 0;) {
        const uint32_t b0 = start + bi * BG;
        const int nb = (int)(top - b0 < (uint32_t)BG ? top - b0 : (uint32_t)BG);
        // 1. stage records
        constexpr int kQ = FS_RECORD_BYTES / 16;
        for (int t = lane; t < nb * kQ; t += 64) {
            const int e = t / kQ, q = t - e * kQ;
            uint32_t rid = vals[b0 + e];
            float4 v4 = make_float4(0.f, 0.f, 0.f, 0.f);
            if ((int64_t)rid < num_records) {
                v4 = reinterpret_cast<const float4*>(records + rid)[q];
            } else {
                rid = 0u;
                if (q == 4) v4.w = __int_as_float((int)0xbff00000);
                if (q == 5) v4.z = __int_as_float(1);
            }
            reinterpret_cast<float4*>(&s_rec[e])[q] = v4;
            if (q == 0) s_recid[e] = rid;
        }
        for (int t = lane; t < BG * kGradFloats; t += 64) (&s_grec[0][0])[t] = 0.f;
        for (int t = lane; t < BG * kChunk; t += 64) (&s_dfeat[0][0])[t] = 0.f;
        __syncthreads();
        // 2. weights, back to front (lanes = pixels)
        uint32_t mask = 0u;
        for (int e = nb - 1; e >= 0; --e) {
            const FsRecord& r = s_rec[e];
            if (r.x1 < wx0 || r.x0 > wx0 + 7 || r.y1 < wy0 || r.y0 > wy0 + 7) continue;
            if ((int)(b0 + e) > last) continue;
            const FsResp rs = fs_response(r, (double)(px - r.ax), (double)(py - r.ay));
            if (rs.d2 <= r.k2 && fs_in_box(r, px, py)) {
                const float Gs = __builtin_amdgcn_exp2f(-0.72134752044448170f * (float)rs.d2);
                const float alpha = fminf(o.alpha_max, r.o * Gs);
                T = T / (1.0 - (double)alpha);
                s_w[e][lane] = (float)((double)alpha * T);
                mask |= 1u << e;
            }
        }
        const uint32_t used = __ockl_wfred_or_u32(mask);
        const uint64_t active_px = __ballot(mask != 0u);
        // 3. feature rows of used entries
        for (int t = lane; t < BG * kChunk; t += 64) {
            const int e = t / kChunk, c = t - e * kChunk;
            // channels >= C are zeroed: the wave-wide dot products read every lane
            if ((used >> e) & 1u) s_feat[e][c] = c < C ? to_f32(feats[fs_surfel_of(s_recid[e], n) * C + c]) : 0.f;
        }
        __syncthreads();
        // 4. lanes = channels: D = g . c per contribution, dL/dc += w g per entry
#pragma unroll
        for (int p = 0; p < 64; ++p) {
            if ((active_px >> p) & 1ull) {
                uint32_t m = __builtin_amdgcn_readlane(mask, p);
                while (m) {
                    const int e = __builtin_ctz(m);
                    m &= m - 1u;
                    float part = 0.f;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) part = fmaf(G[p][c], s_feat[e][lane * CPL + c], part);
                    const float D = wave_sum(part);
                    if (lane == 0) s_D[e][p] = D;
                    const float w = s_w[e][p];
#pragma unroll
                    for (int c = 0; c < CPL; ++c) s_dfeat[e][lane * CPL + c] += w * G[p][c];
                }
            }
        }
        __syncthreads();
        // 5. lanes = pixels: scalar chain back to front
        for (int e = nb - 1; e >= 0; --e) {
            if (!((used >> e) & 1u)) continue;
            const bool mine = (mask >> e) & 1u;
            float g[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) g[k] = 0.f;
            if (mine) {
                const FsRecord& r = s_rec[e];
                const double ddx = (double)(px - r.ax), ddy = (double)(py - r.ay);
                const FsResp rs = fs_response(r, ddx, ddy);
                const float Gs = __builtin_amdgcn_exp2f(-0.72134752044448170f * (float)rs.d2);
                const float ag = r.o * Gs;
                const bool clamped = ag > o.alpha_max;
                const float alpha = clamped ? o.alpha_max : ag;
                const float w = s_w[e][lane];
                const float Tm = w / alpha;
                const float D = s_D[e][lane];
                const float dalpha = Tm * D - suffix / (1.f - alpha);
                suffix = fmaf(w, D, suffix);
                if (!clamped) blend_chain(r, rs, ddx, ddy, Gs, dalpha, g);
            }
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const float sum = wave_sum(g[k]);
                if (lane == 0) s_grec[e][k] = sum;
            }
        }
        __syncthreads();
        // 6. flush per-entry gradients
        for (int t = lane; t < BG * kGradFloats; t += 64) {
            const int e = t / kGradFloats, k = t - e * kGradFloats;
            if (((used >> e) & 1u) && k < 10) atomicAdd(&grad_records[(int64_t)s_recid[e] * kGradFloats + k], s_grec[e][k]);
        }
        for (int t = lane; t < BG * kChunk; t += 64) {
            const int e = t / kChunk, c = t - e * kChunk;
            if (((used >> e) & 1u) && c < C)
                atomicAdd(&grad_feats[fs_surfel_of(s_recid[e], n) * C + c], s_dfeat[e][c]);
        }
        __syncthreads();
    }
}

// dL/dL (anchored, normalised record coefficients; columns: constant, dx, dy)
// back to the surfel parameters.  L = adj(T) A / s with A mapping (1, dx, dy)
// to (x, y, 1) = (xa + dx, ya + dy, 1); since (u, v) does not change when L is
// scaled, the dependence of s on T contributes nothing and dL/dadj = dL/dL A^T / s.
__global__ void __launch_bounds__(256)
preprocess_bwd_kernel(const float* __restrict__ means, const float* __restrict__ scales,
                      const float* __restrict__ quats, const float* __restrict__ opacity, int64_t n,
                      const fs_camera* __restrict__ cams, int num_views, fs_opts o,
                      const float* __restrict__ grad_records, float* __restrict__ gm, float* __restrict__ gs,
                      float* __restrict__ gq, float* __restrict__ go) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double am[3] = {0, 0, 0}, as[2] = {0, 0}, aq[4] = {0, 0, 0, 0}, ao = 0.0;
    for (int v = 0; v < num_views; ++v) {
        const float* gr = grad_records + ((int64_t)v * n + i) * kGradFloats;
        double dl[9];
        bool any = false;
        for (int k = 0; k < 9; ++k) {
            dl[k] = gr[k];
            any = any || dl[k] != 0.0;
        }
        ao += gr[9];
        if (!any) continue;
        const fs_camera& cam = cams[v];
        FsGeo g;
        if (!fs_project(means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i], cam, (double)o.alpha_min, g))
            continue;
        FsFootprint fp;
        fs_footprint(g, cam.width, cam.height, fp);
        const double mx = g.T[2] / g.T[8], my = g.T[5] / g.T[8];
        const double s = (g.H[6] * mx + g.H[7] * my) + g.H[8];
        const double xa = fp.q.ax + 0.5, ya = fp.q.ay + 0.5;
        // dL/dH = dL/dL A^T / s ; A = [[xa,1,0],[ya,0,1],[1,0,0]]  (rows of H act on (x, y, 1))
        double dH[9];
        for (int r = 0; r < 3; ++r) {
            const double l0 = dl[3 * r], l1 = dl[3 * r + 1], l2 = dl[3 * r + 2];
            dH[3 * r + 0] = (l0 * xa + l1) / s;   // column x
            dH[3 * r + 1] = (l0 * ya + l2) / s;   // column y
            dH[3 * r + 2] = l0 / s;               // column 1
        }
        // H columns: T2 x Tw, Tw x T1, T1 x T2 ; for c = a x b: dL/da = b x g, dL/db = g x a
        const double* T1 = g.T;
        const double* T2 = g.T + 3;
        const double* Tw = g.T + 6;
        double gx[3], gy[3], g1[3];
        for (int r = 0; r < 3; ++r) {
            gx[r] = dH[3 * r];
            gy[r] = dH[3 * r + 1];
            g1[r] = dH[3 * r + 2];
        }
        double dT1[3], dT2[3], dTw[3], t0[3], t1[3];
        fs_cross(Tw, gx, t0);          // d(T2 x Tw)/dT2
        fs_cross(T1, g1, t1);          // d(T1 x T2)/dT2 = g1 x T1
        for (int k = 0; k < 3; ++k) dT2[k] = t0[k] - t1[k];
        fs_cross(gx, T2, t0);          // d(T2 x Tw)/dTw
        fs_cross(T1, gy, t1);          // d(Tw x T1)/dTw
        for (int k = 0; k < 3; ++k) dTw[k] = t0[k] + t1[k];
        fs_cross(gy, Tw, t0);          // d(Tw x T1)/dT1
        fs_cross(T2, g1, t1);          // d(T1 x T2)/dT1
        for (int k = 0; k < 3; ++k) dT1[k] = t0[k] + t1[k];
        // T = K [U | V | pc]: rows T1 = fx M0 + cx M2, T2 = fy M1 + cy M2, Tw = M2
        double dM0[3], dM1[3], dM2[3];
        for (int c = 0; c < 3; ++c) {
            dM0[c] = (double)cam.fx * dT1[c];
            dM1[c] = (double)cam.fy * dT2[c];
            dM2[c] = (double)cam.cx * dT1[c] + (double)cam.cy * dT2[c] + dTw[c];
        }
        const double dU[3] = {dM0[0], dM1[0], dM2[0]};
        const double dV[3] = {dM0[1], dM1[1], dM2[1]};
        const double dpc[3] = {dM0[2], dM1[2], dM2[2]};
        FsFrame fr;
        fs_frame(means + 3 * i, scales + 2 * i, quats + 4 * i, cam, fr);
        double Rtu[3], Rtv[3], dtu[3], dtv[3];
        for (int r = 0; r < 3; ++r) {
            const double R0 = cam.R[3 * r], R1 = cam.R[3 * r + 1], R2 = cam.R[3 * r + 2];
            Rtu[r] = (R0 * fr.tu[0] + R1 * fr.tu[1]) + R2 * fr.tu[2];
            Rtv[r] = (R0 * fr.tv[0] + R1 * fr.tv[1]) + R2 * fr.tv[2];
        }
        const double s0 = scales[2 * i], s1 = scales[2 * i + 1];
        for (int k = 0; k < 3; ++k) {
            const double Rk0 = cam.R[k], Rk1 = cam.R[3 + k], Rk2 = cam.R[6 + k];   // column k of R
            am[k] += (Rk0 * dpc[0] + Rk1 * dpc[1]) + Rk2 * dpc[2];
            dtu[k] = s0 * ((Rk0 * dU[0] + Rk1 * dU[1]) + Rk2 * dU[2]);
            dtv[k] = s1 * ((Rk0 * dV[0] + Rk1 * dV[1]) + Rk2 * dV[2]);
        }
        as[0] += fs_dot(Rtu, dU);
        as[1] += fs_dot(Rtv, dV);
        // quaternion: t_u = (1 - f a1, f a2, f a3), t_v = (f b1, 1 - f b2, f b3), f = 2 / |q|^2
        const double w = quats[4 * i], x = quats[4 * i + 1], y = quats[4 * i + 2], z = quats[4 * i + 3];
        const double f = fr.f;
        const double a1 = y * y + z * z, a2 = x * y + w * z, a3 = x * z - w * y;
        const double b1 = x * y - w * z, b2 = x * x + z * z, b3 = y * z + w * x;
        const double sf = -dtu[0] * a1 + dtu[1] * a2 + dtu[2] * a3 + dtv[0] * b1 - dtv[1] * b2 + dtv[2] * b3;
        const double q[4] = {w, x, y, z};
        const double da1[4] = {0, 0, 2 * y, 2 * z}, da2[4] = {z, y, x, w}, da3[4] = {-y, z, -w, x};
        const double db1[4] = {-z, y, x, -w}, db2[4] = {0, 2 * x, 0, 2 * z}, db3[4] = {x, w, z, y};
        for (int k = 0; k < 4; ++k) {
            const double inner = -dtu[0] * da1[k] + dtu[1] * da2[k] + dtu[2] * da3[k] + dtv[0] * db1[k] -
                                 dtv[1] * db2[k] + dtv[2] * db3[k];
            aq[k] += -f * f * q[k] * sf + f * inner;
        }
    }
    for (int k = 0; k < 3; ++k) gm[3 * i + k] += (float)am[k];
    gs[2 * i] += (float)as[0];
    gs[2 * i + 1] += (float)as[1];
    for (int k = 0; k < 4; ++k) gq[4 * i + k] += (float)aq[k];
    go[i] += (float)ao;
}

// ---------------------------------------------------------------------------
// Top-K backward.  The selection pass of the split forward recomputes every
// pixel's (row slot, weight) list and every block's row list; then one
// workgroup per 8x8 block:
//   1. D = g . c for every (pixel, contributor): feature rows are staged in
//      LDS windows (direct global -> LDS loads), TPP threads per pixel each
//      hold one 16-byte channel vector of g in registers and reduce their
//      partial dot products with shuffles inside the pixel's group; the same
//      pass adds w g to per-row LDS accumulators (float atomics), flushed once
//      per (block, row) to dL/dc;
//   2. per contribution, all pairs of the block in parallel: alpha from the
//      record; per pixel (LDS only) the forward's transmittance chain (double
//      precision, same order) and the suffix sums S = sum_{l > m} w_l D_l;
//      then the chain to dL/dL and dL/do, summed per row slot in LDS and
//      flushed once per (block, slot).
// ---------------------------------------------------------------------------
constexpr int kGradThreads = 256;
constexpr int kGradMaxK = 16;
static_assert(kGradMaxK <= FS_TOPK_COMPACT_K, "the gradient pass reads compact lists");
constexpr int kGradSlots = 256;   // row slots whose geometry gradients are summed in LDS

template <typename FT>
struct RowV;
template <>
struct RowV<float> {
    static constexpr int VE = 4;
    FS_DEV static void get(const uint4& r, float* f) {
        f[0] = __uint_as_float(r.x);
        f[1] = __uint_as_float(r.y);
        f[2] = __uint_as_float(r.z);
        f[3] = __uint_as_float(r.w);
    }
};
template <>
struct RowV<uint16_t> {
    static constexpr int VE = 8;
    FS_DEV static void get(const uint4& r, float* f) {
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f[2 * i] = __uint_as_float(w[i] << 16);
            f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    }
};

template <typename FT, int TPP>
__global__ void __launch_bounds__(kGradThreads)
topk_grad_kernel(const FsRecord* __restrict__ records, const uint2* __restrict__ pairs,
                 const int32_t* __restrict__ counts, const uint32_t* __restrict__ rows,
                 const uint32_t* __restrict__ nrows, const FT* __restrict__ feats, int C, int K, int64_t n,
                 const fs_camera* __restrict__ cams, int num_views, int S, int64_t nblocks, fs_opts o,
                 const float* __restrict__ grad_feat, float* __restrict__ grad_records,
                 float* __restrict__ grad_feats) {
    constexpr int VE = RowV<FT>::VE;
    constexpr int kGroups = kGradThreads / TPP;   // row slots handled at once
    constexpr int kPairs = 64 * kGradMaxK;
    __shared__ uint2 s_pairs[kPairs];
    __shared__ float s_D[kPairs];
    __shared__ float s_S[kPairs];    // alpha, then the transmittance before the contribution
    __shared__ float s_T2[kPairs];   // alpha
    __shared__ float s_U[kPairs];    // suffix sums S = sum_{l > m} w_l D_l
    __shared__ int s_soff[kPairs + 1];       // per row slot: first entry of its pair list
    __shared__ int s_sfill[kPairs];          // per row slot: pairs, then the fill cursor
    __shared__ uint16_t s_list[kPairs];      // pair indices p * K + j grouped by row slot
    __shared__ int s_cnt[64];
    __shared__ int s_off[64];                // first pair of each pixel's compact list
    __shared__ int s_wave[kGradThreads / 64];
    __shared__ float s_grec[kGradSlots][10];   // dL/dL and dL/do of the first kGradSlots row slots
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t block = xcd_remap_chunked(blockIdx.x, nblocks, block_row_chunk(cams, S));
    const BlockPos bp = locate_block(block, S, 8, cams, num_views);
    if (!bp.valid) return;           // uniform
    const uint32_t R = nrows[block] & 0xffffu;   // rows (the high half counts the listed pairs)
    if (R == 0) return;              // no pixel of the block blended anything
    const fs_camera& cam = cams[bp.view];
    const int nv = C / VE;           // channel vectors per row (C % VE == 0)
    const int q = tid % TPP, grp = tid / TPP;
    const bool has_vec = q < nv;
    const uint32_t* __restrict__ rowlist = rows + block * 64 * (int64_t)K;
    const int npairs = 64 * K;
    for (int t = tid; t < npairs; t += kGradThreads) s_sfill[t] = 0;
    if (tid < 64) {
        // counts, and the offsets of the pixels' lists in the block's compact
        // list area (the selection writes them back to back)
        const int px = bp.x0 + (tid & 7), py = bp.y0 + (tid >> 3);
        const int c = (px < cam.width && py < cam.height) ? counts[cam.pixel_offset + (int64_t)py * cam.width + px] : 0;
        const int incl = __ockl_wfscan_add_i32(c, true);
        s_cnt[tid] = c;
        s_off[tid] = incl - c;
    }
    __syncthreads();
    // pair j of pixel p at LDS p * K + j
    for (int t = tid; t < npairs; t += kGradThreads) {
        const int p = t / K, j = t - p * K;
        if (j < s_cnt[p]) s_pairs[t] = pairs[block * 64 * (int64_t)K + s_off[p] + j];
    }
    __syncthreads();
    // 1a. pairs grouped by row slot (counting sort in LDS)
    for (int t = tid; t < npairs; t += kGradThreads)
        if (t % K < s_cnt[t / K]) atomicAdd(&s_sfill[s_pairs[t].x], 1);
    __syncthreads();
    {
        constexpr int kPer = (kPairs + kGradThreads - 1) / kGradThreads;
        const int b0 = tid * kPer;
        int c[kPer];
        int sum = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            c[i] = b0 + i < (int)R ? s_sfill[b0 + i] : 0;
            sum += c[i];
        }
        const int incl = __ockl_wfscan_add_i32(sum, true);
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        int off = incl - sum;
        for (int w = 0; w < wave; ++w) off += s_wave[w];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            if (b0 + i < (int)R) {
                s_soff[b0 + i] = off;
                s_sfill[b0 + i] = 0;
            }
            off += c[i];
        }
        if (tid == kGradThreads - 1) s_soff[R] = off;
    }
    __syncthreads();
    for (int t = tid; t < npairs; t += kGradThreads)
        if (t % K < s_cnt[t / K]) {
            const uint32_t slot = s_pairs[t].x;
            s_list[s_soff[slot] + atomicAdd(&s_sfill[slot], 1)] = (uint16_t)t;
        }
    __syncthreads();
    // 1b. slot-major: a group of TPP threads owns a row slot and one channel
    //     vector per thread; it reads the feature row once and, over the
    //     slot's pixels, forms D = g . c (shuffle reduction inside the group)
    //     and dL/dc = sum w g in registers, flushed once per (block, slot)
    for (uint32_t s0 = 0; s0 < R; s0 += kGroups) {
        const uint32_t slot = s0 + (uint32_t)grp;
        const bool live = slot < R;   // uniform inside the group
        float f[VE], acc[VE];
#pragma unroll
        for (int i = 0; i < VE; ++i) acc[i] = f[i] = 0.f;
        uint32_t sidx = 0;
        if (live) {
            sidx = rowlist[slot];
            if (has_vec) RowV<FT>::get(*reinterpret_cast<const uint4*>(feats + (int64_t)sidx * C + q * VE), f);
        }
        const int a = live ? s_soff[slot] : 0, b = live ? s_soff[slot + 1] : 0;
        for (int i = a; i < b; ++i) {
            const int t = s_list[i];
            const int p = t / K;
            const int px = bp.x0 + (p & 7), py = bp.y0 + (p >> 3);
            float gv[VE];
            if (has_vec) {
                const float* src = grad_feat + (cam.pixel_offset + (int64_t)py * cam.width + px) * C + q * VE;
#pragma unroll
                for (int e = 0; e < VE; e += 4) {
                    const float4 v = *reinterpret_cast<const float4*>(src + e);
                    gv[e] = v.x;
                    gv[e + 1] = v.y;
                    gv[e + 2] = v.z;
                    gv[e + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int e = 0; e < VE; ++e) gv[e] = 0.f;
            }
            const float w = __uint_as_float(s_pairs[t].y);
            float part = 0.f;
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                part = fmaf(gv[e], f[e], part);
                acc[e] = fmaf(w, gv[e], acc[e]);
            }
#pragma unroll
            for (int d = 1; d < TPP; d <<= 1) part += __uint_as_float(lane_xor32(__float_as_uint(part), d));
            if (q == 0) s_D[t] = part;
        }
        if (live && has_vec) {
#pragma unroll
            for (int e = 0; e < VE; ++e) atomicAdd(&grad_feats[(int64_t)sidx * C + q * VE + e], acc[e]);
        }
    }
    for (int t = tid; t < kGradSlots * 10; t += kGradThreads) (&s_grec[0][0])[t] = 0.f;
    // 2. per contribution, all pairs of the block in parallel: (a) alpha (the
    //    forward's float value); (b) per pixel, from LDS only, the transmittance
    //    before every contribution (the forward's double-precision product) and
    //    the suffix sums; (c) the chain to dL/dL and dL/do, summed per row slot.
    for (int t = tid; t < npairs; t += kGradThreads) {
        const int p = t / K, j = t - p * K;
        if (j >= s_cnt[p]) continue;
        const int px = bp.x0 + (p & 7), py = bp.y0 + (p >> 3);
        const FsRecord& r = records[(int64_t)bp.view * n + rowlist[s_pairs[t].x]];
        const FsResp rs = fs_response(r, (double)(px - r.ax), (double)(py - r.ay));
        const float Gs = __builtin_amdgcn_exp2f(-0.72134752044448170f * (float)rs.d2);
        s_S[t] = fminf(o.alpha_max, r.o * Gs);   // alpha, for now
    }
    __syncthreads();
    if (tid < 64) {
        const int p = tid;
        const int c = s_cnt[p];
        double T = 1.0;
        for (int j = 0; j < c; ++j) {
            const float al = s_S[p * K + j];
            s_S[p * K + j] = (float)T;   // transmittance before the contribution
            s_T2[p * K + j] = al;
            T = T * (1.0 - (double)al);
        }
        float suffix = 0.f;
        for (int j = c - 1; j >= 0; --j) {
            const float wD = __uint_as_float(s_pairs[p * K + j].y) * s_D[p * K + j];
            s_U[p * K + j] = suffix;
            suffix += wD;
        }
    }
    __syncthreads();
    for (int t = tid; t < npairs; t += kGradThreads) {
        const int p = t / K, j = t - p * K;
        if (j >= s_cnt[p]) continue;
        const int px = bp.x0 + (p & 7), py = bp.y0 + (p >> 3);
        const uint32_t slot = s_pairs[t].x;
        const int64_t rid = (int64_t)bp.view * n + rowlist[slot];
        const FsRecord& r = records[rid];
        const double ddx = (double)(px - r.ax), ddy = (double)(py - r.ay);
        const FsResp rs = fs_response(r, ddx, ddy);
        const float Gs = __builtin_amdgcn_exp2f(-0.72134752044448170f * (float)rs.d2);
        const bool clamped = r.o * Gs > o.alpha_max;
        if (clamped) continue;
        const float alpha = s_T2[t];
        const float dalpha = s_S[t] * s_D[t] - s_U[t] / (1.f - alpha);
        float gg[10];
        blend_chain(r, rs, ddx, ddy, Gs, dalpha, gg);
        if (slot < (uint32_t)kGradSlots) {
#pragma unroll
            for (int k = 0; k < 10; ++k) atomicAdd(&s_grec[slot][k], gg[k]);
        } else {
#pragma unroll
            for (int k = 0; k < 10; ++k) atomicAdd(&grad_records[rid * kGradFloats + k], gg[k]);
        }
    }
    __syncthreads();
    const int nslot = (int)(R < (uint32_t)kGradSlots ? R : (uint32_t)kGradSlots);
    for (int t = tid; t < nslot * 10; t += kGradThreads) {
        const int slot = t / 10, k = t - slot * 10;
        const float v = s_grec[slot][k];
        if (v != 0.f) atomicAdd(&grad_records[((int64_t)bp.view * n + rowlist[slot]) * kGradFloats + k], v);
    }
}

template <typename FT>
hipError_t launch_topk_grad(const FsRecord* records, const void* feats, int C, int64_t n, const fs_camera* cams,
                            int num_views, int64_t nblocks, const fs_opts& o, const float* grad_feat,
                            float* grad_records, float* grad_feats, const FsWorkspace& ws, hipStream_t s) {
    constexpr int VE = RowV<FT>::VE;
    const int nv = C / VE;
    int tpp = 4;
    while (tpp < nv) tpp <<= 1;
    const FT* f = static_cast<const FT*>(feats);
#define FS_GRAD(TPP)                                                                                             \
    hipLaunchKernelGGL((topk_grad_kernel<FT, TPP>), dim3((unsigned)nblocks), dim3(kGradThreads), 0, s, records,    \
                       ws.topk_pairs, ws.topk_counts, ws.topk_rows, ws.topk_nrows, f, C, o.topk, n, cams, num_views, \
                       o.tile, nblocks, o, grad_feat, grad_records, grad_feats)
    switch (tpp) {
        case 4: FS_GRAD(4); break;
        case 8: FS_GRAD(8); break;
        case 16: FS_GRAD(16); break;
        case 32: FS_GRAD(32); break;
        default: FS_GRAD(64); break;
    }
#undef FS_GRAD
    return hipGetLastError();
}

template <int CPL, typename FT>
hipError_t launch_bwd(const FsRecord* records, const uint32_t* vals, const uint32_t* ranges, const void* feats,
                      int C, int64_t n, const fs_camera* cams, int num_views, int64_t total_tiles, const fs_opts& o,
                      const float* out_T, const int32_t* out_last, const float* grad_feat, float* grad_records,
                      float* grad_feats, hipStream_t s) {
    const int sb = o.tile / 8;
    const int64_t blocks = total_tiles * sb * sb;
    hipLaunchKernelGGL((render_bwd_kernel<CPL, FT>), dim3((unsigned)blocks), dim3(64), 0, s, records, vals, ranges,
                       static_cast<const FT*>(feats), C, n, n * num_views, cams, num_views, o.tile, o, out_T,
                       out_last, grad_feat, grad_records, grad_feats);
    return hipGetLastError();
}

}  // namespace

hipError_t fs_launch_render_backward(const float* means, const float* scales, const float* quats,
                                     const float* opacity, const FsRecord* records, const uint32_t* vals,
                                     const uint32_t* ranges, const void* feats, int C, int64_t n,
                                     const fs_camera* cams, int num_views, int64_t total_tiles, const fs_opts& o,
                                     const float* out_T, const int32_t* out_n, const int32_t* out_last,
                                     const float* grad_feat, float* grad_records, float* grad_means,
                                     float* grad_scales, float* grad_quats, float* grad_opacity, float* grad_feats,
                                     const FsWorkspace& ws, hipStream_t s) {
    (void)out_n;
    const int64_t nrec = n * num_views * kGradFloats;
    {
        unsigned blocks = (unsigned)((nrec + 255) / 256);
        blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
        hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks), dim3(256), 0, s, grad_records, nrec);
    }
    hipError_t e;
    const bool bf16 = o.feat_dtype == FS_FEAT_BF16;
    const int ve = bf16 ? 8 : 4;
    const int sb = o.tile / 8;
    const int64_t nblocks = total_tiles * sb * sb;
    if (o.topk > 0 && o.topk <= kGradMaxK && C % ve == 0 && C / ve <= 64 && ws.topk_pairs != nullptr &&
        ws.topk_counts != nullptr && nblocks < (int64_t(1) << 31)) {
        // recompute the selection, then the per-block gradient pass
        e = fs_launch_topk_select(records, nullptr, vals, ranges, n, cams, num_views, total_tiles, o, nullptr,
                                  ws.topk_counts, nullptr, nullptr, nullptr, nullptr, nullptr, ws, s);
        if (e != hipSuccess) return e;
        e = bf16 ? launch_topk_grad<uint16_t>(records, feats, C, n, cams, num_views, nblocks, o, grad_feat,
                                              grad_records, grad_feats, ws, s)
                 : launch_topk_grad<float>(records, feats, C, n, cams, num_views, nblocks, o, grad_feat, grad_records,
                                           grad_feats, ws, s);
    } else if (C <= 64)
        e = bf16 ? launch_bwd<1, uint16_t>(records, vals, ranges, feats, C, n, cams, num_views, total_tiles, o, out_T,
                                           out_last, grad_feat, grad_records, grad_feats, s)
                 : launch_bwd<1, float>(records, vals, ranges, feats, C, n, cams, num_views, total_tiles, o, out_T,
                                        out_last, grad_feat, grad_records, grad_feats, s);
    else
        e = bf16 ? launch_bwd<2, uint16_t>(records, vals, ranges, feats, C, n, cams, num_views, total_tiles, o, out_T,
                                           out_last, grad_feat, grad_records, grad_feats, s)
                 : launch_bwd<2, float>(records, vals, ranges, feats, C, n, cams, num_views, total_tiles, o, out_T,
                                        out_last, grad_feat, grad_records, grad_feats, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(preprocess_bwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, means, scales,
                       quats, opacity, n, cams, num_views, o, grad_records, grad_means, grad_scales, grad_quats,
                       grad_opacity);
    return hipGetLastError();
}
