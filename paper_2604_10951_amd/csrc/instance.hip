// instance.hip -- per-Gaussian instance labels from instance queries (Sec. 3.3).
//
// For every scene Gaussian g (a point p_g with an instance feature f_g of
// dimension D) and every query q (a feature f_q and a 3D Gaussian with
// centre p_q and covariance Sigma_q):
//   S = sigmoid(f_q . f_g)                                (feature similarity)
//   D = phi_q(p_g) / phi_q(p_q) = exp(-|L_q^-1 (p_g - p_q)|^2 / 2)
//       (the query's density relative to its peak; Sigma_q = L_q L_q^T)
//   l(g) = softmax over q of A = S D
// The Q label channels are what the label render blends per pixel.
//
// Per Gaussian the work reads 4 D + 12 bytes and writes 4 Q bytes for 2 D Q
// flops.  With packed FP32 off, the vector form spends about as many issue
// slots on the dot products as on the per-query epilogue, so for the paper's
// Q = D = 32 the dot products go to the matrix cores (instance_label_mfma_kernel,
// 0.066 against 0.078 ms for 1M Gaussians).  Other shapes use the vector form:
// one thread per Gaussian, its feature row against the query features, whose
// addresses are the same for the whole wave (scalar loads, no LDS traffic),
// with the Q dot products kept in registers for the softmax.
#include "fs_internal.h"

namespace {

constexpr int kInstThreads = 256;

// Query centre and the inverse Cholesky factor M = L^-1 (lower triangular,
// stored M11, M21, M22, M31, M32, M33), so that |M d|^2 = d^T Sigma^-1 d is
// a sum of squares.
struct QueryGeom {
    float c[3];
    float m[6];
};

// EXACT: Q == QMAX, so every per-query guard folds away at compile time.
// DC > 0: the feature dimension is DC and the whole row is loaded up front
// (all its loads in flight at once, overlapping the query set-up).
template <int QMAX, bool EXACT, int DC>
__global__ void __launch_bounds__(kInstThreads)
instance_label_kernel(const float* __restrict__ fins, int Drt, const float* __restrict__ means, int64_t n,
                      const float* __restrict__ fq, const float* __restrict__ qmeans,
                      const float* __restrict__ qcovs, int Qrt, float* __restrict__ out) {
    const int Q = EXACT ? QMAX : Qrt;
    const int D = DC > 0 ? DC : Drt;
    __shared__ QueryGeom s_q[QMAX];
    const int tid = (int)threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kInstThreads + tid;
    const bool live = i < n;
    const float4* __restrict__ row = reinterpret_cast<const float4*>(fins + (live ? i : 0) * D);
    constexpr int kPre = DC > 0 ? DC / 4 : 1;
    float4 pre[kPre];
    if constexpr (DC > 0) {
#pragma unroll
        for (int d4 = 0; d4 < kPre; ++d4) pre[d4] = row[d4];
    }
    if (tid < Q) {
        // Cholesky factor of the query covariance and its inverse, in double
        const float* s = qcovs + 6 * tid;   // xx, xy, xz, yy, yz, zz
        const double l11 = sqrt((double)s[0]);
        const double l21 = s[1] / l11, l31 = s[2] / l11;
        const double l22 = sqrt(s[3] - l21 * l21);
        const double l32 = (s[4] - l31 * l21) / l22;
        const double l33 = sqrt(s[5] - l31 * l31 - l32 * l32);
        const double m11 = 1.0 / l11, m22 = 1.0 / l22, m33 = 1.0 / l33;
        const double m21 = -l21 * m11 * m22;
        const double m32 = -l32 * m22 * m33;
        const double m31 = -(l31 * m11 + l32 * m21) * m33;
        QueryGeom g;
        g.c[0] = qmeans[3 * tid];
        g.c[1] = qmeans[3 * tid + 1];
        g.c[2] = qmeans[3 * tid + 2];
        g.m[0] = (float)m11;
        g.m[1] = (float)m21;
        g.m[2] = (float)m22;
        g.m[3] = (float)m31;
        g.m[4] = (float)m32;
        g.m[5] = (float)m33;
        s_q[tid] = g;
    }
    __syncthreads();
    if (!live) return;
    float x[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) x[q] = 0.f;
#pragma unroll(DC > 0 ? DC / 4 : 1)
    for (int d4 = 0; d4 < D / 4; ++d4) {
        const float4 f = DC > 0 ? pre[DC > 0 ? d4 : 0] : row[d4];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            if (q < Q) {
                const float4 w = *reinterpret_cast<const float4*>(fq + (int64_t)q * D + 4 * d4);
                x[q] = fmaf(f.x, w.x, x[q]);
                x[q] = fmaf(f.y, w.y, x[q]);
                x[q] = fmaf(f.z, w.z, x[q]);
                x[q] = fmaf(f.w, w.w, x[q]);
            }
        }
    }
    const float px = means[3 * i], py = means[3 * i + 1], pz = means[3 * i + 2];
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        if (q < Q) {
            const QueryGeom& g = s_q[q];
            const float dx = px - g.c[0], dy = py - g.c[1], dz = pz - g.c[2];
            const float y1 = g.m[0] * dx;
            const float y2 = fmaf(g.m[1], dx, g.m[2] * dy);
            const float y3 = fmaf(g.m[3], dx, fmaf(g.m[4], dy, g.m[5] * dz));
            const float m2 = fmaf(y1, y1, fmaf(y2, y2, y3 * y3));
            // hardware exp2 based exponentials (relative error about
            // |argument| 2^-24) and 1-ulp reciprocals: far below what the
            // fp32 dot product leaves
            const float sim = __builtin_amdgcn_rcpf(1.f + __expf(-x[q]));
            x[q] = __expf(sim * __expf(-0.5f * m2));   // A in [0, 1]: no max shift needed
            sum += x[q];
        }
    }
    const float r = __builtin_amdgcn_rcpf(sum);
    float* __restrict__ o = out + i * Q;
    if (Q % 4 == 0) {
#pragma unroll
        for (int q = 0; q < QMAX; q += 4)
            if (q < Q)
                *reinterpret_cast<float4*>(o + q) = make_float4(x[q] * r, x[q + 1] * r, x[q + 2] * r, x[q + 3] * r);
    } else {
#pragma unroll
        for (int q = 0; q < QMAX; ++q)
            if (q < Q) o[q] = x[q] * r;
    }
}

// Matrix-core form for Q = 32 queries and D = 32 (the paper's feature
// size): per wave two tiles of 32 Gaussians; v_mfma_f32_32x32x2f32 over pairs
// of feature dimensions forms each 32 x 32 block of dot products (rows =
// queries, columns = Gaussians), the dimensions split over two independent
// accumulators.  Lane l feeds query l % 32 and Gaussian l % 32 with
// dimensions 16 (l / 32) + s (the sum over dimensions is order-free), and
// gets back 16 queries of Gaussian l % 32: rows 8 g + 4 (l / 32) + r of
// register 4 g + r.  Both tiles' feature rows are loaded before the query
// set-up.  The two lanes holding a Gaussian's halves exchange their partial
// softmax sums once.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMfmaQ = 32;
constexpr int kMfmaD = 32;

__global__ void __launch_bounds__(kInstThreads)
instance_label_mfma_kernel(const float* __restrict__ fins, const float* __restrict__ means, int64_t n,
                           const float* __restrict__ fq, const float* __restrict__ qmeans,
                           const float* __restrict__ qcovs, float* __restrict__ out) {
    __shared__ QueryGeom s_q[kMfmaQ];
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, col = lane & 31;
    int64_t gi[2];
    float b[2][16];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        gi[t] = (int64_t)blockIdx.x * kInstThreads + wave * 64 + t * 32 + col;
        const int64_t gs = gi[t] < n ? gi[t] : 0;   // every lane takes part in the matrix ops
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const float4 v = *reinterpret_cast<const float4*>(fins + gs * kMfmaD + 16 * half + 4 * s4);
            b[t][4 * s4] = v.x;
            b[t][4 * s4 + 1] = v.y;
            b[t][4 * s4 + 2] = v.z;
            b[t][4 * s4 + 3] = v.w;
        }
    }
    float a[16];   // query col, dimensions 16 half + s
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
        const float4 v = *reinterpret_cast<const float4*>(fq + col * kMfmaD + 16 * half + 4 * s4);
        a[4 * s4] = v.x;
        a[4 * s4 + 1] = v.y;
        a[4 * s4 + 2] = v.z;
        a[4 * s4 + 3] = v.w;
    }
    if (tid < kMfmaQ) {
        const float* sc = qcovs + 6 * tid;   // xx, xy, xz, yy, yz, zz
        const double l11 = sqrt((double)sc[0]);
        const double l21 = sc[1] / l11, l31 = sc[2] / l11;
        const double l22 = sqrt(sc[3] - l21 * l21);
        const double l32 = (sc[4] - l31 * l21) / l22;
        const double l33 = sqrt(sc[5] - l31 * l31 - l32 * l32);
        const double m11 = 1.0 / l11, m22 = 1.0 / l22, m33 = 1.0 / l33;
        const double m21 = -l21 * m11 * m22;
        const double m32 = -l32 * m22 * m33;
        const double m31 = -(l31 * m11 + l32 * m21) * m33;
        QueryGeom g;
        g.c[0] = qmeans[3 * tid];
        g.c[1] = qmeans[3 * tid + 1];
        g.c[2] = qmeans[3 * tid + 2];
        g.m[0] = (float)m11;
        g.m[1] = (float)m21;
        g.m[2] = (float)m22;
        g.m[3] = (float)m31;
        g.m[4] = (float)m32;
        g.m[5] = (float)m33;
        s_q[tid] = g;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x16 acc0, acc1;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc0[v] = 0.f;
            acc1[v] = 0.f;
        }
#pragma unroll
        for (int s = 0; s < 16; s += 2) {
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[t][s], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s + 1], b[t][s + 1], acc1, 0, 0, 0);
        }
        const int64_t gs = gi[t] < n ? gi[t] : 0;
        const float px = means[3 * gs], py = means[3 * gs + 1], pz = means[3 * gs + 2];
        float e[16];
        float sum = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const QueryGeom& g = s_q[8 * (v >> 2) + 4 * half + (v & 3)];
            const float dx = px - g.c[0], dy = py - g.c[1], dz = pz - g.c[2];
            const float y1 = g.m[0] * dx;
            const float y2 = fmaf(g.m[1], dx, g.m[2] * dy);
            const float y3 = fmaf(g.m[3], dx, fmaf(g.m[4], dy, g.m[5] * dz));
            const float m2 = fmaf(y1, y1, fmaf(y2, y2, y3 * y3));
            const float sim = __builtin_amdgcn_rcpf(1.f + __expf(-(acc0[v] + acc1[v])));
            e[v] = __expf(sim * __expf(-0.5f * m2));
            sum += e[v];
        }
        sum += __shfl_xor(sum, 32, 64);   // the other 16 queries of this Gaussian
        const float r = __builtin_amdgcn_rcpf(sum);
        if (gi[t] < n) {
            float* __restrict__ o = out + gi[t] * kMfmaQ + 4 * half;
#pragma unroll
            for (int g = 0; g < 4; ++g)
                *reinterpret_cast<float4*>(o + 8 * g) =
                    make_float4(e[4 * g] * r, e[4 * g + 1] * r, e[4 * g + 2] * r, e[4 * g + 3] * r);
        }
    }
}

}  // namespace

hipError_t fs_launch_instance_labels(const float* fins, int D, const float* means, int64_t n, const float* fq,
                                     const float* qmeans, const float* qcovs, int Q, float* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + kInstThreads - 1) / kInstThreads;
    if (blocks >= (int64_t(1) << 31) || Q < 1 || Q > FS_MAX_QUERIES || D < 4 || D % 4 != 0)
        return hipErrorInvalidValue;
    if (Q == kMfmaQ && D == kMfmaD) {
        hipLaunchKernelGGL(instance_label_mfma_kernel, dim3((unsigned)blocks), dim3(kInstThreads), 0, s, fins, means,
                           n, fq, qmeans, qcovs, out);
        return hipGetLastError();
    }
#define FS_INST_D(QMAX, EXACT)                                                                                 \
    if (D == 32)                                                                                                  \
        hipLaunchKernelGGL((instance_label_kernel<QMAX, EXACT, 32>), dim3((unsigned)blocks), dim3(kInstThreads),  \
                           0, s, fins, D, means, n, fq, qmeans, qcovs, Q, out);                                  \
    else                                                                                                          \
        hipLaunchKernelGGL((instance_label_kernel<QMAX, EXACT, 0>), dim3((unsigned)blocks), dim3(kInstThreads),   \
                           0, s, fins, D, means, n, fq, qmeans, qcovs, Q, out)
#define FS_INST(QMAX)          \
    if (Q == QMAX) {           \
        FS_INST_D(QMAX, true); \
    } else {                   \
        FS_INST_D(QMAX, false); \
    }
    if (Q <= 8) {
        FS_INST(8);
    } else if (Q <= 16) {
        FS_INST(16);
    } else if (Q <= 32) {
        FS_INST(32);
    } else {
        FS_INST(64);
    }
#undef FS_INST
#undef FS_INST_D
    return hipGetLastError();
}
