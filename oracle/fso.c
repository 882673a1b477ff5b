/*
 * fso.c -- CPU oracle for the 2D Gaussian surfel feature rasterizer of
 * Fast-SegSim (arXiv 2604.10951).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference the GPU
 * path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header or constant table with the GPU library.
 *
 * Precision: every quantity is computed in double precision (inputs arrive as
 * doubles converted exactly from the float32 scene).  Compile with
 * -ffp-contract=off: the decisions that produce integers (depth key bits, cull
 * flags, pixel-in-footprint tests, hence tile sets) are evaluated with a fixed
 * operation order and no fused multiply-add, so that they are a pure function
 * of the inputs.
 *
 * What is computed, and where the paper defines it:
 *   - surfel frame from centre p, tangent scales (r_u, r_v) and tangent
 *     vectors t_u, t_v                                 Sec. 3.1, Eq. (1)
 *   - density f(u) = exp(-(u^2+v^2)/2), opacity o      Sec. 3.1
 *   - homogeneous tangent->screen matrix T with rows T1, T2, Tw, x' = T u
 *                                                      Sec. 3.2 (matrix T)
 *   - ray-splat intersection u(x): the tangent-plane point hit by pixel x's
 *     ray, here u ~ (T1 - x Tw) x (T2 - y Tw) = adj(T) (x, y, 1)
 *                                                      Sec. 3.1 (u_i(x))
 *   - front-to-back alpha blending over depth-sorted surfels  Sec. 3.1, Eq. (2)
 *   - Top-K hard selection: the blend restricted to K surfels chosen in depth
 *     order (first K accepted contributors, weight = transmittance)
 *                                                      Sec. 3.4, F_TopK
 *   - the screen conic A x^2 + 2Bxy + C y^2 + 2Dx + 2Ey + F <= 0 of the
 *     cutoff circle u^2+v^2 = k^2, used only to bound which pixels need to be
 *     tested                                           Sec. 3.2 (AccuTile)
 *   - tile sets: a tile holds a surfel iff some pixel of the tile passes the
 *     per-pixel footprint test (the exact result the precise tile
 *     intersection must reach)                         Sec. 3.2
 *   - the gradient of L = sum_p g_p . F_p by the chain rule (no paper
 *     passage: the paper trains through the renderer, Sec. 3.5)
 *   - the paper-literal tile assignment: the linearised projected covariance
 *     Sigma' of Sec. 3.2, read as J J^T with J the Jacobian of the perspective
 *     map at the tangent origin; a tile holds a surfel iff some pixel centre
 *     of the tile lies in (x - mu)^T Sigma'^-1 (x - mu) <= k^2
 *                                                      Sec. 3.2
 *   - pixel depth and normal outputs: blended depth of the ray-splat
 *     intersection point and blended surfel normal n = t_u x t_v (in camera
 *     space, facing the camera)                        Sec. 3.1, Eq. (2)
 *   - the 2D Gaussian splatting screen-space low-pass option: the response
 *     exp(-min(u^2 + v^2, 2 |x - mu|^2) / 2), mu the projected centre
 *     (a screen Gaussian of variance 1/2 px^2 that keeps sub-pixel surfels
 *     visible; not part of the paper, an option of the 2DGS renderer it
 *     builds on)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* camera packed as doubles: W, H, fx, fy, cx, cy, R (row-major 9), t (3), z_near */
enum { CW = 0, CH = 1, CFX = 2, CFY = 3, CCX = 4, CCY = 5, CR = 6, CT = 15, CZN = 18, CAM_LEN = 19 };

/* relative margin below which a threshold decision counts as ambiguous when
 * comparing against a float32 renderer */
#define AMBIG_REL 1e-5

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

static uint32_t float_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Rotation columns t_u, t_v of the (not necessarily unit) quaternion
 * q = (w, x, y, z): the textbook unit-quaternion matrix with the factor 2
 * replaced by 2/|q|^2, which equals normalising q first. */
static void tangent_frame(const double q[4], double f, double tu[3], double tv[3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    tu[0] = 1.0 - f * (y * y + z * z);
    tu[1] = f * (x * y + w * z);
    tu[2] = f * (x * z - w * y);
    tv[0] = f * (x * y - w * z);
    tv[1] = 1.0 - f * (x * x + z * z);
    tv[2] = f * (y * z + w * x);
}

/* Camera-space frame: U = r_u R_cw t_u, V = r_v R_cw t_v, pc = R_cw p + t. */
static void camera_frame(const double* cam, const double p[3], const double s[2], const double tu[3],
                         const double tv[3], double U[3], double V[3], double pc[3])
{
    const double* R = cam + CR;
    for (int r = 0; r < 3; ++r) {
        U[r] = s[0] * ((R[3 * r] * tu[0] + R[3 * r + 1] * tu[1]) + R[3 * r + 2] * tu[2]);
        V[r] = s[1] * ((R[3 * r] * tv[0] + R[3 * r + 1] * tv[1]) + R[3 * r + 2] * tv[2]);
        pc[r] = ((R[3 * r] * p[0] + R[3 * r + 1] * p[1]) + R[3 * r + 2] * p[2]) + cam[CT + r];
    }
}

/* T = K_int [U | V | pc]; rows T1, T2, Tw.  T row-major (9). */
static void screen_matrix(const double* cam, const double U[3], const double V[3], const double pc[3], double T[9])
{
    const double fx = cam[CFX], fy = cam[CFY], cx = cam[CCX], cy = cam[CCY];
    const double M0[3] = {U[0], V[0], pc[0]};
    const double M1[3] = {U[1], V[1], pc[1]};
    const double M2[3] = {U[2], V[2], pc[2]};
    for (int c = 0; c < 3; ++c) {
        T[c] = fx * M0[c] + cx * M2[c];
        T[3 + c] = fy * M1[c] + cy * M2[c];
        T[6 + c] = M2[c];
    }
}

/* H = adj(T) as a row-major 3x3 with h = H (x, y, 1):
 * columns T2 x Tw, Tw x T1, T1 x T2 (expansion of (T1 - x Tw) x (T2 - y Tw)). */
static void adjugate(const double T[9], double H[9])
{
    double cx_[3], cy_[3], c1[3];
    cross3(T + 3, T + 6, cx_);
    cross3(T + 6, T, cy_);
    cross3(T, T + 3, c1);
    for (int r = 0; r < 3; ++r) {
        H[3 * r] = cx_[r];
        H[3 * r + 1] = cy_[r];
        H[3 * r + 2] = c1[r];
    }
}

static int all_finite(const double* v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/*
 * Project one surfel.  Returns 1 if it survives culling.  Culling rules (the
 * paper states none; these keep the footprint a bounded ellipse in front of
 * the camera): non-finite input, |q| = 0, a non-positive scale, centre depth
 * <= z_near, o <= alpha_min, the cutoff disk reaching depth <= z_near, or the
 * surfel seen edge-on (|n . pc| <= 1e-6 |pc|).
 */
static int project_one(const double p[3], const double s[2], const double q[4], double o, const double* cam,
                       double alpha_min, uint32_t* zkey, double T[9], double H[9], double* k2out)
{
    *zkey = 0;
    if (!all_finite(p, 3) || !all_finite(s, 2) || !all_finite(q, 4) || !isfinite(o)) return 0;
    const double qq = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    if (!(qq > 0.0)) return 0;
    if (!(s[0] > 0.0) || !(s[1] > 0.0)) return 0;
    double tu[3], tv[3], U[3], V[3], pc[3];
    tangent_frame(q, 2.0 / qq, tu, tv);
    camera_frame(cam, p, s, tu, tv, U, V, pc);
    *zkey = float_bits((float)pc[2]);
    if (!(pc[2] > cam[CZN])) return 0;
    if (!(o > alpha_min)) return 0;
    const double k2 = 2.0 * log(o / alpha_min);
    const double dz = pc[2] - cam[CZN];
    if (dz * dz <= k2 * (U[2] * U[2] + V[2] * V[2])) return 0;
    double n[3];
    cross3(U, V, n);
    const double det = dot3(n, pc);
    if (det * det <= ((dot3(U, U) * dot3(V, V)) * dot3(pc, pc)) * 1e-12) return 0;
    screen_matrix(cam, U, V, pc, T);
    adjugate(T, H);
    *k2out = k2;
    return 1;
}

/* (u, v) of pixel centre (x, y) on the surfel's tangent plane, as d2 = u^2+v^2. */
static double pixel_d2(const double H[9], double x, double y, double* u, double* v)
{
    const double h0 = (H[0] * x + H[1] * y) + H[2];
    const double h1 = (H[3] * x + H[4] * y) + H[5];
    const double h2 = (H[6] * x + H[7] * y) + H[8];
    if (h2 == 0.0) {
        *u = *v = INFINITY;
        return INFINITY;
    }
    *u = h0 / h2;
    *v = h1 / h2;
    return (*u) * (*u) + (*v) * (*v);
}

/*
 * Axis-aligned bounds of the screen conic q(x, y) <= 0, where
 * q = h0^2 + h1^2 - k2 h2^2 = A x^2 + 2Bxy + C y^2 + 2Dx + 2Ey + F.
 * Returns 0 if the conic is not a bounded ellipse in floating point.
 */
static int conic_bounds(const double H[9], double k2, double bb[4])
{
    const double a0 = H[0], a1 = H[3], a2 = H[6];
    const double b0 = H[1], b1 = H[4], b2 = H[7];
    const double c0 = H[2], c1 = H[5], c2 = H[8];
    const double A = (a0 * a0 + a1 * a1) - k2 * (a2 * a2);
    const double B = (a0 * b0 + a1 * b1) - k2 * (a2 * b2);
    const double C = (b0 * b0 + b1 * b1) - k2 * (b2 * b2);
    const double D = (a0 * c0 + a1 * c1) - k2 * (a2 * c2);
    const double E = (b0 * c0 + b1 * c1) - k2 * (b2 * c2);
    const double F = (c0 * c0 + c1 * c1) - k2 * (c2 * c2);
    const double det = A * C - B * B;
    if (!(A > 0.0) || !(C > 0.0) || !(det > 0.0)) return 0;
    const double bx = B * E - C * D, by = B * D - A * E;
    double rx = bx * bx + det * (E * E - C * F);
    double ry = by * by + det * (D * D - A * F);
    if (!(rx >= 0.0)) rx = 0.0;
    if (!(ry >= 0.0)) ry = 0.0;
    bb[0] = (bx - sqrt(rx)) / det;
    bb[1] = (bx + sqrt(rx)) / det;
    bb[2] = (by - sqrt(ry)) / det;
    bb[3] = (by + sqrt(ry)) / det;
    return all_finite(bb, 4);
}

/* Pixel index range [lo, hi] whose centres may lie inside the footprint.
 * With prefilter != 0: the conic bounds widened by one pixel; otherwise the
 * whole image.  Returns 0 for an empty range. */
static int pixel_range(const double H[9], double k2, int W, int Hh, int prefilter, int r[4])
{
    r[0] = 0;
    r[1] = W - 1;
    r[2] = 0;
    r[3] = Hh - 1;
    double bb[4];
    if (prefilter && conic_bounds(H, k2, bb)) {
        const double lim = 4.0 * (double)(W > Hh ? W : Hh) + 8.0;
        for (int j = 0; j < 4; ++j) {
            if (bb[j] < -lim) bb[j] = -lim;
            if (bb[j] > lim) bb[j] = lim;
        }
        int x0 = (int)ceil(bb[0] - 0.5) - 1, x1 = (int)floor(bb[1] - 0.5) + 1;
        int y0 = (int)ceil(bb[2] - 0.5) - 1, y1 = (int)floor(bb[3] - 0.5) + 1;
        if (x0 > r[0]) r[0] = x0;
        if (x1 < r[1]) r[1] = x1;
        if (y0 > r[2]) r[2] = y0;
        if (y1 < r[3]) r[3] = y1;
    }
    return r[0] <= r[1] && r[2] <= r[3];
}

/* The projected centre mu = (T1 . e3, T2 . e3) / (Tw . e3), e3 = (0, 0, 1):
 * the image of the tangent origin under x' = T u (Sec. 3.2). */
static void projected_centre(const double T[9], double mu[2])
{
    mu[0] = T[2] / T[8];
    mu[1] = T[5] / T[8];
}

/*
 * The linearised projected covariance of Sec. 3.2.  The printed formula is
 * garbled; it is read as the local linearisation of the perspective map
 * x(u, v) = (T1 . (u, v, 1), T2 . (u, v, 1)) / (Tw . (u, v, 1)) at the tangent
 * origin: J_rc = (T_rc - mu_r T_wc) / T_w3 (r, c in {1, 2}) and Sigma' = J J^T
 * (the tangent coordinates have unit variance; the scales are inside T).
 * Outputs mu, Sigma' = (S00, S01, S11) and its inverse P = (P00, P01, P11).
 * Returns 0 if Sigma' is not positive definite in floating point.
 */
static int linearised_ellipse(const double T[9], double mu[2], double Sg[3], double P[3])
{
    projected_centre(T, mu);
    const double J00 = (T[0] - mu[0] * T[6]) / T[8];
    const double J01 = (T[1] - mu[0] * T[7]) / T[8];
    const double J10 = (T[3] - mu[1] * T[6]) / T[8];
    const double J11 = (T[4] - mu[1] * T[7]) / T[8];
    Sg[0] = J00 * J00 + J01 * J01;
    Sg[1] = J00 * J10 + J01 * J11;
    Sg[2] = J10 * J10 + J11 * J11;
    const double det = Sg[0] * Sg[2] - Sg[1] * Sg[1];
    if (!(det > 0.0) || !isfinite(det)) return 0;
    P[0] = Sg[2] / det;
    P[1] = -Sg[1] / det;
    P[2] = Sg[0] / det;
    return 1;
}

/* Mahalanobis distance (x - mu)^T Sigma'^-1 (x - mu) of point (x, y). */
static double linearised_q(const double mu[2], const double P[3], double x, double y)
{
    const double dx = x - mu[0], dy = y - mu[1];
    return (P[0] * dx * dx + 2.0 * P[1] * dx * dy) + P[2] * dy * dy;
}

/* Screen-space term of the low-pass option: 2 |x - mu|^2, i.e. the squared
 * distance to the projected centre in units of a standard deviation of
 * sqrt(1/2) px. */
static double lowpass_r2(const double mu[2], double x, double y)
{
    const double dx = x - mu[0], dy = y - mu[1];
    return 2.0 * (dx * dx + dy * dy);
}

/* Camera depth of the ray-splat intersection point p_c + u U + v V: its third
 * coordinate, Tw . (u, v, 1) (Tw = (U_z, V_z, p_c,z), the last row of T). */
static double intersection_depth(const double T[9], double u, double v)
{
    return (T[6] * u + T[7] * v) + T[8];
}

/* Pixel index range [lo, hi] of pixel centres with a continuous coordinate in
 * [c0, c1], widened by one pixel. */
static void centre_range(double c0, double c1, double lim, int* lo, int* hi)
{
    c0 = c0 < -lim ? -lim : (c0 > lim ? lim : c0);
    c1 = c1 < -lim ? -lim : (c1 > lim ? lim : c1);
    *lo = (int)ceil(c0 - 0.5) - 1;
    *hi = (int)floor(c1 - 0.5) + 1;
}

/* ------------------------------------------------------------------------ */
/* Exported: projection                                                      */
/* ------------------------------------------------------------------------ */

/* Project n surfels with one camera.  Outputs per surfel: valid flag, depth
 * key bits (float32 bits of the camera-space depth of the centre), T (9), H =
 * adj(T) (9) and the cutoff k2 = 2 ln(o / alpha_min). */
int fso_project(const double* means, const double* scales, const double* quats, const double* opacity, int64_t n,
                const double* cam, double alpha_min, int32_t* valid, uint32_t* zkey, double* T, double* H,
                double* k2)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double k = 0.0;
        valid[i] = project_one(means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i], cam, alpha_min, zkey + i,
                               T + 9 * i, H + 9 * i, &k);
        k2[i] = valid[i] ? k : 0.0;
        if (!valid[i]) {
            for (int j = 0; j < 9; ++j) T[9 * i + j] = H[9 * i + j] = 0.0;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exported: per-pixel footprint test and tile sets                          */
/* ------------------------------------------------------------------------ */

/* d2 = u^2 + v^2 at every pixel centre of a W x Hh image for one projected
 * surfel (row-major), for tests of the footprint definition. */
int fso_surfel_d2_image(const double* H, int W, int Hh, double* out)
{
    for (int py = 0; py < Hh; ++py)
        for (int px = 0; px < W; ++px) {
            double u, v;
            out[(int64_t)py * W + px] = pixel_d2(H, px + 0.5, py + 0.5, &u, &v);
        }
    return 0;
}

/* Pixel-centre bounds of the screen conic (x0, x1, y0, y1), 0 if none. */
int fso_conic_bounds(const double* H, double k2, double* bb) { return conic_bounds(H, k2, bb); }

/* Assignment modes of fso_tile_sets (the values of the library's tile modes). */
enum { ASSIGN_EXACT = 0, ASSIGN_LINEARISED = 2 };

/* Candidate pixel range of surfel i for a tile assignment: the union of the
 * closed-form bounds of every shape the assignment tests (the exact conic, or
 * the linearised ellipse, plus the low-pass disc), each widened by one pixel;
 * the whole image if prefilter == 0 or a shape is unbounded. */
static int assign_range(const double T[9], const double H[9], double k2, int mode, int lowpass, int W, int Hh,
                        int prefilter, int r[4])
{
    r[0] = 0;
    r[1] = W - 1;
    r[2] = 0;
    r[3] = Hh - 1;
    if (!prefilter) return 1;
    const double lim = 4.0 * (double)(W > Hh ? W : Hh) + 8.0;
    int lo[2] = {1 << 30, 1 << 30}, hi[2] = {-(1 << 30), -(1 << 30)};
    double bb[4];
    if (mode == ASSIGN_LINEARISED) {
        double mu[2], Sg[3], P[3];
        if (!linearised_ellipse(T, mu, Sg, P)) return 1;
        const double k = sqrt(k2);
        bb[0] = mu[0] - k * sqrt(Sg[0]);
        bb[1] = mu[0] + k * sqrt(Sg[0]);
        bb[2] = mu[1] - k * sqrt(Sg[2]);
        bb[3] = mu[1] + k * sqrt(Sg[2]);
        if (!all_finite(bb, 4)) return 1;
    } else if (!conic_bounds(H, k2, bb)) {
        return 1;
    }
    for (int a = 0; a < 2; ++a) {
        int l, h;
        centre_range(bb[2 * a], bb[2 * a + 1], lim, &l, &h);
        lo[a] = l < lo[a] ? l : lo[a];
        hi[a] = h > hi[a] ? h : hi[a];
    }
    if (lowpass) {
        double mu[2];
        projected_centre(T, mu);
        const double rd = sqrt(0.5 * k2);
        if (!isfinite(mu[0]) || !isfinite(mu[1])) return 1;
        for (int a = 0; a < 2; ++a) {
            int l, h;
            centre_range(mu[a] - rd, mu[a] + rd, lim, &l, &h);
            lo[a] = l < lo[a] ? l : lo[a];
            hi[a] = h > hi[a] ? h : hi[a];
        }
    }
    if (lo[0] > r[0]) r[0] = lo[0];
    if (hi[0] < r[1]) r[1] = hi[0];
    if (lo[1] > r[2]) r[2] = lo[1];
    if (hi[1] < r[3]) r[3] = hi[1];
    return r[0] <= r[1] && r[2] <= r[3];
}

/* Does pixel centre (x, y) assign surfel i to its tile?  exact: u^2 + v^2 <=
 * k2; linearised: the Sec. 3.2 ellipse; with lowpass, also 2 |x - mu|^2 <= k2.
 * *near = 1 if a decision taken lies within 1e-12 relative of k2. */
static int assigns(const double T[9], const double H[9], double k2, int mode, int lowpass, int lin_ok,
                   const double mu[2], const double P[3], double x, double y, int* near)
{
    double q;
    if (mode == ASSIGN_LINEARISED) {
        q = lin_ok ? linearised_q(mu, P, x, y) : INFINITY;
    } else {
        double u, v;
        q = pixel_d2(H, x, y, &u, &v);
    }
    if (fabs(q - k2) < 1e-12 * k2) *near = 1;
    int in = q <= k2;
    if (lowpass) {
        const double r2 = lowpass_r2(mu, x, y);
        if (fabs(r2 - k2) < 1e-12 * k2) *near = 1;
        in = in || r2 <= k2;
    }
    return in;
}

/*
 * Tile sets by the per-pixel definition: tile (tx, ty) holds surfel i iff some
 * pixel centre in the tile assigns it (assigns() above: the exact footprint
 * u^2 + v^2 <= k2 for mode ASSIGN_EXACT, the linearised ellipse of Sec. 3.2
 * for ASSIGN_LINEARISED, and with lowpass != 0 also the low-pass disc).
 * counts[i] = number of tiles.  If keys != NULL, pairs are written (in surfel
 * order, tiles row-major) at offsets[i] (exclusive prefix of counts, computed
 * here serially):
 *   key = ((tile_offset + ty * tiles_x + tx) << 32) | zkey[i],  value = val_offset + i.
 * flag[i] = 1 if any pixel test of surfel i had relative margin below 1e-12
 * (a decision floating point could flip).
 */
int64_t fso_tile_sets(const int32_t* valid, const uint32_t* zkey, const double* T, const double* H, const double* k2,
                      int64_t n, int W, int Hh, int S, int prefilter, int mode, int lowpass, int64_t tile_offset,
                      int64_t val_offset, uint32_t* counts, int8_t* flag, uint64_t* keys, uint32_t* vals)
{
    const int tx_n = (W + S - 1) / S, ty_n = (Hh + S - 1) / S;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    uint8_t* marks = (uint8_t*)calloc((size_t)nthreads * tx_n * ty_n, 1);
    if (!marks) return -1;
    for (int pass = 0; pass < (keys ? 2 : 1); ++pass) {
        int64_t* offsets = NULL;
        if (pass == 1) {
            offsets = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
            offsets[0] = 0;
            for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + counts[i];
        }
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            uint8_t* mk = marks + (size_t)tid * tx_n * ty_n;
            if (pass == 0) {
                counts[i] = 0;
                flag[i] = 0;
            }
            if (!valid[i]) continue;
            const double* Ti = T + 9 * i;
            const double* Hi = H + 9 * i;
            int r[4];
            if (!assign_range(Ti, Hi, k2[i], mode, lowpass, W, Hh, prefilter, r)) continue;
            double mu[2], Sg[3], P[3] = {0.0, 0.0, 0.0};
            int lin_ok = 0;
            if (mode == ASSIGN_LINEARISED)
                lin_ok = linearised_ellipse(Ti, mu, Sg, P);
            else
                projected_centre(Ti, mu);
            uint32_t cnt = 0;
            int fl = 0;
            for (int py = r[2]; py <= r[3]; ++py)
                for (int px = r[0]; px <= r[1]; ++px)
                    if (assigns(Ti, Hi, k2[i], mode, lowpass, lin_ok, mu, P, px + 0.5, py + 0.5, &fl))
                        mk[(py / S) * tx_n + px / S] = 1;
            int64_t o = pass == 1 ? offsets[i] : 0;
            for (int ty = r[2] / S; ty <= r[3] / S; ++ty)
                for (int tx = r[0] / S; tx <= r[1] / S; ++tx) {
                    uint8_t* m = mk + ty * tx_n + tx;
                    if (*m) {
                        if (pass == 1) {
                            keys[o] = ((uint64_t)(tile_offset + (int64_t)ty * tx_n + tx) << 32) | zkey[i];
                            vals[o] = (uint32_t)(val_offset + i);
                            ++o;
                        }
                        ++cnt;
                        *m = 0;
                    }
                }
            if (pass == 0) {
                counts[i] = cnt;
                flag[i] = (int8_t)fl;
            }
        }
        free(offsets);
    }
    free(marks);
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) total += counts[i];
    return total;
}

typedef struct {
    uint64_t key;
    uint32_t val;
} pair_t;

static int pair_cmp(const void* a, const void* b)
{
    const pair_t* x = (const pair_t*)a;
    const pair_t* y = (const pair_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->val != y->val) return x->val < y->val ? -1 : 1;
    return 0;
}

/* Sort (key, value) pairs lexicographically by (key, value), in place. */
int fso_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t m)
{
    pair_t* p = (pair_t*)malloc(sizeof(pair_t) * (m > 0 ? m : 1));
    if (!p) return -1;
    for (int64_t i = 0; i < m; ++i) {
        p[i].key = keys[i];
        p[i].val = vals[i];
    }
    qsort(p, (size_t)m, sizeof(pair_t), pair_cmp);
    for (int64_t i = 0; i < m; ++i) {
        keys[i] = p[i].key;
        vals[i] = p[i].val;
    }
    free(p);
    return 0;
}

/* [start, end) of every tile's run in a sorted pair list (tile = key >> 32). */
int fso_tile_ranges(const uint64_t* keys, int64_t m, int64_t num_tiles, uint32_t* ranges)
{
    for (int64_t t = 0; t < 2 * num_tiles; ++t) ranges[t] = 0;
    for (int64_t i = 0; i < m; ++i) {
        const int64_t t = (int64_t)(keys[i] >> 32);
        if (t < 0 || t >= num_tiles) return -1;
        if (i == 0 || (keys[i - 1] >> 32) != (uint64_t)t) ranges[2 * t] = (uint32_t)i;
        ranges[2 * t + 1] = (uint32_t)(i + 1);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Blending                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t zkey;
    uint32_t idx;
    double d2;   /* u^2 + v^2 (with the low-pass option: min(u^2 + v^2, 2 |x - mu|^2)) */
    double z;    /* camera depth of the ray-splat intersection point (0 if not needed) */
} cand_t;

/* Per-pixel geometry outputs of a blend: GEO_LEN doubles per pixel,
 * [depth, |depth| term sum, normal xyz, |normal| term sums xyz]. */
enum { GEO_LEN = 8 };

static int cand_cmp(const void* a, const void* b)
{
    const cand_t* x = (const cand_t*)a;
    const cand_t* y = (const cand_t*)b;
    if (x->zkey != y->zkey) return x->zkey < y->zkey ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

typedef struct {
    double alpha_min, alpha_max, t_stop;
    int K;      /* 0 = blend every accepted surfel; < 0: the -K of largest weight */
    int kcap;   /* capacity of the per-pixel index output */
} blend_opts;

static int blend_pixel_by_weight(const cand_t* cs, int64_t m, const double* k2, const double* opacity,
                                 const double* feats, int C, int K, const blend_opts* bo, double* F, double* absF,
                                 double* Tout, int32_t* idx, int32_t* amb, int32_t* nclamp, int32_t* last_cand,
                                 const double* normals, double* geo);

/* Adds one contributor (weight w, intersection depth z, normal nrm) to a
 * pixel's geometry outputs. */
static void geo_add(double* geo, double w, double z, const double* nrm)
{
    geo[0] += w * z;
    geo[1] += w * fabs(z);
    for (int k = 0; k < 3; ++k) {
        geo[2 + k] += w * nrm[k];
        geo[5 + k] += w * fabs(nrm[k]);
    }
}

/*
 * Front-to-back blend of one pixel over its candidates sorted by depth key
 * then index (Eq. 2; Top-K of Sec. 3.4 when K > 0):
 *   skip a surfel whose alpha is below alpha_min (u^2+v^2 > k2),
 *   stop before a surfel that would take transmittance below t_stop,
 *   w = alpha T;  F += w c;  T *= (1 - alpha);
 *   with K > 0, stop after the K-th blended surfel.
 * amb = 1 if a decision along the way lies within AMBIG_REL of its threshold.
 * Returns the number of blended surfels.
 */
static int blend_pixel(const cand_t* cs, int64_t m, const double* k2, const double* opacity, const double* feats,
                       int C, const blend_opts* bo, double* F, double* absF, double* Tout, int32_t* idx,
                       int32_t* amb, int32_t* nclamp, int32_t* last_cand, const double* normals, double* geo)
{
    if (geo)
        for (int k = 0; k < GEO_LEN; ++k) geo[k] = 0.0;
    if (bo->K < 0)
        return blend_pixel_by_weight(cs, m, k2, opacity, feats, C, -bo->K, bo, F, absF, Tout, idx, amb, nclamp,
                                     last_cand, normals, geo);
    double T = 1.0;
    int n = 0, a = 0, ncl = 0;
    int32_t lastc = -1;
    for (int c = 0; c < C; ++c) F[c] = absF[c] = 0.0;
    for (int j = 0; j < bo->kcap; ++j) idx[j] = -1;
    for (int64_t j = 0; j < m; ++j) {
        const uint32_t i = cs[j].idx;
        const double d2 = cs[j].d2;
        if (fabs(d2 - k2[i]) < AMBIG_REL * k2[i]) a = 1;
        if (!(d2 <= k2[i])) continue;
        const double G = exp(-0.5 * d2);
        double alpha = opacity[i] * G;
        if (alpha > bo->alpha_max) {
            alpha = bo->alpha_max;
            ++ncl;
        }
        const double Tn = T * (1.0 - alpha);
        if (fabs(Tn - bo->t_stop) < AMBIG_REL * bo->t_stop) a = 1;
        if (Tn < bo->t_stop) break;
        const double w = alpha * T;
        const double* c = feats + (int64_t)i * C;
        for (int ch = 0; ch < C; ++ch) {
            F[ch] += w * c[ch];
            absF[ch] += w * fabs(c[ch]);
        }
        if (geo) geo_add(geo, w, cs[j].z, normals + 3 * (int64_t)i);
        T = Tn;
        if (n < bo->kcap) idx[n] = (int32_t)i;
        ++n;
        lastc = (int32_t)j;
        if (bo->K > 0 && n == bo->K) break;
    }
    *Tout = T;
    *amb = a;
    *nclamp = ncl;
    *last_cand = lastc;
    return n;
}

typedef struct {
    double w;
    int64_t j;
    uint32_t i;
} sel_t;

static int weight_cmp(const void* a, const void* b)
{
    const sel_t* x = (const sel_t*)a;
    const sel_t* y = (const sel_t*)b;
    if (x->w != y->w) return x->w > y->w ? -1 : 1;   /* larger weight first */
    return x->j < y->j ? -1 : (x->j > y->j ? 1 : 0);  /* then the front one */
}

static int position_cmp(const void* a, const void* b)
{
    const sel_t* x = (const sel_t*)a;
    const sel_t* y = (const sel_t*)b;
    return x->j < y->j ? -1 : (x->j > y->j ? 1 : 0);
}

/*
 * Top-K by weight (the alternative reading of Sec. 3.4): the whole
 * front-to-back walk of blend_pixel without the K cutoff gives every
 * contributor's weight w = alpha T and the final transmittance; the K
 * contributors with the largest w (equal weights: the front one first) are
 * blended, front to back, with those weights.  T_final is the walk's.
 * amb also flags a K-th and (K+1)-th weight within AMBIG_REL of each other.
 */
static int blend_pixel_by_weight(const cand_t* cs, int64_t m, const double* k2, const double* opacity,
                                 const double* feats, int C, int K, const blend_opts* bo, double* F, double* absF,
                                 double* Tout, int32_t* idx, int32_t* amb, int32_t* nclamp, int32_t* last_cand,
                                 const double* normals, double* geo)
{
    double T = 1.0;
    int a = 0, ncl = 0;
    int32_t lastc = -1;
    sel_t* ws = (sel_t*)malloc(sizeof(sel_t) * (size_t)(m > 0 ? m : 1));
    int64_t nb = 0;
    for (int c = 0; c < C; ++c) F[c] = absF[c] = 0.0;
    for (int j = 0; j < bo->kcap; ++j) idx[j] = -1;
    for (int64_t j = 0; j < m; ++j) {
        const uint32_t i = cs[j].idx;
        const double d2 = cs[j].d2;
        if (fabs(d2 - k2[i]) < AMBIG_REL * k2[i]) a = 1;
        if (!(d2 <= k2[i])) continue;
        double alpha = opacity[i] * exp(-0.5 * d2);
        if (alpha > bo->alpha_max) {
            alpha = bo->alpha_max;
            ++ncl;
        }
        const double Tn = T * (1.0 - alpha);
        if (fabs(Tn - bo->t_stop) < AMBIG_REL * bo->t_stop) a = 1;
        if (Tn < bo->t_stop) break;
        ws[nb].w = alpha * T;
        ws[nb].j = j;
        ws[nb].i = i;
        ++nb;
        T = Tn;
        lastc = (int32_t)j;
    }
    qsort(ws, (size_t)nb, sizeof(sel_t), weight_cmp);
    const int64_t ns = nb < K ? nb : K;
    if (nb > K && fabs(ws[K - 1].w - ws[K].w) < AMBIG_REL * ws[K - 1].w) a = 1;
    qsort(ws, (size_t)ns, sizeof(sel_t), position_cmp);
    for (int64_t s = 0; s < ns; ++s) {
        const double* c = feats + (int64_t)ws[s].i * C;
        for (int ch = 0; ch < C; ++ch) {
            F[ch] += ws[s].w * c[ch];
            absF[ch] += ws[s].w * fabs(c[ch]);
        }
        if (geo) geo_add(geo, ws[s].w, cs[ws[s].j].z, normals + 3 * (int64_t)ws[s].i);
        if (s < bo->kcap) idx[s] = (int32_t)ws[s].i;
    }
    free(ws);
    *Tout = T;
    *amb = a;
    *nclamp = ncl;
    *last_cand = lastc;
    return (int)ns;
}

/* Candidate test: every surfel whose d2 is within AMBIG_REL above k2 is kept
 * (it either passes, or it is a near miss that makes the pixel ambiguous). */
static int is_candidate(double d2, double k2) { return d2 <= k2 * (1.0 + AMBIG_REL); }

/*
 * Render a list of pixels by brute force: for each pixel every valid surfel is
 * tested, candidates are sorted by (depth key, index), then blended.
 * pix[j] = py * W + px.  Outputs per listed pixel: F (C), absF (C: sum of
 * w |c|, the scale of the rounding error of F), T_final, n, idx (kcap, -1
 * padded), amb, nclamp.
 */
int fso_render_pixels(const int32_t* valid, const uint32_t* zkey, const double* T, const double* H, const double* k2,
                      const double* opacity, const double* feats, const double* normals, int64_t n, int C, int W,
                      const int64_t* pix, int64_t npix, int lowpass, double alpha_min, double alpha_max,
                      double t_stop, int K, int kcap, double* F, double* absF, double* Tout, int32_t* nout,
                      int32_t* idx, int32_t* amb, int32_t* nclamp, double* geo)
{
    (void)alpha_min;
    blend_opts bo = {alpha_min, alpha_max, t_stop, K, kcap};
    int status = 0;
#pragma omp parallel
    {
        int64_t cap = 256;
        cand_t* cs = (cand_t*)malloc(sizeof(cand_t) * cap);
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < npix; ++j) {
            const double x = (double)(pix[j] % W) + 0.5, y = (double)(pix[j] / W) + 0.5;
            int64_t m = 0;
            for (int64_t i = 0; i < n; ++i) {
                if (!valid[i]) continue;
                double u, v;
                double d2 = pixel_d2(H + 9 * i, x, y, &u, &v);
                if (lowpass) {
                    double mu[2];
                    projected_centre(T + 9 * i, mu);
                    const double r2 = lowpass_r2(mu, x, y);
                    d2 = r2 < d2 ? r2 : d2;
                }
                if (!is_candidate(d2, k2[i])) continue;
                if (m == cap) {
                    cap *= 2;
                    cs = (cand_t*)realloc(cs, sizeof(cand_t) * cap);
                }
                cs[m].zkey = zkey[i];
                cs[m].idx = (uint32_t)i;
                cs[m].d2 = d2;
                cs[m].z = geo ? intersection_depth(T + 9 * i, u, v) : 0.0;
                ++m;
            }
            qsort(cs, (size_t)m, sizeof(cand_t), cand_cmp);
            int32_t lc;
            nout[j] = blend_pixel(cs, m, k2, opacity, feats, C, &bo, F + j * C, absF + j * C, Tout + j,
                                  idx + j * kcap, amb + j, nclamp + j, &lc, normals, geo ? geo + j * GEO_LEN : NULL);
        }
        free(cs);
    }
    return status;
}

/*
 * Render pixels from sorted tile lists: pixel (px, py) walks the list of its
 * tile, vals[ranges[2t] .. ranges[2t+1]), t = (py / S) * tiles_x + px / S, in
 * list order (tile, depth key, index), and blends it as blend_pixel does.
 * This is the tiled form of Eq. (2): a surfel missing from a tile's list is
 * never blended there, which is how a tile assignment that misses pixels of a
 * footprint (the linearised one of Sec. 3.2) changes the image.  With lowpass,
 * the response is exp(-min(u^2 + v^2, 2 |x - mu|^2) / 2).  pix = NULL renders
 * every pixel in row-major order; otherwise pix[j] = py * W + px.  geo (NULL
 * or GEO_LEN doubles per pixel) receives depth and normal outputs, normals
 * holding 3 doubles per surfel.  Returns -1 if a list names a surfel >= n.
 */
int fso_render_lists(const int32_t* valid, const uint32_t* zkey, const double* T, const double* H, const double* k2,
                     const double* opacity, const double* feats, const double* normals, int64_t n, int C, int W,
                     int Hh, int S, const uint32_t* vals, const uint32_t* ranges, const int64_t* pix, int64_t npix,
                     int lowpass, double alpha_min, double alpha_max, double t_stop, int K, int kcap, double* F,
                     double* absF, double* Tout, int32_t* nout, int32_t* idx, int32_t* amb, int32_t* nclamp,
                     double* geo)
{
    const int tx_n = (W + S - 1) / S;
    const int64_t m_pix = pix ? npix : (int64_t)W * Hh;
    blend_opts bo = {alpha_min, alpha_max, t_stop, K, kcap};
    int status = 0;
#pragma omp parallel
    {
        int64_t cap = 256;
        cand_t* cs = (cand_t*)malloc(sizeof(cand_t) * cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t j = 0; j < m_pix; ++j) {
            const int64_t p = pix ? pix[j] : j;
            const int px = (int)(p % W), py = (int)(p / W);
            const double x = px + 0.5, y = py + 0.5;
            const int64_t t = (int64_t)(py / S) * tx_n + px / S;
            const uint32_t e0 = ranges[2 * t], e1 = ranges[2 * t + 1];
            int64_t m = 0;
            for (uint32_t e = e0; e < e1; ++e) {
                const uint32_t i = vals[e];
                if ((int64_t)i >= n || !valid[i]) {
#pragma omp atomic write
                    status = -1;
                    continue;
                }
                double u, v;
                double d2 = pixel_d2(H + 9 * (int64_t)i, x, y, &u, &v);
                if (lowpass) {
                    double mu[2];
                    projected_centre(T + 9 * (int64_t)i, mu);
                    const double r2 = lowpass_r2(mu, x, y);
                    d2 = r2 < d2 ? r2 : d2;
                }
                if (m == cap) {
                    cap *= 2;
                    cs = (cand_t*)realloc(cs, sizeof(cand_t) * cap);
                }
                cs[m].zkey = zkey[i];
                cs[m].idx = i;
                cs[m].d2 = d2;
                cs[m].z = geo ? intersection_depth(T + 9 * (int64_t)i, u, v) : 0.0;
                ++m;
            }
            int32_t lc;
            nout[j] = blend_pixel(cs, m, k2, opacity, feats, C, &bo, F + j * C, absF + j * C, Tout + j,
                                  idx + j * kcap, amb + j, nclamp + j, &lc, normals, geo ? geo + j * GEO_LEN : NULL);
        }
        free(cs);
    }
    return status;
}

/*
 * Surfel normals (Sec. 3.1: n = t_u x t_v, the cross product of the tangent
 * vectors), rotated into camera space (n_c = R n, scaled to unit length: the
 * camera rotation arrives in float32 and is orthonormal only to ~1e-7) and
 * flipped where needed so that they face the camera (n_c . p_c <= 0).  Zero
 * for a zero quaternion or non-finite input.  out: 3 doubles per surfel.
 */
int fso_normals(const double* means, const double* quats, int64_t n, const double* cam, double* out)
{
    const double* R = cam + CR;
    for (int64_t i = 0; i < n; ++i) {
        const double* q = quats + 4 * i;
        const double* p = means + 3 * i;
        double* o = out + 3 * i;
        o[0] = o[1] = o[2] = 0.0;
        if (!all_finite(q, 4) || !all_finite(p, 3)) continue;
        const double qq = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
        if (!(qq > 0.0)) continue;
        double tu[3], tv[3], nw[3], nc[3], pc[3];
        tangent_frame(q, 2.0 / qq, tu, tv);
        cross3(tu, tv, nw);
        for (int r = 0; r < 3; ++r) {
            nc[r] = (R[3 * r] * nw[0] + R[3 * r + 1] * nw[1]) + R[3 * r + 2] * nw[2];
            pc[r] = ((R[3 * r] * p[0] + R[3 * r + 1] * p[1]) + R[3 * r + 2] * p[2]) + cam[CT + r];
        }
        const double len = sqrt(dot3(nc, nc));
        const double sgn = dot3(nc, pc) > 0.0 ? -1.0 : 1.0;
        for (int r = 0; r < 3; ++r) o[r] = sgn * nc[r] / len;
    }
    return 0;
}

/*
 * Render a whole W x Hh image.  Candidate lists are built surfel by surfel
 * over each surfel's pixel range (conic bounds widened by one pixel when
 * prefilter != 0, else the whole image), then every pixel sorts its
 * candidates by (depth key, index) and blends them exactly as
 * fso_render_pixels does.  Outputs are per pixel, row-major, as there.
 */
int fso_render_image(const int32_t* valid, const uint32_t* zkey, const double* H, const double* k2,
                     const double* opacity, const double* feats, int64_t n, int C, int W, int Hh, int prefilter,
                     double alpha_min, double alpha_max, double t_stop, int K, int kcap, double* F, double* absF,
                     double* Tout, int32_t* nout, int32_t* idx, int32_t* amb, int32_t* nclamp)
{
    const int64_t npix = (int64_t)W * Hh;
    int64_t* start = (int64_t*)calloc((size_t)npix + 1, sizeof(int64_t));
    if (!start) return -1;
    /* pass 1: count candidates per pixel */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        if (!valid[i]) continue;
        int r[4];
        if (!pixel_range(H + 9 * i, k2[i], W, Hh, prefilter, r)) continue;
        for (int py = r[2]; py <= r[3]; ++py)
            for (int px = r[0]; px <= r[1]; ++px) {
                double u, v;
                const double d2 = pixel_d2(H + 9 * i, px + 0.5, py + 0.5, &u, &v);
                if (is_candidate(d2, k2[i])) {
#pragma omp atomic
                    start[(int64_t)py * W + px + 1] += 1;
                }
            }
    }
    for (int64_t p = 0; p < npix; ++p) start[p + 1] += start[p];
    const int64_t total = start[npix];
    cand_t* cs = (cand_t*)malloc(sizeof(cand_t) * (total > 0 ? total : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (npix > 0 ? npix : 1));
    if (!cs || !fill) {
        free(start);
        free(cs);
        free(fill);
        return -1;
    }
    for (int64_t p = 0; p < npix; ++p) fill[p] = start[p];
    /* pass 2: fill */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        if (!valid[i]) continue;
        int r[4];
        if (!pixel_range(H + 9 * i, k2[i], W, Hh, prefilter, r)) continue;
        for (int py = r[2]; py <= r[3]; ++py)
            for (int px = r[0]; px <= r[1]; ++px) {
                double u, v;
                const double d2 = pixel_d2(H + 9 * i, px + 0.5, py + 0.5, &u, &v);
                if (is_candidate(d2, k2[i])) {
                    int64_t slot;
#pragma omp atomic capture
                    slot = fill[(int64_t)py * W + px]++;
                    cs[slot].zkey = zkey[i];
                    cs[slot].idx = (uint32_t)i;
                    cs[slot].d2 = d2;
                    cs[slot].z = 0.0;
                }
            }
    }
    blend_opts bo = {alpha_min, alpha_max, t_stop, K, kcap};
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < npix; ++p) {
        const int64_t m = start[p + 1] - start[p];
        qsort(cs + start[p], (size_t)m, sizeof(cand_t), cand_cmp);
        int32_t lc;
        nout[p] = blend_pixel(cs + start[p], m, k2, opacity, feats, C, &bo, F + p * C, absF + p * C, Tout + p,
                              idx + p * kcap, amb + p, nclamp + p, &lc, NULL, NULL);
    }
    free(start);
    free(cs);
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gradient                                                                  */
/* ------------------------------------------------------------------------ */

/*
 * Chain dL/dH (H = adj(T), 3x3 row-major) of one surfel back to its
 * parameters: centre (3), scales (2), raw quaternion (4).
 * H columns: T2 x Tw, Tw x T1, T1 x T2.  For c = a x b: dL/da = b x g_c,
 * dL/db = g_c x a.  T = K_int [U | V | pc]; pc = R p + t; U = r_u R t_u;
 * V = r_v R t_v; t_u, t_v from q with factor f = 2/|q|^2.
 */
static void chain_to_params(const double p[3], const double s[2], const double q[4], const double* cam,
                            const double dH[9], double gp[3], double gs[2], double gq[4])
{
    const double qq = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    const double f = 2.0 / qq;
    double tu[3], tv[3], U[3], V[3], pc[3], T[9];
    tangent_frame(q, f, tu, tv);
    camera_frame(cam, p, s, tu, tv, U, V, pc);
    screen_matrix(cam, U, V, pc, T);
    const double* T1 = T;
    const double* T2 = T + 3;
    const double* Tw = T + 6;
    double gx[3], gy[3], g1[3];
    for (int r = 0; r < 3; ++r) {
        gx[r] = dH[3 * r];
        gy[r] = dH[3 * r + 1];
        g1[r] = dH[3 * r + 2];
    }
    double dT1[3] = {0, 0, 0}, dT2[3] = {0, 0, 0}, dTw[3] = {0, 0, 0}, t[3];
    /* col_x = T2 x Tw */
    cross3(Tw, gx, t);
    for (int k = 0; k < 3; ++k) dT2[k] += t[k];
    cross3(gx, T2, t);
    for (int k = 0; k < 3; ++k) dTw[k] += t[k];
    /* col_y = Tw x T1 */
    cross3(T1, gy, t);
    for (int k = 0; k < 3; ++k) dTw[k] += t[k];
    cross3(gy, Tw, t);
    for (int k = 0; k < 3; ++k) dT1[k] += t[k];
    /* col_1 = T1 x T2 */
    cross3(T2, g1, t);
    for (int k = 0; k < 3; ++k) dT1[k] += t[k];
    cross3(g1, T1, t);
    for (int k = 0; k < 3; ++k) dT2[k] += t[k];
    /* T rows: T1 = fx M0 + cx M2, T2 = fy M1 + cy M2, Tw = M2 */
    double dM[3][3];
    for (int c = 0; c < 3; ++c) {
        dM[0][c] = cam[CFX] * dT1[c];
        dM[1][c] = cam[CFY] * dT2[c];
        dM[2][c] = cam[CCX] * dT1[c] + cam[CCY] * dT2[c] + dTw[c];
    }
    const double dU[3] = {dM[0][0], dM[1][0], dM[2][0]};
    const double dV[3] = {dM[0][1], dM[1][1], dM[2][1]};
    const double dpc[3] = {dM[0][2], dM[1][2], dM[2][2]};
    const double* R = cam + CR;
    double Rtu[3], Rtv[3], dtu[3], dtv[3];
    for (int r = 0; r < 3; ++r) {
        Rtu[r] = R[3 * r] * tu[0] + R[3 * r + 1] * tu[1] + R[3 * r + 2] * tu[2];
        Rtv[r] = R[3 * r] * tv[0] + R[3 * r + 1] * tv[1] + R[3 * r + 2] * tv[2];
    }
    for (int k = 0; k < 3; ++k) {
        gp[k] = R[k] * dpc[0] + R[3 + k] * dpc[1] + R[6 + k] * dpc[2];
        dtu[k] = s[0] * (R[k] * dU[0] + R[3 + k] * dU[1] + R[6 + k] * dU[2]);
        dtv[k] = s[1] * (R[k] * dV[0] + R[3 + k] * dV[1] + R[6 + k] * dV[2]);
    }
    gs[0] = dot3(Rtu, dU);
    gs[1] = dot3(Rtv, dV);
    /* t_u = (1 - f a1, f a2, f a3), t_v = (f b1, 1 - f b2, f b3) */
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double a1 = y * y + z * z, a2 = x * y + w * z, a3 = x * z - w * y;
    const double b1 = x * y - w * z, b2 = x * x + z * z, b3 = y * z + w * x;
    const double sum_f = -dtu[0] * a1 + dtu[1] * a2 + dtu[2] * a3 + dtv[0] * b1 - dtv[1] * b2 + dtv[2] * b3;
    /* partial derivatives of a1..b3 w.r.t. (w, x, y, z) */
    const double da1[4] = {0, 0, 2 * y, 2 * z};
    const double da2[4] = {z, y, x, w};
    const double da3[4] = {-y, z, -w, x};
    const double db1[4] = {-z, y, x, -w};
    const double db2[4] = {0, 2 * x, 0, 2 * z};
    const double db3[4] = {x, w, z, y};
    for (int k = 0; k < 4; ++k) {
        const double dfk = -f * f * q[k];
        const double inner = -dtu[0] * da1[k] + dtu[1] * da2[k] + dtu[2] * da3[k] + dtv[0] * db1[k] -
                             dtv[1] * db2[k] + dtv[2] * db3[k];
        gq[k] = dfk * sum_f + f * inner;
    }
}

/*
 * Gradient of L = sum over pixels p and channels c of g[p, c] * F[p, c] for a
 * whole W x Hh image, with the blend's discrete choices (which surfels are
 * accepted, where each pixel stops, the Top-K set, the alpha clamp) held
 * fixed.  Per pixel, contributors m = 1..n front to back with weights
 * w_m = alpha_m T_m:
 *   dL/dc_m      = w_m g
 *   dL/dalpha_m  = T_m (g . c_m) - (sum_{l > m} w_l g . c_l) / (1 - alpha_m)
 *   alpha = o G unless clamped; G = exp(-d2/2); d2 = (h0^2 + h1^2) / h2^2.
 * Outputs: grads w.r.t. means (N x 3), scales (N x 2), raw quaternions
 * (N x 4), opacity (N) and features (N x C).  g is (Hh*W) x C.
 */
int fso_render_grad(const double* means, const double* scales, const double* quats, const double* opacity,
                    const double* feats, int64_t n, int C, const double* cam, int prefilter, double alpha_min,
                    double alpha_max, double t_stop, int K, const double* g, double* gmeans, double* gscales,
                    double* gquats, double* gopac, double* gfeats, double* amean, double* ascale, double* aquat,
                    double* aopac, double* afeat)
{
    /* a* (optional, all or none): sums of the absolute values of the terms
     * each gradient is made of -- per (pixel, contributor) for opacity and
     * features; for centre, scales and quaternion |J| sum_p |dH_p|, with J
     * the (linear) map from dL/dH to the parameters -- the scale against
     * which the rounding error of a float32 gradient is judged. */
    const int want_abs = amean != NULL;
    const int W = (int)cam[CW], Hh = (int)cam[CH];
    int32_t* valid = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    uint32_t* zkey = (uint32_t*)malloc(sizeof(uint32_t) * (n > 0 ? n : 1));
    double* T = (double*)malloc(sizeof(double) * 9 * (n > 0 ? n : 1));
    double* H = (double*)malloc(sizeof(double) * 9 * (n > 0 ? n : 1));
    double* k2 = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
    double* dH = (double*)calloc((size_t)9 * (n > 0 ? n : 1), sizeof(double));
    double* dHa = want_abs ? (double*)calloc((size_t)9 * (n > 0 ? n : 1), sizeof(double)) : NULL;
    if (!valid || !zkey || !T || !H || !k2 || !dH || (want_abs && !dHa)) return -1;
    fso_project(means, scales, quats, opacity, n, cam, alpha_min, valid, zkey, T, H, k2);
    for (int64_t i = 0; i < n; ++i) {
        gopac[i] = 0.0;
        for (int c = 0; c < C; ++c) gfeats[i * C + c] = 0.0;
        if (want_abs) {
            aopac[i] = 0.0;
            for (int c = 0; c < C; ++c) afeat[i * C + c] = 0.0;
        }
    }
    const int64_t npix = (int64_t)W * Hh;
    /* candidate lists, built as in fso_render_image */
    int64_t* start = (int64_t*)calloc((size_t)npix + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        if (!valid[i]) continue;
        int r[4];
        if (!pixel_range(H + 9 * i, k2[i], W, Hh, prefilter, r)) continue;
        for (int py = r[2]; py <= r[3]; ++py)
            for (int px = r[0]; px <= r[1]; ++px) {
                double u, v;
                if (pixel_d2(H + 9 * i, px + 0.5, py + 0.5, &u, &v) <= k2[i]) start[(int64_t)py * W + px + 1]++;
            }
    }
    for (int64_t p = 0; p < npix; ++p) start[p + 1] += start[p];
    cand_t* cs = (cand_t*)malloc(sizeof(cand_t) * (start[npix] > 0 ? start[npix] : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (npix > 0 ? npix : 1));
    for (int64_t p = 0; p < npix; ++p) fill[p] = start[p];
    for (int64_t i = 0; i < n; ++i) {
        if (!valid[i]) continue;
        int r[4];
        if (!pixel_range(H + 9 * i, k2[i], W, Hh, prefilter, r)) continue;
        for (int py = r[2]; py <= r[3]; ++py)
            for (int px = r[0]; px <= r[1]; ++px) {
                double u, v;
                const double d2 = pixel_d2(H + 9 * i, px + 0.5, py + 0.5, &u, &v);
                if (d2 <= k2[i]) {
                    const int64_t slot = fill[(int64_t)py * W + px]++;
                    cs[slot].zkey = zkey[i];
                    cs[slot].idx = (uint32_t)i;
                    cs[slot].d2 = d2;
                }
            }
    }
    int64_t mmax = 1;
    for (int64_t p = 0; p < npix; ++p)
        if (start[p + 1] - start[p] > mmax) mmax = start[p + 1] - start[p];
    double* wts = (double*)malloc(sizeof(double) * mmax);
    double* alphas = (double*)malloc(sizeof(double) * mmax);
    double* Ts = (double*)malloc(sizeof(double) * mmax);
    double* gc = (double*)malloc(sizeof(double) * mmax);
    double* gca = (double*)malloc(sizeof(double) * mmax);   /* sum_ch |g_ch c_ch| */
    int* clamped = (int*)malloc(sizeof(int) * mmax);
    uint32_t* who = (uint32_t*)malloc(sizeof(uint32_t) * mmax);
    double* d2s = (double*)malloc(sizeof(double) * mmax);
    for (int64_t p = 0; p < npix; ++p) {
        const int64_t m = start[p + 1] - start[p];
        cand_t* c = cs + start[p];
        qsort(c, (size_t)m, sizeof(cand_t), cand_cmp);
        const double* gp = g + p * C;
        /* forward walk: the same decisions as blend_pixel */
        double Tcur = 1.0;
        int nc = 0;
        for (int64_t j = 0; j < m; ++j) {
            const uint32_t i = c[j].idx;
            const double G = exp(-0.5 * c[j].d2);
            double alpha = opacity[i] * G;
            int cl = 0;
            if (alpha > alpha_max) {
                alpha = alpha_max;
                cl = 1;
            }
            const double Tn = Tcur * (1.0 - alpha);
            if (Tn < t_stop) break;
            who[nc] = i;
            alphas[nc] = alpha;
            Ts[nc] = Tcur;
            wts[nc] = alpha * Tcur;
            clamped[nc] = cl;
            d2s[nc] = c[j].d2;
            double dotc = 0.0, dota = 0.0;
            for (int ch = 0; ch < C; ++ch) {
                dotc += gp[ch] * feats[(int64_t)i * C + ch];
                dota += fabs(gp[ch] * feats[(int64_t)i * C + ch]);
            }
            gc[nc] = dotc;
            gca[nc] = dota;
            ++nc;
            Tcur = Tn;
            if (K > 0 && nc == K) break;
        }
        /* backward: suffix sums of w_l (g . c_l); with want_abs the same chain
           on absolute values (|g_ch c_ch| summed over channels, so the scale
           covers the rounding of the channel sums too) */
        double suffix = 0.0, suffix_a = 0.0;
        const double x = (double)(p % W) + 0.5, y = (double)(p / W) + 0.5;
        for (int j = nc - 1; j >= 0; --j) {
            const uint32_t i = who[j];
            for (int ch = 0; ch < C; ++ch) gfeats[(int64_t)i * C + ch] += wts[j] * gp[ch];
            if (want_abs)
                for (int ch = 0; ch < C; ++ch) afeat[(int64_t)i * C + ch] += wts[j] * fabs(gp[ch]);
            const double dalpha = Ts[j] * gc[j] - suffix / (1.0 - alphas[j]);
            const double dalpha_a = Ts[j] * gca[j] + suffix_a / (1.0 - alphas[j]);
            suffix += wts[j] * gc[j];
            suffix_a += wts[j] * gca[j];
            if (clamped[j]) continue;
            const double G = exp(-0.5 * d2s[j]);
            gopac[i] += G * dalpha;
            if (want_abs) aopac[i] += G * dalpha_a;
            const double dG = opacity[i] * dalpha;
            const double dd2 = -0.5 * G * dG;
            const double dd2_a = 0.5 * G * opacity[i] * dalpha_a;
            const double* Hi = H + 9 * i;
            const double h0 = (Hi[0] * x + Hi[1] * y) + Hi[2];
            const double h1 = (Hi[3] * x + Hi[4] * y) + Hi[5];
            const double h2 = (Hi[6] * x + Hi[7] * y) + Hi[8];
            const double u = h0 / h2, v = h1 / h2;
            const double du = 2.0 * u * dd2, dv = 2.0 * v * dd2;
            const double dh[3] = {du / h2, dv / h2, -(u * du + v * dv) / h2};
            const double xv[3] = {x, y, 1.0};
            const double dua = 2.0 * fabs(u) * dd2_a, dva = 2.0 * fabs(v) * dd2_a, ah2 = fabs(h2);
            const double dha[3] = {dua / ah2, dva / ah2, (fabs(u) * dua + fabs(v) * dva) / ah2};
            for (int r = 0; r < 3; ++r)
                for (int k = 0; k < 3; ++k) {
                    dH[9 * i + 3 * r + k] += dh[r] * xv[k];
                    if (want_abs) dHa[9 * i + 3 * r + k] += dha[r] * fabs(xv[k]);
                }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) gmeans[3 * i + k] = 0.0;
        gscales[2 * i] = gscales[2 * i + 1] = 0.0;
        for (int k = 0; k < 4; ++k) gquats[4 * i + k] = 0.0;
        if (!valid[i]) continue;
        chain_to_params(means + 3 * i, scales + 2 * i, quats + 4 * i, cam, dH + 9 * i, gmeans + 3 * i,
                        gscales + 2 * i, gquats + 4 * i);
        if (want_abs) {
            for (int k = 0; k < 3; ++k) amean[3 * i + k] = 0.0;
            ascale[2 * i] = ascale[2 * i + 1] = 0.0;
            for (int k = 0; k < 4; ++k) aquat[4 * i + k] = 0.0;
            for (int col = 0; col < 9; ++col) {   /* |J| (sum_p |dH_p|), one column of J at a time */
                double e[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, jm[3], js[2], jq[4];
                e[col] = 1.0;
                chain_to_params(means + 3 * i, scales + 2 * i, quats + 4 * i, cam, e, jm, js, jq);
                const double y = dHa[9 * i + col];
                for (int k = 0; k < 3; ++k) amean[3 * i + k] += fabs(jm[k]) * y;
                for (int k = 0; k < 2; ++k) ascale[2 * i + k] += fabs(js[k]) * y;
                for (int k = 0; k < 4; ++k) aquat[4 * i + k] += fabs(jq[k]) * y;
            }
        }
    }
    if (want_abs)
        for (int64_t i = 0; i < n; ++i)
            if (!valid[i]) {
                for (int k = 0; k < 3; ++k) amean[3 * i + k] = 0.0;
                ascale[2 * i] = ascale[2 * i + 1] = 0.0;
                for (int k = 0; k < 4; ++k) aquat[4 * i + k] = 0.0;
            }
    free(dHa);
    free(valid);
    free(zkey);
    free(T);
    free(H);
    free(k2);
    free(dH);
    free(start);
    free(cs);
    free(fill);
    free(wts);
    free(alphas);
    free(Ts);
    free(gc);
    free(gca);
    free(clamped);
    free(who);
    free(d2s);
    return 0;
}
