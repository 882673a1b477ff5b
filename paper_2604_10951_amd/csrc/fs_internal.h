// fs_internal.h -- device-side definitions shared by the rasterizer kernels.
//
// Geometry (Sec. 3.1 Eq. 1, Sec. 3.2): a surfel with centre p, tangent scales
// (r_u, r_v) and tangent vectors t_u, t_v maps tangent coordinates u = (u, v, 1)
// to homogeneous screen coordinates x' = T u with T = K [U | V | p_c],
// U = r_u R t_u, V = r_v R t_v, p_c = R p + t (camera rows T1, T2, Tw).  The
// ray of pixel point (x, y) meets the tangent plane at u ~ (T1 - x Tw) x
// (T2 - y Tw) = adj(T) (x, y, 1), so (u, v) = (h0 / h2, h1 / h2) with
// h = adj(T) (x, y, 1).  A pixel is in a surfel's footprint iff
// u^2 + v^2 <= k^2 with k^2 = 2 ln(o / alpha_min), i.e. iff o f(u) >= alpha_min.
//
// Integer decisions (depth key, culling, footprint membership and therefore
// tile sets) are taken in double precision with a fixed evaluation order and
// no contraction (the library is built with -ffp-contract=off), so they are a
// pure function of the float32 inputs.  The blend itself runs in float32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fastsegsim.h"

#define FS_DEV __device__ __forceinline__

// ---------------------------------------------------------------------------
// Per (view, surfel) record written by preprocess, read by the renderers.
// Coefficients of h relative to an anchor pixel centre (ax + .5, ay + .5):
// h(px, py) = h_a + (px - ax) g_x + (py - ay) g_y, normalised so that h2 = 1 at
// the projected surfel centre.  They are kept in double precision: for thin or
// grazing surfels the short-axis coordinate u at a pixel L pixels from the
// anchor along the long axis is a cancellation of terms of size L |grad u|, so
// float32 coefficients would leave an absolute error of ~6e-8 L |grad u| in u.
// ---------------------------------------------------------------------------
struct __align__(16) FsRecord {
    double h0, h1, h2;          // h at the anchor
    double gx0, gx1, gx2;       // dh/dx
    double gy0, gy1, gy2;       // dh/dy
    double k2;                  // cutoff k^2 (-1: culled)
    float o;                    // opacity
    int16_t ax, ay;             // anchor pixel (view-local)
    int16_t x0, x1, y0, y1;     // pixel bounding box of the footprint, clamped (x0 > x1: empty)
};
static_assert(sizeof(FsRecord) == FS_RECORD_BYTES, "record size");

// ---------------------------------------------------------------------------
// Double-precision projection.  The evaluation order below is the one the
// depth key, culling and footprint decisions are defined with.
// ---------------------------------------------------------------------------
struct FsGeo {
    double H[9];      // adj(T), row-major: h = H (x, y, 1)
    double T[9];      // rows T1, T2, Tw
    double k2;        // cutoff
    double zc;        // camera depth of the centre
    uint32_t zkey;    // float32 bits of zc
};

FS_DEV void fs_cross(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

FS_DEV double fs_dot(const double a[3], const double b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

FS_DEV bool fs_finite(double x) { return __builtin_isfinite(x); }

// Tangent vectors t_u, t_v: columns 0 and 1 of the rotation of q = (w, x, y, z),
// with the textbook factor 2 replaced by f = 2 / |q|^2 (equal to normalising q).
FS_DEV void fs_tangents(double w, double x, double y, double z, double f, double tu[3], double tv[3]) {
    tu[0] = 1.0 - f * (y * y + z * z);
    tu[1] = f * (x * y + w * z);
    tu[2] = f * (x * z - w * y);
    tv[0] = f * (x * y - w * z);
    tv[1] = 1.0 - f * (x * x + z * z);
    tv[2] = f * (y * z + w * x);
}

struct FsFrame {
    double tu[3], tv[3], U[3], V[3], pc[3];
    double f;
};

// Camera-space frame of a surfel.  Returns false for non-finite input, a zero
// quaternion or a non-positive scale.
FS_DEV bool fs_frame(const float* pm, const float* ps, const float* pq, const fs_camera& cam, FsFrame& fr) {
    const double p0 = pm[0], p1 = pm[1], p2 = pm[2];
    const double s0 = ps[0], s1 = ps[1];
    const double w = pq[0], x = pq[1], y = pq[2], z = pq[3];
    if (!fs_finite(p0) || !fs_finite(p1) || !fs_finite(p2) || !fs_finite(s0) || !fs_finite(s1) || !fs_finite(w) ||
        !fs_finite(x) || !fs_finite(y) || !fs_finite(z))
        return false;
    const double qq = ((w * w + x * x) + y * y) + z * z;
    if (!(qq > 0.0)) return false;
    if (!(s0 > 0.0) || !(s1 > 0.0)) return false;
    fr.f = 2.0 / qq;
    fs_tangents(w, x, y, z, fr.f, fr.tu, fr.tv);
    const double p[3] = {p0, p1, p2};
    for (int r = 0; r < 3; ++r) {
        const double R0 = cam.R[3 * r], R1 = cam.R[3 * r + 1], R2 = cam.R[3 * r + 2];
        fr.U[r] = s0 * ((R0 * fr.tu[0] + R1 * fr.tu[1]) + R2 * fr.tu[2]);
        fr.V[r] = s1 * ((R0 * fr.tv[0] + R1 * fr.tv[1]) + R2 * fr.tv[2]);
        fr.pc[r] = ((R0 * p[0] + R1 * p[1]) + R2 * p[2]) + (double)cam.t[r];
    }
    return true;
}

// T = K [U | V | p_c] (rows T1, T2, Tw) and H = adj(T) with columns
// T2 x Tw, Tw x T1, T1 x T2.
FS_DEV void fs_screen(const fs_camera& cam, const FsFrame& fr, double T[9], double H[9]) {
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
    const double M0[3] = {fr.U[0], fr.V[0], fr.pc[0]};
    const double M1[3] = {fr.U[1], fr.V[1], fr.pc[1]};
    const double M2[3] = {fr.U[2], fr.V[2], fr.pc[2]};
    for (int c = 0; c < 3; ++c) {
        T[c] = fx * M0[c] + cx * M2[c];
        T[3 + c] = fy * M1[c] + cy * M2[c];
        T[6 + c] = M2[c];
    }
    double a[3], b[3], c1[3];
    fs_cross(T + 3, T + 6, a);
    fs_cross(T + 6, T, b);
    fs_cross(T, T + 3, c1);
    for (int r = 0; r < 3; ++r) {
        H[3 * r] = a[r];
        H[3 * r + 1] = b[r];
        H[3 * r + 2] = c1[r];
    }
}

// Full projection with culling: non-finite input, |q| = 0, scale <= 0, centre
// depth <= z_near, o <= alpha_min, cutoff disk reaching depth <= z_near, or
// edge-on (|n . p_c| <= 1e-6 |p_c|).
FS_DEV bool fs_project(const float* pm, const float* ps, const float* pq, float opac, const fs_camera& cam,
                       double alpha_min, FsGeo& g) {
    FsFrame fr;
    g.zkey = 0;
    g.k2 = -1.0;
    if (!fs_frame(pm, ps, pq, cam, fr)) return false;
    const double o = opac;
    if (!fs_finite(o)) return false;
    g.zc = fr.pc[2];
    g.zkey = __float_as_uint((float)fr.pc[2]);
    const double zn = cam.z_near;
    if (!(fr.pc[2] > zn)) return false;
    if (!(o > alpha_min)) return false;
    const double k2 = 2.0 * log(o / alpha_min);
    const double dz = fr.pc[2] - zn;
    if (dz * dz <= k2 * (fr.U[2] * fr.U[2] + fr.V[2] * fr.V[2])) return false;
    double nrm[3];
    fs_cross(fr.U, fr.V, nrm);
    const double det = fs_dot(nrm, fr.pc);
    if (det * det <= ((fs_dot(fr.U, fr.U) * fs_dot(fr.V, fr.V)) * fs_dot(fr.pc, fr.pc)) * 1e-12) return false;
    fs_screen(cam, fr, g.T, g.H);
    g.k2 = k2;
    return true;
}

// 1/x to ~1e-15 relative: the hardware seed (~2^-23) refined by two Newton
// steps (each doubles its bits).
FS_DEV double fs_rcp_approx(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// sqrt(x) (x >= 0) to ~1e-13 relative: the reciprocal square root seed
// (~2^-23) after one Newton step, times x.
FS_DEV double fs_sqrt_line(double x) {
    if (!(x > 0.0)) return 0.0;
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return x * y;
}

// The footprint predicate at pixel (px, py): u^2 + v^2 <= k^2 with
// (u, v) = (h0 / h2, h1 / h2), h = H (px + .5, py + .5, 1).
FS_DEV bool fs_pixel_in(const double H[9], double k2, int px, int py) {
    const double x = (double)px + 0.5, y = (double)py + 0.5;
    const double h0 = (H[0] * x + H[1] * y) + H[2];
    const double h1 = (H[3] * x + H[4] * y) + H[5];
    const double h2 = (H[6] * x + H[7] * y) + H[8];
    if (h2 == 0.0) return false;
    const double u = h0 / h2, v = h1 / h2;
    return u * u + v * v <= k2;
}

// ---------------------------------------------------------------------------
// Screen conic of the cutoff circle, relative to an anchor pixel centre:
// q(dx, dy) = A dx^2 + 2B dx dy + C dy^2 + 2D dx + 2E dy + F <= 0 with
// (x, y) = (ax + .5 + dx, ay + .5 + dy) -- the AccuTile quadratic of Sec. 3.2.
// ---------------------------------------------------------------------------
struct FsConic {
    double A, B, C, D, E, F;
    int ax, ay;
};

FS_DEV void fs_conic(const double H[9], double k2, int ax, int ay, FsConic& q) {
    const double xa = (double)ax + 0.5, ya = (double)ay + 0.5;
    const double a0 = H[0], a1 = H[3], a2 = H[6];
    const double b0 = H[1], b1 = H[4], b2 = H[7];
    const double c0 = (H[0] * xa + H[1] * ya) + H[2];
    const double c1 = (H[3] * xa + H[4] * ya) + H[5];
    const double c2 = (H[6] * xa + H[7] * ya) + H[8];
    q.A = (a0 * a0 + a1 * a1) - k2 * (a2 * a2);
    q.B = (a0 * b0 + a1 * b1) - k2 * (a2 * b2);
    q.C = (b0 * b0 + b1 * b1) - k2 * (b2 * b2);
    q.D = (a0 * c0 + a1 * c1) - k2 * (a2 * c2);
    q.E = (b0 * c0 + b1 * c1) - k2 * (b2 * c2);
    q.F = (c0 * c0 + c1 * c1) - k2 * (c2 * c2);
    q.ax = ax;
    q.ay = ay;
}

// Continuous extent of the ellipse (anchor-relative): dx in [x0, x1], dy in
// [y0, y1].  Returns false if the conic is not a bounded ellipse.
FS_DEV bool fs_conic_extent(const FsConic& q, double e[4]) {
    const double det = q.A * q.C - q.B * q.B;
    if (!(q.A > 0.0) || !(q.C > 0.0) || !(det > 0.0)) return false;
    const double bx = q.B * q.E - q.C * q.D, by = q.B * q.D - q.A * q.E;
    double rx = bx * bx + det * (q.E * q.E - q.C * q.F);
    double ry = by * by + det * (q.D * q.D - q.A * q.F);
    rx = rx > 0.0 ? rx : 0.0;
    ry = ry > 0.0 ? ry : 0.0;
    const double sx = sqrt(rx), sy = sqrt(ry);
    e[0] = (bx - sx) / det;
    e[1] = (bx + sx) / det;
    e[2] = (by - sy) / det;
    e[3] = (by + sy) / det;
    return fs_finite(e[0]) && fs_finite(e[1]) && fs_finite(e[2]) && fs_finite(e[3]);
}

// Surfel footprint in pixel space: the exact predicate (H, k2) plus the
// anchored conic, used to enumerate the footprint line by line.
struct FsFootprint {
    double H[9];
    double k2;
    FsConic q;
    int px0, px1, py0, py1;   // candidate pixel range (inclusive), clamped to the image
};

FS_DEV int fs_clampi(long long v, int lo, int hi) { return (int)(v < lo ? lo : (v > hi ? hi : v)); }

// Build the footprint: anchor at the pixel containing the projected centre
// (clamped to the image), conic, and the candidate pixel range (conic extent
// widened by one pixel).  Returns false if no pixel can be inside.
FS_DEV bool fs_footprint(const FsGeo& g, int W, int Hh, FsFootprint& fp) {
    for (int j = 0; j < 9; ++j) fp.H[j] = g.H[j];
    fp.k2 = g.k2;
    const double mx = g.T[2] / g.T[8], my = g.T[5] / g.T[8];
    const double lim = 1.0e6;
    const double cmx = mx < -lim ? -lim : (mx > lim ? lim : mx);
    const double cmy = my < -lim ? -lim : (my > lim ? lim : my);
    const int ax = fs_clampi((long long)floor(cmx), 0, W - 1);
    const int ay = fs_clampi((long long)floor(cmy), 0, Hh - 1);
    fs_conic(fp.H, fp.k2, ax, ay, fp.q);
    double e[4];
    if (!fs_conic_extent(fp.q, e)) {
        fp.px0 = 0;
        fp.px1 = W - 1;
        fp.py0 = 0;
        fp.py1 = Hh - 1;
        return true;
    }
    const double big = 4.0e6;
    for (int j = 0; j < 4; ++j) e[j] = e[j] < -big ? -big : (e[j] > big ? big : e[j]);
    // pixel centre px + .5 = ax + .5 + dx  ->  px = ax + dx
    fp.px0 = fs_clampi((long long)ceil(e[0]) + ax - 1, 0, W - 1);
    fp.px1 = fs_clampi((long long)floor(e[1]) + ax + 1, 0, W - 1);
    fp.py0 = fs_clampi((long long)ceil(e[2]) + ay - 1, 0, Hh - 1);
    fp.py1 = fs_clampi((long long)floor(e[3]) + ay + 1, 0, Hh - 1);
    if ((long long)floor(e[1]) + ax + 1 < 0 || (long long)ceil(e[0]) + ax - 1 > W - 1) return false;
    if ((long long)floor(e[3]) + ay + 1 < 0 || (long long)ceil(e[2]) + ay - 1 > Hh - 1) return false;
    return fp.px0 <= fp.px1 && fp.py0 <= fp.py1;
}

// Pixels of one line inside a conic shape.  Row mode (rows = true): line is
// pixel row `l`, the result [lo, hi] are pixel columns.  Column mode: line is
// pixel column `l`, result are pixel rows.  The quadratic (the AccuTile
// equation of Sec. 3.2) gives the interval; endpoint pixels whose centres lie
// within 1e-4 px of the conic are re-decided with the shape's exact
// predicate pin(s), so the result equals the per-pixel definition.  Returns
// false if the line is empty.
template <class Pin>
FS_DEV bool fs_conic_line(const FsConic& q, Pin&& pin, bool rows, int l, int lo_lim, int hi_lim, int& lo, int& hi) {
    // along-line coordinate s, across-line offset d (both anchor-relative)
    double a, b, c, d;
    int anchor_s;
    if (rows) {
        d = (double)(l - q.ay);
        a = q.A;
        b = q.B * d + q.D;
        c = (q.C * d + 2.0 * q.E) * d + q.F;
        anchor_s = q.ax;
    } else {
        d = (double)(l - q.ax);
        a = q.C;
        b = q.B * d + q.E;
        c = (q.A * d + 2.0 * q.D) * d + q.F;
        anchor_s = q.ay;
    }
    if (!(a > 0.0)) {
        // degenerate in floating point: decide every pixel of the line
        lo = hi_lim + 1;
        hi = lo_lim - 1;
        for (int s = lo_lim; s <= hi_lim; ++s) {
            if (pin(s)) {
                lo = lo < s ? lo : s;
                hi = s;
            }
        }
        return lo <= hi;
    }
    const double eps = 1e-4;
    const double disc = b * b - a * c;
    if (disc < 0.0) {
        // empty unless the line is tangent within rounding: test the pixel
        // nearest the vertex and grow from it
        if (-disc > 1e-8 * (b * b + fabs(a * c))) return false;
        const double sv = -b / a;
        if (!(fabs(sv) < 4.0e6)) return false;
        const int s0 = (int)rint(sv) + anchor_s;
        if (s0 < lo_lim || s0 > hi_lim || !pin(s0)) return false;
        lo = hi = s0;
        while (lo > lo_lim && pin(lo - 1)) --lo;
        while (hi < hi_lim && pin(hi + 1)) ++hi;
        return true;
    }
    // The roots only locate the interval: every centre within eps of a root
    // is re-decided below with the exact predicate, so they need an absolute
    // error far below eps, not correct rounding.  (-b -+ sqrt(disc)) / a with
    // 1/a (the same for every line of the footprint) and sqrt(disc) from
    // hardware seeds refined by Newton steps: the relative error of sqrt is
    // ~1e-13, and the cancellation in -b + sqrt(disc) leaves an absolute
    // error of a few ulps of |b| / a, so for |s| <= 4e6 every root is within
    // 1e-6 px.
    const double sq = fs_sqrt_line(disc);
    const double ra = fs_rcp_approx(a);
    double s1 = (-b - sq) * ra, s2 = (-b + sq) * ra;
    if (s1 > s2) {
        const double tmp = s1;
        s1 = s2;
        s2 = tmp;
    }
    if (!(s1 > -4.0e6)) s1 = -4.0e6;
    if (!(s2 < 4.0e6)) s2 = 4.0e6;
    // centres strictly inside: s in [ceil(s1), floor(s2)]
    const double cs1 = ceil(s1), fs2 = floor(s2);
    long long L = (long long)cs1 + anchor_s, Hi = (long long)fs2 + anchor_s;
    // re-decide endpoints within eps of the conic
    if (cs1 - s1 < eps) {                     // first centre barely inside
        if (L >= lo_lim && L <= hi_lim && !pin((int)L)) ++L;
    } else if (1.0 - (cs1 - s1) < eps) {      // centre before it barely outside
        if (L - 1 >= lo_lim && L - 1 <= hi_lim && pin((int)(L - 1))) --L;
    }
    if (s2 - fs2 < eps) {
        if (Hi >= lo_lim && Hi <= hi_lim && !pin((int)Hi)) --Hi;
    } else if (1.0 - (s2 - fs2) < eps) {
        if (Hi + 1 >= lo_lim && Hi + 1 <= hi_lim && pin((int)(Hi + 1))) ++Hi;
    }
    if (L < lo_lim) L = lo_lim;
    if (Hi > hi_lim) Hi = hi_lim;
    if (L > Hi) return false;
    lo = (int)L;
    hi = (int)Hi;
    return true;
}

// Pixels of one line inside the exact footprint (fs_conic_line with the
// footprint predicate u^2 + v^2 <= k^2).
FS_DEV bool fs_line_interval(const FsFootprint& fp, bool rows, int l, int lo_lim, int hi_lim, int& lo, int& hi) {
    auto pin = [&](int s) -> bool { return rows ? fs_pixel_in(fp.H, fp.k2, s, l) : fs_pixel_in(fp.H, fp.k2, l, s); };
    return fs_conic_line(fp.q, pin, rows, l, lo_lim, hi_lim, lo, hi);
}

// Enumerate the tiles of the footprint (SnugBox traversal: lines run along the
// shorter side of the pixel range, Sec. 3.2).  For every tile line (a tile
// row in row mode, a tile column in column mode) the tile spans of its pixel
// lines are OR-ed into a 64-bit mask over a window of at most 64 tiles, then
// visit(tx, ty) is called for each tile of the union, in increasing order.
// The lines of a tile line are visited from the one nearest the conic's
// centre outwards, and the visit stops once the mask holds every tile the
// conic's extent along the lines reaches in the window: no further line can
// add a tile, so the union is unchanged (a footprint within one tile column
// usually needs a single line solve per tile line).
template <class Visit>
FS_DEV void fs_sweep_tiles(const FsFootprint& fp, int S, Visit&& visit) {
    const bool rows = (fp.py1 - fp.py0) <= (fp.px1 - fp.px0);
    const int l0 = rows ? fp.py0 : fp.px0, l1 = rows ? fp.py1 : fp.px1;      // lines
    const int s0 = rows ? fp.px0 : fp.py0, s1 = rows ? fp.px1 : fp.py1;      // along-line range
    const int ts0 = s0 / S, ts1 = s1 / S;
    // the line through the conic's centre (the middle of the range if the
    // conic is not a bounded ellipse)
    int lc = (l0 + l1) >> 1;
    {
        const FsConic& q = fp.q;
        const double det = q.A * q.C - q.B * q.B;
        if (q.A > 0.0 && q.C > 0.0 && det > 0.0) {
            const double cen = rows ? (q.B * q.D - q.A * q.E) / det + (double)q.ay
                                    : (q.B * q.E - q.C * q.D) / det + (double)q.ax;
            if (cen > (double)l0 && cen < (double)l1) lc = (int)rint(cen);
        }
    }
    // the tiles any line can reach: the conic's extent along the lines, with
    // a margin of 1e-3 px (far beyond its rounding), within [s0, s1]; for a
    // nearly degenerate conic (det < 1e-6 A C, an extent sensitive to the
    // coefficients' rounding) the whole candidate range
    int tt0 = ts0, tt1 = ts1;
    {
        const FsConic& q = fp.q;
        double e[4];
        if (q.A * q.C - q.B * q.B > 1e-6 * (q.A * q.C) && fs_conic_extent(q, e)) {
            const double a0 = rows ? e[0] : e[2], a1 = rows ? e[1] : e[3];
            const int anchor = rows ? fp.q.ax : fp.q.ay;
            if (a0 > -4.0e6 && a1 < 4.0e6) {
                const long long lo = (long long)ceil(a0 - 1e-3) + anchor, hi = (long long)floor(a1 + 1e-3) + anchor;
                const int clo = fs_clampi(lo, s0, s1), chi = fs_clampi(hi, s0, s1);
                if (clo <= chi) {
                    tt0 = clo / S;
                    tt1 = chi / S;
                }
            }
        }
    }
    for (int wbase = ts0; wbase <= ts1; wbase += 64) {
        // bits tt0 - wbase .. tt1 - wbase of the window (empty if outside it)
        const int f0 = tt0 - wbase > 0 ? tt0 - wbase : 0;
        const int f1 = tt1 - wbase < 63 ? tt1 - wbase : 63;
        const uint64_t full = f0 > f1 ? 0ull
                                      : ((f1 == 63 ? ~0ull : ((1ull << (f1 + 1)) - 1ull)) & ~((1ull << f0) - 1ull));
        for (int tl = l0 / S; tl <= l1 / S; ++tl) {
            uint64_t mask = 0;
            const int la = tl * S > l0 ? tl * S : l0;
            const int lb = tl * S + S - 1 < l1 ? tl * S + S - 1 : l1;
            const int lm = lc < la ? la : (lc > lb ? lb : lc);
            for (int k = 0; k <= lb - la && mask != full; ++k) {
                // lm, lm + 1, .., lb, then lm - 1, .., la
                const int l = lm + k <= lb ? lm + k : lm - (k - (lb - lm));
                int lo, hi;
                if (!fs_line_interval(fp, rows, l, s0, s1, lo, hi)) continue;
                int t1 = lo / S - wbase, t2 = hi / S - wbase;
                if (t2 < 0 || t1 > 63) continue;
                t1 = t1 < 0 ? 0 : t1;
                t2 = t2 > 63 ? 63 : t2;
                const uint64_t hiBits = (t2 == 63) ? ~0ull : ((1ull << (t2 + 1)) - 1ull);
                mask |= hiBits & ~((1ull << t1) - 1ull);
            }
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1ull;
                const int ts = wbase + b;
                if (rows)
                    visit(ts, tl);
                else
                    visit(tl, ts);
            }
        }
    }
}

// Tiles of the square circumscribing the ellipse (centre +- semi-major axis):
// the bounding-box assignment used as the baseline of the tile ablation.
FS_DEV bool fs_bbox_tiles(const FsFootprint& fp, int W, int Hh, int S, int& tx0, int& tx1, int& ty0, int& ty1) {
    const FsConic& q = fp.q;
    const double det = q.A * q.C - q.B * q.B;
    if (!(q.A > 0.0) || !(q.C > 0.0) || !(det > 0.0)) {
        tx0 = fp.px0 / S;
        tx1 = fp.px1 / S;
        ty0 = fp.py0 / S;
        ty1 = fp.py1 / S;
        return true;
    }
    const double xc = (q.B * q.E - q.C * q.D) / det, yc = (q.B * q.D - q.A * q.E) / det;
    const double f0 = -((q.D * xc + q.E * yc) + q.F);
    if (!(f0 > 0.0)) return false;
    const double hm = 0.5 * (q.A + q.C), dd = 0.5 * (q.A - q.C);
    const double lmin = hm - sqrt(dd * dd + q.B * q.B);
    if (!(lmin > 0.0)) return false;
    const double r = sqrt(f0 / lmin) * (1.0 + 1e-9) + 1e-6;
    const double cx = xc + q.ax, cy = yc + q.ay;     // in pixel-index units (centre at +.5)
    const long long x0 = (long long)ceil(cx - r), x1 = (long long)floor(cx + r);
    const long long y0 = (long long)ceil(cy - r), y1 = (long long)floor(cy + r);
    if (x1 < 0 || y1 < 0 || x0 > W - 1 || y0 > Hh - 1 || x0 > x1 || y0 > y1) return false;
    tx0 = fs_clampi(x0, 0, W - 1) / S;
    tx1 = fs_clampi(x1, 0, W - 1) / S;
    ty0 = fs_clampi(y0, 0, Hh - 1) / S;
    ty1 = fs_clampi(y1, 0, Hh - 1) / S;
    return true;
}

// ---------------------------------------------------------------------------
// Extended tile assignment: the paper-literal linearised ellipse (Sec. 3.2)
// in place of the exact footprint, and the low-pass disc (2D Gaussian
// splatting's screen-space filter) added to either.  Every predicate is
// evaluated in double precision with a fixed operation order, so the tile
// sets are a pure function of the inputs.
// ---------------------------------------------------------------------------
// The linearised projected covariance, read as J J^T with J the Jacobian of
// the perspective map (T1 . u, T2 . u) / (Tw . u) at the tangent origin:
// J_rc = (T_rc - mu_r T_wc) / T_w3, mu = (T_13, T_23) / T_w3.  P receives the
// inverse of Sigma' = J J^T as (P00, P01, P11); false if Sigma' is singular.
FS_DEV bool fs_linearised_ellipse(const double T[9], double mu[2], double P[3]) {
    mu[0] = T[2] / T[8];
    mu[1] = T[5] / T[8];
    const double J00 = (T[0] - mu[0] * T[6]) / T[8];
    const double J01 = (T[1] - mu[0] * T[7]) / T[8];
    const double J10 = (T[3] - mu[1] * T[6]) / T[8];
    const double J11 = (T[4] - mu[1] * T[7]) / T[8];
    const double S00 = J00 * J00 + J01 * J01;
    const double S01 = J00 * J10 + J01 * J11;
    const double S11 = J10 * J10 + J11 * J11;
    const double det = S00 * S11 - S01 * S01;
    if (!(det > 0.0) || !fs_finite(det)) return false;
    P[0] = S11 / det;
    P[1] = -S01 / det;
    P[2] = S00 / det;
    return true;
}

// (x - mu)^T Sigma'^-1 (x - mu) <= k^2 at the centre of pixel (px, py).
FS_DEV bool fs_lin_in(const double mu[2], const double P[3], double k2, int px, int py) {
    const double dx = ((double)px + 0.5) - mu[0], dy = ((double)py + 0.5) - mu[1];
    return (P[0] * dx * dx + 2.0 * P[1] * dx * dy) + P[2] * dy * dy <= k2;
}

// Low-pass disc: 2 |x - mu|^2 <= k^2 at the centre of pixel (px, py).
FS_DEV bool fs_disc_in(const double mu[2], double k2, int px, int py) {
    const double dx = ((double)px + 0.5) - mu[0], dy = ((double)py + 0.5) - mu[1];
    return 2.0 * (dx * dx + dy * dy) <= k2;
}

// Conic of (x - c)^T P (x - c) <= k2 (P = (P00, P01, P11)) relative to the
// anchor pixel centre of `like`: only locates line intervals, whose ends the
// shape's predicate re-decides.
FS_DEV void fs_centred_conic(const double c[2], const double P[3], double k2, const FsConic& like, FsConic& q) {
    const double ex = c[0] - ((double)like.ax + 0.5), ey = c[1] - ((double)like.ay + 0.5);
    q.A = P[0];
    q.B = P[1];
    q.C = P[2];
    q.D = -(P[0] * ex + P[1] * ey);
    q.E = -(P[1] * ex + P[2] * ey);
    q.F = (P[0] * ex * ex + 2.0 * P[1] * ex * ey + P[2] * ey * ey) - k2;
    q.ax = like.ax;
    q.ay = like.ay;
}

// Candidate pixel range of a conic (extent widened by one pixel, clamped to
// the image; the whole image if the extent is not finite).  False if it lies
// outside the image.
FS_DEV bool fs_conic_range(const FsConic& q, int W, int Hh, int r[4]) {
    double e[4];
    if (!fs_conic_extent(q, e)) {
        r[0] = 0;
        r[1] = W - 1;
        r[2] = 0;
        r[3] = Hh - 1;
        return true;
    }
    const double big = 4.0e6;
    for (int j = 0; j < 4; ++j) e[j] = e[j] < -big ? -big : (e[j] > big ? big : e[j]);
    const long long x0 = (long long)ceil(e[0]) + q.ax - 1, x1 = (long long)floor(e[1]) + q.ax + 1;
    const long long y0 = (long long)ceil(e[2]) + q.ay - 1, y1 = (long long)floor(e[3]) + q.ay + 1;
    if (x1 < 0 || x0 > W - 1 || y1 < 0 || y0 > Hh - 1) return false;
    r[0] = fs_clampi(x0, 0, W - 1);
    r[1] = fs_clampi(x1, 0, W - 1);
    r[2] = fs_clampi(y0, 0, Hh - 1);
    r[3] = fs_clampi(y1, 0, Hh - 1);
    return r[0] <= r[1] && r[2] <= r[3];
}

FS_DEV void fs_range_union(int r[4], const int a[4], bool& have) {
    if (!have) {
        for (int j = 0; j < 4; ++j) r[j] = a[j];
        have = true;
        return;
    }
    r[0] = a[0] < r[0] ? a[0] : r[0];
    r[1] = a[1] > r[1] ? a[1] : r[1];
    r[2] = a[2] < r[2] ? a[2] : r[2];
    r[3] = a[3] > r[3] ? a[3] : r[3];
}

// The shapes a surfel's tiles come from when the tile mode is LINEARISED or
// the low-pass option is on, and the pixel box the renderers accept it in.
struct FsAssign {
    bool lin;          // the linearised ellipse replaces the exact footprint
    bool lin_ok;       // Sigma' is positive definite
    bool exact_ok;     // the exact footprint's range meets the image
    bool disc;         // the low-pass disc is added
    double mu[2];      // projected centre
    double P[3];       // Sigma'^-1
    FsConic ql, qd;    // linearised and disc conics (anchored like the footprint)
    int ar[4];         // candidate pixel range of the assignment (x0, x1, y0, y1)
    bool have_ar;
    int box[4];        // acceptance box of the record: exact range, plus the disc's
    bool have_box;
};

// Set up the extended assignment of a projected surfel whose exact
// footprint fp was built by fs_footprint (exact_ok = its result).
FS_DEV void fs_assign_setup(const FsGeo& g, const FsFootprint& fp, bool exact_ok, int W, int Hh, bool lin,
                            bool lowpass, FsAssign& a) {
    a.lin = lin;
    a.disc = lowpass;
    a.exact_ok = exact_ok;
    a.lin_ok = false;
    a.have_ar = a.have_box = false;
    a.mu[0] = g.T[2] / g.T[8];
    a.mu[1] = g.T[5] / g.T[8];
    int r[4];
    if (exact_ok) {
        r[0] = fp.px0;
        r[1] = fp.px1;
        r[2] = fp.py0;
        r[3] = fp.py1;
        fs_range_union(a.box, r, a.have_box);
        if (!lin) fs_range_union(a.ar, r, a.have_ar);
    }
    if (lin) {
        a.lin_ok = fs_linearised_ellipse(g.T, a.mu, a.P);
        if (a.lin_ok) {
            fs_centred_conic(a.mu, a.P, g.k2, fp.q, a.ql);
            if (fs_conic_range(a.ql, W, Hh, r)) fs_range_union(a.ar, r, a.have_ar);
        }
    }
    if (lowpass) {
        const double Pd[3] = {2.0, 0.0, 2.0};
        fs_centred_conic(a.mu, Pd, g.k2, fp.q, a.qd);
        if (fs_conic_range(a.qd, W, Hh, r)) {
            fs_range_union(a.ar, r, a.have_ar);
            fs_range_union(a.box, r, a.have_box);
        }
    }
}

// Tiles of the extended assignment, as fs_sweep_tiles: per tile line the
// tile spans of every shape's pixel lines are OR-ed into a 64-bit mask.
template <class Visit>
FS_DEV void fs_sweep_tiles_ext(const FsFootprint& fp, const FsAssign& a, int S, Visit&& visit) {
    if (!a.have_ar) return;
    const int* ar = a.ar;
    const bool rows = (ar[3] - ar[2]) <= (ar[1] - ar[0]);
    const int l0 = rows ? ar[2] : ar[0], l1 = rows ? ar[3] : ar[1];
    const int s0 = rows ? ar[0] : ar[2], s1 = rows ? ar[1] : ar[3];
    const int ts0 = s0 / S, ts1 = s1 / S;
    const bool use_exact = !a.lin && a.exact_ok, use_lin = a.lin && a.lin_ok, use_disc = a.disc;
    for (int wbase = ts0; wbase <= ts1; wbase += 64) {
        for (int tl = l0 / S; tl <= l1 / S; ++tl) {
            uint64_t mask = 0;
            const int la = tl * S > l0 ? tl * S : l0;
            const int lb = tl * S + S - 1 < l1 ? tl * S + S - 1 : l1;
            auto add = [&](int lo, int hi) {
                int t1 = lo / S - wbase, t2 = hi / S - wbase;
                if (t2 < 0 || t1 > 63) return;
                t1 = t1 < 0 ? 0 : t1;
                t2 = t2 > 63 ? 63 : t2;
                const uint64_t hiBits = (t2 == 63) ? ~0ull : ((1ull << (t2 + 1)) - 1ull);
                mask |= hiBits & ~((1ull << t1) - 1ull);
            };
            for (int l = la; l <= lb; ++l) {
                int lo, hi;
                if (use_exact && fs_line_interval(fp, rows, l, s0, s1, lo, hi)) add(lo, hi);
                if (use_lin) {
                    auto pin = [&](int t) -> bool {
                        return rows ? fs_lin_in(a.mu, a.P, fp.k2, t, l) : fs_lin_in(a.mu, a.P, fp.k2, l, t);
                    };
                    if (fs_conic_line(a.ql, pin, rows, l, s0, s1, lo, hi)) add(lo, hi);
                }
                if (use_disc) {
                    auto pin = [&](int t) -> bool {
                        return rows ? fs_disc_in(a.mu, fp.k2, t, l) : fs_disc_in(a.mu, fp.k2, l, t);
                    };
                    if (fs_conic_line(a.qd, pin, rows, l, s0, s1, lo, hi)) add(lo, hi);
                }
            }
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1ull;
                const int ts = wbase + b;
                if (rows)
                    visit(ts, tl);
                else
                    visit(tl, ts);
            }
        }
    }
}

// Bounding-box assignment with the low-pass disc: the tile rectangle
// covering the exact footprint's circumscribed square and the disc's square.
FS_DEV bool fs_bbox_tiles_ext(const FsFootprint& fp, bool exact_ok, const FsAssign& a, int W, int Hh, int S,
                              int& tx0, int& tx1, int& ty0, int& ty1) {
    bool have = exact_ok && fs_bbox_tiles(fp, W, Hh, S, tx0, tx1, ty0, ty1);
    if (a.disc) {
        const double rd = sqrt(0.5 * fp.k2) * (1.0 + 1e-9) + 1e-6;
        const double lo_x = a.mu[0] - 0.5 - rd, hi_x = a.mu[0] - 0.5 + rd;   // pixel-index units
        const double lo_y = a.mu[1] - 0.5 - rd, hi_y = a.mu[1] - 0.5 + rd;
        if (fs_finite(lo_x) && fs_finite(hi_x) && fs_finite(lo_y) && fs_finite(hi_y)) {
            const long long x0 = (long long)ceil(lo_x), x1 = (long long)floor(hi_x);
            const long long y0 = (long long)ceil(lo_y), y1 = (long long)floor(hi_y);
            if (!(x1 < 0 || y1 < 0 || x0 > W - 1 || y0 > Hh - 1 || x0 > x1 || y0 > y1)) {
                const int dx0 = fs_clampi(x0, 0, W - 1) / S, dx1 = fs_clampi(x1, 0, W - 1) / S;
                const int dy0 = fs_clampi(y0, 0, Hh - 1) / S, dy1 = fs_clampi(y1, 0, Hh - 1) / S;
                if (!have) {
                    tx0 = dx0;
                    tx1 = dx1;
                    ty0 = dy0;
                    ty1 = dy1;
                    have = true;
                } else {
                    tx0 = dx0 < tx0 ? dx0 : tx0;
                    tx1 = dx1 > tx1 ? dx1 : tx1;
                    ty0 = dy0 < ty0 ? dy0 : ty0;
                    ty1 = dy1 > ty1 ? dy1 : ty1;
                }
            }
        }
    }
    return have;
}

// ---------------------------------------------------------------------------
// Response of a record at pixel offset (dx, dy) from its anchor: (u, v) and
// d2 = u^2 + v^2 in double precision (fused multiply-adds; 1/h2 from the
// hardware reciprocal refined by one Newton step).  Shared by the forward and
// backward renderers so both take identical accept decisions.
// ---------------------------------------------------------------------------
struct FsResp {
    double u, v, d2, rh;   // tangent coordinates, u^2 + v^2, 1 / h2
};

FS_DEV FsResp fs_response(const FsRecord& r, double dx, double dy) {
    FsResp o;
    const double h0 = fma(dy, r.gy0, fma(dx, r.gx0, r.h0));
    const double h1 = fma(dy, r.gy1, fma(dx, r.gx1, r.h1));
    const double h2 = fma(dy, r.gy2, fma(dx, r.gx2, r.h2));
    double rh = __builtin_amdgcn_rcp(h2);
    rh = fma(rh, fma(-h2, rh, 1.0), rh);
    o.rh = rh;
    o.u = h0 * rh;
    o.v = h1 * rh;
    o.d2 = fma(o.u, o.u, o.v * o.v);
    return o;
}

// Projected centre of a record relative to its anchor pixel centre: the
// point where h0 = h1 = 0 (the tangent origin), solved from the anchored
// coefficients.  Used by the low-pass response.
FS_DEV void fs_record_centre(const FsRecord& r, double& mx, double& my) {
    const double det = r.gx0 * r.gy1 - r.gy0 * r.gx1;
    mx = (r.h1 * r.gy0 - r.h0 * r.gy1) / det;
    my = (r.h0 * r.gx1 - r.h1 * r.gx0) / det;
}

// The low-pass response: d2 = min(u^2 + v^2, 2 |x - mu|^2), the pixel offset
// (dx, dy) and the centre (mx, my) both relative to the anchor.
FS_DEV void fs_lowpass_d2(FsResp& rs, double dx, double dy, double mx, double my) {
    const double ex = dx - mx, ey = dy - my;
    const double r2 = 2.0 * (ex * ex + ey * ey);
    rs.d2 = r2 < rs.d2 ? r2 : rs.d2;
}

// Camera-space normal of a record's plane, facing the camera.  The anchored,
// normalised h2 equals z_c / depth(x) along the ray of pixel point x, a
// linear function of x whose gradient, scaled by the focal lengths, and whose
// value at the principal point form a normal m with m . p_c > 0: the
// camera-facing unit normal is -m / |m|.  (cx, cy) are in pixel-index units
// relative to the anchor pixel centre.
FS_DEV float3 fs_record_normal(const FsRecord& r, const fs_camera& cam) {
    const double ox = (double)cam.cx - ((double)r.ax + 0.5), oy = (double)cam.cy - ((double)r.ay + 0.5);
    const double m0 = (double)cam.fx * r.gx2, m1 = (double)cam.fy * r.gy2;
    const double m2 = r.h2 + ox * r.gx2 + oy * r.gy2;
    const double inv = -1.0 / sqrt(m0 * m0 + m1 * m1 + m2 * m2);
    return make_float3((float)(m0 * inv), (float)(m1 * inv), (float)(m2 * inv));
}

// A pixel is accepted only inside the record's pixel box (it holds every
// pixel centre inside the exact footprint conic; outside it the d2 test can
// only pass by rounding).  Every renderer applies the same test, so their
// accept decisions agree wherever they evaluate a pixel.
FS_DEV bool fs_in_box(const FsRecord& r, int px, int py) {
    return (px >= r.x0) & (px <= r.x1) & (py >= r.y0) & (py <= r.y1);
}

// Record index -> surfel index for record r = v * n + i.
FS_DEV int64_t fs_surfel_of(int64_t rec, int64_t n) { return rec % n; }

// View of a global tile id (binary search over tile offsets; num_views is small).
FS_DEV int fs_view_of_tile(const fs_camera* cams, int num_views, int64_t tile) {
    int lo = 0, hi = num_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)cams[mid].tile_offset <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Render block b of a frame: tile b / (S / RB)^2, sub-block b % (S / RB)^2 of
// RB x RB pixels in row-major order inside the tile.
struct BlockPos {
    int view;
    int x0, y0;      // block origin (view-local pixels)
    int64_t tile;    // global tile id
    bool valid;
};

FS_DEV BlockPos locate_block(int64_t b, int S, int RB, const fs_camera* cams, int num_views) {
    // 32-bit arithmetic: launches keep b < 2^32; S and S / RB are powers of two
    BlockPos bp;
    const uint32_t bb = (uint32_t)b;
    const int lsb = S / RB == 4 ? 2 : (S / RB == 2 ? 1 : 0);   // log2(S / RB)
    const int ls = S == 32 ? 5 : (S == 16 ? 4 : 3);             // log2(S)
    const uint32_t tile = bb >> (2 * lsb);
    const uint32_t sub = bb & ((1u << (2 * lsb)) - 1u);
    const int v = fs_view_of_tile(cams, num_views, tile);
    const fs_camera& cam = cams[v];
    const uint32_t tiles_x = ((uint32_t)cam.width + (uint32_t)S - 1u) >> ls;
    const uint32_t local = tile - (uint32_t)cam.tile_offset;
    const uint32_t ty = local / tiles_x, tx = local - ty * tiles_x;
    bp.view = v;
    bp.tile = tile;
    bp.x0 = (int)(tx << ls) + (int)(sub & ((1u << lsb) - 1u)) * RB;
    bp.y0 = (int)(ty << ls) + (int)(sub >> lsb) * RB;
    bp.valid = bp.x0 < cam.width && bp.y0 < cam.height;
    return bp;
}

// Workgroup -> work item: dispatch hands workgroup g to XCD g mod 8; remap so
// that XCD x takes the contiguous run [x * per, (x + 1) * per).  The last
// G mod 8 workgroups keep their own index.
FS_DEV int64_t xcd_remap(int64_t g, int64_t G) {
    const int64_t per = G / 8;
    if (g >= per * 8) return g;
    return (g % 8) * per + g / 8;
}

// Workgroup -> work item in chunks: the XCDs take turns with runs of `chunk`
// consecutive items (chunk i goes to XCD i mod 8), so all XCDs sweep the
// work in step while neighbouring items still share an XCD.  Items past the
// last whole round of 8 chunks keep their own index.
FS_DEV int64_t xcd_remap_chunked(int64_t g, int64_t G, int64_t chunk) {
    const int64_t round = 8 * chunk;
    if (g >= (G / round) * round) return g;
    const int64_t x = g % 8, s = g / 8;   // XCD and its s-th workgroup
    return ((s / chunk) * 8 + x) * chunk + s % chunk;
}

// 8x8 blocks in one tile row of the first view: the chunk the block passes
// hand to the XCDs in turn (measured best on 1280- and 640-pixel views
// against smaller and larger chunks and against one run per XCD).
FS_DEV int64_t block_row_chunk(const fs_camera* cams, int S) {
    const int64_t tiles_x = ((int64_t)cams[0].width + S - 1) / S;
    const int64_t sb = S / 8;
    return tiles_x * sb * sb;
}

// Bitonic sort of 64 << LOGE keys by one wave, in registers: element
// i = lane * 2^LOGE + e is x[e] of its lane.  Compare-exchange partners
// i ^ j with j < 2^LOGE sit in the same lane; with larger j they are the
// same register of lane ^ (j >> LOGE), fetched by a shuffle.  The network is
// the textbook one (stage k, distance j, ascending where i & k == 0).
// Wave-wide inclusive prefix sums and reductions of the ROCm device library:
// lane shifts and row broadcasts in registers, with no LDS round trip (a
// chain of six shuffles costs six).  Every lane of the wave must be active.
extern "C" __device__ int __ockl_wfscan_add_i32(int, bool);
extern "C" __device__ unsigned int __ockl_wfscan_add_u32(unsigned int, bool);
extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_add_u32(unsigned int);
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_add_u64(unsigned long long);
extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_or_u32(unsigned int);
extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_min_u32(unsigned int);
extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_max_u32(unsigned int);
extern "C" __device__ __attribute__((const)) int __ockl_wfred_max_i32(int);

// Value of lane (lane ^ lm) for lm in {1, 2, 4, 8, 16, 32}.  Distances
// within a 16-lane row use data-parallel-primitive moves, which permute in
// the vector pipeline: quad permutations for 1 and 2, the mirror of an
// 8-lane half-row (lane ^ 7) followed by the reversal of a quad (lane ^ 3)
// for 4, the mirror of a row (lane ^ 15) followed by the half-row mirror for
// 8.  Longer distances go through the LDS crossbar: a swizzle within 32
// lanes for 16, a permute for 32.
FS_DEV uint32_t lane_xor32(uint32_t v, int lm) {
    const int x = (int)v;
    switch (lm) {
        case 1: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        case 2: return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        case 4: {
            const int h = __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false);          // row_half_mirror
            return (uint32_t)__builtin_amdgcn_mov_dpp(h, 0x1B, 0xF, 0xF, false);        // quad_perm [3,2,1,0]
        }
        case 8: {
            const int m = __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false);          // row_mirror
            return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x141, 0xF, 0xF, false);       // row_half_mirror
        }
        case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x1F | (16 << 10));   // xor 16 within 32 lanes
        default: return (uint32_t)__shfl_xor(x, lm, 64);
    }
}

FS_DEV uint64_t lane_xor64(uint64_t v, int lm) {
    const uint32_t lo = lane_xor32((uint32_t)v, lm), hi = lane_xor32((uint32_t)(v >> 32), lm);
    return (uint64_t)hi << 32 | lo;
}

template <int LOGE>
FS_DEV void wave_network(uint64_t (&x)[1 << LOGE]) {
    constexpr int E = 1 << LOGE;
    constexpr int LOGN = 6 + LOGE;
    const int lane = (int)threadIdx.x & 63;
#pragma unroll
    for (int lk = 1; lk <= LOGN; ++lk) {
        const int k = 1 << lk;
#pragma unroll
        for (int lj = lk - 1; lj >= 0; --lj) {
            const int j = 1 << lj;
            if (lj >= LOGE) {
                const int lm = j >> LOGE;   // lane distance
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = lane * E + e;
                    // with 16 keys per lane the vector pipeline is busy with the
                    // compare-exchanges, and the LDS crossbar moves them faster
                    const uint64_t y = LOGE <= 3 ? lane_xor64(x[e], lm) : __shfl_xor(x[e], lm, 64);
                    const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
                    const bool lt = y < x[e];
                    x[e] = (keep_min == lt) ? y : x[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if ((e & j) != 0) continue;
                    const int i = lane * E + e;
                    const uint64_t a = x[e], b = x[e | j];
                    const bool swap = (b < a) == ((i & k) == 0);
                    x[e] = swap ? b : a;
                    x[e | j] = swap ? a : b;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers implemented in the .hip files.
// ---------------------------------------------------------------------------
// Top-K lists in the workspace: for K <= FS_TOPK_COMPACT_K the selection
// writes every 8x8 block's per-pixel (row slot, weight) lists back to back
// (pixel p after pixels 0 .. p - 1) and the block's row count as
// rows | pairs << 16; for larger K pixel p's list starts at p * K.
constexpr int FS_TOPK_COMPACT_K = 16;

struct FsWorkspace {
    // bin (scan + emit)
    uint64_t* scan_status;   // partition totals
    uint32_t* bin_over_sums; // per partition: footprints whose tiles the tile cache does not hold
    uint32_t* scan_ticket;   // [1]: overflow count
    int64_t scan_parts;
    uint2* bin_overflow;     // (record, first offset) of those footprints
    // sort
    uint32_t* tile_cnt;      // pairs per tile
    uint32_t* tile_fill;     // scatter cursor per tile
    uint64_t* sort_status;   // look-back status of the tile-count scan partitions
    uint32_t* sort_ticket;
    uint2* runs;             // pairs grouped by tile, (depth key, record), capacity entries
    uint32_t* long_list;     // tiles whose runs are longer than one wave sorts
    // render
    uint32_t* render_ticket;   // kRenderQueues tickets, kTicketStride words apart
    uint32_t* render_gcnt;        // work order: blocks per cost bucket, per group of 256 blocks
    int64_t render_gcnt_words;
    uint32_t* render_order;
    int64_t render_max_blocks;
    uint32_t* sel_long;     // split Top-K selection: long-list blocks, per 256-block group
    uint32_t* sel_counts;   // their number per group
    // split Top-K render: (row slot, weight bits) of the first K blended
    // surfels of every pixel, indexed [8x8 block][pixel of block][k]; the
    // surfel index of every row slot of a block, [8x8 block][slot]; and the
    // number of row slots of every block
    uint2* topk_pairs;
    uint32_t* topk_rows;
    uint32_t* topk_nrows;
    int64_t topk_pair_slots;
    int32_t* topk_counts;    // backward: blend counts per pixel (at least 64 per 8x8 block)
};

bool fs_workspace_layout(void* base, int64_t n, int32_t num_views, int64_t total_tiles, int64_t pair_capacity,
                         const fs_opts* opts, FsWorkspace* ws, size_t* bytes);

hipError_t fs_launch_preprocess(const float* means, const float* scales, const float* quats, const float* opacity,
                                int64_t n, const fs_camera* cams, int32_t num_views, const fs_opts& o,
                                FsRecord* records, uint32_t* tiles_touched, uint32_t* tile_cache, hipStream_t s);

hipError_t fs_launch_bin(const float* means, const float* scales, const float* quats, const float* opacity, int64_t n,
                         const fs_camera* cams, int32_t num_views, const fs_opts& o, const uint32_t* tiles_touched,
                         const uint32_t* tile_cache, uint64_t* keys, uint32_t* vals, int64_t capacity,
                         int64_t* num_pairs, const FsWorkspace& ws, hipStream_t s);

// Device address and size of the static scratch of fs_bin_noalloc on the
// current device (bin.hip).
hipError_t fs_noalloc_scratch(void** ptr, size_t* bytes);

hipError_t fs_launch_sort(uint64_t* keys, uint32_t* vals, int64_t capacity, const int64_t* num_pairs, int64_t hint,
                          int64_t total_tiles, uint32_t* ranges, const FsWorkspace& ws, hipStream_t s);

hipError_t fs_launch_render_forward(const FsRecord* records, const uint64_t* keys, const uint32_t* vals,
                                    const uint32_t* ranges, const void* feats, int C, int64_t n,
                                    const fs_camera* cams, int num_views, int64_t total_tiles, const fs_opts& o,
                                    float* out_feat, float* out_T, int32_t* out_n, int32_t* out_last,
                                    int32_t* out_idx, float* out_depth, float* out_normal, uint64_t* counters,
                                    const FsWorkspace& ws, hipStream_t s);

// Work queues of the persistent render and the spacing of their tickets
// (256 B apart).  A ticket is a memory-side atomic, serialised per address:
// one ticket for every item of the frame limited the full blend (0.39 ms,
// against 0.336 ms with 8 queues and 0.332 ms with 32).
constexpr uint32_t kRenderQueues = 32;
constexpr uint32_t kTicketStride = 64;

// Work order of render blocks (tile list length, longest first; ties in any
// order) into ws.render_order; zeroes the kRenderQueues tickets of
// ws.render_ticket.
hipError_t fs_launch_block_order(const uint32_t* ranges, int sb2, uint32_t nblocks, const FsWorkspace& ws,
                                 hipStream_t s);

// Selection pass of the split Top-K renderer alone: per-pixel (slot, weight)
// lists, block row lists and counts in the workspace; out_T, out_last,
// out_idx and counters optional.
hipError_t fs_launch_topk_select(const FsRecord* records, const uint64_t* keys, const uint32_t* vals,
                                 const uint32_t* ranges, int64_t n, const fs_camera* cams, int num_views,
                                 int64_t total_tiles, const fs_opts& o, float* out_T, int32_t* out_n,
                                 int32_t* out_last, int32_t* out_idx, float* out_depth, float* out_normal,
                                 uint64_t* counters, const FsWorkspace& ws, hipStream_t s);

// Per-Gaussian instance labels (softmax over queries of similarity x
// proximity); 1 <= Q <= FS_MAX_QUERIES, D % 4 == 0.
hipError_t fs_launch_instance_labels(const float* fins, int D, const float* means, int64_t n, const float* fq,
                                     const float* qmeans, const float* qcovs, int Q, float* out, hipStream_t s);

// Both passes of the split Top-K renderer.  Exactly one of out_feat (feature
// image) and out_label (per-pixel channel argmax, out_score optional) is set.
hipError_t fs_launch_render_topk_split(const FsRecord* records, const uint64_t* keys, const uint32_t* vals,
                                       const uint32_t* ranges, const void* feats, int C, int64_t n,
                                       const fs_camera* cams, int num_views, int64_t total_tiles, const fs_opts& o,
                                       float* out_feat, int32_t* out_label, float* out_score, float* out_T,
                                       int32_t* out_n, int32_t* out_last, int32_t* out_idx, float* out_depth,
                                       float* out_normal, uint64_t* counters, const FsWorkspace& ws,
                                       hipStream_t s);

hipError_t fs_launch_render_backward(const float* means, const float* scales, const float* quats,
                                     const float* opacity, const FsRecord* records, const uint32_t* vals,
                                     const uint32_t* ranges, const void* feats, int C, int64_t n,
                                     const fs_camera* cams, int num_views, int64_t total_tiles, const fs_opts& o,
                                     const float* out_T, const int32_t* out_n, const int32_t* out_last,
                                     const float* grad_feat, float* grad_records, float* grad_means,
                                     float* grad_scales, float* grad_quats, float* grad_opacity, float* grad_feats,
                                     const FsWorkspace& ws, hipStream_t s);
