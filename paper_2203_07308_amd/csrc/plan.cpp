// Host side of a projector plan: geometry validation and the per-stage ray and
// view tables, computed in double precision and stored in float32.
//
// Readings of the fan-beam geometry (the paper fixes none): flat detector,
// one Joseph ray per bin centre, pixel centres at ((c-(nx-1)/2) h, (r-(ny-1)/2) h).
// Stage grids (pooling factor f, Sec. 2.1 Eq. (4)) keep the same isocentre and
// use pixel f h.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fbpnp_impl.h"

namespace fbpnp {

static thread_local std::string g_last_error;

fb_status fail(fb_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

fb_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return FB_EHIP;
}

const char* last_error() { return g_last_error.c_str(); }

fb_status validate_geometry(const fb_geom& g) {
    if (g.nx < 1 || g.ny < 1 || g.n_views < 1 || g.n_bins < 1)
        return fail(FB_EINVAL, "geometry: nx, ny, n_views and n_bins must be positive");
    if (g.nx > 32767 || g.ny > 32767) return fail(FB_EINVAL, "geometry: nx and ny must be at most 32767");
    const double vals[] = {g.pixel_mm, g.sod_mm, g.sdd_mm, g.det_pitch_mm, g.det_offset_mm, g.angle0_rad,
                           g.angle_step_rad};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(FB_EGEOM, "geometry: non-finite parameter");
    if (g.pixel_mm <= 0 || g.sod_mm <= 0 || g.sdd_mm <= 0 || g.det_pitch_mm <= 0)
        return fail(FB_EGEOM, "geometry: pixel, sod, sdd and pitch must be positive");
    double circ = 0.5 * g.pixel_mm * std::sqrt((double)g.nx * g.nx + (double)g.ny * g.ny);
    if (circ >= g.sod_mm) return fail(FB_EGEOM, "geometry: source inside the image circumcircle");
    double umax = std::fabs(0.5 * (g.n_bins - 1) * g.det_pitch_mm) + std::fabs(g.det_offset_mm);
    if (umax >= g.sdd_mm) return fail(FB_EGEOM, "geometry: fan wider than 90 degrees");
    return FB_OK;
}

// Index range [lo, hi] of lines l in [0, nlines) with pos(l) = p0 + l*dp in (pmin, pmax).
static void valid_range(double p0, double dp, int nlines, double pmin, double pmax, int& lo, int& hi) {
    auto ok = [&](int l) {
        double p = p0 + (double)l * dp;
        return p > pmin && p < pmax;
    };
    if (dp == 0.0) {
        if (ok(0)) {
            lo = 0;
            hi = nlines - 1;
        } else {
            lo = 0;
            hi = -1;
        }
        return;
    }
    double a = (pmin - p0) / dp, b = (pmax - p0) / dp;
    if (a > b) std::swap(a, b);
    double flo = std::floor(a) + 1.0, fhi = std::ceil(b) - 1.0;
    flo = std::max(flo, 0.0);
    fhi = std::min(fhi, (double)(nlines - 1));
    if (flo > fhi) {
        lo = 0;
        hi = -1;
        return;
    }
    lo = (int)flo;
    hi = (int)fhi;
    while (lo <= hi && !ok(lo)) ++lo;
    while (hi >= lo && !ok(hi)) --hi;
    if (lo > hi) {
        lo = 0;
        hi = -1;
        return;
    }
    while (lo > 0 && ok(lo - 1)) --lo;
    while (hi < nlines - 1 && ok(hi + 1)) ++hi;
}

fb_status build_stage_tables(const fb_geom& g, int f, std::vector<RayRec>& rays, std::vector<ViewRec>& views,
                             std::vector<int64_t>& view_samples) {
    const int nxs = g.nx / f, nys = g.ny / f, nb = g.n_bins;
    const double hs = g.pixel_mm * f;
    const double cxs = 0.5 * (nxs - 1), cys = 0.5 * (nys - 1);
    rays.assign((size_t)g.n_views * nb, RayRec{0.f, 0.f, 0.f, 0u});
    views.assign(g.n_views, ViewRec{});
    view_samples.assign(g.n_views, 0);
    for (int k = 0; k < g.n_views; ++k) {
        const double beta = g.angle0_rad + (double)k * g.angle_step_rad;
        const double cb = std::cos(beta), sb = std::sin(beta);
        const double sx = g.sod_mm * cb, sy = g.sod_mm * sb;
        const double cx = (g.sod_mm - g.sdd_mm) * cb, cy = (g.sod_mm - g.sdd_mm) * sb;
        int xlo = nb, xhi = -1, ylo = nb, yhi = -1;
        for (int j = 0; j < nb; ++j) {
            const double u = ((double)j - 0.5 * (nb - 1)) * g.det_pitch_mm + g.det_offset_mm;
            const double dx = cx - u * sb - sx, dy = cy + u * cb - sy;
            const double len = std::sqrt(dx * dx + dy * dy);
            const bool xmajor = std::fabs(dx) >= std::fabs(dy);
            double p0, dp, w;
            int nlines, npos;
            if (xmajor) {
                // row coordinate where the ray crosses the centre of column c,
                // rows per column dp (square pixels)
                dp = dy / dx;
                p0 = (sy + (-cxs * hs - sx) * dp) / hs + cys;
                w = hs * len / std::fabs(dx);
                nlines = nxs;
                npos = nys;
                xlo = std::min(xlo, j);
                xhi = std::max(xhi, j);
            } else {
                dp = dx / dy;
                p0 = (sx + (-cys * hs - sy) * dp) / hs + cxs;
                w = hs * len / std::fabs(dy);
                nlines = nys;
                npos = nxs;
                ylo = std::min(ylo, j);
                yhi = std::max(yhi, j);
            }
            // Float position of line k, centred on the grid's middle line and
            // middle position (integers nlines/2, npos/2), exactly as the kernels
            // evaluate it:  p(k) = fmaf(k - nlines/2, dpos, pos_c).
            // A sample exists where p(k) lies in [-1, npos) - npos/2; p is monotone
            // in k, so that is one interval of lines, found exactly in float from
            // a slightly wider double-precision estimate.
            const int lmid = nlines / 2, mid = npos / 2;
            const float dpf = (float)dp;
            const float pcf = (float)(p0 + (double)lmid * dp - (double)mid);
            const float plo = (float)(-1 - mid), phi = (float)(npos - mid);
            auto ok32 = [&](int l) {
                const float q = std::fmaf((float)(l - lmid), dpf, pcf);
                return q >= plo && q < phi;
            };
            // float and double positions differ by less than this margin, so the
            // float interval lies inside the widened double one
            const double margin = 1e-6 * (double)(nlines + npos + 100);
            int lo, hi;
            valid_range(p0, dp, nlines, -1.0 - margin, (double)npos + margin, lo, hi);
            while (hi >= lo && !ok32(lo)) ++lo;
            while (hi >= lo && !ok32(hi)) --hi;
            // A ray without samples keeps its own position: then on every line of
            // the grid it lies outside [-1, npos), which the matched back-projector
            // relies on for every candidate ray.
            RayRec& r = rays[(size_t)k * nb + j];
            r.pos_c = pcf;
            r.dpos = dpf;
            r.len = (float)w;
            r.bits = xmajor ? 0u : 0x80000000u;
            if (hi >= lo) {
                const int n = hi - lo + 1;
                r.bits |= (uint32_t)lo | ((uint32_t)n << 16);
                view_samples[k] += n;
            }
        }
        // each dominance class must be one contiguous bin range
        for (int j = 0; j < nb; ++j) {
            const bool ym = rays[(size_t)k * nb + j].bits >> 31;
            if (!ym && (j < xlo || j > xhi)) return fail(FB_EGEOM, "geometry: x-major bins not contiguous");
            if (ym && (j < ylo || j > yhi)) return fail(FB_EGEOM, "geometry: y-major bins not contiguous");
            if (!ym && j >= ylo && j <= yhi) return fail(FB_EGEOM, "geometry: dominance classes interleave");
        }
        // detector coordinate of the ray through stage pixel (c, r), centred indices
        const double K = g.sdd_mm / g.det_pitch_mm / g.sod_mm;
        ViewRec& v = views[k];
        v.a0 = 0.f;
        v.a1 = (float)(-K * hs * sb);
        v.a2 = (float)(K * hs * cb);
        v.b0 = 1.f;
        v.b1 = (float)(-hs * cb / g.sod_mm);
        v.b2 = (float)(-hs * sb / g.sod_mm);
        v.j0 = (float)(0.5 * (nb - 1) - g.det_offset_mm / g.det_pitch_mm);
        v.pad = 0.f;
        v.xlo = xlo;
        v.xhi = xhi;
        v.ylo = ylo;
        v.yhi = yhi;
    }
    return FB_OK;
}

// Adjacent rays j, j+1 of one dominance class and one view cross every line
// of the grid in the same order, so the distance between rays j and j+m on a
// line is at least m times the smallest adjacent distance dmin, and the
// distance is linear along the lines (smallest at the first or last line). The
// kernels evaluate positions in float (error far below 0.05 cells at these
// sizes), so m >= 2.05 / dmin keeps two such rays at least two cells apart,
// which the scatter backprojector needs to add their taps without a race.
int scatter_gap(const fb_geom& g, int f, const std::vector<RayRec>& rays, const std::vector<ViewRec>& views) {
    const int nxs = g.nx / f, nys = g.ny / f, nb = g.n_bins;
    double dmin = HUGE_VAL;
    for (int k = 0; k < g.n_views; ++k) {
        const ViewRec& v = views[k];
        for (int cls = 0; cls < 2; ++cls) {
            const int lo = cls ? v.ylo : v.xlo, hi = cls ? v.yhi : v.xhi;
            const int nlines = cls ? nys : nxs, lmid = nlines / 2;
            for (int j = lo; j < hi; ++j) {
                const RayRec& a = rays[(size_t)k * nb + j];
                const RayRec& b = rays[(size_t)k * nb + j + 1];
                for (int l : {0, nlines - 1}) {
                    const double t = (double)(l - lmid);
                    const double d = std::fabs(((double)b.pos_c + t * (double)b.dpos) -
                                               ((double)a.pos_c + t * (double)a.dpos));
                    dmin = std::min(dmin, d);
                }
            }
        }
    }
    if (!(dmin > 0.0)) return 1 << 30;  // (no adjacent pair: any gap will do; a zero distance: one part)
    const double m = std::ceil(2.05 / dmin);
    return m >= (double)(1 << 30) ? 1 << 30 : std::max(1, (int)m);
}

// ---------------------------------------------------------------------------
// Bicubic sketch tables (Sec. 3: resizing with bicubic interpolation).
// Output o of an axis of n pixels reduced by f sits at input coordinate
// (o + 1/2) f - 1/2; its weights are Keys' cubic convolution kernel (a = -1/2)
// at (i - u) / f, the taps outside the axis folded back by half-sample
// reflection, normalised to sum 1. The adjoint table lists, for each input i,
// the outputs whose weights reach it.
// ---------------------------------------------------------------------------
static double keys_cubic(double s) {
    const double a = -0.5, t = std::fabs(s);
    if (t <= 1.0) return ((a + 2.0) * t - (a + 3.0)) * t * t + 1.0;
    if (t < 2.0) return ((a * t - 5.0 * a) * t + 8.0 * a) * t - 4.0 * a;
    return 0.0;
}

static int fold_index(int i, int n) {
    while (i < 0 || i >= n) i = i < 0 ? -1 - i : 2 * n - 1 - i;
    return i;
}

fb_status bicubic_axis_tables(int n, int f, bool adjoint, std::vector<int>& lo, std::vector<float>& w, int& taps) {
    if (n < 1 || f < 1 || n % f) return fail(FB_EDIV, "bicubic sketch: size not divisible by f");
    const int m = n / f;
    std::vector<double> S((size_t)m * n, 0.0);
    for (int o = 0; o < m; ++o) {
        const double u = (o + 0.5) * f - 0.5;
        double sum = 0.0;
        for (int i = (int)std::floor(u - 2.0 * f); i <= (int)std::ceil(u + 2.0 * f); ++i) {
            const double k = keys_cubic((i - u) / f);
            if (k == 0.0) continue;
            S[(size_t)o * n + fold_index(i, n)] += k;
            sum += k;
        }
        for (int i = 0; i < n; ++i) S[(size_t)o * n + i] /= sum;
    }
    const int rows = adjoint ? n : m, cols = adjoint ? m : n;
    auto at = [&](int r, int c) { return adjoint ? S[(size_t)c * n + r] : S[(size_t)r * n + c]; };
    std::vector<int> first(rows, cols), last(rows, -1);
    taps = 1;
    for (int r = 0; r < rows; ++r) {
        for (int c = 0; c < cols; ++c)
            if (at(r, c) != 0.0) {
                first[r] = std::min(first[r], c);
                last[r] = c;
            }
        if (last[r] >= first[r]) taps = std::max(taps, last[r] - first[r] + 1);
    }
    taps = std::min(taps, cols);
    lo.assign(rows, 0);
    w.assign((size_t)rows * taps, 0.f);
    for (int r = 0; r < rows; ++r) {
        // a window of `taps` inputs inside the axis that holds every nonzero weight
        const int l = std::max(0, std::min(last[r] >= first[r] ? first[r] : 0, cols - taps));
        if (last[r] >= l + taps) return fail(FB_EINVAL, "bicubic sketch: weight window");
        lo[r] = l;
        for (int t = 0; t < taps; ++t) w[(size_t)r * taps + t] = (float)at(r, l + t);
    }
    return FB_OK;
}

}  // namespace fbpnp

extern "C" const char* fb_last_error(void) { return fbpnp::last_error(); }
