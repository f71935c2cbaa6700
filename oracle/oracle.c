/*
 * FP64 CPU oracle for multi-stage sketched plug-and-play fan-beam CT
 * (Tang, "Accelerating Plug-and-Play Image Reconstruction via Multi-Stage
 * Sketched Gradients", arXiv:2203.07308).
 *
 * TEST INFRASTRUCTURE. This file is the plain, slow reference against which the
 * GPU library is checked. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it. It shares no code, header, table or
 * helper with the GPU library, and the GPU library never calls it.
 *
 * Everything is IEEE double precision, written to be read against the paper:
 *   - measurement model b = A x + w ........................ Sec. 1, Eq. (1)
 *   - least-squares data term and its gradient A^T(Ax - b) .. Sec. 1, Eq. (2); Sec. 2.1, Eq. (5)
 *   - sketched objective f(b, A_s S(x)) ..................... Sec. 2.1, Eq. (4)
 *   - sketched gradient U(A_s^T A_s S(x) - A_s^T b) ......... Sec. 2.1, Eq. (6)
 *   - minibatch (view subset) form with M_k ................. Sec. 2.1, Eq. (7)
 *   - PnP-MS2G iteration (sketch, gradient, step, relaxed
 *     denoiser, momentum) ................................... Sec. 2.1, Algorithm 1
 *   - TV-prox as the denoiser D ............................. Sec. 2.1 (denoiser list after Eq. (5))
 *   - step eta = 1/L, momentum a_i = (i-1)/(i+3), alpha = 1 .. Sec. 3, experimental settings
 *
 * The paper fixes neither the projector nor the fan geometry nor the TV-prox
 * algorithm. The readings used here (all stated again where they are applied):
 *   geometry: pixel (r,c) centre ((c-(nx-1)/2) h, (r-(ny-1)/2) h), stored at
 *     x[r*nx + c]; view k at angle beta = angle0 + k*angle_step; source
 *     S = sod (cos b, sin b); detector centre C = (sod - sdd)(cos b, sin b);
 *     detector direction e_u = (-sin b, cos b); bin j centre
 *     Q_j = C + ((j - (B-1)/2) pitch + det_offset) e_u; ray direction d = Q_j - S.
 *   projector: Joseph's method, one ray per bin centre. A ray is x-major when
 *     |d_x| >= |d_y|; it is then sampled on every pixel-centre column by linear
 *     interpolation between the two nearest pixel-centre rows, pixels outside
 *     the grid being zero, and the sum is weighted by h |d| / |d_x|. y-major rays
 *     swap the roles of rows and columns.
 *   sketch S = average pooling D_f over f x f blocks; upsampler U = D_f^T
 *     (replicate, divide by f^2); A_s = the same projector on the (n/f) grid
 *     with pixel size f h.
 *   denoiser: Chambolle's dual projection iteration for isotropic TV with
 *     forward differences and Neumann boundary, p^0 = 0 on every call.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny;        /* full-resolution grid (pixels) */
    double pixel_mm;       /* full-resolution pixel size h */
    int32_t n_views, n_bins;
    double sod_mm, sdd_mm; /* source-to-isocentre, source-to-detector */
    double det_pitch_mm, det_offset_mm;
    double angle0_rad, angle_step_rad;
} orc_geom;

/* ------------------------------------------------------------------------- */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------- */

/* Source position and ray direction of (view k, bin j). */
static void orc_ray(const orc_geom* g, int k, int j, double* sx, double* sy, double* dx,
                    double* dy) {
    double beta = g->angle0_rad + (double)k * g->angle_step_rad;
    double cb = cos(beta), sb = sin(beta);
    double src_x = g->sod_mm * cb, src_y = g->sod_mm * sb;
    double cen_x = (g->sod_mm - g->sdd_mm) * cb, cen_y = (g->sod_mm - g->sdd_mm) * sb;
    double u = ((double)j - 0.5 * (double)(g->n_bins - 1)) * g->det_pitch_mm + g->det_offset_mm;
    double qx = cen_x + u * (-sb), qy = cen_y + u * cb;
    *sx = src_x;
    *sy = src_y;
    *dx = qx - src_x;
    *dy = qy - src_y;
}

void orc_ray_geometry(const orc_geom* g, int k, int j, double* out4) {
    orc_ray(g, k, j, &out4[0], &out4[1], &out4[2], &out4[3]);
}

/* Pixel value with zero outside the grid. */
static double pix(const double* x, int nx, int ny, int r, int c) {
    if (r < 0 || r >= ny || c < 0 || c >= nx) return 0.0;
    return x[(size_t)r * nx + c];
}

/* ------------------------------------------------------------------------- */
/* Joseph projector on a grid of nxs x nys pixels of size hs                  */
/* ------------------------------------------------------------------------- */

/*
 * One ray of the forward operator A_s (Sec. 1, Eq. (1); Sec. 2.1, Eq. (4)).
 * If count != NULL it receives the number of interpolation samples with at
 * least one in-grid tap of nonzero weight.
 */
static double joseph_ray(const orc_geom* g, int k, int j, int nxs, int nys, double hs,
                         const double* x, long* count) {
    double sx, sy, dx, dy;
    orc_ray(g, k, j, &sx, &sy, &dx, &dy);
    double len = sqrt(dx * dx + dy * dy);
    double acc = 0.0;
    long n_in = 0;
    if (fabs(dx) >= fabs(dy)) {
        /* x-major: one sample on every pixel-centre column */
        for (int c = 0; c < nxs; ++c) {
            double xc = ((double)c - 0.5 * (double)(nxs - 1)) * hs;
            double t = (xc - sx) / dx;
            double yv = sy + t * dy;
            double rho = yv / hs + 0.5 * (double)(nys - 1);
            double r0 = floor(rho);
            double w = rho - r0;
            int ir = (int)r0;
            if (rho > -1.0 && rho < (double)nys) n_in++;
            if (rho > -2.0 && rho < (double)nys + 1.0)
                acc += (1.0 - w) * pix(x, nxs, nys, ir, c) + w * pix(x, nxs, nys, ir + 1, c);
        }
        acc *= hs * len / fabs(dx);
    } else {
        /* y-major: one sample on every pixel-centre row */
        for (int r = 0; r < nys; ++r) {
            double yr = ((double)r - 0.5 * (double)(nys - 1)) * hs;
            double t = (yr - sy) / dy;
            double xv = sx + t * dx;
            double kap = xv / hs + 0.5 * (double)(nxs - 1);
            double c0 = floor(kap);
            double w = kap - c0;
            int ic = (int)c0;
            if (kap > -1.0 && kap < (double)nxs) n_in++;
            if (kap > -2.0 && kap < (double)nxs + 1.0)
                acc += (1.0 - w) * pix(x, nxs, nys, r, ic) + w * pix(x, nxs, nys, r, ic + 1);
        }
        acc *= hs * len / fabs(dy);
    }
    if (count) *count = n_in;
    return acc;
}

/*
 * Transpose of one ray: spread val along the ray with the identical weights.
 * Adds into xt (nys x nxs).
 */
static void joseph_ray_adjoint(const orc_geom* g, int k, int j, int nxs, int nys, double hs,
                               double val, double* xt) {
    double sx, sy, dx, dy;
    orc_ray(g, k, j, &sx, &sy, &dx, &dy);
    double len = sqrt(dx * dx + dy * dy);
    if (fabs(dx) >= fabs(dy)) {
        double wl = val * hs * len / fabs(dx);
        for (int c = 0; c < nxs; ++c) {
            double xc = ((double)c - 0.5 * (double)(nxs - 1)) * hs;
            double t = (xc - sx) / dx;
            double yv = sy + t * dy;
            double rho = yv / hs + 0.5 * (double)(nys - 1);
            if (!(rho > -2.0 && rho < (double)nys + 1.0)) continue;
            double r0 = floor(rho);
            double w = rho - r0;
            int ir = (int)r0;
            if (ir >= 0 && ir < nys) xt[(size_t)ir * nxs + c] += (1.0 - w) * wl;
            if (ir + 1 >= 0 && ir + 1 < nys) xt[(size_t)(ir + 1) * nxs + c] += w * wl;
        }
    } else {
        double wl = val * hs * len / fabs(dy);
        for (int r = 0; r < nys; ++r) {
            double yr = ((double)r - 0.5 * (double)(nys - 1)) * hs;
            double t = (yr - sy) / dy;
            double xv = sx + t * dx;
            double kap = xv / hs + 0.5 * (double)(nxs - 1);
            if (!(kap > -2.0 && kap < (double)nxs + 1.0)) continue;
            double c0 = floor(kap);
            double w = kap - c0;
            int ic = (int)c0;
            if (ic >= 0 && ic < nxs) xt[(size_t)r * nxs + ic] += (1.0 - w) * wl;
            if (ic + 1 >= 0 && ic + 1 < nxs) xt[(size_t)r * nxs + ic + 1] += w * wl;
        }
    }
}

static int view_of(const int32_t* views, int i) { return views ? views[i] : i; }

/*
 * Forward projection y = M A_s x on the grid coarsened by f.
 * x: (ny/f) x (nx/f); y: n_sel x n_bins, rows in the order of `views`
 * (views == NULL selects every view in order, n_sel = n_views).
 */
void orc_fp(const orc_geom* g, int f, const double* x, double* y, const int32_t* views,
            int n_sel) {
    int nxs = g->nx / f, nys = g->ny / f;
    double hs = g->pixel_mm * f;
    int nb = g->n_bins;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_sel; ++i) {
        int k = view_of(views, i);
        for (int j = 0; j < nb; ++j)
            y[(size_t)i * nb + j] = joseph_ray(g, k, j, nxs, nys, hs, x, NULL);
    }
}

/* Number of in-grid Joseph samples of M A_s (used to state projector work). */
long orc_count_samples(const orc_geom* g, int f, const int32_t* views, int n_sel) {
    int nxs = g->nx / f, nys = g->ny / f;
    double hs = g->pixel_mm * f;
    long total = 0;
    double* zero = (double*)calloc((size_t)nxs * nys, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int i = 0; i < n_sel; ++i) {
        int k = view_of(views, i);
        for (int j = 0; j < g->n_bins; ++j) {
            long c = 0;
            joseph_ray(g, k, j, nxs, nys, hs, zero, &c);
            total += c;
        }
    }
    free(zero);
    return total;
}

/*
 * Backprojection x = scale * (M A_s)^T y by scattering the forward weights.
 * The views are split into a fixed number of chunks, each accumulated in its
 * own buffer, and the chunks are summed in order, so the result does not depend
 * on the number of threads.
 */
#define ORC_BP_CHUNKS 16
void orc_bp(const orc_geom* g, int f, const double* y, double* x, const int32_t* views,
            int n_sel, double scale) {
    int nxs = g->nx / f, nys = g->ny / f;
    double hs = g->pixel_mm * f;
    int nb = g->n_bins;
    size_t npix = (size_t)nxs * nys;
    double* part = (double*)calloc(npix * ORC_BP_CHUNKS, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int ch = 0; ch < ORC_BP_CHUNKS; ++ch) {
        double* acc = part + (size_t)ch * npix;
        for (int i = ch; i < n_sel; i += ORC_BP_CHUNKS) {
            int k = view_of(views, i);
            for (int j = 0; j < nb; ++j) {
                double v = y[(size_t)i * nb + j];
                if (v != 0.0) joseph_ray_adjoint(g, k, j, nxs, nys, hs, v, acc);
            }
        }
    }
    for (size_t p = 0; p < npix; ++p) {
        double s = 0.0;
        for (int ch = 0; ch < ORC_BP_CHUNKS; ++ch) s += part[(size_t)ch * npix + p];
        x[p] = scale * s;
    }
    free(part);
}

/*
 * Dense matrix of M A_s for tiny grids, built column by column: column m is
 * the projection of the m-th unit image. A: (n_sel*n_bins) x (nxs*nys), row-major.
 */
void orc_dense_matrix(const orc_geom* g, int f, const int32_t* views, int n_sel, double* A) {
    int nxs = g->nx / f, nys = g->ny / f;
    size_t d = (size_t)nxs * nys, n = (size_t)n_sel * g->n_bins;
    double* e = (double*)calloc(d, sizeof(double));
    double* col = (double*)malloc(n * sizeof(double));
    for (size_t m = 0; m < d; ++m) {
        e[m] = 1.0;
        orc_fp(g, f, e, col, views, n_sel);
        for (size_t i = 0; i < n; ++i) A[i * d + m] = col[i];
        e[m] = 0.0;
    }
    free(e);
    free(col);
}

/* ------------------------------------------------------------------------- */
/* Sketch S = D_f (f x f average pooling) and upsampler U = D_f^T             */
/* ------------------------------------------------------------------------- */

void orc_down(const double* x, int nx, int ny, int f, double* v) {
    int nxs = nx / f, nys = ny / f;
    for (int R = 0; R < nys; ++R)
        for (int C = 0; C < nxs; ++C) {
            double s = 0.0;
            for (int a = 0; a < f; ++a)
                for (int b = 0; b < f; ++b) s += x[(size_t)(f * R + a) * nx + (f * C + b)];
            v[(size_t)R * nxs + C] = s / (double)(f * f);
        }
}

void orc_up(const double* v, int nxs, int nys, int f, double* x) {
    int nx = nxs * f, ny = nys * f;
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) x[(size_t)r * nx + c] = v[(size_t)(r / f) * nxs + c / f] / (double)(f * f);
}

/* ------------------------------------------------------------------------- */
/* Bicubic sketch (Sec. 3: resizing with bicubic interpolation)               */
/* ------------------------------------------------------------------------- */

/* Keys' cubic convolution kernel with a = -1/2. */
static double keys(double s) {
    const double a = -0.5, t = fabs(s);
    if (t <= 1.0) return ((a + 2.0) * t - (a + 3.0)) * t * t + 1.0;
    if (t < 2.0) return ((a * t - 5.0 * a) * t + 8.0 * a) * t - 4.0 * a;
    return 0.0;
}

/* Half-sample symmetric reflection of an index into [0, n). */
static int reflect(int i, int n) {
    while (i < 0 || i >= n) {
        if (i < 0) i = -1 - i;
        if (i >= n) i = 2 * n - 1 - i;
    }
    return i;
}

/*
 * The 1-D bicubic sketch, S (m x n, row-major, m = n / f). Output o sits at the
 * input coordinate u = (o + 1/2) f - 1/2 (pixel centres aligned as when n
 * pixels are resized to n / f); its weights are keys((i - u) / f) for the
 * inputs i with |i - u| < 2 f (the kernel stretched by f against aliasing),
 * folded into the image by half-sample reflection at both ends, then divided
 * by their sum. f = 1 gives the identity.
 */
void orc_bicubic_matrix(int n, int f, double* S) {
    const int m = n / f;
    memset(S, 0, (size_t)m * n * sizeof(double));
    for (int o = 0; o < m; ++o) {
        const double u = (o + 0.5) * f - 0.5;
        double sum = 0.0;
        for (int i = (int)floor(u - 2.0 * f); i <= (int)ceil(u + 2.0 * f); ++i) {
            const double w = keys((i - u) / f);
            if (w == 0.0) continue;
            S[(size_t)o * n + reflect(i, n)] += w;
            sum += w;
        }
        for (int i = 0; i < n; ++i) S[(size_t)o * n + i] /= sum;
    }
}

/* v = S x for the 2-D separable bicubic sketch (rows with S_x, columns with S_y). */
static void bicubic_down(const double* x, int nx, int ny, int f, double* v) {
    const int nxs = nx / f, nys = ny / f;
    double* Sx = (double*)malloc((size_t)nxs * nx * sizeof(double));
    double* Sy = (double*)malloc((size_t)nys * ny * sizeof(double));
    double* t = (double*)calloc((size_t)ny * nxs, sizeof(double));
    orc_bicubic_matrix(nx, f, Sx);
    orc_bicubic_matrix(ny, f, Sy);
    for (int r = 0; r < ny; ++r)
        for (int C = 0; C < nxs; ++C)
            for (int c = 0; c < nx; ++c) t[(size_t)r * nxs + C] += Sx[(size_t)C * nx + c] * x[(size_t)r * nx + c];
    for (int R = 0; R < nys; ++R)
        for (int C = 0; C < nxs; ++C) {
            double acc = 0.0;
            for (int r = 0; r < ny; ++r) acc += Sy[(size_t)R * ny + r] * t[(size_t)r * nxs + C];
            v[(size_t)R * nxs + C] = acc;
        }
    free(Sx);
    free(Sy);
    free(t);
}

/* x = S^T v, the adjoint of bicubic_down. */
static void bicubic_up(const double* v, int nxs, int nys, int f, double* x) {
    const int nx = nxs * f, ny = nys * f;
    double* Sx = (double*)malloc((size_t)nxs * nx * sizeof(double));
    double* Sy = (double*)malloc((size_t)nys * ny * sizeof(double));
    double* t = (double*)calloc((size_t)nys * nx, sizeof(double));
    orc_bicubic_matrix(nx, f, Sx);
    orc_bicubic_matrix(ny, f, Sy);
    for (int R = 0; R < nys; ++R)
        for (int C = 0; C < nxs; ++C)
            for (int c = 0; c < nx; ++c) t[(size_t)R * nx + c] += Sx[(size_t)C * nx + c] * v[(size_t)R * nxs + C];
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            double acc = 0.0;
            for (int R = 0; R < nys; ++R) acc += Sy[(size_t)R * ny + r] * t[(size_t)R * nx + c];
            x[(size_t)r * nx + c] = acc;
        }
    free(Sx);
    free(Sy);
    free(t);
}

/* The sketch S of kind 0 (f x f average pooling D) or 1 (bicubic), and U = S^T. */
void orc_sketch_down(int kind, const double* x, int nx, int ny, int f, double* v) {
    if (kind == 1) bicubic_down(x, nx, ny, f, v);
    else orc_down(x, nx, ny, f, v);
}

void orc_sketch_up(int kind, const double* v, int nxs, int nys, int f, double* x) {
    if (kind == 1) bicubic_up(v, nxs, nys, f, x);
    else orc_up(v, nxs, nys, f, x);
}

/* ------------------------------------------------------------------------- */
/* Sketched (minibatch) gradient, Sec. 2.1, Eqs. (6)-(7)                      */
/* ------------------------------------------------------------------------- */

/*
 * g = sigma * U (M A_s)^T (M A_s S(y) - M b) for the data term 1/2 ||A_s S y - b||^2.
 * b is the full sinogram (n_views x n_bins); M keeps the rows of `views`.
 * y and g are full-resolution (ny x nx).
 */
void orc_grad_k(const orc_geom* g, int kind, int f, const double* y, const double* b, const int32_t* views,
                int n_sel, double sigma, double* grad) {
    int nx = g->nx, ny = g->ny, nxs = nx / f, nys = ny / f, nb = g->n_bins;
    size_t ds = (size_t)nxs * nys, ns = (size_t)n_sel * nb;
    double* v = (double*)malloc(ds * sizeof(double));
    double* r = (double*)malloc(ns * sizeof(double));
    double* gs = (double*)malloc(ds * sizeof(double));
    orc_sketch_down(kind, y, nx, ny, f, v);
    orc_fp(g, f, v, r, views, n_sel);
    for (int i = 0; i < n_sel; ++i) {
        int k = view_of(views, i);
        for (int j = 0; j < nb; ++j) r[(size_t)i * nb + j] -= b[(size_t)k * nb + j];
    }
    orc_bp(g, f, r, gs, views, n_sel, sigma);
    orc_sketch_up(kind, gs, nxs, nys, f, grad);
    free(v);
    free(r);
    free(gs);
}

void orc_grad(const orc_geom* g, int f, const double* y, const double* b, const int32_t* views, int n_sel,
              double sigma, double* grad) {
    orc_grad_k(g, 0, f, y, b, views, n_sel, sigma, grad);
}

/* ------------------------------------------------------------------------- */
/* Denoiser: TV-prox by Chambolle's dual projection                           */
/* ------------------------------------------------------------------------- */

/* (div p)_{r,c} with p1 the row-direction and p2 the column-direction component. */
static void tv_div(const double* p1, const double* p2, int nx, int ny, double* dv) {
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            size_t i = (size_t)r * nx + c;
            double s = 0.0;
            if (r < ny - 1) s += p1[i];
            if (r > 0) s -= p1[i - nx];
            if (c < nx - 1) s += p2[i];
            if (c > 0) s -= p2[i - 1];
            dv[i] = s;
        }
}

/*
 * x = argmin_u 1/2 ||u - z||^2 + lambda TV(u), approximated by n_iter steps of
 *   p <- (p + tau grad(div p - z/lambda)) / (1 + tau |grad(div p - z/lambda)|)
 * from p = 0, then x = z - lambda div p. lambda == 0 returns z.
 */
void orc_tv_prox(const double* z, int nx, int ny, double lambda, int n_iter, double tau,
                 double* x) {
    size_t n = (size_t)nx * ny;
    if (lambda == 0.0) {
        memcpy(x, z, n * sizeof(double));
        return;
    }
    double* p1 = (double*)calloc(n, sizeof(double));
    double* p2 = (double*)calloc(n, sizeof(double));
    double* dv = (double*)calloc(n, sizeof(double));
    double* u = (double*)malloc(n * sizeof(double));
    for (int it = 0; it < n_iter; ++it) {
        tv_div(p1, p2, nx, ny, dv);
        for (size_t i = 0; i < n; ++i) u[i] = dv[i] - z[i] / lambda;
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)r * nx + c;
                double q1 = (r < ny - 1) ? u[i + nx] - u[i] : 0.0;
                double q2 = (c < nx - 1) ? u[i + 1] - u[i] : 0.0;
                double mag = sqrt(q1 * q1 + q2 * q2);
                double den = 1.0 + tau * mag;
                p1[i] = (p1[i] + tau * q1) / den;
                p2[i] = (p2[i] + tau * q2) / den;
            }
    }
    tv_div(p1, p2, nx, ny, dv);
    for (size_t i = 0; i < n; ++i) x[i] = z[i] - lambda * dv[i];
    free(p1);
    free(p2);
    free(dv);
    free(u);
}

/* ------------------------------------------------------------------------- */
/* PnP-MS2G loop, Sec. 2.1 Algorithm 1                                        */
/* ------------------------------------------------------------------------- */

/*
 * Runs T iterations from x_0 = y_0 = x0. Iteration t (1-based) uses
 *   factor[t-1]   pooling factor f of its stage,
 *   views + view_off[t-1], n_sel[t-1]   the minibatch M_t (view list),
 *   sigma[t-1]    minibatch scale (n_views / n_sel for an unbiased estimate),
 *   eta[t-1], a[t-1]   step and momentum,
 * and computes
 *   z   = y_{t-1} - eta_t * G(y_{t-1})
 *   x_t = (1 - alpha) z + alpha TV(z)
 *   y_t = x_t + a_t (x_t - x_{t-1}).
 * history (optional): T x (ny*nx) iterates x_t. x_out: x_T.
 */
void orc_pnp_run_k(const orc_geom* g, int kind, int T, const int32_t* factor, const int32_t* views,
                   const int32_t* view_off, const int32_t* n_sel, const double* sigma, const double* eta,
                   const double* a, double alpha, double lambda, int tv_iters, double tau, const double* b,
                   const double* x0, double* x_out, double* history) {
    size_t n = (size_t)g->nx * g->ny;
    double* x_prev = (double*)malloc(n * sizeof(double));
    double* y = (double*)malloc(n * sizeof(double));
    double* z = (double*)malloc(n * sizeof(double));
    double* x = (double*)malloc(n * sizeof(double));
    double* gr = (double*)malloc(n * sizeof(double));
    memcpy(x_prev, x0, n * sizeof(double));
    memcpy(y, x0, n * sizeof(double));
    for (int t = 0; t < T; ++t) {
        const int32_t* vw = views ? views + view_off[t] : NULL;
        int ns = views ? n_sel[t] : g->n_views;
        orc_grad_k(g, kind, factor[t], y, b, vw, ns, sigma[t], gr);
        for (size_t i = 0; i < n; ++i) z[i] = y[i] - eta[t] * gr[i];
        orc_tv_prox(z, g->nx, g->ny, lambda, tv_iters, tau, x);
        for (size_t i = 0; i < n; ++i) x[i] = (1.0 - alpha) * z[i] + alpha * x[i];
        for (size_t i = 0; i < n; ++i) y[i] = x[i] + a[t] * (x[i] - x_prev[i]);
        if (history) memcpy(history + (size_t)t * n, x, n * sizeof(double));
        memcpy(x_prev, x, n * sizeof(double));
    }
    memcpy(x_out, x_prev, n * sizeof(double));
    free(x_prev);
    free(y);
    free(z);
    free(x);
    free(gr);
}

void orc_pnp_run(const orc_geom* g, int T, const int32_t* factor, const int32_t* views, const int32_t* view_off,
                 const int32_t* n_sel, const double* sigma, const double* eta, const double* a, double alpha,
                 double lambda, int tv_iters, double tau, const double* b, const double* x0, double* x_out,
                 double* history) {
    orc_pnp_run_k(g, 0, T, factor, views, view_off, n_sel, sigma, eta, a, alpha, lambda, tv_iters, tau, b, x0,
                  x_out, history);
}

/* ------------------------------------------------------------------------- */
/* Variance-reduced minibatch gradient (Sec. 2.1, the estimators named after  */
/* Eq. (7); here SVRG over view subsets)                                      */
/* ------------------------------------------------------------------------- */

/*
 * G = g_M(y) - g_M(y_snap) + g(y_snap): the minibatch gradient of orc_grad at y,
 * corrected by the same minibatch at the snapshot y_snap and the full-view
 * gradient there (sigma scales both minibatch terms).
 */
void orc_grad_vr(const orc_geom* g, int f, const double* y, const double* b, const int32_t* views, int n_sel,
                 double sigma, const double* y_snap, double* grad) {
    size_t n = (size_t)g->nx * g->ny;
    double* gs = (double*)malloc(n * sizeof(double));
    double* gf = (double*)malloc(n * sizeof(double));
    orc_grad(g, f, y, b, views, n_sel, sigma, grad);
    orc_grad(g, f, y_snap, b, views, n_sel, sigma, gs);
    orc_grad(g, f, y_snap, b, NULL, g->n_views, 1.0, gf);
    for (size_t i = 0; i < n; ++i) grad[i] = grad[i] - gs[i] + gf[i];
    free(gs);
    free(gf);
}

/*
 * orc_pnp_run with a gradient mode per iteration: mode[t] = 0 the minibatch
 * gradient as in orc_pnp_run; 1 a snapshot: y_snap = y_{t-1} and the full-view
 * gradient there (the step's own gradient); 2 the variance-reduced gradient of
 * orc_grad_vr against the last snapshot (which must use the same factor).
 */
void orc_pnp_run_vr(const orc_geom* g, int T, const int32_t* factor, const int32_t* views,
                    const int32_t* view_off, const int32_t* n_sel, const double* sigma, const int32_t* mode,
                    const double* eta, const double* a, double alpha, double lambda, int tv_iters, double tau,
                    const double* b, const double* x0, double* x_out, double* history) {
    size_t n = (size_t)g->nx * g->ny;
    double* x_prev = (double*)malloc(n * sizeof(double));
    double* y = (double*)malloc(n * sizeof(double));
    double* z = (double*)malloc(n * sizeof(double));
    double* x = (double*)malloc(n * sizeof(double));
    double* gr = (double*)malloc(n * sizeof(double));
    double* y_snap = (double*)calloc(n, sizeof(double));
    memcpy(x_prev, x0, n * sizeof(double));
    memcpy(y, x0, n * sizeof(double));
    for (int t = 0; t < T; ++t) {
        const int32_t* vw = views ? views + view_off[t] : NULL;
        int ns = views ? n_sel[t] : g->n_views;
        if (mode[t] == 1) {
            memcpy(y_snap, y, n * sizeof(double));
            orc_grad(g, factor[t], y, b, NULL, g->n_views, 1.0, gr);
        } else if (mode[t] == 2) {
            orc_grad_vr(g, factor[t], y, b, vw, ns, sigma[t], y_snap, gr);
        } else {
            orc_grad(g, factor[t], y, b, vw, ns, sigma[t], gr);
        }
        for (size_t i = 0; i < n; ++i) z[i] = y[i] - eta[t] * gr[i];
        orc_tv_prox(z, g->nx, g->ny, lambda, tv_iters, tau, x);
        for (size_t i = 0; i < n; ++i) x[i] = (1.0 - alpha) * z[i] + alpha * x[i];
        for (size_t i = 0; i < n; ++i) y[i] = x[i] + a[t] * (x[i] - x_prev[i]);
        if (history) memcpy(history + (size_t)t * n, x, n * sizeof(double));
        memcpy(x_prev, x, n * sizeof(double));
    }
    memcpy(x_out, x_prev, n * sizeof(double));
    free(x_prev);
    free(y);
    free(z);
    free(x);
    free(gr);
    free(y_snap);
}

/* ------------------------------------------------------------------------- */
/* Lipschitz constant of the sketched data term (step eta = 1/L, Sec. 3)      */
/* ------------------------------------------------------------------------- */

/*
 * Power iteration on B^T B with B = A_s D_f over all views, from v = 1/sqrt(d):
 * v <- B^T B v / ||B^T B v||, n_iter times; returns ||B v||^2.
 */
double orc_power_lipschitz_k(const orc_geom* g, int kind, int f, int n_iter) {
    int nx = g->nx, ny = g->ny, nxs = nx / f, nys = ny / f;
    size_t d = (size_t)nx * ny, ds = (size_t)nxs * nys, ns = (size_t)g->n_views * g->n_bins;
    double* v = (double*)malloc(d * sizeof(double));
    double* w = (double*)malloc(d * sizeof(double));
    double* vs = (double*)malloc(ds * sizeof(double));
    double* ws = (double*)malloc(ds * sizeof(double));
    double* s = (double*)malloc(ns * sizeof(double));
    for (size_t i = 0; i < d; ++i) v[i] = 1.0 / sqrt((double)d);
    for (int it = 0; it < n_iter; ++it) {
        orc_sketch_down(kind, v, nx, ny, f, vs);
        orc_fp(g, f, vs, s, NULL, g->n_views);
        orc_bp(g, f, s, ws, NULL, g->n_views, 1.0);
        orc_sketch_up(kind, ws, nxs, nys, f, w);
        double nrm = 0.0;
        for (size_t i = 0; i < d; ++i) nrm += w[i] * w[i];
        nrm = sqrt(nrm);
        for (size_t i = 0; i < d; ++i) v[i] = w[i] / nrm;
    }
    orc_sketch_down(kind, v, nx, ny, f, vs);
    orc_fp(g, f, vs, s, NULL, g->n_views);
    double L = 0.0;
    for (size_t i = 0; i < ns; ++i) L += s[i] * s[i];
    free(v);
    free(w);
    free(vs);
    free(ws);
    free(s);
    return L;
}

double orc_power_lipschitz(const orc_geom* g, int f, int n_iter) { return orc_power_lipschitz_k(g, 0, f, n_iter); }

/* Peak signal-to-noise ratio with peak = max(ref) - min(ref), MSE over all pixels. */
double orc_psnr(const double* x, const double* ref, size_t n) {
    double lo = ref[0], hi = ref[0], se = 0.0;
    for (size_t i = 0; i < n; ++i) {
        if (ref[i] < lo) lo = ref[i];
        if (ref[i] > hi) hi = ref[i];
        double e = x[i] - ref[i];
        se += e * e;
    }
    double mse = se / (double)n;
    return 10.0 * log10((hi - lo) * (hi - lo) / mse);
}

/* ------------------------------------------------------------------------- */
/* Reverse mode (differentiation of the unrolled iteration)                  */
/* ------------------------------------------------------------------------- */

/*
 * zbar = J^T xbar for x = alpha_tv * (TV(z) - z) + z, i.e. the vector-Jacobian
 * product of the relaxed denoiser z -> (1 - alpha) z + alpha TV(z) with the
 * identity part kept at weight 1 (alpha_tv = alpha). The dual iterates p^n,
 * u^n = div p^n - z/lambda and q^n = grad u^n are recomputed, then the steps
 *   p^{n+1} = (p^n + tau q^n) / (1 + tau |q^n|),  x = z - lambda div p^K
 * are reversed. d|q|/dq is taken as 0 at q = 0.
 */
void orc_tv_relax_vjp(const double* z, const double* xbar, int nx, int ny, double lambda, int n_iter,
                      double tau, double alpha, double* zbar) {
    size_t n = (size_t)nx * ny;
    if (lambda == 0.0 || n_iter == 0) {
        memcpy(zbar, xbar, n * sizeof(double));
        return;
    }
    int K = n_iter;
    double* P1 = (double*)calloc(n * (K + 1), sizeof(double)); /* p^0..p^K, row part */
    double* P2 = (double*)calloc(n * (K + 1), sizeof(double)); /* column part */
    double* U = (double*)malloc(n * K * sizeof(double));
    double* dv = (double*)malloc(n * sizeof(double));
    for (int it = 0; it < K; ++it) {
        double *p1 = P1 + it * n, *p2 = P2 + it * n, *u = U + it * n;
        tv_div(p1, p2, nx, ny, dv);
        for (size_t i = 0; i < n; ++i) u[i] = dv[i] - z[i] / lambda;
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)r * nx + c;
                double q1 = (r < ny - 1) ? u[i + nx] - u[i] : 0.0;
                double q2 = (c < nx - 1) ? u[i + 1] - u[i] : 0.0;
                double den = 1.0 + tau * sqrt(q1 * q1 + q2 * q2);
                P1[(it + 1) * n + i] = (p1[i] + tau * q1) / den;
                P2[(it + 1) * n + i] = (p2[i] + tau * q2) / den;
            }
    }
    /* x = z - lambda div p^K, weighted by alpha on the denoiser path */
    double* pb1 = (double*)malloc(n * sizeof(double));
    double* pb2 = (double*)malloc(n * sizeof(double));
    double* qb1 = (double*)malloc(n * sizeof(double));
    double* qb2 = (double*)malloc(n * sizeof(double));
    double* ub = (double*)malloc(n * sizeof(double));
    memcpy(zbar, xbar, n * sizeof(double));
    /* adjoint of div: (div^T w)_1[r,c] = [r<ny-1](w[r,c] - w[r+1,c]), likewise columns */
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            size_t i = (size_t)r * nx + c;
            double w = -lambda * alpha * xbar[i];
            pb1[i] = (r < ny - 1) ? w - (-lambda * alpha * xbar[i + nx]) : 0.0;
            pb2[i] = (c < nx - 1) ? w - (-lambda * alpha * xbar[i + 1]) : 0.0;
        }
    for (int it = K - 1; it >= 0; --it) {
        const double* u = U + it * n;
        const double *pn1 = P1 + (it + 1) * n, *pn2 = P2 + (it + 1) * n;
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)r * nx + c;
                double q1 = (r < ny - 1) ? u[i + nx] - u[i] : 0.0;
                double q2 = (c < nx - 1) ? u[i + 1] - u[i] : 0.0;
                double mag = sqrt(q1 * q1 + q2 * q2);
                double den = 1.0 + tau * mag;
                double nb1 = pb1[i] / den, nb2 = pb2[i] / den;
                double db = -(pb1[i] * pn1[i] + pb2[i] * pn2[i]) / den;
                double magb = tau * db;
                qb1[i] = tau * nb1 + (mag > 0.0 ? magb * q1 / mag : 0.0);
                qb2[i] = tau * nb2 + (mag > 0.0 ? magb * q2 / mag : 0.0);
                pb1[i] = nb1;
                pb2[i] = nb2;
            }
        /* q = masked forward differences of u: u_bar = transpose applied to q_bar */
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)r * nx + c;
                double s = 0.0;
                if (r < ny - 1) s -= qb1[i];
                if (r > 0) s += qb1[i - nx];
                if (c < nx - 1) s -= qb2[i];
                if (c > 0) s += qb2[i - 1];
                ub[i] = s;
            }
        /* u = div p^n - z / lambda */
        for (int r = 0; r < ny; ++r)
            for (int c = 0; c < nx; ++c) {
                size_t i = (size_t)r * nx + c;
                if (r < ny - 1) pb1[i] += ub[i] - ub[i + nx];
                if (c < nx - 1) pb2[i] += ub[i] - ub[i + 1];
                zbar[i] -= ub[i] / lambda;
            }
    }
    free(P1);
    free(P2);
    free(U);
    free(dv);
    free(pb1);
    free(pb2);
    free(qb1);
    free(qb2);
    free(ub);
}

/*
 * Gradient of L(x_T) through T iterations of the loop of orc_pnp_run, given
 * xT_bar = dL/dx_T (y_T does not enter L). Outputs dL/dx_0 (with x_0 = y_0) and
 * dL/deta_t for every t. Each iteration's inputs (x_{t-1}, y_{t-1}) are kept;
 * its gradient and z are recomputed on the way back. With
 *   z = y - eta G(y),  G(y) = sigma U (M A_s)^T (M A_s S y - M b)  (affine, with
 *   symmetric linear part H = sigma U (M A_s)^T M A_s S),
 *   x_t = (1 - alpha) z + alpha D(z),  y_t = x_t + a_t (x_t - x_{t-1}):
 *   xbar_t += (1 + a_t) ybar_t;  xbar_{t-1} = -a_t ybar_t;
 *   zbar = J_relax^T xbar_t;  eta_bar_t = -<zbar, G(y_{t-1})>;
 *   ybar_{t-1} = zbar - eta_t H zbar.
 */
void orc_pnp_vjp(const orc_geom* g, int T, const int32_t* factor, const int32_t* views,
                 const int32_t* view_off, const int32_t* n_sel, const double* sigma, const double* eta,
                 const double* a, double alpha, double lambda, int tv_iters, double tau, const double* b,
                 const double* x0, const double* xT_bar, double* x0_bar, double* eta_bar) {
    size_t n = (size_t)g->nx * g->ny, nb = (size_t)g->n_views * g->n_bins;
    double* X = (double*)malloc(n * (T + 1) * sizeof(double)); /* x_0..x_T */
    double* Y = (double*)malloc(n * (T + 1) * sizeof(double)); /* y_0..y_T */
    double* gr = (double*)malloc(n * sizeof(double));
    double* z = (double*)malloc(n * sizeof(double));
    double* x = (double*)malloc(n * sizeof(double));
    double* zero_b = (double*)calloc(nb, sizeof(double));
    memcpy(X, x0, n * sizeof(double));
    memcpy(Y, x0, n * sizeof(double));
    for (int t = 0; t < T; ++t) {
        const int32_t* vw = views ? views + view_off[t] : NULL;
        int ns = views ? n_sel[t] : g->n_views;
        const double* y = Y + t * n;
        orc_grad(g, factor[t], y, b, vw, ns, sigma[t], gr);
        for (size_t i = 0; i < n; ++i) z[i] = y[i] - eta[t] * gr[i];
        orc_tv_prox(z, g->nx, g->ny, lambda, tv_iters, tau, x);
        double* xt = X + (t + 1) * n;
        double* yt = Y + (t + 1) * n;
        for (size_t i = 0; i < n; ++i) xt[i] = (1.0 - alpha) * z[i] + alpha * x[i];
        for (size_t i = 0; i < n; ++i) yt[i] = xt[i] + a[t] * (xt[i] - X[t * n + i]);
    }
    double* xb = (double*)malloc(n * sizeof(double));
    double* yb = (double*)calloc(n, sizeof(double));
    double* zb = (double*)malloc(n * sizeof(double));
    double* hz = (double*)malloc(n * sizeof(double));
    memcpy(xb, xT_bar, n * sizeof(double));
    for (int t = T - 1; t >= 0; --t) {
        const int32_t* vw = views ? views + view_off[t] : NULL;
        int ns = views ? n_sel[t] : g->n_views;
        const double* y = Y + t * n;
        orc_grad(g, factor[t], y, b, vw, ns, sigma[t], gr);
        for (size_t i = 0; i < n; ++i) z[i] = y[i] - eta[t] * gr[i];
        for (size_t i = 0; i < n; ++i) xb[i] += (1.0 + a[t]) * yb[i];
        orc_tv_relax_vjp(z, xb, g->nx, g->ny, lambda, tv_iters, tau, alpha, zb);
        double e = 0.0;
        for (size_t i = 0; i < n; ++i) e += zb[i] * gr[i];
        eta_bar[t] = -e;
        orc_grad(g, factor[t], zb, zero_b, vw, ns, sigma[t], hz); /* H zbar */
        for (size_t i = 0; i < n; ++i) {
            double ynew = zb[i] - eta[t] * hz[i];
            xb[i] = -a[t] * yb[i];
            yb[i] = ynew;
        }
    }
    for (size_t i = 0; i < n; ++i) x0_bar[i] = xb[i] + yb[i];
    free(X);
    free(Y);
    free(gr);
    free(z);
    free(x);
    free(zero_b);
    free(xb);
    free(yb);
    free(zb);
    free(hz);
}

/* Timing support (no arithmetic of the method): sets the number of OpenMP
 * threads later calls use (n <= 0 leaves it) and returns the number in force
 * before the call (1 when built without OpenMP). */
int orc_set_threads(int n) {
#ifdef _OPENMP
    const int prev = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return prev;
#else
    (void)n;
    return 1;
#endif
}
