// HIP kernels for gfx950 (MI355X) and the C ABI entry points of libfbpnp.
//
// Hot path of one PnP-MS2G iteration (Sec. 2.1, Algorithm 1 with the
// least-squares data term of Eq. (5)-(7)):
//   k_prepare  pooling S = D_f of y_{t-1} into the stage's two "line images"
//   k_fp       Joseph forward projection of the selected views, minus b
//   k_bp       matched backprojection as a pixel-driven gather, fused with the
//              upsampler U = D_f^T and the gradient step z = y - eta U G
//   k_tv       Chambolle TV-prox iterations in LDS, fused with the relaxation
//              and the momentum step
// None of these paths is a dense contraction, so no MFMA is used; the
// projectors gather and interpolate through the L1/L2 caches, laid out so that
// the 64 lanes of a wavefront touch consecutive addresses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fbpnp_impl.h"

using namespace fbpnp;

namespace {

// ---------------------------------------------------------------------------
// Line images: the stage image v (ny_s x nx_s) stored twice, as
//   lx[c][kPad + r] = v[r][c]   (lines = columns, used by x-major rays)
//   ly[r][kPad + c] = v[r][c]   (lines = rows, used by y-major rays)
// with kPad zeros at both ends of every line (written once at plan creation).
// Along a line, the rays of one view that a wavefront handles sample nearby
// positions, so their two interpolation taps are contiguous loads.
// ---------------------------------------------------------------------------
constexpr int kTile = 32;

// v = D_f x (x: ny x nx, full grid; f = 1 copies), written into both line images.
__global__ __launch_bounds__(256) void k_prepare(const float* __restrict__ x, int nx, int f, float inv_ff,
                                                 int nxs, int nys, float* __restrict__ lx, int pitch_x,
                                                 float* __restrict__ ly, int pitch_y) {
    __shared__ float tile[kTile][kTile + 1];
    const int C0 = blockIdx.x * kTile, R0 = blockIdx.y * kTile;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int rr = ty; rr < kTile; rr += 8) {
        const int R = R0 + rr, C = C0 + tx;
        float s = 0.f;
        if (R < nys && C < nxs) {
            if (f == 1) {
                s = x[(size_t)R * nx + C];
            } else {
                for (int a = 0; a < f; ++a) {
                    const float* row = x + (size_t)(f * R + a) * nx + (size_t)f * C;
                    for (int b = 0; b < f; ++b) s += row[b];
                }
                s *= inv_ff;
            }
            ly[(size_t)R * pitch_y + kPad + C] = s;
        }
        tile[rr][tx] = s;
    }
    __syncthreads();
    for (int cc = ty; cc < kTile; cc += 8) {
        const int C = C0 + cc, R = R0 + tx;
        if (R < nys && C < nxs) lx[(size_t)C * pitch_x + kPad + R] = tile[tx][cc];
    }
}

// ---------------------------------------------------------------------------
// Forward projection: one work-item per (selected view, bin). The lanes of a
// wavefront are 64 consecutive bins of one view, so the sinogram write and the
// ray-table read are coalesced and the taps fall on neighbouring positions of
// the same line.
//   y[i][j] = len_j * sum_k [ (1-w) v(line lo+k, p0) + w v(line lo+k, p0+1) ]
//             (- b[view_i][j] when kResid)
// with p = npos/2 + fma(k - n/2, dpos, pos_mid), p0 = floor(p), w = p - p0
// (zero outside the grid).
// ---------------------------------------------------------------------------
template <bool kResid>
__global__ __launch_bounds__(256) void k_fp(const RayRec* __restrict__ rays, int n_bins, int bins_padded,
                                            const int32_t* __restrict__ views, int n_sel, int n_views,
                                            const float* __restrict__ lx, int pitch_x,
                                            const float* __restrict__ ly, int pitch_y, int nxs, int nys,
                                            const float* __restrict__ b, float* __restrict__ y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / bins_padded;
    const int j = t - i * bins_padded;
    if (i >= n_sel || j >= n_bins) return;
    const int v = views ? views[i] : i;
    if ((unsigned)v >= (unsigned)n_views) {  // invalid view index: a zero row
        y[(size_t)i * n_bins + j] = 0.f;
        return;
    }
    const RayRec r = rays[(size_t)v * n_bins + j];
    const uint32_t lo = r.bits & 0xFFFFu, n = (r.bits >> 16) & 0x7FFFu;
    const bool ymaj = (r.bits >> 31) != 0u;
    const int pitch = ymaj ? pitch_y : pitch_x;
    const int npos = ymaj ? nxs : nys;
    const int mid = npos >> 1;
    const float* line = (ymaj ? ly : lx) + (size_t)lo * pitch + kPad + mid;
    // clamping keeps both taps inside the zero padding; it never changes a
    // sample whose taps touch the grid
    const float plo = (float)(-2 - mid), phi = (float)(npos - mid);
    float acc = 0.f, kf = -(float)(n >> 1);
#pragma unroll 4
    for (uint32_t k = 0; k < n; ++k) {
        float p = fmaf(kf, r.dpos, r.pos_mid);
        p = fminf(fmaxf(p, plo), phi);
        const float p0 = floorf(p);
        const float w = p - p0;
        const float* q = line + (int)p0;
        const float a = q[0], c = q[1];
        acc += fmaf(w, c - a, a);
        kf += 1.f;
        line += pitch;
    }
    float val = acc * r.len;
    if (kResid) val -= b[(size_t)v * n_bins + j];
    y[(size_t)i * n_bins + j] = val;
}

// ---------------------------------------------------------------------------
// Matched backprojection, pixel-driven gather.
//
// A wavefront owns a 16 x 16 block of stage pixels, each lane a 2 x 2 block
// (rows r, r+1, columns c, c+1). For every selected view the lane finds the
// rays that can touch its pixels from the detector coordinate j(c, r) of the
// segment ends, and recomputes each candidate's interpolation weight exactly
// as k_fp does (same float operations on the same table entries):
//   x-major ray, column cc: p = nys/2 + fma(cc - lo - n/2, dpos, pos_mid),
//   p0 = floor(p), w = p - p0; row p0 receives (1-w) and row p0+1 receives w.
// The VG wavefronts of a workgroup share the pixel block and split the views;
// their partial sums are added in a fixed order in LDS, so results are
// bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr float kProjEps = 0.02f;  // margin on candidate bin ranges (FP32 error is ~1e-4 bins)

__device__ __forceinline__ float proj_bin(const ViewRec& v, float c, float r) {
    const float num = fmaf(v.a2, r, fmaf(v.a1, c, v.a0));
    const float den = fmaf(v.b2, r, fmaf(v.b1, c, v.b0));
    return num / den + v.j0;
}

// Accumulates the contributions of the candidate rays jl..jh (one class) to a
// strip of two pixels at line l, positions q and q+1; qm = q - npos/2.
__device__ __forceinline__ void gather_strip(const RayRec* __restrict__ rv, const float* __restrict__ yv, int jl,
                                             int jh, int l, int qm, float& s0, float& s1) {
    const float qf = (float)qm;
    for (int j = jl; j <= jh; ++j) {
        const RayRec rr = rv[j];
        const float yy = yv[j] * rr.len;
        const uint32_t lo = rr.bits & 0xFFFFu, n = (rr.bits >> 16) & 0x7FFFu;
        const uint32_t k = (uint32_t)l - lo;
        if (k < n) {
            const float p = fmaf((float)((int)k - (int)(n >> 1)), rr.dpos, rr.pos_mid);
            const float p0 = floorf(p);
            const float w = p - p0;
            const float om = 1.f - w;
            const float d = p0 - qf;
            s0 = fmaf(d == 0.f ? om : (d == -1.f ? w : 0.f), yy, s0);
            s1 = fmaf(d == 1.f ? om : (d == 0.f ? w : 0.f), yy, s1);
        }
    }
}

__device__ __forceinline__ void cand_range(float j1, float j2, int lo, int hi, int& jl, int& jh) {
    const float a = fmaxf(ceilf(fminf(j1, j2) - kProjEps), (float)lo);
    const float b = fminf(floorf(fmaxf(j1, j2) + kProjEps), (float)hi);
    jl = (int)a;
    jh = (int)b;
}

template <int VG, bool kFused>
__global__ __launch_bounds__(64 * VG) void k_bp(const RayRec* __restrict__ rays, const ViewRec* __restrict__ vrec,
                                                int n_bins, const int32_t* __restrict__ views, int n_sel,
                                                int n_views, const float* __restrict__ y, int nxs, int nys,
                                                int blocks_x,
                                                float scale, float* __restrict__ xo, int f, int nx,
                                                const float* __restrict__ yprev, float* __restrict__ z) {
    __shared__ float red[VG > 1 ? VG - 1 : 1][4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bx = blockIdx.x % blocks_x, by = blockIdx.x / blocks_x;
    const int c = bx * 16 + 2 * (lane & 7), r = by * 16 + 2 * (lane >> 3);
    const float cc = (float)c - 0.5f * (float)(nxs - 1), rc = (float)r - 0.5f * (float)(nys - 1);
    float a00 = 0.f, a01 = 0.f, a10 = 0.f, a11 = 0.f;  // (r,c) (r,c+1) (r+1,c) (r+1,c+1)
    for (int i = wave; i < n_sel; i += VG) {
        const int v = __builtin_amdgcn_readfirstlane(views ? views[i] : i);
        if ((unsigned)v >= (unsigned)n_views) continue;  // invalid view index: no contribution
        const ViewRec vr = vrec[v];
        const RayRec* rv = rays + (size_t)v * n_bins;
        const float* yv = y + (size_t)i * n_bins;
        if (vr.xlo <= vr.xhi) {
            int jl, jh;
            cand_range(proj_bin(vr, cc, rc - 1.f), proj_bin(vr, cc, rc + 2.f), vr.xlo, vr.xhi, jl, jh);
            gather_strip(rv, yv, jl, jh, c, r - (nys >> 1), a00, a10);
            cand_range(proj_bin(vr, cc + 1.f, rc - 1.f), proj_bin(vr, cc + 1.f, rc + 2.f), vr.xlo, vr.xhi, jl, jh);
            gather_strip(rv, yv, jl, jh, c + 1, r - (nys >> 1), a01, a11);
        }
        if (vr.ylo <= vr.yhi) {
            int jl, jh;
            cand_range(proj_bin(vr, cc - 1.f, rc), proj_bin(vr, cc + 2.f, rc), vr.ylo, vr.yhi, jl, jh);
            gather_strip(rv, yv, jl, jh, r, c - (nxs >> 1), a00, a01);
            cand_range(proj_bin(vr, cc - 1.f, rc + 1.f), proj_bin(vr, cc + 2.f, rc + 1.f), vr.ylo, vr.yhi, jl,
                       jh);
            gather_strip(rv, yv, jl, jh, r + 1, c - (nxs >> 1), a10, a11);
        }
    }
    if (VG > 1) {
        if (wave > 0) {
            red[wave - 1][0][lane] = a00;
            red[wave - 1][1][lane] = a01;
            red[wave - 1][2][lane] = a10;
            red[wave - 1][3][lane] = a11;
        }
        __syncthreads();
        if (wave > 0) return;
        for (int w = 0; w < VG - 1; ++w) {
            a00 += red[w][0][lane];
            a01 += red[w][1][lane];
            a10 += red[w][2][lane];
            a11 += red[w][3][lane];
        }
    }
    const float g[2][2] = {{a00, a01}, {a10, a11}};
    for (int dr = 0; dr < 2; ++dr)
        for (int dc = 0; dc < 2; ++dc) {
            const int R = r + dr, C = c + dc;
            if (R >= nys || C >= nxs) continue;
            if (!kFused) {
                xo[(size_t)R * nxs + C] = scale * g[dr][dc];
            } else {
                // z = y_prev - (eta sigma / f^2) g on the f x f block of (R, C)
                const float s = scale * g[dr][dc];
                for (int a = 0; a < f; ++a) {
                    const size_t row = (size_t)(f * R + a) * nx + (size_t)f * C;
                    for (int bb = 0; bb < f; ++bb) z[row + bb] = yprev[row + bb] - s;
                }
            }
        }
}

// ---------------------------------------------------------------------------
// TV-prox (Chambolle's dual projection), n_iter <= H-1 steps per launch with
// the tile and a halo of H cells held in LDS. Cells within H of the tile edge
// see incomplete neighbourhoods; the error travels one cell per step, so the
// T x T output tile stays exact.
//   mode 0: x_out = z - lambda div p
//   mode 1: x = (1-alpha) z + alpha (z - lambda div p); y_out = x + a_t (x - x_prev);
//           x_out = x; hist (optional) = x
//   p_in/p_out: optional global dual field [2][ny][nx] for multi-launch runs
//   (p_out set: the launch stores p for its tile instead of producing x).
// ---------------------------------------------------------------------------
template <int T, int H>
__global__ __launch_bounds__(256) void k_tv(const float* __restrict__ z, int nx, int ny, float lam, float tau,
                                            int n_iter, const float* __restrict__ p_in, float* __restrict__ p_out,
                                            int mode, float alpha, float a_t, const float* __restrict__ x_prev,
                                            float* __restrict__ x_out, float* __restrict__ y_out,
                                            float* __restrict__ hist) {
    constexpr int S = T + 2 * H;
    __shared__ float sz[S * S], sp1[S * S], sp2[S * S], su[S * S];
    const int R0 = blockIdx.y * T - H, C0 = blockIdx.x * T - H;
    const size_t plane = (size_t)nx * ny;
    for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
        const int lr = e / S, lc = e - lr * S;
        const int gr = R0 + lr, gc = C0 + lc;
        const bool in = gr >= 0 && gr < ny && gc >= 0 && gc < nx;
        const size_t gi = (size_t)gr * nx + gc;
        sz[e] = in ? z[gi] : 0.f;
        sp1[e] = (in && p_in) ? p_in[gi] : 0.f;
        sp2[e] = (in && p_in) ? p_in[plane + gi] : 0.f;
    }
    __syncthreads();
    const float il = 1.f / lam;
    for (int it = 0; it < n_iter; ++it) {
        for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
            const int lr = e / S, lc = e - lr * S;
            const int gr = R0 + lr, gc = C0 + lc;
            float d = 0.f;
            if (gr < ny - 1) d += sp1[e];
            if (gr > 0 && lr > 0) d -= sp1[e - S];
            if (gc < nx - 1) d += sp2[e];
            if (gc > 0 && lc > 0) d -= sp2[e - 1];
            su[e] = d - sz[e] * il;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
            const int lr = e / S, lc = e - lr * S;
            const int gr = R0 + lr, gc = C0 + lc;
            if (gr < 0 || gr >= ny || gc < 0 || gc >= nx) continue;
            const float q1 = (gr < ny - 1 && lr < S - 1) ? su[e + S] - su[e] : 0.f;
            const float q2 = (gc < nx - 1 && lc < S - 1) ? su[e + 1] - su[e] : 0.f;
            const float den = 1.f + tau * sqrtf(q1 * q1 + q2 * q2);
            sp1[e] = (sp1[e] + tau * q1) / den;
            sp2[e] = (sp2[e] + tau * q2) / den;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int tr = e / T, tc = e - tr * T;
        const int gr = R0 + H + tr, gc = C0 + H + tc;
        if (gr >= ny || gc >= nx) continue;
        const int l = (H + tr) * S + (H + tc);
        const size_t gi = (size_t)gr * nx + gc;
        if (p_out) {
            p_out[gi] = sp1[l];
            p_out[plane + gi] = sp2[l];
            continue;
        }
        float d = 0.f;
        if (gr < ny - 1) d += sp1[l];
        if (gr > 0) d -= sp1[l - S];
        if (gc < nx - 1) d += sp2[l];
        if (gc > 0) d -= sp2[l - 1];
        const float zz = sz[l];
        const float den = zz - lam * d;
        if (mode == 0) {
            x_out[gi] = den;
        } else {
            const float xr = (1.f - alpha) * zz + alpha * den;
            const float yn = xr + a_t * (xr - x_prev[gi]);
            x_out[gi] = xr;
            y_out[gi] = yn;
            if (hist) hist[gi] = xr;
        }
    }
}

// ---------------------------------------------------------------------------
// Standalone sketch kernels and reductions.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_down(const float* __restrict__ x, int nx, int f, float inv_ff, int nxs,
                                              int nys, float* __restrict__ v) {
    const int C = blockIdx.x * blockDim.x + threadIdx.x, R = blockIdx.y;
    if (C >= nxs || R >= nys) return;
    float s = 0.f;
    for (int a = 0; a < f; ++a) {
        const float* row = x + (size_t)(f * R + a) * nx + (size_t)f * C;
        for (int b = 0; b < f; ++b) s += row[b];
    }
    v[(size_t)R * nxs + C] = f == 1 ? s : s * inv_ff;
}

__global__ __launch_bounds__(256) void k_up(const float* __restrict__ v, int nxs, int f, float inv_ff, int nx,
                                            int ny, float* __restrict__ x) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= nx || r >= ny) return;
    x[(size_t)r * nx + c] = v[(size_t)(r / f) * nxs + c / f] * inv_ff;
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ a, size_t n, float val) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = val;
}

// Per-block sums of squares in double, in a fixed order.
constexpr int kRedBlocks = 256;
__global__ __launch_bounds__(256) void k_sumsq_partial(const float* __restrict__ a, size_t n,
                                                       double* __restrict__ part) {
    __shared__ double s[256];
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc += (double)a[i] * (double)a[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ part, int nparts,
                                                   double* __restrict__ out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

__global__ __launch_bounds__(256) void k_normalise(const float* __restrict__ w, float* __restrict__ v, size_t n,
                                                   const double* __restrict__ sumsq) {
    const float inv = (float)(1.0 / sqrt(sumsq[0]));
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        v[i] = w[i] * inv;
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
inline int cdiv(int a, int b) { return (a + b - 1) / b; }

fb_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return FB_OK;
}

fb_status check_stage(const fb_plan* p, int stage) {
    if (!p) return fail(FB_EINVAL, "plan is NULL");
    if (stage < 0 || stage >= (int)p->stages.size()) return fail(FB_EINVAL, "stage index out of range");
    return FB_OK;
}

fb_status check_views(const fb_plan* p, const int32_t* views, int n_sel) {
    if (n_sel < 1) return fail(FB_EINVAL, "n_sel must be positive");
    if (!views && n_sel != p->g.n_views) return fail(FB_EINVAL, "views == NULL requires n_sel == n_views");
    if (n_sel > p->g.n_views) return fail(FB_ESUBSET, "more selected views than views in the geometry");
    return FB_OK;
}

struct StageLines {
    float* lx;
    float* ly;
};

// Line images of a stage live in one plan allocation, one region per stage.
StageLines stage_lines(const fb_plan* p, int stage) {
    size_t off = 0;
    for (int s = 0; s < stage; ++s) {
        const Stage& st = p->stages[s];
        off += (size_t)st.nxs * st.pitch_x + (size_t)st.nys * st.pitch_y;
    }
    const Stage& st = p->stages[stage];
    return {p->line_x + off, p->line_x + off + (size_t)st.nxs * st.pitch_x};
}

fb_status launch_prepare(const fb_plan* p, int stage, const float* x, int nx, int f, hipStream_t s) {
    const Stage& st = p->stages[stage];
    StageLines L = stage_lines(p, stage);
    dim3 grid(cdiv(st.nxs, kTile), cdiv(st.nys, kTile));
    k_prepare<<<grid, 256, 0, s>>>(x, nx, f, 1.f / (float)(f * f), st.nxs, st.nys, L.lx, st.pitch_x, L.ly,
                                   st.pitch_y);
    return check_launch("prepare");
}

fb_status launch_fp(const fb_plan* p, int stage, bool resid, const int32_t* views, int n_sel, const float* b,
                    float* y, hipStream_t s) {
    const Stage& st = p->stages[stage];
    StageLines L = stage_lines(p, stage);
    const int nb = p->g.n_bins, bp = cdiv(nb, 64) * 64;
    const int blocks = cdiv(n_sel * bp, 256);
    if (resid)
        k_fp<true><<<blocks, 256, 0, s>>>(st.rays, nb, bp, views, n_sel, p->g.n_views, L.lx, st.pitch_x, L.ly, st.pitch_y, st.nxs,
                                          st.nys, b, y);
    else
        k_fp<false><<<blocks, 256, 0, s>>>(st.rays, nb, bp, views, n_sel, p->g.n_views, L.lx, st.pitch_x, L.ly, st.pitch_y,
                                           st.nxs, st.nys, b, y);
    return check_launch("fanbeam_fp");
}

template <bool kFused>
fb_status launch_bp_t(const fb_plan* p, int stage, const float* y, const int32_t* views, int n_sel, float scale,
                      float* xo, const float* yprev, float* z, hipStream_t s) {
    const Stage& st = p->stages[stage];
    const int bxs = cdiv(st.nxs, 16), bys = cdiv(st.nys, 16), nblk = bxs * bys;
    int vg = 1;
    while (vg < 16 && nblk * vg < 2048 && vg * 2 <= n_sel) vg *= 2;
    const int nb = p->g.n_bins, f = st.f, nx = p->g.nx;
#define FB_BP(VG)                                                                                           \
    k_bp<VG, kFused><<<nblk, 64 * VG, 0, s>>>(st.rays, st.vrec, nb, views, n_sel, p->g.n_views, y, st.nxs,      \
                                              st.nys, bxs, scale,                                              \
                                              xo, f, nx, yprev, z)
    switch (vg) {
        case 1: FB_BP(1); break;
        case 2: FB_BP(2); break;
        case 4: FB_BP(4); break;
        case 8: FB_BP(8); break;
        default: FB_BP(16); break;
    }
#undef FB_BP
    return check_launch("fanbeam_bp");
}

constexpr int kTvT = 32;
constexpr int kTvMaxFused = 8;

fb_status launch_tv_single(const float* z, int nx, int ny, float lam, float tau, int n_iter, const float* p_in,
                           float* p_out, int mode, float alpha, float a_t, const float* x_prev, float* x_out,
                           float* y_out, float* hist, hipStream_t s) {
    dim3 grid(cdiv(nx, kTvT), cdiv(ny, kTvT));
    if (n_iter <= 5)
        k_tv<kTvT, 6><<<grid, 256, 0, s>>>(z, nx, ny, lam, tau, n_iter, p_in, p_out, mode, alpha, a_t, x_prev,
                                          x_out, y_out, hist);
    else
        k_tv<kTvT, kTvMaxFused + 1><<<grid, 256, 0, s>>>(z, nx, ny, lam, tau, n_iter, p_in, p_out, mode, alpha,
                                                         a_t, x_prev, x_out, y_out, hist);
    return check_launch("tv_prox");
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

fb_status fb_plan_create(const fb_geom* geom, int n_stages, const int32_t* factors, fb_plan** out) {
    if (!geom || !factors || !out || n_stages < 1) return fail(FB_EINVAL, "fb_plan_create: bad arguments");
    *out = nullptr;
    fb_status st = validate_geometry(*geom);
    if (st != FB_OK) return st;
    for (int s = 0; s < n_stages; ++s) {
        const int f = factors[s];
        if (f < 1) return fail(FB_EINVAL, "pooling factor must be >= 1");
        if (geom->nx % f || geom->ny % f) return fail(FB_EDIV, "image size not divisible by the pooling factor");
    }
    fb_plan* p = new fb_plan();
    p->g = *geom;
    (void)hipGetDevice(&p->device);
    auto cleanup = [&](fb_status code) {
        fb_plan_destroy(p);
        return code;
    };
    size_t line_floats = 0;
    for (int s = 0; s < n_stages; ++s) {
        Stage S;
        S.f = factors[s];
        S.nxs = geom->nx / S.f;
        S.nys = geom->ny / S.f;
        S.pitch_x = ((S.nys + 2 * kPad + 3) / 4) * 4;
        S.pitch_y = ((S.nxs + 2 * kPad + 3) / 4) * 4;
        std::vector<RayRec> rays;
        std::vector<ViewRec> vr;
        st = build_stage_tables(*geom, S.f, rays, vr, S.samples);
        if (st != FB_OK) return cleanup(st);
        if (hipMalloc(&S.rays, rays.size() * sizeof(RayRec)) != hipSuccess ||
            hipMalloc(&S.vrec, vr.size() * sizeof(ViewRec)) != hipSuccess) {
            p->stages.push_back(S);
            return cleanup(fail(FB_ENOMEM, "plan: device allocation failed"));
        }
        p->stages.push_back(S);
        hipError_t e = hipMemcpy(S.rays, rays.data(), rays.size() * sizeof(RayRec), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(S.vrec, vr.data(), vr.size() * sizeof(ViewRec), hipMemcpyHostToDevice);
        if (e != hipSuccess) return cleanup(hip_fail(e, "plan: table upload"));
        line_floats += (size_t)S.nxs * S.pitch_x + (size_t)S.nys * S.pitch_y;
    }
    const size_t npix = (size_t)geom->nx * geom->ny, nsino = (size_t)geom->n_views * geom->n_bins;
    p->vec_floats = 3 * npix + 2 + 2 * (kRedBlocks + 1);
    if (hipMalloc(&p->line_x, line_floats * sizeof(float)) != hipSuccess ||
        hipMalloc(&p->resid, nsino * sizeof(float)) != hipSuccess ||
        hipMalloc(&p->zbuf, npix * sizeof(float)) != hipSuccess ||
        hipMalloc(&p->vec, p->vec_floats * sizeof(float)) != hipSuccess)
        return cleanup(fail(FB_ENOMEM, "plan: workspace allocation failed"));
    hipError_t e = hipMemset(p->line_x, 0, line_floats * sizeof(float));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return cleanup(hip_fail(e, "plan: workspace init"));
    *out = p;
    return FB_OK;
}

fb_status fb_plan_destroy(fb_plan* p) {
    if (!p) return FB_OK;
    for (Stage& s : p->stages) {
        if (s.rays) (void)hipFree(s.rays);
        if (s.vrec) (void)hipFree(s.vrec);
    }
    if (p->line_x) (void)hipFree(p->line_x);
    if (p->resid) (void)hipFree(p->resid);
    if (p->zbuf) (void)hipFree(p->zbuf);
    if (p->vec) (void)hipFree(p->vec);
    delete p;
    return FB_OK;
}

fb_status fb_plan_stage_info(const fb_plan* p, int stage, fb_stage_info* out) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!out) return fail(FB_EINVAL, "out is NULL");
    const Stage& S = p->stages[stage];
    out->factor = S.f;
    out->nxs = S.nxs;
    out->nys = S.nys;
    out->samples_all_views = S.samples;
    return FB_OK;
}

fb_status fanbeam_fp(const fb_plan* p, int stage, const float* x, float* y, const int32_t* views, int n_sel,
                     hipStream_t stream) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!x || !y) return fail(FB_EINVAL, "fanbeam_fp: x and y must not be NULL");
    if ((st = check_views(p, views, n_sel)) != FB_OK) return st;
    const Stage& S = p->stages[stage];
    if ((st = launch_prepare(p, stage, x, S.nxs, 1, stream)) != FB_OK) return st;
    return launch_fp(p, stage, false, views, n_sel, nullptr, y, stream);
}

fb_status fanbeam_bp(const fb_plan* p, int stage, const float* y, float* x, const int32_t* views, int n_sel,
                     float scale, hipStream_t stream) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!x || !y) return fail(FB_EINVAL, "fanbeam_bp: x and y must not be NULL");
    if ((st = check_views(p, views, n_sel)) != FB_OK) return st;
    return launch_bp_t<false>(p, stage, y, views, n_sel, scale, x, nullptr, nullptr, stream);
}

fb_status sketch_down(const float* x, int nx, int ny, int f, float* v, hipStream_t stream) {
    if (!x || !v || nx < 1 || ny < 1 || f < 1) return fail(FB_EINVAL, "sketch_down: bad arguments");
    if (nx % f || ny % f) return fail(FB_EDIV, "sketch_down: size not divisible by f");
    const int nxs = nx / f, nys = ny / f;
    k_down<<<dim3(cdiv(nxs, 256), nys), 256, 0, stream>>>(x, nx, f, 1.f / (float)(f * f), nxs, nys, v);
    return check_launch("sketch_down");
}

fb_status sketch_up(const float* v, int nxs, int nys, int f, float* x, hipStream_t stream) {
    if (!x || !v || nxs < 1 || nys < 1 || f < 1) return fail(FB_EINVAL, "sketch_up: bad arguments");
    const int nx = nxs * f, ny = nys * f;
    k_up<<<dim3(cdiv(nx, 256), ny), 256, 0, stream>>>(v, nxs, f, 1.f / (float)(f * f), nx, ny, x);
    return check_launch("sketch_up");
}

size_t fb_tv_workspace_bytes(int nx, int ny, int n_iter) {
    if (n_iter <= kTvMaxFused || nx < 1 || ny < 1) return 0;
    return 4 * (size_t)nx * ny * sizeof(float);
}

fb_status tv_prox(const float* z, float* x, int nx, int ny, float lambda, int n_iter, float tau, void* ws,
                  size_t ws_bytes, hipStream_t stream) {
    if (!z || !x || nx < 1 || ny < 1 || n_iter < 0) return fail(FB_EINVAL, "tv_prox: bad arguments");
    if (!(lambda >= 0.f) || !(tau > 0.f)) return fail(FB_EINVAL, "tv_prox: need lambda >= 0 and tau > 0");
    if (z == x) return fail(FB_EINVAL, "tv_prox: z and x must not alias");
    if (lambda == 0.f || n_iter == 0) {
        hipError_t e = hipMemcpyAsync(x, z, (size_t)nx * ny * sizeof(float), hipMemcpyDeviceToDevice, stream);
        return e == hipSuccess ? FB_OK : hip_fail(e, "tv_prox copy");
    }
    if (n_iter <= kTvMaxFused)
        return launch_tv_single(z, nx, ny, lambda, tau, n_iter, nullptr, nullptr, 0, 0.f, 0.f, nullptr, x, nullptr,
                                nullptr, stream);
    const size_t need = fb_tv_workspace_bytes(nx, ny, n_iter);
    if (!ws || ws_bytes < need) return fail(FB_EINVAL, "tv_prox: workspace too small");
    float* pa = (float*)ws;
    float* pb = pa + 2 * (size_t)nx * ny;
    const float* pin = nullptr;
    int left = n_iter;
    fb_status st;
    while (left > 0) {
        const int m = std::min(left, kTvMaxFused);
        st = launch_tv_single(z, nx, ny, lambda, tau, m, pin, pa, 0, 0.f, 0.f, nullptr, nullptr, nullptr, nullptr,
                              stream);
        if (st != FB_OK) return st;
        pin = pa;
        std::swap(pa, pb);
        left -= m;
    }
    return launch_tv_single(z, nx, ny, lambda, tau, 0, pin, nullptr, 0, 0.f, 0.f, nullptr, x, nullptr, nullptr,
                            stream);
}

fb_status pnp_step(const fb_plan* p, const fb_pnp_args* a, hipStream_t stream) {
    if (!a) return fail(FB_EINVAL, "pnp_step: args is NULL");
    fb_status st = check_stage(p, a->stage);
    if (st != FB_OK) return st;
    if ((st = check_views(p, a->views, a->n_sel)) != FB_OK) return st;
    if (!a->b || !a->y_prev || !a->x_prev || !a->x_out || !a->y_out)
        return fail(FB_EINVAL, "pnp_step: null buffer");
    if (a->tv_iters < 0 || a->tv_iters > kTvMaxFused) return fail(FB_EINVAL, "pnp_step: tv_iters must be in [0, 8]");
    if (!(a->lambda >= 0.f) || !(a->tau > 0.f)) return fail(FB_EINVAL, "pnp_step: need lambda >= 0 and tau > 0");
    const Stage& S = p->stages[a->stage];
    const int nx = p->g.nx, ny = p->g.ny;
    if ((st = launch_prepare(p, a->stage, a->y_prev, nx, S.f, stream)) != FB_OK) return st;
    if ((st = launch_fp(p, a->stage, true, a->views, a->n_sel, a->b, p->resid, stream)) != FB_OK) return st;
    const float step = a->eta * a->sigma / (float)(S.f * S.f);
    if ((st = launch_bp_t<true>(p, a->stage, p->resid, a->views, a->n_sel, step, nullptr, a->y_prev, p->zbuf,
                                stream)) != FB_OK)
        return st;
    // lambda == 0 or no TV iterations: D is the identity, the same kernel then
    // only applies the relaxation and momentum (div p = 0)
    const float lam = a->lambda > 0.f ? a->lambda : 1.f;
    const int iters = a->lambda > 0.f ? a->tv_iters : 0;
    return launch_tv_single(p->zbuf, nx, ny, lam, a->tau, iters, nullptr, nullptr, 1, a->alpha, a->a_t, a->x_prev,
                            a->x_out, a->y_out, a->history, stream);
}

struct fb_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

fb_status fb_graph_create(const fb_plan* p, const fb_pnp_args* steps, int n_steps, fb_graph** out) {
    if (!p || !steps || n_steps < 1 || !out) return fail(FB_EINVAL, "fb_graph_create: bad arguments");
    *out = nullptr;
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "graph: stream");
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(e, "graph: begin capture");
    }
    fb_status st = FB_OK;
    for (int i = 0; i < n_steps && st == FB_OK; ++i) st = pnp_step(p, &steps[i], s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    (void)hipStreamDestroy(s);
    if (st != FB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "graph: end capture");
    fb_graph* G = new fb_graph();
    G->graph = g;
    e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        fb_graph_destroy(G);
        return hip_fail(e, "graph: instantiate");
    }
    *out = G;
    return FB_OK;
}

fb_status fb_graph_launch(fb_graph* G, hipStream_t stream) {
    if (!G || !G->exec) return fail(FB_EINVAL, "fb_graph_launch: graph is NULL");
    hipError_t e = hipGraphLaunch(G->exec, stream);
    return e == hipSuccess ? FB_OK : hip_fail(e, "graph launch");
}

fb_status fb_graph_destroy(fb_graph* G) {
    if (!G) return FB_OK;
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return FB_OK;
}

fb_status fb_power_lipschitz(const fb_plan* p, int stage, int n_iter, double* out, hipStream_t stream) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!out || n_iter < 0) return fail(FB_EINVAL, "fb_power_lipschitz: bad arguments");
    const Stage& S = p->stages[stage];
    const int nx = p->g.nx, ny = p->g.ny, nv = p->g.n_views;
    const size_t npix = (size_t)nx * ny;
    float* v = p->vec;
    float* w = v + npix;
    float* gs = w + npix;  // coarse gradient, nxs * nys <= npix
    double* part = (double*)(p->vec + ((3 * npix + 1) & ~(size_t)1));
    double* sum = part + kRedBlocks;
    const float inv_ff = 1.f / (float)(S.f * S.f);
    const int fill_blocks = std::min<size_t>(1024, (npix + 255) / 256);
    k_fill<<<fill_blocks, 256, 0, stream>>>(v, npix, (float)(1.0 / std::sqrt((double)npix)));
    if ((st = check_launch("power: fill")) != FB_OK) return st;
    for (int it = 0; it <= n_iter; ++it) {
        if ((st = launch_prepare(p, stage, v, nx, S.f, stream)) != FB_OK) return st;
        if ((st = launch_fp(p, stage, false, nullptr, nv, nullptr, p->resid, stream)) != FB_OK) return st;
        if (it == n_iter) break;
        if ((st = launch_bp_t<false>(p, stage, p->resid, nullptr, nv, 1.f, gs, nullptr, nullptr, stream)) != FB_OK)
            return st;
        k_up<<<dim3(cdiv(nx, 256), ny), 256, 0, stream>>>(gs, S.nxs, S.f, inv_ff, nx, ny, w);
        k_sumsq_partial<<<kRedBlocks, 256, 0, stream>>>(w, npix, part);
        k_sum_final<<<1, 256, 0, stream>>>(part, kRedBlocks, sum);
        k_normalise<<<fill_blocks, 256, 0, stream>>>(w, v, npix, sum);
        if ((st = check_launch("power iteration")) != FB_OK) return st;
    }
    k_sumsq_partial<<<kRedBlocks, 256, 0, stream>>>(p->resid, (size_t)nv * p->g.n_bins, part);
    k_sum_final<<<1, 256, 0, stream>>>(part, kRedBlocks, sum);
    if ((st = check_launch("power: norm")) != FB_OK) return st;
    double host = 0.0;
    hipError_t e = hipMemcpyAsync(&host, sum, sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "power: result copy");
    *out = host;
    return FB_OK;
}

}  // extern "C"
