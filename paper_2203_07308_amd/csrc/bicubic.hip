// Bicubic sketch S and its adjoint U = S^T on the GPU (Sec. 3: the paper
// resizes with bicubic interpolation; U is the adjoint so that the sketched
// gradient of Sec. 2.1, Eq. (6), stays the exact gradient of the sketched
// objective). S is separable: a pass along rows (x) into a [ny][nxs]
// intermediate, then one along columns (y) that writes the stage's two line
// images (or a plain image). S^T applies both adjoint tables at once and can
// fuse the gradient step z = y_prev - scale S^T g.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fbpnp_impl.h"

using namespace fbpnp;

namespace {

// tmp[r][C] = sum_t w[C taps + t] x[r][lo[C] + t]
__global__ __launch_bounds__(256) void k_bic_rows(const float* __restrict__ x, int nx, const int* __restrict__ lo,
                                                  const float* __restrict__ w, int taps, int nxs,
                                                  float* __restrict__ tmp) {
    const int C = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (C >= nxs) return;
    const float* xr = x + (size_t)r * nx + lo[C];
    const float* wc = w + (size_t)C * taps;
    float acc = 0.f;
    for (int t = 0; t < taps; ++t) acc = fmaf(wc[t], xr[t], acc);
    tmp[(size_t)r * nxs + C] = acc;
}

// v[R][C] = sum_t w[R taps + t] tmp[lo[R] + t][C], into v and / or the line images
__global__ __launch_bounds__(256) void k_bic_cols(const float* __restrict__ tmp, int nxs, const int* __restrict__ lo,
                                                  const float* __restrict__ w, int taps, float* __restrict__ v,
                                                  float* __restrict__ lx, int pitch_x, float* __restrict__ ly,
                                                  int pitch_y) {
    const int C = blockIdx.x * blockDim.x + threadIdx.x, R = blockIdx.y;
    if (C >= nxs) return;
    const float* tc = tmp + (size_t)lo[R] * nxs + C;
    const float* wr = w + (size_t)R * taps;
    float acc = 0.f;
    for (int t = 0; t < taps; ++t) acc = fmaf(wr[t], tc[(size_t)t * nxs], acc);
    if (v) v[(size_t)R * nxs + C] = acc;
    if (ly) {
        ly[(size_t)R * pitch_y + kPad + C] = acc;
        lx[(size_t)C * pitch_x + kPad + R] = acc;
    }
}

// S^T g at fine pixel (r, c): both adjoint tables; out = yprev - scale (S^T g)
// (or scale (S^T g) without yprev)
__global__ __launch_bounds__(256) void k_bic_up(const float* __restrict__ g, int nxs, const int* __restrict__ lox,
                                                const float* __restrict__ wx, int tx, const int* __restrict__ loy,
                                                const float* __restrict__ wy, int ty, int nx, float scale,
                                                const float* __restrict__ yprev, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= nx) return;
    const float* wrow = wy + (size_t)r * ty;
    const float* wcol = wx + (size_t)c * tx;
    const float* g0 = g + (size_t)loy[r] * nxs + lox[c];
    float acc = 0.f;
    for (int t = 0; t < ty; ++t) {
        float s = 0.f;
        for (int u = 0; u < tx; ++u) s = fmaf(wcol[u], g0[(size_t)t * nxs + u], s);
        acc = fmaf(wrow[t], s, acc);
    }
    const size_t i = (size_t)r * nx + c;
    out[i] = yprev ? fmaf(-scale, acc, yprev[i]) : scale * acc;
}

fb_status upload_axis(int n, int f, bool adjoint, SketchAxis& ax) {
    std::vector<int> lo;
    std::vector<float> w;
    fb_status st = bicubic_axis_tables(n, f, adjoint, lo, w, ax.taps);
    if (st != FB_OK) return st;
    if (hipMalloc(&ax.lo, lo.size() * sizeof(int)) != hipSuccess ||
        hipMalloc(&ax.w, w.size() * sizeof(float)) != hipSuccess)
        return fail(FB_ENOMEM, "bicubic sketch: table allocation");
    hipError_t e = hipMemcpy(ax.lo, lo.data(), lo.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ax.w, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice);
    return e == hipSuccess ? FB_OK : hip_fail(e, "bicubic sketch: table upload");
}

void free_axis(SketchAxis& ax) {
    if (ax.lo) (void)hipFree(ax.lo);
    if (ax.w) (void)hipFree(ax.w);
    ax = SketchAxis();
}

}  // namespace

namespace fbpnp {

void release_sketch(fb_plan* p) {
    for (StageSketch& s : p->sk) {
        free_axis(s.dx);
        free_axis(s.dy);
        free_axis(s.ux);
        free_axis(s.uy);
    }
    p->sk.clear();
    if (p->sk_tmp) (void)hipFree(p->sk_tmp);
    if (p->sk_g) (void)hipFree(p->sk_g);
    p->sk_tmp = p->sk_g = nullptr;
    p->sketch = 0;
}

fb_status launch_bicubic_down(const fb_plan* p, int stage, const float* x, float* v, hipStream_t s) {
    const Stage& S = p->stages[stage];
    const StageSketch& K = p->sk[stage];
    const int nx = p->g.nx, ny = p->g.ny;
    k_bic_rows<<<dim3(cdiv(S.nxs, 256), ny), 256, 0, s>>>(x, nx, K.dx.lo, K.dx.w, K.dx.taps, S.nxs, p->sk_tmp);
    StageLines L = stage_lines(p, stage);
    k_bic_cols<<<dim3(cdiv(S.nxs, 256), S.nys), 256, 0, s>>>(p->sk_tmp, S.nxs, K.dy.lo, K.dy.w, K.dy.taps, v,
                                                             v ? nullptr : L.lx, S.pitch_x, v ? nullptr : L.ly,
                                                             S.pitch_y);
    return check_launch("bicubic sketch");
}

fb_status launch_bicubic_up(const fb_plan* p, int stage, const float* g, float scale, const float* yprev, float* out,
                            hipStream_t s) {
    const Stage& S = p->stages[stage];
    const StageSketch& K = p->sk[stage];
    const int nx = p->g.nx, ny = p->g.ny;
    k_bic_up<<<dim3(cdiv(nx, 256), ny), 256, 0, s>>>(g, S.nxs, K.ux.lo, K.ux.w, K.ux.taps, K.uy.lo, K.uy.w,
                                                     K.uy.taps, nx, scale, yprev, out);
    return check_launch("bicubic adjoint");
}

}  // namespace fbpnp

extern "C" {

fb_status fb_plan_set_sketch(fb_plan* p, int kind) {
    fb_status st = check_stage(p, 0);
    if (st != FB_OK) return st;
    if (kind != 0 && kind != 1) return fail(FB_EINVAL, "fb_plan_set_sketch: kind must be 0 (pooling) or 1 (bicubic)");
    release_sketch(p);
    if (kind == 0) return FB_OK;
    const int nx = p->g.nx, ny = p->g.ny;
    p->sk.resize(p->stages.size());
    int nxs_max = 1, ncoarse_max = 1;
    for (size_t k = 0; k < p->stages.size(); ++k) {
        const int f = p->stages[k].f;
        if (f == 1) continue;
        StageSketch& K = p->sk[k];
        if ((st = upload_axis(nx, f, false, K.dx)) != FB_OK || (st = upload_axis(ny, f, false, K.dy)) != FB_OK ||
            (st = upload_axis(nx, f, true, K.ux)) != FB_OK || (st = upload_axis(ny, f, true, K.uy)) != FB_OK) {
            release_sketch(p);
            return st;
        }
        nxs_max = std::max(nxs_max, nx / f);
        ncoarse_max = std::max(ncoarse_max, (nx / f) * (ny / f));
    }
    if (hipMalloc(&p->sk_tmp, (size_t)ny * nxs_max * sizeof(float)) != hipSuccess ||
        hipMalloc(&p->sk_g, (size_t)ncoarse_max * sizeof(float)) != hipSuccess) {
        release_sketch(p);
        return fail(FB_ENOMEM, "fb_plan_set_sketch: workspace allocation");
    }
    p->sketch = 1;
    return FB_OK;
}

fb_status fb_plan_sketch_down(const fb_plan* p, int stage, const float* x, float* v, hipStream_t stream) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!x || !v) return fail(FB_EINVAL, "fb_plan_sketch_down: null buffer");
    if (!bicubic_stage(p, stage)) return sketch_down(x, p->g.nx, p->g.ny, p->stages[stage].f, v, stream);
    return launch_bicubic_down(p, stage, x, v, stream);
}

fb_status fb_plan_sketch_up(const fb_plan* p, int stage, const float* v, float* x, hipStream_t stream) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!x || !v) return fail(FB_EINVAL, "fb_plan_sketch_up: null buffer");
    const Stage& S = p->stages[stage];
    if (!bicubic_stage(p, stage)) return sketch_up(v, S.nxs, S.nys, S.f, x, stream);
    return launch_bicubic_up(p, stage, v, 1.f, nullptr, x, stream);
}

}  // extern "C"
