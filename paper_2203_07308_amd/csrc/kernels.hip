// HIP kernels for gfx950 (MI355X) and the C ABI entry points of libfbpnp
// (single image per call). The kernel bodies are in device.h:
//   k_prepare  pooling S = D_f of y_{t-1} into the stage's two line images
//   k_fp       Joseph forward projection of the selected views, minus b
//   k_bp       matched gather backprojection fused with U = D_f^T and the step
//   k_tv       Chambolle TV-prox fused with relaxation and momentum
// None of these paths is a dense contraction, so no MFMA is used; the
// projectors gather and interpolate through the L1/L2 caches, laid out so that
// the 64 lanes of a wavefront touch consecutive addresses.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <vector>

#include "device.h"
#include "fbpnp_impl.h"

using namespace fbpnp;

namespace {

using dev::kTile;


// ---------------------------------------------------------------------------
// Single-image kernels: one launch per call, block index = grid position.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prepare(const float* __restrict__ x, int nx, int f, float inv_ff,
                                                 int nxs, int nys, float* __restrict__ lx, int pitch_x,
                                                 float* __restrict__ ly, int pitch_y) {
    dev::prepare_body(blockIdx.x, blockIdx.y, x, nx, f, inv_ff, nxs, nys, lx, pitch_x, ly, pitch_y);
}

template <bool kResid, int SEG>
__global__ __launch_bounds__(256) void k_fp(const RayRec* __restrict__ rays, int n_bins, int bins_padded,
                                            const int32_t* __restrict__ views, int view0, int view_step, int n_sel,
                                            int n_views,
                                            const float* __restrict__ lines, int ly_off, int line_bytes,
                                            int pitch_x, int pitch_y, int nxs, int nys,
                                            const float* __restrict__ b, float* __restrict__ y,
                                            float* __restrict__ proj_out) {
    dev::fp_body<kResid, SEG>(blockIdx.x, rays, n_bins, bins_padded, views, view0, view_step, n_sel, n_views, lines,
                              ly_off, line_bytes, pitch_x, pitch_y, nxs, nys, b, y, proj_out);
}

template <int VG, int PX, bool kFused, bool kAllBins = false>
__global__ __launch_bounds__(64 * VG) void k_bp(const RayRec* __restrict__ rays, const ViewRec* __restrict__ vrec,
                                                int n_bins, const int32_t* __restrict__ views, int view0,
                                                int view_step, int n_sel,
                                                int n_views, const float* __restrict__ y, int nxs, int nys,
                                                int blocks_x, float scale, float* __restrict__ xo, int f, int nx,
                                                const float* __restrict__ yprev, float* __restrict__ z,
                                                const float* __restrict__ mu, float mu_scale,
                                                float* __restrict__ g_out) {
    dev::bp_body<VG, PX, kFused, kAllBins>(dev::xcd_tile(blockIdx.x, gridDim.x), rays, vrec, n_bins, views, view0,
                                           view_step, n_sel, n_views, y,
                                           nxs, nys,
                                           blocks_x, scale, xo, f, nx, yprev, z, mu, mu_scale, g_out);
}

// The line images of a stage small enough to stage in LDS (floats).
constexpr int kFpLdsFloats = 36864;

template <bool kResid, int SEG>
__global__ __launch_bounds__(1024) void k_fp_lds(int lds_floats, int n_blocks, const RayRec* __restrict__ rays,
                                                 int n_bins, int bins_padded, const int32_t* __restrict__ views,
                                                 int view0, int view_step, int n_sel, int n_views,
                                                 const float* __restrict__ lines, int ly_off, int pitch_x,
                                                 int pitch_y, int nxs, int nys, const float* __restrict__ b,
                                                 float* __restrict__ y, float* __restrict__ proj_out) {
    __shared__ float stage_lines_lds[kFpLdsFloats];
    dev::fp_body_lds<kResid, SEG>(stage_lines_lds, lds_floats, n_blocks, rays, n_bins, bins_padded, views, view0,
                                  view_step, n_sel, n_views, lines, ly_off, pitch_x, pitch_y, nxs, nys, b, y,
                                  proj_out);
}

template <int B, int VG, bool kFused>
__global__ __launch_bounds__(64 * VG) void k_bps(const RayRec* __restrict__ rays, const ViewRec* __restrict__ vrec,
                                                 int n_bins, const int32_t* __restrict__ views, int view0,
                                                 int view_step, int n_sel, int n_views, const float* __restrict__ y,
                                                 int nxs, int nys, int blocks_x, int gap, float scale,
                                                 float* __restrict__ xo, int f, int nx, const float* __restrict__ yprev,
                                                 float* __restrict__ z, const float* __restrict__ mu, float mu_scale,
                                                 float* __restrict__ g_out) {
    dev::bps_body<B, VG, kFused>(dev::xcd_tile(blockIdx.x, gridDim.x), rays, vrec, n_bins, views, view0, view_step,
                                 n_sel, n_views, y, nxs, nys,
                                 blocks_x, gap, scale, xo, f, nx, yprev, z, mu, mu_scale, g_out);
}

template <int T, int H, int NT>
__global__ __launch_bounds__(NT) void k_tv(const float* __restrict__ z, int nx, int ny, float lam, float tau,
                                           int n_iter, const float* __restrict__ p_in, float* __restrict__ p_out,
                                           int mode, float alpha, float a_t, const float* __restrict__ x_prev,
                                           float* __restrict__ x_out, float* __restrict__ y_out,
                                           float* __restrict__ hist, int pf, float pinv, float* __restrict__ plx,
                                           int ppx, float* __restrict__ ply, int ppy, int pnxs, int pnys,
                                           unsigned long long* __restrict__ stamp) {
    const int tile = dev::xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    dev::tv_body<T, H, NT>(tile % gridDim.x, tile / gridDim.x, z, nx, ny, lam, tau, n_iter, p_in, p_out, mode, alpha,
                           a_t, x_prev,
                           x_out, y_out, hist, pf, pinv, plx, ppx, ply, ppy, pnxs, pnys, stamp);
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

// The device's constant-rate clock, written once (a start mark for step stamps).
__global__ void k_stamp(unsigned long long* __restrict__ d) { *d = wall_clock64(); }

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ a, size_t n, float val) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = val;
}

// Per-block sums of squares in double, in a fixed order.
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

}  // namespace

// ---------------------------------------------------------------------------
// Host helpers (shared with the reverse-mode entry points)
// ---------------------------------------------------------------------------
namespace fbpnp {

thread_local LaunchEvents t_launch_events;

// kernel launch on stream S, through hipExtLaunchKernelGGL when timing events are set
#define FB_LAUNCH(K, G, B, S, ...)                                                                   \
    do {                                                                                             \
        const LaunchEvents ev_ = t_launch_events;                                                    \
        if (ev_.begin || ev_.end)                                                                    \
            hipExtLaunchKernelGGL(K, G, B, 0, S, ev_.begin, ev_.end, 0, __VA_ARGS__);                \
        else                                                                                         \
            K<<<G, B, 0, S>>>(__VA_ARGS__);                                                          \
    } while (0)

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

ViewSel pnp_views(const fb_pnp_args* a) {
    if (!a->views && a->n_sub > 1) return ViewSel{nullptr, a->n_sel, a->subset, a->n_sub};
    return ViewSel{a->views, a->n_sel};
}

fb_status check_pnp_views(const fb_plan* p, const fb_pnp_args* a) {
    if (a->n_sub > 1 || a->subset != 0) {
        if (a->views) return fail(FB_EINVAL, "pnp_step: give a view list or (n_sub, subset), not both");
        if (a->n_sub < 1 || a->subset < 0 || a->subset >= a->n_sub)
            return fail(FB_EINVAL, "pnp_step: need 0 <= subset < n_sub");
        const int count = (p->g.n_views - a->subset + a->n_sub - 1) / a->n_sub;
        if (count < 1) return fail(FB_EINVAL, "pnp_step: the subset holds no view");
        if (a->n_sel != count) return fail(FB_EINVAL, "pnp_step: n_sel must equal the number of views in the subset");
        return FB_OK;
    }
    if (a->n_sub < 0) return fail(FB_EINVAL, "pnp_step: n_sub must not be negative");
    return check_views(p, a->views, a->n_sel);
}

// Line images of a stage live in one plan allocation, one region per stage.
StageLines stage_lines(const fb_plan* p, int stage) {
    size_t off = 0;
    for (int s = 0; s < stage; ++s) {
        const Stage& st = p->stages[s];
        off += (size_t)st.nxs * st.pitch_x + (size_t)st.nys * st.pitch_y;
    }
    const Stage& st = p->stages[stage];
    const int lxn = st.nxs * st.pitch_x;
    return {p->line_x + off, p->line_x + off + lxn, lxn, (int)((size_t)(lxn + st.nys * st.pitch_y) * sizeof(float))};
}

fb_status launch_prepare(const fb_plan* p, int stage, const float* x, int nx, int f, hipStream_t s) {
    const Stage& st = p->stages[stage];
    StageLines L = stage_lines(p, stage);
    dim3 grid(cdiv(st.nxs, kTile), cdiv(st.nys, kTile));
    k_prepare<<<grid, 256, 0, s>>>(x, nx, f, 1.f / (float)(f * f), st.nxs, st.nys, L.lx, st.pitch_x, L.ly,
                                   st.pitch_y);
    return check_launch("prepare");
}

// ---- launch configurations ------------------------------------------------
// Defaults: split rays over 2 or 4 lanes when one lane per ray gives few
// wavefronts; pixels per lane 4 x 4 on very large grids, 2 x 2 on large ones, 1
// otherwise; views split over up to 16 wavefronts per block (4 with 4 x 4
// pixels, for registers) until ~8192 wavefronts; 32 x 32 TV tiles with 1024
// threads, 16 x 16 when that leaves CUs idle.
int default_fp_seg(long waves1) { return waves1 < 4096 ? 4 : (waves1 < 8192 ? 2 : 1); }
int default_bp_px(long npx) { return npx >= 1024L * 1024 ? 4 : (npx >= 256L * 256 ? 2 : 1); }
int default_bp_vg(int px, long nblk, int n_sel) {
    const int vg_max = px == 4 ? 4 : 16;
    int vg = 1;
    while (vg < vg_max && nblk * vg < 8192 && vg * 2 <= n_sel) vg *= 2;
    return vg;
}
int default_tv_tile(long tiles32) { return tiles32 < 256 ? 16 : 32; }
int bp_block_side(int bp_px) { return bp_px >= 16 ? bp_px : 8 * bp_px; }

bool bp_blocks_reach_source(const fb_geom& g, const Stage& st, int bw) {
    // the union of the blocks grown by one pixel on each side, in centred
    // stage-pixel coordinates: its farthest corner from the isocentre
    const double hx = 0.5 * (st.nxs - 1), hy = 0.5 * (st.nys - 1);
    const double cx = std::max(hx + 1.0, cdiv(st.nxs, bw) * bw - hx);
    const double cy = std::max(hy + 1.0, cdiv(st.nys, bw) * bw - hy);
    return g.pixel_mm * st.f * std::hypot(cx, cy) >= (1.0 - 1e-3) * g.sod_mm;
}

fb_status check_config(const fb_launch_config& c) {
    auto in = [](int v, std::initializer_list<int> ok) {
        if (v == 0) return true;
        for (int o : ok)
            if (v == o) return true;
        return false;
    };
    if (!in(c.fp_seg, {1, 2, 4, 8})) return fail(FB_EINVAL, "launch config: fp_seg must be 0, 1, 2, 4 or 8");
    if (!in(c.bp_px, {1, 2, 4, 16, 32}))
        return fail(FB_EINVAL, "launch config: bp_px must be 0, 1, 2, 4 (gather) or 16, 32 (scatter)");
    if (!in(c.bp_vg, {1, 2, 4, 8, 16})) return fail(FB_EINVAL, "launch config: bp_vg must be 0, 1, 2, 4, 8 or 16");
    if (c.bp_px == 4 && c.bp_vg > 4) return fail(FB_EINVAL, "launch config: bp_px = 4 allows bp_vg <= 4");
    if (!in(c.tv_tile, {16, 32})) return fail(FB_EINVAL, "launch config: tv_tile must be 0, 16 or 32");
    if (!in(c.fp_lds, {1, 2})) return fail(FB_EINVAL, "launch config: fp_lds must be 0, 1 or 2");
    return FB_OK;
}

fb_launch_config plan_config(const fb_plan* p, int stage, int n_sel) {
    const Stage& st = p->stages[stage];
    fb_launch_config c = p->cfg[stage];
    if (!c.fp_seg) c.fp_seg = default_fp_seg((long)n_sel * cdiv(p->g.n_bins, 64));
    if (!c.bp_px) c.bp_px = default_bp_px((long)st.nxs * st.nys);
    if (!c.bp_vg) {
        const int bw = bp_block_side(c.bp_px);
        c.bp_vg = default_bp_vg(c.bp_px, (long)cdiv(st.nxs, bw) * cdiv(st.nys, bw), n_sel);
        if (c.bp_px == 4 && c.bp_vg > 4) c.bp_vg = 4;
    }
    if (!c.tv_tile) c.tv_tile = default_tv_tile((long)cdiv(p->g.nx, 32) * cdiv(p->g.ny, 32));
    if (!c.fp_lds) c.fp_lds = 1;
    return c;
}

bool fp_lds_fits(const fb_plan* p, int stage) {
    const Stage& st = p->stages[stage];
    return (long)st.nxs * st.pitch_x + (long)st.nys * st.pitch_y <= kFpLdsFloats;
}

// work-groups of an LDS-staged projection: one per compute unit at most, each
// taking four blocks of 256 threads at a time
static int cu_count() {
    static int n = 0;
    if (!n) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            n = v;
        else
            n = 256;
    }
    return n;
}

fb_status launch_fp(const fb_plan* p, int stage, bool resid, const ViewSel& sel, const float* b, float* y,
                    hipStream_t s, float* proj_out) {
    const int n_sel = sel.n;
    const Stage& st = p->stages[stage];
    StageLines L = stage_lines(p, stage);
    const int nb = p->g.n_bins;
    const fb_launch_config c = plan_config(p, stage, n_sel);
    const int seg = c.fp_seg;
    const int rays_per_wave = 64 / seg;
    const int bp = cdiv(nb, rays_per_wave) * rays_per_wave;
    const int blocks = cdiv(n_sel * (bp / rays_per_wave), 4);
    if (c.fp_lds == 2 && fp_lds_fits(p, stage)) {
        const int lds_floats = st.nxs * st.pitch_x + st.nys * st.pitch_y;
        const int grid = std::min(cdiv(blocks, 4), cu_count());
#define FB_FPL(RES, SG)                                                                                         \
    FB_LAUNCH((k_fp_lds<RES, SG>), dim3(grid), dim3(1024), s, lds_floats, blocks, st.rays, nb, bp, sel.list,      \
              sel.view0, sel.step, n_sel, p->g.n_views, L.lx, L.ly_off, st.pitch_x, st.pitch_y, st.nxs, st.nys, b, \
              y, proj_out)
        if (resid) {
            if (seg == 8) FB_FPL(true, 8);
            else if (seg == 4) FB_FPL(true, 4);
            else if (seg == 2) FB_FPL(true, 2);
            else FB_FPL(true, 1);
        } else {
            if (seg == 8) FB_FPL(false, 8);
            else if (seg == 4) FB_FPL(false, 4);
            else if (seg == 2) FB_FPL(false, 2);
            else FB_FPL(false, 1);
        }
#undef FB_FPL
        return check_launch("fanbeam_fp");
    }
#define FB_FP(RES, SG)                                                                                        \
    FB_LAUNCH((k_fp<RES, SG>), dim3(blocks), dim3(256), s, st.rays, nb, bp, sel.list, sel.view0, sel.step,      \
              n_sel, p->g.n_views, L.lx,                                                                      \
              L.ly_off, L.bytes, st.pitch_x, st.pitch_y, st.nxs, st.nys, b, y, proj_out)
    if (resid) {
        if (seg == 8) FB_FP(true, 8);
        else if (seg == 4) FB_FP(true, 4);
        else if (seg == 2) FB_FP(true, 2);
        else FB_FP(true, 1);
    } else {
        if (seg == 8) FB_FP(false, 8);
        else if (seg == 4) FB_FP(false, 4);
        else if (seg == 2) FB_FP(false, 2);
        else FB_FP(false, 1);
    }
#undef FB_FP
    return check_launch("fanbeam_fp");
}

template <bool kFused>
static fb_status launch_bp_t(const fb_plan* p, int stage, const float* y, const ViewSel& sel, float scale, float* xo, const float* yprev, float* z, hipStream_t s,
                             const float* mu = nullptr, float mu_scale = 0.f, float* g_out = nullptr) {
    const Stage& st = p->stages[stage];
    const int n_sel = sel.n;
    const fb_launch_config c = plan_config(p, stage, n_sel);
    // blocks that reach the source circle: every bin a candidate, one pixel per lane
    const bool all_bins = bp_blocks_reach_source(p->g, st, bp_block_side(c.bp_px));
    const int px = all_bins ? 1 : c.bp_px, vg = c.bp_vg;
    const int bw = bp_block_side(px);
    const int bxs = cdiv(st.nxs, bw), bys = cdiv(st.nys, bw), nblk = bxs * bys;
    const int nb = p->g.n_bins, f = st.f, nx = p->g.nx;
    if (all_bins) {
        FB_LAUNCH((k_bp<4, 1, kFused, true>), dim3(nblk), dim3(256), s, st.rays, st.vrec, nb, sel.list, sel.view0, sel.step, n_sel,
                  p->g.n_views, y, st.nxs, st.nys, bxs, scale, xo, f, nx, yprev, z, mu, mu_scale, g_out);
        return check_launch("fanbeam_bp");
    }
    if (px >= 16) {
#define FB_BPS(BB, VG)                                                                                         \
    FB_LAUNCH((k_bps<BB, VG, kFused>), dim3(nblk), dim3(64 * VG), s, st.rays, st.vrec, nb, sel.list, sel.view0, \
              sel.step, n_sel, p->g.n_views, y, st.nxs, st.nys, bxs, st.scatter_gap, scale, xo, f, nx, yprev, z, mu, \
              mu_scale, g_out)
#define FB_BPS_VG(BB)                  \
    switch (vg) {                      \
        case 1: FB_BPS(BB, 1); break;  \
        case 2: FB_BPS(BB, 2); break;  \
        case 4: FB_BPS(BB, 4); break;  \
        case 8: FB_BPS(BB, 8); break;  \
        default: FB_BPS(BB, 16); break; \
    }
        if (px == 32) {
            FB_BPS_VG(32)
        } else {
            FB_BPS_VG(16)
        }
#undef FB_BPS_VG
#undef FB_BPS
        return check_launch("fanbeam_bp");
    }
#define FB_BP(VG, PX)                                                                                         \
    FB_LAUNCH((k_bp<VG, PX, kFused>), dim3(nblk), dim3(64 * VG), s, st.rays, st.vrec, nb, sel.list, sel.view0, sel.step, n_sel,         \
              p->g.n_views, y, st.nxs, st.nys, bxs, scale, xo, f, nx, yprev, z, mu, mu_scale, g_out)
#define FB_BP_VG(PX)           \
    switch (vg) {              \
        case 1: FB_BP(1, PX); break;  \
        case 2: FB_BP(2, PX); break;  \
        case 4: FB_BP(4, PX); break;  \
        case 8: FB_BP(8, PX); break;  \
        default: FB_BP(16, PX); break; \
    }
    if (px == 4) {
        switch (vg) {
            case 1: FB_BP(1, 4); break;
            case 2: FB_BP(2, 4); break;
            default: FB_BP(4, 4); break;
        }
    } else if (px == 2) {
        FB_BP_VG(2)
    } else {
        FB_BP_VG(1)
    }
#undef FB_BP_VG
#undef FB_BP
    return check_launch("fanbeam_bp");
}

fb_status launch_bp(const fb_plan* p, int stage, const float* y, const ViewSel& sel, float scale, float* xo,
                    const float* yprev, float* z, bool fused, hipStream_t s) {
    return fused ? launch_bp_t<true>(p, stage, y, sel, scale, xo, yprev, z, s)
                 : launch_bp_t<false>(p, stage, y, sel, scale, xo, yprev, z, s);
}

fb_status capture_graph(const std::function<fb_status(hipStream_t)>& body, fb_graph** out) {
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "graph: stream");
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(e, "graph: begin capture");
    }
    const fb_status st = body(s);
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

fb_status launch_tv_single(const float* z, int nx, int ny, float lam, float tau, int n_iter, const float* p_in,
                           float* p_out, int mode, float alpha, float a_t, const float* x_prev, float* x_out,
                           float* y_out, float* hist, hipStream_t s, const PoolTarget& pt, int tile,
                           unsigned long long* stamp) {
    const int T = tile ? tile : default_tv_tile((long)cdiv(nx, 32) * cdiv(ny, 32));
    if (pt.f > 0 && T % pt.f != 0) return fail(FB_EINVAL, "pooling factor does not divide the TV tile");
    dim3 grid(cdiv(nx, T), cdiv(ny, T));
#define FB_TV(TT, HH, NT)                                                                                     \
    FB_LAUNCH((k_tv<TT, HH, NT>), grid, dim3(NT), s, z, nx, ny, lam, tau, n_iter, p_in, p_out, mode, alpha, a_t, \
              x_prev, x_out, y_out, hist, pt.f, pt.inv, pt.lx, pt.px, pt.ly, pt.py, pt.nxs, pt.nys, stamp)
    if (T == 16) {
        if (n_iter <= 5) FB_TV(16, 6, 256);
        else FB_TV(16, kTvMaxFused + 1, 256);
    } else {
        if (n_iter <= 5) FB_TV(32, 6, 1024);
        else FB_TV(32, kTvMaxFused + 1, 1024);
    }
#undef FB_TV
    return check_launch("tv_prox");
}

}  // namespace fbpnp

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
        if (f < 1 || f > kMaxFactor) return fail(FB_EINVAL, "pooling factor must be in 1..32");
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
    p->cfg.assign(n_stages, fb_launch_config{0, 0, 0, 0, 0});
    for (int s = 0; s < n_stages; ++s) {
        Stage S;
        S.f = factors[s];
        S.nxs = geom->nx / S.f;
        S.nys = geom->ny / S.f;
        S.pitch_x = ((S.nys + 2 * kPad + 3) / 4) * 4;
        S.pitch_y = ((S.nxs + 2 * kPad + 3) / 4) * 4;
        std::vector<RayRec> rays;
        std::vector<ViewRec> vr;
        st = build_stage_tables(*geom, S.f, rays, vr, S.view_samples);
        if (st != FB_OK) return cleanup(st);
        S.scatter_gap = scatter_gap(*geom, S.f, rays, vr);
        for (int64_t n : S.view_samples) S.samples += n;
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
    if (line_floats * sizeof(float) >= ((size_t)1 << 31))
        return cleanup(fail(FB_EINVAL, "plan: image too large for 32-bit line-image offsets"));
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
    release_sketch(p);
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

fb_status fb_plan_set_config(fb_plan* p, int stage, const fb_launch_config* cfg) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    const fb_launch_config c = cfg ? *cfg : fb_launch_config{0, 0, 0, 0, 0};
    if ((st = check_config(c)) != FB_OK) return st;
    if (c.fp_lds == 2 && !fp_lds_fits(p, stage))
        return fail(FB_EINVAL, "launch config: the stage's line images do not fit in LDS (fp_lds = 2)");
    p->cfg[stage] = c;
    return FB_OK;
}

fb_status fb_plan_get_config(const fb_plan* p, int stage, int n_sel, fb_launch_config* out) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!out || n_sel < 1) return fail(FB_EINVAL, "fb_plan_get_config: bad arguments");
    *out = plan_config(p, stage, n_sel);
    return FB_OK;
}

fb_status fb_workspace_bytes(const fb_plan* p, int stage, size_t* out) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!out) return fail(FB_EINVAL, "out is NULL");
    const StageLines L = stage_lines(p, stage);
    *out = (size_t)L.bytes + (size_t)p->g.n_views * p->g.n_bins * sizeof(float) +
           (size_t)p->g.nx * p->g.ny * sizeof(float);
    return FB_OK;
}

fb_status fb_plan_view_samples(const fb_plan* p, int stage, int64_t* out) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!out) return fail(FB_EINVAL, "out is NULL");
    const Stage& S = p->stages[stage];
    std::copy(S.view_samples.begin(), S.view_samples.end(), out);
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
    return launch_fp(p, stage, false, ViewSel{views, n_sel}, nullptr, y, stream);
}

fb_status fanbeam_bp(const fb_plan* p, int stage, const float* y, float* x, const int32_t* views, int n_sel,
                     float scale, hipStream_t stream) {
    fb_status st = check_stage(p, stage);
    if (st != FB_OK) return st;
    if (!x || !y) return fail(FB_EINVAL, "fanbeam_bp: x and y must not be NULL");
    if ((st = check_views(p, views, n_sel)) != FB_OK) return st;
    return launch_bp_t<false>(p, stage, y, ViewSel{views, n_sel}, scale, x, nullptr, nullptr, stream);
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

}  // extern "C"

// The denoiser after its arguments are checked. ws: the two dual fields
// [2][ny][nx] of the multi-launch ping-pong, used only when n_iter > 8 (every
// cell is written by one launch before the next one reads it, so ws needs no
// clearing).
static fb_status tv_prox_run(const float* z, float* x, int nx, int ny, float lambda, int n_iter, float tau,
                             float* ws, hipStream_t stream) {
    if (lambda == 0.f || n_iter == 0) {
        hipError_t e = hipMemcpyAsync(x, z, (size_t)nx * ny * sizeof(float), hipMemcpyDeviceToDevice, stream);
        return e == hipSuccess ? FB_OK : hip_fail(e, "tv_prox copy");
    }
    if (n_iter <= kTvMaxFused)
        return launch_tv_single(z, nx, ny, lambda, tau, n_iter, nullptr, nullptr, 0, 0.f, 0.f, nullptr, x, nullptr,
                                nullptr, stream);
    float* pa = ws;
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

static fb_status tv_prox_check(const char* who, const float* z, const float* x, int nx, int ny, float lambda,
                               int n_iter, float tau) {
    const std::string w(who);
    if (!z || !x || nx < 1 || ny < 1 || n_iter < 0) return fail(FB_EINVAL, w + ": bad arguments");
    if (!(lambda >= 0.f) || !(tau > 0.f)) return fail(FB_EINVAL, w + ": need lambda >= 0 and tau > 0");
    if (z == x) return fail(FB_EINVAL, w + ": z and x must not alias");
    return FB_OK;
}

// Scratch of tv_prox_noalloc: the two dual fields of the multi-launch
// ping-pong, for images of up to kTvScratchPixels pixels (16 MiB, held by
// every device the library runs on until the process ends). In host code the
// array's name is no device address: kernels get the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kTvScratchPixels = (size_t)1 << 20;
static __device__ __align__(256) float scratch[4 * kTvScratchPixels];

// Device address of `scratch` on the current device, looked up once per device.
static fb_status tv_scratch_address(float** out) {
    static std::mutex mu;
    static std::vector<float*> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "tv_prox_noalloc: device");
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)dev >= addr.size()) addr.resize((size_t)dev + 1, nullptr);
    if (!addr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "tv_prox_noalloc: scratch address");
        addr[dev] = static_cast<float*>(ptr);
    }
    *out = addr[dev];
    return FB_OK;
}

extern "C" {

fb_status tv_prox(const float* z, float* x, int nx, int ny, float lambda, int n_iter, float tau, void* ws,
                  size_t ws_bytes, hipStream_t stream) {
    fb_status st = tv_prox_check("tv_prox", z, x, nx, ny, lambda, n_iter, tau);
    if (st != FB_OK) return st;
    if (n_iter > kTvMaxFused && lambda != 0.f && (!ws || ws_bytes < fb_tv_workspace_bytes(nx, ny, n_iter)))
        return fail(FB_EINVAL, "tv_prox: workspace too small");
    return tv_prox_run(z, x, nx, ny, lambda, n_iter, tau, (float*)ws, stream);
}

fb_status tv_prox_noalloc(const float* z, float* x, int nx, int ny, float lambda, int n_iter, float tau,
                          hipStream_t stream) {
    fb_status st = tv_prox_check("tv_prox_noalloc", z, x, nx, ny, lambda, n_iter, tau);
    if (st != FB_OK) return st;
    if ((size_t)nx * (size_t)ny > kTvScratchPixels)
        return fail(FB_EINVAL, "tv_prox_noalloc: image larger than the static scratch (at most 1048576 pixels)");
    float* ws = nullptr;
    if (n_iter > kTvMaxFused && lambda != 0.f && (st = tv_scratch_address(&ws)) != FB_OK) return st;
    return tv_prox_run(z, x, nx, ny, lambda, n_iter, tau, ws, stream);
}


// The TV epilogue's hand-over of y_t to the next step's stage: its pooling
// into that stage's line images (not for bicubic stages, which sketch anew).
static PoolTarget pool_target(const fb_plan* p, int next_stage) {
    PoolTarget pt;
    if (next_stage < 0 || bicubic_stage(p, next_stage)) return pt;
    const Stage& N = p->stages[next_stage];
    StageLines L = stage_lines(p, next_stage);
    pt.f = N.f;
    pt.inv = 1.f / (float)(N.f * N.f);
    pt.lx = L.lx;
    pt.ly = L.ly;
    pt.px = N.pitch_x;
    pt.py = N.pitch_y;
    pt.nxs = N.nxs;
    pt.nys = N.nys;
    return pt;
}

// The denoiser of a step on z (p->zbuf). With next_stage set, y_t is pooled
// for that stage in the TV kernel's epilogue when its factor divides the TV
// tile, else by a pooling launch after it. lambda == 0 or no TV iterations:
// D is the identity, and the same kernel only applies the relaxation and the
// momentum (div p = 0).
static fb_status step_tv(const fb_plan* p, const fb_pnp_args* a, hipStream_t stream) {
    const int tile = plan_config(p, a->stage, a->n_sel).tv_tile;
    PoolTarget pt = pool_target(p, a->next_stage);
    const bool pool_after = pt.f > 0 && tile % pt.f != 0;
    if (pool_after) pt = PoolTarget();
    const float lam = a->lambda > 0.f ? a->lambda : 1.f;
    const int iters = a->lambda > 0.f ? a->tv_iters : 0;
    fb_status st;
    {
        TimedLaunch tl(a->events, 4);
        st = launch_tv_single(p->zbuf, p->g.nx, p->g.ny, lam, a->tau, iters, nullptr, nullptr, 1, a->alpha, a->a_t,
                              a->x_prev, a->x_out, a->y_out, a->history, stream, pt, tile,
                              reinterpret_cast<unsigned long long*>(a->stamp));
    }
    if (st != FB_OK || !pool_after) return st;
    return launch_prepare(p, a->next_stage, a->y_out, p->g.nx, p->stages[a->next_stage].f, stream);
}

// pnp_step at a stage with the bicubic sketch: S into the line images, the
// residual projection, the back-projection into the coarse gradient g, then
// z = y_{t-1} - eta sigma S^T g and the denoiser.
static fb_status pnp_step_bicubic(const fb_plan* p, const fb_pnp_args* a, hipStream_t stream) {
    fb_status st;
    if (a->vr_mode != 0) return fail(FB_EINVAL, "pnp_step: variance reduction is defined with the pooling sketch");
    if ((st = launch_bicubic_down(p, a->stage, a->y_prev, nullptr, stream)) != FB_OK) return st;
    {
        TimedLaunch tl(a->events, 0);
        if ((st = launch_fp(p, a->stage, true, pnp_views(a), a->b, p->resid, stream)) != FB_OK) return st;
    }
    {
        TimedLaunch tl(a->events, 2);
        if ((st = launch_bp_t<false>(p, a->stage, p->resid, pnp_views(a), 1.f, p->sk_g, nullptr, nullptr,
                                     stream)) != FB_OK)
            return st;
    }
    if ((st = launch_bicubic_up(p, a->stage, p->sk_g, a->eta * a->sigma, a->y_prev, p->zbuf, stream)) != FB_OK)
        return st;
    return step_tv(p, a, stream);
}

fb_status pnp_step(const fb_plan* p, const fb_pnp_args* a, hipStream_t stream) {
    if (!a) return fail(FB_EINVAL, "pnp_step: args is NULL");
    fb_status st = check_stage(p, a->stage);
    if (st != FB_OK) return st;
    if ((st = check_pnp_views(p, a)) != FB_OK) return st;
    if (!a->b || !a->y_prev || !a->x_prev || !a->x_out || !a->y_out)
        return fail(FB_EINVAL, "pnp_step: null buffer");
    if (a->tv_iters < 0 || a->tv_iters > kTvMaxFused) return fail(FB_EINVAL, "pnp_step: tv_iters must be in [0, 8]");
    if (!(a->lambda >= 0.f) || !(a->tau > 0.f)) return fail(FB_EINVAL, "pnp_step: need lambda >= 0 and tau > 0");
    if (a->next_stage < -1 || a->next_stage >= (int)p->stages.size())
        return fail(FB_EINVAL, "pnp_step: next_stage out of range");
    if (a->prepared != 0 && a->prepared != 1) return fail(FB_EINVAL, "pnp_step: prepared must be 0 or 1");
    if (a->vr_mode < 0 || a->vr_mode > 2) return fail(FB_EINVAL, "pnp_step: vr_mode must be 0, 1 or 2");
    if (a->vr_mode && (!a->snap_proj || !a->snap_grad))
        return fail(FB_EINVAL, "pnp_step: variance-reduced modes need snap_proj and snap_grad");
    // a snapshot fills every row of snap_proj: all views, in order, each once
    if (a->vr_mode == 1 && (a->views || a->n_sub > 1 || a->n_sel != p->g.n_views))
        return fail(FB_EINVAL, "pnp_step: a snapshot step takes every view (views NULL, no subset)");
    if (a->grad && a->vr_mode != 0) return fail(FB_EINVAL, "pnp_step: grad is for minibatch steps (vr_mode 0)");
    const Stage& S = p->stages[a->stage];
    if (bicubic_stage(p, a->stage)) {
        if (a->grad) return fail(FB_EINVAL, "pnp_step: grad is stored with the pooling sketch only");
        return pnp_step_bicubic(p, a, stream);
    }
    if (!a->prepared && (st = launch_prepare(p, a->stage, a->y_prev, p->g.nx, S.f, stream)) != FB_OK) return st;
    // variance-reduced modes: 1 records the snapshot's projection and coarse
    // gradient; 2 projects against the snapshot's projection and adds its gradient
    const bool snap = a->vr_mode == 1, vr = a->vr_mode == 2;
    {
        TimedLaunch tl(a->events, 0);
        if ((st = launch_fp(p, a->stage, true, pnp_views(a), vr ? a->snap_proj : a->b, p->resid, stream,
                            snap ? a->snap_proj : nullptr)) != FB_OK)
            return st;
    }
    const float step = a->eta * a->sigma / (float)(S.f * S.f);
    {
        TimedLaunch tl(a->events, 2);
        if ((st = launch_bp_t<true>(p, a->stage, p->resid, pnp_views(a), step, nullptr, a->y_prev, p->zbuf,
                                    stream, vr ? a->snap_grad : nullptr, a->eta / (float)(S.f * S.f),
                                    snap ? a->snap_grad : a->grad)) != FB_OK)
            return st;
    }
    return step_tv(p, a, stream);
}

fb_status fb_clock_stamp(uint64_t* dst, hipStream_t stream) {
    if (!dst) return fail(FB_EINVAL, "fb_clock_stamp: dst is NULL");
    k_stamp<<<1, 1, 0, stream>>>(reinterpret_cast<unsigned long long*>(dst));
    return check_launch("fb_clock_stamp");
}

int32_t fb_clock_khz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return khz;
}

fb_status fb_graph_create(const fb_plan* p, const fb_pnp_args* steps, int n_steps, fb_graph** out) {
    if (!p || !steps || n_steps < 1 || !out) return fail(FB_EINVAL, "fb_graph_create: bad arguments");
    *out = nullptr;
    // chain consecutive steps: step i pools its y_t for step i+1 when that
    // step reads it, and step i+1 then skips its own pooling
    std::vector<fb_pnp_args> chain(steps, steps + n_steps);
    for (int i = 0; i < n_steps; ++i) {
        chain[i].prepared = 0;
        chain[i].next_stage = -1;
        chain[i].events = nullptr;  // kernel timing is for direct calls only
    }
    for (int i = 0; i + 1 < n_steps; ++i) {
        if (chain[i + 1].y_prev == chain[i].y_out && chain[i + 1].stage >= 0 &&
            chain[i + 1].stage < (int)p->stages.size()) {
            chain[i].next_stage = chain[i + 1].stage;
            chain[i + 1].prepared = 1;
        }
    }
    return capture_graph(
        [&](hipStream_t s) {
            fb_status st = FB_OK;
            for (int i = 0; i < n_steps && st == FB_OK; ++i) st = pnp_step(p, &chain[i], s);
            return st;
        },
        out);
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
    const bool bic = bicubic_stage(p, stage);
    for (int it = 0; it <= n_iter; ++it) {
        st = bic ? launch_bicubic_down(p, stage, v, nullptr, stream) : launch_prepare(p, stage, v, nx, S.f, stream);
        if (st != FB_OK) return st;
        if ((st = launch_fp(p, stage, false, ViewSel{nullptr, nv}, nullptr, p->resid, stream)) != FB_OK) return st;
        if (it == n_iter) break;
        if ((st = launch_bp_t<false>(p, stage, p->resid, ViewSel{nullptr, nv}, 1.f, gs, nullptr, nullptr, stream)) != FB_OK)
            return st;
        if (bic) {
            if ((st = launch_bicubic_up(p, stage, gs, 1.f, nullptr, w, stream)) != FB_OK) return st;
        } else {
            k_up<<<dim3(cdiv(nx, 256), ny), 256, 0, stream>>>(gs, S.nxs, S.f, inv_ff, nx, ny, w);
        }
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
