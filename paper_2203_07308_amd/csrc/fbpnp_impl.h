// Internal definitions shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "fbpnp.h"

namespace fbpnp {

// Largest pooling factor of a stage (the backprojector's epilogue takes exact
// quotients by f with float reciprocals up to 8 x 4 x 32 fine pixels a side).
constexpr int kMaxFactor = 32;

// Zero padding on both ends of every line of the two line images of a stage.
constexpr int kPad = 2;

// One ray of one stage: Joseph samples on the major-axis lines lo .. lo+n-1.
// On line k the minor-axis pixel-index coordinate is
//   pos(k) = npos/2 + fmaf(k - nlines/2, dpos, pos_c)     (integer npos/2, nlines/2)
// with nlines, npos the grid sizes along the major and minor axis. The plan
// chooses lo, n so that, with exactly this float evaluation, a line has a
// sample if and only if pos(k) lies in [-1, npos); a ray without samples
// (n = 0) keeps its pos_c and dpos, so pos(k) lies outside that interval on
// every line of the grid. Ray weight len = f h |d| / |d_major|.
// bits: lo (16) | n (15) << 16 | axis << 31, axis 0 = x-major (lines are
// columns, positions are rows), 1 = y-major (lines are rows, positions are
// columns).
struct alignas(16) RayRec {
    float pos_c, dpos, len;
    uint32_t bits;
};

// Per view and stage: the detector coordinate of the ray through pixel-index
// point (c, r) of the stage grid is
//   j(c, r) = (a0 + a1 c' + a2 r') / (b0 + b1 c' + b2 r') + j0,
// with centred indices c' = c - (nxs-1)/2, r' = r - (nys-1)/2, and bins
// [xlo, xhi] are x-major, [ylo, yhi] y-major (an empty range has lo > hi).
struct alignas(16) ViewRec {
    float a0, a1, a2, b0, b1, b2, j0, pad;
    int32_t xlo, xhi, ylo, yhi;
};

struct Stage {
    int f = 1, nxs = 0, nys = 0;
    int64_t samples = 0;            // in-grid samples over all views
    std::vector<int64_t> view_samples;  // in-grid samples of each view
    RayRec* rays = nullptr;         // device [n_views][n_bins]
    ViewRec* vrec = nullptr;        // device [n_views]
    int pitch_x = 0, pitch_y = 0;   // line pitches of the two line images
    // smallest bin distance at which two rays of one class and one view lie at
    // least two cells apart on every line of the grid (scatter backprojector)
    int scatter_gap = 1 << 30;
};

}  // namespace fbpnp

namespace fbpnp {
// One axis of a bicubic sketch table on the device: output r reads inputs
// lo[r] .. lo[r] + taps - 1 with weights w[r * taps + t].
struct SketchAxis {
    int* lo = nullptr;
    float* w = nullptr;
    int taps = 0;
};
// S along x (nxs outputs) and y (nys outputs), and S^T along x (nx) and y (ny).
struct StageSketch {
    SketchAxis dx, dy, ux, uy;
};
}  // namespace fbpnp

struct fb_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct fb_plan {
    fb_geom g{};
    std::vector<fbpnp::Stage> stages;
    int device = 0;
    // workspace (device)
    float* line_x = nullptr;   // x-major line image: [nxs][pitch_x], largest stage
    float* line_y = nullptr;   // y-major line image: [nys][pitch_y]
    float* resid = nullptr;    // [n_views][n_bins]
    float* zbuf = nullptr;     // [ny][nx]
    float* vec = nullptr;      // power iteration: 2 x [ny][nx] + reductions
    size_t vec_floats = 0;
    std::vector<fb_launch_config> cfg;  // per stage; zero fields: defaults
    // sketch of the stages with f > 1: 0 average pooling, 1 bicubic (tables below)
    int sketch = 0;
    std::vector<fbpnp::StageSketch> sk;
    float* sk_tmp = nullptr;  // [ny][nx / f] of the largest coarse width
    float* sk_g = nullptr;    // coarse gradient [nys][nxs]
};

namespace fbpnp {

// Thread-local error reporting.
fb_status fail(fb_status code, const std::string& msg);
fb_status hip_fail(hipError_t e, const char* what);

// Host plan construction (double precision tables), in plan.cpp.
fb_status build_stage_tables(const fb_geom& g, int f, std::vector<RayRec>& rays, std::vector<ViewRec>& views,
                             std::vector<int64_t>& view_samples);
fb_status validate_geometry(const fb_geom& g);
// Stage::scatter_gap of a stage's ray and view tables.
int scatter_gap(const fb_geom& g, int f, const std::vector<RayRec>& rays, const std::vector<ViewRec>& views);
// Bicubic sketch table of one axis (n pixels, factor f): S (n / f rows) or its
// adjoint S^T (n rows), each row a window of `taps` consecutive inputs.
fb_status bicubic_axis_tables(int n, int f, bool adjoint, std::vector<int>& lo, std::vector<float>& w, int& taps);

// ---- launch helpers (kernels.hip), used by the forward and reverse entry points
constexpr int kRedBlocks = 256;  // blocks of the two-pass reductions
constexpr int kTvMaxFused = 8;   // TV steps one launch can hold

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
fb_status check_launch(const char* what);

// Timing events for the next projector / denoiser launch of this thread: when
// set, the launch helpers start their kernel with hipExtLaunchKernelGGL, which
// records begin at the kernel's start and end at its completion.
struct LaunchEvents {
    hipEvent_t begin = nullptr, end = nullptr;
};
extern thread_local LaunchEvents t_launch_events;
struct TimedLaunch {  // scoped: events ev[i], ev[i + 1] (ev may be NULL)
    TimedLaunch(hipEvent_t const* ev, int i) {
        if (ev) t_launch_events = {ev[i], ev[i + 1]};
    }
    ~TimedLaunch() { t_launch_events = LaunchEvents(); }
};
fb_status check_stage(const fb_plan* p, int stage);
fb_status check_views(const fb_plan* p, const int32_t* views, int n_sel);

// A selection of n views: list[i] (device) when list is not NULL, else
// view0 + step i.
struct ViewSel {
    const int32_t* list;
    int n;
    int view0 = 0, step = 1;
};
// The selection of a pnp_step (a list, an interleaved subset or every view),
// and its validation.
ViewSel pnp_views(const fb_pnp_args* a);
fb_status check_pnp_views(const fb_plan* p, const fb_pnp_args* a);

struct StageLines {
    float* lx;   // x-major line image [nxs][pitch_x]
    float* ly;   // y-major line image [nys][pitch_y], directly after lx
    int ly_off;  // ly - lx in floats
    int bytes;   // size of both images in bytes
};
StageLines stage_lines(const fb_plan* p, int stage);

// Pooling D_f of x (ny x nx) into the stage's line images.
fb_status launch_prepare(const fb_plan* p, int stage, const float* x, int nx, int f, hipStream_t s);
// Projection of the selected views from the stage's line images (minus b when resid).
// proj_out (optional): the raw projection by view, [n_views][n_bins].
fb_status launch_fp(const fb_plan* p, int stage, bool resid, const ViewSel& sel, const float* b, float* y,
                    hipStream_t s, float* proj_out = nullptr);
// Backprojection: xo = scale A_s^T y (coarse), or fused: z = yprev - scale D^T-replicate(A_s^T y).
fb_status launch_bp(const fb_plan* p, int stage, const float* y, const ViewSel& sel, float scale, float* xo,
                    const float* yprev, float* z, bool fused, hipStream_t s);

// Pooling target for the TV epilogue: the line images of the next stage.
struct PoolTarget {
    int f = 0;  // 0: none
    float inv = 0.f;
    float* lx = nullptr;
    float* ly = nullptr;
    int px = 0, py = 0, nxs = 0, nys = 0;
};
// tile: TV tile width (16 or 32), 0 for the default
fb_status launch_tv_single(const float* z, int nx, int ny, float lam, float tau, int n_iter, const float* p_in,
                           float* p_out, int mode, float alpha, float a_t, const float* x_prev, float* x_out,
                           float* y_out, float* hist, hipStream_t s, const PoolTarget& pt = PoolTarget(),
                           int tile = 0, unsigned long long* stamp = nullptr);

// Bicubic sketch (plans with sketch == 1, stages with f > 1): S of x into the
// stage's line images (or into v when v is set), and out = yprev - scale S^T g
// (out = scale S^T g when yprev is NULL).
fb_status launch_bicubic_down(const fb_plan* p, int stage, const float* x, float* v, hipStream_t s);
fb_status launch_bicubic_up(const fb_plan* p, int stage, const float* g, float scale, const float* yprev, float* out,
                            hipStream_t s);
inline bool bicubic_stage(const fb_plan* p, int stage) { return p->sketch == 1 && p->stages[stage].f > 1; }
void release_sketch(fb_plan* p);  // frees the bicubic tables (back to pooling)

// Captures what body launches on a private stream into an instantiated graph.
fb_status capture_graph(const std::function<fb_status(hipStream_t)>& body, fb_graph** out);

// Launch configurations: defaults, validation, and a plan stage's effective one.
int default_fp_seg(long waves1);
int default_bp_px(long npx);
// Side of a backprojection block in stage pixels: 8 bp_px for the gather form
// (bp_px = 1, 2, 4 pixels per lane), bp_px itself for the scatter form (16, 32).
int bp_block_side(int bp_px);
// Whether a stage's two line images fit in the LDS-staged forward projector.
bool fp_lds_fits(const fb_plan* p, int stage);
int default_bp_vg(int px, long nblk, int n_sel);
int default_tv_tile(long tiles32);
// True when the back-projector's pixel blocks of bw stage pixels, grown by the
// strip ends, reach the source circle (within 0.1 %): there the detector
// coordinate of a block corner is no projective value, and the back-projector
// runs with every bin of a view a candidate.
bool bp_blocks_reach_source(const fb_geom& g, const Stage& st, int bw);
fb_status check_config(const fb_launch_config& c);
fb_launch_config plan_config(const fb_plan* p, int stage, int n_sel);

}  // namespace fbpnp
