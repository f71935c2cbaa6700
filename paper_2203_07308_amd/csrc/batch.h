// Batched form: per-slice descriptors read by the batched kernels, the batch
// object, and the host helpers the autotuner shares.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "fbpnp_impl.h"

namespace fbpnp {

constexpr int kMaxBatchStages = 4;
constexpr int kLocalBits = 20;  // a work item is slice << kLocalBits | block of that slice
constexpr uint32_t kLocalMask = (1u << kLocalBits) - 1;
constexpr int kMaxSlices = 1 << (32 - kLocalBits);

// One stage of one slice, as the batched kernels see it (device memory).
struct BatchStage {
    const RayRec* rays;
    const ViewRec* vrec;
    float* lines;  // x-major line image; the y-major one starts ly_off floats later
    int ly_off, line_bytes, pitch_x, pitch_y, nxs, nys, f;
    int scatter_gap;  // the plan stage's scatter_gap
    float inv_ff;
};

struct SliceDesc {
    int nx, ny, n_views, n_bins;
    long long img_off, sino_off;  // offsets (floats) of the slice in the caller's arenas
    float* resid;                 // the slice plan's residual [n_views][n_bins]
    float* zbuf;                  // the slice plan's z [ny][nx]
    BatchStage st[kMaxBatchStages];
};

struct ItemTable {
    uint32_t* d = nullptr;
    int n = 0;
};

}  // namespace fbpnp

struct fb_batch {
    std::vector<fb_plan*> plans;
    int n_stages = 0;
    std::vector<int> factors;
    std::vector<fbpnp::SliceDesc> h_desc;
    fbpnp::SliceDesc* d_desc = nullptr;
    std::vector<int64_t> img_off, sino_off;  // n_slices + 1 entries
    std::vector<fb_launch_config> cfg;       // per stage; zero fields: defaults
    std::map<std::tuple<int, int, int, int>, fbpnp::ItemTable> tables;
    std::set<int> prepared;  // subset counts whose work lists follow every configuration change
    bool building = false;   // set-up calls only: missing work lists may be built (allocates, synchronises)
};

namespace fbpnp {

fb_launch_config batch_config(const fb_batch* B, int stage, int n_sub);
// Builds every work list that steps with n_sub subsets use under the current
// launch configurations (a set-up call: allocates and synchronises).
fb_status ensure_tables(fb_batch* B, int n_sub);
// Scoped permission for a set-up call to build missing work lists.
struct BuildScope {
    fb_batch* B;
    bool was;
    explicit BuildScope(fb_batch* b) : B(b), was(b->building) { B->building = true; }
    ~BuildScope() { B->building = was; }
};
fb_status launch_prepare_batch(fb_batch* B, int stage, const float* y, hipStream_t s);
fb_status launch_fp_batch(fb_batch* B, int stage, int n_sub, int subset, const float* b, int seg, hipStream_t s);
fb_status launch_bp_batch(fb_batch* B, int stage, int n_sub, int subset, const float* eta, float sigma,
                          const float* y_prev, int px, int vg, hipStream_t s);
fb_status launch_tv_batch(fb_batch* B, int next_stage, float lam, float tau, int n_iter, float alpha, float a_t,
                          const float* x_prev, float* x_out, float* y_out, float* hist, int tile, hipStream_t s);

}  // namespace fbpnp
