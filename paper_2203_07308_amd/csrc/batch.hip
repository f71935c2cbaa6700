// Batched form: one PnP-MS2G iteration (Sec. 2.1, Algorithm 1) for many
// independent slices of different sizes, view counts and detectors, each
// kernel of the iteration issued once for the whole batch.
//
// Every slice keeps its own plan (ray and view tables, line images, residual
// and z buffers). A launch covers all slices: its work-groups read their
// (slice, block) pair from a work-item table, then run the same device body
// as the single-image kernel with that slice's tables. The table lists the
// slices in longest-processing-time order (longest blocks first), and the
// hardware dispatcher hands work-groups to compute units in grid order as
// they free up, so the launch is scheduled greedily longest-first without a
// software queue.
//
// Caller data sits in packed arenas: images back to back (fb_batch_layout
// gives the offsets), sinograms likewise. View subsets are interleaved: with
// n_sub > 1 every slice uses its views k = subset + n_sub i.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <numeric>
#include <tuple>
#include <vector>

#include "batch.h"
#include "device.h"
#include "fbpnp_impl.h"

using namespace fbpnp;

namespace {

__device__ __forceinline__ int dcdiv(int a, int b) { return (a + b - 1) / b; }

// The slice, stage and local block of work-group blockIdx.x.
struct Item {
    const SliceDesc* d;
    int local;
};
__device__ __forceinline__ Item item_of(const SliceDesc* __restrict__ desc, const uint32_t* __restrict__ items) {
    const uint32_t it = items[blockIdx.x];
    return {desc + (it >> kLocalBits), (int)(it & kLocalMask)};
}

__global__ __launch_bounds__(256) void k_prepare_batch(const SliceDesc* __restrict__ desc,
                                                       const uint32_t* __restrict__ items, int stage,
                                                       const float* __restrict__ y) {
    const Item w = item_of(desc, items);
    const SliceDesc& D = *w.d;
    const BatchStage& S = D.st[stage];
    const int bxs = dcdiv(S.nxs, dev::kTile);
    dev::prepare_body(w.local % bxs, w.local / bxs, y + D.img_off, D.nx, S.f, S.inv_ff, S.nxs, S.nys, S.lines,
                      S.pitch_x, S.lines + S.ly_off, S.pitch_y);
}

template <int SEG>
__global__ __launch_bounds__(256) void k_fp_batch(const SliceDesc* __restrict__ desc,
                                                  const uint32_t* __restrict__ items, int stage, int view0,
                                                  int view_step, const float* __restrict__ b) {
    constexpr int R = 64 / SEG;
    const Item w = item_of(desc, items);
    const SliceDesc& D = *w.d;
    const BatchStage& S = D.st[stage];
    const int n_sel = dcdiv(D.n_views, view_step);
    dev::fp_body<true, SEG>(w.local, S.rays, D.n_bins, dcdiv(D.n_bins, R) * R, nullptr, view0, view_step, n_sel,
                            D.n_views, S.lines, S.ly_off, S.line_bytes, S.pitch_x, S.pitch_y, S.nxs, S.nys,
                            b + D.sino_off, D.resid, nullptr);
}

template <int VG, int PX, bool kAllBins = false>
__global__ __launch_bounds__(64 * VG) void k_bp_batch(const SliceDesc* __restrict__ desc,
                                                      const uint32_t* __restrict__ items, int stage, int view0,
                                                      int view_step, const float* __restrict__ eta, float sigma,
                                                      const float* __restrict__ y_prev) {
    const Item w = item_of(desc, items);
    const SliceDesc& D = *w.d;
    const BatchStage& S = D.st[stage];
    const int n_sel = dcdiv(D.n_views, view_step);
    const float scale = eta[w.d - desc] * sigma / (float)(S.f * S.f);
    dev::bp_body<VG, PX, true, kAllBins>(w.local, S.rays, S.vrec, D.n_bins, nullptr, view0, view_step, n_sel,
                                         D.n_views, D.resid, S.nxs, S.nys, dcdiv(S.nxs, 8 * PX), scale, nullptr, S.f,
                                         D.nx, y_prev + D.img_off, D.zbuf);
}

template <int BB, int VG>
__global__ __launch_bounds__(64 * VG) void k_bps_batch(const SliceDesc* __restrict__ desc,
                                                       const uint32_t* __restrict__ items, int stage, int view0,
                                                       int view_step, const float* __restrict__ eta, float sigma,
                                                       const float* __restrict__ y_prev) {
    const Item w = item_of(desc, items);
    const SliceDesc& D = *w.d;
    const BatchStage& S = D.st[stage];
    const int n_sel = dcdiv(D.n_views, view_step);
    const float scale = eta[w.d - desc] * sigma / (float)(S.f * S.f);
    dev::bps_body<BB, VG, true>(w.local, S.rays, S.vrec, D.n_bins, nullptr, view0, view_step, n_sel, D.n_views,
                                D.resid, S.nxs, S.nys, dcdiv(S.nxs, BB), S.scatter_gap, scale, nullptr, S.f, D.nx,
                                y_prev + D.img_off, D.zbuf);
}

template <int T, int H, int NT>
__global__ __launch_bounds__(NT) void k_tv_batch(const SliceDesc* __restrict__ desc,
                                                 const uint32_t* __restrict__ items, int next_stage, float lam,
                                                 float tau, int n_iter, float alpha, float a_t,
                                                 const float* __restrict__ x_prev, float* __restrict__ x_out,
                                                 float* __restrict__ y_out, float* __restrict__ hist) {
    const Item w = item_of(desc, items);
    const SliceDesc& D = *w.d;
    const int bxs = dcdiv(D.nx, T);
    int pf = 0, ppx = 0, ppy = 0, pnxs = 0, pnys = 0;
    float pinv = 0.f;
    float *plx = nullptr, *ply = nullptr;
    if (next_stage >= 0) {
        const BatchStage& N = D.st[next_stage];
        pf = N.f;
        pinv = N.inv_ff;
        plx = N.lines;
        ply = N.lines + N.ly_off;
        ppx = N.pitch_x;
        ppy = N.pitch_y;
        pnxs = N.nxs;
        pnys = N.nys;
    }
    const long long o = D.img_off;
    dev::tv_body<T, H, NT>(w.local % bxs, w.local / bxs, D.zbuf, D.nx, D.ny, lam, tau, n_iter, nullptr, nullptr, 1,
                           alpha, a_t, x_prev + o, x_out + o, y_out + o, hist ? hist + o : nullptr, pf, pinv, plx,
                           ppx, ply, ppy, pnxs, pnys);
}

// kernel launch on stream S, through hipExtLaunchKernelGGL when timing events are set
#define FB_BLAUNCH(K, G, B, S, ...)                                                  \
    do {                                                                             \
        const LaunchEvents ev_ = t_launch_events;                                    \
        if (ev_.begin || ev_.end)                                                    \
            hipExtLaunchKernelGGL(K, G, B, 0, S, ev_.begin, ev_.end, 0, __VA_ARGS__); \
        else                                                                         \
            K<<<G, B, 0, S>>>(__VA_ARGS__);                                          \
    } while (0)

int n_sel_of(int n_views, int n_sub) { return cdiv(n_views, n_sub); }

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace fbpnp {

fb_launch_config batch_config(const fb_batch* B, int stage, int n_sub) {
    fb_launch_config c = B->cfg[stage];
    long waves1 = 0, npx_max = 0, tiles32 = 0;
    int nsel_min = 1 << 30;
    for (const SliceDesc& D : B->h_desc) {
        const BatchStage& S = D.st[stage];
        const int ns = n_sel_of(D.n_views, n_sub);
        waves1 += (long)ns * cdiv(D.n_bins, 64);
        npx_max = std::max(npx_max, (long)S.nxs * S.nys);
        tiles32 += (long)cdiv(D.nx, 32) * cdiv(D.ny, 32);
        nsel_min = std::min(nsel_min, ns);
    }
    if (!c.fp_seg) c.fp_seg = default_fp_seg(waves1);
    if (!c.bp_px) c.bp_px = default_bp_px(npx_max);
    if (!c.bp_vg) {
        long nblk = 0;
        for (const SliceDesc& D : B->h_desc) {
            const BatchStage& S = D.st[stage];
            const int bw = bp_block_side(c.bp_px);
            nblk += (long)cdiv(S.nxs, bw) * cdiv(S.nys, bw);
        }
        c.bp_vg = default_bp_vg(c.bp_px, nblk, nsel_min);
        if (c.bp_px == 4 && c.bp_vg > 4) c.bp_vg = 4;
    }
    if (!c.tv_tile) c.tv_tile = default_tv_tile(tiles32);
    if (!c.fp_lds) c.fp_lds = 1;
    return c;
}

// Work-item table of one launch kind: slices in longest-processing-time
// order, each contributing its blocks in order. kind: 0 pooling, 1 forward
// projection (param = fp_seg), 2 backprojection (param = bp_px, whose block side
// is bp_block_side(bp_px)), 3 TV (param =
// tile side). Tables are built by set-up calls (batch creation, configuration
// changes, fb_batch_prepare, the autotuner, graph creation); a step only looks
// them up, so it never allocates or synchronises.
static fb_status work_items(fb_batch* B, int kind, int stage, int param, int n_sub, const ItemTable** out) {
    const auto key = std::make_tuple(kind, stage, param, n_sub);
    auto found = B->tables.find(key);
    if (found != B->tables.end()) {
        *out = &found->second;
        return FB_OK;
    }
    if (!B->building)
        return fail(FB_EINVAL, "batch: no work list for " + std::to_string(n_sub) +
                                   " subset(s) under the current launch configuration; call fb_batch_prepare "
                                   "first (set-up calls build them)");
    const int n = (int)B->h_desc.size();
    std::vector<long> blocks(n), cost(n);
    for (int i = 0; i < n; ++i) {
        const SliceDesc& D = B->h_desc[i];
        const BatchStage& S = D.st[stage];
        const int ns = n_sel_of(D.n_views, n_sub);
        switch (kind) {
            case 0:
                blocks[i] = (long)cdiv(S.nxs, 32) * cdiv(S.nys, 32);
                cost[i] = 1;
                break;
            case 1: {
                // a block marches 256 / seg rays of one view across the stage grid
                const int R = 64 / param;
                blocks[i] = (long)cdiv(ns * (cdiv(D.n_bins, R)), 4);
                cost[i] = std::max(S.nxs, S.nys);
                break;
            }
            case 2: {
                // a block takes every selected view over its pixel square
                const int bw = bp_block_side(param);
                blocks[i] = (long)cdiv(S.nxs, bw) * cdiv(S.nys, bw);
                cost[i] = (long)ns * S.f;
                break;
            }
            default:
                blocks[i] = (long)cdiv(D.nx, param) * cdiv(D.ny, param);
                cost[i] = 1;
                break;
        }
        if (blocks[i] > (long)kLocalMask) return fail(FB_EINVAL, "batch: a slice has too many blocks for a work item");
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<uint32_t> h;
    for (int i : order)
        for (long k = 0; k < blocks[i]; ++k) h.push_back(((uint32_t)i << kLocalBits) | (uint32_t)k);
    if (h.empty() || h.size() > (size_t)INT32_MAX) return fail(FB_EINVAL, "batch: empty or oversized work list");
    ItemTable t;
    t.n = (int)h.size();
    if (hipMalloc(&t.d, h.size() * sizeof(uint32_t)) != hipSuccess)
        return fail(FB_ENOMEM, "batch: work list allocation failed");
    hipError_t e = hipMemcpy(t.d, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(t.d);
        return hip_fail(e, "batch: work list upload");
    }
    *out = &(B->tables[key] = t);
    return FB_OK;
}

fb_status launch_fp_batch(fb_batch* B, int stage, int n_sub, int subset, const float* b, int seg, hipStream_t s) {
    const ItemTable* t;
    fb_status st = work_items(B, 1, stage, seg, n_sub, &t);
    if (st != FB_OK) return st;
    if (seg == 8) FB_BLAUNCH(k_fp_batch<8>, dim3(t->n), dim3(256), s, B->d_desc, t->d, stage, subset, n_sub, b);
    else if (seg == 4) FB_BLAUNCH(k_fp_batch<4>, dim3(t->n), dim3(256), s, B->d_desc, t->d, stage, subset, n_sub, b);
    else if (seg == 2) FB_BLAUNCH(k_fp_batch<2>, dim3(t->n), dim3(256), s, B->d_desc, t->d, stage, subset, n_sub, b);
    else FB_BLAUNCH(k_fp_batch<1>, dim3(t->n), dim3(256), s, B->d_desc, t->d, stage, subset, n_sub, b);
    return check_launch("batched fp");
}

// A slice whose back-projection blocks (bp_block_side(px) stage pixels) reach the source
// circle: the whole batch's back-projection at that stage takes every bin of a
// view as a candidate, with one pixel per lane.
static bool batch_all_bins(const fb_batch* B, int stage, int px) {
    for (const fb_plan* p : B->plans)
        if (bp_blocks_reach_source(p->g, p->stages[stage], bp_block_side(px))) return true;
    return false;
}

fb_status launch_bp_batch(fb_batch* B, int stage, int n_sub, int subset, const float* eta, float sigma,
                          const float* y_prev, int px, int vg, hipStream_t s) {
    const bool all_bins = batch_all_bins(B, stage, px);
    if (all_bins) px = 1;
    const ItemTable* t;
    fb_status st = work_items(B, 2, stage, px, n_sub, &t);
    if (st != FB_OK) return st;
    if (all_bins) {
        FB_BLAUNCH((k_bp_batch<4, 1, true>), dim3(t->n), dim3(256), s, B->d_desc, t->d, stage, subset, n_sub, eta,
                   sigma, y_prev);
        return check_launch("batched bp");
    }
#define FB_BPB(VG, PX)                                                                                           \
    FB_BLAUNCH((k_bp_batch<VG, PX>), dim3(t->n), dim3(64 * VG), s, B->d_desc, t->d, stage, subset, n_sub, eta, sigma, \
               y_prev)
#define FB_BPB_VG(PX)                 \
    switch (vg) {                     \
        case 1: FB_BPB(1, PX); break;  \
        case 2: FB_BPB(2, PX); break;  \
        case 4: FB_BPB(4, PX); break;  \
        case 8: FB_BPB(8, PX); break;  \
        default: FB_BPB(16, PX); break; \
    }
#define FB_BPSB(BB, VG)                                                                                          \
    FB_BLAUNCH((k_bps_batch<BB, VG>), dim3(t->n), dim3(64 * VG), s, B->d_desc, t->d, stage, subset, n_sub, eta, sigma, \
               y_prev)
#define FB_BPSB_VG(BB)                  \
    switch (vg) {                       \
        case 1: FB_BPSB(BB, 1); break;  \
        case 2: FB_BPSB(BB, 2); break;  \
        case 4: FB_BPSB(BB, 4); break;  \
        case 8: FB_BPSB(BB, 8); break;  \
        default: FB_BPSB(BB, 16); break; \
    }
    if (px == 32) {
        FB_BPSB_VG(32)
    } else if (px == 16) {
        FB_BPSB_VG(16)
    } else if (px == 4) {
        switch (vg) {
            case 1: FB_BPB(1, 4); break;
            case 2: FB_BPB(2, 4); break;
            default: FB_BPB(4, 4); break;
        }
    } else if (px == 2) {
        FB_BPB_VG(2)
    } else {
        FB_BPB_VG(1)
    }
#undef FB_BPSB_VG
#undef FB_BPSB
#undef FB_BPB_VG
#undef FB_BPB
    return check_launch("batched bp");
}

fb_status launch_tv_batch(fb_batch* B, int next_stage, float lam, float tau, int n_iter, float alpha, float a_t,
                          const float* x_prev, float* x_out, float* y_out, float* hist, int tile, hipStream_t s) {
    if (next_stage >= 0 && tile % B->factors[next_stage] != 0)
        return fail(FB_EINVAL, "pooling factor does not divide the TV tile");
    const ItemTable* t;
    fb_status st = work_items(B, 3, 0, tile, 1, &t);
    if (st != FB_OK) return st;
#define FB_TVB(TT, HH, NT)                                                                                      \
    FB_BLAUNCH((k_tv_batch<TT, HH, NT>), dim3(t->n), dim3(NT), s, B->d_desc, t->d, next_stage, lam, tau, n_iter, \
               alpha, a_t, x_prev, x_out, y_out, hist)
    if (tile == 16) {
        if (n_iter <= 5) FB_TVB(16, 6, 256);
        else FB_TVB(16, kTvMaxFused + 1, 256);
    } else {
        if (n_iter <= 5) FB_TVB(32, 6, 1024);
        else FB_TVB(32, kTvMaxFused + 1, 1024);
    }
#undef FB_TVB
    return check_launch("batched tv");
}

fb_status launch_prepare_batch(fb_batch* B, int stage, const float* y, hipStream_t s) {
    const ItemTable* t;
    fb_status st = work_items(B, 0, stage, 0, 1, &t);
    if (st != FB_OK) return st;
    k_prepare_batch<<<t->n, 256, 0, s>>>(B->d_desc, t->d, stage, y);
    return check_launch("batched prepare");
}

static fb_status check_batch_args(const fb_batch* B, const fb_batch_args* a) {
    if (!B || !a) return fail(FB_EINVAL, "batch: NULL batch or args");
    if (a->stage < 0 || a->stage >= B->n_stages) return fail(FB_EINVAL, "batch: stage index out of range");
    if (a->n_sub < 0 || a->subset < 0 || (a->n_sub > 1 && a->subset >= a->n_sub) || (a->n_sub <= 1 && a->subset != 0))
        return fail(FB_ESUBSET, "batch: need 0 <= subset < n_sub (subset 0 without subsets)");
    if (!a->eta || !a->b || !a->y_prev || !a->x_prev || !a->x_out || !a->y_out)
        return fail(FB_EINVAL, "batch: null buffer");
    if (a->tv_iters < 0 || a->tv_iters > kTvMaxFused) return fail(FB_EINVAL, "batch: tv_iters must be in [0, 8]");
    if (!(a->lambda >= 0.f) || !(a->tau > 0.f)) return fail(FB_EINVAL, "batch: need lambda >= 0 and tau > 0");
    if (a->next_stage < -1 || a->next_stage >= B->n_stages) return fail(FB_EINVAL, "batch: next_stage out of range");
    if (a->prepared != 0 && a->prepared != 1) return fail(FB_EINVAL, "batch: prepared must be 0 or 1");
    return FB_OK;
}

fb_status ensure_tables(fb_batch* B, int n_sub) {
    n_sub = std::max(1, n_sub);
    BuildScope scope(B);
    const ItemTable* t;
    fb_status st;
    for (int k = 0; k < B->n_stages; ++k) {
        const fb_launch_config c = batch_config(B, k, n_sub);
        if ((st = work_items(B, 0, k, 0, 1, &t)) != FB_OK) return st;
        if ((st = work_items(B, 1, k, c.fp_seg, n_sub, &t)) != FB_OK) return st;
        const int bp_px = batch_all_bins(B, k, c.bp_px) ? 1 : c.bp_px;  // as launch_bp_batch chooses
        if ((st = work_items(B, 2, k, bp_px, n_sub, &t)) != FB_OK) return st;
        if ((st = work_items(B, 3, 0, c.tv_tile, 1, &t)) != FB_OK) return st;
    }
    B->prepared.insert(n_sub);
    return FB_OK;
}

}  // namespace fbpnp

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

fb_status fb_batch_create(const fb_geom* geoms, int n_slices, int n_stages, const int32_t* factors, fb_batch** out) {
    if (!geoms || !factors || !out || n_slices < 1) return fail(FB_EINVAL, "fb_batch_create: bad arguments");
    if (n_slices > kMaxSlices) return fail(FB_EINVAL, "fb_batch_create: too many slices");
    if (n_stages < 1 || n_stages > kMaxBatchStages) return fail(FB_EINVAL, "fb_batch_create: 1 to 4 stages");
    *out = nullptr;
    fb_batch* B = new fb_batch();
    B->n_stages = n_stages;
    B->factors.assign(factors, factors + n_stages);
    B->cfg.assign(n_stages, fb_launch_config{0, 0, 0, 0, 0});
    int64_t io = 0, so = 0;
    for (int i = 0; i < n_slices; ++i) {
        fb_plan* p = nullptr;
        fb_status st = fb_plan_create(&geoms[i], n_stages, factors, &p);
        if (st != FB_OK) {
            fb_batch_destroy(B);
            return st;
        }
        B->plans.push_back(p);
        SliceDesc D{};
        D.nx = p->g.nx;
        D.ny = p->g.ny;
        D.n_views = p->g.n_views;
        D.n_bins = p->g.n_bins;
        D.img_off = io;
        D.sino_off = so;
        D.resid = p->resid;
        D.zbuf = p->zbuf;
        for (int k = 0; k < n_stages; ++k) {
            const Stage& S = p->stages[k];
            const StageLines L = stage_lines(p, k);
            BatchStage& b = D.st[k];
            b.rays = S.rays;
            b.vrec = S.vrec;
            b.lines = L.lx;
            b.ly_off = L.ly_off;
            b.line_bytes = L.bytes;
            b.pitch_x = S.pitch_x;
            b.pitch_y = S.pitch_y;
            b.nxs = S.nxs;
            b.nys = S.nys;
            b.f = S.f;
            b.scatter_gap = S.scatter_gap;
            b.inv_ff = 1.f / (float)(S.f * S.f);
        }
        B->h_desc.push_back(D);
        B->img_off.push_back(io);
        B->sino_off.push_back(so);
        // 64-float (256-byte) aligned slots
        io += ((int64_t)D.nx * D.ny + 63) / 64 * 64;
        so += ((int64_t)D.n_views * D.n_bins + 63) / 64 * 64;
    }
    B->img_off.push_back(io);
    B->sino_off.push_back(so);
    if (hipMalloc(&B->d_desc, B->h_desc.size() * sizeof(SliceDesc)) != hipSuccess) {
        fb_batch_destroy(B);
        return fail(FB_ENOMEM, "fb_batch_create: descriptor allocation failed");
    }
    hipError_t e = hipMemcpy(B->d_desc, B->h_desc.data(), B->h_desc.size() * sizeof(SliceDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        fb_batch_destroy(B);
        return hip_fail(e, "fb_batch_create: descriptor upload");
    }
    fb_status st = ensure_tables(B, 1);  // steps over all views need no further set-up
    if (st != FB_OK) {
        fb_batch_destroy(B);
        return st;
    }
    *out = B;
    return FB_OK;
}

fb_status fb_batch_destroy(fb_batch* B) {
    if (!B) return FB_OK;
    for (auto& kv : B->tables)
        if (kv.second.d) (void)hipFree(kv.second.d);
    if (B->d_desc) (void)hipFree(B->d_desc);
    for (fb_plan* p : B->plans) fb_plan_destroy(p);
    delete B;
    return FB_OK;
}

fb_status fb_batch_layout(const fb_batch* B, int64_t* image_offsets, int64_t* sino_offsets) {
    if (!B || !image_offsets || !sino_offsets) return fail(FB_EINVAL, "fb_batch_layout: bad arguments");
    std::copy(B->img_off.begin(), B->img_off.end(), image_offsets);
    std::copy(B->sino_off.begin(), B->sino_off.end(), sino_offsets);
    return FB_OK;
}

fb_status fb_batch_slice_plan(fb_batch* B, int slice, fb_plan** out) {
    if (!B || !out || slice < 0 || slice >= (int)B->plans.size()) return fail(FB_EINVAL, "fb_batch_slice_plan: bad arguments");
    *out = B->plans[slice];
    return FB_OK;
}

fb_status fb_batch_set_config(fb_batch* B, int stage, const fb_launch_config* cfg) {
    if (!B || stage < 0 || stage >= B->n_stages) return fail(FB_EINVAL, "fb_batch_set_config: bad arguments");
    const fb_launch_config c = cfg ? *cfg : fb_launch_config{0, 0, 0, 0, 0};
    fb_status st = check_config(c);
    if (st != FB_OK) return st;
    if (c.fp_lds == 2) return fail(FB_EINVAL, "launch config: batches read projector taps from global memory");
    const fb_launch_config old = B->cfg[stage];
    B->cfg[stage] = c;
    for (int n_sub : std::set<int>(B->prepared))
        if ((st = ensure_tables(B, n_sub)) != FB_OK) {
            B->cfg[stage] = old;
            return st;
        }
    return FB_OK;
}

fb_status fb_batch_prepare(fb_batch* B, int n_sub) {
    if (!B || n_sub < 0) return fail(FB_EINVAL, "fb_batch_prepare: bad arguments");
    return ensure_tables(B, n_sub);
}

fb_status fb_batch_get_config(const fb_batch* B, int stage, int n_sub, fb_launch_config* out) {
    if (!B || !out || stage < 0 || stage >= B->n_stages) return fail(FB_EINVAL, "fb_batch_get_config: bad arguments");
    *out = batch_config(B, stage, std::max(1, n_sub));
    return FB_OK;
}

fb_status pnp_step_batched(fb_batch* B, const fb_batch_args* a, hipStream_t stream) {
    fb_status st = check_batch_args(B, a);
    if (st != FB_OK) return st;
    const int n_sub = std::max(1, a->n_sub);
    const fb_launch_config c = batch_config(B, a->stage, n_sub);
    if (!a->prepared && (st = launch_prepare_batch(B, a->stage, a->y_prev, stream)) != FB_OK) return st;
    {
        TimedLaunch tl(a->events, 0);
        if ((st = launch_fp_batch(B, a->stage, n_sub, a->subset, a->b, c.fp_seg, stream)) != FB_OK) return st;
    }
    {
        TimedLaunch tl(a->events, 2);
        if ((st = launch_bp_batch(B, a->stage, n_sub, a->subset, a->eta, a->sigma, a->y_prev, c.bp_px, c.bp_vg,
                                  stream)) != FB_OK)
            return st;
    }
    // lambda == 0 or no TV iterations: the TV kernel only relaxes and applies momentum
    const float lam = a->lambda > 0.f ? a->lambda : 1.f;
    const int iters = a->lambda > 0.f ? a->tv_iters : 0;
    // the next stage's pooling goes into the TV epilogue when its factor
    // divides the TV tile, else into a pooling launch after it
    const bool pool_after = a->next_stage >= 0 && c.tv_tile % B->factors[a->next_stage] != 0;
    {
        TimedLaunch tl(a->events, 4);
        if ((st = launch_tv_batch(B, pool_after ? -1 : a->next_stage, lam, a->tau, iters, a->alpha, a->a_t,
                                  a->x_prev, a->x_out, a->y_out, a->history, c.tv_tile, stream)) != FB_OK)
            return st;
    }
    return pool_after ? launch_prepare_batch(B, a->next_stage, a->y_out, stream) : FB_OK;
}

fb_status fb_batch_graph_create(fb_batch* B, const fb_batch_args* steps, int n_steps, fb_graph** out) {
    if (!B || !steps || n_steps < 1 || !out) return fail(FB_EINVAL, "fb_batch_graph_create: bad arguments");
    *out = nullptr;
    std::vector<fb_batch_args> chain(steps, steps + n_steps);
    fb_status st;
    for (int i = 0; i < n_steps; ++i) {
        if ((st = check_batch_args(B, &chain[i])) != FB_OK) return st;
        chain[i].prepared = 0;
        chain[i].next_stage = -1;
        chain[i].events = nullptr;  // kernel timing is for direct calls only
        if ((st = ensure_tables(B, chain[i].n_sub)) != FB_OK) return st;
    }
    // step i pools its y_t for step i + 1 when that step reads it
    for (int i = 0; i + 1 < n_steps; ++i) {
        if (chain[i + 1].y_prev == chain[i].y_out) {
            chain[i].next_stage = chain[i + 1].stage;
            chain[i + 1].prepared = 1;
        }
    }
    auto body = [&](hipStream_t s) {
        fb_status r = FB_OK;
        for (int i = 0; i < n_steps && r == FB_OK; ++i) r = pnp_step_batched(B, &chain[i], s);
        return r;
    };
    return capture_graph(body, out);
}

}  // extern "C"
