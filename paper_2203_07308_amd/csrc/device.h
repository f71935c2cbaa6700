// Device bodies of the hot-path kernels, shared by the single-image kernels
// (kernels.hip) and the batched ones (batch.hip). Each body computes one
// work-group's share given its block index, so a batched kernel maps its block
// to (slice, block) and calls the same code with that slice's tables.
//
// Hot path of one PnP-MS2G iteration (Sec. 2.1, Algorithm 1 with the
// least-squares data term of Eq. (5)-(7)):
//   prepare_body  pooling S = D_f of y_{t-1} into the stage's two "line images"
//   fp_body       Joseph forward projection of the selected views, minus b
//   bp_body       matched backprojection as a pixel-driven gather, fused with
//                 the upsampler U = D_f^T and the gradient step z = y - eta U G
//   tv_body       Chambolle TV-prox iterations in LDS, fused with the
//                 relaxation and the momentum step
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fbpnp_impl.h"

namespace fbpnp {
namespace dev {

// ---------------------------------------------------------------------------
// Line images: the stage image v (ny_s x nx_s) stored twice, as
//   lx[c][kPad + r] = v[r][c]   (lines = columns, used by x-major rays)
//   ly[r][kPad + c] = v[r][c]   (lines = rows, used by y-major rays)
// with kPad zeros at both ends of every line (written once at plan creation).
// Along a line, the rays of one view that a wavefront handles sample nearby
// positions, so their two interpolation taps are contiguous loads.
// ---------------------------------------------------------------------------
constexpr int kTile = 32;

// Work-groups are handed to the GPU's 8 XCDs (each with its own L2) in turn by
// launch index. Launch index id of n work-groups of a spatial launch gets tile
// xcd_tile(id, n): XCD k = id mod 8 takes the k-th of 8 consecutive runs of
// tiles (tiles are row-major), so the back-projector blocks that write z and
// y_t of a band of image rows and the denoiser tiles that read them run on
// the same XCD and find them in its L2.
__device__ __forceinline__ int xcd_tile(int id, int n) {
    const int q = n >> 3, r = n & 7, k = id & 7, j = id >> 3;
    return k * q + min(k, r) + j;
}

// Sum of an F x F block of an image with row pitch S (global memory or LDS),
// added from zero in row order; all F^2 reads are issued before the sum.
template <int F>
__device__ __forceinline__ float pool_block(const float* __restrict__ b, int S) {
    float v[F * F];
#pragma unroll
    for (int a = 0; a < F; ++a)
#pragma unroll
        for (int c = 0; c < F; ++c) v[a * F + c] = b[a * S + c];
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < F * F; ++k) s += v[k];
    return s;
}

// v = D_f x (x: ny x nx, full grid; f = 1 copies), written into both line images.
__device__ __forceinline__ void prepare_body(int bx, int by, const float* __restrict__ x, int nx, int f,
                                             float inv_ff, int nxs, int nys, float* __restrict__ lx, int pitch_x,
                                             float* __restrict__ ly, int pitch_y) {
    __shared__ float tile[kTile][kTile + 1];
    const int C0 = bx * kTile, R0 = by * kTile;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int rr = ty; rr < kTile; rr += 8) {
        const int R = R0 + rr, C = C0 + tx;
        float s = 0.f;
        if (R < nys && C < nxs) {
            if (f == 1) {
                s = x[(size_t)R * nx + C];
            } else {
                const float* const blk = x + (size_t)(f * R) * nx + (size_t)f * C;
                if (f == 2) s = pool_block<2>(blk, nx);
                else if (f == 3) s = pool_block<3>(blk, nx);
                else if (f == 4) s = pool_block<4>(blk, nx);
                else
                    for (int a = 0; a < f; ++a)
                        for (int b = 0; b < f; ++b) s += blk[(size_t)a * nx + b];
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
// Forward projection: SEG work-items per (selected view, bin), each marching
// a contiguous share of the ray's samples (SEG > 1 when there are too few rays
// to fill the GPU). The 64/SEG rays of a wavefront are consecutive bins of
// one view, so the ray-table read is coalesced and the taps fall on
// neighbouring positions of the same line.
//   y[i][j] = len_j * sum_k [ (1-w) v(line lo+k, p0) + w v(line lo+k, p0+1) ]
//             (- b[view_i][j] when kResid)
// with p = npos/2 + fma(lo + k - nlines/2, dpos, pos_c), p0 = floor(p),
// w = fract(p) (zero outside the grid).
// ---------------------------------------------------------------------------
// Buffer resource word 3 for raw (untyped) buffer loads on CDNA.
constexpr int kBufWord3 = 0x00020000;

// The value of lane (lane ^ o) for a power of two o < 64, by DPP lane moves
// where one exists. kAny: any lane partner inside the same aligned group of 2o
// lanes that lies in the other half will do (min and max reductions); else the
// partner is exactly lane ^ o.
template <bool kAny, typename T>
__device__ __forceinline__ T lane_pair(T v, int o) {
    const int iv = __builtin_bit_cast(int, v);
    int r;
    if (o == 1) r = __builtin_amdgcn_update_dpp(iv, iv, 0xB1, 0xF, 0xF, false);       // quad_perm 1,0,3,2
    else if (o == 2) r = __builtin_amdgcn_update_dpp(iv, iv, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    else if (o == 4 && kAny) r = __builtin_amdgcn_update_dpp(iv, iv, 0x141, 0xF, 0xF, false);  // row_half_mirror
    else if (o == 8) r = __builtin_amdgcn_update_dpp(iv, iv, 0x128, 0xF, 0xF, false);  // row_ror 8
    else r = __shfl_xor(iv, o);
    return __builtin_bit_cast(T, r);
}

// The two interpolation taps at byte offset off of the stage's line images:
// from global memory (through a buffer resource over both images, so a load
// outside them would return zero instead of faulting) or from a copy of the
// images in LDS.
struct TapsGlobal {
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ TapsGlobal(const float* lines, int line_bytes)
        : rsrc(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(lines), (short)0, line_bytes, kBufWord3)) {}
    __device__ __forceinline__ void operator()(int off, float& a, float& c) const {
        const auto t = __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0);
        a = __uint_as_float(t[0]);
        c = __uint_as_float(t[1]);
    }
};
struct TapsLds {
    const float* lds;
    __device__ __forceinline__ void operator()(int off, float& a, float& c) const {
        const float* q = lds + (off >> 2);
        a = q[0];
        c = q[1];
    }
};

// Projection work of 256 threads (local thread index tid), block blk of the
// launch's rays; view i of the selection is views[i], or view0 + i * view_step
// without a list. proj_out (optional): the projection itself, before b is
// subtracted, stored by view ([n_views][n_bins]).
template <bool kResid, int SEG, typename Taps>
__device__ __forceinline__ void fp_block(int blk, int tid, const Taps& taps, const RayRec* __restrict__ rays,
                                         int n_bins, int bins_padded, const int32_t* __restrict__ views, int view0,
                                         int view_step, int n_sel, int n_views, int ly_off, int pitch_x, int pitch_y,
                                         int nxs, int nys, const float* __restrict__ b, float* __restrict__ y,
                                         float* __restrict__ proj_out) {
    constexpr int R = 64 / SEG;  // rays per wavefront; SEG lanes share one ray
    const int lane = tid & 63;
    const int wave = (blk * 256 + tid) >> 6;
    const int waves_per_view = bins_padded / R;
    const int i = wave / waves_per_view;
    const int j = (wave - i * waves_per_view) * R + lane % R;
    const int seg = lane / R;
    const bool active = i < n_sel && j < n_bins;
    int v = 0;
    if (active) v = views ? views[i] : view0 + i * view_step;
    const bool valid = active && (unsigned)v < (unsigned)n_views;  // invalid view index: a zero row
    RayRec r{0.f, 0.f, 0.f, 0u};
    float bj = 0.f;  // b is read with the ray record, ahead of the march
    if (valid) {
        r = rays[(size_t)v * n_bins + j];
        if (kResid && seg == 0) bj = b[(size_t)v * n_bins + j];
    }
    const int lo = (int)(r.bits & 0xFFFFu), n = (int)((r.bits >> 16) & 0x7FFFu);
    const bool ymaj = (r.bits >> 31) != 0u;
    if (n == 0) {  // no samples (or no ray): every position clamps into the padding
        r.pos_c = -1e30f;
        r.dpos = 0.f;
    }
    // All lanes march the same lines in lockstep (the union of the wavefront's
    // sample ranges, split into SEG parts), so one load instruction reads
    // neighbouring positions of one line. Outside its own range a ray's
    // position is clamped into the zero padding and adds nothing. The SEG
    // lanes of a ray hold the same record, so the range is reduced over the R
    // lanes of one segment.
    int L0 = n > 0 ? lo : 1 << 30, L1 = n > 0 ? lo + n : -(1 << 30);
#pragma unroll
    for (int o = 1; o < R; o <<= 1) {
        L0 = min(L0, lane_pair<true>(L0, o));
        L1 = max(L1, lane_pair<true>(L1, o));
    }
    float acc = 0.f;
    if (L1 > L0) {
        // a wavefront can hold rays of both classes, whose lines run along different
        // axes: each lane stops at the end of its own axis (beyond it the position of
        // a ray is not kept out of the grid, and the reads would fall in the other image)
        const int nlines = ymaj ? nys : nxs;
        const int la = L0 + ((L1 - L0) * seg) / SEG, lb = min(L0 + ((L1 - L0) * (seg + 1)) / SEG, nlines);
        const int pitch = ymaj ? pitch_y : pitch_x;
        const int npos = ymaj ? nxs : nys;
        const int mid = npos >> 1, lmid = nlines >> 1;
        const float plo = (float)(-2 - mid), phi = (float)(npos - mid);
        // byte offset of position mid on line la
        int off = ((ymaj ? ly_off : 0) + la * pitch + kPad + mid) * 4;
        const int step = pitch * 4;
        float kf = (float)(la - lmid);
#pragma unroll 4
        for (int l = la; l < lb; ++l) {
            const float p = __builtin_amdgcn_fmed3f(fmaf(kf, r.dpos, r.pos_c), plo, phi);
            const float w = __builtin_amdgcn_fractf(p);
            const int i0 = (int)floorf(p);
            float a, c;
            taps(off + i0 * 4, a, c);
            acc += fmaf(w, c - a, a);
            kf += 1.f;
            off += step;
        }
    }
    // fixed-order sum of the SEG partial sums of each ray
#pragma unroll
    for (int o = R; o < 64; o <<= 1) acc += lane_pair<false>(acc, o);
    if (active && seg == 0) {
        float val = 0.f;
        if (valid) {
            // the residual as an explicit fused multiply-add, so every kernel rounds it alike
            const float p = acc * r.len;
            if (proj_out) proj_out[(size_t)v * n_bins + j] = p;
            val = kResid ? fmaf(acc, r.len, -bj) : p;
        }
        y[(size_t)i * n_bins + j] = val;
    }
}

// Work-group blk (256 threads) of a projection with its taps from global memory.
template <bool kResid, int SEG>
__device__ __forceinline__ void fp_body(int blk, const RayRec* __restrict__ rays, int n_bins, int bins_padded,
                                        const int32_t* __restrict__ views, int view0, int view_step, int n_sel,
                                        int n_views, const float* __restrict__ lines, int ly_off, int line_bytes,
                                        int pitch_x, int pitch_y, int nxs, int nys, const float* __restrict__ b,
                                        float* __restrict__ y, float* __restrict__ proj_out = nullptr) {
    fp_block<kResid, SEG>(blk, (int)threadIdx.x, TapsGlobal(lines, line_bytes), rays, n_bins, bins_padded, views,
                          view0, view_step, n_sel, n_views, ly_off, pitch_x, pitch_y, nxs, nys, b, y, proj_out);
}

// Projection with the stage's two line images staged in LDS (lds_floats of
// them, copied by the whole work-group), for stages small enough to fit:
// every 256-thread quarter of the work-group then takes blocks q + 4
// gridDim.x k of the launch's rays, reading its taps from LDS.
template <bool kResid, int SEG>
__device__ __forceinline__ void fp_body_lds(float* __restrict__ lds, int lds_floats, int n_blocks,
                                            const RayRec* __restrict__ rays, int n_bins, int bins_padded,
                                            const int32_t* __restrict__ views, int view0, int view_step, int n_sel,
                                            int n_views, const float* __restrict__ lines, int ly_off, int pitch_x,
                                            int pitch_y, int nxs, int nys, const float* __restrict__ b,
                                            float* __restrict__ y, float* __restrict__ proj_out) {
    const float4* src = reinterpret_cast<const float4*>(lines);
    float4* dst = reinterpret_cast<float4*>(lds);
    for (int e = threadIdx.x; e < (lds_floats >> 2); e += blockDim.x) dst[e] = src[e];
    __syncthreads();
    const TapsLds taps{lds};
    const int quarter = threadIdx.x >> 8, tid = threadIdx.x & 255;
    for (int blk = blockIdx.x * 4 + quarter; blk < n_blocks; blk += gridDim.x * 4)
        fp_block<kResid, SEG>(blk, tid, taps, rays, n_bins, bins_padded, views, view0, view_step, n_sel, n_views,
                              ly_off, pitch_x, pitch_y, nxs, nys, b, y, proj_out);
}

// ---------------------------------------------------------------------------
// Matched backprojection, pixel-driven gather.
//
// A wavefront owns a block of 8 PX x 8 PX stage pixels, each lane a PX x PX
// block. For every selected view the wavefront first copies the ray records
// of the bins its block can touch (found from the detector coordinate j(c, r)
// of the block corners) into its own LDS slot, with y * len folded in. Each
// lane then finds the rays that can touch its pixels from j(c, r) at the ends
// of its strips and recomputes every candidate's interpolation weight from
// the same float position k_fp uses (same operations on the same table
// entries):
//   x-major ray, column cc: p = nys/2 + fma(cc - nxs/2, dpos, pos_c),
//   row floor(p) receives 1 - fract(p) and row floor(p)+1 receives fract(p).
// A ray without a sample on the strip's line has p outside [-1, npos) there
// (the plan guarantees it), so it adds nothing.
// The VG wavefronts of a workgroup share the pixel block and split the views;
// their partial sums are added in a fixed order in LDS, so results are
// bitwise reproducible (no atomics).
// ---------------------------------------------------------------------------
constexpr float kProjEps = 0.02f;  // margin on candidate bin ranges (FP32 error is ~1e-4 bins)
constexpr int kStageRays = 128;    // ray records staged per wavefront and view

__device__ __forceinline__ float proj_bin(const ViewRec& v, float c, float r) {
    const float num = fmaf(v.a2, r, fmaf(v.a1, c, v.a0));
    const float den = fmaf(v.b2, r, fmaf(v.b1, c, v.b0));
    return fmaf(num, __builtin_amdgcn_rcpf(den), v.j0);
}

__device__ __forceinline__ void cand_range(float j1, float j2, int lo, int hi, int& jl, int& jh) {
    const float a = fmaxf(ceilf(fminf(j1, j2) - kProjEps), (float)lo);
    const float b = fminf(floorf(fmaxf(j1, j2) + kProjEps), (float)hi);
    jl = (int)a;
    jh = (int)b;
}

// Adds one sample (centred position p, weighted value yy) to a strip of PX
// pixels whose first centred position is qf. Pixel qf+t receives the linear
// interpolation weight max(0, 1 - |p - (qf+t)|): 1 - fract(p) on row floor(p)
// and fract(p) on row floor(p)+1, as in k_fp (exactly so for |p| >= 1, where
// every difference involved is representable; within one rounding otherwise).
template <int PX>
__device__ __forceinline__ void strip_add(float p, float qf, float yy, float (&s)[PX]) {
#pragma unroll
    for (int t = 0; t < PX; ++t) {
        // 1 - |p - q| is at most 1, so clamping it to [0, 1] is the max with 0
        // (one subtraction with the output clamp)
        const float wt = __builtin_amdgcn_fmed3f(1.f - fabsf(p - (qf + (float)t)), 0.f, 1.f);
        s[t] = fmaf(wt, yy, s[t]);
    }
}

// Candidate rays jl..jh (one dominance class, staged from bin base) for a
// strip on a line whose offset from the middle line is kf, first centred
// position qm.
template <int PX>
__device__ __forceinline__ void gather_strip(const float* __restrict__ st, int base, int jl, int jh, float kf,
                                             int qm, float (&s)[PX]) {
    const float qf = (float)qm;
    // walk the staged records by address (one counter for the loop and the load)
    const float* const end = st + (jh - base);
    for (const float* e = st + (jl - base); e <= end; ++e) {
        strip_add<PX>(fmaf(kf, e[kStageRays], e[0]), qf, e[2 * kStageRays], s);
    }
}

// All strips of one dominance class for one staged view. The candidate bins
// of a strip come from j(c, r) at its two ends (the numerator and the
// denominator of j are linear in c and r); lo..hi is the class range within
// the staged chunk. kAllBins: every ray of the class range is a candidate
// (for stages whose pixel blocks, grown by the strip ends, reach the source
// circle, where j of the block corners is no longer a valid projective value).
template <int PX, bool kXMajor, bool kAllBins>
__device__ __forceinline__ void bp_class(const ViewRec& vr, const float* __restrict__ st, int base, int lo,
                                         int hi, float cc, float rc, int c, int r, int mid_c, int mid_r,
                                         float (&acc)[PX][PX]) {
    if (lo > hi) return;
    // x-major: strips are columns c+t over rows r-1 .. r+PX;
    // y-major: strips are rows r+t over columns c-1 .. c+PX
    const float n0 = kXMajor ? fmaf(vr.a2, rc - 1.f, fmaf(vr.a1, cc, vr.a0))
                             : fmaf(vr.a2, rc, fmaf(vr.a1, cc - 1.f, vr.a0));
    const float d0 = kXMajor ? fmaf(vr.b2, rc - 1.f, fmaf(vr.b1, cc, vr.b0))
                             : fmaf(vr.b2, rc, fmaf(vr.b1, cc - 1.f, vr.b0));
    const float an = kXMajor ? vr.a2 : vr.a1, bn = kXMajor ? vr.b2 : vr.b1;  // along the strip
    const float at = kXMajor ? vr.a1 : vr.a2, bt = kXMajor ? vr.b1 : vr.b2;  // across strips
    const float dn = an * (float)(PX + 1), dd = bn * (float)(PX + 1);
#pragma unroll
    for (int t = 0; t < PX; ++t) {
        const float nt = fmaf(at, (float)t, n0), dt = fmaf(bt, (float)t, d0);
        int jl = lo, jh = hi;
        if constexpr (!kAllBins)
            cand_range(fmaf(nt, __builtin_amdgcn_rcpf(dt), vr.j0),
                       fmaf(nt + dn, __builtin_amdgcn_rcpf(dt + dd), vr.j0), lo, hi, jl, jh);
        float sacc[PX];
#pragma unroll
        for (int w = 0; w < PX; ++w) sacc[w] = 0.f;
        if (kXMajor) {
            gather_strip<PX>(st, base, jl, jh, (float)(c + t - mid_c), r - mid_r, sacc);
#pragma unroll
            for (int w = 0; w < PX; ++w) acc[w][t] += sacc[w];
        } else {
            gather_strip<PX>(st, base, jl, jh, (float)(r + t - mid_r), c - mid_c, sacc);
#pragma unroll
            for (int w = 0; w < PX; ++w) acc[t][w] += sacc[w];
        }
    }
}

// End of a backprojection work-group. The block's gradient values g (the
// wavefront parts in red, added in wavefront order) are finished by all
// threads together, one output value per thread and pass, in row order:
//   unfused: xo = scale g on the block's stage pixels;
//   fused:   z = y_prev - (eta sigma / f^2) g on the block's f x f fine pixels
//            (explicit fused multiply-adds: every kernel rounds this the same
//            way), with the optional extras mu (z = y_prev - mu_scale mu -
//            scale g) and g_out (g itself, stored once per stage pixel).
// Fine pixel e of block (bx, by) (row-major over its bw f x bw f fine
// pixels): stage pixel (cr, cc) within the block, fine pixel (FR, FC) in the
// image; false if outside. The quotients use float reciprocals rf = 1 / f and
// rfw = 1 / (bw f): a product is within (bw f) 2^-23 of the exact quotient,
// which lies at least 1 / (2 bw f) from an integer, so the truncation is
// exact while bw f < 2048 (bw <= 32 and f <= kMaxFactor give at most 1024).
__device__ __forceinline__ bool bp_fine_pixel(int e, int bw, int bx, int by, int nxs, int nys, int f, float rf,
                                              float rfw, int& cr, int& cc, int& FR, int& FC) {
    const int fw = bw * f;
    const int fr = (int)(((float)e + 0.5f) * rfw), fc = e - fr * fw;
    cr = (int)(((float)fr + 0.5f) * rf);
    cc = (int)(((float)fc + 0.5f) * rf);
    FR = by * bw * f + fr;
    FC = bx * bw * f + fc;
    return by * bw + cr < nys && bx * bw + cc < nxs;
}

// The block's epilogue, NT threads, one output value per thread and pass;
// gval(cr, cc) is the block's gradient value at stage pixel (cr, cc) of the
// block (its parts already added in a fixed order).
template <int BW, int NT, bool kFused, typename GVal>
__device__ __forceinline__ void bp_epilogue(const GVal& gval, int bx, int by, int nxs, int nys, float scale,
                                            float* __restrict__ xo, int f, int nx, const float* __restrict__ yprev,
                                            float* __restrict__ z, const float* __restrict__ mu, float mu_scale,
                                            float* __restrict__ g_out) {
    const int ff = kFused ? f : 1;
    const int n = BW * BW * ff * ff;
    const float rf = 1.f / (float)ff, rfw = 1.f / (float)(BW * ff);
    for (int e = threadIdx.x; e < n; e += NT) {
        int cr, cc, FR, FC;
        if (!bp_fine_pixel(e, BW, bx, by, nxs, nys, ff, rf, rfw, cr, cc, FR, FC)) continue;
        const float g = gval(cr, cc);
        const size_t q = (size_t)(by * BW + cr) * nxs + bx * BW + cc;
        if (!kFused) {
            xo[q] = scale * g;
            continue;
        }
        const float yp = yprev[(size_t)FR * nx + FC];
        if (g_out && (by * BW + cr) * f == FR && (bx * BW + cc) * f == FC) g_out[q] = g;
        const float ms = mu ? mu_scale * mu[q] : 0.f;
        z[(size_t)FR * nx + FC] = fmaf(-scale, g, yp - ms);
    }
}

template <int VG, int PX, bool kFused>
__device__ __forceinline__ void bp_finish(const float (*__restrict__ red)[PX * PX][64], int bx, int by, int nxs,
                                          int nys, float scale, float* __restrict__ xo, int f, int nx,
                                          const float* __restrict__ yprev, float* __restrict__ z,
                                          const float* __restrict__ mu, float mu_scale,
                                          float* __restrict__ g_out) {
    auto gval = [&](int cr, int cc) {
        const int lane = ((cr / PX) << 3) | (cc / PX), slot = (cr % PX) * PX + (cc % PX);
        float g = red[0][slot][lane];
        for (int w = 1; w < VG; ++w) g += red[w][slot][lane];
        return g;
    };
    bp_epilogue<8 * PX, 64 * VG, kFused>(gval, bx, by, nxs, nys, scale, xo, f, nx, yprev, z, mu, mu_scale, g_out);
}

// Work-group blk (64 VG threads) of a backprojection; views as in fp_body.
// Fused form, optional extras: mu (a coarse gradient [nys][nxs]) enters the
// step as z = y_prev - U(scale g + mu_scale mu); g_out receives g itself.
// kAllBins: every bin of a view is staged and every ray of a class is a
// candidate of every strip (launched for stages whose blocks reach the source
// circle; see bp_class).
template <int VG, int PX, bool kFused, bool kAllBins = false>
__device__ __forceinline__ void bp_body(int blk, const RayRec* __restrict__ rays, const ViewRec* __restrict__ vrec,
                                        int n_bins, const int32_t* __restrict__ views, int view0, int view_step,
                                        int n_sel, int n_views, const float* __restrict__ y, int nxs, int nys,
                                        int blocks_x, float scale, float* __restrict__ xo, int f, int nx,
                                        const float* __restrict__ yprev, float* __restrict__ z,
                                        const float* __restrict__ mu = nullptr, float mu_scale = 0.f,
                                        float* __restrict__ g_out = nullptr) {
    constexpr int BW = 8 * PX;  // block width in pixels
    // staged rays as three arrays (position, increment, weighted residual):
    // lanes reading entries up to 31 apart fall in different banks
    __shared__ float stage[VG][3 * kStageRays];
    __shared__ float red[VG][PX * PX][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bx = blk % blocks_x, by = blk / blocks_x;
    const int c = bx * BW + PX * (lane & 7), r = by * BW + PX * (lane >> 3);
    const float hx = 0.5f * (float)(nxs - 1), hy = 0.5f * (float)(nys - 1);
    const float cc = (float)c - hx, rc = (float)r - hy;
    // corners of the block grown by the strip ends (one pixel before, one after)
    const float cb0 = (float)(bx * BW - 1) - hx, cb1 = (float)(bx * BW + BW) - hx;
    const float rb0 = (float)(by * BW - 1) - hy, rb1 = (float)(by * BW + BW) - hy;
    const int mid_r = nys >> 1, mid_c = nxs >> 1;
    float acc[PX][PX];
#pragma unroll
    for (int a = 0; a < PX; ++a)
#pragma unroll
        for (int b = 0; b < PX; ++b) acc[a][b] = 0.f;
    float* st = stage[wave];
    // this wavefront's views are i = wave + VG t, t < n_mine; lane u first
    // finds the bin footprint of view t0 + u (block corners grown by the strip
    // ends), then the wavefront walks those views one by one
    const int n_mine = n_sel > wave ? (n_sel - wave + VG - 1) / VG : 0;
    for (int t0 = 0; t0 < n_mine; t0 += 64) {
        int my_v = -1, my_j0 = 0, my_j1 = -1;
        if (t0 + lane < n_mine) {
            const int iu = wave + VG * (t0 + lane);
            const int vu = views ? views[iu] : view0 + iu * view_step;
            if ((unsigned)vu < (unsigned)n_views) {  // invalid view index: no contribution
                my_v = vu;
                if constexpr (kAllBins) {
                    my_j0 = 0;
                    my_j1 = n_bins - 1;
                } else {
                    const ViewRec vq = vrec[vu];
                    const float q0 = proj_bin(vq, cb0, rb0), q1 = proj_bin(vq, cb1, rb0);
                    const float q2 = proj_bin(vq, cb0, rb1), q3 = proj_bin(vq, cb1, rb1);
                    const float jmin = fminf(fminf(q0, q1), fminf(q2, q3));
                    const float jmax = fmaxf(fmaxf(q0, q1), fmaxf(q2, q3));
                    my_j0 = (int)fmaxf(floorf(jmin - kProjEps), 0.f);
                    my_j1 = (int)fminf(ceilf(jmax + kProjEps), (float)(n_bins - 1));
                }
            }
        }
        const int tn = min(64, n_mine - t0);
        for (int u = 0; u < tn; ++u) {
            const int v = __builtin_amdgcn_readlane(my_v, u);
            if (v < 0) continue;
            const int i = wave + VG * (t0 + u);
            const int j0 = __builtin_amdgcn_readlane(my_j0, u), j1 = __builtin_amdgcn_readlane(my_j1, u);
            const ViewRec vr = vrec[v];
            const RayRec* rv = rays + (size_t)v * n_bins;
            const float* yv = y + (size_t)i * n_bins;
            const bool hasx = vr.xlo <= vr.xhi, hasy = vr.ylo <= vr.yhi;
            // The footprint is staged in chunks of kStageRays bins. The first
            // chunk (in practice the only one) is handled outside any loop, so
            // each class's projections are computed only when it is present.
            auto chunk = [&](int base) {
                const int top = min(j1, base + kStageRays - 1);
                for (int q = lane; q <= top - base; q += 64) {
                    const RayRec rr = rv[base + q];
                    st[q] = rr.pos_c;
                    st[q + kStageRays] = rr.dpos;
                    st[q + 2 * kStageRays] = yv[base + q] * rr.len;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (hasx) bp_class<PX, true, kAllBins>(vr, st, base, max(vr.xlo, base), min(vr.xhi, top), cc, rc, c, r, mid_c,
                                             mid_r, acc);
                if (hasy) bp_class<PX, false, kAllBins>(vr, st, base, max(vr.ylo, base), min(vr.yhi, top), cc, rc, c, r, mid_c,
                                              mid_r, acc);
                // the slot is rewritten only after every lane's reads
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            };
            chunk(j0);
            for (int base = j0 + kStageRays; base <= j1; base += kStageRays) chunk(base);
        }
    }
    // every wavefront parks its partial sums; the work-group then finishes the
    // block together, adding the parts in wavefront order
#pragma unroll
    for (int a = 0; a < PX; ++a)
#pragma unroll
        for (int b = 0; b < PX; ++b) red[wave][a * PX + b][lane] = acc[a][b];
    __syncthreads();
    bp_finish<VG, PX, kFused>(red, bx, by, nxs, nys, scale, xo, f, nx, yprev, z, mu, mu_scale, g_out);
}

// ---------------------------------------------------------------------------
// Matched backprojection, scatter form.
//
// A work-group owns a B x B block of stage pixels (B = 16 or 32); each of its
// VG wavefronts takes every VG-th selected view (as bp_body does) and adds
// that view's samples into its own LDS copy of the block, grown by two guard
// cells on every side. For the rays of one dominance class in the block's
// footprint, lane (slot s, offset q) handles line q of the block (column
// C0 + q for x-major rays, row R0 + q for y-major ones); the S = 64 / B slots
// take S equal parts of the class's bin range and walk them in step, one ray
// each per iteration, with k_fp's float operations:
//   p = fma(kf, dpos, pos_c), kf = line - nlines/2 (centred position),
//   cell floor(p) += (1 - fract(p)) y len,  cell floor(p) + 1 += fract(p) y len.
// The additions are plain LDS reads and writes (LDS float atomics serialise
// lane by lane on this GPU). They are race-free because the rays of one
// iteration never share a cell: the plan gives, per stage, the smallest bin
// distance `gap` at which two rays of one class and view lie at least two
// cells apart on every line of the grid, and the slots run in step only when
// their parts are at least that long (else slot 0 takes the whole range). A
// position outside the block is clamped so that both taps fall in the guard
// cells, which are never read (the slots may collide only there, or on lines
// outside the grid, whose cells are never read either).
// Ray records reach the lanes through registers: in a round, lane (row rho, k)
// holds ray k of its slot's part, and iteration t broadcasts lane t of every
// row of 16 lanes (DPP row_newbcast).
// The wavefronts' copies are added in wavefront order at the end, so results
// are bitwise reproducible run to run.
// ---------------------------------------------------------------------------
template <int B>
struct ScatterTile {
    static constexpr int S = 64 / B;  // slots of B lanes
    static constexpr int P = B + 5;   // row pitch (odd)
    static constexpr int CELLS = (B + 4) * P;  // the block with two guard cells on each side
};

// Lane t of each row of 16 lanes, broadcast to its row.
template <int T>
__device__ __forceinline__ float row_bcast(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x150 + T, 0xF, 0xF, true));
}

// Iteration T of a round: the slot rays held by lane T of each row add their
// sample on this lane's line. A: accumulator stride of the position axis (P
// for x-major rays, whose positions are rows; 1 for y-major ones); cq:
// accumulator index of position 0 on this lane's line.
template <int A, int T>
__device__ __forceinline__ void bps_sample(float pc, float dp, float yl, float kf, float lo, float hi, int cq,
                                           float* __restrict__ acc) {
    const float p = fmaf(kf, row_bcast<T>(dp), row_bcast<T>(pc));
    const float q = __builtin_amdgcn_fmed3f(p, lo, hi);
    const float w = __builtin_amdgcn_fractf(q);
    const int fl = (int)floorf(q);
    const int e = (A == 1 ? fl : __mul24(fl, A)) + cq;
    const float yy = row_bcast<T>(yl);
    const float wy = w * yy;
    const float c0 = acc[e], c1 = acc[e + A];
    acc[e] = c0 + (yy - wy);
    acc[e + A] = c1 + wy;
}

// Iterations T0 .. of a round, in groups of four without branches (so one
// iteration's arithmetic can overlap the previous one's LDS round trip),
// until tn iterations are done; lanes past the round's rays hold a position
// far outside, whose taps fall in the guard cells.
template <int A, int T0 = 0>
__device__ __forceinline__ void bps_round(int tn, float pc, float dp, float yl, float kf, float lo, float hi,
                                          int cq, float* __restrict__ acc) {
    if constexpr (T0 < 16) {
        bps_sample<A, T0>(pc, dp, yl, kf, lo, hi, cq, acc);
        bps_sample<A, T0 + 1>(pc, dp, yl, kf, lo, hi, cq, acc);
        bps_sample<A, T0 + 2>(pc, dp, yl, kf, lo, hi, cq, acc);
        bps_sample<A, T0 + 3>(pc, dp, yl, kf, lo, hi, cq, acc);
        if (T0 + 4 >= tn) return;
        bps_round<A, T0 + 4>(tn, pc, dp, yl, kf, lo, hi, cq, acc);
    }
}

// A round's ray records for this lane: ray first + r0 + k of its slot's part,
// if that lies in the part (L rays) and in the range (up to b); else a
// position far outside with no weight. The loads take no branch (a lane
// without a ray reads bin a of the range), so waiting for one round's records
// can leave the next round's in flight.
__device__ __forceinline__ void bps_fetch(const RayRec* __restrict__ rv, const float* __restrict__ yv, int a,
                                          int first, int r0, int k, int L, int b, bool mine, float& pc, float& dp,
                                          float& len, float& res) {
    const int j = first + r0 + k;
    const bool ok = mine && r0 + k < L && j <= b;
    const int jj = ok ? j : a;
    const RayRec q = rv[jj];
    const float yq = yv[jj];
    pc = ok ? q.pos_c : -1e30f;
    dp = ok ? q.dpos : 0.f;
    len = ok ? q.len : 0.f;
    res = ok ? yq : 0.f;
}

// The rays a .. b of one class of one view: S parts of L rays walked in step
// (one part, slot 0's, when the parts would be shorter than gap), in rounds
// of 16, each round's records loaded during the previous round.
template <int B, int A>
__device__ __forceinline__ void bps_class(const RayRec* __restrict__ rv, const float* __restrict__ yv, int a, int b,
                                          int gap, int slot, int k, float kf, float lo, float hi, int cq,
                                          float* __restrict__ acc) {
    constexpr int S = ScatterTile<B>::S;
    const int n = b - a + 1;
    if (n <= 0) return;
    int L = (n + S - 1) / S;
    const bool parts = L >= gap;
    if (!parts) L = n;
    const int first = a + (parts ? slot * L : 0);
    const bool mine = parts || slot == 0;
    float pc0, dp0, len0, res0, pc1, dp1, len1, res1;
    bps_fetch(rv, yv, a, first, 0, k, L, b, mine, pc0, dp0, len0, res0);
    for (int r0 = 0; r0 < L; r0 += 32) {
        bps_fetch(rv, yv, a, first, r0 + 16, k, L, b, mine, pc1, dp1, len1, res1);
        bps_round<A>(min(16, L - r0), pc0, dp0, res0 * len0, kf, lo, hi, cq, acc);
        if (r0 + 16 >= L) break;
        bps_fetch(rv, yv, a, first, r0 + 32, k, L, b, mine, pc0, dp0, len0, res0);
        bps_round<A>(min(16, L - r0 - 16), pc1, dp1, res1 * len1, kf, lo, hi, cq, acc);
    }
}

// Work-group blk (64 VG threads) of a scatter-form backprojection; arguments
// and results as bp_body's (blocks_x counts B-wide blocks), plus the stage's
// slot gap (Stage::scatter_gap). Stages whose blocks reach the source circle
// take bp_body's every-bin form instead.
template <int B, int VG, bool kFused>
__device__ __forceinline__ void bps_body(int blk, const RayRec* __restrict__ rays, const ViewRec* __restrict__ vrec,
                                         int n_bins, const int32_t* __restrict__ views, int view0, int view_step,
                                         int n_sel, int n_views, const float* __restrict__ y, int nxs, int nys,
                                         int blocks_x, int gap, float scale, float* __restrict__ xo, int f,
                                         int nx, const float* __restrict__ yprev, float* __restrict__ z,
                                         const float* __restrict__ mu = nullptr, float mu_scale = 0.f,
                                         float* __restrict__ g_out = nullptr) {
    using Tl = ScatterTile<B>;
    constexpr int P = Tl::P;
    __shared__ float accs[VG * Tl::CELLS];
    // (the wavefront index is uniform: read it as such, so loops over its views
    // and rounds stay scalar)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int bx = blk % blocks_x, by = blk / blocks_x;
    const int C0 = bx * B, R0 = by * B;
    float* const acc = accs + wave * Tl::CELLS;
    // the wavefront's own copy; its LDS accesses complete in order, so no barrier
    for (int e = lane; e < Tl::CELLS; e += 64) acc[e] = 0.f;
    const int q = lane % B;
    const int mid_r = nys >> 1, mid_c = nxs >> 1;
    // x-major rays: lines are columns C0 + q, positions are rows
    const float kfx = (float)(C0 + q - mid_c);
    const float lox = (float)(R0 - mid_r - 2), hix = (float)(R0 - mid_r + B);
    const int cqx = (mid_r - R0 + 2) * P + q + 2;
    // y-major rays: lines are rows R0 + q, positions are columns
    const float kfy = (float)(R0 + q - mid_r);
    const float loy = (float)(C0 - mid_c - 2), hiy = (float)(C0 - mid_c + B);
    const int cqy = (q + 2) * P + mid_c - C0 + 2;
    // this lane's slot, and the ray of its slot's part it holds in a round
    const int slot = lane / B, k = lane & 15;
    // corners of the block grown by one pixel on each side (a ray reaches a
    // pixel when its position lies within one pixel of it)
    const float hx = 0.5f * (float)(nxs - 1), hy = 0.5f * (float)(nys - 1);
    const float cb0 = (float)(C0 - 1) - hx, cb1 = (float)(C0 + B) - hx;
    const float rb0 = (float)(R0 - 1) - hy, rb1 = (float)(R0 + B) - hy;
    const int n_mine = n_sel > wave ? (n_sel - wave + VG - 1) / VG : 0;
    for (int t0 = 0; t0 < n_mine; t0 += 64) {
        // lane u: view t0 + u of this wavefront, its selection row and the
        // footprint's bins of each class
        int my_v = -1, my_i = 0, xa = 0, xb = -1, ya = 0, yb = -1;
        if (t0 + lane < n_mine) {
            const int iu = wave + VG * (t0 + lane);
            const int vu = views ? views[iu] : view0 + iu * view_step;
            if ((unsigned)vu < (unsigned)n_views) {  // invalid view index: no contribution
                const ViewRec vq = vrec[vu];
                const float q0 = proj_bin(vq, cb0, rb0), q1 = proj_bin(vq, cb1, rb0);
                const float q2 = proj_bin(vq, cb0, rb1), q3 = proj_bin(vq, cb1, rb1);
                const float jmin = fminf(fminf(q0, q1), fminf(q2, q3));
                const float jmax = fmaxf(fmaxf(q0, q1), fmaxf(q2, q3));
                const int j0 = (int)fmaxf(floorf(jmin - kProjEps), 0.f);
                const int j1 = (int)fminf(ceilf(jmax + kProjEps), (float)(n_bins - 1));
                my_v = vu;
                my_i = iu;
                xa = max(vq.xlo, j0);
                xb = min(vq.xhi, j1);
                ya = max(vq.ylo, j0);
                yb = min(vq.yhi, j1);
            }
        }
        const int tn = min(64, n_mine - t0);
        for (int u = 0; u < tn; ++u) {
            const int v = __builtin_amdgcn_readlane(my_v, u);
            if (v < 0) continue;
            const int i = __builtin_amdgcn_readlane(my_i, u);
            const RayRec* rv = rays + (size_t)v * n_bins;
            const float* yv = y + (size_t)i * n_bins;
            bps_class<B, P>(rv, yv, __builtin_amdgcn_readlane(xa, u), __builtin_amdgcn_readlane(xb, u), gap, slot, k,
                            kfx, lox, hix, cqx, acc);
            bps_class<B, 1>(rv, yv, __builtin_amdgcn_readlane(ya, u), __builtin_amdgcn_readlane(yb, u), gap, slot, k,
                            kfy, loy, hiy, cqy, acc);
        }
    }
    __syncthreads();
    auto gval = [&](int cr, int cc) {
        const int e = (cr + 2) * P + cc + 2;
        float g = accs[e];
        for (int w = 1; w < VG; ++w) g += accs[w * Tl::CELLS + e];
        return g;
    };
    bp_epilogue<B, 64 * VG, kFused>(gval, bx, by, nxs, nys, scale, xo, f, nx, yprev, z, mu, mu_scale, g_out);
}

// ---------------------------------------------------------------------------
// TV-prox (Chambolle's dual projection), n_iter <= H-1 steps per launch with
// the tile and a halo of H cells held in LDS. Cells within H of the tile edge
// see incomplete neighbourhoods; the error travels one cell per step, so the
// T x T output tile stays exact.
// The dual field p is zero outside the image and stays zero on the last row
// (p1) and last column (p2), because the masked gradient vanishes there; so
// div p = p1[r] - p1[r-1] + p2[c] - p2[c-1] needs no boundary tests, and the
// Neumann conditions live only in the two gradient masks.
//   mode 0: x_out = z - lambda div p
//   mode 1: x = (1-alpha) z + alpha (z - lambda div p); y_out = x + a_t (x - x_prev);
//           x_out = x; hist (optional) = x
//   p_in/p_out: optional global dual field [2][ny][nx] for multi-launch runs
//   (p_out set: the launch stores p for its tile instead of producing x).
//   stamp (optional): raised to the device clock (wall_clock64) at which each
//   work-group finishes, so that it ends as the launch's last such time.
// ---------------------------------------------------------------------------
// Tile (bx, by) of the TV-prox, NT threads. Each thread owns vertical pairs
// of cells (rows 2i, 2i+1 of one column of the haloed tile): their dual
// values p1, p2 and z / lambda stay in registers, and LDS only carries what a
// neighbour reads (the lower cell's p1, both p2, both u), so a step moves 11
// LDS words per pair instead of 26. Arithmetic and its order are those of the
// plain per-cell form.
template <int T, int H, int NT>
__device__ __forceinline__ void tv_body(int bx, int by, const float* __restrict__ z, int nx, int ny, float lam,
                                        float tau, int n_iter, const float* __restrict__ p_in,
                                        float* __restrict__ p_out, int mode, float alpha, float a_t,
                                        const float* __restrict__ x_prev, float* __restrict__ x_out,
                                        float* __restrict__ y_out, float* __restrict__ hist, int pf, float pinv,
                                        float* __restrict__ plx, int ppx, float* __restrict__ ply, int ppy,
                                        int pnxs, int pnys, unsigned long long* __restrict__ stamp = nullptr) {
    constexpr int S = T + 2 * H;
    static_assert(S % 2 == 0, "pairs of rows need an even tile side");
    constexpr int NPAIR = (S / 2) * S;
    constexpr int NP = (NPAIR + NT - 1) / NT;
    __shared__ float sp1[S * S], sp2[S * S], su[S * S];
    const int R0 = by * T - H, C0 = bx * T - H;
    const size_t plane = (size_t)nx * ny;
    const float il = 1.f / lam;
    // per pair k: column lc, upper row 2 pr; LDS index of the upper cell and
    // of its clamped neighbours (a missing neighbour reads the cell itself)
    int e0[NP], eup[NP], eleft[NP], edown[NP], eright[NP];
    bool live[NP], out0[NP], out1[NP];
    float p1a[NP], p1b[NP], p2a[NP], p2b[NP], za[NP], zb[NP], zla[NP], zlb[NP];
    float m1a[NP], m1b[NP], m2a[NP], m2b[NP], xpa[NP], xpb[NP];
    size_t ga[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int q = threadIdx.x + k * NT;
        live[k] = q < NPAIR;
        const int qq = live[k] ? q : NPAIR - 1;
        const int pr = qq / S, lc = qq - pr * S;
        const int lr = 2 * pr;
        const int e = lr * S + lc;
        e0[k] = e;
        // (the tile's first row reads its pair's lower cell: any finite value
        // there stays outside what the output tile depends on)
        eup[k] = lr > 0 ? e - S : e + S;
        eleft[k] = lc > 0 ? e - 1 : e;
        edown[k] = lr + 2 < S ? e + 2 * S : e + S;
        eright[k] = lc < S - 1 ? e + 1 : e;
        const int gr = R0 + lr, gc = C0 + lc;
        const bool ina = gr >= 0 && gr < ny && gc >= 0 && gc < nx;
        const bool inb = gr + 1 >= 0 && gr + 1 < ny && gc >= 0 && gc < nx;
        m1a[k] = (ina && gr < ny - 1) ? 1.f : 0.f;
        m1b[k] = (inb && gr + 1 < ny - 1) ? 1.f : 0.f;
        m2a[k] = (ina && gc < nx - 1) ? 1.f : 0.f;
        m2b[k] = (inb && gc < nx - 1) ? 1.f : 0.f;
        const size_t gi = (size_t)gr * nx + gc;
        ga[k] = gi;
        za[k] = ina ? z[gi] : 0.f;
        zb[k] = inb ? z[gi + nx] : 0.f;
        p1a[k] = (ina && p_in) ? p_in[gi] : 0.f;
        p1b[k] = (inb && p_in) ? p_in[gi + nx] : 0.f;
        p2a[k] = (ina && p_in) ? p_in[plane + gi] : 0.f;
        p2b[k] = (inb && p_in) ? p_in[plane + gi + nx] : 0.f;
        zla[k] = za[k] * il;
        zlb[k] = zb[k] * il;
        // output cells of the tile
        const bool col_out = lc >= H && lc < H + T && gc < nx;
        out0[k] = live[k] && col_out && lr >= H && lr < H + T && gr < ny;
        out1[k] = live[k] && col_out && lr + 1 >= H && lr + 1 < H + T && gr + 1 < ny;
        if (live[k]) {
            sp1[e + S] = p1b[k];
            sp2[e] = p2a[k];
            sp2[e + S] = p2b[k];
        }
    }
    __syncthreads();
    // x_prev of the output cells, used only at the end: fetched now, after the
    // wait for the loads above, so that its latency overlaps the dual steps
    // (every lane loads, from cell 0 where its cell is no output cell, whose
    // value the epilogue never uses; so the loads take no branch and nothing
    // waits for them before the epilogue)
#pragma unroll
    for (int k = 0; k < NP; ++k) xpa[k] = xpb[k] = 0.f;
    __builtin_amdgcn_s_waitcnt(0);  // the loads above are complete on every path
    if (mode == 1 && !p_out) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            xpa[k] = x_prev[out0[k] ? ga[k] : 0];
            xpb[k] = x_prev[out1[k] ? ga[k] + nx : 0];
        }
    }
    for (int it = 0; it < n_iter; ++it) {
        float ua[NP], ub[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e = e0[k];
            // u = div p - z / lambda on both cells
            ua[k] = (p1a[k] - sp1[eup[k]]) + (p2a[k] - sp2[eleft[k]]) - zla[k];
            ub[k] = (p1b[k] - p1a[k]) + (p2b[k] - sp2[eleft[k] + S]) - zlb[k];
            if (live[k]) {
                su[e] = ua[k];
                su[e + S] = ub[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e = e0[k];
            const float q1a = m1a[k] * (ub[k] - ua[k]);
            const float q1b = m1b[k] * (su[edown[k]] - ub[k]);
            const float q2a = m2a[k] * (su[eright[k]] - ua[k]);
            const float q2b = m2b[k] * (su[eright[k] + S] - ub[k]);
            const float ia = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(fmaf(q1a, q1a, q2a * q2a)), 1.f));
            const float ib = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(fmaf(q1b, q1b, q2b * q2b)), 1.f));
            p1a[k] = fmaf(tau, q1a, p1a[k]) * ia;
            p2a[k] = fmaf(tau, q2a, p2a[k]) * ia;
            p1b[k] = fmaf(tau, q1b, p1b[k]) * ib;
            p2b[k] = fmaf(tau, q2b, p2b[k]) * ib;
            if (live[k]) {
                sp1[e + S] = p1b[k];
                sp2[e] = p2a[k];
                sp2[e + S] = p2b[k];
            }
        }
        __syncthreads();
    }
    float* const yst = su;  // free after the last step: holds y_t for the pooling epilogue
    float yv[NP][2];        // y_t of the pair's two cells, for pooling straight from registers
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e = e0[k];
        const size_t gi = ga[k];
        yv[k][0] = yv[k][1] = 0.f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!(h == 0 ? out0[k] : out1[k])) continue;
            const size_t g = h == 0 ? gi : gi + nx;
            const float p1 = h == 0 ? p1a[k] : p1b[k], p2 = h == 0 ? p2a[k] : p2b[k];
            if (p_out) {
                p_out[g] = p1;
                p_out[plane + g] = p2;
                continue;
            }
            const float p1u = h == 0 ? sp1[eup[k]] : p1a[k];
            const float d = (p1 - p1u) + (p2 - sp2[eleft[k] + h * S]);
            const float zz = h == 0 ? za[k] : zb[k];
            const float den = fmaf(-lam, d, zz);
            if (mode == 0) {
                x_out[g] = den;
            } else {
                const float xr = (1.f - alpha) * zz + alpha * den;
                const float yn = fmaf(a_t, xr - (h == 0 ? xpa[k] : xpb[k]), xr);
                x_out[g] = xr;
                y_out[g] = yn;
                if (hist) hist[g] = xr;
                yst[e + h * S] = yn;
                yv[k][h] = yn;
            }
        }
    }
    if (pf == 1 || (pf == 2 && H % 2 == 0)) {
        // pooling straight from registers, with no barrier: a pair is two rows of
        // one column, and with an even halo the tile's pairs start on even rows and
        // columns, so an f = 2 block is this pair and the next lane's (same sums,
        // in the same order, as k_prepare)
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int q = threadIdx.x + k * NT;
            const int pr = (live[k] ? q : NPAIR - 1) / S;
            const int lc = (live[k] ? q : NPAIR - 1) - pr * S;
            const int gr = R0 + 2 * pr, gc = C0 + lc;
            if (pf == 1) {
                if (H % 2 == 0 && out0[k] && out1[k]) {
                    // the pair's rows are neighbours in the column image, 8-byte aligned
                    // (even first row, even padding, line pitch a multiple of 4)
                    *reinterpret_cast<float2*>(plx + (size_t)gc * ppx + kPad + gr) = make_float2(yv[k][0], yv[k][1]);
                    ply[(size_t)gr * ppy + kPad + gc] = yv[k][0];
                    ply[(size_t)(gr + 1) * ppy + kPad + gc] = yv[k][1];
                } else {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (!(h == 0 ? out0[k] : out1[k])) continue;
                        plx[(size_t)gc * ppx + kPad + gr + h] = yv[k][h];
                        ply[(size_t)(gr + h) * ppy + kPad + gc] = yv[k][h];
                    }
                }
            } else {
                const float ra = __shfl_xor(yv[k][0], 1), rb = __shfl_xor(yv[k][1], 1);
                if (out0[k] && out1[k] && (lc & 1) == 0) {
                    float sum = 0.f;
                    sum += yv[k][0];
                    sum += ra;
                    sum += yv[k][1];
                    sum += rb;
                    sum *= pinv;
                    const int R = gr >> 1, C = gc >> 1;
                    plx[(size_t)C * ppx + kPad + R] = sum;
                    ply[(size_t)R * ppy + kPad + C] = sum;
                }
            }
        }
    } else if (pf > 0) {
        // pooling of y_t for the next iteration's stage (pf x pf blocks inside
        // this tile, pf >= 2 here), with the same arithmetic as k_prepare: one
        // thread per block reads its values from LDS together, adds them in
        // row order and stores the mean into both line images
        __syncthreads();
        const int tc = T / pf;
        const int Rc0 = (R0 + H) / pf, Cc0 = (C0 + H) / pf;
        for (int e = threadIdx.x; e < tc * tc; e += NT) {
            const int cr = e / tc, cc = e - cr * tc;
            const int R = Rc0 + cr, C = Cc0 + cc;
            if (R >= pnys || C >= pnxs) continue;
            const float* const blk = yst + (H + cr * pf) * S + H + cc * pf;
            float sum;
            if (pf == 2) sum = pool_block<2>(blk, S);
            else if (pf == 3) sum = pool_block<3>(blk, S);
            else if (pf == 4) sum = pool_block<4>(blk, S);
            else {
                sum = 0.f;
                for (int a = 0; a < pf; ++a)
                    for (int b = 0; b < pf; ++b) sum += blk[a * S + b];
            }
            sum *= pinv;
            plx[(size_t)C * ppx + kPad + R] = sum;
            ply[(size_t)R * ppy + kPad + C] = sum;
        }
    }
    if (stamp) {
        // the device's constant-rate clock when this work-group has issued all its
        // stores; the latest over the launch marks the end of the step
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(stamp, (unsigned long long)wall_clock64());
    }
}

}  // namespace dev
}  // namespace fbpnp
