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
#include <hip/hip_ext.h>
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

// Wavefront-wide minimum and maximum (every lane gets the result).
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

template <bool kResid, int SEG>
__global__ __launch_bounds__(256) void k_fp(const RayRec* __restrict__ rays, int n_bins, int bins_padded,
                                            const int32_t* __restrict__ views, int n_sel, int n_views,
                                            const float* __restrict__ lines, int ly_off, int line_bytes,
                                            int pitch_x, int pitch_y, int nxs, int nys,
                                            const float* __restrict__ b, float* __restrict__ y) {
    constexpr int R = 64 / SEG;  // rays per wavefront; SEG lanes share one ray
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int waves_per_view = bins_padded / R;
    const int i = wave / waves_per_view;
    const int j = (wave - i * waves_per_view) * R + lane % R;
    const int seg = lane / R;
    const bool active = i < n_sel && j < n_bins;
    // both line images of the stage as one buffer: 32-bit offsets, and a load
    // outside it would return zero instead of faulting
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(lines), (short)0, line_bytes, kBufWord3);
    int v = 0;
    if (active) v = views ? views[i] : i;
    const bool valid = active && (unsigned)v < (unsigned)n_views;  // invalid view index: a zero row
    RayRec r{0.f, 0.f, 0.f, 0u};
    if (valid) r = rays[(size_t)v * n_bins + j];
    const int lo = (int)(r.bits & 0xFFFFu), n = (int)((r.bits >> 16) & 0x7FFFu);
    const bool ymaj = (r.bits >> 31) != 0u;
    if (n == 0) {  // no samples (or no ray): every position clamps into the padding
        r.pos_c = -1e30f;
        r.dpos = 0.f;
    }
    // All lanes march the same lines in lockstep (the union of the wavefront's
    // sample ranges, split into SEG parts), so one load instruction reads
    // neighbouring positions of one line. Outside its own range a ray's
    // position is clamped into the zero padding and adds nothing.
    const int L0 = wave_min(n > 0 ? lo : 1 << 30), L1 = wave_max(n > 0 ? lo + n : -(1 << 30));
    float acc = 0.f;
    if (L1 > L0) {
        const int la = L0 + ((L1 - L0) * seg) / SEG, lb = L0 + ((L1 - L0) * (seg + 1)) / SEG;
        const int pitch = ymaj ? pitch_y : pitch_x;
        const int npos = ymaj ? nxs : nys;
        const int mid = npos >> 1, lmid = (ymaj ? nys : nxs) >> 1;
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
            const auto t = __builtin_amdgcn_raw_buffer_load_b64(rsrc, off + i0 * 4, 0, 0);
            const float a = __uint_as_float(t[0]), c = __uint_as_float(t[1]);
            acc += fmaf(w, c - a, a);
            kf += 1.f;
            off += step;
        }
    }
    // fixed-order sum of the SEG partial sums of each ray
#pragma unroll
    for (int o = R; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
    if (active && seg == 0) {
        float val = 0.f;
        if (valid) {
            val = acc * r.len;
            if (kResid) val -= b[(size_t)v * n_bins + j];
        }
        y[(size_t)i * n_bins + j] = val;
    }
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
    const float e = p - qf;
#pragma unroll
    for (int t = 0; t < PX; ++t) {
        const float wt = fmaxf(1.f - fabsf(e - (float)t), 0.f);
        s[t] = fmaf(wt, yy, s[t]);
    }
}

// Candidate rays jl..jh (one dominance class, staged from bin base) for a
// strip on a line whose offset from the middle line is kf, first centred
// position qm.
template <int PX>
__device__ __forceinline__ void gather_strip(const float4* __restrict__ st, int base, int jl, int jh, float kf,
                                             int qm, float (&s)[PX]) {
    const float qf = (float)qm;
    for (int j = jl; j <= jh; ++j) {
        const float4 e = st[j - base];
        strip_add<PX>(fmaf(kf, e.y, e.x), qf, e.z, s);
    }
}

// All strips of one dominance class for one staged view. The candidate bins
// of a strip come from j(c, r) at its two ends (the numerator and the
// denominator of j are linear in c and r); lo..hi is the class range within
// the staged chunk.
template <int PX, bool kXMajor>
__device__ __forceinline__ void bp_class(const ViewRec& vr, const float4* __restrict__ st, int base, int lo,
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
        int jl, jh;
        cand_range(fmaf(nt, __builtin_amdgcn_rcpf(dt), vr.j0), fmaf(nt + dn, __builtin_amdgcn_rcpf(dt + dd), vr.j0),
                   lo, hi, jl, jh);
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

template <int VG, int PX, bool kFused>
__global__ __launch_bounds__(64 * VG) void k_bp(const RayRec* __restrict__ rays, const ViewRec* __restrict__ vrec,
                                                int n_bins, const int32_t* __restrict__ views, int n_sel,
                                                int n_views, const float* __restrict__ y, int nxs, int nys,
                                                int blocks_x, float scale, float* __restrict__ xo, int f, int nx,
                                                const float* __restrict__ yprev, float* __restrict__ z) {
    constexpr int BW = 8 * PX;  // block width in pixels
    __shared__ float4 stage[VG][kStageRays];
    __shared__ float red[VG > 1 ? VG - 1 : 1][PX * PX][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bx = blockIdx.x % blocks_x, by = blockIdx.x / blocks_x;
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
    float4* st = stage[wave];
    // this wavefront's views are i = wave + VG t, t < n_mine; lane u first
    // finds the bin footprint of view t0 + u (block corners grown by the strip
    // ends), then the wavefront walks those views one by one
    const int n_mine = n_sel > wave ? (n_sel - wave + VG - 1) / VG : 0;
    for (int t0 = 0; t0 < n_mine; t0 += 64) {
        int my_v = -1, my_j0 = 0, my_j1 = -1;
        if (t0 + lane < n_mine) {
            const int iu = wave + VG * (t0 + lane);
            const int vu = views ? views[iu] : iu;
            if ((unsigned)vu < (unsigned)n_views) {  // invalid view index: no contribution
                const ViewRec vq = vrec[vu];
                const float q0 = proj_bin(vq, cb0, rb0), q1 = proj_bin(vq, cb1, rb0);
                const float q2 = proj_bin(vq, cb0, rb1), q3 = proj_bin(vq, cb1, rb1);
                const float jmin = fminf(fminf(q0, q1), fminf(q2, q3));
                const float jmax = fmaxf(fmaxf(q0, q1), fmaxf(q2, q3));
                my_v = vu;
                my_j0 = (int)fmaxf(floorf(jmin - kProjEps), 0.f);
                my_j1 = (int)fminf(ceilf(jmax + kProjEps), (float)(n_bins - 1));
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
                    st[q] = make_float4(rr.pos_c, rr.dpos, yv[base + q] * rr.len, 0.f);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (hasx) bp_class<PX, true>(vr, st, base, max(vr.xlo, base), min(vr.xhi, top), cc, rc, c, r, mid_c,
                                             mid_r, acc);
                if (hasy) bp_class<PX, false>(vr, st, base, max(vr.ylo, base), min(vr.yhi, top), cc, rc, c, r, mid_c,
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
    if (VG > 1) {
        if (wave > 0) {
#pragma unroll
            for (int a = 0; a < PX; ++a)
#pragma unroll
                for (int b = 0; b < PX; ++b) red[wave - 1][a * PX + b][lane] = acc[a][b];
        }
        __syncthreads();
        if (wave > 0) return;
        for (int w = 0; w < VG - 1; ++w)
#pragma unroll
            for (int a = 0; a < PX; ++a)
#pragma unroll
                for (int b = 0; b < PX; ++b) acc[a][b] += red[w][a * PX + b][lane];
    }
#pragma unroll
    for (int dr = 0; dr < PX; ++dr)
#pragma unroll
        for (int dc = 0; dc < PX; ++dc) {
            const int R = r + dr, C = c + dc;
            if (R >= nys || C >= nxs) continue;
            if (!kFused) {
                xo[(size_t)R * nxs + C] = scale * acc[dr][dc];
            } else {
                // z = y_prev - (eta sigma / f^2) g on the f x f block of (R, C)
                const float sg = scale * acc[dr][dc];
                for (int a = 0; a < f; ++a) {
                    const size_t row = (size_t)(f * R + a) * nx + (size_t)f * C;
                    for (int bb = 0; bb < f; ++bb) z[row + bb] = yprev[row + bb] - sg;
                }
            }
        }
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
// ---------------------------------------------------------------------------
template <int T, int H, int NT>
__global__ __launch_bounds__(NT) void k_tv(const float* __restrict__ z, int nx, int ny, float lam, float tau,
                                           int n_iter, const float* __restrict__ p_in, float* __restrict__ p_out,
                                           int mode, float alpha, float a_t, const float* __restrict__ x_prev,
                                           float* __restrict__ x_out, float* __restrict__ y_out,
                                           float* __restrict__ hist, int pf, float pinv, float* __restrict__ plx,
                                           int ppx, float* __restrict__ ply, int ppy, int pnxs, int pnys) {
    constexpr int S = T + 2 * H;
    constexpr int NC = (S * S + NT - 1) / NT;
    __shared__ float sz[S * S], sp1[S * S], sp2[S * S], su[S * S];
    const int R0 = blockIdx.y * T - H, C0 = blockIdx.x * T - H;
    const size_t plane = (size_t)nx * ny;
    // per-thread cells, their clamped neighbour indices and gradient masks
    int ce[NC], cup[NC], cleft[NC], cdown[NC], cright[NC];
    float m1[NC], m2[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int e = threadIdx.x + k * NT;
        const int ee = e < S * S ? e : S * S - 1;
        const int lr = ee / S, lc = ee - lr * S;
        const int gr = R0 + lr, gc = C0 + lc;
        const bool in = gr >= 0 && gr < ny && gc >= 0 && gc < nx;
        ce[k] = e;
        cup[k] = lr > 0 ? ee - S : ee;
        cleft[k] = lc > 0 ? ee - 1 : ee;
        cdown[k] = lr < S - 1 ? ee + S : ee;
        cright[k] = lc < S - 1 ? ee + 1 : ee;
        m1[k] = (in && gr < ny - 1) ? 1.f : 0.f;
        m2[k] = (in && gc < nx - 1) ? 1.f : 0.f;
        if (e < S * S) {
            const size_t gi = (size_t)gr * nx + gc;
            sz[e] = in ? z[gi] : 0.f;
            sp1[e] = (in && p_in) ? p_in[gi] : 0.f;
            sp2[e] = (in && p_in) ? p_in[plane + gi] : 0.f;
        }
    }
    __syncthreads();
    const float il = 1.f / lam;
    for (int it = 0; it < n_iter; ++it) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int e = ce[k];
            if (e < S * S) su[e] = (sp1[e] - sp1[cup[k]]) + (sp2[e] - sp2[cleft[k]]) - sz[e] * il;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int e = ce[k];
            if (e < S * S) {
                const float u = su[e];
                const float q1 = m1[k] * (su[cdown[k]] - u);
                const float q2 = m2[k] * (su[cright[k]] - u);
                const float inv = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(fmaf(q1, q1, q2 * q2)), 1.f));
                sp1[e] = fmaf(tau, q1, sp1[e]) * inv;
                sp2[e] = fmaf(tau, q2, sp2[e]) * inv;
            }
        }
        __syncthreads();
    }
    float* const yst = su;  // free after the last step: holds y_t for the pooling epilogue
    for (int e = threadIdx.x; e < T * T; e += NT) {
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
        const float d = (sp1[l] - sp1[l - S]) + (sp2[l] - sp2[l - 1]);
        const float zz = sz[l];
        const float den = fmaf(-lam, d, zz);
        if (mode == 0) {
            x_out[gi] = den;
        } else {
            const float xr = (1.f - alpha) * zz + alpha * den;
            const float yn = fmaf(a_t, xr - x_prev[gi], xr);
            x_out[gi] = xr;
            y_out[gi] = yn;
            if (hist) hist[gi] = xr;
            yst[l] = yn;
        }
    }
    if (pf > 0) {
        // pooling of y_t for the next iteration's stage (pf x pf blocks inside
        // this tile), written into that stage's two line images with the same
        // arithmetic as k_prepare
        __syncthreads();
        const int tc = T / pf;
        const int Rc0 = (R0 + H) / pf, Cc0 = (C0 + H) / pf;
        for (int pass = 0; pass < 2; ++pass) {
            for (int e = threadIdx.x; e < tc * tc; e += NT) {
                // consecutive threads walk the contiguous axis of the image written
                const int u = e % tc, w = e / tc;
                const int cr = pass == 0 ? u : w, cc = pass == 0 ? w : u;
                const int R = Rc0 + cr, C = Cc0 + cc;
                if (R >= pnys || C >= pnxs) continue;
                float sum = 0.f;
                if (pf == 1) {
                    sum = yst[(H + cr) * S + H + cc];
                } else {
                    for (int a = 0; a < pf; ++a)
                        for (int b = 0; b < pf; ++b) sum += yst[(H + cr * pf + a) * S + H + cc * pf + b];
                    sum *= pinv;
                }
                if (pass == 0) plx[(size_t)C * ppx + kPad + R] = sum;
                else ply[(size_t)R * ppy + kPad + C] = sum;
            }
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

fb_status launch_fp(const fb_plan* p, int stage, bool resid, const int32_t* views, int n_sel, const float* b,
                    float* y, hipStream_t s) {
    const Stage& st = p->stages[stage];
    StageLines L = stage_lines(p, stage);
    const int nb = p->g.n_bins;
    // split rays over 2 or 4 lanes when one lane per ray gives few wavefronts
    const int waves1 = n_sel * cdiv(nb, 64);
    const int seg = waves1 < 4096 ? 4 : (waves1 < 8192 ? 2 : 1);
    const int rays_per_wave = 64 / seg;
    const int bp = cdiv(nb, rays_per_wave) * rays_per_wave;
    const int blocks = cdiv(n_sel * (bp / rays_per_wave), 4);
#define FB_FP(RES, SG)                                                                                        \
    FB_LAUNCH((k_fp<RES, SG>), dim3(blocks), dim3(256), s, st.rays, nb, bp, views, n_sel, p->g.n_views, L.lx,   \
              L.ly_off, L.bytes, st.pitch_x, st.pitch_y, st.nxs, st.nys, b, y)
    if (resid) {
        if (seg == 4) FB_FP(true, 4);
        else if (seg == 2) FB_FP(true, 2);
        else FB_FP(true, 1);
    } else {
        if (seg == 4) FB_FP(false, 4);
        else if (seg == 2) FB_FP(false, 2);
        else FB_FP(false, 1);
    }
#undef FB_FP
    return check_launch("fanbeam_fp");
}

template <bool kFused>
static fb_status launch_bp_t(const fb_plan* p, int stage, const float* y, const int32_t* views, int n_sel,
                             float scale, float* xo, const float* yprev, float* z, hipStream_t s) {
    const Stage& st = p->stages[stage];
    // pixels per lane: 4 x 4 on very large grids, 2 x 2 on large ones, 1
    // otherwise (more wavefronts); views split over up to 16 wavefronts per
    // block (4 with 4 x 4 pixels, for registers) until ~8192 wavefronts
    const long npx = (long)st.nxs * st.nys;
    const int px = npx >= 1024L * 1024 ? 4 : (npx >= 256L * 256 ? 2 : 1);
    const int vg_max = px == 4 ? 4 : 16;
    const int bw = 8 * px;
    const int bxs = cdiv(st.nxs, bw), bys = cdiv(st.nys, bw), nblk = bxs * bys;
    int vg = 1;
    while (vg < vg_max && nblk * vg < 8192 && vg * 2 <= n_sel) vg *= 2;
    const int nb = p->g.n_bins, f = st.f, nx = p->g.nx;
#define FB_BP(VG, PX)                                                                                         \
    FB_LAUNCH((k_bp<VG, PX, kFused>), dim3(nblk), dim3(64 * VG), s, st.rays, st.vrec, nb, views, n_sel,         \
              p->g.n_views, y, st.nxs, st.nys, bxs, scale, xo, f, nx, yprev, z)
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

fb_status launch_bp(const fb_plan* p, int stage, const float* y, const int32_t* views, int n_sel, float scale,
                    float* xo, const float* yprev, float* z, bool fused, hipStream_t s) {
    return fused ? launch_bp_t<true>(p, stage, y, views, n_sel, scale, xo, yprev, z, s)
                 : launch_bp_t<false>(p, stage, y, views, n_sel, scale, xo, yprev, z, s);
}

fb_status launch_tv_single(const float* z, int nx, int ny, float lam, float tau, int n_iter, const float* p_in,
                           float* p_out, int mode, float alpha, float a_t, const float* x_prev, float* x_out,
                           float* y_out, float* hist, hipStream_t s, const PoolTarget& pt) {
    // 32 x 32 tiles with 1024 threads; 16 x 16 tiles when that leaves CUs idle
    const bool small = cdiv(nx, 32) * cdiv(ny, 32) < 256;
    const int T = small ? 16 : 32;
    if (pt.f > 0 && T % pt.f != 0) return fail(FB_EINVAL, "pooling factor does not divide the TV tile");
    dim3 grid(cdiv(nx, T), cdiv(ny, T));
#define FB_TV(TT, HH, NT)                                                                                     \
    FB_LAUNCH((k_tv<TT, HH, NT>), grid, dim3(NT), s, z, nx, ny, lam, tau, n_iter, p_in, p_out, mode, alpha, a_t, \
              x_prev, x_out, y_out, hist, pt.f, pt.inv, pt.lx, pt.px, pt.ly, pt.py, pt.nxs, pt.nys)
    if (small) {
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
        st = build_stage_tables(*geom, S.f, rays, vr, S.view_samples);
        if (st != FB_OK) return cleanup(st);
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
    if (a->next_stage < -1 || a->next_stage >= (int)p->stages.size())
        return fail(FB_EINVAL, "pnp_step: next_stage out of range");
    if (a->prepared != 0 && a->prepared != 1) return fail(FB_EINVAL, "pnp_step: prepared must be 0 or 1");
    const Stage& S = p->stages[a->stage];
    const int nx = p->g.nx, ny = p->g.ny;
    if (!a->prepared && (st = launch_prepare(p, a->stage, a->y_prev, nx, S.f, stream)) != FB_OK) return st;
    {
        TimedLaunch tl(a->events, 0);
        if ((st = launch_fp(p, a->stage, true, a->views, a->n_sel, a->b, p->resid, stream)) != FB_OK) return st;
    }
    const float step = a->eta * a->sigma / (float)(S.f * S.f);
    {
        TimedLaunch tl(a->events, 2);
        if ((st = launch_bp_t<true>(p, a->stage, p->resid, a->views, a->n_sel, step, nullptr, a->y_prev, p->zbuf,
                                    stream)) != FB_OK)
            return st;
    }
    PoolTarget pt;
    if (a->next_stage >= 0) {
        const Stage& N = p->stages[a->next_stage];
        StageLines L = stage_lines(p, a->next_stage);
        pt.f = N.f;
        pt.inv = 1.f / (float)(N.f * N.f);
        pt.lx = L.lx;
        pt.ly = L.ly;
        pt.px = N.pitch_x;
        pt.py = N.pitch_y;
        pt.nxs = N.nxs;
        pt.nys = N.nys;
    }
    // lambda == 0 or no TV iterations: D is the identity, the same kernel then
    // only applies the relaxation and momentum (div p = 0)
    const float lam = a->lambda > 0.f ? a->lambda : 1.f;
    const int iters = a->lambda > 0.f ? a->tv_iters : 0;
    TimedLaunch tl(a->events, 4);
    return launch_tv_single(p->zbuf, nx, ny, lam, a->tau, iters, nullptr, nullptr, 1, a->alpha, a->a_t, a->x_prev,
                            a->x_out, a->y_out, a->history, stream, pt);
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
    fb_status st = FB_OK;
    for (int i = 0; i < n_steps && st == FB_OK; ++i) st = pnp_step(p, &chain[i], s);
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
