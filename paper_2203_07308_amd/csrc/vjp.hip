// Reverse mode of one PnP-MS2G iteration (Sec. 2.1, Algorithm 1) for
// differentiating unrolled reconstructions: vector-Jacobian products of the
// relaxed TV-prox denoiser and of a whole pnp_step, built from the matched
// projector pair (the backprojector is the transpose of the projector, so the
// symmetric Hessian part of the sketched gradient reuses both as they are).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "fbpnp_impl.h"

using namespace fbpnp;

namespace {

// ---------------------------------------------------------------------------
// TV-prox forward recomputation in global memory (one launch per half step).
// The dual field p is zero outside the image and on the last row (p1) and
// last column (p2), so div p needs no boundary tests; the gradient masks carry
// the Neumann boundary.
// ---------------------------------------------------------------------------

// u = div p - z / lambda
__global__ __launch_bounds__(256) void k_tvf_u(const float* __restrict__ p1, const float* __restrict__ p2,
                                               const float* __restrict__ z, float il, int nx, int ny,
                                               float* __restrict__ u) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= nx) return;
    const size_t i = (size_t)r * nx + c;
    const float up = r > 0 ? p1[i - nx] : 0.f, left = c > 0 ? p2[i - 1] : 0.f;
    u[i] = (p1[i] - up) + (p2[i] - left) - z[i] * il;
}

// p' = (p + tau q) / (1 + tau |q|), q = masked forward differences of u
__global__ __launch_bounds__(256) void k_tvf_p(const float* __restrict__ u, const float* __restrict__ p1,
                                               const float* __restrict__ p2, float tau, int nx, int ny,
                                               float* __restrict__ o1, float* __restrict__ o2) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= nx) return;
    const size_t i = (size_t)r * nx + c;
    const float q1 = r < ny - 1 ? u[i + nx] - u[i] : 0.f;
    const float q2 = c < nx - 1 ? u[i + 1] - u[i] : 0.f;
    const float inv = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(fmaf(q1, q1, q2 * q2)), 1.f));
    o1[i] = fmaf(tau, q1, p1[i]) * inv;
    o2[i] = fmaf(tau, q2, p2[i]) * inv;
}

// ---------------------------------------------------------------------------
// TV-prox reverse sweep. With x = (1-alpha) z + alpha (z - lambda div p^K):
//   zbar = xbar (direct), pbar^K = -lambda alpha div^T xbar,
// and for n = K-1 .. 0, with N = p^n + tau q^n, d = 1 + tau |q^n|, p^{n+1} = N/d:
//   Nbar = pbar/d, dbar = -<pbar, p^{n+1}>/d, qbar = tau Nbar + tau dbar q/|q|
//   (0 at q = 0), pbar^n = Nbar + div^T ubar, zbar -= ubar/lambda,
//   ubar = (masked grad)^T qbar.
// (div^T w)_1[r,c] = [r < ny-1](w[r,c] - w[r+1,c]), likewise for columns.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tvb_init(const float* __restrict__ xbar, float lam_alpha, int nx, int ny,
                                                  float* __restrict__ pb1, float* __restrict__ pb2,
                                                  float* __restrict__ zbar) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= nx) return;
    const size_t i = (size_t)r * nx + c;
    const float xb = xbar[i];
    zbar[i] = xb;
    pb1[i] = r < ny - 1 ? -lam_alpha * (xb - xbar[i + nx]) : 0.f;
    pb2[i] = c < nx - 1 ? -lam_alpha * (xb - xbar[i + 1]) : 0.f;
}

__global__ __launch_bounds__(256) void k_tvb_q(const float* __restrict__ u, const float* __restrict__ pn1,
                                               const float* __restrict__ pn2, float tau, int nx, int ny,
                                               float* __restrict__ pb1, float* __restrict__ pb2,
                                               float* __restrict__ qb1, float* __restrict__ qb2) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= nx) return;
    const size_t i = (size_t)r * nx + c;
    const float q1 = r < ny - 1 ? u[i + nx] - u[i] : 0.f;
    const float q2 = c < nx - 1 ? u[i + 1] - u[i] : 0.f;
    const float mag = sqrtf(fmaf(q1, q1, q2 * q2));
    const float den = fmaf(tau, mag, 1.f);
    const float b1 = pb1[i], b2 = pb2[i];
    const float nb1 = b1 / den, nb2 = b2 / den;
    const float db = -fmaf(b1, pn1[i], b2 * pn2[i]) / den;
    const float mb = mag > 0.f ? tau * db / mag : 0.f;
    qb1[i] = fmaf(tau, nb1, mb * q1);
    qb2[i] = fmaf(tau, nb2, mb * q2);
    pb1[i] = nb1;
    pb2[i] = nb2;
}

// ubar at (rr, cc): transpose of the masked forward differences applied to qbar
__device__ __forceinline__ float ubar_at(const float* __restrict__ qb1, const float* __restrict__ qb2, int rr, int cc,
                                         int nx, int ny) {
    const size_t i = (size_t)rr * nx + cc;
    float s = 0.f;
    if (rr < ny - 1) s -= qb1[i];
    if (rr > 0) s += qb1[i - nx];
    if (cc < nx - 1) s -= qb2[i];
    if (cc > 0) s += qb2[i - 1];
    return s;
}

__global__ __launch_bounds__(256) void k_tvb_up(const float* __restrict__ qb1, const float* __restrict__ qb2,
                                                float il, int nx, int ny, float* __restrict__ pb1,
                                                float* __restrict__ pb2, float* __restrict__ zbar) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= nx) return;
    const size_t i = (size_t)r * nx + c;
    const float u0 = ubar_at(qb1, qb2, r, c, nx, ny);
    if (r < ny - 1) pb1[i] += u0 - ubar_at(qb1, qb2, r + 1, c, nx, ny);
    if (c < nx - 1) pb2[i] += u0 - ubar_at(qb1, qb2, r, c + 1, nx, ny);
    zbar[i] -= u0 * il;
}

// ---------------------------------------------------------------------------
// pnp_step reverse helpers
// ---------------------------------------------------------------------------

// z = y_prev - (eta / f^2) gs[r/f][c/f];  xtot = xbar + (1 + a) ybar;  xbar_prev = -a ybar
__global__ __launch_bounds__(256) void k_vjp_front(const float* __restrict__ yprev, const float* __restrict__ g,
                                                   int f, int nxs, float step, const float* __restrict__ xbar,
                                                   const float* __restrict__ ybar, float a_t, int nx,
                                                   float* __restrict__ z, float* __restrict__ xtot,
                                                   float* __restrict__ xbar_prev) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= nx) return;
    const size_t i = (size_t)r * nx + c;
    // the forward step's z, with its rounding (the fused back-projector's epilogue)
    z[i] = fmaf(-step, g[(size_t)(r / f) * nxs + c / f], yprev[i]);
    const float yb = ybar ? ybar[i] : 0.f;
    xtot[i] = fmaf(1.f + a_t, yb, xbar[i]);
    if (xbar_prev) xbar_prev[i] = -a_t * yb;
}

// per-block partial sums of zbar[r][c] * gs[r/f][c/f] in double, fixed order
__global__ __launch_bounds__(256) void k_dot_rep(const float* __restrict__ zb, const float* __restrict__ gs, int f,
                                                 int nxs, int nx, size_t n, double* __restrict__ part) {
    __shared__ double sm[256];
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / nx), c = (int)(i - (size_t)r * nx);
        acc += (double)zb[i] * (double)gs[(size_t)(r / f) * nxs + c / f];
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ part, int nparts, double scale,
                                                   float* __restrict__ out) {
    __shared__ double sm[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(scale * sm[0]);
}

__global__ __launch_bounds__(256) void k_zero(float* __restrict__ y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) y[i] = 0.f;
}

// y += a x
__global__ __launch_bounds__(256) void k_axpy(const float* __restrict__ x, float a, size_t n, float* __restrict__ y) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = fmaf(a, x[i], y[i]);
}

// ---------------------------------------------------------------------------
// TV-prox reverse sweep in one launch: each work-group recomputes the K dual
// steps on a 32 x 32 output tile grown by a 12-cell halo (the recomputation
// and the sweep back each move the influence of the tile's unknown
// surroundings one cell per step, 2K + 1 <= 11 cells in all), keeping every
// level p^1..p^K and u^0..u^{K-1} of its cells in registers and exchanging
// neighbour values through LDS, then sweeps back through the levels and
// writes zbar for the tile. Each cell's operations and their order are
// those of the launch chain above (k_tvf_u, k_tvf_p, k_tvb_init, k_tvb_q,
// k_tvb_up), so both give the same floats; the image-boundary conditions are
// taken on global coordinates, and cells outside the image (halo) never feed
// cells inside it. A thread owns vertical pairs of cells, as in the
// denoiser.
// ---------------------------------------------------------------------------
constexpr int kVjpTile = 32, kVjpHalo = 12, kVjpMaxFused = 5;

template <int K>
__global__ __launch_bounds__(1024) void k_tv_vjp_tile(const float* __restrict__ z, const float* __restrict__ xbar,
                                                      float* __restrict__ zbar, int nx, int ny, float il,
                                                      float lam_alpha, float tau) {
    constexpr int T = kVjpTile, H = kVjpHalo, S = T + 2 * H, NT = 1024;
    constexpr int NPAIR = (S / 2) * S, NP = (NPAIR + NT - 1) / NT;
    __shared__ float sa[S * S], sb[S * S], sc[S * S], sd[S * S];
    const int R0 = blockIdx.y * T - H, C0 = blockIdx.x * T - H;
    int e[NP], eu[NP][2], el[NP][2], ed[NP][2], er[NP][2], gr[NP], gc[NP];
    bool live[NP], in[NP][2];
    float zz[NP][2], xb[NP][2];
    float P1[K + 1][NP][2], P2[K + 1][NP][2], U[K][NP][2];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int q = threadIdx.x + k * NT;
        live[k] = q < NPAIR;
        const int qq = live[k] ? q : NPAIR - 1;
        const int pr = qq / S, lc = qq - pr * S, lr = 2 * pr;
        e[k] = lr * S + lc;
        gr[k] = R0 + lr;
        gc[k] = C0 + lc;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = lr + h, ei = e[k] + h * S;
            // neighbours inside the tile (at its edge the cell itself: those cells are halo)
            eu[k][h] = r > 0 ? ei - S : ei;
            ed[k][h] = r < S - 1 ? ei + S : ei;
            el[k][h] = lc > 0 ? ei - 1 : ei;
            er[k][h] = lc < S - 1 ? ei + 1 : ei;
            const int g = gr[k] + h;
            in[k][h] = g >= 0 && g < ny && gc[k] >= 0 && gc[k] < nx;
            const size_t gi = (size_t)(in[k][h] ? g : 0) * nx + (in[k][h] ? gc[k] : 0);
            zz[k][h] = in[k][h] ? z[gi] : 0.f;
            xb[k][h] = in[k][h] ? xbar[gi] : 0.f;
            P1[0][k][h] = P2[0][k][h] = 0.f;
            if (live[k]) sa[ei] = sb[ei] = 0.f;
        }
    }
    __syncthreads();
    // forward: u^n = div p^n - z / lambda, p^{n+1} = (p^n + tau q^n) / (1 + tau |q^n|)
#pragma unroll
    for (int n = 0; n < K; ++n) {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float up = gr[k] + h > 0 ? sa[eu[k][h]] : 0.f;
                const float left = gc[k] > 0 ? sb[el[k][h]] : 0.f;
                U[n][k][h] = (P1[n][k][h] - up) + (P2[n][k][h] - left) - zz[k][h] * il;
            }
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (live[k]) sc[e[k] + h * S] = U[n][k][h];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float q1 = gr[k] + h < ny - 1 ? sc[ed[k][h]] - U[n][k][h] : 0.f;
                const float q2 = gc[k] < nx - 1 ? sc[er[k][h]] - U[n][k][h] : 0.f;
                const float inv =
                    __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(fmaf(q1, q1, q2 * q2)), 1.f));
                P1[n + 1][k][h] = fmaf(tau, q1, P1[n][k][h]) * inv;
                P2[n + 1][k][h] = fmaf(tau, q2, P2[n][k][h]) * inv;
            }
        if (n + 1 < K) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (live[k]) {
                        sa[e[k] + h * S] = P1[n + 1][k][h];
                        sb[e[k] + h * S] = P2[n + 1][k][h];
                    }
        }
        __syncthreads();
    }
    // reverse: zbar = xbar, pbar^K = -lambda alpha div^T xbar
    float zb[NP][2], pb1[NP][2], pb2[NP][2];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (live[k]) {
                sc[e[k] + h * S] = xb[k][h];
                sd[e[k] + h * S] = U[K - 1][k][h];
            }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            zb[k][h] = xb[k][h];
            pb1[k][h] = gr[k] + h < ny - 1 ? -lam_alpha * (xb[k][h] - sc[ed[k][h]]) : 0.f;
            pb2[k][h] = gc[k] < nx - 1 ? -lam_alpha * (xb[k][h] - sc[er[k][h]]) : 0.f;
        }
#pragma unroll
    for (int n = K - 1; n >= 0; --n) {
        // qbar from pbar^{n+1}, q^n (u^n of the cell and its neighbours) and p^{n+1}
        float qb1[NP][2], qb2[NP][2];
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float q1 = gr[k] + h < ny - 1 ? sd[ed[k][h]] - U[n][k][h] : 0.f;
                const float q2 = gc[k] < nx - 1 ? sd[er[k][h]] - U[n][k][h] : 0.f;
                const float mag = sqrtf(fmaf(q1, q1, q2 * q2));
                const float den = fmaf(tau, mag, 1.f);
                const float b1 = pb1[k][h], b2 = pb2[k][h];
                const float nb1 = b1 / den, nb2 = b2 / den;
                const float db = -fmaf(b1, P1[n + 1][k][h], b2 * P2[n + 1][k][h]) / den;
                const float mb = mag > 0.f ? tau * db / mag : 0.f;
                qb1[k][h] = fmaf(tau, nb1, mb * q1);
                qb2[k][h] = fmaf(tau, nb2, mb * q2);
                pb1[k][h] = nb1;
                pb2[k][h] = nb2;
            }
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (live[k]) {
                    sa[e[k] + h * S] = qb1[k][h];
                    sb[e[k] + h * S] = qb2[k][h];
                }
        __syncthreads();
        // ubar = (masked grad)^T qbar at the cell
        float ub[NP][2];
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int rr = gr[k] + h, cc = gc[k];
                float s = 0.f;
                if (rr < ny - 1) s -= qb1[k][h];
                if (rr > 0) s += sa[eu[k][h]];
                if (cc < nx - 1) s -= qb2[k][h];
                if (cc > 0) s += sb[el[k][h]];
                ub[k][h] = s;
            }
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (live[k]) sc[e[k] + h * S] = ub[k][h];
        __syncthreads();
        // pbar^n = Nbar + div^T ubar, zbar -= ubar / lambda; and u^{n-1} for the next step
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float u0 = ub[k][h];
                if (gr[k] + h < ny - 1) pb1[k][h] += u0 - sc[ed[k][h]];
                if (gc[k] < nx - 1) pb2[k][h] += u0 - sc[er[k][h]];
                zb[k][h] -= u0 * il;
                if (n > 0 && live[k]) sd[e[k] + h * S] = U[n - 1][k][h];
            }
        __syncthreads();
    }
    // the output tile
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int pr = (live[k] ? threadIdx.x + k * NT : NPAIR - 1) / S;
        const int lc = e[k] - 2 * pr * S;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lr = 2 * pr + h;
            if (live[k] && in[k][h] && lr >= H && lr < H + T && lc >= H && lc < H + T)
                zbar[(size_t)(gr[k] + h) * nx + gc[k]] = zb[k][h];
        }
    }
}

size_t tv_ws_floats(int nx, int ny, int n_iter) {
    // up to kVjpMaxFused steps the one-launch sweep keeps every level on chip;
    // beyond, p levels 0..K (two planes each), u levels 0..K-1, pbar, qbar
    if (n_iter <= kVjpMaxFused) return 0;
    return (size_t)nx * ny * (size_t)(2 * (n_iter + 1) + n_iter + 4);
}

// zbar = J^T xbar for z -> (1 - alpha) z + alpha TV_prox(z); ws holds tv_ws_floats.
fb_status launch_tv_vjp(const float* z, const float* xbar, float* zbar, int nx, int ny, float lam, int K, float tau,
                        float alpha, float* ws, hipStream_t s) {
    const size_t n = (size_t)nx * ny;
    dim3 grid(cdiv(nx, 256), ny);
    if (lam == 0.f || K == 0 || alpha == 0.f) {
        hipError_t e = hipMemcpyAsync(zbar, xbar, n * sizeof(float), hipMemcpyDeviceToDevice, s);
        return e == hipSuccess ? FB_OK : hip_fail(e, "tv vjp copy");
    }
    if (K <= kVjpMaxFused) {
        const dim3 tiles(cdiv(nx, kVjpTile), cdiv(ny, kVjpTile));
        const float il = 1.f / lam, la = lam * alpha;
        switch (K) {
            case 1: k_tv_vjp_tile<1><<<tiles, 1024, 0, s>>>(z, xbar, zbar, nx, ny, il, la, tau); break;
            case 2: k_tv_vjp_tile<2><<<tiles, 1024, 0, s>>>(z, xbar, zbar, nx, ny, il, la, tau); break;
            case 3: k_tv_vjp_tile<3><<<tiles, 1024, 0, s>>>(z, xbar, zbar, nx, ny, il, la, tau); break;
            case 4: k_tv_vjp_tile<4><<<tiles, 1024, 0, s>>>(z, xbar, zbar, nx, ny, il, la, tau); break;
            default: k_tv_vjp_tile<5><<<tiles, 1024, 0, s>>>(z, xbar, zbar, nx, ny, il, la, tau); break;
        }
        return check_launch("tv_prox_vjp");
    }
    float* P = ws;                       // level k: P + 2 k n (p1), + n (p2)
    float* U = P + 2 * (size_t)(K + 1) * n;  // level k: U + k n
    float* pb1 = U + (size_t)K * n;
    float* pb2 = pb1 + n;
    float* qb1 = pb2 + n;
    float* qb2 = qb1 + n;
    const float il = 1.f / lam;
    k_zero<<<cdiv((int)std::min<size_t>(2 * n, 1 << 20), 256), 256, 0, s>>>(P, 2 * n);  // p^0 = 0
    for (int k = 0; k < K; ++k) {
        float* p1 = P + 2 * (size_t)k * n;
        k_tvf_u<<<grid, 256, 0, s>>>(p1, p1 + n, z, il, nx, ny, U + (size_t)k * n);
        k_tvf_p<<<grid, 256, 0, s>>>(U + (size_t)k * n, p1, p1 + n, tau, nx, ny, p1 + 2 * n, p1 + 3 * n);
    }
    k_tvb_init<<<grid, 256, 0, s>>>(xbar, lam * alpha, nx, ny, pb1, pb2, zbar);
    for (int k = K - 1; k >= 0; --k) {
        float* pn = P + 2 * (size_t)(k + 1) * n;
        k_tvb_q<<<grid, 256, 0, s>>>(U + (size_t)k * n, pn, pn + n, tau, nx, ny, pb1, pb2, qb1, qb2);
        k_tvb_up<<<grid, 256, 0, s>>>(qb1, qb2, il, nx, ny, pb1, pb2, zbar);
    }
    return check_launch("tv_prox_vjp");
}

}  // namespace

extern "C" {

size_t fb_tv_vjp_workspace_bytes(int nx, int ny, int n_iter) {
    if (nx < 1 || ny < 1 || n_iter < 0) return 0;
    return tv_ws_floats(nx, ny, n_iter) * sizeof(float);
}

fb_status tv_prox_vjp(const float* z, const float* xbar, float* zbar, int nx, int ny, float lambda, int n_iter,
                      float tau, float alpha, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!z || !xbar || !zbar || nx < 1 || ny < 1 || n_iter < 0) return fail(FB_EINVAL, "tv_prox_vjp: bad arguments");
    if (!(lambda >= 0.f) || !(tau > 0.f)) return fail(FB_EINVAL, "tv_prox_vjp: need lambda >= 0 and tau > 0");
    if (zbar == xbar || zbar == z) return fail(FB_EINVAL, "tv_prox_vjp: zbar must not alias the inputs");
    const size_t need = fb_tv_vjp_workspace_bytes(nx, ny, n_iter);
    if (need > 0 && (!ws || ws_bytes < need)) return fail(FB_EINVAL, "tv_prox_vjp: workspace too small");
    return launch_tv_vjp(z, xbar, zbar, nx, ny, lambda, n_iter, tau, alpha, (float*)ws, stream);
}

// Float offset of the double-precision reduction partials in a pnp_step_vjp
// workspace: after z, xtot, zbar, the coarse gradient and the TV reverse sweep,
// rounded up to 256 bytes so the doubles are aligned for any image size.
static size_t vjp_part_offset_floats(int nx, int ny, int tv_iters) {
    const size_t n = (size_t)nx * ny;
    return (4 * n + tv_ws_floats(nx, ny, tv_iters) + 63) / 64 * 64;
}

size_t fb_pnp_vjp_workspace_bytes(const fb_plan* p, int tv_iters) {
    if (!p || tv_iters < 0) return 0;
    // the float buffers, then the reduction partials (+1 result)
    return vjp_part_offset_floats(p->g.nx, p->g.ny, tv_iters) * sizeof(float) + (kRedBlocks + 2) * sizeof(double);
}

fb_status pnp_step_vjp(const fb_plan* p, const fb_pnp_args* a, const float* xbar, const float* ybar, float* xbar_prev,
                       float* ybar_prev, float* eta_bar, int combine, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!a || !xbar || !ybar_prev || !eta_bar) return fail(FB_EINVAL, "pnp_step_vjp: null argument");
    fb_status st = check_stage(p, a->stage);
    if (st != FB_OK) return st;
    if ((st = check_pnp_views(p, a)) != FB_OK) return st;
    if (!a->b || !a->y_prev) return fail(FB_EINVAL, "pnp_step_vjp: null buffer in args");
    if (a->vr_mode != 0) return fail(FB_EINVAL, "pnp_step_vjp: variance-reduced steps are not differentiated");
    if (bicubic_stage(p, a->stage)) return fail(FB_EINVAL, "pnp_step_vjp: differentiated with the pooling sketch only");
    if (a->tv_iters < 0 || a->tv_iters > 64) return fail(FB_EINVAL, "pnp_step_vjp: tv_iters out of range");
    if (!(a->lambda >= 0.f) || !(a->tau > 0.f)) return fail(FB_EINVAL, "pnp_step_vjp: need lambda >= 0 and tau > 0");
    if (!ws || ws_bytes < fb_pnp_vjp_workspace_bytes(p, a->tv_iters))
        return fail(FB_EINVAL, "pnp_step_vjp: workspace too small");
    if ((uintptr_t)ws % 256 != 0) return fail(FB_EINVAL, "pnp_step_vjp: workspace must be 256-byte aligned");
    const float* outs[] = {xbar_prev, ybar_prev};
    const float* ins[] = {xbar, ybar, a->y_prev, a->x_prev, a->b, a->grad};
    for (const float* o : outs)
        for (const float* q : ins)
            if (o && o == q) return fail(FB_EINVAL, "pnp_step_vjp: outputs must not alias inputs");
    if (xbar_prev && xbar_prev == ybar_prev) return fail(FB_EINVAL, "pnp_step_vjp: xbar_prev aliases ybar_prev");
    const Stage& S = p->stages[a->stage];
    const int nx = p->g.nx, ny = p->g.ny, f = S.f;
    const size_t n = (size_t)nx * ny;
    float* z = (float*)ws;
    float* xtot = z + n;
    float* zbar = xtot + n;
    float* gs = zbar + n;
    float* tvws = gs + n;
    double* part = (double*)((float*)ws + vjp_part_offset_floats(nx, ny, a->tv_iters));
    const dim3 grid(cdiv(nx, 256), ny);
    // the unscaled coarse gradient g = A_s^T M (M A_s S y - M b) of the step
    // (G = sigma g): stored by the forward step, or recomputed with the same
    // kernels and launch configuration, so it has the same bits either way
    const float* g = a->grad;
    if (!g) {
        if ((st = launch_prepare(p, a->stage, a->y_prev, nx, f, stream)) != FB_OK) return st;
        if ((st = launch_fp(p, a->stage, true, pnp_views(a), a->b, p->resid, stream)) != FB_OK) return st;
        if ((st = launch_bp(p, a->stage, p->resid, pnp_views(a), 1.f, gs, nullptr, nullptr, false, stream)) != FB_OK)
            return st;
        g = gs;
    }
    // z = y - eta sigma U g, as the forward step rounds it
    const float inv_ff = 1.f / (float)(f * f);
    const float step = a->eta * a->sigma / (float)(f * f);
    k_vjp_front<<<grid, 256, 0, stream>>>(a->y_prev, g, f, S.nxs, step, xbar, ybar, a->a_t, nx, z, xtot,
                                          combine ? nullptr : xbar_prev);
    if ((st = check_launch("pnp_step_vjp front")) != FB_OK) return st;
    // zbar = J_relax^T xtot
    const int K = a->lambda > 0.f ? a->tv_iters : 0;
    if ((st = launch_tv_vjp(z, xtot, zbar, nx, ny, a->lambda, K, a->tau, a->alpha, tvws, stream)) != FB_OK) return st;
    // eta_bar = -<zbar, U G> = -(sigma / f^2) <zbar, g replicated>
    k_dot_rep<<<kRedBlocks, 256, 0, stream>>>(zbar, g, f, S.nxs, nx, n, part);
    k_dot_final<<<1, 256, 0, stream>>>(part, kRedBlocks, -(double)a->sigma / (double)(f * f), eta_bar);
    if ((st = check_launch("pnp_step_vjp eta")) != FB_OK) return st;
    // ybar_prev = zbar - eta sigma U A_s^T M^T M A_s S zbar
    if ((st = launch_prepare(p, a->stage, zbar, nx, f, stream)) != FB_OK) return st;
    if ((st = launch_fp(p, a->stage, false, pnp_views(a), nullptr, p->resid, stream)) != FB_OK) return st;
    if ((st = launch_bp(p, a->stage, p->resid, pnp_views(a), a->eta * a->sigma * inv_ff, nullptr, zbar, ybar_prev,
                        true, stream)) != FB_OK)
        return st;
    if (combine && ybar) {
        // adjoint of x_0 = y_0: ybar_prev + xbar_prev, xbar_prev = -a ybar
        k_axpy<<<cdiv((int)std::min<size_t>(n, 1 << 20), 256), 256, 0, stream>>>(ybar, -a->a_t, n, ybar_prev);
        if ((st = check_launch("pnp_step_vjp combine")) != FB_OK) return st;
    }
    return FB_OK;
}

}  // extern "C"
