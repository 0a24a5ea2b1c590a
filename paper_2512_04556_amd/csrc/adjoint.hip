// Adjoint of a uniform-Theta sparse layer (the end-to-end differentiation of
// Sec. 4.1): gradients w.r.t. every tap's offset and weight, and w.r.t. the
// layer input.
//
// For a tap with corner offset (ix, iy) = floor(-o), fractions (fx, fy) and
// weight w, let S_ab = sum_p G[p] X[map(p + (ix + a, iy + b))] (channels summed,
// map = the boundary rule).  Then
//   dL/dw   = sum_ab c_ab S_ab / w          (c_ab = w * bilinear corner weight)
//   dL/dox  = -w [(1-fy)(S01 - S00) + fy (S11 - S10)]
//   dL/doy  = -w [(1-fx)(S10 - S00) + fx (S11 - S01)]
// so a tap costs four correlation sums per pixel.  Sums are reduced per block
// (wave butterflies then a fixed LDS order) into partials, then across blocks
// in a fixed order: results are bitwise reproducible.
//
// The input adjoint is the exact transpose of the gather:
//   Gprev[q] = sum_i sum_ab c_ab sum_{p : map(p + d_ab) = q} G[p].
// For ZERO the preimage is the single pixel q - d (if inside); for CLAMP a
// border pixel's preimage is a run (edge) or block (corner) of pixels, which
// the kernel sums directly.
#include "common.hpp"
#include "internal.hpp"

namespace disk {

constexpr int kTW = 64;
constexpr int kRows = 8;
constexpr int kTH = 4 * kRows;

int adjoint_tap_blocks(int H, int W) {
    const int ntiles = ((W + kTW - 1) / kTW) * ((H + kTH - 1) / kTH);
    return 8 * ((ntiles + 7) / 8);
}

struct SrcF32 {
    const float* p;
    __device__ __forceinline__ float load(size_t i) const { return p[i]; }
};
struct SrcBF16 {
    const uint16_t* p;
    __device__ __forceinline__ float load(size_t i) const { return bf16_to_f32(p[i]); }
};
struct SrcImpulse {
    size_t centre;
    __device__ __forceinline__ float load(size_t i) const { return i == centre ? 1.0f : 0.0f; }
};

template <int C, int BOUND, class Src>
__global__ __launch_bounds__(256) void adjoint_taps_kernel(Src src, const float* __restrict__ G,
                                                           const TapU* __restrict__ taps, int N, int H,
                                                           int W, int tiles_x, int per, int ntiles,
                                                           float* __restrict__ partial) {
    __shared__ float red[4][4];
    const int tile = xcd_tile(blockIdx.x, per);
    const bool active = tile < ntiles;
    const int x = active ? (tile % tiles_x) * kTW + (threadIdx.x & 63) : W;
    const int yb = active ? (tile / tiles_x) * kTH + (threadIdx.x >> 6) * kRows : H;
    const size_t plane = static_cast<size_t>(H) * W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    for (int i = 0; i < N; ++i) {
        const TapU t = taps[i];
        float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (x < W) {
            int x0 = x + t.ix, x1 = x0 + 1;
            const bool vx0 = x0 >= 0 && x0 < W, vx1 = x1 >= 0 && x1 < W;
            x0 = min(max(x0, 0), W - 1);
            x1 = min(max(x1, 0), W - 1);
            for (int r = 0; r < kRows; ++r) {
                const int y = yb + r;
                if (y >= H) break;
                int y0 = y + t.iy, y1 = y0 + 1;
                const bool vy0 = y0 >= 0 && y0 < H, vy1 = y1 >= 0 && y1 < H;
                y0 = min(max(y0, 0), H - 1);
                y1 = min(max(y1, 0), H - 1);
                const size_t r0 = static_cast<size_t>(y0) * W, r1 = static_cast<size_t>(y1) * W;
                const size_t pix = static_cast<size_t>(y) * W + x;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float g = G[c * plane + pix];
                    float v00 = src.load(c * plane + r0 + x0), v01 = src.load(c * plane + r0 + x1);
                    float v10 = src.load(c * plane + r1 + x0), v11 = src.load(c * plane + r1 + x1);
                    if (BOUND == DISK_ZERO) {
                        v00 = (vx0 && vy0) ? v00 : 0.0f;
                        v01 = (vx1 && vy0) ? v01 : 0.0f;
                        v10 = (vx0 && vy1) ? v10 : 0.0f;
                        v11 = (vx1 && vy1) ? v11 : 0.0f;
                    }
                    s[0] = fmaf(g, v00, s[0]);
                    s[1] = fmaf(g, v01, s[1]);
                    s[2] = fmaf(g, v10, s[2]);
                    s[3] = fmaf(g, v11, s[3]);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) s[a] = wave_sum(s[a]);
        if (lane == 0)
#pragma unroll
            for (int a = 0; a < 4; ++a) red[wave][a] = s[a];
        __syncthreads();
        if (threadIdx.x < 4) {
            const int a = threadIdx.x;
            const float v = (red[0][a] + red[1][a]) + (red[2][a] + red[3][a]);
            partial[(static_cast<size_t>(blockIdx.x) * N + i) * 4 + a] = v;
        }
        __syncthreads();
    }
}

// One work-group per tap: the four corner sums S_ab over the nblk block
// partials (thread t adds blocks t, t + 256, ... in order, then a fixed tree),
// and from them the tap's gradient (the bilinear weights' derivatives).
__device__ __forceinline__ void finish_tap(const float* __restrict__ partial, int nblk, int N, int i,
                                           const float* __restrict__ theta, float* __restrict__ dtheta) {
    __shared__ float buf[4][256];
    const int t = threadIdx.x;
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int b = t; b < nblk; b += 256) {
        const float* q = partial + (static_cast<size_t>(b) * N + i) * 4;
#pragma unroll
        for (int a = 0; a < 4; ++a) v[a] += q[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) buf[a][t] = v[a];
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if (t < m)
#pragma unroll
            for (int a = 0; a < 4; ++a) buf[a][t] += buf[a][t + m];
        __syncthreads();
    }
    if (t != 0) return;
    const float ox = theta[3 * i + 0], oy = theta[3 * i + 1], w = theta[3 * i + 2];
    int ix, iy;
    float fx, fy;
    floor_frac(-ox, ix, fx);
    floor_frac(-oy, iy, fy);
    const float S00 = buf[0][0], S01 = buf[1][0], S10 = buf[2][0], S11 = buf[3][0];
    const float gw = (1.0f - fy) * ((1.0f - fx) * S00 + fx * S01) + fy * ((1.0f - fx) * S10 + fx * S11);
    const float gx = -w * ((1.0f - fy) * (S01 - S00) + fy * (S11 - S10));
    const float gy = -w * ((1.0f - fx) * (S10 - S00) + fx * (S11 - S01));
    dtheta[3 * i + 0] = gx;
    dtheta[3 * i + 1] = gy;
    dtheta[3 * i + 2] = gw;
}

__global__ __launch_bounds__(256) void adjoint_finish_kernel(const float* __restrict__ partial, int nblk, int N,
                                                             const float* __restrict__ theta,
                                                             float* __restrict__ dtheta) {
    finish_tap(partial, nblk, N, blockIdx.x, theta, dtheta);
}

// The finish of several layers in one launch: work-group b takes tap
// b - first[l] of entry l (first[] ascending).
__global__ __launch_bounds__(256) void adjoint_finish_layers_kernel(FinishLayers a, const float* __restrict__ partial,
                                                                    const float* __restrict__ theta,
                                                                    float* __restrict__ dtheta) {
    int l = 0;
    while (l + 1 < a.n && static_cast<int>(blockIdx.x) >= a.first[l + 1]) ++l;
    finish_tap(partial + a.pofs[l], a.nblk[l], a.N[l], blockIdx.x - a.first[l], theta + 3 * a.tap0[l],
               dtheta + 3 * a.tap0[l]);
}

template <int C, int BOUND, class Src>
static hipError_t taps_launch(Src src, const float* G, const TapU* taps, int N, int H, int W, float* partial,
                              hipStream_t s) {
    const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + kTH - 1) / kTH;
    const int ntiles = tiles_x * tiles_y;
    const int per = (ntiles + 7) / 8;
    hipLaunchKernelGGL((adjoint_taps_kernel<C, BOUND, Src>), dim3(8 * per), dim3(256), 0, s, src, G, taps, N, H,
                       W, tiles_x, per, ntiles, partial);
    return hipGetLastError();
}

template <int C, int BOUND>
static hipError_t taps_src(int src_kind, const void* X, const float* G, const TapU* taps, int N, int H, int W,
                           float* partial, hipStream_t s) {
    if (src_kind == 0) return taps_launch<C, BOUND>(SrcF32{static_cast<const float*>(X)}, G, taps, N, H, W, partial, s);
    if (src_kind == 1) return taps_launch<C, BOUND>(SrcBF16{static_cast<const uint16_t*>(X)}, G, taps, N, H, W, partial, s);
    const size_t centre = static_cast<size_t>((H - 1) / 2) * W + (W - 1) / 2;
    return taps_launch<C, BOUND>(SrcImpulse{centre}, G, taps, N, H, W, partial, s);
}

template <int C>
static hipError_t taps_bound(int boundary, int src_kind, const void* X, const float* G, const TapU* taps, int N,
                             int H, int W, float* partial, hipStream_t s) {
    if (boundary == DISK_ZERO) return taps_src<C, DISK_ZERO>(src_kind, X, G, taps, N, H, W, partial, s);
    return taps_src<C, DISK_CLAMP>(src_kind, X, G, taps, N, H, W, partial, s);
}

hipError_t launch_adjoint_taps(int C, int boundary, int src_kind, const void* X, const float* G,
                               const TapU* taps, int N, int H, int W, float* partial, hipStream_t s) {
    switch (C) {
        case 1: return taps_bound<1>(boundary, src_kind, X, G, taps, N, H, W, partial, s);
        case 2: return taps_bound<2>(boundary, src_kind, X, G, taps, N, H, W, partial, s);
        case 3: return taps_bound<3>(boundary, src_kind, X, G, taps, N, H, W, partial, s);
        default: return taps_bound<4>(boundary, src_kind, X, G, taps, N, H, W, partial, s);
    }
}

// `partial` holds nblk * N * 4 block partials (the workspace carving also
// reserves N * 4 floats after them).
hipError_t launch_adjoint_finish_layers(const FinishLayers& a, const float* partial, const float* theta, float* dtheta,
                                        hipStream_t s) {
    if (a.n < 1 || a.n > DISK_MAX_LAYERS) return hipErrorInvalidValue;
    const int nwg = a.first[a.n - 1] + a.N[a.n - 1];
    hipLaunchKernelGGL(adjoint_finish_layers_kernel, dim3(nwg), dim3(256), 0, s, a, partial, theta, dtheta);
    return hipGetLastError();
}

hipError_t launch_adjoint_finish(float* partial, int nblk, const float* theta_layer, int N, float* dtheta_layer,
                                 hipStream_t s) {
    hipLaunchKernelGGL(adjoint_finish_kernel, dim3(N), dim3(256), 0, s, partial, nblk, N, theta_layer,
                       dtheta_layer);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// input adjoint
// ---------------------------------------------------------------------------
// Preimage range along one axis of corner shift d: all p in [0, n) with
// map(p + d) == q.
template <int BOUND>
__device__ __forceinline__ void preimage(int q, int d, int n, int& lo, int& hi) {
    if (BOUND == DISK_ZERO) {
        lo = hi = q - d;
    } else {
        lo = (q == 0) ? -0x3fffffff : q - d;
        hi = (q == n - 1) ? 0x3fffffff : q - d;
    }
    lo = max(lo, 0);
    hi = min(hi, n - 1);
}

// Gprev at pixel (x, y): the exact transpose (border pixels of CLAMP sum the
// run or block of output pixels whose clamped corner lands on them).
template <int C, int BOUND>
__device__ __forceinline__ void input_adjoint_pixel(const float* __restrict__ G, const TapU* __restrict__ taps, int N,
                                                    int H, int W, int x, int y, float (&acc)[C]) {
    const size_t plane = static_cast<size_t>(H) * W;
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0f;
    const bool border = (BOUND == DISK_CLAMP) && (x == 0 || y == 0 || x == W - 1 || y == H - 1);
    for (int i = 0; i < N; ++i) {
        const TapU t = taps[i];
        const float cw[4] = {t.c00, t.c01, t.c10, t.c11};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int dx = t.ix + (a & 1), dy = t.iy + (a >> 1);
            if (!border) {
                const int px = x - dx, py = y - dy;
                if (px >= 0 && px < W && py >= 0 && py < H) {
                    const size_t pi = static_cast<size_t>(py) * W + px;
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c] = fmaf(cw[a], G[c * plane + pi], acc[c]);
                }
            } else {
                int xl, xh, yl, yh;
                preimage<BOUND>(x, dx, W, xl, xh);
                preimage<BOUND>(y, dy, H, yl, yh);
                for (int py = yl; py <= yh; ++py)
                    for (int px = xl; px <= xh; ++px) {
                        const size_t pi = static_cast<size_t>(py) * W + px;
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[c] = fmaf(cw[a], G[c * plane + pi], acc[c]);
                    }
            }
        }
    }
}

template <int C, int BOUND>
__global__ __launch_bounds__(256) void adjoint_input_kernel(const float* __restrict__ G,
                                                            const TapU* __restrict__ taps, int N, int H,
                                                            int W, float* __restrict__ Gprev) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const size_t plane = static_cast<size_t>(H) * W;
    float acc[C];
    input_adjoint_pixel<C, BOUND>(G, taps, N, H, W, x, y, acc);
#pragma unroll
    for (int c = 0; c < C; ++c) Gprev[c * plane + static_cast<size_t>(y) * W + x] = acc[c];
}

// The CLAMP border pixels only (rows 0 and H-1, columns 0 and W-1): run after
// the interior was produced by the zero-padded transposed gather, one wave
// per border pixel.
__device__ __forceinline__ long border_count(int H, int W) {
    return (H <= 2 || W <= 2) ? static_cast<long>(H) * W : 2L * W + 2L * (H - 2);
}
// Border pixel i (wave-uniform) of the input adjoint: lane l takes the (tap,
// corner) pairs l, l + 64, ... and sums their preimage runs; a fixed
// butterfly adds the lanes.
template <int C>
__device__ __forceinline__ void input_border_pixel(const float* __restrict__ G, const TapU* __restrict__ taps, int N,
                                                   int H, int W, long i, float* __restrict__ Gprev) {
    const int lane = threadIdx.x & 63;
    int x, y;
    if (H <= 2 || W <= 2) {
        y = static_cast<int>(i / W);
        x = static_cast<int>(i - static_cast<long>(y) * W);
    } else if (i < 2L * W) {
        y = i < W ? 0 : H - 1;
        x = static_cast<int>(i < W ? i : i - W);
    } else {
        const int j = static_cast<int>(i - 2L * W);
        x = j < H - 2 ? 0 : W - 1;
        y = 1 + (j < H - 2 ? j : j - (H - 2));
    }
    const size_t plane = static_cast<size_t>(H) * W;
    float acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0f;
    for (int pr = lane; pr < 4 * N; pr += 64) {
        const TapU t = taps[pr >> 2];
        const int a = pr & 3;
        const float cw = a == 0 ? t.c00 : a == 1 ? t.c01 : a == 2 ? t.c10 : t.c11;
        int xl, xh, yl, yh;
        preimage<DISK_CLAMP>(x, t.ix + (a & 1), W, xl, xh);
        preimage<DISK_CLAMP>(y, t.iy + (a >> 1), H, yl, yh);
        for (int py = yl; py <= yh; ++py)
            for (int px = xl; px <= xh; ++px) {
                const size_t pi = static_cast<size_t>(py) * W + px;
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] = fmaf(cw, G[c * plane + pi], acc[c]);
            }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = wave_sum(acc[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < C; ++c) Gprev[c * plane + static_cast<size_t>(y) * W + x] = acc[c];
}

template <int C>
__global__ __launch_bounds__(256) void adjoint_input_border_kernel(const float* __restrict__ G,
                                                                   const TapU* __restrict__ taps, int N, int H,
                                                                   int W, float* __restrict__ Gprev) {
    const long i = (static_cast<long>(blockIdx.x) * 256 + threadIdx.x) >> 6;   // one wave per border pixel
    if (i < border_count(H, W)) input_border_pixel<C>(G, taps, N, H, W, i, Gprev);
}

hipError_t launch_adjoint_input_border(int C, const float* G, const TapU* taps, int N, int H, int W, float* Gprev,
                                       hipStream_t s) {
    const long nb = (H <= 2 || W <= 2) ? static_cast<long>(H) * W : 2L * W + 2L * (H - 2);
    const dim3 grid(static_cast<unsigned>((nb + 3) / 4)), block(256);   // one wave per border pixel
    if (C == 3)
        hipLaunchKernelGGL((adjoint_input_border_kernel<3>), grid, block, 0, s, G, taps, N, H, W, Gprev);
    else if (C == 4)
        hipLaunchKernelGGL((adjoint_input_border_kernel<4>), grid, block, 0, s, G, taps, N, H, W, Gprev);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CLAMP border work of one fused backward layer, in one launch
// ---------------------------------------------------------------------------
struct BorderArgs {
    const float* G;         // the layer's output gradient
    const float* X;         // its input
    const float* theta;     // its N taps
    const TapU* taps;
    int N, NS, H, W, hmax, parts, nA, nrows;
    float* partial;         // nrows rows of N * 4 correlation partials; the last `parts` are written here
    float* Gprev;           // the input adjoint, whose border pixels are written here
};

// Work-groups [0, nA): the CLAMP samples the fused pass leaves out, for tap i
// < NS and corner ab: over the pixels p whose sample p + d + ab (d =
// floor(-o_i)) leaves the image, G(p) X(clamp(p + d + ab)) summed over the
// channels (zero for i >= NS, and for every tap when the layer's halo exceeds
// hmax: the fused kernel's fallback then reads those samples itself).  The
// pixels (the rows whose sample row leaves the image, whole, then the sample
// columns that leave it in the other rows) are split into `parts`; (tap,
// corner, part) writes entry 4 i + ab of border row `part` (rows nrows - parts
// .. nrows - 1).  Work-groups [nA, ...): the input adjoint's border pixels, one
// wave each (input_border_pixel).  Fixed-order sums.
// (dTheta then needs every row: adjoint_finish_kernel, launched after this.
// Reducing it in the last correlation work-group instead needs a device-scope
// release per work-group, an L2 write-back each on this GPU: far slower.)
template <int C>
__global__ __launch_bounds__(256) void adjoint_border_kernel(BorderArgs a) {
    __shared__ float red[4];
    const int t = threadIdx.x;
    if (static_cast<int>(blockIdx.x) < a.nA) {
        const int part = blockIdx.x % a.parts, ia = blockIdx.x / a.parts, i = ia >> 2, ab = ia & 3;
        const int N = a.N, H = a.H, W = a.W;
        float m = 0.0f;
        for (int k = 0; k < N; ++k) {
            float mk = fmaxf(fabsf(a.theta[3 * k]), fabsf(a.theta[3 * k + 1]));
            if (!(mk <= 1.0e6f)) mk = 1.0e6f;   // non-finite or huge
            m = fmaxf(m, mk);
        }
        const int halo = static_cast<int>(ceilf(m)) + 1;
        float v = 0.0f;
        if (i < a.NS && halo <= a.hmax) {
            const int dx = static_cast<int>(floorf(-a.theta[3 * i])) + (ab & 1);
            const int dy = static_cast<int>(floorf(-a.theta[3 * i + 1])) + (ab >> 1);
            const int rlo = dy < 0 ? min(-dy, H) : 0, rhi = dy > 0 ? min(dy, H - rlo) : 0;
            const int clo = dx < 0 ? min(-dx, W) : 0, chi = dx > 0 ? min(dx, W - clo) : 0;
            const int ncol = clo + chi, nin = H - rlo - rhi;
            const long n1 = static_cast<long>(rlo + rhi) * W, n = n1 + static_cast<long>(nin) * ncol;
            const size_t plane = static_cast<size_t>(H) * W;
            const long u0 = n * part / a.parts, u1 = n * (part + 1) / a.parts;
            for (long u = u0 + t; u < u1; u += 256) {
                int x, y;
                if (u < n1) {
                    const int r = static_cast<int>(u / W);
                    x = static_cast<int>(u - static_cast<long>(r) * W);
                    y = r < rlo ? r : H - rhi + (r - rlo);
                } else {
                    const long w = u - n1;
                    const int r = static_cast<int>(w / ncol), k = static_cast<int>(w - static_cast<long>(r) * ncol);
                    y = rlo + r;
                    x = k < clo ? k : W - chi + (k - clo);
                }
                const int sx = min(max(x + dx, 0), W - 1), sy = min(max(y + dy, 0), H - 1);
                const size_t pg = static_cast<size_t>(y) * W + x, px = static_cast<size_t>(sy) * W + sx;
#pragma unroll
                for (int c = 0; c < C; ++c) v = fmaf(a.G[c * plane + pg], a.X[c * plane + px], v);
            }
        }
        // fixed-order block sum: wave butterflies, then the four waves in order
        v = wave_sum(v);
        if ((t & 63) == 0) red[t >> 6] = v;
        __syncthreads();
        if (t == 0) {
            float* row = a.partial + static_cast<size_t>(a.nrows - a.parts + part) * N * 4;
            row[4 * i + ab] = (red[0] + red[1]) + (red[2] + red[3]);
        }
        return;
    }
    const long i = (static_cast<long>(blockIdx.x) - a.nA) * 4 + (t >> 6);   // wave-uniform
    if (i < border_count(a.H, a.W)) input_border_pixel<C>(a.G, a.taps, a.N, a.H, a.W, i, a.Gprev);
}

hipError_t launch_adjoint_border(int C, const float* G, const float* X, const float* theta_layer, const TapU* taps,
                                 int N, int NS, int H, int W, int hmax, float* partial, int nrows, int parts,
                                 float* Gprev, hipStream_t s) {
    if (N < 1 || N > 32 || parts < 1 || nrows < parts) return hipErrorInvalidValue;
    BorderArgs a{G, X, theta_layer, taps, N, NS, H, W, hmax, parts, 4 * N * parts, nrows, partial, Gprev};
    const long nb = (H <= 2 || W <= 2) ? static_cast<long>(H) * W : 2L * W + 2L * (H - 2);
    const dim3 grid(static_cast<unsigned>(a.nA + (nb + 3) / 4)), block(256);
    if (C == 3)
        hipLaunchKernelGGL(adjoint_border_kernel<3>, grid, block, 0, s, a);
    else if (C == 4)
        hipLaunchKernelGGL(adjoint_border_kernel<4>, grid, block, 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int C>
static hipError_t input_bound(int boundary, const float* G, const TapU* taps, int N, int H, int W, float* Gprev,
                              hipStream_t s) {
    dim3 grid((W + 63) / 64, (H + 3) / 4), block(256);
    if (boundary == DISK_ZERO)
        hipLaunchKernelGGL((adjoint_input_kernel<C, DISK_ZERO>), grid, block, 0, s, G, taps, N, H, W, Gprev);
    else
        hipLaunchKernelGGL((adjoint_input_kernel<C, DISK_CLAMP>), grid, block, 0, s, G, taps, N, H, W, Gprev);
    return hipGetLastError();
}

hipError_t launch_adjoint_input(int C, int boundary, const float* G, const TapU* taps, int N, int H, int W,
                                float* Gprev, hipStream_t s) {
    switch (C) {
        case 1: return input_bound<1>(boundary, G, taps, N, H, W, Gprev, s);
        case 2: return input_bound<2>(boundary, G, taps, N, H, W, Gprev, s);
        case 3: return input_bound<3>(boundary, G, taps, N, H, W, Gprev, s);
        default: return input_bound<4>(boundary, G, taps, N, H, W, Gprev, s);
    }
}

}  // namespace disk
