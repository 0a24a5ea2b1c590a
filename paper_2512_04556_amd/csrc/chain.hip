// Uniform-Theta sparse layers on images and impulse canvases (Sec. 3.2 Eq. 2-3,
// impulse response Sec. 4.4 Eq. 10).
//
// A layer is Y[p] = sum_i w_i B(X, p - o_i).  Because Theta is spatially
// uniform, each tap's integer corner offset (floor(-o)) and its four bilinear
// corner weights are the same for every pixel: they are prepared once per call
// (TapU) and read through the scalar cache, so the per-pixel work of a tap is
// four reads and 4 FMAs per channel.  Reads go through L1/L2: neighbouring
// lanes read neighbouring addresses for every tap, so each wave's accesses
// coalesce into a few cache lines.
#include "common.hpp"
#include "internal.hpp"

namespace disk {

__global__ void prep_uniform_kernel(const float* __restrict__ theta, int T, TapU* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T) return;
    const float ox = theta[3 * i + 0], oy = theta[3 * i + 1], w = theta[3 * i + 2];
    int ix, iy;
    float fx, fy;
    floor_frac(-ox, ix, fx);
    floor_frac(-oy, iy, fy);
    const float wy1 = w * fy, wy0 = w - wy1;
    TapU t;
    t.ix = ix;
    t.iy = iy;
    t.c01 = wy0 * fx;
    t.c00 = wy0 - t.c01;
    t.c11 = wy1 * fx;
    t.c10 = wy1 - t.c11;
    t.pad0 = t.pad1 = 0;
    out[i] = t;
}

hipError_t launch_prep_uniform(const float* theta, int T, TapU* out, hipStream_t s) {
    hipLaunchKernelGGL(prep_uniform_kernel, dim3((T + 63) / 64), dim3(64), 0, s, theta, T, out);
    return hipGetLastError();
}

// Sources: a stored image (f32 / bf16) or the implicit Dirac impulse.
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

constexpr int kTW = 64;   // tile width (one wave per row)
constexpr int kRows = 4;  // rows per thread
constexpr int kTH = 4 * kRows;

template <int C, int BOUND, class Src, typename TOut>
__global__ __launch_bounds__(256) void layer_uniform_kernel(Src src, TOut* __restrict__ Y,
                                                            const TapU* __restrict__ taps, int N,
                                                            int H, int W, int tiles_x, int per,
                                                            int ntiles) {
    const int tile = xcd_tile(blockIdx.x, per);
    if (tile >= ntiles) return;
    const int x = (tile % tiles_x) * kTW + (threadIdx.x & 63);
    const int yb = (tile / tiles_x) * kTH + (threadIdx.x >> 6) * kRows;
    const size_t plane = static_cast<size_t>(H) * W;
    float acc[kRows][C];
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[r][c] = 0.0f;

    for (int i = 0; i < N; ++i) {
        const TapU t = taps[i];
        int x0 = x + t.ix, x1 = x0 + 1;
        const bool vx0 = x0 >= 0 && x0 < W, vx1 = x1 >= 0 && x1 < W;
        x0 = min(max(x0, 0), W - 1);
        x1 = min(max(x1, 0), W - 1);
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            int y0 = yb + r + t.iy, y1 = y0 + 1;
            const bool vy0 = y0 >= 0 && y0 < H, vy1 = y1 >= 0 && y1 < H;
            y0 = min(max(y0, 0), H - 1);
            y1 = min(max(y1, 0), H - 1);
            const size_t r0 = static_cast<size_t>(y0) * W, r1 = static_cast<size_t>(y1) * W;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float v00 = src.load(c * plane + r0 + x0);
                float v01 = src.load(c * plane + r0 + x1);
                float v10 = src.load(c * plane + r1 + x0);
                float v11 = src.load(c * plane + r1 + x1);
                if (BOUND == DISK_ZERO) {
                    v00 = (vx0 && vy0) ? v00 : 0.0f;
                    v01 = (vx1 && vy0) ? v01 : 0.0f;
                    v10 = (vx0 && vy1) ? v10 : 0.0f;
                    v11 = (vx1 && vy1) ? v11 : 0.0f;
                }
                float a = acc[r][c];
                a = fmaf(t.c00, v00, a);
                a = fmaf(t.c01, v01, a);
                a = fmaf(t.c10, v10, a);
                a = fmaf(t.c11, v11, a);
                acc[r][c] = a;
            }
        }
    }
    if (x >= W) return;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int y = yb + r;
        if (y < H) {
#pragma unroll
            for (int c = 0; c < C; ++c) IO<TOut>::store(Y, c * plane + static_cast<size_t>(y) * W + x, acc[r][c]);
        }
    }
}

template <int C, int BOUND, class Src>
static hipError_t dispatch_dst(Src src, int dst_kind, void* dst, const TapU* taps, int N, int H, int W,
                               hipStream_t s) {
    const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + kTH - 1) / kTH;
    const int ntiles = tiles_x * tiles_y;
    const int per = (ntiles + 7) / 8;
    dim3 grid(8 * per), block(256);
    if (dst_kind == 0)
        hipLaunchKernelGGL((layer_uniform_kernel<C, BOUND, Src, float>), grid, block, 0, s, src,
                           static_cast<float*>(dst), taps, N, H, W, tiles_x, per, ntiles);
    else
        hipLaunchKernelGGL((layer_uniform_kernel<C, BOUND, Src, uint16_t>), grid, block, 0, s, src,
                           static_cast<uint16_t*>(dst), taps, N, H, W, tiles_x, per, ntiles);
    return hipGetLastError();
}

template <int C, int BOUND>
static hipError_t dispatch_src(int src_kind, const void* src, int dst_kind, void* dst, const TapU* taps,
                               int N, int H, int W, hipStream_t s) {
    if (src_kind == 0) return dispatch_dst<C, BOUND>(SrcF32{static_cast<const float*>(src)}, dst_kind, dst, taps, N, H, W, s);
    if (src_kind == 1) return dispatch_dst<C, BOUND>(SrcBF16{static_cast<const uint16_t*>(src)}, dst_kind, dst, taps, N, H, W, s);
    const size_t centre = static_cast<size_t>((H - 1) / 2) * W + (W - 1) / 2;
    return dispatch_dst<C, BOUND>(SrcImpulse{centre}, dst_kind, dst, taps, N, H, W, s);
}

template <int C>
static hipError_t dispatch_bound(int boundary, int src_kind, const void* src, int dst_kind, void* dst,
                                 const TapU* taps, int N, int H, int W, hipStream_t s) {
    if (boundary == DISK_ZERO) return dispatch_src<C, DISK_ZERO>(src_kind, src, dst_kind, dst, taps, N, H, W, s);
    return dispatch_src<C, DISK_CLAMP>(src_kind, src, dst_kind, dst, taps, N, H, W, s);
}

hipError_t launch_layer_uniform(int C, int boundary, int src_kind, const void* src, int dst_kind,
                                void* dst, const TapU* taps, int N, int H, int W, hipStream_t s) {
    switch (C) {
        case 1: return dispatch_bound<1>(boundary, src_kind, src, dst_kind, dst, taps, N, H, W, s);
        case 2: return dispatch_bound<2>(boundary, src_kind, src, dst_kind, dst, taps, N, H, W, s);
        case 3: return dispatch_bound<3>(boundary, src_kind, src, dst_kind, dst, taps, N, H, W, s);
        default: return dispatch_bound<4>(boundary, src_kind, src, dst_kind, dst, taps, N, H, W, s);
    }
}

}  // namespace disk
