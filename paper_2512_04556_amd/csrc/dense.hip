// Dense spatially varying convolution: the per-pixel kernel that the sparse
// filter approximates (Eq. 1 with a kernel chosen per output pixel, Sec. 4.3),
// computed directly as the quality and speed reference.
//
//   out[p] = sum_q K_p[q] I[clamp(p - q)] / sum_q K_p[q],  |qx|, |qy| <= half
//   disk:    K_p[q] = clamp(r + 1/2 - |q|, 0, 1),           r = r0 + (r1 - r0) clamp(P0, 0, 1)
//   ellipse: K_p[q] = clamp(1/2 - (rho - 1) |q| / rho, 0, 1) (rho > 0; clamp(1/2 + min(ax, ay)) at q = 0),
//            rho = |(qx / ax, qy / ay)|, ax = r sqrt(a), ay = r / sqrt(a),
//            a = a0 (a1 / a0)^clamp(P1, 0, 1)
//
// One wave owns 64 consecutive pixels of a row; it visits the window of the
// largest kernel among its pixels (pixels with smaller kernels get zero
// weights there).  Reads go through L1/L2 (the image is re-read by
// neighbouring waves); per tap a pixel costs one weight, C FMAs and C loads.
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace disk {

namespace {

struct DenseArgs {
    int kind, C, H, W, half;
    float r0, r1, a0, a1;
};

template <int C, typename TIn, typename TOut, int KIND>
__global__ __launch_bounds__(256) void dense_sv_kernel(DenseArgs a, const TIn* __restrict__ X,
                                                       const float* __restrict__ P, TOut* __restrict__ Y) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int segs = (a.W + 63) / 64;
    const int y = wave / segs;
    if (y >= a.H) return;
    const int x = (wave - y * segs) * 64 + lane;
    const bool live = x < a.W;
    const int xc = live ? x : a.W - 1;
    const size_t plane = static_cast<size_t>(a.H) * a.W;
    const size_t pix = static_cast<size_t>(y) * a.W + xc;
    const float u0 = fminf(fmaxf(P[pix], 0.0f), 1.0f);
    const float r = a.r0 + (a.r1 - a.r0) * u0;
    float ax = r, ay = r;
    if (KIND == 1) {
        const float u1 = fminf(fmaxf(P[plane + pix], 0.0f), 1.0f);
        const float asp = a.a0 * powf(a.a1 / a.a0, u1);
        const float s = sqrtf(asp);
        ax = r * s;
        ay = r / s;
    }
    // window of this wave: the largest semi-axis among its live pixels, capped at half
    const float reach = live ? fmaxf(ax, ay) + 0.5f : 0.0f;
    const int R = min(a.half, static_cast<int>(ceilf(wave_max(reach))));
    const float iax = 1.0f / ax, iay = 1.0f / ay;
    float acc[C], z = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0f;
    const TIn* Xc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Xc[c] = X + c * plane;
    for (int qy = -R; qy <= R; ++qy) {
        const uint32_t row = static_cast<uint32_t>(min(max(y - qy, 0), a.H - 1)) * static_cast<uint32_t>(a.W);
        const float fqy = static_cast<float>(qy);
        for (int qx0 = -R; qx0 <= R; qx0 += 64) {
            // |q| of the next 64 taps, one per lane, broadcast tap by tap
            const float lqx = static_cast<float>(qx0 + lane);
            const float nql = sqrtf(lqx * lqx + fqy * fqy);
            const int cnt = min(64, R - qx0 + 1);
            for (int k = 0; k < cnt; ++k) {
                const int qx = qx0 + k;
                const float nq = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, nql), k));
                float w;
                if (KIND == 0) {
                    w = fminf(fmaxf(r + 0.5f - nq, 0.0f), 1.0f);
                } else {
                    const float fqx = static_cast<float>(qx);
                    const float ex = fqx * iax, ey = fqy * iay;
                    const float rho = sqrtf(ex * ex + ey * ey);
                    const float d = rho > 0.0f ? (rho - 1.0f) * (nq / rho) : -fminf(ax, ay);
                    w = fminf(fmaxf(0.5f - d, 0.0f), 1.0f);
                }
                const uint32_t off = (row + static_cast<uint32_t>(min(max(xc - qx, 0), a.W - 1))) *
                                     static_cast<uint32_t>(sizeof(TIn));
                z += w;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    acc[c] = fmaf(w, IO<TIn>::load(reinterpret_cast<const TIn*>(reinterpret_cast<const char*>(Xc[c]) + off), 0),
                                  acc[c]);
            }
        }
    }
    if (!live) return;
    const float inv = 1.0f / z;
#pragma unroll
    for (int c = 0; c < C; ++c) IO<TOut>::store(Y, c * plane + pix, acc[c] * inv);
}

template <int C, typename TIn, typename TOut>
hipError_t launch_c(const DenseArgs& a, const void* X, const float* P, void* Y, hipStream_t s) {
    const long waves = static_cast<long>(a.H) * ((a.W + 63) / 64);
    const dim3 grid(static_cast<unsigned>((waves + 3) / 4));
    if (a.kind == 0)
        hipLaunchKernelGGL((dense_sv_kernel<C, TIn, TOut, 0>), grid, dim3(256), 0, s, a,
                           static_cast<const TIn*>(X), P, static_cast<TOut*>(Y));
    else
        hipLaunchKernelGGL((dense_sv_kernel<C, TIn, TOut, 1>), grid, dim3(256), 0, s, a,
                           static_cast<const TIn*>(X), P, static_cast<TOut*>(Y));
    return hipGetLastError();
}

template <typename TIn, typename TOut>
hipError_t launch_t(const DenseArgs& a, const void* X, const float* P, void* Y, hipStream_t s) {
    switch (a.C) {
        case 1: return launch_c<1, TIn, TOut>(a, X, P, Y, s);
        case 2: return launch_c<2, TIn, TOut>(a, X, P, Y, s);
        case 3: return launch_c<3, TIn, TOut>(a, X, P, Y, s);
        default: return launch_c<4, TIn, TOut>(a, X, P, Y, s);
    }
}

}  // namespace

hipError_t launch_dense_sv(int kind, float r0, float r1, float a0, float a1, int half, const void* image,
                           const float* pmap, void* out, int C, int H, int W, int bf16, hipStream_t s) {
    DenseArgs a{kind, C, H, W, half, r0, r1, a0, a1};
    if (bf16) return launch_t<uint16_t, uint16_t>(a, image, pmap, out, s);
    return launch_t<float, float>(a, image, pmap, out, s);
}

}  // namespace disk
