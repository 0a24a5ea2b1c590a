// Spatially varying sparse filtering by filter-space interpolation (Sec. 4.3,
// Eq. 8-9), one launch per sparse layer (the multi-pass filter of Sec. 4.4).
//
// Per pixel p and layer l:
//   u = clamp(P(p), 0, 1) * (G - 1) per axis, k = min(floor(u), G - 1), t = u - k,
//   Theta(p) = Theta_k + t (Theta_{k+1} - Theta_k)          (1-D; hat weights)
//            = A + s D0 + t D1 + s t D01                    (2-D; bilinear weights)
//   X_l[p] = sum_i w_i(p) B_CLAMP(X_{l-1}, p - o_i(p)).
// With k = min(floor(u), G - 1) and the difference of the last node set to 0,
// every basis node is reproduced exactly (t = 0 there).
//
// Design (gfx950):
// * The basis is turned, once per call, into a coefficient table: per (entry,
//   tap) the negated offset intercepts/slopes and the weight intercept/slope,
//   plus the slope change to the next entry (for waves that straddle a node).
// * A work-group owns a 64 x (4*PY) output tile.  The input tile plus a clamped
//   halo of `halo` pixels is staged in LDS as [row][col][C] FP32 (clamping at
//   staging time removes all per-tap boundary logic).  Each wave owns PY
//   consecutive 64-pixel rows; lanes are consecutive in x, so the gathers of a
//   wave read consecutive LDS words (conflict-free) shifted by the tap offset.
// * P varies slowly, so most 64-pixel rows share one basis interval k: the tap
//   coefficients are then wave-uniform and come from the scalar cache, and the
//   per-pixel interpolation is one FMA per component.  Rows straddling one node
//   use a two-FMA kinked line; anything else reads per-lane coefficients.
// * Blocks map to tiles XCD-contiguously so halo re-reads stay in one L2.
#include "common.hpp"
#include "internal.hpp"

#include <cstdlib>

namespace disk {

constexpr int kRow1D = 9;   // nAx nDx nAy nDy Aw Dw nDDx nDDy DDw
constexpr int kRow2D = 12;  // (nA nD0 nD1 nD01) for x, y; (A D0 D1 D01) for w

size_t sv_table_floats(int dims, int G, int T) {
    // one spare row: the pipelined loop reads (but never uses) the row after the last tap
    return (static_cast<size_t>(G) * T + 1) * (dims == 1 ? kRow1D : kRow2D);
}

struct PrepArgs {
    int dims, G0, G1, T, L;
    int layer_of_tap_start[DISK_MAX_LAYERS + 1];
    int halo[DISK_MAX_LAYERS];
};

__device__ __forceinline__ const float* brow(const float* basis, int T, int entry, int tap) {
    return basis + (static_cast<size_t>(entry) * T + tap) * 3;
}

// One work-group: clears the flag, then fills the table and checks every
// offset against its layer's halo.
__global__ __launch_bounds__(1024) void sv_prep_kernel(PrepArgs a, const float* __restrict__ basis,
                                                       float* __restrict__ table, int* __restrict__ flag) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int G = a.dims == 1 ? a.G0 : a.G0 * a.G1;
    const int n = G * a.T;
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
        const int e = idx / a.T, tap = idx - e * a.T;
        int l = 0;
        while (l + 1 < a.L && tap >= a.layer_of_tap_start[l + 1]) ++l;
        const float lim = static_cast<float>(a.halo[l] - 1);
        const float* A = brow(basis, a.T, e, tap);
        if (!(fabsf(A[0]) <= lim && fabsf(A[1]) <= lim) || !isfinite(A[2])) atomicOr(&bad, 1);
        if (a.dims == 1) {
            const float* B = brow(basis, a.T, min(e + 1, G - 1), tap);
            const float* Cn = brow(basis, a.T, min(e + 2, G - 1), tap);
            float D[3], D2[3];
            for (int j = 0; j < 3; ++j) {
                D[j] = (e + 1 < G) ? B[j] - A[j] : 0.0f;
                D2[j] = (e + 2 < G) ? Cn[j] - B[j] : 0.0f;
            }
            float* r = table + static_cast<size_t>(idx) * kRow1D;
            r[0] = -A[0];
            r[1] = -D[0];
            r[2] = -A[1];
            r[3] = -D[1];
            r[4] = A[2];
            r[5] = D[2];
            r[6] = -(D2[0] - D[0]);
            r[7] = -(D2[1] - D[1]);
            r[8] = D2[2] - D[2];
        } else {
            const int i0 = e / a.G1, i1 = e - i0 * a.G1;
            const bool h0 = i0 + 1 < a.G0, h1 = i1 + 1 < a.G1;
            const float* P10 = brow(basis, a.T, (h0 ? i0 + 1 : i0) * a.G1 + i1, tap);
            const float* P01 = brow(basis, a.T, i0 * a.G1 + (h1 ? i1 + 1 : i1), tap);
            const float* P11 = brow(basis, a.T, (h0 ? i0 + 1 : i0) * a.G1 + (h1 ? i1 + 1 : i1), tap);
            float* r = table + static_cast<size_t>(idx) * kRow2D;
            for (int j = 0; j < 3; ++j) {
                const float sg = j < 2 ? -1.0f : 1.0f;
                const float d0 = h0 ? P10[j] - A[j] : 0.0f;
                const float d1 = h1 ? P01[j] - A[j] : 0.0f;
                const float d01 = (h0 && h1) ? (P11[j] - P10[j]) - (P01[j] - A[j]) : 0.0f;
                r[4 * j + 0] = sg * A[j];
                r[4 * j + 1] = sg * d0;
                r[4 * j + 2] = sg * d1;
                r[4 * j + 3] = sg * d01;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *flag = bad;
}

hipError_t launch_sv_prep(int dims, int G0, int G1, const LayerSpec& spec, const int* halo,
                          const float* basis, float* table, int* flag, hipStream_t s) {
    PrepArgs a{};
    a.dims = dims;
    a.G0 = G0;
    a.G1 = G1;
    a.T = spec.T;
    a.L = spec.L;
    for (int l = 0; l < spec.L; ++l) {
        a.layer_of_tap_start[l] = spec.tap0[l];
        a.halo[l] = halo[l];
    }
    a.layer_of_tap_start[spec.L] = spec.T;
    hipLaunchKernelGGL(sv_prep_kernel, dim3(1), dim3(1024), 0, s, a, basis, table, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the pass kernel
// ---------------------------------------------------------------------------
constexpr int kTW = 64;

// LDS byte offsets <-> LDS pointers (address space 3 pointers are 32-bit offsets).
typedef __attribute__((address_space(3))) float lds_float;
__device__ __forceinline__ int lds_offset(float* p) {
    return static_cast<int>(reinterpret_cast<uintptr_t>((lds_float*)p));
}
__device__ __forceinline__ const lds_float* lds_ptr(int byte_offset) {
    return reinterpret_cast<const lds_float*>(static_cast<uintptr_t>(static_cast<uint32_t>(byte_offset)));
}

// Single-instruction VALU helpers (arithmetic only).
__device__ __forceinline__ int cvt_flr(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
__device__ __forceinline__ int mad24(int a, int b, int c) {
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// Accumulate one tap with per-lane (nx, ny) = -offset and weight w.  `base` is
// the byte address of the pixel's own position in the staged [row][col][C]
// tile; rowB / colB are the byte strides of a row and a column.
template <int C>
__device__ __forceinline__ void gather_tap(float* acc, int base, int rowB, float nx, float ny, float w) {
    const int ix = cvt_flr(nx), iy = cvt_flr(ny);
    const float fx = __builtin_amdgcn_fractf(nx), fy = __builtin_amdgcn_fractf(ny);
    const float wy1 = w * fy, wy0 = w - wy1;
    const float c01 = wy0 * fx, c00 = wy0 - c01;
    const float c11 = wy1 * fx, c10 = wy1 - c11;
    const int a0 = mad24(ix, C * 4, mad24(iy, rowB, base));
    const lds_float* r0 = lds_ptr(a0);
    const lds_float* r1 = lds_ptr(a0 + rowB);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float a = acc[c];
        a = fmaf(c00, r0[c], a);
        a = fmaf(c01, r0[C + c], a);
        a = fmaf(c10, r1[c], a);
        a = fmaf(c11, r1[C + c], a);
        acc[c] = a;
    }
}

template <int C, int DIMS, typename TIn, typename TOut, int PY>
__global__ __launch_bounds__(256, 2) void sv_pass_kernel(
    const TIn* __restrict__ X, TOut* __restrict__ Y, const float* __restrict__ P,
    const float* __restrict__ table, int tap0, int N, int T, int G0, int G1, int H, int W, int halo,
    int tiles_x, int per, int ntiles, const int* __restrict__ flag) {
    extern __shared__ float lds[];
    constexpr int TH = 4 * PY;
    constexpr int RW = DIMS == 1 ? kRow1D : kRow2D;
    const int tile = xcd_tile(blockIdx.x, per);
    if (tile >= ntiles) return;
    const size_t plane = static_cast<size_t>(H) * W;
    const int tx0 = (tile % tiles_x) * kTW, ty0 = (tile / tiles_x) * TH;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int x = tx0 + lane;

    if (*flag) {  // an offset exceeds its declared halo: refuse to gather
        if (x < W)
            for (int j = 0; j < PY; ++j) {
                const int y = ty0 + wave * PY + j;
                if (y < H)
                    for (int c = 0; c < C; ++c)
                        IO<TOut>::store(Y, c * plane + static_cast<size_t>(y) * W + x, __builtin_nanf(""));
            }
        return;
    }

    const int SX = kTW + 2 * halo, SY = TH + 2 * halo;
    const int rowC = SX * C;
    // Stage the tile + clamped halo.  Loads are batched (4 rows x up to 3
    // column chunks x C per lane in flight) before any LDS store, so the
    // memory latency is paid once per batch rather than once per row.
    const int nq = (SX + 63) >> 6;
    for (int r0 = wave; r0 < SY; r0 += 16) {
        float v[4][3][C];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int gy = min(max(ty0 - halo + r0 + 4 * rr, 0), H - 1);
            const size_t grow = static_cast<size_t>(gy) * W;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (q < nq) {
                    const int gx = min(max(tx0 - halo + lane + 64 * q, 0), W - 1);
#pragma unroll
                    for (int c = 0; c < C; ++c) v[rr][q][c] = IO<TIn>::load(X, c * plane + grow + gx);
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int ly = r0 + 4 * rr;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int lx = lane + 64 * q;
                if (q < nq && ly < SY && lx < SX) {
                    float* d = lds + ly * rowC + lx * C;
#pragma unroll
                    for (int c = 0; c < C; ++c) d[c] = v[rr][q][c];
                }
            }
        }
    }

    // decode the parameter map for this lane's PY pixels
    const int xc = min(x, W - 1);
    float ta[PY], tb[PY];
    int kk[PY];
#pragma unroll
    for (int j = 0; j < PY; ++j) {
        const int yc = min(ty0 + wave * PY + j, H - 1);
        const size_t pi = static_cast<size_t>(yc) * W + xc;
        const float u0 = fminf(fmaxf(P[pi], 0.0f), 1.0f) * static_cast<float>(G0 - 1);
        const int k0 = min(static_cast<int>(floorf(u0)), G0 - 1);
        ta[j] = u0 - static_cast<float>(k0);
        if (DIMS == 1) {
            kk[j] = k0;
            tb[j] = u0;  // kept for the two-interval path
        } else {
            const float u1 = fminf(fmaxf(P[plane + pi], 0.0f), 1.0f) * static_cast<float>(G1 - 1);
            const int k1 = min(static_cast<int>(floorf(u1)), G1 - 1);
            tb[j] = u1 - static_cast<float>(k1);
            kk[j] = k0 * G1 + k1;
        }
    }
    __syncthreads();

    const int lds_base = lds_offset(lds);
    const int rowB = rowC * 4;
    int base[PY];
#pragma unroll
    for (int j = 0; j < PY; ++j) base[j] = lds_base + ((wave * PY + j + halo) * rowC + (lane + halo) * C) * 4;
    float acc[PY][C];
#pragma unroll
    for (int j = 0; j < PY; ++j)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[j][c] = 0.0f;

    int lo = kk[0], hi = kk[0];
#pragma unroll
    for (int j = 1; j < PY; ++j) {
        lo = min(lo, kk[j]);
        hi = max(hi, kk[j]);
    }
    const int k0u = uniform(kk[0]);
    const bool same = __all(lo == k0u && hi == k0u);

    if (same) {
        // every pixel of the wave lies in one interval: wave-uniform coefficients
        const float* e = table + (static_cast<size_t>(k0u) * T + tap0) * RW;
        if (DIMS == 1) {
            // software-pipelined: the next tap's scalar coefficients load while
            // this tap computes (the table carries one spare row at its end)
            float Ax = e[0], Dx = e[1], Ay = e[2], Dy = e[3], Aw = e[4], Dw = e[5];
            for (int i = 0; i < N; ++i) {
                const float* r = e + (i + 1) * RW;
                const float nAx = r[0], nDx = r[1], nAy = r[2], nDy = r[3], nAw = r[4], nDw = r[5];
#pragma unroll
                for (int j = 0; j < PY; ++j)
                    gather_tap<C>(acc[j], base[j], rowB, fmaf(ta[j], Dx, Ax), fmaf(ta[j], Dy, Ay), fmaf(ta[j], Dw, Aw));
                Ax = nAx; Dx = nDx; Ay = nAy; Dy = nDy; Aw = nAw; Dw = nDw;
            }
        } else {
        for (int i = 0; i < N; ++i) {
            const float* r = e + i * RW;
            {
#pragma unroll
                for (int j = 0; j < PY; ++j) {
                    const float st = ta[j] * tb[j];
                    const float nx = fmaf(st, r[3], fmaf(tb[j], r[2], fmaf(ta[j], r[1], r[0])));
                    const float ny = fmaf(st, r[7], fmaf(tb[j], r[6], fmaf(ta[j], r[5], r[4])));
                    const float w = fmaf(st, r[11], fmaf(tb[j], r[10], fmaf(ta[j], r[9], r[8])));
                    gather_tap<C>(acc[j], base[j], rowB, nx, ny, w);
                }
            }
        }
        }
    } else {
        const int bmin = wave_min_i(lo), bmax = wave_max_i(hi);
        if (DIMS == 1 && bmax == bmin + 1) {
            // the block straddles one node: kinked line from interval bmin
            const int kb = uniform(bmin);
            float t0[PY], e1[PY];
#pragma unroll
            for (int j = 0; j < PY; ++j) {
                t0[j] = tb[j] - static_cast<float>(kb);
                e1[j] = fmaxf(t0[j] - 1.0f, 0.0f);
            }
            const float* e = table + (static_cast<size_t>(kb) * T + tap0) * RW;
            for (int i = 0; i < N; ++i) {
                const float* r = e + i * RW;
                const float Ax = r[0], Dx = r[1], Ay = r[2], Dy = r[3], Aw = r[4], Dw = r[5];
                const float Ex = r[6], Ey = r[7], Ew = r[8];
#pragma unroll
                for (int j = 0; j < PY; ++j)
                    gather_tap<C>(acc[j], base[j], rowB, fmaf(e1[j], Ex, fmaf(t0[j], Dx, Ax)),
                                  fmaf(e1[j], Ey, fmaf(t0[j], Dy, Ay)), fmaf(e1[j], Ew, fmaf(t0[j], Dw, Aw)));
            }
        } else {
            // general case: per-lane coefficients
            for (int i = 0; i < N; ++i) {
#pragma unroll
                for (int j = 0; j < PY; ++j) {
                    const float* r = table + (static_cast<size_t>(kk[j]) * T + tap0 + i) * RW;
                    if (DIMS == 1) {
                        gather_tap<C>(acc[j], base[j], rowB, fmaf(ta[j], r[1], r[0]), fmaf(ta[j], r[3], r[2]),
                                      fmaf(ta[j], r[5], r[4]));
                    } else {
                        const float st = ta[j] * tb[j];
                        const float nx = fmaf(st, r[3], fmaf(tb[j], r[2], fmaf(ta[j], r[1], r[0])));
                        const float ny = fmaf(st, r[7], fmaf(tb[j], r[6], fmaf(ta[j], r[5], r[4])));
                        const float w = fmaf(st, r[11], fmaf(tb[j], r[10], fmaf(ta[j], r[9], r[8])));
                        gather_tap<C>(acc[j], base[j], rowB, nx, ny, w);
                    }
                }
            }
        }
    }

    if (x < W) {
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            const int y = ty0 + wave * PY + j;
            if (y < H)
#pragma unroll
                for (int c = 0; c < C; ++c) IO<TOut>::store(Y, c * plane + static_cast<size_t>(y) * W + x, acc[j][c]);
        }
    }
}

int sv_rows_per_wave(int halo, int C) {
    // Tuning override (rows per wave: 2, 4, 8 or 16), read once.
    static const int forced = [] {
        const char* e = std::getenv("DISK_SV_ROWS");
        const int v = e ? std::atoi(e) : 0;
        return (v == 2 || v == 4 || v == 8 || v == 16) ? v : 0;
    }();
    if (forced && sv_lds_bytes(halo, C, forced) <= 160 * 1024) return forced;
    // Larger tiles amortise the halo; keep the staged tile within 80 KB so two
    // work-groups share a CU.
    for (int py : {8, 4}) {
        if (sv_lds_bytes(halo, C, py) <= 80 * 1024) return py;
    }
    return 2;
}

size_t sv_lds_bytes(int halo, int C, int py) {
    return static_cast<size_t>(kTW + 2 * halo) * (4 * py + 2 * halo) * C * sizeof(float);
}

template <int C, int DIMS, typename TIn, typename TOut, int PY>
static hipError_t launch_typed(const void* src, void* dst, const float* pmap, const float* table, int tap0,
                               int N, int T, int G0, int G1, int H, int W, int halo, const int* flag,
                               hipStream_t s) {
    const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + 4 * PY - 1) / (4 * PY);
    const int ntiles = tiles_x * tiles_y;
    const int per = (ntiles + 7) / 8;
    const size_t lds = sv_lds_bytes(halo, C, PY);
    auto fn = sv_pass_kernel<C, DIMS, TIn, TOut, PY>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(8 * per), dim3(256), lds, s, static_cast<const TIn*>(src),
                       static_cast<TOut*>(dst), pmap, table, tap0, N, T, G0, G1, H, W, halo, tiles_x, per,
                       ntiles, flag);
    return hipGetLastError();
}

template <int C, int DIMS, int PY>
static hipError_t launch_io(int src_bf16, const void* src, int dst_bf16, void* dst, const float* pmap,
                            const float* table, int tap0, int N, int T, int G0, int G1, int H, int W, int halo,
                            const int* flag, hipStream_t s) {
    if (!src_bf16 && !dst_bf16)
        return launch_typed<C, DIMS, float, float, PY>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
    if (src_bf16 && !dst_bf16)
        return launch_typed<C, DIMS, uint16_t, float, PY>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
    if (!src_bf16 && dst_bf16)
        return launch_typed<C, DIMS, float, uint16_t, PY>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
    return launch_typed<C, DIMS, uint16_t, uint16_t, PY>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
}

template <int C, int DIMS>
static hipError_t launch_py(int src_bf16, const void* src, int dst_bf16, void* dst, const float* pmap,
                            const float* table, int tap0, int N, int T, int G0, int G1, int H, int W, int halo,
                            const int* flag, hipStream_t s) {
    const int py = sv_rows_per_wave(halo, C);
    if (py == 16) return launch_io<C, DIMS, 16>(src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
    if (py == 8) return launch_io<C, DIMS, 8>(src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
    if (py == 4) return launch_io<C, DIMS, 4>(src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
    return launch_io<C, DIMS, 2>(src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
}

template <int C>
static hipError_t launch_dims(int dims, int src_bf16, const void* src, int dst_bf16, void* dst, const float* pmap,
                              const float* table, int tap0, int N, int T, int G0, int G1, int H, int W, int halo,
                              const int* flag, hipStream_t s) {
    if (dims == 1) return launch_py<C, 1>(src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
    return launch_py<C, 2>(src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
}

hipError_t launch_sv_pass(int C, int dims, int src_bf16, const void* src, int dst_bf16, void* dst,
                          const float* pmap, const float* table, int tap0, int N, int T, int G0, int G1,
                          int H, int W, int halo, const int* flag, hipStream_t s) {
    switch (C) {
        case 1: return launch_dims<1>(dims, src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
        case 2: return launch_dims<2>(dims, src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
        case 3: return launch_dims<3>(dims, src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
        default: return launch_dims<4>(dims, src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
    }
}

}  // namespace disk
