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
// * P varies slowly, so most 16 x 8 wave blocks share one basis interval k: the
//   tap coefficients are then wave-uniform (broadcast LDS reads of the layer's
//   table rows staged after the tile, or the scalar cache where the table does
//   not fit), and the per-pixel interpolation is one FMA per component.  Blocks
//   straddling up to three nodes use a kinked line; anything else reads
//   per-lane coefficients.
// * Blocks map to tiles XCD-contiguously so halo re-reads stay in one L2.
#include "common.hpp"
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <type_traits>

namespace disk {

constexpr int kRow1D = 9;   // nAx nDx nAy nDy Aw Dw nDDx nDDy DDw
constexpr int kRow2D = 12;  // (nA nD0 nD1 nD01) for x, y; (A D0 D1 D01) for w

size_t sv_table_floats(int dims, int G, int T) {
    // spare rows: the chunked loops read (but never use) up to 8 rows past the last tap
    return (static_cast<size_t>(G) * T + 8) * (dims == 1 ? kRow1D : kRow2D);
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

// base + a 32-bit byte offset (lets a load take a scalar base and a 32-bit
// vector offset)
template <typename T>
__device__ __forceinline__ const T* byte_at(const T* base, uint32_t byte_off) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
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
// the byte address of the pixel's own position in the staged tile, laid out
// [row][col][C] with a row stride of rowB bytes.
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

// The same tap for C = 3 or 4 with the tile stored as one float4 per pixel
// (RGB padded, or RGBA): the four corners are four 128-bit LDS reads, the
// widest and fastest LDS access on gfx950.  Floors are taken in FP32 and the
// LDS byte address is formed with two exact FP32 FMAs (integers < 2^24) and one
// conversion, cheaper than integer conversion plus 24-bit multiplies.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) v4f lds_v4f;
typedef __attribute__((address_space(3))) v2f lds_v2f;
__device__ __forceinline__ v4f lds_ld4(int byte_off) {
    return *reinterpret_cast<const lds_v4f*>(static_cast<uintptr_t>(static_cast<uint32_t>(byte_off)));
}
__device__ __forceinline__ v2f lds_ld2(int byte_off) {
    return *reinterpret_cast<const lds_v2f*>(static_cast<uintptr_t>(static_cast<uint32_t>(byte_off)));
}
// ROWB > 0: the row stride is a compile-time constant, so the second row's
// reads take it in their offset field (no address add, and no register reuse
// that would make the second pair wait for the first).
template <int C, int ROWB = 0>
__device__ __forceinline__ void gather_tap4(float* acc, float basef, float rowBf, int rowB, float nx, float ny,
                                            float w) {
    if (ROWB > 0) {
        rowB = ROWB;
        rowBf = static_cast<float>(ROWB);
    }
    const float flx = floorf(nx), fly = floorf(ny);
    const float fx = nx - flx, fy = ny - fly;
    const float wy1 = w * fy, wy0 = w - wy1;
    const float c01 = wy0 * fx, c00 = wy0 - c01;
    const float c11 = wy1 * fx, c10 = wy1 - c11;
    const int a0 = static_cast<int>(fmaf(flx, 16.0f, fmaf(fly, rowBf, basef)));
    const lds_v4f* r0 = reinterpret_cast<const lds_v4f*>(static_cast<uintptr_t>(static_cast<uint32_t>(a0)));
    const lds_v4f* r1 = reinterpret_cast<const lds_v4f*>(static_cast<uintptr_t>(static_cast<uint32_t>(a0 + rowB)));
    const v4f v00 = r0[0], v01 = r0[1], v10 = r1[0], v11 = r1[1];
    const float q00[4] = {v00.x, v00.y, v00.z, v00.w}, q01[4] = {v01.x, v01.y, v01.z, v01.w};
    const float q10[4] = {v10.x, v10.y, v10.z, v10.w}, q11[4] = {v11.x, v11.y, v11.z, v11.w};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float a = acc[c];
        a = fmaf(c00, q00[c], a);
        a = fmaf(c01, q01[c], a);
        a = fmaf(c10, q10[c], a);
        a = fmaf(c11, q11[c], a);
        acc[c] = a;
    }
}

// Staged-tile row stride in dwords: (64 + 2 halo) pixels of C channels, padded
// so that the four 16-lane rows of a wave fall in disjoint LDS banks
// (row stride = 16, 33, 48, 1 mod 64 for C = 1..4).
// LDS row stride of the staged tile.  The LDS has 128 four-byte banks and a
// 128-bit read serves 32 lanes per cycle: two 16-pixel lane rows.  With float4
// pixels the two rows of a pass are conflict-free when their starts are 256 B
// apart modulo 512 B, so the C >= 3 stride is padded to 64 dwords mod 128.
__host__ __device__ __forceinline__ int sv_row_dwords(int halo, int C, bool pad = true) {
    if (C >= 3) {
        const int raw = (kTW + 2 * halo) * 4;
        return pad ? raw + ((64 - raw % 128) + 128) % 128 : raw;
    }
    const int raw = (kTW + 2 * halo) * C;
    const int target = C == 1 ? 16 : C == 2 ? 33 : C == 3 ? 48 : 1;
    return raw + ((target - raw % 64) + 64) % 64;
}

// Lane geometry shared by both pass kernels.  A work-group of NW waves owns a
// 64 x (NW/4 * 4*PY) output tile.  Wave w owns columns [16 (w%4), 16 (w%4) + 16)
// of row band w/4; lane (lx, ly) = (lane & 15, lane >> 4) handles rows 4j + ly,
// j < PY, of its band.  Every per-wave decision (interval span) therefore covers
// a 16 x 4PY block, small enough that a slowly varying map rarely spans a node.

// Decode P for this lane's PY pixels: interval k and the fractions ta (axis 0)
// and tb (axis 1 in 2-D, u itself in 1-D for the multi-interval path).
template <int DIMS, int PY>
__device__ __forceinline__ void sv_decode(const float (&pv)[PY][DIMS], int G0, int G1, float (&ta)[PY],
                                          float (&tb)[PY], int (&kk)[PY]) {
#pragma unroll
    for (int j = 0; j < PY; ++j) {
        const float u0 = fminf(fmaxf(pv[j][0], 0.0f), 1.0f) * static_cast<float>(G0 - 1);
        const int k0 = min(static_cast<int>(floorf(u0)), G0 - 1);
        ta[j] = u0 - static_cast<float>(k0);
        if (DIMS == 1) {
            kk[j] = k0;
            tb[j] = u0;
        } else {
            const float u1 = fminf(fmaxf(pv[j][DIMS - 1], 0.0f), 1.0f) * static_cast<float>(G1 - 1);
            const int k1 = min(static_cast<int>(floorf(u1)), G1 - 1);
            tb[j] = u1 - static_cast<float>(k1);
            kk[j] = k0 * G1 + k1;
        }
    }
}

// Layer table staged in LDS (1-D bases): one 48-byte row per (entry, tap),
// entry-major: nAx nDx nAy nDy | Aw Dw 0 0 | nDDx nDDy DDw 0, plus one zero row
// at the end (the pipelined loops read one row past the last tap).
constexpr int kRowLB = 48;
__host__ __device__ __forceinline__ int sv_ltab_bytes(int G, int N) { return (G * N + 1) * kRowLB; }

// All N taps of one layer for this lane's PY pixels of a staged tile.
// ROWB > 0 fixes the staged row stride at compile time; TL reads the
// coefficients of uniform and straddling waves from the LDS table at byte
// offset tabL (wave-uniform broadcast reads, pipelined one tap ahead) instead
// of the scalar cache.
template <int C, int DIMS, int PY, int ROWB = 0, bool TL = false>
__device__ __forceinline__ void sv_tile_taps(float (&acc)[PY][C], const float (&ta)[PY], const float (&tb)[PY],
                                             const int (&kk)[PY], int base0, int rowB,
                                             const float* __restrict__ table, int tap0, int N, int T,
                                             int tabL = 0) {
    constexpr int RW = DIMS == 1 ? kRow1D : kRow2D;
    if (ROWB > 0) rowB = ROWB;
    const float rowBf = static_cast<float>(rowB);
    float basef[PY];
#pragma unroll
    for (int j = 0; j < PY; ++j) basef[j] = static_cast<float>(base0 + j * 4 * rowB);
#pragma unroll
    for (int j = 0; j < PY; ++j)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[j][c] = 0.0f;
#define SV_TAP(j, nx, ny, w)                                                                       \
    do {                                                                                           \
        if (C >= 3)                                                                                \
            gather_tap4<C, ROWB>(acc[j], basef[j], rowBf, rowB, (nx), (ny), (w));                  \
        else                                                                                       \
            gather_tap<C>(acc[j], base0 + (j) * 4 * rowB, rowB, (nx), (ny), (w));                  \
    } while (0)

    int lo = kk[0], hi = kk[0];
#pragma unroll
    for (int j = 1; j < PY; ++j) {
        lo = min(lo, kk[j]);
        hi = max(hi, kk[j]);
    }
    const int k0u = uniform(kk[0]);
    const bool same = __all(lo == k0u && hi == k0u);

    if constexpr (TL && DIMS == 1) {
        // Every coefficient comes from this layer's LDS rows: row (k, i) at
        // byte tabL + (k N + i) kRowLB.  `table` is not read on this path.
        if (same) {
            // one interval for the whole wave: wave-uniform (broadcast) reads
            int r = uniform(tabL + k0u * N * kRowLB);
            v4f a = lds_ld4(r);
            v2f b = lds_ld2(r + 16);
            for (int i = 0; i < N; ++i) {
                r += kRowLB;
                v4f na = lds_ld4(r);
                v2f nb = lds_ld2(r + 16);
#pragma unroll
                for (int j = 0; j < PY; ++j)
                    SV_TAP(j, fmaf(ta[j], a.y, a.x), fmaf(ta[j], a.w, a.z), fmaf(ta[j], b.y, b.x));
                // the next tap's coefficients are needed only here: keeps their
                // reads ahead of this tap's gathers
                asm volatile("" : "+v"(na), "+v"(nb));
                a = na;
                b = nb;
            }
            return;
        }
        const int bmin = uniform(wave_min_i(lo)), bmax = uniform(wave_max_i(hi));
        const int span = bmax - bmin;
        if (span <= 3) {
            // entry bmin's line plus one hinge per interior node; the slope
            // changes are stored with entries bmin .. bmax - 1 (same tap)
            const int estep = N * kRowLB;
            const int e0 = uniform(tabL + bmin * estep);
            auto hinge_lds = [&](auto span_c) {
                constexpr int SP = decltype(span_c)::value;
                float t0[PY], h[SP][PY];
#pragma unroll
                for (int j = 0; j < PY; ++j) {
                    t0[j] = tb[j] - static_cast<float>(bmin);
#pragma unroll
                    for (int m = 0; m < SP; ++m) h[m][j] = fmaxf(t0[j] - static_cast<float>(m + 1), 0.0f);
                }
                int r = e0;
                for (int i = 0; i < N; ++i, r += kRowLB) {
                    const v4f a = lds_ld4(r);
                    const v2f b = lds_ld2(r + 16);
                    v4f E[SP];
#pragma unroll
                    for (int m = 0; m < SP; ++m) E[m] = lds_ld4(r + m * estep + 32);
#pragma unroll
                    for (int j = 0; j < PY; ++j) {
                        float nx = fmaf(t0[j], a.y, a.x), ny = fmaf(t0[j], a.w, a.z), w = fmaf(t0[j], b.y, b.x);
#pragma unroll
                        for (int m = 0; m < SP; ++m) {
                            nx = fmaf(h[m][j], E[m].x, nx);
                            ny = fmaf(h[m][j], E[m].y, ny);
                            w = fmaf(h[m][j], E[m].z, w);
                        }
                        SV_TAP(j, nx, ny, w);
                    }
                }
            };
            if (span == 1)
                hinge_lds(std::integral_constant<int, 1>{});
            else if (span == 2)
                hinge_lds(std::integral_constant<int, 2>{});
            else
                hinge_lds(std::integral_constant<int, 3>{});
            return;
        }
        // any other wave: per-lane rows (kk[j] <= G - 1, so inside the table)
        for (int i = 0; i < N; ++i) {
#pragma unroll
            for (int j = 0; j < PY; ++j) {
                const int r = tabL + (kk[j] * N + i) * kRowLB;
                const v4f a = lds_ld4(r);
                const v2f b = lds_ld2(r + 16);
                SV_TAP(j, fmaf(ta[j], a.y, a.x), fmaf(ta[j], a.w, a.z), fmaf(ta[j], b.y, b.x));
            }
        }
        return;
    }

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
                    SV_TAP(j, fmaf(ta[j], Dx, Ax), fmaf(ta[j], Dy, Ay), fmaf(ta[j], Dw, Aw));
                Ax = nAx; Dx = nDx; Ay = nAy; Dy = nDy; Aw = nAw; Dw = nDw;
            }
        } else {
            for (int i = 0; i < N; ++i) {
                const float* r = e + i * RW;
#pragma unroll
                for (int j = 0; j < PY; ++j) {
                    const float st = ta[j] * tb[j];
                    const float nx = fmaf(st, r[3], fmaf(tb[j], r[2], fmaf(ta[j], r[1], r[0])));
                    const float ny = fmaf(st, r[7], fmaf(tb[j], r[6], fmaf(ta[j], r[5], r[4])));
                    const float w = fmaf(st, r[11], fmaf(tb[j], r[10], fmaf(ta[j], r[9], r[8])));
                    SV_TAP(j, nx, ny, w);
                }
            }
        }
        return;
    }
    const int bmin = uniform(wave_min_i(lo)), bmax = uniform(wave_max_i(hi));
    const int span = bmax - bmin;
    if (DIMS == 1 && span <= 3) {
        // The block straddles `span` nodes: the piecewise-linear Theta(u) over
        // intervals bmin..bmax is the line of interval bmin plus one hinge
        // max(0, u - m) (D_m - D_{m-1}) per interior node m.
        const float* e = table + (static_cast<size_t>(bmin) * T + tap0) * RW;
        const size_t step = static_cast<size_t>(T) * RW;
        auto hinge_loop = [&](auto span_c) {
            constexpr int SP = decltype(span_c)::value;
            float t0[PY], h[SP][PY];
#pragma unroll
            for (int j = 0; j < PY; ++j) {
                t0[j] = tb[j] - static_cast<float>(bmin);
#pragma unroll
                for (int m = 0; m < SP; ++m) h[m][j] = fmaxf(t0[j] - static_cast<float>(m + 1), 0.0f);
            }
            for (int i = 0; i < N; ++i) {
                const float* r = e + i * RW;
                const float Ax = r[0], Dx = r[1], Ay = r[2], Dy = r[3], Aw = r[4], Dw = r[5];
                float Ex[SP], Ey[SP], Ew[SP];
#pragma unroll
                for (int m = 0; m < SP; ++m) {
                    Ex[m] = r[m * step + 6];
                    Ey[m] = r[m * step + 7];
                    Ew[m] = r[m * step + 8];
                }
#pragma unroll
                for (int j = 0; j < PY; ++j) {
                    float nx = fmaf(t0[j], Dx, Ax), ny = fmaf(t0[j], Dy, Ay), w = fmaf(t0[j], Dw, Aw);
#pragma unroll
                    for (int m = 0; m < SP; ++m) {
                        nx = fmaf(h[m][j], Ex[m], nx);
                        ny = fmaf(h[m][j], Ey[m], ny);
                        w = fmaf(h[m][j], Ew[m], w);
                    }
                    SV_TAP(j, nx, ny, w);
                }
            }
        };
        if (span == 1)
            hinge_loop(std::integral_constant<int, 1>{});
        else if (span == 2)
            hinge_loop(std::integral_constant<int, 2>{});
        else
            hinge_loop(std::integral_constant<int, 3>{});
        return;
    }
    // general case: per-lane coefficients, all rows' loads in flight together
    for (int i = 0; i < N; ++i) {
        float rr[PY][RW];
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            const float* r = table + (static_cast<size_t>(kk[j]) * T + tap0 + i) * RW;
#pragma unroll
            for (int q = 0; q < RW; ++q) rr[j][q] = r[q];
        }
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            const float* r = rr[j];
            if (DIMS == 1) {
                SV_TAP(j, fmaf(ta[j], r[1], r[0]), fmaf(ta[j], r[3], r[2]), fmaf(ta[j], r[5], r[4]));
            } else {
                const float st = ta[j] * tb[j];
                const float nx = fmaf(st, r[3], fmaf(tb[j], r[2], fmaf(ta[j], r[1], r[0])));
                const float ny = fmaf(st, r[7], fmaf(tb[j], r[6], fmaf(ta[j], r[5], r[4])));
                const float w = fmaf(st, r[11], fmaf(tb[j], r[10], fmaf(ta[j], r[9], r[8])));
                SV_TAP(j, nx, ny, w);
            }
        }
    }
#undef SV_TAP
}

// Store one staged pixel (C channels) into the LDS tile.
template <int C>
__device__ __forceinline__ void sv_put(float* lds, int rowW, int ly, int cx, const float (&v)[C]) {
    if (C >= 3) {
        reinterpret_cast<float4*>(lds + ly * rowW)[cx] = make_float4(v[0], v[1], v[2], C == 4 ? v[C - 1] : 0.0f);
    } else {
        float* d = lds + ly * rowW + cx * C;
#pragma unroll
        for (int c = 0; c < C; ++c) d[c] = v[c];
    }
}

template <int C, typename TOut, int PY>
__device__ __forceinline__ void sv_store(TOut* __restrict__ Y, size_t plane, int W, int H, int x, int y0,
                                         const float (&acc)[PY][C]) {
    if (x >= W) return;
#pragma unroll
    for (int j = 0; j < PY; ++j) {
        const int y = y0 + 4 * j;
        if (y < H) {
            const uint32_t off = (static_cast<uint32_t>(y) * static_cast<uint32_t>(W) + static_cast<uint32_t>(x)) *
                                 static_cast<uint32_t>(sizeof(TOut));
#pragma unroll
            for (int c = 0; c < C; ++c)
                IO<TOut>::store(const_cast<TOut*>(byte_at(Y + c * plane, off)), 0, acc[j][c]);
        }
    }
}

// General pass kernel: one tile per work-group, any halo up to 64.
template <int C, int DIMS, typename TIn, typename TOut, int PY, int NW>
__global__ __launch_bounds__(64 * NW) void sv_pass_kernel(
    const TIn* __restrict__ X, TOut* __restrict__ Y, const float* __restrict__ P,
    const float* __restrict__ table, int tap0, int N, int T, int G0, int G1, int H, int W, int halo,
    int tiles_x, int per, int ntiles, const int* __restrict__ flag, int rowW) {
    extern __shared__ float lds[];
    constexpr int TH = 4 * PY * (NW / 4);
    const int tile = xcd_tile(blockIdx.x, per);
    if (tile >= ntiles) return;
    const size_t plane = static_cast<size_t>(H) * W;
    const int tx0 = (tile % tiles_x) * kTW, ty0 = (tile / tiles_x) * TH;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = ((wave & 3) << 4) + (lane & 15), lyb = (wave >> 2) * 4 * PY + (lane >> 4);
    const int x = tx0 + lx;

    if (*flag) {  // an offset exceeds its declared halo: refuse to gather
        float nan[PY][C];
        for (int j = 0; j < PY; ++j)
            for (int c = 0; c < C; ++c) nan[j][c] = __builtin_nanf("");
        sv_store<C, TOut, PY>(Y, plane, W, H, x, ty0 + lyb, nan);
        return;
    }

    const int SX = kTW + 2 * halo, SY = TH + 2 * halo;
    // decode loads first: their latency overlaps the staging below
    const int xc = min(x, W - 1);
    float pv[PY][DIMS];
#pragma unroll
    for (int j = 0; j < PY; ++j) {
        const size_t pi = static_cast<size_t>(min(ty0 + 4 * j + lyb, H - 1)) * W + xc;
#pragma unroll
        for (int d = 0; d < DIMS; ++d) pv[j][d] = P[d * plane + pi];
    }
    // Stage the tile + clamped halo, loads batched (4 rows x up to 3 column
    // chunks x C per lane in flight) before the LDS stores.
    const int nq = (SX + 63) >> 6;
    for (int r0 = wave; r0 < SY; r0 += 4 * NW) {
        float v[4][3][C];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int gy = min(max(ty0 - halo + r0 + NW * rr, 0), H - 1);
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
            const int ly = r0 + NW * rr;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int cx = lane + 64 * q;
                if (q < nq && ly < SY && cx < SX) sv_put<C>(lds, rowW, ly, cx, v[rr][q]);
            }
        }
    }
    float ta[PY], tb[PY];
    int kk[PY];
    sv_decode<DIMS, PY>(pv, G0, G1, ta, tb, kk);
    __syncthreads();

    const int rowB = rowW * 4;
    constexpr int PXB = C >= 3 ? 16 : 4 * C;  // bytes per staged pixel
    const int base0 = lds_offset(lds) + (lyb + halo) * rowB + (lx + halo) * PXB;
    float acc[PY][C];
    sv_tile_taps<C, DIMS, PY>(acc, ta, tb, kk, base0, rowB, table, tap0, N, T);
    sv_store<C, TOut, PY>(Y, plane, W, H, x, ty0 + lyb, acc);
}

// Persistent, software-pipelined pass kernel (halo <= kPipeHalo): each
// work-group walks a contiguous run of tiles of its XCD; while it gathers from
// the tile in LDS, the next tile's inputs and parameter values are already in
// flight into registers, so HBM/L2 latency overlaps the gather.  16 waves,
// 2 row-steps per wave: a 64 x 32 tile.
constexpr int kPipeHalo = 24;
#ifndef DISK_SV_HALO8
#define DISK_SV_HALO8 12
#endif
constexpr int kPipeHalo8 = DISK_SV_HALO8;   // 8-wave variant
constexpr int kPipePY = 2;
// Halos 25..30 (2-D bases with a wide layer): 8-wave 64 x 16 tiles, one per
// CU, two waves per SIMD (the 74-76 staged rows take 60 staging registers),
// row stride 124 pixels (no bank padding: it would not fit the LDS).
constexpr int kPipeHaloWide = 30;
constexpr int kPipeRowBWide = (kTW + 2 * kPipeHaloWide) * 16;
// C <= 2 (and the plane groups of a C >= 3 image whose halo is beyond the
// staged C >= 3 kernels): 16-wave 64 x 32 tiles up to halo 42 (at C = 2 the
// 116 staged rows of 8-byte pixels take 160 KB of LDS).
constexpr int kPipeHaloBig = 42;
template <int NW, int HMAX>
struct PipeShape {
    static constexpr int TH = 4 * kPipePY * (NW / 4);                     // tile rows
    static constexpr int RPW = (TH + 2 * HMAX + NW - 1) / NW;              // staged rows per wave
    static constexpr int NQ = (kTW + 2 * HMAX + 63) / 64;                  // 64-column chunks
    static constexpr int WPE = NW < 16 && HMAX > kPipeHalo ? 2 : 4;       // waves per SIMD
};

// Staging registers of the pipelined kernel hold what each load returned,
// untouched until the LDS store: arithmetic on a loaded value (the BF16
// widening, the zero select outside the image) would make the compiler wait
// for that load inside the prefetch, before the gathers it should overlap.
template <typename T>
struct Staged {
    using type = float;
    __device__ __forceinline__ static float load(const float* p) { return *p; }
    __device__ __forceinline__ static float widen(float v) { return v; }
};
template <>
struct Staged<uint16_t> {
    using type = uint32_t;
    __device__ __forceinline__ static uint32_t load(const uint16_t* p) { return *p; }
    __device__ __forceinline__ static float widen(uint32_t v) { return __uint_as_float(v << 16); }
};

// Uniform chain layer whose offsets exceed the staged halo (or are not
// finite): the work-group's tiles with corners read straight from the clamped
// source planes, in the staged path's arithmetic and order.
// tr: the transposed layer (offsets negated, reads outside the image are 0).
template <int C, typename TIn, typename TOut, int PY, int TH>
__device__ __forceinline__ void chain_tiles_global(const TIn* __restrict__ X, TOut* __restrict__ Y, const float* __restrict__ raw,
                                   int tap0, int N, int H, int W, int tile, int tend, int nwg, int tiles_x, int lx,
                                   int lyb, bool tr) {
    const size_t plane = static_cast<size_t>(H) * W;
    for (; tile < tend; tile += nwg) {
        const int x = (tile % tiles_x) * kTW + lx, y0 = (tile / tiles_x) * TH + lyb;
        float acc[PY][C];
#pragma unroll
        for (int j = 0; j < PY; ++j)
#pragma unroll
            for (int c = 0; c < C; ++c) acc[j][c] = 0.0f;
        for (int i = 0; i < N; ++i) {
            const float* r = raw + static_cast<size_t>(tap0 + i) * 3;
            const float nx = tr ? r[0] : -r[0], ny = tr ? r[1] : -r[1], w = r[2];
            const float flx = floorf(nx), fly = floorf(ny);
            const float fx = nx - flx, fy = ny - fly;
            const float wy1 = w * fy, wy0 = w - wy1;
            const float c01 = wy0 * fx, c00 = wy0 - c01;
            const float c11 = wy1 * fx, c10 = wy1 - c11;
            // integer parts bounded before conversion (a non-finite offset
            // still reads in bounds; its NaN weights carry to the output)
            const int dx = static_cast<int>(fminf(fmaxf(flx, -1048576.0f), 1048576.0f));
            const int dy = static_cast<int>(fminf(fmaxf(fly, -1048576.0f), 1048576.0f));
            const int xa = min(max(x + dx, 0), W - 1), xb = min(max(x + dx + 1, 0), W - 1);
            // ZERO reads (tr): a corner outside the image contributes 0
            const bool ia = !tr || (x + dx >= 0 && x + dx < W), ib = !tr || (x + dx + 1 >= 0 && x + dx + 1 < W);
#pragma unroll
            for (int j = 0; j < PY; ++j) {
                const int y = y0 + 4 * j;
                const size_t ra = static_cast<size_t>(min(max(y + dy, 0), H - 1)) * W;
                const size_t rb = static_cast<size_t>(min(max(y + dy + 1, 0), H - 1)) * W;
                const bool ja = !tr || (y + dy >= 0 && y + dy < H), jb = !tr || (y + dy + 1 >= 0 && y + dy + 1 < H);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const size_t o = c * plane;
                    float a = acc[j][c];
                    a = fmaf(c00, (ja && ia) ? IO<TIn>::load(X, o + ra + xa) : 0.0f, a);
                    a = fmaf(c01, (ja && ib) ? IO<TIn>::load(X, o + ra + xb) : 0.0f, a);
                    a = fmaf(c10, (jb && ia) ? IO<TIn>::load(X, o + rb + xa) : 0.0f, a);
                    a = fmaf(c11, (jb && ib) ? IO<TIn>::load(X, o + rb + xb) : 0.0f, a);
                    acc[j][c] = a;
                }
            }
        }
        sv_store<C, TOut, PY>(Y, plane, W, H, x, y0, acc);
    }
}

// Tap correlations S_ab = sum_p sum_c G[c][p] X[c][map(p + d_ab)] of a chunk
// of <= kCorrTaps uniform taps (the tap gradients of a chain layer), for the
// PY pixels of a lane, added to s.  ZR: reads outside the image are 0, else
// clamped.  Direct global reads: the path for offsets beyond the staged halo.
constexpr int kCorrTaps = 8;
template <int C, typename TIn, int PY, int TH, bool ZR>
__device__ __forceinline__ void corr_tiles_global(const TIn* __restrict__ X, const float* __restrict__ G,
                                  const float* __restrict__ raw, int tap0, int N, int H, int W, int tile, int tend,
                                  int nwg, int tiles_x, int lx, int lyb, float (&s)[kCorrTaps][4]) {
    const size_t plane = static_cast<size_t>(H) * W;
    for (; tile < tend; tile += nwg) {
        const int x = (tile % tiles_x) * kTW + lx, y0 = (tile / tiles_x) * TH + lyb;
        float g[PY][C];
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            const int y = y0 + 4 * j;
            const bool in = x < W && y < H;
#pragma unroll
            for (int c = 0; c < C; ++c) g[j][c] = in ? G[c * plane + static_cast<size_t>(y) * W + x] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < kCorrTaps; ++i) {
            if (i < N) {
                const float* r = raw + static_cast<size_t>(tap0 + i) * 3;
                const float flx = floorf(-r[0]), fly = floorf(-r[1]);
                const int dx = static_cast<int>(fminf(fmaxf(flx, -1048576.0f), 1048576.0f));
                const int dy = static_cast<int>(fminf(fmaxf(fly, -1048576.0f), 1048576.0f));
#pragma unroll
                for (int j = 0; j < PY; ++j) {
                    const int y = y0 + 4 * j;
#pragma unroll
                    for (int ab = 0; ab < 4; ++ab) {
                        const int cx = x + dx + (ab & 1), cy = y + dy + (ab >> 1);
                        const bool ok = !ZR || (cx >= 0 && cx < W && cy >= 0 && cy < H);
                        const size_t o = static_cast<size_t>(min(max(cy, 0), H - 1)) * W + min(max(cx, 0), W - 1);
                        float v = s[i][ab];
#pragma unroll
                        for (int c = 0; c < C; ++c) v = fmaf(g[j][c], ok ? IO<TIn>::load(X, c * plane + o) : 0.0f, v);
                        s[i][ab] = v;
                    }
                }
            }
        }
    }
}

// Work-group sum of s (wave butterflies, then waves in order) into
// part[(blockIdx.x * pN + pofs + i) * 4 + ab]; red: >= NW * kCorrTaps * 4 floats of LDS.
template <int NW>
__device__ __forceinline__ void corr_block_reduce(float (&s)[kCorrTaps][4], int N, float* red, float* __restrict__ part, int pN,
                                  int pofs) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < kCorrTaps; ++i)
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
            const float v = wave_sum(s[i][ab]);
            if (lane == 0) red[(wave * kCorrTaps + i) * 4 + ab] = v;
        }
    __syncthreads();
    if (threadIdx.x < 4 * N) {
        const int i = threadIdx.x >> 2, ab = threadIdx.x & 3;
        float v = 0.0f;
        for (int w = 0; w < NW; ++w) v += red[(w * kCorrTaps + i) * 4 + ab];
        part[(static_cast<size_t>(blockIdx.x) * pN + pofs + i) * 4 + ab] = v;
    }
}

// Staged tap correlations of one tile: the chunk's taps (LDS rows, t = 0:
// -o = (nAx, nAy)) read their four corners from the tile for the lane's PY
// pixels, weighted by the pixel's gradient over the channels.
template <int C, int PY, int ROWB>
__device__ __forceinline__ void corr_tile_taps(float (&s)[kCorrTaps][4], const float (&g)[PY][C], int base0, int tabL,
                                               int N) {
    float basef[PY];
#pragma unroll
    for (int j = 0; j < PY; ++j) basef[j] = static_cast<float>(base0 + j * 4 * ROWB);
#pragma unroll
    for (int i = 0; i < kCorrTaps; ++i) {
        if (i < N) {
            const v4f a = lds_ld4(tabL + i * kRowLB);
            const float flx = floorf(a.x), fly = floorf(a.z);
#pragma unroll
            for (int j = 0; j < PY; ++j) {
                const int a0 = static_cast<int>(fmaf(flx, 16.0f, fmaf(fly, static_cast<float>(ROWB), basef[j])));
                const v4f v[4] = {lds_ld4(a0), lds_ld4(a0 + 16), lds_ld4(a0 + ROWB), lds_ld4(a0 + ROWB + 16)};
#pragma unroll
                for (int ab = 0; ab < 4; ++ab) {
                    float t = s[i][ab];
#pragma unroll
                    for (int c = 0; c < C; ++c) t = fmaf(g[j][c], v[ab][c], t);
                    s[i][ab] = t;
                }
            }
        }
    }
}

// Staged transposed gather fused with the tap correlations (modes 5 and 6).
// The tile holds G (zero outside the image).  For tap i with d = floor(-o_i)
// and the forward's corner weights c_ab, the exact ZERO transpose is
// G'(q) = sum_i sum_ab c_ab G(q - d - ab), and the same four values give the
// part of S_ab(i) = sum_p G(p) X(p + d + ab) whose samples stay in the image:
// with q = p + d + ab it is sum_q X(q) G(q - d - ab) (X at the lane's pixels,
// zero outside the image).  All N taps enter G', the first NS <= kCorrTaps
// taps the sums.
template <int C, int PY, int ROWB>
__device__ __forceinline__ void fused_tile_taps(float (&s)[kCorrTaps][4], float (&acc)[PY][C],
                                                const float (&xq)[PY][C], int base0, int tabL, int N, int NS) {
    float basef[PY];
#pragma unroll
    for (int j = 0; j < PY; ++j) {
        basef[j] = static_cast<float>(base0 + j * 4 * ROWB);
#pragma unroll
        for (int c = 0; c < C; ++c) acc[j][c] = 0.0f;
    }
    // tap i: its weights, then for each of the lane's pixels the four G corners
    // (corner (1, 1) = q - d - (1, 1); (0, 1) one pixel right, (1, 0) one row
    // down), G' accumulated; `sum(j, q00, q01, q10, q11)` takes the corners
    auto tap = [&](int i, auto&& sum) {
        const v4f a = lds_ld4(tabL + i * kRowLB);
        const v2f b = lds_ld2(tabL + i * kRowLB + 16);
        const float flx = floorf(a.x), fly = floorf(a.z);
        const float fx = a.x - flx, fy = a.z - fly, w = b.x;
        const float wy1 = w * fy, wy0 = w - wy1;
        const float c01 = wy0 * fx, c00 = wy0 - c01;
        const float c11 = wy1 * fx, c10 = wy1 - c11;
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            const int a0 =
                static_cast<int>(fmaf(-1.0f - flx, 16.0f, fmaf(-1.0f - fly, static_cast<float>(ROWB), basef[j])));
            const v4f g11 = lds_ld4(a0), g10 = lds_ld4(a0 + 16), g01 = lds_ld4(a0 + ROWB),
                      g00 = lds_ld4(a0 + ROWB + 16);
            const float q00[4] = {g00.x, g00.y, g00.z, g00.w}, q01[4] = {g01.x, g01.y, g01.z, g01.w};
            const float q10[4] = {g10.x, g10.y, g10.z, g10.w}, q11[4] = {g11.x, g11.y, g11.z, g11.w};
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float v = acc[j][c];
                v = fmaf(c00, q00[c], v);
                v = fmaf(c01, q01[c], v);
                v = fmaf(c10, q10[c], v);
                v = fmaf(c11, q11[c], v);
                acc[j][c] = v;
            }
            sum(j, q00, q01, q10, q11);
        }
    };
    // the first kCorrTaps taps: sums of the first NS in registers (the loop is
    // unrolled, so the sums' indices are fixed)
#pragma unroll
    for (int i = 0; i < kCorrTaps; ++i) {
        if (i < N) {
            const bool sums = i < NS;
            tap(i, [&](int j, const float (&q00)[4], const float (&q01)[4], const float (&q10)[4],
                       const float (&q11)[4]) {
                if (sums) {
                    float t0 = s[i][0], t1 = s[i][1], t2 = s[i][2], t3 = s[i][3];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        t0 = fmaf(xq[j][c], q00[c], t0);
                        t1 = fmaf(xq[j][c], q01[c], t1);
                        t2 = fmaf(xq[j][c], q10[c], t2);
                        t3 = fmaf(xq[j][c], q11[c], t3);
                    }
                    s[i][0] = t0, s[i][1] = t1, s[i][2] = t2, s[i][3] = t3;
                }
            });
        }
    }
    for (int i = kCorrTaps; i < N; ++i)
        tap(i, [](int, const float (&)[4], const float (&)[4], const float (&)[4], const float (&)[4]) {});
}

// ROWB > 0 (C >= 3): the staged row stride in bytes, fixed at compile time
// (rowW is then ROWB / 4).  TL (1-D bases): the layer's coefficient rows are
// staged in LDS after the tile, at byte offset SY * rowB.
// MODE 0: a spatially varying pass.  MODE 1 (TL, raw = Theta, G0 = 1, P ==
// nullptr): one layer of a uniform chain.  MODE 2: that layer's transpose.
template <int C, int DIMS, typename TIn, typename TOut, int NW, int HMAX, int ROWB, bool TL, int MODE = 0>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(PipeShape<NW, HMAX>::WPE,
                                                                           PipeShape<NW, HMAX>::WPE))) void
sv_pass_pipe_kernel(
    const TIn* __restrict__ X, TOut* __restrict__ Y, const float* __restrict__ P,
    const float* __restrict__ table, int tap0, int N, int T, int G0, int G1, int H, int W, int halo,
    int tiles_x, int per, int ntiles, const int* __restrict__ flag, int rowW, const float* __restrict__ raw,
    int pN, int pofs, float* __restrict__ part, int ntf, int pfs) {
    // Frames: tiles run over F stacked frames of C planes each (ntiles = F
    // ntf); a tile's frame is tile / ntf.  The parameter map is shared by
    // every frame (pfs = 0) or one per frame (pfs = DIMS planes apart).
    extern __shared__ float lds[];
    if (ROWB > 0) rowW = ROWB / 4;
    constexpr int PY = kPipePY;
    constexpr int TH = PipeShape<NW, HMAX>::TH;
    constexpr int kPipeRPW = PipeShape<NW, HMAX>::RPW, kPipeNQ = PipeShape<NW, HMAX>::NQ;
    const int xcd = blockIdx.x & 7, nwg = gridDim.x >> 3;
    const int tend = min((xcd + 1) * per, ntiles);
    int tile = xcd * per + (blockIdx.x >> 3);
    // MODE 3, 4: tap correlations of a chain layer (CLAMP / ZERO): X = the
    // layer input, P = G (its output gradient), Y = the partial sums
    // [grid][pN][4]; taps tap0 .. tap0 + N - 1 (N <= kCorrTaps) are entries
    // pofs .. pofs + N - 1 of the layer.
    // MODE 5, 6: the transpose of a chain layer (G' into Y; X = G, P = the
    // layer input) fused with the in-image part of its tap correlations (for
    // the first min(N, kCorrTaps) taps, into part [grid][pN][4]); the forward
    // boundary is CLAMP (5) or ZERO (6): it only matters in the fallback.
    constexpr bool corr = MODE >= 3, fused = MODE >= 5;
    float s[kCorrTaps][4];
    if constexpr (corr) {
#pragma unroll
        for (int i = 0; i < kCorrTaps; ++i)
#pragma unroll
            for (int ab = 0; ab < 4; ++ab) s[i][ab] = 0.0f;
    }
    auto corr_finish = [&]() {
        if constexpr (corr) {
            __syncthreads();   // the LDS is free again
            if constexpr (fused)
                corr_block_reduce<NW>(s, min(N, kCorrTaps), lds, part, pN, pofs);
            else
                corr_block_reduce<NW>(s, N, lds, reinterpret_cast<float*>(Y), pN, pofs);
        }
    };
    if (tile >= tend) {
        corr_finish();
        return;
    }
    const size_t plane = static_cast<size_t>(H) * W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = ((wave & 3) << 4) + (lane & 15), lyb = (wave >> 2) * 4 * PY + (lane >> 4);

    // Chain layers (MODE 1, 2): no parameter map (every pixel at k = 0, t = 0);
    // the transpose (MODE 2) negates the offsets and stages the tile with zeros
    // outside the image (the input adjoint away from CLAMP-border pixels).  The
    // halo comes from the layer's own taps (every wave reads the N <= 32 taps):
    // ceil(max |offset|) + 1; beyond HMAX the tiles take the global path.
    constexpr bool chain = MODE != 0, trans = MODE == 2, zstage = MODE == 2 || MODE == 4 || MODE >= 5;
    if constexpr (TL && chain) {
        float m = 0.0f;
        if (lane < N) {
            const float* r = raw + static_cast<size_t>(tap0 + lane) * 3;
            m = fmaxf(fabsf(r[0]), fabsf(r[1]));
            if (!(m <= 1.0e6f)) m = 1.0e6f;    // non-finite or huge
        }
        halo = uniform(static_cast<int>(ceilf(wave_max(m))) + 1);
        if (halo > HMAX) {
            if constexpr (fused) {
                // the transpose as mode 2 does, the correlations (in-image and
                // border samples alike) as mode 3 or 4 does
                chain_tiles_global<C, TIn, TOut, PY, TH>(X, Y, raw, tap0, N, H, W, tile, tend, nwg, tiles_x, lx,
                                                         lyb, true);
                corr_tiles_global<C, TIn, PY, TH, MODE == 6>(reinterpret_cast<const TIn*>(P),
                                                             reinterpret_cast<const float*>(X), raw, tap0,
                                                             min(N, kCorrTaps), H, W, tile, tend, nwg, tiles_x,
                                                             lx, lyb, s);
                corr_finish();
            } else if constexpr (corr) {
                corr_tiles_global<C, TIn, PY, TH, zstage>(X, P, raw, tap0, N, H, W, tile, tend, nwg, tiles_x, lx, lyb,
                                                          s);
                corr_finish();
            } else {
                chain_tiles_global<C, TIn, TOut, PY, TH>(X, Y, raw, tap0, N, H, W, tile, tend, nwg, tiles_x, lx,
                                                         lyb, trans);
            }
            return;
        }
    }

    const int SX = kTW + 2 * halo, SY = TH + 2 * halo;
    const int rowB = rowW * 4;
    constexpr int PXB = C >= 3 ? 16 : 4 * C;
    const int base0 = lds_offset(lds) + (lyb + halo) * rowB + (lx + halo) * PXB;
    const int wv = uniform(wave);                // the wave index, in a scalar register
    const int nq = (SX + 63) >> 6;               // <= kPipeNQ
    const int tabL = lds_offset(lds) + SY * rowB;
    // raw == nullptr: the prepared table and its flag (set when an offset
    // exceeds its declared halo).  raw != nullptr (TL only): the basis itself;
    // this layer's rows are derived here with the same arithmetic as the table
    // preparation, and its offsets checked against this layer's halo.
    int bad = raw ? 0 : *flag;
    if (TL) {
        // this layer's rows of the coefficient table -> LDS (visible after the
        // first barrier below); the extra last row is zero
        const int nrow = G0 * N;
        const float lim = static_cast<float>(halo - 1);
        int mine = 0;
        for (int r = threadIdx.x; r <= nrow; r += 64 * NW) {
            v4f q0 = {0.0f, 0.0f, 0.0f, 0.0f}, q1 = q0, q2 = q0;
            if (r < nrow) {
                const int k = r / N, i = r - k * N;
                if (raw) {
                    const int tap = tap0 + i;
                    const float* A = raw + (static_cast<size_t>(k) * T + tap) * 3;
                    const float* B = raw + (static_cast<size_t>(min(k + 1, G0 - 1)) * T + tap) * 3;
                    const float* Cn = raw + (static_cast<size_t>(min(k + 2, G0 - 1)) * T + tap) * 3;
                    float D[3], D2[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        D[j] = (k + 1 < G0) ? B[j] - A[j] : 0.0f;
                        D2[j] = (k + 2 < G0) ? Cn[j] - B[j] : 0.0f;
                    }
                    if constexpr (trans)
                        q0 = v4f{A[0], D[0], A[1], D[1]};
                    else
                        q0 = v4f{-A[0], -D[0], -A[1], -D[1]};
                    q1 = v4f{A[2], D[2], 0.0f, 0.0f};
                    q2 = v4f{-(D2[0] - D[0]), -(D2[1] - D[1]), D2[2] - D[2], 0.0f};
                    if (!chain && (!(fabsf(A[0]) <= lim && fabsf(A[1]) <= lim) || !isfinite(A[2]))) mine = 1;
                } else {
                    const float* g = table + (static_cast<size_t>(k) * T + tap0 + i) * kRow1D;
                    q0 = v4f{g[0], g[1], g[2], g[3]};
                    q1 = v4f{g[4], g[5], 0.0f, 0.0f};
                    q2 = v4f{g[6], g[7], g[8], 0.0f};
                }
            }
            lds_v4f* d = reinterpret_cast<lds_v4f*>(static_cast<uintptr_t>(static_cast<uint32_t>(tabL + r * kRowLB)));
            d[0] = q0;
            d[1] = q1;
            d[2] = q2;
        }
        if (raw) bad = __syncthreads_or(mine);
    }
    if (bad) {  // an offset exceeds its declared halo: refuse to gather
        float nan[PY][C];
        for (int j = 0; j < PY; ++j)
            for (int c = 0; c < C; ++c) nan[j][c] = __builtin_nanf("");
        for (; tile < tend; tile += nwg) {
            const int f = MODE == 0 ? tile / ntf : 0, tt = tile - f * ntf;
            sv_store<C, TOut, PY>(Y + static_cast<size_t>(f) * C * plane, plane, W, H, (tt % tiles_x) * kTW + lx,
                                  (tt / tiles_x) * TH + lyb, nan);
        }
        return;
    }
    const int nr = (SY - wv + NW - 1) / NW;      // staged rows of this wave, <= kPipeRPW
    // one base pointer per plane and 32-bit element offsets inside a plane
    // (H W <= 2^30): the loads take a scalar base plus one vector offset
    const TIn* Xc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Xc[c] = X + c * plane;
    const float* Pd[DIMS];
#pragma unroll
    for (int d = 0; d < DIMS; ++d) Pd[d] = chain ? nullptr : P + d * plane;

    static_assert(kPipeRPW * kPipeNQ <= 32, "one outside-the-image bit per staged (row, chunk)");
    typename Staged<TIn>::type stg[kPipeRPW][kPipeNQ][C];
    uint32_t zmask = 0;   // zstage: bit rr * kPipeNQ + q set when that staged value lies outside the image
    float pv[PY][DIMS];
    float gv[PY][C];   // corr: the tile's output gradient at the lane's pixels (as loaded)
    uint32_t gmask = 0;   // corr: bit j set when the lane's pixel j lies outside the image
    // (frame, tile within the frame) of the current and the prefetched tile,
    // advanced by nwg without a division (nwg <= tiles per frame is not
    // assumed); chain layers (MODE != 0) always cover one frame
    int cur_f = 0, cur_t = tile;
    if constexpr (MODE == 0) {
        while (cur_t >= ntf) {
            cur_t -= ntf;
            ++cur_f;
        }
    }
    int nxt_f = cur_f, nxt_t = cur_t;
    auto advance = [&](int& f, int& t) {
        t += nwg;
        if constexpr (MODE == 0) {
            while (t >= ntf) {
                t -= ntf;
                ++f;
            }
        }
    };
    auto issue = [&](int f, int tt) {
        const size_t xfo = static_cast<size_t>(f) * C * plane, pfo = static_cast<size_t>(f) * pfs * plane;
        const int tx0 = (tt % tiles_x) * kTW, ty0 = (tt / tiles_x) * TH;
        uint32_t gx[kPipeNQ];
        bool vx[kPipeNQ];
#pragma unroll
        for (int q = 0; q < kPipeNQ; ++q) {
            const int cx = tx0 - halo + lane + 64 * q;
            gx[q] = static_cast<uint32_t>(min(max(cx, 0), W - 1));
            vx[q] = zstage ? static_cast<unsigned>(cx) < static_cast<unsigned>(W) : true;
        }
        if constexpr (zstage) zmask = 0;
#pragma unroll
        for (int rr = 0; rr < kPipeRPW; ++rr) {
            if (rr < nr) {
                const int ry = ty0 - halo + wv + NW * rr;
                const uint32_t grow = static_cast<uint32_t>(min(max(ry, 0), H - 1)) * static_cast<uint32_t>(W);
                const bool vy = zstage ? static_cast<unsigned>(ry) < static_cast<unsigned>(H) : true;
#pragma unroll
                for (int q = 0; q < kPipeNQ; ++q) {
                    if (q < nq) {
                        const uint32_t off = (grow + gx[q]) * static_cast<uint32_t>(sizeof(TIn));   // bytes
#pragma unroll
                        for (int c = 0; c < C; ++c) stg[rr][q][c] = Staged<TIn>::load(byte_at(Xc[c] + xfo, off));
                        if constexpr (zstage)
                            if (!(vy && vx[q])) zmask |= 1u << (rr * kPipeNQ + q);
                    }
                }
            }
        }
        const uint32_t xc = static_cast<uint32_t>(min(tx0 + lx, W - 1));
        if constexpr (corr) {
            gmask = 0;
#pragma unroll
            for (int j = 0; j < PY; ++j) {
                const int y = ty0 + 4 * j + lyb;
                const bool in = tx0 + lx < W && y < H;
                const uint32_t pi = (static_cast<uint32_t>(min(y, H - 1)) * static_cast<uint32_t>(W) + xc) * 4u;
#pragma unroll
                for (int c = 0; c < C; ++c) gv[j][c] = *byte_at(P + c * plane, pi);
                if (!in) gmask |= 1u << j;
            }
        }
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            const uint32_t pi = (static_cast<uint32_t>(min(ty0 + 4 * j + lyb, H - 1)) * static_cast<uint32_t>(W) + xc) * 4u;
#pragma unroll
            for (int d = 0; d < DIMS; ++d) {
                if constexpr (chain)
                    pv[j][d] = 0.0f;
                else
                    pv[j][d] = *byte_at(Pd[d] + pfo, pi);
            }
        }
    };

    // A tile's output is stored after the next tile has been staged, ahead of
    // that tile's prefetch: the loop-top wait for the prefetched loads then
    // never waits for stores (vmcnt retires in order, and exec-masked stores
    // are not counted by the compiler's wait), and the stores have a whole
    // tile of gathers to drain.
    float pacc[PY][C];
    TOut* pY = nullptr;
    int px = 0, py0 = 0;
    issue(cur_f, cur_t);
    for (;;) {
        // the staged registers of `tile` -> LDS
#pragma unroll
        for (int rr = 0; rr < kPipeRPW; ++rr) {
            const int ly = wv + NW * rr;
#pragma unroll
            for (int q = 0; q < kPipeNQ; ++q) {
                const int cx = lane + 64 * q;
                if (rr < nr && q < nq && cx < SX) {
                    float v[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) v[c] = Staged<TIn>::widen(stg[rr][q][c]);
                    if constexpr (zstage)
                        if ((zmask >> (rr * kPipeNQ + q)) & 1u)
#pragma unroll
                            for (int c = 0; c < C; ++c) v[c] = 0.0f;
                    sv_put<C>(lds, rowW, ly, cx, v);
                }
            }
        }
        float ta[PY], tb[PY];
        int kk[PY];
        sv_decode<DIMS, PY>(pv, G0, G1, ta, tb, kk);
        // Keep the decode (and its wait on this tile's P loads) ahead of the
        // next tile's prefetch: vmcnt retires in order, so a decode sunk below
        // the prefetch would wait for the whole prefetch.
#pragma unroll
        for (int j = 0; j < PY; ++j) asm volatile("" ::"v"(ta[j]), "v"(tb[j]), "v"(kk[j]));
        __syncthreads();
        const int fr = cur_f, tr = cur_t;
        advance(nxt_f, nxt_t);
        TOut* const Yf = Y + static_cast<size_t>(fr) * C * plane;
        const int x = (tr % tiles_x) * kTW + lx, y0 = (tr / tiles_x) * TH + lyb;
        const int next = tile + nwg;
        if constexpr (!corr || fused) {
            if (pY) sv_store<C, TOut, PY>(pY, plane, W, H, px, py0, pacc);
            asm volatile("" ::: "memory");   // the stores stay ahead of the prefetch
        }
        if constexpr (fused) {
            float xq[PY][C];
#pragma unroll
            for (int j = 0; j < PY; ++j)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    xq[j][c] = ((gmask >> j) & 1u) ? 0.0f : gv[j][c];
                    asm volatile("" ::"v"(xq[j][c]));   // this tile's X ahead of the prefetch
                }
            if (next < tend) issue(nxt_f, nxt_t);
            fused_tile_taps<C, PY, ROWB>(s, pacc, xq, base0, tabL, N, min(N, kCorrTaps));
            pY = Yf;
            px = x;
            py0 = y0;
        } else if constexpr (corr) {
            float gc[PY][C];
#pragma unroll
            for (int j = 0; j < PY; ++j)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    gc[j][c] = ((gmask >> j) & 1u) ? 0.0f : gv[j][c];
                    asm volatile("" ::"v"(gc[j][c]));   // this tile's G ahead of the prefetch
                }
            if (next < tend) issue(nxt_f, nxt_t);
            corr_tile_taps<C, PY, ROWB>(s, gc, base0, tabL, N);
        } else {
            if (next < tend) issue(nxt_f, nxt_t);
            sv_tile_taps<C, DIMS, PY, ROWB, TL>(pacc, ta, tb, kk, base0, rowB, table, tap0, N, T, tabL);
            pY = Yf;
            px = x;
            py0 = y0;
        }
        if (next >= tend) break;
        tile = next;
        cur_f = nxt_f;
        cur_t = nxt_t;
        __syncthreads();  // every wave is done reading this tile before the next is written
    }
    if constexpr (!corr || fused) {
        if (pY) sv_store<C, TOut, PY>(pY, plane, W, H, px, py0, pacc);
    }
    corr_finish();
}

// Fallback for halos whose staged tile does not fit in LDS: one pixel per
// thread, corners read straight from the (clamped) source planes through L1/L2.
// Same decode, coefficients, corner weights and accumulation order as the
// staged kernels, so the results are identical.
template <int C, int DIMS, typename TIn, typename TOut>
__global__ __launch_bounds__(256) void sv_pass_global_kernel(const TIn* __restrict__ X, TOut* __restrict__ Y,
                                                             const float* __restrict__ P,
                                                             const float* __restrict__ table, int tap0, int N, int T,
                                                             int G0, int G1, int H, int W,
                                                             const int* __restrict__ flag) {
    constexpr int RW = DIMS == 1 ? kRow1D : kRow2D;
    const long idx = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= static_cast<long>(H) * W) return;
    const int y = static_cast<int>(idx / W), x = static_cast<int>(idx - static_cast<long>(y) * W);
    const size_t plane = static_cast<size_t>(H) * W;
    float acc[C];
    if (*flag) {
#pragma unroll
        for (int c = 0; c < C; ++c) IO<TOut>::store(Y, c * plane + idx, __builtin_nanf(""));
        return;
    }
    float pv[1][DIMS];
#pragma unroll
    for (int d = 0; d < DIMS; ++d) pv[0][d] = P[d * plane + idx];
    float ta[1], tb[1];
    int kk[1];
    sv_decode<DIMS, 1>(pv, G0, G1, ta, tb, kk);
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0f;
    // one base per plane, 32-bit element offsets inside it (H W <= 2^30)
    const TIn* Xc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Xc[c] = X + c * plane;
    auto tap = [&](const float* __restrict__ r) {
        float nx, ny, w;
        if (DIMS == 1) {
            nx = fmaf(ta[0], r[1], r[0]);
            ny = fmaf(ta[0], r[3], r[2]);
            w = fmaf(ta[0], r[5], r[4]);
        } else {
            const float st = ta[0] * tb[0];
            nx = fmaf(st, r[3], fmaf(tb[0], r[2], fmaf(ta[0], r[1], r[0])));
            ny = fmaf(st, r[7], fmaf(tb[0], r[6], fmaf(ta[0], r[5], r[4])));
            w = fmaf(st, r[11], fmaf(tb[0], r[10], fmaf(ta[0], r[9], r[8])));
        }
        const float flx = floorf(nx), fly = floorf(ny);
        const float fx = nx - flx, fy = ny - fly;
        const float wy1 = w * fy, wy0 = w - wy1;
        const float c01 = wy0 * fx, c00 = wy0 - c01;
        const float c11 = wy1 * fx, c10 = wy1 - c11;
        const int x0 = x + static_cast<int>(flx), y0 = y + static_cast<int>(fly);
        const uint32_t xa = static_cast<uint32_t>(min(max(x0, 0), W - 1));
        const uint32_t xb = static_cast<uint32_t>(min(max(x0 + 1, 0), W - 1));
        const uint32_t ra = static_cast<uint32_t>(min(max(y0, 0), H - 1)) * static_cast<uint32_t>(W);
        const uint32_t rb = static_cast<uint32_t>(min(max(y0 + 1, 0), H - 1)) * static_cast<uint32_t>(W);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            constexpr uint32_t E = sizeof(TIn);
            float a = acc[c];
            a = fmaf(c00, IO<TIn>::load(byte_at(Xc[c], (ra + xa) * E), 0), a);
            a = fmaf(c01, IO<TIn>::load(byte_at(Xc[c], (ra + xb) * E), 0), a);
            a = fmaf(c10, IO<TIn>::load(byte_at(Xc[c], (rb + xa) * E), 0), a);
            a = fmaf(c11, IO<TIn>::load(byte_at(Xc[c], (rb + xb) * E), 0), a);
            acc[c] = a;
        }
    };
    // a wave whose pixels share one interval reads its coefficient rows at a
    // wave-uniform address (scalar loads); same arithmetic either way
    const int k0 = uniform(kk[0]);
    if (__all(kk[0] == k0)) {
        const float* e = table + (static_cast<size_t>(k0) * T + tap0) * RW;
        for (int i = 0; i < N; ++i) tap(e + i * RW);
    } else {
        for (int i = 0; i < N; ++i) tap(table + (static_cast<size_t>(kk[0]) * T + tap0 + i) * RW);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) IO<TOut>::store(Y, c * plane + idx, acc[c]);
}

// Angle axis of a 2-D basis: out[(i0 G1 + i1)][t] = base[i0][t] with its offset
// rotated by angle i1 (cos, sin given), weight copied.
struct RotArgs {
    int G0, G1, T;
    float cs[2 * 64];
};
__global__ __launch_bounds__(256) void rotate_basis_kernel(RotArgs a, const float* __restrict__ base,
                                                           float* __restrict__ out) {
    const long n = static_cast<long>(a.G0) * a.G1 * a.T;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * 256) {
        const int t = static_cast<int>(i % a.T);
        const long e = i / a.T;
        const int i1 = static_cast<int>(e % a.G1), i0 = static_cast<int>(e / a.G1);
        const float* b = base + (static_cast<size_t>(i0) * a.T + t) * 3;
        const float c = a.cs[2 * i1], s = a.cs[2 * i1 + 1];
        float* o = out + static_cast<size_t>(i) * 3;
        o[0] = fmaf(c, b[0], -s * b[1]);
        o[1] = fmaf(s, b[0], c * b[1]);
        o[2] = b[2];
    }
}

hipError_t launch_rotate_basis(int G0, int G1, int T, const double* angles, const float* base, float* out,
                               hipStream_t s) {
    RotArgs a{};
    a.G0 = G0;
    a.G1 = G1;
    a.T = T;
    for (int j = 0; j < G1; ++j) {
        a.cs[2 * j] = static_cast<float>(std::cos(angles[j]));
        a.cs[2 * j + 1] = static_cast<float>(std::sin(angles[j]));
    }
    const long n = static_cast<long>(G0) * G1 * T;
    hipLaunchKernelGGL(rotate_basis_kernel, dim3(static_cast<unsigned>(std::min<long>((n + 255) / 256, 1024))),
                       dim3(256), 0, s, a, base, out);
    return hipGetLastError();
}

// Tile choice.  DISK_SV_PIPE=0 forces the one-tile-per-work-group kernel (a
// tuning override, read once).
static int env_int(const char* name, int dflt) {
    const char* e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

// LDS bytes of a tile of 4*rows rows.
size_t sv_lds_bytes(int halo, int C, int rows, bool pad) {
    return static_cast<size_t>(sv_row_dwords(halo, C, pad)) * (4 * rows + 2 * halo) * sizeof(float);
}

int sv_rows_per_wave(int halo, int C) { return sv_lds_bytes(halo, C, 8) <= 160 * 1024 ? 4 : 2; }

static int cu_count() {
    static const int n = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        return v;
    }();
    return n;
}

// Staged-tile row stride of the C >= 3 pipe kernels: 448 dwords (112 float4
// pixels) holds 64 + 2 * 24 columns and is 64 mod 128 dwords (bank rule above)
// for every halo up to 24.
constexpr int kPipeRowB = 448 * 4;

template <int C, int DIMS, typename TIn, typename TOut, int NW, int HMAX, int ROWB, bool TL>
static size_t pipe_lds_bytes(int halo, int G0, int N) {
    constexpr int TH = PipeShape<NW, HMAX>::TH;
    const size_t rowB = ROWB > 0 ? ROWB : static_cast<size_t>(sv_row_dwords(halo, C)) * 4;
    return rowB * (TH + 2 * halo) + (TL ? sv_ltab_bytes(G0, N) : 0);
}

template <int C, int DIMS, typename TIn, typename TOut, int NW, int HMAX, int ROWB, bool TL, int MODE = 0>
static hipError_t launch_pipe(const void* src, void* dst, const float* pmap, const float* table, int tap0, int N,
                              int T, int G0, int G1, int H, int W, int halo, const int* flag, const float* raw,
                              hipStream_t s, int pN = 0, int pofs = 0, int* grid_out = nullptr,
                              float* part = nullptr, int grid = 0, Frames fr = Frames{}) {
    constexpr int TH = PipeShape<NW, HMAX>::TH;
    const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + TH - 1) / TH;
    const int ntf = tiles_x * tiles_y;
    const int ntiles = ntf * fr.F;
    const int per = (ntiles + 7) / 8;
    const int hs = MODE != 0 ? HMAX : halo;   // chain layers size the tile for HMAX
    const size_t lds = pipe_lds_bytes<C, DIMS, TIn, TOut, NW, HMAX, ROWB, TL>(hs, G0, N);
    const int rowW = ROWB > 0 ? ROWB / 4 : sv_row_dwords(hs, C);
    auto fn = sv_pass_pipe_kernel<C, DIMS, TIn, TOut, NW, HMAX, ROWB, TL, MODE>;
    // Host queries once per kernel and LDS size (launches of a frame repeat them)
    static std::mutex mu;
    static size_t attr_lds = 0, occ_lds = 0;
    static int occ_cached = 1;
    int occ = 1;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (lds > attr_lds) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
            if (e != hipSuccess) return e;
            attr_lds = lds;
        }
        if (lds != occ_lds) {
            int o = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, reinterpret_cast<const void*>(fn), 64 * NW, lds) !=
                    hipSuccess ||
                o < 1)
                o = 1;
            occ_cached = o;
            occ_lds = lds;
        }
        occ = occ_cached;
    }
    int per_xcd = (cu_count() * occ) / 8;                 // work-groups per XCD
    per_xcd = std::max(1, std::min(per_xcd, per));
    if (grid > 0) per_xcd = grid / 8;                     // a given grid (a multiple of 8): partials laid out alike
    hipLaunchKernelGGL(fn, dim3(8 * per_xcd), dim3(64 * NW), lds, s, static_cast<const TIn*>(src),
                       static_cast<TOut*>(dst), pmap, table, tap0, N, T, G0, G1, H, W, halo, tiles_x, per, ntiles,
                       flag, rowW, raw, pN, pofs, part, ntf, fr.pmap_shared ? 0 : DIMS);
    if (grid_out) *grid_out = 8 * per_xcd;
    return hipGetLastError();
}

template <int C, int DIMS, typename TIn, typename TOut, int PY, int NW>
static hipError_t launch_tiles(const void* src, void* dst, const float* pmap, const float* table, int tap0, int N,
                               int T, int G0, int G1, int H, int W, int halo, const int* flag, hipStream_t s,
                               bool pad = true) {
    constexpr int TH = 4 * PY * (NW / 4);
    const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + TH - 1) / TH;
    const int ntiles = tiles_x * tiles_y;
    const int per = (ntiles + 7) / 8;
    const size_t lds = sv_lds_bytes(halo, C, PY * (NW / 4), pad);
    const int rowW = sv_row_dwords(halo, C, pad);
    auto fn = sv_pass_kernel<C, DIMS, TIn, TOut, PY, NW>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(8 * per), dim3(64 * NW), lds, s, static_cast<const TIn*>(src),
                       static_cast<TOut*>(dst), pmap, table, tap0, N, T, G0, G1, H, W, halo, tiles_x, per,
                       ntiles, flag, rowW);
    return hipGetLastError();
}

template <int C, int DIMS, typename TIn, typename TOut>
static hipError_t launch_typed(const void* src, void* dst, const float* pmap, const float* table, int tap0, int N,
                               int T, int G0, int G1, int H, int W, int halo, const int* flag, const float* raw,
                               hipStream_t s, Frames fr) {
    static const int pipe = env_int("DISK_SV_PIPE", 1);
    // small halos: 8-wave work-groups of 64 x 16 tiles, two per CU, whose
    // staging and gather phases drift apart and overlap; larger ones: 16-wave
    // work-groups of 64 x 32 tiles, one per CU.  C >= 3 with a 1-D basis: fixed
    // row stride and the layer table in LDS when it fits, else the scalar-cache
    // table; C < 3 or 2-D: runtime stride, scalar-cache table.
#define SV_TRY_PIPE(NW, HMAX, ROWB, TL, BUDGET)                                                              \
    if (pipe && halo <= HMAX &&                                                                              \
        pipe_lds_bytes<C, DIMS, TIn, TOut, NW, HMAX, ROWB, TL>(halo, G0, N) <= static_cast<size_t>(BUDGET)) \
        return launch_pipe<C, DIMS, TIn, TOut, NW, HMAX, ROWB, TL>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, \
                                                                  halo, flag, raw, s, 0, 0, nullptr, nullptr, 0, fr);
    if constexpr (C >= 3 && DIMS == 1) {
        SV_TRY_PIPE(8, kPipeHalo8, kPipeRowB, true, 80 * 1024)
        SV_TRY_PIPE(16, kPipeHalo, kPipeRowB, true, 160 * 1024)
    }
    if (raw) return hipErrorInvalidValue;   // the raw-basis path exists only in the kernels above
    if constexpr (C >= 3) {
        SV_TRY_PIPE(8, kPipeHalo8, kPipeRowB, false, 80 * 1024)
        SV_TRY_PIPE(16, kPipeHalo, kPipeRowB, false, 160 * 1024)
        SV_TRY_PIPE(8, kPipeHaloWide, kPipeRowBWide, false, 160 * 1024)
    } else {
        SV_TRY_PIPE(8, kPipeHalo8, 0, false, 80 * 1024)
        SV_TRY_PIPE(16, kPipeHalo, 0, false, 160 * 1024)
        SV_TRY_PIPE(16, kPipeHaloBig, 0, false, 160 * 1024)
    }
#undef SV_TRY_PIPE
    // A staged tile pays for its halo only when it is tall: 64 x 32 tiles while
    // they fit (for a C >= 3 image, its planes in groups of two and one); below
    // that the halo rows dominate (measured: an 8-row tile at halo 33 is slower
    // than reading the corners through L1), so larger halos take the
    // one-pixel-per-thread kernel.  The kernels below take one frame per launch.
    const size_t fsz = static_cast<size_t>(C) * H * W, psz = fr.pmap_shared ? 0 : static_cast<size_t>(DIMS) * H * W;
    for (int f = 0; f < fr.F; ++f) {
        const TIn* xs = static_cast<const TIn*>(src) + f * fsz;
        TOut* ys = static_cast<TOut*>(dst) + f * fsz;
        const float* ps = pmap + f * psz;
        hipError_t e;
        if (sv_rows_per_wave(halo, C) == 4) {
            e = launch_tiles<C, DIMS, TIn, TOut, 4, 8>(xs, ys, ps, table, tap0, N, T, G0, G1, H, W, halo, flag, s);
        } else if (C >= 3 && sv_rows_per_wave(halo, 2) == 4) {
            // Every plane is filtered with the same per-pixel coefficients and
            // independently of the others: groups of two planes stage 8-byte
            // pixels, whose 64 x 32 tiles still fit the LDS at this halo.
            if constexpr (C >= 3) {
                const size_t plane = static_cast<size_t>(H) * W;
                e = launch_typed<2, DIMS, TIn, TOut>(xs, ys, ps, table, tap0, N, T, G0, G1, H, W, halo, flag, nullptr,
                                                     s, Frames{});
                if (e == hipSuccess)
                    e = launch_typed<C - 2, DIMS, TIn, TOut>(xs + 2 * plane, ys + 2 * plane, ps, table, tap0, N, T,
                                                             G0, G1, H, W, halo, flag, nullptr, s, Frames{});
            } else {
                e = hipErrorInvalidValue;   // not reached: C < 3 never takes this branch
            }
        } else {
            const long px = static_cast<long>(H) * W;
            hipLaunchKernelGGL((sv_pass_global_kernel<C, DIMS, TIn, TOut>), dim3(static_cast<unsigned>((px + 255) / 256)),
                               dim3(256), 0, s, xs, ys, ps, table, tap0, N, T, G0, G1, H, W, flag);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int C, int DIMS>
static hipError_t launch_py(int src_bf16, const void* src, int dst_bf16, void* dst, const float* pmap,
                            const float* table, int tap0, int N, int T, int G0, int G1, int H, int W, int halo,
                            const int* flag, const float* raw, hipStream_t s, Frames fr) {
    if (!src_bf16 && !dst_bf16)
        return launch_typed<C, DIMS, float, float>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
    if (src_bf16 && !dst_bf16)
        return launch_typed<C, DIMS, uint16_t, float>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
    if (!src_bf16 && dst_bf16)
        return launch_typed<C, DIMS, float, uint16_t>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
    return launch_typed<C, DIMS, uint16_t, uint16_t>(src, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
}

template <int C>
static hipError_t launch_dims(int dims, int src_bf16, const void* src, int dst_bf16, void* dst, const float* pmap,
                              const float* table, int tap0, int N, int T, int G0, int G1, int H, int W, int halo,
                              const int* flag, const float* raw, hipStream_t s, Frames fr) {
    if (dims == 1) return launch_py<C, 1>(src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
    return launch_py<C, 2>(src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
}

// One layer of a uniform chain on an image (CLAMP), as a pass of the staged
// kernel with a single-entry basis (Theta itself) and no parameter map: every
// pixel sits in the one interval at t = 0, so its coefficients are Theta's.
template <int C, typename TIn, typename TOut>
static hipError_t chain_typed(const void* src, void* dst, const float* theta, int tap0, int N, int T, int H, int W,
                              hipStream_t s) {
    return launch_pipe<C, 1, TIn, TOut, 16, kPipeHalo, kPipeRowB, true, 1>(src, dst, nullptr, nullptr, tap0, N, T, 1,
                                                                           1, H, W, 0, nullptr, theta, s);
}
template <int C>
static hipError_t chain_io(int src_bf16, const void* src, int dst_bf16, void* dst, const float* theta, int tap0,
                           int N, int T, int H, int W, hipStream_t s) {
    if (!src_bf16 && !dst_bf16) return chain_typed<C, float, float>(src, dst, theta, tap0, N, T, H, W, s);
    if (src_bf16 && !dst_bf16) return chain_typed<C, uint16_t, float>(src, dst, theta, tap0, N, T, H, W, s);
    if (!src_bf16 && dst_bf16) return chain_typed<C, float, uint16_t>(src, dst, theta, tap0, N, T, H, W, s);
    return chain_typed<C, uint16_t, uint16_t>(src, dst, theta, tap0, N, T, H, W, s);
}
template <int C>
static hipError_t chain_trans_c(const float* G, float* Gprev, const float* theta, int tap0, int N, int T, int H, int W,
                                hipStream_t s) {
    return launch_pipe<C, 1, float, float, 16, kPipeHalo, kPipeRowB, true, 2>(G, Gprev, nullptr, nullptr, tap0, N, T, 1,
                                                                             1, H, W, 0, nullptr, theta, s);
}
hipError_t launch_chain_transpose(int C, const float* G, float* Gprev, const float* theta, int tap0, int N, int T,
                                  int H, int W, hipStream_t s) {
    if (C == 3) return chain_trans_c<3>(G, Gprev, theta, tap0, N, T, H, W, s);
    if (C == 4) return chain_trans_c<4>(G, Gprev, theta, tap0, N, T, H, W, s);
    return hipErrorInvalidValue;
}
// Tap correlations of one chain layer (C = 3, 4) into partial[grid][N][4]
// (taps first .. N - 1, chunks of kCorrTaps per launch); *nblk = the grid
// (rows of partial), or `grid` when given.
template <int C, typename TIn, int MODE>
static hipError_t corr_typed(const void* X, const float* G, const float* theta, int tap0, int N, int T, int H, int W,
                             float* partial, int* nblk, hipStream_t s, int first, int grid) {
    for (int c0 = first; c0 < N; c0 += kCorrTaps) {
        const hipError_t e = launch_pipe<C, 1, TIn, float, 16, kPipeHalo, kPipeRowB, true, MODE>(
            X, partial, G, nullptr, tap0 + c0, std::min(kCorrTaps, N - c0), T, 1, 1, H, W, 0, nullptr, theta, s, N,
            c0, nblk, nullptr, grid);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
template <int C>
static hipError_t corr_c(int zero, const float* X, const float* G, const float* theta, int tap0, int N, int T, int H,
                         int W, float* partial, int* nblk, hipStream_t s, int first, int grid) {
    if (zero) return corr_typed<C, float, 4>(X, G, theta, tap0, N, T, H, W, partial, nblk, s, first, grid);
    return corr_typed<C, float, 3>(X, G, theta, tap0, N, T, H, W, partial, nblk, s, first, grid);
}
hipError_t launch_adjoint_corr(int C, int boundary, const float* X, const float* G, const float* theta, int tap0,
                               int N, int T, int H, int W, float* partial, int* nblk, hipStream_t s) {
    const int zero = boundary == DISK_ZERO;
    if (C == 3) return corr_c<3>(zero, X, G, theta, tap0, N, T, H, W, partial, nblk, s, 0, 0);
    if (C == 4) return corr_c<4>(zero, X, G, theta, tap0, N, T, H, W, partial, nblk, s, 0, 0);
    return hipErrorInvalidValue;
}

template <int C>
static hipError_t fused_c(int zero, const float* G, const float* X, float* Gn, const float* theta, int tap0, int N,
                          int T, int H, int W, float* partial, const TapU* taps, int* nrows_out, hipStream_t s) {
    int nb = 0;
    hipError_t e = zero ? launch_pipe<C, 1, float, float, 16, kPipeHalo, kPipeRowB, true, 6>(
                              G, Gn, X, nullptr, tap0, N, T, 1, 1, H, W, 0, nullptr, theta, s, N, 0, &nb, partial)
                        : launch_pipe<C, 1, float, float, 16, kPipeHalo, kPipeRowB, true, 5>(
                              G, Gn, X, nullptr, tap0, N, T, 1, 1, H, W, 0, nullptr, theta, s, N, 0, &nb, partial);
    if (e != hipSuccess) return e;
    if (N > kCorrTaps) {   // the other taps' correlations, on the same grid (rows of partial)
        int nb2 = 0;
        e = corr_c<C>(zero, X, G, theta, tap0, N, T, H, W, partial, &nb2, s, kCorrTaps, nb);
        if (e != hipSuccess) return e;
    }
    int nrows = nb;
    if (!zero) {
        // CLAMP: the border samples into up to 16 rows after the grid's (the
        // partial buffer holds at least adjoint_tap_blocks(H, W) + 1 rows of
        // the layer's widest N) and the border pixels of Gn, in one launch
        const int parts = std::max(1, std::min(16, adjoint_tap_blocks(H, W) + 1 - nb));
        nrows = nb + parts;
        e = launch_adjoint_border(C, G, X, theta + 3 * tap0, taps, N, std::min(N, kCorrTaps), H, W, kPipeHalo,
                                  partial, nrows, parts, Gn, s);
        if (e != hipSuccess) return e;
    }
    *nrows_out = nrows;
    return hipSuccess;
}
hipError_t launch_chain_fused(int C, int boundary, const float* G, const float* X, float* Gn, const float* theta,
                              int tap0, int N, int T, int H, int W, float* partial, const TapU* taps,
                              int* nrows, hipStream_t s) {
    const int zero = boundary == DISK_ZERO;
    if (C == 3) return fused_c<3>(zero, G, X, Gn, theta, tap0, N, T, H, W, partial, taps, nrows, s);
    if (C == 4) return fused_c<4>(zero, G, X, Gn, theta, tap0, N, T, H, W, partial, taps, nrows, s);
    return hipErrorInvalidValue;
}

bool chain_pass_ok(int C, int boundary) {
    static const int pipe = env_int("DISK_SV_PIPE", 1);
    return pipe && C >= 3 && C <= 4 && boundary == DISK_CLAMP;
}
hipError_t launch_chain_pass(int C, int src_bf16, const void* src, int dst_bf16, void* dst, const float* theta,
                             int tap0, int N, int T, int H, int W, hipStream_t s) {
    if (C == 3) return chain_io<3>(src_bf16, src, dst_bf16, dst, theta, tap0, N, T, H, W, s);
    if (C == 4) return chain_io<4>(src_bf16, src, dst_bf16, dst, theta, tap0, N, T, H, W, s);
    return hipErrorInvalidValue;
}

bool sv_pass_raw_ok(int C, int dims, int halo, int G0, int N) {
    static const int pipe = env_int("DISK_SV_PIPE", 1);
    if (C < 3 || dims != 1 || !pipe) return false;
    // the same conditions as the table-in-LDS branches of launch_typed
    if (halo <= kPipeHalo8 &&
        pipe_lds_bytes<3, 1, float, float, 8, kPipeHalo8, kPipeRowB, true>(halo, G0, N) <= 80 * 1024)
        return true;
    return halo <= kPipeHalo &&
           pipe_lds_bytes<3, 1, float, float, 16, kPipeHalo, kPipeRowB, true>(halo, G0, N) <= 160 * 1024;
}

hipError_t launch_sv_pass(int C, int dims, int src_bf16, const void* src, int dst_bf16, void* dst,
                          const float* pmap, const float* table, int tap0, int N, int T, int G0, int G1,
                          int H, int W, int halo, const int* flag, const float* raw, hipStream_t s, Frames fr) {
    if (fr.F < 1) return hipErrorInvalidValue;
    switch (C) {
        case 1: return launch_dims<1>(dims, src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
        case 2: return launch_dims<2>(dims, src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
        case 3: return launch_dims<3>(dims, src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
        default: return launch_dims<4>(dims, src_bf16, src, dst_bf16, dst, pmap, table, tap0, N, T, G0, G1, H, W, halo, flag, raw, s, fr);
    }
}

}  // namespace disk
