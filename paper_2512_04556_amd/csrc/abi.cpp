// C ABI of libdisk: argument validation, workspace carving and dispatch to
// the HIP kernels.  Nothing here allocates device memory, throws, exits or
// prints; failures return a negative disk_status with a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"

using namespace disk;

namespace {

thread_local std::string g_err;

disk_status fail(disk_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

disk_status ok() {
    g_err.clear();
    return DISK_OK;
}

disk_status hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(DISK_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return DISK_OK;
}

#define DISK_TRY(expr)                          \
    do {                                        \
        disk_status _s = (expr);                \
        if (_s != DISK_OK) return _s;           \
    } while (0)
#define DISK_HIP(expr, what) DISK_TRY(hip_check((expr), what))

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

disk_status check_ptr(const void* p, const char* name, bool nullable = false) {
    if (!p) return nullable ? DISK_OK : fail(DISK_INVALID_ARG, "%s is NULL", name);
    if (!aligned16(p)) return fail(DISK_INVALID_ARG, "%s is not 16-byte aligned", name);
    return DISK_OK;
}

disk_status check_complex(const disk_complex* cx) {
    if (!cx) return fail(DISK_INVALID_ARG, "complex is NULL");
    if (cx->L < 1 || cx->L > DISK_MAX_LAYERS) return fail(DISK_BAD_SHAPE, "L=%d out of [1,%d]", cx->L, DISK_MAX_LAYERS);
    for (int l = 0; l < cx->L; ++l)
        if (cx->taps[l] < 1 || cx->taps[l] > DISK_MAX_TAPS)
            return fail(DISK_BAD_SHAPE, "taps[%d]=%d out of [1,%d]", l, cx->taps[l], DISK_MAX_TAPS);
    return DISK_OK;
}

disk_status check_image(int C, int H, int W) {
    if (C < 1 || C > DISK_MAX_CHANNELS) return fail(DISK_BAD_SHAPE, "C=%d out of [1,%d]", C, DISK_MAX_CHANNELS);
    if (H < 1 || W < 1) return fail(DISK_BAD_SHAPE, "H=%d W=%d must be >= 1", H, W);
    if (static_cast<int64_t>(H) * W > (int64_t(1) << 30)) return fail(DISK_BAD_SHAPE, "image too large");
    return DISK_OK;
}

// Bump allocator over the caller's workspace (256-byte aligned slices).
struct Carve {
    char* base;
    size_t cap, used = 0;
    Carve(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
    template <typename T>
    T* take(size_t n) {
        used = (used + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += n * sizeof(T);
        return p;
    }
};

size_t image_floats(int C, int H, int W) { return static_cast<size_t>(C) * H * W; }

}  // namespace

extern "C" {

const char* disk_status_string(disk_status s) {
    switch (s) {
        case DISK_OK: return "DISK_OK";
        case DISK_INVALID_ARG: return "DISK_INVALID_ARG";
        case DISK_BAD_SHAPE: return "DISK_BAD_SHAPE";
        case DISK_WORKSPACE_TOO_SMALL: return "DISK_WORKSPACE_TOO_SMALL";
        case DISK_DEVICE: return "DISK_DEVICE";
        case DISK_UNSUPPORTED: return "DISK_UNSUPPORTED";
    }
    return "DISK_UNKNOWN";
}

const char* disk_last_error(void) { return g_err.c_str(); }
const char* disk_version(void) { return "libdisk 0.1 gfx950"; }

int64_t disk_clock_rate_khz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return khz;
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
static size_t forward_ws(const disk_complex* cx, int C, int H, int W, bool has_saved, Carve& cv,
                         TapU** tapu, float** buf0, float** buf1) {
    const LayerSpec sp = make_spec(*cx);
    *tapu = cv.take<TapU>(sp.T);
    const int nbuf = has_saved ? 0 : std::min(cx->L - 1, 2);
    *buf0 = nbuf >= 1 ? cv.take<float>(image_floats(C, H, W)) : nullptr;
    *buf1 = nbuf >= 2 ? cv.take<float>(image_floats(C, H, W)) : nullptr;
    return cv.used;
}

size_t disk_forward_workspace_size(const disk_complex* cx, int32_t C, int32_t H, int32_t W, disk_dtype,
                                   int32_t, int32_t has_saved) {
    if (!cx || cx->L < 1 || cx->L > DISK_MAX_LAYERS) return 0;
    Carve cv(nullptr, 0);
    TapU* t;
    float *a, *b;
    return forward_ws(cx, C, H, W, has_saved != 0, cv, &t, &a, &b) + 256;
}

disk_status disk_forward(const disk_complex* cx, const float* theta, const void* in, void* out, int32_t C,
                         int32_t H, int32_t W, disk_dtype io, disk_boundary boundary, float* saved, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
    DISK_TRY(check_complex(cx));
    DISK_TRY(check_image(C, H, W));
    DISK_TRY(check_ptr(theta, "theta"));
    DISK_TRY(check_ptr(in, "in", true));
    DISK_TRY(check_ptr(out, "out"));
    DISK_TRY(check_ptr(saved, "saved", true));
    DISK_TRY(check_ptr(ws, "ws", true));
    if (io != DISK_F32 && io != DISK_BF16) return fail(DISK_INVALID_ARG, "bad dtype %d", int(io));
    if (boundary != DISK_ZERO && boundary != DISK_CLAMP) return fail(DISK_INVALID_ARG, "bad boundary %d", int(boundary));
    const bool impulse = in == nullptr;
    if (impulse) {
        if (C != 1) return fail(DISK_BAD_SHAPE, "impulse mode needs C == 1");
        if ((H & 1) == 0 || (W & 1) == 0) return fail(DISK_BAD_SHAPE, "impulse mode needs odd sides (H=%d W=%d)", H, W);
        if (boundary != DISK_ZERO) return fail(DISK_INVALID_ARG, "impulse mode needs DISK_ZERO");
        if (io != DISK_F32) return fail(DISK_INVALID_ARG, "impulse mode needs DISK_F32");
    }
    Carve cv(ws, ws_bytes);
    TapU* tapu;
    float *b0, *b1;
    forward_ws(cx, C, H, W, saved != nullptr, cv, &tapu, &b0, &b1);
    if (!ws || cv.used > ws_bytes)
        return fail(DISK_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, cv.used);
    const LayerSpec sp = make_spec(*cx);
    const size_t n = image_floats(C, H, W);
    const int io_kind = io == DISK_BF16 ? 1 : 0;
    if (!impulse && chain_pass_ok(C, boundary)) {
        // images with C = 3, 4 and CLAMP: the LDS-staged pass kernel, taps from Theta
        for (int l = 0; l < sp.L; ++l) {
            const void* src = l == 0 ? in : (saved ? saved + (l - 1) * n : ((l - 1) % 2 ? b1 : b0));
            void* dst = l == sp.L - 1 ? out : (saved ? saved + l * n : (l % 2 ? b1 : b0));
            const int sb = (l == 0 && io_kind) ? 1 : 0;
            const int db = (l == sp.L - 1 && io_kind) ? 1 : 0;
            DISK_HIP(launch_chain_pass(C, sb, src, db, dst, theta, sp.tap0[l], sp.taps[l], sp.T, H, W, stream),
                     "chain layer");
        }
        return ok();
    }
    DISK_HIP(launch_prep_uniform(theta, sp.T, tapu, stream), "prep");
    for (int l = 0; l < sp.L; ++l) {
        const void* src;
        int src_kind;
        if (l == 0) {
            src = in;
            src_kind = impulse ? 2 : io_kind;
        } else {
            src = saved ? saved + (l - 1) * n : ((l - 1) % 2 ? b1 : b0);
            src_kind = 0;
        }
        void* dst;
        int dst_kind;
        if (l == sp.L - 1) {
            dst = out;
            dst_kind = io_kind;
        } else {
            dst = saved ? saved + l * n : (l % 2 ? b1 : b0);
            dst_kind = 0;
        }
        DISK_HIP(launch_layer_uniform(C, boundary, src_kind, src, dst_kind, dst, tapu + sp.tap0[l], sp.taps[l], H, W,
                                      stream),
                 "layer");
    }
    return ok();
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
static size_t partial_slot(int nblk, int maxN) { return static_cast<size_t>(nblk) * maxN * 4 + maxN * 4; }

static size_t backward_ws(const disk_complex* cx, int C, int H, int W, Carve& cv, TapU** tapu, float** partial,
                          float** g0, float** g1) {
    const LayerSpec sp = make_spec(*cx);
    int maxN = 0;
    for (int l = 0; l < sp.L; ++l) maxN = std::max(maxN, sp.taps[l]);
    const int nblk = adjoint_tap_blocks(H, W);
    *tapu = cv.take<TapU>(sp.T);
    // one slot of partial rows per layer (their finish runs after the last layer)
    *partial = cv.take<float>(static_cast<size_t>(sp.L) * partial_slot(nblk, maxN));
    *g0 = cv.take<float>(image_floats(C, H, W));
    *g1 = cv.take<float>(image_floats(C, H, W));
    return cv.used;
}

size_t disk_backward_workspace_size(const disk_complex* cx, int32_t C, int32_t H, int32_t W) {
    if (!cx || cx->L < 1 || cx->L > DISK_MAX_LAYERS || H < 1 || W < 1) return 0;
    Carve cv(nullptr, 0);
    TapU* t;
    float *p, *a, *b;
    return backward_ws(cx, C, H, W, cv, &t, &p, &a, &b) + 256;
}

disk_status disk_backward(const disk_complex* cx, const float* theta, const float* in, const float* saved,
                          const float* grad_out, float* grad_theta, float* grad_in, int32_t C, int32_t H, int32_t W,
                          disk_boundary boundary, void* ws, size_t ws_bytes, hipStream_t stream) {
    DISK_TRY(check_complex(cx));
    DISK_TRY(check_image(C, H, W));
    DISK_TRY(check_ptr(theta, "theta"));
    DISK_TRY(check_ptr(in, "in", true));
    DISK_TRY(check_ptr(grad_out, "grad_out"));
    DISK_TRY(check_ptr(grad_theta, "grad_theta", true));
    DISK_TRY(check_ptr(grad_in, "grad_in", true));
    if (boundary != DISK_ZERO && boundary != DISK_CLAMP) return fail(DISK_INVALID_ARG, "bad boundary %d", int(boundary));
    if (cx->L > 1) DISK_TRY(check_ptr(saved, "saved"));
    const bool impulse = in == nullptr;
    if (impulse) {
        if (C != 1) return fail(DISK_BAD_SHAPE, "impulse mode needs C == 1");
        if ((H & 1) == 0 || (W & 1) == 0) return fail(DISK_BAD_SHAPE, "impulse mode needs odd sides (H=%d W=%d)", H, W);
        if (boundary != DISK_ZERO) return fail(DISK_INVALID_ARG, "impulse mode needs DISK_ZERO");
    }
    Carve cv(ws, ws_bytes);
    TapU* tapu;
    float *partial, *g0, *g1;
    backward_ws(cx, C, H, W, cv, &tapu, &partial, &g0, &g1);
    if (!ws || cv.used > ws_bytes)
        return fail(DISK_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, cv.used);
    const LayerSpec sp = make_spec(*cx);
    const size_t n = image_floats(C, H, W);
    const int nblk = adjoint_tap_blocks(H, W);
    int maxN = 0;
    for (int l = 0; l < sp.L; ++l) maxN = std::max(maxN, sp.taps[l]);
    const size_t slot = partial_slot(nblk, maxN);
    DISK_HIP(launch_prep_uniform(theta, sp.T, tapu, stream), "prep");
    const float* G = grad_out;
    FinishLayers fin;   // the fused layers' dTheta, reduced in one launch after the last layer
    for (int l = sp.L - 1; l >= 0; --l) {
        const void* X = l == 0 ? static_cast<const void*>(in) : static_cast<const void*>(saved + (l - 1) * n);
        const int src_kind = (l == 0 && impulse) ? 2 : 0;
        float* partial_l = partial + l * slot;
        if (grad_theta && (l > 0 || grad_in) && !impulse && chain_pass_ok(C, DISK_CLAMP)) {
            // the input adjoint and the tap correlations in one staged pass
            float* Gn = l == 0 ? grad_in : (G == g0 ? g1 : g0);
            int nrows = 0;
            DISK_HIP(launch_chain_fused(C, boundary, G, static_cast<const float*>(X), Gn, theta, sp.tap0[l],
                                        sp.taps[l], sp.T, H, W, partial_l, tapu + sp.tap0[l], &nrows, stream),
                     "adjoint fused");
            const int k = fin.n++;
            fin.first[k] = k == 0 ? 0 : fin.first[k - 1] + fin.N[k - 1];
            fin.N[k] = sp.taps[l];
            fin.nblk[k] = nrows;
            fin.tap0[k] = sp.tap0[l];
            fin.pofs[k] = static_cast<long long>(l) * static_cast<long long>(slot);
            G = Gn;
            continue;
        }
        if (grad_theta) {
            int nb = nblk;
            if (!impulse && chain_pass_ok(C, DISK_CLAMP)) {
                DISK_HIP(launch_adjoint_corr(C, boundary, static_cast<const float*>(X), G, theta, sp.tap0[l], sp.taps[l],
                                             sp.T, H, W, partial_l, &nb, stream),
                         "adjoint taps");
            } else {
                DISK_HIP(launch_adjoint_taps(C, boundary, src_kind, X, G, tapu + sp.tap0[l], sp.taps[l], H, W,
                                             partial_l, stream),
                         "adjoint taps");
            }
            DISK_HIP(launch_adjoint_finish(partial_l, nb, theta + 3 * sp.tap0[l], sp.taps[l],
                                           grad_theta + 3 * sp.tap0[l], stream),
                     "adjoint finish");
        }
        if (l > 0 || grad_in) {
            float* Gn = l == 0 ? grad_in : (G == g0 ? g1 : g0);
            if (!impulse && chain_pass_ok(C, DISK_CLAMP)) {
                // staged transposed gather; CLAMP border pixels recomputed exactly
                DISK_HIP(launch_chain_transpose(C, G, Gn, theta, sp.tap0[l], sp.taps[l], sp.T, H, W, stream),
                         "adjoint input");
                if (boundary == DISK_CLAMP)
                    DISK_HIP(launch_adjoint_input_border(C, G, tapu + sp.tap0[l], sp.taps[l], H, W, Gn, stream),
                             "adjoint input border");
            } else {
                DISK_HIP(launch_adjoint_input(C, boundary, G, tapu + sp.tap0[l], sp.taps[l], H, W, Gn, stream),
                         "adjoint input");
            }
            G = Gn;
        }
    }
    if (fin.n > 0) DISK_HIP(launch_adjoint_finish_layers(fin, partial, theta, grad_theta, stream), "adjoint finish");
    return ok();
}

// ---------------------------------------------------------------------------
// spatially varying filter
// ---------------------------------------------------------------------------
static int basis_entries(const disk_basis* b) { return b->dims == 1 ? b->grid[0] : b->grid[0] * b->grid[1]; }

static disk_status check_basis(const disk_basis* b) {
    if (!b) return fail(DISK_INVALID_ARG, "basis is NULL");
    DISK_TRY(check_complex(&b->cx));
    if (b->dims != 1 && b->dims != 2) return fail(DISK_BAD_SHAPE, "basis dims=%d (1 or 2)", b->dims);
    if (b->grid[0] < 1 || (b->dims == 2 && b->grid[1] < 1) || basis_entries(b) > 4096)
        return fail(DISK_BAD_SHAPE, "basis grid out of range");
    for (int l = 0; l < b->cx.L; ++l)
        if (b->halo[l] < 1 || b->halo[l] > DISK_MAX_HALO)
            return fail(DISK_UNSUPPORTED, "halo[%d]=%d outside [1,%d]", l, b->halo[l], DISK_MAX_HALO);
    return DISK_OK;
}

disk_status disk_basis_set_halo(disk_basis* b, const float* basis_theta_host) {
    if (!b || !basis_theta_host) return fail(DISK_INVALID_ARG, "NULL argument");
    DISK_TRY(check_complex(&b->cx));
    if (b->dims != 1 && b->dims != 2) return fail(DISK_BAD_SHAPE, "basis dims=%d (1 or 2)", b->dims);
    const LayerSpec sp = make_spec(b->cx);
    const int G = basis_entries(b);
    for (int l = 0; l < sp.L; ++l) {
        double m = 0.0;
        for (int e = 0; e < G; ++e)
            for (int i = sp.tap0[l]; i < sp.tap0[l] + sp.taps[l]; ++i) {
                const float* r = basis_theta_host + (static_cast<size_t>(e) * sp.T + i) * 3;
                if (!std::isfinite(r[0]) || !std::isfinite(r[1]) || !std::isfinite(r[2]))
                    return fail(DISK_INVALID_ARG, "non-finite basis value (entry %d tap %d)", e, i);
                m = std::max(m, std::max(std::fabs(double(r[0])), std::fabs(double(r[1]))));
            }
        b->halo[l] = static_cast<int32_t>(std::ceil(m)) + 1;
    }
    for (int l = sp.L; l < DISK_MAX_LAYERS; ++l) b->halo[l] = 0;
    return ok();
}

static size_t sv_table_bytes_of(const disk_basis* b) {
    const LayerSpec sp = make_spec(b->cx);
    return ((sv_table_floats(b->dims, basis_entries(b), sp.T) * sizeof(float) + 255) & ~size_t(255)) + 256;
}

static size_t sv_apply_ws(const disk_basis* b, int C, int H, int W, Carve& cv, float** b0, float** b1, int F = 1) {
    const int nbuf = std::min(b->cx.L - 1, 2);
    *b0 = nbuf >= 1 ? cv.take<float>(image_floats(C, H, W) * F) : nullptr;
    *b1 = nbuf >= 2 ? cv.take<float>(image_floats(C, H, W) * F) : nullptr;
    return cv.used;
}

size_t disk_sv_table_bytes(const disk_basis* b) {
    if (!b || b->cx.L < 1 || b->cx.L > DISK_MAX_LAYERS || (b->dims != 1 && b->dims != 2)) return 0;
    return sv_table_bytes_of(b);
}

size_t disk_sv_apply_workspace_size(const disk_basis* b, int32_t C, int32_t H, int32_t W, disk_dtype) {
    if (!b || b->cx.L < 1 || b->cx.L > DISK_MAX_LAYERS) return 0;
    Carve cv(nullptr, 0);
    float *a, *c;
    return sv_apply_ws(b, C, H, W, cv, &a, &c) + 256;
}

size_t disk_sv_filter_workspace_size(const disk_basis* b, int32_t C, int32_t H, int32_t W, disk_dtype io) {
    const size_t t = disk_sv_table_bytes(b);
    if (!t) return 0;
    return t + disk_sv_apply_workspace_size(b, C, H, W, io);
}

disk_status disk_sv_prepare(const disk_basis* b, const float* basis_theta, void* table, size_t table_bytes,
                            hipStream_t stream) {
    DISK_TRY(check_basis(b));
    DISK_TRY(check_ptr(basis_theta, "basis_theta"));
    DISK_TRY(check_ptr(table, "table"));
    if (table_bytes < sv_table_bytes_of(b))
        return fail(DISK_WORKSPACE_TOO_SMALL, "table %zu < %zu bytes", table_bytes, sv_table_bytes_of(b));
    const LayerSpec sp = make_spec(b->cx);
    const int G0 = b->grid[0], G1 = b->dims == 2 ? b->grid[1] : 1;
    float* tab = static_cast<float*>(table);
    int* flag = reinterpret_cast<int*>(static_cast<char*>(table) + sv_table_bytes_of(b) - 256);
    DISK_HIP(launch_sv_prep(b->dims, G0, G1, sp, b->halo, basis_theta, tab, flag, stream), "sv prep");
    return ok();
}

// The L passes, ping-ponging through b0/b1: coefficients from a prepared table
// and its flag, or (raw != nullptr) derived by each pass from the basis.
static disk_status sv_passes(const disk_basis* b, const void* image, const float* pmap, void* out, int C, int H,
                             int W, disk_dtype io, float* b0, float* b1, const float* tab, const int* flag,
                             const float* raw, hipStream_t stream, Frames fr = Frames{}) {
    const LayerSpec sp = make_spec(b->cx);
    const int G0 = b->grid[0], G1 = b->dims == 2 ? b->grid[1] : 1;
    for (int l = 0; l < sp.L; ++l) {
        const void* src = l == 0 ? image : ((l - 1) % 2 ? b1 : b0);
        void* dst = l == sp.L - 1 ? out : (l % 2 ? b1 : b0);
        const int sb = (l == 0 && io == DISK_BF16) ? 1 : 0;
        const int db = (l == sp.L - 1 && io == DISK_BF16) ? 1 : 0;
        DISK_HIP(launch_sv_pass(C, b->dims, sb, src, db, dst, pmap, tab, sp.tap0[l], sp.taps[l], sp.T, G0, G1, H, W,
                                b->halo[l], flag, raw, stream, fr),
                 "sv pass");
    }
    return ok();
}

disk_status disk_sv_apply(const disk_basis* b, const void* table, const void* image, const float* pmap, void* out,
                          int32_t C, int32_t H, int32_t W, disk_dtype io, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
    DISK_TRY(check_basis(b));
    DISK_TRY(check_image(C, H, W));
    DISK_TRY(check_ptr(table, "table"));
    DISK_TRY(check_ptr(image, "image"));
    DISK_TRY(check_ptr(pmap, "pmap"));
    DISK_TRY(check_ptr(out, "out"));
    DISK_TRY(check_ptr(ws, "ws", true));
    if (io != DISK_F32 && io != DISK_BF16) return fail(DISK_INVALID_ARG, "bad dtype %d", int(io));
    if (image == out) return fail(DISK_INVALID_ARG, "image and out must not alias");
    Carve cv(ws, ws_bytes);
    float *b0, *b1;
    sv_apply_ws(b, C, H, W, cv, &b0, &b1);
    if (cv.used > 0 && (!ws || cv.used > ws_bytes))
        return fail(DISK_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, cv.used);
    const float* tab = static_cast<const float*>(table);
    const int* flag = reinterpret_cast<const int*>(static_cast<const char*>(table) + sv_table_bytes_of(b) - 256);
    return sv_passes(b, image, pmap, out, C, H, W, io, b0, b1, tab, flag, nullptr, stream);
}

size_t disk_sv_filter_frames_workspace_size(const disk_basis* b, int32_t F, int32_t C, int32_t H, int32_t W,
                                            disk_dtype) {
    const size_t t = disk_sv_table_bytes(b);
    if (!t || F < 1 || F > DISK_MAX_FRAMES) return 0;
    Carve cv(nullptr, 0);
    float *a, *c;
    return t + sv_apply_ws(b, C, H, W, cv, &a, &c, F) + 256;
}

disk_status disk_sv_filter_frames(const disk_basis* b, const float* basis_theta, const void* images,
                                  const float* pmaps, int32_t pmap_per_frame, void* outs, int32_t F, int32_t C,
                                  int32_t H, int32_t W, disk_dtype io, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
    DISK_TRY(check_basis(b));
    DISK_TRY(check_image(C, H, W));
    if (F < 1 || F > DISK_MAX_FRAMES) return fail(DISK_BAD_SHAPE, "F=%d out of [1,%d]", F, DISK_MAX_FRAMES);
    DISK_TRY(check_ptr(basis_theta, "basis_theta"));
    DISK_TRY(check_ptr(images, "images"));
    DISK_TRY(check_ptr(pmaps, "pmaps"));
    DISK_TRY(check_ptr(outs, "outs"));
    DISK_TRY(check_ptr(ws, "ws", true));
    if (io != DISK_F32 && io != DISK_BF16) return fail(DISK_INVALID_ARG, "bad dtype %d", int(io));
    const size_t tb = sv_table_bytes_of(b);
    const size_t need = disk_sv_filter_frames_workspace_size(b, F, C, H, W, io);
    if (!ws || ws_bytes < need) return fail(DISK_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, need);
    if (images == outs) return fail(DISK_INVALID_ARG, "images and outs must not alias");
    const Frames fr{F, pmap_per_frame ? 0 : 1};
    Carve cv(static_cast<char*>(ws) + tb, ws_bytes - tb);
    float *b0, *b1;
    sv_apply_ws(b, C, H, W, cv, &b0, &b1, F);
    // 1-D basis with C >= 3: every pass derives its layer's coefficients from
    // the basis itself (no separate preparation launch); otherwise the table
    // is prepared at the start of the workspace.
    const LayerSpec sp = make_spec(b->cx);
    bool raw = true;
    for (int l = 0; l < sp.L; ++l) raw = raw && sv_pass_raw_ok(C, b->dims, b->halo[l], b->grid[0], sp.taps[l]);
    if (raw) return sv_passes(b, images, pmaps, outs, C, H, W, io, b0, b1, nullptr, nullptr, basis_theta, stream, fr);
    DISK_TRY(disk_sv_prepare(b, basis_theta, ws, tb, stream));
    const float* tab = static_cast<const float*>(ws);
    const int* flag = reinterpret_cast<const int*>(static_cast<const char*>(ws) + tb - 256);
    return sv_passes(b, images, pmaps, outs, C, H, W, io, b0, b1, tab, flag, nullptr, stream, fr);
}

disk_status disk_sv_filter(const disk_basis* b, const float* basis_theta, const void* image, const float* pmap,
                           void* out, int32_t C, int32_t H, int32_t W, disk_dtype io, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
    return disk_sv_filter_frames(b, basis_theta, image, pmap, 0, out, 1, C, H, W, io, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// batched optimisation, initialisers
// ---------------------------------------------------------------------------
static disk_status check_meta(const disk_batch_meta* m) {
    if (!m) return fail(DISK_INVALID_ARG, "meta is NULL");
    if (m->B < 1) return fail(DISK_BAD_SHAPE, "B=%d must be >= 1", m->B);
    if (m->max_side < 1 || m->max_side > DISK_MAX_SIDE || (m->max_side & 1) == 0)
        return fail(DISK_BAD_SHAPE, "max_side=%d must be odd in [1,%d]", m->max_side, DISK_MAX_SIDE);
    if (m->max_T < 1 || m->max_T > DISK_MAX_LAYERS * DISK_MAX_TAPS)
        return fail(DISK_BAD_SHAPE, "max_T=%d out of range", m->max_T);
    return DISK_OK;
}

static disk_status check_opt_params(const disk_opt_params* params) {
    if (!params) return fail(DISK_INVALID_ARG, "params is NULL");
    const disk_opt_params& p = *params;
    if (p.max_steps < 0) return fail(DISK_INVALID_ARG, "max_steps=%d < 0", p.max_steps);
    if (!(p.beta1 >= 0.0f && p.beta1 < 1.0f) || !(p.beta2 >= 0.0f && p.beta2 < 1.0f) || !(p.eps > 0.0f))
        return fail(DISK_INVALID_ARG, "bad Adam hyper-parameters");
    if (!std::isfinite(p.lr0) || !std::isfinite(p.lr1)) return fail(DISK_INVALID_ARG, "non-finite learning rate");
    if (p.loss != DISK_LOSS_NMSE && p.loss != DISK_LOSS_CHARBONNIER) return fail(DISK_INVALID_ARG, "bad loss %d", p.loss);
    if (p.loss == DISK_LOSS_CHARBONNIER && !(p.charb_eps > 0.0f)) return fail(DISK_INVALID_ARG, "charb_eps must be > 0");
    if (p.offset_units != DISK_OFFSETS_PIXELS && p.offset_units != DISK_OFFSETS_HALF_WIDTH)
        return fail(DISK_INVALID_ARG, "bad offset_units %d", p.offset_units);
    return DISK_OK;
}

static bool tune_ok(const disk_opt_tune* t) {
    return !t || (t->threads == 256 && t->wgs_per_cu >= 1 && t->wgs_per_cu <= 4) ||
           (t->threads == 1024 && t->wgs_per_cu == 1);
}

static disk_status check_tune(const disk_opt_tune* t) {
    if (!tune_ok(t))
        return fail(DISK_INVALID_ARG, "tune: threads=%d wgs_per_cu=%d (256 x 1..4, or 1024 x 1)", t->threads,
                    t->wgs_per_cu);
    return DISK_OK;
}

static disk_opt_tune launch_shape(const disk_batch_meta* m, const disk_opt_tune* t) {
    return t ? *t : opt_default_tune(*m);
}

static size_t optimize_ws(const disk_batch_meta* m, const disk_opt_tune* t, Carve& cv, int** order, int** queue,
                          float** scratch, size_t* slot, int* nwg) {
    const disk_opt_tune sh = launch_shape(m, t);
    *nwg = opt_workgroups(m->B, sh.wgs_per_cu, sh.threads);
    *slot = opt_slot_floats(m->max_side, std::min(m->max_T, DISK_MAX_LAYERS));
    *order = cv.take<int>(m->B);
    *queue = cv.take<int>(64);
    *scratch = cv.take<float>(*slot * *nwg);
    return cv.used;
}

size_t disk_optimize_workspace_size(const disk_batch_meta* meta, const disk_opt_tune* tune) {
    if (!meta || meta->B < 1 || meta->max_side < 1 || meta->max_T < 1) return 0;
    if (!tune_ok(tune)) return 0;
    Carve cv(nullptr, 0);
    int *o, *q, nwg;
    float* sc;
    size_t slot;
    return optimize_ws(meta, tune, cv, &o, &q, &sc, &slot, &nwg) + 256;
}

disk_status disk_optimize_default_tune(const disk_batch_meta* meta, disk_opt_tune* out) {
    if (!meta || !out) return fail(DISK_INVALID_ARG, "meta and out must not be NULL");
    if (meta->B < 1 || meta->max_side < 1 || meta->max_T < 1)
        return fail(DISK_INVALID_ARG, "bad batch meta (B=%d max_side=%d max_T=%d)", int(meta->B),
                    int(meta->max_side), int(meta->max_T));
    *out = opt_default_tune(*meta);
    return ok();
}

disk_status disk_optimize_batch(const disk_batch_meta* meta, const disk_target* desc, const int32_t* taps,
                                const float* targets, float* theta, float* psnr_db, int32_t* steps, int32_t* status,
                                uint64_t* finish_ticks, const disk_opt_params* params, const disk_opt_state* state,
                                const disk_opt_tune* tune, void* ws, size_t ws_bytes, hipStream_t stream) {
    DISK_TRY(check_meta(meta));
    DISK_TRY(check_ptr(desc, "desc"));
    DISK_TRY(check_ptr(taps, "taps"));
    DISK_TRY(check_ptr(targets, "targets"));
    DISK_TRY(check_ptr(theta, "theta"));
    DISK_TRY(check_ptr(psnr_db, "psnr_db"));
    DISK_TRY(check_ptr(steps, "steps"));
    DISK_TRY(check_ptr(status, "status"));
    DISK_TRY(check_opt_params(params));
    DISK_TRY(check_tune(tune));
    const disk_opt_params& p = *params;
    Carve cv(ws, ws_bytes);
    int *order, *queue, nwg;
    float* scratch;
    size_t slot;
    optimize_ws(meta, tune, cv, &order, &queue, &scratch, &slot, &nwg);
    if (!ws || cv.used > ws_bytes)
        return fail(DISK_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, cv.used);
    DISK_TRY(check_ptr(finish_ticks, "finish_ticks", true));
    OptExtra x;
    x.ticks = reinterpret_cast<unsigned long long*>(finish_ticks);
    if (state) {
        if ((state->adam_m == nullptr) != (state->adam_v == nullptr))
            return fail(DISK_INVALID_ARG, "state: adam_m and adam_v must be given together");
        if (state->max_updates < 0) return fail(DISK_INVALID_ARG, "state->max_updates=%d < 0", state->max_updates);
        DISK_TRY(check_ptr(state->adam_m, "state->adam_m", true));
        DISK_TRY(check_ptr(state->adam_v, "state->adam_v", true));
        DISK_TRY(check_ptr(state->start_step, "state->start_step", true));
        DISK_TRY(check_ptr(state->loss, "state->loss", true));
        x.adam_m = state->adam_m;
        x.adam_v = state->adam_v;
        x.start = state->start_step;
        x.loss = state->loss;
        x.max_updates = state->max_updates;
    }
    DISK_HIP(launch_optimize(meta->B, desc, taps, targets, theta, psnr_db, steps, status, p, order, queue, scratch,
                             slot, nwg, meta->max_side, meta->max_T, x, launch_shape(meta, tune).threads, stream),
             "optimize");
    return ok();
}

disk_status disk_fit_basis(const disk_batch_meta* meta, const disk_target* desc, const int32_t* taps,
                           const float* targets, float* theta, float* psnr_db, int32_t* steps, int32_t* status,
                           const float* scale, const disk_opt_params* params, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
    DISK_TRY(check_meta(meta));
    DISK_TRY(check_ptr(desc, "desc"));
    DISK_TRY(check_ptr(taps, "taps"));
    DISK_TRY(check_ptr(targets, "targets"));
    DISK_TRY(check_ptr(theta, "theta"));
    DISK_TRY(check_ptr(psnr_db, "psnr_db"));
    DISK_TRY(check_ptr(steps, "steps"));
    DISK_TRY(check_ptr(status, "status"));
    if (!scale) return fail(DISK_INVALID_ARG, "scale is NULL");
    for (int k = 1; k < meta->B; ++k)
        if (!(std::isfinite(scale[k]) && scale[k] > 0.0f))
            return fail(DISK_INVALID_ARG, "scale[%d]=%g must be finite and > 0", k, static_cast<double>(scale[k]));
    DISK_TRY(check_opt_params(params));
    const disk_batch_meta one{1, meta->max_side, meta->max_T};
    Carve cv(ws, ws_bytes);
    int *order, *queue, nwg;
    float* scratch;
    size_t slot;
    optimize_ws(&one, nullptr, cv, &order, &queue, &scratch, &slot, &nwg);
    if (!ws || cv.used > ws_bytes)
        return fail(DISK_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, cv.used);
    for (int k = 0; k < meta->B; ++k) {
        if (k > 0) DISK_HIP(launch_continue(desc, taps, theta, k, scale[k], stream), "continuation start");
        DISK_HIP(launch_optimize(1, desc + k, taps, targets, theta, psnr_db + k, steps + k, status + k, *params,
                                 order, queue, scratch, slot, nwg, meta->max_side, meta->max_T, OptExtra{},
                                 launch_shape(&one, nullptr).threads, stream),
                 "optimize");
    }
    return ok();
}

size_t disk_fit_basis_workspace_size(const disk_batch_meta* meta) {
    if (check_meta(meta) != DISK_OK) return 0;
    const disk_batch_meta one{1, meta->max_side, meta->max_T};
    Carve cv(nullptr, 0);
    int *order, *queue, nwg;
    float* scratch;
    size_t slot;
    optimize_ws(&one, nullptr, cv, &order, &queue, &scratch, &slot, &nwg);
    return cv.used;
}

disk_status disk_init_radial(const disk_batch_meta* meta, const disk_target* desc, const int32_t* taps,
                             const float* targets, float* theta, hipStream_t stream) {
    DISK_TRY(check_meta(meta));
    DISK_TRY(check_ptr(desc, "desc"));
    DISK_TRY(check_ptr(taps, "taps"));
    DISK_TRY(check_ptr(targets, "targets"));
    DISK_TRY(check_ptr(theta, "theta"));
    DISK_HIP(launch_init_radial(meta->B, desc, taps, targets, theta, meta->max_side, meta->max_T, stream),
             "init radial");
    return ok();
}

disk_status disk_basis_rotate(const float* base, int32_t G0, int32_t T, const double* angles, int32_t G1,
                              float* out, hipStream_t stream) {
    if (G0 < 1 || G1 < 1 || G1 > 64 || T < 1 || T > DISK_MAX_LAYERS * DISK_MAX_TAPS)
        return fail(DISK_BAD_SHAPE, "G0=%d G1=%d T=%d out of range", G0, G1, T);
    DISK_TRY(check_ptr(base, "base"));
    DISK_TRY(check_ptr(out, "out"));
    if (!angles) return fail(DISK_INVALID_ARG, "angles is NULL");
    for (int j = 0; j < G1; ++j)
        if (!std::isfinite(angles[j])) return fail(DISK_INVALID_ARG, "angles[%d] is not finite", j);
    const char* b = reinterpret_cast<const char*>(base);
    const char* o = reinterpret_cast<const char*>(out);
    if (o < b + static_cast<size_t>(G0) * T * 12 && b < o + static_cast<size_t>(G0) * G1 * T * 12)
        return fail(DISK_INVALID_ARG, "out overlaps base");
    DISK_HIP(launch_rotate_basis(G0, G1, T, angles, base, out, stream), "rotate basis");
    return ok();
}

// ---------------------------------------------------------------------------
// dense reference
// ---------------------------------------------------------------------------
disk_status disk_dense_sv(const disk_dense_params* p, const void* image, const float* pmap, void* out, int32_t C,
                          int32_t H, int32_t W, disk_dtype io, hipStream_t stream) {
    if (!p) return fail(DISK_INVALID_ARG, "params is NULL");
    DISK_TRY(check_image(C, H, W));
    if (p->kind != DISK_DENSE_DISK && p->kind != DISK_DENSE_ELLIPSE) return fail(DISK_INVALID_ARG, "bad kind %d", p->kind);
    if (p->half < 0 || p->half > 127) return fail(DISK_BAD_SHAPE, "half=%d out of [0,127]", p->half);
    if (!(std::isfinite(p->r0) && std::isfinite(p->r1) && p->r0 >= 0.0f && p->r1 >= 0.0f))
        return fail(DISK_INVALID_ARG, "radii must be finite and >= 0");
    if (p->kind == DISK_DENSE_ELLIPSE && !(p->a0 > 0.0f && p->a1 > 0.0f && std::isfinite(p->a0) && std::isfinite(p->a1)))
        return fail(DISK_INVALID_ARG, "aspects must be finite and > 0");
    if (io != DISK_F32 && io != DISK_BF16) return fail(DISK_INVALID_ARG, "bad dtype %d", int(io));
    DISK_TRY(check_ptr(image, "image"));
    DISK_TRY(check_ptr(pmap, "pmap"));
    DISK_TRY(check_ptr(out, "out"));
    if (image == out) return fail(DISK_INVALID_ARG, "out must not alias image");
    DISK_HIP(launch_dense_sv(p->kind, p->r0, p->r1, p->a0, p->a1, p->half, image, pmap, out, C, H, W,
                             io == DISK_BF16 ? 1 : 0, stream),
             "dense sv");
    return ok();
}

// ---------------------------------------------------------------------------
// learned initialiser
// ---------------------------------------------------------------------------
static disk_status check_net_batch(int32_t B) {
    if (B < 1 || B > DISK_NET_MAX_BATCH) return fail(DISK_BAD_SHAPE, "B=%d out of [1,%d]", B, DISK_NET_MAX_BATCH);
    return DISK_OK;
}

int64_t disk_net_param_count(void) { return net_param_count(); }

size_t disk_net_workspace_size(int32_t B) {
    if (B < 1 || B > DISK_NET_MAX_BATCH) return 0;
    return net_ws_layout(B, true).total;
}

size_t disk_net_predict_workspace_size(int32_t B) {
    if (B < 1 || B > DISK_NET_MAX_BATCH) return 0;
    return net_ws_layout(B, false).total;
}

disk_status disk_init_predict(const float* params, const uint16_t* targets64, const float* half_width, float* theta,
                              int32_t B, void* ws, size_t ws_bytes, hipStream_t stream) {
    DISK_TRY(check_net_batch(B));
    DISK_TRY(check_ptr(params, "params"));
    DISK_TRY(check_ptr(targets64, "targets64"));
    DISK_TRY(check_ptr(half_width, "half_width"));
    DISK_TRY(check_ptr(theta, "theta"));
    const NetWs w = net_ws_layout(B, false);
    if (!ws || ws_bytes < w.total) return fail(DISK_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, w.total);
    DISK_TRY(check_ptr(ws, "ws"));
    DISK_HIP(net_forward(params, targets64, B, static_cast<char*>(ws), w, theta, half_width, stream), "net forward");
    return ok();
}

disk_status disk_net_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr,
                                const uint16_t* targets64, const float* half_width, const float* theta_ref, int32_t B,
                                float* loss_out, float* grad_out, void* ws, size_t ws_bytes, hipStream_t stream) {
    DISK_TRY(check_net_batch(B));
    DISK_TRY(check_ptr(params, "params"));
    DISK_TRY(check_ptr(adam_m, "adam_m"));
    DISK_TRY(check_ptr(adam_v, "adam_v"));
    DISK_TRY(check_ptr(targets64, "targets64"));
    DISK_TRY(check_ptr(half_width, "half_width"));
    DISK_TRY(check_ptr(theta_ref, "theta_ref"));
    DISK_TRY(check_ptr(loss_out, "loss_out"));
    if (grad_out) DISK_TRY(check_ptr(grad_out, "grad_out"));
    if (params == adam_m || params == adam_v || adam_m == adam_v || (grad_out && (grad_out == params ||
                                                                                   grad_out == adam_m ||
                                                                                   grad_out == adam_v)))
        return fail(DISK_INVALID_ARG, "params, adam_m, adam_v and grad_out must be distinct");
    if (step < 1) return fail(DISK_INVALID_ARG, "step=%d must be >= 1", step);
    if (!std::isfinite(lr) || lr < 0.0f) return fail(DISK_INVALID_ARG, "lr must be finite and >= 0");
    const NetWs w = net_ws_layout(B, true);
    if (!ws || ws_bytes < w.total) return fail(DISK_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, w.total);
    DISK_TRY(check_ptr(ws, "ws"));
    char* base = static_cast<char*>(ws);
    float* grad = grad_out ? grad_out : reinterpret_cast<float*>(base + w.grad);
    DISK_HIP(net_forward(params, targets64, B, base, w, reinterpret_cast<float*>(base + w.yhat), nullptr, stream),
             "net forward");
    DISK_HIP(net_backward(params, targets64, theta_ref, half_width, B, base, w, grad, loss_out, stream), "net backward");
    DISK_HIP(net_adam(params, adam_m, adam_v, grad, step, lr, stream), "net adam");
    return ok();
}

disk_status disk_net_prepare_inputs(const disk_batch_meta* meta, const disk_target* desc, const float* targets,
                                    uint16_t* targets64, float* half_width, hipStream_t stream) {
    DISK_TRY(check_meta(meta));
    DISK_TRY(check_ptr(desc, "desc"));
    DISK_TRY(check_ptr(targets, "targets"));
    DISK_TRY(check_ptr(targets64, "targets64"));
    DISK_TRY(check_ptr(half_width, "half_width"));
    DISK_HIP(net_prepare(meta->B, desc, targets, targets64, half_width, meta->max_side, stream), "net prepare");
    return ok();
}

disk_status disk_net_scatter_theta(const disk_batch_meta* meta, const disk_target* desc, const int32_t* taps,
                                   const float* theta48, float* theta, hipStream_t stream) {
    DISK_TRY(check_meta(meta));
    DISK_TRY(check_ptr(desc, "desc"));
    DISK_TRY(check_ptr(taps, "taps"));
    DISK_TRY(check_ptr(theta48, "theta48"));
    DISK_TRY(check_ptr(theta, "theta"));
    DISK_HIP(net_scatter(meta->B, desc, taps, theta48, theta, stream), "net scatter");
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// disk_sv_filter_noalloc: disk_sv_filter with its scratch (the coefficient
// table and the two FP32 ping-pong images between passes) in a file-scope
// device array, for callers that cannot allocate device memory.  In host code
// the array's name is only a stand-in: its device address is looked up once
// per device with hipGetSymbolAddress (with that device current) and only that
// address reaches the kernels.  All calls on one device share its array, so
// calls that overlap on one device race.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoallocBytes = size_t(DISK_SV_NOALLOC_MAX_BYTES);
constexpr int kNoallocDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoallocBytes];
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoallocDevices] = {};

disk_status noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DISK_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kNoallocDevices)
        return fail(DISK_UNSUPPORTED, "device %d beyond the %d supported", dev, kNoallocDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(DISK_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return DISK_OK;
}
}  // namespace

size_t disk_sv_noalloc_max_bytes(void) { return kNoallocBytes; }

disk_status disk_sv_filter_noalloc(const disk_basis* b, const float* basis_theta, const void* image,
                                   const float* pmap, void* out, int32_t C, int32_t H, int32_t W, disk_dtype io,
                                   hipStream_t stream) {
    DISK_TRY(check_basis(b));
    DISK_TRY(check_image(C, H, W));
    const size_t need = disk_sv_filter_workspace_size(b, C, H, W, io);
    if (need == 0) return fail(DISK_BAD_SHAPE, "invalid basis or image shape");
    if (need > kNoallocBytes)
        return fail(DISK_WORKSPACE_TOO_SMALL,
                    "needs %zu bytes of scratch, more than the fixed %zu-byte device array of the allocation-free "
                    "entry point (use disk_sv_filter with a workspace)",
                    need, kNoallocBytes);
    void* ws = nullptr;
    DISK_TRY(noalloc_scratch(&ws));
    return disk_sv_filter(b, basis_theta, image, pmap, out, C, H, W, io, ws, kNoallocBytes, stream);
}
