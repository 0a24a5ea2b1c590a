// Internal launch interface between the C ABI (abi.cpp) and the HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/disk.h"

namespace disk {

// One uniform tap, prepared once per call: integer corner offset of the
// gather at p - o and the four bilinear corner weights premultiplied by w.
struct TapU {
    int ix, iy;          // floor(-ox), floor(-oy)
    float c00, c01, c10, c11;
    int pad0, pad1;
};
static_assert(sizeof(TapU) == 32, "TapU layout");

struct LayerSpec {
    int L;
    int taps[DISK_MAX_LAYERS];
    int tap0[DISK_MAX_LAYERS];
    int T;
};

inline LayerSpec make_spec(const disk_complex& cx) {
    LayerSpec s{};
    s.L = cx.L;
    int o = 0;
    for (int l = 0; l < cx.L; ++l) {
        s.taps[l] = cx.taps[l];
        s.tap0[l] = o;
        o += cx.taps[l];
    }
    s.T = o;
    return s;
}

// ---- chain.hip: uniform-Theta chain on images / impulse canvases ----------
// Prepares TapU[T] from theta[T][3].
hipError_t launch_prep_uniform(const float* theta, int T, TapU* out, hipStream_t s);
// One layer.  src_kind: 0 = f32 image, 1 = bf16 image, 2 = impulse (centre).
// dst_kind: 0 = f32, 1 = bf16.
hipError_t launch_layer_uniform(int C, int boundary, int src_kind, const void* src, int dst_kind,
                                void* dst, const TapU* taps, int N, int H, int W, hipStream_t s);

// ---- adjoint.hip -------------------------------------------------------------
// Per-tap correlation sums S_ab = sum_p G[p] X[p + (ix+a, iy+b)] (boundary
// mapped) into partial[nblk][N][4]; returns nblk through *nblk_out.
int adjoint_tap_blocks(int H, int W);
hipError_t launch_adjoint_taps(int C, int boundary, int src_kind, const void* X, const float* G,
                               const TapU* taps, int N, int H, int W, float* partial,
                               hipStream_t s);
// Reduces partials (fixed order) and writes dtheta rows [N][3] of this layer.
hipError_t launch_adjoint_finish(float* partial, int nblk, const float* theta_layer, int N, float* dtheta_layer,
                                 hipStream_t s);
// The same for n layers in one launch: entry l has N[l] taps from tap0[l] of
// the complex, nblk[l] partial rows at partial + pofs[l] (floats), and
// first[l] = the sum of N over the entries before it.
struct FinishLayers {
    int n = 0;
    int first[DISK_MAX_LAYERS], N[DISK_MAX_LAYERS], nblk[DISK_MAX_LAYERS], tap0[DISK_MAX_LAYERS];
    long long pofs[DISK_MAX_LAYERS];
};
hipError_t launch_adjoint_finish_layers(const FinishLayers& a, const float* partial, const float* theta, float* dtheta,
                                        hipStream_t s);
// Input adjoint: Gprev = A^T G (exact transpose incl. CLAMP border folding).
// pad: scratch of (H+2R)*(W+2R)*C floats for CLAMP (R = halo); may be null for ZERO.
hipError_t launch_adjoint_input(int C, int boundary, const float* G, const TapU* taps, int N, int H, int W,
                                float* Gprev, hipStream_t s);

// ---- filter.hip: spatially varying filter ------------------------------------
// Table row widths: 1-D 9 floats, 2-D 12 floats per (entry, tap).
size_t sv_table_floats(int dims, int G, int T);
hipError_t launch_sv_prep(int dims, int G0, int G1, const LayerSpec& spec, const int* halo,
                          const float* basis, float* table, int* flag, hipStream_t s);
int sv_rows_per_wave(int halo, int C);
size_t sv_lds_bytes(int halo, int C, int py, bool pad = true);
// table + flag from launch_sv_prep (raw == nullptr), or raw = the basis itself
// (1-D, C >= 3 layers for which sv_pass_raw_ok holds): the pass derives its
// layer's coefficient rows and checks its offsets against `halo` on its own.
// F frames [F][C][H][W] in one pass (the pipelined kernel walks the tiles of
// all frames in one launch); the parameter map is shared by the frames or one
// [dims][H][W] per frame.
struct Frames {
    int F = 1;
    int pmap_shared = 1;
};
hipError_t launch_sv_pass(int C, int dims, int src_bf16, const void* src, int dst_bf16, void* dst,
                          const float* pmap, const float* table, int tap0, int N, int T, int G0,
                          int G1, int H, int W, int halo, const int* flag, const float* raw, hipStream_t s,
                          Frames fr = Frames{});
bool sv_pass_raw_ok(int C, int dims, int halo, int G0, int N);
// One uniform-chain layer on a C = 3 or 4 image with the CLAMP boundary through
// the staged pass kernel (halo derived on the device from the layer's taps).
bool chain_pass_ok(int C, int boundary);
// Input adjoint of one uniform layer (C = 3, 4) through the staged kernel:
// the zero-padded gather at negated offsets, exact except on CLAMP border
// pixels, which launch_adjoint_input_border then recomputes.
hipError_t launch_chain_transpose(int C, const float* G, float* Gprev, const float* theta, int tap0, int N, int T,
                                  int H, int W, hipStream_t s);
hipError_t launch_adjoint_input_border(int C, const float* G, const TapU* taps, int N, int H, int W, float* Gprev,
                                       hipStream_t s);
// Tap correlations of one uniform layer (C = 3, 4) through the staged kernel:
// partial[nblk][N][4] in the layout adjoint_finish_kernel sums (*nblk set to
// the grid, <= adjoint_tap_blocks(H, W)).  X: the layer input, G: its output
// gradient (both FP32).
hipError_t launch_adjoint_corr(int C, int boundary, const float* X, const float* G, const float* theta, int tap0,
                               int N, int T, int H, int W, float* partial, int* nblk, hipStream_t s);
// The backward of a chain layer (C = 3, 4; ZERO or CLAMP forward): its
// transpose G' into Gn fused with its tap correlations (the in-image part of
// the first taps from the fused pass, the other taps from correlation passes
// on the same grid, as rows of partial[][N][4]; *nrows is set to their
// count, for launch_adjoint_finish or launch_adjoint_finish_layers).  For
// CLAMP one launch after the pass adds the samples that leave the image and
// recomputes the border pixels of Gn exactly (launch_adjoint_border).  taps:
// the layer's prepared taps.
hipError_t launch_chain_fused(int C, int boundary, const float* G, const float* X, float* Gn, const float* theta,
                              int tap0, int N, int T, int H, int W, float* partial, const TapU* taps, int* nrows,
                              hipStream_t s);
// The CLAMP border work of one fused backward layer in one launch: the
// correlation samples that leave the image into rows nrows - parts .. nrows -
// 1 of partial, and the input adjoint on the border pixels of Gprev.
hipError_t launch_adjoint_border(int C, const float* G, const float* X, const float* theta_layer, const TapU* taps,
                                 int N, int NS, int H, int W, int hmax, float* partial, int nrows, int parts,
                                 float* Gprev, hipStream_t s);
hipError_t launch_chain_pass(int C, int src_bf16, const void* src, int dst_bf16, void* dst, const float* theta,
                             int tap0, int N, int T, int H, int W, hipStream_t s);

// ---- optimize.hip: batched optimiser and radial init --------------------------
// optional outputs and resumed state of one optimiser launch
struct OptExtra {
    unsigned long long* ticks = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    const int* start = nullptr;
    float* loss = nullptr;
    int max_updates = 0;
};
int opt_workgroups(int B, int per_cu, int threads);
// the built-in launch table (opt_tune.cpp)
disk_opt_tune opt_default_tune(const disk_batch_meta& m);
size_t opt_slot_floats(int max_side, int max_L);
hipError_t launch_optimize(int B, const disk_target* desc, const int* taps, const float* targets, float* theta,
                           float* psnr, int* steps, int* status, const disk_opt_params& p, int* order, int* queue,
                           float* scratch, size_t slot_floats, int nwg, int max_side, int max_T,
                           const OptExtra& x, int threads, hipStream_t s);
hipError_t launch_continue(const disk_target* desc, const int* taps, float* theta, int k, float scale,
                           hipStream_t s);
hipError_t launch_init_radial(int B, const disk_target* desc, const int* taps, const float* targets, float* theta,
                              int max_side, int max_T, hipStream_t s);

hipError_t launch_rotate_basis(int G0, int G1, int T, const double* angles, const float* base, float* out,
                               hipStream_t s);

// ---- dense reference (dense.hip) ----
hipError_t launch_dense_sv(int kind, float r0, float r1, float a0, float a1, int half, const void* image,
                           const float* pmap, void* out, int C, int H, int W, int bf16, hipStream_t s);

// ---- learned initialiser (net.hip) ----
struct NetWs {   // byte offsets into the caller's workspace
    size_t wp, act, yhat, g32[2], gq[2], part, cpart, cslab, grad, total;
};
long net_param_count();
NetWs net_ws_layout(int B, bool train);
void net_wgrad_splits(int cout, int Kp, int Mred, int* S, int* kchunk);
hipError_t net_forward(const float* params, const uint16_t* x0, int B, char* ws, const NetWs& w, float* out,
                       const float* hw, hipStream_t s);
hipError_t net_backward(const float* params, const uint16_t* x0, const float* ref, const float* hw, int B, char* ws,
                        const NetWs& w, float* grad, float* loss_out, hipStream_t s);
hipError_t net_adam(float* params, float* m, float* v, const float* grad, int step, float lr, hipStream_t s);
hipError_t net_prepare(int B, const disk_target* desc, const float* targets, uint16_t* x64, float* hw, int max_side,
                       hipStream_t s);
hipError_t net_scatter(int B, const disk_target* desc, const int* taps, const float* th48, float* theta,
                       hipStream_t s);

}  // namespace disk
