// Batched optimisation of sparse kernel complexes (Sec. 4.1 Eq. 4; impulse
// supervision Sec. 4.4 Eq. 10-11; Adam with linear learning-rate decay,
// Sec. 5.1), and the radial initialiser (Eq. 6), for thousands of targets of
// uneven size in one persistent launch.
//
// One work-group owns one target at a time and runs every step of it
// in-kernel: forward chain on the impulse canvas, loss and PSNR, the adjoint,
// and the Adam update.  Work-groups pull targets from a queue ordered by
// decreasing cost (side^2 x taps), so the longest targets start first.
//
// Canvases.  Each target keeps L canvases of side S = M + 2P (P = (M+1)/2 + 1)
// in a per-work-group slot of the workspace: X_1..X_{L-1} and K_syn / G_L.
// The zero frame of width P is the ZERO boundary: every gather whose corner
// offsets stay within the frame (|offset| < ~M/2) is unconditional; taps
// beyond it take a masked path.  During the backward pass G_{l-1} overwrites
// X_{l-1}, which is dead once layer l's tap gradients are done.  The first
// layer acts on the impulse, so X_1 is the deterministic sum of its taps'
// bilinear splats and the first layer's tap gradients are point reads of G_1.
//
// Lanes: each wave walks 8 x 8 pixel blocks of the canvas, so lane utilisation
// stays high from M = 15 to M = 255.  All reductions are fixed-order wave
// butterflies plus an ordered LDS combine: results are bitwise reproducible.
#include <algorithm>
#include <cstdlib>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace disk {

// Work-group sizes: 256 threads (four resident per CU, one target each) for
// large batches; 1024 threads (one per CU, sixteen waves on one target) for
// batches too small to fill the chip.
constexpr int kOptThreads = 256;
constexpr int kOptThreadsWide = 1024;
constexpr int kMaxT = DISK_MAX_LAYERS * DISK_MAX_TAPS;  // 256
constexpr int kChunk = 8;                               // taps per gradient chunk

struct OptArgs {
    int B;
    const disk_target* desc;
    const int* taps;
    const float* targets;
    float* theta;
    float* psnr;
    int* steps;
    int* status;
    disk_opt_params p;
    const int* order;
    int* queue;
    float* scratch;
    size_t slot_floats;
    int max_side, max_T;
    unsigned long long* ticks;   // optional: device clock when each target finished
    // optional Adam state carried across calls, per Theta row like theta
    float* adam_m;
    float* adam_v;
    const int* start;            // optional: updates already applied per target
    float* loss;                 // optional: loss of the returned Theta per target
    int max_updates;             // > 0: at most this many updates per target in this call
};

struct TapO {
    int ix, iy;                 // floor(-o)
    float c00, c01, c10, c11;   // w * bilinear corner weights
    float fx, fy;               // fractions of -o
    int off;                    // iy * S + ix: the corner's canvas offset
    int inside;                 // tap_inside(P): all four corners within the zero frame
};

// Canvas element at a 32-bit element index: a scalar base plus one 32-bit
// vector byte offset per load (no 64-bit address arithmetic per tap).
__device__ __forceinline__ const float* at(const float* base, int idx) {
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) +
                                          static_cast<uint32_t>(idx) * 4u);
}

__device__ __forceinline__ int opt_pad(int M) { return (M + 1) / 2 + 1; }

// Reduce v over the work-group (NW waves) in a fixed order; every thread gets the sum.
template <int NW>
__device__ __forceinline__ float wg_sum(float v, float* red) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    return s;
}

template <int NW>
__device__ __forceinline__ float wg_max(float v, float* red) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float s = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = fmaxf(s, red[w]);
    return s;
}

// Lane geometry of an 8 x 8 block walk.
struct Walk {
    int M, S, P, nbx, nblk, inv;
    __device__ Walk(int M_, int S_, int P_) : M(M_), S(S_), P(P_) {
        nbx = (M + 7) >> 3;
        nblk = nbx * nbx;
        inv = (65536 + nbx - 1) / nbx;   // blk / nbx == (blk * inv) >> 16 for nbx <= 32, blk < 1024
    }
    // pixel of block `blk` for this lane; `act` false for lanes past the edge
    // (their index is clamped onto the canvas so every read stays in bounds)
    __device__ __forceinline__ int pixel(int blk, int& x, int& y, bool& act) const {
        const int lane = threadIdx.x & 63;
        const int by = (blk * inv) >> 16, bx = blk - by * nbx;
        x = (bx << 3) + (lane & 7);
        y = (by << 3) + (lane >> 3);
        act = x < M && y < M;
        return (min(y, M - 1) + P) * S + min(x, M - 1) + P;
    }
};

// Support boxes.  X_1 (the first layer's splats on the impulse) is nonzero
// only in a box around the centre, and X_{l+1}(p) reads X_l(p + d_i + ab), so
// the box of X_{l+1} is that of X_l moved by -d_i - ab over the layer's taps
// (clipped to the M x M interior).  Passes skip the 8 x 8 blocks that miss the
// box they need; an empty box has x0 > x1.
struct Box {
    int x0, x1, y0, y1;
};
__device__ __forceinline__ bool block_meets(const Walk& wk, int blk, const Box& b) {
    const int by = (blk * wk.inv) >> 16, bx = blk - by * wk.nbx;
    const int x = bx << 3, y = by << 3;
    return x <= b.x1 && x + 7 >= b.x0 && y <= b.y1 && y + 7 >= b.y0;
}
__device__ __forceinline__ Box load_box(const int* v) {
    return Box{uniform(v[0]), uniform(v[1]), uniform(v[2]), uniform(v[3])};
}

// Value of a corner read that may leave the frame (masked path).
__device__ __forceinline__ float masked(const float* buf, int x, int y, int dx, int dy, int M, int S, int P) {
    const int xx = x + dx, yy = y + dy;
    if (xx < 0 || xx >= M || yy < 0 || yy >= M) return 0.0f;
    return buf[(yy + P) * S + xx + P];
}

__device__ __forceinline__ bool tap_inside(const TapO& t, int P) {
    return t.ix >= -P && t.ix <= P - 1 && t.iy >= -P && t.iy <= P - 1;
}

// One tap's contribution at a pixel: forward p + (ix+a, iy+b); transpose q - (ix+a, iy+b).
template <int SGN>
__device__ __forceinline__ float gather_tap(float acc, const TapO& t, const float* __restrict__ src, int base, int x,
                                            int y, const Walk& wk) {
    const int M = wk.M, S = wk.S, P = wk.P;
    if (t.inside) {
        const int q = base + SGN * t.off;
        acc = fmaf(t.c00, *at(src, q), acc);
        acc = fmaf(t.c01, *at(src, q + SGN), acc);
        acc = fmaf(t.c10, *at(src, q + SGN * S), acc);
        acc = fmaf(t.c11, *at(src, q + SGN * (S + 1)), acc);
    } else {
        const int xc = min(x, M - 1), yc = min(y, M - 1);
        acc = fmaf(t.c00, masked(src, xc, yc, SGN * t.ix, SGN * t.iy, M, S, P), acc);
        acc = fmaf(t.c01, masked(src, xc, yc, SGN * (t.ix + 1), SGN * t.iy, M, S, P), acc);
        acc = fmaf(t.c10, masked(src, xc, yc, SGN * t.ix, SGN * (t.iy + 1), M, S, P), acc);
        acc = fmaf(t.c11, masked(src, xc, yc, SGN * (t.ix + 1), SGN * (t.iy + 1), M, S, P), acc);
    }
    return acc;
}

// Where a gathered pixel goes: a plain store, or, for the last forward layer,
// the loss terms of the chain output (NMSE, Eq. 11, or Charbonnier) and
// dL/dK_syn written in place of K_syn.
struct StoreOut {
    static constexpr bool kEvery = false;   // blocks outside both boxes need no store
    float* dst;
    __device__ __forceinline__ void operator()(int base, int, int, bool act, float acc) {
        if (act) dst[base] = acc;
    }
};
struct LossOut {
    static constexpr bool kEvery = true;    // every pixel enters the loss
    float* dst;
    const float* tgt;
    int M, charb;
    float pk, inv_pk2, n, ce;
    float se, ch;   // this lane's sums, in block order
    __device__ __forceinline__ void operator()(int base, int x, int y, bool act, float acc) {
        if (act) {
            const float dv = acc - tgt[y * M + x];
            se = fmaf(dv, dv, se);
            float g;
            if (charb) {
                const float dn = dv / pk;
                const float r = sqrtf(fmaf(dn, dn, ce * ce));
                ch += r;
                g = dn / (r * n * pk);
            } else {
                g = 2.0f * dv * inv_pk2 / n;
            }
            dst[base] = g;
        }
    }
};

// out(p, sum_taps sum_ab c_ab src[p + sgn * d_ab]) over the interior (sgn = +1:
// forward gather; sgn = -1: the transpose, used for G_{l-1}).  Taps go four at
// a time: when all four stay inside the zero frame their 16 reads are issued
// together before the FMAs (same accumulation order as one tap at a time).
// Blocks that miss `box` (where the sum is zero, or not needed) take 0 without
// reading; of those, the ones that also miss `zbox` are skipped unless Out
// needs every pixel.
template <int NW, int SGN, class Out>
__device__ void gather_layer(const float* __restrict__ src, const TapO* tp, int N, const Walk& wk, Out& out,
                             const Box& box, const Box& zbox) {
    const int wave = threadIdx.x >> 6;
    const int S = wk.S;
    for (int blk = wave; blk < wk.nblk; blk += NW) {
        const bool hit = block_meets(wk, blk, box);
        if (!hit && !Out::kEvery && !block_meets(wk, blk, zbox)) continue;
        int x, y;
        bool act;
        const int base = wk.pixel(blk, x, y, act);
        float acc = 0.0f;
        int i = 0;
        if (!hit) i = N;
        for (; i + 4 <= N; i += 4) {
            TapO t[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) t[k] = tp[i + k];
            if (t[0].inside & t[1].inside & t[2].inside & t[3].inside) {
                float v[4][4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int q = base + SGN * uniform(t[k].off);
                    v[k][0] = *at(src, q);
                    v[k][1] = *at(src, q + SGN);
                    v[k][2] = *at(src, q + SGN * S);
                    v[k][3] = *at(src, q + SGN * (S + 1));
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    acc = fmaf(t[k].c00, v[k][0], acc);
                    acc = fmaf(t[k].c01, v[k][1], acc);
                    acc = fmaf(t[k].c10, v[k][2], acc);
                    acc = fmaf(t[k].c11, v[k][3], acc);
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) acc = gather_tap<SGN>(acc, t[k], src, base, x, y, wk);
            }
        }
        for (; i < N; ++i) acc = gather_tap<SGN>(acc, tp[i], src, base, x, y, wk);
        out(base, x, y, act, acc);
    }
}

// Backward of a layer past the first, in one pass over the canvas.  The tap
// correlations S_ab(i) = sum_p G(p) X(p + d_i + ab) equal, with q = p + d_i +
// ab, sum_q X(q) G(q - d_i - ab): the same G values the transposed gather
// G'(q) = sum_i sum_ab c_ab G(q - d_i - ab) reads.  So each lane reads X(q)
// once and the 4 N values of G once, and accumulates both: G' of all N <= NT
// taps (in the order of gather_layer<-1>) and the sums of the first NS taps
// (registers; the later taps' sums are taken beforehand by the plain
// correlation pass, since G'(q) then overwrites X(q), which only this lane
// reads).  The sums go through the fixed-order wave + LDS reduction into sS.
constexpr int kFuseS = 8;      // taps whose sums the fused pass accumulates
constexpr int kFuseMax = 12;   // taps per layer up to which the fused pass runs
template <int NW, int NS, int NT>
__device__ __forceinline__ void fused_backward(const float* __restrict__ G, float* X, const TapO* tp, int N,
                                               const Walk& wk, float (*sS)[4], float* red, const Box& box) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int S = wk.S;
    float s[NS][4];
    int off[NT];
    bool all_in = true;
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) s[k][ab] = 0.0f;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        off[k] = 0;
        if (k < N) {
            off[k] = uniform(tp[k].off);
            all_in = all_in && tp[k].inside;
        }
    }
    for (int blk = wave; blk < wk.nblk; blk += NW) {
        // outside the box of X: X = 0 (no sums) and G' is not needed
        if (!block_meets(wk, blk, box)) continue;
        int x, y;
        bool act;
        const int base = wk.pixel(blk, x, y, act);
        const float xv = act ? *at(X, base) : 0.0f;
        float gl = 0.0f;
        if (all_in) {
#pragma unroll
            for (int k0 = 0; k0 < NT; k0 += 4) {
                if (k0 < N) {
                    float v[4][4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int q = base - off[k0 + k];
                        v[k][0] = *at(G, q);
                        v[k][1] = *at(G, q - 1);
                        v[k][2] = *at(G, q - S);
                        v[k][3] = *at(G, q - (S + 1));
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (k0 + k < N) {
                            const TapO& t = tp[k0 + k];
                            gl = fmaf(t.c00, v[k][0], gl);
                            gl = fmaf(t.c01, v[k][1], gl);
                            gl = fmaf(t.c10, v[k][2], gl);
                            gl = fmaf(t.c11, v[k][3], gl);
                            if (k0 + k < NS)
#pragma unroll
                                for (int ab = 0; ab < 4; ++ab)
                                    s[k0 + k][ab] = fmaf(xv, v[k][ab], s[k0 + k][ab]);
                        }
                    }
                }
            }
        } else {
            const int M = wk.M, P = wk.P;
            const int xc = min(x, M - 1), yc = min(y, M - 1);
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                if (k < N) {
                    const TapO t = tp[k];
                    float v[4];
                    if (t.inside) {
                        const int q = base - t.off;
                        v[0] = *at(G, q);
                        v[1] = *at(G, q - 1);
                        v[2] = *at(G, q - S);
                        v[3] = *at(G, q - (S + 1));
                    } else {
                        v[0] = masked(G, xc, yc, -t.ix, -t.iy, M, S, P);
                        v[1] = masked(G, xc, yc, -(t.ix + 1), -t.iy, M, S, P);
                        v[2] = masked(G, xc, yc, -t.ix, -(t.iy + 1), M, S, P);
                        v[3] = masked(G, xc, yc, -(t.ix + 1), -(t.iy + 1), M, S, P);
                    }
                    gl = fmaf(t.c00, v[0], gl);
                    gl = fmaf(t.c01, v[1], gl);
                    gl = fmaf(t.c10, v[2], gl);
                    gl = fmaf(t.c11, v[3], gl);
                    if (k < NS)
#pragma unroll
                        for (int ab = 0; ab < 4; ++ab) s[k][ab] = fmaf(xv, v[ab], s[k][ab]);
                }
            }
        }
        if (act) X[base] = gl;
    }
    // fixed-order reduction of the first min(N, NS) taps' sums
    const int ns = min(N, NS);
#pragma unroll
    for (int k = 0; k < NS; ++k)
        if (k < ns)
#pragma unroll
            for (int ab = 0; ab < 4; ++ab) {
                const float v = wave_sum(s[k][ab]);
                if (lane == 0) red[(wave * NS + k) * 4 + ab] = v;
            }
    __syncthreads();
    if (tid < 4 * ns) {
        const int k = tid >> 2, ab = tid & 3;
        float v = 0.0f;
        for (int w = 0; w < NW; ++w) v += red[(w * NS + k) * 4 + ab];
        sS[k][ab] = v;
    }
}

template <int NTH>
__global__ __launch_bounds__(NTH, NTH == kOptThreads ? 4 : 1) void opt_kernel(OptArgs a) {
    constexpr int kOptWaves = NTH / 64;
    constexpr int kOptThreads = NTH;
    __shared__ float th[kMaxT * 3], am[kMaxT * 3], av[kMaxT * 3], gr[kMaxT * 3];
    __shared__ TapO tap[kMaxT];
    __shared__ float sS[kMaxT][4];
    __shared__ float red[kOptWaves * (kChunk > kFuseS ? kChunk : kFuseS) * 4];
    __shared__ int s_q;
    __shared__ int t0[DISK_MAX_LAYERS + 1];
    // support boxes (x0, x1, y0, y1) of X_1..X_L this step and the last one
    __shared__ int s_box[DISK_MAX_LAYERS + 1][4], s_pbox[DISK_MAX_LAYERS + 1][4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    float* slot = a.scratch + blockIdx.x * a.slot_floats;

    for (;;) {
        if (tid == 0) s_q = atomicAdd(a.queue, 1);
        __syncthreads();
        const int q = s_q;
        __syncthreads();
        if (q >= a.B) break;
        const int b = a.order[q];
        const disk_target d = a.desc[b];
        const int M = d.side, L = d.L, P = opt_pad(M), S = M + 2 * P;
        const int* ntap = a.taps + d.taps_off;
        // validate the descriptor (it lives on the device): a malformed target
        // is skipped with status 3
        bool bad = M < 1 || (M & 1) == 0 || M > a.max_side || L < 1 || L > DISK_MAX_LAYERS ||
                   d.taps_off < 0 || d.theta_off < 0 || d.target_off < 0;
        int T = 0;
        if (!bad)
            for (int l = 0; l < L; ++l) {
                bad |= ntap[l] < 1 || ntap[l] > DISK_MAX_TAPS;
                T += ntap[l];
            }
        bad |= T > a.max_T || static_cast<size_t>(M + 2 * P) * (M + 2 * P) * L > a.slot_floats;
        const int s0 = a.start ? a.start[b] : 0;   // resumed schedule position
        bad |= s0 < 0;
        if (bad) {
            if (tid == 0) {
                a.psnr[b] = 0.0f;
                a.steps[b] = 0;
                a.status[b] = 3;
                if (a.loss) a.loss[b] = 0.0f;
                if (a.ticks) a.ticks[b] = wall_clock64();
            }
            __syncthreads();
            continue;
        }
        if (tid == 0) {
            t0[0] = 0;
            for (int l = 0; l < L; ++l) t0[l + 1] = t0[l] + ntap[l];
        }
        const float* tgt = a.targets + d.target_off;
        float* theta_g = a.theta + 3 * static_cast<size_t>(d.theta_off);
        const size_t SS = static_cast<size_t>(S) * S;
        const Walk wk(M, S, P);
        const int c = (M - 1) / 2;          // impulse centre (both axes)
        const float n = static_cast<float>(M) * M;

        // ---- target setup: parameters, moments, zeroed canvases, peak -------
        {
            const float* am_g = a.adam_m ? a.adam_m + 3 * static_cast<size_t>(d.theta_off) : nullptr;
            const float* av_g = a.adam_v ? a.adam_v + 3 * static_cast<size_t>(d.theta_off) : nullptr;
            for (int i = tid; i < 3 * T; i += kOptThreads) {
                th[i] = theta_g[i];
                am[i] = am_g ? am_g[i] : 0.0f;
                av[i] = av_g ? av_g[i] : 0.0f;
            }
        }
        // the last schedule position this call may reach
        const int step_end = a.max_updates > 0 ? min(a.p.max_steps, s0 + a.max_updates) : a.p.max_steps;
        for (size_t i = tid; i < SS * L; i += kOptThreads) slot[i] = 0.0f;
        if (tid < 4 * (DISK_MAX_LAYERS + 1)) s_box[tid >> 2][tid & 3] = (tid & 1) ? -1 : M;   // empty: the canvases are zero
        float pk = -INFINITY;
        for (int i = tid; i < M * M; i += kOptThreads) pk = fmaxf(pk, tgt[i]);
        pk = wg_max<kOptWaves>(pk, red);
        const float inv_pk2 = 1.0f / (pk * pk);
        // beta^t after the s0 updates already applied (the same products an
        // uninterrupted run forms one step at a time)
        float b1t = 1.0f, b2t = 1.0f;
        for (int k = 0; k < s0; ++k) {
            b1t *= a.p.beta1;
            b2t *= a.p.beta2;
        }
        float psnr = 0.0f, loss = 0.0f;
        int status = 0, step = 0;
        __syncthreads();

        for (step = s0;; ++step) {
            // ---- taps of the current Theta --------------------------------
            for (int i = tid; i < T; i += kOptThreads) {
                const float ox = th[3 * i], oy = th[3 * i + 1], w = th[3 * i + 2];
                TapO t;
                floor_frac(-ox, t.ix, t.fx);
                floor_frac(-oy, t.iy, t.fy);
                const float wy1 = w * t.fy, wy0 = w - wy1;
                t.c01 = wy0 * t.fx;
                t.c00 = wy0 - t.c01;
                t.c11 = wy1 * t.fx;
                t.c10 = wy1 - t.c11;
                t.off = t.iy * S + t.ix;
                t.inside = tap_inside(t, P) ? 1 : 0;
                tap[i] = t;
            }
            __syncthreads();
            if (tid == 0) {
                // last step's boxes: where the canvases may still hold values
                for (int j = 0; j <= L; ++j)
                    for (int k = 0; k < 4; ++k) s_pbox[j][k] = s_box[j][k];
                int bx0 = 0, bx1 = -1, by0 = 0, by1 = -1;
                for (int l = 0; l < L; ++l) {
                    // X_{l+1} from X_l (l = 0: the impulse at (c, c))
                    if (l == 0) {
                        bx0 = bx1 = by0 = by1 = c;
                    } else if (bx0 > bx1 || by0 > by1) {
                        s_box[l + 1][0] = M, s_box[l + 1][1] = -1, s_box[l + 1][2] = M, s_box[l + 1][3] = -1;
                        continue;
                    }
                    int mnx = tap[t0[l]].ix, mxx = mnx, mny = tap[t0[l]].iy, mxy = mny;
                    for (int i = t0[l] + 1; i < t0[l + 1]; ++i) {
                        mnx = min(mnx, tap[i].ix);
                        mxx = max(mxx, tap[i].ix);
                        mny = min(mny, tap[i].iy);
                        mxy = max(mxy, tap[i].iy);
                    }
                    bx0 = max(bx0 - mxx - 1, 0);
                    bx1 = min(bx1 - mnx, M - 1);
                    by0 = max(by0 - mxy - 1, 0);
                    by1 = min(by1 - mny, M - 1);
                    const bool empty = bx0 > bx1 || by0 > by1;
                    s_box[l + 1][0] = empty ? M : bx0;
                    s_box[l + 1][1] = empty ? -1 : bx1;
                    s_box[l + 1][2] = empty ? M : by0;
                    s_box[l + 1][3] = empty ? -1 : by1;
                }
            }
            __syncthreads();

            // ---- forward: X_1 = splats of layer 1 on the impulse ------------
            float* X1 = slot + (L == 1 ? 0 : SS);
            // blocks outside X_1's box hold zeros (written only where last step's
            // values may remain; a one-layer chain's canvas holds G everywhere)
            const Box b1 = load_box(s_box[1]);
            const Box z1 = L == 1 ? Box{0, M - 1, 0, M - 1} : load_box(s_pbox[1]);
            for (int blk = wave; blk < wk.nblk; blk += kOptWaves) {
                const bool hit = block_meets(wk, blk, b1);
                if (!hit && !block_meets(wk, blk, z1)) continue;
                int x, y;
                bool act;
                const int base = wk.pixel(blk, x, y, act);
                float acc = 0.0f;
                for (int i = 0; hit && i < ntap[0]; ++i) {
                    const TapO t = tap[i];
                    // corner (a, b) of pixel p reads p + (ix+a, iy+b); the impulse is at c
                    const int ax = c - x - t.ix, ay = c - y - t.iy;
                    if (ax >= 0 && ax <= 1 && ay >= 0 && ay <= 1)
                        acc += ay == 0 ? (ax == 0 ? t.c00 : t.c01) : (ax == 0 ? t.c10 : t.c11);
                }
                if (act) X1[base] = acc;
            }
            __syncthreads();
            // ---- loss, PSNR, G_L (in place of K_syn): in the last layer's pass,
            // or over X_1 for a one-layer chain -----------------------------
            float se = 0.0f, ch = 0.0f;
            const float ce = a.p.charb_eps;
            for (int l = 1; l < L; ++l) {
                const float* src = slot + l * SS;
                const Box bo = load_box(s_box[l + 1]);
                if (l < L - 1) {
                    StoreOut o{slot + (l + 1) * SS};
                    gather_layer<kOptWaves, 1>(src, tap + t0[l], ntap[l], wk, o, bo, load_box(s_pbox[l + 1]));
                } else {
                    LossOut o{slot, tgt, M, a.p.loss == DISK_LOSS_CHARBONNIER, pk, inv_pk2, n, ce, 0.0f, 0.0f};
                    gather_layer<kOptWaves, 1>(src, tap + t0[l], ntap[l], wk, o, bo, bo);
                    se = o.se;
                    ch = o.ch;
                }
                __syncthreads();
            }
            if (L == 1) {
                LossOut o{slot, tgt, M, a.p.loss == DISK_LOSS_CHARBONNIER, pk, inv_pk2, n, ce, 0.0f, 0.0f};
                for (int blk = wave; blk < wk.nblk; blk += kOptWaves) {
                    int x, y;
                    bool act;
                    const int base = wk.pixel(blk, x, y, act);
                    o(base, x, y, act, slot[base]);
                }
                se = o.se;
                ch = o.ch;
            }
            se = wg_sum<kOptWaves>(se, red);
            if (a.p.loss == DISK_LOSS_CHARBONNIER) ch = wg_sum<kOptWaves>(ch, red);
            const float nmse = se * inv_pk2 / n;
            loss = a.p.loss == DISK_LOSS_CHARBONNIER ? ch / n : nmse;
            psnr = nmse > 0.0f ? -10.0f * log10f(nmse) : INFINITY;
            if (!isfinite(loss)) {
                status = 2;
                break;
            }
            if (psnr >= a.p.psnr_stop_db) {
                status = 1;
                break;
            }
            if (step >= step_end) break;

            // ---- backward ----------------------------------------------------
            for (int l = L - 1; l >= 0; --l) {
                const float* G = slot + (l == L - 1 ? 0 : (l + 1) * SS);   // G_{l+1} (1-based l+1)
                const TapO* tp = tap + t0[l];
                const int N = ntap[l];
                if (l == 0) {
                    // layer 1 reads the impulse: S_ab = G_1[c - d_ab]
                    for (int i = tid; i < N; i += kOptThreads) {
                        const TapO t = tp[i];
#pragma unroll
                        for (int ab = 0; ab < 4; ++ab) {
                            const int px = c - t.ix - (ab & 1), py = c - t.iy - (ab >> 1);
                            sS[i][ab] = (px >= 0 && px < M && py >= 0 && py < M) ? G[(py + P) * S + px + P] : 0.0f;
                        }
                    }
                } else {
                    const float* X = slot + l * SS;   // X_l (1-based), input of this layer
                    // up to kFuseMax taps the fused pass below takes the first kFuseS
                    // taps' sums; the rest (all of them for wider layers) come from
                    // the correlation pass here, which must precede it
                    const bool fuse = N <= kFuseMax;
                    // p outside the output's box reads only zeros of X: G(p) X(p + d) = 0
                    const Box ob = load_box(s_box[l + 1]);
                    for (int i0 = fuse ? kFuseS : 0; i0 < N; i0 += kChunk) {
                        const int nc = min(kChunk, N - i0);
                        float s[kChunk][4];
#pragma unroll
                        for (int k = 0; k < kChunk; ++k)
#pragma unroll
                            for (int ab = 0; ab < 4; ++ab) s[k][ab] = 0.0f;
                        // the chunk's canvas offsets (wave-uniform); when all taps stay
                        // inside the zero frame the 4 kChunk reads of a pixel go out together
                        int off[kChunk];
                        bool all_in = (nc & 3) == 0;
#pragma unroll
                        for (int k = 0; k < kChunk; ++k) {
                            off[k] = 0;
                            if (k < nc) {
                                const TapO t = tp[i0 + k];
                                off[k] = uniform(t.off);
                                all_in = all_in && t.inside;
                            }
                        }
                        if (all_in) {
                            for (int blk = wave; blk < wk.nblk; blk += kOptWaves) {
                                if (!block_meets(wk, blk, ob)) continue;
                                int x, y;
                                bool act;
                                const int base = wk.pixel(blk, x, y, act);
                                const float g = act ? G[base] : 0.0f;
#pragma unroll
                                for (int k0 = 0; k0 < kChunk; k0 += 4) {
                                    if (k0 >= nc) break;
                                    float v[4][4];
#pragma unroll
                                    for (int k = 0; k < 4; ++k) {
                                        const int q = base + off[k0 + k];
                                        v[k][0] = *at(X, q);
                                        v[k][1] = *at(X, q + 1);
                                        v[k][2] = *at(X, q + S);
                                        v[k][3] = *at(X, q + S + 1);
                                    }
#pragma unroll
                                    for (int k = 0; k < 4; ++k)
#pragma unroll
                                        for (int ab = 0; ab < 4; ++ab)
                                            s[k0 + k][ab] = fmaf(g, v[k][ab], s[k0 + k][ab]);
                                }
                            }
                        } else {
                        for (int blk = wave; blk < wk.nblk; blk += kOptWaves) {
                            if (!block_meets(wk, blk, ob)) continue;
                            int x, y;
                            bool act;
                            const int base = wk.pixel(blk, x, y, act);
                            const float g = act ? G[base] : 0.0f;
#pragma unroll
                            for (int k = 0; k < kChunk; ++k) {
                                if (k < nc) {
                                    const TapO t = tp[i0 + k];
                                    float v00, v01, v10, v11;
                                    if (t.inside) {
                                        const int q = base + t.off;
                                        v00 = *at(X, q);
                                        v01 = *at(X, q + 1);
                                        v10 = *at(X, q + S);
                                        v11 = *at(X, q + S + 1);
                                    } else {
                                        const int xc = min(x, M - 1), yc = min(y, M - 1);
                                        v00 = masked(X, xc, yc, t.ix, t.iy, M, S, P);
                                        v01 = masked(X, xc, yc, t.ix + 1, t.iy, M, S, P);
                                        v10 = masked(X, xc, yc, t.ix, t.iy + 1, M, S, P);
                                        v11 = masked(X, xc, yc, t.ix + 1, t.iy + 1, M, S, P);
                                    }
                                    s[k][0] = fmaf(g, v00, s[k][0]);
                                    s[k][1] = fmaf(g, v01, s[k][1]);
                                    s[k][2] = fmaf(g, v10, s[k][2]);
                                    s[k][3] = fmaf(g, v11, s[k][3]);
                                }
                            }
                        }
                        }
                        // fixed-order reduction of the chunk's 4 * nc sums
#pragma unroll
                        for (int k = 0; k < kChunk; ++k)
#pragma unroll
                            for (int ab = 0; ab < 4; ++ab) {
                                const float v = wave_sum(s[k][ab]);
                                if (lane == 0) red[(wave * kChunk + k) * 4 + ab] = v;
                            }
                        __syncthreads();
                        if (tid < 4 * nc) {
                            const int k = tid >> 2, ab = tid & 3;
                            float v = 0.0f;
                            for (int w = 0; w < kOptWaves; ++w) v += red[(w * kChunk + k) * 4 + ab];
                            sS[i0 + k][ab] = v;
                        }
                        __syncthreads();
                    }
                    // correlations of the first taps and G_l (1-based) in one pass; G_l replaces X_l
                    if (fuse) fused_backward<kOptWaves, kFuseS, kFuseMax>(G, slot + l * SS, tp, N, wk, sS, red, load_box(s_box[l]));
                }
                __syncthreads();
                // dTheta of this layer's taps
                for (int i = tid; i < N; i += kOptThreads) {
                    const TapO t = tp[i];
                    const float w = th[3 * (t0[l] + i) + 2];
                    const float S00 = sS[i][0], S01 = sS[i][1], S10 = sS[i][2], S11 = sS[i][3];
                    const float fx = t.fx, fy = t.fy;
                    gr[3 * (t0[l] + i) + 0] = -w * ((1.0f - fy) * (S01 - S00) + fy * (S11 - S10));
                    gr[3 * (t0[l] + i) + 1] = -w * ((1.0f - fx) * (S10 - S00) + fx * (S11 - S01));
                    gr[3 * (t0[l] + i) + 2] =
                        (1.0f - fy) * ((1.0f - fx) * S00 + fx * S01) + fy * ((1.0f - fx) * S10 + fx * S11);
                }
                if (l > 0 && N > kFuseMax) {
                    // G_l (1-based) = transpose of layer l+1 applied to G_{l+1}, into X_l's canvas
                    StoreOut o{slot + l * SS};
                    // needed (and written) only in X_l's box: the canvas keeps its zeros elsewhere
                    const Box none{M, -1, M, -1};
                    gather_layer<kOptWaves, -1>(G, tp, N, wk, o, load_box(s_box[l]), none);
                }
                __syncthreads();
            }

            // ---- Adam ----------------------------------------------------------
            const float lr = a.p.max_steps > 1
                                 ? a.p.lr0 + (a.p.lr1 - a.p.lr0) * (static_cast<float>(step) /
                                                                     static_cast<float>(a.p.max_steps - 1))
                                 : a.p.lr0;
            b1t *= a.p.beta1;
            b2t *= a.p.beta2;
            const float bc1 = 1.0f - b1t, bc2 = 1.0f - b2t;
            // learning-rate unit of the offsets: pixels, or the target's half-width
            const float lr_o =
                a.p.offset_units == DISK_OFFSETS_HALF_WIDTH ? lr * (0.5f * static_cast<float>(M - 1)) : lr;
            for (int i = tid; i < 3 * T; i += kOptThreads) {
                const float g = gr[i];
                const float m = fmaf(a.p.beta1, am[i], (1.0f - a.p.beta1) * g);
                const float v = fmaf(a.p.beta2, av[i], (1.0f - a.p.beta2) * g * g);
                am[i] = m;
                av[i] = v;
                th[i] -= (i % 3 == 2 ? lr : lr_o) * (m / bc1) / (sqrtf(v / bc2) + a.p.eps);
            }
            __syncthreads();
        }

        {
            float* am_g = a.adam_m ? a.adam_m + 3 * static_cast<size_t>(d.theta_off) : nullptr;
            float* av_g = a.adam_v ? a.adam_v + 3 * static_cast<size_t>(d.theta_off) : nullptr;
            for (int i = tid; i < 3 * T; i += kOptThreads) {
                theta_g[i] = th[i];
                if (am_g) am_g[i] = am[i];
                if (av_g) av_g[i] = av[i];
            }
        }
        if (tid == 0) {
            a.psnr[b] = psnr;
            a.steps[b] = step;
            a.status[b] = status;
            if (a.loss) a.loss[b] = loss;
            if (a.ticks) a.ticks[b] = wall_clock64();
        }
        __syncthreads();
    }
}

// Order targets by decreasing cost (side^2 x taps) with a bucketed counting
// sort in one work-group, and reset the work queue.
constexpr int kOrderBuckets = 4096;
__global__ __launch_bounds__(1024) void opt_order_kernel(int B, const disk_target* __restrict__ desc,
                                                         const int* __restrict__ taps, int* __restrict__ order,
                                                         int* __restrict__ queue, unsigned long long* ticks) {
    if (ticks && threadIdx.x == 0) ticks[B] = wall_clock64();   // the launch's start
    __shared__ int hist[kOrderBuckets];
    for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    auto key = [&](int b) {
        const disk_target d = desc[b];
        int T = 0;
        for (int l = 0; l < d.L; ++l) T += taps[d.taps_off + l];
        const float cost = static_cast<float>(d.side) * d.side * max(T, 1);
        // log-spaced buckets, largest cost -> bucket 0
        const int k = static_cast<int>(log2f(cost) * 128.0f);
        return kOrderBuckets - 1 - min(max(k, 0), kOrderBuckets - 1);
    };
    for (int b = threadIdx.x; b < B; b += blockDim.x) atomicAdd(&hist[key(b)], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int i = 0; i < kOrderBuckets; ++i) {
            const int h = hist[i];
            hist[i] = run;
            run += h;
        }
        *queue = 0;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x) order[atomicAdd(&hist[key(b)], 1)] = b;
}

// Continuation start of basis entry k (k >= 1): Theta_k = Theta*_{k-1} with its
// offsets scaled by `scale` and its weights copied, when both entries have the
// same layer structure; otherwise Theta_k stays as given.
__global__ __launch_bounds__(64) void continue_kernel(const disk_target* __restrict__ desc,
                                                      const int* __restrict__ taps, float* __restrict__ theta, int k,
                                                      float scale) {
    const disk_target a = desc[k - 1], b = desc[k];
    if (a.L != b.L || a.L < 1 || a.L > DISK_MAX_LAYERS || a.taps_off < 0 || b.taps_off < 0 || a.theta_off < 0 ||
        b.theta_off < 0)
        return;
    int T = 0;
    for (int l = 0; l < a.L; ++l) {
        const int na = taps[a.taps_off + l], nb = taps[b.taps_off + l];
        if (na != nb || na < 1 || na > DISK_MAX_TAPS) return;
        T += na;
    }
    const float* src = theta + 3 * static_cast<size_t>(a.theta_off);
    float* dst = theta + 3 * static_cast<size_t>(b.theta_off);
    for (int i = threadIdx.x; i < 3 * T; i += 64) dst[i] = (i % 3 == 2) ? src[i] : src[i] * scale;
}

hipError_t launch_continue(const disk_target* desc, const int* taps, float* theta, int k, float scale,
                           hipStream_t s) {
    hipLaunchKernelGGL(continue_kernel, dim3(1), dim3(64), 0, s, desc, taps, theta, k, scale);
    return hipGetLastError();
}

// Resident work-groups: `per_cu` per compute unit (each owns one target at a
// time; at most 4 of 256 threads, or 1 of 1024), at most one per target.
int opt_workgroups(int B, int per_cu, int threads) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        n = 256;
    per_cu = std::max(1, std::min(per_cu, threads == kOptThreadsWide ? 1 : 4));
    return std::max(1, std::min(B, per_cu * n));
}

size_t opt_slot_floats(int max_side, int max_L) {
    const int S = max_side + 2 * ((max_side + 1) / 2 + 1);
    return (static_cast<size_t>(S) * S * max_L + 63) & ~size_t(63);
}

hipError_t launch_optimize(int B, const disk_target* desc, const int* taps, const float* targets, float* theta,
                           float* psnr, int* steps, int* status, const disk_opt_params& p, int* order, int* queue,
                           float* scratch, size_t slot_floats, int nwg, int max_side, int max_T,
                           const OptExtra& x, int threads, hipStream_t s) {
    hipLaunchKernelGGL(opt_order_kernel, dim3(1), dim3(1024), 0, s, B, desc, taps, order, queue, x.ticks);
    OptArgs a{B,     desc,  taps,    targets,     theta,    psnr,     steps,   status, p,
              order, queue, scratch, slot_floats, max_side, max_T,    x.ticks, x.adam_m, x.adam_v,
              x.start, x.loss, x.max_updates};
    if (threads == kOptThreadsWide)
        hipLaunchKernelGGL(opt_kernel<kOptThreadsWide>, dim3(nwg), dim3(kOptThreadsWide), 0, s, a);
    else
        hipLaunchKernelGGL(opt_kernel<kOptThreads>, dim3(nwg), dim3(kOptThreads), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Radial initialisation (Eq. 6), one work-group per target.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void init_radial_kernel(int B, const disk_target* __restrict__ desc,
                                                          const int* __restrict__ taps,
                                                          const float* __restrict__ targets,
                                                          float* __restrict__ theta, int max_side,
                                                          int max_T) {
    __shared__ float red[4];
    const int tid = threadIdx.x;
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        const disk_target d = desc[b];
        const int M = d.side, h = (M - 1) / 2;
        // same descriptor checks as the optimiser; a malformed target is left alone
        bool bad = M < 1 || (M & 1) == 0 || M > max_side || d.L < 1 || d.L > DISK_MAX_LAYERS ||
                   d.taps_off < 0 || d.theta_off < 0 || d.target_off < 0;
        if (!bad) {
            int T = 0;
            for (int l = 0; l < d.L; ++l) {
                bad |= taps[d.taps_off + l] < 1 || taps[d.taps_off + l] > DISK_MAX_TAPS;
                T += taps[d.taps_off + l];
            }
            bad |= T > max_T;
        }
        if (bad) continue;   // uniform across the block: every thread reads the same descriptor
        const float* K = targets + d.target_off;
        // total mass, then the smallest integer squared radius whose disk holds 99%
        float tot = 0.0f;
        for (int i = tid; i < M * M; i += 256) tot += K[i];
        auto wsum = [&](float v) {
            v = wave_sum(v);
            __syncthreads();
            if ((tid & 63) == 0) red[tid >> 6] = v;
            __syncthreads();
            return (red[0] + red[1]) + (red[2] + red[3]);
        };
        tot = wsum(tot);
        int lo = 0, hi = 2 * h * h;   // mass(hi) = tot
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            float m = 0.0f;
            for (int i = tid; i < M * M; i += 256) {
                const int y = i / M, x = i - y * M;
                const int dx = x - h, dy = y - h;
                if (dx * dx + dy * dy <= mid) m += K[i];
            }
            m = wsum(m);
            if (m >= 0.99f * tot)
                hi = mid;
            else
                lo = mid + 1;
        }
        const float R = fminf(static_cast<float>(h), sqrtf(static_cast<float>(lo)));
        const int L = d.L;
        const float dr = 2.0f * R / static_cast<float>(L * (L + 1));
        float* out = theta + 3 * static_cast<size_t>(d.theta_off);
        int off = 0;
        for (int l = 0; l < L; ++l) {
            const int N = taps[d.taps_off + l];
            const float r = static_cast<float>(l + 1) * dr;
            for (int i = tid; i < N; i += 256) {
                const float ang = 6.283185307179586f * static_cast<float>(i + 1) / static_cast<float>(N);
                out[3 * (off + i) + 0] = r * cosf(ang);
                out[3 * (off + i) + 1] = r * sinf(ang);
                out[3 * (off + i) + 2] = 1.0f / static_cast<float>(N);
            }
            off += N;
        }
        __syncthreads();
    }
}

hipError_t launch_init_radial(int B, const disk_target* desc, const int* taps, const float* targets, float* theta,
                              int max_side, int max_T, hipStream_t s) {
    const int nblk = std::max(1, std::min(B, 4096));
    hipLaunchKernelGGL(init_radial_kernel, dim3(nblk), dim3(256), 0, s, B, desc, taps, targets, theta,
                       max_side, max_T);
    return hipGetLastError();
}

}  // namespace disk
