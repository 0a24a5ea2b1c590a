// Learned initialiser: conv encoder + MLP on MFMA (gfx950), forward, backward
// and Adam.  Every contraction is one BF16 GEMM kernel with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16), fed by operand loaders that read the matrices
// in whichever layout they live in (row-major, column-major, or the 3x3
// stride-2 im2col view of an NHWC activation) and stage 64 x 32 tiles in LDS.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace disk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kConvWidth[6] = {32, 64, 128, 128, 256, 256};
constexpr int kFc0 = 512, kOut = 144, kSide = 64;
constexpr bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
static_assert(pow2(kSide) && pow2(kConvWidth[0]) && pow2(kConvWidth[1]) && pow2(kConvWidth[2]) &&
                  pow2(kConvWidth[3]) && pow2(kConvWidth[4]) && pow2(kConvWidth[5]),
              "the im2col index splits are shifts");
constexpr int kBM = 64, kBN = 64, kBK = 32;
// Operand tiles in LDS: rows of kBK BF16 (64 B: four 16-B chunks) with chunk c
// of row r stored at chunk c ^ ((r >> 2) & 3), so that the 16-B stores of four
// consecutive rows and the MFMA fragment reads (one chunk of 16 rows) fall on
// distinct banks.
__host__ __device__ constexpr int tile_off(int r, int c) { return r * kBK + ((c ^ ((r >> 2) & 3)) << 3); }
constexpr int kPre = 3;    // GEMM k-steps of operand loads in flight

__device__ __forceinline__ uint4 zero4() { return make_uint4(0u, 0u, 0u, 0u); }

// 16 zero bytes in device memory (never written): the source of the operand
// pieces that fall outside a matrix or into the convolution's zero padding.
__device__ uint4 g_zero16;

// 8 BF16 at p[off] when in, else zeros, as one unconditional load: the chosen
// address passes through an empty asm statement, so the compiler can neither
// make the load conditional nor select afterwards (conditional loads make it
// wait for every load in flight).
// (The pointer stays in the global address space: a generic one would make
// these flat loads, which the LDS waits count as well.)
typedef const __attribute__((address_space(1))) uint4 GlobalU4;
__device__ __forceinline__ uint4 load8_or_zero(const uint16_t* p, size_t off, bool in) {
    GlobalU4* q = in ? (GlobalU4*)(p + off) : (GlobalU4*)&g_zero16;
    asm volatile("" : "+v"(q));
    return *(const uint4*)q;
}

// ---- operand loaders ------------------------------------------------------
// A loader describes a matrix Op(row, k).  kContig loaders return the 8
// elements (row, k..k+7); the others return (row..row+7, k).
struct LdRow {   // Op(r, k) = p[r * ld + k]
    const uint16_t* p;
    int ld, rows, K;
    static constexpr bool kContig = true;
    __device__ void limit(int ke) { K = min(K, ke); }   // zeros from reduction index ke on
    __device__ uint4 fetch(int r, int k) const {
        return load8_or_zero(p, static_cast<size_t>(r) * ld + k, r < rows && k < K);
    }
};

struct LdCol {   // Op(r, k) = p[k * ld + r]
    const uint16_t* p;
    int ld, rows, K;
    static constexpr bool kContig = false;
    __device__ void limit(int ke) { K = min(K, ke); }
    __device__ uint4 fetch(int r, int k) const {
        return load8_or_zero(p, static_cast<size_t>(k) * ld + r, r < rows && k < K);
    }
};

// im2col of a 3x3 / stride 2 / zero-padding 1 convolution over NHWC x:
// Op(m, k) with m = (b, oy, ox) and k = (ky * 3 + kx) * Cin + ci.
// Every extent of this network is a power of two (64 x 64 input, stride 2,
// widths 32..256): the index splits are shifts (lg*), and tap / 3 for a tap
// below 9 is (tap * 11) >> 5.
struct Im2col {
    const uint16_t* x;
    int H, W, Cin, Ho, Wo, M, K;   // K = 9 Cin
    int lgHW, lgWo, lgCin;         // log2(Ho Wo), log2 Wo, log2 Cin
    // Cin >= 8: 8 channels of one tap (branch-free, so that loads of several
    // k-steps can be in flight at once).
    __device__ uint4 fetch_wide(int m, int k) const {
        const int b = m >> lgHW, r = m - (b << lgHW), oy = r >> lgWo, ox = r - (oy << lgWo);
        const int tap = k >> lgCin, ci = k - (tap << lgCin);
        const int ky = (tap * 11) >> 5, kx = tap - 3 * ky;
        const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
        return load8_or_zero(x, ((static_cast<size_t>(b) * H + iy) * W + ix) * Cin + ci,
                             m < M && k < K && iy >= 0 && iy < H && ix >= 0 && ix < W);
    }
    __device__ uint4 fetch8(int m, int k) const {
        if (Cin >= 8) return fetch_wide(m, k);
        if (m >= M || k >= K) return zero4();
        const int b = m >> lgHW, r = m - (b << lgHW), oy = r >> lgWo, ox = r - (oy << lgWo);
        // Cin == 1: 8 consecutive taps
        uint16_t e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int tap = k + j;   // used only below 9
            const int ky = (tap * 11) >> 5, kx = tap - 3 * ky;
            const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
            e[j] = (tap < 9 && iy >= 0 && iy < H && ix >= 0 && ix < W)
                       ? x[(static_cast<size_t>(b) * H + iy) * W + ix]
                       : static_cast<uint16_t>(0);
        }
        uint4 v;
        __builtin_memcpy(&v, e, 16);
        return v;
    }
};
struct LdIm2col : Im2col {   // Op(m, k); Cin >= 8 (the first convolution has its own kernel)
    static constexpr bool kContig = true;
    __device__ void limit(int ke) { K = min(K, ke); }
    __device__ uint4 fetch(int r, int k) const { return fetch_wide(r, k); }
};
struct LdIm2colT : Im2col {  // Op(j, m) = im2col(m, j): rows j..j+7 at reduction index m
    static constexpr bool kContig = false;
    __device__ void limit(int ke) { M = min(M, ke); }
    __device__ uint4 fetch(int r, int k) const { return fetch8(k, r); }
};

// Input gradient of a 3 x 3 / stride 2 / padding 1 convolution by parity
// class: input pixel (iy, ix) = (2 j + py, 2 i + px) receives from the taps
// with iy + 1 - ky even, i.e. ky = 1 (py = 0) or ky = 0, 2 (py = 1), from
// output row oy = (iy + 1 - ky) / 2 (likewise x).  Per class (py, px) the
// gradient is a GEMM with rows m = (b, j, i) over B * Ho * Ho pixels, columns
// ci, and reduction index k = t * Cout + co over the class's (1 + py)(1 + px)
// taps t (ty = t / nx, tx = t % nx, nx = 1 + px).
struct SubpixTap {
    int py, px, lgHo, lgCo, Ho, Co;
    __device__ __forceinline__ void tap(int t, int& ky, int& kx) const {
        const int ty = px ? t >> 1 : t, tx = px ? t & 1 : 0;
        ky = py ? 2 * ty : 1;
        kx = px ? 2 * tx : 1;
    }
};
struct LdSubpixG : SubpixTap {   // Op(m, k) = g(b, oy, ox, co): 8 consecutive co
    const uint16_t* g;           // output gradient, NHWC [B][Ho][Ho][Co]
    int M, K;
    static constexpr bool kContig = true;
    __device__ void limit(int ke) { K = min(K, ke); }
    __device__ uint4 fetch(int m, int k) const {
        const int b = m >> (2 * lgHo), j = (m >> lgHo) & (Ho - 1), i = m & (Ho - 1);
        const int t = k >> lgCo, co = k & (Co - 1);
        int ky, kx;
        tap(t, ky, kx);
        const int oy = (2 * j + py + 1 - ky) >> 1, ox = (2 * i + px + 1 - kx) >> 1;
        return load8_or_zero(g, ((static_cast<size_t>(b) * Ho + oy) * Ho + ox) * Co + co,
                             m < M && k < K && oy < Ho && ox < Ho);
    }
};
struct LdSubpixW : SubpixTap {   // Op(ci, k) = W(co, ky, kx, ci): rows ci..ci+7 at k
    const uint16_t* wp;          // packed weights [Co][Kp], k = (ky 3 + kx) Cin + ci
    int Kp, Cin, K;
    static constexpr bool kContig = false;
    __device__ void limit(int ke) { K = min(K, ke); }
    __device__ uint4 fetch(int ci, int k) const {
        const int t = k >> lgCo, co = k & (Co - 1);
        int ky, kx;
        tap(t, ky, kx);
        return load8_or_zero(wp, static_cast<size_t>(co) * Kp + (ky * 3 + kx) * Cin + ci, ci < Cin && k < K);
    }
};

template <class LD>
__device__ __forceinline__ uint4 tile_fetch(const LD& ld, int row0, int k0, int t) {
    if constexpr (LD::kContig)
        return ld.fetch(row0 + (t >> 2), k0 + (t & 3) * 8);
    else
        return ld.fetch(row0 + (t & 7) * 8, k0 + (t >> 3));
}

template <class LD>
__device__ __forceinline__ void tile_store(uint16_t* S, int t, uint4 v) {
    if constexpr (LD::kContig) {
        *reinterpret_cast<uint4*>(S + tile_off(t >> 2, t & 3)) = v;
    } else {
        uint16_t e[8];
        __builtin_memcpy(e, &v, 16);
        const int r = (t & 7) * 8, k = t >> 3;
#pragma unroll
        for (int j = 0; j < 8; ++j) S[tile_off(r + j, k >> 3) + (k & 7)] = e[j];
    }
}

// ---- epilogues ------------------------------------------------------------
// Staged epilogues (kStaged) produce BF16 values that the GEMM gathers in LDS
// and stores eight at a time (put8: columns n..n+7, N a multiple of 8).
struct EpAct {   // hidden layer: out = bf16(ReLU(acc + bias))
    uint16_t* out;
    const float* bias;
    int ld;
    static constexpr bool kStaged = true;
    __device__ uint16_t value(int n, float acc) const { return f32_to_bf16(fmaxf(acc + bias[n], 0.0f)); }
    __device__ void put8(int m, int n, uint4 v) const {
        *reinterpret_cast<uint4*>(out + static_cast<size_t>(m) * ld + n) = v;
    }
};
struct EpOut {   // last layer: out = acc + bias, offsets times hw[m] when hw is given
    float* out;
    const float* bias;
    const float* hw;
    int ld;
    static constexpr bool kStaged = false;
    __device__ void put(int m, int n, float acc, int) const {
        float v = acc + bias[n];
        if (hw && (n % 3) < 2) v *= hw[m];
        out[static_cast<size_t>(m) * ld + n] = v;
    }
};
struct EpStore {  // plain FP32 store; split z writes its own M x N slab
    float* out;
    int ld;
    size_t slab;
    static constexpr bool kStaged = false;
    __device__ void put(int m, int n, float acc, int z) const {
        out[z * slab + static_cast<size_t>(m) * ld + n] = acc;
    }
};
// Input-gradient epilogues (kColSum): g = acc * [x > 0] in FP32 is the
// gradient of the lower layer's pre-activation; its BF16 rounding is stored
// for that layer's contractions, and the GEMM sums g over each tile's rows in
// a fixed order into colpart[(cls nM + m-tile)][n], the partial column sums
// from which that layer's bias gradient is formed (the FP32 g itself is not
// stored).
struct EpMaskGrad {  // FC input gradient
    uint16_t* gq;
    const uint16_t* x;
    int ld;
    float* colpart;
    static constexpr bool kStaged = false, kColSum = true;
    static constexpr int cls = 0;
    __device__ float put(int m, int n, float acc, int) const {
        const size_t i = static_cast<size_t>(m) * ld + n;
        const float g = (x[i] & 0x7fffu) != 0 && !(x[i] & 0x8000u) ? acc : 0.0f;
        gq[i] = f32_to_bf16(g);
        return g;
    }
};

struct EpSubpix {   // conv input gradient of one parity class at (b, 2j+py, 2i+px, ci)
    uint16_t* gq;
    const uint16_t* x;   // the layer input, NHWC [B][Hin][Hin][Cin]
    int py, px, lgHo, Ho, Cin;
    float* colpart;
    int cls;             // the parity class, 2 py + px
    static constexpr bool kStaged = false, kColSum = true;
    __device__ float put(int m, int ci, float acc, int) const {
        const int b = m >> (2 * lgHo), j = (m >> lgHo) & (Ho - 1), i = m & (Ho - 1);
        const size_t idx = ((static_cast<size_t>(b) * 2 * Ho + 2 * j + py) * 2 * Ho + 2 * i + px) * Cin + ci;
        const float g = (x[idx] & 0x7fffu) != 0 && !(x[idx] & 0x8000u) ? acc : 0.0f;
        gq[idx] = f32_to_bf16(g);
        return g;
    }
};

template <class EP, class = void>
struct ColSumOf {
    static constexpr bool value = false;
};
template <class EP>
struct ColSumOf<EP, decltype(void(EP::kColSum))> {
    static constexpr bool value = EP::kColSum;
};

// C[M][N] = sum_k A(m, k) B(k, n), B given as Op(n, k).  Block: 64 x 64 tile,
// four waves of 32 x 32 (2 x 2 MFMA blocks of 16 x 16), k-steps of 32.
// Grid: x = M tiles (rounded up to eight when xcd is set) x N tiles, z =
// splits of the k range (kchunk each).
template <class LA, class LB, class EP>
__global__ __launch_bounds__(256) void gemm_kernel(LA la, LB lb, EP ep, int M, int N, int K, int kchunk,
                                                   int xcd) {
    constexpr int kCs = kBN + 8;   // staged C tile row stride, BF16 elements (144 B)
    constexpr int kSmem = (kBM + kBN) * kBK > kBM * kCs ? (kBM + kBN) * kBK : kBM * kCs;
    __shared__ __attribute__((aligned(16))) uint16_t smem[kSmem];
    uint16_t* const As = smem;
    uint16_t* const Bs = smem + kBM * kBK;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    // Tile order.  Work-groups are dealt to the eight XCDs in turn; with xcd set
    // the N tiles of one M tile take ids eight apart: same XCD (same L2) and
    // dispatched together, so the A rows they share are read from HBM once.
    // Otherwise M tiles run fastest.
    const int nM = (M + kBM - 1) / kBM, nN = (N + kBN - 1) / kBN;
    int mt, nt;
    if (xcd) {
        const int slot = blockIdx.x >> 3;
        mt = (slot / nN) * 8 + (blockIdx.x & 7);
        nt = slot - (slot / nN) * nN;
        if (mt >= nM) return;   // padding tiles of the last group of eight
    } else {
        nt = blockIdx.x / nM;
        mt = blockIdx.x - nt * nM;
    }
    const int row0 = mt * kBM, col0 = nt * kBN;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // kPre k-steps of operand loads in flight (registers, rotating): a step's
    // LDS store waits only for the loads issued kPre steps earlier.  The step
    // count is rounded up to a multiple of kPre and the loaders return zeros
    // from ke on, so the loop body is straight-line code.
    la.limit(ke);
    lb.limit(ke);
    uint4 va[kPre], vb[kPre];
#pragma unroll
    for (int p = 0; p < kPre; ++p) {
        va[p] = tile_fetch(la, row0, kb + p * kBK, t);
        vb[p] = tile_fetch(lb, col0, kb + p * kBK, t);
    }
    const int groups = (ke - kb + kPre * kBK - 1) / (kPre * kBK);
    for (int g = 0, k0 = kb; g < groups; ++g, k0 += kPre * kBK) {
#pragma unroll
        for (int p = 0; p < kPre; ++p) {
            __syncthreads();
            tile_store<LA>(As, t, va[p]);
            tile_store<LB>(Bs, t, vb[p]);
            __syncthreads();
            va[p] = tile_fetch(la, row0, k0 + (p + kPre) * kBK, t);
            vb[p] = tile_fetch(lb, col0, k0 + (p + kPre) * kBK, t);
            bf16x8 af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                af[i] = *reinterpret_cast<const bf16x8*>(As + tile_off(wm * 32 + i * 16 + (lane & 15), lane >> 4));
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bf[j] = *reinterpret_cast<const bf16x8*>(Bs + tile_off(wn * 32 + j * 16 + (lane & 15), lane >> 4));
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    }
    // C block (i, j): lane holds rows 4 (lane >> 4) + r, column lane & 15
    if constexpr (EP::kStaged) {
        // BF16 tile through LDS (over the operand tiles): each store
        // instruction then writes eight whole 128-byte tile rows
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = wm * 32 + i * 16 + 4 * (lane >> 4) + r, cc = wn * 32 + j * 16 + (lane & 15);
                    smem[rr * kCs + cc] = ep.value(col0 + cc, acc[i][j][r]);
                }
        __syncthreads();
#pragma unroll
        for (int c = t; c < kBM * kBN / 8; c += 256) {
            const int rr = c / (kBN / 8), c8 = (c % (kBN / 8)) * 8;
            if (row0 + rr < M && col0 + c8 < N)
                ep.put8(row0 + rr, col0 + c8, *reinterpret_cast<const uint4*>(smem + rr * kCs + c8));
        }
    } else if constexpr (ColSumOf<EP>::value) {
        // column sums of the stored values over the tile's rows: this lane's
        // eight rows in order, then the four lane groups of a column (fixed
        // butterfly), then the two waves along M through LDS
        float cs[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            cs[j] = 0.0f;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = row0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                    const int n = col0 + wn * 32 + j * 16 + (lane & 15);
                    if (m < M && n < N) cs[j] += ep.put(m, n, acc[i][j][r], blockIdx.z);
                }
            cs[j] += __shfl_xor(cs[j], 16, 64);
            cs[j] += __shfl_xor(cs[j], 32, 64);
        }
        float* red = reinterpret_cast<float*>(smem);   // 2 x 64 floats over the operand tiles
        __syncthreads();
        if (lane < 16) {
#pragma unroll
            for (int j = 0; j < 2; ++j) red[wm * kBN + wn * 32 + j * 16 + lane] = cs[j];
        }
        __syncthreads();
        if (t < kBN && col0 + t < N)
            ep.colpart[(static_cast<size_t>(ep.cls) * nM + mt) * N + col0 + t] = red[t] + red[kBN + t];
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = row0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                    const int n = col0 + wn * 32 + j * 16 + (lane & 15);
                    if (m < M && n < N) ep.put(m, n, acc[i][j][r], blockIdx.z);
                }
    }
}

template <class LA, class LB, class EP>
hipError_t gemm(const LA& la, const LB& lb, const EP& ep, int M, int N, int K, int splits, int kchunk,
                hipStream_t s) {
    if (EP::kStaged && N % 8 != 0) return hipErrorInvalidValue;
    const long nM = (M + kBM - 1) / kBM, nN = (N + kBN - 1) / kBN;
    const int xcd = nM >= 8 && nN > 1;
    const long nx = (xcd ? (nM + 7) / 8 * 8 : nM) * nN;
    if (nx > 0x7fffffffL) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(nx), 1, splits);
    hipLaunchKernelGGL((gemm_kernel<LA, LB, EP>), grid, dim3(256), 0, s, la, lb, ep, M, N, K, kchunk, xcd);
    return hipGetLastError();
}

// ---- layer table ----------------------------------------------------------
struct Layer {
    int conv, cin, cout, hin, hout;   // fc: hin = hout = 1
    int K, Kp;                        // reduction length (9 cin or fin), padded to 32
    long w_off, b_off;                // in the parameter blob
    long wp_off;                      // in the packed BF16 weights
    long act_in;                      // activation (layer input) offset per sample, BF16 elements; -1: the input
};
struct Table {
    Layer l[8];
    long params, packed, act_per_sample;
};

Table make_table() {
    Table T{};
    long off = 0, wp = 0, act = 0;
    int cin = 1, h = kSide;
    for (int i = 0; i < 8; ++i) {
        Layer& L = T.l[i];
        L.conv = i < 6;
        L.cin = cin;
        L.cout = i < 6 ? kConvWidth[i] : (i == 6 ? kFc0 : kOut);
        L.hin = L.conv ? h : 1;
        L.hout = L.conv ? (h + 1) / 2 : 1;
        L.K = L.conv ? 9 * cin : cin;
        L.Kp = (L.K + kBK - 1) / kBK * kBK;
        L.w_off = off;
        off += static_cast<long>(L.cout) * L.K;
        L.b_off = off;
        off += L.cout;
        L.wp_off = wp;
        wp += static_cast<long>(L.cout) * L.Kp;
        if (i == 0) {
            L.act_in = -1;
        } else {
            L.act_in = act;
            act += static_cast<long>(L.hin) * L.hin * L.cin;
        }
        cin = L.cout;
        h = L.hout;
    }
    T.params = off;
    T.packed = wp;
    T.act_per_sample = act;
    return T;
}

const Table& table() {
    static const Table T = make_table();
    return T;
}

static int lg2(int v) {   // v a power of two
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}
static void set_shifts(Im2col& a, const Layer& L) {
    a.lgHW = lg2(L.hout * L.hout);
    a.lgWo = lg2(L.hout);
    a.lgCin = lg2(L.cin);
}

// First convolution (one input channel, kSide x kSide in, kConvWidth[0] out):
// as a GEMM its reduction is only 9 long (padded to 32) and its 64-wide column
// tile half used, so it runs as a direct 3 x 3 / stride 2 stencil instead, one
// output pixel per thread and all output channels, eight at a time with those
// eight channels' weights in scalar registers.  The work-group's 256 pixels x
// kC0 channels are one contiguous stretch of the NHWC output: they go through
// LDS so that each store instruction writes 1 KB contiguous.  Same arithmetic
// as the GEMM path: BF16 operands, exact products summed in FP32 in tap
// order, then bias, ReLU and BF16 rounding.
constexpr int kHo0 = kSide / 2, kC0 = kConvWidth[0];
static_assert(kSide % 2 == 0 && kC0 % 8 == 0 && (kHo0 * kHo0) % 256 == 0, "conv_first_kernel tiling");
__global__ __launch_bounds__(256) void conv_first_kernel(const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ wp, int Kp,
                                                         const float* __restrict__ bias, uint16_t* __restrict__ y) {
    constexpr int Q = kC0 / 8;   // uint4 pieces per pixel
    static_assert(Q == 4, "stage_slot swizzles four pieces per pixel");
    // piece q of pixel p at slot 4 p + (q ^ ((p >> 2) & 3)): sixteen lanes
    // writing one piece of sixteen pixels, or reading four pieces of four
    // pixels, use sixteen distinct bank groups
    auto stage_slot = [](int p, int q) { return 4 * p + (q ^ ((p >> 2) & 3)); };
    __shared__ uint4 stage[256 * Q];
    const int tid = threadIdx.x;
    const long m = blockIdx.x * 256L + tid;   // grid: B * kHo0 * kHo0 / 256 blocks exactly
    const int b = static_cast<int>(m / (kHo0 * kHo0)), r = static_cast<int>(m % (kHo0 * kHo0));
    const int oy = r / kHo0, ox = r % kHo0;
    const uint16_t* xb = x + static_cast<size_t>(b) * kSide * kSide;
    float xv[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
        xv[tap] = (iy >= 0 && iy < kSide && ix >= 0 && ix < kSide) ? bf16_to_f32(xb[iy * kSide + ix]) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        float acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            // row co of the packed weights: taps 0..8, then zeros up to Kp
            const uint32_t* wr = reinterpret_cast<const uint32_t*>(wp + (8 * q + j) * Kp);
            acc[j] = 0.0f;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const uint32_t u = wr[tap >> 1];
                acc[j] = fmaf(xv[tap], __uint_as_float((tap & 1) ? (u & 0xffff0000u) : (u << 16)), acc[j]);
            }
        }
        uint32_t pk[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            pk[j] = static_cast<uint32_t>(f32_to_bf16(fmaxf(acc[2 * j] + bias[8 * q + 2 * j], 0.0f))) |
                    static_cast<uint32_t>(f32_to_bf16(fmaxf(acc[2 * j + 1] + bias[8 * q + 2 * j + 1], 0.0f))) << 16;
        stage[stage_slot(tid, q)] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    }
    __syncthreads();
    uint4* dst = reinterpret_cast<uint4*>(y + blockIdx.x * 256L * kC0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int c = tid + 256 * i;   // 16-B piece c of the stretch: pixel c / Q, piece c % Q
        dst[c] = stage[stage_slot(c / Q, c % Q)];
    }
}

// ---- small kernels ----------------------------------------------------------
struct PackArgs {
    Layer l[8];
};

// FP32 master weights (PyTorch layout) -> BF16, K-contiguous with conv taps
// ordered (ky, kx, ci), rows padded with zeros to Kp.
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a, const float* __restrict__ params,
                                                   uint16_t* __restrict__ wp, long total) {
    for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += static_cast<long>(gridDim.x) * 256) {
        int li = 0;
        while (li < 7 && i >= a.l[li + 1].wp_off) ++li;
        const Layer& L = a.l[li];
        const long e = i - L.wp_off;
        const int co = static_cast<int>(e / L.Kp), k = static_cast<int>(e - static_cast<long>(co) * L.Kp);
        float v = 0.0f;
        if (k < L.K) {
            if (L.conv) {
                const int tap = k / L.cin, ci = k - tap * L.cin;
                v = params[L.w_off + (static_cast<long>(co) * L.cin + ci) * 9 + tap];
            } else {
                v = params[L.w_off + static_cast<long>(co) * L.K + k];
            }
        }
        wp[i] = f32_to_bf16(v);
    }
}

// Loss (before the update) and dL/dy_hat = 2 (y_hat - y) / (B 144), y the
// reference in network units.  Grid-stride over the B x 144 outputs; each
// block writes its partial sum of squares (fixed order inside the block), and
// loss_final_kernel adds the partials in block order.
constexpr int kLossBlocks = 256;
__global__ __launch_bounds__(256) void loss_grad_kernel(int B, const float* __restrict__ yhat,
                                                        const float* __restrict__ ref, const float* __restrict__ hw,
                                                        float* __restrict__ g32, uint16_t* __restrict__ gq,
                                                        float* __restrict__ part) {
    __shared__ float red[4];
    const long n = static_cast<long>(B) * kOut;
    const float fn = static_cast<float>(n);
    float s = 0.0f;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * 256) {
        const int b = static_cast<int>(i / kOut), c = static_cast<int>(i - static_cast<long>(b) * kOut);
        const float y = (c % 3) < 2 ? ref[i] / hw[b] : ref[i];
        const float d = yhat[i] - y;
        s += d * d;
        const float g = (2.0f * d) / fn;   // correctly rounded: exact whenever 2d/n is representable
        g32[i] = g;
        gq[i] = f32_to_bf16(g);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ __launch_bounds__(256) void loss_final_kernel(const float* __restrict__ part, int nb, long n,
                                                         float* __restrict__ loss_out) {
    __shared__ float buf[256];
    float v = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 256) v += part[b];
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if (threadIdx.x < m) buf[threadIdx.x] += buf[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_out[0] = buf[0] / static_cast<float>(n);
}

// Column sums of g [M][N] (FP32, N a multiple of 4, at most 1024): stage 1
// writes part[blk][N] for 256-row slabs, stage 2 adds the slabs in order.
// Stage 1 reads whole rows as float4: thread t owns column quad q = t % (N/4)
// of rows r0 + j * rpi (r0 = t / (N/4), rpi = 256 / (N/4) rows per sweep), and
// the rpi partial sums of each quad are then added in order of r0.
constexpr int kColRows = 256;
__global__ __launch_bounds__(256) void colsum_part_kernel(const float* __restrict__ g, int M, int N,
                                                          float* __restrict__ part) {
    __shared__ float4 red[256];
    const int nq = N >> 2, rpi = 256 / nq;
    const int t = threadIdx.x, q = t % nq, r0 = t / nq;
    const int s0 = blockIdx.x * kColRows, s1 = min(M, s0 + kColRows);
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (r0 < rpi) {
        const float4* g4 = reinterpret_cast<const float4*>(g);
        for (int r = s0 + r0; r < s1; r += rpi) {
            const float4 v = g4[static_cast<size_t>(r) * nq + q];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
    }
    red[t] = acc;
    __syncthreads();
    if (t < nq) {
        float4 s = red[t];
        for (int k = 1; k < rpi; ++k) {
            const float4 v = red[k * nq + t];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
        reinterpret_cast<float4*>(part + static_cast<size_t>(blockIdx.x) * N)[t] = s;
    }
}
// One work-group per column: strided partial sums, then a fixed tree.
__global__ __launch_bounds__(256) void colsum_final_kernel(const float* __restrict__ part, int nblk, int N,
                                                           float* __restrict__ out) {
    __shared__ float buf[256];
    const int n = blockIdx.x;
    float s = 0.0f;
    for (int b = threadIdx.x; b < nblk; b += 256) s += part[static_cast<size_t>(b) * N + n];
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if (threadIdx.x < m) buf[threadIdx.x] += buf[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = buf[0];
}

// Sum the split-K slabs of a weight gradient [S][cout][Kp] into the blob's
// PyTorch layout.
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(Layer L, const float* __restrict__ part, int S,
                                                           float* __restrict__ grad) {
    const long n = static_cast<long>(L.cout) * L.K;
    const size_t slab = static_cast<size_t>(L.cout) * L.Kp;
    // i walks the packed columns (co, k), so the S slab reads of consecutive
    // threads are consecutive floats; each sum goes to its blob position
    // (for a convolution, packed column k = tap * cin + ci is blob entry
    // (co, ci, tap))
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * 256) {
        const int co = static_cast<int>(i / L.K), k = static_cast<int>(i - static_cast<long>(co) * L.K);
        float s = 0.0f;
        for (int z = 0; z < S; ++z) s += part[z * slab + static_cast<size_t>(co) * L.Kp + k];
        long dst = i;
        if (L.conv) {
            const int tap = k / L.cin, ci = k - tap * L.cin;
            dst = static_cast<long>(co) * L.K + 9 * ci + tap;
        }
        grad[L.w_off + dst] = s;
    }
}

__global__ __launch_bounds__(256) void adam_kernel(long n, float* __restrict__ p, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ g, float lr,
                                                   float bc1, float bc2) {
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * 256) {
        const float gi = g[i];
        const float mi = fmaf(0.9f, m[i], 0.1f * gi);
        const float vi = fmaf(0.999f, v[i], 0.001f * gi * gi);
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
    }
}

// Network input of one target per work-group (exact area overlap onto 64 x 64
// cells of side s centred on the target's centre, peak-normalised, BF16).
__global__ __launch_bounds__(256) void prepare_kernel(int B, const disk_target* __restrict__ desc,
                                                      const float* __restrict__ targets, uint16_t* __restrict__ x64,
                                                      float* __restrict__ hw, int max_side) {
    __shared__ float red[4];
    const int tid = threadIdx.x;
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        const disk_target d = desc[b];
        const int M = d.side;
        uint16_t* out = x64 + static_cast<size_t>(b) * kSide * kSide;
        if (M < 1 || (M & 1) == 0 || M > max_side || d.target_off < 0) {
            for (int i = tid; i < kSide * kSide; i += 256) out[i] = 0;
            if (tid == 0) hw[b] = 0.0f;
            continue;
        }
        const float* K = targets + d.target_off;
        const float s = fmaxf(1.0f, static_cast<float>(M) / kSide);
        const float c = 0.5f * static_cast<float>(M - 1);
        const float inv_s2 = 1.0f / (s * s);
        float val[16];
        float mx = 0.0f;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int idx = tid + 256 * q, i = idx >> 6, j = idx & 63;
            const float lo_y = c + static_cast<float>(i - 32) * s, hi_y = lo_y + s;
            const float lo_x = c + static_cast<float>(j - 32) * s, hi_x = lo_x + s;
            const int y0 = max(0, static_cast<int>(floorf(lo_y + 0.5f))), y1 = min(M - 1, static_cast<int>(floorf(hi_y + 0.5f)));
            const int x0 = max(0, static_cast<int>(floorf(lo_x + 0.5f))), x1 = min(M - 1, static_cast<int>(floorf(hi_x + 0.5f)));
            float acc = 0.0f;
            for (int y = y0; y <= y1; ++y) {
                const float wy = fminf(hi_y, y + 0.5f) - fmaxf(lo_y, y - 0.5f);
                if (wy <= 0.0f) continue;
                float row = 0.0f;
                for (int x = x0; x <= x1; ++x) {
                    const float wx = fminf(hi_x, x + 0.5f) - fmaxf(lo_x, x - 0.5f);
                    if (wx > 0.0f) row += wx * K[y * M + x];
                }
                acc += wy * row;
            }
            val[q] = acc * inv_s2;
            mx = fmaxf(mx, val[q]);
        }
        mx = wave_max(mx);
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = mx;
        __syncthreads();
        const float pk = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
#pragma unroll
        for (int q = 0; q < 16; ++q) out[tid + 256 * q] = f32_to_bf16(pk > 0.0f ? val[q] / pk : 0.0f);
        if (tid == 0) hw[b] = 0.5f * kSide * s;
    }
}

__global__ __launch_bounds__(64) void scatter_kernel(int B, const disk_target* __restrict__ desc,
                                                     const int* __restrict__ taps, const float* __restrict__ th48,
                                                     float* __restrict__ theta) {
    const int b = blockIdx.x;
    if (b >= B) return;
    const disk_target d = desc[b];
    if (d.L != 4 || d.taps_off < 0 || d.theta_off < 0) return;
    for (int l = 0; l < 4; ++l)
        if (taps[d.taps_off + l] != 12) return;
    for (int i = threadIdx.x; i < kOut; i += 64)
        theta[3 * static_cast<size_t>(d.theta_off) + i] = th48[static_cast<size_t>(b) * kOut + i];
}

int grid_for(long n) { return static_cast<int>(std::min<long>((n + 255) / 256, 8192)); }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
long net_param_count() { return table().params; }

// Workspace layout (offsets in bytes, 256-aligned), for batch B.
// Rows of partial column sums from which layer i's bias gradient is formed
// (i < 7): the tiles of the GEMMs that produce its output gradient, i.e. the
// input gradient of layer i + 1 (four parity classes for a convolution).
static size_t bias_part_rows(int B, int i) {
    const Layer& P = table().l[i + 1];
    const size_t M = static_cast<size_t>(B) * P.hout * P.hout;
    const size_t nM = (M + kBM - 1) / kBM;
    return P.conv ? 4 * nM : nM;
}

NetWs net_ws_layout(int B, bool train) {
    const Table& T = table();
    NetWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        const size_t o = off;
        off += bytes;
        return o;
    };
    w.wp = take(T.packed * 2);
    w.act = take(static_cast<size_t>(B) * T.act_per_sample * 2);
    w.yhat = take(static_cast<size_t>(B) * kOut * 4);
    if (!train) {
        w.total = take(0);
        return w;
    }
    // gradient buffers: BF16 copies of the largest layer output (layer 1: 32 x
    // 32 x 32 per sample); FP32 only for the output layer's (the loss gradient)
    size_t gmax = 0, part = 0, cpart = ((static_cast<size_t>(B) + kColRows - 1) / kColRows) * kOut, cslab = 0;
    for (int i = 0; i < 8; ++i) {
        const Layer& L = T.l[i];
        const size_t M = static_cast<size_t>(B) * L.hout * L.hout;
        gmax = std::max(gmax, M * L.cout);
        int S, kc;
        net_wgrad_splits(L.cout, L.Kp, static_cast<int>(M), &S, &kc);
        part = std::max(part, static_cast<size_t>(S) * L.cout * L.Kp);
        if (i < 7) {
            cpart = std::max(cpart, bias_part_rows(B, i) * L.cout);
            cslab = std::max(cslab, (bias_part_rows(B, i) + kColRows - 1) / kColRows * L.cout);
        }
    }
    w.g32[0] = take(static_cast<size_t>(B) * kOut * 4);
    w.g32[1] = w.g32[0];
    w.gq[0] = take(gmax * 2);
    w.gq[1] = take(gmax * 2);
    w.part = take(part * 4);
    w.cpart = take(cpart * 4);
    w.cslab = take(cslab * 4);
    w.grad = take(T.params * 4);
    w.total = take(0);
    return w;
}

void net_wgrad_splits(int cout, int Kp, int Mred, int* S, int* kchunk) {
    const int tiles = ((cout + kBM - 1) / kBM) * ((Kp + kBN - 1) / kBN);
    int s = std::max(1, 512 / tiles);
    const int steps = (Mred + kBK - 1) / kBK;
    s = std::min(s, steps);
    const int per = (steps + s - 1) / s;
    *kchunk = per * kBK;
    *S = (Mred + *kchunk - 1) / *kchunk;
}

static uint16_t* act_ptr(char* ws, const NetWs& w, int B, const Layer& L, const uint16_t* x0) {
    if (L.act_in < 0) return const_cast<uint16_t*>(x0);
    return reinterpret_cast<uint16_t*>(ws + w.act) + static_cast<size_t>(B) * L.act_in;
}

hipError_t net_forward(const float* params, const uint16_t* x0, int B, char* ws, const NetWs& w,
                       float* out, const float* hw, hipStream_t s) {
    const Table& T = table();
    PackArgs pa;
    for (int i = 0; i < 8; ++i) pa.l[i] = T.l[i];
    uint16_t* wp = reinterpret_cast<uint16_t*>(ws + w.wp);
    hipLaunchKernelGGL(pack_kernel, dim3(grid_for(T.packed)), dim3(256), 0, s, pa, params, wp, T.packed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int i = 0; i < 8; ++i) {
        const Layer& L = T.l[i];
        const uint16_t* xin = act_ptr(ws, w, B, L, x0);
        const int M = B * L.hout * L.hout;
        const float* bias = params + L.b_off;
        LdRow wb{wp + L.wp_off, L.Kp, L.cout, L.Kp};
        if (i < 7) {
            EpAct ep{act_ptr(ws, w, B, T.l[i + 1], x0), bias, L.cout};
            if (i == 0) {
                const long nblk = static_cast<long>(B) * kHo0 * kHo0 / 256;
                hipLaunchKernelGGL(conv_first_kernel, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, s, xin, wb.p,
                                   L.Kp, bias, ep.out);
                e = hipGetLastError();
            } else if (L.conv) {
                LdIm2col a;
                a.x = xin; a.H = L.hin; a.W = L.hin; a.Cin = L.cin; a.Ho = L.hout; a.Wo = L.hout; a.M = M; a.K = L.K;
                set_shifts(a, L);
                e = gemm(a, wb, ep, M, L.cout, L.Kp, 1, L.Kp, s);
            } else {
                LdRow a{xin, L.K, M, L.K};
                e = gemm(a, wb, ep, M, L.cout, L.Kp, 1, L.Kp, s);
            }
        } else {
            LdRow a{xin, L.K, M, L.K};
            EpOut ep{out, bias, hw, kOut};
            e = gemm(a, wb, ep, M, L.cout, L.Kp, 1, L.Kp, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t net_backward(const float* params, const uint16_t* x0, const float* ref, const float* hw, int B, char* ws,
                        const NetWs& w, float* grad, float* loss_out, hipStream_t s) {
    const Table& T = table();
    const uint16_t* wp = reinterpret_cast<const uint16_t*>(ws + w.wp);
    const float* yhat = reinterpret_cast<const float*>(ws + w.yhat);
    float* g32 = reinterpret_cast<float*>(ws + w.g32[0]);
    uint16_t* gq[2] = {reinterpret_cast<uint16_t*>(ws + w.gq[0]), reinterpret_cast<uint16_t*>(ws + w.gq[1])};
    float* part = reinterpret_cast<float*>(ws + w.part);
    float* cpart = reinterpret_cast<float*>(ws + w.cpart);
    {
        // the loss partials use the column-sum scratch (>= 128 B floats: layer 1's slab count x 32)
        const long n = static_cast<long>(B) * kOut;
        const int nb = static_cast<int>(std::min<long>(kLossBlocks, (n + 1023) / 1024));
        hipLaunchKernelGGL(loss_grad_kernel, dim3(nb), dim3(256), 0, s, B, yhat, ref, hw, g32, gq[0], cpart);
        hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, cpart, nb, n, loss_out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int cur = 0;
    for (int i = 7; i >= 0; --i) {
        const Layer& L = T.l[i];
        const int M = B * L.hout * L.hout;
        const uint16_t* xin = act_ptr(ws, w, B, L, x0);
        // bias gradient: column sums of g (FP32).  The output layer's g is the
        // loss gradient in FP32; every other layer's comes as the partial
        // column sums that the epilogues of the input-gradient GEMMs of layer
        // i + 1 left in cpart (one row per tile, parity classes in order)
        if (i == 7) {
            if ((L.cout & 3) != 0 || L.cout > 1024) return hipErrorInvalidValue;   // the column-sum layout
            const int nblk = (M + kColRows - 1) / kColRows;
            hipLaunchKernelGGL(colsum_part_kernel, dim3(nblk), dim3(256), 0, s, g32, M, L.cout, cpart);
            hipLaunchKernelGGL(colsum_final_kernel, dim3(L.cout), dim3(256), 0, s, cpart, nblk, L.cout,
                               grad + L.b_off);
        } else {
            // the tile partials, [rows][cout]; many rows: 256-row slabs read as
            // whole rows, then the slabs in order (reading 64K rows a column at
            // a time took 23 us per layer at batch 4096; for a few thousand
            // rows the extra launch costs more than it saves)
            const int rows = static_cast<int>(bias_part_rows(B, i));
            if (rows > 8192) {
                if ((L.cout & 3) != 0 || L.cout > 1024) return hipErrorInvalidValue;
                const int nslab = (rows + kColRows - 1) / kColRows;
                float* cslab = reinterpret_cast<float*>(ws + w.cslab);
                hipLaunchKernelGGL(colsum_part_kernel, dim3(nslab), dim3(256), 0, s, cpart, rows, L.cout, cslab);
                hipLaunchKernelGGL(colsum_final_kernel, dim3(L.cout), dim3(256), 0, s, cslab, nslab, L.cout,
                                   grad + L.b_off);
            } else {
                hipLaunchKernelGGL(colsum_final_kernel, dim3(L.cout), dim3(256), 0, s, cpart, rows, L.cout,
                                   grad + L.b_off);
            }
        }
        // weight gradient: dW(co, j) = sum_m g(m, co) x_col(m, j), split over m
        int S, kc;
        net_wgrad_splits(L.cout, L.Kp, M, &S, &kc);
        LdCol ga{gq[cur], L.cout, L.cout, M};
        EpStore ps{part, L.Kp, static_cast<size_t>(L.cout) * L.Kp};
        if (L.conv) {
            LdIm2colT xb;
            xb.x = xin; xb.H = L.hin; xb.W = L.hin; xb.Cin = L.cin; xb.Ho = L.hout; xb.Wo = L.hout; xb.M = M; xb.K = L.K;
            set_shifts(xb, L);
            e = gemm(ga, xb, ps, L.cout, L.Kp, M, S, kc, s);
        } else {
            LdCol xb{xin, L.K, L.K, M};
            e = gemm(ga, xb, ps, L.cout, L.Kp, M, S, kc, s);
        }
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(grid_for(static_cast<long>(L.cout) * L.K)), dim3(256), 0, s, L,
                           part, S, grad);
        if (i == 0) break;
        // input gradient, masked by the layer input's ReLU, into the other buffer
        const int nxt = cur ^ 1;
        LdRow gr{gq[cur], L.cout, M, L.cout};
        LdCol wc{wp + L.wp_off, L.Kp, L.Kp, L.cout};
        if (L.conv) {
            // four parity classes of input pixels, each a GEMM over its taps
            const int lgHo = lg2(L.hout), lgCo = lg2(L.cout);
            for (int py = 0; py < 2; ++py)
                for (int px = 0; px < 2; ++px) {
                    const SubpixTap st{py, px, lgHo, lgCo, L.hout, L.cout};
                    const int Kc = (1 + py) * (1 + px) * L.cout;
                    LdSubpixG a;
                    static_cast<SubpixTap&>(a) = st;
                    a.g = gq[cur]; a.M = M; a.K = Kc;
                    LdSubpixW wb;
                    static_cast<SubpixTap&>(wb) = st;
                    wb.wp = wp + L.wp_off; wb.Kp = L.Kp; wb.Cin = L.cin; wb.K = Kc;
                    EpSubpix ep{gq[nxt], xin, py, px, lgHo, L.hout, L.cin, cpart, 2 * py + px};
                    e = gemm(a, wb, ep, M, L.cin, Kc, 1, Kc, s);
                    if (e != hipSuccess) return e;
                }
        } else {
            EpMaskGrad ep{gq[nxt], xin, L.K, cpart};
            e = gemm(gr, wc, ep, M, L.K, L.cout, 1, L.cout, s);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur = nxt;
    }
    return hipGetLastError();
}

hipError_t net_adam(float* params, float* m, float* v, const float* grad, int step, float lr, hipStream_t s) {
    const long n = table().params;
    const float bc1 = static_cast<float>(1.0 - std::pow(0.9, step));
    const float bc2 = static_cast<float>(1.0 - std::pow(0.999, step));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, params, m, v, grad, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t net_prepare(int B, const disk_target* desc, const float* targets, uint16_t* x64, float* hw, int max_side,
                       hipStream_t s) {
    hipLaunchKernelGGL(prepare_kernel, dim3(std::min(B, 8192)), dim3(256), 0, s, B, desc, targets, x64, hw, max_side);
    return hipGetLastError();
}

hipError_t net_scatter(int B, const disk_target* desc, const int* taps, const float* th48, float* theta,
                       hipStream_t s) {
    hipLaunchKernelGGL(scatter_kernel, dim3(B), dim3(64), 0, s, B, desc, taps, th48, theta);
    return hipGetLastError();
}

}  // namespace disk
