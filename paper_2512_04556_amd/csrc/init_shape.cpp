// Shape-aware (sparse-sampling) initialisation of Theta (Sec. 4.2, Eq. 7), on
// the host in FP64.  The first layer's taps are dart-thrown over the support of
// the target, {K > 0.01 max K}: S = |support|, r = sqrt(S / (N_1 pi)); a draw is
// a uniformly chosen support pixel jittered by U[-1/2, 1/2)^2 and is accepted
// when it lies at least r from every accepted point; after 100 N_1 consecutive
// rejections r shrinks by 0.9.  Layer-1 weights are the target at the rounded
// points, normalised to unit sum.  Layers 2..L take the radial pattern of Eq. 6
// with extent r and layer indices 1..L-1 (their radii sum to r).
//
// Random numbers: SplitMix64 (Steele, Lea, Flood 2014), counter-based: output n
// of key k is mix64(k + (n + 1) * 0x9E3779B97F4A7C15); the key of target b
// under seed s is output b of key s; a uniform double is (z >> 11) * 2^-53.
// Compiled with FP contraction off so each double operation rounds as written.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/disk.h"

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Counter {
    uint64_t key, n = 0;
    double uniform() {
        const uint64_t z = mix64(key + (n + 1) * kGolden);
        ++n;
        return static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0);
    }
};

void radial(double R, const int32_t* taps, int L, int index0, float* out) {
    // radii r_j = j * dr for j = index0 .. index0 + L - 1, summing to R
    const int jmax = index0 + L - 1;
    const double jsum = 0.5 * (static_cast<double>(jmax) * (jmax + 1) - static_cast<double>(index0 - 1) * index0);
    const double dr = jsum > 0.0 ? R / jsum : 0.0;
    int o = 0;
    for (int l = 0; l < L; ++l) {
        const int N = taps[l];
        const double r = (l + index0) * dr;
        for (int i = 1; i <= N; ++i) {
            const double a = 2.0 * M_PI * i / N;
            out[3 * o + 0] = static_cast<float>(r * std::cos(a));
            out[3 * o + 1] = static_cast<float>(r * std::sin(a));
            out[3 * o + 2] = static_cast<float>(1.0 / N);
            ++o;
        }
    }
}

}  // namespace

extern "C" disk_status disk_init_shape(const float* target, int32_t M, int32_t L, const int32_t* taps, uint64_t seed,
                                       int32_t index, float* theta, double* r_out) {
    if (!target || !taps || !theta) return DISK_INVALID_ARG;
    if (M < 1 || (M & 1) == 0 || M > DISK_MAX_SIDE || L < 1 || L > DISK_MAX_LAYERS) return DISK_BAD_SHAPE;
    for (int l = 0; l < L; ++l)
        if (taps[l] < 1 || taps[l] > DISK_MAX_TAPS) return DISK_BAD_SHAPE;
    const double c = (M - 1) / 2.0;
    double pk = -INFINITY;
    for (int i = 0; i < M * M; ++i) pk = std::fmax(pk, static_cast<double>(target[i]));
    if (!(pk > 0.0)) {  // degenerate target: the radial pattern over the half-width
        radial(c, taps, L, 1, theta);
        if (r_out) *r_out = 0.0;
        return DISK_OK;
    }
    std::vector<int> sx, sy;  // support, row-major
    for (int y = 0; y < M; ++y)
        for (int x = 0; x < M; ++x)
            if (static_cast<double>(target[y * M + x]) > 0.01 * pk) {
                sx.push_back(x);
                sy.push_back(y);
            }
    const int S = static_cast<int>(sx.size());
    const int Ns = taps[0];
    double r = std::sqrt(S / (Ns * M_PI));
    Counter st{mix64(seed + (static_cast<uint64_t>(index) + 1) * kGolden)};
    std::vector<double> ax, ay;
    int rejections = 0;
    while (static_cast<int>(ax.size()) < Ns) {
        int j = static_cast<int>(st.uniform() * S);
        if (j > S - 1) j = S - 1;
        const double px = static_cast<double>(sx[j]) + (st.uniform() - 0.5);
        const double py = static_cast<double>(sy[j]) + (st.uniform() - 0.5);
        const double r2 = r * r;
        bool ok = true;
        for (size_t k = 0; k < ax.size(); ++k) {
            const double dx = px - ax[k], dy = py - ay[k];
            if (dx * dx + dy * dy < r2) {
                ok = false;
                break;
            }
        }
        if (ok) {
            ax.push_back(px);
            ay.push_back(py);
            rejections = 0;
        } else if (++rejections >= 100 * Ns) {
            r = 0.9 * r;
            rejections = 0;
        }
    }
    std::vector<double> w(Ns);
    double wsum = 0.0;
    for (int k = 0; k < Ns; ++k) {
        int rx = static_cast<int>(std::floor(ax[k] + 0.5)), ry = static_cast<int>(std::floor(ay[k] + 0.5));
        rx = rx < 0 ? 0 : (rx > M - 1 ? M - 1 : rx);
        ry = ry < 0 ? 0 : (ry > M - 1 ? M - 1 : ry);
        w[k] = target[ry * M + rx];
        wsum += w[k];
    }
    for (int k = 0; k < Ns; ++k) {
        theta[3 * k + 0] = static_cast<float>(ax[k] - c);
        theta[3 * k + 1] = static_cast<float>(ay[k] - c);
        theta[3 * k + 2] = static_cast<float>(wsum > 0.0 ? w[k] / wsum : 1.0 / Ns);
    }
    if (L > 1) radial(r, taps + 1, L - 1, 1, theta + 3 * Ns);
    if (r_out) *r_out = r;
    return DISK_OK;
}

// ---------------------------------------------------------------------------
// Random-position initialisation (the baseline of Sec. 4.2): tap i of layer l
// uniform in [-r_l, r_l]^2 with r_l = l dr the radial rule's radius (Eq. 6,
// dr = 2R / (L (L + 1)), R = min((M-1)/2, r99)), w = 1 / N_l.  Two draws per
// tap (x, then y) from the same counter stream as the shape-aware init.
// ---------------------------------------------------------------------------
namespace {

// Smallest pixel-centre distance whose closed disk holds >= 99% of the mass:
// pixels ordered by squared distance (stable), masses accumulated in that order.
double r99(const float* K, int M) {
    const int h = (M - 1) / 2;
    std::vector<std::pair<int, int>> d2i;   // (d2, row-major index)
    d2i.reserve(static_cast<size_t>(M) * M);
    for (int y = 0; y < M; ++y)
        for (int x = 0; x < M; ++x) d2i.emplace_back((x - h) * (x - h) + (y - h) * (y - h), y * M + x);
    std::stable_sort(d2i.begin(), d2i.end(),
                     [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first < b.first; });
    double total = 0.0;
    for (const auto& p : d2i) total += static_cast<double>(K[p.second]);
    double cum = 0.0;
    const size_t n = d2i.size();
    for (size_t i = 0; i < n; ++i) {
        cum += static_cast<double>(K[d2i[i].second]);
        const bool last = i + 1 == n || d2i[i + 1].first != d2i[i].first;
        if (last && cum >= 0.99 * total) return std::sqrt(static_cast<double>(d2i[i].first));
    }
    return std::sqrt(static_cast<double>(d2i.back().first));
}

}  // namespace

extern "C" disk_status disk_init_random(const float* target, int32_t M, int32_t L, const int32_t* taps, uint64_t seed,
                                        int32_t index, float* theta, double* R_out) {
    if (!target || !taps || !theta) return DISK_INVALID_ARG;
    if (M < 1 || (M & 1) == 0 || M > DISK_MAX_SIDE || L < 1 || L > DISK_MAX_LAYERS) return DISK_BAD_SHAPE;
    for (int l = 0; l < L; ++l)
        if (taps[l] < 1 || taps[l] > DISK_MAX_TAPS) return DISK_BAD_SHAPE;
    const double R = std::fmin(0.5 * (M - 1), r99(target, M));
    const double dr = 2.0 * R / (static_cast<double>(L) * (L + 1));
    Counter st{mix64(seed + (static_cast<uint64_t>(index) + 1) * kGolden)};
    int o = 0;
    for (int l = 0; l < L; ++l) {
        const double r = (l + 1) * dr;
        for (int i = 0; i < taps[l]; ++i) {
            const double ox = (2.0 * st.uniform() - 1.0) * r;
            const double oy = (2.0 * st.uniform() - 1.0) * r;
            theta[3 * o + 0] = static_cast<float>(ox);
            theta[3 * o + 1] = static_cast<float>(oy);
            theta[3 * o + 2] = static_cast<float>(1.0 / taps[l]);
            ++o;
        }
    }
    if (R_out) *R_out = R;
    return DISK_OK;
}
