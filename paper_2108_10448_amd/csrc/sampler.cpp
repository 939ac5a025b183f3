// Host sampler for Algorithm 1's sampling step: uniform index sets I_i and
// J_i drawn without replacement, sorted ascending.
//
// Generator: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).  One stream per
// key (seed, t, mode, which): x = out(seed); x = out(x ^ t);
// x = out(x ^ (2*mode + which)); draws are the successive SplitMix64 outputs
// from state x.  A bounded draw in [0, N) is the high 64 bits of u * N.
// Subsets: Floyd's algorithm (Bentley & Floyd, CACM 1987), then sorted.
// Chidori J_i is the product of the I_j (j != i), last remaining mode fastest;
// fiber J_i is a uniform subset of the C-order columns of the unfolding.
#include "internal.h"

#include <algorithm>
#include <unordered_set>

namespace rtcur {

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

inline uint64_t finalize(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct SplitMix {
    uint64_t state;
    uint64_t next() {
        state += kGamma;
        return finalize(state);
    }
    uint64_t below(uint64_t n) {
        unsigned __int128 p = (unsigned __int128)next() * n;
        return (uint64_t)(p >> 64);
    }
};

inline uint64_t out_of(uint64_t x) { return finalize(x + kGamma); }

SplitMix stream_for(uint64_t seed, int64_t t, int mode, int which) {
    uint64_t x = out_of(seed);
    x = out_of(x ^ (uint64_t)t);
    x = out_of(x ^ (uint64_t)(2 * mode + which));
    return SplitMix{x};
}

// Floyd: for j = N-m .. N-1 draw t in [0, j]; take t unless already taken,
// in which case take j.
std::vector<int64_t> floyd(SplitMix& g, int64_t m, int64_t N) {
    std::unordered_set<int64_t> taken;
    taken.reserve((size_t)m * 2 + 1);
    std::vector<int64_t> out;
    out.reserve((size_t)m);
    for (int64_t j = N - m; j < N; ++j) {
        int64_t t = (int64_t)g.below((uint64_t)(j + 1));
        int64_t pick = taken.count(t) ? j : t;
        taken.insert(pick);
        out.push_back(pick);
    }
    std::sort(out.begin(), out.end());
    return out;
}

}  // namespace

void chidori_columns(const Shape& sh, SampleHost& out) {
    const int n = sh.n;
    out.Jcols.resize(n);
    out.Jtup.resize(n);
    for (int i = 0; i < n; ++i) {
        // remaining modes, increasing; last fastest
        int rest[kMaxModes];
        int nr = 0;
        for (int j = 0; j < n; ++j)
            if (j != i) rest[nr++] = j;
        std::vector<int64_t>& cols = out.Jcols[i];
        std::vector<int32_t>& tup = out.Jtup[i];  // [ncols][n-1]
        int64_t m = 1;
        for (int q = 0; q < nr; ++q) m *= sh.s[rest[q]];
        cols.resize((size_t)m);
        tup.resize((size_t)m * nr);
        // column c <-> positions (pos_0, .., pos_{nr-1}) in the I of the
        // remaining modes, last fastest: an odometer over the positions; the
        // unfolding column is sum_q I[pos_q] * prod_{q' > q} d
        int64_t stride[kMaxModes];
        stride[nr - 1] = 1;
        for (int q = nr - 2; q >= 0; --q) stride[q] = stride[q + 1] * sh.d[rest[q + 1]];
        int64_t pos[kMaxModes] = {0, 0, 0, 0};
        for (int64_t c = 0; c < m; ++c) {
            int64_t col = 0;
            for (int q = 0; q < nr; ++q) {
                const int64_t v = out.I[rest[q]][pos[q]];
                tup[(size_t)c * nr + q] = (int32_t)v;
                col += v * stride[q];
            }
            cols[(size_t)c] = col;
            for (int q = nr - 1; q >= 0; --q) {
                if (++pos[q] < sh.s[rest[q]]) break;
                pos[q] = 0;
            }
        }
    }
}

void draw_sample(uint64_t seed, int64_t t, const Shape& sh, bool chidori,
                 SampleHost& out, bool with_cols) {
    const int n = sh.n;
    // resized, not cleared: a reused sample keeps its vectors' storage
    out.I.resize(n);
    out.Jcols.resize(n);
    out.Jtup.resize(n);
    for (int i = 0; i < n; ++i) {
        SplitMix g = stream_for(seed, t, i, 0);
        out.I[i] = floyd(g, sh.s[i], sh.d[i]);
    }
    if (chidori) {
        if (with_cols) {
            chidori_columns(sh, out);
        } else {
            for (int i = 0; i < n; ++i) {
                out.Jcols[i].clear();
                out.Jtup[i].clear();
            }
        }
        return;
    }
    for (int i = 0; i < n; ++i) {
        int rest[kMaxModes];
        int nr = 0;
        for (int j = 0; j < n; ++j)
            if (j != i) rest[nr++] = j;
        std::vector<int64_t>& cols = out.Jcols[i];
        std::vector<int32_t>& tup = out.Jtup[i];  // [ncols][n-1]
        int64_t P = 1;
        for (int q = 0; q < nr; ++q) P *= sh.d[rest[q]];
        SplitMix g = stream_for(seed, t, i, 1);
        cols = floyd(g, sh.m[i], P);
        tup.resize(cols.size() * nr);
        for (size_t c = 0; c < cols.size(); ++c) {
            int64_t rem = cols[c];
            for (int q = nr - 1; q >= 0; --q) {
                int64_t dq = sh.d[rest[q]];
                tup[c * nr + q] = (int32_t)(rem % dq);
                rem /= dq;
            }
        }
    }
}

}  // namespace rtcur
