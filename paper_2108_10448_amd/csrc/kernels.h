// Device kernels of the RTCUR hot loop for gfx950 (wave64).
//
// Data layout in HBM (all block-sized buffers share one layout):
//   block 0 (R) then blocks 1..n (C_i), each row-major nrows x ncols;
//   B_i factors d_i x RP (RP = rank padded to 4/8/16 with zero columns);
//   H_b = (G x_{j != mode} B_j)(columns of block b), RP x ncols per block;
//   W_i, Y_i (float64) s_i x RP; Z_i (float64) RP x m_i.
// With these, L on any block entry (x, c) is sum_p B_mode[x][p] H_b[p][c]:
// the Tucker form G x_i B_i of L = R x_i (C_i U_i^+) (equation 8), where
// U_i^+ = V_i S_i^-1 W_i^T, G = R x_i W_i^T and B_i = C_i V_i S_i^-1.
//
// Cross-workgroup reductions never use in-kernel fences: each launch writes
// per-workgroup partials and the next launch (after the kernel boundary has
// made them visible) sums them in a fixed order, so every result is bitwise
// reproducible.  Streaming loops issue all their global loads before using
// any of them, so that many loads are in flight per wave.
#pragma once

#include <hip/hip_bf16.h>

#include "internal.h"

namespace rtcur {

constexpr int kThreads = 256;      // 4 waves of 64
constexpr int kTileRows = 16;      // rows per gather / threshold tile
constexpr int kTileCols = 256;     // one column per thread
constexpr int kGramMinChunk = 2048; // Gram: columns per work item (at least)
constexpr int kGramMaxKC = 64;     // Gram: column chunks per output tile (at most)
constexpr int kGramKCGroup = 4;    // chunks summed per load round in the eigensolver
constexpr int kBfacRowsPerWave = 4;
constexpr int kBfacRows = 4 * kBfacRowsPerWave;

enum HtFlags { kHaveL = 1, kDoE = 2, kDoHT = 4, kDecide = 8, kFirstGather = 16,
               kIfRunning = 32 /* gather: skip once the stop flag is raised */ };

typedef double v4d __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- helpers

// Wave64 reductions on DPP lane moves (no LDS round trips): quad swaps,
// half-row and row mirrors, then row broadcasts 15 and 31 fold the four
// rows into lane 63, which is read back for every lane.  Fixed order.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane63(double v) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// v of lane l (l wave-uniform), in every lane
__device__ __forceinline__ double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// sum over each quad of lanes (xor 1, xor 2), result in all four lanes
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_mov<0xB1, 0xF>(v);  // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E, 0xF>(v);  // quad_perm [2,3,0,1]
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    v = quad_sum(v);
    v += dpp_mov<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_mov<0x140, 0xF>(v);  // row_mirror
    v += dpp_mov<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
    v += dpp_mov<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
    return lane63(v);
}

__device__ __forceinline__ double wave_max(double v) {
    // max is idempotent: moves from disabled rows contribute 0 <= |x|, so
    // this is only used on non-negative values
    v = fmax(v, dpp_mov<0xB1, 0xF>(v));
    v = fmax(v, dpp_mov<0x4E, 0xF>(v));
    v = fmax(v, dpp_mov<0x141, 0xF>(v));
    v = fmax(v, dpp_mov<0x140, 0xF>(v));
    v = fmax(v, dpp_mov<0x142, 0xA>(v));
    v = fmax(v, dpp_mov<0x143, 0xC>(v));
    return lane63(v);
}

// Sum over all threads of the workgroup in a fixed order (NW waves); every
// thread gets the result.  red must hold NW doubles.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += red[w];
    return t;
}

template <int NW>
__device__ __forceinline__ double block_max(double v, double* red) {
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t = fmax(t, red[w]);
    return t;
}

// The stop flag is only ever raised by an earlier launch (or by a
// workgroup whose siblings' results are then discarded), so a plain load
// after the kernel boundary sees it.
__device__ __forceinline__ bool stopped(const DevState* st) {
    return *(volatile const int*)&st->stop != 0;
}

// The same flag for kernels that issue their first loads before testing it:
// a relaxed device-scope atomic load, which (unlike a volatile one) lets the
// compiler place its wait at the first use, so that the flag's round trip
// overlaps the kernel's first data loads instead of stalling every wave at
// entry.  Only an earlier launch raises the flag where a kernel tests it
// per thread; where a sibling workgroup of the same launch can raise it,
// the kernel shares one thread's value through LDS.
__device__ __forceinline__ int stop_flag(const DevState* st) {
    return __hip_atomic_load(&st->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------------------- set-up

// Loop state of a new solve, and zeroed factors (so that a k = 0 result
// reconstructs to L = 0) and error history, in one launch.
// The iteration index k of a launch: its argument, or with k = -1 the
// device's own count (set by k_set_iter before a replayed iteration graph,
// advanced once per iteration by the Gram launch).
__device__ __forceinline__ int iter_of(int kcur, const DevState* st) {
    return kcur >= 0 ? kcur : st->iter;
}

__global__ void k_set_iter(DevState* st, int k) {
    if (threadIdx.x == 0) st->iter = k;
}

__global__ __launch_bounds__(kThreads) void k_init_state(DevState* st, double zeta0,
                                                         uint32_t* bf, int64_t bf_words,
                                                         double* bd, int64_t nbd, double* gd,
                                                         int ngd, double* hist, int nhist) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->stop = 0;
        st->status = 0;
        st->final_iter = 0;
        st->converged = 0;
        st->zeta0 = zeta0;
        st->den = 0.0;
        st->eig_steps = 0;
        st->eig_unconverged = 0;
        st->e_prev = -1.0;
        st->e_last = -1.0;
        st->iter = 0;
        for (int j = 0; j < 4; ++j) st->counter[j] = 0u;
        for (int j = 0; j < kMaxModes; ++j) st->eigest[j] = 0.0;
    }
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = t; e < bf_words; e += stride) bf[e] = 0u;
    for (int64_t e = t; e < nbd; e += stride) bd[e] = 0.0;
    for (int64_t e = t; e < ngd; e += stride) gd[e] = 0.0;
    for (int64_t e = t; e < nhist; e += stride) hist[e] = 0.0;
}

// Clear the stop flag to continue the loop from the current iterate (the
// FP32 refinement sweep after the bfloat16 iterations); the loop state
// otherwise stays.
__global__ void k_resume(DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->stop = 0;
        st->status = 0;
        st->converged = 0;
    }
}

// The next sample's index data from its staging slot into the index region
// (RTCUR-R with iterations queued ahead), unless the loop has stopped: the
// returned iterate keeps its own sample.  nbytes is a multiple of 16.
__global__ __launch_bounds__(kThreads) void k_take_sample(uint4* __restrict__ dst,
                                                          const uint4* __restrict__ src,
                                                          int64_t n16, const DevState* st) {
    if (stopped(st)) return;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n16;
         e += (int64_t)gridDim.x * kThreads)
        dst[e] = src[e];
}

// Column index data of the blocks whose columns are the Cartesian product
// of the other modes' sampled indices (bit b of prod_mask: block b; the R
// block always, the C_i under chidori sampling): column c of block b takes
// the other modes in increasing order, the last fastest, and gets
// cidx[q][c] = I_{j_q}[pos_q] and colx[c] = sum_q I_{j_q}[pos_q] * xstride_{j_q}.
// Block b = blockIdx.y.  With st, returns at once when the loop has stopped
// (the index data then stays that of the returned iterate).
__global__ __launch_bounds__(kThreads) void k_expand_cols(Prob P, int prod_mask,
                                                          const DevState* st) {
    if (st && stopped(st)) return;
    const int b = blockIdx.y;
    if (!((prod_mask >> b) & 1)) return;
    const BlockDev& bd = P.blk[b];
    int rest[kMaxModes - 1];
    int nr = 0;
    for (int j = 0; j < P.n; ++j)
        if (j != bd.mode) rest[nr++] = j;
    const int64_t nc = bd.ncols;
    int64_t* colx = const_cast<int64_t*>(bd.colx);
    int32_t* cidx = const_cast<int32_t*>(bd.cidx);
    for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < nc;
         c += (int64_t)gridDim.x * kThreads) {
        int64_t rem = c, off = 0;
        for (int q = nr - 1; q >= 0; --q) {
            const int j = rest[q];
            const int64_t pos = rem % P.s[j];
            rem /= P.s[j];
            const int32_t v = P.I[j][pos];
            off += (int64_t)v * P.xstride[j];
            cidx[(int64_t)q * nc + c] = v;
        }
        colx[c] = off;
    }
}

// bfloat16 block entries to float (exact).
__global__ __launch_bounds__(kThreads) void k_widen(const __hip_bfloat16* __restrict__ in,
                                                    int64_t N, float* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < N;
         e += (int64_t)gridDim.x * kThreads)
        out[e] = (float)in[e];
}

// zeta_0 = ||X||_inf over the whole tensor (one full read) plus a
// non-finite check; part: 2 doubles per workgroup, finished by k_absmax_fin.
template <typename TX>
__global__ __launch_bounds__(kThreads) void k_absmax(const TX* __restrict__ X,
                                                     int64_t N, double* part) {
    __shared__ double red[4];
    constexpr int U = 8;
    double mx = 0.0, bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; e0 < N;
         e0 += stride * U) {
        TX v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * stride;
            v[u] = X[e < N ? e : e0];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double d = (double)v[u];
            if (!isfinite(d)) bad = 1.0;
            mx = fmax(mx, fabs(d));
        }
    }
    const double bm = block_max<4>(mx, red);
    const double bb = block_max<4>(bad, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = bm;
        part[2 * blockIdx.x + 1] = bb;
    }
}

__global__ __launch_bounds__(kThreads) void k_absmax_fin(const double* part, int nparts,
                                                         DevState* st) {
    __shared__ double red[4];
    double m = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < nparts; t += kThreads) {
        m = fmax(m, part[2 * t]);
        b = fmax(b, part[2 * t + 1]);
    }
    m = block_max<4>(m, red);
    b = block_max<4>(b, red);
    if (threadIdx.x == 0) {
        st->zeta0 = m;
        if (b != 0.0) {
            st->stop = 1;
            st->status = RTCUR_E_NONFINITE;
        }
    }
}

// ------------------------------------------------------------------ gather
// X_Omega: R = X(I_1..I_n), C_i = X_(i)(:, J_i) (Algorithm 1, equation 9),
// with per-tile squared sums for the denominator of e^(k) (equation 14).
template <typename TX, typename T, int TR = kTileRows>
__global__ __launch_bounds__(kThreads) void k_gather(
    const TX* __restrict__ X, Prob P, const int4* __restrict__ tiles,
    T* __restrict__ XO, double* part, const DevState* st, int flags) {
    __shared__ double red[4];
    if ((flags & kIfRunning) && stopped(st)) return;  // uniform
    const int4 tl = tiles[blockIdx.x];
    const BlockDev& bd = P.blk[tl.x];
    const int c = tl.z + threadIdx.x;
    const int rows = min(TR, bd.nrows - tl.y);
    const bool valid = c < bd.ncols;
    const int cc = valid ? c : bd.ncols - 1;
    const int64_t cx = bd.colx[cc];
    const int64_t rs = P.xstride[bd.mode];
    TX v[TR];
#pragma unroll
    for (int x = 0; x < TR; ++x) {
        const int xr = tl.y + (x < rows ? x : rows - 1);
        const int64_t xi = bd.rowidx ? bd.rowidx[xr] : xr;
        v[x] = X[xi * rs + cx];
    }
    double acc = 0.0, bad = 0.0;
#pragma unroll
    for (int x = 0; x < TR; ++x) {
        if (valid && x < rows) {
            const T t = (T)v[x];
            XO[bd.off + (int64_t)(tl.y + x) * bd.ncols + c] = t;
            const double dv = (double)t;
            if (!isfinite(dv)) bad = 1.0;
            acc += dv * dv;
        }
    }
    const double sa = block_sum<4>(acc, red);
    const double sb = block_sum<4>(bad, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa;
        part[2 * blockIdx.x + 1] = sb;
    }
}

// Denominator of e^(k): sum over blocks (in block order) of the block norms.
__global__ __launch_bounds__(kThreads) void k_den(Prob P, const double* part, int flags,
                                                  DevState* st) {
    __shared__ double red[4];
    if ((flags & kIfRunning) && stopped(st)) return;  // uniform
    double den = 0.0, badall = 0.0;
    for (int b = 0; b < P.nblk; ++b) {
        double v = 0.0, w = 0.0;
        for (int t = P.blk[b].tile0 + threadIdx.x; t < P.blk[b].tile1; t += kThreads) {
            v += part[2 * t];
            w += part[2 * t + 1];
        }
        v = block_sum<4>(v, red);
        w = block_sum<4>(w, red);
        den += sqrt(v);
        badall += w;
    }
    if (threadIdx.x == 0) {
        st->den = den;
        if (badall != 0.0) {
            st->stop = 1;
            st->status = RTCUR_E_NONFINITE;
        } else if (den == 0.0 && (flags & kFirstGather)) {
            // every sampled entry is zero: L = 0 is the answer (k = 0)
            st->stop = 1;
            st->status = RTCUR_OK;
            st->final_iter = 0;
            st->converged = 1;
        }
    }
}

// ---------------------------------------------- fused residual + threshold
// For iteration k+1 on every block entry (Section 3.3, equations 11, 13, 14):
//   L^k = sum_p B[x][p] H[p][c]              (formed on the fly, never stored)
//   E   = C^k - L^k  -> per-tile sums of E^2 (numerator of e^(k))
//   D   = X - L^k;  S = D if |D| > zeta_{k+1} else 0;  C^{k+1} = X - S
// zeta_{k+1} = gamma^(k+1) zeta_0 by repeated multiplication (equation 12),
// or, with a schedule of multipliers c_j of zeta_0, zeta_j = c_j zeta_0 for
// j <= nsched and the decay by gamma from the last of them beyond.
// T: factor and arithmetic type; TB: block storage type (T, or bfloat16
// with T = float).
template <typename T, int RP, typename TB = T, int TR = kTileRows>
__global__ __launch_bounds__(kThreads) void k_ht(
    Prob P, const int4* __restrict__ tiles, const TB* __restrict__ XO,
    const TB* __restrict__ Cold, TB* __restrict__ Cnew,
    uint64_t* __restrict__ mask, const T* __restrict__ Bf,
    const T* __restrict__ H, double gamma, int kcur, int flags,
    double* __restrict__ part, const DevState* st) {
    const int sf = stop_flag(st);
    __shared__ T brow[TR][RP];
    __shared__ double red[4];
    const bool haveL = flags & kHaveL, doE = flags & kDoE, doHT = flags & kDoHT;
    const int4 tl = tiles[blockIdx.x];
    const BlockDev& bd = P.blk[tl.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int c = tl.z + tid;
    const bool valid = c < bd.ncols;
    const int cc = valid ? c : bd.ncols - 1;
    const int rows = min(TR, bd.nrows - tl.y);
    // all loads first (the threshold below comes after them: its chain of
    // dependent loads of the loop state would otherwise delay every one)
    TB xb[TR], cb[TR];
    const int64_t base = bd.off + (int64_t)tl.y * bd.ncols + cc;
#pragma unroll
    for (int x = 0; x < TR; ++x) {
        const int64_t e = base + (int64_t)(x < rows ? x : rows - 1) * bd.ncols;
        xb[x] = doHT ? XO[e] : TB(0.0f);
        cb[x] = doE ? Cold[e] : TB(0.0f);
    }
    T h[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) h[p] = T(0);
    if (haveL) {
        // rows p >= r of a block's H are padding: never written, not read
#pragma unroll
        for (int p = 0; p < RP; ++p)
            if (p < bd.r) h[p] = H[bd.hoff + (int64_t)p * bd.ncols + cc];  // (uniform)
    }
    kcur = iter_of(kcur, st);
    double zeta = st->zeta0;
    if (kcur < P.nsched) {
        zeta *= P.zsched[kcur];
    } else {
        int j = 0;
        if (P.nsched > 0) {
            zeta *= P.zsched[P.nsched - 1];
            j = P.nsched;
        }
        for (; j <= kcur; ++j) zeta *= gamma;
    }
    if (sf) return;
    if (haveL) {
        for (int q = tid; q < (TR * RP <= kThreads ? kThreads : TR * RP); q += kThreads) {
            if (TR * RP <= kThreads && q >= TR * RP) break;
            const int x = q / RP, p = q % RP;
            const int xr = tl.y + (x < rows ? x : rows - 1);
            const int64_t xi = bd.rowidx ? bd.rowidx[xr] : xr;
            brow[x][p] = Bf[P.boff[bd.mode] + xi * RP + p];
        }
        __syncthreads();
    }
    double e2 = 0.0;
#pragma unroll
    for (int x = 0; x < TR; ++x) {
        if (x >= rows) break;  // uniform
        T L = T(0);
        if (haveL) {
#pragma unroll
            for (int p = 0; p < RP; ++p) L = fma(brow[x][p], h[p], L);
        }
        const int64_t e = bd.off + (int64_t)(tl.y + x) * bd.ncols + c;
        if (doE && valid) {
            const double dv = (double)(T)cb[x] - (double)L;
            e2 += dv * dv;
        }
        if (doHT) {
            const T xv = (T)xb[x];
            const T D = xv - L;
            const bool keep = valid && fabs((double)D) > zeta;
            const T S = keep ? D : T(0);
            if (valid) Cnew[e] = (TB)(xv - S);
            const uint64_t bal = __ballot(keep);
            if (lane == 0 && tl.z + wv * 64 < bd.ncols)
                mask[bd.moff + (int64_t)(tl.y + x) * bd.words + (tl.z >> 6) + wv] = bal;
        }
    }
    if (flags & kDecide) {
        const double se = block_sum<4>(e2, red);
        if (tid == 0) part[blockIdx.x] = se;
    }
}

// e^(k) = sum_b ||E_b||_F / den from the per-tile partials of k_ht; raises
// the stop flag when e^(k) <= tol (or is not finite).  One workgroup.
__device__ void decide_block(const Prob& P, const double* part, int kcur, double tol,
                             double* err_hist, DevState* st, double* red) {
    double num = 0.0;
    for (int b = 0; b < P.nblk; ++b) {
        double v = 0.0;
        for (int t = P.blk[b].tile0 + threadIdx.x; t < P.blk[b].tile1; t += kThreads)
            v += part[t];
        v = block_sum<4>(v, red);
        num += sqrt(v);
    }
    if (threadIdx.x == 0) {
        const double e = num / st->den;
        err_hist[kcur] = e;
        st->e_prev = st->e_last;
        st->e_last = e;
        if (!isfinite(e)) {
            st->stop = 1;
            st->status = RTCUR_E_NONFINITE;
            st->final_iter = kcur;
        } else if (e <= tol) {
            st->stop = 1;
            st->status = RTCUR_OK;
            st->converged = 1;
            st->final_iter = kcur;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_decide(Prob P, const double* part, int kcur,
                                                     double tol, double* err_hist,
                                                     DevState* st) {
    __shared__ double red[4];
    if (stopped(st)) return;
    decide_block(P, part, kcur, tol, err_hist, st, red);
}

// -------------------------------------------------------- Gram of U_i rows
// Gram_i = U_i U_i^T, U_i = C_i(I_i, :) (the matrix whose truncated SVD gives
// U_i^+, equation 9), in float64 on the matrix cores.  One work item is a
// 16x16 output tile (upper triangle only) over one column chunk: the tile's
// 16 + 16 rows are staged through LDS in panels of 256 columns with
// coalesced loads (the loads of the panel after next in flight during this
// panel's products), and each wave runs a chain of V_MFMA_F64_16X16X4 over its 64
// columns of the panel (lane l feeds row l%16 at column 4q + l/16 of
// product q; the accumulator's register v of lane l is row 4v + l/16,
// column l%16).  The eigensolver adds the per-chunk tiles in order.  With
// `decide`, one extra workgroup forms e^(k) from the threshold pass's
// partials.
constexpr int kGramPanel = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gram(
    Prob P, const T* __restrict__ C, const int4* __restrict__ items, int nitems,
    double* __restrict__ gpart, int decide, const double* hpart, int kcur, double tol,
    double* err_hist, DevState* st) {
    const int sf = stop_flag(st);
    constexpr int LD = kGramPanel + (sizeof(T) == 8 ? 1 : 2);  // bank-spread row stride
    __shared__ T pan[32 * LD];
    __shared__ double sacc[4][256];
    if ((int)blockIdx.x == nitems) {
        if (decide && !sf) {
            const int kc = iter_of(kcur, st);
            decide_block(P, hpart, kc, tol, err_hist, st, &sacc[0][0]);
            // (every thread read the count before decide_block's barriers)
            if (kcur < 0 && threadIdx.x == 0) st->iter = kc + 1;
        }
        return;
    }
    const int4 it = items[blockIdx.x];
    const int i = it.x, ta = it.y & 0xffff, tb = it.y >> 16;
    const int kc = it.z & 0xffff;
    const bool same = ta == tb;  // diagonal tile: B rows are the A rows
    const BlockDev& bd = P.blk[1 + i];
    const int s = P.s[i], m = bd.ncols;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, rr = lane & 15;
    const int cb = kc * P.gchunk[i], ce = min(cb + P.gchunk[i], m);
    // this thread loads column (panel + tid) of the tile's rows
    const T* rowp[32];
    bool rowok[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const int a = (j < 16 ? ta : tb) * 16 + (j & 15);
        rowok[j] = a < s && (j < 16 || !same);
        rowp[j] = C + bd.off + (int64_t)P.I[i][a < s ? a : s - 1] * m;
    }
    // unconditional loads at clamped addresses (a branch per load would
    // serialise them); the mask is applied when a panel goes to LDS.  Two
    // register sets alternate, so each panel's loads have two panels of
    // products to arrive.
    T va[32], vb[32];
    bool ina = false, inb = false;
    auto load = [&](T (&vv)[32], bool& in, int p0) {
        const int c = p0 + tid;
        in = c < ce;
        const int cs = in ? c : cb;
#pragma unroll
        for (int j = 0; j < 32; ++j) vv[j] = rowp[j][cs];
    };
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    const int boff = same ? 0 : 16;
    load(va, ina, cb);
    if (cb + kGramPanel < ce) load(vb, inb, cb + kGramPanel);
    // the decision workgroup of this launch may raise the stop flag while
    // the waves of this one read it: thread 0's value decides for all
    __shared__ int sflag;
    if (tid == 0) sflag = sf;
    __syncthreads();
    if (sflag) return;  // uniform
    for (int p0 = cb; p0 < ce; p0 += 2 * kGramPanel) {
        {
            const bool in = ina;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 32; ++j) pan[j * LD + tid] = (in && rowok[j]) ? va[j] : T(0);
            __syncthreads();
            if (p0 + 2 * kGramPanel < ce) load(va, ina, p0 + 2 * kGramPanel);
            const T* pa = pan + rr * LD + 64 * w + g;
            const T* pb = pan + (boff + rr) * LD + 64 * w + g;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)pa[4 * q], (double)pb[4 * q],
                                                           acc, 0, 0, 0);
        }
        if (p0 + kGramPanel >= ce) break;
        {
            const bool in = inb;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 32; ++j) pan[j * LD + tid] = (in && rowok[j]) ? vb[j] : T(0);
            __syncthreads();
            if (p0 + 3 * kGramPanel < ce) load(vb, inb, p0 + 3 * kGramPanel);
            const T* pa = pan + rr * LD + 64 * w + g;
            const T* pb = pan + (boff + rr) * LD + 64 * w + g;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)pa[4 * q], (double)pb[4 * q],
                                                           acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) sacc[w][(4 * u + g) * 16 + rr] = acc[u];
    __syncthreads();
    gpart[(int64_t)blockIdx.x * 256 + tid] =
        ((sacc[0][tid] + sacc[1][tid]) + sacc[2][tid]) + sacc[3][tid];
}

// ------------------------------------------------ truncated eigensolver
// Top-r eigenspace of Gram_i = U_i U_i^T in float64, one 256-thread
// workgroup per mode, thread a owning row a of the s x r iterates: the Gram
// is assembled (in LDS when it fits) from k_gram's tiles; subspace
// iteration (warm-started from the previous iterate's W_i under RTCUR-F,
// from the previous B_i's rows at the new I_i under RTCUR-R) with
// Cholesky-QR orthonormalisation runs until the residual
// ||G Q - Q T||_F <= rtol ||T||_F with T = Q^T G Q.  Then W_i = Q and
// Y_i = Q T^-1, so that the truncated pseudo-inverse is
// U_i^+ = U_i^T Y_i W_i^T: the operator V_r S_r^-1 W_r^T of the SVD written
// in another orthonormal basis of the same subspace.  Padded columns
// r..RP-1 stay zero.

__device__ __forceinline__ uint32_t eig_hash(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return h;
}

// Start-block entry (row a, column p) uniform in (-1, 1) from the hash's top
// 24 bits: such a block has full column rank with probability one (a +-1
// pattern need not: the 10 x 5 one of this hash has rank 4).
__device__ __forceinline__ double eig_start(uint32_t a, uint32_t p, uint32_t salt) {
    return (double)(eig_hash(a, p + 131u * salt) >> 8) * 0x1p-23 - 1.0 + 0x1p-24;
}

// Element (row, col) of the eigensolver's row-major s x RP blocks in LDS
// (sh.qs, sh.zs): the column index XOR the row's low bits, so that a
// thread's own row (lanes on consecutive rows, RP doubles apart) spreads
// over the banks instead of landing on one, while a row stays contiguous
// for the matrix-core operand loads (lanes on the columns of one row).
template <int RP>
__device__ __forceinline__ int rsw(int row, int col) {
    return row * RP + (col ^ (row & (RP - 1)));
}

template <int RP>
// The small arrays come first so that their fixed addresses fit the 16-bit
// immediate offset of LDS instructions (no address register each); the row
// arrays, addressed per thread anyway, come last.
struct EigShared {
    double tm[RP * RP], mm[RP * RP];       // T = Q^T Z, M = Z^T Z
    double vv[RP * RP];                    // Rayleigh-Ritz: eigenvectors of T
    double dv[RP];                         // RP = 16: 1 / R_jj of the factor in mm
    double th[RP], jc[RP], js[RP];         // eigenvalues; one Jacobi round's rotations
    double red[4];
    int jp[RP], ord[RP];                   // rotation partners; decreasing order
    int gsteps;                            // steps of the guarded iteration
    int stopf;                             // the stop flag at entry
    int ok;
    int cok;                               // RP = 16: the factor's pivots were positive
    double part[4][256];                   // per-wave 16 x 16 MFMA partials
    double part2[4][256];                  // second set (T and M together)
    double qs[kMaxS * RP];                 // Q rows; rows s..sp-1 stay zero
    double zs[kMaxS * RP];                 // Z = G Q rows; rows s..sp-1 stay zero
};

// T = Q^T Z (when wantT) and M = Z^T Z from the rows in LDS (sp = s rounded
// up to 16, rows beyond s zero) on the float64 matrix cores: waves 0 and 1
// sum T over the two halves of the rows, waves 2 and 3 sum M; lane l feeds
// column l%16 at row 4j + l/16 of product j.  The halves are added in a
// fixed order.
template <int RP>
__device__ void eig_tm(int sp, bool wantT, EigShared<RP>& sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4, cc = col < RP ? col : RP - 1;
    const bool isM = w >= 2;
    const int nk = sp >> 2, half = w & 1;
    const int j0 = half ? nk / 2 : 0, j1 = half ? nk : nk / 2;
    // two independent chains (even and odd products), added at the end
    v4d acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    if (isM || wantT) {
        for (int j = j0; j < j1; j += 2) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int jj = j + u < j1 ? j + u : j0;
                const int b = 4 * jj + kq;
                double zv = sh.zs[rsw<RP>(b, cc)];
                double qv = sh.qs[rsw<RP>(b, cc)];
                zv = (col < RP && j + u < j1) ? zv : 0.0;
                qv = col < RP ? qv : 0.0;
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(isM ? zv : qv, zv, acc[u], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sh.part[w][(4 * v + kq) * 16 + col] = acc[0][v] + acc[1][v];
    __syncthreads();
    if (threadIdx.x < RP * RP) {
        const int p = threadIdx.x / RP, t = threadIdx.x % RP;
        if (wantT) sh.tm[threadIdx.x] = sh.part[0][p * 16 + t] + sh.part[1][p * 16 + t];
        sh.mm[threadIdx.x] = sh.part[2][p * 16 + t] + sh.part[3][p * 16 + t];
    }
    __syncthreads();
}

// Cholesky of M's r x r block (M in LDS, row stride RP) into upper R in
// registers, in every thread, with Rinv_jj = 1 / R_jj from one reciprocal
// square root (no divisions); identity beyond r.  Returns false if a pivot
// is not positive.
template <int RP>
__device__ __forceinline__ bool eig_chol(const double* M, int r, double (&R)[RP][RP],
                                         double (&dinv)[RP]) {
    // straight-line code (selects, no branches on r) so that the LDS reads
    // of M are not serialised
    bool ok = true;
#pragma unroll
    for (int j = 0; j < RP; ++j) {
#pragma unroll
        for (int q = 0; q < RP; ++q) R[j][q] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < RP; ++j) {
        const bool jin = j < r;
        double d = M[j * RP + j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= R[k][j] * R[k][j];
        ok = ok && (!jin || d > 0.0);
        const double ri = rsqrt((jin && d > 0.0) ? d : 1.0);
        dinv[j] = ri;
        R[j][j] = jin ? d * ri : 1.0;
#pragma unroll
        for (int q = j + 1; q < RP; ++q) {
            double v = M[j * RP + q];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= R[k][j] * R[k][q];
            R[j][q] = (jin && q < r) ? v * ri : 0.0;
        }
    }
    return ok;
}

// q = z R^-1 for this thread's row.
template <int RP>
__device__ __forceinline__ void eig_trsm(const double (&z)[RP], const double (&R)[RP][RP],
                                         const double (&dinv)[RP], double (&q)[RP]) {
#pragma unroll
    for (int p = 0; p < RP; ++p) {
        double v = z[p];
#pragma unroll
        for (int k = 0; k < p; ++k) v -= q[k] * R[k][p];
        q[p] = v * dinv[p];
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky-QR factor of an RP x RP matrix M in LDS (its r x r block; the
// identity beyond r) and the solve q = z R^-1 of a thread's row.  RP <= 8: R
// in the registers of every thread (eig_chol, eig_trsm).  RP = 16 (where R
// would not fit in every thread's registers): wave 0 factors M with one
// column of R per lane (the same operations, in the same order, as eig_chol)
// and writes R over M's upper triangle, 1 / R_jj to sh.dv; the solve reads R
// from there.  M must be sh.mm.  Called by every thread.
template <int RP, bool kLds = (RP > 8)>
struct EigChol {
    double R[RP][RP], di[RP];
    __device__ __forceinline__ bool factor(double* M, int r, EigShared<RP>& sh) {
        (void)sh;
        return eig_chol<RP>(M, r, R, di);  // same value in every thread
    }
    __device__ __forceinline__ void solve(const double (&z)[RP], double (&q)[RP],
                                          const EigShared<RP>& sh) const {
        (void)sh;
        eig_trsm<RP>(z, R, di, q);
    }
};

template <int RP>
struct EigChol<RP, true> {
    __device__ __forceinline__ bool factor(double* M, int r, EigShared<RP>& sh) {
        if (threadIdx.x < 64) {
            // lane c < RP holds column c of R in registers and forms it left
            // to right: R[j][c] = (M[j][c] - sum_{k<j} R[k][j] R[k][c]) / R_jj,
            // the R[k][j] read from lane j; the terms are subtracted in
            // increasing k, the order in which a right-looking update applies
            // them, so that R is the same to the bit.  Lanes >= RP shadow
            // lane c % RP and store nothing.
            const int lane = threadIdx.x, c = lane & (RP - 1);
            double R[RP];
#pragma unroll
            for (int k = 0; k < RP; ++k) R[k] = M[k * RP + c];
            bool ok = true;
            double dc = 1.0;  // 1 / R_cc
#pragma unroll
            for (int j = 0; j < RP; ++j) {
                double v = R[j];
#pragma unroll
                for (int k = 0; k < j; ++k) v -= lane_value(R[k], j) * R[k];
                const bool jin = j < r;
                const double d = lane_value(v, j);  // the pivot
                ok = ok && (!jin || d > 0.0);
                const double ri = rsqrt((jin && d > 0.0) ? d : 1.0);
                if (c == j) dc = ri;
                // row j of R: the pivot, the scaled entries right of it
                // inside the r x r block, zero elsewhere (identity beyond r);
                // entries below the diagonal (j > c) are not part of R
                R[j] = c == j ? (jin ? d * ri : 1.0) : (c > j ? ((jin && c < r) ? v * ri : 0.0) : 0.0);
            }
            if (lane < RP) {
#pragma unroll
                for (int k = 0; k < RP; ++k)
                    if (k <= c) M[k * RP + c] = R[k];
                sh.dv[c] = c < r ? dc : 1.0;
            }
            if (lane == 0) sh.cok = ok ? 1 : 0;
        }
        __syncthreads();
        return sh.cok != 0;
    }
    __device__ __forceinline__ void solve(const double (&z)[RP], double (&q)[RP],
                                          const EigShared<RP>& sh) const {
        // (a scheduling barrier per column keeps the compiler from hoisting
        // all of R's loads at once, which would not fit in registers)
#pragma unroll
        for (int p = 0; p < RP; ++p) {
            double v = z[p];
#pragma unroll
            for (int k = 0; k < p; ++k) v -= q[k] * sh.mm[k * RP + p];
            q[p] = v * sh.dv[p];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
};

// The Gram of a mode (sp x sp, sp = s rounded up to 16, zero beyond s) is
// kept as its upper-triangular 16 x 16 tiles (ta <= tb) in the order
// ta-major, tb increasing -- the order of k_gram's tile pairs -- 256 doubles
// each, entry (r, c) of a tile at r * 16 + (c ^ r): the XOR spreads both a
// tile's rows and its columns over the LDS banks.  Entry (a, b) of a lower
// tile is entry (b, a) of its mirror.  Returns the offset of G[16 t + x][16 kt + y]
// for x, y < 16.
__device__ __forceinline__ int gram_at(int t, int kt, int x, int y, int nt) {
    const bool up = t <= kt;
    const int ta = up ? t : kt, tb = up ? kt : t;
    const int tile = ta * nt - ta * (ta - 1) / 2 + (tb - ta);
    const int r = up ? x : y, c = up ? y : x;
    return tile * 256 + r * 16 + (c ^ r);
}

// Index of the tile pair (min(t, kt), max(t, kt)) in gram_at's order.
__device__ __forceinline__ int gram_tile(int t, int kt, int nt) {
    const int ta = t <= kt ? t : kt, tb = t <= kt ? kt : t;
    return ta * nt - ta * (ta - 1) / 2 + (tb - ta);
}

// A lane's operand offsets for the products Z = G Q below (lane l: Gram
// tile row l % 16 at k-step 4u + l / 16, and Q's row 4u + l / 16 of a
// 16-row set at column l % 16): gram_at's offset within a tile is gu[u]
// (upper tile) or gl[u] (lower tile, read through its mirror), and
// rsw(16 j + 4u + l / 16, cc) is 16 j RP + qo[u].  Computed once, so that a
// step's addresses are a wave-uniform base plus one of these registers.
template <int RP>
struct GqLane {
    int gu[4], gl[4], qo[4];
    __device__ __forceinline__ GqLane(int col, int kq, int cc) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int y = 4 * u + kq;
            gu[u] = col * 16 + (y ^ col);
            gl[u] = y * 16 + (col ^ y);
            qo[u] = y * RP + (cc ^ (y & (RP - 1)));
        }
    }
};

// Z = G Q into zs (rows < s, columns < RP) on the float64 matrix cores, G in
// the tile layout above, Q's rows s..sp-1 zero.  Wave w takes the 16-row
// tiles w, w + 4, ...; per tile one accumulator chain over the rows of Q:
// lane l feeds G row 16t + l%16 and Q column l%16 at row 4j + l/16 of
// product j; accumulator register v of lane l is row 4v + l/16, column l%16.
template <int RP>
__device__ __forceinline__ void eig_gq(const double* G, int sp, int s, EigShared<RP>& sh) {
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (wave-uniform)
    const int col = lane & 15, kq = lane >> 4, cc = col < RP ? col : RP - 1;
    const int nt = sp >> 4;
    const GqLane<RP> L(col, kq, cc);
    for (int t = w; t < nt; t += 4) {
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < sp; j += 16) {  // sp is a multiple of 16
            double av[4], bv[4];
            const bool up = t <= (j >> 4);
            const double* Gt = G + gram_tile(t, j >> 4, nt) * 256;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = Gt[up ? L.gu[u] : L.gl[u]];
                bv[u] = sh.qs[j * RP + L.qo[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], col < RP ? bv[u] : 0.0, acc,
                                                           0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * t + 4 * v + kq;
            if (row < s && col < RP) sh.zs[rsw<RP>(row, col)] = acc[v];
        }
    }
    __syncthreads();
}

// Eigen-decomposition of the symmetric RP x RP matrix in sh.mm by cyclic
// Jacobi rotations (Golub and Van Loan, the symmetric Schur step with the
// round-robin ordering of RP/2 disjoint rotations per round), run by wave 0
// alone: on return sh.vv holds the eigenvectors as columns, sh.th the
// eigenvalues and sh.ord the indices by decreasing eigenvalue.  Sweeps stop
// once the off-diagonal mass is below 1e-29 of the diagonal's (squares).
template <int RP>
__device__ void eig_jacobi(EigShared<RP>& sh) {
    const int lane = threadIdx.x;  // 0..63
    constexpr int NE = (RP * RP + 63) / 64;
    double* A = sh.mm;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        const int e = lane + 64 * u;
        if (e < RP * RP) sh.vv[e] = (e / RP == e % RP) ? 1.0 : 0.0;
    }
    wave_sync();
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dg = 0.0;
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = lane + 64 * u;
            const double v = e < RP * RP ? A[e] : 0.0;
            if (e / RP == e % RP) dg += v * v;
            else off += v * v;
        }
        off = wave_sum(off);
        dg = wave_sum(dg);
        if (!(off > 1e-29 * dg)) break;
        for (int k = 0; k < RP - 1; ++k) {
            if (lane < RP / 2) {
                int p = RP - 1, q = k;
                if (lane > 0) {
                    p = (k + lane) % (RP - 1);
                    q = (k - lane + RP - 1) % (RP - 1);
                }
                const double app = A[p * RP + p], aqq = A[q * RP + q], apq = A[p * RP + q];
                double c = 1.0, sn = 0.0;
                if (apq != 0.0) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    sn = t * c;
                }
                // J[p][p] = J[q][q] = c, J[p][q] = sn, J[q][p] = -sn; column i of
                // J is c at row i and js[i] at row jp[i]
                sh.jp[p] = q;
                sh.jp[q] = p;
                sh.jc[p] = c;
                sh.jc[q] = c;
                sh.js[p] = -sn;
                sh.js[q] = sn;
            }
            wave_sync();
            double na[NE], nv[NE];
#pragma unroll
            for (int u = 0; u < NE; ++u) {
                const int e = lane + 64 * u < RP * RP ? lane + 64 * u : 0;
                const int i = e / RP, j = e % RP;
                const int i2 = sh.jp[i], j2 = sh.jp[j];
                const double ci = sh.jc[i], si = sh.js[i], cj = sh.jc[j], sj = sh.js[j];
                // (J^T A J)[i][j] and (V J)[i][j]
                na[u] = ci * (cj * A[i * RP + j] + sj * A[i * RP + j2]) +
                        si * (cj * A[i2 * RP + j] + sj * A[i2 * RP + j2]);
                nv[u] = cj * sh.vv[i * RP + j] + sj * sh.vv[i * RP + j2];
            }
            wave_sync();
#pragma unroll
            for (int u = 0; u < NE; ++u) {
                const int e = lane + 64 * u;
                if (e < RP * RP) {
                    A[e] = na[u];
                    sh.vv[e] = nv[u];
                }
            }
            wave_sync();
        }
    }
    if (lane < RP) {
        const double t = A[lane * RP + lane];
        int rank = 0;
        for (int k = 0; k < RP; ++k) {
            const double u = A[k * RP + k];
            rank += (u > t || (u == t && k < lane)) ? 1 : 0;
        }
        sh.th[lane] = t;
        sh.ord[rank] = lane;
    }
    wave_sync();
}

constexpr int kEigCheck = 4;     // guarded iteration: Rayleigh-Ritz every 4 steps
constexpr int kEigGuardMax = 400;

// (defined below, with the plain iteration it serves first)
template <int RP>
__device__ __forceinline__ void eig_gq_tm(const double* G, int sp, int s, EigShared<RP>& sh);

// Guarded subspace iteration for a slow gap (lambda_{r+1} / lambda_r close
// to 1): the iterate gets m - r extra columns (m = min(RP, s)), so that the
// top-r part converges at lambda_{m+1} / lambda_r, with a Rayleigh-Ritz
// step (T = Q^T G Q diagonalised by eig_jacobi) every kEigCheck steps that
// rotates the basis to Ritz vectors in decreasing order and tests the top-r
// residual ||G q_p - theta_p q_p|| against rtol ||theta_{1..r}||.  Cholesky-QR
// is applied twice per step, because the m-column iterate is worse
// conditioned than the r-column one.  The iterate enters and leaves in
// sh.qs (rows < s): on return it holds the top-r Ritz vectors (zero beyond
// r) when converged (result 1) or the best r columns found (0); after a rank
// loss of the m-column iterate (-1) it is left as it came.  *steps counts
// the steps taken.  Kept out of line so that its registers do not weigh on
// the plain iteration of the caller.
template <int RP>
__device__ __noinline__ int eig_guarded(const double* G, int sp, int s, int r, int m,
                                        double rtol, EigShared<RP>* shp, int* steps_out) {
    EigShared<RP>& sh = *shp;
    const int a = threadIdx.x;
    const bool act = a < s;
    int steps = 0;
    double x[RP], z[RP], q[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) q[p] = act ? sh.qs[rsw<RP>(a, p)] : 0.0;
#pragma unroll
    for (int p = 0; p < RP; ++p)
        x[p] = p < r ? q[p] : ((act && p < m) ? eig_start(a, p, 7u) : 0.0);
    int res = 0;
    for (int it = 0; it <= kEigGuardMax; ++it, ++steps) {
        __syncthreads();
        if (act) {
#pragma unroll
            for (int p = 0; p < RP; ++p) sh.qs[rsw<RP>(a, p)] = x[p];
        }
        __syncthreads();
        eig_gq_tm<RP>(G, sp, s, sh);  // Z = G X, T = X^T Z, M = Z^T Z
#pragma unroll
        for (int p = 0; p < RP; ++p) z[p] = act ? sh.zs[rsw<RP>(a, p)] : 0.0;
        // sh.mm holds Z^T Z of the rows in sh.zs until a Rayleigh-Ritz check
        // rotates them
        bool mfresh = true;
        if (it > 0 && (it % kEigCheck == 0 || it == kEigGuardMax)) {
            mfresh = false;
            if (threadIdx.x < RP * RP) {
                const int p = threadIdx.x / RP, t = threadIdx.x % RP;
                sh.mm[threadIdx.x] = 0.5 * (sh.tm[p * RP + t] + sh.tm[t * RP + p]);
            }
            __syncthreads();
            if (threadIdx.x < 64) eig_jacobi<RP>(sh);
            __syncthreads();
            double xr[RP], zr[RP], rn = 0.0, tn = 0.0;
#pragma unroll
            for (int p = 0; p < RP; ++p) {
                const int o = sh.ord[p] & (RP - 1);  // in range even if a NaN broke the ranking
                double u = 0.0, v = 0.0;
#pragma unroll
                for (int k = 0; k < RP; ++k) {
                    const double w = sh.vv[k * RP + o];
                    u += x[k] * w;
                    v += z[k] * w;
                }
                xr[p] = u;
                zr[p] = v;
                if (p < r) {
                    const double t = sh.th[o];
                    const double d = v - t * u;
                    rn += act ? d * d : 0.0;
                    tn += t * t;
                }
            }
            rn = block_sum<4>(rn, sh.red);
#pragma unroll
            for (int p = 0; p < RP; ++p) {
                x[p] = xr[p];
                z[p] = zr[p];
            }
            if (rn <= rtol * rtol * tn || it == kEigGuardMax) {
                res = rn <= rtol * rtol * tn ? 1 : 0;
                break;
            }
        }
        // Cholesky-QR twice over the m columns
        if (!mfresh) {
            __syncthreads();
            if (act) {
#pragma unroll
                for (int p = 0; p < RP; ++p) sh.zs[rsw<RP>(a, p)] = z[p];
            }
            __syncthreads();
        }
        bool ok = true;
        for (int rep = 0; rep < 2; ++rep) {
            if (rep > 0 || !mfresh) eig_tm<RP>(sp, false, sh);  // M = Z^T Z
            EigChol<RP> ch;
            ok = ch.factor(sh.mm, m, sh);
            if (!ok) break;
            ch.solve(z, x, sh);
            if (rep == 0) {
#pragma unroll
                for (int p = 0; p < RP; ++p) z[p] = x[p];
                if (act) {
#pragma unroll
                    for (int p = 0; p < RP; ++p) sh.zs[rsw<RP>(a, p)] = z[p];
                }
                __syncthreads();
            }
        }
        if (!ok) {
            res = -1;
            break;
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int p = 0; p < RP; ++p) sh.qs[rsw<RP>(a, p)] = res < 0 ? q[p] : (p < r ? x[p] : 0.0);
    }
    if (threadIdx.x == 0) *steps_out = steps;
    __syncthreads();
    return res;
}

// The Gram of one mode from k_gram's per-chunk 16 x 16 tiles into G (the
// tile layout of gram_at): E entries per thread and KG chunks per
// load round, every load of a round issued before the first add; with
// kMulti the rounds repeat over the chunks, which are always added in chunk
// order.
template <int E, int KG, bool kMulti>
__device__ __forceinline__ void gram_assemble(const double* __restrict__ src0, int total,
                                              int nkc, double* G) {
    for (int f0 = threadIdx.x; f0 < total; f0 += E * kThreads) {
        double sum[E];
#pragma unroll
        for (int u = 0; u < E; ++u) sum[u] = 0.0;
        for (int q0 = 0; q0 < (kMulti ? nkc : 1); q0 += KG) {
            double v[E][KG];
#pragma unroll
            for (int u = 0; u < E; ++u) {
                const int f = f0 + u * kThreads < total ? f0 + u * kThreads : f0;
                const double* src = src0 + (int64_t)(f >> 8) * nkc * 256 + (f & 255);
#pragma unroll
                for (int q = 0; q < KG; ++q)  // masked in the sum
                    v[u][q] = src[(int64_t)(q0 + q < nkc ? q0 + q : q0) * 256];
            }
#pragma unroll
            for (int u = 0; u < E; ++u)
#pragma unroll
                for (int q = 0; q < KG; ++q)
                    if (q0 + q < nkc) sum[u] += v[u][q];
        }
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int f = f0 + u * kThreads;
            if (f >= total) continue;
            // tile f / 256, entry (r, c); rows and columns beyond s come out
            // of k_gram as zeros
            const int r = (f >> 4) & 15, c = f & 15;
            G[(f & ~255) + r * 16 + (c ^ r)] = sum[u];
        }
    }
}

// As gram_assemble for at most KG chunks, two neighbouring entries of a tile
// per thread and 16-byte loads: half the load instructions, so that all of
// them (E2 x KG) are in flight at once.
template <int E2, int KG>
__device__ __forceinline__ void gram_assemble2(const double* __restrict__ src0, int total,
                                               int nkc, double* G) {
    for (int f0 = 2 * threadIdx.x; f0 < total; f0 += 2 * E2 * kThreads) {
        double2 v[E2][KG];
#pragma unroll
        for (int u = 0; u < E2; ++u) {
            const int f = f0 + 2 * u * kThreads < total ? f0 + 2 * u * kThreads : f0;
            const double* src = src0 + (int64_t)(f >> 8) * nkc * 256 + (f & 255);
#pragma unroll
            for (int q = 0; q < KG; ++q)  // masked in the sum
                v[u][q] = *reinterpret_cast<const double2*>(src + (int64_t)(q < nkc ? q : 0) * 256);
        }
#pragma unroll
        for (int u = 0; u < E2; ++u) {
            const int f = f0 + 2 * u * kThreads;
            if (f >= total) continue;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int q = 0; q < KG; ++q)
                if (q < nkc) {
                    s0 += v[u][q].x;
                    s1 += v[u][q].y;
                }
            const int r = (f >> 4) & 15, c = f & 15;  // c even: c, c + 1 in one row
            G[(f & ~255) + r * 16 + (c ^ r)] = s0;
            G[(f & ~255) + r * 16 + ((c + 1) ^ r)] = s1;
        }
    }
}

// NP (1 or 2) Z tiles of eig_gq_tm, t and t + 4, side by side: each
// 16-column operand set of Q is loaded once for both, and the two tiles'
// product chains interleave (each chain in its own k order, as alone);
// the epilogues run in tile order.
template <int RP, int NP>
__device__ __forceinline__ void gq_tm_tiles(const double* G, int sp, int s, int nt, int t,
                                            const GqLane<RP>& L, int col, int kq,
                                            EigShared<RP>& sh, v4d& tacc, v4d& macc) {
    // Q^T as the A operand of the T product: A[p][k] = Q[16t + 4v + k][p]
    // (loaded up front, so that a tile's epilogue does not wait on LDS)
    double qa[NP][4];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            qa[k][v] = col < RP ? sh.qs[16 * (t + 4 * k) * RP + L.qo[v]] : 0.0;
    v4d acc[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = v4d{0.0, 0.0, 0.0, 0.0};
    // two operand sets of 16 columns, each loaded while the other one's
    // products run
    double a0[NP][4], b0[4], a1[NP][4], b1[4];
    auto load = [&](double (&av)[NP][4], double (&bv)[4], int j) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int tk = t + 4 * k;
            const bool up = tk <= (j >> 4);
            const double* Gt = G + gram_tile(tk, j >> 4, nt) * 256;
#pragma unroll
            for (int u = 0; u < 4; ++u) av[k][u] = Gt[up ? L.gu[u] : L.gl[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) bv[u] = sh.qs[j * RP + L.qo[u]];
    };
    auto mul = [&](const double (&av)[NP][4], const double (&bv)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double b = col < RP ? bv[u] : 0.0;
#pragma unroll
            for (int k = 0; k < NP; ++k)
                acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[k][u], b, acc[k], 0, 0, 0);
        }
    };
    // (the scheduling barriers keep each set's loads ahead of the other
    // set's products instead of next to their own use)
    load(a0, b0, 0);
    int j = 0;
    for (; j + 32 <= sp; j += 32) {  // sp is a multiple of 16
        load(a1, b1, j + 16);
        __builtin_amdgcn_sched_barrier(0);
        mul(a0, b0);
        load(a0, b0, j + 32 < sp ? j + 32 : j);  // (at the end: reloaded, unused)
        __builtin_amdgcn_sched_barrier(0);
        mul(a1, b1);
    }
    if (j < sp) mul(a0, b0);  // an odd number of 16-column sets
#pragma unroll
    for (int k = 0; k < NP; ++k) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * (t + 4 * k) + 4 * v + kq;
            if (row < s && col < RP) sh.zs[rsw<RP>(row, col)] = acc[k][v];
            tacc = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[k][v], acc[k][v], tacc, 0, 0, 0);
            macc = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[k][v], acc[k][v], macc, 0, 0, 0);
        }
    }
}

// Z = G Q into zs as eig_gq, with T = Q^T Z and M = Z^T Z formed from each
// Z tile while it is still in the accumulators: register v of lane l holds
// Z[16t + 4v + l/16][l%16], which is exactly the B operand (row k = l/16,
// column l%16) of the k-step v over the tile's rows, and for M also its A
// operand (A[m][k] = Z[k][m]).  Per-wave partials are added in wave order.
template <int RP>
__device__ __forceinline__ void eig_gq_tm(const double* G, int sp, int s, EigShared<RP>& sh) {
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (wave-uniform)
    const int col = lane & 15, kq = lane >> 4, cc = col < RP ? col : RP - 1;
    const int nt = sp >> 4;
    const GqLane<RP> L(col, kq, cc);
    v4d tacc = {0.0, 0.0, 0.0, 0.0}, macc = {0.0, 0.0, 0.0, 0.0};
    // wave w takes the tiles w, w + 4, w + 8, ..., two at a time
    for (int t = w; t < nt; t += 8) {
        if (t + 4 < nt)  // (uniform)
            gq_tm_tiles<RP, 2>(G, sp, s, nt, t, L, col, kq, sh, tacc, macc);
        else
            gq_tm_tiles<RP, 1>(G, sp, s, nt, t, L, col, kq, sh, tacc, macc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        sh.part[w][(4 * v + kq) * 16 + col] = tacc[v];
        sh.part2[w][(4 * v + kq) * 16 + col] = macc[v];
    }
    __syncthreads();
    if (threadIdx.x < RP * RP) {
        const int p = threadIdx.x / RP, t = threadIdx.x % RP;
        const int e = p * 16 + t;
        sh.tm[threadIdx.x] = ((sh.part[0][e] + sh.part[1][e]) + sh.part[2][e]) + sh.part[3][e];
        sh.mm[threadIdx.x] = ((sh.part2[0][e] + sh.part2[1][e]) + sh.part2[2][e]) + sh.part2[3][e];
    }
    __syncthreads();
}

// W_i = Q and Y_i = Q T^-1 with T = R^T R (Cholesky of the symmetrised T,
// in sh.mm), the rank test on T, and the step counts; RP <= 8: R in the
// registers of every thread, y = (q R^-1) R^-T by two triangular solves.
// The rank test's ||T^-1||_F is formed by wave 0: lane t < RP solves for
// column t of R^-1 (into sh.vv), then lane (p, t) forms entry (p, t) of
// T^-1 = R^-1 R^-T.
template <int RP>
__device__ __forceinline__ void eig_finish_regs(const Prob& P, int i, int s, int r, int a, bool act,
                                                const double (&q)[RP], bool conv, int steps,
                                                double* __restrict__ Wi, double* __restrict__ Y,
                                                DevState* st, EigShared<RP>& sh) {
    double R[RP][RP], di[RP];
    const bool tok = eig_chol<RP>(sh.mm, r, R, di);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane < RP) {
            double x[RP];
#pragma unroll
            for (int j = RP - 1; j >= 0; --j) {
                double v = j == lane ? 1.0 : 0.0;
#pragma unroll
                for (int k = j + 1; k < RP; ++k) v -= R[j][k] * x[k];
                x[j] = v * di[j];
            }
#pragma unroll
            for (int j = 0; j < RP; ++j) sh.vv[j * RP + lane] = x[j];  // R^-1[j][lane]
        }
        wave_sync();
        // rank test on ||T||_F >= lambda_1 and 1/||T^-1||_F <= lambda_r
        // (flag when lambda_r / lambda_1 may be <= 64 s 2^-52); the padded
        // rows and columns of T and R^-1 are masked out
        double tf = 0.0, tif = 0.0;
        if (lane < RP * RP) {
            const int p = lane / RP, t = lane % RP;
            const bool in = p < r && t < r;
            const double tv = in ? sh.mm[p * RP + t] : 0.0;
            double v = 0.0;  // (R^-1 R^-T)[p][t]
#pragma unroll
            for (int k = 0; k < RP; ++k)
                v += (k >= p && k >= t) ? sh.vv[p * RP + k] * sh.vv[t * RP + k] : 0.0;
            tf = tv * tv;
            tif = in ? v * v : 0.0;
        }
        tf = wave_sum(tf);
        tif = wave_sum(tif);
        if (threadIdx.x == 0) {
            atomicAdd(&st->eig_steps, steps);
            if (!conv) atomicAdd(&st->eig_unconverged, 1);
            // 1 / (||T||_F ||T^-1||_F) <= lambda_r / lambda_1: the next call's
            // stopping scale
            const double qq = tf * tif;
            st->eigest[i] = (qq > 0.0 && isfinite(qq)) ? 1.0 / sqrt(qq) : 0.0;
            if (!isfinite(tf) || !isfinite(tif)) {
                st->stop = 1;
                st->status = RTCUR_E_NONFINITE;
            } else if (!tok || !(tf > 0.0) || 1.0 <= 64.0 * s * 0x1p-52 * sqrt(tf * tif)) {
                st->stop = 1;
                st->status = RTCUR_E_RANK;
            }
        }
    }
    if (act) {
        // y = q T^-1: u = q R^-1, then y R^T = u
        double u[RP], y[RP];
        eig_trsm<RP>(q, R, di, u);
#pragma unroll
        for (int p = RP - 1; p >= 0; --p) {
            double v = u[p];
#pragma unroll
            for (int k = p + 1; k < RP; ++k) v -= R[p][k] * y[k];
            y[p] = v * di[p];
        }
        double* Yi = Y + P.woff[i];
#pragma unroll
        for (int p = 0; p < RP; ++p) {
            Wi[a * RP + p] = p < r ? q[p] : 0.0;
            Yi[a * RP + p] = p < r ? y[p] : 0.0;
        }
    }
}

// As eig_finish_regs for RP = 16: R factored in LDS (EigChol), R^-1 formed
// column by column by the lanes of wave 0 into sh.vv, the rank test's sums
// spread over wave 0's lanes, and Y read back from LDS by every thread.
template <int RP>
__device__ __forceinline__ void eig_finish_lds(const Prob& P, int i, int s, int r, int a, bool act,
                                               bool conv, int steps,
                                               double* __restrict__ Wi, double* __restrict__ Y,
                                               DevState* st, EigShared<RP>& sh) {
    EigChol<RP> ch;
    const bool tok = ch.factor(sh.mm, r, sh);  // R in the upper triangle of sh.mm
    if (threadIdx.x < RP) {
        // column c of R^-1: Ri[c][c] = 1 / R_cc, Ri[j][c] = -(sum_{j < k <= c}
        // R[j][k] Ri[k][c]) / R_jj for j < c, zero below the diagonal
        const int c = threadIdx.x;
        double col[RP];
#pragma unroll
        for (int j = RP - 1; j >= 0; --j) {
            double v = 0.0;
#pragma unroll
            for (int k = j + 1; k < RP; ++k) v += k <= c ? sh.mm[j * RP + k] * col[k] : 0.0;
            col[j] = j > c ? 0.0 : (j == c ? sh.dv[j] : -v * sh.dv[j]);
        }
#pragma unroll
        for (int k = 0; k < RP; ++k) sh.vv[k * RP + c] = col[k];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // rank test on ||T||_F >= lambda_1 and 1/||T^-1||_F <= lambda_r
        // (flag when lambda_r / lambda_1 may be <= 64 s 2^-52); the padded
        // rows and columns of T and R^-1 are masked out
        double tf = 0.0, tif = 0.0;
        for (int e = threadIdx.x; e < RP * RP; e += 64) {
            const int p = e / RP, t = e % RP;
            const bool in = p < r && t < r;
            const double tv = in ? 0.5 * (sh.tm[p * RP + t] + sh.tm[t * RP + p]) : 0.0;
            double v = 0.0;  // (R^-1 R^-T)[p][t]
#pragma unroll
            for (int k = 0; k < RP; ++k)
                v += (k >= p && k >= t) ? sh.vv[p * RP + k] * sh.vv[t * RP + k] : 0.0;
            tf += tv * tv;
            tif += in ? v * v : 0.0;
        }
        tf = wave_sum(tf);
        tif = wave_sum(tif);
        if (threadIdx.x == 0) {
            atomicAdd(&st->eig_steps, steps);
            if (!conv) atomicAdd(&st->eig_unconverged, 1);
            // 1 / (||T||_F ||T^-1||_F) <= lambda_r / lambda_1: the next call's
            // stopping scale
            const double q = tf * tif;
            st->eigest[i] = (q > 0.0 && isfinite(q)) ? 1.0 / sqrt(q) : 0.0;
            if (!isfinite(tf) || !isfinite(tif)) {
                st->stop = 1;
                st->status = RTCUR_E_NONFINITE;
            } else if (!tok || !(tf > 0.0) || 1.0 <= 64.0 * s * 0x1p-52 * sqrt(tf * tif)) {
                st->stop = 1;
                st->status = RTCUR_E_RANK;
            }
        }
    }
    if (act) {
        // y = q T^-1 = (q R^-1) R^-T, q the thread's row of sh.qs
        double qr[RP], u[RP];
#pragma unroll
        for (int k = 0; k < RP; ++k) qr[k] = sh.qs[rsw<RP>(a, k)];
        double* Yi = Y + P.woff[i];
#pragma unroll
        for (int p = 0; p < RP; ++p) Wi[a * RP + p] = p < r ? qr[p] : 0.0;
#pragma unroll
        for (int p = 0; p < RP; ++p) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k <= p; ++k) v += qr[k] * sh.vv[k * RP + p];
            u[p] = v;
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int p = 0; p < RP; ++p) {
            double v = 0.0;
#pragma unroll
            for (int k = p; k < RP; ++k) v += u[k] * sh.vv[p * RP + k];
            Yi[a * RP + p] = p < r ? v : 0.0;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// kLdsGram: the Gram sits in dynamic LDS (else in `gram`); a compile-time
// choice so that its accesses compile to LDS (or global) instructions rather
// than generic ones.
template <int RP, bool kLdsGram>
__global__ __launch_bounds__(kThreads) void k_eig(Prob P, const double* __restrict__ gpart,
                                                  double* __restrict__ gram,
                                                  double* __restrict__ W,
                                                  double* __restrict__ Y,
                                                  const double* __restrict__ Bd, int warm,
                                                  int maxit, double rtol_arg, DevState* st) {
    extern __shared__ double Gl[];  // the Gram's tiles (layout of gram_at), when they fit
    __shared__ EigShared<RP> sh;
    const int i = blockIdx.x;
    const int s = P.s[i], r = P.r[i];
    // rtol_arg > 0: a fixed relative residual.  rtol_arg = -u (the blocks'
    // unit roundoff): scaled to the weakest wanted pair, u sqrt(lambda_r /
    // lambda_1) from the previous call's bound (1e-10 on a first call), so
    // that the subspace error rtol lambda_1 / lambda_r stays at the level
    // u kappa that the blocks' rounding already puts there
    double rtol = rtol_arg;
    if (rtol_arg < 0.0) {
        const double est = st->eigest[i];
        rtol = est > 0.0 ? fmax(1e-12, -rtol_arg * sqrt(est)) : 1e-10;
    }
    const int sp = (s + 15) & ~15;
    const int a = threadIdx.x;
    const bool act = a < s;
    double* G = kLdsGram ? Gl : gram + P.goff[i];
    const int nt = sp >> 4;
    const int npairs = nt * (nt + 1) / 2;
    // the warm start's rows load while the Gram is assembled
    double* Wi = W + P.woff[i];
    double qw[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) qw[p] = warm == 1 ? Wi[(act ? a : 0) * RP + p] : 0.0;
    // the stop flag, loaded by thread 0 now (its round trip overlaps the
    // Gram assembly, whose reads stay inside this shape's partials either
    // way) and shared through LDS afterwards, so that the whole workgroup
    // takes the same branch: a sibling mode's workgroup of this launch may
    // raise the flag meanwhile
    const int sf0 = threadIdx.x == 0 ? stop_flag(st) : 0;
    {
        // the Gram from k_gram's per-chunk 16 x 16 tiles, chunks added in
        // order; every load of a thread is issued before the first use
        const int nkc = P.gnkc[i];
        const int total = npairs * 256;
        const double* src0 = gpart + (int64_t)P.gitem0[i] * 256;
        // chunk counts up to 4 or 8 (and 16 at RP = 16): pairs of entries,
        // every chunk's load of a round in flight at once; more: rounds of
        // 16 chunks, added in chunk order.  (Wider rounds at RP <= 8 raise
        // the whole kernel's register count and measured slower.)
        if (nkc <= 4) {
            gram_assemble2<12, 4>(src0, total, nkc, G);
        } else if (nkc <= 8) {
            gram_assemble2<6, 8>(src0, total, nkc, G);
        } else if (RP == 16 && nkc <= 16) {
            gram_assemble2<3, 16>(src0, total, nkc, G);
        } else {
            gram_assemble<4, 16, true>(src0, total, nkc, G);
        }
    }
    // Q and Z rows s..sp-1 stay zero for the padded products (written after
    // the assembly's loads were issued; the barrier below orders both)
    for (int e = s * RP + threadIdx.x; e < sp * RP; e += kThreads) {
        sh.qs[e] = 0.0;
        sh.zs[e] = 0.0;
    }
    if (threadIdx.x == 0) {
        sh.stopf = sf0;
        sh.ok = 1;
    }
    __syncthreads();
    if (sh.stopf) return;  // uniform: one value for the whole workgroup
    double q[RP], z[RP];
    if (warm == 1) {
#pragma unroll
        for (int p = 0; p < RP; ++p) q[p] = (act && p < r) ? qw[p] : 0.0;
    } else {
        // start block G * Omega, then Cholesky-QR twice.  Omega: with
        // warm == 2 (a new sample under RTCUR-R) the previous mode-i factor's
        // rows at the new I_i, which span nearly the wanted subspace; else,
        // or if that block loses rank, a fixed pseudo-random block (a second
        // one if G * Omega still loses rank; only a Gram of rank below r
        // fails both)
        bool ok = false;
        for (int att = warm == 2 ? 0 : 1; att < 3 && !ok; ++att) {
            __syncthreads();
            for (int e = threadIdx.x; e < s * RP; e += kThreads) {
                const int b = e / RP, p = e % RP;
                const double v = att == 0 ? Bd[P.boff[i] + (int64_t)P.I[i][b] * RP + p]
                                          : eig_start(b, p, att);
                sh.qs[rsw<RP>(b, p)] = p < r ? v : 0.0;
            }
            __syncthreads();
            eig_gq<RP>(G, sp, s, sh);
#pragma unroll
            for (int p = 0; p < RP; ++p) z[p] = act ? sh.zs[rsw<RP>(a, p)] : 0.0;
            ok = true;
            for (int rep = 0; rep < 2 && ok; ++rep) {
                eig_tm<RP>(sp, false, sh);  // M = Z^T Z
                EigChol<RP> ch;
                ok = ch.factor(sh.mm, r, sh);
                if (ok) {
                    ch.solve(z, q, sh);
#pragma unroll
                    for (int p = 0; p < RP; ++p) z[p] = q[p];
                    if (rep == 0 && act) {
#pragma unroll
                        for (int p = 0; p < RP; ++p) sh.zs[rsw<RP>(a, p)] = z[p];
                    }
                    __syncthreads();
                }
            }
        }
        if (!ok) {
            if (threadIdx.x == 0) {
                st->stop = 1;
                st->status = RTCUR_E_RANK;
            }
            return;
        }
    }
    // RP = 16: the iterate's rows stay in sh.qs (and Z's in sh.zs) from here
    // on instead of in registers, which would not hold them beside the rest
    constexpr bool kRowsLds = RP > 8;
    if constexpr (kRowsLds) {
        __syncthreads();
        if (act) {
#pragma unroll
            for (int p = 0; p < RP; ++p) sh.qs[rsw<RP>(a, p)] = q[p];
        }
    }
    int steps = 0;
    const int m = s < RP ? s : RP;  // columns available to the guarded iteration
    // Plain subspace iteration on r columns for at most `limit` steps:
    // 0 = converged, 1 = limit reached, 2 = too slow (the contraction per
    // step predicts more than 30 further steps; only with allow_guard),
    // 3 = Cholesky breakdown (sh.ok cleared).  Every branch is uniform: rn
    // and tn come out of a block-wide sum.
    auto plain = [&](int limit, bool allow_guard) -> int {
        double prev = 0.0;
        for (int it = 0;; ++it, ++steps) {
            __syncthreads();
            if (act) {
#pragma unroll
                for (int p = 0; p < RP; ++p) sh.qs[rsw<RP>(a, p)] = q[p];
            }
            __syncthreads();
            eig_gq_tm<RP>(G, sp, s, sh);  // Z = G Q, T = Q^T Z, M = Z^T Z
#pragma unroll
            for (int p = 0; p < RP; ++p) z[p] = act ? sh.zs[rsw<RP>(a, p)] : 0.0;
            // (RP <= 8 only: RP = 16 runs plain_lds) T in registers
            double rn = 0.0, tn = 0.0;
            double Tr[RP][RP];
#pragma unroll
            for (int k = 0; k < RP; ++k)
#pragma unroll
                for (int p = 0; p < RP; ++p) {
                    Tr[k][p] = sh.tm[k * RP + p];
                    tn += Tr[k][p] * Tr[k][p];
                }
#pragma unroll
            for (int p = 0; p < RP; ++p) {
                double v = z[p];
#pragma unroll
                for (int k = 0; k < RP; ++k) v -= q[k] * Tr[k][p];
                rn += act ? v * v : 0.0;
            }
            rn = block_sum<4>(rn, sh.red);
            if (rn <= rtol * rtol * tn) return 0;
            if (it >= limit) return 1;
            if (allow_guard && m > r && it >= 4 && prev > 0.0) {
                // more than 30 further steps at this contraction rho = rn / prev:
                // rtol^2 tn / rn < rho^30 (a tiny rho underflows to 0: fast)
                const double r2 = (rn / prev) * (rn / prev), r4 = r2 * r2, r8 = r4 * r4;
                const double r30 = r8 * r8 * r8 * r4 * r2;
                if (rn >= prev || rtol * rtol * tn < r30 * rn) return 2;
            }
            prev = rn;
            EigChol<RP> ch;
            if (!ch.factor(sh.mm, r, sh)) {
                if (threadIdx.x == 0) sh.ok = 0;
                return 3;
            }
            ch.solve(z, q, sh);
        }
    };
    // As plain, with the rows of Q (and Z) kept in LDS between steps (read
    // into registers within a step): q_a = Z_a R^-1 goes back to the thread's
    // row of sh.qs.
    auto plain_lds = [&](int limit, bool allow_guard) -> int {
        double prev = 0.0;
        for (int it = 0;; ++it, ++steps) {
            __syncthreads();
            eig_gq_tm<RP>(G, sp, s, sh);  // Z = G Q, T = Q^T Z, M = Z^T Z
            // the thread's rows of Q and Z in registers for this step only
            // (every row index below kMaxS is in range; the inactive rows'
            // terms are dropped); T read from LDS one column at a time
            double qr[RP], zr[RP];
#pragma unroll
            for (int k = 0; k < RP; ++k) {
                qr[k] = sh.qs[rsw<RP>(a, k)];
                zr[k] = sh.zs[rsw<RP>(a, k)];
            }
            // ||T||_F^2: four entries per lane and a wave sum, the same in
            // every wave
            double tn = 0.0;
#pragma unroll
            for (int u = 0; u < RP * RP / 64; ++u) {
                const double t = sh.tm[(threadIdx.x & 63) + 64 * u];
                tn += t * t;
            }
            tn = wave_sum(tn);
            // the row's residual z - q T, one row of T at a time (RP
            // independent sums; the next row's loads issued before this
            // row's products, two rows in flight at most)
            double v[RP], tr[2][RP];
#pragma unroll
            for (int p = 0; p < RP; ++p) {
                v[p] = zr[p];
                tr[0][p] = sh.tm[p];
            }
#pragma unroll
            for (int k = 0; k < RP; ++k) {
                if (k + 1 < RP) {
#pragma unroll
                    for (int p = 0; p < RP; ++p) tr[(k + 1) & 1][p] = sh.tm[(k + 1) * RP + p];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int p = 0; p < RP; ++p) v[p] -= qr[k] * tr[k & 1][p];
            }
            double rn = 0.0;
#pragma unroll
            for (int p = 0; p < RP; ++p) rn += v[p] * v[p];
            rn = block_sum<4>(act ? rn : 0.0, sh.red);
            if (rn <= rtol * rtol * tn) return 0;
            if (it >= limit) return 1;
            if (allow_guard && m > r && it >= 4 && prev > 0.0) {
                const double r2 = (rn / prev) * (rn / prev), r4 = r2 * r2, r8 = r4 * r4;
                const double r30 = r8 * r8 * r8 * r4 * r2;
                if (rn >= prev || rtol * rtol * tn < r30 * rn) return 2;
            }
            prev = rn;
            EigChol<RP> ch;
            if (!ch.factor(sh.mm, r, sh)) {
                if (threadIdx.x == 0) sh.ok = 0;
                return 3;
            }
            ch.solve(zr, qr, sh);
            if (act) {
#pragma unroll
                for (int p = 0; p < RP; ++p) sh.qs[rsw<RP>(a, p)] = qr[p];
            }
        }
    };
    int pr;
    if constexpr (kRowsLds) pr = plain_lds(maxit, true);
    else pr = plain(maxit, true);
    if (pr == 2) {
        __syncthreads();
        if constexpr (!kRowsLds) {
            if (act) {
#pragma unroll
                for (int p = 0; p < RP; ++p) sh.qs[rsw<RP>(a, p)] = q[p];
            }
        }
        if (threadIdx.x == 0) sh.gsteps = 0;
        __syncthreads();
        const int g = eig_guarded<RP>(G, sp, s, r, m, rtol, &sh, &sh.gsteps);
        if constexpr (!kRowsLds) {
#pragma unroll
            for (int p = 0; p < RP; ++p) q[p] = act ? sh.qs[rsw<RP>(a, p)] : 0.0;
        }
        steps += sh.gsteps;
        // a few plain steps from the Ritz vectors (or, after a breakdown of
        // the guarded iterate, the plain iterate) polish the basis and form
        // the T used below
        if constexpr (kRowsLds) pr = plain_lds(g >= 0 ? 8 : maxit, false);
        else pr = plain(g >= 0 ? 8 : maxit, false);
    }
    const bool conv = pr == 0;
    __syncthreads();
    if (!sh.ok) {
        if (threadIdx.x == 0) {
            st->stop = 1;
            st->status = RTCUR_E_RANK;
        }
        return;
    }
    // Q spans the top-r eigenspace and T = Q^T G Q, so the truncated
    // pseudo-inverse of the Gram is Q T^-1 Q^T: W_i = Q, Y_i = Q T^-1 with
    // T = R^T R (Cholesky of the symmetrised T, every thread).
    __syncthreads();
    if (threadIdx.x < RP * RP) {
        const int p = threadIdx.x / RP, t = threadIdx.x % RP;
        sh.mm[threadIdx.x] = 0.5 * (sh.tm[p * RP + t] + sh.tm[t * RP + p]);
    }
    __syncthreads();
    if constexpr (RP <= 8) {
        eig_finish_regs<RP>(P, i, s, r, a, act, q, conv, steps, Wi, Y, st, sh);
    } else {
        eig_finish_lds<RP>(P, i, s, r, a, act, conv, steps, Wi, Y, st, sh);
    }
}

// --------------------------- Z_i = Y_i^T U_i  and the core's first phase
// Workgroups [0, s_0 cparts): T[a] = R(a, :, ..) x_{l >= 1} W_l^T (or a
// part of its middle-mode rows), the core G = R x_i W_i^T before its last
// contraction (with W_0, finished beside the B-factor items).
// Workgroups [s_0 cparts, s_0 cparts + nz): Z_i (m_i x r_i, float64, row per
// column) with U_i = C_i(I_i, :), so that V_i S_i^-1 = Z_i; 64 columns per
// workgroup, one per lane, each wave summing a quarter of the s_i rows.
template <typename T, int RP>
__device__ void zmat_tile(const Prob& P, const T* __restrict__ C, const double* __restrict__ Y,
                          double* __restrict__ Zbuf, int2 tl, double* ys, double* red, int sf) {
    const int i = tl.x;
    const BlockDev& bd = P.blk[1 + i];
    const int s = P.s[i], m = bd.ncols;
    const double* Yi = Y + P.woff[i];
    for (int e = threadIdx.x; e < s * RP; e += kThreads) ys[e] = Yi[e];
    if (sf) return;
    __syncthreads();
    // lane = column (64 per workgroup: each row's loads are one coalesced
    // 64-column segment per wave), wave = a quarter of the rows of U_i (its
    // row index is uniform: a scalar load); the four waves' partial sums are
    // added in wave order through LDS
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (wave-uniform)
    const int c = tl.y + lane;
    const int cc = c < m ? c : m - 1;
    const int qlen = (s + 3) / 4;
    const int a0 = w * qlen, a1 = min(s, a0 + qlen);
    const int32_t* Ii = P.I[i];
    const T* base = C + bd.off + cc;
    double acc[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) acc[p] = 0.0;
    constexpr int U = 16;
    for (int b0 = a0; b0 < a1; b0 += U) {
        T u[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int a = b0 + q < a1 ? b0 + q : a0;  // (masked below)
            u[q] = base[(int64_t)Ii[a] * m];
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (b0 + q < a1) {  // uniform
                const double uv = (double)u[q];
#pragma unroll
                for (int p = 0; p < RP; ++p) acc[p] = fma(uv, ys[(b0 + q) * RP + p], acc[p]);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < RP; ++p) red[(w * RP + p) * 64 + lane] = acc[p];
    __syncthreads();
    // Z_i is stored compactly, r_i doubles per column (the padded columns
    // p >= r_i of Y_i are zero); consecutive threads write consecutive words
    const int r = P.r[i];
    for (int e = threadIdx.x; e < 64 * r; e += kThreads) {
        const int col = e / r, p = e - col * r;
        const double z = ((red[p * 64 + col] + red[(RP + p) * 64 + col]) +
                          red[(2 * RP + p) * 64 + col]) + red[(3 * RP + p) * 64 + col];
        if (tl.y + col < m) Zbuf[P.zoff[i] + (int64_t)(tl.y + col) * r + p] = z;
    }
}

// sum_k x[k * xs] * y[k * ys] over LDS operands, in a fixed order: loads
// issued eight terms at a time, alternate terms into two accumulators.
template <typename TX>
__device__ __forceinline__ double lds_dot(const TX* x, int xs, const double* y, int ys, int K) {
    double acc[2] = {0.0, 0.0};
    for (int k = 0; k < K; k += 8) {
        double xv[8], yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int kk = k + u < K ? k + u : K - 1;
            xv[u] = (double)x[kk * xs];
            yv[u] = y[kk * ys];
            xv[u] = k + u < K ? xv[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u & 1] = fma(xv[u], yv[u], acc[u & 1]);
    }
    return acc[0] + acc[1];
}

constexpr int kCoreLds = 4096;  // doubles of LDS for one slice's partial core
constexpr int kSliceBytes = 16384;  // bytes of R staged per pass (in buf's second half)
// three-mode slices of more than kCoreLds / 2 entries (r_2 s_1 <= 4096): a
// second kernel instance with the partial core in the first 4096 doubles and
// the staging behind them
constexpr int kCoreSliceBig = 4096;
constexpr int kCoreLdsBig = kCoreSliceBig + kSliceBytes / 8;

// T[a] for one slice a of the R block (row-major s_0 x ... x s_{n-1}):
// contract the last mode (R staged through LDS), then the others in LDS;
// each step puts the new rank index first, so T[a] ends up ordered
// (r_1, .., r_{n-1}).  buf: the partial core in [0, half), the staged rows
// (rs) and the next contraction's output from buf + half.
template <typename T, int RP>
__device__ void core_slice(const Prob& P, const T* __restrict__ R, const double* __restrict__ W,
                           double* __restrict__ Tbuf, int a, double* buf, double* ws, T* rs,
                           int sf, int half) {
    const int n = P.n;
    const int tid = threadIdx.x;
    int rows = 1;
    for (int l = 1; l < n - 1; ++l) rows *= P.s[l];
    const int K = P.s[n - 1];
    const int rq = P.r[n - 1];
    // this item's rows [rb, re) of the slice (the whole slice unless the
    // middle mode is split into P.cparts parts; the parts' partial cores
    // are added by core_finish)
    const int part = a % P.cparts;
    a /= P.cparts;
    const int rb = part * P.crows, re = min(rows, rb + P.crows);
    const T* Ra = R + (int64_t)a * rows * K;
    const int RC = max(1, kSliceBytes / (int)sizeof(T) / K);
    // every load of the first pass (its R rows and W_{n-1}) and of the next
    // mode's W rows is issued before the first store
    constexpr int NV = kSliceBytes / (int)sizeof(T) / kThreads;  // R entries per thread
    constexpr int NW = kMaxS * RP / kThreads;                   // W entries per thread
    const int nr0 = min(RC, re - rb), ne0 = nr0 * K;
    T v0[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const int e = tid + u * kThreads;
        v0[u] = Ra[(int64_t)rb * K + (e < ne0 ? e : 0)];
    }
    double w0[NW], w1[NW];
    const int l1 = n - 2;  // the next mode contracted (none when n == 2)
#pragma unroll
    for (int u = 0; u < NW; ++u) {
        const int e = tid + u * kThreads;
        w0[u] = W[P.woff[n - 1] + (e < K * RP ? e : 0)];
        w1[u] = l1 >= 1 ? W[P.woff[l1 >= 1 ? l1 : 0] + (e < P.s[l1 >= 1 ? l1 : 0] * RP ? e : 0)]
                        : 0.0;
    }
    if (sf) return;
#pragma unroll
    for (int u = 0; u < NW; ++u) {
        const int e = tid + u * kThreads;
        if (e < K * RP) ws[e] = w0[u];
    }
    if (P.cparts > 1) {
        for (int o = tid; o < rq * rows; o += kThreads) {
            const int row = o % rows;
            if (row < rb || row >= re) buf[o] = 0.0;
        }
    }
    for (int r0 = rb; r0 < re; r0 += RC) {
        const int nr = min(RC, re - r0);
        const int ne = nr * K;
        __syncthreads();
        if (r0 == rb) {
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                const int e = tid + u * kThreads;
                if (e < ne) rs[e] = v0[u];
            }
        } else {
            for (int e0 = tid; e0 < ne; e0 += 8 * kThreads) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * kThreads;
                    v[u] = Ra[(int64_t)r0 * K + (e < ne ? e : e0)];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * kThreads;
                    if (e < ne) rs[e] = v[u];
                }
            }
        }
        __syncthreads();
        for (int o = tid; o < rq * nr; o += kThreads) {
            const int p = o / nr, row = o % nr;
            buf[p * rows + r0 + row] = lds_dot<T>(rs + row * K, 1, ws + p, RP, K);
        }
    }
    __syncthreads();
    // remaining modes n-2 .. 1 in LDS: [lead][rest][K'] -> [r'][lead][rest]
    int lead = rq;
    int rest = rows;
    double* cur = buf;
    double* nxt = buf + half;
    for (int l = n - 2; l >= 1; --l) {
        const int Kl = P.s[l], rl = P.r[l];
        rest /= Kl;
        const int M = lead * rest;
        __syncthreads();
        if (l == l1) {
#pragma unroll
            for (int u = 0; u < NW; ++u) {
                const int e = tid + u * kThreads;
                if (e < Kl * RP) ws[e] = w1[u];
            }
        } else {
            for (int e = tid; e < Kl * RP; e += kThreads) ws[e] = W[P.woff[l] + e];
        }
        __syncthreads();
        for (int o = tid; o < rl * M; o += kThreads) {
            const int p = o / M, row = o % M;
            nxt[o] = lds_dot<double>(cur + row * Kl, 1, ws + p, RP, Kl);
        }
        __syncthreads();
        double* t = cur;
        cur = nxt;
        nxt = t;
        lead *= rl;
    }
    int tot = 1;
    for (int l = 1; l < n; ++l) tot *= P.r[l];
    for (int e = tid; e < tot; e += kThreads)
        Tbuf[((int64_t)a * P.cparts + part) * tot + e] = cur[e];
}

// G = sum_a W_0[a]^T T[a] (the last contraction of the core, the parts of
// each slice added in order with it), one workgroup, T and W_0 rows staged
// through the caller's LDS buffer of `cap` doubles.
template <int RP>
__device__ void core_finish(const Prob& P, const double* __restrict__ W,
                            const double* __restrict__ Tbuf, double* __restrict__ Gd,
                            double* buf, int cap) {
    const int s0 = P.s[0] * P.cparts, r0 = P.r[0];  // slices: (a, part), part fastest
    const int tot = P.core / r0;
    // as many slices per round as the LDS buffer holds (all of them when
    // possible), their T rows and W_0 rows staged together
    const int A = max(1, min(s0, cap / (tot + RP)));
    double* tb = buf;
    double* wb = buf + A * tot;
    // G groups of threads split the slices of a round; the groups' partial
    // sums are added in group order
    const int G = P.core <= kThreads ? max(1, min(8, kThreads / P.core)) : 1;
    const int g = threadIdx.x / P.core;
    constexpr int JM = kMaxCore / kThreads;
    double acc[JM];
#pragma unroll
    for (int j = 0; j < JM; ++j) acc[j] = 0.0;
    for (int a0 = 0; a0 < s0; a0 += A) {
        const int na = min(A, s0 - a0);
        __syncthreads();
        for (int e = threadIdx.x; e < na * tot; e += kThreads)
            tb[e] = Tbuf[(int64_t)a0 * tot + e];
        for (int e = threadIdx.x; e < na * RP; e += kThreads)
            wb[e] = W[P.woff[0] + (int64_t)((a0 + e / RP) / P.cparts) * RP + e % RP];
        __syncthreads();
        if (G > 1) {
            if (g < G) {
                const int o = threadIdx.x - g * P.core;
                const int p = o / tot, rest = o % tot;
                const int k0 = g * na / G, k1 = (g + 1) * na / G;
                acc[0] += lds_dot<double>(wb + k0 * RP + p, RP, tb + k0 * tot + rest, tot, k1 - k0);
            }
        } else {
#pragma unroll
            for (int j = 0; j < JM; ++j) {
                const int o = threadIdx.x + j * kThreads;
                if (o < P.core) {
                    const int p = o / tot, rest = o % tot;
                    acc[j] += lds_dot<double>(wb + p, RP, tb + rest, tot, na);
                }
            }
        }
    }
    if (G > 1) {
        __syncthreads();
        if (g < G) buf[threadIdx.x] = acc[0];
        __syncthreads();
        if (threadIdx.x < P.core) {
            double v = 0.0;
            for (int q = 0; q < G; ++q) v += buf[q * P.core + threadIdx.x];
            Gd[threadIdx.x] = v;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < JM; ++j) {
        const int o = threadIdx.x + j * kThreads;
        if (o < P.core) Gd[o] = acc[j];
    }
}

// kBig: three modes with r_2 s_1 > kCoreLds / 2 (the larger buffer).
template <typename T, int RP, bool kBig>
__global__ __launch_bounds__(kThreads) void k_zcore(Prob P, const T* __restrict__ C,
                                                    const double* __restrict__ Y,
                                                    double* __restrict__ Zbuf,
                                                    const int2* __restrict__ ztiles, int nz,
                                                    const double* __restrict__ W,
                                                    double* __restrict__ Tbuf,
                                                    const DevState* st) {
    const int sf = stop_flag(st);
    constexpr int NB = kBig ? kCoreLdsBig : kCoreLds;
    constexpr int HALF = kBig ? kCoreSliceBig : kCoreLds / 2;
    __shared__ double sh[kMaxS * RP];
    __shared__ double buf[NB];
    // the slice's staged rows share buf's second part (free until the
    // contraction of the middle modes)
    static_assert(kSliceBytes <= (int)sizeof(double) * (NB - HALF), "staging fits");
    static_assert(NB >= 4 * 16 * 64, "zmat_tile's wave partials fit");
    T* rs = reinterpret_cast<T*>(buf + HALF);
    // the core slices (the longer workgroups) first, so that they are
    // dispatched first and the Z tiles fill the CUs around them
    const int ncore = P.s[0] * P.cparts;
    if ((int)blockIdx.x < ncore) {
        core_slice<T, RP>(P, C + P.blk[0].off, W, Tbuf, (int)blockIdx.x, buf, sh, rs, sf, HALF);
        return;
    }
    const int zt = (int)blockIdx.x - ncore;  // < nz: the grid is nz + ncore
    if (zt < nz) zmat_tile<T, RP>(P, C, Y, Zbuf, ztiles[zt], sh, buf, sf);
}

// -------------------------------------------------------- B_i = C_i Z_i
// B_i (d_i x RP) = C_i V_i S_i^-1 = C_i Z_i.  Work item = (mode, 16 rows,
// 1024 columns): Z_i's chunk is staged in LDS, each wave owns 4 rows and its
// lanes stride the columns; k_bred adds the chunks' partial rows in order.
// One extra workgroup finishes the core G from the slices of k_zcore.
constexpr int kBfacKC = 1024;
constexpr int kBfacMaxKC = 64;  // column chunks (partial rows) per entry at most
// columns per B-factor work item (its Z chunk in LDS: KC x RP doubles)
constexpr int bfac_kc(int rp) { return rp <= 8 ? kBfacKC : kBfacKC / 2; }

// Entry (c, p) of a B-factor work item's staged Z chunk (column c of the
// chunk, RP doubles each) in LDS: p XOR bits of c above the columns that
// share one 256-byte bank row, so that the lanes of a wave, on consecutive
// columns and reading the same p, fall on distinct banks.
template <int RP>
__device__ __forceinline__ int zsw(int c, int p) {
    constexpr int sh = RP == 4 ? 3 : (RP == 8 ? 2 : 1);
    return c * RP + (p ^ ((c >> sh) & (RP - 1)));
}

// kSub: some mode stages several Z sub-chunks per work item (P.bsub > 1).
template <typename T, int RP, bool kSub>
__global__ __launch_bounds__(kThreads) void k_bfac(Prob P, const T* __restrict__ C,
                                                   const double* __restrict__ Zbuf,
                                                   const int4* __restrict__ items, int nitems,
                                                   double* __restrict__ bpart,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ Tbuf,
                                                   double* __restrict__ Gd, const DevState* st) {
    const int sf = stop_flag(st);
    constexpr int KC = bfac_kc(RP);
    static_assert(KC * RP >= kCoreLds, "core_finish staging fits in zs");
    __shared__ double zs[KC * RP];
    if (blockIdx.x == 0) {
        // the core G = sum_a W_0[a]^T T[a] from k_zcore's slices, beside the
        // B-factor items: workgroup 0, so that it is dispatched first (it is
        // the longest single workgroup) and overlaps the items
        if (sf) return;
        core_finish<RP>(P, W, Tbuf, Gd, zs, KC * RP);
        return;
    }
    const int item = (int)blockIdx.x - 1;  // the grid is nitems + 1
    if (item >= nitems) return;
    const int4 it = items[item];
    const int i = it.x, rb = it.y, kc = it.z;
    const BlockDev& bd = P.blk[1 + i];
    const int m = bd.ncols, d = bd.nrows;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double acc[kBfacRowsPerWave][RP];
    if constexpr (!kSub) {
        const int c0 = kc * KC, cn = min(KC, m - c0);
        const int r = P.r[i];
        const double* Zc = Zbuf + P.zoff[i] + (int64_t)c0 * r;
        const int xb = rb * kBfacRows + w * kBfacRowsPerWave;
        const T* rowp[kBfacRowsPerWave];
#pragma unroll
        for (int j = 0; j < kBfacRowsPerWave; ++j)
            rowp[j] = C + bd.off + (int64_t)(xb + j < d ? xb + j : d - 1) * m + c0;
        constexpr int U = 8;
        auto load_c = [&](T (&cv)[kBfacRowsPerWave][U], int u0) {
#pragma unroll
            for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = lane + 64 * (u0 + u);
                    cv[j][u] = rowp[j][c < cn ? c : 0];
                }
        };
        // the first batch of C is in flight while the Z chunk is staged
        T cv[kBfacRowsPerWave][U];
        load_c(cv, 0);
        {
            // Z chunk -> LDS: every load of a thread issued before the stores
            // (Z_i holds r doubles per column; the padding p >= r is staged as
            // zero, its lanes loading a word the others fetch anyway)
            constexpr int ZE = KC * RP / kThreads;
            double zv[ZE];
#pragma unroll
            for (int q = 0; q < ZE; ++q) {
                const int e = tid + q * kThreads, c = e / RP, p = e % RP;
                zv[q] = Zc[(e < cn * RP && p < r) ? c * r + p : 0];
            }
#pragma unroll
            for (int q = 0; q < ZE; ++q) {
                const int e = tid + q * kThreads, c = e / RP, p = e % RP;
                zs[zsw<RP>(c, p)] = (e < cn * RP && p < r) ? zv[q] : 0.0;
            }
        }
        if (sf) return;
#pragma unroll
        for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
            for (int p = 0; p < RP; ++p) acc[j][p] = 0.0;
        __syncthreads();
        for (int u0 = 0; u0 < KC / 64; u0 += U) {
            T cn_[kBfacRowsPerWave][U];
            if (u0 + U < KC / 64) load_c(cn_, u0 + U);  // next batch in flight
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = lane + 64 * (u0 + u);
                if (c < cn) {
                    double z[RP];
#pragma unroll
                    for (int p = 0; p < RP; ++p) z[p] = zs[zsw<RP>(c, p)];
#pragma unroll
                    for (int j = 0; j < kBfacRowsPerWave; ++j) {
                        const double x = (double)cv[j][u];
#pragma unroll
                        for (int p = 0; p < RP; ++p) acc[j][p] = fma(x, z[p], acc[j][p]);
                    }
                }
            }
            if (u0 + U < KC / 64) {
#pragma unroll
                for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
                    for (int u = 0; u < U; ++u) cv[j][u] = cn_[j][u];
            }
        }
    } else {
        const int xb = rb * kBfacRows + w * kBfacRowsPerWave;
        const int nsub = P.bsub[i];
        for (int sc = 0; sc < nsub; ++sc) {
            const int c0 = (kc * nsub + sc) * KC;
            if (c0 >= m) break;  // uniform
            const int cn = min(KC, m - c0);
            const int r = P.r[i];
            const double* Zc = Zbuf + P.zoff[i] + (int64_t)c0 * r;
            const T* rowp[kBfacRowsPerWave];
#pragma unroll
            for (int j = 0; j < kBfacRowsPerWave; ++j)
                rowp[j] = C + bd.off + (int64_t)(xb + j < d ? xb + j : d - 1) * m + c0;
            constexpr int U = 8;
            auto load_c = [&](T (&cv)[kBfacRowsPerWave][U], int u0) {
#pragma unroll
                for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int c = lane + 64 * (u0 + u);
                        cv[j][u] = rowp[j][c < cn ? c : 0];
                    }
            };
            // the first batch of C is in flight while the Z chunk is staged
            T cv[kBfacRowsPerWave][U];
            load_c(cv, 0);
            {
                // Z chunk -> LDS: every load of a thread issued before the stores
                // (Z_i holds r doubles per column; the padding p >= r is staged as
                // zero, its lanes loading a word the others fetch anyway)
                constexpr int ZE = KC * RP / kThreads;
                double zv[ZE];
#pragma unroll
                for (int q = 0; q < ZE; ++q) {
                    const int e = tid + q * kThreads, c = e / RP, p = e % RP;
                    zv[q] = Zc[(e < cn * RP && p < r) ? c * r + p : 0];
                }
#pragma unroll
                for (int q = 0; q < ZE; ++q) {
                    const int e = tid + q * kThreads, c = e / RP, p = e % RP;
                    zs[zsw<RP>(c, p)] = (e < cn * RP && p < r) ? zv[q] : 0.0;
                }
            }
            if (sf) return;
            if (sc == 0) {
                // zeroed after the first staging: one sub-chunk keeps the
                // accumulators out of the staging's registers
#pragma unroll
                for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
                    for (int p = 0; p < RP; ++p) acc[j][p] = 0.0;
            }
            __syncthreads();
            for (int u0 = 0; u0 < KC / 64; u0 += U) {
                T cn_[kBfacRowsPerWave][U];
                if (u0 + U < KC / 64) load_c(cn_, u0 + U);  // next batch in flight
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = lane + 64 * (u0 + u);
                    if (c < cn) {
                        double z[RP];
#pragma unroll
                        for (int p = 0; p < RP; ++p) z[p] = zs[zsw<RP>(c, p)];
#pragma unroll
                        for (int j = 0; j < kBfacRowsPerWave; ++j) {
                            const double x = (double)cv[j][u];
#pragma unroll
                            for (int p = 0; p < RP; ++p) acc[j][p] = fma(x, z[p], acc[j][p]);
                        }
                    }
                }
                if (u0 + U < KC / 64) {
#pragma unroll
                    for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
                        for (int u = 0; u < U; ++u) cv[j][u] = cn_[j][u];
                }
            }
            __syncthreads();  // the next sub-chunk overwrites zs
        }
    }
#pragma unroll
    for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
        for (int p = 0; p < RP; ++p) acc[j][p] = wave_sum(acc[j][p]);
    double* out = bpart + ((int64_t)item * kBfacRows + w * kBfacRowsPerWave) * RP;
    if (lane < RP) {
#pragma unroll
        for (int j = 0; j < kBfacRowsPerWave; ++j) {
            double v = 0.0;
#pragma unroll
            for (int p = 0; p < RP; ++p)
                if (p == lane) v = acc[j][p];
            out[j * RP + lane] = v;
        }
    }
}

// B_i rows: the column-chunk partials of k_bfac added in chunk order (one
// thread per entry).
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_bred(Prob P, const double* __restrict__ bpart,
                                                   const int4* __restrict__ items,
                                                   T* __restrict__ Bf, double* __restrict__ Bd,
                                                   const DevState* st) {
    const int sf = stop_flag(st);
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    int i = 0;
    int64_t base = 0;
    while (i < P.n - 1 && e >= base + (int64_t)P.d[i] * RP) {
        base += (int64_t)P.d[i] * RP;
        ++i;
    }
    if (e >= base + (int64_t)P.d[i] * RP) return;
    const int x = (int)((e - base) / RP), p = (int)((e - base) % RP);
    const int rb = x / kBfacRows, xr = x % kBfacRows;
    const int nkc = P.bnkc[i];
    const double* src = bpart + ((int64_t)(P.bitem0[i] + rb * nkc) * kBfacRows + xr) * RP + p;
    double sum = 0.0;
    for (int q0 = 0; q0 < nkc; q0 += 16) {  // 16 loads in flight, added in order
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q] = src[(int64_t)(q0 + q < nkc ? q0 + q : q0) * kBfacRows * RP];
        if (sf) return;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (q0 + q < nkc) sum += v[q];
    }
    Bf[P.boff[i] + (int64_t)x * RP + p] = (T)sum;
    Bd[P.boff[i] + (int64_t)x * RP + p] = sum;
}

// ------------------------------------------------ H_b = G x_{j != mode} B_j
// For every column of a block (or, with a negative block id, every column of
// the full mode-`dense_mode` unfolding), H[p][c] = sum over the other modes'
// core indices of G[..p..] * prod_j B_j[idx_j(c)][q_j].  G sits in LDS
// permuted so that the block's own mode comes first (at the true ranks).
// k_hexp contracts per column with each thread's B rows in LDS, so the loops
// run to the true ranks.  k_hexp_fac serves three or more modes with columns
// that come in runs sharing every other-mode index but the last (R, chidori
// blocks, the dense unfolding) and a long per-column contraction: per run,
// T[p][z] = sum over the leading other-mode core indices of G[..p..z] *
// prod B (in LDS), then per column H[p][c] = sum_z T[p][z] B_last[idx_last(c)][z].
constexpr int kHexpFactorMin = 256;  // prod r_i above which k_hexp_fac is used

template <typename T, int RP, int N>
__global__ __launch_bounds__(kThreads) void k_hexp_fac(
    Prob P, const int2* __restrict__ tiles, const T* __restrict__ Bf,
    const double* __restrict__ Gd, T* __restrict__ H, const DevState* st,
    int dense_mode, int64_t dense_cols) {
    const int sf = st ? stop_flag(st) : 0;
    constexpr int GPAD = N == 2 ? RP * RP : (N == 3 ? RP * RP * RP : RP * RP * RP * RP);
    constexpr int GP = GPAD < kMaxCore ? GPAD : kMaxCore;
    __shared__ double gp[GP];
    __shared__ double vs[RP * (kThreads + 2 * RP)];  // the runs' T
    const int2 tl = tiles[blockIdx.x];
    const bool dense = tl.x < 0;
    const int mode = dense ? dense_mode : P.blk[tl.x].mode;
    const int64_t ncols = dense ? dense_cols : P.blk[tl.x].ncols;
    int others[kMaxModes - 1] = {0, 0, 0};
    int no = 0;
    for (int j = 0; j < N; ++j)
        if (j != mode) others[no++] = j;
    const int rm = P.r[mode];
    const int r0 = P.r[others[0]];
    const int r1 = N >= 3 ? P.r[others[1]] : 1;
    const int r2 = N >= 4 ? P.r[others[2]] : 1;
    // permuted core at the true ranks: gp[((p*r0 + q)*r1 + u)*r2 + z] = G[...]
    // with p at `mode` and q, u, z at the other modes in increasing order
    int gstr[kMaxModes];
    gstr[N - 1] = 1;
    for (int j = N - 2; j >= 0; --j) gstr[j] = gstr[j + 1] * P.r[j + 1];
    const int gcount = rm * r0 * r1 * r2;
    for (int e = threadIdx.x; e < gcount; e += kThreads) {
        int rem = e;
        const int z = rem % r2;
        rem /= r2;
        const int u = rem % r1;
        rem /= r1;
        const int q = rem % r0;
        const int p = rem / r0;
        int off = p * gstr[mode] + q * gstr[others[0]];
        if (N >= 3) off += u * gstr[others[1]];
        if (N >= 4) off += z * gstr[others[2]];
        gp[e] = Gd[off];
    }
    const int tid = threadIdx.x;
    const int64_t c = (int64_t)tl.y * kThreads + tid;
    const int64_t cc = c < ncols ? c : ncols - 1;
    const int plen = dense ? P.d[others[N - 2]] : P.blk[tl.x].plen;
    {
        if (sf) return;  // uniform
        const int rl = P.r[others[N - 2]];          // rank of the last other mode
        const int64_t c0 = (int64_t)tl.y * kThreads;
        const int64_t g0 = c0 / plen;
        const int64_t cl = (c0 + kThreads < ncols ? c0 + kThreads : ncols) - 1;
        const int npre = (int)(cl / plen - g0 + 1);
        double* Tb = vs;  // [npre][rm][rl]: at most RP (256 + 2 RP) doubles
        const int nt = npre * rm * rl;
        // the rows of the leading other modes at a column
        auto lead_rows = [&](int64_t col, int64_t (&ro)[kMaxModes - 1]) {
            if (dense) {
                int64_t rem = col / plen;
                for (int q = N - 3; q >= 0; --q) {
                    const int j = others[q];
                    ro[q] = P.boff[j] + (rem % P.d[j]) * RP;
                    rem /= P.d[j];
                }
            } else {
                const BlockDev& bd = P.blk[tl.x];
                for (int q = 0; q < N - 2; ++q)
                    ro[q] = P.boff[others[q]] + (int64_t)bd.cidx[(int64_t)q * ncols + col] * RP;
            }
        };
        __syncthreads();  // gp staged
        for (int e = tid; e < nt; e += kThreads) {
            const int z = e % rl;
            const int p = (e / rl) % rm;
            const int g = e / (rl * rm);
            int64_t ro[kMaxModes - 1] = {0, 0, 0};
            lead_rows((g0 + g) * plen, ro);
            double b0[RP], b1[RP];
#pragma unroll
            for (int k = 0; k < RP; ++k) {
                b0[k] = (double)Bf[ro[0] + k];
                b1[k] = N >= 4 ? (double)Bf[ro[1] + k] : 0.0;
            }
            double t = 0.0;
            if constexpr (N == 3) {
                // gp[(p*r0 + q)*r1 + z], z at the last other mode
#pragma unroll
                for (int q = 0; q < RP; ++q)
                    if (q < r0) t = fma(gp[(p * r0 + q) * r1 + z], b0[q], t);
            } else {
#pragma unroll
                for (int q = 0; q < RP; ++q) {
                    if (q < r0) {
                        double t1 = 0.0;
#pragma unroll
                        for (int u = 0; u < RP; ++u)
                            if (u < r1) t1 = fma(gp[((p * r0 + q) * r1 + u) * r2 + z], b1[u], t1);
                        t = fma(t1, b0[q], t);
                    }
                }
            }
            Tb[e] = t;
        }
        // this column's row of the last other mode
        int64_t rlast;
        if (dense) {
            rlast = P.boff[others[N - 2]] + (cc % plen) * RP;
        } else {
            const BlockDev& bd = P.blk[tl.x];
            rlast = P.boff[others[N - 2]] +
                    (int64_t)bd.cidx[(int64_t)(N - 2) * ncols + cc] * RP;
        }
        double bl[RP];
#pragma unroll
        for (int k = 0; k < RP; ++k) bl[k] = (double)Bf[rlast + k];
        __syncthreads();
        const double* Tg = Tb + (int)(cc / plen - g0) * rm * rl;
        const int64_t hoff = dense ? 0 : P.blk[tl.x].hoff;
        // a sampled block's H has the mode's r rows (the threshold pass reads
        // no more); the full-unfolding H of a reconstruction all RP
        const int prows = dense ? RP : rm;
        for (int p = 0; p < prows; ++p) {
            double a = 0.0;
            if (p < rm) {
#pragma unroll
                for (int z = 0; z < RP; ++z)
                    if (z < rl) a = fma(Tg[p * rl + z], bl[z], a);
            }
            if (c < ncols) H[hoff + (int64_t)p * ncols + c] = (T)a;
        }
        return;
    }
}

template <typename T, int RP, int N>
__global__ __launch_bounds__(kThreads) void k_hexp(
    Prob P, const int2* __restrict__ tiles, const T* __restrict__ Bf,
    const double* __restrict__ Gd, T* __restrict__ H, const DevState* st,
    int dense_mode, int64_t dense_cols) {
    const int sf = st ? stop_flag(st) : 0;
    constexpr int GPAD = N == 2 ? RP * RP : (N == 3 ? RP * RP * RP : RP * RP * RP * RP);
    constexpr int GP = GPAD < kMaxCore ? GPAD : kMaxCore;
    __shared__ double gp[GP];
    __shared__ double vs[(N - 1) * RP * kThreads];
    const int2 tl = tiles[blockIdx.x];
    const bool dense = tl.x < 0;
    const int mode = dense ? dense_mode : P.blk[tl.x].mode;
    const int64_t ncols = dense ? dense_cols : P.blk[tl.x].ncols;
    int others[kMaxModes - 1] = {0, 0, 0};
    int no = 0;
    for (int j = 0; j < N; ++j)
        if (j != mode) others[no++] = j;
    const int rm = P.r[mode];
    const int r0 = P.r[others[0]];
    const int r1 = N >= 3 ? P.r[others[1]] : 1;
    const int r2 = N >= 4 ? P.r[others[2]] : 1;
    // permuted core at the true ranks: gp[((p*r0 + q)*r1 + u)*r2 + z] = G[...]
    // with p at `mode` and q, u, z at the other modes in increasing order
    int gstr[kMaxModes];
    gstr[N - 1] = 1;
    for (int j = N - 2; j >= 0; --j) gstr[j] = gstr[j + 1] * P.r[j + 1];
    const int gcount = rm * r0 * r1 * r2;
    for (int e = threadIdx.x; e < gcount; e += kThreads) {
        int rem = e;
        const int z = rem % r2;
        rem /= r2;
        const int u = rem % r1;
        rem /= r1;
        const int q = rem % r0;
        const int p = rem / r0;
        int off = p * gstr[mode] + q * gstr[others[0]];
        if (N >= 3) off += u * gstr[others[1]];
        if (N >= 4) off += z * gstr[others[2]];
        gp[e] = Gd[off];
    }
    const int tid = threadIdx.x;
    const int64_t c = (int64_t)tl.y * kThreads + tid;
    const int64_t cc = c < ncols ? c : ncols - 1;
    // this column's rows of the other modes' B factors -> vs[(q*RP+k)*256+tid]
    int64_t rowoff[kMaxModes - 1];
    if (dense) {
        int64_t rem = cc;
        for (int q = N - 2; q >= 0; --q) {
            const int j = others[q];
            rowoff[q] = P.boff[j] + (rem % P.d[j]) * RP;
            rem /= P.d[j];
        }
    } else {
        const BlockDev& bd = P.blk[tl.x];
        for (int q = 0; q < N - 1; ++q)
            rowoff[q] = P.boff[others[q]] + (int64_t)bd.cidx[(int64_t)q * ncols + cc] * RP;
    }
    T bv[N - 1][RP];
#pragma unroll
    for (int q = 0; q < N - 1; ++q)
#pragma unroll
        for (int k = 0; k < RP; ++k) bv[q][k] = Bf[rowoff[q] + k];
    if (sf) return;
    const int64_t hoff = dense ? 0 : P.blk[tl.x].hoff;
    // a sampled block's H has the mode's r rows (the threshold pass reads no
    // more); the full-unfolding H of a reconstruction all RP
    const int prows = dense ? RP : rm;
    if constexpr (N <= 3) {
        // the B rows stay in registers: the q and u loops are unrolled to RP
        // and masked at the true ranks, so the core's LDS reads pipeline
        double v0[RP], v1[RP];
#pragma unroll
        for (int k = 0; k < RP; ++k) {
            v0[k] = (double)bv[0][k];
            v1[k] = N == 3 ? (double)bv[N == 3 ? 1 : 0][k] : 0.0;
        }
        __syncthreads();  // gp staged
        for (int p = 0; p < prows; ++p) {
            double a = 0.0;
            if (p < rm) {
#pragma unroll
                for (int q = 0; q < RP; ++q) {
                    if (q < r0) {
                        double t1;
                        if constexpr (N == 2) {
                            t1 = gp[p * r0 + q];
                        } else {
                            t1 = 0.0;
#pragma unroll
                            for (int u = 0; u < RP; ++u)
                                if (u < r1) t1 = fma(gp[(p * r0 + q) * r1 + u], v1[u], t1);
                        }
                        a = fma(t1, v0[q], a);
                    }
                }
            }
            if (c < ncols) H[hoff + (int64_t)p * ncols + c] = (T)a;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < N - 1; ++q)
#pragma unroll
        for (int k = 0; k < RP; ++k) vs[(q * RP + k) * kThreads + tid] = (double)bv[q][k];
    __syncthreads();
    const double* v0 = vs + tid;
    const double* v1 = vs + RP * kThreads + tid;
    const double* v2 = vs + 2 * RP * kThreads + tid;
    for (int p = 0; p < prows; ++p) {
        double a = 0.0;
        if (p < rm) {
            for (int q = 0; q < r0; ++q) {
                double t1 = 0.0;
                for (int u = 0; u < r1; ++u) {
                    double t2 = 0.0;
                    for (int z = 0; z < r2; ++z)
                        t2 = fma(gp[((p * r0 + q) * r1 + u) * r2 + z], v2[z * kThreads], t2);
                    t1 = fma(t2, v1[u * kThreads], t1);
                }
                a = fma(t1, v0[q * kThreads], a);
            }
        }
        if (c < ncols) H[hoff + (int64_t)p * ncols + c] = (T)a;
    }
}

// ------------------------------------------------------- full reconstruction
// L = G x_i B_i over every entry: out[x][c] = sum_p B_0[x][p] Hfull[p][c],
// Hfull = G x_{j >= 1} B_j over the full mode-0 unfolding columns.
template <typename T, typename TO, int RP>
__global__ __launch_bounds__(kThreads) void k_recon(int d0, int64_t ncols,
                                                    const T* __restrict__ B0,
                                                    const T* __restrict__ Hf,
                                                    TO* __restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int x0 = blockIdx.y * kTileRows;
    __shared__ T bs[kTileRows][RP];
    if (threadIdx.x < kTileRows * RP) {
        const int x = threadIdx.x / RP, p = threadIdx.x % RP;
        bs[x][p] = (x0 + x < d0) ? B0[(int64_t)(x0 + x) * RP + p] : T(0);
    }
    __syncthreads();
    if (c >= ncols) return;
    T h[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) h[p] = Hf[(int64_t)p * ncols + c];
    const int rows = min(kTileRows, d0 - x0);
    for (int x = 0; x < rows; ++x) {
        T L = T(0);
#pragma unroll
        for (int p = 0; p < RP; ++p) L = fma(bs[x][p], h[p], L);
        out[(int64_t)(x0 + x) * ncols + c] = (TO)L;
    }
}

// Full-grid outliers fused with the reconstruction (the S-update of
// equation 11 applied to every entry of X instead of the sampled blocks):
// L = sum_p B_0[x][p] H[p][c] on the mode-0 unfolding, D = X - L in the
// compute type, S = D where |D| > zeta (strict, equation 10) else 0.  One
// read of X, one write of S (and of L when L_out is given).
template <typename T, typename TX, typename TO, int RP>
__global__ __launch_bounds__(kThreads) void k_outliers(int d0, int64_t ncols,
                                                       const T* __restrict__ B0,
                                                       const T* __restrict__ Hf,
                                                       const TX* __restrict__ X, double zeta,
                                                       TO* __restrict__ S_out,
                                                       TO* __restrict__ L_out) {
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int x0 = blockIdx.y * kTileRows;
    __shared__ T bs[kTileRows][RP];
    if (threadIdx.x < kTileRows * RP) {
        const int x = threadIdx.x / RP, p = threadIdx.x % RP;
        bs[x][p] = (x0 + x < d0) ? B0[(int64_t)(x0 + x) * RP + p] : T(0);
    }
    __syncthreads();
    if (c >= ncols) return;
    const int rows = min(kTileRows, d0 - x0);
    TX xv[kTileRows];
#pragma unroll
    for (int x = 0; x < kTileRows; ++x)
        xv[x] = X[(int64_t)(x0 + (x < rows ? x : rows - 1)) * ncols + c];
    T h[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) h[p] = Hf[(int64_t)p * ncols + c];
#pragma unroll
    for (int x = 0; x < kTileRows; ++x) {
        if (x >= rows) break;  // uniform
        T L = T(0);
#pragma unroll
        for (int p = 0; p < RP; ++p) L = fma(bs[x][p], h[p], L);
        const T D = (T)xv[x] - L;
        const int64_t e = (int64_t)(x0 + x) * ncols + c;
        S_out[e] = (TO)(fabs((double)D) > zeta ? D : T(0));
        if (L_out) L_out[e] = (TO)L;
    }
}

// L on one sampled block (for inspection): out[x][c] = sum_p B[x][p] H[p][c].
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_evalblock(Prob P, int b,
                                                        const T* __restrict__ Bf,
                                                        const T* __restrict__ H,
                                                        double* __restrict__ out) {
    const BlockDev& bd = P.blk[b];
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= (int64_t)bd.nrows * bd.ncols) return;
    const int x = (int)(e / bd.ncols);
    const int c = (int)(e % bd.ncols);
    const int64_t xi = bd.rowidx ? bd.rowidx[x] : x;
    T L = T(0);
#pragma unroll
    for (int p = 0; p < RP; ++p)
        if (p < bd.r)  // (the block's H has r rows)
            L = fma(Bf[P.boff[bd.mode] + xi * RP + p], H[bd.hoff + (int64_t)p * bd.ncols + c], L);
    out[e] = (double)L;
}

// support bitmask of a block -> 0/1 doubles
__global__ void k_unpack_mask(const uint64_t* __restrict__ mask, int64_t moff, int words,
                              int nrows, int ncols, double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= (int64_t)nrows * ncols) return;
    const int x = (int)(e / ncols), c = (int)(e % ncols);
    const uint64_t wd = mask[moff + (int64_t)x * words + (c >> 6)];
    out[e] = ((wd >> (c & 63)) & 1ull) ? 1.0 : 0.0;
}

// out[0..N) = 0 (a fill kernel rather than a memset: safe inside a captured
// graph)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_zero(T* __restrict__ out, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < N; e += stride)
        out[e] = T(0);
}

// The work list of an H expansion over the full mode-0 unfolding: tile q
// covers columns [256 q, 256 q + 256) (block id -1: dense).
__global__ __launch_bounds__(kThreads) void k_dense_tiles(int2* __restrict__ tiles,
                                                          int64_t ntile) {
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q < ntile) tiles[q] = make_int2(-1, (int)q);
}

template <typename T>
__global__ void k_to_double(const T* __restrict__ in, int64_t N, double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e < N) out[e] = (double)in[e];
}

}  // namespace rtcur
