// Device kernels of the RTCUR hot loop for gfx950 (wave64).
//
// Data layout in HBM (all block-sized buffers share one layout):
//   block 0 (R) then blocks 1..n (C_i), each row-major nrows x ncols;
//   B_i factors d_i x RP (RP = rank padded to 4/8/16 with zero columns);
//   H_b = (G x_{j != mode} B_j)(columns of block b), RP x ncols per block;
//   W_i, Y_i (float64) s_i x RP; Z_i (float64) RP x m_i.
// With these, L on any block entry (x, c) is sum_p B_mode[x][p] H_b[p][c]:
// the Tucker form G x_i B_i of L = R x_i (C_i U_i^+) (equation 5), where
// U_i^+ = V_i S_i^-1 W_i^T, G = R x_i W_i^T and B_i = C_i V_i S_i^-1.
//
// Cross-workgroup reductions never use in-kernel fences: each launch writes
// per-workgroup partials and the next launch (after the kernel boundary has
// made them visible) sums them in a fixed order, so every result is bitwise
// reproducible.  Streaming loops issue all their global loads before using
// any of them, so that many loads are in flight per wave.
#pragma once

#include "internal.h"

namespace rtcur {

constexpr int kThreads = 256;      // 4 waves of 64
constexpr int kEigThreads = 1024;  // 16 waves for the eigensolver
constexpr int kTileRows = 16;      // rows per gather / threshold tile
constexpr int kTileCols = 256;     // one column per thread
constexpr int kGramMinChunk = 2048; // Gram: columns per work item (at least)
constexpr int kGramMaxKC = 16;     // Gram: column chunks per output tile (at most)
constexpr int kBfacRowsPerWave = 4;
constexpr int kBfacRows = 4 * kBfacRowsPerWave;

enum HtFlags { kHaveL = 1, kDoE = 2, kDoHT = 4, kDecide = 8, kFirstGather = 16 };

typedef double v4d __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
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

// --------------------------------------------------------------- set-up

__global__ void k_init_state(DevState* st, double zeta0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->stop = 0;
        st->status = 0;
        st->final_iter = 0;
        st->converged = 0;
        st->zeta0 = zeta0;
        st->den = 0.0;
        st->eig_steps = 0;
        st->eig_unconverged = 0;
        for (int j = 0; j < 4; ++j) st->counter[j] = 0u;
    }
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
// X_Omega: R = X(I_1..I_n), C_i = X_(i)(:, J_i) (Algorithm 1, equation 6),
// with per-tile squared sums for the denominator of e^(k) (equation 11).
template <typename TX, typename T>
__global__ __launch_bounds__(kThreads) void k_gather(
    const TX* __restrict__ X, Prob P, const int4* __restrict__ tiles,
    T* __restrict__ XO, double* part) {
    __shared__ double red[4];
    const int4 tl = tiles[blockIdx.x];
    const BlockDev& bd = P.blk[tl.x];
    const int c = tl.z + threadIdx.x;
    const int rows = min(kTileRows, bd.nrows - tl.y);
    const bool valid = c < bd.ncols;
    const int cc = valid ? c : bd.ncols - 1;
    const int64_t cx = bd.colx[cc];
    const int64_t rs = P.xstride[bd.mode];
    TX v[kTileRows];
#pragma unroll
    for (int x = 0; x < kTileRows; ++x) {
        const int xr = tl.y + (x < rows ? x : rows - 1);
        const int64_t xi = bd.rowidx ? bd.rowidx[xr] : xr;
        v[x] = X[xi * rs + cx];
    }
    double acc = 0.0, bad = 0.0;
#pragma unroll
    for (int x = 0; x < kTileRows; ++x) {
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
// For iteration k+1 on every block entry (Section 3.3, equations 8, 10, 11):
//   L^k = sum_p B[x][p] H[p][c]              (formed on the fly, never stored)
//   E   = C^k - L^k  -> per-tile sums of E^2 (numerator of e^(k))
//   D   = X - L^k;  S = D if |D| > zeta_{k+1} else 0;  C^{k+1} = X - S
// zeta_{k+1} = gamma^(k+1) zeta_0 by repeated multiplication (equation 9).
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_ht(
    Prob P, const int4* __restrict__ tiles, const T* __restrict__ XO,
    const T* __restrict__ Cold, T* __restrict__ Cnew,
    uint64_t* __restrict__ mask, const T* __restrict__ Bf,
    const T* __restrict__ H, double gamma, int kcur, int flags,
    double* __restrict__ part, const DevState* st) {
    if (stopped(st)) return;
    __shared__ T brow[kTileRows][RP];
    __shared__ double red[4];
    const bool haveL = flags & kHaveL, doE = flags & kDoE, doHT = flags & kDoHT;
    const int4 tl = tiles[blockIdx.x];
    const BlockDev& bd = P.blk[tl.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int c = tl.z + tid;
    const bool valid = c < bd.ncols;
    const int cc = valid ? c : bd.ncols - 1;
    const int rows = min(kTileRows, bd.nrows - tl.y);
    double zeta = st->zeta0;
    for (int j = 0; j <= kcur; ++j) zeta *= gamma;

    // all loads first
    T xv[kTileRows], co[kTileRows];
    const int64_t base = bd.off + (int64_t)tl.y * bd.ncols + cc;
#pragma unroll
    for (int x = 0; x < kTileRows; ++x) {
        const int64_t e = base + (int64_t)(x < rows ? x : rows - 1) * bd.ncols;
        xv[x] = doHT ? XO[e] : T(0);
        co[x] = doE ? Cold[e] : T(0);
    }
    T h[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) h[p] = T(0);
    if (haveL) {
#pragma unroll
        for (int p = 0; p < RP; ++p) h[p] = H[bd.hoff + (int64_t)p * bd.ncols + cc];
        if (tid < kTileRows * RP) {
            const int x = tid / RP, p = tid % RP;
            const int xr = tl.y + (x < rows ? x : rows - 1);
            const int64_t xi = bd.rowidx ? bd.rowidx[xr] : xr;
            brow[x][p] = Bf[P.boff[bd.mode] + xi * RP + p];
        }
        __syncthreads();
    }
    double e2 = 0.0;
#pragma unroll
    for (int x = 0; x < kTileRows; ++x) {
        if (x >= rows) break;  // uniform
        T L = T(0);
        if (haveL) {
#pragma unroll
            for (int p = 0; p < RP; ++p) L = fma(brow[x][p], h[p], L);
        }
        const int64_t e = bd.off + (int64_t)(tl.y + x) * bd.ncols + c;
        if (doE && valid) {
            const double dv = (double)co[x] - (double)L;
            e2 += dv * dv;
        }
        if (doHT) {
            const T D = xv[x] - L;
            const bool keep = valid && fabs((double)D) > zeta;
            const T S = keep ? D : T(0);
            if (valid) Cnew[e] = xv[x] - S;
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
// U_i^+, equation 6), in float64 on the matrix cores: one work item is a
// 16x16 output tile (upper triangle only) over one column chunk (at least
// 2048 columns, a quarter per wave),
// as a chain of V_MFMA_F64_16X16X4 (lane l feeds row l%16, k-slot l/16; the
// accumulator's register v of lane l is row 4v + l/16, column l%16).  The
// per-item tiles are summed by the eigensolver.  With `decide`, one extra
// workgroup forms e^(k) from the threshold pass's partials.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gram(
    Prob P, const T* __restrict__ C, const int4* __restrict__ items, int nitems,
    double* __restrict__ gpart, int decide, const double* hpart, int kcur, double tol,
    double* err_hist, DevState* st) {
    if (stopped(st)) return;
    __shared__ double sacc[4][256];
    if ((int)blockIdx.x == nitems) {
        if (decide) decide_block(P, hpart, kcur, tol, err_hist, st, &sacc[0][0]);
        return;
    }
    const int4 it = items[blockIdx.x];
    const int i = it.x, ta = it.y & 0xffff, tb = it.y >> 16;
    const int kc = it.z & 0xffff;
    const BlockDev& bd = P.blk[1 + i];
    const int s = P.s[i], m = bd.ncols;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ia = ta * 16 + (lane & 15), ib = tb * 16 + (lane & 15);
    const int g = lane >> 4;
    const bool okA = ia < s, okB = ib < s;
    const T* rowA = C + bd.off + (int64_t)P.I[i][okA ? ia : s - 1] * m;
    const T* rowB = C + bd.off + (int64_t)P.I[i][okB ? ib : s - 1] * m;
    const int kw = P.gchunk[i] / 4;
    const int kbeg = kc * P.gchunk[i] + w * kw;
    const int kend = min(kbeg + kw, m);
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = kbeg; k0 < kend; k0 += 64) {
        // 4 k-steps of 16 columns: 16 loads of A and 16 of B in flight
        T ra[16], rb[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int kk = k0 + 16 * (q >> 2) + 4 * g + (q & 3);
            const int ks = kk < kend ? kk : kbeg;
            ra[q] = rowA[ks];
            rb[q] = rowB[ks];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int kk = k0 + 16 * (q >> 2) + 4 * g + (q & 3);
            const bool in = kk < kend;
            const double av = (okA && in) ? (double)ra[q] : 0.0;
            const double bv = (okB && in) ? (double)rb[q] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sacc[w][(4 * v + g) * 16 + (lane & 15)] = acc[v];
    __syncthreads();
    gpart[(int64_t)blockIdx.x * 256 + tid] =
        ((sacc[0][tid] + sacc[1][tid]) + sacc[2][tid]) + sacc[3][tid];
}

// ------------------------------------------------ truncated eigensolver
// Top-r eigenpairs of Gram_i = U_i U_i^T in float64, one 1024-thread
// workgroup per mode: the Gram is assembled in LDS from the k_gram tiles,
// then subspace iteration (warm-started from the previous iterate's W_i
// under RTCUR-F) with Cholesky-QR orthonormalisation runs until the residual
// ||G Q - Q T||_F <= rtol ||T||_F with T = Q^T G Q, and a Rayleigh-Ritz step
// T = V diag(lambda) V^T (cyclic Jacobi) gives W_i = Q V.  The singular
// values of U_i are sqrt(lambda); Y_i = W_i diag(1/lambda) so that
// U_i^+ = U_i^T Y_i W_i^T.  Rank test: lambda_r <= 64 s 2^-52 lambda_1.

__device__ __forceinline__ uint32_t eig_hash(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return h;
}

constexpr int kEigWaves = kEigThreads / 64;

// Out (r x r) = A^T B for s x r row-major A, B in LDS; wave-parallel dots.
__device__ void eig_atb(const double* A, const double* B, int s, int r, double* Out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = w; q < r * r; q += kEigWaves) {
        const int p = q / r, t = q % r;
        double v = 0.0;
        for (int a = lane; a < s; a += 64) v += A[a * r + p] * B[a * r + t];
        v = wave_sum(v);
        if (lane == 0) Out[q] = v;
    }
}

// Cholesky of the r x r SPD matrix M (row-major) into upper R, M = R^T R.
// Single thread.  Returns false if a pivot is not positive.
__device__ bool eig_chol(const double* M, double* R, int r) {
    for (int p = 0; p < r * r; ++p) R[p] = 0.0;
    for (int j = 0; j < r; ++j) {
        double d = M[j * r + j];
        for (int k = 0; k < j; ++k) d -= R[k * r + j] * R[k * r + j];
        if (!(d > 0.0)) return false;
        const double rjj = sqrt(d);
        R[j * r + j] = rjj;
        for (int q = j + 1; q < r; ++q) {
            double v = M[j * r + q];
            for (int k = 0; k < j; ++k) v -= R[k * r + j] * R[k * r + q];
            R[j * r + q] = v / rjj;
        }
    }
    return true;
}

// Q = Z R^-1 (row by row), R upper triangular r x r.
__device__ void eig_trsm(const double* Z, const double* R, int s, int r, double* Q) {
    for (int a = threadIdx.x; a < s; a += kEigThreads) {
        double q[kMaxRank];
        for (int p = 0; p < r; ++p) {
            double v = Z[a * r + p];
            for (int k = 0; k < p; ++k) v -= q[k] * R[k * r + p];
            q[p] = v / R[p * r + p];
        }
        for (int p = 0; p < r; ++p) Q[a * r + p] = q[p];
    }
}

// Z = G Q (s x s times s x r): 4 threads share one output, each summing a
// quarter of b, combined with two shuffles.
__device__ void eig_gq(const double* G, const double* Q, int s, int r, double* Z) {
    const int sub = threadIdx.x & 3;
    for (int idx = threadIdx.x >> 2; idx < ((s * r + 63) / 64) * 64; idx += kEigThreads / 4) {
        const bool ok = idx < s * r;
        const int id = ok ? idx : 0;
        const int a = id / r, p = id % r;
        const double* g = G + a * s;
        double v0 = 0.0, v1 = 0.0;
        int b = sub;
        for (; b + 4 < s; b += 8) {
            v0 = fma(g[b], Q[b * r + p], v0);
            v1 = fma(g[b + 4], Q[(b + 4) * r + p], v1);
        }
        if (b < s) v0 = fma(g[b], Q[b * r + p], v0);
        double v = v0 + v1;
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        if (ok && sub == 0) Z[idx] = v;
    }
}

// Cyclic Jacobi on the symmetric r x r matrix A (single thread): A is
// overwritten by its diagonalisation, V accumulates the rotations.
__device__ void eig_jacobi(double* A, double* V, int r) {
    for (int p = 0; p < r; ++p)
        for (int q = 0; q < r; ++q) V[p * r + q] = (p == q) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int p = 0; p < r; ++p)
            for (int q = 0; q < r; ++q) {
                const double v = A[p * r + q] * A[p * r + q];
                tot += v;
                if (p != q) off += v;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < r - 1; ++p) {
            for (int q = p + 1; q < r; ++q) {
                const double apq = A[p * r + q];
                if (apq == 0.0) continue;
                const double app = A[p * r + p], aqq = A[q * r + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) /
                                 (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < r; ++k) {  // A <- A J (columns p, q)
                    const double akp = A[k * r + p], akq = A[k * r + q];
                    A[k * r + p] = cs * akp - sn * akq;
                    A[k * r + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < r; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = A[p * r + k], aqk = A[q * r + k];
                    A[p * r + k] = cs * apk - sn * aqk;
                    A[q * r + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < r; ++k) {  // V <- V J
                    const double vkp = V[k * r + p], vkq = V[k * r + q];
                    V[k * r + p] = cs * vkp - sn * vkq;
                    V[k * r + q] = sn * vkp + cs * vkq;
                }
            }
        }
    }
}

__global__ __launch_bounds__(kEigThreads) void k_eig(Prob P,
                                                     const double* __restrict__ gpart,
                                                     double* __restrict__ gram,
                                                     double* __restrict__ W,
                                                     double* __restrict__ Y,
                                                     double* __restrict__ lam,
                                                     int warm, int maxit, double rtol,
                                                     int use_lds_gram, DevState* st) {
    if (stopped(st)) return;
    extern __shared__ double lds[];
    __shared__ double red[kEigWaves];
    __shared__ double Tm[kMaxRank * kMaxRank], Mm[kMaxRank * kMaxRank],
        Rm[kMaxRank * kMaxRank], Vm[kMaxRank * kMaxRank];
    __shared__ double lamv[kMaxRank];
    __shared__ int order[kMaxRank];
    __shared__ int s_ok;
    const int i = blockIdx.x;
    const int s = P.s[i], r = P.r[i], RP = P.rp;
    const int tid = threadIdx.x;
    double* Q = lds;
    double* Z = Q + s * r;
    double* G = use_lds_gram ? Z + s * r : gram + P.goff[i];
    double* Wi = W + P.woff[i];
    if (tid == 0) s_ok = 1;

    // assemble the Gram from the per-item tiles (fixed chunk order)
    {
        const int nt = (s + 15) / 16;
        const int npairs = nt * (nt + 1) / 2;
        const int it0 = P.gitem0[i];
        const int nkc = P.gnkc[i];
        const int total = npairs * 256;
        for (int f = tid; f < total; f += kEigThreads) {
            const int q = f >> 8, t = f & 255;
            const double* src = gpart + (int64_t)(it0 + q * nkc) * 256 + t;
            double v[kGramMaxKC];
#pragma unroll
            for (int kc = 0; kc < kGramMaxKC; ++kc)
                v[kc] = src[(int64_t)(kc < nkc ? kc : 0) * 256];
            double sum = 0.0;
#pragma unroll
            for (int kc = 0; kc < kGramMaxKC; ++kc)
                if (kc < nkc) sum += v[kc];
            // pair q -> (ta, tb), ta <= tb, ta-major
            int ta = 0, rem = q;
            while (rem >= nt - ta) {
                rem -= nt - ta;
                ++ta;
            }
            const int tb = ta + rem;
            const int a = ta * 16 + (t >> 4), b = tb * 16 + (t & 15);
            if (a < s && b < s) {
                G[a * s + b] = sum;
                G[b * s + a] = sum;
            }
        }
    }
    __syncthreads();

    if (warm) {
        for (int e = tid; e < s * r; e += kEigThreads) Q[e] = Wi[(e / r) * RP + e % r];
    } else {
        // start block G * Omega, Omega a fixed +-1 pattern, then CholQR twice
        for (int e = tid; e < s * r; e += kEigThreads)
            Z[e] = (eig_hash(e / r, e % r) & 1u) ? 1.0 : -1.0;
        __syncthreads();
        eig_gq(G, Z, s, r, Q);
        __syncthreads();
        for (int rep = 0; rep < 2; ++rep) {
            eig_atb(Q, Q, s, r, Mm);
            __syncthreads();
            if (tid == 0) s_ok = eig_chol(Mm, Rm, r);
            __syncthreads();
            if (!s_ok) break;
            for (int e = tid; e < s * r; e += kEigThreads) Z[e] = Q[e];
            __syncthreads();
            eig_trsm(Z, Rm, s, r, Q);
            __syncthreads();
        }
        if (!s_ok) {
            if (tid == 0) {
                st->stop = 1;
                st->status = RTCUR_E_RANK;
            }
            return;
        }
    }
    __syncthreads();
    int steps = 0;
    bool conv = false;
    for (; steps <= maxit; ++steps) {
        eig_gq(G, Q, s, r, Z);
        __syncthreads();
        eig_atb(Q, Z, s, r, Tm);
        __syncthreads();
        double rn = 0.0;
        for (int e = tid; e < s * r; e += kEigThreads) {
            const int a = e / r, p = e % r;
            double v = Z[e];
            for (int k = 0; k < r; ++k) v -= Q[a * r + k] * Tm[k * r + p];
            rn += v * v;
        }
        rn = block_sum<kEigWaves>(rn, red);
        double tn = 0.0;
        for (int e = 0; e < r * r; ++e) tn += Tm[e] * Tm[e];
        if (rn <= rtol * rtol * tn) {
            conv = true;
            break;
        }
        if (steps == maxit) break;
        eig_atb(Z, Z, s, r, Mm);
        __syncthreads();
        if (tid == 0) s_ok = eig_chol(Mm, Rm, r);
        __syncthreads();
        if (!s_ok) break;
        eig_trsm(Z, Rm, s, r, Q);
        __syncthreads();
    }
    if (!s_ok) {
        if (tid == 0) {
            st->stop = 1;
            st->status = RTCUR_E_RANK;
        }
        return;
    }
    // Rayleigh-Ritz: T = Q^T G Q (symmetrised), T = V diag(lambda) V^T
    if (tid == 0) {
        for (int p = 0; p < r; ++p)
            for (int q = 0; q < r; ++q) Mm[p * r + q] = 0.5 * (Tm[p * r + q] + Tm[q * r + p]);
        eig_jacobi(Mm, Vm, r);
        for (int p = 0; p < r; ++p) {
            lamv[p] = Mm[p * r + p];
            order[p] = p;
        }
        for (int p = 1; p < r; ++p) {  // insertion sort, descending
            int o = order[p], q = p;
            while (q > 0 && lamv[order[q - 1]] < lamv[o]) {
                order[q] = order[q - 1];
                --q;
            }
            order[q] = o;
        }
        atomicAdd(&st->eig_steps, steps);
        if (!conv) atomicAdd(&st->eig_unconverged, 1);
        const double l1 = lamv[order[0]], lr = lamv[order[r - 1]];
        if (!isfinite(l1)) {
            st->stop = 1;
            st->status = RTCUR_E_NONFINITE;
        } else if (!(l1 > 0.0) || lr <= 64.0 * s * 0x1p-52 * l1) {
            st->stop = 1;
            st->status = RTCUR_E_RANK;
        }
    }
    __syncthreads();
    double* Yi = Y + P.woff[i];
    double* li = lam + P.loff[i];
    for (int e = tid; e < s * RP; e += kEigThreads) {
        const int a = e / RP, p = e % RP;
        double wv = 0.0, yv = 0.0;
        if (p < r) {
            const int o = order[p];
            for (int k = 0; k < r; ++k) wv += Q[a * r + k] * Vm[k * r + o];
            yv = wv / lamv[o];
        }
        Wi[e] = wv;
        Yi[e] = yv;
    }
    if (tid < RP) li[tid] = tid < r ? lamv[order[tid]] : 0.0;
}

// --------------------------- Z_i = Y_i^T U_i  and the core's first phase
// Workgroups [0, nz): Z_i (m_i x RP, float64, row per column) with
// U_i = C_i(I_i, :), so that V_i S_i^-1 = Z_i; 64 columns per workgroup,
// four threads per column each summing a quarter of the s_i rows.
// Workgroups [nz, nz + s_0): T[a] = R(a, :, ..) x_{l >= 1} W_l^T, the core
// G = R x_i W_i^T before its last contraction (with W_0, done by k_hexp).
template <typename T, int RP>
__device__ void zmat_tile(const Prob& P, const T* __restrict__ C, const double* __restrict__ Y,
                          double* __restrict__ Zbuf, int2 tl, double* ys) {
    const int i = tl.x;
    const BlockDev& bd = P.blk[1 + i];
    const int s = P.s[i], m = bd.ncols;
    const double* Yi = Y + P.woff[i];
    for (int e = threadIdx.x; e < s * RP; e += kThreads) ys[e] = Yi[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int quarter = lane >> 4;
    const int c = tl.y + w * 16 + (lane & 15);
    const int cc = c < m ? c : m - 1;
    const int qlen = (s + 3) / 4;
    const int a0 = quarter * qlen;
    const int32_t* Ii = P.I[i];
    const T* base = C + bd.off + cc;
    double acc[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) acc[p] = 0.0;
    constexpr int U = 16;
    for (int b0 = 0; b0 < qlen; b0 += U) {
        T u[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            int a = a0 + b0 + q;
            a = (b0 + q < qlen && a < s) ? a : a0;
            u[q] = base[(int64_t)Ii[a < s ? a : s - 1] * m];
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int a = a0 + b0 + q;
            if (b0 + q < qlen && a < s) {
                const double uv = (double)u[q];
#pragma unroll
                for (int p = 0; p < RP; ++p) acc[p] = fma(uv, ys[a * RP + p], acc[p]);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < RP; ++p) {
        acc[p] += __shfl_xor(acc[p], 16, 64);
        acc[p] += __shfl_xor(acc[p], 32, 64);
    }
    if (quarter == 0 && c < m) {
        double* Zi = Zbuf + P.zoff[i] + (int64_t)c * RP;
#pragma unroll
        for (int p = 0; p < RP; ++p) Zi[p] = acc[p];
    }
}

constexpr int kCoreLds = 4096;  // doubles of LDS for one slice's partial core

// T[a] for one slice a of the R block (row-major s_0 x ... x s_{n-1}):
// contract the last mode from global memory, the others in LDS; each step
// puts the new rank index first, so T[a] ends up ordered (r_1, .., r_{n-1}).
template <typename T, int RP>
__device__ void core_slice(const Prob& P, const T* __restrict__ R, const double* __restrict__ W,
                           double* __restrict__ Tbuf, int a, double* buf, double* ws) {
    const int n = P.n;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int rows = 1;
    for (int l = 1; l < n - 1; ++l) rows *= P.s[l];
    const int K = P.s[n - 1];
    const int rq = P.r[n - 1];
    for (int e = tid; e < K * RP; e += kThreads) ws[e] = W[P.woff[n - 1] + e];
    __syncthreads();
    const T* Ra = R + (int64_t)a * rows * K;
    // step 1: buf[p][row] = sum_k Ra[row][k] W_{n-1}[k][p], one wave per row
    for (int row0 = w * 4; row0 < rows; row0 += 16) {
        double v[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = row0 + j < rows ? row0 + j : rows - 1;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = lane + 64 * u;
                v[j][u] = k < K ? (double)Ra[(int64_t)row * K + k] : 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double acc[RP];
#pragma unroll
            for (int p = 0; p < RP; ++p) acc[p] = 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = lane + 64 * u;
                if (k < K) {
#pragma unroll
                    for (int p = 0; p < RP; ++p) acc[p] = fma(v[j][u], ws[k * RP + p], acc[p]);
                }
            }
#pragma unroll
            for (int p = 0; p < RP; ++p) acc[p] = wave_sum(acc[p]);
            if (lane < rq && row0 + j < rows) {
                double o = 0.0;
#pragma unroll
                for (int p = 0; p < RP; ++p)
                    if (p == lane) o = acc[p];
                buf[lane * rows + row0 + j] = o;
            }
        }
    }
    __syncthreads();
    // remaining modes n-2 .. 1 in LDS: [lead][rest][K'] -> [r'][lead][rest]
    int lead = rq;
    int rest = rows;
    double* cur = buf;
    double* nxt = buf + kCoreLds / 2;
    for (int l = n - 2; l >= 1; --l) {
        const int Kl = P.s[l], rl = P.r[l];
        rest /= Kl;
        const int M = lead * rest;
        __syncthreads();
        for (int e = tid; e < Kl * RP; e += kThreads) ws[e] = W[P.woff[l] + e];
        __syncthreads();
        for (int o = tid; o < rl * M; o += kThreads) {
            const int p = o / M, row = o % M;
            double acc = 0.0;
            for (int k = 0; k < Kl; ++k) acc = fma(cur[row * Kl + k], ws[k * RP + p], acc);
            nxt[o] = acc;
        }
        __syncthreads();
        double* t = cur;
        cur = nxt;
        nxt = t;
        lead *= rl;
    }
    int tot = 1;
    for (int l = 1; l < n; ++l) tot *= P.r[l];
    for (int e = tid; e < tot; e += kThreads) Tbuf[(int64_t)a * tot + e] = cur[e];
}

template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_zcore(Prob P, const T* __restrict__ C,
                                                    const double* __restrict__ Y,
                                                    double* __restrict__ Zbuf,
                                                    const int2* __restrict__ ztiles, int nz,
                                                    const double* __restrict__ W,
                                                    double* __restrict__ Tbuf,
                                                    const DevState* st) {
    if (stopped(st)) return;
    __shared__ double sh[kMaxS * RP];
    __shared__ double buf[kCoreLds];
    if ((int)blockIdx.x < nz) {
        zmat_tile<T, RP>(P, C, Y, Zbuf, ztiles[blockIdx.x], sh);
        return;
    }
    core_slice<T, RP>(P, C + P.blk[0].off, W, Tbuf, (int)blockIdx.x - nz, buf, sh);
}

// -------------------------------------------------------- B_i = C_i Z_i
// B_i (d_i x RP) = C_i V_i S_i^-1 = C_i Z_i.  Work item = (mode, 16 rows,
// 1024 columns): Z_i's chunk is staged in LDS, each wave owns 4 rows and its
// lanes stride the columns; partial rows go to bpart and k_bred adds the
// column chunks in order.
constexpr int kBfacKC = 1024;

template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_bfac(Prob P, const T* __restrict__ C,
                                                   const double* __restrict__ Zbuf,
                                                   const int4* __restrict__ items,
                                                   double* __restrict__ bpart,
                                                   const DevState* st) {
    if (stopped(st)) return;
    constexpr int KC = RP <= 8 ? kBfacKC : kBfacKC / 2;
    __shared__ double zs[KC * RP];
    const int4 it = items[blockIdx.x];
    const int i = it.x, rb = it.y, kc = it.z;
    const BlockDev& bd = P.blk[1 + i];
    const int m = bd.ncols, d = bd.nrows;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int c0 = kc * KC, cn = min(KC, m - c0);
    const double* Zc = Zbuf + P.zoff[i] + (int64_t)c0 * RP;
    for (int e = tid; e < KC * RP; e += kThreads) zs[e] = e < cn * RP ? Zc[e] : 0.0;
    const int xb = rb * kBfacRows + w * kBfacRowsPerWave;
    const T* rowp[kBfacRowsPerWave];
#pragma unroll
    for (int j = 0; j < kBfacRowsPerWave; ++j)
        rowp[j] = C + bd.off + (int64_t)(xb + j < d ? xb + j : d - 1) * m + c0;
    double acc[kBfacRowsPerWave][RP];
#pragma unroll
    for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
        for (int p = 0; p < RP; ++p) acc[j][p] = 0.0;
    __syncthreads();
    constexpr int U = 8;
    for (int u0 = 0; u0 < KC / 64; u0 += U) {
        T cv[kBfacRowsPerWave][U];
#pragma unroll
        for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = lane + 64 * (u0 + u);
                cv[j][u] = rowp[j][c < cn ? c : 0];
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = lane + 64 * (u0 + u);
            if (c < cn) {
                double z[RP];
#pragma unroll
                for (int p = 0; p < RP; ++p) z[p] = zs[c * RP + p];
#pragma unroll
                for (int j = 0; j < kBfacRowsPerWave; ++j) {
                    const double x = (double)cv[j][u];
#pragma unroll
                    for (int p = 0; p < RP; ++p) acc[j][p] = fma(x, z[p], acc[j][p]);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
        for (int p = 0; p < RP; ++p) acc[j][p] = wave_sum(acc[j][p]);
    double* out = bpart + ((int64_t)blockIdx.x * kBfacRows + w * kBfacRowsPerWave) * RP;
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

// G = sum_a W_0[a]^T T[a] (the last contraction of the core), one
// workgroup, T staged through LDS in slices of whole a-rows.
template <int RP>
__device__ void core_finish(const Prob& P, const double* __restrict__ W,
                            const double* __restrict__ Tbuf, double* __restrict__ Gd) {
    __shared__ double tb[kCoreLds / 2];
    __shared__ double wb[kCoreLds / 2];
    const int s0 = P.s[0], r0 = P.r[0];
    const int tot = P.core / r0;
    const int A = max(1, min((kCoreLds / 2) / tot, (kCoreLds / 2) / RP));
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
            wb[e] = W[P.woff[0] + (int64_t)a0 * RP + e];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < JM; ++j) {
            const int o = threadIdx.x + j * kThreads;
            if (o < P.core) {
                const int p = o / tot, rest = o % tot;
                double v = acc[j];
                for (int a = 0; a < na; ++a) v = fma(wb[a * RP + p], tb[a * tot + rest], v);
                acc[j] = v;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < JM; ++j) {
        const int o = threadIdx.x + j * kThreads;
        if (o < P.core) Gd[o] = acc[j];
    }
}

// B_i rows: sum of the column-chunk partials of k_bfac, in chunk order; the
// workgroup after the last one finishes the core G.
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_bred(Prob P, const double* __restrict__ bpart,
                                                   T* __restrict__ Bf, double* __restrict__ Bd,
                                                   int nred, const double* __restrict__ W,
                                                   const double* __restrict__ Tbuf,
                                                   double* __restrict__ Gd,
                                                   const DevState* st) {
    if (stopped(st)) return;
    if ((int)blockIdx.x == nred) {
        core_finish<RP>(P, W, Tbuf, Gd);
        return;
    }
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    // locate mode i of flat entry e over sum_i d_i * RP
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
    double v = 0.0;
    for (int kc = 0; kc < nkc; ++kc) v += src[(int64_t)kc * kBfacRows * RP];
    Bf[P.boff[i] + (int64_t)x * RP + p] = (T)v;
    Bd[P.boff[i] + (int64_t)x * RP + p] = v;
}

// ------------------------------------------------ H_b = G x_{j != mode} B_j
// For every column of a block (or, with a negative block id, every column of
// the full mode-`dense_mode` unfolding), H[p][c] = sum over the other modes'
// core indices of G[..p..] * prod_j B_j[idx_j(c)][q_j].  G sits in LDS
// permuted so that the block's own mode comes first (padded to RP per mode);
// each thread's B rows sit in LDS too, so the loops run to the true ranks.
template <typename T, int RP, int N>
__global__ __launch_bounds__(kThreads) void k_hexp(
    Prob P, const int2* __restrict__ tiles, const T* __restrict__ Bf,
    const double* __restrict__ Gd, T* __restrict__ H, const DevState* st,
    int dense_mode, int64_t dense_cols) {
    if (st && stopped(st)) return;
    constexpr int GP = N == 2 ? RP * RP : (N == 3 ? RP * RP * RP : RP * RP * RP * RP);
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
    // permuted, padded core: gp[p][q_0]..[q_{N-2}] = G[...] with p at `mode`
    int gstr[kMaxModes];
    gstr[N - 1] = 1;
    for (int j = N - 2; j >= 0; --j) gstr[j] = gstr[j + 1] * P.r[j + 1];
    for (int e = threadIdx.x; e < GP; e += kThreads) {
        int rem = e, idx[kMaxModes];
        for (int q = N - 2; q >= 0; --q) {
            idx[q] = rem % RP;
            rem /= RP;
        }
        const int p = rem;
        bool ok = p < P.r[mode];
        int off = p * gstr[mode];
        for (int q = 0; q < N - 1; ++q) {
            ok = ok && idx[q] < P.r[others[q]];
            off += idx[q] * gstr[others[q]];
        }
        gp[e] = ok ? Gd[off] : 0.0;
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
    {
        T bv[N - 1][RP];
#pragma unroll
        for (int q = 0; q < N - 1; ++q)
#pragma unroll
            for (int k = 0; k < RP; ++k) bv[q][k] = Bf[rowoff[q] + k];
#pragma unroll
        for (int q = 0; q < N - 1; ++q)
#pragma unroll
            for (int k = 0; k < RP; ++k) vs[(q * RP + k) * kThreads + tid] = (double)bv[q][k];
    }
    __syncthreads();
    const int rm = P.r[mode];
    const int r0 = P.r[others[0]];
    const int r1 = N >= 3 ? P.r[others[1]] : 1;
    const int r2 = N >= 4 ? P.r[others[2]] : 1;
    const double* v0 = vs + tid;
    const double* v1 = vs + RP * kThreads + tid;
    const double* v2 = vs + 2 * RP * kThreads + tid;
    const int64_t hoff = dense ? 0 : P.blk[tl.x].hoff;
    for (int p = 0; p < RP; ++p) {
        double a = 0.0;
        if (p < rm) {
            for (int q = 0; q < r0; ++q) {
                double t1;
                if constexpr (N == 2) {
                    t1 = gp[p * RP + q];
                } else {
                    t1 = 0.0;
                    for (int u = 0; u < r1; ++u) {
                        double t2;
                        if constexpr (N == 3) {
                            t2 = gp[(p * RP + q) * RP + u];
                        } else {
                            t2 = 0.0;
                            for (int z = 0; z < r2; ++z)
                                t2 = fma(gp[((p * RP + q) * RP + u) * RP + z],
                                         v2[z * kThreads], t2);
                        }
                        t1 = fma(t2, v1[u * kThreads], t1);
                    }
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

template <typename T>
__global__ void k_to_double(const T* __restrict__ in, int64_t N, double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e < N) out[e] = (double)in[e];
}

}  // namespace rtcur
