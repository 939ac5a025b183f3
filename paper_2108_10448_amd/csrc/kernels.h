// Device kernels of the RTCUR hot loop for gfx950 (wave64).
//
// Data layout in HBM (all block-sized buffers share one layout):
//   block 0 (R) then blocks 1..n (C_i), each row-major nrows x ncols;
//   B_i factors d_i x RP (RP = rank padded to 4/8/16 with zero columns);
//   H_b = (G x_{j != mode} B_j)(columns of block b), RP x ncols per block;
//   W_i, Y_i (float64) s_i x RP; Z_i (float64) RP x m_i; Gram_i s_i x s_i.
// With these, L on any block entry (x, c) is sum_p B_mode[x][p] H_b[p][c]:
// the Tucker form G x_i B_i of L = R x_i (C_i U_i^+) (equation 5), where
// U_i^+ = V_i S_i^-1 W_i^T, G = R x_i W_i^T and B_i = C_i V_i S_i^-1.
#pragma once

#include "internal.h"

namespace rtcur {

constexpr int kThreads = 256;     // every kernel runs 4 waves of 64
constexpr int kTileRows = 16;     // rows per gather / threshold tile
constexpr int kTileCols = 256;    // one column per thread
constexpr int kGramKW = 256;      // Gram: columns per wave per work item
constexpr int kGramKCW = 4 * kGramKW;
constexpr int kBfacRowsPerWave = 4;
constexpr int kBfacRows = 4 * kBfacRowsPerWave;
constexpr int kBfacKC = 1024;     // B_i: columns per work item
constexpr int kContractRowsPerWave = 8;

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

// Sum over the 256 threads in a fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

__device__ __forceinline__ void st_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Last-arriving workgroup of a group of `total`: returns true in exactly one
// workgroup, after every other workgroup's prior agent-scope stores are
// visible.  The counter is reset by that workgroup for the next launch.
__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned total) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == total - 1u);
        if (s_last)
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last != 0;
}

__device__ __forceinline__ bool stopped(const DevState* st) {
    return __hip_atomic_load(const_cast<int*>(&st->stop), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT) != 0;
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

// zeta_0 = ||X||_inf over the whole tensor (one full read), with a
// non-finite check.  part: 2 doubles per workgroup.
template <typename TX>
__global__ __launch_bounds__(kThreads) void k_absmax(const TX* __restrict__ X,
                                                     int64_t N, double* part,
                                                     DevState* st) {
    __shared__ double red[4];
    double mx = 0.0, bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < N;
         e += stride) {
        double v = (double)X[e];
        if (!isfinite(v)) bad = 1.0;
        mx = fmax(mx, fabs(v));
    }
    mx = wave_max(mx);
    bad = wave_max(bad);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    double bm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bad;
    __syncthreads();
    double bb = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (threadIdx.x == 0) {
        st_agent(&part[2 * blockIdx.x], bm);
        st_agent(&part[2 * blockIdx.x + 1], bb);
    }
    if (!arrive_last(&st->counter[0], gridDim.x)) return;
    double m2 = 0.0, b2 = 0.0;
    for (unsigned t = threadIdx.x; t < gridDim.x; t += kThreads) {
        m2 = fmax(m2, ld_agent(&part[2 * t]));
        b2 = fmax(b2, ld_agent(&part[2 * t + 1]));
    }
    m2 = wave_max(m2);
    b2 = wave_max(b2);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m2;
    __syncthreads();
    double fm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b2;
    __syncthreads();
    double fb = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (threadIdx.x == 0) {
        st->zeta0 = fm;
        if (fb != 0.0) {
            st->stop = 1;
            st->status = RTCUR_E_NONFINITE;
        }
    }
}

// ------------------------------------------------------------------ gather
// X_Omega: R = X(I_1..I_n), C_i = X_(i)(:, J_i) (Algorithm 1, equation 6),
// plus the per-block squared norms that form the denominator of e^(k)
// (equation 11).  One tile = kTileRows rows x 256 columns of one block.
template <typename TX, typename T>
__global__ __launch_bounds__(kThreads) void k_gather(
    const TX* __restrict__ X, Prob P, const int4* __restrict__ tiles,
    T* __restrict__ XO, double* part, int flags, DevState* st) {
    __shared__ double red[4];
    const int4 tl = tiles[blockIdx.x];
    const BlockDev& bd = P.blk[tl.x];
    const int c = tl.z + threadIdx.x;
    const int rows = min(kTileRows, bd.nrows - tl.y);
    double acc = 0.0, bad = 0.0;
    if (c < bd.ncols) {
        const int64_t cx = bd.colx[c];
        const int64_t rs = P.xstride[bd.mode];
        for (int x = 0; x < rows; ++x) {
            const int xr = tl.y + x;
            const int64_t xi = bd.rowidx ? bd.rowidx[xr] : xr;
            const T v = (T)X[xi * rs + cx];
            XO[bd.off + (int64_t)xr * bd.ncols + c] = v;
            const double dv = (double)v;
            if (!isfinite(dv)) bad = 1.0;
            acc += dv * dv;
        }
    }
    const double sa = block_sum(acc, red);
    const double sb = block_sum(bad, red);
    if (threadIdx.x == 0) {
        st_agent(&part[2 * blockIdx.x], sa);
        st_agent(&part[2 * blockIdx.x + 1], sb);
    }
    if (!arrive_last(&st->counter[0], gridDim.x)) return;
    double den = 0.0, badall = 0.0;
    for (int b = 0; b < P.nblk; ++b) {
        double v = 0.0, w = 0.0;
        for (int t = P.blk[b].tile0 + threadIdx.x; t < P.blk[b].tile1; t += kThreads) {
            v += ld_agent(&part[2 * t]);
            w += ld_agent(&part[2 * t + 1]);
        }
        v = block_sum(v, red);
        w = block_sum(w, red);
        den += sqrt(v);
        badall += w;
    }
    if (threadIdx.x == 0) {
        st->den = den;
        if (badall != 0.0) {
            st->stop = 1;
            st->status = RTCUR_E_NONFINITE;
        } else if (den == 0.0 && (flags & kFirstGather)) {
            // all sampled entries are zero: L = 0 is the answer (k = 0)
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
//   E   = C^k - L^k  -> block sums of E^2    (numerator of e^(k))
//   D   = X - L^k;  S = D if |D| > zeta_{k+1} else 0;  C^{k+1} = X - S
// zeta_{k+1} = gamma^(k+1) zeta_0 by repeated multiplication (equation 9).
// The last workgroup forms e^(k) = sum_b ||E_b|| / den and raises `stop`
// when e^(k) <= tol, so iterations can be queued without host round trips.
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_ht(
    Prob P, const int4* __restrict__ tiles, const T* __restrict__ XO,
    const T* __restrict__ Cold, T* __restrict__ Cnew,
    uint64_t* __restrict__ mask, const T* __restrict__ Bf,
    const T* __restrict__ H, double gamma, int kcur, int flags, double tol,
    double* part, double* err_hist, DevState* st) {
    if (stopped(st)) return;
    __shared__ T brow[kTileRows][RP];
    __shared__ double red[4];
    const bool haveL = flags & kHaveL, doE = flags & kDoE, doHT = flags & kDoHT;
    const int4 tl = tiles[blockIdx.x];
    const BlockDev& bd = P.blk[tl.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int c = tl.z + tid;
    const bool valid = c < bd.ncols;
    const int rows = min(kTileRows, bd.nrows - tl.y);
    double zeta = st->zeta0;
    for (int j = 0; j <= kcur; ++j) zeta *= gamma;

    T h[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) h[p] = T(0);
    if (haveL) {
        if (valid) {
#pragma unroll
            for (int p = 0; p < RP; ++p)
                h[p] = H[bd.hoff + (int64_t)p * bd.ncols + c];
        }
        if (tid < kTileRows * RP) {
            const int x = tid / RP, p = tid % RP;
            T v = T(0);
            if (x < rows) {
                const int64_t xi = bd.rowidx ? bd.rowidx[tl.y + x] : (tl.y + x);
                v = Bf[P.boff[bd.mode] + xi * RP + p];
            }
            brow[x][p] = v;
        }
        __syncthreads();
    }
    double e2 = 0.0, ns = 0.0;
    for (int x = 0; x < rows; ++x) {
        const int64_t e = bd.off + (int64_t)(tl.y + x) * bd.ncols + c;
        T L = T(0);
        if (haveL) {
#pragma unroll
            for (int p = 0; p < RP; ++p) L = fma(brow[x][p], h[p], L);
        }
        bool keep = false;
        if (valid) {
            if (doE) {
                const double dv = (double)Cold[e] - (double)L;
                e2 += dv * dv;
            }
            if (doHT) {
                const T xv = XO[e];
                const T D = xv - L;
                keep = fabs((double)D) > zeta;
                const T S = keep ? D : T(0);
                Cnew[e] = xv - S;
                ns += keep ? 1.0 : 0.0;
            }
        }
        if (doHT) {
            const uint64_t bal = __ballot(keep);
            if (lane == 0 && tl.z + wv * 64 < bd.ncols)
                mask[bd.moff + (int64_t)(tl.y + x) * bd.words + (tl.z >> 6) + wv] = bal;
        }
    }
    if (!(flags & kDecide)) return;
    const double se = block_sum(e2, red);
    if (tid == 0) st_agent(&part[blockIdx.x], se);
    if (!arrive_last(&st->counter[1], gridDim.x)) return;
    double num = 0.0;
    for (int b = 0; b < P.nblk; ++b) {
        double v = 0.0;
        for (int t = P.blk[b].tile0 + tid; t < P.blk[b].tile1; t += kThreads)
            v += ld_agent(&part[t]);
        v = block_sum(v, red);
        num += sqrt(v);
    }
    if (tid == 0) {
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

// -------------------------------------------------------- Gram of U_i rows
// Gram_i = U_i U_i^T, U_i = C_i(I_i, :) (the matrix whose truncated SVD gives
// U_i^+, equation 6), in float64 on the matrix cores: one work item is a
// 16x16 output tile (upper triangle only) over 1024 columns, one
// V_MFMA_F64_16X16X4 chain per wave.  Per-item partial tiles are summed in
// item order by the last item of each tile.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gram(
    Prob P, const T* __restrict__ C, const int4* __restrict__ items,
    double* gpart, unsigned* gcnt, double* __restrict__ gram, DevState* st) {
    if (stopped(st)) return;
    __shared__ double sacc[4][256];
    const int4 it = items[blockIdx.x];
    const int i = it.x, ta = it.y & 0xffff, tb = it.y >> 16;
    const int kc = it.z & 0xffff, nkc = it.z >> 16, pid = it.w;
    const BlockDev& bd = P.blk[1 + i];
    const int s = P.s[i], m = bd.ncols;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ia = ta * 16 + (lane & 15), ib = tb * 16 + (lane & 15);
    const int g = lane >> 4;
    const T* rowA = ia < s ? C + bd.off + (int64_t)P.I[i][ia] * m : nullptr;
    const T* rowB = ib < s ? C + bd.off + (int64_t)P.I[i][ib] * m : nullptr;
    const int kbeg = kc * kGramKCW + w * kGramKW;
    const int kend = min(kbeg + kGramKW, m);
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = kbeg; k0 < kend; k0 += 16) {
        double av[4], bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int kk = k0 + 4 * g + j;
            const bool in = kk < kend;
            av[j] = (rowA && in) ? (double)rowA[kk] : 0.0;
            bv[j] = (rowB && in) ? (double)rowB[kk] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[j], acc, 0, 0, 0);
    }
    // accumulator layout (gfx950): lane l, register v holds row 4*v + l/16,
    // column l%16 of the 16x16 tile
#pragma unroll
    for (int v = 0; v < 4; ++v) sacc[w][(4 * v + g) * 16 + (lane & 15)] = acc[v];
    __syncthreads();
    const double tv = ((sacc[0][tid] + sacc[1][tid]) + sacc[2][tid]) + sacc[3][tid];
    st_agent(&gpart[(int64_t)blockIdx.x * 256 + tid], tv);
    if (!arrive_last(&gcnt[pid], nkc)) return;
    double sum = 0.0;
    const int64_t base = (int64_t)(blockIdx.x - kc) * 256 + tid;
    for (int q = 0; q < nkc; ++q) sum += ld_agent(&gpart[base + (int64_t)q * 256]);
    const int a = ta * 16 + tid / 16, b = tb * 16 + tid % 16;
    if (a < s && b < s) {
        double* G = gram + P.goff[i];
        G[(int64_t)a * s + b] = sum;
        if (ta != tb) G[(int64_t)b * s + a] = sum;
    }
}

// ------------------------------------------------ truncated eigensolver
// Top-r eigenpairs of Gram_i = U_i U_i^T in float64, one workgroup per mode:
// subspace iteration (warm-started from the previous iterate's W_i under
// RTCUR-F) with Cholesky-QR orthonormalisation, stopped when the residual
// ||G Q - Q T||_F <= rtol ||T||_F with T = Q^T G Q, then a Rayleigh-Ritz
// step: T = V diag(lambda) V^T by cyclic Jacobi, W_i = Q V.  The singular
// values of U_i are sqrt(lambda); Y_i = W_i diag(1/lambda) so that
// U_i^+ = U_i^T Y_i W_i^T.  Rank test: lambda_r <= 64 s 2^-52 lambda_1.

__device__ __forceinline__ uint32_t eig_hash(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return h;
}

// Out (r x r) = A^T B for s x r row-major A, B in LDS.  Wave-parallel dots.
__device__ void eig_atb(const double* A, const double* B, int s, int r,
                        double* Out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = w; q < r * r; q += 4) {
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
    for (int p = 0; p < r; ++p) {
        for (int q = 0; q < r; ++q) R[p * r + q] = 0.0;
    }
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
__device__ void eig_trsm(const double* Z, const double* R, int s, int r,
                         double* Q) {
    for (int a = threadIdx.x; a < s; a += kThreads) {
        double q[kMaxRank];
        for (int p = 0; p < r; ++p) {
            double v = Z[a * r + p];
            for (int k = 0; k < p; ++k) v -= q[k] * R[k * r + p];
            q[p] = v / R[p * r + p];
        }
        for (int p = 0; p < r; ++p) Q[a * r + p] = q[p];
    }
}

// Z = G Q (s x s times s x r).
__device__ void eig_gq(const double* G, const double* Q, int s, int r,
                       double* Z) {
    for (int idx = threadIdx.x; idx < s * r; idx += kThreads) {
        const int a = idx / r, p = idx % r;
        const double* g = G + (int64_t)a * s;
        double v = 0.0;
        for (int b = 0; b < s; ++b) v = fma(g[b], Q[b * r + p], v);
        Z[idx] = v;
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

__global__ __launch_bounds__(kThreads) void k_eig(Prob P,
                                                  const double* __restrict__ gram,
                                                  double* __restrict__ W,
                                                  double* __restrict__ Y,
                                                  double* __restrict__ lam,
                                                  int warm, int maxit,
                                                  double rtol, int use_lds_gram,
                                                  DevState* st) {
    if (stopped(st)) return;
    extern __shared__ double lds[];
    __shared__ double red[4];
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
    double* Gl = Z + s * r;
    const double* Gg = gram + P.goff[i];
    const bool in_lds = use_lds_gram != 0;
    if (tid == 0) s_ok = 1;
    if (in_lds) {
        for (int e = tid; e < s * s; e += kThreads) Gl[e] = Gg[e];
    }
    const double* G = in_lds ? Gl : Gg;
    double* Wi = W + P.woff[i];
    __syncthreads();

    if (warm) {
        for (int e = tid; e < s * r; e += kThreads) Q[e] = Wi[(e / r) * RP + e % r];
    } else {
        // start block G * Omega, Omega a fixed +-1 pattern, then CholQR twice
        for (int e = tid; e < s * r; e += kThreads)
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
            for (int e = tid; e < s * r; e += kThreads) Z[e] = Q[e];
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
    int steps = 0;
    bool conv = false;
    for (; steps <= maxit; ++steps) {
        eig_gq(G, Q, s, r, Z);
        __syncthreads();
        eig_atb(Q, Z, s, r, Tm);
        __syncthreads();
        double rn = 0.0;
        for (int e = tid; e < s * r; e += kThreads) {
            const int a = e / r, p = e % r;
            double v = Z[e];
            for (int k = 0; k < r; ++k) v -= Q[a * r + k] * Tm[k * r + p];
            rn += v * v;
        }
        rn = block_sum(rn, red);
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
            for (int q = 0; q < r; ++q)
                Mm[p * r + q] = 0.5 * (Tm[p * r + q] + Tm[q * r + p]);
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
        if (!(l1 > 0.0) || lr <= 64.0 * s * 0x1p-52 * l1) {
            st->stop = 1;
            st->status = RTCUR_E_RANK;
        } else if (!isfinite(l1)) {
            st->stop = 1;
            st->status = RTCUR_E_NONFINITE;
        }
    }
    __syncthreads();
    double* Yi = Y + P.woff[i];
    double* li = lam + P.loff[i];
    for (int e = tid; e < s * RP; e += kThreads) {
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

// ------------------------------------------------------------ Z_i = U_i^T Y_i
// Z_i (RP x m_i, float64) with U_i = C_i(I_i, :); then V_i S_i^-1 = Z_i^T.
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_zmat(Prob P, const T* __restrict__ C,
                                                   const double* __restrict__ Y,
                                                   double* __restrict__ Zbuf,
                                                   const int2* __restrict__ tiles,
                                                   DevState* st) {
    if (stopped(st)) return;
    __shared__ double ys[kMaxS * RP];
    const int2 tl = tiles[blockIdx.x];
    const int i = tl.x;
    const BlockDev& bd = P.blk[1 + i];
    const int s = P.s[i], m = bd.ncols;
    const double* Yi = Y + P.woff[i];
    for (int e = threadIdx.x; e < s * RP; e += kThreads) ys[e] = Yi[e];
    __syncthreads();
    const int c = tl.y + threadIdx.x;
    if (c >= m) return;
    double acc[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) acc[p] = 0.0;
    const int32_t* Ii = P.I[i];
    const T* base = C + bd.off + c;
    for (int a = 0; a < s; ++a) {
        const double u = (double)base[(int64_t)Ii[a] * m];
#pragma unroll
        for (int p = 0; p < RP; ++p) acc[p] = fma(u, ys[a * RP + p], acc[p]);
    }
    double* Zi = Zbuf + P.zoff[i];
#pragma unroll
    for (int p = 0; p < RP; ++p) Zi[(int64_t)p * m + c] = acc[p];
}

// --------------------------------------------------------- B_i = C_i Z_i^T
// B_i (d_i x RP) = C_i V_i S_i^-1.  Work item = (mode, 16-row block, 1024
// columns); each wave owns 4 rows, lanes stride the columns.  Partial sums
// are added in column-chunk order by the last item of each row block.
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_bfac(
    Prob P, const T* __restrict__ C, const double* __restrict__ Zbuf,
    const int4* __restrict__ items, double* bpart, unsigned* bcnt,
    T* __restrict__ Bf, double* __restrict__ Bd, DevState* st) {
    if (stopped(st)) return;
    const int4 it = items[blockIdx.x];
    const int i = it.x, rb = it.y, kc = it.z & 0xffff, nkc = it.z >> 16;
    const int cid = it.w;
    const BlockDev& bd = P.blk[1 + i];
    const int m = bd.ncols, d = bd.nrows;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double* Zi = Zbuf + P.zoff[i];
    const int c0 = kc * kBfacKC, c1 = min(c0 + kBfacKC, m);
    double acc[kBfacRowsPerWave][RP];
#pragma unroll
    for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
        for (int p = 0; p < RP; ++p) acc[j][p] = 0.0;
    const int xb = rb * kBfacRows + w * kBfacRowsPerWave;
    for (int c = c0 + lane; c < c1; c += 64) {
        double z[RP];
#pragma unroll
        for (int p = 0; p < RP; ++p) z[p] = Zi[(int64_t)p * m + c];
#pragma unroll
        for (int j = 0; j < kBfacRowsPerWave; ++j) {
            const int x = xb + j;
            const double cv = x < d ? (double)C[bd.off + (int64_t)x * m + c] : 0.0;
#pragma unroll
            for (int p = 0; p < RP; ++p) acc[j][p] = fma(cv, z[p], acc[j][p]);
        }
    }
#pragma unroll
    for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
        for (int p = 0; p < RP; ++p) acc[j][p] = wave_sum(acc[j][p]);
    double* mine = bpart + (int64_t)blockIdx.x * kBfacRows * RP;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < kBfacRowsPerWave; ++j)
#pragma unroll
            for (int p = 0; p < RP; ++p)
                st_agent(&mine[(w * kBfacRowsPerWave + j) * RP + p], acc[j][p]);
    }
    if (!arrive_last(&bcnt[cid], nkc)) return;
    const double* first = bpart + (int64_t)(blockIdx.x - kc) * kBfacRows * RP;
    for (int e = tid; e < kBfacRows * RP; e += kThreads) {
        double v = 0.0;
        for (int q = 0; q < nkc; ++q) v += ld_agent(&first[(int64_t)q * kBfacRows * RP + e]);
        const int x = rb * kBfacRows + e / RP, p = e % RP;
        if (x < d) {
            Bf[P.boff[i] + (int64_t)x * RP + p] = (T)v;
            Bd[P.boff[i] + (int64_t)x * RP + p] = v;
        }
    }
}

// ------------------------------------------- core G = R x_i W_i^T, by stages
// out[p][row] = sum_k in[row][k] W[k][p]: contract the last axis of a
// row-major M x K array and put the new axis first.  Applied n times to R
// (last mode first), this yields G with modes in their natural order.
template <typename TIN, int RP>
__global__ __launch_bounds__(kThreads) void k_contract(
    const TIN* __restrict__ in, int M, int K, const double* __restrict__ W,
    int r, double* __restrict__ out, DevState* st) {
    if (stopped(st)) return;
    __shared__ double ws[kMaxS * RP];
    for (int e = threadIdx.x; e < K * RP; e += kThreads) ws[e] = W[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row0 = (blockIdx.x * 4 + w) * kContractRowsPerWave;
    for (int j = 0; j < kContractRowsPerWave; ++j) {
        const int row = row0 + j;
        if (row >= M) break;
        double acc[RP];
#pragma unroll
        for (int p = 0; p < RP; ++p) acc[p] = 0.0;
        for (int k = lane; k < K; k += 64) {
            const double v = (double)in[(int64_t)row * K + k];
#pragma unroll
            for (int p = 0; p < RP; ++p) acc[p] = fma(v, ws[k * RP + p], acc[p]);
        }
#pragma unroll
        for (int p = 0; p < RP; ++p) acc[p] = wave_sum(acc[p]);
        if (lane == 0) {
            for (int p = 0; p < r; ++p) out[(int64_t)p * M + row] = acc[p];
        }
    }
}

// ------------------------------------------------ H_b = G x_{j != mode} B_j
// For every column of a block (or, with cidx == nullptr, every column of the
// full mode-`mode` unfolding), H[p][c] = sum over the other modes' core
// indices of G[..p..] * prod_j B_j[idx_j(c)][q_j].  G is held in LDS.
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_hexp(
    Prob P, const int2* __restrict__ tiles, const T* __restrict__ Bf,
    const double* __restrict__ Gd, T* __restrict__ H, DevState* st,
    int dense_mode, int64_t dense_cols) {
    if (st && stopped(st)) return;
    __shared__ double gs[kMaxCore];
    for (int e = threadIdx.x; e < P.core; e += kThreads) gs[e] = Gd[e];
    __syncthreads();
    const int2 tl = tiles[blockIdx.x];
    const bool dense = tl.x < 0;
    const int mode = dense ? dense_mode : P.blk[tl.x].mode;
    const int64_t ncols = dense ? dense_cols : P.blk[tl.x].ncols;
    const int64_t c = (int64_t)tl.y * kThreads + threadIdx.x;
    if (c >= ncols) return;
    const int n = P.n;
    int others[kMaxModes - 1];
    int no = 0;
    for (int j = 0; j < n; ++j)
        if (j != mode) others[no++] = j;
    // row of B_j used by this column, for each other mode
    int64_t rowoff[kMaxModes - 1];
    if (dense) {
        int64_t rem = c;
        for (int q = no - 1; q >= 0; --q) {
            const int j = others[q];
            rowoff[q] = P.boff[j] + (rem % P.d[j]) * RP;
            rem /= P.d[j];
        }
    } else {
        const BlockDev& bd = P.blk[tl.x];
        for (int q = 0; q < no; ++q)
            rowoff[q] = P.boff[others[q]] + (int64_t)bd.cidx[(int64_t)q * ncols + c] * RP;
    }
    // core strides (C order)
    int gstr[kMaxModes];
    gstr[n - 1] = 1;
    for (int j = n - 2; j >= 0; --j) gstr[j] = gstr[j + 1] * P.r[j + 1];
    double acc[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) acc[p] = 0.0;
    // odometer over the other modes' core indices
    int qi[kMaxModes - 1] = {0, 0, 0};
    const int rm = P.r[mode], sm = gstr[mode];
    while (true) {
        double prod = 1.0;
        int goff = 0;
        for (int q = 0; q < no; ++q) {
            prod *= (double)Bf[rowoff[q] + qi[q]];
            goff += qi[q] * gstr[others[q]];
        }
#pragma unroll
        for (int p = 0; p < RP; ++p)
            if (p < rm) acc[p] = fma(gs[goff + p * sm], prod, acc[p]);
        int q = no - 1;
        while (q >= 0 && ++qi[q] == P.r[others[q]]) {
            qi[q] = 0;
            --q;
        }
        if (q < 0) break;
    }
    const int64_t hoff = dense ? 0 : P.blk[tl.x].hoff;
#pragma unroll
    for (int p = 0; p < RP; ++p) H[hoff + (int64_t)p * ncols + c] = (T)acc[p];
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

// core G (float64, prod r_i) -> also unpack the support bitmask of a block
__global__ void k_unpack_mask(const uint64_t* __restrict__ mask, int64_t moff,
                              int words, int nrows, int ncols,
                              double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= (int64_t)nrows * ncols) return;
    const int x = (int)(e / ncols), c = (int)(e % ncols);
    const uint64_t wd = mask[moff + (int64_t)x * words + (c >> 6)];
    out[e] = ((wd >> (c & 63)) & 1ull) ? 1.0 : 0.0;
}

template <typename T>
__global__ void k_to_double(const T* __restrict__ in, int64_t N,
                            double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e < N) out[e] = (double)in[e];
}

}  // namespace rtcur
