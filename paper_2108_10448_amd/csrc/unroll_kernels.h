// Device kernels of the differentiable unrolled RTCUR-F (float64): K
// iterations of Algorithm 1 on one fixed chidori sample with per-iteration
// thresholds zeta_1..zeta_K, the L-update in its literal form (equations 8-9,
// A_i = C_i U_i^+, L = R x_i A_i on the blocks), and the hand-written adjoint
// of every step.  The threshold of equation 10 is replaced, for the
// derivative, by the gate S = D sigmoid((|D| / zeta - 1) / tau) (tau = 0:
// the hard threshold itself).
//
// Building blocks: a strided, batched GEMM on the float64 matrix cores; a
// cyclic Jacobi eigensolver for the s_i x s_i Grams (one workgroup per
// matrix, everything in LDS); mode-k unfold / fold of 3-mode tensors; the
// gate and its derivative; gathers and scatter-adds between the dense tensor
// and the block buffer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rtcur {
namespace ur {

constexpr int kT = 256;  // threads per workgroup (4 waves of 64)

typedef double v4d __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ GEMM
// C[b] = alpha op(A[b]) op(B[b]) + beta C[b] for b < gridDim.z, row-major:
//   op(A) (M x K): element (i, k) at A[b sa + (ta ? k lda + i : i lda + k)]
//   op(B) (K x N): element (k, j) at B[b sb + (tb ? j ldb + k : k ldb + j)]
//   C (M x N): element (i, j) at C[b sc + i ldc + j]
// beta = 0 never reads C.  A 32 x 32 tile of C per workgroup, one 16 x 16
// V_MFMA_F64_16X16X4 tile per wave, K staged through LDS 16 at a time (each
// operand tile loaded along its contiguous index).  Lane l feeds A row l%16
// at k = l/16 and B column l%16 at k = l/16; accumulator register v of lane
// l is row 4v + l/16, column l%16.
// With ksplit > 1 (long K, few output tiles): blockIdx.z = batch * ksplit +
// slice; the workgroup sums slice `slice` of K (kper columns, a multiple of
// 16) and writes its partial tile, alpha = 1 and beta = 0, to C + blockIdx.z
// * sc (the partial buffer); k_splitk_sum adds the slices in order.
__global__ __launch_bounds__(kT) void k_gemm(int M, int N, int K, double alpha,
                                             const double* __restrict__ A, int64_t lda,
                                             int64_t sa, int ta, const double* __restrict__ B,
                                             int64_t ldb, int64_t sb, int tb, double beta,
                                             double* __restrict__ C, int64_t ldc, int64_t sc,
                                             int ksplit, int kper) {
    __shared__ double As[32][17];
    __shared__ double Bs[16][33];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row0 = blockIdx.y * 32, col0 = blockIdx.x * 32;
    const int64_t bz = blockIdx.z / ksplit;
    const int slice = (int)(blockIdx.z % ksplit);
    const int kb = slice * kper, ke = min(K, kb + kper);
    A += bz * sa;
    B += bz * sb;
    C += (ksplit > 1 ? (int64_t)blockIdx.z : bz) * sc;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = tid + u * kT;  // 512 entries of each tile
            // A tile 32 x 16: along k when A is row-major, along i when transposed
            const int ai = ta ? (e & 31) : (e >> 4), ak = ta ? (e >> 5) : (e & 15);
            const int gi = row0 + ai, gk = k0 + ak;
            As[ai][ak] = (gi < M && gk < ke) ? A[ta ? (int64_t)gk * lda + gi : (int64_t)gi * lda + gk]
                                             : 0.0;
            // B tile 16 x 32: along j when B is row-major, along k when transposed
            const int bk = tb ? (e & 15) : (e >> 5), bj = tb ? (e >> 4) : (e & 31);
            const int hk = k0 + bk, hj = col0 + bj;
            Bs[bk][bj] = (hk < ke && hj < N) ? B[tb ? (int64_t)hj * ldb + hk : (int64_t)hk * ldb + hj]
                                             : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[16 * wr + (lane & 15)][4 * q + (lane >> 4)],
                                                       Bs[4 * q + (lane >> 4)][16 * wc + (lane & 15)],
                                                       acc, 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = row0 + 16 * wr + 4 * v + (lane >> 4), j = col0 + 16 * wc + (lane & 15);
        if (i < M && j < N) {
            double* c = C + (int64_t)i * ldc + j;
            *c = beta == 0.0 ? alpha * acc[v] : alpha * acc[v] + beta * *c;
        }
    }
}

// C = alpha sum_slice P[b * ksplit + slice] + beta C over batch x M x N, the
// slices added in order (P: M x N per slice, contiguous).
__global__ __launch_bounds__(kT) void k_splitk_sum(int M, int N, int batch, int ksplit,
                                                   const double* __restrict__ P, double alpha,
                                                   double beta, double* __restrict__ C,
                                                   int64_t ldc, int64_t sc) {
    const int64_t mn = (int64_t)M * N, tot = mn * batch;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * kT) {
        const int64_t b = e / mn, ij = e % mn;
        const int i = (int)(ij / N), j = (int)(ij % N);
        double v = 0.0;
        for (int q = 0; q < ksplit; ++q) v += P[(b * ksplit + q) * mn + ij];
        double* c = C + b * sc + (int64_t)i * ldc + j;
        *c = beta == 0.0 ? alpha * v : alpha * v + beta * *c;
    }
}

// ------------------------------------------------- 3-mode unfold and fold
// dir = 0: out = T_(k), the mode-k unfolding (d_k x the other two in C
// order) of the C-order tensor T (d0 x d1 x d2); dir = 1: the inverse.
__global__ __launch_bounds__(kT) void k_unfold3(const double* __restrict__ in,
                                                double* __restrict__ out, int d0, int d1, int d2,
                                                int k, int dir) {
    const int64_t n = (int64_t)d0 * d1 * d2;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kT) {
        const int64_t a = e / ((int64_t)d1 * d2), b = (e / d2) % d1, c = e % d2;  // tensor index
        int64_t u;                                                              // unfolded index
        if (k == 0) u = e;
        else if (k == 1) u = (b * d0 + a) * d2 + c;
        else u = (c * d0 + a) * d1 + b;
        if (dir == 0) out[u] = in[e];
        else out[e] = in[u];
    }
}

// ------------------------------------------------ gathers and scatters
// out[e] = X[idx[e]] (float64 or float32 X)
template <typename TX>
__global__ __launch_bounds__(kT) void k_gather_idx(const TX* __restrict__ X,
                                                   const int64_t* __restrict__ idx, int64_t n,
                                                   double* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kT)
        out[e] = (double)X[idx[e]];
}

// Xbar[idx[e]] += v[e] for the block entries, one block at a time (within a
// block every entry of X appears once, so no two threads of a launch touch
// the same address)
__global__ __launch_bounds__(kT) void k_scatter_add(const double* __restrict__ v,
                                                    const int64_t* __restrict__ idx, int64_t n,
                                                    double* __restrict__ Xbar) {
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kT)
        Xbar[idx[e]] += v[e];
}

// U (s x m) = rows I (s of them) of the d x m block C
__global__ __launch_bounds__(kT) void k_rows(const double* __restrict__ C,
                                             const int32_t* __restrict__ I, int s, int64_t m,
                                             double* __restrict__ U) {
    const int64_t n = (int64_t)s * m;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kT)
        U[e] = C[(int64_t)I[e / m] * m + e % m];
}

// rows I of the d x m block Cbar += Ubar (s x m); I has distinct entries
__global__ __launch_bounds__(kT) void k_rows_add(double* __restrict__ Cbar,
                                                 const int32_t* __restrict__ I, int s, int64_t m,
                                                 const double* __restrict__ Ubar) {
    const int64_t n = (int64_t)s * m;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kT)
        Cbar[(int64_t)I[e / m] * m + e % m] += Ubar[e];
}

// -------------------------------------------------------------- the gate
// phi(D) = HT_zeta(D) (tau = 0) or D sigmoid((|D| / zeta - 1) / tau), with
// its partial derivatives in D and zeta.
__device__ __forceinline__ void gate_eval(double D, double zeta, double tau, double& phi,
                                          double& dD, double& dz) {
    if (tau == 0.0) {
        const bool keep = fabs(D) > zeta;
        phi = keep ? D : 0.0;
        dD = keep ? 1.0 : 0.0;
        dz = 0.0;
        return;
    }
    const double ad = fabs(D);
    const double u = (ad / zeta - 1.0) / tau;
    const double sg = 1.0 / (1.0 + exp(-u));
    const double sp = sg * (1.0 - sg);  // sigmoid'(u)
    phi = D * sg;
    dD = sg + ad * sp / (zeta * tau);
    dz = -D * sp * ad / (zeta * zeta * tau);
}

// C = X - phi(X - L) on n block entries (L may be null: L = 0)
__global__ __launch_bounds__(kT) void k_gate_fwd(const double* __restrict__ X,
                                                 const double* __restrict__ L, int64_t n,
                                                 double zeta, double tau, double* __restrict__ C) {
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kT) {
        const double x = X[e];
        const double D = x - (L ? L[e] : 0.0);
        double phi, dD, dz;
        gate_eval(D, zeta, tau, phi, dD, dz);
        C[e] = x - phi;
    }
}

// Adjoint of C = X - phi(X - L): Xbar += Cbar (1 - phi_D); Lbar = Cbar phi_D
// (when Lbar is not null); per-workgroup partial sums of -Cbar phi_zeta
// into zpart[blockIdx.x], added in order by the host.
__global__ __launch_bounds__(kT) void k_gate_bwd(const double* __restrict__ X,
                                                 const double* __restrict__ L, int64_t n,
                                                 double zeta, double tau,
                                                 const double* __restrict__ Cbar,
                                                 double* __restrict__ Xbar,
                                                 double* __restrict__ Lbar,
                                                 double* __restrict__ zpart) {
    __shared__ double red[kT / 64];
    double zs = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kT) {
        const double D = X[e] - (L ? L[e] : 0.0);
        double phi, dD, dz;
        gate_eval(D, zeta, tau, phi, dD, dz);
        const double cb = Cbar[e];
        Xbar[e] += cb * (1.0 - dD);
        if (Lbar) Lbar[e] = cb * dD;
        zs -= cb * dz;
    }
    // fixed-order workgroup sum
    for (int o = 32; o > 0; o >>= 1) zs += __shfl_down(zs, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = zs;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kT / 64; ++q) t += red[q];
        zpart[blockIdx.x] = t;
    }
}

// ------------------------------------------------------- small elementwise
// y = a x + b y over n entries
__global__ __launch_bounds__(kT) void k_axpby(int64_t n, double a, const double* __restrict__ x,
                                              double b, double* __restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kT)
        y[e] = a * x[e] + (b == 0.0 ? 0.0 : b * y[e]);
}

// The truncated pseudo-inverse of the Gram, Gh = V_r diag(1 / lambda_r) V_r^T
// (s x s, V column-major eigenvectors in decreasing eigenvalue order:
// V[i * s + j] is component i of eigenvector j), and its symmetric gradient
// weights for the adjoint: F[j][k] of the divided differences of f(lambda)
// = 1 / lambda on the top r eigenvalues, 0 on the rest.
__global__ __launch_bounds__(kT) void k_ghat(const double* __restrict__ V,
                                             const double* __restrict__ lam, int s, int r,
                                             double* __restrict__ Gh) {
    for (int e = blockIdx.x * kT + threadIdx.x; e < s * s; e += gridDim.x * kT) {
        const int i = e / s, j = e % s;
        double v = 0.0;
        for (int p = 0; p < r; ++p) v += V[i * s + p] * V[j * s + p] / lam[p];
        Gh[e] = v;
    }
}

// W = F o ((W + W^T) / 2) in place on an s x s matrix given in the eigenbasis
// (W = V^T Xbar V): the Daleckii-Krein weights of f = 1/lambda on the top r
// eigenvalues (0 on the rest):
//   j, k < r:        -1 / (lambda_j lambda_k)
//   j < r <= k:       1 / (lambda_j (lambda_j - lambda_k))   (and symmetric)
//   j, k >= r:        0
// Symmetrising first is the adjoint of the symmetric perturbations dG.
__global__ __launch_bounds__(kT) void k_dk_weights(double* __restrict__ W,
                                                   const double* __restrict__ lam, int s, int r) {
    // each thread owns the pairs (j, k) with j <= k so the in-place update
    // of (j, k) and (k, j) is done by one thread
    for (int e = blockIdx.x * kT + threadIdx.x; e < s * s; e += gridDim.x * kT) {
        const int j = e / s, k = e % s;
        if (k < j) continue;
        const double sym = 0.5 * (W[j * s + k] + W[k * s + j]);
        double f;
        const bool jin = j < r, kin = k < r;
        if (jin && kin) f = -1.0 / (lam[j] * lam[k]);
        else if (jin) f = 1.0 / (lam[j] * (lam[j] - lam[k]));
        else if (kin) f = 1.0 / (lam[k] * (lam[k] - lam[j]));
        else f = 0.0;
        W[j * s + k] = f * sym;
        W[k * s + j] = f * sym;
    }
}

// Rank floor of the truncated SVD of U (s x m) read off the Gram's
// eigenvalues (decreasing): sigma_r <= max(s, m) 2^-52 sigma_1, i.e.
// lambda_r <= (max(s, m) 2^-52)^2 lambda_1 (or lambda_r <= 0), sets bit 1 of
// *flag; a non-finite eigenvalue sets bit 2.
__global__ void k_rank_check(const double* __restrict__ lam, int r, double smax, int* flag) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double l1 = lam[0], lr = lam[r - 1];
    if (!isfinite(l1) || !isfinite(lr)) {
        atomicOr(flag, 2);
        return;
    }
    const double f = smax * 0x1p-52;
    if (!(lr > 0.0) || lr <= f * f * l1) atomicOr(flag, 1);
}

// -------------------------------------------------------- Jacobi eigensolver
// Eigendecomposition of the symmetric s x s matrix G (s <= kJacMax) by
// cyclic Jacobi with the round-robin parallel ordering (n2/2 disjoint
// rotations per round, n2 = s rounded up to even, index n2-1 fixed when s is
// odd... every index meets every other once per sweep), one workgroup per
// matrix (blockIdx.x selects it), A and V in LDS.  A round applies its
// rotations in place, first to the rows of each pair, then to the columns
// (of A and V): the pairs are disjoint, so each work item reads and writes
// only its own two entries.  Sweeps stop when the off-diagonal mass is below
// 1e-30 of the diagonal's (squares) or after 40.
// Output: lam (s, decreasing) and V (s x s, V[i * s + j] = component i of
// eigenvector j, in the same order).
constexpr int kJacMax = 96;
constexpr int kJT = 512;  // threads of k_jacobi

__global__ __launch_bounds__(kJT) void k_jacobi(const double* __restrict__ Gall, int64_t gstride,
                                               int s, double* __restrict__ lam_all,
                                               int64_t lstride, double* __restrict__ V_all,
                                               int64_t vstride) {
    extern __shared__ double jsm[];
    const int ld = kJacMax + 1;
    double* A = jsm;                       // s x ld
    double* V = jsm + kJacMax * ld;        // s x ld
    __shared__ double jc[kJacMax], js[kJacMax];  // one round's rotations, per pair
    __shared__ int jp[kJacMax], jq[kJacMax], ord[kJacMax];
    __shared__ double red[2][kJT / 64];
    __shared__ int stop;
    const double* G = Gall + blockIdx.x * gstride;
    double* lam = lam_all + blockIdx.x * lstride;
    double* Vout = V_all + blockIdx.x * vstride;
    const int tid = threadIdx.x;
    const int n2 = s + (s & 1);
    for (int e = tid; e < s * s; e += kJT) {
        const int i = e / s, j = e % s;
        A[i * ld + j] = 0.5 * (G[i * s + j] + G[j * s + i]);
        V[i * ld + j] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int e = tid; e < s * s; e += kJT) {
            const int i = e / s, j = e % s;
            const double v = A[i * ld + j];
            if (i == j) dg += v * v;
            else off += v * v;
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_down(off, o, 64);
            dg += __shfl_down(dg, o, 64);
        }
        if ((tid & 63) == 0) {
            red[0][tid >> 6] = off;
            red[1][tid >> 6] = dg;
        }
        __syncthreads();
        if (tid == 0) {
            double a = 0.0, b = 0.0;
            for (int q = 0; q < kJT / 64; ++q) {
                a += red[0][q];
                b += red[1][q];
            }
            stop = !(a > 1e-30 * b);
        }
        __syncthreads();
        if (stop) break;
        for (int k = 0; k < n2 - 1; ++k) {
            if (tid < n2 / 2) {
                int p = n2 - 1, q = k;
                if (tid > 0) {
                    p = (k + tid) % (n2 - 1);
                    q = (k - tid + n2 - 1) % (n2 - 1);
                }
                double c = 1.0, sn = 0.0;
                if (p < s && q < s) {
                    const double app = A[p * ld + p], aqq = A[q * ld + q], apq = A[p * ld + q];
                    if (apq != 0.0) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                    }
                }
                // J[p][p] = J[q][q] = c, J[p][q] = sn, J[q][p] = -sn (the
                // identity for a pair with the padding index)
                const bool in = p < s && q < s;
                jp[tid] = in ? p : -1;
                jq[tid] = q;
                jc[tid] = c;
                js[tid] = sn;
            }
            __syncthreads();
            // A <- J^T A (the rows of each pair), then A <- A J and V <- V J
            // (its columns), in place: the pairs are disjoint, so each item
            // reads and writes only its own two entries
            const int npair = n2 / 2, items = npair * s;
            for (int e = tid; e < items; e += kJT) {
                const int t = e / s, j = e - t * s;
                const int p = jp[t];
                if (p < 0) continue;
                const int q = jq[t];
                const double c = jc[t], sn = js[t];
                const double a = A[p * ld + j], b = A[q * ld + j];
                A[p * ld + j] = c * a - sn * b;
                A[q * ld + j] = sn * a + c * b;
            }
            __syncthreads();
            for (int e = tid; e < items; e += kJT) {
                const int t = e / s, i = e - t * s;
                const int p = jp[t];
                if (p < 0) continue;
                const int q = jq[t];
                const double c = jc[t], sn = js[t];
                const double a = A[i * ld + p], b = A[i * ld + q];
                A[i * ld + p] = c * a - sn * b;
                A[i * ld + q] = sn * a + c * b;
                const double va = V[i * ld + p], vb = V[i * ld + q];
                V[i * ld + p] = c * va - sn * vb;
                V[i * ld + q] = sn * va + c * vb;
            }
            __syncthreads();
        }
    }
    // decreasing order (ties by index)
    if (tid < s) {
        const double t = A[tid * ld + tid];
        int rank = 0;
        for (int k = 0; k < s; ++k) {
            const double u = A[k * ld + k];
            rank += (u > t || (u == t && k < tid)) ? 1 : 0;
        }
        ord[rank] = tid;
    }
    __syncthreads();
    if (tid < s) lam[tid] = A[ord[tid] * ld + ord[tid]];
    for (int e = tid; e < s * s; e += kJT) {
        const int i = e / s, j = e % s;
        Vout[i * s + j] = V[i * ld + ord[j]];
    }
}

}  // namespace ur
}  // namespace rtcur
