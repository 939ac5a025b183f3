// Differentiable unrolled RTCUR-F on one gfx950 device (float64): the forward
// pass of K iterations of Algorithm 1 on a fixed chidori sample with given
// thresholds zeta_1..zeta_K (Section 3.2's schedule made an input), and the
// hand-written adjoint of those K iterations with respect to the thresholds
// and to X.  Three modes.
//
// Forward, iteration k (L^0 = 0):
//   C = X - phi(X - L^(k-1)) on every block (phi: the threshold of equation
//       10, or its gate D sigmoid((|D| / zeta_k - 1) / tau));
//   per mode i: U_i = C_i(I_i, :), G_i = U_i U_i^T = V diag(lambda) V^T
//       (Jacobi), Gh_i = V_r diag(1 / lambda_r) V_r^T, A_i = C_i U_i^T Gh_i
//       (= C_i U_i^+ of the rank-r_i truncation, equation 8);
//   L^k = R x_i A_i on the blocks (R = C on the core block; on R every factor
//       enters through its rows at I_i, on C_i factor i enters whole).
// Checkpoints, per iteration: R^k, A_i^k and the Grams' eigenpairs (the
// factor form of L^k; never a block-sized array), so the memory held grows
// with K only by the factors.
//
// Backward, k = K .. 1: L^(k-1) and C^k are recomputed from checkpoint k-1;
// then, in reverse order, the adjoints of the evaluation L = R x_i A_i, of
// A_i = C_i U_i^T Gh_i, of Gh_i as a spectral function of G_i (the
// Daleckii-Krein divided differences of f = 1/lambda on the top r
// eigenvalues), of G_i = U_i U_i^T, and of the threshold step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "unroll_kernels.h"

using namespace rtcur::ur;

struct rtcur_unroll_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    int d[3], r[3], s[3];
    int64_t m[3], NR = 0, N = 0, off[4], nb[4];
    int K = 0;
    uint64_t seed = 0;
    bool have_forward = false;
    double tau = 0.0;
    std::vector<double> zetas;
    // device memory: one arena
    void* arena = nullptr;
    int64_t* idx = nullptr;      // X offset of every block entry
    int32_t* I[3] = {nullptr, nullptr, nullptr};
    double *XB = nullptr, *LB = nullptr, *CB = nullptr, *LbarB = nullptr, *CbarB = nullptr,
           *XbarB = nullptr;
    double *ck = nullptr;        // K checkpoints
    int64_t ck_stride = 0, ck_A[3], ck_V[3], ck_lam[3];
    double *T1 = nullptr, *T2 = nullptr, *T3 = nullptr, *T4 = nullptr, *T5 = nullptr;
    double *U = nullptr, *Mm = nullptr, *Mbar = nullptr, *Ubar = nullptr;
    double *G = nullptr, *Gh = nullptr, *Wa = nullptr, *Wb = nullptr, *Gbar = nullptr;
    double *At[3] = {nullptr, nullptr, nullptr}, *Atb[3] = {nullptr, nullptr, nullptr},
           *Ab[3] = {nullptr, nullptr, nullptr};
    double *Rbar = nullptr, *zpart = nullptr;
    int* flag = nullptr;         // rank-test status of the forward pass
    double* sk = nullptr;        // split-K partial tiles (grown on demand)
    size_t sk_bytes = 0;
    int nzp = 0;
    std::vector<double> zhost;
};

namespace {

#define UCHK(expr)                                                                  \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) {                                                     \
            u->last_error = std::string(#expr) + ": " + hipGetErrorString(e_);      \
            return RTCUR_E_HIP;                                                     \
        }                                                                           \
    } while (0)

int ufail(rtcur_unroll_s* u, int st, const char* msg) {
    if (u) u->last_error = msg;
    return st;
}

unsigned grid_for(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kT - 1) / kT));
}

// C = alpha op(A) op(B) + beta C (see k_gemm), optionally batched.  A long
// K over few output tiles is split into slices (about 512 workgroups in all,
// at least 256 columns each) whose partial tiles k_splitk_sum adds in order.
int gemm(rtcur_unroll_s* u, int M, int N, int Kd, double alpha, const double* A, int64_t lda,
         bool ta, const double* B, int64_t ldb, bool tb, double beta, double* C, int64_t ldc,
         int batch = 1, int64_t sa = 0, int64_t sb = 0, int64_t sc = 0) {
    if (M <= 0 || N <= 0) return 0;
    const int64_t tiles = (int64_t)((N + 31) / 32) * ((M + 31) / 32) * batch;
    int ksplit = 1;
    if (tiles < 256 && Kd >= 512)
        ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(Kd / 256, 512 / tiles));
    const int kper = ksplit > 1 ? ((Kd + ksplit - 1) / ksplit + 15) / 16 * 16 : Kd;
    if (ksplit > 1) ksplit = (Kd + kper - 1) / kper;  // (no empty slice)
    if (ksplit > 1) {
        const size_t need = sizeof(double) * (size_t)M * N * batch * ksplit;
        if (need > u->sk_bytes) {
            if (u->sk) {
                UCHK(hipStreamSynchronize(u->stream));  // (earlier slices may still read it)
                UCHK(hipFree(u->sk));
            }
            u->sk = nullptr;
            u->sk_bytes = 0;
            if (hipMalloc(reinterpret_cast<void**>(&u->sk), need) != hipSuccess) {
                (void)hipGetLastError();
                return ufail(u, RTCUR_E_NOMEM, "split-K workspace allocation failed");
            }
            u->sk_bytes = need;
        }
        dim3 grid((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32),
                  (unsigned)(batch * ksplit));
        hipLaunchKernelGGL(k_gemm, grid, dim3(kT), 0, u->stream, M, N, Kd, 1.0, A, lda, sa,
                           ta ? 1 : 0, B, ldb, sb, tb ? 1 : 0, 0.0, u->sk, (int64_t)N,
                           (int64_t)M * N, ksplit, kper);
        UCHK(hipGetLastError());
        hipLaunchKernelGGL(k_splitk_sum, dim3(grid_for((int64_t)M * N * batch)), dim3(kT), 0,
                           u->stream, M, N, batch, ksplit, (const double*)u->sk, alpha, beta, C,
                           ldc, sc);
        UCHK(hipGetLastError());
        return 0;
    }
    dim3 grid((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32), (unsigned)batch);
    hipLaunchKernelGGL(k_gemm, grid, dim3(kT), 0, u->stream, M, N, Kd, alpha, A, lda, sa,
                       ta ? 1 : 0, B, ldb, sb, tb ? 1 : 0, beta, C, ldc, sc, 1, Kd);
    UCHK(hipGetLastError());
    return 0;
}

// out = T x_k Mat (Mat: s_k x s_k, or its transpose when tr) on the
// s0 x s1 x s2 tensors of the core block
int mode_product(rtcur_unroll_s* u, const double* T, const double* Mat, int k, bool tr,
                 double* out) {
    const int s0 = u->s[0], s1 = u->s[1], s2 = u->s[2];
    if (k == 0)
        return gemm(u, s0, s1 * s2, s0, 1.0, Mat, s0, tr, T, (int64_t)s1 * s2, false, 0.0, out,
                    (int64_t)s1 * s2);
    if (k == 1)
        return gemm(u, s1, s2, s1, 1.0, Mat, s1, tr, T, s2, false, 0.0, out, s2, s0, 0,
                    (int64_t)s1 * s2, (int64_t)s1 * s2);
    // (s0 s1 x s2) x Mat^T
    return gemm(u, s0 * s1, s2, s2, 1.0, T, s2, false, Mat, s2, !tr, 0.0, out, s2);
}

int unfold(rtcur_unroll_s* u, const double* in, double* out, int k, int dir) {
    hipLaunchKernelGGL(k_unfold3, dim3(grid_for(u->NR)), dim3(kT), 0, u->stream, in, out,
                       u->s[0], u->s[1], u->s[2], k, dir);
    UCHK(hipGetLastError());
    return 0;
}

// P (s_j x s_j) += unfold_j(X) unfold_j(Y)^T (X, Y: core-block tensors);
// uses T4, T5
int unfold_product(rtcur_unroll_s* u, const double* X, const double* Y, int j, double* P) {
    const int sj = u->s[j];
    const int64_t kk = u->NR / sj;
    const double *Xu = X, *Yu = Y;
    int rc;
    if (j != 0) {
        if ((rc = unfold(u, X, u->T4, j, 0)) || (rc = unfold(u, Y, u->T5, j, 0))) return rc;
        Xu = u->T4;
        Yu = u->T5;
    }
    return gemm(u, sj, sj, (int)kk, 1.0, Xu, kk, false, Yu, kk, true, 1.0, P, sj);
}

// rows I_i of a d_i x w matrix into an s_i x w one
int rows(rtcur_unroll_s* u, const double* C, int i, int64_t w, double* out) {
    hipLaunchKernelGGL(k_rows, dim3(grid_for(u->s[i] * w)), dim3(kT), 0, u->stream, C, u->I[i],
                       u->s[i], w, out);
    UCHK(hipGetLastError());
    return 0;
}

int rows_add(rtcur_unroll_s* u, double* C, int i, int64_t w, const double* add) {
    hipLaunchKernelGGL(k_rows_add, dim3(grid_for(u->s[i] * w)), dim3(kT), 0, u->stream, C,
                       u->I[i], u->s[i], w, add);
    UCHK(hipGetLastError());
    return 0;
}

int axpby(rtcur_unroll_s* u, int64_t n, double a, const double* x, double b, double* y) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kT), 0, u->stream, n, a, x, b, y);
    UCHK(hipGetLastError());
    return 0;
}

int zero(rtcur_unroll_s* u, double* y, int64_t n) { return axpby(u, n, 0.0, y, 0.0, y); }

double* ck_R(rtcur_unroll_s* u, int k) { return u->ck + (int64_t)(k - 1) * u->ck_stride; }
double* ck_A(rtcur_unroll_s* u, int k, int i) { return ck_R(u, k) + u->ck_A[i]; }
double* ck_V(rtcur_unroll_s* u, int k, int i) { return ck_R(u, k) + u->ck_V[i]; }
double* ck_lam(rtcur_unroll_s* u, int k, int i) { return ck_R(u, k) + u->ck_lam[i]; }

// the others of mode i, increasing
void others(int i, int& j1, int& j2) {
    j1 = i == 0 ? 1 : 0;
    j2 = i == 2 ? 1 : 2;
}

// L on every block from checkpoint k (R^k, A_i^k) into LB; leaves the rows
// At_j = A_j(I_j, :)
int evaluate(rtcur_unroll_s* u, int k) {
    int rc;
    const double* R = ck_R(u, k);
    for (int j = 0; j < 3; ++j)
        if ((rc = rows(u, ck_A(u, k, j), j, u->s[j], u->At[j]))) return rc;
    // L on R: R x_0 At_0 x_1 At_1 x_2 At_2
    if ((rc = mode_product(u, R, u->At[0], 0, false, u->T1)) ||
        (rc = mode_product(u, u->T1, u->At[1], 1, false, u->T2)) ||
        (rc = mode_product(u, u->T2, u->At[2], 2, false, u->LB + u->off[0])))
        return rc;
    // L on C_i: A_i unfold_i(R x_j1 At_j1 x_j2 At_j2)
    for (int i = 0; i < 3; ++i) {
        int j1, j2;
        others(i, j1, j2);
        if ((rc = mode_product(u, R, u->At[j1], j1, false, u->T1)) ||
            (rc = mode_product(u, u->T1, u->At[j2], j2, false, u->T2)))
            return rc;
        const double* Phi = u->T2;
        if (i != 0) {
            if ((rc = unfold(u, u->T2, u->T3, i, 0))) return rc;
            Phi = u->T3;
        }
        if ((rc = gemm(u, u->d[i], (int)u->m[i], u->s[i], 1.0, ck_A(u, k, i), u->s[i], false, Phi,
                       u->m[i], false, 0.0, u->LB + u->off[1 + i], u->m[i])))
            return rc;
    }
    return 0;
}

int gate_fwd(rtcur_unroll_s* u, int k) {
    hipLaunchKernelGGL(k_gate_fwd, dim3(grid_for(u->N)), dim3(kT), 0, u->stream, u->XB,
                       k > 1 ? (const double*)u->LB : nullptr, u->N, u->zetas[k - 1], u->tau,
                       u->CB);
    UCHK(hipGetLastError());
    return 0;
}

// The Grams' eigenpairs of C^k (into checkpoint k) and A_i^k = C_i U_i^T Gh_i
int lupdate(rtcur_unroll_s* u, int k) {
    int rc;
    for (int i = 0; i < 3; ++i) {
        const int s = u->s[i];
        const int64_t m = u->m[i];
        double* Ci = u->CB + u->off[1 + i];
        if ((rc = rows(u, Ci, i, m, u->U))) return rc;
        // G_i = U U^T into the i-th Gram slot (kJacMax^2 apart)
        if ((rc = gemm(u, s, s, (int)m, 1.0, u->U, m, false, u->U, m, true, 0.0,
                       u->G + (int64_t)i * kJacMax * kJacMax, s)))
            return rc;
    }
    // From the second iteration on, each Gram is first expressed in the
    // previous iteration's eigenbasis (V^T G V, nearly diagonal: the Grams
    // change little from one iteration to the next), so that the Jacobi
    // sweeps start from a nearly diagonal matrix and stop after a few; the
    // eigenvectors are rotated back afterwards.  Same eigenpairs up to
    // rounding.
    const bool warm = k >= 2;
    if (warm) {
        for (int i = 0; i < 3; ++i) {
            const int s = u->s[i];
            double* Gi = u->G + (int64_t)i * kJacMax * kJacMax;
            const double* Vp = ck_V(u, k - 1, i);
            if ((rc = gemm(u, s, s, s, 1.0, Gi, s, false, Vp, s, false, 0.0, u->Wa, s)) ||
                (rc = gemm(u, s, s, s, 1.0, Vp, s, true, u->Wa, s, false, 0.0, Gi, s)))
                return rc;
        }
    }
    // one workgroup per mode (equal s: one launch; else one per mode)
    const size_t lds = sizeof(double) * 2 * kJacMax * (kJacMax + 1);
    const bool same = u->s[0] == u->s[1] && u->s[1] == u->s[2];
    for (int i = 0; i < 3; i += same ? 3 : 1) {
        const int nm = same ? 3 : 1;
        // eigenpairs straight into checkpoint k (slots kJacMax^2 and kJacMax
        // apart; one launch covers the three modes when their sizes agree)
        hipLaunchKernelGGL(k_jacobi, dim3(nm), dim3(kJT), lds, u->stream,
                           u->G + (int64_t)i * kJacMax * kJacMax, (int64_t)kJacMax * kJacMax,
                           u->s[i], ck_lam(u, k, i), (int64_t)kJacMax, ck_V(u, k, i),
                           (int64_t)kJacMax * kJacMax);
        UCHK(hipGetLastError());
    }
    if (warm) {
        for (int i = 0; i < 3; ++i) {
            const int s = u->s[i];
            double* Vk = ck_V(u, k, i);
            if ((rc = gemm(u, s, s, s, 1.0, ck_V(u, k - 1, i), s, false, Vk, s, false, 0.0, u->Wb,
                           s)))
                return rc;
            UCHK(hipMemcpyAsync(Vk, u->Wb, sizeof(double) * s * s, hipMemcpyDeviceToDevice,
                                u->stream));
        }
    }
    for (int i = 0; i < 3; ++i) {
        const int s = u->s[i];
        const int64_t m = u->m[i];
        double* Ci = u->CB + u->off[1 + i];
        hipLaunchKernelGGL(k_ghat, dim3(grid_for((int64_t)s * s)), dim3(kT), 0, u->stream,
                           ck_V(u, k, i), ck_lam(u, k, i), s, u->r[i], u->Gh);
        UCHK(hipGetLastError());
        // rank floor of the truncated SVD: lambda_r <= (max(s, m) eps)^2 lambda_1
        hipLaunchKernelGGL(k_rank_check, dim3(1), dim3(64), 0, u->stream, ck_lam(u, k, i),
                           u->r[i], std::max<double>(s, (double)m), u->flag);
        UCHK(hipGetLastError());
        if ((rc = rows(u, Ci, i, m, u->U))) return rc;
        // M = U^T Gh (m x s), A = C_i M (d x s)
        if ((rc = gemm(u, (int)m, s, s, 1.0, u->U, m, true, u->Gh, s, false, 0.0, u->Mm, s)) ||
            (rc = gemm(u, u->d[i], s, (int)m, 1.0, Ci, m, false, u->Mm, s, false, 0.0,
                       ck_A(u, k, i), s)))
            return rc;
    }
    // R^k = C on the core block
    UCHK(hipMemcpyAsync(ck_R(u, k), u->CB + u->off[0], sizeof(double) * u->NR,
                        hipMemcpyDeviceToDevice, u->stream));
    return 0;
}

// Adjoint of one block's evaluation F unfold_i(R x_j1 At_j1 x_j2 At_j2)
// (rowsF x m_i) given its upstream Gb: Fbar += Gb Phi^T, and the
// contributions to Rbar and to Atb_j1, Atb_j2.  Checkpoint k's R.
int eval_adjoint_block(rtcur_unroll_s* u, int k, int i, const double* F, int rowsF, double* Fbar,
                       const double* Gb) {
    int rc;
    int j1, j2;
    others(i, j1, j2);
    const double* R = ck_R(u, k);
    const int si = u->s[i];
    const int64_t mi = u->m[i];
    if ((rc = mode_product(u, R, u->At[j1], j1, false, u->T1)) ||
        (rc = mode_product(u, u->T1, u->At[j2], j2, false, u->T2)))
        return rc;
    const double* Phi = u->T2;
    if (i != 0) {
        if ((rc = unfold(u, u->T2, u->T3, i, 0))) return rc;
        Phi = u->T3;
    }
    // Fbar += Gb Phi^T; Phibar = F^T Gb (into T3 unfolded), Ybar = fold_i
    if ((rc = gemm(u, rowsF, si, (int)mi, 1.0, Gb, mi, false, Phi, mi, true, 1.0, Fbar, si)))
        return rc;
    double* Ybar = u->T2;  // T2 (Y) is no longer needed
    if (i == 0) {
        if ((rc = gemm(u, si, (int)mi, rowsF, 1.0, F, si, true, Gb, mi, false, 0.0, Ybar, mi)))
            return rc;
    } else {
        if ((rc = gemm(u, si, (int)mi, rowsF, 1.0, F, si, true, Gb, mi, false, 0.0, u->T3, mi)) ||
            (rc = unfold(u, u->T3, Ybar, i, 1)))
            return rc;
    }
    // Y = T1 x_j2 At_j2: Atb_j2 += unfold_j2(Ybar) unfold_j2(T1)^T,
    // T1bar = Ybar x_j2 At_j2^T
    if ((rc = unfold_product(u, Ybar, u->T1, j2, u->Atb[j2])) ||
        (rc = mode_product(u, Ybar, u->At[j2], j2, true, u->T3)))
        return rc;
    // T1 = R x_j1 At_j1: Atb_j1 += unfold_j1(T1bar) unfold_j1(R)^T,
    // Rbar += T1bar x_j1 At_j1^T
    if ((rc = unfold_product(u, u->T3, R, j1, u->Atb[j1])) ||
        (rc = mode_product(u, u->T3, u->At[j1], j1, true, u->T1)) ||
        (rc = axpby(u, u->NR, 1.0, u->T1, 1.0, u->Rbar)))
        return rc;
    return 0;
}

int release(rtcur_unroll_s* u) {
    if (u->arena) (void)hipFree(u->arena);
    u->arena = nullptr;
    if (u->sk) (void)hipFree(u->sk);
    u->sk = nullptr;
    u->sk_bytes = 0;
    return 0;
}

}  // namespace

extern "C" {

int rtcur_unroll_create(rtcur_unroll_t* out, int device, void* hip_stream, int32_t n,
                        const int64_t* dims, const int32_t* ranks, const int64_t* I_sizes,
                        int32_t K, uint64_t seed) {
    if (!out) return RTCUR_E_INVAL;
    *out = nullptr;
    if (n != 3 || !dims || !ranks || !I_sizes || K < 1 || K > 1000) return RTCUR_E_INVAL;
    for (int i = 0; i < 3; ++i) {
        if (dims[i] < 1 || dims[i] > (1 << 20) || ranks[i] < 1 || I_sizes[i] < ranks[i] ||
            I_sizes[i] > dims[i] || I_sizes[i] > kJacMax)
            return RTCUR_E_INVAL;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return RTCUR_E_HIP;
    if (device < 0 || device >= count) return RTCUR_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return RTCUR_E_HIP;
    rtcur_unroll_s* u = new (std::nothrow) rtcur_unroll_s();
    if (!u) return RTCUR_E_NOMEM;
    u->device = device;
    u->stream = static_cast<hipStream_t>(hip_stream);
    u->K = K;
    u->seed = seed;
    rtcur::Shape sh;
    sh.n = 3;
    sh.chidori = true;
    for (int i = 0; i < 3; ++i) {
        u->d[i] = (int)dims[i];
        u->r[i] = ranks[i];
        u->s[i] = (int)I_sizes[i];
        sh.d[i] = dims[i];
        sh.r[i] = ranks[i];
        sh.s[i] = I_sizes[i];
    }
    for (int i = 0; i < 3; ++i) {
        int j1, j2;
        others(i, j1, j2);
        u->m[i] = (int64_t)u->s[j1] * u->s[j2];
        sh.m[i] = u->m[i];
    }
    u->NR = (int64_t)u->s[0] * u->s[1] * u->s[2];
    u->off[0] = 0;
    u->nb[0] = u->NR;
    int64_t N = u->NR;
    for (int i = 0; i < 3; ++i) {
        u->off[1 + i] = N;
        u->nb[1 + i] = (int64_t)u->d[i] * u->m[i];
        N += u->nb[1 + i];
    }
    u->N = N;
    // the sample (resample counter 0) and every block entry's X offset
    rtcur::SampleHost smp;
    std::vector<int64_t> idx;
    try {
        rtcur::draw_sample(seed, 0, sh, true, smp, true);
        idx.resize((size_t)N);
    } catch (...) {
        delete u;
        return RTCUR_E_NOMEM;
    }
    const int64_t xs[3] = {(int64_t)u->d[1] * u->d[2], (int64_t)u->d[2], 1};
    {
        int64_t e = 0;
        for (int a = 0; a < u->s[0]; ++a)
            for (int b = 0; b < u->s[1]; ++b)
                for (int c = 0; c < u->s[2]; ++c)
                    idx[(size_t)e++] = smp.I[0][a] * xs[0] + smp.I[1][b] * xs[1] + smp.I[2][c];
        for (int i = 0; i < 3; ++i) {
            int j1, j2;
            others(i, j1, j2);
            for (int x = 0; x < u->d[i]; ++x)
                for (int64_t c = 0; c < u->m[i]; ++c) {
                    const int32_t* t = &smp.Jtup[i][(size_t)c * 2];
                    idx[(size_t)e++] = x * xs[i] + t[0] * xs[j1] + t[1] * xs[j2];
                }
        }
    }
    // arena
    int64_t smax = std::max(u->s[0], std::max(u->s[1], u->s[2]));
    int64_t dmax = std::max(u->d[0], std::max(u->d[1], u->d[2]));
    int64_t mmax = std::max(u->m[0], std::max(u->m[1], u->m[2]));
    // one checkpoint: R, A_i, V_i (s_i^2, kJacMax^2 apart), lambda_i
    u->ck_A[0] = u->NR;
    for (int i = 1; i < 3; ++i) u->ck_A[i] = u->ck_A[i - 1] + (int64_t)u->d[i - 1] * u->s[i - 1];
    u->ck_V[0] = u->ck_A[2] + (int64_t)u->d[2] * u->s[2];
    for (int i = 1; i < 3; ++i) u->ck_V[i] = u->ck_V[i - 1] + (int64_t)kJacMax * kJacMax;
    u->ck_lam[0] = u->ck_V[2] + (int64_t)kJacMax * kJacMax;
    for (int i = 1; i < 3; ++i) u->ck_lam[i] = u->ck_lam[i - 1] + kJacMax;
    u->ck_stride = (u->ck_lam[2] + kJacMax + 31) / 32 * 32;
    u->nzp = (int)grid_for(N);
    size_t total = 0;
    auto take = [&](size_t bytes) {
        size_t o = total;
        total += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_idx = take(sizeof(int64_t) * N);
    size_t o_I[3];
    for (int i = 0; i < 3; ++i) o_I[i] = take(sizeof(int32_t) * u->s[i]);
    const size_t o_blk = take(sizeof(double) * N * 6);
    const size_t o_ck = take(sizeof(double) * u->ck_stride * K);
    const size_t o_t = take(sizeof(double) * u->NR * 5);
    const size_t o_u = take(sizeof(double) * smax * mmax * 2 + sizeof(double) * mmax * smax * 2);
    const size_t o_g = take(sizeof(double) * 3 * kJacMax * kJacMax);
    const size_t o_s = take(sizeof(double) * kJacMax * kJacMax * 4);
    const size_t o_a = take(sizeof(double) * (smax * smax * 6 + dmax * smax * 3));
    const size_t o_r = take(sizeof(double) * u->NR);
    const size_t o_z = take(sizeof(double) * u->nzp);
    const size_t o_f = take(sizeof(int) * 4);
    if (hipMalloc(&u->arena, total) != hipSuccess) {
        (void)hipGetLastError();
        delete u;
        return RTCUR_E_NOMEM;
    }
    char* a = static_cast<char*>(u->arena);
    u->idx = reinterpret_cast<int64_t*>(a + o_idx);
    for (int i = 0; i < 3; ++i) u->I[i] = reinterpret_cast<int32_t*>(a + o_I[i]);
    double* blk = reinterpret_cast<double*>(a + o_blk);
    u->XB = blk;
    u->LB = blk + N;
    u->CB = blk + 2 * N;
    u->LbarB = blk + 3 * N;
    u->CbarB = blk + 4 * N;
    u->XbarB = blk + 5 * N;
    u->ck = reinterpret_cast<double*>(a + o_ck);
    double* t = reinterpret_cast<double*>(a + o_t);
    u->T1 = t;
    u->T2 = t + u->NR;
    u->T3 = t + 2 * u->NR;
    u->T4 = t + 3 * u->NR;
    u->T5 = t + 4 * u->NR;
    double* uu = reinterpret_cast<double*>(a + o_u);
    u->U = uu;
    u->Ubar = uu + smax * mmax;
    u->Mm = uu + 2 * smax * mmax;
    u->Mbar = uu + 3 * smax * mmax;
    u->G = reinterpret_cast<double*>(a + o_g);
    double* sq = reinterpret_cast<double*>(a + o_s);
    u->Gh = sq;
    u->Wa = sq + kJacMax * kJacMax;
    u->Wb = sq + 2 * kJacMax * kJacMax;
    u->Gbar = sq + 3 * kJacMax * kJacMax;
    double* aa = reinterpret_cast<double*>(a + o_a);
    for (int i = 0; i < 3; ++i) {
        u->At[i] = aa + (2 * i) * smax * smax;
        u->Atb[i] = aa + (2 * i + 1) * smax * smax;
        u->Ab[i] = aa + 6 * smax * smax + i * dmax * smax;
    }
    u->Rbar = reinterpret_cast<double*>(a + o_r);
    u->zpart = reinterpret_cast<double*>(a + o_z);
    u->flag = reinterpret_cast<int*>(a + o_f);
    // uploads (synchronous: the host vectors are pageable and die here)
    int rc = RTCUR_OK;
    if (hipMemcpy(u->idx, idx.data(), sizeof(int64_t) * N, hipMemcpyHostToDevice) != hipSuccess)
        rc = RTCUR_E_HIP;
    for (int i = 0; i < 3 && rc == RTCUR_OK; ++i) {
        std::vector<int32_t> Ii(smp.I[i].begin(), smp.I[i].end());
        if (hipMemcpy(u->I[i], Ii.data(), sizeof(int32_t) * u->s[i], hipMemcpyHostToDevice) !=
            hipSuccess)
            rc = RTCUR_E_HIP;
    }
    const void* fn = reinterpret_cast<const void*>(k_jacobi);
    if (rc == RTCUR_OK &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * 2 * kJacMax * (kJacMax + 1))) != hipSuccess)
        rc = RTCUR_E_HIP;
    if (rc != RTCUR_OK) {
        (void)hipGetLastError();
        release(u);
        delete u;
        return rc;
    }
    *out = u;
    return RTCUR_OK;
}

int rtcur_unroll_destroy(rtcur_unroll_t u) {
    if (!u) return RTCUR_OK;
    (void)hipSetDevice(u->device);
    release(u);
    delete u;
    return RTCUR_OK;
}

int rtcur_unroll_blocks(rtcur_unroll_t u, int64_t* n_blk, int64_t* idx_out, int64_t cap) {
    if (!u) return RTCUR_E_INVAL;
    if (n_blk) *n_blk = u->N;
    if (!idx_out) return RTCUR_OK;
    if (cap < u->N) return ufail(u, RTCUR_E_INVAL, "index buffer too small");
    UCHK(hipSetDevice(u->device));
    UCHK(hipMemcpy(idx_out, u->idx, sizeof(int64_t) * u->N, hipMemcpyDeviceToHost));
    return RTCUR_OK;
}

int rtcur_unroll_forward(rtcur_unroll_t u, const void* X, int x_dtype, const double* zetas,
                         double tau, double* L_out) {
    if (!u) return RTCUR_E_INVAL;
    u->have_forward = false;
    if (!X || !zetas || !L_out) return ufail(u, RTCUR_E_INVAL, "null argument");
    if (x_dtype != RTCUR_F64 && x_dtype != RTCUR_F32)
        return ufail(u, RTCUR_E_INVAL, "x_dtype must be RTCUR_F64 or RTCUR_F32");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return ufail(u, RTCUR_E_INVAL, "tau must be >= 0");
    for (int k = 0; k < u->K; ++k)
        if (!(zetas[k] > 0.0) || !std::isfinite(zetas[k]))
            return ufail(u, RTCUR_E_INVAL, "thresholds must be positive and finite");
    UCHK(hipSetDevice(u->device));
    u->zetas.assign(zetas, zetas + u->K);
    u->tau = tau;
    int rc;
    if (x_dtype == RTCUR_F64)
        hipLaunchKernelGGL((k_gather_idx<double>), dim3(grid_for(u->N)), dim3(kT), 0, u->stream,
                           (const double*)X, u->idx, u->N, u->XB);
    else
        hipLaunchKernelGGL((k_gather_idx<float>), dim3(grid_for(u->N)), dim3(kT), 0, u->stream,
                           (const float*)X, u->idx, u->N, u->XB);
    UCHK(hipGetLastError());
    UCHK(hipMemsetAsync(u->flag, 0, sizeof(int), u->stream));
    for (int k = 1; k <= u->K; ++k) {
        if ((rc = gate_fwd(u, k)) || (rc = lupdate(u, k)) || (rc = evaluate(u, k))) return rc;
    }
    UCHK(hipMemcpyAsync(L_out, u->LB, sizeof(double) * u->N, hipMemcpyDeviceToDevice, u->stream));
    int flag = 0;
    UCHK(hipMemcpyAsync(&flag, u->flag, sizeof(int), hipMemcpyDeviceToHost, u->stream));
    UCHK(hipStreamSynchronize(u->stream));
    if (flag & 2) return ufail(u, RTCUR_E_NONFINITE, "non-finite eigenvalue");
    if (flag & 1) return ufail(u, RTCUR_E_RANK, "U_i has numerical rank below r_i");
    u->have_forward = true;
    return RTCUR_OK;
}

int rtcur_unroll_backward(rtcur_unroll_t u, const double* L_bar, double* zeta_bar,
                          double* X_bar) {
    if (!u) return RTCUR_E_INVAL;
    if (!u->have_forward) return ufail(u, RTCUR_E_STATE, "no forward pass to differentiate");
    if (!L_bar || !zeta_bar || !X_bar) return ufail(u, RTCUR_E_INVAL, "null argument");
    UCHK(hipSetDevice(u->device));
    int rc;
    if ((rc = zero(u, u->XbarB, u->N))) return rc;
    UCHK(hipMemcpyAsync(u->LbarB, L_bar, sizeof(double) * u->N, hipMemcpyDeviceToDevice,
                        u->stream));
    u->zhost.assign((size_t)u->nzp, 0.0);
    for (int k = u->K; k >= 1; --k) {
        // L^(k-1) and C^k again (L^0 = 0)
        if (k > 1 && (rc = evaluate(u, k - 1))) return rc;
        if ((rc = gate_fwd(u, k))) return rc;
        // adjoint of L^k = R^k x_i A_i^k on the blocks
        for (int j = 0; j < 3; ++j) {
            if ((rc = rows(u, ck_A(u, k, j), j, u->s[j], u->At[j])) ||
                (rc = zero(u, u->Atb[j], (int64_t)u->s[j] * u->s[j])) ||
                (rc = zero(u, u->Ab[j], (int64_t)u->d[j] * u->s[j])))
                return rc;
        }
        if ((rc = zero(u, u->Rbar, u->NR))) return rc;
        if ((rc = eval_adjoint_block(u, k, 0, u->At[0], u->s[0], u->Atb[0], u->LbarB + u->off[0])))
            return rc;
        for (int i = 0; i < 3; ++i)
            if ((rc = eval_adjoint_block(u, k, i, ck_A(u, k, i), u->d[i], u->Ab[i],
                                         u->LbarB + u->off[1 + i])))
                return rc;
        for (int i = 0; i < 3; ++i)
            if ((rc = rows_add(u, u->Ab[i], i, u->s[i], u->Atb[i]))) return rc;
        // adjoint of A_i = C_i U_i^T Gh_i into Cbar (C_i blocks), Rbar into R's
        if ((rc = zero(u, u->CbarB, u->N))) return rc;
        for (int i = 0; i < 3; ++i) {
            const int s = u->s[i], d = u->d[i];
            const int64_t m = u->m[i];
            const double* V = ck_V(u, k, i);
            const double* lam = ck_lam(u, k, i);
            double* Ci = u->CB + u->off[1 + i];
            double* Cbi = u->CbarB + u->off[1 + i];
            hipLaunchKernelGGL(k_ghat, dim3(grid_for((int64_t)s * s)), dim3(kT), 0, u->stream, V,
                               lam, s, u->r[i], u->Gh);
            UCHK(hipGetLastError());
            if ((rc = rows(u, Ci, i, m, u->U)) ||
                // M = U^T Gh
                (rc = gemm(u, (int)m, s, s, 1.0, u->U, m, true, u->Gh, s, false, 0.0, u->Mm, s)) ||
                // Cbar_i += Abar M^T
                (rc = gemm(u, d, (int)m, s, 1.0, u->Ab[i], s, false, u->Mm, s, true, 1.0, Cbi, m)) ||
                // Mbar = C_i^T Abar
                (rc = gemm(u, (int)m, s, d, 1.0, Ci, m, true, u->Ab[i], s, false, 0.0, u->Mbar, s)) ||
                // Ubar = Gh Mbar^T
                (rc = gemm(u, s, (int)m, s, 1.0, u->Gh, s, false, u->Mbar, s, true, 0.0, u->Ubar, m)) ||
                // Ghbar = U Mbar (into Gbar)
                (rc = gemm(u, s, s, (int)m, 1.0, u->U, m, false, u->Mbar, s, false, 0.0, u->Gbar, s)) ||
                // W = V^T Ghbar V, weighted, Gbar = V W V^T
                (rc = gemm(u, s, s, s, 1.0, V, s, true, u->Gbar, s, false, 0.0, u->Wa, s)) ||
                (rc = gemm(u, s, s, s, 1.0, u->Wa, s, false, V, s, false, 0.0, u->Wb, s)))
                return rc;
            hipLaunchKernelGGL(k_dk_weights, dim3(grid_for((int64_t)s * s)), dim3(kT), 0, u->stream,
                               u->Wb, lam, s, u->r[i]);
            UCHK(hipGetLastError());
            if ((rc = gemm(u, s, s, s, 1.0, V, s, false, u->Wb, s, false, 0.0, u->Wa, s)) ||
                (rc = gemm(u, s, s, s, 1.0, u->Wa, s, false, V, s, true, 0.0, u->Gbar, s)) ||
                // G = U U^T: Ubar += (Gbar + Gbar^T) U = 2 Gbar U (Gbar symmetric)
                (rc = gemm(u, s, (int)m, s, 2.0, u->Gbar, s, false, u->U, m, false, 1.0, u->Ubar, m)) ||
                (rc = rows_add(u, Cbi, i, m, u->Ubar)))
                return rc;
        }
        if ((rc = axpby(u, u->NR, 1.0, u->Rbar, 1.0, u->CbarB + u->off[0]))) return rc;
        // adjoint of C = X - phi(X - L^(k-1)): Xbar, Lbar^(k-1), zeta_k's share
        hipLaunchKernelGGL(k_gate_bwd, dim3(u->nzp), dim3(kT), 0, u->stream, u->XB,
                           k > 1 ? (const double*)u->LB : nullptr, u->N, u->zetas[k - 1], u->tau,
                           u->CbarB, u->XbarB, k > 1 ? u->LbarB : nullptr, u->zpart);
        UCHK(hipGetLastError());
        UCHK(hipMemcpyAsync(u->zhost.data(), u->zpart, sizeof(double) * u->nzp,
                            hipMemcpyDeviceToHost, u->stream));
        UCHK(hipStreamSynchronize(u->stream));
        double z = 0.0;
        for (int q = 0; q < u->nzp; ++q) z += u->zhost[(size_t)q];
        zeta_bar[k - 1] = z;
    }
    // X's gradient: every block's share added at its entries (a block never
    // holds an entry of X twice)
    {
        int64_t total = (int64_t)u->d[0] * u->d[1] * u->d[2];
        if ((rc = zero(u, X_bar, total))) return rc;
        for (int b = 0; b < 4; ++b) {
            hipLaunchKernelGGL(k_scatter_add, dim3(grid_for(u->nb[b])), dim3(kT), 0, u->stream,
                               u->XbarB + u->off[b], u->idx + u->off[b], u->nb[b], X_bar);
            UCHK(hipGetLastError());
        }
    }
    UCHK(hipStreamSynchronize(u->stream));
    return RTCUR_OK;
}

const char* rtcur_unroll_last_error(rtcur_unroll_t u) {
    if (!u) return "null handle";
    return u->last_error.c_str();
}

}  // extern "C"
