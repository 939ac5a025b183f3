// extern "C" entry points of librtcur (declared in include/rtcur.h):
// argument validation, handle lifetime, status strings and host copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

using rtcur::Shape;

namespace {

int fail(rtcur_t h, int status, const char* msg) {
    if (h) h->last_error = msg;
    return status;
}

// Checks of the Algorithm 1 inputs; fills the shape.
int validate(rtcur_t h, int32_t n, const int64_t* dims, const int32_t* ranks,
             const int64_t* I_sizes, const int64_t* J_sizes, double gamma, double tol,
             int32_t max_iter, int x_dtype, Shape& sh) {
    if (n < 2 || n > rtcur::kMaxModes)
        return fail(h, RTCUR_E_INVAL, "number of modes must be 2..4");
    if (!dims || !ranks || !I_sizes) return fail(h, RTCUR_E_INVAL, "null size array");
    if (x_dtype != RTCUR_F64 && x_dtype != RTCUR_F32)
        return fail(h, RTCUR_E_INVAL, "x_dtype must be RTCUR_F64 or RTCUR_F32");
    if (!(gamma > 0.0 && gamma < 1.0)) return fail(h, RTCUR_E_INVAL, "gamma must lie in (0,1)");
    if (!(tol >= 0.0)) return fail(h, RTCUR_E_INVAL, "tol must be >= 0");
    if (max_iter < 1) return fail(h, RTCUR_E_INVAL, "max_iter must be >= 1");
    sh.n = n;
    sh.chidori = (J_sizes == nullptr);
    int64_t core = 1;
    for (int i = 0; i < n; ++i) {
        sh.d[i] = dims[i];
        sh.r[i] = ranks[i];
        sh.s[i] = I_sizes[i];
        if (dims[i] < 1 || dims[i] > (int64_t)1 << 30)
            return fail(h, RTCUR_E_INVAL, "dims out of range");
        if (ranks[i] < 1 || ranks[i] > rtcur::kMaxRank)
            return fail(h, RTCUR_E_INVAL, "ranks must be 1..16");
        if (I_sizes[i] < ranks[i] || I_sizes[i] > dims[i])
            return fail(h, RTCUR_E_INVAL, "need r_i <= |I_i| <= d_i");
        if (I_sizes[i] > rtcur::kMaxS) return fail(h, RTCUR_E_INVAL, "|I_i| must be <= 256");
        core *= ranks[i];
    }
    if (core > rtcur::kMaxCore) return fail(h, RTCUR_E_INVAL, "prod(r_i) must be <= 4096");
    {
        // one slice of the core, r_{n-1} x prod_{0 < l < n-1} |I_l|, fits in
        // LDS: 4096 entries with three modes (always, as r_2 <= 16 and
        // |I_1| <= 256), 2048 with four (whose next contraction also stays
        // in LDS)
        int64_t slice = ranks[n - 1];
        for (int l = 1; l < n - 1; ++l) slice *= I_sizes[l];
        if (slice > (n == 3 ? 4096 : 2048))
            return fail(h, RTCUR_E_INVAL, "sampled core slice too large");
    }
    int64_t total = 1;
    for (int i = 0; i < n; ++i) total *= sh.d[i];
    if (total > ((int64_t)1 << 40)) return fail(h, RTCUR_E_INVAL, "tensor too large");
    int64_t nblk = 1;
    for (int i = 1; i < n; ++i) nblk *= sh.s[i];
    nblk *= sh.s[0];
    for (int i = 0; i < n; ++i) {
        int64_t P = 1, m = 1;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            P *= sh.d[j];
            m *= sh.s[j];
        }
        if (J_sizes) m = J_sizes[i];
        if (m < ranks[i] || m > P) return fail(h, RTCUR_E_INVAL, "need r_i <= |J_i| <= prod of other dims");
        if (m > ((int64_t)1 << 31) - 1) return fail(h, RTCUR_E_INVAL, "|J_i| too large");
        sh.m[i] = m;
        nblk += sh.d[i] * m;
    }
    if (nblk > ((int64_t)1 << 36)) return fail(h, RTCUR_E_INVAL, "sampled blocks too large");
    return RTCUR_OK;
}

}  // namespace

extern "C" {

int rtcur_create(rtcur_t* out, int device, void* hip_stream, int variant, int compute_dtype) {
    if (!out) return RTCUR_E_INVAL;
    *out = nullptr;
    if (variant != RTCUR_FIXED && variant != RTCUR_RESAMPLE) return RTCUR_E_INVAL;
    if (compute_dtype != RTCUR_F64 && compute_dtype != RTCUR_F32 && compute_dtype != RTCUR_BF16)
        return RTCUR_E_INVAL;
    if (compute_dtype == RTCUR_BF16 && variant != RTCUR_FIXED) return RTCUR_E_INVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return RTCUR_E_HIP;
    if (device < 0 || device >= count) return RTCUR_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return RTCUR_E_HIP;
    // the device's static scratch (rtcur_reconstruct_noalloc), looked up once
    if (rtcur::static_scratch_init(device) != RTCUR_OK) return RTCUR_E_HIP;
    rtcur_t h = new (std::nothrow) rtcur_s();
    if (!h) return RTCUR_E_NOMEM;
    h->device = device;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->variant = variant;
    h->dtype = compute_dtype;
    *out = h;
    return RTCUR_OK;
}

int rtcur_solve(rtcur_t h, const void* X, int x_dtype, int32_t n, const int64_t* dims,
                const int32_t* ranks, const int64_t* I_sizes, const int64_t* J_sizes,
                double zeta0, double gamma, double tol, int32_t max_iter, uint64_t seed,
                rtcur_info* info) {
    if (!h) return RTCUR_E_INVAL;
    h->have_result = false;
    if (!X) return fail(h, RTCUR_E_INVAL, "X is null");
    if (std::isnan(zeta0) || std::isinf(zeta0)) return fail(h, RTCUR_E_INVAL, "zeta0 not finite");
    Shape sh;
    int rc = validate(h, n, dims, ranks, I_sizes, J_sizes, gamma, tol, max_iter, x_dtype, sh);
    if (rc != RTCUR_OK) {
        h->info.status = rc;
        if (info) *info = h->info;
        return rc;
    }
    const auto t0 = std::chrono::steady_clock::now();
    try {
        rc = rtcur::solve(h, X, x_dtype, sh, zeta0, gamma, tol, max_iter, seed);
    } catch (const std::bad_alloc&) {
        rc = fail(h, RTCUR_E_NOMEM, "host allocation failed");
    } catch (...) {
        rc = fail(h, RTCUR_E_STATE, "internal error");
    }
    if (rc < 0) {
        std::memset(&h->info, 0, sizeof(h->info));
        h->info.status = rc;
    }
    h->info.solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    h->info.batch_slot = -1;
    h->info.batch_seq = -1;
    if (info) *info = h->info;
    return rc;
}

int rtcur_reconstruct(rtcur_t h, void* L_out, int out_dtype) {
    if (!h) return RTCUR_E_INVAL;
    if (!L_out) return fail(h, RTCUR_E_INVAL, "L_out is null");
    if (out_dtype != RTCUR_F64 && out_dtype != RTCUR_F32)
        return fail(h, RTCUR_E_INVAL, "out_dtype must be RTCUR_F64 or RTCUR_F32");
    return rtcur::reconstruct(h, L_out, out_dtype);
}

int rtcur_reconstruct_noalloc(rtcur_t h, void* L_out, int out_dtype) {
    if (!h) return RTCUR_E_INVAL;
    if (!L_out) return fail(h, RTCUR_E_INVAL, "L_out is null");
    if (out_dtype != RTCUR_F64 && out_dtype != RTCUR_F32)
        return fail(h, RTCUR_E_INVAL, "out_dtype must be RTCUR_F64 or RTCUR_F32");
    try {
        return rtcur::reconstruct_noalloc(h, L_out, out_dtype);
    } catch (...) {
        return fail(h, RTCUR_E_STATE, "internal error");
    }
}

int rtcur_outliers(rtcur_t h, const void* X, int x_dtype, double zeta, void* S_out,
                   void* L_out, int out_dtype) {
    if (!h) return RTCUR_E_INVAL;
    if (!X || !S_out) return fail(h, RTCUR_E_INVAL, "X and S_out must not be null");
    if (x_dtype != RTCUR_F64 && x_dtype != RTCUR_F32)
        return fail(h, RTCUR_E_INVAL, "x_dtype must be RTCUR_F64 or RTCUR_F32");
    if (out_dtype != RTCUR_F64 && out_dtype != RTCUR_F32)
        return fail(h, RTCUR_E_INVAL, "out_dtype must be RTCUR_F64 or RTCUR_F32");
    if (!std::isfinite(zeta)) return fail(h, RTCUR_E_INVAL, "zeta must be finite");
    return rtcur::outliers(h, X, x_dtype, zeta, S_out, L_out, out_dtype);
}

// Solve times of batch instances, by problem: the batch queue's order.
static std::mutex g_batch_mu;
static std::map<std::vector<int64_t>, double> g_batch_ms;

static std::vector<int64_t> batch_key(rtcur_t h, int32_t j, int x_dtype, const int32_t* n,
                                      const int64_t* dims, const int32_t* ranks,
                                      const int64_t* I_sizes, const int64_t* J_sizes,
                                      double gamma, double tol, int32_t max_iter) {
    std::vector<int64_t> k = {h->dtype, h->variant, x_dtype, n[j], max_iter, J_sizes ? 1 : 0};
    int64_t tb, gb;
    std::memcpy(&tb, &tol, sizeof(tb));
    std::memcpy(&gb, &gamma, sizeof(gb));
    k.push_back(tb);
    k.push_back(gb);
    for (int32_t q = 0; q < n[j] && q < rtcur::kMaxModes; ++q) {
        const int64_t o = (int64_t)j * rtcur::kMaxModes + q;
        k.push_back(dims[o]);
        k.push_back(ranks[o]);
        k.push_back(I_sizes[o]);
        if (J_sizes) k.push_back(J_sizes[o]);
    }
    return k;
}

int rtcur_solve_batch(rtcur_t* hs, int32_t nh, int32_t count, const void* const* X,
                      int x_dtype, const int32_t* n, const int64_t* dims,
                      const int32_t* ranks, const int64_t* I_sizes, const int64_t* J_sizes,
                      const double* zeta0, double gamma, double tol, int32_t max_iter,
                      const uint64_t* seeds, void* const* L_out, int out_dtype,
                      rtcur_info* infos, int32_t* status) {
    if (!hs || nh < 1 || count < 0 || (count > 0 && (!X || !n || !dims || !ranks ||
                                                     !I_sizes || !seeds || !status)))
        return RTCUR_E_INVAL;
    if (L_out && out_dtype != RTCUR_F64 && out_dtype != RTCUR_F32) return RTCUR_E_INVAL;
    for (int32_t t = 0; t < nh; ++t) {
        if (!hs[t]) return RTCUR_E_INVAL;
        for (int32_t u = 0; u < t; ++u)
            if (hs[u] == hs[t]) return RTCUR_E_INVAL;  // one thread per handle
    }
    const int32_t nt = count < nh ? count : nh;
    // one work queue, longest first: instances in decreasing number of
    // entries (ties by index); each handle's thread takes the next one when
    // its previous solve has returned
    std::vector<int32_t> order;
    std::vector<std::thread> pool;
    std::vector<char> inline_list;
    std::atomic<int32_t> next{0};
    try {
        order.resize(count);
        inline_list.assign(nt > 0 ? nt : 0, 0);
        pool.reserve(nt > 1 ? nt - 1 : 0);
    } catch (...) {
        return RTCUR_E_NOMEM;
    }
    for (int32_t j = 0; j < count; ++j) order[j] = j;
    auto entries = [&](int32_t j) {
        double v = 1.0;
        for (int32_t q = 0; q < n[j] && q < rtcur::kMaxModes; ++q)
            v *= (double)dims[(int64_t)j * rtcur::kMaxModes + q];
        return v;
    };
    // expected cost, longest first: the solve times last measured in this
    // process for the same problem (sizes, ranks, sample sizes, the first
    // handle's compute dtype and variant, gamma, tol, max_iter) when every
    // instance has one, else the number of entries
    std::vector<std::vector<int64_t>> keys;
    std::vector<double> cost;
    try {
        keys.resize(count);
        cost.resize(count);
        for (int32_t j = 0; j < count; ++j)
            keys[j] = batch_key(hs[0], j, x_dtype, n, dims, ranks, I_sizes, J_sizes, gamma, tol,
                                max_iter);
        bool all = count > 0;
        {
            std::lock_guard<std::mutex> lk(g_batch_mu);
            for (int32_t j = 0; j < count; ++j) {
                auto it = g_batch_ms.find(keys[j]);
                if (it == g_batch_ms.end()) all = false;
                else cost[j] = it->second;
            }
        }
        if (!all)
            for (int32_t j = 0; j < count; ++j) cost[j] = entries(j);
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    } catch (...) {
        return RTCUR_E_NOMEM;  // before any solve started
    }
    auto work = [&](int32_t t) {
        for (int32_t seq = 0;; ++seq) {
            const int32_t q = next.fetch_add(1);
            if (q >= count) break;
            const int32_t j = order[q];
            const int64_t* Js = J_sizes ? J_sizes + (int64_t)j * rtcur::kMaxModes : nullptr;
            rtcur_info inf;
            std::memset(&inf, 0, sizeof(inf));
            int rc = rtcur_solve(hs[t], X[j], x_dtype, n[j], dims + (int64_t)j * rtcur::kMaxModes,
                                 ranks + (int64_t)j * rtcur::kMaxModes,
                                 I_sizes + (int64_t)j * rtcur::kMaxModes, Js,
                                 zeta0 ? zeta0[j] : 0.0, gamma, tol, max_iter, seeds[j], &inf);
            if (rc >= 0 && L_out && L_out[j]) {
                const int rr = rtcur_reconstruct(hs[t], L_out[j], out_dtype);
                if (rr != RTCUR_OK) rc = rr;
            }
            status[j] = rc;
            inf.batch_slot = t;
            inf.batch_seq = seq;
            if (infos) infos[j] = inf;
            if (rc >= 0) {
                try {
                    std::lock_guard<std::mutex> lk(g_batch_mu);
                    g_batch_ms[keys[j]] = inf.solve_ms;
                } catch (...) {
                    // (the cost record is an optimisation of the order only)
                }
            }
        }
    };
    // Handles whose thread cannot be started run their lists on the calling
    // thread; every started thread is joined before returning, whatever
    // happened, so no joinable std::thread is ever destroyed.
    for (int32_t t = 1; t < nt; ++t) {
        try {
            pool.emplace_back(work, t);
        } catch (...) {
            inline_list[t] = 1;
        }
    }
    if (nt > 0) inline_list[0] = 1;
    for (int32_t t = 0; t < nt; ++t)
        if (inline_list[t]) work(t);
    for (auto& th : pool) th.join();
    int rc = RTCUR_OK;
    for (int32_t j = 0; j < count; ++j)
        if (status[j] < 0) return status[j];
        else if (status[j] == RTCUR_NOT_CONVERGED) rc = RTCUR_NOT_CONVERGED;
    return rc;
}

int rtcur_autotune(rtcur_t h, const void* X, int x_dtype, int32_t n, const int64_t* dims,
                   const int32_t* ranks, const int64_t* I_sizes, const int64_t* J_sizes,
                   int32_t iters, int32_t reps, uint64_t seed, int32_t* tile,
                   double* tuned_ms, double* default_ms) {
    if (!h) return RTCUR_E_INVAL;
    if (!X || !tile) return fail(h, RTCUR_E_INVAL, "X and tile must not be null");
    if (iters < 1 || iters > 1000 || reps < 1 || reps > 100)
        return fail(h, RTCUR_E_INVAL, "iters must be in [1, 1000] and reps in [1, 100]");
    rtcur::Shape sh;
    int rc = validate(h, n, dims, ranks, I_sizes, J_sizes, 0.7, 0.0, iters, x_dtype, sh);
    if (rc != RTCUR_OK) return rc;
    rtcur::Tune best;
    double bm = 0.0, dm = 0.0;
    try {
        rc = rtcur::autotune(h, X, x_dtype, sh, iters, reps, seed, &best, &bm, &dm);
    } catch (const std::bad_alloc&) {
        rc = fail(h, RTCUR_E_NOMEM, "host allocation failed");
    } catch (...) {
        rc = fail(h, RTCUR_E_STATE, "internal error");
    }
    h->tune_forced = false;
    if (rc < 0) return rc;
    tile[0] = best.ht_rows;
    tile[1] = best.gram_chunk;
    tile[2] = best.bfac_sub;
    if (tuned_ms) *tuned_ms = bm;
    if (default_ms) *default_ms = dm;
    return RTCUR_OK;
}

int rtcur_set_tiles(rtcur_t h, const int32_t* tile) {
    if (!h) return RTCUR_E_INVAL;
    if (!tile) {
        h->tune_user_set = false;
        return RTCUR_OK;
    }
    if ((tile[0] != 8 && tile[0] != 16 && tile[0] != 32) || tile[1] < 0 ||
        (tile[1] > 0 && (tile[1] < 256 || tile[1] % 256 != 0)) || tile[2] < 0 || tile[2] > 64)
        return fail(h, RTCUR_E_INVAL,
                    "tile: rows 8, 16 or 32; Gram chunk 0 or a multiple of 256; B sub-chunks "
                    "0..64");
    h->tune_user.ht_rows = tile[0];
    h->tune_user.gram_chunk = tile[1];
    h->tune_user.bfac_sub = tile[2];
    h->tune_user_set = true;
    return RTCUR_OK;
}

int rtcur_set_graphs(rtcur_t h, int32_t enable) {
    if (!h) return RTCUR_E_INVAL;
    h->graphs = enable != 0;
    return RTCUR_OK;
}

int rtcur_autotune_clear(void) {
    rtcur::autotune_clear();
    return RTCUR_OK;
}

int rtcur_set_schedule(rtcur_t h, const double* multipliers, int32_t n) {
    if (!h) return RTCUR_E_INVAL;
    if (n < 0 || (n > 0 && !multipliers)) return fail(h, RTCUR_E_INVAL, "bad schedule");
    for (int32_t k = 0; k < n; ++k)
        if (!(multipliers[k] > 0.0) || !std::isfinite(multipliers[k]))
            return fail(h, RTCUR_E_INVAL, "schedule multipliers must be positive and finite");
    try {
        h->sched.assign(multipliers, multipliers + n);
    } catch (...) {
        return fail(h, RTCUR_E_NOMEM, "host allocation failed");
    }
    return RTCUR_OK;
}

int rtcur_destroy(rtcur_t h) {
    if (!h) return RTCUR_OK;
    rtcur::release(h);
    delete h;
    return RTCUR_OK;
}

int rtcur_get_indices(rtcur_t h, int32_t mode, int32_t which, int64_t* out, int64_t cap,
                      int64_t* len) {
    if (!h) return RTCUR_E_INVAL;
    if (!h->have_result) return fail(h, RTCUR_E_STATE, "no successful solve");
    if (mode < 0 || mode >= h->shape.n || (which != 0 && which != 1))
        return fail(h, RTCUR_E_INVAL, "mode or which out of range");
    // chidori column lists are formed from the I_i on first request
    if (which == 1 && h->shape.chidori &&
        (int64_t)h->sample.Jcols[mode].size() != h->shape.m[mode]) {
        try {
            rtcur::chidori_columns(h->shape, h->sample);
        } catch (...) {
            return fail(h, RTCUR_E_NOMEM, "column list allocation failed");
        }
    }
    const std::vector<int64_t>& v = which == 0 ? h->sample.I[mode] : h->sample.Jcols[mode];
    if (len) *len = (int64_t)v.size();
    if (out) {
        const int64_t k = cap < (int64_t)v.size() ? cap : (int64_t)v.size();
        if (k > 0) std::memcpy(out, v.data(), sizeof(int64_t) * k);
    }
    return RTCUR_OK;
}

int rtcur_get_history(rtcur_t h, double* err, double* zeta, int32_t cap, int32_t* len) {
    if (!h) return RTCUR_E_INVAL;
    if (!h->have_result) return fail(h, RTCUR_E_STATE, "no successful solve");
    const int32_t k = (int32_t)h->err_hist.size();
    if (len) *len = k;
    const int32_t q = cap < k ? cap : k;
    for (int32_t j = 0; j < q; ++j) {
        if (err) err[j] = h->err_hist[j];
        if (zeta) zeta[j] = h->zeta_hist[j];
    }
    return RTCUR_OK;
}

int rtcur_get_block(rtcur_t h, int32_t block, int32_t what, double* out, int64_t cap,
                    int64_t* len) {
    if (!h) return RTCUR_E_INVAL;
    return rtcur::get_block(h, block, what, out, cap, len);
}

int rtcur_get_tucker(rtcur_t h, double* core, double* const* B) {
    if (!h) return RTCUR_E_INVAL;
    return rtcur::get_tucker(h, core, B);
}

int rtcur_sample(uint64_t seed, int64_t t, int32_t n, const int64_t* dims,
                 const int64_t* I_sizes, const int64_t* J_sizes, int32_t mode, int32_t which,
                 int64_t* out, int64_t cap, int64_t* len) {
    if (n < 2 || n > rtcur::kMaxModes || !dims || !I_sizes) return RTCUR_E_INVAL;
    if (mode < 0 || mode >= n || (which != 0 && which != 1) || t < 0) return RTCUR_E_INVAL;
    Shape sh;
    sh.n = n;
    sh.chidori = (J_sizes == nullptr);
    for (int i = 0; i < n; ++i) {
        if (dims[i] < 1 || I_sizes[i] < 0 || I_sizes[i] > dims[i]) return RTCUR_E_INVAL;
        sh.d[i] = dims[i];
        sh.s[i] = I_sizes[i];
        sh.r[i] = 1;
    }
    for (int i = 0; i < n; ++i) {
        int64_t P = 1, m = 1;
        for (int j = 0; j < n; ++j)
            if (j != i) {
                P *= dims[j];
                m *= I_sizes[j];
            }
        if (J_sizes) {
            if (J_sizes[i] < 0 || J_sizes[i] > P) return RTCUR_E_INVAL;
            m = J_sizes[i];
        }
        sh.m[i] = m;
    }
    rtcur::SampleHost smp;
    try {
        rtcur::draw_sample(seed, t, sh, sh.chidori, smp);
    } catch (...) {
        return RTCUR_E_NOMEM;
    }
    const std::vector<int64_t>& v = which == 0 ? smp.I[mode] : smp.Jcols[mode];
    if (len) *len = (int64_t)v.size();
    if (out) {
        const int64_t k = cap < (int64_t)v.size() ? cap : (int64_t)v.size();
        if (k > 0) std::memcpy(out, v.data(), sizeof(int64_t) * k);
    }
    return RTCUR_OK;
}

int rtcur_set_profiling(rtcur_t h, int32_t mask) {
    if (!h) return RTCUR_E_INVAL;
    const uint32_t all = (1u << rtcur::kProfKinds) - 1u;
    const uint32_t m = mask < 0 ? all : ((uint32_t)mask & all);
    if (m && !h->prof_mask) {
        for (int k = 0; k < rtcur::kProfKinds; ++k) {
            h->prof_ms[k] = 0.0;
            h->prof_count[k] = 0;
        }
    }
    h->prof_mask = m;
    return RTCUR_OK;
}

int rtcur_get_profile(rtcur_t h, int32_t kind, char* name, int32_t name_cap,
                      double* total_ms, int64_t* launches) {
    if (!h) return RTCUR_E_INVAL;
    if (kind < 0 || kind >= rtcur::kProfKinds) return RTCUR_E_INVAL;
    if (name && name_cap > 0) {
        std::strncpy(name, rtcur::kProfNames[kind], (size_t)name_cap - 1);
        name[name_cap - 1] = 0;
    }
    if (total_ms) *total_ms = h->prof_ms[kind];
    if (launches) *launches = h->prof_count[kind];
    return RTCUR_OK;
}

const char* rtcur_strerror(int status) {
    switch (status) {
        case RTCUR_OK: return "ok";
        case RTCUR_NOT_CONVERGED: return "not converged within max_iter";
        case RTCUR_E_INVAL: return "invalid argument";
        case RTCUR_E_NOMEM: return "out of memory";
        case RTCUR_E_HIP: return "HIP runtime error";
        case RTCUR_E_RANK: return "rank-deficient U_i";
        case RTCUR_E_NONFINITE: return "non-finite value";
        case RTCUR_E_STATE: return "invalid call order";
        default: return "unknown status";
    }
}

const char* rtcur_last_error(rtcur_t h) {
    if (!h) return "null handle";
    return h->last_error.c_str();
}

}  // extern "C"
