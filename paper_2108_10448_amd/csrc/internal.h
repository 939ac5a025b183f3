// Internal declarations of librtcur: problem shape, host sample, the device
// problem descriptor passed to kernels, the device-side loop state, and the
// handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rtcur.h"

namespace rtcur {

constexpr int kMaxModes = 4;
constexpr int kMaxBlocks = kMaxModes + 1;
constexpr int kMaxRank = 16;
constexpr int kMaxCore = 4096;   // prod(r_i), the Tucker core held in LDS
constexpr int kMaxS = 256;       // |I_i|, the eigensolver's matrix side

// ---------------------------------------------------------------- host side

struct Shape {
    int n = 0;
    int64_t d[kMaxModes] = {};
    int r[kMaxModes] = {};
    int64_t s[kMaxModes] = {};   // |I_i|
    int64_t m[kMaxModes] = {};   // |J_i| (chidori: prod_{j != i} s_j)
    bool chidori = true;
};

struct SampleHost {
    std::vector<std::vector<int64_t>> I;      // per mode, sorted
    std::vector<std::vector<int64_t>> Jcols;  // per mode: unfolding columns
    std::vector<std::vector<int32_t>> Jtup;   // per mode: [m_i][n-1] tuples
};

// I_i always; under fiber sampling also J_i; under chidori J_i only when
// with_cols (else left empty: chidori_columns forms them from the I_i).
void draw_sample(uint64_t seed, int64_t t, const Shape& sh, bool chidori,
                 SampleHost& out, bool with_cols = true);
void chidori_columns(const Shape& sh, SampleHost& out);

// ------------------------------------------------------- device descriptors

// One sampled block.  Block 0 is R (rows I_0, columns the product of
// I_1..I_{n-1}); block 1+i is C_i (rows all of mode i, columns J_i).  Blocks
// are stored row-major, one after another, in every block-sized buffer.
struct BlockDev {
    int mode;                 // mode that indexes the block's rows
    int r;                    // rank of that mode
    int nrows;
    int ncols;
    int64_t off;              // element offset of the block
    int64_t hoff;             // element offset of the block's H (RP x ncols)
    int64_t moff;             // 64-bit word offset of the support bitmask
    int words;                // bitmask words per row
    int tile0, tile1;         // range of the block's tiles in the tile table
    int plen;                 // consecutive columns that share every other-mode
                              // index but the last (chidori: s of the last
                              // other mode); 0 when columns have no such runs
    const int32_t* rowidx;    // row -> index in `mode` (nullptr: identity)
    const int64_t* colx;      // column -> X offset of the other modes' indices
    const int32_t* cidx;      // [n-1][ncols] other-mode index of each column
};

struct Prob {
    int n;
    int nblk;
    int rp;                   // padded rank: 4, 8 or 16
    int core;                 // prod r_i
    int d[kMaxModes];
    int r[kMaxModes];
    int s[kMaxModes];
    int m[kMaxModes];
    int64_t xstride[kMaxModes];
    int64_t boff[kMaxModes];  // offset of B_i (d_i x rp) in the factor buffer
    int64_t woff[kMaxModes];  // offset of W_i / Y_i (s_i x rp), float64
    int64_t goff[kMaxModes];  // offset of the Gram of mode i (s_i x s_i)
    int64_t zoff[kMaxModes];  // offset of Z_i (m_i x r_i, row per column), float64
    int gitem0[kMaxModes];    // first Gram work item of mode i
    int gnkc[kMaxModes];      // Gram column chunks per output tile of mode i
    int gchunk[kMaxModes];    // columns per Gram chunk (multiple of 256)
    int cparts;               // core slices per a (middle-mode row parts, 3 modes)
    int crows;                // middle-mode rows per part
    int bitem0[kMaxModes];    // first B-factor work item of mode i
    int bnkc[kMaxModes];      // B-factor column chunks per row block of mode i
    int bsub[kMaxModes];      // staged Z sub-chunks per B-factor column chunk
    const int32_t* I[kMaxModes];   // sampled rows of each mode (device)
    const double* zsched;     // threshold multipliers c_1..c_nsched of zeta_0 (device)
    int nsched;               // 0: the geometric decay of equation 12 throughout
    BlockDev blk[kMaxBlocks];
};

// Loop state that lives on the device so that iterations can be queued ahead
// of the host: every iteration kernel returns at once when `stop` is set.
struct DevState {
    int stop;            // 1: stop (converged, zero data, or error)
    int status;          // rtcur_status of the stop
    int final_iter;      // k of the returned iterate
    int converged;
    double zeta0;
    double den;          // denominator of e^(k) on the current sample
    int eig_steps;
    int eig_unconverged;
    double e_prev, e_last;  // the last two e^(k) decided (host chunk planning)
    int iter;            // k of the next threshold pass when its launch passes
                         // k = -1 (replayed iteration graphs): advanced by the
                         // Gram launch's decision workgroup
    unsigned counter[4]; // last-workgroup counters (gather, ht, spare)
    double eigest[kMaxModes];  // per mode: lower bound of lambda_r / lambda_1 of
                               // the Gram at the last eigensolver call (0: none)
};

// ------------------------------------------------------------------ handle

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct rtcur_handle_impl;  // fwd

// Tile shapes of a layout (0: the built-in rule): rows per gather /
// threshold tile (8, 16 or 32), columns per Gram work item (sets the number
// of column chunks per Gram tile), Z sub-chunks per B-factor work item.
struct Tune {
    int ht_rows = 0;
    int gram_chunk = 0;
    int bfac_sub = 0;
    bool operator==(const Tune& o) const {
        return ht_rows == o.ht_rows && gram_chunk == o.gram_chunk && bfac_sub == o.bfac_sub;
    }
};

}  // namespace rtcur

struct rtcur_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int variant = RTCUR_FIXED;
    int dtype = RTCUR_F64;
    std::string last_error;
    // results of the last solve
    bool have_result = false;
    rtcur::Shape shape;
    rtcur::SampleHost sample;
    std::vector<double> err_hist, zeta_hist;
    std::vector<double> sched;  // rtcur_set_schedule: multipliers of zeta_0
    rtcur_info info{};
    // device workspace (owned; grown on demand, freed by destroy)
    std::vector<rtcur::DevBuf> bufs;
    void* impl = nullptr;      // solver-private state (see solver.hip)
    // kernel timing (rtcur_set_profiling)
    uint32_t prof_mask = 0;   // bit k: time kernel kind k
    double prof_ms[16] = {};
    int64_t prof_count[16] = {};
    // tile shapes: the autotuner's candidate under test, else the caller's
    // (rtcur_set_tiles), else the tuned table's entry, else the built-in rule
    bool tune_forced = false;
    rtcur::Tune tune_force;
    bool tune_user_set = false;
    rtcur::Tune tune_user;
    // rtcur_set_graphs: RTCUR-F's steady-state iterations as replayed graphs
    bool graphs = false;
};

namespace rtcur {
int solve(rtcur_s* h, const void* X, int x_dtype, const Shape& sh,
          double zeta0, double gamma, double tol, int max_iter,
          uint64_t seed);
int reconstruct(rtcur_s* h, void* out, int out_dtype);
int outliers(rtcur_s* h, const void* X, int x_dtype, double zeta, void* S_out, void* L_out,
             int out_dtype);
int get_block(rtcur_s* h, int block, int what, double* out, int64_t cap,
              int64_t* len);
int get_tucker(rtcur_s* h, double* core, double* const* B);
void release(rtcur_s* h);
// bytes of the per-device static scratch of the allocation-free entry point
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
// looks up (once per device, `device` current) the static scratch's address
int static_scratch_init(int device);
int reconstruct_noalloc(rtcur_s* h, void* out, int out_dtype);
// Times candidate tile shapes for this problem (coordinate descent over
// ht_rows, gram_chunk, bfac_sub; each candidate the best of `reps` solves of
// `iters` iterations after one warm-up) and records the fastest for its
// sizes in the process-wide table that later layouts of those sizes use.
int autotune(rtcur_s* h, const void* X, int x_dtype, const Shape& sh, int iters, int reps,
             uint64_t seed, Tune* best, double* best_ms, double* default_ms);
void autotune_clear();
constexpr int kProfKinds = 10;
extern const char* const kProfNames[kProfKinds];
}  // namespace rtcur
