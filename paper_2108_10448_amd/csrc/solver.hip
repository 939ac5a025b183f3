// Host orchestration of the RTCUR hot loop on one gfx950 device.
//
// Per iteration (RTCUR-F), all on the handle's stream and queued ahead of
// the host (every kernel returns at once after the device-side stop flag is
// raised, so the host only checks the flag every few iterations):
//   k_ht     fused residual, e^(k) numerator partials, hard threshold,
//            support bits (Step I, equations 11-14)
//   k_gram   Gram_i = U_i U_i^T on the float64 matrix cores, plus the
//            e^(k) decision from k_ht's partials
//   k_eig    top-r_i eigenspace of Gram_i -> W_i, Y_i
//   k_zcore  Z_i = U_i^T Y_i (so V_i S_i^-1 = Z_i) and the core slices
//            T[a] = R(a, ..) x_{l >= 1} W_l^T
//   k_bfac   B_i = C_i Z_i partials over column chunks
//   k_bred   B_i from the partials (k_bfac's extra workgroup finishes the
//            core G = sum_a W_0[a]^T T[a])
//   k_hexp   H_b = G x_{j != mode} B_j on each block's columns
// so that the next k_ht forms L on the blocks as B_mode H_b (Section 3.3).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <chrono>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace rtcur {

#define HIPCHK(expr)                                                           \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            h->last_error = std::string(#expr) + ": " + hipGetErrorString(e_); \
            return RTCUR_E_HIP;                                                \
        }                                                                      \
    } while (0)

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int pad_rank(int r) { return r <= 4 ? 4 : (r <= 8 ? 8 : 16); }

// Offsets of named regions inside one device arena.
struct Arena {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t off = total;
        total = align_up(total + std::max<size_t>(bytes, 1), 256);
        return off;
    }
};

constexpr int kAbsmaxWG = 2048;

}  // namespace

enum ProfKind { PK_ABSMAX = 0, PK_GATHER, PK_HT, PK_GRAM, PK_EIG, PK_ZCORE, PK_BFAC,
                PK_BRED, PK_HEXP, PK_DECIDE };
const char* const kProfNames[kProfKinds] = {"absmax", "gather", "ht",   "gram", "eig",
                                            "zcore",  "bfac",   "bred", "hexp", "decide"};

struct ProfRec {
    int kind, iter, a, b;  // a, b: indices into the event pool
};

// Device scratch of the allocation-free entry point (rtcur_reconstruct_noalloc):
// one static array in the code object, of which every GPU that loads the
// library holds its own copy, at its own address, until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory:
// kernels and copies only ever get the address that hipGetSymbolAddress
// returned for the current device (scratch_dev below).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices] = {};
}  // namespace

int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return RTCUR_E_INVAL;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_dev[device]) return RTCUR_OK;
    void* p = nullptr;
    // the caller made `device` current
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return RTCUR_E_HIP;
    }
    scratch_dev[device] = p;
    return RTCUR_OK;
}

// Solver-private state kept in the handle between calls.
struct Impl {
    std::vector<hipEvent_t> events;  // pool for kernel timing
    std::vector<ProfRec> recs;
    size_t ev_used = 0;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    void* scratch = nullptr;        // getters / reconstruct temporaries
    size_t scratch_bytes = 0;
    DevState* st_host = nullptr;    // pinned mirror of the device state and,
    size_t st_host_bytes = 0;       //   behind it, of the e^(k) history
    char* d_stage = nullptr;        // RTCUR-R: index data of queued samples
    char* h_stage = nullptr;        //   (device slots and their pinned source)
    size_t stage_bytes = 0;
    char* h_idx = nullptr;          // pinned source of the index upload
    size_t h_idx_bytes = 0;
    hipEvent_t idx_ev = nullptr;    // recorded after that upload
    bool idx_pending = false;       //   (the buffer is rewritten only after it)
    int max_dyn_lds[3] = {0, 0, 0};  // k_eig<4|8|16, true>: room for the Gram
    bool max_dyn_set = false;
    std::vector<int64_t> plan_key;  // sizes the current layout was planned for

    // layout of the current solve
    Prob P{};
    int ht_rows = kTileRows;        // rows per gather / threshold tile
    int64_t nblk_elems = 0;
    int64_t h_elems = 0, mask_words = 0, bf_elems = 0, w_elems = 0, z_elems = 0,
            g_elems = 0, t_elems = 0;
    std::vector<int4> ht_tiles, gram_items, bfac_items;
    std::vector<int2> z_tiles, h_tiles;
    int n_pairs = 0, n_bgroups = 0, n_bred_wg = 0;

    // device regions (inside the arena)
    void *XO = nullptr, *C[2] = {nullptr, nullptr}, *Bf = nullptr, *H = nullptr;
    uint64_t* mask[2] = {nullptr, nullptr};
    double* zsched = nullptr;       // threshold schedule (max_iter doubles)
    double *W = nullptr, *Y = nullptr, *Z = nullptr, *gram = nullptr,
           *gpart = nullptr, *bpart = nullptr, *Bd = nullptr, *Gd = nullptr, *Tc = nullptr,
           *part = nullptr, *hpart = nullptr, *err_hist = nullptr;
    DevState* st = nullptr;
    int4 *d_ht_tiles = nullptr, *d_gram_items = nullptr, *d_bfac_items = nullptr;
    int2 *d_z_tiles = nullptr, *d_h_tiles = nullptr;
    char* d_idx = nullptr;          // sample-dependent index data
    size_t idx_bytes = 0;
    size_t hist_len = 0;

    // replayed iteration pair (RTCUR-F steady state), captured on cstream
    // (two entries: the bfloat16 runner and its FP32 refinement sweep)
    hipStream_t cstream = nullptr;
    struct PairGraph {
        std::vector<char> key;      // what the captured launches depend on
        hipGraphExec_t exec = nullptr;
    };
    std::vector<PairGraph> graphs;  // most recently captured last
    bool graph_off = false;         // capture failed once: direct launches only

    // result bookkeeping
    int final_iter = 0;
    int cur = 0;                    // which C / mask buffer holds C^k
};

static Impl* impl_of(rtcur_s* h) {
    if (!h->impl) h->impl = new Impl();
    return static_cast<Impl*>(h->impl);
}

void release(rtcur_s* h) {
    Impl* im = static_cast<Impl*>(h->impl);
    if (!im) return;
    (void)hipSetDevice(h->device);
    if (im->arena) (void)hipFree(im->arena);
    if (im->scratch) (void)hipFree(im->scratch);
    if (im->st_host) (void)hipHostFree(im->st_host);
    if (im->d_stage) (void)hipFree(im->d_stage);
    if (im->h_stage) (void)hipHostFree(im->h_stage);
    if (im->idx_ev) (void)hipEventSynchronize(im->idx_ev);
    if (im->h_idx) (void)hipHostFree(im->h_idx);
    if (im->idx_ev) (void)hipEventDestroy(im->idx_ev);
    for (hipEvent_t e : im->events) (void)hipEventDestroy(e);
    for (auto& g : im->graphs) (void)hipGraphExecDestroy(g.exec);
    if (im->cstream) (void)hipStreamDestroy(im->cstream);
    delete im;
    h->impl = nullptr;
}

// --------------------------------------------------------------- layout

// Host-side index data for one sample, packed for a single upload.
struct IdxPack {
    size_t bytes = 0;        // whole index region
    size_t host_bytes = 0;   // leading part the host fills (the rest: k_expand_cols)
    int prod_mask = 0;       // blocks whose column data k_expand_cols forms
    size_t I_off[kMaxModes], rowidx_off, colx_off[kMaxBlocks], cidx_off[kMaxBlocks];
};

// Offsets of the index regions for this shape (they depend on sizes only):
// first the sampled indices I_i and the column data of the fiber-sampled
// blocks (packed on the host), then the column data of the blocks whose
// columns are products of the I_j (formed on the device).
static void index_layout(const Shape& sh, IdxPack& pk) {
    const int n = sh.n;
    size_t off = 0;
    auto reserve = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    for (int i = 0; i < n; ++i) pk.I_off[i] = reserve(sizeof(int32_t) * sh.s[i]);
    pk.rowidx_off = pk.I_off[0];  // the R block's rows are I_0
    int64_t ncol[kMaxBlocks];
    ncol[0] = 1;
    for (int j = 1; j < n; ++j) ncol[0] *= sh.s[j];
    for (int i = 0; i < n; ++i) ncol[1 + i] = sh.m[i];
    pk.prod_mask = 0;
    for (int b = 0; b <= n; ++b)
        if (b == 0 || sh.chidori) pk.prod_mask |= 1 << b;
    for (int pass = 0; pass < 2; ++pass) {
        for (int b = 0; b <= n; ++b) {
            if (((pk.prod_mask >> b) & 1) != pass) continue;
            pk.colx_off[b] = reserve(sizeof(int64_t) * ncol[b]);
            pk.cidx_off[b] = reserve(sizeof(int32_t) * ncol[b] * (n - 1));
        }
        if (pass == 0) pk.host_bytes = off;
    }
    pk.bytes = off;
}

// The host part of the sample's index data into base (pk.host_bytes bytes,
// laid out by index_layout; the alignment gaps are left as they are).
static void pack_indices(const Shape& sh, const SampleHost& smp, const IdxPack& pk,
                         char* base) {
    const int n = sh.n;
    for (int i = 0; i < n; ++i) {
        int32_t* p = reinterpret_cast<int32_t*>(base + pk.I_off[i]);
        for (int64_t a = 0; a < sh.s[i]; ++a) p[a] = (int32_t)smp.I[i][a];
    }
    if (sh.chidori) return;
    int64_t xstride[kMaxModes];
    xstride[n - 1] = 1;
    for (int j = n - 2; j >= 0; --j) xstride[j] = xstride[j + 1] * sh.d[j + 1];
    // fiber-sampled C_i: the drawn unfolding columns
    for (int i = 0; i < n; ++i) {
        int64_t* cx = reinterpret_cast<int64_t*>(base + pk.colx_off[1 + i]);
        int32_t* ci = reinterpret_cast<int32_t*>(base + pk.cidx_off[1 + i]);
        const int64_t m = sh.m[i];
        const int32_t* tup = smp.Jtup[i].data();
        for (int64_t c = 0; c < m; ++c) {
            int64_t off2 = 0;
            int q = 0;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                const int64_t v = tup[c * (n - 1) + q];
                off2 += v * xstride[j];
                ci[(int64_t)q * m + c] = (int32_t)v;
                ++q;
            }
            cx[c] = off2;
        }
    }
}

// Region offsets of one solve's arena.
struct Regions {
    size_t XO, C0, C1, m0, m1, Bf, H, W, Y, Z, gram, gpart, bpart, Bd, Gd, Tc, part,
        hpart, hist, st, tiles, idx, zs;
};

// Block descriptors, offsets and work lists for this shape; sizes the arena.
static void plan(Impl& im, const Shape& sh, int esize, size_t idx_bytes, int max_iter,
                 const Tune& tune, Arena& ar, Regions& rg) {
    const int n = sh.n;
    Prob& P = im.P;
    std::memset(&P, 0, sizeof(P));
    P.n = n;
    P.nblk = n + 1;
    int rmax = 1;
    P.core = 1;
    for (int i = 0; i < n; ++i) {
        P.d[i] = (int)sh.d[i];
        P.r[i] = sh.r[i];
        P.s[i] = (int)sh.s[i];
        P.m[i] = (int)sh.m[i];
        rmax = std::max(rmax, sh.r[i]);
        P.core *= sh.r[i];
    }
    const int RP = pad_rank(rmax);
    P.rp = RP;
    P.xstride[n - 1] = 1;
    for (int j = n - 2; j >= 0; --j) P.xstride[j] = P.xstride[j + 1] * sh.d[j + 1];
    int64_t off = 0, hoff = 0, moff = 0;
    im.ht_tiles.clear();
    im.ht_rows = tune.ht_rows == 8 || tune.ht_rows == 32 ? tune.ht_rows : kTileRows;
    if (esize == 8 && im.ht_rows == 32) im.ht_rows = kTileRows;  // (registers)
    for (int b = 0; b <= n; ++b) {
        BlockDev& bd = P.blk[b];
        if (b == 0) {
            bd.mode = 0;
            bd.nrows = (int)sh.s[0];
            int64_t nc = 1;
            for (int j = 1; j < n; ++j) nc *= sh.s[j];
            bd.ncols = (int)nc;
        } else {
            bd.mode = b - 1;
            bd.nrows = (int)sh.d[b - 1];
            bd.ncols = (int)sh.m[b - 1];
        }
        bd.r = sh.r[bd.mode];
        {
            // the columns run over the other modes in C order (last fastest)
            // for R and for chidori blocks
            const int last = bd.mode == n - 1 ? n - 2 : n - 1;
            bd.plen = (b == 0 || sh.chidori) ? (int)sh.s[last] : 0;
        }
        bd.off = off;
        bd.hoff = hoff;
        bd.moff = moff;
        bd.words = (bd.ncols + 63) / 64;
        off += (int64_t)bd.nrows * bd.ncols;
        hoff += (int64_t)RP * bd.ncols;
        moff += (int64_t)bd.nrows * bd.words;
    }
    // gather / threshold tiles of the blocks with the most rows first (a
    // block of fewer rows than a tile has short tiles: they fill in at the
    // end); a block's tiles stay contiguous, in row-major tile order, as the
    // error sums read them
    {
        int tord[kMaxBlocks];
        for (int b = 0; b <= n; ++b) tord[b] = b;
        std::stable_sort(tord, tord + n + 1, [&](int a, int b) {
            return std::min(P.blk[a].nrows, im.ht_rows) > std::min(P.blk[b].nrows, im.ht_rows);
        });
        for (int q = 0; q <= n; ++q) {
            BlockDev& bd = P.blk[tord[q]];
            bd.tile0 = (int)im.ht_tiles.size();
            for (int r0 = 0; r0 < bd.nrows; r0 += im.ht_rows)
                for (int c0 = 0; c0 < bd.ncols; c0 += kTileCols)
                    im.ht_tiles.push_back(make_int4(tord[q], r0, c0, 0));
            bd.tile1 = (int)im.ht_tiles.size();
        }
    }
    im.nblk_elems = off;
    im.h_elems = hoff;
    im.mask_words = moff;
    im.bf_elems = im.w_elems = im.z_elems = im.g_elems = 0;
    for (int i = 0; i < n; ++i) {
        P.boff[i] = im.bf_elems;
        im.bf_elems += (int64_t)sh.d[i] * RP;
        P.woff[i] = im.w_elems;
        im.w_elems += sh.s[i] * RP;
        P.goff[i] = im.g_elems;
        // the upper-triangular 16 x 16 tiles of the Gram
        const int64_t nt = (sh.s[i] + 15) / 16;
        im.g_elems += 256 * (nt * (nt + 1) / 2);
        P.zoff[i] = im.z_elems;
        im.z_elems += (int64_t)sh.r[i] * sh.m[i];  // r_i words per column
    }
    // Gram work: upper-triangular 16x16 tile pairs x column chunks
    im.gram_items.clear();
    int npairs_all = 0;
    for (int i = 0; i < n; ++i) {
        const int nt = (int)((sh.s[i] + 15) / 16);
        npairs_all += nt * (nt + 1) / 2;
    }
    int pid = 0;
    for (int i = 0; i < n; ++i) {
        const int nt = (int)((sh.s[i] + 15) / 16);
        // at least kGramMinChunk columns per chunk; at most kGramMaxKC chunks,
        // and about 1024 tiles per mode for the eigensolver to add up
        const int npi = nt * (nt + 1) / 2;
        int nkc;
        if (tune.gram_chunk > 0) {
            nkc = (int)std::min<int64_t>(kGramMaxKC, (sh.m[i] + tune.gram_chunk - 1) /
                                                         tune.gram_chunk);
            nkc = std::max(1, nkc);
        } else {
            nkc = (int)std::min<int64_t>(kGramMaxKC, (sh.m[i] + kGramMinChunk - 1) / kGramMinChunk);
            nkc = std::max(1, std::min(nkc, std::max(kGramKCGroup, 1024 / npi)));
        }
        const int chunk = (int)align_up((size_t)((sh.m[i] + nkc - 1) / nkc), 256);
        P.gnkc[i] = nkc;
        P.gchunk[i] = chunk;
    }
    // items of the modes with the longest chunks (the longer workgroups)
    // first, so that they are dispatched first; a mode's items stay
    // contiguous in (tile pair, chunk) order, as the eigensolver reads them
    int gord[kMaxModes];
    for (int i = 0; i < n; ++i) gord[i] = i;
    std::stable_sort(gord, gord + n, [&](int a, int b) { return P.gchunk[a] > P.gchunk[b]; });
    for (int q = 0; q < n; ++q) {
        const int i = gord[q];
        const int nt = (int)((sh.s[i] + 15) / 16);
        P.gitem0[i] = (int)im.gram_items.size();
        for (int ta = 0; ta < nt; ++ta)
            for (int tb = ta; tb < nt; ++tb, ++pid)
                for (int kc = 0; kc < P.gnkc[i]; ++kc)
                    im.gram_items.push_back(make_int4(i, ta | (tb << 16), kc, pid));
    }
    im.n_pairs = pid;
    (void)npairs_all;
    // Z_i: 64 columns per work item; B_i: 16 rows x column chunks
    im.z_tiles.clear();
    im.bfac_items.clear();
    im.n_bgroups = 0;
    const int bkc = bfac_kc(RP);
    // Z tiles of the modes with more sampled rows (the longer workgroups)
    // first
    {
        int zord[kMaxModes];
        for (int i = 0; i < n; ++i) zord[i] = i;
        std::stable_sort(zord, zord + n, [&](int a, int b) { return sh.s[a] > sh.s[b]; });
        for (int q = 0; q < n; ++q)
            for (int64_t c0 = 0; c0 < sh.m[zord[q]]; c0 += 64)
                im.z_tiles.push_back(make_int2(zord[q], (int)c0));
    }
    for (int i = 0; i < n; ++i) {
        // at most kBfacMaxKC partial rows per entry for k_bred: long modes
        // stage several Z sub-chunks per work item
        const int nsc = (int)((sh.m[i] + bkc - 1) / bkc);
        const int nsub = std::min(nsc, std::max((nsc + kBfacMaxKC - 1) / kBfacMaxKC,
                                                tune.bfac_sub));
        P.bnkc[i] = (nsc + nsub - 1) / nsub;
        P.bsub[i] = nsub;
    }
    // items of the modes with the most sub-chunks per item (the longest
    // workgroups) first, so that they are dispatched first and the shorter
    // ones fill the CUs around them; a mode's items stay contiguous in (row
    // block, chunk) order, as k_bred reads them
    int border[kMaxModes];
    for (int i = 0; i < n; ++i) border[i] = i;
    std::stable_sort(border, border + n, [&](int a, int b) { return P.bsub[a] > P.bsub[b]; });
    for (int q = 0; q < n; ++q) {
        const int i = border[q];
        P.bitem0[i] = (int)im.bfac_items.size();
        for (int rb = 0; rb * kBfacRows < sh.d[i]; ++rb, ++im.n_bgroups)
            for (int kc = 0; kc < P.bnkc[i]; ++kc)
                im.bfac_items.push_back(make_int4(i, rb, kc, im.n_bgroups));
    }
    int64_t bent = 0;
    for (int i = 0; i < n; ++i) bent += sh.d[i] * RP;
    im.n_bred_wg = (int)((bent + kThreads - 1) / kThreads);
    // H tiles of the blocks with more H rows (the block mode's rank: the
    // longer workgroups) first; order does not change what a tile computes
    im.h_tiles.clear();
    int hord[kMaxBlocks];
    for (int b = 0; b <= n; ++b) hord[b] = b;
    std::stable_sort(hord, hord + n + 1,
                     [&](int a, int b) { return P.blk[a].r > P.blk[b].r; });
    for (int q = 0; q <= n; ++q) {
        const int b = hord[q];
        for (int cb = 0; cb * kThreads < P.blk[b].ncols; ++cb)
            im.h_tiles.push_back(make_int2(b, cb));
    }
    // core slices T[a] = R(a, ..) x_{l >= 1} W_l^T: s_0 x prod_{l >= 1} r_l
    // with three modes the slice's middle-mode rows are split so that each
    // part is staged in one pass
    P.cparts = 1;
    P.crows = 1;  // all middle-mode rows of a slice
    for (int l = 1; l < n - 1; ++l) P.crows *= (int)sh.s[l];
    if (n == 3) {
        const int rc = std::max<int>(1, kSliceBytes / esize / (int)sh.s[2]);
        P.cparts = (P.crows + rc - 1) / rc;
        P.crows = (P.crows + P.cparts - 1) / P.cparts;
    }
    im.t_elems = sh.s[0] * P.cparts * (P.core / sh.r[0]);

    const size_t nb = (size_t)im.nblk_elems;
    rg.XO = ar.add(nb * esize);
    rg.C0 = ar.add(nb * esize);
    rg.C1 = ar.add(nb * esize);
    rg.m0 = ar.add(sizeof(uint64_t) * im.mask_words);
    rg.m1 = ar.add(sizeof(uint64_t) * im.mask_words);
    rg.Bf = ar.add(im.bf_elems * esize);
    rg.H = ar.add(im.h_elems * esize);
    rg.W = ar.add(sizeof(double) * im.w_elems);
    rg.Y = ar.add(sizeof(double) * im.w_elems);
    rg.Z = ar.add(sizeof(double) * im.z_elems);
    rg.gram = ar.add(sizeof(double) * im.g_elems);
    rg.gpart = ar.add(sizeof(double) * 256 * im.gram_items.size());
    rg.bpart = ar.add(sizeof(double) * kBfacRows * RP * im.bfac_items.size());
    rg.Bd = ar.add(sizeof(double) * im.bf_elems);
    rg.Gd = ar.add(sizeof(double) * P.core);
    rg.Tc = ar.add(sizeof(double) * im.t_elems);
    rg.part = ar.add(sizeof(double) * 2 * std::max<size_t>(im.ht_tiles.size(), kAbsmaxWG));
    rg.hpart = ar.add(sizeof(double) * im.ht_tiles.size());
    im.hist_len = (size_t)max_iter + 2;
    rg.st = ar.add(sizeof(DevState));  // the history right behind: one read-back
    rg.hist = ar.add(sizeof(double) * im.hist_len);
    rg.tiles = ar.add(sizeof(int4) * (im.ht_tiles.size() + im.gram_items.size() +
                                      im.bfac_items.size()) +
                      sizeof(int2) * (im.z_tiles.size() + im.h_tiles.size()));
    rg.idx = ar.add(idx_bytes);
    rg.zs = ar.add(sizeof(double) * (size_t)max_iter);  // threshold schedule
}

// ------------------------------------------------------------ the solver

// H_b expansion launch: the run-factored kernel when the columns come in
// runs and the per-column contraction (prod r_i) is long, else the
// per-column one.
template <typename T, int RP>
static void launch_hexp(const Prob& P, bool runs, unsigned grid, hipStream_t st,
                        const int2* tiles, const T* Bf, const double* Gd, T* H,
                        const DevState* ds, int dense_mode, int64_t dense_cols) {
    const bool fac = P.n >= 3 && runs && P.core > kHexpFactorMin;
    switch (P.n) {
        case 2:
            hipLaunchKernelGGL((k_hexp<T, RP, 2>), dim3(grid), dim3(kThreads), 0, st, P, tiles,
                               Bf, Gd, H, ds, dense_mode, dense_cols);
            break;
        case 3:
            if (fac)
                hipLaunchKernelGGL((k_hexp_fac<T, RP, 3>), dim3(grid), dim3(kThreads), 0, st, P,
                                   tiles, Bf, Gd, H, ds, dense_mode, dense_cols);
            else
                hipLaunchKernelGGL((k_hexp<T, RP, 3>), dim3(grid), dim3(kThreads), 0, st, P,
                                   tiles, Bf, Gd, H, ds, dense_mode, dense_cols);
            break;
        default:
            if (fac)
                hipLaunchKernelGGL((k_hexp_fac<T, RP, 4>), dim3(grid), dim3(kThreads), 0, st, P,
                                   tiles, Bf, Gd, H, ds, dense_mode, dense_cols);
            else
                hipLaunchKernelGGL((k_hexp<T, RP, 4>), dim3(grid), dim3(kThreads), 0, st, P,
                                   tiles, Bf, Gd, H, ds, dense_mode, dense_cols);
            break;
    }
}

constexpr int kRChunk = 8;  // RTCUR-R: iterations queued per state read

// T: factor and arithmetic type; TB: block storage type (T, or bfloat16
// with T = float for the bfloat16 iterations).
template <typename T, int RP, typename TB = T>
struct Runner {
    rtcur_s* h;
    Impl& im;
    hipStream_t s;
    int tag = 0;    // iteration the next launches belong to (0: set-up)
    int open = -1;  // pending profile record

    // Event pair around one launch when profiling is on.
    hipError_t pb(int kind) {
        open = -1;
        if (!(h->prof_mask & (1u << kind))) return hipSuccess;
        if (im.ev_used + 2 > im.events.size()) {
            for (int q = 0; q < 64; ++q) {
                hipEvent_t e;
                hipError_t err = hipEventCreate(&e);
                if (err != hipSuccess) return err;
                im.events.push_back(e);
            }
        }
        const int a = (int)im.ev_used++, b = (int)im.ev_used++;
        im.recs.push_back(ProfRec{kind, tag, a, b});
        open = (int)im.recs.size() - 1;
        return hipEventRecord(im.events[a], s);
    }
    hipError_t pe() {
        if (open < 0) return hipSuccess;
        const int b = im.recs[open].b;
        open = -1;
        return hipEventRecord(im.events[b], s);
    }
    // Accumulate the launches that did work: iteration tags up to K, and up
    // to K + 1 for the kernels whose pass at K + 1 decides the stop.
    int prof_collect(int K) {
        if (im.recs.empty()) return 0;
        HIPCHK(hipStreamSynchronize(s));
        for (const ProfRec& r : im.recs) {
            const bool deciding = r.kind == PK_HT || r.kind == PK_GRAM || r.kind == PK_DECIDE;
            if (r.iter > K + (deciding ? 1 : 0)) continue;
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, im.events[r.a], im.events[r.b]));
            h->prof_ms[r.kind] += ms;
            h->prof_count[r.kind] += 1;
        }
        im.recs.clear();
        im.ev_used = 0;
        return 0;
    }

    template <int TR>
    void gather_tr(const void* X, int xdt, int flags, int nt) {
        if (xdt == RTCUR_F64)
            hipLaunchKernelGGL((k_gather<double, TB, TR>), dim3(nt), dim3(kThreads), 0, s,
                               (const double*)X, im.P, im.d_ht_tiles, (TB*)im.XO, im.part,
                               (const DevState*)im.st, flags);
        else
            hipLaunchKernelGGL((k_gather<float, TB, TR>), dim3(nt), dim3(kThreads), 0, s,
                               (const float*)X, im.P, im.d_ht_tiles, (TB*)im.XO, im.part,
                               (const DevState*)im.st, flags);
    }

    int gather(const void* X, int xdt, int flags) {
        const int nt = (int)im.ht_tiles.size();
        HIPCHK(pb(PK_GATHER));
        if (im.ht_rows == 8) gather_tr<8>(X, xdt, flags, nt);
        else if (im.ht_rows == 32 && sizeof(TB) <= 4) gather_tr<32>(X, xdt, flags, nt);
        else gather_tr<kTileRows>(X, xdt, flags, nt);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_den, dim3(1), dim3(kThreads), 0, s, im.P, (const double*)im.part,
                           flags, im.st);
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        return 0;
    }

    int ht(int kcur, int flags, const TB* Cold, TB* Cnew, uint64_t* mask, double gamma) {
        const int nt = (int)im.ht_tiles.size();
        HIPCHK(pb(PK_HT));
        auto go = [&](auto tr) {
            constexpr int TR = decltype(tr)::value;
            hipLaunchKernelGGL((k_ht<T, RP, TB, TR>), dim3(nt), dim3(kThreads), 0, s, im.P,
                               im.d_ht_tiles, (const TB*)im.XO, Cold, Cnew, mask,
                               (const T*)im.Bf, (const T*)im.H, gamma, kcur, flags, im.hpart,
                               im.st);
        };
        if (im.ht_rows == 8) go(std::integral_constant<int, 8>{});
        else if (im.ht_rows == 32 && sizeof(TB) <= 4) go(std::integral_constant<int, 32>{});
        else go(std::integral_constant<int, kTileRows>{});
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        return 0;
    }

    int decide(int kcur, double tol) {
        HIPCHK(pb(PK_DECIDE));
        hipLaunchKernelGGL(k_decide, dim3(1), dim3(kThreads), 0, s, im.P,
                           (const double*)im.hpart, kcur, tol, im.err_hist, im.st);
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        return 0;
    }

    int hexp() {
        HIPCHK(pb(PK_HEXP));
        const unsigned nt = (unsigned)im.h_tiles.size();
        // every block comes in column runs only under chidori sampling
        launch_hexp<T, RP>(im.P, h->shape.chidori, nt, s, im.d_h_tiles, (const T*)im.Bf,
                           im.Gd, (T*)im.H, im.st, 0, 0);
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        return 0;
    }

    // Step (II): L-update from C (equations 8-9) into B_i, G, H_b.  With
    // `decide`, the Gram launch also forms e^(kcur) from k_ht's partials.
    int lupdate(const TB* C, int warm, int decide_flag, int kcur, double tol) {
        const Prob& P = im.P;
        const int n = P.n;
        const int ng = (int)im.gram_items.size();
        HIPCHK(pb(PK_GRAM));
        hipLaunchKernelGGL((k_gram<TB>), dim3(ng + 1), dim3(kThreads), 0, s, P, C,
                           im.d_gram_items, ng, im.gpart, decide_flag,
                           (const double*)im.hpart, kcur, tol, im.err_hist, im.st);
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        int smax = 0;
        for (int i = 0; i < n; ++i) smax = std::max(smax, (P.s[i] + 15) / 16 * 16);
        const size_t lds_g = sizeof(double) * 256 * (size_t)(smax / 16) * (smax / 16 + 1) / 2;
        const int use_lds = lds_g <= (size_t)im.max_dyn_lds[RP == 4 ? 0 : RP == 8 ? 1 : 2];
        // float64 blocks: subspace to 1e-13; float32 (and bfloat16) blocks:
        // the residual scaled to the weakest wanted pair from float32's unit
        // roundoff (see k_eig)
        const double rtol = sizeof(T) == 8 ? 1e-13 : -0x1p-24;
        HIPCHK(pb(PK_EIG));
        if (use_lds)
            hipLaunchKernelGGL((k_eig<RP, true>), dim3(n), dim3(kThreads), lds_g, s, P,
                               (const double*)im.gpart, im.gram, im.W, im.Y, im.Bd, warm, 200, rtol,
                               im.st);
        else
            hipLaunchKernelGGL((k_eig<RP, false>), dim3(n), dim3(kThreads), 0, s, P,
                               (const double*)im.gpart, im.gram, im.W, im.Y, im.Bd, warm, 200, rtol,
                               im.st);
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        const int nz = (int)im.z_tiles.size();
        HIPCHK(pb(PK_ZCORE));
        int srows = 1;  // rows of a sampled core slice
        for (int l = 1; l < n - 1; ++l) srows *= P.s[l];
        if (P.r[n - 1] * srows > kCoreLds / 2)  // (three modes only)
            hipLaunchKernelGGL((k_zcore<TB, RP, true>), dim3(nz + P.s[0] * P.cparts),
                               dim3(kThreads), 0, s, P, C, (const double*)im.Y, im.Z,
                               im.d_z_tiles, nz, (const double*)im.W, im.Tc, im.st);
        else
            hipLaunchKernelGGL((k_zcore<TB, RP, false>), dim3(nz + P.s[0] * P.cparts),
                               dim3(kThreads), 0, s, P, C, (const double*)im.Y, im.Z,
                               im.d_z_tiles, nz, (const double*)im.W, im.Tc, im.st);
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        HIPCHK(pb(PK_BFAC));
        const int nb = (int)im.bfac_items.size();
        bool sub = false;
        for (int i = 0; i < n; ++i) sub = sub || P.bsub[i] > 1;
        if (sub)
            hipLaunchKernelGGL((k_bfac<TB, RP, true>), dim3(nb + 1), dim3(kThreads), 0, s, P, C,
                               (const double*)im.Z, im.d_bfac_items, nb, im.bpart,
                               (const double*)im.W, (const double*)im.Tc, im.Gd, im.st);
        else
            hipLaunchKernelGGL((k_bfac<TB, RP, false>), dim3(nb + 1), dim3(kThreads), 0, s, P, C,
                               (const double*)im.Z, im.d_bfac_items, nb, im.bpart,
                               (const double*)im.W, (const double*)im.Tc, im.Gd, im.st);
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        HIPCHK(pb(PK_BRED));
        hipLaunchKernelGGL((k_bred<T, RP>), dim3(im.n_bred_wg), dim3(kThreads), 0, s, P,
                           (const double*)im.bpart, im.d_bfac_items, (T*)im.Bf, im.Bd, im.st);
        HIPCHK(hipGetLastError());
        HIPCHK(pe());
        return hexp();
    }

    int read_state(DevState& out) {
        // the state and the e^(k) history behind it in one copy
        const size_t bytes = (size_t)(reinterpret_cast<char*>(im.err_hist + im.hist_len) -
                                      reinterpret_cast<char*>(im.st));
        if (bytes > im.st_host_bytes) {
            if (im.st_host) HIPCHK(hipHostFree(im.st_host));
            im.st_host = nullptr;
            im.st_host_bytes = 0;
            HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&im.st_host), bytes,
                                 hipHostMallocDefault));
            im.st_host_bytes = bytes;
        }
        HIPCHK(hipMemcpyAsync(im.st_host, im.st, bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        out = *im.st_host;
        return 0;
    }

    int upload_sample(const SampleHost& smp, const Shape& sh) {
        IdxPack pk;
        index_layout(sh, pk);
        if (pk.bytes > im.idx_bytes) {
            h->last_error = "internal: index region too small";
            return RTCUR_E_STATE;
        }
        // packed into pinned memory and copied in stream order; the host
        // rewrites that memory only once the previous copy has finished
        if (im.idx_pending) {
            HIPCHK(hipEventSynchronize(im.idx_ev));
            im.idx_pending = false;
        }
        if (pk.bytes > im.h_idx_bytes) {
            if (im.h_idx) HIPCHK(hipHostFree(im.h_idx));
            im.h_idx = nullptr;
            im.h_idx_bytes = 0;
            if (hipHostMalloc(reinterpret_cast<void**>(&im.h_idx), pk.bytes,
                              hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                h->last_error = "pinned index buffer allocation failed";
                return RTCUR_E_NOMEM;
            }
            im.h_idx_bytes = pk.bytes;
        }
        if (!im.idx_ev)
            HIPCHK(hipEventCreateWithFlags(&im.idx_ev, hipEventDisableTiming));
        pack_indices(sh, smp, pk, im.h_idx);
        HIPCHK(hipMemcpyAsync(im.d_idx, im.h_idx, pk.host_bytes, hipMemcpyHostToDevice, s));
        HIPCHK(hipEventRecord(im.idx_ev, s));
        im.idx_pending = true;
        Prob& P = im.P;
        for (int i = 0; i < sh.n; ++i)
            P.I[i] = reinterpret_cast<const int32_t*>(im.d_idx + pk.I_off[i]);
        for (int b = 0; b <= sh.n; ++b) {
            P.blk[b].rowidx = b == 0 ? reinterpret_cast<const int32_t*>(im.d_idx + pk.rowidx_off)
                                     : nullptr;
            P.blk[b].colx = reinterpret_cast<const int64_t*>(im.d_idx + pk.colx_off[b]);
            P.blk[b].cidx = reinterpret_cast<const int32_t*>(im.d_idx + pk.cidx_off[b]);
        }
        return expand_cols(pk, nullptr);
    }

    // The product blocks' column data from the I_i now in the index region.
    int expand_cols(const IdxPack& pk, const DevState* stp) {
        if (!pk.prod_mask) return 0;
        int64_t cmax = 0;
        for (int b = 0; b < im.P.nblk; ++b)
            if ((pk.prod_mask >> b) & 1) cmax = std::max<int64_t>(cmax, im.P.blk[b].ncols);
        const unsigned gx = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>(256, (cmax + kThreads - 1) / kThreads));
        hipLaunchKernelGGL(k_expand_cols, dim3(gx, im.P.nblk), dim3(kThreads), 0, s, im.P,
                           pk.prod_mask, stp);
        HIPCHK(hipGetLastError());
        return 0;
    }

    // Queue a sample's index data for an iteration ahead (RTCUR-R): packed
    // into pinned slot `slot`, copied to its device slot in stream order and
    // taken into the index region by k_take_sample unless the loop stopped.
    int stage_sample(const SampleHost& smp, const Shape& sh, int slot) {
        IdxPack pk;
        index_layout(sh, pk);
        if (pk.bytes != im.idx_bytes || im.idx_bytes % 16) {
            h->last_error = "internal: index layout changed";
            return RTCUR_E_STATE;
        }
        const size_t need = (size_t)kRChunk * im.idx_bytes;
        if (need > im.stage_bytes) {
            if (im.d_stage) HIPCHK(hipFree(im.d_stage));
            if (im.h_stage) HIPCHK(hipHostFree(im.h_stage));
            im.d_stage = im.h_stage = nullptr;
            im.stage_bytes = 0;
            if (hipMalloc(reinterpret_cast<void**>(&im.d_stage), need) != hipSuccess ||
                hipHostMalloc(reinterpret_cast<void**>(&im.h_stage), need,
                              hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                h->last_error = "staging allocation failed";
                return RTCUR_E_NOMEM;
            }
            im.stage_bytes = need;
        }
        char* hs = im.h_stage + (size_t)slot * im.idx_bytes;
        char* ds = im.d_stage + (size_t)slot * im.idx_bytes;
        pack_indices(sh, smp, pk, hs);
        HIPCHK(hipMemcpyAsync(ds, hs, pk.host_bytes, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_take_sample, dim3(64), dim3(kThreads), 0, s,
                           reinterpret_cast<uint4*>(im.d_idx), reinterpret_cast<const uint4*>(ds),
                           (int64_t)(pk.host_bytes / 16), (const DevState*)im.st);
        HIPCHK(hipGetLastError());
        return expand_cols(pk, im.st);
    }

    // Set-up of a solve: sample, loop state, zeroed factors, zeta_0 and the
    // first gather (with the denominator of e^(k)).
    int start(const void* X, int xdt, const Shape& sh, double zeta0, uint64_t seed) {
        int rc;
        im.recs.clear();
        im.ev_used = 0;
        // the threshold schedule (multipliers of zeta_0), at most max_iter of
        // them; a pageable copy, finished before the call returns
        const int ns = (int)std::min<size_t>(h->sched.size(), im.hist_len - 2);
        im.P.zsched = im.zsched;
        im.P.nsched = ns;
        if (ns > 0)
            HIPCHK(hipMemcpyAsync(im.zsched, h->sched.data(), sizeof(double) * ns,
                                  hipMemcpyHostToDevice, s));
        draw_sample(seed, 0, sh, sh.chidori, h->sample, false);
        if ((rc = upload_sample(h->sample, sh))) return rc;
        hipLaunchKernelGGL(k_init_state, dim3(16), dim3(kThreads), 0, s, im.st,
                           zeta0 > 0 ? zeta0 : 0.0, static_cast<uint32_t*>(im.Bf),
                           (int64_t)(im.bf_elems * sizeof(T) / 4), im.Bd, im.bf_elems, im.Gd,
                           im.P.core, im.err_hist, (int)im.hist_len);
        HIPCHK(hipGetLastError());
        if (!(zeta0 > 0)) {
            int64_t N = 1;
            for (int i = 0; i < sh.n; ++i) N *= sh.d[i];
            HIPCHK(pb(PK_ABSMAX));
            if (xdt == RTCUR_F64)
                hipLaunchKernelGGL((k_absmax<double>), dim3(kAbsmaxWG), dim3(kThreads), 0, s,
                                   (const double*)X, N, im.part);
            else
                hipLaunchKernelGGL((k_absmax<float>), dim3(kAbsmaxWG), dim3(kThreads), 0, s,
                                   (const float*)X, N, im.part);
            HIPCHK(hipGetLastError());
            hipLaunchKernelGGL(k_absmax_fin, dim3(1), dim3(kThreads), 0, s,
                               (const double*)im.part, kAbsmaxWG, im.st);
            HIPCHK(hipGetLastError());
            HIPCHK(pe());
        }
        return gather(X, xdt, kFirstGather);
    }

    int run(const void* X, int xdt, const Shape& sh, double zeta0, double gamma,
            double tol, int max_iter, uint64_t seed) {
        const bool resample = h->variant == RTCUR_RESAMPLE;
        int rc;
        if ((rc = start(X, xdt, sh, zeta0, seed))) return rc;
        DevState ds;
        const bool skip = tol >= 1.0;  // e^(0) = 1 <= tol: no iteration
        if (!skip) {
            rc = resample ? loop_resample(X, xdt, sh, gamma, tol, max_iter, seed, ds)
                          : loop_fixed(gamma, tol, max_iter, ds, 0);
            if (rc) return rc;
        } else if ((rc = read_state(ds))) {
            return rc;
        }
        return finish(ds, skip, gamma, tol, max_iter);
    }

    // Histories, profile totals and the summary of the returned iterate.
    int finish(const DevState& ds, bool skip, double gamma, double tol, int max_iter) {
        int rc;
        if (ds.status < 0) {
            h->last_error = ds.status == RTCUR_E_RANK ? "U_i has numerical rank below r_i"
                                                      : "non-finite value in X or e^(k)";
            h->have_result = false;
            im.recs.clear();
            im.ev_used = 0;
            return ds.status;
        }
        int K = ds.stop ? ds.final_iter : max_iter;
        if (skip) K = 0;
        if ((rc = prof_collect(K))) return rc;
        im.final_iter = K;
        im.cur = K % 2;
        // histories
        h->err_hist.assign(K, 0.0);
        if (K > 0) {
            // every path reads the state (and the history behind it) last
            const double* eh = reinterpret_cast<const double*>(
                reinterpret_cast<const char*>(im.st_host) +
                (reinterpret_cast<const char*>(im.err_hist) - reinterpret_cast<const char*>(im.st)));
            for (int j = 1; j <= K; ++j) h->err_hist[j - 1] = eh[j];
        }
        h->zeta_hist.assign(K, 0.0);
        // the thresholds the kernels used: the schedule's multipliers of
        // zeta_0, then the decay by gamma from the last of them
        const int ns = im.P.nsched;
        double z = ds.zeta0;
        for (int j = 0; j < K; ++j) {
            if (j < ns) {
                z = ds.zeta0 * h->sched[(size_t)j];
            } else {
                z *= gamma;
            }
            h->zeta_hist[j] = z;
        }
        rtcur_info& info = h->info;
        info.iters = K;
        info.err = K > 0 ? h->err_hist[K - 1] : (ds.den == 0.0 ? 0.0 : 1.0);
        info.converged = (K > 0 ? info.err <= tol : (tol >= 1.0 || ds.den == 0.0)) ? 1 : 0;
        info.zeta = K > 0 ? h->zeta_hist[K - 1] : ds.zeta0;
        info.zeta0 = ds.zeta0;
        info.eig_steps = ds.eig_steps;
        info.eig_unconverged = ds.eig_unconverged;
        info.status = info.converged ? RTCUR_OK : RTCUR_NOT_CONVERGED;
        h->have_result = true;
        return info.status;
    }

    // Continue the loop from iterate k0 with the blocks re-gathered in this
    // runner's block type (the FP32 refinement sweep).
    int resume(const void* X, int xdt) {
        hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s, im.st);
        HIPCHK(hipGetLastError());
        return gather(X, xdt, 0);
    }

    // The returned iterate's blocks in float after bfloat16 iterations: X_Omega
    // re-gathered, C^K widened (through the other C buffer).
    int widen(const void* X, int xdt, int K) {
        int rc;
        if ((rc = gather(X, xdt, 0))) return rc;
        if (K > 0) {
            const int64_t N = im.nblk_elems;
            float* tmp = static_cast<float*>(im.C[(K + 1) % 2]);
            hipLaunchKernelGGL(k_widen, dim3(1024), dim3(kThreads), 0, s,
                               static_cast<const __hip_bfloat16*>(im.C[K % 2]), N, tmp);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(im.C[K % 2], tmp, sizeof(float) * N, hipMemcpyDeviceToDevice,
                                  s));
        }
        return 0;
    }

    // C^j lives in C[j % 2]; C^0 is X_Omega itself.
    TB* cbuf(int j) { return j == 0 ? (TB*)im.XO : (TB*)im.C[j % 2]; }

    // The steady-state iteration pair as one executable graph: iterations j
    // (odd, C^{j-1} in C[0]) and j + 1, every error and decision formed, k
    // taken from the device's count (launch argument -1).  Captured on the
    // handle's own capture stream (the caller's stream may be the null
    // stream, which cannot be captured) and kept while the launches would be
    // the same: runner type, gamma, tol, the arena and the whole layout.
    // Sets *out to null when capturing is not possible (then the iterations
    // are launched one by one).
    int pair_graph(double gamma, double tol, hipGraphExec_t* out) {
        *out = nullptr;
        if (im.graph_off) return 0;
        std::vector<char> key(sizeof(int) * 3 + sizeof(double) * 2 + sizeof(void*) + sizeof(Prob));
        {
            char* q = key.data();
            const int tp[3] = {(int)sizeof(T), RP, (int)sizeof(TB)};
            const void* ar = im.arena;
            std::memcpy(q, tp, sizeof(tp));
            q += sizeof(tp);
            std::memcpy(q, &gamma, sizeof(double));
            q += sizeof(double);
            std::memcpy(q, &tol, sizeof(double));
            q += sizeof(double);
            std::memcpy(q, &ar, sizeof(void*));
            q += sizeof(void*);
            std::memcpy(q, &im.P, sizeof(Prob));
        }
        for (auto& g : im.graphs)
            if (g.key == key) {
                *out = g.exec;
                return 0;
            }
        if (im.graphs.size() >= 2) {
            HIPCHK(hipStreamSynchronize(s));  // no replay of it still queued
            HIPCHK(hipGraphExecDestroy(im.graphs.front().exec));
            im.graphs.erase(im.graphs.begin());
        }
        if (!im.cstream) HIPCHK(hipStreamCreateWithFlags(&im.cstream, hipStreamNonBlocking));
        const hipStream_t s0 = s;
        if (hipStreamBeginCapture(im.cstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            im.graph_off = true;
            return 0;
        }
        s = im.cstream;
        const int flags = kDoHT | kHaveL | kDoE | kDecide;
        int rc = ht(-1, flags, (TB*)im.C[0], (TB*)im.C[1], im.mask[1], gamma);
        if (!rc) rc = lupdate((TB*)im.C[1], 1, 1, -1, tol);
        if (!rc) rc = ht(-1, flags, (TB*)im.C[1], (TB*)im.C[0], im.mask[0], gamma);
        if (!rc) rc = lupdate((TB*)im.C[0], 1, 1, -1, tol);
        s = s0;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(im.cstream, &g);
        hipError_t ei = hipErrorUnknown;
        hipGraphExec_t ex = nullptr;
        if (!rc && ec == hipSuccess && g) ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (rc || ec != hipSuccess || ei != hipSuccess) {
            (void)hipGetLastError();
            im.graph_off = true;
            return rc;
        }
        im.graphs.push_back(Impl::PairGraph{std::move(key), ex});
        *out = ex;
        return 0;
    }

    // Iterations j0 + 1 .. (stop or max_iter).  The first of them has no
    // e^(j0) to form when j0 > 0 (it was formed before the loop was resumed).
    // Iterations are queued in chunks (4 first, then as many as the observed
    // decay of e^(k) predicts, at most 12); the host reads the device state
    // once per chunk.  A stop raised inside a chunk makes its remaining
    // launches return at once.
    int loop_fixed(double gamma, double tol, int max_iter, DevState& ds, int j0) {
        int done = j0;
        int rc;
        double e_prev = -1.0, e_last = -1.0;
        while (done < max_iter) {
            int chunk = done - j0 < 4 ? 4 : 8;
            if (e_last > 0 && e_prev > 0 && e_last < e_prev) {
                const double rate = e_last / e_prev;
                const double need = std::log(tol / e_last) / std::log(rate);
                if (std::isfinite(need)) chunk = (int)std::min(12.0, std::max(1.0, std::ceil(need)));
            }
            chunk = std::min(chunk, max_iter - done);
            for (int q = 0; q < chunk;) {
                const int j = done + 1 + q;  // iteration j computes S^j, L^j
                tag = j;
                // steady state from an odd j >= 3 on (C^{j-1} in C[0], every
                // error formed): the rest of the chunk as replayed pairs, with
                // the device's iteration count set to j - 1 first
                if (h->graphs && h->prof_mask == 0 && j % 2 == 1 && j >= 3 && j >= j0 + 2 &&
                    chunk - q >= 2) {
                    hipGraphExec_t gx = nullptr;
                    if ((rc = pair_graph(gamma, tol, &gx))) return rc;
                    if (gx) {
                        hipLaunchKernelGGL(k_set_iter, dim3(1), dim3(64), 0, s, im.st, j - 1);
                        HIPCHK(hipGetLastError());
                        const int np = (chunk - q) / 2;
                        for (int p = 0; p < np; ++p) HIPCHK(hipGraphLaunch(gx, s));
                        q += 2 * np;
                        continue;
                    }
                }
                const bool err = j > 1 && j > j0 + 1;  // e^(j-1) formed here
                const int flags = kDoHT | (j > 1 ? kHaveL : 0) | (err ? (kDoE | kDecide) : 0);
                if ((rc = ht(j - 1, flags, cbuf(j - 1), cbuf(j), im.mask[j % 2], gamma)))
                    return rc;
                if ((rc = lupdate(cbuf(j), j > 1 ? 1 : 0, err ? 1 : 0, j - 1, tol))) return rc;
                ++q;
            }
            done += chunk;
            if ((rc = read_state(ds))) return rc;
            if (ds.stop) return 0;
            e_prev = ds.e_prev;
            e_last = ds.e_last;
        }
        // e^(max_iter): one error-only pass
        tag = max_iter + 1;
        if ((rc = ht(max_iter, kHaveL | kDoE | kDecide, cbuf(max_iter), nullptr, nullptr, gamma)))
            return rc;
        if ((rc = decide(max_iter, tol))) return rc;
        return read_state(ds);
    }

    // RTCUR-R with iterations queued in chunks as under RTCUR-F: the host
    // draws the chunk's samples ahead and stages their index data; a stop
    // raised inside the chunk makes the rest of it (sample take, gathers and
    // kernels) return at once, so the device keeps the returned iterate's
    // sample and blocks, and the host keeps that sample too.
    int loop_resample(const void* X, int xdt, const Shape& sh, double gamma, double tol,
                      int max_iter, uint64_t seed, DevState& ds) {
        int rc;
        std::vector<SampleHost> smp(kRChunk);
        int done = 0;
        double e_prev = -1.0, e_last = -1.0;
        while (done < max_iter) {
            int chunk = done < 4 ? 4 : kRChunk;
            if (e_last > 0 && e_prev > 0 && e_last < e_prev) {
                const double rate = e_last / e_prev;
                const double need = std::log(tol / e_last) / std::log(rate);
                if (std::isfinite(need))
                    chunk = (int)std::min<double>(kRChunk, std::max(1.0, std::ceil(need)));
            }
            chunk = std::min(chunk, max_iter - done);
            for (int q = 0; q < chunk; ++q) {
                const int j = done + 1 + q;
                tag = j;
                if (j > 1) {
                    // new sample (t = j-1), gather there, L^(j-1) on its columns
                    draw_sample(seed, j - 1, sh, sh.chidori, smp[q], false);
                    if ((rc = stage_sample(smp[q], sh, q))) return rc;
                    if ((rc = gather(X, xdt, kIfRunning))) return rc;
                    if ((rc = hexp())) return rc;
                }
                const int flags = kDoHT | (j > 1 ? kHaveL : 0);
                if ((rc = ht(j - 1, flags, nullptr, cbuf(j), im.mask[j % 2], gamma))) return rc;
                // the eigensolver starts from the previous factors' rows at the
                // new sample (j > 1)
                if ((rc = lupdate(cbuf(j), j > 1 ? 2 : 0, 0, j - 1, tol))) return rc;
                // e^(j) on this sample
                if ((rc = ht(j, kHaveL | kDoE | kDecide, cbuf(j), nullptr, nullptr, gamma)))
                    return rc;
                if ((rc = decide(j, tol))) return rc;
            }
            if ((rc = read_state(ds))) return rc;
            const int last = ds.stop ? ds.final_iter : done + chunk;
            // iteration j > 1 of this chunk drew smp[j - done - 1]; iteration 1
            // kept the sample of the set-up
            if (last > 1 && last > done && last <= done + chunk)
                h->sample = std::move(smp[last - done - 1]);
            if (ds.stop) return 0;
            done += chunk;
            e_prev = ds.e_prev;
            e_last = ds.e_last;
        }
        return 0;
    }
};

// Lay out the arena for this problem and point every region into it.
// ---------------------------------------------------------- tile autotuner
// Process-wide table: problem sizes (and block element size) -> the tile
// shapes the autotuner found fastest for them.
static std::mutex g_tune_mu;
static std::map<std::vector<int64_t>, Tune> g_tune;

static std::vector<int64_t> tune_key(const Shape& sh, int esize) {
    std::vector<int64_t> key = {sh.n, sh.chidori ? 1 : 0, esize};
    for (int i = 0; i < sh.n; ++i) {
        key.push_back(sh.d[i]);
        key.push_back(sh.r[i]);
        key.push_back(sh.s[i]);
        key.push_back(sh.m[i]);
    }
    return key;
}

static Tune tuned_for(const Shape& sh, int esize) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(sh, esize));
    return it == g_tune.end() ? Tune{} : it->second;
}

void autotune_clear() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

template <typename T>
static int prepare(rtcur_s* h, Impl& im, const Shape& sh, int max_iter) {
    IdxPack pk;
    index_layout(sh, pk);
    // the layout and work lists depend on the sizes and the tile shapes only:
    // a solve of the same sizes as the previous one on this handle reuses
    // them.  Tile shapes: the autotuner's candidate while it runs, else the
    // caller's (rtcur_set_tiles), else the table's entry for these sizes,
    // else the built-in rule.
    const Tune tune = h->tune_forced     ? h->tune_force
                      : h->tune_user_set ? h->tune_user
                                         : tuned_for(sh, (int)sizeof(T));
    std::vector<int64_t> key = tune_key(sh, (int)sizeof(T));
    key.push_back(max_iter);
    key.push_back((int64_t)pk.bytes);
    key.push_back(tune.ht_rows);
    key.push_back(tune.gram_chunk);
    key.push_back(tune.bfac_sub);
    if (im.arena && key == im.plan_key) return 0;
    im.plan_key.clear();
    Arena ar;
    Regions rg;
    plan(im, sh, sizeof(T), pk.bytes, max_iter, tune, ar, rg);
    if (ar.total > im.arena_bytes) {
        if (im.arena) HIPCHK(hipFree(im.arena));
        im.arena = nullptr;
        im.arena_bytes = 0;
        hipError_t e = hipMalloc(&im.arena, ar.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            im.arena = nullptr;
            h->last_error = "device workspace allocation failed";
            return RTCUR_E_NOMEM;
        }
        im.arena_bytes = ar.total;
    }
    char* a = static_cast<char*>(im.arena);
    auto dp = [&](size_t off) { return reinterpret_cast<double*>(a + off); };
    im.XO = a + rg.XO;
    im.C[0] = a + rg.C0;
    im.C[1] = a + rg.C1;
    im.mask[0] = reinterpret_cast<uint64_t*>(a + rg.m0);
    im.mask[1] = reinterpret_cast<uint64_t*>(a + rg.m1);
    im.Bf = a + rg.Bf;
    im.H = a + rg.H;
    im.W = dp(rg.W);
    im.Y = dp(rg.Y);
    im.Z = dp(rg.Z);
    im.gram = dp(rg.gram);
    im.gpart = dp(rg.gpart);
    im.bpart = dp(rg.bpart);
    im.Bd = dp(rg.Bd);
    im.Gd = dp(rg.Gd);
    im.Tc = dp(rg.Tc);
    im.part = dp(rg.part);
    im.hpart = dp(rg.hpart);
    im.err_hist = dp(rg.hist);
    im.st = reinterpret_cast<DevState*>(a + rg.st);
    char* t = a + rg.tiles;
    im.d_ht_tiles = reinterpret_cast<int4*>(t);
    t += sizeof(int4) * im.ht_tiles.size();
    im.d_gram_items = reinterpret_cast<int4*>(t);
    t += sizeof(int4) * im.gram_items.size();
    im.d_bfac_items = reinterpret_cast<int4*>(t);
    t += sizeof(int4) * im.bfac_items.size();
    im.d_z_tiles = reinterpret_cast<int2*>(t);
    t += sizeof(int2) * im.z_tiles.size();
    im.d_h_tiles = reinterpret_cast<int2*>(t);
    im.d_idx = a + rg.idx;
    im.idx_bytes = pk.bytes;
    im.zsched = dp(rg.zs);
    // work lists (one upload)
    std::vector<char> tb(sizeof(int4) * (im.ht_tiles.size() + im.gram_items.size() +
                                         im.bfac_items.size()) +
                         sizeof(int2) * (im.z_tiles.size() + im.h_tiles.size()));
    char* q = tb.data();
    auto put = [&](const void* src, size_t bytes) {
        if (bytes) std::memcpy(q, src, bytes);
        q += bytes;
    };
    put(im.ht_tiles.data(), sizeof(int4) * im.ht_tiles.size());
    put(im.gram_items.data(), sizeof(int4) * im.gram_items.size());
    put(im.bfac_items.data(), sizeof(int4) * im.bfac_items.size());
    put(im.z_tiles.data(), sizeof(int2) * im.z_tiles.size());
    put(im.h_tiles.data(), sizeof(int2) * im.h_tiles.size());
    HIPCHK(hipMemcpyAsync(a + rg.tiles, tb.data(), tb.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    im.plan_key = std::move(key);
    return 0;
}

// RTCUR_BF16: the blocks in bfloat16 (factors, arithmetic and L in float;
// Gram, eigensolver and norms in float64) until e^(k) <= max(tol,
// kBf16Switch), then the FP32 refinement sweep continues from that iterate
// with the blocks re-gathered in float until e^(k) <= tol.
constexpr double kBf16Switch = 1e-2;

template <int RP>
static int run_bf16(rtcur_s* h, Impl& im, const void* X, int xdt, const Shape& sh,
                    double zeta0, double gamma, double tol, int max_iter, uint64_t seed) {
    Runner<float, RP, __hip_bfloat16> R1{h, im, h->stream};
    Runner<float, RP, float> R2{h, im, h->stream};
    int rc;
    if ((rc = R1.start(X, xdt, sh, zeta0, seed))) return rc;
    DevState ds;
    const bool skip = tol >= 1.0;
    if (skip) {
        if ((rc = R2.widen(X, xdt, 0)) || (rc = R2.read_state(ds))) return rc;
        return R2.finish(ds, true, gamma, tol, max_iter);
    }
    if ((rc = R1.loop_fixed(gamma, std::max(tol, kBf16Switch), max_iter, ds, 0))) return rc;
    if (ds.status < 0) return R2.finish(ds, false, gamma, tol, max_iter);
    const int k1 = ds.stop ? ds.final_iter : max_iter;
    double e1 = 1.0;
    if (k1 > 0)
        HIPCHK(hipMemcpy(&e1, im.err_hist + k1, sizeof(double), hipMemcpyDeviceToHost));
    if (k1 >= max_iter || e1 <= tol || (ds.stop && ds.final_iter == 0)) {
        if ((rc = R2.widen(X, xdt, k1)) || (rc = R2.read_state(ds))) return rc;
        return R2.finish(ds, false, gamma, tol, max_iter);
    }
    if ((rc = R2.resume(X, xdt))) return rc;
    if ((rc = R2.loop_fixed(gamma, tol, max_iter, ds, k1))) return rc;
    return R2.finish(ds, false, gamma, tol, max_iter);
}

template <typename T, int RP>
static int run_rp(rtcur_s* h, Impl& im, const void* X, int xdt, const Shape& sh,
                  double zeta0, double gamma, double tol, int max_iter, uint64_t seed) {
    if constexpr (std::is_same<T, float>::value) {
        if (h->dtype == RTCUR_BF16)
            return run_bf16<RP>(h, im, X, xdt, sh, zeta0, gamma, tol, max_iter, seed);
    }
    Runner<T, RP> R{h, im, h->stream};
    return R.run(X, xdt, sh, zeta0, gamma, tol, max_iter, seed);
}

template <typename T>
static int run_t(rtcur_s* h, Impl& im, const void* X, int xdt, const Shape& sh,
                 double zeta0, double gamma, double tol, int max_iter, uint64_t seed) {
    int rc = prepare<T>(h, im, sh, max_iter);
    if (rc) return rc;
    switch (im.P.rp) {
        case 4: return run_rp<T, 4>(h, im, X, xdt, sh, zeta0, gamma, tol, max_iter, seed);
        case 8: return run_rp<T, 8>(h, im, X, xdt, sh, zeta0, gamma, tol, max_iter, seed);
        default: return run_rp<T, 16>(h, im, X, xdt, sh, zeta0, gamma, tol, max_iter, seed);
    }
}

int solve(rtcur_s* h, const void* X, int x_dtype, const Shape& sh, double zeta0,
          double gamma, double tol, int max_iter, uint64_t seed) {
    Impl& im = *impl_of(h);
    h->have_result = false;
    HIPCHK(hipSetDevice(h->device));
    if (!im.max_dyn_set) {
        im.max_dyn_set = true;
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, h->device));
        // k_eig keeps the Gram in dynamic LDS when it fits beside its
        // static arrays
        const void* fns[3] = {reinterpret_cast<const void*>(k_eig<4, true>),
                              reinterpret_cast<const void*>(k_eig<8, true>),
                              reinterpret_cast<const void*>(k_eig<16, true>)};
        for (int k = 0; k < 3; ++k) {
            hipFuncAttributes fa;
            int room = 0;
            if (hipFuncGetAttributes(&fa, fns[k]) == hipSuccess)
                room = (int)prop.sharedMemPerBlock - (int)fa.sharedSizeBytes - 1024;
            if (room > 0 && hipFuncSetAttribute(fns[k], hipFuncAttributeMaxDynamicSharedMemorySize,
                                                room) != hipSuccess)
                room = 0;
            (void)hipGetLastError();  // a refused attribute leaves a sticky error
            im.max_dyn_lds[k] = room > 0 ? room : 0;
        }
    }
    h->shape = sh;
    if (h->dtype == RTCUR_F64)
        return run_t<double>(h, im, X, x_dtype, sh, zeta0, gamma, tol, max_iter, seed);
    return run_t<float>(h, im, X, x_dtype, sh, zeta0, gamma, tol, max_iter, seed);
}

// Coordinate descent over the tile shapes, one at a time from the built-in
// rule: rows per gather / threshold tile, then the Gram's column chunk, then
// the B-factor sub-chunks; a candidate whose work lists equal one already
// timed is skipped.  Each candidate: one warm-up solve (layout, graph
// capture), then the best of `reps` timed solves of `iters` iterations
// (tol 0, so every candidate does the same iterations), host wall clock.
int autotune(rtcur_s* h, const void* X, int x_dtype, const Shape& sh, int iters, int reps,
             uint64_t seed, Tune* best, double* best_ms, double* default_ms) {
    const int esize = h->dtype == RTCUR_F64 ? 8 : 4;
    int rc = 0;
    auto time_of = [&](const Tune& t, double* ms) -> int {
        h->tune_forced = true;
        h->tune_force = t;
        int r = solve(h, X, x_dtype, sh, 0.0, 0.7, 0.0, iters, seed);
        double bt = 1e300;
        for (int q = 0; q < reps && r >= 0; ++q) {
            const auto t0 = std::chrono::steady_clock::now();
            r = solve(h, X, x_dtype, sh, 0.0, 0.7, 0.0, iters, seed);
            const double dt = std::chrono::duration<double, std::milli>(
                                  std::chrono::steady_clock::now() - t0).count();
            bt = std::min(bt, dt);
        }
        h->tune_forced = false;
        *ms = bt;
        return r < 0 ? r : 0;
    };
    // the work split a tune gives (to skip candidates equal to one timed)
    auto gram_split = [&](const Tune& t) {
        std::vector<int> v;
        for (int i = 0; i < sh.n; ++i) {
            const int nt = (int)((sh.s[i] + 15) / 16), npi = nt * (nt + 1) / 2;
            int nkc;
            if (t.gram_chunk > 0) {
                nkc = std::max(1, (int)std::min<int64_t>(kGramMaxKC, (sh.m[i] + t.gram_chunk - 1) /
                                                                         t.gram_chunk));
            } else {
                nkc = (int)std::min<int64_t>(kGramMaxKC, (sh.m[i] + kGramMinChunk - 1) /
                                                             kGramMinChunk);
                nkc = std::max(1, std::min(nkc, std::max(kGramKCGroup, 1024 / npi)));
            }
            v.push_back(nkc);
        }
        return v;
    };
    int rmax = 1;
    for (int i = 0; i < sh.n; ++i) rmax = std::max(rmax, sh.r[i]);
    const int bkc = bfac_kc(pad_rank(rmax));
    auto bfac_split = [&](const Tune& t) {
        std::vector<int> v;
        for (int i = 0; i < sh.n; ++i) {
            const int nsc = (int)((sh.m[i] + bkc - 1) / bkc);
            v.push_back(std::min(nsc, std::max((nsc + kBfacMaxKC - 1) / kBfacMaxKC, t.bfac_sub)));
        }
        return v;
    };
    Tune cur;
    cur.ht_rows = kTileRows;
    double cur_ms = 0.0;
    if ((rc = time_of(cur, &cur_ms))) return rc;
    *default_ms = cur_ms;
    auto consider = [&](const Tune& t) -> int {
        double ms = 0.0;
        const int r = time_of(t, &ms);
        if (r) return r;
        if (ms < cur_ms) {
            cur = t;
            cur_ms = ms;
        }
        return 0;
    };
    for (int tr : {8, 32}) {
        if (esize == 8 && tr == 32) continue;
        Tune t = cur;
        t.ht_rows = tr;
        if ((rc = consider(t))) return rc;
    }
    {
        std::vector<std::vector<int>> seen = {gram_split(cur)};
        const Tune base = cur;
        for (int c : {512, 1024, 2048, 4096, 8192}) {
            Tune t = base;
            t.gram_chunk = c;
            const std::vector<int> v = gram_split(t);
            if (std::find(seen.begin(), seen.end(), v) != seen.end()) continue;
            seen.push_back(v);
            if ((rc = consider(t))) return rc;
        }
    }
    {
        std::vector<std::vector<int>> seen = {bfac_split(cur)};
        const Tune base = cur;
        for (int b : {2, 4, 8}) {
            Tune t = base;
            t.bfac_sub = b;
            const std::vector<int> v = bfac_split(t);
            if (std::find(seen.begin(), seen.end(), v) != seen.end()) continue;
            seen.push_back(v);
            if ((rc = consider(t))) return rc;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(sh, esize)] = cur;
    }
    *best = cur;
    *best_ms = cur_ms;
    return 0;
}

// ------------------------------------------------------------ outputs

static int ensure_scratch(rtcur_s* h, Impl& im, size_t bytes) {
    if (bytes <= im.scratch_bytes) return 0;
    if (im.scratch) HIPCHK(hipFree(im.scratch));
    im.scratch = nullptr;
    im.scratch_bytes = 0;
    if (hipMalloc(&im.scratch, bytes) != hipSuccess) {
        (void)hipGetLastError();
        h->last_error = "scratch allocation failed";
        return RTCUR_E_NOMEM;
    }
    im.scratch_bytes = bytes;
    return 0;
}

// H of the full mode-0 unfolding (RP x prod_{j>0} d_j) into the scratch
// buffer, for the dense reconstruction and the full-grid outliers.
template <typename T, int RP>
static int dense_h(rtcur_s* h, Impl& im, int64_t ncols, T** Hf_out) {
    const Prob& P = im.P;
    const int64_t ntile = (ncols + kThreads - 1) / kThreads;
    size_t need = align_up(sizeof(T) * RP * ncols, 256) + sizeof(int2) * ntile + 256;
    int rc = ensure_scratch(h, im, need);
    if (rc) return rc;
    T* Hf = static_cast<T*>(im.scratch);
    int2* tiles = reinterpret_cast<int2*>(static_cast<char*>(im.scratch) +
                                          align_up(sizeof(T) * RP * ncols, 256));
    std::vector<int2> tl(ntile);
    for (int64_t q = 0; q < ntile; ++q) tl[q] = make_int2(-1, (int)q);
    HIPCHK(hipMemcpyAsync(tiles, tl.data(), sizeof(int2) * ntile, hipMemcpyHostToDevice,
                          h->stream));
    launch_hexp<T, RP>(P, true, (unsigned)ntile, h->stream, tiles, (const T*)im.Bf, im.Gd, Hf,
                       (const DevState*)nullptr, 0, ncols);
    HIPCHK(hipGetLastError());
    *Hf_out = Hf;
    return 0;
}

template <typename T, typename TO, int RP>
static int recon_t(rtcur_s* h, Impl& im, void* out) {
    const Prob& P = im.P;
    int64_t ncols = 1;
    for (int j = 1; j < P.n; ++j) ncols *= P.d[j];
    const int64_t total = ncols * P.d[0];
    if (im.final_iter == 0) {
        HIPCHK(hipMemsetAsync(out, 0, total * sizeof(TO), h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        return 0;
    }
    T* Hf = nullptr;
    int rc = dense_h<T, RP>(h, im, ncols, &Hf);
    if (rc) return rc;
    const int64_t ntile = (ncols + kThreads - 1) / kThreads;
    dim3 grid((unsigned)ntile, (unsigned)((P.d[0] + kTileRows - 1) / kTileRows));
    hipLaunchKernelGGL((k_recon<T, TO, RP>), grid, dim3(kThreads), 0, h->stream, P.d[0],
                       ncols, (const T*)im.Bf + P.boff[0], (const T*)Hf, (TO*)out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return 0;
}

template <typename T>
static int recon_rp(rtcur_s* h, Impl& im, void* out, int odt) {
    switch (im.P.rp) {
        case 4: return odt == RTCUR_F64 ? recon_t<T, double, 4>(h, im, out) : recon_t<T, float, 4>(h, im, out);
        case 8: return odt == RTCUR_F64 ? recon_t<T, double, 8>(h, im, out) : recon_t<T, float, 8>(h, im, out);
        default: return odt == RTCUR_F64 ? recon_t<T, double, 16>(h, im, out) : recon_t<T, float, 16>(h, im, out);
    }
}

// Full-grid outliers S = HT_zeta(X - L) and optionally L itself, in one pass.
template <typename T, typename TX, typename TO, int RP>
static int outl_t(rtcur_s* h, Impl& im, const void* X, double zeta, void* S, void* L) {
    const Prob& P = im.P;
    int64_t ncols = 1;
    for (int j = 1; j < P.n; ++j) ncols *= P.d[j];
    T* Hf = nullptr;
    const T* B0 = (const T*)im.Bf + P.boff[0];
    if (im.final_iter == 0) {
        // L = 0: H = 0 (B is never read then: H zero makes every L zero)
        const size_t need = align_up(sizeof(T) * RP * ncols, 256) + 256;
        int rc = ensure_scratch(h, im, need);
        if (rc) return rc;
        Hf = static_cast<T*>(im.scratch);
        HIPCHK(hipMemsetAsync(Hf, 0, sizeof(T) * RP * ncols, h->stream));
    } else {
        int rc = dense_h<T, RP>(h, im, ncols, &Hf);
        if (rc) return rc;
    }
    const int64_t ntile = (ncols + kThreads - 1) / kThreads;
    dim3 grid((unsigned)ntile, (unsigned)((P.d[0] + kTileRows - 1) / kTileRows));
    hipLaunchKernelGGL((k_outliers<T, TX, TO, RP>), grid, dim3(kThreads), 0, h->stream, P.d[0],
                       ncols, B0, (const T*)Hf, (const TX*)X, zeta, (TO*)S, (TO*)L);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return 0;
}

template <typename T, int RP>
static int outl_rp(rtcur_s* h, Impl& im, const void* X, int xdt, double zeta, void* S, void* L,
                   int odt) {
    if (xdt == RTCUR_F64)
        return odt == RTCUR_F64 ? outl_t<T, double, double, RP>(h, im, X, zeta, S, L)
                                : outl_t<T, double, float, RP>(h, im, X, zeta, S, L);
    return odt == RTCUR_F64 ? outl_t<T, float, double, RP>(h, im, X, zeta, S, L)
                            : outl_t<T, float, float, RP>(h, im, X, zeta, S, L);
}

template <typename T>
static int outl_t2(rtcur_s* h, Impl& im, const void* X, int xdt, double zeta, void* S, void* L,
                   int odt) {
    switch (im.P.rp) {
        case 4: return outl_rp<T, 4>(h, im, X, xdt, zeta, S, L, odt);
        case 8: return outl_rp<T, 8>(h, im, X, xdt, zeta, S, L, odt);
        default: return outl_rp<T, 16>(h, im, X, xdt, zeta, S, L, odt);
    }
}

int outliers(rtcur_s* h, const void* X, int x_dtype, double zeta, void* S_out, void* L_out,
             int out_dtype) {
    Impl* im = static_cast<Impl*>(h->impl);
    if (!h->have_result || !im) {
        h->last_error = "no successful solve";
        return RTCUR_E_STATE;
    }
    HIPCHK(hipSetDevice(h->device));
    // default: the threshold of the returned iterate, zeta_K (zeta_0 when K = 0)
    if (!(zeta > 0.0)) zeta = h->info.zeta;
    if (h->dtype == RTCUR_F64)
        return outl_t2<double>(h, *im, X, x_dtype, zeta, S_out, L_out, out_dtype);
    return outl_t2<float>(h, *im, X, x_dtype, zeta, S_out, L_out, out_dtype);
}

int reconstruct(rtcur_s* h, void* out, int out_dtype) {
    Impl* im = static_cast<Impl*>(h->impl);
    if (!h->have_result || !im) {
        h->last_error = "no successful solve to reconstruct";
        return RTCUR_E_STATE;
    }
    HIPCHK(hipSetDevice(h->device));
    if (h->dtype == RTCUR_F64) return recon_rp<double>(h, *im, out, out_dtype);
    return recon_rp<float>(h, *im, out, out_dtype);
}

// The allocation-free reconstruction: the dense H and its tile list in the
// device's static scratch (no hipMalloc, no host-to-device copy, no memset:
// every step is a kernel launch on the handle's stream), queued without
// waiting for the device.
template <typename T, typename TO, int RP>
static int recon_static_t(rtcur_s* h, Impl& im, void* out, char* base) {
    const Prob& P = im.P;
    int64_t ncols = 1;
    for (int j = 1; j < P.n; ++j) ncols *= P.d[j];
    const int64_t total = ncols * P.d[0];
    if (im.final_iter == 0) {
        const unsigned nwg = (unsigned)std::min<int64_t>(4096, (total + kThreads - 1) / kThreads);
        hipLaunchKernelGGL((k_fill_zero<TO>), dim3(std::max(1u, nwg)), dim3(kThreads), 0,
                           h->stream, (TO*)out, total);
        HIPCHK(hipGetLastError());
        return 0;
    }
    const int64_t ntile = (ncols + kThreads - 1) / kThreads;
    const size_t hbytes = align_up(sizeof(T) * RP * (size_t)ncols, 256);
    const size_t need = hbytes + sizeof(int2) * (size_t)ntile;
    if (need > kStaticScratchBytes) {
        h->last_error = "reconstruction needs " + std::to_string(need) +
                        " bytes of scratch; the static scratch holds " +
                        std::to_string(kStaticScratchBytes);
        return RTCUR_E_INVAL;
    }
    T* Hf = reinterpret_cast<T*>(base);
    int2* tiles = reinterpret_cast<int2*>(base + hbytes);
    hipLaunchKernelGGL(k_dense_tiles, dim3((unsigned)((ntile + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, h->stream, tiles, ntile);
    HIPCHK(hipGetLastError());
    launch_hexp<T, RP>(P, true, (unsigned)ntile, h->stream, tiles, (const T*)im.Bf, im.Gd, Hf,
                       (const DevState*)nullptr, 0, ncols);
    HIPCHK(hipGetLastError());
    dim3 grid((unsigned)ntile, (unsigned)((P.d[0] + kTileRows - 1) / kTileRows));
    hipLaunchKernelGGL((k_recon<T, TO, RP>), grid, dim3(kThreads), 0, h->stream, P.d[0],
                       ncols, (const T*)im.Bf + P.boff[0], (const T*)Hf, (TO*)out);
    HIPCHK(hipGetLastError());
    return 0;
}

template <typename T>
static int recon_static_rp(rtcur_s* h, Impl& im, void* out, int odt, char* base) {
    switch (im.P.rp) {
        case 4: return odt == RTCUR_F64 ? recon_static_t<T, double, 4>(h, im, out, base)
                                        : recon_static_t<T, float, 4>(h, im, out, base);
        case 8: return odt == RTCUR_F64 ? recon_static_t<T, double, 8>(h, im, out, base)
                                        : recon_static_t<T, float, 8>(h, im, out, base);
        default: return odt == RTCUR_F64 ? recon_static_t<T, double, 16>(h, im, out, base)
                                         : recon_static_t<T, float, 16>(h, im, out, base);
    }
}

int reconstruct_noalloc(rtcur_s* h, void* out, int out_dtype) {
    Impl* im = static_cast<Impl*>(h->impl);
    if (!h->have_result || !im) {
        h->last_error = "no successful solve to reconstruct";
        return RTCUR_E_STATE;
    }
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(scratch_mu);
        if (h->device >= 0 && h->device < kMaxDevices) base = scratch_dev[h->device];
    }
    if (!base) {
        h->last_error = "static scratch address of this device unknown";
        return RTCUR_E_STATE;
    }
    HIPCHK(hipSetDevice(h->device));
    char* b = static_cast<char*>(base);
    if (h->dtype == RTCUR_F64) return recon_static_rp<double>(h, *im, out, out_dtype, b);
    return recon_static_rp<float>(h, *im, out, out_dtype, b);
}

template <typename T, int RP>
static int block_t(rtcur_s* h, Impl& im, int b, int what, double* dst, int64_t len) {
    const Prob& P = im.P;
    const BlockDev& bd = P.blk[b];
    int rc = ensure_scratch(h, im, sizeof(double) * len + 256);
    if (rc) return rc;
    double* tmp = static_cast<double*>(im.scratch);
    const unsigned nwg = (unsigned)((len + kThreads - 1) / kThreads);
    const int K = im.final_iter;
    if (what == RTCUR_BLOCK_X || (what == RTCUR_BLOCK_C && K == 0)) {
        hipLaunchKernelGGL((k_to_double<T>), dim3(nwg), dim3(kThreads), 0, h->stream,
                           (const T*)im.XO + bd.off, len, tmp);
    } else if (what == RTCUR_BLOCK_C) {
        hipLaunchKernelGGL((k_to_double<T>), dim3(nwg), dim3(kThreads), 0, h->stream,
                           (const T*)im.C[im.cur] + bd.off, len, tmp);
    } else if (K == 0) {
        HIPCHK(hipMemsetAsync(tmp, 0, sizeof(double) * len, h->stream));
    } else if (what == RTCUR_BLOCK_L) {
        hipLaunchKernelGGL((k_evalblock<T, RP>), dim3(nwg), dim3(kThreads), 0, h->stream, P, b,
                           (const T*)im.Bf, (const T*)im.H, tmp);
    } else {
        hipLaunchKernelGGL(k_unpack_mask, dim3(nwg), dim3(kThreads), 0, h->stream,
                           im.mask[im.cur], bd.moff, bd.words, bd.nrows, bd.ncols, tmp);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(dst, tmp, sizeof(double) * len, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return 0;
}

int get_block(rtcur_s* h, int block, int what, double* out, int64_t cap, int64_t* len) {
    Impl* im = static_cast<Impl*>(h->impl);
    if (!h->have_result || !im) {
        h->last_error = "no successful solve";
        return RTCUR_E_STATE;
    }
    if (block < 0 || block > im->P.n || what < 0 || what > 3) {
        h->last_error = "block or what out of range";
        return RTCUR_E_INVAL;
    }
    const BlockDev& bd = im->P.blk[block];
    const int64_t n = (int64_t)bd.nrows * bd.ncols;
    if (len) *len = n;
    if (!out) return 0;
    if (cap < n) {
        h->last_error = "output buffer too small";
        return RTCUR_E_INVAL;
    }
    HIPCHK(hipSetDevice(h->device));
    const int rp = im->P.rp;
    if (h->dtype == RTCUR_F64) {
        if (rp == 4) return block_t<double, 4>(h, *im, block, what, out, n);
        if (rp == 8) return block_t<double, 8>(h, *im, block, what, out, n);
        return block_t<double, 16>(h, *im, block, what, out, n);
    }
    if (rp == 4) return block_t<float, 4>(h, *im, block, what, out, n);
    if (rp == 8) return block_t<float, 8>(h, *im, block, what, out, n);
    return block_t<float, 16>(h, *im, block, what, out, n);
}

int get_tucker(rtcur_s* h, double* core, double* const* B) {
    Impl* im = static_cast<Impl*>(h->impl);
    if (!h->have_result || !im) {
        h->last_error = "no successful solve";
        return RTCUR_E_STATE;
    }
    HIPCHK(hipSetDevice(h->device));
    const Prob& P = im->P;
    if (core)
        HIPCHK(hipMemcpy(core, im->Gd, sizeof(double) * P.core, hipMemcpyDeviceToHost));
    if (B) {
        std::vector<double> tmp((size_t)im->bf_elems);
        HIPCHK(hipMemcpy(tmp.data(), im->Bd, sizeof(double) * im->bf_elems,
                         hipMemcpyDeviceToHost));
        for (int i = 0; i < P.n; ++i) {
            if (!B[i]) continue;
            for (int x = 0; x < P.d[i]; ++x)
                for (int p = 0; p < P.r[i]; ++p)
                    B[i][(size_t)x * P.r[i] + p] =
                        im->final_iter == 0 ? 0.0 : tmp[P.boff[i] + (size_t)x * P.rp + p];
        }
    }
    return 0;
}

}  // namespace rtcur
