// C ABI of libfrg: argument checks, context and workspace ownership, the rhs
// pipeline (bubbles -> operand layout -> channel contractions -> combine) and
// the explicit flow of Eq. (1) in s = ln T with on-device step control.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "frg_internal.h"


// Column tiles of one class: positions (tile order) -> natural columns, the
// combine's map of every natural column to (position << 3) | C4v element, and
// per tile and K part the list of active k chunks.
struct TileSet {
    int ncol = 0;
    int kparts = 1;   // K parts the chunk lists are cut into
    int32_t *d_cperm = nullptr, *d_cmap = nullptr, *d_koff = nullptr, *d_klist = nullptr;
    int64_t chunks = 0;
    // host copies for cutting the lists into another number of K parts: chunk id
    // of every list entry, and where each tile's entries begin (tiles + 1 values)
    std::vector<int32_t> h_chunk, h_begin;
};

// Kernel timing with HIP events (frg_profile_* and frg_batch_profile_*): a pool
// of events and the (class, start, end) records made while it is on.
struct EvProf {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int cls; hipEvent_t a, b; };
    std::vector<Rec> recs;
    hipEvent_t next() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin() { recs.clear(); used = 0; on = true; }
    void destroy() {
        for (hipEvent_t e : pool) hipEventDestroy(e);
        pool.clear();
    }
};

struct frg_ctx_s {
    frg::Geometry g;
    int device = 0;
    int Trows = 0;
    int64_t n3 = 0;
    // temperature-independent device tables
    double *d_bnd = nullptr, *d_xi = nullptr, *d_w = nullptr, *d_trig_row = nullptr,
           *d_trig_pt = nullptr;
    uint8_t *d_bins = nullptr;
    int32_t *d_count = nullptr;   // energy-angle grid: live points per patch
    // self-energy flowing with the vertex: V and F hold N^3 + N doubles (S after V);
    // se_sym: the caller's S is C4v invariant, so the bubble rows stay C4v images
    // of each other and pp/ph pairs (checked at flow start)
    bool se_on = false, se_sym = false;
    bool batch_member = false;    // owned by a batch (frg_batch_context)
    double *d_sigD = nullptr;     // [N] patch sums of the self-energy flow
    int32_t *d_colrow_pp = nullptr, *d_colrow_ph = nullptr;   // (row << 3): every row stored
    // C4v orbit reduction of the bubble rows
    bool sym_avail = false, sym_on = false;
    int n_rep_pp = 0, n_rep_ph = 0;
    std::vector<int32_t> h_rowlist, h_rowlist_ph;   // host copies of the two lists below
    int32_t *d_rowlist = nullptr;      // representative pp rows
    int32_t *d_rowlist_ph = nullptr;   // per representative pp row q: the ph row of -q (its pair)
    int32_t *d_colsym_pp = nullptr, *d_colsym_ph = nullptr;   // (compact rep << 3) | element
    // column tiles of the contraction, per class ([0]: pp columns, [1]: ph):
    // all columns in Hilbert order with their active 8-wide k chunks (ts_full);
    // one column per C4v orbit of column pairs, for a C4v-invariant vertex
    // (ts_vsym); all columns in natural order with every chunk (ts_dense, made
    // on demand)
    bool kskip_on = true;
    bool vsym_on = false;
    // interaction flow: the context's bubble buffer holds L_T for this T and
    // precision (set by frg_iflow_init, cleared by any other bubble sweep into it)
    double iflow_T = 0.0;
    int iflow_prec = -1;
    TileSet ts_full[2], ts_vsym[2], ts_dense[2];
    int16_t *d_perm8 = nullptr;   // [8][N] C4v patch maps (identity rows when N % 8 != 0)
    // tuning (frg_set_tuning / frg_tune; 0 = the built-in choice): bubble rows
    // per block of the sweep, output rows per contraction block
    int rpb = 0, bm = 0;
    // K parts of the contraction: enough blocks (ks_target per flow) over the
    // tiles of the column set in use, at least ks_lo
    int ks_target = 3456, ks_lo = 1;
    bool kfixed = false;   // parts by fixed chunk ranges (FRG_KPARTS=fixed) or equal shares
    // rhs workspace
    double *d_pa64 = nullptr, *d_T = nullptr;
    float *d_pa32 = nullptr;
    double *d_B64 = nullptr;
    float *d_B32 = nullptr;
    double *d_perm = nullptr;
    uint16_t *d_ahl = nullptr;
    float *d_g32 = nullptr;
    double *d_C = nullptr;
    // flow workspace
    double *d_k[7] = {nullptr};
    double *d_yt = nullptr, *d_y5 = nullptr, *d_partial = nullptr, *d_state = nullptr;
    double *h_state = nullptr;
    // reduced flow state (symmetric-vertex mode with orbit columns): nst entries,
    // one per representative pp column and free index; y, the stage input and y5
    int64_t nst = 0;
    double *d_yr = nullptr, *d_ytr = nullptr, *d_y5r = nullptr;
    int nred = 256;
    size_t c_elems = 0;     // doubles the channel buffer d_C holds
    // bumped whenever a workspace buffer is freed and allocated again: captured
    // graphs and batch descriptors that hold its old address are stale then
    uint64_t ws_gen = 0;
    int ks_override = 0;    // FRG_KSPLIT
    size_t ws_bytes = 0;
    // the library's static scratch on this context's device (frg_rhs_noalloc)
    void *d_scratch = nullptr;
    // event timing (frg_profile_begin/end)
    EvProf pf;
    // one captured step of a single flow, replayed while its key matches
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        hipStream_t stream = nullptr;       // the context's own stream (capture needs one)
        hipEvent_t ev_in = nullptr, ev_out = nullptr;
        std::vector<double> key;
    } sg;
};

namespace {

thread_local std::string g_err;

frg_status fail(frg_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? FRG_ENOMEM : FRG_EDEVICE,         \
                        std::string(#expr) + ": " + hipGetErrorString(e_));           \
    } while (0)

template <class T>
frg_status dalloc(frg_ctx ctx, T **p, size_t n) {
    if (*p) return FRG_OK;
    void *q = nullptr;
    const size_t bytes = sizeof(T) * (n ? n : 1);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(FRG_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    *p = static_cast<T *>(q);
    ctx->ws_bytes += bytes;
    return FRG_OK;
}

template <class T>
frg_status upload(frg_ctx ctx, T **p, const T *src, size_t n) {
    frg_status st = dalloc(ctx, p, n);
    if (st) return st;
    HIPCHK(hipMemcpy(*p, src, sizeof(T) * n, hipMemcpyHostToDevice));
    return FRG_OK;
}

#define TRY(x)                        \
    do {                              \
        frg_status s_ = (x);          \
        if (s_ != FRG_OK) return s_;  \
    } while (0)

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

frg_status check_prec(frg_precision p) {
    if (p != FRG_PREC_FP64 && p != FRG_PREC_SPLIT_BF16)
        return fail(FRG_EINVAL, "unknown precision");
    return FRG_OK;
}

frg_status ensure_rhs_ws(frg_ctx ctx, frg_precision prec) {
    const auto &g = ctx->g;
    const size_t NN = static_cast<size_t>(g.N) * g.N;
    TRY(dalloc(ctx, &ctx->d_T, 4));
    if (prec == FRG_PREC_FP64) {
        TRY(dalloc(ctx, &ctx->d_pa64, 3 * static_cast<size_t>(g.np)));
        TRY(dalloc(ctx, &ctx->d_B64, NN * ctx->Trows));
        TRY(dalloc(ctx, &ctx->d_perm, 5 * static_cast<size_t>(ctx->n3)));
    } else {
        TRY(dalloc(ctx, &ctx->d_pa32, 3 * static_cast<size_t>(g.np)));
        TRY(dalloc(ctx, &ctx->d_B32, NN * ctx->Trows));
        TRY(dalloc(ctx, &ctx->d_ahl, 6 * static_cast<size_t>(ctx->n3)));
        TRY(dalloc(ctx, &ctx->d_g32, 3 * static_cast<size_t>(ctx->n3)));
    }
    return FRG_OK;
}

frg_status ensure_flow_ws(frg_ctx ctx) {
    // N more entries after V: the self-energy's place when it flows along
    const size_t nfull = static_cast<size_t>(ctx->n3) + static_cast<size_t>(ctx->g.N);
    for (int j = 0; j < 7; ++j) TRY(dalloc(ctx, &ctx->d_k[j], nfull));
    TRY(dalloc(ctx, &ctx->d_yt, nfull));
    TRY(dalloc(ctx, &ctx->d_y5, nfull));
    if (ctx->nst > 0) {
        // a reduced stage vector holds nst entries and, with a self-energy, N more
        TRY(dalloc(ctx, &ctx->d_yr, static_cast<size_t>(ctx->nst + ctx->g.N)));
        TRY(dalloc(ctx, &ctx->d_ytr, static_cast<size_t>(ctx->nst + ctx->g.N)));
        TRY(dalloc(ctx, &ctx->d_y5r, static_cast<size_t>(ctx->nst + ctx->g.N)));
    }
    TRY(dalloc(ctx, &ctx->d_partial, 2 * static_cast<size_t>(ctx->nred)));
    TRY(dalloc(ctx, &ctx->d_state, FRG_STATE_LEN));
    if (!ctx->h_state) HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&ctx->h_state),
                                            sizeof(double) * FRG_STATE_LEN, hipHostMallocDefault));
    return FRG_OK;
}

// Records events around the launches made while it is alive (profiling only).
struct KTimer {
    EvProf &pf;
    int cls;
    hipStream_t s;
    hipEvent_t a = nullptr;
    KTimer(EvProf &p, int k, hipStream_t st) : pf(p), cls(k), s(st) {
        if (pf.on && (a = pf.next())) hipEventRecord(a, s);
    }
    KTimer(frg_ctx c, int k, hipStream_t st) : KTimer(c->pf, k, st) {}
    ~KTimer() {
        if (!a) return;
        hipEvent_t b = pf.next();
        if (!b) return;
        hipEventRecord(b, s);
        pf.recs.push_back({cls, a, b});
    }
};

// summed milliseconds and launch counts per kernel class of the records
frg_status prof_collect(EvProf &pf, double *ms, int32_t *counts) {
    pf.on = false;
    double acc[FRG_KERNEL_CLASSES] = {0};
    int32_t cnt[FRG_KERNEL_CLASSES] = {0};
    for (const auto &r : pf.recs) {
        HIPCHK(hipEventSynchronize(r.b));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        acc[r.cls] += t;
        cnt[r.cls] += 1;
    }
    pf.recs.clear();
    pf.used = 0;
    for (int k = 0; k < FRG_KERNEL_CLASSES; ++k) {
        if (ms) ms[k] = acc[k];
        if (counts) counts[k] = cnt[k];
    }
    return FRG_OK;
}

frg::BubbleArgs bubble_args(frg_ctx ctx, bool fp32, void *bpp, void *bph, const double *pa64, const float *pa32,
                            const double *Tdev) {
    const auto &g = ctx->g;
    frg::BubbleArgs a;
    a.N = g.N;
    a.nf = g.nf;
    a.np = g.np;
    a.n_rad = g.n_rad;
    a.n_ang = g.n_ang;
    a.Tpp = g.Tpp;
    a.Trows = ctx->Trows;
    a.mt2 = -2.0 * g.t;
    a.mt4p = 4.0 * g.tp;
    a.mu = g.mu;
    a.bins = ctx->d_bins;
    a.trig_row = ctx->d_trig_row;
    a.trig_pt = ctx->d_trig_pt;
    a.pa64 = fp32 ? nullptr : pa64;
    a.pa32 = fp32 ? pa32 : nullptr;
    a.Tdev = Tdev;
    a.Bpp = bpp;
    a.Bph = bph;
    a.nrows = ctx->Trows;
    a.npp_out = g.Tpp;
    a.rowlist = nullptr;
    a.rowlist_ph = nullptr;
    a.rpb = ctx->rpb;
    a.count = ctx->d_count;
    a.sigma = nullptr;
    return a;
}

// output rows per block of the contraction (a tuning, else by N)
int block_rows(frg_ctx ctx) { return ctx->bm > 0 ? ctx->bm : frg::contract_block_rows(ctx->g.N); }

int c4v_patch_host(int o, int j, int N) {
    const int q = N / 4;
    const int v = (o & 1) ? ((o + 1) / 2) * q - 1 - j : j + (o / 2) * q;
    return ((v % N) + N) % N;
}

// C4v orbits of the transfer rows (N % 8 == 0 only: the grid is then
// bitwise symmetric).  Builds the representative list, the per-column
// (compact rep, element) tables and checks B_{g t}(g a, g b) = B_t(a, b)
// on the device's second-line table; the reduction is enabled only if the
// check finds no exception.
//
// Only pp rows have representatives of their own.  With patch j + N/2
// opposite to j (k_{j+N/2} = -k_j bitwise), every ph transfer
// Q = k_x - k_y = -(k_y + k_{x+N/2}) is the opposite of a pp transfer, and the
// ph row of -q has the second-line energy of the pp row q at every fine point.
// So each representative pp row q is evaluated together with the ph row of -q
// (its pair), and a ph row Q = g (-q) is the g-image of the pair's ph row.
frg_status build_orbits(frg_ctx ctx) {
    const auto &g = ctx->g;
    const int N = g.N;
    if (N % 8 != 0) return FRG_OK;
    std::vector<int> pi(g.Tpp), pj(g.Tpp), px(g.Tph), py(g.Tph);
    for (int i = 0; i < N; ++i)
        for (int j = i; j < N; ++j) { const int t = g.row_pp[i * N + j]; pi[t] = i; pj[t] = j; }
    for (int x = 0; x < N; ++x)
        for (int y = 0; y < N; ++y) { const int t = g.row_ph[x * N + y]; px[t] = x; py[t] = y; }
    auto img_pp = [&](int o, int t) {
        return g.row_pp[c4v_patch_host(o, pi[t], N) * N + c4v_patch_host(o, pj[t], N)];
    };
    auto img_ph = [&](int o, int t) {
        if (t == 0) return 0;
        return g.row_ph[c4v_patch_host(o, px[t], N) * N + c4v_patch_host(o, py[t], N)];
    };
    std::vector<int> rep_pp(g.Tpp), el_pp(g.Tpp), rep_ph(g.Tph), el_ph(g.Tph);
    for (int t = 0; t < g.Tpp; ++t) {
        int r = t;
        for (int o = 1; o < 8; ++o) r = std::min(r, img_pp(o, t));
        rep_pp[t] = r;
        el_pp[t] = -1;
        for (int o = 0; o < 8 && el_pp[t] < 0; ++o)
            if (img_pp(o, r) == t) el_pp[t] = o;
    }
    std::vector<int32_t> rowlist, rowlist_ph, cidx_pp(g.Tpp, -1), orbit(ctx->Trows);
    const int H = N / 2;
    auto pair_ph = [&](int t) { return g.row_ph[((pi[t] + H) % N) * N + pj[t]]; };   // ph row of -q_t
    for (int t = 0; t < g.Tpp; ++t)
        if (rep_pp[t] == t) {
            cidx_pp[t] = static_cast<int32_t>(rowlist.size());
            rowlist.push_back(t);
            rowlist_ph.push_back(g.Tpp + pair_ph(t));
        }
    const int npp = static_cast<int>(rowlist.size());
    // ph row t = (x, y): -Q_t = k_y + k_{x+N/2} is the pp transfer t' = o . rep, so
    // Q_t = o (-q_rep): the o-image of the pair row of rep
    for (int t = 0; t < g.Tph; ++t) {
        const int x = px[t], y = py[t];
        const int u = (x + H) % N, lo = std::min(y, u), hi = std::max(y, u);
        const int tp = g.row_pp[lo * N + hi];
        rep_ph[t] = rep_pp[tp];
        el_ph[t] = el_pp[tp];
    }
    (void)img_ph;
    for (int t = 0; t < g.Tpp; ++t) orbit[t] = (rep_pp[t] << 3) | el_pp[t];
    for (int t = 0; t < g.Tph; ++t) orbit[g.Tpp + t] = ((g.Tpp + pair_ph(rep_ph[t])) << 3) | el_ph[t];
    std::vector<int32_t> cs_pp(static_cast<size_t>(N) * N), cs_ph(static_cast<size_t>(N) * N);
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            const int tp = g.row_pp[y * N + x];
            cs_pp[y * N + x] = (cidx_pp[rep_pp[tp]] << 3) | el_pp[tp];
            const int th = g.row_ph[x * N + y];
            cs_ph[y * N + x] = (cidx_pp[rep_ph[th]] << 3) | el_ph[th];
        }
    int32_t *d_orbit = nullptr;
    int *d_bad = nullptr;
    TRY(upload(ctx, &d_orbit, orbit.data(), orbit.size()));
    TRY(dalloc(ctx, &d_bad, 1));
    HIPCHK(hipMemset(d_bad, 0, sizeof(int)));
    // a reflected polar patch lists its sub-rays in reverse; the energy-angle
    // lists keep their order
    frg::launch_sym_check(ctx->d_bins, d_orbit, N, g.n_rad, g.n_ang, ctx->Trows, !g.egrid, d_bad, nullptr);
    int bad = -1;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost);
    hipFree(d_orbit);
    hipFree(d_bad);
    ctx->ws_bytes -= sizeof(int32_t) * orbit.size() + sizeof(int);
    if (e != hipSuccess) return fail(FRG_EDEVICE, std::string("symmetry check: ") + hipGetErrorString(e));
    if (bad != 0) return FRG_OK;   // an exception to exact covariance: keep every row
    TRY(upload(ctx, &ctx->d_rowlist, rowlist.data(), rowlist.size()));
    TRY(upload(ctx, &ctx->d_rowlist_ph, rowlist_ph.data(), rowlist_ph.size()));
    {   // the paired sweep takes the ph row's patches from the pp row's (+ N/2)
        int *d_pbad = nullptr;
        TRY(dalloc(ctx, &d_pbad, 1));
        HIPCHK(hipMemset(d_pbad, 0, sizeof(int)));
        frg::launch_pair_check(ctx->d_bins, ctx->d_rowlist, ctx->d_rowlist_ph, static_cast<int>(rowlist.size()),
                               g.np, N, d_pbad, nullptr);
        int pbad = -1;
        hipError_t pe = hipGetLastError();
        if (pe == hipSuccess) pe = hipMemcpy(&pbad, d_pbad, sizeof(int), hipMemcpyDeviceToHost);
        hipFree(d_pbad);
        ctx->ws_bytes -= sizeof(int);
        if (pe != hipSuccess) return fail(FRG_EDEVICE, std::string("pair check: ") + hipGetErrorString(pe));
        if (pbad != 0) return FRG_OK;   // keep every row, unpaired
    }
    ctx->h_rowlist = rowlist;
    ctx->h_rowlist_ph = rowlist_ph;
    TRY(upload(ctx, &ctx->d_colsym_pp, cs_pp.data(), cs_pp.size()));
    TRY(upload(ctx, &ctx->d_colsym_ph, cs_ph.data(), cs_ph.size()));
    ctx->n_rep_pp = npp;
    ctx->n_rep_ph = npp;
    ctx->sym_avail = true;
    ctx->sym_on = std::getenv("FRG_NO_SYM") == nullptr;
    return FRG_OK;
}

// K parts of the fused contraction over ncol columns: enough blocks for several
// rounds over the 256 compute units (measured best at N = 96: 8 parts for all
// columns, 16 for one column per C4v orbit; in a batch of 16, 2 for all
// columns and 8 for the orbit columns); FRG_KSPLIT overrides
int ksplit_for(frg_ctx ctx, int ncol, int hi) {
    if (ctx->ks_override > 0) return ctx->ks_override;
    const int N = ctx->g.N;
    const int bm = block_rows(ctx);
    const int64_t tiles = 3LL * ((N + bm - 1) / bm) * ((ncol + 63) / 64);
    const int64_t ks = (ctx->ks_target + tiles - 1) / tiles;
    return static_cast<int>(std::min<int64_t>(hi, std::max<int64_t>(ctx->ks_lo, ks)));
}

// entry of a chunk list: chunk id j (k = 8j .. 8j+7) and the patch pair
// (a, b) of k = 8j = a*N + b, packed as j | a << 13 | b << 21 (N <= 256)
int32_t list_entry(int j, int N) {
    const int k = j * frg::kContractChunk;
    return static_cast<int32_t>(j | ((k / N) << 13) | ((k % N) << 21));
}

// position along a Hilbert curve over the Brillouin zone [-pi, pi)^2 (2^16 x 2^16 cells)
uint64_t hilbert_key(double qx, double qy) {
    const uint32_t n = 1u << 16;
    auto quant = [&](double v) {
        const double u = (v + M_PI) / (2.0 * M_PI) * n;
        return u <= 0.0 ? 0u : (u >= n - 1.0 ? n - 1u : static_cast<uint32_t>(u));
    };
    uint32_t x = quant(qx), y = quant(qy);
    uint64_t d = 0;
    for (uint32_t sq = n / 2; sq > 0; sq /= 2) {
        const uint32_t rx = (x & sq) ? 1u : 0u, ry = (y & sq) ? 1u : 0u;
        d += static_cast<uint64_t>(sq) * sq * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) { x = n - 1 - x; y = n - 1 - y; }
            std::swap(x, y);
        }
    }
    return d;
}

// Column tiles of the contraction.  Columns (pp: (j1, j2), ph: (y, x)) are
// ordered along the Hilbert curve of their transfer momentum; for every tile
// of 64 consecutive columns the second-line table gives the k chunks where
// any of its bubble rows can be nonzero (T independent).  Tile t's list is cut
// into the contraction's KS parts: part ks is klist[koff[t*(KS+1)+ks] ..
// koff[t*(KS+1)+ks+1]), either an equal share of the entries (cut at multiples
// of 4 entries, one split-path step) or, with FRG_KPARTS=fixed, the entries
// with chunk ids in [ks*nch/KS, (ks+1)*nch/KS) (the same k range in every
// tile, so the blocks of one part share one slice of the A operands).
void cut_parts(const std::vector<int32_t> &chunk_of_entry, int begin, int end, int KS, int nch, bool fixed,
               int32_t *off) {
    const int n = end - begin;
    for (int ks = 0; ks <= KS; ++ks) {
        if (!fixed) {
            const int64_t e = (static_cast<int64_t>((n + 3) / 4) * ks / KS) * 4;
            off[ks] = begin + static_cast<int32_t>(std::min<int64_t>(e, n));
        } else {
            const int lim = static_cast<int>(static_cast<int64_t>(nch) * ks / KS);
            int i = begin;
            while (i < end && chunk_of_entry[i] < lim) ++i;
            off[ks] = i;
        }
    }
}

// (Re)cut every tile's chunk list of ts into KS parts (the offsets koff); the
// lists themselves stay.  A new offset table replaces the old one.
frg_status cut_tileset(frg_ctx ctx, TileSet &ts, int KS) {
    const int tiles = static_cast<int>(ts.h_begin.size()) - 1;
    const int nch = ctx->g.N * ctx->g.N / frg::kContractChunk;
    std::vector<int32_t> koff(static_cast<size_t>(tiles) * (KS + 1));
    for (int t = 0; t < tiles; ++t)
        cut_parts(ts.h_chunk, ts.h_begin[t], ts.h_begin[t + 1], KS, nch, ctx->kfixed,
                  &koff[static_cast<size_t>(t) * (KS + 1)]);
    if (ts.d_koff) {
        hipFree(ts.d_koff);
        ctx->ws_bytes -= sizeof(int32_t) * static_cast<size_t>(tiles) * (ts.kparts + 1);
        ts.d_koff = nullptr;
    }
    TRY(upload(ctx, &ts.d_koff, koff.data(), koff.size()));
    ts.kparts = KS;
    return FRG_OK;
}

// Tile set of class cls over the columns `cols` (natural indices; rep[c] and
// h[c] give, for every natural column c, the computed column whose values it
// takes and the C4v element carrying c's free index to it).  Hilbert order of
// the columns' transfer momenta unless natural; active chunks from the
// second-line table unless every chunk is kept.
frg_status build_tileset(frg_ctx ctx, int cls, const std::vector<int32_t> &cols, const std::vector<int32_t> &rep,
                         const std::vector<int8_t> &h, bool natural, bool all_chunks, int KS, TileSet &ts) {
    const auto &g = ctx->g;
    const int N = g.N, NC = N * N;
    const int ncol = static_cast<int>(cols.size());
    const int tiles = (ncol + frg::kContractCols - 1) / frg::kContractCols;
    const int nch = NC / frg::kContractChunk;
    std::vector<int32_t> colfull(NC), perm(cols);
    std::vector<uint64_t> key(NC);
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            const int c = y * N + x;
            const int row = cls == 0 ? g.row_pp[y * N + x] : g.row_ph[x * N + y];
            const double *q = cls == 0 ? &g.qpp[2 * row] : &g.qph[2 * row];
            colfull[c] = cls == 0 ? row : g.Tpp + row;
            key[c] = hilbert_key(q[0], q[1]);
        }
    if (!natural) std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<int32_t> pos(NC, -1), cmap(NC);
    for (int i = 0; i < ncol; ++i) pos[perm[i]] = i;
    for (int c = 0; c < NC; ++c) cmap[c] = (pos[rep[c]] << 3) | h[c];
    TRY(upload(ctx, &ts.d_cperm, perm.data(), perm.size()));
    TRY(upload(ctx, &ts.d_cmap, cmap.data(), cmap.size()));
    std::vector<uint8_t> flags(static_cast<size_t>(tiles) * nch, 1);
    if (!all_chunks) {
        int32_t *d_colfull = nullptr;
        uint8_t *d_flags = nullptr;
        hipError_t e = hipMalloc(&d_colfull, sizeof(int32_t) * NC);
        if (e == hipSuccess) e = hipMalloc(&d_flags, flags.size());
        if (e == hipSuccess) e = hipMemcpy(d_colfull, colfull.data(), sizeof(int32_t) * NC, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(d_flags, 0, flags.size());
        if (e == hipSuccess) {
            frg::launch_tile_pattern(ctx->d_bins, d_colfull, ts.d_cperm, ncol, N, g.nf, g.np, d_flags, nullptr);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpy(flags.data(), d_flags, flags.size(), hipMemcpyDeviceToHost);
        if (d_colfull) hipFree(d_colfull);
        if (d_flags) hipFree(d_flags);
        if (e != hipSuccess) return fail(FRG_EDEVICE, std::string("column tiles: ") + hipGetErrorString(e));
    }
    std::vector<int32_t> klist, chunk, begin(tiles + 1);
    for (int t = 0; t < tiles; ++t) {
        begin[t] = static_cast<int32_t>(klist.size());
        for (int j = 0; j < nch; ++j)
            if (flags[static_cast<size_t>(t) * nch + j]) {
                klist.push_back(list_entry(j, N));
                chunk.push_back(j);
            }
    }
    begin[tiles] = static_cast<int32_t>(klist.size());
    ts.ncol = ncol;
    ts.chunks = static_cast<int64_t>(klist.size());
    ts.h_chunk = std::move(chunk);
    ts.h_begin = std::move(begin);
    TRY(upload(ctx, &ts.d_klist, klist.data(), klist.size()));
    return cut_tileset(ctx, ts, KS);
}

// every column computed, each its own representative
void all_columns(int N, std::vector<int32_t> &cols, std::vector<int32_t> &rep, std::vector<int8_t> &h) {
    cols.resize(static_cast<size_t>(N) * N);
    std::iota(cols.begin(), cols.end(), 0);
    rep = cols;
    h.assign(cols.size(), 0);
}

// Tile sets made at creation: ts_full (and, where the grid is exactly C4v
// covariant, ts_vsym: one column per orbit of the pair action
// g (y, x) = (g y, g x), and h[c] = g^-1 for c = g rep, because
// F(g c, g m) = F(c, m) for a C4v-invariant vertex).  Also the [8][N] patch
// maps.
//
// Each channel class picks its own representative per orbit: the member whose
// transfer momentum lies in the wedge 0 <= q_y <= q_x (smallest natural index
// among ties, and where no member's does).  The representatives' transfers
// then fill one eighth of the zone densely, so 64 consecutive columns in
// Hilbert order have nearly the same bubble-row pattern: at N = 96 a tile
// visits 45% of the dense k chunks instead of 59% with the smallest natural
// index as representative (which scatters the transfers over the whole zone).
frg_status build_ktiles(frg_ctx ctx) {
    const int N = ctx->g.N, NC = N * N;
    const char *kp = std::getenv("FRG_KPARTS");
    ctx->kfixed = kp && std::strcmp(kp, "fixed") == 0;
    std::vector<int16_t> perm8(8 * static_cast<size_t>(N));
    for (int o = 0; o < 8; ++o)
        for (int j = 0; j < N; ++j)
            perm8[o * N + j] = static_cast<int16_t>(N % 8 == 0 ? c4v_patch_host(o, j, N) : j);
    TRY(upload(ctx, &ctx->d_perm8, perm8.data(), perm8.size()));
    std::vector<int32_t> cols, rep;
    std::vector<int8_t> h;
    all_columns(N, cols, rep, h);
    const int ks_full = ksplit_for(ctx, NC, 8);
    for (int cls = 0; cls < 2; ++cls)
        TRY(build_tileset(ctx, cls, cols, rep, h, false, false, ks_full, ctx->ts_full[cls]));
    if (!ctx->sym_avail) return FRG_OK;
    const auto &g = ctx->g;
    for (int cls = 0; cls < 2; ++cls) {
        // 0: transfer in the wedge, 1: not; then the natural index
        auto score = [&](int c) -> int64_t {
            const int y = c / N, x = c % N;
            const int row = cls == 0 ? g.row_pp[y * N + x] : g.row_ph[x * N + y];
            const double *q = cls == 0 ? &g.qpp[2 * row] : &g.qph[2 * row];
            const bool wedge = q[1] >= -1e-9 && q[1] <= q[0] + 1e-9;
            return (wedge ? 0 : static_cast<int64_t>(NC)) + c;
        };
        cols.clear();
        for (int c = 0; c < NC; ++c) {
            const int y = c / N, x = c % N;
            int r = c, ro = 0;
            int64_t best = score(c);
            for (int o = 1; o < 8; ++o) {
                const int gc = c4v_patch_host(o, y, N) * N + c4v_patch_host(o, x, N);
                const int64_t sc = score(gc);
                if (sc < best) { best = sc; r = gc; ro = o; }
            }
            // c = g rep with g the inverse of the element ro that carries c to rep;
            // the value at c, m is the value at rep, ro(m)
            rep[c] = r;
            h[c] = static_cast<int8_t>(ro);
            if (r == c) cols.push_back(c);
        }
        // up to 24 parts at N >= 96 (a single split flow at N = 96: 5980 -> 6177 rhs/s
        // against 16 parts; FP64 1% slower), 16 below
        const int ks_v = ksplit_for(ctx, static_cast<int>(cols.size()), N >= 96 ? 24 : 16);
        TRY(build_tileset(ctx, cls, cols, rep, h, false, false, ks_v, ctx->ts_vsym[cls]));
    }
    ctx->nst = static_cast<int64_t>(ctx->ts_vsym[0].ncol) * N;
    return FRG_OK;
}

// natural column order with every k chunk (the dense contraction)
frg_status ensure_dense_tiles(frg_ctx ctx) {
    if (ctx->ts_dense[0].d_klist) return FRG_OK;
    std::vector<int32_t> cols, rep;
    std::vector<int8_t> h;
    all_columns(ctx->g.N, cols, rep, h);
    for (int cls = 0; cls < 2; ++cls)
        TRY(build_tileset(ctx, cls, cols, rep, h, true, true, ctx->ts_full[0].kparts, ctx->ts_dense[cls]));
    return FRG_OK;
}

// Operand pointers of the fused contraction in the layout the layout kernels
// write: FP64 perm = [pp A, phc A, phd A (chunk-major), phc gather, phd
// gather]; split ahl = the three A operands x (hi, lo), g32 = [V, phc gather,
// phd gather].  Both contractions take the direct-ph sum as
// V(j2,a,b) V(j1,b,j3) + V(a,j2,b) (V(j1,b,a) - 2 V(j1,b,j3)), so the first phd
// operand is the phc operand V(m,a,b).
void set_operands(frg::FusedContractArgs &a, bool split, const double *V, const double *P, const uint16_t *H,
                  const float *G, int64_t n3) {
    using frg::TERM_PP;
    using frg::TERM_PHC;
    using frg::TERM_PHD;
    if (!split) {
        a.A64[TERM_PP][0] = P;           a.G64[TERM_PP][0] = V;
        a.A64[TERM_PHC][0] = P + n3;     a.G64[TERM_PHC][0] = P + 3 * n3;
        a.A64[TERM_PHD][0] = P + n3;     a.G64[TERM_PHD][0] = P + 4 * n3;
        a.A64[TERM_PHD][1] = P + 2 * n3; a.G64[TERM_PHD][1] = P + 4 * n3;
    } else {
        a.Ahl[TERM_PP][0] = H;           a.G32[TERM_PP][0] = G;
        a.Ahl[TERM_PHC][0] = H + 2 * n3; a.G32[TERM_PHC][0] = G + n3;
        a.Ahl[TERM_PHD][0] = H + 2 * n3; a.G32[TERM_PHD][0] = G + 2 * n3;
        a.Ahl[TERM_PHD][1] = H + 4 * n3; a.G32[TERM_PHD][1] = G + 2 * n3;
    }
}

// bubble-row operands of the contraction: pointers, sizes and whether the
// split path may take its buffer-load fast path
void set_bubbles(frg_ctx ctx, bool split, bool sym, void *bpp, void *bph, frg::FusedContractArgs &a) {
    const auto &g = ctx->g;
    const int64_t NN = static_cast<int64_t>(g.N) * g.N;
    const int64_t elem = split ? 4 : 8;
    const int64_t bpp_bytes = (sym ? ctx->n_rep_pp : g.Tpp) * NN * elem;
    const int64_t bph_bytes = (sym ? ctx->n_rep_ph : g.Tph) * NN * elem;
    a.B[frg::TERM_PP] = bpp;
    a.B[frg::TERM_PHC] = a.B[frg::TERM_PHD] = bph;
    a.Bbytes[frg::TERM_PP] = bpp_bytes;
    a.Bbytes[frg::TERM_PHC] = a.Bbytes[frg::TERM_PHD] = bph_bytes;
    const int64_t lim = int64_t(1) << 31;
    a.fast = split && g.N % 32 == 0 && bpp_bytes < lim && bph_bytes < lim && 4 * ctx->n3 < lim &&
             std::getenv("FRG_NO_FAST") == nullptr;
}

// the tile set in use for class cls
const TileSet &tiles_of(frg_ctx ctx, int cls) {
    if (!ctx->kskip_on) return ctx->ts_dense[cls];
    return ctx->vsym_on ? ctx->ts_vsym[cls] : ctx->ts_full[cls];
}
const int32_t *col_pos(frg_ctx ctx, int cls) { return tiles_of(ctx, cls).d_cmap; }
// Flows keep their stage vectors reduced while the orbit columns are computed:
// the rhs is then known at the representative columns only, and every other
// entry is a copy (a C4v-invariant vertex stays invariant).
// A C4v-invariant self-energy rides along after the nst reduced entries.
bool red_state(frg_ctx ctx) {
    return ctx->vsym_on && ctx->kskip_on && ctx->nst > 0 && (!ctx->se_on || ctx->se_sym);
}
// K parts of the column set in use
int ksplit(frg_ctx ctx) { return tiles_of(ctx, 0).kparts; }

// channel elements one rhs computes (computed columns x N), for the K-part sum
int64_t computed_elems(frg_ctx ctx) {
    return static_cast<int64_t>(std::max(tiles_of(ctx, 0).ncol, tiles_of(ctx, 1).ncol)) * ctx->g.N;
}

void set_tiles(frg_ctx ctx, frg::FusedContractArgs &a) {
    for (int t = 0; t < 3; ++t) {
        const TileSet &ts = tiles_of(ctx, t == frg::TERM_PP ? 0 : 1);
        a.cperm[t] = ts.d_cperm;
        a.koff[t] = ts.d_koff;
        a.klist[t] = ts.d_klist;
        a.ncol[t] = ts.ncol;
    }
}

// Per-call workspace of one rhs: the point factors and temperature, the bubble
// rows, the operand layout and the channel partials ([3][KS][cs], then their
// sums [3][cs], cs = elements computed per channel).  The context's own
// buffers (ctx_ws, sized by ensure_rhs_ws / ensure_c), or pieces of the static
// scratch (frg_rhs_noalloc).
struct RhsWs {
    double *pa64 = nullptr, *T = nullptr;
    float *pa32 = nullptr;
    double *B64 = nullptr;
    float *B32 = nullptr;
    double *perm = nullptr;
    uint16_t *ahl = nullptr;
    float *g32 = nullptr;
    double *C = nullptr;
    bool own = true;   // the context's buffers
};

RhsWs ctx_ws(frg_ctx ctx) {
    RhsWs w;
    w.pa64 = ctx->d_pa64; w.T = ctx->d_T; w.pa32 = ctx->d_pa32;
    w.B64 = ctx->d_B64; w.B32 = ctx->d_B32;
    w.perm = ctx->d_perm; w.ahl = ctx->d_ahl; w.g32 = ctx->d_g32;
    w.C = ctx->d_C;
    return w;
}

// prep + bubbles into the context's bubble tensor (or caller buffers)
frg_status run_bubbles(frg_ctx ctx, bool split, double T_host, const double *state, double c,
                       void *bpp, void *bph, hipStream_t s, bool reps_only = false, bool full = false,
                       const RhsWs *wsp = nullptr, const double *sigma = nullptr) {
    const RhsWs w = wsp ? *wsp : ctx_ws(ctx);
    {
        KTimer kt(ctx, FRG_K_PREP, s);
        frg::launch_point_prep(ctx->d_xi, ctx->d_w, ctx->g.np, T_host, state, c,
                               split ? nullptr : w.pa64, split ? w.pa32 : nullptr, w.T, s, sigma, ctx->g.nf);
    }
    {
        KTimer kt(ctx, FRG_K_BUBBLES, s);
        frg::BubbleArgs ba = bubble_args(ctx, split, bpp, bph, w.pa64, w.pa32, w.T);
        ba.sigma = sigma;
        if (reps_only) {
            ba.rowlist = ctx->d_rowlist;
            ba.rowlist_ph = ctx->d_rowlist_ph;
            ba.nrows = ctx->n_rep_pp;
            ba.npp_out = ctx->n_rep_pp;
        }
        frg::launch_bubbles(ba, split, full, s);
    }
    HIPCHK(hipGetLastError());
    return FRG_OK;
}

// channel stride: the elements one rhs computes per channel (computed columns
// x N; N^3 when every column is computed)
int64_t chan_stride(frg_ctx ctx) { return computed_elems(ctx); }
// doubles of the channel buffer for the column set in use: K-part partials
// [3][KS][cs] (float in the split path, in the first half of each part) and
// their FP64 sums [3][cs]
size_t c_elems_needed(frg_ctx ctx) {
    return 3 * static_cast<size_t>(ksplit(ctx) + 1) * static_cast<size_t>(chan_stride(ctx));
}

frg_status ensure_c(frg_ctx ctx) {
    const size_t need = c_elems_needed(ctx);
    if (ctx->c_elems >= need) return FRG_OK;
    if (ctx->d_C) {
        // a captured step writes the old buffer: drop it before the buffer goes
        if (ctx->sg.exec) {
            hipGraphExecDestroy(ctx->sg.exec);
            ctx->sg.exec = nullptr;
        }
        ctx->ws_gen++;
        hipFree(ctx->d_C);
        ctx->ws_bytes -= sizeof(double) * ctx->c_elems;
        ctx->d_C = nullptr;
    }
    TRY(dalloc(ctx, &ctx->d_C, need));
    ctx->c_elems = need;
    return FRG_OK;
}

// where the rhs takes its bubbles from
enum RhsMode {
    RHS_DT = 0,       // dL/dT at T (temperature flow)
    RHS_FULL = 1,     // L at T (interaction flow, one evaluation)
    RHS_STORED = 2    // the L_T already in the context's buffer (interaction flow steps)
};

// full rhs: F = scale * (-Cpp + Cc + Cd); scale = T when scale_by_T.  red_out:
// F at the representative entries only (the reduced flow state).  Vred: the
// split path reads its input from this reduced state instead of V
frg_status run_rhs(frg_ctx ctx, bool split, double T_host, const double *state, double c,
                   const double *V, double *F, int scale_by_T, hipStream_t s, RhsMode mode = RHS_DT,
                   bool red_out = false, const double *Vred = nullptr, const RhsWs *wsp = nullptr) {
    const auto &g = ctx->g;
    const int N = g.N;
    const size_t NN = static_cast<size_t>(N) * N;
    const int64_t n3 = ctx->n3;
    // with a general self-energy the rows are not C4v images of each other:
    // every row; with a C4v-invariant one they are, and the pairs hold
    const bool se = ctx->se_on && mode == RHS_DT;
    const bool sym = ctx->sym_on && (!se || ctx->se_sym);
    // the self-energy: after V, or, when a split stage of a reduced flow hands
    // over the reduced vector itself (V == Vred), after its nst entries
    const double *Sv = se ? (Vred ? Vred + ctx->nst : V + ctx->n3) : nullptr;
    const int KS = ksplit(ctx);
    const int64_t cs = chan_stride(ctx);
    if (!wsp) TRY(ensure_c(ctx));
    const RhsWs w = wsp ? *wsp : ctx_ws(ctx);
    const size_t npp_rows = sym ? static_cast<size_t>(ctx->n_rep_pp) : static_cast<size_t>(g.Tpp);
    void *bpp = split ? static_cast<void *>(w.B32) : static_cast<void *>(w.B64);
    void *bph = split ? static_cast<void *>(w.B32 + NN * npp_rows) : static_cast<void *>(w.B64 + NN * npp_rows);
    if (mode != RHS_STORED) {
        if (w.own) ctx->iflow_prec = -1;   // the context's bubble buffer is overwritten
        TRY(run_bubbles(ctx, split, T_host, state, c, bpp, bph, s, sym, mode == RHS_FULL, &w, Sv));
    }
    double *Cpp = w.C, *Cc = w.C + KS * cs, *Cd = w.C + 2 * KS * cs;
    frg::FusedContractArgs a;
    std::memset(&a, 0, sizeof(a));
    a.N = N;
    a.KS = KS;
    a.n3 = n3;
    a.pstride = cs;
    a.bm = block_rows(ctx);
    set_bubbles(ctx, split, sym, bpp, bph, a);
    a.colrow[frg::TERM_PP] = sym ? ctx->d_colsym_pp : ctx->d_colrow_pp;
    a.colrow[frg::TERM_PHC] = a.colrow[frg::TERM_PHD] = sym ? ctx->d_colsym_ph : ctx->d_colrow_ph;
    set_tiles(ctx, a);
    a.C[frg::TERM_PP] = Cpp;
    a.C[frg::TERM_PHC] = Cc;
    a.C[frg::TERM_PHD] = Cd;
    {
        KTimer kt(ctx, FRG_K_LAYOUT, s);
        if (!split) frg::launch_layout_f64(V, N, w.perm, s);
        else if (Vred) frg::launch_layout_split_red(Vred, N, col_pos(ctx, 0), tiles_of(ctx, 1).d_cperm,
                                                    tiles_of(ctx, 1).ncol, w.ahl, w.g32, s);
        else frg::launch_layout_split(V, N, w.ahl, w.g32, s);
    }
    set_operands(a, split, V, w.perm, w.ahl, w.g32, n3);
    {
        KTimer kt(ctx, FRG_K_CONTRACT, s);
        frg::launch_contract_fused(a, split, s);
    }
    {
        KTimer kt(ctx, FRG_K_COMBINE, s);
        double *Cs = w.C + 3 * KS * cs;
        frg::launch_sum_parts(w.C, split, KS, cs, cs, Cs, s);
        if (red_out)
            frg::launch_combine_red(Cs, cs, N, ctx->nst, tiles_of(ctx, 0).d_cperm, col_pos(ctx, 1), ctx->d_perm8,
                                    w.T, scale_by_T, F, s);
        else
            frg::launch_combine(Cs, Cs + cs, Cs + 2 * cs, false, N, 1, col_pos(ctx, 0), col_pos(ctx, 1),
                                ctx->d_perm8, w.T, scale_by_T, F, s);
        if (se)   // the self-energy's derivative after F (always FP64)
            frg::launch_dsigma(ctx->d_xi, ctx->d_w, N, g.nf, Vred ? Vred : V, Sv, w.T, scale_by_T, ctx->d_sigD,
                               F + (red_out ? ctx->nst : n3), s, Vred ? col_pos(ctx, 0) : nullptr);
    }
    HIPCHK(hipGetLastError());
    return FRG_OK;
}

// max over g, j of |V(g j) - V(j)| / max |V| (synchronises the stream)
constexpr double kVsymTol = 1e-12;
frg_status vsym_deviation(frg_ctx ctx, const double *V, hipStream_t s, double *rel) {
    const int nb = frg::vsym_check_blocks(ctx->g.N);
    double *d_part = nullptr;
    HIPCHK(hipMalloc(&d_part, sizeof(double) * 2 * nb));
    std::vector<double> h(2 * static_cast<size_t>(nb));
    frg::launch_vsym_check(V, ctx->g.N, ctx->d_perm8, d_part, s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d_part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(d_part);
    if (e != hipSuccess) return fail(FRG_EDEVICE, std::string("symmetry check: ") + hipGetErrorString(e));
    double dev = 0.0, vmax = 0.0;
    for (int i = 0; i < nb; ++i) {
        dev = std::max(dev, h[i]);
        vmax = std::max(vmax, h[nb + i]);
    }
    *rel = vmax > 0.0 ? dev / vmax : dev;
    return FRG_OK;
}

// S (N doubles on the device) C4v invariant to 1e-12 relative: S(g j) = S(j)
// for every C4v element g (synchronises the stream)
frg_status check_se_sym(frg_ctx ctx, const double *d_S, hipStream_t s) {
    const int N = ctx->g.N;
    std::vector<double> S(static_cast<size_t>(N));
    HIPCHK(hipMemcpyAsync(S.data(), d_S, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double dev = 0.0, smax = 0.0;
    for (int j = 0; j < N; ++j) {
        smax = std::max(smax, std::fabs(S[j]));
        for (int o = 1; o < 8; ++o) dev = std::max(dev, std::fabs(S[c4v_patch_host(o, j, N)] - S[j]));
    }
    if (!(dev <= kVsymTol * smax))
        return fail(FRG_EINVAL, "a C4v-invariant self-energy was announced, but S deviates by " +
                                    std::to_string(dev) + " (max |S| " + std::to_string(smax) + ")");
    return FRG_OK;
}

frg_status check_ctx(frg_ctx ctx) {
    if (!ctx) return fail(FRG_EINVAL, "null context");
    return FRG_OK;
}

frg_status check_opts(frg_ctx ctx, const frg_flow_opts *o) {
    (void)ctx;
    if (!o) return fail(FRG_EINVAL, "null flow options");
    TRY(check_prec(o->prec));
    if (o->stepper != FRG_RK4 && o->stepper != FRG_DP54) return fail(FRG_EINVAL, "unknown stepper");
    if (!(o->T0 > 0.0) || !std::isfinite(o->T0) || !(o->T_min > 0.0) || !std::isfinite(o->T_min) ||
        o->T0 == o->T_min)
        return fail(FRG_EINVAL, "need finite T0 > 0, T_min > 0, T0 != T_min");
    if (!(o->vmax > 0.0)) return fail(FRG_EINVAL, "vmax must be > 0");
    if (o->stepper == FRG_RK4 && o->fixed_steps <= 0)
        return fail(FRG_EINVAL, "RK4 needs fixed_steps > 0");
    if (o->stepper == FRG_DP54 && (!(o->rtol > 0.0) || !(o->atol >= 0.0) || !std::isfinite(o->h0)))
        return fail(FRG_EINVAL, "DP54 needs rtol > 0, atol >= 0, finite h0");
    if (o->max_steps < 0) return fail(FRG_EINVAL, "max_steps must be >= 0");
    return FRG_OK;
}

// Dormand & Prince (1980) 5(4) tableau
const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
const double DP_A[7][6] = {{0},
                           {1.0 / 5},
                           {3.0 / 40, 9.0 / 40},
                           {44.0 / 45, -56.0 / 15, 32.0 / 9},
                           {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
                           {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656},
                           {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
const double DP_E[7] = {35.0 / 384 - 5179.0 / 57600, 0.0, 500.0 / 1113 - 7571.0 / 16695,
                        125.0 / 192 - 393.0 / 640, -2187.0 / 6784 + 92097.0 / 339200,
                        11.0 / 84 - 187.0 / 2100, -1.0 / 40};

int red_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return static_cast<int>(b < 256 ? (b < 1 ? 1 : b) : 256);
}

}  // namespace

static frg_status check_params(const frg_params *p);
extern "C" frg_status frg_batch_destroy(frg_batch b);

extern "C" {

const char *frg_status_str(frg_status st) {
    switch (st) {
    case FRG_OK: return "ok";
    case FRG_EINVAL: return "invalid argument";
    case FRG_ENOMEM: return "out of memory";
    case FRG_EDEVICE: return "device error";
    case FRG_ENOTSUP: return "not supported";
    case FRG_ENONFINITE: return "non-finite state";
    }
    return "unknown status";
}

const char *frg_last_error(void) { return g_err.c_str(); }

static frg_status create_impl(const frg_params *p, int n_batch, frg_ctx *out, const frg_egrid *eg = nullptr);

frg_status frg_create(const frg_params *p, frg_ctx *out) { return create_impl(p, 1, out); }

// largest padded n_f of the energy-angle grid
constexpr int kMaxEgridPoints = 1 << 17;

static frg_status check_egrid(const frg_params *p, const frg_egrid *e) {
    if (!p || !e) return fail(FRG_EINVAL, "null parameters");
    if (p->N < 4 || p->N > 256 || p->N % 4 != 0)
        return fail(FRG_EINVAL, "N must satisfy 4 <= N <= 256 and N % 4 == 0");
    if (!std::isfinite(p->t) || !std::isfinite(p->tp) || !std::isfinite(p->mu) || !std::isfinite(p->U) ||
        p->t == 0.0)
        return fail(FRG_EINVAL, "model parameters must be finite and t != 0");
    if (!(std::fabs(p->tp) < 0.5 * std::fabs(p->t)))
        return fail(FRG_EINVAL, "the energy-angle grid needs |t'| < t/2 (eps monotone along rays from Gamma)");
    if (e->n_E < 1 || e->max_level < 1 || e->max_level > 12 || !(e->rtol > 0.0) || !std::isfinite(e->rtol))
        return fail(FRG_EINVAL, "egrid needs n_E >= 1, 1 <= max_level <= 12 and rtol > 0");
    return FRG_OK;
}

frg_status frg_create_egrid(const frg_params *p, const frg_egrid *e, frg_ctx *out) {
    if (!out) return fail(FRG_EINVAL, "null output handle");
    *out = nullptr;
    TRY(check_egrid(p, e));
    return create_impl(p, 1, out, e);
}

frg_status frg_points(frg_ctx ctx, int32_t *n_f, int32_t *counts) {
    TRY(check_ctx(ctx));
    const auto &g = ctx->g;
    if (n_f) *n_f = g.nf;
    if (counts)
        for (int a = 0; a < g.N; ++a) counts[a] = g.egrid ? g.count[a] : g.nf;
    return FRG_OK;
}

// n_batch: flows of the batch this context belongs to (1 alone): a batch
// needs fewer K parts per flow to fill the chip; FRG_KSPLIT overrides
static frg_status create_impl(const frg_params *p, int n_batch, frg_ctx *out, const frg_egrid *eg) {
    if (!out) return fail(FRG_EINVAL, "null output handle");
    *out = nullptr;
    if (eg) TRY(check_egrid(p, eg));
    else TRY(check_params(p));
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(FRG_EDEVICE, "no HIP device");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(FRG_EDEVICE, std::string("libfrg is built for gfx950, device is ") + prop.gcnArchName);

    frg_ctx ctx = new frg_ctx_s();
    ctx->device = dev;
    {   // the static scratch of this device, looked up once per device with it current
        const hipError_t e = frg::scratch_address(&ctx->d_scratch);
        if (e != hipSuccess) {
            delete ctx;
            return fail(FRG_EDEVICE, std::string("static scratch: ") + hipGetErrorString(e));
        }
    }
    if (n_batch > 1) {   // measured at N = 96: 8 parts for 16 flows, 4 for 64
        ctx->ks_target = (6912 + n_batch - 1) / n_batch;
        ctx->ks_lo = 4;
    }
    if (const char *e = std::getenv("FRG_KSPLIT")) ctx->ks_override = std::atoi(e);
    if (!eg) {
        frg::build_geometry(*p, ctx->g);
    } else if (!frg::build_geometry_egrid(*p, *eg, kMaxEgridPoints, ctx->g)) {
        delete ctx;
        return fail(FRG_ENOTSUP, "energy-angle grid: more than " + std::to_string(kMaxEgridPoints) +
                                     " points in a patch");
    }
    const auto &g = ctx->g;
    ctx->Trows = g.Tpp + g.Tph;
    ctx->n3 = static_cast<int64_t>(g.N) * g.N * g.N;
    auto bail = [&](frg_status st) { std::string m = g_err; frg_destroy(ctx); g_err = m; return st; };

    std::vector<double> qrow(2 * static_cast<size_t>(ctx->Trows)), trig_row(4 * static_cast<size_t>(ctx->Trows));
    for (int r = 0; r < ctx->Trows; ++r) {
        const double *q = r < g.Tpp ? &g.qpp[2 * r] : &g.qph[2 * (r - g.Tpp)];
        qrow[2 * r] = q[0];
        qrow[2 * r + 1] = q[1];
        trig_row[4 * r] = std::cos(q[0]);
        trig_row[4 * r + 1] = std::sin(q[0]);
        trig_row[4 * r + 2] = std::cos(q[1]);
        trig_row[4 * r + 3] = std::sin(q[1]);
    }
    std::vector<double> trig_pt(4 * static_cast<size_t>(g.np));
    for (int i = 0; i < g.np; ++i) {
        trig_pt[i] = std::cos(g.px[i]);
        trig_pt[g.np + i] = std::sin(g.px[i]);
        trig_pt[2 * g.np + i] = std::cos(g.py[i]);
        trig_pt[3 * g.np + i] = std::sin(g.py[i]);
    }
    std::vector<int32_t> cpp(static_cast<size_t>(g.N) * g.N), cph(static_cast<size_t>(g.N) * g.N);
    for (int y = 0; y < g.N; ++y)
        for (int x = 0; x < g.N; ++x) {
            cpp[y * g.N + x] = g.row_pp[y * g.N + x] << 3;   // column (j1=y, j2=x)
            cph[y * g.N + x] = g.row_ph[x * g.N + y] << 3;   // column (y, x): transfer k_x - k_y
        }
    double *d_px = nullptr, *d_py = nullptr, *d_qrow = nullptr;
    frg_status st;
    if ((st = upload(ctx, &ctx->d_bnd, g.bnd.data(), g.bnd.size())) ||
        (st = upload(ctx, &ctx->d_xi, g.xi.data(), g.xi.size())) ||
        (st = upload(ctx, &ctx->d_w, g.w.data(), g.w.size())) ||
        (st = upload(ctx, &ctx->d_trig_row, trig_row.data(), trig_row.size())) ||
        (st = upload(ctx, &ctx->d_trig_pt, trig_pt.data(), trig_pt.size())) ||
        (st = upload(ctx, &ctx->d_colrow_pp, cpp.data(), cpp.size())) ||
        (st = upload(ctx, &ctx->d_colrow_ph, cph.data(), cph.size())) ||
        (st = dalloc(ctx, &ctx->d_bins, static_cast<size_t>(ctx->Trows) * g.np)) ||
        (g.egrid && (st = upload(ctx, &ctx->d_count, g.count.data(), g.count.size()))))
        return bail(st);
    size_t tmp_bytes = 0;
    if ((st = upload(ctx, &d_px, g.px.data(), g.px.size())) ||
        (st = upload(ctx, &d_py, g.py.data(), g.py.size())) ||
        (st = upload(ctx, &d_qrow, qrow.data(), qrow.size()))) {
        hipFree(d_px); hipFree(d_py); hipFree(d_qrow);
        return bail(st);
    }
    tmp_bytes = sizeof(double) * (2 * g.np + qrow.size());
    frg::launch_bins(ctx->d_bnd, d_px, d_py, d_qrow, g.N, g.n_rad, g.n_ang, g.Tpp, ctx->Trows, ctx->d_bins,
                     nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    hipFree(d_px);
    hipFree(d_py);
    hipFree(d_qrow);
    ctx->ws_bytes -= tmp_bytes;
    if (e != hipSuccess) {
        g_err = std::string("second-line table: ") + hipGetErrorString(e);
        return bail(FRG_EDEVICE);
    }
    if ((st = build_orbits(ctx))) return bail(st);
    if ((st = build_ktiles(ctx))) return bail(st);
    *out = ctx;
    return FRG_OK;
}

frg_status frg_destroy(frg_ctx ctx) {
    if (!ctx) return FRG_OK;
    void *ptrs[] = {ctx->d_bnd, ctx->d_xi, ctx->d_w, ctx->d_trig_row, ctx->d_trig_pt, ctx->d_bins, ctx->d_count,
                    ctx->d_sigD,
                    ctx->d_colrow_pp, ctx->d_colrow_ph, ctx->d_pa64, ctx->d_T, ctx->d_pa32,
                    ctx->d_B64, ctx->d_B32, ctx->d_perm, ctx->d_ahl, ctx->d_g32, ctx->d_C,
                    ctx->d_yt, ctx->d_y5, ctx->d_partial, ctx->d_state, ctx->d_rowlist, ctx->d_rowlist_ph,
                    ctx->d_colsym_pp, ctx->d_colsym_ph, ctx->d_perm8, ctx->d_yr, ctx->d_ytr, ctx->d_y5r};
    for (void *p : ptrs)
        if (p) hipFree(p);
    for (int c = 0; c < 2; ++c)
        for (TileSet *ts : {&ctx->ts_full[c], &ctx->ts_vsym[c], &ctx->ts_dense[c]})
            for (int32_t *p : {ts->d_cperm, ts->d_cmap, ts->d_koff, ts->d_klist})
                if (p) hipFree(p);
    for (int j = 0; j < 7; ++j)
        if (ctx->d_k[j]) hipFree(ctx->d_k[j]);
    if (ctx->h_state) hipHostFree(ctx->h_state);
    ctx->pf.destroy();
    if (ctx->sg.exec) hipGraphExecDestroy(ctx->sg.exec);
    if (ctx->sg.ev_in) hipEventDestroy(ctx->sg.ev_in);
    if (ctx->sg.ev_out) hipEventDestroy(ctx->sg.ev_out);
    if (ctx->sg.stream) hipStreamDestroy(ctx->sg.stream);
    delete ctx;
    return FRG_OK;
}

frg_status frg_sizes(frg_ctx ctx, size_t *n_v, size_t *n_bpp, size_t *n_bph, size_t *ws) {
    TRY(check_ctx(ctx));
    const size_t NN = static_cast<size_t>(ctx->g.N) * ctx->g.N;
    if (n_v) *n_v = static_cast<size_t>(ctx->n3);
    if (n_bpp) *n_bpp = NN * ctx->g.Tpp;
    if (n_bph) *n_bph = NN * ctx->g.Tph;
    if (ws) *ws = ctx->ws_bytes;
    return FRG_OK;
}

frg_status frg_tables(frg_ctx ctx, double *kc, double *bnd, double *fine, double *qpp, double *qph,
                      int32_t *idx4) {
    TRY(check_ctx(ctx));
    const auto &g = ctx->g;
    if (kc) std::memcpy(kc, g.kc.data(), sizeof(double) * g.kc.size());
    if (bnd) std::memcpy(bnd, g.bnd.data(), sizeof(double) * g.bnd.size());
    if (fine)
        for (int i = 0; i < g.np; ++i) {
            fine[4 * i] = g.px[i];
            fine[4 * i + 1] = g.py[i];
            fine[4 * i + 2] = g.w[i];
            fine[4 * i + 3] = g.xi[i];
        }
    if (qpp) std::memcpy(qpp, g.qpp.data(), sizeof(double) * g.qpp.size());
    if (qph) std::memcpy(qph, g.qph.data(), sizeof(double) * g.qph.size());
    if (idx4) frg::host_idx4(g, idx4);
    return FRG_OK;
}

static frg_status check_params(const frg_params *p) {
    if (!p) return fail(FRG_EINVAL, "null parameters");
    if (p->N < 4 || p->N > 256 || p->N % 4 != 0)
        return fail(FRG_EINVAL, "N must satisfy 4 <= N <= 256 and N % 4 == 0");
    if (p->n_rad < 1 || p->n_ang < 1) return fail(FRG_EINVAL, "n_rad, n_ang must be >= 1");
    if (static_cast<int64_t>(p->n_rad) * p->n_ang > 1024)
        return fail(FRG_ENOTSUP, "n_rad * n_ang > 1024 points per patch is not supported");
    if (!std::isfinite(p->t) || !std::isfinite(p->tp) || !std::isfinite(p->mu) ||
        !std::isfinite(p->U) || p->t == 0.0)
        return fail(FRG_EINVAL, "model parameters must be finite and t != 0");
    return FRG_OK;
}

frg_status frg_host_tables(const frg_params *p, double *kc, double *bnd, double *fine, double *qpp,
                           double *qph, int32_t *idx4) {
    TRY(check_params(p));
    frg_ctx_s tmp;
    frg::build_geometry(*p, tmp.g);
    return frg_tables(&tmp, kc, bnd, fine, qpp, qph, idx4);
}

frg_status frg_host_tables_egrid(const frg_params *p, const frg_egrid *e, int32_t *n_f, int32_t *counts,
                                 double *kc, double *bnd, double *fine, double *qpp, double *qph, int32_t *idx4) {
    TRY(check_egrid(p, e));
    frg_ctx_s tmp;
    if (!frg::build_geometry_egrid(*p, *e, kMaxEgridPoints, tmp.g))
        return fail(FRG_ENOTSUP, "energy-angle grid: more than " + std::to_string(kMaxEgridPoints) +
                                     " points in a patch");
    TRY(frg_points(&tmp, n_f, counts));
    return frg_tables(&tmp, kc, bnd, fine, qpp, qph, idx4);
}

frg_status frg_bins(frg_ctx ctx, int32_t kind, uint8_t *d_out, void *stream) {
    TRY(check_ctx(ctx));
    if (!d_out) return fail(FRG_EINVAL, "null output");
    if (kind != 0 && kind != 1) return fail(FRG_EINVAL, "kind must be 0 (ph) or 1 (pp)");
    const auto &g = ctx->g;
    frg::launch_bins_export(ctx->d_bins, g.N, g.n_rad, g.n_ang, kind == 1 ? 0 : g.Tpp, kind == 1 ? g.Tpp : g.Tph,
                            d_out, static_cast<hipStream_t>(stream));
    HIPCHK(hipGetLastError());
    return FRG_OK;
}

frg_status frg_bubbles(frg_ctx ctx, double T, frg_precision prec, void *d_bpp, void *d_bph,
                       void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_prec(prec));
    if (!(T > 0.0) || !std::isfinite(T)) return fail(FRG_EINVAL, "T must be finite and > 0");
    if ((d_bpp && !aligned8(d_bpp)) || (d_bph && !aligned8(d_bph)))
        return fail(FRG_EINVAL, "misaligned output");
    TRY(ensure_rhs_ws(ctx, prec));
    return run_bubbles(ctx, prec == FRG_PREC_SPLIT_BF16, T, nullptr, 0.0, d_bpp, d_bph,
                       static_cast<hipStream_t>(stream));
}

frg_status frg_bubble_reps(frg_ctx ctx, int32_t *n_rep, int32_t *pp_rows, int32_t *ph_rows) {
    TRY(check_ctx(ctx));
    if (!ctx->sym_avail) return fail(FRG_ENOTSUP, "no C4v row reduction on this grid (N % 8 != 0)");
    const size_t n = ctx->h_rowlist.size();
    if (n_rep) *n_rep = static_cast<int32_t>(n);
    for (size_t i = 0; i < n; ++i) {
        if (pp_rows) pp_rows[i] = ctx->h_rowlist[i];
        if (ph_rows) ph_rows[i] = ctx->h_rowlist_ph[i] - ctx->g.Tpp;
    }
    return FRG_OK;
}

frg_status frg_bubbles_reps(frg_ctx ctx, double T, frg_precision prec, void *d_bpp, void *d_bph,
                            void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_prec(prec));
    if (!ctx->sym_avail) return fail(FRG_ENOTSUP, "no C4v row reduction on this grid (N % 8 != 0)");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(FRG_EINVAL, "T must be finite and > 0");
    if (!d_bpp || !d_bph) return fail(FRG_EINVAL, "the paired sweep writes both outputs");
    if (!aligned8(d_bpp) || !aligned8(d_bph)) return fail(FRG_EINVAL, "misaligned output");
    TRY(ensure_rhs_ws(ctx, prec));
    return run_bubbles(ctx, prec == FRG_PREC_SPLIT_BF16, T, nullptr, 0.0, d_bpp, d_bph,
                       static_cast<hipStream_t>(stream), true);
}

frg_status frg_rhs(frg_ctx ctx, double T, const double *d_V, double *d_F, frg_precision prec,
                   void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_prec(prec));
    if (!(T > 0.0) || !std::isfinite(T)) return fail(FRG_EINVAL, "T must be finite and > 0");
    if (!d_V || !d_F) return fail(FRG_EINVAL, "null V or F");
    if (!aligned8(d_V) || !aligned8(d_F)) return fail(FRG_EINVAL, "V and F must be 8-byte aligned");
    const size_t bytes = sizeof(double) * (static_cast<size_t>(ctx->n3) + (ctx->se_on ? ctx->g.N : 0));
    if (overlap(d_V, bytes, d_F, bytes)) return fail(FRG_EINVAL, "V and F overlap");
    TRY(ensure_rhs_ws(ctx, prec));
    return run_rhs(ctx, prec == FRG_PREC_SPLIT_BF16, T, nullptr, 0.0, d_V, d_F, 0,
                   static_cast<hipStream_t>(stream));
}

frg_status frg_rhs_noalloc(frg_ctx ctx, double T, const double *d_V, double *d_F, frg_precision prec,
                           void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_prec(prec));
    if (!(T > 0.0) || !std::isfinite(T)) return fail(FRG_EINVAL, "T must be finite and > 0");
    if (!d_V || !d_F) return fail(FRG_EINVAL, "null V or F");
    if (!aligned8(d_V) || !aligned8(d_F)) return fail(FRG_EINVAL, "V and F must be 8-byte aligned");
    const size_t bytes = sizeof(double) * static_cast<size_t>(ctx->n3);
    if (overlap(d_V, bytes, d_F, bytes)) return fail(FRG_EINVAL, "V and F overlap");
    if (!ctx->d_scratch) return fail(FRG_EDEVICE, "no static scratch on this device");
    if (ctx->se_on) return fail(FRG_ENOTSUP, "frg_rhs_noalloc takes no self-energy");
    // the workspace of one rhs, carved from the scratch in 256-byte aligned pieces
    const bool split = prec == FRG_PREC_SPLIT_BF16;
    const auto &g = ctx->g;
    const size_t NN = static_cast<size_t>(g.N) * g.N, n3 = static_cast<size_t>(ctx->n3);
    const size_t np = static_cast<size_t>(g.np);
    const size_t rows = ctx->sym_on ? static_cast<size_t>(ctx->n_rep_pp + ctx->n_rep_ph)
                                    : static_cast<size_t>(ctx->Trows);
    size_t off = 0;
    auto take = [&off](size_t nbytes) {
        const size_t o = off;
        off += (nbytes + 255) & ~static_cast<size_t>(255);
        return o;
    };
    const size_t o_T = take(4 * sizeof(double));
    const size_t esz = split ? sizeof(float) : sizeof(double);
    const size_t o_pa = take(3 * np * esz);
    const size_t o_B = take(rows * NN * esz);
    const size_t o_perm = split ? 0 : take(5 * n3 * sizeof(double));
    const size_t o_ahl = split ? take(6 * n3 * sizeof(uint16_t)) : 0;
    const size_t o_g32 = split ? take(3 * n3 * sizeof(float)) : 0;
    const size_t o_C = take(c_elems_needed(ctx) * sizeof(double));
    if (off > frg::kScratchBytes)
        return fail(FRG_ENOTSUP, "frg_rhs_noalloc: this context and precision need " + std::to_string(off) +
                                     " bytes of workspace; the static scratch holds " +
                                     std::to_string(frg::kScratchBytes));
    char *base = static_cast<char *>(ctx->d_scratch);
    RhsWs w;
    w.own = false;
    w.T = reinterpret_cast<double *>(base + o_T);
    if (split) {
        w.pa32 = reinterpret_cast<float *>(base + o_pa);
        w.B32 = reinterpret_cast<float *>(base + o_B);
        w.ahl = reinterpret_cast<uint16_t *>(base + o_ahl);
        w.g32 = reinterpret_cast<float *>(base + o_g32);
    } else {
        w.pa64 = reinterpret_cast<double *>(base + o_pa);
        w.B64 = reinterpret_cast<double *>(base + o_B);
        w.perm = reinterpret_cast<double *>(base + o_perm);
    }
    w.C = reinterpret_cast<double *>(base + o_C);
    // event timing would create events: not in this call
    const bool prof = ctx->pf.on;
    ctx->pf.on = false;
    const frg_status st = run_rhs(ctx, split, T, nullptr, 0.0, d_V, d_F, 0, static_cast<hipStream_t>(stream),
                                  RHS_DT, false, nullptr, &w);
    ctx->pf.on = prof;
    return st;
}

frg_status frg_flow_init(frg_ctx ctx, const frg_flow_opts *o, const double *d_V, double *d_state,
                         void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_opts(ctx, o));
    if (!d_V || !d_state || !aligned8(d_V) || !aligned8(d_state))
        return fail(FRG_EINVAL, "null or misaligned V / state");
    if (ctx->vsym_on) {   // a flow from a C4v-invariant vertex stays invariant
        double dev = 0.0;
        TRY(vsym_deviation(ctx, d_V, static_cast<hipStream_t>(stream), &dev));
        if (!(dev <= kVsymTol))
            return fail(FRG_EINVAL, "symmetric-vertex mode needs a C4v-invariant V (relative deviation " +
                                        std::to_string(dev) + ")");
    }
    if (ctx->se_on && ctx->se_sym) TRY(check_se_sym(ctx, d_V + ctx->n3, static_cast<hipStream_t>(stream)));
    TRY(ensure_rhs_ws(ctx, o->prec));
    TRY(ensure_flow_ws(ctx));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double s0 = std::log(o->T0), smin = std::log(o->T_min);
    const double dir = smin < s0 ? -1.0 : 1.0;
    double h;
    if (o->stepper == FRG_RK4) {
        h = (smin - s0) / static_cast<double>(o->fixed_steps);
    } else {
        h = o->h0 == 0.0 ? 0.01 : std::fabs(o->h0);
        h *= dir;
    }
    frg::launch_state_init(d_state, s0, h, smin, s);
    if (o->stepper == FRG_RK4) frg::launch_state_set(d_state, 27, o->fixed_steps, s);
    const int64_t nflow = ctx->n3 + (ctx->se_on ? ctx->g.N : 0);
    frg::launch_maxabs_to(nflow, d_V, d_state, 24, ctx->d_partial, red_blocks(nflow), s);
    if (o->stepper == FRG_DP54) {
        // first stage of the first step (later steps reuse the last stage: FSAL)
        TRY(run_rhs(ctx, o->prec == FRG_PREC_SPLIT_BF16, 0.0, d_state, 0.0, d_V, ctx->d_k[0], 1, s, RHS_DT,
                    red_state(ctx)));
        frg::launch_state_set(d_state, FRG_ST_RHS, 1.0, s);
    }
    HIPCHK(hipGetLastError());
    return FRG_OK;
}

// one step attempt; iflow: an interaction-flow step (stored bubbles, rhs not
// scaled by T), else a temperature-flow step in s = ln T
static frg_status flow_step_impl(frg_ctx ctx, const frg_flow_opts *o, double *V, double *state,
                                 double *log, int log_cap, hipStream_t s, bool iflow = false) {
    const RhsMode mode = iflow ? RHS_STORED : RHS_DT;
    const int scale = iflow ? 0 : 1;
    const bool split = o->prec == FRG_PREC_SPLIT_BF16;
    // reduced state: the stages combine nst-entry vectors (y gathered from V),
    // and each stage input is expanded into a full vertex for the rhs
    const bool red = red_state(ctx);
    // the self-energy flows in the same array, after V (after the reduced
    // entries in a reduced state)
    const bool se = ctx->se_on && !iflow;
    const int N = ctx->g.N;
    const int64_t n = (red ? ctx->nst : ctx->n3) + (se ? N : 0);
    double *y = red ? ctx->d_yr : V, *yt = red ? ctx->d_ytr : ctx->d_yt, *y5 = red ? ctx->d_y5r : ctx->d_y5;
    const int32_t *cperm = tiles_of(ctx, 0).d_cperm, *cmap = col_pos(ctx, 0);
    // the rhs input of a stage whose combination went to out (its full form;
    // the split layout reads a reduced one directly)
    auto full_of = [&](double *out) -> const double * {
        if (!red || split) return out;
        double *full = out == y5 ? ctx->d_y5 : ctx->d_yt;
        KTimer kt(ctx, FRG_K_RK, s);
        frg::launch_vred_expand(out, N, cmap, ctx->d_perm8, nullptr, full, s);
        if (se) frg::launch_accept_copy(N, nullptr, out + ctx->nst, full + ctx->n3, s);
        return full;
    };
    // accepted step: V <- y5 (expanded when reduced)
    auto accept_v = [&]() {
        if (red) {
            frg::launch_vred_expand(y5, N, cmap, ctx->d_perm8, state, V, s);
            if (se) frg::launch_accept_copy(N, state, y5 + ctx->nst, V + ctx->n3, s);
        } else {
            frg::launch_accept_copy(n, state, y5, V, s);
        }
    };
    if (red) {
        KTimer kt(ctx, FRG_K_RK, s);
        frg::launch_vred_gather(V, N, cperm, ctx->nst, y, s);
        if (se) frg::launch_accept_copy(N, nullptr, V + ctx->n3, y + ctx->nst, s);
    }
    frg::RkStageArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.n = n;
    sa.y = y;
    sa.state = state;
    for (int j = 0; j < 7; ++j) sa.k[j] = ctx->d_k[j];
    if (o->stepper == FRG_DP54) {
        for (int st = 1; st < 7; ++st) {
            sa.nk = st;
            for (int j = 0; j < 7; ++j) sa.coef[j] = j < st ? DP_A[st][j] : 0.0;
            sa.out = st == 6 ? y5 : yt;
            {
                KTimer kt(ctx, FRG_K_RK, s);
                if (st == 1) frg::launch_pre_step(state, FRG_DP54, s);
                frg::launch_rk_stage(sa, s);
            }
            TRY(run_rhs(ctx, split, 0.0, state, DP_C[st], full_of(sa.out), ctx->d_k[st], scale, s, mode, red,
                        red && split ? sa.out : nullptr));
        }
        const double *kk[7];
        for (int j = 0; j < 7; ++j) kk[j] = ctx->d_k[j];
        KTimer kt(ctx, FRG_K_RK, s);
        frg::launch_dp_error(n, y, y5, kk, DP_E, o->rtol, o->atol, state, ctx->d_partial, red_blocks(n), s);
        frg::launch_dp_control(state, log, log_cap, o->vmax, o->max_steps, FRG_DP54, s);
        accept_v();
        frg::launch_accept_copy(n, state, ctx->d_k[6], ctx->d_k[0], s);
    } else {
        frg::launch_pre_step(state, FRG_RK4, s);
        const double cs[4] = {0.0, 0.5, 0.5, 1.0};
        for (int st = 0; st < 4; ++st) {
            const double *in = V;
            if (st > 0) {
                sa.nk = st;
                for (int j = 0; j < 7; ++j) sa.coef[j] = (j == st - 1) ? cs[st] : 0.0;
                sa.out = yt;
                frg::launch_rk_stage(sa, s);
                in = full_of(yt);
            }
            TRY(run_rhs(ctx, split, 0.0, state, cs[st], in, ctx->d_k[st], scale, s, mode, red,
                        red && split && st > 0 ? yt : nullptr));
        }
        sa.nk = 4;
        const double b[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
        for (int j = 0; j < 7; ++j) sa.coef[j] = j < 4 ? b[j] : 0.0;
        sa.out = y5;
        frg::launch_rk_stage(sa, s);
        frg::launch_maxabs_to(n, y5, state, 20, ctx->d_partial, red_blocks(n), s);
        frg::launch_dp_control(state, log, log_cap, o->vmax, o->max_steps, FRG_RK4, s);
        accept_v();
    }
    HIPCHK(hipGetLastError());
    return FRG_OK;
}

// One step through a captured graph of flow_step_impl, replayed while the
// step's inputs are the same (buffers, stepper options, tile settings); the
// eager path when kernels are being timed or FRG_NO_GRAPH is set.  The graph
// runs on the context's own stream, ordered after the caller's stream by
// events.  The workspace is sized before the capture, so nothing is
// allocated inside it.
static frg_status flow_step_graph(frg_ctx ctx, const frg_flow_opts *o, double *V, double *state, double *log,
                                  int log_cap, hipStream_t cs, bool iflow) {
    if (ctx->pf.on || std::getenv("FRG_NO_GRAPH")) return flow_step_impl(ctx, o, V, state, log, log_cap, cs, iflow);
    if (!iflow) ctx->iflow_prec = -1;   // a replayed temperature step overwrites the bubbles too
    // the channel buffer the step writes is sized first, so that its address
    // (and the generation of the workspace) is part of the key
    TRY(ensure_c(ctx));
    auto P = [](const void *p) { return static_cast<double>(reinterpret_cast<uintptr_t>(p)); };
    const std::vector<double> key = {P(V), P(state), P(log), static_cast<double>(log_cap),
                                     static_cast<double>(o->stepper), static_cast<double>(o->prec), o->rtol,
                                     o->atol, o->vmax, static_cast<double>(o->max_steps), iflow ? 1.0 : 0.0,
                                     ctx->sym_on ? 1.0 : 0.0, ctx->vsym_on ? 1.0 : 0.0, ctx->kskip_on ? 1.0 : 0.0,
                                     ctx->se_on ? 1.0 : 0.0, ctx->se_sym ? 1.0 : 0.0,
                                     P(ctx->d_C), static_cast<double>(ctx->c_elems),
                                     static_cast<double>(ctx->ws_gen)};
    auto &g = ctx->sg;
    if (!g.stream) {
        HIPCHK(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&g.ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&g.ev_out, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(g.ev_in, cs));
    HIPCHK(hipStreamWaitEvent(g.stream, g.ev_in, 0));
    if (!g.exec || g.key != key) {
        if (g.exec) {
            hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(g.stream, hipStreamCaptureModeThreadLocal));
        const frg_status st = flow_step_impl(ctx, o, V, state, log, log_cap, g.stream, iflow);
        const hipError_t ce = hipStreamEndCapture(g.stream, &graph);
        if (st != FRG_OK) {
            if (graph) hipGraphDestroy(graph);
            return st;
        }
        if (ce != hipSuccess) return fail(FRG_EDEVICE, std::string("step capture: ") + hipGetErrorString(ce));
        const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.exec = nullptr;
            return fail(FRG_EDEVICE, std::string("step graph: ") + hipGetErrorString(e));
        }
        g.key = key;
    }
    HIPCHK(hipGraphLaunch(g.exec, g.stream));
    HIPCHK(hipEventRecord(g.ev_out, g.stream));
    HIPCHK(hipStreamWaitEvent(cs, g.ev_out, 0));
    return FRG_OK;
}

frg_status frg_flow_step(frg_ctx ctx, const frg_flow_opts *o, double *d_V, double *d_state,
                         void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_opts(ctx, o));
    if (!d_V || !d_state || !aligned8(d_V) || !aligned8(d_state))
        return fail(FRG_EINVAL, "null or misaligned V / state");
    TRY(ensure_rhs_ws(ctx, o->prec));
    TRY(ensure_flow_ws(ctx));
    return flow_step_graph(ctx, o, d_V, d_state, nullptr, 0, static_cast<hipStream_t>(stream), false);
}

frg_status frg_flow(frg_ctx ctx, const frg_flow_opts *o, double *d_V, double *d_log,
                    int32_t log_cap, frg_flow_result *r, void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_opts(ctx, o));
    if (!r) return fail(FRG_EINVAL, "null result");
    if (log_cap < 0 || (log_cap > 0 && !d_log)) return fail(FRG_EINVAL, "bad log buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    TRY(ensure_rhs_ws(ctx, o->prec));
    TRY(ensure_flow_ws(ctx));
    TRY(frg_flow_init(ctx, o, d_V, ctx->d_state, stream));
    const int cap = o->max_steps > 0 ? 4 * o->max_steps + 64 : 1000000;
    double *hs = ctx->h_state;
    for (int it = 0; it < cap; ++it) {
        TRY(flow_step_graph(ctx, o, d_V, ctx->d_state, d_log, log_cap, s, false));
        HIPCHK(hipMemcpyAsync(hs, ctx->d_state, sizeof(double) * FRG_STATE_LEN,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hs[FRG_ST_REASON] != 0.0) break;
    }
    std::memset(r, 0, sizeof(*r));
    r->reason = static_cast<frg_stop>(static_cast<int>(hs[FRG_ST_REASON]));
    r->T_end = std::exp(hs[FRG_ST_S]);
    r->T_c = std::exp(hs[FRG_ST_SC]);
    r->T_c_interp = std::exp(hs[FRG_ST_SC_INTERP]);
    r->accepted = static_cast<int32_t>(hs[FRG_ST_ACCEPTED]);
    r->rejected = static_cast<int32_t>(hs[FRG_ST_REJECTED]);
    r->rhs_evals = static_cast<int32_t>(hs[FRG_ST_RHS]);
    r->first_step_rhs = static_cast<int32_t>(hs[FRG_ST_FIRST_RHS]);
    if (r->reason == FRG_STOP_NONFINITE) return fail(FRG_ENONFINITE, "flow state became non-finite");
    return FRG_OK;
}

}  // extern "C"

// ---- interaction flow (Sec. 4's working example): dV/dg = F_L[V] at fixed T

namespace {

frg_status check_iopts(const frg_iflow_opts *o) {
    if (!o) return fail(FRG_EINVAL, "null interaction-flow options");
    TRY(check_prec(o->prec));
    if (o->stepper != FRG_RK4 && o->stepper != FRG_DP54) return fail(FRG_EINVAL, "unknown stepper");
    if (!(o->T > 0.0) || !std::isfinite(o->T)) return fail(FRG_EINVAL, "T must be finite and > 0");
    if (!std::isfinite(o->g0) || !std::isfinite(o->g1) || o->g0 == o->g1)
        return fail(FRG_EINVAL, "need finite g0 != g1");
    if (!(o->vmax > 0.0)) return fail(FRG_EINVAL, "vmax must be > 0");
    if (o->stepper == FRG_RK4 && o->fixed_steps <= 0) return fail(FRG_EINVAL, "RK4 needs fixed_steps > 0");
    if (o->stepper == FRG_DP54 && (!(o->rtol > 0.0) || !(o->atol >= 0.0) || !std::isfinite(o->h0)))
        return fail(FRG_EINVAL, "DP54 needs rtol > 0, atol >= 0, finite h0");
    if (o->max_steps < 0) return fail(FRG_EINVAL, "max_steps must be >= 0");
    return FRG_OK;
}

// the stepper options of an interaction flow (the temperature fields are unused)
frg_flow_opts stepper_opts(const frg_iflow_opts *o) {
    frg_flow_opts f;
    std::memset(&f, 0, sizeof(f));
    f.stepper = o->stepper;
    f.prec = o->prec;
    f.T0 = 1.0;
    f.T_min = 0.5;
    f.rtol = o->rtol;
    f.atol = o->atol;
    f.vmax = o->vmax;
    f.h0 = o->h0;
    f.fixed_steps = o->fixed_steps;
    f.max_steps = o->max_steps;
    return f;
}

// A toggle that changes the form of the flow state converts the rhs a running
// flow keeps for its next step (k[0], first same as last) to the new form.
frg_status convert_k0(frg_ctx ctx, bool was_red) {
    const bool now = red_state(ctx);
    if (was_red == now || !ctx->d_k[0] || !ctx->d_ytr) return FRG_OK;
    HIPCHK(hipDeviceSynchronize());
    const int N = ctx->g.N;
    // a self-energy's N entries follow the nst reduced or the N^3 full entries
    const size_t tail = ctx->se_on ? static_cast<size_t>(N) : 0;
    double *k0 = ctx->d_k[0];
    if (now) {
        frg::launch_vred_gather(k0, N, ctx->ts_vsym[0].d_cperm, ctx->nst, ctx->d_ytr, nullptr);
        HIPCHK(hipGetLastError());
        if (tail) HIPCHK(hipMemcpy(ctx->d_ytr + ctx->nst, k0 + ctx->n3, sizeof(double) * tail, hipMemcpyDeviceToDevice));
        HIPCHK(hipMemcpy(k0, ctx->d_ytr, sizeof(double) * (ctx->nst + tail), hipMemcpyDeviceToDevice));
    } else {
        if (tail) HIPCHK(hipMemcpy(ctx->d_yt + ctx->n3, k0 + ctx->nst, sizeof(double) * tail, hipMemcpyDeviceToDevice));
        frg::launch_vred_expand(k0, N, ctx->ts_vsym[0].d_cmap, ctx->d_perm8, nullptr, ctx->d_yt, nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpy(k0, ctx->d_yt, sizeof(double) * (ctx->n3 + tail), hipMemcpyDeviceToDevice));
    }
    HIPCHK(hipDeviceSynchronize());
    return FRG_OK;
}

frg_status check_vsym_v(frg_ctx ctx, const double *d_V, hipStream_t s) {
    if (!ctx->vsym_on) return FRG_OK;   // a flow from a C4v-invariant vertex stays invariant
    double dev = 0.0;
    TRY(vsym_deviation(ctx, d_V, s, &dev));
    if (!(dev <= kVsymTol))
        return fail(FRG_EINVAL, "symmetric-vertex mode needs a C4v-invariant V (relative deviation " +
                                    std::to_string(dev) + ")");
    return FRG_OK;
}

}  // namespace

extern "C" {

frg_status frg_bubbles_full(frg_ctx ctx, double T, frg_precision prec, void *d_bpp, void *d_bph,
                            void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_prec(prec));
    if (!(T > 0.0) || !std::isfinite(T)) return fail(FRG_EINVAL, "T must be finite and > 0");
    TRY(ensure_rhs_ws(ctx, prec));
    return run_bubbles(ctx, prec == FRG_PREC_SPLIT_BF16, T, nullptr, 0.0, d_bpp, d_bph,
                       static_cast<hipStream_t>(stream), false, true);
}

frg_status frg_rhs_full(frg_ctx ctx, double T, const double *d_V, double *d_F, frg_precision prec,
                        void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_prec(prec));
    if (!(T > 0.0) || !std::isfinite(T)) return fail(FRG_EINVAL, "T must be finite and > 0");
    if (!d_V || !d_F) return fail(FRG_EINVAL, "null V or F");
    if (!aligned8(d_V) || !aligned8(d_F)) return fail(FRG_EINVAL, "V and F must be 8-byte aligned");
    const size_t bytes = sizeof(double) * static_cast<size_t>(ctx->n3);
    if (overlap(d_V, bytes, d_F, bytes)) return fail(FRG_EINVAL, "V and F overlap");
    TRY(ensure_rhs_ws(ctx, prec));
    return run_rhs(ctx, prec == FRG_PREC_SPLIT_BF16, T, nullptr, 0.0, d_V, d_F, 0,
                   static_cast<hipStream_t>(stream), RHS_FULL);
}

frg_status frg_iflow_init(frg_ctx ctx, const frg_iflow_opts *o, const double *d_V, double *d_state,
                          void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_iopts(o));
    if (!d_V || !d_state || !aligned8(d_V) || !aligned8(d_state))
        return fail(FRG_EINVAL, "null or misaligned V / state");
    hipStream_t s = static_cast<hipStream_t>(stream);
    TRY(check_vsym_v(ctx, d_V, s));
    TRY(ensure_rhs_ws(ctx, o->prec));
    TRY(ensure_flow_ws(ctx));
    const bool split = o->prec == FRG_PREC_SPLIT_BF16;
    // the bubbles L_T, once for the whole flow, into the buffer the rhs reads
    {
        const size_t NN = static_cast<size_t>(ctx->g.N) * ctx->g.N;
        const bool sym = ctx->sym_on;
        const size_t npp_rows = sym ? static_cast<size_t>(ctx->n_rep_pp) : static_cast<size_t>(ctx->g.Tpp);
        void *bpp = split ? static_cast<void *>(ctx->d_B32) : static_cast<void *>(ctx->d_B64);
        void *bph = split ? static_cast<void *>(ctx->d_B32 + NN * npp_rows)
                          : static_cast<void *>(ctx->d_B64 + NN * npp_rows);
        TRY(run_bubbles(ctx, split, o->T, nullptr, 0.0, bpp, bph, s, sym, true));
        ctx->iflow_T = o->T;
        ctx->iflow_prec = o->prec;
    }
    const double dir = o->g1 < o->g0 ? -1.0 : 1.0;
    double h;
    if (o->stepper == FRG_RK4) {
        h = (o->g1 - o->g0) / static_cast<double>(o->fixed_steps);
    } else {
        h = o->h0 == 0.0 ? 0.01 : std::fabs(o->h0);
        h *= dir;
    }
    frg::launch_state_init(d_state, o->g0, h, o->g1, s);
    if (o->stepper == FRG_RK4) frg::launch_state_set(d_state, 27, o->fixed_steps, s);
    frg::launch_maxabs_to(ctx->n3, d_V, d_state, 24, ctx->d_partial, red_blocks(ctx->n3), s);
    if (o->stepper == FRG_DP54) {
        TRY(run_rhs(ctx, split, o->T, d_state, 0.0, d_V, ctx->d_k[0], 0, s, RHS_STORED, red_state(ctx)));
        frg::launch_state_set(d_state, FRG_ST_RHS, 1.0, s);
    }
    HIPCHK(hipGetLastError());
    return FRG_OK;
}

frg_status frg_iflow_step(frg_ctx ctx, const frg_iflow_opts *o, double *d_V, double *d_state, void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_iopts(o));
    if (!d_V || !d_state || !aligned8(d_V) || !aligned8(d_state))
        return fail(FRG_EINVAL, "null or misaligned V / state");
    if (ctx->iflow_prec != o->prec || ctx->iflow_T != o->T)
        return fail(FRG_EINVAL, "the context no longer holds the bubbles of this interaction flow "
                                "(call frg_iflow_init again)");
    const frg_flow_opts f = stepper_opts(o);
    return flow_step_graph(ctx, &f, d_V, d_state, nullptr, 0, static_cast<hipStream_t>(stream), true);
}

frg_status frg_iflow(frg_ctx ctx, const frg_iflow_opts *o, double *d_V, double *d_log, int32_t log_cap,
                     frg_iflow_result *r, void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_iopts(o));
    if (!r) return fail(FRG_EINVAL, "null result");
    if (log_cap < 0 || (log_cap > 0 && !d_log)) return fail(FRG_EINVAL, "bad log buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    TRY(ensure_rhs_ws(ctx, o->prec));
    TRY(ensure_flow_ws(ctx));
    TRY(frg_iflow_init(ctx, o, d_V, ctx->d_state, stream));
    const frg_flow_opts f = stepper_opts(o);
    const int cap = o->max_steps > 0 ? 4 * o->max_steps + 64 : 1000000;
    double *hs = ctx->h_state;
    for (int it = 0; it < cap; ++it) {
        TRY(flow_step_graph(ctx, &f, d_V, ctx->d_state, d_log, log_cap, s, true));
        HIPCHK(hipMemcpyAsync(hs, ctx->d_state, sizeof(double) * FRG_STATE_LEN, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hs[FRG_ST_REASON] != 0.0) break;
    }
    std::memset(r, 0, sizeof(*r));
    r->reason = static_cast<frg_stop>(static_cast<int>(hs[FRG_ST_REASON]));
    r->g_end = hs[FRG_ST_S];
    r->g_c = hs[FRG_ST_SC];
    r->g_c_interp = hs[FRG_ST_SC_INTERP];
    r->accepted = static_cast<int32_t>(hs[FRG_ST_ACCEPTED]);
    r->rejected = static_cast<int32_t>(hs[FRG_ST_REJECTED]);
    r->rhs_evals = static_cast<int32_t>(hs[FRG_ST_RHS]);
    r->first_step_rhs = static_cast<int32_t>(hs[FRG_ST_FIRST_RHS]);
    if (r->reason == FRG_STOP_NONFINITE) return fail(FRG_ENONFINITE, "flow state became non-finite");
    return FRG_OK;
}

}  // extern "C"

extern "C" {

frg_status frg_set_symmetry(frg_ctx ctx, int32_t enable) {
    TRY(check_ctx(ctx));
    if (enable && !ctx->sym_avail)
        return fail(FRG_ENOTSUP, "C4v row reduction unavailable (N % 8 != 0 or covariance check failed)");
    if (ctx->sym_on != (enable != 0)) ctx->iflow_prec = -1;   // the bubble rows change layout
    ctx->sym_on = enable != 0;
    return FRG_OK;
}

frg_status frg_symmetry(frg_ctx ctx, int32_t *active, int32_t *rows_computed) {
    TRY(check_ctx(ctx));
    if (active) *active = ctx->sym_on ? 1 : 0;
    if (rows_computed) *rows_computed = ctx->sym_on ? ctx->n_rep_pp + ctx->n_rep_ph : ctx->Trows;
    return FRG_OK;
}

frg_status frg_set_vsym(frg_ctx ctx, int32_t enable) {
    TRY(check_ctx(ctx));
    if (enable && ctx->se_on && !ctx->se_sym)
        return fail(FRG_EINVAL, "symmetric-vertex mode with a general (not C4v-invariant) self-energy");
    if (enable && !ctx->sym_avail)
        return fail(FRG_ENOTSUP, "symmetric-vertex mode needs an exactly C4v covariant grid (N % 8 == 0)");
    const bool was_red = red_state(ctx);
    ctx->vsym_on = enable != 0;
    return convert_k0(ctx, was_red);
}

frg_status frg_set_self_energy(frg_ctx ctx, int32_t enable) {
    TRY(check_ctx(ctx));
    if (enable < 0 || enable > 2) return fail(FRG_EINVAL, "self-energy switch: 0, 1 (general) or 2 (C4v invariant)");
    if (enable == 1 && ctx->vsym_on)
        return fail(FRG_EINVAL, "a general self-energy needs the symmetric-vertex mode off");
    if (enable && ctx->batch_member)
        return fail(FRG_ENOTSUP, "the self-energy runs on single flows only");
    if (enable == 2 && !ctx->sym_avail)
        return fail(FRG_ENOTSUP, "a C4v-invariant self-energy needs an exactly C4v covariant grid (N % 8 == 0)");
    if (enable && !ctx->d_sigD) TRY(dalloc(ctx, &ctx->d_sigD, static_cast<size_t>(ctx->g.N)));
    ctx->se_on = enable != 0;
    ctx->se_sym = enable == 2;
    return FRG_OK;
}

frg_status frg_self_energy(frg_ctx ctx, int32_t *active) {
    TRY(check_ctx(ctx));
    if (active) *active = ctx->se_on ? (ctx->se_sym ? 2 : 1) : 0;
    return FRG_OK;
}

frg_status frg_vsym(frg_ctx ctx, int32_t *active, int32_t *columns) {
    TRY(check_ctx(ctx));
    if (active) *active = ctx->vsym_on ? 1 : 0;
    if (columns) *columns = ctx->vsym_on ? ctx->ts_vsym[0].ncol : ctx->g.N * ctx->g.N;
    return FRG_OK;
}

frg_status frg_check_vsym(frg_ctx ctx, const double *d_V, double *rel_dev, void *stream) {
    TRY(check_ctx(ctx));
    if (!d_V || !rel_dev || !aligned8(d_V)) return fail(FRG_EINVAL, "null or misaligned argument");
    return vsym_deviation(ctx, d_V, static_cast<hipStream_t>(stream), rel_dev);
}

frg_status frg_set_kskip(frg_ctx ctx, int32_t enable) {
    TRY(check_ctx(ctx));
    if (!enable) TRY(ensure_dense_tiles(ctx));
    const bool was_red = red_state(ctx);
    ctx->kskip_on = enable != 0;
    return convert_k0(ctx, was_red);
}

frg_status frg_kskip(frg_ctx ctx, int32_t *active, double *executed_frac) {
    TRY(check_ctx(ctx));
    if (active) *active = ctx->kskip_on ? 1 : 0;
    if (executed_frac) {
        // against every chunk of every column (natural tiles); work weights of
        // the channels: pp 1, phc 1, phd 2 products per chunk
        const int NC = ctx->g.N * ctx->g.N;
        const double dense = static_cast<double>((NC + frg::kContractCols - 1) / frg::kContractCols) *
                             (NC / frg::kContractChunk);
        const TileSet &pp = tiles_of(ctx, 0), &ph = tiles_of(ctx, 1);
        *executed_frac = ctx->kskip_on ? (pp.chunks + 3.0 * ph.chunks) / (4.0 * dense) : 1.0;
    }
    return FRG_OK;
}

frg_status frg_profile_begin(frg_ctx ctx) {
    TRY(check_ctx(ctx));
    ctx->pf.begin();
    return FRG_OK;
}

frg_status frg_profile_end(frg_ctx ctx, double *ms, int32_t *counts) {
    TRY(check_ctx(ctx));
    return prof_collect(ctx->pf, ms, counts);
}

}  // extern "C"

namespace {

frg_status check_tuning(frg_ctx ctx, const frg_tuning *t) {
    if (!t) return fail(FRG_EINVAL, "null tuning");
    if (t->kparts < 0 || t->kparts > 64) return fail(FRG_EINVAL, "kparts must be in 1..64 (0: keep)");
    if (t->sweep_rows < 0 || t->sweep_rows > 256 || t->sweep_rows % 4 != 0)
        return fail(FRG_EINVAL, "sweep_rows must be a multiple of 4 in 4..256 (0: keep)");
    if (t->block_rows != 0 && t->block_rows != 32 && t->block_rows != 64 && t->block_rows != 96)
        return fail(FRG_EINVAL, "block_rows must be 32, 64 or 96 (0: keep)");
    (void)ctx;
    return FRG_OK;
}

// apply a checked tuning; K parts go to the tile sets of the column set in use
frg_status apply_tuning(frg_ctx ctx, const frg_tuning *t) {
    const bool moved = (t->kparts > 0 && t->kparts != ksplit(ctx)) || (t->block_rows > 0 && t->block_rows != block_rows(ctx));
    if (t->kparts > 0 && t->kparts != ksplit(ctx)) {
        const int cls_sets = 2;
        for (int cls = 0; cls < cls_sets; ++cls) {
            TileSet *ts = !ctx->kskip_on ? &ctx->ts_dense[cls] : (ctx->vsym_on ? &ctx->ts_vsym[cls] : &ctx->ts_full[cls]);
            TRY(cut_tileset(ctx, *ts, t->kparts));
        }
    }
    if (t->sweep_rows > 0) ctx->rpb = t->sweep_rows;
    if (t->block_rows > 0) ctx->bm = t->block_rows;
    // captured steps and batch descriptors hold the old offset tables and launch shapes
    if (ctx->sg.exec) {
        hipGraphExecDestroy(ctx->sg.exec);
        ctx->sg.exec = nullptr;
    }
    if (moved || t->sweep_rows > 0) ctx->ws_gen++;
    return FRG_OK;
}

frg_tuning tuning_of(frg_ctx ctx) {
    frg_tuning t;
    t.kparts = ksplit(ctx);
    t.sweep_rows = ctx->rpb > 0 ? ctx->rpb : 64;
    t.block_rows = block_rows(ctx);
    return t;
}

// the tuners' record of their candidates: per row kparts, sweep_rows,
// block_rows and the per-rhs times of the bubble, contraction + K-part sum
// classes and of all classes (ms)
struct TuneLog {
    double *p;
    int cap, rows;
    void add(const frg_tuning &t, const double *ms) {
        if (p && rows < cap) {
            double *r = p + 6 * static_cast<size_t>(rows);
            double tot = 0.0;
            for (int k = 0; k < FRG_KERNEL_CLASSES; ++k) tot += ms[k];
            r[0] = t.kparts; r[1] = t.sweep_rows; r[2] = t.block_rows;
            r[3] = ms[FRG_K_BUBBLES]; r[4] = ms[FRG_K_CONTRACT] + ms[FRG_K_COMBINE]; r[5] = tot;
        }
        rows++;
    }
};

// candidate values searched by the tuners
const int kTuneKparts[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
const int kTuneRows[] = {16, 32, 64, 128, 160, 256};
const int kTuneBm[] = {32, 64, 96};

}  // namespace

extern "C" {

frg_status frg_get_tuning(frg_ctx ctx, frg_tuning *t) {
    TRY(check_ctx(ctx));
    if (!t) return fail(FRG_EINVAL, "null tuning");
    *t = tuning_of(ctx);
    return FRG_OK;
}

frg_status frg_set_tuning(frg_ctx ctx, const frg_tuning *t) {
    TRY(check_ctx(ctx));
    TRY(check_tuning(ctx, t));
    return apply_tuning(ctx, t);
}

// Coordinate search with event-timed rhs evaluations: the sweep's rows per
// block against the bubble class time, then (block rows, K parts) against the
// contraction and combine time (the K-part sum grows with the parts).
frg_status frg_tune(frg_ctx ctx, double T, const double *d_V, double *d_F, frg_precision prec, int32_t reps,
                    frg_tuning *best, double *best_ms, double *log, int32_t log_cap, int32_t *log_rows,
                    void *stream) {
    TRY(check_ctx(ctx));
    TRY(check_prec(prec));
    if (!(T > 0.0) || !std::isfinite(T)) return fail(FRG_EINVAL, "T must be finite and > 0");
    if (!d_V || !d_F || reps < 1) return fail(FRG_EINVAL, "need V, F and reps >= 1");
    if (ctx->pf.on) return fail(FRG_EINVAL, "frg_tune while kernel timing is on");
    const bool split = prec == FRG_PREC_SPLIT_BF16;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TRY(ensure_rhs_ws(ctx, prec));
    // per-class milliseconds of one rhs, averaged over reps (one warm-up rhs first)
    auto timed = [&](double *cls_ms) -> frg_status {
        TRY(run_rhs(ctx, split, T, nullptr, 0.0, d_V, d_F, 0, s));
        ctx->pf.begin();
        for (int r = 0; r < reps; ++r) {
            const frg_status st = run_rhs(ctx, split, T, nullptr, 0.0, d_V, d_F, 0, s);
            if (st) { ctx->pf.on = false; return st; }
        }
        double ms[FRG_KERNEL_CLASSES];
        TRY(prof_collect(ctx->pf, ms, nullptr));
        for (int k = 0; k < FRG_KERNEL_CLASSES; ++k) cls_ms[k] = ms[k] / reps;
        return FRG_OK;
    };
    TuneLog tl{log, log_cap, 0};
    frg_tuning cur = tuning_of(ctx);
    double ms[FRG_KERNEL_CLASSES];
    double best_bub = 1e300;
    for (int rows : kTuneRows) {
        frg_tuning t = cur;
        t.sweep_rows = rows;
        TRY(apply_tuning(ctx, &t));
        TRY(timed(ms));
        tl.add(t, ms);
        if (ms[FRG_K_BUBBLES] < best_bub) { best_bub = ms[FRG_K_BUBBLES]; cur.sweep_rows = rows; }
    }
    TRY(apply_tuning(ctx, &cur));
    const int N = ctx->g.N;
    const int ncol = std::max(tiles_of(ctx, 0).ncol, tiles_of(ctx, 1).ncol);
    double best_con = 1e300;
    for (int bm : kTuneBm) {
        if (bm > 32 && bm - 32 >= N) continue;   // no larger tile than the rows need
        for (int ks : kTuneKparts) {
            const int64_t blocks = static_cast<int64_t>(frg::contract_kinds(split)) * ((N + bm - 1) / bm) *
                                   ((ncol + 63) / 64) * ks;
            if (blocks > 65536) continue;
            frg_tuning t = cur;
            t.block_rows = bm;
            t.kparts = ks;
            TRY(apply_tuning(ctx, &t));
            TRY(timed(ms));
            tl.add(t, ms);
            const double c = ms[FRG_K_CONTRACT] + ms[FRG_K_COMBINE];
            if (c < best_con) { best_con = c; cur.block_rows = bm; cur.kparts = ks; }
        }
    }
    TRY(apply_tuning(ctx, &cur));
    TRY(timed(ms));
    double total = 0.0;
    for (int k = 0; k < FRG_KERNEL_CLASSES; ++k) total += ms[k];
    if (best) *best = cur;
    if (best_ms) *best_ms = total;
    if (log_rows) *log_rows = tl.rows;
    return FRG_OK;
}

}  // extern "C"

// =====================================================================
// Batches of independent flows (uneven N, different model parameters):
// every kernel of an RK stage runs once for all flows, driven by work lists
// of (flow, block); the contraction is one persistent launch over the
// cost-sorted work of all flows.  A whole DP5(4) step is captured once in a
// hipGraph and replayed.
// =====================================================================
struct frg_batch_s {
    std::vector<frg_ctx> ctx;
    int n = 0, nf = 0, maxN = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    frg::FlowArgs *d_fa = nullptr;
    frg::BubbleArgs *d_ba = nullptr;
    frg::FusedContractArgs *d_ca[3] = {nullptr, nullptr, nullptr};   // per source (V, yt, y5)
    double **d_states = nullptr;
    double *d_state_all = nullptr, *h_state_all = nullptr;
    int2 *d_it_st = nullptr;   // (flow, block of 256 entries of its state: reduced or full)
    int n_st = 0;
    int2 *d_it_prep = nullptr, *d_it_bub = nullptr, *d_it_n3 = nullptr, *d_it_red = nullptr,
         *d_it_con = nullptr, *d_it_comb = nullptr, *d_it_sum = nullptr, *d_it_lay = nullptr;
    int n_bub_pair = 0;   // leading items of it_bub that belong to flows with row pairs
    int n_prep = 0, n_bub = 0, n_n3 = 0, n_red = 0, n_con = 0, n_comb = 0, n_sum = 0, n_lay = 0;
    // contraction work list grouped by block height class (32, 64, 96), each cut
    // into 8 per-XCD queues: d_q[class] = {start[8], count[8]}
    int con_count[3] = {0, 0, 0};
    int *d_q = nullptr;         // [3][16]
    int *d_counter = nullptr;   // [3][8]
    int2 *d_it_flat = nullptr;  // same items, per class in flow order (one block per item)
    int flat_start[3] = {0, 0, 0};
    // contraction dispatch: one block per work item in cost order (default), or
    // persistent blocks pulling from per-XCD queues (FRG_BATCH_DISPATCH=persistent;
    // measured 1.95x slower at N = 96)
    bool persistent = false;
    int persistent_grid = 1024;
    int built_prec = -1;            // precision the device arrays describe
    std::vector<uint64_t> built_gen;   // members' workspace generations the descriptors hold
    hipGraphExec_t exec = nullptr;
    int exec_prec = -1;
    double *d_log = nullptr;
    int log_cap = 0;
    frg_flow_opts opts{};
    bool initialised = false;
    EvProf pf;   // frg_batch_profile_begin/end: steps run eagerly with events per kernel class
};

namespace {

frg_status batch_fail_free(frg_batch b);

template <class T>
frg_status bupload(T **p, const std::vector<T> &v) {
    if (*p) { hipFree(*p); *p = nullptr; }
    void *q = nullptr;
    HIPCHK(hipMalloc(&q, sizeof(T) * (v.empty() ? 1 : v.size())));
    *p = static_cast<T *>(q);
    if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return FRG_OK;
}

// per-flow descriptors for precision prec; V of flow f is Vs[f]
frg_status batch_build(frg_batch b, frg_precision prec, double *const *Vs) {
    const bool split = prec == FRG_PREC_SPLIT_BF16;
    std::vector<frg::FlowArgs> fa(b->n);
    std::vector<frg::BubbleArgs> ba(b->n);
    std::vector<frg::FusedContractArgs> ca[3];
    for (int s = 0; s < 3; ++s) ca[s].resize(b->n);
    std::vector<double *> st(b->n);
    std::vector<int2> it_prep, it_bub, it_bub_single, it_n3, it_st, it_red, it_comb, it_sum, it_lay;
    struct Item { int2 it; int cls, queue; double flow_cost, cost; };
    std::vector<Item> con;
    for (int f = 0; f < b->n; ++f) {
        frg_ctx c = b->ctx[f];
        const auto &g = c->g;
        TRY(ensure_rhs_ws(c, prec));
        TRY(ensure_flow_ws(c));
        // the single-flow K split keeps concurrently running blocks of a flow on
        // one K range of its operands (L2 reuse); the same buffer serves frg_flow_init
        const int KS = ksplit(c);
        TRY(ensure_c(c));
        const int64_t n3 = c->n3;
        const int64_t cs = chan_stride(c);
        const size_t NN = static_cast<size_t>(g.N) * g.N;
        const bool sym = c->sym_on;
        const size_t npp_rows = sym ? static_cast<size_t>(c->n_rep_pp) : static_cast<size_t>(g.Tpp);
        void *bpp = split ? static_cast<void *>(c->d_B32) : static_cast<void *>(c->d_B64);
        void *bph = split ? static_cast<void *>(c->d_B32 + NN * npp_rows)
                          : static_cast<void *>(c->d_B64 + NN * npp_rows);
        frg::FlowArgs &A = fa[f];
        std::memset(&A, 0, sizeof(A));
        A.N = g.N; A.np = g.np; A.nred = red_blocks(n3); A.n3 = n3;
        A.xi = c->d_xi; A.w = c->d_w; A.pa64 = c->d_pa64; A.pa32 = c->d_pa32; A.Tdev = c->d_T;
        A.V = Vs[f]; A.state = b->d_state_all + static_cast<size_t>(f) * FRG_STATE_LEN;
        for (int j = 0; j < 7; ++j) A.k[j] = c->d_k[j];
        A.yt = c->d_yt; A.y5 = c->d_y5; A.partial = c->d_partial;
        A.perm = c->d_perm; A.ahl = c->d_ahl; A.g32 = c->d_g32; A.C = c->d_C; A.KS = KS;
        A.f32parts = split ? 1 : 0;
        A.cs = cs;
        A.Csum = c->d_C + 3 * KS * cs;
        A.ppos = col_pos(c, 0); A.phpos = col_pos(c, 1);
        A.perm8 = c->d_perm8;
        A.nel = computed_elems(c);
        A.red = red_state(c) ? 1 : 0;
        A.nst = c->nst;
        A.yr = c->d_yr; A.ytr = c->d_ytr; A.y5r = c->d_y5r;
        A.cperm_pp = tiles_of(c, 0).d_cperm;
        A.cperm_ph = tiles_of(c, 1).d_cperm;
        A.ncol_ph = tiles_of(c, 1).ncol;
        st[f] = A.state;
        frg::BubbleArgs bb = bubble_args(c, split, bpp, bph, c->d_pa64, c->d_pa32, c->d_T);
        if (sym) {
            bb.rowlist = c->d_rowlist;
            bb.rowlist_ph = c->d_rowlist_ph;
            bb.nrows = c->n_rep_pp;
            bb.npp_out = c->n_rep_pp;
        }
        ba[f] = bb;
        const double *srcs[3] = {Vs[f], c->d_yt, c->d_y5};
        for (int s = 0; s < 3; ++s) {
            frg::FusedContractArgs &a = ca[s][f];
            std::memset(&a, 0, sizeof(a));
            const double *V = srcs[s];
            a.N = g.N; a.KS = KS; a.n3 = n3;
            const int bm = block_rows(c);
            a.bm = bm;
            a.mtiles = (g.N + bm - 1) / bm;
            set_bubbles(c, split, sym, bpp, bph, a);
            a.colrow[frg::TERM_PP] = sym ? c->d_colsym_pp : c->d_colrow_pp;
            a.colrow[frg::TERM_PHC] = a.colrow[frg::TERM_PHD] = sym ? c->d_colsym_ph : c->d_colrow_ph;
            set_tiles(c, a);
            a.ctiles = (std::max(a.ncol[frg::TERM_PP], a.ncol[frg::TERM_PHC]) + 63) / 64;
            a.pstride = cs;
            a.C[frg::TERM_PP] = c->d_C;
            a.C[frg::TERM_PHC] = c->d_C + KS * cs;
            a.C[frg::TERM_PHD] = c->d_C + 2 * KS * cs;
            set_operands(a, split, V, c->d_perm, c->d_ahl, c->d_g32, n3);
        }
        for (int k = 0; k < (g.np + 255) / 256; ++k) it_prep.push_back(make_int2(f, k));
        const int rpb = c->rpb > 0 ? c->rpb : frg::bubble_batched_rows_per_block(bb.nrows);
        ba[f].rpb = rpb;
        const int chunks = (bb.nrows + rpb - 1) / rpb;
        for (int ch = 0; ch < chunks; ++ch)
            for (int a = 0; a < g.N; ++a)
                (bb.rowlist_ph ? it_bub : it_bub_single).push_back(make_int2(f, (ch << 8) | a));
        for (int64_t k = 0; k < (n3 + 255) / 256; ++k) it_n3.push_back(make_int2(f, static_cast<int>(k)));
        const int64_t nst = A.red ? c->nst : n3;
        for (int64_t k = 0; k < (nst + 255) / 256; ++k) it_st.push_back(make_int2(f, static_cast<int>(k)));
        for (int k = 0; k < frg::layout_blocks(g.N); ++k) it_lay.push_back(make_int2(f, k));
        const int ncomb = A.red ? static_cast<int>((c->nst + 255) / 256) : frg::combine_tiles(g.N);
        for (int k = 0; k < ncomb; ++k) it_comb.push_back(make_int2(f, k));
        for (int64_t k = 0; k < (3 * A.nel + frg::kSumPartsPerBlock - 1) / frg::kSumPartsPerBlock; ++k)
            it_sum.push_back(make_int2(f, static_cast<int>(k)));
        for (int k = 0; k < A.nred; ++k) it_red.push_back(make_int2(f, k));
        const frg::FusedContractArgs &a0 = ca[0][f];
        const int per_term = a0.mtiles * a0.ctiles * KS;
        const int bm = block_rows(c);
        const double kwork = static_cast<double>(NN) / KS * bm;
        const double fcost = 4.0 * per_term * kwork;   // whole flow
        const int cls = bm == 32 ? 0 : (bm == 64 ? 1 : 2);
        // K part ks of this flow is served by the XCDs q with q * KS / 8 == ks
        std::vector<int> rr(KS, 0);
        for (int id = 0; id < frg::contract_kinds(split) * per_term; ++id) {
            const double np_ = frg::contract_kind_products(split, id / per_term);   // heaviest kind first
            const int ks = id % KS;
            int q;
            if (KS >= 8) {
                q = ks % 8;
            } else {
                const int lo = (ks * 8 + KS - 1) / KS, hi = ((ks + 1) * 8 + KS - 1) / KS;  // [lo, hi)
                q = lo + (rr[ks]++ % std::max(1, hi - lo));
            }
            con.push_back({make_int2(f, id), cls, q, fcost, np_ * kwork});
        }
    }
    // largest flows first; within a flow its own order (heaviest channel first), so
    // the blocks running together share one flow's operands
    std::stable_sort(con.begin(), con.end(), [](const Item &x, const Item &y) {
        if (x.cls != y.cls) return x.cls > y.cls;
        if (x.queue != y.queue) return x.queue < y.queue;
        if (x.flow_cost != y.flow_cost) return x.flow_cost > y.flow_cost;
        if (x.it.x != y.it.x) return x.it.x < y.it.x;
        return x.cost > y.cost;
    });
    std::vector<int2> it_con(con.size());
    std::vector<int> qtab(3 * 16, 0);
    for (int k = 0; k < 3; ++k) b->con_count[k] = 0;
    for (size_t i = 0; i < con.size(); ++i) {
        it_con[i] = con[i].it;
        const int k = con[i].cls, q = con[i].queue;
        b->con_count[k]++;
        if (qtab[k * 16 + 8 + q]++ == 0) qtab[k * 16 + q] = static_cast<int>(i);
    }
    TRY(bupload(&b->d_q, qtab));
    {
        std::vector<Item> flat = con;
        std::stable_sort(flat.begin(), flat.end(), [](const Item &x, const Item &y) {
            if (x.cls != y.cls) return x.cls > y.cls;
            if (x.flow_cost != y.flow_cost) return x.flow_cost > y.flow_cost;
            if (x.it.x != y.it.x) return x.it.x < y.it.x;
            return x.it.y < y.it.y;
        });
        std::vector<int2> fl(flat.size());
        int seen[3] = {0, 0, 0};
        for (size_t i = 0; i < flat.size(); ++i) {
            fl[i] = flat[i].it;
            if (seen[flat[i].cls]++ == 0) b->flat_start[flat[i].cls] = static_cast<int>(i);
        }
        TRY(bupload(&b->d_it_flat, fl));
    }
    TRY(bupload(&b->d_fa, fa));
    TRY(bupload(&b->d_ba, ba));
    for (int s = 0; s < 3; ++s) TRY(bupload(&b->d_ca[s], ca[s]));
    TRY(bupload(&b->d_states, st));
    TRY(bupload(&b->d_it_prep, it_prep));
    b->n_bub_pair = static_cast<int>(it_bub.size());
    it_bub.insert(it_bub.end(), it_bub_single.begin(), it_bub_single.end());
    TRY(bupload(&b->d_it_bub, it_bub));
    TRY(bupload(&b->d_it_n3, it_n3));
    TRY(bupload(&b->d_it_st, it_st));
    TRY(bupload(&b->d_it_red, it_red));
    TRY(bupload(&b->d_it_con, it_con));
    TRY(bupload(&b->d_it_comb, it_comb));
    TRY(bupload(&b->d_it_sum, it_sum));
    TRY(bupload(&b->d_it_lay, it_lay));
    b->n_prep = static_cast<int>(it_prep.size());
    b->n_bub = static_cast<int>(it_bub.size());
    b->n_n3 = static_cast<int>(it_n3.size());
    b->n_st = static_cast<int>(it_st.size());
    b->n_red = static_cast<int>(it_red.size());
    b->n_con = static_cast<int>(it_con.size());
    b->n_comb = static_cast<int>(it_comb.size());
    b->n_sum = static_cast<int>(it_sum.size());
    b->n_lay = static_cast<int>(it_lay.size());
    b->built_prec = prec;
    b->built_gen.resize(b->n);
    for (int f = 0; f < b->n; ++f) b->built_gen[f] = b->ctx[f]->ws_gen;
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; b->exec_prec = -1; }
    return FRG_OK;
}

// rhs of every flow: input src (V, yt or y5), result T*F into k[stage]
void batch_rhs_launch(frg_batch b, bool split, double c_stage, int src, int stage, hipStream_t s) {
    const double *const *states = b->d_states;
    {
        KTimer kt(b->pf, FRG_K_PREP, s);
        frg::launch_prep_b(b->d_fa, b->d_it_prep, b->n_prep, c_stage, split, s);
    }
    {
        KTimer kt(b->pf, FRG_K_BUBBLES, s);
        frg::launch_bubbles_batched(b->d_ba, b->d_it_bub, b->n_bub_pair, b->n_bub, states, b->nf, b->maxN, split, s);
    }
    {
        KTimer kt(b->pf, FRG_K_LAYOUT, s);
        frg::launch_layout_b(b->d_fa, b->d_it_lay, b->n_lay, src, split, s);
    }
    KTimer kc(b->pf, FRG_K_CONTRACT, s);
    const int bms[3] = {32, 64, 96};
    for (int k = 2; k >= 0; --k) {
        if (!b->con_count[k]) continue;
        if (!b->persistent) {
            frg::launch_contract_items(b->d_ca[src], b->d_it_flat + b->flat_start[k], b->con_count[k], states,
                                       bms[k], split, s);
            continue;
        }
        const int grid = std::min(std::max(8, b->con_count[k]), b->persistent_grid);
        frg::launch_contract_persistent(b->d_ca[src], b->d_it_con, b->d_q + k * 16, b->d_q + k * 16 + 8,
                                        b->d_counter + 8 * k, states, grid, bms[k], split, s);
    }
}

// channel sums and the combine of every flow (the rhs into k[stage])
void batch_combine_launch(frg_batch b, int stage, hipStream_t s) {
    KTimer kt(b->pf, FRG_K_COMBINE, s);
    frg::launch_sum_parts_b(b->d_fa, b->d_it_sum, b->n_sum, s);
    frg::launch_combine_b(b->d_fa, b->d_it_comb, b->n_comb, stage, s);
}

void batch_step_launch(frg_batch b, const frg_flow_opts *o, hipStream_t s) {
    const bool split = o->prec == FRG_PREC_SPLIT_BF16;
    {
        KTimer kt(b->pf, FRG_K_RK, s);
        frg::launch_step_ctl_b(b->d_fa, b->n, 1, nullptr, 0, o->vmax, o->max_steps, s);
        frg::launch_vred_b(b->d_fa, b->d_it_st, b->n_st, frg::SRC_V, s);   // reduced flows: y from V
    }
    for (int st = 1; st < 7; ++st) {
        double coef[7] = {0};
        for (int j = 0; j < st; ++j) coef[j] = DP_A[st][j];
        const int dst = st == 6 ? frg::SRC_Y5 : frg::SRC_YT;
        {
            KTimer kt(b->pf, FRG_K_RK, s);
            frg::launch_rk_stage_b(b->d_fa, b->d_it_st, b->n_st, coef, st, dst, s);
            // reduced flows: the full rhs input (the split layout reads the reduced one)
            if (!split) frg::launch_vred_b(b->d_fa, b->d_it_n3, b->n_n3, dst, s);
        }
        batch_rhs_launch(b, split, DP_C[st], dst, st, s);
        batch_combine_launch(b, st, s);
    }
    KTimer kt(b->pf, FRG_K_RK, s);
    frg::launch_dp_error_b(b->d_fa, b->d_it_red, b->n_red, b->n, DP_E, o->rtol, o->atol, s);
    frg::launch_step_ctl_b(b->d_fa, b->n, 2, b->d_log, b->log_cap, o->vmax, o->max_steps, s);
    frg::launch_accept_b(b->d_fa, b->d_it_n3, b->n_n3, s);
}

frg_status batch_fail_free(frg_batch b) {
    std::string m = g_err;
    frg_batch_destroy(b);
    g_err = m;
    return FRG_EINVAL;
}

}  // namespace

extern "C" {

frg_status frg_batch_create(const frg_params *params, int32_t n_flows, frg_batch *out) {
    if (!out || !params || n_flows < 1) return fail(FRG_EINVAL, "need params[n_flows] with n_flows >= 1");
    *out = nullptr;
    for (int f = 0; f < n_flows; ++f) {
        TRY(check_params(&params[f]));
        if (params[f].n_rad != params[0].n_rad || params[f].n_ang != params[0].n_ang)
            return fail(FRG_EINVAL, "all flows of a batch must have the same n_rad and n_ang");
    }
    frg_batch b = new frg_batch_s();
    b->n = n_flows;
    if (const char *d = std::getenv("FRG_BATCH_DISPATCH")) b->persistent = std::strcmp(d, "persistent") == 0;
    b->nf = params[0].n_rad * params[0].n_ang;
    for (int f = 0; f < n_flows; ++f) {
        frg_ctx c = nullptr;
        frg_status st = create_impl(&params[f], n_flows, &c);
        if (st) { std::string m = g_err; frg_batch_destroy(b); g_err = m; return st; }
        c->batch_member = true;
        b->ctx.push_back(c);
        b->maxN = std::max(b->maxN, params[f].N);
    }
    hipError_t e = hipStreamCreate(&b->stream);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&b->d_counter), 24 * sizeof(int));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&b->d_state_all), sizeof(double) * FRG_STATE_LEN * n_flows);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&b->h_state_all), sizeof(double) * FRG_STATE_LEN * n_flows,
                          hipHostMallocDefault);
    if (e == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, b->ctx[0]->device) == hipSuccess)
            b->persistent_grid = 4 * prop.multiProcessorCount;
    }
    if (e != hipSuccess) {
        g_err = std::string("batch setup: ") + hipGetErrorString(e);
        frg_batch_destroy(b);
        return FRG_EDEVICE;
    }
    *out = b;
    return FRG_OK;
}

frg_status frg_batch_destroy(frg_batch b) {
    if (!b) return FRG_OK;
    for (frg_ctx c : b->ctx) frg_destroy(c);
    void *ptrs[] = {b->d_fa, b->d_ba, b->d_ca[0], b->d_ca[1], b->d_ca[2], b->d_states, b->d_state_all,
                    b->d_it_prep, b->d_it_bub, b->d_it_n3, b->d_it_st, b->d_it_red, b->d_it_con, b->d_counter,
                    b->d_q, b->d_it_flat, b->d_it_comb, b->d_it_sum, b->d_it_lay};
    for (void *p : ptrs)
        if (p) hipFree(p);
    if (b->h_state_all) hipHostFree(b->h_state_all);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->ev_in) hipEventDestroy(b->ev_in);
    if (b->ev_out) hipEventDestroy(b->ev_out);
    if (b->stream) hipStreamDestroy(b->stream);
    b->pf.destroy();
    delete b;
    return FRG_OK;
}

frg_status frg_batch_set_vsym(frg_batch b, int32_t enable) {
    if (!b) return fail(FRG_EINVAL, "null batch");
    for (frg_ctx c : b->ctx)
        if (enable && !c->sym_avail)
            return fail(FRG_ENOTSUP, "symmetric-vertex mode needs N % 8 == 0 for every flow");
    for (frg_ctx c : b->ctx) c->vsym_on = enable != 0;
    // descriptors and the captured step describe the old mode: flow_init again
    b->initialised = false;
    b->built_prec = -1;
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; b->exec_prec = -1; }
    return FRG_OK;
}

frg_status frg_batch_context(frg_batch b, int32_t i, frg_ctx *out) {
    if (!b || !out || i < 0 || i >= b->n) return fail(FRG_EINVAL, "bad batch or flow index");
    *out = b->ctx[i];
    return FRG_OK;
}

frg_status frg_batch_flow_init(frg_batch b, const frg_flow_opts *o, double *const *d_V, double *d_log,
                               int32_t log_cap, void *stream) {
    if (!b) return fail(FRG_EINVAL, "null batch");
    TRY(check_opts(b->ctx[0], o));
    if (o->stepper != FRG_DP54) return fail(FRG_ENOTSUP, "batched flows use DP54");
    if (!d_V) return fail(FRG_EINVAL, "null V array");
    if (log_cap < 0 || (log_cap > 0 && !d_log)) return fail(FRG_EINVAL, "bad log buffer");
    for (int f = 0; f < b->n; ++f)
        if (!d_V[f] || !aligned8(d_V[f])) return fail(FRG_EINVAL, "null or misaligned V");
    hipStream_t cs = static_cast<hipStream_t>(stream);
    hipStream_t s = b->stream;
    HIPCHK(hipEventRecord(b->ev_in, cs));
    HIPCHK(hipStreamWaitEvent(s, b->ev_in, 0));
    b->d_log = d_log;
    b->log_cap = log_cap;
    b->opts = *o;
    TRY(batch_build(b, o->prec, d_V));
    for (int f = 0; f < b->n; ++f)
        TRY(frg_flow_init(b->ctx[f], o, d_V[f], b->d_state_all + static_cast<size_t>(f) * FRG_STATE_LEN, s));
    HIPCHK(hipEventRecord(b->ev_out, s));
    HIPCHK(hipStreamWaitEvent(cs, b->ev_out, 0));
    b->initialised = true;
    return FRG_OK;
}

frg_status frg_batch_flow_step(frg_batch b, void *stream) {
    if (!b || !b->initialised) return fail(FRG_EINVAL, "batch flow not initialised");
    for (int f = 0; f < b->n; ++f)
        if (b->ctx[f]->ws_gen != b->built_gen[f]) {
            // a member's workspace moved (work on its context through frg_batch_context):
            // the descriptors and the captured step point at freed memory
            if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
            b->initialised = false;
            return fail(FRG_EINVAL, "the workspace of a flow of the batch was reallocated since "
                                    "frg_batch_flow_init; call it again");
        }
    hipStream_t cs = static_cast<hipStream_t>(stream);
    hipStream_t s = b->stream;
    HIPCHK(hipEventRecord(b->ev_in, cs));
    HIPCHK(hipStreamWaitEvent(s, b->ev_in, 0));
    if (std::getenv("FRG_NO_GRAPH") == nullptr && !b->pf.on) {
        if (!b->exec) {
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            batch_step_launch(b, &b->opts, s);
            HIPCHK(hipStreamEndCapture(s, &graph));
            hipError_t e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(FRG_EDEVICE, std::string("graph: ") + hipGetErrorString(e));
        }
        HIPCHK(hipGraphLaunch(b->exec, s));
    } else {
        batch_step_launch(b, &b->opts, s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(b->ev_out, s));
    HIPCHK(hipStreamWaitEvent(cs, b->ev_out, 0));
    return FRG_OK;
}

frg_status frg_batch_results(frg_batch b, frg_flow_result *r, int32_t *all_stopped) {
    if (!b || !r) return fail(FRG_EINVAL, "null argument");
    HIPCHK(hipMemcpyAsync(b->h_state_all, b->d_state_all, sizeof(double) * FRG_STATE_LEN * b->n,
                          hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    frg_status ret = FRG_OK;
    bool all = true;
    for (int f = 0; f < b->n; ++f) {
        const double *h = b->h_state_all + f * FRG_STATE_LEN;
        frg_flow_result &R = r[f];
        std::memset(&R, 0, sizeof(R));
        R.reason = static_cast<frg_stop>(static_cast<int>(h[FRG_ST_REASON]));
        R.T_end = std::exp(h[FRG_ST_S]);
        R.T_c = std::exp(h[FRG_ST_SC]);
        R.T_c_interp = std::exp(h[FRG_ST_SC_INTERP]);
        R.accepted = static_cast<int32_t>(h[FRG_ST_ACCEPTED]);
        R.rejected = static_cast<int32_t>(h[FRG_ST_REJECTED]);
        R.rhs_evals = static_cast<int32_t>(h[FRG_ST_RHS]);
        R.first_step_rhs = static_cast<int32_t>(h[FRG_ST_FIRST_RHS]);
        if (R.reason == FRG_STOP_NONFINITE) ret = FRG_ENONFINITE;
        all = all && R.reason != FRG_STOP_NONE;
    }
    if (all_stopped) *all_stopped = all ? 1 : 0;
    if (ret) return fail(ret, "a flow of the batch became non-finite");
    return FRG_OK;
}

frg_status frg_batch_flow(frg_batch b, const frg_flow_opts *o, double *const *d_V, double *d_log,
                          int32_t log_cap, frg_flow_result *r, void *stream) {
    if (!r) return fail(FRG_EINVAL, "null results");
    TRY(frg_batch_flow_init(b, o, d_V, d_log, log_cap, stream));
    const int cap = o->max_steps > 0 ? 4 * o->max_steps + 64 : 1000000;
    frg_status st = FRG_OK;
    for (int it = 0; it < cap; ++it) {
        TRY(frg_batch_flow_step(b, stream));
        int32_t all = 0;
        st = frg_batch_results(b, r, &all);
        if (st != FRG_OK || all) break;
    }
    // the captured step bakes in the options and the log buffer: re-capture next time
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    b->initialised = false;
    return st;
}

frg_status frg_batch_profile_begin(frg_batch b) {
    if (!b) return fail(FRG_EINVAL, "null batch");
    b->pf.begin();
    return FRG_OK;
}

frg_status frg_batch_profile_end(frg_batch b, double *ms, int32_t *counts) {
    if (!b) return fail(FRG_EINVAL, "null batch");
    return prof_collect(b->pf, ms, counts);
}

frg_status frg_batch_set_tuning(frg_batch b, const frg_tuning *t) {
    if (!b) return fail(FRG_EINVAL, "null batch");
    TRY(check_tuning(b->ctx[0], t));
    for (frg_ctx c : b->ctx) TRY(apply_tuning(c, t));
    // descriptors and the captured step describe the old tuning: flow_init again
    b->initialised = false;
    b->built_prec = -1;
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; b->exec_prec = -1; }
    return FRG_OK;
}

// The batch's coordinate search: every member takes the same candidate; the
// batched rhs of all flows is timed per kernel class with events.
frg_status frg_batch_tune(frg_batch b, const double *T, double *const *d_V, double *const *d_F,
                          frg_precision prec, int32_t reps, frg_tuning *best, double *best_ms, double *log,
                          int32_t log_cap, int32_t *log_rows, void *stream) {
    if (!b) return fail(FRG_EINVAL, "null batch");
    TRY(check_prec(prec));
    if (!T || !d_V || !d_F || reps < 1) return fail(FRG_EINVAL, "need T, V, F and reps >= 1");
    if (b->pf.on) return fail(FRG_EINVAL, "frg_batch_tune while kernel timing is on");
    for (int f = 0; f < b->n; ++f)
        if (!(T[f] > 0.0) || !std::isfinite(T[f]) || !d_V[f] || !d_F[f])
            return fail(FRG_EINVAL, "bad T, V or F of a flow");
    const bool split = prec == FRG_PREC_SPLIT_BF16;
    hipStream_t cs = static_cast<hipStream_t>(stream);
    hipStream_t s = b->stream;
    HIPCHK(hipEventRecord(b->ev_in, cs));
    HIPCHK(hipStreamWaitEvent(s, b->ev_in, 0));
    auto timed = [&](double *cls_ms) -> frg_status {
        TRY(batch_build(b, prec, d_V));
        for (int f = 0; f < b->n; ++f) {
            double *h = b->h_state_all + f * FRG_STATE_LEN;
            for (int i = 0; i < FRG_STATE_LEN; ++i) h[i] = 0.0;
            h[FRG_ST_S] = std::log(T[f]);
        }
        HIPCHK(hipMemcpyAsync(b->d_state_all, b->h_state_all, sizeof(double) * FRG_STATE_LEN * b->n,
                              hipMemcpyHostToDevice, s));
        batch_rhs_launch(b, split, 0.0, frg::SRC_V, 0, s);
        batch_combine_launch(b, 0, s);
        b->pf.begin();
        for (int r = 0; r < reps; ++r) {
            batch_rhs_launch(b, split, 0.0, frg::SRC_V, 0, s);
            batch_combine_launch(b, 0, s);
        }
        double ms[FRG_KERNEL_CLASSES];
        TRY(prof_collect(b->pf, ms, nullptr));
        for (int k = 0; k < FRG_KERNEL_CLASSES; ++k) cls_ms[k] = ms[k] / reps;
        HIPCHK(hipGetLastError());
        return FRG_OK;
    };
    TuneLog tl{log, log_cap, 0};
    frg_tuning cur = tuning_of(b->ctx[0]);
    cur.sweep_rows = frg::bubble_batched_rows_per_block(b->ctx[0]->sym_on ? b->ctx[0]->n_rep_pp
                                                                           : b->ctx[0]->Trows);
    for (frg_ctx c : b->ctx) TRY(apply_tuning(c, &cur));
    double ms[FRG_KERNEL_CLASSES];
    double best_bub = 1e300;
    for (int rows : kTuneRows) {
        frg_tuning t = cur;
        t.sweep_rows = rows;
        for (frg_ctx c : b->ctx) TRY(apply_tuning(c, &t));
        TRY(timed(ms));
        tl.add(t, ms);
        if (ms[FRG_K_BUBBLES] < best_bub) { best_bub = ms[FRG_K_BUBBLES]; cur.sweep_rows = rows; }
    }
    double best_con = 1e300;
    for (int bm : kTuneBm) {
        if (bm > 32 && bm - 32 >= b->maxN) continue;
        for (int ks : kTuneKparts) {
            if (ks > 32) continue;
            frg_tuning t = cur;
            t.block_rows = bm;
            t.kparts = ks;
            for (frg_ctx c : b->ctx) TRY(apply_tuning(c, &t));
            TRY(timed(ms));
            tl.add(t, ms);
            const double c = ms[FRG_K_CONTRACT] + ms[FRG_K_COMBINE];
            if (c < best_con) { best_con = c; cur.block_rows = bm; cur.kparts = ks; }
        }
    }
    for (frg_ctx c : b->ctx) TRY(apply_tuning(c, &cur));
    TRY(timed(ms));
    HIPCHK(hipStreamSynchronize(s));
    double total = 0.0;
    for (int k = 0; k < FRG_KERNEL_CLASSES; ++k) total += ms[k];
    b->initialised = false;
    b->built_prec = -1;
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; b->exec_prec = -1; }
    if (best) *best = cur;
    if (best_ms) *best_ms = total;
    if (log_rows) *log_rows = tl.rows;
    HIPCHK(hipEventRecord(b->ev_out, s));
    HIPCHK(hipStreamWaitEvent(cs, b->ev_out, 0));
    return FRG_OK;
}

frg_status frg_batch_rhs(frg_batch b, const double *T, double *const *d_V, double *const *d_F,
                         frg_precision prec, void *stream) {
    if (!b) return fail(FRG_EINVAL, "null batch");
    TRY(check_prec(prec));
    if (!T || !d_V || !d_F) return fail(FRG_EINVAL, "null argument");
    for (int f = 0; f < b->n; ++f) {
        if (!(T[f] > 0.0) || !std::isfinite(T[f])) return fail(FRG_EINVAL, "T must be finite and > 0");
        if (!d_V[f] || !d_F[f] || !aligned8(d_V[f]) || !aligned8(d_F[f]))
            return fail(FRG_EINVAL, "null or misaligned V/F");
        const size_t bytes = sizeof(double) * static_cast<size_t>(b->ctx[f]->n3);
        if (overlap(d_V[f], bytes, d_F[f], bytes)) return fail(FRG_EINVAL, "V and F overlap");
    }
    hipStream_t cs = static_cast<hipStream_t>(stream);
    hipStream_t s = b->stream;
    HIPCHK(hipEventRecord(b->ev_in, cs));
    HIPCHK(hipStreamWaitEvent(s, b->ev_in, 0));
    TRY(batch_build(b, prec, d_V));
    // per-flow state: s = ln T, h = 0, running; the result goes to k[0], then to F
    for (int f = 0; f < b->n; ++f) {
        double *h = b->h_state_all + f * FRG_STATE_LEN;
        for (int i = 0; i < FRG_STATE_LEN; ++i) h[i] = 0.0;
        h[FRG_ST_S] = std::log(T[f]);
    }
    HIPCHK(hipMemcpyAsync(b->d_state_all, b->h_state_all, sizeof(double) * FRG_STATE_LEN * b->n,
                          hipMemcpyHostToDevice, s));
    batch_rhs_launch(b, prec == FRG_PREC_SPLIT_BF16, 0.0, frg::SRC_V, 0, s);
    batch_combine_launch(b, 0, s);
    for (int f = 0; f < b->n; ++f) {
        frg_ctx c = b->ctx[f];
        // F from the channel partials (the batched combine left T*F in k[0])
        const int KS = ksplit(c);
        const int64_t cs = chan_stride(c);
        double *Cs = c->d_C + 3 * KS * cs;
        frg::launch_sum_parts(c->d_C, prec == FRG_PREC_SPLIT_BF16, KS, cs, cs, Cs, s);
        frg::launch_combine(Cs, Cs + cs, Cs + 2 * cs, false, c->g.N, 1,
                            col_pos(c, 0), col_pos(c, 1), c->d_perm8, c->d_T, 0, d_F[f], s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(b->ev_out, s));
    HIPCHK(hipStreamWaitEvent(cs, b->ev_out, 0));
    HIPCHK(hipStreamSynchronize(s));
    return FRG_OK;
}

}  // extern "C"
