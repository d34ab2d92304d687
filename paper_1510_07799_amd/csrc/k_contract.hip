// Contraction of the bubble rows with the vertex (the three one-loop channels
// of Sec. 4), as GEMM-shaped products on the matrix cores.
//
// Every channel term has the form
//     C[m, c] = sum_{k=(a,b)} A[m][k] * B_row(c)[k] * g(c, k)
// with m the free external index, c an ordered pair of the other two external
// indices, row(c) the bubble row of the transfer momentum of c, A a permuted
// copy of V (shared by all columns) and g a gathered vertex factor:
//   pp : m = j3, c = (j1,j2), A = V(a,b,j3),   g = V(j1,j2,a)
//   phc: m = j1, c = (j2,j3), A = V(j1,a,b),   g = V(b,j2,j3)
//   phd: m = j2, c = (j1,j3), A = -2V(a,j2,b)+V(j2,a,b) with g = V(j1,b,j3),
//                              plus A = V(a,j2,b)           with g = V(j1,b,a),
//        computed regrouped: A = V(j2,a,b) (the phc operand) with g = V(j1,b,j3),
//                       plus A = V(a,j2,b) with g = V(j1,b,a) - 2 V(j1,b,j3)
//
// One launch covers all three channels.  A block owns a BM x BC output tile
// of one channel over one K range (K split in KS parts to fill the chip; the
// parts are summed in a fixed order afterwards, so the result is
// deterministic).
//
// A bubble row is zero wherever no fine point of patch a has its second
// momentum in patch b (about 80% of the entries at N = 96); which entries
// these are does not depend on T.  Columns are ordered along a Hilbert curve
// of their transfer momentum, so the 64 columns of a tile have nearly the
// same nonzero pattern, and each tile iterates only over the 8-wide k chunks
// where any of its rows has a point (a list made once per context from the
// second-line table).  The skipped products are exact zeros.
//
// Per K step the A tile is read with 16-byte loads and the
// B-side tile Z = B_row(c)[k] g(c,k) is formed in registers from one bubble
// row per column; both are stored to LDS in the matrix-core operand layout,
// and the global loads of the next step are issued before the MFMAs of the
// current one.  Four waves in a 2 x 2 arrangement each own (BM/2) x (BC/2),
// so every operand fragment read from LDS feeds several MFMAs.
//   FP64:  v_mfma_f64_16x16x4f64, K step 16 (two list chunks).
//   split: A and Z as bf16 hi + lo, three v_mfma_f32_16x16x32_bf16 per
//          k-step (hi*hi + hi*lo + lo*hi), FP32 accumulation, K step 32
//          (four list chunks).
#include <algorithm>

#include "frg_internal.h"

namespace frg {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int BC = kContractCols;   // output columns (c) per block

// Pointers read from a descriptor in memory are generic to the compiler, which
// then emits FLAT accesses (they share the LDS wait counter and serialise the
// prefetch against the operand reads); every operand is in global memory, so
// say so.
#define GLOBAL_AS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const GLOBAL_AS T *gload_ptr(const T *p) {
    return reinterpret_cast<const GLOBAL_AS T *>(reinterpret_cast<uintptr_t>(p));
}
template <class T>
__device__ __forceinline__ GLOBAL_AS T *gstore_ptr(T *p) {
    return reinterpret_cast<GLOBAL_AS T *>(reinterpret_cast<uintptr_t>(p));
}
constexpr int kThreads = 256;

struct Work {
    int term, mtile, ctile, ks;
};

__host__ __device__ __forceinline__ int block_rows_of(int N) { return N <= 32 ? 32 : (N <= 64 ? 64 : 96); }

// Where a column's bubble row comes from: the stored row `row`, read through
// the inverse of C4v element o (identity for o = 0).  Patch j of the image
// row reads patch map(j) of the stored row: rotations shift, reflections
// reverse.
struct RowMap {
    int row;      // stored row
    bool refl;    // inverse element is a reflection
    int shR;      // rotation: shift; reflection: R with map(j) = R - j (mod N)
    __device__ __forceinline__ int map(int j, int N) const {
        const int v = refl ? shR - j : j + shR;
        return v >= N ? v - N : (v < 0 ? v + N : v);
    }
};

__device__ __forceinline__ RowMap decode_rowmap(int info, int N) {
    RowMap r;
    r.row = info >> 3;
    const int o = info & 7;
    const int oinv = (o & 1) ? o : ((8 - o) & 7);
    const int q = N >> 2;
    r.refl = (oinv & 1) != 0;
    r.shR = r.refl ? ((oinv + 1) >> 1) * q - 1 : (oinv >> 1) * q;
    if (r.shR >= N) r.shR -= N;
    return r;
}

// A list entry: chunk id (bits 0-12) and the patch pair (a, b) of its first
// k = 8 * chunk = a*N + b (bits 13-20 and 21-28), so no division by N is
// needed in the loop.
__device__ __forceinline__ int ent_chunk(int e) { return e & 0x1fff; }
__device__ __forceinline__ int ent_a(int e) { return (e >> 13) & 0xff; }
__device__ __forceinline__ int ent_b(int e) { return (e >> 21) & 0xff; }

// ZK consecutive entries k = kb .. kb+ZK-1 of a column's bubble row
// (k = a'*N + b', kb = a1*N + b1), gathered through the row map; VW-wide vector
// loads when the source window is contiguous and aligned, scalar loads otherwise.
template <int ZK, int VW, typename T, typename VT>
__device__ __forceinline__ void load_bubble_window(const GLOBAL_AS T *brow, const RowMap &rm, int N, int K,
                                                   int kb, int a1, int b1, bool ok, T *out) {
    if (!ok) {
#pragma unroll
        for (int q = 0; q < ZK; ++q) out[q] = T(0);
        return;
    }
    if (kb + ZK <= K && b1 + ZK <= N) {
        const int a = rm.map(a1, N);
        const int bt = rm.map(b1, N);
        const int lo = rm.refl ? bt - (ZK - 1) : bt;
        if (lo >= 0 && lo + ZK <= N && ((a * N + lo) % VW) == 0) {
            const GLOBAL_AS T *src = brow + a * N + lo;
            T tmp[ZK];
#pragma unroll
            for (int q = 0; q < ZK; q += VW) {
                const VT v = *reinterpret_cast<const GLOBAL_AS VT *>(src + q);
#pragma unroll
                for (int e = 0; e < VW; ++e) tmp[q + e] = v[e];
            }
            // a per-lane select between two fixed register orders (an index
            // computed from refl would become a dynamic register-array access)
            const bool refl = rm.refl;
#pragma unroll
            for (int q = 0; q < ZK; ++q) {
                const T fwd = tmp[q], rev = tmp[ZK - 1 - q];
                out[q] = refl ? rev : fwd;
            }
            return;
        }
    }
    int aa = a1, bb = b1;
#pragma unroll
    for (int q = 0; q < ZK; ++q) {
        out[q] = kb + q < K ? brow[rm.map(aa, N) * N + rm.map(bb, N)] : T(0);
        if (++bb == N) { bb = 0; ++aa; }
    }
}

// block -> (kind, m tile, c tile, K part); heaviest kind first
template <bool SPLIT>
__device__ __forceinline__ Work decode_block(const FusedContractArgs &P, int id) {
    const int per_term = P.mtiles * P.ctiles * P.KS;
    Work w;
    const int t = id / per_term;
    w.term = t == 0 ? TERM_PHD : (t == 1 ? TERM_PHC : TERM_PP);
    id -= t * per_term;
    w.ks = id % P.KS;
    id /= P.KS;
    w.ctile = id % P.ctiles;
    w.mtile = id / P.ctiles;
    return w;
}

// The active k chunks of a block: the entries of its K part of its column
// tile's list, G chunks per step; entries past the part read as -1 (a zero
// chunk).  Each
// thread reads only the entries of the list slots its loads serve, one step
// ahead of their use, as ordinary vector loads: a uniform (scalar) load would
// share its wait counter with the LDS traffic of the MFMA loop.
template <int G>
struct TileK {
    const GLOBAL_AS int32_t *kl;
    int nk, st_lo, st_hi;
    __device__ __forceinline__ TileK(const FusedContractArgs &P, int term, const Work &w) {
        const GLOBAL_AS int32_t *koff = gload_ptr(P.koff[term]) + static_cast<int64_t>(w.ctile) * (P.KS + 1) + w.ks;
        const int kbeg = koff[0];
        nk = koff[1] - kbeg;
        kl = gload_ptr(P.klist[term]) + kbeg;
        st_lo = 0;
        st_hi = (nk + G - 1) / G;
    }
    // chunk id in slot `slot` (0 .. G-1) of step st
    __device__ __forceinline__ int entry(int st, int slot) const {
        const int i = st * G + slot;
        return i < nk ? kl[i] : -1;
    }
};

// ------------------------------------------------------------------ FP64
template <int TERM, int BM>
__device__ __forceinline__ void body_f64(const FusedContractArgs &P, const Work &w, double *smem) {
    constexpr int BK = 16;
    constexpr int ZK = BK / 4;                          // k per thread in the Z loader
    constexpr int NP = TERM == TERM_PHD ? 2 : 1;
    constexpr int LDA = BK + 1;
    constexpr int G = BK / kContractChunk;
    constexpr int NCH = G * BM * 4;                     // 16-byte A pieces per operand and step
    constexpr int ACH = (NCH + kThreads - 1) / kThreads;
    double *sA = smem;                        // [NP][BM][LDA]
    double *sZ = smem + NP * BM * LDA;        // [NP][BC][LDA]
    const int N = P.N;
    const int K = N * N;
    const int NC = P.ncol[TERM];
    const int m0 = w.mtile * BM, c0 = w.ctile * BC;
    if (c0 >= NC) return;
    const TileK<G> tk(P, TERM, w);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const GLOBAL_AS double *A0 = gload_ptr(P.A64[TERM][0]);
    const GLOBAL_AS double *A1 = gload_ptr(P.A64[TERM][1]);
    const GLOBAL_AS double *B = gload_ptr(static_cast<const double *>(P.B[TERM]));
    const GLOBAL_AS int32_t *colrow = gload_ptr(P.colrow[TERM]);

    // A loader (chunk-major operand): piece ch is 16 bytes of row `row` of list
    // slot `slot`; consecutive lanes read consecutive bytes of one chunk
    auto apiece = [&](int i, int &slot, int &row, int &part) {
        const int ch = tid + i * kThreads;
        slot = ch / (BM * 4);
        row = (ch % (BM * 4)) >> 2;
        part = ch & 3;
    };
    // Z loader: column at tile position cl, ZK consecutive k of one list chunk
    const int cl = tid >> 2, zk = (tid & 3) * ZK;
    const int zslot = zk / kContractChunk, zoff = zk % kContractChunk;
    const bool cvalid = c0 + cl < NC;
    const int c = cvalid ? gload_ptr(P.cperm[TERM])[c0 + cl] : 0;
    const RowMap rm = decode_rowmap(cvalid ? colrow[c] : 0, N);
    const GLOBAL_AS double *brow = B + static_cast<int64_t>(rm.row) * K;
    const GLOBAL_AS double *g0 = gload_ptr(P.G64[TERM][0]) + static_cast<int64_t>(c) * N;
    const GLOBAL_AS double *g1 = TERM == TERM_PHD
                                     ? gload_ptr(P.G64[TERM][1]) + static_cast<int64_t>(c / N) * K
                                     : nullptr;

    d2_t ra[NP][ACH];
    double rb[ZK], rg0[ZK], rg1[ZK];

    // ea[i]: list entry of the slot of A piece i; ez: of the Z window
    auto load = [&](const int (&ea)[ACH], int ez) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const GLOBAL_AS double *Ap = p == 0 ? A0 : A1;
#pragma unroll
            for (int i = 0; i < ACH; ++i) {
                int slot, row, part;
                apiece(i, slot, row, part);
                const int m = m0 + row;
                if (tid + i * kThreads < NCH && ea[i] >= 0 && m < N)
                    ra[p][i] = *reinterpret_cast<const GLOBAL_AS d2_t *>(
                        Ap + (static_cast<int64_t>(ent_chunk(ea[i])) * N + m) * kContractChunk + part * 2);
                else
                    ra[p][i] = d2_t{0.0, 0.0};
            }
        }
        const bool zok = cvalid && ez >= 0;
        const int kb = zok ? ent_chunk(ez) * kContractChunk + zoff : 0;
        int a = zok ? ent_a(ez) : 0, b = zok ? ent_b(ez) + zoff : 0;
        if (b >= N) { b -= N; ++a; }
        load_bubble_window<ZK, 2, double, d2_t>(brow, rm, N, K, kb, a, b, zok, rb);
#pragma unroll
        for (int q = 0; q < ZK; ++q) {
            const bool ok = zok && kb + q < K;
            if (TERM == TERM_PP) rg0[q] = ok ? g0[a] : 0.0;
            else rg0[q] = ok ? g0[b] : 0.0;
            if (TERM == TERM_PHD) rg1[q] = ok ? g1[kb + q] : 0.0;
            if (++b == N) { b = 0; ++a; }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < ACH; ++i) {
                if (tid + i * kThreads >= NCH) continue;
                int slot, row, part;
                apiece(i, slot, row, part);
                const int kp = slot * kContractChunk + part * 2;
                sA[(p * BM + row) * LDA + kp] = ra[p][i][0];
                sA[(p * BM + row) * LDA + kp + 1] = ra[p][i][1];
            }
#pragma unroll
        for (int q = 0; q < ZK; ++q) {
            sZ[cl * LDA + zk + q] = rb[q] * rg0[q];
            // second phd product: V(j1,b,a) - 2 V(j1,b,j3) (the regrouped phd term)
            if (TERM == TERM_PHD) sZ[(BC + cl) * LDA + zk + q] = rb[q] * fma(-2.0, rg0[q], rg1[q]);
        }
    };

    constexpr int RT = BM / 32;   // row tiles of 16 per wave
    const int wm = wave & 1, wc = wave >> 1;
    d4_t acc[RT][2];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        acc[i][0] = d4_t{0.0, 0.0, 0.0, 0.0};
        acc[i][1] = d4_t{0.0, 0.0, 0.0, 0.0};
    }
    int aslot[ACH];
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
        int row, part;
        apiece(i, aslot[i], row, part);
    }
    int ea[ACH], ez;
    auto fetch = [&](int st) {
#pragma unroll
        for (int i = 0; i < ACH; ++i) ea[i] = tid + i * kThreads < NCH ? tk.entry(st, aslot[i]) : -1;
        ez = tk.entry(st, zslot);
    };
    fetch(tk.st_lo);
    if (tk.st_lo < tk.st_hi) load(ea, ez);
    fetch(tk.st_lo + 1);
    for (int st = tk.st_lo; st < tk.st_hi; ++st) {
        store();
        __syncthreads();
        if (st + 1 < tk.st_hi) {
            load(ea, ez);
            fetch(st + 2);
        }
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                double bf[2];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
                    bf[ci] = sZ[(p * BC + wc * 32 + ci * 16 + (lane & 15)) * LDA + kk * 4 + (lane >> 4)];
#pragma unroll
                for (int ri = 0; ri < RT; ++ri) {
                    const double af = sA[(p * BM + wm * (BM / 2) + ri * 16 + (lane & 15)) * LDA + kk * 4 + (lane >> 4)];
#pragma unroll
                    for (int ci = 0; ci < 2; ++ci)
                        acc[ri][ci] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf[ci], acc[ri][ci], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // f64 16x16x4 accumulator layout: lane l, register r holds row (l>>4) + 4r, column l&15;
    // output C[ks][tile position][m] (part stride pstride): a block's tile is one contiguous range
    GLOBAL_AS double *Cout = gstore_ptr(static_cast<double *>(P.C[TERM])) + static_cast<int64_t>(w.ks) * P.pstride;
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) {
        const int pos = c0 + wc * 32 + ci * 16 + (lane & 15);
        if (pos >= NC) continue;
#pragma unroll
        for (int ri = 0; ri < RT; ++ri)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * (BM / 2) + ri * 16 + (lane >> 4) + 4 * r;
                if (m < N) Cout[static_cast<int64_t>(pos) * N + m] = acc[ri][ci][r];
            }
    }
}

// ------------------------------------------------------------------ split BF16
// bf16 offset of (row r, 16-byte chunk c) in a [rows][32] LDS tile (64-byte
// rows): the four chunks of a row are XOR-swizzled by (r >> 1) ^ (r >> 3), so
// any 8 aligned consecutive rows at one chunk fill the 8 16-byte slots of a
// 128-byte bank line, and any 16 those of a 256-byte line.  The MFMA operand
// reads (16 consecutive rows per chunk) and the A stores (consecutive rows)
// then avoid the address conflicts of a 128-bit access served 8 or 16 lanes at
// a time; XOR with bits 2-3 alone gives rows r and r + 2 the same banks in the
// former case.
__device__ __forceinline__ int swz(int r, int c) { return r * 32 + ((c ^ (((r >> 1) ^ (r >> 3)) & 3)) << 3); }

// KIND = TERM_PP or TERM_PHC: one product.  KIND = TERM_PHD: two products into
// one accumulator.  The phd sum (-2 V(a,j2,b) + V(j2,a,b)) V(j1,b,j3) +
// V(a,j2,b) V(j1,b,a) is regrouped as V(j2,a,b) V(j1,b,j3) + V(a,j2,b)
// (V(j1,b,a) - 2 V(j1,b,j3)): its first operand is the phc operand V(m,a,b)
// (operand aop(p): 0 for p = 0, 1 for p = 1).  The phc and phd kinds read the
// same ph bubble rows and tile lists.  Computing phc and both phd products in
// one block would load each window once, but its two accumulator sets hold the
// kernel at 2 waves per SIMD (137 VGPRs + 48 AGPRs); apart, the kinds need at
// most 115 + 24 and run 3 waves per SIMD, which outweighs reading the phc
// operand and the windows twice.
template <int KIND, int BM, bool FAST>
__device__ __forceinline__ void body_split(const FusedContractArgs &P, const Work &w, uint16_t *smem) {
    constexpr bool PHD = KIND == TERM_PHD;
    constexpr bool PH = KIND != TERM_PP;          // a ph kind (phc or phd)
    constexpr int TT = PH ? TERM_PHC : TERM_PP;   // term whose bubble rows and tile lists are read
    constexpr int BK = 32;
    constexpr int ZK = BK / 4;    // k per thread in the Z loader
    constexpr int LD = BK;        // bf16 row pitch; chunks swizzled by swz()
    constexpr int NP = PHD ? 2 : 1;    // products (Z tiles)
    constexpr int NA = PHD ? 2 : 1;    // A operands
    constexpr int NACC = 1;
    constexpr int G = BK / kContractChunk;
    constexpr int NCH = G * BM;                         // 16-byte A pieces (one chunk of one row)
    constexpr int ACH = (NCH + kThreads - 1) / kThreads;
    uint16_t *sA = smem;                           // [NA][2][BM][LD]
    uint16_t *sZ = smem + NA * 2 * BM * LD;        // [NP][2][BC][LD]
    const int N = P.N;
    const int K = N * N;
    const int NC = P.ncol[TT];
    const int64_t n3 = P.n3;
    const int m0 = w.mtile * BM, c0 = w.ctile * BC;
    if (c0 >= NC) return;
    const TileK<G> tk(P, TT, w);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const GLOBAL_AS uint16_t *Ahl[NA];
    if constexpr (PH) {
        Ahl[0] = gload_ptr(P.Ahl[TERM_PHC][0]);
        if constexpr (PHD) Ahl[1] = gload_ptr(P.Ahl[TERM_PHD][1]);
    } else {
        Ahl[0] = gload_ptr(P.Ahl[TERM_PP][0]);
    }
    const GLOBAL_AS float *B = gload_ptr(static_cast<const float *>(P.B[TT]));
    const GLOBAL_AS int32_t *colrow = gload_ptr(P.colrow[TT]);

    // A piece ch = tid + i * kThreads: row ch % BM of list slot ch / BM, so
    // consecutive lanes read consecutive rows of one chunk (chunk-major operand)
    static_assert(ZK == kContractChunk && G == 4, "split slots");
    // Z loader: column at tile position cl, list slot zslot (one chunk)
    const int zslot = tid & 3;
    const int cl = tid >> 2;
    const bool cvalid = c0 + cl < NC;
    const int c = cvalid ? gload_ptr(P.cperm[TT])[c0 + cl] : 0;
    const RowMap rm = decode_rowmap(cvalid ? colrow[c] : 0, N);
    const GLOBAL_AS float *brow = B + static_cast<int64_t>(rm.row) * K;
    // gather factors: pp V(j1,j2,a); phc V(b,j2,j3); phd V(j1,b,j3) and V(j1,b,a)
    const GLOBAL_AS float *g0 = gload_ptr(P.G32[TT][0]) + static_cast<int64_t>(c) * N;
    const GLOBAL_AS float *gd = PHD ? gload_ptr(P.G32[TERM_PHD][0]) + static_cast<int64_t>(c) * N : nullptr;
    const GLOBAL_AS float *g1 = PHD ? gload_ptr(P.G32[TERM_PHD][1]) + static_cast<int64_t>(c / N) * K : nullptr;

    u32x4_t ra[NA][2][ACH];
    float rb[ZK], rg[2][ZK];   // pp, phc: rg[0] = the gather; phd: V(j1,b,j3), V(j1,b,a)

    // Buffer resources for the FAST path: 32-bit offsets, and an offset past
    // the end (kOOB) reads zeros, so padding entries and invalid columns need
    // no branches.  FAST needs N % 32 == 0 (a window of 8 k then stays in one
    // row of patches and contiguous after every C4v patch map) and bubble
    // rows below 2 GiB; the host checks both.
    constexpr uint32_t kOOB = 0x80000000u;
    constexpr int kFlags = 0x00020000;   // raw buffer, 32-bit data format (gfx9)
    __amdgpu_buffer_rsrc_t rA[NA], rB, rG0, rGd, rG1;
    if constexpr (FAST) {
        const uint16_t *Araw[2] = {PH ? P.Ahl[TERM_PHC][0] : P.Ahl[TERM_PP][0], P.Ahl[TERM_PHD][1]};
#pragma unroll
        for (int p = 0; p < NA; ++p)
            rA[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(Araw[p]), 0, static_cast<int>(4 * n3),
                                                      kFlags);
        rB = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(P.B[TT]), 0, static_cast<int>(P.Bbytes[TT]),
                                               kFlags);
        rG0 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(P.G32[TT][0]), 0, static_cast<int>(4 * n3),
                                                kFlags);
        if constexpr (PHD) {
            rGd = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(P.G32[TERM_PHD][0]), 0,
                                                    static_cast<int>(4 * n3), kFlags);
            rG1 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(P.G32[TERM_PHD][1]), 0,
                                                    static_cast<int>(4 * n3), kFlags);
        }
    }
    // byte offsets of the column's bubble row and gather rows
    const uint32_t brow_off = static_cast<uint32_t>(rm.row) * static_cast<uint32_t>(K) * 4u;
    const uint32_t g0_off = static_cast<uint32_t>(c) * static_cast<uint32_t>(N) * 4u;
    const uint32_t g1_off = static_cast<uint32_t>(c / N) * static_cast<uint32_t>(K) * 4u;

    auto load_fast = [&](const int (&ea)[ACH], int e) {
#pragma unroll
        for (int p = 0; p < NA; ++p)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl)
#pragma unroll
                for (int i = 0; i < ACH; ++i) {
                    const int ch = tid + i * kThreads;
                    if (ch >= NCH) continue;   // uniform per wave
                    const int m = m0 + ch % BM;
                    const uint32_t off = (ea[i] >= 0 && m < N)
                        ? ((static_cast<uint32_t>(ent_chunk(ea[i])) * N + m) * kContractChunk +
                           static_cast<uint32_t>(hl * n3)) * 2u
                        : kOOB;
                    ra[p][hl][i] = __builtin_bit_cast(u32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rA[p], off, 0, 0));
                }
        const bool zok = cvalid && e >= 0;
        const int a = ent_a(e), b = ent_b(e);
        // bubble-row window: 8 contiguous floats at (map(a), lo) of the stored row
        const int am = rm.map(a, N), bt = rm.map(b, N);
        const int lo = rm.refl ? bt - (ZK - 1) : bt;
        const uint32_t boff = zok ? brow_off + static_cast<uint32_t>(am * N + lo) * 4u : kOOB;
        const f4_t w0 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rB, boff, 0, 0));
        const f4_t w1 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rB, boff + 16u, 0, 0));
        const bool refl = rm.refl;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rb[q] = refl ? w1[3 - q] : w0[q];
            rb[q + 4] = refl ? w0[3 - q] : w1[q];
        }
        if constexpr (!PH) {
            const uint32_t go = zok ? g0_off + static_cast<uint32_t>(a) * 4u : kOOB;
            const float v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rG0, go, 0, 0));
#pragma unroll
            for (int q = 0; q < ZK; ++q) rg[0][q] = v;
        } else if constexpr (!PHD) {
            const uint32_t go = zok ? g0_off + static_cast<uint32_t>(b) * 4u : kOOB;
            const f4_t u0 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rG0, go, 0, 0));
            const f4_t u1 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rG0, go + 16u, 0, 0));
#pragma unroll
            for (int q = 0; q < 4; ++q) { rg[0][q] = u0[q]; rg[0][q + 4] = u1[q]; }
        } else {
            const uint32_t go = zok ? g0_off + static_cast<uint32_t>(b) * 4u : kOOB;
            const uint32_t g1o = zok ? g1_off + static_cast<uint32_t>(ent_chunk(e) * kContractChunk) * 4u : kOOB;
            const f4_t v0 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rGd, go, 0, 0));
            const f4_t v1 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rGd, go + 16u, 0, 0));
            const f4_t x0 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rG1, g1o, 0, 0));
            const f4_t x1 = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(rG1, g1o + 16u, 0, 0));
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                rg[0][q] = v0[q]; rg[0][q + 4] = v1[q];
                rg[1][q] = x0[q]; rg[1][q + 4] = x1[q];
            }
        }
    };

    // ea[i]: list entry of the slot of A piece i; e: of the Z window
    auto load_general = [&](const int (&ea)[ACH], int e) {
#pragma unroll
        for (int p = 0; p < NA; ++p)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl)
#pragma unroll
                for (int i = 0; i < ACH; ++i) {
                    const int ch = tid + i * kThreads;
                    const int m = m0 + ch % BM;
                    if (ch < NCH && ea[i] >= 0 && m < N)
                        ra[p][hl][i] = *reinterpret_cast<const GLOBAL_AS u32x4_t *>(
                            Ahl[p] + hl * n3 + (static_cast<int64_t>(ent_chunk(ea[i])) * N + m) * kContractChunk);
                    else
                        ra[p][hl][i] = u32x4_t{0u, 0u, 0u, 0u};
                }
        const bool zok = cvalid && e >= 0;
        const int kb = zok ? ent_chunk(e) * kContractChunk : 0;
        const int a = zok ? ent_a(e) : 0, b = zok ? ent_b(e) : 0;
        load_bubble_window<ZK, 4, float, f4_t>(brow, rm, N, K, kb, a, b, zok, rb);
        if (!zok) {
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < ZK; ++q) rg[p][q] = 0.f;
            return;
        }
        const bool inrow = b + ZK <= N;   // the window stays in one a (always when N % 8 == 0)
        if constexpr (!PH) {
            if (inrow) {
                const float v = g0[a];
#pragma unroll
                for (int q = 0; q < ZK; ++q) rg[0][q] = v;
            } else {
                int aa = a, bb = b;
#pragma unroll
                for (int q = 0; q < ZK; ++q) {
                    rg[0][q] = kb + q < K ? g0[aa] : 0.f;
                    if (++bb == N) { bb = 0; ++aa; }
                }
            }
        } else {
            // phc: V(b,j2,j3) from g0; phd: V(j1,b,j3) from gd, then V(j1,b,a) from g1
            const GLOBAL_AS float *gb = PHD ? gd : g0;
            if (inrow && (b & 3) == 0) {
#pragma unroll
                for (int q = 0; q < ZK; q += 4) {
                    const f4_t u = *reinterpret_cast<const GLOBAL_AS f4_t *>(gb + b + q);
#pragma unroll
                    for (int t = 0; t < 4; ++t) rg[0][q + t] = u[t];
                }
            } else {
                int bb = b;
#pragma unroll
                for (int q = 0; q < ZK; ++q) {
                    rg[0][q] = kb + q < K ? gb[bb] : 0.f;
                    if (++bb == N) bb = 0;
                }
            }
            if constexpr (PHD) {
                if (kb + ZK <= K) {
#pragma unroll
                    for (int q = 0; q < ZK; q += 4) {
                        const f4_t v = *reinterpret_cast<const GLOBAL_AS f4_t *>(g1 + kb + q);
#pragma unroll
                        for (int t = 0; t < 4; ++t) rg[1][q + t] = v[t];
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < ZK; ++q) rg[1][q] = kb + q < K ? g1[kb + q] : 0.f;
                }
            }
        }
    };
    auto load = [&](const int (&ea)[ACH], int e) {
        if constexpr (FAST) load_fast(ea, e);
        else load_general(ea, e);
    };
    auto store = [&]() {
#pragma unroll
        for (int p = 0; p < NA; ++p)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl)
#pragma unroll
                for (int i = 0; i < ACH; ++i) {
                    const int ch = tid + i * kThreads;
                    if (ch >= NCH) continue;
                    *reinterpret_cast<u32x4_t *>(sA + (p * 2 + hl) * BM * LD + swz(ch % BM, ch / BM)) = ra[p][hl][i];
                }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            bf8_t hi, lo;   // round-to-nearest-even conversions (v_cvt_pk_bf16_f32)
#pragma unroll
            for (int q = 0; q < ZK; ++q) {
                // phd product 1: V(j1,b,a) - 2 V(j1,b,j3) (the regrouped phd term)
                const float gq = (PHD && p == 1) ? fmaf(-2.0f, rg[0][q], rg[1][q]) : rg[0][q];
                const float z = rb[q] * gq;
                const __bf16 zh = static_cast<__bf16>(z);
                hi[q] = zh;
                lo[q] = static_cast<__bf16>(z - static_cast<float>(zh));
            }
            *reinterpret_cast<bf8_t *>(sZ + (p * 2 + 0) * BC * LD + swz(cl, zslot)) = hi;
            *reinterpret_cast<bf8_t *>(sZ + (p * 2 + 1) * BC * LD + swz(cl, zslot)) = lo;
        }
    };

    constexpr int RT = BM / 32;
    const int wm = wave & 1, wc = wave >> 1;
    f4_t acc[NACC][RT][2];
#pragma unroll
    for (int u = 0; u < NACC; ++u)
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            acc[u][i][0] = f4_t{0.f, 0.f, 0.f, 0.f};
            acc[u][i][1] = f4_t{0.f, 0.f, 0.f, 0.f};
        }
    int ea[ACH], ez;
    auto fetch = [&](int st) {
#pragma unroll
        for (int i = 0; i < ACH; ++i) {
            const int ch = tid + i * kThreads;
            ea[i] = ch < NCH ? tk.entry(st, ch / BM) : -1;
        }
        ez = tk.entry(st, zslot);
    };
    fetch(tk.st_lo);
    if (tk.st_lo < tk.st_hi) load(ea, ez);
    fetch(tk.st_lo + 1);
    for (int st = tk.st_lo; st < tk.st_hi; ++st) {
        store();
        __syncthreads();
        if (st + 1 < tk.st_hi) {
            load(ea, ez);
            fetch(st + 2);
        }
        const int kch = lane >> 4;   // the lane's 8-wide k chunk of the step
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            constexpr int u = 0;
            bf8_t zh[2], zl[2];
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
                const int zr = wc * 32 + ci * 16 + (lane & 15);
                zh[ci] = *reinterpret_cast<const bf8_t *>(sZ + (p * 2 + 0) * BC * LD + swz(zr, kch));
                zl[ci] = *reinterpret_cast<const bf8_t *>(sZ + (p * 2 + 1) * BC * LD + swz(zr, kch));
            }
#pragma unroll
            for (int ri = 0; ri < RT; ++ri) {
                const int ar = wm * (BM / 2) + ri * 16 + (lane & 15);
                const int aop = (PHD && p == 1) ? 1 : 0;
                const bf8_t ah = *reinterpret_cast<const bf8_t *>(sA + (aop * 2 + 0) * BM * LD + swz(ar, kch));
                const bf8_t al = *reinterpret_cast<const bf8_t *>(sA + (aop * 2 + 1) * BM * LD + swz(ar, kch));
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) {
                    f4_t &d = acc[u][ri][ci];
                    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, zh[ci], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, zl[ci], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, zh[ci], d, 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // bf16 16x16x32 accumulator layout: lane l, register r holds row 4(l>>4) + r, column l&15
    // output C[ks][tile position][m] in float (the accumulators' own precision):
    // four consecutive m per lane, one 16-byte store (N % 4 == 0, so a group of
    // four rows is either wholly inside or outside)
#pragma unroll
    for (int u = 0; u < NACC; ++u) {
        const int term = PHD ? TERM_PHD : (PH ? TERM_PHC : TERM_PP);
        GLOBAL_AS float *Cout = gstore_ptr(static_cast<float *>(P.C[term])) + static_cast<int64_t>(w.ks) * P.pstride;
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) {
            const int pos = c0 + wc * 32 + ci * 16 + (lane & 15);
            if (pos >= NC) continue;
#pragma unroll
            for (int ri = 0; ri < RT; ++ri) {
                const int m = m0 + wm * (BM / 2) + ri * 16 + 4 * (lane >> 4);
                if (m < N)
                    *reinterpret_cast<GLOBAL_AS f4_t *>(Cout + static_cast<int64_t>(pos) * N + m) = acc[u][ri][ci];
            }
        }
    }
}

template <int BM, bool SPLIT>
__device__ __forceinline__ void run_work(const FusedContractArgs &P, const Work &w, double *smem_d) {
    if (SPLIT) {
        uint16_t *smem = reinterpret_cast<uint16_t *>(smem_d);
        if (P.fast) {
            if (w.term == TERM_PHD) body_split<TERM_PHD, BM, true>(P, w, smem);
            else if (w.term == TERM_PHC) body_split<TERM_PHC, BM, true>(P, w, smem);
            else body_split<TERM_PP, BM, true>(P, w, smem);
        } else {
            if (w.term == TERM_PHD) body_split<TERM_PHD, BM, false>(P, w, smem);
            else if (w.term == TERM_PHC) body_split<TERM_PHC, BM, false>(P, w, smem);
            else body_split<TERM_PP, BM, false>(P, w, smem);
        }
    } else {
        if (w.term == TERM_PHD) body_f64<TERM_PHD, BM>(P, w, smem_d);
        else if (w.term == TERM_PHC) body_f64<TERM_PHC, BM>(P, w, smem_d);
        else body_f64<TERM_PP, BM>(P, w, smem_d);
    }
}

// The FP64 phd kind needs 133 VGPRs + 48 AGPRs, 2 waves per SIMD; held to 3
// waves the compiler spills 12 registers, and the kernel still runs 1-6% faster
// (every column most).  The split kinds fit 3 waves without the hint.
template <int BM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void contract_f64_fused(
    FusedContractArgs P) {
    extern __shared__ double smem_d[];
    run_work<BM, false>(P, decode_block<false>(P, blockIdx.x), smem_d);
}

template <int BM>
__global__ __launch_bounds__(kThreads) void contract_split_fused(FusedContractArgs P) {
    extern __shared__ double smem_d[];
    run_work<BM, true>(P, decode_block<true>(P, blockIdx.x), smem_d);
}

// Persistent launch over a work list of many flows.  The list of one block
// height class is cut into 8 queues, one per XCD: items of K part p of a flow
// go to the queues of the XCDs that own p (block b runs on XCD b mod 8), so
// each XCD's L2 sees one K range of the operands, as in the single-flow
// launch.  A block drains its own queue, then steals from the others; within a
// queue the items are sorted by cost, largest first, and items of flows that
// have stopped are skipped.
template <bool SPLIT, int BM>
__global__ __launch_bounds__(kThreads) void contract_persistent(const FusedContractArgs *__restrict__ args,
                                                                const int2 *__restrict__ items,
                                                                const int *__restrict__ qstart,
                                                                const int *__restrict__ qcount, int *counters,
                                                                const double *const *__restrict__ states) {
    extern __shared__ double smem_d[];
    __shared__ int next;
    const int q0 = blockIdx.x & 7;
    for (int r = 0; r < 8; ++r) {
        const int q = (q0 + r) & 7;
        const int n = qcount[q];
        const int2 *qi = items + qstart[q];
        for (;;) {
            if (threadIdx.x == 0) next = atomicAdd(&counters[q], 1);
            __syncthreads();
            const int i = __builtin_amdgcn_readfirstlane(next);
            __syncthreads();
            if (i >= n) break;
            const int2 it = qi[i];
            if (states && states[it.x][FRG_ST_REASON] != 0.0) continue;
            const FusedContractArgs P = args[it.x];
            run_work<BM, SPLIT>(P, decode_block<SPLIT>(P, it.y), smem_d);
            __syncthreads();
        }
    }
}

// One block per work item of the list, dealt by the hardware dispatcher in
// list order (the alternative to the persistent queues).
template <bool SPLIT, int BM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void contract_items(
    const FusedContractArgs *__restrict__ args, const int2 *__restrict__ items,
    const double *const *__restrict__ states) {
    extern __shared__ double smem_d[];
    const int2 it = items[blockIdx.x];
    if (states && states[it.x][FRG_ST_REASON] != 0.0) return;
    const FusedContractArgs P = args[it.x];
    run_work<BM, SPLIT>(P, decode_block<SPLIT>(P, it.y), smem_d);
}

__global__ void reset_counters(int *counters, int n) {
    if (static_cast<int>(threadIdx.x) < n) counters[threadIdx.x] = 0;
}

constexpr int contract_kinds_of(bool) { return 3; }

// LDS of one block: split [2 A operands][hi, lo] A (BM x 32) and [2 products]
// [hi, lo] Z (64 x 32) bf16 tiles (40 KB at BM = 96: three blocks per CU);
// FP64 [2 products] A (BM x 17) and Z (64 x 17) tiles
constexpr size_t lds_bytes(bool split, int bm) {
    return split ? sizeof(uint16_t) * (2 * 2 * bm * 32 + 2 * 2 * BC * 32)
                 : sizeof(double) * (2 * bm * 17 + 2 * BC * 17);
}

template <int BM>
void launch_bm(FusedContractArgs a, bool split, hipStream_t s) {
    a.mtiles = (a.N + BM - 1) / BM;
    a.ctiles = (std::max(a.ncol[TERM_PP], a.ncol[TERM_PHC]) + BC - 1) / BC;
    const int blocks = contract_kinds_of(split) * a.mtiles * a.ctiles * a.KS;
    if (split)
        hipLaunchKernelGGL(contract_split_fused<BM>, dim3(blocks), dim3(kThreads), lds_bytes(true, BM), s, a);
    else
        hipLaunchKernelGGL(contract_f64_fused<BM>, dim3(blocks), dim3(kThreads), lds_bytes(false, BM), s, a);
}

// flags of the k chunks of the column tiles: block p scans the second-line
// table row of the column at tile position p and marks, in its tile's flags
// (zeroed by the caller), every chunk k / 8 with k = a*N + b that holds a point
// (byte stores of 1, so concurrent blocks of one tile need no atomics)
__global__ __launch_bounds__(256) void tile_pattern_kernel(const uint8_t *__restrict__ bins,
                                                           const int32_t *__restrict__ colfull,
                                                           const int32_t *__restrict__ cperm, int ncol, int N,
                                                           int nf, int np, uint8_t *__restrict__ flags) {
    const int NC = N * N, nch = NC / kContractChunk;
    const int p = blockIdx.x;
    if (p >= ncol) return;
    uint8_t *tf = flags + static_cast<int64_t>(p / BC) * nch;
    const uint8_t *row = bins + static_cast<int64_t>(colfull[cperm[p]]) * np;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const int k = (i / nf) * N + row[i];
        tf[k / kContractChunk] = 1;
    }
}

}  // namespace


int contract_block_rows(int N) { return block_rows_of(N); }

void launch_tile_pattern(const uint8_t *bins, const int32_t *colfull, const int32_t *cperm, int ncol, int N,
                         int nf, int np, uint8_t *flags, hipStream_t s) {
    hipLaunchKernelGGL(tile_pattern_kernel, dim3(ncol), dim3(256), 0, s, bins, colfull, cperm, ncol, N, nf, np,
                       flags);
}

size_t contract_lds_bytes(bool split) { return lds_bytes(split, 96); }

int contract_kinds(bool split) { return contract_kinds_of(split); }

int contract_kind_products(bool split, int kind) {
    if (split) return kind == 0 ? 2 : 1;
    return kind == 0 ? 2 : 1;
}

template <bool SPLIT, int BM>
void launch_persistent_bm(const FusedContractArgs *args, const int2 *items, const int *qstart,
                          const int *qcount, int *counters, const double *const *states, int grid,
                          hipStream_t s) {
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, counters, 8);
    hipLaunchKernelGGL((contract_persistent<SPLIT, BM>), dim3(grid), dim3(kThreads), contract_lds_bytes(SPLIT),
                       s, args, items, qstart, qcount, counters, states);
}

template <bool SPLIT, int BM>
void launch_items_bm(const FusedContractArgs *args, const int2 *items, int nitems, const double *const *states,
                     hipStream_t s) {
    hipLaunchKernelGGL((contract_items<SPLIT, BM>), dim3(nitems), dim3(kThreads), contract_lds_bytes(SPLIT), s,
                       args, items, states);
}

void launch_contract_items(const FusedContractArgs *args, const int2 *items, int nitems,
                           const double *const *states, int bm, bool split, hipStream_t s) {
    if (split) {
        if (bm == 32) launch_items_bm<true, 32>(args, items, nitems, states, s);
        else if (bm == 64) launch_items_bm<true, 64>(args, items, nitems, states, s);
        else launch_items_bm<true, 96>(args, items, nitems, states, s);
    } else {
        if (bm == 32) launch_items_bm<false, 32>(args, items, nitems, states, s);
        else if (bm == 64) launch_items_bm<false, 64>(args, items, nitems, states, s);
        else launch_items_bm<false, 96>(args, items, nitems, states, s);
    }
}

// items of flows whose block height is bm, cut into 8 per-XCD queues
void launch_contract_persistent(const FusedContractArgs *args, const int2 *items, const int *qstart,
                                const int *qcount, int *counters, const double *const *states, int grid,
                                int bm, bool split, hipStream_t s) {
    if (split) {
        if (bm == 32) launch_persistent_bm<true, 32>(args, items, qstart, qcount, counters, states, grid, s);
        else if (bm == 64) launch_persistent_bm<true, 64>(args, items, qstart, qcount, counters, states, grid, s);
        else launch_persistent_bm<true, 96>(args, items, qstart, qcount, counters, states, grid, s);
    } else {
        if (bm == 32) launch_persistent_bm<false, 32>(args, items, qstart, qcount, counters, states, grid, s);
        else if (bm == 64) launch_persistent_bm<false, 64>(args, items, qstart, qcount, counters, states, grid, s);
        else launch_persistent_bm<false, 96>(args, items, qstart, qcount, counters, states, grid, s);
    }
}

void launch_contract_fused(const FusedContractArgs &a, bool split, hipStream_t s) {
    const int bm = a.bm > 0 ? a.bm : contract_block_rows(a.N);
    if (bm == 32) launch_bm<32>(a, split, s);
    else if (bm == 64) launch_bm<64>(a, split, s);
    else launch_bm<96>(a, split, s);
}

}  // namespace frg
