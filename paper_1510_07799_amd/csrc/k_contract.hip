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
//                              plus A = V(a,j2,b)           with g = V(j1,b,a)
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
#include "frg_internal.h"

namespace frg {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));
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

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

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

// ZK consecutive entries k = kb .. kb+ZK-1 of a column's bubble row
// (k = a'*N + b'), gathered through the row map; VW-wide vector loads when the
// source window is contiguous and aligned, scalar loads otherwise.
template <int ZK, int VW, typename T, typename VT>
__device__ __forceinline__ void load_bubble_window(const GLOBAL_AS T *brow, const RowMap &rm, int N, int K,
                                                   int kb, bool ok, T *out) {
    if (!ok) {
#pragma unroll
        for (int q = 0; q < ZK; ++q) out[q] = T(0);
        return;
    }
    const int a1 = kb / N, b1 = kb - a1 * N;
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
#pragma unroll
            for (int q = 0; q < ZK; ++q) out[q] = rm.refl ? tmp[ZK - 1 - q] : tmp[q];
            return;
        }
    }
#pragma unroll
    for (int q = 0; q < ZK; ++q) {
        const int k = kb + q;
        if (k < K) {
            const int aa = k / N, bb = k - aa * N;
            out[q] = brow[rm.map(aa, N) * N + rm.map(bb, N)];
        } else {
            out[q] = T(0);
        }
    }
}

// block -> (term, m tile, c tile, K part); heaviest channel (phd) first
__device__ __forceinline__ Work decode_block(const FusedContractArgs &P, int id) {
    const int per_term = P.mtiles * P.ctiles * P.KS;
    Work w;
    const int order[3] = {TERM_PHD, TERM_PHC, TERM_PP};
    const int t = id / per_term;
    w.term = order[t];
    id -= t * per_term;
    w.ks = id % P.KS;
    id /= P.KS;
    w.ctile = id % P.ctiles;
    w.mtile = id / P.ctiles;
    return w;
}

// The active k chunks of a block: entries [st_lo*G, st_hi*G) of its column
// tile's list, G chunks per step (K part ks of KS takes an equal share of the
// tile's steps).  Entries past the list read as -1 (a zero chunk).  Each
// thread reads only the entries of the list slots its loads serve, one step
// ahead of their use, as ordinary vector loads: a uniform (scalar) load would
// share its wait counter with the LDS traffic of the MFMA loop.
template <int G>
struct TileK {
    const GLOBAL_AS int32_t *kl;
    int nk, st_lo, st_hi;
    __device__ __forceinline__ TileK(const FusedContractArgs &P, int term, const Work &w) {
        const GLOBAL_AS int32_t *koff = gload_ptr(P.koff[term]);
        const int kbeg = koff[w.ctile];
        nk = koff[w.ctile + 1] - kbeg;
        kl = gload_ptr(P.klist[term]) + kbeg;
        const int nst = (nk + G - 1) / G;
        st_lo = static_cast<int>((static_cast<int64_t>(nst) * w.ks) / P.KS);
        st_hi = static_cast<int>((static_cast<int64_t>(nst) * (w.ks + 1)) / P.KS);
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
    const int NC = N * N;
    const int m0 = w.mtile * BM, c0 = w.ctile * BC;
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
                        Ap + (static_cast<int64_t>(ea[i]) * N + m) * kContractChunk + part * 2);
                else
                    ra[p][i] = d2_t{0.0, 0.0};
            }
        }
        const bool zok = cvalid && ez >= 0;
        const int kb = zok ? ez * kContractChunk + zoff : 0;
        load_bubble_window<ZK, 2, double, d2_t>(brow, rm, N, K, kb, zok, rb);
        int a = kb / N, b = kb - a * N;
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
            if (TERM == TERM_PHD) sZ[(BC + cl) * LDA + zk + q] = rb[q] * rg1[q];
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
    // output C[ks][tile position][m]: a block's tile is one contiguous range
    GLOBAL_AS double *Cout = gstore_ptr(P.C[TERM]) + static_cast<int64_t>(w.ks) * P.n3;
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
template <int TERM, int BM>
__device__ __forceinline__ void body_split(const FusedContractArgs &P, const Work &w, uint16_t *smem) {
    constexpr int BK = 32;
    constexpr int ZK = BK / 4;    // k per thread in the Z loader
    constexpr int LD = BK + 8;    // bf16 row pitch: rows stay 16-byte aligned
    constexpr int NP = TERM == TERM_PHD ? 2 : 1;
    constexpr int G = BK / kContractChunk;
    constexpr int NCH = G * BM;                         // 16-byte A pieces (one chunk of one row)
    constexpr int ACH = (NCH + kThreads - 1) / kThreads;
    uint16_t *sA = smem;                           // [NP][2][BM][LD]
    uint16_t *sZ = smem + NP * 2 * BM * LD;        // [NP][2][BC][LD]
    const int N = P.N;
    const int K = N * N;
    const int NC = N * N;
    const int64_t n3 = P.n3;
    const int m0 = w.mtile * BM, c0 = w.ctile * BC;
    const TileK<G> tk(P, TERM, w);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const GLOBAL_AS uint16_t *Ahl[2] = {gload_ptr(P.Ahl[TERM][0]), gload_ptr(P.Ahl[TERM][1])};
    const GLOBAL_AS float *B = gload_ptr(static_cast<const float *>(P.B[TERM]));
    const GLOBAL_AS int32_t *colrow = gload_ptr(P.colrow[TERM]);

    // A piece ch = tid + i * kThreads: row ch % BM of list slot ch / BM, so
    // consecutive lanes read consecutive rows of one chunk (chunk-major operand)
    static_assert(ZK == kContractChunk && G == 4, "split slots");
    // Z loader: column at tile position cl, list slot zslot (one chunk)
    const int zslot = tid & 3;
    const int cl = tid >> 2, zk = zslot * ZK;
    const bool cvalid = c0 + cl < NC;
    const int c = cvalid ? gload_ptr(P.cperm[TERM])[c0 + cl] : 0;
    const RowMap rm = decode_rowmap(cvalid ? colrow[c] : 0, N);
    const GLOBAL_AS float *brow = B + static_cast<int64_t>(rm.row) * K;
    const GLOBAL_AS float *g0 = gload_ptr(P.G32[TERM][0]) + static_cast<int64_t>(c) * N;
    const GLOBAL_AS float *g1 = TERM == TERM_PHD
                                    ? gload_ptr(P.G32[TERM][1]) + static_cast<int64_t>(c / N) * K
                                    : nullptr;

    u32x4_t ra[NP][2][ACH];
    float rb[ZK], rg0[ZK], rg1[ZK];

    // ea[i]: list entry of the slot of A piece i; e: of the Z window
    auto load = [&](const int (&ea)[ACH], int e) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl)
#pragma unroll
                for (int i = 0; i < ACH; ++i) {
                    const int ch = tid + i * kThreads;
                    const int m = m0 + ch % BM;
                    if (ch < NCH && ea[i] >= 0 && m < N)
                        ra[p][hl][i] = *reinterpret_cast<const GLOBAL_AS u32x4_t *>(
                            Ahl[p] + hl * n3 + (static_cast<int64_t>(ea[i]) * N + m) * kContractChunk);
                    else
                        ra[p][hl][i] = u32x4_t{0u, 0u, 0u, 0u};
                }
        const bool zok = cvalid && e >= 0;
        const int kb = zok ? e * kContractChunk : 0;
        load_bubble_window<ZK, 4, float, f4_t>(brow, rm, N, K, kb, zok, rb);
        int a = kb / N, b = kb - a * N;
        if (TERM != TERM_PP && zok && b + ZK <= N && (b & 3) == 0 && (N & 3) == 0) {
#pragma unroll
            for (int q = 0; q < ZK; q += 4) {
                const f4_t v = *reinterpret_cast<const GLOBAL_AS f4_t *>(g0 + b + q);
                rg0[q] = v[0]; rg0[q + 1] = v[1]; rg0[q + 2] = v[2]; rg0[q + 3] = v[3];
            }
        } else {
            int aa = a, bb = b;
#pragma unroll
            for (int q = 0; q < ZK; ++q) {
                const bool ok = zok && kb + q < K;
                rg0[q] = ok ? (TERM == TERM_PP ? g0[aa] : g0[bb]) : 0.f;
                if (++bb == N) { bb = 0; ++aa; }
            }
        }
        if (TERM == TERM_PHD) {
            if (zok && kb + ZK <= K) {
#pragma unroll
                for (int q = 0; q < ZK; q += 4) {
                    const f4_t v = *reinterpret_cast<const GLOBAL_AS f4_t *>(g1 + kb + q);
                    rg1[q] = v[0]; rg1[q + 1] = v[1]; rg1[q + 2] = v[2]; rg1[q + 3] = v[3];
                }
            } else {
#pragma unroll
                for (int q = 0; q < ZK; ++q) rg1[q] = (zok && kb + q < K) ? g1[kb + q] : 0.f;
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl)
#pragma unroll
                for (int i = 0; i < ACH; ++i) {
                    const int ch = tid + i * kThreads;
                    if (ch >= NCH) continue;
                    const int row = ch % BM, kq = (ch / BM) * kContractChunk;
                    *reinterpret_cast<u32x4_t *>(sA + ((p * 2 + hl) * BM + row) * LD + kq) = ra[p][hl][i];
                }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            u16x8_t hi, lo;
#pragma unroll
            for (int q = 0; q < ZK; ++q) {
                const float z = rb[q] * (p == 0 ? rg0[q] : rg1[q]);
                const uint16_t zh = bf16_rne(z);
                hi[q] = zh;
                lo[q] = bf16_rne(z - bf16_to_f(zh));
            }
            *reinterpret_cast<u16x8_t *>(sZ + ((p * 2 + 0) * BC + cl) * LD + zk) = hi;
            *reinterpret_cast<u16x8_t *>(sZ + ((p * 2 + 1) * BC + cl) * LD + zk) = lo;
        }
    };

    constexpr int RT = BM / 32;
    const int wm = wave & 1, wc = wave >> 1;
    f4_t acc[RT][2];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        acc[i][0] = f4_t{0.f, 0.f, 0.f, 0.f};
        acc[i][1] = f4_t{0.f, 0.f, 0.f, 0.f};
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
#pragma unroll
        for (int ks = 0; ks < BK / 32; ++ks) {
            const int kof = ks * 32 + (lane >> 4) * 8;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                bf8_t zh[2], zl[2];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) {
                    const int zr = wc * 32 + ci * 16 + (lane & 15);
                    zh[ci] = *reinterpret_cast<const bf8_t *>(sZ + ((p * 2 + 0) * BC + zr) * LD + kof);
                    zl[ci] = *reinterpret_cast<const bf8_t *>(sZ + ((p * 2 + 1) * BC + zr) * LD + kof);
                }
#pragma unroll
                for (int ri = 0; ri < RT; ++ri) {
                    const int ar = wm * (BM / 2) + ri * 16 + (lane & 15);
                    const bf8_t ah = *reinterpret_cast<const bf8_t *>(sA + ((p * 2 + 0) * BM + ar) * LD + kof);
                    const bf8_t al = *reinterpret_cast<const bf8_t *>(sA + ((p * 2 + 1) * BM + ar) * LD + kof);
#pragma unroll
                    for (int ci = 0; ci < 2; ++ci) {
                        acc[ri][ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, zh[ci], acc[ri][ci], 0, 0, 0);
                        acc[ri][ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, zl[ci], acc[ri][ci], 0, 0, 0);
                        acc[ri][ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, zh[ci], acc[ri][ci], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
    // bf16 16x16x32 accumulator layout: lane l, register r holds row 4(l>>4) + r, column l&15
    // output C[ks][tile position][m]: four consecutive m per lane, one 32-byte store
    // (N % 4 == 0, so a group of four rows is either wholly inside or outside)
    GLOBAL_AS double *Cout = gstore_ptr(P.C[TERM]) + static_cast<int64_t>(w.ks) * P.n3;
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) {
        const int pos = c0 + wc * 32 + ci * 16 + (lane & 15);
        if (pos >= NC) continue;
#pragma unroll
        for (int ri = 0; ri < RT; ++ri) {
            const int m = m0 + wm * (BM / 2) + ri * 16 + 4 * (lane >> 4);
            if (m < N) {
                const d4_t v{static_cast<double>(acc[ri][ci][0]), static_cast<double>(acc[ri][ci][1]),
                             static_cast<double>(acc[ri][ci][2]), static_cast<double>(acc[ri][ci][3])};
                *reinterpret_cast<GLOBAL_AS d4_t *>(Cout + static_cast<int64_t>(pos) * N + m) = v;
            }
        }
    }
}

template <int BM, bool SPLIT>
__device__ __forceinline__ void run_work(const FusedContractArgs &P, const Work &w, double *smem_d) {
    if (SPLIT) {
        uint16_t *smem = reinterpret_cast<uint16_t *>(smem_d);
        if (w.term == TERM_PHD) body_split<TERM_PHD, BM>(P, w, smem);
        else if (w.term == TERM_PHC) body_split<TERM_PHC, BM>(P, w, smem);
        else body_split<TERM_PP, BM>(P, w, smem);
    } else {
        if (w.term == TERM_PHD) body_f64<TERM_PHD, BM>(P, w, smem_d);
        else if (w.term == TERM_PHC) body_f64<TERM_PHC, BM>(P, w, smem_d);
        else body_f64<TERM_PP, BM>(P, w, smem_d);
    }
}

template <int BM>
__global__ __launch_bounds__(kThreads) void contract_f64_fused(FusedContractArgs P) {
    extern __shared__ double smem_d[];
    run_work<BM, false>(P, decode_block(P, blockIdx.x), smem_d);
}

template <int BM>
__global__ __launch_bounds__(kThreads) void contract_split_fused(FusedContractArgs P) {
    extern __shared__ double smem_d[];
    run_work<BM, true>(P, decode_block(P, blockIdx.x), smem_d);
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
            run_work<BM, SPLIT>(P, decode_block(P, it.y), smem_d);
            __syncthreads();
        }
    }
}

// One block per work item of the list, dealt by the hardware dispatcher in
// list order (the alternative to the persistent queues).
template <bool SPLIT, int BM>
__global__ __launch_bounds__(kThreads) void contract_items(const FusedContractArgs *__restrict__ args,
                                                           const int2 *__restrict__ items,
                                                           const double *const *__restrict__ states) {
    extern __shared__ double smem_d[];
    const int2 it = items[blockIdx.x];
    if (states && states[it.x][FRG_ST_REASON] != 0.0) return;
    const FusedContractArgs P = args[it.x];
    run_work<BM, SPLIT>(P, decode_block(P, it.y), smem_d);
}

__global__ void reset_counters(int *counters, int n) {
    if (static_cast<int>(threadIdx.x) < n) counters[threadIdx.x] = 0;
}

template <int BM>
void launch_bm(FusedContractArgs a, bool split, hipStream_t s) {
    a.mtiles = (a.N + BM - 1) / BM;
    a.ctiles = (a.N * a.N + BC - 1) / BC;
    const int blocks = 3 * a.mtiles * a.ctiles * a.KS;
    if (split) {
        const size_t lds = sizeof(uint16_t) * (2 * 2 * BM * (32 + 8) + 2 * 2 * BC * (32 + 8));
        hipLaunchKernelGGL(contract_split_fused<BM>, dim3(blocks), dim3(kThreads), lds, s, a);
    } else {
        const size_t lds = sizeof(double) * (2 * BM * 17 + 2 * BC * 17);
        hipLaunchKernelGGL(contract_f64_fused<BM>, dim3(blocks), dim3(kThreads), lds, s, a);
    }
}

// flags of the k chunks of one column tile (block = tile)
__global__ __launch_bounds__(256) void tile_pattern_kernel(const uint8_t *__restrict__ bins,
                                                           const int32_t *__restrict__ colfull,
                                                           const int32_t *__restrict__ cperm, int N,
                                                           int nf, int np, uint8_t *__restrict__ flags) {
    extern __shared__ uint8_t sflag[];
    const int NC = N * N, nch = NC / kContractChunk;
    for (int j = threadIdx.x; j < nch; j += blockDim.x) sflag[j] = 0;
    __syncthreads();
    const int p0 = blockIdx.x * BC;
    for (int cl = 0; cl < BC && p0 + cl < NC; ++cl) {
        const uint8_t *row = bins + static_cast<int64_t>(colfull[cperm[p0 + cl]]) * np;
        for (int p = threadIdx.x; p < np; p += blockDim.x) {
            const int k = (p / nf) * N + row[p];
            sflag[k / kContractChunk] = 1;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nch; j += blockDim.x) flags[static_cast<int64_t>(blockIdx.x) * nch + j] = sflag[j];
}

}  // namespace


int contract_block_rows(int N) { return block_rows_of(N); }

void launch_tile_pattern(const uint8_t *bins, const int32_t *colfull, const int32_t *cperm, int N, int nf,
                         int np, uint8_t *flags, hipStream_t s) {
    const int tiles = (N * N + BC - 1) / BC;
    const size_t lds = static_cast<size_t>(N) * N / kContractChunk;
    hipLaunchKernelGGL(tile_pattern_kernel, dim3(tiles), dim3(256), lds, s, bins, colfull, cperm, N, nf, np,
                       flags);
}

size_t contract_lds_bytes(bool split) {
    return split ? sizeof(uint16_t) * (2 * 2 * 96 * (32 + 8) + 2 * 2 * BC * (32 + 8))
                 : sizeof(double) * (2 * 96 * 17 + 2 * BC * 17);
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
    const int bm = contract_block_rows(a.N);
    if (bm == 32) launch_bm<32>(a, split, s);
    else if (bm == 64) launch_bm<64>(a, split, s);
    else launch_bm<96>(a, split, s);
}

}  // namespace frg
