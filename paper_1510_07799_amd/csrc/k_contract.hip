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
// The A tile is staged through LDS; the B-side tile Z = B_row(c)[k] g(c,k) is
// formed in registers from one bubble row per column and written to LDS in
// the matrix-core operand layout.  FP64: v_mfma_f64_16x16x4f64.  Split path:
// A and Z as bf16 hi + lo, three v_mfma_f32_16x16x32_bf16 per k-step
// (hi*hi + hi*lo + lo*hi), FP32 accumulation, result widened to FP64.
#include "frg_internal.h"

namespace frg {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4_t __attribute__((ext_vector_type(4)));

constexpr int BM = 32;   // output rows (m) per block
constexpr int BC = 64;   // output columns (c) per block
constexpr int kThreads = 256;

// output index of C[m, c] in the F layout of the term
template <int TERM>
__device__ __forceinline__ int64_t out_index(int N, int m, int c) {
    const int64_t K = static_cast<int64_t>(N) * N;
    if (TERM == TERM_PP) return static_cast<int64_t>(c) * N + m;          // F[j1][j2][j3=m]
    if (TERM == TERM_PHC) return static_cast<int64_t>(m) * K + c;         // F[j1=m][j2][j3], c=j2*N+j3
    return static_cast<int64_t>(c / N) * K + static_cast<int64_t>(m) * N + (c % N);  // F[j1][j2=m][j3]
}

// ------------------------------------------------------------------ FP64
template <int TERM>
__global__ __launch_bounds__(kThreads) void contract_f64_kernel(ContractArgs P) {
    constexpr int BK = 16;
    constexpr int NP = TERM == TERM_PHD ? 2 : 1;
    __shared__ double sA[NP][BM][BK + 1];
    __shared__ double sZ[NP][BC][BK + 1];
    const int N = P.N;
    const int K = N * N;
    const int NC = N * N;
    const int m0 = blockIdx.y * BM, c0 = blockIdx.x * BC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double *B = static_cast<const double *>(P.B);

    // A loader: row ml, two consecutive k
    const int ml = tid >> 3, ak = (tid & 7) * 2;
    const bool mvalid = (m0 + ml) < N;
    // Z loader: column cl, four consecutive k
    const int cl = tid >> 2, zk = (tid & 3) * 4;
    const int c = c0 + cl;
    const bool cvalid = c < NC;
    const double *brow = B + static_cast<int64_t>(cvalid ? P.colrow[c] : 0) * K;
    const double *g0 = P.G64[0] + static_cast<int64_t>(cvalid ? c : 0) * N;
    const double *g1 = TERM == TERM_PHD ? P.G64[1] + static_cast<int64_t>(cvalid ? c / N : 0) * K
                                        : nullptr;

    const int mb = wave & 1, cb0 = (wave >> 1) * 2;
    d4_t acc[2];
    acc[0] = d4_t{0.0, 0.0, 0.0, 0.0};
    acc[1] = d4_t{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const double *Ap = P.A64[p] + static_cast<int64_t>(m0 + ml) * K;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int k = k0 + ak + q;
                sA[p][ml][ak + q] = (mvalid && k < K) ? Ap[k] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + zk + q;
            const bool ok = cvalid && k < K;
            const int a = k / N, b = k - a * N;
            const double bv = ok ? brow[k] : 0.0;
            if (TERM == TERM_PP) {
                sZ[0][cl][zk + q] = ok ? bv * g0[a] : 0.0;
            } else if (TERM == TERM_PHC) {
                sZ[0][cl][zk + q] = ok ? bv * g0[b] : 0.0;
            } else {
                sZ[0][cl][zk + q] = ok ? bv * g0[b] : 0.0;
                sZ[NP - 1][cl][zk + q] = ok ? bv * g1[k] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const double af = sA[p][mb * 16 + (lane & 15)][kk * 4 + (lane >> 4)];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) {
                    const double bf = sZ[p][(cb0 + ci) * 16 + (lane & 15)][kk * 4 + (lane >> 4)];
                    acc[ci] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, acc[ci], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // f64 16x16x4 accumulator layout: lane l, register r holds row (l>>4) + 4r, column l&15
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) {
        const int cc = c0 + (cb0 + ci) * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = m0 + mb * 16 + (lane >> 4) + 4 * r;
            if (m < N && cc < NC) P.C[out_index<TERM>(N, m, cc)] = acc[ci][r];
        }
    }
}

// ------------------------------------------------------------------ split BF16
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

template <int TERM>
__global__ __launch_bounds__(kThreads) void contract_split_kernel(ContractArgs P) {
    constexpr int BK = 32;
    constexpr int LD = BK + 8;   // bf16 row pitch (16-byte aligned rows)
    constexpr int NP = TERM == TERM_PHD ? 2 : 1;
    __shared__ __attribute__((aligned(16))) uint16_t sA[NP][2][BM][LD];
    __shared__ __attribute__((aligned(16))) uint16_t sZ[NP][2][BC][LD];
    const int N = P.N;
    const int K = N * N;
    const int NC = N * N;
    const int64_t n3 = static_cast<int64_t>(N) * K;
    const int m0 = blockIdx.y * BM, c0 = blockIdx.x * BC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float *B = static_cast<const float *>(P.B);

    const int ml = tid >> 3, ak = (tid & 7) * 4;       // A loader: 4 k per thread
    const bool mvalid = (m0 + ml) < N;
    const int cl = tid >> 2, zk = (tid & 3) * 8;       // Z loader: 8 k per thread
    const int c = c0 + cl;
    const bool cvalid = c < NC;
    const float *brow = B + static_cast<int64_t>(cvalid ? P.colrow[c] : 0) * K;
    const float *g0 = P.G32[0] + static_cast<int64_t>(cvalid ? c : 0) * N;
    const float *g1 = TERM == TERM_PHD ? P.G32[1] + static_cast<int64_t>(cvalid ? c / N : 0) * K
                                       : nullptr;

    const int mb = wave & 1, cb0 = (wave >> 1) * 2;
    f4_t acc[2];
    acc[0] = f4_t{0.f, 0.f, 0.f, 0.f};
    acc[1] = f4_t{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int hl = 0; hl < 2; ++hl) {
                const uint16_t *Ap = P.Ahl[p] + hl * n3 + static_cast<int64_t>(m0 + ml) * K;
                u16x4_t v;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = k0 + ak + q;
                    v[q] = (mvalid && k < K) ? Ap[k] : static_cast<uint16_t>(0);
                }
                *reinterpret_cast<u16x4_t *>(&sA[p][hl][ml][ak]) = v;
            }
        }
        u16x8_t zh[NP], zl[NP];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = k0 + zk + q;
            const bool ok = cvalid && k < K;
            const int a = k / N, b = k - a * N;
            const float bv = ok ? brow[k] : 0.f;
            float z[NP];
            if (TERM == TERM_PP) {
                z[0] = ok ? bv * g0[a] : 0.f;
            } else if (TERM == TERM_PHC) {
                z[0] = ok ? bv * g0[b] : 0.f;
            } else {
                z[0] = ok ? bv * g0[b] : 0.f;
                z[NP - 1] = ok ? bv * g1[k] : 0.f;
            }
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const uint16_t hi = bf16_rne(z[p]);
                zh[p][q] = hi;
                zl[p][q] = bf16_rne(z[p] - bf16_to_f(hi));
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            *reinterpret_cast<u16x8_t *>(&sZ[p][0][cl][zk]) = zh[p];
            *reinterpret_cast<u16x8_t *>(&sZ[p][1][cl][zk]) = zl[p];
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int arow = mb * 16 + (lane & 15), kof = (lane >> 4) * 8;
            const bf8_t ahi = *reinterpret_cast<const bf8_t *>(&sA[p][0][arow][kof]);
            const bf8_t alo = *reinterpret_cast<const bf8_t *>(&sA[p][1][arow][kof]);
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
                const int zrow = (cb0 + ci) * 16 + (lane & 15);
                const bf8_t zhi = *reinterpret_cast<const bf8_t *>(&sZ[p][0][zrow][kof]);
                const bf8_t zlo = *reinterpret_cast<const bf8_t *>(&sZ[p][1][zrow][kof]);
                acc[ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, zhi, acc[ci], 0, 0, 0);
                acc[ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, zlo, acc[ci], 0, 0, 0);
                acc[ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, zhi, acc[ci], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // bf16 16x16x32 accumulator layout: lane l, register r holds row 4(l>>4) + r, column l&15
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) {
        const int cc = c0 + (cb0 + ci) * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = m0 + mb * 16 + 4 * (lane >> 4) + r;
            if (m < N && cc < NC) P.C[out_index<TERM>(N, m, cc)] = static_cast<double>(acc[ci][r]);
        }
    }
}

template <int TERM>
void launch_term(const ContractArgs &a, bool split, hipStream_t s) {
    const int NC = a.N * a.N;
    dim3 grid((NC + BC - 1) / BC, (a.N + BM - 1) / BM);
    if (split)
        hipLaunchKernelGGL(contract_split_kernel<TERM>, grid, dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(contract_f64_kernel<TERM>, grid, dim3(kThreads), 0, s, a);
}

}  // namespace

void launch_contract(const ContractArgs &a, bool split, hipStream_t s) {
    if (a.term == TERM_PP) launch_term<TERM_PP>(a, split, s);
    else if (a.term == TERM_PHC) launch_term<TERM_PHC>(a, split, s);
    else launch_term<TERM_PHD>(a, split, s);
}

}  // namespace frg
