// Bubble sweep: for every transfer row and every patch a, the temperature
// derivative of the one-loop bubble binned by the patch b of the second line,
//   B_row(a, b) = sum_{p in a, bin(row,p) = b} w_p dL/dT(xi_p, eps(second line); T)
// (Sec. 4: the three one-loop diagrams integrated over the Brillouin zone;
// here each transfer's bubble row is shared by every vertex entry that uses it).
//
// Work decomposition: one block per (patch a, chunk of rows); the patch's fine
// points are staged once in LDS (lane-major so lane L's P points sit at
// slot j*64 + L), and each wave sweeps whole rows: lane L evaluates the P
// consecutive points L*P .. L*P+P-1 (radially adjacent, so mostly one bin),
// accumulates runs of equal bin in registers and flushes each run into the
// wave's private LDS bins with one LDS add; the wave then writes the row
// B_row(a, 0..N-1) with coalesced stores.  The bin table (one byte per
// evaluation) and the cos/sin of points and transfers are temperature
// independent; eps(second line) uses cos(q -/+ p) = cos q cos p +/- sin q sin p.
//
// FP64 path: everything in double.  Split path: eps in double (its absolute
// error is divided by 2T), the integrand in FP32 with hardware exp/rcp, runs
// summed with Kahan compensation, bins accumulated in double, output float.
#include <cmath>

#include "frg_internal.h"

namespace frg {

namespace {

constexpr int kRowsPerBlock = 64;   // 16 rows per wave
constexpr int kThreads = 256;

// divided difference of h(x) = x sech^2 x, with the Taylor form near x = y
__device__ __forceinline__ double div_h64(double a, double ha, double b) {
    const double d = a - b;
    if (fabs(d) < 2e-3) {
        const double m = 0.5 * (a + b);
        const double e = exp(-2.0 * fabs(m));
        const double q = 1.0 + e;
        const double S = 4.0 * e / (q * q);
        const double tau = copysign((1.0 - e) / q, m);
        const double h1 = S * (1.0 - 2.0 * m * tau);
        const double h3 = 12.0 * S - 18.0 * S * S - 8.0 * m * S * tau * (1.0 - 3.0 * S);
        return h1 + d * d * h3 / 24.0;
    }
    const double e = exp(-2.0 * fabs(b));
    const double q = 1.0 + e;
    const double hb = b * (4.0 * e / (q * q));
    return (ha - hb) / d;
}

__device__ __forceinline__ float div_h32(float a, float ha, float b) {
    const float d = a - b;
    if (fabsf(d) < 0.1f) {
        const float m = 0.5f * (a + b);
        const float e = __expf(-2.0f * fabsf(m));
        const float q = 1.0f + e;
        const float S = 4.0f * e * __builtin_amdgcn_rcpf(q * q);
        const float tau = copysignf((1.0f - e) * __builtin_amdgcn_rcpf(q), m);
        const float h1 = S * (1.0f - 2.0f * m * tau);
        const float h3 = 12.0f * S - 18.0f * S * S - 8.0f * m * S * tau * (1.0f - 3.0f * S);
        return h1 + d * d * h3 * (1.0f / 24.0f);
    }
    const float e = __expf(-2.0f * fabsf(b));
    const float q = 1.0f + e;
    const float hb = b * (4.0f * e * __builtin_amdgcn_rcpf(q * q));
    return (ha - hb) * __builtin_amdgcn_rcpf(d);
}

template <int P, bool F32>
__device__ __forceinline__ void bubble_body(const BubbleArgs &A, int chunk, int a_patch, double *smem) {
    constexpr int S = P * 64;          // slots per array
    double *pt = smem;                 // [7][S]: cpx spx cpy spy a ha wf
    const int N = A.N, nf = A.nf, np = A.np;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *bins = smem + 7 * S + wave * N;

    for (int k = threadIdx.x; k < S; k += kThreads) {
        const int L = k / P, j = k % P;
        const int slot = j * 64 + L;
        if (k < nf) {
            const int i = a_patch * nf + k;
            pt[0 * S + slot] = A.trig_pt[i];
            pt[1 * S + slot] = A.trig_pt[np + i];
            pt[2 * S + slot] = A.trig_pt[2 * np + i];
            pt[3 * S + slot] = A.trig_pt[3 * np + i];
            if (F32) {
                pt[4 * S + slot] = A.pa32[i];
                pt[5 * S + slot] = A.pa32[np + i];
                pt[6 * S + slot] = A.pa32[2 * np + i];
            } else {
                pt[4 * S + slot] = A.pa64[i];
                pt[5 * S + slot] = A.pa64[np + i];
                pt[6 * S + slot] = A.pa64[2 * np + i];
            }
        } else {
            for (int q = 0; q < 7; ++q) pt[q * S + slot] = 0.0;
        }
    }
    const double inv2T = A.Tdev[1];
    const double mt2 = A.mt2, mt4p = A.mt4p, mu = A.mu;
    __syncthreads();

    const int row0 = chunk * kRowsPerBlock;
    for (int rr = wave; rr < kRowsPerBlock; rr += 4) {
        const int slot_out = row0 + rr;                 // output row position
        const bool active = slot_out < A.nrows;
        const int r = active ? (A.rowlist ? A.rowlist[slot_out] : slot_out) : 0;   // transfer row
        if (active)
            for (int b = lane; b < N; b += 64) bins[b] = 0.0;
        __syncthreads();
        if (active) {
            const bool pp = r < A.Tpp;
            const double cqx = A.trig_row[4 * r], sqx = A.trig_row[4 * r + 1];
            const double cqy = A.trig_row[4 * r + 2], sqy = A.trig_row[4 * r + 3];
            const uint8_t *brow = A.bins + static_cast<size_t>(r) * np + static_cast<size_t>(a_patch) * nf;
            int bcur = -1;
            double acc64 = 0.0;
            float acc32 = 0.0f, comp32 = 0.0f;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int k = lane * P + j;
                if (k < nf) {
                    const int slot = j * 64 + lane;
                    const double cpx = pt[slot], spx = pt[S + slot];
                    const double cpy = pt[2 * S + slot], spy = pt[3 * S + slot];
                    double cx, cy;
                    if (pp) {   // cos(q - p)
                        cx = cqx * cpx + sqx * spx;
                        cy = cqy * cpy + sqy * spy;
                    } else {    // cos(p + Q)
                        cx = cpx * cqx - spx * sqx;
                        cy = cpy * cqy - spy * sqy;
                    }
                    const double xi2 = mt2 * (cx + cy) - mt4p * (cx * cy) - mu;
                    double b2 = xi2 * inv2T;
                    if (pp) b2 = -b2;
                    const int bin = brow[k];
                    if (F32) {
                        const float v = static_cast<float>(pt[6 * S + slot]) *
                                        div_h32(static_cast<float>(pt[4 * S + slot]),
                                                static_cast<float>(pt[5 * S + slot]),
                                                static_cast<float>(b2));
                        if (bin != bcur) {
                            if (bcur >= 0)
                                atomicAdd(&bins[bcur], static_cast<double>(acc32) - static_cast<double>(comp32));
                            bcur = bin;
                            acc32 = v;
                            comp32 = 0.0f;
                        } else {   // Kahan step
                            const float y = v - comp32;
                            const float t = acc32 + y;
                            comp32 = (t - acc32) - y;
                            acc32 = t;
                        }
                    } else {
                        const double v = pt[6 * S + slot] * div_h64(pt[4 * S + slot], pt[5 * S + slot], b2);
                        if (bin != bcur) {
                            if (bcur >= 0) atomicAdd(&bins[bcur], acc64);
                            bcur = bin;
                            acc64 = v;
                        } else {
                            acc64 += v;
                        }
                    }
                }
            }
            if (bcur >= 0) {
                if (F32) atomicAdd(&bins[bcur], static_cast<double>(acc32) - static_cast<double>(comp32));
                else atomicAdd(&bins[bcur], acc64);
            }
        }
        __syncthreads();
        if (active) {
            const size_t NN = static_cast<size_t>(N) * N;
            const bool pp = slot_out < A.npp_out;
            const size_t base = (pp ? static_cast<size_t>(slot_out) : static_cast<size_t>(slot_out - A.npp_out)) * NN +
                                static_cast<size_t>(a_patch) * N;
            void *outp = pp ? A.Bpp : A.Bph;
            if (outp) {
                for (int b = lane; b < N; b += 64) {
                    if (F32) static_cast<float *>(outp)[base + b] = static_cast<float>(bins[b]);
                    else static_cast<double *>(outp)[base + b] = bins[b];
                }
            }
        }
        __syncthreads();
    }
}

template <int P, bool F32>
__global__ __launch_bounds__(kThreads) void bubble_kernel(BubbleArgs A) {
    extern __shared__ double smem[];
    bubble_body<P, F32>(A, blockIdx.x, blockIdx.y, smem);
}

// batched: item = (flow, chunk << 8 | patch); skips flows whose state says stop
template <int P, bool F32>
__global__ __launch_bounds__(kThreads) void bubble_kernel_batched(const BubbleArgs *__restrict__ args,
                                                                  const int2 *__restrict__ items,
                                                                  const double *const *__restrict__ states) {
    extern __shared__ double smem[];
    const int2 it = items[blockIdx.x];
    if (states && states[it.x][FRG_ST_REASON] != 0.0) return;
    const BubbleArgs A = args[it.x];
    bubble_body<P, F32>(A, it.y >> 8, it.y & 255, smem);
}

template <int P>
void launch_p(const BubbleArgs &a, bool fp32, hipStream_t s) {
    dim3 grid((a.nrows + kRowsPerBlock - 1) / kRowsPerBlock, a.N);
    const size_t lds = sizeof(double) * (7 * P * 64 + 4 * a.N);
    if (fp32)
        hipLaunchKernelGGL((bubble_kernel<P, true>), grid, dim3(kThreads), lds, s, a);
    else
        hipLaunchKernelGGL((bubble_kernel<P, false>), grid, dim3(kThreads), lds, s, a);
}

template <int P>
void launch_pb(const BubbleArgs *args, const int2 *items, int nitems, const double *const *states,
               int maxN, bool fp32, hipStream_t s) {
    const size_t lds = sizeof(double) * (7 * P * 64 + 4 * maxN);
    if (fp32)
        hipLaunchKernelGGL((bubble_kernel_batched<P, true>), dim3(nitems), dim3(kThreads), lds, s, args,
                           items, states);
    else
        hipLaunchKernelGGL((bubble_kernel_batched<P, false>), dim3(nitems), dim3(kThreads), lds, s, args,
                           items, states);
}

}  // namespace

int bubble_rows_per_block() { return kRowsPerBlock; }

void launch_bubbles_batched(const BubbleArgs *args, const int2 *items, int nitems,
                            const double *const *states, int nf, int maxN, bool fp32, hipStream_t s) {
    const int P = (nf + 63) / 64;
    if (P <= 1) launch_pb<1>(args, items, nitems, states, maxN, fp32, s);
    else if (P <= 2) launch_pb<2>(args, items, nitems, states, maxN, fp32, s);
    else if (P <= 4) launch_pb<4>(args, items, nitems, states, maxN, fp32, s);
    else if (P <= 8) launch_pb<8>(args, items, nitems, states, maxN, fp32, s);
    else launch_pb<16>(args, items, nitems, states, maxN, fp32, s);
}

void launch_bubbles(const BubbleArgs &a, bool fp32, hipStream_t s) {
    const int P = (a.nf + 63) / 64;
    if (P <= 1) launch_p<1>(a, fp32, s);
    else if (P <= 2) launch_p<2>(a, fp32, s);
    else if (P <= 4) launch_p<4>(a, fp32, s);
    else if (P <= 8) launch_p<8>(a, fp32, s);
    else launch_p<16>(a, fp32, s);
}

}  // namespace frg
