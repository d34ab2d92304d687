// Bubble sweep: for every transfer row and every patch a, the temperature
// derivative of the one-loop bubble binned by the patch b of the second line,
//   B_row(a, b) = sum_{p in a, bin(row,p) = b} w_p dL/dT(xi_p, eps(second line); T)
// (Sec. 4: the three one-loop diagrams integrated over the Brillouin zone;
// here each transfer's bubble row is shared by every vertex entry that uses it).
//
// Work decomposition: one block per (patch a, chunk of rows); lane L holds the
// P fine points at table positions L*P .. L*P+P-1 of the patch (angular
// neighbours at one radius, so mostly one bin) in registers for all rows, and
// each wave sweeps whole rows independently (in the FP64 path the points sit in
// LDS instead, to keep the register count down): it accumulates runs of equal
// bin in registers, flushes each run into the wave's private LDS bins with one
// LDS add, and writes the row B_row(a, 0..N-1) with coalesced stores (no
// block-wide barrier after the set-up).  The bin table (one byte per evaluation) and the cos/sin
// of points and transfers are temperature independent; eps(second line) uses
// cos(q -/+ p) = cos q cos p +/- sin q sin p.
//
// FP64 path: everything in double.  Split path: eps in double (its absolute
// error is divided by 2T), the integrand in FP32 with hardware exp2/rcp, runs
// of at most P points summed in FP32, bins accumulated in double, output float.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "frg_internal.h"

namespace frg {

namespace {

constexpr int kRowsPerBlock = 64;          // 16 rows per wave (default; a tuning may set 4..256)
// Batches have blocks to spare: blocks of about 160 rows (at most 40 per wave)
// cut the per-block point set-up, in chunks evened out over a flow's rows.
constexpr int kRowsPerBlockBatched = 160;
constexpr int kThreads = 256;

// Weighted divided difference w (h(a) - h(b)) / (a - b) of h(x) = x sech^2 x,
// given c1 = w h(a) and c2 = -4 w.  With e = exp(-2|x|), sech^2 x = 4e / (1+e)^2
// and tanh x = sign(x) (1 - e) / (1 + e).  Away from the diagonal (wdiv_*_far)
// the difference is taken over one common denominator,
//   w (h(a) - h(b)) / d = (c1 (1+e)^2 + c2 b e) / ((1+e)^2 d),   e = exp(-2|b|),
// so one division (one reciprocal in FP32) serves it.  Near it (small d = a - b)
// the FP64 path (wdiv_*64_near) takes the Taylor form h1(m) + d^2 h3(m) / 24
// around m = (a + b) / 2 (h1, h3: first and third derivatives of h), scaled by
// w = -c2 / 4; the FP32 path expands around a (below).
// The far form has no branch, so a lane's points are evaluated side by side and
// the few near ones are redone afterwards.
__device__ __forceinline__ double wdiv_h64_far(double c1, double c2, double b, double d) {
    const double e = exp(-2.0 * fabs(b));
    const double q = 1.0 + e;
    const double q2 = q * q;
    return fma(c2, b * e, c1 * q2) / (q2 * d);
}
__device__ __forceinline__ double wdiv_h64_near(double a, double c2, double b) {
    const double d = a - b;
    const double m = 0.5 * (a + b);
    const double e = exp(-2.0 * fabs(m));
    const double r = 1.0 / (1.0 + e);
    const double S = 4.0 * e * r * r;
    const double tau = copysign((1.0 - e) * r, m);
    const double h1 = S * (1.0 - 2.0 * m * tau);
    const double h3 = S * (12.0 - 18.0 * S - 8.0 * m * tau * (1.0 - 3.0 * S));
    return (-0.25 * c2) * (h1 + d * d * h3 / 24.0);
}
constexpr double kTaylor64 = 2e-3;

// FP32 forms with hardware exp2 and reciprocal.  Near the diagonal (|d| < 0.02)
// the split path expands around the point's own a instead of the midpoint,
//   w (h(a) - h(b)) / d = C0 + C1 d + C2 d^2 + C3 d^3,
//   C0 = w h1(a), C1 = -w h2(a) / 2, C2 = w h3(a) / 6, C3 = -w h4(a) / 24
// (hk: k-th derivative of h), whose coefficients depend on the point alone and
// are made once per block (taylor_consts); the branch is then three FMAs.  The
// truncation (the d^4 term, h5 / 120) stays below about 1e-7 of w there, and the
// far form beyond it loses at most about 2e-7 / |d| < 1e-5 (relative to w) to
// the rounding of h(a) and of the exponential.
constexpr float kTaylor32 = 0.02f;
constexpr float kM2Log2e = -2.8853900817779268f;   // -2 / ln 2: exp(-2x) = exp2(kM2Log2e x)
__device__ __forceinline__ float wdiv_h32_far(float c1, float c2, float b, float d) {
    const float e = __builtin_amdgcn_exp2f(kM2Log2e * fabsf(b));
    const float q = 1.0f + e;
    const float q2 = q * q;
    return fmaf(c2, b * e, c1 * q2) * __builtin_amdgcn_rcpf(q2 * d);
}
__device__ __forceinline__ float taylor_poly(const float4 &C, float d) {
    return fmaf(d, fmaf(d, fmaf(d, C.w, C.z), C.y), C.x);
}
// The coefficients C0..C3 above at x (in FP64), for h (FULL false, weight w) or
// for tanh (FULL true, weight W; its derivatives are S, -2 S tau, 4 S - 6 S^2
// and -8 S tau (1 - 3 S)), with S = sech^2 x and tau = tanh x.
template <bool FULL>
__device__ __forceinline__ float4 taylor_consts(double x, double w) {
    const double e = exp(-2.0 * fabs(x));
    const double r = 1.0 / (1.0 + e);
    const double S = 4.0 * e * r * r;
    const double tau = copysign((1.0 - e) * r, x);
    double k1, k2, k3, k4;
    if constexpr (FULL) {
        k1 = S;
        k2 = -2.0 * S * tau;
        k3 = S * (4.0 - 6.0 * S);
        k4 = -8.0 * S * tau * (1.0 - 3.0 * S);
    } else {
        k1 = S * (1.0 - 2.0 * x * tau);
        k2 = -2.0 * S * (2.0 * tau - 2.0 * x + 3.0 * x * S);
        k3 = S * (12.0 - 18.0 * S - 8.0 * x * tau * (1.0 - 3.0 * S));
        k4 = 8.0 * S * (tau * (12.0 * S - 4.0) + x * (2.0 - 15.0 * S + 15.0 * S * S));
    }
    return make_float4(static_cast<float>(w * k1), static_cast<float>(-w * k2 / 2.0),
                       static_cast<float>(w * k3 / 6.0), static_cast<float>(-w * k4 / 24.0));
}

// The full bubble (not its T-derivative) has the weighted divided difference
// W (tanh a - tanh b) / (a - b) with W = w_p / 4T, given c1 = W tanh(a) and
// c2 = W: far from the diagonal over one common denominator,
//   (c1 (1+e) - c2 sign(b) (1-e)) / ((1+e) d),   e = exp(-2|b|),
// near it the Taylor form S(m) + d^2 (4S - 6S^2)(m) / 24 with S = sech^2 (the
// first and third derivatives of tanh).
__device__ __forceinline__ double wdiv_t64_far(double c1, double c2, double b, double d) {
    const double e = exp(-2.0 * fabs(b));
    const double q = 1.0 + e;
    return (c1 * q - c2 * copysign(1.0 - e, b)) / (q * d);
}
__device__ __forceinline__ double wdiv_t64_near(double a, double c2, double b) {
    const double d = a - b;
    const double m = 0.5 * (a + b);
    const double e = exp(-2.0 * fabs(m));
    const double r = 1.0 / (1.0 + e);
    const double S = 4.0 * e * r * r;
    return c2 * (S + d * d * (4.0 * S - 6.0 * S * S) / 24.0);
}
__device__ __forceinline__ float wdiv_t32_far(float c1, float c2, float b, float d) {
    const float e = __builtin_amdgcn_exp2f(kM2Log2e * fabsf(b));
    const float q = 1.0f + e;
    return (c1 * q - c2 * copysignf(1.0f - e, b)) * __builtin_amdgcn_rcpf(q * d);
}

// Both rows of a pair (reading below): the second lines of the pp row q and of
// the ph row -q have one energy, so b_ph = -b_pp exactly, and the two weighted
// divided differences share exp(-2|b|) and the numerator's terms.  In FP32 each
// value is bitwise the one the single-row form gives, and the near forms of a
// pair fetch the point's coefficients once (coef()).  The FP64 temperature
// derivative pair takes both quotients from one division, 1 / (t0 t1) with
// t = (1+e)^2 d (a few ulp instead of a correctly rounded quotient each; an
// FP64 division is a dozen instructions).
template <class G>
__device__ __forceinline__ void near32_pair(const G &coef, float d0, float d1, float &v0, float &v1) {
    const bool n0 = fabsf(d0) < kTaylor32, n1 = fabsf(d1) < kTaylor32;
    if (n0 || n1) {
        const float4 C = coef();
        if (n0) v0 = taylor_poly(C, d0);
        if (n1) v1 = taylor_poly(C, d1);
    }
}
template <class G>
__device__ __forceinline__ void wdiv_h32_pair(float a, float c1, float c2, float b, const G &coef,
                                              float &v0, float &v1) {
    const float e = __builtin_amdgcn_exp2f(kM2Log2e * fabsf(b));
    const float q = 1.0f + e;
    const float q2 = q * q;
    const float A = c1 * q2, be = b * e;
    const float d0 = a - b, d1 = a + b;
    v0 = fmaf(c2, be, A) * __builtin_amdgcn_rcpf(q2 * d0);
    v1 = fmaf(c2, -be, A) * __builtin_amdgcn_rcpf(q2 * d1);
    near32_pair(coef, d0, d1, v0, v1);
}
template <class G>
__device__ __forceinline__ void wdiv_t32_pair(float a, float c1, float c2, float b, const G &coef,
                                              float &v0, float &v1) {
    const float e = __builtin_amdgcn_exp2f(kM2Log2e * fabsf(b));
    const float q = 1.0f + e;
    const float A = c1 * q, t = c2 * copysignf(1.0f - e, b);
    const float d0 = a - b, d1 = a + b;
    v0 = (A - t) * __builtin_amdgcn_rcpf(q * d0);
    v1 = (A + t) * __builtin_amdgcn_rcpf(q * d1);
    near32_pair(coef, d0, d1, v0, v1);
}
__device__ __forceinline__ void wdiv_h64_pair(double a, double c1, double c2, double b, double &v0, double &v1) {
    const double e = exp(-2.0 * fabs(b));
    const double q = 1.0 + e;
    const double q2 = q * q;
    const double A = c1 * q2, be = b * e;
    const double d0 = a - b, d1 = a + b;
    const bool n0 = fabs(d0) < kTaylor64, n1 = fabs(d1) < kTaylor64;
    // a near term's denominator is replaced by 1 (its value comes from the
    // Taylor form), so a zero d cannot reach the other term
    const double t0 = q2 * (n0 ? 1.0 : d0), t1 = q2 * (n1 ? 1.0 : d1);
    const double inv = 1.0 / (t0 * t1);
    v0 = fma(c2, be, A) * (t1 * inv);
    v1 = fma(c2, -be, A) * (t0 * inv);
    if (n0) v0 = wdiv_h64_near(a, c2, b);
    if (n1) v1 = wdiv_h64_near(a, c2, -b);
}
__device__ __forceinline__ void wdiv_t64_pair(double a, double c1, double c2, double b, double &v0, double &v1) {
    const double e = exp(-2.0 * fabs(b));
    const double q = 1.0 + e;
    const double A = c1 * q, t = c2 * copysign(1.0 - e, b);
    const double d0 = a - b, d1 = a + b;
    v0 = (A - t) / (q * d0);
    v1 = (A + t) / (q * d1);
    if (fabs(d0) < kTaylor64) v0 = wdiv_t64_near(a, c2, b);
    if (fabs(d1) < kTaylor64) v1 = wdiv_t64_near(a, c2, -b);
}

__device__ __forceinline__ double tanh_d(double x) {
    const double e = exp(-2.0 * fabs(x));
    return copysign((1.0 - e) / (1.0 + e), x);
}

// a wave-uniform double held in scalar registers
__device__ __forceinline__ double uniform_f64(double x) {
    const uint64_t u = __double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// order the LDS accesses of one wave (its bins are private to it); the fences
// cover LDS only, so they need no wait for the wave's global loads and stores
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Pointers read from the argument block are generic to the compiler, which then
// emits FLAT accesses: those count against the LDS wait counter as well, so
// every LDS wait of a row would also wait for the loads in flight.  Every
// operand here is in global memory (address space 1); the transfer-row
// constants are wave-uniform and read through the scalar cache (address
// space 4).
#define GLOBAL_AS __attribute__((address_space(1)))
#define CONST_AS __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const GLOBAL_AS T *gld(const T *p) {
    return reinterpret_cast<const GLOBAL_AS T *>(reinterpret_cast<uintptr_t>(p));
}
template <class T>
__device__ __forceinline__ GLOBAL_AS T *gst(T *p) {
    return reinterpret_cast<GLOBAL_AS T *>(reinterpret_cast<uintptr_t>(p));
}
template <class T>
__device__ __forceinline__ const CONST_AS T *cld(const T *p) {
    return reinterpret_cast<const CONST_AS T *>(reinterpret_cast<uintptr_t>(p));
}

// Bins of wave w at smem[w*N ..) (a pair's two rows interleaved at
// smem[2*w*N ..)); in LDS mode the point data follow them.
template <int P, bool F32>
constexpr bool points_in_registers() { return F32 && P <= 8; }

// With the points in registers, the points' Taylor coefficients (one float4 per
// point, lane-major) follow the bins instead.
template <int P, bool F32>
size_t bubble_lds_bytes(int N, bool paired) {
    return sizeof(double) * ((paired ? 8 : 4) * static_cast<size_t>(N)) +
           (points_in_registers<P, F32>() ? sizeof(float4) * P * 64 : sizeof(double) * 7 * P * 64);
}

// FULL: the full bubble L instead of dL/dT (the interaction flow).  PAIRED: each
// output position evaluates a pp row q and the ph row of -q at once (rowlist,
// rowlist_ph): their second lines q - p and p - q have one energy.
// PF: the next row's table bytes are loaded while a row is evaluated (the
// batched kernel and the paired single-flow kernel, which then stay within 128
// registers; the unpaired single-flow kernel spills with it)
// SE: a self-energy per patch (A.sigma) shifts the second line's energy by
// its bin's value (dL/dT only); the table S/2T sits in LDS after the point
// data.  A pair takes the pp row's bin: the ph row's bin is the pp bin + N/2,
// whose self-energy is the same when S is C4v invariant (the host pairs rows
// only then), so the ph energy stays the negative of the pp one.
template <int P, bool F32, bool FULL, bool PAIRED, bool PF, bool SE = false>
__device__ __forceinline__ void bubble_body(const BubbleArgs &A, int chunk, int a_patch, double *smem, int rpb) {
    static_assert(!SE || !FULL, "self-energy rows are dL/dT rows");
    using PT = typename std::conditional<F32, float, double>::type;
    // The lane's P points (table positions lane*P .. lane*P+P-1, angular
    // neighbours at one radius): in registers for every row (split path with up
    // to 8 points per lane), or, where that would cost too many registers (the
    // FP64 path), staged once in LDS lane-major (lane L's point j at slot j*64 + L).
    constexpr bool REG = points_in_registers<P, F32>();
    constexpr int PR = REG ? P : 1;
    constexpr int S = P * 64;
    const int N = A.N, nf = A.nf, np = A.np;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // a pair's two rows interleaved (pp at 2b, ph at 2b + 1): one address per run
    constexpr int BS = PAIRED ? 2 : 1;
    double *bins = smem + wave * N * BS;
    // a pair's ph row, indexed by the pp row's bin: the ph second line p - q is
    // the inverse of the pp one q - p, so its patch is the pp bin + N/2 (checked
    // on the table at context creation); the output pass undoes the shift
    double *bins2 = bins + 1;
    double *pt = smem + (PAIRED ? 8 : 4) * N;  // LDS mode: [7][S] cpx spx cpy spy a c1 c2
    float4 *tay = reinterpret_cast<float4 *>(pt);  // register mode: [S] Taylor coefficients
    double *sgl = pt + (REG ? 2 * S : 7 * S);      // SE: S_b / 2T of every patch b
    if constexpr (SE)
        for (int b = threadIdx.x; b < N; b += kThreads) sgl[b] = A.sigma[b] * A.Tdev[1];

    // per point: cos/sin of px, py; a = xi / 2T; c1 = w h(a), c2 = -4 w with
    // w = -w_p / 4T^2 (the weighted divided difference takes these); for the
    // full bubble c1 = W tanh(a), c2 = W with W = w_p / 4T = -w T
    const double Tcur = A.Tdev[0];
    const GLOBAL_AS float *pa32 = gld(A.pa32);
    const GLOBAL_AS double *pa64 = gld(A.pa64), *trig_pt = gld(A.trig_pt);
    auto point_consts = [&](bool ok, int i, PT &a, PT &c1, PT &c2) {
        const double wf = ok ? (F32 ? static_cast<double>(pa32[2 * np + i]) : pa64[2 * np + i]) : 0.0;
        const double av = ok ? (F32 ? static_cast<double>(pa32[i]) : pa64[i]) : 0.0;
        a = static_cast<PT>(av);
        if constexpr (FULL) {
            const double W = -wf * Tcur;
            c1 = static_cast<PT>(W * tanh_d(av));
            c2 = static_cast<PT>(W);
        } else {
            const PT w = static_cast<PT>(wf);
            c1 = w * (ok ? static_cast<PT>(F32 ? pa32[np + i] : pa64[np + i]) : PT(0));
            c2 = PT(-4) * w;
        }
    };
    double cpx[PR], spx[PR], cpy[PR], spy[PR];
    PT pa[PR], pc1[PR], pc2[PR];
    if constexpr (REG) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int k = lane * P + j;   // table position; fine point (s, m) = (k % n_ang, k / n_ang)
            const bool ok = k < nf;
            const int i = a_patch * nf + (ok ? (k % A.n_ang) * A.n_rad + k / A.n_ang : 0);
            cpx[j] = ok ? trig_pt[i] : 1.0;
            spx[j] = ok ? trig_pt[np + i] : 0.0;
            cpy[j] = ok ? trig_pt[2 * np + i] : 1.0;
            spy[j] = ok ? trig_pt[3 * np + i] : 0.0;
            point_consts(ok, i, pa[j], pc1[j], pc2[j]);
            // the block's waves share the coefficients: wave j % 4 makes point j's
            // (expanded around the a the sweep uses, rounded to FP32)
            if ((j & 3) == wave) {
                const double wf = ok ? static_cast<double>(pa32[2 * np + i]) : 0.0;
                tay[j * 64 + lane] = taylor_consts<FULL>(static_cast<double>(pa[j]), FULL ? -wf * Tcur : wf);
            }
        }
        __syncthreads();
    } else {
        for (int k = threadIdx.x; k < S; k += kThreads) {
            const int slot = (k % P) * 64 + k / P;
            const bool ok = k < nf;
            const int i = a_patch * nf + (ok ? (k % A.n_ang) * A.n_rad + k / A.n_ang : 0);
            pt[0 * S + slot] = ok ? trig_pt[i] : 1.0;
            pt[1 * S + slot] = ok ? trig_pt[np + i] : 0.0;
            pt[2 * S + slot] = ok ? trig_pt[2 * np + i] : 1.0;
            pt[3 * S + slot] = ok ? trig_pt[3 * np + i] : 0.0;
            PT a, c1, c2;
            point_consts(ok, i, a, c1, c2);
            pt[4 * S + slot] = a;
            pt[5 * S + slot] = c1;
            pt[6 * S + slot] = c2;
        }
        __syncthreads();
    }
    auto pval = [&](int q, int j) -> double {
        if constexpr (REG) {
            return q == 0 ? cpx[j] : q == 1 ? spx[j] : q == 2 ? cpy[j] : q == 3 ? spy[j]
                 : q == 4 ? static_cast<double>(pa[j]) : q == 5 ? static_cast<double>(pc1[j])
                 : static_cast<double>(pc2[j]);
        } else {
            return pt[q * S + j * 64 + lane];
        }
    };
    // eps / 2T = K1 (cx + cy) - K2 cx cy - K3, the constants computed once and
    // kept in scalar registers
    const double inv2T = A.Tdev[1];
    const double K1 = uniform_f64(A.mt2 * inv2T), K3 = uniform_f64(A.mu * inv2T);
    const double G = uniform_f64(A.mt4p / (A.mt2 * A.mt2) * (1.0 / inv2T));   // K2 / K1^2 (t != 0)
    // second-line patches of the lane's points: one P-byte load when aligned
    const bool vec_bins = (nf % P) == 0 && (P == 4 || P == 8 || P == 16);
    constexpr int W = (P + 3) / 4;
    // second-line patches of the lane's points in table row r, four to a word
    // the argument block's pointers, read once (stores in the row loop could alias
    // the block for the compiler, which would otherwise reload them every row)
    const GLOBAL_AS uint8_t *const gbins = gld(A.bins);
    const CONST_AS double *const gtrig = cld(A.trig_row);
    auto load_bins = [&](int r, uint32_t *bw) {
        const GLOBAL_AS uint8_t *brow = gbins + static_cast<size_t>(r) * np + static_cast<size_t>(a_patch) * nf;
        if (vec_bins) {   // wave-uniform; lanes past n_f read the patch start (zero-weight points)
            const GLOBAL_AS uint8_t *src = brow + (lane * P < nf ? lane * P : 0);
            if constexpr (P == 4) {
                bw[0] = *reinterpret_cast<const GLOBAL_AS uint32_t *>(src);
            } else if constexpr (P >= 8) {
#pragma unroll
                for (int h = 0; h < P / 8; ++h) {
                    const uint64_t v = *reinterpret_cast<const GLOBAL_AS uint64_t *>(src + 8 * h);
                    bw[2 * h] = static_cast<uint32_t>(v);
                    bw[2 * h + 1] = static_cast<uint32_t>(v >> 32);
                }
            }
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) bw[w] = 0;
#pragma unroll
            for (int j = 0; j < P; ++j)
                bw[j >> 2] |= static_cast<uint32_t>(lane * P + j < nf ? brow[lane * P + j] : 0) << (8 * (j & 3));
        }
    };
    const size_t NN = static_cast<size_t>(N) * N;

    const int row0 = chunk * rpb;
    // the wave's bins start at zero; each row's output pass clears them again
    for (int b = lane; b < N; b += 64) bins[BS * b] = 0.0;
    if constexpr (PAIRED)
        for (int b = lane; b < N; b += 64) bins2[BS * b] = 0.0;
    // the wave's 16 transfer rows (and a pair's second rows), one per lane, read
    // once: each row then takes them with a lane read instead of a global load
    const int rows_per_wave = rpb >> 2;   // at most 64: one row index per lane
    const int my_slot = row0 + wave + 4 * lane;
    const bool my_ok = lane < rows_per_wave && my_slot < A.nrows;
    const int my_r = my_ok ? (A.rowlist ? A.rowlist[my_slot] : my_slot) : 0;
    // second-line patches of the lane's points, loaded one row ahead so that a
    // row's table bytes are in flight while the previous row is evaluated
    auto row_valid = [&](int it) { return it < rows_per_wave && row0 + wave + 4 * it < A.nrows; };
    uint32_t nbw[W];
    if (PF && row_valid(0)) load_bins(__builtin_amdgcn_readlane(my_r, 0), nbw);
    for (int it = 0; it < rows_per_wave; ++it) {
        const int rr = wave + 4 * it;
        const int slot_out = row0 + rr;                 // output row position (wave-uniform)
        if (slot_out >= A.nrows) break;
        // transfer row (wave-uniform: kept in scalar registers with its constants);
        // a pair's second row is the ph row of the opposite transfer
        const int r = __builtin_amdgcn_readlane(my_r, it);
        // Row-uniform factors.  pp: cos(q - p) = cos q cos p + sin q sin p and the
        // second line enters as -eps / 2T; ph: cos(p + Q) = cos p cos Q - sin p sin Q
        // and +eps / 2T, so b = k1 (cx + cy) - k2 cx cy - k3 with the channel's
        // signs in k1, k2, k3.  With X = k1 cx = (k1 cqx) cos px + (k1 sx) sin px and
        // Y = k1 cy likewise, b = X (1 - (k2 / k1^2) Y) + (Y - k3): seven FP64
        // operations, each with one scalar operand.  In a pair, r is the pp row.
        const bool pp = PAIRED || r < A.Tpp;
        const double k1 = pp ? -K1 : K1, g = pp ? -G : G, k3 = pp ? -K3 : K3;
        const CONST_AS double *tr = gtrig + 4 * r;
        const double cqx = uniform_f64(k1 * tr[0]), cqy = uniform_f64(k1 * tr[2]);
        const double sx = uniform_f64((pp ? k1 : -k1) * tr[1]);
        const double sy = uniform_f64((pp ? k1 : -k1) * tr[3]);
        uint32_t bw[W];
        if constexpr (PF) {
#pragma unroll
            for (int w = 0; w < W; ++w) bw[w] = nbw[w];
            if (row_valid(it + 1)) load_bins(__builtin_amdgcn_readlane(my_r, it + 1), nbw);
        } else {
            load_bins(r, bw);
        }
        auto bin_of = [&](const uint32_t *w, int j) -> int { return (w[j >> 2] >> (8 * (j & 3))) & 0xff; };
        // FP32 Taylor coefficients of point j: from LDS in register mode, else made
        // on the spot (w = -c2 / 4, or W = c2 for the full bubble)
        auto coef = [&](int j) -> float4 {
            if constexpr (REG) {
                return tay[j * 64 + lane];
            } else {
                const double c2 = pval(6, j);
                return taylor_consts<FULL>(pval(4, j), FULL ? c2 : -0.25 * c2);
            }
        };
        // weighted divided difference(s) of point j: the far form for every
        // lane, then the Taylor form where the lane is close to the diagonal
        auto value = [&](int j, PT &v, PT &v2) {
            const double Y = cqy * pval(2, j) + sy * pval(3, j);
            const double X = cqx * pval(0, j) + sx * pval(1, j);
            double bd = fma(X, fma(-g, Y, 1.0), Y - k3);
            // pp rows take the second line's energy with a minus sign
            if constexpr (SE) bd += (pp ? -1.0 : 1.0) * sgl[bin_of(bw, j)];
            const PT b = static_cast<PT>(bd);
            const PT a = static_cast<PT>(pval(4, j)), c1 = static_cast<PT>(pval(5, j)),
                     c2 = static_cast<PT>(pval(6, j));
            if constexpr (PAIRED) {
                if constexpr (F32 && FULL) wdiv_t32_pair(a, c1, c2, b, [&] { return coef(j); }, v, v2);
                else if constexpr (F32) wdiv_h32_pair(a, c1, c2, b, [&] { return coef(j); }, v, v2);
                else if constexpr (FULL) wdiv_t64_pair(a, c1, c2, b, v, v2);
                else wdiv_h64_pair(a, c1, c2, b, v, v2);
                return;
            }
            const PT d = a - b;
            if constexpr (F32) {
                v = FULL ? wdiv_t32_far(c1, c2, b, d) : wdiv_h32_far(c1, c2, b, d);
                if (fabsf(d) < kTaylor32) v = taylor_poly(coef(j), d);
            } else {
                if constexpr (FULL) {
                    v = wdiv_t64_far(c1, c2, b, d);
                    if (fabs(d) < kTaylor64) v = wdiv_t64_near(a, c2, b);
                } else {
                    v = wdiv_h64_far(c1, c2, b, d);
                    if (fabs(d) < kTaylor64) v = wdiv_h64_near(a, c2, b);
                }
            }
        };
        wave_sync();
        // Runs of equal bin summed in registers (at most P terms), one FP64 LDS
        // add per run.  Padding points (past n_f) carry zero weight.
        PT acc, acc2 = PT(0);
        value(0, acc, acc2);
        int bcur = bin_of(bw, 0);
#pragma unroll
        for (int j = 1; j < P; ++j) {
            PT v, v2 = PT(0);
            value(j, v, v2);
            const int bin = bin_of(bw, j);
            if (bin != bcur) {   // a pair's ph run ends with its pp run
                atomicAdd(&bins[BS * bcur], static_cast<double>(acc));
                acc = PT(0);
                if constexpr (PAIRED) {
                    atomicAdd(&bins2[BS * bcur], static_cast<double>(acc2));
                    acc2 = PT(0);
                }
            }
            acc += v;
            if constexpr (PAIRED) acc2 += v2;
            bcur = bin;
        }
        atomicAdd(&bins[BS * bcur], static_cast<double>(acc));
        if constexpr (PAIRED) atomicAdd(&bins2[BS * bcur], static_cast<double>(acc2));
        wave_sync();
        // outputs: a pair writes its pp row and its ph row at the same position.
        // A lane takes bins b and b + 64 of both rows at once (all reads issued
        // before the first store), and clears them.
        constexpr int NO = PAIRED ? 2 : 1;
        size_t base[NO];
        void *outp[NO];
        double *src[NO];
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const bool pp_out = PAIRED ? k == 0 : slot_out < A.npp_out;
            const size_t pos = PAIRED ? static_cast<size_t>(slot_out)
                                      : (pp_out ? static_cast<size_t>(slot_out)
                                                : static_cast<size_t>(slot_out - A.npp_out));
            base[k] = pos * NN + static_cast<size_t>(a_patch) * N;
            outp[k] = pp_out ? A.Bpp : A.Bph;
            src[k] = k == 0 ? bins : bins2;
        }
        const int H = N >> 1;
        if constexpr (PAIRED) {
            // a lane takes bins b, b + 1 (b even) of both rows: 32 contiguous bytes
            // of the interleaved bins; the ph row's values at pp-bin positions b,
            // b + 1 are its output bins b + N/2, b + N/2 + 1 (mod N; N % 8 == 0, so
            // the pair does not wrap), so both rows take one 2-wide store
            for (int b = 2 * lane; b < N; b += 128) {
                double2 *q = reinterpret_cast<double2 *>(bins + 2 * b);
                const double2 u0 = q[0], u1 = q[1];   // (pp b, ph@b), (pp b+1, ph@b+1)
                q[0] = make_double2(0.0, 0.0);
                q[1] = make_double2(0.0, 0.0);
                const int bph = b + H >= N ? b + H - N : b + H;
                typedef float f2v __attribute__((ext_vector_type(2)));
                typedef double d2v __attribute__((ext_vector_type(2)));
                if (F32) {
                    if (outp[0])
                        *reinterpret_cast<GLOBAL_AS f2v *>(gst(static_cast<float *>(outp[0])) + base[0] + b) =
                            f2v{static_cast<float>(u0.x), static_cast<float>(u1.x)};
                    if (outp[1])
                        *reinterpret_cast<GLOBAL_AS f2v *>(gst(static_cast<float *>(outp[1])) + base[1] + bph) =
                            f2v{static_cast<float>(u0.y), static_cast<float>(u1.y)};
                } else {
                    if (outp[0])
                        *reinterpret_cast<GLOBAL_AS d2v *>(gst(static_cast<double *>(outp[0])) + base[0] + b) =
                            d2v{u0.x, u1.x};
                    if (outp[1])
                        *reinterpret_cast<GLOBAL_AS d2v *>(gst(static_cast<double *>(outp[1])) + base[1] + bph) =
                            d2v{u0.y, u1.y};
                }
            }
            wave_sync();
            continue;
        }
        for (int b0 = lane; b0 < N; b0 += 128) {
            const int b1 = b0 + 64;
            const bool has1 = b1 < N;
            // ph output bin b sits at pp-bin position b + N/2 (an involution, so
            // every position is read and cleared by exactly one lane)
            int i0[NO], i1[NO];
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                i0[k] = k == 0 ? b0 : (b0 + H >= N ? b0 + H - N : b0 + H);
                i1[k] = k == 0 ? b1 : (b1 + H >= N ? b1 + H - N : b1 + H);
            }
            double v[NO][2];
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                v[k][0] = src[k][BS * i0[k]];
                v[k][1] = has1 ? src[k][BS * i1[k]] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < NO; ++k) {   // read and cleared by the same lane
                src[k][BS * i0[k]] = 0.0;
                if (has1) src[k][BS * i1[k]] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                if (!outp[k]) continue;
                if (F32) {
                    GLOBAL_AS float *o = gst(static_cast<float *>(outp[k])) + base[k];
                    o[b0] = static_cast<float>(v[k][0]);
                    if (has1) o[b1] = static_cast<float>(v[k][1]);
                } else {
                    GLOBAL_AS double *o = gst(static_cast<double *>(outp[k])) + base[k];
                    o[b0] = v[k][0];
                    if (has1) o[b1] = v[k][1];
                }
            }
        }
        wave_sync();
    }
}

// ----------------------------------------------------------------- segmented sweep
// The energy-angle grid holds thousands of points per patch (A.count[a] live,
// the rest zero-weight padding up to n_f, a multiple of kSegPoints).  A block
// (patch a, chunk of rows) walks the patch's live points in segments of
// kSegPoints = 64 lanes x 8: per segment the points are set up once (registers
// or LDS as in the unsegmented sweep), then every row of the block is evaluated
// on them into that row's own FP64 LDS bins, which therefore hold a whole
// block's rows (rpb x N doubles, twice for pairs) until the last segment; the
// rows are written after it.
constexpr int kSegP = kSegPoints / 64;

template <bool F32>
size_t seg_point_lds_bytes() {
    return points_in_registers<kSegP, F32>() ? sizeof(float4) * kSegPoints : sizeof(double) * 7 * kSegPoints;
}

// rows per block of the segmented sweep: the request (a multiple of 4), cut so
// that the block's LDS stays within 64 KB.  Default (measured at N = 96 with
// the paper's quadrature, 4..36 rows): 24 for the split path, where more rows
// amortise the per-segment point set-up until the LDS bins cut the blocks per
// CU; 8 for FP64, whose points sit in LDS and whose rows cost more registers.
template <bool F32>
int seg_rows_per_block(int N, bool paired, int req) {
    const size_t per_row = sizeof(double) * static_cast<size_t>(N) * (paired ? 2 : 1);
    // the points and a self-energy table (N doubles) take their part first
    const size_t room = 65536 - seg_point_lds_bytes<F32>() - sizeof(double) * static_cast<size_t>(N);
    int lim = static_cast<int>(room / per_row) / 4 * 4;
    lim = std::max(4, lim);
    const int r = req > 0 ? req : (F32 ? 24 : 8);
    return std::min(std::min(r, lim), 256);   // at most 64 rows per wave
}

template <bool F32>
size_t seg_lds_bytes(int N, bool paired, int rpb, bool se) {
    return sizeof(double) * static_cast<size_t>(rpb) * N * (paired ? 2 : 1) + seg_point_lds_bytes<F32>() +
           (se ? sizeof(double) * static_cast<size_t>(N) : 0);
}

// SE: the second line's energy carries its bin's self-energy (A.sigma, as S/2T
// in LDS after the point data); dL/dT rows only, paired as in bubble_body
template <bool F32, bool FULL, bool PAIRED, bool SE = false>
__global__ __launch_bounds__(kThreads) void bubble_seg_kernel(BubbleArgs A, int rpb) {
    static_assert(!SE || !FULL, "self-energy rows are dL/dT rows");
    extern __shared__ double smem[];
    using PT = typename std::conditional<F32, float, double>::type;
    constexpr int P = kSegP;
    constexpr bool REG = points_in_registers<P, F32>();
    constexpr int PR = REG ? P : 1;
    constexpr int S = kSegPoints;
    const int N = A.N, nf = A.nf, np = A.np;
    const int chunk = blockIdx.x, a_patch = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rpw = rpb >> 2;   // rows per wave
    constexpr int BS = PAIRED ? 2 : 1;   // a pair's rows interleaved: pp at 2b, ph (at the pp bin) at 2b + 1
    double *bins = smem + static_cast<size_t>(wave) * rpw * N * BS;          // [rpw][N][BS]
    double *pt = smem + static_cast<size_t>(PAIRED ? 8 : 4) * rpw * N;       // LDS mode: [7][S]
    float4 *tay = reinterpret_cast<float4 *>(pt);                            // register mode: [S]
    double *sgl = pt + (REG ? 2 * S : 7 * S);                                // SE: S_b / 2T
    if constexpr (SE)
        for (int b = threadIdx.x; b < N; b += kThreads) sgl[b] = A.sigma[b] * A.Tdev[1];

    const double Tcur = A.Tdev[0];
    const GLOBAL_AS float *pa32 = gld(A.pa32);
    const GLOBAL_AS double *pa64 = gld(A.pa64), *trig_pt = gld(A.trig_pt);
    const GLOBAL_AS uint8_t *const gbins = gld(A.bins);
    const CONST_AS double *const gtrig = cld(A.trig_row);
    auto point_consts = [&](int i, PT &a, PT &c1, PT &c2) {
        const double wf = F32 ? static_cast<double>(pa32[2 * np + i]) : pa64[2 * np + i];
        const double av = F32 ? static_cast<double>(pa32[i]) : pa64[i];
        a = static_cast<PT>(av);
        if constexpr (FULL) {
            const double W = -wf * Tcur;
            c1 = static_cast<PT>(W * tanh_d(av));
            c2 = static_cast<PT>(W);
        } else {
            const PT w = static_cast<PT>(wf);
            c1 = w * static_cast<PT>(F32 ? pa32[np + i] : pa64[np + i]);
            c2 = PT(-4) * w;
        }
    };
    const double inv2T = A.Tdev[1];
    const double K1 = uniform_f64(A.mt2 * inv2T), K3 = uniform_f64(A.mu * inv2T);
    const double G = uniform_f64(A.mt4p / (A.mt2 * A.mt2) * (1.0 / inv2T));
    const size_t NN = static_cast<size_t>(N) * N;

    const int row0 = chunk * rpb;
    for (int k = lane; k < rpw * N * BS; k += 64) bins[k] = 0.0;
    // the wave's rows, one per lane (at most 64 rows per wave)
    const int my_slot = row0 + wave + 4 * lane;
    const bool my_ok = lane < rpw && my_slot < A.nrows;
    const int my_r = my_ok ? (A.rowlist ? A.rowlist[my_slot] : my_slot) : 0;
    int nrow_w = 0;   // rows this wave evaluates
    while (nrow_w < rpw && row0 + wave + 4 * nrow_w < A.nrows) ++nrow_w;

    const int nseg = (A.count[a_patch] + S - 1) / S;
    double cpx[PR], spx[PR], cpy[PR], spy[PR];
    PT pa[PR], pc1[PR], pc2[PR];
    // the lane's 8 table bytes of row r in segment sg (in bounds: n_f is a
    // multiple of the segment)
    auto load_bins = [&](int r, int sg, uint32_t *bw) {
        const GLOBAL_AS uint8_t *src = gbins + static_cast<size_t>(r) * np + static_cast<size_t>(a_patch) * nf +
                                       sg * S + lane * P;
        const uint64_t v = *reinterpret_cast<const GLOBAL_AS uint64_t *>(src);
        bw[0] = static_cast<uint32_t>(v);
        bw[1] = static_cast<uint32_t>(v >> 32);
    };
    // the next row's table bytes are loaded while a row is evaluated (and the
    // first row's of a segment while its points are set up)
    uint32_t nbw[2] = {0u, 0u};
    if (nseg > 0 && nrow_w > 0) load_bins(__builtin_amdgcn_readlane(my_r, 0), 0, nbw);
    for (int sg = 0; sg < nseg; ++sg) {
        const int k0 = sg * S;
        // every wave is done with the previous segment's shared point data
        if (sg > 0) __syncthreads();
        if constexpr (REG) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int i = a_patch * nf + k0 + lane * P + j;
                cpx[j] = trig_pt[i];
                spx[j] = trig_pt[np + i];
                cpy[j] = trig_pt[2 * np + i];
                spy[j] = trig_pt[3 * np + i];
                point_consts(i, pa[j], pc1[j], pc2[j]);
                if ((j & 3) == wave) {
                    const double wf = static_cast<double>(pa32[2 * np + i]);
                    tay[j * 64 + lane] = taylor_consts<FULL>(static_cast<double>(pa[j]), FULL ? -wf * Tcur : wf);
                }
            }
        } else {
            for (int k = threadIdx.x; k < S; k += kThreads) {
                const int slot = (k % P) * 64 + k / P;
                const int i = a_patch * nf + k0 + k;
                pt[0 * S + slot] = trig_pt[i];
                pt[1 * S + slot] = trig_pt[np + i];
                pt[2 * S + slot] = trig_pt[2 * np + i];
                pt[3 * S + slot] = trig_pt[3 * np + i];
                PT a, c1, c2;
                point_consts(i, a, c1, c2);
                pt[4 * S + slot] = a;
                pt[5 * S + slot] = c1;
                pt[6 * S + slot] = c2;
            }
        }
        __syncthreads();
        auto pval = [&](int q, int j) -> double {
            if constexpr (REG) {
                return q == 0 ? cpx[j] : q == 1 ? spx[j] : q == 2 ? cpy[j] : q == 3 ? spy[j]
                     : q == 4 ? static_cast<double>(pa[j]) : q == 5 ? static_cast<double>(pc1[j])
                     : static_cast<double>(pc2[j]);
            } else {
                return pt[q * S + j * 64 + lane];
            }
        };
        auto coef = [&](int j) -> float4 {
            if constexpr (REG) {
                return tay[j * 64 + lane];
            } else {
                const double c2 = pval(6, j);
                return taylor_consts<FULL>(pval(4, j), FULL ? c2 : -0.25 * c2);
            }
        };
        auto bin_of = [&](const uint32_t *w, int j) -> int { return (w[j >> 2] >> (8 * (j & 3))) & 0xff; };
        for (int it = 0; it < nrow_w; ++it) {
            const int r = __builtin_amdgcn_readlane(my_r, it);
            const bool pp = PAIRED || r < A.Tpp;
            const double k1 = pp ? -K1 : K1, g = pp ? -G : G, k3 = pp ? -K3 : K3;
            const CONST_AS double *tr = gtrig + 4 * r;
            const double cqx = uniform_f64(k1 * tr[0]), cqy = uniform_f64(k1 * tr[2]);
            const double sx = uniform_f64((pp ? k1 : -k1) * tr[1]);
            const double sy = uniform_f64((pp ? k1 : -k1) * tr[3]);
            uint32_t bw[2] = {nbw[0], nbw[1]};
            if (it + 1 < nrow_w) load_bins(__builtin_amdgcn_readlane(my_r, it + 1), sg, nbw);
            else if (sg + 1 < nseg) load_bins(__builtin_amdgcn_readlane(my_r, 0), sg + 1, nbw);
            auto value = [&](int j, PT &v, PT &v2) {
                const double Y = cqy * pval(2, j) + sy * pval(3, j);
                const double X = cqx * pval(0, j) + sx * pval(1, j);
                double bd = fma(X, fma(-g, Y, 1.0), Y - k3);
                // pp rows take the second line's energy with a minus sign
                if constexpr (SE) bd += (pp ? -1.0 : 1.0) * sgl[bin_of(bw, j)];
                const PT b = static_cast<PT>(bd);
                const PT a = static_cast<PT>(pval(4, j)), c1 = static_cast<PT>(pval(5, j)),
                         c2 = static_cast<PT>(pval(6, j));
                if constexpr (PAIRED) {
                    if constexpr (F32 && FULL) wdiv_t32_pair(a, c1, c2, b, [&] { return coef(j); }, v, v2);
                    else if constexpr (F32) wdiv_h32_pair(a, c1, c2, b, [&] { return coef(j); }, v, v2);
                    else if constexpr (FULL) wdiv_t64_pair(a, c1, c2, b, v, v2);
                    else wdiv_h64_pair(a, c1, c2, b, v, v2);
                    return;
                }
                const PT d = a - b;
                if constexpr (F32) {
                    v = FULL ? wdiv_t32_far(c1, c2, b, d) : wdiv_h32_far(c1, c2, b, d);
                    if (fabsf(d) < kTaylor32) v = taylor_poly(coef(j), d);
                } else {
                    if constexpr (FULL) {
                        v = wdiv_t64_far(c1, c2, b, d);
                        if (fabs(d) < kTaylor64) v = wdiv_t64_near(a, c2, b);
                    } else {
                        v = wdiv_h64_far(c1, c2, b, d);
                        if (fabs(d) < kTaylor64) v = wdiv_h64_near(a, c2, b);
                    }
                }
            };
            double *rb = bins + static_cast<size_t>(it) * N * BS;
            double *rb2 = rb + 1;
            PT acc, acc2 = PT(0);
            value(0, acc, acc2);
            int bcur = bin_of(bw, 0);
#pragma unroll
            for (int j = 1; j < P; ++j) {
                PT v, v2 = PT(0);
                value(j, v, v2);
                const int bin = bin_of(bw, j);
                if (bin != bcur) {   // a pair's ph run ends with its pp run
                    atomicAdd(&rb[BS * bcur], static_cast<double>(acc));
                    acc = PT(0);
                    if constexpr (PAIRED) {
                        atomicAdd(&rb2[BS * bcur], static_cast<double>(acc2));
                        acc2 = PT(0);
                    }
                }
                acc += v;
                if constexpr (PAIRED) acc2 += v2;
                bcur = bin;
            }
            atomicAdd(&rb[BS * bcur], static_cast<double>(acc));
            if constexpr (PAIRED) atomicAdd(&rb2[BS * bcur], static_cast<double>(acc2));
        }
    }
    wave_sync();
    // the wave's rows out (each row's bins were written by this wave only)
    constexpr int NO = PAIRED ? 2 : 1;
    for (int it = 0; it < nrow_w; ++it) {
        const int slot_out = row0 + wave + 4 * it;
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const bool pp_out = PAIRED ? k == 0 : slot_out < A.npp_out;
            const size_t pos = PAIRED ? static_cast<size_t>(slot_out)
                                      : (pp_out ? static_cast<size_t>(slot_out)
                                                : static_cast<size_t>(slot_out - A.npp_out));
            const size_t base = pos * NN + static_cast<size_t>(a_patch) * N;
            void *outp = pp_out ? A.Bpp : A.Bph;
            if (!outp) continue;
            const double *src = bins + static_cast<size_t>(it) * N * BS + k;
            const int sh = k == 0 ? 0 : N >> 1;   // ph bins sit at the pp bin + N/2
            for (int b = lane; b < N; b += 64) {
                const int i = b + sh >= N ? b + sh - N : b + sh;
                if (F32) gst(static_cast<float *>(outp))[base + b] = static_cast<float>(src[BS * i]);
                else gst(static_cast<double *>(outp))[base + b] = src[BS * i];
            }
        }
    }
}

template <bool F32, bool FULL>
void launch_seg(const BubbleArgs &a, hipStream_t s) {
    const bool paired = a.rowlist_ph != nullptr;
    const int rpb = seg_rows_per_block<F32>(a.N, paired, a.rpb);
    dim3 grid((a.nrows + rpb - 1) / rpb, a.N);
    const bool se = a.sigma != nullptr && !FULL;   // dL/dT rows only
    const size_t lds = seg_lds_bytes<F32>(a.N, paired, rpb, se);
    if (se) {
        if constexpr (!FULL) {
            if (paired)
                hipLaunchKernelGGL((bubble_seg_kernel<F32, false, true, true>), grid, dim3(kThreads), lds, s, a, rpb);
            else
                hipLaunchKernelGGL((bubble_seg_kernel<F32, false, false, true>), grid, dim3(kThreads), lds, s, a,
                                   rpb);
        }
    } else if (paired) {
        hipLaunchKernelGGL((bubble_seg_kernel<F32, FULL, true>), grid, dim3(kThreads), lds, s, a, rpb);
    } else {
        hipLaunchKernelGGL((bubble_seg_kernel<F32, FULL, false>), grid, dim3(kThreads), lds, s, a, rpb);
    }
}

template <int P, bool F32, bool FULL, bool PAIRED, bool SE = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void bubble_kernel(BubbleArgs A) {
    extern __shared__ double smem[];
    bubble_body<P, F32, FULL, PAIRED, PAIRED, SE>(A, blockIdx.x, blockIdx.y, smem,
                                                  A.rpb > 0 ? A.rpb : kRowsPerBlock);
}

// batched: item = (flow, chunk << 8 | patch); skips flows whose state says stop.
// The items of flows with row pairs and of flows without are separate launches.
template <int P, bool F32, bool PAIRED>
__global__ __launch_bounds__(kThreads) void bubble_kernel_batched(
        const BubbleArgs *__restrict__ args, const int2 *__restrict__ items,
        const double *const *__restrict__ states) {
    extern __shared__ double smem[];
    const int2 it = items[blockIdx.x];
    if (states && states[it.x][FRG_ST_REASON] != 0.0) return;
    const BubbleArgs &A = args[it.x];
    bubble_body<P, F32, false, PAIRED, true>(A, it.y >> 8, it.y & 255, smem, A.rpb);
}

template <int P, bool PAIRED>
void launch_pp(const BubbleArgs &a, bool fp32, bool full, hipStream_t s) {
    const int rpb = a.rpb > 0 ? a.rpb : kRowsPerBlock;
    dim3 grid((a.nrows + rpb - 1) / rpb, a.N);
    const size_t lds = fp32 ? bubble_lds_bytes<P, true>(a.N, PAIRED) : bubble_lds_bytes<P, false>(a.N, PAIRED);
    if (a.sigma && !full) {   // a self-energy: dL/dT rows only (paired when it is C4v invariant)
        const size_t l = lds + sizeof(double) * static_cast<size_t>(a.N);
        if (fp32) hipLaunchKernelGGL((bubble_kernel<P, true, false, PAIRED, true>), grid, dim3(kThreads), l, s, a);
        else hipLaunchKernelGGL((bubble_kernel<P, false, false, PAIRED, true>), grid, dim3(kThreads), l, s, a);
        return;
    }
    if (fp32 && !full)
        hipLaunchKernelGGL((bubble_kernel<P, true, false, PAIRED>), grid, dim3(kThreads), lds, s, a);
    else if (!fp32 && !full)
        hipLaunchKernelGGL((bubble_kernel<P, false, false, PAIRED>), grid, dim3(kThreads), lds, s, a);
    else if (fp32)
        hipLaunchKernelGGL((bubble_kernel<P, true, true, PAIRED>), grid, dim3(kThreads), lds, s, a);
    else
        hipLaunchKernelGGL((bubble_kernel<P, false, true, PAIRED>), grid, dim3(kThreads), lds, s, a);
}

template <int P>
void launch_p(const BubbleArgs &a, bool fp32, bool full, hipStream_t s) {
    if (a.rowlist_ph) launch_pp<P, true>(a, fp32, full, s);
    else launch_pp<P, false>(a, fp32, full, s);
}

template <int P, bool PAIRED>
void launch_pbp(const BubbleArgs *args, const int2 *items, int nitems, const double *const *states,
                int maxN, bool fp32, hipStream_t s) {
    if (nitems <= 0) return;
    const size_t lds = fp32 ? bubble_lds_bytes<P, true>(maxN, PAIRED) : bubble_lds_bytes<P, false>(maxN, PAIRED);
    if (fp32)
        hipLaunchKernelGGL((bubble_kernel_batched<P, true, PAIRED>), dim3(nitems), dim3(kThreads), lds, s, args,
                           items, states);
    else
        hipLaunchKernelGGL((bubble_kernel_batched<P, false, PAIRED>), dim3(nitems), dim3(kThreads), lds, s, args,
                           items, states);
}

template <int P>
void launch_pb(const BubbleArgs *args, const int2 *items, int npaired, int nitems, const double *const *states,
               int maxN, bool fp32, hipStream_t s) {
    launch_pbp<P, true>(args, items, npaired, states, maxN, fp32, s);
    launch_pbp<P, false>(args, items + npaired, nitems - npaired, states, maxN, fp32, s);
}

}  // namespace

int bubble_batched_rows_per_block(int nrows) {
    const int nch = std::max(1, (nrows + kRowsPerBlockBatched - 1) / kRowsPerBlockBatched);
    const int per = (nrows + nch - 1) / nch;
    return std::min(256, (per + 3) / 4 * 4);
}

void launch_bubbles_batched(const BubbleArgs *args, const int2 *items, int npaired, int nitems,
                            const double *const *states, int nf, int maxN, bool fp32, hipStream_t s) {
    const int P = (nf + 63) / 64;
    if (P <= 1) launch_pb<1>(args, items, npaired, nitems, states, maxN, fp32, s);
    else if (P <= 2) launch_pb<2>(args, items, npaired, nitems, states, maxN, fp32, s);
    else if (P <= 4) launch_pb<4>(args, items, npaired, nitems, states, maxN, fp32, s);
    else if (P <= 8) launch_pb<8>(args, items, npaired, nitems, states, maxN, fp32, s);
    else launch_pb<16>(args, items, npaired, nitems, states, maxN, fp32, s);
}

void launch_bubbles(const BubbleArgs &a, bool fp32, bool full, hipStream_t s) {
    if (a.count) {   // energy-angle grid: segments of the patch's live points
        if (fp32 && !full) launch_seg<true, false>(a, s);
        else if (!fp32 && !full) launch_seg<false, false>(a, s);
        else if (fp32) launch_seg<true, true>(a, s);
        else launch_seg<false, true>(a, s);
        return;
    }
    const int P = (a.nf + 63) / 64;
    if (P <= 1) launch_p<1>(a, fp32, full, s);
    else if (P <= 2) launch_p<2>(a, fp32, full, s);
    else if (P <= 4) launch_p<4>(a, fp32, full, s);
    else if (P <= 8) launch_p<8>(a, fp32, full, s);
    else launch_p<16>(a, fp32, full, s);
}

}  // namespace frg
