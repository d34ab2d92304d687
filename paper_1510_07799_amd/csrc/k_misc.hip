// Small device kernels: second-line patch table, per-point temperature
// factors, contraction operand layout, channel combine and the explicit
// Runge-Kutta machinery (stage sums, FP64 error norm, on-device step control).
#include <algorithm>
#include <cmath>

#include <mutex>
#include <vector>

#include "frg_internal.h"

namespace frg {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;

__device__ __forceinline__ double dev_fold(double x) {
    while (x >= kPi) x -= kTwoPi;
    while (x < -kPi) x += kTwoPi;
    return x;
}

// cross(b, k) >= 0 and cross(b', k) < 0 with each product rounded on its own
__device__ __forceinline__ bool dev_in_sector(const double *bnd, int j, double kx, double ky) {
    const double u0 = __dmul_rn(bnd[2 * j], ky), v0 = __dmul_rn(bnd[2 * j + 1], kx);
    const double u1 = __dmul_rn(bnd[2 * j + 2], ky), v1 = __dmul_rn(bnd[2 * j + 3], kx);
    return __dsub_rn(u0, v0) >= 0.0 && __dsub_rn(u1, v1) < 0.0;
}

// patch of a folded momentum: unique sector j with cross(b_j,k) >= 0 and
// cross(b_{j+1},k) < 0; an FP32 atan2 only picks where the search starts
__device__ int dev_patch(const double *bnd, int N, double kx, double ky) {
    if (kx == 0.0 && ky == 0.0) return 0;
    float th = atan2f(static_cast<float>(ky), static_cast<float>(kx));
    if (th < 0.f) th += 6.28318530717958647f;
    int j0 = static_cast<int>(th * (static_cast<float>(N) * 0.159154943091895336f));
    j0 = j0 < 0 ? 0 : (j0 >= N ? N - 1 : j0);
    for (int d = 0; d <= N / 2; ++d) {
        int j = j0 + d;
        j = j >= N ? j - N : j;
        if (dev_in_sector(bnd, j, kx, ky)) return j;
        j = j0 - d;
        j = j < 0 ? j + N : j;
        if (dev_in_sector(bnd, j, kx, ky)) return j;
    }
    return 0;
}

// The table keeps each patch's points in angular-fastest order: fine point
// (s, m) of patch a (sub-ray s, radius m; fine-grid index a*n_f + s*n_rad + m)
// sits at a*n_f + m*n_ang + s.  A lane of the bubble sweep takes consecutive
// entries, i.e. angular neighbours at one radius, whose second lines mostly
// share a patch.
__device__ __forceinline__ int bin_slot(int i, int n_rad, int n_ang) {
    const int nf = n_rad * n_ang;
    const int a = i / nf, loc = i - a * nf;
    const int s = loc / n_rad, m = loc - s * n_rad;
    return a * nf + m * n_ang + s;
}

__global__ void bins_kernel(const double *__restrict__ bnd, const double *__restrict__ px,
                            const double *__restrict__ py, const double *__restrict__ qrow,
                            int N, int n_rad, int n_ang, int Tpp, int Trows, uint8_t *__restrict__ bins) {
    const int np = N * n_rad * n_ang;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const int slot = bin_slot(i, n_rad, n_ang);
    for (int r = blockIdx.y; r < Trows; r += gridDim.y) {
        const double qx = qrow[2 * r], qy = qrow[2 * r + 1];
        double kx, ky;
        if (r < Tpp) {          // pp: second line q - p
            kx = dev_fold(qx - px[i]);
            ky = dev_fold(qy - py[i]);
        } else {                // ph: second line p + Q
            kx = dev_fold(px[i] + qx);
            ky = dev_fold(py[i] + qy);
        }
        bins[static_cast<size_t>(r) * np + slot] = static_cast<uint8_t>(dev_patch(bnd, N, kx, ky));
    }
}

// the table in fine-grid order (rows r0 .. r0 + nrows - 1)
__global__ void bins_export_kernel(const uint8_t *__restrict__ bins, int N, int n_rad, int n_ang, int r0,
                                   int nrows, uint8_t *__restrict__ out) {
    const int np = N * n_rad * n_ang;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const int slot = bin_slot(i, n_rad, n_ang);
    for (int r = blockIdx.y; r < nrows; r += gridDim.y)
        out[static_cast<size_t>(r) * np + i] = bins[static_cast<size_t>(r0 + r) * np + slot];
}

// image of patch j under C4v element o (o even: rotation by o/2 quarter
// turns; o odd: reflection about the axis at (o+1) pi/8)
__device__ __forceinline__ int c4v_patch(int o, int j, int N) {
    const int q = N >> 2;
    int v = (o & 1) ? ((o + 1) >> 1) * q - 1 - j : j + (o >> 1) * q;   // in (-N, 2N)
    v += v < 0 ? N : 0;
    return v >= N ? v - N : v;
}

// orbit[t'] = (rep row << 3) | o with t' = o . rep
__global__ void sym_check_kernel(const uint8_t *__restrict__ bins, const int32_t *__restrict__ orbit,
                                 int N, int n_rad, int n_ang, int Trows, bool rev, int *mismatch) {
    const int nf = n_rad * n_ang, np = N * nf;
    const int ip = blockIdx.x * blockDim.x + threadIdx.x;
    if (ip >= np) return;
    const int a1 = ip / nf, loc = ip - a1 * nf;
    const int s1 = loc / n_rad, m = loc - s1 * n_rad;
    int bad = 0;
    for (int t = blockIdx.y; t < Trows; t += gridDim.y) {
        const int info = orbit[t];
        const int rep = info >> 3, o = info & 7;
        if (o == 0) continue;
        const int oinv = (o & 1) ? o : ((8 - o) & 7);
        const int a = c4v_patch(oinv, a1, N);
        const int s = (rev && (o & 1)) ? n_ang - 1 - s1 : s1;
        const int b = bins[static_cast<size_t>(rep) * np + a * nf + m * n_ang + s];
        if (bins[static_cast<size_t>(t) * np + a1 * nf + m * n_ang + s1] != c4v_patch(o, b, N)) ++bad;
    }
    if (bad) atomicAdd(mismatch, bad);
}

// pairs of bubble rows (pp row q, ph row of -q): the ph second line p - q is
// the inverse of the pp one q - p, so its patch must be the pp patch + N/2 at
// every point; counts the (pair, point) entries where the table says otherwise
__global__ void pair_check_kernel(const uint8_t *__restrict__ bins, const int32_t *__restrict__ rows_pp,
                                  const int32_t *__restrict__ rows_ph, int npairs, int np, int N,
                                  int *mismatch) {
    const int ip = blockIdx.x * blockDim.x + threadIdx.x;
    if (ip >= np) return;
    const int H = N >> 1;
    int bad = 0;
    for (int i = blockIdx.y; i < npairs; i += gridDim.y) {
        const int b = bins[static_cast<size_t>(rows_pp[i]) * np + ip];
        const int b2 = bins[static_cast<size_t>(rows_ph[i]) * np + ip];
        if (b2 != (b + H >= N ? b + H - N : b + H)) ++bad;
    }
    if (bad) atomicAdd(mismatch, bad);
}

__device__ __forceinline__ double sech2_d(double x) {
    const double e = exp(-2.0 * fabs(x));
    const double d = 1.0 + e;
    return 4.0 * e / (d * d);
}

__global__ void point_prep_kernel(const double *__restrict__ xi, const double *__restrict__ w,
                                  int np, double T_host, const double *__restrict__ state,
                                  double c_stage, double *__restrict__ pa64,
                                  float *__restrict__ pa32, double *__restrict__ Tout,
                                  const double *__restrict__ sigma, int nf) {
    const double T = state ? exp(state[FRG_ST_S] + c_stage * state[FRG_ST_H]) : T_host;
    const double inv2T = 0.5 / T;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        Tout[0] = T;
        Tout[1] = inv2T;
    }
    if (i >= np) return;
    // with a self-energy the point's energy carries its patch's value
    const double a = (sigma ? xi[i] + sigma[i / nf] : xi[i]) * inv2T;
    const double ha = a * sech2_d(a);
    const double wf = -w[i] / (4.0 * T * T);
    if (pa64) {
        pa64[i] = a;
        pa64[np + i] = ha;
        pa64[2 * np + i] = wf;
    }
    if (pa32) {
        pa32[i] = static_cast<float>(a);
        pa32[np + i] = static_cast<float>(ha);
        pa32[2 * np + i] = static_cast<float>(wf);
    }
}

// Self-energy flow, patch sums: block a adds w_p d/dT n_F(x/T) = w_p x/(4T^2)
// sech^2(x/2T), x = xi_p + S_a, over the patch's points (thread t takes points
// t, t + 256, ...; then a fixed tree over the block), so the sum is reproducible.
__global__ __launch_bounds__(256) void dsigma_patch_kernel(const double *__restrict__ xi,
                                                           const double *__restrict__ w, int nf,
                                                           const double *__restrict__ S,
                                                           const double *__restrict__ Tdev,
                                                           double *__restrict__ D) {
    __shared__ double part[256];
    const int a = blockIdx.x;
    const double T = Tdev[0];
    const double sa = S[a];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nf; k += 256) {
        const int i = a * nf + k;
        const double x = xi[i] + sa;
        acc += w[i] * (x / (4.0 * T * T) * sech2_d(x / (2.0 * T)));
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) D[a] = part[0];
}

// dS_j = scale * sum_a D_a (2 V(j,a,j) - V(a,j,j)): block j, thread a, summed
// by a fixed tree (bit-reproducible).  V is the full vertex, or (ppos given) a
// reduced flow state read through the pp column map: V(a, b, m) =
// Vr[pos N + patch of m under the column's element] with (pos, element) =
// ppos[a N + b], the same values an expansion writes.  N <= 256.
__global__ __launch_bounds__(256) void dsigma_kernel(int N, const double *__restrict__ V,
                                                     const int32_t *__restrict__ ppos,
                                                     const double *__restrict__ D,
                                                     const double *__restrict__ Tdev, int scale_by_T,
                                                     double *__restrict__ dS) {
    __shared__ double part[256];
    const int j = blockIdx.x, a = threadIdx.x;
    const size_t NN = static_cast<size_t>(N) * N;
    auto at = [&](int x, int y, int m) -> double {
        if (!ppos) return V[static_cast<size_t>(x) * NN + static_cast<size_t>(y) * N + m];
        const int32_t cm = ppos[x * N + y];
        return V[static_cast<size_t>(cm >> 3) * N + c4v_patch(cm & 7, m, N)];
    };
    part[a] = a < N ? D[a] * (2.0 * at(j, a, j) - at(a, j, j)) : 0.0;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (a < h) part[a] += part[a + h];
        __syncthreads();
    }
    if (a == 0) dS[j] = (scale_by_T ? Tdev[0] : 1.0) * part[0];
}

// Contraction operands of V (each N^3; row m = i, contraction index
// kk = j*N + k, i.e. (a, b) = (j, k)).  The A operands are stored chunk-major,
// [kk / 8][m][kk % 8], so that one 8-wide k chunk of all rows is one
// contiguous run: the contraction reads the chunks of a column tile's active
// list, which need not be adjacent.  The gather tables stay row-major.
//   FP64 perm blocks:
//     0: V[j][k][i]                pp A       (row j3 = i)
//     1: V[i][j][k]                phc A      (row j1 = i)
//     2: V[j][i][k]                phd A      (row j2 = i)
//     3: V[k][i][j]                phc gather (column (y, x) = (i, j), b = k)
//     4: V[i][k][j]                phd gather (column (y, x) = (i, j), b = k;
//                                              and y = i, (a, b) = (j, k))
//   The contractions take the direct-ph sum (-2 V(a,j2,b) + V(j2,a,b)) V(j1,b,j3)
//   + V(a,j2,b) V(j1,b,a) as V(j2,a,b) V(j1,b,j3) + V(a,j2,b) (V(j1,b,a) -
//   2 V(j1,b,j3)): blocks 1 and 2 serve it.
//   split: ahl = A blocks 0, 1 and 2 as bf16 hi, lo ([3][2][N^3], chunk-major);
//          g32 = [V (pp gather), block 3, block 4] in FP32.
//
// One layout pass is a grid of layout_blocks(N) blocks of 256 threads:
//  - A part: a thread makes one (chunk c, row i) run of 8 entries of every A
//    operand (i fastest, so a wave's stores are contiguous).  pp reads
//    V[kk][i] (coalesced across the rows i); phc and phd read 8 consecutive
//    entries of a row of V.  The split path also writes the pp gather table
//    (a copy of V in FP32) from the phc reads.
//  - gather part: 32 x 32 tiles transposed through LDS, block 4 as the
//    transpose of V seen as [k][(i, j)], block 5 per i as that of V[i] seen as
//    [k][j].
constexpr int kLayoutTile = 32;

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

__host__ __device__ __forceinline__ int layout_a_blocks(int N) {
    return static_cast<int>((static_cast<int64_t>(N) * N * N / 8 + 255) / 256);
}
__host__ __device__ __forceinline__ int layout_t_tiles(int N) { return (N + kLayoutTile - 1) / kLayoutTile; }

// The split layout can read a flow's reduced state directly (one entry per
// representative pp column and free index): V(a, b, m) = Vr[pos N + perm8[o][m]]
// with (pos, o) = ppos[a N + b].  Only the gather rows of representative columns
// are written then (the contraction reads no others).
struct RedSrc {
    const double *Vr;
    const int32_t *ppos;           // pp column map: position << 3 | C4v element
    const int32_t *cperm_ph;       // representative ph columns (natural index), ncol_ph of them
    int ncol_ph;
    __device__ __forceinline__ double at(int N, int a, int b, int m) const {
        const int32_t cm = ppos[a * N + b];
        return Vr[(cm >> 3) * N + c4v_patch(cm & 7, m, N)];
    }
};

// A operands of chunk c, row i
template <bool SPLIT, bool RED = false>
__device__ __forceinline__ void layout_a_unit(const double *__restrict__ V, int N, int64_t n3, int64_t u,
                                              uint16_t *__restrict__ ahl, float *__restrict__ g32,
                                              double *__restrict__ perm, const RedSrc &R) {
    const int64_t NN = static_cast<int64_t>(N) * N;
    // u < N^3 / 8 <= 2^21: 32-bit divisions
    const uint32_t u32 = static_cast<uint32_t>(u), cu = u32 / static_cast<uint32_t>(N);
    const int i = static_cast<int>(u32 - cu * N);
    const int64_t c = cu;
    const int64_t kk0 = 8 * c;
    double pp[8], phc[8], phd[8];
    bool write_g = true;
    if constexpr (RED) {   // N % 8 == 0 here (a C4v-covariant grid)
        const int kk = static_cast<int>(kk0), j = kk / N, k0 = kk - j * N;
        const int32_t cc = R.ppos[i * N + j], cd = R.ppos[j * N + i];
        const double *rc = R.Vr + (cc >> 3) * N, *rd = R.Vr + (cd >> 3) * N;
        if (N % 32 == 0) {
            // k0 and the rotations' shifts (multiples of N/4) are multiples of 8, so
            // the 8 patches k0 .. k0+7 map to one aligned run of 8 entries of the
            // row, in reverse order for a reflection: 16-byte loads
            auto run8 = [&](const double *row, int o, double *out) {
                const bool refl = (o & 1) != 0;
                const double2 *src = reinterpret_cast<const double2 *>(row + c4v_patch(o, refl ? k0 + 7 : k0, N));
                double tmp[8];
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const double2 v = src[h];
                    tmp[2 * h] = v.x;
                    tmp[2 * h + 1] = v.y;
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) out[t] = refl ? tmp[7 - t] : tmp[t];
            };
            run8(rc, cc & 7, phc);
            run8(rd, cd & 7, phd);
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                phc[t] = rc[c4v_patch(cc & 7, k0 + t, N)];
                phd[t] = rd[c4v_patch(cd & 7, k0 + t, N)];
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) pp[t] = R.at(N, j, k0 + t, i);
        write_g = (cc & 7) == 0;   // gather row (i, j) of a representative pp column
    }
    const double *vrow = V + i * NN + kk0;
    if constexpr (RED) {
    } else if (N % 8 == 0) {   // the chunk lies in one j row: contiguous 64-byte runs
        const int j = static_cast<int>(kk0 / N), k0 = static_cast<int>(kk0 - static_cast<int64_t>(j) * N);
        const double *drow = V + (static_cast<int64_t>(j) * N + i) * N + k0;
#pragma unroll
        for (int t = 0; t < 8; t += 2) {
            const double2 a = *reinterpret_cast<const double2 *>(vrow + t);
            const double2 b = *reinterpret_cast<const double2 *>(drow + t);
            phc[t] = a.x; phc[t + 1] = a.y;
            phd[t] = b.x; phd[t + 1] = b.y;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t kk = kk0 + t;
            const int64_t j = kk / N, k = kk - j * N;
            phc[t] = vrow[t];
            phd[t] = V[(j * N + i) * N + k];
        }
    }
    if constexpr (!RED) {
#pragma unroll
        for (int t = 0; t < 8; ++t) pp[t] = V[(kk0 + t) * N + i];
    }
    const int64_t cm = (c * N + i) * 8;
    if constexpr (SPLIT) {
        float ops[3][8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            ops[0][t] = static_cast<float>(pp[t]);
            ops[1][t] = static_cast<float>(phc[t]);
            ops[2][t] = static_cast<float>(phd[t]);
        }
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            uint32_t hw[4], lw[4];
#pragma unroll
            for (int t = 0; t < 8; t += 2) {
                const uint16_t h0 = bf16_rne(ops[o][t]), h1 = bf16_rne(ops[o][t + 1]);
                const uint16_t l0 = bf16_rne(ops[o][t] - bf16_to_f(h0));
                const uint16_t l1 = bf16_rne(ops[o][t + 1] - bf16_to_f(h1));
                hw[t / 2] = static_cast<uint32_t>(h0) | (static_cast<uint32_t>(h1) << 16);
                lw[t / 2] = static_cast<uint32_t>(l0) | (static_cast<uint32_t>(l1) << 16);
            }
            *reinterpret_cast<uint4 *>(ahl + (2 * o) * n3 + cm) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
            *reinterpret_cast<uint4 *>(ahl + (2 * o + 1) * n3 + cm) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
        }
        if (write_g) {
            float4 *g = reinterpret_cast<float4 *>(g32 + i * NN + kk0);
            g[0] = make_float4(ops[1][0], ops[1][1], ops[1][2], ops[1][3]);
            g[1] = make_float4(ops[1][4], ops[1][5], ops[1][6], ops[1][7]);
        }
    } else {
#pragma unroll
        for (int t = 0; t < 8; t += 2) {
            *reinterpret_cast<double2 *>(perm + cm + t) = make_double2(pp[t], pp[t + 1]);
            *reinterpret_cast<double2 *>(perm + n3 + cm + t) = make_double2(phc[t], phc[t + 1]);
            *reinterpret_cast<double2 *>(perm + 2 * n3 + cm + t) = make_double2(phd[t], phd[t + 1]);
        }
    }
}

// one 32 x 32 tile of out[col][r] = get(r, col) for the output rows col that
// keep(col) accepts (rows x cols input), stored as OUT
template <typename OUT, class GET, class KEEP, class OROW>
__device__ __forceinline__ void layout_transpose_gen(GET get, KEEP keep, OROW orow, int rows, int64_t cols, int r0,
                                                     int64_t c0, OUT *__restrict__ out, int64_t ld_out,
                                                     double (*tile)[kLayoutTile + 1]) {
    const int tx = threadIdx.x & (kLayoutTile - 1), ty = threadIdx.x / kLayoutTile;   // 32 x 8
#pragma unroll
    for (int p = 0; p < kLayoutTile; p += 8) {
        const int r = r0 + ty + p;
        const int64_t c = c0 + tx;
        tile[ty + p][tx] = (r < rows && c < cols && keep(c)) ? get(r, c) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kLayoutTile; p += 8) {
        const int64_t c = c0 + ty + p;
        const int r = r0 + tx;
        if (r < rows && c < cols && keep(c)) out[orow(c) * ld_out + r] = static_cast<OUT>(tile[tx][ty + p]);
    }
}

// one 32 x 32 tile of out[r][col] = in[col][r] (in: rows x cols, row stride ld_in;
// out: cols x rows, row stride ld_out), stored as OUT
template <typename OUT>
__device__ __forceinline__ void layout_transpose_tile(const double *__restrict__ in, int rows, int64_t cols,
                                                      int64_t ld_in, int r0, int64_t c0, OUT *__restrict__ out,
                                                      int64_t ld_out, double (*tile)[kLayoutTile + 1]) {
    const int tx = threadIdx.x & (kLayoutTile - 1), ty = threadIdx.x / kLayoutTile;   // 32 x 8
#pragma unroll
    for (int p = 0; p < kLayoutTile; p += 8) {
        const int r = r0 + ty + p;
        const int64_t c = c0 + tx;
        tile[ty + p][tx] = (r < rows && c < cols) ? in[r * ld_in + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kLayoutTile; p += 8) {
        const int64_t c = c0 + ty + p;
        const int r = r0 + tx;
        if (r < rows && c < cols) out[c * ld_out + r] = static_cast<OUT>(tile[tx][ty + p]);
    }
}

typedef double LayoutTile[kLayoutTile + 1];   // rows of the 32 x 33 LDS tile a layout block uses

// block blk of a layout pass
template <bool SPLIT>
__device__ __forceinline__ void layout_block(const double *__restrict__ V, int N, int64_t n3, int blk,
                                             uint16_t *__restrict__ ahl, float *__restrict__ g32,
                                             double *__restrict__ perm, LayoutTile *tile) {
    
    const int na = layout_a_blocks(N), nt = layout_t_tiles(N);
    const int64_t NN = static_cast<int64_t>(N) * N;
    if (blk < na) {
        const int64_t u = static_cast<int64_t>(blk) * 256 + threadIdx.x;
        if (u < n3 / 8) layout_a_unit<SPLIT>(V, N, n3, u, ahl, g32, perm, RedSrc{});
        return;
    }
    blk -= na;
    const int nt1 = nt * static_cast<int>((NN + kLayoutTile - 1) / kLayoutTile);
    if (blk < nt1) {   // block 4: out[(i, j)][k] = V[k][(i, j)]
        const int rt = blk % nt;
        const int64_t ct = blk / nt;
        if constexpr (SPLIT)
            layout_transpose_tile<float>(V, N, NN, NN, rt * kLayoutTile, ct * kLayoutTile, g32 + n3, N, tile);
        else
            layout_transpose_tile<double>(V, N, NN, NN, rt * kLayoutTile, ct * kLayoutTile, perm + 3 * n3, N, tile);
        return;
    }
    blk -= nt1;        // block 5: out[i][j][k] = V[i][k][j]
    const int i = blk / (nt * nt), rem = blk - i * nt * nt;
    const int rt = rem % nt, ct = rem / nt;
    if constexpr (SPLIT)
        layout_transpose_tile<float>(V + i * NN, N, N, N, rt * kLayoutTile, ct * kLayoutTile, g32 + 2 * n3 + i * NN,
                                     N, tile);
    else
        layout_transpose_tile<double>(V + i * NN, N, N, N, rt * kLayoutTile, ct * kLayoutTile,
                                      perm + 4 * n3 + i * NN, N, tile);
}

__global__ __launch_bounds__(256) void layout_f64_kernel(const double *__restrict__ V, int N,
                                                         double *__restrict__ perm) {
    const int64_t n3 = static_cast<int64_t>(N) * N * N;
    __shared__ LayoutTile tile[kLayoutTile];
    layout_block<false>(V, N, n3, blockIdx.x, nullptr, nullptr, perm, tile);
}

// block blk of a split layout pass from a reduced state: the A units as in
// layout_block<true>, then the phd gather (block 5) in full, then the phc gather
// (block 4) of the representative ph columns only, in 32 x 32 tiles of (k,
// position in the representative list); blocks past layout_blocks_red(N, ncol_ph)
// have nothing to do
__host__ __device__ __forceinline__ int layout_blocks_red(int N, int ncol_ph) {
    const int nt = layout_t_tiles(N);
    return layout_a_blocks(N) + N * nt * nt + nt * ((ncol_ph + kLayoutTile - 1) / kLayoutTile);
}
__device__ __forceinline__ void layout_block_red(const RedSrc &R, int N, int64_t n3, int blk,
                                                 uint16_t *__restrict__ ahl, float *__restrict__ g32,
                                                 LayoutTile *tile) {
    const int na = layout_a_blocks(N), nt = layout_t_tiles(N);
    const int64_t NN = static_cast<int64_t>(N) * N;
    if (blk < na) {
        const int64_t u = static_cast<int64_t>(blk) * 256 + threadIdx.x;
        if (u < n3 / 8) layout_a_unit<true, true>(nullptr, N, n3, u, ahl, g32, nullptr, R);
        return;
    }
    blk -= na;
    const int n5 = N * nt * nt;
    if (blk < n5) {    // block 5: out[i][j][k] = V(i, k, j)
        const int i = blk / (nt * nt), rem = blk - i * nt * nt;
        const int rt = rem % nt, ct = rem / nt;
        layout_transpose_gen<float>([&](int k, int64_t j) { return R.at(N, i, k, static_cast<int>(j)); },
                                    [](int64_t) { return true; }, [](int64_t j) { return j; }, N, N,
                                    rt * kLayoutTile, ct * kLayoutTile, g32 + 2 * n3 + i * NN, N, tile);
        return;
    }
    blk -= n5;
    const int npt = (R.ncol_ph + kLayoutTile - 1) / kLayoutTile;
    if (blk >= nt * npt) return;
    // block 4: out[c][k] = V(k, i, j) for the representative ph columns c = (i, j)
    const int rt = blk % nt, pt = blk / nt;
    layout_transpose_gen<float>(
        [&](int k, int64_t pos) {
            const int c = R.cperm_ph[pos], i = c / N;   // c < N^2: 32-bit division
            return R.at(N, k, i, c - i * N);
        },
        [](int64_t) { return true; }, [&](int64_t pos) { return static_cast<int64_t>(R.cperm_ph[pos]); }, N,
        R.ncol_ph, rt * kLayoutTile, pt * kLayoutTile, g32 + n3, N, tile);
}

__global__ __launch_bounds__(256) void layout_split_red_kernel(RedSrc R, int N, uint16_t *__restrict__ ahl,
                                                               float *__restrict__ g32) {
    const int64_t n3 = static_cast<int64_t>(N) * N * N;
    __shared__ LayoutTile tile[kLayoutTile];
    layout_block_red(R, N, n3, blockIdx.x, ahl, g32, tile);
}

__global__ __launch_bounds__(256) void layout_split_kernel(const double *__restrict__ V, int N,
                                                           uint16_t *__restrict__ ahl, float *__restrict__ g32) {
    const int64_t n3 = static_cast<int64_t>(N) * N * N;
    __shared__ LayoutTile tile[kLayoutTile];
    layout_block<true>(V, N, n3, blockIdx.x, ahl, g32, nullptr, tile);
}

// The channel partials are stored per column tile position, [p][m], so each
// channel sees F through its own index frame.  A block assembles an 8 x 8 x 32
// cube (j1, j2, j3) of F in LDS, reading each channel along its contiguous
// index: pp along j3 (32 values), phc along j1 and phd along j2 (8 values).
constexpr int CB_J = 8, CB_K = 32, CB_P = CB_K + 1;

int combine_tiles_of(int N) {
    const int nj = (N + CB_J - 1) / CB_J, nk = (N + CB_K - 1) / CB_K;
    return nj * nj * nk;
}

template <typename PT>
__device__ void combine_body(int N, int KS, int64_t n3, const PT *__restrict__ Cpp,
                             const PT *__restrict__ Cc, const PT *__restrict__ Cd,
                             const int32_t *__restrict__ ppos, const int32_t *__restrict__ phpos,
                             const int16_t *__restrict__ perm8, double scale, double *__restrict__ F, int tile,
                             double *sF) {
    // channel value at column map entry cm and free index m
    auto at_of = [&](int32_t cm, int m) -> int64_t {
        return static_cast<int64_t>(cm >> 3) * N + perm8[(cm & 7) * N + m];
    };
    const int nj = (N + CB_J - 1) / CB_J, nk = (N + CB_K - 1) / CB_K;
    const int t3 = tile % nk, t2 = (tile / nk) % nj, t1 = tile / (nk * nj);
    const int a0 = t1 * CB_J, b0 = t2 * CB_J, c0 = t3 * CB_K;
    constexpr int NE = CB_J * CB_J * CB_K;
    // pp: lanes along j3
    for (int e = threadIdx.x; e < NE; e += blockDim.x) {
        const int i3 = e % CB_K, i2 = (e / CB_K) % CB_J, i1 = e / (CB_K * CB_J);
        const int j1 = a0 + i1, j2 = b0 + i2, j3 = c0 + i3;
        if (j1 >= N || j2 >= N || j3 >= N) continue;
        const int64_t at = at_of(ppos[j1 * N + j2], j3);
        double v = 0.0;
        for (int s = 0; s < KS; ++s) v += Cpp[s * n3 + at];
        sF[(i1 * CB_J + i2) * CB_P + i3] = -v;
    }
    __syncthreads();
    // phc: m = j1, column (j2, j3); lanes along j1
    for (int e = threadIdx.x; e < NE; e += blockDim.x) {
        const int i1 = e % CB_J, i3 = (e / CB_J) % CB_K, i2 = e / (CB_J * CB_K);
        const int j1 = a0 + i1, j2 = b0 + i2, j3 = c0 + i3;
        if (j1 >= N || j2 >= N || j3 >= N) continue;
        const int64_t at = at_of(phpos[j2 * N + j3], j1);
        double v = 0.0;
        for (int s = 0; s < KS; ++s) v += Cc[s * n3 + at];
        sF[(i1 * CB_J + i2) * CB_P + i3] += v;
    }
    __syncthreads();
    // phd: m = j2, column (j1, j3); lanes along j2
    for (int e = threadIdx.x; e < NE; e += blockDim.x) {
        const int i2 = e % CB_J, i3 = (e / CB_J) % CB_K, i1 = e / (CB_J * CB_K);
        const int j1 = a0 + i1, j2 = b0 + i2, j3 = c0 + i3;
        if (j1 >= N || j2 >= N || j3 >= N) continue;
        const int64_t at = at_of(phpos[j1 * N + j3], j2);
        double v = 0.0;
        for (int s = 0; s < KS; ++s) v += Cd[s * n3 + at];
        sF[(i1 * CB_J + i2) * CB_P + i3] += v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NE; e += blockDim.x) {
        const int i3 = e % CB_K, i2 = (e / CB_K) % CB_J, i1 = e / (CB_K * CB_J);
        const int j1 = a0 + i1, j2 = b0 + i2, j3 = c0 + i3;
        if (j1 >= N || j2 >= N || j3 >= N) continue;
        F[(static_cast<int64_t>(j1) * N + j2) * N + j3] = scale * sF[(i1 * CB_J + i2) * CB_P + i3];
    }
}

// Reduced flow state of the symmetric-vertex mode: entry i = pos * N + m holds
// V(c, m) for the representative pp column c = cperm[pos] = j1 N + j2 (the
// column tile order of the orbit columns); any column follows from
//   V(c, m) = Vr[(cmap[c] >> 3) N + perm8[cmap[c] & 7][m]],
// the relation the channel values of those columns obey.  Indices fit 32 bits
// (N^3 <= 2^24), so the divisions by N are 32-bit ones.
__device__ __forceinline__ double vred_at(const double *__restrict__ Vr, int N, const int32_t *__restrict__ cmap,
                                          const int16_t *__restrict__ perm8, int64_t i) {
    const uint32_t ii = static_cast<uint32_t>(i), c = ii / static_cast<uint32_t>(N);
    const int32_t cm = cmap[c];
    (void)perm8;
    return Vr[(cm >> 3) * N + c4v_patch(cm & 7, static_cast<int>(ii - c * N), N)];
}
__device__ __forceinline__ double vred_gather_at(const double *__restrict__ V, int N,
                                                 const int32_t *__restrict__ cperm, int64_t i) {
    const uint32_t ii = static_cast<uint32_t>(i), pos = ii / static_cast<uint32_t>(N);
    return V[static_cast<uint32_t>(cperm[pos]) * N + (ii - pos * N)];
}
// -Cpp + Cc + Cd at reduced entry i (the same sums, in the same order, as the
// full assembly above; the pp value is the stored column itself)
__device__ __forceinline__ double combine_red_at(int N, const double *__restrict__ Cpp,
                                                 const double *__restrict__ Cc, const double *__restrict__ Cd,
                                                 const int32_t *__restrict__ cperm, const int32_t *__restrict__ phpos,
                                                 const int16_t *__restrict__ perm8, int64_t i) {
    const uint32_t ii = static_cast<uint32_t>(i), pos = ii / static_cast<uint32_t>(N);
    const int j3 = static_cast<int>(ii - pos * N);
    const int c = cperm[pos], j1 = c / N, j2 = c - j1 * N;
    (void)perm8;
    auto at_of = [&](int32_t cm, int m) -> int64_t {
        return static_cast<int64_t>(cm >> 3) * N + c4v_patch(cm & 7, m, N);
    };
    double v = -Cpp[i];
    v += Cc[at_of(phpos[j2 * N + j3], j1)];
    v += Cd[at_of(phpos[j1 * N + j3], j2)];
    return v;
}

__global__ __launch_bounds__(256) void vred_gather_kernel(const double *__restrict__ V, int N,
                                                          const int32_t *__restrict__ cperm, int64_t nst,
                                                          double *__restrict__ Vr) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nst) Vr[i] = vred_gather_at(V, N, cperm, i);
}

// gate: when given, only accepted steps (state slot 23) write
__global__ __launch_bounds__(256) void vred_expand_kernel(const double *__restrict__ Vr, int N,
                                                          const int32_t *__restrict__ cmap,
                                                          const int16_t *__restrict__ perm8, int64_t n3,
                                                          const double *gate, double *__restrict__ V) {
    if (gate && gate[23] == 0.0) return;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n3) V[i] = vred_at(Vr, N, cmap, perm8, i);
}

__global__ __launch_bounds__(256) void combine_red_kernel(const double *__restrict__ Cs, int64_t cs, int N,
                                                          int64_t nst, const int32_t *__restrict__ cperm,
                                                          const int32_t *__restrict__ phpos,
                                                          const int16_t *__restrict__ perm8,
                                                          const double *__restrict__ Tdev, int scale_by_T,
                                                          double *__restrict__ F) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nst) return;
    const double scale = scale_by_T ? Tdev[0] : 1.0;
    F[i] = scale * combine_red_at(N, Cs, Cs + cs, Cs + 2 * cs, cperm, phpos, perm8, i);
}

// Sum of the K-part partials, four consecutive elements per thread (streams
// of contiguous loads, one per part).
template <typename PT>
__device__ __forceinline__ void sum_parts_body(const double *__restrict__ C, int KS, int64_t cs, int64_t nel,
                                               double *__restrict__ out, int64_t q) {
    // q runs over [3][nel / 4] quads (nel % 4 == 0: nel = ncol * N, N % 4 == 0)
    const int64_t qpt = nel / 4;
    if (q >= 3 * qpt) return;
    // q < 3 N^3 / 4 < 2^24: a 32-bit division
    const uint32_t q32 = static_cast<uint32_t>(q), qpt32 = static_cast<uint32_t>(qpt);
    const int t = static_cast<int>(q32 / qpt32);
    const int64_t i = 4 * static_cast<int64_t>(q32 - static_cast<uint32_t>(t) * qpt32);
    const PT *Ct = reinterpret_cast<const PT *>(C + t * static_cast<int64_t>(KS) * cs);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < KS; ++s) {
        const PT *src = Ct + s * cs + i;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] += static_cast<double>(src[e]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) out[t * cs + i + e] = v[e];
}

template <typename PT>
__global__ __launch_bounds__(256) void sum_parts_kernel(const double *__restrict__ C, int KS, int64_t cs,
                                                        int64_t nel, double *__restrict__ out) {
    sum_parts_body<PT>(C, KS, cs, nel, out, static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x);
}

// V(g j1, g j2, g j3) - V(j1, j2, j3) over the seven non-trivial C4v elements:
// per block the largest deviation and the largest |V| (fixed-order host max)
constexpr int kVsymBlocks = 1024;
__global__ __launch_bounds__(256) void vsym_check_kernel(const double *__restrict__ V, int N,
                                                         const int16_t *__restrict__ perm8,
                                                         double *__restrict__ partials) {
    __shared__ double sd[256], sv[256];
    const int64_t n3 = static_cast<int64_t>(N) * N * N;
    double dev = 0.0, vmax = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n3;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int j3 = static_cast<int>(i % N), j2 = static_cast<int>((i / N) % N);
        const int j1 = static_cast<int>(i / (static_cast<int64_t>(N) * N));
        const double v = V[i];
        vmax = fmax(vmax, fabs(v));
        for (int o = 1; o < 8; ++o) {
            const int64_t k = (static_cast<int64_t>(perm8[o * N + j1]) * N + perm8[o * N + j2]) * N +
                              perm8[o * N + j3];
            dev = fmax(dev, fabs(V[k] - v));
        }
    }
    sd[threadIdx.x] = dev;
    sv[threadIdx.x] = vmax;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + w]);
            sv[threadIdx.x] = fmax(sv[threadIdx.x], sv[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = sd[0];
        partials[gridDim.x + blockIdx.x] = sv[0];
    }
}

template <typename PT>
__global__ __launch_bounds__(256) void combine_kernel(const PT *__restrict__ Cpp,
                                                      const PT *__restrict__ Cc,
                                                      const PT *__restrict__ Cd, int N, int parts,
                                                      const int32_t *__restrict__ ppos,
                                                      const int32_t *__restrict__ phpos,
                                                      const int16_t *__restrict__ perm8,
                                                      const double *__restrict__ Tdev, int scale_by_T,
                                                      double *__restrict__ F) {
    __shared__ double sF[CB_J * CB_J * CB_P];
    const int64_t n3 = static_cast<int64_t>(N) * N * N;
    combine_body(N, parts, n3, Cpp, Cc, Cd, ppos, phpos, perm8, scale_by_T ? Tdev[0] : 1.0, F, blockIdx.x, sF);
}

// ----------------------------------------------------------------- RK
__global__ void rk_stage_kernel(RkStageArgs a) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const double h = a.state[FRG_ST_H];
    double acc = 0.0;
    for (int j = 0; j < a.nk; ++j)
        if (a.coef[j] != 0.0) acc += a.coef[j] * a.k[j][i];
    a.out[i] = a.y[i] + h * acc;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = (o > v || o != o) ? o : v;   // propagate NaN
    }
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) {
            const double o = sh[w];
            v = (o > v || o != o) ? o : v;
        }
    }
    return v;
}

struct ErrArgs {
    int64_t n;
    const double *y, *y5;
    const double *k[7];
    double e[7];
    double rtol, atol;
    const double *state;
    double *partial;
};

__global__ void dp_error_partial(ErrArgs a) {
    __shared__ double sh[2][16];
    const double h = a.state[FRG_ST_H];
    double emax = 0.0, vmax = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double d = 0.0;
#pragma unroll
        for (int j = 0; j < 7; ++j) d += a.e[j] * a.k[j][i];
        d = fabs(h * d);
        const double y5 = a.y5[i];
        const double sc = a.atol + a.rtol * fmax(fabs(a.y[i]), fabs(y5));
        const double q = d / sc;
        emax = (q > emax || q != q) ? q : emax;
        const double av = fabs(y5);
        vmax = (av > vmax || av != av) ? av : vmax;
    }
    emax = block_max(emax, sh[0]);
    vmax = block_max(vmax, sh[1]);
    if (threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = emax;
        a.partial[2 * blockIdx.x + 1] = vmax;
    }
}

__global__ void maxabs_partial(int64_t n, const double *__restrict__ y, double *partial) {
    __shared__ double sh[16];
    double vmax = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double av = fabs(y[i]);
        vmax = (av > vmax || av != av) ? av : vmax;
    }
    vmax = block_max(vmax, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = 0.0;
        partial[2 * blockIdx.x + 1] = vmax;
    }
}

// final reduction of the partials: error norm into state[slot_e] (if >= 0),
// max|y| into state[slot_v]; fixed order, so the result is deterministic
// the largest (error, |y|) partials, NaN-propagating, by one wave: lane l takes
// blocks l, l + 64, ..., then a butterfly.  A maximum is exact, so the result
// is the same for any order of the partials.
__device__ __forceinline__ void wave_max_partials(const double *partial, int nblocks, double &e, double &v) {
    e = 0.0;
    v = 0.0;
    for (int b = static_cast<int>(threadIdx.x & 63); b < nblocks; b += 64) {
        const double pe = partial[2 * b], pv = partial[2 * b + 1];
        e = (pe > e || pe != pe) ? pe : e;
        v = (pv > v || pv != pv) ? pv : v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double oe = __shfl_xor(e, off, 64), ov = __shfl_xor(v, off, 64);
        e = (oe > e || oe != oe) ? oe : e;
        v = (ov > v || ov != ov) ? ov : v;
    }
}

// launched as one wave
__global__ void reduce_partials(const double *partial, int nblocks, double *state, int slot_e,
                                int slot_v) {
    double e, v;
    wave_max_partials(partial, nblocks, e, v);
    if (threadIdx.x != 0) return;
    if (slot_e >= 0) state[slot_e] = e;
    state[slot_v] = v;
}

__global__ void state_set_kernel(double *state, int slot, double v) {
    if (threadIdx.x == 0) state[slot] = v;
}

// pre-step: clip the step onto s_min (DP54) and remember whether this is the last
__device__ void pre_step_body(double *state, int stepper) {
    if (stepper == FRG_DP54) {
        const double s = state[FRG_ST_S], smin = state[FRG_ST_SMIN];
        double h = state[FRG_ST_H];
        const double dir = state[21];
        state[22] = 0.0;
        if ((s + h - smin) * dir >= 0.0) {
            h = smin - s;
            state[22] = 1.0;
        }
        state[FRG_ST_H] = h;
    }
    state[23] = 0.0;  // accept flag of this attempt
}

__global__ void pre_step_kernel(double *state, int stepper) {
    if (threadIdx.x == 0) pre_step_body(state, stepper);
}

// step control (one thread).  DP54: G10 rules; RK4: fixed step index.
// state slots: 20 max|y_new|, 21 direction, 22 last, 23 accept, 24 m_prev,
// 25 s0, 26 RK4 step index, 27 RK4 step count
__device__ void control_body(double *state, double *log, int log_cap, double vmax,
                             int max_steps, int stepper) {
    if (state[FRG_ST_REASON] != 0.0) { state[23] = 0.0; return; }
    const double mx = state[20];
    const double s = state[FRG_ST_S], h = state[FRG_ST_H];
    int accept;
    double s_new;
    if (stepper == FRG_DP54) {
        const double err = state[FRG_ST_ERR];
        state[FRG_ST_RHS] += 6.0;
        if (!(err == err) || !(mx == mx) || isinf(err) || isinf(mx)) {
            state[FRG_ST_REASON] = FRG_STOP_NONFINITE;
            state[23] = 0.0;
            return;
        }
        double fac = err == 0.0 ? 5.0 : 0.9 * pow(err, -0.2);
        fac = fac < 0.2 ? 0.2 : (fac > 5.0 ? 5.0 : fac);
        accept = err <= 1.0;
        s_new = state[22] != 0.0 ? state[FRG_ST_SMIN] : s + h;
        if (!accept) {
            state[FRG_ST_REJECTED] += 1.0;
            state[FRG_ST_H] = h * fac;
            state[23] = 0.0;
            if (!(fabs(h * fac) > 1e-14 * (1.0 + fabs(s)))) state[FRG_ST_REASON] = FRG_STOP_HMIN;
            return;
        }
        state[FRG_ST_H] = h * fac;
    } else {
        state[FRG_ST_RHS] += 4.0;
        if (!(mx == mx) || isinf(mx)) {
            state[FRG_ST_REASON] = FRG_STOP_NONFINITE;
            state[23] = 0.0;
            return;
        }
        accept = 1;
        const double idx = state[26] + 1.0;
        state[26] = idx;
        s_new = state[25] + idx * h;
    }
    state[23] = 1.0;
    state[FRG_ST_ACCEPTED] += 1.0;
    if (state[FRG_ST_ACCEPTED] == 1.0) state[FRG_ST_FIRST_RHS] = state[FRG_ST_RHS];
    const double s_prev = s, m_prev = state[24];
    state[FRG_ST_S] = s_new;
    state[FRG_ST_VMAX] = mx;
    double reason = 0.0;
    if (mx > vmax) {
        reason = FRG_STOP_DIVERGED;
        state[FRG_ST_SC] = s_new;
        state[FRG_ST_SC_INTERP] = s_prev + (vmax - m_prev) / (mx - m_prev) * (s_new - s_prev);
    } else if (stepper == FRG_DP54 ? state[22] != 0.0 : state[26] >= state[27]) {
        reason = FRG_STOP_TMIN;
    } else if (max_steps > 0 && state[FRG_ST_ACCEPTED] >= max_steps) {
        reason = FRG_STOP_MAXSTEPS;
    }
    state[24] = mx;
    state[FRG_ST_REASON] = reason;
    const int row = static_cast<int>(state[FRG_ST_ACCEPTED]) - 1;
    if (log && row < log_cap) {
        double *L = log + 8 * row;
        L[0] = s_new; L[1] = h; L[2] = state[FRG_ST_ERR]; L[3] = mx;
        L[4] = state[FRG_ST_RHS]; L[5] = state[FRG_ST_REJECTED]; L[6] = state[FRG_ST_ACCEPTED];
        L[7] = reason;
    }
}

__global__ void control_kernel(double *state, double *log, int log_cap, double vmax,
                               int max_steps, int stepper) {
    if (threadIdx.x == 0) control_body(state, log, log_cap, vmax, max_steps, stepper);
}

__global__ void accept_copy_kernel(int64_t n, const double *state, const double *__restrict__ src,
                                   double *__restrict__ dst) {
    if (state && state[23] == 0.0) return;   // no state: copy unconditionally
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void state_init_kernel(double *state, double s0, double h, double s_min) {
    if (threadIdx.x != 0) return;
    for (int i = 0; i < FRG_STATE_LEN; ++i) state[i] = 0.0;
    state[FRG_ST_S] = s0;
    state[FRG_ST_H] = h;
    state[FRG_ST_SMIN] = s_min;
    state[FRG_ST_SC] = NAN;
    state[FRG_ST_SC_INTERP] = NAN;
    state[21] = (s_min < s0) ? -1.0 : 1.0;
    state[25] = s0;
}


// ----------------------------------------------------------------- batched (work list of (flow, block))
__device__ __forceinline__ bool flow_stopped(const FlowArgs &f) { return f.state[FRG_ST_REASON] != 0.0; }

__global__ void prep_b_kernel(const FlowArgs *__restrict__ fa, const int2 *__restrict__ items,
                              double c_stage, int split) {
    const int2 it = items[blockIdx.x];
    const FlowArgs &f = fa[it.x];
    if (flow_stopped(f)) return;
    const double T = exp(f.state[FRG_ST_S] + c_stage * f.state[FRG_ST_H]);
    const double inv2T = 0.5 / T;
    const int i = it.y * blockDim.x + threadIdx.x;
    if (i == 0) {
        f.Tdev[0] = T;
        f.Tdev[1] = inv2T;
    }
    if (i >= f.np) return;
    const double a = f.xi[i] * inv2T;
    const double ha = a * sech2_d(a);
    const double wf = -f.w[i] / (4.0 * T * T);
    if (split) {
        f.pa32[i] = static_cast<float>(a);
        f.pa32[f.np + i] = static_cast<float>(ha);
        f.pa32[2 * f.np + i] = static_cast<float>(wf);
    } else {
        f.pa64[i] = a;
        f.pa64[f.np + i] = ha;
        f.pa64[2 * f.np + i] = wf;
    }
}

__device__ __forceinline__ const double *src_of(const FlowArgs &f, int src) {
    return src == SRC_V ? f.V : (src == SRC_YT ? f.yt : f.y5);
}

// items: (flow, block of that flow's layout pass)
__global__ __launch_bounds__(256) void layout_b_kernel(const FlowArgs *__restrict__ fa,
                                                       const int2 *__restrict__ items, int src, int split) {
    __shared__ LayoutTile tile[kLayoutTile];
    const int2 it = items[blockIdx.x];
    const FlowArgs &f = fa[it.x];
    if (flow_stopped(f)) return;
    if (!split) {
        layout_block<false>(src_of(f, src), f.N, f.n3, it.y, nullptr, nullptr, f.perm, tile);
    } else if (f.red && src != SRC_V) {   // straight from the reduced stage vector
        const RedSrc R{src == SRC_YT ? f.ytr : f.y5r, f.ppos, f.cperm_ph, f.ncol_ph};
        layout_block_red(R, f.N, f.n3, it.y, f.ahl, f.g32, tile);
    } else {
        layout_block<true>(src_of(f, src), f.N, f.n3, it.y, f.ahl, f.g32, nullptr, tile);
    }
}

__global__ __launch_bounds__(256) void combine_b_kernel(const FlowArgs *__restrict__ fa,
                                                        const int2 *__restrict__ items, int stage) {
    __shared__ double sF[CB_J * CB_J * CB_P];
    const int2 it = items[blockIdx.x];
    const FlowArgs &f = fa[it.x];
    if (flow_stopped(f)) return;
    const int64_t n = f.n3;
    if (f.red) {   // item = block of 256 reduced entries
        const int64_t i = static_cast<int64_t>(it.y) * blockDim.x + threadIdx.x;
        if (i < f.nst)
            f.k[stage][i] = f.Tdev[0] * combine_red_at(f.N, f.Csum, f.Csum + f.cs, f.Csum + 2 * f.cs, f.cperm_pp,
                                                       f.phpos, f.perm8, i);
        return;
    }
    combine_body(f.N, 1, n, static_cast<const double *>(f.Csum), f.Csum + f.cs, f.Csum + 2 * f.cs, f.ppos, f.phpos,
                 f.perm8, f.Tdev[0], f.k[stage], it.y, sF);
}

// batched sum of the K parts: item = (flow, block of kSumPartsPerBlock elements)
__global__ __launch_bounds__(256) void sum_parts_b_kernel(const FlowArgs *__restrict__ fa,
                                                          const int2 *__restrict__ items) {
    const int2 it = items[blockIdx.x];
    const FlowArgs &f = fa[it.x];
    if (flow_stopped(f)) return;
    const int64_t q = static_cast<int64_t>(it.y) * (kSumPartsPerBlock / 4) + threadIdx.x;
    if (f.f32parts) sum_parts_body<float>(f.C, f.KS, f.cs, f.nel, f.Csum, q);
    else sum_parts_body<double>(f.C, f.KS, f.cs, f.nel, f.Csum, q);
}

struct Coef7 { double c[7]; };

__global__ void rk_stage_b_kernel(const FlowArgs *__restrict__ fa, const int2 *__restrict__ items,
                                  Coef7 coef, int nk, int dst) {
    const int2 it = items[blockIdx.x];
    const FlowArgs &f = fa[it.x];
    if (flow_stopped(f)) return;
    const int64_t i = static_cast<int64_t>(it.y) * blockDim.x + threadIdx.x;
    if (i >= (f.red ? f.nst : f.n3)) return;
    const double h = f.state[FRG_ST_H];
    double acc = 0.0;
    for (int j = 0; j < nk; ++j)
        if (coef.c[j] != 0.0) acc += coef.c[j] * f.k[j][i];
    double *out = dst == SRC_YT ? (f.red ? f.ytr : f.yt) : (f.red ? f.y5r : f.y5);
    out[i] = (f.red ? f.yr : f.V)[i] + h * acc;
}

// reduced flows: y <- the representative entries of V (step start), or the full
// rhs input yt / y5 <- the expansion of its reduced stage vector
__global__ __launch_bounds__(256) void vred_b_kernel(const FlowArgs *__restrict__ fa, const int2 *__restrict__ items,
                                                     int dst) {
    const int2 it = items[blockIdx.x];
    const FlowArgs &f = fa[it.x];
    if (!f.red || flow_stopped(f)) return;
    const int64_t i = static_cast<int64_t>(it.y) * blockDim.x + threadIdx.x;
    if (dst == SRC_V) {
        if (i < f.nst) f.yr[i] = vred_gather_at(f.V, f.N, f.cperm_pp, i);
    } else if (i < f.n3) {
        (dst == SRC_YT ? f.yt : f.y5)[i] = vred_at(dst == SRC_YT ? f.ytr : f.y5r, f.N, f.ppos, f.perm8, i);
    }
}

// error norm partials: item block it.y of flow it.x covers a grid-stride slice
__global__ void dp_error_b_kernel(const FlowArgs *__restrict__ fa, const int2 *__restrict__ items,
                                  Coef7 e, double rtol, double atol) {
    __shared__ double sh[2][16];
    const int2 it = items[blockIdx.x];
    const FlowArgs &f = fa[it.x];
    if (flow_stopped(f)) return;
    const double h = f.state[FRG_ST_H];
    double emax = 0.0, vmax = 0.0;
    const int64_t n = f.red ? f.nst : f.n3;
    const double *yv = f.red ? f.yr : f.V, *y5v = f.red ? f.y5r : f.y5;
    for (int64_t i = static_cast<int64_t>(it.y) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(f.nred) * blockDim.x) {
        double d = 0.0;
#pragma unroll
        for (int j = 0; j < 7; ++j) d += e.c[j] * f.k[j][i];
        d = fabs(h * d);
        const double y5 = y5v[i];
        const double q = d / (atol + rtol * fmax(fabs(yv[i]), fabs(y5)));
        emax = (q > emax || q != q) ? q : emax;
        const double av = fabs(y5);
        vmax = (av > vmax || av != av) ? av : vmax;
    }
    emax = block_max(emax, sh[0]);
    vmax = block_max(vmax, sh[1]);
    if (threadIdx.x == 0) {
        f.partial[2 * it.y] = emax;
        f.partial[2 * it.y + 1] = vmax;
    }
}

// one wave per flow: the error norm and max|y5| from the flow's partials
__global__ void reduce_partials_b_kernel(const FlowArgs *__restrict__ fa) {
    const FlowArgs &f = fa[blockIdx.x];
    if (flow_stopped(f)) return;
    double e, v;
    wave_max_partials(f.partial, f.nred, e, v);
    if (threadIdx.x != 0) return;
    f.state[FRG_ST_ERR] = e;
    f.state[20] = v;
}

// one thread per flow: phase 1 = pre-step, 2 = step control (the error partials
// are reduced by reduce_partials_b_kernel)
__global__ void step_ctl_b_kernel(const FlowArgs *__restrict__ fa, int nflows, int phase, double *log_base,
                                  int log_cap, double vmax, int max_steps) {
    const int fl = blockIdx.x * blockDim.x + threadIdx.x;
    if (fl >= nflows) return;
    const FlowArgs &f = fa[fl];
    if (phase == 1) {
        if (flow_stopped(f)) return;
        pre_step_body(f.state, FRG_DP54);
    } else {
        control_body(f.state, log_base ? log_base + static_cast<size_t>(fl) * 8 * log_cap : nullptr,
                     log_cap, vmax, max_steps, FRG_DP54);
    }
}

// accepted steps: V <- y5 and the first stage <- last stage (FSAL)
__global__ void accept_b_kernel(const FlowArgs *__restrict__ fa, const int2 *__restrict__ items) {
    const int2 it = items[blockIdx.x];
    const FlowArgs &f = fa[it.x];
    if (f.state[23] == 0.0) return;
    const int64_t i = static_cast<int64_t>(it.y) * blockDim.x + threadIdx.x;
    if (i >= f.n3) return;
    if (f.red) {
        f.V[i] = vred_at(f.y5r, f.N, f.ppos, f.perm8, i);
        if (i < f.nst) f.k[0][i] = f.k[6][i];
        return;
    }
    f.V[i] = f.y5[i];
    f.k[0][i] = f.k[6][i];
}

inline unsigned blocks_for(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

}  // namespace

void launch_bins(const double *bnd, const double *px, const double *py, const double *qrow,
                 int N, int n_rad, int n_ang, int Tpp, int Trows, uint8_t *bins, hipStream_t s) {
    const int np = N * n_rad * n_ang;
    dim3 grid(blocks_for(np, 256), Trows < 65535 ? Trows : 65535);
    hipLaunchKernelGGL(bins_kernel, grid, dim3(256), 0, s, bnd, px, py, qrow, N, n_rad, n_ang, Tpp, Trows,
                       bins);
}

void launch_bins_export(const uint8_t *bins, int N, int n_rad, int n_ang, int r0, int nrows, uint8_t *out,
                        hipStream_t s) {
    const int np = N * n_rad * n_ang;
    if (nrows <= 0) return;
    dim3 grid(blocks_for(np, 256), nrows < 65535 ? nrows : 65535);
    hipLaunchKernelGGL(bins_export_kernel, grid, dim3(256), 0, s, bins, N, n_rad, n_ang, r0, nrows, out);
}

void launch_sym_check(const uint8_t *bins, const int32_t *orbit, int N, int n_rad, int n_ang,
                      int Trows, bool rev, int *mismatch, hipStream_t s) {
    const int np = N * n_rad * n_ang;
    dim3 grid(blocks_for(np, 256), Trows < 4096 ? Trows : 4096);
    hipLaunchKernelGGL(sym_check_kernel, grid, dim3(256), 0, s, bins, orbit, N, n_rad, n_ang, Trows, rev,
                       mismatch);
}

void launch_pair_check(const uint8_t *bins, const int32_t *rows_pp, const int32_t *rows_ph, int npairs, int np,
                       int N, int *mismatch, hipStream_t s) {
    if (npairs <= 0) return;
    dim3 grid(blocks_for(np, 256), npairs < 4096 ? npairs : 4096);
    hipLaunchKernelGGL(pair_check_kernel, grid, dim3(256), 0, s, bins, rows_pp, rows_ph, npairs, np, N, mismatch);
}

void launch_point_prep(const double *xi, const double *w, int np, double T_host,
                       const double *state, double c_stage, double *pa64, float *pa32,
                       double *Tout, hipStream_t s, const double *sigma, int nf) {
    hipLaunchKernelGGL(point_prep_kernel, dim3(blocks_for(np, 256)), dim3(256), 0, s, xi, w, np,
                       T_host, state, c_stage, pa64, pa32, Tout, sigma, nf);
}

void launch_dsigma(const double *xi, const double *w, int N, int nf, const double *V, const double *S,
                   const double *Tdev, int scale_by_T, double *D, double *dS, hipStream_t s,
                   const int32_t *ppos) {
    hipLaunchKernelGGL(dsigma_patch_kernel, dim3(N), dim3(256), 0, s, xi, w, nf, S, Tdev, D);
    hipLaunchKernelGGL(dsigma_kernel, dim3(N), dim3(256), 0, s, N, V, ppos, D, Tdev, scale_by_T, dS);
}

int layout_blocks(int N) {
    const int nt = layout_t_tiles(N);
    const int64_t NN = static_cast<int64_t>(N) * N;
    return layout_a_blocks(N) + nt * static_cast<int>((NN + kLayoutTile - 1) / kLayoutTile) + N * nt * nt;
}

void launch_layout_f64(const double *V, int N, double *perm, hipStream_t s) {
    hipLaunchKernelGGL(layout_f64_kernel, dim3(layout_blocks(N)), dim3(256), 0, s, V, N, perm);
}

void launch_layout_split_red(const double *Vr, int N, const int32_t *ppos, const int32_t *cperm_ph, int ncol_ph,
                             uint16_t *ahl, float *g32, hipStream_t s) {
    hipLaunchKernelGGL(layout_split_red_kernel, dim3(layout_blocks_red(N, ncol_ph)), dim3(256), 0, s,
                       RedSrc{Vr, ppos, cperm_ph, ncol_ph}, N, ahl, g32);
}

void launch_layout_split(const double *V, int N, uint16_t *ahl, float *g32, hipStream_t s) {
    hipLaunchKernelGGL(layout_split_kernel, dim3(layout_blocks(N)), dim3(256), 0, s, V, N, ahl, g32);
}

int combine_tiles(int N) { return combine_tiles_of(N); }

void launch_combine(const void *Cpp, const void *Cc, const void *Cd, bool f32parts, int N, int parts,
                    const int32_t *ppos, const int32_t *phpos, const int16_t *perm8,
                    const double *Tdev, int scale_by_T, double *F, hipStream_t s) {
    if (f32parts)
        hipLaunchKernelGGL(combine_kernel<float>, dim3(combine_tiles_of(N)), dim3(256), 0, s,
                           static_cast<const float *>(Cpp), static_cast<const float *>(Cc),
                           static_cast<const float *>(Cd), N, parts, ppos, phpos, perm8, Tdev, scale_by_T, F);
    else
        hipLaunchKernelGGL(combine_kernel<double>, dim3(combine_tiles_of(N)), dim3(256), 0, s,
                           static_cast<const double *>(Cpp), static_cast<const double *>(Cc),
                           static_cast<const double *>(Cd), N, parts, ppos, phpos, perm8, Tdev, scale_by_T, F);
}

void launch_rk_stage(const RkStageArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(rk_stage_kernel, dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a);
}

void launch_dp_error(int64_t n, const double *y, const double *y5, const double *const k[7],
                     const double e[7], double rtol, double atol, double *state, double *partial,
                     int nblocks, hipStream_t s) {
    ErrArgs a;
    a.n = n;
    a.y = y;
    a.y5 = y5;
    for (int j = 0; j < 7; ++j) { a.k[j] = k[j]; a.e[j] = e[j]; }
    a.rtol = rtol;
    a.atol = atol;
    a.state = state;
    a.partial = partial;
    hipLaunchKernelGGL(dp_error_partial, dim3(nblocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(64), 0, s, partial, nblocks, state,
                       static_cast<int>(FRG_ST_ERR), 20);
}

void launch_maxabs_to(int64_t n, const double *y, double *state, int slot, double *partial,
                      int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(maxabs_partial, dim3(nblocks), dim3(256), 0, s, n, y, partial);
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(64), 0, s, partial, nblocks, state, -1, slot);
}

void launch_state_set(double *state, int slot, double v, hipStream_t s) {
    hipLaunchKernelGGL(state_set_kernel, dim3(1), dim3(64), 0, s, state, slot, v);
}

void launch_dp_control(double *state, double *log, int log_cap, double vmax, int max_steps,
                       int stepper, hipStream_t s) {
    hipLaunchKernelGGL(control_kernel, dim3(1), dim3(64), 0, s, state, log, log_cap, vmax,
                       max_steps, stepper);
}

void launch_pre_step(double *state, int stepper, hipStream_t s) {
    hipLaunchKernelGGL(pre_step_kernel, dim3(1), dim3(64), 0, s, state, stepper);
}

void launch_vred_gather(const double *V, int N, const int32_t *cperm, int64_t nst, double *Vr, hipStream_t s) {
    hipLaunchKernelGGL(vred_gather_kernel, dim3(blocks_for(nst, 256)), dim3(256), 0, s, V, N, cperm, nst, Vr);
}
void launch_vred_expand(const double *Vr, int N, const int32_t *cmap, const int16_t *perm8, const double *gate,
                        double *V, hipStream_t s) {
    const int64_t n3 = static_cast<int64_t>(N) * N * N;
    hipLaunchKernelGGL(vred_expand_kernel, dim3(blocks_for(n3, 256)), dim3(256), 0, s, Vr, N, cmap, perm8, n3,
                       gate, V);
}
void launch_combine_red(const double *Cs, int64_t cs, int N, int64_t nst, const int32_t *cperm,
                        const int32_t *phpos, const int16_t *perm8, const double *Tdev, int scale_by_T, double *F,
                        hipStream_t s) {
    hipLaunchKernelGGL(combine_red_kernel, dim3(blocks_for(nst, 256)), dim3(256), 0, s, Cs, cs, N, nst, cperm,
                       phpos, perm8, Tdev, scale_by_T, F);
}
void launch_vred_b(const FlowArgs *fa, const int2 *items, int nitems, int dst, hipStream_t s) {
    if (nitems > 0) hipLaunchKernelGGL(vred_b_kernel, dim3(nitems), dim3(256), 0, s, fa, items, dst);
}

void launch_accept_copy(int64_t n, const double *state, const double *src, double *dst,
                        hipStream_t s) {
    hipLaunchKernelGGL(accept_copy_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, state,
                       src, dst);
}

void launch_prep_b(const FlowArgs *fa, const int2 *items, int nitems, double c_stage, bool split,
                   hipStream_t s) {
    hipLaunchKernelGGL(prep_b_kernel, dim3(nitems), dim3(256), 0, s, fa, items, c_stage, split ? 1 : 0);
}
void launch_layout_b(const FlowArgs *fa, const int2 *items, int nitems, int src, bool split,
                     hipStream_t s) {
    hipLaunchKernelGGL(layout_b_kernel, dim3(nitems), dim3(256), 0, s, fa, items, src, split ? 1 : 0);
}
void launch_sum_parts(const double *C, bool f32parts, int KS, int64_t cs, int64_t nel, double *out,
                      hipStream_t s) {
    const int64_t quads = 3 * (nel / 4);
    if (f32parts)
        hipLaunchKernelGGL(sum_parts_kernel<float>, dim3(blocks_for(quads, 256)), dim3(256), 0, s, C, KS, cs, nel,
                           out);
    else
        hipLaunchKernelGGL(sum_parts_kernel<double>, dim3(blocks_for(quads, 256)), dim3(256), 0, s, C, KS, cs, nel,
                           out);
}

int vsym_check_blocks(int N) {
    const int64_t n3 = static_cast<int64_t>(N) * N * N;
    return static_cast<int>(std::min<int64_t>(kVsymBlocks, (n3 + 255) / 256));
}

void launch_vsym_check(const double *V, int N, const int16_t *perm8, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(vsym_check_kernel, dim3(vsym_check_blocks(N)), dim3(256), 0, s, V, N, perm8, partials);
}

void launch_sum_parts_b(const FlowArgs *fa, const int2 *items, int nitems, hipStream_t s) {
    hipLaunchKernelGGL(sum_parts_b_kernel, dim3(nitems), dim3(kSumPartsPerBlock / 4), 0, s, fa, items);
}

void launch_combine_b(const FlowArgs *fa, const int2 *items, int nitems, int stage, hipStream_t s) {
    hipLaunchKernelGGL(combine_b_kernel, dim3(nitems), dim3(256), 0, s, fa, items, stage);
}
void launch_rk_stage_b(const FlowArgs *fa, const int2 *items, int nitems, const double coef[7],
                       int nk, int dst, hipStream_t s) {
    Coef7 c;
    for (int j = 0; j < 7; ++j) c.c[j] = coef[j];
    hipLaunchKernelGGL(rk_stage_b_kernel, dim3(nitems), dim3(256), 0, s, fa, items, c, nk, dst);
}
void launch_dp_error_b(const FlowArgs *fa, const int2 *items, int nitems, int nflows,
                       const double e[7], double rtol, double atol, hipStream_t s) {
    Coef7 c;
    for (int j = 0; j < 7; ++j) c.c[j] = e[j];
    hipLaunchKernelGGL(dp_error_b_kernel, dim3(nitems), dim3(256), 0, s, fa, items, c, rtol, atol);
    hipLaunchKernelGGL(reduce_partials_b_kernel, dim3(nflows), dim3(64), 0, s, fa);
}
void launch_step_ctl_b(const FlowArgs *fa, int nflows, int phase, double *log_base, int log_cap,
                       double vmax, int max_steps, hipStream_t s) {
    hipLaunchKernelGGL(step_ctl_b_kernel, dim3(blocks_for(nflows, 64)), dim3(64), 0, s, fa, nflows, phase,
                       log_base, log_cap, vmax, max_steps);
}
void launch_accept_b(const FlowArgs *fa, const int2 *items, int nitems, hipStream_t s) {
    hipLaunchKernelGGL(accept_b_kernel, dim3(nitems), dim3(256), 0, s, fa, items);
}

void launch_state_init(double *state, double s0, double h, double s_min, hipStream_t s) {
    hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, state, s0, h, s_min);
}

// ----------------------------------------------------------------- static scratch
// Workspace of frg_rhs_noalloc: a file-scope device array, so that callers that
// cannot allocate (code under graph capture, tight serving loops) get an rhs
// without hipMalloc.  Every device the library runs on holds its own copy from
// the load of the code object until the process ends.  In host code the name
// is only a stand-in: kernels receive the device address that
// hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void **out) {
    static std::mutex mu;
    static std::vector<void *> addr;   // per device
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if (static_cast<int>(addr.size()) <= dev) addr.resize(static_cast<size_t>(dev) + 1, nullptr);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace frg
