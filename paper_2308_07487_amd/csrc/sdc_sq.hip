// q-resolved dynamic structure factor, Eq. (3), at arbitrary wave vectors for
// any point set (lattice or not), on gfx950.
//
// The phase of a pair factorises, exp(-i q.(r_j - r_i)) = conj(e_i) e_j with
// e_j(q) = exp(-i q.r_j), so the double sum over pairs in Eq. (3) becomes
//     S(q, t) = (1 / (N n_o)) sum_o sum_a conj(F_a(q, o s)) F_a(q, o s + t),
//     F_a(q, f) = sum_j e_j(q) S_j^a(f),
// the dense contraction of the phase matrix [n_q x N] with the spin matrix
// [N x 3T] (FP64 MFMA, phases computed on the fly as in the on-the-fly Q of
// Sec. 3.4 but per site instead of per pair), followed by a short
// correlation over the origins.  The connected form (Eq. (4) with its second
// term, i.e. Eq. (5)) centres the origin side: F_a(q, o s) minus its average
// over the origins, which is the transform of the per-site averages.
#include <hip/hip_runtime.h>

#include "sdc_internal.h"

namespace sdc {

typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kSqQ = 16;                    // wave vectors per workgroup (MFMA rows)
constexpr int kSqSites = 32;                // sites per LDS chunk (8 MFMA K-steps of 4)
constexpr int kSqCB = 4;                    // 16-column blocks per wave
constexpr int kSqCols = 4 * kSqCB * 16;     // spin-matrix columns per workgroup
constexpr int kSqRow = kSqCols + 16;        // LDS row pitch (floats), staggers the banks

// One workgroup: 16 wave vectors x 256 columns (f, a) x one range of sites.
// Per chunk of 32 sites the workgroup computes the 512 phases (cos, -sin of
// q.r in FP64) and stages the spins of its columns in LDS; each wave then runs
// 8 K-steps of 4 sites, two FP64 MFMAs (real and imaginary phase rows) per
// 16-column block.  The partial transform of the site range goes to its own
// slice of `part` (no atomics; the slices are summed in a fixed order).
__global__ __launch_bounds__(256) void sq_transform_kernel(SqTransformArgs a) {
    __shared__ double ph[2][kSqSites][kSqQ];
    __shared__ float sb[kSqSites][kSqRow];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q0 = blockIdx.x * kSqQ;
    const int64_t c0 = (int64_t)blockIdx.y * kSqCols;
    const int64_t n_cols = 3 * (int64_t)a.n_frames_used;
    const int64_t jb = (int64_t)blockIdx.z * a.sites_per_split;
    const int64_t je = jb + a.sites_per_split < a.n ? jb + a.sites_per_split : a.n;
    // frames whose three columns meet [c0, c0 + kSqCols)
    const int64_t f_first = c0 / 3;
    const int n_f = (int)((c0 + kSqCols - 1) / 3 - f_first + 1);
    f64x4 acc_re[kSqCB], acc_im[kSqCB];
#pragma unroll
    for (int b = 0; b < kSqCB; ++b) {
        acc_re[b] = f64x4{0.0, 0.0, 0.0, 0.0};
        acc_im[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    for (int64_t j0 = jb; j0 < je; j0 += kSqSites) {
        __syncthreads();  // the previous chunk has been consumed
        for (int e = tid; e < kSqSites * kSqQ; e += 256) {
            const int s = e / kSqQ, qi = e % kSqQ;
            const int64_t j = j0 + s;
            const int qq = q0 + qi;
            double cs = 0.0, sn = 0.0;
            if (j < je && qq < a.n_q) {
                const double th = a.q[3 * qq] * (double)a.pos[3 * j] + a.q[3 * qq + 1] * (double)a.pos[3 * j + 1] +
                                  a.q[3 * qq + 2] * (double)a.pos[3 * j + 2];
                sincos(th, &sn, &cs);
            }
            ph[0][s][qi] = cs;   // Re exp(-i q.r)
            ph[1][s][qi] = -sn;  // Im exp(-i q.r)
        }
        // spins of the chunk: frame-major so that each frame's sites x 3
        // components are one contiguous run of the [T][N][3] array
        for (int e = tid; e < n_f * 3 * kSqSites; e += 256) {
            const int fl = e / (3 * kSqSites);
            const int r = e - fl * 3 * kSqSites;
            const int s = r / 3, al = r - 3 * s;
            const int64_t f = f_first + fl;
            const int64_t c = 3 * f + al - c0;
            if (c < 0 || c >= kSqCols) continue;
            const int64_t j = j0 + s;
            float v = 0.0f;
            if (f < a.n_frames_used && j < je) v = a.frames[(f * a.n + j) * 3 + al];
            sb[s][c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < kSqSites; k4 += 4) {
            // A[i][k] = phase of wave vector i at site k: lane i + 16 k;
            // B[k][c] = spin column c at site k: lane c + 16 k
            const int s = k4 + (lane >> 4);
            const double are = ph[0][s][lane & 15], aim = ph[1][s][lane & 15];
#pragma unroll
            for (int b = 0; b < kSqCB; ++b) {
                const double bv = (double)sb[s][(wave * kSqCB + b) * 16 + (lane & 15)];
                acc_re[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(are, bv, acc_re[b], 0, 0, 0);
                acc_im[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim, bv, acc_im[b], 0, 0, 0);
            }
        }
    }
    // D[i][c] of the FP64 16x16x4 form: lane l, item v holds row 4 v + l / 16
    // of column l % 16 (rows interleave across the lane groups, unlike the
    // FP32 forms)
    double* out = a.part + (int64_t)blockIdx.z * a.n_q * 2 * n_cols;
#pragma unroll
    for (int b = 0; b < kSqCB; ++b) {
        const int64_t c = c0 + (wave * kSqCB + b) * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int qq = q0 + 4 * v + (lane >> 4);
            if (qq < a.n_q && c < n_cols) {
                out[(int64_t)qq * 2 * n_cols + c] = acc_re[b][v];
                out[((int64_t)qq * 2 + 1) * n_cols + c] = acc_im[b][v];
            }
        }
    }
}

// F[q][f][a] = sum over the site ranges of the partial transforms, in range
// order (deterministic), as interleaved (re, im).
__global__ __launch_bounds__(256) void sq_reduce_kernel(SqTransformArgs a, double* __restrict__ F) {
    const int64_t n_cols = 3 * (int64_t)a.n_frames_used;
    const int64_t per = (int64_t)a.n_q * 2 * n_cols;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < per; x += (int64_t)gridDim.x * blockDim.x) {
        double sum = 0.0;
        for (int sp = 0; sp < a.n_split; ++sp) sum += a.part[sp * per + x];
        const int64_t c = x % n_cols, qr = x / n_cols;
        F[((qr >> 1) * n_cols + c) * 2 + (qr & 1)] = sum;
    }
}

// One workgroup per wave vector, one thread per lag:
// raw[q][t] += sum_o sum_a conj(F_a(q, o s) - <F_a>) F_a(q, o s + t), FP64,
// <F_a> the average over the origins in the connected form (else 0).
__global__ __launch_bounds__(256) void sq_corr_kernel(SqCorrArgs a) {
    const int qq = blockIdx.x;
    const double* F = a.F + (int64_t)qq * a.n_cols * 2;
    double mre[3] = {0.0, 0.0, 0.0}, mim[3] = {0.0, 0.0, 0.0};
    if (a.connected) {
        for (int o = 0; o < a.n_origins; ++o)
            for (int al = 0; al < 3; ++al) {
                const int64_t x = ((int64_t)o * a.stride * 3 + al) * 2;
                mre[al] += F[x];
                mim[al] += F[x + 1];
            }
        for (int al = 0; al < 3; ++al) {
            mre[al] /= a.n_origins;
            mim[al] /= a.n_origins;
        }
    }
    for (int t = threadIdx.x; t < a.n_lags; t += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int o = 0; o < a.n_origins; ++o) {
            const int64_t f0 = (int64_t)o * a.stride, f1 = f0 + t;
            for (int al = 0; al < 3; ++al) {
                const double ar = F[(f0 * 3 + al) * 2] - mre[al], ai = F[(f0 * 3 + al) * 2 + 1] - mim[al];
                const double br = F[(f1 * 3 + al) * 2], bi = F[(f1 * 3 + al) * 2 + 1];
                re += ar * br + ai * bi;
                im += ar * bi - ai * br;
            }
        }
        double* r = a.raw + ((int64_t)qq * a.n_lags + t) * 2;
        r[0] += re;
        r[1] += im;
    }
    if (qq == 0 && threadIdx.x == 0) a.n_org[0] += (double)a.n_origins;
}

__global__ __launch_bounds__(256) void sq_norm_kernel(const double* __restrict__ raw, const double* __restrict__ n_org,
                                                      int64_t n_sites, int64_t count, double* __restrict__ sqt) {
    const double d = (double)n_sites * n_org[0];
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < count; x += (int64_t)gridDim.x * blockDim.x)
        sqt[x] = d > 0.0 ? raw[x] / d : 0.0;
}

dim3 sq_transform_grid(int n_q, int n_frames_used, int n_split) {
    const int64_t n_cols = 3 * (int64_t)n_frames_used;
    return dim3((unsigned)((n_q + kSqQ - 1) / kSqQ), (unsigned)((n_cols + kSqCols - 1) / kSqCols),
                (unsigned)n_split);
}

int64_t blocks_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return b > 8192 ? 8192 : (b < 1 ? 1 : b);
}

}  // namespace

int64_t sq_tiles_per_split(int n_q, int n_frames_used) {
    const dim3 g = sq_transform_grid(n_q, n_frames_used, 1);
    return (int64_t)g.x * g.y;
}

int sq_site_chunk() { return kSqSites; }

int launch_sq_transform(const SqTransformArgs& a, double* F, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(sq_transform_kernel, sq_transform_grid(a.n_q, a.n_frames_used, a.n_split), dim3(256), 0, s,
                       a);
    const int64_t per = (int64_t)a.n_q * 2 * 3 * (int64_t)a.n_frames_used;
    hipLaunchKernelGGL(sq_reduce_kernel, dim3((unsigned)blocks_for(per)), dim3(256), 0, s, a, F);
    return (int)hipGetLastError();
}

int launch_sq_corr(const SqCorrArgs& a, void* stream) {
    hipLaunchKernelGGL(sq_corr_kernel, dim3((unsigned)a.n_q), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_sq_finalize(const double* raw, const double* n_org, int64_t n_sites, int n_q, int n_lags, double* sqt,
                       double* sqw, void* stream) {
    const int64_t count = (int64_t)n_q * n_lags * 2;
    hipLaunchKernelGGL(sq_norm_kernel, dim3((unsigned)blocks_for(count)), dim3(256), 0, (hipStream_t)stream, raw,
                       n_org, n_sites, count, sqt);
    const int e = (int)hipGetLastError();
    return e != 0 ? e : launch_sqw(sqt, sqw, n_q, n_lags, stream);
}

}  // namespace sdc
