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

// sin and cos of x in FP64 for |x| < 2^20, without branches: Cody-Waite
// reduction x = k pi/2 + r with pi/2 in two parts (FMA), Taylor polynomials
// of sin r and cos r on |r| <= pi/4 (terms to r^15 and r^16; the first left
// out is below 1e-16), and the quadrant k mod 4 choosing and signing them.
// Absolute error a few 1e-16, a quarter of the library routine's work.
__device__ inline void sincos_small(double x, double* s, double* c) {
    const double two_over_pi = 0x1.45f306dc9c883p-1;
    const double pio2_hi = 0x1.921fb54442d18p+0;   // pi/2 rounded to double
    const double pio2_lo = 0x1.1a62633145c07p-54;  // pi/2 - pio2_hi, rounded
    const double k = rint(x * two_over_pi);
    const double r = fma(-k, pio2_lo, fma(-k, pio2_hi, x));
    const double r2 = r * r;
    double ps = -1.0 / 1307674368000.0;            // -1/15!
    ps = fma(ps, r2, 1.0 / 6227020800.0);          //  1/13!
    ps = fma(ps, r2, -1.0 / 39916800.0);           // -1/11!
    ps = fma(ps, r2, 1.0 / 362880.0);              //  1/9!
    ps = fma(ps, r2, -1.0 / 5040.0);               // -1/7!
    ps = fma(ps, r2, 1.0 / 120.0);                 //  1/5!
    ps = fma(ps, r2, -1.0 / 6.0);                  // -1/3!
    const double sn = fma(ps * r2, r, r);
    double pc = 1.0 / 20922789888000.0;            //  1/16!
    pc = fma(pc, r2, -1.0 / 87178291200.0);        // -1/14!
    pc = fma(pc, r2, 1.0 / 479001600.0);           //  1/12!
    pc = fma(pc, r2, -1.0 / 3628800.0);            // -1/10!
    pc = fma(pc, r2, 1.0 / 40320.0);               //  1/8!
    pc = fma(pc, r2, -1.0 / 720.0);                // -1/6!
    pc = fma(pc, r2, 1.0 / 24.0);                  //  1/4!
    pc = fma(pc, r2, -0.5);                        // -1/2!
    const double cs = fma(pc, r2, 1.0);
    // quadrant: (sin, cos)(k pi/2 + r) = (sn, cs), (cs, -sn), (-sn, -cs), (-cs, sn)
    const int q = (int)((long long)k & 3);
    const double s0 = (q & 1) ? cs : sn;
    const double c0 = (q & 1) ? sn : cs;
    *s = (q & 2) ? -s0 : s0;
    *c = ((q + 1) & 2) ? -c0 : c0;
}

constexpr int kSqQBlocks = 4;               // 16-row wave-vector blocks per workgroup
constexpr int kSqColParts = 3;              // column ranges per wave-vector block
constexpr int kSqWaves = kSqQBlocks * kSqColParts;  // consumer waves (MFMA), three per SIMD
constexpr int kSqProdWaves = 4;             // producer waves, one per SIMD
constexpr int kSqThreads = 64 * (kSqWaves + kSqProdWaves);
constexpr int kSqQ = 16 * kSqQBlocks;       // wave vectors per workgroup
constexpr int kSqSites = 24;                // sites per chunk (6 MFMA K-steps of 4)
constexpr int kSqCB = 12;                   // 16-column blocks per workgroup
constexpr int kSqCBW = kSqCB / kSqColParts;   // 16-column blocks per consumer wave
constexpr int kSqCols = kSqCB * 16;         // 192 spin-matrix columns = 64 whole frames
constexpr int kSqFrames = kSqCols / 3;
constexpr int kSqPitch = 3 * kSqSites + 4;  // LDS doubles per staged frame (padded against bank conflicts)
constexpr int kSqPhBuf = 2 * kSqSites * kSqQ;    // doubles of one phase buffer (cos, -sin)
constexpr int kSqSbBuf = kSqFrames * kSqPitch;   // doubles of one spin buffer
constexpr int kSqLdsBytes = 2 * (kSqPhBuf + kSqSbBuf) * (int)sizeof(double);
static_assert(kSqCols % 3 == 0, "a column range must cover whole frames");
static_assert(kSqCB % kSqColParts == 0 && kSqSites % 4 == 0, "consumer split");
static_assert(kSqLdsBytes <= 160 * 1024, "two chunk buffers must fit in LDS");

constexpr int kSqProducers = 64 * kSqProdWaves;
constexpr int kSqPhPer = kSqSites * kSqQ / kSqProducers;         // phases per producer thread
constexpr int kSqSbPer = kSqFrames * 3 * kSqSites / kSqProducers;  // spin values per producer thread
static_assert(kSqPhPer * kSqProducers == kSqSites * kSqQ && kSqProducers % kSqQ == 0, "phase split");
static_assert(kSqSbPer * kSqProducers == kSqFrames * 3 * kSqSites && kSqSbPer % 2 == 0, "spin split");
static_assert(kSqPitch % 2 == 0, "16-byte LDS rows");

// Producer side: the phases of the 64 wave vectors at the 24 sites of chunk
// j0 and the chunk's spins of 64 frames (one contiguous FP64 block of the
// packed spins) into one buffer.  Producer thread p keeps wave vector p % 64
// (qv, zero past n_q) and takes sites p / 64 + 4 i; every global load of the
// chunk is issued before the first is used.
__device__ __forceinline__ void sq_produce(const SqTransformArgs& a, int ptid, const double (&qv)[3], int64_t f_first,
                                           int64_t j0, int64_t je, double* __restrict__ ph,
                                           double* __restrict__ sb) {
    float px[kSqPhPer], py[kSqPhPer], pz[kSqPhPer];
#pragma unroll
    for (int i = 0; i < kSqPhPer; ++i) {
        const int64_t j = j0 + ptid / kSqQ + (kSqProducers / kSqQ) * i;
        const bool in = j < je;
        px[i] = in ? a.pos[3 * j] : 0.0f;
        py[i] = in ? a.pos[3 * j + 1] : 0.0f;
        pz[i] = in ? a.pos[3 * j + 2] : 0.0f;
    }
    // the chunk's 64 frames x 24 sites x 3 components, as pairs of doubles
    const double2* src =
        (const double2*)(a.packed + ((j0 / kSqSites) * a.t_pad + f_first) * (3 * kSqSites));
    double2 v[kSqSbPer / 2];
#pragma unroll
    for (int i = 0; i < kSqSbPer / 2; ++i) v[i] = src[ptid + kSqProducers * i];
#pragma unroll
    for (int i = 0; i < kSqPhPer; ++i) {
        const int64_t j = j0 + ptid / kSqQ + (kSqProducers / kSqQ) * i;
        double cs = 0.0, sn = 0.0;
        if (j < je) {
            const double th = qv[0] * (double)px[i] + qv[1] * (double)py[i] + qv[2] * (double)pz[i];
            sincos_small(th, &sn, &cs);
        }
        const int e = ptid + kSqProducers * i;  // = site * 64 + wave vector
        ph[e] = cs;                             // Re exp(-i q.r), [site][q]
        ph[kSqSites * kSqQ + e] = -sn;          // Im exp(-i q.r)
    }
#pragma unroll
    for (int i = 0; i < kSqSbPer / 2; ++i) {
        const int e = ptid + kSqProducers * i;  // pair index: frame e / 36, values 2 (e % 36), +1
        const int fl = e / (3 * kSqSites / 2), r = 2 * (e - fl * (3 * kSqSites / 2));
        *(double2*)(sb + fl * kSqPitch + r) = v[i];
    }
}

// Packed spins for the contraction: P[c][f][s][a] = S_j^a(f), j = 24 c + s,
// FP64, zero for sites past N and frames past n_frames_used (t_pad frames
// per chunk, a multiple of 64), so that a block's 64 frames are one
// contiguous block.
__global__ __launch_bounds__(256) void sq_pack_kernel(SqTransformArgs a) {
    const int64_t per_chunk = (int64_t)a.t_pad * 3 * kSqSites;
    const int64_t total = (a.n + kSqSites - 1) / kSqSites * per_chunk;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ch = x / per_chunk, rem = x - ch * per_chunk;
        const int64_t f = rem / (3 * kSqSites);
        const int r = (int)(rem - f * 3 * kSqSites);
        const int64_t j = ch * kSqSites + r / 3;
        a.packed[x] = (f < a.n_frames_used && j < a.n) ? (double)a.frames[(f * a.n + j) * 3 + r % 3] : 0.0;
    }
}

// One workgroup: 64 wave vectors x 192 columns (64 frames x 3 components) x
// one range of sites, in chunks of 24 sites with two LDS buffers.  Four
// producer waves fill the next chunk's buffer (64 x 24 phases, cos and -sin
// of q.r in FP64, and the spins) while twelve consumer waves, three per SIMD so
// that one issues MFMAs while the others wait, run the current chunk:
// consumer w takes wave vectors 16 (w % 4) .. +15 and column blocks
// 4 (w / 4) .. +3 through 6 K-steps of 4 sites, two FP64 MFMAs (real and
// imaginary phase rows) per 16-column block sharing the spin operand.  One
// barrier per chunk.  Spins are read from memory once per 64 wave vectors and
// each phase is computed once per 192 columns (the FP64 vector work of the
// phases takes issue cycles from the FP64 MFMAs).  The
// partial transform of the site range goes to its own slice of `part` (no
// atomics; the slices are summed in a fixed order).
__global__ __launch_bounds__(kSqThreads, 1) void sq_transform_kernel(SqTransformArgs a) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool producer = wave >= kSqWaves;
    const int q0 = blockIdx.x * kSqQ;
    const int64_t f_first = (int64_t)blockIdx.y * kSqFrames;
    const int64_t c0 = 3 * f_first;
    const int64_t n_cols = 3 * (int64_t)a.n_frames_used;
    const int64_t jb = (int64_t)blockIdx.z * a.sites_per_split;
    const int64_t je = jb + a.sites_per_split < a.n ? jb + a.sites_per_split : a.n;
    // Producer and consumer waves run separate loops with the same barrier
    // count (one before the first chunk, one per chunk), so the consumers'
    // accumulators are not live in the producers' code.
    if (producer) {
        const int ptid = tid - 64 * kSqWaves;
        double qv[3] = {0.0, 0.0, 0.0};  // zero past n_q: rows nobody stores
        if (q0 + ptid % kSqQ < a.n_q) {
            qv[0] = a.q[3 * (q0 + ptid % kSqQ)];
            qv[1] = a.q[3 * (q0 + ptid % kSqQ) + 1];
            qv[2] = a.q[3 * (q0 + ptid % kSqQ) + 2];
        }
        sq_produce(a, ptid, qv, f_first, jb, je, lds, lds + 2 * kSqPhBuf);
        __syncthreads();
        int nxt = 1;
        for (int64_t j0 = jb; j0 < je; j0 += kSqSites) {
            if (j0 + kSqSites < je)
                sq_produce(a, ptid, qv, f_first, j0 + kSqSites, je, lds + nxt * kSqPhBuf,
                           lds + 2 * kSqPhBuf + nxt * kSqSbBuf);
            __syncthreads();  // the consumers are done with the other buffer
            nxt ^= 1;
        }
        return;
    }
    const int qb = wave % kSqQBlocks, cb0 = (wave / kSqQBlocks) * kSqCBW;
    const bool active = q0 + 16 * qb < a.n_q;  // wave-uniform
    // LDS offset of this lane's column in each block (frame row, component)
    int boff[kSqCBW];
#pragma unroll
    for (int b = 0; b < kSqCBW; ++b) {
        const int c = (cb0 + b) * 16 + (lane & 15);
        boff[b] = (c / 3) * kSqPitch + c % 3;
    }
    f64x4 acc_re[kSqCBW], acc_im[kSqCBW];
#pragma unroll
    for (int b = 0; b < kSqCBW; ++b) {
        acc_re[b] = f64x4{0.0, 0.0, 0.0, 0.0};
        acc_im[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    // this lane's first phase and spin in a buffer: A[i][k] = phase of wave
    // vector i at site k sits in lane i + 16 k, B[k][c] = spin column c at
    // site k in lane c + 16 k
    const int a_off = (lane >> 4) * kSqQ + 16 * qb + (lane & 15);
#pragma unroll
    for (int b = 0; b < kSqCBW; ++b) boff[b] += 3 * (lane >> 4);
    __syncthreads();  // the first chunk is staged
    int cur = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kSqSites) {
        if (active) {
            const double* ph = lds + cur * kSqPhBuf + a_off;
            const double* sb = lds + 2 * kSqPhBuf + cur * kSqSbBuf;
            // Two register sets: the operands of K-step k + 1 are read from
            // LDS while the MFMAs of step k run.
            double are[2], aim[2], bv[2][kSqCBW];
            auto fetch = [&](int k, int r) {
                are[r] = ph[4 * k * kSqQ];
                aim[r] = ph[kSqSites * kSqQ + 4 * k * kSqQ];
#pragma unroll
                for (int b = 0; b < kSqCBW; ++b) bv[r][b] = sb[boff[b] + 12 * k];
            };
            fetch(0, 0);
#pragma unroll
            for (int k = 0; k < kSqSites / 4; ++k) {
                const int r = k & 1;
                if (k + 1 < kSqSites / 4) fetch(k + 1, r ^ 1);
#pragma unroll
                for (int b = 0; b < kSqCBW; ++b) {
                    acc_re[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[r], bv[r][b], acc_re[b], 0, 0, 0);
                    acc_im[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[r], bv[r][b], acc_im[b], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // done with `cur`; the producers have filled the other buffer
        cur ^= 1;
    }
    if (!active) return;
    // D[i][c] of the FP64 16x16x4 form: lane l, item v holds row 4 v + l / 16
    // of column l % 16 (rows interleave across the lane groups, unlike the
    // FP32 forms)
    double* out = a.part + (int64_t)blockIdx.z * a.n_q * 2 * n_cols;
#pragma unroll
    for (int b = 0; b < kSqCBW; ++b) {
        const int64_t c = c0 + (cb0 + b) * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int qq = q0 + 16 * qb + 4 * v + (lane >> 4);
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
    return dim3((unsigned)((n_q + kSqQ - 1) / kSqQ), (unsigned)((n_frames_used + kSqFrames - 1) / kSqFrames),
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

int prepare_sq_kernels() {
    return (int)hipFuncSetAttribute((const void*)sq_transform_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    kSqLdsBytes);
}

int sq_frames_per_block() { return kSqFrames; }

int launch_sq_pack(const SqTransformArgs& a, void* stream) {
    const int64_t total = (a.n + kSqSites - 1) / kSqSites * (int64_t)a.t_pad * 3 * kSqSites;
    hipLaunchKernelGGL(sq_pack_kernel, dim3((unsigned)blocks_for(total)), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_sq_transform(const SqTransformArgs& a, void* stream) {
    hipLaunchKernelGGL(sq_transform_kernel, sq_transform_grid(a.n_q, a.n_frames_used, a.n_split), dim3(kSqThreads),
                       kSqLdsBytes, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_sq_corr(const SqTransformArgs& t, const SqCorrArgs& a, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int64_t per = (int64_t)t.n_q * 2 * 3 * (int64_t)t.n_frames_used;
    hipLaunchKernelGGL(sq_reduce_kernel, dim3((unsigned)blocks_for(per)), dim3(256), 0, s, t, a.F);
    hipLaunchKernelGGL(sq_corr_kernel, dim3((unsigned)a.n_q), dim3(256), 0, s, a);
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
