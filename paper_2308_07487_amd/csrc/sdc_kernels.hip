// gfx950 kernels of the sdc library.
//
//  pack    : [T][N][3] fp32 trajectory -> component-major, site-permuted,
//            K-contiguous blocks of 8 time samples (Sec. 3.2: the N x 3M
//            rearrangement; Sec. 3.1: realization-major storage for
//            coalescing), split into hi + lo halves for reduced precision.
//  fused   : per lag the N x N x 3*n_origins product on MFMA with the bin key
//            and the histogram fused into the epilogue (Sec. 3.3-3.4, Fig. 2,
//            Eq. (6)); LDS histograms in FP64, merged into global FP64 bins.
//  count   : exact integer pair counts per bin with the same tile walk.
//  self    : the i = j term per lag in FP64.
//  final   : normalisation, site sum and the windowed time DFT (Sec. 2.2).
//  traj    : Landau-Lifshitz RK4 (Eq. (2), Sec. 3.1) with Philox4x32-10 starts.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "sdc_internal.h"

namespace sdc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// 32-byte pack element: 8 time samples of one component of one site.
// Split precisions: 8 hi halves then 8 lo halves.  FP32: 8 floats.
struct alignas(16) Chunk {
    uint4 x, y;
};
// 48-byte pack element of the three-piece BF16 form: 8 hi, 8 mid, 8 lo.
struct alignas(16) Chunk3 {
    uint4 x, y, z;
};
template <int PREC>
using PackElem = typename std::conditional<PREC == SDC_PREC_BF16X3, Chunk3, Chunk>::type;

// ---------------------------------------------------------------------------
// pack
// ---------------------------------------------------------------------------

__device__ inline uint32_t bf16_bits(float v) {
    __bf16 b = (__bf16)v;  // round to nearest even
    return (uint32_t)__builtin_bit_cast(uint16_t, b);
}
__device__ inline uint32_t f16_bits(float v) {
    _Float16 b = (_Float16)v;
    return (uint32_t)__builtin_bit_cast(uint16_t, b);
}
__device__ inline float bf16_val(uint32_t bits) {
    return (float)__builtin_bit_cast(__bf16, (uint16_t)bits);
}
__device__ inline float f16_val(uint32_t bits) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits);
}

template <int PREC>
__device__ inline PackElem<PREC> make_chunk(const float v[8]) {
    PackElem<PREC> c;
    if constexpr (PREC == SDC_PREC_BF16X3) {
        // x = hi + mid + lo exactly: each difference has at most 16 (then 8)
        // significant bits and is exact in fp32
        uint32_t hi[8], mi[8], lo[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            hi[e] = bf16_bits(v[e]);
            const float r1 = v[e] - bf16_val(hi[e]);
            mi[e] = bf16_bits(r1);
            lo[e] = bf16_bits(r1 - bf16_val(mi[e]));
        }
        c.x = make_uint4(hi[0] | hi[1] << 16, hi[2] | hi[3] << 16, hi[4] | hi[5] << 16, hi[6] | hi[7] << 16);
        c.y = make_uint4(mi[0] | mi[1] << 16, mi[2] | mi[3] << 16, mi[4] | mi[5] << 16, mi[6] | mi[7] << 16);
        c.z = make_uint4(lo[0] | lo[1] << 16, lo[2] | lo[3] << 16, lo[4] | lo[5] << 16, lo[6] | lo[7] << 16);
    } else if constexpr (PREC == SDC_PREC_FP32) {
        c.x = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                         __float_as_uint(v[3]));
        c.y = make_uint4(__float_as_uint(v[4]), __float_as_uint(v[5]), __float_as_uint(v[6]),
                         __float_as_uint(v[7]));
    } else {
        uint32_t hi[8], lo[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if constexpr (PREC == SDC_PREC_SPLIT_BF16) {
                hi[e] = bf16_bits(v[e]);
                lo[e] = bf16_bits(v[e] - bf16_val(hi[e]));  // v - hi is exact in fp32
            } else {
                hi[e] = f16_bits(v[e]);
                lo[e] = f16_bits(v[e] - f16_val(hi[e]));
            }
        }
        c.x = make_uint4(hi[0] | hi[1] << 16, hi[2] | hi[3] << 16, hi[4] | hi[5] << 16,
                         hi[6] | hi[7] << 16);
        c.y = make_uint4(lo[0] | lo[1] << 16, lo[2] | lo[3] << 16, lo[4] | lo[5] << 16,
                         lo[6] | lo[7] << 16);
    }
    return c;
}

// One thread per (block of 8 samples, packed site); writes the three
// components.  Rows 0..3*O8 of the work index the A pack (origins o*s),
// the rest the B packs (phase copies: sample g of phase ph is frame s*g + ph).
template <int PREC>
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_pad) return;
    const int row = blockIdx.y;  // 0..O8 + n_phase*F8 - 1
    const int32_t orig = a.perm[p];
    float v[3][8];
    const bool isA = row < a.O8;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int64_t f;
        bool ok;
        if (isA) {
            const int o = row * 8 + e;
            f = (int64_t)o * a.stride;
            ok = o < a.n_origins;
        } else {
            const int r = row - a.O8;
            const int ph = r / a.F8;
            const int g = (r % a.F8) * 8 + e;
            f = (int64_t)g * a.stride + ph;
            ok = true;
        }
        ok = ok && orig >= 0 && f < a.frames_valid;
        const float* src = a.frames + (f * a.n + (ok ? orig : 0)) * 3;
        v[0][e] = ok ? src[0] : 0.0f;
        v[1][e] = ok ? src[1] : 0.0f;
        v[2][e] = ok ? src[2] : 0.0f;
        // connected form: the origin side is centred on its average over the
        // origins (Eq. (5)); since the centred values sum to zero over the
        // origins, the later side needs no centring
        if (isA && ok && a.mean) {
            v[0][e] -= a.mean[4 * orig];
            v[1][e] -= a.mean[4 * orig + 1];
            v[2][e] -= a.mean[4 * orig + 2];
        }
    }
    PackElem<PREC>* dst;
    int64_t comp_stride;
    if (isA) {
        dst = (PackElem<PREC>*)a.A + (int64_t)row * a.n_pad + p;
        comp_stride = (int64_t)a.O8 * a.n_pad;
    } else {
        const int r = row - a.O8;
        const int ph = r / a.F8;
        dst = (PackElem<PREC>*)a.B + ((int64_t)ph * 3 * a.F8 + (r % a.F8)) * a.n_pad + p;
        comp_stride = (int64_t)a.F8 * a.n_pad;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[c * comp_stride] = make_chunk<PREC>(v[c]);
}

int launch_pack(const PackArgs& a, void* stream) {
    dim3 block(256);
    dim3 grid((unsigned)((a.n_pad + 255) / 256), (unsigned)(a.O8 + a.n_phase * a.F8));
    hipStream_t s = (hipStream_t)stream;
    switch (a.precision) {
        case SDC_PREC_FP32: hipLaunchKernelGGL(pack_kernel<SDC_PREC_FP32>, grid, block, 0, s, a); break;
        case SDC_PREC_SPLIT_BF16: hipLaunchKernelGGL(pack_kernel<SDC_PREC_SPLIT_BF16>, grid, block, 0, s, a); break;
        case SDC_PREC_SPLIT_FP16: hipLaunchKernelGGL(pack_kernel<SDC_PREC_SPLIT_FP16>, grid, block, 0, s, a); break;
        case SDC_PREC_BF16X3: hipLaunchKernelGGL(pack_kernel<SDC_PREC_BF16X3>, grid, block, 0, s, a); break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused product + binning epilogue
// ---------------------------------------------------------------------------
//
// Work: task = (lag group, stream).  A workgroup of 4 waves takes one task
// and walks the stream's tile pairs (64 i-sites x 64 j-sites).  Wave w owns
// the 32x32 quadrant (w >> 1, w & 1) for all LG lags of the group: LG MFMA
// accumulator tiles.  The K loop runs over the 3 components and over
// K-steps of 16 origins; in a K-step, lane (i, h) holds origins
// 16c + 8h + [0, 8) of its site and lane (j, h) holds the 8*NB samples
// 16c + 8h + u0 + [0, 8*NB) of its site, from which the operand of lag
// u0 + m is the 8-sample slice starting at m (a register select for even m,
// a byte align for odd m).  No operand goes through LDS; LDS holds the
// histogram.  Two workgroups share a CU, so one workgroup's epilogue and
// memory waits overlap the other's MFMA work.

__device__ inline uint32_t align2(uint32_t hi, uint32_t lo) {
    return __builtin_amdgcn_alignbyte(hi, lo, 2);
}

// Operand of lag u0 + M: the 8 halves starting at window element M.
template <int M, int NW>
__device__ inline uint4 slice8(const uint32_t (&w)[NW]) {
    constexpr int e = M / 2;
    static_assert(e + 4 + (M & 1) <= NW, "window too short");
    if constexpr ((M & 1) == 0) {
        return make_uint4(w[e], w[e + 1], w[e + 2], w[e + 3]);
    } else {
        return make_uint4(align2(w[e + 1], w[e]), align2(w[e + 2], w[e + 1]),
                          align2(w[e + 3], w[e + 2]), align2(w[e + 4], w[e + 3]));
    }
}

template <int PREC>
__device__ inline f32x16 mfma16(uint4 a, uint4 b, f32x16 c) {
    if constexpr (PREC == SDC_PREC_SPLIT_BF16 || PREC == SDC_PREC_BF16X3) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
}

// Products one K loop forms (PASS):
//  kPassAll   : every product of the form; the large ones into acc.v, the
//               small ones into acc.s (one-pass and lag-split schedules);
//  kPassSmall : hi*lo + lo*hi into acc.v (first loop of the two-pass
//               schedule, from zero);
//  kPassLarge : hi*hi into acc.v (second loop, on top of the small sums).
// The small products are never added to a sum that already holds the large
// ones: the BF16/FP16 matrix cores align every addend of an instruction to
// the largest one and drop the bits that fall below a fixed window, always
// downwards, so the low bits of small products added to a large sum would
// bias each element by a fraction of its last place per K-step.  Added to a
// sum of their own size they keep every bit, and the large products added
// afterwards (16 significant bits each) lose none either.
//  kPassFold  : every product of the form; per K-step and lag the small
//               products are summed from zero in a transient tile, which FP32
//               vector adds (round to nearest) then add to acc.v, next to
//               the hi*hi MFMA (fold schedule).
constexpr int kPassAll = 0, kPassLarge = 1, kPassSmall = 2, kPassFold = 3;

__device__ inline void add16(f32x16& acc, const f32x16& t) {
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += t[r];
}

// Three-product split for the wave's lag M (its window slice OFF + M):
// hi*hi + hi*lo + lo*hi.
template <int PREC, int PASS, int OFF, int M, int NW, int LW>
__device__ inline void split_step(const Chunk& av, const uint32_t (&wh)[NW],
                                  const uint32_t (&wl)[NW], f32x16 (&acc)[LW], f32x16 (&acc_s)[LW]) {
    const uint4 bh = slice8<OFF + M, NW>(wh);
    if constexpr (PASS == kPassLarge) {
        acc[M] = mfma16<PREC>(av.x, bh, acc[M]);
    } else {
        const uint4 bl = slice8<OFF + M, NW>(wl);
        if constexpr (PASS == kPassAll) {
            acc[M] = mfma16<PREC>(av.x, bh, acc[M]);
            acc_s[M] = mfma16<PREC>(av.x, bl, acc_s[M]);
            acc_s[M] = mfma16<PREC>(av.y, bh, acc_s[M]);
        } else if constexpr (PASS == kPassFold) {
            f32x16 t = {};
            t = mfma16<PREC>(av.x, bl, t);
            t = mfma16<PREC>(av.y, bh, t);
            acc[M] = mfma16<PREC>(av.x, bh, acc[M]);
            add16(acc[M], t);
        } else {
            acc[M] = mfma16<PREC>(av.x, bl, acc[M]);
            acc[M] = mfma16<PREC>(av.y, bh, acc[M]);
        }
    }
}

// Three-piece BF16 for the wave's lag M: the six products hh, hm, mh, mm,
// hl, lh (the dropped ml, lm, ll are below 2^-24 of the product); hh goes to
// the main accumulator, the other five (2^-8 and smaller) to the second one.
template <int OFF, int M, int NW, int LW>
__device__ inline void x3_step(const Chunk3& av, const uint32_t (&wh)[NW], const uint32_t (&wm)[NW],
                               const uint32_t (&wl)[NW], f32x16 (&acc)[LW], f32x16 (&acc_s)[LW]) {
    const uint4 bh = slice8<OFF + M, NW>(wh);
    const uint4 bm = slice8<OFF + M, NW>(wm);
    const uint4 bl = slice8<OFF + M, NW>(wl);
    acc[M] = mfma16<SDC_PREC_BF16X3>(av.x, bh, acc[M]);
    acc_s[M] = mfma16<SDC_PREC_BF16X3>(av.x, bm, acc_s[M]);
    acc_s[M] = mfma16<SDC_PREC_BF16X3>(av.y, bh, acc_s[M]);
    acc_s[M] = mfma16<SDC_PREC_BF16X3>(av.y, bm, acc_s[M]);
    acc_s[M] = mfma16<SDC_PREC_BF16X3>(av.x, bl, acc_s[M]);
    acc_s[M] = mfma16<SDC_PREC_BF16X3>(av.z, bh, acc_s[M]);
}

// The same with the small products folded into the main sums per K-step.
template <int OFF, int M, int NW, int LW>
__device__ inline void x3_fold_step(const Chunk3& av, const uint32_t (&wh)[NW], const uint32_t (&wm)[NW],
                                    const uint32_t (&wl)[NW], f32x16 (&acc)[LW]) {
    const uint4 bh = slice8<OFF + M, NW>(wh);
    const uint4 bm = slice8<OFF + M, NW>(wm);
    const uint4 bl = slice8<OFF + M, NW>(wl);
    f32x16 t = {};
    t = mfma16<SDC_PREC_BF16X3>(av.x, bm, t);
    t = mfma16<SDC_PREC_BF16X3>(av.y, bh, t);
    t = mfma16<SDC_PREC_BF16X3>(av.y, bm, t);
    t = mfma16<SDC_PREC_BF16X3>(av.x, bl, t);
    t = mfma16<SDC_PREC_BF16X3>(av.z, bh, t);
    acc[M] = mfma16<SDC_PREC_BF16X3>(av.x, bh, acc[M]);
    add16(acc[M], t);
}

template <int OFF, int NW, int LW, int... Ms>
__device__ inline void x3_all(const Chunk3& av, const uint32_t (&wh)[NW], const uint32_t (&wm)[NW],
                              const uint32_t (&wl)[NW], f32x16 (&acc)[LW], f32x16 (&acc_s)[LW],
                              std::integer_sequence<int, Ms...>) {
    (x3_step<OFF, Ms, NW, LW>(av, wh, wm, wl, acc, acc_s), ...);
}

template <int OFF, int NW, int LW, int... Ms>
__device__ inline void x3_fold_all(const Chunk3& av, const uint32_t (&wh)[NW], const uint32_t (&wm)[NW],
                                   const uint32_t (&wl)[NW], f32x16 (&acc)[LW], std::integer_sequence<int, Ms...>) {
    (x3_fold_step<OFF, Ms, NW, LW>(av, wh, wm, wl, acc), ...);
}

template <int PREC, int PASS, int OFF, int NW, int LW, int... Ms>
__device__ inline void split_all(const Chunk& av, const uint32_t (&wh)[NW], const uint32_t (&wl)[NW],
                                 f32x16 (&acc)[LW], f32x16 (&acc_s)[LW], std::integer_sequence<int, Ms...>) {
    (split_step<PREC, PASS, OFF, Ms, NW, LW>(av, wh, wl, acc, acc_s), ...);
}

// FP32: MFMA q of the K-step takes origin 16c + 8h + q on both sides.
template <int Q, int OFF, int M, int NF, int LW>
__device__ inline void f32_step(const float (&a)[8], const float (&w)[NF], f32x16 (&acc)[LW]) {
    acc[M] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[Q], w[Q + OFF + M], acc[M], 0, 0, 0);
}
template <int Q, int OFF, int NF, int LW, int... Ms>
__device__ inline void f32_q(const float (&a)[8], const float (&w)[NF], f32x16 (&acc)[LW],
                             std::integer_sequence<int, Ms...>) {
    (f32_step<Q, OFF, Ms, NF, LW>(a, w, acc), ...);
}
template <int OFF, int NF, int LW, int... Qs>
__device__ inline void f32_all(const float (&a)[8], const float (&w)[NF], f32x16 (&acc)[LW],
                               std::integer_sequence<int, Qs...>) {
    (f32_q<Qs, OFF, NF, LW>(a, w, acc, std::make_integer_sequence<int, LW>{}), ...);
}

// Fixed-point image of v (deterministic mode), rounded to nearest.
__device__ inline unsigned long long to_fixed(double v) {
    return (unsigned long long)__double2ll_rn(v * kFixedScale);
}

__device__ inline int pmod_dev(int a, int m) {
    int r = a % m;
    return r < 0 ? r + m : r;
}

// Accumulators of one wave: LW 32x32 tiles, and for the schedules that
// keep them apart a second set for the small products of the reduced forms.
template <int PREC, int SCHED, int LW>
struct Acc {
    f32x16 v[LW];
    f32x16 s[(PREC == SDC_PREC_FP32 || SCHED == kSchedTwoPass || SCHED == kSchedFold) ? 1 : LW];
};

// Operands of one K-step for one lane: A (8 origins, hi/lo or fp32) and the
// B window of NB pack elements.
template <int PREC, int NB>
struct Stage {
    PackElem<PREC> a;
    PackElem<PREC> b[NB];
};

template <int PREC, int PASS, int SCHED, int NB, int LW, int OFF>
__device__ inline void stage_mma(const Stage<PREC, NB>& s, Acc<PREC, SCHED, LW>& ac) {
    f32x16 (&acc)[LW] = ac.v;
    constexpr int NW = 4 * NB;
    if constexpr (PREC == SDC_PREC_BF16X3) {
        uint32_t wh[NW], wm[NW], wl[NW];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const uint32_t h4[4] = {s.b[k].x.x, s.b[k].x.y, s.b[k].x.z, s.b[k].x.w};
            const uint32_t m4[4] = {s.b[k].y.x, s.b[k].y.y, s.b[k].y.z, s.b[k].y.w};
            const uint32_t l4[4] = {s.b[k].z.x, s.b[k].z.y, s.b[k].z.z, s.b[k].z.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                wh[4 * k + e] = h4[e];
                wm[4 * k + e] = m4[e];
                wl[4 * k + e] = l4[e];
            }
        }
        if constexpr (PASS == kPassFold)
            x3_fold_all<OFF, NW, LW>(s.a, wh, wm, wl, acc, std::make_integer_sequence<int, LW>{});
        else
            x3_all<OFF, NW, LW>(s.a, wh, wm, wl, acc, ac.s, std::make_integer_sequence<int, LW>{});
    } else if constexpr (PREC == SDC_PREC_FP32) {
        float af[8], w[8 * NB];
        const uint32_t ar[8] = {s.a.x.x, s.a.x.y, s.a.x.z, s.a.x.w, s.a.y.x, s.a.y.y, s.a.y.z, s.a.y.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) af[e] = __uint_as_float(ar[e]);
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const uint32_t r[8] = {s.b[k].x.x, s.b[k].x.y, s.b[k].x.z, s.b[k].x.w,
                                   s.b[k].y.x, s.b[k].y.y, s.b[k].y.z, s.b[k].y.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) w[8 * k + e] = __uint_as_float(r[e]);
        }
        f32_all<OFF, 8 * NB, LW>(af, w, acc, std::make_integer_sequence<int, 8>{});
    } else {
        uint32_t wh[NW], wl[NW];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            wh[4 * k] = s.b[k].x.x;
            wh[4 * k + 1] = s.b[k].x.y;
            wh[4 * k + 2] = s.b[k].x.z;
            wh[4 * k + 3] = s.b[k].x.w;
            wl[4 * k] = s.b[k].y.x;
            wl[4 * k + 1] = s.b[k].y.y;
            wl[4 * k + 2] = s.b[k].y.z;
            wl[4 * k + 3] = s.b[k].y.w;
        }
        // the two-pass schedule has no second accumulator set (its passes
        // never write one)
        if constexpr (SCHED == kSchedTwoPass || SCHED == kSchedFold)
            split_all<PREC, PASS, OFF, NW, LW>(s.a, wh, wl, acc, acc, std::make_integer_sequence<int, LW>{});
        else
            split_all<PREC, PASS, OFF, NW, LW>(s.a, wh, wl, acc, ac.s, std::make_integer_sequence<int, LW>{});
    }
}

int fused_lds_bytes(int win, int precision) {
    return lag_group(precision) * win * (int)sizeof(double) + 1024 * (int)sizeof(float);
}

// MFMA instructions one stage_mma call issues per wave.
template <int PREC, int PASS, int LW>
constexpr int mfma_per_stage() {
    if constexpr (PREC == SDC_PREC_FP32) return 8 * LW;
    else if constexpr (PREC == SDC_PREC_BF16X3) return 6 * LW;
    else if constexpr (PASS == kPassLarge) return LW;
    else if constexpr (PASS == kPassSmall) return 2 * LW;
    else return 3 * LW;
}

// Instruction order of one K-step for the schedules with a second
// accumulator set (one-pass, lag-split): the next stage's loads first, then
// each MFMA followed by up to NV vector instructions (the operand shuffles of
// the following lags), so that the shuffles issue while the matrix core works
// instead of in a burst in front of it (about 5% at the 36^3 workload).  The
// two-pass and fold loops keep the compiler's order with the loads fenced
// off from the MFMAs: there the interleave gains nothing (two-pass) or costs
// register spills (fold, and the batch kernel).
template <int NMF, int NV>
__device__ __forceinline__ void interleave() {
    __builtin_amdgcn_sched_group_barrier(0x020, 16, 0);  // vector memory reads
#pragma unroll
    for (int i = 0; i < NMF; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, NV, 0);  // vector ALU
    }
}

// One K loop over all K-steps of a tile pair with NS register buffers: the
// loads of the next NS - 1 K-steps are in flight while one step's MFMAs run
// (load indices clamp to the last step, so the last round's extra loads are
// harmless re-reads).  For the interleaved schedules the main loop takes NS
// steps per trip without a branch, so loads and MFMAs of a step share one
// scheduling region, and the fewer than NS steps left after it (loaded
// already) follow; the others skip the steps past the end inside the loop
// and fence the loads off from the MFMAs.
template <int PREC, int PASS, int SCHED, int NB, int LW, int OFF, int NS, class Load>
__device__ __forceinline__ void k_loop(int nk, const Load& load, Acc<PREC, SCHED, LW>& acc) {
    Stage<PREC, NB> s[NS];
#pragma unroll
    for (int j = 0; j < NS - 1; ++j) load(s[j], j);
    if constexpr (SCHED == kSchedOnePass || SCHED == kSchedLagSplit) {
        constexpr int NMF = mfma_per_stage<PREC, PASS, LW>();
        int kk = 0;
        for (; kk + NS <= nk; kk += NS) {
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                load(s[(j + NS - 1) % NS], kk + j + NS - 1);
                stage_mma<PREC, PASS, SCHED, NB, LW, OFF>(s[j], acc);
                interleave<NMF, 4>();
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int j = 0; j < NS - 1; ++j)
            if (kk + j < nk) stage_mma<PREC, PASS, SCHED, NB, LW, OFF>(s[j], acc);
    } else {
        for (int kk = 0; kk < nk; kk += NS) {
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                load(s[(j + NS - 1) % NS], kk + j + NS - 1);
                __builtin_amdgcn_sched_barrier(0);
                if (j == 0 || kk + j < nk) stage_mma<PREC, PASS, SCHED, NB, LW, OFF>(s[j], acc);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

// What the tile-pair loop of one wave needs of its task.
struct TaskCtx {
    const FusedArgs* a;
    KGroup grp;
    KStream st;
    double* hist;
    const float* e2s;
    int quadrant;  // 32x32 quadrant of the 64x64 tile pair (wave index mod 4)
};

// The tile pairs of a task for one wave: its quadrant, its LW lags starting
// at lag OFF of the group (all LG of them unless the lag-split schedule
// gives the group's two halves to two waves).
template <int PREC, int RADIAL, int PAIRED, int SCHED, int LW, int OFF>
__device__ __forceinline__ void pair_loop(const TaskCtx& c) {
    constexpr int LG = lag_group(PREC);
    constexpr int NB = win_blocks(LG);
    constexpr bool TWO = SCHED == kSchedTwoPass;
    constexpr bool FOLD = SCHED == kSchedFold;
    const FusedArgs& a = *c.a;
    const KGroup grp = c.grp;
    double* hist = c.hist;
    const int lane = threadIdx.x & 63;
    const int wi = c.quadrant >> 1, wj = c.quadrant & 1, h = lane >> 5, l32 = lane & 31;

    using Elem = PackElem<PREC>;
    const Elem* Ab = (const Elem*)a.A;
    const Elem* Bb = (const Elem*)a.B + (int64_t)grp.phase * a.phase_stride;
    // K-steps run over the 3 O8 origin blocks of all components, two blocks
    // per step (one per lane half); a half past the last block reads the A
    // pack's zero block 3 O8
    const int nk = a.nk;
    const int nblk = 3 * a.O8;
    const int ublk = grp.u0 / 8;
    const int dF = a.F8 - a.O8;  // B block of A block k (component c): k + c dF + ublk
    const int n_c = a.O8 / 2;    // PAIRED: K-steps per component

    // lane byte offsets from a block's tile base: the site within the tile
    // and, for the upper lane half, the next block (the plan keeps two pack
    // blocks within 4 GiB)
    const uint32_t offA = (uint32_t)(((int64_t)h * a.n_pad + wi * 32 + l32) * (int64_t)sizeof(Elem));
    const uint32_t offB = (uint32_t)(((int64_t)h * a.n_pad + wj * 32 + l32) * (int64_t)sizeof(Elem));

    for (int p = c.st.p0; p < c.st.p1; ++p) {
        const KPair pr = a.pairs[p];
        const int64_t sj = (int64_t)pr.tj * kTile + wj * 32 + l32;
        Acc<PREC, SCHED, LW> acc;
#pragma unroll
        for (int m = 0; m < LW; ++m)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc.v[m][r] = 0.0f;
        if constexpr (PREC != SDC_PREC_FP32 && !TWO && !FOLD) {
#pragma unroll
            for (int m = 0; m < LW; ++m)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc.s[m][r] = 0.0f;
        }

        // Register buffers: while K-step kk is multiplied the loads of later
        // steps are in flight (indices clamp to the last block).  Parts of
        // an element a pass does not use are not loaded (dead loads).  Each
        // load is a uniform block address plus the lane's fixed byte offset.
        const Elem* At = Ab + (int64_t)pr.ti * kTile;
        const Elem* Bt = Bb + (int64_t)pr.tj * kTile;
        auto load = [&](Stage<PREC, NB>& b, int kk) {
            kk = kk < nk ? kk : nk - 1;
            const int64_t np = a.n_pad;
            // A block of lane half h: 2 kk + h (the zero block for the half
            // past the last block)
            const Elem* pa = At + (int64_t)(2 * kk) * np;
            const Elem* pb;
            uint32_t ob = offB;
            if constexpr (PAIRED) {
                // both halves in component alpha: B block 2 kk + h + alpha dF + ublk
                const int alpha = (kk >= n_c) + (kk >= 2 * n_c);
                pb = Bt + (int64_t)(2 * kk + alpha * dF + ublk) * np;
            } else {
                // block indices of both lane halves from the step index
                // (uniform); A: [3][O8] blocks flattened, then the zero block
                const int k0 = 2 * kk;
                const int k1 = k0 + 1 < nblk ? k0 + 1 : nblk - 1;
                const int b0 = k0 + ((k0 >= a.O8) + (k0 >= 2 * a.O8)) * dF + ublk;
                const int b1 = k1 + ((k1 >= a.O8) + (k1 >= 2 * a.O8)) * dF + ublk;
                pb = Bt + (int64_t)b0 * np;
                // offB holds one block for the upper half; it needs b1 - b0
                ob += h ? (uint32_t)((int64_t)(b1 - b0 - 1) * np * (int64_t)sizeof(Elem)) : 0u;
            }
            b.a = *(const Elem*)((const char*)pa + offA);
#pragma unroll
            for (int q = 0; q < NB; ++q) b.b[q] = *(const Elem*)((const char*)(pb + q * np) + ob);
        };

        // Epilogue: bin of each accumulator element, LDS FP64 add per lag.
        // Accumulator register r of lane (l32, h) holds row 8(r/4) + 4h + r%4,
        // column l32 of the wave's 32x32 quadrant.
        int bin[16];
        auto bins = [&]() {
            const int64_t rowbase = (int64_t)pr.ti * kTile + wi * 32 + 4 * h;
            if constexpr (RADIAL) {
                if (a.keys) {
                    // the pair's shells, computed once per plan for all lag groups
                    const uint4* kp =
                        (const uint4*)(a.keys + (((int64_t)p * 4 + c.quadrant) * 64 + lane) * 16);
                    const uint4 k0 = kp[0], k1 = kp[1];
                    const uint32_t kw[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
#pragma unroll
                    for (int r = 0; r < 16; ++r) bin[r] = (int)((kw[r / 2] >> (16 * (r & 1))) & 0xFFFFu);
                } else {
                    const float4 pj = *(const float4*)(a.pos4 + 4 * sj);
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float4 pi = *(const float4*)(a.pos4 + 4 * (rowbase + 8 * (r / 4) + (r % 4)));
                        const float d2 = dist2_f32(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z);
                        bin[r] = shell_of(d2, c.e2s, a.n_shells, a.inv_w);
                    }
                }
            } else {
                const int gj = a.gtab[sj] + pr.shift;
#pragma unroll
                for (int r = 0; r < 16; ++r) bin[r] = gj - a.gtab[rowbase + 8 * (r / 4) + (r % 4)];
            }
        };
        auto add_hist = [&](auto with_small) {
#pragma unroll
            for (int m = 0; m < LW; ++m) {
                if ((grp.mask >> (OFF + m)) & 1) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        double v = (double)acc.v[m][r];
                        if constexpr (decltype(with_small)::value) v += (double)acc.s[m][r];
                        if (a.det)
                            atomicAdd(reinterpret_cast<unsigned long long*>(hist) + (OFF + m) * a.win + bin[r],
                                      to_fixed(v));
                        else
                            atomicAdd(&hist[(OFF + m) * a.win + bin[r]], v);
                    }
                }
            }
        };

        if constexpr (TWO) {
            // small products first, while the sums are still small, then the
            // large ones on top (see the pass constants)
            k_loop<PREC, kPassSmall, SCHED, NB, LW, OFF, kStagesTwoPassSmall>(nk, load, acc);
            k_loop<PREC, kPassLarge, SCHED, NB, LW, OFF, kStagesTwoPassLarge>(nk, load, acc);
            bins();
            add_hist(std::false_type{});
        } else if constexpr (FOLD) {
            k_loop<PREC, kPassFold, SCHED, NB, LW, OFF, kStagesFold>(nk, load, acc);
            bins();
            add_hist(std::false_type{});
        } else {
            k_loop<PREC, kPassAll, SCHED, NB, LW, OFF, kStagesOnePass>(nk, load, acc);
            bins();
            add_hist(std::integral_constant<bool, PREC != SDC_PREC_FP32>{});
        }
    }
}

// One task of a plan: the stream's tile pairs for one lag group, histogram
// in LDS (`hist`: [LG][win] FP64, then the radial edge table), merged into
// the plan's global bins at the end.  Called by the whole workgroup.
// PAIRED: O8 is even, so a K-step's two origin blocks always lie in one
// component and the block offsets follow from the step with one scalar
// division; otherwise the blocks of all components are taken in turn and a
// step may straddle two components.
// SCHED: kSchedOnePass, kSchedTwoPass (hi/lo splits only) or kSchedLagSplit
// (eight waves: wave w takes quadrant w mod 4 and the lag half w / 4).
template <int PREC, int RADIAL, int PAIRED, int SCHED>
__device__ __forceinline__ void fused_task(const FusedArgs& a, int task, double* hist) {
    constexpr int LG = lag_group(PREC);
    constexpr int NT = threads_per_wg(SCHED);
    float* e2s = (float*)(hist + LG * a.win);
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    TaskCtx c;
    c.a = &a;
    c.grp = a.groups[task % a.n_groups];
    c.st = a.streams[task / a.n_groups];
    c.hist = hist;
    c.e2s = e2s;
    c.quadrant = wave & 3;

    for (int x = tid; x < LG * a.win; x += NT) hist[x] = 0.0;
    if constexpr (RADIAL) {
        for (int x = tid; x < a.n_shells; x += NT) e2s[x] = a.e2[x];
    }
    __syncthreads();

    if constexpr (SCHED == kSchedLagSplit) {
        if (wave < 4)
            pair_loop<PREC, RADIAL, PAIRED, SCHED, LG / 2, 0>(c);
        else
            pair_loop<PREC, RADIAL, PAIRED, SCHED, LG / 2, LG / 2>(c);
    } else {
        pair_loop<PREC, RADIAL, PAIRED, SCHED, LG, 0>(c);
    }
    __syncthreads();

    // Merge the stream's histogram into the global bins.
    const KGroup grp = c.grp;
    const KStream st = c.st;
    for (int x = tid; x < LG * a.win; x += NT) {
        const int m = x / a.win;
        const int w = x - m * a.win;
        const double v = hist[x];
        const unsigned long long vq = reinterpret_cast<const unsigned long long*>(hist)[x];
        if (vq != 0ull && ((grp.mask >> m) & 1)) {
            int64_t b;
            if constexpr (RADIAL) {
                b = w;
            } else {
                const int w0 = w / (a.W1 * a.W2);
                const int w1 = (w / a.W2) % a.W1;
                const int w2 = w % a.W2;
                const int k0 = pmod_dev(st.base[0] + w0, a.L0);
                const int k1 = pmod_dev(st.base[1] + w1, a.L1);
                const int k2 = pmod_dev(st.base[2] + w2, a.L2);
                b = ((int64_t)k0 * a.L1 + k1) * a.L2 + k2;
                if (a.kind == SDC_BINS_PERIODIC_BCC) b = 2 * b + st.parity;
            }
            const int64_t t = (int64_t)a.stride * (grp.u0 + m) + grp.phase;
            if (a.det)
                atomicAdd(&a.Hq[t * a.n_bins + b], vq);
            else
                unsafeAtomicAdd(&a.H[t * a.n_bins + b], v);
        }
    }
}

template <int PREC, int RADIAL, int PAIRED, int SCHED>
__global__ __launch_bounds__(threads_per_wg(SCHED), waves_per_simd(SCHED)) void fused_kernel(FusedArgs a) {
    extern __shared__ double hist[];
    // XCD-aware task order: consecutive tasks land on the same XCD (work-
    // groups are dealt to the 8 XCDs round-robin), and consecutive tasks are
    // the lag groups of one stream.  The workgroups running together on an
    // XCD then walk the same tile pairs in step: they share the i-tile
    // operand and overlapping time windows of the j-tile operand in L2.
    const int n_tasks = a.n_groups * a.n_streams;
    const int per = (n_tasks + 7) / 8;
    const int task = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (task >= n_tasks) return;
    fused_task<PREC, RADIAL, PAIRED, SCHED>(a, task, hist);
}

// Persistent kernel over the tasks of several plans (one launch for a
// batch of samples).  The global task list (plan-major, then stream, then
// lag group) is cut into 8 contiguous ranges of about equal work, at stream
// boundaries, one queue per XCD; a workgroup takes tasks from its own XCD's
// queue with an atomic counter and, once that queue is empty, from the
// following queues in turn.  Equal work keeps the XCDs on their own queues
// until the end, so the lag groups of a stream segment run on one XCD and
// share its operands in L2 (ranges of equal task counts let the XCDs with
// the small samples' short tasks steal the large samples' tasks for most of
// the launch, and the operand fetches grew 8x).  Every counter only grows
// and each queue is visited until it is found empty, so every workgroup
// leaves the loop after at most total + 8 claims.  The K-step addressing
// follows each plan's origin-block count (per component when it is even).
template <int PREC, int RADIAL, int SCHED>
__global__ __launch_bounds__(threads_per_wg(SCHED), waves_per_simd(SCHED)) void fused_batch_kernel(
    const FusedArgs* __restrict__ args, const int64_t* __restrict__ task_start, int n_plans,
    unsigned* __restrict__ queue, const int32_t* __restrict__ ranges, int total) {
    extern __shared__ double hist[];
    __shared__ int s_task, s_plan, s_queue, s_exhausted;
    if (threadIdx.x == 0) {
        s_queue = (int)(blockIdx.x % 8);
        s_exhausted = 0;
    }
    for (;;) {
        if (threadIdx.x == 0) {
            // queue state in LDS: no registers stay live across a task
            int x = s_queue, exhausted = s_exhausted;
            int t = -1;
            while (exhausted < 8) {
                const int lo = ranges[x];
                const int hi = min(ranges[x + 1], total);
                if (lo < hi) {
                    const unsigned k = atomicAdd(&queue[x], 1u);
                    if (k < (unsigned)(hi - lo)) {
                        t = lo + (int)k;
                        break;
                    }
                }
                x = (x + 1) % 8;
                ++exhausted;
            }
            int pl = 0;
            if (t >= 0) {  // last plan whose first task is <= t
                int lo = 0, hi = n_plans - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) / 2;
                    if (task_start[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                pl = lo;
                t -= (int)task_start[pl];
            }
            s_task = t;
            s_plan = pl;
            s_queue = x;
            s_exhausted = exhausted;
        }
        __syncthreads();
        const int task = __builtin_amdgcn_readfirstlane(s_task);
        const int pl = __builtin_amdgcn_readfirstlane(s_plan);
        __syncthreads();
        if (task < 0) break;
        const int paired = __builtin_amdgcn_readfirstlane(args[pl].O8 % 2 == 0);
        if (paired)
            fused_task<PREC, RADIAL, 1, SCHED>(args[pl], task, hist);
        else
            fused_task<PREC, RADIAL, 0, SCHED>(args[pl], task, hist);
        __syncthreads();  // the histogram is reused by the next task
    }
}

// Instantiated kernels: (precision, schedule) pairs the library runs.
template <int PREC, int SCHED, int RADIAL, int PAIRED>
static const void* fused_fn() {
    return (const void*)fused_kernel<PREC, RADIAL, PAIRED, SCHED>;
}
template <int PREC, int SCHED, int RADIAL>
static const void* batch_fn() {
    return (const void*)fused_batch_kernel<PREC, RADIAL, SCHED>;
}

template <int PREC, int SCHED>
static const void* pick_fused(int radial, int paired, bool batch) {
    if (batch) return radial ? batch_fn<PREC, SCHED, 1>() : batch_fn<PREC, SCHED, 0>();
    if (radial) return paired ? fused_fn<PREC, SCHED, 1, 1>() : fused_fn<PREC, SCHED, 1, 0>();
    return paired ? fused_fn<PREC, SCHED, 0, 1>() : fused_fn<PREC, SCHED, 0, 0>();
}

template <int PREC>
static const void* pick_sched(int sched, int radial, int paired, bool batch) {
    switch (sched) {
        case kSchedOnePass: return pick_fused<PREC, kSchedOnePass>(radial, paired, batch);
        case kSchedLagSplit: return pick_fused<PREC, kSchedLagSplit>(radial, paired, batch);
        case kSchedTwoPass:
            if constexpr (PREC == SDC_PREC_SPLIT_BF16 || PREC == SDC_PREC_SPLIT_FP16)
                return pick_fused<PREC, kSchedTwoPass>(radial, paired, batch);
            return nullptr;
        case kSchedFold:
            if constexpr (PREC != SDC_PREC_FP32) return pick_fused<PREC, kSchedFold>(radial, paired, batch);
            return nullptr;
        default: return nullptr;
    }
}

// Kernel of a fused launch, or null for a (precision, schedule) pair that
// does not exist.
static const void* fused_kernel_of(int precision, int sched, int radial, int paired, bool batch) {
    switch (precision) {
        case SDC_PREC_FP32: return pick_sched<SDC_PREC_FP32>(sched, radial, paired, batch);
        case SDC_PREC_BF16X3: return pick_sched<SDC_PREC_BF16X3>(sched, radial, paired, batch);
        case SDC_PREC_SPLIT_BF16: return pick_sched<SDC_PREC_SPLIT_BF16>(sched, radial, paired, batch);
        case SDC_PREC_SPLIT_FP16: return pick_sched<SDC_PREC_SPLIT_FP16>(sched, radial, paired, batch);
        default: return nullptr;
    }
}

int launch_fused(const FusedArgs& a, void* stream) {
    if (a.n_groups * a.n_streams == 0) return 0;
    if (!sched_valid(a.precision, a.sched)) return (int)hipErrorInvalidValue;
    const void* fn = fused_kernel_of(a.precision, a.sched, a.kind == SDC_BINS_RADIAL, a.O8 % 2 == 0, false);
    if (!fn) return (int)hipErrorInvalidValue;
    const int lds = fused_lds_bytes(a.win, a.precision);
    const int n_tasks = a.n_groups * a.n_streams;
    const int grid = 8 * ((n_tasks + 7) / 8);
    void* params[] = {(void*)&a};
    return (int)hipLaunchKernel(fn, dim3(grid), dim3(threads_per_wg(a.sched)), params, lds, (hipStream_t)stream);
}

int batch_grid(int precision, int sched, int radial, int lds, int device, int total, int* grid) {
    const void* fn = fused_kernel_of(precision, sched, radial, 0, true);
    if (!fn) return (int)hipErrorInvalidValue;
    int per_cu = 0, n_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads_per_wg(sched), lds);
    if (e != hipSuccess) return (int)e;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return (int)e;
    if (per_cu < 1) per_cu = 1;
    int64_t g = (int64_t)per_cu * n_cu;
    if (g > total) g = total;
    g = 8 * ((g + 7) / 8);
    *grid = (int)(g < 8 ? 8 : g);
    return 0;
}

int launch_fused_batch(const BatchLaunch& b, void* stream) {
    if (b.total == 0) return 0;
    const void* fn = fused_kernel_of(b.precision, b.sched, b.radial, 0, true);
    if (!fn) return (int)hipErrorInvalidValue;
    int e = launch_zero(b.queue, 8 * sizeof(unsigned), stream);
    if (e != 0) return e;
    const FusedArgs* args = b.args;
    const int64_t* task_start = b.task_start;
    int n_plans = b.n_plans;
    unsigned* queue = b.queue;
    const int32_t* ranges = b.ranges;
    int total = b.total;
    void* params[] = {(void*)&args, (void*)&task_start, (void*)&n_plans, (void*)&queue, (void*)&ranges,
                      (void*)&total};
    return (int)hipLaunchKernel(fn, dim3(b.grid), dim3(threads_per_wg(b.sched)), params, b.lds,
                                (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// exact pair counts
// ---------------------------------------------------------------------------

template <int RADIAL>
__global__ __launch_bounds__(256) void count_kernel(CountArgs a) {
    extern __shared__ unsigned int hcount[];  // [win], then radial edges
    float* e2s = (float*)(hcount + a.win);
    const int tid = threadIdx.x;
    const KStream st = a.streams[blockIdx.x];
    for (int x = tid; x < a.win; x += 256) hcount[x] = 0u;
    if constexpr (RADIAL) {
        for (int x = tid; x < a.n_shells; x += 256) e2s[x] = a.e2[x];
    }
    __syncthreads();
    for (int p = st.p0; p < st.p1; ++p) {
        const KPair pr = a.pairs[p];
        for (int e = tid; e < kTile * kTile; e += 256) {
            const int64_t pi = (int64_t)pr.ti * kTile + (e >> 6);
            const int64_t pj = (int64_t)pr.tj * kTile + (e & 63);
            if (a.perm[pi] < 0 || a.perm[pj] < 0) continue;
            int w;
            if constexpr (RADIAL) {
                const float4 ri = *(const float4*)(a.pos4 + 4 * pi);
                const float4 rj = *(const float4*)(a.pos4 + 4 * pj);
                w = shell_of(dist2_f32(ri.x, ri.y, ri.z, rj.x, rj.y, rj.z), e2s, a.n_shells, a.inv_w);
            } else {
                w = a.gtab[pj] - a.gtab[pi] + pr.shift;
            }
            atomicAdd(&hcount[w], 1u);
        }
    }
    __syncthreads();
    for (int w = tid; w < a.win; w += 256) {
        const unsigned int v = hcount[w];
        if (v == 0u) continue;
        int64_t b;
        if constexpr (RADIAL) {
            b = w;
        } else {
            const int w0 = w / (a.W1 * a.W2);
            const int w1 = (w / a.W2) % a.W1;
            const int w2 = w % a.W2;
            const int k0 = pmod_dev(st.base[0] + w0, a.L0);
            const int k1 = pmod_dev(st.base[1] + w1, a.L1);
            const int k2 = pmod_dev(st.base[2] + w2, a.L2);
            b = ((int64_t)k0 * a.L1 + k1) * a.L2 + k2;
            if (a.kind == SDC_BINS_PERIODIC_BCC) b = 2 * b + st.parity;
        }
        atomicAdd(&a.counts[b], (unsigned long long)v);
    }
}

// One workgroup per tile pair; thread (wave, lane) writes the 16 shells its
// accumulator registers hold in the fused kernel (same row/column mapping).
__global__ __launch_bounds__(256) void radial_keys_kernel(CountArgs a, int64_t n_pairs, uint16_t* __restrict__ keys) {
    __shared__ float e2s[1024];
    const int tid = threadIdx.x;
    for (int x = tid; x < a.n_shells; x += 256) e2s[x] = a.e2[x];
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int wi = wave >> 1, wj = wave & 1, h = lane >> 5, l32 = lane & 31;
    for (int64_t p = blockIdx.x; p < n_pairs; p += gridDim.x) {
        const KPair pr = a.pairs[p];
        const int64_t sj = (int64_t)pr.tj * kTile + wj * 32 + l32;
        const int64_t rowbase = (int64_t)pr.ti * kTile + wi * 32 + 4 * h;
        const float4 pj = *(const float4*)(a.pos4 + 4 * sj);
        uint32_t kw[8];
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
            const float4 p0 = *(const float4*)(a.pos4 + 4 * (rowbase + 8 * (r / 4) + (r % 4)));
            const float4 p1 = *(const float4*)(a.pos4 + 4 * (rowbase + 8 * ((r + 1) / 4) + ((r + 1) % 4)));
            const uint32_t k0 = (uint32_t)shell_of(dist2_f32(p0.x, p0.y, p0.z, pj.x, pj.y, pj.z), e2s, a.n_shells, a.inv_w);
            const uint32_t k1 = (uint32_t)shell_of(dist2_f32(p1.x, p1.y, p1.z, pj.x, pj.y, pj.z), e2s, a.n_shells, a.inv_w);
            kw[r / 2] = k0 | (k1 << 16);
        }
        uint4* dst = (uint4*)(keys + ((p * 4 + wave) * 64 + lane) * 16);
        dst[0] = make_uint4(kw[0], kw[1], kw[2], kw[3]);
        dst[1] = make_uint4(kw[4], kw[5], kw[6], kw[7]);
    }
}

int launch_radial_keys(const CountArgs& a, int64_t n_pairs, uint16_t* keys, void* stream) {
    if (n_pairs == 0) return 0;
    if (a.n_shells > 1024) return (int)hipErrorInvalidValue;
    const int64_t grid = n_pairs < 65536 ? n_pairs : 65536;
    hipLaunchKernelGGL(radial_keys_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, a, n_pairs,
                       keys);
    return (int)hipGetLastError();
}

int launch_count(const CountArgs& a, void* stream) {
    if (a.n_streams == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    const int lds = a.win * 4 + (a.kind == SDC_BINS_RADIAL ? a.n_shells * 4 : 0);
    hipError_t e;
    if (a.kind == SDC_BINS_RADIAL) {
        e = hipFuncSetAttribute((const void*)count_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(count_kernel<1>, dim3(a.n_streams), dim3(256), lds, s, a);
    } else {
        e = hipFuncSetAttribute((const void*)count_kernel<0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(count_kernel<0>, dim3(a.n_streams), dim3(256), lds, s, a);
    }
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// self term: sum_o sum_i S_i(o s) . S_i(o s + t) in FP64
// ---------------------------------------------------------------------------

// Low part of the hi/lo split exactly as the pack kernel forms it.
template <int PREC>
__device__ inline double split_lo(float v) {
    if constexpr (PREC == SDC_PREC_SPLIT_BF16) return (double)bf16_val(bf16_bits(v - bf16_val(bf16_bits(v))));
    else if constexpr (PREC == SDC_PREC_SPLIT_FP16) return (double)f16_val(f16_bits(v - f16_val(f16_bits(v))));
    else return 0.0;
}

// The part of x*y that the reduced-precision contraction leaves out, from
// the pieces the pack kernel forms (FP64, exact): lo*lo for the hi/lo splits;
// mid*lo + lo*mid + lo*lo for the three-piece form.
template <int PREC>
__device__ inline double dropped_product(float x, float y) {
    if constexpr (PREC == SDC_PREC_BF16X3) {
        const float rx = x - bf16_val(bf16_bits(x)), ry = y - bf16_val(bf16_bits(y));
        const double mx = (double)bf16_val(bf16_bits(rx)), my = (double)bf16_val(bf16_bits(ry));
        const double lx = (double)bf16_val(bf16_bits(rx - (float)mx));
        const double ly = (double)bf16_val(bf16_bits(ry - (float)my));
        return mx * ly + lx * my + lx * ly;
    } else {
        return split_lo<PREC>(x) * split_lo<PREC>(y);
    }
}

// Block: up to 16 consecutive sites.  With USE_LDS their whole time series
// sits in LDS; otherwise the samples are read from global memory.
// Thread (site q = tid / 16, lane r = tid % 16) takes lags r, r + 16, ...
// Besides the exact self sum it forms, for split precisions, the lo*lo
// product that the three-product contraction leaves out, restricted to the
// i = j pairs, and adds it to bin 0 (the bin of zero displacement for every
// bin kind).  On the diagonal that term has a fixed sign, so dropping it
// would bias C(0, 0); off the diagonal it is unbiased rounding noise.
template <bool USE_LDS, int PREC>
__global__ __launch_bounds__(256) void self_kernel(SelfArgs a, int sites_per_block) {
    extern __shared__ float ser[];  // [t_need][sites_per_block][3]
    __shared__ double part[1024];
    __shared__ double part_lo[1024];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * sites_per_block;
    const int nsb = (int)((a.n - i0) < sites_per_block ? (a.n - i0) : sites_per_block);
    if constexpr (USE_LDS) {
        for (int64_t x = tid; x < a.t_need * nsb * 3; x += 256) {
            const int64_t f = x / (nsb * 3);
            const int64_t rem = x - f * nsb * 3;
            ser[f * sites_per_block * 3 + rem] = a.frames[(f * a.n + i0) * 3 + rem];
        }
    }
    for (int x = tid; x < a.n_sel; x += 256) {
        part[x] = 0.0;
        part_lo[x] = 0.0;
    }
    __syncthreads();
    const int q = tid / 16, r = tid % 16;
    float mu[3] = {0.0f, 0.0f, 0.0f};  // origin-side average (connected form)
    if (a.mean && q < nsb)
        for (int c = 0; c < 3; ++c) mu[c] = a.mean[4 * (i0 + q) + c];
    if (q < nsb) {
        for (int l = r; l < a.n_sel; l += 16) {
            const int t = a.lags[l];
            double s = 0.0, sl = 0.0;
            for (int o = 0; o < a.n_origins; ++o) {
                const int64_t f0 = (int64_t)o * a.stride, f1 = f0 + t;
                const float* x0;
                const float* x1;
                if constexpr (USE_LDS) {
                    x0 = ser + (f0 * sites_per_block + q) * 3;
                    x1 = ser + (f1 * sites_per_block + q) * 3;
                } else {
                    x0 = a.frames + (f0 * a.n + i0 + q) * 3;
                    x1 = a.frames + (f1 * a.n + i0 + q) * 3;
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float u = x0[c] - mu[c];  // as the pack kernel forms it
                    s += (double)u * (double)x1[c];
                    if constexpr (PREC != SDC_PREC_FP32) sl += dropped_product<PREC>(u, x1[c]);
                }
            }
            if (a.det) {
                atomicAdd(reinterpret_cast<unsigned long long*>(part) + l, to_fixed(s));
                if constexpr (PREC != SDC_PREC_FP32)
                    atomicAdd(reinterpret_cast<unsigned long long*>(part_lo) + l, to_fixed(sl));
            } else {
                atomicAdd(&part[l], s);
                if constexpr (PREC != SDC_PREC_FP32) atomicAdd(&part_lo[l], sl);
            }
        }
    }
    __syncthreads();
    // origin totals live on the device so that replays of a captured
    // accumulate count their origins too
    if (blockIdx.x == 0)
        for (int l = tid; l < a.n_sel; l += 256) a.norg[a.lags[l]] += (double)a.n_origins;
    for (int l = tid; l < a.n_sel; l += 256) {
        if (a.det) {
            atomicAdd(&a.selfq[a.lags[l]], reinterpret_cast<const unsigned long long*>(part)[l]);
            if constexpr (PREC != SDC_PREC_FP32)
                atomicAdd(&a.Hq[(int64_t)a.lags[l] * a.n_bins], reinterpret_cast<const unsigned long long*>(part_lo)[l]);
        } else {
            unsafeAtomicAdd(&a.self[a.lags[l]], part[l]);
            if constexpr (PREC != SDC_PREC_FP32)
                unsafeAtomicAdd(&a.H[(int64_t)a.lags[l] * a.n_bins], part_lo[l]);
        }
    }
}

template <bool USE_LDS>
static void launch_self_kind(const SelfArgs& a, dim3 grid, int lds, hipStream_t s, int spb) {
    switch (a.precision) {
        case SDC_PREC_SPLIT_BF16:
            hipLaunchKernelGGL((self_kernel<USE_LDS, SDC_PREC_SPLIT_BF16>), grid, dim3(256), lds, s, a, spb);
            break;
        case SDC_PREC_SPLIT_FP16:
            hipLaunchKernelGGL((self_kernel<USE_LDS, SDC_PREC_SPLIT_FP16>), grid, dim3(256), lds, s, a, spb);
            break;
        case SDC_PREC_BF16X3:
            hipLaunchKernelGGL((self_kernel<USE_LDS, SDC_PREC_BF16X3>), grid, dim3(256), lds, s, a, spb);
            break;
        default:
            hipLaunchKernelGGL((self_kernel<USE_LDS, SDC_PREC_FP32>), grid, dim3(256), lds, s, a, spb);
            break;
    }
}

// Site-summed spin M(f) = sum_i S_i(f) of every frame the accumulate reads,
// in FP64: one workgroup per frame.
__global__ __launch_bounds__(256) void magnet_kernel(const float* __restrict__ frames, int64_t n,
                                                     double* __restrict__ M) {
    __shared__ double red[3][256];
    const int64_t f = blockIdx.x;
    const float* x = frames + f * n * 3;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        s0 += (double)x[3 * i];
        s1 += (double)x[3 * i + 1];
        s2 += (double)x[3 * i + 2];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) M[f * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// Site-summed correlation of each selected lag: the sum over all ordered
// pairs of S_i(o s) . S_j(o s + t) equals M(o s) . M(o s + t), summed over
// the origins in FP64 (one thread per lag).
// For the connected form the origin side is centred: the sum over all pairs
// of (S_i(o s) - <S_i>) . S_j(o s + t) is (M(o s) - <M>) . M(o s + t).
__global__ __launch_bounds__(256) void msum_kernel(SelfArgs a) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.n_sel) return;
    const int t = a.lags[l];
    double mb[3] = {0.0, 0.0, 0.0};
    if (a.mean) {
        for (int o = 0; o < a.n_origins; ++o)
            for (int c = 0; c < 3; ++c) mb[c] += a.mframe[(int64_t)o * a.stride * 3 + c];
        for (int c = 0; c < 3; ++c) mb[c] /= (double)a.n_origins;
    }
    double s = 0.0;
    for (int o = 0; o < a.n_origins; ++o) {
        const double* m0 = a.mframe + (int64_t)o * a.stride * 3;
        const double* m1 = m0 + (int64_t)t * 3;
        s += (m0[0] - mb[0]) * m1[0] + (m0[1] - mb[1]) * m1[1] + (m0[2] - mb[2]) * m1[2];
    }
    a.msum[t] += s;
}

__global__ __launch_bounds__(256) void mean_kernel(const float* __restrict__ frames, int64_t n, int n_origins,
                                                   int stride, float* __restrict__ mean) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int o = 0; o < n_origins; ++o) {
        const float* x = frames + ((int64_t)o * stride * n + i) * 3;
        s0 += (double)x[0];
        s1 += (double)x[1];
        s2 += (double)x[2];
    }
    const double inv = 1.0 / (double)n_origins;
    mean[4 * i] = (float)(s0 * inv);
    mean[4 * i + 1] = (float)(s1 * inv);
    mean[4 * i + 2] = (float)(s2 * inv);
    mean[4 * i + 3] = 0.0f;
}

int launch_mean(const float* frames, int64_t n, int n_origins, int stride, float* mean, void* stream) {
    hipLaunchKernelGGL(mean_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       frames, n, n_origins, stride, mean);
    return (int)hipGetLastError();
}

int launch_self(const SelfArgs& a, void* stream) {
    if (a.n_sel == 0) return 0;
    if (a.n_sel > 1024) return (int)hipErrorInvalidValue;
    const int64_t budget = kSelfLdsBudget;
    const int64_t per_site = a.t_need * 3 * (int64_t)sizeof(float);
    hipStream_t s = (hipStream_t)stream;
    if (per_site <= budget) {
        int spb = (int)(budget / per_site);
        if (spb > 16) spb = 16;
        const int lds = (int)(a.t_need * spb * 3 * sizeof(float));
        launch_self_kind<true>(a, dim3((unsigned)((a.n + spb - 1) / spb)), lds, s, spb);
    } else {
        launch_self_kind<false>(a, dim3((unsigned)((a.n + 15) / 16)), 0, s, 16);
    }
    hipLaunchKernelGGL(magnet_kernel, dim3((unsigned)a.t_need), dim3(256), 0, s, a.frames, a.n, a.mframe);
    hipLaunchKernelGGL(msum_kernel, dim3((unsigned)((a.n_sel + 255) / 256)), dim3(256), 0, s, a);
    return (int)hipGetLastError();
}

// Dynamic-LDS limits of every kernel that takes more than the default, set
// once per device at plan creation so that the launch paths make no attribute
// calls (they stay legal under stream capture).
int prepare_kernels() {
    for (int prec = SDC_PREC_FP32; prec <= SDC_PREC_BF16X3; ++prec)
        for (int sched = kSchedOnePass; sched <= kSchedFold; ++sched)
            for (int k = 0; k < 6; ++k) {  // (radial, paired) of the single-plan kernels, then the batch ones
                const bool batch = k >= 4;
                const int radial = batch ? (k & 1) : ((k >> 1) & 1), paired = batch ? 0 : (k & 1);
                const void* f = fused_kernel_of(prec, sched, radial, paired, batch);
                if (!f) continue;
                hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxFusedLds);
                if (e != hipSuccess) return (int)e;
            }
    const void* self[] = {(const void*)self_kernel<true, SDC_PREC_FP32>,
                          (const void*)self_kernel<true, SDC_PREC_SPLIT_BF16>,
                          (const void*)self_kernel<true, SDC_PREC_SPLIT_FP16>,
                          (const void*)self_kernel<true, SDC_PREC_BF16X3>};
    for (const void* f : self) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSelfLdsBudget);
        if (e != hipSuccess) return (int)e;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// finalize: normalisation, site sums, windowed DFT (all FP64)
// ---------------------------------------------------------------------------

__global__ void normalize_kernel(FinalArgs a) {
    const int64_t total = (int64_t)a.n_lags * a.n_bins;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = x / a.n_bins;
        const int64_t b = x - t * a.n_bins;
        const double den = a.n_org[t] * (double)a.counts[b];
        a.C[x] = den > 0.0 ? a.H[x] / den : 0.0;
    }
}

// Site-summed and self correlations per lag.  The site sum comes from the
// magnetisation products (an exact identity for the sum of H over all
// bins), which keeps the per-bin rounding of the reduced-precision products
// from adding up over N^2 pairs.
__global__ __launch_bounds__(256) void sums_kernel(FinalArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_lags) return;
    const double d = (double)a.n_sites * a.n_org[t];
    a.csum[t] = d > 0.0 ? a.msum[t] / d : 0.0;
    a.cself[t] = d > 0.0 ? a.self[t] / d : 0.0;
}

__global__ void dft_kernel(FinalArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = a.n_lags;
    if (k >= m) return;
    double re0 = 0, im0 = 0, re1 = 0, im1 = 0;
    for (int t = 0; t < m; ++t) {
        const double w = 0.5 * (1.0 + cospi((double)t / (double)m));
        const int64_t kt = ((int64_t)k * t) % m;
        double sn, cs;
        sincospi(-2.0 * (double)kt / (double)m, &sn, &cs);
        re0 += w * a.csum[t] * cs;
        im0 += w * a.csum[t] * sn;
        re1 += w * a.cself[t] * cs;
        im1 += w * a.cself[t] * sn;
    }
    a.ssum[2 * k] = re0;
    a.ssum[2 * k + 1] = im0;
    a.sself[2 * k] = re1;
    a.sself[2 * k + 1] = im1;
}

// One workgroup per (q, lag): S(q, t) = sum_b exp(-i q.d_b) H(b, t) / (N n_org),
// d_b the displacement of bin b (bcc: the parity adds half a cell on every
// axis).  FP64 throughout; the phase is reduced exactly in integers first.
__global__ __launch_bounds__(256) void sqt_kernel(SqtArgs a) {
    __shared__ double red[2][256];
    const int qi = blockIdx.x, t = blockIdx.y;
    const int64_t m0 = a.m[3 * qi], m1 = a.m[3 * qi + 1], m2 = a.m[3 * qi + 2];
    const bool bcc = a.kind == SDC_BINS_PERIODIC_BCC;
    double re = 0.0, im = 0.0;
    for (int64_t b = threadIdx.x; b < a.n_bins; b += 256) {
        const int64_t c = bcc ? b >> 1 : b;
        const int par = bcc ? (int)(b & 1) : 0;
        const int64_t k0 = c / ((int64_t)a.L1 * a.L2), k1 = (c / a.L2) % a.L1, k2 = c % a.L2;
        // q.d / pi = sum_a 2 m_a (k_a + p/2) / L_a = sum_a m_a (2 k_a + p) / L_a, taken mod 2
        // per axis in integers: m_a (2 k_a + p) mod 2 L_a
        const int64_t n0 = (m0 * (2 * k0 + par)) % (2 * (int64_t)a.L0);
        const int64_t n1 = (m1 * (2 * k1 + par)) % (2 * (int64_t)a.L1);
        const int64_t n2 = (m2 * (2 * k2 + par)) % (2 * (int64_t)a.L2);
        const double x = (double)n0 / a.L0 + (double)n1 / a.L1 + (double)n2 / a.L2;
        double sn, cs;
        sincospi(-x, &sn, &cs);
        const double h = a.H[(int64_t)t * a.n_bins + b];
        re += cs * h;
        im += sn * h;
    }
    red[0][threadIdx.x] = re;
    red[1][threadIdx.x] = im;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double d = (double)a.n_sites * a.n_org[t];
        const int64_t o = ((int64_t)qi * a.n_lags + t) * 2;
        a.sqt[o] = d > 0.0 ? red[0][0] / d : 0.0;
        a.sqt[o + 1] = d > 0.0 ? red[1][0] / d : 0.0;
    }
}

// Windowed DFT over the lags of each q (same window as the site sums).
__global__ void sqw_kernel(const double* __restrict__ sqt, double* __restrict__ sqw, int m) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int qi = blockIdx.y;
    if (k >= m) return;
    const double* x = sqt + (int64_t)qi * m * 2;
    double re = 0.0, im = 0.0;
    for (int t = 0; t < m; ++t) {
        const double w = 0.5 * (1.0 + cospi((double)t / (double)m));
        const int64_t kt = ((int64_t)k * t) % m;
        double sn, cs;
        sincospi(-2.0 * (double)kt / (double)m, &sn, &cs);
        // (x_re + i x_im)(cs + i sn)
        re += w * (x[2 * t] * cs - x[2 * t + 1] * sn);
        im += w * (x[2 * t] * sn + x[2 * t + 1] * cs);
    }
    sqw[((int64_t)qi * m + k) * 2] = re;
    sqw[((int64_t)qi * m + k) * 2 + 1] = im;
}

int launch_sqw(const double* sqt, double* sqw, int n_q, int n_lags, void* stream) {
    if (n_q == 0) return 0;
    hipLaunchKernelGGL(sqw_kernel, dim3((unsigned)((n_lags + 63) / 64), (unsigned)n_q), dim3(64), 0,
                       (hipStream_t)stream, sqt, sqw, n_lags);
    return (int)hipGetLastError();
}

int launch_sqt(const SqtArgs& a, void* stream) {
    if (a.n_q == 0) return 0;
    hipLaunchKernelGGL(sqt_kernel, dim3((unsigned)a.n_q, (unsigned)a.n_lags), dim3(256), 0, (hipStream_t)stream, a);
    const int e = (int)hipGetLastError();
    return e != 0 ? e : launch_sqw(a.sqt, a.sqw, a.n_q, a.n_lags, stream);
}

int launch_finalize(const FinalArgs& a, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (a.C) {
        const int64_t total = (int64_t)a.n_lags * a.n_bins;
        int64_t blocks = (total + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(sums_kernel, dim3((a.n_lags + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(dft_kernel, dim3((a.n_lags + 63) / 64), dim3(64), 0, s, a);
    return (int)hipGetLastError();
}

__global__ void zero_kernel(uint32_t* p, int64_t words) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < words;
         x += (int64_t)gridDim.x * blockDim.x)
        p[x] = 0u;
}

__global__ void fixed_to_double_kernel(const unsigned long long* __restrict__ q, double* __restrict__ d, int64_t n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        d[x] = (double)(long long)q[x] / kFixedScale;
}

__global__ void double_to_fixed_kernel(const double* __restrict__ d, unsigned long long* __restrict__ q, int64_t n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        q[x] = to_fixed(d[x]);
}

static int64_t grid_for(int64_t n) {
    int64_t blocks = (n + 255) / 256;
    return blocks > 8192 ? 8192 : (blocks < 1 ? 1 : blocks);
}

int launch_fixed_to_double(const unsigned long long* q, double* d, int64_t n, void* stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(fixed_to_double_kernel, dim3((unsigned)grid_for(n)), dim3(256), 0, (hipStream_t)stream, q, d, n);
    return (int)hipGetLastError();
}

int launch_double_to_fixed(const double* d, unsigned long long* q, int64_t n, void* stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(double_to_fixed_kernel, dim3((unsigned)grid_for(n)), dim3(256), 0, (hipStream_t)stream, d, q, n);
    return (int)hipGetLastError();
}

int launch_zero(void* ptr, int64_t bytes, void* stream) {
    if (bytes <= 0) return 0;
    const int64_t words = bytes / 4;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t*)ptr, words);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// trajectory: Philox starts and LL RK4
// ---------------------------------------------------------------------------

__device__ inline float u24(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

// Independent uniform unit vectors for every (frame, site): Philox4x32-10,
// key = seed, counter = (site low, frame, site high, 7); z = 2u0 - 1,
// phi = 2 pi u1 (the autotuner's input; any spins time the same).
__global__ void unit_spins_kernel(float* __restrict__ out, int64_t n, int64_t n_frames, uint64_t seed) {
    const int64_t total = n * n_frames;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = x / n, i = x - f * n;
        uint32_t c[4] = {(uint32_t)i, (uint32_t)f, (uint32_t)((uint64_t)i >> 32), 7u};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double z = 2.0 * ((double)(c[0] >> 8) * (1.0 / 16777216.0)) - 1.0;
        const double r = sqrt(fmax(0.0, 1.0 - z * z));
        double sn, cs;
        sincospi(2.0 * ((double)(c[1] >> 8) * (1.0 / 16777216.0)), &sn, &cs);
        out[3 * x] = (float)(r * cs);
        out[3 * x + 1] = (float)(r * sn);
        out[3 * x + 2] = (float)z;
    }
}

int launch_unit_spins(float* out, int64_t n, int64_t n_frames, uint64_t seed, void* stream) {
    const int64_t total = n * n_frames;
    if (total <= 0) return 0;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(unit_spins_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, out, n,
                       n_frames, seed);
    return (int)hipGetLastError();
}

__global__ void traj_init_kernel(TrajArgs a, float* S) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    double x, y, z;
    if (a.init == SDC_INIT_GIVEN) {
        x = a.init_dev[3 * i];
        y = a.init_dev[3 * i + 1];
        z = a.init_dev[3 * i + 2];
    } else {
        uint32_t c[4] = {(uint32_t)i, 0u, (uint32_t)((uint64_t)i >> 32), 0u};
        philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
        const double u0 = (double)(c[0] >> 8) * (1.0 / 16777216.0);
        const double u1 = (double)(c[1] >> 8) * (1.0 / 16777216.0);
        if (a.init == SDC_INIT_UNIFORM) {
            z = 2.0 * u0 - 1.0;
            const double r = sqrt(fmax(0.0, 1.0 - z * z));
            double sn, cs;
            sincospi(2.0 * u1, &sn, &cs);
            x = r * cs;
            y = r * sn;
        } else {
            const double rr = sqrt(-2.0 * log(1.0 - u0));
            double sn, cs;
            sincospi(2.0 * u1, &sn, &cs);
            const double v0 = a.sigma * rr * cs, v1 = a.sigma * rr * sn;
            const double ang = sqrt(v0 * v0 + v1 * v1);
            const double f = ang > 0.0 ? sin(ang) / ang : 1.0;
            x = f * v0;
            y = f * v1;
            z = cos(ang);
        }
    }
    S[3 * i] = (float)x;
    S[3 * i + 1] = (float)y;
    S[3 * i + 2] = (float)z;
    a.frames[3 * i] = (float)x;
    a.frames[3 * i + 1] = (float)y;
    a.frames[3 * i + 2] = (float)z;
}

// One RK4 stage: k = h_i x X_i with the effective field of Eq. (1),
// h_i = sum_j (J_ij X_j + D_ij x X_j) - 2 A X_i^z z - H_z z.
//  stage 0: acc = k;      Tout = S + dt/2 k
//  stage 1: acc += 2k;    Tout = S + dt/2 k
//  stage 2: acc += 2k;    Tout = S + dt k
//  stage 3: S += dt/6 (acc + k), frame written
__global__ __launch_bounds__(256) void traj_stage_kernel(TrajArgs a, int stage, float* S,
                                                         const float* X, float* Tout, float* acc,
                                                         float* frame) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    float h0 = 0.f, h1 = 0.f, h2 = 0.f;
    for (int e = 0; e < a.z_max; ++e) {
        const int32_t j = a.nbr[i * a.z_max + e];
        if (j < 0) continue;
        const float J = a.jval[i * a.z_max + e];
        const float y0 = X[3 * (int64_t)j], y1 = X[3 * (int64_t)j + 1], y2 = X[3 * (int64_t)j + 2];
        h0 += J * y0;
        h1 += J * y1;
        h2 += J * y2;
        if (a.dvec) {
            const float* d = a.dvec + 3 * (i * a.z_max + e);
            h0 += d[1] * y2 - d[2] * y1;
            h1 += d[2] * y0 - d[0] * y2;
            h2 += d[0] * y1 - d[1] * y0;
        }
    }
    const float x0 = X[3 * i], x1 = X[3 * i + 1], x2 = X[3 * i + 2];
    h2 += -a.aniso2 * x2 - a.hz;
    const float k0 = h1 * x2 - h2 * x1;
    const float k1 = h2 * x0 - h0 * x2;
    const float k2 = h0 * x1 - h1 * x0;
    const float s0 = S[3 * i], s1 = S[3 * i + 1], s2 = S[3 * i + 2];
    if (stage == 0) {
        acc[3 * i] = k0;
        acc[3 * i + 1] = k1;
        acc[3 * i + 2] = k2;
    } else if (stage < 3) {
        acc[3 * i] += 2.f * k0;
        acc[3 * i + 1] += 2.f * k1;
        acc[3 * i + 2] += 2.f * k2;
    }
    if (stage < 3) {
        const float c = stage == 2 ? a.dt : 0.5f * a.dt;
        Tout[3 * i] = s0 + c * k0;
        Tout[3 * i + 1] = s1 + c * k1;
        Tout[3 * i + 2] = s2 + c * k2;
    } else {
        const float c = a.dt / 6.0f;
        const float n0 = s0 + c * (acc[3 * i] + k0);
        const float n1 = s1 + c * (acc[3 * i + 1] + k1);
        const float n2 = s2 + c * (acc[3 * i + 2] + k2);
        S[3 * i] = n0;
        S[3 * i + 1] = n1;
        S[3 * i + 2] = n2;
        frame[3 * i] = n0;
        frame[3 * i + 1] = n1;
        frame[3 * i + 2] = n2;
    }
}

int launch_traj(const TrajArgs& a, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const unsigned grid = (unsigned)((a.n + 255) / 256);
    float* S = a.work;
    float* T1 = a.work + 3 * a.n;
    float* T2 = a.work + 6 * a.n;
    float* acc = a.work + 9 * a.n;
    hipLaunchKernelGGL(traj_init_kernel, dim3(grid), dim3(256), 0, s, a, S);
    for (int64_t f = 1; f < a.n_frames; ++f) {
        float* frame = a.frames + f * a.n * 3;
        hipLaunchKernelGGL(traj_stage_kernel, dim3(grid), dim3(256), 0, s, a, 0, S, (const float*)S, T1, acc, frame);
        hipLaunchKernelGGL(traj_stage_kernel, dim3(grid), dim3(256), 0, s, a, 1, S, (const float*)T1, T2, acc, frame);
        hipLaunchKernelGGL(traj_stage_kernel, dim3(grid), dim3(256), 0, s, a, 2, S, (const float*)T2, T1, acc, frame);
        hipLaunchKernelGGL(traj_stage_kernel, dim3(grid), dim3(256), 0, s, a, 3, S, (const float*)T1, T2, acc, frame);
    }
    return (int)hipGetLastError();
}

}  // namespace sdc
