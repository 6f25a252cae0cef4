// Internal declarations of the sdc library: tile layout, kernel arguments and
// launch wrappers.  Not part of the public ABI (include/sdc.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "sdc.h"

namespace sdc {

// Sites are grouped in tiles of 64.  Periodic lattices: a tile is a brick of
// at most 4x4x4 cells of one sublattice, slot (ox*4 + oy)*4 + oz.  Radial:
// 64 consecutive points in Morton order.  Unused slots are padding (zero
// spins, no counts).
constexpr int kTile = 64;
// Lags handled together by one fused task (consecutive lag indices u): 8
// for the reduced-precision forms (128 accumulator registers per wave for
// one set of sums), 16 for FP32 (its MFMA is 16x slower per flop, so operand
// reuse across more lags matters more than overlap).
constexpr int lag_group(int precision) { return precision == SDC_PREC_FP32 ? 16 : 8; }
// Schedules of the fused product (a tuning choice per plan and batch; the
// results differ only by rounding).  The small products of the reduced forms
// always get sums of their own (see the pass constants of the kernel).
//  kSchedOnePass: every product in one K loop per tile pair; the reduced
//    forms keep a second accumulator set for the small products (256
//    registers), so one workgroup fits on a CU; three-stage register
//    prefetch.  Every precision has it.
//  kSchedTwoPass: hi/lo splits only: per tile pair one K loop for hi*lo +
//    lo*hi from zero, then one for hi*hi on top of those sums, in the same
//    128 registers, then the histogram adds; two workgroups per CU, so one
//    workgroup's epilogue and memory waits overlap the other's MFMAs.
//  kSchedLagSplit: one K loop as in kSchedOnePass, but workgroups of eight
//    waves in which two waves share each 32x32 quadrant and take half of the
//    lag group each: 2 x 64 accumulator registers for the reduced forms (128
//    for FP32), two waves per SIMD.  Every precision.
//  kSchedFold: reduced forms only: one K loop; per K-step and lag the
//    small products are summed from zero in a transient 32x32 tile and added
//    to the large sums with FP32 vector adds (round to nearest, no bias),
//    beside the hi*hi MFMA; 128 accumulator registers, two workgroups per
//    CU.
constexpr int kSchedOnePass = 0, kSchedTwoPass = 1, kSchedLagSplit = 2, kSchedFold = 3;
constexpr int threads_per_wg(int sched) { return sched == kSchedLagSplit ? 512 : 256; }
// Register buffers of the K loops (loads of NS - 1 K-steps ahead in flight).
// At two workgroups per CU the other workgroup covers the rest of the load
// latency: two to six buffers in either loop of the two-pass schedule time
// the same (1085-1102 ms at sc 36^3), so the fewest registers win.
constexpr int kStagesOnePass = 3, kStagesTwoPassSmall = 2, kStagesTwoPassLarge = 2, kStagesFold = 2;
// Kernel schedule of a public sdc_schedule (ONE_PASS or TWO_PASS).
constexpr int sched_index(int schedule) {
    return schedule == SDC_SCHED_TWO_PASS  ? kSchedTwoPass
           : schedule == SDC_SCHED_LAG_SPLIT ? kSchedLagSplit
           : schedule == SDC_SCHED_FOLD      ? kSchedFold
                                             : kSchedOnePass;
}
constexpr int wg_per_cu(int sched) { return sched == kSchedTwoPass || sched == kSchedFold ? 2 : 1; }
// Waves per SIMD at that occupancy: the launch-bounds minimum that sets the
// register budget (four SIMDs per CU, 64-lane waves).
constexpr int waves_per_simd(int sched) { return wg_per_cu(sched) * threads_per_wg(sched) / 256; }
constexpr bool sched_valid(int precision, int sched) {
    return sched == kSchedOnePass || sched == kSchedLagSplit ||
           (sched == kSchedTwoPass && (precision == SDC_PREC_SPLIT_BF16 || precision == SDC_PREC_SPLIT_FP16)) ||
           (sched == kSchedFold && precision != SDC_PREC_FP32);
}
// Pack elements (8 samples each) in one lane's B window: LG - 1 + 8 samples.
constexpr int win_blocks(int lg) { return (lg + 14) / 8; }
// Origins per pack block; a K-step of the fused product takes two blocks
// (one per lane half of the 32x32 MFMA), running over the blocks of all three
// components in turn.
constexpr int kOriginBlock = 8;

// One tile pair of a stream: i-tile, j-tile and the window shift of this pair.
struct KPair {
    int32_t ti, tj, shift, pad;
};

// A stream is a run of tile pairs whose epilogue shares one LDS histogram.
// Periodic: all pairs (I, I + db) for a fixed brick offset db and fixed
// sublattices; the histogram is indexed by the window coordinate and maps to
// global bins through base/parity.  Radial: all pairs (I, J) of one I; the
// histogram is indexed by shell.
struct KStream {
    int32_t p0, p1;
    int32_t base[3];
    int32_t parity;
    int32_t pad[2];
};

// Lag group: lags t = s*(u0 + m) + phase for m in [0, 16) with bit m of mask.
struct KGroup {
    int32_t phase, u0, mask, pad;
};

struct Layout {
    int kind = 0;
    int L[3] = {0, 0, 0};
    int64_t n = 0;
    int64_t n_bins = 0;
    int64_t n_pad = 0;
    int32_t n_tiles = 0;
    int W[3] = {1, 1, 1};   // periodic window extents
    int win = 0;            // histogram bins per lag (window size or n_shells)
    int n_shells = 0;
    std::vector<int32_t> perm;   // [n_pad] original site index, -1 = padding
    std::vector<int32_t> gtab;   // [n_pad] window coordinate of the slot
    std::vector<float> pos4;     // [n_pad][4] radial positions, packed order
    std::vector<float> e2;       // [n_shells] radial squared edges
    std::vector<KPair> pairs;
    std::vector<KStream> streams;
};

// Records the thread-local error text returned by sdc_last_error(); returns s.
sdc_status set_error(sdc_status s, const std::string& msg);

// Builds the tile layout of a sample, streams cut into segments of at most
// segment_pairs tile pairs.  Returns SDC_OK or an error with text.
sdc_status build_layout(const float* pos, int64_t n, const sdc_bin_spec* spec, int segment_pairs,
                        Layout* out, std::string* err);

// Default tile pairs per fused task: periodic streams cut into segments of
// 96 pairs, radial streams (all j-tiles of an i-tile) whole.
constexpr int kDefaultSegmentPeriodic = 96;
constexpr int kMaxSegmentPairs = 1 << 20;
constexpr int default_segment_pairs(int kind) {
    return kind == SDC_BINS_RADIAL ? kMaxSegmentPairs : kDefaultSegmentPeriodic;
}

// Tuning a plan runs with (sdc_tune.cpp): the caller's fields where set,
// else the entry of the tuning file named by SDC_TUNING_FILE for the plan's
// size class, else the defaults.  Every field of *out is set (no zeros).
sdc_status resolve_tuning(const sdc_tuning* given, int64_t n_sites, const sdc_bin_spec* bins,
                          const sdc_corr_spec* corr, int device, sdc_tuning* out);

// Global bin of window coordinate w of stream s (periodic kinds).
int64_t window_bin(const Layout& lay, const KStream& s, int w);

// Radial shell of a squared distance: the largest k with e2[k] <= d2.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline int shell_of(float d2, const float* e2, int n_shells, float inv_w) {
    // first guess from the square root, then move to the exact rule
    float r = __builtin_sqrtf(d2);
    int k = (int)(r * inv_w);
    if (k < 0) k = 0;
    if (k > n_shells - 1) k = n_shells - 1;
    while (k > 0 && e2[k] > d2) --k;
    while (k + 1 < n_shells && e2[k + 1] <= d2) ++k;
    return k;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor bijection with Weyl key increments.  c is updated in place.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// FP32 squared distance in the fixed order ((dx*dx + dy*dy) + dz*dz), no
// contraction.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline float dist2_f32(float xi, float yi, float zi, float xj, float yj, float zj) {
#pragma clang fp contract(off)
    float dx = xj - xi;
    float dy = yj - yi;
    float dz = zj - zi;
    float a = dx * dx;
    float b = dy * dy;
    float c = dz * dz;
    return (a + b) + c;
}

// ---------------------------------------------------------------------------
// Kernel launch wrappers (sdc_kernels.hip).  All return hipError_t as int.
// ---------------------------------------------------------------------------

struct PackArgs {
    const float* frames;  // [n_frames][n][3]
    int64_t n, n_frames, n_pad;
    const int32_t* perm;  // [n_pad]
    int n_origins, stride, precision;
    int O8;               // origin blocks of 8 in the A pack (per component)
    int F8;               // frame blocks of 8 in each B phase pack
    int n_phase;          // = stride
    int64_t frames_valid; // frames usable: min(n_frames, required)
    const float* mean;    // [n][4] per-site origin averages subtracted from A, or null
    void* A;              // [3][O8][n_pad] x 32 B
    void* B;              // [n_phase][3][F8][n_pad] x 32 B
};
int launch_pack(const PackArgs& a, void* stream);

struct FusedArgs {
    const void* A;
    const void* B;
    int64_t n_pad;
    int O8, F8;                    // origin blocks per component (A), window blocks (B)
    int nk;                        // K-steps: ceil(3 O8 / 2)
    int64_t phase_stride;          // elements of 32 B per B phase
    const KPair* pairs;
    const KStream* streams;
    int n_streams;
    const KGroup* groups;
    int n_groups;
    const int32_t* gtab;
    const float* pos4;
    const uint16_t* keys;          // radial: per-pair key tiles, or null (computed in the epilogue)
    const float* e2;
    int n_shells;
    float inv_w;
    int kind, L0, L1, L2, W1, W2, win;
    double* H;
    int det;                       // deterministic mode: fixed-point bins in Hq
    unsigned long long* Hq;
    int64_t n_bins;
    int stride;
    int precision;
    int sched;                     // kSchedOnePass / kSchedTwoPass
};
int launch_fused(const FusedArgs& a, void* stream);

// One persistent launch over the tasks of several plans (same precision and
// bin class): args[n_plans] and task_start[n_plans + 1] in device memory,
// queue = 8 device counters (zeroed by the launch itself).
struct BatchLaunch {
    const FusedArgs* args;
    const int64_t* task_start;
    int n_plans;
    unsigned* queue;
    const int32_t* ranges;  // [9]: XCD queue x holds tasks [ranges[x], ranges[x + 1])
    int total;
    int precision, radial, sched;
    int lds, grid;
};
int launch_fused_batch(const BatchLaunch& b, void* stream);
// Workgroups that fit on the device at once (a multiple of 8, at most `total`
// rounded up to 8).
int batch_grid(int precision, int sched, int radial, int lds, int device, int total, int* grid);

struct CountArgs {
    const KPair* pairs;
    const KStream* streams;
    int n_streams;
    const int32_t* perm;
    const int32_t* gtab;
    const float* pos4;
    const float* e2;
    int n_shells;
    float inv_w;
    int kind, L0, L1, L2, W1, W2, win;
    unsigned long long* counts;
};
int launch_count(const CountArgs& a, void* stream);
// Radial key table: keys[((p*4 + wave)*64 + lane)*16 + r] = shell of the pair
// element that accumulator register r of that lane holds for tile pair p.
int launch_radial_keys(const CountArgs& a, int64_t n_pairs, uint16_t* keys, void* stream);

struct SelfArgs {
    const float* frames;
    int64_t n, n_frames;
    int n_origins, stride;
    const int32_t* lags;  // device [n_sel]
    int n_sel;
    int64_t t_need;       // frames read: (n_origins - 1) * stride + max lag + 1
    double* self;         // [n_lags] indexed by lag value
    int precision;        // split precisions: add the diagonal lo*lo term to H
    double* H;            // [n_lags][n_bins]; the i = j pairs all fall in bin 0
    int64_t n_bins;
    double* norg;         // [n_lags] origin totals, += n_origins per selected lag
    double* mframe;       // [t_need][3] scratch: site-summed spin of each frame
    double* msum;         // [n_lags] += sum_o M(o s) . M(o s + t)
    const float* mean;    // [n][4] origin averages (connected form), or null
    int det;              // deterministic mode: fixed-point self sums and bins
    unsigned long long* selfq;
    unsigned long long* Hq;
};
int launch_self(const SelfArgs& a, void* stream);
// Per-site averages over the origins of one accumulate (connected form):
// mean[4 i + c] = fp32((1/n_o) sum_o S_i^c(o s)), summed in FP64.
int launch_mean(const float* frames, int64_t n, int n_origins, int stride, float* mean, void* stream);

struct FinalArgs {
    const double* H;
    const unsigned long long* counts;
    const double* n_org;   // device [n_lags]
    const double* self;    // device [n_lags]
    const double* msum;    // device [n_lags] site-summed raw correlation
    int64_t n_bins, n_sites;
    int n_lags;
    double* C;             // [n_lags][n_bins] or null
    double* csum;          // [n_lags]
    double* cself;         // [n_lags]
    double* ssum;          // [n_lags][2]
    double* sself;         // [n_lags][2]
};
int launch_finalize(const FinalArgs& a, void* stream);

// S(q, t) of Eq. (3) from the bins of a periodic plan, for wave vectors
// q_a = 2 pi m_a / L_a (integer m), and its windowed time transform.
struct SqtArgs {
    const double* H;       // [n_lags][n_bins]
    const double* n_org;   // [n_lags]
    int64_t n_bins, n_sites;
    int n_lags;
    int kind, L0, L1, L2;  // periodic bin enumeration (sc / bcc)
    const int32_t* m;      // [n_q][3]
    int n_q;
    double* sqt;           // [n_q][n_lags][2]
    double* sqw;           // [n_q][n_lags][2]
};
int launch_sqt(const SqtArgs& a, void* stream);
// Windowed time transform of S(q, t) for every q (the window of the site sums):
// sqw[q][k] = sum_t w_t sqt[q][t] exp(-2 pi i k t / n_lags), (re, im) pairs.
int launch_sqw(const double* sqt, double* sqw, int n_q, int n_lags, void* stream);

// q-resolved S(q, t) of Eq. (3) at arbitrary wave vectors (sdc_sq.hip).
struct SqTransformArgs {
    const float* frames;      // [>= n_frames_used][n][3] fp32, caller's site order (pack input)
    double* packed;           // [ceil(n / chunk)][t_pad][chunk][3] FP64, chunk = sq_site_chunk() (pack output, contraction input)
    int t_pad;                // n_frames_used rounded up to whole 48-frame column blocks
    const float* pos;         // [n][3] fp32
    const double* q;          // [n_q][3]
    int64_t n;
    int n_q;
    int n_frames_used;        // (n_origins - 1) * stride + n_lags
    int n_split;              // site ranges, one partial transform each
    int64_t sites_per_split;
    double* part;             // [n_split][n_q][2][3 n_frames_used]
};
struct SqCorrArgs {
    double* F;                // [n_q][n_frames_used][3][2], written by the range sum
    int n_q;
    int64_t n_cols;           // 3 n_frames_used
    int n_origins, stride, n_lags;
    int connected;
    double* raw;              // [n_q][n_lags][2], accumulated
    double* n_org;            // [1] origins accumulated
};
// Workgroups of the transform per site range, and the sites one workgroup
// stages per step (site ranges are multiples of it).
int64_t sq_tiles_per_split(int n_q, int n_frames_used);
// Set the contraction kernel's dynamic-LDS limit on the current device.
int prepare_sq_kernels();
int sq_site_chunk();
int sq_frames_per_block();
// Packs the frames site-chunk-major in FP64 (a.frames -> a.packed).
int launch_sq_pack(const SqTransformArgs& a, void* stream);
// The phase contraction alone (partial transforms of the site ranges).
int launch_sq_transform(const SqTransformArgs& a, void* stream);
// Sum of the site ranges into a.F, then the origin correlation.
int launch_sq_corr(const SqTransformArgs& t, const SqCorrArgs& a, void* stream);
int launch_sq_finalize(const double* raw, const double* n_org, int64_t n_sites, int n_q, int n_lags, double* sqt,
                       double* sqw, void* stream);

int launch_zero(void* ptr, int64_t bytes, void* stream);

// Fixed device scratch of the entry points that allocate nothing
// (sdc_static.hip): kStaticScratchBytes per device, shared by every call on
// that device.  static_scratch() returns the device address of `device`'s
// copy, looked up on the first call for that device (with it current).
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
int static_scratch(int device, void** ptr);

// Deterministic mode: every sum that several threads add into is kept as a
// two's-complement 64-bit fixed-point number with 2^-20 resolution, so
// integer atomics make the result independent of the order of the adds.
constexpr double kFixedScale = 1048576.0;
int launch_fixed_to_double(const unsigned long long* q, double* d, int64_t n, void* stream);
int launch_double_to_fixed(const double* d, unsigned long long* q, int64_t n, void* stream);

struct TrajArgs {
    int64_t n;
    int z_max;                 // neighbours per site (ELL width)
    const int32_t* nbr;        // [n][z_max], -1 = none
    const float* jval;         // [n][z_max]
    const float* dvec;         // [n][z_max][3] DMI vectors D_ij, or null
    float aniso2, hz;          // 2 A and H_z of Eq. (1)
    float dt;
    int init, pad;
    double sigma;
    uint64_t seed;
    const float* init_dev;
    float* frames;             // [n_frames][n][3]
    int64_t n_frames;
    float* work;               // [5][n][3] fp32 scratch: S, T, acc, k
};
int launch_traj(const TrajArgs& a, void* stream);
// Seeded independent uniform unit vectors, [n_frames][n][3] fp32.
int launch_unit_spins(float* out, int64_t n, int64_t n_frames, uint64_t seed, void* stream);

// Metropolis sweeps (sdc_mc.hip).
struct McArgs {
    int64_t n;
    int z_max;
    const int32_t* site_of;    // [n] site of each slot (slots colour-major)
    const int32_t* nbr;        // [n slots][z_max] neighbour slots, -1 = none
    const float* jval;         // [n slots][z_max]
    const float* dvec;         // [n slots][z_max][3] DMI vectors, or null
    double A, Hz;              // anisotropy and field of Eq. (1)
    uint64_t seed;             // Philox key of the moves
    double acc_target;         // acceptance-rate target of the cone adaptation
    double* S;                 // [n slots][3] FP64 state
    double* cone;              // [2]: cone half-angle, its cosine
    unsigned long long* accepted;  // accepted moves of the current sweep (mc_counter_bytes())
    // Lattice stencil (set only when the host has checked that it reproduces
    // the tables above slot for slot): periodic sc box L0 x L1 x L2, every edge
    // even, site (x L1 + y) L2 + z, two colour classes (the checkerboard),
    // class c in slots c n/2 .. (c + 1) n/2 in site order, bonds +x, -x, +y,
    // -y, +z, -z with coupling st_j and DMI vectors (st_dp, st_dz, st_dz)
    // rotated onto each axis, st_dn for the negative directions.
    int stencil;
    int L0, L1, L2;
    float st_j, st_dp, st_dn, st_dz;
};
int mc_energy_blocks(int64_t n);
size_t mc_counter_bytes();
// Loads init (fp32, or keeps the FP64 state when init is null), sets the cone.
int launch_mc_setup(const McArgs& a, const float* init, double cone0, void* stream);
// One sweep: every colour class in order (class c = slots class_start[c] ..
// class_start[c + 1]), then the cone update (history[sweep] receives the
// accepted moves when history is not null).
int launch_mc_sweep(const McArgs& a, const int64_t* class_start, int n_classes, double T, int64_t sweep,
                    long long* history, void* stream);
// Energy per site, final cone and temperature into info[0..2]; state as fp32.
int launch_mc_finish(const McArgs& a, double* partial, double T_last, float* out, double* info, void* stream);

int fused_lds_bytes(int win, int precision);
// Largest dynamic LDS of a fused launch (the CU's 160 KB less room for the
// batch kernel's few static words) and the self kernel's staging budget.
constexpr int kMaxFusedLds = 160 * 1024 - 256;
constexpr int64_t kSelfLdsBudget = 96 * 1024;
// Set the kernels' dynamic-LDS limits on the current device.
int prepare_kernels();

}  // namespace sdc
