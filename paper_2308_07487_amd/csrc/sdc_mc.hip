// Metropolis Monte Carlo with an adaptive trial cone and simulated annealing
// (Sec. 2.1, Sec. 4.3) on the Hamiltonian of Eq. (1), on gfx950.
//
// Sites are split into colour classes that share no bond (greedy colouring
// on the host), so one class is updated in parallel, one thread per site.
// The state is FP64 and stored colour-major: slot k holds site site_of[k],
// the slots of one class are contiguous and the bond tables are in slot
// order with neighbours given as slots, so a class's own states, bond
// tables and its neighbours' states are read as contiguous runs.  Every random number is a Philox4x32-10 draw of the
// (site, sweep) counter, so a sweep's result does not depend on the order in
// which threads run; the cone and the acceptance counter live in device
// memory and are updated by a one-thread kernel after each sweep, so a whole
// schedule is queued without host round trips.
#include <hip/hip_runtime.h>

#include "sdc_internal.h"

namespace sdc {

namespace {

constexpr double kPi = 3.14159265358979323846;
// The accepted moves of a sweep are counted in kMcCounters counters, one per
// 128-byte line (workgroup b adds to counter b mod kMcCounters), so that the
// workgroups' atomics do not all queue on one address.
constexpr int kMcCounters = 64;
constexpr int kMcCounterStride = 16;  // u64 words between counters

// One colour class of one sweep.  Site i's move: trial spin in a cone of
// half-angle `cone` about S_i (cos a uniform in [cos cone, 1], azimuth
// uniform), Metropolis acceptance at temperature T.  Counter = (i low,
// sweep low, i high, 2^31 | sweep high), key = seed: u_k = (w_k + 1/2) 2^-32.
// Workgroups go to the 8 XCDs in turn; workgroup b takes block
// x q + min(x, r) + b / 8 of the class (x = b mod 8, nb = 8 q + r blocks), so
// each XCD sweeps one contiguous stretch of slots in order and its L2 keeps
// the neighbour planes that the following slots read again.
// STENCIL: the site and its neighbours' slots follow from the slot by
// lattice arithmetic (McArgs::stencil), so the slot -> site map and the bond
// tables are not read; the sums run over the bonds in table order with the
// table's values, so both forms give the same bits.
template <int STENCIL>
__global__ __launch_bounds__(256) void mc_colour_kernel(McArgs a, int64_t k0, int64_t count, double T,
                                                        int64_t sweep) {
    const int64_t nb = gridDim.x, q = nb / 8, r = nb % 8, x = blockIdx.x % 8;
    const int64_t lb = x * q + (x < r ? x : r) + blockIdx.x / 8;
    const int64_t t = lb * blockDim.x + threadIdx.x;
    bool accepted = false;
    if (t < count) {
        const int64_t k = k0 + t;           // slot
        int64_t i;                          // site index: the Philox counter
        // field of the neighbours: sum_j (J_ij S_j + D_ij x S_j)
        double w0 = 0.0, w1 = 0.0, w2 = 0.0;
        auto bond = [&](int64_t j, double J, double d0, double d1, double d2, bool dmi) {
            const double y0 = a.S[3 * j], y1 = a.S[3 * j + 1], y2 = a.S[3 * j + 2];
            w0 += J * y0;
            w1 += J * y1;
            w2 += J * y2;
            if (dmi) {
                w0 += d1 * y2 - d2 * y1;
                w1 += d2 * y0 - d0 * y2;
                w2 += d0 * y1 - d1 * y0;
            }
        };
        if constexpr (STENCIL) {
            // class c = (k0 > 0) holds the sites of parity c of x + y + z in
            // site order; with L2 even its t-th site is 2t or 2t + 1
            const int64_t half = a.n / 2, s0 = 2 * t;
            const int64_t row = s0 / a.L2, z0 = s0 - row * a.L2;
            const int64_t y = row % a.L1, xx = row / a.L1;
            const int64_t dl = (k0 > 0 ? 1 : 0) ^ ((xx + y) & 1);
            const int64_t z = z0 + dl;
            i = s0 + dl;
            const int64_t other = k0 > 0 ? 0 : half;  // first slot of the neighbours' class
            const int64_t xp = xx + 1 < a.L0 ? xx + 1 : 0, xm = xx > 0 ? xx - 1 : a.L0 - 1;
            const int64_t yp = y + 1 < a.L1 ? y + 1 : 0, ym = y > 0 ? y - 1 : a.L1 - 1;
            const int64_t zp = z + 1 < a.L2 ? z + 1 : 0, zm = z > 0 ? z - 1 : a.L2 - 1;
            const int64_t rxy = row * a.L2;  // (x L1 + y) L2
            const int64_t sj[6] = {((xp * a.L1 + y) * a.L2 + z), ((xm * a.L1 + y) * a.L2 + z),
                                   ((xx * a.L1 + yp) * a.L2 + z), ((xx * a.L1 + ym) * a.L2 + z),
                                   rxy + zp, rxy + zm};
            const bool dmi = a.dvec != nullptr;
            const double J = a.st_j, dp = a.st_dp, dn = a.st_dn, dz = a.st_dz;
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const double dd = (e & 1) ? dn : dp;
                bond(other + (sj[e] >> 1), J, e / 2 == 0 ? dd : dz, e / 2 == 1 ? dd : dz, e / 2 == 2 ? dd : dz, dmi);
            }
        } else {
            i = a.site_of[k];
            for (int e = 0; e < a.z_max; ++e) {
                const int32_t j = a.nbr[k * a.z_max + e];
                if (j < 0) continue;
                const float* d = a.dvec ? a.dvec + 3 * (k * a.z_max + e) : nullptr;
                bond(j, a.jval[k * a.z_max + e], d ? d[0] : 0.0, d ? d[1] : 0.0, d ? d[2] : 0.0, d != nullptr);
            }
        }
        double* si = a.S + 3 * k;
        const double s0 = si[0], s1 = si[1], s2 = si[2];
        uint32_t c[4] = {(uint32_t)i, (uint32_t)sweep, (uint32_t)((uint64_t)i >> 32),
                         0x80000000u | (uint32_t)((uint64_t)sweep >> 32)};
        philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
        const double u0 = ((double)c[0] + 0.5) * (1.0 / 4294967296.0);
        const double u1 = ((double)c[1] + 0.5) * (1.0 / 4294967296.0);
        const double u2 = ((double)c[2] + 0.5) * (1.0 / 4294967296.0);
        const double cosa = 1.0 - u0 * (1.0 - a.cone[1]);
        const double sina = sqrt(fmax(0.0, 1.0 - cosa * cosa));
        double sb, cb;
        sincospi(2.0 * u1, &sb, &cb);
        // frame about S_i: e1 from z (x when S_i is near z), e2 = S_i x e1
        const bool near_z = fabs(s2) >= 0.9;
        const double ax = near_z ? 1.0 : 0.0, az = near_z ? 0.0 : 1.0;
        const double as = ax * s0 + az * s2;
        double e10 = ax - as * s0, e11 = -as * s1, e12 = az - as * s2;
        const double l1 = sqrt(e10 * e10 + e11 * e11 + e12 * e12);
        e10 /= l1;
        e11 /= l1;
        e12 /= l1;
        const double e20 = s1 * e12 - s2 * e11, e21 = s2 * e10 - s0 * e12, e22 = s0 * e11 - s1 * e10;
        double t0 = cosa * s0 + sina * (cb * e10 + sb * e20);
        double t1 = cosa * s1 + sina * (cb * e11 + sb * e21);
        double t2 = cosa * s2 + sina * (cb * e12 + sb * e22);
        const double lt = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
        t0 /= lt;
        t1 /= lt;
        t2 /= lt;
        const double dE = ((t0 - s0) * w0 + (t1 - s1) * w1 + (t2 - s2) * w2) - a.A * (t2 * t2 - s2 * s2) -
                          a.Hz * (t2 - s2);
        if (dE <= 0.0 || u2 < exp(-dE / T)) {
            si[0] = t0;
            si[1] = t1;
            si[2] = t2;
            accepted = true;
        }
    }
    __shared__ unsigned int wave_acc[4];
    const unsigned long long ball = __ballot(accepted);
    if ((threadIdx.x & 63) == 0) wave_acc[threadIdx.x >> 6] = (unsigned int)__popcll(ball);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long sum = (unsigned long long)wave_acc[0] + wave_acc[1] + wave_acc[2] + wave_acc[3];
        if (sum) atomicAdd(a.accepted + (blockIdx.x % kMcCounters) * kMcCounterStride, sum);
    }
}

// After a sweep (one wave): gather the counters, clear them, record the
// accepted moves, adapt the cone.
__global__ __launch_bounds__(64) void mc_cone_kernel(McArgs a, long long* history, int64_t sweep) {
    __shared__ unsigned long long part[kMcCounters];
    const int t = threadIdx.x;
    part[t] = a.accepted[t * kMcCounterStride];
    a.accepted[t * kMcCounterStride] = 0ull;
    __syncthreads();
    if (t != 0) return;
    unsigned long long acc = 0ull;
    for (int c = 0; c < kMcCounters; ++c) acc += part[c];
    if (history) history[sweep] = (long long)acc;
    const double rate = (double)acc / (double)a.n;
    double c = a.cone[0];
    if (rate < a.acc_target)
        c = fmax(1e-3, 0.9 * c);
    else if (rate > 2.0 * a.acc_target)
        c = fmin(kPi, 1.1 * c);
    a.cone[0] = c;
    a.cone[1] = cos(c);
}

__global__ __launch_bounds__(64) void mc_setup_kernel(McArgs a, double cone0) {
    a.accepted[threadIdx.x * kMcCounterStride] = 0ull;
    if (threadIdx.x != 0) return;
    a.cone[0] = cone0;
    a.cone[1] = cos(cone0);
}

__global__ __launch_bounds__(256) void mc_load_kernel(McArgs a, const float* __restrict__ init) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < 3 * a.n; x += (int64_t)gridDim.x * blockDim.x)
        a.S[x] = (double)init[3 * (int64_t)a.site_of[x / 3] + x % 3];
}

// Energy of Eq. (1) per block: half of each site's bond energies (each bond
// is seen from both ends) plus its single-site terms; partial sums per block.
__global__ __launch_bounds__(256) void mc_energy_kernel(McArgs a, double* __restrict__ partial) {
    __shared__ double red[256];
    double e = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n; k += (int64_t)gridDim.x * blockDim.x) {
        const double* si = a.S + 3 * k;
        double eb = 0.0;
        for (int e = 0; e < a.z_max; ++e) {
            const int32_t j = a.nbr[k * a.z_max + e];
            if (j < 0) continue;
            const double* sj = a.S + 3 * (int64_t)j;
            eb += (double)a.jval[k * a.z_max + e] * (si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2]);
            if (a.dvec) {
                const float* d = a.dvec + 3 * (k * a.z_max + e);
                const double cx = si[1] * sj[2] - si[2] * sj[1];
                const double cy = si[2] * sj[0] - si[0] * sj[2];
                const double cz = si[0] * sj[1] - si[1] * sj[0];
                eb -= (double)d[0] * cx + (double)d[1] * cy + (double)d[2] * cz;
            }
        }
        e += 0.5 * eb - a.A * si[2] * si[2] - a.Hz * si[2];
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Final state as fp32 and the info block: energy per site (partials summed
// in block order), cone, last temperature.
__global__ __launch_bounds__(256) void mc_out_kernel(McArgs a, float* __restrict__ out) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < 3 * a.n; x += (int64_t)gridDim.x * blockDim.x)
        out[3 * (int64_t)a.site_of[x / 3] + x % 3] = (float)a.S[x];
}

// One workgroup: thread t sums partials t, t + 256, ... in order, then a
// fixed tree (the same result on every run).
__global__ __launch_bounds__(256) void mc_info_kernel(McArgs a, const double* __restrict__ partial, int n_partial,
                                                      double T_last, double* __restrict__ info) {
    __shared__ double red[256];
    double e = 0.0;
    for (int b = threadIdx.x; b < n_partial; b += 256) e += partial[b];
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    info[0] = red[0] / (double)a.n;
    info[1] = a.cone[0];
    info[2] = T_last;
}

unsigned grid_of(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

}  // namespace

int mc_energy_blocks(int64_t n) { return (int)grid_of(n); }

size_t mc_counter_bytes() { return (size_t)kMcCounters * kMcCounterStride * sizeof(unsigned long long); }

int launch_mc_setup(const McArgs& a, const float* init, double cone0, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (init) hipLaunchKernelGGL(mc_load_kernel, dim3(grid_of(3 * a.n)), dim3(256), 0, s, a, init);
    hipLaunchKernelGGL(mc_setup_kernel, dim3(1), dim3(64), 0, s, a, cone0);
    return (int)hipGetLastError();
}

int launch_mc_sweep(const McArgs& a, const int64_t* class_start, int n_classes, double T, int64_t sweep,
                    long long* history, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    for (int c = 0; c < n_classes; ++c) {
        const int64_t count = class_start[c + 1] - class_start[c];
        if (count == 0) continue;
        const unsigned grid = (unsigned)((count + 255) / 256);
        if (a.stencil)
            hipLaunchKernelGGL(mc_colour_kernel<1>, dim3(grid), dim3(256), 0, s, a, class_start[c], count, T, sweep);
        else
            hipLaunchKernelGGL(mc_colour_kernel<0>, dim3(grid), dim3(256), 0, s, a, class_start[c], count, T, sweep);
    }
    hipLaunchKernelGGL(mc_cone_kernel, dim3(1), dim3(64), 0, s, a, history, sweep);
    return (int)hipGetLastError();
}

int launch_mc_finish(const McArgs& a, double* partial, double T_last, float* out, double* info, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const unsigned g = grid_of(a.n);
    hipLaunchKernelGGL(mc_energy_kernel, dim3(g), dim3(256), 0, s, a, partial);
    hipLaunchKernelGGL(mc_out_kernel, dim3(grid_of(3 * a.n)), dim3(256), 0, s, a, out);
    hipLaunchKernelGGL(mc_info_kernel, dim3(1), dim3(256), 0, s, a, (const double*)partial, (int)g, T_last, info);
    return (int)hipGetLastError();
}

}  // namespace sdc
