// Trajectory generator entry point: bond tables on the host (nearest
// neighbours of sc/bcc lattices, or J(r) pairs within a cutoff for open
// samples, with their DMI vectors), then the RK4 kernels of sdc_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "sdc_internal.h"

namespace {

int64_t pmod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

// Random bond sign from Philox: counter (min(i,j), max(i,j), 1, 0).
float bond_sign(uint64_t seed, int64_t i, int64_t j) {
    const uint32_t a = (uint32_t)std::min(i, j), b = (uint32_t)std::max(i, j);
    uint32_t c[4] = {a, b, 1u, 0u};
    sdc::philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return (c[0] & 1u) ? -1.0f : 1.0f;
}

struct Bonds {
    int z = 0;
    std::vector<int32_t> nbr;
    std::vector<float> jv;
    std::vector<float> dv;  // [n][z][3] D (r_j - r_i)/|r_j - r_i|, filled when D != 0
};

sdc_status lattice_bonds(const float* pos, int64_t n, const sdc_traj_spec* sp, Bonds* b, std::string* err) {
    const bool bcc = sp->kind == SDC_BINS_PERIODIC_BCC;
    int64_t L[3];
    for (int a = 0; a < 3; ++a) {
        if (sp->cells[a] < 1) {
            *err = "cells must be >= 1";
            return SDC_ERR_INVALID_ARG;
        }
        L[a] = sp->cells[a];
    }
    const int64_t expect = (bcc ? 2 : 1) * L[0] * L[1] * L[2];
    if (n != expect) {
        *err = "n_sites must equal the lattice sites of the box";
        return SDC_ERR_INVALID_ARG;
    }
    // doubled integer coordinates D = 2r (sc: even), periodic modulo 2L
    std::vector<int64_t> D(3 * n);
    std::unordered_map<int64_t, int64_t> index;
    index.reserve((size_t)n * 2);
    auto code = [&](const int64_t d[3]) {
        return (pmod(d[0], 2 * L[0]) * (2 * L[1]) + pmod(d[1], 2 * L[1])) * (2 * L[2]) + pmod(d[2], 2 * L[2]);
    };
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            const double p = 2.0 * pos[3 * i + a];
            const double r = std::floor(p + 0.5);
            if (!(std::fabs(p - r) <= 2e-3) || (!bcc && pmod((int64_t)r, 2) != 0)) {
                *err = "position is not a lattice point";
                return SDC_ERR_INVALID_ARG;
            }
            D[3 * i + a] = (int64_t)r;
        }
        if (bcc && (pmod(D[3 * i], 2) != pmod(D[3 * i + 1], 2) || pmod(D[3 * i], 2) != pmod(D[3 * i + 2], 2))) {
            *err = "position is not a bcc lattice point";
            return SDC_ERR_INVALID_ARG;
        }
        if (!index.emplace(code(&D[3 * i]), i).second) {
            *err = "duplicate lattice site";
            return SDC_ERR_INVALID_ARG;
        }
    }
    std::vector<std::array<int, 3>> deltas;
    if (!bcc) {
        deltas = {{2, 0, 0}, {-2, 0, 0}, {0, 2, 0}, {0, -2, 0}, {0, 0, 2}, {0, 0, -2}};
    } else {
        for (int sx = -1; sx <= 1; sx += 2)
            for (int sy = -1; sy <= 1; sy += 2)
                for (int sz = -1; sz <= 1; sz += 2) deltas.push_back({sx, sy, sz});
    }
    b->z = (int)deltas.size();
    b->nbr.resize((size_t)n * b->z);
    b->jv.resize((size_t)n * b->z);
    if (sp->D != 0.0) b->dv.resize((size_t)n * b->z * 3);
    for (int64_t i = 0; i < n; ++i)
        for (int e = 0; e < b->z; ++e) {
            const int64_t d[3] = {D[3 * i] + deltas[e][0], D[3 * i + 1] + deltas[e][1], D[3 * i + 2] + deltas[e][2]};
            auto it = index.find(code(d));
            if (it == index.end()) {
                *err = "lattice neighbour missing";
                return SDC_ERR_INVALID_ARG;
            }
            const int64_t j = it->second;
            if (j == i) {  // a box one cell wide: the bond closes on the site itself and is dropped
                b->nbr[i * b->z + e] = -1;
                b->jv[i * b->z + e] = 0.0f;
                continue;
            }
            b->nbr[i * b->z + e] = (int32_t)j;
            float J = (float)sp->J;
            if (sp->coupling == SDC_COUPLING_NN_RANDOM_SIGN) J = (float)std::fabs(sp->J) * bond_sign(sp->seed, i, j);
            b->jv[i * b->z + e] = J;
            if (!b->dv.empty()) {
                // unit bond vector from the doubled-coordinate step (minimal image)
                const double len = std::sqrt((double)(deltas[e][0] * deltas[e][0] + deltas[e][1] * deltas[e][1] +
                                                      deltas[e][2] * deltas[e][2]));
                for (int c = 0; c < 3; ++c) b->dv[(i * b->z + e) * 3 + c] = (float)(sp->D * deltas[e][c] / len);
            }
        }
    return SDC_OK;
}

sdc_status cutoff_bonds(const float* pos, int64_t n, const sdc_traj_spec* sp, Bonds* b, std::string* err) {
    if (!(sp->r_cut > 0.0f) || !std::isfinite(sp->r_cut)) {
        *err = "r_cut must be finite and > 0";
        return SDC_ERR_INVALID_ARG;
    }
    const float rc = sp->r_cut;
    const float rc2 = rc * rc;
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(pos[3 * i + a])) {
                *err = "non-finite position";
                return SDC_ERR_INVALID_ARG;
            }
            lo[a] = std::min(lo[a], pos[3 * i + a]);
        }
    // cell list with cell edge r_cut
    std::unordered_map<int64_t, std::vector<int64_t>> cells;
    auto cell_of = [&](int64_t i, int64_t c[3]) {
        for (int a = 0; a < 3; ++a) c[a] = (int64_t)std::floor((pos[3 * i + a] - lo[a]) / rc);
    };
    auto key = [](int64_t x, int64_t y, int64_t z) { return (x * 1048573 + y) * 1048573 + z; };
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        cell_of(i, c);
        cells[key(c[0], c[1], c[2])].push_back(i);
    }
    std::vector<std::vector<std::pair<int32_t, float>>> nb(n);
    size_t zmax = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        cell_of(i, c);
        for (int64_t dx = -1; dx <= 1; ++dx)
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dz = -1; dz <= 1; ++dz) {
                    auto it = cells.find(key(c[0] + dx, c[1] + dy, c[2] + dz));
                    if (it == cells.end()) continue;
                    for (int64_t j : it->second) {
                        if (j == i) continue;
                        const float d2 = sdc::dist2_f32(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], pos[3 * j],
                                                        pos[3 * j + 1], pos[3 * j + 2]);
                        if (d2 <= rc2) nb[i].push_back({(int32_t)j, (float)(sp->J * std::exp(-std::sqrt((double)d2)))});
                    }
                }
        zmax = std::max(zmax, nb[i].size());
    }
    if (zmax > 4096) {
        *err = "too many neighbours within r_cut";
        return SDC_ERR_UNSUPPORTED;
    }
    b->z = (int)std::max<size_t>(zmax, 1);
    b->nbr.assign((size_t)n * b->z, -1);
    b->jv.assign((size_t)n * b->z, 0.0f);
    if (sp->D != 0.0) b->dv.assign((size_t)n * b->z * 3, 0.0f);
    for (int64_t i = 0; i < n; ++i) {
        std::sort(nb[i].begin(), nb[i].end());
        for (size_t e = 0; e < nb[i].size(); ++e) {
            const int64_t j = nb[i][e].first;
            b->nbr[i * b->z + e] = (int32_t)j;
            b->jv[i * b->z + e] = nb[i][e].second;
            if (!b->dv.empty()) {
                double d[3], len2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    d[c] = (double)pos[3 * j + c] - (double)pos[3 * i + c];
                    len2 += d[c] * d[c];
                }
                const double len = std::sqrt(len2);
                for (int c = 0; c < 3; ++c)
                    b->dv[(i * b->z + e) * 3 + c] = len > 0.0 ? (float)(sp->D * d[c] / len) : 0.0f;
            }
        }
    }
    return SDC_OK;
}

sdc_status build_bonds(const float* pos, int64_t n, const sdc_traj_spec* sp, Bonds* b, std::string* err) {
    try {
        if ((sp->kind == SDC_BINS_PERIODIC_SC || sp->kind == SDC_BINS_PERIODIC_BCC) &&
            (sp->coupling == SDC_COUPLING_NN_UNIFORM || sp->coupling == SDC_COUPLING_NN_RANDOM_SIGN))
            return lattice_bonds(pos, n, sp, b, err);
        if (sp->kind == SDC_BINS_RADIAL && sp->coupling == SDC_COUPLING_EXP_CUTOFF) return cutoff_bonds(pos, n, sp, b, err);
    } catch (const std::bad_alloc&) {
        *err = "host allocation failed";
        return SDC_ERR_OOM;
    }
    *err = "unsupported kind/coupling combination";
    return SDC_ERR_UNSUPPORTED;
}

// The annealing schedule: T_k = T_start cool^k while T_k > T_end,
// sweeps_per_T sweeps each, then sweeps_final sweeps at T_end.  Calls
// visit(T) once per sweep, in order; returns the number of sweeps.
template <class F>
int64_t mc_schedule(const sdc_mc_spec* m, F visit) {
    int64_t s = 0;
    for (double T = m->T_start; T > m->T_end; T *= m->cool)
        for (int64_t k = 0; k < m->sweeps_per_T; ++k, ++s) visit(T);
    for (int64_t k = 0; k < m->sweeps_final; ++k, ++s) visit(m->T_end);
    return s;
}

sdc_status mc_check(const sdc_mc_spec* m) {
    const double pi = 3.14159265358979323846;
    if (!std::isfinite(m->J) || !std::isfinite(m->D) || !std::isfinite(m->A) || !std::isfinite(m->Hz))
        return sdc::set_error(SDC_ERR_INVALID_ARG, "J, D, A and Hz must be finite");
    if (!(m->T_end > 0.0) || !std::isfinite(m->T_end) || !(m->T_start > 0.0) || !std::isfinite(m->T_start))
        return sdc::set_error(SDC_ERR_INVALID_ARG, "temperatures must be finite and > 0");
    if (!(m->cool > 0.0 && m->cool < 1.0)) return sdc::set_error(SDC_ERR_INVALID_ARG, "cool must be in (0, 1)");
    if (m->sweeps_per_T < 1 || m->sweeps_final < 0)
        return sdc::set_error(SDC_ERR_INVALID_ARG, "sweeps_per_T must be >= 1 and sweeps_final >= 0");
    if (!(m->cone0 > 0.0 && m->cone0 <= pi)) return sdc::set_error(SDC_ERR_INVALID_ARG, "cone0 must be in (0, pi]");
    if (!(m->acc_target > 0.0 && m->acc_target <= 0.5))
        return sdc::set_error(SDC_ERR_INVALID_ARG, "acc_target must be in (0, 0.5]");
    // at most 2^40 sweeps (the ladder has log(T_end / T_start) / log(cool) rungs)
    const double rungs = m->T_start > m->T_end ? std::ceil(std::log(m->T_end / m->T_start) / std::log(m->cool)) + 1 : 0;
    if (rungs * (double)m->sweeps_per_T + (double)m->sweeps_final > 1099511627776.0)
        return sdc::set_error(SDC_ERR_UNSUPPORTED, "schedule longer than 2^40 sweeps");
    return SDC_OK;
}

}  // namespace

extern "C" sdc_status sdc_traj_generate(const float* positions_host, int64_t n_sites, const sdc_traj_spec* spec,
                                        float* frames_dev, int64_t n_frames, int device, void* stream) {
    auto sdc_internal_set_error = [](sdc_status st, const std::string& msg) { return sdc::set_error(st, msg); };
    if (!positions_host || !spec || !frames_dev) return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "null pointer");
    if (n_sites < 1 || n_sites > ((int64_t)1 << 26))
        return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "n_sites out of range");
    if (n_frames < 1) return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "n_frames must be >= 1");
    if (!(spec->dt > 0.0) || !std::isfinite(spec->dt) || !std::isfinite(spec->J))
        return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "dt must be > 0 and J finite");
    if (!std::isfinite(spec->D) || !std::isfinite(spec->A) || !std::isfinite(spec->Hz))
        return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "D, A and Hz must be finite");
    if (spec->init < SDC_INIT_UNIFORM || spec->init > SDC_INIT_GIVEN)
        return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "unknown init");
    if (spec->init == SDC_INIT_GIVEN && !spec->init_dev)
        return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "init_dev is null");
    if (spec->init == SDC_INIT_PERTURBED_Z && !(spec->sigma >= 0.0))
        return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "sigma must be >= 0");
    Bonds b;
    std::string err;
    const sdc_status s = build_bonds(positions_host, n_sites, spec, &b, &err);
    if (s != SDC_OK) return sdc_internal_set_error(s, err.c_str());

    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
        return sdc_internal_set_error(SDC_ERR_NO_DEVICE, "no HIP device");
    if (device < 0 || device >= count) return sdc_internal_set_error(SDC_ERR_INVALID_ARG, "device out of range");
    if (hipSetDevice(device) != hipSuccess) return sdc_internal_set_error(SDC_ERR_HIP, "hipSetDevice");
    int32_t* d_nbr = nullptr;
    float* d_j = nullptr;
    float* d_dv = nullptr;
    float* d_work = nullptr;
    auto cleanup = [&]() {
        if (d_nbr) (void)hipFree(d_nbr);
        if (d_j) (void)hipFree(d_j);
        if (d_dv) (void)hipFree(d_dv);
        if (d_work) (void)hipFree(d_work);
    };
    if (hipMalloc(&d_nbr, b.nbr.size() * 4) != hipSuccess || hipMalloc(&d_j, b.jv.size() * 4) != hipSuccess ||
        (!b.dv.empty() && hipMalloc(&d_dv, b.dv.size() * 4) != hipSuccess) ||
        hipMalloc(&d_work, (size_t)12 * n_sites * 4) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return sdc_internal_set_error(SDC_ERR_OOM, "hipMalloc failed");
    }
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d_nbr, b.nbr.data(), b.nbr.size() * 4, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(d_j, b.jv.data(), b.jv.size() * 4, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && d_dv) e = hipMemcpyAsync(d_dv, b.dv.data(), b.dv.size() * 4, hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) {
        cleanup();
        return sdc_internal_set_error(SDC_ERR_HIP, hipGetErrorString(e));
    }
    sdc::TrajArgs ta{};
    ta.n = n_sites;
    ta.z_max = b.z;
    ta.nbr = d_nbr;
    ta.jval = d_j;
    ta.dvec = d_dv;
    ta.aniso2 = (float)(2.0 * spec->A);
    ta.hz = (float)spec->Hz;
    ta.dt = (float)spec->dt;
    ta.init = spec->init;
    ta.sigma = spec->sigma;
    ta.seed = spec->seed;
    ta.init_dev = spec->init_dev;
    ta.frames = frames_dev;
    ta.n_frames = n_frames;
    ta.work = d_work;
    int le = sdc::launch_traj(ta, stream);
    hipError_t se = hipStreamSynchronize(hs);
    cleanup();
    if (le != 0) return sdc_internal_set_error(SDC_ERR_HIP, hipGetErrorString((hipError_t)le));
    if (se != hipSuccess) return sdc_internal_set_error(SDC_ERR_HIP, hipGetErrorString(se));
    return sdc_internal_set_error(SDC_OK, "");
}

extern "C" sdc_status sdc_mc_n_sweeps(const sdc_mc_spec* spec, int64_t* n_sweeps) {
    if (!spec || !n_sweeps) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    const sdc_status s = mc_check(spec);
    if (s != SDC_OK) return s;
    *n_sweeps = mc_schedule(spec, [](double) {});
    return sdc::set_error(SDC_OK, "");
}

struct sdc_mc {
    int device = 0;
    sdc_mc_spec spec{};
    int64_t n = 0;
    int n_col = 0;
    std::vector<int64_t> start;          // first slot of each colour class, and n
    std::vector<void*> owned;
    sdc::McArgs args{};
    double* d_partial = nullptr;
    double* d_info = nullptr;
    long long* d_hist = nullptr;
    int64_t hist_cap = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool timed = false;
    bool loaded = false;                 // the FP64 state holds a configuration

    ~sdc_mc() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        for (void* p : owned) (void)hipFree(p);
    }
};

namespace {

uint32_t float_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, sizeof u);
    return u;
}

// The colour kernel's lattice stencil (McArgs::stencil) for a periodic sc box
// with even edges and one uniform coupling: turned on only when it gives the
// slot -> site map and every neighbour slot, coupling and DMI vector of the
// slot-ordered tables bit for bit, so both kernels compute the same sweep.
void mc_stencil(const sdc_mc_spec* spec, int64_t n, int n_col, const std::vector<int64_t>& start,
                const std::vector<int32_t>& order, const Bonds& b, sdc::McArgs* ma) {
    ma->stencil = 0;
    if (spec->kind != SDC_BINS_PERIODIC_SC || spec->coupling != SDC_COUPLING_NN_UNIFORM || n_col != 2 || b.z != 6 ||
        n % 2 != 0 || start[1] != n / 2)
        return;
    for (int a = 0; a < 3; ++a)
        if (spec->cells[a] < 2 || spec->cells[a] % 2 != 0) return;
    const int64_t L0 = spec->cells[0], L1 = spec->cells[1], L2 = spec->cells[2], half = n / 2;
    const float jf = (float)spec->J;
    // the DMI table entries D (r_j - r_i) / |r_j - r_i| for steps of +-2 or 0
    // in doubled coordinates, rounded as the table rounds them
    const float dp = (float)(spec->D * 2 / 2.0), dn = (float)(spec->D * -2 / 2.0), dz = (float)(spec->D * 0 / 2.0);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t c = k >= half ? 1 : 0, s0 = 2 * (k - c * half);
        const int64_t row = s0 / L2, z0 = s0 - row * L2, y = row % L1, x = row / L1;
        const int64_t dl = c ^ ((x + y) & 1), z = z0 + dl;
        if (order[(size_t)k] != s0 + dl) return;
        const int64_t other = c ? 0 : half;
        const int64_t sj[6] = {((((x + 1) % L0) * L1 + y) * L2 + z), ((((x + L0 - 1) % L0) * L1 + y) * L2 + z),
                               ((x * L1 + (y + 1) % L1) * L2 + z), ((x * L1 + (y + L1 - 1) % L1) * L2 + z),
                               row * L2 + (z + 1) % L2, row * L2 + (z + L2 - 1) % L2};
        for (int e = 0; e < 6; ++e) {
            const size_t be = (size_t)(k * 6 + e);
            if (b.nbr[be] != other + (sj[e] >> 1) || float_bits(b.jv[be]) != float_bits(jf)) return;
            if (!b.dv.empty())
                for (int a = 0; a < 3; ++a)
                    if (float_bits(b.dv[be * 3 + a]) != float_bits(a == e / 2 ? ((e & 1) ? dn : dp) : dz)) return;
        }
    }
    ma->stencil = 1;
    ma->L0 = (int)L0;
    ma->L1 = (int)L1;
    ma->L2 = (int)L2;
    ma->st_j = jf;
    ma->st_dp = dp;
    ma->st_dn = dn;
    ma->st_dz = dz;
}

bool mc_alloc(sdc_mc* m, void** p, size_t bytes) {
    if (hipMalloc(p, bytes ? bytes : 1) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    m->owned.push_back(*p);
    return true;
}

}  // namespace

extern "C" sdc_status sdc_mc_create(const float* positions_host, int64_t n_sites, const sdc_mc_spec* spec, int device,
                                    sdc_mc** out) {
    if (!out) return sdc::set_error(SDC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (!positions_host || !spec) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    if (n_sites < 1 || n_sites > ((int64_t)1 << 26)) return sdc::set_error(SDC_ERR_INVALID_ARG, "n_sites out of range");
    sdc_status s = mc_check(spec);
    if (s != SDC_OK) return s;
    sdc_traj_spec ts{};
    ts.kind = spec->kind;
    for (int a = 0; a < 3; ++a) ts.cells[a] = spec->cells[a];
    ts.coupling = spec->coupling;
    ts.r_cut = spec->r_cut;
    ts.J = spec->J;
    ts.D = spec->D;
    ts.seed = spec->seed;
    Bonds b;
    std::string err;
    s = build_bonds(positions_host, n_sites, &ts, &b, &err);
    if (s != SDC_OK) return sdc::set_error(s, err);
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count == 0)
        return sdc::set_error(SDC_ERR_NO_DEVICE, "no HIP device");
    if (device < 0 || device >= dev_count) return sdc::set_error(SDC_ERR_INVALID_ARG, "device out of range");
    if (hipSetDevice(device) != hipSuccess) return sdc::set_error(SDC_ERR_HIP, "hipSetDevice");
    sdc_mc* m = nullptr;
    try {
        m = new sdc_mc();
        m->device = device;
        m->spec = *spec;
        m->n = n_sites;
        // greedy colouring in site order, then the sites grouped by colour
        std::vector<int32_t> colour((size_t)n_sites, -1);
        std::vector<char> used;
        for (int64_t i = 0; i < n_sites; ++i) {
            used.assign((size_t)m->n_col + 1, 0);
            for (int e = 0; e < b.z; ++e) {
                const int32_t j = b.nbr[i * b.z + e];
                if (j >= 0 && j < i) used[(size_t)colour[j]] = 1;
            }
            int c = 0;
            while (used[(size_t)c]) ++c;
            colour[i] = c;
            m->n_col = std::max(m->n_col, c + 1);
        }
        // colour-major slots: class c takes slots start[c] .. start[c + 1], sites
        // in index order; bond tables rewritten in slot order with slot
        // neighbours
        std::vector<int64_t>& start = m->start;
        start.assign((size_t)m->n_col + 1, 0);
        for (int64_t i = 0; i < n_sites; ++i) ++start[(size_t)colour[i] + 1];
        for (int c = 0; c < m->n_col; ++c) start[(size_t)c + 1] += start[(size_t)c];
        std::vector<int32_t> order((size_t)n_sites), slot((size_t)n_sites);
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n_sites; ++i) {
            const int64_t k = fill[(size_t)colour[i]]++;
            order[(size_t)k] = (int32_t)i;
            slot[(size_t)i] = (int32_t)k;
        }
        {
            std::vector<int32_t> nbr(b.nbr.size());
            std::vector<float> jv(b.jv.size()), dv(b.dv.size());
            for (int64_t k = 0; k < n_sites; ++k) {
                const int64_t i = order[(size_t)k];
                for (int e = 0; e < b.z; ++e) {
                    const int32_t j = b.nbr[i * b.z + e];
                    nbr[k * b.z + e] = j < 0 ? -1 : slot[(size_t)j];
                    jv[k * b.z + e] = b.jv[i * b.z + e];
                    if (!dv.empty())
                        for (int c = 0; c < 3; ++c) dv[(k * b.z + e) * 3 + c] = b.dv[(i * b.z + e) * 3 + c];
                }
            }
            b.nbr.swap(nbr);
            b.jv.swap(jv);
            b.dv.swap(dv);
        }

        int32_t* d_nbr = nullptr;
        int32_t* d_order = nullptr;
        float* d_j = nullptr;
        float* d_dv = nullptr;
        double* d_S = nullptr;
        double* d_cone = nullptr;
        unsigned long long* d_acc = nullptr;
        const int n_part = sdc::mc_energy_blocks(n_sites);
        const bool ok = mc_alloc(m, (void**)&d_nbr, b.nbr.size() * 4) && mc_alloc(m, (void**)&d_j, b.jv.size() * 4) &&
                        (b.dv.empty() || mc_alloc(m, (void**)&d_dv, b.dv.size() * 4)) &&
                        mc_alloc(m, (void**)&d_order, (size_t)n_sites * 4) &&
                        mc_alloc(m, (void**)&d_S, (size_t)n_sites * 24) && mc_alloc(m, (void**)&d_cone, 16) &&
                        mc_alloc(m, (void**)&d_acc, sdc::mc_counter_bytes()) && mc_alloc(m, (void**)&m->d_partial, (size_t)n_part * 8) &&
                        mc_alloc(m, (void**)&m->d_info, 24);
        if (!ok) {
            delete m;
            return sdc::set_error(SDC_ERR_OOM, "hipMalloc failed");
        }
        hipError_t e = hipMemcpy(d_nbr, b.nbr.data(), b.nbr.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_j, b.jv.data(), b.jv.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && d_dv) e = hipMemcpy(d_dv, b.dv.data(), b.dv.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_order, order.data(), (size_t)n_sites * 4, hipMemcpyHostToDevice);
        for (hipEvent_t& ev : m->ev)
            if (e == hipSuccess) e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            delete m;
            return sdc::set_error(SDC_ERR_HIP, hipGetErrorString(e));
        }
        sdc::McArgs& ma = m->args;
        ma.n = n_sites;
        ma.z_max = b.z;
        ma.site_of = d_order;
        ma.nbr = d_nbr;
        ma.jval = d_j;
        ma.dvec = d_dv;
        ma.A = spec->A;
        ma.Hz = spec->Hz;
        ma.S = d_S;
        ma.cone = d_cone;
        ma.accepted = d_acc;
        mc_stencil(spec, n_sites, m->n_col, m->start, order, b, &ma);
    } catch (const std::bad_alloc&) {
        delete m;
        return sdc::set_error(SDC_ERR_OOM, "host allocation failed");
    }
    *out = m;
    return sdc::set_error(SDC_OK, "");
}

extern "C" sdc_status sdc_mc_run(sdc_mc* m, const sdc_mc_spec* schedule, const float* init_dev, float* state_dev,
                                 int64_t* accepted_host, double* info_host, void* stream) {
    if (!m || !schedule || !state_dev) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    if (!init_dev && !m->loaded) return sdc::set_error(SDC_ERR_STATE, "no configuration yet: pass init_dev");
    sdc_status s = mc_check(schedule);
    if (s != SDC_OK) return s;
    const int64_t n_sweeps = mc_schedule(schedule, [](double) {});
    if (hipSetDevice(m->device) != hipSuccess) return sdc::set_error(SDC_ERR_HIP, "hipSetDevice");
    if (accepted_host && n_sweeps > m->hist_cap) {
        void* p = nullptr;
        if (!mc_alloc(m, &p, (size_t)n_sweeps * 8)) return sdc::set_error(SDC_ERR_OOM, "hipMalloc failed");
        m->d_hist = (long long*)p;
        m->hist_cap = n_sweeps;
    }
    sdc::McArgs ma = m->args;
    ma.seed = schedule->seed;
    ma.acc_target = schedule->acc_target;
    hipStream_t hs = (hipStream_t)stream;
    int le = sdc::launch_mc_setup(ma, init_dev, schedule->cone0, stream);
    if (le == 0) le = (int)hipEventRecord(m->ev[0], hs);
    int64_t sweep = 0;
    double T_last = schedule->T_start;
    long long* hist = accepted_host ? m->d_hist : nullptr;
    mc_schedule(schedule, [&](double T) {
        if (le == 0)
            le = sdc::launch_mc_sweep(ma, m->start.data(), m->n_col, T, sweep, hist, stream);
        ++sweep;
        T_last = T;
    });
    if (le == 0) le = (int)hipEventRecord(m->ev[1], hs);
    if (le == 0) le = sdc::launch_mc_finish(ma, m->d_partial, T_last, state_dev, m->d_info, stream);
    if (le != 0) return sdc::set_error(SDC_ERR_HIP, hipGetErrorString((hipError_t)le));
    m->loaded = true;
    m->timed = true;
    if (!accepted_host && !info_host) return sdc::set_error(SDC_OK, "");
    double info[3] = {0.0, 0.0, 0.0};
    le = (int)hipMemcpyAsync(info, m->d_info, 24, hipMemcpyDeviceToHost, hs);
    if (le == 0 && accepted_host && n_sweeps > 0)
        le = (int)hipMemcpyAsync(accepted_host, m->d_hist, (size_t)n_sweeps * 8, hipMemcpyDeviceToHost, hs);
    const hipError_t se = hipStreamSynchronize(hs);
    if (le != 0) return sdc::set_error(SDC_ERR_HIP, hipGetErrorString((hipError_t)le));
    if (se != hipSuccess) return sdc::set_error(SDC_ERR_HIP, hipGetErrorString(se));
    if (info_host) {
        info_host[0] = info[0];
        info_host[1] = info[1];
        info_host[2] = info[2];
        info_host[3] = (double)m->n_col;
    }
    return sdc::set_error(SDC_OK, "");
}

extern "C" sdc_status sdc_mc_timings(sdc_mc* m, double* ms) {
    if (!m || !ms) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    if (!m->timed) return sdc::set_error(SDC_ERR_STATE, "no run yet");
    if (hipEventSynchronize(m->ev[1]) != hipSuccess) return sdc::set_error(SDC_ERR_HIP, "hipEventSynchronize");
    float t = 0.0f;
    if (hipEventElapsedTime(&t, m->ev[0], m->ev[1]) != hipSuccess)
        return sdc::set_error(SDC_ERR_HIP, "hipEventElapsedTime");
    *ms = t;
    return sdc::set_error(SDC_OK, "");
}

extern "C" sdc_status sdc_mc_uses_stencil(const sdc_mc* m, int32_t* stencil) {
    if (!m || !stencil) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    *stencil = m->args.stencil;
    return sdc::set_error(SDC_OK, "");
}

extern "C" sdc_status sdc_mc_destroy(sdc_mc* m) {
    if (!m) return SDC_OK;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    delete m;
    return sdc::set_error(SDC_OK, "");
}

extern "C" sdc_status sdc_mc_anneal(const float* positions_host, int64_t n_sites, const sdc_mc_spec* spec,
                                    const float* init_dev, float* state_dev, int64_t* accepted_host,
                                    double* info_host, int device, void* stream) {
    if (!init_dev || !state_dev) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    sdc_mc* m = nullptr;
    sdc_status s = sdc_mc_create(positions_host, n_sites, spec, device, &m);
    if (s != SDC_OK) return s;
    s = sdc_mc_run(m, spec, init_dev, state_dev, accepted_host, info_host, stream);
    if (s == SDC_OK && !accepted_host && !info_host && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        s = sdc::set_error(SDC_ERR_HIP, "hipStreamSynchronize");
    const std::string keep = sdc_last_error();
    (void)sdc_mc_destroy(m);
    return s == SDC_OK ? s : sdc::set_error(s, keep);
}
