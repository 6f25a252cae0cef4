// C ABI of the sdc library: argument validation, plan state, device memory,
// and the sequence of kernels behind each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "sdc_internal.h"

using sdc::KGroup;
using sdc::KPair;
using sdc::KStream;
using sdc::Layout;

namespace {

thread_local std::string g_err;

sdc_status set_err(sdc_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

sdc_status hip_err(int e, const char* what) {
    return set_err(SDC_ERR_HIP, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
}

#define SDC_HIP(call, what)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_err((int)e_, what); \
    } while (0)

// Checks that a usable gfx950 device exists and makes it current.
sdc_status use_device(int device) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
        return set_err(SDC_ERR_NO_DEVICE, "no HIP device");
    if (device < 0 || device >= count) return set_err(SDC_ERR_INVALID_ARG, "device ordinal out of range");
    hipDeviceProp_t prop;
    SDC_HIP(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_err(SDC_ERR_NO_DEVICE, std::string("device is not gfx950: ") + prop.gcnArchName);
    SDC_HIP(hipSetDevice(device), "hipSetDevice");
    return SDC_OK;
}

// Makes `device` current only if it is not already (a no-op call sequence
// inside a stream capture).
hipError_t select_device(int device) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    return cur == device ? hipSuccess : hipSetDevice(device);
}

template <class T>
sdc_status dalloc(T** p, size_t count, std::vector<void*>* owned) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(SDC_ERR_OOM, "hipMalloc failed");
    }
    owned->push_back(*p);
    return SDC_OK;
}

// Groups of lags for one lag selection: lag t = s*u + phase, grouped by
// (phase, 16-aligned block of u), with a mask of the selected members.
std::vector<KGroup> make_groups(const std::vector<int>& lags, int s, int lg) {
    std::map<std::pair<int, int>, int> mask;
    for (int t : lags) {
        const int ph = t % s, u = t / s, u0 = (u / lg) * lg;
        mask[{ph, u0}] |= 1 << (u - u0);
    }
    std::vector<KGroup> g;
    for (auto& kv : mask) g.push_back(KGroup{kv.first.first, kv.first.second, kv.second, 0});
    return g;
}

}  // namespace

sdc_status sdc::set_error(sdc_status s, const std::string& msg) { return set_err(s, msg); }

// Largest radial key table kept per plan (2 bytes per ordered tile-pair slot).
constexpr size_t kMaxKeyTableBytes = (size_t)32 << 30;

struct LagSel {
    KGroup* d_groups = nullptr;
    int n_groups = 0;
    int32_t* d_lags = nullptr;
    int n_sel = 0;
    int max_lag = 0;
    std::vector<int> lags;
};

struct sdc_plan {
    int device = 0;
    sdc_bin_spec bins{};
    sdc_corr_spec corr{};
    Layout lay;
    int nk = 0, O8 = 0, F8 = 0;
    int64_t t_req = 0;
    std::vector<void*> owned;
    int32_t* d_perm = nullptr;
    int32_t* d_gtab = nullptr;
    float* d_pos4 = nullptr;
    float* d_e2 = nullptr;
    KPair* d_pairs = nullptr;
    KStream* d_streams = nullptr;
    unsigned long long* d_counts = nullptr;
    double* d_H = nullptr;
    double* d_self = nullptr;
    double* d_norg = nullptr;
    double* d_msum = nullptr;    // [n_lags] sum_o M . M (site-summed raw correlation)
    double* d_mframe = nullptr;  // [t_req][3] per-frame site sums (scratch)
    float* d_mean = nullptr;     // [n][4] origin averages (connected form, scratch)
    uint16_t* d_keys = nullptr;  // radial: per-pair shell tiles, 8 KiB per tile pair
    unsigned long long* d_Hq = nullptr;     // deterministic mode: fixed-point H
    unsigned long long* d_selfq = nullptr;  // deterministic mode: fixed-point self sums
    double* d_C = nullptr;
    double* d_fin = nullptr;  // csum, cself, ssum[2], sself[2]
    void* d_A = nullptr;
    void* d_B = nullptr;
    size_t bytes_A = 0, bytes_B = 0;
    std::map<std::vector<int>, LagSel> sels;
    sdc_tuning tuning{};  // resolved: schedule (never SDC_SCHED_DEFAULT) and segment length
    bool failed = false;
    int batch_refs = 0;  // batches that hold this plan
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool timed = false;

    ~sdc_plan() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        for (void* p : owned) (void)hipFree(p);
    }
};

namespace {

sdc_status get_sel(sdc_plan* p, const int32_t* lags_host, int32_t n_sel, const LagSel** out) {
    std::vector<int> lags;
    if (!lags_host) {
        lags.resize(p->corr.n_lags);
        for (int t = 0; t < p->corr.n_lags; ++t) lags[t] = t;
    } else {
        if (n_sel < 1 || n_sel > p->corr.n_lags)
            return set_err(SDC_ERR_INVALID_ARG, "n_lags_sel must be in [1, n_lags]");
        lags.assign(lags_host, lags_host + n_sel);
        std::vector<int> sorted = lags;
        std::sort(sorted.begin(), sorted.end());
        for (size_t k = 0; k < sorted.size(); ++k) {
            if (sorted[k] < 0 || sorted[k] >= p->corr.n_lags)
                return set_err(SDC_ERR_INVALID_ARG, "lag out of [0, n_lags)");
            if (k > 0 && sorted[k] == sorted[k - 1]) return set_err(SDC_ERR_INVALID_ARG, "duplicate lag");
        }
        lags = sorted;
    }
    auto it = p->sels.find(lags);
    if (it != p->sels.end()) {
        *out = &it->second;
        return SDC_OK;
    }
    LagSel sel;
    sel.lags = lags;
    sel.n_sel = (int)lags.size();
    sel.max_lag = lags.back();
    std::vector<KGroup> g = make_groups(lags, p->corr.origin_stride, sdc::lag_group(p->corr.precision));
    sel.n_groups = (int)g.size();
    sdc_status s = dalloc(&sel.d_groups, g.size(), &p->owned);
    if (s != SDC_OK) return s;
    s = dalloc(&sel.d_lags, lags.size(), &p->owned);
    if (s != SDC_OK) return s;
    // one-time upload per distinct selection; later calls reuse it and stay
    // asynchronous (and capturable)
    SDC_HIP(hipMemcpy(sel.d_groups, g.data(), g.size() * sizeof(KGroup), hipMemcpyHostToDevice), "upload groups");
    SDC_HIP(hipMemcpy(sel.d_lags, lags.data(), lags.size() * sizeof(int32_t), hipMemcpyHostToDevice), "upload lags");
    auto res = p->sels.emplace(lags, sel);
    *out = &res.first->second;
    return SDC_OK;
}

sdc_status check_specs(const sdc_bin_spec* bins, const sdc_corr_spec* corr) {
    if (!bins || !corr) return set_err(SDC_ERR_INVALID_ARG, "null spec");
    if (corr->n_origins < 1 || corr->n_origins > 4096)
        return set_err(SDC_ERR_INVALID_ARG, "n_origins must be in [1, 4096]");
    if (corr->n_lags < 1 || corr->n_lags > 1024) return set_err(SDC_ERR_INVALID_ARG, "n_lags must be in [1, 1024]");
    if (corr->origin_stride < 1 || corr->origin_stride > 64)
        return set_err(SDC_ERR_INVALID_ARG, "origin_stride must be in [1, 64]");
    if (corr->precision < SDC_PREC_FP32 || corr->precision > SDC_PREC_BF16X3)
        return set_err(SDC_ERR_INVALID_ARG, "unknown precision");
    if ((corr->flags & ~(SDC_FLAG_TIMING | SDC_FLAG_CONNECTED | SDC_FLAG_NO_KEY_TABLE | SDC_FLAG_DETERMINISTIC)) != 0)
        return set_err(SDC_ERR_INVALID_ARG, "unknown flags");
    if (bins->kind < SDC_BINS_PERIODIC_SC || bins->kind > SDC_BINS_RADIAL)
        return set_err(SDC_ERR_INVALID_ARG, "unknown bin kind");
    return SDC_OK;
}

sdc_status plan_usable(const sdc_plan* p) {
    if (!p) return set_err(SDC_ERR_INVALID_ARG, "null plan");
    if (p->failed) return set_err(SDC_ERR_STATE, "plan is unusable after an earlier device failure");
    return SDC_OK;
}

sdc_status fused_args(const sdc_plan* p, const LagSel& sel, sdc::FusedArgs* a) {
    const Layout& L = p->lay;
    std::memset(a, 0, sizeof(*a));
    a->A = p->d_A;
    a->B = p->d_B;
    a->n_pad = L.n_pad;
    a->O8 = p->O8;
    a->F8 = p->F8;
    a->nk = p->nk;
    a->phase_stride = (int64_t)3 * p->F8 * L.n_pad;
    a->pairs = p->d_pairs;
    a->streams = p->d_streams;
    a->n_streams = (int)L.streams.size();
    a->groups = sel.d_groups;
    a->n_groups = sel.n_groups;
    a->gtab = p->d_gtab;
    a->pos4 = p->d_pos4;
    a->keys = p->d_keys;
    a->e2 = p->d_e2;
    a->n_shells = L.n_shells;
    a->inv_w = L.n_shells ? (float)((double)L.n_shells / (double)p->bins.r_max) : 0.0f;
    a->kind = L.kind;
    a->L0 = L.L[0];
    a->L1 = L.L[1];
    a->L2 = L.L[2];
    a->W1 = L.W[1];
    a->W2 = L.W[2];
    a->win = L.win;
    a->H = p->d_H;
    a->det = p->d_Hq != nullptr;
    a->Hq = p->d_Hq;
    a->n_bins = L.n_bins;
    a->stride = p->corr.origin_stride;
    a->precision = p->corr.precision;
    a->sched = sdc::sched_index(p->tuning.schedule);
    if ((int64_t)a->n_groups * a->n_streams > (int64_t)INT32_MAX / 2)
        return set_err(SDC_ERR_UNSUPPORTED, "too many fused tasks");
    return SDC_OK;
}

sdc_status check_frames(const sdc_plan* p, const LagSel& sel, int64_t n_frames) {
    const int64_t need = (int64_t)(p->corr.n_origins - 1) * p->corr.origin_stride + sel.max_lag + 1;
    if (n_frames < need) return set_err(SDC_ERR_INVALID_ARG, "n_frames too small for the origins and lags");
    return SDC_OK;
}

// Queue the pack and self kernels of one accumulate (the current device is
// the plan's); with `timing`, events 0 and 1 bracket them.
sdc_status queue_pack_self(sdc_plan* p, const LagSel& sel, const float* spins_dev, int64_t n_frames, void* stream,
                           bool timing) {
    const Layout& L = p->lay;
    hipStream_t hs = (hipStream_t)stream;
    sdc::PackArgs pa{};
    pa.frames = spins_dev;
    pa.n = L.n;
    pa.n_frames = n_frames;
    pa.n_pad = L.n_pad;
    pa.perm = p->d_perm;
    pa.n_origins = p->corr.n_origins;
    pa.stride = p->corr.origin_stride;
    pa.precision = p->corr.precision;
    pa.O8 = p->O8;
    pa.F8 = p->F8;
    pa.n_phase = p->corr.origin_stride;
    pa.frames_valid = std::min<int64_t>(n_frames, p->t_req);
    pa.A = p->d_A;
    pa.B = p->d_B;
    pa.mean = p->d_mean;
    if (timing) SDC_HIP(hipEventRecord(p->ev[0], hs), "hipEventRecord");
    int e = 0;
    if (p->d_mean)
        e = sdc::launch_mean(spins_dev, L.n, p->corr.n_origins, p->corr.origin_stride, p->d_mean, stream);
    if (e == 0) e = sdc::launch_pack(pa, stream);
    if (e != 0) {
        p->failed = true;
        return hip_err(e, "pack kernel");
    }
    sdc::SelfArgs sa{};
    sa.frames = spins_dev;
    sa.n = L.n;
    sa.n_frames = n_frames;
    sa.n_origins = p->corr.n_origins;
    sa.stride = p->corr.origin_stride;
    sa.lags = sel.d_lags;
    sa.n_sel = sel.n_sel;
    sa.t_need = (int64_t)(p->corr.n_origins - 1) * p->corr.origin_stride + sel.max_lag + 1;
    sa.self = p->d_self;
    sa.precision = p->corr.precision;
    sa.H = p->d_H;
    sa.n_bins = L.n_bins;
    sa.norg = p->d_norg;
    sa.mframe = p->d_mframe;
    sa.msum = p->d_msum;
    sa.mean = p->d_mean;
    sa.det = p->d_Hq != nullptr;
    sa.selfq = p->d_selfq;
    sa.Hq = p->d_Hq;
    if (timing) SDC_HIP(hipEventRecord(p->ev[1], hs), "hipEventRecord");
    e = sdc::launch_self(sa, stream);
    if (e != 0) {
        p->failed = true;
        return hip_err(e, "self kernel");
    }
    return SDC_OK;
}

// Deterministic mode: refresh the FP64 views (H, self sums) from the
// fixed-point accumulators, queued on the stream.
int refresh_fixed(sdc_plan* p, void* stream) {
    if (!p->d_Hq) return 0;
    int e = sdc::launch_fixed_to_double(p->d_Hq, p->d_H, (int64_t)p->corr.n_lags * p->lay.n_bins, stream);
    if (e == 0) e = sdc::launch_fixed_to_double(p->d_selfq, p->d_self, p->corr.n_lags, stream);
    return e;
}

}  // namespace

struct sdc_batch {
    int device = 0;
    std::vector<sdc_plan*> plans;
    std::vector<const LagSel*> sels;
    std::vector<void*> owned;
    sdc::BatchLaunch bl{};
    int flags = 0;
    int schedule = SDC_SCHED_ONE_PASS;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool timed = false;
    ~sdc_batch() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        for (sdc_plan* p : plans) --p->batch_refs;
        for (void* q : owned) (void)hipFree(q);
    }
};

extern "C" {

const char* sdc_status_string(sdc_status s) {
    switch (s) {
        case SDC_OK: return "ok";
        case SDC_ERR_INVALID_ARG: return "invalid argument";
        case SDC_ERR_STATE: return "invalid state";
        case SDC_ERR_OOM: return "out of memory";
        case SDC_ERR_HIP: return "HIP error";
        case SDC_ERR_UNSUPPORTED: return "unsupported";
        case SDC_ERR_NO_DEVICE: return "no usable device";
    }
    return "unknown status";
}

const char* sdc_last_error(void) { return g_err.c_str(); }

sdc_status sdc_layout_keys(const float* positions_host, int64_t n_sites, const sdc_bin_spec* bins,
                           int64_t* keys_out) {
    g_err.clear();
    if (!positions_host || !bins || !keys_out) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    if (n_sites < 1 || n_sites > 4096) return set_err(SDC_ERR_INVALID_ARG, "n_sites must be in [1, 4096]");
    Layout lay;
    std::string err;
    sdc_status s;
    try {
        s = sdc::build_layout(positions_host, n_sites, bins, sdc::default_segment_pairs(bins->kind), &lay, &err);
    } catch (const std::bad_alloc&) {
        return set_err(SDC_ERR_OOM, "host allocation failed");
    }
    if (s != SDC_OK) return set_err(s, err);
    const int64_t n = n_sites;
    std::vector<uint8_t> seen((size_t)(n * n), 0);
    const float inv_w = lay.n_shells ? (float)((double)lay.n_shells / (double)bins->r_max) : 0.0f;
    for (const KStream& st : lay.streams) {
        for (int p = st.p0; p < st.p1; ++p) {
            const KPair& pr = lay.pairs[p];
            for (int a = 0; a < sdc::kTile; ++a)
                for (int b = 0; b < sdc::kTile; ++b) {
                    const int64_t pi = (int64_t)pr.ti * sdc::kTile + a;
                    const int64_t pj = (int64_t)pr.tj * sdc::kTile + b;
                    const int32_t i = lay.perm[pi], j = lay.perm[pj];
                    if (lay.kind != SDC_BINS_RADIAL) {
                        // every slot, padding included, must land inside the window:
                        // the kernels bin padded slots too (with zero spins)
                        const int w = lay.gtab[pj] - lay.gtab[pi] + pr.shift;
                        if (w < 0 || w >= lay.win)
                            return set_err(SDC_ERR_INVALID_ARG, "window coordinate out of range");
                    }
                    if (i < 0 || j < 0) continue;
                    int64_t key;
                    if (lay.kind == SDC_BINS_RADIAL) {
                        const float* ri = &lay.pos4[4 * pi];
                        const float* rj = &lay.pos4[4 * pj];
                        key = sdc::shell_of(sdc::dist2_f32(ri[0], ri[1], ri[2], rj[0], rj[1], rj[2]),
                                            lay.e2.data(), lay.n_shells, inv_w);
                    } else {
                        const int w = lay.gtab[pj] - lay.gtab[pi] + pr.shift;
                        if (w < 0 || w >= lay.win) return set_err(SDC_ERR_INVALID_ARG, "window coordinate out of range");
                        key = sdc::window_bin(lay, st, w);
                    }
                    const int64_t x = (int64_t)i * n + j;
                    if (seen[x]) return set_err(SDC_ERR_INVALID_ARG, "pair visited twice");
                    seen[x] = 1;
                    keys_out[x] = key;
                }
        }
    }
    for (uint8_t v : seen)
        if (!v) return set_err(SDC_ERR_INVALID_ARG, "pair not visited");
    return SDC_OK;
}

sdc_status sdc_plan_create(const float* positions_host, int64_t n_sites, const sdc_bin_spec* bins,
                           const sdc_corr_spec* corr, int device, sdc_plan** out) {
    return sdc_plan_create_tuned(positions_host, n_sites, bins, corr, nullptr, device, out);
}

sdc_status sdc_plan_create_tuned(const float* positions_host, int64_t n_sites, const sdc_bin_spec* bins,
                                 const sdc_corr_spec* corr, const sdc_tuning* tuning, int device, sdc_plan** out) {
    g_err.clear();
    if (!out) return set_err(SDC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (!positions_host) return set_err(SDC_ERR_INVALID_ARG, "null positions");
    sdc_status s = check_specs(bins, corr);
    if (s != SDC_OK) return s;
    sdc_tuning tu{};
    s = sdc::resolve_tuning(tuning, n_sites, bins, corr, device, &tu);
    if (s != SDC_OK) return s;
    sdc_plan* p = nullptr;
    try {
        p = new sdc_plan();
        p->bins = *bins;
        p->corr = *corr;
        p->tuning = tu;
        std::string err;
        s = sdc::build_layout(positions_host, n_sites, bins, tu.segment_pairs, &p->lay, &err);
        if (s != SDC_OK) {
            delete p;
            return set_err(s, err);
        }
    } catch (const std::bad_alloc&) {
        delete p;
        return set_err(SDC_ERR_OOM, "host allocation failed");
    }
    s = use_device(device);
    if (s != SDC_OK) {
        delete p;
        return s;
    }
    p->device = device;
    const Layout& L = p->lay;
    const int sstr = corr->origin_stride;
    p->O8 = (corr->n_origins + sdc::kOriginBlock - 1) / sdc::kOriginBlock;
    p->nk = (3 * p->O8 + 1) / 2;
    const int u_max = (corr->n_lags - 1) / sstr;
    const int lg = sdc::lag_group(corr->precision);
    const int u0_max = (u_max / lg) * lg;
    // largest block read: (O8 - 1) + u0_max / 8 + win_blocks - 1
    p->F8 = p->O8 + u0_max / 8 + sdc::win_blocks(lg) - 1;
    p->t_req = (int64_t)(corr->n_origins - 1) * sstr + corr->n_lags;
    const size_t elem = corr->precision == SDC_PREC_BF16X3 ? 48 : 32;  // bytes per pack element
    // A: [3][O8] blocks plus one zero block, read by the lane half past the
    // last block when 3 O8 is odd
    p->bytes_A = ((size_t)3 * p->O8 + 1) * L.n_pad * elem;
    p->bytes_B = (size_t)sstr * 3 * p->F8 * L.n_pad * elem;
    if (sdc::fused_lds_bytes(L.win, corr->precision) > sdc::kMaxFusedLds) {
        delete p;
        return set_err(SDC_ERR_UNSUPPORTED, "histogram window does not fit in LDS");
    }
    if ((uint64_t)2 * L.n_pad * elem > (uint64_t)UINT32_MAX) {
        // the fused kernel addresses two pack blocks with a 32-bit lane offset
        delete p;
        return set_err(SDC_ERR_UNSUPPORTED, "too many sites for the pack layout (two blocks must fit in 4 GiB)");
    }

#define TRY(x)                  \
    do {                        \
        sdc_status s_ = (x);    \
        if (s_ != SDC_OK) {     \
            delete p;           \
            return s_;          \
        }                       \
    } while (0)
#define TRYHIP(call, what)                              \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) {                         \
            delete p;                                   \
            return hip_err((int)e_, what);              \
        }                                               \
    } while (0)

    {
        const int e = sdc::prepare_kernels();
        if (e != 0) {
            delete p;
            return hip_err(e, "kernel attributes");
        }
    }
    TRY(dalloc(&p->d_perm, L.n_pad, &p->owned));
    TRY(dalloc(&p->d_gtab, L.n_pad, &p->owned));
    TRY(dalloc(&p->d_pos4, L.pos4.size(), &p->owned));
    TRY(dalloc(&p->d_e2, L.e2.size(), &p->owned));
    TRY(dalloc(&p->d_pairs, L.pairs.size(), &p->owned));
    TRY(dalloc(&p->d_streams, L.streams.size(), &p->owned));
    TRY(dalloc(&p->d_counts, (size_t)L.n_bins, &p->owned));
    TRY(dalloc(&p->d_H, (size_t)corr->n_lags * L.n_bins, &p->owned));
    TRY(dalloc(&p->d_self, (size_t)corr->n_lags, &p->owned));
    TRY(dalloc(&p->d_norg, (size_t)corr->n_lags, &p->owned));
    TRY(dalloc(&p->d_msum, (size_t)corr->n_lags, &p->owned));
    TRY(dalloc(&p->d_mframe, (size_t)p->t_req * 3, &p->owned));
    if (corr->flags & SDC_FLAG_CONNECTED) TRY(dalloc(&p->d_mean, (size_t)L.n * 4, &p->owned));
    if (corr->flags & SDC_FLAG_DETERMINISTIC) {
        TRY(dalloc(&p->d_Hq, (size_t)corr->n_lags * L.n_bins, &p->owned));
        TRY(dalloc(&p->d_selfq, (size_t)corr->n_lags, &p->owned));
        TRYHIP(hipMemset(p->d_Hq, 0, (size_t)corr->n_lags * L.n_bins * 8), "zero fixed-point H");
        TRYHIP(hipMemset(p->d_selfq, 0, (size_t)corr->n_lags * 8), "zero fixed-point self sums");
    }
    TRY(dalloc(&p->d_fin, (size_t)6 * corr->n_lags, &p->owned));
    TRY(dalloc((char**)&p->d_A, p->bytes_A, &p->owned));
    TRY(dalloc((char**)&p->d_B, p->bytes_B, &p->owned));

    TRYHIP(hipMemcpy(p->d_perm, L.perm.data(), L.n_pad * sizeof(int32_t), hipMemcpyHostToDevice), "upload perm");
    TRYHIP(hipMemcpy(p->d_gtab, L.gtab.data(), L.n_pad * sizeof(int32_t), hipMemcpyHostToDevice), "upload gtab");
    if (!L.pos4.empty())
        TRYHIP(hipMemcpy(p->d_pos4, L.pos4.data(), L.pos4.size() * sizeof(float), hipMemcpyHostToDevice), "upload pos");
    if (!L.e2.empty())
        TRYHIP(hipMemcpy(p->d_e2, L.e2.data(), L.e2.size() * sizeof(float), hipMemcpyHostToDevice), "upload edges");
    TRYHIP(hipMemcpy(p->d_pairs, L.pairs.data(), L.pairs.size() * sizeof(KPair), hipMemcpyHostToDevice), "upload pairs");
    TRYHIP(hipMemcpy(p->d_streams, L.streams.data(), L.streams.size() * sizeof(KStream), hipMemcpyHostToDevice),
           "upload streams");
    if (corr->flags & SDC_FLAG_TIMING)
        for (int k = 0; k < 4; ++k) TRYHIP(hipEventCreate(&p->ev[k]), "hipEventCreate");
    TRYHIP(hipMemset(p->d_A, 0, p->bytes_A), "zero A pack");
    TRYHIP(hipMemset(p->d_counts, 0, (size_t)L.n_bins * 8), "zero counts");
    TRYHIP(hipMemset(p->d_H, 0, (size_t)corr->n_lags * L.n_bins * 8), "zero H");
    TRYHIP(hipMemset(p->d_self, 0, (size_t)corr->n_lags * 8), "zero self");
    TRYHIP(hipMemset(p->d_norg, 0, (size_t)corr->n_lags * 8), "zero origin totals");
    TRYHIP(hipMemset(p->d_msum, 0, (size_t)corr->n_lags * 8), "zero site sums");

    sdc::CountArgs ca{};
    ca.pairs = p->d_pairs;
    ca.streams = p->d_streams;
    ca.n_streams = (int)L.streams.size();
    ca.perm = p->d_perm;
    ca.gtab = p->d_gtab;
    ca.pos4 = p->d_pos4;
    ca.e2 = p->d_e2;
    ca.n_shells = L.n_shells;
    ca.inv_w = L.n_shells ? (float)((double)L.n_shells / (double)bins->r_max) : 0.0f;
    ca.kind = L.kind;
    ca.L0 = L.L[0];
    ca.L1 = L.L[1];
    ca.L2 = L.L[2];
    ca.W1 = L.W[1];
    ca.W2 = L.W[2];
    ca.win = L.win;
    ca.counts = p->d_counts;
    int e = sdc::launch_count(ca, nullptr);
    if (e != 0) {
        delete p;
        return hip_err(e, "count kernel");
    }
    // Radial: the shells of every tile pair, once, for all lag groups of all
    // accumulates (2 bytes per ordered pair), when the table fits the budget.
    if (L.kind == SDC_BINS_RADIAL && !(corr->flags & SDC_FLAG_NO_KEY_TABLE)) {
        const size_t bytes = L.pairs.size() * (size_t)sdc::kTile * sdc::kTile * sizeof(uint16_t);
        size_t free_b = 0, total_b = 0;
        TRYHIP(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        if (bytes <= kMaxKeyTableBytes && bytes <= free_b / 4) {
            TRY(dalloc((char**)&p->d_keys, bytes, &p->owned));
            e = sdc::launch_radial_keys(ca, (int64_t)L.pairs.size(), p->d_keys, nullptr);
            if (e != 0) {
                delete p;
                return hip_err(e, "radial key kernel");
            }
        }
    }
    TRYHIP(hipDeviceSynchronize(), "count kernel");
#undef TRY
#undef TRYHIP
    *out = p;
    return SDC_OK;
}

sdc_status sdc_plan_get_tuning(const sdc_plan* plan, sdc_tuning* tuning) {
    g_err.clear();
    if (!plan || !tuning) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    *tuning = plan->tuning;
    return SDC_OK;
}

sdc_status sdc_plan_n_bins(const sdc_plan* plan, int64_t* n_bins) {
    g_err.clear();
    if (!plan || !n_bins) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    *n_bins = plan->lay.n_bins;
    return SDC_OK;
}

sdc_status sdc_accumulate(sdc_plan* p, const float* spins_dev, int64_t n_frames, const int32_t* lags_host,
                          int32_t n_lags_sel, void* stream) {
    g_err.clear();
    sdc_status s = plan_usable(p);
    if (s != SDC_OK) return s;
    if (!spins_dev) return set_err(SDC_ERR_INVALID_ARG, "null spins");
    const LagSel* sel = nullptr;
    s = get_sel(p, lags_host, n_lags_sel, &sel);
    if (s != SDC_OK) return s;
    s = check_frames(p, *sel, n_frames);
    if (s != SDC_OK) return s;
    sdc::FusedArgs fa;
    s = fused_args(p, *sel, &fa);
    if (s != SDC_OK) return s;
    SDC_HIP(select_device(p->device), "hipSetDevice");
    const bool timing = (p->corr.flags & SDC_FLAG_TIMING) != 0;
    hipStream_t hs = (hipStream_t)stream;
    s = queue_pack_self(p, *sel, spins_dev, n_frames, stream, timing);
    if (s != SDC_OK) return s;
    if (timing) SDC_HIP(hipEventRecord(p->ev[2], hs), "hipEventRecord");
    const int e = sdc::launch_fused(fa, stream);
    if (e != 0) {
        p->failed = true;
        return hip_err(e, "fused kernel");
    }
    if (timing) {
        SDC_HIP(hipEventRecord(p->ev[3], hs), "hipEventRecord");
        p->timed = true;
    }
    return SDC_OK;
}

sdc_status sdc_finalize(sdc_plan* p, double* C_host, uint64_t* counts_host, double* Csum_host,
                        double* Cself_host, double* Ssum_host, double* Sself_host, void* stream) {
    g_err.clear();
    sdc_status s = plan_usable(p);
    if (s != SDC_OK) return s;
    SDC_HIP(select_device(p->device), "hipSetDevice");
    const Layout& L = p->lay;
    const int nl = p->corr.n_lags;
    hipStream_t hs = (hipStream_t)stream;
    if (C_host && !p->d_C) {
        s = dalloc(&p->d_C, (size_t)nl * L.n_bins, &p->owned);
        if (s != SDC_OK) return s;
    }
    {
        const int e = refresh_fixed(p, stream);
        if (e != 0) {
            p->failed = true;
            return hip_err(e, "fixed-point conversion");
        }
    }
    sdc::FinalArgs fa{};
    fa.H = p->d_H;
    fa.counts = p->d_counts;
    fa.n_org = p->d_norg;
    fa.self = p->d_self;
    fa.msum = p->d_msum;
    fa.n_bins = L.n_bins;
    fa.n_sites = L.n;
    fa.n_lags = nl;
    fa.C = C_host ? p->d_C : nullptr;
    fa.csum = p->d_fin;
    fa.cself = p->d_fin + nl;
    fa.ssum = p->d_fin + 2 * nl;
    fa.sself = p->d_fin + 4 * nl;
    int e = sdc::launch_finalize(fa, stream);
    if (e != 0) {
        p->failed = true;
        return hip_err(e, "finalize kernels");
    }
    std::vector<double> fin(6 * (size_t)nl);
    SDC_HIP(hipMemcpyAsync(fin.data(), p->d_fin, fin.size() * sizeof(double), hipMemcpyDeviceToHost, hs), "copy out");
    if (C_host)
        SDC_HIP(hipMemcpyAsync(C_host, p->d_C, (size_t)nl * L.n_bins * sizeof(double), hipMemcpyDeviceToHost, hs),
                "copy C");
    if (counts_host)
        SDC_HIP(hipMemcpyAsync(counts_host, p->d_counts, (size_t)L.n_bins * 8, hipMemcpyDeviceToHost, hs), "copy counts");
    hipError_t se = hipStreamSynchronize(hs);
    if (se != hipSuccess) {
        p->failed = true;
        return hip_err((int)se, "finalize (or earlier queued work)");
    }
    if (Csum_host) std::memcpy(Csum_host, fin.data(), nl * sizeof(double));
    if (Cself_host) std::memcpy(Cself_host, fin.data() + nl, nl * sizeof(double));
    if (Ssum_host) std::memcpy(Ssum_host, fin.data() + 2 * nl, 2 * nl * sizeof(double));
    if (Sself_host) std::memcpy(Sself_host, fin.data() + 4 * nl, 2 * nl * sizeof(double));
    return SDC_OK;
}

sdc_status sdc_plan_structure_factor(sdc_plan* p, const int32_t* m_host, int32_t n_q, double* Sqt_host,
                                     double* Sqw_host, void* stream) {
    g_err.clear();
    sdc_status s = plan_usable(p);
    if (s != SDC_OK) return s;
    if (!m_host || (!Sqt_host && !Sqw_host)) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    if (n_q < 1 || n_q > 65535) return set_err(SDC_ERR_INVALID_ARG, "n_q must be in [1, 65535]");
    if (p->lay.kind == SDC_BINS_RADIAL)
        return set_err(SDC_ERR_UNSUPPORTED, "S(q, t) from bins needs a periodic plan");
    for (int64_t x = 0; x < 3 * (int64_t)n_q; ++x)
        if (m_host[x] < -(1 << 20) || m_host[x] > (1 << 20))
            return set_err(SDC_ERR_INVALID_ARG, "wave-vector index out of range");
    SDC_HIP(select_device(p->device), "hipSetDevice");
    const int nl = p->corr.n_lags;
    const size_t out_n = (size_t)n_q * nl * 2;
    std::vector<void*> tmp;
    int32_t* d_m = nullptr;
    double* d_out = nullptr;
    s = dalloc(&d_m, (size_t)3 * n_q, &tmp);
    if (s == SDC_OK) s = dalloc(&d_out, 2 * out_n, &tmp);
    auto release = [&]() {
        for (void* q : tmp) (void)hipFree(q);
    };
    if (s != SDC_OK) {
        release();
        return s;
    }
    hipStream_t hs = (hipStream_t)stream;
    hipError_t he = hipMemcpyAsync(d_m, m_host, (size_t)3 * n_q * sizeof(int32_t), hipMemcpyHostToDevice, hs);
    if (he == hipSuccess) he = (hipError_t)refresh_fixed(p, stream);
    sdc::SqtArgs a{};
    a.H = p->d_H;
    a.n_org = p->d_norg;
    a.n_bins = p->lay.n_bins;
    a.n_sites = p->lay.n;
    a.n_lags = nl;
    a.kind = p->lay.kind;
    a.L0 = p->lay.L[0];
    a.L1 = p->lay.L[1];
    a.L2 = p->lay.L[2];
    a.m = d_m;
    a.n_q = n_q;
    a.sqt = d_out;
    a.sqw = d_out + out_n;
    int e = he == hipSuccess ? sdc::launch_sqt(a, stream) : (int)he;
    if (e == 0 && Sqt_host)
        e = (int)hipMemcpyAsync(Sqt_host, a.sqt, out_n * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == 0 && Sqw_host)
        e = (int)hipMemcpyAsync(Sqw_host, a.sqw, out_n * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == 0) e = (int)hipStreamSynchronize(hs);
    release();
    if (e != 0) {
        p->failed = true;
        return hip_err(e, "structure factor");
    }
    return SDC_OK;
}

sdc_status sdc_plan_structure_factor_static(sdc_plan* p, const int32_t* m_host, int32_t n_q, double* Sqt_host,
                                            double* Sqw_host, void* stream) {
    g_err.clear();
    sdc_status s = plan_usable(p);
    if (s != SDC_OK) return s;
    if (!m_host || (!Sqt_host && !Sqw_host)) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    if (n_q < 1 || n_q > 65535) return set_err(SDC_ERR_INVALID_ARG, "n_q must be in [1, 65535]");
    if (p->lay.kind == SDC_BINS_RADIAL)
        return set_err(SDC_ERR_UNSUPPORTED, "S(q, t) from bins needs a periodic plan");
    for (int64_t x = 0; x < 3 * (int64_t)n_q; ++x)
        if (m_host[x] < -(1 << 20) || m_host[x] > (1 << 20))
            return set_err(SDC_ERR_INVALID_ARG, "wave-vector index out of range");
    // scratch layout: m [3 n_q] int32 (padded to 256 bytes), S(q, t), S(q, w)
    const int nl = p->corr.n_lags;
    const size_t out_n = (size_t)n_q * nl * 2;
    const size_t m_bytes = ((size_t)3 * n_q * sizeof(int32_t) + 255) / 256 * 256;
    if (m_bytes + 2 * out_n * sizeof(double) > sdc::kStaticScratchBytes)
        return set_err(SDC_ERR_UNSUPPORTED, "n_q * n_lags too large for the fixed scratch (16 MiB: "
                                            "12 n_q + 32 n_q n_lags bytes)");
    SDC_HIP(select_device(p->device), "hipSetDevice");
    void* base = nullptr;
    {
        const int e = sdc::static_scratch(p->device, &base);
        if (e != 0) return hip_err(e, "fixed scratch address");
    }
    hipStream_t hs = (hipStream_t)stream;
    int32_t* d_m = (int32_t*)base;
    double* d_out = (double*)((char*)base + m_bytes);
    hipError_t he = hipMemcpyAsync(d_m, m_host, (size_t)3 * n_q * sizeof(int32_t), hipMemcpyHostToDevice, hs);
    if (he == hipSuccess) he = (hipError_t)refresh_fixed(p, stream);
    sdc::SqtArgs a{};
    a.H = p->d_H;
    a.n_org = p->d_norg;
    a.n_bins = p->lay.n_bins;
    a.n_sites = p->lay.n;
    a.n_lags = nl;
    a.kind = p->lay.kind;
    a.L0 = p->lay.L[0];
    a.L1 = p->lay.L[1];
    a.L2 = p->lay.L[2];
    a.m = d_m;
    a.n_q = n_q;
    a.sqt = d_out;
    a.sqw = d_out + out_n;
    int e = he == hipSuccess ? sdc::launch_sqt(a, stream) : (int)he;
    if (e == 0 && Sqt_host)
        e = (int)hipMemcpyAsync(Sqt_host, a.sqt, out_n * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == 0 && Sqw_host)
        e = (int)hipMemcpyAsync(Sqw_host, a.sqw, out_n * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == 0) e = (int)hipStreamSynchronize(hs);
    if (e != 0) {
        p->failed = true;
        return hip_err(e, "structure factor (fixed scratch)");
    }
    return SDC_OK;
}

sdc_status sdc_plan_raw(sdc_plan* p, double* H_host, double* n_org_host, double* self_host, double* msum_host,
                        void* stream) {
    g_err.clear();
    sdc_status s = plan_usable(p);
    if (s != SDC_OK) return s;
    SDC_HIP(select_device(p->device), "hipSetDevice");
    hipStream_t hs = (hipStream_t)stream;
    const int nl = p->corr.n_lags;
    {
        const int e = refresh_fixed(p, stream);
        if (e != 0) {
            p->failed = true;
            return hip_err(e, "fixed-point conversion");
        }
    }
    if (H_host)
        SDC_HIP(hipMemcpyAsync(H_host, p->d_H, (size_t)nl * p->lay.n_bins * 8, hipMemcpyDeviceToHost, hs), "copy H");
    if (self_host) SDC_HIP(hipMemcpyAsync(self_host, p->d_self, (size_t)nl * 8, hipMemcpyDeviceToHost, hs), "copy self");
    if (n_org_host)
        SDC_HIP(hipMemcpyAsync(n_org_host, p->d_norg, (size_t)nl * 8, hipMemcpyDeviceToHost, hs), "copy origin totals");
    if (msum_host)
        SDC_HIP(hipMemcpyAsync(msum_host, p->d_msum, (size_t)nl * 8, hipMemcpyDeviceToHost, hs), "copy site sums");
    hipError_t se = hipStreamSynchronize(hs);
    if (se != hipSuccess) {
        p->failed = true;
        return hip_err((int)se, "raw copy (or earlier queued work)");
    }
    return SDC_OK;
}

sdc_status sdc_plan_load_raw(sdc_plan* p, const double* H_host, const double* n_org_host, const double* self_host,
                             const double* msum_host, void* stream) {
    g_err.clear();
    sdc_status s = plan_usable(p);
    if (s != SDC_OK) return s;
    if (!H_host || !n_org_host || !self_host || !msum_host) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    const int nl = p->corr.n_lags;
    for (int t = 0; t < nl; ++t)
        if (!(n_org_host[t] >= 0.0)) return set_err(SDC_ERR_INVALID_ARG, "negative or NaN origin total");
    SDC_HIP(select_device(p->device), "hipSetDevice");
    hipStream_t hs = (hipStream_t)stream;
    SDC_HIP(hipMemcpyAsync(p->d_H, H_host, (size_t)nl * p->lay.n_bins * 8, hipMemcpyHostToDevice, hs), "load H");
    SDC_HIP(hipMemcpyAsync(p->d_self, self_host, (size_t)nl * 8, hipMemcpyHostToDevice, hs), "load self");
    SDC_HIP(hipMemcpyAsync(p->d_norg, n_org_host, (size_t)nl * 8, hipMemcpyHostToDevice, hs), "load origin totals");
    SDC_HIP(hipMemcpyAsync(p->d_msum, msum_host, (size_t)nl * 8, hipMemcpyHostToDevice, hs), "load site sums");
    if (p->d_Hq) {
        int e = sdc::launch_double_to_fixed(p->d_H, p->d_Hq, (int64_t)nl * p->lay.n_bins, stream);
        if (e == 0) e = sdc::launch_double_to_fixed(p->d_self, p->d_selfq, nl, stream);
        if (e != 0) {
            p->failed = true;
            return hip_err(e, "fixed-point conversion");
        }
    }
    hipError_t se = hipStreamSynchronize(hs);
    if (se != hipSuccess) {
        p->failed = true;
        return hip_err((int)se, "load raw");
    }
    return SDC_OK;
}

sdc_status sdc_plan_timings(sdc_plan* p, double* ms) {
    g_err.clear();
    sdc_status s = plan_usable(p);
    if (s != SDC_OK) return s;
    if (!ms) return set_err(SDC_ERR_INVALID_ARG, "null output");
    if (!(p->corr.flags & SDC_FLAG_TIMING) || !p->timed)
        return set_err(SDC_ERR_STATE, "no timed accumulate (create the plan with SDC_FLAG_TIMING)");
    SDC_HIP(hipEventSynchronize(p->ev[3]), "hipEventSynchronize");
    for (int k = 0; k < 3; ++k) {
        float t = 0.0f;
        SDC_HIP(hipEventElapsedTime(&t, p->ev[k], p->ev[k + 1]), "hipEventElapsedTime");
        ms[k] = t;
    }
    return SDC_OK;
}

sdc_status sdc_plan_reset(sdc_plan* p, void* stream) {
    g_err.clear();
    sdc_status s = plan_usable(p);
    if (s != SDC_OK) return s;
    SDC_HIP(select_device(p->device), "hipSetDevice");
    int e = sdc::launch_zero(p->d_H, (int64_t)p->corr.n_lags * p->lay.n_bins * 8, stream);
    if (e == 0) e = sdc::launch_zero(p->d_self, (int64_t)p->corr.n_lags * 8, stream);
    if (e == 0) e = sdc::launch_zero(p->d_norg, (int64_t)p->corr.n_lags * 8, stream);
    if (e == 0) e = sdc::launch_zero(p->d_msum, (int64_t)p->corr.n_lags * 8, stream);
    if (e == 0 && p->d_Hq) e = sdc::launch_zero(p->d_Hq, (int64_t)p->corr.n_lags * p->lay.n_bins * 8, stream);
    if (e == 0 && p->d_selfq) e = sdc::launch_zero(p->d_selfq, (int64_t)p->corr.n_lags * 8, stream);
    if (e != 0) {
        p->failed = true;
        return hip_err(e, "reset");
    }
    return SDC_OK;
}

sdc_status sdc_plan_destroy(sdc_plan* p) {
    g_err.clear();
    if (!p) return SDC_OK;
    if (p->batch_refs > 0) return set_err(SDC_ERR_STATE, "plan is held by a batch; destroy the batch first");
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    delete p;
    return SDC_OK;
}

sdc_status sdc_batch_create(sdc_plan* const* plans, int32_t n_plans, int32_t flags, sdc_batch** out) {
    return sdc_batch_create_tuned(plans, n_plans, flags, nullptr, out);
}

sdc_status sdc_batch_create_tuned(sdc_plan* const* plans, int32_t n_plans, int32_t flags, const sdc_tuning* tuning,
                                  sdc_batch** out) {
    g_err.clear();
    if (!out) return set_err(SDC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (!plans) return set_err(SDC_ERR_INVALID_ARG, "null plan list");
    if ((flags & ~SDC_FLAG_TIMING) != 0) return set_err(SDC_ERR_INVALID_ARG, "unknown flags");
    if (n_plans < 1 || n_plans > 4096) return set_err(SDC_ERR_INVALID_ARG, "n_plans must be in [1, 4096]");
    for (int k = 0; k < n_plans; ++k) {
        sdc_status s = plan_usable(plans[k]);
        if (s != SDC_OK) return s;
        for (int q = 0; q < k; ++q)
            if (plans[q] == plans[k]) return set_err(SDC_ERR_INVALID_ARG, "a plan appears twice in the batch");
        if (plans[k]->device != plans[0]->device) return set_err(SDC_ERR_INVALID_ARG, "plans on different devices");
        if (plans[k]->corr.precision != plans[0]->corr.precision)
            return set_err(SDC_ERR_INVALID_ARG, "plans of different precisions");
        if ((plans[k]->lay.kind == SDC_BINS_RADIAL) != (plans[0]->lay.kind == SDC_BINS_RADIAL))
            return set_err(SDC_ERR_INVALID_ARG, "radial and periodic plans in one batch");
    }
    const int device = plans[0]->device;
    const int prec = plans[0]->corr.precision;
    const int radial = plans[0]->lay.kind == SDC_BINS_RADIAL ? 1 : 0;
    // Schedule of the one launch: the caller's, else the one the plans' own
    // tunings give the most work (pair-terms times origins).
    int schedule = tuning ? tuning->schedule : SDC_SCHED_DEFAULT;
    if (schedule != SDC_SCHED_DEFAULT) {
        if (schedule < SDC_SCHED_ONE_PASS || schedule > SDC_SCHED_FOLD)
            return set_err(SDC_ERR_INVALID_ARG, "unknown schedule");
        if (!sdc::sched_valid(prec, sdc::sched_index(schedule)))
            return set_err(SDC_ERR_UNSUPPORTED, "schedule not available for this precision");
    } else {
        double w[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < n_plans; ++k)
            w[plans[k]->tuning.schedule] += (double)plans[k]->lay.n * (double)plans[k]->lay.n *
                                             plans[k]->corr.n_lags * plans[k]->corr.n_origins;
        schedule = SDC_SCHED_ONE_PASS;
        for (int sch = SDC_SCHED_TWO_PASS; sch <= SDC_SCHED_FOLD; ++sch)
            if (w[sch] > w[schedule]) schedule = sch;
    }
    SDC_HIP(hipSetDevice(device), "hipSetDevice");
    sdc_batch* b = nullptr;
    try {
        b = new sdc_batch();
    } catch (const std::bad_alloc&) {
        return set_err(SDC_ERR_OOM, "host allocation failed");
    }
    b->device = device;
    b->flags = flags;
    if (flags & SDC_FLAG_TIMING) {
        for (hipEvent_t& e : b->ev) {
            const hipError_t he = hipEventCreate(&e);
            if (he != hipSuccess) {
                delete b;
                return hip_err((int)he, "hipEventCreate");
            }
        }
    }
    // The launch's task list takes the plans in order of decreasing task
    // length (K-steps times tile pairs per segment), so the workgroups finish
    // on the short tasks of the small samples and the launch's tail is short;
    // the plans keep the caller's order everywhere else.
    std::vector<int> order((size_t)n_plans);
    for (int k = 0; k < n_plans; ++k) order[k] = k;
    auto task_len = [&](int k) {
        const sdc_plan* p = plans[k];
        return (double)p->nk * (double)p->lay.pairs.size() / (double)std::max<size_t>(1, p->lay.streams.size());
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return task_len(x) > task_len(y); });
    std::vector<sdc::FusedArgs> args((size_t)n_plans);
    std::vector<int64_t> start((size_t)n_plans + 1, 0);
    int lds = 0;
    for (int k = 0; k < n_plans; ++k) {
        sdc_plan* p = plans[k];
        const LagSel* sel = nullptr;
        sdc_status s = get_sel(p, nullptr, 0, &sel);
        if (s != SDC_OK) {
            delete b;
            return s;
        }
        b->plans.push_back(p);
        ++p->batch_refs;
        b->sels.push_back(sel);
    }
    for (int k = 0; k < n_plans; ++k) {
        const int q = order[k];
        sdc_status s = fused_args(plans[q], *b->sels[q], &args[k]);
        if (s != SDC_OK) {
            delete b;
            return s;
        }
        args[k].sched = sdc::sched_index(schedule);
        start[k + 1] = start[k] + (int64_t)args[k].n_groups * args[k].n_streams;
        lds = std::max(lds, sdc::fused_lds_bytes(args[k].win, prec));
    }
    if (start[n_plans] > (int64_t)INT32_MAX / 2) {
        delete b;
        return set_err(SDC_ERR_UNSUPPORTED, "too many fused tasks in the batch");
    }
    // XCD queue ranges of about equal work, cut at stream boundaries (all
    // lag groups of a stream segment in one queue).  Work of a stream's task:
    // its tile pairs times (K-steps + 4), the 4 standing for the per-pair
    // epilogue.
    std::vector<int32_t> ranges(9, 0);
    {
        std::vector<int64_t> cut;     // task index at the end of every stream, in list order
        std::vector<double> cum;      // work up to there
        double w = 0.0;
        for (int k = 0; k < n_plans; ++k) {
            const sdc_plan* p = plans[order[k]];
            for (size_t st = 0; st < p->lay.streams.size(); ++st) {
                const KStream& ks = p->lay.streams[st];
                w += (double)(ks.p1 - ks.p0) * (double)(p->nk + 4) * (double)args[k].n_groups;
                cut.push_back(start[k] + (int64_t)(st + 1) * args[k].n_groups);
                cum.push_back(w);
            }
        }
        size_t c = 0;
        for (int x = 1; x < 8; ++x) {
            const double target = w * x / 8.0;
            while (c < cum.size() && cum[c] < target) ++c;
            // the stream end nearest to the target, never before the previous cut
            int64_t r = c < cut.size() ? cut[c] : start[n_plans];
            if (c > 0 && c < cum.size() && target - cum[c - 1] < cum[c] - target) r = cut[c - 1];
            ranges[x] = (int32_t)std::max<int64_t>(r, ranges[x - 1]);
        }
        ranges[8] = (int32_t)start[n_plans];
    }
    sdc::FusedArgs* d_args = nullptr;
    int64_t* d_start = nullptr;
    unsigned* d_queue = nullptr;
    int32_t* d_ranges = nullptr;
    sdc_status s = dalloc(&d_args, args.size(), &b->owned);
    if (s == SDC_OK) s = dalloc(&d_start, start.size(), &b->owned);
    if (s == SDC_OK) s = dalloc(&d_queue, 8, &b->owned);
    if (s == SDC_OK) s = dalloc(&d_ranges, 9, &b->owned);
    if (s != SDC_OK) {
        delete b;
        return s;
    }
    hipError_t he = hipMemcpy(d_args, args.data(), args.size() * sizeof(sdc::FusedArgs), hipMemcpyHostToDevice);
    if (he == hipSuccess)
        he = hipMemcpy(d_start, start.data(), start.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(d_ranges, ranges.data(), 9 * sizeof(int32_t), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
        delete b;
        return hip_err((int)he, "upload batch tables");
    }
    sdc::BatchLaunch& bl = b->bl;
    bl.args = d_args;
    bl.task_start = d_start;
    bl.n_plans = n_plans;
    bl.queue = d_queue;
    bl.ranges = d_ranges;
    bl.total = (int)start[n_plans];
    bl.precision = prec;
    bl.radial = radial;
    bl.sched = sdc::sched_index(schedule);
    bl.lds = lds;
    b->schedule = schedule;
    const int e = sdc::batch_grid(prec, bl.sched, radial, lds, device, std::max(bl.total, 1), &bl.grid);
    if (e != 0) {
        delete b;
        return hip_err(e, "batch occupancy");
    }
    *out = b;
    return SDC_OK;
}

sdc_status sdc_batch_accumulate(sdc_batch* b, const float* const* spins_dev, const int64_t* n_frames, void* stream) {
    g_err.clear();
    if (!b) return set_err(SDC_ERR_INVALID_ARG, "null batch");
    if (!spins_dev || !n_frames) return set_err(SDC_ERR_INVALID_ARG, "null spins or frame counts");
    const size_t n = b->plans.size();
    for (size_t k = 0; k < n; ++k) {
        sdc_status s = plan_usable(b->plans[k]);
        if (s != SDC_OK) return s;
        if (!spins_dev[k]) return set_err(SDC_ERR_INVALID_ARG, "null spins");
        s = check_frames(b->plans[k], *b->sels[k], n_frames[k]);
        if (s != SDC_OK) return s;
    }
    SDC_HIP(select_device(b->device), "hipSetDevice");
    const bool timing = (b->flags & SDC_FLAG_TIMING) != 0;
    hipStream_t hs = (hipStream_t)stream;
    if (timing) SDC_HIP(hipEventRecord(b->ev[0], hs), "hipEventRecord");
    for (size_t k = 0; k < n; ++k) {
        sdc_status s = queue_pack_self(b->plans[k], *b->sels[k], spins_dev[k], n_frames[k], stream, false);
        if (s != SDC_OK) {
            for (sdc_plan* p : b->plans) p->failed = true;
            return s;
        }
    }
    if (timing) SDC_HIP(hipEventRecord(b->ev[1], hs), "hipEventRecord");
    const int e = sdc::launch_fused_batch(b->bl, stream);
    if (e != 0) {
        for (sdc_plan* p : b->plans) p->failed = true;
        return hip_err(e, "batched fused kernel");
    }
    if (timing) {
        SDC_HIP(hipEventRecord(b->ev[2], hs), "hipEventRecord");
        b->timed = true;
    }
    return SDC_OK;
}

sdc_status sdc_batch_timings(sdc_batch* b, double* ms) {
    g_err.clear();
    if (!b || !ms) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    if (!(b->flags & SDC_FLAG_TIMING) || !b->timed)
        return set_err(SDC_ERR_STATE, "no timed batch accumulate (create the batch with SDC_FLAG_TIMING)");
    SDC_HIP(hipEventSynchronize(b->ev[2]), "hipEventSynchronize");
    for (int k = 0; k < 2; ++k) {
        float t = 0.0f;
        SDC_HIP(hipEventElapsedTime(&t, b->ev[k], b->ev[k + 1]), "hipEventElapsedTime");
        ms[k] = t;
    }
    return SDC_OK;
}

sdc_status sdc_batch_info(const sdc_batch* b, int64_t* n_tasks, int32_t* grid) {
    g_err.clear();
    if (!b) return set_err(SDC_ERR_INVALID_ARG, "null batch");
    if (n_tasks) *n_tasks = b->bl.total;
    if (grid) *grid = b->bl.grid;
    return SDC_OK;
}

sdc_status sdc_batch_schedule(const sdc_batch* b, int32_t* schedule) {
    g_err.clear();
    if (!b || !schedule) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    *schedule = b->schedule;
    return SDC_OK;
}

sdc_status sdc_batch_destroy(sdc_batch* b) {
    g_err.clear();
    if (!b) return SDC_OK;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    delete b;
    return SDC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// q-resolved S(q, t) at arbitrary wave vectors
// ---------------------------------------------------------------------------

// Largest memory of the per-site-range partial transforms.
constexpr size_t kMaxSqPartBytes = (size_t)1 << 30;

struct sdc_sq {
    int device = 0;
    sdc_sq_spec spec{};
    int64_t n = 0;
    int n_q = 0;
    int t_used = 0;
    int t_pad = 0;
    int n_split = 1;
    int64_t sites_per_split = 0;
    std::vector<void*> owned;
    float* d_pos = nullptr;
    double* d_q = nullptr;
    double* d_pack = nullptr;  // [ceil(n / chunk)][t_pad][chunk][3] packed spins (chunk = sq_site_chunk())
    double* d_part = nullptr;  // [n_split][n_q][2][3 t_used]
    double* d_F = nullptr;     // [n_q][t_used][3][2]
    double* d_raw = nullptr;   // [n_q][n_lags][2]
    double* d_norg = nullptr;  // [1]
    double* d_out = nullptr;   // [2][n_q][n_lags][2]: S(q, t), S(q, w)
    bool failed = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool timed = false;

    ~sdc_sq() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        for (void* p : owned) (void)hipFree(p);
    }
};

namespace {

sdc_status sq_usable(const sdc_sq* q) {
    if (!q) return set_err(SDC_ERR_INVALID_ARG, "null accumulator");
    if (q->failed) return set_err(SDC_ERR_STATE, "accumulator is unusable after an earlier device failure");
    return SDC_OK;
}

}  // namespace

sdc_status sdc_sq_create(const float* positions_host, int64_t n_sites, const double* q_host, int32_t n_q,
                         const sdc_sq_spec* spec, int device, sdc_sq** out) {
    g_err.clear();
    if (!out) return set_err(SDC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (!positions_host || !q_host || !spec) return set_err(SDC_ERR_INVALID_ARG, "null pointer");
    if (n_sites < 1 || n_sites > ((int64_t)1 << 31)) return set_err(SDC_ERR_INVALID_ARG, "n_sites must be in [1, 2^31]");
    if (n_q < 1 || n_q > 65536) return set_err(SDC_ERR_INVALID_ARG, "n_q must be in [1, 65536]");
    if (spec->n_origins < 1 || spec->n_origins > 4096)
        return set_err(SDC_ERR_INVALID_ARG, "n_origins must be in [1, 4096]");
    if (spec->n_lags < 1 || spec->n_lags > 1024) return set_err(SDC_ERR_INVALID_ARG, "n_lags must be in [1, 1024]");
    if (spec->origin_stride < 1 || spec->origin_stride > 64)
        return set_err(SDC_ERR_INVALID_ARG, "origin_stride must be in [1, 64]");
    if ((spec->flags & ~(SDC_FLAG_TIMING | SDC_FLAG_CONNECTED)) != 0)
        return set_err(SDC_ERR_INVALID_ARG, "unknown flags (only TIMING and CONNECTED apply)");
    for (int64_t x = 0; x < 3 * n_sites; ++x)
        if (!std::isfinite(positions_host[x])) return set_err(SDC_ERR_INVALID_ARG, "non-finite position");
    for (int64_t x = 0; x < 3 * (int64_t)n_q; ++x)
        if (!std::isfinite(q_host[x])) return set_err(SDC_ERR_INVALID_ARG, "non-finite wave vector");
    // the kernels' sine and cosine take |q.r| < 2^20 (a bound through the
    // largest |q|_1 and the largest coordinate)
    double q1 = 0.0, rmax = 0.0;
    for (int32_t k = 0; k < n_q; ++k)
        q1 = std::max(q1, std::fabs(q_host[3 * k]) + std::fabs(q_host[3 * k + 1]) + std::fabs(q_host[3 * k + 2]));
    for (int64_t x = 0; x < 3 * n_sites; ++x) rmax = std::max(rmax, (double)std::fabs(positions_host[x]));
    if (q1 * rmax >= 1048576.0) return set_err(SDC_ERR_UNSUPPORTED, "phases |q.r| may reach 2^20 rad");
    sdc_status s = use_device(device);
    if (s != SDC_OK) return s;
    {
        const int e = sdc::prepare_sq_kernels();
        if (e != 0) return hip_err(e, "kernel attributes");
    }
    sdc_sq* q = nullptr;
    try {
        q = new sdc_sq();
    } catch (const std::bad_alloc&) {
        return set_err(SDC_ERR_OOM, "host allocation failed");
    }
    q->device = device;
    q->spec = *spec;
    q->n = n_sites;
    q->n_q = n_q;
    q->t_used = (spec->n_origins - 1) * spec->origin_stride + spec->n_lags;
    const int fb = sdc::sq_frames_per_block();
    q->t_pad = (q->t_used + fb - 1) / fb * fb;
    const int64_t n_cols = 3 * (int64_t)q->t_used;
    // Site ranges: enough workgroups to fill the chip (one per compute unit
    // at a time; 1536 to 3072 of them, the count that leaves the last round
    // of the chip fullest), at least four staged chunks per range, partials
    // within kMaxSqPartBytes.
    const int64_t chunk = sdc::sq_site_chunk();
    const int64_t tiles = sdc::sq_tiles_per_split(n_q, q->t_used);
    const size_t per_split = (size_t)n_q * 2 * n_cols * sizeof(double);
    int n_cu = 256;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n_cu < 1)
        n_cu = 256;
    const int64_t split_cap = std::max<int64_t>(1, std::min<int64_t>({n_sites / (4 * chunk),
        (int64_t)(kMaxSqPartBytes / per_split), 65535}));
    int64_t best_sps = 0, best_split = 0;
    double best_fill = -1.0;
    for (int64_t s = std::max<int64_t>(1, 1536 / tiles); s <= std::max<int64_t>(1, 3072 / tiles); ++s) {
        int64_t sps = (n_sites + std::min(s, split_cap) - 1) / std::min(s, split_cap);
        sps = (sps + chunk - 1) / chunk * chunk;
        const int64_t ns = (n_sites + sps - 1) / sps;
        const int64_t wg = tiles * ns, rounds = (wg + n_cu - 1) / n_cu;
        const double fill = (double)wg / (double)(rounds * n_cu);
        if (fill > best_fill + 1e-9) {
            best_fill = fill;
            best_sps = sps;
            best_split = ns;
        }
    }
    q->sites_per_split = best_sps;
    q->n_split = (int)best_split;
    const size_t out_n = (size_t)n_q * spec->n_lags * 2;
#define SQ_TRY(x)               \
    do {                        \
        sdc_status s_ = (x);    \
        if (s_ != SDC_OK) {     \
            delete q;           \
            return s_;          \
        }                       \
    } while (0)
    SQ_TRY(dalloc(&q->d_pos, (size_t)3 * n_sites, &q->owned));
    SQ_TRY(dalloc(&q->d_q, (size_t)3 * n_q, &q->owned));
    SQ_TRY(dalloc(&q->d_pack, (size_t)((n_sites + chunk - 1) / chunk) * q->t_pad * 3 * chunk, &q->owned));
    SQ_TRY(dalloc(&q->d_part, (size_t)q->n_split * n_q * 2 * n_cols, &q->owned));
    SQ_TRY(dalloc(&q->d_F, (size_t)n_q * 2 * n_cols, &q->owned));
    SQ_TRY(dalloc(&q->d_raw, out_n, &q->owned));
    SQ_TRY(dalloc(&q->d_norg, 1, &q->owned));
    SQ_TRY(dalloc(&q->d_out, 2 * out_n, &q->owned));
#undef SQ_TRY
    hipError_t e = hipMemcpy(q->d_pos, positions_host, (size_t)3 * n_sites * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(q->d_q, q_host, (size_t)3 * n_q * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = (hipError_t)sdc::launch_zero(q->d_raw, (int64_t)out_n * 8, nullptr);
    if (e == hipSuccess) e = (hipError_t)sdc::launch_zero(q->d_norg, 8, nullptr);
    if (e == hipSuccess && (spec->flags & SDC_FLAG_TIMING))
        for (hipEvent_t& ev : q->ev)
            if (e == hipSuccess) e = hipEventCreate(&ev);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete q;
        return hip_err((int)e, "accumulator set-up");
    }
    *out = q;
    return SDC_OK;
}

sdc_status sdc_sq_accumulate(sdc_sq* q, const float* spins_dev, int64_t n_frames, void* stream) {
    g_err.clear();
    sdc_status s = sq_usable(q);
    if (s != SDC_OK) return s;
    if (!spins_dev) return set_err(SDC_ERR_INVALID_ARG, "null spins");
    if (n_frames < q->t_used)
        return set_err(SDC_ERR_INVALID_ARG, "n_frames must be >= (n_origins - 1) * stride + n_lags");
    SDC_HIP(select_device(q->device), "hipSetDevice");
    const bool timing = (q->spec.flags & SDC_FLAG_TIMING) != 0;
    hipStream_t hs = (hipStream_t)stream;
    sdc::SqTransformArgs ta{};
    ta.frames = spins_dev;
    ta.packed = q->d_pack;
    ta.t_pad = q->t_pad;
    ta.pos = q->d_pos;
    ta.q = q->d_q;
    ta.n = q->n;
    ta.n_q = q->n_q;
    ta.n_frames_used = q->t_used;
    ta.n_split = q->n_split;
    ta.sites_per_split = q->sites_per_split;
    ta.part = q->d_part;
    sdc::SqCorrArgs ca{};
    ca.F = q->d_F;
    ca.n_q = q->n_q;
    ca.n_cols = 3 * (int64_t)q->t_used;
    ca.n_origins = q->spec.n_origins;
    ca.stride = q->spec.origin_stride;
    ca.n_lags = q->spec.n_lags;
    ca.connected = (q->spec.flags & SDC_FLAG_CONNECTED) ? 1 : 0;
    ca.raw = q->d_raw;
    ca.n_org = q->d_norg;
    if (timing) SDC_HIP(hipEventRecord(q->ev[0], hs), "hipEventRecord");
    int e = sdc::launch_sq_pack(ta, stream);
    if (e == 0 && timing) e = (int)hipEventRecord(q->ev[1], hs);
    if (e == 0) e = sdc::launch_sq_transform(ta, stream);
    if (e == 0 && timing) e = (int)hipEventRecord(q->ev[2], hs);
    if (e == 0) e = sdc::launch_sq_corr(ta, ca, stream);
    if (e == 0 && timing) e = (int)hipEventRecord(q->ev[3], hs);
    if (e != 0) {
        q->failed = true;
        return hip_err(e, "structure factor kernels");
    }
    if (timing) q->timed = true;
    return SDC_OK;
}

sdc_status sdc_sq_finalize(sdc_sq* q, double* Sqt_host, double* Sqw_host, void* stream) {
    g_err.clear();
    sdc_status s = sq_usable(q);
    if (s != SDC_OK) return s;
    if (!Sqt_host && !Sqw_host) return set_err(SDC_ERR_INVALID_ARG, "no output requested");
    SDC_HIP(select_device(q->device), "hipSetDevice");
    hipStream_t hs = (hipStream_t)stream;
    const size_t out_n = (size_t)q->n_q * q->spec.n_lags * 2;
    int e = sdc::launch_sq_finalize(q->d_raw, q->d_norg, q->n, q->n_q, q->spec.n_lags, q->d_out, q->d_out + out_n,
                                    stream);
    if (e == 0 && Sqt_host)
        e = (int)hipMemcpyAsync(Sqt_host, q->d_out, out_n * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == 0 && Sqw_host)
        e = (int)hipMemcpyAsync(Sqw_host, q->d_out + out_n, out_n * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == 0) e = (int)hipStreamSynchronize(hs);
    if (e != 0) {
        q->failed = true;
        return hip_err(e, "structure factor finalize (or earlier queued work)");
    }
    return SDC_OK;
}

sdc_status sdc_sq_timings(sdc_sq* q, double* ms) {
    g_err.clear();
    sdc_status s = sq_usable(q);
    if (s != SDC_OK) return s;
    if (!ms) return set_err(SDC_ERR_INVALID_ARG, "null output");
    if (!(q->spec.flags & SDC_FLAG_TIMING) || !q->timed)
        return set_err(SDC_ERR_STATE, "no timed accumulate (create with SDC_FLAG_TIMING)");
    SDC_HIP(hipEventSynchronize(q->ev[3]), "hipEventSynchronize");
    for (int k = 0; k < 3; ++k) {
        float t = 0.0f;
        SDC_HIP(hipEventElapsedTime(&t, q->ev[k], q->ev[k + 1]), "hipEventElapsedTime");
        ms[k] = t;
    }
    return SDC_OK;
}

sdc_status sdc_sq_reset(sdc_sq* q, void* stream) {
    g_err.clear();
    sdc_status s = sq_usable(q);
    if (s != SDC_OK) return s;
    SDC_HIP(select_device(q->device), "hipSetDevice");
    int e = sdc::launch_zero(q->d_raw, (int64_t)q->n_q * q->spec.n_lags * 16, stream);
    if (e == 0) e = sdc::launch_zero(q->d_norg, 8, stream);
    if (e != 0) {
        q->failed = true;
        return hip_err(e, "reset");
    }
    return SDC_OK;
}

sdc_status sdc_sq_destroy(sdc_sq* q) {
    g_err.clear();
    if (!q) return SDC_OK;
    (void)hipSetDevice(q->device);
    (void)hipDeviceSynchronize();
    delete q;
    return SDC_OK;
}
