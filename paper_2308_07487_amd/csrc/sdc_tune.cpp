// Autotuner of the fused product and the tuning file it writes.
//
// What is tuned per size class (device architecture, bin kind,
// floor(2 log2 N), K-steps, precision):
//  - the schedule of the fused kernel (one-pass, two-pass, lag-split or
//    fold; how the small split products are kept out of the large sums), and
//  - the number of tile pairs per fused task (segment length): the tasks of
//    one segment share a histogram and are merged into the global bins once;
//    shorter segments keep the lag groups that run together on an XCD close
//    enough in the pair list to share its L2, longer ones merge less.  The
//    lag groups of a segment start as the XCD's workgroup slots free up, so
//    unless their count divides the slots they drift apart by a fraction of
//    the segment (on a bcc 40^3 sample with 19 lag groups: 1.8 TB fetched
//    per launch with 16-pair segments, 12.3 TB with 96).
// The tuner times every candidate on the device (HIP events around the
// fused launch) and keeps the fastest; the results go to a small JSON file
// that plan creation reads (SDC_TUNING_FILE).  The paper's CUTLASS variants
// are tuned by hand per tile shape (Sec. 3.3-3.4, Fig. 2); here the choice is
// measured on the target device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include "sdc_internal.h"

namespace {

struct TuneKey {
    std::string arch;
    int kind = 0, n_class = 0, k_steps = 0, precision = 0;
    bool operator==(const TuneKey& o) const {
        return arch == o.arch && kind == o.kind && n_class == o.n_class && k_steps == o.k_steps &&
               precision == o.precision;
    }
};

struct TuneEntry {
    TuneKey key;
    sdc_tuning tuning{};
    double fused_ms = 0.0;
    std::string candidates;  // "schedule/segment:ms ..." of every candidate timed
};

// Size class of a sample: floor(2 log2 N) (half octaves), and the K-steps of
// the product, ceil(3 ceil(n_origins / 8) / 2).
TuneKey make_key(const std::string& arch, int64_t n_sites, const sdc_bin_spec* bins, const sdc_corr_spec* corr) {
    TuneKey k;
    k.arch = arch;
    k.kind = bins->kind;
    k.n_class = (int)std::floor(2.0 * std::log2((double)std::max<int64_t>(n_sites, 1)));
    const int o8 = (corr->n_origins + sdc::kOriginBlock - 1) / sdc::kOriginBlock;
    k.k_steps = (3 * o8 + 1) / 2;
    k.precision = corr->precision;
    return k;
}

sdc_status device_arch(int device, std::string* arch) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
        return sdc::set_error(SDC_ERR_NO_DEVICE, "no HIP device");
    if (device < 0 || device >= count) return sdc::set_error(SDC_ERR_INVALID_ARG, "device ordinal out of range");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return sdc::set_error(SDC_ERR_NO_DEVICE, "hipGetDeviceProperties failed");
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');  // "gfx950:sramecc+:xnack-" -> "gfx950"
    *arch = colon == std::string::npos ? a : a.substr(0, colon);
    return SDC_OK;
}

// --- the tuning file -------------------------------------------------------
//
// {"sdc_tuning": 1, "entries": [
//   {"arch": "gfx950", "kind": 0, "n_class": 31, "k_steps": 24, "precision": 1,
//    "schedule": 2, "segment_pairs": 96, "fused_ms": 12.5}, ...]}
//
// The reader takes every object of the "entries" array and the string or
// number value of each of its keys; unknown keys are ignored, an entry
// missing a key is skipped.

bool parse_entry(const std::string& obj, TuneEntry* e) {
    int have = 0;
    size_t i = 0;
    while (true) {
        const size_t q0 = obj.find('"', i);
        if (q0 == std::string::npos) break;
        const size_t q1 = obj.find('"', q0 + 1);
        if (q1 == std::string::npos) return false;
        const std::string key = obj.substr(q0 + 1, q1 - q0 - 1);
        size_t c = obj.find(':', q1 + 1);
        if (c == std::string::npos) return false;
        ++c;
        while (c < obj.size() && std::isspace((unsigned char)obj[c])) ++c;
        std::string val;
        if (c < obj.size() && obj[c] == '"') {
            const size_t v1 = obj.find('"', c + 1);
            if (v1 == std::string::npos) return false;
            val = obj.substr(c + 1, v1 - c - 1);
            i = v1 + 1;
        } else {
            size_t v1 = c;
            while (v1 < obj.size() && obj[v1] != ',' && obj[v1] != '}' && !std::isspace((unsigned char)obj[v1])) ++v1;
            val = obj.substr(c, v1 - c);
            i = v1;
        }
        char* end = nullptr;
        const double num = std::strtod(val.c_str(), &end);
        const bool is_num = end && *end == '\0' && !val.empty();
        if (key == "arch") {
            e->key.arch = val;
            have |= 1;
        } else if (key == "candidates") {
            e->candidates = val;
        } else if (is_num) {
            if (key == "kind") e->key.kind = (int)num, have |= 2;
            else if (key == "n_class") e->key.n_class = (int)num, have |= 4;
            else if (key == "k_steps") e->key.k_steps = (int)num, have |= 8;
            else if (key == "precision") e->key.precision = (int)num, have |= 16;
            else if (key == "schedule") e->tuning.schedule = (int32_t)num, have |= 32;
            else if (key == "segment_pairs") e->tuning.segment_pairs = (int32_t)num, have |= 64;
            else if (key == "fused_ms") e->fused_ms = num;
        }
    }
    return have == 127;
}

std::vector<TuneEntry> read_file(const char* path) {
    std::vector<TuneEntry> out;
    if (!path || !*path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos) return out;
    pos = text.find('[', pos);
    if (pos == std::string::npos) return out;
    while (true) {
        const size_t o0 = text.find_first_of("{]", pos);
        if (o0 == std::string::npos || text[o0] == ']') break;
        const size_t o1 = text.find('}', o0);
        if (o1 == std::string::npos) break;
        TuneEntry e;
        if (parse_entry(text.substr(o0 + 1, o1 - o0 - 1), &e)) out.push_back(e);
        pos = o1 + 1;
    }
    return out;
}

bool write_file(const char* path, std::vector<TuneEntry> entries) {
    std::sort(entries.begin(), entries.end(), [](const TuneEntry& a, const TuneEntry& b) {
        if (a.key.arch != b.key.arch) return a.key.arch < b.key.arch;
        if (a.key.kind != b.key.kind) return a.key.kind < b.key.kind;
        if (a.key.precision != b.key.precision) return a.key.precision < b.key.precision;
        if (a.key.n_class != b.key.n_class) return a.key.n_class < b.key.n_class;
        return a.key.k_steps < b.key.k_steps;
    });
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\"sdc_tuning\": 1, \"entries\": [\n");
    for (size_t k = 0; k < entries.size(); ++k) {
        const TuneEntry& e = entries[k];
        std::fprintf(f,
                     "  {\"arch\": \"%s\", \"kind\": %d, \"n_class\": %d, \"k_steps\": %d, \"precision\": %d, "
                     "\"schedule\": %d, \"segment_pairs\": %d, \"fused_ms\": %.4f, \"candidates\": \"%s\"}%s\n",
                     e.key.arch.c_str(), e.key.kind, e.key.n_class, e.key.k_steps, e.key.precision,
                     (int)e.tuning.schedule, (int)e.tuning.segment_pairs, e.fused_ms, e.candidates.c_str(),
                     k + 1 < entries.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

const TuneEntry* find(const std::vector<TuneEntry>& v, const TuneKey& k) {
    for (const TuneEntry& e : v)
        if (e.key == k) return &e;
    return nullptr;
}

bool split_precision(int p) { return p == SDC_PREC_SPLIT_BF16 || p == SDC_PREC_SPLIT_FP16; }

}  // namespace

namespace sdc {

sdc_status resolve_tuning(const sdc_tuning* given, int64_t n_sites, const sdc_bin_spec* bins,
                          const sdc_corr_spec* corr, int device, sdc_tuning* out) {
    sdc_tuning t{};
    if (given) t = *given;
    if (t.schedule < SDC_SCHED_DEFAULT || t.schedule > SDC_SCHED_FOLD)
        return set_error(SDC_ERR_INVALID_ARG, "unknown schedule");
    if (t.segment_pairs < 0 || t.segment_pairs > kMaxSegmentPairs)
        return set_error(SDC_ERR_INVALID_ARG, "segment_pairs must be 0 or in [1, 2^20]");
    if (t.schedule == SDC_SCHED_DEFAULT || t.segment_pairs == 0) {
        const char* path = std::getenv("SDC_TUNING_FILE");
        std::string arch;
        if (path && *path && device_arch(device, &arch) == SDC_OK) {
            const std::vector<TuneEntry> v = read_file(path);
            const TuneEntry* e = find(v, make_key(arch, n_sites, bins, corr));
            if (e) {
                if (t.schedule == SDC_SCHED_DEFAULT) t.schedule = e->tuning.schedule;
                if (t.segment_pairs == 0) t.segment_pairs = e->tuning.segment_pairs;
            }
        }
    }
    if (t.schedule == SDC_SCHED_DEFAULT)
        t.schedule = split_precision(corr->precision) ? SDC_SCHED_TWO_PASS : SDC_SCHED_ONE_PASS;
    if (t.schedule < SDC_SCHED_ONE_PASS || t.schedule > SDC_SCHED_FOLD)
        return set_error(SDC_ERR_INVALID_ARG, "unknown schedule in the tuning file");
    if (!sched_valid(corr->precision, sched_index(t.schedule)))
        return set_error(SDC_ERR_UNSUPPORTED, "schedule not available for this precision");
    if (t.segment_pairs <= 0 || t.segment_pairs > kMaxSegmentPairs) t.segment_pairs = default_segment_pairs(bins->kind);
    *out = t;
    return SDC_OK;
}

}  // namespace sdc

extern "C" {

sdc_status sdc_tuning_lookup(const char* cache_path, int64_t n_sites, const sdc_bin_spec* bins,
                             const sdc_corr_spec* corr, int device, sdc_tuning* tuning, int32_t* found) {
    if (!cache_path || !bins || !corr || !tuning || !found) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    std::string arch;
    sdc_status s = device_arch(device, &arch);
    if (s != SDC_OK) return s;
    const std::vector<TuneEntry> v = read_file(cache_path);
    const TuneEntry* e = find(v, make_key(arch, n_sites, bins, corr));
    *found = e ? 1 : 0;
    if (e) *tuning = e->tuning;
    sdc::set_error(SDC_OK, "");
    return SDC_OK;
}

sdc_status sdc_autotune_candidates(const sdc_bin_spec* bins, const sdc_corr_spec* corr, sdc_tuning* out,
                                   int32_t max_out, int32_t* n_out) {
    if (!bins || !corr || !n_out || (max_out > 0 && !out)) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    std::vector<int32_t> schedules = {SDC_SCHED_ONE_PASS, SDC_SCHED_LAG_SPLIT};
    if (split_precision(corr->precision)) schedules.push_back(SDC_SCHED_TWO_PASS);
    if (corr->precision != SDC_PREC_FP32) schedules.push_back(SDC_SCHED_FOLD);
    std::vector<int32_t> segments;
    if (bins->kind == SDC_BINS_RADIAL) segments = {64, 256, sdc::kMaxSegmentPairs};
    else segments = {16, 32, 48, 96, 192};
    int32_t n = 0;
    for (int32_t sch : schedules)
        for (int32_t seg : segments) {
            if (n < max_out) out[n] = sdc_tuning{sch, seg};
            ++n;
        }
    *n_out = n;
    sdc::set_error(SDC_OK, "");
    return SDC_OK;
}

sdc_status sdc_autotune(const float* positions_host, int64_t n_sites, const sdc_bin_spec* bins,
                        const sdc_corr_spec* corr, int device, int32_t max_lags, const sdc_tuning* candidates,
                        int32_t n_candidates, const char* cache_path, sdc_tuning* best, double* best_ms,
                        double* candidate_ms) {
    if (!positions_host || !bins || !corr || !best) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    std::string arch;
    sdc_status s = device_arch(device, &arch);
    if (s != SDC_OK) return s;
    if (corr->n_lags < 1 || corr->n_origins < 1 || corr->origin_stride < 1)
        return sdc::set_error(SDC_ERR_INVALID_ARG, "invalid correlation spec");
    std::vector<sdc_tuning> cands;
    if (candidates) {
        if (n_candidates < 1 || n_candidates > 4096) return sdc::set_error(SDC_ERR_INVALID_ARG, "n_candidates");
        cands.assign(candidates, candidates + n_candidates);
    } else {
        int32_t n = 0;
        sdc_autotune_candidates(bins, corr, nullptr, 0, &n);
        cands.resize(n);
        sdc_autotune_candidates(bins, corr, cands.data(), n, &n);
    }
    for (const sdc_tuning& t : cands)
        if (t.schedule == SDC_SCHED_DEFAULT || t.segment_pairs == 0)
            return sdc::set_error(SDC_ERR_INVALID_ARG, "candidates must set every field");

    const int n_use = max_lags > 0 ? std::min(max_lags, corr->n_lags) : corr->n_lags;
    std::vector<int32_t> lags(n_use);
    for (int t = 0; t < n_use; ++t) lags[t] = t;
    const int64_t n_frames = (int64_t)(corr->n_origins - 1) * corr->origin_stride + n_use;
    if (hipSetDevice(device) != hipSuccess) return sdc::set_error(SDC_ERR_HIP, "hipSetDevice failed");
    float* spins = nullptr;
    if (hipMalloc((void**)&spins, (size_t)n_frames * n_sites * 3 * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return sdc::set_error(SDC_ERR_OOM, "hipMalloc of the tuning spins failed");
    }
    int e = sdc::launch_unit_spins(spins, n_sites, n_frames, 0x5DC07E57ull, nullptr);
    if (e == 0) e = (int)hipDeviceSynchronize();
    if (e != 0) {
        (void)hipFree(spins);
        return sdc::set_error(SDC_ERR_HIP, std::string("tuning spins: ") + hipGetErrorString((hipError_t)e));
    }
    sdc_corr_spec c = *corr;
    c.flags |= SDC_FLAG_TIMING;
    // SDC_TUNE_VERBOSE set and not "0": one stderr line per candidate timed
    const char* env_verbose = std::getenv("SDC_TUNE_VERBOSE");
    const bool verbose = env_verbose && *env_verbose && std::strcmp(env_verbose, "0") != 0;
    std::vector<double> meds(cands.size(), 0.0);
    std::string summary;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        {
            const sdc_tuning cand = cands[ci];
            sdc_plan* p = nullptr;
            s = sdc_plan_create_tuned(positions_host, n_sites, bins, &c, &cand, device, &p);
            if (s != SDC_OK) {
                (void)hipFree(spins);
                return s;
            }
            std::vector<double> ms;
            for (int rep = 0; rep < 4 && s == SDC_OK; ++rep) {
                s = sdc_accumulate(p, spins, n_frames, lags.data(), n_use, nullptr);
                double t3[3];
                if (s == SDC_OK) s = sdc_plan_timings(p, t3);
                if (s == SDC_OK && rep > 0) ms.push_back(t3[2]);
            }
            const std::string err = sdc_last_error();
            sdc_plan_destroy(p);
            if (s != SDC_OK) {
                (void)hipFree(spins);
                return sdc::set_error(s, err);
            }
            std::sort(ms.begin(), ms.end());
            const double med = ms[ms.size() / 2];
            if (candidate_ms) candidate_ms[ci] = med;
            if (verbose)
                std::fprintf(stderr, "sdc_autotune: candidate %zu/%zu schedule %d segment %d: %.3f ms\n", ci + 1,
                             cands.size(), (int)cand.schedule, (int)cand.segment_pairs, med);
            char buf[64];
            std::snprintf(buf, sizeof buf, "%s%d/%d:%.3f", summary.empty() ? "" : " ", (int)cand.schedule,
                          (int)cand.segment_pairs, med);
            summary += buf;
            meds[ci] = med;
        }
    }
    (void)hipFree(spins);
    // Candidates within 0.5% of the fastest are ties within the timing
    // noise; of those the longest segment wins (fewer histogram merges, less
    // write traffic), then the faster.
    const double fastest = *std::min_element(meds.begin(), meds.end());
    size_t pick = 0;
    bool have = false;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        if (meds[ci] > fastest * 1.005) continue;
        if (!have || cands[ci].segment_pairs > cands[pick].segment_pairs ||
            (cands[ci].segment_pairs == cands[pick].segment_pairs && meds[ci] < meds[pick]))
            pick = ci;
        have = true;
    }
    *best = cands[pick];
    const double best_t = meds[pick];
    if (best_ms) *best_ms = best_t;
    if (cache_path) {
        std::vector<TuneEntry> v = read_file(cache_path);
        const TuneKey key = make_key(arch, n_sites, bins, corr);
        v.erase(std::remove_if(v.begin(), v.end(), [&](const TuneEntry& x) { return x.key == key; }), v.end());
        TuneEntry ne;
        ne.key = key;
        ne.tuning = *best;
        ne.fused_ms = best_t;
        ne.candidates = summary;
        v.push_back(ne);
        if (!write_file(cache_path, v)) return sdc::set_error(SDC_ERR_INVALID_ARG, "cannot write the tuning file");
    }
    sdc::set_error(SDC_OK, "");
    return SDC_OK;
}

}  // extern "C"
