// Tile layout of a sample: site permutation into tiles of 64, window tables
// and the stream/pair work lists of the fused kernel.
//
// Periodic lattices (bins = displacements modulo the box): sites are grouped
// in bricks of at most 4x4x4 cells of one sublattice.  For a fixed brick
// offset db every pair of bricks (I, I + db) sees displacements inside one
// small window, so one LDS histogram of window coordinates serves a whole
// stream of tile pairs and is mapped to global bins once.  This is the
// position-derived epilogue value of the paper's on-the-fly variant
// (Sec. 3.4, Eq. (6)) turned into a bin index.
//
// Radial shells: Morton-ordered tiles; one stream per i-tile over all j-tiles
// with a histogram over all shells.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "sdc_internal.h"

namespace sdc {

namespace {

int64_t pmod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

sdc_status fail(std::string* err, sdc_status s, const std::string& msg) {
    if (err) *err = msg;
    return s;
}

// Even chunking of [0, L) into nb chunks (sizes floor or ceil of L / nb).
void chunks(int L, int nb, std::vector<int>* start) {
    start->resize(nb + 1);
    for (int k = 0; k <= nb; ++k) (*start)[k] = (int)(((int64_t)k * L) / nb);
}

// Brick shape: chunk counts per axis such that a brick (at most
// ceil(L_a / nb_a) cells per axis) fits a 64-slot tile.  The product costs
// O(tiles^2), so the fewest tiles win; ties go to the smaller histogram
// window, then to the shape closest to 4 x 4 x 4.  Edges that are multiples
// of 4 keep 4 x 4 x 4 bricks with no padding; other edges avoid the up to
// 2.4x padding of fixed 4-cell chunks (a 10^3 box: 20 tiles of 5 x 5 x 2
// instead of 27 tiles of 4 x 4 x 4 slots).
void choose_bricks(const int L[3], int nb[3]) {
    int64_t best_tiles = -1, best_win = 0, best_dev = 0;
    for (int s0 = 1; s0 <= std::min(L[0], kTile); ++s0) {
        const int n0 = (L[0] + s0 - 1) / s0, m0 = (L[0] + n0 - 1) / n0;
        if (m0 != s0) continue;  // every chunk count once, by its largest chunk
        for (int s1 = 1; s1 <= std::min(L[1], kTile / s0); ++s1) {
            const int n1 = (L[1] + s1 - 1) / s1, m1 = (L[1] + n1 - 1) / n1;
            if (m1 != s1) continue;
            for (int s2 = 1; s2 <= std::min(L[2], kTile / (s0 * s1)); ++s2) {
                const int n2 = (L[2] + s2 - 1) / s2, m2 = (L[2] + n2 - 1) / n2;
                if (m2 != s2) continue;
                const int64_t tiles = (int64_t)n0 * n1 * n2;
                const int64_t win = (int64_t)(2 * s0) * (2 * s1) * (2 * s2);
                const int64_t dev = std::abs(s0 - 4) + std::abs(s1 - 4) + std::abs(s2 - 4);
                if (best_tiles < 0 || tiles < best_tiles || (tiles == best_tiles && win < best_win) ||
                    (tiles == best_tiles && win == best_win && dev < best_dev)) {
                    best_tiles = tiles;
                    best_win = win;
                    best_dev = dev;
                    nb[0] = n0;
                    nb[1] = n1;
                    nb[2] = n2;
                }
            }
        }
    }
}

uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

// Cut every stream into consecutive segments of at most `seg` pairs (same
// window, same bins).  The lag groups of a segment run as neighbouring tasks
// on one XCD and share its operands in L2 only while they are in step; over
// a whole stream (up to ~1000 pairs) they drift apart and the operand
// re-reads miss L2.  Shorter segments keep them in step at the price of
// more histogram merges (one per segment, lag group and window bin).
void split_streams(Layout* lay, int seg) {
    std::vector<KStream> out;
    for (const KStream& s : lay->streams) {
        const int len = s.p1 - s.p0;
        const int nseg = (len + seg - 1) / seg;
        for (int k = 0; k < nseg; ++k) {
            KStream t = s;
            t.p0 = s.p0 + (int)((int64_t)k * len / nseg);
            t.p1 = s.p0 + (int)((int64_t)(k + 1) * len / nseg);
            out.push_back(t);
        }
    }
    lay->streams.swap(out);
}

sdc_status build_periodic(const float* pos, int64_t n, const sdc_bin_spec* spec, int seg, Layout* lay,
                          std::string* err) {
    const bool bcc = spec->kind == SDC_BINS_PERIODIC_BCC;
    const int nsub = bcc ? 2 : 1;
    int L[3];
    for (int a = 0; a < 3; ++a) {
        L[a] = spec->cells[a];
        if (L[a] < 1 || L[a] > 4096) return fail(err, SDC_ERR_INVALID_ARG, "cells must be in [1, 4096]");
        lay->L[a] = L[a];
    }
    const int64_t cells = (int64_t)L[0] * L[1] * L[2];
    if (n != nsub * cells)
        return fail(err, SDC_ERR_INVALID_ARG, "n_sites must equal the number of lattice sites of the box");
    lay->n_bins = n;

    std::vector<int> st[3];
    std::vector<int> chunk_of[3];
    int nb[3], maxsz[3];
    choose_bricks(L, nb);
    for (int a = 0; a < 3; ++a) {
        chunks(L[a], nb[a], &st[a]);
        maxsz[a] = 0;
        chunk_of[a].assign(L[a], 0);
        for (int k = 0; k < nb[a]; ++k) {
            maxsz[a] = std::max(maxsz[a], st[a][k + 1] - st[a][k]);
            for (int x = st[a][k]; x < st[a][k + 1]; ++x) chunk_of[a][x] = k;
        }
    }
    // anchor differences A(k, db) = (start[(k + db) mod nb] - start[k]) mod L
    std::vector<int> amin[3], spread(3, 0);
    for (int a = 0; a < 3; ++a) {
        amin[a].assign(nb[a], 0);
        for (int d = 0; d < nb[a]; ++d) {
            int lo = 1 << 30, hi = -1;
            for (int k = 0; k < nb[a]; ++k) {
                int A = (int)pmod(st[a][(k + d) % nb[a]] - st[a][k], L[a]);
                lo = std::min(lo, A);
                hi = std::max(hi, A);
            }
            amin[a][d] = lo;
            spread[a] = std::max(spread[a], hi - lo);
        }
        lay->W[a] = 2 * (maxsz[a] - 1) + 1 + spread[a];
    }
    const int W0 = lay->W[0], W1 = lay->W[1], W2 = lay->W[2];
    lay->win = W0 * W1 * W2;
    const int nbt = nb[0] * nb[1] * nb[2];
    lay->n_tiles = nsub * nbt;
    lay->n_pad = (int64_t)lay->n_tiles * kTile;
    lay->perm.assign(lay->n_pad, -1);
    lay->gtab.assign(lay->n_pad, 0);

    auto tile_of = [&](int beta, int k0, int k1, int k2) {
        return ((beta * nb[0] + k0) * nb[1] + k1) * nb[2] + k2;
    };
    // slot q of a tile = brick cell (o0, o1, o2) with q = (o0 * s1 + o1) * s2 + o2,
    // s = largest chunk per axis; its window coordinate does not depend on the
    // tile, so padded slots (zero spins) get one in range as well
    const int brick = maxsz[0] * maxsz[1] * maxsz[2];
    for (int64_t p = 0; p < lay->n_pad; ++p) {
        const int q = (int)(p % kTile);
        if (q >= brick) continue;
        const int o0 = q / (maxsz[1] * maxsz[2]), o1 = (q / maxsz[2]) % maxsz[1], o2 = q % maxsz[2];
        lay->gtab[p] = (o0 * W1 + o1) * W2 + o2;
    }
    for (int64_t i = 0; i < n; ++i) {
        int c[3], beta = 0;
        if (!bcc) {
            for (int a = 0; a < 3; ++a) {
                double p = pos[3 * i + a];
                double r = std::floor(p + 0.5);
                if (!(std::fabs(p - r) <= 1e-3))
                    return fail(err, SDC_ERR_INVALID_ARG, "position is not a lattice point");
                c[a] = (int)pmod((int64_t)r, L[a]);
            }
        } else {
            int64_t d[3];
            for (int a = 0; a < 3; ++a) {
                double p = 2.0 * pos[3 * i + a];
                double r = std::floor(p + 0.5);
                if (!(std::fabs(p - r) <= 2e-3))
                    return fail(err, SDC_ERR_INVALID_ARG, "position is not a bcc lattice point");
                d[a] = (int64_t)r;
            }
            beta = (int)pmod(d[0], 2);
            if (pmod(d[1], 2) != beta || pmod(d[2], 2) != beta)
                return fail(err, SDC_ERR_INVALID_ARG, "position is not a bcc lattice point");
            for (int a = 0; a < 3; ++a) c[a] = (int)pmod((d[a] - beta) / 2, L[a]);
        }
        int k[3], o[3];
        for (int a = 0; a < 3; ++a) {
            k[a] = chunk_of[a][c[a]];
            o[a] = c[a] - st[a][k[a]];
        }
        int64_t p = (int64_t)tile_of(beta, k[0], k[1], k[2]) * kTile + (o[0] * maxsz[1] + o[1]) * maxsz[2] + o[2];
        if (lay->perm[p] >= 0) return fail(err, SDC_ERR_INVALID_ARG, "duplicate lattice site");
        lay->perm[p] = (int32_t)i;
    }
    const int stride[3] = {W1 * W2, W2, 1};
    lay->streams.reserve((size_t)nsub * nsub * nbt);
    lay->pairs.reserve((size_t)nsub * nsub * nbt * nbt);
    for (int bi = 0; bi < nsub; ++bi)
        for (int bj = 0; bj < nsub; ++bj)
            for (int d0 = 0; d0 < nb[0]; ++d0)
                for (int d1 = 0; d1 < nb[1]; ++d1)
                    for (int d2 = 0; d2 < nb[2]; ++d2) {
                        const int d[3] = {d0, d1, d2};
                        KStream s{};
                        s.p0 = (int32_t)lay->pairs.size();
                        const int cshift = (bcc && bj < bi) ? 1 : 0;
                        for (int a = 0; a < 3; ++a) s.base[a] = amin[a][d[a]] - (maxsz[a] - 1) - cshift;
                        s.parity = (int)pmod(bj - bi, 2);
                        for (int k0 = 0; k0 < nb[0]; ++k0)
                            for (int k1 = 0; k1 < nb[1]; ++k1)
                                for (int k2 = 0; k2 < nb[2]; ++k2) {
                                    const int k[3] = {k0, k1, k2};
                                    int kj[3], shift = 0;
                                    for (int a = 0; a < 3; ++a) {
                                        kj[a] = (k[a] + d[a]) % nb[a];
                                        int A = (int)pmod(st[a][kj[a]] - st[a][k[a]], L[a]);
                                        shift += (A - amin[a][d[a]] + maxsz[a] - 1) * stride[a];
                                    }
                                    KPair pr{};
                                    pr.ti = tile_of(bi, k0, k1, k2);
                                    pr.tj = tile_of(bj, kj[0], kj[1], kj[2]);
                                    pr.shift = shift;
                                    lay->pairs.push_back(pr);
                                }
                        s.p1 = (int32_t)lay->pairs.size();
                        lay->streams.push_back(s);
                    }
    split_streams(lay, seg);
    return SDC_OK;
}

sdc_status build_radial(const float* pos, int64_t n, const sdc_bin_spec* spec, int seg, Layout* lay,
                        std::string* err) {
    if (spec->n_shells < 1 || spec->n_shells > 1024)
        return fail(err, spec->n_shells < 1 ? SDC_ERR_INVALID_ARG : SDC_ERR_UNSUPPORTED,
                    "n_shells must be in [1, 1024]");
    if (!(spec->r_max > 0.0f) || !std::isfinite(spec->r_max))
        return fail(err, SDC_ERR_INVALID_ARG, "r_max must be finite and > 0");
    const int ns = spec->n_shells;
    lay->n_shells = ns;
    lay->n_bins = ns;
    lay->win = ns;
    lay->e2.resize(ns);
    const double w = (double)spec->r_max / (double)ns;
    for (int k = 0; k < ns; ++k) {
        double e = (double)k * w;
        lay->e2[k] = (float)(e * e);
    }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            float v = pos[3 * i + a];
            if (!std::isfinite(v)) return fail(err, SDC_ERR_INVALID_ARG, "non-finite position");
            lo[a] = std::min(lo[a], v);
            hi[a] = std::max(hi[a], v);
        }
    std::vector<std::pair<uint64_t, int64_t>> code(n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t m = 0;
        for (int a = 0; a < 3; ++a) {
            double ext = (double)hi[a] - lo[a];
            double u = ext > 0 ? ((double)pos[3 * i + a] - lo[a]) / ext : 0.0;
            uint64_t q = (uint64_t)std::min(1023.0, std::max(0.0, std::floor(u * 1024.0)));
            m |= spread3(q) << (2 - a);
        }
        code[i] = {m, i};
    }
    std::stable_sort(code.begin(), code.end());
    lay->n_tiles = (int32_t)((n + kTile - 1) / kTile);
    lay->n_pad = (int64_t)lay->n_tiles * kTile;
    lay->perm.assign(lay->n_pad, -1);
    lay->gtab.assign(lay->n_pad, 0);
    lay->pos4.assign(lay->n_pad * 4, 0.0f);
    for (int64_t p = 0; p < n; ++p) {
        int64_t i = code[p].second;
        lay->perm[p] = (int32_t)i;
        for (int a = 0; a < 3; ++a) lay->pos4[4 * p + a] = pos[3 * i + a];
    }
    lay->streams.reserve(lay->n_tiles);
    lay->pairs.reserve((size_t)lay->n_tiles * lay->n_tiles);
    for (int ti = 0; ti < lay->n_tiles; ++ti) {
        KStream s{};
        s.p0 = (int32_t)lay->pairs.size();
        for (int tj = 0; tj < lay->n_tiles; ++tj) lay->pairs.push_back(KPair{ti, tj, 0, 0});
        s.p1 = (int32_t)lay->pairs.size();
        lay->streams.push_back(s);
    }
    split_streams(lay, seg);
    return SDC_OK;
}

}  // namespace

sdc_status build_layout(const float* pos, int64_t n, const sdc_bin_spec* spec, int segment_pairs, Layout* lay,
                        std::string* err) {
    if (!pos || !spec || !lay) return fail(err, SDC_ERR_INVALID_ARG, "null pointer");
    if (segment_pairs < 1) return fail(err, SDC_ERR_INVALID_ARG, "segment_pairs must be >= 1");
    if (n < 1) return fail(err, SDC_ERR_INVALID_ARG, "n_sites must be >= 1");
    if (n > (int64_t)1 << 26) return fail(err, SDC_ERR_UNSUPPORTED, "n_sites above 2^26");
    *lay = Layout();
    lay->kind = spec->kind;
    lay->n = n;
    sdc_status s;
    if (spec->kind == SDC_BINS_PERIODIC_SC || spec->kind == SDC_BINS_PERIODIC_BCC)
        s = build_periodic(pos, n, spec, segment_pairs, lay, err);
    else if (spec->kind == SDC_BINS_RADIAL)
        s = build_radial(pos, n, spec, segment_pairs, lay, err);
    else
        return fail(err, SDC_ERR_INVALID_ARG, "unknown bin kind");
    if (s != SDC_OK) return s;
    if ((int64_t)lay->pairs.size() > (int64_t)INT32_MAX)
        return fail(err, SDC_ERR_UNSUPPORTED, "too many tile pairs");
    return SDC_OK;
}

int64_t window_bin(const Layout& lay, const KStream& s, int w) {
    const int w0 = w / (lay.W[1] * lay.W[2]);
    const int w1 = (w / lay.W[2]) % lay.W[1];
    const int w2 = w % lay.W[2];
    const int64_t k0 = pmod((int64_t)s.base[0] + w0, lay.L[0]);
    const int64_t k1 = pmod((int64_t)s.base[1] + w1, lay.L[1]);
    const int64_t k2 = pmod((int64_t)s.base[2] + w2, lay.L[2]);
    int64_t b = (k0 * lay.L[1] + k1) * lay.L[2] + k2;
    if (lay.kind == SDC_BINS_PERIODIC_BCC) b = 2 * b + s.parity;
    return b;
}

}  // namespace sdc
