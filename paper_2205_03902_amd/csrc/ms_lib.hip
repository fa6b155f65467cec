// libimsp host side: validation, plans, workspace layout and kernel launches
// behind the C ABI declared in include/ms.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ms.h"
#include "line_kernels.hpp"
#include "ms_kernels.hpp"

using namespace imsp;

namespace {

thread_local std::string g_err;

ms_status fail(ms_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

constexpr int kMaxBlocks = 256;    // partial-maximum blocks per segment
constexpr long long kScatterBlocks = 32768;   // target grid of the scatter pass
// Distinct sub-pixel probe shifts per plan.  A raster has a few; refined positions have one per
// position.  The class tables and partial sums take about (kChunks + 5) C N^2 8 bytes.
constexpr int kMaxClasses = 4096;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workgroups of a line launch per window: N / 16 groups of 16 lines aligned in object coordinates
// take N / 16 + 1 (line_kernels.hpp).
int line_groups(int n) { return n / 16 + 1; }

bool supported_n(int n) { return n == 16 || n == 32 || n == 64 || n == 128 || n == 256; }

// Windows up to 128 fit one workgroup (fused kernel); larger ones use the line kernels.
bool fused_fits(int n) { return n <= 128; }

ms_status validate(const ms_problem *pb)
{
    if (!pb) return fail(MS_ERR_INVALID_ARG, "problem is NULL");
    const int n = pb->n;
    if (n < 16 || n > 256 || (n & (n - 1)))
        return fail(MS_ERR_INVALID_ARG, "n must be a power of two in [16, 256]");
    if (!supported_n(n)) return fail(MS_ERR_UNSUPPORTED, "n = " + std::to_string(n) + " is not implemented");
    if (pb->obj_h < n || pb->obj_w < n) return fail(MS_ERR_INVALID_ARG, "object must be at least N x N");
    if (pb->obj_h > (1 << 20) || pb->obj_w > (1 << 20) || (int64_t)pb->obj_h * pb->obj_w > (int64_t)1 << 30)
        return fail(MS_ERR_INVALID_ARG, "object too large");
    if (pb->n_slices < 1 || pb->n_slices > 4096) return fail(MS_ERR_INVALID_ARG, "n_slices must be in [1, 4096]");
    if (pb->n_pos < 1 || pb->n_pos > ((int64_t)1 << 30)) return fail(MS_ERR_INVALID_ARG, "n_pos must be in [1, 2^30]");
    if (!pb->positions) return fail(MS_ERR_INVALID_ARG, "positions is NULL");
    if (pb->n_slices > 1 && !pb->dz) return fail(MS_ERR_INVALID_ARG, "dz is NULL");
    if (!(pb->pixel_size > 0.0) || !std::isfinite(pb->pixel_size))
        return fail(MS_ERR_INVALID_ARG, "pixel_size must be positive and finite");
    if (!(pb->wavelength > 0.0) || !std::isfinite(pb->wavelength))
        return fail(MS_ERR_INVALID_ARG, "wavelength must be positive and finite");
    if (!std::isfinite(pb->tilt_y) || !std::isfinite(pb->tilt_x)) return fail(MS_ERR_INVALID_ARG, "tilts must be finite");
    for (int64_t i = 0; i < 2 * pb->n_pos; ++i)
        if (!std::isfinite(pb->positions[i]) || std::fabs(pb->positions[i]) > 1e9)
            return fail(MS_ERR_INVALID_ARG, "position " + std::to_string(i / 2) + " is not finite or too large");
    for (int m = 0; m + 1 < pb->n_slices; ++m)
        if (!std::isfinite(pb->dz[m])) return fail(MS_ERR_INVALID_ARG, "dz is not finite");
    if (pb->checkpoint_every < 0) return fail(MS_ERR_INVALID_ARG, "checkpoint_every must be >= 0");
    return MS_OK;
}

// Host-side description derived from the problem: patch origins, shift classes,
// batches and scatter lists.
struct HostPlan {
    int n = 0, H = 0, W = 0, M = 0, C = 0;
    int K = 1;                                // incident waves stored every K slices (1: all)
    int64_t S = 0, B = 0;
    int nb = 0, tiles_x = 0, tiles_y = 0, n_tiles = 0;
    // 64 x 4 scatter tiles for the fused path's patches (natural layout), where that path exists
    bool wide = false;
    int wtiles_x = 0, wtiles_y = 0, n_wtiles = 0;
    std::vector<int4> pos_info;
    std::vector<double> cls_fy, cls_fx;
    std::vector<double> dz_unique;            // distinct slice distances
    std::vector<int> gap_table;               // M - 1 entries: index into dz_unique
    // Scatter lists.  Each batch is cut into at most kChunks chunks of consecutive
    // positions; per (batch, chunk, tile) the entries (batch-local s, origin y, origin x)
    // of the windows that touch the tile, per (batch, chunk, class) its positions.  The lists of
    // 16 x 16 tiles, then (wide) those of 64 x 4 tiles, back to back.
    std::vector<int> tile_off;                // nb x kChunks x (n_tiles + 1) [+ nb x kChunks x (n_wtiles + 1)]
    std::vector<int4> tile_list;              // entries of both, the offsets absolute
    std::vector<int> class_off, class_list;   // nb x kChunks x (C + 1), absolute offsets
    // Band sums of the line path's gradient patches (line_band_kernel).  Orientation o = 0: even
    // slices (natural frame), bands of one origin x ordered by origin y; o = 1: odd slices
    // (transposed frame), bands of one origin y ordered by origin x.  Per batch: the bands' members
    // (batch-local positions, absolute offsets) with their offsets from the band's first origin,
    // the workgroups (batch-local band, member range, first band line) and the scatter lists of the
    // band images (entries (batch-local band, origin y, origin x, spread)), chunked like the patch
    // lists with a count common to both orientations.
    bool bands[2] = {false, false};                  // per orientation: whether its bands pay
    int band_rows = 0;                               // lines of a band image (of N), a multiple of 16
    int64_t band_count = 0;                          // most bands of one batch and used orientation
    std::vector<int> wg_first[2];                    // nb + 1: first workgroup of each batch
    std::vector<int4> wg[2];
    std::vector<int> bmem[2], bdelta[2];
    std::vector<int> btile_off[2];                   // nb x kChunks x (n_tiles + 1), absolute offsets
    std::vector<int4> btile_list[2];
    std::vector<int> band_nch;                       // chunks per batch
};

// A batch of `count` positions is reduced in nch chunks of cs consecutive positions.
struct Chunking {
    int cs, nch;
};

Chunking chunking(int64_t count)
{
    Chunking c;
    c.cs = (int)((count + kChunks - 1) / kChunks);
    if (c.cs < 1) c.cs = 1;
    c.nch = (int)((count + c.cs - 1) / c.cs);
    return c;
}

// Chunk partial planes a scatter of a batch of B positions may write per slice: the chunks of any
// list of at most B entries (positions or bands).  chunking(B).nch can be fewer: 9 for B = 17,
// whose 16 bands would take 16.
int partial_chunks(int64_t B) { return (int)std::min<int64_t>(std::max<int64_t>(B, 1), kChunks); }

void derive_positions(const ms_problem *pb, HostPlan &hp)
{
    hp.n = pb->n; hp.H = pb->obj_h; hp.W = pb->obj_w; hp.M = pb->n_slices; hp.S = pb->n_pos;
    hp.tiles_y = (hp.H + kTileH - 1) / kTileH;
    hp.tiles_x = (hp.W + kTileW - 1) / kTileW;
    hp.n_tiles = hp.tiles_y * hp.tiles_x;
    hp.wide = hp.n <= 128;
    hp.wtiles_y = hp.wide ? (hp.H + kWideH - 1) / kWideH : 0;
    hp.wtiles_x = hp.wide ? (hp.W + kWideW - 1) / kWideW : 0;
    hp.n_wtiles = hp.wtiles_y * hp.wtiles_x;
    hp.pos_info.resize(hp.S);
    std::map<std::pair<double, double>, int> classes;
    for (int64_t s = 0; s < hp.S; ++s) {
        double py = pb->positions[2 * s], px = pb->positions[2 * s + 1];
        double fly = std::floor(py), flx = std::floor(px);
        int64_t iy = (int64_t)fly % hp.H, ix = (int64_t)flx % hp.W;
        if (iy < 0) iy += hp.H;
        if (ix < 0) ix += hp.W;
        std::pair<double, double> key(py - fly, px - flx);
        auto it = classes.find(key);
        int c;
        if (it == classes.end()) {
            c = (int)hp.cls_fy.size();
            classes.emplace(key, c);
            hp.cls_fy.push_back(key.first);
            hp.cls_fx.push_back(key.second);
        } else {
            c = it->second;
        }
        hp.pos_info[s] = make_int4((int)iy, (int)ix, c, 0);
    }
    hp.C = (int)hp.cls_fy.size();
    hp.gap_table.assign(std::max(hp.M - 1, 1), 0);
    for (int g = 0; g + 1 < hp.M; ++g) {
        auto it = std::find(hp.dz_unique.begin(), hp.dz_unique.end(), pb->dz[g]);
        if (it == hp.dz_unique.end()) {
            hp.gap_table[g] = (int)hp.dz_unique.size();
            hp.dz_unique.push_back(pb->dz[g]);
        } else {
            hp.gap_table[g] = (int)(it - hp.dz_unique.begin());
        }
    }
    if (hp.dz_unique.empty()) hp.dz_unique.push_back(0.0);
}

// Distinct slice distances the fused kernel keeps in LDS (HCap in ms_kernels.hpp).
int table_capacity(int n)
{
    switch (n) {
        case 16: return HCap<16>::U;
        case 32: return HCap<32>::U;
        case 64: return HCap<64>::U;
        case 128: return HCap<128>::U;
        default: return 1 << 30;   // the line kernels stage the two tables each launch needs
    }
}

bool too_many_classes(const HostPlan &hp) { return hp.C > kMaxClasses; }

// A tiling of the object for the scatter: tiles of tw x th pixels, tiles_x a row.
struct Tiling {
    int tw, th, tiles_x, tiles_y, n_tiles;
};
Tiling square_tiles(const HostPlan &hp) { return {kTileW, kTileH, hp.tiles_x, hp.tiles_y, hp.n_tiles}; }
Tiling wide_tiles(const HostPlan &hp) { return {kWideW, kWideH, hp.wtiles_x, hp.wtiles_y, hp.n_wtiles}; }

// Tiles (row-major) covered by the window of one position.
void window_tiles(const HostPlan &hp, const Tiling &tg, const int4 &info, std::vector<int> &rows,
                  std::vector<int> &cols, std::vector<char> &mark_y, std::vector<char> &mark_x)
{
    rows.clear(); cols.clear();
    std::fill(mark_y.begin(), mark_y.end(), 0);
    std::fill(mark_x.begin(), mark_x.end(), 0);
    for (int i = 0; i < hp.n; ++i) {
        int ty = ((info.x + i) % hp.H) / tg.th;
        if (!mark_y[ty]) { mark_y[ty] = 1; rows.push_back(ty); }
        int tx = ((info.y + i) % hp.W) / tg.tw;
        if (!mark_x[tx]) { mark_x[tx] = 1; cols.push_back(tx); }
    }
}

// The position lists of tiling tg appended to hp.tile_off / hp.tile_list (offsets absolute), and
// with classes also the class lists.
void append_lists(HostPlan &hp, const Tiling &tg, bool classes)
{
    const int64_t B = hp.B;
    std::vector<int> rows, cols;
    std::vector<char> my(tg.tiles_y), mx(tg.tiles_x);
    std::vector<std::vector<int>> per_pos(hp.S);
    size_t total = 0;
    for (int64_t s = 0; s < hp.S; ++s) {
        window_tiles(hp, tg, hp.pos_info[s], rows, cols, my, mx);
        per_pos[s].reserve(rows.size() * cols.size());
        for (int ty : rows)
            for (int tx : cols) per_pos[s].push_back(ty * tg.tiles_x + tx);
        total += per_pos[s].size();
    }
    const size_t tstride = (size_t)tg.n_tiles + 1, cstride = (size_t)hp.C + 1;
    const size_t off0 = hp.tile_off.size(), list0 = hp.tile_list.size();
    hp.tile_off.resize(off0 + (size_t)hp.nb * kChunks * tstride, 0);
    hp.tile_list.resize(list0 + total, make_int4(0, 0, 0, 0));
    if (classes) {
        hp.class_off.assign((size_t)hp.nb * kChunks * cstride, 0);
        hp.class_list.assign(hp.S, 0);
    }
    int base = (int)list0, cbase = 0;
    std::vector<int> cnt(tg.n_tiles), ccnt(hp.C);
    for (int b = 0; b < hp.nb; ++b) {
        const int64_t s0 = (int64_t)b * B, count = std::min(hp.S, s0 + B) - s0;
        const Chunking ch = chunking(count);
        for (int c = 0; c < kChunks; ++c) {
            const int64_t a0 = std::min<int64_t>((int64_t)c * ch.cs, count);
            const int64_t a1 = std::min<int64_t>(a0 + ch.cs, count);
            std::fill(cnt.begin(), cnt.end(), 0);
            std::fill(ccnt.begin(), ccnt.end(), 0);
            for (int64_t a = a0; a < a1; ++a) {
                for (int t : per_pos[s0 + a]) cnt[t]++;
                ccnt[hp.pos_info[s0 + a].z]++;
            }
            int *off = &hp.tile_off[off0 + ((size_t)b * kChunks + c) * tstride];
            off[0] = base;
            for (int t = 0; t < tg.n_tiles; ++t) off[t + 1] = off[t] + cnt[t];
            std::vector<int> cur(off, off + tg.n_tiles);
            for (int64_t a = a0; a < a1; ++a) {
                const int4 info = hp.pos_info[s0 + a];
                for (int t : per_pos[s0 + a]) hp.tile_list[cur[t]++] = make_int4((int)a, info.x, info.y, 0);
            }
            base = off[tg.n_tiles];
            if (!classes) continue;
            int *coff = &hp.class_off[((size_t)b * kChunks + c) * cstride];
            coff[0] = cbase;
            for (int k = 0; k < hp.C; ++k) coff[k + 1] = coff[k] + ccnt[k];
            std::vector<int> ccur(coff, coff + hp.C);
            for (int64_t a = a0; a < a1; ++a) hp.class_list[ccur[hp.pos_info[s0 + a].z]++] = (int)a;
            cbase = coff[hp.C];
        }
    }
}

void build_lists(HostPlan &hp, int64_t B)
{
    hp.B = B;
    hp.nb = (int)((hp.S + B - 1) / B);
    hp.tile_off.clear();
    hp.tile_list.clear();
    append_lists(hp, square_tiles(hp), true);
    if (hp.wide) append_lists(hp, wide_tiles(hp), false);
}

// Entries of the position lists of both tilings.
size_t tile_entries(const HostPlan &hp)
{
    std::vector<int> rows, cols;
    size_t total = 0;
    for (int w = 0; w < (hp.wide ? 2 : 1); ++w) {
        const Tiling tg = w ? wide_tiles(hp) : square_tiles(hp);
        std::vector<char> my(tg.tiles_y), mx(tg.tiles_x);
        for (int64_t s = 0; s < hp.S; ++s) {
            window_tiles(hp, tg, hp.pos_info[s], rows, cols, my, mx);
            total += rows.size() * cols.size();
        }
    }
    return total;
}

// One band: its members in order (batch-local positions), their offsets from the first origin
// along the cross axis, and the first member's origin.
struct Band {
    std::vector<int> mem, delta;
    int oy = 0, ox = 0;
};

// Bands of positions [s0, s0 + count) in orientation o (see HostPlan).  A band ends where the next
// origin lies more than N beyond the previous one (the windows would leave a gap) or more than
// H - N (W - N) beyond the first (the band image would wrap onto itself).
void make_bands(const HostPlan &hp, int64_t s0, int64_t count, int o, std::vector<Band> &out)
{
    out.clear();
    std::vector<int> idx((size_t)count);
    for (int64_t a = 0; a < count; ++a) idx[(size_t)a] = (int)a;
    auto key = [&](int a) {
        const int4 &q = hp.pos_info[s0 + a];
        return o == 0 ? std::make_tuple(q.y, q.x) : std::make_tuple(q.x, q.y);
    };
    std::sort(idx.begin(), idx.end(), [&](int a, int b) {
        const auto ka = key(a), kb = key(b);
        return ka != kb ? ka < kb : a < b;
    });
    const int limit = o == 0 ? hp.H - hp.n : hp.W - hp.n;
    for (size_t i = 0; i < idx.size();) {
        Band bd;
        const auto k0 = key(idx[i]);
        const int first = std::get<1>(k0);
        int prev = first;
        size_t e = i;
        while (e < idx.size()) {
            const auto k = key(idx[e]);
            if (std::get<0>(k) != std::get<0>(k0)) break;
            const int along = std::get<1>(k);
            if (e > i && (along - prev > hp.n || along - first > limit)) break;
            bd.mem.push_back(idx[e]);
            bd.delta.push_back(along - first);
            prev = along;
            ++e;
        }
        const int4 &q = hp.pos_info[s0 + idx[i]];
        bd.oy = q.x;
        bd.ox = q.y;
        out.push_back(std::move(bd));
        i = e;
    }
}

// Lines of a band image (rows of the object for o = 0, columns for o = 1): N plus the spread of
// its origins.
int band_extent(const HostPlan &hp, const Band &bd) { return hp.n + bd.delta.back(); }

// First line of a band's first workgroup: groups of 16 lines aligned in object coordinates (the
// band's first origin across the lines plus u0 is a multiple of 16).
int band_u_start(const Band &bd, int o) { return -((o == 0 ? bd.oy : bd.ox) & 15); }

// Workgroups of a band: its lines from band_u_start to the extent in groups of 16.
int band_groups(const HostPlan &hp, const Band &bd, int o)
{
    return (band_extent(hp, bd) - band_u_start(bd, o) + 15) / 16;
}

// Tiles covered by an image of rows x cols at origin (oy, ox), wrapping.
void image_tiles(const HostPlan &hp, int oy, int ox, int rows, int cols, std::vector<int> &out,
                 std::vector<char> &mark_y, std::vector<char> &mark_x)
{
    std::vector<int> ty_list, tx_list;
    std::fill(mark_y.begin(), mark_y.end(), 0);
    std::fill(mark_x.begin(), mark_x.end(), 0);
    for (int i = 0; i < rows; ++i) {
        const int ty = ((oy + i) % hp.H) / kTileH;
        if (!mark_y[ty]) { mark_y[ty] = 1; ty_list.push_back(ty); }
    }
    for (int i = 0; i < cols; ++i) {
        const int tx = ((ox + i) % hp.W) / kTileW;
        if (!mark_x[tx]) { mark_x[tx] = 1; tx_list.push_back(tx); }
    }
    out.clear();
    for (int ty : ty_list)
        for (int tx : tx_list) out.push_back(ty * hp.tiles_x + tx);
}

// Tiles of the band image of orientation o.
void band_tiles(const HostPlan &hp, const Band &bd, int o, std::vector<int> &out, std::vector<char> &my,
                std::vector<char> &mx)
{
    const int ext = band_extent(hp, bd);
    image_tiles(hp, bd.oy, bd.ox, o == 0 ? ext : hp.n, o == 0 ? hp.n : ext, out, my, mx);
}

// Band sizes for batches of B.  Bands of an orientation pay when their images take at most three
// quarters of the elements of the patches they replace; a band image holds the longest band of
// the used orientations (lines of N, rounded up to 16 lines).
struct BandStats {
    bool on[2] = {false, false};
    int rows = 0;
    int64_t count_max = 0, count[2] = {0, 0}, entries[2] = {0, 0}, workgroups[2] = {0, 0};
};

BandStats band_stats(const HostPlan &hp, int64_t B)
{
    BandStats bs;
    if (hp.n < 32) return bs;
    const int64_t nb = (hp.S + B - 1) / B;
    std::vector<Band> bands;
    std::vector<int> tiles;
    std::vector<char> my(hp.tiles_y), mx(hp.tiles_x);
    int64_t maxc[2] = {0, 0};
    int maxe[2] = {0, 0};
    double elems[2] = {0.0, 0.0};
    for (int o = 0; o < 2; ++o)
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t s0 = b * B, count = std::min(hp.S, s0 + B) - s0;
            make_bands(hp, s0, count, o, bands);
            bs.count[o] += (int64_t)bands.size();
            maxc[o] = std::max(maxc[o], (int64_t)bands.size());
            for (const Band &bd : bands) {
                const int ext = band_extent(hp, bd);
                maxe[o] = std::max(maxe[o], ext);
                elems[o] += (double)ext * hp.n;
                band_tiles(hp, bd, o, tiles, my, mx);
                bs.entries[o] += (int64_t)tiles.size();
                bs.workgroups[o] += band_groups(hp, bd, o);
            }
        }
    const double patches = (double)hp.S * hp.n * hp.n;
    for (int o = 0; o < 2; ++o) {
        bs.on[o] = elems[o] <= 0.75 * patches;
        if (bs.on[o]) bs.count_max = std::max(bs.count_max, maxc[o]);
    }
    const int longest = std::max(bs.on[0] ? maxe[0] : 0, bs.on[1] ? maxe[1] : 0);
    bs.rows = (longest + 15) / 16 * 16;
    return bs;
}

// Elements of one band image (the stride between a slice's band images).
size_t band_elems(const HostPlan &hp) { return (size_t)hp.n * hp.band_rows; }

void build_band_lists(HostPlan &hp)
{
    const int64_t B = hp.B;
    const size_t tstride = (size_t)hp.n_tiles + 1;
    std::vector<int> tiles;
    std::vector<char> my(hp.tiles_y), mx(hp.tiles_x);
    std::vector<std::vector<Band>> per(2 * (size_t)hp.nb);
    hp.band_nch.assign(hp.nb, 1);
    for (int o = 0; o < 2; ++o)
        for (int b = 0; b < hp.nb; ++b) {
            const int64_t s0 = (int64_t)b * B, count = std::min(hp.S, s0 + B) - s0;
            make_bands(hp, s0, count, o, per[(size_t)o * hp.nb + b]);
        }
    for (int b = 0; b < hp.nb; ++b)
        for (int o = 0; o < 2; ++o)
            if (hp.bands[o]) hp.band_nch[b] = std::max(hp.band_nch[b], chunking((int64_t)per[(size_t)o * hp.nb + b].size()).nch);
    for (int o = 0; o < 2; ++o) {
        hp.wg_first[o].assign(hp.nb + 1, 0);
        if (!hp.bands[o]) continue;
        hp.wg[o].clear(); hp.bmem[o].clear(); hp.bdelta[o].clear();
        hp.btile_off[o].assign((size_t)hp.nb * kChunks * tstride, 0);
        hp.btile_list[o].clear();
        std::vector<int> cnt(hp.n_tiles);
        int base = 0;
        for (int b = 0; b < hp.nb; ++b) {
            const std::vector<Band> &bands = per[(size_t)o * hp.nb + b];
            // members and workgroups: each 16 band lines, the members whose window meets them;
            // the longest first (ties in band and line order) so that the launch ends evenly
            hp.wg_first[o][b] = (int)hp.wg[o].size();
            std::vector<int4> wgs;
            for (size_t g = 0; g < bands.size(); ++g) {
                const Band &bd = bands[g];
                const int m0 = (int)hp.bmem[o].size();
                hp.bmem[o].insert(hp.bmem[o].end(), bd.mem.begin(), bd.mem.end());
                hp.bdelta[o].insert(hp.bdelta[o].end(), bd.delta.begin(), bd.delta.end());
                const int u_first = band_u_start(bd, o), groups = band_groups(hp, bd, o);
                size_t lo = 0, hi = 0;
                for (int k = 0; k < groups; ++k) {
                    const int u0 = u_first + 16 * k;
                    while (lo < bd.delta.size() && bd.delta[lo] + hp.n <= u0) ++lo;
                    while (hi < bd.delta.size() && bd.delta[hi] < u0 + 16) ++hi;
                    if (hi > lo) wgs.push_back(make_int4((int)g, m0 + (int)lo, m0 + (int)hi, u0));
                }
            }
            std::stable_sort(wgs.begin(), wgs.end(), [](const int4 &x, const int4 &y) { return x.z - x.y > y.z - y.y; });
            hp.wg[o].insert(hp.wg[o].end(), wgs.begin(), wgs.end());
            // scatter lists of the band images, chunks of consecutive bands
            const int64_t ng = (int64_t)bands.size();
            std::vector<std::vector<int>> cover((size_t)ng);
            for (int64_t g = 0; g < ng; ++g) band_tiles(hp, bands[(size_t)g], o, cover[(size_t)g], my, mx);
            const Chunking ch = chunking(ng);
            for (int c = 0; c < kChunks; ++c) {
                const int64_t a0 = std::min<int64_t>((int64_t)c * ch.cs, ng);
                const int64_t a1 = std::min<int64_t>(a0 + ch.cs, ng);
                std::fill(cnt.begin(), cnt.end(), 0);
                for (int64_t g = a0; g < a1; ++g)
                    for (int t : cover[(size_t)g]) cnt[t]++;
                int *off = &hp.btile_off[o][((size_t)b * kChunks + c) * tstride];
                off[0] = base;
                for (int t = 0; t < hp.n_tiles; ++t) off[t + 1] = off[t] + cnt[t];
                hp.btile_list[o].resize((size_t)off[hp.n_tiles]);
                std::vector<int> cur(off, off + hp.n_tiles);
                for (int64_t g = a0; g < a1; ++g) {
                    const Band &bd = bands[(size_t)g];
                    const int4 e = make_int4((int)g, bd.oy, bd.ox, bd.delta.back());
                    for (int t : cover[(size_t)g]) hp.btile_list[o][(size_t)cur[t]++] = e;
                }
                base = off[hp.n_tiles];
            }
        }
        hp.wg_first[o][hp.nb] = (int)hp.wg[o].size();
    }
}

// Stored incident waves per position: all M with K = 1; otherwise the checkpoints psi_K,
// psi_2K, ... (floor((M - 1) / K) of them) and one work slot, which holds the recomputed wave
// of the slice being taken and then its gradient patch.
int checkpoints(int M, int K) { return K > 1 ? (M - 1) / K : 0; }
int wave_slots(int M, int K) { return K > 1 ? checkpoints(M, K) + 1 : M; }
int overlap_slots(int M, int K) { return K > 1 ? 1 : M; }

// Workspace layout.  Every region is 256-byte aligned.
struct Layout {
    size_t tw, hy, hx, gap_table, ry, rx, ident, dry, drx, zero_ident, dprobe, pgrad, pcurv;
    size_t pos_info, pos_list, sub_list;
    size_t class_probe, class_acc, class_tmp, gp, layer_g, layer_w, maxt2, partial, maxw, scal;
    size_t full_g, full_w, maxw_all, mu_all;
    size_t tile_off, tile_list, class_off, class_list, sub_class_off, sub_class_list;
    size_t spart, wpart, cpart;
    size_t waves, probe_patch, overlap, loss_pos, half, replay, slices_t, loss_part, energy;
    size_t wg[2], bmem[2], bdelta[2], btile_off[2], btile_list[2], band;
    size_t total;
};

Layout make_layout(const HostPlan &hp, int64_t B, size_t n_entries)
{
    Layout L{};
    const size_t n = hp.n, NN = n * n, HW = (size_t)hp.H * hp.W, M = hp.M, C = hp.C, S = hp.S;
    const size_t gaps = std::max<size_t>(M - 1, 1);
    const size_t nb = (size_t)((S + B - 1) / B);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align_up(std::max<size_t>(bytes, 1)); return r; };
    L.tw = take((n / 16) * 17 * 8);
    L.hy = take(hp.dz_unique.size() * n * 8);
    L.hx = take(hp.dz_unique.size() * n * 8);
    L.gap_table = take(gaps * 4);
    L.ry = take(C * n * 8);
    L.rx = take(C * n * 8);
    L.ident = take(C * 4);
    L.dry = take(C * n * 8);
    L.drx = take(C * n * 8);
    L.zero_ident = take(C * 4);
    L.dprobe = take(2 * C * NN * 8);
    L.pgrad = take(S * 2 * 8);
    L.pcurv = take(S * 2 * 8);
    L.pos_info = take(S * 16);
    L.pos_list = take(S * 4);
    L.sub_list = take(S * 4);
    L.class_probe = take(C * NN * 8);
    L.class_acc = take(C * NN * 8);
    L.class_tmp = take(C * NN * 8);
    L.gp = take(NN * 8);
    L.layer_g = take(HW * 8);
    L.layer_w = take(HW * 4);
    L.maxt2 = take(M * 4);
    L.partial = take(M * kMaxBlocks * 4 + kMaxBlocks * 4);
    L.maxw = take(4);
    L.scal = take(8 * 8);
    L.full_g = take(M * HW * 8);
    L.full_w = take(M * HW * 4);
    L.maxw_all = take(M * 4);
    L.mu_all = take(M * 8);
    L.tile_off = take(nb * kChunks * ((size_t)hp.n_tiles + 1 + (hp.wide ? (size_t)hp.n_wtiles + 1 : 0)) * 4);
    L.tile_list = take(n_entries * 16);
    L.class_off = take(nb * kChunks * (C + 1) * 4);
    L.class_list = take(S * 4);
    L.sub_class_off = take(nb * kChunks * (C + 1) * 4);
    L.sub_class_list = take(S * 4);
    // chunk partials of the slices one scatter takes: all M at once, or one at a time when the
    // waves are recomputed slice by slice; a batch's band lists may have more chunks than its
    // position lists (at most min(B, 16))
    const size_t nch = (size_t)partial_chunks(B), scattered = hp.K > 1 ? 1 : M;
    L.spart = take(nch * scattered * HW * 8);
    L.wpart = take(nch * scattered * HW * 4);
    L.cpart = take(nch * C * NN * 8);
    L.waves = take((size_t)B * wave_slots(hp.M, hp.K) * NN * 8);
    L.probe_patch = take((size_t)B * NN * 8);
    L.overlap = take((size_t)B * overlap_slots(hp.M, hp.K) * NN * 4);
    L.loss_pos = take((size_t)B * 8);
    // line kernels: the two half-propagated windows per position that a chain of launches
    // alternates between (two more for recomputed waves), the odd slices transposed, per-line-group
    // partials; recomputation on the fused kernel parks its adjoint state in the first
    const bool lines_possible = hp.n >= 32;
    const size_t NA = n * (n + 16);    // a line window: rows of N + 16 (line_kernels.hpp)
    L.half = take(lines_possible ? 2 * (size_t)B * NA * 8 : (hp.K > 1 ? (size_t)B * NN * 8 : 0));
    L.replay = take((lines_possible && hp.K > 1) ? 2 * (size_t)B * NA * 8 : 0);
    L.slices_t = take(lines_possible ? (M / 2) * HW * 8 : 0);
    L.loss_part = take(lines_possible ? (size_t)B * line_groups(hp.n) * 8 : 0);
    L.energy = take((n / 16) * 8);
    // band sums of the line path: workgroups, members, scatter lists and the band images of the
    // slices one scatter takes
    const BandStats bs = band_stats(hp, B);
    for (int d = 0; d < 2; ++d) {
        const bool on = bs.on[d];
        L.wg[d] = take(on ? (size_t)bs.workgroups[d] * 16 : 0);
        L.bmem[d] = take(on ? S * 4 : 0);
        L.bdelta[d] = take(on ? S * 4 : 0);
        L.btile_off[d] = take(on ? nb * kChunks * (hp.n_tiles + 1) * 4 : 0);
        L.btile_list[d] = take(on ? (size_t)bs.entries[d] * 16 : 0);
    }
    L.band = take(scattered * (size_t)bs.count_max * n * bs.rows * 8);
    L.total = o;
    return L;
}

int64_t choose_batch(const HostPlan &hp, size_t n_entries, size_t budget)
{
    if (budget == 0) return hp.S;
    if (make_layout(hp, hp.S, n_entries).total <= budget) return hp.S;
    int64_t lo = 0, hi = hp.S;   // invariant: lo fits (or 0), hi does not
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(hp, mid, n_entries).total <= budget) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Wave storage and batch: a requested interval k (>= M means none stored) is kept and only
// the batch adapts to the budget; k = 0 takes every wave (K = 1) unless the budget cannot hold
// all positions that way, then the smallest K whose waves fit all positions, and only when K = M
// does not fit either, smaller batches.  Sets hp.K; returns the batch (0 if nothing fits).
int64_t choose_storage(HostPlan &hp, size_t n_entries, size_t budget, int k_req)
{
    if (hp.M < 2) {
        hp.K = 1;
        return choose_batch(hp, n_entries, budget);
    }
    if (k_req > 0) {
        hp.K = std::min(k_req, hp.M);
        return choose_batch(hp, n_entries, budget);
    }
    hp.K = 1;
    if (budget == 0) return hp.S;
    for (int k = 1; k <= hp.M; ++k) {
        if (k > 1 && k < hp.M && wave_slots(hp.M, k) == wave_slots(hp.M, k - 1)) continue;
        hp.K = k;
        if (make_layout(hp, hp.S, n_entries).total <= budget) return hp.S;
    }
    hp.K = hp.M;
    return choose_batch(hp, n_entries, budget);
}

}  // namespace

struct ms_plan {
    HostPlan hp;
    Layout L;
    double dx = 0, lambda = 0, tilt_y = 0, tilt_x = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    // host staging for subset uploads (kept alive until the next call)
    std::vector<int> sub_list, sub_class_off, sub_class_list;
    // optional timing of the fused kernel
    std::vector<hipEvent_t> ev_start, ev_stop;
    size_t ev_used = 0;
    bool lines = false;   // line kernels instead of the fused per-position kernel
    // the line path sums gradient patches into band images when the plan has them: of row and
    // column launches (MS_BANDS_ALL), row launches only, or none
    int band_mode = MS_BANDS_ALL;
    // with bands in both frames, the forward chain keeps each launch's window for the adjoint in
    // place of the wave (ms_plan_set_kept_windows)
    bool keep_windows = true;
    // Algorithm 1 on the line path (ms_plan_set_layer_carry): the layer whose incident wave slot 1
    // of the waves holds from the last layer step (-1: none), and the buffers it came from
    bool layer_carry = false;
    int carry_layer = -1;
    const void *carry_key[3] = {nullptr, nullptr, nullptr};
    // A second stream (default priority) for the probe-gradient reductions, which only read
    // what the per-position kernel wrote and so run beside the slice scatter; fork and join
    // through events on the caller's stream.
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int objective = MS_OBJECTIVE_AMPLITUDE;

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    // elements per position of the wave and overlap regions
    long long wave_stride() const { return (long long)wave_slots(hp.M, hp.K) * hp.n * hp.n; }
    long long ovl_stride() const { return (long long)overlap_slots(hp.M, hp.K) * hp.n * hp.n; }
    bool recompute() const { return hp.K > 1; }
    bool bands_active(int o) const
    {
        return lines && hp.bands[o] && (band_mode == MS_BANDS_ALL || (band_mode == MS_BANDS_ROWS && o == 0));
    }
    // whether the plain adjoint's forward chain keeps windows: every wave stored (K = 1) and the
    // M - 1 windows, rows of N + 16, fit where the M waves would be
    bool kept_windows() const
    {
        const long long n = hp.n;
        return lines && keep_windows && hp.K == 1 && hp.M > 1 && bands_active(0) && bands_active(1) &&
               (hp.M - 1) * n * (n + 16) <= hp.M * n * n;
    }
    // the fused path scatters its patches (natural layout) over 64 x 4 tiles
    bool wide_scatter() const { return !lines && hp.wide; }
    // offset of batch b's position-list offsets of the square (or the wide) tiling
    size_t tile_off_at(int b, bool wide) const
    {
        const size_t sq = (size_t)hp.nb * kChunks * (hp.n_tiles + 1);
        return wide ? sq + (size_t)b * kChunks * (hp.n_wtiles + 1) : (size_t)b * kChunks * (hp.n_tiles + 1);
    }
    long long band_stride() const { return (long long)band_elems(hp); }
    long long band_slice_stride() const { return (long long)hp.band_count * band_stride(); }
};

namespace {

ms_status check_hip(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return MS_OK;
}

template <int N>
void launch_fused_n(int mode, const FusedParams &fp, int count, hipStream_t st)
{
    dim3 grid(count), block(Win<N>::NT);
    switch (mode) {
        case kForward: fused_kernel<N, kForward><<<grid, block, 0, st>>>(fp); break;
        case kAdjoint: fused_kernel<N, kAdjoint><<<grid, block, 0, st>>>(fp); break;
        case kLayer: fused_kernel<N, kLayer><<<grid, block, 0, st>>>(fp); break;
        case kReplay: fused_kernel<N, kReplay><<<grid, block, 0, st>>>(fp); break;
        default: fused_kernel<N, kProbe><<<grid, block, 0, st>>>(fp); break;
    }
}

void launch_fused_raw(int n, int mode, const FusedParams &fp, int count, hipStream_t st)
{
    switch (n) {
        case 16: launch_fused_n<16>(mode, fp, count, st); break;
        case 32: launch_fused_n<32>(mode, fp, count, st); break;
        case 64: launch_fused_n<64>(mode, fp, count, st); break;
        case 128: launch_fused_n<128>(mode, fp, count, st); break;
        default: break;   // larger windows always take the line kernels
    }
}

template <int N>
void launch_line(bool tr, const LineParams &lp, int stage, int count, hipStream_t st)
{
    dim3 grid(line_groups(N), count), block(kLinesPerGroup * Win<N>::R);
    if (tr) line_kernel<N, true><<<grid, block, 0, st>>>(lp, stage);
    else line_kernel<N, false><<<grid, block, 0, st>>>(lp, stage);
}

// A line launch in frame tr (the transposed frame of odd slices).
void launch_line_n(int n, bool tr, const LineParams &lp, int stage, int count, hipStream_t st)
{
    switch (n) {
        case 32: launch_line<32>(tr, lp, stage, count, st); break;
        case 64: launch_line<64>(tr, lp, stage, count, st); break;
        case 128: launch_line<128>(tr, lp, stage, count, st); break;
        default: launch_line<256>(tr, lp, stage, count, st); break;
    }
}

template <int N>
void launch_band(bool tr, bool recomp, const LineParams &lp, const BandParams &bp, int workgroups, hipStream_t st)
{
    const dim3 block(kLinesPerGroup * Win<N>::R);
    if (recomp) {
        if (tr) line_band_kernel<N, true, true><<<workgroups, block, 0, st>>>(lp, bp);
        else line_band_kernel<N, false, true><<<workgroups, block, 0, st>>>(lp, bp);
    } else {
        if (tr) line_band_kernel<N, true, false><<<workgroups, block, 0, st>>>(lp, bp);
        else line_band_kernel<N, false, false><<<workgroups, block, 0, st>>>(lp, bp);
    }
}

// The two half-propagation buffers of a chain of line launches: each launch reads the one the
// previous launch wrote and writes the other.
struct PingPong {
    float2 *buf[2];
    int cur = 0;
    PingPong(float2 *base, long long elems) : buf{base, base + elems} {}
    void next(LineParams &lp)
    {
        lp.A_in = buf[cur];
        lp.A_out = buf[cur ^ 1];
        cur ^= 1;
    }
};

// The odd slices transposed (the rows of the line path's odd launches).
void transpose_odd(ms_plan *p, const float2 *slices, hipStream_t st)
{
    const HostPlan &hp = p->hp;
    if (hp.M < 2) return;
    const dim3 grid((hp.W + 31) / 32, (hp.H + 31) / 32, hp.M / 2);
    transpose_odd_kernel<<<grid, 256, 0, st>>>(slices, p->at<float2>(p->L.slices_t), hp.H, hp.W);
}

// Adjoint launch of slice lp.m for batch b with the gradient patches summed into the band images
// at out (in the frame of slice m); recomp: lp.psi_in holds the forward launch's windows of slice m
// rather than psi_m.
void launch_band_n(ms_plan *p, int b, const LineParams &lp, float2 *out, hipStream_t st, bool recomp = false)
{
    const HostPlan &hp = p->hp;
    const int o = lp.m & 1;
    const int first = hp.wg_first[o][b], workgroups = hp.wg_first[o][b + 1] - first;
    if (workgroups < 1) return;
    BandParams bp{};
    bp.wg = p->at<int4>(p->L.wg[o]) + first;
    bp.mem = p->at<int>(p->L.bmem[o]);
    bp.delta = p->at<int>(p->L.bdelta[o]);
    bp.band = out;
    bp.band_stride = p->band_stride();
    bp.rows = hp.band_rows;
    const bool tr = o == 1;
    switch (hp.n) {
        case 32: launch_band<32>(tr, recomp, lp, bp, workgroups, st); break;
        case 64: launch_band<64>(tr, recomp, lp, bp, workgroups, st); break;
        case 128: launch_band<128>(tr, recomp, lp, bp, workgroups, st); break;
        default: launch_band<256>(tr, recomp, lp, bp, workgroups, st); break;
    }
}

// Line-kernel parameters shared by every launch of one batch (per-launch fields cleared).
LineParams line_params(ms_plan *p, const FusedParams &fp, int mode)
{
    const HostPlan &hp = p->hp;
    LineParams lp{};
    lp.class_probe = fp.class_probe; lp.slices = fp.slices; lp.pos_info = fp.pos_info; lp.pos_list = fp.pos_list;
    lp.slices_t = p->at<float2>(p->L.slices_t);
    lp.tw = fp.tw; lp.hy = fp.hy; lp.hx = fp.hx; lp.gap_table = fp.gap_table;
    lp.measured = fp.measured; lp.intensity = fp.intensity; lp.exit_waves = fp.exit_waves;
    lp.probe_patch = fp.probe_patch;
    lp.loss_part = p->at<double>(p->L.loss_part);
    lp.H = hp.H; lp.W = hp.W; lp.M = hp.M;
    lp.mode = mode;
    lp.objective = fp.objective;
    return lp;
}

// Forward launches m = 0..M-1 (layout of slice m: rows for even m), the far-field launch
// in the other layout, then (unless forward-only) the adjoint launches m = M-1 .. m_stop.
// Every wave the mode needs is stored (K = 1 layout; the layer mode uses slot 0).
// Batch b >= 0 of a plain adjoint sums the gradient patches into bands when the plan has them;
// when both frames do, the forward chain writes the window of each launch m = 1 .. M-1 into a
// kept slot instead of a ping-pong buffer and stores no wave, and the band launches finish psi_m
// from it (kept_windows).
void run_lines(ms_plan *p, int mode, const FusedParams &fp, int count, hipStream_t st, int b)
{
    const HostPlan &hp = p->hp;
    const int M = hp.M;
    const long long NN = (long long)hp.n * hp.n, NA = (long long)hp.n * (hp.n + 16);
    float2 *waves = fp.waves;
    LineParams lp = line_params(p, fp, mode);
    PingPong A(p->at<float2>(p->L.half), (long long)hp.B * NA);
    const bool bands = mode == kAdjoint && !fp.full && b >= 0;
    const bool keep = bands && p->kept_windows();
    auto kept = [&](int m) { return waves + (long long)(m - 1) * hp.B * NA; };
    transpose_odd(p, fp.slices, st);
    // the layer mode's wave of its slice: slot 0, or slot 1 when it is carried to the next step
    float2 *layer_wave = (mode == kLayer && fp.carry) ? waves + NN : waves;
    const int m_first = (mode == kLayer) ? fp.chain_from : 0;
    for (int m = m_first; m < M; ++m) {
        lp.m = m;
        lp.psi_out = nullptr;
        lp.ovl_out = nullptr;
        lp.restart = (m == m_first && m > 0) ? fp.chain_wave : nullptr;
        lp.restart_stride = fp.wave_stride;
        if (m > 0 && mode == kAdjoint && !keep) { lp.psi_out = waves + m * NN; lp.psi_out_stride = fp.wave_stride; }
        // a restart at the layer's own slice reads the wave already there
        if (m > 0 && mode == kLayer && m == fp.layer && !(lp.restart == layer_wave)) {
            lp.psi_out = layer_wave;
            lp.psi_out_stride = fp.wave_stride;
        }
        if (mode == kLayer && m == fp.layer) { lp.ovl_out = fp.overlap_patch; lp.ovl_stride = fp.ovl_stride; }
        A.next(lp);
        if (keep) {
            if (m > 0) lp.A_in = kept(m);
            if (m + 1 < M) lp.A_out = kept(m + 1);
        }
        launch_line_n(hp.n, (m & 1) != 0, lp, kStageForward, count, st);
    }
    // the adjoint chain keeps A with per-position offsets from its first launch on when band
    // workgroups take part in it (the far field writes aligned windows)
    const bool obj = bands && (p->bands_active(0) || p->bands_active(1));
    lp.psi_out = nullptr;
    lp.ovl_out = nullptr;
    lp.restart = nullptr;
    lp.m = M - 1;
    A.next(lp);    // the buffer the last forward launch wrote, also when the others were kept
    launch_line_n(hp.n, (M & 1) != 0, lp, kStageFar, count, st);
    if (mode == kForward) return;
    lp.obj_out = obj ? 1 : 0;
    const int m_stop = (mode == kLayer) ? fp.layer : 0;
    for (int m = M - 1; m >= m_stop; --m) {
        lp.m = m;
        lp.patch_out = nullptr;
        lp.psi_in = nullptr;
        lp.ovl_out = nullptr;
        if (mode == kAdjoint) {
            lp.patch_out = waves + m * NN;
            lp.psi_in = m > 0 ? waves + m * NN : nullptr;
            if (fp.full) { lp.ovl_out = fp.overlap_patch + m * NN; lp.ovl_stride = fp.ovl_stride; }
        } else if (mode == kLayer && m == fp.layer) {
            lp.patch_out = waves;
            lp.psi_in = m > 0 ? layer_wave : nullptr;
        }
        lp.patch_stride = lp.psi_in_stride = fp.wave_stride;
        if (keep) {
            lp.psi_in = m > 0 ? kept(m) : nullptr;
            lp.psi_in_stride = NA;
        }
        lp.go_on = (m > m_stop) || (mode != kLayer);
        A.next(lp);
        if (bands && p->bands_active(m & 1))
            launch_band_n(p, b, lp, p->at<float2>(p->L.band) + m * p->band_slice_stride(), st, keep);
        else
            launch_line_n(hp.n, (m & 1) != 0, lp, kStageAdjoint, count, st);
        lp.obj_in = lp.obj_out;
    }
}

// Event pair around a group of per-position launches, while profiling is on.
struct TimedRegion {
    ms_plan *p;
    hipStream_t st;
    bool on;
    TimedRegion(ms_plan *plan, hipStream_t stream) : p(plan), st(stream), on(plan->ev_used < plan->ev_start.size())
    {
        if (on) (void)hipEventRecord(p->ev_start[p->ev_used], st);
    }
    ~TimedRegion()
    {
        if (on) (void)hipEventRecord(p->ev_stop[p->ev_used++], st);
    }
};

// All per-position work of one batch, with optional timing.
void launch_fused(ms_plan *p, int mode, const FusedParams &fp, int count, hipStream_t st, int b = -1)
{
    TimedRegion t(p, st);
    if (p->lines) run_lines(p, mode, fp, count, st, b);
    else launch_fused_raw(p->hp.n, mode, fp, count, st);
}

void scatter(ms_plan *p, int b, int count, const float2 *patches, long long pos_stride, const float *wpatch,
             long long w_stride, int m0, int n_m, float2 *out, float *wout, int accumulate, hipStream_t st);
void scatter_slices(ms_plan *p, int b, int count, const float2 *patches, long long pos_stride, int m0, int n_m,
                    float2 *out, int accumulate, hipStream_t st);

// Adjoint of one batch with recomputed incident waves (K > 1): the forward chain stores psi_K,
// psi_2K, ... and the head slice M - 1; then, slice by slice from M - 1 down to 0, the wave of the
// slice is recomputed from the nearest stored one below (or the probe), its gradient patch written
// to the work slot and scattered into g (and |psi|^2 into w when the step sizes need it) before
// the next slice overwrites the slot.  Each slice's launches are one timed region.
void adjoint_recompute(ms_plan *p, FusedParams fp, int b, int count, hipStream_t st, float2 *g, float *w,
                       int accumulate)
{
    const HostPlan &hp = p->hp;
    const int M = hp.M, K = hp.K, nck = checkpoints(M, K);
    const long long NN = (long long)hp.n * hp.n, hw = (long long)hp.H * hp.W;
    float2 *waves = fp.waves;
    float2 *work = waves + nck * NN;
    auto ck_slot = [&](int m) { return waves + (long long)(m / K - 1) * NN; };
    const float *ovl = w ? fp.overlap_patch : nullptr;
    fp.full = w ? 1 : 0;
    if (!p->lines) {
        for (int seg = M - 1; seg >= 0; --seg) {
            fp.seg = seg;
            {
                TimedRegion t(p, st);
                launch_fused_raw(hp.n, kReplay, fp, count, st);
            }
            scatter(p, b, count, work, fp.wave_stride, ovl, fp.ovl_stride, seg, 1, g + seg * hw,
                    w ? w + seg * hw : nullptr, accumulate, st);
        }
        return;
    }
    LineParams lp = line_params(p, fp, kAdjoint);
    const long long pair = (long long)hp.B * hp.n * (hp.n + 16);
    PingPong A(p->at<float2>(p->L.half), pair);
    transpose_odd(p, fp.slices, st);
    // the adjoint chain keeps A with per-position offsets when band workgroups take part in it
    const bool obj = !w && (p->bands_active(0) || p->bands_active(1));
    {
        TimedRegion t(p, st);
        for (int m = 0; m < M; ++m) {
            lp.m = m;
            lp.psi_out = nullptr;
            if (m > 0 && m % K == 0) lp.psi_out = ck_slot(m);
            else if (m == M - 1) lp.psi_out = work;
            lp.psi_out_stride = fp.wave_stride;
            A.next(lp);
            launch_line_n(hp.n, (m & 1) != 0, lp, kStageForward, count, st);
        }
        lp.psi_out = nullptr;
        lp.m = M - 1;
        A.next(lp);
        launch_line_n(hp.n, (M & 1) != 0, lp, kStageFar, count, st);
    }
    lp.obj_out = obj ? 1 : 0;
    lp.patch_out = work;
    lp.patch_stride = lp.psi_in_stride = fp.wave_stride;
    lp.go_on = 1;
    if (w) { lp.ovl_out = fp.overlap_patch; lp.ovl_stride = fp.ovl_stride; }
    for (int m = M - 1; m >= 0; --m) {
        TimedRegion t(p, st);
        if (m < M - 1 && m % K != 0) {
            // psi_m again: from the stored wave psi_c (or the probe), the forward launches c .. m
            // in the second pair of half-propagation buffers, the last one ending at psi_m in the
            // work slot
            const int c = m - m % K;
            LineParams rp = lp;
            PingPong Rb(p->at<float2>(p->L.replay), pair);
            rp.obj_in = rp.obj_out = 0;
            rp.patch_out = nullptr;
            rp.psi_in = nullptr;
            rp.ovl_out = nullptr;
            rp.probe_patch = nullptr;
            rp.go_on = 0;
            for (int mm = c; mm <= m; ++mm) {
                rp.m = mm;
                rp.restart = (mm == c && c > 0) ? ck_slot(c) : nullptr;
                rp.restart_stride = fp.wave_stride;
                rp.psi_out = (mm == m) ? work : nullptr;
                rp.psi_out_stride = fp.wave_stride;
                rp.stop_after_psi = (mm == m) ? 1 : 0;
                Rb.next(rp);
                launch_line_n(hp.n, (mm & 1) != 0, rp, kStageForward, count, st);
            }
        }
        lp.m = m;
        lp.psi_in = (m == 0) ? nullptr : (m % K == 0 ? ck_slot(m) : work);
        A.next(lp);
        const LineParams cur = lp;
        lp.obj_in = lp.obj_out;      // the next adjoint launch reads what this one writes
        if (!w && p->bands_active(m & 1)) {
            launch_band_n(p, b, cur, p->at<float2>(p->L.band), st);
            scatter_slices(p, b, count, work, fp.wave_stride, m, 1, g + m * hw, accumulate, st);
            continue;
        }
        launch_line_n(hp.n, (m & 1) != 0, cur, kStageAdjoint, count, st);
        scatter(p, b, count, work, fp.wave_stride, ovl, fp.ovl_stride, m, 1, g + m * hw, w ? w + m * hw : nullptr,
                accumulate, st);
    }
}

// Per-position losses of the last batch: where they are and how many.
const double *loss_entries(ms_plan *p, int count, int *n_entries)
{
    if (p->lines) {
        *n_entries = count * line_groups(p->hp.n);
        return p->at<double>(p->L.loss_part);
    }
    *n_entries = count;
    return p->at<double>(p->L.loss_pos);
}

template <int N>
void launch_filter_n(bool conj, const float2 *in, long long in_stride, float2 *out, const float2 *my,
                     const float2 *mx, const int *ident, const float2 *tw, int count, hipStream_t st)
{
    dim3 grid(count), block(Win<N>::NT);
    if (conj) window_filter_kernel<N, true><<<grid, block, 0, st>>>(in, in_stride, out, my, mx, ident, tw);
    else window_filter_kernel<N, false><<<grid, block, 0, st>>>(in, in_stride, out, my, mx, ident, tw);
}

void launch_filter(int n, bool conj, const float2 *in, long long in_stride, float2 *out, const float2 *my,
                   const float2 *mx, const int *ident, const float2 *tw, int count, hipStream_t st)
{
    switch (n) {
        case 16: launch_filter_n<16>(conj, in, in_stride, out, my, mx, ident, tw, count, st); break;
        case 32: launch_filter_n<32>(conj, in, in_stride, out, my, mx, ident, tw, count, st); break;
        case 64: launch_filter_n<64>(conj, in, in_stride, out, my, mx, ident, tw, count, st); break;
        case 128: launch_filter_n<128>(conj, in, in_stride, out, my, mx, ident, tw, count, st); break;
        default: break;
    }
}

template <int N>
void launch_line_filter(bool row, bool conj, const float2 *in, long long in_stride, float2 *out,
                        const float2 *table, const int *ident, const float2 *tw, int count, hipStream_t st)
{
    dim3 grid(N / kLinesPerGroup, count), block(kLinesPerGroup * Win<N>::R);
    if (row && conj) line_filter_kernel<N, true, true><<<grid, block, 0, st>>>(in, in_stride, out, table, ident, tw);
    else if (row) line_filter_kernel<N, true, false><<<grid, block, 0, st>>>(in, in_stride, out, table, ident, tw);
    else if (conj) line_filter_kernel<N, false, true><<<grid, block, 0, st>>>(in, in_stride, out, table, ident, tw);
    else line_filter_kernel<N, false, false><<<grid, block, 0, st>>>(in, in_stride, out, table, ident, tw);
}

void line_filter(int n, bool row, bool conj, const float2 *in, long long in_stride, float2 *out, const float2 *table,
                 const int *ident, const float2 *tw, int count, hipStream_t st)
{
    switch (n) {
        case 32: launch_line_filter<32>(row, conj, in, in_stride, out, table, ident, tw, count, st); break;
        case 64: launch_line_filter<64>(row, conj, in, in_stride, out, table, ident, tw, count, st); break;
        case 128: launch_line_filter<128>(row, conj, in, in_stride, out, table, ident, tw, count, st); break;
        default: launch_line_filter<256>(row, conj, in, in_stride, out, table, ident, tw, count, st); break;
    }
}

// Shifted probes P_c = F^{-1}(F P o ramp_c) for every shift class.
void class_probes(ms_plan *p, const ms_c64 *probe, hipStream_t st)
{
    const HostPlan &hp = p->hp;
    if (p->lines) {
        // x ramps on rows into class_tmp, then y ramps on columns into class_probe
        line_filter(hp.n, true, false, reinterpret_cast<const float2 *>(probe), 0, p->at<float2>(p->L.class_tmp),
                    p->at<float2>(p->L.rx), p->at<int>(p->L.ident), p->at<float2>(p->L.tw), hp.C, st);
        line_filter(hp.n, false, false, p->at<float2>(p->L.class_tmp), (long long)hp.n * hp.n,
                    p->at<float2>(p->L.class_probe), p->at<float2>(p->L.ry), p->at<int>(p->L.ident),
                    p->at<float2>(p->L.tw), hp.C, st);
        return;
    }
    launch_filter(hp.n, false, reinterpret_cast<const float2 *>(probe), 0, p->at<float2>(p->L.class_probe),
                  p->at<float2>(p->L.ry), p->at<float2>(p->L.rx), p->at<int>(p->L.ident), p->at<float2>(p->L.tw),
                  hp.C, st);
}

// Derivatives of the shifted probes in their shifts, dP_c/df_y then dP_c/df_x, into dprobe.
void class_probe_derivatives(ms_plan *p, const ms_c64 *probe, hipStream_t st)
{
    const HostPlan &hp = p->hp;
    const long long plane = (long long)hp.C * hp.n * hp.n;
    float2 *dy = p->at<float2>(p->L.dprobe), *dx = dy + plane;
    const float2 *in = reinterpret_cast<const float2 *>(probe);
    const int *none = p->at<int>(p->L.zero_ident);
    const float2 *tw = p->at<float2>(p->L.tw);
    if (p->lines) {
        float2 *tmp = p->at<float2>(p->L.class_tmp);
        line_filter(hp.n, true, false, in, 0, tmp, p->at<float2>(p->L.rx), none, tw, hp.C, st);
        line_filter(hp.n, false, false, tmp, (long long)hp.n * hp.n, dy, p->at<float2>(p->L.dry), none, tw, hp.C, st);
        line_filter(hp.n, true, false, in, 0, tmp, p->at<float2>(p->L.drx), none, tw, hp.C, st);
        line_filter(hp.n, false, false, tmp, (long long)hp.n * hp.n, dx, p->at<float2>(p->L.ry), none, tw, hp.C, st);
        return;
    }
    launch_filter(hp.n, false, in, 0, dy, p->at<float2>(p->L.dry), p->at<float2>(p->L.rx), none, tw, hp.C, st);
    launch_filter(hp.n, false, in, 0, dx, p->at<float2>(p->L.ry), p->at<float2>(p->L.drx), none, tw, hp.C, st);
}

// max |t_m|^2 of every slice into maxt2[M].
void slice_maxima(ms_plan *p, const ms_c64 *slices, hipStream_t st)
{
    const HostPlan &hp = p->hp;
    const long long hw = (long long)hp.H * hp.W;
    const int blocks = (int)std::min<long long>(kMaxBlocks, (hw + 255) / 256);
    max_partial_kernel<<<dim3(blocks, hp.M), 256, 0, st>>>(reinterpret_cast<const float2 *>(slices), nullptr, hw,
                                                           p->at<float>(p->L.partial));
    max_final_kernel<<<hp.M, 256, 0, st>>>(p->at<float>(p->L.partial), blocks, p->at<float>(p->L.maxt2));
}

FusedParams fused_params(ms_plan *p, const ms_c64 *slices, const float *measured)
{
    const HostPlan &hp = p->hp;
    FusedParams fp{};
    fp.class_probe = p->at<float2>(p->L.class_probe);
    fp.slices = reinterpret_cast<const float2 *>(slices);
    fp.pos_info = p->at<int4>(p->L.pos_info);
    fp.tw = p->at<float2>(p->L.tw);
    fp.hy = p->at<float2>(p->L.hy);
    fp.hx = p->at<float2>(p->L.hx);
    fp.gap_table = p->at<int>(p->L.gap_table);
    fp.n_tables = (int)hp.dz_unique.size();
    fp.measured = measured;
    fp.waves = p->at<float2>(p->L.waves);
    fp.probe_patch = p->at<float2>(p->L.probe_patch);
    fp.overlap_patch = p->at<float>(p->L.overlap);
    fp.loss_pos = p->at<double>(p->L.loss_pos);
    fp.H = hp.H; fp.W = hp.W; fp.M = hp.M; fp.layer = 0;
    fp.objective = p->objective;
    fp.full = 0;
    fp.wave_stride = p->wave_stride();
    fp.ovl_stride = p->ovl_stride();
    fp.ck = hp.K;
    fp.seg = hp.M - 1;
    fp.park = p->at<float2>(p->L.half);
    return fp;
}

// N^2 of the step-size denominator; doubled (half step) for the Poisson objective.
double step_norm(const ms_plan *p)
{
    const double nn = (double)p->hp.n * p->hp.n;
    return p->objective == MS_OBJECTIVE_POISSON ? 2.0 * nn : nn;
}

int grid_for(long long count) { return (int)std::max<long long>(1, std::min<long long>(8192, (count + 255) / 256)); }

// Pass 1 over nch chunks of images and pass 2 (chunk partials in order) for n_m slices.
void scatter_launch(ms_plan *p, ScatterParams &sp, int nch, int n_m, float2 *out, float *wout, int accumulate,
                    hipStream_t st, bool wide)
{
    const HostPlan &hp = p->hp;
    const Tiling tg = wide ? wide_tiles(hp) : square_tiles(hp);
    sp.partial = p->at<float2>(p->L.spart);
    sp.wpartial = wout ? p->at<float>(p->L.wpart) : nullptr;
    sp.H = hp.H; sp.W = hp.W; sp.N = hp.n; sp.tiles_x = tg.tiles_x; sp.n_tiles = tg.n_tiles;
    // Consecutive chunks are summed in one block (in ascending order, as one longer chunk) while
    // the grid keeps about kScatterBlocks blocks: fewer partial planes to write and reduce when
    // many slices are scattered at once.
    const long long per_group = (long long)tg.n_tiles * n_m;
    const int groups = (int)std::min<long long>(nch, std::max<long long>(1, (kScatterBlocks + per_group - 1) / per_group));
    sp.nch = nch;
    sp.cpb = (nch + groups - 1) / groups;
    const int ngrp = (nch + sp.cpb - 1) / sp.cpb;
    if (wide) scatter_partial_kernel<kWideW, kWideH><<<dim3(tg.n_tiles, ngrp, n_m), 256, 0, st>>>(sp);
    else scatter_partial_kernel<kTileW, kTileH><<<dim3(tg.n_tiles, ngrp, n_m), 256, 0, st>>>(sp);
    const long long plane = (long long)n_m * hp.H * hp.W;
    chunk_reduce_kernel<float2><<<grid_for(plane), 256, 0, st>>>(sp.partial, ngrp, plane, out, accumulate);
    if (wout) {
        const long long hw = (long long)hp.H * hp.W;
        chunk_reduce_kernel<float><<<grid_for(n_m * hw), 256, 0, st>>>(sp.wpartial, ngrp, n_m * hw, wout,
                                                                        accumulate);
    }
}

// Gradient patches of batch b for slices m0 .. m0 + n_m - 1 into out (n_m x H x W), and the
// overlap patches into wout if given; accumulate adds to what out already holds.  patches:
// slice i of position a at patches + a * pos_stride + i * N^2 (wpatch likewise with w_stride).
void scatter(ms_plan *p, int b, int count, const float2 *patches, long long pos_stride, const float *wpatch,
             long long w_stride, int m0, int n_m, float2 *out, float *wout, int accumulate, hipStream_t st)
{
    const HostPlan &hp = p->hp;
    ScatterParams sp{};
    sp.m0 = m0;
    sp.trans1 = p->lines ? 1 : 0;    // the line path stores odd slices' patches transposed
    sp.patches0 = sp.patches1 = patches;
    sp.wpatch = wpatch;
    sp.pos_stride0 = sp.pos_stride1 = pos_stride;
    sp.slice_stride0 = sp.slice_stride1 = (long long)hp.n * hp.n;
    const bool wide = p->wide_scatter();
    sp.tile_off0 = sp.tile_off1 = p->at<int>(p->L.tile_off) + p->tile_off_at(b, wide);
    sp.entries0 = sp.entries1 = p->at<int4>(p->L.tile_list);
    sp.ld0 = sp.ld1 = hp.n;
    sp.w_stride = w_stride;
    scatter_launch(p, sp, chunking(count).nch, n_m, out, wout, accumulate, st, wide);
}

// Gradient images of batch b for slices m0 .. m0 + n_m - 1 into out (n_m x H x W): for each
// parity the band images (slice i's at the band buffer + i * band slice stride) when its launches
// sum bands, else the per-position patches (slice i of position a at patches + a * pos_stride +
// i * N^2).
void scatter_slices(ms_plan *p, int b, int count, const float2 *patches, long long pos_stride, int m0, int n_m,
                    float2 *out, int accumulate, hipStream_t st)
{
    const HostPlan &hp = p->hp;
    ScatterParams sp{};
    const size_t toff = (size_t)b * kChunks * (hp.n_tiles + 1);
    const bool wide = p->wide_scatter();     // no bands then: patches in the natural layout
    int nch = chunking(count).nch;
    for (int o = 0; o < 2; ++o) {
        // list o serves the slices m0 + i of parity o
        const float2 *img = patches;
        long long ps = pos_stride, ss = (long long)hp.n * hp.n;
        const int *off = p->at<int>(p->L.tile_off) + p->tile_off_at(b, wide);
        const int4 *ent = p->at<int4>(p->L.tile_list);
        // the line path stores odd slices' images transposed
        const int trans = (p->lines && o == 1) ? 1 : 0;
        int vert = 0;
        if (p->bands_active(o)) {
            img = p->at<float2>(p->L.band);
            ps = p->band_stride();
            ss = p->band_slice_stride();
            off = p->at<int>(p->L.btile_off[o]) + toff;
            ent = p->at<int4>(p->L.btile_list[o]);
            vert = o == 0 ? 1 : 0;    // the spread runs along y (even slices) or x (odd slices)
            nch = std::max(nch, hp.band_nch[b]);
        }
        if (o == 0) {
            sp.patches0 = img; sp.pos_stride0 = ps; sp.slice_stride0 = ss;
            sp.tile_off0 = off; sp.entries0 = ent; sp.ld0 = hp.n; sp.vert0 = vert; sp.trans0 = trans;
        } else {
            sp.patches1 = img; sp.pos_stride1 = ps; sp.slice_stride1 = ss;
            sp.tile_off1 = off; sp.entries1 = ent; sp.ld1 = hp.n; sp.vert1 = vert; sp.trans1 = trans;
        }
    }
    sp.m0 = m0;
    scatter_launch(p, sp, nch, n_m, out, nullptr, accumulate, st, wide);
}

// Probe patches of one batch summed per shift class into class_acc (accumulate adds).
void class_sums(ms_plan *p, const int *class_off, const int *class_list, int count, int accumulate,
                hipStream_t st)
{
    const HostPlan &hp = p->hp;
    const int nn = hp.n * hp.n;
    const Chunking ch = chunking(count);
    class_partial_kernel<<<dim3((nn + 255) / 256, hp.C, ch.nch), 256, 0, st>>>(
        p->at<float2>(p->L.probe_patch), class_off, class_list, p->at<float2>(p->L.cpart), hp.C, nn);
    const long long plane = (long long)hp.C * nn;
    chunk_reduce_kernel<float2><<<grid_for(plane), 256, 0, st>>>(p->at<float2>(p->L.cpart), ch.nch, plane,
                                                                 p->at<float2>(p->L.class_acc), accumulate);
}

// Probe gradient from the per-class sums: sum_c S_c^H acc_c.
void probe_gradient(ms_plan *p, float2 *out, hipStream_t st)
{
    const HostPlan &hp = p->hp;
    const int nn = hp.n * hp.n;
    if (p->lines) {
        line_filter(hp.n, true, true, p->at<float2>(p->L.class_acc), nn, p->at<float2>(p->L.class_tmp),
                    p->at<float2>(p->L.rx), p->at<int>(p->L.ident), p->at<float2>(p->L.tw), hp.C, st);
        line_filter(hp.n, false, true, p->at<float2>(p->L.class_tmp), nn, p->at<float2>(p->L.class_acc),
                    p->at<float2>(p->L.ry), p->at<int>(p->L.ident), p->at<float2>(p->L.tw), hp.C, st);
        sum_classes_kernel<<<(nn + 255) / 256, 256, 0, st>>>(p->at<float2>(p->L.class_acc), hp.C, nn, out);
        return;
    }
    launch_filter(hp.n, true, p->at<float2>(p->L.class_acc), nn, p->at<float2>(p->L.class_tmp),
                  p->at<float2>(p->L.ry), p->at<float2>(p->L.rx), p->at<int>(p->L.ident), p->at<float2>(p->L.tw),
                  hp.C, st);
    sum_classes_kernel<<<(nn + 255) / 256, 256, 0, st>>>(p->at<float2>(p->L.class_tmp), hp.C, nn, out);
}

bool aligned8(const void *ptr) { return ((uintptr_t)ptr & 7) == 0; }

}  // namespace

extern "C" {

const char *ms_last_error(void) { return g_err.c_str(); }

ms_status ms_reconstruction_error(hipStream_t st, const ms_c64 *est, const ms_c64 *ref, const float *mask,
                                  int32_t n_slices, int32_t obj_h, int32_t obj_w, int32_t max_shift, double *work,
                                  double *err_out, int32_t *shift_out)
{
    g_err.clear();
    if (!est || !ref || !err_out || !work) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    if (n_slices < 1 || n_slices > 4096 || obj_h < 1 || obj_w < 1 || (int64_t)obj_h * obj_w > ((int64_t)1 << 30))
        return fail(MS_ERR_INVALID_ARG, "n_slices must be in [1, 4096] and obj_h obj_w in [1, 2^30]");
    if (max_shift < 0 || max_shift > 64 || max_shift >= obj_h || max_shift >= obj_w)
        return fail(MS_ERR_INVALID_ARG, "max_shift must be in [0, 64] and below the object's sides");
    if (!aligned8(est) || !aligned8(ref) || !aligned8(err_out) || !aligned8(work) || ((uintptr_t)mask & 3) ||
        ((uintptr_t)shift_out & 3))
        return fail(MS_ERR_INVALID_ARG, "misaligned buffer");
    const int side = 2 * max_shift + 1, n_shifts = side * side;
    recon_shift_kernel<<<dim3(n_shifts, n_slices), 256, 0, st>>>(reinterpret_cast<const float2 *>(est),
                                                                  reinterpret_cast<const float2 *>(ref), mask, obj_h,
                                                                  obj_w, max_shift, n_slices, work);
    recon_select_kernel<<<1, 1, 0, st>>>(work, n_shifts, n_slices, max_shift, err_out, shift_out);
    return check_hip("ms_reconstruction_error");
}

ms_status ms_workspace_size(const ms_problem *pb, size_t budget_bytes, size_t *ws_bytes)
{
    try {
        g_err.clear();
        ms_status st = validate(pb);
        if (st != MS_OK) return st;
        if (!ws_bytes) return fail(MS_ERR_INVALID_ARG, "ws_bytes is NULL");
        HostPlan hp;
        derive_positions(pb, hp);
        if (too_many_classes(hp))
            return fail(MS_ERR_UNSUPPORTED, "more than " + std::to_string(kMaxClasses) + " distinct sub-pixel offsets");
        if ((int)hp.dz_unique.size() > table_capacity(hp.n))
            return fail(MS_ERR_UNSUPPORTED, "more than " + std::to_string(table_capacity(hp.n)) + " distinct slice distances");
        size_t ne = tile_entries(hp);
        int64_t B = choose_storage(hp, ne, budget_bytes, pb->checkpoint_every);
        if (B < 1) return fail(MS_ERR_BUDGET, "budget too small for a single position");
        *ws_bytes = make_layout(hp, B, ne).total;
        return MS_OK;
    } catch (const std::bad_alloc &) {
        return fail(MS_ERR_INVALID_ARG, "host out of memory");
    } catch (...) {
        return fail(MS_ERR_INVALID_ARG, "unexpected host error");
    }
}

}  // extern "C"

namespace {

// A plan's host description and tables for problem pb in the workspace ws of ws_bytes: derives
// positions, shift classes, wave storage and batch (the workspace is the budget), builds the
// scatter lists and uploads every table (blocking copies).  Creates no stream or event.
ms_status build_plan(ms_plan *p, const ms_problem *pb, char *ws, size_t ws_bytes, const char *ws_name)
{
    HostPlan &hp = p->hp;
    derive_positions(pb, hp);
    if (too_many_classes(hp))
        return fail(MS_ERR_UNSUPPORTED, "more than " + std::to_string(kMaxClasses) + " distinct sub-pixel offsets");
    if ((int)hp.dz_unique.size() > table_capacity(hp.n))
        return fail(MS_ERR_UNSUPPORTED, "more than " + std::to_string(table_capacity(hp.n)) + " distinct slice distances");
    size_t ne = tile_entries(hp);
    int64_t B = choose_storage(hp, ne, ws_bytes, pb->checkpoint_every);
    if (B < 1) {
        HostPlan one = hp;
        one.K = std::max(hp.M, 1);
        return fail(MS_ERR_BUDGET, std::string(ws_name) + " of " + std::to_string(ws_bytes) +
                                       " bytes is too small for a single position (it needs " +
                                       std::to_string(make_layout(one, 1, ne).total) + ")");
    }
    build_lists(hp, B);
    {
        const BandStats bs = band_stats(hp, B);
        hp.bands[0] = bs.on[0];
        hp.bands[1] = bs.on[1];
        hp.band_rows = bs.rows;
        hp.band_count = bs.count_max;
        if (bs.on[0] || bs.on[1]) build_band_lists(hp);
    }
    p->L = make_layout(hp, B, ne);
    if (p->L.total > ws_bytes) return fail(MS_ERR_BUDGET, std::string(ws_name) + " too small");
    p->ws = ws;
    p->lines = !fused_fits(hp.n);
    p->ws_bytes = ws_bytes;
    p->dx = pb->pixel_size; p->lambda = pb->wavelength; p->tilt_y = pb->tilt_y; p->tilt_x = pb->tilt_x;
    // Tables, computed in FP64 and rounded once.
    const int n = hp.n, C = hp.C;
    const double PI = 3.14159265358979323846264338327950288;
    // twiddles W_N^{j k1} of lane j, rows of 17 (see Win::TW_WORDS)
    const int R = n / 16;
    std::vector<float2> tw((size_t)R * 17, make_float2(1.f, 0.f));
    for (int j = 0; j < R; ++j)
        for (int k1 = 0; k1 < 16; ++k1) {
            double a = -2.0 * PI * (double)(j * k1) / n;
            tw[(size_t)j * 17 + k1] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
    auto freq = [&](int i) { return (double)(i < (n + 1) / 2 ? i : i - n); };
    const int U = (int)hp.dz_unique.size();
    std::vector<float2> hy((size_t)U * n), hx((size_t)U * n);
    for (int g = 0; g < U; ++g) {
        double dz = hp.dz_unique[g];
        for (int i = 0; i < n; ++i) {
            double q = freq(i) / ((double)n * pb->pixel_size);
            // eq. (fresnel_element) split per axis: exp(-pi i dz (lambda q^2 + 2 q sin(theta)))
            double py = -PI * dz * (pb->wavelength * q * q + 2.0 * q * std::sin(pb->tilt_y));
            double px = -PI * dz * (pb->wavelength * q * q + 2.0 * q * std::sin(pb->tilt_x));
            hy[(size_t)g * n + i] = make_float2((float)(std::cos(py) / n), (float)(std::sin(py) / n));
            hx[(size_t)g * n + i] = make_float2((float)(std::cos(px) / n), (float)(std::sin(px) / n));
        }
    }
    std::vector<float2> ry((size_t)C * n), rx((size_t)C * n), dry((size_t)C * n), drx((size_t)C * n);
    std::vector<int> ident(C), zero_ident(C, 0);
    for (int c = 0; c < C; ++c) {
        ident[c] = (hp.cls_fy[c] == 0.0 && hp.cls_fx[c] == 0.0) ? 1 : 0;
        for (int i = 0; i < n; ++i) {
            double ay = -2.0 * PI * freq(i) * hp.cls_fy[c] / n;
            double ax = -2.0 * PI * freq(i) * hp.cls_fx[c] / n;
            ry[(size_t)c * n + i] = make_float2((float)(std::cos(ay) / n), (float)(std::sin(ay) / n));
            rx[(size_t)c * n + i] = make_float2((float)(std::cos(ax) / n), (float)(std::sin(ax) / n));
            // the ramp differentiated in its shift: times -2 pi i k / N
            const double th = 2.0 * PI * freq(i) / n;
            dry[(size_t)c * n + i] = make_float2((float)(th * std::sin(ay) / n), (float)(-th * std::cos(ay) / n));
            drx[(size_t)c * n + i] = make_float2((float)(th * std::sin(ax) / n), (float)(-th * std::cos(ax) / n));
        }
    }
    std::vector<int> pos_list(hp.S);
    for (int64_t s = 0; s < hp.S; ++s) pos_list[s] = (int)s;

    auto up = [&](size_t off, const void *src, size_t bytes) -> bool {
        if (bytes == 0) return true;
        return hipMemcpy(p->ws + off, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = up(p->L.tw, tw.data(), tw.size() * 8) && up(p->L.hy, hy.data(), hy.size() * 8) &&
              up(p->L.hx, hx.data(), hx.size() * 8) && up(p->L.ry, ry.data(), ry.size() * 8) &&
              up(p->L.gap_table, hp.gap_table.data(), hp.gap_table.size() * 4) &&
              up(p->L.rx, rx.data(), rx.size() * 8) && up(p->L.ident, ident.data(), ident.size() * 4) &&
              up(p->L.dry, dry.data(), dry.size() * 8) && up(p->L.drx, drx.data(), drx.size() * 8) &&
              up(p->L.zero_ident, zero_ident.data(), zero_ident.size() * 4) &&
              up(p->L.pos_info, hp.pos_info.data(), hp.pos_info.size() * 16) &&
              up(p->L.pos_list, pos_list.data(), pos_list.size() * 4) &&
              up(p->L.tile_off, hp.tile_off.data(), hp.tile_off.size() * 4) &&
              up(p->L.tile_list, hp.tile_list.data(), hp.tile_list.size() * 16) &&
              up(p->L.class_off, hp.class_off.data(), hp.class_off.size() * 4) &&
              up(p->L.class_list, hp.class_list.data(), hp.class_list.size() * 4);
    for (int d = 0; ok && d < 2; ++d)
        ok = !hp.bands[d] || (up(p->L.wg[d], hp.wg[d].data(), hp.wg[d].size() * 16) &&
             up(p->L.bmem[d], hp.bmem[d].data(), hp.bmem[d].size() * 4) &&
             up(p->L.bdelta[d], hp.bdelta[d].data(), hp.bdelta[d].size() * 4) &&
             up(p->L.btile_off[d], hp.btile_off[d].data(), hp.btile_off[d].size() * 4) &&
             up(p->L.btile_list[d], hp.btile_list[d].data(), hp.btile_list[d].size() * 16));
    if (!ok) {
        hipError_t e = hipGetLastError();
        return fail(MS_ERR_HIP, std::string("table upload failed: ") + hipGetErrorString(e));
    }
    // the per-position tile vectors are no longer needed on the host
    hp.tile_list.clear();
    hp.tile_list.shrink_to_fit();
    for (int d = 0; d < 2; ++d) {
        std::vector<int4>().swap(hp.wg[d]);
        std::vector<int>().swap(hp.bmem[d]);
        std::vector<int>().swap(hp.bdelta[d]);
        std::vector<int>().swap(hp.btile_off[d]);
        std::vector<int4>().swap(hp.btile_list[d]);
    }
    return MS_OK;
}

}  // namespace

extern "C" {

ms_status ms_plan_create(const ms_problem *pb, void *workspace, size_t ws_bytes, ms_plan **out)
{
    try {
        g_err.clear();
        ms_status st = validate(pb);
        if (st != MS_OK) return st;
        if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
        if (!workspace) return fail(MS_ERR_INVALID_ARG, "workspace is NULL");
        if ((uintptr_t)workspace % kAlign) return fail(MS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        ms_plan *p = new ms_plan();
        st = build_plan(p, pb, static_cast<char *>(workspace), ws_bytes, "workspace");
        if (st != MS_OK) {
            delete p;
            return st;
        }
        if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess) {
            hipError_t e = hipGetLastError();
            ms_plan_destroy(p);
            return fail(MS_ERR_HIP, std::string("stream or event creation failed: ") + hipGetErrorString(e));
        }
        *out = p;
        return MS_OK;
    } catch (const std::bad_alloc &) {
        return fail(MS_ERR_INVALID_ARG, "host out of memory");
    } catch (...) {
        return fail(MS_ERR_INVALID_ARG, "unexpected host error");
    }
}

void ms_plan_destroy(ms_plan *plan)
{
    if (!plan) return;
    for (hipEvent_t e : plan->ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : plan->ev_stop) (void)hipEventDestroy(e);
    if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
    if (plan->ev_join) (void)hipEventDestroy(plan->ev_join);
    if (plan->side) (void)hipStreamDestroy(plan->side);
    delete plan;
}

ms_status ms_profile_begin(ms_plan *p, int32_t max_launches)
{
    g_err.clear();
    if (!p || max_launches < 1 || max_launches > 100000) return fail(MS_ERR_INVALID_ARG, "bad profiling request");
    for (hipEvent_t e : p->ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->ev_stop) (void)hipEventDestroy(e);
    p->ev_start.clear();
    p->ev_stop.clear();
    p->ev_used = 0;
    for (int i = 0; i < max_launches; ++i) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return check_hip("hipEventCreate");
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return check_hip("hipEventCreate");
        }
        p->ev_start.push_back(a);
        p->ev_stop.push_back(b);
    }
    return MS_OK;
}

ms_status ms_profile_end(ms_plan *p, double *total_ms, int64_t *launches)
{
    g_err.clear();
    if (!p || !total_ms || !launches) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    double tot = 0.0;
    ms_status st = MS_OK;
    if (p->ev_used > 0 && hipEventSynchronize(p->ev_stop[p->ev_used - 1]) != hipSuccess)
        st = check_hip("hipEventSynchronize");
    for (size_t i = 0; i < p->ev_used && st == MS_OK; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev_start[i], p->ev_stop[i]) != hipSuccess) st = check_hip("hipEventElapsedTime");
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)p->ev_used;
    for (hipEvent_t e : p->ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->ev_stop) (void)hipEventDestroy(e);
    p->ev_start.clear();
    p->ev_stop.clear();
    p->ev_used = 0;
    return st;
}

int64_t ms_plan_batch(const ms_plan *plan) { return plan ? plan->hp.B : 0; }

int32_t ms_plan_shift_classes(const ms_plan *plan) { return plan ? plan->hp.C : 0; }

int32_t ms_plan_checkpoint_every(const ms_plan *plan) { return plan ? plan->hp.K : 0; }

ms_status ms_plan_set_objective(ms_plan *p, int32_t objective)
{
    g_err.clear();
    if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
    p->carry_layer = -1;    // the carried wave no longer holds
    if (objective != MS_OBJECTIVE_AMPLITUDE && objective != MS_OBJECTIVE_POISSON)
        return fail(MS_ERR_INVALID_ARG, "unknown objective");
    p->objective = objective;
    return MS_OK;
}

ms_status ms_plan_set_path(ms_plan *p, int32_t path)
{
    g_err.clear();
    if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
    p->carry_layer = -1;    // the carried wave no longer holds
    const int n = p->hp.n;
    switch (path) {
        case MS_PATH_AUTO:
            p->lines = !fused_fits(n);
            return MS_OK;
        case MS_PATH_FUSED:
            if (!fused_fits(n)) return fail(MS_ERR_UNSUPPORTED, "the fused kernel holds windows up to 128 x 128");
            p->lines = false;
            return MS_OK;
        case MS_PATH_LINES:
            if (n < 32) return fail(MS_ERR_UNSUPPORTED, "the line kernels need n >= 32");
            p->lines = true;
            return MS_OK;
        default:
            return fail(MS_ERR_INVALID_ARG, "unknown path");
    }
}

ms_status ms_plan_set_bands(ms_plan *p, int32_t mode)
{
    g_err.clear();
    if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
    p->carry_layer = -1;    // the carried wave no longer holds
    if (mode != MS_BANDS_NONE && mode != MS_BANDS_ROWS && mode != MS_BANDS_ALL)
        return fail(MS_ERR_INVALID_ARG, "unknown band mode");
    p->band_mode = mode;
    return MS_OK;
}

int32_t ms_plan_has_bands(const ms_plan *p) { return p ? (p->hp.bands[0] ? 1 : 0) | (p->hp.bands[1] ? 2 : 0) : 0; }

ms_status ms_plan_set_kept_windows(ms_plan *p, int32_t on)
{
    g_err.clear();
    if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
    p->carry_layer = -1;    // the carried wave no longer holds
    p->keep_windows = on != 0;
    return MS_OK;
}

int32_t ms_plan_kept_windows(const ms_plan *p) { return p && p->kept_windows() ? 1 : 0; }

ms_status ms_plan_set_layer_carry(ms_plan *p, int32_t on)
{
    g_err.clear();
    if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
    p->layer_carry = on != 0;
    p->carry_layer = -1;
    return MS_OK;
}

namespace {

ms_status make_probe(ms_plan *p, hipStream_t st, double alpha, const Aberrations &ab, ms_c64 *probe_out)
{
    float2 *out = reinterpret_cast<float2 *>(probe_out);
    const float2 *tw = p->at<float2>(p->L.tw);
    if (p->hp.n == 256) {
        // rows: aperture and inverse DFT along x; columns: inverse DFT along y; unit energy
        constexpr int N = 256, G = N / kLinesPerGroup;
        double *part = p->at<double>(p->L.energy);
        dim3 grid(G, 1), block(kLinesPerGroup * Win<N>::R);
        line_probe_kernel<N, true><<<grid, block, 0, st>>>(out, part, tw, p->dx, p->lambda, alpha, ab);
        line_probe_kernel<N, false><<<grid, block, 0, st>>>(out, part, tw, p->dx, p->lambda, alpha, ab);
        scale_unit_energy_kernel<<<64, 256, 0, st>>>(out, (long long)N * N, part, G);
        return check_hip("ms_make_probe");
    }
    switch (p->hp.n) {
        case 16: make_probe_kernel<16><<<1, Win<16>::NT, 0, st>>>(out, tw, p->dx, p->lambda, alpha, ab); break;
        case 32: make_probe_kernel<32><<<1, Win<32>::NT, 0, st>>>(out, tw, p->dx, p->lambda, alpha, ab); break;
        case 64: make_probe_kernel<64><<<1, Win<64>::NT, 0, st>>>(out, tw, p->dx, p->lambda, alpha, ab); break;
        default: make_probe_kernel<128><<<1, Win<128>::NT, 0, st>>>(out, tw, p->dx, p->lambda, alpha, ab); break;
    }
    return check_hip("ms_make_probe");
}

}  // namespace

ms_status ms_make_probe(ms_plan *p, hipStream_t st, double alpha, double defocus, ms_c64 *probe_out)
{
    g_err.clear();
    if (!p || !probe_out) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    p->carry_layer = -1;    // the carried wave no longer holds
    if (!aligned8(probe_out)) return fail(MS_ERR_INVALID_ARG, "probe_out must be 8-byte aligned");
    if (!(alpha > 0.0) || !std::isfinite(alpha) || !std::isfinite(defocus))
        return fail(MS_ERR_INVALID_ARG, "alpha must be positive, both finite");
    return make_probe(p, st, alpha, Aberrations{defocus, 0.0, 1.0, 0.0, 0.0}, probe_out);
}

ms_status ms_make_probe_aberrated(ms_plan *p, hipStream_t st, double alpha, const double *aberrations,
                                  ms_c64 *probe_out)
{
    g_err.clear();
    if (!p || !probe_out || !aberrations) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    p->carry_layer = -1;    // the carried wave no longer holds
    if (!aligned8(probe_out)) return fail(MS_ERR_INVALID_ARG, "probe_out must be 8-byte aligned");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(aberrations[i])) return fail(MS_ERR_INVALID_ARG, "aberrations must be finite");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(MS_ERR_INVALID_ARG, "alpha must be positive and finite");
    const Aberrations ab{aberrations[0], aberrations[1], std::cos(2.0 * aberrations[2]), std::sin(2.0 * aberrations[2]),
                         aberrations[3]};
    return make_probe(p, st, alpha, ab, probe_out);
}

ms_status ms_forward(ms_plan *p, hipStream_t st, const ms_c64 *probe, const ms_c64 *slices, float *intensity_out,
                     ms_c64 *exit_out)
{
    g_err.clear();
    if (!p || !probe || !slices || !intensity_out) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    p->carry_layer = -1;    // the carried wave no longer holds
    if (!aligned8(probe) || !aligned8(slices) || !aligned8(exit_out) || ((uintptr_t)intensity_out & 3))
        return fail(MS_ERR_INVALID_ARG, "misaligned buffer");
    const HostPlan &hp = p->hp;
    class_probes(p, probe, st);
    FusedParams fp = fused_params(p, slices, nullptr);
    fp.intensity = intensity_out;
    fp.exit_waves = reinterpret_cast<float2 *>(exit_out);
    fp.waves = nullptr;
    for (int b = 0; b < hp.nb; ++b) {
        int64_t s0 = (int64_t)b * hp.B;
        int count = (int)std::min<int64_t>(hp.B, hp.S - s0);
        fp.pos_list = p->at<int>(p->L.pos_list) + s0;
        launch_fused(p, kForward, fp, count, st);
    }
    return check_hip("ms_forward");
}

}  // extern "C"

// The workspace of ms_adjoint_scratch: every call on a device shares that device's copy, which
// keeps the last call's contents (nothing in it needs to start at zero).
static __device__ __align__(256) unsigned char scratch[MS_SCRATCH_BYTES];

namespace {

bool adjoint_args_ok(const ms_c64 *probe, const ms_c64 *slices, const float *measured, const ms_c64 *grad_slices,
                     const ms_c64 *grad_probe, const double *loss_out, ms_status *st)
{
    if (!probe || !slices || !measured || !grad_slices || !loss_out) {
        *st = fail(MS_ERR_INVALID_ARG, "NULL argument");
        return false;
    }
    if (!aligned8(probe) || !aligned8(slices) || !aligned8(grad_slices) || !aligned8(grad_probe) ||
        !aligned8(loss_out) || ((uintptr_t)measured & 3)) {
        *st = fail(MS_ERR_INVALID_ARG, "misaligned buffer");
        return false;
    }
    return true;
}

// The loss-and-gradient pass of a plan.  With a side stream (a plan from ms_plan_create) the loss
// and probe-gradient reductions run beside the slice scatter; without one, after it on st.
ms_status adjoint_impl(ms_plan *p, hipStream_t st, const ms_c64 *probe, const ms_c64 *slices, const float *measured,
                       ms_c64 *grad_slices, ms_c64 *grad_probe, double *loss_out)
{
    const HostPlan &hp = p->hp;
    class_probes(p, probe, st);
    FusedParams fp = fused_params(p, slices, measured);
    if (!grad_probe) fp.probe_patch = nullptr;
    const bool fork = p->side != nullptr;
    hipStream_t aux = fork ? p->side : st;
    for (int b = 0; b < hp.nb; ++b) {
        int64_t s0 = (int64_t)b * hp.B;
        int count = (int)std::min<int64_t>(hp.B, hp.S - s0);
        fp.pos_list = p->at<int>(p->L.pos_list) + s0;
        if (p->recompute())
            adjoint_recompute(p, fp, b, count, st, reinterpret_cast<float2 *>(grad_slices), nullptr, b > 0);
        else
            launch_fused(p, kAdjoint, fp, count, st, b);
        // the loss and the probe-gradient reductions read only the per-position outputs: they
        // run on the side stream while the slice scatter runs here; the next batch (which
        // overwrites those outputs) and the return wait for them
        if (fork && (hipEventRecord(p->ev_fork, st) != hipSuccess || hipStreamWaitEvent(aux, p->ev_fork, 0) != hipSuccess))
            return check_hip("ms_adjoint fork");
        {
            int n_loss;
            const double *lsrc = loss_entries(p, count, &n_loss);
            loss_sum_kernel<<<1, 256, 0, aux>>>(lsrc, n_loss, loss_out, b > 0);
        }
        if (grad_probe) {
            class_sums(p, p->at<int>(p->L.class_off) + (size_t)b * kChunks * (hp.C + 1), p->at<int>(p->L.class_list),
                       count, b > 0, aux);
            if (b + 1 == hp.nb) probe_gradient(p, reinterpret_cast<float2 *>(grad_probe), aux);
        }
        if (fork && hipEventRecord(p->ev_join, aux) != hipSuccess) return check_hip("ms_adjoint join");
        if (!p->recompute())
            scatter_slices(p, b, count, fp.waves, fp.wave_stride, 0, hp.M, reinterpret_cast<float2 *>(grad_slices),
                           b > 0, st);
        if (fork && hipStreamWaitEvent(st, p->ev_join, 0) != hipSuccess) return check_hip("ms_adjoint join");
    }
    return check_hip("ms_adjoint");
}

// Device address of the static scratch per device (looked up once per device, with that device
// current): host code passes these, never the array's name, which is a host-side stand-in.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

ms_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return check_hip("hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MS_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MS_OK;
}

}  // namespace

extern "C" {

ms_status ms_adjoint(ms_plan *p, hipStream_t st, const ms_c64 *probe, const ms_c64 *slices, const float *measured,
                     ms_c64 *grad_slices, ms_c64 *grad_probe, double *loss_out)
{
    g_err.clear();
    if (!p) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    p->carry_layer = -1;    // the carried wave no longer holds
    ms_status bad;
    if (!adjoint_args_ok(probe, slices, measured, grad_slices, grad_probe, loss_out, &bad)) return bad;
    return adjoint_impl(p, st, probe, slices, measured, grad_slices, grad_probe, loss_out);
}

ms_status ms_adjoint_scratch(const ms_problem *pb, hipStream_t st, const ms_c64 *probe, const ms_c64 *slices,
                             const float *measured, ms_c64 *grad_slices, ms_c64 *grad_probe, double *loss_out)
{
    try {
        g_err.clear();
        ms_status status = validate(pb);
        if (status != MS_OK) return status;
        if (!adjoint_args_ok(probe, slices, measured, grad_slices, grad_probe, loss_out, &status)) return status;
        void *ws = nullptr;
        status = scratch_address(&ws);
        if (status != MS_OK) return status;
        // work enqueued earlier on st may still read the scratch: let it finish before the tables
        // of this problem overwrite it
        if (hipStreamSynchronize(st) != hipSuccess) return check_hip("ms_adjoint_scratch: hipStreamSynchronize");
        ms_plan plan;   // host description only: no stream, no event, no device memory of its own
        status = build_plan(&plan, pb, static_cast<char *>(ws), MS_SCRATCH_BYTES, "the static scratch");
        if (status != MS_OK) return status;
        return adjoint_impl(&plan, st, probe, slices, measured, grad_slices, grad_probe, loss_out);
    } catch (const std::bad_alloc &) {
        return fail(MS_ERR_INVALID_ARG, "host out of memory");
    } catch (...) {
        return fail(MS_ERR_INVALID_ARG, "unexpected host error");
    }
}

ms_status ms_layer_step(ms_plan *p, hipStream_t st, int32_t layer, int32_t k_steps, const ms_c64 *probe,
                        ms_c64 *slices, const float *measured, double *loss_out, double *mu_out)
{
    g_err.clear();
    if (!p || !probe || !slices || !measured) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    const HostPlan &hp = p->hp;
    if (layer < 0 || layer >= hp.M) return fail(MS_ERR_INVALID_ARG, "layer out of range");
    if (k_steps < 0) return fail(MS_ERR_INVALID_ARG, "k_steps must be >= 0");
    if (!aligned8(probe) || !aligned8(slices) || !aligned8(loss_out) || !aligned8(mu_out) || ((uintptr_t)measured & 3))
        return fail(MS_ERR_INVALID_ARG, "misaligned buffer");
    if (k_steps == 0) return MS_OK;
    const long long hw = (long long)hp.H * hp.W;
    class_probes(p, probe, st);
    slice_maxima(p, slices, st);
    FusedParams fp = fused_params(p, slices, measured);
    fp.layer = layer;
    fp.probe_patch = nullptr;
    // the incident wave carried from the previous layer step: kept in slot 1 (one batch, two slots)
    // and usable when that step took this layer or the one before with the same buffers
    const bool carry = p->layer_carry && p->lines && hp.nb == 1 && wave_slots(hp.M, hp.K) >= 2;
    if (!carry || p->carry_key[0] != probe || p->carry_key[1] != slices || p->carry_key[2] != measured)
        p->carry_layer = -1;
    fp.carry = carry ? 1 : 0;
    const float2 *carried = fp.waves + (long long)hp.n * hp.n;
    double *mu = p->at<double>(p->L.scal);
    double *total = mu + 1;
    float2 *g = p->at<float2>(p->L.layer_g);
    float *w = p->at<float>(p->L.layer_w);
    const int wblocks = (int)std::min<long long>(kMaxBlocks, (hw + 255) / 256);
    for (int k = 0; k < k_steps; ++k) {
        for (int b = 0; b < hp.nb; ++b) {
            int64_t s0 = (int64_t)b * hp.B;
            int count = (int)std::min<int64_t>(hp.B, hp.S - s0);
            fp.pos_list = p->at<int>(p->L.pos_list) + s0;
            // psi_layer unchanged since it was carried (the slices before this layer are), or
            // psi_{layer-1}, whose slice the last step updated, continued from there
            fp.chain_from = 0;
            fp.chain_wave = nullptr;
            if (carry && layer >= 1 && p->carry_layer == layer) {
                fp.chain_from = layer;
                fp.chain_wave = carried;
            } else if (carry && layer >= 2 && p->carry_layer == layer - 1) {
                fp.chain_from = layer - 1;
                fp.chain_wave = carried;
            }
            launch_fused(p, kLayer, fp, count, st);
            if (carry) {
                p->carry_layer = layer;
                p->carry_key[0] = probe;
                p->carry_key[1] = slices;
                p->carry_key[2] = measured;
            }
            scatter(p, b, count, fp.waves, fp.wave_stride, fp.overlap_patch, fp.ovl_stride, layer, 1, g, w, b > 0, st);
            {
                int n_loss;
                const double *lsrc = loss_entries(p, count, &n_loss);
                loss_sum_kernel<<<1, 256, 0, st>>>(lsrc, n_loss, total, b > 0);
            }
        }
        float *part = p->at<float>(p->L.partial) + (size_t)hp.M * kMaxBlocks;
        max_partial_kernel<<<dim3(wblocks, 1), 256, 0, st>>>(nullptr, w, hw, part);
        max_final_kernel<<<1, 256, 0, st>>>(part, wblocks, p->at<float>(p->L.maxw));
        const bool last = (k + 1 == k_steps);
        step_size_kernel<<<1, 1, 0, st>>>(p->at<float>(p->L.maxt2), layer + 1, hp.M, p->at<float>(p->L.maxw),
                                          step_norm(p), 1.0, mu, last ? mu_out : nullptr, total,
                                          last ? loss_out : nullptr);
        update_kernel<<<(int)std::min<long long>(4096, (hw + 255) / 256), 256, 0, st>>>(
            reinterpret_cast<float2 *>(slices) + (size_t)layer * hw, g, hw, mu);
    }
    return check_hip("ms_layer_step");
}

ms_status ms_full_step(ms_plan *p, hipStream_t st, int32_t k_steps, double step_scale, const ms_c64 *probe,
                       ms_c64 *slices, const float *measured, double *loss_out, double *mu_out)
{
    g_err.clear();
    if (!p || !probe || !slices || !measured) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    p->carry_layer = -1;    // the carried wave no longer holds
    const HostPlan &hp = p->hp;
    if (k_steps < 0) return fail(MS_ERR_INVALID_ARG, "k_steps must be >= 0");
    if (!(step_scale > 0.0) || !std::isfinite(step_scale)) return fail(MS_ERR_INVALID_ARG, "step_scale must be > 0");
    if (!aligned8(probe) || !aligned8(slices) || !aligned8(loss_out) || !aligned8(mu_out) || ((uintptr_t)measured & 3))
        return fail(MS_ERR_INVALID_ARG, "misaligned buffer");
    if (k_steps == 0) return MS_OK;
    const long long hw = (long long)hp.H * hp.W;
    const int M = hp.M;
    class_probes(p, probe, st);
    FusedParams fp = fused_params(p, slices, measured);
    fp.probe_patch = nullptr;
    fp.full = 1;
    double *total = p->at<double>(p->L.scal) + 1;
    double *mu = p->at<double>(p->L.mu_all);
    float *maxw = p->at<float>(p->L.maxw_all);
    float2 *g = p->at<float2>(p->L.full_g);
    float *w = p->at<float>(p->L.full_w);
    float *part = p->at<float>(p->L.partial) + (size_t)M * kMaxBlocks;
    const int wblocks = (int)std::min<long long>(kMaxBlocks, (hw + 255) / 256);
    for (int k = 0; k < k_steps; ++k) {
        // every step size is taken at the current iterate, before any slice changes
        slice_maxima(p, slices, st);
        for (int b = 0; b < hp.nb; ++b) {
            int64_t s0 = (int64_t)b * hp.B;
            int count = (int)std::min<int64_t>(hp.B, hp.S - s0);
            fp.pos_list = p->at<int>(p->L.pos_list) + s0;
            if (p->recompute()) {
                adjoint_recompute(p, fp, b, count, st, g, w, b > 0);
            } else {
                launch_fused(p, kAdjoint, fp, count, st);
                scatter(p, b, count, fp.waves, fp.wave_stride, fp.overlap_patch, fp.ovl_stride, 0, M, g, w, b > 0, st);
            }
            int n_loss;
            const double *lsrc = loss_entries(p, count, &n_loss);
            loss_sum_kernel<<<1, 256, 0, st>>>(lsrc, n_loss, total, b > 0);
        }
        const bool last = (k + 1 == k_steps);
        for (int m = 0; m < M; ++m) {
            max_partial_kernel<<<dim3(wblocks, 1), 256, 0, st>>>(nullptr, w + (size_t)m * hw, hw, part);
            max_final_kernel<<<1, 256, 0, st>>>(part, wblocks, maxw + m);
            step_size_kernel<<<1, 1, 0, st>>>(p->at<float>(p->L.maxt2), m + 1, M, maxw + m, step_norm(p) / step_scale, 1.0,
                                              mu + m, (last && mu_out) ? mu_out + m : nullptr, total,
                                              last ? loss_out : nullptr);
        }
        for (int m = 0; m < M; ++m)
            update_kernel<<<(int)std::min<long long>(4096, (hw + 255) / 256), 256, 0, st>>>(
                reinterpret_cast<float2 *>(slices) + (size_t)m * hw, g + (size_t)m * hw, hw, mu + m);
    }
    return check_hip("ms_full_step");
}

ms_status ms_probe_step(ms_plan *p, hipStream_t st, int32_t k_steps, ms_c64 *probe, const ms_c64 *slices,
                        const float *measured, const int64_t *subset, int64_t n_subset, double *loss_out,
                        double *mu_out)
{
    g_err.clear();
    if (!p || !probe || !slices || !measured) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    p->carry_layer = -1;    // the carried wave no longer holds
    const HostPlan &hp = p->hp;
    if (k_steps < 0) return fail(MS_ERR_INVALID_ARG, "k_steps must be >= 0");
    if (!aligned8(probe) || !aligned8(slices) || !aligned8(loss_out) || !aligned8(mu_out) || ((uintptr_t)measured & 3))
        return fail(MS_ERR_INVALID_ARG, "misaligned buffer");
    int64_t count_all = hp.S;
    const int *list = p->at<int>(p->L.pos_list);
    const int *coff = p->at<int>(p->L.class_off);
    const int *clist = p->at<int>(p->L.class_list);
    if (subset) {
        if (n_subset < 1 || n_subset > hp.S) return fail(MS_ERR_INVALID_ARG, "n_subset must be in [1, S]");
        for (int64_t i = 0; i < n_subset; ++i)
            if (subset[i] < 0 || subset[i] >= hp.S) return fail(MS_ERR_INVALID_ARG, "subset index out of range");
        count_all = n_subset;
    }
    if (k_steps == 0) return MS_OK;
    try {
        if (subset) {
            // the subset, cut into batches and chunks like the full position list
            const int64_t nbs = (n_subset + hp.B - 1) / hp.B;
            p->sub_list.assign(n_subset, 0);
            p->sub_class_off.assign((size_t)nbs * kChunks * (hp.C + 1), 0);
            p->sub_class_list.assign(n_subset, 0);
            std::vector<int> cnt(hp.C);
            int base = 0;
            for (int64_t b = 0; b < nbs; ++b) {
                const int64_t s0 = b * hp.B, count = std::min(n_subset, s0 + hp.B) - s0;
                const Chunking ch = chunking(count);
                for (int c = 0; c < kChunks; ++c) {
                    const int64_t a0 = std::min<int64_t>((int64_t)c * ch.cs, count);
                    const int64_t a1 = std::min<int64_t>(a0 + ch.cs, count);
                    std::fill(cnt.begin(), cnt.end(), 0);
                    for (int64_t a = a0; a < a1; ++a) {
                        p->sub_list[s0 + a] = (int)subset[s0 + a];
                        cnt[hp.pos_info[subset[s0 + a]].z]++;
                    }
                    int *o = &p->sub_class_off[((size_t)b * kChunks + c) * (hp.C + 1)];
                    o[0] = base;
                    for (int k = 0; k < hp.C; ++k) o[k + 1] = o[k] + cnt[k];
                    std::vector<int> cur(o, o + hp.C);
                    for (int64_t a = a0; a < a1; ++a) p->sub_class_list[cur[hp.pos_info[subset[s0 + a]].z]++] = (int)a;
                    base = o[hp.C];
                }
            }
            bool ok = hipMemcpyAsync(p->ws + p->L.sub_list, p->sub_list.data(), p->sub_list.size() * 4,
                                     hipMemcpyHostToDevice, st) == hipSuccess &&
                      hipMemcpyAsync(p->ws + p->L.sub_class_off, p->sub_class_off.data(),
                                     p->sub_class_off.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
                      hipMemcpyAsync(p->ws + p->L.sub_class_list, p->sub_class_list.data(),
                                     p->sub_class_list.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
            if (!ok) return check_hip("ms_probe_step subset upload");
            list = p->at<int>(p->L.sub_list);
            coff = p->at<int>(p->L.sub_class_off);
            clist = p->at<int>(p->L.sub_class_list);
        }
    } catch (const std::bad_alloc &) {
        return fail(MS_ERR_INVALID_ARG, "host out of memory");
    }
    const int nn = hp.n * hp.n;
    const int nbs = (int)((count_all + hp.B - 1) / hp.B);
    slice_maxima(p, slices, st);
    FusedParams fp = fused_params(p, slices, measured);
    double *mu = p->at<double>(p->L.scal);
    double *total = mu + 1;
    float2 *gp = p->at<float2>(p->L.gp);
    for (int k = 0; k < k_steps; ++k) {
        class_probes(p, probe, st);
        for (int b = 0; b < nbs; ++b) {
            int64_t s0 = (int64_t)b * hp.B;
            int count = (int)std::min<int64_t>(hp.B, count_all - s0);
            fp.pos_list = list + s0;
            launch_fused(p, kProbe, fp, count, st);
            class_sums(p, coff + (size_t)b * kChunks * (hp.C + 1), clist, count, b > 0, st);
            {
                int n_loss;
                const double *lsrc = loss_entries(p, count, &n_loss);
                loss_sum_kernel<<<1, 256, 0, st>>>(lsrc, n_loss, total, b > 0);
            }
        }
        probe_gradient(p, gp, st);
        const bool last = (k + 1 == k_steps);
        step_size_kernel<<<1, 1, 0, st>>>(p->at<float>(p->L.maxt2), 0, hp.M, nullptr, step_norm(p), (double)count_all,
                                          mu, last ? mu_out : nullptr, total, last ? loss_out : nullptr);
        update_kernel<<<(nn + 255) / 256, 256, 0, st>>>(reinterpret_cast<float2 *>(probe), gp, nn, mu);
    }
    return check_hip("ms_probe_step");
}

// Probe-mode passes over every batch, then the per-position gradient (and curvature bound).
static ms_status position_pass(ms_plan *p, hipStream_t st, const ms_c64 *probe, const ms_c64 *slices,
                               const float *measured, double *grad, double *curv, double *loss_out)
{
    const HostPlan &hp = p->hp;
    const int nn = hp.n * hp.n;
    slice_maxima(p, slices, st);
    class_probes(p, probe, st);
    class_probe_derivatives(p, probe, st);
    FusedParams fp = fused_params(p, slices, measured);
    double *total = p->at<double>(p->L.scal) + 1;
    const int *list = p->at<int>(p->L.pos_list);
    for (int b = 0; b < hp.nb; ++b) {
        const int64_t s0 = (int64_t)b * hp.B;
        const int count = (int)std::min<int64_t>(hp.B, hp.S - s0);
        fp.pos_list = list + s0;
        launch_fused(p, kProbe, fp, count, st);
        int n_loss;
        const double *lsrc = loss_entries(p, count, &n_loss);
        loss_sum_kernel<<<1, 256, 0, st>>>(lsrc, n_loss, total, b > 0);
        position_grad_kernel<<<count, 256, 0, st>>>(p->at<float2>(p->L.probe_patch), list + s0,
                                                    p->at<int4>(p->L.pos_info), p->at<float2>(p->L.dprobe),
                                                    (long long)hp.C * nn, nn, p->at<float>(p->L.maxt2), hp.M, grad,
                                                    curv);
    }
    if (loss_out) copy_scalar_kernel<<<1, 1, 0, st>>>(total, loss_out);
    return MS_OK;
}

ms_status ms_position_grad(ms_plan *p, hipStream_t st, const ms_c64 *probe, const ms_c64 *slices,
                           const float *measured, double *grad_pos, double *curv_pos, double *loss_out)
{
    g_err.clear();
    if (!p || !probe || !slices || !measured || !grad_pos) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    p->carry_layer = -1;    // the carried wave no longer holds
    if (!aligned8(probe) || !aligned8(slices) || !aligned8(grad_pos) || !aligned8(curv_pos) || !aligned8(loss_out) ||
        ((uintptr_t)measured & 3))
        return fail(MS_ERR_INVALID_ARG, "misaligned buffer");
    position_pass(p, st, probe, slices, measured, grad_pos, curv_pos, loss_out);
    return check_hip("ms_position_grad");
}

ms_status ms_position_step(ms_plan *p, hipStream_t st, double step_scale, const ms_c64 *probe, const ms_c64 *slices,
                           const float *measured, double *positions, double *loss_out)
{
    g_err.clear();
    if (!p || !probe || !slices || !measured || !positions) return fail(MS_ERR_INVALID_ARG, "NULL argument");
    p->carry_layer = -1;    // the carried wave no longer holds
    if (!(step_scale > 0.0) || !std::isfinite(step_scale)) return fail(MS_ERR_INVALID_ARG, "step_scale must be > 0");
    if (!aligned8(probe) || !aligned8(slices) || !aligned8(positions) || !aligned8(loss_out) ||
        ((uintptr_t)measured & 3))
        return fail(MS_ERR_INVALID_ARG, "misaligned buffer");
    double *grad = p->at<double>(p->L.pgrad), *curv = p->at<double>(p->L.pcurv);
    position_pass(p, st, probe, slices, measured, grad, curv, loss_out);
    const long long count = 2 * (long long)p->hp.S;
    position_update_kernel<<<(int)std::min<long long>(1024, (count + 255) / 256), 256, 0, st>>>(positions, grad, curv,
                                                                                               count, step_scale);
    return check_hip("ms_position_step");
}

}  // extern "C"
