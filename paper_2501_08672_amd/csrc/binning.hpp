// Binning walk shared by the projection (which counts the tiles each splat
// reaches) and the emission of instances (sort.hip): the exact ellipse-tile
// test, the tile-part masks, and the wave-wide flat expansion of a wave's
// records over their bbox tiles.  Both kernels run this same code, so the
// emitted instances are exactly the counted ones.
#pragma once
#include "common.hpp"

namespace gsl {

namespace {

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (lane == 0) ? 0ull : (~0ull >> (64 - lane)); }

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v, int lane)
{
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

// Which parts of tile (tx, ty) the splat's alpha_min ellipse reaches: for
// 32x32 tiles the 16x16 quadrants (bit 2 * row half + column half), for 16x16
// tiles the quarter-row bands (bit q: rows [4q, 4q + 4)), for 8x8 tiles none.
// A part is marked when the ellipse reaches the rectangle of its pixel
// centres (clipped to the image): the same exact test as the tile's, on the
// part, so a pixel of an unmarked part has alpha < alpha_min.
__device__ __forceinline__ uint32_t tile_parts(const EllipseTest &e, int W, int H, int tile, int tx, int ty)
{
    uint32_t b = 0;
    if (tile == 32) {
#pragma unroll
        for (int rh = 0; rh < 2; rh++)
#pragma unroll
            for (int ch = 0; ch < 2; ch++) {
                const float x0 = (float)(tx * 32 + ch * 16) + 0.5f, x1 = (float)min(tx * 32 + ch * 16 + 16, W) - 0.5f;
                const float y0 = (float)(ty * 32 + rh * 16) + 0.5f, y1 = (float)min(ty * 32 + rh * 16 + 16, H) - 0.5f;
                if (x0 <= x1 && y0 <= y1 && ellipse_hits_rect(e, x0, x1, y0, y1)) b |= 1u << (2 * rh + ch);
            }
    } else if (tile == 16) {
        const float x0 = (float)(tx * 16) + 0.5f, x1 = (float)min(tx * 16 + 16, W) - 0.5f;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float y0 = (float)(ty * 16 + 4 * q) + 0.5f, y1 = (float)min(ty * 16 + 4 * q + 4, H) - 0.5f;
            if (y0 <= y1 && ellipse_hits_rect(e, x0, x1, y0, y1)) b |= 1u << q;
        }
    }
    return b;
}

// Does the splat's alpha_min ellipse reach tile (tx, ty), and which parts of
// it (tile_parts; only when `bands` is given)?
__device__ __forceinline__ bool tile_hit(const EllipseTest &e, int W, int H, int tile, int tx, int ty,
                                         uint32_t *bands)
{
    float rx0, rx1, ry0, ry1;
    tile_rect(tx, ty, tile, W, H, rx0, rx1, ry0, ry1);
    if (!ellipse_hits_rect(e, rx0, rx1, ry0, ry1)) return false;
    if (bands) *bands = tile_parts(e, W, H, tile, tx, ty);
    return true;
}

// Counting and emitting share one walk.  A wave expands the bbox tiles of its
// records into one flat list (an exclusive scan of the bbox tile counts gives
// each record its segment) and tests 64 list entries per step, lane l entry
// t0 + l.  The records with at least one bbox tile sit in LDS in lane order,
// compacted, so an entry's record index is the number of segments starting at
// or before it, minus one: each record's lane marks its segment start in the
// `mark` word of the array slot at that window position (tagged with the
// step; these words are not part of the record in the slot), one ballot over
// the marks gives the starts inside the window, and a popcount finishes the
// lookup (one LDS round trip per step).  Every lane is busy whatever the mix of small and
// large splats, and no step waits on a global load.  Within a record the hits
// keep bbox order (row-major), so an instance's slot is the record's hits
// before this window plus the hits of the same record on lower lanes.
struct alignas(16) RecTiles {
    float mx, my, l11, l12, l22, kq, kv, kh;
    int32_t tx0, ty0, nx, tiles_x;
    int32_t tile_base;
    uint32_t wh;  // image width | height << 16 (both below 2^15)
    uint32_t gid;
    uint32_t base, limit, excl;
    float rnx;     // 1 / nx
    uint32_t mark;  // walk: segment-start tag of this window position
};
static_assert(sizeof(RecTiles) == 80, "RecTiles layout");

__device__ __forceinline__ int bbox_tiles(const gsl_binrec &s, int tile)
{
    if (s.x0 > s.x1) return 0;
    return (s.x1 / tile - s.x0 / tile + 1) * (s.y1 / tile - s.y0 / tile + 1);
}

__device__ __forceinline__ void rec_fill(RecTiles &r, const gsl_binrec &s, const DevCam &cam, int tile,
                                         uint32_t gid, uint32_t base, uint32_t limit, uint32_t excl)
{
    const EllipseTest e = ellipse_test(s);
    r.mx = e.mx;
    r.my = e.my;
    r.l11 = e.l11;
    r.l12 = e.l12;
    r.l22 = e.l22;
    r.kq = e.kq;
    r.kv = e.kv;
    r.kh = e.kh;
    r.tx0 = s.x0 / tile;
    r.ty0 = s.y0 / tile;
    r.nx = s.x1 / tile - r.tx0 + 1;
    r.tiles_x = cam.tiles_x;
    r.tile_base = cam.tile_offset;
    r.wh = (uint32_t)cam.W | ((uint32_t)cam.H << 16);
    r.gid = gid;
    r.base = base;
    r.limit = limit;
    r.excl = excl;
    r.rnx = 1.0f / (float)r.nx;
}

// Lanes [lo, hi) of a wave, lo and hi clamped to [0, 64].
__device__ __forceinline__ uint64_t lane_range(int64_t lo, int64_t hi)
{
    lo = lo < 0 ? 0 : (lo > kWave ? kWave : lo);
    hi = hi < 0 ? 0 : (hi > kWave ? kWave : hi);
    const uint64_t below_hi = hi >= kWave ? ~0ull : ((1ull << hi) - 1ull);
    const uint64_t below_lo = lo >= kWave ? ~0ull : ((1ull << lo) - 1ull);
    return below_hi & ~below_lo;
}

// Highest set bit of a non-zero 64-bit mask.
__device__ __forceinline__ int top_bit(uint64_t m) { return 63 - __clzll(m); }

// The caller's slot among the lanes of its wave that have bbox tiles (records
// are stored at this index in the wave's RecTiles array).
__device__ __forceinline__ int rec_slot(uint32_t nt, int lane)
{
    return __popcll(__ballot(nt != 0u) & lanemask_lt(lane));
}

// Walks the flat tile list of the wave's records.  rec: the wave's 64 slots,
// holding its records with at least one bbox tile compacted in lane order
// (rec_slot), visible to all its lanes.  [excl, incl) is the calling lane's own segment (empty for a lane without
// bbox tiles).  Returns the hit count of the calling lane's own record.
template <bool emit>
__device__ __forceinline__ uint32_t expand_tiles(RecTiles *rec, int lane, uint32_t excl, uint32_t incl, uint32_t total,
                                                 int tile, uint32_t *__restrict__ tile_ids,
                                                 uint32_t *__restrict__ gauss_ids)
{
    uint32_t own = 0;
    int started = 0;      // records whose segment starts before this window
    uint32_t carry = 0;   // hits of the record running into this window, before it
    const uint64_t upto = ~0ull >> (kWave - 1 - lane);  // lanes 0 .. lane
    const uint64_t below = lanemask_lt(lane);
    rec[lane].mark = 0u;  // no step's tag (t0 + 1 >= 1)
    __builtin_amdgcn_wave_barrier();
    for (uint32_t t0 = 0; t0 < total; t0 += kWave) {
        const uint32_t g = t0 + (uint32_t)lane;
        const uint32_t tag = t0 + 1u;
        if (incl > excl && excl >= t0 && excl - t0 < (uint32_t)kWave) rec[excl - t0].mark = tag;
        __builtin_amdgcn_wave_barrier();
        const uint64_t starts = __ballot(rec[lane].mark == tag);
        __builtin_amdgcn_wave_barrier();
        const uint64_t mine = starts & upto;  // starts at or below this entry
        int o = started + __popcll(mine) - 1;  // the entry's record (>= 0 for g < total)
        o = o < 0 ? 0 : o;
        bool hit = false;
        uint32_t bands = 0;
        int tx = 0, ty = 0;
        const RecTiles &r = rec[o];
        if (g < total) {
            const uint32_t t = g - r.excl;
            uint32_t q = (uint32_t)((float)t * r.rnx);
            if (q * (uint32_t)r.nx > t) q--;
            else if ((q + 1) * (uint32_t)r.nx <= t) q++;
            ty = r.ty0 + (int)q;
            tx = r.tx0 + (int)(t - q * (uint32_t)r.nx);
            EllipseTest e;
            e.mx = r.mx;
            e.my = r.my;
            e.l11 = r.l11;
            e.l12 = r.l12;
            e.l22 = r.l22;
            e.kq = r.kq;
            e.kv = r.kv;
            e.kh = r.kh;
            hit = tile_hit(e, (int)(r.wh & 0xffffu), (int)(r.wh >> 16), tile, tx, ty, emit ? &bands : nullptr);
        }
        const uint64_t mask = __ballot(hit);
        if (emit && hit) {
            // the entry's record starts at the highest start at or below it,
            // else it runs in from before the window with `carry` hits
            const uint64_t seg = mine ? below & ~lanemask_lt(top_bit(mine)) : below;
            const uint32_t slot = (mine ? 0u : carry) + (uint32_t)__popcll(mask & seg);
            if (slot < r.limit) {  // never beyond the record's counted range
                tile_ids[r.base + slot] = (uint32_t)(r.tile_base + ty * r.tiles_x + tx);
                gauss_ids[r.base + slot] = r.gid | (bands << kGidBits);
            }
        }
        // the record running into the next window: its hits up to there
        const uint64_t last = starts ? ~lanemask_lt(top_bit(starts)) : ~0ull;
        carry = (starts ? 0u : carry) + (uint32_t)__popcll(mask & last);
        started += __popcll(starts);
        own += (uint32_t)__popcll(mask & lane_range((int64_t)excl - (int64_t)t0, (int64_t)incl - (int64_t)t0));
    }
    return own;
}

// Records whose bbox spans more than kBigTiles tiles leave the wave-wide walk
// for a list that a second kernel takes one record per workgroup.  In depth
// order the largest splats (the nearest) are contiguous: left in the flat
// walk they would load a few waves with most of the work while the rest of
// the chip idles.
constexpr uint32_t kBigTiles = 256;
constexpr int kBigBlocks = 1024;  // workgroups of the per-record kernels (grid-stride over the list)

__device__ __forceinline__ void push_big(uint32_t *__restrict__ list, uint32_t *__restrict__ n, uint32_t v)
{
    list[atomicAdd(n, 1u)] = v;
}

}  // namespace

}  // namespace gsl
