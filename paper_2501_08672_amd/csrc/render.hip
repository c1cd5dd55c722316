// Front-to-back alpha compositing (eq. eq:raster) and its hand-written
// adjoint (eq. eq:gaussian_optimization), per (camera, tile) work item.
//
// Layout for wave64: a workgroup of NW waves owns one TS x TS tile; each
// wave owns a region of it (a 16x16 quadrant of a 32x32 tile, the whole of
// a 16x16 or 8x8 tile) and each lane owns PPL pixels of one column of that
// region (PPL = 4, or 1 for 8x8).  The tile's depth-ordered instance list is
// staged through LDS in chunks of up to 256 splats (one lane loads one 48-B
// record as three float4 and stores it in the form the walks use, see
// stage_splat) and every lane walks the chunk with broadcast LDS reads,
// evaluating its PPL pixels against each splat.  The walk ends for the wave
// as soon as none of its pixels is still open.
//
// Per pixel (centre x = (u + 0.5, v + 0.5)):
//   power = -1/2 |L (x - mu)|^2,  alpha = min(alpha_max, sigma exp(power))
//   alpha < alpha_min          -> skip
//   T (1 - alpha) < T_min      -> stop before this Gaussian
//   C += alpha T c,  T *= 1 - alpha
//
// The backward pass stores nothing beyond T_final and the walk length per
// pixel: it walks the same list from the back, recovers T before each
// contributor by dividing by (1 - alpha), and carries the suffix
// S = sum_{j>k} c_j alpha_j T_j + T_final bg, so that
//   dI/dc_k = alpha_k T_k,  dI/dalpha_k = T_k c_k - S / (1 - alpha_k)
// (only v . S is kept, v the pixel's cotangent).
// Each lane first sums the nine 2D gradients of a splat over its own pixels;
// the wave then reduce-scatters them on the VALU (lane swaps and DPP, no LDS
// permutes) so that nine lanes hold the nine totals, and a single atomic
// instruction with those nine lanes active adds them into the
// per-(camera, Gaussian) record.  A splat no pixel of the wave used costs no
// reduction and no atomic.
//
// The fused kernel runs the forward walk, the per-pixel loss and its
// gradient against the target image (L1 or L2, local to the pixel) and the
// backward walk for one item, keeping T, the walk lengths and the colours in
// registers, plus one bit per list position and wave (in LDS) telling the
// backward walk where the forward walk found no contributor.  Its persistent variant launches a few workgroups per CU that
// take items from an atomic counter.
#include "common.hpp"

namespace gsl {

namespace {

// Staged splats hold L' = kPowScale L (L the Cholesky factor of the conic)
// and log2 of the opacity, so that sigma exp(-|L d|^2 / 2) is one exp2 of
// log2(sigma) - |L' d|^2.  kPowScale^2 = log2(e) / 2; conic terms built from
// L' are scaled back by kPowScaleInv2 = 1 / kPowScale^2 = 2 ln 2.
constexpr float kPowScale = 0.84932180028801904f;
constexpr float kPowScaleInv2 = 1.3862943611198906f;

__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// Does any active lane hold p?  The ballot's mask feeds the branch directly
// (no round trip of the condition through a VGPR).
__device__ __forceinline__ bool any_lane(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0ull; }

// Where the pixels of a workgroup are.  Wave w owns a region of CW columns
// by ROWS rows of the TS x TS tile: with four waves on a 32x32 tile each
// takes a 16x16 quadrant (QUAD), otherwise a full-width strip of TS/NW rows.
// Lane l holds column l % CW of the region and rows l / CW + k * RSTEP,
// k < PPL.
//
// Each instance carries a 4-bit mask of the tile parts its alpha_min ellipse
// reaches: for 32x32 tiles the quadrants (bit 2 * row half + column half),
// for 16x16 tiles the quarter-row bands of 4 rows, none for 8x8.  need(w, k)
// is the set of bits covering pixel slot k of wave w: an instance with none
// of them set has alpha < alpha_min on every pixel of the slot.
template <int TS, int NW>
struct Geo {
    static constexpr int BS = kWave * NW;                // lanes per workgroup
    static constexpr bool QUAD = TS == 32 && NW == 4;     // 16x16 quadrant per wave
    static constexpr int CW = QUAD ? 16 : TS;             // columns per wave region
    static constexpr int ROWS = QUAD ? 16 : TS / NW;      // rows per wave region
    static constexpr int PPL = CW * ROWS / kWave;         // pixels per lane
    static constexpr int RSTEP = kWave / CW;              // row stride between a lane's pixels
    static constexpr int CH = BS;                         // splats staged per chunk
    // workgroups per CU the compositing kernels ask the compiler to fit: four
    // waves per workgroup, eight workgroups = eight waves per SIMD (at most 64
    // VGPRs, which the fused kernel fits without spilling); the persistent
    // kernel keeps seven (72 VGPRs: it spills at 64)
    static constexpr int MIN_WG = BS == 256 ? 8 : 1;
    static constexpr int MIN_WG_PERSISTENT = BS == 256 ? 7 : 1;
    static constexpr bool MASKED = TS >= 16;
    static_assert(CW * ROWS % kWave == 0 && PPL >= 1 && ROWS * (QUAD ? 2 : NW) == TS, "tile/wave layout");
    __device__ static int col0(int w) { return QUAD ? (w & 1) * 16 : 0; }
    __device__ static int row0(int w) { return QUAD ? (w >> 1) * 16 : w * ROWS; }
    __device__ static uint32_t need(int w, int k)
    {
        const int r0 = row0(w) + k * RSTEP, r1 = r0 + RSTEP - 1;  // rows of the slot
        if (TS == 32) {
            const uint32_t cols = CW == 16 ? 1u << (col0(w) / 16) : 3u;  // column halves of the region
            uint32_t m = 0;
            for (int h = r0 / 16; h <= r1 / 16; h++) m |= cols << (2 * h);
            return m;
        }
        uint32_t m = 0;
        for (int b = r0 / 4; b <= r1 / 4; b++) m |= 1u << b;
        return m;
    }
    // the slots of a wave need the same bits: the test is per splat
    static constexpr bool ONE_BAND = MASKED && (TS == 32 ? ROWS <= 16 : ROWS <= 4);
};

// DPP sum of a wave: the total lands in lane 63.
__device__ __forceinline__ float dpp_sum63(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));  // row_half_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));  // row_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));  // row_bcast:15
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));  // row_bcast:31
    return v;
}

__device__ __forceinline__ float wave_total(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dpp_sum63(v)), 63));
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0xB1, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x4E, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x141, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x140, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x142, 0xA, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint32_t wave_total_u32(uint32_t v)
{
    v += __builtin_amdgcn_update_dpp(0u, v, 0xB1, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x4E, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x141, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x140, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xA, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xC, 0xF, false);
    return __builtin_amdgcn_readlane(v, 63);
}

// ---- reduce-scatter of the nine 2D-gradient slots across a wave ----------
// Level 32 and 16 pair up slots with the gfx950 half/row swaps (each pair of
// values becomes one value whose two halves, then four rows, carry different
// slots), levels 8 and 4 with DPP mirrors inside a row, and the last two with
// quad permutes.  Each lane ends with the complete sum of one slot (shared by
// the four lanes of a quad) or of a padding slot.  ~27 VALU instead of nine
// full wave reductions.
__device__ __forceinline__ float swap_add32(float a, float b)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_add16(float a, float b)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// lanes with `hi` keep b's partial, the others a's; partner = mirror lane
template <int CTRL>
__device__ __forceinline__ float mirror_add(float a, float b, bool hi)
{
    const float keep = hi ? b : a, send = hi ? a : b;
    return keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float reduce9(const float (&g)[kG2], int lane)
{
    const float y0 = swap_add32(g[0], g[1]);
    const float y1 = swap_add32(g[2], g[3]);
    const float y2 = swap_add32(g[4], g[5]);
    const float y3 = swap_add32(g[6], g[7]);
    const float y4 = swap_add32(g[8], 0.f);
    const float z0 = swap_add16(y0, y1);
    const float z1 = swap_add16(y2, y3);
    const float z2 = swap_add16(y4, 0.f);
    const bool h8 = (lane & 8) != 0, h4 = (lane & 4) != 0;
    const float w0 = mirror_add<0x140>(z0, z1, h8);   // row_mirror
    const float w1 = mirror_add<0x140>(z2, 0.f, h8);
    float u = mirror_add<0x141>(w0, w1, h4);          // row_half_mirror
    u += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(u), 0xB1, 0xF, 0xF, false));  // quad [1,0,3,2]
    u += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(u), 0x4E, 0xF, 0xF, false));  // quad [2,3,0,1]
    return u;
}

// Slot whose total reduce9 leaves in this lane (-1 for a padding slot), found
// by pushing slot tags through the same network.  Call with all lanes active.
__device__ __forceinline__ int reduce9_slot(int lane)
{
    float tag[kG2];
#pragma unroll
    for (int f = 0; f < kG2; f++) tag[f] = lane == 0 ? (float)(f + 1) : 0.f;
    return (int)reduce9(tag, lane) - 1;
}

__device__ __forceinline__ int find_cam(const DevCam *__restrict__ cams, int C, int t)
{
    int lo = 0, hi = C - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cams[mid].tile_offset <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Where one lane's pixels are.
template <int TS, int NW>
struct TileInfo {
    using G = Geo<TS, NW>;
    int c;
    int W, H;
    int px;             // column of this lane
    int py0;            // row of the lane's first pixel; pixel k is at py0 + k * RSTEP
    uint32_t rs, re;    // the tile's instance range
    int64_t pix0;       // packed pixel index of the lane's first pixel
    int64_t plane0;     // float offset of the camera's image
    int64_t npix;       // W * H
    __device__ bool inside(int k) const { return px < W && py0 + k * G::RSTEP < H; }
    __device__ int64_t pix(int k) const { return pix0 + (int64_t)k * G::RSTEP * W; }
    __device__ int64_t off(int k) const { return (int64_t)(py0 + k * G::RSTEP) * W + px; }
};

template <int TS, int NW>
__device__ __forceinline__ TileInfo<TS, NW> tile_info(const RenderArgs &a, int t)
{
    using G = Geo<TS, NW>;
    TileInfo<TS, NW> ti;
    ti.c = find_cam(a.cams, a.C, t);
    const DevCam &cam = a.cams[ti.c];
    ti.W = cam.W;
    ti.H = cam.H;
    const int local = t - cam.tile_offset;
    const int ty = local / cam.tiles_x, tx = local - ty * cam.tiles_x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    ti.px = tx * TS + G::col0(w) + lane % G::CW;
    ti.py0 = ty * TS + G::row0(w) + lane / G::CW;
    ti.rs = a.ranges[2 * (int64_t)t];
    ti.re = a.ranges[2 * (int64_t)t + 1];
    ti.npix = (int64_t)ti.W * ti.H;
    ti.pix0 = cam.pix_offset + (int64_t)ti.py0 * ti.W + ti.px;
    ti.plane0 = 3 * cam.pix_offset;
    return ti;
}

// Index of a chunk entry in a per-wave list: bytes while the chunk and its
// sentinel (index CH) fit, else 16-bit.
template <int CH>
using list_t = typename std::conditional<(CH < 255), uint8_t, uint16_t>::type;

// A chunk of CH staged splats (the LDS chunk depth, 64, 128 or 256) for a
// workgroup of NWV waves.  Entry CH is a sentinel whose alpha is 0 at every
// pixel (log2 opacity = -inf, no tile parts): the forward walk pads its lists
// with it to whole groups of four entries.
// One staged splat, 48 bytes: a walk reads an entry through one address
// (two 16-byte loads and one 8-byte load).
struct StageEntry {
    float4 p0;     // mx, my, l11', l12'  (factor scaled by kPowScale)
    float4 p1;     // l22', log2(opacity), r, g
    float p2;      // b
    uint32_t gid;  // Gaussian index | band mask << 28
    uint32_t pad[2];
};

template <int CH, int NWV>
struct Stage {
    StageEntry e[CH + 1];
    __device__ uint32_t gid_at(int k) const { return e[k].gid; }
    // per wave: the chunk entries that reach its region, in order (rows start
    // 8-byte aligned: groups of four entries are read with one load)
    alignas(8) list_t<CH> wl[NWV][CH + 4];
};

// Entries [j4, j4 + 4) of wave wv's list (j4 a multiple of four) as one
// scalar, entry u in bits [u * 8 * sizeof(list_t), ...).
template <int CH, int NWV>
__device__ __forceinline__ uint64_t list_group(const Stage<CH, NWV> &st, int wv, int j4)
{
    static_assert(((CH + 4) * sizeof(list_t<CH>)) % (4 * sizeof(list_t<CH>)) == 0, "list rows hold whole groups");
    const list_t<CH> *p = &st.wl[wv][j4];
    if (sizeof(list_t<CH>) == 2) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        return (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(v.x) |
               ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(v.y) << 32);
    }
    return (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(*reinterpret_cast<const uint32_t *>(p));
}

template <typename St, int CH>
__device__ __forceinline__ void stage_sentinel(St &st)
{
    st.e[CH].p0 = make_float4(0.f, 0.f, 0.f, 0.f);
    st.e[CH].p1 = make_float4(0.f, -__builtin_inff(), 0.f, 0.f);
    st.e[CH].p2 = 0.f;
    st.e[CH].gid = 0u;
}

// A projection record (mx, my, l11, l12 | l22, opacity, r, g | b ...) in the
// staged form that eval_pair reads.
__device__ __forceinline__ void stage_splat(const float4 *__restrict__ r4, float4 &p0, float4 &p1)
{
    p0 = r4[0];
    p1 = r4[1];
    p0.z *= kPowScale;
    p0.w *= kPowScale;
    p1.x *= kPowScale;
    p1.y = log2f(p1.y);
}

// Stages list positions [start, min(start + CH, end)) into entries 0.. of the
// chunk, each of the BS lanes of the workgroup loading every BS-th entry
// (all loads of a lane issued before the first store).
template <int CH, int BS, typename St>
__device__ __forceinline__ void stage_load(St &st, const RenderArgs &a, const gsl_splat *__restrict__ rec,
                                           uint32_t start, uint32_t end)
{
    constexpr int PER = CH > BS ? CH / BS : 1;
    uint32_t val[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int e = (int)threadIdx.x + q * BS;
        val[q] = (e < CH && start + (uint32_t)e < end) ? a.gauss_ids[start + e] : 0xffffffffu;
    }
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int e = (int)threadIdx.x + q * BS;
        if (e < CH && start + (uint32_t)e < end) {
            const float4 *r4 = reinterpret_cast<const float4 *>(rec + (val[q] & kGidMask));
            stage_splat(r4, st.e[e].p0, st.e[e].p1);
            st.e[e].p2 = r4[2].x;
            st.e[e].gid = val[q];
        }
    }
}

// Does splat `val` reach the band of pixel slot k of this wave?
template <int TS, int NW>
__device__ __forceinline__ bool in_band(uint32_t val, int w, int k)
{
    if (!Geo<TS, NW>::MASKED) return true;
    return ((val >> kGidBits) & Geo<TS, NW>::need(w, k)) != 0u;
}

// Alpha of one (pixel, splat) pair.  Every walk (forward, backward,
// counting) evaluates it with this same instruction sequence — the file is
// compiled without floating-point contraction and the fused multiply-adds are
// explicit — so the backward reproduces the forward's alpha bit for bit and
// the result does not depend on the tile size or the lane layout.
// With the staged form (ax = l11' dx): s = sigma G = exp2(log2 sigma - t1'^2 - t2'^2),
// t1' = l11' dx + l12' dy, t2' = l22' dy.
struct PairEval {
    float dy, s, alpha;
};

__device__ __forceinline__ PairEval eval_pair(const float4 &p0, const float4 &p1, float ax, float fy, float amax)
{
    PairEval e;
    e.dy = fy - p0.y;
    const float t1 = fmaf(p0.w, e.dy, ax);
    const float t2 = p1.x * e.dy;
    const float lg = fmaf(-t1, t1, fmaf(-t2, t2, p1.y));
    e.s = __builtin_amdgcn_exp2f(lg);
    // min(alpha_max, s) on the bit patterns: both are >= 0 (exp2 never
    // returns a negative value), where the unsigned order is the float order,
    // and a NaN s (any sign) gives alpha_max as fminf does.  One integer min
    // instead of a float min that re-canonicalises alpha_max at every step.
    e.alpha = __uint_as_float(min(__float_as_uint(e.s), __float_as_uint(amax)));
    return e;
}

// One front-to-back step of a pixel of transmittance T (negative once the
// pixel is finished) past a Gaussian of alpha a: hit = a >= alpha_min; the
// transmittance behind it T (1 - a), formed as T - a T with one rounding; the
// Gaussian contributes when hit and that stays >= T_min (never for a finished
// pixel, whose product is negative).  The colour weight is T minus the new
// transmittance (a T up to that rounding, 0 when it does not contribute), so
// the weights of a pixel add up to 1 - T_final.  A hit that would cross T_min
// finishes the pixel (T becomes -|T|).  Every walk that composites uses this,
// so their images agree bit for bit.
// Order tests on float bit patterns as integer compares, which issue beside
// the walks' floating-point work instead of taking its slots.  For x, y >= 0
// the unsigned order of the bits is the float order; for a bound y >= 0 and
// any x other than -0 and NaN (neither occurs where these are used) the
// signed order decides x >= y as the float compare does, a negative x having
// the sign bit set.
__device__ __forceinline__ bool ge_nonneg(float x, float y) { return __float_as_uint(x) >= __float_as_uint(y); }
__device__ __forceinline__ bool lt_nonneg(float x, float y) { return __float_as_uint(x) < __float_as_uint(y); }
__device__ __forceinline__ bool ge_bound(float x, float y) { return __float_as_int(x) >= __float_as_int(y); }
__device__ __forceinline__ bool positive(float x) { return __float_as_int(x) > 0; }

struct CompStep {
    float T, w;
    bool acc;
};

__device__ __forceinline__ CompStep comp_step(float T, float a, float amin, float Tmin)
{
    CompStep r;
    const bool hit = ge_nonneg(a, amin);  // alpha and alpha_min are >= 0
    const float Tn = fmaf(-T, a, T);
    r.acc = hit && ge_bound(Tn, Tmin);     // Tn < 0 for a finished pixel, never -0
    float Tsel = r.acc ? Tn : T;
    r.w = T - Tsel;
    // A hit that does not contribute keeps Tsel == T, so the new state is
    // formed from Tsel alone.  The empty statement orders the weight first:
    // T's last use is then the weight and the new state takes T's register
    // (no copy at the loop's back edge).  It emits no instruction.
    asm("" : "+v"(Tsel) : "v"(r.w));
    r.T = (hit && !r.acc) ? -fabsf(Tsel) : Tsel;
    return r;
}

// Builds this wave's list of the chunk entries that reach its region (one
// band test per splat and wave) in Stage::wl; returns its length.  Every lane
// of the workgroup calls it after the chunk is staged; on return the lists
// are visible to their waves.
// The list is followed by sentinel entries up to the next multiple of four
// (for lists with room for them).
template <int TS, int NW, int CH, typename St>
__device__ __forceinline__ int wave_list(St &st, int n, int wv, int lane)
{
    static_assert(CH <= 256, "chunk entries");
    using L = typename std::remove_reference<decltype(st.wl[0][0])>::type;
    constexpr int cap = sizeof(st.wl[0]) / sizeof(L);
    const uint64_t below = (1ull << lane) - 1ull;
    int c = 0;
#pragma unroll
    for (int g = 0; g < CH; g += kWave) {
        const int e = g + lane;
        const bool in = e < n && in_band<TS, NW>(st.gid_at(e), wv, 0);
        const uint64_t m = __ballot(in);
        if (in) st.wl[wv][c + __popcll(m & below)] = (L)e;
        c += __popcll(m);
    }
    if (cap >= CH + 4 && lane < ((c + 3) & ~3) - c) st.wl[wv][c + lane] = (L)CH;
    __syncthreads();
    return c;
}

template <int PPL>
struct PixState {
    float T[PPL];
    float C0[PPL], C1[PPL], C2[PPL];
    uint32_t nwalk[PPL];
};

// Work counters of the forward walk (only the counting kernel uses them).
// `bwd` counts, per pixel, the in-band list positions up to its last
// contributor: the pairs the backward walk has to evaluate.
struct NoCount {
    __device__ void eval(int, bool) {}
    __device__ void contrib(int, bool) {}
};
template <int PPL>
struct Count {
    uint32_t evald = 0, ncontrib = 0;
    uint32_t seen[PPL] = {}, bwd[PPL] = {};
    __device__ void eval(int k, bool b)
    {
        evald += b ? 1u : 0u;
        seen[k] += b ? 1u : 0u;
    }
    __device__ void contrib(int k, bool b)
    {
        ncontrib += b ? 1u : 0u;
        bwd[k] = b ? seen[k] : bwd[k];
    }
};

// Per-wave record of the list positions where at least one pixel of the wave
// contributed (forward walk), consulted by the backward walk of the same
// item to skip positions nothing used.  Positions beyond the record are
// always walked.
constexpr int kHitWords = 128;  // 4096 positions

// Forward walk over the tile list; every lane of the workgroup calls it.
// `hits` (may be null) receives this wave's contribution bits.
template <int TS, int NW, int CH, typename Counter>
__device__ __forceinline__ PixState<Geo<TS, NW>::PPL> fwd_walk(const RenderArgs &a, const TileInfo<TS, NW> &ti,
                                                                Stage<CH, NW> &st, Counter &cnt,
                                                                uint32_t *hits = nullptr)
{
    using G = Geo<TS, NW>;
    constexpr int PPL = G::PPL;
    const gsl_splat *rec = a.splats + (int64_t)ti.c * a.N;
    const float fx = ti.px + 0.5f;
    const float amin = a.o.alpha_min, amax = a.o.alpha_max, Tmin = a.o.T_min;
    // A pixel's transmittance carries its state in the sign: T > 0 while the
    // walk is open, -T once a Gaussian would take it below T_min.  With
    // T_min > 0 and alpha < 1 a finished pixel has T (1 - alpha) < 0 < T_min,
    // so the same test that finishes a pixel keeps it finished.
    PixState<PPL> ps;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        ps.T[k] = ti.inside(k) ? 1.f : -1.f;
        ps.C0[k] = ps.C1[k] = ps.C2[k] = 0.f;
        ps.nwalk[k] = 0;
    }
    float fy[PPL];
#pragma unroll
    for (int k = 0; k < PPL; k++) fy[k] = (float)(ti.py0 + k * G::RSTEP) + 0.5f;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t hbits = 0;
    int hword = 0;
    auto open = [&]() {
        bool o = false;
#pragma unroll
        for (int k = 0; k < PPL; k++) o |= positive(ps.T[k]);
        return o;
    };
    if (threadIdx.x == 0) stage_sentinel<Stage<CH, NW>, CH>(st);
    for (uint32_t start = ti.rs; start < ti.re; start += CH) {
        if (__syncthreads_count(open()) == 0) break;
        stage_load<CH, G::BS>(st, a, rec, start, ti.re);
        __syncthreads();
        const int n = (int)min((uint32_t)CH, ti.re - start);
        // With one band test per wave, the wave walks only the entries that
        // reach its region (a band the ellipse misses has alpha < alpha_min
        // everywhere), listed in order: no skip branch in the walk.
        const int nw_list = G::ONE_BAND ? wave_list<TS, NW, CH>(st, n, wv, lane) : n;
        // Groups of four entries, the last one padded with the sentinel, and
        // the open-pixel test once per group (finished pixels change
        // nothing): one exit from the loop, straight-line groups.
        // (one loop with one exit test, at the end of each group: nested
        // loops make the register allocator copy every accumulator at each
        // group's end)
        constexpr int EB = 8 * (int)sizeof(list_t<CH>);
        const int nw_pad = (nw_list + 3) & ~3;
        uint64_t grp = 0;
        bool go = nw_pad > 0 && any_lane(open());
        for (int jj = 0; go; ) {
            const int u = jj & 3;
            if (G::ONE_BAND && u == 0) grp = list_group(st, wv, jj);
            const int j = G::ONE_BAND ? (int)((grp >> (u * EB)) & ((1u << EB) - 1u)) : (jj < nw_list ? jj : CH);
            const StageEntry &se = st.e[j];
            const float4 p0 = se.p0;
            const float4 p1 = se.p1;
            const float cb = se.p2;
            const uint32_t val = __builtin_amdgcn_readfirstlane(se.gid);  // same for every lane
            const float dx = fx - p0.x;
            const float ax = p0.z * dx;
            const uint32_t pos1 = start + (uint32_t)j + 1u - ti.rs;
            bool used = false;
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (!G::ONE_BAND && !in_band<TS, NW>(val, wv, k)) continue;
                // predicated: every lane evaluates, selects decide what changes
                const PairEval e = eval_pair(p0, p1, ax, fy[k], amax);
                const float T = ps.T[k];
                cnt.eval(k, positive(T) && j < CH);  // the sentinel is not a pair
                const CompStep cs = comp_step(T, e.alpha, amin, Tmin);
                cnt.contrib(k, cs.acc);
                ps.C0[k] = fmaf(cs.w, p1.z, ps.C0[k]);
                ps.C1[k] = fmaf(cs.w, p1.w, ps.C1[k]);
                ps.C2[k] = fmaf(cs.w, cb, ps.C2[k]);
                ps.T[k] = cs.T;
                ps.nwalk[k] = cs.acc ? pos1 : ps.nwalk[k];
                const bool acc = cs.acc;
                used = used || acc;
            }
            if (hits) {
                const int pos = (int)pos1 - 1, wd = pos >> 5;
                if (wd != hword) {
                    // every lane stores the same word: no divergent branch in the loop
                    if (hword < kHitWords) hits[hword] = hbits;
                    hbits = 0;
                    hword = wd;
                }
                if (any_lane(used)) hbits |= 1u << (pos & 31);
            }
            jj++;
            if ((jj & 3) == 0) go = jj < nw_pad && any_lane(open());
        }
        __syncthreads();
    }
    if (hits && lane == 0 && hword < kHitWords) hits[hword] = hbits;
#pragma unroll
    for (int k = 0; k < PPL; k++) ps.T[k] = fabsf(ps.T[k]);
    return ps;
}

// The backward walk's list: entries that reach the wave's region, lie before
// the wave's last contributor (pos < maxn) and, within the first 32 *
// kHitWords positions, where the forward walk saw one of its contributors.
template <int TS, int NW, int CH>
__device__ __forceinline__ int wave_list_bwd(Stage<CH, NW> &st, int n, uint32_t pos0, uint32_t maxn,
                                             const uint32_t *hits, int wv, int lane)
{
    static_assert(CH <= 256, "chunk entries");
    const uint64_t below = (1ull << lane) - 1ull;
    int c = 0;
#pragma unroll
    for (int g = 0; g < CH; g += kWave) {
        const int e = g + lane;
        const uint32_t pos = pos0 + (uint32_t)e;
        bool in = e < n && pos < maxn && (!Geo<TS, NW>::ONE_BAND || in_band<TS, NW>(st.e[e].gid, wv, 0));
        if (in && hits && pos < 32u * kHitWords) in = ((hits[pos >> 5] >> (pos & 31)) & 1u) != 0u;
        const uint64_t m = __ballot(in);
        if (in) st.wl[wv][c + __popcll(m & below)] = (list_t<CH>)e;
        c += __popcll(m);
    }
    __syncthreads();
    return c;
}

// Backward walk.  Tf[k] is the final transmittance of pixel k, v its cotangent.
template <int TS, int NW, int CH>
__device__ __forceinline__ void bwd_walk(const RenderArgs &a, const TileInfo<TS, NW> &ti, Stage<CH, NW> &st,
                                         const float (&Tf)[Geo<TS, NW>::PPL],
                                         const uint32_t (&nw_in)[Geo<TS, NW>::PPL],
                                         const float (&v)[Geo<TS, NW>::PPL][3], uint32_t *s_max,
                                         const uint32_t *hits = nullptr)
{
    using G = Geo<TS, NW>;
    constexpr int PPL = G::PPL;
    const gsl_splat *rec = a.splats + (int64_t)ti.c * a.N;
    float *g2d = a.g2d + (int64_t)ti.c * a.N * kG2;
    const float fx = ti.px + 0.5f;
    const float amin = a.o.alpha_min, amax = a.o.alpha_max;
    const int lane = threadIdx.x & (kWave - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t len = ti.re - ti.rs;
    // SV[k] = v . S with S the colour composited behind the current splat
    // (background included): dI/dalpha = T c - S / (1 - alpha) enters only as
    // v . dI/dalpha, so one scalar per pixel carries the suffix.
    float T[PPL], SV[PPL], fy[PPL];
    uint32_t nw[PPL];
    uint32_t lane_max = 0;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        T[k] = Tf[k];
        SV[k] = T[k] * fmaf(v[k][0], a.o.bg[0], fmaf(v[k][1], a.o.bg[1], v[k][2] * a.o.bg[2]));
        nw[k] = ti.inside(k) ? min(nw_in[k], len) : 0u;  // never walk past the tile's list
        lane_max = max(lane_max, nw[k]);
        fy[k] = (float)(ti.py0 + k * G::RSTEP) + 0.5f;
    }
    __syncthreads();
    if (threadIdx.x == 0) *s_max = 0;
    __syncthreads();
    if (lane_max) atomicMax(s_max, lane_max);
    __syncthreads();
    const uint32_t maxn = *s_max;
    const int slot = reduce9_slot(lane);
    const bool writer = slot >= 0 && (lane & 3) == 0;
    const int64_t lo = ti.rs;
    // the last list position any pixel of this wave walks to
    const uint32_t wave_max = __builtin_amdgcn_readfirstlane(wave_max_u32(lane_max));
    for (int64_t end = lo + maxn; end > lo; end -= CH) {
        const int64_t start = end - CH > lo ? end - CH : lo;
        __syncthreads();
        stage_load<CH, G::BS>(st, a, rec, (uint32_t)start, (uint32_t)end);
        __syncthreads();
        // the entries this wave has to visit, in order (walked in reverse)
        const int nl = wave_list_bwd<TS, NW, CH>(st, (int)(end - start), (uint32_t)(start - lo), wave_max, hits, wv,
                                                 lane);
        constexpr int EB = 8 * (int)sizeof(list_t<CH>);
        uint64_t grp = 0;
        for (int jj = nl - 1; jj >= 0; jj--) {
            // the group of four holding jj (entries past the list are read, never used)
            const int u = jj & 3;
            if (u == 3 || jj == nl - 1) grp = list_group(st, wv, jj & ~3);
            const int j = (int)((grp >> (u * EB)) & ((1u << EB) - 1u));
            const uint32_t pos = (uint32_t)(start - lo) + (uint32_t)j;
            const StageEntry &se = st.e[j];
            const float4 p0 = se.p0;
            const float4 p1 = se.p1;
            const float cb = se.p2;
            const uint32_t val = __builtin_amdgcn_readfirstlane(se.gid);  // same for every lane
            const float dx = fx - p0.x;
            const float ax = p0.z * dx;
            // Per lane: gp = dL/dpower of each pixel; the lane's pixels share
            // dx, so the 2D-mean and conic gradients need only P = sum gp,
            // Q = sum gp dy and R = sum gp dy^2 (t1 = l11 dx + l12 dy,
            // t2 = l22 dy, power = -(t1^2 + t2^2) / 2).  dalpha/dsigma = G =
            // s / sigma, so the opacity gradient is P / sigma.
            float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, P = 0.f, Q = 0.f, R = 0.f;
            bool used = false;
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (!G::ONE_BAND && !in_band<TS, NW>(val, wv, k)) continue;  // wave-uniform skips
                const bool inwalk = pos < nw[k];
                if (!any_lane(inwalk)) continue;    // wave-uniform skips
                const PairEval e = eval_pair(p0, p1, ax, fy[k], amax);
                const float ae = inwalk ? e.alpha : 0.f;
                const bool hit = ge_nonneg(ae, amin);  // one compare: its mask feeds the ballot
                if (!any_lane(hit)) continue;
                used = true;
                // predicated from here: a non-contributing lane takes alpha = 0,
                // so its T stays (r = 1), its colour weight is 0 and its
                // suffix does not change; its alpha gradient is zeroed below
                const float al = hit ? ae : 0.f;
                const float r = rcp_fast(1.f - al);
                const float Tk = T[k] * r;  // transmittance before this Gaussian
                T[k] = Tk;
                const float w = al * Tk;
                gc0 = fmaf(w, v[k][0], gc0);
                gc1 = fmaf(w, v[k][1], gc1);
                gc2 = fmaf(w, v[k][2], gc2);
                const float vc = fmaf(v[k][0], p1.z, fmaf(v[k][1], p1.w, v[k][2] * cb));
                const float ga = fmaf(Tk, vc, -SV[k] * r);
                SV[k] = fmaf(w, vc, SV[k]);
                // alpha is clamped where sigma G >= alpha_max: no gradient to sigma, G
                const float gam = (hit && lt_nonneg(e.s, amax)) ? ga : 0.f;
                const float gp = e.s * gam;
                const float hy = gp * e.dy;
                P += gp;
                Q += hy;
                R = fmaf(hy, e.dy, R);
            }
            if (used) {
                float g[kG2];
                const float u = fmaf(ax, P, p0.w * Q);  // kPowScale * sum of gp t1
                g[0] = kPowScaleInv2 * (p0.z * u);
                g[1] = kPowScaleInv2 * fmaf(p0.w, u, p1.x * (p1.x * Q));
                g[2] = -0.5f * (dx * dx) * P;
                g[3] = -dx * Q;
                g[4] = -0.5f * R;
                g[5] = P * __builtin_amdgcn_exp2f(-p1.y);
                g[6] = gc0;
                g[7] = gc1;
                g[8] = gc2;
                const float tot = reduce9(g, lane);
                if (writer && tot != 0.f) unsafeAtomicAdd(g2d + (int64_t)(val & kGidMask) * kG2 + slot, tot);
            }
        }
    }
}

template <int TS, int NW>
__global__ __launch_bounds__((Geo<TS, NW>::BS), (Geo<TS, NW>::MIN_WG)) void k_render_fwd(RenderArgs a)
{
    using G = Geo<TS, NW>;
    __shared__ Stage<G::CH, NW> st;
    const TileInfo<TS, NW> ti = tile_info<TS, NW>(a, (int)blockIdx.x);
    NoCount nc;
    const PixState<G::PPL> ps = fwd_walk<TS, NW, G::CH>(a, ti, st, nc);
#pragma unroll
    for (int k = 0; k < G::PPL; k++) {
        if (!ti.inside(k)) continue;
        const int64_t off = ti.off(k);
        a.image[ti.plane0 + off] = ps.C0[k] + ps.T[k] * a.o.bg[0];
        a.image[ti.plane0 + ti.npix + off] = ps.C1[k] + ps.T[k] * a.o.bg[1];
        a.image[ti.plane0 + 2 * ti.npix + off] = ps.C2[k] + ps.T[k] * a.o.bg[2];
        a.T_final[ti.pix(k)] = ps.T[k];
        a.n_walk[ti.pix(k)] = ps.nwalk[k];
    }
}

template <int TS, int NW>
__global__ __launch_bounds__((Geo<TS, NW>::BS)) void k_render_bwd(RenderArgs a)
{
    using G = Geo<TS, NW>;
    __shared__ Stage<G::CH, NW> st;
    __shared__ uint32_t s_max;
    const TileInfo<TS, NW> ti = tile_info<TS, NW>(a, (int)blockIdx.x);
    float T[G::PPL], v[G::PPL][3];
    uint32_t nw[G::PPL];
#pragma unroll
    for (int k = 0; k < G::PPL; k++) {
        T[k] = 1.f;
        nw[k] = 0;
        v[k][0] = v[k][1] = v[k][2] = 0.f;
        if (ti.inside(k)) {
            const int64_t off = ti.off(k);
            T[k] = a.T_final[ti.pix(k)];
            nw[k] = a.n_walk[ti.pix(k)];
            v[k][0] = a.dL_dimage[ti.plane0 + off];
            v[k][1] = a.dL_dimage[ti.plane0 + ti.npix + off];
            v[k][2] = a.dL_dimage[ti.plane0 + 2 * ti.npix + off];
        }
    }
    bwd_walk<TS, NW, G::CH>(a, ti, st, T, nw, v, &s_max);
}

// Forward, per-pixel loss and its gradient, backward for one item.
template <int TS, int NW, int CH>
__device__ __forceinline__ void fused_item(const RenderArgs &a, int t, Stage<CH, NW> &st, uint32_t *s_max,
                                           float *s_loss, uint32_t (*s_hits)[kHitWords])
{
    using G = Geo<TS, NW>;
    constexpr int PPL = G::PPL;
    const TileInfo<TS, NW> ti = tile_info<TS, NW>(a, t);
    NoCount nc;
    uint32_t *hits = s_hits[threadIdx.x / kWave];
    const PixState<PPL> ps = fwd_walk<TS, NW, CH>(a, ti, st, nc, hits);
    float v[PPL][3];
    float lsum = 0.f;
    const float inv = 1.f / (3.f * (float)ti.npix);
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        v[k][0] = v[k][1] = v[k][2] = 0.f;
        if (!ti.inside(k)) continue;
        const int64_t off = ti.off(k);
        const float I0 = ps.C0[k] + ps.T[k] * a.o.bg[0];
        const float I1 = ps.C1[k] + ps.T[k] * a.o.bg[1];
        const float I2 = ps.C2[k] + ps.T[k] * a.o.bg[2];
        if (a.image) {
            a.image[ti.plane0 + off] = I0;
            a.image[ti.plane0 + ti.npix + off] = I1;
            a.image[ti.plane0 + 2 * ti.npix + off] = I2;
        }
        const float r0 = I0 - a.target[ti.plane0 + off];
        const float r1 = I1 - a.target[ti.plane0 + ti.npix + off];
        const float r2 = I2 - a.target[ti.plane0 + 2 * ti.npix + off];
        if (a.loss == GSL_LOSS_L1) {
            auto sgn = [](float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); };
            v[k][0] = sgn(r0) * inv;
            v[k][1] = sgn(r1) * inv;
            v[k][2] = sgn(r2) * inv;
            lsum += (fabsf(r0) + fabsf(r1) + fabsf(r2)) * inv;
        } else {
            v[k][0] = r0;
            v[k][1] = r1;
            v[k][2] = r2;
            lsum += 0.5f * (r0 * r0 + r1 * r1 + r2 * r2);
        }
    }
    // per-item loss partial
    const float ls = wave_total(lsum);
    if ((threadIdx.x & (kWave - 1)) == 0) s_loss[threadIdx.x / kWave] = ls;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0;
        for (int w = 0; w < NW; w++) tot += s_loss[w];
        a.loss_part[t] = tot;
    }
    bwd_walk<TS, NW, CH>(a, ti, st, ps.T, ps.nwalk, v, s_max, hits);
}

// Item of workgroup b.  Workgroups are dispatched to the 8 XCDs round-robin
// (b mod 8); with `xcd_chunks` each XCD gets a contiguous run of tiles
// (b mod 8) * chunk + b / 8, so neighbouring tiles, which share most of
// their splats, meet in the same L2.
__device__ __forceinline__ int item_of_block(const RenderArgs &a, uint32_t b, bool xcd_chunks)
{
    if (a.order) return (int)a.order[b];
    if (!xcd_chunks) return (int)b;
    const uint32_t chunk = (uint32_t)((a.T_total + 7) / 8);
    return (int)((b & 7u) * chunk + (b >> 3));
}

template <int TS, int NW, bool XCD, int CH>
__global__ __launch_bounds__((Geo<TS, NW>::BS), (Geo<TS, NW>::MIN_WG)) void k_render_fused(RenderArgs a)
{
    __shared__ Stage<CH, NW> st;
    __shared__ uint32_t s_max;
    __shared__ float s_loss[NW];
    __shared__ uint32_t s_hits[NW][kHitWords];
    const int t = item_of_block(a, blockIdx.x, XCD);
    if (t >= a.T_total) return;  // padding of the XCD-chunked grid (uniform per workgroup)
    fused_item<TS, NW, CH>(a, t, st, &s_max, s_loss, s_hits);
}

template <int TS, int NW, int CH>
__global__ __launch_bounds__((Geo<TS, NW>::BS), (Geo<TS, NW>::MIN_WG_PERSISTENT)) void k_render_fused_persistent(
    RenderArgs a)
{
    __shared__ Stage<CH, NW> st;
    __shared__ uint32_t s_max;
    __shared__ uint32_t s_item;
    __shared__ float s_loss[NW];
    __shared__ uint32_t s_hits[NW][kHitWords];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= (uint32_t)a.T_total) break;
        const int t = a.order ? (int)a.order[item] : (int)item;
        fused_item<TS, NW, CH>(a, t, st, &s_max, s_loss, s_hits);
    }
}

// Work counts of the compositing, by the per-pixel rule on the tile lists:
// counts[0] = (pixel, Gaussian) pairs the forward walk evaluates (up to and
// including the Gaussian that stops it), counts[1] = contributors,
// counts[2] = pairs the backward walk evaluates (sum of walk lengths).
template <int TS, int NW>
__global__ __launch_bounds__((Geo<TS, NW>::BS)) void k_render_count(RenderArgs a, unsigned long long *counts)
{
    using G = Geo<TS, NW>;
    __shared__ Stage<G::CH, NW> st;
    const TileInfo<TS, NW> ti = tile_info<TS, NW>(a, (int)blockIdx.x);
    Count<G::PPL> cnt;
    const PixState<G::PPL> ps = fwd_walk<TS, NW, G::CH>(a, ti, st, cnt);
    (void)ps;
    uint32_t nw = 0;
#pragma unroll
    for (int k = 0; k < G::PPL; k++) nw += cnt.bwd[k];
    const uint32_t e = wave_total_u32(cnt.evald), c = wave_total_u32(cnt.ncontrib), w = wave_total_u32(nw);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicAdd(&counts[0], (unsigned long long)e);
        atomicAdd(&counts[1], (unsigned long long)c);
        atomicAdd(&counts[2], (unsigned long long)w);
    }
}

// Work order of the fused launch: tiles by descending list length (buckets
// of equal floor(log2 length), empty tiles last), so that the longest items
// start first.  One workgroup; the order inside a bucket is whatever the LDS
// atomics give, which only affects scheduling.
__global__ __launch_bounds__(1024) void k_order_by_length(const uint32_t *__restrict__ ranges, int64_t T,
                                                          uint32_t *__restrict__ order)
{
    __shared__ uint32_t s_hist[33];
    __shared__ uint32_t s_cur[33];
    auto bucket = [&](int64_t t) {
        const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
        return len == 0 ? 32u : (uint32_t)__clz(len);  // 31 - floor(log2 len): longest first
    };
    if (threadIdx.x < 33) s_hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) atomicAdd(&s_hist[bucket(t)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int b = 0; b < 33; b++) {
            s_cur[b] = run;
            run += s_hist[b];
        }
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) order[atomicAdd(&s_cur[bucket(t)], 1u)] = (uint32_t)t;
}

__global__ __launch_bounds__(256) void k_reduce_f64(const double *__restrict__ part, int64_t n, double *__restrict__ out)
{
    __shared__ double s[256 / kWave];
    double acc = 0;
    int64_t k = threadIdx.x;
    for (; k + 7 * 256 < n; k += 8 * 256) {  // eight loads in flight, added in the same order
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = part[k + q * 256];
#pragma unroll
        for (int q = 0; q < 8; q++) acc += v[q];
    }
    for (; k < n; k += 256) acc += part[k];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < 256 / kWave; w++) t += s[w];
        *out = t;
    }
}

// ------------------------------------------------------------------ pose Jacobian

// Forward-mode walk for the IESKF visual update (Sec. II-D, Appendix A):
// per pixel, alongside T and the colour, the six tangents dT and the 3 x 6
// tangents of the colour with respect to the camera twist, with every
// threshold decision taken exactly as in the forward walk (same alpha
// evaluation), so the contributor set is the image's.  For a contributor with
// alpha a (da = 0 where the clamp holds, else a dpower, dpower = (Q d) . dmu
// - 1/2 d^T dQ d from the splat's tangent record):
//   dC += c (T da + a dT),   dT <- dT (1 - a) - T da,
// and at the end dI = dC + bg dT.  The item then sums, over its pixels, the
// normal-equation terms of the stacked model z + H xi with z = I - target:
// H^T R^-1 H (21), H^T R^-1 z (6) and z^T R^-1 z, R^-1 a per-pixel weight.
// One pixel per lane for 8x8 and 16x16 tiles, two for 32x32; the splats and
// their tangent records are staged in chunks of up to 256.
template <int CH, int NQ, int NWV>
struct TanStage {
    float4 p0[CH];
    float4 p1[CH];
    float p2[CH];
    uint32_t gid[CH];
    float4 t[NQ][CH];
    uint8_t wl[NWV][CH];  // per wave: the entries that reach its region
    __device__ uint32_t gid_at(int k) const { return gid[k]; }
};

template <int TS, int NW, bool SHC>
__global__ __launch_bounds__((Geo<TS, NW>::BS)) void k_render_jvp(RenderArgs a)
{
    using G = Geo<TS, NW>;
    constexpr int PPL = G::PPL;
    constexpr int CH = G::BS < 256 ? G::BS : 256;
    constexpr int STRIDE = SHC ? kTangentSH : kTangent;
    __shared__ TanStage<CH, STRIDE / 4, NW> st;
    __shared__ double s_nrm[NW][kNrm];
    const int t = (int)blockIdx.x;
    const TileInfo<TS, NW> ti = tile_info<TS, NW>(a, t);
    const gsl_splat *rec = a.splats + (int64_t)ti.c * a.N;
    const float *tan = a.tangent + (int64_t)ti.c * a.N * STRIDE;
    const float fx = ti.px + 0.5f;
    const float amin = a.o.alpha_min, amax = a.o.alpha_max, Tmin = a.o.T_min;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    // T < 0 marks a finished pixel, as in the forward walk
    float T[PPL], C0[PPL], C1[PPL], C2[PPL], fy[PPL], dT[PPL][6], dC[PPL][3][6];
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        T[k] = ti.inside(k) ? 1.f : -1.f;
        C0[k] = C1[k] = C2[k] = 0.f;
        fy[k] = (float)(ti.py0 + k * G::RSTEP) + 0.5f;
#pragma unroll
        for (int j = 0; j < 6; j++) {
            dT[k][j] = 0.f;
            dC[k][0][j] = dC[k][1][j] = dC[k][2][j] = 0.f;
        }
    }
    auto open = [&]() {
        bool o = false;
#pragma unroll
        for (int k = 0; k < PPL; k++) o |= positive(T[k]);
        return o;
    };
    for (uint32_t start = ti.rs; start < ti.re; start += CH) {
        if (__syncthreads_count(open()) == 0) break;
        if (threadIdx.x < CH && start + threadIdx.x < ti.re) {
            const uint32_t val = a.gauss_ids[start + threadIdx.x];
            const uint32_t gi = val & kGidMask;
            const float4 *r4 = reinterpret_cast<const float4 *>(rec + gi);
            stage_splat(r4, st.p0[threadIdx.x], st.p1[threadIdx.x]);
            st.p2[threadIdx.x] = r4[2].x;
            st.gid[threadIdx.x] = val;
            const float4 *t4 = reinterpret_cast<const float4 *>(tan + (int64_t)gi * STRIDE);
#pragma unroll
            for (int q = 0; q < STRIDE / 4; q++) st.t[q][threadIdx.x] = t4[q];
        }
        __syncthreads();
        const int n = (int)min((uint32_t)CH, ti.re - start);
        const int nl = G::ONE_BAND ? wave_list<TS, NW, CH>(st, n, wv, lane) : n;
        for (int jj = 0; jj < nl; jj++) {
            if (!__any(open())) break;
            const int j = G::ONE_BAND ? __builtin_amdgcn_readfirstlane((int)st.wl[wv][jj]) : jj;
            const uint32_t val = __builtin_amdgcn_readfirstlane(st.gid[j]);
            const float4 p0 = st.p0[j];
            const float4 p1 = st.p1[j];
            const float cb = st.p2[j];
            const float dx = fx - p0.x;
            const float ax = p0.z * dx;
            // conic (A, B, C) = L^T L from the staged factor (l11', l12'; 0, l22')
            const float cA = kPowScaleInv2 * (p0.z * p0.z), cB = kPowScaleInv2 * (p0.z * p0.w),
                        cC = kPowScaleInv2 * fmaf(p0.w, p0.w, p1.x * p1.x);
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (!G::ONE_BAND && !in_band<TS, NW>(val, wv, k)) continue;
                const PairEval e = eval_pair(p0, p1, ax, fy[k], amax);
                const CompStep cs = comp_step(T[k], e.alpha, amin, Tmin);
                const bool acc = cs.acc;
                if (!any_lane(acc)) {
                    T[k] = cs.T;
                    continue;
                }
                // a contributor moves the state; others act as alpha = 0, dalpha = 0
                const float al = acc ? e.alpha : 0.f;
                const float sg = (acc && lt_nonneg(e.s, amax)) ? e.alpha : 0.f;  // dalpha = sg * dpower
                const float gx = fmaf(cA, dx, cB * e.dy), gy = fmaf(cB, dx, cC * e.dy);
                const float k2 = -0.5f * dx * dx, k3 = -dx * e.dy, k4 = -0.5f * e.dy * e.dy;
                float da[6];
                {
                    const float4 t0 = st.t[0][j], t1 = st.t[1][j], t2 = st.t[2][j], t3 = st.t[3][j];
                    const float4 t4 = st.t[4][j], t5 = st.t[5][j], t6 = st.t[6][j], t7 = st.t[7][j];
                    const float tv[30] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w, t2.x, t2.y,
                                          t2.z, t2.w, t3.x, t3.y, t3.z, t3.w, t4.x, t4.y, t4.z, t4.w,
                                          t5.x, t5.y, t5.z, t5.w, t6.x, t6.y, t6.z, t6.w, t7.x, t7.y};
#pragma unroll
                    for (int q = 0; q < 6; q++) {
                        float dp = gx * tv[q];
                        dp = fmaf(gy, tv[6 + q], dp);
                        dp = fmaf(k2, tv[12 + q], dp);
                        dp = fmaf(k3, tv[18 + q], dp);
                        dp = fmaf(k4, tv[24 + q], dp);
                        da[q] = sg * dp;
                    }
                }
                const float Tk = T[k];
#pragma unroll
                for (int q = 0; q < 6; q++) {
                    const float w = fmaf(Tk, da[q], al * dT[k][q]);
                    dC[k][0][q] = fmaf(p1.z, w, dC[k][0][q]);
                    dC[k][1][q] = fmaf(p1.w, w, dC[k][1][q]);
                    dC[k][2][q] = fmaf(cb, w, dC[k][2][q]);
                    dT[k][q] = fmaf(dT[k][q], 1.f - al, -Tk * da[q]);
                }
                const float wgt = cs.w;  // al Tk up to the rounding of the transmittance
                if (SHC) {  // the colour's own derivative along dt: + alpha T dc
                    const float4 c0 = st.t[7][j], c1 = st.t[8][j], c2 = st.t[9][j];
                    const float dc[9] = {c0.z, c0.w, c1.x, c1.y, c1.z, c1.w, c2.x, c2.y, c2.z};
#pragma unroll
                    for (int ch = 0; ch < 3; ch++)
#pragma unroll
                        for (int q = 0; q < 3; q++) dC[k][ch][3 + q] = fmaf(wgt, dc[3 * ch + q], dC[k][ch][3 + q]);
                }
                C0[k] = fmaf(wgt, p1.z, C0[k]);
                C1[k] = fmaf(wgt, p1.w, C1[k]);
                C2[k] = fmaf(wgt, cb, C2[k]);
                T[k] = cs.T;
            }
        }
        __syncthreads();
    }
    // per-pixel outputs and the item's normal-equation sums
    float nrm[kNrm];
#pragma unroll
    for (int q = 0; q < kNrm; q++) nrm[q] = 0.f;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        if (!ti.inside(k)) continue;
        const int64_t off = ti.off(k);
        // the same expression as the forward kernels, so the colour matches theirs bit for bit
        const float Tf = fabsf(T[k]);
        const float I[3] = {C0[k] + Tf * a.o.bg[0], C1[k] + Tf * a.o.bg[1], C2[k] + Tf * a.o.bg[2]};
        float Jp[3][6];
#pragma unroll
        for (int ch = 0; ch < 3; ch++)
#pragma unroll
            for (int q = 0; q < 6; q++) Jp[ch][q] = fmaf(a.o.bg[ch], dT[k][q], dC[k][ch][q]);
        if (a.image)
            for (int ch = 0; ch < 3; ch++) a.image[ti.plane0 + ch * ti.npix + off] = I[ch];
        if (a.jac)
            for (int ch = 0; ch < 3; ch++)
                for (int q = 0; q < 6; q++) a.jac[(int64_t)(6 * ch + q) * a.P_total + ti.pix(k)] = Jp[ch][q];
        if (a.target) {
            const float w = a.weight ? a.weight[ti.pix(k)] : 1.f;
            float z[3];
            for (int ch = 0; ch < 3; ch++) z[ch] = I[ch] - a.target[ti.plane0 + ch * ti.npix + off];
            int idx = 0;
#pragma unroll
            for (int r = 0; r < 6; r++)
#pragma unroll
                for (int q = r; q < 6; q++) {
                    float h = Jp[0][r] * Jp[0][q];
                    h = fmaf(Jp[1][r], Jp[1][q], h);
                    h = fmaf(Jp[2][r], Jp[2][q], h);
                    nrm[idx] = fmaf(w, h, nrm[idx]);
                    idx++;
                }
#pragma unroll
            for (int r = 0; r < 6; r++) {
                float h = Jp[0][r] * z[0];
                h = fmaf(Jp[1][r], z[1], h);
                h = fmaf(Jp[2][r], z[2], h);
                nrm[21 + r] = fmaf(w, h, nrm[21 + r]);
            }
            nrm[27] = fmaf(w, fmaf(z[0], z[0], fmaf(z[1], z[1], z[2] * z[2])), nrm[27]);
        }
    }
    if (a.nrm_part) {
#pragma unroll
        for (int q = 0; q < kNrm; q++) {
            const float v = wave_total(nrm[q]);
            if (lane == 0) s_nrm[wv][q] = (double)v;
        }
        __syncthreads();
        if (threadIdx.x < kNrm) {
            double v = 0.0;
            for (int w = 0; w < NW; w++) v += s_nrm[w][threadIdx.x];
            a.nrm_part[(int64_t)t * kNrm + threadIdx.x] = v;
        }
    }
}

// Per-camera FP64 sums of the item partials (the camera's tiles are the
// contiguous range [tile_offset, tile_offset + tiles_x * tiles_y)).
__global__ __launch_bounds__(256) void k_normal_reduce(const double *__restrict__ part,
                                                       const DevCam *__restrict__ cams, double *__restrict__ HtH,
                                                       double *__restrict__ Htz, double *__restrict__ zz)
{
    __shared__ double s[256 / kWave][kNrm];
    const int c = blockIdx.x;
    const int64_t t0 = cams[c].tile_offset, nt = (int64_t)cams[c].tiles_x * cams[c].tiles_y;
    double acc[kNrm];
    for (int q = 0; q < kNrm; q++) acc[q] = 0.0;
    for (int64_t t = threadIdx.x; t < nt; t += 256)
        for (int q = 0; q < kNrm; q++) acc[q] += part[(t0 + t) * kNrm + q];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (int q = 0; q < kNrm; q++) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
        if (lane == 0) s[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNrm) {
        double v = 0.0;
        for (int w = 0; w < 256 / kWave; w++) v += s[w][threadIdx.x];
        const int q = threadIdx.x;
        if (q < 21) {
            if (HtH) {
                // upper-triangle index q -> (r, col)
                int r = 0, k = q;
                while (k >= 6 - r) {
                    k -= 6 - r;
                    r++;
                }
                const int col = r + k;
                HtH[(int64_t)c * 36 + r * 6 + col] = v;
                HtH[(int64_t)c * 36 + col * 6 + r] = v;
            }
        } else if (q < 27) {
            if (Htz) Htz[(int64_t)c * 6 + (q - 21)] = v;
        } else if (zz) {
            zz[c] = v;
        }
    }
}

// waves per tile for each tile size
template <int TS>
struct Waves {
    static constexpr int NW = TS == 32 ? 4 : 1;
};

template <int TS>
void launch_fwd_t(const RenderArgs &a, hipStream_t s)
{
    constexpr int NW = Waves<TS>::NW;
    hipLaunchKernelGGL((k_render_fwd<TS, NW>), dim3((unsigned)a.T_total), dim3(Geo<TS, NW>::BS), 0, s, a);
}
template <int TS>
void launch_bwd_t(const RenderArgs &a, hipStream_t s)
{
    constexpr int NW = Waves<TS>::NW;
    hipLaunchKernelGGL((k_render_bwd<TS, NW>), dim3((unsigned)a.T_total), dim3(Geo<TS, NW>::BS), 0, s, a);
}
template <int TS>
void launch_count_t(const RenderArgs &a, unsigned long long *counts, hipStream_t s)
{
    constexpr int NW = Waves<TS>::NW;
    hipLaunchKernelGGL((k_render_count<TS, NW>), dim3((unsigned)a.T_total), dim3(Geo<TS, NW>::BS), 0, s, a, counts);
}
template <int TS, int CH>
void launch_fused_tc(const RenderArgs &a, int variant, int num_cus, hipStream_t s)
{
    constexpr int NW = Waves<TS>::NW;
    if (variant & 1) {
        const int per_cu = 32 / NW;
        int64_t g = (int64_t)num_cus * per_cu;
        if (g > a.T_total) g = a.T_total;
        hipLaunchKernelGGL((k_render_fused_persistent<TS, NW, CH>), dim3((unsigned)g), dim3(Geo<TS, NW>::BS), 0, s,
                           a);
    } else if ((variant & 4) && !a.order) {
        const int64_t g = 8 * ((a.T_total + 7) / 8);
        hipLaunchKernelGGL((k_render_fused<TS, NW, true, CH>), dim3((unsigned)g), dim3(Geo<TS, NW>::BS), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_render_fused<TS, NW, false, CH>), dim3((unsigned)a.T_total), dim3(Geo<TS, NW>::BS), 0,
                           s, a);
    }
}
template <int TS>
void launch_fused_t(const RenderArgs &a, int variant, int chunk, int num_cus, hipStream_t s)
{
    switch (chunk) {
    case 64: launch_fused_tc<TS, 64>(a, variant, num_cus, s); break;
    case 128: launch_fused_tc<TS, 128>(a, variant, num_cus, s); break;
    default: launch_fused_tc<TS, 256>(a, variant, num_cus, s); break;
    }
}

}  // namespace

void launch_render_count(const RenderArgs &a, unsigned long long *counts, hipStream_t s)
{
    if (a.T_total == 0) return;
    switch (a.o.tile) {
    case 8: launch_count_t<8>(a, counts, s); break;
    case 16: launch_count_t<16>(a, counts, s); break;
    default: launch_count_t<32>(a, counts, s); break;
    }
}

void launch_render_fwd(const RenderArgs &a, hipStream_t s)
{
    if (a.T_total == 0) return;
    switch (a.o.tile) {
    case 8: launch_fwd_t<8>(a, s); break;
    case 16: launch_fwd_t<16>(a, s); break;
    default: launch_fwd_t<32>(a, s); break;
    }
}

void launch_render_bwd(const RenderArgs &a, hipStream_t s)
{
    if (a.T_total == 0) return;
    switch (a.o.tile) {
    case 8: launch_bwd_t<8>(a, s); break;
    case 16: launch_bwd_t<16>(a, s); break;
    default: launch_bwd_t<32>(a, s); break;
    }
}

void launch_render_fused(const RenderArgs &a, int variant, int chunk, int num_cus, hipStream_t s)
{
    if (a.T_total == 0) return;
    switch (a.o.tile) {
    case 8: launch_fused_t<8>(a, variant, chunk, num_cus, s); break;
    case 16: launch_fused_t<16>(a, variant, chunk, num_cus, s); break;
    default: launch_fused_t<32>(a, variant, chunk, num_cus, s); break;
    }
}

void launch_order_by_length(const uint32_t *ranges, int64_t T, uint32_t *order, hipStream_t s)
{
    if (T > 0) hipLaunchKernelGGL(k_order_by_length, dim3(1), dim3(1024), 0, s, ranges, T, order);
}

void launch_render_jvp(const RenderArgs &a, hipStream_t s)
{
    if (a.T_total == 0) return;
    switch (a.o.tile) {
        case 8:
            if (a.sh_colour) hipLaunchKernelGGL((k_render_jvp<8, 1, true>), dim3((unsigned)a.T_total), dim3(64), 0, s, a);
            else hipLaunchKernelGGL((k_render_jvp<8, 1, false>), dim3((unsigned)a.T_total), dim3(64), 0, s, a);
            break;
        case 16:
            if (a.sh_colour) hipLaunchKernelGGL((k_render_jvp<16, 4, true>), dim3((unsigned)a.T_total), dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_render_jvp<16, 4, false>), dim3((unsigned)a.T_total), dim3(256), 0, s, a);
            break;
        default:
            if (a.sh_colour) hipLaunchKernelGGL((k_render_jvp<32, 8, true>), dim3((unsigned)a.T_total), dim3(512), 0, s, a);
            else hipLaunchKernelGGL((k_render_jvp<32, 8, false>), dim3((unsigned)a.T_total), dim3(512), 0, s, a);
            break;
    }
}

void launch_normal_reduce(const double *nrm_part, const DevCam *cams, int C, double *HtH, double *Htz, double *zz,
                          hipStream_t s)
{
    if (C == 0) return;
    hipLaunchKernelGGL(k_normal_reduce, dim3((unsigned)C), dim3(256), 0, s, nrm_part, cams, HtH, Htz, zz);
}

void launch_reduce_f64(const double *part, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, s, part, n, out);
}

}  // namespace gsl
