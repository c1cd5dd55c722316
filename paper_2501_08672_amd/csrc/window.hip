// Device-side maintenance of the sliding window of Gaussians (Sec. II-C,
// the incremental window update, Steps 1-4).
//
// The window's per-Gaussian data live at a fixed capacity in HBM: R rows of
// ld 4-byte words (row r of Gaussian i at r * ld + i), plus one 64-bit
// root-voxel key per Gaussian (Sec. II-A, eq. HashKey).  A frame's update is
// two calls:
//   classify  the keys of the current LiDAR frame's points go into an
//             open-addressing hash set (one 16-byte slot per key: the key,
//             the index of its first point, and whether a window Gaussian
//             carries it).  Each window Gaussian looks its key up: absent
//             means DELETE (Step 1).  Each point that is the first of its key
//             and whose key no window Gaussian carries yields an ADD key
//             (Step 3).  Two exclusive scans order the DELETE slots and the
//             ADD keys (window order, first-point order).
//   compact   in place: the DELETE Gaussians are gathered out (their
//             parameters go back to the global map), then the k-th DELETE
//             slot below n - D receives the k-th kept Gaussian of the rear
//             [n - D, n) (Step 2), then the caller's new Gaussians are
//             appended at n - D (Step 4).  Only the D evicted, the at most D
//             moved and the A appended Gaussians are touched.
// The three compaction phases are separate launches because each reads
// slots that the next one overwrites.  Every compaction kernel first checks
// that the caller's (n, D) equal what classify found on the device and does
// nothing otherwise, so a stale count can never index out of bounds.
#include "common.hpp"

namespace gsl {

namespace {

constexpr uint64_t kEmptyKey = ~0ull;  // no packed key has its top bit set
constexpr uint32_t kNoSlot = 0xffffffffu;
constexpr int kKeyBits = 21;
constexpr double kKeyBias = (double)(1 << 20);
constexpr int64_t kWinMagic = 0x67736c77696e6477ll;  // marks a header written by classify

struct __align__(16) Slot {
    uint64_t key;    // kEmptyKey when free
    uint32_t first;  // smallest index of a point with this key
    uint32_t inwin;  // 1 once a window Gaussian carries this key
};
static_assert(sizeof(Slot) == 16, "hash slot is 16 bytes");

// splitmix64's output function (Steele, Lea, Flood, OOPSLA 2014): a bijective
// 64-bit mix, so neighbouring voxel keys land on unrelated slots.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// floor(p / v_s) per axis in fp64 (IEEE division, exact floor for float32
// inputs), biased by 2^20 into three 21-bit fields.
__device__ __forceinline__ bool point_key(const float *__restrict__ p, double vs, uint64_t &key)
{
    uint64_t k = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const float c = p[a];
        if (!isfinite(c)) return false;
        const double f = floor((double)c / vs);
        if (!(f >= -kKeyBias && f < kKeyBias)) return false;
        k = (k << kKeyBits) | (uint64_t)(int64_t)(f + kKeyBias);
    }
    key = k;
    return true;
}

__global__ __launch_bounds__(256) void k_voxel_keys(const float *__restrict__ xyz, int64_t P, int64_t ps, int64_t as,
                                                    double vs, uint64_t *__restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float p[3] = {xyz[i * ps], xyz[i * ps + as], xyz[i * ps + 2 * as]};
    uint64_t key;
    keys[i] = point_key(p, vs, key) ? key : kEmptyKey;
}

__global__ void k_win_init(Slot *__restrict__ tab, uint64_t cap, int64_t *__restrict__ hdr, int64_t n, int64_t P)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < cap) {
        Slot e;
        e.key = kEmptyKey;
        e.first = kNoSlot;
        e.inwin = 0;
        tab[s] = e;
    }
    if (s == 0) {
        hdr[2] = n;
        hdr[3] = P;
        hdr[4] = kWinMagic;
    }
}

// Step 3, first half: every valid point inserts its key.  The table holds at
// least twice as many slots as points, so a free slot or the key itself is
// always reached within `mask + 1` probes.
__global__ __launch_bounds__(256) void k_win_insert(const float *__restrict__ pts, int64_t P, double vs,
                                                    Slot *__restrict__ tab, uint64_t mask, uint32_t *__restrict__ pslot)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    uint64_t key;
    uint32_t slot = kNoSlot;
    if (point_key(pts + 3 * i, vs, key)) {
        uint64_t s = mix64(key) & mask;
        for (uint64_t probe = 0; probe <= mask; probe++) {
            const unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long *>(&tab[s].key),
                                                      (unsigned long long)kEmptyKey, (unsigned long long)key);
            if (prev == kEmptyKey || prev == key) {
                atomicMin(&tab[s].first, (uint32_t)i);
                slot = (uint32_t)s;
                break;
            }
            s = (s + 1) & mask;
        }
    }
    pslot[i] = slot;
}

// Step 1: a window Gaussian whose key is not in the frame's set is DELETE.
__global__ __launch_bounds__(256) void k_win_mark(const uint64_t *__restrict__ keys, int64_t n,
                                                  Slot *__restrict__ tab, uint64_t mask, uint32_t *__restrict__ del)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = keys[i];
    uint32_t d = 1;
    if (key != kEmptyKey) {
        uint64_t s = mix64(key) & mask;
        for (uint64_t probe = 0; probe <= mask; probe++) {
            const uint64_t cur = tab[s].key;
            if (cur == key) {
                tab[s].inwin = 1u;  // every writer stores the same value
                d = 0;
                break;
            }
            if (cur == kEmptyKey) break;
            s = (s + 1) & mask;
        }
    }
    del[i] = d;
}

// Step 3, second half: the first point of a key no window Gaussian carries.
__global__ __launch_bounds__(256) void k_win_addflag(const uint32_t *__restrict__ pslot, int64_t P,
                                                     const Slot *__restrict__ tab, uint32_t *__restrict__ addf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const uint32_t s = pslot[i];
    uint32_t f = 0;
    if (s != kNoSlot) {
        const Slot e = tab[s];
        f = (e.first == (uint32_t)i && e.inwin == 0u) ? 1u : 0u;
    }
    addf[i] = f;
}

__global__ __launch_bounds__(256) void k_win_addkeys(const uint32_t *__restrict__ addf,
                                                     const uint32_t *__restrict__ arank,
                                                     const uint32_t *__restrict__ pslot, int64_t P,
                                                     const Slot *__restrict__ tab, uint64_t *__restrict__ add_keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P || !addf[i]) return;
    add_keys[arank[i]] = tab[pslot[i]].key;
}

// Position of the e-th DELETE Gaussian, and the two counts for the caller.
__global__ __launch_bounds__(256) void k_win_evpos(const uint32_t *__restrict__ del, const uint32_t *__restrict__ drank,
                                                   int64_t n, uint32_t *__restrict__ evpos,
                                                   const int64_t *__restrict__ hdr, int32_t *__restrict__ counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && counts) {
        counts[0] = (int32_t)hdr[0];
        counts[1] = (int32_t)hdr[1];
    }
    if (i < n && del[i]) evpos[drank[i]] = (uint32_t)i;
}

__device__ __forceinline__ bool counts_match(const int64_t *hdr, int64_t n, int64_t D)
{
    return hdr[4] == kWinMagic && hdr[2] == n && hdr[0] == D;
}

__global__ void k_win_status(const int64_t *__restrict__ hdr, int64_t n, int64_t D, int32_t *__restrict__ status)
{
    *status = counts_match(hdr, n, D) ? 0 : 1;
}

// Compaction phase 1: gather the DELETE Gaussians (window order).
__global__ __launch_bounds__(256) void k_win_evict(const uint64_t *__restrict__ keys, const float *__restrict__ rows,
                                                   int R, int64_t ld, int64_t n, int64_t D,
                                                   const uint32_t *__restrict__ evpos, const int64_t *__restrict__ hdr,
                                                   uint64_t *__restrict__ ek, float *__restrict__ er)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D || !counts_match(hdr, n, D)) return;
    const int64_t i = evpos[e];
    if (ek) ek[e] = keys[i];
    if (er)
        for (int r = 0; r < R; r++) er[r * D + e] = rows[r * ld + i];
}

// Compaction phase 2: the kept Gaussians of [n - D, n) fill the DELETE slots
// below n - D in order.  Reads only [n - D, n), writes only below n - D.
__global__ __launch_bounds__(256) void k_win_fill(uint64_t *__restrict__ keys, float *__restrict__ rows, int R,
                                                  int64_t ld, int64_t n, int64_t D, const uint32_t *__restrict__ del,
                                                  const uint32_t *__restrict__ drank,
                                                  const uint32_t *__restrict__ evpos, const int64_t *__restrict__ hdr)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= D || !counts_match(hdr, n, D)) return;
    const int64_t i = n - D + t;
    if (del[i]) return;
    const int64_t d_front = drank[n - D];        // DELETE slots below n - D
    const int64_t k = t - ((int64_t)drank[i] - d_front);  // rank among the rear's kept Gaussians
    const int64_t dest = evpos[k];
    keys[dest] = keys[i];
    for (int r = 0; r < R; r++) rows[r * ld + dest] = rows[r * ld + i];
}

// Compaction phase 3: append the new Gaussians at n - D.
__global__ __launch_bounds__(256) void k_win_append(uint64_t *__restrict__ keys, float *__restrict__ rows, int R,
                                                    int64_t ld, int64_t n, int64_t D,
                                                    const uint64_t *__restrict__ akeys,
                                                    const float *__restrict__ arows, int64_t A,
                                                    const int64_t *__restrict__ hdr)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A || !counts_match(hdr, n, D)) return;
    const int64_t dest = n - D + a;
    keys[dest] = akeys[a];
    for (int r = 0; r < R; r++) rows[r * ld + dest] = arows[r * A + a];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

uint64_t window_table_slots(int64_t P)
{
    uint64_t cap = 1024;
    while (cap < 2 * (uint64_t)P) cap <<= 1;
    return cap;
}

void launch_voxel_keys(const float *xyz, int64_t P, int64_t ps, int64_t as, float voxel_size, uint64_t *keys,
                       hipStream_t s)
{
    if (P > 0)
        hipLaunchKernelGGL(k_voxel_keys, dim3(blocks_for(P)), dim3(256), 0, s, xyz, P, ps, as, (double)voxel_size,
                           keys);
}

void launch_window_classify(const float *pts, int64_t P, float voxel_size, const uint64_t *keys, int64_t n,
                            const WinWs &w, int32_t *counts, uint64_t *add_keys, hipStream_t s)
{
    Slot *tab = reinterpret_cast<Slot *>(w.table);
    const uint64_t mask = w.slots - 1;
    hipLaunchKernelGGL(k_win_init, dim3(blocks_for((int64_t)w.slots)), dim3(256), 0, s, tab, w.slots, w.hdr, n, P);
    if (P > 0)
        hipLaunchKernelGGL(k_win_insert, dim3(blocks_for(P)), dim3(256), 0, s, pts, P, (double)voxel_size, tab, mask,
                           w.pslot);
    if (n > 0) hipLaunchKernelGGL(k_win_mark, dim3(blocks_for(n)), dim3(256), 0, s, keys, n, tab, mask, w.del);
    launch_scan_u32(w.del, w.drank, n, w.partial, &w.hdr[0], s);
    if (P > 0) hipLaunchKernelGGL(k_win_addflag, dim3(blocks_for(P)), dim3(256), 0, s, w.pslot, P, tab, w.addf);
    launch_scan_u32(w.addf, w.arank, P, w.partial, &w.hdr[1], s);
    if (P > 0 && add_keys)
        hipLaunchKernelGGL(k_win_addkeys, dim3(blocks_for(P)), dim3(256), 0, s, w.addf, w.arank, w.pslot, P, tab,
                           add_keys);
    hipLaunchKernelGGL(k_win_evpos, dim3(n > 0 ? blocks_for(n) : 1), dim3(256), 0, s, w.del, w.drank, n, w.evpos,
                       w.hdr, counts);
}

void launch_window_compact(uint64_t *keys, float *rows, int R, int64_t ld, int64_t n, int64_t D,
                           const uint64_t *add_keys, const float *add_rows, int64_t A, uint64_t *evicted_keys,
                           float *evicted_rows, const WinWs &w, int32_t *status, hipStream_t s)
{
    if (status) hipLaunchKernelGGL(k_win_status, dim3(1), dim3(1), 0, s, w.hdr, n, D, status);
    if (D > 0 && (evicted_keys || evicted_rows))
        hipLaunchKernelGGL(k_win_evict, dim3(blocks_for(D)), dim3(256), 0, s, keys, rows, R, ld, n, D, w.evpos,
                           w.hdr, evicted_keys, evicted_rows);
    if (D > 0)
        hipLaunchKernelGGL(k_win_fill, dim3(blocks_for(D)), dim3(256), 0, s, keys, rows, R, ld, n, D, w.del, w.drank,
                           w.evpos, w.hdr);
    if (A > 0)
        hipLaunchKernelGGL(k_win_append, dim3(blocks_for(A)), dim3(256), 0, s, keys, rows, R, ld, n, D, add_keys,
                           add_rows, A, w.hdr);
}

}  // namespace gsl
