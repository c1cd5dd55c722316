// Tile binning and the device radix sort.
//
// The paper's renderer orders each tile's Gaussians by depth (tile-based
// depth sorting, Sec. II-C).  Here the order is built in two stable passes
// that together equal one sort by the 64-bit key (tile << 32 | depth bits)
// with ties by Gaussian index:
//   1. the C*N projection records are sorted by their 32-bit depth key
//      (LSD radix, 4 passes over the records, culled records last);
//   2. every record, in that order, emits one (tile id, Gaussian index)
//      instance per overlapped tile, and the K instances are sorted by tile
//      id alone (LSD radix over only the ceil(log2 T) significant bits).
// Stability of pass 2 keeps the depth order inside each tile, so the K-sized
// sort moves 8 B per instance per pass over 1-3 passes instead of 12 B over
// 6-7 passes.
//
// Radix pass design for wave64: per 4096-key block, each wave ranks its keys
// with a ballot-based multisplit (8 ballots give the mask of lanes sharing a
// digit; the rank is the popcount of that mask below the lane), the block
// reorders its keys by digit in LDS, and writes them out in digit runs so the
// global stores are contiguous.  Digit histograms are stored digit-major
// ([256][blocks]) so one exclusive scan gives every block's output offsets.
#include "binning.hpp"

namespace gsl {

namespace {


// ------------------------------------------------------------------ fills

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}
__global__ void k_fill_f32(float *p, float v, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

inline unsigned fill_blocks(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// ------------------------------------------------------------------ scan


// Sum of each kScanTile-sized block.
// With d_n, entries at or beyond *d_n count as 0.
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                              const int64_t *__restrict__ d_n,
                                                              uint64_t *__restrict__ partial)
{
    __shared__ uint64_t s[kScanThreads / kWave];
    if (d_n && *d_n < n) n = *d_n;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t v[kScanItems];  // all loads in flight before the first add
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const int64_t j = base + (int64_t)k * kScanThreads + threadIdx.x;
        v[k] = j < n ? in[j] : 0u;
    }
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) acc += v[k];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kScanThreads / kWave; w++) t += s[w];
        partial[blockIdx.x] = t;
    }
}

// Exclusive scan of the block sums in one workgroup (four consecutive sums
// per thread, 4096 per step); writes the total.
constexpr int kPartialItems = 4;

__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t *__restrict__ partial, int64_t nb,
                                                        int64_t *__restrict__ d_total)
{
    __shared__ uint64_t s_w[1024 / kWave];
    __shared__ uint64_t s_carry;
    const int lane = threadIdx.x & 63, wv = threadIdx.x / kWave;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024 * kPartialItems) {
        const int64_t j0 = base + (int64_t)threadIdx.x * kPartialItems;
        uint64_t v[kPartialItems], sum = 0;
#pragma unroll
        for (int q = 0; q < kPartialItems; q++) {
            v[q] = j0 + q < nb ? partial[j0 + q] : 0;
            sum += v[q];
        }
        const uint64_t inc = wave_incl_scan_u64(sum, lane);
        if (lane == 63) s_w[wv] = inc;
        __syncthreads();
        uint64_t wbase = 0, tot = 0;
        for (int w = 0; w < 1024 / kWave; w++) {
            if (w < wv) wbase += s_w[w];
            tot += s_w[w];
        }
        uint64_t run = s_carry + wbase + inc - sum;
#pragma unroll
        for (int q = 0; q < kPartialItems; q++) {
            if (j0 + q < nb) partial[j0 + q] = run;
            run += v[q];
        }
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && d_total) *d_total = (int64_t)s_carry;
}

// Block-local exclusive scan plus the block's offset.  Offsets beyond 2^32
// wrap; the callers compare the 64-bit total against their capacity first.
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *__restrict__ in, int64_t n,
                                                            const int64_t *__restrict__ d_n,
                                                            const uint64_t *__restrict__ partial,
                                                            uint32_t *__restrict__ out)
{
    __shared__ uint64_t s_w[kScanThreads / kWave];
    const int64_t n_all = n;  // every position gets an offset; those at or beyond *d_n add 0
    if (d_n && *d_n < n) n = *d_n;
    const int lane = threadIdx.x & 63, wv = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // each thread owns kScanItems consecutive elements
    uint32_t v[kScanItems];
    uint64_t sum = 0;
    const int64_t mybase = base + (int64_t)threadIdx.x * kScanItems;
    for (int k = 0; k < kScanItems; k++) {
        const int64_t j = mybase + k;
        v[k] = j < n ? in[j] : 0u;
        sum += v[k];
    }
    const uint64_t inc = wave_incl_scan_u64(sum, lane);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint64_t wbase = 0;
    for (int w = 0; w < wv; w++) wbase += s_w[w];
    uint64_t run = partial[blockIdx.x] + wbase + inc - sum;
    for (int k = 0; k < kScanItems; k++) {
        const int64_t j = mybase + k;
        if (j < n_all) out[j] = (uint32_t)run;
        run += v[k];
    }
}

// ------------------------------------------------------------------ radix sort

__device__ __forceinline__ int64_t live_count(const int64_t *d_n, int64_t n_max)
{
    if (!d_n) return n_max;
    const int64_t n = *d_n;
    return n < n_max ? n : n_max;
}

// Mask of the lanes of this wave whose digit equals this lane's digit: per
// bit, the ballot of lanes with the bit set, taken as is where this lane's
// bit is set and complemented where it is clear (xnor with the bit spread
// over the word by a signed one-bit extract).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid, int db)
{
    uint64_t peers = __builtin_amdgcn_ballot_w64(valid);
    for (int b = 0; b < db; b++) {
        const uint32_t sb = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);  // 0 or all ones
        const uint64_t m = __builtin_amdgcn_ballot_w64(sb != 0u);
        const uint64_t s2 = ((uint64_t)sb << 32) | sb;
        peers &= ~(m ^ s2);
    }
    return peers;
}

// Digit histogram of one 4096-key block, digit-major output hist[d * nb + block].
// With `drop`, keys equal to kDropKey are left out (the first pass of a sort
// that also compacts).
constexpr uint32_t kDropKey = 0xffffffffu;

// With first_tiles (the first pass of the depth sort), the key of record j
// is keys[j] where first_tiles[j] > 0 and kDropKey elsewhere.
__global__ __launch_bounds__(kSortThreads) void k_rs_hist(const uint32_t *__restrict__ keys, int64_t n_max,
                                                          const int64_t *__restrict__ d_n, int shift, int db,
                                                          uint32_t *__restrict__ hist, int64_t nb, bool drop,
                                                          const int32_t *__restrict__ first_tiles,
                                                          uint32_t *__restrict__ zero_word)
{
    if (zero_word && blockIdx.x == 0 && threadIdx.x == 0) *zero_word = 0u;
    __shared__ uint32_t s_cnt[kSortThreads / kWave][256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x / kWave;
    for (int k = threadIdx.x; k < (kSortThreads / kWave) * 256; k += kSortThreads) (&s_cnt[0][0])[k] = 0;
    __syncthreads();
    const uint32_t dmask = (1u << db) - 1u;
    const int64_t n = live_count(d_n, n_max);
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)wv * (kSortTile / (kSortThreads / kWave));
    uint32_t kk[kSortItems];  // all loads in flight before the first ballot
    int32_t tt[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t j = base + (int64_t)r * kWave + lane;
        kk[r] = j < n ? keys[j] : kDropKey;
        tt[r] = (first_tiles && j < n) ? first_tiles[j] : 1;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; r++) kk[r] = tt[r] > 0 ? kk[r] : kDropKey;
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t j = base + (int64_t)r * kWave + lane;
        const uint32_t kj = kk[r];
        const bool valid = j < n && !(drop && kj == kDropKey);
        const uint32_t d = (kj >> shift) & dmask;
        // the counts do not depend on the order of the adds; a wave whose
        // keys share one digit (the top byte of depth keys, mostly) adds its
        // count once instead of 64 conflicting LDS atomics on one counter
        const uint64_t vm = __builtin_amdgcn_ballot_w64(valid);
        if (vm == 0ull) continue;
        const int first = __builtin_amdgcn_readfirstlane((int)__ffsll((unsigned long long)vm) - 1);
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, first);
        if (__builtin_amdgcn_ballot_w64(valid && d != d0) == 0ull) {
            if (lane == first) atomicAdd(&s_cnt[wv][d0], (uint32_t)__popcll(vm));
        } else if (valid) {
            atomicAdd(&s_cnt[wv][d], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < (1 << db); d += kSortThreads) {
        uint32_t t = 0;
        for (int w = 0; w < kSortThreads / kWave; w++) t += s_cnt[w][d];
        hist[(int64_t)d * nb + blockIdx.x] = t;
    }
}

// Exclusive scan of one digit's row of the digit-major histogram (workgroup
// d scans hist[d][0 .. nb)), and the row's total in totals[d].  The scatter
// adds the digit's base, the exclusive scan of the totals, itself.
constexpr int kRowItems = 4;

__global__ __launch_bounds__(256) void k_rs_rowscan(const uint32_t *__restrict__ hist, int64_t nb,
                                                    uint32_t *__restrict__ hist_off, uint32_t *__restrict__ totals)
{
    __shared__ uint32_t s_w[256 / kWave];
    __shared__ uint32_t s_carry;
    const int lane = threadIdx.x & 63, wv = threadIdx.x / kWave;
    const uint32_t *row = hist + (int64_t)blockIdx.x * nb;
    uint32_t *out = hist_off + (int64_t)blockIdx.x * nb;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 256 * kRowItems) {
        const int64_t j0 = base + (int64_t)threadIdx.x * kRowItems;
        uint32_t v[kRowItems], sum = 0;
#pragma unroll
        for (int q = 0; q < kRowItems; q++) {
            v[q] = j0 + q < nb ? row[j0 + q] : 0u;
            sum += v[q];
        }
        uint32_t inc = sum;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        if (lane == kWave - 1) s_w[wv] = inc;
        __syncthreads();
        uint32_t wbase = 0, tot = 0;
        for (int w = 0; w < 256 / kWave; w++) {
            wbase += w < wv ? s_w[w] : 0u;
            tot += s_w[w];
        }
        uint32_t run = s_carry + wbase + inc - sum;
#pragma unroll
        for (int q = 0; q < kRowItems; q++) {
            if (j0 + q < nb) out[j0 + q] = run;
            run += v[q];
        }
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = s_carry;
}

// Stable scatter of one block using the row-scanned digit-major histogram
// and the digit totals.  With d_kept (the first pass of a dropping sort),
// workgroup 0 writes the number of keys kept.
__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(const uint32_t *__restrict__ kin,
                                                             const uint32_t *__restrict__ vin,
                                                             uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                             int64_t n_max, const int64_t *__restrict__ d_n, int shift,
                                                             int db, const uint32_t *__restrict__ hist_off, int64_t nb,
                                                             const uint32_t *__restrict__ totals, bool drop,
                                                             int64_t *__restrict__ d_kept,
                                                             const int32_t *__restrict__ first_tiles,
                                                             const int32_t *__restrict__ gather_tiles,
                                                             uint32_t *__restrict__ counts_out, int pack_shift)
{
    const uint32_t dmask = (1u << db) - 1u;
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint32_t s_cnt[NW][256];   // per-wave running digit counts, then wave bases
    __shared__ uint32_t s_loc[256];       // block-local first position of each digit
    __shared__ uint32_t s_glob[256];      // digit bases, then global first position of each digit for this block
    __shared__ uint32_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t s_nloc;           // keys of this block that are kept
    const int lane = threadIdx.x & 63, wv = threadIdx.x / kWave;
    for (int k = threadIdx.x; k < NW * 256; k += kSortThreads) (&s_cnt[0][0])[k] = 0;
    if (threadIdx.x < kWave) {
        // digit bases: exclusive scan of the 256 digit totals by one wave (4 per lane)
        uint32_t t[4], sum = 0;
        for (int k = 0; k < 4; k++) {
            const int d = lane * 4 + k;
            t[k] = d <= (int)dmask ? totals[d] : 0u;
            sum += t[k];
        }
        uint32_t inc = sum;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        uint32_t run = inc - sum;
        for (int k = 0; k < 4; k++) {
            s_glob[lane * 4 + k] = run;
            run += t[k];
        }
        if (d_kept && blockIdx.x == 0 && lane == kWave - 1) *d_kept = (int64_t)run;  // every key kept
    }
    __syncthreads();
    const int64_t n = live_count(d_n, n_max);
    const int64_t block_base = (int64_t)blockIdx.x * kSortTile;
    if (block_base >= n) return;
    const int64_t base = block_base + (int64_t)wv * (kSortTile / NW);
    uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
    int32_t tt[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {  // all loads in flight before the first ballot
        const int64_t j = base + (int64_t)r * kWave + lane;
        key[r] = j < n ? kin[j] : kDropKey;
        // the first pass of the depth sort: values are the record indices
        val[r] = j < n ? (first_tiles ? (uint32_t)j : vin[j]) : 0u;
        tt[r] = (first_tiles && j < n) ? first_tiles[j] : 1;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; r++) key[r] = tt[r] > 0 ? key[r] : kDropKey;
    // with pack_shift, the record index takes the low pack_shift bits of the
    // value and the tile count the rest (all-ones: look it up)
    const uint32_t cnt_cap = pack_shift ? (0xffffffffu >> pack_shift) : 0u;
    if (first_tiles && pack_shift) {
#pragma unroll
        for (int r = 0; r < kSortItems; r++)
            val[r] |= min((uint32_t)max(tt[r], 0), cnt_cap) << pack_shift;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t j = base + (int64_t)r * kWave + lane;
        const bool valid = j < n && !(drop && key[r] == kDropKey);
        if (!valid) val[r] = 0u;
        const uint32_t d = (key[r] >> shift) & dmask;
        const uint64_t peers = digit_peers(d, valid, db);
        const uint32_t before = valid ? s_cnt[wv][d] : 0u;
        rank[r] = before + (uint32_t)__popcll(peers & lanemask_lt(lane));
        if (valid && (int)(__ffsll((unsigned long long)peers) - 1) == lane) s_cnt[wv][d] = before + __popcll(peers);
        if (!valid) rank[r] = 0xffffffffu;
    }
    __syncthreads();
    // block-local digit starts and per-wave bases
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        uint32_t run = 0;
        for (int w = 0; w < NW; w++) {
            const uint32_t c = s_cnt[w][d];
            s_cnt[w][d] = run;
            run += c;
        }
        s_loc[d] = run;  // total of digit d in this block (scanned below)
        if (d <= (int)dmask) s_glob[d] += hist_off[(int64_t)d * nb + blockIdx.x];
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        // exclusive scan of the 256 digit totals by one wave (4 per lane)
        uint32_t t[4], sum = 0;
        for (int k = 0; k < 4; k++) {
            t[k] = s_loc[lane * 4 + k];
            sum += t[k];
        }
        uint32_t inc = sum;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        uint32_t run = inc - sum;
        for (int k = 0; k < 4; k++) {
            s_loc[lane * 4 + k] = run;
            run += t[k];
        }
        if (lane == kWave - 1) s_nloc = run;
    }
    __syncthreads();
    for (int r = 0; r < kSortItems; r++) {
        if (rank[r] == 0xffffffffu) continue;
        const uint32_t d = (key[r] >> shift) & dmask;
        const uint32_t pos = s_loc[d] + s_cnt[wv][d] + rank[r];
        s_key[pos] = key[r];
        s_val[pos] = val[r];
    }
    __syncthreads();
    const int nloc = (int)s_nloc;
    for (int p = threadIdx.x; p < nloc; p += kSortThreads) {
        const uint32_t k = s_key[p];
        const uint32_t d = (k >> shift) & dmask;
        const uint32_t dst = s_glob[d] + (uint32_t)p - s_loc[d];
        kout[dst] = k;
        const uint32_t v = s_val[p];
        if (counts_out) {
            // the last pass of the depth sort: the record index, and its tile
            // count at its place in depth order
            const uint32_t idx = pack_shift ? (v & ((1u << pack_shift) - 1u)) : v;
            const uint32_t c = pack_shift ? (v >> pack_shift) : cnt_cap;
            vout[dst] = idx;
            counts_out[dst] = c != cnt_cap ? c : (uint32_t)gather_tiles[idx];
        } else {
            vout[dst] = v;
        }
    }
}

// ------------------------------------------------------------------ one-block sort

// The whole sort of n <= kOneBlockSortKeys pairs by one workgroup of 1024
// lanes.  The keys stay in registers: R per lane, R the smallest power of two
// with 1024 R >= n_max; wave w owns positions [64 R w, 64 R (w + 1)), row r
// at 64 R w + 64 r + lane, so a small sort spreads over every wave.  Each
// pass ranks them with the same ballot multisplit as the multi-block
// scatter, reorders them through LDS and reads them back in position order:
// a stable sort, so the result is the multi-block sort's, bit for bit.  The
// depth sort's extras are folded in as there (the first pass reads
// first_keys, drops records without tiles and packs each tile count beside
// its record index; the last pass unpacks them and writes counts_out), and
// with offsets_out the counts' exclusive scan and total follow; with ranges
// (the tile sort), every tile's range of positions.
constexpr int kObThreads = 1024;
constexpr int kObWaves = kObThreads / kWave;

template <int R>
__global__ __launch_bounds__(kObThreads) void k_rs_one_block(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n_max, const int64_t *__restrict__ d_n, int bits, int db, int64_t *d_kept,
    const int32_t *__restrict__ first_tiles, const int32_t *__restrict__ gather_tiles,
    uint32_t *__restrict__ counts_out, uint32_t *__restrict__ offsets_out, int64_t *__restrict__ d_total,
    int pack_shift, uint32_t *__restrict__ zero_word, uint32_t *__restrict__ ranges, int64_t T_total)
{
    constexpr int kObItems = R;
    __shared__ uint32_t s_key[kObThreads * R];
    __shared__ uint32_t s_val[kObThreads * R];
    __shared__ uint32_t s_cnt[kObWaves][256];
    __shared__ uint32_t s_loc[256];
    __shared__ uint32_t s_wsum[kObWaves];
    __shared__ uint32_t s_n;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (zero_word && threadIdx.x == 0) *zero_word = 0u;
    const uint32_t dmask = (1u << db) - 1u;
    const uint32_t cnt_cap = pack_shift ? (0xffffffffu >> pack_shift) : 0u;
    int64_t n = live_count(d_n, n_max);
    uint32_t key[kObItems], val[kObItems];
    int rank[kObItems];
#pragma unroll
    for (int r = 0; r < kObItems; r++) {
        const int64_t p = (int64_t)wv * (kObItems * kWave) + r * kWave + lane;
        key[r] = p < n ? kin[p] : kDropKey;
        val[r] = p < n ? (first_tiles ? (uint32_t)p : vin[p]) : 0u;
        if (first_tiles) {
            const int32_t t = p < n ? first_tiles[p] : 0;
            key[r] = t > 0 ? key[r] : kDropKey;
            if (pack_shift) val[r] |= min((uint32_t)max(t, 0), cnt_cap) << pack_shift;
        }
    }
    const bool drop = d_kept != nullptr;  // the first pass drops kDropKey keys
    for (int shift = 0; shift < bits; shift += db) {
        const bool first = shift == 0;
        for (int k = threadIdx.x; k < kObWaves * 256; k += kObThreads) (&s_cnt[0][0])[k] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kObItems; r++) {
            const int64_t p = (int64_t)wv * (kObItems * kWave) + r * kWave + lane;
            const bool valid = p < n && !(drop && first && key[r] == kDropKey);
            const uint32_t d = (key[r] >> shift) & dmask;
            const uint64_t peers = digit_peers(d, valid, db);
            const uint32_t before = valid ? s_cnt[wv][d] : 0u;
            rank[r] = valid ? (int)(before + (uint32_t)__popcll(peers & lanemask_lt(lane))) : -1;
            if (valid && (int)(__ffsll((unsigned long long)peers) - 1) == lane) s_cnt[wv][d] = before + __popcll(peers);
        }
        __syncthreads();
        if (threadIdx.x < 256) {
            const int d = threadIdx.x;
            uint32_t run = 0;
            for (int w = 0; w < kObWaves; w++) {
                const uint32_t c = s_cnt[w][d];
                s_cnt[w][d] = run;
                run += c;
            }
            s_loc[d] = run;
        }
        __syncthreads();
        if (threadIdx.x < kWave) {
            // exclusive scan of the 256 digit totals (4 per lane)
            uint32_t t[4], sum = 0;
            for (int k = 0; k < 4; k++) {
                t[k] = s_loc[lane * 4 + k];
                sum += t[k];
            }
            uint32_t inc = sum;
            for (int off = 1; off < kWave; off <<= 1) {
                const uint32_t o = __shfl_up(inc, off, kWave);
                if (lane >= off) inc += o;
            }
            uint32_t run = inc - sum;
            for (int k = 0; k < 4; k++) {
                s_loc[lane * 4 + k] = run;
                run += t[k];
            }
            if (lane == kWave - 1) s_n = run;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kObItems; r++) {
            if (rank[r] < 0) continue;
            const uint32_t d = (key[r] >> shift) & dmask;
            const uint32_t pos = s_loc[d] + s_cnt[wv][d] + (uint32_t)rank[r];
            s_key[pos] = key[r];
            s_val[pos] = val[r];
        }
        __syncthreads();
        n = s_n;  // the kept keys (all of them after the first pass)
        if (first && d_kept && threadIdx.x == 0) *d_kept = n;
#pragma unroll
        for (int r = 0; r < kObItems; r++) {
            const int64_t p = (int64_t)wv * (kObItems * kWave) + r * kWave + lane;
            key[r] = p < n ? s_key[p] : kDropKey;
            val[r] = p < n ? s_val[p] : 0u;
        }
        __syncthreads();
    }
    // out, in position order (the last pass left it in LDS and in registers)
    uint32_t cnt[kObItems];
#pragma unroll
    for (int r = 0; r < kObItems; r++) {
        const int64_t p = (int64_t)wv * (kObItems * kWave) + r * kWave + lane;
        cnt[r] = 0u;
        if (p >= n) continue;
        kout[p] = key[r];
        if (counts_out) {
            const uint32_t idx = pack_shift ? (val[r] & ((1u << pack_shift) - 1u)) : val[r];
            const uint32_t c = pack_shift ? (val[r] >> pack_shift) : cnt_cap;
            cnt[r] = c != cnt_cap ? c : (uint32_t)gather_tiles[idx];
            vout[p] = idx;
            counts_out[p] = cnt[r];
        } else {
            vout[p] = val[r];
        }
    }
    if (ranges) {
        // the tile sort: every tile's first and one-past-last position (empty
        // tiles [0, 0)), from the sorted keys still in LDS.  A live count above
        // n_max (the instances overflowed their capacity and were never
        // emitted) leaves every tile empty, so nothing reads those keys' ids.
        for (int64_t t = threadIdx.x; t < 2 * T_total; t += kObThreads) ranges[t] = 0u;
        __syncthreads();
        const bool overflow = d_n && *d_n > n_max;
#pragma unroll
        for (int r = 0; r < kObItems; r++) {
            if (overflow) break;
            const int64_t p = (int64_t)wv * (kObItems * kWave) + r * kWave + lane;
            if (p >= n || (int64_t)key[r] >= T_total) continue;  // never trust an id as an index
            if (p == 0 || s_key[p - 1] != key[r]) ranges[2 * (int64_t)key[r]] = (uint32_t)p;
            if (p == n - 1 || s_key[p + 1] != key[r]) ranges[2 * (int64_t)key[r] + 1] = (uint32_t)(p + 1);
        }
    }
    if (!offsets_out) return;
    // exclusive scan of the counts in position order: a wave's rows in turn,
    // then the waves' totals
    uint32_t run = 0;
    uint32_t excl[kObItems];
#pragma unroll
    for (int r = 0; r < kObItems; r++) {
        uint32_t inc = cnt[r];
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        excl[r] = run + inc - cnt[r];
        run += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) s_wsum[wv] = run;
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (int w = 0; w < kObWaves; w++) {
        base += w < wv ? s_wsum[w] : 0u;
        total += s_wsum[w];
    }
#pragma unroll
    for (int r = 0; r < kObItems; r++) {
        const int64_t p = (int64_t)wv * (kObItems * kWave) + r * kWave + lane;
        if (p < n_max) offsets_out[p] = p < n ? base + excl[r] : total;
    }
    if (d_total && threadIdx.x == 0) *d_total = (int64_t)total;
}

// ------------------------------------------------------------------ binning

// The listed records, one per workgroup of 256 lanes (grid-stride over the
// list): 256 bbox tiles per step in row-major order, a hit's slot from the
// ballots of the four waves, so the instances come out exactly as the
// wave-wide walk would write them.  Counting: list entries are record
// indices m.  Emitting: list entries are depth-order positions j.
template <bool emit>
__global__ __launch_bounds__(256) void k_tiles_big(const gsl_binrec *__restrict__ binrecs,
                                                   const DevCam *__restrict__ cams, int N, int tile,
                                                   const uint32_t *__restrict__ big_list,
                                                   const uint32_t *__restrict__ big_n, int32_t *__restrict__ tiles,
                                                   const uint32_t *__restrict__ order,
                                                   const uint32_t *__restrict__ offsets,
                                                   const uint32_t *__restrict__ counts,
                                                   const int64_t *__restrict__ d_K, int64_t capacity,
                                                   uint32_t *__restrict__ tile_ids, uint32_t *__restrict__ gauss_ids)
{
    __shared__ uint32_t s_cnt[4];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (emit && *d_K > capacity) return;  // uniform: nothing was counted into place
    const uint32_t nbig = *big_n;
    for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const uint32_t entry = big_list[b];
        const uint32_t m = emit ? order[entry] : entry;
        const uint32_t base = emit ? offsets[entry] : 0u, limit = emit ? counts[entry] : 0u;
        const gsl_binrec s = binrecs[m];
        const uint32_t c = m / (uint32_t)N;
        const uint32_t gid = m - c * (uint32_t)N;
        const DevCam &cam = cams[c];
        const EllipseTest e = ellipse_test(s);
        const int tx0 = s.x0 / tile, ty0 = s.y0 / tile;
        const int nx = s.x1 / tile - tx0 + 1;
        const uint32_t nt = (uint32_t)bbox_tiles(s, tile);
        uint32_t run = 0;
        for (uint32_t t0 = 0; t0 < nt; t0 += 256) {
            const uint32_t t = t0 + threadIdx.x;
            bool hit = false;
            uint32_t bands = 0;
            int tx = 0, ty = 0;
            if (t < nt) {
                ty = ty0 + (int)(t / (uint32_t)nx);
                tx = tx0 + (int)(t - (uint32_t)(ty - ty0) * (uint32_t)nx);
                hit = tile_hit(e, cam.W, cam.H, tile, tx, ty, emit ? &bands : nullptr);
            }
            const uint64_t mask = __ballot(hit);
            if (lane == 0) s_cnt[wv] = (uint32_t)__popcll(mask);
            __syncthreads();
            uint32_t before = run, tot = 0;
            for (int k = 0; k < 4; k++) {
                before += k < wv ? s_cnt[k] : 0u;
                tot += s_cnt[k];
            }
            if (emit && hit) {
                const uint32_t slot = before + (uint32_t)__popcll(mask & lanemask_lt(lane));
                if (slot < limit) {  // never beyond the record's counted range
                    tile_ids[base + slot] = (uint32_t)(cam.tile_offset + ty * cam.tiles_x + tx);
                    gauss_ids[base + slot] = gid | (bands << kGidBits);
                }
            }
            run += tot;
            __syncthreads();
        }
        if (!emit && threadIdx.x == 0) tiles[m] = (int32_t)run;
    }
}

// One (tile, Gaussian | bands) instance per reached tile, records in depth order.
__global__ __launch_bounds__(256) void k_emit(const uint32_t *__restrict__ order, const uint32_t *__restrict__ offsets,
                                              const uint32_t *__restrict__ counts,
                                              const gsl_binrec *__restrict__ binrecs,
                                              const DevCam *__restrict__ cams, int N, int64_t M, int tile,
                                              const int64_t *__restrict__ d_K, int64_t capacity,
                                              uint32_t *__restrict__ tile_ids, uint32_t *__restrict__ gauss_ids,
                                              int32_t *__restrict__ d_status, uint32_t *__restrict__ big_list,
                                              uint32_t *__restrict__ big_n, const int64_t *__restrict__ d_V)
{
    __shared__ RecTiles rec[256];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t K = *d_K;
    if (j == 0) *d_status = K > capacity ? GSL_ECAPACITY : GSL_OK;
    if (K > capacity) return;  // uniform: every thread reads the same K
    const int64_t V = *d_V;    // records kept by the depth sort (the positions beyond carry no count)
    uint32_t nt = 0, cnt = 0, m = 0, off = 0;
    gsl_binrec s;
    if (j < V) {
        // three independent loads first (order[j] is only used where cnt != 0)
        cnt = counts[j];
        m = order[j];
        off = offsets[j];
        if (cnt) {
            s = binrecs[m];
            nt = (uint32_t)bbox_tiles(s, tile);
            if (nt > kBigTiles) {
                push_big(big_list, big_n, (uint32_t)j);
                nt = 0;
            }
        }
    }
    const uint32_t incl = (uint32_t)wave_incl_scan_u64(nt, lane), excl = incl - nt;
    const int wave0 = threadIdx.x & ~(kWave - 1);
    const int slot = rec_slot(nt, lane);
    if (nt) {
        const uint32_t c = m / (uint32_t)N;
        rec_fill(rec[wave0 + slot], s, cams[c], tile, m - c * (uint32_t)N, off, cnt, excl);
    }
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    __syncthreads();
    expand_tiles<true>(rec + wave0, lane, excl, incl, total, tile, tile_ids, gauss_ids);
}

// Four consecutive positions per thread: the ids at k0-1 .. k0+4 (a sentinel
// outside [0, K), never equal to a valid id) mark where runs start and end.
constexpr int kRangeItems = 4;

__global__ void k_ranges(const uint32_t *__restrict__ tile_ids, const int64_t *__restrict__ d_K, int64_t capacity,
                         int64_t T_total, uint32_t *__restrict__ ranges)
{
    constexpr uint32_t kNone = 0xffffffffu;
    const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeItems;
    const int64_t K = *d_K;
    if (K > capacity) return;
    if (k0 >= K) return;
    uint32_t t[kRangeItems + 2];
    t[0] = k0 > 0 ? tile_ids[k0 - 1] : kNone;
    if (k0 + kRangeItems <= K && (reinterpret_cast<uintptr_t>(tile_ids) & 15u) == 0) {
        const uint4 v = *reinterpret_cast<const uint4 *>(tile_ids + k0);
        t[1] = v.x;
        t[2] = v.y;
        t[3] = v.z;
        t[4] = v.w;
    } else {
#pragma unroll
        for (int q = 0; q < kRangeItems; q++) t[1 + q] = k0 + q < K ? tile_ids[k0 + q] : kNone;
    }
    t[kRangeItems + 1] = k0 + kRangeItems < K ? tile_ids[k0 + kRangeItems] : kNone;
#pragma unroll
    for (int q = 0; q < kRangeItems; q++) {
        const uint32_t cur = t[1 + q];
        if ((int64_t)cur >= T_total) continue;  // never trust an id as an index (also skips positions >= K)
        const int64_t k = k0 + q;
        if (t[q] != cur) ranges[2 * (int64_t)cur] = (uint32_t)k;
        if (t[q + 2] != cur) ranges[2 * (int64_t)cur + 1] = (uint32_t)(k + 1);
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_f32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

void launch_scan_u32(const uint32_t *counts, uint32_t *offsets, int64_t n, uint64_t *partial, int64_t *d_total,
                     hipStream_t s, const int64_t *d_n)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        if (d_total) launch_fill_f64(reinterpret_cast<double *>(d_total), 0.0, 1, s);  // all-zero bits == int64 0
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, n, d_n, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partial, nb, d_total);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, n, d_n, partial, offsets);
}

int launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2, int64_t n_max,
                      const int64_t *d_n, int bits, uint32_t *hist, uint32_t *hist_off, uint32_t *totals,
                      hipStream_t s, int64_t *d_kept, const DepthSortIO *io, uint32_t *ranges, int64_t T_total)
{
    const int64_t nb = (n_max + kSortTile - 1) / kSortTile;
    if (nb == 0 || bits <= 0) {
        if (d_kept) launch_fill_f64(reinterpret_cast<double *>(d_kept), 0.0, 1, s);  // all-zero bits == int64 0
        if (io && io->zero_word) launch_fill_u32(io->zero_word, 0u, 1, s);
        return 0;
    }
    uint32_t *kin = keys, *vin = vals, *kout = keys2, *vout = vals2;
    const uint32_t *kin0 = io ? io->first_keys : keys;  // the first pass reads its keys from here
    if (radix_one_block(n_max)) {
        const int passes1 = (bits + 7) / 8, db1 = (bits + passes1 - 1) / passes1;
        int ps = 0;
        if (io && io->counts_out) {
            int ib = 1;
            while (ib < 32 && ((uint64_t)1 << ib) < (uint64_t)n_max) ib++;
            if (ib <= 28) ps = ib;
        }
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(1), dim3(kObThreads), 0, s, kin0, vals, keys2, vals2, n_max, d_n, bits, db1,
                               d_kept, io ? io->first_tiles : nullptr, io ? io->gather_tiles : nullptr,
                               io ? io->counts_out : nullptr, io ? io->offsets_out : nullptr,
                               io ? io->d_total : nullptr, ps, io ? io->zero_word : nullptr, ranges, T_total);
        };
        if (n_max <= kObThreads) go(k_rs_one_block<1>);
        else if (n_max <= 2 * kObThreads) go(k_rs_one_block<2>);
        else if (n_max <= 4 * kObThreads) go(k_rs_one_block<4>);
        else if (n_max <= 8 * kObThreads) go(k_rs_one_block<8>);
        else go(k_rs_one_block<16>);
        return 1;
    }
    int where = 0;
    // as few passes of at most 8 bits as cover `bits`, the digits split evenly
    // (fewer buckets per pass write longer runs)
    const int passes = (bits + 7) / 8, db = (bits + passes - 1) / passes;
    // the depth sort's values carry the tile counts in their free high bits
    // when the record indices leave at least four
    int pack_shift = 0;
    if (io && io->counts_out) {
        int ib = 1;
        while (ib < 32 && ((uint64_t)1 << ib) < (uint64_t)n_max) ib++;
        if (ib <= 28) pack_shift = ib;
    }
    for (int shift = 0; shift < bits; shift += db) {
        // with d_kept the first pass drops kDropKey keys and counts the rest
        const bool drop = d_kept && shift == 0;
        const bool first = shift == 0, last = shift + db >= bits;
        const uint32_t *kp = first ? kin0 : kin;
        const int32_t *ft = (io && first) ? io->first_tiles : nullptr;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, kp, n_max, d_n, shift, db, hist,
                           nb, drop, ft, (io && first) ? io->zero_word : nullptr);
        hipLaunchKernelGGL(k_rs_rowscan, dim3(1u << db), dim3(256), 0, s, hist, nb, hist_off, totals);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, kp, vin, kout, vout, n_max,
                           d_n, shift, db, hist_off, nb, totals, drop, drop ? d_kept : nullptr, ft,
                           (io && last) ? io->gather_tiles : nullptr, (io && last) ? io->counts_out : nullptr,
                           pack_shift);
        if (drop) d_n = d_kept;
        uint32_t *tk = kin, *tv = vin;
        kin = kout; vin = vout;
        kout = tk; vout = tv;
        where ^= 1;
    }
    return where;
}

void launch_count_big(const gsl_binrec *binrecs, const DevCam *cams, const Layout &L, int32_t *tiles_touched,
                      uint32_t *big_list, uint32_t *big_n, hipStream_t s)
{
    if (L.M == 0) return;
    hipLaunchKernelGGL((k_tiles_big<false>), dim3(kBigBlocks), dim3(256), 0, s, binrecs, cams, L.N, L.tile, big_list,
                       big_n, tiles_touched, nullptr, nullptr, nullptr, nullptr, (int64_t)0, nullptr, nullptr);
}

void launch_emit(const uint32_t *order, const uint32_t *offsets, const uint32_t *counts, const gsl_binrec *binrecs,
                 const DevCam *cams, const Layout &L, const int64_t *d_K, int64_t capacity, uint32_t *tile_ids,
                 uint32_t *gauss_ids, int32_t *d_status, uint32_t *big_list, uint32_t *big_n, const int64_t *d_V,
                 hipStream_t s)
{
    const int64_t blocks = L.M > 0 ? (L.M + 255) / 256 : 1;
    // *big_n is zero here: the depth sort's first histogram pass cleared it
    hipLaunchKernelGGL(k_emit, dim3((unsigned)blocks), dim3(256), 0, s, order, offsets, counts, binrecs, cams, L.N,
                       L.M, L.tile, d_K, capacity, tile_ids, gauss_ids, d_status, big_list, big_n, d_V);
    if (L.M > 0)
        hipLaunchKernelGGL((k_tiles_big<true>), dim3(kBigBlocks), dim3(256), 0, s, binrecs, cams, L.N, L.tile,
                           big_list, big_n, nullptr, order, offsets, counts, d_K, capacity, tile_ids, gauss_ids);
}

void launch_ranges(const uint32_t *tile_ids, const int64_t *d_K, int64_t capacity, int64_t T_total,
                   uint32_t *ranges, hipStream_t s)
{
    launch_fill_u32(ranges, 0u, 2 * T_total, s);
    if (capacity > 0)
        hipLaunchKernelGGL(k_ranges, dim3((unsigned)((capacity + 256 * kRangeItems - 1) / (256 * kRangeItems))),
                           dim3(256), 0, s, tile_ids, d_K, capacity, T_total, ranges);
}

}  // namespace gsl
