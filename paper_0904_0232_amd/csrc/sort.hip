// Stable cell sort of the particle slots and compaction of the removed ones.
// Key = rank(tile) T^3 + the cell's place in its tile, with (i,j,k) = floor(x)
// (FP64) or the packed cell (FP32-mixed), tiles of T^3 cells ranked along a
// path of face-adjacent tiles and cells in layers across the path
// (tile_key); removed particles take the all-ones key of key_bits bits and
// so sort to the end.
//
// The ordering is a least-significant-digit radix sort over digits of at most
// 9 bits (ceil(key_bits / 9) passes, 3 at 256^3).  Each pass is
//   upsweep:   per tile of 4096 slots, a histogram of the digit in LDS,
//              written digit-major, counts[d * ntiles + tile];
//   scan:      one exclusive scan over that array gives, for every (digit,
//              tile), where the tile's elements of that digit start;
//   downsweep: the tile re-reads its keys and ranks each element among the
//              earlier elements of its digit (wave ballots give the rank
//              inside 64 slots, a wave-private count table in LDS the rank
//              across the wave's rounds, a prefix over the waves the rank in
//              the tile), stages the tile in LDS in digit order and writes it
//              out, so consecutive lanes write consecutive addresses.
// Ranks follow slot order within a tile and tiles follow slot order within a
// digit, so every pass is stable, and the whole sort equals a stable sort on
// the key.  A last kernel moves the particle records (the SoA gather) in
// output order.  No pass waits on another block, and every loop is bounded
// by the tile.
#include "grpic_dev.h"
#include "grpic_impl.h"

namespace grpic {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;  // slots per tile
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kSortMaxBits = 9;
constexpr int kSortMaxBins = 1 << kSortMaxBits;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kSortBlock * kScanItems;  // scan entries per block
constexpr int kScanTopBlock = 1024;

struct SortPlan {
    int passes;
    int shift[4];
    int bits[4];
};

// Digits of at most 9 bits, as even as possible, low digits first.
SortPlan sort_plan(int key_bits) {
    SortPlan P;
    P.passes = (key_bits + kSortMaxBits - 1) / kSortMaxBits;
    if (P.passes < 1) P.passes = 1;
    const int base = key_bits / P.passes, extra = key_bits % P.passes;
    int sh = 0;
    for (int p = 0; p < P.passes; p++) {
        P.bits[p] = base + (p < extra ? 1 : 0);
        P.shift[p] = sh;
        sh += P.bits[p];
    }
    return P;
}

int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

size_t sort_temp_bytes(int64_t capacity) {
    const int64_t entries = (int64_t)kSortMaxBins * sort_tiles(capacity > 0 ? capacity : 1);
    const int64_t chunks = (entries + kScanChunk - 1) / kScanChunk;
    return (size_t)(entries + chunks + 64) * 4;
}

// ---------------------------------------------------------------------------
// Keys.  The first block also resets the live count, which the last pass
// lowers to the position of the first removed particle.

// Tiles ranked along a boustrophedon path (planes tz in order, rows ty
// reversed in odd planes, tiles tx reversed in odd rows), so consecutive
// tiles share a face.  Inside a tile the cells go in layers across the
// direction in which the path leaves it (along the row; at a row's end to
// the next row; at a plane's end to the next plane), from the face it
// entered by to the face it leaves by; inside a layer the lower remaining
// axis runs fastest.  So the last layer of a tile and the first layer of the
// next one are neighbours, and a block of consecutive sorted particles that
// spans two tiles covers two or three thin layers instead of both tiles.
__device__ __forceinline__ uint32_t tile_key(int T, int nTx, int nTy, const int c[3]) {
    const int tx = c[0] / T, ty = c[1] / T, tz = c[2] / T;
    const int lx = c[0] - tx * T, ly = c[1] - ty * T, lz = c[2] - tz * T;
    const int in_plane = (tz & 1) ? nTy - 1 - ty : ty;
    const int row = tz * nTy + in_plane;
    const int along = (row & 1) ? nTx - 1 - tx : tx;
    int layer, slow, fast;
    if (along < nTx - 1) {  // leaves along x
        layer = (row & 1) ? T - 1 - lx : lx;
        slow = lz;
        fast = ly;
    } else if (in_plane < nTy - 1) {  // leaves to the next row, along y
        layer = (tz & 1) ? T - 1 - ly : ly;
        slow = lz;
        fast = lx;
    } else {  // leaves to the next plane, along z
        layer = lz;
        slow = ly;
        fast = lx;
    }
    return ((uint32_t)row * (uint32_t)nTx + (uint32_t)along) * (uint32_t)(T * T * T) +
           (uint32_t)((layer * T + slow) * T + fast);
}

// Key of slot id (every slot below n); slot 0 also resets the live count.
__device__ __forceinline__ void sort_key_slot(const Grid &G, int T, int nTx, int nTy, uint32_t sentinel,
                                              const ParticlePtrs &in, int64_t n, uint32_t *__restrict__ keys,
                                              unsigned long long *counters, int64_t id) {
    if (id == 0) counters[C_NALIVE] = (unsigned long long)n;
    if (id >= n) return;
    if (in.sp[id] == kDead) {
        keys[id] = sentinel;
        return;
    }
    int c[3];
    for (int ax = 0; ax < 3; ax++) {
        const int ci = (int)floor(in.x[ax][id]);
        const int nn = G.dim(ax);
        c[ax] = ci < 0 ? 0 : (ci > nn - 1 ? nn - 1 : ci);
    }
    keys[id] = tile_key(T, nTx, nTy, c);
}

__device__ __forceinline__ void sort_key_slot32(const Grid &G, int T, int nTx, int nTy, uint32_t sentinel,
                                                const ParticlePtrs32 &in, int64_t n, uint32_t *__restrict__ keys,
                                                unsigned long long *counters, int64_t id) {
    if (id == 0) counters[C_NALIVE] = (unsigned long long)n;
    if (id >= n) return;
    if (in.sp[id] == kDead) {
        keys[id] = sentinel;
        return;
    }
    int c[3];
    unpack_cell(in.cell[id], c[0], c[1], c[2]);
    for (int ax = 0; ax < 3; ax++) {
        const int nn = G.dim(ax);
        c[ax] = c[ax] < 0 ? 0 : (c[ax] > nn - 1 ? nn - 1 : c[ax]);
    }
    keys[id] = tile_key(T, nTx, nTy, c);
}

__global__ void k_sort_keys(Grid G, int T, int nTx, int nTy, uint32_t sentinel, ParticlePtrs in, int64_t n,
                            uint32_t *__restrict__ keys, unsigned long long *counters) {
    sort_key_slot(G, T, nTx, nTy, sentinel, in, n, keys, counters, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void k_sort_keys32(Grid G, int T, int nTx, int nTy, uint32_t sentinel, ParticlePtrs32 in, int64_t n,
                              uint32_t *__restrict__ keys, unsigned long long *counters) {
    sort_key_slot32(G, T, nTx, nTy, sentinel, in, n, keys, counters, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Upsweep: digit histogram of one tile.

// Digit histogram of tile t.  hist: kSortMaxBins LDS entries.  Every thread
// of the block calls it; the caller orders earlier uses of hist before it.
__device__ __forceinline__ void upsweep_tile(const uint32_t *__restrict__ keys, int64_t n, int shift, int bits,
                                             int64_t ntiles, uint32_t *__restrict__ counts, int64_t t,
                                             uint32_t *hist) {
    const int R = 1 << bits;
    for (int d = threadIdx.x; d < R; d += kSortBlock) hist[d] = 0u;
    __syncthreads();
    const int64_t base = t * kSortTile;
    uint32_t k[kSortItems];
#pragma unroll
    for (int q = 0; q < kSortItems; q++) {
        const int64_t i = base + q * kSortBlock + threadIdx.x;
        k[q] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kSortItems; q++)
        if (base + q * kSortBlock + threadIdx.x < n) atomicAdd(&hist[(k[q] >> shift) & (uint32_t)(R - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += kSortBlock) counts[(int64_t)d * ntiles + t] = hist[d];
}

__global__ __launch_bounds__(kSortBlock) void k_sort_upsweep(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                              int bits, int64_t ntiles, uint32_t *__restrict__ counts) {
    __shared__ uint32_t hist[kSortMaxBins];
    upsweep_tile(keys, n, shift, bits, ntiles, counts, blockIdx.x, hist);
}

// ---------------------------------------------------------------------------
// Exclusive scan of m uint32 entries in place (the totals fit 32 bits: they
// sum to the slot count).  Chunks of kScanChunk entries: chunk sums, a scan
// of the sums in one block, then each chunk scanned from its base.

// Exclusive scan of one value per thread over the block; *total receives
// the block's sum.  Every thread of the block calls it.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[kScanTopBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int k = 0; k < nw; k++) {
        const uint32_t s = wsum[k];
        if (k < w) before += s;
        all += s;
    }
    __syncthreads();  // wsum may be reused by the next call
    *total = all;
    return before + x - v;
}

// Sum of chunk c of a[0, m).
__device__ __forceinline__ void scan_reduce_chunk(const uint32_t *__restrict__ a, int64_t m,
                                                  uint32_t *__restrict__ sums, int64_t c) {
    const int64_t base = c * kScanChunk;
    uint32_t s = 0;
    for (int q = 0; q < kScanItems; q++) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + q;
        if (i < m) s += a[i];
    }
    uint32_t total;
    (void)block_exclusive_scan(s, &total);
    if (threadIdx.x == 0) sums[c] = total;
}

// Exclusive scan of the nchunks chunk sums by one block.
__device__ __forceinline__ void scan_top_sums(uint32_t *__restrict__ sums, int64_t nchunks) {
    const int64_t per = (nchunks + blockDim.x - 1) / blockDim.x;
    const int64_t lo = (int64_t)threadIdx.x * per;
    uint32_t s = 0;
    for (int64_t i = lo; i < lo + per && i < nchunks; i++) s += sums[i];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, &total);
    for (int64_t i = lo; i < lo + per && i < nchunks; i++) {
        const uint32_t v = sums[i];
        sums[i] = run;
        run += v;
    }
}

// Chunk c of a[0, m) scanned in place from its base sums[c].
__device__ __forceinline__ void scan_down_chunk(uint32_t *__restrict__ a, int64_t m,
                                                const uint32_t *__restrict__ sums, int64_t c) {
    const int64_t base = c * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; q++) {
        v[q] = base + q < m ? a[base + q] : 0u;
        s += v[q];
    }
    uint32_t total;
    uint32_t run = sums[c] + block_exclusive_scan(s, &total);
#pragma unroll
    for (int q = 0; q < kScanItems; q++) {
        if (base + q < m) a[base + q] = run;
        run += v[q];
    }
}

__global__ __launch_bounds__(kSortBlock) void k_scan_reduce(const uint32_t *__restrict__ a, int64_t m,
                                                            uint32_t *__restrict__ sums) {
    scan_reduce_chunk(a, m, sums, blockIdx.x);
}

// One block of kScanTopBlock threads: exclusive scan of the chunk sums.
__global__ __launch_bounds__(kScanTopBlock) void k_scan_top(uint32_t *__restrict__ sums, int64_t nchunks) {
    scan_top_sums(sums, nchunks);
}

__global__ __launch_bounds__(kSortBlock) void k_scan_down(uint32_t *__restrict__ a, int64_t m,
                                                          const uint32_t *__restrict__ sums) {
    scan_down_chunk(a, m, sums, blockIdx.x);
}

void launch_scan(uint32_t *a, int64_t m, uint32_t *sums, hipStream_t s) {
    const int64_t nchunks = (m + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nchunks), dim3(kSortBlock), 0, s, a, m, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTopBlock), 0, s, sums, nchunks);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nchunks), dim3(kSortBlock), 0, s, a, m, sums);
}

// ---------------------------------------------------------------------------
// Downsweep.  Out writes one element to its sorted position (PassOut: the
// key and value arrays of the next pass).

struct PassOut {
    uint32_t *keys, *vals;
    __device__ __forceinline__ void operator()(int64_t dest, uint32_t key, uint32_t val) const {
        keys[dest] = key;
        vals[dest] = val;
    }
};

// The particle records in sorted order: out[i] = in[idx[i]].  Reads follow
// the output order, which for particles sorted a few steps earlier is close
// to the input order, so they stay nearly coalesced.
__device__ __forceinline__ void gather_slot(const ParticlePtrs &in, const ParticlePtrs &out,
                                            const uint32_t *__restrict__ idx, int64_t n, int64_t i) {
    if (i >= n) return;
    const uint32_t s = idx[i];
    for (int q = 0; q < 3; q++) out.x[q][i] = in.x[q][s];
    for (int q = 0; q < 4; q++) out.u[q][i] = in.u[q][s];
    out.sp[i] = in.sp[s];
}

__device__ __forceinline__ void gather_slot32(const ParticlePtrs32 &in, const ParticlePtrs32 &out,
                                              const uint32_t *__restrict__ idx, int64_t n, int64_t i) {
    if (i >= n) return;
    const uint32_t s = idx[i];
    out.cell[i] = in.cell[s];
    for (int q = 0; q < 3; q++) out.off[q][i] = in.off[q][s];
    for (int q = 0; q < 4; q++) out.u[q][i] = in.u[q][s];
    out.sp[i] = in.sp[s];
}

__global__ void k_sort_gather(ParticlePtrs in, ParticlePtrs out, const uint32_t *__restrict__ idx, int64_t n) {
    gather_slot(in, out, idx, n, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void k_sort_gather32(ParticlePtrs32 in, ParticlePtrs32 out, const uint32_t *__restrict__ idx, int64_t n) {
    gather_slot32(in, out, idx, n, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// FIRST: the values are the slot indices (not read).  LAST: lower the live
// count to the sorted position of the first removed particle.
//
// Wave w ranks the tile's slots [w * kSortTile / 4, (w + 1) * kSortTile / 4)
// in rounds of 64 consecutive slots against its own count table: the lanes
// of one digit (wave ballots) read the table entry, and the lowest of them
// adds their number.  LDS instructions of one wave complete in order, so no
// barrier is needed inside the rounds; one barrier, then per digit a prefix
// over the four waves and a scan over the digits place every element.
struct DownLds {
    uint32_t key[kSortTile];
    uint32_t val[kSortTile];
    uint32_t start[kSortMaxBins];            // where each digit starts in the staged tile
    uint32_t goff[kSortMaxBins];             // where the tile's digit starts in the output
    uint16_t wc[kSortWaves][kSortMaxBins];   // per-wave counts, then per-wave prefixes
};

// Tile t of one pass.  Every thread of the block calls it; the caller orders
// earlier uses of L before it.
template <bool FIRST, bool LAST, class Out>
__device__ __forceinline__ void downsweep_tile(const uint32_t *__restrict__ keys_in,
                                               const uint32_t *__restrict__ vals_in, int64_t n, int shift, int bits,
                                               int64_t ntiles, const uint32_t *__restrict__ offsets, const Out &out,
                                               uint32_t sentinel, unsigned long long *counters, int64_t t,
                                               DownLds &L) {
    constexpr int kWaveSpan = kSortTile / kSortWaves;  // slots ranked by one wave
    uint32_t *s_key = L.key, *s_val = L.val, *s_start = L.start, *s_goff = L.goff;
    uint16_t(*s_wc)[kSortMaxBins] = L.wc;
    const int R = 1 << bits, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t mask = (uint32_t)(R - 1);
    const int64_t base = t * kSortTile;
    const int tile_n = (int)(n - base < kSortTile ? n - base : kSortTile);
    for (int d = tid; d < R; d += kSortBlock) {
        s_goff[d] = offsets[(int64_t)d * ntiles + t];
        for (int k = 0; k < kSortWaves; k++) s_wc[k][d] = 0;
    }
    uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
    for (int q = 0; q < kSortItems; q++) {
        const int l = w * kWaveSpan + q * 64 + lane;
        const bool valid = l < tile_n;
        key[q] = valid ? keys_in[base + l] : 0u;
        val[q] = valid ? (FIRST ? (uint32_t)(base + l) : vals_in[base + l]) : 0u;
    }
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int q = 0; q < kSortItems; q++) {
        const bool valid = w * kWaveSpan + q * 64 + lane < tile_n;
        const uint32_t d = (key[q] >> shift) & mask;
        // lanes of this wave with the same digit
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < bits; b++) {
            const bool on = (d >> b) & 1u;
            const unsigned long long bal = __ballot(on);
            peers &= on ? bal : ~bal;
        }
        const unsigned long long lower = peers & below;
        const uint32_t before = valid ? (uint32_t)s_wc[w][d] : 0u;
        rank[q] = before + (uint32_t)__popcll(lower);
        if (valid && lower == 0ull) s_wc[w][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
    }
    __syncthreads();
    // per digit: the waves' prefixes and the tile's count; then the digits'
    // starts in the staged tile (exclusive scan over the digits)
    {
        uint32_t c[2] = {0u, 0u};
        for (int h = 0; h < 2; h++) {
            const int d = 2 * tid + h;
            if (d < R) {
                uint32_t run = 0;
                for (int k = 0; k < kSortWaves; k++) {
                    const uint32_t v = s_wc[k][d];
                    s_wc[k][d] = (uint16_t)run;
                    run += v;
                }
                c[h] = run;
            }
        }
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(c[0] + c[1], &total);
        if (2 * tid < R) s_start[2 * tid] = ex;
        if (2 * tid + 1 < R) s_start[2 * tid + 1] = ex + c[0];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSortItems; q++) {
        if (w * kWaveSpan + q * 64 + lane < tile_n) {
            const uint32_t d = (key[q] >> shift) & mask;
            const uint32_t pos = s_start[d] + s_wc[w][d] + rank[q];
            s_key[pos] = key[q];
            s_val[pos] = val[q];
        }
    }
    __syncthreads();
    for (int l = tid; l < tile_n; l += kSortBlock) {
        const uint32_t k = s_key[l];
        const uint32_t d = (k >> shift) & mask;
        const int64_t dest = (int64_t)s_goff[d] + (int64_t)(l - (int)s_start[d]);
        out(dest, k, s_val[l]);
        if (LAST && k == sentinel && (l == 0 || s_key[l - 1] != sentinel))
            atomicMin(&counters[C_NALIVE], (unsigned long long)dest);
    }
}

template <bool FIRST, bool LAST, class Out>
__global__ __launch_bounds__(kSortBlock) void k_sort_downsweep(const uint32_t *__restrict__ keys_in,
                                                                const uint32_t *__restrict__ vals_in, int64_t n,
                                                                int shift, int bits, int64_t ntiles,
                                                                const uint32_t *__restrict__ offsets, Out out,
                                                                uint32_t sentinel, unsigned long long *counters) {
    __shared__ DownLds L;
    downsweep_tile<FIRST, LAST, Out>(keys_in, vals_in, n, shift, bits, ntiles, offsets, out, sentinel, counters,
                                     blockIdx.x, L);
}

// The passes over the keys; returns where the sorted keys and the original
// slot of each sorted position are.
void run_passes(int64_t n, int key_bits, uint32_t *keys, uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt,
                void *temp, uint32_t sentinel, unsigned long long *counters, uint32_t **final_keys,
                uint32_t **final_idx, hipStream_t s) {
    const SortPlan P = sort_plan(key_bits);
    const int64_t ntiles = sort_tiles(n);
    uint32_t *counts = (uint32_t *)temp;
    uint32_t *sums = counts + (int64_t)kSortMaxBins * ntiles;
    uint32_t *kin = keys, *vin = nullptr, *kout = keys_alt, *vout = idx_alt;
    for (int p = 0; p < P.passes; p++) {
        const int R = 1 << P.bits[p];
        hipLaunchKernelGGL(k_sort_upsweep, dim3((unsigned)ntiles), dim3(kSortBlock), 0, s, kin, n, P.shift[p],
                           P.bits[p], ntiles, counts);
        launch_scan(counts, (int64_t)R * ntiles, sums, s);
        const bool first = p == 0, last = p == P.passes - 1;
        PassOut po{kout, vout};
        if (first && last)
            hipLaunchKernelGGL((k_sort_downsweep<true, true, PassOut>), dim3((unsigned)ntiles), dim3(kSortBlock), 0, s,
                               kin, vin, n, P.shift[p], P.bits[p], ntiles, counts, po, sentinel, counters);
        else if (first)
            hipLaunchKernelGGL((k_sort_downsweep<true, false, PassOut>), dim3((unsigned)ntiles), dim3(kSortBlock), 0,
                               s, kin, vin, n, P.shift[p], P.bits[p], ntiles, counts, po, sentinel, counters);
        else if (last)
            hipLaunchKernelGGL((k_sort_downsweep<false, true, PassOut>), dim3((unsigned)ntiles), dim3(kSortBlock), 0,
                               s, kin, vin, n, P.shift[p], P.bits[p], ntiles, counts, po, sentinel, counters);
        else
            hipLaunchKernelGGL((k_sort_downsweep<false, false, PassOut>), dim3((unsigned)ntiles), dim3(kSortBlock), 0,
                               s, kin, vin, n, P.shift[p], P.bits[p], ntiles, counts, po, sentinel, counters);
        // the next pass reads what this one wrote and writes the pair this
        // one read (pass 0 read keys, with implicit values: idx is free)
        uint32_t *nk = kin, *nv = kin == keys ? idx : idx_alt;
        kin = kout;
        vin = vout;
        kout = nk;
        vout = nv;
    }
    *final_keys = kin;
    *final_idx = vin;
}

void launch_sort(const Grid &G, int tile, int64_t n, ParticlePtrs in, ParticlePtrs out, uint32_t *keys,
                 uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, int key_bits, bool keep,
                 uint32_t **final_keys, uint32_t **final_idx, unsigned long long *counters, hipStream_t s) {
    if (n <= 0) return;
    const int nTx = (G.nx + tile - 1) / tile, nTy = (G.ny + tile - 1) / tile;
    const uint32_t sentinel = key_bits >= 32 ? 0xFFFFFFFFu : ((1u << key_bits) - 1u);
    hipLaunchKernelGGL(k_sort_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, tile, nTx, nTy, sentinel,
                       in, n, keys, counters);
    uint32_t *fk, *fi;
    run_passes(n, key_bits, keys, keys_alt, idx, idx_alt, temp, sentinel, counters, &fk, &fi, s);
    hipLaunchKernelGGL(k_sort_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, fi, n);
    if (final_keys) *final_keys = keep ? fk : nullptr;
    if (final_idx) *final_idx = keep ? fi : nullptr;
}

void launch_sort32(const Grid &G, int tile, int64_t n, ParticlePtrs32 in, ParticlePtrs32 out, uint32_t *keys,
                   uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, int key_bits, bool keep,
                   uint32_t **final_keys, uint32_t **final_idx, unsigned long long *counters, hipStream_t s) {
    if (n <= 0) return;
    const int nTx = (G.nx + tile - 1) / tile, nTy = (G.ny + tile - 1) / tile;
    const uint32_t sentinel = key_bits >= 32 ? 0xFFFFFFFFu : ((1u << key_bits) - 1u);
    hipLaunchKernelGGL(k_sort_keys32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, tile, nTx, nTy,
                       sentinel, in, n, keys, counters);
    uint32_t *fk, *fi;
    run_passes(n, key_bits, keys, keys_alt, idx, idx_alt, temp, sentinel, counters, &fk, &fi, s);
    hipLaunchKernelGGL(k_sort_gather32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, fi, n);
    if (final_keys) *final_keys = keep ? fk : nullptr;
    if (final_idx) *final_idx = keep ? fi : nullptr;
}

// ---------------------------------------------------------------------------
// Serving batch: the sorts of every run that falls due in an iteration, as
// persistent launches over the logical blocks of those runs (slots in blocks
// of kSortBlock, tiles, scan chunks), captured with the rest of the
// iteration.  The bodies are the ones above, so a run sorts exactly as alone.

void batch_sort_job(const Grid &G, int tile, int64_t n, ParticlePtrs32 in, ParticlePtrs32 out, uint32_t *keys,
                    uint32_t *keys_alt, uint32_t *idx, uint32_t *idx_alt, void *temp, int key_bits, BatchSort &J) {
    J = BatchSort{};
    if (n <= 0) return;
    const SortPlan P = sort_plan(key_bits);
    J.n = n;
    J.ntiles = sort_tiles(n);
    J.tile = tile;
    J.nTx = (G.nx + tile - 1) / tile;
    J.nTy = (G.ny + tile - 1) / tile;
    J.sentinel = key_bits >= 32 ? 0xFFFFFFFFu : ((1u << key_bits) - 1u);
    J.passes = P.passes;
    int widest = 0;
    J.counts = (uint32_t *)temp;
    J.sums = J.counts + (int64_t)kSortMaxBins * J.ntiles;
    // the ping-pong of run_passes
    uint32_t *kin = keys, *vin = nullptr, *kout = keys_alt, *vout = idx_alt;
    for (int p = 0; p < P.passes; p++) {
        J.shift[p] = P.shift[p];
        J.bits[p] = P.bits[p];
        widest = P.bits[p] > widest ? P.bits[p] : widest;
        J.kin[p] = kin;
        J.vin[p] = vin;
        J.kout[p] = kout;
        J.vout[p] = vout;
        uint32_t *nk = kin, *nv = kin == keys ? idx : idx_alt;
        kin = kout;
        vin = vout;
        kout = nk;
        vout = nv;
    }
    J.final_idx = vin;
    J.nchunks = (((int64_t)1 << widest) * J.ntiles + kScanChunk - 1) / kScanChunk;
    J.in = in;
    J.out = out;
}

int64_t batch_sort_blocks(int kind, const BatchSort &J) {
    if (J.n <= 0) return 0;
    switch (kind) {
    case BK_SORT_SLOT: return (J.n + kSortBlock - 1) / kSortBlock;
    case BK_SORT_TILE: return J.ntiles;
    case BK_SORT_SCAN: return J.nchunks;
    }
    return 0;
}

namespace {

__device__ __forceinline__ int64_t scan_entries(const BatchSort &J, int p) {
    return ((int64_t)1 << J.bits[p]) * J.ntiles;
}

__global__ __launch_bounds__(kSortBlock) void k_batch_sort_keys32(const BatchTable *__restrict__ T) {
    const int64_t total = T->total[BK_SORT_SLOT];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        const BatchRun32 &R = T->run[batch_run_of(T, BK_SORT_SLOT, lb)];
        const BatchSort &J = R.sort;
        sort_key_slot32(R.G, J.tile, J.nTx, J.nTy, J.sentinel, J.in, J.n, J.kin[0], R.counters,
                        (lb - R.off[BK_SORT_SLOT]) * kSortBlock + threadIdx.x);
    }
}

__global__ __launch_bounds__(kSortBlock) void k_batch_sort_upsweep(const BatchTable *__restrict__ T, int p) {
    __shared__ uint32_t hist[kSortMaxBins];
    const int64_t total = T->total[BK_SORT_TILE];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        const BatchRun32 &R = T->run[batch_run_of(T, BK_SORT_TILE, lb)];
        const BatchSort &J = R.sort;
        if (p >= J.passes) continue;  // the same for the whole block
        __syncthreads();              // the previous tile is done with hist
        upsweep_tile(J.kin[p], J.n, J.shift[p], J.bits[p], J.ntiles, J.counts, lb - R.off[BK_SORT_TILE], hist);
    }
}

__global__ __launch_bounds__(kSortBlock) void k_batch_scan_reduce(const BatchTable *__restrict__ T, int p) {
    const int64_t total = T->total[BK_SORT_SCAN];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        const BatchRun32 &R = T->run[batch_run_of(T, BK_SORT_SCAN, lb)];
        const BatchSort &J = R.sort;
        if (p >= J.passes) continue;
        const int64_t m = scan_entries(J, p), c = lb - R.off[BK_SORT_SCAN];
        if (c * kScanChunk >= m) continue;
        scan_reduce_chunk(J.counts, m, J.sums, c);
    }
}

// One block per run.
__global__ __launch_bounds__(kScanTopBlock) void k_batch_scan_top(const BatchTable *__restrict__ T, int p) {
    for (int r = blockIdx.x; r < T->nruns; r += gridDim.x) {
        const BatchSort &J = T->run[r].sort;
        if (J.n <= 0 || p >= J.passes) continue;
        const int64_t m = scan_entries(J, p);
        scan_top_sums(J.sums, (m + kScanChunk - 1) / kScanChunk);
    }
}

__global__ __launch_bounds__(kSortBlock) void k_batch_scan_down(const BatchTable *__restrict__ T, int p) {
    const int64_t total = T->total[BK_SORT_SCAN];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        const BatchRun32 &R = T->run[batch_run_of(T, BK_SORT_SCAN, lb)];
        const BatchSort &J = R.sort;
        if (p >= J.passes) continue;
        const int64_t m = scan_entries(J, p), c = lb - R.off[BK_SORT_SCAN];
        if (c * kScanChunk >= m) continue;
        scan_down_chunk(J.counts, m, J.sums, c);
    }
}

template <bool FIRST>
__global__ __launch_bounds__(kSortBlock) void k_batch_sort_downsweep(const BatchTable *__restrict__ T, int p) {
    __shared__ DownLds L;
    const int64_t total = T->total[BK_SORT_TILE];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        const BatchRun32 &R = T->run[batch_run_of(T, BK_SORT_TILE, lb)];
        const BatchSort &J = R.sort;
        if (p >= J.passes) continue;
        __syncthreads();  // the previous tile is done with L
        const PassOut po{J.kout[p], J.vout[p]};
        const int64_t t = lb - R.off[BK_SORT_TILE];
        if (p == J.passes - 1)
            downsweep_tile<FIRST, true, PassOut>(J.kin[p], J.vin[p], J.n, J.shift[p], J.bits[p], J.ntiles, J.counts,
                                                 po, J.sentinel, R.counters, t, L);
        else
            downsweep_tile<FIRST, false, PassOut>(J.kin[p], J.vin[p], J.n, J.shift[p], J.bits[p], J.ntiles, J.counts,
                                                  po, J.sentinel, R.counters, t, L);
    }
}

__global__ __launch_bounds__(kSortBlock) void k_batch_sort_gather32(const BatchTable *__restrict__ T) {
    const int64_t total = T->total[BK_SORT_SLOT];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        const BatchRun32 &R = T->run[batch_run_of(T, BK_SORT_SLOT, lb)];
        const BatchSort &J = R.sort;
        gather_slot32(J.in, J.out, J.final_idx, J.n, (lb - R.off[BK_SORT_SLOT]) * kSortBlock + threadIdx.x);
    }
}

// Persistent grids: 8 blocks per compute unit, 3 for the downsweep (40 KiB
// of LDS each), one block per run for the scan of the chunk sums.
constexpr int kBatchSortGrid = 256 * 8;
constexpr int kBatchDownGrid = 256 * 3;

}  // namespace

void launch_batch_sort(const BatchTable *table, int passes, hipStream_t s) {
    if (passes <= 0) return;
    hipLaunchKernelGGL(k_batch_sort_keys32, dim3(kBatchSortGrid), dim3(kSortBlock), 0, s, table);
    for (int p = 0; p < passes; p++) {
        hipLaunchKernelGGL(k_batch_sort_upsweep, dim3(kBatchSortGrid), dim3(kSortBlock), 0, s, table, p);
        hipLaunchKernelGGL(k_batch_scan_reduce, dim3(kBatchSortGrid), dim3(kSortBlock), 0, s, table, p);
        hipLaunchKernelGGL(k_batch_scan_top, dim3(kMaxBatchRuns), dim3(kScanTopBlock), 0, s, table, p);
        hipLaunchKernelGGL(k_batch_scan_down, dim3(kBatchSortGrid), dim3(kSortBlock), 0, s, table, p);
        if (p == 0)
            hipLaunchKernelGGL(k_batch_sort_downsweep<true>, dim3(kBatchDownGrid), dim3(kSortBlock), 0, s, table, p);
        else
            hipLaunchKernelGGL(k_batch_sort_downsweep<false>, dim3(kBatchDownGrid), dim3(kSortBlock), 0, s, table, p);
    }
    hipLaunchKernelGGL(k_batch_sort_gather32, dim3(kBatchSortGrid), dim3(kSortBlock), 0, s, table);
}

}  // namespace grpic
