// Device prefix sums and a stable LSD radix sort of (64-bit key, 32-bit
// value) pairs.
//
// The library is ordered by (charge, precursor m/z, library index) so that a
// query's candidates (same charge, precursor m/z within the tolerance;
// Section 3.4) are one contiguous run of rows, and queries are ordered by
// (charge, precursor m/z) so that neighbouring queries share candidate
// ranges. Both orders come from the radix sort below; the CSR offsets of the
// device preprocessing (Section 3.2) come from the exclusive scan.
//
// Scan: reduce-then-scan over 4096-element tiles (256 threads x 16 items):
// per-tile totals, one workgroup scanning the totals in chunks with a running
// carry, then each tile scanned through LDS with wave shuffles and offset by
// its total's prefix. Any n in [0, 2^31) takes three launches.
//
// Radix sort: 8-bit digits, least significant first, one pass per digit:
// count (per tile, per digit), exclusive scan of the digit-major count table
// (digit d of tile t lands at d * tiles + t, so the scan gives every tile the
// global position of its first item of each digit), scatter. Within a tile
// the items are taken in rounds of 256 in input order; lanes of a wave that
// carry the same digit find each other with eight ballots (one per digit
// bit), rank themselves by the lanes below them, and the per-wave counts of a
// round are turned into per-wave bases in LDS. Every pass is therefore stable
// and deterministic, and so is the whole sort.
#include "internal.h"

namespace homs {
namespace {

constexpr int kThreads = 256;  // 4 waves
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // 4096 elements per tile
constexpr int kRadix = 256;
constexpr int kWaves = kThreads / 64;

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
inline int64_t tiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive scan of one value per thread across the workgroup; *total gets
// the sum of all values. s_wave: kWaves entries of LDS.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* s_wave, T* total)
{
    const T incl = wave_inclusive_scan(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) s_wave[w] = incl;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        const T x = s_wave[i];
        if (i < w) base += x;
        tot += x;
    }
    __syncthreads();  // s_wave may be rewritten by the caller's next scan
    *total = tot;
    return base + incl - v;
}

// tile totals (in may alias the scan's output; it is read before any write)
template <typename T>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const T* __restrict__ in, int64_t n,
                                                               T* __restrict__ sums)
{
    __shared__ T s_wave[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int64_t j = base + i * kThreads + threadIdx.x;
        if (j < n) acc += in[j];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int i = 0; i < kWaves; ++i) t += s_wave[i];
        sums[blockIdx.x] = t;
    }
}

// Scans `n` elements of one tile-sized chunk at `src` into `dst` (may alias)
// with exclusive prefix `carry`; returns the chunk's total (every thread).
// s_tile: kTile elements of LDS.
template <typename T>
__device__ __forceinline__ T scan_chunk(const T* src, T* dst, int64_t n, T carry,
                                        T* s_tile, T* s_wave)
{
    // coalesced load into LDS, then each thread scans 16 consecutive elements
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int j = i * kThreads + threadIdx.x;
        s_tile[j] = (j < n) ? src[j] : (T)0;
    }
    __syncthreads();
    T* mine = s_tile + threadIdx.x * kItems;
    T run = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const T v = mine[i];
        mine[i] = run;
        run += v;
    }
    T total;
    const T base = block_exclusive_scan(run, s_wave, &total) + carry;
#pragma unroll
    for (int i = 0; i < kItems; ++i) mine[i] += base;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int j = i * kThreads + threadIdx.x;
        if (j < n) dst[j] = s_tile[j];
    }
    __syncthreads();  // s_tile is reused by the next chunk
    return total;
}

// one workgroup: exclusive scan of the tile totals, chunk by chunk
template <typename T>
__global__ __launch_bounds__(kThreads) void scan_top_kernel(T* __restrict__ sums, int64_t n)
{
    __shared__ T s_tile[kTile];
    __shared__ T s_wave[kWaves];
    T carry = 0;
    for (int64_t b = 0; b < n; b += kTile) {
        const int64_t m = (n - b) < kTile ? (n - b) : kTile;
        carry += scan_chunk<T>(sums + b, sums + b, m, carry, s_tile, s_wave);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scan_down_kernel(const T* in, int64_t n,
                                                             const T* __restrict__ offs, T* out)
{
    __shared__ T s_tile[kTile];
    __shared__ T s_wave[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int64_t m = (n - base) < kTile ? (n - base) : kTile;
    (void)scan_chunk<T>(in + base, out + base, m, offs[blockIdx.x], s_tile, s_wave);
}

// lanes of the calling wave whose `valid` flag is set and whose digit equals
// this lane's (all lanes of the wave must call it together)
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t set = __ballot(bit);
        m &= bit ? set : ~set;
    }
    return m;
}

__device__ __forceinline__ uint64_t lanes_below()
{
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// per tile and digit: number of items; counts are digit-major
__global__ __launch_bounds__(kThreads) void radix_count_kernel(const uint64_t* __restrict__ keys,
                                                               int64_t n, int shift,
                                                               uint32_t* __restrict__ counts,
                                                               int64_t tiles)
{
    __shared__ uint32_t s_cnt[kWaves][kRadix];
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s_cnt[i][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const uint64_t below = lanes_below();
    for (int r = 0; r < kItems; ++r) {
        const int64_t j = base + r * kThreads + t;
        const bool valid = j < n;
        const uint32_t d = valid ? (uint32_t)(keys[j] >> shift) & (kRadix - 1) : 0u;
        const uint64_t peers = digit_peers(d, valid);
        // the lowest lane of each digit group adds the group's size (each
        // wave owns its own counters, so no two lanes add to one at once)
        if (valid && (peers & below) == 0) s_cnt[w][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    counts[(int64_t)t * tiles + blockIdx.x] = s_cnt[0][t] + s_cnt[1][t] + s_cnt[2][t] + s_cnt[3][t];
}

// stable scatter of one tile to the positions given by the scanned counts
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, int64_t n, int shift,
    const uint32_t* __restrict__ offs, int64_t tiles, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout)
{
    __shared__ uint32_t s_next[kRadix];               // next free position per digit
    __shared__ uint32_t s_wave[2][kWaves][kRadix];    // per-wave counts, then bases (by round parity)
    const int t = threadIdx.x, w = t >> 6;
    s_next[t] = offs[(int64_t)t * tiles + blockIdx.x];
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s_wave[0][i][t] = 0;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const uint64_t below = lanes_below();
    __syncthreads();
    for (int r = 0; r < kItems; ++r) {
        uint32_t(*cur)[kRadix] = s_wave[r & 1];
        uint32_t(*nxt)[kRadix] = s_wave[(r & 1) ^ 1];
        const int64_t j = base + r * kThreads + t;
        const bool valid = j < n;
        const uint64_t k = valid ? kin[j] : 0ull;
        const uint32_t v = valid ? vin[j] : 0u;
        const uint32_t d = (uint32_t)(k >> shift) & (kRadix - 1);
        const uint64_t peers = digit_peers(d, valid);
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0) cur[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        // every read of the other buffer (the previous round's scatter) came
        // before this barrier and the next round writes it only after the
        // next one: clear it now
#pragma unroll
        for (int i = 0; i < kWaves; ++i) nxt[i][t] = 0;
        {  // thread t owns digit t: counts of the four waves -> their bases
            const uint32_t c0 = cur[0][t], c1 = cur[1][t], c2 = cur[2][t], c3 = cur[3][t];
            const uint32_t b = s_next[t];
            cur[0][t] = b;
            cur[1][t] = b + c0;
            cur[2][t] = b + c0 + c1;
            cur[3][t] = b + c0 + c1 + c2;
            s_next[t] = b + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = cur[w][d] + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
    }
}

}  // namespace

size_t scan_temp_bytes(int64_t n) { return al((size_t)(tiles_of(n) > 0 ? tiles_of(n) : 1) * 8); }

template <typename T>
hipError_t exclusive_scan(const T* in, T* out, int64_t n, void* temp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t tiles = tiles_of(n);
    T* sums = (T*)temp;
    scan_reduce_kernel<T><<<(uint32_t)tiles, kThreads, 0, s>>>(in, n, sums);
    scan_top_kernel<T><<<1, kThreads, 0, s>>>(sums, tiles);
    scan_down_kernel<T><<<(uint32_t)tiles, kThreads, 0, s>>>(in, n, sums, out);
    return hipGetLastError();
}

template hipError_t exclusive_scan<uint32_t>(const uint32_t*, uint32_t*, int64_t, void*,
                                             hipStream_t);
template hipError_t exclusive_scan<int64_t>(const int64_t*, int64_t*, int64_t, void*,
                                            hipStream_t);

size_t radix_sort_temp_bytes(int64_t n)
{
    const int64_t cells = (int64_t)kRadix * (tiles_of(n) > 0 ? tiles_of(n) : 1);
    return al((size_t)cells * 4) + scan_temp_bytes(cells);
}

hipError_t radix_sort_pairs(int64_t n, uint64_t* keys, uint64_t* keys_alt, uint32_t* vals,
                            uint32_t* vals_alt, int begin_bit, int end_bit, void* temp,
                            hipStream_t s, bool* in_alt)
{
    *in_alt = false;
    if (n <= 0 || begin_bit >= end_bit) return hipSuccess;
    if (n > 0xFFFFFFFFll || begin_bit < 0 || end_bit > 64 || (end_bit - begin_bit) % 8 != 0)
        return hipErrorInvalidValue;
    const int64_t tiles = tiles_of(n);
    const int64_t cells = (int64_t)kRadix * tiles;
    uint32_t* counts = (uint32_t*)temp;
    void* scan_tmp = (char*)temp + al((size_t)cells * 4);
    uint64_t *ki = keys, *ko = keys_alt;
    uint32_t *vi = vals, *vo = vals_alt;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        radix_count_kernel<<<(uint32_t)tiles, kThreads, 0, s>>>(ki, n, shift, counts, tiles);
        hipError_t e = exclusive_scan<uint32_t>(counts, counts, cells, scan_tmp, s);
        if (e != hipSuccess) return e;
        radix_scatter_kernel<<<(uint32_t)tiles, kThreads, 0, s>>>(ki, vi, n, shift, counts, tiles,
                                                                  ko, vo);
        std::swap(ki, ko);
        std::swap(vi, vo);
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

}  // namespace homs
