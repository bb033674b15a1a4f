// Open-window Hamming top-1 search with XOR + population count (Section 3.4;
// the bit-packed representation and popcount similarity of Section 4.1).
//
// Work decomposition. Queries are ordered by (charge, precursor m/z) and cut
// into tiles of 256; neighbouring queries share almost all of their
// candidates, so a tile's candidates are one contiguous range of the sorted
// library (the union of its queries' windows, a few rows wider than any one
// window). The range is cut into chunks of kChunk rows; one workgroup of
// four waves handles one (tile, chunk) pair, every lane owning one query.
//
// Inner loop. A wave walks its chunk kRefs rows at a time. For each block of
// kWords words of the packed vectors the lane loads that slice of its own
// query into VGPRs, and every reference row slice is fetched with scalar
// loads (the row index is wave-uniform, so one s_load_dwordx16 feeds all 64
// queries of the wave through SGPR operands). Each 32-bit word then costs
// exactly two VALU instructions per (query, reference) pair: v_xor_b32 and
// v_bcnt_u32_b32 (population count with accumulate) into a per-reference
// accumulator. The wave's four-wave workgroup walks the same rows, so the
// scalar cache serves one fetch of a row to all 256 queries of the tile.
// Scalar loads are software-pipelined two rows ahead: without it every row
// waits out a full scalar-load round trip and the kernel sits near 70% of
// the VALU issue rate; with it, above 90%.
//
// Selection. After a block's distances are complete each lane keeps the
// lexicographic minimum of (distance, library index) over rows inside its
// own window [lo, hi); the lane's minimum is merged into the query's 64-bit
// key (distance << 32 | library index) with one global atomicMin.
#include "popcount_tile.h"

namespace homs {
namespace {

using namespace popc;

__global__ __launch_bounds__(kTile) void search_popcount_kernel(
    uint32_t words, int64_t nq, const uint32_t* __restrict__ q_hv,
    const uint32_t* __restrict__ qperm, const int64_t* __restrict__ lo,
    const int64_t* __restrict__ hi, const int64_t* __restrict__ tile_lo,
    const int64_t* __restrict__ tile_hi, const uint32_t* __restrict__ lib_hv,
    const uint32_t* __restrict__ lib_orig, uint64_t* __restrict__ keys)
{
    const int64_t tile = blockIdx.x;
    const int64_t t_lo = tile_lo[tile];
    const int64_t t_hi = tile_hi[tile];
    const int64_t a64 = t_lo + (int64_t)blockIdx.y * kChunk;
    if (a64 >= t_hi) return;  // this tile's range has fewer chunks
    popcount_tile_rows(words, nq, q_hv, qperm, lo, hi, tile, (uint32_t)a64,
                       (uint32_t)min(a64 + kChunk, t_hi), lib_hv, lib_orig, keys);
}

__global__ void tile_bounds_kernel(int64_t nq, int64_t n_tiles, int tile,
                                   const uint32_t* __restrict__ qperm,
                                   const int64_t* __restrict__ lo, const int64_t* __restrict__ hi,
                                   int64_t* __restrict__ tile_lo, int64_t* __restrict__ tile_hi)
{
    // one wave per tile: lanes stride over its queries, then a wave reduction
    const int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (t >= n_tiles) return;  // wave-uniform
    int64_t mn = INT64_MAX, mx = 0;
    const int64_t end = min((t + 1) * (int64_t)tile, nq);
    for (int64_t i = t * tile + l; i < end; i += 64) {
        const uint32_t q = qperm[i];
        const int64_t a = lo[q], b = hi[q];
        if (b > a) {
            mn = min(mn, a);
            mx = max(mx, b);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mn = min(mn, (int64_t)__shfl_xor((long long)mn, off));
        mx = max(mx, (int64_t)__shfl_xor((long long)mx, off));
    }
    if (l == 0) {
        if (mn == INT64_MAX) mn = mx = 0;
        tile_lo[t] = mn;
        tile_hi[t] = mx;
    }
}

}  // namespace

int search_popcount_tile() { return kTile; }

hipError_t launch_tile_bounds(int64_t nq, const uint32_t* qperm, const int64_t* lo,
                              const int64_t* hi, int tile, int64_t* tile_lo, int64_t* tile_hi,
                              hipStream_t s)
{
    const int64_t n_tiles = (nq + tile - 1) / tile;
    if (n_tiles <= 0) return hipSuccess;
    tile_bounds_kernel<<<(uint32_t)((n_tiles + 3) / 4), 256, 0, s>>>(nq, n_tiles, tile, qperm, lo,
                                                                     hi, tile_lo, tile_hi);
    return hipGetLastError();
}

hipError_t launch_search_popcount(const homs_ctx* c, int64_t nq, const uint32_t* q_hv,
                                  const uint32_t* qperm, const int64_t* lo, const int64_t* hi,
                                  const int64_t* tile_lo, const int64_t* tile_hi,
                                  const TilePlan& plan, uint64_t* keys, hipStream_t s)
{
    (void)plan;
    const int64_t n_tiles = (nq + kTile - 1) / kTile;
    if (n_tiles <= 0 || c->lib.n <= 0) return hipSuccess;
    const int64_t max_chunks = (c->lib.n + kChunk - 1) / kChunk;
    if (max_chunks > 65535) return hipErrorInvalidConfiguration;
    search_popcount_kernel<<<dim3((uint32_t)n_tiles, (uint32_t)max_chunks), kTile, 0, s>>>(
        c->words, nq, q_hv, qperm, lo, hi, tile_lo, tile_hi, c->lib.hv, c->lib.orig, keys);
    return hipGetLastError();
}

}  // namespace homs
