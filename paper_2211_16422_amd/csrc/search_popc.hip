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
#include "internal.h"

namespace homs {
namespace {

constexpr int kTile = 256;        // queries per workgroup (4 waves)
constexpr int kRefs = 32;         // reference rows per accumulator block
constexpr int kWords = 16;        // words per slice (one s_load_dwordx16 per row)
constexpr int kGroup = 2;         // rows per scalar prefetch group
constexpr int64_t kChunk = 2048;  // reference rows per workgroup

typedef __attribute__((address_space(4))) const uint32_t const_u32;

struct Slice {
    uint32_t v[kWords];
};

// 16 consecutive words at a wave-uniform address, fetched into SGPRs
__device__ __forceinline__ Slice scalar_slice(const uint32_t* p)
{
    const const_u32* q = (const const_u32*)p;
    Slice s;
#pragma unroll
    for (int i = 0; i < kWords; ++i) s.v[i] = q[i];
    return s;
}

// s_waitcnt with lgkmcnt(0) (vmcnt and expcnt left at their maxima): scalar
// loads return out of order, so only a full drain proves a group has landed
constexpr int kWaitScalar = 0xC07F;

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
    const uint32_t a = (uint32_t)a64;
    const uint32_t b = (uint32_t)min(a64 + kChunk, t_hi);

    const int64_t qs = tile * kTile + threadIdx.x;  // position in sorted order
    const bool valid = qs < nq;
    const uint32_t qi = valid ? qperm[qs] : 0u;
    uint32_t q_lo = 0, q_hi = 0;
    if (valid) {
        q_lo = (uint32_t)lo[qi];
        q_hi = (uint32_t)hi[qi];
    }
    const uint32_t* qrow = q_hv + (size_t)qi * words;

    uint32_t best_d = 0xFFFFFFFFu, best_o = 0xFFFFFFFFu;

    for (uint32_t rb = a; rb < b; rb += kRefs) {
        uint32_t acc[kRefs];
#pragma unroll
        for (int r = 0; r < kRefs; ++r) acc[r] = 0u;

        // rows past the chunk end re-read its last row; they are masked below
        Slice cur[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k)
            cur[k] = scalar_slice(lib_hv + (size_t)min(rb + (uint32_t)k, b - 1u) * words);

        for (uint32_t c = 0; c < words; c += kWords) {
            uint32_t qv[kWords];
#pragma unroll
            for (int i = 0; i < kWords; i += 4) {
                const uint4 t = *reinterpret_cast<const uint4*>(qrow + c + i);
                qv[i] = t.x;
                qv[i + 1] = t.y;
                qv[i + 2] = t.z;
                qv[i + 3] = t.w;
            }
#pragma unroll
            for (int r0 = 0; r0 < kRefs; r0 += kGroup) {
                // the current group has landed; start fetching the next one
                // (next rows of this slice, or the first rows of the next
                // slice) so its latency hides behind this group's VALU work
                __builtin_amdgcn_s_waitcnt(kWaitScalar);
                __builtin_amdgcn_sched_barrier(0);
                const bool same = r0 + kGroup < kRefs;
                const int nr = same ? r0 + kGroup : 0;
                const uint32_t nc = same ? c : (c + kWords < words ? c + kWords : c);
                Slice nxt[kGroup];
#pragma unroll
                for (int k = 0; k < kGroup; ++k)
                    nxt[k] = scalar_slice(lib_hv + (size_t)min(rb + (uint32_t)(nr + k), b - 1u) *
                                                       words + nc);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < kGroup; ++k)
#pragma unroll
                    for (int i = 0; i < kWords; ++i) acc[r0 + k] += __popc(qv[i] ^ cur[k].v[i]);
#pragma unroll
                for (int k = 0; k < kGroup; ++k) cur[k] = nxt[k];
            }
        }
        __builtin_amdgcn_s_waitcnt(kWaitScalar);

#pragma unroll
        for (int r = 0; r < kRefs; ++r) {
            const uint32_t g = rb + (uint32_t)r;
            const uint32_t gc = min(g, b - 1u);
            const uint32_t o = ((const const_u32*)lib_orig)[gc];
            const bool in = (g < b) && (g >= q_lo) && (g < q_hi);
            const uint32_t d = acc[r];
            if (in && (d < best_d || (d == best_d && o < best_o))) {
                best_d = d;
                best_o = o;
            }
        }
    }
    if (valid && best_d != 0xFFFFFFFFu)
        atomicMin(reinterpret_cast<unsigned long long*>(keys + qi),
                  ((unsigned long long)best_d << 32) | (unsigned long long)best_o);
}

__global__ void tile_bounds_kernel(int64_t nq, int64_t n_tiles, const uint32_t* __restrict__ qperm,
                                   const int64_t* __restrict__ lo, const int64_t* __restrict__ hi,
                                   int64_t* __restrict__ tile_lo, int64_t* __restrict__ tile_hi)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    int64_t mn = INT64_MAX, mx = 0;
    const int64_t end = min((t + 1) * (int64_t)kTile, nq);
    for (int64_t i = t * kTile; i < end; ++i) {
        const uint32_t q = qperm[i];
        if (hi[q] > lo[q]) {
            mn = min(mn, lo[q]);
            mx = max(mx, hi[q]);
        }
    }
    if (mn == INT64_MAX) mn = mx = 0;
    tile_lo[t] = mn;
    tile_hi[t] = mx;
}

}  // namespace

int search_popcount_tile() { return kTile; }

hipError_t launch_tile_bounds(int64_t nq, const uint32_t* qperm, const int64_t* lo,
                              const int64_t* hi, int tile, int64_t* tile_lo, int64_t* tile_hi,
                              hipStream_t s)
{
    (void)tile;
    const int64_t n_tiles = (nq + kTile - 1) / kTile;
    if (n_tiles <= 0) return hipSuccess;
    tile_bounds_kernel<<<(uint32_t)((n_tiles + 255) / 256), 256, 0, s>>>(nq, n_tiles, qperm, lo,
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
