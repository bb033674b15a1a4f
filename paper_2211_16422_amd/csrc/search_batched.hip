// Batched search of a mixed query stream (narrow ppm and open Da windows,
// Table 1) in one persistent launch.
//
// A batch mixes windows of a few dozen candidates with windows of a million.
// Queries are split by window size: a "wide" query (more than
// cfg.narrow_max candidates) goes into 256-query tiles that share one
// candidate range, scored with the XOR + popcount tile code of the plain
// search; a "narrow" query is scored by one wave with one candidate row per
// lane. Both kinds become work items of one queue: items [0, W) are
// (wide tile, row chunk) pairs, items [W, W + N) are groups of narrow
// queries. A persistent grid of workgroups pulls items with an atomic
// counter until the queue is empty, so every wave reaches the exit.
//
// Everything between the inputs and the outputs is device work with a fixed
// launch shape (no host synchronisation, no memset or copy nodes, no library
// sort), so the whole batch can be captured once in a hipGraph and replayed:
//   window bounds -> bucket histogram -> scan -> scatter (counting sort by
//   (wide/narrow, charge, precursor bucket)) -> plan -> reset keys ->
//   persistent search -> finalize.
#include "mfma_direct.h"
#include "popcount_tile.h"

namespace homs {
namespace {

constexpr int kThreads = 256;
constexpr int kScanBlock = 1024;          // elements per first-level scan block
constexpr int kCharges = 16;              // charges 0..15 get buckets; others clamp
constexpr int kPmzBuckets = 8192;         // precursor buckets of cfg width each
constexpr int kClassBuckets = kCharges * kPmzBuckets;
constexpr int kBuckets = 2 * kClassBuckets;  // wide first, then narrow

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + kThreads - 1) / kThreads); }

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_u64_kernel(uint64_t* __restrict__ p, int64_t n, uint64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// bucket of every query: (narrow?, charge, floor(pmz / width)), clamped
__global__ void bucket_kernel(int64_t nq, const double* __restrict__ q_pmz,
                              const int8_t* __restrict__ q_charge, bool use_charge,
                              const int64_t* __restrict__ lo, const int64_t* __restrict__ hi,
                              uint32_t narrow_max, double inv_width,
                              uint32_t* __restrict__ bucket, uint32_t* __restrict__ hist)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const bool narrow = (hi[q] - lo[q]) <= (int64_t)narrow_max;
    int c = use_charge ? (int)q_charge[q] : 0;
    c = c < 0 ? 0 : (c >= kCharges ? kCharges - 1 : c);
    const double x = q_pmz[q] * inv_width;
    int p = (x >= 0.0) ? (x < (double)(kPmzBuckets - 1) ? (int)x : kPmzBuckets - 1) : 0;
    const uint32_t bkt = (narrow ? kClassBuckets : 0) + (uint32_t)(c * kPmzBuckets + p);
    bucket[q] = bkt;
    atomicAdd(hist + bkt, 1u);
}

// exclusive scan, level 1: each block scans kScanBlock entries in place and
// records its total
__global__ __launch_bounds__(kThreads) void scan_blocks_kernel(uint32_t* __restrict__ a, int64_t n,
                                                               uint32_t* __restrict__ block_sums)
{
    __shared__ uint32_t s[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    for (int i = threadIdx.x; i < kScanBlock; i += kThreads)
        s[i] = (base + i < n) ? a[base + i] : 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < kScanBlock; ++i) {
            const uint32_t v = s[i];
            s[i] = run;
            run += v;
        }
        block_sums[blockIdx.x] = run;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kScanBlock; i += kThreads)
        if (base + i < n) a[base + i] = s[i];
}

// level 2: one thread scans the block totals; level 3 adds them back
__global__ void scan_sums_kernel(uint32_t* __restrict__ sums, int64_t n)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t run = 0;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t v = sums[i];
        sums[i] = run;
        run += v;
    }
}

__global__ void scan_add_kernel(uint32_t* __restrict__ a, int64_t n,
                                const uint32_t* __restrict__ block_sums)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += block_sums[i / kScanBlock];
}

// counting-sort scatter; the order inside a bucket is arbitrary and results
// do not depend on it (keys merge with atomicMin)
__global__ void scatter_kernel(int64_t nq, const uint32_t* __restrict__ bucket,
                               uint32_t* __restrict__ cursor, uint32_t* __restrict__ order)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const uint32_t pos = atomicAdd(cursor + bucket[q], 1u);
    order[pos] = (uint32_t)q;
}

struct Plan {
    uint32_t n_wide;       // wide queries occupy order[0, n_wide)
    uint32_t wide_items;   // (tile, chunk) items
    uint32_t total_items;  // wide items + narrow groups
    uint32_t next_item;    // queue head
};

// One workgroup: wide-tile candidate ranges, their chunk counts and the
// item prefix, and the queue counters. After the scatter, the cursor of the
// last wide bucket has advanced to the first narrow position, i.e. n_wide.
__global__ __launch_bounds__(1024) void plan_kernel(
    int64_t nq, const uint32_t* __restrict__ cursor, const uint32_t* __restrict__ order,
    const int64_t* __restrict__ lo, const int64_t* __restrict__ hi, uint32_t chunk_rows,
    uint32_t narrow_group, int64_t max_tiles, int64_t* __restrict__ tile_lo,
    int64_t* __restrict__ tile_hi, uint32_t* __restrict__ tile_item, Plan* __restrict__ plan)
{
    __shared__ uint32_t s_nwide;
    __shared__ uint32_t s_part[1024];
    if (threadIdx.x == 0) s_nwide = cursor[kClassBuckets - 1];
    __syncthreads();
    const uint32_t n_wide = s_nwide;
    const int64_t n_tiles = (n_wide + popc::kTile - 1) / popc::kTile;
    // per tile: candidate range union and number of chunks
    for (int64_t t = threadIdx.x; t < max_tiles; t += blockDim.x) {
        int64_t mn = INT64_MAX, mx = 0;
        if (t < n_tiles) {
            const int64_t end = min((t + 1) * (int64_t)popc::kTile, (int64_t)n_wide);
            for (int64_t i = t * popc::kTile; i < end; ++i) {
                const uint32_t q = order[i];
                if (hi[q] > lo[q]) {
                    mn = min(mn, lo[q]);
                    mx = max(mx, hi[q]);
                }
            }
        }
        if (mn == INT64_MAX) mn = mx = 0;
        tile_lo[t] = mn;
        tile_hi[t] = mx;
        tile_item[t] = (uint32_t)((mx - mn + chunk_rows - 1) / chunk_rows);
    }
    __syncthreads();
    // exclusive prefix of chunk counts: contiguous segment per thread
    const int64_t per = (max_tiles + blockDim.x - 1) / blockDim.x;
    const int64_t s0 = threadIdx.x * per, s1 = min(s0 + per, max_tiles);
    uint32_t part = 0;
    for (int64_t t = s0; t < s1; ++t) part += tile_item[t];
    s_part[threadIdx.x] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (unsigned i = 0; i < blockDim.x; ++i) {
            const uint32_t v = s_part[i];
            s_part[i] = run;
            run += v;
        }
        plan->n_wide = n_wide;
        plan->wide_items = run;
        const uint32_t n_narrow = (uint32_t)(nq - n_wide);
        plan->total_items = run + (n_narrow + narrow_group - 1) / narrow_group;
        plan->next_item = 0;
    }
    __syncthreads();
    uint32_t run = s_part[threadIdx.x];
    for (int64_t t = s0; t < s1; ++t) {
        const uint32_t v = tile_item[t];
        tile_item[t] = run;  // first item of tile t
        run += v;
    }
}

// ENGINE 0: popcount tiles, 256 threads; ENGINE 2 / 3: fp8 / fp4 matrix-core
// tiles (mfd::tile_rows), 512 threads. Narrow queries are spread over the waves.
template <int ENGINE>
__global__ __launch_bounds__(ENGINE == 0 ? popc::kTile : mfd::kThreads) void
persistent_search_kernel(uint32_t words, const uint32_t* __restrict__ q_hv,
                         const uint32_t* __restrict__ order, const int64_t* __restrict__ lo,
                         const int64_t* __restrict__ hi, int64_t nq,
                         const int64_t* __restrict__ tile_lo, const int64_t* __restrict__ tile_hi,
                         const uint32_t* __restrict__ tile_item, int64_t max_tiles,
                         uint32_t chunk_rows, uint32_t narrow_group, Plan* __restrict__ plan,
                         const uint32_t* __restrict__ lib_hv,
                         const uint32_t* __restrict__ lib_orig, const int32_t* __restrict__ qoff,
                         const float* __restrict__ rowk, uint64_t* __restrict__ keys)
{
    static_assert(popc::kTile == mfd::kQueries, "all engines use 256-query tiles");
    constexpr int kFormat = ENGINE == HOMS_ENGINE_MFMA_F4 ? 4 : 0;  // f8f6f4 element format
    __shared__ uint32_t s_item;
    const uint32_t n_wide = plan->n_wide;
    const uint32_t wide_items = plan->wide_items;
    const uint32_t total = plan->total_items;
    const uint32_t waves = blockDim.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&plan->next_item, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total) break;  // uniform: every wave of every workgroup exits here
        if (item < wide_items) {
            // largest tile whose first item <= item
            int64_t l = 0, r = max_tiles - 1;
            while (l < r) {
                const int64_t m = (l + r + 1) >> 1;
                if (tile_item[m] <= item)
                    l = m;
                else
                    r = m - 1;
            }
            const int64_t tile = l;
            const int64_t a = tile_lo[tile] + (int64_t)(item - tile_item[tile]) * chunk_rows;
            const int64_t b = min(a + (int64_t)chunk_rows, tile_hi[tile]);
            if (a < b) {
                if constexpr (ENGINE == 0)
                    popc::popcount_tile_rows(words, (int64_t)n_wide, q_hv, order, lo, hi, tile,
                                             (uint32_t)a, (uint32_t)b, lib_hv, lib_orig, keys);
                else
                    mfd::tile_rows<kFormat>(words, (int64_t)n_wide, q_hv, order, lo, hi, tile,
                                            (uint32_t)a, (uint32_t)b, lib_hv, lib_orig, qoff,
                                            rowk, keys);
            }
        } else {
            const int64_t first = (int64_t)n_wide + (int64_t)(item - wide_items) * narrow_group;
            const int64_t last = min(first + (int64_t)narrow_group, nq);
            for (int64_t p = first + (threadIdx.x >> 6); p < last; p += waves) {
                const uint32_t qi = order[p];
                if (hi[qi] > lo[qi])
                    popc::window_rows_wave(words, qi, q_hv, (uint32_t)lo[qi], (uint32_t)hi[qi],
                                           lib_hv, lib_orig, keys);
            }
        }
    }
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t batched_scratch_bytes(int64_t nq)
{
    const int64_t max_tiles = (nq + popc::kTile - 1) / popc::kTile + 1;
    const int64_t scan_blocks = (kBuckets + kScanBlock - 1) / kScanBlock;
    return 2 * al(nq * 8) + al(nq * 8) + 2 * al(nq * 4) + al(kBuckets * 4) +
           al(scan_blocks * 4) + 2 * al(max_tiles * 8) + al(max_tiles * 4) + al(nq * 4) +
           al(sizeof(Plan));
}

hipError_t launch_search_batched(const homs_ctx* c, const BatchedConfig& cfg, void* scratch,
                                 int64_t nq, const uint32_t* q_hv, const double* q_pmz,
                                 const int8_t* q_charge, const int8_t* kinds,
                                 const double* values, int64_t* out_idx, int32_t* out_dist,
                                 hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    const int64_t max_tiles = (nq + popc::kTile - 1) / popc::kTile + 1;
    const int64_t scan_blocks = (kBuckets + kScanBlock - 1) / kScanBlock;
    char* p = (char*)scratch;
    int64_t* lo = (int64_t*)p;
    p += al(nq * 8);
    int64_t* hi = (int64_t*)p;
    p += al(nq * 8);
    uint64_t* keys = (uint64_t*)p;
    p += al(nq * 8);
    uint32_t* bucket = (uint32_t*)p;
    p += al(nq * 4);
    uint32_t* order = (uint32_t*)p;
    p += al(nq * 4);
    uint32_t* hist = (uint32_t*)p;  // counts, then bucket starts, then cursors
    p += al(kBuckets * 4);
    uint32_t* sums = (uint32_t*)p;
    p += al(scan_blocks * 4);
    int64_t* tile_lo = (int64_t*)p;
    p += al(max_tiles * 8);
    int64_t* tile_hi = (int64_t*)p;
    p += al(max_tiles * 8);
    uint32_t* tile_item = (uint32_t*)p;
    p += al(max_tiles * 4);
    int32_t* qoff = (int32_t*)p;  // per-query constants of the fp4 engine
    p += al(nq * 4);
    Plan* plan = (Plan*)p;

    hipError_t e = launch_window_bounds(c, nq, q_pmz, q_charge, HOMS_TOL_DA, 0.0, kinds, values,
                                        lo, hi, s);
    if (e != hipSuccess) return e;
    fill_u32_kernel<<<blocks_for(kBuckets), kThreads, 0, s>>>(hist, kBuckets, 0u);
    bucket_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, q_pmz, q_charge, c->p.charge_match != 0,
                                                      lo, hi, cfg.narrow_max,
                                                      1.0 / cfg.bucket_da, bucket, hist);
    scan_blocks_kernel<<<(uint32_t)scan_blocks, kThreads, 0, s>>>(hist, kBuckets, sums);
    scan_sums_kernel<<<1, 1, 0, s>>>(sums, scan_blocks);
    scan_add_kernel<<<blocks_for(kBuckets), kThreads, 0, s>>>(hist, kBuckets, sums);
    scatter_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, bucket, hist, order);
    plan_kernel<<<1, 1024, 0, s>>>(nq, hist, order, lo, hi, cfg.chunk_rows, cfg.narrow_group,
                                   max_tiles, tile_lo, tile_hi, tile_item, plan);
    fill_u64_kernel<<<blocks_for(nq), kThreads, 0, s>>>(keys, nq, ~0ull);
    if (cfg.engine == HOMS_ENGINE_MFMA_F8) {
        persistent_search_kernel<HOMS_ENGINE_MFMA_F8><<<cfg.grid, mfd::kThreads, 0, s>>>(
            c->words, q_hv, order, lo, hi, nq, tile_lo, tile_hi, tile_item, max_tiles,
            cfg.chunk_rows, cfg.narrow_group, plan, c->lib.hv, c->lib.orig, nullptr, nullptr,
            keys);
    } else if (cfg.engine == HOMS_ENGINE_MFMA_F4) {
        e = launch_fp4_query_offsets(c, nq, q_hv, qoff, s);
        if (e != hipSuccess) return e;
        persistent_search_kernel<HOMS_ENGINE_MFMA_F4><<<cfg.grid, mfd::kThreads, 0, s>>>(
            c->words, q_hv, order, lo, hi, nq, tile_lo, tile_hi, tile_item, max_tiles,
            cfg.chunk_rows, cfg.narrow_group, plan, c->lib.hv, c->lib.orig, qoff, c->lib.rowk,
            keys);
    } else {
        persistent_search_kernel<HOMS_ENGINE_POPCOUNT><<<cfg.grid, popc::kTile, 0, s>>>(
            c->words, q_hv, order, lo, hi, nq, tile_lo, tile_hi, tile_item, max_tiles,
            cfg.chunk_rows, cfg.narrow_group, plan, c->lib.hv, c->lib.orig, nullptr, nullptr,
            keys);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(nq, keys, out_idx, out_dist, s);
}

}  // namespace homs
