// Shortlist search with the learned embedding.
//
// For every query the k candidates of its window (Section 3.4) with the
// largest embedding scores e_q . e_r are kept (ties to the lower library
// index) and rescored exactly by Hamming distance; the result is the
// exhaustive top-1 restricted to that shortlist.
//
// Selecting k of up to a few million scores per query is done in one scoring
// pass over the window:
//  1. threshold: per tile of 128 m/z-ordered queries, score a regular sample
//     of the union of its windows (every 2^j-th sorted row, at most kSample
//     rows) on matrix cores; per query take the r-th largest of its in-window
//     sample scores (radix select), r chosen so that about t1 window
//     candidates are expected at or above it (t1 between a quarter and a half
//     of the kCapacity buffer, growing with k; see shortlist_targets);
//     windows of at most kSample (= kCapacity) candidates keep everything;
//  2. collect: score every (query, candidate) pair on matrix cores (E4M3
//     scoring embeddings, fp32 accumulation; a workgroup takes 128
//     m/z-ordered queries and an 8,192-row chunk of the library in 32-row
//     block steps) and append in-window pairs at or above the query's
//     threshold to its buffer of kCapacity 64-bit keys (order-preserving
//     score << 32 | sorted row), in two passes: pass 0 over every eighth
//     absolute 128-row block with the sampled threshold; then per query a
//     threshold refined from pass 0's hits (the r-th best of them, about t2
//     window candidates expected above it, t2 leaving k a margin of four
//     standard deviations); pass 1 over the other blocks with the refined
//     threshold, where hits are rare enough that most tiles need only one
//     ballot;
//  3. select: the k largest keys of each buffer in descending order (a
//     buffer of at most 2k keys sorted whole in LDS, a larger one first cut
//     to its k best by a radix select); a query whose buffer overflowed,
//     whose sampled threshold kept fewer than min(k, window) candidates, or
//     whose k-th kept key scores below the refined threshold (so that a
//     better candidate of pass 1 could have been missed) is flagged for the
//     exhaustive fallback and gets no shortlist;
//  4. rescore: one wave per query, 16 lanes per shortlist entry, computes the
//     exact Hamming distances; the wave minimum of (distance << 32 | library
//     index) is merged into the query's key;
//  5. fallback: the flagged queries are listed on the device and their whole
//     windows scanned, one wave per 512-row unit, into the same keys.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "gemm_bf16.h"
#include "learned.h"
#include "popcount_tile.h"

namespace homs {
namespace {

constexpr int kSample = 8192;    // most sampled candidates per window
constexpr int kCapacity = 8192;  // buffer entries per query
// Per-query buffer counters one per 128-byte line: the atomics of one flush
// (entries of up to 64 queries) then spread over L2 channels instead of
// serialising on two lines.
constexpr int kCountStride = 32;
constexpr int kTileQ = 128;      // queries per collection workgroup
constexpr int64_t kCollectChunk = 8192;  // library rows per collection workgroup
constexpr int kRowGroups = 1;  // row groups of a collection workgroup (32-row block steps)
constexpr int kThreads = 256;
constexpr int64_t kFallbackRows = 512;   // window rows per wave in the exhaustive fallback

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + kThreads - 1) / kThreads); }


// order-preserving map of a float onto uint32 (larger float, larger key)
__device__ __forceinline__ uint32_t fkey(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (b >> 31) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float fkey_inv(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// dst row p = src row perm[p]; 16-byte pieces
__global__ void permute_rows_kernel(int64_t n, int E, const uint32_t* __restrict__ perm,
                                    const uint16_t* __restrict__ src, uint16_t* __restrict__ dst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int per = E / 8;
    if (t >= n * per) return;
    const int64_t r = t / per;
    const int c = (int)(t - r * per);
    ((uint4*)(dst + r * E))[c] = ((const uint4*)(src + (size_t)perm[r] * E))[c];
}

// dst row p = src row perm[p] for rows of E bytes; 16-byte pieces
__global__ void permute_rows8_kernel(int64_t n, int E, const uint32_t* __restrict__ perm,
                                     const uint8_t* __restrict__ src, uint8_t* __restrict__ dst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int per = E / 16;
    if (t >= n * per) return;
    const int64_t r = t / per;
    const int c = (int)(t - r * per);
    ((uint4*)(dst + r * E))[c] = ((const uint4*)(src + (size_t)perm[r] * E))[c];
}

// Bitonic sort, descending, of n = 2^j keys in LDS by one workgroup.
__device__ void bitonic_desc(uint64_t* a, int n)
{
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool desc = (lo & size) == 0;
                const uint64_t x = a[lo], y = a[hi];
                if (desc ? (x < y) : (x > y)) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

// Sample grid of a tile of 128 m/z-ordered queries: the rows g0 + m 2^sh
// (m < n) of the sorted library inside the union of the tile's windows, with
// the smallest sh that keeps n <= kSample (n = 0 when the union itself has at
// most kSample rows, so no query of the tile needs a threshold).
struct SampleGrid {
    int64_t g0;
    int32_t sh;
    int32_t n;
};

// Scores of every query of a tile against its sample grid, on matrix cores:
// S[q][m] = e_q . e_(row m), fp32. kSampleSplit workgroups per tile take
// 128-row steps of the grid in turn; the queries are the A operand, so that
// each accumulator register holds 32 consecutive samples of one query and
// the stores are contiguous.
constexpr int kSampleSplit = 8;
__global__ __launch_bounds__(256) void sample_scores_kernel(
    int E, int64_t q_begin, int64_t q_end, const uint16_t* __restrict__ q_sorted,
    const int64_t* __restrict__ tile_lo, const int64_t* __restrict__ tile_hi,
    const uint16_t* __restrict__ lib_emb, SampleGrid* __restrict__ grids, float* __restrict__ S)
{
    using namespace gemm;
    __shared__ __attribute__((aligned(16))) uint8_t sA[2][kTM * kRowBytes];
    __shared__ __attribute__((aligned(16))) uint8_t sB[2][kTN * kRowBytes];
    const int64_t tile = blockIdx.x / kSampleSplit;
    const int split = (int)(blockIdx.x % kSampleSplit);
    const int64_t u0 = tile_lo[tile], u1 = tile_hi[tile];
    SampleGrid gr{u0, 0, 0};
    if (u1 - u0 > kSample) {
        int sh = 1;
        while (((u1 - u0 + ((int64_t)1 << sh) - 1) >> sh) > kSample) ++sh;
        const int64_t st = (int64_t)1 << sh;
        gr.g0 = (u0 + st - 1) & ~(st - 1);
        gr.sh = sh;
        gr.n = (int32_t)((u1 - gr.g0 + st - 1) >> sh);
    }
    if (threadIdx.x == 0 && split == 0) grids[tile] = gr;
    if (gr.n == 0) return;  // uniform
    const int t = threadIdx.x, l = t & 63, w = t >> 6, wr = w & 1, wn = w >> 1;
    const int64_t p0 = q_begin + tile * kTileQ;
    const int64_t qlast = q_end - 1;
    const int row0 = t >> 1, part0 = (t * 2) & 3;
    const uint16_t* b_row = q_sorted + (size_t)min(p0 + row0, qlast) * E + part0 * 8;
    uint8_t* sa_dst = &sA[0][0] + row0 * kRowBytes + part0 * 16;
    uint8_t* sb_dst = &sB[0][0] + row0 * kRowBytes + part0 * 16;
    float* Sq = S + (size_t)(tile * kTileQ) * kSample;
    for (int m0 = split * kTM; m0 < gr.n; m0 += kSampleSplit * kTM) {
        const int64_t mrow = gr.g0 + ((int64_t)min(m0 + row0, gr.n - 1) << gr.sh);
        const uint16_t* a_row = lib_emb + (size_t)mrow * E + part0 * 8;
        Stage st;
        f32x16 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{0};
        const int nk = E / kTK;
        st = load_stage(a_row, b_row, 0);
        store_stage(st, sa_dst, sb_dst, 0);
        __syncthreads();
        for (int s = 0; s < nk; ++s) {
            const int b = s & 1;
            if (s + 1 < nk) st = load_stage(a_row, b_row, (s + 1) * kTK);
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                bf16x8 av[2], bv[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    av[i] = *(const bf16x8*)(sA[b] + (wr * 64 + i * 32 + (l & 31)) * kRowBytes +
                                             ks * 32 + 16 * (l >> 5));
                    bv[i] = *(const bf16x8*)(sB[b] + (wn * 64 + i * 32 + (l & 31)) * kRowBytes +
                                             ks * 32 + 16 * (l >> 5));
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bv[j], av[i],
                                                                           acc[i][j], 0, 0, 0);
            }
            if (s + 1 < nk) store_stage(st, sa_dst, sb_dst, b ^ 1);
            __syncthreads();
        }
        // register r of acc[i][j]: query wn 64 + 32 j + 8 (r / 4) + 4 (l / 32) + r % 4,
        // sample m0 + wr 64 + 32 i + l % 32
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = m0 + wr * 64 + i * 32 + (l & 31);
            if (m >= gr.n) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int q = wn * 64 + j * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
                    Sq[(size_t)q * kSample + m] = acc[i][j][r];
                }
        }
    }
}

// One round of a radix select, by the first wave of the workgroup: from the
// 256 digit counts, the largest digit d with (keys above d) < r <= (keys at
// or above d), the count above it and hist[d] (digit 0 when r exceeds the
// total). Lane l sums digits 255 - 4 l .. 252 - 4 l, a wave scan orders the
// lanes, and the first lane whose running count reaches r walks its four.
struct RadixDigit {
    uint32_t digit, above, eq;
};
__device__ RadixDigit radix_digit(const uint32_t* hist, uint32_t r)
{
    const int l = threadIdx.x & 63;
    uint32_t h[4], sum = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        h[c] = hist[255 - 4 * l - c];
        sum += h[c];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off);
        if (l >= off) inc += y;
    }
    const uint64_t m = __ballot(inc >= r);
    RadixDigit out;
    if (m == 0) {
        const uint32_t h0 = hist[0];
        out.digit = 0;
        out.above = __shfl(inc, 63) - h0;
        out.eq = h0;
        return out;
    }
    const int L = __ffsll((unsigned long long)m) - 1;
    uint32_t d = 0, ab = 0, e = 0, cum = inc - sum;
    bool found = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) {  // digit 255 - 4 l - c, from the top
        if (!found && cum + h[c] >= r) {
            found = true;
            d = (uint32_t)(255 - 4 * l - c);
            ab = cum;
            e = h[c];
        }
        cum += h[c];
    }
    out.digit = __shfl(d, L);
    out.above = __shfl(ab, L);
    out.eq = __shfl(e, L);
    return out;
}

// One workgroup per query of the pass: the r-th largest of its in-window
// sample scores (radix select over order-preserving keys, 8 bits per round),
// with r chosen so that about `target` window candidates are expected at or
// above it; -inf keeps the whole window.
__global__ __launch_bounds__(kThreads) void threshold_kernel(
    int64_t q_begin, int64_t target, const uint32_t* __restrict__ qperm,
    const int64_t* __restrict__ lo, const int64_t* __restrict__ hi,
    const SampleGrid* __restrict__ grids, const float* __restrict__ S, float* __restrict__ thr)
{
    __shared__ uint32_t hist[256];
    __shared__ RadixDigit s_rd;
    const int64_t qp = blockIdx.x;  // position in the pass
    const int64_t p = q_begin + qp;
    const uint32_t qi = qperm[p];
    const int64_t a = lo[qi], b = hi[qi], w = b - a;
    const SampleGrid gr = grids[qp / kTileQ];
    int64_t i0 = 0, i1 = 0;
    if (w > kSample && gr.n > 0) {
        const int64_t st = (int64_t)1 << gr.sh;
        i0 = a <= gr.g0 ? 0 : (a - gr.g0 + st - 1) >> gr.sh;
        i1 = b <= gr.g0 ? 0 : min((int64_t)gr.n, (b - gr.g0 + st - 1) >> gr.sh);
    }
    const int ns = (int)max((int64_t)0, i1 - i0);
    if (ns == 0) {  // uniform
        if (threadIdx.x == 0) thr[p] = -INFINITY;
        return;
    }
    const float* v = S + (size_t)qp * kSample + i0;
    int64_t r64 = (target * ns + w - 1) / w;
    uint32_t r = (uint32_t)(r64 < 1 ? 1 : (r64 > ns ? ns : r64));
    // the sample keys stay in registers for the four rounds
    constexpr int kPer = kSample / kThreads;
    uint32_t key[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = (int)threadIdx.x + j * kThreads;
        key[j] = i < ns ? fkey(v[i]) : 0u;
    }
    uint32_t prefix = 0, mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = (int)threadIdx.x + j * kThreads;
            if (i < ns && (key[j] & mask) == prefix)
                atomicAdd(&hist[(key[j] >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const RadixDigit rd = radix_digit(hist, r);
            if (threadIdx.x == 0) s_rd = rd;
        }
        __syncthreads();
        prefix |= s_rd.digit << shift;
        mask |= 255u << shift;
        r -= s_rd.above;
    }
    if (threadIdx.x == 0) thr[p] = fkey_inv(prefix);
}

// Library rows are scored in two passes over absolute 128-row blocks: pass 0
// takes the blocks whose index is a multiple of kPassStride (an evenly spread
// 1 / kPassStride of every window) with the sampled threshold, pass 1 the
// others with a threshold refined from pass 0's hits.
constexpr int64_t kPassStride = 8;

// rows below x (absolute) that lie in pass-0 blocks
__host__ __device__ inline int64_t pass0_rows_below(int64_t x)
{
    const int64_t span = 128 * kPassStride;
    return (x / span) * 128 + min(x % span, (int64_t)128);
}

// One workgroup per query of the pass: the refined threshold. Pass 0 kept,
// from its 1 / kPassStride share of the window, every candidate scoring at
// or above the sampled threshold; the r-th largest of them, r = ceil(target x
// share / window) (about `target` window candidates are then expected at or
// above it), is the threshold of pass 1. Windows kept whole (-inf), a pass-0
// buffer that overflowed, or fewer than r pass-0 candidates keep the sampled
// threshold.
__global__ __launch_bounds__(kThreads) void refine_threshold_kernel(
    int64_t q_begin, int64_t target, const uint32_t* __restrict__ qperm,
    const int64_t* __restrict__ lo,
    const int64_t* __restrict__ hi, const uint32_t* __restrict__ count,
    const uint64_t* __restrict__ buf, const float* __restrict__ thr, float* __restrict__ thr2)
{
    __shared__ uint32_t hist[256];
    __shared__ RadixDigit s_rd;
    const int64_t qp = blockIdx.x;
    const int64_t p = q_begin + qp;
    const float t1 = thr[p];
    const uint32_t qi = qperm[p];
    const int64_t a = lo[qi], b = hi[qi], w = b - a;
    const uint32_t cnt = count[qp * kCountStride];
    const int64_t share = pass0_rows_below(b) - pass0_rows_below(a);
    const int64_t r64 = w > 0 ? (target * share + w - 1) / w : 0;
    // uniform
    if (t1 == -INFINITY || cnt > (uint32_t)kCapacity || r64 < 1 || (int64_t)cnt < r64) {
        if (threadIdx.x == 0) thr2[p] = t1;
        return;
    }
    const int n = (int)cnt;
    uint32_t r = (uint32_t)r64;
    const uint64_t* keys = buf + (size_t)qp * kCapacity;
    constexpr int kPer = kCapacity / kThreads;
    uint32_t key[kPer];  // score halves of the keys, in registers
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = (int)threadIdx.x + j * kThreads;
        key[j] = i < n ? (uint32_t)(keys[i] >> 32) : 0u;
    }
    uint32_t prefix = 0, mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = (int)threadIdx.x + j * kThreads;
            if (i < n && (key[j] & mask) == prefix) atomicAdd(&hist[(key[j] >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const RadixDigit rd = radix_digit(hist, r);
            if (threadIdx.x == 0) s_rd = rd;
        }
        __syncthreads();
        prefix |= s_rd.digit << shift;
        mask |= 255u << shift;
        r -= s_rd.above;
    }
    if (threadIdx.x == 0) thr2[p] = fmaxf(t1, fkey_inv(prefix));
}

// Scores BR = 32 NWR library rows x 128 m/z-ordered queries per block step on
// matrix cores and appends every in-window pair at or above the query's
// threshold.
//
// Operands are the scoring embeddings as E4M3 codes of 16 e (one byte per
// component, v_mfma_f32_32x32x64_f8f6f4, fp32 accumulation): every product
// of two codes is exact in fp32, and the accumulator holds 256 times the
// score of the rounded embeddings.
//
// 2 NWR waves per workgroup, two per SIMD: wave (wr, wn) owns rows 32 wr ..
// + 31 of each block and the 64 queries of half wn (two 32-query tiles),
// whose codes are its B operands for the whole chunk (E / 64 steps of 32
// bytes per tile), so every A operand read from LDS feeds two matrix
// instructions. Library rows
// stream through four LDS buffers filled by direct global-to-LDS loads
// (global_load_lds_dwordx4, no staging registers): one load moves 1 KB (64
// lanes x 16 bytes) of a block's rows, so a block of BR E-byte rows takes
// E / 64 loads per wave. The barrier of a block step couples only the waves
// of one workgroup: with NWR = 1 (32-row steps, two waves) four workgroups
// share a compute unit and the matrix cores run the waves of the others
// while one workgroup waits at its barrier (with 1M + 1M rows and 100k
// queries the scoring takes 22.4 ms with NWR = 2 and 21.0 ms with NWR = 1,
// against 27.3 ms with NWR = 4, one workgroup per compute unit). Per block
// step, the block's A operands are in registers (read from LDS one step
// ahead), the next block waits in LDS and
// two more are in flight; one barrier per block both publishes the landed
// block and frees the buffer of the block in registers. The 16-byte piece
// p of row R sits at slot p ^ swz(R) of the row, swz(R) = (R / (16 / P)) mod
// P with P = E / 16 pieces per row, so the 16 rows a quarter-wave reads
// together land on 16 distinct 16-byte bank groups. The loads are issued
// from inline asm with explicit vmcnt waits: the compiler would otherwise
// drain every outstanding LDS load before any LDS read and cap the prefetch
// at one block.
//
// Epilogue, software-pipelined: two accumulator sets are used in turn. The
// straight-line part of a step's other work (the hit pre-check of block
// b - 1, the next loads, the next block's LDS reads, bookkeeping) is placed
// between block b's matrix instructions, where the wave issues it while the
// matrix core runs; the hits of block b - 1 follow the matrix instructions.
// When the wave's 32 rows of the block lie inside every window of its
// queries (the usual case), one ballot per query tile on each lane's largest
// score first tells whether the tile has any hit; only such tiles take a
// compare and a ballot per position (skipped unless some lane hits).
// Otherwise the block's positions are masked row by row. Hits go to the
// wave's own LDS list at positions counted from the ballot (no atomics, no
// global loads), flushed to the per-query global buffers when half full and
// at the end.
constexpr int kWaveList = 384;  // LDS entries per wave

// s_waitcnt immediate: vmcnt(n), expcnt and lgkmcnt left at their maxima
constexpr int waitcnt_vm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x70 | 0xF00; }
// vmcnt(n) and lgkmcnt(0)
constexpr int waitcnt_vm_lgkm0(int n) { return (n & 15) | ((n >> 4) << 14) | 0x70; }

typedef int v8i32 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float max16(const gemm::f32x16& v)
{
    const float a = fmaxf(fmaxf(v[0], v[1]), v[2]), b = fmaxf(fmaxf(v[3], v[4]), v[5]);
    const float c = fmaxf(fmaxf(v[6], v[7]), v[8]), d = fmaxf(fmaxf(v[9], v[10]), v[11]);
    const float e = fmaxf(fmaxf(v[12], v[13]), v[14]);
    return fmaxf(fmaxf(fmaxf(a, b), c), fmaxf(fmaxf(d, e), v[15]));
}

template <int E, int pass, int NWR>
__global__ __launch_bounds__(64 * 2 * NWR, 2) void collect_kernel(
    int64_t q_begin, int64_t q_end, const uint8_t* __restrict__ q_sorted8,
    const uint32_t* __restrict__ qperm, const int64_t* __restrict__ lo,
    const int64_t* __restrict__ hi, const float* __restrict__ thr,
    const int64_t* __restrict__ tile_lo, const int64_t* __restrict__ tile_hi,
    const uint8_t* __restrict__ lib_emb8, uint32_t* __restrict__ count,
    uint64_t* __restrict__ buf, int64_t n_tiles, int64_t n_chunks)
{
    using namespace gemm;
    constexpr int KS = E / 64;                    // 32 x 32 x 64 steps
    constexpr int PPK = 16 / KS;                  // epilogue positions per step
    constexpr int P = E / 16;                     // 16-byte pieces per row
    constexpr int RPS = 16 / P;                   // rows sharing one swizzle value
    constexpr int NW = 2 * NWR;                   // waves: NWR row groups x 2 query halves
    constexpr int BR = 32 * NWR;                  // rows per block step
    constexpr uint32_t S = 128 / BR;              // block steps per 128-row pass block
    constexpr int NL = E / 64;                    // direct loads per wave per block
    constexpr float kScoreScale2 = kScoreScale * kScoreScale;
    constexpr int kBufs = 4;                      // LDS block buffers: kBufs blocks in flight
    static_assert(KS * PPK == 16 && NL >= 1, "E in {64, 128, 256}");
    static_assert(NWR == 1 || NWR == 2 || NWR == 4, "32-, 64- or 128-row block steps");
    __shared__ __attribute__((aligned(16))) uint8_t sA[kBufs][BR * E];
    __shared__ uint64_t s_key[NW][kWaveList];
    __shared__ uint8_t s_col[NW][kWaveList];  // query of the entry within the tile
    // Chunks are fixed row ranges of the sorted library, clipped to the
    // tile's candidate range. Workgroups go to the eight XCDs in turn
    // (workgroup i to XCD i mod 8, each with its own L2): XCD x takes chunks
    // x, x + 8, ... and, for each, every tile, so a chunk's rows are fetched
    // into one L2 and read there by all the tiles that cover it.
    const int64_t wg = blockIdx.x;
    const int64_t slot = wg >> 3;
    const int64_t chunk = (slot / n_tiles) * 8 + (wg & 7);
    const int64_t tile = slot % n_tiles;
    if (chunk >= n_chunks) return;
    const int64_t r0 = chunk * kCollectChunk;
    const int64_t c0 = max(r0, tile_lo[tile]);
    const int64_t c1 = min(r0 + kCollectChunk, tile_hi[tile]);
    if (c0 >= c1) return;
    // the chunk's end row in a scalar register (32-bit: the library has
    // fewer than 2^31 rows)
    const uint32_t e1 = __builtin_amdgcn_readfirstlane((uint32_t)c1);
    // the wave index in a scalar register: everything derived from it is
    // wave-uniform scalar work
    const int t = threadIdx.x, l = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wr = w % NWR, wn = w / NWR;
    const int64_t p0 = q_begin + tile * kTileQ;  // first sorted query of the tile
    // This pass's BR-row blocks meeting [c0, c1), in the absolute 128-row
    // blocks of the pass (pass 0 the multiples of kPassStride, pass 1 the
    // others): block g lies in pass-0 block g / S when g mod G < S. Rows of a
    // block below c0 lie below every window of the tile (c0 is the chunk's
    // first row or the tile's lowest window start) and are masked like any
    // row outside a window.
    constexpr int64_t G = kPassStride * S;
    const int64_t g_lo = c0 / BR, g_hi = (c1 + BR - 1) / BR;
    auto below0 = [](int64_t x) { return x / G * S + min(x % G, (int64_t)S); };
    const int64_t n0 = below0(g_hi) - below0(g_lo);
    const int nblk = (int)(pass == 0 ? n0 : (g_hi - g_lo) - n0);
    if (nblk == 0) return;
    // The pass's blocks in order (32-bit: the library has fewer than 2^31
    // rows): two walkers, one for the loads (kBufs - 1 blocks ahead) and one
    // for the epilogue, each stepping to the next block of the pass.
    const bool lo_in0 = g_lo % G < (int64_t)S;
    const uint32_t first =
        pass == 0 ? (uint32_t)(lo_in0 ? g_lo : (g_lo / G + 1) * G)
                  : (uint32_t)(lo_in0 ? g_lo - g_lo % G + S : g_lo);
    auto next_block = [&](uint32_t g) -> uint32_t {
        g += 1;
        if (pass == 0) return g % (uint32_t)G == S ? g + (uint32_t)(G - S) : g;
        return g % (uint32_t)G == 0 ? g + S : g;
    };
    uint32_t g_issue = first, g_epi = first;
    // the pass's last block in the chunk: the loads issued for block steps
    // past the end re-read it into a buffer that is never scored, so that
    // every step waits for the same number of loads, with no branch
    const int64_t y = g_hi - 1, ym = y % G;
    const uint32_t g_last = pass == 0 ? (uint32_t)(ym < (int64_t)S ? y : y - ym + S - 1)
                                      : (uint32_t)(ym >= (int64_t)S ? y : y - ym - 1);

    // rows [BR g, + BR) of the block g_issue points to into sA[b % kBufs]:
    // load x of wave w fills bytes [1024 (NL w + x), + 1024) of the buffer
    // (the destination of a direct load is M0 + 16 x lane), lane l the slot
    // of row R = o / E, o the byte offset of the lane, with the row's piece
    // (slot ^ swz(R)); rows past c1 repeat the last row
    auto issue = [&](int b) {  // block b, the one g_issue points to
        const uint32_t mb = (b < nblk ? g_issue : g_last) * (uint32_t)BR;
        g_issue = next_block(g_issue);
        const uint32_t base = (uint32_t)(uintptr_t)&sA[b % kBufs][0];
        const uint8_t* gbase = lib_emb8 + (size_t)mb * E;  // wave-uniform
        const int last = (int)min((uint32_t)BR - 1u, e1 - 1u - mb);
#pragma unroll
        for (int x = 0; x < NL; ++x) {
            const int ci = w * NL + x;
            const int o = ci * 1024 + 16 * l;
            const int R = o / E;
            const int sl = (o % E) / 16;
            const int pc = sl ^ ((R / RPS) % P);
            const uint32_t voff = (uint32_t)(min(R, last) * E + pc * 16);
            const uint32_t lds = __builtin_amdgcn_readfirstlane(base + (uint32_t)(ci * 1024));
            asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1"
                         :
                         : "v"(voff), "s"(gbase), "s"(lds)
                         : "memory", "m0");
        }
    };

    // this lane's two query columns: epilogue state (32-bit rows: the library
    // has fewer than 2^31 rows) and B operands
    int col[2];
    bool qok[2];
    uint32_t qlo[2], qhi[2];
    float qthr[2];
    v8i32 bq[2][KS];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        col[j] = wn * 64 + j * 32 + (l & 31);
        const int64_t p = p0 + col[j];
        qok[j] = p < q_end;
        qlo[j] = qhi[j] = 0;
        qthr[j] = INFINITY;
        if (qok[j]) {
            const uint32_t qi = qperm[p];
            qlo[j] = (uint32_t)lo[qi];
            qhi[j] = (uint32_t)hi[qi];
            qthr[j] = thr[p] * kScoreScale2;  // exact: a power of two
        }
        const uint8_t* qrow = q_sorted8 + (size_t)min(p, q_end - 1) * E + 32 * (l >> 5);
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const uint4 u0 = *(const uint4*)(qrow + kk * 64);
            const uint4 u1 = *(const uint4*)(qrow + kk * 64 + 16);
            bq[j][kk] = v8i32{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w,
                              (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
        }
    }
    // LDS offsets of this lane's A operand: row R = 32 wr + l % 32, pieces
    // 4 kk + 2 (l / 32) + c of the 64-byte step kk
    uint32_t aoff[KS][2];
    {
        const int R = wr * 32 + (l & 31);
        const int sw = (R / RPS) % P;
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                aoff[kk][c] = (uint32_t)(R * E + 16 * ((4 * kk + 2 * (l >> 5) + c) ^ sw));
    }
    // rows [wlo, whi) lie inside the chunk and inside the window of every
    // query of the wave (wave-uniform): a block whose 32 rows of the wave
    // fall in it needs no per-row window test
    uint32_t wlo, whi;
    {
        uint32_t lo_all = 0, hi_all = e1;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (qok[j]) {
                lo_all = max(lo_all, qlo[j]);
                hi_all = min(hi_all, qhi[j]);
            }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo_all = max(lo_all, (uint32_t)__shfl_xor((int)lo_all, o));
            hi_all = min(hi_all, (uint32_t)__shfl_xor((int)hi_all, o));
        }
        wlo = __builtin_amdgcn_readfirstlane(lo_all);
        whi = __builtin_amdgcn_readfirstlane(hi_all);
    }
    // The B operands are in registers before the pipeline starts, so that no
    // wait for them is left inside the loop, where it would also wait for the
    // prefetched blocks (vmcnt counts in issue order). The empty asm
    // statements consume the loaded values here, so the compiler can neither
    // sink the loads below the prefetch (the restrict-qualified query rows
    // would let it) nor leave their wait to the loop.
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) asm volatile("" : "+v"(bq[j][kk]));
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    for (int b = 0; b < kBufs; ++b) issue(b);

    // the wave's LDS hit list and its flush to the per-query global buffers
    uint32_t wcount = 0;  // wave-uniform
    const int64_t qbase = tile * kTileQ;  // pass slot of the tile's first query
    // one hit straight to the global buffer (score key << 32 | sorted row:
    // the select kernel turns rows into library indices)
    auto put = [&](int64_t qs, uint64_t v) {
        const uint32_t slot = atomicAdd(count + qs * kCountStride, 1u);
        if (slot < (uint32_t)kCapacity) buf[(size_t)qs * kCapacity + slot] = v;
    };
    // the wave's list to the global buffers, four entries per lane at a time
    // so that their atomics are in flight together
    auto flush = [&]() {
        for (uint32_t e0 = 0; e0 < wcount; e0 += 256) {
            uint32_t slot[4];
            int64_t qs[4];
            uint64_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t e = e0 + 64 * u + l;
                qs[u] = e < wcount ? qbase + s_col[w][e] : -1;
                v[u] = e < wcount ? s_key[w][e] : 0;
                slot[u] = qs[u] >= 0 ? atomicAdd(count + qs[u] * kCountStride, 1u) : 0xFFFFFFFFu;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (slot[u] < (uint32_t)kCapacity) buf[(size_t)qs[u] * kCapacity + slot[u]] = v[u];
        }
        wcount = 0;
    };
    // append the hits of one position of query tile j (m: the wave's hit
    // mask, uniform; sc: 256 times the score)
    auto append = [&](uint64_t m, bool ok, float sc, uint32_t g, int j) {
        const uint64_t v = ((uint64_t)fkey(sc * (1.f / kScoreScale2)) << 32) | (uint64_t)g;
        if (wcount + 64 <= kWaveList) {
            // the sorted row: its library index is looked up by the select
            // kernel, so no global load (and no vmcnt wait, which would also
            // drain the prefetch) happens in this kernel
            if (ok) {
                const uint32_t pos =
                    wcount + __builtin_amdgcn_mbcnt_hi(
                                 (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                s_key[w][pos] = v;
                s_col[w][pos] = (uint8_t)col[j];
            }
            wcount += (uint32_t)__popcll(m);
        } else if (ok) {  // list full inside a dense block: direct
            put(qbase + col[j], v);
        }
    };

    // Accumulator register r of query tile j holds matrix row
    // i = 8 (r / 4) + 4 (l / 32) + r % 4 of the wave's tile, library row
    // wb + i with wb = the block's first row + 32 wr: gl + roff(r) with
    // gl = wb + 4 (l / 32).
    auto roff = [](int r) -> uint32_t { return (uint32_t)(8 * (r >> 2) + (r & 3)); };
    // The scores of a scored block are examined while the next block's
    // matrix instructions run: gl = the row of accumulator register 0 in this
    // lane, fast = every row of the wave lies inside every window of its
    // queries. The pre-check (fast case): which query tiles have a hit at
    // all, from the largest of each lane's 16 scores (one query, 16 rows)
    // against its threshold, one ballot per tile; straight-line code, so it
    // can sit between matrix instructions.
    auto precheck = [&](const f32x16(&a)[2], uint64_t (&hit)[2]) {
#pragma unroll
        for (int j = 0; j < 2; ++j) hit[j] = __ballot(max16(a[j]) >= qthr[j]);
    };
    // the hits themselves: in the fast case a compare and a ballot per
    // position of the tiles the pre-check flagged, else per-row masks
    auto examine = [&](const f32x16(&a)[2], uint32_t gl, bool fast, const uint64_t (&hit)[2]) {
        if (fast) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (hit[j] == 0) continue;  // one test per tile, not per position
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float sc = a[j][r];
                    const uint64_t m = __ballot(sc >= qthr[j]);
                    if (m != 0) append(m, sc >= qthr[j], sc, gl + roff(r), j);
                }
            }
        } else {  // window or chunk edge inside the wave's rows: per-row masks
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t g = gl + roff(r);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const float sc = a[j][r];
                    const bool ok = sc >= qthr[j] && g < e1 && g >= qlo[j] && g < qhi[j];
                    const uint64_t m = __ballot(ok);
                    if (m != 0) append(m, ok, sc, g, j);
                }
            }
        }
    };
    auto block_info = [&](uint32_t& gl, bool& fast) {  // the block g_epi points to
        const uint32_t wb = g_epi * (uint32_t)BR + wr * 32;
        g_epi = next_block(g_epi);
        gl = wb + 4u * (uint32_t)(l >> 5);
        fast = wb >= wlo && wb + 32 <= whi;
    };
    // block b's A operands (this lane's row, all E / 64 steps) from LDS
    auto read_a = [&](int b, v8i32(&av)[KS]) {
        const uint8_t* Ab = sA[b % kBufs];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const uint4 u0 = *(const uint4*)(Ab + aoff[kk][0]);
            const uint4 u1 = *(const uint4*)(Ab + aoff[kk][1]);
            av[kk] = v8i32{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w,
                           (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
        }
    };

    // Software pipeline, one step per block b: block b's A operands are in
    // registers (read from LDS during step b - 1), block b + 1 sits in LDS,
    // blocks b + 2 and b + 3 are in flight. Step b waits for block b + 1 (own
    // loads, then the barrier for everyone's; the barrier also means every
    // wave has its block-b operands, so block b's buffer is free), issues the
    // loads of block b + 4 into that buffer and runs block b's matrix
    // instructions with the rest of the step's work placed between them:
    // the pre-check of block b - 1, the loads, the LDS reads of block b + 1
    // and the block bookkeeping. A wave keeps issuing while its matrix
    // instruction runs, so that work is hidden behind the matrix core; the
    // scheduling barriers keep the compiler from regrouping it. The hits of
    // block b - 1 (branches, rare) follow the matrix instructions. Two
    // accumulator and two operand sets are used in turn.
    auto step = [&](int b, f32x16(&cur)[2], const f32x16(&prev)[2], const v8i32(&avc)[KS],
                    v8i32(&avn)[KS], uint32_t glp, bool fastp, uint32_t& glc, bool& fastc) {
        // this wave's LDS reads of block b are complete before the barrier,
        // so no wave can refill block b's buffer under them
        __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0((kBufs - 2) * NL));
        __syncthreads();
        uint64_t hit[2];
        // work item t runs after matrix instruction min(at[t], 2 KS - 1); the
        // LDS reads of block b + 1 come late, when most of block b's operand
        // registers are free again
        constexpr int at[5] = {0, 1, 2, 3, 5};
        auto work = [&](int t) {
            if (t == 0) hit[0] = __ballot(max16(prev[0]) >= qthr[0]);
            if (t == 1) hit[1] = __ballot(max16(prev[1]) >= qthr[1]);
            if (t == 2) issue(b + kBufs);
            if (t == 3) block_info(glc, fastc);
            if (t == 4) read_a(b + 1, avn);
        };
        constexpr int kWork = 5;
#pragma unroll
        for (int i = 0; i < 2 * KS; ++i) {
            const int kk = i >> 1, j = i & 1;
            cur[j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                avc[kk], bq[j][kk], kk == 0 ? f32x16{0} : cur[j], 0, 0, 0, 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < kWork; ++t)
                if (min(at[t], 2 * KS - 1) == i) {
                    work(t);
                    __builtin_amdgcn_sched_barrier(0);
                }
        }
        if (b > 0) examine(prev, glp, fastp, hit);
        if (wcount > kWaveList / 2) flush();  // wave-uniform
    };

    f32x16 accA[2], accB[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) accA[j] = accB[j] = f32x16{0};
    v8i32 avA[KS], avB[KS];
    uint32_t glA = 0, glB = 0;
    bool fastA = false, fastB = false;
    // block 0 landed (the loads of blocks 1 .. kBufs - 1 stay in flight)
    __builtin_amdgcn_s_waitcnt(waitcnt_vm((kBufs - 1) * NL));
    __syncthreads();
    read_a(0, avA);
    for (int b = 0; b < nblk; b += 2) {
        step(b, accA, accB, avA, avB, glB, fastB, glA, fastA);
        if (b + 1 < nblk) step(b + 1, accB, accA, avB, avA, glA, fastA, glB, fastB);
    }
    {  // the last block's hits
        uint64_t hit[2];
        if (nblk & 1) {
            precheck(accA, hit);
            examine(accA, glA, fastA, hit);
        } else {
            precheck(accB, hit);
            examine(accB, glB, fastB, hit);
        }
    }
    flush();
    // the re-reads issued past the end land before the LDS is released
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
}

// One workgroup per query of the pass: the k largest keys of its buffer, in
// descending order. When more than twice k candidates were kept, the keys
// stay in registers; a radix select over the scores (8 bits per round, each
// round's digit found by one wave) gives the k-th largest score and how many
// keys share it, a second select over library indices runs only among those
// ties when not all of them are kept, and only the k kept keys are translated
// from sorted rows to library indices and sorted (bitonic, in LDS).
constexpr int kMaxK = kCapacity / 8;  // largest k the search takes

__global__ __launch_bounds__(kThreads) void select_kernel(
    int64_t q_begin, int k, const uint32_t* __restrict__ count, const uint64_t* __restrict__ buf,
    const float* __restrict__ thr, const uint32_t* __restrict__ qperm,
    const int64_t* __restrict__ lo, const int64_t* __restrict__ hi,
    const uint32_t* __restrict__ lib_orig, int64_t* __restrict__ shortlist,
    uint8_t* __restrict__ fallback)
{
    __shared__ uint64_t s_sel[kMaxK];
    __shared__ uint32_t hist[256];
    __shared__ RadixDigit s_rd;
    __shared__ uint32_t s_nsel;
    const int64_t p = q_begin + blockIdx.x;
    const uint32_t qi = qperm[p];
    const int64_t w = hi[qi] - lo[qi];
    const uint32_t cnt = count[blockIdx.x * kCountStride];
    const int n = (int)min(cnt, (uint32_t)kCapacity);
    const int need = (int)min((int64_t)k, w);
    const bool sampled = thr[p] != -INFINITY;
    // fallback reason: 1 the buffer overflowed, 2 fewer than min(k, window)
    // candidates were kept, 3 the k-th kept scores below the threshold
    uint8_t why = cnt > (uint32_t)kCapacity ? 1 : (sampled && n < need) ? 2 : 0;
    bool bad = why != 0;
    const uint64_t* keys = buf + (size_t)blockIdx.x * kCapacity;
    const int kk = min(k, n);  // keys kept
    // The scoring kernel stored (score << 32 | sorted row); the result keys
    // are (score << 32 | ~library index), so that equal scores go to the
    // lower library index.
    auto lib_key = [&](uint64_t v) {
        return (v & 0xFFFFFFFF00000000ull) | (uint64_t)(0xFFFFFFFFu - lib_orig[(uint32_t)v]);
    };
    // a buffer of at most twice the kept count (and at most kMaxK keys) is
    // sorted whole; a larger one first has its kk-th key selected, so that
    // only the kept keys are translated and sorted
    const bool whole = n <= 2 * kk && n <= kMaxK;
    if (!bad && kk > 0) {  // uniform
        if (whole) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) s_sel[i] = lib_key(keys[i]);
        } else {
            constexpr int kPer = kCapacity / kThreads;
            uint64_t kv[kPer];  // this thread's keys, in registers
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int i = (int)threadIdx.x + j * kThreads;
                kv[j] = i < n ? keys[i] : 0ull;
            }
            // radix select of the kk-th largest score (high halves)
            uint32_t prefix = 0, mask = 0, r = (uint32_t)kk, eq = 0;
            for (int shift = 24; shift >= 0; shift -= 8) {
                for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kPer; ++j) {
                    const uint32_t h = (uint32_t)(kv[j] >> 32);
                    if ((int)threadIdx.x + j * kThreads < n && (h & mask) == prefix)
                        atomicAdd(&hist[(h >> shift) & 255u], 1u);
                }
                __syncthreads();
                if (threadIdx.x < 64) {
                    const RadixDigit rd = radix_digit(hist, r);
                    if (threadIdx.x == 0) s_rd = rd;
                }
                __syncthreads();
                prefix |= s_rd.digit << shift;
                mask |= 255u << shift;
                r -= s_rd.above;
                eq = s_rd.eq;
            }
            // Every key scoring above `prefix` is kept, and r of the eq keys
            // scoring exactly `prefix`: all of them when r == eq (the usual
            // case), else those with the r lowest library indices, found by a
            // second radix select over ~library index among the ties only.
            const bool all_ties = r == eq;
            uint32_t lp = 0, lmask = 0;
            if (!all_ties) {
                for (int shift = 24; shift >= 0; shift -= 8) {
                    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < kPer; ++j) {
                        if ((int)threadIdx.x + j * kThreads < n &&
                            (uint32_t)(kv[j] >> 32) == prefix) {
                            const uint32_t lw = (uint32_t)lib_key(kv[j]);
                            if ((lw & lmask) == lp) atomicAdd(&hist[(lw >> shift) & 255u], 1u);
                        }
                    }
                    __syncthreads();
                    if (threadIdx.x < 64) {
                        const RadixDigit rd = radix_digit(hist, r);
                        if (threadIdx.x == 0) s_rd = rd;
                    }
                    __syncthreads();
                    lp |= s_rd.digit << shift;
                    lmask |= 255u << shift;
                    r -= s_rd.above;
                }
            }
            // gather the kk kept keys, translated to library indices
            if (threadIdx.x == 0) s_nsel = 0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const uint32_t h = (uint32_t)(kv[j] >> 32);
                if ((int)threadIdx.x + j * kThreads >= n || h < prefix) continue;
                const uint64_t key = lib_key(kv[j]);
                if (h > prefix || all_ties || (uint32_t)key >= lp)
                    s_sel[atomicAdd(&s_nsel, 1u)] = key;
            }
        }
        __syncthreads();
        const int m = whole ? n : kk;  // keys now in s_sel
        int np = 1;
        while (np < m) np <<= 1;
        for (int i = m + threadIdx.x; i < np; i += blockDim.x) s_sel[i] = 0ull;
        __syncthreads();
        if (np > 1) bitonic_desc(s_sel, np);
        // Every window candidate scoring at or above thr is in the buffer
        // (pass 1 kept those, pass 0 kept more of its blocks); the kk kept
        // keys are the window's best only if the kk-th scores at least thr.
        if (sampled && (uint32_t)(s_sel[kk - 1] >> 32) < fkey(thr[p])) {
            bad = true;
            why = 3;
        }
    }
    int64_t* out = shortlist + (size_t)qi * k;
    for (int i = threadIdx.x; i < k; i += blockDim.x)
        out[i] = (!bad && i < kk) ? (int64_t)(0xFFFFFFFFu - (uint32_t)s_sel[i]) : -1;
    if (threadIdx.x == 0) fallback[qi] = why;
}

// one wave per query: exact distances of the shortlist, minimum merged
__global__ __launch_bounds__(kThreads) void rescore_kernel(
    int64_t q_begin, int64_t q_end, int k, uint32_t words, const uint32_t* __restrict__ q_hv,
    const uint32_t* __restrict__ qperm, const int64_t* __restrict__ shortlist,
    const uint32_t* __restrict__ lib_slot, const uint32_t* __restrict__ lib_hv,
    uint64_t* __restrict__ keys)
{
    const int64_t p = q_begin + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (p >= q_end) return;
    const uint32_t qi = qperm[p];
    const uint32_t* qrow = q_hv + (size_t)qi * words;
    const int64_t* sl = shortlist + (size_t)qi * k;
    // four entries per step, 16 lanes each: lane li of group g reads 16-byte
    // pieces li, li + 16, ... of entry base + g, so a load instruction takes
    // four contiguous 256-byte runs
    const int g = l >> 4, li = l & 15;
    const uint32_t nc = words / 4;  // 16-byte pieces per row
    const uint4* qp = (const uint4*)qrow;
    uint64_t best = ~0ull;
    for (int base = 0; base < k; base += 4) {
        const int j = base + g;
        const int64_t o = j < k ? sl[j] : -1;
        uint32_t d = 0;
        if (o >= 0) {
            const uint4* rp = (const uint4*)(lib_hv + (size_t)lib_slot[o] * words);
            for (uint32_t c = li; c < nc; c += 16) {
                const uint4 q4 = qp[c];
                const uint4 r4 = rp[c];
                d += __builtin_popcount(q4.x ^ r4.x) + __builtin_popcount(q4.y ^ r4.y) +
                     __builtin_popcount(q4.z ^ r4.z) + __builtin_popcount(q4.w ^ r4.w);
            }
        }
        d += __shfl_xor(d, 8);
        d += __shfl_xor(d, 4);
        d += __shfl_xor(d, 2);
        d += __shfl_xor(d, 1);
        if (o >= 0) {
            const uint64_t key = ((uint64_t)d << 32) | (uint64_t)o;
            best = key < best ? key : best;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t x = __shfl_xor(best, off);
        best = x < best ? x : best;
    }
    if (l == 0 && best != ~0ull)
        atomicMin((unsigned long long*)(keys + qi), (unsigned long long)best);
}

// list of the queries that fell back (order irrelevant: results merge by atomicMin)
__global__ void fallback_compact_kernel(int64_t nq, const uint8_t* __restrict__ fallback,
                                        uint32_t* __restrict__ list, uint32_t* __restrict__ count)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq && fallback[q]) list[atomicAdd(count, 1u)] = (uint32_t)q;
}

// Exhaustive pass over the windows of the listed queries: unit u = (library
// rows [(u / n) R, + R) clipped to the window of list entry u % n), n listed
// queries, one wave per unit, grid-stride so that a fixed launch covers any
// count. Units are block-major: the waves that run together read the same
// rows for different queries, so a block comes from HBM about once rather
// than once per query.
__global__ __launch_bounds__(kThreads) void fallback_scan_kernel(
    uint32_t words, const uint32_t* __restrict__ q_hv, const int64_t* __restrict__ lo,
    const int64_t* __restrict__ hi, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ count, int64_t max_units, const uint32_t* __restrict__ lib_hv,
    const uint32_t* __restrict__ lib_orig, uint64_t* __restrict__ keys)
{
    const int64_t n = (int64_t)*count;
    const int64_t total = n * max_units;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); u < total;
         u += waves) {
        const int64_t blk = u / n;
        const uint32_t qi = list[u - blk * n];
        const int64_t a = max(blk * kFallbackRows, lo[qi]);
        const int64_t b = min((blk + 1) * kFallbackRows, hi[qi]);
        if (a < b)  // wave-uniform
            popc::window_rows_wave(words, qi, q_hv, (uint32_t)a, (uint32_t)b, lib_hv, lib_orig,
                                   keys);
    }
}

__global__ void zero_u32_kernel(int64_t n, uint32_t* __restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Window candidates expected at or above each threshold for shortlists of k.
// Pass 1's target t2 leaves k a margin of four standard deviations of the
// count estimated from the r = t2 / kPassStride best pass-0 hits (relative
// spread about 1 / sqrt(r)): the smallest t2 with t2 - 4 sqrt(8 t2) >= k, and
// at least 256. The sampled threshold targets eight times that, between
// kCapacity / 4 and kCapacity / 2: on the widest windows the sample holds
// only a few rows per candidate above the threshold (r of 4 at 2,048 of 2.5M
// rows), and pass 0 must still find the r hits the refinement needs and,
// where it does not, keep at least k candidates itself.
void shortlist_targets(int k, int64_t* t1, int64_t* t2)
{
    const double c = 4.0 * std::sqrt((double)kPassStride);
    const double x = 0.5 * (c + std::sqrt(c * c + 4.0 * (double)k));
    *t2 = std::max<int64_t>(256, (int64_t)std::ceil(x * x));
    *t1 = std::min<int64_t>(kCapacity / 2, std::max<int64_t>(kCapacity / 4, 8 * *t2));
}

}  // namespace

int learned_max_k() { return kMaxK; }

bool learned_search_supports(int E) { return E == 64 || E == 128 || E == 256; }

size_t learned_scratch_bytes(int64_t nq, int64_t E, LearnedScratchPlan* plan)
{
    LearnedScratchPlan pl;
    const int64_t budget = (int64_t)1 << 30;  // bytes of candidate buffers per pass
    pl.batch = std::max<int64_t>(kTileQ, budget / ((int64_t)kCapacity * 8) / kTileQ * kTileQ);
    pl.batch = std::min<int64_t>(pl.batch, (nq + kTileQ - 1) / kTileQ * kTileQ);
    pl.batch = std::max<int64_t>(pl.batch, kTileQ);
    if (plan) *plan = pl;
    const int64_t tiles = pl.batch / kTileQ;
    return al(nq * E * 2) + al(nq * E) + 2 * al(nq * 4) + al(pl.batch * 4 * kCountStride) +
           al(pl.batch * (int64_t)kCapacity * 8) +
           2 * al(tiles * 8) + al(tiles * sizeof(SampleGrid)) + al(pl.batch * (int64_t)kSample * 4);
}

hipError_t launch_search_learned(const homs_ctx* c, const homs_model* m, void* scratch,
                                 const LearnedScratchPlan& plan, int64_t nq,
                                 const uint32_t* q_hv, const uint16_t* q_emb,
                                 const uint8_t* q_emb8, const uint32_t* qperm, const int64_t* lo,
                                 const int64_t* hi, int k, uint64_t* keys, uint8_t* fallback,
                                 int64_t* shortlist, const SpanHook& hook, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    const int E = m->E;
    if (!learned_search_supports(E)) return hipErrorInvalidValue;
    const int64_t tiles_max = plan.batch / kTileQ;
    char* p = (char*)scratch;
    uint16_t* q_sorted = (uint16_t*)p;
    p += al(nq * E * 2);
    uint8_t* q_sorted8 = (uint8_t*)p;
    p += al(nq * E);
    float* thr = (float*)p;
    p += al(nq * 4);
    float* thr2 = (float*)p;
    p += al(nq * 4);
    uint32_t* count = (uint32_t*)p;
    p += al(plan.batch * 4 * kCountStride);
    uint64_t* buf = (uint64_t*)p;
    p += al(plan.batch * (int64_t)kCapacity * 8);
    int64_t* tlo = (int64_t*)p;
    p += al(tiles_max * 8);
    int64_t* thi = (int64_t*)p;
    p += al(tiles_max * 8);
    SampleGrid* grids = (SampleGrid*)p;
    p += al(tiles_max * sizeof(SampleGrid));
    float* S = (float*)p;

    permute_rows_kernel<<<blocks_for(nq * (E / 8)), kThreads, 0, s>>>(nq, E, qperm, q_emb,
                                                                     q_sorted);
    permute_rows8_kernel<<<blocks_for(nq * (E / 16)), kThreads, 0, s>>>(nq, E, qperm, q_emb8,
                                                                       q_sorted8);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t max_chunks = (c->lib.n + kCollectChunk - 1) / kCollectChunk;
    if (max_chunks > 65535) return hipErrorInvalidConfiguration;
    int64_t t1, t2;
    shortlist_targets(k, &t1, &t2);
    for (int64_t b0 = 0; b0 < nq; b0 += plan.batch) {
        const int64_t b1 = std::min(nq, b0 + plan.batch), nb = b1 - b0;
        const int64_t tiles = (nb + kTileQ - 1) / kTileQ;
        e = launch_tile_bounds(nb, qperm + b0, lo, hi, kTileQ, tlo, thi, s);
        if (e != hipSuccess) return e;
        sample_scores_kernel<<<(uint32_t)(tiles * kSampleSplit), 256, 0, s>>>(
            E, b0, b1, q_sorted, tlo, thi, m->lib_emb, grids, S);
        threshold_kernel<<<(uint32_t)nb, kThreads, 0, s>>>(b0, t1, qperm, lo, hi, grids, S, thr);
        zero_u32_kernel<<<blocks_for(nb * kCountStride), kThreads, 0, s>>>(nb * kCountStride,
                                                                           count);
        hipEvent_t ea = hook.mark ? hook.mark(hook.user, s) : nullptr;
        // whole rounds of 8 chunks, so every XCD's sequence is complete
        const int64_t cwg = tiles * ((max_chunks + 7) / 8) * 8;
        if (cwg > 0x7FFFFFFF) return hipErrorInvalidConfiguration;
        const uint32_t cgrid = (uint32_t)cwg;
        auto collect = [&](auto pass_tag, const float* t) {
            constexpr int P = decltype(pass_tag)::value;
            constexpr int nt = 128 * kRowGroups;
            auto go = [&](auto kern) {
                kern<<<cgrid, nt, 0, s>>>(b0, b1, q_sorted8, qperm, lo, hi, t, tlo, thi,
                                          m->lib_emb8, count, buf, tiles, max_chunks);
            };
            if (E == 256) go(collect_kernel<256, P, kRowGroups>);
            else if (E == 128) go(collect_kernel<128, P, kRowGroups>);
            else go(collect_kernel<64, P, kRowGroups>);
        };
        // pass 0 with the sampled threshold, the refined threshold from its
        // hits, pass 1 with the refined one (same buffers, appended)
        collect(std::integral_constant<int, 0>{}, thr);
        refine_threshold_kernel<<<(uint32_t)nb, kThreads, 0, s>>>(b0, t2, qperm, lo, hi, count,
                                                                  buf, thr, thr2);
        collect(std::integral_constant<int, 1>{}, thr2);
        if (hook.mark && ea) hook.span(hook.user, ea, hook.mark(hook.user, s));
        select_kernel<<<(uint32_t)nb, kThreads, 0, s>>>(b0, k, count, buf, thr2, qperm, lo, hi,
                                                          c->lib.orig, shortlist, fallback);
        rescore_kernel<<<(uint32_t)((nb + 3) / 4), kThreads, 0, s>>>(
            b0, b1, k, c->words, q_hv, qperm, shortlist, c->lib.slot, c->lib.hv, keys);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t fallback_scratch_bytes(int64_t nq) { return al(nq * 4) + al(4); }

hipError_t launch_fallback_scan(const homs_ctx* c, int64_t nq, const uint32_t* q_hv,
                                const uint8_t* fallback, const int64_t* lo, const int64_t* hi,
                                void* scratch, uint64_t* keys, hipStream_t s)
{
    if (nq <= 0 || c->lib.n <= 0) return hipSuccess;
    uint32_t* list = (uint32_t*)scratch;
    uint32_t* count = (uint32_t*)((char*)scratch + al(nq * 4));
    zero_u32_kernel<<<1, 64, 0, s>>>(1, count);
    fallback_compact_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, fallback, list, count);
    const int64_t max_units = (c->lib.n + kFallbackRows - 1) / kFallbackRows;
    fallback_scan_kernel<<<2048, kThreads, 0, s>>>(c->words, q_hv, lo, hi, list, count, max_units,
                                                   c->lib.hv, c->lib.orig, keys);
    return hipGetLastError();
}

}  // namespace homs
