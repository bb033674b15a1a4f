// Device code of the XOR + popcount tile search, shared by the one-shot
// search kernel and the persistent batched kernel. See search_popc.hip for
// the design.
#pragma once

#include "internal.h"

namespace homs {
namespace popc {

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

// acc += popcount(row_word ^ query_word) as exactly v_xor_b32 (row word in
// an SGPR) + v_bcnt_u32_b32 with its built-in accumulate. Written out so the
// compiler cannot reassociate the sum into bcnt(x, 0) + add3 trees, which
// costs a third more VALU issue.
__device__ __forceinline__ void xor_popcount_add(uint32_t& acc, uint32_t row_word,
                                                 uint32_t query_word)
{
    uint32_t t;
    asm("v_xor_b32 %0, %1, %2" : "=v"(t) : "s"(row_word), "v"(query_word));
    asm("v_bcnt_u32_b32 %0, %1, %0" : "+v"(acc) : "v"(t));
}

// s_waitcnt with lgkmcnt(0) (vmcnt and expcnt left at their maxima): scalar
// loads return out of order, so only a full drain proves a group has landed
constexpr int kWaitScalar = 0xC07F;

// Scores rows [a, b) of the sorted library against the 256 queries of
// m/z-ordered tile `tile` (one per thread) and merges each query's best
// (distance, library index) into keys[] with a 64-bit atomicMin.
__device__ __forceinline__ void popcount_tile_rows(
    uint32_t words, int64_t nq, const uint32_t* __restrict__ q_hv,
    const uint32_t* __restrict__ qperm, const int64_t* __restrict__ lo,
    const int64_t* __restrict__ hi, int64_t tile, uint32_t a, uint32_t b,
    const uint32_t* __restrict__ lib_hv, const uint32_t* __restrict__ lib_orig,
    uint64_t* __restrict__ keys)
{
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
                    for (int i = 0; i < kWords; ++i) xor_popcount_add(acc[r0 + k], cur[k].v[i], qv[i]);
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

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

// One wave scores library rows [q_lo, q_hi) against query qi (one row per
// lane, query words through scalar loads, row words through 16-byte vector
// loads) and merges the wave's best (distance, library index) into keys[qi].
__device__ __forceinline__ void window_rows_wave(uint32_t words, uint32_t qi,
                                             const uint32_t* __restrict__ q_hv,
                                             uint32_t q_lo, uint32_t q_hi,
                                             const uint32_t* __restrict__ lib_hv,
                                             const uint32_t* __restrict__ lib_orig,
                                             uint64_t* __restrict__ keys)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t* qrow = q_hv + (size_t)qi * words;
    uint64_t best = ~0ull;
    for (uint32_t base = q_lo; base < q_hi; base += 64) {
        const uint32_t row = base + lane;
        const uint32_t rr = min(row, q_hi - 1u);
        const uint32_t* rp = lib_hv + (size_t)rr * words;
        uint32_t acc = 0;
        for (uint32_t c = 0; c < words; c += kWords) {
            const Slice qs = scalar_slice(qrow + c);
            uint32_t rv[kWords];
#pragma unroll
            for (int i = 0; i < kWords; i += 4) {
                const uint4 t = *reinterpret_cast<const uint4*>(rp + c + i);
                rv[i] = t.x;
                rv[i + 1] = t.y;
                rv[i + 2] = t.z;
                rv[i + 3] = t.w;
            }
#pragma unroll
            for (int i = 0; i < kWords; ++i) xor_popcount_add(acc, qs.v[i], rv[i]);
        }
        const uint64_t key =
            row < q_hi ? (((uint64_t)acc << 32) | (uint64_t)lib_orig[rr]) : ~0ull;
        best = key < best ? key : best;
    }
    best = wave_min_u64(best);
    if (lane == 0 && best != ~0ull)
        atomicMin(reinterpret_cast<unsigned long long*>(keys + qi), (unsigned long long)best);
}

}  // namespace popc
}  // namespace homs
