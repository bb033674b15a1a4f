// Register-direct matrix-core search tile: scores library rows [a, b) of the
// sorted library against the 256 m/z-ordered queries of tile `tile`
// (positions tile * 256 .. in qperm, of which the first nq exist) and merges
// each query's best (distance, library index) into keys[] with one 64-bit
// atomicMin. Used by the fp8 and fp4 engines of the one-shot search and by
// the batched persistent search. Needs a workgroup of 512 threads (8 waves in
// a 2 x 4 grid, each owning 128 rows x 64 queries of a 256 x 256 block), D a
// multiple of 512, and an orig array padded by 256 entries past the library.
//
// With bit 0 = +1 and bit 1 = -1, H = (D - <x, y>) / 2 and <x, y> is exact in
// fp32 (integers of magnitude <= D), so the distances equal the popcount
// ones bit for bit. +-1 is exact in both element formats (fp8 e4m3 0x38 /
// 0xB8, fp4 e2m1 0x2 / 0xA), and so is every product. No LDS: every lane
// loads the packed bits of its own operand rows from global memory one group
// (256 components) ahead and expands them in registers right before the
// matrix instructions. fp4 operands take half the register bytes and half
// the matrix cycles of fp8 ones for the same 64 components.
#pragma once

#include "internal.h"

namespace homs {
namespace mfd {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int WR = 2, WQ = 4, TR = 4, TQ = 2;
constexpr int kThreads = 64 * WR * WQ;   // 512
constexpr int kRows = WR * TR * 32;      // library rows per block step (256)
constexpr int kQueries = WQ * TQ * 32;   // queries per tile (256)

// 32 packed bits -> 32 fp8 e4m3 bytes of +-1.0 (0x38 / 0xB8). Byte j of dword
// m carries bit m + 8 j in its sign position: one shift and one v_bfi_b32
// (bit insert of the sign into 0x38383838) per dword. This orders the
// components of a k group differently from the packed order, but the same
// way for both operands, which leaves every dot product unchanged. sel =
// 0x80808080 and one = 0x38383838 are passed in VGPRs (VOP3 takes no
// literal operands here).
__device__ __forceinline__ v8i expand_pm1_fp8(uint32_t w, uint32_t sel, uint32_t one) {
  v8i o;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const uint32_t x = w << (7 - m);
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(sel), "v"(x), "v"(one));
    o[m] = (int)r;
  }
  return o;
}

// 32 packed bits -> 32 fp4 e2m1 nibbles of +-1.0 (0x2 / 0xA) in the low four
// dwords of the operand (the fp4 form reads no others). Nibble j of dword m
// carries bit m + 4 j in its sign position: one shift and one bit insert per
// 8 components, the same order for both operands.
__device__ __forceinline__ v8i expand_pm1_fp4(uint32_t w, uint32_t sel, uint32_t one) {
  v8i o = v8i{0};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const uint32_t x = w << (3 - m);
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(sel), "v"(x), "v"(one));
    o[m] = (int)r;
  }
  return o;
}

// element format code of the f8f6f4 matrix instruction: 0 = fp8 e4m3, 4 = fp4 e2m1
template <int F>
__device__ __forceinline__ v8i expand_pm1(uint32_t w, uint32_t sel, uint32_t one) {
  static_assert(F == 0 || F == 4, "fp8 e4m3 or fp4 e2m1");
  if constexpr (F == 0)
    return expand_pm1_fp8(w, sel, one);
  else
    return expand_pm1_fp4(w, sel, one);
}

// Operand loads: within a group of 256 components (8 words per row), k half h
// of every 32 x 32 x 64 step takes words 4h .. 4h + 3 of the group, stage s
// word 4h + s, so each lane fetches 16 bytes per row per group; A (library
// rows) and B (queries) use the same assignment. The next group is in flight
// while the current one is expanded and multiplied. The four waves of a row
// half share library rows, and the two waves of a query quarter share query
// rows, through L1.
template <int F>
__device__ __forceinline__ void tile_rows(uint32_t words, int64_t nq,
    const uint32_t* __restrict__ q_hv, const uint32_t* __restrict__ qperm,
    const int64_t* __restrict__ lo, const int64_t* __restrict__ hi, int64_t tile, uint32_t a,
    uint32_t b, const uint32_t* __restrict__ lib, const uint32_t* __restrict__ orig,
    uint64_t* __restrict__ keys)
{
  constexpr int MR = kRows, NQ = kQueries;
  const uint32_t D = words * 32;
  const int t = threadIdx.x, l = t & 63, w = t >> 6, wr = w % WR, wq = w / WR;
  const int h = l >> 5;

  // query columns of this lane (B rows and epilogue columns coincide)
  const uint32_t* qrow[TQ];
  uint32_t qlo[TQ], qhi[TQ], qid[TQ];
  uint64_t bk[TQ];
  bool qok[TQ];
#pragma unroll
  for (int j = 0; j < TQ; ++j) {
    const int64_t qs = tile * NQ + wq * TQ * 32 + j * 32 + (l & 31);
    qok[j] = qs < nq;
    qid[j] = qok[j] ? qperm[qs] : qperm[nq - 1];
    qlo[j] = qok[j] ? (uint32_t)lo[qid[j]] : 0u;
    qhi[j] = qok[j] ? (uint32_t)hi[qid[j]] : 0u;
    qrow[j] = q_hv + (size_t)qid[j] * words + 4 * h;
    bk[j] = ~0ull;
  }
  const uint32_t G = words / 8;
  const uint32_t nblk = (b - a + MR - 1) / MR;
  uint32_t sel = F == 0 ? 0x80808080u : 0x88888888u, one = F == 0 ? 0x38383838u : 0x22222222u;
  asm volatile("" : "+v"(sel), "+v"(one));  // keep both in VGPRs

  for (uint32_t blk = 0; blk < nblk; ++blk) {
    const uint32_t* arow[TR];
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const uint32_t row = a + blk * MR + wr * TR * 32 + i * 32 + (l & 31);
      arow[i] = lib + (size_t)min(row, b - 1u) * words + 4 * h;
    }
    v16f acc[TR][TQ];
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
      for (int j = 0; j < TQ; ++j) acc[i][j] = v16f{0};
    // packed words of two groups in flight: x* is consumed while y* loads
    uint4 xa[TR], xb[TQ], ya[TR], yb[TQ];
    auto load = [&](uint32_t g, uint4 (&da)[TR], uint4 (&db)[TQ]) {
      const uint32_t off = (g < G ? g : G - 1) * 8;
#pragma unroll
      for (int i = 0; i < TR; ++i) da[i] = *(const uint4*)(arow[i] + off);
#pragma unroll
      for (int j = 0; j < TQ; ++j) db[j] = *(const uint4*)(qrow[j] + off);
      __builtin_amdgcn_sched_barrier(0);  // issued before the group's work
    };
    auto group = [&](const uint4 (&ca)[TR], const uint4 (&cb)[TQ]) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        v8i bv[TQ];
#pragma unroll
        for (int j = 0; j < TQ; ++j) {
          const uint32_t x = st == 0 ? cb[j].x : st == 1 ? cb[j].y : st == 2 ? cb[j].z : cb[j].w;
          bv[j] = expand_pm1<F>(x, sel, one);
        }
#pragma unroll
        for (int i = 0; i < TR; ++i) {
          const uint32_t x = st == 0 ? ca[i].x : st == 1 ? ca[i].y : st == 2 ? ca[i].z : ca[i].w;
          const v8i av = expand_pm1<F>(x, sel, one);
#pragma unroll
          for (int j = 0; j < TQ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv[j], acc[i][j], F, F,
                                                                         0, 0, 0, 0);
        }
      }
    };
    load(0, xa, xb);
    for (uint32_t g = 0; g < G; g += 2) {  // G = D / 256 is even
      load(g + 1, ya, yb);
      group(xa, xb);
      load(g + 2, xa, xb);
      group(ya, yb);
    }
    const uint32_t base = a + blk * MR + wr * TR * 32;
#pragma unroll
    for (int i = 0; i < TR; ++i) {
#pragma unroll
      for (int rg = 0; rg < 4; ++rg) {
        const uint32_t g0 = base + i * 32 + 8 * rg + 4 * (l >> 5);
        const uint4 o4 = *(const uint4*)(orig + g0);  // orig is padded past the end
        const uint32_t ov[4] = {o4.x, o4.y, o4.z, o4.w};
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          const uint32_t g = g0 + r4;
#pragma unroll
          for (int j = 0; j < TQ; ++j) {
            const int dot = (int)acc[i][j][4 * rg + r4];
            const uint32_t d = (uint32_t)((int)D - dot) >> 1;
            const bool in = (g < b) && (g >= qlo[j]) && (g < qhi[j]);
            const uint64_t key = in ? (((uint64_t)d << 32) | ov[r4]) : ~0ull;
            bk[j] = key < bk[j] ? key : bk[j];
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < TQ; ++j) {
    const uint64_t k = bk[j];
    const uint64_t k2 = __shfl_xor(k, 32);
    const uint64_t km = k < k2 ? k : k2;
    if (l < 32 && qok[j] && km != ~0ull)
      atomicMin((unsigned long long*)(keys + qid[j]), (unsigned long long)km);
  }
}


}  // namespace mfd
}  // namespace homs
