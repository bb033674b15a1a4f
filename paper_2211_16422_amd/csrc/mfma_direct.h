// Matrix-core search tile (int8, fp8 and fp4 engines of the one-shot search
// and the fp8 and fp4 engines of the batched persistent search): scores library rows [a, b) of the sorted
// library against the 256 m/z-ordered queries of tile `tile` (positions
// tile * 256 .. in qperm, of which the first nq exist) and merges each
// query's best (distance, library index) into keys[] with one 64-bit
// atomicMin. Needs a workgroup of 512 threads (8 waves in a 2 x 4 grid, each
// owning 128 rows x 64 queries of a 256 x 256 block), D a multiple of 512,
// and an orig array padded by 256 entries past the library.
//
// fp8: with bit 0 = +1 and bit 1 = -1 on both sides, H = (D - <x, y>) / 2,
// and <x, y> is an integer of magnitude <= D, exact in fp32.
//
// int8: the same components scaled to +-64 (0x40 / 0xC0, which, like the fp8
// bytes of +-1.0, differ only in the sign bit, so the expansion is the fp8
// one with another constant); the int32 dot product is 4096 (D - 2H), at most
// 2^27 in magnitude, and is shifted down by 12 before the same epilogue.
//
// fp4 (half the operand bytes and half the matrix cycles of fp8): both sides
// map component c of class m = c mod 4 with bit x to u_m + 2 x s_m, where
// (u, u + 2 s) = (4, 6), (2, 4), (0, 2), (1, -1): each pair differs in bit m
// of its e2m1 code alone (mantissa, exponent low, exponent high, sign), so
// the bit stays where it is in its word and one v_bfi_b32 (a v_and_b32 for
// class 2) expands 8 components, with no shift on either side. A product is
// u^2 + 2 u s (x + y) + 4 x y, so <x, y> = 21D/4 + sum_m 2 u_m s_m (|a|_m +
// |b|_m) + 4 a.b (|a|_m: a row's set bits of class m), and with H = |a| +
// |b| - 2 a.b: 2H = K(a) + Q(b) - <x, y>, where K(a) = 10 |a|_0 + 6 |a|_1 +
// 2 |a|_2 is a per-row constant (stored with the library as a float) and
// Q(b) = 21D/4 + 10 |b|_0 + 6 |b|_1 + 2 |b|_2 a per-query constant. The
// epilogue works on t = <x, y> - K (largest t = smallest H; H = (Q - t) / 2).
// Every product is an integer of magnitude <= 36 and every sum below 2^24,
// so t and H are exact.
//
// Data movement: the packed bits of the block's 256 library rows and 256
// query rows move into LDS in stages of 4 groups (1,024 components, one
// 128-byte line per row) by direct global-to-LDS loads, one stage ahead of
// their use, with one barrier per stage; every wave reads its operands from
// LDS (16 bytes per row and group) and expands them in registers right before
// the matrix instructions. Staging loads every line once per workgroup
// instead of once per wave, which was the bound of an earlier version whose
// lanes loaded their own operand rows from global memory.
#pragma once

#include <type_traits>

#include "internal.h"

namespace homs {
namespace mfd {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

// operand formats: 0 and 4 are the fp8 e4m3 and fp4 e2m1 codes of the
// f8f6f4 matrix instruction; kFmtI8 selects the int8 instruction
constexpr int kFmtF8 = 0, kFmtF4 = 4, kFmtI8 = 8;

// Wave layouts of the 256-row x 256-query workgroup tile: WR x WQ waves,
// each owning TR x TQ matrix tiles of 32 x 32 (TR 32-row tiles of library
// rows, TQ 32-query tiles). An expanded library operand feeds TQ matrix
// instructions and an expanded query operand TR of them.
template <int WR_, int WQ_, int TR_, int TQ_>
struct Layout {
  static constexpr int WR = WR_, WQ = WQ_, TR = TR_, TQ = TQ_;
  static constexpr int NW = WR * WQ;
  static constexpr int kThreads = 64 * NW;
  static constexpr int kRows = WR * TR * 32;
  static constexpr int kQueries = WQ * TQ * 32;
  static constexpr int kLoadRows = 256 / NW;  // rows of each operand a wave moves per stage
  static_assert(kRows == 256 && kQueries == 256, "256 x 256 workgroup tiles");
};
// 8 waves (two per SIMD) of 4 x 2 tiles: 8 accumulators of 16 registers
using Layout8 = Layout<2, 4, 4, 2>;
// 4 waves (one per SIMD) of 4 x 4 tiles: 16 accumulators (AGPRs), each
// expanded library operand feeding four matrix instructions
using Layout4 = Layout<2, 2, 4, 4>;

constexpr int kThreads = Layout8::kThreads;   // 512 (the persistent kernel's layout)
constexpr int kRows = 256;      // library rows per block step
constexpr int kQueries = 256;   // queries per tile

// s_waitcnt immediate: vmcnt(n), expcnt and lgkmcnt left at their maxima
constexpr int waitcnt_vm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x70 | 0xF00; }

// 32 packed bits -> 32 bytes of +-v whose two values differ only in the sign
// bit: fp8 e4m3 +-1.0 (0x38 / 0xB8) or int8 +-64 (0x40 / 0xC0). Byte j of
// dword m carries bit m + 8 j in its sign position: one shift and one
// v_bfi_b32 (bit insert of the sign into `one`, the +v byte repeated) per
// dword. This orders the components of a k group differently from the packed
// order, but the same way for both operands, which leaves every dot product
// unchanged. sel = 0x80808080 and one are passed in VGPRs (VOP3 takes no
// literal operands here).
__device__ __forceinline__ v8i expand_pm1(uint32_t w, uint32_t sel, uint32_t one) {
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

// 32 packed bits -> 32 fp4 e2m1 nibbles in the low four dwords of the operand
// (the fp4 form reads no others); nibble j of dword m is component m + 4 j of
// the word, the same order and the same map on both sides: the bit stays in
// place (bit m of the nibble) and selects between the codes of u_m and
// u_m + 2 s_m (sel[m] = 0x11111111 << m, base[m] = 0x66666666 (4.0),
// 0x44444444 (2.0), 0 (0.0), 0x22222222 (1.0)).
struct Fp4Consts {
  uint32_t c11, c22, c44, c88, c66;  // kept in VGPRs (VOP3 takes no literals)
};
__device__ __forceinline__ uint32_t bfi(uint32_t sel, uint32_t x, uint32_t y) {
  uint32_t r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(sel), "v"(x), "v"(y));
  return r;
}
__device__ __forceinline__ v8i expand_fp4(uint32_t w, const Fp4Consts& k) {
  v8i o = v8i{0};
  o[0] = (int)bfi(k.c11, w, k.c66);
  o[1] = (int)bfi(k.c22, w, k.c44);
  o[2] = (int)(w & k.c44);
  o[3] = (int)bfi(k.c88, w, k.c22);
  return o;
}

// dot product held in accumulator register r, exact in fp32: the fp32
// accumulators hold it as is, the int8 ones 4096 times it
__device__ __forceinline__ float dot_of(const v16f& a, int r) { return a[r]; }
__device__ __forceinline__ float dot_of(const v16i& a, int r) { return (float)(a[r] >> 12); }

// Stage buffers: per stage, 256 library rows and 256 query rows of kSG * 32
// bytes. The 16-byte piece p of row r is stored at position p ^ f(r) with
// f(r) = (r / kRPB) mod kP, so that the 16 rows read together by a quarter
// wave fall in 16 distinct bank groups. One allocation shared by both stage
// sizes (kSG = 4, or 2 when D / 256 is not a multiple of 4).
constexpr int kStageBytes = 2 * (kRows + kQueries) * 128;  // two 4-group stages
__device__ __forceinline__ char* stage_lds() {
  __shared__ __attribute__((aligned(16))) char buf[kStageBytes];
  return buf;
}
// library indices of each wave's rows of a block, two blocks in flight
__device__ __forceinline__ uint32_t* orig_lds() {
  __shared__ __attribute__((aligned(16))) uint32_t buf[2 * Layout8::NW * Layout8::TR * 32];
  return buf;
}
// the fp4 row constants K of the same rows
__device__ __forceinline__ float* rowk_lds() {
  __shared__ __attribute__((aligned(16))) float buf[2 * Layout8::NW * Layout8::TR * 32];
  return buf;
}

// qoff / rowk: the per-query constant Q and the per-row constant K of the fp4
// form (by query index and by sorted row, rowk padded like orig; unused by fp8
// and int8)
template <int F, int kSG, bool kAhead, class L>
__device__ __forceinline__ void tile_rows_staged(uint32_t words, int64_t nq,
    const uint32_t* __restrict__ q_hv, const uint32_t* __restrict__ qperm,
    const int64_t* __restrict__ lo, const int64_t* __restrict__ hi, int64_t tile, uint32_t a,
    uint32_t b, const uint32_t* __restrict__ lib, const uint32_t* __restrict__ orig,
    const int32_t* __restrict__ qoff, const float* __restrict__ rowk,
    uint64_t* __restrict__ keys)
{
  constexpr int MR = kRows, NQ = kQueries;
  constexpr int WR = L::WR, WQ = L::WQ, TR = L::TR, TQ = L::TQ, RPW = L::kLoadRows;
  static_assert(L::NW * TR <= Layout8::NW * Layout8::TR, "library index buffer");
  constexpr int kRowBytes = kSG * 32;    // bytes of a row per stage
  constexpr int kP = 2 * kSG;            // 16-byte pieces per row and stage
  constexpr int kRPB = 64 / (8 * kSG);   // rows between repeats of the bank pattern
  constexpr int kRPI = 64 / kP;          // rows per direct-load instruction
  constexpr int kLI = RPW / kRPI;        // instructions per wave and operand (RPW rows)
  constexpr int kBuf = (MR + NQ) * kRowBytes;
  static_assert(2 * kBuf <= kStageBytes, "stage buffers");
  const uint32_t D = words * 32;
  const int t = threadIdx.x, l = t & 63, w = t >> 6, wr = w % WR, wq = w / WR;
  const int h = l >> 5;
  char* const lds = stage_lds();
  uint32_t* const s_orig = orig_lds();
  float* const s_rowk = rowk_lds();

  // query columns of this lane (B rows and epilogue columns coincide);
  // distance = (Q - t) / 2: t the dot product and Q = D (fp8, int8), or t the
  // dot product minus the row's K and Q the query's constant (fp4)
  uint32_t qlo[TQ], qhi[TQ], qid[TQ];
  int Q[TQ];
  uint64_t bk[TQ];
  bool qok[TQ];
  float need[TQ];
#pragma unroll
  for (int j = 0; j < TQ; ++j) {
    const int64_t qs = tile * NQ + wq * TQ * 32 + j * 32 + (l & 31);
    qok[j] = qs < nq;
    qid[j] = qok[j] ? qperm[qs] : qperm[nq - 1];
    qlo[j] = qok[j] ? (uint32_t)lo[qid[j]] : 0u;
    qhi[j] = qok[j] ? (uint32_t)hi[qid[j]] : 0u;
    Q[j] = F == 4 ? qoff[qid[j]] : (int)D;
    bk[j] = ~0ull;
    // Dot product a row must reach to matter: that of the query's best so
    // far (from other workgroups; equal dots still matter for the index
    // rule). Absent queries never update.
    const uint64_t k0 = qok[j] ? keys[qid[j]] : 0ull;
    need[j] = !qok[j] ? INFINITY
              : k0 == ~0ull ? -INFINITY
                            : (float)(Q[j] - 2 * (int)(uint32_t)(k0 >> 32));
  }
  // query rows this lane moves into LDS: rows w * RPW + x * kRPI + l / kP
  const char* qld[kLI];
#pragma unroll
  for (int x = 0; x < kLI; ++x) {
    const int64_t qs = tile * NQ + w * RPW + x * kRPI + l / kP;
    const uint32_t qi = qs < nq ? qperm[qs] : qperm[nq - 1];
    qld[x] = (const char*)(q_hv + (size_t)qi * words);
  }
  // Consume these loads here: the compiler does not see the direct loads
  // below, and a wait of its own placed after them would drain them too.
#pragma unroll
  for (int j = 0; j < TQ; ++j)
    asm volatile("" : "+v"(qlo[j]), "+v"(qhi[j]), "+v"(qid[j]), "+v"(need[j]), "+v"(Q[j]));
#pragma unroll
  for (int x = 0; x < kLI; ++x) asm volatile("" : "+v"(qld[x]));

  const uint32_t SPB = words / (8 * kSG);  // stages per block
  const uint32_t nblk = (b - a + MR - 1) / MR;
  const uint32_t total = nblk * SPB;
  uint32_t sel = 0x80808080u, one = F == kFmtI8 ? 0x40404040u : 0x38383838u;  // int8 / fp8
  Fp4Consts k4{0x11111111u, 0x22222222u, 0x44444444u, 0x88888888u, 0x66666666u};
  if constexpr (F != kFmtF4)
    asm volatile("" : "+v"(sel), "+v"(one));  // keep in VGPRs
  else
    asm volatile("" : "+v"(k4.c11), "+v"(k4.c22), "+v"(k4.c44), "+v"(k4.c88), "+v"(k4.c66));

  // piece loaded by this lane in instruction x: LDS position l % kP of row
  // w * RPW + x * kRPI + l / kP holds piece position ^ f(row)
  auto lpos = [&](int x) {
    const uint32_t row = (uint32_t)(w * RPW + x * kRPI + l / kP);
    return (uint32_t)(l % kP) ^ ((row / kRPB) % kP);
  };
  // Stage S into buffer S % 2: library rows (clamped to the chunk's last
  // row) and query rows, preceded at a block's first stage by the block's
  // library indices. A direct load writes lane l's 16 (4) bytes to M0 + 16 l
  // (M0 + 4 l). 2 kLI loads per stage, 2 more at a block's first stage.
  auto issue = [&](uint32_t S) {
    const uint32_t B = S / SPB, sp = S % SPB;
    const uint32_t rb = a + B * MR;
    const uint32_t lim = b - 1u - rb;
    if (sp == 0) {
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const uint32_t voff = (rb + wr * TR * 32 + 64 * x + l) * 4u;  // orig is padded
        const uint32_t m0 = __builtin_amdgcn_readfirstlane(
            (uint32_t)(uintptr_t)(s_orig + ((B & 1) * WR * WQ + w) * TR * 32 + 64 * x));
        asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dword %0, %1"
                     :
                     : "v"(voff), "s"(orig), "s"(m0)
                     : "memory", "m0");
        if constexpr (F == kFmtF4) {  // the rows' K, same positions (rowk is padded)
          const uint32_t mk = __builtin_amdgcn_readfirstlane(
              (uint32_t)(uintptr_t)(s_rowk + ((B & 1) * WR * WQ + w) * TR * 32 + 64 * x));
          asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dword %0, %1"
                       :
                       : "v"(voff), "s"(rowk), "s"(mk)
                       : "memory", "m0");
        }
      }
    }
    char* const sA = lds + (S & 1) * kBuf;
    char* const sB = sA + MR * kRowBytes;
    const char* gA = (const char*)(lib + (size_t)rb * words);  // uniform
#pragma unroll
    for (int x = 0; x < kLI; ++x) {
      const uint32_t row = (uint32_t)(w * RPW + x * kRPI + l / kP);
      const uint32_t voff = min(row, lim) * words * 4u + sp * kRowBytes + lpos(x) * 16u;
      const uint32_t m0 = __builtin_amdgcn_readfirstlane(
          (uint32_t)(uintptr_t)(sA + (w * RPW + x * kRPI) * kRowBytes));
      asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1"
                   :
                   : "v"(voff), "s"(gA), "s"(m0)
                   : "memory", "m0");
    }
#pragma unroll
    for (int x = 0; x < kLI; ++x) {
      const char* src = qld[x] + sp * kRowBytes + lpos(x) * 16u;
      const uint32_t m0 = __builtin_amdgcn_readfirstlane(
          (uint32_t)(uintptr_t)(sB + (w * RPW + x * kRPI) * kRowBytes));
      asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off"
                   :
                   : "v"(src), "s"(m0)
                   : "memory", "m0");
    }
  };

  // Operand reads: row (l & 31) of a 32-row tile, piece 2 g + h (k half h of
  // group g takes words 4h .. 4h + 3 of the group's 8 words, the same for A
  // and B). Every tile of a wave starts at a multiple of 32 rows, so the
  // position of the piece depends on the lane only.
  const uint32_t r31 = (uint32_t)(l & 31);
  uint32_t roff[kSG];
#pragma unroll
  for (int g = 0; g < kSG; ++g)
    roff[g] = r31 * kRowBytes + 16u * ((uint32_t)(2 * g + h) ^ ((r31 / kRPB) % kP));

  issue(0);
  using Acc = typename std::conditional<F == kFmtI8, v16i, v16f>::type;
  Acc acc[TR][TQ];
  for (uint32_t S = 0; S < total; ++S) {
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));  // this wave's loads of stage S
    __syncthreads();  // every wave's loads landed; stage S - 1 is fully read
    if (S + 1 < total) issue(S + 1);
    const uint32_t sp = S % SPB;
    if (sp == 0) {
#pragma unroll
      for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TQ; ++j) acc[i][j] = Acc{0};
    }
    const char* bufA = lds + (S & 1) * kBuf + wr * TR * 32 * kRowBytes;
    const char* bufB = lds + (S & 1) * kBuf + MR * kRowBytes + wq * TQ * 32 * kRowBytes;
    // kAhead: the operand words of group g + 1 are read while group g
    // computes (the scheduling barrier keeps the compiler from sinking the
    // reads back to their use); 24 more registers
    uint4 pa[2][TR], pb[2][TQ];
    if constexpr (kAhead) {
#pragma unroll
      for (int i = 0; i < TR; ++i) pa[0][i] = *(const uint4*)(bufA + i * 32 * kRowBytes + roff[0]);
#pragma unroll
      for (int j = 0; j < TQ; ++j) pb[0][j] = *(const uint4*)(bufB + j * 32 * kRowBytes + roff[0]);
    }
#pragma unroll
    for (int g = 0; g < kSG; ++g) {
      uint4 ca[TR], cb[TQ];
      if constexpr (kAhead) {
        if (g + 1 < kSG) {
#pragma unroll
          for (int i = 0; i < TR; ++i)
            pa[(g + 1) & 1][i] = *(const uint4*)(bufA + i * 32 * kRowBytes + roff[g + 1]);
#pragma unroll
          for (int j = 0; j < TQ; ++j)
            pb[(g + 1) & 1][j] = *(const uint4*)(bufB + j * 32 * kRowBytes + roff[g + 1]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < TR; ++i) ca[i] = pa[g & 1][i];
#pragma unroll
        for (int j = 0; j < TQ; ++j) cb[j] = pb[g & 1][j];
      } else {
#pragma unroll
        for (int i = 0; i < TR; ++i) ca[i] = *(const uint4*)(bufA + i * 32 * kRowBytes + roff[g]);
#pragma unroll
        for (int j = 0; j < TQ; ++j) cb[j] = *(const uint4*)(bufB + j * 32 * kRowBytes + roff[g]);
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        v8i bv[TQ];
#pragma unroll
        for (int j = 0; j < TQ; ++j) {
          const uint32_t x = st == 0 ? cb[j].x : st == 1 ? cb[j].y : st == 2 ? cb[j].z : cb[j].w;
          if constexpr (F == kFmtF4)
            bv[j] = expand_fp4(x, k4);
          else
            bv[j] = expand_pm1(x, sel, one);
        }
#pragma unroll
        for (int i = 0; i < TR; ++i) {
          const uint32_t x = st == 0 ? ca[i].x : st == 1 ? ca[i].y : st == 2 ? ca[i].z : ca[i].w;
          v8i av;
          if constexpr (F == kFmtF4)
            av = expand_fp4(x, k4);
          else
            av = expand_pm1(x, sel, one);
#pragma unroll
          for (int j = 0; j < TQ; ++j) {
            if constexpr (F == kFmtI8) {
              // bytes 0-15 and 16-31 of each lane: two K = 32 halves of the
              // same 64 components, split alike on both operands
              const v4i a0 = {av[0], av[1], av[2], av[3]}, a1 = {av[4], av[5], av[6], av[7]};
              const v4i b0 = {bv[j][0], bv[j][1], bv[j][2], bv[j][3]};
              const v4i b1 = {bv[j][4], bv[j][5], bv[j][6], bv[j][7]};
              acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc[i][j], 0, 0, 0);
            } else {
              acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv[j], acc[i][j], F,
                                                                           F, 0, 0, 0, 0);
            }
          }
        }
      }
    }
    if (sp != SPB - 1) continue;

    // Epilogue of block blk. Accumulator register r of tile (i, j) holds row
    // base + 32 i + 8 (r / 4) + 4 (l / 32) + r % 4 and query column j; the
    // block's library indices are in LDS (their load is older than stage S's).
    const uint32_t blk = S / SPB;
    const uint32_t base = a + blk * MR + wr * TR * 32;
    const uint32_t* so = s_orig + ((blk & 1) * WR * WQ + w) * TR * 32 + 4 * (l >> 5);
    if constexpr (F == kFmtF4) {
      // fp4: t = <x, y> - K(row) in place (the accumulators restart with the
      // next block); from here on the epilogue is that of fp8 with t for the
      // dot product and Q(b) for D
      const float* sk = s_rowk + ((blk & 1) * WR * WQ + w) * TR * 32 + 4 * (l >> 5);
#pragma unroll
      for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) {
          const float4 kq = *(const float4*)(sk + i * 32 + 8 * rg);
          const float kv[4] = {kq.x, kq.y, kq.z, kq.w};
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4)
#pragma unroll
            for (int j = 0; j < TQ; ++j) acc[i][j][4 * rg + r4] -= kv[r4];
        }
    }
    bool inner = base + TR * 32 <= b;
#pragma unroll
    for (int j = 0; j < TQ; ++j)
      inner = inner && (!qok[j] || (qlo[j] <= base && base + TR * 32 <= qhi[j]));
    if (__ballot(!inner) == 0) {
      // every row of the wave is a candidate of every query column: the
      // column maximum decides, and only a maximum that reaches the best so
      // far looks up library indices
#pragma unroll
      for (int j = 0; j < TQ; ++j) {
        float m = dot_of(acc[0][j], 0);
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) m = fmaxf(m, dot_of(acc[i][j], r));
        if (m >= need[j]) {
          uint32_t o_min = ~0u;
#pragma unroll
          for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
              const uint4 o4 = *(const uint4*)(so + i * 32 + 8 * rg);
              const uint32_t ov[4] = {o4.x, o4.y, o4.z, o4.w};
#pragma unroll
              for (int r4 = 0; r4 < 4; ++r4)
                if (dot_of(acc[i][j], 4 * rg + r4) == m) o_min = min(o_min, ov[r4]);
            }
          const uint32_t d = (uint32_t)(Q[j] - (int)m) >> 1;
          const uint64_t key = ((uint64_t)d << 32) | o_min;
          bk[j] = key < bk[j] ? key : bk[j];
          need[j] = m;
        }
      }
    } else {
      // window or chunk edge inside the wave's rows: per-row masks
#pragma unroll
      for (int i = 0; i < TR; ++i) {
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) {
          const uint32_t g0 = base + i * 32 + 8 * rg + 4 * (l >> 5);
          const uint4 o4 = *(const uint4*)(so + i * 32 + 8 * rg);
          const uint32_t ov[4] = {o4.x, o4.y, o4.z, o4.w};
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) {
            const uint32_t g = g0 + r4;
#pragma unroll
            for (int j = 0; j < TQ; ++j) {
              const int dot = (int)dot_of(acc[i][j], 4 * rg + r4);
              const uint32_t d = (uint32_t)(Q[j] - dot) >> 1;
              const bool in = (g < b) && (g >= qlo[j]) && (g < qhi[j]);
              const uint64_t key = in ? (((uint64_t)d << 32) | ov[r4]) : ~0ull;
              bk[j] = key < bk[j] ? key : bk[j];
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < TQ; ++j)
        if (bk[j] != ~0ull)
          need[j] = fmaxf(need[j], (float)(Q[j] - 2 * (int)(uint32_t)(bk[j] >> 32)));
    }
  }
  __syncthreads();  // LDS is free again when the caller starts another tile
#pragma unroll
  for (int j = 0; j < TQ; ++j) {
    const uint64_t k = bk[j];
    const uint64_t k2 = __shfl_xor(k, 32);
    const uint64_t km = k < k2 ? k : k2;
    if (l < 32 && qok[j] && km != ~0ull)
      atomicMin((unsigned long long*)(keys + qid[j]), (unsigned long long)km);
  }
}

// 4-group stages when D / 256 is a multiple of 4, else 2-group stages;
// kAhead reads each group's operands one group early (for callers with 24
// registers to spare)
template <int F, bool kAhead = false, class L = Layout8>
__device__ __forceinline__ void tile_rows(uint32_t words, int64_t nq,
    const uint32_t* __restrict__ q_hv, const uint32_t* __restrict__ qperm,
    const int64_t* __restrict__ lo, const int64_t* __restrict__ hi, int64_t tile, uint32_t a,
    uint32_t b, const uint32_t* __restrict__ lib, const uint32_t* __restrict__ orig,
    const int32_t* __restrict__ qoff, const float* __restrict__ rowk,
    uint64_t* __restrict__ keys)
{
  if (words % 32 == 0)
    tile_rows_staged<F, 4, kAhead, L>(words, nq, q_hv, qperm, lo, hi, tile, a, b, lib, orig,
                                      qoff, rowk, keys);
  else
    tile_rows_staged<F, 2, kAhead, L>(words, nq, q_hv, qperm, lo, hi, tile, a, b, lib, orig,
                                      qoff, rowk, keys);
}

}  // namespace mfd
}  // namespace homs
