// Open-window Hamming top-1 search on matrix cores (the precision form).
//
// With bit 0 standing for +1 and bit 1 for -1, the Hamming distance of two
// D-component vectors is H = (D - <x, y>) / 2 (the bipolar reading of
// Section 3.3 with the Hamming similarity of Section 3.4), and <x, y> over a
// window of candidates is a dense matrix product. Every partial sum is an
// integer of magnitude at most D <= 32768, exactly representable in int32 and
// in fp32, so both engines reproduce the popcount distances bit for bit.
//
// Work decomposition (both engines): as in the popcount kernel, a workgroup
// takes one tile of 256 m/z-ordered queries and one chunk of its candidate
// rows, in blocks of 256 library rows (the M dimension). Eight waves form a
// 2 x 4 grid; each owns a 128-row x 64-query accumulator tile (4 x 2 tiles of
// 32 x 32) in VGPRs, so two waves share every SIMD and one wave's bit
// expansion overlaps the other's matrix instructions.
//
// int8 engine (mfma_search_kernel): the packed bits of the 256 rows and 256
// queries are read 64 components at a time and expanded once per workgroup
// to int8 +-1 bytes (a 4-bit group is spread to four bytes with one multiply
// and a mask, v_perm_b32 maps 0/1 bytes to +-1); the expanded stage (rows
// padded to 80 bytes so 16 lanes of a 16-byte LDS read touch 64 distinct
// banks) is double-buffered in LDS while the other buffer feeds the MFMAs.
//
// fp8 and fp4 engines (mfma_direct_kernel<F>): no LDS. Every lane loads the
// packed bits of its own operand rows and expands them in registers right
// before the matrix instructions, with one shift and one bit insert per 4
// (fp8) or 8 (fp4) components; an LDS variant of the fp8 engine spent as
// many LDS cycles on operand traffic as matrix cycles.
//
// Epilogue per block: distance = (D - dot) / 2, masked by each query's own
// window and the chunk end, folded into a per-lane 64-bit running minimum of
// (distance << 32 | library index); lanes l and l+32 hold the same query
// columns and are merged with a shuffle before one atomicMin per query.
#include "internal.h"
#include "mfma_direct.h"

namespace homs {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int KC = 64, LROW = 80, GRP = 4;

// 32 packed bits -> 32 bytes of +-1 in the encoding held by the byte table `lut`
__device__ __forceinline__ void expand32(uint32_t w, uint32_t lut, uint32_t* o) {
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const uint32_t nib = (w >> (4 * m)) & 0xFu;
    const uint32_t spread = (nib * 0x00204081u) & 0x01010101u;
    o[m] = __builtin_amdgcn_perm(0u, lut, spread);
  }
}

template <int FMT, int WR, int WQ, int TR, int TQ>
__global__ __launch_bounds__(64 * WR * WQ, 1) void mfma_search_kernel(uint32_t words, int64_t nq, const uint32_t* __restrict__ q_hv,
    const uint32_t* __restrict__ qperm, const int64_t* __restrict__ lo, const int64_t* __restrict__ hi,
    const int64_t* __restrict__ tlo, const int64_t* __restrict__ thi,
    const uint32_t* __restrict__ lib, const uint32_t* __restrict__ orig, uint64_t* __restrict__ keys, int64_t chunk)
{
  constexpr int NTHR = 64 * WR * WQ, MR = WR * TR * 32, NQ = WQ * TQ * 32;
  constexpr int ROWS = MR + NQ, RPT = (ROWS + NTHR - 1) / NTHR;
  static_assert(FMT == 0, "the LDS kernel is the int8 engine");
  typedef v16i AccT;
  __shared__ __attribute__((aligned(16))) uint8_t sbuf[2][ROWS * LROW];
  const int64_t tile = blockIdx.x;
  const int64_t a64 = tlo[tile] + (int64_t)blockIdx.y * chunk;
  const int64_t t_hi = thi[tile];
  if (a64 >= t_hi) return;
  const uint32_t a = (uint32_t)a64, b = (uint32_t)min(a64 + chunk, t_hi);
  const uint32_t D = words * 32;
  const int t = threadIdx.x, l = t & 63, w = t >> 6, wr = w % WR, wq = w / WR;
  const uint32_t lut = 0x0000FF01u;  // byte 0 -> +1 (0x01), byte 1 -> -1 (0xFF)

  // expansion rows of this thread: row < MR is a library row of the block,
  // row >= MR is query row - MR of the tile
  const uint32_t* qrow_e[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int row = t + k * NTHR;
    const int qrel = row - MR;
    const int64_t qs = tile * NQ + (qrel >= 0 && qrel < NQ ? qrel : 0);
    const uint32_t q = qs < nq ? qperm[qs] : 0u;
    qrow_e[k] = q_hv + (size_t)q * words;
  }

  uint32_t qlo[TQ], qhi[TQ], qid[TQ];
  uint64_t bk[TQ];
  bool qok[TQ];
#pragma unroll
  for (int j = 0; j < TQ; ++j) {
    const int64_t qs = tile * NQ + wq * TQ * 32 + j * 32 + (l & 31);
    qok[j] = qs < nq;
    qid[j] = qok[j] ? qperm[qs] : 0u;
    qlo[j] = qok[j] ? (uint32_t)lo[qid[j]] : 0u;
    qhi[j] = qok[j] ? (uint32_t)hi[qid[j]] : 0u;
    bk[j] = ~0ull;
  }

  const uint32_t S = words * 32 / KC;
  const uint32_t nblk = (b - a + MR - 1) / MR;
  const uint32_t T = nblk * S;

  uint4 p0[RPT][2], p1[RPT][2];
  auto load_group = [&](uint32_t g, uint4 (&d)[RPT][2]) {
    const uint32_t t0 = min(g, T / GRP - 1) * GRP;
    const uint32_t blk = t0 / S, s0 = t0 % S;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int row = t + k * NTHR;
      if (row < ROWS) {
        const uint32_t* src = row < MR ? lib + (size_t)min(a + blk * MR + (uint32_t)row, b - 1u) * words : qrow_e[k];
        const uint4* p = (const uint4*)((const uint8_t*)src + s0 * (KC / 8));
        d[k][0] = p[0]; d[k][1] = p[1];
      }
    }
  };
  auto expand_stage = [&](int j, const uint4 (&d)[RPT][2], int buf) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int row = t + k * NTHR;
      if (row < ROWS) {
        const uint4 v = d[k][j >> 1];
        const uint32_t x0 = (j & 1) ? v.z : v.x, x1 = (j & 1) ? v.w : v.y;
        uint32_t o[8];
        uint4* dst = (uint4*)(sbuf[buf] + row * LROW);
        expand32(x0, lut, o);
        dst[0] = make_uint4(o[0], o[1], o[2], o[3]); dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
        expand32(x1, lut, o);
        dst[2] = make_uint4(o[0], o[1], o[2], o[3]); dst[3] = make_uint4(o[4], o[5], o[6], o[7]);
      }
    }
  };
  auto mfma_stage = [&](int buf, AccT (&acc)[TR][TQ]) {
    const uint8_t* A = sbuf[buf];
    const uint8_t* B = sbuf[buf] + MR * LROW;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      v4i av[TR], bv[TQ];
#pragma unroll
      for (int i = 0; i < TR; ++i)
        av[i] = *(const v4i*)(A + (wr * TR * 32 + i * 32 + (l & 31)) * LROW + ks * 32 + 16 * (l >> 5));
#pragma unroll
      for (int j = 0; j < TQ; ++j)
        bv[j] = *(const v4i*)(B + (wq * TQ * 32 + j * 32 + (l & 31)) * LROW + ks * 32 + 16 * (l >> 5));
#pragma unroll
      for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TQ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  };

  load_group(0, p0);
  load_group(1, p1);
  expand_stage(0, p0, 0);
  __syncthreads();

  for (uint32_t blk = 0; blk < nblk; ++blk) {
    AccT acc[TR][TQ];
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
      for (int j = 0; j < TQ; ++j) acc[i][j] = AccT{0};
    for (uint32_t s = 0; s < S; s += 8) {
      const uint32_t g0 = (blk * S + s) / GRP;
      expand_stage(1, p0, 1); mfma_stage(0, acc); __syncthreads();
      expand_stage(2, p0, 0); mfma_stage(1, acc); __syncthreads();
      expand_stage(3, p0, 1); mfma_stage(0, acc); __syncthreads();
      expand_stage(0, p1, 0); mfma_stage(1, acc);
      load_group(g0 + 2, p0);
      __syncthreads();
      expand_stage(1, p1, 1); mfma_stage(0, acc); __syncthreads();
      expand_stage(2, p1, 0); mfma_stage(1, acc); __syncthreads();
      expand_stage(3, p1, 1); mfma_stage(0, acc); __syncthreads();
      expand_stage(0, p0, 0); mfma_stage(1, acc);
      load_group(g0 + 3, p1);
      __syncthreads();
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

// XCD-aware work map of the register-direct kernels. Workgroups are handed
// to the eight XCDs in turn (workgroup i to XCD i mod 8), and each XCD has its
// own L2. Work items are (query tile, library chunk) pairs on absolute chunk
// boundaries; they are grouped into patches of 4 adjacent tiles x 8 adjacent
// chunks, and consecutive patches go to consecutive XCDs, so the 32
// workgroups an XCD runs side by side share 8 chunks of library rows and 4
// tiles of query rows (about 3 MB per 256-row step) in their L2.
constexpr int kXcds = 8, kPatchTiles = 4, kPatchChunks = 8;
constexpr int kPatch = kPatchTiles * kPatchChunks;

template <int F>
__global__ __launch_bounds__(mfd::kThreads, 1) void mfma_direct_kernel(uint32_t words, int64_t nq,
    const uint32_t* __restrict__ q_hv, const uint32_t* __restrict__ qperm,
    const int64_t* __restrict__ lo, const int64_t* __restrict__ hi,
    const int64_t* __restrict__ tlo, const int64_t* __restrict__ thi,
    const uint32_t* __restrict__ lib, const uint32_t* __restrict__ orig,
    const int32_t* __restrict__ qoff, uint64_t* __restrict__ keys, int64_t chunk, int64_t n_tiles,
    int64_t chunk_patches, int64_t patches)
{
  const int64_t wg = blockIdx.x;
  const int64_t slot = wg / kXcds;  // position in this XCD's sequence
  const int64_t patch = (slot / kPatch) * kXcds + wg % kXcds;
  if (patch >= patches) return;
  const int local = (int)(slot % kPatch);
  const int64_t tile = (patch / chunk_patches) * kPatchTiles + local / kPatchChunks;
  const int64_t cidx = (patch % chunk_patches) * kPatchChunks + local % kPatchChunks;
  if (tile >= n_tiles) return;
  const int64_t a64 = max(cidx * chunk, tlo[tile]);
  const int64_t b64 = min(cidx * chunk + chunk, thi[tile]);
  if (a64 >= b64) return;
  mfd::tile_rows<F, true>(words, nq, q_hv, qperm, lo, hi, tile, (uint32_t)a64, (uint32_t)b64,
                          lib, orig, qoff, keys);
}

// The fp4 form's per-query constant Q = -3D/4 + 10 |b|_0 + 2 |b|_1 + 2 |b|_2,
// |b|_m the query's set bits at components of class m (component mod 4), one
// wave per query.
__global__ __launch_bounds__(256) void fp4_query_offsets_kernel(int64_t nq, uint32_t words,
    const uint32_t* __restrict__ q_hv, int32_t* __restrict__ qoff)
{
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (q >= nq) return;
  const uint32_t* row = q_hv + (size_t)q * words;
  int s = 0;
  for (uint32_t i = l; i < words; i += 64) {
    const uint32_t w = row[i];
    s += 10 * __builtin_popcount(w & 0x11111111u) + 2 * __builtin_popcount(w & 0x66666666u);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (l == 0) qoff[q] = s - (int)(3 * words * 8);
}

constexpr int kMfWR = 2, kMfWQ = 4, kMfTR = 4, kMfTQ = 2;
constexpr int kMfQueries = kMfWQ * kMfTQ * 32;  // 256 per workgroup
constexpr int64_t kMfChunk = 4096;

}  // namespace

int search_mfma_tile() { return kMfQueries; }
int64_t search_mfma_row_pad() { return kMfWR * kMfTR * 32; }

hipError_t launch_fp4_query_offsets(const homs_ctx* c, int64_t nq, const uint32_t* q_hv,
                                    int32_t* qoff, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    fp4_query_offsets_kernel<<<(uint32_t)((nq + 3) / 4), 256, 0, s>>>(nq, c->words, q_hv, qoff);
    return hipGetLastError();
}

hipError_t launch_search_mfma(const homs_ctx* c, int fmt, int64_t nq, const uint32_t* q_hv,
                              const uint32_t* qperm, const int64_t* lo, const int64_t* hi,
                              const int64_t* tile_lo, const int64_t* tile_hi, int32_t* qoff,
                              uint64_t* keys, hipStream_t s)
{
    const int64_t n_tiles = (nq + kMfQueries - 1) / kMfQueries;
    if (n_tiles <= 0 || c->lib.n <= 0) return hipSuccess;
    const int64_t max_chunks = (c->lib.n + kMfChunk - 1) / kMfChunk;
    if (max_chunks > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid((uint32_t)n_tiles, (uint32_t)max_chunks), block(64 * kMfWR * kMfWQ);
    if (fmt == 0)
        mfma_search_kernel<0, kMfWR, kMfWQ, kMfTR, kMfTQ><<<grid, block, 0, s>>>(
            c->words, nq, q_hv, qperm, lo, hi, tile_lo, tile_hi, c->lib.hv, c->lib.orig, keys,
            kMfChunk);
    else {
        const int64_t tile_groups = (n_tiles + kPatchTiles - 1) / kPatchTiles;
        const int64_t chunk_patches = (max_chunks + kPatchChunks - 1) / kPatchChunks;
        const int64_t patches = tile_groups * chunk_patches;
        // whole rounds of kXcds patches, so every XCD's sequence is complete
        const int64_t blocks = (patches + kXcds - 1) / kXcds * kXcds * kPatch;
        if (blocks > 0x7FFFFFFF) return hipErrorInvalidConfiguration;
        if (fmt == 1) {
            mfma_direct_kernel<0><<<(uint32_t)blocks, block, 0, s>>>(
                c->words, nq, q_hv, qperm, lo, hi, tile_lo, tile_hi, c->lib.hv, c->lib.orig,
                nullptr, keys, kMfChunk, n_tiles, chunk_patches, patches);
        } else {
            const hipError_t e = launch_fp4_query_offsets(c, nq, q_hv, qoff, s);
            if (e != hipSuccess) return e;
            mfma_direct_kernel<4><<<(uint32_t)blocks, block, 0, s>>>(
                c->words, nq, q_hv, qperm, lo, hi, tile_lo, tile_hi, c->lib.hv, c->lib.orig,
                qoff, keys, kMfChunk, n_tiles, chunk_patches, patches);
        }
    }
    return hipGetLastError();
}

}  // namespace homs
