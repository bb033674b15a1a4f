// Open-window Hamming top-1 search on matrix cores (the precision form).
//
// With bit 0 standing for +1 and bit 1 for -1, the Hamming distance of two
// D-component vectors is H = (D - <x, y>) / 2 (the bipolar reading of
// Section 3.3 with the Hamming similarity of Section 3.4), and <x, y> over a
// window of candidates is a dense matrix product. Every partial sum is an
// integer of magnitude at most D <= 32768, exactly representable in int32 and
// in fp32 (int8 works on +-64 components: 4096 times the same integers), so
// every engine reproduces the popcount distances bit for bit.
//
// Work decomposition (every engine): a workgroup takes one tile of 256
// m/z-ordered queries and one chunk of its candidate rows, in blocks of 256
// library rows (the M dimension). Eight waves form a 2 x 4 grid; each owns a
// 128-row x 64-query accumulator tile (4 x 2 tiles of 32 x 32) in
// registers, so two waves share every SIMD and one wave's bit expansion
// overlaps the other's matrix instructions.
//
// Data movement (mfma_direct.h): the packed bits of a block's rows and of the
// tile's queries move into LDS in stages of 1,024 components by direct
// global-to-LDS loads, one stage ahead of their use; each wave reads its
// operand words from LDS and expands them in registers right before the
// matrix instructions, with one shift and one bit insert per 4 components
// (int8 +-64, fp8 +-1.0) or per 8 (fp4, asymmetric on the library side).
//
// Epilogue per block: distance = (Q - dot) / 2 (Q = D, or the fp4 form's
// per-query constant), masked by each query's own window and the chunk end,
// folded into a per-lane 64-bit running minimum of (distance << 32 | library
// index); lanes l and l+32 hold the same query columns and are merged with a
// shuffle before one atomicMin per query.
#include "internal.h"
#include "mfma_direct.h"

namespace homs {
namespace {

// XCD-aware work map of the direct kernels. Workgroups are handed
// to the eight XCDs in turn (workgroup i to XCD i mod 8), and each XCD has its
// own L2. Work items are (query tile, library chunk) pairs on absolute chunk
// boundaries; they are grouped into patches of 4 adjacent tiles x 8 adjacent
// chunks, and consecutive patches go to consecutive XCDs, so the 32
// workgroups an XCD runs side by side share 8 chunks of library rows and 4
// tiles of query rows (about 3 MB per 256-row step) in their L2.
constexpr int kXcds = 8, kPatchTiles = 4, kPatchChunks = 8;
constexpr int kPatch = kPatchTiles * kPatchChunks;

// wave layout of the one-shot kernels
using DirectLayout = mfd::Layout8;

template <int F>
__global__ __launch_bounds__(DirectLayout::kThreads, 1) void mfma_direct_kernel(uint32_t words,
    int64_t nq,
    const uint32_t* __restrict__ q_hv, const uint32_t* __restrict__ qperm,
    const int64_t* __restrict__ lo, const int64_t* __restrict__ hi,
    const int64_t* __restrict__ tlo, const int64_t* __restrict__ thi,
    const uint32_t* __restrict__ lib, const uint32_t* __restrict__ orig,
    const int32_t* __restrict__ qoff, const float* __restrict__ rowk,
    uint64_t* __restrict__ keys, int64_t chunk, int64_t n_tiles,
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
  mfd::tile_rows<F, true, DirectLayout>(words, nq, q_hv, qperm, lo, hi, tile, (uint32_t)a64,
                                        (uint32_t)b64, lib, orig, qoff, rowk, keys);
}

// 10 |x|_0 + 6 |x|_1 + 2 |x|_2 of a packed row, |x|_m its set bits at
// components of class m (component mod 4): the fp4 form's per-row constant
// K (and, plus 21D/4, its per-query constant Q); one wave per row
__device__ __forceinline__ int fp4_class_weight(const uint32_t* __restrict__ row, uint32_t words)
{
  const int l = threadIdx.x & 63;
  int s = 0;
  for (uint32_t i = l; i < words; i += 64) {
    const uint32_t w = row[i];
    s += 10 * __builtin_popcount(w & 0x11111111u) + 6 * __builtin_popcount(w & 0x22222222u) +
         2 * __builtin_popcount(w & 0x44444444u);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

__global__ __launch_bounds__(256) void fp4_query_offsets_kernel(int64_t nq, uint32_t words,
    const uint32_t* __restrict__ q_hv, int32_t* __restrict__ qoff)
{
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;
  const int s = fp4_class_weight(q_hv + (size_t)q * words, words);
  if ((threadIdx.x & 63) == 0) qoff[q] = s + (int)(21 * words * 8);  // 21D/4
}

// the per-row constants, n rows, then `pad` zeros
__global__ __launch_bounds__(256) void fp4_row_consts_kernel(int64_t n, int64_t pad, uint32_t words,
    const uint32_t* __restrict__ hv, float* __restrict__ rowk)
{
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n + pad) return;
  const int s = r < n ? fp4_class_weight(hv + (size_t)r * words, words) : 0;
  if ((threadIdx.x & 63) == 0) rowk[r] = (float)s;
}

constexpr int kMfQueries = mfd::kQueries;  // 256 per workgroup
constexpr int64_t kMfChunk = 4096;

}  // namespace

int search_mfma_tile() { return kMfQueries; }
int64_t search_mfma_row_pad() { return mfd::kRows; }

hipError_t launch_fp4_row_consts(int64_t n, uint32_t words, const uint32_t* hv, float* rowk,
                                 hipStream_t s)
{
  const int64_t pad = mfd::kRows;  // the epilogue reads whole groups past the last row
  if (n + pad <= 0) return hipSuccess;
  fp4_row_consts_kernel<<<(uint32_t)((n + pad + 3) / 4), 256, 0, s>>>(n, pad, words, hv, rowk);
  return hipGetLastError();
}

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
    const dim3 block(DirectLayout::kThreads);
    const int64_t tile_groups = (n_tiles + kPatchTiles - 1) / kPatchTiles;
    const int64_t chunk_patches = (max_chunks + kPatchChunks - 1) / kPatchChunks;
    const int64_t patches = tile_groups * chunk_patches;
    // whole rounds of kXcds patches, so every XCD's sequence is complete
    const int64_t blocks = (patches + kXcds - 1) / kXcds * kXcds * kPatch;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidConfiguration;
    if (fmt == 0) {
        mfma_direct_kernel<mfd::kFmtI8><<<(uint32_t)blocks, block, 0, s>>>(
            c->words, nq, q_hv, qperm, lo, hi, tile_lo, tile_hi, c->lib.hv, c->lib.orig,
            nullptr, nullptr, keys, kMfChunk, n_tiles, chunk_patches, patches);
    } else if (fmt == 1) {
        mfma_direct_kernel<mfd::kFmtF8><<<(uint32_t)blocks, block, 0, s>>>(
            c->words, nq, q_hv, qperm, lo, hi, tile_lo, tile_hi, c->lib.hv, c->lib.orig,
            nullptr, nullptr, keys, kMfChunk, n_tiles, chunk_patches, patches);
    } else {
        const hipError_t e = launch_fp4_query_offsets(c, nq, q_hv, qoff, s);
        if (e != hipSuccess) return e;
        mfma_direct_kernel<mfd::kFmtF4><<<(uint32_t)blocks, block, 0, s>>>(
            c->words, nq, q_hv, qperm, lo, hi, tile_lo, tile_hi, c->lib.hv, c->lib.orig,
            qoff, c->lib.rowk, keys, kMfChunk, n_tiles, chunk_patches, patches);
    }
    return hipGetLastError();
}

}  // namespace homs
