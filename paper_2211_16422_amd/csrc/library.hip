// Library layout, candidate windows and result keys.
//
// The library is sorted once by (charge, precursor m/z, library index) so
// that the candidates of a query (same charge, precursor m/z within the
// tolerance; Section 3.4) form one contiguous range of sorted rows, found by
// two binary searches in float64. Results travel as 64-bit keys
// (distance << 32 | library index): the smallest key is the smallest
// distance with ties to the lowest library index, so partial results of
// different workgroups merge with one 64-bit atomicMin. The sorts are the
// stable radix sort of sort_scan.hip.
#include "internal.h"

namespace homs {
namespace {

constexpr int kThreads = 256;

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + kThreads - 1) / kThreads); }

// Order-preserving map of a double onto uint64 (negative values reversed).
// Values that compare equal get one key: -0 sorts as +0, and every NaN as
// one NaN after +inf, so rows of equal precursors stay in library order.
__device__ __forceinline__ uint64_t order_key(double x)
{
    if (x == 0.0) x = 0.0;
    const uint64_t b = (x != x) ? 0x7FF8000000000000ull : (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void make_keys_kernel(int64_t n, const double* __restrict__ pmz,
                                 uint64_t* __restrict__ k64, uint32_t* __restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    k64[i] = order_key(pmz[i]);
    vals[i] = (uint32_t)i;
}

// second sort key: the charge of each row in the order of the first sort
__global__ void charge_keys_kernel(int64_t n, const int8_t* __restrict__ charge, bool use_charge,
                                   const uint32_t* __restrict__ perm, uint64_t* __restrict__ k)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    k[i] = use_charge ? (uint64_t)((uint8_t)charge[perm[i]] ^ 0x80u) : 0ull;
}

__global__ void scatter_sorted_kernel(int64_t n, const uint32_t* __restrict__ perm,
                                      const double* __restrict__ pmz,
                                      const int8_t* __restrict__ charge, bool use_charge,
                                      double* __restrict__ pmz_out, int8_t* __restrict__ charge_out,
                                      uint32_t* __restrict__ slot)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t i = perm[j];
    pmz_out[j] = pmz[i];
    charge_out[j] = use_charge ? charge[i] : (int8_t)0;
    slot[i] = (uint32_t)j;
}

__global__ void slot_kernel(int64_t n, const uint32_t* __restrict__ orig, uint32_t* __restrict__ slot)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) slot[orig[j]] = (uint32_t)j;
}

__global__ void gather_rows_kernel(int64_t n, uint32_t w4, const uint4* __restrict__ src,
                                   const uint32_t* __restrict__ orig, uint4* __restrict__ dst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * (int64_t)w4) return;
    const int64_t j = t / w4;
    const uint32_t w = (uint32_t)(t - j * w4);
    dst[(size_t)orig[j] * w4 + w] = src[(size_t)j * w4 + w];
}

// first j in [0, n) with (ch[j], pmz[j]) >= (c, x) (strict: > when `upper`)
__device__ __forceinline__ int64_t lex_bound(const int8_t* __restrict__ ch,
                                             const double* __restrict__ pmz, int64_t n, int8_t c,
                                             double x, bool upper)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const int8_t cm = ch[mid];
        bool before;  // row mid precedes the bound
        if (cm != c)
            before = cm < c;
        else
            before = upper ? (pmz[mid] <= x) : (pmz[mid] < x);
        if (before)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ void window_kernel(int64_t nq, const double* __restrict__ q_pmz,
                              const int8_t* __restrict__ q_charge, bool use_charge, int32_t kind,
                              double value, const int8_t* __restrict__ kinds,
                              const double* __restrict__ values, const double* __restrict__ lib_pmz,
                              const int8_t* __restrict__ lib_charge, int64_t nlib,
                              int64_t* __restrict__ lo_out, int64_t* __restrict__ hi_out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const double pmz = q_pmz[q];
    const int32_t k = kinds ? (int32_t)kinds[q] : kind;
    const double v = values ? values[q] : value;
    // tolerance in Da, or ppm of the precursor m/z: (pmz * v) / 1e6
    const double tol = (k == HOMS_TOL_DA) ? v : __ddiv_rn(__dmul_rn(pmz, v), 1.0e6);
    const double lo_b = __dsub_rn(pmz, tol);
    const double hi_b = __dadd_rn(pmz, tol);
    const int8_t c = use_charge ? q_charge[q] : (int8_t)0;
    const int64_t lo = lex_bound(lib_charge, lib_pmz, nlib, c, lo_b, false);
    int64_t hi = lex_bound(lib_charge, lib_pmz, nlib, c, hi_b, true);
    if (hi < lo) hi = lo;  // NaN precursor or negative tolerance: empty
    lo_out[q] = lo;
    hi_out[q] = hi;
}

__global__ void query_keys_kernel(int64_t nq, const double* __restrict__ q_pmz,
                                  const int8_t* __restrict__ q_charge, bool use_charge,
                                  uint64_t* __restrict__ k, uint32_t* __restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    // charge in the top 8 bits, the upper 56 bits of the ordered m/z below;
    // the order only shapes tiles, results never depend on it
    const uint64_t ch = use_charge ? (uint64_t)((uint8_t)q_charge[i] ^ 0x80u) : 0ull;
    k[i] = (ch << 56) | (order_key(q_pmz[i]) >> 8);
    vals[i] = (uint32_t)i;
}

__global__ void init_keys_kernel(int64_t n, uint64_t* __restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = ~0ull;
}

__global__ void finalize_kernel(int64_t n, const uint64_t* __restrict__ keys,
                                int64_t* __restrict__ idx, int32_t* __restrict__ dist)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    if (k == ~0ull) {
        idx[i] = -1;
        dist[i] = -1;
    } else {
        idx[i] = (int64_t)(uint32_t)k;
        dist[i] = (int32_t)(k >> 32);
    }
}

// one workgroup per query; each thread computes whole distances of candidates
__global__ void debug_distances_kernel(int64_t nq, uint32_t words, const uint32_t* __restrict__ q_hv,
                                       const uint32_t* __restrict__ lib_hv,
                                       const uint32_t* __restrict__ orig,
                                       const int64_t* __restrict__ lo,
                                       const int64_t* __restrict__ hi,
                                       const int64_t* __restrict__ row_off,
                                       int64_t* __restrict__ out_idx, int32_t* __restrict__ out_dist)
{
    const int64_t q = blockIdx.x;
    if (q >= nq) return;
    const uint32_t* qr = q_hv + (size_t)q * words;
    for (int64_t j = lo[q] + threadIdx.x; j < hi[q]; j += blockDim.x) {
        const uint32_t* rr = lib_hv + (size_t)j * words;
        int32_t d = 0;
        for (uint32_t w = 0; w < words; ++w) d += __popc(qr[w] ^ rr[w]);
        const int64_t o = row_off[q] + (j - lo[q]);
        out_idx[o] = (int64_t)orig[j];
        out_dist[o] = d;
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ---------------------------------------------------------------------------

size_t library_sort_temp_bytes(int64_t n)
{
    return 2 * align_up((size_t)n * 8) + align_up((size_t)n * 4) + radix_sort_temp_bytes(n);
}

hipError_t launch_library_sort(int64_t n, const double* pmz, const int8_t* charge, bool use_charge,
                               void* temp, size_t temp_bytes, uint32_t* perm_out, double* pmz_out,
                               int8_t* charge_out, uint32_t* slot_out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    char* p = (char*)temp;
    uint64_t* ka = (uint64_t*)p;
    p += align_up((size_t)n * 8);
    uint64_t* kb = (uint64_t*)p;
    p += align_up((size_t)n * 8);
    uint32_t* va = (uint32_t*)p;
    p += align_up((size_t)n * 4);
    void* sort_tmp = p;
    p += radix_sort_temp_bytes(n);
    if ((size_t)(p - (char*)temp) > temp_bytes) return hipErrorInvalidValue;

    // stable sort by precursor m/z (8 passes: back in ka / va), then a stable
    // pass by charge (into kb's partner ka and perm_out): ties of both keys
    // keep library order
    make_keys_kernel<<<blocks_for(n), kThreads, 0, s>>>(n, pmz, ka, va);
    bool alt = false;
    hipError_t e = radix_sort_pairs(n, ka, kb, va, slot_out, 0, 64, sort_tmp, s, &alt);
    if (e != hipSuccess) return e;
    if (alt) return hipErrorInvalidValue;  // an even number of passes ends in ka / va
    charge_keys_kernel<<<blocks_for(n), kThreads, 0, s>>>(n, charge, use_charge, va, kb);
    e = radix_sort_pairs(n, kb, ka, va, perm_out, 0, 8, sort_tmp, s, &alt);
    if (e != hipSuccess) return e;
    if (!alt) return hipErrorInvalidValue;  // one pass ends in ka / perm_out
    scatter_sorted_kernel<<<blocks_for(n), kThreads, 0, s>>>(n, perm_out, pmz, charge, use_charge,
                                                             pmz_out, charge_out, slot_out);
    return hipGetLastError();
}

hipError_t launch_slots(int64_t n, const uint32_t* orig, uint32_t* slot, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    slot_kernel<<<blocks_for(n), kThreads, 0, s>>>(n, orig, slot);
    return hipGetLastError();
}

hipError_t launch_gather_rows(int64_t n, uint32_t words, const uint32_t* src, const uint32_t* orig,
                              uint32_t* dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const uint32_t w4 = words / 4;
    gather_rows_kernel<<<blocks_for(n * (int64_t)w4), kThreads, 0, s>>>(
        n, w4, (const uint4*)src, orig, (uint4*)dst);
    return hipGetLastError();
}

hipError_t launch_window_bounds(const homs_ctx* c, int64_t nq, const double* q_pmz,
                                const int8_t* q_charge, int32_t kind, double value,
                                const int8_t* kinds, const double* values, int64_t* lo,
                                int64_t* hi, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    window_kernel<<<blocks_for(nq), kThreads, 0, s>>>(
        nq, q_pmz, q_charge, c->p.charge_match != 0, kind, value, kinds, values, c->lib.pmz,
        c->lib.charge, c->lib.n, lo, hi);
    return hipGetLastError();
}

size_t query_sort_temp_bytes(int64_t nq) { return radix_sort_temp_bytes(nq); }

hipError_t launch_query_sort(int64_t nq, const double* q_pmz, const int8_t* q_charge,
                             bool use_charge, void* temp, size_t temp_bytes, uint64_t* keys_a,
                             uint64_t* keys_b, uint32_t* perm_a, uint32_t* perm_b,
                             uint32_t** perm_out, hipStream_t s)
{
    *perm_out = perm_a;
    if (nq <= 0) return hipSuccess;
    if (temp_bytes < radix_sort_temp_bytes(nq)) return hipErrorInvalidValue;
    query_keys_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, q_pmz, q_charge, use_charge, keys_a,
                                                          perm_a);
    // the charge and the upper 32 bits of the ordered m/z (relative resolution
    // 2^-20) are enough to make tiles of neighbouring precursors
    bool alt = false;
    hipError_t e = radix_sort_pairs(nq, keys_a, keys_b, perm_a, perm_b, 24, 64, temp, s, &alt);
    *perm_out = alt ? perm_b : perm_a;
    return e;
}

hipError_t launch_init_keys(int64_t nq, uint64_t* keys, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    init_keys_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, keys);
    return hipGetLastError();
}

hipError_t launch_finalize(int64_t nq, const uint64_t* keys, int64_t* idx, int32_t* dist,
                           hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    finalize_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, keys, idx, dist);
    return hipGetLastError();
}

hipError_t launch_debug_distances(const homs_ctx* c, int64_t nq, const uint32_t* q_hv,
                                  const int64_t* lo, const int64_t* hi, const int64_t* row_off,
                                  int64_t* out_idx, int32_t* out_dist, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    debug_distances_kernel<<<(uint32_t)nq, kThreads, 0, s>>>(nq, c->words, q_hv, c->lib.hv,
                                                             c->lib.orig, lo, hi, row_off, out_idx,
                                                             out_dist);
    return hipGetLastError();
}

}  // namespace homs
