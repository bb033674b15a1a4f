// Cascade search (Section 3.4) with target-decoy FDR filtering (Section 2.1,
// at the fixed 1% level of Section 4.1): the kernels between the two search
// stages.
//
// A stage's PSMs are the top-1 matches of the queries it searched; a PSM is a
// decoy match when its library entry is a decoy. FDR at distance threshold d
// (accept every PSM at distance <= d) is decoys / targets among those PSMs,
// undefined (never accepted) without a target; a PSM's q-value is the
// minimum FDR over thresholds d' >= its distance; targets with q-value <= the
// level are identifications. Because distances are integers in [0, D], the
// FDR needs no sort: a histogram of targets and decoys by distance, one scan
// for the cumulative counts and FDR(d), one reverse scan for the running
// minimum. Counts are exact integers and FDR(d) one IEEE double division.
#include <cmath>

#include "internal.h"

namespace homs {
namespace {

constexpr int kThreads = 256;
constexpr int kScanThreads = 1024;

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + kThreads - 1) / kThreads); }

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// PSMs of the stage by distance (hist[0 .. nbins) targets, hist[nbins ..)
// decoys). Stage 2 counts only queries the narrow stage did not identify.
__global__ void fdr_hist_kernel(int64_t nq, const int64_t* __restrict__ idx,
                                const int32_t* __restrict__ dist, const int8_t* __restrict__ stage,
                                int second, const uint8_t* __restrict__ lib_decoy, uint32_t nbins,
                                uint32_t* __restrict__ hist)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nq) return;
    if (second && stage[q] == 1) return;
    const int64_t i = idx[q];
    if (i < 0) return;
    const uint32_t d = (uint32_t)dist[q];
    if (d >= nbins) return;  // cannot happen: distances are <= D
    atomicAdd(hist + (lib_decoy[i] ? nbins : 0u) + d, 1u);
}

// q-value of every distance, one workgroup: each thread owns a contiguous
// run of distances; run totals are scanned across threads in LDS.
__global__ __launch_bounds__(kScanThreads) void fdr_qtable_kernel(
    uint32_t nbins, const uint32_t* __restrict__ hist, double* __restrict__ qtab)
{
    __shared__ uint64_t s_t[kScanThreads], s_d[kScanThreads];
    __shared__ double s_m[kScanThreads];
    const int t = threadIdx.x;
    const uint32_t per = (nbins + kScanThreads - 1) / kScanThreads;
    const uint32_t b0 = min(nbins, t * per), b1 = min(nbins, b0 + per);
    uint64_t nt = 0, nd = 0;
    for (uint32_t d = b0; d < b1; ++d) {
        nt += hist[d];
        nd += hist[nbins + d];
    }
    s_t[t] = nt;
    s_d[t] = nd;
    __syncthreads();
    // inclusive scan of the run totals (Hillis-Steele)
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const uint64_t at = t >= o ? s_t[t - o] : 0, ad = t >= o ? s_d[t - o] : 0;
        __syncthreads();
        s_t[t] += at;
        s_d[t] += ad;
        __syncthreads();
    }
    // FDR at every distance of the run, and the run's minimum
    uint64_t ct = s_t[t] - nt, cd = s_d[t] - nd;  // counts below the run
    double m = INFINITY;
    for (uint32_t d = b0; d < b1; ++d) {
        ct += hist[d];
        cd += hist[nbins + d];
        const double f = ct > 0 ? (double)cd / (double)ct : INFINITY;
        qtab[d] = f;
        m = fmin(m, f);
    }
    s_m[t] = m;
    __syncthreads();
    // suffix minimum of the run minima (reverse Hillis-Steele)
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const double v = t + o < kScanThreads ? s_m[t + o] : INFINITY;
        __syncthreads();
        s_m[t] = fmin(s_m[t], v);
        __syncthreads();
    }
    double run = t + 1 < kScanThreads ? s_m[t + 1] : INFINITY;  // minimum above the run
    for (uint32_t d = b1; d-- > b0;) {
        run = fmin(run, qtab[d]);
        qtab[d] = run;
    }
}

// Stage 1: identified = a target match with q <= level; every query keeps its
// narrow-stage result and q-value for now.
__global__ void fdr_apply_first_kernel(int64_t nq, const int64_t* __restrict__ idx,
                                       const int32_t* __restrict__ dist,
                                       const uint8_t* __restrict__ lib_decoy,
                                       const double* __restrict__ qtab, double level,
                                       int8_t* __restrict__ stage, double* __restrict__ qvalue)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const int64_t i = idx[q];
    const double qv = i >= 0 ? qtab[dist[q]] : INFINITY;
    stage[q] = (i >= 0 && !lib_decoy[i] && qv <= level) ? 1 : 0;
    qvalue[q] = qv;
}

// Stage 2: every query the narrow stage did not identify takes the open
// stage's result, q-value and verdict.
__global__ void fdr_apply_second_kernel(int64_t nq, const int64_t* __restrict__ idx2,
                                        const int32_t* __restrict__ dist2,
                                        const uint8_t* __restrict__ lib_decoy,
                                        const double* __restrict__ qtab, double level,
                                        int8_t* __restrict__ stage, double* __restrict__ qvalue,
                                        int64_t* __restrict__ out_idx,
                                        int32_t* __restrict__ out_dist)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nq || stage[q] == 1) return;
    const int64_t i = idx2[q];
    const double qv = i >= 0 ? qtab[dist2[q]] : INFINITY;
    out_idx[q] = i;
    out_dist[q] = dist2[q];
    qvalue[q] = qv;
    stage[q] = (i >= 0 && !lib_decoy[i] && qv <= level) ? 2 : 0;
}

// Open-stage precursors: an identified query gets +inf, which leaves its
// window empty and sorts it after every other query of its charge.
__global__ void mask_pmz_kernel(int64_t nq, const double* __restrict__ pmz,
                                const int8_t* __restrict__ stage, double* __restrict__ pmz2)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nq) return;
    pmz2[q] = stage[q] == 1 ? INFINITY : pmz[q];
}

}  // namespace

size_t cascade_scratch_bytes(int64_t nq, uint32_t dim)
{
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t nbins = (size_t)dim + 1;
    return al(nq * 8) + al(nq * 8) + al(nq * 4) + al(2 * nbins * 4) + al(nbins * 8);
}

CascadeScratch cascade_carve(void* base, int64_t nq, uint32_t dim)
{
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t nbins = (size_t)dim + 1;
    char* p = (char*)base;
    CascadeScratch w{};
    w.pmz2 = (double*)p;
    p += al(nq * 8);
    w.idx2 = (int64_t*)p;
    p += al(nq * 8);
    w.dist2 = (int32_t*)p;
    p += al(nq * 4);
    w.hist = (uint32_t*)p;
    p += al(2 * nbins * 4);
    w.qtab = (double*)p;
    return w;
}

hipError_t launch_fdr_stage(int second, int64_t nq, uint32_t dim, const int64_t* idx,
                            const int32_t* dist, const uint8_t* lib_decoy, double level,
                            const CascadeScratch& w, int8_t* stage, double* qvalue,
                            int64_t* out_idx, int32_t* out_dist, hipStream_t s)
{
    const uint32_t nbins = dim + 1;
    fill_u32_kernel<<<blocks_for(2 * (int64_t)nbins), kThreads, 0, s>>>(w.hist, 2 * nbins, 0u);
    fdr_hist_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, idx, dist, stage, second, lib_decoy,
                                                         nbins, w.hist);
    fdr_qtable_kernel<<<1, kScanThreads, 0, s>>>(nbins, w.hist, w.qtab);
    if (!second)
        fdr_apply_first_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, idx, dist, lib_decoy,
                                                                    w.qtab, level, stage, qvalue);
    else
        fdr_apply_second_kernel<<<blocks_for(nq), kThreads, 0, s>>>(
            nq, idx, dist, lib_decoy, w.qtab, level, stage, qvalue, out_idx, out_dist);
    return hipGetLastError();
}

hipError_t launch_mask_identified(int64_t nq, const double* pmz, const int8_t* stage,
                                  double* pmz2, hipStream_t s)
{
    mask_pmz_kernel<<<blocks_for(nq), kThreads, 0, s>>>(nq, pmz, stage, pmz2);
    return hipGetLastError();
}

}  // namespace homs
