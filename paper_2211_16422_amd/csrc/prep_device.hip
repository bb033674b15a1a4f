// Preprocessing on the device (Section 3.2, Table 1): raw peaks -> spectrum
// vectors, the same steps and float64 arithmetic as the host path
// (homs_preprocess), so encoding can start from raw m/z and intensities
// already in HBM.
//
// Spectra of up to kWaveCap raw peaks (the usual case): one wave per
// spectrum, no barriers. In-range peaks are compacted into the wave's LDS
// (ballot positions), the noise floor is a wave maximum, a kept peak's place
// in the top-N is its rank under (intensity desc, m/z asc, input position
// asc) counted by the lane that owns it, the N kept peaks are placed in
// (m/z asc, position asc) order by a second rank, and colliding bins are
// summed by the lane holding their first peak, sequentially in m/z order (the
// order that fixes the sums' rounding); normalisation and quantisation are
// per bin. Larger spectra go to a workgroup kernel with bitonic sorts in LDS
// and one thread for the in-order sums; one with more than kPrepCap raw peaks
// first has the peaks that can reach the top-N gathered into LDS (all kept
// peaks, or, when more than kPrepCap are kept, the top_n found by a radix
// select over (intensity desc, m/z asc, position asc) keys read from global
// memory), and only a spectrum that would keep more than kPrepCap peaks
// (top_n above kPrepCap) raises kErrPeaks and yields no entries. Every double
// operation is an IEEE operation (no contraction; the device double square
// root is correctly rounded), so results equal the host path's.
//
// Two passes over the spectra: the first counts each spectrum's unique bins,
// an exclusive scan gives the CSR offsets, the second recomputes and writes.

#include <cmath>
#include <type_traits>

#include "internal.h"

namespace homs {
namespace {

constexpr int kPrepThreads = 128;
constexpr int kPrepCap = 2048;
constexpr int kWaveCap = 256;
constexpr int kWaves = 4;  // spectra per workgroup of the wave kernel

struct PrepArgs {
    double mz_min, mz_max, bins_per_da, noise_frac;
    int64_t nbins;
    uint32_t top_n, Q;
};

// Kernel modes: 0 counts each spectrum's entries, 1 writes them at the
// scanned offsets, 2 (staged single pass) writes the count and the entries at
// s * stage_cap (at most min(top_n, kPrepCap) entries per spectrum), moved to
// their final place once the counts are scanned.
__device__ __forceinline__ int64_t stage_cap(const PrepArgs& pa)
{
    return pa.top_n < (uint32_t)kPrepCap ? (int64_t)pa.top_n : (int64_t)kPrepCap;
}

// bitonic sort of s[0, P) (P a power of two) under `before`, by the workgroup
template <typename Before>
__device__ void bitonic(double* a_mz, double* a_in, uint32_t* a_pos, int P, Before before)
{
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const bool swap = up ? before(l, i) : before(i, l);
                    if (swap) {
                        const double tm = a_mz[i], ti = a_in[i];
                        const uint32_t tp = a_pos[i];
                        a_mz[i] = a_mz[l];
                        a_in[i] = a_in[l];
                        a_pos[i] = a_pos[l];
                        a_mz[l] = tm;
                        a_in[l] = ti;
                        a_pos[l] = tp;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// order-preserving key of a finite double (-0 and +0 share one)
__device__ __forceinline__ uint64_t order_key(double x)
{
    if (x == 0.0) x = 0.0;
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// A spectrum of np > kPrepCap raw peaks: gathers into s_mz / s_in / s_pos
// (count in *s_m, which starts at 0) the kept peaks (in range, not below
// floor_i) that can reach the top-N: all of them when at most kPrepCap are
// kept, else the T = min(kept, top_n) first under (intensity desc, m/z asc,
// position asc), found by a radix select, 8 bits per round, over the 160-bit
// keys (~key(intensity), key(m/z), position) read from global memory. Returns
// false (uniform) when T exceeds kPrepCap. The whole workgroup calls it.
__device__ bool gather_large(int64_t p0, int64_t np, const double* __restrict__ mz,
                             const double* __restrict__ inten, const PrepArgs& pa, double floor_i,
                             double* s_mz, double* s_in, uint32_t* s_pos, int* s_m)
{
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_kept, s_dig, s_below, s_eq;
    auto kept_at = [&](int64_t p, double& m, double& v) {
        m = mz[p0 + p];
        v = inten[p0 + p];
        return m >= pa.mz_min && m < pa.mz_max && !(v < floor_i);
    };
    if (threadIdx.x == 0) s_kept = 0;
    __syncthreads();
    uint32_t c = 0;
    for (int64_t p = threadIdx.x; p < np; p += blockDim.x) {
        double m, v;
        c += kept_at(p, m, v) ? 1u : 0u;
    }
    atomicAdd(&s_kept, c);
    __syncthreads();
    const uint32_t kept = s_kept;
    auto put = [&](int64_t p, double m, double v) {
        const int slot = atomicAdd(s_m, 1);
        if (slot < kPrepCap) {  // always, by the counts above; kept as a bound
            s_mz[slot] = m;
            s_in[slot] = v;
            s_pos[slot] = (uint32_t)p;
        }
    };
    if (kept <= (uint32_t)kPrepCap) {  // uniform
        for (int64_t p = threadIdx.x; p < np; p += blockDim.x) {
            double m, v;
            if (kept_at(p, m, v)) put(p, m, v);
        }
        return true;
    }
    uint32_t r = kept < pa.top_n ? kept : pa.top_n;  // rank sought, 1-based
    if (r > (uint32_t)kPrepCap) return false;
    // prefix and mask of the decided digits of the three keys
    uint64_t pre1 = 0, msk1 = 0, pre2 = 0, msk2 = 0;
    uint32_t pre3 = 0, msk3 = 0;
    auto keys = [&](int64_t p, double m, double v, uint64_t& k1, uint64_t& k2, uint32_t& k3) {
        k1 = ~order_key(v);  // descending intensity
        k2 = order_key(m);
        k3 = (uint32_t)p;
    };
    for (int d = 0; d < 20; ++d) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) s_hist[i] = 0;
        __syncthreads();
        for (int64_t p = threadIdx.x; p < np; p += blockDim.x) {
            double m, v;
            if (!kept_at(p, m, v)) continue;
            uint64_t k1, k2;
            uint32_t k3;
            keys(p, m, v, k1, k2, k3);
            if ((k1 & msk1) != pre1 || (k2 & msk2) != pre2 || (k3 & msk3) != pre3) continue;
            const uint32_t dig = d < 8 ? (uint32_t)(k1 >> (56 - 8 * d)) & 255u
                                 : d < 16 ? (uint32_t)(k2 >> (56 - 8 * (d - 8))) & 255u
                                          : (k3 >> (24 - 8 * (d - 16))) & 255u;
            atomicAdd(&s_hist[dig], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {  // the digit holding the r-th smallest key
            uint32_t cum = 0, dg = 0;
            while (dg < 255 && cum + s_hist[dg] < r) cum += s_hist[dg++];
            s_dig = dg;
            s_below = cum;
            s_eq = s_hist[dg];
        }
        __syncthreads();
        const uint32_t dig = s_dig, eq = s_eq;
        r -= s_below;
        if (d < 8) {
            pre1 |= (uint64_t)dig << (56 - 8 * d);
            msk1 |= (uint64_t)255 << (56 - 8 * d);
        } else if (d < 16) {
            pre2 |= (uint64_t)dig << (56 - 8 * (d - 8));
            msk2 |= (uint64_t)255 << (56 - 8 * (d - 8));
        } else {
            pre3 |= dig << (24 - 8 * (d - 16));
            msk3 |= 255u << (24 - 8 * (d - 16));
        }
        if (eq == r) break;  // uniform: every key sharing the prefix is taken
    }
    // every kept peak whose decided digits are at most the prefix: T of them
    for (int64_t p = threadIdx.x; p < np; p += blockDim.x) {
        double m, v;
        if (!kept_at(p, m, v)) continue;
        uint64_t k1, k2;
        uint32_t k3;
        keys(p, m, v, k1, k2, k3);
        k1 &= msk1;
        k2 &= msk2;
        k3 &= msk3;
        const bool le = k1 != pre1 ? k1 < pre1 : k2 != pre2 ? k2 < pre2 : k3 <= pre3;
        if (le) put(p, m, v);
    }
    return true;
}

__global__ __launch_bounds__(kPrepThreads) void preprocess_kernel(
    int write, int64_t n, const int64_t* __restrict__ off, const double* __restrict__ mz,
    const double* __restrict__ inten, PrepArgs pa, int64_t* __restrict__ counts,
    const int64_t* __restrict__ out_off, int32_t* __restrict__ out_bin,
    uint8_t* __restrict__ out_level, uint32_t* __restrict__ err)
{
    __shared__ double s_mz[kPrepCap], s_in[kPrepCap];
    __shared__ uint32_t s_pos[kPrepCap];
    __shared__ double s_red[kPrepThreads];
    __shared__ int s_m, s_k;
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        const int64_t p0 = off[s];
        const int64_t np = off[s + 1] - p0;
        if (np <= kWaveCap) continue;  // the wave kernel's
        const bool large = np > kPrepCap;  // uniform
        if (threadIdx.x == 0) s_m = 0;
        __syncthreads();
        // 1. m/z range; 2. the maximum intensity of the peaks in range (those
        // peaks go to LDS unless the spectrum is larger than LDS holds)
        double imax = 0.0;
        for (int64_t p = threadIdx.x; p < np; p += blockDim.x) {
            const double m = mz[p0 + p];
            if (m >= pa.mz_min && m < pa.mz_max) {
                const double v = inten[p0 + p];
                if (!large) {
                    const int slot = atomicAdd(&s_m, 1);
                    s_mz[slot] = m;
                    s_in[slot] = v;
                    s_pos[slot] = (uint32_t)p;
                }
                imax = v > imax ? v : imax;
            }
        }
        s_red[threadIdx.x] = imax;
        __syncthreads();
        for (int o = kPrepThreads / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o)
                s_red[threadIdx.x] = fmax(s_red[threadIdx.x], s_red[threadIdx.x + o]);
            __syncthreads();
        }
        const double floor_i = pa.noise_frac * s_red[0];
        if (large) {
            if (!gather_large(p0, np, mz, inten, pa, floor_i, s_mz, s_in, s_pos, &s_m)) {
                if (threadIdx.x == 0) {
                    atomicOr(err, kErrPeaks);
                    if (write != 1) counts[s] = 0;
                }
                __syncthreads();
                continue;
            }
            __syncthreads();
        }
        const int m = s_m < kPrepCap ? s_m : kPrepCap;
        // peaks below the noise floor sort after the kept ones (kept >= 0),
        // padding after everything
        int P = 1;
        while (P < m) P <<= 1;
        for (int i = threadIdx.x; i < P; i += blockDim.x) {
            if (i >= m) {
                s_in[i] = -INFINITY;
                s_mz[i] = INFINITY;
                s_pos[i] = 0xFFFFFFFFu;
            } else if (s_in[i] < floor_i) {
                s_in[i] = -1.0;
            }
        }
        __syncthreads();
        // 3. top-N: intensity desc, m/z asc, input position asc
        bitonic(s_mz, s_in, s_pos, P, [&](int x, int y) {
            if (s_in[x] != s_in[y]) return s_in[x] > s_in[y];
            if (s_mz[x] != s_mz[y]) return s_mz[x] < s_mz[y];
            return s_pos[x] < s_pos[y];
        });
        if (threadIdx.x == 0) {
            int k = 0;
            while (k < m && s_in[k] >= 0.0) ++k;  // kept peaks come first
            s_k = k < (int)pa.top_n ? k : (int)pa.top_n;
        }
        __syncthreads();
        const int k = s_k;
        // 4. square roots of the kept intensities; the rest become padding
        int P2 = 1;
        while (P2 < k) P2 <<= 1;
        for (int i = threadIdx.x; i < P2; i += blockDim.x) {
            if (i < k) {
                s_in[i] = sqrt(s_in[i]);
            } else {
                s_mz[i] = INFINITY;
                s_pos[i] = 0xFFFFFFFFu;
            }
        }
        __syncthreads();
        // 5. ascending m/z, then input position
        bitonic(s_mz, s_in, s_pos, P2, [&](int x, int y) {
            if (s_mz[x] != s_mz[y]) return s_mz[x] < s_mz[y];
            return s_pos[x] < s_pos[y];
        });
        // 5-6. bins, sums of colliding peaks in ascending m/z, normalisation,
        // levels: one thread, in order (the sums' rounding depends on it)
        if (threadIdx.x == 0) {
            int u = 0;
            int32_t last = -1;
            for (int i = 0; i < k; ++i) {
                int64_t bn = (int64_t)floor((s_mz[i] - pa.mz_min) * pa.bins_per_da);
                if (bn > pa.nbins - 1) bn = pa.nbins - 1;
                if (bn < 0) bn = 0;
                if (u > 0 && last == (int32_t)bn) {
                    s_in[u - 1] = s_in[u - 1] + s_in[i];
                } else {
                    s_in[u] = s_in[i];  // u <= i: in place
                    s_pos[u] = (uint32_t)bn;
                    last = (int32_t)bn;
                    ++u;
                }
            }
            if (write != 1) counts[s] = u;
            if (write != 0) {
                double smax = 0.0;
                for (int i = 0; i < u; ++i) smax = s_in[i] > smax ? s_in[i] : smax;
                const int64_t w0 = write == 2 ? s * stage_cap(pa) : out_off[s];
                for (int i = 0; i < u; ++i) {
                    int64_t lv = 0;
                    if (smax > 0.0) {
                        const double v = s_in[i] / smax;
                        lv = (int64_t)floor(v * (double)pa.Q);
                        if (lv > (int64_t)pa.Q - 1) lv = (int64_t)pa.Q - 1;
                    }
                    out_bin[w0 + i] = (int32_t)s_pos[i];
                    out_level[w0 + i] = (uint8_t)lv;
                }
            }
        }
        __syncthreads();  // LDS is reused by the next spectrum
    }
}

// total order of the top-N selection: does peak x come before peak y?
__device__ __forceinline__ bool before_int(double ix, double mx, uint32_t px, double iy, double my,
                                           uint32_t py)
{
    if (ix != iy) return ix > iy;
    if (mx != my) return mx < my;
    return px < py;
}

__global__ __launch_bounds__(64 * kWaves) void preprocess_wave_kernel(
    int write, int64_t n, const int64_t* __restrict__ off, const double* __restrict__ mz,
    const double* __restrict__ inten, PrepArgs pa, int64_t* __restrict__ counts,
    const int64_t* __restrict__ out_off, int32_t* __restrict__ out_bin,
    uint8_t* __restrict__ out_level)
{
    __shared__ double s_mz[kWaves][kWaveCap], s_in[kWaves][kWaveCap];
    __shared__ double s_tmz[kWaves][kWaveCap];
    __shared__ uint16_t s_pos[kWaves][kWaveCap], s_top[kWaves][kWaveCap],
        s_ord[kWaves][kWaveCap], s_tpos[kWaves][kWaveCap];
    __shared__ int32_t s_bin[kWaves][kWaveCap];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double* const smz = s_mz[w];
    double* const sin_ = s_in[w];
    uint16_t* const spos = s_pos[w];
    uint16_t* const stop = s_top[w];
    uint16_t* const sord = s_ord[w];
    double* const tmz = s_tmz[w];
    uint16_t* const tpos = s_tpos[w];
    int32_t* const sbin = s_bin[w];
    const int64_t stride = (int64_t)gridDim.x * kWaves;
    for (int64_t s = (int64_t)blockIdx.x * kWaves + w; s < n; s += stride) {
        const int64_t p0 = off[s];
        const int np = (int)(off[s + 1] - p0);
        if (np > kWaveCap) continue;  // the workgroup kernel's (uniform per wave)
        // 1. in-range peaks into LDS, in input order; their maximum intensity
        int m = 0;
        double imax = 0.0;
        for (int c = 0; c < np; c += 64) {
            const int p = c + l;
            double pm = 0.0, pi = 0.0;
            bool ok = false;
            if (p < np) {
                pm = mz[p0 + p];
                pi = inten[p0 + p];
                ok = pm >= pa.mz_min && pm < pa.mz_max;
            }
            const uint64_t b = __ballot(ok);
            if (ok) {
                const int slot = m + (int)__builtin_amdgcn_mbcnt_hi(
                                         (uint32_t)(b >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
                smz[slot] = pm;
                sin_[slot] = pi;
                spos[slot] = (uint16_t)p;
                imax = pi > imax ? pi : imax;
            }
            m += __popcll(b);
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double v = __shfl_xor(imax, o);
            imax = v > imax ? v : imax;
        }
        __builtin_amdgcn_wave_barrier();
        // 2. noise floor; 3. rank of each kept peak in the top-N order
        const double floor_i = pa.noise_frac * imax;
        int kept = 0;
        for (int e = l; e < m; e += 64) kept += !(sin_[e] < floor_i);
        for (int o = 32; o > 0; o >>= 1) kept += __shfl_xor(kept, o);
        const int k = kept < (int)pa.top_n ? kept : (int)pa.top_n;
        // one pass over the peaks ranks all of the lane's peaks at once
        // (held in registers); peak j's fields are broadcast LDS reads, and
        // the loop carries no dependence between iterations, so the reads of
        // several iterations are in flight together
        auto rank_top = [&](auto per_tag) {
            constexpr int P = decltype(per_tag)::value;  // peaks per lane
            double ie[P], me[P];
            uint32_t pe[P];
            int r[P];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int e = l + 64 * q < m ? l + 64 * q : m - 1;
                ie[q] = sin_[e];
                me[q] = smz[e];
                pe[q] = spos[e];
                r[q] = 0;
            }
#pragma unroll 4
            for (int j = 0; j < m; ++j) {
                const double ij = sin_[j], mj = smz[j];
                const uint32_t pj = spos[j];
                const bool kj = !(ij < floor_i);
#pragma unroll
                for (int q = 0; q < P; ++q)
                    r[q] += (kj && before_int(ij, mj, pj, ie[q], me[q], pe[q])) ? 1 : 0;
            }
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int e = l + 64 * q;
                if (e < m && !(ie[q] < floor_i) && r[q] < k) stop[r[q]] = (uint16_t)e;
            }
        };
        static_assert(kWaveCap == 256, "up to four peaks per lane");
        if (m > 0) {  // wave-uniform
            const int per = (m + 63) >> 6;
            if (per == 1)
                rank_top(std::integral_constant<int, 1>{});
            else if (per == 2)
                rank_top(std::integral_constant<int, 2>{});
            else if (per == 3)
                rank_top(std::integral_constant<int, 3>{});
            else
                rank_top(std::integral_constant<int, 4>{});
        }
        __builtin_amdgcn_wave_barrier();
        // 4-5. the top-N in (m/z asc, position asc) order, ranked over a
        // compact copy of their m/z and positions
        for (int t = l; t < k; t += 64) {
            const int e = stop[t];
            tmz[t] = smz[e];
            tpos[t] = spos[e];
        }
        __builtin_amdgcn_wave_barrier();
        for (int t = l; t < k; t += 64) {
            const double me = tmz[t];
            const uint32_t pe = tpos[t];
            int r = 0;
#pragma unroll 4
            for (int u = 0; u < k; ++u) {
                const double mf = tmz[u];
                r += (mf < me || (mf == me && (uint32_t)tpos[u] < pe)) ? 1 : 0;
            }
            sord[r] = stop[t];
        }
        __builtin_amdgcn_wave_barrier();
        for (int t = l; t < k; t += 64) {
            int64_t bn = (int64_t)floor((smz[sord[t]] - pa.mz_min) * pa.bins_per_da);
            if (bn > pa.nbins - 1) bn = pa.nbins - 1;
            if (bn < 0) bn = 0;
            sbin[t] = (int32_t)bn;
        }
        __builtin_amdgcn_wave_barrier();
        // 5-6. bins: the lane of a bin's first peak sums its peaks' square
        // roots in m/z order; then the largest sum, levels and output
        int u_total = 0;
        double smax = 0.0;
        for (int c = 0; c < k; c += 64) {
            const int t = c + l;
            const bool first = t < k && (t == 0 || sbin[t] != sbin[t - 1]);
            if (first) {
                double sum = sqrt(sin_[sord[t]]);
                for (int v = t + 1; v < k && sbin[v] == sbin[t]; ++v) sum = sum + sqrt(sin_[sord[v]]);
                smax = sum > smax ? sum : smax;
            }
            u_total += __popcll(__ballot(first));
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double v = __shfl_xor(smax, o);
            smax = v > smax ? v : smax;
        }
        if (write != 1 && l == 0) counts[s] = u_total;
        if (write == 0) continue;
        int64_t w0 = write == 2 ? s * stage_cap(pa) : out_off[s];
        for (int c = 0; c < k; c += 64) {
            const int t = c + l;
            const bool first = t < k && (t == 0 || sbin[t] != sbin[t - 1]);
            const uint64_t b = __ballot(first);
            if (first) {
                double sum = sqrt(sin_[sord[t]]);
                for (int v = t + 1; v < k && sbin[v] == sbin[t]; ++v) sum = sum + sqrt(sin_[sord[v]]);
                int64_t lv = 0;
                if (smax > 0.0) {
                    const double val = sum / smax;
                    lv = (int64_t)floor(val * (double)pa.Q);
                    if (lv > (int64_t)pa.Q - 1) lv = (int64_t)pa.Q - 1;
                }
                const int64_t at = w0 + (int64_t)__builtin_amdgcn_mbcnt_hi(
                                            (uint32_t)(b >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
                out_bin[at] = sbin[t];
                out_level[at] = (uint8_t)lv;
            }
            w0 += __popcll(b);
        }
        __builtin_amdgcn_wave_barrier();  // LDS is reused by the wave's next spectrum
    }
}

// one wave per spectrum, grid-stride
__global__ void compact_stage_kernel(int64_t n, PrepArgs pa, const int64_t* __restrict__ counts,
                                     const int64_t* __restrict__ out_off,
                                     const int32_t* __restrict__ st_bin,
                                     const uint8_t* __restrict__ st_level,
                                     int32_t* __restrict__ out_bin, uint8_t* __restrict__ out_level)
{
    const int l = threadIdx.x & 63;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t cap = stage_cap(pa);
    for (int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; s < n; s += waves) {
        const int64_t c = counts[s], o = out_off[s];
        for (int64_t j = l; j < c; j += 64) {
            out_bin[o + j] = st_bin[s * cap + j];
            out_level[o + j] = st_level[s * cap + j];
        }
    }
}

__global__ void offsets_tail_kernel(int64_t n, const int64_t* counts, int64_t* out_off)
{
    // out_off[0, n) holds the exclusive scan; the total closes the CSR
    out_off[n] = n > 0 ? out_off[n - 1] + counts[n - 1] : 0;
}

}  // namespace

int prep_device_max_peaks() { return kPrepCap; }

namespace {
constexpr size_t kStageBudget = (size_t)2 << 30;  // staged single pass up to this many bytes
size_t al256(size_t b) { return (b + 255) / 256 * 256; }
size_t stage_bytes(int64_t n, uint32_t top_n)
{
    const size_t cap = top_n < (uint32_t)kPrepCap ? top_n : (uint32_t)kPrepCap;
    return al256((size_t)n * cap * 4) + al256((size_t)n * cap);
}
}  // namespace

size_t prep_device_scratch_bytes(int64_t n, uint32_t top_n)
{
    const size_t temp = scan_temp_bytes(n);
    const size_t st = stage_bytes(n, top_n);
    return al256((size_t)n * 8) + al256(temp) + (st <= kStageBudget ? st : 0);
}

hipError_t launch_preprocess_device(const homs_ctx* c, int64_t n, const int64_t* off,
                                    const double* mz, const double* inten, int64_t* out_off,
                                    int32_t* out_bin, uint8_t* out_level, void* scratch,
                                    hipStream_t s)
{
    if (n <= 0) {
        return hipMemsetAsync(out_off, 0, sizeof(int64_t), s);
    }
    PrepArgs pa{c->p.mz_min, c->p.mz_max, c->p.bins_per_da, c->p.noise_frac, c->n_bins,
                c->p.top_n, c->p.n_levels};
    int64_t* counts = (int64_t*)scratch;
    void* temp = (char*)scratch + al256((size_t)n * 8);
    const size_t temp_bytes = scan_temp_bytes(n);
    hipError_t e = hipSuccess;
    const uint32_t grid = (uint32_t)(n < 8192 ? n : 8192);
    const int64_t wgrid64 = (n + kWaves - 1) / kWaves;
    const uint32_t wgrid = (uint32_t)(wgrid64 < 65536 ? wgrid64 : 65536);
    if (stage_bytes(n, pa.top_n) <= kStageBudget) {
        // one pass into the staging area, scan, move into place
        char* st = (char*)temp + al256(temp_bytes);
        const size_t cap = pa.top_n < (uint32_t)kPrepCap ? pa.top_n : (uint32_t)kPrepCap;
        int32_t* st_bin = (int32_t*)st;
        uint8_t* st_level = (uint8_t*)(st + al256((size_t)n * cap * 4));
        preprocess_wave_kernel<<<wgrid, 64 * kWaves, 0, s>>>(2, n, off, mz, inten, pa, counts,
                                                             out_off, st_bin, st_level);
        preprocess_kernel<<<grid, kPrepThreads, 0, s>>>(2, n, off, mz, inten, pa, counts, out_off,
                                                        st_bin, st_level, c->d_err);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = exclusive_scan<int64_t>(counts, out_off, n, temp, s);
        if (e != hipSuccess) return e;
        offsets_tail_kernel<<<1, 1, 0, s>>>(n, counts, out_off);
        const int64_t cgrid64 = (n + 3) / 4;
        compact_stage_kernel<<<(uint32_t)(cgrid64 < 65536 ? cgrid64 : 65536), 256, 0, s>>>(
            n, pa, counts, out_off, st_bin, st_level, out_bin, out_level);
        return hipGetLastError();
    }
    // two passes (count, scan, write) when the staging area would be too large
    for (int write = 0; write < 2; ++write) {
        preprocess_wave_kernel<<<wgrid, 64 * kWaves, 0, s>>>(write, n, off, mz, inten, pa, counts,
                                                             out_off, out_bin, out_level);
        preprocess_kernel<<<grid, kPrepThreads, 0, s>>>(write, n, off, mz, inten, pa, counts,
                                                        out_off, out_bin, out_level, c->d_err);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (!write) {
            e = exclusive_scan<int64_t>(counts, out_off, n, temp, s);
            if (e != hipSuccess) return e;
            offsets_tail_kernel<<<1, 1, 0, s>>>(n, counts, out_off);
        }
    }
    return hipGetLastError();
}

}  // namespace homs
