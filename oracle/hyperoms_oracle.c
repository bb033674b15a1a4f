/*
 * HyperOMS oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU implementation of what the HyperOMS hot path computes
 * (Kang, Xu, Bittremieux, Rosing, "Massively Parallel Open Modification
 * Spectral Library Searching with Hyperdimensional Computing", arXiv
 * 2211.16422). Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it; the product library never does.
 *
 * Every function follows the paper's definition directly, with no blocking,
 * bit tricks or reordering beyond what the definition states:
 *   - preprocessing: Section 3.2 and Table 1 (noise filter, top-N, binning,
 *     summing colliding peaks), plus intensity quantisation to Q levels
 *     (Section 3.3);
 *   - position and level hypervectors: Sections 3.3.1 and 3.3.2;
 *   - encoding: Section 3.3, Eq. 1, followed by binarisation;
 *   - candidate filter and Hamming top-1: Section 3.4 and Section 2.1.
 * Where the paper is silent the readings are stated at each function.
 *
 * Floating point is float64 throughout and uses only correctly rounded IEEE
 * operations (+, -, *, /, sqrt, floor) in a fixed order; build with
 * -ffp-contract=off.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the state advances by the golden-ratio gamma and
 * each output is the variant-13 finaliser of the new state.               */
static uint64_t sm64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

ORACLE_API void oracle_splitmix64(uint64_t seed, int64_t n, uint64_t *out)
{
    uint64_t s = seed;
    for (int64_t i = 0; i < n; ++i) out[i] = sm64_next(&s);
}

/* ------------------------------------------------------------------------ */
/* Helpers on one packed hypervector: bit d lives in word d/32 at bit d%32;
 * a 0 bit stands for the bipolar component +1 and a 1 bit for -1.         */
static void flip_bit(uint32_t *hv, uint32_t d) { hv[d >> 5] ^= (1u << (d & 31)); }

/* Draws D random bits, 64 per SplitMix64 output (bit d from output d/64,
 * bit position d%64).                                                       */
static void random_bits(uint64_t *state, uint32_t D, uint32_t *hv)
{
    memset(hv, 0, (size_t)(D / 32) * sizeof(uint32_t));
    for (uint32_t k = 0; k < D / 64; ++k) {
        uint64_t r = sm64_next(state);
        for (uint32_t b = 0; b < 64; ++b)
            if ((r >> b) & 1u) flip_bit(hv, k * 64 + b);
    }
}

/* Fisher-Yates (Durstenfeld) shuffle of 0..D-1: for i = D-1 down to 1 swap
 * entry i with entry j = (next output) mod (i+1).                           */
static void random_permutation(uint64_t *state, uint32_t D, uint32_t *perm)
{
    for (uint32_t i = 0; i < D; ++i) perm[i] = i;
    for (uint32_t i = D - 1; i >= 1; --i) {
        uint32_t j = (uint32_t)(sm64_next(state) % (uint64_t)(i + 1));
        uint32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
}

/*
 * Position (ID) and level hypervector tables (Sections 3.3.1 and 3.3.2).
 *
 * Reading of Section 3.3.1: one random base vector F_0 and one random order
 * of the D components; F_i is F_0 with the first k_i components of that
 * order flipped, k_i = floor(alpha * i / (f - 1)), so F_0 and F_{f-1} differ
 * in exactly alpha components and H(F_i, F_j) = |k_i - k_j|.
 * Reading of Section 3.3.2: level j of Q is the level-0 base vector with
 * m_j = floor((D/2) * j / (Q - 1)) components flipped, again cumulatively
 * along one random order, so H(L_0, L_{Q-1}) = D/2.
 *
 * Random stream: a single SplitMix64 stream started at `seed`, consumed in
 * this order: F_0 bits, the F order, L_0 bits, the L order.
 *
 * id_out: f rows of D/32 words; lv_out: Q rows of D/32 words.
 * Returns 0, or -1 for D not a multiple of 64, f == 0, Q < 2, alpha > D.
 */
/* encoding 0: position vectors with locality (Section 3.3.1); 1 and 2 (the
 * random-ID and random-projection baselines of Section 4.2): every position
 * vector is independent random bits, drawn row after row from the same
 * stream after the level table. */
ORACLE_API int oracle_codebook(uint32_t D, uint32_t f, uint32_t Q, uint32_t alpha,
                               uint64_t seed, uint32_t encoding, uint32_t *id_out,
                               uint32_t *lv_out)
{
    if (D == 0 || D % 64 != 0 || f == 0 || Q < 2 || alpha > D) return -1;
    const uint32_t W = D / 32;
    uint64_t state = seed;
    uint32_t *base = (uint32_t *)malloc((size_t)W * sizeof(uint32_t));
    uint32_t *perm = (uint32_t *)malloc((size_t)D * sizeof(uint32_t));
    if (!base || !perm) { free(base); free(perm); return -1; }

    random_bits(&state, D, base);
    random_permutation(&state, D, perm);
    for (uint32_t i = 0; i < f; ++i) {
        uint64_t k = (f == 1) ? 0 : ((uint64_t)alpha * i) / (uint64_t)(f - 1);
        uint32_t *row = id_out + (size_t)i * W;
        memcpy(row, base, (size_t)W * sizeof(uint32_t));
        for (uint64_t t = 0; t < k; ++t) flip_bit(row, perm[t]);
    }

    random_bits(&state, D, base);
    random_permutation(&state, D, perm);
    for (uint32_t j = 0; j < Q; ++j) {
        uint64_t m = ((uint64_t)(D / 2) * j) / (uint64_t)(Q - 1);
        uint32_t *row = lv_out + (size_t)j * W;
        memcpy(row, base, (size_t)W * sizeof(uint32_t));
        for (uint64_t t = 0; t < m; ++t) flip_bit(row, perm[t]);
    }
    if (encoding != 0)
        for (uint32_t i = 0; i < f; ++i) random_bits(&state, D, id_out + (size_t)i * W);
    free(base);
    free(perm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Preprocessing (Section 3.2; Table 1).                                     */

typedef struct {
    double mz, inten;
    int64_t pos;  /* position within the spectrum's input peaks */
} peak_t;

/* intensity descending, then m/z ascending, then input position ascending */
static int by_intensity(const void *a, const void *b)
{
    const peak_t *x = (const peak_t *)a, *y = (const peak_t *)b;
    if (x->inten != y->inten) return x->inten > y->inten ? -1 : 1;
    if (x->mz != y->mz) return x->mz < y->mz ? -1 : 1;
    return (x->pos > y->pos) - (x->pos < y->pos);
}

/* m/z ascending, then input position ascending */
static int by_mz(const void *a, const void *b)
{
    const peak_t *x = (const peak_t *)a, *y = (const peak_t *)b;
    if (x->mz != y->mz) return x->mz < y->mz ? -1 : 1;
    return (x->pos > y->pos) - (x->pos < y->pos);
}

/* number of m/z bins: ceil((mz_max - mz_min) * bins_per_da) */
ORACLE_API int64_t oracle_num_bins(double mz_min, double mz_max, double bins_per_da)
{
    return (int64_t)ceil((mz_max - mz_min) * bins_per_da);
}

/*
 * For every spectrum, in this order (Section 3.2, with the readings noted):
 *  1. keep peaks with mz_min <= mz < mz_max (Table 1 m/z range);
 *  2. drop peaks whose intensity is below noise_frac times the most intense
 *     remaining peak (the 1% noise rule);
 *  3. keep the top_n most intense peaks (Table 1: 50); ties go to the lower
 *     m/z, then the earlier input peak;
 *  4. scale each intensity by its square root (the workloads' "sqrt scaling";
 *     the paper does not say);
 *  5. bin = floor((mz - mz_min) * bins_per_da), clamped to the last bin;
 *     peaks sharing a bin are merged by summing their scaled intensities,
 *     added in ascending m/z order;
 *  6. divide each bin value by the largest one and quantise to one of Q
 *     levels: level = min(Q - 1, floor(v * Q)) (Section 3.3 quantises the
 *     intensity range into Q levels); if every value is 0 all levels are 0.
 * Output per spectrum: unique bins in ascending order with their levels.
 * out_off has n+1 entries; out_bin/out_level need room for off[n] entries.
 * Returns the total number of output peaks, or -1 on allocation failure.
 */
ORACLE_API int64_t oracle_preprocess(int64_t n, const int64_t *off, const double *mz,
                                     const double *inten, double mz_min, double mz_max,
                                     double bins_per_da, double noise_frac, uint32_t top_n,
                                     uint32_t Q, int64_t *out_off, int32_t *out_bin,
                                     uint8_t *out_level)
{
    const int64_t nbins = oracle_num_bins(mz_min, mz_max, bins_per_da);
    int64_t maxp = 0;
    for (int64_t s = 0; s < n; ++s)
        if (off[s + 1] - off[s] > maxp) maxp = off[s + 1] - off[s];
    peak_t *pk = (peak_t *)malloc((size_t)(maxp > 0 ? maxp : 1) * sizeof(peak_t));
    double *sum = (double *)malloc((size_t)(maxp > 0 ? maxp : 1) * sizeof(double));
    int32_t *bins = (int32_t *)malloc((size_t)(maxp > 0 ? maxp : 1) * sizeof(int32_t));
    if (!pk || !sum || !bins) { free(pk); free(sum); free(bins); return -1; }

    int64_t w = 0;
    out_off[0] = 0;
    for (int64_t s = 0; s < n; ++s) {
        /* 1. m/z range */
        int64_t m = 0;
        for (int64_t p = off[s]; p < off[s + 1]; ++p) {
            if (mz[p] >= mz_min && mz[p] < mz_max) {
                pk[m].mz = mz[p];
                pk[m].inten = inten[p];
                pk[m].pos = p - off[s];
                ++m;
            }
        }
        /* 2. noise filter */
        double imax = 0.0;
        for (int64_t p = 0; p < m; ++p)
            if (pk[p].inten > imax) imax = pk[p].inten;
        const double floor_i = noise_frac * imax;
        int64_t k = 0;
        for (int64_t p = 0; p < m; ++p)
            if (!(pk[p].inten < floor_i)) pk[k++] = pk[p];
        /* 3. top-N by intensity */
        qsort(pk, (size_t)k, sizeof(peak_t), by_intensity);
        if (k > (int64_t)top_n) k = top_n;
        /* 4. square-root scaling */
        for (int64_t p = 0; p < k; ++p) pk[p].inten = sqrt(pk[p].inten);
        /* 5. binning and summing of colliding peaks, in ascending m/z */
        qsort(pk, (size_t)k, sizeof(peak_t), by_mz);
        int64_t u = 0;
        for (int64_t p = 0; p < k; ++p) {
            int64_t b = (int64_t)floor((pk[p].mz - mz_min) * bins_per_da);
            if (b > nbins - 1) b = nbins - 1;
            if (b < 0) b = 0;
            if (u > 0 && bins[u - 1] == (int32_t)b) {
                sum[u - 1] = sum[u - 1] + pk[p].inten;
            } else {
                bins[u] = (int32_t)b;
                sum[u] = pk[p].inten;
                ++u;
            }
        }
        /* 6. normalise by the largest bin value and quantise */
        double smax = 0.0;
        for (int64_t p = 0; p < u; ++p)
            if (sum[p] > smax) smax = sum[p];
        for (int64_t p = 0; p < u; ++p) {
            int64_t lv = 0;
            if (smax > 0.0) {
                double v = sum[p] / smax;
                lv = (int64_t)floor(v * (double)Q);
                if (lv > (int64_t)Q - 1) lv = (int64_t)Q - 1;
            }
            out_bin[w] = bins[p];
            out_level[w] = (uint8_t)lv;
            ++w;
        }
        out_off[s + 1] = w;
    }
    free(pk);
    free(sum);
    free(bins);
    return w;
}

/* ------------------------------------------------------------------------ */
/*
 * Encoding (Section 3.3, Eq. 1): I = sum over peaks (i, j) of F_i (*) L_j in
 * bipolar form, then every positive component becomes +1 and every other
 * component -1. With bit 0 standing for +1 the element-wise product of two
 * bipolar vectors is the XOR of their bits, and a component whose sum is
 * zero (including every component of a spectrum with no peaks) becomes -1,
 * i.e. bit 1.
 * Per spectrum s the peaks are bin[off[s]..off[s+1]) with levels level[...];
 * out has n rows of D/32 words.
 */
ORACLE_API void oracle_encode(uint32_t D, const uint32_t *id, const uint32_t *lv, int64_t n,
                              const int64_t *off, const int32_t *bin, const uint8_t *level,
                              uint32_t *out)
{
    const uint32_t W = D / 32;
#pragma omp parallel
    {
        int32_t *I = (int32_t *)malloc((size_t)D * sizeof(int32_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t s = 0; s < n; ++s) {
            for (uint32_t d = 0; d < D; ++d) I[d] = 0;
            for (int64_t p = off[s]; p < off[s + 1]; ++p) {
                const uint32_t *F = id + (size_t)bin[p] * W;
                const uint32_t *L = lv + (size_t)level[p] * W;
                for (uint32_t wd = 0; wd < W; ++wd) {
                    const uint32_t x = F[wd] ^ L[wd];
                    for (uint32_t b = 0; b < 32; ++b)
                        I[wd * 32 + b] += ((x >> b) & 1u) ? -1 : +1;
                }
            }
            uint32_t *o = out + (size_t)s * W;
            for (uint32_t wd = 0; wd < W; ++wd) o[wd] = 0;
            for (uint32_t d = 0; d < D; ++d)
                if (!(I[d] > 0)) o[d >> 5] |= (1u << (d & 31));
        }
        free(I);
    }
}

/* Random-projection LSH baseline (Section 4.2): the spectrum vector, with
 * each kept bin weighted by (level + 1), projected on the random +-1 rows
 * (bit 0 = +1): S_d = sum over peaks of w * (+1 or -1); bit d = 0 if S_d > 0,
 * else 1 (the tie rule of Eq. 1's binarisation). */
ORACLE_API void oracle_encode_lsh(uint32_t D, const uint32_t *id, int64_t n, const int64_t *off,
                                  const int32_t *bin, const uint8_t *level, uint32_t *out)
{
    const uint32_t W = D / 32;
#pragma omp parallel
    {
        int64_t *S = (int64_t *)malloc((size_t)D * sizeof(int64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t s = 0; s < n; ++s) {
            for (uint32_t d = 0; d < D; ++d) S[d] = 0;
            for (int64_t p = off[s]; p < off[s + 1]; ++p) {
                const uint32_t *R = id + (size_t)bin[p] * W;
                const int64_t w = (int64_t)level[p] + 1;
                for (uint32_t d = 0; d < D; ++d)
                    S[d] += ((R[d >> 5] >> (d & 31)) & 1u) ? -w : w;
            }
            uint32_t *o = out + (size_t)s * W;
            for (uint32_t wd = 0; wd < W; ++wd) o[wd] = 0;
            for (uint32_t d = 0; d < D; ++d)
                if (!(S[d] > 0)) o[d >> 5] |= (1u << (d & 31));
        }
        free(S);
    }
}

/* ------------------------------------------------------------------------ */
/* Candidate filter (Section 3.4) and Hamming distance (Section 3.4; the
 * paper's Hamming similarity is D minus this distance).                     */

/* window kind: 0 = tolerance in Da, 1 = tolerance in ppm of the query's
 * precursor m/z, i.e. tol = (pmz_q * value) / 1e6. */
static void bounds(double pmz, int32_t kind, double value, double *lo, double *hi)
{
    double tol = (kind == 0) ? value : (pmz * value) / 1.0e6;
    *lo = pmz - tol;
    *hi = pmz + tol;
}

/* A reference is a candidate of a query when both have the same charge (if
 * charge_match) and lo <= pmz_ref <= hi. */
static int in_window(double pr, int8_t cr, int8_t cq, double lo, double hi, int charge_match)
{
    if (charge_match && cr != cq) return 0;
    return (lo <= pr) && (pr <= hi);
}

static int32_t hamming(const uint32_t *a, const uint32_t *b, uint32_t W)
{
    int32_t h = 0;
    for (uint32_t w = 0; w < W; ++w) h += __builtin_popcount(a[w] ^ b[w]);
    return h;
}

/*
 * Top-1 search: for every query, among its candidates, the reference with
 * the smallest Hamming distance (largest Hamming similarity); equal
 * distances go to the lowest library index. A query with no candidate gets
 * (-1, -1). kinds/values give each query's window (Section 3.4; Table 1).
 */
ORACLE_API void oracle_search(uint32_t D, int64_t nlib, const uint32_t *lib_hv,
                              const double *lib_pmz, const int8_t *lib_charge, int64_t nq,
                              const uint32_t *q_hv, const double *q_pmz, const int8_t *q_charge,
                              const int32_t *kinds, const double *values, int32_t charge_match,
                              int64_t *out_idx, int32_t *out_dist)
{
    const uint32_t W = D / 32;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
        double lo, hi;
        bounds(q_pmz[q], kinds[q], values[q], &lo, &hi);
        int64_t best_i = -1;
        int32_t best_d = -1;
        for (int64_t r = 0; r < nlib; ++r) {
            if (!in_window(lib_pmz[r], lib_charge[r], q_charge[q], lo, hi, charge_match)) continue;
            int32_t h = hamming(q_hv + (size_t)q * W, lib_hv + (size_t)r * W, W);
            if (best_i < 0 || h < best_d) {
                best_i = r;
                best_d = h;
            }
        }
        out_idx[q] = best_i;
        out_dist[q] = best_d;
    }
}

/* Number of candidates of every query (same rule as oracle_search). */
ORACLE_API void oracle_window_counts(int64_t nlib, const double *lib_pmz, const int8_t *lib_charge,
                                     int64_t nq, const double *q_pmz, const int8_t *q_charge,
                                     const int32_t *kinds, const double *values,
                                     int32_t charge_match, int64_t *out_count)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        double lo, hi;
        bounds(q_pmz[q], kinds[q], values[q], &lo, &hi);
        int64_t c = 0;
        for (int64_t r = 0; r < nlib; ++r)
            c += in_window(lib_pmz[r], lib_charge[r], q_charge[q], lo, hi, charge_match);
        out_count[q] = c;
    }
}

/* Every candidate of every query with its distance, in library order;
 * query q's entries start at row_off[q] (prefix sums of oracle_window_counts). */
ORACLE_API void oracle_window_distances(uint32_t D, int64_t nlib, const uint32_t *lib_hv,
                                        const double *lib_pmz, const int8_t *lib_charge,
                                        int64_t nq, const uint32_t *q_hv, const double *q_pmz,
                                        const int8_t *q_charge, const int32_t *kinds,
                                        const double *values, int32_t charge_match,
                                        const int64_t *row_off, int64_t *out_idx,
                                        int32_t *out_dist)
{
    const uint32_t W = D / 32;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nq; ++q) {
        double lo, hi;
        bounds(q_pmz[q], kinds[q], values[q], &lo, &hi);
        int64_t o = row_off[q];
        for (int64_t r = 0; r < nlib; ++r) {
            if (!in_window(lib_pmz[r], lib_charge[r], q_charge[q], lo, hi, charge_match)) continue;
            out_idx[o] = r;
            out_dist[o] = hamming(q_hv + (size_t)q * W, lib_hv + (size_t)r * W, W);
            ++o;
        }
    }
}

ORACLE_API int32_t oracle_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
