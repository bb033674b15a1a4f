/*
 * hyperoms.h — C ABI of libhyperoms, an MI355X (gfx950) implementation of the
 * data-parallel hot path of HyperOMS open modification spectral library
 * search (Kang, Xu, Bittremieux, Rosing; arXiv 2211.16422):
 *
 *   spectrum vectors --(Eq. 1 encoding, Section 3.3)--> binary hypervectors
 *   --(charge + precursor m/z filter and Hamming top-1, Section 3.4)--> best
 *   library match per query.
 *
 * Conventions
 *  - Every function returns homs_status (0 = success, < 0 = error) unless it
 *    is documented otherwise; no C++ exception crosses this boundary. The
 *    message of the last failure on a context is homs_last_error(ctx); errors
 *    raised before a context exists are reported by homs_last_error(NULL)
 *    (per thread).
 *  - Pointers prefixed h_ are host memory, d_ are device memory on the
 *    context's device. All buffers are owned by the caller and only used for
 *    the duration of the call, except where stated; the context owns its
 *    codebook, its sorted library and its workspaces.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it; calls documented as synchronous wait for
 *    it before returning.
 *  - Hypervectors are packed rows of D/32 uint32 words: bit d of a row is bit
 *    (d % 32) of word d / 32. A 0 bit stands for the bipolar component +1 and
 *    a 1 bit for -1, so the element-wise product of Eq. 1 is XOR.
 *  - After HOMS_E_DEVICE the context is unusable and only homs_destroy is
 *    valid. Other failures leave the context as it was.
 */
#ifndef HYPEROMS_H
#define HYPEROMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t homs_status;

#define HOMS_OK 0
#define HOMS_E_INVALID (-1)     /* bad argument */
#define HOMS_E_OOM (-2)         /* device or host allocation failed */
#define HOMS_E_DEVICE (-3)      /* HIP runtime or kernel failure (sticky) */
#define HOMS_E_STATE (-4)       /* call not valid in the context's state */
#define HOMS_E_UNSUPPORTED (-5) /* valid request this library version does not handle */

/*
 * Test hook: with the environment variable HOMS_TEST_FAIL_ALLOC=n, the n-th
 * device allocation of the library after the variable last changed value
 * fails without allocating, and the call that made it returns HOMS_E_OOM
 * (text after the number, as in "3:b", only re-arms the count). An
 * allocation failure leaves the context usable; unset, the variable costs
 * one getenv per allocation.
 */

typedef struct homs_ctx homs_ctx;

/*
 * Method parameters (Table 1; Section 4.2).
 *  dim          D, hypervector bits; a multiple of 512 in [512, 32768]
 *               (Section 4.2 uses 8192).
 *  n_levels     Q, intensity levels, 2..255 (Section 4.2 uses 16).
 *  top_n        most intense peaks kept per spectrum (Table 1: 50), >= 1.
 *  mz_min/max   fragment m/z range [mz_min, mz_max) (Table 1: 101 / 1500).
 *  bins_per_da  1 / bin width (Table 1: 20 for 0.05 Da, 25 for 0.04 Da).
 *  noise_frac   peaks below noise_frac x the most intense peak are dropped
 *               (Section 3.2: 0.01).
 *  id_flips     alpha, components flipped between the first and the last
 *               position hypervector (Section 3.3.1); 0 means D/2.
 *  charge_match 1: candidates must share the query's charge (Section 3.4);
 *               0: charge is ignored.
 *  seed         seed of the codebook's SplitMix64 stream.
 *  encoding     HOMS_ENCODING_*: the paper's ID-level encoding (Section 3.3),
 *               or one of the two baselines it is compared with in Section
 *               4.2 (Fig. 4(c)).
 */
typedef struct homs_params {
    uint32_t struct_size; /* sizeof(homs_params) */
    uint32_t dim;
    uint32_t n_levels;
    uint32_t top_n;
    double mz_min;
    double mz_max;
    double bins_per_da;
    double noise_frac;
    uint32_t id_flips;
    uint32_t charge_match;
    uint64_t seed;
    uint32_t encoding;
    uint32_t reserved;
} homs_params;

/* Encodings. ID_LEVEL: Eq. 1 with position vectors that keep locality
 * (Section 3.3.1) bound to level vectors (Section 3.3.2). RANDOM_ID: the same
 * binding and majority with independent random position vectors (the
 * ID-level HDC baseline of Section 4.2). LSH: random-projection hashing of
 * the spectrum vector (Section 4.2): bit d = 0 if sum over kept bins of
 * (level + 1) x (+1 or -1, bit d of the bin's random row) > 0, else 1. For
 * RANDOM_ID and LSH, row i of the position table is the next D/64 outputs of
 * the codebook stream after the level table's draws. */
#define HOMS_ENCODING_ID_LEVEL 0
#define HOMS_ENCODING_RANDOM_ID 1
#define HOMS_ENCODING_LSH 2

/* Precursor tolerance (Section 3.4; Table 1): kind 0 = +-value Da,
 * kind 1 = +-value ppm of the query precursor m/z, i.e. pmz * value / 1e6.
 * A library spectrum is a candidate when lo <= pmz_ref <= hi with
 * lo = pmz - tol and hi = pmz + tol computed in float64. */
#define HOMS_TOL_DA 0
#define HOMS_TOL_PPM 1
typedef struct homs_window {
    int32_t kind;
    int32_t reserved;
    double value;
} homs_window;

/* Search engines for homs_search_window. POPCOUNT: XOR + population count
 * on packed words (Section 3.4 with the bit packing of Section 4.1).
 * MFMA_I8 / MFMA_F8 / MFMA_F4: the same distances from the dot products of
 * the bipolar vectors (Section 3.3), H = (D - <x, y>) / 2, contracted on
 * matrix cores with operands expanded from the packed bits on the fly: int8
 * +-64 (int32 accumulate, 4096 <x, y>), fp8 e4m3 +-1.0, or fp4 e2m1 values
 * whose per-query dot product is an exact affine function of H (fp32
 * accumulate). Every partial sum is an integer exactly representable in its
 * accumulator, so all engines return identical results. */
#define HOMS_ENGINE_POPCOUNT 0
#define HOMS_ENGINE_MFMA_I8 1
#define HOMS_ENGINE_MFMA_F8 2
#define HOMS_ENGINE_MFMA_F4 3

/* Fills *p with Table 1 / Section 4.2 defaults (D = 8192, Q = 16, top 50,
 * [101, 1500) m/z, 0.05 Da bins, 1% noise floor, alpha = D/2, charge match,
 * seed 0). */
homs_status homs_params_default(homs_params *p);

/* Number of m/z bins f = ceil((mz_max - mz_min) * bins_per_da), i.e. the
 * number of position hypervectors; -1 if p is invalid. */
int64_t homs_num_bins(const homs_params *p);

const char *homs_status_string(homs_status s);
const char *homs_last_error(const homs_ctx *ctx);

/*
 * Host preprocessing of raw spectra into spectrum vectors (Section 3.2;
 * Table 1). Per spectrum: keep peaks with mz_min <= mz < mz_max; drop peaks
 * below noise_frac x the most intense remaining peak; keep the top_n most
 * intense (ties: lower m/z, then earlier peak); take the square root of each
 * intensity; bin = floor((mz - mz_min) * bins_per_da) (clamped to f - 1);
 * sum the values of peaks sharing a bin in ascending m/z order; divide by
 * the largest bin value; level = min(Q - 1, floor(v * Q)).
 * In:  n spectra; h_offsets[n + 1] (CSR, non-decreasing, h_offsets[0] = 0);
 *      h_mz and h_intensity[h_offsets[n]] (finite; intensity >= 0).
 * Out: h_out_offsets[n + 1]; h_out_bin (int32) and h_out_level (uint8), each
 *      with room for h_offsets[n] entries, receive per spectrum its unique
 *      bins in ascending order; *out_total = number of entries written.
 * Synchronous, host only; uses up to n_threads host threads (0 = all).
 */
homs_status homs_preprocess(const homs_params *p, int64_t n, const int64_t *h_offsets,
                            const double *h_mz, const double *h_intensity,
                            int64_t *h_out_offsets, int32_t *h_out_bin,
                            uint8_t *h_out_level, int64_t *out_total, int32_t n_threads);

/*
 * The same preprocessing (Section 3.2; Table 1) on the context's device, with
 * the context's parameters and identical results (float64 throughout), so
 * that encoding can start from raw peaks already in device memory.
 * In:  n spectra; d_offsets[n + 1] (int64 CSR, non-decreasing, d_offsets[0]
 *      = 0); d_mz and d_intensity[d_offsets[n]] (float64, finite; intensity
 *      >= 0). Spectra of any size; one that would keep more than 2048 peaks
 *      (min(peaks at or above the noise floor, top_n) > 2048, so only with
 *      top_n above 2048) gets no entries and raises device error bit 1
 *      (homs_device_errors).
 * Out: d_out_offsets[n + 1]; d_out_bin (int32) and d_out_level (uint8) with
 *      room for min(d_offsets[n], n * top_n) entries: per spectrum its unique
 *      bins in ascending order. All device pointers.
 * Asynchronous on `stream`; uses the context's workspace (grows on first use
 * of a larger n).
 */
homs_status homs_preprocess_device(homs_ctx *ctx, int64_t n, const int64_t *d_offsets,
                                   const double *d_mz, const double *d_intensity,
                                   int64_t *d_out_offsets, int32_t *d_out_bin,
                                   uint8_t *d_out_level, void *stream);

/*
 * Creates a context on HIP device `device` and generates the position and
 * level hypervectors from p->seed (Sections 3.3.1, 3.3.2): F_0 and the level
 * base L_0 are random bits, F_i flips the first floor(alpha*i/(f-1))
 * components of a random order of the D components, L_j flips the first
 * floor((D/2)*j/(Q-1)) components of another random order. Random numbers
 * come from one SplitMix64 stream (Steele et al., OOPSLA 2014) started at
 * the seed and consumed as: F_0 bits (D/64 outputs, bit d = bit d%64 of
 * output d/64), Fisher-Yates order of F (i = D-1..1, j = output mod (i+1)),
 * L_0 bits, order of L. Synchronous.
 */
homs_status homs_create(const homs_params *p, int32_t device, homs_ctx **out);

/* The same tables as homs_create generates, computed on the host into
 * h_id (f x D/32 words) and h_level (Q x D/32 words); no device needed. */
homs_status homs_generate_codebook(const homs_params *p, uint32_t *h_id, uint32_t *h_level);
void homs_destroy(homs_ctx *ctx);

/* Replaces the position table (f rows of D/32 words) and/or the level table
 * (Q rows) with caller-supplied host tables; NULL keeps the current one.
 * Invalidates an encoded library (state error on the next search until the
 * library is encoded again). Synchronous. */
homs_status homs_set_codebook(homs_ctx *ctx, const uint32_t *h_id, const uint32_t *h_level);
/* Copies the current tables to host buffers of f x D/32 and Q x D/32 words
 * (either may be NULL). Synchronous. */
homs_status homs_get_codebook(homs_ctx *ctx, uint32_t *h_id, uint32_t *h_level);

/*
 * Encodes n spectrum vectors with Eq. 1 (Section 3.3): I = sum over peaks
 * (bin i, level j) of F_i (*) L_j, then bit d = 0 if I_d > 0 and 1 otherwise
 * (so a tie, and every bit of a spectrum without peaks, is 1).
 * In:  d_offsets[n + 1] (int64 CSR); d_bin[...] (int32, each < f, unique
 *      within a spectrum), d_level[...] (uint8, each < Q).
 * Out: d_out[n][D/32] packed rows (uint32, 16-byte aligned) in input order.
 * Asynchronous on `stream`. A peak with an out-of-range bin or level is
 * skipped and raises a device error flag read by homs_device_errors().
 */
homs_status homs_encode_queries(homs_ctx *ctx, int64_t n, const int64_t *d_offsets,
                                const int32_t *d_bin, const uint8_t *d_level, uint32_t *d_out,
                                void *stream);

/*
 * Encodes the reference library (Section 3.3; references are encoded once
 * and reused) and keeps it on the device sorted by (charge, precursor m/z,
 * library index), which makes every query's candidates (Section 3.4) one
 * contiguous range. Library index = position in the input (references and
 * decoys as the caller orders them); 0 <= n < 2^31.
 * In: CSR as for homs_encode_queries; d_pmz[n] float64; d_charge[n] int8.
 * Replaces any previous library. Synchronous (waits for `stream`); returns
 * HOMS_E_INVALID if a bin or level was out of range.
 */
homs_status homs_encode_library(homs_ctx *ctx, int64_t n, const int64_t *d_offsets,
                                const int32_t *d_bin, const uint8_t *d_level,
                                const double *d_pmz, const int8_t *d_charge, void *stream);

/* Number of library spectra (0 before homs_encode_library). */
homs_status homs_library_size(const homs_ctx *ctx, int64_t *n);

/* Copies the encoded library into d_out[n][D/32] in library-index order.
 * Asynchronous on `stream`. */
homs_status homs_library_export(homs_ctx *ctx, uint32_t *d_out, void *stream);

/* The library's sorted order (test support): d_out_orig[j] (uint32) is the
 * library index of sorted row j, rows ordered by (charge, precursor m/z,
 * library index) (by (precursor m/z, library index) when charge_match = 0),
 * the order that makes every Section 3.4 candidate set one run of rows.
 * d_out_orig holds homs_library_size() entries. Asynchronous on `stream`. */
homs_status homs_library_order(homs_ctx *ctx, uint32_t *d_out_orig, void *stream);

/*
 * Candidate ranges (Section 3.4): for each query, [d_lo[q], d_hi[q]) in the
 * context's sorted library order; the count of candidates is hi - lo. NaN
 * precursors give empty ranges. Asynchronous on `stream`.
 */
homs_status homs_window_bounds(homs_ctx *ctx, int64_t nq, const double *d_q_pmz,
                               const int8_t *d_q_charge, const homs_window *win,
                               int64_t *d_lo, int64_t *d_hi, void *stream);

/*
 * Open (or standard) search, Section 3.4: for every query, the candidate
 * with the smallest Hamming distance (largest Hamming similarity
 * D - distance), equal distances going to the lowest library index.
 * In:  d_q_hv[nq][D/32] (16-byte aligned), d_q_pmz[nq], d_q_charge[nq],
 *      one window for all queries, engine = HOMS_ENGINE_*.
 * Out: d_out_idx[nq] (int64 library index, -1 if no candidate),
 *      d_out_dist[nq] (int32 Hamming distance, -1 if no candidate).
 * Asynchronous on `stream`; the context's workspace grows on first use of a
 * larger nq (a device allocation), so concurrent calls on one context race.
 */
homs_status homs_search_window(homs_ctx *ctx, int64_t nq, const uint32_t *d_q_hv,
                               const double *d_q_pmz, const int8_t *d_q_charge,
                               const homs_window *win, int32_t engine, int64_t *d_out_idx,
                               int32_t *d_out_dist, void *stream);

/*
 * homs_search_window without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, results and errors as
 * homs_search_window (the same kernels run), but the per-call scratch (window
 * bounds, query order, result keys) lives in a static device array of 8 MiB
 * that the library holds on each GPU it runs on until the process ends; the
 * call makes no hipMalloc, hipFree or other allocating call and records no
 * profiling events.
 * Limit: nq <= HOMS_NOALLOC_MAX_QUERIES; larger nq returns HOMS_E_INVALID.
 * Every call on one GPU (from any context) shares that GPU's array, and it
 * keeps the last call's contents: calls that overlap on one GPU (different
 * streams, threads or contexts) race and must be serialised by the caller.
 * Asynchronous on `stream`.
 */
#define HOMS_NOALLOC_MAX_QUERIES 131072
homs_status homs_search_window_noalloc(homs_ctx *ctx, int64_t nq, const uint32_t *d_q_hv,
                                       const double *d_q_pmz, const int8_t *d_q_charge,
                                       const homs_window *win, int32_t engine,
                                       int64_t *d_out_idx, int32_t *d_out_dist, void *stream);

/*
 * Cascade search, Section 3.4, with target-decoy FDR filtering (Section 2.1;
 * the fixed 1% level of Section 4.1 is fdr_level = 0.01). Stage 1 searches
 * every query with the narrow window; stage 2 searches, with the wide
 * window, every query that stage 1 did not identify. In each stage a PSM is a
 * query's top-1 match (score D - distance) and is a decoy match when
 * d_lib_decoy[its library index] != 0; FDR at distance threshold d = decoy
 * PSMs / target PSMs at distance <= d over that stage's PSMs (undefined,
 * never accepted, without a target); a PSM's q-value is the minimum FDR over
 * thresholds at or above its distance; a target PSM with q-value <=
 * fdr_level is an identification. Counts are exact and each FDR one IEEE
 * double division, so results are deterministic.
 * In:  queries as for homs_search_window; narrow and wide windows; engine =
 *      HOMS_ENGINE_*; d_lib_decoy[library size] (device, library order, the
 *      caller's indices); fdr_level in [0, 1].
 * Out: d_out_stage[nq] (int8): 1 = identified in stage 1, 2 = in stage 2,
 *      0 = not identified; d_out_idx / d_out_dist / d_out_qvalue[nq] (int64,
 *      int32, double): the stage-1 match and q-value for stage-1
 *      identifications, the stage-2 ones for every other query (-1, -1, +inf
 *      when its wide window is empty).
 * Asynchronous on `stream`; the workspace grows on first use of a larger nq.
 */
homs_status homs_cascade_search(homs_ctx *ctx, int64_t nq, const uint32_t *d_q_hv,
                                const double *d_q_pmz, const int8_t *d_q_charge,
                                const homs_window *narrow, const homs_window *wide,
                                int32_t engine, const uint8_t *d_lib_decoy, double fdr_level,
                                int64_t *d_out_idx, int32_t *d_out_dist, int8_t *d_out_stage,
                                double *d_out_qvalue, void *stream);

/*
 * Tunables of homs_search_batched, chosen by homs_autotune_batched or set by
 * the caller.
 *  narrow_max    a query with at most this many candidates is scored on its
 *                own by one wave (one candidate per lane); larger windows are
 *                scored in 256-query tiles sharing one candidate range.
 *  chunk_rows    candidate rows per tile work item.
 *  narrow_group  narrow queries per work item, a multiple of 4 (>= 4).
 *  grid          workgroups of the persistent kernel (1..65535).
 *  bucket_da     precursor bucket width (Da) used to order queries into tiles.
 *  engine        how wide tiles are scored: HOMS_ENGINE_POPCOUNT,
 *                HOMS_ENGINE_MFMA_F8 or HOMS_ENGINE_MFMA_F4 (the default)
 *                (all exact, see homs_search_window).
 */
typedef struct homs_batched_config {
    uint32_t narrow_max;
    uint32_t chunk_rows;
    uint32_t narrow_group;
    uint32_t grid;
    double bucket_da;
    int32_t engine;
} homs_batched_config;
homs_status homs_batched_config_get(const homs_ctx *ctx, homs_batched_config *out);
homs_status homs_batched_config_set(homs_ctx *ctx, const homs_batched_config *cfg);

/*
 * Search of a mixed query stream (Section 3.4, cascade search: narrow
 * standard windows and wide open windows, Table 1) in one persistent
 * launch: per query q the window is d_kinds[q] (HOMS_TOL_DA or
 * HOMS_TOL_PPM) with tolerance d_values[q]. Results are defined exactly as
 * for homs_search_window. Every step runs on the device with a fixed launch
 * shape and no host synchronisation; with use_graph = 1 the batch is
 * captured into a hipGraph on first use and replayed while nq, every
 * pointer argument, the configuration and the library stay the same (a
 * change re-captures). Asynchronous on `stream`; grows the workspace (a
 * device allocation) on first use of a larger nq. Calls on one context must
 * not overlap.
 */
homs_status homs_search_batched(homs_ctx *ctx, int64_t nq, const uint32_t *d_q_hv,
                                const double *d_q_pmz, const int8_t *d_q_charge,
                                const int8_t *d_kinds, const double *d_values,
                                int64_t *d_out_idx, int32_t *d_out_dist, int32_t use_graph,
                                void *stream);

/*
 * Autotuner of the batched search: times candidate configurations on the
 * given batch (coordinate descent over engine, chunk_rows, grid, narrow_max
 * and narrow_group from the current configuration, `reps` timed runs each after
 * one warm-up), keeps the fastest in the context and returns it with its
 * time per batch in *best_ms. The outputs hold the last run's (identical)
 * results. Synchronous.
 */
homs_status homs_autotune_batched(homs_ctx *ctx, int64_t nq, const uint32_t *d_q_hv,
                                  const double *d_q_pmz, const int8_t *d_q_charge,
                                  const int8_t *d_kinds, const double *d_values,
                                  int64_t *d_out_idx, int32_t *d_out_dist, int32_t reps,
                                  homs_batched_config *best, double *best_ms, void *stream);

/*
 * Every candidate of every query with its Hamming distance (test support).
 * d_row_off[nq + 1] are prefix sums of hi - lo from homs_window_bounds; query
 * q's candidates are written to [d_row_off[q], d_row_off[q + 1]) of d_out_idx
 * (library index) and d_out_dist, in sorted-library order. Asynchronous.
 */
homs_status homs_debug_distances(homs_ctx *ctx, int64_t nq, const uint32_t *d_q_hv,
                                 const double *d_q_pmz, const int8_t *d_q_charge,
                                 const homs_window *win, const int64_t *d_row_off,
                                 int64_t *d_out_idx, int32_t *d_out_dist, void *stream);

/* Reads and clears the context's device error flags (bit 0: a bin or level
 * out of range in an encode; bit 1: a spectrum over the device preprocessing
 * limit). Synchronous (waits for `stream`). */
homs_status homs_device_errors(homs_ctx *ctx, uint32_t *flags, void *stream);

/*
 * Kernel timing (measurement support). While enabled, every search and
 * encode call records HIP events on its stream around its main kernels;
 * homs_profile_read waits for those events, returns the accumulated times
 * and launch counts since the last read, and resets them.
 *  search_ms/search_launches: the Hamming search kernel (any engine);
 *  encode_ms/encode_launches: the encode kernels of homs_encode_queries and
 *           homs_encode_library (and the device preprocessing kernels);
 *  prep_ms: window, ordering and result kernels around the search kernel
 *           (and the query embedding of homs_search_learned), and the
 *           library sort of homs_encode_library;
 *  score_ms/score_launches: the matrix-core scoring kernels of
 *           homs_search_learned (two scoring launches and the threshold
 *           refinement between them, per pass of queries); their time is
 *           also part of search_ms.
 */
typedef struct homs_profile {
    double search_ms;
    double encode_ms;
    double prep_ms;
    int64_t search_launches;
    int64_t encode_launches;
    double score_ms;
    int64_t score_launches;
} homs_profile;
homs_status homs_profile_enable(homs_ctx *ctx, int32_t enable);
homs_status homs_profile_read(homs_ctx *ctx, homs_profile *out);

/*
 * ---- Learned shortlist ------------------------------------------------------
 * An extension beyond the paper: a small MLP embeds hypervectors into unit
 * vectors so that a query's exact nearest reference scores high; the search
 * then rescores only the k best-scoring candidates of each Section 3.4
 * window exactly by Hamming distance. The answer is the Section 3.4 top-1
 * restricted to that shortlist (exact whenever the true nearest candidate is
 * in it); queries whose shortlist cannot be formed fall back to the
 * exhaustive window search.
 *
 * Network (D -> hidden -> embed): x = bipolar form of the hypervector (bit 0
 * -> +1, bit 1 -> -1); h = ReLU(W1 x + b1); z = W2 h + b2;
 * e = z / sqrt(z.z + 1e-12); score(q, r) = e_q . e_r. Weights are fp32 masters
 * (row-major W1[hidden][D], W2[embed][hidden]) with bf16 copies feeding
 * matrix-core GEMMs that accumulate in fp32; hidden activations are rounded
 * to bf16 between the layers.
 * Training: InfoNCE over a batch of B (query, reference) pairs with in-batch
 * negatives, S_ij = e_qi . e_rj / tau, loss = mean_i (logsumexp_j S_ij - S_ii),
 * both towers sharing the weights; Adam (0.9, 0.999, 1e-8) updates them.
 *
 * A model belongs to one context, must be destroyed before it, and its calls
 * must not overlap with other calls on that context. Failures are reported
 * through homs_last_error(ctx).
 */
typedef struct homs_model homs_model;

/* New model on ctx's device with the given initial weights (host fp32:
 * h_W1[hidden][D], h_b1[hidden], h_W2[embed][hidden], h_b2[embed]); hidden and
 * embed are multiples of 32 (hidden <= 8192, embed <= 4096). Synchronous. */
homs_status homs_model_create(homs_ctx *ctx, int32_t hidden, int32_t embed, const float *h_W1,
                              const float *h_b1, const float *h_W2, const float *h_b2,
                              homs_model **out);
void homs_model_destroy(homs_model *model);

/* Replaces the weights and resets the optimiser state. Synchronous. */
homs_status homs_model_set_weights(homs_model *model, const float *h_W1, const float *h_b1,
                                   const float *h_W2, const float *h_b2);

/* Copies the fp32 weights to the host (NULL skips an array). Synchronous
 * (waits for the device). */
homs_status homs_model_get_weights(homs_model *model, float *h_W1, float *h_b1, float *h_W2,
                                   float *h_b2);

/* Unit embeddings d_out[n][embed] (fp32) of d_hv[n][D/32]. Asynchronous. */
homs_status homs_model_embed(homs_model *model, int64_t n, const uint32_t *d_hv, float *d_out,
                             void *stream);

/* Loss and gradients of one batch without updating the weights: d_q_hv and
 * d_r_hv hold `batch` rows each (16-byte aligned; batch a multiple of 32 in
 * [32, 16384]), pair i = (query row i, reference row i). Host outputs with the
 * weights' shapes (NULL skips one). Synchronous. */
homs_status homs_model_gradients(homs_model *model, int32_t batch, const uint32_t *d_q_hv,
                                 const uint32_t *d_r_hv, float tau, float *h_loss, float *h_gW1,
                                 float *h_gb1, float *h_gW2, float *h_gb2, void *stream);

/* One training step (loss, gradients, Adam update with learning rate lr); the
 * batch loss is written to d_loss[0] (device float). Asynchronous. */
homs_status homs_model_train_step(homs_model *model, int32_t batch, const uint32_t *d_q_hv,
                                  const uint32_t *d_r_hv, float tau, float lr, float *d_loss,
                                  void *stream);

/* Training schedule of homs_model_train (homs_train_config_default: 2
 * epochs, batch 1024, lr 3e-5, tau 0.02, seed 0). */
typedef struct homs_train_config {
    uint32_t struct_size; /* sizeof(homs_train_config) */
    int32_t epochs;       /* passes over the pairs, 1..1000 */
    int32_t batch;        /* pairs per step: a multiple of 32 in [32, 16384] */
    float lr;             /* Adam learning rate, >= 0 */
    float tau;            /* InfoNCE temperature, > 0 */
    uint32_t reserved;
    uint64_t seed;        /* seed of the epochs' batch order */
} homs_train_config;
homs_status homs_train_config_default(homs_train_config *cfg);

/*
 * Trains the model on (query, exact top-1 reference) pairs, the reference
 * being a row of the context's encoded library (the Section 3.4 search's
 * answer is the label). Pair i is query row d_q_hv[i] ([n][D/32], 16-byte
 * aligned) and library index d_target_idx[i] (int64, caller's library
 * order); a pair whose index is outside [0, library size) is skipped.
 * Schedule: the valid pairs are ordered by their reference's place in the
 * library's (charge, precursor m/z, library index) order, ties keeping pair
 * order, and cut into batches of cfg->batch consecutive pairs (a last partial
 * batch is dropped), so a batch's in-batch negatives are references of
 * neighbouring precursors. Epoch e takes the nb batches in increasing order of
 * key(b) = output e * nb + b (0-based) of the SplitMix64 stream seeded with
 * cfg->seed (ties: lower b), one homs_model_train_step per batch: the weights
 * after the call equal those after that sequence of homs_model_train_step
 * calls on the gathered rows.
 * Out: *out_steps = epochs * nb; d_losses (optional, device float, room for
 * epochs * floor(n / batch)) receives each step's loss in step order.
 * Synchronous (waits for `stream`); allocates and frees its own device
 * buffers.
 */
homs_status homs_model_train(homs_model *model, int64_t n, const uint32_t *d_q_hv,
                             const int64_t *d_target_idx, const homs_train_config *cfg,
                             float *d_losses, int64_t *out_steps, void *stream);

/* Embeds the context's encoded library into the model's scoring
 * embeddings (sorted library order): for each row the unit embedding e
 * rounded as E4M3(16 e) (the 8-bit E4M3 format of the OCP 8-bit floating
 * point specification, nearest value, ties to even), kept as E4M3 codes and,
 * divided by 16, as bf16. Needed before homs_search_learned and again after
 * the library or the weights change. Asynchronous; grows its buffers (device
 * allocations) when the library grew. */
homs_status homs_model_embed_library(homs_model *model, void *stream);

/* Test support: copies the stored scoring embeddings of the library (sorted
 * order, the order of homs_library_order) to d_out_fp8 [n][E] (E4M3 codes of
 * 16 e) and/or d_out_bf16 [n][E] (those values / 16, bf16 bits); either may
 * be NULL. HOMS_E_STATE without homs_model_embed_library. Asynchronous. */
homs_status homs_model_library_embeddings(homs_model *model, uint8_t *d_out_fp8,
                                          uint16_t *d_out_bf16, void *stream);

/*
 * Shortlist search: for each query, the k (1 <= k <= 1024) candidates of its
 * window with the largest scores (score = dot product of the two scoring
 * embeddings, see homs_model_embed_library; ties to the lower library index)
 * are rescored exactly; d_out_idx / d_out_dist are the Hamming top-1 over
 * them (lowest library index among equal distances; -1 / -1 without
 * candidates). Candidates are found with score thresholds (one estimated
 * from a sample of the window, then one refined from the hits in every
 * eighth 128-row block of the sorted library). d_out_fallback[q] != 0 marks
 * a query whose shortlist could not be formed this way, with the reason: 1
 * its candidate buffer overflowed, 2 a threshold kept fewer than
 * min(k, window) candidates, 3 the k-th kept candidate scores below the
 * refined threshold; its result is the exhaustive window search. d_out_shortlist (optional, [nq][k] int64) receives each query's
 * shortlist by descending score, -1 past the window's size and for fallback
 * queries. Same query arguments as homs_search_window. The model's embed size
 * must be 64, 128 or 256 (HOMS_E_UNSUPPORTED otherwise). Asynchronous; grows
 * the context's workspace on first use of a larger nq.
 */
homs_status homs_search_learned(homs_ctx *ctx, homs_model *model, int64_t nq,
                                const uint32_t *d_q_hv, const double *d_q_pmz,
                                const int8_t *d_q_charge, const homs_window *win, int32_t k,
                                int64_t *d_out_idx, int32_t *d_out_dist, uint8_t *d_out_fallback,
                                int64_t *d_out_shortlist, void *stream);

/*
 * ---- Library and model files --------------------------------------------------
 * The paper keeps preprocessed spectra in a reusable binary file (Section 3.2)
 * and encodes reference hypervectors once for reuse (Sections 3.3 and 4.4);
 * these calls keep an encoded library, and a trained model, across
 * processes. All numbers are little-endian; each file ends with a 64-bit
 * checksum of every byte before it: h = 0xcbf29ce484222325, then for each
 * 8-byte little-endian word w (the last one zero-padded) h = (h ^ w) *
 * 0x100000001b3 mod 2^64.
 *
 * Library file (96-byte header, then the sorted library):
 *   char magic[8] = "HOMSLIB1"; uint32 version (1), dim, n_levels, top_n,
 *   id_flips (resolved: D/2 when the parameter was 0), charge_match,
 *   encoding, reserved (0); double mz_min, mz_max, bins_per_da, noise_frac;
 *   uint64 seed; uint64 codebook_hash (the checksum above over the position
 *   table's words, then the level table's); int64 n;
 *   uint32 orig[n] (library index of each sorted row); double pmz[n];
 *   int8 charge[n] (0 when charge_match = 0); uint32 hv[n][D/32];
 *   uint64 checksum.
 * Model file (32-byte header):
 *   char magic[8] = "HOMSMDL1"; uint32 version (1), dim; int32 hidden,
 *   embed; int64 step (Adam steps taken); then float32 W1[hidden][D],
 *   b1[hidden], W2[embed][hidden], b2[embed] and the Adam first and second
 *   moments of each, in the order mW1, vW1, mb1, vb1, mW2, vW2, mb2, vb2;
 *   uint64 checksum.
 */
#define HOMS_FILE_LIBRARY 1
#define HOMS_FILE_MODEL 2

/* Writes the context's encoded library to `path` (replacing the file).
 * Synchronous; on failure no file is left behind. */
homs_status homs_library_save(homs_ctx *ctx, const char *path);

/* Replaces the context's library with the one in `path`. The file must have
 * been written with the context's parameters and codebook (HOMS_E_INVALID
 * otherwise, as for a damaged or inconsistent file: a checksum mismatch, a
 * size that does not match the header, an order that is not a permutation
 * sorted by (charge, precursor m/z, library index)); the context is then as
 * after homs_encode_library of the same spectra. Synchronous. */
homs_status homs_library_load(homs_ctx *ctx, const char *path);

/* Writes the model (weights, Adam moments and step count) to `path`, so
 * training can resume where it stopped. Synchronous. */
homs_status homs_model_save(homs_model *model, const char *path);

/* New model on ctx from a model file (dim must equal the context's D).
 * Library embeddings are not stored: call homs_model_embed_library before
 * homs_search_learned. Synchronous. */
homs_status homs_model_load(homs_ctx *ctx, const char *path, homs_model **out);

/* homs_file_inspect: what a file holds, read and checked on the host (no
 * device needed): kind (HOMS_FILE_LIBRARY or HOMS_FILE_MODEL), version, dim;
 * for a library n, codebook_hash and the parameters it was encoded with
 * (other fields of params at their defaults); for a model hidden, embed and
 * step. Verifies the size and the checksum (HOMS_E_INVALID when the file is
 * damaged). */
typedef struct homs_file_info {
    uint32_t kind;
    uint32_t version;
    uint32_t dim;
    int32_t hidden;
    int32_t embed;
    int32_t reserved;
    int64_t n;
    int64_t step;
    uint64_t codebook_hash;
    homs_params params;
} homs_file_info;
homs_status homs_file_inspect(const char *path, homs_file_info *out);

/*
 * Measurement support: sustained rate, in 32-bit lane operations per second,
 * of the v_xor_b32 + v_bcnt_u32_b32 pair the popcount search is made of,
 * from a kernel of 16 independent chains per lane filling every compute unit
 * of `device` (best of three runs). Synchronous; allocates and frees a small
 * device buffer.
 */
homs_status homs_measure_xor_popcount_rate(int32_t device, double *lane_ops_per_s);

#ifdef __cplusplus
}
#endif

#endif /* HYPEROMS_H */
