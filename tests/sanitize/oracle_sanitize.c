/* Address and undefined-behaviour sanitizer run of the oracle
 * (oracle/hyperoms_oracle.c, built into this program without OpenMP by
 * tests/test_sanitizers_cpu.py with gcc -fsanitize=address,undefined). It
 * drives every oracle function with small ragged and edge-case inputs and
 * checks invariants that need no reference (distances in [0, D], counts
 * equal to the listed candidates, top-1 equal to the smallest listed
 * distance). Exit status 0 means no sanitizer report and no failed check. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_codebook(uint32_t D, uint32_t f, uint32_t Q, uint32_t alpha, uint64_t seed,
                    uint32_t encoding, uint32_t *id_out, uint32_t *lv_out);
int64_t oracle_num_bins(double mz_min, double mz_max, double bins_per_da);
int64_t oracle_preprocess(int64_t n, const int64_t *off, const double *mz, const double *inten,
                          double mz_min, double mz_max, double bins_per_da, double noise_frac,
                          uint32_t top_n, uint32_t Q, int64_t *out_off, int32_t *out_bin,
                          uint8_t *out_level);
void oracle_encode(uint32_t D, const uint32_t *id, const uint32_t *lv, int64_t n,
                   const int64_t *off, const int32_t *bin, const uint8_t *level, uint32_t *out);
void oracle_encode_lsh(uint32_t D, const uint32_t *id, int64_t n, const int64_t *off,
                       const int32_t *bin, const uint8_t *level, uint32_t *out);
void oracle_search(uint32_t D, int64_t nlib, const uint32_t *lib_hv, const double *lib_pmz,
                   const int8_t *lib_charge, int64_t nq, const uint32_t *q_hv,
                   const double *q_pmz, const int8_t *q_charge, const int32_t *kinds,
                   const double *values, int32_t charge_match, int64_t *out_idx,
                   int32_t *out_dist);
void oracle_window_counts(int64_t nlib, const double *lib_pmz, const int8_t *lib_charge,
                          int64_t nq, const double *q_pmz, const int8_t *q_charge,
                          const int32_t *kinds, const double *values, int32_t charge_match,
                          int64_t *out_count);
void oracle_window_distances(uint32_t D, int64_t nlib, const uint32_t *lib_hv,
                             const double *lib_pmz, const int8_t *lib_charge, int64_t nq,
                             const uint32_t *q_hv, const double *q_pmz, const int8_t *q_charge,
                             const int32_t *kinds, const double *values, int32_t charge_match,
                             const int64_t *row_off, int64_t *out_idx, int32_t *out_dist);
int32_t oracle_max_threads(void);

static int failures = 0;
static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "check failed: %s\n", what);
        ++failures;
    }
}

static uint64_t rng_state = 12345;
static uint64_t next_u64(void) /* xorshift64*, test data only */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545F4914F6CDD1Dull;
}
static double uniform(double a, double b) { return a + (b - a) * (double)(next_u64() >> 11) / 9007199254740992.0; }

int main(void)
{
    const uint32_t D = 512, W = D / 32, Q = 16;
    const double mz_min = 101.0, mz_max = 1500.0, bpd = 25.0;
    const int64_t nb = oracle_num_bins(mz_min, mz_max, bpd);
    check(nb == 34975, "bin count");
    check(oracle_codebook(100, 10, Q, 50, 1, 0, NULL, NULL) == -1, "D not a multiple of 64");
    check(oracle_codebook(D, 0, Q, 50, 1, 0, NULL, NULL) == -1, "f = 0");
    check(oracle_max_threads() >= 1, "thread count");

    uint32_t *id = malloc((size_t)nb * W * 4), *lv = malloc((size_t)Q * W * 4);
    check(oracle_codebook(D, (uint32_t)nb, Q, D / 2, 7, 0, id, lv) == 0, "codebook");

    /* ragged spectra: empty, out of range, ties, one large */
    enum { NS = 60 };
    int64_t off[NS + 1];
    off[0] = 0;
    int64_t cap = 0;
    int np[NS];
    for (int s = 0; s < NS; ++s) {
        np[s] = s == 0 ? 0 : s == 1 ? 3 : s == 2 ? 4 : s == NS - 1 ? 3000 : (int)(next_u64() % 200);
        cap += np[s];
        off[s + 1] = cap;
    }
    double *mz = malloc((size_t)(cap + 1) * 8), *in = malloc((size_t)(cap + 1) * 8);
    for (int64_t p = 0; p < cap; ++p) {
        mz[p] = uniform(50.0, 1600.0);
        in[p] = uniform(0.0, 1000.0);
    }
    mz[off[1]] = 10.0; mz[off[1] + 1] = 1600.0; mz[off[1] + 2] = mz_max; /* out of range */
    for (int k = 0; k < 4; ++k) { mz[off[2] + k] = 500.0; in[off[2] + k] = 5.0; } /* ties */
    int64_t out_off[NS + 1];
    int32_t *bin = malloc((size_t)(cap + 1) * 4);
    uint8_t *level = malloc((size_t)(cap + 1));
    const int64_t total = oracle_preprocess(NS, off, mz, in, mz_min, mz_max, bpd, 0.01, 50, Q,
                                            out_off, bin, level);
    check(total >= 0 && out_off[NS] == total, "preprocess total");
    check(out_off[1] - out_off[0] == 0 && out_off[2] - out_off[1] == 0, "empty spectra stay empty");
    check(out_off[3] - out_off[2] == 1, "ties share one bin");
    for (int s = 0; s < NS; ++s)
        for (int64_t e = out_off[s]; e < out_off[s + 1]; ++e) {
            check(bin[e] >= 0 && bin[e] < nb && level[e] < Q, "entry in range");
            if (e > out_off[s]) check(bin[e] > bin[e - 1], "bins ascend");
        }

    uint32_t *hv = malloc((size_t)NS * W * 4), *hv2 = malloc((size_t)NS * W * 4);
    oracle_encode(D, id, lv, NS, out_off, bin, level, hv);
    uint32_t *rid = malloc((size_t)nb * W * 4), *rlv = malloc((size_t)Q * W * 4);
    check(oracle_codebook(D, (uint32_t)nb, Q, D / 2, 7, 2, rid, rlv) == 0, "LSH codebook");
    oracle_encode_lsh(D, rid, NS, out_off, bin, level, hv2);

    /* library = the spectra, queries = the same spectra with shifted precursors */
    double pmz[NS], qpmz[NS], values[NS];
    int8_t ch[NS], qch[NS];
    int32_t kinds[NS];
    for (int s = 0; s < NS; ++s) {
        pmz[s] = uniform(400.0, 1200.0);
        ch[s] = (int8_t)(2 + s % 2);
        qpmz[s] = s == 5 ? NAN : pmz[(s * 7) % NS] + uniform(-1.0, 1.0);
        qch[s] = s == 6 ? 9 : ch[(s * 7) % NS];
        kinds[s] = s % 3 == 0 ? 1 : 0;
        values[s] = s % 3 == 0 ? 20.0 : s % 3 == 1 ? 500.0 : 0.0;
    }
    int64_t cnt[NS], ridx[NS], rowoff[NS + 1];
    int32_t rdist[NS];
    oracle_window_counts(NS, pmz, ch, NS, qpmz, qch, kinds, values, 1, cnt);
    rowoff[0] = 0;
    for (int s = 0; s < NS; ++s) rowoff[s + 1] = rowoff[s] + cnt[s];
    int64_t *lidx = malloc((size_t)(rowoff[NS] + 1) * 8);
    int32_t *ldist = malloc((size_t)(rowoff[NS] + 1) * 4);
    oracle_window_distances(D, NS, hv, pmz, ch, NS, hv, qpmz, qch, kinds, values, 1, rowoff,
                            lidx, ldist);
    oracle_search(D, NS, hv, pmz, ch, NS, hv, qpmz, qch, kinds, values, 1, ridx, rdist);
    check(cnt[5] == 0 && cnt[6] == 0, "NaN precursor and absent charge have no candidates");
    for (int s = 0; s < NS; ++s) {
        int64_t bi = -1;
        int32_t bd = -1;
        for (int64_t e = rowoff[s]; e < rowoff[s + 1]; ++e) {
            check(ldist[e] >= 0 && ldist[e] <= (int32_t)D, "distance in [0, D]");
            if (bi < 0 || ldist[e] < bd) { bi = lidx[e]; bd = ldist[e]; }
        }
        check(ridx[s] == bi && rdist[s] == bd, "top-1 is the smallest listed distance");
    }
    oracle_search(D, 0, hv, pmz, ch, NS, hv, qpmz, qch, kinds, values, 0, ridx, rdist);
    for (int s = 0; s < NS; ++s) check(ridx[s] == -1 && rdist[s] == -1, "empty library");

    free(id); free(lv); free(rid); free(rlv); free(mz); free(in); free(bin); free(level);
    free(hv); free(hv2); free(lidx); free(ldist);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: all checks passed\n");
    return 0;
}
