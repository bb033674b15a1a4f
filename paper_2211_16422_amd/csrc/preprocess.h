// Host-side preprocessing of raw spectra into spectrum vectors.
#pragma once
#include <stdint.h>

#include <string>

namespace homs {

struct PreprocessParams {
    double mz_min, mz_max, bins_per_da, noise_frac;
    uint32_t top_n, n_levels;
    int64_t n_bins;
};

// Returns false (with *why set) on invalid input; see homs_preprocess.
bool preprocess_spectra(const PreprocessParams& p, int64_t n, const int64_t* off,
                        const double* mz, const double* intensity, int64_t* out_off,
                        int32_t* out_bin, uint8_t* out_level, int64_t* out_total,
                        int n_threads, std::string* why);

}  // namespace homs
