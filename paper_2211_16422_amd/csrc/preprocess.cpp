// Host preprocessing (Section 3.2; Table 1): raw peaks -> unique
// (m/z bin, intensity level) pairs per spectrum, ready for encoding.
//
// Order of the steps: m/z range filter, 1% noise floor relative to the most
// intense peak in range, top-N most intense (ties: lower m/z, then earlier
// peak), square-root scaling, binning with floor((mz - mz_min) * bins/Da)
// and summing of colliding peaks in ascending m/z, normalisation by the
// largest bin and quantisation to Q levels (min(Q - 1, floor(v * Q))).
// All arithmetic is float64 with correctly rounded operations in this fixed
// order (the library is built with -ffp-contract=off), so the result is
// reproducible bit for bit.
#include "preprocess.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace homs {
namespace {

struct Peak {
    double mz;
    double inten;
    int64_t pos;
};

// writes the spectrum's unique bins to bin_out/level_out, returns how many
int64_t one_spectrum(const PreprocessParams& p, const double* mz, const double* it, int64_t np,
                     std::vector<Peak>& pk, int32_t* bin_out, uint8_t* level_out,
                     std::vector<double>& sums)
{
    pk.clear();
    for (int64_t i = 0; i < np; ++i)
        if (mz[i] >= p.mz_min && mz[i] < p.mz_max) pk.push_back(Peak{mz[i], it[i], i});

    double imax = 0.0;
    for (const Peak& k : pk) imax = std::max(imax, k.inten);
    const double floor_i = p.noise_frac * imax;
    pk.erase(std::remove_if(pk.begin(), pk.end(), [&](const Peak& k) { return k.inten < floor_i; }),
             pk.end());

    if (pk.size() > (size_t)p.top_n) {
        auto stronger = [](const Peak& a, const Peak& b) {
            if (a.inten != b.inten) return a.inten > b.inten;
            if (a.mz != b.mz) return a.mz < b.mz;
            return a.pos < b.pos;
        };
        std::partial_sort(pk.begin(), pk.begin() + p.top_n, pk.end(), stronger);
        pk.resize(p.top_n);
    }
    for (Peak& k : pk) k.inten = std::sqrt(k.inten);
    std::sort(pk.begin(), pk.end(), [](const Peak& a, const Peak& b) {
        if (a.mz != b.mz) return a.mz < b.mz;
        return a.pos < b.pos;
    });

    int64_t u = 0;
    sums.clear();
    for (const Peak& k : pk) {
        int64_t b = (int64_t)std::floor((k.mz - p.mz_min) * p.bins_per_da);
        b = std::min<int64_t>(std::max<int64_t>(b, 0), p.n_bins - 1);
        if (u > 0 && bin_out[u - 1] == (int32_t)b) {
            sums[u - 1] = sums[u - 1] + k.inten;
        } else {
            bin_out[u] = (int32_t)b;
            sums.push_back(k.inten);
            ++u;
        }
    }
    double smax = 0.0;
    for (int64_t i = 0; i < u; ++i) smax = std::max(smax, sums[i]);
    for (int64_t i = 0; i < u; ++i) {
        int64_t lv = 0;
        if (smax > 0.0) {
            const double v = sums[i] / smax;
            lv = std::min<int64_t>((int64_t)std::floor(v * (double)p.n_levels),
                                   (int64_t)p.n_levels - 1);
        }
        level_out[i] = (uint8_t)lv;
    }
    return u;
}

template <class F>
void parallel_ranges(int64_t n, int threads, F&& fn)
{
    if (threads <= 1 || n < 1024) {
        fn(0, n, 0);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t step = (n + threads - 1) / threads;
    for (int t = 0; t < threads; ++t) {
        const int64_t a = t * step, b = std::min(n, a + step);
        if (a >= b) break;
        pool.emplace_back([&, a, b, t] { fn(a, b, t); });
    }
    for (auto& th : pool) th.join();
}

}  // namespace

bool preprocess_spectra(const PreprocessParams& p, int64_t n, const int64_t* off, const double* mz,
                        const double* intensity, int64_t* out_off, int32_t* out_bin,
                        uint8_t* out_level, int64_t* out_total, int n_threads, std::string* why)
{
    if (n < 0) {
        *why = "n < 0";
        return false;
    }
    if (off[0] != 0) {
        *why = "offsets[0] != 0";
        return false;
    }
    for (int64_t s = 0; s < n; ++s)
        if (off[s + 1] < off[s]) {
            *why = "offsets decrease at spectrum " + std::to_string(s);
            return false;
        }
    int threads = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    threads = std::min(threads, 64);
    const int64_t total_in = off[n];
    std::vector<char> bad(threads, 0);
    parallel_ranges(total_in, threads, [&](int64_t a, int64_t b, int t) {
        for (int64_t i = a; i < b; ++i)
            if (!std::isfinite(mz[i]) || !std::isfinite(intensity[i]) || intensity[i] < 0.0) {
                bad[t] = 1;
                return;
            }
    });
    for (char c : bad)
        if (c) {
            *why = "non-finite m/z or intensity, or negative intensity";
            return false;
        }

    // pass 1: each spectrum's result at its input offset (there is room:
    // unique bins <= input peaks); pass 2: compact left.
    std::vector<int64_t> count(n);
    parallel_ranges(n, threads, [&](int64_t a, int64_t b, int) {
        std::vector<Peak> pk;
        std::vector<double> sums;
        for (int64_t s = a; s < b; ++s)
            count[s] = one_spectrum(p, mz + off[s], intensity + off[s], off[s + 1] - off[s], pk,
                                    out_bin + off[s], out_level + off[s], sums);
    });
    int64_t w = 0;
    out_off[0] = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (w != off[s] && count[s] > 0) {
            std::memmove(out_bin + w, out_bin + off[s], (size_t)count[s] * sizeof(int32_t));
            std::memmove(out_level + w, out_level + off[s], (size_t)count[s]);
        }
        w += count[s];
        out_off[s + 1] = w;
    }
    *out_total = w;
    return true;
}

}  // namespace homs
