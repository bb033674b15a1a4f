// Address and undefined-behaviour sanitizer run of the library's host code
// (preprocessing, codebook generation, checksummed file IO), built with g++
// -fsanitize=address,undefined by tests/test_sanitizers_cpu.py. It drives
// every entry point with ordinary and edge-case inputs and checks the few
// invariants that need no reference; the results themselves are checked
// against the oracle elsewhere. Exit status 0 means no sanitizer report and
// no failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include <unistd.h>

#include "codebook.h"
#include "persist.h"
#include "preprocess.h"

namespace {

int failures = 0;

void check(bool ok, const char* what)
{
    if (!ok) {
        std::fprintf(stderr, "check failed: %s\n", what);
        ++failures;
    }
}

// ragged spectra with every awkward case in one batch
struct Batch {
    std::vector<int64_t> off{0};
    std::vector<double> mz, in;
    void add(const std::vector<double>& m, const std::vector<double>& i)
    {
        mz.insert(mz.end(), m.begin(), m.end());
        in.insert(in.end(), i.begin(), i.end());
        off.push_back((int64_t)mz.size());
    }
};

void run_preprocess()
{
    homs::PreprocessParams p{};
    p.mz_min = 101.0;
    p.mz_max = 1500.0;
    p.bins_per_da = 1.0 / 0.04;
    p.noise_frac = 0.01;
    p.top_n = 50;
    p.n_levels = 16;
    p.n_bins = (int64_t)std::ceil((p.mz_max - p.mz_min) * p.bins_per_da);
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> umz(50.0, 1600.0), uin(0.0, 1000.0);
    Batch b;
    b.add({}, {});                                      // no peaks
    b.add({50.0, 1600.0, 100.99}, {1.0, 2.0, 3.0});    // all out of range
    b.add({101.0, 1499.999}, {0.0, 0.0});              // range edges, zero intensities
    b.add({500.0, 500.0, 500.0}, {5.0, 5.0, 5.0});     // exact ties, one bin
    b.add({200.0, 200.01, 200.02}, {1e-300, 1e300, 4.0});  // colliding bins, extreme values
    for (int s = 0; s < 200; ++s) {                     // ragged random spectra
        const int np = (int)(rng() % 400);
        std::vector<double> m(np), i(np);
        for (int k = 0; k < np; ++k) {
            m[k] = umz(rng);
            i[k] = uin(rng);
        }
        b.add(m, i);
    }
    {  // one very large spectrum
        std::vector<double> m(20000), i(20000);
        for (int k = 0; k < 20000; ++k) {
            m[k] = umz(rng);
            i[k] = uin(rng);
        }
        b.add(m, i);
    }
    const int64_t n = (int64_t)b.off.size() - 1;
    for (int threads : {1, 4}) {
        for (uint32_t top_n : {1u, 50u, 100000u}) {
            p.top_n = top_n;
            std::vector<int64_t> out_off(n + 1, -1);
            std::vector<int32_t> out_bin(b.mz.size() + 1);
            std::vector<uint8_t> out_level(b.mz.size() + 1);
            int64_t total = -1;
            std::string why;
            const bool ok = homs::preprocess_spectra(p, n, b.off.data(), b.mz.data(), b.in.data(),
                                                     out_off.data(), out_bin.data(),
                                                     out_level.data(), &total, threads, &why);
            check(ok, "preprocess on valid input");
            check(out_off[0] == 0 && out_off[n] == total, "offsets frame the output");
            for (int64_t s = 0; s < n; ++s) {
                check(out_off[s + 1] >= out_off[s], "offsets ascend");
                check(out_off[s + 1] - out_off[s] <= (int64_t)top_n, "at most top_n entries");
                for (int64_t e = out_off[s]; e < out_off[s + 1]; ++e) {
                    check(out_bin[e] >= 0 && out_bin[e] < p.n_bins, "bin in range");
                    check(out_level[e] < p.n_levels, "level in range");
                    if (e > out_off[s]) check(out_bin[e] > out_bin[e - 1], "bins ascend");
                }
            }
        }
    }
    {  // an empty batch; invalid input is refused
        std::vector<int64_t> off{0}, out_off(1);
        int64_t total = -1;
        std::string why;
        check(homs::preprocess_spectra(p, 0, off.data(), nullptr, nullptr, out_off.data(),
                                       nullptr, nullptr, &total, 2, &why) && total == 0,
              "empty batch");
        std::vector<int64_t> out_off2(n + 1);
        std::vector<int32_t> ob(b.mz.size() + 1);
        std::vector<uint8_t> ol(b.mz.size() + 1);
        std::vector<double> nan_in = b.in;
        nan_in[b.off[6]] = std::numeric_limits<double>::quiet_NaN();
        const bool ok = homs::preprocess_spectra(p, n, b.off.data(), b.mz.data(), nan_in.data(),
                                                 out_off2.data(), ob.data(), ol.data(), &total, 3,
                                                 &why);
        check(!ok && !why.empty(), "a NaN intensity is refused");
        std::vector<int64_t> bad_off{0, 5, 3};
        const bool ok2 = homs::preprocess_spectra(p, 2, bad_off.data(), b.mz.data(), b.in.data(),
                                                  out_off2.data(), ob.data(), ol.data(), &total, 1,
                                                  &why);
        check(!ok2, "descending offsets are refused");
    }
}

void run_codebook()
{
    for (uint32_t D : {64u, 512u, 8192u})
        for (uint32_t f : {1u, 37u})
            for (uint32_t Q : {2u, 16u})
                for (uint32_t enc : {0u, 1u, 2u}) {
                    const uint32_t W = D / 32;
                    std::vector<uint32_t> id((size_t)f * W + 1, 0xDEADBEEFu),
                        lv((size_t)Q * W + 1, 0xDEADBEEFu);
                    homs::generate_codebook(D, f, Q, D / 2, 42, enc, id.data(), lv.data());
                    check(id[(size_t)f * W] == 0xDEADBEEFu, "no write past the ID table");
                    check(lv[(size_t)Q * W] == 0xDEADBEEFu, "no write past the level table");
                    // the two extreme levels differ in alpha = D / 2 bits
                    int diff = 0;
                    for (uint32_t w = 0; w < W; ++w)
                        diff += __builtin_popcount(lv[w] ^ lv[(size_t)(Q - 1) * W + w]);
                    check(diff == (int)(D / 2), "extreme levels differ in alpha bits");
                }
}

void run_files()
{
    char path[] = "/tmp/homs_sanitize_XXXXXX";
    const int fd = mkstemp(path);
    check(fd >= 0, "temporary file");
    if (fd < 0) return;
    close(fd);
    std::mt19937_64 rng(3);
    std::vector<uint8_t> data(1 << 20);
    for (auto& x : data) x = (uint8_t)rng();
    const size_t chunks[] = {0, 1, 7, 8, 9, 4095, 65536, 3, 100000};
    {
        homs::FileWriter w;
        std::string err;
        check(w.open(path, &err), "open for writing");
        size_t at = 0;
        for (size_t c : chunks) {
            check(w.write(data.data() + at, c), "write");
            at += c;
        }
        check(w.finish(&err), "finish writing");
    }
    size_t total = 0;
    for (size_t c : chunks) total += c;
    {  // read back in other chunk sizes
        homs::FileReader r;
        std::string err;
        check(r.open(path, &err), "open for reading");
        std::vector<uint8_t> back(total);
        size_t at = 0;
        while (at < total) {
            const size_t c = std::min<size_t>(total - at, 1 + (rng() % 5000));
            check(r.read(back.data() + at, c), "read");
            at += c;
        }
        check(r.finish(&err), "checksum verified");
        check(std::memcmp(back.data(), data.data(), total) == 0, "bytes read back");
    }
    {  // one flipped byte fails the checksum
        FILE* f = std::fopen(path, "r+b");
        check(f != nullptr, "reopen");
        if (f) {
            std::fseek(f, 12345, SEEK_SET);
            const int c = std::fgetc(f);
            std::fseek(f, 12345, SEEK_SET);
            std::fputc(c ^ 1, f);
            std::fclose(f);
        }
        homs::FileReader r;
        std::string err;
        check(r.open(path, &err), "open the damaged file");
        std::vector<uint8_t> back(total);
        check(r.read(back.data(), total), "read the damaged file");
        check(!r.finish(&err) && !err.empty(), "damaged file refused");
    }
    {  // a read past the end fails cleanly
        homs::FileReader r;
        std::string err;
        check(r.open(path, &err), "open");
        std::vector<uint8_t> back(total + 100);
        check(!r.read(back.data(), total + 100), "short read reported");
    }
    {  // an abandoned writer removes its file
        homs::FileWriter w;
        std::string err;
        check(w.open(path, &err), "open for writing");
        check(w.write(data.data(), 10), "write");
        w.abandon();
        FILE* f = std::fopen(path, "rb");
        check(f == nullptr, "abandoned file removed");
        if (f) std::fclose(f);
    }
    std::remove(path);
    homs::Checksum a, b;
    a.update(data.data(), 1000);
    b.update(data.data(), 3);
    b.update(data.data() + 3, 997);
    check(a.value() == b.value(), "checksum independent of chunking");
}

}  // namespace

int main()
{
    run_preprocess();
    run_codebook();
    run_files();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host sanitizer run: all checks passed\n");
    return 0;
}
