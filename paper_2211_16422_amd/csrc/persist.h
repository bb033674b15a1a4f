// Host side of the library and model files (homs_library_save/load,
// homs_model_save/load, homs_file_info): buffered writing and reading with
// a running 64-bit checksum. Not part of the C ABI.
#pragma once

#include <stdint.h>
#include <stdio.h>

#include <string>

namespace homs {

// FNV-1a over little-endian 64-bit words: h = (h ^ w) * 0x100000001b3 from
// h = 0xcbf29ce484222325, the last word zero-padded.
class Checksum {
public:
    void update(const void* p, size_t n);
    uint64_t value() const;  // of every byte given so far

private:
    uint64_t h_ = 0xcbf29ce484222325ull;
    uint8_t tail_[8] = {0};
    size_t ntail_ = 0;
};

class FileWriter {
public:
    ~FileWriter();
    bool open(const std::string& path, std::string* err);
    bool write(const void* p, size_t n);  // adds to the checksum
    bool finish(std::string* err);        // appends the checksum, closes
    void abandon();                       // closes and removes the file

private:
    FILE* f_ = nullptr;
    std::string path_;
    Checksum sum_;
    bool ok_ = true;
};

class FileReader {
public:
    ~FileReader();
    bool open(const std::string& path, std::string* err);
    bool read(void* p, size_t n);  // false on a short read; adds to the checksum
    // reads the stored checksum, compares it with the running one and
    // checks that nothing follows it
    bool finish(std::string* err);
    int64_t size() const { return size_; }

private:
    FILE* f_ = nullptr;
    Checksum sum_;
    int64_t size_ = 0;
};

constexpr char kLibraryMagic[8] = {'H', 'O', 'M', 'S', 'L', 'I', 'B', '1'};
constexpr char kModelMagic[8] = {'H', 'O', 'M', 'S', 'M', 'D', 'L', '1'};
constexpr uint32_t kFileVersion = 1;

// fixed-size header of a library file (little-endian, no padding)
#pragma pack(push, 1)
struct LibraryHeader {
    char magic[8];
    uint32_t version, dim, n_levels, top_n, id_flips, charge_match, encoding, reserved;
    double mz_min, mz_max, bins_per_da, noise_frac;
    uint64_t seed, codebook_hash;
    int64_t n;
};
struct ModelHeader {
    char magic[8];
    uint32_t version, dim;
    int32_t hidden, embed;
    int64_t step;
};
#pragma pack(pop)
static_assert(sizeof(LibraryHeader) == 96, "library header layout");
static_assert(sizeof(ModelHeader) == 32, "model header layout");

}  // namespace homs
