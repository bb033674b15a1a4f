// Buffered file writing and reading with a running checksum for the library
// and model files.
#include "persist.h"

#include <cstring>

namespace homs {

namespace {
constexpr uint64_t kPrime = 0x100000001b3ull;

inline uint64_t load_le64(const uint8_t* b)
{
    uint64_t w = 0;
    for (int i = 7; i >= 0; --i) w = (w << 8) | b[i];
    return w;
}
}  // namespace

void Checksum::update(const void* p, size_t n)
{
    const uint8_t* b = (const uint8_t*)p;
    while (n > 0 && ntail_ > 0) {  // complete a pending word
        tail_[ntail_++] = *b++;
        --n;
        if (ntail_ == 8) {
            h_ = (h_ ^ load_le64(tail_)) * kPrime;
            ntail_ = 0;
        }
    }
    for (; n >= 8; n -= 8, b += 8) h_ = (h_ ^ load_le64(b)) * kPrime;
    for (; n > 0; --n) tail_[ntail_++] = *b++;
}

uint64_t Checksum::value() const
{
    if (ntail_ == 0) return h_;
    uint8_t w[8] = {0};
    std::memcpy(w, tail_, ntail_);
    return (h_ ^ load_le64(w)) * kPrime;
}

FileWriter::~FileWriter() { abandon(); }

bool FileWriter::open(const std::string& path, std::string* err)
{
    path_ = path;
    f_ = fopen(path.c_str(), "wb");
    if (!f_) {
        *err = "cannot open " + path + " for writing";
        return false;
    }
    return true;
}

bool FileWriter::write(const void* p, size_t n)
{
    if (!ok_ || !f_) return false;
    sum_.update(p, n);
    ok_ = fwrite(p, 1, n, f_) == n;
    return ok_;
}

bool FileWriter::finish(std::string* err)
{
    if (!f_) return false;
    uint64_t v = sum_.value();
    uint8_t b[8];
    for (int i = 0; i < 8; ++i) b[i] = (uint8_t)(v >> (8 * i));
    ok_ = ok_ && fwrite(b, 1, 8, f_) == 8;
    ok_ = (fclose(f_) == 0) && ok_;
    f_ = nullptr;
    if (!ok_) {
        *err = "write to " + path_ + " failed";
        std::remove(path_.c_str());
    }
    return ok_;
}

void FileWriter::abandon()
{
    if (f_) {
        fclose(f_);
        f_ = nullptr;
        std::remove(path_.c_str());
    }
}

FileReader::~FileReader()
{
    if (f_) fclose(f_);
}

bool FileReader::open(const std::string& path, std::string* err)
{
    f_ = fopen(path.c_str(), "rb");
    if (!f_) {
        *err = "cannot open " + path;
        return false;
    }
    if (fseek(f_, 0, SEEK_END) == 0) size_ = (int64_t)ftell(f_);
    fseek(f_, 0, SEEK_SET);
    return true;
}

bool FileReader::read(void* p, size_t n)
{
    if (!f_ || fread(p, 1, n, f_) != n) return false;
    sum_.update(p, n);
    return true;
}

bool FileReader::finish(std::string* err)
{
    uint8_t b[8];
    if (!f_ || fread(b, 1, 8, f_) != 8) {
        *err = "file is truncated";
        return false;
    }
    uint64_t stored = 0;
    for (int i = 7; i >= 0; --i) stored = (stored << 8) | b[i];
    if (stored != sum_.value()) {
        *err = "checksum mismatch (the file is damaged)";
        return false;
    }
    if (fgetc(f_) != EOF) {
        *err = "unexpected bytes after the checksum";
        return false;
    }
    return true;
}

}  // namespace homs
