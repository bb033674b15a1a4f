// Host generation of the position (ID) and level hypervector tables
// (Sections 3.3.1 and 3.3.2) from a SplitMix64 stream.
//
// Position vectors: a random base F_0 and a random order of the D
// components; F_i flips the first k_i = floor(alpha * i / (f - 1)) entries of
// that order, so neighbouring bins share almost every component (spatial
// locality) and F_0, F_{f-1} differ in exactly alpha components. Level
// vectors: the same construction with m_j = floor((D / 2) * j / (Q - 1)),
// so the lowest and highest levels differ in D/2 components (value
// locality). Rows are built incrementally: row i is row i - 1 with the order
// entries k_{i-1} .. k_i - 1 flipped.
#include "codebook.h"

#include <cstring>
#include <vector>

namespace homs {
namespace {

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014)
struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

void base_row(SplitMix64& g, uint32_t D, uint32_t* row)
{
    for (uint32_t k = 0; k < D / 64; ++k) {
        const uint64_t r = g.next();
        row[2 * k] = (uint32_t)r;
        row[2 * k + 1] = (uint32_t)(r >> 32);
    }
}

std::vector<uint32_t> flip_order(SplitMix64& g, uint32_t D)
{
    std::vector<uint32_t> order(D);
    for (uint32_t i = 0; i < D; ++i) order[i] = i;
    for (uint32_t i = D - 1; i > 0; --i) {
        const uint32_t j = (uint32_t)(g.next() % (uint64_t)(i + 1));
        const uint32_t t = order[i];
        order[i] = order[j];
        order[j] = t;
    }
    return order;
}

void fill_table(uint32_t D, uint32_t rows, uint64_t total_flips, const uint32_t* base,
                const std::vector<uint32_t>& order, uint32_t* out)
{
    const uint32_t W = D / 32;
    std::memcpy(out, base, (size_t)W * sizeof(uint32_t));
    uint64_t done = 0;
    for (uint32_t i = 1; i < rows; ++i) {
        uint32_t* row = out + (size_t)i * W;
        std::memcpy(row, row - W, (size_t)W * sizeof(uint32_t));
        const uint64_t want = (total_flips * i) / (uint64_t)(rows - 1);
        for (; done < want; ++done) {
            const uint32_t d = order[done];
            row[d >> 5] ^= 1u << (d & 31u);
        }
    }
}

}  // namespace

void generate_codebook(uint32_t D, uint32_t f, uint32_t Q, uint32_t alpha, uint64_t seed,
                       uint32_t encoding, uint32_t* id_table, uint32_t* level_table)
{
    SplitMix64 g{seed};
    std::vector<uint32_t> base(D / 32);
    base_row(g, D, base.data());
    std::vector<uint32_t> order = flip_order(g, D);
    fill_table(D, f, alpha, base.data(), order, id_table);
    base_row(g, D, base.data());
    order = flip_order(g, D);
    fill_table(D, Q, D / 2, base.data(), order, level_table);
    // the baselines of Section 4.2: independent random position vectors,
    // drawn row after row after the level table's draws
    if (encoding != 0)
        for (uint32_t i = 0; i < f; ++i) base_row(g, D, id_table + (size_t)i * (D / 32));
}

}  // namespace homs
