// Host-side generation of the position and level hypervector tables.
#pragma once
#include <stdint.h>

namespace homs {

// id_table: f rows of D/32 words; level_table: Q rows of D/32 words.
// Requires D % 64 == 0, f >= 1, Q >= 2, alpha <= D.
// encoding: HOMS_ENCODING_* (random position rows unless ID_LEVEL)
void generate_codebook(uint32_t D, uint32_t f, uint32_t Q, uint32_t alpha, uint64_t seed,
                       uint32_t encoding, uint32_t* id_table, uint32_t* level_table);

}  // namespace homs
