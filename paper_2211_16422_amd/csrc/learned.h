// Internal declarations of the learned shortlist (model state, training and
// embedding steps, shortlist search). Not part of the C ABI.
#pragma once

#include <string>

#include "internal.h"

struct homs_model {
    homs_ctx* ctx = nullptr;
    int D = 0, H = 0, E = 0;
    // fp32 masters, Adam moments, bf16 copies (W2 also transposed), gradients
    float *W1 = nullptr, *b1 = nullptr, *W2 = nullptr, *b2 = nullptr;
    float *mW1 = nullptr, *vW1 = nullptr, *mb1 = nullptr, *vb1 = nullptr;
    float *mW2 = nullptr, *vW2 = nullptr, *mb2 = nullptr, *vb2 = nullptr;
    uint16_t *W1h = nullptr, *W2h = nullptr, *W2Th = nullptr;
    float *gW1 = nullptr, *gb1 = nullptr, *gW2 = nullptr, *gb2 = nullptr;
    int64_t step = 0;
    uint64_t weights_gen = 0;  // bumped by every weight change
    float* loss_scratch = nullptr;  // device float for losses nobody asked for
    void* train_ws = nullptr;
    size_t train_ws_bytes = 0;
    void* emb_ws = nullptr;
    size_t emb_ws_bytes = 0;
    // scoring embeddings of the context's library in sorted order: E4M3 codes
    // of 16 e [n][E] (the scoring kernel's operands) and the same values / 16
    // in bf16 [n][E] (the threshold samples' operands)
    uint8_t* lib_emb8 = nullptr;
    uint16_t* lib_emb = nullptr;
    int64_t lib_emb_n = 0;
    uint64_t lib_emb_lib_gen = 0;  // ctx->lib_gen and weights_gen the embeddings
    uint64_t lib_emb_w_gen = 0;    // were made from (stale when either moved on)
    bool lib_emb_valid = false;
};

namespace homs {

constexpr int64_t kEmbedBatch = 16384;  // rows expanded to bf16 per embedding pass

// Scoring embeddings: the E4M3 format of the OCP 8-bit floating point
// specification (v1.0, 2023): sign, 4 exponent bits with bias 7, 3 fraction
// bits; subnormals m 2^-9; largest finite value 448. A unit embedding is
// scaled by kScoreScale first, so its components lie in the normal range;
// scores of two scaled rows are kScoreScale^2 times the scores of the
// rounded embeddings.
constexpr float kScoreScale = 16.f;

// nearest E4M3 code, ties to even; magnitudes beyond 448 saturate
__device__ __forceinline__ uint32_t to_e4m3(float x)
{
    const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
    const float a = fminf(fabsf(x), 448.f);
    uint32_t code;
    if (a < 0.015625f) {  // below 2^-6: multiples of 2^-9 (8 is 2^-6 itself)
        code = (uint32_t)rintf(a * 512.f);
    } else {  // keep 3 fraction bits, ties to even; a carry moves into the exponent
        uint32_t u = __float_as_uint(a);
        u += 0x7FFFFu + ((u >> 20) & 1u);
        code = (((u >> 23) - 120u) << 3) | ((u >> 20) & 7u);  // exponent bias 127 -> 7
    }
    return sign | code;
}

__device__ __forceinline__ float from_e4m3(uint32_t c)
{
    const uint32_t e = (c >> 3) & 15u, m = c & 7u;
    const float mag = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * (1.f / 512.f);
    return (c & 0x80u) ? -mag : mag;
}

void model_free(homs_model* m);
hipError_t model_alloc(homs_model* m);
hipError_t model_refresh_bf16(homs_model* m, hipStream_t s);
// Embeddings of n packed rows: fp32 unit embeddings (out_f32), and/or the
// scoring embeddings (out_fp8: E4M3 codes of kScoreScale e; out_bf16: those
// values / kScoreScale). Without out_fp8, out_bf16 holds bf16(e).
hipError_t model_embed(homs_model* m, int64_t n, const uint32_t* hv, float* out_f32,
                       uint16_t* out_bf16, uint8_t* out_fp8, hipStream_t s);
// Rows of a training batch taken through device index arrays: at `step`, row
// r of the batch is query q_rows[perm[step] * B + r] and reference (sorted
// library row) r_rows[perm[step] * B + r].
struct RowSelect {
    const uint32_t* q_rows;
    const uint32_t* r_rows;
    const uint32_t* perm;
    int64_t step;
};
// One training step on B pairs: rows [0, B) of q_hv and r_hv, or, with sel,
// the rows sel picks out of q_hv and r_hv.
hipError_t model_step(homs_model* m, int B, const uint32_t* q_hv, const uint32_t* r_hv, float tau,
                      float lr, bool update, float* loss, hipStream_t s,
                      const RowSelect* sel = nullptr);
// The training schedule of homs_model_train (pairs ordered by their
// reference's sorted library row, batches of B, each epoch's batch order
// from the SplitMix64 stream of `seed`); synchronous.
hipError_t model_train(homs_model* m, int64_t n, const uint32_t* q_hv, const int64_t* target,
                       int epochs, int B, float lr, float tau, uint64_t seed, float* losses,
                       int64_t* steps_out, hipStream_t s);

// learned_search.hip: shortlist of k per query, exact rescoring; sets
// fallback[q] = 1 where the shortlist could not be formed (the caller then
// runs the exhaustive search for those queries)
// Optional timing of the scoring kernel: mark() records an event on the
// stream (or returns nullptr), span() files an interval between two marks.
struct SpanHook {
    void* user = nullptr;
    hipEvent_t (*mark)(void* user, hipStream_t s) = nullptr;
    void (*span)(void* user, hipEvent_t a, hipEvent_t b) = nullptr;
};

struct LearnedScratchPlan {
    int64_t batch;  // queries per collection pass
};
int learned_max_k();
bool learned_search_supports(int embed);  // embedding sizes the search kernels take
size_t learned_scratch_bytes(int64_t nq, int64_t E, LearnedScratchPlan* plan);
hipError_t launch_search_learned(const homs_ctx* c, const homs_model* m, void* scratch,
                                 const LearnedScratchPlan& plan, int64_t nq,
                                 const uint32_t* q_hv, const uint16_t* q_emb,
                                 const uint8_t* q_emb8,
                                 const uint32_t* qperm, const int64_t* lo, const int64_t* hi,
                                 int k, uint64_t* keys, uint8_t* fallback, int64_t* shortlist,
                                 const SpanHook& hook, hipStream_t s);
// exhaustive search of the windows of the queries with fallback[q] set,
// merged into keys (scratch: fallback_scratch_bytes)
size_t fallback_scratch_bytes(int64_t nq);
hipError_t launch_fallback_scan(const homs_ctx* c, int64_t nq, const uint32_t* q_hv,
                                const uint8_t* fallback, const int64_t* lo, const int64_t* hi,
                                void* scratch, uint64_t* keys, hipStream_t s);
size_t embed_ws_bytes(const homs_model* m, int64_t rows);
size_t train_ws_bytes(const homs_model* m, int B);

}  // namespace homs
