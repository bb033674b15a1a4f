// Learned shortlist: a small MLP embeds hypervectors into unit vectors,
// trained on the GPU on (query, exact top-1) pairs produced by the search
// itself; at query time it proposes the k best-scoring candidates of each
// window, which are rescored exactly by Hamming distance. Queries whose
// shortlist cannot be formed reliably fall back to the exhaustive search.
//
// Network: x (bipolar hypervector, D) -> a1 = W1 x + b1 -> h = ReLU(a1) (H)
// -> z = W2 h + b2 (E) -> e = z / sqrt(z.z + eps). Weights are fp32 masters
// with bf16 copies for the matrix-core GEMMs (fp32 accumulation). Loss:
// InfoNCE over a batch of B pairs with in-batch negatives, temperature tau.
// Optimizer: Adam (beta1 0.9, beta2 0.999, eps 1e-8).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gemm_bf16.h"
#include "learned.h"

namespace homs {
namespace {

using gemm::to_bf16;
constexpr int kThreads = 256;
constexpr float kEpsNorm = 1e-12f;

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + kThreads - 1) / kThreads); }

// packed rows [n][D/32] -> bipolar bf16 rows [n][ld] (+1 = 0x3F80, -1 = 0xBF80)
__global__ void expand_bits_kernel(int64_t n, uint32_t words, const uint32_t* __restrict__ hv,
                                   uint16_t* __restrict__ X, int64_t ld)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * (int64_t)words) return;
    const int64_t r = t / words;
    const uint32_t w = (uint32_t)(t - r * words);
    const uint32_t v = hv[r * words + w];
    uint16_t* o = X + r * ld + (int64_t)w * 32;
#pragma unroll
    for (int b = 0; b < 32; b += 2) {
        const uint32_t lo = ((v >> b) & 1u) ? 0xBF80u : 0x3F80u;
        const uint32_t hi = ((v >> (b + 1)) & 1u) ? 0xBF80u : 0x3F80u;
        *(uint32_t*)(o + b) = lo | (hi << 16);
    }
}

// the same expansion for the rows of one training batch taken through index
// arrays: row r of the batch is hv[rows[perm[step] * n + r]]
__global__ void expand_rows_kernel(int64_t n, uint32_t words, const uint32_t* __restrict__ hv,
                                   const uint32_t* __restrict__ rows,
                                   const uint32_t* __restrict__ perm, int64_t step,
                                   uint16_t* __restrict__ X, int64_t ld)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * (int64_t)words) return;
    const int64_t r = t / words;
    const uint32_t w = (uint32_t)(t - r * words);
    const int64_t src = (int64_t)rows[(int64_t)perm[step] * n + r];
    const uint32_t v = hv[src * words + w];
    uint16_t* o = X + r * ld + (int64_t)w * 32;
#pragma unroll
    for (int b = 0; b < 32; b += 2) {
        const uint32_t lo = ((v >> b) & 1u) ? 0xBF80u : 0x3F80u;
        const uint32_t hi = ((v >> (b + 1)) & 1u) ? 0xBF80u : 0x3F80u;
        *(uint32_t*)(o + b) = lo | (hi << 16);
    }
}

// bf16 [R][C] (ld_in) -> bf16 [C][R] (ld_out), 32 x 32 tiles through LDS
__global__ void transpose_bf16_kernel(int R, int C, const uint16_t* __restrict__ in, int ld_in,
                                      uint16_t* __restrict__ out, int ld_out)
{
    __shared__ uint16_t tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < R && c < C) ? in[(size_t)r * ld_in + c] : (uint16_t)0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int c = c0 + i, r = r0 + tx;
        if (c < C && r < R) out[(size_t)c * ld_out + r] = tile[tx][i];
    }
}

// unit embedding rows: e = z / sqrt(z.z + eps); one wave per row. With eb8,
// the scoring embeddings: eb8 = E4M3 code of kScoreScale e and eb = that
// value / kScoreScale (exact in bf16); otherwise eb = bf16(e).
__global__ void normalize_kernel(int64_t M, int E, const float* __restrict__ z,
                                 float* __restrict__ e, uint16_t* __restrict__ eb,
                                 float* __restrict__ s, float* __restrict__ out_f32,
                                 uint8_t* __restrict__ eb8 = nullptr)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (row >= M) return;
    const float* zr = z + row * E;
    float ss = 0.f;
    for (int j = l; j < E; j += 64) ss += zr[j] * zr[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    const float sc = sqrtf(ss + kEpsNorm);
    for (int j = l; j < E; j += 64) {
        const float v = zr[j] / sc;
        if (e) e[row * E + j] = v;
        if (eb8) {
            const uint32_t c = to_e4m3(v * kScoreScale);
            eb8[row * E + j] = (uint8_t)c;
            if (eb) eb[row * E + j] = to_bf16(from_e4m3(c) * (1.f / kScoreScale));
        } else if (eb) {
            eb[row * E + j] = to_bf16(v);
        }
        if (out_f32) out_f32[row * E + j] = v;
    }
    if (s && l == 0) s[row] = sc;
}

// InfoNCE over logits S [B][B] (already divided by tau): per row softmax,
// loss += (logsumexp - S_ii) / B, dS = (P - I) / B stored as bf16 and its
// transpose. One workgroup per row.
__global__ void info_nce_kernel(int B, const float* __restrict__ S, uint16_t* __restrict__ dS,
                                uint16_t* __restrict__ dST, float* __restrict__ loss)
{
    __shared__ float red[kThreads / 64];
    const int i = blockIdx.x;
    const float* row = S + (size_t)i * B;
    float mx = -INFINITY;
    for (int j = threadIdx.x; j < B; j += kThreads) mx = fmaxf(mx, row[j]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    float sum = 0.f;
    for (int j = threadIdx.x; j < B; j += kThreads) sum += __expf(row[j] - mx);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    sum = red[0] + red[1] + red[2] + red[3];
    for (int j = threadIdx.x; j < B; j += kThreads) {
        const float p = __expf(row[j] - mx) / sum;
        const float g = (p - (j == i ? 1.f : 0.f)) / (float)B;
        dS[(size_t)i * B + j] = to_bf16(g);
        dST[(size_t)j * B + i] = to_bf16(g);
    }
    if (threadIdx.x == 0) atomicAdd(loss, (logf(sum) + mx - row[i]) / (float)B);
}

// dz = (dE - e (e.dE)) / s, one wave per row; fp32 and bf16 copies
__global__ void normalize_backward_kernel(int64_t M, int E, const float* __restrict__ e,
                                          const float* __restrict__ s,
                                          const float* __restrict__ dE, float* __restrict__ dz,
                                          uint16_t* __restrict__ dzb)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (row >= M) return;
    float dot = 0.f;
    for (int j = l; j < E; j += 64) dot += e[row * E + j] * dE[row * E + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off);
    const float sc = s[row];
    for (int j = l; j < E; j += 64) {
        const float v = (dE[row * E + j] - e[row * E + j] * dot) / sc;
        dz[row * E + j] = v;
        dzb[row * E + j] = to_bf16(v);
    }
}

// column sums of a [M][N] fp32 matrix in two deterministic passes: partial
// sums of kColRows-row slabs (grid.y = slab), then the slabs in order
constexpr int kColRows = 128;

__global__ void colsum_partial_kernel(int M, int N, const float* __restrict__ a,
                                      float* __restrict__ part)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int m0 = blockIdx.y * kColRows, m1 = min(m0 + kColRows, M);
    float acc = 0.f;
    for (int m = m0; m < m1; ++m) acc += a[(size_t)m * N + n];
    part[(size_t)blockIdx.y * N + n] = acc;
}

__global__ void colsum_final_kernel(int P, int N, const float* __restrict__ part,
                                    float* __restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float acc = 0.f;
    for (int p = 0; p < P; ++p) acc += part[(size_t)p * N + n];
    out[n] = acc;
}

inline void colsum(int M, int N, const float* a, float* part, float* out, hipStream_t s)
{
    const int P = (M + kColRows - 1) / kColRows;
    colsum_partial_kernel<<<dim3((unsigned)((N + 255) / 256), (unsigned)P), 256, 0, s>>>(M, N, a,
                                                                                         part);
    colsum_final_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(P, N, part, out);
}

__global__ void adam_kernel(int64_t n, float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float c1,
                            float c2, uint16_t* __restrict__ wb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    w[i] = wi;
    if (wb) wb[i] = to_bf16(wi);
}

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ a, uint16_t* __restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = to_bf16(a[i]);
}

__global__ void fill_f32_kernel(int64_t n, float* __restrict__ p, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ---------------------------------------------------------------------------
// model lifetime and weights

void model_free(homs_model* m)
{
    for (void* p : {(void*)m->W1, (void*)m->b1, (void*)m->W2, (void*)m->b2, (void*)m->mW1,
                    (void*)m->vW1, (void*)m->mb1, (void*)m->vb1, (void*)m->mW2, (void*)m->vW2,
                    (void*)m->mb2, (void*)m->vb2, (void*)m->W1h, (void*)m->W2h, (void*)m->W2Th,
                    (void*)m->gW1, (void*)m->gb1, (void*)m->gW2, (void*)m->gb2, m->train_ws,
                    m->emb_ws, (void*)m->lib_emb, (void*)m->lib_emb8, (void*)m->loss_scratch})
        if (p) (void)hipFree(p);
}

hipError_t model_alloc(homs_model* m)
{
    const size_t n1 = (size_t)m->H * m->D, n2 = (size_t)m->E * m->H;
    hipError_t e = hipSuccess;
    auto A = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = dev_malloc(p, bytes);
        if (e == hipSuccess) e = hipMemset(*p, 0, bytes);
    };
    A((void**)&m->W1, n1 * 4);
    A((void**)&m->b1, m->H * 4);
    A((void**)&m->W2, n2 * 4);
    A((void**)&m->b2, m->E * 4);
    A((void**)&m->mW1, n1 * 4);
    A((void**)&m->vW1, n1 * 4);
    A((void**)&m->mb1, m->H * 4);
    A((void**)&m->vb1, m->H * 4);
    A((void**)&m->mW2, n2 * 4);
    A((void**)&m->vW2, n2 * 4);
    A((void**)&m->mb2, m->E * 4);
    A((void**)&m->vb2, m->E * 4);
    A((void**)&m->W1h, n1 * 2);
    A((void**)&m->W2h, n2 * 2);
    A((void**)&m->W2Th, n2 * 2);
    A((void**)&m->gW1, n1 * 4);
    A((void**)&m->gb1, m->H * 4);
    A((void**)&m->gW2, n2 * 4);
    A((void**)&m->gb2, m->E * 4);
    A((void**)&m->loss_scratch, 256);
    return e;
}

// bf16 copies of the weights (and W2 transposed) from the fp32 masters
hipError_t model_refresh_bf16(homs_model* m, hipStream_t s)
{
    const int64_t n1 = (int64_t)m->H * m->D, n2 = (int64_t)m->E * m->H;
    to_bf16_kernel<<<blocks_for(n1), kThreads, 0, s>>>(n1, m->W1, m->W1h);
    to_bf16_kernel<<<blocks_for(n2), kThreads, 0, s>>>(n2, m->W2, m->W2h);
    transpose_bf16_kernel<<<dim3((m->H + 31) / 32, (m->E + 31) / 32), 256, 0, s>>>(
        m->E, m->H, m->W2h, m->H, m->W2Th, m->E);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// embedding inference: n packed rows -> unit embeddings (fp32 and/or bf16)

size_t embed_ws_bytes(const homs_model* m, int64_t rows)
{
    return al(rows * m->D * 2) + al(rows * m->H * 2) + 2 * al(rows * m->E * 4) + al(rows * 4);
}

hipError_t model_embed(homs_model* m, int64_t n, const uint32_t* hv, float* out_f32,
                       uint16_t* out_bf16, uint8_t* out_fp8, hipStream_t s)
{
    const int64_t rows = std::min<int64_t>(n, kEmbedBatch);
    if (n <= 0) return hipSuccess;
    const size_t need = embed_ws_bytes(m, rows);
    if (m->emb_ws_bytes < need) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (m->emb_ws) (void)hipFree(m->emb_ws);
        m->emb_ws = nullptr;
        m->emb_ws_bytes = 0;
        e = dev_malloc(&m->emb_ws, need);
        if (e != hipSuccess) return e;
        m->emb_ws_bytes = need;
    }
    char* p = (char*)m->emb_ws;
    uint16_t* X = (uint16_t*)p;
    p += al(rows * m->D * 2);
    uint16_t* hb = (uint16_t*)p;
    p += al(rows * m->H * 2);
    float* a1 = (float*)p;  // also reused for z
    p += al(rows * m->E * 4);
    (void)p;
    const uint32_t words = (uint32_t)(m->D / 32);
    for (int64_t r0 = 0; r0 < n; r0 += rows) {
        const int64_t nr = std::min(rows, n - r0);
        expand_bits_kernel<<<blocks_for(nr * words), kThreads, 0, s>>>(nr, words,
                                                                        hv + r0 * words, X, m->D);
        hipError_t e = gemm::gemm_nt<gemm::kBias | gemm::kStoreBf16 | gemm::kReluBf16>(
            s, (int)nr, m->H, m->D, X, m->D, m->W1h, m->D, 1.f, m->b1, nullptr, nullptr, m->H, hb,
            m->H);
        if (e != hipSuccess) return e;
        e = gemm::gemm_nt<gemm::kBias | gemm::kStoreF32>(s, (int)nr, m->E, m->H, hb, m->H, m->W2h,
                                                         m->H, 1.f, m->b2, nullptr, a1, m->E,
                                                         nullptr, 0);
        if (e != hipSuccess) return e;
        normalize_kernel<<<(uint32_t)((nr + 3) / 4), 256, 0, s>>>(
            nr, m->E, a1, nullptr, out_bf16 ? out_bf16 + r0 * m->E : nullptr, nullptr,
            out_f32 ? out_f32 + r0 * m->E : nullptr, out_fp8 ? out_fp8 + r0 * m->E : nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// one training step (forward, loss, backward; Adam when `update`)

size_t train_ws_bytes(const homs_model* m, int B)
{
    const size_t M2 = 2 * (size_t)B, D = m->D, H = m->H, E = m->E;
    return 2 * al(M2 * D * 2) + al(M2 * H * 4) + 2 * al(M2 * H * 2) + 3 * al(M2 * E * 4) +
           al(M2 * E * 2) + al(M2 * 4) + al(E * M2 * 2) + al((size_t)B * B * 4) +
           2 * al((size_t)B * B * 2) + al(M2 * E * 4) + al(M2 * E * 2) + al(E * M2 * 2) +
           al(M2 * H * 4) + al(M2 * H * 2) + al(H * M2 * 2) +
           al(((M2 + kColRows - 1) / kColRows) * std::max(H, E) * 4);
}

hipError_t model_step(homs_model* m, int B, const uint32_t* q_hv, const uint32_t* r_hv, float tau,
                      float lr, bool update, float* loss, hipStream_t s, const RowSelect* sel)
{
    const int M2 = 2 * B, D = m->D, H = m->H, E = m->E;
    const uint32_t words = (uint32_t)(D / 32);
    const size_t need = train_ws_bytes(m, B);
    if (m->train_ws_bytes < need) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (m->train_ws) (void)hipFree(m->train_ws);
        m->train_ws = nullptr;
        m->train_ws_bytes = 0;
        e = dev_malloc(&m->train_ws, need);
        if (e != hipSuccess) return e;
        m->train_ws_bytes = need;
    }
    char* p = (char*)m->train_ws;
    auto take = [&](size_t bytes) {
        void* r = p;
        p += al(bytes);
        return r;
    };
    uint16_t* X = (uint16_t*)take((size_t)M2 * D * 2);
    uint16_t* XT = (uint16_t*)take((size_t)M2 * D * 2);
    float* a1 = (float*)take((size_t)M2 * H * 4);
    uint16_t* hb = (uint16_t*)take((size_t)M2 * H * 2);
    uint16_t* hT = (uint16_t*)take((size_t)M2 * H * 2);
    float* z = (float*)take((size_t)M2 * E * 4);
    float* e = (float*)take((size_t)M2 * E * 4);
    float* dz = (float*)take((size_t)M2 * E * 4);
    uint16_t* eb = (uint16_t*)take((size_t)M2 * E * 2);
    float* sc = (float*)take((size_t)M2 * 4);
    uint16_t* eT = (uint16_t*)take((size_t)E * M2 * 2);
    float* S = (float*)take((size_t)B * B * 4);
    uint16_t* dS = (uint16_t*)take((size_t)B * B * 2);
    uint16_t* dST = (uint16_t*)take((size_t)B * B * 2);
    float* dE = (float*)take((size_t)M2 * E * 4);
    uint16_t* dzb = (uint16_t*)take((size_t)M2 * E * 2);
    uint16_t* dzT = (uint16_t*)take((size_t)E * M2 * 2);
    float* da1 = (float*)take((size_t)M2 * H * 4);
    uint16_t* da1b = (uint16_t*)take((size_t)M2 * H * 2);
    uint16_t* da1T = (uint16_t*)take((size_t)H * M2 * 2);
    float* colpart = (float*)take((size_t)((M2 + kColRows - 1) / kColRows) * std::max(H, E) * 4);

    using namespace gemm;
    hipError_t err = hipSuccess;
#define STEP(x)                              \
    do {                                     \
        err = (x);                           \
        if (err != hipSuccess) return err;   \
    } while (0)
    // forward, both towers stacked: rows [0, B) queries, [B, 2B) references
    if (sel) {
        expand_rows_kernel<<<blocks_for((int64_t)B * words), kThreads, 0, s>>>(
            B, words, q_hv, sel->q_rows, sel->perm, sel->step, X, D);
        expand_rows_kernel<<<blocks_for((int64_t)B * words), kThreads, 0, s>>>(
            B, words, r_hv, sel->r_rows, sel->perm, sel->step, X + (size_t)B * D, D);
    } else {
        expand_bits_kernel<<<blocks_for((int64_t)B * words), kThreads, 0, s>>>(B, words, q_hv, X,
                                                                                D);
        expand_bits_kernel<<<blocks_for((int64_t)B * words), kThreads, 0, s>>>(
            B, words, r_hv, X + (size_t)B * D, D);
    }
    STEP(gemm_nt<kBias | kStoreF32 | kStoreBf16 | kReluBf16>(s, M2, H, D, X, D, m->W1h, D, 1.f,
                                                             m->b1, nullptr, a1, H, hb, H));
    STEP(gemm_nt<kBias | kStoreF32>(s, M2, E, H, hb, H, m->W2h, H, 1.f, m->b2, nullptr, z, E,
                                    nullptr, 0));
    normalize_kernel<<<(uint32_t)((M2 + 3) / 4), 256, 0, s>>>(M2, E, z, e, eb, sc, nullptr);
    // logits and loss
    STEP(gemm_nt<kStoreF32>(s, B, B, E, eb, E, eb + (size_t)B * E, E, 1.f / tau, nullptr, nullptr,
                            S, B, nullptr, 0));
    fill_f32_kernel<<<1, 64, 0, s>>>(1, loss, 0.f);
    info_nce_kernel<<<B, kThreads, 0, s>>>(B, S, dS, dST, loss);
    // dE_q = dS E_r / tau, dE_r = dS^T E_q / tau (B operands are E^T slices)
    transpose_bf16_kernel<<<dim3((E + 31) / 32, (M2 + 31) / 32), 256, 0, s>>>(M2, E, eb, E, eT,
                                                                                M2);
    STEP(gemm_nt<kStoreF32>(s, B, E, B, dS, B, eT + B, M2, 1.f / tau, nullptr, nullptr, dE, E,
                            nullptr, 0));
    STEP(gemm_nt<kStoreF32>(s, B, E, B, dST, B, eT, M2, 1.f / tau, nullptr, nullptr,
                            dE + (size_t)B * E, E, nullptr, 0));
    normalize_backward_kernel<<<(uint32_t)((M2 + 3) / 4), 256, 0, s>>>(M2, E, e, sc, dE, dz, dzb);
    colsum(M2, E, dz, colpart, m->gb2, s);
    transpose_bf16_kernel<<<dim3((E + 31) / 32, (M2 + 31) / 32), 256, 0, s>>>(M2, E, dzb, E, dzT,
                                                                                M2);
    transpose_bf16_kernel<<<dim3((H + 31) / 32, (M2 + 31) / 32), 256, 0, s>>>(M2, H, hb, H, hT,
                                                                                M2);
    // dW2 = dz^T h
    STEP(gemm_nt<kStoreF32>(s, E, H, M2, dzT, M2, hT, M2, 1.f, nullptr, nullptr, m->gW2, H,
                            nullptr, 0));
    // da1 = (dz W2) * [a1 > 0]
    STEP(gemm_nt<kMask | kStoreF32 | kStoreBf16>(s, M2, H, E, dzb, E, m->W2Th, E, 1.f, nullptr,
                                                 a1, da1, H, da1b, H));
    colsum(M2, H, da1, colpart, m->gb1, s);
    transpose_bf16_kernel<<<dim3((H + 31) / 32, (M2 + 31) / 32), 256, 0, s>>>(M2, H, da1b, H,
                                                                                da1T, M2);
    // dW1 = da1^T X
    transpose_bf16_kernel<<<dim3((D + 31) / 32, (M2 + 31) / 32), 256, 0, s>>>(M2, D, X, D, XT,
                                                                                M2);
    STEP(gemm_nt<kStoreF32>(s, H, D, M2, da1T, M2, XT, M2, 1.f, nullptr, nullptr, m->gW1, D,
                            nullptr, 0));
    STEP(hipGetLastError());
    if (!update) return hipSuccess;
    m->step += 1;
    const float c1 = 1.f - powf(0.9f, (float)m->step), c2 = 1.f - powf(0.999f, (float)m->step);
    const int64_t n1 = (int64_t)H * D, n2 = (int64_t)E * H;
    adam_kernel<<<blocks_for(n1), kThreads, 0, s>>>(n1, m->W1, m->gW1, m->mW1, m->vW1, lr, c1, c2,
                                                    m->W1h);
    adam_kernel<<<blocks_for(H), kThreads, 0, s>>>(H, m->b1, m->gb1, m->mb1, m->vb1, lr, c1, c2,
                                                   nullptr);
    adam_kernel<<<blocks_for(n2), kThreads, 0, s>>>(n2, m->W2, m->gW2, m->mW2, m->vW2, lr, c1, c2,
                                                    m->W2h);
    adam_kernel<<<blocks_for(E), kThreads, 0, s>>>(E, m->b2, m->gb2, m->mb2, m->vb2, lr, c1, c2,
                                                   nullptr);
    transpose_bf16_kernel<<<dim3((H + 31) / 32, (E + 31) / 32), 256, 0, s>>>(E, H, m->W2h, H,
                                                                              m->W2Th, E);
#undef STEP
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// training schedule over (query, reference) pairs

namespace {

// output k (0-based) of the SplitMix64 stream started at `seed` (Steele, Lea,
// Flood, OOPSLA 2014): the state after k + 1 increments of the golden gamma,
// through the generator's output mix
__device__ __forceinline__ uint64_t splitmix64_output(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// pair k -> key = sorted library row of its reference (2^32 - 1 when the
// index is outside the library), value = k; counts the valid pairs
__global__ void pair_keys_kernel(int64_t n, const int64_t* __restrict__ target,
                                 const uint32_t* __restrict__ slot, int64_t nlib,
                                 uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                 unsigned long long* __restrict__ n_valid)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = k < n;
    const int64_t t = in ? target[k] : -1;
    const bool valid = t >= 0 && t < nlib;
    if (in) {
        keys[k] = valid ? (uint64_t)slot[t] : 0xFFFFFFFFull;
        vals[k] = (uint32_t)k;
    }
    const uint64_t m = __ballot(valid);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(n_valid, (unsigned long long)__popcll(m));
}

// ordered pair j -> its query row and its reference's sorted library row
__global__ void pair_rows_kernel(int64_t n, const uint64_t* __restrict__ keys,
                                 const uint32_t* __restrict__ vals, uint32_t* __restrict__ q_rows,
                                 uint32_t* __restrict__ r_rows)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    q_rows[j] = vals[j];
    r_rows[j] = (uint32_t)keys[j];
}

// batch b of epoch e -> key = SplitMix64 output e * nb + b, value = b
__global__ void epoch_keys_kernel(int64_t nb, int64_t epoch, uint64_t seed,
                                  uint64_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    keys[b] = splitmix64_output(seed, (uint64_t)(epoch * nb + b));
    vals[b] = (uint32_t)b;
}

}  // namespace

hipError_t model_train(homs_model* m, int64_t n, const uint32_t* q_hv, const int64_t* target,
                       int epochs, int B, float lr, float tau, uint64_t seed, float* losses,
                       int64_t* steps_out, hipStream_t s)
{
    *steps_out = 0;
    const homs_ctx* c = m->ctx;
    const int64_t cap = n > 1 ? n : 1;
    const size_t sort_tmp = radix_sort_temp_bytes(cap);
    const size_t need = 2 * al((size_t)cap * 8) + 4 * al((size_t)cap * 4) + al(sort_tmp) + al(8);
    char* base = nullptr;
    hipError_t e = dev_malloc((void**)&base, need);
    if (e != hipSuccess) return e;
    char* p = base;
    auto take = [&](size_t bytes) {
        void* r = p;
        p += al(bytes);
        return r;
    };
    uint64_t* ka = (uint64_t*)take((size_t)cap * 8);
    uint64_t* kb = (uint64_t*)take((size_t)cap * 8);
    uint32_t* va = (uint32_t*)take((size_t)cap * 4);
    uint32_t* vb = (uint32_t*)take((size_t)cap * 4);
    uint32_t* q_rows = (uint32_t*)take((size_t)cap * 4);
    uint32_t* r_rows = (uint32_t*)take((size_t)cap * 4);
    void* tmp = take(sort_tmp);
    unsigned long long* d_valid = (unsigned long long*)take(8);
    unsigned long long n_valid = 0;
    int64_t nb = 0;
    bool alt = false;

    e = hipMemsetAsync(d_valid, 0, 8, s);
    if (e == hipSuccess && n > 0) {
        pair_keys_kernel<<<blocks_for(n), kThreads, 0, s>>>(n, target, c->lib.slot, c->lib.n, ka,
                                                            va, d_valid);
        // stable: pairs of one reference keep their input order
        e = radix_sort_pairs(n, ka, kb, va, vb, 0, 32, tmp, s, &alt);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&n_valid, d_valid, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
        nb = (int64_t)n_valid / B;
        if (nb > 0) {
            // invalid pairs sorted last; the last partial batch is dropped
            pair_rows_kernel<<<blocks_for(nb * B), kThreads, 0, s>>>(
                nb * B, alt ? kb : ka, alt ? vb : va, q_rows, r_rows);
            e = hipGetLastError();
        }
    }
    for (int ep = 0; ep < epochs && e == hipSuccess && nb > 0; ++ep) {
        epoch_keys_kernel<<<blocks_for(nb), kThreads, 0, s>>>(nb, ep, seed, ka, va);
        e = radix_sort_pairs(nb, ka, kb, va, vb, 0, 64, tmp, s, &alt);
        const uint32_t* perm = alt ? vb : va;
        for (int64_t j = 0; j < nb && e == hipSuccess; ++j) {
            const RowSelect sel{q_rows, r_rows, perm, j};
            e = model_step(m, B, q_hv, c->lib.hv, tau, lr, true,
                           losses ? losses + (int64_t)ep * nb + j : m->loss_scratch, s, &sel);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(base);
    if (e == hipSuccess) *steps_out = (int64_t)epochs * nb;
    return e;
}

}  // namespace homs
