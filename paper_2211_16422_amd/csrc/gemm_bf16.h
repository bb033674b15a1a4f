// bf16 matrix-core GEMM used by the learned shortlist:
//     C[m][n] = alpha * sum_k A[m][k] * B[n][k]   (+ epilogue)
// A is M x K and B is N x K, both row-major bf16 with K contiguous ("NT"),
// fp32 accumulation on v_mfma_f32_32x32x16_bf16. K must be a multiple of 32;
// M and N are arbitrary (loads clamp, stores mask).
//
// Workgroup tile 128 x 128 with four waves in a 2 x 2 grid (64 x 64 per
// wave, 2 x 2 MFMA tiles of 32 x 32). K advances 32 at a time through a
// double-buffered LDS stage (rows padded to 80 bytes so 16 lanes of a
// 16-byte read hit 64 distinct banks); the global loads of the next two
// stages are in flight while the current stage's MFMAs run.
//
// Operand layout of 32x32x16 bf16 (checked on gfx950): lane l supplies row
// (l % 32) and the 8 consecutive k of group (l / 32); accumulator register r
// of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
#pragma once

#include "internal.h"

namespace homs {
namespace gemm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTM = 128, kTN = 128, kTK = 32, kRowBytes = 80;

enum Epi : int {
    kBias = 1,       // + bias[n]
    kRelu = 2,       // max(., 0)
    kMask = 4,       // * (mask[m][n] > 0), mask fp32 with C's layout
    kStoreF32 = 8,   // C (fp32, ldc)
    kStoreBf16 = 16, // Cb (bf16, ldcb)
    kReluBf16 = 32   // ReLU applied to the bf16 store only (C keeps the pre-activation)
};

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    // round to nearest even; inputs here are finite
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One thread's share of a K step: pieces c = 2t and 2t + 1 of the 512
// 16-byte pieces of a 128 x 32 bf16 tile (row c / 4, piece c % 4), for A and B.
struct Stage {
    uint4 a0, a1, b0, b1;
};

__device__ __forceinline__ Stage load_stage(const uint16_t* a_row, const uint16_t* b_row, int k0)
{
    Stage st;
    st.a0 = *(const uint4*)(a_row + k0);
    st.a1 = *(const uint4*)(a_row + k0 + 8);
    st.b0 = *(const uint4*)(b_row + k0);
    st.b1 = *(const uint4*)(b_row + k0 + 8);
    return st;
}

__device__ __forceinline__ void store_stage(const Stage& st, uint8_t* sa, uint8_t* sb, int buf)
{
    const int off = buf * (kTM * kRowBytes);
    *(uint4*)(sa + off) = st.a0;
    *(uint4*)(sa + off + 16) = st.a1;
    *(uint4*)(sb + off) = st.b0;
    *(uint4*)(sb + off + 16) = st.b1;
}

template <int EPI>
__global__ __launch_bounds__(256) void gemm_nt_kernel(
    int M, int N, int K, const uint16_t* __restrict__ A, int lda, const uint16_t* __restrict__ B,
    int ldb, float alpha, const float* __restrict__ bias, const float* __restrict__ mask,
    float* __restrict__ C, int ldc, uint16_t* __restrict__ Cb, int ldcb)
{
    __shared__ __attribute__((aligned(16))) uint8_t sA[2][kTM * kRowBytes];
    __shared__ __attribute__((aligned(16))) uint8_t sB[2][kTN * kRowBytes];
    const int t = threadIdx.x, l = t & 63, w = t >> 6, wr = w & 1, wn = w >> 1;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;

    // global -> register staging: 2 x 16 bytes of A and of B per thread
    const int row0 = t >> 1, part0 = (t * 2) & 3;  // pieces c = 2t, 2t + 1
    const uint16_t* a_row = A + (size_t)min(m0 + row0, M - 1) * lda + part0 * 8;
    const uint16_t* b_row = B + (size_t)min(n0 + row0, N - 1) * ldb + part0 * 8;
    uint8_t* sa_dst = &sA[0][0] + row0 * kRowBytes + part0 * 16;
    uint8_t* sb_dst = &sB[0][0] + row0 * kRowBytes + part0 * 16;
    Stage st;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{0};

    const int nk = K / kTK;
    // Two K steps of loads in flight, in two named register sets (a copy
    // from one set to the other would wait for the newer loads): at step s
    // the set of step s + 1 is stored to LDS while the loads of step s + 2
    // fill the other set, so each load has two steps of matrix work to land.
    // The loads are unconditional (past the last step they re-read it), so
    // that the compiler's wait before a store counts only the older set.
    auto compute = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = *(const bf16x8*)(sA[buf] + (wr * 64 + i * 32 + (l & 31)) * kRowBytes +
                                         ks * 32 + 16 * (l >> 5));
                bv[i] = *(const bf16x8*)(sB[buf] + (wn * 64 + i * 32 + (l & 31)) * kRowBytes +
                                         ks * 32 + 16 * (l >> 5));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0,
                                                                       0, 0);
        }
    };
    Stage st1;
    st = load_stage(a_row, b_row, 0);
    store_stage(st, sa_dst, sb_dst, 0);
    if (nk > 1) st1 = load_stage(a_row, b_row, kTK);
    __syncthreads();
    for (int s = 0; s < nk; s += 2) {
        // LDS buffer 0 holds step s, st1 step s + 1
        st = load_stage(a_row, b_row, min(s + 2, nk - 1) * kTK);
        compute(0);
        if (s + 1 < nk) store_stage(st1, sa_dst, sb_dst, 1);
        __syncthreads();
        if (s + 1 >= nk) break;
        // LDS buffer 1 holds step s + 1, st step s + 2
        st1 = load_stage(a_row, b_row, min(s + 3, nk - 1) * kTK);
        compute(1);
        if (s + 2 < nk) store_stage(st, sa_dst, sb_dst, 0);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 64 + j * 32 + (l & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wr * 64 + i * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
                if (m >= M || n >= N) continue;
                float v = alpha * acc[i][j][r];
                if (EPI & kBias) v += bias[n];
                if (EPI & kRelu) v = v > 0.f ? v : 0.f;
                if (EPI & kMask) v = mask[(size_t)m * ldc + n] > 0.f ? v : 0.f;
                if (EPI & kStoreF32) C[(size_t)m * ldc + n] = v;
                if (EPI & kStoreBf16)
                    Cb[(size_t)m * ldcb + n] = to_bf16((EPI & kReluBf16) && v < 0.f ? 0.f : v);
            }
        }
}

template <int EPI>
inline hipError_t gemm_nt(hipStream_t s, int M, int N, int K, const uint16_t* A, int lda,
                          const uint16_t* B, int ldb, float alpha, const float* bias,
                          const float* mask, float* C, int ldc, uint16_t* Cb, int ldcb)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K % kTK != 0 || lda % 8 != 0 || ldb % 8 != 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((N + kTN - 1) / kTN), (unsigned)((M + kTM - 1) / kTM));
    gemm_nt_kernel<EPI><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, alpha, bias, mask, C, ldc,
                                             Cb, ldcb);
    return hipGetLastError();
}

}  // namespace gemm
}  // namespace homs
