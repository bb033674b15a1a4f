// Eq. 1 encoding (Section 3.3) on gfx950.
//
// One group of D/128 consecutive lanes encodes one spectrum; lane w owns the
// 128 components 128w .. 128w+127 (one uint4 of the packed row). For every
// peak (bin i, level j) the lane loads its uint4 of F_i (a coalesced 16-byte
// load: the group reads the whole 1 KiB row at D = 8192) and of L_j, binds
// them with XOR (bit 0 = +1, so the bipolar product is XOR) and adds the
// 128 resulting bits into bit-sliced counters: plane k holds bit k of the
// number of -1 components seen so far. Peaks are taken eight at a time: the
// 16 row loads of a group are issued together (the kernel waits on gathered
// rows, so loads in flight set its speed), and the eight bound rows enter the
// counters through a carry-save tree of full adders on the three low planes
// (the Harley-Seal scheme: planes 0, 1 and 2 take the ones, twos and fours,
// one carry of weight 8 ripples into the planes above): 21 + 2(P - 3)
// operations per word for eight peaks (27 at P = 6) where a ripple of half
// adders takes 2P per peak (96). The last, partial group is masked. The bipolar sum is I = n - 2c
// (n peaks, c components equal to -1), so the binarised bit (1 unless I > 0)
// is c >= ceil(n/2), evaluated on the planes with a bit-sliced comparison
// against that constant.
//
// The random-projection baseline of Section 4.2 weights bin i's random row by
// w = level + 1 instead of binding it with a level vector: S = W - 2c with
// W = sum of the weights and c the weighted count of -1 components, added to
// the planes as w's binary digits (the row's bits enter plane k for every
// set bit k of w); the bit is c >= ceil(W/2) again.
#include "internal.h"

namespace homs {
namespace {

struct U4 {
    uint32_t v[4];
};

// one bit-sliced full adder: a + b + c = sum + 2 carry in every bit position
// (carry = majority, one bitfield select)
__device__ __forceinline__ void full_add(uint32_t a, uint32_t b, uint32_t c, uint32_t& sum,
                                         uint32_t& carry)
{
    const uint32_t u = a ^ b;
    sum = u ^ c;
    carry = (u & c) | (~u & a);
}

// add eight 0/1 slices to the counters (P >= 4): the low three planes act as
// carry-save accumulators of weight 1, 2 and 4 and the carry of weight 8
// ripples from plane 3 up, so the count is sum_k plane_k 2^k after every group
template <int P>
__device__ __forceinline__ void add_eight(U4 (&c)[P], const U4 (&x)[8])
{
    static_assert(P >= 4, "the carry-save tree needs planes 0..3");
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint32_t ta, tb, fa, fb, y;
        full_add(c[0].v[e], x[0].v[e], x[1].v[e], c[0].v[e], ta);
        full_add(c[0].v[e], x[2].v[e], x[3].v[e], c[0].v[e], tb);
        full_add(c[1].v[e], ta, tb, c[1].v[e], fa);
        full_add(c[0].v[e], x[4].v[e], x[5].v[e], c[0].v[e], ta);
        full_add(c[0].v[e], x[6].v[e], x[7].v[e], c[0].v[e], tb);
        full_add(c[1].v[e], ta, tb, c[1].v[e], fb);
        full_add(c[2].v[e], fa, fb, c[2].v[e], y);
#pragma unroll
        for (int k = 3; k < P; ++k) {
            const uint32_t carry = c[k].v[e] & y;
            c[k].v[e] ^= y;
            y = carry;
        }
    }
}

// bit-sliced (count >= t) for a constant t < 2^P
template <int P>
__device__ __forceinline__ U4 at_least(const U4 (&c)[P], uint32_t t)
{
    U4 gt, eq;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        gt.v[e] = 0u;
        eq.v[e] = ~0u;
    }
#pragma unroll
    for (int k = P - 1; k >= 0; --k) {
        const bool tk = (t >> k) & 1u;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (tk) {
                eq.v[e] &= c[k].v[e];
            } else {
                gt.v[e] |= eq.v[e] & c[k].v[e];
                eq.v[e] &= ~c[k].v[e];
            }
        }
    }
    U4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r.v[e] = gt.v[e] | eq.v[e];
    return r;
}

template <int P>
__device__ __forceinline__ U4 encode_one(const uint4* __restrict__ id, const uint4* __restrict__ lv,
                                         uint32_t w4, uint32_t lane, int64_t a, int64_t b,
                                         const int32_t* __restrict__ bin,
                                         const uint8_t* __restrict__ level, int64_t n_bins,
                                         uint32_t n_levels, uint32_t* __restrict__ err)
{
    U4 c[P];
#pragma unroll
    for (int k = 0; k < P; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) c[k].v[e] = 0u;
    uint32_t n_ok = 0;
    bool bad = false;
    // one group of eight peaks from p on; with `partial`, the slots from b on
    // re-read peak b - 1 and are masked off. A peak out of range adds nothing
    // and is not counted (row 0 is loaded in its place and masked off).
    auto group = [&](int64_t p, bool partial) {
        U4 x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const bool present = !partial || p + i < b;
            const int64_t q = present ? p + i : b - 1;
            const int32_t bi = bin[q];
            const uint32_t lj = level[q];
            const bool in_range = bi >= 0 && (int64_t)bi < n_bins && lj < n_levels;
            const bool ok = present && in_range;
            const uint4 f = id[(ok ? (size_t)bi : 0) * w4 + lane];
            const uint4 l = lv[(ok ? (size_t)lj : 0) * w4 + lane];
            const uint32_t m = ok ? ~0u : 0u;
            x[i].v[0] = (f.x ^ l.x) & m;
            x[i].v[1] = (f.y ^ l.y) & m;
            x[i].v[2] = (f.z ^ l.z) & m;
            x[i].v[3] = (f.w ^ l.w) & m;
            n_ok += ok ? 1u : 0u;
            bad |= present && !in_range;
        }
        add_eight<P>(c, x);
    };
    int64_t p = a;
    for (; p + 8 <= b; p += 8) group(p, false);
    if (p < b) group(p, true);
    if (bad && lane == 0) atomicOr(err, kErrRange);
    return at_least<P>(c, (n_ok + 1u) / 2u);
}

// add x * w to the counters: x enters plane k for every set bit k of w
template <int P>
__device__ __forceinline__ void add_weighted(U4 (&c)[P], const U4& x, uint32_t w)
{
#pragma unroll
    for (int k0 = 0; k0 < 9; ++k0) {  // w <= 256
        if (!((w >> k0) & 1u)) continue;  // uniform over the lane group
        U4 y = x;
#pragma unroll
        for (int k = k0; k < P; ++k) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t carry = c[k].v[e] & y.v[e];
                c[k].v[e] ^= y.v[e];
                y.v[e] = carry;
            }
        }
    }
}

template <int P>
__device__ __forceinline__ U4 encode_one_lsh(const uint4* __restrict__ id, uint32_t w4,
                                             uint32_t lane, int64_t a, int64_t b,
                                             const int32_t* __restrict__ bin,
                                             const uint8_t* __restrict__ level, int64_t n_bins,
                                             uint32_t n_levels, uint32_t* __restrict__ err)
{
    U4 c[P];
#pragma unroll
    for (int k = 0; k < P; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) c[k].v[e] = 0u;
    uint32_t W = 0;
    for (int64_t p = a; p < b; ++p) {
        const int32_t bi = bin[p];
        const uint32_t lj = level[p];
        if (bi < 0 || (int64_t)bi >= n_bins || lj >= n_levels) {
            if (lane == 0) atomicOr(err, kErrRange);
            continue;
        }
        const uint4 f = id[(size_t)bi * w4 + lane];
        U4 x;
        x.v[0] = f.x;
        x.v[1] = f.y;
        x.v[2] = f.z;
        x.v[3] = f.w;
        add_weighted<P>(c, x, lj + 1u);
        W += lj + 1u;
    }
    return at_least<P>(c, (W + 1u) / 2u);
}

// Spectra by size class: kClass 0 below 64 peaks, 1 from 64 to 255, 2 from
// 256 on (wider counters). The launches write disjoint spectra; splitting
// keeps the register count, and so the occupancy, of the common case
// independent of the counters that larger spectra need.
__device__ __forceinline__ int size_class(int64_t np) { return np < 64 ? 0 : np < 256 ? 1 : 2; }

template <int kClass>
__global__ __launch_bounds__(256) void encode_lsh_kernel(
    const uint4* __restrict__ id, uint32_t w4, uint32_t per_block, int64_t n,
    const int64_t* __restrict__ off, const int32_t* __restrict__ bin,
    const uint8_t* __restrict__ level, int64_t n_bins, uint32_t n_levels,
    const uint32_t* __restrict__ slot, uint4* __restrict__ out, uint32_t* __restrict__ err)
{
    const uint32_t t = threadIdx.x;
    const uint32_t sub = t / w4;
    const uint32_t lane = t - sub * w4;
    if (sub >= per_block) return;
    const int64_t s = (int64_t)blockIdx.x * per_block + sub;
    if (s >= n) return;
    const int64_t a = off[s], b = off[s + 1];
    const int64_t np = b - a;
    // planes for the largest weighted count: np * 256
    if (size_class(np) != kClass) return;
    U4 r;
    if constexpr (kClass == 0)
        r = encode_one_lsh<14>(id, w4, lane, a, b, bin, level, n_bins, n_levels, err);
    else if constexpr (kClass == 1)
        r = encode_one_lsh<16>(id, w4, lane, a, b, bin, level, n_bins, n_levels, err);
    else
        r = encode_one_lsh<32>(id, w4, lane, a, b, bin, level, n_bins, n_levels, err);
    const int64_t row = slot ? (int64_t)slot[s] : s;
    out[(size_t)row * w4 + lane] = make_uint4(r.v[0], r.v[1], r.v[2], r.v[3]);
}

template <int kClass>
__global__ __launch_bounds__(256) void encode_kernel(
    const uint4* __restrict__ id, const uint4* __restrict__ lv, uint32_t w4, uint32_t per_block,
    int64_t n, const int64_t* __restrict__ off, const int32_t* __restrict__ bin,
    const uint8_t* __restrict__ level, int64_t n_bins, uint32_t n_levels,
    const uint32_t* __restrict__ slot, uint4* __restrict__ out, uint32_t* __restrict__ err)
{
    const uint32_t t = threadIdx.x;
    const uint32_t sub = t / w4;
    const uint32_t lane = t - sub * w4;
    if (sub >= per_block) return;
    const int64_t s = (int64_t)blockIdx.x * per_block + sub;
    if (s >= n) return;
    const int64_t a = off[s], b = off[s + 1];
    const int64_t np = b - a;
    if (size_class(np) != kClass) return;
    U4 r;
    if constexpr (kClass == 0) {
        r = encode_one<6>(id, lv, w4, lane, a, b, bin, level, n_bins, n_levels, err);
    } else if constexpr (kClass == 1) {
        r = encode_one<8>(id, lv, w4, lane, a, b, bin, level, n_bins, n_levels, err);
    } else {
        if (np < 65536)
            r = encode_one<16>(id, lv, w4, lane, a, b, bin, level, n_bins, n_levels, err);
        else
            r = encode_one<32>(id, lv, w4, lane, a, b, bin, level, n_bins, n_levels, err);
    }
    const int64_t row = slot ? (int64_t)slot[s] : s;
    out[(size_t)row * w4 + lane] = make_uint4(r.v[0], r.v[1], r.v[2], r.v[3]);
}

}  // namespace

hipError_t launch_encode(const homs_ctx* c, int64_t n, const int64_t* off, const int32_t* bin,
                         const uint8_t* level, const uint32_t* slot, uint32_t* out,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const uint32_t w4 = c->words / 4;  // lanes per spectrum
    const uint32_t per_block = 256u / w4;
    const int64_t blocks = (n + per_block - 1) / per_block;
    // one launch per size class (each returns at once for the spectra of the
    // other classes)
    if (c->p.encoding == HOMS_ENCODING_LSH) {
        auto lsh = [&](auto kern) {
            kern<<<dim3((uint32_t)blocks), dim3(per_block * w4), 0, s>>>(
                reinterpret_cast<const uint4*>(c->d_id), w4, per_block, n, off, bin, level,
                c->n_bins, c->p.n_levels, slot, reinterpret_cast<uint4*>(out), c->d_err);
        };
        lsh(encode_lsh_kernel<0>);
        lsh(encode_lsh_kernel<1>);
        lsh(encode_lsh_kernel<2>);
        return hipGetLastError();
    }
    auto idl = [&](auto kern) {
        kern<<<dim3((uint32_t)blocks), dim3(per_block * w4), 0, s>>>(
            reinterpret_cast<const uint4*>(c->d_id), reinterpret_cast<const uint4*>(c->d_level),
            w4, per_block, n, off, bin, level, c->n_bins, c->p.n_levels, slot,
            reinterpret_cast<uint4*>(out), c->d_err);
    };
    idl(encode_kernel<0>);
    idl(encode_kernel<1>);
    idl(encode_kernel<2>);
    return hipGetLastError();
}

}  // namespace homs
