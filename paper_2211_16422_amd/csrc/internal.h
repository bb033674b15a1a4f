// Internal declarations shared by the host side of libhyperoms and its kernel
// launchers. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "hyperoms.h"

namespace homs {

// Device-side error flag bits.
constexpr uint32_t kErrRange = 1u;  // bin >= f or level >= Q in an encode
constexpr uint32_t kErrPeaks = 2u;  // a spectrum keeping more peaks than device preprocessing holds

struct Library {
    int64_t n = 0;
    uint32_t* hv = nullptr;      // [n][W] rows in sorted order
    double* pmz = nullptr;       // [n] sorted precursor m/z
    int8_t* charge = nullptr;    // [n] sorted charge (all 0 when charge is ignored)
    uint32_t* orig = nullptr;    // [n] library index of each sorted row
    uint32_t* slot = nullptr;    // [n] sorted row of each library index
    float* rowk = nullptr;       // [n + pad] the fp4 search's per-row constant K
};

struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Tunables of the batched persistent search (homs_batched_config).
struct BatchedConfig {
    uint32_t narrow_max = 1024;   // windows up to this size are scored per query
    uint32_t chunk_rows = 2048;   // candidate rows per wide work item
    uint32_t narrow_group = 32;   // narrow queries per work item (multiple of 4)
    uint32_t grid = 1024;         // persistent workgroups
    double bucket_da = 0.5;       // precursor bucket width for query ordering
    int32_t engine = HOMS_ENGINE_MFMA_F4;  // wide tiles: popcount, fp8 or fp4 matrix cores
};

// A captured batched search, replayed while its arguments stay the same.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<uintptr_t> key;
};

// Event-based kernel timing (homs_profile_*).
enum ProfKind { kProfSearch = 0, kProfEncode = 1, kProfPrep = 2, kProfScore = 3 };
struct Profiler {
    bool on = false;
    struct Span {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Span> pending;
    std::vector<hipEvent_t> pool;
    double ms[4] = {0, 0, 0, 0};
    int64_t launches[4] = {0, 0, 0, 0};
};

}  // namespace homs

struct homs_ctx {
    homs_params p{};
    int device = 0;
    int64_t n_bins = 0;  // f
    uint32_t words = 0;  // W = D / 32
    uint32_t* d_id = nullptr;     // [f][W]
    uint32_t* d_level = nullptr;  // [Q][W]
    uint32_t* d_err = nullptr;    // device error flags
    homs::Library lib;
    bool lib_valid = false;
    uint64_t lib_gen = 0;  // bumped by every homs_encode_library
    homs::Workspace ws;
    homs::Profiler prof;
    homs::BatchedConfig batched;
    homs::GraphCache graph;
    hipStream_t capture_stream = nullptr;
    void* noalloc_scratch = nullptr;  // device address of this device's static scratch
    bool dead = false;
    std::string err;
};

namespace homs {

// Every device allocation of the library: hipMalloc, except under the test
// hook HOMS_TEST_FAIL_ALLOC=n (environment variable, read at every call):
// the n-th call after the variable last changed value fails with
// hipErrorOutOfMemory and allocates nothing (text after the number, as in
// "3:b", only re-arms the count). api.hip.
hipError_t dev_malloc(void** p, size_t bytes);
template <class T>
inline hipError_t dev_malloc(T** p, size_t bytes)
{
    return dev_malloc(reinterpret_cast<void**>(p), bytes);
}

// ---- kernel launchers (each in its own translation unit) -------------------

// encode.hip
hipError_t launch_encode(const homs_ctx* c, int64_t n, const int64_t* off, const int32_t* bin,
                         const uint8_t* level, const uint32_t* slot, uint32_t* out,
                         hipStream_t s);

// sort_scan.hip: exclusive prefix sums (uint32_t and int64_t; in and out may
// be the same buffer) and a stable LSD radix sort of (uint64 key, uint32
// value) pairs over key bits [begin_bit, end_bit) (a multiple of 8 wide);
// the sorted pairs end in the *_alt buffers when *in_alt is set on return.
size_t scan_temp_bytes(int64_t n);
template <typename T>
hipError_t exclusive_scan(const T* in, T* out, int64_t n, void* temp, hipStream_t s);
size_t radix_sort_temp_bytes(int64_t n);
hipError_t radix_sort_pairs(int64_t n, uint64_t* keys, uint64_t* keys_alt, uint32_t* vals,
                            uint32_t* vals_alt, int begin_bit, int end_bit, void* temp,
                            hipStream_t s, bool* in_alt);

// library.hip
size_t library_sort_temp_bytes(int64_t n);
hipError_t launch_library_sort(int64_t n, const double* pmz, const int8_t* charge,
                               bool use_charge, void* temp, size_t temp_bytes,
                               uint32_t* perm_out, double* pmz_out, int8_t* charge_out,
                               uint32_t* slot_out, hipStream_t s);
hipError_t launch_gather_rows(int64_t n, uint32_t words, const uint32_t* src,
                              const uint32_t* orig, uint32_t* dst, hipStream_t s);
// slot[orig[j]] = j; orig must be a permutation of [0, n)
hipError_t launch_slots(int64_t n, const uint32_t* orig, uint32_t* slot, hipStream_t s);
hipError_t launch_window_bounds(const homs_ctx* c, int64_t nq, const double* q_pmz,
                                const int8_t* q_charge, int32_t kind, double value,
                                const int8_t* kinds, const double* values, int64_t* lo,
                                int64_t* hi, hipStream_t s);
size_t query_sort_temp_bytes(int64_t nq);
hipError_t launch_query_sort(int64_t nq, const double* q_pmz, const int8_t* q_charge,
                             bool use_charge, void* temp, size_t temp_bytes,
                             uint64_t* keys_a, uint64_t* keys_b, uint32_t* perm_a,
                             uint32_t* perm_b, uint32_t** perm_out, hipStream_t s);
hipError_t launch_init_keys(int64_t nq, uint64_t* keys, hipStream_t s);
hipError_t launch_finalize(int64_t nq, const uint64_t* keys, int64_t* idx, int32_t* dist,
                           hipStream_t s);
hipError_t launch_debug_distances(const homs_ctx* c, int64_t nq, const uint32_t* q_hv,
                                  const int64_t* lo, const int64_t* hi,
                                  const int64_t* row_off, int64_t* out_idx, int32_t* out_dist,
                                  hipStream_t s);

// search_popc.hip
struct TilePlan {
    int64_t n_tiles = 0;
    int64_t max_chunks = 0;
    int64_t chunk_rows = 0;
};
hipError_t launch_tile_bounds(int64_t nq, const uint32_t* qperm, const int64_t* lo,
                              const int64_t* hi, int tile, int64_t* tile_lo, int64_t* tile_hi,
                              hipStream_t s);
hipError_t launch_search_popcount(const homs_ctx* c, int64_t nq, const uint32_t* q_hv,
                                  const uint32_t* qperm, const int64_t* lo, const int64_t* hi,
                                  const int64_t* tile_lo, const int64_t* tile_hi,
                                  const TilePlan& plan, uint64_t* keys, hipStream_t s);
int search_popcount_tile();

// search_batched.hip
size_t batched_scratch_bytes(int64_t nq);
hipError_t launch_search_batched(const homs_ctx* c, const BatchedConfig& cfg, void* scratch,
                                 int64_t nq, const uint32_t* q_hv, const double* q_pmz,
                                 const int8_t* q_charge, const int8_t* kinds,
                                 const double* values, int64_t* out_idx, int32_t* out_dist,
                                 hipStream_t s);

// search_mfma.hip (fmt 0: int8, 1: fp8 e4m3, 2: fp4 e2m1)
int search_mfma_tile();
int64_t search_mfma_row_pad();  // rows of padding the library's orig array needs
// qoff: workspace of nq int32 (the fp4 form's per-query constants)
hipError_t launch_search_mfma(const homs_ctx* c, int fmt, int64_t nq, const uint32_t* q_hv,
                              const uint32_t* qperm, const int64_t* lo, const int64_t* hi,
                              const int64_t* tile_lo, const int64_t* tile_hi, int32_t* qoff,
                              uint64_t* keys, hipStream_t s);
// the fp4 form's per-row constants K of n rows of hv, then search_mfma_row_pad() zeros
hipError_t launch_fp4_row_consts(int64_t n, uint32_t words, const uint32_t* hv, float* rowk,
                                 hipStream_t s);
hipError_t launch_fp4_query_offsets(const homs_ctx* c, int64_t nq, const uint32_t* q_hv,
                                    int32_t* qoff, hipStream_t s);

// prep_device.hip: preprocessing of raw spectra on the device
int prep_device_max_peaks();
size_t prep_device_scratch_bytes(int64_t n, uint32_t top_n);
hipError_t launch_preprocess_device(const homs_ctx* c, int64_t n, const int64_t* off,
                                    const double* mz, const double* inten, int64_t* out_off,
                                    int32_t* out_bin, uint8_t* out_level, void* scratch,
                                    hipStream_t s);

// cascade.hip: FDR filtering between the stages of homs_cascade_search
struct CascadeScratch {
    double* pmz2;     // [nq] open-stage precursors (+inf for identified queries)
    int64_t* idx2;    // [nq] open-stage top-1
    int32_t* dist2;   // [nq]
    uint32_t* hist;   // [2 (D + 1)] PSMs by distance: targets, then decoys
    double* qtab;     // [D + 1] q-value of each distance
};
size_t cascade_scratch_bytes(int64_t nq, uint32_t dim);
CascadeScratch cascade_carve(void* base, int64_t nq, uint32_t dim);
// second = 0: PSMs of every query (idx, dist: narrow stage), sets stage and
// qvalue; second = 1: PSMs of the queries with stage != 1 (idx, dist: open
// stage), which also take these results into out_idx / out_dist
hipError_t launch_fdr_stage(int second, int64_t nq, uint32_t dim, const int64_t* idx,
                            const int32_t* dist, const uint8_t* lib_decoy, double level,
                            const CascadeScratch& w, int8_t* stage, double* qvalue,
                            int64_t* out_idx, int32_t* out_dist, hipStream_t s);
hipError_t launch_mask_identified(int64_t nq, const double* pmz, const int8_t* stage,
                                  double* pmz2, hipStream_t s);

}  // namespace homs
