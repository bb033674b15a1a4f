// C ABI of libhyperoms: argument validation, context and memory management,
// and the order of kernel launches for each entry point.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "codebook.h"
#include "internal.h"
#include "learned.h"
#include "persist.h"
#include "preprocess.h"

namespace homs {

hipError_t dev_malloc(void** p, size_t bytes)
{
    const char* v = std::getenv("HOMS_TEST_FAIL_ALLOC");
    if (v && *v) {
        static std::mutex mu;
        static std::string armed;
        static long calls = 0;
        std::lock_guard<std::mutex> lock(mu);
        if (armed != v) {
            armed = v;
            calls = 0;
        }
        if (++calls == std::strtol(v, nullptr, 10)) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    return hipMalloc(p, bytes);
}

}  // namespace homs

namespace {

thread_local std::string g_last_error;

homs_status fail(homs_ctx* c, homs_status s, const std::string& msg)
{
    if (c) {
        c->err = msg;
        if (s == HOMS_E_DEVICE) c->dead = true;
    } else {
        g_last_error = msg;
    }
    return s;
}

homs_status hip_fail(homs_ctx* c, hipError_t e, const char* what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        return fail(c, HOMS_E_OOM, msg);
    }
    return fail(c, HOMS_E_DEVICE, msg);
}

#define HIP_TRY(c, expr, what)                      \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hip_fail((c), e_, (what)); \
    } while (0)

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool params_valid(const homs_params* p, std::string* why)
{
    if (!p) {
        *why = "params is NULL";
        return false;
    }
    if (p->struct_size != sizeof(homs_params)) {
        *why = "params.struct_size != sizeof(homs_params)";
        return false;
    }
    if (p->dim < 512 || p->dim > 32768 || p->dim % 512 != 0) {
        *why = "dim must be a multiple of 512 in [512, 32768]";
        return false;
    }
    if (p->n_levels < 2 || p->n_levels > 255) {
        *why = "n_levels must be in [2, 255]";
        return false;
    }
    if (p->encoding != HOMS_ENCODING_ID_LEVEL && p->encoding != HOMS_ENCODING_RANDOM_ID &&
        p->encoding != HOMS_ENCODING_LSH) {
        *why = "encoding must be HOMS_ENCODING_ID_LEVEL, _RANDOM_ID or _LSH";
        return false;
    }
    if (p->top_n < 1) {
        *why = "top_n must be >= 1";
        return false;
    }
    if (!std::isfinite(p->mz_min) || !std::isfinite(p->mz_max) || !(p->mz_max > p->mz_min) ||
        !std::isfinite(p->bins_per_da) || !(p->bins_per_da > 0.0) ||
        !std::isfinite(p->noise_frac) || p->noise_frac < 0.0 || p->noise_frac > 1.0) {
        *why = "invalid m/z range, bin width or noise fraction";
        return false;
    }
    const double f = std::ceil((p->mz_max - p->mz_min) * p->bins_per_da);
    if (!(f >= 1.0) || f > 16777216.0) {
        *why = "number of m/z bins must be in [1, 2^24]";
        return false;
    }
    if (p->id_flips > p->dim) {
        *why = "id_flips must be <= dim";
        return false;
    }
    if (p->charge_match > 1) {
        *why = "charge_match must be 0 or 1";
        return false;
    }
    return true;
}

bool window_valid(const homs_window* w, std::string* why)
{
    if (!w) {
        *why = "window is NULL";
        return false;
    }
    if (w->kind != HOMS_TOL_DA && w->kind != HOMS_TOL_PPM) {
        *why = "window kind must be HOMS_TOL_DA or HOMS_TOL_PPM";
        return false;
    }
    if (!std::isfinite(w->value) || w->value < 0.0) {
        *why = "window value must be finite and >= 0";
        return false;
    }
    return true;
}

homs_status usable(homs_ctx* c)
{
    if (!c) return fail(nullptr, HOMS_E_INVALID, "ctx is NULL");
    if (c->dead) return fail(c, HOMS_E_DEVICE, "context is in a device-error state: " + c->err);
    return HOMS_OK;
}

void free_library(homs::Library& L)
{
    if (L.hv) (void)hipFree(L.hv);
    if (L.pmz) (void)hipFree(L.pmz);
    if (L.charge) (void)hipFree(L.charge);
    if (L.orig) (void)hipFree(L.orig);
    if (L.slot) (void)hipFree(L.slot);
    if (L.rowk) (void)hipFree(L.rowk);
    L = homs::Library{};
}

void drop_graph(homs_ctx* c);

// Grows the context's workspace to at least `bytes` (synchronising first).
homs_status ensure_workspace(homs_ctx* c, size_t bytes, hipStream_t s)
{
    if (c->ws.bytes >= bytes) return HOMS_OK;
    HIP_TRY(c, hipStreamSynchronize(s), "hipStreamSynchronize");
    drop_graph(c);
    if (c->ws.ptr) (void)hipFree(c->ws.ptr);
    c->ws = homs::Workspace{};
    const size_t want = bytes + bytes / 4;
    HIP_TRY(c, homs::dev_malloc(&c->ws.ptr, want), "hipMalloc(workspace)");
    c->ws.bytes = want;
    return HOMS_OK;
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch of homs_search_window_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends. Host code never passes the symbol
// itself to a kernel (on the host it is only a stand-in): the device address
// of each GPU's copy is taken once per device with hipGetSymbolAddress while
// that device is current, and that address is what the kernels get.
constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
__device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;  // by device ordinal; nullptr until looked up

// The device address of `scratch` on `device`, which must be current.
hipError_t scratch_address(int device, void** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)device >= g_scratch_addr.size()) g_scratch_addr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_addr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = ptr;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

// Per-call search scratch carved out of the workspace.
struct SearchScratch {
    int64_t* lo;
    int64_t* hi;
    uint64_t* keys;
    uint64_t* qk_a;
    uint64_t* qk_b;
    uint32_t* qp_a;
    uint32_t* qp_b;
    int64_t* tile_lo;
    int64_t* tile_hi;
    int32_t* qoff;  // per-query constants of the fp4 engine
    void* sort_tmp;
    size_t sort_bytes;
};

size_t search_scratch_bytes(int64_t nq, int tile)
{
    const int64_t nt = (nq + tile - 1) / tile;
    return 2 * al(nq * 8) + al(nq * 8) + 2 * al(nq * 8) + 2 * al(nq * 4) + 2 * al(nt * 8) +
           al(nq * 4) + homs::query_sort_temp_bytes(nq);
}

SearchScratch carve(void* base, int64_t nq, int tile)
{
    const int64_t nt = (nq + tile - 1) / tile;
    char* p = (char*)base;
    SearchScratch s{};
    s.lo = (int64_t*)p;
    p += al(nq * 8);
    s.hi = (int64_t*)p;
    p += al(nq * 8);
    s.keys = (uint64_t*)p;
    p += al(nq * 8);
    s.qk_a = (uint64_t*)p;
    p += al(nq * 8);
    s.qk_b = (uint64_t*)p;
    p += al(nq * 8);
    s.qp_a = (uint32_t*)p;
    p += al(nq * 4);
    s.qp_b = (uint32_t*)p;
    p += al(nq * 4);
    s.tile_lo = (int64_t*)p;
    p += al(nt * 8);
    s.tile_hi = (int64_t*)p;
    p += al(nt * 8);
    s.qoff = (int32_t*)p;
    p += al(nq * 4);
    s.sort_tmp = p;
    s.sort_bytes = homs::query_sort_temp_bytes(nq);
    return s;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Records an event on `s` for profiling (nullptr when profiling is off).
hipEvent_t prof_mark(homs_ctx* c, hipStream_t s)
{
    if (!c->prof.on) return nullptr;
    hipEvent_t e = nullptr;
    if (!c->prof.pool.empty()) {
        e = c->prof.pool.back();
        c->prof.pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return nullptr;
    }
    if (hipEventRecord(e, s) != hipSuccess) {
        c->prof.pool.push_back(e);
        return nullptr;
    }
    return e;
}

void prof_span(homs_ctx* c, hipEvent_t a, hipEvent_t b, int kind)
{
    if (a && b) c->prof.pending.push_back({a, b, kind});
}

}  // namespace

extern "C" {

homs_status homs_params_default(homs_params* p)
{
    if (!p) return fail(nullptr, HOMS_E_INVALID, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(homs_params);
    p->dim = 8192;
    p->n_levels = 16;
    p->top_n = 50;
    p->mz_min = 101.0;
    p->mz_max = 1500.0;
    p->bins_per_da = 20.0;
    p->noise_frac = 0.01;
    p->id_flips = 0;
    p->charge_match = 1;
    p->seed = 0;
    return HOMS_OK;
}

int64_t homs_num_bins(const homs_params* p)
{
    std::string why;
    if (!params_valid(p, &why)) return -1;
    return (int64_t)std::ceil((p->mz_max - p->mz_min) * p->bins_per_da);
}

const char* homs_status_string(homs_status s)
{
    switch (s) {
    case HOMS_OK: return "ok";
    case HOMS_E_INVALID: return "invalid argument";
    case HOMS_E_OOM: return "out of memory";
    case HOMS_E_DEVICE: return "device error";
    case HOMS_E_STATE: return "invalid state";
    case HOMS_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char* homs_last_error(const homs_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

homs_status homs_preprocess(const homs_params* p, int64_t n, const int64_t* h_offsets,
                            const double* h_mz, const double* h_intensity, int64_t* h_out_offsets,
                            int32_t* h_out_bin, uint8_t* h_out_level, int64_t* out_total,
                            int32_t n_threads)
{
    std::string why;
    if (!params_valid(p, &why)) return fail(nullptr, HOMS_E_INVALID, why);
    if (n < 0 || !h_offsets || !h_out_offsets || !out_total)
        return fail(nullptr, HOMS_E_INVALID, "n < 0 or NULL offsets/out_total");
    if (n > 0 && h_offsets[n] > 0 && (!h_mz || !h_intensity || !h_out_bin || !h_out_level))
        return fail(nullptr, HOMS_E_INVALID, "NULL peak arrays");
    homs::PreprocessParams pp{p->mz_min,      p->mz_max, p->bins_per_da, p->noise_frac,
                              p->top_n,       p->n_levels, homs_num_bins(p)};
    try {
        if (!homs::preprocess_spectra(pp, n, h_offsets, h_mz, h_intensity, h_out_offsets,
                                      h_out_bin, h_out_level, out_total, n_threads, &why))
            return fail(nullptr, HOMS_E_INVALID, why);
    } catch (const std::bad_alloc&) {
        return fail(nullptr, HOMS_E_OOM, "host allocation failed in preprocess");
    } catch (const std::exception& e) {
        return fail(nullptr, HOMS_E_INVALID, e.what());
    }
    return HOMS_OK;
}

homs_status homs_create(const homs_params* p, int32_t device, homs_ctx** out)
{
    std::string why;
    if (!out) return fail(nullptr, HOMS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!params_valid(p, &why)) return fail(nullptr, HOMS_E_INVALID, why);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
        return fail(nullptr, HOMS_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(nullptr, HOMS_E_INVALID, "device out of range");
    DeviceGuard g(device);
    if (!g.ok) return fail(nullptr, HOMS_E_DEVICE, "hipSetDevice failed");

    homs_ctx* c = new (std::nothrow) homs_ctx();
    if (!c) return fail(nullptr, HOMS_E_OOM, "host allocation failed");
    c->p = *p;
    if (c->p.id_flips == 0) c->p.id_flips = c->p.dim / 2;
    c->device = device;
    c->n_bins = homs_num_bins(p);
    c->words = p->dim / 32;

    std::vector<uint32_t> id, lv;
    try {
        id.resize((size_t)c->n_bins * c->words);
        lv.resize((size_t)p->n_levels * c->words);
    } catch (const std::bad_alloc&) {
        delete c;
        return fail(nullptr, HOMS_E_OOM, "host allocation failed (codebook)");
    }
    homs::generate_codebook(p->dim, (uint32_t)c->n_bins, p->n_levels, c->p.id_flips, p->seed,
                            p->encoding, id.data(), lv.data());
    hipError_t e = homs::dev_malloc(&c->d_id, id.size() * 4);
    if (e == hipSuccess) e = homs::dev_malloc(&c->d_level, lv.size() * 4);
    if (e == hipSuccess) e = homs::dev_malloc(&c->d_err, 256);
    if (e == hipSuccess) e = hipMemcpy(c->d_id, id.data(), id.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_level, lv.data(), lv.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->d_err, 0, 256);
    if (e == hipSuccess) e = scratch_address(device, &c->noalloc_scratch);
    if (e != hipSuccess) {
        std::string msg = std::string("context setup: ") + hipGetErrorString(e);
        homs_destroy(c);
        return fail(nullptr, e == hipErrorOutOfMemory ? HOMS_E_OOM : HOMS_E_DEVICE, msg);
    }
    *out = c;
    return HOMS_OK;
}

homs_status homs_generate_codebook(const homs_params* p, uint32_t* h_id, uint32_t* h_level)
{
    std::string why;
    if (!params_valid(p, &why)) return fail(nullptr, HOMS_E_INVALID, why);
    if (!h_id || !h_level) return fail(nullptr, HOMS_E_INVALID, "NULL output table");
    const uint32_t alpha = p->id_flips == 0 ? p->dim / 2 : p->id_flips;
    homs::generate_codebook(p->dim, (uint32_t)homs_num_bins(p), p->n_levels, alpha, p->seed,
                            p->encoding, h_id, h_level);
    return HOMS_OK;
}

void homs_destroy(homs_ctx* c)
{
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    free_library(c->lib);
    if (c->d_id) (void)hipFree(c->d_id);
    if (c->d_level) (void)hipFree(c->d_level);
    if (c->d_err) (void)hipFree(c->d_err);
    if (c->ws.ptr) (void)hipFree(c->ws.ptr);
    drop_graph(c);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (auto& sp : c->prof.pending) {
        c->prof.pool.push_back(sp.a);
        c->prof.pool.push_back(sp.b);
    }
    std::sort(c->prof.pool.begin(), c->prof.pool.end());
    c->prof.pool.erase(std::unique(c->prof.pool.begin(), c->prof.pool.end()), c->prof.pool.end());
    for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
    delete c;
}

homs_status homs_set_codebook(homs_ctx* c, const uint32_t* h_id, const uint32_t* h_level)
{
    if (homs_status s = usable(c)) return s;
    DeviceGuard g(c->device);
    if (h_id)
        HIP_TRY(c, hipMemcpy(c->d_id, h_id, (size_t)c->n_bins * c->words * 4, hipMemcpyHostToDevice),
                "hipMemcpy(id table)");
    if (h_level)
        HIP_TRY(c, hipMemcpy(c->d_level, h_level, (size_t)c->p.n_levels * c->words * 4,
                             hipMemcpyHostToDevice),
                "hipMemcpy(level table)");
    if (h_id || h_level) {
        c->lib_valid = false;
        drop_graph(c);
    }
    return HOMS_OK;
}

homs_status homs_get_codebook(homs_ctx* c, uint32_t* h_id, uint32_t* h_level)
{
    if (homs_status s = usable(c)) return s;
    DeviceGuard g(c->device);
    if (h_id)
        HIP_TRY(c, hipMemcpy(h_id, c->d_id, (size_t)c->n_bins * c->words * 4, hipMemcpyDeviceToHost),
                "hipMemcpy(id table)");
    if (h_level)
        HIP_TRY(c, hipMemcpy(h_level, c->d_level, (size_t)c->p.n_levels * c->words * 4,
                             hipMemcpyDeviceToHost),
                "hipMemcpy(level table)");
    return HOMS_OK;
}

homs_status homs_encode_queries(homs_ctx* c, int64_t n, const int64_t* d_offsets,
                                const int32_t* d_bin, const uint8_t* d_level, uint32_t* d_out,
                                void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "n must be in [0, 2^31)");
    if (n == 0) return HOMS_OK;
    if (!d_offsets || !d_bin || !d_level || !d_out)
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    if (!aligned16(d_out)) return fail(c, HOMS_E_INVALID, "d_out must be 16-byte aligned");
    DeviceGuard g(c->device);
    hipEvent_t e0 = prof_mark(c, (hipStream_t)stream);
    HIP_TRY(c, homs::launch_encode(c, n, d_offsets, d_bin, d_level, nullptr, d_out,
                                   (hipStream_t)stream),
            "encode kernel");
    prof_span(c, e0, prof_mark(c, (hipStream_t)stream), homs::kProfEncode);
    return HOMS_OK;
}

homs_status homs_encode_library(homs_ctx* c, int64_t n, const int64_t* d_offsets,
                                const int32_t* d_bin, const uint8_t* d_level, const double* d_pmz,
                                const int8_t* d_charge, void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "n must be in [0, 2^31)");
    if (n > 0 && (!d_offsets || !d_bin || !d_level || !d_pmz || !d_charge))
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(c, hipStreamSynchronize(s), "hipStreamSynchronize");
    free_library(c->lib);
    c->lib_valid = false;
    drop_graph(c);
    c->lib_gen += 1;
    if (n == 0) {
        c->lib_valid = true;
        return HOMS_OK;
    }
    homs::Library L;
    L.n = n;
    const size_t tmp_bytes = homs::library_sort_temp_bytes(n);
    void* tmp = nullptr;
    hipError_t e = homs::dev_malloc(&L.hv, (size_t)n * c->words * 4);
    if (e == hipSuccess) e = homs::dev_malloc(&L.pmz, (size_t)n * 8);
    if (e == hipSuccess) e = homs::dev_malloc(&L.charge, (size_t)n);
    // the MFMA epilogue reads library indices in groups past the last row
    const size_t orig_pad = (size_t)homs::search_mfma_row_pad();
    if (e == hipSuccess) e = homs::dev_malloc(&L.orig, ((size_t)n + orig_pad) * 4);
    if (e == hipSuccess) e = hipMemsetAsync(L.orig + n, 0, orig_pad * 4, s);
    if (e == hipSuccess) e = homs::dev_malloc(&L.slot, (size_t)n * 4);
    if (e == hipSuccess) e = homs::dev_malloc(&L.rowk, ((size_t)n + orig_pad) * 4);
    if (e == hipSuccess) e = homs::dev_malloc(&tmp, tmp_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_err, 0, 4, s);
    hipEvent_t e0 = e == hipSuccess ? prof_mark(c, s) : nullptr;
    if (e == hipSuccess)
        e = homs::launch_library_sort(n, d_pmz, d_charge, c->p.charge_match != 0, tmp, tmp_bytes,
                                      L.orig, L.pmz, L.charge, L.slot, s);
    hipEvent_t e1 = e == hipSuccess ? prof_mark(c, s) : nullptr;
    if (e == hipSuccess) e = homs::launch_encode(c, n, d_offsets, d_bin, d_level, L.slot, L.hv, s);
    hipEvent_t e2 = e == hipSuccess ? prof_mark(c, s) : nullptr;
    if (e == hipSuccess) e = homs::launch_fp4_row_consts(n, c->words, L.hv, L.rowk, s);
    prof_span(c, e0, e1, homs::kProfPrep);
    prof_span(c, e1, e2, homs::kProfEncode);
    uint32_t flags = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flags, c->d_err, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) {
        free_library(L);
        return hip_fail(c, e, "encode_library");
    }
    if (flags & homs::kErrRange) {
        free_library(L);
        (void)hipMemset(c->d_err, 0, 4);
        return fail(c, HOMS_E_INVALID, "a bin or level is out of range");
    }
    c->lib = L;
    c->lib_valid = true;
    c->lib_gen += 1;
    return HOMS_OK;
}

homs_status homs_library_size(const homs_ctx* c, int64_t* n)
{
    if (!c || !n) return fail(nullptr, HOMS_E_INVALID, "NULL argument");
    *n = c->lib_valid ? c->lib.n : 0;
    return HOMS_OK;
}

homs_status homs_library_export(homs_ctx* c, uint32_t* d_out, void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (c->lib.n == 0) return HOMS_OK;
    if (!d_out || !aligned16(d_out)) return fail(c, HOMS_E_INVALID, "d_out NULL or misaligned");
    DeviceGuard g(c->device);
    HIP_TRY(c, homs::launch_gather_rows(c->lib.n, c->words, c->lib.hv, c->lib.orig, d_out,
                                        (hipStream_t)stream),
            "export kernel");
    return HOMS_OK;
}

homs_status homs_library_order(homs_ctx* c, uint32_t* d_out_orig, void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (c->lib.n == 0) return HOMS_OK;
    if (!d_out_orig) return fail(c, HOMS_E_INVALID, "d_out_orig is NULL");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipMemcpyAsync(d_out_orig, c->lib.orig, (size_t)c->lib.n * 4,
                              hipMemcpyDeviceToDevice, (hipStream_t)stream),
            "hipMemcpyAsync(order)");
    return HOMS_OK;
}

homs_status homs_window_bounds(homs_ctx* c, int64_t nq, const double* d_q_pmz,
                               const int8_t* d_q_charge, const homs_window* win, int64_t* d_lo,
                               int64_t* d_hi, void* stream)
{
    if (homs_status s = usable(c)) return s;
    std::string why;
    if (!window_valid(win, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "nq out of range");
    if (nq == 0) return HOMS_OK;
    if (!d_q_pmz || !d_q_charge || !d_lo || !d_hi) return fail(c, HOMS_E_INVALID, "NULL pointer");
    DeviceGuard g(c->device);
    HIP_TRY(c, homs::launch_window_bounds(c, nq, d_q_pmz, d_q_charge, win->kind, win->value,
                                          nullptr, nullptr, d_lo, d_hi, (hipStream_t)stream),
            "window kernel");
    return HOMS_OK;
}

}  // extern "C"

namespace {

bool engine_valid(int32_t engine)
{
    return engine == HOMS_ENGINE_POPCOUNT || engine == HOMS_ENGINE_MFMA_I8 ||
           engine == HOMS_ENGINE_MFMA_F8 || engine == HOMS_ENGINE_MFMA_F4;
}

int engine_tile(int32_t engine)
{
    return engine == HOMS_ENGINE_POPCOUNT ? homs::search_popcount_tile()
                                          : homs::search_mfma_tile();
}

// The search of homs_search_window on validated arguments. The workspace must
// already hold search_scratch_bytes(nq, engine_tile(engine)) bytes; callers
// may keep their own buffers after that region.
homs_status run_search(homs_ctx* c, int64_t nq, const uint32_t* d_q_hv, const double* d_q_pmz,
                       const int8_t* d_q_charge, const homs_window* win, int32_t engine,
                       int64_t* d_out_idx, int32_t* d_out_dist, hipStream_t s,
                       void* scratch_base = nullptr, bool profile = true)
{
    const int tile = engine_tile(engine);
    SearchScratch w = carve(scratch_base ? scratch_base : c->ws.ptr, nq, tile);
    // without profiling no event is created or recorded
    auto mark = [&]() -> hipEvent_t { return profile ? prof_mark(c, s) : nullptr; };

    hipEvent_t e0 = mark();
    HIP_TRY(c, homs::launch_window_bounds(c, nq, d_q_pmz, d_q_charge, win->kind, win->value,
                                          nullptr, nullptr, w.lo, w.hi, s),
            "window kernel");
    uint32_t* qperm = nullptr;
    HIP_TRY(c, homs::launch_query_sort(nq, d_q_pmz, d_q_charge, c->p.charge_match != 0, w.sort_tmp,
                                       w.sort_bytes, w.qk_a, w.qk_b, w.qp_a, w.qp_b, &qperm, s),
            "query sort");
    HIP_TRY(c, homs::launch_tile_bounds(nq, qperm, w.lo, w.hi, tile, w.tile_lo, w.tile_hi, s),
            "tile bounds kernel");
    HIP_TRY(c, homs::launch_init_keys(nq, w.keys, s), "init keys kernel");
    homs::TilePlan plan;
    hipEvent_t e1 = mark();
    if (engine == HOMS_ENGINE_POPCOUNT)
        HIP_TRY(c, homs::launch_search_popcount(c, nq, d_q_hv, qperm, w.lo, w.hi, w.tile_lo,
                                                w.tile_hi, plan, w.keys, s),
                "search kernel");
    else
        HIP_TRY(c, homs::launch_search_mfma(c, engine == HOMS_ENGINE_MFMA_I8   ? 0
                                               : engine == HOMS_ENGINE_MFMA_F8 ? 1
                                                                               : 2,
                                            nq, d_q_hv,
                                            qperm, w.lo, w.hi, w.tile_lo, w.tile_hi, w.qoff, w.keys,
                                            s),
                "MFMA search kernel");
    hipEvent_t e2 = mark();
    HIP_TRY(c, homs::launch_finalize(nq, w.keys, d_out_idx, d_out_dist, s), "finalize kernel");
    hipEvent_t e3 = mark();
    prof_span(c, e0, e1, homs::kProfPrep);
    prof_span(c, e1, e2, homs::kProfSearch);
    prof_span(c, e2, e3, homs::kProfPrep);
    return HOMS_OK;
}

}  // namespace

extern "C" {

homs_status homs_search_window(homs_ctx* c, int64_t nq, const uint32_t* d_q_hv,
                               const double* d_q_pmz, const int8_t* d_q_charge,
                               const homs_window* win, int32_t engine, int64_t* d_out_idx,
                               int32_t* d_out_dist, void* stream)
{
    if (homs_status s = usable(c)) return s;
    std::string why;
    if (!window_valid(win, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!engine_valid(engine)) return fail(c, HOMS_E_INVALID, "unknown engine");
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "nq out of range");
    if (nq == 0) return HOMS_OK;
    if (!d_q_hv || !d_q_pmz || !d_q_charge || !d_out_idx || !d_out_dist)
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    if (!aligned16(d_q_hv)) return fail(c, HOMS_E_INVALID, "d_q_hv must be 16-byte aligned");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (homs_status st = ensure_workspace(c, search_scratch_bytes(nq, engine_tile(engine)), s))
        return st;
    return run_search(c, nq, d_q_hv, d_q_pmz, d_q_charge, win, engine, d_out_idx, d_out_dist, s);
}

homs_status homs_search_window_noalloc(homs_ctx* c, int64_t nq, const uint32_t* d_q_hv,
                                       const double* d_q_pmz, const int8_t* d_q_charge,
                                       const homs_window* win, int32_t engine,
                                       int64_t* d_out_idx, int32_t* d_out_dist, void* stream)
{
    if (homs_status s = usable(c)) return s;
    std::string why;
    if (!window_valid(win, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!engine_valid(engine)) return fail(c, HOMS_E_INVALID, "unknown engine");
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (nq < 0 || nq > HOMS_NOALLOC_MAX_QUERIES)
        return fail(c, HOMS_E_INVALID,
                    "nq out of range for homs_search_window_noalloc (at most " +
                        std::to_string(HOMS_NOALLOC_MAX_QUERIES) + " queries)");
    if (search_scratch_bytes(nq, engine_tile(engine)) > kNoAllocScratchBytes)
        return fail(c, HOMS_E_INVALID, "nq needs more than the static scratch holds");
    if (nq == 0) return HOMS_OK;
    if (!d_q_hv || !d_q_pmz || !d_q_charge || !d_out_idx || !d_out_dist)
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    if (!aligned16(d_q_hv)) return fail(c, HOMS_E_INVALID, "d_q_hv must be 16-byte aligned");
    if (!c->noalloc_scratch) return fail(c, HOMS_E_STATE, "static scratch not set up");
    DeviceGuard g(c->device);
    return run_search(c, nq, d_q_hv, d_q_pmz, d_q_charge, win, engine, d_out_idx, d_out_dist,
                      (hipStream_t)stream, c->noalloc_scratch, false);
}

homs_status homs_preprocess_device(homs_ctx* c, int64_t n, const int64_t* d_offsets,
                                   const double* d_mz, const double* d_intensity,
                                   int64_t* d_out_offsets, int32_t* d_out_bin,
                                   uint8_t* d_out_level, void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "n out of range");
    if (!d_offsets || !d_out_offsets) return fail(c, HOMS_E_INVALID, "NULL device pointer");
    if (n > 0 && (!d_mz || !d_intensity || !d_out_bin || !d_out_level))
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (homs_status st = ensure_workspace(c, homs::prep_device_scratch_bytes(n, c->p.top_n), s))
        return st;
    hipEvent_t e0 = prof_mark(c, s);
    HIP_TRY(c, homs::launch_preprocess_device(c, n, d_offsets, d_mz, d_intensity, d_out_offsets,
                                              d_out_bin, d_out_level, c->ws.ptr, s),
            "preprocess kernels");
    hipEvent_t e1 = prof_mark(c, s);
    prof_span(c, e0, e1, homs::kProfEncode);
    return HOMS_OK;
}

homs_status homs_cascade_search(homs_ctx* c, int64_t nq, const uint32_t* d_q_hv,
                                const double* d_q_pmz, const int8_t* d_q_charge,
                                const homs_window* narrow, const homs_window* wide,
                                int32_t engine, const uint8_t* d_lib_decoy, double fdr_level,
                                int64_t* d_out_idx, int32_t* d_out_dist, int8_t* d_out_stage,
                                double* d_out_qvalue, void* stream)
{
    if (homs_status s = usable(c)) return s;
    std::string why;
    if (!window_valid(narrow, &why)) return fail(c, HOMS_E_INVALID, "narrow: " + why);
    if (!window_valid(wide, &why)) return fail(c, HOMS_E_INVALID, "wide: " + why);
    if (!engine_valid(engine)) return fail(c, HOMS_E_INVALID, "unknown engine");
    if (!std::isfinite(fdr_level) || fdr_level < 0.0 || fdr_level > 1.0)
        return fail(c, HOMS_E_INVALID, "fdr_level must be in [0, 1]");
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "nq out of range");
    if (nq == 0) return HOMS_OK;
    if (!d_q_hv || !d_q_pmz || !d_q_charge || !d_lib_decoy || !d_out_idx || !d_out_dist ||
        !d_out_stage || !d_out_qvalue)
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    if (!aligned16(d_q_hv)) return fail(c, HOMS_E_INVALID, "d_q_hv must be 16-byte aligned");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t dim = c->words * 32;
    const size_t search_bytes = search_scratch_bytes(nq, engine_tile(engine));
    const size_t off = (search_bytes + 255) & ~(size_t)255;
    if (homs_status st = ensure_workspace(c, off + homs::cascade_scratch_bytes(nq, dim), s))
        return st;
    const homs::CascadeScratch w = homs::cascade_carve((char*)c->ws.ptr + off, nq, dim);

    // stage 1: standard search with the narrow window, FDR over all its PSMs
    if (homs_status st = run_search(c, nq, d_q_hv, d_q_pmz, d_q_charge, narrow, engine,
                                    d_out_idx, d_out_dist, s))
        return st;
    hipEvent_t e0 = prof_mark(c, s);
    HIP_TRY(c, homs::launch_fdr_stage(0, nq, dim, d_out_idx, d_out_dist, d_lib_decoy, fdr_level,
                                      w, d_out_stage, d_out_qvalue, nullptr, nullptr, s),
            "FDR kernels (narrow stage)");
    HIP_TRY(c, homs::launch_mask_identified(nq, d_q_pmz, d_out_stage, w.pmz2, s),
            "mask kernel");
    hipEvent_t e1 = prof_mark(c, s);
    prof_span(c, e0, e1, homs::kProfPrep);
    // stage 2: open search of the queries not identified, FDR over their PSMs
    if (homs_status st = run_search(c, nq, d_q_hv, w.pmz2, d_q_charge, wide, engine, w.idx2,
                                    w.dist2, s))
        return st;
    hipEvent_t e2 = prof_mark(c, s);
    HIP_TRY(c, homs::launch_fdr_stage(1, nq, dim, w.idx2, w.dist2, d_lib_decoy, fdr_level, w,
                                      d_out_stage, d_out_qvalue, d_out_idx, d_out_dist, s),
            "FDR kernels (open stage)");
    hipEvent_t e3 = prof_mark(c, s);
    prof_span(c, e2, e3, homs::kProfPrep);
    return HOMS_OK;
}

}  // extern "C"

namespace {

bool batched_config_valid(const homs_batched_config* b, std::string* why)
{
    if (!b) {
        *why = "config is NULL";
        return false;
    }
    if (b->chunk_rows < 32 || b->chunk_rows > (1u << 24)) {
        *why = "chunk_rows must be in [32, 2^24]";
        return false;
    }
    if (b->narrow_group < 4 || b->narrow_group % 4 != 0 || b->narrow_group > 4096) {
        *why = "narrow_group must be a multiple of 4 in [4, 4096]";
        return false;
    }
    if (b->grid < 1 || b->grid > 65535) {
        *why = "grid must be in [1, 65535]";
        return false;
    }
    if (!std::isfinite(b->bucket_da) || !(b->bucket_da > 0.0)) {
        *why = "bucket_da must be finite and > 0";
        return false;
    }
    if (b->engine != HOMS_ENGINE_POPCOUNT && b->engine != HOMS_ENGINE_MFMA_F8 &&
        b->engine != HOMS_ENGINE_MFMA_F4) {
        *why = "engine must be HOMS_ENGINE_POPCOUNT, HOMS_ENGINE_MFMA_F8 or HOMS_ENGINE_MFMA_F4";
        return false;
    }
    return true;
}

homs::BatchedConfig to_internal(const homs_batched_config& b)
{
    homs::BatchedConfig c;
    c.narrow_max = b.narrow_max;
    c.chunk_rows = b.chunk_rows;
    c.narrow_group = b.narrow_group;
    c.grid = b.grid;
    c.bucket_da = b.bucket_da;
    c.engine = b.engine;
    return c;
}

homs_batched_config to_public(const homs::BatchedConfig& c)
{
    homs_batched_config b;
    b.narrow_max = c.narrow_max;
    b.chunk_rows = c.chunk_rows;
    b.narrow_group = c.narrow_group;
    b.grid = c.grid;
    b.bucket_da = c.bucket_da;
    b.engine = c.engine;
    return b;
}

void drop_graph(homs_ctx* c)
{
    if (c->graph.exec) (void)hipGraphExecDestroy(c->graph.exec);
    if (c->graph.graph) (void)hipGraphDestroy(c->graph.graph);
    c->graph = homs::GraphCache{};
}

homs_status batched_check(homs_ctx* c, int64_t nq, const uint32_t* q_hv, const double* q_pmz,
                          const int8_t* q_charge, const int8_t* kinds, const double* values,
                          int64_t* out_idx, int32_t* out_dist)
{
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "nq out of range");
    if (nq == 0) return HOMS_OK;
    if (!q_hv || !q_pmz || !q_charge || !kinds || !values || !out_idx || !out_dist)
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    if (!aligned16(q_hv)) return fail(c, HOMS_E_INVALID, "d_q_hv must be 16-byte aligned");
    return HOMS_OK;
}

// One batched search, eager or through the cached graph.
homs_status run_batched(homs_ctx* c, const homs::BatchedConfig& cfg, int64_t nq,
                        const uint32_t* q_hv, const double* q_pmz, const int8_t* q_charge,
                        const int8_t* kinds, const double* values, int64_t* out_idx,
                        int32_t* out_dist, bool use_graph, hipStream_t s)
{
    if (homs_status st = ensure_workspace(c, homs::batched_scratch_bytes(nq), s)) return st;
    hipEvent_t e0 = prof_mark(c, s);
    if (!use_graph) {
        HIP_TRY(c, homs::launch_search_batched(c, cfg, c->ws.ptr, nq, q_hv, q_pmz, q_charge, kinds,
                                               values, out_idx, out_dist, s),
                "batched search");
    } else {
        std::vector<uintptr_t> key = {
            (uintptr_t)nq,        (uintptr_t)q_hv,       (uintptr_t)q_pmz,
            (uintptr_t)q_charge,  (uintptr_t)kinds,      (uintptr_t)values,
            (uintptr_t)out_idx,   (uintptr_t)out_dist,   (uintptr_t)c->ws.ptr,
            (uintptr_t)c->lib.hv, (uintptr_t)c->lib.n,   (uintptr_t)cfg.narrow_max,
            (uintptr_t)cfg.chunk_rows, (uintptr_t)cfg.narrow_group, (uintptr_t)cfg.grid,
            (uintptr_t)(cfg.bucket_da * 1e9), (uintptr_t)cfg.engine};
        if (!c->graph.exec || c->graph.key != key) {
            drop_graph(c);
            if (!c->capture_stream)
                HIP_TRY(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking),
                        "hipStreamCreateWithFlags");
            HIP_TRY(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal),
                    "hipStreamBeginCapture");
            hipError_t le = homs::launch_search_batched(c, cfg, c->ws.ptr, nq, q_hv, q_pmz,
                                                        q_charge, kinds, values, out_idx,
                                                        out_dist, c->capture_stream);
            hipGraph_t graph = nullptr;
            hipError_t ce = hipStreamEndCapture(c->capture_stream, &graph);
            if (le != hipSuccess || ce != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return hip_fail(c, le != hipSuccess ? le : ce, "capturing the batched search");
            }
            hipGraphExec_t exec = nullptr;
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return hip_fail(c, ie, "hipGraphInstantiate");
            }
            c->graph.graph = graph;
            c->graph.exec = exec;
            c->graph.key = key;
        }
        HIP_TRY(c, hipGraphLaunch(c->graph.exec, s), "hipGraphLaunch");
    }
    prof_span(c, e0, prof_mark(c, s), homs::kProfSearch);
    return HOMS_OK;
}

}  // namespace

extern "C" {

homs_status homs_batched_config_get(const homs_ctx* c, homs_batched_config* out)
{
    if (!c || !out) return fail(nullptr, HOMS_E_INVALID, "NULL argument");
    *out = to_public(c->batched);
    return HOMS_OK;
}

homs_status homs_batched_config_set(homs_ctx* c, const homs_batched_config* cfg)
{
    if (homs_status s = usable(c)) return s;
    std::string why;
    if (!batched_config_valid(cfg, &why)) return fail(c, HOMS_E_INVALID, why);
    c->batched = to_internal(*cfg);
    return HOMS_OK;
}

homs_status homs_search_batched(homs_ctx* c, int64_t nq, const uint32_t* d_q_hv,
                                const double* d_q_pmz, const int8_t* d_q_charge,
                                const int8_t* d_kinds, const double* d_values,
                                int64_t* d_out_idx, int32_t* d_out_dist, int32_t use_graph,
                                void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (homs_status s = batched_check(c, nq, d_q_hv, d_q_pmz, d_q_charge, d_kinds, d_values,
                                      d_out_idx, d_out_dist))
        return s;
    if (nq == 0) return HOMS_OK;
    DeviceGuard g(c->device);
    return run_batched(c, c->batched, nq, d_q_hv, d_q_pmz, d_q_charge, d_kinds, d_values,
                       d_out_idx, d_out_dist, use_graph != 0, (hipStream_t)stream);
}

homs_status homs_autotune_batched(homs_ctx* c, int64_t nq, const uint32_t* d_q_hv,
                                  const double* d_q_pmz, const int8_t* d_q_charge,
                                  const int8_t* d_kinds, const double* d_values,
                                  int64_t* d_out_idx, int32_t* d_out_dist, int32_t reps,
                                  homs_batched_config* best, double* best_ms, void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (homs_status s = batched_check(c, nq, d_q_hv, d_q_pmz, d_q_charge, d_kinds, d_values,
                                      d_out_idx, d_out_dist))
        return s;
    if (reps < 1 || reps > 1000) return fail(c, HOMS_E_INVALID, "reps must be in [1, 1000]");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const bool prof = c->prof.on;
    c->prof.on = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    HIP_TRY(c, hipEventCreate(&t0), "hipEventCreate");
    HIP_TRY(c, hipEventCreate(&t1), "hipEventCreate");
    auto time_cfg = [&](const homs::BatchedConfig& cfg, double* ms) -> homs_status {
        if (nq == 0) {
            *ms = 0.0;
            return HOMS_OK;
        }
        if (homs_status st = run_batched(c, cfg, nq, d_q_hv, d_q_pmz, d_q_charge, d_kinds,
                                         d_values, d_out_idx, d_out_dist, false, s))
            return st;
        HIP_TRY(c, hipEventRecord(t0, s), "hipEventRecord");
        for (int r = 0; r < reps; ++r)
            if (homs_status st = run_batched(c, cfg, nq, d_q_hv, d_q_pmz, d_q_charge, d_kinds,
                                             d_values, d_out_idx, d_out_dist, false, s))
                return st;
        HIP_TRY(c, hipEventRecord(t1, s), "hipEventRecord");
        HIP_TRY(c, hipEventSynchronize(t1), "hipEventSynchronize");
        float f = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&f, t0, t1), "hipEventElapsedTime");
        *ms = (double)f / reps;
        return HOMS_OK;
    };
    homs::BatchedConfig cur = c->batched;
    double cur_ms = 0.0;
    homs_status st = time_cfg(cur, &cur_ms);
    const uint32_t chunks[] = {1024, 2048, 4096, 8192};
    const uint32_t grids[] = {512, 1024, 2048, 4096};
    const uint32_t narrows[] = {256, 1024, 4096};
    const uint32_t groups[] = {16, 32, 64};
    const uint32_t engines[] = {HOMS_ENGINE_POPCOUNT, HOMS_ENGINE_MFMA_F8, HOMS_ENGINE_MFMA_F4};
    auto sweep = [&](auto set, const auto& vals) {
        for (size_t i = 0; i < sizeof(vals) / sizeof(vals[0]) && st == HOMS_OK; ++i) {
            homs::BatchedConfig cand = cur;
            set(cand, vals[i]);
            double ms = 0.0;
            st = time_cfg(cand, &ms);
            if (st == HOMS_OK && ms < cur_ms) {
                cur = cand;
                cur_ms = ms;
            }
        }
    };
    sweep([](homs::BatchedConfig& b, uint32_t v) { b.engine = (int32_t)v; }, engines);
    sweep([](homs::BatchedConfig& b, uint32_t v) { b.chunk_rows = v; }, chunks);
    sweep([](homs::BatchedConfig& b, uint32_t v) { b.grid = v; }, grids);
    sweep([](homs::BatchedConfig& b, uint32_t v) { b.narrow_max = v; }, narrows);
    sweep([](homs::BatchedConfig& b, uint32_t v) { b.narrow_group = v; }, groups);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    c->prof.on = prof;
    if (st != HOMS_OK) return st;
    c->batched = cur;
    if (best) *best = to_public(cur);
    if (best_ms) *best_ms = cur_ms;
    return HOMS_OK;
}

homs_status homs_debug_distances(homs_ctx* c, int64_t nq, const uint32_t* d_q_hv,
                                 const double* d_q_pmz, const int8_t* d_q_charge,
                                 const homs_window* win, const int64_t* d_row_off,
                                 int64_t* d_out_idx, int32_t* d_out_dist, void* stream)
{
    if (homs_status s = usable(c)) return s;
    std::string why;
    if (!window_valid(win, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "nq out of range");
    if (nq == 0) return HOMS_OK;
    if (!d_q_hv || !d_q_pmz || !d_q_charge || !d_row_off || !d_out_idx || !d_out_dist)
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const int tile = homs::search_popcount_tile();
    if (homs_status st = ensure_workspace(c, search_scratch_bytes(nq, tile), s)) return st;
    SearchScratch w = carve(c->ws.ptr, nq, tile);
    HIP_TRY(c, homs::launch_window_bounds(c, nq, d_q_pmz, d_q_charge, win->kind, win->value,
                                          nullptr, nullptr, w.lo, w.hi, s),
            "window kernel");
    HIP_TRY(c, homs::launch_debug_distances(c, nq, d_q_hv, w.lo, w.hi, d_row_off, d_out_idx,
                                            d_out_dist, s),
            "debug distances kernel");
    return HOMS_OK;
}

homs_status homs_device_errors(homs_ctx* c, uint32_t* flags, void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (!flags) return fail(c, HOMS_E_INVALID, "flags is NULL");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    uint32_t f = 0;
    HIP_TRY(c, hipMemcpyAsync(&f, c->d_err, 4, hipMemcpyDeviceToHost, s), "read error flags");
    HIP_TRY(c, hipStreamSynchronize(s), "hipStreamSynchronize");
    HIP_TRY(c, hipMemsetAsync(c->d_err, 0, 4, s), "clear error flags");
    HIP_TRY(c, hipStreamSynchronize(s), "hipStreamSynchronize");
    *flags = f;
    return HOMS_OK;
}

homs_status homs_profile_enable(homs_ctx* c, int32_t enable)
{
    if (homs_status s = usable(c)) return s;
    c->prof.on = enable != 0;
    return HOMS_OK;
}

homs_status homs_profile_read(homs_ctx* c, homs_profile* out)
{
    if (homs_status s = usable(c)) return s;
    if (!out) return fail(c, HOMS_E_INVALID, "out is NULL");
    DeviceGuard g(c->device);
    for (auto& sp : c->prof.pending) {
        float ms = 0.f;
        HIP_TRY(c, hipEventSynchronize(sp.b), "hipEventSynchronize");
        HIP_TRY(c, hipEventElapsedTime(&ms, sp.a, sp.b), "hipEventElapsedTime");
        c->prof.ms[sp.kind] += ms;
        c->prof.launches[sp.kind] += 1;
    }
    // spans share their boundary events; return each event to the pool once
    std::vector<hipEvent_t> seen;
    for (auto& sp : c->prof.pending)
        for (hipEvent_t e : {sp.a, sp.b})
            if (std::find(seen.begin(), seen.end(), e) == seen.end()) seen.push_back(e);
    for (hipEvent_t e : seen) c->prof.pool.push_back(e);
    c->prof.pending.clear();
    out->search_ms = c->prof.ms[homs::kProfSearch];
    out->encode_ms = c->prof.ms[homs::kProfEncode];
    out->prep_ms = c->prof.ms[homs::kProfPrep];
    out->search_launches = c->prof.launches[homs::kProfSearch];
    out->encode_launches = c->prof.launches[homs::kProfEncode];
    out->score_ms = c->prof.ms[homs::kProfScore];
    out->score_launches = c->prof.launches[homs::kProfScore];
    for (int k = 0; k < 4; ++k) {
        c->prof.ms[k] = 0;
        c->prof.launches[k] = 0;
    }
    return HOMS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned shortlist

namespace {

homs_status model_usable(homs_model* m)
{
    if (!m) return fail(nullptr, HOMS_E_INVALID, "model is NULL");
    if (homs_status s = usable(m->ctx)) return s;
    return HOMS_OK;
}

homs_status model_copy_weights(homs_model* m, const float* W1, const float* b1, const float* W2,
                               const float* b2)
{
    homs_ctx* c = m->ctx;
    const size_t n1 = (size_t)m->H * m->D, n2 = (size_t)m->E * m->H;
    HIP_TRY(c, hipMemcpy(m->W1, W1, n1 * 4, hipMemcpyHostToDevice), "hipMemcpy(W1)");
    HIP_TRY(c, hipMemcpy(m->b1, b1, (size_t)m->H * 4, hipMemcpyHostToDevice), "hipMemcpy(b1)");
    HIP_TRY(c, hipMemcpy(m->W2, W2, n2 * 4, hipMemcpyHostToDevice), "hipMemcpy(W2)");
    HIP_TRY(c, hipMemcpy(m->b2, b2, (size_t)m->E * 4, hipMemcpyHostToDevice), "hipMemcpy(b2)");
    for (void* p : {(void*)m->mW1, (void*)m->vW1, (void*)m->mW2, (void*)m->vW2})
        HIP_TRY(c, hipMemset(p, 0, (p == m->mW1 || p == m->vW1 ? n1 : n2) * 4), "hipMemset");
    HIP_TRY(c, hipMemset(m->mb1, 0, (size_t)m->H * 4), "hipMemset");
    HIP_TRY(c, hipMemset(m->vb1, 0, (size_t)m->H * 4), "hipMemset");
    HIP_TRY(c, hipMemset(m->mb2, 0, (size_t)m->E * 4), "hipMemset");
    HIP_TRY(c, hipMemset(m->vb2, 0, (size_t)m->E * 4), "hipMemset");
    HIP_TRY(c, homs::model_refresh_bf16(m, nullptr), "weight conversion kernels");
    HIP_TRY(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
    m->step = 0;
    m->weights_gen += 1;
    return HOMS_OK;
}

bool pairs_valid(int32_t batch, const uint32_t* q, const uint32_t* r, std::string* why)
{
    if (batch < 32 || batch > 16384 || batch % 32 != 0) {
        *why = "batch must be a multiple of 32 in [32, 16384]";
        return false;
    }
    if (!q || !r || !aligned16(q) || !aligned16(r)) {
        *why = "pair rows must be non-NULL and 16-byte aligned";
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

homs_status homs_model_create(homs_ctx* c, int32_t hidden, int32_t embed, const float* h_W1,
                              const float* h_b1, const float* h_W2, const float* h_b2,
                              homs_model** out)
{
    if (!out) return fail(nullptr, HOMS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (homs_status s = usable(c)) return s;
    if (hidden < 32 || hidden > 8192 || hidden % 32 != 0 || embed < 32 || embed > 4096 ||
        embed % 32 != 0)
        return fail(c, HOMS_E_INVALID, "hidden and embed must be multiples of 32 (hidden <= 8192, "
                                       "embed <= 4096)");
    if (!h_W1 || !h_b1 || !h_W2 || !h_b2) return fail(c, HOMS_E_INVALID, "NULL weight array");
    DeviceGuard g(c->device);
    homs_model* m = new (std::nothrow) homs_model();
    if (!m) return fail(c, HOMS_E_OOM, "host allocation failed");
    m->ctx = c;
    m->D = (int)c->p.dim;
    m->H = hidden;
    m->E = embed;
    hipError_t e = homs::model_alloc(m);
    if (e != hipSuccess) {
        homs::model_free(m);
        delete m;
        return hip_fail(c, e, "model allocation");
    }
    if (homs_status s = model_copy_weights(m, h_W1, h_b1, h_W2, h_b2)) {
        homs::model_free(m);
        delete m;
        return s;
    }
    *out = m;
    return HOMS_OK;
}

void homs_model_destroy(homs_model* m)
{
    if (!m) return;
    DeviceGuard g(m->ctx->device);
    (void)hipDeviceSynchronize();
    homs::model_free(m);
    delete m;
}

homs_status homs_model_set_weights(homs_model* m, const float* h_W1, const float* h_b1,
                                   const float* h_W2, const float* h_b2)
{
    if (homs_status s = model_usable(m)) return s;
    if (!h_W1 || !h_b1 || !h_W2 || !h_b2) return fail(m->ctx, HOMS_E_INVALID, "NULL weight array");
    DeviceGuard g(m->ctx->device);
    return model_copy_weights(m, h_W1, h_b1, h_W2, h_b2);
}

homs_status homs_model_get_weights(homs_model* m, float* h_W1, float* h_b1, float* h_W2,
                                   float* h_b2)
{
    if (homs_status s = model_usable(m)) return s;
    homs_ctx* c = m->ctx;
    DeviceGuard g(c->device);
    HIP_TRY(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
    const size_t n1 = (size_t)m->H * m->D, n2 = (size_t)m->E * m->H;
    if (h_W1) HIP_TRY(c, hipMemcpy(h_W1, m->W1, n1 * 4, hipMemcpyDeviceToHost), "hipMemcpy(W1)");
    if (h_b1)
        HIP_TRY(c, hipMemcpy(h_b1, m->b1, (size_t)m->H * 4, hipMemcpyDeviceToHost), "hipMemcpy(b1)");
    if (h_W2) HIP_TRY(c, hipMemcpy(h_W2, m->W2, n2 * 4, hipMemcpyDeviceToHost), "hipMemcpy(W2)");
    if (h_b2)
        HIP_TRY(c, hipMemcpy(h_b2, m->b2, (size_t)m->E * 4, hipMemcpyDeviceToHost), "hipMemcpy(b2)");
    return HOMS_OK;
}

homs_status homs_model_embed(homs_model* m, int64_t n, const uint32_t* d_hv, float* d_out,
                             void* stream)
{
    if (homs_status s = model_usable(m)) return s;
    homs_ctx* c = m->ctx;
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "n out of range");
    if (n == 0) return HOMS_OK;
    if (!d_hv || !d_out) return fail(c, HOMS_E_INVALID, "NULL device pointer");
    DeviceGuard g(c->device);
    HIP_TRY(c, homs::model_embed(m, n, d_hv, d_out, nullptr, nullptr, (hipStream_t)stream),
            "embedding kernels");
    return HOMS_OK;
}

homs_status homs_model_gradients(homs_model* m, int32_t batch, const uint32_t* d_q_hv,
                                 const uint32_t* d_r_hv, float tau, float* h_loss, float* h_gW1,
                                 float* h_gb1, float* h_gW2, float* h_gb2, void* stream)
{
    if (homs_status s = model_usable(m)) return s;
    homs_ctx* c = m->ctx;
    std::string why;
    if (!pairs_valid(batch, d_q_hv, d_r_hv, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!(tau > 0.f) || !std::isfinite(tau)) return fail(c, HOMS_E_INVALID, "tau must be > 0");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    float* d_loss = nullptr;
    HIP_TRY(c, homs::dev_malloc(&d_loss, 256), "hipMalloc(loss)");
    hipError_t e = homs::model_step(m, batch, d_q_hv, d_r_hv, tau, 0.f, false, d_loss, s);
    float loss = 0.f;
    if (e == hipSuccess) e = hipMemcpyAsync(&loss, d_loss, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_loss);
    if (e != hipSuccess) return hip_fail(c, e, "training kernels");
    const size_t n1 = (size_t)m->H * m->D, n2 = (size_t)m->E * m->H;
    if (h_loss) *h_loss = loss;
    if (h_gW1) HIP_TRY(c, hipMemcpy(h_gW1, m->gW1, n1 * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    if (h_gb1) HIP_TRY(c, hipMemcpy(h_gb1, m->gb1, (size_t)m->H * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    if (h_gW2) HIP_TRY(c, hipMemcpy(h_gW2, m->gW2, n2 * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    if (h_gb2) HIP_TRY(c, hipMemcpy(h_gb2, m->gb2, (size_t)m->E * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    return HOMS_OK;
}

homs_status homs_model_train_step(homs_model* m, int32_t batch, const uint32_t* d_q_hv,
                                  const uint32_t* d_r_hv, float tau, float lr, float* d_loss,
                                  void* stream)
{
    if (homs_status s = model_usable(m)) return s;
    homs_ctx* c = m->ctx;
    std::string why;
    if (!pairs_valid(batch, d_q_hv, d_r_hv, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!(tau > 0.f) || !std::isfinite(tau)) return fail(c, HOMS_E_INVALID, "tau must be > 0");
    if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(c, HOMS_E_INVALID, "lr must be >= 0");
    if (!d_loss) return fail(c, HOMS_E_INVALID, "d_loss is NULL");
    DeviceGuard g(c->device);
    HIP_TRY(c, homs::model_step(m, batch, d_q_hv, d_r_hv, tau, lr, true, d_loss,
                                (hipStream_t)stream),
            "training kernels");
    m->weights_gen += 1;
    return HOMS_OK;
}

homs_status homs_train_config_default(homs_train_config* cfg)
{
    if (!cfg) return fail(nullptr, HOMS_E_INVALID, "cfg is NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->struct_size = sizeof(homs_train_config);
    cfg->epochs = 2;
    cfg->batch = 1024;
    cfg->lr = 3e-5f;
    cfg->tau = 0.02f;
    cfg->seed = 0;
    return HOMS_OK;
}

homs_status homs_model_train(homs_model* m, int64_t n, const uint32_t* d_q_hv,
                             const int64_t* d_target_idx, const homs_train_config* cfg,
                             float* d_losses, int64_t* out_steps, void* stream)
{
    if (homs_status s = model_usable(m)) return s;
    homs_ctx* c = m->ctx;
    if (!out_steps) return fail(c, HOMS_E_INVALID, "out_steps is NULL");
    *out_steps = 0;
    if (!cfg || cfg->struct_size != sizeof(homs_train_config))
        return fail(c, HOMS_E_INVALID, "cfg is NULL or cfg.struct_size != sizeof(homs_train_config)");
    if (cfg->epochs < 1 || cfg->epochs > 1000)
        return fail(c, HOMS_E_INVALID, "epochs must be in [1, 1000]");
    if (cfg->batch < 32 || cfg->batch > 16384 || cfg->batch % 32 != 0)
        return fail(c, HOMS_E_INVALID, "batch must be a multiple of 32 in [32, 16384]");
    if (!(cfg->tau > 0.f) || !std::isfinite(cfg->tau))
        return fail(c, HOMS_E_INVALID, "tau must be > 0");
    if (!(cfg->lr >= 0.f) || !std::isfinite(cfg->lr))
        return fail(c, HOMS_E_INVALID, "lr must be >= 0");
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "n out of range");
    if (n > 0 && (!d_q_hv || !d_target_idx))
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    if (d_q_hv && !aligned16(d_q_hv)) return fail(c, HOMS_E_INVALID, "d_q_hv must be 16-byte aligned");
    if (n == 0 || c->lib.n == 0) return HOMS_OK;
    DeviceGuard g(c->device);
    int64_t steps = 0;
    hipError_t e = homs::model_train(m, n, d_q_hv, d_target_idx, cfg->epochs, cfg->batch, cfg->lr,
                                     cfg->tau, cfg->seed, d_losses, &steps, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "training kernels");
    if (steps > 0) m->weights_gen += 1;
    *out_steps = steps;
    return HOMS_OK;
}

homs_status homs_model_embed_library(homs_model* m, void* stream)
{
    if (homs_status s = model_usable(m)) return s;
    homs_ctx* c = m->ctx;
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = c->lib.n;
    m->lib_emb_valid = false;
    if (m->lib_emb_n < n) {
        HIP_TRY(c, hipStreamSynchronize(s), "hipStreamSynchronize");
        if (m->lib_emb) (void)hipFree(m->lib_emb);
        if (m->lib_emb8) (void)hipFree(m->lib_emb8);
        m->lib_emb = nullptr;
        m->lib_emb8 = nullptr;
        m->lib_emb_n = 0;
        const size_t rows = (size_t)std::max<int64_t>(n, 1);
        HIP_TRY(c, homs::dev_malloc(&m->lib_emb, rows * m->E * 2),
                "hipMalloc(library embeddings)");
        HIP_TRY(c, homs::dev_malloc(&m->lib_emb8, rows * m->E),
                "hipMalloc(library embeddings)");
        m->lib_emb_n = n;
    }
    if (n > 0)
        HIP_TRY(c, homs::model_embed(m, n, c->lib.hv, nullptr, m->lib_emb, m->lib_emb8, s),
                "embedding kernels");
    m->lib_emb_lib_gen = c->lib_gen;
    m->lib_emb_w_gen = m->weights_gen;
    m->lib_emb_valid = true;
    return HOMS_OK;
}

homs_status homs_model_library_embeddings(homs_model* m, uint8_t* d_out_fp8, uint16_t* d_out_bf16,
                                          void* stream)
{
    if (homs_status s = model_usable(m)) return s;
    homs_ctx* c = m->ctx;
    if (!m->lib_emb_valid) return fail(c, HOMS_E_STATE, "no library embeddings");
    const size_t n = (size_t)c->lib.n * m->E;
    if (n == 0) return HOMS_OK;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (d_out_fp8)
        HIP_TRY(c, hipMemcpyAsync(d_out_fp8, m->lib_emb8, n, hipMemcpyDeviceToDevice, s),
                "hipMemcpyAsync(embeddings)");
    if (d_out_bf16)
        HIP_TRY(c, hipMemcpyAsync(d_out_bf16, m->lib_emb, n * 2, hipMemcpyDeviceToDevice, s),
                "hipMemcpyAsync(embeddings)");
    return HOMS_OK;
}

homs_status homs_search_learned(homs_ctx* c, homs_model* m, int64_t nq, const uint32_t* d_q_hv,
                                const double* d_q_pmz, const int8_t* d_q_charge,
                                const homs_window* win, int32_t k, int64_t* d_out_idx,
                                int32_t* d_out_dist, uint8_t* d_out_fallback,
                                int64_t* d_out_shortlist, void* stream)
{
    if (homs_status s = usable(c)) return s;
    if (!m || m->ctx != c) return fail(c, HOMS_E_INVALID, "model is NULL or of another context");
    std::string why;
    if (!window_valid(win, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    if (!m->lib_emb_valid || m->lib_emb_lib_gen != c->lib_gen || m->lib_emb_w_gen != m->weights_gen)
        return fail(c, HOMS_E_STATE, "library embeddings are missing or stale "
                                     "(call homs_model_embed_library)");
    if (!homs::learned_search_supports(m->E))
        return fail(c, HOMS_E_UNSUPPORTED, "the shortlist search takes embed = 64, 128 or 256");
    if (k < 1 || k > homs::learned_max_k())
        return fail(c, HOMS_E_INVALID,
                    "k must be in [1, " + std::to_string(homs::learned_max_k()) + "]");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(c, HOMS_E_INVALID, "nq out of range");
    if (nq == 0) return HOMS_OK;
    if (!d_q_hv || !d_q_pmz || !d_q_charge || !d_out_idx || !d_out_dist || !d_out_fallback)
        return fail(c, HOMS_E_INVALID, "NULL device pointer");
    if (!aligned16(d_q_hv)) return fail(c, HOMS_E_INVALID, "d_q_hv must be 16-byte aligned");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const int tile = homs::search_popcount_tile();
    homs::LearnedScratchPlan plan;
    const size_t base = search_scratch_bytes(nq, tile);
    const size_t extra = al(homs::fallback_scratch_bytes(nq)) + al(nq * (size_t)m->E * 2) +
                         al(nq * (size_t)m->E) +
                         (d_out_shortlist ? 0 : al(nq * (size_t)k * 8)) +
                         homs::learned_scratch_bytes(nq, m->E, &plan);
    if (homs_status st = ensure_workspace(c, base + extra, s)) return st;
    SearchScratch w = carve(c->ws.ptr, nq, tile);
    char* p = (char*)c->ws.ptr + base;
    void* fb_scratch = p;
    p += al(homs::fallback_scratch_bytes(nq));
    uint16_t* q_emb = (uint16_t*)p;
    p += al(nq * (size_t)m->E * 2);
    uint8_t* q_emb8 = (uint8_t*)p;
    p += al(nq * (size_t)m->E);
    int64_t* shortlist = d_out_shortlist;
    if (!shortlist) {
        shortlist = (int64_t*)p;
        p += al(nq * (size_t)k * 8);
    }
    void* lscratch = p;

    hipEvent_t e0 = prof_mark(c, s);
    HIP_TRY(c, homs::launch_window_bounds(c, nq, d_q_pmz, d_q_charge, win->kind, win->value,
                                          nullptr, nullptr, w.lo, w.hi, s),
            "window kernel");
    uint32_t* qperm = nullptr;
    HIP_TRY(c, homs::launch_query_sort(nq, d_q_pmz, d_q_charge, c->p.charge_match != 0, w.sort_tmp,
                                       w.sort_bytes, w.qk_a, w.qk_b, w.qp_a, w.qp_b, &qperm, s),
            "query sort");
    HIP_TRY(c, homs::launch_init_keys(nq, w.keys, s), "init keys kernel");
    HIP_TRY(c, homs::model_embed(m, nq, d_q_hv, nullptr, q_emb, q_emb8, s), "embedding kernels");
    hipEvent_t e1 = prof_mark(c, s);
    homs::SpanHook hook;
    if (c->prof.on) {
        hook.user = c;
        hook.mark = [](void* u, hipStream_t st) { return prof_mark((homs_ctx*)u, st); };
        hook.span = [](void* u, hipEvent_t a, hipEvent_t b) {
            prof_span((homs_ctx*)u, a, b, homs::kProfScore);
        };
    }
    HIP_TRY(c, homs::launch_search_learned(c, m, lscratch, plan, nq, d_q_hv, q_emb, q_emb8, qperm,
                                           w.lo, w.hi, k, w.keys, d_out_fallback, shortlist, hook,
                                           s),
            "shortlist kernels");
    // exhaustive pass over the windows of the queries that fell back
    HIP_TRY(c, homs::launch_fallback_scan(c, nq, d_q_hv, d_out_fallback, w.lo, w.hi, fb_scratch,
                                          w.keys, s),
            "fallback search kernels");
    hipEvent_t e2 = prof_mark(c, s);
    HIP_TRY(c, homs::launch_finalize(nq, w.keys, d_out_idx, d_out_dist, s), "finalize kernel");
    hipEvent_t e3 = prof_mark(c, s);
    prof_span(c, e0, e1, homs::kProfPrep);
    prof_span(c, e1, e2, homs::kProfSearch);
    prof_span(c, e2, e3, homs::kProfPrep);
    return HOMS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// library and model files

namespace {

constexpr size_t kIoChunk = (size_t)64 << 20;  // bytes staged through the host per copy

// checksum of the context's position and level tables (the codebook a
// library was encoded with)
homs_status codebook_hash(homs_ctx* c, uint64_t* out)
{
    std::vector<uint32_t> id, lv;
    try {
        id.resize((size_t)c->n_bins * c->words);
        lv.resize((size_t)c->p.n_levels * c->words);
    } catch (const std::bad_alloc&) {
        return fail(c, HOMS_E_OOM, "host allocation failed (codebook)");
    }
    HIP_TRY(c, hipMemcpy(id.data(), c->d_id, id.size() * 4, hipMemcpyDeviceToHost),
            "hipMemcpy(id table)");
    HIP_TRY(c, hipMemcpy(lv.data(), c->d_level, lv.size() * 4, hipMemcpyDeviceToHost),
            "hipMemcpy(level table)");
    homs::Checksum h;
    h.update(id.data(), id.size() * 4);
    h.update(lv.data(), lv.size() * 4);
    *out = h.value();
    return HOMS_OK;
}

void fill_library_header(const homs_ctx* c, homs::LibraryHeader* hd)
{
    std::memset(hd, 0, sizeof(*hd));
    std::memcpy(hd->magic, homs::kLibraryMagic, 8);
    hd->version = homs::kFileVersion;
    hd->dim = c->p.dim;
    hd->n_levels = c->p.n_levels;
    hd->top_n = c->p.top_n;
    hd->id_flips = c->p.id_flips;
    hd->charge_match = c->p.charge_match;
    hd->encoding = c->p.encoding;
    hd->mz_min = c->p.mz_min;
    hd->mz_max = c->p.mz_max;
    hd->bins_per_da = c->p.bins_per_da;
    hd->noise_frac = c->p.noise_frac;
    hd->seed = c->p.seed;
}

// the bytes of a library file of n rows of W words
int64_t library_file_bytes(int64_t n, uint32_t words)
{
    return (int64_t)sizeof(homs::LibraryHeader) + n * (4 + 8 + 1 + 4 * (int64_t)words) + 8;
}

int64_t model_file_bytes(int64_t D, int64_t H, int64_t E)
{
    return (int64_t)sizeof(homs::ModelHeader) + 3 * 4 * (H * D + H + E * H + E) + 8;
}

// device -> file through a host staging buffer
homs_status write_device(homs_ctx* c, homs::FileWriter& f, const void* d, size_t bytes,
                         std::vector<char>& buf)
{
    for (size_t off = 0; off < bytes; off += buf.size()) {
        const size_t m = std::min(buf.size(), bytes - off);
        HIP_TRY(c, hipMemcpy(buf.data(), (const char*)d + off, m, hipMemcpyDeviceToHost),
                "hipMemcpy(save)");
        if (!f.write(buf.data(), m)) return fail(c, HOMS_E_INVALID, "file write failed");
    }
    return HOMS_OK;
}

// file -> device through a host staging buffer
homs_status read_device(homs_ctx* c, homs::FileReader& f, void* d, size_t bytes,
                        std::vector<char>& buf)
{
    for (size_t off = 0; off < bytes; off += buf.size()) {
        const size_t m = std::min(buf.size(), bytes - off);
        if (!f.read(buf.data(), m)) return fail(c, HOMS_E_INVALID, "file is truncated");
        HIP_TRY(c, hipMemcpy((char*)d + off, buf.data(), m, hipMemcpyHostToDevice),
                "hipMemcpy(load)");
    }
    return HOMS_OK;
}

// host copy of the device sort key of a precursor m/z (negative values
// reversed), so a file's row order is checked exactly as the sort made it
uint64_t order_key_host(double x)
{
    uint64_t b;
    std::memcpy(&b, &x, 8);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

}  // namespace

extern "C" {

homs_status homs_library_save(homs_ctx* c, const char* path)
{
    if (homs_status s = usable(c)) return s;
    if (!path) return fail(c, HOMS_E_INVALID, "path is NULL");
    if (!c->lib_valid) return fail(c, HOMS_E_STATE, "no encoded library");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
    homs::LibraryHeader hd;
    fill_library_header(c, &hd);
    if (homs_status s = codebook_hash(c, &hd.codebook_hash)) return s;
    hd.n = c->lib.n;
    std::vector<char> buf;
    try {
        buf.resize(kIoChunk);
    } catch (const std::bad_alloc&) {
        return fail(c, HOMS_E_OOM, "host allocation failed (staging)");
    }
    std::string why;
    homs::FileWriter f;
    if (!f.open(path, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!f.write(&hd, sizeof(hd))) return fail(c, HOMS_E_INVALID, "file write failed");
    const size_t n = (size_t)c->lib.n;
    for (auto part : {std::make_pair((const void*)c->lib.orig, n * 4),
                      std::make_pair((const void*)c->lib.pmz, n * 8),
                      std::make_pair((const void*)c->lib.charge, n),
                      std::make_pair((const void*)c->lib.hv, n * c->words * 4)})
        if (part.second)
            if (homs_status s = write_device(c, f, part.first, part.second, buf)) return s;
    if (!f.finish(&why)) return fail(c, HOMS_E_INVALID, why);
    return HOMS_OK;
}

homs_status homs_library_load(homs_ctx* c, const char* path)
{
    if (homs_status s = usable(c)) return s;
    if (!path) return fail(c, HOMS_E_INVALID, "path is NULL");
    DeviceGuard g(c->device);
    std::string why;
    homs::FileReader f;
    if (!f.open(path, &why)) return fail(c, HOMS_E_INVALID, why);
    homs::LibraryHeader hd;
    if (!f.read(&hd, sizeof(hd)) || std::memcmp(hd.magic, homs::kLibraryMagic, 8) != 0)
        return fail(c, HOMS_E_INVALID, "not a library file");
    if (hd.version != homs::kFileVersion)
        return fail(c, HOMS_E_UNSUPPORTED, "library file version " + std::to_string(hd.version));
    homs::LibraryHeader want;
    fill_library_header(c, &want);
    if (hd.dim != want.dim || hd.n_levels != want.n_levels || hd.top_n != want.top_n ||
        hd.id_flips != want.id_flips || hd.charge_match != want.charge_match ||
        hd.encoding != want.encoding || hd.mz_min != want.mz_min || hd.mz_max != want.mz_max ||
        hd.bins_per_da != want.bins_per_da || hd.noise_frac != want.noise_frac ||
        hd.seed != want.seed)
        return fail(c, HOMS_E_INVALID, "the library was encoded with other parameters");
    if (homs_status s = codebook_hash(c, &want.codebook_hash)) return s;
    if (hd.codebook_hash != want.codebook_hash)
        return fail(c, HOMS_E_INVALID, "the library was encoded with another codebook");
    if (hd.n < 0 || hd.n >= ((int64_t)1 << 31) || f.size() != library_file_bytes(hd.n, c->words))
        return fail(c, HOMS_E_INVALID, "library file size does not match its header");
    const int64_t n = hd.n;
    std::vector<uint32_t> orig;
    std::vector<double> pmz;
    std::vector<int8_t> charge;
    std::vector<char> buf;
    try {
        orig.resize(n);
        pmz.resize(n);
        charge.resize(n);
        buf.resize(kIoChunk);
    } catch (const std::bad_alloc&) {
        return fail(c, HOMS_E_OOM, "host allocation failed (library file)");
    }
    if (!f.read(orig.data(), n * 4) || !f.read(pmz.data(), n * 8) || !f.read(charge.data(), n))
        return fail(c, HOMS_E_INVALID, "file is truncated");
    // the order must be a permutation sorted as the library sort makes it
    {
        std::vector<uint8_t> seen(n, 0);
        for (int64_t j = 0; j < n; ++j) {
            if (orig[j] >= (uint64_t)n || seen[orig[j]])
                return fail(c, HOMS_E_INVALID, "library file order is not a permutation");
            seen[orig[j]] = 1;
            if (!hd.charge_match && charge[j] != 0)
                return fail(c, HOMS_E_INVALID, "library file has charges without charge_match");
            if (j > 0) {
                const uint64_t a = order_key_host(pmz[j - 1]), b = order_key_host(pmz[j]);
                const bool ordered = charge[j - 1] != charge[j] ? charge[j - 1] < charge[j]
                                     : a != b                 ? a < b
                                                              : orig[j - 1] < orig[j];
                if (!ordered) return fail(c, HOMS_E_INVALID, "library file rows are not sorted");
            }
        }
    }
    homs::Library L;
    L.n = n;
    const size_t orig_pad = (size_t)homs::search_mfma_row_pad();
    hipError_t e = hipSuccess;
    if (n > 0) {
        e = homs::dev_malloc(&L.hv, (size_t)n * c->words * 4);
        if (e == hipSuccess) e = homs::dev_malloc(&L.pmz, (size_t)n * 8);
        if (e == hipSuccess) e = homs::dev_malloc(&L.charge, (size_t)n);
        if (e == hipSuccess) e = homs::dev_malloc(&L.orig, ((size_t)n + orig_pad) * 4);
        if (e == hipSuccess) e = homs::dev_malloc(&L.slot, (size_t)n * 4);
        if (e == hipSuccess) e = homs::dev_malloc(&L.rowk, ((size_t)n + orig_pad) * 4);
        if (e == hipSuccess) e = hipMemcpy(L.orig, orig.data(), (size_t)n * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(L.orig + n, 0, orig_pad * 4);
        if (e == hipSuccess) e = hipMemcpy(L.pmz, pmz.data(), (size_t)n * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(L.charge, charge.data(), (size_t)n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = homs::launch_slots(n, L.orig, L.slot, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        free_library(L);
        return hip_fail(c, e, "library load");
    }
    if (homs_status s = read_device(c, f, L.hv, (size_t)n * c->words * 4, buf)) {
        free_library(L);
        return s;
    }
    if (n > 0) {
        const hipError_t ek = homs::launch_fp4_row_consts(n, c->words, L.hv, L.rowk, nullptr);
        if (ek != hipSuccess) {
            free_library(L);
            return hip_fail(c, ek, "library load");
        }
    }
    if (!f.finish(&why)) {
        free_library(L);
        return fail(c, HOMS_E_INVALID, why);
    }
    HIP_TRY(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
    free_library(c->lib);
    drop_graph(c);
    c->lib = L;
    c->lib_valid = true;
    c->lib_gen += 2;
    return HOMS_OK;
}

homs_status homs_model_save(homs_model* m, const char* path)
{
    if (homs_status s = model_usable(m)) return s;
    homs_ctx* c = m->ctx;
    if (!path) return fail(c, HOMS_E_INVALID, "path is NULL");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipDeviceSynchronize(), "hipDeviceSynchronize");
    homs::ModelHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    std::memcpy(hd.magic, homs::kModelMagic, 8);
    hd.version = homs::kFileVersion;
    hd.dim = (uint32_t)m->D;
    hd.hidden = m->H;
    hd.embed = m->E;
    hd.step = m->step;
    std::vector<char> buf;
    try {
        buf.resize(kIoChunk);
    } catch (const std::bad_alloc&) {
        return fail(c, HOMS_E_OOM, "host allocation failed (staging)");
    }
    std::string why;
    homs::FileWriter f;
    if (!f.open(path, &why)) return fail(c, HOMS_E_INVALID, why);
    if (!f.write(&hd, sizeof(hd))) return fail(c, HOMS_E_INVALID, "file write failed");
    const size_t n1 = (size_t)m->H * m->D, n2 = (size_t)m->E * m->H;
    const std::pair<const float*, size_t> parts[] = {
        {m->W1, n1}, {m->b1, (size_t)m->H}, {m->W2, n2}, {m->b2, (size_t)m->E},
        {m->mW1, n1}, {m->vW1, n1}, {m->mb1, (size_t)m->H}, {m->vb1, (size_t)m->H},
        {m->mW2, n2}, {m->vW2, n2}, {m->mb2, (size_t)m->E}, {m->vb2, (size_t)m->E}};
    for (const auto& part : parts)
        if (homs_status s = write_device(c, f, part.first, part.second * 4, buf)) return s;
    if (!f.finish(&why)) return fail(c, HOMS_E_INVALID, why);
    return HOMS_OK;
}

homs_status homs_model_load(homs_ctx* c, const char* path, homs_model** out)
{
    if (!out) return fail(nullptr, HOMS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (homs_status s = usable(c)) return s;
    if (!path) return fail(c, HOMS_E_INVALID, "path is NULL");
    DeviceGuard g(c->device);
    std::string why;
    homs::FileReader f;
    if (!f.open(path, &why)) return fail(c, HOMS_E_INVALID, why);
    homs::ModelHeader hd;
    if (!f.read(&hd, sizeof(hd)) || std::memcmp(hd.magic, homs::kModelMagic, 8) != 0)
        return fail(c, HOMS_E_INVALID, "not a model file");
    if (hd.version != homs::kFileVersion)
        return fail(c, HOMS_E_UNSUPPORTED, "model file version " + std::to_string(hd.version));
    if (hd.dim != c->p.dim) return fail(c, HOMS_E_INVALID, "model dimension differs from D");
    if (hd.hidden < 32 || hd.hidden > 8192 || hd.hidden % 32 != 0 || hd.embed < 32 ||
        hd.embed > 4096 || hd.embed % 32 != 0 || hd.step < 0)
        return fail(c, HOMS_E_INVALID, "invalid model shape in file");
    if (f.size() != model_file_bytes(hd.dim, hd.hidden, hd.embed))
        return fail(c, HOMS_E_INVALID, "model file size does not match its header");
    const size_t n1 = (size_t)hd.hidden * hd.dim, n2 = (size_t)hd.embed * hd.hidden;
    std::vector<float> w;
    try {
        w.resize(3 * (n1 + n2 + hd.hidden + hd.embed));
    } catch (const std::bad_alloc&) {
        return fail(c, HOMS_E_OOM, "host allocation failed (model file)");
    }
    if (!f.read(w.data(), w.size() * 4)) return fail(c, HOMS_E_INVALID, "file is truncated");
    if (!f.finish(&why)) return fail(c, HOMS_E_INVALID, why);
    float* p = w.data();
    auto take = [&](size_t k) {
        float* r = p;
        p += k;
        return r;
    };
    float *W1 = take(n1), *b1 = take(hd.hidden), *W2 = take(n2), *b2 = take(hd.embed);
    homs_model* m = nullptr;
    if (homs_status s = homs_model_create(c, hd.hidden, hd.embed, W1, b1, W2, b2, &m)) return s;
    const std::pair<float*, size_t> moments[] = {
        {m->mW1, n1}, {m->vW1, n1}, {m->mb1, (size_t)hd.hidden}, {m->vb1, (size_t)hd.hidden},
        {m->mW2, n2}, {m->vW2, n2}, {m->mb2, (size_t)hd.embed}, {m->vb2, (size_t)hd.embed}};
    for (const auto& mo : moments) {
        hipError_t e = hipMemcpy(mo.first, take(mo.second), mo.second * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            homs_model_destroy(m);
            return hip_fail(c, e, "hipMemcpy(model moments)");
        }
    }
    m->step = hd.step;
    *out = m;
    return HOMS_OK;
}

homs_status homs_file_inspect(const char* path, homs_file_info* out)
{
    if (!path || !out) return fail(nullptr, HOMS_E_INVALID, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    std::string why;
    homs::FileReader f;
    if (!f.open(path, &why)) return fail(nullptr, HOMS_E_INVALID, why);
    char magic[8];
    if (!f.read(magic, 8)) return fail(nullptr, HOMS_E_INVALID, "not a libhyperoms file");
    int64_t payload = 0;
    if (std::memcmp(magic, homs::kLibraryMagic, 8) == 0) {
        homs::LibraryHeader hd;
        std::memcpy(hd.magic, magic, 8);
        if (!f.read((char*)&hd + 8, sizeof(hd) - 8))
            return fail(nullptr, HOMS_E_INVALID, "file is truncated");
        if (hd.version != homs::kFileVersion)
            return fail(nullptr, HOMS_E_UNSUPPORTED, "file version " + std::to_string(hd.version));
        if (hd.dim < 512 || hd.dim > 32768 || hd.dim % 512 != 0 || hd.n < 0 ||
            hd.n >= ((int64_t)1 << 31) || f.size() != library_file_bytes(hd.n, hd.dim / 32))
            return fail(nullptr, HOMS_E_INVALID, "library file size does not match its header");
        out->kind = HOMS_FILE_LIBRARY;
        out->version = hd.version;
        out->dim = hd.dim;
        out->n = hd.n;
        out->codebook_hash = hd.codebook_hash;
        homs_params_default(&out->params);
        out->params.dim = hd.dim;
        out->params.n_levels = hd.n_levels;
        out->params.top_n = hd.top_n;
        out->params.mz_min = hd.mz_min;
        out->params.mz_max = hd.mz_max;
        out->params.bins_per_da = hd.bins_per_da;
        out->params.noise_frac = hd.noise_frac;
        out->params.id_flips = hd.id_flips;
        out->params.charge_match = hd.charge_match;
        out->params.seed = hd.seed;
        out->params.encoding = hd.encoding;
        payload = f.size() - (int64_t)sizeof(hd) - 8;
    } else if (std::memcmp(magic, homs::kModelMagic, 8) == 0) {
        homs::ModelHeader hd;
        std::memcpy(hd.magic, magic, 8);
        if (!f.read((char*)&hd + 8, sizeof(hd) - 8))
            return fail(nullptr, HOMS_E_INVALID, "file is truncated");
        if (hd.version != homs::kFileVersion)
            return fail(nullptr, HOMS_E_UNSUPPORTED, "file version " + std::to_string(hd.version));
        if (hd.hidden < 32 || hd.hidden > 8192 || hd.embed < 32 || hd.embed > 4096 ||
            hd.dim < 512 || hd.dim > 32768 ||
            f.size() != model_file_bytes(hd.dim, hd.hidden, hd.embed))
            return fail(nullptr, HOMS_E_INVALID, "model file size does not match its header");
        out->kind = HOMS_FILE_MODEL;
        out->version = hd.version;
        out->dim = hd.dim;
        out->hidden = hd.hidden;
        out->embed = hd.embed;
        out->step = hd.step;
        payload = f.size() - (int64_t)sizeof(hd) - 8;
    } else {
        return fail(nullptr, HOMS_E_INVALID, "not a libhyperoms file");
    }
    std::vector<char> buf;
    try {
        buf.resize(kIoChunk);
    } catch (const std::bad_alloc&) {
        return fail(nullptr, HOMS_E_OOM, "host allocation failed (staging)");
    }
    for (int64_t off = 0; off < payload; off += (int64_t)buf.size()) {
        const size_t m = (size_t)std::min<int64_t>((int64_t)buf.size(), payload - off);
        if (!f.read(buf.data(), m)) return fail(nullptr, HOMS_E_INVALID, "file is truncated");
    }
    if (!f.finish(&why)) return fail(nullptr, HOMS_E_INVALID, why);
    return HOMS_OK;
}

}  // extern "C"
