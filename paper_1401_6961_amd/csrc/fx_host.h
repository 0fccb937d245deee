// Internal declarations shared by the host sources of the exchange library
// (tree build and C ABI in fx_host.cpp, exchange execution in fx_exec.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fx.h"
#include "fx_costmodel.h"
#include "fx_internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
extern thread_local std::string g_last_error;

struct FxError {
    fx_status st;
    std::string msg;
};

[[noreturn]] inline void fx_fail(fx_status st, const std::string& msg) { throw FxError{st, msg}; }

#define FX_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) fx_fail(FX_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline fx_status fx_guard_status(const FxError& e) {
    g_last_error = e.msg;
    return e.st;
}

template <typename F>
inline fx_status fx_guard(F&& f) {
    try {
        f();
        g_last_error.clear();
        return FX_OK;
    } catch (const FxError& e) {
        return fx_guard_status(e);
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return FX_ERR_OOM;
    } catch (...) {
        g_last_error = "internal error";
        return FX_ERR_INTERNAL;
    }
}

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
extern fx_alloc_fn g_alloc;
extern fx_free_fn g_free;
extern void* g_alloc_ctx;

inline void* fx_dalloc(size_t bytes, hipStream_t st, bool persistent = false) {
    if (bytes == 0) bytes = 8;
    void* p = nullptr;
    if (persistent) {
        // memory owned by a tree handle outlives the caller's stream
        if (hipMalloc(&p, bytes) != hipSuccess || !p) {
            (void)hipGetLastError();
            fx_fail(FX_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
        return p;
    }
    if (g_alloc) {
        p = g_alloc(bytes, (void*)st, g_alloc_ctx);
        if (!p) fx_fail(FX_ERR_OOM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
        return p;
    }
    hipError_t e = hipMallocAsync(&p, bytes, st);
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        fx_fail(FX_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

inline void fx_dfree(void* p, hipStream_t st, bool persistent = false) {
    if (!p) return;
    if (persistent) {
        (void)hipFree(p);
        return;
    }
    if (g_free) g_free(p, (void*)st, g_alloc_ctx);
    else (void)hipFreeAsync(p, st);
}

// RAII set of device allocations tied to a stream
struct DevArena {
    hipStream_t st;
    bool persistent;
    std::vector<void*> ptrs;
    explicit DevArena(hipStream_t s, bool pers = false) : st(s), persistent(pers) {}
    template <typename T>
    T* get(size_t count) {
        T* p = (T*)fx_dalloc(sizeof(T) * count, st, persistent);
        ptrs.push_back(p);
        return p;
    }
    void release(void* p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            fx_dfree(p, st, persistent);
            ptrs.erase(it);
        }
    }
    ~DevArena() {
        for (void* p : ptrs) fx_dfree(p, st, persistent);
    }
};

template <typename T>
inline T* upload(DevArena& A, const std::vector<T>& v) {
    T* d = A.get<T>(v.size());
    if (!v.empty()) FX_HIP(hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, A.st));
    return d;
}

template <typename T>
inline T read1(const T* dptr, hipStream_t st) {
    T v;
    FX_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, st));
    FX_HIP(hipStreamSynchronize(st));
    return v;
}

inline int ncart(int l) { return (l + 1) * (l + 2) / 2; }


// ---------------------------------------------------------------------------
// host plan: ordering + ragged bisection
// ---------------------------------------------------------------------------
struct Level {
    std::vector<int> sL, sR, ch0, nch;  // nodes of this level; ch0/nch index level+1
};

struct Plan {
    std::vector<int> order;   // tree position -> caller shell index
    std::vector<Level> levels;
};

// ---------------------------------------------------------------------------
// the tree handle
// ---------------------------------------------------------------------------
// Buffer sizes learned from earlier calls on a tree: a call sizes its
// traversal buffers from them, so it needs no size read-back (fx_exec.cpp).
struct FxSizeHint {
    long e_in = 0;      // largest entry count of an inner level of the whole traversal (0: not known yet)
    long e_leaf = 0;    // leaf-level entry count of the whole traversal
    // measured for one split of K into row ranges: the largest inner-level and
    // leaf-level entry counts of any one range (0: not measured)
    int range_chunks = 0;
    long range_e_in = 0, range_e_leaf = 0;
    std::vector<long> leaf_rows;   // leaf entries per leaf row of the whole traversal (empty: unknown)
    // largest unit count per (la, ld) of one row range, at units_chunks ranges (0: not seen)
    int units_chunks = 0;
    long units_max[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // the row-range count last chosen, and what it was chosen for
    int plan_chunks = 0, plan_range_chunks = 0, plan_screen = 0;
    size_t plan_budget = 0;
    long plan_e_in = 0, plan_e_leaf = 0;
};
struct FxGraphCache;                        // fx_exec.cpp
void fx_graph_cache_free(FxGraphCache* g);  // fx_exec.cpp

struct fx_tree {
    int S = 0, n = 0, lmax = 0;
    uint64_t id = 0;                 // unique per handle (never reused)
    mutable std::mutex mu;           // guards hint, usage and the graph cache
    mutable FxSizeHint hint;
    mutable FxDevRun* usage = nullptr;       // pinned, written by the last call's copy
    mutable hipEvent_t usage_ev = nullptr;   // recorded after that copy
    mutable bool usage_pending = false;
    mutable int usage_nchunks = 1;           // row ranges of the call that wrote it
    mutable FxGraphCache* gcache = nullptr;
    std::vector<int> order;          // tree position -> caller shell
    std::vector<int> l, nprim;       // tree order
    std::vector<int> f0;             // tree order, caller function offset
    std::vector<Level> levels;
    std::vector<int> leaf_lofs;      // host copy
    bool single_shell_leaves = false;
    hipStream_t build_stream = nullptr;
    DevArena* arena = nullptr;
    FxDevBasis basis{};
    double* boys = nullptr;
    std::vector<int*> d_sL, d_sR, d_ch0, d_nch;
    std::vector<int*> d_nf;          // per level: functions of each node
    std::vector<double*> d_Qsq;      // per level (nk x nk)
    std::vector<double*> d_Smx;      // per level (nk x nk): block maxima of the shell-pair overlaps
    double* qrow = nullptr;          // max_b Qn[s][b]
    float mean_np[3] = {1, 1, 1};    // mean primitive count of the shells of each l
    ~fx_tree() {
        if (arena) (void)hipDeviceSynchronize();
        fx_graph_cache_free(gcache);
        if (usage_ev) (void)hipEventDestroy(usage_ev);
        if (usage) (void)hipHostFree(usage);
        delete arena;
    }
};

struct fx_costmodel {
    std::vector<float> W, norm;    // FX_MLP_NPARAM, FX_MLP_NNORM
    float* dW = nullptr;
    float* dnorm = nullptr;
    ~fx_costmodel() {
        if (dW) (void)hipFree(dW);
        if (dnorm) (void)hipFree(dnorm);
    }
    void upload() {
        if (!dW) {
            if (hipMalloc(&dW, sizeof(float) * FX_MLP_NPARAM) != hipSuccess ||
                hipMalloc(&dnorm, sizeof(float) * FX_MLP_NNORM) != hipSuccess)
                fx_fail(FX_ERR_OOM, "cost model allocation failed");
        }
        FX_HIP(hipMemcpy(dW, W.data(), sizeof(float) * FX_MLP_NPARAM, hipMemcpyHostToDevice));
        FX_HIP(hipMemcpy(dnorm, norm.data(), sizeof(float) * FX_MLP_NNORM, hipMemcpyHostToDevice));
    }
};

struct fx_task_timings {
    std::vector<float> feat;    // 4 per sample
    std::vector<float> log2ns;  // measured unit time
    std::vector<int> cls;       // cls * 2 + fp32
};

// per class and precision: kernel variant and launch flags (fx_host.cpp)
extern int g_variant[81][2];
extern int g_flags[81][2];
// timing-probe collection of the calling thread (fx_record_task_timings)
extern thread_local fx_task_timings* g_recording;

// Exchange of `count` systems with `ndens` densities each (fx_exec.cpp).
// Ps, Ks: count * ndens device pointers, system-major; scratch: a device
// block of scratch_bytes to work in (nothing is allocated), or null.
void fx_exchange_run(const fx_tree* const* trees, const double* const* Ps, double* const* Ks, int count, int ndens,
                     double tau, const fx_exchange_opts* opts, fx_stats* stats, hipStream_t st, void* scratch,
                     size_t scratch_bytes);
