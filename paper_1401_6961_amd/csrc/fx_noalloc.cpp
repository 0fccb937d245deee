// Exchange without device allocation, for callers that cannot allocate
// (code under stream capture, serving loops with a fixed memory budget).
//
// The work runs in a file-scope device array of FX_SCRATCH_BYTES that every
// call on a GPU shares (each GPU holds its own copy, at its own address, for
// the life of the process).  Host code never passes the array's name to a
// kernel or a copy: its device address is looked up once per device with
// hipGetSymbolAddress and kept, and that address is what the exchange uses.
// Every buffer a kernel reads before writing (counters, accumulators,
// flags) is cleared by a fill kernel at the start of each call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/fx.h"
#include "fx_host.h"

#define FX_SCRATCH_BYTES (256ull << 20)
#define FX_SCRATCH_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[FX_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[FX_SCRATCH_MAX_DEVICES];

// Device address of `scratch` on the current device (looked up once per device).
static void* scratch_address() {
    int dev = 0;
    FX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= FX_SCRATCH_MAX_DEVICES) fx_fail(FX_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fx_fail(FX_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

extern "C" {

size_t fx_noalloc_scratch_bytes(void) { return (size_t)FX_SCRATCH_BYTES; }

fx_status fx_exchange_noalloc(const fx_tree* tree, const double* P, double tau, double* K,
                              const fx_exchange_opts* opts, fx_stats* stats, void* stream) {
    return fx_guard([&] {
        if (opts && (opts->use_graph || opts->profile))
            fx_fail(FX_ERR_INVALID_ARG, "use_graph and profile allocate; fx_exchange_noalloc takes neither");
        void* base = scratch_address();
        fx_exchange_run(&tree, &P, &K, 1, 1, tau, opts, stats, (hipStream_t)stream, base, (size_t)FX_SCRATCH_BYTES);
    });
}

}  // extern "C"
