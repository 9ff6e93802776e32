// The matching sweep for callers that cannot allocate memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation): the
// same computation as rich_match_sweep, with its device work arrays in a
// fixed file-scope device array instead of hipMalloc'd buffers and its host
// read-back into a local variable instead of pinned memory.
#include <mutex>

#include "common.hpp"

namespace {

// The work arrays of every call on a device.  Each GPU the library runs on
// holds its own copy for the life of the process.  Host code never uses this
// name as an address (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) char scratch[RICH_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch_dev[MAX_DEVICES] = {};  // device address of `scratch`, per device

// The device address of the current device's array, looked up once per
// device (with that device current) and kept.
rich_status scratch_address(void **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return RICH_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return RICH_EHIP;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return RICH_OK;
}

}  // namespace

extern "C" rich_status rich_match_sweep_noalloc(int64_t n, const int64_t *rowptr_dev, const int32_t *col_dev,
                                                const double *val_dev, int32_t *agg_dev, int64_t *n_coarse_host,
                                                void *hip_stream) {
    if (n < 0 || n >= ((int64_t)1 << 31) || !rowptr_dev || !col_dev || !val_dev || !agg_dev || !n_coarse_host)
        return RICH_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (n == 0) {
        *n_coarse_host = 0;
        return RICH_OK;
    }
    int64_t nnz = 0;
    HIP_TRY(hipMemcpyAsync(&nnz, rowptr_dev + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (nnz < 0) return RICH_EINVAL;
    if (rich::match_ws_bytes(n, nnz) > (size_t)RICH_NOALLOC_SCRATCH_BYTES) return RICH_EBUDGET;
    void *base = nullptr;
    RICH_TRY(scratch_address(&base));
    int still = 0;
    return rich::match_sweep_ws(n, rowptr_dev, col_dev, val_dev, agg_dev, n_coarse_host,
                                rich::match_ws_carve(base, n, nnz), &still, s);
}
