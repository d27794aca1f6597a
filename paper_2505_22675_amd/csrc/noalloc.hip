// Binning + IDW without any device allocation: the bins and the binning
// scratch live in a file-scope device array (one copy per GPU, resident from
// the library's load until the process ends) instead of a caller workspace.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address reaches kernels.
#include "auv_internal.hpp"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = AUV_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up on the first call
// on each device, with that device current).
auv_status scratch_on_current_device(char **out)
{
    int dev = -1;
    AUV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return auv::fail(AUV_ERR_RANGE, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return auv::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0)
            return auv::fail(AUV_ERR_HIP, "scratch symbol address missing or misaligned");
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return AUV_OK;
}

}  // namespace

extern "C" {

auv_status auv_grid_idw_noalloc(const auv_grid *grid, const double *x, const double *y,
                                const double *z, int64_t n, int32_t bin_log2,
                                const auv_idw_params *params, float *z_out, int32_t *cnt_out,
                                int32_t *nn_idx_out, float *nn_z_out, auv_stream stream)
{
    if (!grid || !params)
        return auv::fail(AUV_ERR_INVALID, "grid or params is null");
    size_t need = 0;
    const auv_status qs = auv_bin_workspace_size(grid, n, params->radius, bin_log2, &need);
    if (qs != AUV_OK)
        return qs;
    if (need > kScratchBytes)
        return auv::fail(AUV_ERR_BUDGET,
                         "binning needs " + std::to_string(need) +
                             " bytes, more than the static scratch (" +
                             std::to_string(kScratchBytes) + " bytes)");
    char *ws = nullptr;
    const auv_status ss = scratch_on_current_device(&ws);
    if (ss != AUV_OK)
        return ss;
    auv_bins b{};
    const auv_status bs = auv::bin_into(grid, x, y, z, n, params->radius, bin_log2, ws,
                                        kScratchBytes, static_cast<hipStream_t>(stream), &b);
    if (bs != AUV_OK)
        return bs;
    return auv_interp_idw(grid, &b, params, z_out, cnt_out, nn_idx_out, nn_z_out, stream);
}

}  // extern "C"
