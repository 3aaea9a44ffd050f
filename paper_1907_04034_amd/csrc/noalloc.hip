// noalloc.hip -- sph_step without a caller workspace, for callers that cannot
// allocate device memory: the workspace is a file-scope device array of
// SPH_STATIC_SCRATCH_BYTES that every GPU the library runs on holds from its
// load until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (with that
// device current) and only that address is used afterwards.
#include <mutex>

#include "sph_launch.h"

namespace {

constexpr size_t kScratchBytes = SPH_STATIC_SCRATCH_BYTES;
static_assert(kScratchBytes % 16 == 0, "the clear writes 16-byte words");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device, then kept). Returns SPH_OK or an error code.
int device_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return sph::api_error(SPH_EHIP, "sph_step_static: no current HIP device");
    if (dev >= kMaxDevices)
        return sph::api_error(SPH_EUNSUPPORTED, "sph_step_static: device index above 63");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return sph::api_error(SPH_EHIP, "sph_step_static: hipGetSymbolAddress failed");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SPH_OK;
}

// The used part of the scratch is cleared at every call: the workspace of a
// step must start zeroed (counters are consumed and re-zeroed by their own
// kernels), and the previous call may have laid the same bytes out for
// another capacity or cell grid. A kernel rather than hipMemsetAsync, so that
// the call can be captured into a HIP graph.
__global__ void __launch_bounds__(sph::kBlock) k_clear(uint4 *p, size_t n16)
{
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = uint4{0u, 0u, 0u, 0u};
}

// The call's device error word (the workspace's first word) to the caller.
__global__ void k_take_error(const uint32_t *err, uint32_t *out) { *out = *err; }

}  // namespace

extern "C" int sph_step_static(const sph_params *prm, sph_state *st, sph_state *alt,
                               sph_nlist *nl, sph_derived *out, int32_t nsteps,
                               double *drag_hist, uint32_t *err_out, void *stream)
{
    if (!st) return sph::api_error(SPH_EINVAL, "sph_step_static: state is NULL");
    size_t need = 0;
    int rc = sph_workspace_size(prm, st->cap, &need);
    if (rc) return rc;
    if (need > kScratchBytes)
        return sph::api_error(SPH_ECAPACITY,
                              "sph_step_static: this capacity and cell grid need a larger "
                              "workspace than the static scratch holds; use sph_step");
    void *ws = nullptr;
    if ((rc = device_scratch(&ws))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n16 = (need + 15) / 16;
    const int64_t blocks = (int64_t(n16) + sph::kBlock - 1) / sph::kBlock;
    hipLaunchKernelGGL(k_clear, dim3(unsigned(blocks < 4096 ? blocks : 4096)),
                       dim3(sph::kBlock), 0, s, static_cast<uint4 *>(ws), n16);
    rc = sph::step_on_workspace(prm, st, alt, nl, out, nsteps, drag_hist, ws, need, stream);
    if (rc) return rc;
    if (err_out)
        hipLaunchKernelGGL(k_take_error, dim3(1), dim3(1), 0, s,
                           static_cast<const uint32_t *>(ws), err_out);
    if (hipGetLastError() != hipSuccess)
        return sph::api_error(SPH_EHIP, "sph_step_static: kernel launch failed");
    return SPH_OK;
}
