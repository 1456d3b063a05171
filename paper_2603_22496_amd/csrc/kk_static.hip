// kk_beamform without a caller workspace, for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops, harnesses that forbid allocation).  The pair
// shares of a split plan (partial images, summed in a fixed order afterwards) live in a
// file-scope device array of fixed size instead of the caller's workspace; every other step is
// kk_beamform's.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/kk.h"
#include "kk_internal.h"
#include "kk_plan.h"

// The shares live in `scratch` (one copy per GPU; every call overwrites the part it reads before
// reading it, so nothing needs clearing).  Host code reaches the array only through the device
// address hipGetSymbolAddress returns for the current GPU.
static constexpr size_t kStaticScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace kk {
namespace {

constexpr int kMaxDevices = 64;

std::mutex scratch_mutex;
void* scratch_ptr[kMaxDevices];  // device address of `scratch` per GPU, set on first use

// The array's device address on the current GPU (looked up once per GPU, with it current).
void* device_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        scratch_ptr[dev] = p;
    }
    return scratch_ptr[dev];
}

}  // namespace
}  // namespace kk

extern "C" {

size_t kk_beamform_static_max_bytes(void) { return kStaticScratchBytes; }

int32_t kk_beamform_static(const float* rf_theta, int32_t N, int32_t M, int32_t T, const void* plan_host,
                           const void* plan_dev, size_t plan_bytes, float* image, float* intensity, int32_t mode,
                           void* stream) {
    using namespace kk;
    if (!rf_theta || !plan_host || !plan_dev || !image) return KK_E_NULL;
    const int32_t* h = static_cast<const int32_t*>(plan_host);
    if (!gather_plan_ok(h, plan_bytes, false)) return KK_E_WORKSPACE;
    if (h[PW_N] != N || h[PW_M] != M || h[PW_T] != T || N < 1 || M < 1 || T < 1) return KK_E_ARG;
    if (intensity && mode != KK_COMPOUND_COHERENT && mode != KK_COMPOUND_INCOHERENT) return KK_E_ARG;
    if (gather_workspace_bytes(h) > kStaticScratchBytes) return KK_E_WORKSPACE;
    void* ws = device_scratch();
    if (!ws) return KK_E_HIP;
    const hipError_t e = run_gather(reinterpret_cast<const float2*>(rf_theta), h, static_cast<const int32_t*>(plan_dev),
                                    reinterpret_cast<float2*>(image), intensity, mode, ws, false,
                                    (hipStream_t)stream);
    return e == hipSuccess ? KK_OK : KK_E_HIP;
}

}  // extern "C"
