// Placeholder: decomposition and DAS kernels are added next.
#include <hip/hip_runtime.h>
#include "../../include/kk.h"
extern "C" {
size_t kk_decompose_workspace_bytes(const kk_geom*, int32_t, int32_t, int32_t, int32_t) { return 0; }
int32_t kk_decompose(const int16_t*, int32_t, const kk_geom*, const int32_t*, int32_t, int32_t, int32_t, float*,
                     void*, size_t, void*) { return KK_E_UNSUPPORTED; }
size_t das_workspace_bytes(const kk_geom*, int32_t) { return 0; }
int32_t das_beamform(const int16_t*, int32_t, const kk_geom*, const void*, const void*, size_t, float*, void*,
                     size_t, void*) { return KK_E_UNSUPPORTED; }
}
