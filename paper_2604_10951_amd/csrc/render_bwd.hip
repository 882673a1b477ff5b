// render_bwd.hip -- backward of the blend (written next).
#include "fs_internal.h"

hipError_t fs_launch_render_backward(const float*, const float*, const float*, const float*, const FsRecord*,
                                     const uint32_t*, const uint32_t*, const void*, int, int64_t, const fs_camera*,
                                     int, int64_t, const fs_opts&, const float*, const int32_t*, const int32_t*,
                                     const float*, float*, float*, float*, float*, float*, float*,
                                     const FsWorkspace&, hipStream_t) {
    return hipErrorNotSupported;
}
