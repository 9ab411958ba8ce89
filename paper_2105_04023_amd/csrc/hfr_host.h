// Host-side pieces shared by the translation units of the library: the
// context, allocation through the caller's hooks and error reporting.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <string>

#include "../../include/im.h"
#include "hfr_internal.h"

struct im_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;  // bytes all handles of the context may hold (0 = no bound)
    size_t in_use = 0;
    im_alloc_fn af = nullptr;
    im_free_fn ff = nullptr;
    void* user = nullptr;
};

namespace hfr {

extern thread_local std::string g_last_error;

// Records a thread-local message for im_last_error() and returns st.
im_status fail(im_status st, const char* fmt, ...);

// Device memory through the context's hooks (hipMalloc/hipFree without
// hooks); sizes are rounded up to 256 bytes.  Returns nullptr on failure.
void* ctx_alloc(im_ctx* c, size_t bytes);
void ctx_free(im_ctx* c, void* p);

}  // namespace hfr
