// Host-side pieces shared by the translation units of the library: the
// context, allocation through the caller's hooks and error reporting.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <atomic>
#include <string>

#include "../../include/im.h"
#include "hfr_internal.h"

struct im_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;  // bytes all handles of the context may hold (0 = no bound)
    std::atomic<size_t> in_use{0};  // sketches of several threads may be released into one context
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

// Offsets of a caller's CSR, int64 or int32 per im_csr.offset_bits.
// csr_offsets_check: IM_OK, or the error (with its message) of an invalid offset_bits.
im_status csr_offsets_check(const im_csr* g);
// Offset i (host read, or a small device-to-host copy for device arrays); -1 on a copy failure.
int64_t csr_offset_at(const im_csr* g, int64_t i);
// All n+1 offsets as int64 into device memory dst (widened on the device for int32 inputs).
hipError_t csr_copy_offsets(const im_csr* g, int64_t* dst, hipStream_t s);
// All n+1 offsets as int64 into host memory.
hipError_t csr_offsets_to_host(const im_csr* g, int64_t* dst);

// Moves an idle sketch (no work of it in flight) to another context of the same
// device: its later calls run on that context's stream and count against that
// context's bytes in use.  Both contexts must use the same allocator.
void sketch_rebind(im_sketch* sk, im_ctx* ctx);

}  // namespace hfr
