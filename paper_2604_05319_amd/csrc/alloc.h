// Device memory of the library: every allocation goes through the process-wide
// allocator hook (hnessi_set_allocator), stream-ordered on the stream of the
// call that allocates.
#pragma once

#include <string>
#include <vector>

#include "../../include/hnessi.h"
#include "common.h"

namespace hn {

// Allocations made with one snapshot of the hook (a handle keeps the hook it
// was created with, so a later hnessi_set_allocator does not change how its
// memory is returned).
struct DevAlloc {
    hnessi_alloc_fn fa = nullptr;
    hnessi_free_fn ff = nullptr;
    void* ctx = nullptr;
    hipStream_t st = nullptr;   // stream of the allocations (and of zero fills)
    std::vector<void*> ptrs;
    size_t bytes = 0;

    static DevAlloc current(hipStream_t st);
    // nbytes of device memory, or nullptr when the hook fails; zero = fill with zeros
    // on st (a kernel, not a memset node)
    void* raw(size_t nbytes, bool zero);
    // return every allocation through the hook; on_stream: stream-ordered on st,
    // otherwise on the NULL stream (the caller has synchronized the work using it)
    void release(bool on_stream);
};

// allocate count elements of T; HNESSI_OK or HNESSI_E_NOMEM (message set)
template <class T>
int dev_alloc(DevAlloc& al, T*& p, size_t count, bool zero) {
    if (count == 0) count = 1;
    p = static_cast<T*>(al.raw(count * sizeof(T), zero));
    return p ? HNESSI_OK : HNESSI_E_NOMEM;
}

// thread-local last-error message of the C ABI
int set_error(int code, const std::string& msg);
int lib_init();

}  // namespace hn
