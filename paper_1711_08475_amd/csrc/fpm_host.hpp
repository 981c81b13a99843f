// fpm_host.hpp -- host-side helpers shared by the C ABI sources: error
// reporting (thread-local last error) and device allocation.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/fpm.h"

namespace fpm {

extern thread_local std::string g_last_error;

fpm_status fail(fpm_status st, const char *fmt, ...);
fpm_status hip_fail(hipError_t e, const char *what);

// Every device buffer of the library goes through these two: they keep the
// process-wide count of live bytes that fpm_device_memory_in_use reports,
// and refuse an allocation that would take it past the limit set with
// fpm_set_device_memory_limit (hipErrorOutOfMemory, i.e. FPM_ENOMEM).
hipError_t dev_alloc(void **p, size_t bytes);
void dev_free(void *p);

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    return dev_alloc((void **)p, bytes);
}

template <typename T>
void dfree(T *&p)
{
    if (p)
        dev_free((void *)p);
    p = nullptr;
}

}  // namespace fpm

#define HIPCHK(expr)                                   \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess)                          \
            return fpm::hip_fail(_e, #expr);           \
    } while (0)
