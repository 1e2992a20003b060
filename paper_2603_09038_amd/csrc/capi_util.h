// Error-handling and allocation helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <new>
#include <string>

#include "internal.h"

#define PA_TRY try {
#define PA_CATCH                                                  \
    }                                                             \
    catch (const std::bad_alloc &) {                              \
        hexpa::set_error("host allocation failed");                      \
        return PA_ERR_ARG;                                        \
    }                                                             \
    catch (...) {                                                 \
        hexpa::set_error("unexpected host exception");                   \
        return PA_ERR_ARG;                                        \
    }

#define HIP_OK(expr)                                                                   \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) {                                                        \
            hexpa::set_error(std::string(#expr) + " failed: " + hipGetErrorString(_e));       \
            return PA_ERR_HIP;                                                         \
        }                                                                              \
    } while (0)

inline int arg_error(const char *msg)
{
    hexpa::set_error(msg);
    return PA_ERR_ARG;
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

template <class T>
inline hipError_t dalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, n * sizeof(T) + 16);
}
