// Shared host/device helpers of libddf: status handling and small vector types.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/ddf.h"

namespace ddf {

void set_error(const char *fmt, ...);
void clear_error();

// Validation helper: record a message and return the status.
#define DDF_REQUIRE(cond, status, ...)          \
    do {                                        \
        if (!(cond)) {                          \
            ::ddf::set_error(__VA_ARGS__);      \
            return (status);                    \
        }                                       \
    } while (0)

// Map a HIP launch error to DDF_ERR_HIP.
inline ddf_status launch_status(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return DDF_ERR_HIP;
    }
    return DDF_OK;
}

inline hipStream_t as_stream(ddf_stream s) { return reinterpret_cast<hipStream_t>(s); }

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

}  // namespace ddf
