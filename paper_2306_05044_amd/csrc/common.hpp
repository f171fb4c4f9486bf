// Host-side helpers shared by the C entry points: error reporting, argument
// checks and launch checks.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "capvndf.h"

namespace capvndf {

// Record a printf-style message for capvndf_last_error() and return code.
int32_t fail(int32_t code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// CAPVNDF_OK if the last launch succeeded, else CAPVNDF_ERR_HIP with a message.
int32_t check_launch(const char* what);

// CAPVNDF_OK if e == hipSuccess, else CAPVNDF_ERR_HIP naming the call.
int32_t check_hip(hipError_t e, const char* what);

inline bool aligned_to(const void* p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

// Checks one array argument: non-NULL and 4-byte aligned.
int32_t check_array(const void* p, const char* name);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline uint32_t key_lo(uint64_t seed) { return (uint32_t)seed; }
inline uint32_t key_hi(uint64_t seed) { return (uint32_t)(seed >> 32); }

}  // namespace capvndf
