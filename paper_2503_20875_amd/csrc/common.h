// Internal helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "cetra.h"

namespace cetra {

// Thread-local last-error message; returns `status` for tail calls.
int set_error(int status, const char *fmt, ...);
void clear_error();

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Checks the launch that was just enqueued.
int check_launch(const char *what);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Launch tuning currently in force (process-wide).
cetra_tuning current_tuning();

// LDS bytes of the linear tile (W windows per lane) for duration j, and its
// staged span (0 = the span does not fit `cap` bytes and is read directly).
constexpr int kMaxLinearLdsBytes = 64 * 1024;
size_t linear_lds_bytes(const cetra_grid *g, int j, int W, size_t cap, int32_t *span_cap);

// Validates the parts of a grid plan that kernels rely on.
int check_grid(const cetra_grid *g);

constexpr double kTwo32 = 4294967296.0;

}  // namespace cetra

#define CETRA_REQUIRE(cond, ...)                                          \
    do {                                                                  \
        if (!(cond)) return ::cetra::set_error(CETRA_ERR_INVALID, __VA_ARGS__); \
    } while (0)
