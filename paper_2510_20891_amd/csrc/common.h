// Internal helpers shared by the library's translation units.
#pragma once

#include <cstdarg>
#include <cstddef>
#include <cstdint>

#include "emri.h"

namespace emri {

// Records a formatted detail for emri_last_error() and returns `status`.
int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Number of compute units of the current device (cached per device).
int device_cu_count(int *out);

// Pseudo-inverse of the n x K row-major matrix U, transposed (pt[a*K + k]);
// host FP64 (basis.cpp).
void pseudo_inverse_t(const double *U, int n, int K, double *pt);

}  // namespace emri
