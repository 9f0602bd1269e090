// Bounds check of a caller buffer against the device allocation that holds it.
// Plain C++ (no HIP): the host validation calls it with the range reported by
// hipMemGetAddressRange, and a host-only unit test compiles it on its own.
#pragma once

#include <stddef.h>
#include <stdint.h>

// true when [p, p + bytes) lies inside [base, base + size); no intermediate sum
// can wrap around
inline bool sp6_range_inside(uintptr_t base, size_t size, uintptr_t p, size_t bytes) {
  if (p < base) return false;
  const uintptr_t off = p - base;
  if (off > size) return false;
  return bytes <= size - off;
}
