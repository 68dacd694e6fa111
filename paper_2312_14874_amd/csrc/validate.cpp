#include "validate.hpp"

namespace mi355scan {

int check_dtype(int dtype) {
  if (dtype >= 0 && dtype <= 2) return kOk;
  return is_dtype64(dtype) ? kNotSupported : kInvalid;   // 64-bit: scan_flat only
}

int check_flags(uint32_t flags) { return (flags & ~kKnownFlags) ? kInvalid : kOk; }

int kernel_kind(int dtype, uint32_t flags) {
  switch (op_of(flags)) {
    case kOpSum: return dtype == 2 ? 1 : 0;
    case kOpMax:
    case kOpMin: return 2;
    default: return 3;
  }
}

uint32_t op_key(int dtype, uint32_t flags) {
  const bool sgn = dtype == 0;
  switch (op_of(flags)) {
    case kOpMax: return sgn ? 0x80000000u : 0u;
    case kOpMin: return sgn ? 0x7FFFFFFFu : 0xFFFFFFFFu;
    default: return 0u;
  }
}

int check_operator(int dtype, uint32_t flags) {
  if (op_of(flags) == kOpSum) return kOk;
  if (dtype == 2) return kNotSupported;
  if ((flags & kFlagReverse) && op_key(dtype, flags) != 0u) return kNotSupported;
  return kOk;
}

int check_flat(const void *in, const void *out, int64_t n) { return check_flat_sz(in, out, n, 4); }

int check_flat_sz(const void *in, const void *out, int64_t n, int esize) {
  if (n < 0) return kInvalid;
  if (n == 0) return kOk;
  if (!in || !out) return kInvalid;
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if ((a % (uintptr_t)esize) || (b % (uintptr_t)esize)) return kInvalid;
  if (n > (int64_t)(UINTPTR_MAX / 16)) return kInvalid;
  const uintptr_t bytes = (uintptr_t)n * (uintptr_t)esize;
  if (a + bytes < a || b + bytes < b) return kInvalid;   // address wrap
  if (a != b && a < b + bytes && b < a + bytes) return kOverlap;
  return kOk;
}

int check_segmented(const void *in, const void *out, const void *offsets,
                    int64_t num_segments, int64_t n) {
  if (num_segments < 0) return kInvalid;
  const int r = check_flat(in, out, n);
  if (r != kOk) return r;
  if (n == 0) return kOk;
  if (num_segments == 0) return kInvalid;     // offsets[S] = n > 0 needs a segment
  if (!offsets || ((uintptr_t)offsets & 7u)) return kInvalid;
  return kOk;
}

}  // namespace mi355scan
