// Host-side argument validation for the C ABI.  No HIP calls: every check
// here runs before anything is enqueued, and can be tested without a GPU.
#pragma once
#include <stdint.h>

namespace mi355scan {

// Mirrors scan_status_t.
enum Status : int {
  kOk = 0, kInvalid = 1, kOverlap = 2, kOom = 3, kLaunch = 4,
  kNotSupported = 5, kCapture = 6, kTimeout = 7
};

constexpr uint32_t kFlagExclusive = 0x1u;
constexpr uint32_t kFlagReverse = 0x2u;
constexpr uint32_t kOpShift = 2;               // operator field: bits 2-3
constexpr uint32_t kOpMask = 0x3u << kOpShift;
enum Operator : uint32_t { kOpSum = 0, kOpMax = 1, kOpMin = 2, kOpXor = 3 };
constexpr uint32_t kKnownFlags = kFlagExclusive | kFlagReverse | kOpMask;

inline uint32_t op_of(uint32_t flags) { return (flags & kOpMask) >> kOpShift; }
// Kernel kind for (dtype, operator): 0 integer sum, 1 float32 sum, 2 keyed
// max (max and min), 3 xor.
int kernel_kind(int dtype, uint32_t flags);
// Key of the keyed max: the order (anti-)isomorphism x -> x ^ key that turns
// the operator into an unsigned max with identity 0.
uint32_t op_key(int dtype, uint32_t flags);
// Operator combinations the kernels do not provide: max / min / xor of
// float32, and a reverse scan whose identity is not 0 before keying (the
// buffer loads beyond n return 0, which a reverse scan meets first).
int check_operator(int dtype, uint32_t flags);

// dtype: 0 = i32, 1 = u32, 2 = f32
int check_dtype(int dtype);
int check_flags(uint32_t flags);
// in/out arrays of n 4-byte elements; in == out allowed, other overlap refused
int check_flat(const void *in, const void *out, int64_t n);
// the same for elements of esize bytes (aligned to esize)
int check_flat_sz(const void *in, const void *out, int64_t n, int esize);
// 64-bit dtypes (3 = int64, 4 = uint64, 5 = float64): scan_flat only
inline bool is_dtype64(int dtype) { return dtype >= 3 && dtype <= 5; }
// segmented batch: offsets (S+1 int64, 8-byte aligned) required when n > 0
int check_segmented(const void *in, const void *out, const void *offsets,
                    int64_t num_segments, int64_t n);

}  // namespace mi355scan
