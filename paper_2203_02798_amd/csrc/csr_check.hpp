// Validity of a matrix operand, shared by the checking kernel (k_check.hip)
// and its host-built test.
//
// A CSR matrix (Section 1, notation) of n rows, d columns and nnz stored
// entries is well formed when its row offsets start at 0, never decrease and
// end at nnz, and every column index lies in [0, d).  Those three facts are
// what every kernel that walks A's rows relies on: a decreasing offset or one
// past nnz sends a row's loop outside the entry arrays, an index outside
// [0, d) addresses outside the d-wide row sums.  Separately, a value that is
// not finite (NaN or an infinity) is reported under its own bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psk {

enum : uint32_t {
  kCheckStructure = 1u,  // offsets or an index break the CSR definition
  kCheckNonFinite = 2u,  // a stored value is NaN or infinite
};

// Row i (0 <= i < n) of the offsets: lo = indptr[i], hi = indptr[i + 1].
// Checking lo <= hi for every row, indptr[0] == 0 and indptr[n] == nnz bounds
// every offset to [0, nnz].
__host__ __device__ __forceinline__ uint32_t csr_row_code(int64_t lo, int64_t hi, int64_t i,
                                                          int64_t n, int64_t nnz) {
  bool bad = lo > hi;
  if (i == 0) bad |= lo != 0;
  if (i == n - 1) bad |= hi != nnz;
  return bad ? kCheckStructure : 0u;
}

// One stored column index against d (negative indices fail as large unsigned).
__host__ __device__ __forceinline__ uint32_t csr_index_code(int32_t c, int64_t d) {
  return (uint64_t)(uint32_t)c >= (uint64_t)d ? kCheckStructure : 0u;
}

// A stored value: finite or not, from its exponent field alone (all ones for
// NaN and both infinities), so no floating-point comparison decides it.
__host__ __device__ __forceinline__ uint32_t value_code(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  return ((b >> 52) & 0x7ffu) == 0x7ffu ? kCheckNonFinite : 0u;
}
__host__ __device__ __forceinline__ uint32_t value_code(float v) {
  const uint32_t b = __builtin_bit_cast(uint32_t, v);
  return ((b >> 23) & 0xffu) == 0xffu ? kCheckNonFinite : 0u;
}

}  // namespace psk
