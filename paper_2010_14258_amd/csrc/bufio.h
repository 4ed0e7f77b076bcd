// Buffer-resource loads and stores of complex values for gfx950.
//
// A workgroup that streams a region of a waveform builds one buffer resource for it (the base must
// be the same for the whole wave) and addresses elements with a 32-bit per-lane byte offset plus a
// uniform byte offset, so sixteen loads along a team's sequence share one address register.  Reads
// past num_records return zero and writes past it are dropped by the hardware, which bounds every
// access to the region the resource names.
#pragma once

#include "common.h"

namespace ldbp {

// word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data, no swizzle, no index stride)
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0), static_cast<int>(bytes),
                                           kBufWord3);
}

template <typename R>
__device__ __forceinline__ cx_t<R> buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  cx_t<R> v;
  if constexpr (sizeof(R) == 4) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(voff), static_cast<int>(soff), 0);
    __builtin_memcpy(&v, &u, sizeof(v));
  } else {
    const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(voff), static_cast<int>(soff), 0);
    __builtin_memcpy(&v, &u, sizeof(v));
  }
  return v;
}

template <typename R>
__device__ __forceinline__ void buf_store(cx_t<R> v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(R) == 4) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    u2 u;
    __builtin_memcpy(&u, &v, sizeof(v));
    __builtin_amdgcn_raw_buffer_store_b64(u, r, static_cast<int>(voff), static_cast<int>(soff), 0);
  } else {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 u;
    __builtin_memcpy(&u, &v, sizeof(v));
    __builtin_amdgcn_raw_buffer_store_b128(u, r, static_cast<int>(voff), static_cast<int>(soff), 0);
  }
}

}  // namespace ldbp
