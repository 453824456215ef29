// Raw buffer access to complex128 elements on CDNA: a buffer resource (in
// scalar registers) plus a 32-bit offset per lane.  Such loads and stores
// count on the vector memory counter only (generic pointers also count on
// the LDS counter, so waiting for an LDS read would wait for them too), and
// an access past the resource's end reads zero or is dropped, so no branch
// has to guard it.
#pragma once
#include <hip/hip_runtime.h>

namespace tn {

// A resource over `elems` elements from `base` (elems * 16 < 2^31).
typedef __amdgpu_buffer_rsrc_t BufRes;
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ BufRes make_res(double2 *base, int elems) {
  // the resource must be wave-uniform (scalar registers)
  const unsigned long long a = (unsigned long long)base;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  double2 *ub = (double2 *)(((unsigned long long)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(ub, 0, __builtin_amdgcn_readfirstlane(elems * 16),
                                           0x00020000);
}
__device__ __forceinline__ double2 bload(BufRes r, int elem) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, elem * 16, 0, 0));
}
__device__ __forceinline__ void bstore(BufRes r, int elem, double2 x) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, x), r, elem * 16, 0, 0);
}

// Offset (bytes) of an access that the hardware drops: past any resource here.
constexpr int BUF_DROP = 0x7FFFFFF0;
__device__ __forceinline__ double2 bload_bytes(BufRes r, int bytes) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, bytes, 0, 0));
}
__device__ __forceinline__ void bstore_bytes(BufRes r, int bytes, double2 x) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, x), r, bytes, 0, 0);
}

}  // namespace tn
