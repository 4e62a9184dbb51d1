// Streaming access to state amplitudes in HBM. Every plain gate touches each amplitude once
// (read, then write), so loads and stores carry the nontemporal hint: the state streams through
// the caches without displacing what is still reused there. Device code only.
#pragma once
#include <hip/hip_runtime.h>

namespace qd {

typedef double qd_v2d __attribute__((ext_vector_type(2)));
typedef float qd_v2f __attribute__((ext_vector_type(2)));
typedef unsigned qd_v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const qd_v2d t = __builtin_nontemporal_load(reinterpret_cast<const qd_v2d*>(p));
  return double2{t.x, t.y};
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const qd_v2f t = __builtin_nontemporal_load(reinterpret_cast<const qd_v2f*>(p));
  return float2{t.x, t.y};
}
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
  const qd_v4u t = __builtin_nontemporal_load(reinterpret_cast<const qd_v4u*>(p));
  return uint4{t.x, t.y, t.z, t.w};
}
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  __builtin_nontemporal_store(qd_v2d{v.x, v.y}, reinterpret_cast<qd_v2d*>(p));
}
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
  __builtin_nontemporal_store(qd_v2f{v.x, v.y}, reinterpret_cast<qd_v2f*>(p));
}
__device__ __forceinline__ void st_stream(uint4* p, uint4 v) {
  __builtin_nontemporal_store(qd_v4u{v.x, v.y, v.z, v.w}, reinterpret_cast<qd_v4u*>(p));
}

}  // namespace qd
