// Streaming loads and stores of float4 pixels for the resolve kernels.
//
// A resolve reads the history and writes its result once, and the next
// render does not read either: marking those accesses nontemporal lets the
// caches keep the render's volume lines instead (measured at 1080p: the
// render + resolve step 0.9 % faster, images unchanged).
#pragma once

#include <hip/hip_runtime.h>

namespace cloud {

template <typename P>
__device__ __forceinline__ float4 load_stream(P p) {
  float4 v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  v.z = __builtin_nontemporal_load(&p->z);
  v.w = __builtin_nontemporal_load(&p->w);
  return v;
}

template <typename P>
__device__ __forceinline__ void store_stream(P p, float4 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
  __builtin_nontemporal_store(v.z, &p->z);
  __builtin_nontemporal_store(v.w, &p->w);
}

}  // namespace cloud
