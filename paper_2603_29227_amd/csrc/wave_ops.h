// Wave-level helpers shared by the query and the backward.
#pragma once

#include <hip/hip_runtime.h>

namespace ksdf {
namespace {

// Wave-aggregated counting-sort steps over small integer keys: the lanes that share
// a key take one atomic between them (the lowest lane issues it).
__device__ __forceinline__ void wave_count(int* count, int key, bool valid) {
  unsigned long long pending = __ballot(valid);
  const int lane = threadIdx.x & 63;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int k = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long mask = __ballot(valid && key == k);
    if (lane == leader) atomicAdd(count + k, (int)__popcll(mask));
    pending &= ~mask;
  }
}
// position of each valid lane in its key's range (cursor: running start per key)
__device__ __forceinline__ int wave_slot(int* cursor, int key, bool valid) {
  unsigned long long pending = __ballot(valid);
  const int lane = threadIdx.x & 63;
  int pos = -1;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int k = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long mask = __ballot(valid && key == k);
    int base = 0;
    if (lane == leader) base = atomicAdd(cursor + k, (int)__popcll(mask));
    base = __builtin_amdgcn_readlane(base, leader);
    if (valid && key == k) pos = base + (int)__popcll(mask & ((1ull << lane) - 1ull));
    pending &= ~mask;
  }
  return pos;
}

}  // namespace
}  // namespace ksdf
