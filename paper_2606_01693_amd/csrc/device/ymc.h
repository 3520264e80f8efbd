// G-WFQ-YMC (Section III-A): placeholder until the slow path lands; gq_create
// refuses GQ_WFQ_YMC while this header only declares the interface.
#pragma once
#include "common.h"
namespace gq {
namespace ymc {
__device__ __forceinline__ int enqueue(const gq_dev& q, uint64_t, uint32_t, uint32_t&) {
  latch_error(q.err, (uint64_t)(-GQ_ERR_INVALID));
  return GQ_ERR_INVALID;
}
__device__ __forceinline__ int dequeue(const gq_dev& q, uint64_t*, uint32_t, uint32_t&) {
  latch_error(q.err, (uint64_t)(-GQ_ERR_INVALID));
  return GQ_ERR_INVALID;
}
}  // namespace ymc
}  // namespace gq
