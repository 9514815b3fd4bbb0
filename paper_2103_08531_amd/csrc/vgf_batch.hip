// vgf_batch.hip -- device side of batched solves: refreshing the per-entry
// pointer tables that the captured passes read. The new pointers travel as
// kernel arguments (copied at launch), so the update is stream-ordered and
// needs no host staging buffer.
#include "vgf_internal.hpp"

namespace vgf {

namespace {

__global__ void k_set_pointers(void** dst, PtrChunk c) {
  const int i = (int)threadIdx.x;
  if (i < c.n) dst[i] = c.p[i];
}

}  // namespace

hipError_t launch_set_pointers(void** dst, const PtrChunk& c, hipStream_t s) {
  if (c.n <= 0) return hipSuccess;
  if (c.n > PtrChunk::kMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_set_pointers, dim3(1), dim3(PtrChunk::kMax), 0, s, dst, c);
  return hipGetLastError();
}

}  // namespace vgf
