// Batched-ISTA instantiation for one decimation, d = 2 * CS_D2.
#include "launch.hpp"
#include "batch.hpp"

#ifndef CS_D2
#error "compile with -DCS_D2=<d/2>"
#endif

namespace cs {

template <>
hipError_t launch_batch_ista<CS_D2>(const BatchSig* sigs, int count, unsigned* queue, int iters, int grid,
                                    hipStream_t s) {
  k_batch_ista<CS_D2><<<dim3(grid), dim3(kBThreads), 0, s>>>(sigs, count, queue, iters);
  return hipGetLastError();
}

template <>
int batch_blocks_per_cu<CS_D2>() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_batch_ista<CS_D2>),
                                                   kBThreads, 0) != hipSuccess)
    return 0;
  return nb;
}

}  // namespace cs
