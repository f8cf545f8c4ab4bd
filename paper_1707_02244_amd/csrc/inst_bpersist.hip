// Persistent batched-solver instantiation for one algorithm (CS_ALG: 0 ISTA,
// 1 ADMM); every length and decimation of the batch is dispatched inside the
// kernel.
#include "launch.hpp"
#include "batch_persist.hpp"

#ifndef CS_ALG
#error "compile with -DCS_ALG=<0 for ISTA, 1 for ADMM>"
#endif

namespace cs {

template <>
const void* batch_persist_kernel<CS_ALG>() {
  return reinterpret_cast<const void*>(&k_batch_persist<CS_ALG>);
}

template <>
int batch_persist_blocks_per_cu<CS_ALG>() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_persist_kernel<CS_ALG>(), kPBThreads, 0) !=
      hipSuccess)
    return 0;
  return nb;
}

}  // namespace cs
