// Direct (FFT-free) A x and A^T r kernels, one instantiation per decimation.
#include "direct.hpp"
#include "launch.hpp"

namespace cs {

hipError_t launch_direct(int transpose, int d, const float* c, const float* in, float* out, long long n,
                         hipStream_t s) {
  const dim3 b(kDirT);
  const long long m = n / d;
  switch (d) {
#define CS_CASE(D)                                                                              \
  case D:                                                                                       \
    if (transpose)                                                                              \
      k_direct_adj<D><<<dim3((unsigned)((n + kDirOutT - 1) / kDirOutT)), b, 0, s>>>(c, in, out, n); \
    else                                                                                        \
      k_direct_fwd<D><<<dim3((unsigned)((m + dir_fwd_outputs<D>() - 1) / dir_fwd_outputs<D>())), b, 0, s>>>( \
          c, in, out, n);                                                                       \
    break;
    CS_CASE(2) CS_CASE(4) CS_CASE(8) CS_CASE(16)
#undef CS_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cs
