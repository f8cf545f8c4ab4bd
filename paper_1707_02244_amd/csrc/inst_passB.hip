// Pass-B instantiation for one column length N1 = CS_LEN.
#include "launch.hpp"

#ifndef CS_LEN
#error "compile with -DCS_LEN=<column length>"
#endif

namespace cs {

template <>
hipError_t launch_passB<CS_LEN>(int mode, int grid, const PassBArgs& a, hipStream_t s) {
  constexpr int L = CS_LEN;
  const dim3 g(grid), b(kThreads);
  switch (mode) {
    case B_FWD_REAL: k_passB<L, B_FWD_REAL><<<g, b, 0, s>>>(a); break;
    case B_FWD_UP: k_passB<L, B_FWD_UP><<<g, b, 0, s>>>(a); break;
    case B_FWD_ZMU: k_passB<L, B_FWD_ZMU><<<g, b, 0, s>>>(a); break;
    case B_ISTA: k_passB<L, B_ISTA><<<g, b, 0, s>>>(a); break;
    case B_ADMM: k_passB<L, B_ADMM><<<g, b, 0, s>>>(a); break;
    case B_OUT_ALL: k_passB<L, B_OUT_ALL><<<g, b, 0, s>>>(a); break;
    case B_OUT_DEC: k_passB<L, B_OUT_DEC><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cs
