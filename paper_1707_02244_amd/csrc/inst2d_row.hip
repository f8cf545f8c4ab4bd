// 2-D row-pass instantiation for one packed row length H = CS_LEN.
#include "launch.hpp"
#include "kernels2d.hpp"

#ifndef CS_LEN
#error "compile with -DCS_LEN=<packed row length>"
#endif

namespace cs {

template <>
hipError_t launch2_row<CS_LEN>(int mode, int grid, const Row2Args& a, hipStream_t s) {
  constexpr int L = CS_LEN;
  const dim3 g(grid), b(row2_threads<L>());
  switch (mode) {
    case R2_FWD_REAL: k2_row<L, R2_FWD_REAL><<<g, b, 0, s>>>(a); break;
    case R2_FWD_UP: k2_row<L, R2_FWD_UP><<<g, b, 0, s>>>(a); break;
    case R2_FWD_ZMU: k2_row<L, R2_FWD_ZMU><<<g, b, 0, s>>>(a); break;
    case R2_ISTA: k2_row<L, R2_ISTA><<<g, b, 0, s>>>(a); break;
    case R2_ADMM: k2_row<L, R2_ADMM><<<g, b, 0, s>>>(a); break;
    case R2_OUT_ALL: k2_row<L, R2_OUT_ALL><<<g, b, 0, s>>>(a); break;
    case R2_OUT_DEC: k2_row<L, R2_OUT_DEC><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cs
