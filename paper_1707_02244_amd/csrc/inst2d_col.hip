// 2-D column-pass instantiation for one column length R = CS_LEN.
#include "launch.hpp"
#include "kernels2d.hpp"

#ifndef CS_LEN
#error "compile with -DCS_LEN=<column length>"
#endif

namespace cs {

template <>
hipError_t launch2_col<CS_LEN>(int op, int grid, const Col2Args& a, hipStream_t s) {
  constexpr int L = CS_LEN;
  const dim3 g(grid), b(col2_threads<L>());
  switch (op) {
    case C2_ISTA: k2_col<L, C2_ISTA><<<g, b, 0, s>>>(a); break;
    case C2_ADMM: k2_col<L, C2_ADMM><<<g, b, 0, s>>>(a); break;
    case C2_RES: k2_col<L, C2_RES><<<g, b, 0, s>>>(a); break;
    case C2_MUL: k2_col<L, C2_MUL><<<g, b, 0, s>>>(a); break;
    case C2_MULC: k2_col<L, C2_MULC><<<g, b, 0, s>>>(a); break;
    case C2_SPEC: k2_col<L, C2_SPEC><<<g, b, 0, s>>>(a); break;
    case C2_SPECMUL: k2_col<L, C2_SPECMUL><<<g, b, 0, s>>>(a); break;
    case C2_YHAT: k2_col<L, C2_YHAT><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cs
