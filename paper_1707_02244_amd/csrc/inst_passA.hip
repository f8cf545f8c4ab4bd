// Pass-A instantiation for one row length N2 = CS_LEN.
#include "launch.hpp"
#include "unrolled.hpp"
#include "cpadmm.hpp"

#ifndef CS_LEN
#error "compile with -DCS_LEN=<row length>"
#endif

namespace cs {

template <>
hipError_t launch_passA<CS_LEN>(int op, int d2, int grid, const PassAArgs& a, hipStream_t s) {
  constexpr int L = CS_LEN;
  const dim3 g(grid), b(pass_a_threads(L));
#define CS_GROUP_OP(OPV)                                                              \
  switch (d2) {                                                                       \
    case 0: k_passA<L, OPV, 0><<<g, b, 0, s>>>(a); break;                             \
    case 1: k_passA<L, OPV, 1><<<g, b, 0, s>>>(a); break;                             \
    case 2: k_passA<L, OPV, 2><<<g, b, 0, s>>>(a); break;                             \
    case 4: k_passA<L, OPV, 4><<<g, b, 0, s>>>(a); break;                             \
    case 8: k_passA<L, OPV, 8><<<g, b, 0, s>>>(a); break;                             \
    default: return hipErrorInvalidValue;                                             \
  }
  switch (op) {
    case A_ISTA: CS_GROUP_OP(A_ISTA); break;
    case A_ADMM: CS_GROUP_OP(A_ADMM); break;
    case A_RES: CS_GROUP_OP(A_RES); break;
    case A_MUL: k_passA<L, A_MUL, 1><<<g, b, 0, s>>>(a); break;
    case A_MULC: k_passA<L, A_MULC, 1><<<g, b, 0, s>>>(a); break;
    case A_SPEC: k_passA<L, A_SPEC, 1><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
#undef CS_GROUP_OP
  return hipGetLastError();
}

template <>
hipError_t launch_urow<CS_LEN>(int op, int d2, int grid, int batch, const PassAArgs& a, const UStride& st,
                               hipStream_t s) {
  constexpr int L = CS_LEN;
  const dim3 g(grid, batch), b(kThreads);
#define CS_U(OPV)                                                                      \
  switch (d2) {                                                                        \
    case 1: k_urow<L, OPV, 1><<<g, b, 0, s>>>(a, st); break;                           \
    case 2: k_urow<L, OPV, 2><<<g, b, 0, s>>>(a, st); break;                           \
    case 4: k_urow<L, OPV, 4><<<g, b, 0, s>>>(a, st); break;                           \
    case 8: k_urow<L, OPV, 8><<<g, b, 0, s>>>(a, st); break;                           \
    default: return hipErrorInvalidValue;                                              \
  }
  switch (op) {
    case A_ISTA: CS_U(A_ISTA); break;
    case A_ADJ: CS_U(A_ADJ); break;
    case A_TILE: CS_U(A_TILE); break;
    case A_SPEC: k_urow<L, A_SPEC, 1><<<g, b, 0, s>>>(a, st); break;
    default: return hipErrorInvalidValue;
  }
#undef CS_U
  return hipGetLastError();
}

template <>
hipError_t launch_cp_row<CS_LEN>(int grid, const CpArgs& a, hipStream_t s) {
  if constexpr (CS_LEN <= kCpMaxN2) {
    k_cp_row<CS_LEN, cp_row_threads(CS_LEN)><<<dim3(grid), dim3(cp_row_threads(CS_LEN)), 0, s>>>(a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

}  // namespace cs
