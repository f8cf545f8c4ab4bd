// Pass-B instantiation for one column length N1 = CS_LEN.
#include "launch.hpp"
#include "unrolled.hpp"
#include "cpadmm.hpp"

#ifndef CS_LEN
#error "compile with -DCS_LEN=<column length>"
#endif

namespace cs {

template <>
hipError_t launch_passB<CS_LEN>(int mode, int grid, const PassBArgs& a, hipStream_t s) {
  constexpr int L = CS_LEN;
  const dim3 g(grid), b(pass_b_threads(L));
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

template <>
hipError_t launch_ucol<CS_LEN>(int mode, int grid, int batch, const PassBArgs& a, const UStride& st,
                               hipStream_t s) {
  constexpr int L = CS_LEN;
  const dim3 g(grid, batch), b(kThreads);
  if constexpr (L > 2048) {   // the unrolled solver takes n <= 2^25
    (void)g; (void)b; (void)mode; (void)a; (void)st; (void)s;
    return hipErrorInvalidValue;
  } else {
  switch (mode) {
    case B_FWD_REAL: k_ucol<L, B_FWD_REAL><<<g, b, 0, s>>>(a, st); break;
    case B_FWD_UP: k_ucol<L, B_FWD_UP><<<g, b, 0, s>>>(a, st); break;
    case B_ISTA: k_ucol<L, B_ISTA><<<g, b, 0, s>>>(a, st); break;
    case B_ISTA_REC: k_ucol<L, B_ISTA_REC><<<g, b, 0, s>>>(a, st); break;
    case B_ADJ_V: k_ucol<L, B_ADJ_V><<<g, b, 0, s>>>(a, st); break;
    case B_ADJ_X: k_ucol<L, B_ADJ_X><<<g, b, 0, s>>>(a, st); break;
    case B_ADJ_XV: k_ucol<L, B_ADJ_XV><<<g, b, 0, s>>>(a, st); break;
    case B_OUT_DEC: k_ucol<L, B_OUT_DEC><<<g, b, 0, s>>>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
  }
}

template <>
hipError_t launch_cp_col<CS_LEN>(int last, int grid, const CpArgs& a, hipStream_t s) {
  if constexpr (CS_LEN <= kCpMaxN1) {
    constexpr int CB = cp_cb(CS_LEN);
    constexpr int T = cp_col_threads(CS_LEN);
    if (last) k_cp_col<CS_LEN, CB, T, true><<<dim3(grid), dim3(T), 0, s>>>(a);
    else k_cp_col<CS_LEN, CB, T, false><<<dim3(grid), dim3(T), 0, s>>>(a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

}  // namespace cs
